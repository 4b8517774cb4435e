/* sanitize_oracle.c -- drives the oracle's C library (box and spherical
 * formal solutions, operator columns, nearest-neighbour stencil, 1D
 * reductions, tracker templates) on tiny grids under AddressSanitizer /
 * UndefinedBehaviorSanitizer.  Exits non-zero on a failed invariant; the
 * sanitizers abort on any memory or undefined-behaviour error. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_fs_box(int Nx, int Ny, int Nz, int n_mu, int n_phi, const double *chi, const double *S, double I_top,
               double I_bot, int lstar_kind, double *J, double *lstar, int nthreads);
int orc_fs_box_dirs(int Nx, int Ny, int Nz, int n_mu, int n_phi, const double *chi, const double *S, double I_top,
                    double I_bot, int lstar_kind, int n_sub, const int *dirs, double *J, double *lstar, int nthreads);
int orc_fs_box_sampled(int Nx, int Ny, int Nz, int n_mu, int n_phi, const double *chi, const double *S, double I_top,
                       double I_bot, int lstar_kind, int nsamp, const long *vox, double *J, double *lstar,
                       int nthreads);
int orc_fs_box_op(int Nx, int Ny, int Nz, int n_mu, int n_phi, const double *chi, const double *S, double I_top,
                  double I_bot, int op, double *J);
int orc_lstar_stencil_box(int Nx, int Ny, int Nz, int n_mu, int n_phi, const double *chi, int op, double *out,
                          int nthreads);
int orc_box_template(int Nz, double mu, double phi, int cap, int *di, int *dj, int *kk, double *s, double *t0);
int orc_fs_1d(int Nz, int n_mu, int n_phi, const double *chi_k, const double *S_k, double I_top, double I_bot,
              int lstar_kind, double *J_k, double *L_k);
int orc_fs_1d_dirs(int Nz, int n_mu, int n_phi, const double *chi_k, const double *S_k, double I_top, double I_bot,
                   double *Iout);
int orc_fs_sphere(int Nr, int Nt, int Np, double rc, double ro, int n_mu, int n_phi, double dsrc, double B_sub,
                  const double *chi, const double *S, const double *Bv, double I_out, int lstar_kind, double *J,
                  double *lstar, int nthreads);
int orc_lstar_stencil_sphere(int Nr, int Nt, int Np, double rc, double ro, int n_mu, int n_phi, const double *chi,
                             int op, double *out, int nthreads);

static int fails = 0;
static long checks = 0;
#define CHECK(c)                                                                  \
    do {                                                                          \
        ++checks;                                                                 \
        if (!(c)) {                                                               \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__);       \
            ++fails;                                                              \
        }                                                                         \
    } while (0)

static double urand(unsigned *st)
{
    *st = *st * 1664525u + 1013904223u;
    return (*st >> 8) * (1.0 / 16777216.0);
}

static void box_case(int Nx, int Ny, int Nz, int n_mu, int n_phi, unsigned seed)
{
    const long n = (long)Nx * Ny * Nz;
    const int ndir = n_mu * n_phi;
    double *chi = malloc(sizeof(double) * n), *S = malloc(sizeof(double) * n);
    double *J = malloc(sizeof(double) * n), *L = malloc(sizeof(double) * n);
    double *J1 = calloc(n, sizeof(double)), *L1 = calloc(n, sizeof(double));
    double *Jp = malloc(sizeof(double) * n), *Lp = malloc(sizeof(double) * n);
    double *st = malloc(sizeof(double) * 27 * n), *col = malloc(sizeof(double) * n);
    int *dirs = malloc(sizeof(int) * ndir);
    for (long v = 0; v < n; ++v) {
        chi[v] = 0.05 + 3.0 * urand(&seed);
        S[v] = 0.2 + urand(&seed);
    }
    for (int kind = 0; kind < 2; ++kind) {
        CHECK(orc_fs_box(Nx, Ny, Nz, n_mu, n_phi, chi, S, 0.0, 1.0, kind, J, L, 2) == 0);
        for (long v = 0; v < n; ++v) CHECK(isfinite(J[v]) && L[v] >= 0.0 && L[v] < 1.0);
        /* direction subsets sum to the full solution */
        memset(J1, 0, sizeof(double) * n);
        memset(L1, 0, sizeof(double) * n);
        for (int part = 0; part < 2; ++part) {
            int m = 0;
            for (int d = part; d < ndir; d += 2) dirs[m++] = d;
            CHECK(orc_fs_box_dirs(Nx, Ny, Nz, n_mu, n_phi, chi, S, 0.0, 1.0, kind, m, dirs, Jp, Lp, 2) == 0);
            for (long v = 0; v < n; ++v) {
                J1[v] += Jp[v];
                L1[v] += Lp[v];
            }
        }
        for (long v = 0; v < n; ++v) CHECK(fabs(J1[v] - J[v]) <= 1e-13 * fabs(J[v]) + 1e-15);
        /* sampled voxels */
        long vox[3] = {0, n / 2, n - 1};
        double Js[3], Ls[3];
        CHECK(orc_fs_box_sampled(Nx, Ny, Nz, n_mu, n_phi, chi, S, 0.0, 1.0, kind, 3, vox, Js, Ls, 2) == 0);
        for (int i = 0; i < 3; ++i) CHECK(fabs(Js[i] - J[vox[i]]) <= 1e-12 * fabs(J[vox[i]]));
    }
    /* operator column and stencil of both operators */
    for (int op = 0; op < 2; ++op) {
        memset(col, 0, sizeof(double) * n);
        col[n / 2] = 1.0;
        CHECK(orc_fs_box_op(Nx, Ny, Nz, n_mu, n_phi, chi, col, 0.0, 0.0, op, J) == 0);
        CHECK(orc_lstar_stencil_box(Nx, Ny, Nz, n_mu, n_phi, chi, op, st, 2) == 0);
        for (long i = 0; i < 27 * n; ++i) CHECK(isfinite(st[i]));
    }
    free(chi); free(S); free(J); free(L); free(J1); free(L1); free(Jp); free(Lp); free(st); free(col); free(dirs);
}

int main(void)
{
    box_case(1, 1, 1, 2, 1, 1u);
    box_case(5, 4, 3, 2, 4, 2u);
    box_case(7, 5, 6, 4, 8, 3u);
    box_case(9, 9, 1, 2, 4, 4u);
    {
        int di[4096], dj[4096], kk[4096];
        double s[4096], t0[4096];
        const int M = orc_box_template(7, -0.3, 1.1, 4096, di, dj, kk, s, t0);
        CHECK(M > 0);
        double sum = 0.0;
        for (int m = 0; m < M; ++m) sum += s[m];
        CHECK(fabs(sum - 7.0 / 0.3) < 1e-9);
        CHECK(orc_box_template(7, -0.3, 1.1, 2, di, dj, kk, s, t0) < 0); /* capacity reported, nothing overrun */
    }
    {
        enum { Nz = 12, NMU = 4, NPHI = 2 };
        double chi[Nz], S[Nz], J[Nz], L[Nz], I[NMU * NPHI * Nz];
        for (int k = 0; k < Nz; ++k) {
            chi[k] = pow(10.0, -2.0 + 0.3 * k);
            S[k] = 1.0;
        }
        CHECK(orc_fs_1d(Nz, NMU, NPHI, chi, S, 0.0, 1.0, 1, J, L) == 0);
        CHECK(orc_fs_1d_dirs(Nz, NMU, NPHI, chi, S, 0.0, 1.0, I) == 0);
        for (int k = 0; k < Nz; ++k) CHECK(isfinite(J[k]) && L[k] >= 0.0 && L[k] < 1.0);
    }
    {
        enum { NR = 4, NT = 3, NP = 6 };
        const long n = NR * NT * NP;
        double chi[NR * NT * NP], S[NR * NT * NP], Bv[NR * NT * NP], J[NR * NT * NP], L[NR * NT * NP];
        unsigned seed = 9u;
        for (long v = 0; v < n; ++v) {
            chi[v] = 0.1 + urand(&seed);
            S[v] = 0.5 + urand(&seed);
            Bv[v] = 1.0;
        }
        CHECK(orc_fs_sphere(NR, NT, NP, 1.0, 3.0, 2, 4, 0.0, 1.0, chi, S, Bv, 0.0, 0, J, L, 2) == 0);
        for (long v = 0; v < n; ++v) CHECK(isfinite(J[v]) && J[v] >= 0.0);
        CHECK(orc_fs_sphere(NR, NT, NP, 0.5, 2.0, 2, 4, 4.0, 1.0, chi, S, Bv, 0.0, 1, J, L, 2) == 0);
        for (long v = 0; v < n; ++v) CHECK(isfinite(J[v]) && J[v] >= 0.0);
        double *st = malloc(sizeof(double) * 27 * n);
        for (int op = 0; op < 2; ++op) {
            CHECK(orc_lstar_stencil_sphere(NR, NT, NP, 1.0, 3.0, 2, 4, chi, op, st, 2) == 0);
            for (long i = 0; i < 27 * n; ++i) CHECK(isfinite(st[i]));
        }
        CHECK(orc_lstar_stencil_sphere(NR, NT, 2, 1.0, 3.0, 2, 4, chi, 0, st, 2) != 0); /* Nphi < 3 refused */
        free(st);
    }
    if (fails) {
        fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    printf("%ld oracle checks passed\n", checks);
    return 0;
}
