/*
 * rt_oracle.c -- plain FP64 reference ("oracle") for the discrete formal
 * solution of the static 3D radiative transfer equation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or constant generator with the GPU library.
 *
 * What it computes (Hauschildt & Baron, "A 3D radiative transfer framework
 * XII", arXiv 2102.01734):
 *   - the transfer equation n.grad I = eta - chi I, S = eta/chi  (Sec. 2.1, eq. 1)
 *   - the formal solution J = Lambda S, i.e. I integrated along long
 *     characteristics for all solid angles and angle-averaged    (Sec. 2.2, eq. frmsol)
 *   - the approximate operator Lambda* (diagonal here) built in the same sweep
 *     (Sec. 4, "Method"; Listing 1 steps 4-4b)
 *   - per characteristic point: previous/next S and chi, optical steps,
 *     interpolation weights alpha, beta, gamma, boundary/vacuum fix-up and the
 *     Delta-I / exp(-dtau) update (Listing 1, steps 1-5).
 * The discretisation details the paper leaves open are read as follows
 * (each one is also listed in the design notes):
 *   - cubic voxels of edge 1, centres on integers, x,y periodic (Sec. 3.1);
 *   - directions: midpoint rule, equally spaced in mu and phi, equal weights
 *     (Sec. 3.1, "equally spaced in mu = cos(theta) and phi");
 *   - one characteristic per inflow-face voxel centre; all rays of one direction
 *     are integer translates of the ray through column (0,0);
 *   - points at segment midpoints carrying the voxel's S and chi; optical step
 *     between neighbouring points = half-sum of the two segment depths;
 *   - piecewise-parabolic interpolation of S in optical depth (Olson-Kunasz
 *     form) with a geometric fallback to linear interpolation;
 *   - voxel intensity = path-length weighted mean over all visits of the voxel.
 *
 * Compile with -ffp-contract=off: the optical steps are formed as
 * tau = chi*s and D = 0.5*(tau_a + tau_b), each correctly rounded.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_TIE 1e-12         /* crossings closer than 1e-12*(t+1) are one crossing */
#define ORC_SERIES_BELOW 0.25 /* small optical steps use the power series */

enum { ORC_LSTAR_LINEAR = 0, ORC_LSTAR_PARABOLIC = 1 };

/* ------------------------------------------------------------------------ */
/* Angle quadrature (Sec. 3.1 and 3.2: equally spaced in mu and phi).       */
/* Direction index d = i_mu * n_phi + j_phi.                                */
/* ------------------------------------------------------------------------ */
void orc_quadrature(int n_mu, int n_phi, double *mu, double *phi, double *w)
{
    for (int i = 0; i < n_mu; i++) {
        for (int j = 0; j < n_phi; j++) {
            int d = i * n_phi + j;
            mu[d] = -1.0 + (2.0 * i + 1.0) / n_mu;
            phi[d] = 2.0 * M_PI * (j + 0.5) / n_phi;
            w[d] = 1.0 / ((double)n_mu * (double)n_phi);
        }
    }
}

void orc_direction_vector(double mu, double phi, double *n3)
{
    double st = sqrt(1.0 - mu * mu);
    n3[0] = st * cos(phi);
    n3[1] = st * sin(phi);
    n3[2] = mu;
}

/* ------------------------------------------------------------------------ */
/* Tracker for the periodic box: the geometric path of the characteristic   */
/* that enters through the inflow face at the centre of column (0,0).      */
/* Method: list every plane crossing, sort them, merge crossings closer than */
/* the tie tolerance, and locate each segment by the voxel that contains    */
/* its midpoint.                                                            */
/*   di, dj : unwrapped voxel offsets from the entry column                 */
/*   kk     : layer index, 0 = top layer (z max), Nz-1 = bottom layer       */
/*   s      : path length of the segment inside that voxel                  */
/*   t0     : parameter (distance from the entry point) of the segment start*/
/* Returns the number of segments, or -1 if cap is too small.               */
/* ------------------------------------------------------------------------ */
static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x < y) ? -1 : (x > y) ? 1 : 0;
}

int orc_trace_box(int Nz, double nx, double ny, double nz, int cap,
                  int *di, int *dj, int *kk, double *s, double *t0)
{
    double ax = fabs(nx), ay = fabs(ny), az = fabs(nz);
    if (az <= 0.0 || Nz <= 0)
        return -1;
    double t_exit = Nz / az;
    /* count crossings */
    long nxc = 0, nyc = 0;
    if (ax > 0.0)
        while ((nxc + 0.5) / ax < t_exit) nxc++;
    if (ay > 0.0)
        while ((nyc + 0.5) / ay < t_exit) nyc++;
    long ntot = nxc + nyc + Nz; /* Nz-1 interior z planes + the exit plane */
    double *tc = (double *)malloc(sizeof(double) * (size_t)ntot);
    long n = 0;
    for (long i = 0; i < nxc; i++) tc[n++] = (i + 0.5) / ax;
    for (long i = 0; i < nyc; i++) tc[n++] = (i + 0.5) / ay;
    for (long k = 1; k <= Nz; k++) tc[n++] = k / az;
    qsort(tc, (size_t)n, sizeof(double), cmp_double);

    /* merge near-coincident crossings; the exit ends the ray */
    double prev = 0.0;
    int m = 0;
    for (long i = 0; i < n; i++) {
        double t = tc[i];
        int is_exit = (t >= t_exit);
        if (t - prev > ORC_TIE * (prev + 1.0)) {
            if (m >= cap) { free(tc); return -1; }
            double tm = 0.5 * (prev + t);
            di[m] = (int)floor(nx * tm + 0.5);
            dj[m] = (int)floor(ny * tm + 0.5);
            int depth = (int)floor(az * tm);
            if (depth > Nz - 1) depth = Nz - 1;
            kk[m] = (nz < 0.0) ? depth : (Nz - 1 - depth);
            s[m] = t - prev;
            t0[m] = prev;
            m++;
            prev = t;
        }
        if (is_exit) break;
    }
    free(tc);
    return m;
}

/* ------------------------------------------------------------------------ */
/* Moments of the attenuation kernel over one optical step D:               */
/*   e_n = integral_0^D t^n exp(-(D-t)) dt,  n = 0,1,2                      */
/*   e0 = 1 - exp(-D), e1 = D - e0, e2 = D^2 - 2 e1.                        */
/* For D < 0.25 e1 and e2 come from their power series (the closed forms    */
/* cancel catastrophically there).                                          */
/* ------------------------------------------------------------------------ */
void orc_moments(double D, double *e0, double *e1, double *e2)
{
    *e0 = -expm1(-D);
    if (D < ORC_SERIES_BELOW) {
        /* e1 = sum_{n>=2} (-1)^n D^n/n!,  e2 = 2 sum_{n>=3} (-1)^(n+1) D^n/n! */
        double term = 0.5 * D * D; /* D^n/n! for n = 2 */
        double s1 = 0.0, s2 = 0.0;
        for (int n = 2; n <= 17; n++) {
            double sg = (n % 2 == 0) ? 1.0 : -1.0;
            s1 += sg * term;
            if (n >= 3) s2 -= sg * term;
            term *= D / (n + 1);
        }
        *e1 = s1;
        *e2 = 2.0 * s2;
    } else {
        *e1 = D - *e0;
        *e2 = D * D - 2.0 * (*e1);
    }
}

/* D coth(D/2) - 2: the largest downwind step D' for which the parabolic
   weight beta reaches 1 (beta >= 1 <=> D' <= D coth(D/2) - 2). */
double orc_beta_limit(double D)
{
    if (D < 0.1) {
        double D2 = D * D;
        return D2 / 6.0 - D2 * D2 / 360.0 + D2 * D2 * D2 / 15120.0 - D2 * D2 * D2 * D2 / 604800.0;
    }
    return D / tanh(0.5 * D) - 2.0;
}

/*
 * Weights of one segment P_{m-1} -> P_m (upwind step D, downwind step Dp):
 *   I_m = I_{m-1} exp(-D) + alpha S_{m-1} + beta S_m + gamma S_{m+1}.
 * They integrate the Lagrange quadratic through (0,S_{m-1}), (D,S_m),
 * (D+Dp,S_{m+1}) against exp(-(D-t)) (Listing 1, step 4).  The linear
 * interpolant (gamma = 0) is used on the last segment of a ray, when
 * Dp < D/2, or when the parabolic beta would reach 1.  D = 0 (vacuum
 * segment) gives all-zero weights (Listing 1, step 4a).
 * Returns 1 if the linear form was used.
 */
int orc_weights(double D, double Dp, int last, double *a, double *b, double *g)
{
    double e0, e1, e2;
    if (!(D > 0.0)) {
        *a = *b = *g = 0.0;
        return 1;
    }
    orc_moments(D, &e0, &e1, &e2);
    int lin = last || (Dp < 0.5 * D) || (Dp <= orc_beta_limit(D));
    if (lin) {
        *a = e0 - e1 / D;
        *b = e1 / D;
        *g = 0.0;
    } else {
        *a = e0 + (e2 - (2.0 * D + Dp) * e1) / (D * (D + Dp));
        *b = ((D + Dp) * e1 - e2) / (D * Dp);
        *g = (e2 - D * e1) / (Dp * (D + Dp));
    }
    return lin;
}

/*
 * Formal solution along one characteristic with M points.
 *   tau[m] : optical depth chi*s of segment m (m = 0..M-1)
 *   S[m]   : source function of the voxel of segment m
 *   I_bc   : intensity entering the ray
 * Output: I[m] at the segment midpoints P_m, and the local operator diagonal
 * d[m] = dI_m/dS_m (parabolic: the weights actually used; linear: the
 * linear-interpolation weight e1/D).
 */
void orc_ray(int M, const double *tau, const double *S, double I_bc,
             int lstar_kind, double *I, double *d)
{
    if (M <= 0) return;
    /* entry half segment: S constant from the entry point to P_1 */
    double D0 = 0.5 * tau[0];
    double x0 = exp(-D0);
    double e00 = -expm1(-D0);
    I[0] = I_bc * x0 + S[0] * e00;
    if (d) d[0] = e00;
    double gprev = 0.0; /* downwind weight used for the previous point */
    for (int m = 1; m < M; m++) {
        int last = (m == M - 1);
        double D = 0.5 * (tau[m - 1] + tau[m]);
        double Dp = last ? 0.0 : 0.5 * (tau[m] + tau[m + 1]);
        double a, b, g;
        orc_weights(D, Dp, last, &a, &b, &g);
        double ex = exp(-D);
        double Sn = last ? 0.0 : S[m + 1];
        I[m] = I[m - 1] * ex + a * S[m - 1] + b * S[m] + g * Sn;
        if (d) {
            if (lstar_kind == ORC_LSTAR_PARABOLIC) {
                d[m] = b + gprev * ex;
            } else {
                double e0, e1, e2;
                if (D > 0.0) {
                    orc_moments(D, &e0, &e1, &e2);
                    d[m] = e1 / D;
                } else {
                    d[m] = 0.0;
                }
            }
        }
        gprev = g;
    }
}

/* ------------------------------------------------------------------------ */
/* Full formal solution on the periodic box.                                */
/* Arrays are [k][y][x] with k = 0 the top layer; x fastest.                */
/* I_top enters rays going down (mu < 0), I_bot rays going up (mu > 0).     */
/* J and lstar (lstar may be NULL) are overwritten.                         */
/* Returns 0 on success, <0 on error.                                       */
/* ------------------------------------------------------------------------ */
typedef struct {
    int M;
    int *di, *dj, *kk;
    double *s, *t0;
} orc_path;

static int orc_make_path(int Nz, const double *n3, orc_path *p)
{
    double az = fabs(n3[2]);
    double st = sqrt(n3[0] * n3[0] + n3[1] * n3[1]);
    /* generous cap: every unit of parameter crosses at most 3 planes */
    int cap = (int)(3.0 * (Nz / az) * (1.0 + st) + 16.0);
    p->di = (int *)malloc(sizeof(int) * cap);
    p->dj = (int *)malloc(sizeof(int) * cap);
    p->kk = (int *)malloc(sizeof(int) * cap);
    p->s = (double *)malloc(sizeof(double) * cap);
    p->t0 = (double *)malloc(sizeof(double) * cap);
    p->M = orc_trace_box(Nz, n3[0], n3[1], n3[2], cap, p->di, p->dj, p->kk, p->s, p->t0);
    return p->M;
}

static void orc_free_path(orc_path *p)
{
    free(p->di); free(p->dj); free(p->kk); free(p->s); free(p->t0);
}

static inline int wrap(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

/* Formal solution restricted to the listed directions (dirs = NULL: all of
   them); J and lstar then hold the partial angle sums over those directions. */
int orc_fs_box_dirs(int Nx, int Ny, int Nz, int n_mu, int n_phi,
                    const double *chi, const double *S, double I_top, double I_bot,
                    int lstar_kind, int n_sub, const int *dirs, double *J, double *lstar, int nthreads)
{
    int ndir = n_mu * n_phi;
    int nloop = dirs ? n_sub : ndir;
    long nvox = (long)Nx * Ny * Nz;
    double *mu = (double *)malloc(sizeof(double) * ndir);
    double *ph = (double *)malloc(sizeof(double) * ndir);
    double *w = (double *)malloc(sizeof(double) * ndir);
    orc_quadrature(n_mu, n_phi, mu, ph, w);
    memset(J, 0, sizeof(double) * nvox);
    if (lstar) memset(lstar, 0, sizeof(double) * nvox);
    int err = 0;
    if (nthreads <= 0) nthreads = 1;
    /* per-thread accumulators, combined in thread order at the end */
    double *Jt = (double *)calloc((size_t)nthreads * nvox, sizeof(double));
    double *Lt = lstar ? (double *)calloc((size_t)nthreads * nvox, sizeof(double)) : NULL;

#pragma omp parallel num_threads(nthreads)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *num = (double *)malloc(sizeof(double) * nvox);
        double *den = (double *)malloc(sizeof(double) * nvox);
        double *lnum = lstar ? (double *)malloc(sizeof(double) * nvox) : NULL;
        double *Jmy = Jt + (size_t)tid * nvox;
        double *Lmy = lstar ? Lt + (size_t)tid * nvox : NULL;
#pragma omp for schedule(static, 1)
        for (int q = 0; q < nloop; q++) {
            int d = dirs ? dirs[q] : q;
            double n3[3];
            orc_direction_vector(mu[d], ph[d], n3);
            orc_path p;
            if (orc_make_path(Nz, n3, &p) <= 0) {
#pragma omp atomic write
                err = -2;
                orc_free_path(&p);
                continue;
            }
            int M = p.M;
            double *tau = (double *)malloc(sizeof(double) * M);
            double *Sv = (double *)malloc(sizeof(double) * M);
            double *I = (double *)malloc(sizeof(double) * M);
            double *dd = (double *)malloc(sizeof(double) * M);
            long *vid = (long *)malloc(sizeof(long) * M);
            memset(num, 0, sizeof(double) * nvox);
            memset(den, 0, sizeof(double) * nvox);
            if (lnum) memset(lnum, 0, sizeof(double) * nvox);
            double Ibc = (mu[d] < 0.0) ? I_top : I_bot;
            for (int y0 = 0; y0 < Ny; y0++) {
                for (int x0 = 0; x0 < Nx; x0++) {
                    for (int m = 0; m < M; m++) {
                        long v = ((long)p.kk[m] * Ny + wrap(y0 + p.dj[m], Ny)) * Nx + wrap(x0 + p.di[m], Nx);
                        vid[m] = v;
                        tau[m] = chi[v] * p.s[m];
                        Sv[m] = S[v];
                    }
                    orc_ray(M, tau, Sv, Ibc, lstar_kind, I, lnum ? dd : NULL);
                    for (int m = 0; m < M; m++) {
                        num[vid[m]] += p.s[m] * I[m];
                        den[vid[m]] += p.s[m];
                        if (lnum) lnum[vid[m]] += p.s[m] * dd[m];
                    }
                }
            }
            for (long v = 0; v < nvox; v++) {
                if (den[v] > 0.0) {
                    Jmy[v] += w[d] * num[v] / den[v];
                    if (Lmy) Lmy[v] += w[d] * lnum[v] / den[v];
                }
            }
            free(tau); free(Sv); free(I); free(dd); free(vid);
            orc_free_path(&p);
        }
        free(num); free(den); free(lnum);
    }
    for (int t = 0; t < nthreads; t++) {
        for (long v = 0; v < nvox; v++) {
            J[v] += Jt[(size_t)t * nvox + v];
            if (lstar) lstar[v] += Lt[(size_t)t * nvox + v];
        }
    }
    free(Jt); free(Lt);
    free(mu); free(ph); free(w);
    return err;
}

int orc_fs_box(int Nx, int Ny, int Nz, int n_mu, int n_phi,
               const double *chi, const double *S, double I_top, double I_bot,
               int lstar_kind, double *J, double *lstar, int nthreads)
{
    return orc_fs_box_dirs(Nx, Ny, Nz, n_mu, n_phi, chi, S, I_top, I_bot, lstar_kind, 0, NULL, J, lstar,
                           nthreads);
}

/*
 * The same formal solution evaluated only at a list of voxels: for every
 * direction and every visit of the voxel, the characteristic through it is
 * integrated from its entry point up to that visit.  Used to check large
 * grids one voxel at a time.
 */
int orc_fs_box_sampled(int Nx, int Ny, int Nz, int n_mu, int n_phi,
                       const double *chi, const double *S, double I_top, double I_bot,
                       int lstar_kind, int nsamp, const long *vox,
                       double *J, double *lstar, int nthreads)
{
    int ndir = n_mu * n_phi;
    double *mu = (double *)malloc(sizeof(double) * ndir);
    double *ph = (double *)malloc(sizeof(double) * ndir);
    double *w = (double *)malloc(sizeof(double) * ndir);
    orc_quadrature(n_mu, n_phi, mu, ph, w);
    int err = 0;
    if (nthreads <= 0) nthreads = 1;
    double *Jd = (double *)calloc((size_t)ndir * nsamp, sizeof(double));
    double *Ld = (double *)calloc((size_t)ndir * nsamp, sizeof(double));
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
    for (int d = 0; d < ndir; d++) {
        double n3[3];
        orc_direction_vector(mu[d], ph[d], n3);
        orc_path p;
        if (orc_make_path(Nz, n3, &p) <= 0) {
#pragma omp atomic write
            err = -2;
            orc_free_path(&p);
            continue;
        }
        int M = p.M;
        double *tau = (double *)malloc(sizeof(double) * M);
        double *Sv = (double *)malloc(sizeof(double) * M);
        double *I = (double *)malloc(sizeof(double) * M);
        double *dd = (double *)malloc(sizeof(double) * M);
        double Ibc = (mu[d] < 0.0) ? I_top : I_bot;
        for (int q = 0; q < nsamp; q++) {
            long v = vox[q];
            int xv = (int)(v % Nx), yv = (int)((v / Nx) % Ny), kv = (int)(v / ((long)Nx * Ny));
            double num = 0.0, den = 0.0, lnum = 0.0;
            for (int m = 0; m < M; m++) {
                if (p.kk[m] != kv) continue;
                /* the ray whose m-th segment lies in voxel v */
                int x0 = wrap(xv - p.di[m], Nx), y0 = wrap(yv - p.dj[m], Ny);
                int Mq = (m + 2 < M) ? m + 2 : M; /* up to and incl. the downwind point */
                for (int j = 0; j < Mq; j++) {
                    long u = ((long)p.kk[j] * Ny + wrap(y0 + p.dj[j], Ny)) * Nx + wrap(x0 + p.di[j], Nx);
                    tau[j] = chi[u] * p.s[j];
                    Sv[j] = S[u];
                }
                /* a ray truncated after m+1 points must still treat point m
                   as interior when the full ray continues: integrate Mq points
                   but only use I[m]; point m is "last" only if m == M-1 */
                orc_ray(Mq, tau, Sv, Ibc, lstar_kind, I, dd);
                num += p.s[m] * I[m];
                lnum += p.s[m] * dd[m];
                den += p.s[m];
            }
            if (den > 0.0) {
                Jd[(size_t)d * nsamp + q] = w[d] * num / den;
                Ld[(size_t)d * nsamp + q] = w[d] * lnum / den;
            }
        }
        free(tau); free(Sv); free(I); free(dd);
        orc_free_path(&p);
    }
    for (int q = 0; q < nsamp; q++) {
        double a = 0.0, b = 0.0;
        for (int d = 0; d < ndir; d++) {
            a += Jd[(size_t)d * nsamp + q];
            b += Ld[(size_t)d * nsamp + q];
        }
        J[q] = a;
        if (lstar) lstar[q] = b;
    }
    free(Jd); free(Ld); free(mu); free(ph); free(w);
    return err;
}

/* Template of one direction, exported for tracker tests. */
int orc_box_template(int Nz, double mu, double phi, int cap,
                     int *di, int *dj, int *kk, double *s, double *t0)
{
    double n3[3];
    orc_direction_vector(mu, phi, n3);
    return orc_trace_box(Nz, n3[0], n3[1], n3[2], cap, di, dj, kk, s, t0);
}

/*
 * x,y-homogeneous reduction: when chi and S depend on the layer only, every
 * ray of a direction sees the same sequence of values, so J of a layer is the
 * path-length weighted mean of I over that layer along the single template
 * ray, summed over directions.  chi_k, S_k, J_k, L_k have Nz entries (k = 0
 * top).  Used for plane-parallel checks (sqrt(eps) law, flux conservation).
 */
int orc_fs_1d(int Nz, int n_mu, int n_phi, const double *chi_k, const double *S_k,
              double I_top, double I_bot, int lstar_kind, double *J_k, double *L_k)
{
    int ndir = n_mu * n_phi;
    double *mu = (double *)malloc(sizeof(double) * ndir);
    double *ph = (double *)malloc(sizeof(double) * ndir);
    double *w = (double *)malloc(sizeof(double) * ndir);
    orc_quadrature(n_mu, n_phi, mu, ph, w);
    double *num = (double *)malloc(sizeof(double) * Nz);
    double *den = (double *)malloc(sizeof(double) * Nz);
    double *lnum = (double *)malloc(sizeof(double) * Nz);
    memset(J_k, 0, sizeof(double) * Nz);
    if (L_k) memset(L_k, 0, sizeof(double) * Nz);
    int err = 0;
    for (int d = 0; d < ndir; d++) {
        double n3[3];
        orc_direction_vector(mu[d], ph[d], n3);
        orc_path p;
        if (orc_make_path(Nz, n3, &p) <= 0) { err = -2; orc_free_path(&p); continue; }
        int M = p.M;
        double *tau = (double *)malloc(sizeof(double) * M);
        double *Sv = (double *)malloc(sizeof(double) * M);
        double *I = (double *)malloc(sizeof(double) * M);
        double *dd = (double *)malloc(sizeof(double) * M);
        for (int m = 0; m < M; m++) {
            tau[m] = chi_k[p.kk[m]] * p.s[m];
            Sv[m] = S_k[p.kk[m]];
        }
        orc_ray(M, tau, Sv, (mu[d] < 0.0) ? I_top : I_bot, lstar_kind, I, dd);
        memset(num, 0, sizeof(double) * Nz);
        memset(den, 0, sizeof(double) * Nz);
        memset(lnum, 0, sizeof(double) * Nz);
        for (int m = 0; m < M; m++) {
            num[p.kk[m]] += p.s[m] * I[m];
            den[p.kk[m]] += p.s[m];
            lnum[p.kk[m]] += p.s[m] * dd[m];
        }
        for (int k = 0; k < Nz; k++) {
            if (den[k] > 0.0) {
                J_k[k] += w[d] * num[k] / den[k];
                if (L_k) L_k[k] += w[d] * lnum[k] / den[k];
            }
        }
        free(tau); free(Sv); free(I); free(dd);
        orc_free_path(&p);
    }
    free(num); free(den); free(lnum); free(mu); free(ph); free(w);
    return err;
}

/*
 * Directional intensities of the x,y-homogeneous reduction, for flux checks:
 * Iout[d*Nz + k] = path-length weighted mean intensity of direction d in
 * layer k.
 */
int orc_fs_1d_dirs(int Nz, int n_mu, int n_phi, const double *chi_k, const double *S_k,
                   double I_top, double I_bot, double *Iout)
{
    int ndir = n_mu * n_phi;
    double *mu = (double *)malloc(sizeof(double) * ndir);
    double *ph = (double *)malloc(sizeof(double) * ndir);
    double *w = (double *)malloc(sizeof(double) * ndir);
    orc_quadrature(n_mu, n_phi, mu, ph, w);
    double *num = (double *)malloc(sizeof(double) * Nz);
    double *den = (double *)malloc(sizeof(double) * Nz);
    int err = 0;
    for (int d = 0; d < ndir; d++) {
        double n3[3];
        orc_direction_vector(mu[d], ph[d], n3);
        orc_path p;
        if (orc_make_path(Nz, n3, &p) <= 0) { err = -2; orc_free_path(&p); continue; }
        int M = p.M;
        double *tau = (double *)malloc(sizeof(double) * M);
        double *Sv = (double *)malloc(sizeof(double) * M);
        double *I = (double *)malloc(sizeof(double) * M);
        for (int m = 0; m < M; m++) {
            tau[m] = chi_k[p.kk[m]] * p.s[m];
            Sv[m] = S_k[p.kk[m]];
        }
        orc_ray(M, tau, Sv, (mu[d] < 0.0) ? I_top : I_bot, ORC_LSTAR_LINEAR, I, NULL);
        memset(num, 0, sizeof(double) * Nz);
        memset(den, 0, sizeof(double) * Nz);
        for (int m = 0; m < M; m++) {
            num[p.kk[m]] += p.s[m] * I[m];
            den[p.kk[m]] += p.s[m];
        }
        for (int k = 0; k < Nz; k++)
            Iout[(size_t)d * Nz + k] = den[k] > 0.0 ? num[k] / den[k] : 0.0;
        free(tau); free(Sv); free(I);
        orc_free_path(&p);
    }
    free(num); free(den); free(mu); free(ph); free(w);
    return err;
}
