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

/* ------------------------------------------------------------------------ */
/* Operators and the nearest-neighbour Lambda* (Sec. 2, eq. alo; Sec. 3:    */
/* the paper's runs use a non-local Lambda*).                              */
/*                                                                          */
/* The formal solution is linear in S: I_p = I_{p-1} ex_p + a_p S_{p-1}     */
/* + b_p S_p + g_p S_{p+1} along a characteristic.  Two operators are       */
/* used: op = parabolic, the formal solution itself (Lambda), and op =      */
/* linear, linear interpolation at every point (the operator whose          */
/* diagonal is the default Lambda*).  The nearest-neighbour Lambda* is      */
/* Lambda_op restricted to the 27 voxels u with |u - v| <= 1 per axis:      */
/*   Lambda*_{v,u} = sum_d w_d sum_{m: v_m = v} s_m dI_m/dS_u / sum s_m.     */
/* dI_m/dS_u is the sum, over the points p whose update uses S_u, of that   */
/* weight times the attenuation from p to m.  A voxel more than three       */
/* points upstream of m differs from v_m by 2 or more along some axis (each */
/* step of a straight ray moves at least one coordinate by one, never back),*/
/* and points downstream of m + 1 do not enter I_m, so only the points      */
/* m - 3 .. m + 1 can be neighbours that contribute.                        */
/* Components c = (dz+1)*9 + (dy+1)*3 + (dx+1) with (dx,dy,dz) = u - v      */
/* (periodic in x and y; dz = +1 is the next layer down).                   */
/* ------------------------------------------------------------------------ */

/* Weights of point p of a characteristic with M points for operator op.
   p = 0 is the entry half-segment: I_0 = I_bc ex_0 + b_0 S_0. */
static void orc_point_op(int op, int M, const double *tau, int p, double *ex, double *a, double *b, double *g)
{
    if (p == 0) {
        double D0 = 0.5 * tau[0];
        *ex = exp(-D0);
        *a = 0.0;
        *b = -expm1(-D0);
        *g = 0.0;
        return;
    }
    int last = (p == M - 1);
    double D = 0.5 * (tau[p - 1] + tau[p]);
    double Dp = last ? 0.0 : 0.5 * (tau[p] + tau[p + 1]);
    *ex = exp(-D);
    if (op == ORC_LSTAR_PARABOLIC) {
        orc_weights(D, Dp, last, a, b, g);
        return;
    }
    if (D > 0.0) {
        double e0, e1, e2;
        orc_moments(D, &e0, &e1, &e2);
        *a = e0 - e1 / D;
        *b = e1 / D;
    } else {
        *a = 0.0;
        *b = 0.0;
    }
    *g = 0.0;
}

/* Formal solution of operator op along one characteristic (I only). */
void orc_ray_op(int op, int M, const double *tau, const double *S, double I_bc, double *I)
{
    for (int p = 0; p < M; p++) {
        double ex, a, b, g;
        orc_point_op(op, M, tau, p, &ex, &a, &b, &g);
        if (p == 0) {
            I[0] = I_bc * ex + b * S[0];
        } else {
            double Sn = (p + 1 < M) ? S[p + 1] : 0.0;
            I[p] = I[p - 1] * ex + a * S[p - 1] + b * S[p] + g * Sn;
        }
    }
}

/* J = Lambda_op S + boundary term on the periodic box (single thread; used
   on small grids to build operator columns). */
int orc_fs_box_op(int Nx, int Ny, int Nz, int n_mu, int n_phi, const double *chi, const double *S,
                  double I_top, double I_bot, int op, double *J)
{
    int ndir = n_mu * n_phi;
    long nvox = (long)Nx * Ny * Nz;
    double *mu = (double *)malloc(sizeof(double) * ndir);
    double *ph = (double *)malloc(sizeof(double) * ndir);
    double *w = (double *)malloc(sizeof(double) * ndir);
    double *num = (double *)malloc(sizeof(double) * nvox);
    double *den = (double *)malloc(sizeof(double) * nvox);
    orc_quadrature(n_mu, n_phi, mu, ph, w);
    memset(J, 0, sizeof(double) * nvox);
    int err = 0;
    for (int d = 0; d < ndir && !err; d++) {
        double n3[3];
        orc_direction_vector(mu[d], ph[d], n3);
        orc_path p;
        if (orc_make_path(Nz, n3, &p) <= 0) {
            err = -2;
            orc_free_path(&p);
            break;
        }
        int M = p.M;
        double *tau = (double *)malloc(sizeof(double) * M);
        double *Sv = (double *)malloc(sizeof(double) * M);
        double *I = (double *)malloc(sizeof(double) * M);
        long *vid = (long *)malloc(sizeof(long) * M);
        memset(num, 0, sizeof(double) * nvox);
        memset(den, 0, sizeof(double) * nvox);
        for (int y0 = 0; y0 < Ny; y0++)
            for (int x0 = 0; x0 < Nx; x0++) {
                for (int m = 0; m < M; m++) {
                    long v = ((long)p.kk[m] * Ny + wrap(y0 + p.dj[m], Ny)) * Nx + wrap(x0 + p.di[m], Nx);
                    vid[m] = v;
                    tau[m] = chi[v] * p.s[m];
                    Sv[m] = S[v];
                }
                orc_ray_op(op, M, tau, Sv, (mu[d] < 0.0) ? I_top : I_bot, I);
                for (int m = 0; m < M; m++) {
                    num[vid[m]] += p.s[m] * I[m];
                    den[vid[m]] += p.s[m];
                }
            }
        for (long v = 0; v < nvox; v++)
            if (den[v] > 0.0) J[v] += w[d] * num[v] / den[v];
        free(tau); free(Sv); free(I); free(vid);
        orc_free_path(&p);
    }
    free(num); free(den); free(mu); free(ph); free(w);
    return err;
}

/* Nearest-neighbour Lambda* of operator op: out[c * nvox + v], c as above. */
int orc_lstar_stencil_box(int Nx, int Ny, int Nz, int n_mu, int n_phi, const double *chi, int op, double *out,
                          int nthreads)
{
    int ndir = n_mu * n_phi;
    long nvox = (long)Nx * Ny * Nz;
    double *mu = (double *)malloc(sizeof(double) * ndir);
    double *ph = (double *)malloc(sizeof(double) * ndir);
    double *w = (double *)malloc(sizeof(double) * ndir);
    orc_quadrature(n_mu, n_phi, mu, ph, w);
    memset(out, 0, sizeof(double) * 27 * nvox);
    if (nthreads <= 0) nthreads = 1;
    double *acc = (double *)calloc((size_t)nthreads * 27 * nvox, sizeof(double));
    int err = 0;
#pragma omp parallel num_threads(nthreads)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *num = (double *)malloc(sizeof(double) * 27 * nvox);
        double *den = (double *)malloc(sizeof(double) * nvox);
        double *mine = acc + (size_t)tid * 27 * nvox;
#pragma omp for schedule(static, 1)
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
            double *ex = (double *)malloc(sizeof(double) * M);
            double *wa = (double *)malloc(sizeof(double) * M);
            double *wb = (double *)malloc(sizeof(double) * M);
            double *wg = (double *)malloc(sizeof(double) * M);
            long *vid = (long *)malloc(sizeof(long) * M);
            memset(num, 0, sizeof(double) * 27 * nvox);
            memset(den, 0, sizeof(double) * nvox);
            for (int y0 = 0; y0 < Ny; y0++)
                for (int x0 = 0; x0 < Nx; x0++) {
                    for (int m = 0; m < M; m++) {
                        long v = ((long)p.kk[m] * Ny + wrap(y0 + p.dj[m], Ny)) * Nx + wrap(x0 + p.di[m], Nx);
                        vid[m] = v;
                        tau[m] = chi[v] * p.s[m];
                    }
                    for (int q = 0; q < M; q++) orc_point_op(op, M, tau, q, &ex[q], &wa[q], &wb[q], &wg[q]);
                    for (int m = 0; m < M; m++) {
                        den[vid[m]] += p.s[m];
                        for (int j = -1; j <= 3; j++) {
                            int u = m - j; /* point whose voxel carries the S */
                            if (u < 0 || u >= M) continue;
                            int dx = p.di[u] - p.di[m], dy = p.dj[u] - p.dj[m], dz = p.kk[u] - p.kk[m];
                            if (dx < -1 || dx > 1 || dy < -1 || dy > 1 || dz < -1 || dz > 1) continue;
                            /* dI_m/dS_u: updates of points u-1, u, u+1 (those up to m) */
                            double coef = 0.0;
                            for (int q = (u > 0 ? u - 1 : 0); q <= m && q <= u + 1; q++) {
                                double wq = (q == u + 1) ? wa[q] : (q == u) ? wb[q] : wg[q];
                                double att = 1.0;
                                for (int r = q + 1; r <= m; r++) att *= ex[r];
                                coef += wq * att;
                            }
                            int c = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
                            num[(size_t)c * nvox + vid[m]] += p.s[m] * coef;
                        }
                    }
                }
            for (int c = 0; c < 27; c++)
                for (long v = 0; v < nvox; v++)
                    if (den[v] > 0.0) mine[(size_t)c * nvox + v] += w[d] * num[(size_t)c * nvox + v] / den[v];
            free(tau); free(ex); free(wa); free(wb); free(wg); free(vid);
            orc_free_path(&p);
        }
        free(num); free(den);
    }
    for (int t = 0; t < nthreads; t++)
        for (long i = 0; i < 27 * nvox; i++) out[i] += acc[(size_t)t * 27 * nvox + i];
    free(acc); free(mu); free(ph); free(w);
    return err;
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

/* ======================================================================== */
/* Spherical grid (Sec. 3.2: r, theta, phi voxels around a core).           */
/* Reading: voxels are bounded by spheres r_i = rc + i (ro-rc)/Nr, cones    */
/* theta_k = k pi/Nt and half-planes phi_j = 2 pi j/Np; index              */
/* v = (ip*Nt + it)*Nr + ir (r fastest).  Rays of one direction: a square   */
/* lattice of spacing h on the plane through the origin normal to n, axes   */
/* e1 = normalise(z x n) (x if n is parallel to z), e2 = n x e1, lattice    */
/* points with |p| < ro; then, in voxel order, one ray through the centre   */
/* of every voxel no ray has visited yet.  A ray meeting the core (|p| <   */
/* rc) gives two characteristics: inward to the core surface, and outward   */
/* from it.  Crossings are collected, sorted and merged as on the box, and  */
/* each segment is located by its midpoint.                                 */
/* ======================================================================== */
typedef struct {
    int Nr, Nt, Np;
    double rc, ro;
} orc_sph;

static void orc_sph_locate(const orc_sph *g, const double *x, int *ir, int *it, int *ip)
{
    double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    double th = acos(fmax(-1.0, fmin(1.0, x[2] / r)));
    double ph = atan2(x[1], x[0]);
    if (ph < 0.0) ph += 2.0 * M_PI;
    int a = (int)floor((r - g->rc) / (g->ro - g->rc) * g->Nr);
    int b = (int)floor(th / M_PI * g->Nt);
    int c = (int)floor(ph / (2.0 * M_PI) * g->Np);
    *ir = a < 0 ? 0 : (a >= g->Nr ? g->Nr - 1 : a);
    *it = b < 0 ? 0 : (b >= g->Nt ? g->Nt - 1 : b);
    *ip = c < 0 ? 0 : (c >= g->Np ? g->Np - 1 : c);
}

/* Crossings of the line p + t n (p.n = 0, |n| = 1) with every voxel
   boundary, restricted to (t0, t1).  Returns the count written to tc. */
static int orc_sph_crossings(const orc_sph *g, const double *p, const double *n, double t0, double t1,
                             double *tc, int cap)
{
    int m = 0;
    double pp = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
#define PUSH(t_) do { double tt_ = (t_); if (tt_ > t0 && tt_ < t1 && m < cap) tc[m++] = tt_; } while (0)
    for (int i = 1; i < g->Nr; i++) {
        double r = g->rc + i * (g->ro - g->rc) / g->Nr;
        double q = r * r - pp;
        if (q > 0.0) { double s = sqrt(q); PUSH(-s); PUSH(s); }
    }
    for (int k = 1; k < g->Nt; k++) {
        double th = k * M_PI / g->Nt;
        double c = cos(th);
        if (2 * k == g->Nt) {                 /* equatorial plane */
            if (n[2] != 0.0) PUSH(-p[2] / n[2]);
            continue;
        }
        double c2 = c * c;
        double A = n[2] * n[2] - c2, Bq = 2.0 * p[2] * n[2], C = p[2] * p[2] - c2 * pp;
        double roots[2];
        int nr = 0;
        if (fabs(A) < 1e-300) {
            if (Bq != 0.0) roots[nr++] = -C / Bq;
        } else {
            double disc = Bq * Bq - 4.0 * A * C;
            if (disc >= 0.0) {
                double sq = sqrt(disc);
                roots[nr++] = (-Bq - sq) / (2.0 * A);
                roots[nr++] = (-Bq + sq) / (2.0 * A);
            }
        }
        for (int q = 0; q < nr; q++) {
            double z = p[2] + roots[q] * n[2];
            if ((z > 0.0) == (c > 0.0)) PUSH(roots[q]);   /* the cone's own nappe */
        }
    }
    for (int j = 0; j < g->Np; j++) {
        double ph = 2.0 * M_PI * j / g->Np;
        double cs = cos(ph), sn = sin(ph);
        double den = -sn * n[0] + cs * n[1];
        if (den == 0.0) continue;
        double t = (sn * p[0] - cs * p[1]) / den;
        double x = p[0] + t * n[0], y = p[1] + t * n[1];
        if (cs * x + sn * y > 0.0) PUSH(t);       /* the half-plane, not its mirror */
    }
#undef PUSH
    return m;
}

/* One characteristic from ta to tb: segments (voxel, length, start) in order. */
static int orc_sph_segments(const orc_sph *g, const double *p, const double *n, double ta, double tb,
                            int *vox, double *s, double *t0s, int cap, double *tc, int tcap)
{
    int nc = orc_sph_crossings(g, p, n, ta, tb, tc, tcap);
    qsort(tc, (size_t)nc, sizeof(double), cmp_double);
    double prev = ta;
    int m = 0;
    for (int i = 0; i <= nc; i++) {
        double t = (i < nc) ? tc[i] : tb;
        if (t - prev > ORC_TIE * (fabs(prev) + 1.0)) {
            if (m >= cap) return -1;
            double tm = 0.5 * (prev + t), x[3];
            for (int a = 0; a < 3; a++) x[a] = p[a] + tm * n[a];
            int ir, it, ip;
            orc_sph_locate(g, x, &ir, &it, &ip);
            vox[m] = (ip * g->Nt + it) * g->Nr + ir;
            s[m] = t - prev;
            t0s[m] = prev - ta;
            m++;
            prev = t;
        }
    }
    return m;
}

static void orc_sph_frame(const double *n, double *e1, double *e2)
{
    double a[3] = {-n[1], n[0], 0.0};          /* z x n */
    double l = sqrt(a[0] * a[0] + a[1] * a[1]);
    if (l < 1e-12) { a[0] = 1.0; a[1] = 0.0; l = 1.0; }
    e1[0] = a[0] / l; e1[1] = a[1] / l; e1[2] = 0.0;
    e2[0] = n[1] * e1[2] - n[2] * e1[1];
    e2[1] = n[2] * e1[0] - n[0] * e1[2];
    e2[2] = n[0] * e1[1] - n[1] * e1[0];
}

/* Lattice spacing: median over voxels of the cube root of the voxel volume. */
static int cmp_dbl_asc(const void *a, const void *b) { return cmp_double(a, b); }
double orc_sph_spacing(int Nr, int Nt, int Np, double rc, double ro)
{
    int nv = Nr * Nt;
    double *v = (double *)malloc(sizeof(double) * nv);
    for (int it = 0; it < Nt; it++)
        for (int ir = 0; ir < Nr; ir++) {
            double r0 = rc + ir * (ro - rc) / Nr, r1 = rc + (ir + 1) * (ro - rc) / Nr;
            double c0 = cos(it * M_PI / Nt), c1 = cos((it + 1) * M_PI / Nt);
            double vol = (r1 * r1 * r1 - r0 * r0 * r0) / 3.0 * (c0 - c1) * (2.0 * M_PI / Np);
            v[it * Nr + ir] = cbrt(vol);
        }
    qsort(v, (size_t)nv, sizeof(double), cmp_dbl_asc);
    double h = (nv % 2) ? v[nv / 2] : 0.5 * (v[nv / 2 - 1] + v[nv / 2]);
    free(v);
    return h;
}

/*
 * Rays of one direction.  Writes, for every characteristic c: its start
 * point offset (foot point p and [ta, tb]), kind (0 = enters from outside,
 * 1 = leaves the core) and the entry point's position for boundary
 * intensities.  Returns the number of characteristics, or -1 (cap).
 *   chars: [c][8] = p0,p1,p2, ta, tb, kind, 0, 0
 */
int orc_sph_rays(int Nr, int Nt, int Np, double rc, double ro, double h, const double *n, int cap, double *chars)
{
    orc_sph g = {Nr, Nt, Np, rc, ro};
    int nvox = Nr * Nt * Np;
    unsigned char *seen = (unsigned char *)calloc((size_t)nvox, 1);
    int tcap = 4 * (Nr + Nt + Np) + 16, scap = tcap + 4;
    double *tc = (double *)malloc(sizeof(double) * tcap);
    int *vox = (int *)malloc(sizeof(int) * scap);
    double *s = (double *)malloc(sizeof(double) * scap), *t0s = (double *)malloc(sizeof(double) * scap);
    double e1[3], e2[3];
    orc_sph_frame(n, e1, e2);
    int nc = 0, K = (int)ceil(ro / h) + 1;
    /* p enumerates the lattice, then fill-in foot points */
    for (int pass = 0; pass < 2; pass++) {
        int nitems = pass == 0 ? (2 * K + 1) * (2 * K + 1) : nvox;
        for (int q = 0; q < nitems; q++) {
            double p[3];
            if (pass == 0) {
                int a = q / (2 * K + 1) - K, b = q % (2 * K + 1) - K;
                for (int k = 0; k < 3; k++) p[k] = a * h * e1[k] + b * h * e2[k];
            } else {
                if (seen[q]) continue;
                int ir = q % Nr, it = (q / Nr) % Nt, ip = q / (Nr * Nt);
                double r = rc + (ir + 0.5) * (ro - rc) / Nr, th = (it + 0.5) * M_PI / Nt, ph = (ip + 0.5) * 2.0 * M_PI / Np;
                double c[3] = {r * sin(th) * cos(ph), r * sin(th) * sin(ph), r * cos(th)};
                double cn = c[0] * n[0] + c[1] * n[1] + c[2] * n[2];
                for (int k = 0; k < 3; k++) p[k] = c[k] - cn * n[k];
            }
            double pp = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
            if (!(pp < ro * ro)) continue;
            double to = sqrt(ro * ro - pp);
            double seg[2][3];
            int nseg = 0;
            if (pp < rc * rc) {
                double ti = sqrt(rc * rc - pp);
                seg[nseg][0] = -to; seg[nseg][1] = -ti; seg[nseg][2] = 0; nseg++;
                seg[nseg][0] = ti; seg[nseg][1] = to; seg[nseg][2] = 1; nseg++;
            } else {
                seg[nseg][0] = -to; seg[nseg][1] = to; seg[nseg][2] = 0; nseg++;
            }
            for (int k = 0; k < nseg; k++) {
                int M = orc_sph_segments(&g, p, n, seg[k][0], seg[k][1], vox, s, t0s, scap, tc, tcap);
                if (M <= 0) continue;
                if (nc >= cap) { nc = -1; goto done; }
                double *cc = chars + 8 * (size_t)nc;
                cc[0] = p[0]; cc[1] = p[1]; cc[2] = p[2];
                cc[3] = seg[k][0]; cc[4] = seg[k][1]; cc[5] = seg[k][2]; cc[6] = 0; cc[7] = 0;
                nc++;
                for (int m = 0; m < M; m++) seen[vox[m]] = 1;
            }
        }
    }
done:
    free(seen); free(tc); free(vox); free(s); free(t0s);
    return nc;
}

/* Segments of one characteristic (for tests and the formal solution). */
int orc_sph_char(int Nr, int Nt, int Np, double rc, double ro, const double *ch, const double *n, int cap,
                 int *vox, double *s, double *t0s)
{
    orc_sph g = {Nr, Nt, Np, rc, ro};
    int tcap = 4 * (Nr + Nt + Np) + 16;
    double *tc = (double *)malloc(sizeof(double) * tcap);
    int M = orc_sph_segments(&g, ch, n, ch[3], ch[4], vox, s, t0s, cap, tc, tcap);
    free(tc);
    return M;
}

/* Boundary intensity of a characteristic entering from outside, from a point
   source on the +z axis at distance dsrc*ro: the discrete inward direction
   closest to the light's direction at the entry point receives
   J_inc/w with J_inc = B_sub (ro (dsrc-1))^2 / |x - x_src|^2 (= B_sub at the
   sub-source point); lit points only.  Returns the intensity for direction d. */
double orc_sph_irradiation(int n_mu, int n_phi, int d, const double *x, double ro, double dsrc, double B_sub)
{
    if (dsrc <= 1.0) return 0.0;
    double xs[3] = {0.0, 0.0, dsrc * ro};
    double u[3] = {x[0] - xs[0], x[1] - xs[1], x[2] - xs[2]};
    double L = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    for (int k = 0; k < 3; k++) u[k] /= L;
    if (u[0] * x[0] + u[1] * x[1] + u[2] * x[2] >= 0.0) return 0.0;   /* not lit */
    int ndir = n_mu * n_phi, best = -1;
    double bestdot = -2.0;
    for (int q = 0; q < ndir; q++) {
        int i = q / n_phi, j = q % n_phi;
        double mu = -1.0 + (2.0 * i + 1.0) / n_mu, ph = 2.0 * M_PI * (j + 0.5) / n_phi, v[3];
        orc_direction_vector(mu, ph, v);
        double dot = v[0] * u[0] + v[1] * u[1] + v[2] * u[2];
        if (dot > bestdot) { bestdot = dot; best = q; }
    }
    if (best != d) return 0.0;
    double w = 1.0 / ((double)n_mu * n_phi);
    double Jinc = B_sub * (ro * (dsrc - 1.0)) * (ro * (dsrc - 1.0)) / (L * L);
    return Jinc / w;
}

/*
 * Formal solution on the spherical grid: J and Lambda* for source S and
 * opacity chi ([ip][it][ir]).  Characteristics entering from outside start
 * with I_out + irradiation; those leaving the core start with the core
 * intensity B of their first voxel (Bv).
 */
int orc_fs_sphere(int Nr, int Nt, int Np, double rc, double ro, int n_mu, int n_phi, double dsrc, double B_sub,
                  const double *chi, const double *S, const double *Bv, double I_out, int lstar_kind,
                  double *J, double *lstar, int nthreads)
{
    int ndir = n_mu * n_phi;
    long nvox = (long)Nr * Nt * Np;
    double h = orc_sph_spacing(Nr, Nt, Np, rc, ro);
    memset(J, 0, sizeof(double) * nvox);
    if (lstar) memset(lstar, 0, sizeof(double) * nvox);
    if (nthreads <= 0) nthreads = 1;
    double *Jt = (double *)calloc((size_t)nthreads * nvox, sizeof(double));
    double *Lt = (double *)calloc((size_t)nthreads * nvox, sizeof(double));
    int err = 0;
    int K = (int)ceil(ro / h) + 1;
    int cap = 2 * ((2 * K + 1) * (2 * K + 1) + (int)nvox) + 16;
#pragma omp parallel num_threads(nthreads)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *num = (double *)malloc(sizeof(double) * nvox), *den = (double *)malloc(sizeof(double) * nvox);
        double *lnum = (double *)malloc(sizeof(double) * nvox);
        double *chars = (double *)malloc(sizeof(double) * 8 * (size_t)cap);
        int scap = 4 * (Nr + Nt + Np) + 20;
        int *vox = (int *)malloc(sizeof(int) * scap);
        double *s = (double *)malloc(sizeof(double) * scap), *t0s = (double *)malloc(sizeof(double) * scap);
        double *tau = (double *)malloc(sizeof(double) * scap), *Sv = (double *)malloc(sizeof(double) * scap);
        double *I = (double *)malloc(sizeof(double) * scap), *dd = (double *)malloc(sizeof(double) * scap);
#pragma omp for schedule(static, 1)
        for (int d = 0; d < ndir; d++) {
            int i = d / n_phi, j = d % n_phi;
            double mu = -1.0 + (2.0 * i + 1.0) / n_mu, ph = 2.0 * M_PI * (j + 0.5) / n_phi, n[3];
            orc_direction_vector(mu, ph, n);
            double w = 1.0 / ((double)n_mu * n_phi);
            int nc = orc_sph_rays(Nr, Nt, Np, rc, ro, h, n, cap, chars);
            if (nc < 0) {
#pragma omp atomic write
                err = -3;
                continue;
            }
            memset(num, 0, sizeof(double) * nvox);
            memset(den, 0, sizeof(double) * nvox);
            memset(lnum, 0, sizeof(double) * nvox);
            for (int c = 0; c < nc; c++) {
                const double *ch = chars + 8 * (size_t)c;
                int M = orc_sph_char(Nr, Nt, Np, rc, ro, ch, n, scap, vox, s, t0s);
                if (M <= 0) continue;
                for (int m = 0; m < M; m++) { tau[m] = chi[vox[m]] * s[m]; Sv[m] = S[vox[m]]; }
                double Ibc;
                if (ch[5] == 1.0) {
                    Ibc = Bv[vox[0]];
                } else {
                    double x[3];
                    for (int k = 0; k < 3; k++) x[k] = ch[k] + ch[3] * n[k];
                    Ibc = I_out + orc_sph_irradiation(n_mu, n_phi, d, x, ro, dsrc, B_sub);
                }
                orc_ray(M, tau, Sv, Ibc, lstar_kind, I, dd);
                for (int m = 0; m < M; m++) {
                    num[vox[m]] += s[m] * I[m];
                    den[vox[m]] += s[m];
                    lnum[vox[m]] += s[m] * dd[m];
                }
            }
            double *Jm = Jt + (size_t)tid * nvox, *Lm = Lt + (size_t)tid * nvox;
            for (long v = 0; v < nvox; v++) {
                if (den[v] > 0.0) { Jm[v] += w * num[v] / den[v]; Lm[v] += w * lnum[v] / den[v]; }
            }
        }
        free(num); free(den); free(lnum); free(chars); free(vox); free(s); free(t0s);
        free(tau); free(Sv); free(I); free(dd);
    }
    for (int t = 0; t < nthreads; t++)
        for (long v = 0; v < nvox; v++) {
            J[v] += Jt[(size_t)t * nvox + v];
            if (lstar) lstar[v] += Lt[(size_t)t * nvox + v];
        }
    free(Jt); free(Lt);
    return err;
}

/*
 * Nearest-neighbour Lambda* of operator op on the spherical grid:
 * out[c * nvox + v], c = (dp+1)*9 + (dt+1)*3 + (dr+1) for the neighbour
 * u = (ir+dr, it+dt, ip+dp) of v = (ir, it, ip) (phi periodic, r and theta
 * not; Np >= 3).  As on the box, a point m of a characteristic takes
 * dI_m/dS at the points m+1 .. m-3 of the same characteristic whose voxel is
 * such a neighbour (Sec. 2: the paper's non-local operator), weighted like
 * the formal solution's voxel average (s_m over the sum of s of the voxel's
 * visits in that direction).  Points further upstream that still lie in a
 * neighbour (possible where voxels are small against the ray spacing) and
 * neighbours across the pole are not indices of this stencil.
 */
int orc_lstar_stencil_sphere(int Nr, int Nt, int Np, double rc, double ro, int n_mu, int n_phi, const double *chi,
                             int op, double *out, int nthreads)
{
    if (Np < 3) return -4;
    int ndir = n_mu * n_phi;
    long nvox = (long)Nr * Nt * Np;
    double h = orc_sph_spacing(Nr, Nt, Np, rc, ro);
    memset(out, 0, sizeof(double) * 27 * nvox);
    if (nthreads <= 0) nthreads = 1;
    double *acc = (double *)calloc((size_t)nthreads * 27 * nvox, sizeof(double));
    int err = 0;
    int K = (int)ceil(ro / h) + 1;
    int cap = 2 * ((2 * K + 1) * (2 * K + 1) + (int)nvox) + 16;
#pragma omp parallel num_threads(nthreads)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *num = (double *)malloc(sizeof(double) * 27 * nvox);
        double *den = (double *)malloc(sizeof(double) * nvox);
        double *mine = acc + (size_t)tid * 27 * nvox;
        double *chars = (double *)malloc(sizeof(double) * 8 * (size_t)cap);
        int scap = 4 * (Nr + Nt + Np) + 20;
        int *vox = (int *)malloc(sizeof(int) * scap);
        double *s = (double *)malloc(sizeof(double) * scap), *t0s = (double *)malloc(sizeof(double) * scap);
        double *tau = (double *)malloc(sizeof(double) * scap);
        double *ex = (double *)malloc(sizeof(double) * scap), *wa = (double *)malloc(sizeof(double) * scap);
        double *wb = (double *)malloc(sizeof(double) * scap), *wg = (double *)malloc(sizeof(double) * scap);
#pragma omp for schedule(static, 1)
        for (int d = 0; d < ndir; d++) {
            int i = d / n_phi, j = d % n_phi;
            double mu = -1.0 + (2.0 * i + 1.0) / n_mu, ph = 2.0 * M_PI * (j + 0.5) / n_phi, n[3];
            orc_direction_vector(mu, ph, n);
            double w = 1.0 / ((double)n_mu * n_phi);
            int nc = orc_sph_rays(Nr, Nt, Np, rc, ro, h, n, cap, chars);
            if (nc < 0) {
#pragma omp atomic write
                err = -3;
                continue;
            }
            memset(num, 0, sizeof(double) * 27 * nvox);
            memset(den, 0, sizeof(double) * nvox);
            for (int c = 0; c < nc; c++) {
                int M = orc_sph_char(Nr, Nt, Np, rc, ro, chars + 8 * (size_t)c, n, scap, vox, s, t0s);
                if (M <= 0) continue;
                for (int m = 0; m < M; m++) tau[m] = chi[vox[m]] * s[m];
                for (int q = 0; q < M; q++) orc_point_op(op, M, tau, q, &ex[q], &wa[q], &wb[q], &wg[q]);
                for (int m = 0; m < M; m++) {
                    den[vox[m]] += s[m];
                    int irm = vox[m] % Nr, itm = (vox[m] / Nr) % Nt, ipm = vox[m] / (Nr * Nt);
                    for (int jj = -1; jj <= 3; jj++) {
                        int u = m - jj;
                        if (u < 0 || u >= M) continue;
                        int dr = vox[u] % Nr - irm, dt = (vox[u] / Nr) % Nt - itm;
                        int dp = wrap(vox[u] / (Nr * Nt) - ipm, Np);
                        dp = dp == Np - 1 ? -1 : dp;
                        if (dr < -1 || dr > 1 || dt < -1 || dt > 1 || dp < -1 || dp > 1) continue;
                        double coef = 0.0;
                        for (int q = (u > 0 ? u - 1 : 0); q <= m && q <= u + 1; q++) {
                            double wq = (q == u + 1) ? wa[q] : (q == u) ? wb[q] : wg[q];
                            double att = 1.0;
                            for (int r = q + 1; r <= m; r++) att *= ex[r];
                            coef += wq * att;
                        }
                        int cc = (dp + 1) * 9 + (dt + 1) * 3 + (dr + 1);
                        num[(size_t)cc * nvox + vox[m]] += s[m] * coef;
                    }
                }
            }
            for (int cc = 0; cc < 27; cc++)
                for (long v = 0; v < nvox; v++)
                    if (den[v] > 0.0) mine[(size_t)cc * nvox + v] += w * num[(size_t)cc * nvox + v] / den[v];
        }
        free(num); free(den); free(chars); free(vox); free(s); free(t0s); free(tau);
        free(ex); free(wa); free(wb); free(wg);
    }
    for (int t = 0; t < nthreads; t++)
        for (long i2 = 0; i2 < 27 * nvox; i2++) out[i2] += acc[(size_t)t * 27 * nvox + i2];
    free(acc);
    return err;
}
