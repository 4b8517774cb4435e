/*
 * rt3d.h -- C ABI of the MI355X (gfx950) library for the 3D radiative
 * transfer formal solution and its operator-splitting (ALI) iteration.
 *
 * Method: P. H. Hauschildt & E. Baron, "A 3D radiative transfer framework.
 * XII. Many-core, vector and GPU methods" (arXiv 2102.01734):
 *   - static transfer equation n.grad I = eta - chi I, S = eta/chi      (Sec. 2.1, eq. 1)
 *   - formal solution J = Lambda S along characteristics for all solid
 *     angles, with the approximate operator Lambda*                      (Sec. 2.2 eq. frmsol; Sec. 4)
 *   - per-point steps: gather previous/next S and chi, optical steps,
 *     interpolation weights, boundary/vacuum fix-up, Lambda* data,
 *     Delta I and exp(-dtau)                                            (Listing 1, steps 0-5)
 *   - operator splitting [1 - Lambda*(1-eps)] J_new = J_fs - Lambda*(1-eps) J_old,
 *     S = (1-eps) J + eps B                                             (Sec. 2.2, eq. alo)
 *   - geometry (tracker) computed once and reused for every wavelength  (Sec. 4.1)
 *
 * Conventions shared by every entry point:
 *   - Box grid: cubic voxels of unit edge, Nx x Ny x Nz voxels, periodic in
 *     x and y.  Layer k = 0 is the top (outer boundary, z max), k = Nz-1 the
 *     bottom (inner boundary).  Field arrays are structure-of-arrays,
 *     [lambda][k][y][x], x fastest, contiguous, one value per voxel.
 *   - Spherical grid (Sec. 3.2): Nr x Ntheta x Nphi voxels between the core
 *     radius r_core and the outer radius r_out, bounded by the spheres
 *     r_i = r_core + i (r_out - r_core)/Nr, the cones theta_k = k pi/Ntheta
 *     and the half-planes phi_j = 2 pi j/Nphi.  Voxel index
 *     v = (iphi Ntheta + itheta) Nr + ir (r fastest); field arrays are
 *     [lambda][v].  The core is opaque: characteristics that hit it end
 *     there, characteristics leaving it start with I_core.  Characteristics
 *     entering through r_out start with I_out plus, optionally, the
 *     irradiation of a point source on the +z axis.
 *   - Directions: n_mu x n_phi, mu_i = -1 + (2i+1)/n_mu, phi_j = 2 pi (j+1/2)/n_phi,
 *     equal weights 1/(n_mu n_phi) (Sec. 3.1: equally spaced in mu and phi).
 *   - Precision: RT_FP64 grids take double fields and compute the formal
 *     solution in double.  RT_FP32 grids take float fields, run the formal
 *     solution recurrence and J accumulation in float, and keep the optical
 *     steps, interpolation weights and all ALI state (J, S, Ng, norms) in
 *     double.
 *   - Pointers marked "device" are HIP device pointers (e.g. from
 *     torch.Tensor.data_ptr()); the caller allocates and owns them and the
 *     library never frees them.  The grid handle owns its geometry tables,
 *     partial-sum buffers and scratch; rt_destroy_grid frees all of them.
 *   - stream: a hipStream_t cast to void* (NULL = the default stream).  Work is
 *     enqueued asynchronously on it unless stated otherwise.  Part of a call's
 *     work may run on a stream the grid owns (the nearest-neighbour Lambda*
 *     build of an ALI step): it starts after the work enqueued on `stream`
 *     before the call, and work enqueued on `stream` after the call waits
 *     for it, as if it had been enqueued on `stream` itself.
 *   - Device: a grid belongs to the device that is current when it is
 *     created; make that device current for every call on the grid.
 *   - Errors: every call returns an rt_status; arguments are validated before
 *     anything is launched.  rt_last_error() returns a message for the most
 *     recent failure on the calling thread.  A handle must not be used from two
 *     threads at once; different handles are independent.
 */
#ifndef RT3D_H
#define RT3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RT_OK = 0,
    RT_E_INVALID = 1,       /* bad argument or descriptor                      */
    RT_E_NOMEM = 2,         /* device allocation failed                        */
    RT_E_HIP = 3,           /* a HIP runtime call failed                       */
    RT_E_NOT_CONVERGED = 4, /* rt_solve reached max_iter; state stays valid    */
    RT_E_NUMERIC = 5,       /* NaN or Inf met in the iteration                 */
    RT_E_UNSUPPORTED = 6    /* valid request the library cannot serve          */
} rt_status;

typedef enum { RT_GEOM_BOX_PERIODIC_XY = 0, RT_GEOM_SPHERICAL = 1 } rt_geom;
typedef enum { RT_FP64 = 0, RT_FP32 = 1 } rt_prec;

/* rt_grid_desc.flags */
#define RT_F_LSTAR_PARABOLIC 0x1u /* Lambda* = exact diagonal of the parabolic
                                     formal solution; default: diagonal of the
                                     linear-interpolation operator            */
#define RT_F_BAND_TILES 0x2u      /* box: accumulate J / Lambda* of a workgroup
                                     in a band of rows of the layer instead of
                                     the whole layer.  Used by itself for layers
                                     whose tile does not fit the LDS of a CU
                                     (e.g. 257 x 257), or fits only with
                                     kernels that spill registers (e.g.
                                     129 x 129); the flag forces it for any box
                                     grid (results differ only in the
                                     summation order).  Single-precision band
                                     tiles of J-only or Lambda*-only sweeps
                                     are two layer rows wide (twice the LDS
                                     per row), so that no ray's column wraps. */
#define RT_F_LSTAR_NONLOCAL 0x4u  /* box or sphere (Nphi >= 3, geometry cache
                                     in device memory): the ALI uses the
                                     nearest-neighbour
                                     Lambda* (Sec. 2, Sec. 3: the non-local
                                     operator of the paper's runs) -- the
                                     operator selected by RT_F_LSTAR_PARABOLIC
                                     restricted to the 27 neighbours of each
                                     voxel (see rt_lstar_stencil) -- and solves
                                     the operator-splitting system with Jacobi
                                     or Gauss-Seidel sweeps
                                     (rt_solve_opts.os_sweeps, os_method).  The
                                     state's lstar array still receives the
                                     diagonal; on box grids it is the
                                     stencil's centre component (the same
                                     sum; on RT_FP32 grids in the sweep's
                                     float rounding), on spherical grids the
                                     centre also holds the window points of a
                                     characteristic that re-enters the voxel. */
#define RT_F_HOST_CACHE 0x8u      /* sphere: keep every chunk of the geometry
                                     cache in pinned host memory and stream it
                                     to the GPU for each formal solution (the
                                     paper's SmallGPU mode, Sec. 5).  Without
                                     the flag, chunks stay in device memory
                                     while it lasts and only the rest is
                                     streamed.  Streamed grids run their ALI
                                     steps without graph capture.  Results are
                                     bitwise those of a device-resident cache. */

typedef struct rt_grid *rt_grid_t;

typedef struct {
    uint32_t struct_size;  /* sizeof(rt_grid_desc)                              */
    int32_t geom;          /* rt_geom                                           */
    int32_t n[3];          /* box: Nx, Ny, Nz; sphere: Nr, Ntheta, Nphi (>= 1)  */
    double h[3];           /* box: ignored (unit voxels); sphere: r_core, r_out,
                              source distance in units of r_out (> 1, or 0 for
                              no irradiation)                                   */
    int32_t n_mu, n_phi;   /* direction quadrature; n_mu even, n_phi >= 1       */
    int32_t n_lambda_max;  /* largest wavelength batch any call will pass       */
    int32_t prec;          /* rt_prec                                           */
    uint32_t flags;        /* RT_F_*                                            */
} rt_grid_desc;

/*
 * Builds the tracker output on the host in double precision, uploads it once,
 * and sizes the work schedule and partial-sum buffers for up to n_lambda_max
 * wavelengths (Sec. 4.1: the geometry cache is built once and reused for all
 * wavelengths).
 *   box: one characteristic template per direction (every other
 *        characteristic of that direction is an integer translate of it).
 *   sphere: every characteristic of every direction (see rt_sphere_tracks),
 *        traced on up to 16 host threads, with per-visit voxel, path length
 *        and averaging weight (float on RT_FP32 grids, double on RT_FP64),
 *        uploaded in chunks of consecutive directions.
 * Blocks until the upload is complete.  Errors: RT_E_INVALID (descriptor),
 * RT_E_UNSUPPORTED (box layer larger than the on-chip tile allows),
 * RT_E_NOMEM, RT_E_HIP.  *out is NULL on error.
 * RT_E_NOMEM: a box grid whose working set -- geometry, the partial sums of a
 * formal solution with J and Lambda* of n_lambda_max wavelengths, the padded
 * inputs, the ALI state (Ng history, double anchors on RT_FP32 grids) and,
 * with RT_F_LSTAR_NONLOCAL, the stencil -- exceeds the free device memory is
 * refused before anything is allocated; so is a spherical grid with
 * RT_F_LSTAR_NONLOCAL whose geometry cache does not fit device memory.  Every
 * entry point returns RT_E_NOMEM when a device or pinned-host allocation
 * fails later on.
 */
rt_status rt_create_grid(const rt_grid_desc *desc, rt_grid_t *out);

/* Frees every device buffer of the handle (after synchronising its device). */
rt_status rt_destroy_grid(rt_grid_t grid);

/* Read-only facts about a grid.  Any out pointer may be NULL. */
rt_status rt_grid_info(rt_grid_t grid, int64_t *n_vox, int32_t *n_dir,
                       int64_t *n_visits_total, int32_t *n_workgroups);

/*
 * Formal solution J = Lambda S + Lambda_bc (Sec. 2.2 eq. frmsol) and,
 * optionally, the diagonal Lambda* (Sec. 4; Listing 1 step 4b), for n_lambda
 * independent wavelengths on the same grid.
 *   chi, S     device, [n_lambda][Nz][Ny][Nx], grid precision (float/double);
 *              chi >= 0 (chi = 0 marks vacuum: Listing 1 step 4a)
 *   I_bc       device, grid precision; NULL = all zero.  Box: [n_lambda][2],
 *              intensity entering at the top (mu < 0 rays) and at the bottom
 *              (mu > 0 rays).  Sphere: [n_lambda][3] = I_out (entering through
 *              r_out), I_core (leaving the core), J_sub (mean intensity of the
 *              point source at the sub-source point r_out z; each lit entry
 *              point adds J_sub (r_out (d - 1))^2 / |x - x_src|^2 / w to the
 *              quadrature direction closest to the light's direction, ties to
 *              the lower index)
 *   J_out      device, [n_lambda][Nz][Ny][Nx], grid precision
 *   lstar_out  device, same shape, or NULL to skip Lambda*
 * n_lambda = 0 is a no-op.  Deterministic: the same inputs give bitwise the
 * same outputs (fixed summation order, no floating-point atomics across
 * workgroups).  Errors: RT_E_INVALID (NULL pointer, n_lambda out of range),
 * RT_E_HIP.
 */
rt_status rt_formal_solution(rt_grid_t grid, int32_t n_lambda, const void *chi, const void *S,
                             const void *I_bc, void *J_out, void *lstar_out, void *stream);

/*
 * The formal solution over a subset of the directions (box grids): J and
 * Lambda* summed over the listed directions only, i.e. the partial sums one
 * of several GPUs holding those directions would contribute before the
 * all-reduce of J over solid angles (Sec. 4).  Summing the results over
 * disjoint subsets that cover all directions gives rt_formal_solution's
 * output up to the summation order.
 *   dirs  host, n_dirs >= 1 direction indices (i_mu * n_phi + j_phi),
 *         strictly increasing
 * Other arguments and errors as rt_formal_solution; RT_E_UNSUPPORTED on
 * spherical grids.
 */
rt_status rt_formal_solution_dirs(rt_grid_t grid, int32_t n_lambda, const void *chi, const void *S,
                                  const void *I_bc, int32_t n_dirs, const int32_t *dirs, void *J_out,
                                  void *lstar_out, void *stream);

/*
 * Host-side planning of a solid-angle decomposition: directions are dealt,
 * longest characteristic first, to the shard with the fewest visits so far,
 * so shards carry nearly equal work (shallow directions cost up to ~7x the
 * mean).  Writes shard `shard` of `n_shards` (sorted) to dirs_out (host, may
 * be NULL for a size query) and its size to *n_out.  No device work.
 */
rt_status rt_shard_directions(rt_grid_t grid, int32_t n_shards, int32_t shard, int32_t *dirs_out, int32_t *n_out);

/*
 * State of the ALI iteration for a batch of wavelengths.
 * The caller owns every array.  Besides them, a grid keeps scratch that
 * belongs to the state it stepped last: the padded formal-solution inputs,
 * the Ng history (the last four iterates), on RT_FP32 grids the double
 * anchor (S_a, J_a = Lambda S_a + Lambda_bc), and with RT_F_LSTAR_NONLOCAL the
 * nearest-neighbour stencil.  A step on a state whose array pointers or
 * n_lambda differ from those of the previous step (or the first step after
 * a BiCGStab solve on the grid) rebuilds all of it from that state: S from
 * J, a new anchor, the stencil from chi, and an empty Ng history -- the path
 * to the fixed point changes, the fixed point does not.  Several states can
 * therefore share one grid, stepped alternately.  After changing J, chi, eps
 * or B in place between steps, set iter = 0 (and lstar_valid = 0 if chi
 * changed), which restarts the same way.
 */
typedef struct {
    uint32_t struct_size; /* sizeof(rt_state)                                   */
    int32_t n_lambda;     /* 1 .. n_lambda_max                                  */
    const void *chi;      /* device [n_lambda][vox], grid precision             */
    const void *eps;      /* device [n_lambda][vox], grid precision, 0<=eps<=1  */
    const void *B;        /* device [n_lambda][vox], grid precision             */
    const void *I_bc;     /* device [n_lambda][2] (box) or [n_lambda][3]
                             (sphere), grid precision, as in
                             rt_formal_solution; NULL = 0                       */
    double *J;            /* device [n_lambda][vox] double: current iterate;
                             on entry the start value (e.g. B), on exit the
                             result.  Resuming from any J is allowed (iter = 0
                             for a J the library did not write last).           */
    double *S;            /* device [n_lambda][vox] double: S = (1-eps)J + eps B
                             of the returned J (written by the library)         */
    void *lstar;          /* device [n_lambda][vox] grid precision: Lambda*     */
    int32_t lstar_valid;  /* in/out: 0 = compute Lambda* on the next step       */
    int32_t iter;         /* in/out: ALI steps taken since the last restart     */
    double *rel_change;   /* device [n_lambda] double, out: max_v |dJ/J| of the
                             last step (0 for wavelengths already converged)   */
} rt_state;

/* rt_solve_opts.method */
#define RT_SOLVER_ALI 0
#define RT_SOLVER_BICGSTAB 1

typedef struct {
    uint32_t struct_size; /* sizeof(rt_solve_opts)                              */
    double tol;           /* stop when max_v |J_new - J_old|/|J_new| < tol      */
    int32_t max_iter;     /* ALI steps per rt_solve call                        */
    int32_t ng_every;     /* Ng acceleration every k plain steps (0 = off)      */
    int32_t ng_start;     /* first step at which Ng may be applied              */
    int32_t reanchor;     /* FP32 grids: new FP64 anchor once max |dJ/J| has
                             fallen by this factor since the last anchor
                             (0 = library default 100)                          */
    int32_t use_graph;    /* 1: plain steps (no anchor, Ng or Lambda* pass) run
                             as a captured HIP graph, replayed per step; needs
                             a non-NULL stream.  Results are bitwise those of
                             eager launches.                                    */
    int32_t method;       /* rt_solve: RT_SOLVER_ALI (operator splitting with
                             Ng) or RT_SOLVER_BICGSTAB (see rt_solve)           */
    int32_t net_every;    /* rt_solve with a preconditioner network set
                             (rt_set_preconditioner): propose a learned
                             correction after every net_every-th step
                             (0 = never); see rt_set_preconditioner             */
    int32_t os_sweeps;    /* grids with RT_F_LSTAR_NONLOCAL: sweeps of the
                             operator-splitting system per step, started from
                             the diagonal solution (0 = library default 16);
                             ignored otherwise                                  */
    int32_t os_method;    /* those sweeps: RT_OS_JACOBI or RT_OS_GAUSS_SEIDEL
                             (Sec. 3 names both): in place, over 18 colour
                             classes in the order cz*9 + cy*3 + cx with
                             cz = z mod 2, cx = x mod 2, cy = y mod 2, except
                             the last column (row) of an odd periodic axis of
                             length >= 3, which takes class 2.  Voxels of a
                             class share no stencil coupling, so the sweep is
                             the sequential Gauss-Seidel sweep in that voxel
                             order (each class updated in parallel) and is
                             bitwise reproducible.                              */
} rt_solve_opts;

/* rt_solve_opts.os_method */
#define RT_OS_JACOBI 0
#define RT_OS_GAUSS_SEIDEL 1

typedef struct {
    int32_t iters;          /* ALI steps taken by this call                     */
    int32_t n_fs;           /* formal solutions (all precisions)                */
    int32_t n_fs64;         /* of which double-precision anchors                */
    int32_t n_ng;           /* Ng extrapolations applied                        */
    int32_t n_converged;    /* wavelengths below tol at return                  */
    double max_rel_change;  /* max over wavelengths of the last step's change   */
    double seconds;         /* wall time of the call                            */
    int32_t n_net_accept;   /* learned corrections kept (per wavelength)        */
    int32_t n_net_reject;   /* learned corrections rejected (per wavelength)    */
} rt_solve_report;

/*
 * One ALI step (Sec. 2.2 eq. alo with the diagonal Lambda*, or with the
 * nearest-neighbour Lambda* on RT_F_LSTAR_NONLOCAL grids): formal solution
 * of the current S (building Lambda* first when lstar_valid == 0), the
 * operator-splitting update of J (pointwise for the diagonal Lambda*; for the
 * non-local one, J_new = J_old + dJ with dJ from os_sweeps Jacobi or
 * Gauss-Seidel sweeps (os_method) of [1 - Lambda*(1-eps)] dJ = J_fs - J_old),
 * S = (1-eps)J + eps B, the
 * per-wavelength norm max_v |dJ/J| into state->rel_change, and -- when the
 * schedule in opts says so -- the Ng extrapolation of the last four iterates.
 * Asynchronous on `stream`.  For RT_FP32 grids the formal solution of the
 * step is single precision on S - S_anchor; the anchor (a double-precision
 * formal solution) is taken on the first step and refreshed by rt_solve.
 * Errors: RT_E_INVALID, RT_E_HIP.
 */
rt_status rt_ali_step(rt_grid_t grid, rt_state *state, const rt_solve_opts *opts, void *stream);

/*
 * The nearest-neighbour Lambda* of a box grid (Sec. 2, Sec. 3): for each voxel
 * v and each of its 27 neighbours u = v + (dx, dy, dz) (x, y periodic), the
 * part of the operator element Lambda[v][u] that characteristics carry
 * directly from u to v (points at most three apart along a characteristic;
 * on periods longer than a characteristic's horizontal reach within the
 * neighbourhood this is the whole element).  The operator is the
 * linear-interpolation one, or the formal solution itself with
 * RT_F_LSTAR_PARABOLIC; component 13 (the voxel itself) is the diagonal
 * Lambda* of rt_formal_solution.  Elements of neighbours beyond the top or
 * bottom layer are 0.
 *   chi  device [n_lambda][Nz][Ny][Nx], grid precision
 *   out  device [n_lambda][27][Nz][Ny][Nx], grid precision, component
 *        c = (dz+1)*9 + (dy+1)*3 + (dx+1)
 * Spherical grids (Nphi >= 3, geometry cache in device memory): chi
 * [n_lambda][Nphi][Ntheta][Nr], out [n_lambda][27][Nphi][Ntheta][Nr] with
 * c = (dp+1)*9 + (dt+1)*3 + (dr+1) for the neighbour (ir+dr, it+dt, ip+dp),
 * phi periodic, r and theta bounded; a point m of a characteristic takes
 * dI_m/dS at its points m+1 .. m-3 that lie in such a neighbour (further
 * points and neighbours across the pole are not elements of this stencil);
 * one thread per characteristic adds with 64-bit fixed-point atomics.
 * Sums are accumulated in 64-bit fixed point (2^-52), so the result is
 * bitwise reproducible.  Per wavelength and direction, workgroups gather
 * the contributions of bundles of ray rows in LDS and add each target row to
 * device memory once per layer; layers too wide for that (more than 2048
 * voxels a row, or a tile of two rows beyond the LDS), or any grid when the
 * environment variable RT3D_STENCIL_PER_CHARACTERISTIC=1 is set at grid
 * creation, add every contribution to device memory directly.  Both give
 * bitwise the same result.  Asynchronous on `stream`.  Errors: RT_E_INVALID
 * (also Nphi < 3 on a spherical grid), RT_E_UNSUPPORTED (a spherical cache
 * streamed from host memory), RT_E_NOMEM, RT_E_HIP.
 */
rt_status rt_lstar_stencil(rt_grid_t grid, int32_t n_lambda, const void *chi, void *out, void *stream);

/*
 * RT_SOLVER_ALI: runs ALI steps until every wavelength has max_v |dJ/J| < tol
 * or max_iter steps were taken.  Wavelengths that converge drop out of later
 * steps.
 * RT_SOLVER_BICGSTAB: BiCGStab (van der Vorst 1992; the paper names it among
 * the solvers of the operator-splitting system, Sec. 4) on
 * [1 - diag(1-eps) Lambda] S = (1-eps) Lambda_bc + eps B, right-preconditioned
 * by 1 - (1-eps) Lambda*, from S(J) of the state's J, until
 * ||b - A S||_2 / ||b||_2 < tol per wavelength (at most max_iter iterations,
 * two formal solutions each, all in double precision); then J = Lambda S +
 * Lambda_bc and S = (1-eps) J + eps B.  rel_change receives the final
 * relative residuals and iter is reset to 0 (a later ALI step restarts from
 * this J).  Ng and net options are ignored.
 * Blocks (reads a few bytes per step back to the host).  Returns
 * RT_E_NOT_CONVERGED (state valid and resumable) or RT_E_NUMERIC (NaN/Inf).
 */
rt_status rt_solve(rt_grid_t grid, rt_state *state, const rt_solve_opts *opts,
                   rt_solve_report *report, void *stream);

/*
 * Learned ALI correction (an addition to the paper's method; box grids only).
 * A 3D U-Net maps, per voxel, the features
 *   f0 = r / max|r|,  r = (J_fs - J) / J   (the formal-solution residual of
 *                                           the iterate before an ALI update)
 *   f1 = log10(chi) / 4,  f2 = log10(eps) / 3 + 1
 * to a relative correction c; the ALI iterate becomes
 *   J <- J (1 + clamp(max|r| c, -1/2, 1)).
 * Network: levels l = 0..L-1 with C_l in {16, 32, 64} channels and
 * n_l = (n_{l-1} + 1)/2 points per axis; 3x3x3 convolutions (periodic in x, y,
 * zero-padded in z) with ReLU, stride-2 convolutions down, linear 2x
 * upsampling plus a convolution up, additive skips, a 1x1 head.  Inference
 * runs in bf16 on the matrix cores with fp32 accumulation.
 * Inside rt_solve (opts->net_every > 0) a correction is proposed after every
 * net_every-th plain step k.  One ALI sweep smooths the corrected iterate, and
 * the next sweep's formal solution gives the residual of the smoothed
 * candidate; the correction is kept only where that residual is below
 * res_k q^2, q = res_k / res_{k-1} the recent contraction of the plain
 * iteration (per wavelength).  Otherwise J returns to the plain ALI iterate of
 * step k, at the cost of two formal solutions, and the plain trajectory
 * continues bitwise as without the network.  The fixed point is that of
 * plain ALI, whatever the network.
 *   blob   host memory: "RTUN", uint32 version = 1, uint32 L, uint32 C[L],
 *          then for each convolution in the order input (3 -> C0), level-0
 *          (C0 -> C0), for l = 1..L-1 down_l (C_{l-1} -> C_l, stride 2) and
 *          conv_l (C_l -> C_l), for l = L-1..1 up_l (C_l -> C_{l-1}) and
 *          dec_{l-1} (C_{l-1} -> C_{l-1}), head (C0 -> 1, one tap): float32
 *          weights [tap][c_out][c_in] (tap = (dz*3 + dy)*3 + dx) and biases
 *          [c_out].  Copied; the caller keeps ownership.  NULL removes the net.
 * Errors: RT_E_INVALID (malformed blob), RT_E_UNSUPPORTED (spherical grid),
 * RT_E_HIP.
 */
rt_status rt_set_preconditioner(rt_grid_t grid, const void *blob, size_t bytes);

/*
 * Network inference alone (for tests and tools): out = network(features) on
 * the grid's Nz x Ny x Nx volume.  features: device float [Nz][Ny][Nx][3];
 * out: device float [Nz][Ny][Nx].  Asynchronous on stream.  RT_E_INVALID if
 * no network is set.
 */
rt_status rt_precond_forward(rt_grid_t grid, const float *features, float *out, void *stream);

/*
 * Host-only tracker output for one direction of the box (no GPU needed): the
 * characteristic entering the centre of the inflow face of column (0,0),
 * segment by segment -- unwrapped voxel offsets di, dj from the entry column,
 * layer kk (0 = top) and path length s.  dir = i_mu * n_phi + j_phi.
 * *M receives the segment count; the arrays (host memory, cap entries each)
 * are filled when cap >= *M.  For inspection and tests of the geometry cache.
 */
rt_status rt_box_template(int32_t Nz, int32_t n_mu, int32_t n_phi, int32_t dir, int32_t cap, int32_t *di,
                          int32_t *dj, int32_t *kk, double *s, int32_t *M);

/*
 * The characteristics of direction `dir` of a spherical grid, as the library
 * traces them (host only, no device needed).  Per direction: a square lattice
 * of foot points p (spacing h = median cube root of the voxel volumes, axes
 * e1 = normalise(z x n), or x when n is along z, and e2 = n x e1) with
 * |p| < r_out, then, in voxel-index order, one line through the centre of
 * every voxel not visited yet.  A line meeting the core gives an inward
 * characteristic ending on it and an outward one starting on it.  Crossings
 * with spheres, cones and half-planes are sorted; crossings within
 * 1e-12 (|t| + 1) of the previous segment end are merged; each segment
 * belongs to the voxel containing its midpoint.
 *   h_out        spacing h (may be NULL)
 *   n_chars, n_visits  in: capacity of the arrays; out: counts
 *   chars        [n_chars][6] = p (3), t_a, t_b, kind (0 outer, 1 core):
 *                the characteristic is p + t n for t in [t_a, t_b]
 *   visit_begin  [n_chars + 1]; vox, s: [n_visits] voxel and path length
 * With any of chars, visit_begin, vox, s NULL only the counts are returned.
 */
rt_status rt_sphere_tracks(const rt_grid_desc *desc, int32_t dir, double *h_out, int64_t *n_chars,
                           int64_t *n_visits, double *chars, int64_t *visit_begin, int32_t *vox, double *s);

/*
 * Launch-shape autotuner (the "run-time configuration optimisation" the paper
 * suggests, Sec. 6): times the single-output (J) formal-solution kernel of the
 * grid's precision for every compiled (workgroup size, rays per thread) shape
 * that can hold one direction's rays, on the caller's fields (n_lambda
 * wavelengths of chi and S, device, as in rt_formal_solution, zero boundary
 * intensity), and keeps the fastest for all later formal solutions and ALI
 * steps of this grid.  Row-band tile shapes compete on every box grid (their
 * flush covers only the rows a bundle reaches, which can beat whole-layer
 * tiles even where those fit); whole-layer shapes only on grids without
 * RT_F_BAND_TILES whose layer fits the LDS.  rt_launch_shape reports which
 * kind was kept.  The shape changes only how directions are grouped
 * into workgroup partial sums, i.e. the summation order of J (differences
 * at the rounding level of the grid precision).  Blocks.  Box grids only
 * (RT_E_UNSUPPORTED on spherical grids).
 * threads_out / rays_out (may be NULL) receive the chosen shape (workgroup
 * size bound and rays per thread, as rt_set_launch_shape takes them).
 */
rt_status rt_autotune(rt_grid_t grid, int32_t n_lambda, const void *chi, const void *S, int32_t *threads_out,
                      int32_t *rays_out, void *stream);

/*
 * rt_autotune on the formal solution over a subset of the directions (as
 * rt_formal_solution_dirs takes them: host, strictly increasing indices), for
 * a grid that will sweep only that share, e.g. one GPU's directions of a
 * solid-angle decomposition (Sec. 4): few directions need more ray bundles
 * per direction (RT_F_BAND_TILES shapes) to keep every CU busy.  Errors as
 * rt_autotune and rt_formal_solution_dirs.
 */
rt_status rt_autotune_dirs(rt_grid_t grid, int32_t n_lambda, const void *chi, const void *S, int32_t n_dirs,
                           const int32_t *dirs, int32_t *threads_out, int32_t *rays_out, void *stream);

/*
 * Fixes the launch shape of the grid's single-output formal-solution kernel
 * to one of the compiled shapes (threads = workgroup size bound, rays = rays
 * per thread), e.g. one that rt_autotune chose in an earlier process, so that
 * runs are reproducible without re-tuning.  A launch may use fewer threads
 * than the bound when a direction has fewer rays.  RT_E_INVALID if no
 * compiled shape matches or the shape cannot hold one direction's rays in
 * the device's LDS; RT_E_UNSUPPORTED on spherical grids.  Does not launch
 * anything.  Where a shape is compiled for both tile kinds, the grid's own
 * kind (row bands with RT_F_BAND_TILES or a layer beyond the LDS, else whole
 * layers) is taken; rt_set_launch_shape_tiles names the kind.
 */
rt_status rt_set_launch_shape(rt_grid_t grid, int32_t threads, int32_t rays);

/*
 * rt_set_launch_shape with the tile kind named: band = 1 for row-band tiles,
 * 0 for whole-layer tiles (as rt_launch_shape reports it), so that a shape
 * kept by rt_autotune can be set again exactly.  Whole-layer tiles on a grid
 * that needs row bands are RT_E_INVALID; other errors as rt_set_launch_shape.
 */
rt_status rt_set_launch_shape_tiles(rt_grid_t grid, int32_t threads, int32_t rays, int32_t band);

/*
 * RT_FP32 box grids: fixes the launch shape of the double-precision anchor
 * sweep (the defect-correction anchors of rt_solve), e.g. to the shape that
 * rt_autotune picked on a double-precision grid of the same size (band as
 * rt_set_launch_shape_tiles takes it).  Shapes and errors as
 * rt_set_launch_shape_tiles; RT_E_INVALID on double-precision grids.
 */
rt_status rt_set_anchor_shape(rt_grid_t grid, int32_t threads, int32_t rays, int32_t band);

/*
 * The launch shape that the grid's single-output formal-solution kernel
 * uses now (box grids): workgroup size bound, rays per thread, ray bundles
 * per direction (workgroups that share one direction, each with its own tile
 * and partial sums), and band = 1 if the tiles are row bands
 * (RT_F_BAND_TILES, or a layer too wide for a whole-layer tile in LDS), else
 * 0.  Any out pointer may be NULL.  RT_E_UNSUPPORTED on spherical grids.
 */
rt_status rt_launch_shape(rt_grid_t grid, int32_t *threads, int32_t *rays, int32_t *bundles, int32_t *band);

/*
 * Bytes of the grid's geometry cache held in device memory and in pinned
 * host memory (streamed chunks of a spherical grid; 0 for box grids, whose
 * cache is one template per direction).  Any out pointer may be NULL.
 */
rt_status rt_cache_bytes(rt_grid_t grid, int64_t *device_bytes, int64_t *host_bytes);

/*
 * Measurement hooks.  While enabled, every formal-solution kernel launch of
 * this grid is bracketed by HIP events recorded on the launch stream; plain
 * ALI steps run as HIP graphs (use_graph) are captured with two one-wave
 * kernels around their sweep that store the device wall clock, and the time
 * of each replay is collected before that graph is replayed again (the call
 * then waits for the previous replay) and by rt_profile_read.  rt_profile_read waits for those events and
 * returns the summed kernel time (ms), the number of launches and the number
 * of characteristic points they evaluated (visits x rays, summed over work
 * items) since the previous read, then starts a new interval.  Out pointers
 * may be NULL.
 */
rt_status rt_profile_enable(rt_grid_t grid, int32_t enable);
rt_status rt_profile_read(rt_grid_t grid, double *fs_ms, int32_t *fs_launches, int64_t *fs_points);

/* Size of the fixed device scratch of rt_formal_solution_noalloc (per GPU). */
#define RT_NOALLOC_SCRATCH_BYTES (64u << 20)

/*
 * rt_formal_solution for callers that cannot allocate device memory: code
 * being captured into a HIP graph, serving loops and harnesses that forbid
 * hipMalloc.  Same arguments, outputs and errors as rt_formal_solution (box
 * grids; RT_E_UNSUPPORTED on spherical grids).  Every scratch buffer of the
 * call -- the work schedule, the padded (chi, S) input and the workgroup
 * partial sums -- lives in one fixed device array of RT_NOALLOC_SCRATCH_BYTES
 * that the library holds on each GPU it runs on until the process ends (set
 * up by rt_create_grid); the call itself allocates no device memory and
 * frees none.  When the partial sums of the grid's usual workgroup count do
 * not fit, fewer persistent workgroups are launched (results then differ
 * from rt_formal_solution's in the summation order only); a call whose
 * padded input plus one workgroup's partial sums per ray bundle exceed the
 * array is refused with RT_E_INVALID before anything is enqueued.  All calls
 * on one GPU share the array: calls that overlap in time on one GPU (e.g.
 * on two streams, or from two threads) race and give wrong results.
 * The work schedule is copied from host memory the grid keeps; nothing in
 * the array needs to start at zero.
 */
rt_status rt_formal_solution_noalloc(rt_grid_t grid, int32_t n_lambda, const void *chi, const void *S,
                                     const void *I_bc, void *J_out, void *lstar_out, void *stream);

/* Message of the last failed call on this thread ("" if none). */
const char *rt_last_error(void);

/* Library version string. */
const char *rt_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RT3D_H */
