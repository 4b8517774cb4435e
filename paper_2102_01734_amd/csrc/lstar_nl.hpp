// lstar_nl.hpp -- nearest-neighbour (non-local) Lambda* on the box and the
// Jacobi solver of the operator-splitting system it defines.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rt3d {

// Stencil components: c = (dz+1)*9 + (dy+1)*3 + (dx+1) for the neighbour
// u = v + (dx, dy, dz) (x, y periodic; dz = +1 is the next layer down);
// c = 13 is the voxel itself.
constexpr int kStencil = 27;
constexpr int kStencilCentre = 13;

// Per visit of a template (StencilArgs::comp): the stencil components of the
// voxels that the points m+1, m, m-1, m-2, m-3 of a characteristic lie in,
// seen from the voxel of point m, 6 bits each (j + 1 = 0..4 for point m - j),
// kNoComp (rt_internal.hpp) when that point is not a neighbour or does not
// exist.

struct StencilArgs {
    int Nx, Ny, Nz;
    int64_t n_vox;
    const uint32_t *dxy;       // per visit: di mod Nx | (dj mod Ny) << 15 | layer-end flag
    const double *s;           // per visit: path length
    const uint32_t *comp;      // per visit: packed stencil components (see above)
    const int64_t *dir_vbegin;
    const int32_t *dir_M;
    const double *dir_wmu;     // w_d |mu_d|
    const double *dir_mu;
    const void *chi;           // caller opacity [lambda][Nz][Ny][Nx], grid precision
    const int32_t *lambda_of;  // batch entry -> wavelength
    unsigned long long *acc;   // [lambda][27][n_vox] fixed point (2^-52), cleared by the caller
    int skip_centre;           // 1: leave the centre component (the diagonal Lambda*) out
    // row-window kernel (used when dir_plane is set): per visit the row
    // relative to the lowest template row of its layer; per direction
    // kPlaneStride entries: [0, 27) component -> tile plane (-1: never added,
    // including the centre when skip_centre), [32, 32 + planes) plane ->
    // component (32-bit entries: the kernel reads them with scalar loads);
    // planes: the largest plane count of any direction; rows: ray rows per
    // workgroup (set by the launcher)
    const int32_t *brow;
    const int32_t *dir_plane;
    int planes;
    int rows;
};

constexpr int kPlaneStride = 64;

// Nearest-neighbour Lambda* on a spherical grid, one chunk of the geometry
// cache: one thread per characteristic and batch entry follows the
// characteristic's visits (same recurrence as the box), and adds
// w_m G_j (w_m the visit's voxel-averaging weight) to component
// c = (dp+1)*9 + (dt+1)*3 + (dr+1) of its voxel for the points m+1 .. m-3
// whose voxel is an index neighbour (phi periodic, r and theta bounded) with
// one 64-bit fixed-point atomic each.
struct SphereStencilArgs {
    int Nr, Nt, Np;
    int64_t n_vox;
    int64_t n_bundles;
    const int64_t *bundle_begin;  // entry of visit m of characteristic c of bundle b: bundle_begin[b] + 64 m + c
    const int32_t *char_len;
    const int32_t *vox;
    const void *s, *w;            // geometry type
    const void *chi;              // [lambda][n_vox], grid precision
    const int32_t *lambda_of;
    int n_batch;
    unsigned long long *acc;      // [lambda][27][n_vox]
    int skip_centre;
};
hipError_t lstar_stencil_sphere_accumulate(const SphereStencilArgs &a, bool grid_double, bool geom_double,
                                           bool parabolic, hipStream_t st);

// Adds every characteristic's contributions to the stencil of the linear-
// interpolation operator (parabolic = false) or of the formal solution
// itself (parabolic = true), for n_batch wavelengths and all directions.
// max_lds: shared memory per workgroup (bytes); layers too wide for a tile of
// two rows use a per-characteristic kernel with one global atomic per
// contribution instead.
hipError_t lstar_stencil_accumulate(const StencilArgs &a, bool grid_double, bool parabolic, int n_dir, int n_batch,
                                    size_t max_lds, hipStream_t st);

// out[lam][c][v] = acc[lam][c][v] * 2^-52 (T = float or double); with
// `centre` (T, [lambda][n_vox]: a diagonal Lambda* of the same operator) the
// centre component is copied from it instead.
hipError_t lstar_stencil_finish(const unsigned long long *acc, const int32_t *lambda_of, int64_t n_vox, int n_batch,
                                const void *centre, void *out, bool out_double, hipStream_t st);

// One Jacobi sweep of [1 - Lambda*(1-eps)] x = r per wavelength of the batch
// (first: x = r / (1 - Lambda*_vv (1-eps_v)), the diagonal solution).
struct OsJacobiArgs {
    int Nx, Ny, Nz;        // voxel v = (z Ny + y) Nx + x (sphere: x = r, y = theta, z = phi)
    int per[3];            // per axis x, y, z: 1 periodic, 0 bounded (box 1, 1, 0; sphere 0, 0, 1)
    int64_t n_vox;
    const int32_t *lambda_of;
    const void *st;       // [lambda][27][n_vox], grid precision
    const void *eps;      // [lambda][n_vox], grid precision
    const double *r;      // [lambda][n_vox]
    const double *x_in;   // [lambda][n_vox] (unused when first)
    double *x_out;        // [lambda][n_vox]
};
hipError_t os_jacobi_sweep(const OsJacobiArgs &a, bool grid_double, bool first, int n_batch, hipStream_t st);
// One Gauss-Seidel sweep, in place on x_out (x_in unused), over the 18
// colour classes in the order cz * 9 + cy * 3 + cx, where c = index mod 2
// along each axis, except the last index of an odd periodic axis of length
// >= 3, which takes class 2.  Voxels of one class share no stencil coupling,
// so each class is updated in parallel.
hipError_t os_gs_sweep(const OsJacobiArgs &a, bool grid_double, int n_batch, hipStream_t st);

}  // namespace rt3d
