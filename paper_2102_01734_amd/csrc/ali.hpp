// ali.hpp -- launch interface of the padding, reduction, ALI and Ng kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rt3d {

// Writes component comp (0 = chi, 1 = S) of the interleaved doubly periodic
// padded formal-solution input (see ali.hip).  Ny == 0 selects the
// voxel-major pair layout [voxel][Nx][2] of the spherical grid, Nx the
// wavelength stride and Nz the number of voxels.
template <typename TS, typename TD>
hipError_t pad_field(const TS *src, const double *anchor, TD *dst, int Nx, int Ny, int Nz, int n_lambda, int comp,
                     hipStream_t st);

template <typename TP, typename TO>
hipError_t reduce_partials(const TP *part, const int32_t *slot_begin, const int32_t *slot_ids,
                           const int32_t *lambda_of, int n_batch, TO *out, int64_t n_vox, hipStream_t st);

template <typename G, typename TN>
hipError_t source_update(const double *J, const G *eps, const G *B, double *S, const double *S_anchor, TN *next_pad,
                         int Nx, int Ny, int64_t n_vox, const int32_t *lambda_of, int n_batch, hipStream_t st);

template <typename TS, typename TD>
hipError_t cast_array(const TS *src, TD *dst, int64_t n, hipStream_t st);

hipError_t fill_u64(unsigned long long *p, unsigned long long v, int n, hipStream_t st);

// p[0] = the device wall clock (hipDeviceAttributeWallClockRate kHz) when the
// one-wave stamp kernel runs, in stream order.
hipError_t wall_stamp(unsigned long long *p, hipStream_t st);

// Smallest operator-splitting denominator 1 - (1-eps) Lambda*_vv.  Where
// eps -> 0 and the medium is optically thick, Lambda* approaches 1; stored
// in single precision it can round to exactly 1 (a pure-scattering medium
// then gives a zero denominator), so single-precision data clamp at 1e-7
// (about their rounding unit), double-precision data at 1e-12.
template <typename G>
__host__ __device__ constexpr double os_den_min()
{
    return sizeof(G) == 4 ? 1e-7 : 1e-12;
}

struct AliUpdateArgs {
    int Nx, Ny;
    int64_t n_vox;
    const int32_t *lambda_of;   // batch entry -> wavelength index
    const void *part;           // partial slots of the formal solution, or null
    const int32_t *slot_begin;  // per batch entry
    const int32_t *slot_ids;
    const double *J_anchor;     // double-precision anchor J_fs(S_anchor), or null
    const double *S_anchor;     // anchor source, or null
    const void *eps, *B, *lstar;  // grid precision
    double *J;                  // in/out
    double *S;                  // out
    double *hist;               // out: copy of the new J into the Ng ring, or null
    void *next_pad;             // out: S - S_anchor into the interleaved padded input
    double *rel_change;         // out: per wavelength max |dJ/J| (atomic max)
    double *resid;              // out: per wavelength max |J_fs - J_old| / |J_old| (atomic max), or null
    float *net_r;               // out: (J_fs - J_old) / J_old per voxel (network input), or null
    // operator-splitting system solved outside (non-local Lambda*):
    double *rfs_out;            // if set: only write J_fs - J_old here and return
    const double *rfs_in;       // if set: J_fs = J_old + rfs_in (part and J_anchor unused)
    const double *dJ;           // if set: J_new = J_old + dJ instead of the diagonal solution
};

hipError_t ali_update(const AliUpdateArgs &a, bool part_double, bool grid_double, bool next_double, int n_batch,
                      hipStream_t st);

struct NgApplyArgs {
    int Nx, Ny;
    int64_t n_vox;
    const int32_t *lambda_of;
    const double *x0, *x1, *x2, *x3;  // newest .. oldest iterate
    double *coef;                     // [batch][3]: a, b, applied
    const void *eps, *B;
    const double *S_anchor;
    double *J, *S;
    void *next_pad;
};

hipError_t ng_accelerate(const NgApplyArgs &a, double *blk, int nblk, int n_batch, bool grid_double,
                         hipStream_t st);

}  // namespace rt3d
