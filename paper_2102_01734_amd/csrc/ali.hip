// ali.hip -- field padding, partial-sum reduction, the operator-splitting
// update, Ng acceleration and convergence norms (gfx950).
//
// Operator splitting with a diagonal Lambda* (Sec. 2.2, eq. alo of the paper):
//   [1 - Lambda*(1-eps)] J_new = J_fs - Lambda*(1-eps) J_old
// written as the increment J_new = J_old + (J_fs - J_old) / (1 - (1-eps) Lambda*),
// then S = (1-eps) J_new + eps B.  All ALI state is double precision.
//
// Ng acceleration (Ng 1974; least-squares form of Auer 1987, not part of the
// paper): with the last four iterates x0 (newest) .. x3, d_i = x_i - x_{i+1},
// Q1 = d0 - d1, Q2 = d0 - d2 and weights 1/x0^2, (a, b) minimise
// sum w (d0 - a Q1 - b Q2)^2 and x <- (1-a-b) x0 + a x1 + b x2.
//
// Every reduction over voxels runs in a fixed order (per-block partials, then
// one block per wavelength), so results are bitwise reproducible; the only
// atomics are max-reductions of non-negative doubles, which are exact.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ali.hpp"

namespace rt3d {

// ---------------------------------------------------------------------------
// Formal-solution input layout: for every wavelength a doubly periodic padded
// copy [k][y2][x2] (y2 < 2Ny, x2 < 2Nx) of the pair (chi, S), interleaved so a
// point's opacity and source are one 8- (16-) byte load:
//   dst[((l*Nz + k)*2Ny + y2)*2Nx + x2][comp] = src[l][k][y2 mod Ny][x2 mod Nx],
// comp 0 = chi, comp 1 = S (optionally minus an anchor), in the kernel type.
// Ny == 0 selects the voxel-major layout of the spherical grid, pairs
// [voxel][Nx][2] with Nx the wavelength stride (no periodic directions), so
// the wavelengths of one voxel are contiguous.
// ---------------------------------------------------------------------------
template <typename TD>
__device__ __forceinline__ void store_padded(TD *dst, int64_t l, int64_t n_vox, int64_t v, int Nx, int Ny, int comp,
                                             TD val)
{
    if (Ny == 0) {
        dst[2 * (v * Nx + l) + comp] = val;
        return;
    }
    const int x = (int)(v % Nx);
    const int64_t r = v / Nx;
    const int y = (int)(r % Ny);
    const int64_t k = r / Ny;
    TD *base = dst + 2 * (l * 4 * n_vox + k * (4LL * Nx * Ny)) + comp;
    const int64_t W = 2 * Nx;
    base[2 * ((int64_t)y * W + x)] = val;
    base[2 * ((int64_t)y * W + x + Nx)] = val;
    base[2 * ((int64_t)(y + Ny) * W + x)] = val;
    base[2 * ((int64_t)(y + Ny) * W + x + Nx)] = val;
}

template <typename TS, typename TD>
__global__ void pad_kernel(const TS *__restrict__ src, const double *__restrict__ anchor, TD *__restrict__ dst,
                           int Nx, int Ny, int64_t per_lambda, int64_t total, int comp)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int64_t l = i / per_lambda;
    const int64_t v = i - l * per_lambda;
    double val = (double)src[i];
    if (anchor) val -= anchor[i];
    store_padded<TD>(dst, l, per_lambda, v, Nx, Ny, comp, (TD)val);
}

template <typename TS, typename TD>
hipError_t pad_field(const TS *src, const double *anchor, TD *dst, int Nx, int Ny, int Nz, int n_lambda, int comp,
                     hipStream_t st)
{
    const int64_t per = Ny > 0 ? (int64_t)Nx * Ny * Nz : (int64_t)Nz;
    const int64_t total = per * n_lambda;
    if (total == 0) return hipSuccess;
    const int bs = 256;
    hipLaunchKernelGGL((pad_kernel<TS, TD>), dim3((unsigned)((total + bs - 1) / bs)), dim3(bs), 0, st, src, anchor,
                       dst, Nx, Ny, per, total, comp);
    return hipGetLastError();
}

template hipError_t pad_field<float, float>(const float *, const double *, float *, int, int, int, int, int,
                                             hipStream_t);
template hipError_t pad_field<float, double>(const float *, const double *, double *, int, int, int, int, int,
                                             hipStream_t);
template hipError_t pad_field<double, double>(const double *, const double *, double *, int, int, int, int, int,
                                             hipStream_t);
template hipError_t pad_field<double, float>(const double *, const double *, float *, int, int, int, int, int,
                                             hipStream_t);

// ---------------------------------------------------------------------------
// out[lambda_of[b]][v] = sum over slots of batch entry b of part[slot][v]
// (double accumulation, fixed slot order)
// ---------------------------------------------------------------------------
template <typename TP, typename TO>
__global__ void reduce_kernel(const TP *__restrict__ part, const int32_t *__restrict__ slot_begin,
                              const int32_t *__restrict__ slot_ids, const int32_t *__restrict__ lambda_of,
                              TO *__restrict__ out, int64_t n_vox)
{
    const int b = blockIdx.y;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n_vox) return;
    double acc = 0.0;
    const int s1 = slot_begin[b + 1];
    for (int s = slot_begin[b]; s < s1; ++s) acc += (double)part[(int64_t)slot_ids[s] * n_vox + v];
    out[(int64_t)lambda_of[b] * n_vox + v] = (TO)acc;
}

template <typename TP, typename TO>
hipError_t reduce_partials(const TP *part, const int32_t *slot_begin, const int32_t *slot_ids,
                           const int32_t *lambda_of, int n_batch, TO *out, int64_t n_vox, hipStream_t st)
{
    if (n_batch == 0 || n_vox == 0) return hipSuccess;
    const int bs = 256;
    dim3 grid((unsigned)((n_vox + bs - 1) / bs), (unsigned)n_batch);
    hipLaunchKernelGGL((reduce_kernel<TP, TO>), grid, dim3(bs), 0, st, part, slot_begin, slot_ids, lambda_of, out,
                       n_vox);
    return hipGetLastError();
}

template hipError_t reduce_partials<float, float>(const float *, const int32_t *, const int32_t *, const int32_t *,
                                                  int, float *, int64_t, hipStream_t);
template hipError_t reduce_partials<float, double>(const float *, const int32_t *, const int32_t *,
                                                   const int32_t *, int, double *, int64_t, hipStream_t);
template hipError_t reduce_partials<double, double>(const double *, const int32_t *, const int32_t *,
                                                    const int32_t *, int, double *, int64_t, hipStream_t);
template hipError_t reduce_partials<double, float>(const double *, const int32_t *, const int32_t *,
                                                   const int32_t *, int, float *, int64_t, hipStream_t);

template <typename TS, typename TD>
__global__ void cast_kernel(const TS *__restrict__ src, TD *__restrict__ dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (TD)src[i];
}

template <typename TS, typename TD>
hipError_t cast_array(const TS *src, TD *dst, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((cast_kernel<TS, TD>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

template hipError_t cast_array<float, double>(const float *, double *, int64_t, hipStream_t);

// ---------------------------------------------------------------------------
// small fills (used instead of memset so the step can live in a graph)
// ---------------------------------------------------------------------------
__global__ void fill_u64_kernel(unsigned long long *p, unsigned long long v, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t fill_u64(unsigned long long *p, unsigned long long v, int n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u64_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

// Stores the device's constant-rate wall clock: stream-ordered time stamps
// around a kernel inside a captured graph.
__global__ void wall_stamp_kernel(unsigned long long *p)
{
    if (threadIdx.x == 0) *p = (unsigned long long)wall_clock64();
}

hipError_t wall_stamp(unsigned long long *p, hipStream_t st)
{
    hipLaunchKernelGGL(wall_stamp_kernel, dim3(1), dim3(64), 0, st, p);
    return hipGetLastError();
}

__device__ __forceinline__ void atomic_max_nonneg(double *addr, double v)
{
    // non-negative doubles (and NaN, whose bits sort above +inf) order like
    // their bit patterns read as unsigned integers
    atomicMax(reinterpret_cast<unsigned long long *>(addr), (unsigned long long)__double_as_longlong(v));
}

template <int BS>
__device__ __forceinline__ double block_max(double v)
{
    __shared__ double red[BS / 64];
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int w = threadIdx.x / 64, ln = threadIdx.x % 64;
    if (ln == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x < 64) {
        v = threadIdx.x < BS / 64 ? red[threadIdx.x] : 0.0;
        for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    }
    return v;
}

// S = (1-eps) J + eps B, evaluated the same way (no contraction) wherever S
// is formed, so a source recomputed from a restored J is bitwise the one the
// update produced
__device__ __forceinline__ double source_value(double e, double j, double b)
{
#pragma clang fp contract(off)
    return (1.0 - e) * j + e * b;
}

// ---------------------------------------------------------------------------
// S = (1-eps) J + eps B and the padded formal-solution input (S - anchor)
// ---------------------------------------------------------------------------
template <typename G, typename TN>
__global__ void source_kernel(const double *__restrict__ J, const G *__restrict__ eps, const G *__restrict__ B,
                              double *__restrict__ S, const double *__restrict__ S_anchor, TN *__restrict__ next_pad,
                              int Nx, int Ny, int64_t n_vox, const int32_t *__restrict__ lambda_of)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n_vox) return;
    const int64_t i = (int64_t)lambda_of[blockIdx.y] * n_vox + v;
    const double e = (double)eps[i];
    const double s = source_value(e, J[i], (double)B[i]);
    S[i] = s;
    const TN out = (TN)(S_anchor ? s - S_anchor[i] : s);
    store_padded<TN>(next_pad, lambda_of[blockIdx.y], n_vox, v, Nx, Ny, 1, out);
}

template <typename G, typename TN>
hipError_t source_update(const double *J, const G *eps, const G *B, double *S, const double *S_anchor, TN *next_pad,
                         int Nx, int Ny, int64_t n_vox, const int32_t *lambda_of, int n_batch, hipStream_t st)
{
    if (n_batch == 0 || n_vox == 0) return hipSuccess;
    const int bs = 256;
    dim3 grid((unsigned)((n_vox + bs - 1) / bs), (unsigned)n_batch);
    hipLaunchKernelGGL((source_kernel<G, TN>), grid, dim3(bs), 0, st, J, eps, B, S, S_anchor, next_pad, Nx, Ny, n_vox,
                       lambda_of);
    return hipGetLastError();
}

template hipError_t source_update<float, float>(const double *, const float *, const float *, double *,
                                                const double *, float *, int, int, int64_t, const int32_t *, int,
                                                hipStream_t);
template hipError_t source_update<double, double>(const double *, const double *, const double *, double *,
                                                  const double *, double *, int, int, int64_t, const int32_t *, int,
                                                  hipStream_t);
template hipError_t source_update<float, double>(const double *, const float *, const float *, double *,
                                                 const double *, double *, int, int, int64_t, const int32_t *, int,
                                                 hipStream_t);

// ---------------------------------------------------------------------------
// fused: J_fs = J_anchor + sum of partial slots; operator-splitting update;
// S; next padded input; Ng history; per-wavelength max |dJ/J|
// ---------------------------------------------------------------------------
template <typename TP, typename G, typename TN>
__global__ void __launch_bounds__(256) ali_update_kernel(AliUpdateArgs a)
{
    const int b = blockIdx.y;
    const int lam = a.lambda_of[b];
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double rel = 0.0, res = 0.0;
    if (a.rfs_out) {  // uniform over the launch: no thread reaches the block reductions
        if (v < a.n_vox) {
            const int64_t i = (int64_t)lam * a.n_vox + v;
            double jfs = a.J_anchor ? a.J_anchor[i] : 0.0;
            if (a.part) {
                const TP *part = reinterpret_cast<const TP *>(a.part);
                const int s1 = a.slot_begin[b + 1];
                double acc = 0.0;
                for (int s = a.slot_begin[b]; s < s1; ++s) acc += (double)part[(int64_t)a.slot_ids[s] * a.n_vox + v];
                jfs += acc;
            }
            a.rfs_out[i] = jfs - a.J[i];
        }
        return;
    }
    if (v < a.n_vox) {
        const int64_t i = (int64_t)lam * a.n_vox + v;
        double jfs = a.J_anchor ? a.J_anchor[i] : 0.0;
        if (a.rfs_in) {
            jfs = a.J[i] + a.rfs_in[i];
        } else if (a.part) {
            const TP *part = reinterpret_cast<const TP *>(a.part);
            const int s1 = a.slot_begin[b + 1];
            double acc = 0.0;
            for (int s = a.slot_begin[b]; s < s1; ++s) acc += (double)part[(int64_t)a.slot_ids[s] * a.n_vox + v];
            jfs += acc;
        }
        const double e = (double)reinterpret_cast<const G *>(a.eps)[i];
        const double L = (double)reinterpret_cast<const G *>(a.lstar)[i];
        const double Bv = (double)reinterpret_cast<const G *>(a.B)[i];
        const double jo = a.J[i];
        const double rr = (jfs - jo) / jo;
        res = fabs(rr);
        if (!(res <= 1.0e308)) res = __builtin_inf();
        if (a.net_r) a.net_r[i] = (float)rr;
        double den = 1.0 - (1.0 - e) * L;
        den = den < os_den_min<G>() ? os_den_min<G>() : den;
        const double jn = a.dJ ? jo + a.dJ[i] : jo + (jfs - jo) / den;
        a.J[i] = jn;
        if (a.hist) a.hist[i] = jn;
        const double dj = fabs(jn - jo);
        rel = dj == 0.0 ? 0.0 : dj / fabs(jn);
        if (!(rel <= 1.0e308)) rel = __builtin_inf();  // NaN or Inf: reported as non-finite
        const double s = source_value(e, jn, Bv);
        a.S[i] = s;
        const TN out = (TN)(a.S_anchor ? s - a.S_anchor[i] : s);
        store_padded<TN>(reinterpret_cast<TN *>(a.next_pad), lam, a.n_vox, v, a.Nx, a.Ny, 1, out);
    }
    rel = block_max<256>(rel);
    if (threadIdx.x == 0) atomic_max_nonneg(&a.rel_change[lam], rel);
    if (a.resid) {
        __syncthreads();  // the reduction scratch of block_max is reused
        res = block_max<256>(res);
        if (threadIdx.x == 0) atomic_max_nonneg(&a.resid[lam], res);
    }
}

template <typename TP, typename G, typename TN>
static hipError_t ali_update_t(const AliUpdateArgs &a, int n_batch, hipStream_t st)
{
    const int bs = 256;
    dim3 grid((unsigned)((a.n_vox + bs - 1) / bs), (unsigned)n_batch);
    hipLaunchKernelGGL((ali_update_kernel<TP, G, TN>), grid, dim3(bs), 0, st, a);
    return hipGetLastError();
}

hipError_t ali_update(const AliUpdateArgs &a, bool part_double, bool grid_double, bool next_double, int n_batch,
                      hipStream_t st)
{
    if (n_batch == 0 || a.n_vox == 0) return hipSuccess;
    if (grid_double) {
        if (part_double && next_double) return ali_update_t<double, double, double>(a, n_batch, st);
        return hipErrorInvalidValue;
    }
    if (next_double) return hipErrorInvalidValue;
    if (part_double) return ali_update_t<double, float, float>(a, n_batch, st);
    return ali_update_t<float, float, float>(a, n_batch, st);
}

// ---------------------------------------------------------------------------
// Ng: five weighted dot products per wavelength (per-block partials, then a
// fixed-order sum), the 2x2 solve, and the extrapolation
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) ng_dots_kernel(const double *__restrict__ x0, const double *__restrict__ x1,
                                                      const double *__restrict__ x2, const double *__restrict__ x3,
                                                      const int32_t *__restrict__ lambda_of, int64_t n_vox,
                                                      double *__restrict__ blk)
{
    const int b = blockIdx.y;
    const int64_t lam = lambda_of[b];
    double acc[5] = {0, 0, 0, 0, 0};
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n_vox; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = lam * n_vox + v;
        const double a0 = x0[i], a1 = x1[i], a2 = x2[i], a3 = x3[i];
        const double d0 = a0 - a1, d1 = a1 - a2, d2 = a2 - a3;
        const double q1 = d0 - d1, q2 = d0 - d2;
        const double w = 1.0 / (a0 * a0);
        acc[0] += w * q1 * q1;
        acc[1] += w * q1 * q2;
        acc[2] += w * q2 * q2;
        acc[3] += w * d0 * q1;
        acc[4] += w * d0 * q2;
    }
    __shared__ double red[5][4];
    const int wv = threadIdx.x / 64, ln = threadIdx.x % 64;
    for (int c = 0; c < 5; ++c) {
        double v = acc[c];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (ln == 0) red[c][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        const double s = ((red[threadIdx.x][0] + red[threadIdx.x][1]) + red[threadIdx.x][2]) + red[threadIdx.x][3];
        blk[((int64_t)b * gridDim.x + blockIdx.x) * 5 + threadIdx.x] = s;
    }
}

__global__ void ng_solve_kernel(const double *__restrict__ blk, int nblk, double *__restrict__ coef)
{
    const int b = blockIdx.x;
    if (threadIdx.x != 0) return;
    double A[5] = {0, 0, 0, 0, 0};
    for (int k = 0; k < nblk; ++k)
        for (int c = 0; c < 5; ++c) A[c] += blk[((int64_t)b * nblk + k) * 5 + c];
    const double det = A[0] * A[2] - A[1] * A[1];
    double ca = 0.0, cb = 0.0, ok = 0.0;
    if (det > 1e-10 * A[0] * A[2] && det == det && det < 1e300) {
        ca = (A[3] * A[2] - A[4] * A[1]) / det;
        cb = (A[4] * A[0] - A[3] * A[1]) / det;
        ok = 1.0;
    }
    coef[3 * b + 0] = ca;
    coef[3 * b + 1] = cb;
    coef[3 * b + 2] = ok;
}

template <typename G, typename TN>
__global__ void ng_apply_kernel(NgApplyArgs a)
{
    const int b = blockIdx.y;
    const int lam = a.lambda_of[b];
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= a.n_vox) return;
    if (a.coef[3 * b + 2] == 0.0) return;  // singular system: keep the plain iterate
    const double ca = a.coef[3 * b + 0], cb = a.coef[3 * b + 1];
    const int64_t i = (int64_t)lam * a.n_vox + v;
    const double jn = (1.0 - ca - cb) * a.x0[i] + ca * a.x1[i] + cb * a.x2[i];
    a.J[i] = jn;
    const double e = (double)reinterpret_cast<const G *>(a.eps)[i];
    const double s = source_value(e, jn, (double)reinterpret_cast<const G *>(a.B)[i]);
    a.S[i] = s;
    const TN out = (TN)(a.S_anchor ? s - a.S_anchor[i] : s);
    store_padded<TN>(reinterpret_cast<TN *>(a.next_pad), lam, a.n_vox, v, a.Nx, a.Ny, 1, out);
}

hipError_t ng_accelerate(const NgApplyArgs &a, double *blk, int nblk, int n_batch, bool grid_double, hipStream_t st)
{
    if (n_batch == 0 || a.n_vox == 0) return hipSuccess;
    hipLaunchKernelGGL(ng_dots_kernel, dim3(nblk, n_batch), dim3(256), 0, st, a.x0, a.x1, a.x2, a.x3, a.lambda_of,
                       a.n_vox, blk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(ng_solve_kernel, dim3(n_batch), dim3(64), 0, st, blk, nblk, a.coef);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int bs = 256;
    dim3 grid((unsigned)((a.n_vox + bs - 1) / bs), (unsigned)n_batch);
    if (grid_double)
        hipLaunchKernelGGL((ng_apply_kernel<double, double>), grid, dim3(bs), 0, st, a);
    else
        hipLaunchKernelGGL((ng_apply_kernel<float, float>), grid, dim3(bs), 0, st, a);
    return hipGetLastError();
}

}  // namespace rt3d
