// fs_sphere.hip -- formal solution on the spherical grid (gfx950).
//
// Characteristics of a spherical grid are not translates of one another, so
// every one is listed in the geometry cache (visits: voxel, path length,
// averaging weight).  One thread integrates one characteristic of one
// wavelength with the same per-point arithmetic as the box sweep
// (fs_point.hpp): entry half-segment with constant S, then the parabolic /
// linear recurrence.  It writes w_v,d I_m (and w_v,d times the point's
// Lambda* entry) for every visit, where w_v,d = w_d s_m / (sum of s over the
// visits of voxel v in direction d).  A second kernel sums these per voxel
// over a fixed CSR order, so J is bitwise reproducible and independent of how
// wavelengths are batched.
//
// Boundary intensities (Sec. 3.2 of the paper): characteristics entering
// from outside start with I_out plus the irradiation of the point source,
// J_sub times the characteristic's precomputed factor; characteristics that
// leave the opaque core start with I_core (the diffusion-limit value, B at
// the core for constant B).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fs_point.hpp"
#include "fs_sphere.hpp"

namespace rt3d {

namespace {

template <typename T>
struct SPair {
    T chi, S;
};

template <typename T>
__device__ __forceinline__ SPair<T> load_pair(const SPair<T> *__restrict__ f, int32_t v)
{
    return f[v];
}

}  // namespace

template <typename T, typename TG, bool WJ, bool WL, bool PARA>
__global__ void __launch_bounds__(256) fs_sphere_kernel(FsSphereArgs a)
{
    const int b = blockIdx.y;
    const int64_t c = a.char0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.char0 + a.n_chars) return;
    const int lam = a.lambda_of[b];
    const SPair<T> *__restrict__ F = reinterpret_cast<const SPair<T> *>(a.field) + (int64_t)lam * a.n_vox;
    const TG *__restrict__ sv = reinterpret_cast<const TG *>(a.s);
    const TG *__restrict__ wv = reinterpret_cast<const TG *>(a.w);
    const int32_t *__restrict__ vx = a.vox;
    T *__restrict__ oJ = WJ ? reinterpret_cast<T *>(a.outJ) + (int64_t)b * a.out_stride - a.visit0 : nullptr;
    T *__restrict__ oL = WL ? reinterpret_cast<T *>(a.outL) + (int64_t)b * a.out_stride - a.visit0 : nullptr;

    const int64_t k0 = a.char_begin[c], k1 = a.char_begin[c + 1];
    T I0 = T(0);
    if (WJ && a.I_bc) {
        const T *bc = reinterpret_cast<const T *>(a.I_bc) + 3 * lam;
        const double g = a.char_g[c];
        I0 = g < 0.0 ? bc[1] : bc[0] + bc[2] * T(g);
    }

    // first point: entry half-segment with constant S
    SPair<T> fp = load_pair<T>(F, vx[k0]);
    double tp = seg_depth((double)fp.chi, (double)sv[k0]);
    T I;
    {
        T ex, e0;
        entry_weights<T>(0.5 * tp, ex, e0);
        I = I0 * ex + fp.S * e0;
        const T w0 = T(wv[k0]);
        if (WJ) oJ[k0] = w0 * I;
        if (WL) oL[k0] = w0 * e0;
    }
    if (k0 + 1 >= k1) return;
    SPair<T> fc = load_pair<T>(F, vx[k0 + 1]);
    double tc = seg_depth((double)fc.chi, (double)sv[k0 + 1]);
    T gprev = T(0);
    for (int64_t k = k0 + 1; k < k1; ++k) {
        const bool last = k + 1 == k1;
        SPair<T> fn{T(0), T(0)};
        double tn = 0.0;
        if (!last) {
            fn = load_pair<T>(F, vx[k + 1]);
            tn = seg_depth((double)fn.chi, (double)sv[k + 1]);
        }
        const double D = half_sum(tp, tc);
        const double Dp = last ? 0.0 : half_sum(tc, tn);
        const PointW<T> pw = point_weights<T>(D, Dp, last);
        const T wk = T(wv[k]);
        if (WJ) {
            I = I * pw.ex + pw.a * fp.S + pw.b * fc.S + (last ? T(0) : pw.g * fn.S);
            oJ[k] = wk * I;
        }
        if (WL) {
            T dloc;
            if (PARA) {
                dloc = pw.b + gprev * pw.ex;
                gprev = pw.g;
            } else {
                dloc = pw.dlin;
            }
            oL[k] = wk * dloc;
        }
        fp = fc;
        tp = tc;
        fc = fn;
        tc = tn;
    }
}

template <typename T, typename TG, bool WJ, bool WL, bool PARA>
static hipError_t launch_t(const FsSphereArgs &a, int n_batch, hipStream_t st)
{
    if (a.n_chars == 0 || n_batch == 0) return hipSuccess;
    const int bs = 256;
    dim3 grid((unsigned)((a.n_chars + bs - 1) / bs), (unsigned)n_batch);
    hipLaunchKernelGGL((fs_sphere_kernel<T, TG, WJ, WL, PARA>), grid, dim3(bs), 0, st, a);
    return hipGetLastError();
}

template <typename T, typename TG>
static hipError_t launch_flags(const FsSphereArgs &a, bool wj, bool wl, bool para, int n_batch, hipStream_t st)
{
    if (wj && wl && para) return launch_t<T, TG, true, true, true>(a, n_batch, st);
    if (wj && wl) return launch_t<T, TG, true, true, false>(a, n_batch, st);
    if (wj) return launch_t<T, TG, true, false, false>(a, n_batch, st);
    if (wl && para) return launch_t<T, TG, false, true, true>(a, n_batch, st);
    if (wl) return launch_t<T, TG, false, true, false>(a, n_batch, st);
    return hipErrorInvalidValue;
}

hipError_t fs_sphere_launch(const FsSphereArgs &a, bool is_double, bool gdouble, bool want_j, bool want_l,
                            bool parabolic_lstar, int n_batch, hipStream_t st)
{
    if (is_double && gdouble) return launch_flags<double, double>(a, want_j, want_l, parabolic_lstar, n_batch, st);
    if (is_double) return launch_flags<double, float>(a, want_j, want_l, parabolic_lstar, n_batch, st);
    if (!gdouble) return launch_flags<float, float>(a, want_j, want_l, parabolic_lstar, n_batch, st);
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// fixed-order gather of the per-visit contributions into voxels
// ---------------------------------------------------------------------------
template <typename TS, typename TD>
__global__ void __launch_bounds__(256) sphere_gather_kernel(const TS *__restrict__ src, int64_t src_stride,
                                                            const int32_t *__restrict__ row,
                                                            const int32_t *__restrict__ idx, int64_t n_vox,
                                                            TD *__restrict__ dst, int accumulate)
{
    const int b = blockIdx.y;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n_vox) return;
    const TS *s = src + (int64_t)b * src_stride;
    double acc = 0.0;
    const int32_t e = row[v + 1];
    for (int32_t k = row[v]; k < e; ++k) acc += (double)s[idx[k]];
    TD *d = dst + (int64_t)b * n_vox + v;
    *d = accumulate ? (TD)((double)*d + acc) : (TD)acc;
}

template <typename TS, typename TD>
static hipError_t gather_t(const void *src, int64_t src_stride, const int32_t *row, const int32_t *idx,
                           int64_t n_vox, int n_batch, void *dst, bool accumulate, hipStream_t st)
{
    if (n_vox == 0 || n_batch == 0) return hipSuccess;
    const int bs = 256;
    dim3 grid((unsigned)((n_vox + bs - 1) / bs), (unsigned)n_batch);
    hipLaunchKernelGGL((sphere_gather_kernel<TS, TD>), grid, dim3(bs), 0, st, reinterpret_cast<const TS *>(src),
                       src_stride, row, idx, n_vox, reinterpret_cast<TD *>(dst), accumulate ? 1 : 0);
    return hipGetLastError();
}

hipError_t sphere_gather(const void *src, bool src_double, int64_t src_stride, const int32_t *row, const int32_t *idx,
                         int64_t n_vox, int n_batch, void *dst, bool dst_double, bool accumulate, hipStream_t st)
{
    if (src_double && dst_double)
        return gather_t<double, double>(src, src_stride, row, idx, n_vox, n_batch, dst, accumulate, st);
    if (src_double) return gather_t<double, float>(src, src_stride, row, idx, n_vox, n_batch, dst, accumulate, st);
    if (dst_double) return gather_t<float, double>(src, src_stride, row, idx, n_vox, n_batch, dst, accumulate, st);
    return gather_t<float, float>(src, src_stride, row, idx, n_vox, n_batch, dst, accumulate, st);
}

}  // namespace rt3d
