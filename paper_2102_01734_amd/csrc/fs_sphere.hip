// fs_sphere.hip -- formal solution on the spherical grid (gfx950).
//
// Characteristics of a spherical grid are not translates of one another, so
// every one is listed in the geometry cache (visits: voxel, path length,
// averaging weight), bundle-major: 64 characteristics of similar length per
// bundle, visit m of all 64 in one contiguous row.  One thread integrates one
// characteristic for one wavelength with the same per-point arithmetic as the
// box sweep (fs_point.hpp): entry half-segment with constant S, then the
// parabolic / linear recurrence.  The L lanes of a characteristic are L
// wavelengths: they share each cache entry (one broadcast load) and read the
// (chi, S) pairs of one voxel as one contiguous run (voxel-major field).  Each
// visit's w_v,d I_m (and w_v,d times the point's Lambda* term) is stored
// [entry][batch], w_v,d = w_d s_m / (sum of s over the visits of voxel v in
// direction d).  A second kernel sums these per voxel in a fixed CSR order, so
// J is bitwise reproducible and independent of how wavelengths are batched.
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

}  // namespace

template <typename T, typename TG, bool WJ, bool WL, bool PARA>
__global__ void __launch_bounds__(256) fs_sphere_kernel(FsSphereArgs a)
{
    // wavefront -> (bundle, batch group, slice of the bundle); lane -> (characteristic, batch entry)
    const int L = a.L, C = 64 / L;
    const int n_groups = (a.n_batch + L - 1) / L;
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t per_bundle = (int64_t)n_groups * L;
    const int64_t bundle = wave / per_bundle;
    if (bundle >= a.n_bundles) return;
    const int rem = (int)(wave - bundle * per_bundle);
    const int grp = rem / L, slice = rem - grp * L;
    const int c = slice * C + lane / L;
    const int b = grp * L + lane % L;
    if (b >= a.n_batch) return;
    const int len = a.char_len[bundle * 64 + c];
    if (len <= 0) return;
    const int lam = a.lambda_of[b];
    const SPair<T> *__restrict__ F = reinterpret_cast<const SPair<T> *>(a.field) + lam;
    const int ls = a.lam_stride;
    const TG *__restrict__ sv = reinterpret_cast<const TG *>(a.s);
    const TG *__restrict__ wv = reinterpret_cast<const TG *>(a.w);
    const int32_t *__restrict__ vx = a.vox;
    const int nb = a.n_batch;
    T *__restrict__ oJ = WJ ? reinterpret_cast<T *>(a.outJ) + b : nullptr;
    T *__restrict__ oL = WL ? reinterpret_cast<T *>(a.outL) + b : nullptr;
    const int64_t e0 = a.bundle_begin[bundle] + c;  // entry of visit m: e0 + 64 m

    T I0 = T(0);
    if (WJ && a.I_bc) {
        const T *bc = reinterpret_cast<const T *>(a.I_bc) + 3 * lam;
        const double g = a.char_g[bundle * 64 + c];
        I0 = g < 0.0 ? bc[1] : bc[0] + bc[2] * T(g);
    }
    auto pair = [&](int64_t e) { return F[(int64_t)vx[e] * ls]; };

    // first point: entry half-segment with constant S
    SPair<T> fp = pair(e0);
    double tp = seg_depth((double)fp.chi, (double)sv[e0]);
    T I;
    {
        T ex, e0w;
        entry_weights<T, true>(0.5 * tp, ex, e0w);
        I = I0 * ex + fp.S * e0w;
        const T w0 = T(wv[e0]);
        if (WJ) oJ[e0 * nb] = w0 * I;
        if (WL) oL[e0 * nb] = w0 * e0w;
    }
    if (len < 2) return;
    SPair<T> fc = pair(e0 + 64);
    double tc = seg_depth((double)fc.chi, (double)sv[e0 + 64]);
    T gprev = T(0);
    // software pipeline: the (chi, S) pair and path length of a point are read
    // one visit before it is used, its voxel index two visits before
    SPair<T> fq{T(0), T(0)};
    TG sq = TG(0);
    int32_t vq = 0;
    if (len > 2) {
        fq = pair(e0 + 128);
        sq = sv[e0 + 128];
    }
    if (len > 3) vq = vx[e0 + 192];
    for (int m = 1; m < len; ++m) {
        const int64_t e = e0 + 64 * (int64_t)m;
        const bool last = m + 1 == len;
        SPair<T> fn{T(0), T(0)};
        double tn = 0.0;
        if (!last) {
            fn = fq;  // point m + 1
            const TG sn = sq;
            if (m + 2 < len) {
                fq = F[(int64_t)vq * ls];  // point m + 2
                sq = sv[e + 128];
                if (m + 3 < len) vq = vx[e + 192];  // point m + 3
            }
            tn = seg_depth((double)fn.chi, (double)sn);
        }
        const double D = half_sum(tp, tc);
        const double Dp = last ? 0.0 : half_sum(tc, tn);
        const PointW<T> pw = point_weights<T, sizeof(T) == 8, true, true, WL && !PARA>(D, Dp, last);
        const T wk = T(wv[e]);
        if (WJ) {
            I = I * pw.ex + pw.a * fp.S + pw.b * fc.S + (last ? T(0) : pw.g * fn.S);
            oJ[e * nb] = wk * I;
        }
        if (WL) {
            T dloc;
            if (PARA) {
                dloc = pw.b + gprev * pw.ex;
                gprev = pw.g;
            } else {
                dloc = pw.dlin;
            }
            oL[e * nb] = wk * dloc;
        }
        fp = fc;
        tp = tc;
        fc = fn;
        tc = tn;
    }
}

template <typename T, typename TG, bool WJ, bool WL, bool PARA>
static hipError_t launch_t(const FsSphereArgs &a, hipStream_t st)
{
    if (a.n_bundles == 0 || a.n_batch == 0) return hipSuccess;
    const int64_t n_groups = (a.n_batch + a.L - 1) / a.L;
    const int64_t waves = a.n_bundles * n_groups * a.L;
    hipLaunchKernelGGL((fs_sphere_kernel<T, TG, WJ, WL, PARA>), dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st,
                       a);
    return hipGetLastError();
}

template <typename T, typename TG>
static hipError_t launch_flags(const FsSphereArgs &a, bool wj, bool wl, bool para, hipStream_t st)
{
    if (wj && wl && para) return launch_t<T, TG, true, true, true>(a, st);
    if (wj && wl) return launch_t<T, TG, true, true, false>(a, st);
    if (wj) return launch_t<T, TG, true, false, false>(a, st);
    if (wl && para) return launch_t<T, TG, false, true, true>(a, st);
    if (wl) return launch_t<T, TG, false, true, false>(a, st);
    return hipErrorInvalidValue;
}

hipError_t fs_sphere_launch(const FsSphereArgs &a, bool is_double, bool gdouble, bool want_j, bool want_l,
                            bool parabolic_lstar, hipStream_t st)
{
    if (a.L != 1 && a.L != 2 && a.L != 4 && a.L != 8 && a.L != 16) return hipErrorInvalidValue;
    if (is_double && gdouble) return launch_flags<double, double>(a, want_j, want_l, parabolic_lstar, st);
    if (is_double) return launch_flags<double, float>(a, want_j, want_l, parabolic_lstar, st);
    if (!gdouble) return launch_flags<float, float>(a, want_j, want_l, parabolic_lstar, st);
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// fixed-order gather of the per-visit contributions into voxels
// ---------------------------------------------------------------------------
template <typename TS, typename TD>
__global__ void __launch_bounds__(256) sphere_gather_kernel(const TS *__restrict__ src, const int32_t *__restrict__ row,
                                                            const int32_t *__restrict__ idx, int64_t n_vox, int nb,
                                                            TD *__restrict__ dst, int accumulate)
{
    // thread -> (voxel, batch entry), batch fastest: the entries of one voxel are read as contiguous rows
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n_vox * nb) return;
    const int64_t v = id / nb;
    const int b = (int)(id - v * nb);
    double acc = 0.0;
    const int32_t e = row[v + 1];
    int32_t k = row[v];
    // eight visits' loads in flight at a time; the sum keeps the order of k
    constexpr int U = 8;
    for (; k + U <= e; k += U) {
        int64_t i[U];
        TS s[U];
#pragma unroll
        for (int u = 0; u < U; ++u) i[u] = idx[k + u];
#pragma unroll
        for (int u = 0; u < U; ++u) s[u] = src[i[u] * nb + b];
#pragma unroll
        for (int u = 0; u < U; ++u) acc += (double)s[u];
    }
    for (; k < e; ++k) acc += (double)src[(int64_t)idx[k] * nb + b];
    TD *d = dst + (int64_t)b * n_vox + v;
    *d = accumulate ? (TD)((double)*d + acc) : (TD)acc;
}

template <typename TS, typename TD>
static hipError_t gather_t(const void *src, const int32_t *row, const int32_t *idx, int64_t n_vox, int n_batch,
                           void *dst, bool accumulate, hipStream_t st)
{
    if (n_vox == 0 || n_batch == 0) return hipSuccess;
    const int64_t n = n_vox * n_batch;
    hipLaunchKernelGGL((sphere_gather_kernel<TS, TD>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       reinterpret_cast<const TS *>(src), row, idx, n_vox, n_batch, reinterpret_cast<TD *>(dst),
                       accumulate ? 1 : 0);
    return hipGetLastError();
}

hipError_t sphere_gather(const void *src, bool src_double, const int32_t *row, const int32_t *idx, int64_t n_vox,
                         int n_batch, void *dst, bool dst_double, bool accumulate, hipStream_t st)
{
    if (src_double && dst_double) return gather_t<double, double>(src, row, idx, n_vox, n_batch, dst, accumulate, st);
    if (src_double) return gather_t<double, float>(src, row, idx, n_vox, n_batch, dst, accumulate, st);
    if (dst_double) return gather_t<float, double>(src, row, idx, n_vox, n_batch, dst, accumulate, st);
    return gather_t<float, float>(src, row, idx, n_vox, n_batch, dst, accumulate, st);
}

}  // namespace rt3d
