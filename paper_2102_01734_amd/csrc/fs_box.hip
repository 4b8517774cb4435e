// fs_box.hip -- formal solution on the x,y-periodic box (gfx950).
//
// One workgroup sweeps all characteristics of one (wavelength, direction)
// work item through the grid, layer by layer in the direction of travel
// (top to bottom for mu < 0).  Every thread carries the intensity of R rays in
// registers; all rays of a direction share the visit template, so at visit m
// every lane reads the same template entry (scalar loads) and ray r touches
// voxel r + offset_m.  At a fixed m that map is one-to-one, so after a
// workgroup barrier per visit step the layer's J (and Lambda*) tile in LDS is
// updated without collisions and in a fixed order (bitwise reproducible).
// When the template leaves a layer the tile is added into the workgroup's own
// partial-sum slot in HBM.
//
// Per point (Listing 1 of the paper): gather previous/current/next S and chi
// (step 1-2), optical steps (3), interpolation weights with the linear
// fallback (4) and vacuum fix-up (4a), Lambda* data (4b), exp(-dtau) and the
// intensity update (5).  Optical steps and weights are evaluated in double;
// the recurrence and the J accumulation run in the field type T.
//
// Fields are read from doubly periodic padded copies [Nz][2Ny][2Nx], so the
// address of ray r at visit m is base_r + offset_m with no wrap arithmetic.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fs_box.hpp"

namespace rt3d {

// ---------------------------------------------------------------------------
// double-precision point arithmetic
// ---------------------------------------------------------------------------
__device__ __forceinline__ double seg_depth(double chi, double s)
{
#pragma clang fp contract(off)
    return chi * s;
}

__device__ __forceinline__ double half_sum(double a, double b)
{
#pragma clang fp contract(off)
    return 0.5 * (a + b);
}

__device__ __forceinline__ double rcp_f64(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}

// Attenuation moments over an optical step D >= 0:
//   ex = exp(-D), e0 = 1 - ex, e1 = D - e0, e2 = D^2 - 2 e1.
// Below D = 1/4 e2 comes from its Taylor series 2 D^3 sum_j (-D)^j/(j+3)!,
// and e1, e0, ex follow from it without cancellation.
__device__ __forceinline__ void kernel_moments(double D, double &ex, double &e0, double &e1, double &e2)
{
    if (D < 0.25) {
        double p = 1.0 / 87178291200.0;           // 1/14!
        p = __builtin_fma(-D, p, 1.0 / 6227020800.0);  // 1/13!
        p = __builtin_fma(-D, p, 1.0 / 479001600.0);   // 1/12!
        p = __builtin_fma(-D, p, 1.0 / 39916800.0);    // 1/11!
        p = __builtin_fma(-D, p, 1.0 / 3628800.0);     // 1/10!
        p = __builtin_fma(-D, p, 1.0 / 362880.0);      // 1/9!
        p = __builtin_fma(-D, p, 1.0 / 40320.0);       // 1/8!
        p = __builtin_fma(-D, p, 1.0 / 5040.0);        // 1/7!
        p = __builtin_fma(-D, p, 1.0 / 720.0);         // 1/6!
        p = __builtin_fma(-D, p, 1.0 / 120.0);         // 1/5!
        p = __builtin_fma(-D, p, 1.0 / 24.0);          // 1/4!
        p = __builtin_fma(-D, p, 1.0 / 6.0);           // 1/3!
        const double D2 = D * D;
        e2 = 2.0 * D2 * D * p;
        e1 = 0.5 * (D2 - e2);
        e0 = D - e1;
        ex = 1.0 - e0;
    } else {
        ex = exp(-D);
        e0 = 1.0 - ex;
        e1 = D - e0;
        e2 = D * D - 2.0 * e1;
    }
}

struct PointWeights {
    double a, b, g;  // weights of S_{m-1}, S_m, S_{m+1}
    double ex;       // exp(-D)
    double dlin;     // e1/D: linear-interpolation diagonal
};

// Weights of the segment from the previous point (upwind optical step D) to
// the current one, the downwind step being Dp (ignored when last).
// Parabolic (Lagrange quadratic through the three points integrated against
// exp(-(D-t))), falling back to linear on the last point of a ray, when
// Dp < D/2, or when the parabolic beta would reach 1 (Dp e0 <= D e1 - e2).
// D = 0 is a vacuum segment: no change of the intensity.
__device__ __forceinline__ PointWeights point_weights(double D, double Dp, bool last)
{
    PointWeights w;
    double e0, e1, e2;
    kernel_moments(D, w.ex, e0, e1, e2);
    if (!(D > 0.0)) {
        w.a = w.b = w.g = 0.0;
        w.dlin = 0.0;
        w.ex = 1.0;
        return w;
    }
    const double rD = rcp_f64(D);
    w.dlin = e1 * rD;
    const bool lin = last || (Dp < 0.5 * D) || (Dp * e0 <= D * e1 - e2);
    if (lin) {
        w.a = e0 - w.dlin;
        w.b = w.dlin;
        w.g = 0.0;
    } else {
        const double Ds = D + Dp;
        const double r = rcp_f64(D * Dp * Ds);
        w.a = e0 + (e2 - (D + Ds) * e1) * (Dp * r);
        w.b = (Ds * e1 - e2) * (Ds * r);
        w.g = (e2 - D * e1) * (D * r);
    }
    return w;
}

// ---------------------------------------------------------------------------
// the sweep kernel
// ---------------------------------------------------------------------------
template <typename T, int R, bool WJ, bool WL, bool PARA>
__global__ void __launch_bounds__(1024) fs_box_kernel(FsBoxArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int Nx = a.Nx, Ny = a.Ny;
    const int NxNy = Nx * Ny;
    T *tJ = reinterpret_cast<T *>(smem_raw);
    T *tL = tJ + (WJ ? NxNy : 0);
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;

    for (int i = tid; i < NxNy; i += nthr) {
        if (WJ) tJ[i] = T(0);
        if (WL) tL[i] = T(0);
    }

    // rays of this thread: q = tid + j*nthr, origin (x0, y0)
    int gbase[R];
    int xy0[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int q = tid + j * nthr;
        if (q < NxNy) {
            const int y0 = q / Nx;
            const int x0 = q - y0 * Nx;
            gbase[j] = y0 * (2 * Nx) + x0;
            xy0[j] = x0 | (y0 << 16);
        } else {
            gbase[j] = 0;
            xy0[j] = -1;
        }
    }
    __syncthreads();

    const int it_end = a.wg_begin[blockIdx.x + 1];
    for (int it = a.wg_begin[blockIdx.x]; it < it_end; ++it) {
        const WorkItem item = a.items[it];
        const int lam = item.lambda;
        const int d = item.dir;
        const T *__restrict__ chi = reinterpret_cast<const T *>(a.chi_pad) + (int64_t)lam * a.pad_stride;
        const T *__restrict__ S = reinterpret_cast<const T *>(a.S_pad) + (int64_t)lam * a.pad_stride;
        T *__restrict__ pJ = WJ ? reinterpret_cast<T *>(a.partJ) + (int64_t)item.slot * a.n_vox : nullptr;
        T *__restrict__ pL = WL ? reinterpret_cast<T *>(a.partL) + (int64_t)item.slot * a.n_vox : nullptr;
        const bool first = item.first != 0;
        const int64_t vb = a.dir_vbegin[d];
        const int M = a.dir_M[d];
        const double wmu = a.dir_wmu[d];
        const bool down = a.dir_mu[d] < 0.0;
        const T Ibc = a.I_bc ? reinterpret_cast<const T *>(a.I_bc)[2 * lam + (down ? 0 : 1)] : T(0);
        const int32_t *__restrict__ goff = a.goff + vb;
        const uint32_t *__restrict__ dxy = a.dxy + vb;
        const double *__restrict__ sv = a.s + vb;

        T I[R];
        T gprev[R];
#pragma unroll
        for (int j = 0; j < R; ++j) { I[j] = Ibc; gprev[j] = T(0); }

        int layer = down ? 0 : a.Nz - 1;
        const int dlayer = down ? 1 : -1;

        // sliding window of template entries: previous (p), current (c), next (n)
        int g_p = 0, g_c = goff[0];
        double s_p = 0.0, s_c = sv[0];
        int g_n = M > 1 ? goff[1] : 0;
        double s_n = M > 1 ? sv[1] : 0.0;
        uint32_t w_c = dxy[0];

        for (int m = 0; m < M; ++m) {
            const bool last = (m == M - 1);
            const int di = (int)(w_c & kOffMask);
            const int dj = (int)((w_c >> kOffBits) & kOffMask);
            const T cw = T(wmu * s_c);
#pragma unroll
            for (int j = 0; j < R; ++j) {
                if (xy0[j] < 0) continue;
                const int gb = gbase[j];
                const T chi_c = chi[gb + g_c];
                const T S_c = WJ ? S[gb + g_c] : T(0);
                T dloc = T(0);
                if (m == 0) {
                    // entry half-segment, constant S (Listing 1 step 4a)
                    const double D0 = 0.5 * seg_depth((double)chi_c, s_c);
                    double ex, e0, e1, e2;
                    kernel_moments(D0, ex, e0, e1, e2);
                    if (WJ) I[j] = I[j] * T(ex) + S_c * T(e0);
                    dloc = T(e0);
                } else {
                    const T chi_p = chi[gb + g_p];
                    const T S_p = WJ ? S[gb + g_p] : T(0);
                    T chi_n = T(0), S_n = T(0);
                    if (!last) {
                        chi_n = chi[gb + g_n];
                        if (WJ) S_n = S[gb + g_n];
                    }
                    const double tp = seg_depth((double)chi_p, s_p);
                    const double tc = seg_depth((double)chi_c, s_c);
                    const double D = half_sum(tp, tc);
                    const double Dp = last ? 0.0 : half_sum(tc, seg_depth((double)chi_n, s_n));
                    const PointWeights pw = point_weights(D, Dp, last);
                    const T ex = T(pw.ex);
                    if (WJ) I[j] = I[j] * ex + T(pw.a) * S_p + T(pw.b) * S_c + T(pw.g) * S_n;
                    if (WL) {
                        if (PARA) {
                            dloc = T(pw.b) + gprev[j] * ex;
                            gprev[j] = T(pw.g);
                        } else {
                            dloc = T(pw.dlin);
                        }
                    }
                }
                const int x0 = xy0[j] & 0xffff, y0 = xy0[j] >> 16;
                int xl = x0 + di;
                xl = xl >= Nx ? xl - Nx : xl;
                int yl = y0 + dj;
                yl = yl >= Ny ? yl - Ny : yl;
                const int idx = yl * Nx + xl;
                if (WJ) atomicAdd(&tJ[idx], cw * I[j]);
                if (WL) atomicAdd(&tL[idx], cw * dloc);
            }
            __syncthreads();
            if (w_c & kLayerEnd) {
                const int64_t lo = (int64_t)layer * NxNy;
                for (int i = tid; i < NxNy; i += nthr) {
                    if (WJ) {
                        const T v = tJ[i];
                        tJ[i] = T(0);
                        pJ[lo + i] = first ? v : pJ[lo + i] + v;
                    }
                    if (WL) {
                        const T v = tL[i];
                        tL[i] = T(0);
                        pL[lo + i] = first ? v : pL[lo + i] + v;
                    }
                }
                layer += dlayer;
                __syncthreads();
            }
            // advance the window
            g_p = g_c; s_p = s_c;
            g_c = g_n; s_c = s_n;
            if (m + 1 < M) w_c = dxy[m + 1];
            if (m + 2 < M) { g_n = goff[m + 2]; s_n = sv[m + 2]; }
        }
    }
}

// ---------------------------------------------------------------------------
// host-side dispatch
// ---------------------------------------------------------------------------
template <typename T, int R, bool WJ, bool WL, bool PARA>
static hipError_t launch_r(const FsBoxArgs &a, int n_wg, int nthr, size_t lds, hipStream_t st)
{
    auto k = fs_box_kernel<T, R, WJ, WL, PARA>;
    hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(n_wg), dim3(nthr), lds, st, a);
    return hipGetLastError();
}

template <typename T, bool WJ, bool WL, bool PARA>
static hipError_t launch_flags(const FsBoxArgs &a, int R, int n_wg, int nthr, size_t lds, hipStream_t st)
{
    switch (R) {
    case 1: return launch_r<T, 1, WJ, WL, PARA>(a, n_wg, nthr, lds, st);
    case 2: return launch_r<T, 2, WJ, WL, PARA>(a, n_wg, nthr, lds, st);
    case 4: return launch_r<T, 4, WJ, WL, PARA>(a, n_wg, nthr, lds, st);
    case 8: return launch_r<T, 8, WJ, WL, PARA>(a, n_wg, nthr, lds, st);
    case 12: return launch_r<T, 12, WJ, WL, PARA>(a, n_wg, nthr, lds, st);
    case 17: return launch_r<T, 17, WJ, WL, PARA>(a, n_wg, nthr, lds, st);
    case 24: return launch_r<T, 24, WJ, WL, PARA>(a, n_wg, nthr, lds, st);
    default: return hipErrorInvalidValue;
    }
}

int fs_box_pick_r(int n_rays, int max_threads, int *nthr)
{
    static const int Rs[] = {1, 2, 4, 8, 12, 17, 24};
    for (int R : Rs) {
        const int need = (n_rays + R - 1) / R;
        if (need <= max_threads) {
            int t = ((need + 63) / 64) * 64;
            if (t > max_threads) t = max_threads;
            *nthr = t;
            return R;
        }
    }
    return 0;
}

template <typename T>
static hipError_t launch_t(const FsBoxArgs &a, bool wj, bool wl, bool para, int R, int n_wg, int nthr, size_t lds,
                           hipStream_t st)
{
    if (wj && wl && para) return launch_flags<T, true, true, true>(a, R, n_wg, nthr, lds, st);
    if (wj && wl) return launch_flags<T, true, true, false>(a, R, n_wg, nthr, lds, st);
    if (wj) return launch_flags<T, true, false, false>(a, R, n_wg, nthr, lds, st);
    if (wl && para) return launch_flags<T, false, true, true>(a, R, n_wg, nthr, lds, st);
    if (wl) return launch_flags<T, false, true, false>(a, R, n_wg, nthr, lds, st);
    return hipSuccess;
}

hipError_t fs_box_launch(const FsBoxArgs &a, bool is_double, bool want_j, bool want_l, bool para, int R,
                         int n_wg, int nthr, size_t lds, hipStream_t st)
{
    if (n_wg <= 0) return hipSuccess;
    return is_double ? launch_t<double>(a, want_j, want_l, para, R, n_wg, nthr, lds, st)
                     : launch_t<float>(a, want_j, want_l, para, R, n_wg, nthr, lds, st);
}

template <typename T, int R, bool WJ, bool WL, bool PARA>
static int occ_r(int nthr, size_t lds)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fs_box_kernel<T, R, WJ, WL, PARA>, nthr, lds) != hipSuccess)
        return 0;
    return n;
}

template <typename T, bool WJ, bool WL, bool PARA>
static int occ_flags(int R, int nthr, size_t lds)
{
    switch (R) {
    case 1: return occ_r<T, 1, WJ, WL, PARA>(nthr, lds);
    case 2: return occ_r<T, 2, WJ, WL, PARA>(nthr, lds);
    case 4: return occ_r<T, 4, WJ, WL, PARA>(nthr, lds);
    case 8: return occ_r<T, 8, WJ, WL, PARA>(nthr, lds);
    case 12: return occ_r<T, 12, WJ, WL, PARA>(nthr, lds);
    case 17: return occ_r<T, 17, WJ, WL, PARA>(nthr, lds);
    case 24: return occ_r<T, 24, WJ, WL, PARA>(nthr, lds);
    default: return 0;
    }
}

template <typename T>
static int occ_t(bool wj, bool wl, bool para, int R, int nthr, size_t lds)
{
    if (wj && wl && para) return occ_flags<T, true, true, true>(R, nthr, lds);
    if (wj && wl) return occ_flags<T, true, true, false>(R, nthr, lds);
    if (wj) return occ_flags<T, true, false, false>(R, nthr, lds);
    if (wl && para) return occ_flags<T, false, true, true>(R, nthr, lds);
    if (wl) return occ_flags<T, false, true, false>(R, nthr, lds);
    return 0;
}

int fs_box_occupancy(bool is_double, bool want_j, bool want_l, bool para, int R, int nthr, size_t lds)
{
    return is_double ? occ_t<double>(want_j, want_l, para, R, nthr, lds)
                     : occ_t<float>(want_j, want_l, para, R, nthr, lds);
}

}  // namespace rt3d
