// lstar_nl.hip -- nearest-neighbour Lambda* of the box (gfx950) and the
// Jacobi sweeps of the operator-splitting system it defines.
//
// The paper's production runs use a non-local Lambda* (Sec. 2, Sec. 3: the
// nearest-neighbour operator, built in the first iteration, with the OS
// system [1 - Lambda*(1-eps)] J_new = J_fs - Lambda*(1-eps) J_old solved by
// Jacobi, Gauss-Seidel or BiCGStab).  Here Lambda* is the exact restriction
// of an operator (the linear-interpolation operator by default, or the
// formal solution itself) to the 27 neighbours of each voxel, as far as a
// characteristic carries it directly from the neighbour to the voxel.
//
// Along one characteristic the intensity is linear in S:
//   I_m = I_{m-1} ex_m + a_m S_{m-1} + b_m S_m + g_m S_{m+1}.
// The derivatives G_j = dI_m / dS(point m - j), j = -1..3, obey
//   G_-1 = g_m,  G_0 = ex_m G_-1' + b_m,  G_1 = ex_m G_0' + a_m,
//   G_2 = ex_m G_1',  G_3 = ex_m G_2'           (' = values at point m - 1),
// and a voxel more than three points upstream cannot be a neighbour of the
// voxel of point m (each step of a straight ray moves some coordinate by
// one and never back), so these five numbers give every neighbour's
// element; G_0 is the local diagonal of the diagonal Lambda*.  Each point
// adds w_d |mu_d| s_m G_j to component c_j of its voxel (the path-length
// weighted mean over the voxel's visits, sum of s = 1/|mu_d|).
//
// The sums are fixed-point integers (2^-52 units): integer addition is
// associative, so the result is bitwise independent of the order in which
// contributions arrive.  |sum| <= 1 per element, so 2^52 leaves ample
// headroom below 2^63.
//
// Row-window kernel: a workgroup takes one wavelength, one direction and a
// bundle of H consecutive ray rows (all Nx rays of each row), its rays in
// lockstep.  At visit m every ray of bundle row yr adds to target row
// yr + brow_m of the current layer (brow: the visit's row above the lowest
// row the template reaches in that layer), so the live target rows form a
// window of H rows that moves by at most one row per visit and only one way
// within a layer.  The window lives in LDS as H + 1 circular rows of Nx
// words for each stencil component the direction uses; contributions go in
// with LDS integer atomics.  A row that leaves the window (and every live row
// at the end of a layer) is added to HBM with one 64-bit atomic per non-zero
// word and cleared.  Layers too wide for such a tile fall back to one thread
// per characteristic with a global atomic per contribution.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "ali.hpp"
#include "fs_point.hpp"
#include "lstar_nl.hpp"
#include "rt_internal.hpp"

namespace rt3d {

// One contribution w G in fixed point, round(w G 2^52) as a signed 64-bit
// integer (ties to even).
__device__ __forceinline__ long long fix52(double cw52, double G) { return __double2ll_rn(cw52 * G); }

template <typename G, bool PARA>
__global__ void __launch_bounds__(256) lstar_stencil_kernel(StencilArgs a)
{
    const int Nx = a.Nx, Ny = a.Ny;
    const int NxNy = Nx * Ny;
    const int q = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (q >= NxNy) return;
    const int d = blockIdx.y;
    const int lam = a.lambda_of[blockIdx.z];
    const int y0 = q / Nx, x0 = q - y0 * Nx;
    const G *__restrict__ chi = reinterpret_cast<const G *>(a.chi) + (int64_t)lam * a.n_vox;
    unsigned long long *__restrict__ acc = a.acc + (int64_t)lam * kStencil * a.n_vox;
    const int64_t vb = a.dir_vbegin[d];
    const int M = a.dir_M[d];
    const double wmu = a.dir_wmu[d];
    const int dl = a.dir_mu[d] < 0.0 ? 1 : -1;
    const uint32_t *__restrict__ dxy = a.dxy + vb;
    const double *__restrict__ sv = a.s + vb;
    const uint32_t *__restrict__ comp = a.comp + vb;

    auto voxel = [&](uint32_t w, int k) -> int64_t {
        int x = x0 + (int)(w & kOffMask);
        if (x >= Nx) x -= Nx;
        int y = y0 + (int)((w >> kOffBits) & kOffMask);
        if (y >= Ny) y -= Ny;
        return (int64_t)k * NxNy + (int64_t)y * Nx + x;
    };
    // adds w |mu| s_m G_j to component c_j of voxel v (j = -1..3)
    auto add = [&](int64_t v, double cw, uint32_t comps, const double (&Gv)[5]) {
        const double cw52 = cw * 0x1p52;
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            if (!PARA && j == 0) continue;  // no downwind weight in the linear operator
            const uint32_t c = (comps >> (6 * j)) & 63u;
            if (c == kNoComp || (a.skip_centre && c == (uint32_t)kStencilCentre)) continue;
            const long long f = fix52(cw52, Gv[j]);
            if (f != 0) atomicAdd(&acc[(int64_t)c * a.n_vox + v], (unsigned long long)f);
        }
    };

    // visit 0 and the look-ahead to visit 1; the layer advances after each layer-end visit
    int k_cur = dl > 0 ? 0 : a.Nz - 1;
    uint32_t w_cur = dxy[0];
    int64_t v_cur = voxel(w_cur, k_cur);
    double t_cur = seg_depth((double)chi[v_cur], sv[0]);
    int k_nxt = k_cur + ((w_cur & kLayerEnd) ? dl : 0);
    uint32_t w_nxt = 0;
    int64_t v_nxt = 0;
    double t_nxt = 0.0;
    if (M > 1) {
        w_nxt = dxy[1];
        v_nxt = voxel(w_nxt, k_nxt);
        t_nxt = seg_depth((double)chi[v_nxt], sv[1]);
    }
    double Gv[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // G_-1, G_0, G_1, G_2, G_3
    {
        double ex0, e00;
        entry_weights<double>(0.5 * t_cur, ex0, e00);
        Gv[1] = e00;
        add(v_cur, wmu * sv[0], comp[0], Gv);
    }
    for (int m = 1; m < M; ++m) {
        const double t_prev = t_cur;
        w_cur = w_nxt;
        v_cur = v_nxt;
        t_cur = t_nxt;
        k_cur = k_nxt;
        k_nxt = k_cur + ((w_cur & kLayerEnd) ? dl : 0);
        const bool last = m + 1 == M;
        if (!last) {
            w_nxt = dxy[m + 1];
            v_nxt = voxel(w_nxt, k_nxt);
            t_nxt = seg_depth((double)chi[v_nxt], sv[m + 1]);
        }
        const double D = half_sum(t_prev, t_cur);
        const double Dp = last ? 0.0 : half_sum(t_cur, t_nxt);
        double ex, wa, wb, wg;
        // single-precision grids keep the stencil in float: the shorter
        // moment forms of the float sweep suffice there
        if (PARA) {
            const PointW<double> pw = point_weights<double, sizeof(G) == 8>(D, Dp, last);
            ex = pw.ex; wa = pw.a; wb = pw.b; wg = pw.g;
        } else {
            const double Dv = D < kMinStep ? kMinStep : D;
            double e0, e1, e2;
            kernel_moments<sizeof(G) == 8>(Dv, ex, e0, e1, e2);
            wb = e1 * rcp_f64<sizeof(G) == 8>(Dv);
            wa = e0 - wb;
            wg = 0.0;
        }
        Gv[4] = ex * Gv[3];
        Gv[3] = ex * Gv[2];
        Gv[2] = ex * Gv[1] + wa;
        Gv[1] = ex * Gv[0] + wb;
        Gv[0] = wg;
        add(v_cur, wmu * sv[m], comp[m], Gv);
    }
}

constexpr int kFlushWords = 4;

template <typename G, bool PARA, int R>
__global__ void __launch_bounds__(1024) lstar_stencil_rows_kernel(StencilArgs a)
{
    extern __shared__ unsigned long long tile[];  // [plane][H + 1 circular rows][Nx]
    const int Nx = a.Nx, Ny = a.Ny, H = a.rows, W = H + 1, P = a.planes;
    const int64_t NxNy = (int64_t)Nx * Ny;
    const int nthr = (int)blockDim.x, tid = (int)threadIdx.x;
    const int d = blockIdx.y;
    const int lam = a.lambda_of[blockIdx.z];
    const int yb = (int)blockIdx.x * H;
    const G *__restrict__ chi = reinterpret_cast<const G *>(a.chi) + (int64_t)lam * a.n_vox;
    unsigned long long *__restrict__ acc = a.acc + (int64_t)lam * kStencil * a.n_vox;
    const int64_t vb = a.dir_vbegin[d];
    const int M = a.dir_M[d];
    const double wmu = a.dir_wmu[d];
    const int dl = a.dir_mu[d] < 0.0 ? 1 : -1;
    const uint32_t *__restrict__ dxy = a.dxy + vb;
    const double *__restrict__ sv = a.s + vb;
    const uint32_t *__restrict__ comp = a.comp + vb;
    const int32_t *__restrict__ brow = a.brow + vb;
    const int32_t *__restrict__ plane_of = a.dir_plane + (int64_t)d * kPlaneStride;
    const int32_t *__restrict__ comp_of = plane_of + 32;

    __shared__ int64_t coff[kStencil];  // plane -> offset of its component in the sums
    for (int i = tid; i < P * W * Nx; i += nthr) tile[i] = 0;
    if (tid < P) coff[tid] = comp_of[tid] >= 0 ? (int64_t)comp_of[tid] * a.n_vox : 0;
    const int fdp = nthr / Nx, fdx = nthr - fdp * Nx;  // flush stride in planes and columns
    const int fp0 = tid / Nx, fx0 = tid - fp0 * Nx;

    // ray slots: slot tid + r nthr is ray (x0, yb + yr) of the bundle
    int x0[R], y0[R], yr[R];
    bool act[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int l = tid + r * nthr;
        yr[r] = l / Nx;
        x0[r] = l - yr[r] * Nx;
        y0[r] = yb + yr[r];
        act[r] = yr[r] < H && y0[r] < Ny;
        if (!act[r]) { x0[r] = 0; y0[r] = 0; yr[r] = 0; }  // follows ray (0, 0) without adding
    }
    auto col = [&](int x, uint32_t w) { x += (int)(w & kOffMask); return x >= Nx ? x - Nx : x; };
    auto row = [&](int y, uint32_t w) { y += (int)((w >> kOffBits) & kOffMask); return y >= Ny ? y - Ny : y; };
    // first absolute row of the window's relative row 0 in the layer of visit word w at relative row br
    auto row_base = [&](uint32_t w, int br) {
        int j = ((int)((w >> kOffBits) & kOffMask) - br) % Ny;
        return j < 0 ? j + Ny : j;
    };

    int k_cur = dl > 0 ? 0 : a.Nz - 1;
    uint32_t w_cur = dxy[0];
    int br_cur = brow[0];
    int k_nxt = k_cur + ((w_cur & kLayerEnd) ? dl : 0);
    uint32_t w_nxt = M > 1 ? dxy[1] : 0u;
    int slot[R], x_cur[R], x_nxt[R];
    double t_cur[R], t_nxt[R], Gv[R][5];  // G_-1, G_0, G_1, G_2, G_3 per ray
#pragma unroll
    for (int r = 0; r < R; ++r) {
        slot[r] = (yr[r] + br_cur) % W;
        x_cur[r] = col(x0[r], w_cur);
        t_cur[r] = seg_depth((double)chi[(int64_t)k_cur * NxNy + (int64_t)row(y0[r], w_cur) * Nx + x_cur[r]], sv[0]);
        x_nxt[r] = 0;
        t_nxt[r] = 0.0;
        if (M > 1) {
            x_nxt[r] = col(x0[r], w_nxt);
            t_nxt[r] = seg_depth((double)chi[(int64_t)k_nxt * NxNy + (int64_t)row(y0[r], w_nxt) * Nx + x_nxt[r]],
                                 sv[1]);
        }
#pragma unroll
        for (int j = 0; j < 5; ++j) Gv[r][j] = 0.0;
    }
    __syncthreads();  // tile cleared, component offsets set
    // a row of P x Nx words that fits kFlushWords words a thread is flushed
    // from a per-thread list of tile and sum offsets, its LDS reads issued
    // together; wider rows by a strided loop
    const bool f_list = P * Nx <= kFlushWords * nthr;
    int f_lds[kFlushWords];
    int64_t f_glob[kFlushWords];
#pragma unroll
    for (int j = 0; j < kFlushWords; ++j) {
        const int i = tid + j * nthr;
        const int p = i / Nx, x = i - p * Nx;
        f_lds[j] = p < P ? p * W * Nx + x : -1;
        f_glob[j] = p < P ? coff[p] + x : 0;
    }

    // adds w |mu| s_m G_j of every active ray to its target word of component c_j
    auto add = [&](double cw, uint32_t comps) {
        const double cw52 = cw * 0x1p52;
        int word[R];  // the ray's target word in plane 0
#pragma unroll
        for (int r = 0; r < R; ++r) word[r] = slot[r] * Nx + x_cur[r];
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            if (!PARA && j == 0) continue;  // no downwind weight in the linear operator
            const uint32_t c = (comps >> (6 * j)) & 63u;
            if (c == kNoComp) continue;
            const int p = plane_of[c];
            if (p < 0) continue;
            unsigned long long *plane = tile + p * W * Nx;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const long long f = fix52(cw52, Gv[r][j]);
                if (act[r] && f != 0) atomicAdd(&plane[word[r]], (unsigned long long)f);
            }
        }
    };
    // adds relative row rel of layer k (row 0 at absolute row jb) to HBM and
    // clears it; thread tid takes the words tid, tid + nthr, ... of the row's
    // P x Nx words (plane-major), stepping plane and column without division
    auto flush = [&](int rel, int k, int jb) {
        unsigned long long *trow = tile + (rel % W) * Nx;
        const int64_t base = (int64_t)k * NxNy + (int64_t)((yb + jb + rel) % Ny) * Nx;
        if (f_list) {
            unsigned long long v[kFlushWords];
#pragma unroll
            for (int j = 0; j < kFlushWords; ++j) v[j] = f_lds[j] >= 0 ? trow[f_lds[j]] : 0ull;
#pragma unroll
            for (int j = 0; j < kFlushWords; ++j)
                if (v[j] != 0ull) {
                    trow[f_lds[j]] = 0ull;
                    atomicAdd(&acc[f_glob[j] + base], v[j]);
                }
            return;
        }
        int p = fp0, x = fx0;
        while (p < P) {
            unsigned long long *t = trow + p * W * Nx + x;
            const unsigned long long v = *t;
            if (v != 0ull) {
                *t = 0ull;
                atomicAdd(&acc[coff[p] + base + x], v);
            }
            x += fdx;
            p += fdp;
            if (x >= Nx) {
                x -= Nx;
                ++p;
            }
        }
    };
    // after visit m: at a layer end every live row leaves; else the row that the next visit no longer reaches
    auto advance = [&](int m) {
        if (w_cur & kLayerEnd) {
            __syncthreads();
            const int jb = row_base(w_cur, br_cur);
            for (int rr = 0; rr < H; ++rr) flush(br_cur + rr, k_cur, jb);
            __syncthreads();
            if (m + 1 < M) {
                const int br_n = brow[m + 1];
#pragma unroll
                for (int r = 0; r < R; ++r) slot[r] = (yr[r] + br_n) % W;
            }
            return;
        }
        const int br_n = brow[m + 1];
        if (br_n == br_cur) return;
        __syncthreads();
        const bool up = br_n > br_cur;
        flush(up ? br_cur : br_cur + H - 1, k_cur, row_base(w_cur, br_cur));
#pragma unroll
        for (int r = 0; r < R; ++r) slot[r] = up ? (slot[r] + 1 == W ? 0 : slot[r] + 1) : (slot[r] == 0 ? W - 1 : slot[r] - 1);
    };

#pragma unroll
    for (int r = 0; r < R; ++r) {
        double ex0, e00;
        entry_weights<double>(0.5 * t_cur[r], ex0, e00);
        Gv[r][1] = e00;
    }
    add(wmu * sv[0], comp[0]);
    advance(0);
    br_cur = M > 1 ? brow[1] : br_cur;
    for (int m = 1; m < M; ++m) {
        w_cur = w_nxt;
        k_cur = k_nxt;
        k_nxt = k_cur + ((w_cur & kLayerEnd) ? dl : 0);
        const bool last = m + 1 == M;
        if (!last) w_nxt = dxy[m + 1];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double t_prev = t_cur[r];
            x_cur[r] = x_nxt[r];
            t_cur[r] = t_nxt[r];
            if (!last) {
                x_nxt[r] = col(x0[r], w_nxt);
                t_nxt[r] = seg_depth(
                    (double)chi[(int64_t)k_nxt * NxNy + (int64_t)row(y0[r], w_nxt) * Nx + x_nxt[r]], sv[m + 1]);
            }
            const double D = half_sum(t_prev, t_cur[r]);
            const double Dp = last ? 0.0 : half_sum(t_cur[r], t_nxt[r]);
            double ex, wa, wb, wg;
            if (PARA) {
                const PointW<double> pw = point_weights<double, sizeof(G) == 8>(D, Dp, last);
                ex = pw.ex; wa = pw.a; wb = pw.b; wg = pw.g;
            } else {
                const double Dv = D < kMinStep ? kMinStep : D;
                double e0, e1, e2;
                kernel_moments<sizeof(G) == 8>(Dv, ex, e0, e1, e2);
                wb = e1 * rcp_f64<sizeof(G) == 8>(Dv);
                wa = e0 - wb;
                wg = 0.0;
            }
            Gv[r][4] = ex * Gv[r][3];
            Gv[r][3] = ex * Gv[r][2];
            Gv[r][2] = ex * Gv[r][1] + wa;
            Gv[r][1] = ex * Gv[r][0] + wb;
            Gv[r][0] = wg;
        }
        add(wmu * sv[m], comp[m]);
        advance(m);
        if (!last) br_cur = brow[m + 1];
    }
}

// Tile rows per workgroup for the row-window kernel: about 800 rays (two per
// thread), within half the LDS (two workgroups per CU) where possible;
// measured on a 129 x 129 layer against 4..16 rows and one to four rays per
// thread, on both operators.  The bundles are then evened out.  0 when not
// even one row fits.
static int stencil_rows(const StencilArgs &a, size_t max_lds)
{
    const size_t row_bytes = (size_t)a.planes * a.Nx * 8;
    const size_t fixed = 256;  // the kernel's static LDS (component offsets)
    if (row_bytes == 0 || max_lds < 2 * fixed || a.Nx > 2048) return 0;
    int h = std::max(1, (800 + a.Nx / 2) / a.Nx);
    const int fit2 = (int)((max_lds / 2 - fixed) / row_bytes) - 1;
    const int fit1 = (int)((max_lds - fixed) / row_bytes) - 1;
    h = std::min(h, fit2 >= 1 ? fit2 : fit1);
    h = std::min(h, a.Ny);
    if (h < 1) return 0;
    const int nb = (a.Ny + h - 1) / h;
    return (a.Ny + nb - 1) / nb;
}

template <typename G, bool PARA, int R>
static hipError_t launch_rows(const StencilArgs &a, int n_dir, int n_batch, hipStream_t st)
{
    const int rays = a.rows * a.Nx;
    const int nthr = ((rays + R - 1) / R + 63) / 64 * 64;
    const size_t lds = (size_t)a.planes * (a.rows + 1) * a.Nx * 8;
    auto k = lstar_stencil_rows_kernel<G, PARA, R>;
    hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    dim3 grid((unsigned)((a.Ny + a.rows - 1) / a.rows), (unsigned)n_dir, (unsigned)n_batch);
    hipLaunchKernelGGL(k, grid, dim3(nthr), lds, st, a);
    return hipGetLastError();
}

template <typename G, bool PARA>
static hipError_t launch_rows_r(const StencilArgs &a, int n_dir, int n_batch, hipStream_t st)
{
    if (a.rows * a.Nx <= 512) return launch_rows<G, PARA, 1>(a, n_dir, n_batch, st);
    return launch_rows<G, PARA, 2>(a, n_dir, n_batch, st);
}

hipError_t lstar_stencil_accumulate(const StencilArgs &a0, bool grid_double, bool parabolic, int n_dir, int n_batch,
                                    size_t max_lds, hipStream_t st)
{
    if (n_dir <= 0 || n_batch <= 0) return hipSuccess;
    if (a0.dir_plane && a0.brow) {
        StencilArgs a = a0;
        a.rows = a.planes > 0 ? stencil_rows(a, max_lds) : 0;
        if (a.planes == 0) return hipSuccess;  // no component is ever added
        if (a.rows > 0) {
            if (grid_double)
                return parabolic ? launch_rows_r<double, true>(a, n_dir, n_batch, st)
                                 : launch_rows_r<double, false>(a, n_dir, n_batch, st);
            return parabolic ? launch_rows_r<float, true>(a, n_dir, n_batch, st)
                             : launch_rows_r<float, false>(a, n_dir, n_batch, st);
        }
    }
    const StencilArgs &a = a0;
    const int NxNy = a.Nx * a.Ny;
    dim3 grid((unsigned)((NxNy + 255) / 256), (unsigned)n_dir, (unsigned)n_batch);
    if (grid_double) {
        if (parabolic) hipLaunchKernelGGL((lstar_stencil_kernel<double, true>), grid, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((lstar_stencil_kernel<double, false>), grid, dim3(256), 0, st, a);
    } else {
        if (parabolic) hipLaunchKernelGGL((lstar_stencil_kernel<float, true>), grid, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((lstar_stencil_kernel<float, false>), grid, dim3(256), 0, st, a);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// spherical grid: one thread per (characteristic, batch entry)
// ---------------------------------------------------------------------------
template <typename G, typename TG, bool PARA>
__global__ void __launch_bounds__(256) lstar_stencil_sphere_kernel(SphereStencilArgs a)
{
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int c = threadIdx.x & 63;
    const int64_t bundle = wave / a.n_batch;
    if (bundle >= a.n_bundles) return;
    const int b = (int)(wave - bundle * a.n_batch);
    const int len = a.char_len[bundle * 64 + c];
    if (len <= 0) return;
    const int lam = a.lambda_of[b];
    const G *__restrict__ chi = reinterpret_cast<const G *>(a.chi) + (int64_t)lam * a.n_vox;
    unsigned long long *__restrict__ acc = a.acc + (int64_t)lam * kStencil * a.n_vox;
    const TG *__restrict__ sv = reinterpret_cast<const TG *>(a.s);
    const TG *__restrict__ wv = reinterpret_cast<const TG *>(a.w);
    const int64_t e0 = a.bundle_begin[bundle] + c;
    const int Nr = a.Nr, Nt = a.Nt, Np = a.Np;

    // voxel coordinates of the points m+1, m, m-1, m-2, m-3 (slot j+1 for point m-j)
    int vr[5], vt[5], vp[5], vv[5];
    auto set = [&](int slot, int v) {
        vv[slot] = v;
        vr[slot] = v % Nr;
        const int q = v / Nr;
        vt[slot] = q % Nt;
        vp[slot] = q / Nt;
    };
#pragma unroll
    for (int j = 0; j < 5; ++j) { vv[j] = -1; vr[j] = vt[j] = vp[j] = 0; }
    // adds w G_j for every point m-j (slot j+1) that is an index neighbour of point m (slot 1)
    auto add = [&](double cw, const double (&Gv)[5]) {
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            if (!PARA && j == 0) continue;  // no downwind weight in the linear operator
            if (vv[j] < 0) continue;
            const int dr = vr[j] - vr[1], dt = vt[j] - vt[1];
            int dp = vp[j] - vp[1];
            dp = dp < 0 ? dp + Np : dp;
            dp = dp == Np - 1 ? -1 : dp;
            if (dr < -1 || dr > 1 || dt < -1 || dt > 1 || dp > 1) continue;
            const int comp = (dp + 1) * 9 + (dt + 1) * 3 + (dr + 1);
            if (a.skip_centre && comp == kStencilCentre) continue;
            const long long f = fix52(cw * 0x1p52, Gv[j]);
            if (f != 0) atomicAdd(&acc[(int64_t)comp * a.n_vox + vv[1]], (unsigned long long)f);
        }
    };

    set(1, a.vox[e0]);
    double t_cur = seg_depth((double)chi[vv[1]], (double)sv[e0]);
    double t_nxt = 0.0;
    if (len > 1) {
        set(0, a.vox[e0 + 64]);
        t_nxt = seg_depth((double)chi[vv[0]], (double)sv[e0 + 64]);
    }
    double Gv[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // G_-1, G_0, G_1, G_2, G_3
    {
        double ex0, e00;
        entry_weights<double>(0.5 * t_cur, ex0, e00);
        Gv[1] = e00;
        add((double)wv[e0], Gv);
    }
    for (int m = 1; m < len; ++m) {
        const int64_t e = e0 + 64 * (int64_t)m;
        const bool last = m + 1 == len;
        // shift the window: point m becomes slot 1
#pragma unroll
        for (int j = 4; j >= 1; --j) {
            vv[j] = vv[j - 1]; vr[j] = vr[j - 1]; vt[j] = vt[j - 1]; vp[j] = vp[j - 1];
        }
        const double t_prev = t_cur;
        t_cur = t_nxt;
        if (!last) {
            set(0, a.vox[e + 64]);
            t_nxt = seg_depth((double)chi[vv[0]], (double)sv[e + 64]);
        } else {
            vv[0] = -1;
        }
        const double D = half_sum(t_prev, t_cur);
        const double Dp = last ? 0.0 : half_sum(t_cur, t_nxt);
        double ex, wa, wb, wg;
        if (PARA) {
            const PointW<double> pw = point_weights<double, sizeof(G) == 8>(D, Dp, last);
            ex = pw.ex; wa = pw.a; wb = pw.b; wg = pw.g;
        } else {
            const double Dv = D < kMinStep ? kMinStep : D;
            double e0m, e1, e2;
            kernel_moments<sizeof(G) == 8>(Dv, ex, e0m, e1, e2);
            wb = e1 * rcp_f64<sizeof(G) == 8>(Dv);
            wa = e0m - wb;
            wg = 0.0;
        }
        Gv[4] = ex * Gv[3];
        Gv[3] = ex * Gv[2];
        Gv[2] = ex * Gv[1] + wa;
        Gv[1] = ex * Gv[0] + wb;
        Gv[0] = wg;
        add((double)wv[e], Gv);
    }
}

hipError_t lstar_stencil_sphere_accumulate(const SphereStencilArgs &a, bool grid_double, bool geom_double,
                                           bool parabolic, hipStream_t st)
{
    if (a.n_bundles <= 0 || a.n_batch <= 0) return hipSuccess;
    const int64_t waves = a.n_bundles * a.n_batch;
    const dim3 grid((unsigned)((waves + 3) / 4));
#define RT_SPH_ST(G, TG, P) hipLaunchKernelGGL((lstar_stencil_sphere_kernel<G, TG, P>), grid, dim3(256), 0, st, a)
    if (grid_double) {
        if (geom_double) { if (parabolic) RT_SPH_ST(double, double, true); else RT_SPH_ST(double, double, false); }
        else { if (parabolic) RT_SPH_ST(double, float, true); else RT_SPH_ST(double, float, false); }
    } else {
        if (geom_double) { if (parabolic) RT_SPH_ST(float, double, true); else RT_SPH_ST(float, double, false); }
        else { if (parabolic) RT_SPH_ST(float, float, true); else RT_SPH_ST(float, float, false); }
    }
#undef RT_SPH_ST
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(256) stencil_finish_kernel(const unsigned long long *__restrict__ acc,
                                                             const int32_t *__restrict__ lambda_of, int64_t n_vox,
                                                             const T *__restrict__ centre, T *__restrict__ out)
{
    const int64_t n = (int64_t)kStencil * n_vox;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t lam = lambda_of[blockIdx.y];
    const int64_t base = lam * n;
    const int64_t c0 = (int64_t)kStencilCentre * n_vox;
    if (centre && i >= c0 && i < c0 + n_vox)
        out[base + i] = centre[lam * n_vox + (i - c0)];
    else
        out[base + i] = (T)((double)(long long)acc[base + i] * 0x1p-52);
}

hipError_t lstar_stencil_finish(const unsigned long long *acc, const int32_t *lambda_of, int64_t n_vox, int n_batch,
                                const void *centre, void *out, bool out_double, hipStream_t st)
{
    if (n_vox <= 0 || n_batch <= 0) return hipSuccess;
    const int64_t n = (int64_t)kStencil * n_vox;
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)n_batch);
    if (out_double)
        hipLaunchKernelGGL((stencil_finish_kernel<double>), grid, dim3(256), 0, st, acc, lambda_of, n_vox,
                           reinterpret_cast<const double *>(centre), reinterpret_cast<double *>(out));
    else
        hipLaunchKernelGGL((stencil_finish_kernel<float>), grid, dim3(256), 0, st, acc, lambda_of, n_vox,
                           reinterpret_cast<const float *>(centre), reinterpret_cast<float *>(out));
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Operator-splitting sweeps on [1 - Lambda*(1-eps)] x = r:
//   x_v <- (r_v + sum_{c != centre} L_c(v) (1 - eps_u) x_u) / (1 - L_centre(v) (1 - eps_v)),
// neighbours u in component order (a fixed order: reproducible).  Jacobi
// reads x_in and writes x_out; Gauss-Seidel updates x in place, one colour
// class at a time.
// ---------------------------------------------------------------------------
template <typename G>
__device__ __forceinline__ double os_row(const OsJacobiArgs &a, int64_t base, int x, int y, int k,
                                         const double *__restrict__ xs, bool first)
{
    const int64_t n = a.n_vox;
    const int Nx = a.Nx, Ny = a.Ny;
    const int64_t NxNy = (int64_t)Nx * Ny;
    const int64_t v = (int64_t)k * NxNy + (int64_t)y * Nx + x;
    const G *__restrict__ st = reinterpret_cast<const G *>(a.st) + base * kStencil;
    const G *__restrict__ eps = reinterpret_cast<const G *>(a.eps) + base;
    double den = 1.0 - (double)st[kStencilCentre * n + v] * (1.0 - (double)eps[v]);
    den = den < os_den_min<G>() ? os_den_min<G>() : den;
    double acc = a.r[base + v];
    if (!first) {
        for (int c = 0; c < kStencil; ++c) {
            if (c == kStencilCentre) continue;
            const double L = (double)st[(int64_t)c * n + v];
            if (L == 0.0) continue;
            int ku = k + c / 9 - 1;
            if (a.per[2]) ku = ku < 0 ? ku + a.Nz : (ku >= a.Nz ? ku - a.Nz : ku);
            else if (ku < 0 || ku >= a.Nz) continue;
            int yu = y + (c / 3) % 3 - 1;
            if (a.per[1]) yu = yu < 0 ? yu + Ny : (yu >= Ny ? yu - Ny : yu);
            else if (yu < 0 || yu >= Ny) continue;
            int xu = x + c % 3 - 1;
            if (a.per[0]) xu = xu < 0 ? xu + Nx : (xu >= Nx ? xu - Nx : xu);
            else if (xu < 0 || xu >= Nx) continue;
            const int64_t u = (int64_t)ku * NxNy + (int64_t)yu * Nx + xu;
            acc += L * (1.0 - (double)eps[u]) * xs[base + u];
        }
    }
    return acc / den;
}

template <typename G>
__global__ void __launch_bounds__(256) os_jacobi_kernel(OsJacobiArgs a, int first)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= a.n_vox) return;
    const int64_t base = (int64_t)a.lambda_of[blockIdx.y] * a.n_vox;
    const int64_t NxNy = (int64_t)a.Nx * a.Ny;
    const int k = (int)(v / NxNy);
    const int rem = (int)(v - (int64_t)k * NxNy);
    const int y = rem / a.Nx, x = rem - y * a.Nx;
    a.x_out[base + v] = os_row<G>(a, base, x, y, k, a.x_in, first != 0);
}

hipError_t os_jacobi_sweep(const OsJacobiArgs &a, bool grid_double, bool first, int n_batch, hipStream_t st)
{
    if (a.n_vox <= 0 || n_batch <= 0) return hipSuccess;
    dim3 grid((unsigned)((a.n_vox + 255) / 256), (unsigned)n_batch);
    if (grid_double)
        hipLaunchKernelGGL((os_jacobi_kernel<double>), grid, dim3(256), 0, st, a, first ? 1 : 0);
    else
        hipLaunchKernelGGL((os_jacobi_kernel<float>), grid, dim3(256), 0, st, a, first ? 1 : 0);
    return hipGetLastError();
}

// One colour class: coordinates (cx + 2 i, cy + 2 j, cz + 2 l) for colours 0
// and 1, the last index of the axis for colour 2; n[3] class sizes.
struct OsColour {
    int c[3];
    int n[3];
};

template <typename G>
__global__ void __launch_bounds__(256) os_gs_kernel(OsJacobiArgs a, OsColour col)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nxy = (int64_t)col.n[0] * col.n[1];
    if (i >= nxy * col.n[2]) return;
    const int iz = (int)(i / nxy);
    const int rem = (int)(i - (int64_t)iz * nxy);
    const int iy = rem / col.n[0], ix = rem - iy * col.n[0];
    const int x = col.c[0] == 2 ? a.Nx - 1 : col.c[0] + 2 * ix;
    const int y = col.c[1] == 2 ? a.Ny - 1 : col.c[1] + 2 * iy;
    const int k = col.c[2] == 2 ? a.Nz - 1 : col.c[2] + 2 * iz;
    const int64_t base = (int64_t)a.lambda_of[blockIdx.y] * a.n_vox;
    const double xn = os_row<G>(a, base, x, y, k, a.x_out, false);
    a.x_out[base + (int64_t)k * a.Nx * a.Ny + (int64_t)y * a.Nx + x] = xn;
}

// Size of colour class c along an axis of N voxels: parity classes 0 and 1,
// and on a periodic axis of odd length >= 3 the last voxel in class 2 (it
// neighbours voxel 0 across the period).
static int colour_size(int N, int c, bool periodic)
{
    const bool odd_wrap = periodic && N >= 3 && (N & 1);
    if (c == 2) return odd_wrap ? 1 : 0;
    const int lim = odd_wrap ? N - 1 : N;
    return lim > c ? (lim - c + 1) / 2 : 0;
}

hipError_t os_gs_sweep(const OsJacobiArgs &a, bool grid_double, int n_batch, hipStream_t st)
{
    if (a.n_vox <= 0 || n_batch <= 0) return hipSuccess;
    for (int cz = 0; cz < 3; ++cz)
        for (int cy = 0; cy < 3; ++cy)
            for (int cx = 0; cx < 3; ++cx) {
                OsColour col{{cx, cy, cz}, {colour_size(a.Nx, cx, a.per[0] != 0), colour_size(a.Ny, cy, a.per[1] != 0),
                                            colour_size(a.Nz, cz, a.per[2] != 0)}};
                const int64_t n = (int64_t)col.n[0] * col.n[1] * col.n[2];
                if (n == 0) continue;
                dim3 grid((unsigned)((n + 255) / 256), (unsigned)n_batch);
                if (grid_double)
                    hipLaunchKernelGGL((os_gs_kernel<double>), grid, dim3(256), 0, st, a, col);
                else
                    hipLaunchKernelGGL((os_gs_kernel<float>), grid, dim3(256), 0, st, a, col);
                hipError_t e = hipGetLastError();
                if (e != hipSuccess) return e;
            }
    return hipSuccess;
}

}  // namespace rt3d
