// fs_box.hip -- formal solution on the x,y-periodic box (gfx950).
//
// One workgroup sweeps all characteristics of one (wavelength, direction)
// work item through the grid, layer by layer in the direction of travel
// (top to bottom for mu < 0).  Every thread carries the intensity of R rays in
// registers; all rays of a direction share the visit template, so at visit m
// every lane reads the same template entry (scalar loads) and ray r touches
// voxel r + offset_m.  At a fixed m that map is one-to-one, so with a
// workgroup barrier per visit step the layer's J (and Lambda*) tile in LDS is
// updated by plain read-add-write without collisions and in a fixed order
// (bitwise reproducible; no LDS atomics, whose queueing cost a third of the
// kernel time).
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
//
// Band tiles (layers too wide for LDS): the rays of a direction are split
// into bundles of whole ray rows, and a workgroup's tile holds only the rows
// that its bundle reaches within the current layer.  Within one layer the
// template's row offsets span at most `span` rows (its horizontal travel per
// layer), so rays of origin rows [yb, yb + h) land in the h + span + 1 rows
// that start at yb + (lowest template row of the layer); the visit table
// carries each visit's row relative to that lowest row.  The tile index is
// then (origin row - yb + relative row) * Nx + x, and the flush maps tile
// word i to layer word (base * Nx + i) mod NxNy.  The workgroup clears its
// partial slot when it opens it, because a band touches only part of it.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "fs_box.hpp"
#include "fs_point.hpp"

namespace rt3d {

// ---------------------------------------------------------------------------
// field loads: one raw buffer load per point fetches the (chi, S) pair; the
// per-ray byte offset sits in a VGPR, the per-visit byte offset in an SGPR,
// so there is no per-lane address arithmetic
// ---------------------------------------------------------------------------
__device__ __forceinline__ __amdgpu_buffer_rsrc_t field_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}

template <typename T>
struct Pair {
    T chi, S;
};

template <typename T>
__device__ __forceinline__ Pair<T> ld_pair(__amdgpu_buffer_rsrc_t r, int voff, int soff);

template <>
__device__ __forceinline__ Pair<float> ld_pair<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    return __builtin_bit_cast(Pair<float>, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

template <>
__device__ __forceinline__ Pair<double> ld_pair<double>(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    return __builtin_bit_cast(Pair<double>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

// ---------------------------------------------------------------------------
// the sweep kernel
// ---------------------------------------------------------------------------
// Fused multiply-add in the recurrence type.
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// A value that is the same in every lane, kept in a scalar register: the
// weight of a visit, formed by vector instructions from scalar inputs, then
// serves every ray of the thread as a scalar operand.  Double values stay
// as they are.
__device__ __forceinline__ float uniform(float v)
{
    // by an explicit v_readfirstlane (the builtin would be moved ahead of the
    // conversion to single precision, which is then redone per ray).  A
    // readlane of a VGPR that the previous VALU instruction wrote needs wait
    // states in between, which the compiler inserts only around its own
    // instructions: the s_nop gives them here.
    float s;
    asm("s_nop 1\n\tv_readfirstlane_b32 %0, %1" : "=s"(s) : "v"(v));
    return s;
}
__device__ __forceinline__ double uniform(double v) { return v; }

template <typename T, int LB, int R, bool WJ, bool WL, bool PARA, int OCC, bool BAND>
__global__ void __launch_bounds__(LB) __attribute__((amdgpu_waves_per_eu(OCC * LB / 256 > 0 ? OCC * LB / 256 : 1)))
fs_box_kernel(FsBoxArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int Nx = a.Nx, Ny = a.Ny;
    const int NxNy = Nx * Ny;
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    // tiles of tile_words words plus one scratch word per thread (padding slots)
    const int TW = a.tile_words;
    T *tJ = reinterpret_cast<T *>(smem_raw);
    T *tL = tJ + (WJ ? TW + nthr : 0);
    constexpr int ES = 2 * (int)sizeof(T);  // bytes per (chi, S) pair

    for (int i = tid; i < TW + nthr; i += nthr) {
        if (WJ) tJ[i] = T(0);
        if (WL) tL[i] = T(0);
    }

    // The rays of a direction may be split into bundles of consecutive ray
    // indices; workgroup w always sweeps bundle w mod n_bundles (its own layer
    // tile and partial slot), so smaller workgroups with fewer rays per thread
    // can share a CU.  Rays of this thread: local index l = tid + j*nthr of
    // the bundle, origin (x0, y0) of ray q_lo + l.  Slots past the bundle's
    // last ray repeat an earlier ray of the bundle and contribute exactly
    // zero.  The host admits a launch shape only if nthr * (R - 1) is below
    // the smallest bundle, so only the last slot (j = R - 1) of a thread can
    // be such a padding slot and the other R - 1 copies of the point body
    // carry no padding logic.
    const int bundle = a.n_bundles > 1 ? (int)(blockIdx.x % (unsigned)a.n_bundles) : 0;
    int q_lo, q_n, yb = 0, hb = 0;
    if (BAND) {
        yb = (int)(((int64_t)bundle * Ny) / a.n_bundles);
        hb = (int)(((int64_t)(bundle + 1) * Ny) / a.n_bundles) - yb;
        q_lo = yb * Nx;
        q_n = hb * Nx;
    } else {
        q_lo = bundle * a.bundle_rays;
        q_n = min(a.bundle_rays, NxNy - q_lo);
    }
    // Two constants per ray j of this thread: vb[j], the byte offset of its
    // origin in the padded field (the per-visit part of the address is
    // scalar), and tw[j] = x0 << 19 | (tile word of its origin) * sizeof(T):
    // its high field decides the x wrap of a visit by one unsigned comparison
    // with a scalar, its low field (< 2^19: LDS bytes) is the tile address
    // before the visit's scalar offset.  Rows are relative to the bundle's
    // first row yb for band tiles.  Only the last slot of a thread can be a
    // padding slot (padj).
    const uint32_t row_bytes = (uint32_t)(2 * Nx * ES);
    // Single-precision band tiles of single-output sweeps are two layer rows
    // wide, like the padded field: a ray's column x0 + dx (below 2 Nx) then
    // needs no wrap, and the layer flush adds word x + Nx of a tile row to
    // column x.  (Two outputs at twice the width would leave room for fewer
    // rows per band.)
    constexpr bool WIDE = BAND && sizeof(T) == 4 && !(WJ && WL);
    const uint32_t tpitch = WIDE ? 2u * (uint32_t)Nx : (uint32_t)Nx;
    const int gshift = BAND ? (int)((uint32_t)yb * row_bytes) : 0;
    constexpr uint32_t kTileMask = (1u << 19) - 1u;
    int vb[R];
    uint32_t tw[R];
    bool padj = false;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        int l = tid + j * nthr;
        bool pad = false;
        while (l >= q_n) { l -= q_n; pad = true; }
        const int q = q_lo + l;
        const int y0 = q / Nx;
        const int x0 = q - y0 * Nx;
        const uint32_t yr = (uint32_t)(y0 - yb);
        vb[j] = (int)(yr * row_bytes + (uint32_t)x0 * ES);
        tw[j] = ((uint32_t)x0 << 19) | ((yr * tpitch + (uint32_t)x0) * (uint32_t)sizeof(T));
        if (j == R - 1) padj = pad;
    }
    unsigned char *const tJb = reinterpret_cast<unsigned char *>(tJ);
    unsigned char *const tLb = reinterpret_cast<unsigned char *>(tL);
    const uint32_t pad_addr = (uint32_t)(TW + tid) * (uint32_t)sizeof(T);
    const int f_row0 = tid / Nx, f_x0 = tid - f_row0 * Nx;    // flush position of this thread
    const int f_drow = nthr / Nx, f_dx = nthr - f_drow * Nx;  // and its step
    __syncthreads();

    const uint32_t slice_bytes = (uint32_t)(a.pad_stride * ES);
    const int it_end = a.wg_begin[blockIdx.x + 1];
    for (int it = a.wg_begin[blockIdx.x]; it < it_end; ++it) {
        const WorkItem item = a.items[it];
        const int lam = item.lambda;
        const int d = item.dir;
        const __amdgpu_buffer_rsrc_t rf =
            field_rsrc(reinterpret_cast<const T *>(a.field) + 2 * (int64_t)lam * a.pad_stride, slice_bytes);
        T *__restrict__ pJ = WJ ? reinterpret_cast<T *>(a.partJ) + (int64_t)item.slot * a.n_vox : nullptr;
        T *__restrict__ pL = WL ? reinterpret_cast<T *>(a.partL) + (int64_t)item.slot * a.n_vox : nullptr;
        const bool first = item.first != 0;
        const int64_t vbeg = a.dir_vbegin[d];
        const int M = a.dir_M[d];
        const double wmu = a.dir_wmu[d];
        const bool down = a.dir_mu[d] < 0.0;
        const T Ibc = a.I_bc ? reinterpret_cast<const T *>(a.I_bc)[2 * lam + (down ? 0 : 1)] : T(0);
        const int32_t *__restrict__ goff = a.goff + vbeg;
        const uint32_t *__restrict__ dxy = a.dxy + vbeg;
        const double *__restrict__ sv = a.s + vbeg;
        const int32_t *__restrict__ brow = BAND ? a.brow + vbeg : nullptr;
        const int span = BAND ? a.dir_span[d] : 0;

        if (BAND && first) {
            // a band touches only part of the slot: clear all of it once
            for (int64_t i = tid; i < a.n_vox; i += nthr) {
                if (WJ) pJ[i] = T(0);
                if (WL) pL[i] = T(0);
            }
            __syncthreads();
        }

        T I[R];
        T gprev[R];
        int layer = down ? 0 : a.Nz - 1;
        const int dlayer = down ? 1 : -1;

        // w, r: offsets word and relative row of the layer's last visit
        auto flush_layer = [&](uint32_t w, int r) {
            const int64_t lo = (int64_t)layer * NxNy;
            if (BAND) {
                // tile row 0 is layer row yb + (lowest template row of the layer)
                int base = (yb + (int)((w >> kOffBits) & kOffMask) - r) % Ny;
                if (base < 0) base += Ny;
                const uint32_t g0 = (uint32_t)base * (uint32_t)Nx;
                const int n = (hb + span + 1) * Nx;
                if (WIDE) {
                    // output word i = row Nx + x takes tile words row 2Nx + x and
                    // row 2Nx + x + Nx; row and x advance without division.  A
                    // single-output sweep (one tile, one slot); eight words of a
                    // thread at a time, their slot reads issued together
                    T *const tile = WJ ? tJ : tL;
                    T *__restrict__ const part = WJ ? pJ : pL;
                    int row = f_row0, x = f_x0;
                    auto word = [&](int i, uint32_t &gi, int &t0) {
                        gi = g0 + (uint32_t)i;
                        gi = min(gi, gi - (uint32_t)NxNy);
                        t0 = i + row * Nx;
                        x += f_dx;
                        row += f_drow;
                        if (x >= Nx) {
                            x -= Nx;
                            ++row;
                        }
                    };
                    constexpr int U = 8;
                    for (int i = tid; i < n; i += U * nthr) {
                        uint32_t gi[U];
                        int t0[U];
                        T old[U];
                        // slots past the band end only the thread's last group
#pragma unroll
                        for (int u = 0; u < U; ++u)
                            if (i + u * nthr < n) word(i + u * nthr, gi[u], t0[u]);
#pragma unroll
                        for (int u = 0; u < U; ++u)
                            if (i + u * nthr < n) old[u] = part[lo + gi[u]];
#pragma unroll
                        for (int u = 0; u < U; ++u)
                            if (i + u * nthr < n) {
                                const T v = tile[t0[u]] + tile[t0[u] + Nx];
                                tile[t0[u]] = T(0);
                                tile[t0[u] + Nx] = T(0);
                                part[lo + gi[u]] = old[u] + v;
                            }
                    }
                    layer += dlayer;
                    __syncthreads();
                    return;
                }
                // four words of a thread at a time, their slot reads issued together
                constexpr int U = 4;
                for (int i = tid; i < n; i += U * nthr) {
                    uint32_t gi[U];
                    T oJ[U], oL[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        gi[u] = g0 + (uint32_t)(i + u * nthr);
                        gi[u] = min(gi[u], gi[u] - (uint32_t)NxNy);
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        if (i + u * nthr < n) {
                            if (WJ) oJ[u] = pJ[lo + gi[u]];
                            if (WL) oL[u] = pL[lo + gi[u]];
                        }
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int k = i + u * nthr;
                        if (k < n) {
                            if (WJ) {
                                const T v = tJ[k];
                                tJ[k] = T(0);
                                pJ[lo + gi[u]] = oJ[u] + v;
                            }
                            if (WL) {
                                const T v = tL[k];
                                tL[k] = T(0);
                                pL[lo + gi[u]] = oL[u] + v;
                            }
                        }
                    }
                }
            } else {
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
            }
            layer += dlayer;
            __syncthreads();
        };
        // Scalar part of a visit's tile addresses: byte offset of the visit's
        // horizontal offsets (dx, and the relative row r or dy), the x-wrap
        // threshold (Nx - dx) << 19 on tw, and for layer tiles the y-wrap
        // threshold on the tile address.
        struct TileStep {
            uint32_t off, thx, thy;
        };
        auto tile_step = [&](uint32_t w, int r) {
            const uint32_t dx = w & kOffMask;
            TileStep s;
            s.thx = ((uint32_t)Nx - dx) << 19;
            if (BAND) {
                s.off = ((uint32_t)r * tpitch + dx) * (uint32_t)sizeof(T);
                s.thy = 0;
            } else {
                const uint32_t dy = (w >> kOffBits) & kOffMask;
                s.off = (dy * (uint32_t)Nx + dx) * (uint32_t)sizeof(T);
                s.thy = ((uint32_t)Ny - dy) * (uint32_t)Nx * (uint32_t)sizeof(T);
            }
            return s;
        };
        // LDS byte address of ray j's voxel at a visit; padding slots go to
        // this thread's own word past the tile, so no two lanes ever update
        // the same word in one step
        auto tile_addr = [&](int j, const TileStep &s) {
            const uint32_t base = tw[j] & kTileMask;
            uint32_t a4 = base + s.off;
            if (!WIDE) a4 -= tw[j] >= s.thx ? (uint32_t)Nx * (uint32_t)sizeof(T) : 0u;
            if (!BAND) a4 -= base >= s.thy ? (uint32_t)NxNy * (uint32_t)sizeof(T) : 0u;
            return (j == R - 1 && padj) ? pad_addr : a4;
        };
        // the visit weight, zero for a padding slot
        auto ray_weight = [&](int j, T cw) { return (j == R - 1 && padj) ? T(0) : cw; };
        auto tile_add = [&](unsigned char *tile, uint32_t addr, T v) {
            T *w = reinterpret_cast<T *>(tile + addr);
            *w += v;
        };

        // Single-precision sweeps carry along each ray, from one visit to the
        // next, the sources of the previous and current points (Sp, Sc), the
        // opacity of the current point (Xc) and the optical step from the
        // previous point to the current one (Dc): each visit then reads only
        // the next point's (chi, S) pair and forms one optical depth.  Double
        // sweeps (twice the registers per value) read the previous, current
        // and next pairs at every visit instead.
        constexpr bool CARRY = sizeof(T) == 4;
        T Sp[CARRY ? R : 1], Sc[CARRY ? R : 1], Xc[CARRY ? R : 1];
        double Dc[CARRY ? R : 1];
        int g_p = 0;
        double s_p = 0.0;

        // first point: entry half-segment with constant S; the second point's
        // pair is read too (the first optical step between points needs it)
        int g_c = goff[0] * ES + gshift;
        double s_c = sv[0];
        uint32_t w_c = dxy[0];
        int r_c = BAND ? brow[0] : 0;
        int g_n = g_c;
        double s_n = s_c;
        if (M > 1) {
            g_n = goff[1] * ES + gshift;
            s_n = sv[1];
        }
        {
            const T cw = T(wmu * s_c);
            const TileStep ts = tile_step(w_c, r_c);
#pragma unroll
            for (int j = 0; j < R; ++j) {
                gprev[j] = T(0);
                const Pair<T> f0 = ld_pair<T>(rf, vb[j], g_c);
                const double t0 = seg_depth((double)f0.chi, s_c);
                T ex, e0;
                entry_weights<T>(0.5 * t0, ex, e0);
                I[j] = WJ ? Ibc * ex + f0.S * e0 : T(0);
                const uint32_t ad = tile_addr(j, ts);
                const T cj = ray_weight(j, cw);
                if (WJ) tile_add(tJb, ad, cj * I[j]);
                if (WL) tile_add(tLb, ad, cj * e0);
                if constexpr (CARRY) {
                    const Pair<T> f1 = ld_pair<T>(rf, vb[j], g_n);
                    Sp[j] = f0.S;
                    Sc[j] = f1.S;
                    Xc[j] = f1.chi;
                    Dc[j] = step_depth(t0, seg_depth((double)f1.chi, s_n));
                }
            }
            __syncthreads();
            if (w_c & kLayerEnd) flush_layer(w_c, r_c);
        }

        // one point of every ray of this thread; LAST: the final point, which
        // has no downwind neighbour
        auto step = [&](auto last_tag) {
            constexpr bool LAST = decltype(last_tag)::value;
            const T cw = uniform(T(wmu * s_c));
            const TileStep ts = tile_step(w_c, r_c);
            // software pipeline over the rays of this thread: the loads of
            // ray j+1 are in flight while ray j is computed
            const Pair<T> zero{T(0), T(0)};
            Pair<T> nn = LAST ? zero : ld_pair<T>(rf, vb[0], g_n);
            Pair<T> np = CARRY ? zero : ld_pair<T>(rf, vb[0], g_p);
            Pair<T> nc = CARRY ? zero : ld_pair<T>(rf, vb[0], g_c);
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const Pair<T> fn = nn, fp = np, fc = nc;
                if (j + 1 < R) {
                    if (!LAST) nn = ld_pair<T>(rf, vb[j + 1], g_n);
                    if (!CARRY) {
                        np = ld_pair<T>(rf, vb[j + 1], g_p);
                        nc = ld_pair<T>(rf, vb[j + 1], g_c);
                    }
                }
                double D, Dp = 0.0;
                T S_prev, S_cur;
                if constexpr (CARRY) {
                    D = Dc[j];
                    S_prev = Sp[j];
                    S_cur = Sc[j];
                    if (!LAST) Dp = step_depth(seg_depth((double)Xc[j], s_c), seg_depth((double)fn.chi, s_n));
                } else {
                    const double tc = seg_depth((double)fc.chi, s_c);
                    D = step_depth(seg_depth((double)fp.chi, s_p), tc);
                    if (!LAST) Dp = step_depth(tc, seg_depth((double)fn.chi, s_n));
                    S_prev = fp.S;
                    S_cur = fc.S;
                }
                const PointW<T> pw = point_weights_pos<T, LAST, WL && !PARA>(D, Dp);
                if (WJ) {
                    // accumulated in place: I ex, then the three source terms
                    T Ij = I[j] * pw.ex;
                    Ij = fma_t(pw.a, S_prev, Ij);
                    Ij = fma_t(pw.b, S_cur, Ij);
                    if (!LAST) Ij = fma_t(pw.g, fn.S, Ij);
                    I[j] = Ij;
                }
                const uint32_t ad = tile_addr(j, ts);
                const T cj = ray_weight(j, cw);
                if (WJ) tile_add(tJb, ad, cj * I[j]);
                if (WL) {
                    T dloc;
                    if (PARA) {
                        dloc = pw.b + gprev[j] * pw.ex;
                        gprev[j] = pw.g;
                    } else {
                        dloc = pw.dlin;
                    }
                    tile_add(tLb, ad, cj * dloc);
                }
                if constexpr (CARRY && !LAST) {
                    Sp[j] = Sc[j];
                    Sc[j] = fn.S;
                    Xc[j] = fn.chi;
                    Dc[j] = Dp;
                }
            }
            __syncthreads();
            if (w_c & kLayerEnd) flush_layer(w_c, r_c);
        };

        // template entries of the current visit (c) and the next one (n); the
        // final point is taken after the loop, so that the loop body has a
        // single path (no merge of the carried per-ray state)
        for (int m = 1; m + 1 < M; ++m) {
            g_p = g_c;
            s_p = s_c;
            g_c = g_n;
            s_c = s_n;
            w_c = dxy[m];
            if (BAND) r_c = brow[m];
            g_n = goff[m + 1] * ES + gshift;
            s_n = sv[m + 1];
            step(std::false_type{});
        }
        if (M > 1) {
            g_p = g_c;
            s_p = s_c;
            g_c = g_n;
            s_c = s_n;
            w_c = dxy[M - 1];
            if (BAND) r_c = brow[M - 1];
            step(std::true_type{});
        }
    }
}

// ---------------------------------------------------------------------------
// host-side dispatch
//
// Launch shapes: (threads per workgroup bound LB, rays per thread R).  All
// output combinations exist for LB = 1024; the other shapes exist for the
// J-only kernel, which runs every ALI step and is the one the autotuner
// (rt_autotune) times.
// ---------------------------------------------------------------------------
// Launch shapes (threads bound LB, rays per thread R, workgroups per CU OCC).
// OCC = 2 shapes split each direction's rays into two bundles so that two
// workgroups (two layer tiles) share a CU: twice the resident waves to hide
// the latency of the double-precision point arithmetic.  Band-tile shapes
// serve layers too wide for a whole-layer tile (and grids that ask for band
// tiles); their bundle count follows from the LDS left per workgroup.
#define RT_FS_SHAPES_FULL(X)                                                                                 \
    X(1024, 1, 1) X(1024, 2, 1) X(1024, 4, 1) X(1024, 8, 1) X(1024, 12, 1) X(1024, 17, 1) X(1024, 24, 1) \
        X(768, 6, 1) X(768, 11, 1)
#define RT_FS_SHAPES_TUNE(X)                                                                                     \
    X(768, 2, 1) X(768, 8, 1) X(768, 22, 1) X(768, 32, 1) X(512, 33, 1) X(256, 5, 1) X(256, 17, 1) X(256, 34, 1) \
        X(512, 3, 2) X(512, 7, 2) X(512, 9, 2) X(512, 17, 2)
#define RT_FS_SHAPES_BAND_FULL(X)                                                                            \
    X(1024, 1, 1) X(1024, 2, 1) X(1024, 4, 1) X(1024, 8, 1) X(1024, 12, 1) X(1024, 17, 1) X(768, 6, 1) \
        X(768, 11, 1)
#define RT_FS_SHAPES_BAND_TUNE(X) \
    X(768, 8, 1) X(768, 10, 1) X(896, 10, 1) X(768, 22, 1) X(512, 6, 2) X(512, 7, 2) X(512, 9, 2) X(512, 17, 2)

static const FsShape kShapes[] = {
#define RT_LIST(lb, r, o) {lb, r, true, o, false},
    RT_FS_SHAPES_FULL(RT_LIST)
#undef RT_LIST
#define RT_LIST(lb, r, o) {lb, r, false, o, false},
    RT_FS_SHAPES_TUNE(RT_LIST)
#undef RT_LIST
#define RT_LIST(lb, r, o) {lb, r, true, o, true},
    RT_FS_SHAPES_BAND_FULL(RT_LIST)
#undef RT_LIST
#define RT_LIST(lb, r, o) {lb, r, false, o, true},
    RT_FS_SHAPES_BAND_TUNE(RT_LIST)
#undef RT_LIST
};

int fs_box_shapes(const FsShape **out)
{
    *out = kShapes;
    return (int)(sizeof(kShapes) / sizeof(kShapes[0]));
}

template <typename T, int LB, int R, bool WJ, bool WL, bool PARA, int OCC, bool BAND>
static hipError_t launch_one(const FsBoxArgs &a, int n_wg, int nthr, size_t lds, hipStream_t st)
{
    auto k = fs_box_kernel<T, LB, R, WJ, WL, PARA, OCC, BAND>;
    hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(n_wg), dim3(nthr), lds, st, a);
    return hipGetLastError();
}

// Resident workgroups per CU; negative when the compiled kernel spills
// registers to scratch memory (the host then prefers other shapes).
template <typename T, int LB, int R, bool WJ, bool WL, bool PARA, int OCC, bool BAND>
static int occ_one(int nthr, size_t lds)
{
    const auto k = fs_box_kernel<T, LB, R, WJ, WL, PARA, OCC, BAND>;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, nthr, lds) != hipSuccess) return 0;
    hipFuncAttributes attr{};
    if (hipFuncGetAttributes(&attr, (const void *)k) != hipSuccess) return 0;
    return attr.localSizeBytes > 0 ? -n : n;
}

template <typename T, int LB, int R, int OCC, bool BAND>
static hipError_t launch_flags(const FsBoxArgs &a, bool wj, bool wl, bool para, int n_wg, int nthr, size_t lds,
                               hipStream_t st)
{
    if (wj && wl && para) return launch_one<T, LB, R, true, true, true, OCC, BAND>(a, n_wg, nthr, lds, st);
    if (wj && wl) return launch_one<T, LB, R, true, true, false, OCC, BAND>(a, n_wg, nthr, lds, st);
    if (wj) return launch_one<T, LB, R, true, false, false, OCC, BAND>(a, n_wg, nthr, lds, st);
    if (wl && para) return launch_one<T, LB, R, false, true, true, OCC, BAND>(a, n_wg, nthr, lds, st);
    if (wl) return launch_one<T, LB, R, false, true, false, OCC, BAND>(a, n_wg, nthr, lds, st);
    return hipSuccess;
}

template <typename T, int LB, int R, int OCC, bool BAND>
static int occ_flags(bool wj, bool wl, bool para, int nthr, size_t lds)
{
    if (wj && wl && para) return occ_one<T, LB, R, true, true, true, OCC, BAND>(nthr, lds);
    if (wj && wl) return occ_one<T, LB, R, true, true, false, OCC, BAND>(nthr, lds);
    if (wj) return occ_one<T, LB, R, true, false, false, OCC, BAND>(nthr, lds);
    if (wl && para) return occ_one<T, LB, R, false, true, true, OCC, BAND>(nthr, lds);
    if (wl) return occ_one<T, LB, R, false, true, false, OCC, BAND>(nthr, lds);
    return 0;
}

template <typename T>
static hipError_t launch_t(const FsBoxArgs &a, bool wj, bool wl, bool para, bool band, int lb, int R, int n_wg,
                           int nthr, size_t lds, hipStream_t st)
{
    const bool j_only = wj && !wl;
    if (!band) {
#define RT_CASE(LBv, Rv, Ov) \
    if (lb == LBv && R == Rv) return launch_flags<T, LBv, Rv, Ov, false>(a, wj, wl, para, n_wg, nthr, lds, st);
        RT_FS_SHAPES_FULL(RT_CASE)
#undef RT_CASE
        if (!j_only) return hipErrorInvalidValue;
#define RT_CASE(LBv, Rv, Ov) \
    if (lb == LBv && R == Rv) return launch_one<T, LBv, Rv, true, false, false, Ov, false>(a, n_wg, nthr, lds, st);
        RT_FS_SHAPES_TUNE(RT_CASE)
#undef RT_CASE
    } else {
#define RT_CASE(LBv, Rv, Ov) \
    if (lb == LBv && R == Rv) return launch_flags<T, LBv, Rv, Ov, true>(a, wj, wl, para, n_wg, nthr, lds, st);
        RT_FS_SHAPES_BAND_FULL(RT_CASE)
#undef RT_CASE
        if (!j_only) return hipErrorInvalidValue;
#define RT_CASE(LBv, Rv, Ov) \
    if (lb == LBv && R == Rv) return launch_one<T, LBv, Rv, true, false, false, Ov, true>(a, n_wg, nthr, lds, st);
        RT_FS_SHAPES_BAND_TUNE(RT_CASE)
#undef RT_CASE
    }
    return hipErrorInvalidValue;
}

template <typename T>
static int occ_t(bool wj, bool wl, bool para, bool band, int lb, int R, int nthr, size_t lds)
{
    const bool j_only = wj && !wl;
    if (!band) {
#define RT_CASE(LBv, Rv, Ov) \
    if (lb == LBv && R == Rv) return occ_flags<T, LBv, Rv, Ov, false>(wj, wl, para, nthr, lds);
        RT_FS_SHAPES_FULL(RT_CASE)
#undef RT_CASE
        if (!j_only) return 0;
#define RT_CASE(LBv, Rv, Ov) \
    if (lb == LBv && R == Rv) return occ_one<T, LBv, Rv, true, false, false, Ov, false>(nthr, lds);
        RT_FS_SHAPES_TUNE(RT_CASE)
#undef RT_CASE
    } else {
#define RT_CASE(LBv, Rv, Ov) \
    if (lb == LBv && R == Rv) return occ_flags<T, LBv, Rv, Ov, true>(wj, wl, para, nthr, lds);
        RT_FS_SHAPES_BAND_FULL(RT_CASE)
#undef RT_CASE
        if (!j_only) return 0;
#define RT_CASE(LBv, Rv, Ov) \
    if (lb == LBv && R == Rv) return occ_one<T, LBv, Rv, true, false, false, Ov, true>(nthr, lds);
        RT_FS_SHAPES_BAND_TUNE(RT_CASE)
#undef RT_CASE
    }
    return 0;
}

hipError_t fs_box_launch(const FsBoxArgs &a, bool is_double, bool want_j, bool want_l, bool para, bool band, int lb,
                         int R, int n_wg, int nthr, size_t lds, hipStream_t st)
{
    if (n_wg <= 0) return hipSuccess;
    return is_double ? launch_t<double>(a, want_j, want_l, para, band, lb, R, n_wg, nthr, lds, st)
                     : launch_t<float>(a, want_j, want_l, para, band, lb, R, n_wg, nthr, lds, st);
}

int fs_box_occupancy(bool is_double, bool want_j, bool want_l, bool para, bool band, int lb, int R, int nthr,
                     size_t lds)
{
    return is_double ? occ_t<double>(want_j, want_l, para, band, lb, R, nthr, lds)
                     : occ_t<float>(want_j, want_l, para, band, lb, R, nthr, lds);
}

}  // namespace rt3d
