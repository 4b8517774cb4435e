// rt_api.cpp -- the C ABI declared in include/rt3d.h.
//
// Host side of the library: argument validation, the geometry cache upload,
// workgroup schedules, lazily sized device buffers, and the order of kernel
// launches for one formal solution, one ALI step and a full solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "ali.hpp"
#include "fs_box.hpp"
#include "fs_sphere.hpp"
#include "krylov.hpp"
#include "lstar_nl.hpp"
#include "rt_internal.hpp"
#include "unet.hpp"

using namespace rt3d;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static rt_status fail(rt_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHK(...)                                                                         \
    do {                                                                                    \
        hipError_t e_ = (__VA_ARGS__);                                                      \
        if (e_ != hipSuccess)                                                               \
            return fail(RT_E_HIP, "HIP error %s at %s:%d", hipGetErrorString(e_), __FILE__, \
                        __LINE__);                                                          \
    } while (0)

// ---------------------------------------------------------------------------
// device buffer helper
// ---------------------------------------------------------------------------
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    ~DevBuf() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    // grows (never shrinks); contents are not preserved
    hipError_t ensure(size_t n)
    {
        if (n <= bytes) return hipSuccess;
        release();
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) { p = nullptr; return e; }
        bytes = n;
        return hipSuccess;
    }
    template <typename T> T *as() const { return reinterpret_cast<T *>(p); }
};

// One kernel variant: element type, outputs, launch shape and resident count.
struct Variant {
    bool dbl = false, wj = false, wl = false;
    int lb = 0, R = 0, nthr = 0, n_wg = 0;
    int nb = 1, Q = 0;  // ray bundles per direction and rays per (largest) bundle
    bool band = false;  // band tiles (bundles of whole ray rows) instead of layer tiles
    int tile_words = 0;
    size_t lds = 0;
    bool ok = false;
};

struct DevSchedule {
    int n_wg = 0, n_slots = 0, n_batch = 0;
    int64_t points = 0;  // characteristic points evaluated by one launch
    DevBuf wg_begin, items, slot_begin, slot_ids, lambda_of;
};

// One chunk of the spherical geometry cache, bundle-major (chunk-local
// indices; see fs_sphere.hpp).  Either resident in device memory (one
// buffer per array) or, when device memory runs short or the grid asks for
// it, packed into one pinned host block that is streamed through a device
// staging buffer for every formal solution (the paper's SmallGPU mode,
// Sec. 5: caches kept on the host and sent to the GPU per solid angle).
struct SphereChunkDev {
    SphereChunk info;
    int64_t n_chars = 0, n_visits = 0, n_bundles = 0, n_entries = 0;
    DevBuf bundle_begin;  // int64 [n_bundles]
    DevBuf char_len;      // int32 [n_bundles * 64]
    DevBuf char_g;        // double [n_bundles * 64]
    DevBuf vox;           // int32 [n_entries]
    DevBuf s, w;          // geometry type [n_entries]
    DevBuf row, idx;      // CSR voxel -> entries: int32 [n_vox + 1], int32 [n_visits]
    // host placement: the same eight arrays packed at 256-byte aligned offsets
    void *host = nullptr;
    size_t bytes = 0;     // packed size (either placement)
    size_t off[8] = {};
    ~SphereChunkDev()
    {
        if (host) (void)hipHostFree(host);
    }
};

// Device pointers of a chunk's arrays (staged chunks: inside the staging buffer).
struct ChunkPtrs {
    const int64_t *bundle_begin;
    const int32_t *char_len;
    const double *char_g;
    const int32_t *vox;
    const void *s, *w;
    const int32_t *row, *idx;
};

static ChunkPtrs chunk_ptrs(const SphereChunkDev &ch, const void *stage)
{
    ChunkPtrs p{};
    if (ch.host) {
        const char *b = static_cast<const char *>(stage);
        p.bundle_begin = reinterpret_cast<const int64_t *>(b + ch.off[0]);
        p.char_len = reinterpret_cast<const int32_t *>(b + ch.off[1]);
        p.char_g = reinterpret_cast<const double *>(b + ch.off[2]);
        p.vox = reinterpret_cast<const int32_t *>(b + ch.off[3]);
        p.s = b + ch.off[4];
        p.w = b + ch.off[5];
        p.row = reinterpret_cast<const int32_t *>(b + ch.off[6]);
        p.idx = reinterpret_cast<const int32_t *>(b + ch.off[7]);
    } else {
        p.bundle_begin = ch.bundle_begin.as<int64_t>();
        p.char_len = ch.char_len.as<int32_t>();
        p.char_g = ch.char_g.as<double>();
        p.vox = ch.vox.as<int32_t>();
        p.s = ch.s.p;
        p.w = ch.w.p;
        p.row = ch.row.as<int32_t>();
        p.idx = ch.idx.as<int32_t>();
    }
    return p;
}

struct rt_grid {
    rt_grid_desc desc{};
    BoxGeometry geo;
    // spherical grids
    bool sphere = false;
    bool sph_gdouble = false;  // geometry cache in double (double grids) or float
    SphereCache sph;
    std::vector<std::unique_ptr<SphereChunkDev>> sph_chunks;
    DevBuf sph_outJ, sph_outL;  // per-visit contributions of one chunk
    // streamed chunks: two staging buffers, a copy stream and its events
    bool sph_host_cache = false;  // RT_F_HOST_CACHE: every chunk on the host
    bool sph_streaming = false;   // some chunk lives on the host
    DevBuf sph_stage[2];
    hipStream_t sph_copy = nullptr;
    hipEvent_t sph_copied[2] = {nullptr, nullptr}, sph_done[2] = {nullptr, nullptr};
    int64_t cache_dev_bytes = 0, cache_host_bytes = 0;
    // layout of the formal-solution input: box (Nx, Ny, Nz); sphere (n_vox, 0, 1)
    int lx = 0, ly = 0, lz = 0;
    int nbc = 2;  // boundary values per wavelength in I_bc
    int device = 0;
    int n_cu = 0;
    size_t max_lds = 0;
    bool dbl = false;
    bool para = false;
    int64_t n_vox = 0;
    int n_dir = 0;
    int64_t n_visits = 0;

    DevBuf goff, dxy, s, vbegin, M, wmu, mu, brow, span, comp;
    // nearest-neighbour Lambda*: fixed-point sums, stencil [lambda][27][vox]
    // (grid precision), OS right-hand side and Jacobi iterates [lambda][vox]
    bool nonlocal = false;
    DevBuf nl_acc, nl_st, os_r, os_x0, os_x1;
    // the stencil of an ALI step runs on a side stream beside its formal solutions
    hipStream_t nl_side = nullptr;
    hipEvent_t nl_fork = nullptr, nl_join = nullptr;
    int span_max = 0;   // largest per-layer row extent of any template
    bool band = false;  // the box sweep uses band tiles (see fs_box.hip)
    Variant var[2][2][2];  // [dbl][wj][wl]
    bool tuned = false;

    std::map<std::string, std::unique_ptr<DevSchedule>> schedules;

    // formal-solution inputs: interleaved (chi, S) doubly periodic padded copies
    DevBuf fs_fld;           // rt_formal_solution
    DevBuf fld, fld64, ibc64;  // ALI (sized for n_lambda_max); fld64: double anchors of FP32 grids
    DevBuf partJ, partL, partJ64, partL64;
    // ALI state owned by the library
    DevBuf J_anchor, S_anchor, hist, ng_blk, ng_coef;
    int hist_count = 0;
    const void *chi_src = nullptr;
    // captured plain ALI steps, keyed by batch, ring slot and state pointers
    std::map<std::string, hipGraphExec_t> graphs;
    // BiCGStab vectors and reduction scratch
    DevBuf kvec, kblk, kout, kc;
    // learned ALI correction
    UNetDev *net = nullptr;
    DevBuf net_r, net_f, net_out, J_save, resid;
    // measurement hooks
    bool prof = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_events;
    int64_t prof_points = 0;
    void drop_graphs()
    {
        for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
        graphs.clear();
    }
    ~rt_grid()
    {
        for (int i = 0; i < 2; ++i) {
            if (sph_copied[i]) (void)hipEventDestroy(sph_copied[i]);
            if (sph_done[i]) (void)hipEventDestroy(sph_done[i]);
        }
        if (sph_copy) (void)hipStreamDestroy(sph_copy);
        if (nl_fork) (void)hipEventDestroy(nl_fork);
        if (nl_join) (void)hipEventDestroy(nl_join);
        if (nl_side) (void)hipStreamDestroy(nl_side);
        for (auto &e : prof_events) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
        drop_graphs();
        if (net) unet_destroy(net);
    }
};

static Variant &variant(rt_grid *g, bool dbl, bool wj, bool wl) { return g->var[dbl][wj][wl]; }

// Resident-workgroup count and LDS size of one launch shape; ok = false when
// the shape cannot hold all rays of a bundle or its tiles do not fit.
static Variant make_variant(rt_grid *g, bool dbl, bool wj, bool wl, int lb, int R, int occ = 1, bool band = false)
{
    Variant v;
    v.dbl = dbl; v.wj = wj; v.wl = wl; v.lb = lb; v.R = R; v.band = band;
    const int Nx = g->geo.Nx, Ny = g->geo.Ny;
    const int rays = Nx * Ny;
    const size_t esz = dbl ? 8 : 4;
    const size_t nout = (wj ? 1 : 0) + (wl ? 1 : 0);
    // the padded field of one wavelength must stay addressable by 32-bit buffer offsets
    if ((int64_t)4 * g->n_vox * 2 * (int64_t)esz > (int64_t)INT_MAX) return v;
    if (!band) {
        const int nb = occ;
        const int Q = (rays + nb - 1) / nb;
        const int q_last = rays - (nb - 1) * Q;  // the smallest bundle
        if (q_last <= 0) return v;
        v.nb = nb;
        v.Q = Q;
        const int need = (Q + R - 1) / R;
        if (need > lb) return v;
        v.nthr = std::min(lb, ((need + 63) / 64) * 64);
        // the sweep kernel expects padding slots only in each thread's last ray slot
        if ((int64_t)v.nthr * (R - 1) >= q_last) return v;
        // per tile: one word per voxel of a layer plus one scratch word per thread
        v.tile_words = rays;
    } else {
        // fewest bundles of whole rows (sizes Ny/nb rounded down or up) whose
        // rays fit the shape and whose band tiles leave room for `occ`
        // workgroups per CU
        const int span = g->span_max;
        bool found = false;
        for (int nb = 2; nb <= Ny && !found; ++nb) {
            const int H = (Ny + nb - 1) / nb, Hmin = Ny / nb;
            if (H + span + 1 > Ny) continue;
            const int64_t Q = (int64_t)H * Nx;
            const int64_t need = (Q + R - 1) / R;
            if (need > lb) continue;
            const int nthr = std::min(lb, (int)((need + 63) / 64) * 64);
            if ((int64_t)nthr * (R - 1) >= (int64_t)Hmin * Nx) continue;
            const int tw = (H + span + 1) * Nx;
            if ((size_t)(tw + nthr) * esz * nout * (size_t)occ > g->max_lds) continue;
            v.nb = nb; v.Q = (int)Q; v.nthr = nthr; v.tile_words = tw;
            found = true;
        }
        if (!found) return v;
    }
    v.lds = (size_t)(v.tile_words + v.nthr) * esz * nout;
    if (v.lds > g->max_lds) return v;
    const int res = fs_box_occupancy(dbl, wj, wl, g->para, band, lb, R, v.nthr, v.lds);
    if (res <= 0) return v;
    v.n_wg = res * g->n_cu;
    v.n_wg -= v.n_wg % v.nb;  // equal classes of workgroups per bundle
    if (v.n_wg < v.nb) return v;
    v.ok = true;
    return v;
}

// Default shape: 1024-thread workgroups.  Layer tiles: the fewest rays per
// thread.  Band tiles: the fewest bundles (widest bands, least flush traffic
// per ray), then the fewest rays per thread.
static void setup_variant(rt_grid *g, bool dbl, bool wj, bool wl)
{
    const FsShape *sh = nullptr;
    const int n = fs_box_shapes(&sh);
    Variant &best = variant(g, dbl, wj, wl);
    best = Variant();
    for (int i = 0; i < n; ++i) {
        if (!sh[i].full || sh[i].lb != 1024 || sh[i].band != g->band) continue;
        Variant v = make_variant(g, dbl, wj, wl, sh[i].lb, sh[i].R, sh[i].occ, sh[i].band);
        if (!v.ok) continue;
        if (!g->band) { best = v; return; }
        if (!best.ok || v.nb < best.nb) best = v;
    }
}

// Rays swept by the workgroups of bundle b of a launch.
static int64_t bundle_ray_count(const rt_grid *g, const Variant *v, int b)
{
    const int64_t Nx = g->geo.Nx, Ny = g->geo.Ny;
    if (!v || v->nb <= 1) return Nx * Ny;
    if (v->band) return ((int64_t)(b + 1) * Ny / v->nb - (int64_t)b * Ny / v->nb) * Nx;
    return std::min<int64_t>(v->Q, Nx * Ny - (int64_t)b * v->Q);
}

// ---------------------------------------------------------------------------
// schedules
// ---------------------------------------------------------------------------
static rt_status get_schedule(rt_grid *g, int n_wg, const std::vector<int32_t> &lambdas, DevSchedule **out,
                              const std::vector<int32_t> *subset = nullptr, const Variant *v = nullptr)
{
    const int nb = v ? v->nb : 1;
    std::string key = std::to_string(n_wg) + "/" + std::to_string(nb) + (v && v->band ? "b" : "") + ":";
    for (int l : lambdas) key += std::to_string(l) + ",";
    if (subset) {
        key += "|d";
        for (int d : *subset) key += std::to_string(d) + ",";
    }
    auto it = g->schedules.find(key);
    if (it != g->schedules.end()) {
        *out = it->second.get();
        return RT_OK;
    }
    Schedule sc;
    auto ds = std::make_unique<DevSchedule>();
    if (g->sphere) {
        // one slot per batch entry: the gather writes each wavelength's J directly
        const int nb = (int)lambdas.size();
        sc.n_wg = 0;
        sc.wg_begin.assign(1, 0);
        sc.n_slots = nb;
        for (int b = 0; b <= nb; ++b) sc.slot_begin.push_back(b);
        for (int b = 0; b < nb; ++b) sc.slot_ids.push_back(b);
        ds->points = g->n_visits * nb;
    } else {
        build_schedule(g->geo, lambdas, n_wg, sc, subset, nb);
        for (int w = 0; w < sc.n_wg; ++w) {
            const int64_t nr = bundle_ray_count(g, v, w % nb);
            for (int k = sc.wg_begin[w]; k < sc.wg_begin[w + 1]; ++k)
                ds->points += (int64_t)g->geo.dirs[sc.items[k].dir].M * nr;
        }
    }
    ds->n_wg = sc.n_wg;
    ds->n_slots = sc.n_slots;
    ds->n_batch = (int)lambdas.size();
    auto up = [](DevBuf &b, const void *src, size_t n) -> hipError_t {
        hipError_t e = b.ensure(n > 0 ? n : 16);
        if (e != hipSuccess) return e;
        if (n > 0) return hipMemcpy(b.p, src, n, hipMemcpyHostToDevice);
        return hipSuccess;
    };
    HIPCHK(up(ds->wg_begin, sc.wg_begin.data(), sc.wg_begin.size() * sizeof(int32_t)));
    HIPCHK(up(ds->items, sc.items.data(), sc.items.size() * sizeof(WorkItem)));
    HIPCHK(up(ds->slot_begin, sc.slot_begin.data(), sc.slot_begin.size() * sizeof(int32_t)));
    HIPCHK(up(ds->slot_ids, sc.slot_ids.data(), sc.slot_ids.size() * sizeof(int32_t)));
    HIPCHK(up(ds->lambda_of, lambdas.data(), lambdas.size() * sizeof(int32_t)));
    if (g->schedules.size() > 64) {
        g->drop_graphs();  // captured graphs reference schedule buffers
        g->schedules.clear();
    }
    *out = ds.get();
    g->schedules[key] = std::move(ds);
    return RT_OK;
}

// ---------------------------------------------------------------------------
// formal solution on padded inputs already in place
// ---------------------------------------------------------------------------
// Spherical grid: per chunk, the characteristic kernel writes per-visit
// contributions and the gather sums them into partJ / partL [batch][voxel]
// (stored by the first chunk, accumulated by the others).
static rt_status run_fs_sphere(rt_grid *g, const Variant &v, const std::vector<int32_t> &lambdas, const void *fld,
                               const void *I_bc, DevBuf &partJ, DevBuf &partL, DevSchedule **sched_out,
                               hipStream_t st)
{
    const bool dbl = v.dbl, wj = v.wj, wl = v.wl;
    if (!dbl && g->sph_gdouble) return fail(RT_E_INVALID, "single-precision sweep on a double geometry cache");
    DevSchedule *sc = nullptr;
    rt_status rs = get_schedule(g, 0, lambdas, &sc);
    if (rs != RT_OK) return rs;
    const int nb = (int)lambdas.size();
    const size_t esz = dbl ? 8 : 4;
    if (wj) HIPCHK(partJ.ensure((size_t)nb * g->n_vox * esz));
    if (wl) HIPCHK(partL.ensure((size_t)nb * g->n_vox * esz));
    if ((size_t)nb * g->sph.max_chunk_visits * esz > g->sph_outJ.bytes)
        return fail(RT_E_INVALID, "batch larger than n_lambda_max");
    // lanes per characteristic: the batch entries, up to 16
    int L = 1;
    while (L < nb && L < 16) L *= 2;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (g->prof) {
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        HIPCHK(hipEventRecord(e0, st));
    }
    // chunks kept on the host go through two staging buffers: the copy of the
    // next one (copy stream) overlaps the sweep and gather of the current one
    const size_t n_ch = g->sph_chunks.size();
    std::vector<int> slot_of(n_ch, -1);
    std::vector<size_t> host_order;
    for (size_t c = 0; c < n_ch; ++c)
        if (g->sph_chunks[c]->host) {
            slot_of[c] = (int)(host_order.size() % 2);
            host_order.push_back(c);
        }
    auto issue_copy = [&](size_t k) -> hipError_t {
        const size_t c = host_order[k];
        const int sl = slot_of[c];
        const SphereChunkDev &ch = *g->sph_chunks[c];
        hipError_t e = hipStreamWaitEvent(g->sph_copy, g->sph_done[sl], 0);  // the buffer's last reader is done
        if (e == hipSuccess)
            e = hipMemcpyAsync(g->sph_stage[sl].p, ch.host, ch.bytes, hipMemcpyHostToDevice, g->sph_copy);
        if (e == hipSuccess) e = hipEventRecord(g->sph_copied[sl], g->sph_copy);
        return e;
    };
    size_t next_copy = 0;
    if (!host_order.empty()) {
        HIPCHK(issue_copy(0));
        next_copy = 1;
    }
    for (size_t c = 0; c < n_ch; ++c) {
        const SphereChunkDev &ch = *g->sph_chunks[c];
        const int sl = slot_of[c];
        if (sl >= 0) HIPCHK(hipStreamWaitEvent(st, g->sph_copied[sl], 0));
        const ChunkPtrs cp = chunk_ptrs(ch, sl >= 0 ? g->sph_stage[sl].p : nullptr);
        FsSphereArgs a{};
        a.n_bundles = ch.n_bundles;
        a.bundle_begin = cp.bundle_begin;
        a.char_len = cp.char_len;
        a.char_g = cp.char_g;
        a.vox = cp.vox;
        a.s = cp.s;
        a.w = cp.w;
        a.lambda_of = sc->lambda_of.as<int32_t>();
        a.n_batch = nb;
        a.lam_stride = g->lx;
        a.L = L;
        a.field = fld;
        a.I_bc = I_bc;
        a.outJ = wj ? g->sph_outJ.p : nullptr;
        a.outL = wl ? g->sph_outL.p : nullptr;
        HIPCHK(fs_sphere_launch(a, dbl, g->sph_gdouble, wj, wl, g->para, st));
        if (wj)
            HIPCHK(sphere_gather(g->sph_outJ.p, dbl, cp.row, cp.idx, g->n_vox, nb, partJ.p, dbl, c > 0, st));
        if (wl)
            HIPCHK(sphere_gather(g->sph_outL.p, dbl, cp.row, cp.idx, g->n_vox, nb, partL.p, dbl, c > 0, st));
        if (sl >= 0) {
            HIPCHK(hipEventRecord(g->sph_done[sl], st));
            if (next_copy < host_order.size()) HIPCHK(issue_copy(next_copy++));
        }
    }
    if (g->prof) {
        HIPCHK(hipEventRecord(e1, st));
        g->prof_events.push_back({e0, e1});
        g->prof_points += sc->points;
    }
    *sched_out = sc;
    return RT_OK;
}

static rt_status run_fs_with(rt_grid *g, const Variant &v, const std::vector<int32_t> &lambdas, const void *fld,
                             const void *I_bc, DevBuf &partJ, DevBuf &partL, DevSchedule **sched_out,
                             hipStream_t st, const std::vector<int32_t> *subset = nullptr)
{
    if (g->sphere) return run_fs_sphere(g, v, lambdas, fld, I_bc, partJ, partL, sched_out, st);
    const bool dbl = v.dbl, wj = v.wj, wl = v.wl;
    if (!v.ok) return fail(RT_E_UNSUPPORTED, "no kernel configuration fits this grid (layer tile of %d voxels)",
                           g->geo.Nx * g->geo.Ny);
    DevSchedule *sc = nullptr;
    rt_status rs = get_schedule(g, v.n_wg, lambdas, &sc, subset, &v);
    if (rs != RT_OK) return rs;
    const size_t esz = dbl ? 8 : 4;
    if (wj) HIPCHK(partJ.ensure((size_t)sc->n_slots * g->n_vox * esz));
    if (wl) HIPCHK(partL.ensure((size_t)sc->n_slots * g->n_vox * esz));
    FsBoxArgs a{};
    a.Nx = g->geo.Nx; a.Ny = g->geo.Ny; a.Nz = g->geo.Nz;
    a.n_vox = g->n_vox;
    a.goff = g->goff.as<int32_t>();
    a.dxy = g->dxy.as<uint32_t>();
    a.s = g->s.as<double>();
    a.dir_vbegin = g->vbegin.as<int64_t>();
    a.dir_M = g->M.as<int32_t>();
    a.dir_wmu = g->wmu.as<double>();
    a.dir_mu = g->mu.as<double>();
    a.wg_begin = sc->wg_begin.as<int32_t>();
    a.items = sc->items.as<WorkItem>();
    a.field = fld;
    a.pad_stride = 4 * g->n_vox;
    a.I_bc = I_bc;
    a.partJ = wj ? partJ.p : nullptr;
    a.partL = wl ? partL.p : nullptr;
    a.n_bundles = v.nb;
    a.bundle_rays = v.Q;
    a.tile_words = v.tile_words;
    a.brow = g->brow.as<int32_t>();
    a.dir_span = g->span.as<int32_t>();
    if (g->prof) {
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        HIPCHK(hipEventRecord(e0, st));
        HIPCHK(fs_box_launch(a, dbl, wj, wl, g->para, v.band, v.lb, v.R, sc->n_wg, v.nthr, v.lds, st));
        HIPCHK(hipEventRecord(e1, st));
        g->prof_events.push_back({e0, e1});
        g->prof_points += sc->points;
    } else {
        HIPCHK(fs_box_launch(a, dbl, wj, wl, g->para, v.band, v.lb, v.R, sc->n_wg, v.nthr, v.lds, st));
    }
    *sched_out = sc;
    return RT_OK;
}

static rt_status run_fs(rt_grid *g, bool dbl, bool wj, bool wl, const std::vector<int32_t> &lambdas,
                        const void *fld, const void *I_bc, DevBuf &partJ, DevBuf &partL, DevSchedule **sched_out,
                        hipStream_t st, const std::vector<int32_t> *subset = nullptr)
{
    return run_fs_with(g, variant(g, dbl, wj, wl), lambdas, fld, I_bc, partJ, partL, sched_out, st, subset);
}

// ---------------------------------------------------------------------------
// API
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// spherical geometry cache: traced on host threads direction by direction,
// then uploaded in chunks of consecutive directions
// ---------------------------------------------------------------------------
namespace {

// One direction's characteristics in kernel order (longest first) with
// averaging weights and boundary factors.
struct SphereDirCache {
    std::vector<int64_t> len;     // visits per characteristic
    std::vector<double> g;        // boundary factor
    std::vector<int32_t> vox;
    std::vector<double> s, w;
};

void prepare_sphere_direction(const SphereSpec &spec, double h, const std::vector<Direction> &dirs, int d,
                              std::vector<double> &den, SphereDirCache &out)
{
    SphereTracks tr;
    trace_sphere_direction(spec, h, dirs[d].n, tr);
    const int64_t nc = (int64_t)tr.kind.size();
    // sum of path lengths per voxel in this direction, in trace order
    for (size_t k = 0; k < tr.vox.size(); ++k) den[(size_t)tr.vox[k]] += tr.s[k];
    std::vector<int64_t> order((size_t)nc);
    for (int64_t c = 0; c < nc; ++c) order[(size_t)c] = c;
    std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
        return tr.begin[x + 1] - tr.begin[x] > tr.begin[y + 1] - tr.begin[y];
    });
    out = SphereDirCache();
    out.vox.reserve(tr.vox.size());
    out.s.reserve(tr.vox.size());
    out.w.reserve(tr.vox.size());
    const double wd = dirs[d].w;
    for (int64_t c : order) {
        const int64_t b = tr.begin[c], e = tr.begin[c + 1];
        out.len.push_back(e - b);
        double gc = -1.0;
        if (tr.kind[c] == 0) {
            const double *p = &tr.p[3 * c];
            const double x[3] = {p[0] + tr.ta[c] * dirs[d].n[0], p[1] + tr.ta[c] * dirs[d].n[1],
                                 p[2] + tr.ta[c] * dirs[d].n[2]};
            gc = sphere_irradiation(spec, dirs, d, x);
        }
        out.g.push_back(gc);
        for (int64_t k = b; k < e; ++k) {
            out.vox.push_back(tr.vox[k]);
            out.s.push_back(tr.s[k]);
            out.w.push_back(wd * tr.s[k] / den[(size_t)tr.vox[k]]);
        }
    }
    for (int32_t v : tr.vox) den[(size_t)v] = 0.0;
}

template <typename TG>
hipError_t upload_chunk(SphereChunkDev &ch, const std::vector<SphereDirCache> &dirs, int64_t n_vox, bool force_host)
{
    // every characteristic of the chunk, longest first (ties in direction and trace order)
    struct Ref { int d; int64_t c, off, len; };
    std::vector<Ref> refs;
    int64_t nv = 0;
    for (int d = 0; d < (int)dirs.size(); ++d) {
        int64_t off = 0;
        for (size_t c = 0; c < dirs[d].len.size(); ++c) {
            refs.push_back(Ref{d, (int64_t)c, off, dirs[d].len[c]});
            off += dirs[d].len[c];
        }
        nv += off;
    }
    std::stable_sort(refs.begin(), refs.end(), [](const Ref &a, const Ref &b) { return a.len > b.len; });
    const int64_t nc = (int64_t)refs.size();
    const int64_t nbun = (nc + 63) / 64;
    std::vector<int64_t> bb((size_t)nbun);
    std::vector<int32_t> clen((size_t)nbun * 64, 0);
    std::vector<double> cg((size_t)nbun * 64, 0.0);
    int64_t ne = 0;
    for (int64_t b = 0; b < nbun; ++b) {
        bb[(size_t)b] = ne;
        ne += 64 * refs[(size_t)(b * 64)].len;  // the bundle's first characteristic is its longest
    }
    std::vector<int32_t> vx((size_t)ne, 0);
    std::vector<TG> sv((size_t)ne, TG(0)), wv((size_t)ne, TG(0));
    for (int64_t k = 0; k < nc; ++k) {
        const Ref &r = refs[(size_t)k];
        const int64_t b = k / 64, c = k % 64;
        clen[(size_t)k] = (int32_t)r.len;
        cg[(size_t)k] = dirs[r.d].g[(size_t)r.c];
        for (int64_t m = 0; m < r.len; ++m) {
            const size_t e = (size_t)(bb[(size_t)b] + 64 * m + c);
            const size_t src = (size_t)(r.off + m);
            vx[e] = dirs[r.d].vox[src];
            sv[e] = (TG)dirs[r.d].s[src];
            wv[e] = (TG)dirs[r.d].w[src];
        }
    }
    ch.n_chars = nc;
    ch.n_visits = nv;
    ch.n_bundles = nbun;
    ch.n_entries = ne;
    // CSR voxel -> entries, in entry order
    std::vector<int32_t> row((size_t)n_vox + 1, 0), idx((size_t)nv);
    for (int64_t k = 0; k < nc; ++k) {
        const Ref &r = refs[(size_t)k];
        for (int64_t m = 0; m < r.len; ++m) row[(size_t)dirs[r.d].vox[(size_t)(r.off + m)] + 1]++;
    }
    for (int64_t v = 0; v < n_vox; ++v) row[(size_t)v + 1] += row[(size_t)v];
    std::vector<int32_t> fill(row.begin(), row.end() - 1);
    for (int64_t b = 0; b < nbun; ++b)
        for (int64_t e = bb[(size_t)b]; e < (b + 1 < nbun ? bb[(size_t)b + 1] : ne); ++e) {
            const int64_t m = (e - bb[(size_t)b]) / 64, c = (e - bb[(size_t)b]) % 64;
            if (m < clen[(size_t)(b * 64 + c)]) idx[(size_t)fill[(size_t)vx[(size_t)e]]++] = (int32_t)e;
        }
    // placement: device memory while it lasts (a reserve stays free for the
    // per-visit outputs, partial sums and state), else pinned host memory
    const void *src[8] = {bb.data(), clen.data(), cg.data(), vx.data(), sv.data(), wv.data(), row.data(), idx.data()};
    const size_t len[8] = {bb.size() * 8, clen.size() * 4, cg.size() * 8, vx.size() * 4,
                           sv.size() * sizeof(TG), wv.size() * sizeof(TG), row.size() * 4, idx.size() * 4};
    size_t total = 0;
    for (int i = 0; i < 8; ++i) {
        ch.off[i] = total;
        total += (len[i] + 255) / 256 * 256;
    }
    ch.bytes = total;
    bool to_host = force_host;
    if (!to_host) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return hipErrorOutOfMemory;
        const size_t reserve = std::max<size_t>((size_t)2 << 30, std::min<size_t>((size_t)32 << 30, tot / 8));
        to_host = fr < total + reserve;
    }
    if (to_host) {
        hipError_t e = hipHostMalloc(&ch.host, total, hipHostMallocDefault);
        if (e != hipSuccess) {
            ch.host = nullptr;
            return e;
        }
        for (int i = 0; i < 8; ++i)
            if (len[i]) std::memcpy(static_cast<char *>(ch.host) + ch.off[i], src[i], len[i]);
        return hipSuccess;
    }
    auto up = [](DevBuf &d, const void *src, size_t n) -> hipError_t {
        hipError_t e = d.ensure(n > 0 ? n : 16);
        if (e != hipSuccess || n == 0) return e;
        return hipMemcpy(d.p, src, n, hipMemcpyHostToDevice);
    };
    hipError_t e;
    if ((e = up(ch.bundle_begin, bb.data(), bb.size() * 8)) != hipSuccess) return e;
    if ((e = up(ch.char_len, clen.data(), clen.size() * 4)) != hipSuccess) return e;
    if ((e = up(ch.char_g, cg.data(), cg.size() * 8)) != hipSuccess) return e;
    if ((e = up(ch.vox, vx.data(), vx.size() * 4)) != hipSuccess) return e;
    if ((e = up(ch.s, sv.data(), sv.size() * sizeof(TG))) != hipSuccess) return e;
    if ((e = up(ch.w, wv.data(), wv.size() * sizeof(TG))) != hipSuccess) return e;
    if ((e = up(ch.row, row.data(), row.size() * 4)) != hipSuccess) return e;
    return up(ch.idx, idx.data(), idx.size() * 4);
}

}  // namespace

// Visits per chunk: the per-visit outputs of a chunk take n_lambda_max x
// entries x 16 bytes (double J and Lambda* for the anchors of single-precision
// grids); chunks are sized so that this stays near 8 GiB (of the 288 GB of an
// MI355X; fewer chunks mean fewer gather passes over the voxels).  The
// environment variable RT3D_SPHERE_CHUNK_VISITS overrides the size (smaller
// chunks: less memory, more launches).
static int64_t sphere_chunk_cap(int n_lambda_max)
{
    int64_t cap = ((int64_t)8 << 30) / (16 * (int64_t)n_lambda_max);
    if (const char *e = std::getenv("RT3D_SPHERE_CHUNK_VISITS")) {
        const long long v = std::atoll(e);
        if (v > 0) cap = v;
    }
    return std::min<int64_t>(cap, ((int64_t)1 << 30));  // entries (with bundle padding) stay below 2^31
}

static rt_status build_sphere_grid(rt_grid *g, const rt_grid_desc *desc)
{
    SphereSpec spec;
    spec.Nr = desc->n[0]; spec.Nt = desc->n[1]; spec.Np = desc->n[2];
    spec.rc = desc->h[0]; spec.ro = desc->h[1]; spec.dsrc = desc->h[2];
    spec.n_mu = desc->n_mu; spec.n_phi = desc->n_phi;
    const std::string err = check_sphere_spec(spec);
    if (!err.empty()) return fail(RT_E_INVALID, "%s", err.c_str());
    SphereCache &sc = g->sph;
    sc.spec = spec;
    sc.h = sphere_spacing(spec);
    for (int i = 0; i < spec.n_mu; ++i)
        for (int j = 0; j < spec.n_phi; ++j) sc.dirs.push_back(quadrature_direction(i, j, spec.n_mu, spec.n_phi));
    const int nd = (int)sc.dirs.size();
    const int64_t nvox = (int64_t)spec.Nr * spec.Nt * spec.Np;
    const int64_t cap = sphere_chunk_cap(desc->n_lambda_max);
    unsigned hw = std::thread::hardware_concurrency();
    const int nthr = (int)std::max(1u, std::min(hw == 0 ? 1u : hw, 16u));

    std::vector<SphereDirCache> pending;  // directions of the open chunk
    int64_t pend_visits = 0;
    int chunk_dir0 = 0;
    auto flush = [&](int dir_end) -> rt_status {
        if (pending.empty()) return RT_OK;
        auto ch = std::make_unique<SphereChunkDev>();
        ch->info.dir_begin = chunk_dir0;
        ch->info.dir_end = dir_end;
        hipError_t e = g->sph_gdouble ? upload_chunk<double>(*ch, pending, nvox, g->sph_host_cache)
                                      : upload_chunk<float>(*ch, pending, nvox, g->sph_host_cache);
        if (e != hipSuccess) return fail(RT_E_HIP, "geometry upload: %s", hipGetErrorString(e));
        if (ch->host) {
            g->sph_streaming = true;
            g->cache_host_bytes += (int64_t)ch->bytes;
        } else {
            g->cache_dev_bytes += (int64_t)ch->bytes;
        }
        for (const auto &d : pending)
            for (int64_t l : d.len) ch->info.max_len = std::max<int64_t>(ch->info.max_len, l);
        sc.n_chars += ch->n_chars;
        sc.n_visits += ch->n_visits;
        sc.max_chunk_visits = std::max(sc.max_chunk_visits, ch->n_entries);
        g->sph_chunks.push_back(std::move(ch));
        pending.clear();
        pend_visits = 0;
        chunk_dir0 = dir_end;
        return RT_OK;
    };
    // directions are traced in windows of 2 x threads and consumed in order
    const int win = 2 * nthr;
    for (int d0 = 0; d0 < nd; d0 += win) {
        const int d1 = std::min(nd, d0 + win);
        std::vector<SphereDirCache> res((size_t)(d1 - d0));
        std::atomic<int> next(d0);
        std::vector<std::thread> pool;
        for (int t = 0; t < std::min(nthr, d1 - d0); ++t)
            pool.emplace_back([&]() {
                std::vector<double> den((size_t)nvox, 0.0);
                for (int d = next++; d < d1; d = next++)
                    prepare_sphere_direction(spec, sc.h, sc.dirs, d, den, res[(size_t)(d - d0)]);
            });
        for (auto &th : pool) th.join();
        for (int d = d0; d < d1; ++d) {
            SphereDirCache &dc = res[(size_t)(d - d0)];
            const int64_t nv = (int64_t)dc.vox.size();
            if (nv > cap) return fail(RT_E_INVALID, "direction %d has %lld visits, above the chunk size %lld", d,
                                      (long long)nv, (long long)cap);
            if (pend_visits + nv > cap) {
                rt_status rs = flush(d);
                if (rs != RT_OK) return rs;
            }
            pend_visits += nv;
            pending.push_back(std::move(dc));
        }
    }
    return flush(nd);
}

static rt_status compute_stencil(rt_grid *g, const void *chi, int n_lambda, int nb, const int32_t *lambda_of,
                                 void *out, bool out_double, hipStream_t st);

extern "C" {

const char *rt_last_error(void) { return g_err.c_str(); }

const char *rt_version(void) { return "rt3d 0.1 (gfx950)"; }

rt_status rt_box_template(int32_t Nz, int32_t n_mu, int32_t n_phi, int32_t dir, int32_t cap, int32_t *di,
                          int32_t *dj, int32_t *kk, double *s, int32_t *M)
{
    if (Nz < 1 || n_mu < 2 || (n_mu % 2) || n_phi < 1 || dir < 0 || dir >= n_mu * n_phi || !M)
        return fail(RT_E_INVALID, "bad template request");
    const int i = dir / n_phi, j = dir % n_phi;
    double n[3];
    const double mu = -1.0 + (2.0 * i + 1.0) / n_mu;
    const double phi = 2.0 * M_PI * (j + 0.5) / n_phi;
    const double st = std::sqrt(1.0 - mu * mu);
    n[0] = st * std::cos(phi);
    n[1] = st * std::sin(phi);
    n[2] = mu;
    std::vector<int32_t> a, b, c;
    std::vector<double> l;
    const int m = trace_box_ray(Nz, n, a, b, c, l);
    if (m < 0) return fail(RT_E_INVALID, "tracker failed");
    *M = m;
    if (!di || !dj || !kk || !s) return RT_OK;  // size query
    if (m > cap) return fail(RT_E_INVALID, "cap %d < %d segments", cap, m);
    for (int q = 0; q < m; ++q) { di[q] = a[q]; dj[q] = b[q]; kk[q] = c[q]; s[q] = l[q]; }
    return RT_OK;
}

rt_status rt_sphere_tracks(const rt_grid_desc *desc, int32_t dir, double *h_out, int64_t *n_chars, int64_t *n_visits,
                           double *chars, int64_t *visit_begin, int32_t *vox, double *s)
{
    if (!desc || !n_chars || !n_visits) return fail(RT_E_INVALID, "desc, n_chars and n_visits must not be NULL");
    if (desc->struct_size != sizeof(rt_grid_desc)) return fail(RT_E_INVALID, "desc->struct_size mismatch");
    if (desc->geom != RT_GEOM_SPHERICAL) return fail(RT_E_INVALID, "not a spherical grid");
    SphereSpec spec;
    spec.Nr = desc->n[0]; spec.Nt = desc->n[1]; spec.Np = desc->n[2];
    spec.rc = desc->h[0]; spec.ro = desc->h[1]; spec.dsrc = desc->h[2];
    spec.n_mu = desc->n_mu; spec.n_phi = desc->n_phi;
    const std::string err = check_sphere_spec(spec);
    if (!err.empty()) return fail(RT_E_INVALID, "%s", err.c_str());
    if (dir < 0 || dir >= spec.n_mu * spec.n_phi) return fail(RT_E_INVALID, "direction %d out of range", dir);
    const double h = sphere_spacing(spec);
    const Direction d = quadrature_direction(dir / spec.n_phi, dir % spec.n_phi, spec.n_mu, spec.n_phi);
    SphereTracks tr;
    trace_sphere_direction(spec, h, d.n, tr);
    const int64_t nc = (int64_t)tr.kind.size(), nv = (int64_t)tr.vox.size();
    if (h_out) *h_out = h;
    const bool fill = chars && visit_begin && vox && s;
    if (fill) {
        if (*n_chars < nc || *n_visits < nv) return fail(RT_E_INVALID, "output arrays too small");
        for (int64_t c = 0; c < nc; ++c) {
            double *o = chars + 6 * c;
            o[0] = tr.p[3 * c]; o[1] = tr.p[3 * c + 1]; o[2] = tr.p[3 * c + 2];
            o[3] = tr.ta[c]; o[4] = tr.tb[c]; o[5] = tr.kind[c];
        }
        std::memcpy(visit_begin, tr.begin.data(), (size_t)(nc + 1) * 8);
        std::memcpy(vox, tr.vox.data(), (size_t)nv * 4);
        std::memcpy(s, tr.s.data(), (size_t)nv * 8);
    }
    *n_chars = nc;
    *n_visits = nv;
    return RT_OK;
}

rt_status rt_create_grid(const rt_grid_desc *desc, rt_grid_t *out)
{
    if (!out) return fail(RT_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!desc) return fail(RT_E_INVALID, "desc is NULL");
    if (desc->struct_size != sizeof(rt_grid_desc)) return fail(RT_E_INVALID, "desc->struct_size mismatch");
    if (desc->geom != RT_GEOM_BOX_PERIODIC_XY && desc->geom != RT_GEOM_SPHERICAL)
        return fail(RT_E_INVALID, "unknown geometry %d", desc->geom);
    if (desc->prec != RT_FP32 && desc->prec != RT_FP64) return fail(RT_E_INVALID, "unknown precision %d", desc->prec);
    if (desc->n_lambda_max < 1) return fail(RT_E_INVALID, "n_lambda_max must be >= 1");
    if (desc->flags & ~(RT_F_LSTAR_PARABOLIC | RT_F_BAND_TILES | RT_F_LSTAR_NONLOCAL | RT_F_HOST_CACHE))
        return fail(RT_E_INVALID, "unknown flags 0x%x", desc->flags);
    if (desc->geom == RT_GEOM_BOX_PERIODIC_XY && (desc->flags & RT_F_HOST_CACHE))
        return fail(RT_E_INVALID, "RT_F_HOST_CACHE applies to spherical grids only");
    if (desc->geom == RT_GEOM_SPHERICAL && (desc->flags & (RT_F_BAND_TILES | RT_F_LSTAR_NONLOCAL)))
        return fail(RT_E_INVALID, "RT_F_BAND_TILES and RT_F_LSTAR_NONLOCAL apply to box grids only");
    if (desc->geom == RT_GEOM_SPHERICAL) {
        const int64_t nv = (int64_t)desc->n[0] * desc->n[1] * desc->n[2];
        if (desc->n[0] < 1 || desc->n[1] < 1 || desc->n[2] < 1) return fail(RT_E_INVALID, "grid sizes must be >= 1");
        if (nv > ((int64_t)1 << 30) || nv * 4 * desc->n_lambda_max > (int64_t)1 << 40)
            return fail(RT_E_INVALID, "grid x batch too large");
        if (desc->n_mu > 4096 || desc->n_phi > 4096) return fail(RT_E_INVALID, "direction counts out of range");
        auto g = std::make_unique<rt_grid>();
        g->desc = *desc;
        g->sphere = true;
        g->dbl = desc->prec == RT_FP64;
        g->sph_gdouble = g->dbl;
        g->para = (desc->flags & RT_F_LSTAR_PARABOLIC) != 0;
        g->n_vox = nv;
        g->lx = desc->n_lambda_max; g->ly = 0; g->lz = (int)nv;  // voxel-major pairs [v][n_lambda_max]
        g->nbc = 3;
        g->sph_host_cache = (desc->flags & RT_F_HOST_CACHE) != 0;
        HIPCHK(hipGetDevice(&g->device));
        rt_status rs = build_sphere_grid(g.get(), desc);
        if (rs != RT_OK) return rs;
        if (g->sph_streaming) {
            size_t stage = 0;
            for (const auto &ch : g->sph_chunks)
                if (ch->host) stage = std::max(stage, ch->bytes);
            for (int i = 0; i < 2; ++i) {
                HIPCHK(g->sph_stage[i].ensure(stage));
                HIPCHK(hipEventCreateWithFlags(&g->sph_copied[i], hipEventDisableTiming));
                HIPCHK(hipEventCreateWithFlags(&g->sph_done[i], hipEventDisableTiming));
            }
            HIPCHK(hipStreamCreateWithFlags(&g->sph_copy, hipStreamNonBlocking));
        }
        g->n_dir = (int)g->sph.dirs.size();
        g->n_visits = g->sph.n_visits;
        // per-visit output buffers at their largest size (double, n_lambda_max), so
        // that captured graphs never see them move
        const size_t ob = (size_t)desc->n_lambda_max * (size_t)std::max<int64_t>(g->sph.max_chunk_visits, 1) * 8;
        HIPCHK(g->sph_outJ.ensure(ob));
        HIPCHK(g->sph_outL.ensure(ob));
        // every output combination runs through the same characteristic kernel
        for (int d = 0; d < 2; ++d)
            for (int j = 0; j < 2; ++j)
                for (int l = 0; l < 2; ++l) {
                    Variant &v = variant(g.get(), d, j, l);
                    v = Variant();
                    v.dbl = d; v.wj = j; v.wl = l;
                    v.ok = (j || l) && (d || !g->sph_gdouble);
                }
        *out = g.release();
        g_err.clear();
        return RT_OK;
    }
    const int64_t nv = (int64_t)desc->n[0] * desc->n[1] * desc->n[2];
    if (desc->n[0] < 1 || desc->n[1] < 1 || desc->n[2] < 1) return fail(RT_E_INVALID, "grid sizes must be >= 1");
    if (desc->n[0] > 4096 || desc->n[1] > 4096 || desc->n[2] > 1000000)
        return fail(RT_E_INVALID, "grid sizes out of range");
    if (nv * 4 * desc->n_lambda_max > (int64_t)1 << 40) return fail(RT_E_INVALID, "grid x batch too large");
    if (desc->n_mu > 4096 || desc->n_phi > 4096) return fail(RT_E_INVALID, "direction counts out of range");

    auto g = std::make_unique<rt_grid>();
    g->desc = *desc;
    g->dbl = desc->prec == RT_FP64;
    g->para = (desc->flags & RT_F_LSTAR_PARABOLIC) != 0;
    std::string err = build_box_geometry(desc->n[0], desc->n[1], desc->n[2], desc->n_mu, desc->n_phi, g->geo);
    if (!err.empty()) return fail(RT_E_INVALID, "%s", err.c_str());
    g->n_vox = nv;
    g->n_dir = (int)g->geo.dirs.size();
    g->n_visits = (int64_t)g->geo.s.size();
    g->lx = g->geo.Nx; g->ly = g->geo.Ny; g->lz = g->geo.Nz;
    g->nbc = 2;

    HIPCHK(hipGetDevice(&g->device));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, g->device));
    g->n_cu = prop.multiProcessorCount;
    g->max_lds = prop.sharedMemPerBlock;
    if (prop.maxSharedMemoryPerMultiProcessor > 0 && (size_t)prop.maxSharedMemoryPerMultiProcessor < g->max_lds)
        g->max_lds = prop.maxSharedMemoryPerMultiProcessor;

    const size_t nvis = (size_t)g->n_visits;
    HIPCHK(g->goff.ensure(nvis * 4));
    HIPCHK(g->dxy.ensure(nvis * 4));
    HIPCHK(g->s.ensure(nvis * 8));
    HIPCHK(hipMemcpy(g->goff.p, g->geo.goff.data(), nvis * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(g->dxy.p, g->geo.dxy.data(), nvis * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(g->s.p, g->geo.s.data(), nvis * 8, hipMemcpyHostToDevice));
    HIPCHK(g->brow.ensure(nvis * 4));
    HIPCHK(hipMemcpy(g->brow.p, g->geo.brow.data(), nvis * 4, hipMemcpyHostToDevice));
    HIPCHK(g->comp.ensure(nvis * 4));
    HIPCHK(hipMemcpy(g->comp.p, g->geo.comp.data(), nvis * 4, hipMemcpyHostToDevice));
    g->nonlocal = (desc->flags & RT_F_LSTAR_NONLOCAL) != 0;
    if (g->n_dir > 65535) return fail(RT_E_INVALID, "more than 65535 directions");
    std::vector<int64_t> vb(g->n_dir);
    std::vector<int32_t> Ms(g->n_dir), sp(g->n_dir);
    std::vector<double> wmu(g->n_dir), mu(g->n_dir);
    for (int d = 0; d < g->n_dir; ++d) {
        vb[d] = g->geo.dirs[d].vbegin;
        Ms[d] = g->geo.dirs[d].M;
        sp[d] = g->geo.dirs[d].span;
        g->span_max = std::max(g->span_max, sp[d]);
        wmu[d] = g->geo.dirs[d].w * std::fabs(g->geo.dirs[d].mu);
        mu[d] = g->geo.dirs[d].mu;
    }
    HIPCHK(g->vbegin.ensure(g->n_dir * 8));
    HIPCHK(g->M.ensure(g->n_dir * 4));
    HIPCHK(g->wmu.ensure(g->n_dir * 8));
    HIPCHK(g->mu.ensure(g->n_dir * 8));
    HIPCHK(hipMemcpy(g->vbegin.p, vb.data(), g->n_dir * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(g->M.p, Ms.data(), g->n_dir * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(g->wmu.p, wmu.data(), g->n_dir * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(g->mu.p, mu.data(), g->n_dir * 8, hipMemcpyHostToDevice));
    HIPCHK(g->span.ensure(g->n_dir * 4));
    HIPCHK(hipMemcpy(g->span.p, sp.data(), g->n_dir * 4, hipMemcpyHostToDevice));

    // whole-layer tiles where they fit, else (or when asked for) band tiles
    auto setup_all = [&]() {
        for (int d = 0; d < 2; ++d)
            for (int j = 0; j < 2; ++j)
                for (int l = 0; l < 2; ++l)
                    if (j || l) setup_variant(g.get(), d, j, l);
        const bool self_ok = variant(g.get(), g->dbl, true, false).ok && variant(g.get(), g->dbl, false, true).ok;
        const bool anchor_ok = g->dbl || variant(g.get(), true, true, false).ok;
        return self_ok && anchor_ok;
    };
    g->band = (desc->flags & RT_F_BAND_TILES) != 0;
    bool ok = setup_all();
    if (!ok && !g->band) {
        g->band = true;
        ok = setup_all();
    }
    if (!ok)
        return fail(RT_E_UNSUPPORTED,
                    "layer of %d x %d voxels (row span %d per layer) fits neither a layer tile nor a band tile in "
                    "%zu bytes of LDS",
                    g->geo.Nx, g->geo.Ny, g->span_max, g->max_lds);
    *out = g.release();
    g_err.clear();
    return RT_OK;
}

rt_status rt_destroy_grid(rt_grid_t grid)
{
    if (!grid) return fail(RT_E_INVALID, "grid is NULL");
    (void)hipDeviceSynchronize();
    delete grid;
    return RT_OK;
}

static rt_status autotune(rt_grid *g, int32_t n_lambda, const void *chi, const void *S,
                         const std::vector<int32_t> *subset, int32_t *threads_out, int32_t *rays_out, void *stream)
{
    if (!g) return fail(RT_E_INVALID, "grid is NULL");
    if (n_lambda < 1 || n_lambda > g->desc.n_lambda_max)
        return fail(RT_E_INVALID, "n_lambda %d outside [1, %d]", n_lambda, g->desc.n_lambda_max);
    if (!chi || !S) return fail(RT_E_INVALID, "chi and S must not be NULL");
    if (g->sphere) return fail(RT_E_UNSUPPORTED, "launch shapes apply to the box sweep only");
    hipStream_t st = (hipStream_t)stream;
    const bool dbl = g->dbl;
    const int Nx = g->geo.Nx, Ny = g->geo.Ny, Nz = g->geo.Nz;
    HIPCHK(g->fs_fld.ensure(8 * (size_t)n_lambda * g->n_vox * (dbl ? 8 : 4)));
    if (dbl) {
        HIPCHK(pad_field<double, double>((const double *)chi, nullptr, g->fs_fld.as<double>(), Nx, Ny, Nz, n_lambda, 0, st));
        HIPCHK(pad_field<double, double>((const double *)S, nullptr, g->fs_fld.as<double>(), Nx, Ny, Nz, n_lambda, 1, st));
    } else {
        HIPCHK(pad_field<float, float>((const float *)chi, nullptr, g->fs_fld.as<float>(), Nx, Ny, Nz, n_lambda, 0, st));
        HIPCHK(pad_field<float, float>((const float *)S, nullptr, g->fs_fld.as<float>(), Nx, Ny, Nz, n_lambda, 1, st));
    }
    std::vector<int32_t> lams(n_lambda);
    for (int i = 0; i < n_lambda; ++i) lams[i] = i;
    const FsShape *sh = nullptr;
    const int n = fs_box_shapes(&sh);
    Variant best = variant(g, dbl, true, false);
    float best_ms = 1e30f;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const bool prof = g->prof;
    g->prof = false;
    rt_status rs = RT_OK;
    for (int i = 0; i < n && rs == RT_OK; ++i) {
        // band tiles compete on every grid (their flush covers only the rows a
        // bundle reaches); layer tiles only where the grid is not in band mode
        if (g->band && !sh[i].band) continue;
        const Variant v = make_variant(g, dbl, true, false, sh[i].lb, sh[i].R, sh[i].occ, sh[i].band);
        if (!v.ok) continue;
        DevSchedule *sc = nullptr;
        DevBuf &pJ = dbl ? g->partJ64 : g->partJ;
        DevBuf &pL = dbl ? g->partL64 : g->partL;
        rs = run_fs_with(g, v, lams, g->fs_fld.p, nullptr, pJ, pL, &sc, st, subset);  // warm-up
        if (rs != RT_OK) break;
        if (hipEventRecord(e0, st) != hipSuccess) { rs = fail(RT_E_HIP, "event record failed"); break; }
        rs = run_fs_with(g, v, lams, g->fs_fld.p, nullptr, pJ, pL, &sc, st, subset);
        if (rs != RT_OK) break;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            rs = fail(RT_E_HIP, "event timing failed");
            break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best_ms) { best_ms = ms; best = v; }
    }
    g->prof = prof;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rs != RT_OK) return rs;
    variant(g, dbl, true, false) = best;
    g->tuned = true;
    if (threads_out) *threads_out = best.lb;
    if (rays_out) *rays_out = best.R;
    return RT_OK;
}

rt_status rt_autotune(rt_grid_t g, int32_t n_lambda, const void *chi, const void *S, int32_t *threads_out,
                      int32_t *rays_out, void *stream)
{
    return autotune(g, n_lambda, chi, S, nullptr, threads_out, rays_out, stream);
}

rt_status rt_autotune_dirs(rt_grid_t g, int32_t n_lambda, const void *chi, const void *S, int32_t n_dirs,
                           const int32_t *dirs, int32_t *threads_out, int32_t *rays_out, void *stream)
{
    if (!g) return fail(RT_E_INVALID, "grid is NULL");
    if (g->sphere) return fail(RT_E_UNSUPPORTED, "launch shapes apply to the box sweep only");
    if (n_dirs < 1 || !dirs) return fail(RT_E_INVALID, "need at least one direction");
    std::vector<int32_t> sub(dirs, dirs + n_dirs);
    for (int32_t i = 0; i < n_dirs; ++i) {
        if (sub[i] < 0 || sub[i] >= g->n_dir) return fail(RT_E_INVALID, "direction %d out of range", sub[i]);
        if (i > 0 && sub[i] <= sub[i - 1]) return fail(RT_E_INVALID, "directions must be strictly increasing");
    }
    return autotune(g, n_lambda, chi, S, &sub, threads_out, rays_out, stream);
}

static rt_status set_shape(rt_grid *g, bool dbl, int32_t threads, int32_t rays, int band)
{
    const FsShape *sh = nullptr;
    const int n = fs_box_shapes(&sh);
    for (int pass = 0; pass < 2; ++pass)  // the grid's own tile kind first when band < 0
        for (int i = 0; i < n; ++i) {
            if (sh[i].lb != threads || sh[i].R != rays) continue;
            if (band >= 0 ? sh[i].band != (band != 0) : (sh[i].band != g->band) != (pass == 1)) continue;
            if (g->band && !sh[i].band) continue;
            const Variant v = make_variant(g, dbl, true, false, threads, rays, sh[i].occ, sh[i].band);
            if (!v.ok) continue;
            variant(g, dbl, true, false) = v;
            return RT_OK;
        }
    return fail(RT_E_INVALID, "no compiled launch shape %d threads x %d rays%s that holds the rays of a direction",
                threads, rays, band < 0 ? "" : (band ? " (band tiles)" : " (layer tiles)"));
}

rt_status rt_set_launch_shape_tiles(rt_grid_t g, int32_t threads, int32_t rays, int32_t band)
{
    if (!g) return fail(RT_E_INVALID, "grid is NULL");
    if (g->sphere) return fail(RT_E_UNSUPPORTED, "launch shapes apply to the box sweep only");
    rt_status rs = set_shape(g, g->dbl, threads, rays, band ? 1 : 0);
    if (rs == RT_OK) g->tuned = true;
    return rs;
}

rt_status rt_set_launch_shape(rt_grid_t g, int32_t threads, int32_t rays)
{
    if (!g) return fail(RT_E_INVALID, "grid is NULL");
    if (g->sphere) return fail(RT_E_UNSUPPORTED, "launch shapes apply to the box sweep only");
    rt_status rs = set_shape(g, g->dbl, threads, rays, -1);
    if (rs == RT_OK) g->tuned = true;
    return rs;
}

rt_status rt_set_anchor_shape(rt_grid_t g, int32_t threads, int32_t rays, int32_t band)
{
    if (!g) return fail(RT_E_INVALID, "grid is NULL");
    if (g->sphere) return fail(RT_E_UNSUPPORTED, "launch shapes apply to the box sweep only");
    if (g->dbl) return fail(RT_E_INVALID, "double-precision grids have no anchor sweep");
    return set_shape(g, true, threads, rays, band ? 1 : 0);
}

rt_status rt_lstar_stencil(rt_grid_t g, int32_t n_lambda, const void *chi, void *out, void *stream)
{
    if (!g) return fail(RT_E_INVALID, "grid is NULL");
    if (g->sphere) return fail(RT_E_UNSUPPORTED, "the nearest-neighbour Lambda* is built on box grids");
    if (n_lambda == 0) return RT_OK;
    if (n_lambda < 0 || n_lambda > g->desc.n_lambda_max)
        return fail(RT_E_INVALID, "n_lambda %d outside [0, %d]", n_lambda, g->desc.n_lambda_max);
    if (!chi || !out) return fail(RT_E_INVALID, "chi and out must not be NULL");
    std::vector<int32_t> lams(n_lambda);
    for (int i = 0; i < n_lambda; ++i) lams[i] = i;
    DevSchedule *sc = nullptr;
    rt_status rs = get_schedule(g, variant(g, g->dbl, true, false).n_wg, lams, &sc);
    if (rs != RT_OK) return rs;
    return compute_stencil(g, chi, n_lambda, n_lambda, sc->lambda_of.as<int32_t>(), out, g->dbl,
                           (hipStream_t)stream);
}

rt_status rt_cache_bytes(rt_grid_t g, int64_t *device_bytes, int64_t *host_bytes)
{
    if (!g) return fail(RT_E_INVALID, "grid is NULL");
    int64_t d = g->cache_dev_bytes, h = g->cache_host_bytes;
    if (!g->sphere) d = (int64_t)(g->goff.bytes + g->dxy.bytes + g->s.bytes + g->brow.bytes + g->comp.bytes);
    if (device_bytes) *device_bytes = d;
    if (host_bytes) *host_bytes = h;
    return RT_OK;
}

rt_status rt_launch_shape(rt_grid_t g, int32_t *threads, int32_t *rays, int32_t *bundles, int32_t *band)
{
    if (!g) return fail(RT_E_INVALID, "grid is NULL");
    if (g->sphere) return fail(RT_E_UNSUPPORTED, "launch shapes apply to the box sweep only");
    const Variant &v = variant(g, g->dbl, true, false);
    if (threads) *threads = v.lb;
    if (rays) *rays = v.R;
    if (bundles) *bundles = v.nb;
    if (band) *band = v.band ? 1 : 0;
    return RT_OK;
}

rt_status rt_profile_enable(rt_grid_t g, int32_t enable)
{
    if (!g) return fail(RT_E_INVALID, "grid is NULL");
    g->prof = enable != 0;
    return RT_OK;
}

rt_status rt_profile_read(rt_grid_t g, double *fs_ms, int32_t *fs_launches, int64_t *fs_points)
{
    if (!g) return fail(RT_E_INVALID, "grid is NULL");
    double ms = 0.0;
    for (auto &e : g->prof_events) {
        HIPCHK(hipEventSynchronize(e.second));
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, e.first, e.second));
        ms += t;
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    if (fs_ms) *fs_ms = ms;
    if (fs_launches) *fs_launches = (int32_t)g->prof_events.size();
    if (fs_points) *fs_points = g->prof_points;
    g->prof_events.clear();
    g->prof_points = 0;
    return RT_OK;
}

rt_status rt_grid_info(rt_grid_t g, int64_t *n_vox, int32_t *n_dir, int64_t *n_visits_total, int32_t *n_wg)
{
    if (!g) return fail(RT_E_INVALID, "grid is NULL");
    if (n_vox) *n_vox = g->n_vox;
    if (n_dir) *n_dir = g->n_dir;
    if (n_visits_total) *n_visits_total = g->n_visits;
    if (n_wg) *n_wg = g->sphere ? (int32_t)g->sph_chunks.size() : variant(g, g->dbl, true, false).n_wg;
    return RT_OK;
}

static rt_status formal_solution(rt_grid *g, int32_t n_lambda, const void *chi, const void *S, const void *I_bc,
                                 void *J_out, void *lstar_out, void *stream, const std::vector<int32_t> *subset);

rt_status rt_formal_solution(rt_grid_t g, int32_t n_lambda, const void *chi, const void *S, const void *I_bc,
                             void *J_out, void *lstar_out, void *stream)
{
    return formal_solution(g, n_lambda, chi, S, I_bc, J_out, lstar_out, stream, nullptr);
}

rt_status rt_formal_solution_dirs(rt_grid_t g, int32_t n_lambda, const void *chi, const void *S, const void *I_bc,
                                  int32_t n_dirs, const int32_t *dirs, void *J_out, void *lstar_out, void *stream)
{
    if (!g) return fail(RT_E_INVALID, "grid is NULL");
    if (g->sphere) return fail(RT_E_UNSUPPORTED, "direction subsets apply to box grids");
    if (n_dirs < 1 || !dirs) return fail(RT_E_INVALID, "need at least one direction");
    std::vector<int32_t> sub(dirs, dirs + n_dirs);
    for (int32_t i = 0; i < n_dirs; ++i) {
        if (sub[i] < 0 || sub[i] >= g->n_dir) return fail(RT_E_INVALID, "direction %d out of range", sub[i]);
        if (i > 0 && sub[i] <= sub[i - 1]) return fail(RT_E_INVALID, "directions must be strictly increasing");
    }
    return formal_solution(g, n_lambda, chi, S, I_bc, J_out, lstar_out, stream, &sub);
}

rt_status rt_shard_directions(rt_grid_t g, int32_t n_shards, int32_t shard, int32_t *dirs_out, int32_t *n_out)
{
    if (!g || !n_out) return fail(RT_E_INVALID, "grid and n_out must not be NULL");
    if (g->sphere) return fail(RT_E_UNSUPPORTED, "direction shards apply to box grids");
    if (n_shards < 1 || shard < 0 || shard >= n_shards) return fail(RT_E_INVALID, "shard %d of %d", shard, n_shards);
    const std::vector<int32_t> d = shard_directions(g->geo, n_shards, shard);
    if (dirs_out) std::memcpy(dirs_out, d.data(), d.size() * sizeof(int32_t));
    *n_out = (int32_t)d.size();
    return RT_OK;
}

}  // extern "C"

static rt_status formal_solution(rt_grid *g, int32_t n_lambda, const void *chi, const void *S, const void *I_bc,
                                 void *J_out, void *lstar_out, void *stream, const std::vector<int32_t> *subset)
{
    if (!g) return fail(RT_E_INVALID, "grid is NULL");
    if (n_lambda < 0 || n_lambda > g->desc.n_lambda_max)
        return fail(RT_E_INVALID, "n_lambda %d outside [0, %d]", n_lambda, g->desc.n_lambda_max);
    if (n_lambda == 0) return RT_OK;
    if (!chi || !S || !J_out) return fail(RT_E_INVALID, "chi, S and J_out must not be NULL");
    hipStream_t st = (hipStream_t)stream;
    const bool dbl = g->dbl;
    const size_t esz = dbl ? 8 : 4;
    const size_t padn = g->sphere ? (size_t)g->desc.n_lambda_max * g->n_vox : (size_t)n_lambda * 4 * g->n_vox;
    const int Nx = g->lx, Ny = g->ly, Nz = g->lz;
    HIPCHK(g->fs_fld.ensure(2 * padn * esz));
    if (dbl) {
        HIPCHK(pad_field<double, double>((const double *)chi, nullptr, g->fs_fld.as<double>(), Nx, Ny, Nz, n_lambda, 0, st));
        HIPCHK(pad_field<double, double>((const double *)S, nullptr, g->fs_fld.as<double>(), Nx, Ny, Nz, n_lambda, 1, st));
    } else {
        HIPCHK(pad_field<float, float>((const float *)chi, nullptr, g->fs_fld.as<float>(), Nx, Ny, Nz, n_lambda, 0, st));
        HIPCHK(pad_field<float, float>((const float *)S, nullptr, g->fs_fld.as<float>(), Nx, Ny, Nz, n_lambda, 1, st));
    }
    std::vector<int32_t> lams(n_lambda);
    for (int i = 0; i < n_lambda; ++i) lams[i] = i;
    const bool wl = lstar_out != nullptr;
    DevBuf &pJ = dbl ? g->partJ64 : g->partJ;
    DevBuf &pL = dbl ? g->partL64 : g->partL;
    const bool joint = wl && variant(g, dbl, true, true).ok;
    DevSchedule *sc = nullptr;
    rt_status rs;
    if (joint) {
        rs = run_fs(g, dbl, true, true, lams, g->fs_fld.p, I_bc, pJ, pL, &sc, st, subset);
        if (rs != RT_OK) return rs;
    } else {
        if (wl) {
            rs = run_fs(g, dbl, false, true, lams, g->fs_fld.p, I_bc, pJ, pL, &sc, st, subset);
            if (rs != RT_OK) return rs;
            if (dbl)
                HIPCHK(reduce_partials<double, double>(pL.as<double>(), sc->slot_begin.as<int32_t>(), sc->slot_ids.as<int32_t>(),
                                                       sc->lambda_of.as<int32_t>(), n_lambda, (double *)lstar_out, g->n_vox, st));
            else
                HIPCHK(reduce_partials<float, float>(pL.as<float>(), sc->slot_begin.as<int32_t>(), sc->slot_ids.as<int32_t>(),
                                                     sc->lambda_of.as<int32_t>(), n_lambda, (float *)lstar_out, g->n_vox, st));
        }
        rs = run_fs(g, dbl, true, false, lams, g->fs_fld.p, I_bc, pJ, pL, &sc, st, subset);
        if (rs != RT_OK) return rs;
    }
    if (dbl) {
        HIPCHK(reduce_partials<double, double>(pJ.as<double>(), sc->slot_begin.as<int32_t>(), sc->slot_ids.as<int32_t>(),
                                               sc->lambda_of.as<int32_t>(), n_lambda, (double *)J_out, g->n_vox, st));
        if (joint)
            HIPCHK(reduce_partials<double, double>(pL.as<double>(), sc->slot_begin.as<int32_t>(), sc->slot_ids.as<int32_t>(),
                                                   sc->lambda_of.as<int32_t>(), n_lambda, (double *)lstar_out, g->n_vox, st));
    } else {
        HIPCHK(reduce_partials<float, float>(pJ.as<float>(), sc->slot_begin.as<int32_t>(), sc->slot_ids.as<int32_t>(),
                                             sc->lambda_of.as<int32_t>(), n_lambda, (float *)J_out, g->n_vox, st));
        if (joint)
            HIPCHK(reduce_partials<float, float>(pL.as<float>(), sc->slot_begin.as<int32_t>(), sc->slot_ids.as<int32_t>(),
                                                 sc->lambda_of.as<int32_t>(), n_lambda, (float *)lstar_out, g->n_vox, st));
    }
    return RT_OK;
}

// ---------------------------------------------------------------------------
// ALI
// ---------------------------------------------------------------------------
static rt_status check_state(rt_grid *g, const rt_state *s)
{
    if (!s) return fail(RT_E_INVALID, "state is NULL");
    if (s->struct_size != sizeof(rt_state)) return fail(RT_E_INVALID, "state->struct_size mismatch");
    if (s->n_lambda < 1 || s->n_lambda > g->desc.n_lambda_max)
        return fail(RT_E_INVALID, "state->n_lambda %d outside [1, %d]", s->n_lambda, g->desc.n_lambda_max);
    if (!s->chi || !s->eps || !s->B || !s->J || !s->S || !s->lstar || !s->rel_change)
        return fail(RT_E_INVALID, "state arrays chi, eps, B, J, S, lstar, rel_change must not be NULL");
    if (s->iter < 0) return fail(RT_E_INVALID, "state->iter < 0");
    return RT_OK;
}

static rt_status check_opts(const rt_solve_opts *o)
{
    if (!o) return fail(RT_E_INVALID, "opts is NULL");
    if (o->struct_size != sizeof(rt_solve_opts)) return fail(RT_E_INVALID, "opts->struct_size mismatch");
    if (!(o->tol > 0.0)) return fail(RT_E_INVALID, "opts->tol must be > 0");
    if (o->max_iter < 1) return fail(RT_E_INVALID, "opts->max_iter must be >= 1");
    if (o->ng_every < 0 || o->ng_start < 0 || o->reanchor < 0) return fail(RT_E_INVALID, "negative Ng/anchor option");
    if (o->use_graph != 0 && o->use_graph != 1) return fail(RT_E_INVALID, "opts->use_graph must be 0 or 1");
    if (o->net_every < 0) return fail(RT_E_INVALID, "opts->net_every must be >= 0");
    if (o->method != RT_SOLVER_ALI && o->method != RT_SOLVER_BICGSTAB)
        return fail(RT_E_INVALID, "unknown solver method %d", o->method);
    if (o->os_sweeps < 0 || o->os_sweeps > 1000) return fail(RT_E_INVALID, "opts->os_sweeps outside [0, 1000]");
    return RT_OK;
}

// Allocates the per-state buffers (sized for n_lambda_max) once.
static rt_status ensure_state_buffers(rt_grid *g)
{
    const size_t nl = (size_t)g->desc.n_lambda_max;
    const size_t nv = (size_t)g->n_vox;
    const size_t esz = g->dbl ? 8 : 4;
    HIPCHK(g->fld.ensure(nl * 8 * nv * esz));
    if (!g->dbl) {
        HIPCHK(g->fld64.ensure(nl * 8 * nv * 8));
        HIPCHK(g->J_anchor.ensure(nl * nv * 8));
        HIPCHK(g->S_anchor.ensure(nl * nv * 8));
        HIPCHK(g->ibc64.ensure(nl * 3 * 8));
    }
    HIPCHK(g->hist.ensure(4 * nl * nv * 8));
    HIPCHK(g->ng_blk.ensure(nl * 256 * 5 * 8));
    HIPCHK(g->ng_coef.ensure(nl * 3 * 8));
    HIPCHK(g->resid.ensure(nl * 8));
    if (g->nonlocal) {
        HIPCHK(g->nl_st.ensure(nl * kStencil * nv * esz));
        HIPCHK(g->os_r.ensure(nl * nv * 8));
        HIPCHK(g->os_x0.ensure(nl * nv * 8));
        HIPCHK(g->os_x1.ensure(nl * nv * 8));
    }
    if (g->net) {
        HIPCHK(g->net_r.ensure(nl * nv * 4));
        HIPCHK(g->J_save.ensure(nl * nv * 8));
        HIPCHK(g->net_f.ensure(nv * 3 * 4));
        HIPCHK(g->net_out.ensure(nv * 4));
    }
    return RT_OK;
}

static int os_sweeps_of(const rt_solve_opts *o) { return o->os_sweeps > 0 ? o->os_sweeps : 16; }

// Nearest-neighbour Lambda* of the batch from the caller's opacity, in two
// parts: clear the fixed-point sums and accumulate every characteristic
// (without the centre component when skip_centre), then convert into `out`
// ([lambda][27][vox], double or float), the centre taken from `centre` (the
// diagonal Lambda* of the same operator, [lambda][vox]) when given.
static rt_status accumulate_stencil(rt_grid *g, const void *chi, int n_lambda, int nb, const int32_t *lambda_of,
                                    bool skip_centre, hipStream_t st)
{
    const int64_t per = (int64_t)kStencil * g->n_vox;
    HIPCHK(g->nl_acc.ensure((size_t)n_lambda * per * 8));
    for (int64_t off = 0; off < (int64_t)n_lambda * per; off += (int64_t)1 << 30) {
        const int64_t cnt = std::min<int64_t>((int64_t)1 << 30, (int64_t)n_lambda * per - off);
        HIPCHK(fill_u64(g->nl_acc.as<unsigned long long>() + off, 0ull, (int)cnt, st));
    }
    StencilArgs a{};
    a.Nx = g->geo.Nx; a.Ny = g->geo.Ny; a.Nz = g->geo.Nz;
    a.n_vox = g->n_vox;
    a.dxy = g->dxy.as<uint32_t>();
    a.s = g->s.as<double>();
    a.comp = g->comp.as<uint32_t>();
    a.dir_vbegin = g->vbegin.as<int64_t>();
    a.dir_M = g->M.as<int32_t>();
    a.dir_wmu = g->wmu.as<double>();
    a.dir_mu = g->mu.as<double>();
    a.chi = chi;
    a.lambda_of = lambda_of;
    a.acc = g->nl_acc.as<unsigned long long>();
    a.skip_centre = skip_centre ? 1 : 0;
    HIPCHK(lstar_stencil_accumulate(a, g->dbl, g->para, g->n_dir, nb, st));
    return RT_OK;
}

static rt_status finish_stencil(rt_grid *g, int nb, const int32_t *lambda_of, const void *centre, void *out,
                                bool out_double, hipStream_t st)
{
    HIPCHK(lstar_stencil_finish(g->nl_acc.as<unsigned long long>(), lambda_of, g->n_vox, nb, centre, out, out_double,
                                st));
    return RT_OK;
}

static rt_status compute_stencil(rt_grid *g, const void *chi, int n_lambda, int nb, const int32_t *lambda_of,
                                 void *out, bool out_double, hipStream_t st)
{
    rt_status rs = accumulate_stencil(g, chi, n_lambda, nb, lambda_of, false, st);
    if (rs != RT_OK) return rs;
    return finish_stencil(g, nb, lambda_of, nullptr, out, out_double, st);
}

// The operator-splitting update.  Diagonal Lambda*: the fused pointwise
// kernel.  Nearest-neighbour Lambda*: J_fs - J_old, `sweeps` Jacobi sweeps of
// [1 - Lambda*(1-eps)] dJ = J_fs - J_old started from the diagonal solution,
// then the same update kernel with that dJ (norms, Ng history, S, next input).
static rt_status os_update(rt_grid *g, int n_lambda, AliUpdateArgs ua, bool part_double, bool grid_double,
                           bool next_double, int nb, int sweeps, hipStream_t st)
{
    if (!g->nonlocal) {
        HIPCHK(ali_update(ua, part_double, grid_double, next_double, nb, st));
        return RT_OK;
    }
    (void)n_lambda;
    AliUpdateArgs ra = ua;
    ra.rfs_out = g->os_r.as<double>();
    HIPCHK(ali_update(ra, part_double, grid_double, next_double, nb, st));
    OsJacobiArgs ja{};
    ja.Nx = g->geo.Nx; ja.Ny = g->geo.Ny; ja.Nz = g->geo.Nz;
    ja.n_vox = g->n_vox;
    ja.lambda_of = ua.lambda_of;
    ja.st = g->nl_st.p;
    ja.eps = ua.eps;
    ja.r = g->os_r.as<double>();
    double *x[2] = {g->os_x0.as<double>(), g->os_x1.as<double>()};
    ja.x_in = nullptr;
    ja.x_out = x[0];
    HIPCHK(os_jacobi_sweep(ja, g->dbl, true, nb, st));
    for (int k = 0; k < sweeps; ++k) {
        ja.x_in = x[k % 2];
        ja.x_out = x[(k + 1) % 2];
        HIPCHK(os_jacobi_sweep(ja, g->dbl, false, nb, st));
    }
    ua.rfs_in = g->os_r.as<double>();
    ua.dJ = x[sweeps % 2];
    HIPCHK(ali_update(ua, part_double, grid_double, next_double, nb, st));
    return RT_OK;
}

// The plain step (Lambda* known, no anchor, no Ng): clear the norms, formal
// solution of the current S (FP64 grids) or of S - S_anchor (FP32 grids), and
// the fused update.  Issues only kernel launches, so it can be captured.
static rt_status plain_step_launches(rt_grid *g, rt_state *s, const std::vector<int32_t> &lams,
                                     const int32_t *lambda_of, hipStream_t st, int sweeps, bool keep_hist = true)
{
    const int nl = s->n_lambda, nb = (int)lams.size();
    const int64_t nv = g->n_vox;
    HIPCHK(fill_u64(reinterpret_cast<unsigned long long *>(s->rel_change), 0ull, nl, st));
    HIPCHK(fill_u64(g->resid.as<unsigned long long>(), 0ull, nl, st));
    AliUpdateArgs ua{};
    ua.Nx = g->lx; ua.Ny = g->ly; ua.n_vox = nv;
    ua.resid = g->resid.as<double>();
    ua.net_r = g->net ? g->net_r.as<float>() : nullptr;
    ua.lambda_of = lambda_of;
    ua.eps = s->eps; ua.B = s->B; ua.lstar = s->lstar;
    ua.J = s->J; ua.S = s->S;
    ua.hist = keep_hist ? g->hist.as<double>() + (size_t)(g->hist_count % 4) * nl * nv : nullptr;
    ua.rel_change = s->rel_change;
    ua.next_pad = g->fld.p;
    DevSchedule *sc = nullptr;
    rt_status rs;
    if (g->dbl) {
        rs = run_fs(g, true, true, false, lams, g->fld.p, s->I_bc, g->partJ64, g->partL64, &sc, st);
        if (rs != RT_OK) return rs;
        ua.part = g->partJ64.p;
    } else {
        rs = run_fs(g, false, true, false, lams, g->fld.p, nullptr, g->partJ, g->partL, &sc, st);
        if (rs != RT_OK) return rs;
        ua.part = g->partJ.p;
        ua.S_anchor = g->S_anchor.as<double>();
        ua.J_anchor = g->J_anchor.as<double>();
    }
    ua.slot_begin = sc->slot_begin.as<int32_t>();
    ua.slot_ids = sc->slot_ids.as<int32_t>();
    return os_update(g, nl, ua, g->dbl, g->dbl, g->dbl, nb, sweeps, st);
}

// The plain step through a captured HIP graph: captured on first use for this
// batch, Ng ring slot and state, then replayed.  Schedules and partial-slot
// buffers are prepared before capture so the capture sees launches only.
static rt_status graph_plain_step(rt_grid *g, rt_state *s, const std::vector<int32_t> &lams,
                                  const int32_t *lambda_of, hipStream_t st, int sweeps)
{
    const Variant &v = variant(g, g->dbl, true, false);
    DevSchedule *sc = nullptr;
    rt_status rs = get_schedule(g, v.n_wg, lams, &sc, nullptr, &v);
    if (rs != RT_OK) return rs;
    DevBuf &pJ = g->dbl ? g->partJ64 : g->partJ;
    HIPCHK(pJ.ensure((size_t)sc->n_slots * g->n_vox * (g->dbl ? 8 : 4)));
    char buf[512];
    snprintf(buf, sizeof buf, "%d|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%d|%d|%d|%d:", g->hist_count % 4, (void *)s->J,
             (void *)s->S, s->lstar, s->eps, s->B, (void *)s->rel_change, pJ.p, (void *)st,
             g->net ? g->net_r.p : nullptr, g->resid.p, s->n_lambda, v.lb, v.R, g->nonlocal ? sweeps : -1);
    std::string key(buf);
    for (int l : lams) key += std::to_string(l) + ",";
    auto it = g->graphs.find(key);
    if (it == g->graphs.end()) {
        if (g->graphs.size() > 32) g->drop_graphs();
        const bool prof = g->prof;
        g->prof = false;
        HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        rs = plain_step_launches(g, s, lams, lambda_of, st, sweeps);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(st, &graph);
        g->prof = prof;
        if (rs != RT_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return rs;
        }
        HIPCHK(e);
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCHK(e);
        it = g->graphs.emplace(key, exec).first;
    }
    HIPCHK(hipGraphLaunch(it->second, st));
    return RT_OK;
}

// One ALI step over the wavelengths in `lams` (all of them must be indices < n_lambda).
// candidate: J holds a proposed (learned) iterate; the step neither applies Ng
// nor enters the result into the Ng history, so that a rejected proposal
// leaves the history of plain iterates untouched.
static rt_status ali_step_batch(rt_grid *g, rt_state *s, const rt_solve_opts *o, const std::vector<int32_t> &lams,
                                bool anchor, hipStream_t st, int *fs_count, int *fs64_count, int *ng_count,
                                bool candidate = false)
{
    const int Nx = g->lx, Ny = g->ly, Nz = g->lz;
    const int nl = s->n_lambda;
    const int64_t nv = g->n_vox;
    const int nb = (int)lams.size();
    rt_status rs = ensure_state_buffers(g);
    if (rs != RT_OK) return rs;
    DevSchedule *lam_sc = nullptr;  // for lambda_of of the batch
    rs = get_schedule(g, variant(g, g->dbl, true, false).n_wg, lams, &lam_sc);
    if (rs != RT_OK) return rs;
    const int32_t *lambda_of = lam_sc->lambda_of.as<int32_t>();

    // (re)initialisation: padded opacity, S from J, fresh Ng history
    if (s->iter == 0 || s->chi != g->chi_src) {
        if (g->dbl) {
            HIPCHK(pad_field<double, double>((const double *)s->chi, nullptr, g->fld.as<double>(), Nx, Ny, Nz, nl, 0, st));
        } else {
            HIPCHK(pad_field<float, float>((const float *)s->chi, nullptr, g->fld.as<float>(), Nx, Ny, Nz, nl, 0, st));
            HIPCHK(pad_field<float, double>((const float *)s->chi, nullptr, g->fld64.as<double>(), Nx, Ny, Nz, nl, 0, st));
        }
        g->chi_src = s->chi;
    }
    if (s->iter == 0) {
        g->hist_count = 0;
        if (g->dbl)
            HIPCHK(source_update<double, double>(s->J, (const double *)s->eps, (const double *)s->B, s->S, nullptr,
                                                 g->fld.as<double>(), Nx, Ny, nv, lambda_of, nb, st));
        anchor = true;
    }

    // Ng extrapolation of the last four iterates, due before this step's formal solution
    if (!candidate && o->ng_every > 0 && g->hist_count >= 4 && s->iter >= o->ng_start) {
        NgApplyArgs na{};
        na.Nx = Nx; na.Ny = Ny; na.n_vox = nv;
        na.lambda_of = lambda_of;
        const size_t hs = (size_t)nl * nv;
        double *h = g->hist.as<double>();
        const int c = g->hist_count;  // newest iterate sits in ring slot (c-1) mod 4
        na.x0 = h + (size_t)((c - 1) % 4) * hs;
        na.x1 = h + (size_t)((c - 2) % 4) * hs;
        na.x2 = h + (size_t)((c - 3) % 4) * hs;
        na.x3 = h + (size_t)((c - 4) % 4) * hs;
        na.coef = g->ng_coef.as<double>();
        na.eps = s->eps; na.B = s->B;
        na.S_anchor = g->dbl ? nullptr : g->S_anchor.as<double>();
        na.J = s->J; na.S = s->S;
        na.next_pad = g->fld.p;
        HIPCHK(ng_accelerate(na, g->ng_blk.as<double>(), 256, nb, g->dbl, st));
        g->hist_count = 0;
        ++*ng_count;
    }

    const bool want_l = s->lstar_valid == 0;
    if (!want_l && (g->dbl || !anchor)) {
        if (o->use_graph && st != nullptr && !candidate && !g->sph_streaming)
            rs = graph_plain_step(g, s, lams, lambda_of, st, os_sweeps_of(o));
        else
            rs = plain_step_launches(g, s, lams, lambda_of, st, os_sweeps_of(o), !candidate);
        if (rs != RT_OK) return rs;
        ++*fs_count;
        if (g->dbl) ++*fs64_count;
        if (!candidate) g->hist_count++;
        s->iter++;
        return RT_OK;
    }
    HIPCHK(fill_u64(reinterpret_cast<unsigned long long *>(s->rel_change), 0ull, nl, st));
    HIPCHK(fill_u64(g->resid.as<unsigned long long>(), 0ull, nl, st));
    AliUpdateArgs ua{};
    ua.Nx = Nx; ua.Ny = Ny; ua.n_vox = nv;
    ua.resid = g->resid.as<double>();
    ua.net_r = g->net ? g->net_r.as<float>() : nullptr;
    ua.lambda_of = lambda_of;
    ua.eps = s->eps; ua.B = s->B; ua.lstar = s->lstar;
    ua.J = s->J; ua.S = s->S;
    ua.hist = candidate ? nullptr : g->hist.as<double>() + (size_t)(g->hist_count % 4) * nl * nv;
    ua.rel_change = s->rel_change;
    ua.next_pad = g->fld.p;
    DevSchedule *sc = nullptr;
    const int sweeps = os_sweeps_of(o);
    // The stencil needs only chi and is read only by the OS update: it runs
    // on a side stream, ready from the start of the step and enqueued after
    // the step's sweeps (so that the first sweep's persistent workgroups are
    // placed before its many small ones), and is joined before the update.
    // The atomic-bound stencil build then shares the CUs with the first
    // ALU-bound sweep; a later sweep waits for CUs until the stencil drains.
    // Its sums are integers, so the result does not depend on the overlap.
    bool stencil_pending = want_l && g->nonlocal, stencil_forked = false;
    if (stencil_pending) {
        if (!g->nl_side) HIPCHK(hipStreamCreateWithFlags(&g->nl_side, hipStreamNonBlocking));
        if (!g->nl_fork) HIPCHK(hipEventCreateWithFlags(&g->nl_fork, hipEventDisableTiming));
        if (!g->nl_join) HIPCHK(hipEventCreateWithFlags(&g->nl_join, hipEventDisableTiming));
        HIPCHK(g->nl_acc.ensure((size_t)nl * kStencil * (size_t)nv * 8));  // no reallocation once forked
        HIPCHK(hipEventRecord(g->nl_fork, st));  // chi and the work before this step are ready
    }
    auto fork_stencil = [&]() -> rt_status {
        if (!stencil_pending || stencil_forked) return RT_OK;
        HIPCHK(hipStreamWaitEvent(g->nl_side, g->nl_fork, 0));
        rt_status r = accumulate_stencil(g, s->chi, nl, nb, lambda_of, true, g->nl_side);
        if (r != RT_OK) return r;
        HIPCHK(hipEventRecord(g->nl_join, g->nl_side));
        stencil_forked = true;
        return RT_OK;
    };
    // after the step's diagonal Lambda* is reduced into s->lstar: it is the
    // stencil's centre component (the same sum over the same points)
    auto join_stencil = [&]() -> rt_status {
        rt_status r = fork_stencil();
        if (r != RT_OK) return r;
        if (!stencil_forked) return RT_OK;
        HIPCHK(hipStreamWaitEvent(st, g->nl_join, 0));
        return finish_stencil(g, nb, lambda_of, s->lstar, g->nl_st.p, g->dbl, st);
    };

    if (g->dbl) {
        const bool joint = want_l && variant(g, true, true, true).ok;
        DevSchedule *scL = nullptr;
        if (want_l && !joint) {
            rs = run_fs(g, true, false, true, lams, g->fld.p, s->I_bc, g->partJ64, g->partL64, &scL, st);
            if (rs != RT_OK) return rs;
            ++*fs_count; ++*fs64_count;
        }
        rs = run_fs(g, true, true, joint, lams, g->fld.p, s->I_bc, g->partJ64, g->partL64, &sc, st);
        if (rs != RT_OK) return rs;
        rs = fork_stencil();
        if (rs != RT_OK) return rs;
        ++*fs_count; ++*fs64_count;
        if (scL)  // after the J sweep, so that the two sweeps are queued back to back
            HIPCHK(reduce_partials<double, double>(g->partL64.as<double>(), scL->slot_begin.as<int32_t>(),
                                                   scL->slot_ids.as<int32_t>(), scL->lambda_of.as<int32_t>(), nb,
                                                   (double *)s->lstar, nv, st));
        if (joint)
            HIPCHK(reduce_partials<double, double>(g->partL64.as<double>(), sc->slot_begin.as<int32_t>(), sc->slot_ids.as<int32_t>(),
                                                   sc->lambda_of.as<int32_t>(), nb, (double *)s->lstar, nv, st));
        ua.part = g->partJ64.p;
        ua.slot_begin = sc->slot_begin.as<int32_t>();
        ua.slot_ids = sc->slot_ids.as<int32_t>();
        rs = join_stencil();
        if (rs != RT_OK) return rs;
        rs = os_update(g, nl, ua, true, true, true, nb, sweeps, st);
        if (rs != RT_OK) return rs;
    } else {
        ua.S_anchor = g->S_anchor.as<double>();
        ua.J_anchor = g->J_anchor.as<double>();
        // The anchor's inputs (which the Lambda*-only sweep does not read) are
        // prepared first and the Lambda* reduction follows the anchor sweep, so
        // that the two sweeps are queued back to back.
        const void *ibc = nullptr;
        if (anchor) {
            // double-precision anchor: S_a = S, J_a = Lambda S_a + Lambda_bc
            if (s->iter == 0)
                HIPCHK(source_update<float, double>(s->J, (const float *)s->eps, (const float *)s->B, s->S, nullptr,
                                                    g->fld64.as<double>(), Nx, Ny, nv, lambda_of, nb, st));
            else
                HIPCHK(pad_field<double, double>(s->S, nullptr, g->fld64.as<double>(), Nx, Ny, Nz, nl, 1, st));
            HIPCHK(hipMemcpyAsync(g->S_anchor.p, s->S, (size_t)nl * nv * 8, hipMemcpyDeviceToDevice, st));
            if (s->I_bc) {
                HIPCHK(cast_array<float, double>((const float *)s->I_bc, g->ibc64.as<double>(), (int64_t)g->nbc * nl, st));
                ibc = g->ibc64.p;
            }
        }
        DevSchedule *scL = nullptr;
        if (want_l) {
            rs = run_fs(g, false, false, true, lams, g->fld.p, nullptr, g->partJ, g->partL, &scL, st);
            if (rs != RT_OK) return rs;
            ++*fs_count;
        }
        auto reduce_lstar = [&]() -> rt_status {
            if (scL)
                HIPCHK(reduce_partials<float, float>(g->partL.as<float>(), scL->slot_begin.as<int32_t>(),
                                                     scL->slot_ids.as<int32_t>(), scL->lambda_of.as<int32_t>(), nb,
                                                     (float *)s->lstar, nv, st));
            return RT_OK;
        };
        if (anchor) {
            rs = run_fs(g, true, true, false, lams, g->fld64.p, ibc, g->partJ64, g->partL64, &sc, st);
            if (rs != RT_OK) return rs;
            rs = fork_stencil();
            if (rs != RT_OK) return rs;
            rs = reduce_lstar();
            if (rs != RT_OK) return rs;
            HIPCHK(reduce_partials<double, double>(g->partJ64.as<double>(), sc->slot_begin.as<int32_t>(), sc->slot_ids.as<int32_t>(),
                                                   sc->lambda_of.as<int32_t>(), nb, g->J_anchor.as<double>(), nv, st));
            ++*fs_count; ++*fs64_count;
            ua.part = nullptr;
            ua.slot_begin = sc->slot_begin.as<int32_t>();
            ua.slot_ids = sc->slot_ids.as<int32_t>();
            rs = join_stencil();
            if (rs != RT_OK) return rs;
            rs = os_update(g, nl, ua, false, false, false, nb, sweeps, st);
            if (rs != RT_OK) return rs;
        } else {
            rs = reduce_lstar();
            if (rs != RT_OK) return rs;
            rs = run_fs(g, false, true, false, lams, g->fld.p, nullptr, g->partJ, g->partL, &sc, st);
            if (rs != RT_OK) return rs;
            rs = fork_stencil();
            if (rs != RT_OK) return rs;
            ++*fs_count;
            ua.part = g->partJ.p;
            ua.slot_begin = sc->slot_begin.as<int32_t>();
            ua.slot_ids = sc->slot_ids.as<int32_t>();
            rs = join_stencil();
            if (rs != RT_OK) return rs;
            rs = os_update(g, nl, ua, false, false, false, nb, sweeps, st);
            if (rs != RT_OK) return rs;
        }
    }
    s->lstar_valid = 1;
    if (!candidate) g->hist_count++;
    s->iter++;
    return RT_OK;
}

extern "C" {

rt_status rt_ali_step(rt_grid_t g, rt_state *s, const rt_solve_opts *o, void *stream)
{
    if (!g) return fail(RT_E_INVALID, "grid is NULL");
    rt_status rs = check_state(g, s);
    if (rs != RT_OK) return rs;
    rs = check_opts(o);
    if (rs != RT_OK) return rs;
    std::vector<int32_t> lams(s->n_lambda);
    for (int i = 0; i < s->n_lambda; ++i) lams[i] = i;
    int nfs = 0, nfs64 = 0, nng = 0;
    return ali_step_batch(g, s, o, lams, false, (hipStream_t)stream, &nfs, &nfs64, &nng);
}

// Learned correction of the wavelengths in `lams`: save the plain ALI
// iterate, evaluate the network on (r / max|r|, chi, eps) and scale J.
static rt_status net_propose(rt_grid *g, rt_state *s, const std::vector<int32_t> &lams, const std::vector<double> &res,
                             hipStream_t st)
{
    const int64_t nv = g->n_vox;
    const size_t esz = g->dbl ? 8 : 4;
    for (int l : lams) {
        double *J = s->J + (size_t)l * nv;
        HIPCHK(hipMemcpyAsync(g->J_save.as<double>() + (size_t)l * nv, J, nv * 8, hipMemcpyDeviceToDevice, st));
        const float *r = g->net_r.as<float>() + (size_t)l * nv;
        const char *chi = (const char *)s->chi + (size_t)l * nv * esz;
        const char *eps = (const char *)s->eps + (size_t)l * nv * esz;
        if (g->dbl)
            HIPCHK(unet_features<double>(r, res[l], (const double *)chi, (const double *)eps, nv, g->net_f.as<float>(), st));
        else
            HIPCHK(unet_features<float>(r, res[l], (const float *)chi, (const float *)eps, nv, g->net_f.as<float>(), st));
        HIPCHK(unet_forward(g->net, g->net_f.as<float>(), g->net_out.as<float>(), st));
        HIPCHK(unet_apply(g->net_out.as<float>(), res[l], J, nv, st));
    }
    return RT_OK;
}

// S and the formal-solution input from the current J of the wavelengths in `lams`.
static rt_status refresh_source(rt_grid *g, rt_state *s, const std::vector<int32_t> &lams, hipStream_t st)
{
    DevSchedule *sc = nullptr;
    rt_status rs = get_schedule(g, variant(g, g->dbl, true, false).n_wg, lams, &sc);
    if (rs != RT_OK) return rs;
    const int nb = (int)lams.size();
    if (g->dbl)
        HIPCHK(source_update<double, double>(s->J, (const double *)s->eps, (const double *)s->B, s->S, nullptr,
                                             g->fld.as<double>(), g->lx, g->ly, g->n_vox, sc->lambda_of.as<int32_t>(),
                                             nb, st));
    else
        HIPCHK(source_update<float, float>(s->J, (const float *)s->eps, (const float *)s->B, s->S,
                                           g->S_anchor.as<double>(), g->fld.as<float>(), g->lx, g->ly, g->n_vox,
                                           sc->lambda_of.as<int32_t>(), nb, st));
    return RT_OK;
}

// BiCGStab on A S = b (A = 1 - diag(1-eps) Lambda, b = (1-eps) Lambda_bc + eps B),
// right-preconditioned by M = 1 - (1-eps) Lambda*; every formal solution in
// double precision (single-precision grids use their double anchor input).
static rt_status solve_bicgstab(rt_grid *g, rt_state *s, const rt_solve_opts *o, rt_solve_report *rep, hipStream_t st)
{
    const auto t0 = std::chrono::steady_clock::now();
    rt_solve_report r{};
    const int nl = s->n_lambda;
    const int64_t nv = g->n_vox;
    const size_t vn = (size_t)nl * nv;
    rt_status rs = ensure_state_buffers(g);
    if (rs != RT_OK) return rs;
    std::vector<int32_t> lams(nl);
    for (int i = 0; i < nl; ++i) lams[i] = i;
    DevSchedule *lsc = nullptr;
    rs = get_schedule(g, variant(g, g->dbl, true, false).n_wg, lams, &lsc);
    if (rs != RT_OK) return rs;
    const int32_t *lambda_of = lsc->lambda_of.as<int32_t>();
    const int nblk = 64;
    HIPCHK(g->kvec.ensure(13 * vn * 8));
    HIPCHK(g->kblk.ensure((size_t)nl * nblk * 4 * 8));
    HIPCHK(g->kout.ensure((size_t)nl * 4 * 8));
    HIPCHK(g->kc.ensure((size_t)nl * 4 * 8));
    double *V = g->kvec.as<double>();
    KVec a{};
    a.eps = s->eps; a.B = s->B; a.lstar = s->lstar; a.c = g->kc.as<double>();
    a.x = V; a.y = V + vn; a.u = V + 2 * vn; a.b = V + 3 * vn; a.r = V + 4 * vn; a.rh = V + 5 * vn;
    a.p = V + 6 * vn; a.v = V + 7 * vn; a.ph = V + 8 * vn; a.s = V + 9 * vn; a.sh = V + 10 * vn; a.t = V + 11 * vn;
    double *zero = V + 12 * vn;
    a.J = s->J;
    const int lx = g->lx, ly = g->ly, lz = g->lz;
    double *fpad = g->dbl ? g->fld.as<double>() : g->fld64.as<double>();
    // opacity into the double formal-solution input; Lambda* in grid precision if needed
    if (g->dbl) {
        HIPCHK(pad_field<double, double>((const double *)s->chi, nullptr, fpad, lx, ly, lz, nl, 0, st));
    } else {
        HIPCHK(pad_field<float, double>((const float *)s->chi, nullptr, fpad, lx, ly, lz, nl, 0, st));
        HIPCHK(pad_field<float, float>((const float *)s->chi, nullptr, g->fld.as<float>(), lx, ly, lz, nl, 0, st));
    }
    g->chi_src = nullptr;  // the ALI inputs are re-initialised by the next ALI step
    DevSchedule *sc = nullptr;
    if (s->lstar_valid == 0) {
        if (g->dbl) {
            rs = run_fs(g, true, false, true, lams, fpad, nullptr, g->partJ64, g->partL64, &sc, st);
            if (rs != RT_OK) return rs;
            HIPCHK(reduce_partials<double, double>(g->partL64.as<double>(), sc->slot_begin.as<int32_t>(),
                                                   sc->slot_ids.as<int32_t>(), sc->lambda_of.as<int32_t>(), nl,
                                                   (double *)s->lstar, nv, st));
        } else {
            rs = run_fs(g, false, false, true, lams, g->fld.p, nullptr, g->partJ, g->partL, &sc, st);
            if (rs != RT_OK) return rs;
            HIPCHK(reduce_partials<float, float>(g->partL.as<float>(), sc->slot_begin.as<int32_t>(),
                                                 sc->slot_ids.as<int32_t>(), sc->lambda_of.as<int32_t>(), nl,
                                                 (float *)s->lstar, nv, st));
        }
        s->lstar_valid = 1;
        r.n_fs++;
        if (g->dbl) r.n_fs64++;
    }
    const void *ibc = s->I_bc;
    if (s->I_bc && !g->dbl) {
        HIPCHK(cast_array<float, double>((const float *)s->I_bc, g->ibc64.as<double>(), (int64_t)g->nbc * nl, st));
        ibc = g->ibc64.p;
    }
    // y = Lambda src (+ Lambda_bc when bc), double precision
    auto fs64 = [&](const double *src, const void *bc, double *out) -> rt_status {
        HIPCHK(pad_field<double, double>(src, nullptr, fpad, lx, ly, lz, nl, 1, st));
        DevSchedule *sc2 = nullptr;
        rt_status rs2 = run_fs(g, true, true, false, lams, fpad, bc, g->partJ64, g->partL64, &sc2, st);
        if (rs2 != RT_OK) return rs2;
        HIPCHK(reduce_partials<double, double>(g->partJ64.as<double>(), sc2->slot_begin.as<int32_t>(),
                                               sc2->slot_ids.as<int32_t>(), sc2->lambda_of.as<int32_t>(), nl, out, nv,
                                               st));
        r.n_fs++;
        r.n_fs64++;
        return RT_OK;
    };
    std::vector<double> dots(4 * nl), c(4 * nl, 0.0);
    auto dot = [&](int n, const double *x0, const double *y0, const double *x1 = nullptr,
                   const double *y1 = nullptr) -> rt_status {
        KDots d{};
        d.n = n;
        d.a[0] = x0; d.b[0] = y0; d.a[1] = x1 ? x1 : x0; d.b[1] = y1 ? y1 : y0;
        d.a[2] = d.a[3] = x0; d.b[2] = d.b[3] = y0;
        HIPCHK(krylov_dots(d, nv, nl, g->kblk.as<double>(), nblk, g->kout.as<double>(), st));
        HIPCHK(hipMemcpyAsync(dots.data(), g->kout.p, 4 * nl * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        return RT_OK;
    };
    auto put = [&]() -> rt_status {
        HIPCHK(hipMemcpyAsync(g->kc.p, c.data(), 4 * nl * sizeof(double), hipMemcpyHostToDevice, st));
        return RT_OK;
    };
    auto vec = [&](int op) -> rt_status {
        HIPCHK(krylov_vec(a, op, nv, nl, g->dbl, st));
        return RT_OK;
    };
#define RT_TRY(x) do { rt_status rs_ = (x); if (rs_ != RT_OK) return rs_; } while (0)
    // b, x0 = S(J), r0
    HIPCHK(hipMemsetAsync(zero, 0, vn * 8, st));
    RT_TRY(fs64(zero, ibc, a.u));  // Lambda_bc
    if (g->dbl)
        HIPCHK(source_update<double, double>(s->J, (const double *)s->eps, (const double *)s->B, a.x, nullptr, fpad,
                                             lx, ly, nv, lambda_of, nl, st));
    else
        HIPCHK(source_update<float, double>(s->J, (const float *)s->eps, (const float *)s->B, a.x, nullptr, fpad, lx,
                                            ly, nv, lambda_of, nl, st));
    RT_TRY(fs64(a.x, nullptr, a.y));
    RT_TRY(vec(KOP_RHS));
    RT_TRY(dot(2, a.b, a.b, a.r, a.r));
    std::vector<double> bnorm(nl), res(nl), rho_old(nl, 1.0), alpha(nl, 1.0), omega(nl, 1.0);
    std::vector<char> done(nl, 0);
    for (int l = 0; l < nl; ++l) {
        bnorm[l] = std::sqrt(dots[4 * l]);
        res[l] = bnorm[l] > 0.0 ? std::sqrt(dots[4 * l + 1]) / bnorm[l] : 0.0;
        done[l] = !(res[l] >= o->tol);
    }
    auto all_done = [&]() {
        for (int l = 0; l < nl; ++l)
            if (!done[l]) return false;
        return true;
    };
    for (int it = 0; it < o->max_iter && !all_done(); ++it) {
        r.iters++;
        RT_TRY(dot(1, a.rh, a.r));
        for (int l = 0; l < nl; ++l) {
            const double rho = dots[4 * l];
            if (done[l] || rho == 0.0) { done[l] = 1; c[4 * l] = 0.0; c[4 * l + 1] = 0.0; continue; }
            c[4 * l] = it == 0 ? 0.0 : (rho / rho_old[l]) * (alpha[l] / omega[l]);
            c[4 * l + 1] = omega[l];
            rho_old[l] = rho;
        }
        RT_TRY(put());
        RT_TRY(vec(KOP_P));
        RT_TRY(fs64(a.ph, nullptr, a.y));
        RT_TRY(vec(KOP_AV));
        RT_TRY(dot(1, a.rh, a.v));
        for (int l = 0; l < nl; ++l) {
            const double rv = dots[4 * l];
            alpha[l] = (!done[l] && rv != 0.0) ? rho_old[l] / rv : 0.0;
            c[4 * l] = alpha[l];
        }
        RT_TRY(put());
        RT_TRY(vec(KOP_S));
        RT_TRY(dot(1, a.s, a.s));
        bool s_conv = true;
        for (int l = 0; l < nl; ++l)
            if (!done[l] && !(std::sqrt(dots[4 * l]) / bnorm[l] < o->tol)) s_conv = false;
        if (s_conv) {
            RT_TRY(vec(KOP_XH));
            for (int l = 0; l < nl; ++l)
                if (!done[l]) { res[l] = std::sqrt(dots[4 * l]) / bnorm[l]; done[l] = 1; }
            break;
        }
        RT_TRY(fs64(a.sh, nullptr, a.y));
        RT_TRY(vec(KOP_AT));
        RT_TRY(dot(2, a.t, a.s, a.t, a.t));
        for (int l = 0; l < nl; ++l) {
            const double ts = dots[4 * l], tt = dots[4 * l + 1];
            omega[l] = (!done[l] && tt > 0.0) ? ts / tt : 0.0;
            c[4 * l] = done[l] ? 0.0 : alpha[l];
            c[4 * l + 1] = omega[l];
            if (!done[l] && omega[l] == 0.0) done[l] = 1;  // breakdown: keep the last iterate
        }
        RT_TRY(put());
        RT_TRY(vec(KOP_X));
        RT_TRY(dot(1, a.r, a.r));
        for (int l = 0; l < nl; ++l) {
            if (done[l]) continue;
            res[l] = std::sqrt(dots[4 * l]) / bnorm[l];
            if (!(res[l] <= 1e308)) {
                r.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
                if (rep) *rep = r;
                return fail(RT_E_NUMERIC, "non-finite BiCGStab residual in wavelength %d", l);
            }
            if (res[l] < o->tol) done[l] = 1;
        }
    }
    // J = Lambda S + Lambda_bc, S = (1-eps) J + eps B; the state restarts its ALI history
    RT_TRY(fs64(a.x, nullptr, a.y));
    RT_TRY(vec(KOP_J));
    if (g->dbl)
        HIPCHK(source_update<double, double>(s->J, (const double *)s->eps, (const double *)s->B, s->S, nullptr,
                                             g->fld.as<double>(), lx, ly, nv, lambda_of, nl, st));
    else
        HIPCHK(source_update<float, double>(s->J, (const float *)s->eps, (const float *)s->B, s->S, nullptr, fpad, lx,
                                            ly, nv, lambda_of, nl, st));
#undef RT_TRY
    HIPCHK(hipMemcpyAsync(s->rel_change, res.data(), nl * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    s->iter = 0;
    g->hist_count = 0;
    int nconv = 0;
    double mx = 0.0;
    for (int l = 0; l < nl; ++l) {
        if (res[l] < o->tol) nconv++;
        mx = std::max(mx, res[l]);
    }
    r.n_converged = nconv;
    r.max_rel_change = mx;
    r.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rep) *rep = r;
    if (nconv < nl)
        return fail(RT_E_NOT_CONVERGED, "%d of %d wavelengths above the BiCGStab tolerance after %d iterations",
                    nl - nconv, nl, o->max_iter);
    g_err.clear();
    return RT_OK;
}

rt_status rt_solve(rt_grid_t g, rt_state *s, const rt_solve_opts *o, rt_solve_report *rep, void *stream)
{
    if (!g) return fail(RT_E_INVALID, "grid is NULL");
    rt_status rs = check_state(g, s);
    if (rs != RT_OK) return rs;
    rs = check_opts(o);
    if (rs != RT_OK) return rs;
    hipStream_t st = (hipStream_t)stream;
    if (o->method == RT_SOLVER_BICGSTAB) return solve_bicgstab(g, s, o, rep, st);
    const auto t0 = std::chrono::steady_clock::now();
    rt_solve_report r{};
    const int nl = s->n_lambda;
    const int64_t nv = g->n_vox;
    std::vector<int32_t> active(nl);
    for (int i = 0; i < nl; ++i) active[i] = i;
    std::vector<double> rel(nl, 0.0), res(nl, 0.0), res_before(nl, 0.0), res_prev(nl, 0.0), res_goal(nl, 0.0);
    const double refac = o->reanchor > 0 ? (double)o->reanchor : 100.0;
    const bool use_net = g->net != nullptr && o->net_every > 0;
    // Learned corrections: after a proposal, one ALI sweep smooths the candidate
    // (phase 1), and the residual of the smoothed candidate, measured by the
    // sweep after it (phase 2), decides.  The network removes smooth error that
    // the residual hardly sees and leaves small-scale error that the residual
    // amplifies and one sweep removes, so the raw candidate's residual would
    // misjudge it.  The goal is the residual the plain iteration would reach
    // in the same two steps, from its recent contraction.
    std::vector<int32_t> pending;  // wavelengths whose J descends from a learned candidate
    int phase = 0;
    int since_net = 0;
    double rel_at_anchor = 1e300;
    bool anchor_next = true;
    rt_status out = RT_E_NOT_CONVERGED;
    for (int it = 0; it < o->max_iter; ++it) {
        const bool cand = !pending.empty();
        const bool anchor = !g->dbl && !cand && (anchor_next || s->iter == 0);
        rs = ali_step_batch(g, s, o, active, anchor, st, &r.n_fs, &r.n_fs64, &r.n_ng, cand);
        if (rs != RT_OK) return rs;
        HIPCHK(hipMemcpyAsync(rel.data(), s->rel_change, nl * sizeof(double), hipMemcpyDeviceToHost, st));
        if (use_net) HIPCHK(hipMemcpyAsync(res.data(), g->resid.p, nl * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        r.iters++;
        // verdict on pending candidates: this step's residual is that of the smoothed candidate
        std::vector<int32_t> rejected;
        if (!pending.empty() && phase == 1) {
            phase = 2;
        } else if (!pending.empty()) {
            for (int l : pending) {
                if (res[l] < res_goal[l]) r.n_net_accept++;
                else rejected.push_back(l);
            }
            r.n_net_reject += (int)rejected.size();
            for (int l : rejected)
                HIPCHK(hipMemcpyAsync(s->J + (size_t)l * nv, g->J_save.as<double>() + (size_t)l * nv, nv * 8,
                                      hipMemcpyDeviceToDevice, st));
            if (!rejected.empty()) {
                rs = refresh_source(g, s, rejected, st);
                if (rs != RT_OK) return rs;
            }
            // an accepted correction breaks the sequence of plain iterates Ng works on;
            // when every proposal is rejected the plain trajectory continues unchanged
            if (rejected.size() != pending.size()) g->hist_count = 0;
            pending.clear();
            phase = 0;
        }
        double mx = 0.0;
        std::vector<int32_t> still;
        for (int l : active) {
            // a rejected candidate's step is discarded, whatever it produced
            if (std::find(rejected.begin(), rejected.end(), l) != rejected.end()) {
                still.push_back(l);
                continue;
            }
            if (!(rel[l] <= 1e308)) {
                r.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
                if (rep) *rep = r;
                return fail(RT_E_NUMERIC, "non-finite J in wavelength %d at step %d", l, s->iter);
            }
            if (rel[l] >= o->tol) still.push_back(l);
            mx = rel[l] > mx ? rel[l] : mx;
        }
        r.max_rel_change = mx;
        if (!cand) {  // candidate steps do not move the anchor schedule
            if (anchor) rel_at_anchor = mx;
            anchor_next = !g->dbl && mx < rel_at_anchor / refac;
        }
        active.swap(still);
        if (!pending.empty()) {  // candidates that converged during smoothing need no verdict
            std::vector<int32_t> keep;
            for (int l : pending)
                if (std::find(active.begin(), active.end(), l) != active.end()) keep.push_back(l);
                else r.n_net_accept++;
            pending.swap(keep);
            if (pending.empty()) phase = 0;
        }
        if (active.empty()) { out = RT_OK; break; }
        // propose a learned correction for the wavelengths still iterating
        if (!cand) {
            ++since_net;
            for (int l : active) {
                res_prev[l] = res_before[l];
                res_before[l] = res[l];
            }
        }
        if (use_net && !cand && since_net >= o->net_every && it + 2 < o->max_iter) {
            for (int l : active)
                if (res[l] > 0.0 && res[l] <= 1e308) pending.push_back(l);
            if (!pending.empty()) {
                rs = net_propose(g, s, pending, res, st);
                if (rs != RT_OK) return rs;
                rs = refresh_source(g, s, pending, st);
                if (rs != RT_OK) return rs;
                for (int l : pending) {
                    const double q = res_prev[l] > 0.0 ? std::min(1.0, res[l] / res_prev[l]) : 1.0;
                    res_goal[l] = res[l] * q * q;
                }
                phase = 1;
            }
            since_net = 0;
        }
    }
    // a candidate still pending at max_iter has not been checked: return the plain iterate
    if (!pending.empty()) {
        for (int l : pending)
            HIPCHK(hipMemcpyAsync(s->J + (size_t)l * nv, g->J_save.as<double>() + (size_t)l * nv, nv * 8,
                                  hipMemcpyDeviceToDevice, st));
        rs = refresh_source(g, s, pending, st);
        if (rs != RT_OK) return rs;
        HIPCHK(hipStreamSynchronize(st));
    }
    r.n_converged = nl - (int)active.size();
    r.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rep) *rep = r;
    if (out != RT_OK) return fail(RT_E_NOT_CONVERGED, "%d of %d wavelengths not converged after %d steps",
                                  (int)active.size(), nl, o->max_iter);
    g_err.clear();
    return RT_OK;
}

rt_status rt_set_preconditioner(rt_grid_t g, const void *blob, size_t bytes)
{
    if (!g) return fail(RT_E_INVALID, "grid is NULL");
    if (g->sphere) return fail(RT_E_UNSUPPORTED, "the learned correction is available on box grids only");
    HIPCHK(hipDeviceSynchronize());
    g->drop_graphs();
    if (g->net) { unet_destroy(g->net); g->net = nullptr; }
    if (!blob) return RT_OK;
    UNetSpec spec;
    std::string err = parse_unet(blob, bytes, spec);
    if (!err.empty()) return fail(RT_E_INVALID, "%s", err.c_str());
    UNetDev *u = unet_create(spec, g->geo.Nx, g->geo.Ny, g->geo.Nz, err);
    if (!u) return fail(RT_E_HIP, "%s", err.c_str());
    g->net = u;
    return RT_OK;
}

rt_status rt_precond_forward(rt_grid_t g, const float *features, float *out, void *stream)
{
    if (!g) return fail(RT_E_INVALID, "grid is NULL");
    if (!g->net) return fail(RT_E_INVALID, "no network set (rt_set_preconditioner)");
    if (!features || !out) return fail(RT_E_INVALID, "features and out must not be NULL");
    HIPCHK(unet_forward(g->net, features, out, (hipStream_t)stream));
    return RT_OK;
}

}  // extern "C"
