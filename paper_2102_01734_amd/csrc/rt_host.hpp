// rt_host.hpp -- host-side internals shared by the api_*.cpp modules of the C
// ABI (include/rt3d.h): the grid handle, device buffers, launch variants,
// schedules, error reporting, and the functions one module calls in another.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
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

// internal header of the api_*.cpp modules only
using namespace rt3d;

// ---------------------------------------------------------------------------
// errors: a thread-local message for rt_last_error
// ---------------------------------------------------------------------------
rt_status fail(rt_status st, const char *fmt, ...);
void clear_error();

// Maps a failed HIP call to RT_E_NOMEM (out of device or pinned memory) or
// RT_E_HIP, with the message for rt_last_error.
rt_status hip_fail(hipError_t e, const char *file, int line);

#define HIPCHK(...)                                              \
    do {                                                         \
        hipError_t e_ = (__VA_ARGS__);                           \
        if (e_ != hipSuccess) return hip_fail(e_, __FILE__, __LINE__); \
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
    bool spill = false;  // the compiled kernel keeps part of its state in scratch memory
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
    // per direction, the stencil components it adds to and their LDS planes in
    // the row-window stencil kernel ([with centre, without][dir][kPlaneStride]),
    // the plane counts, and whether every template's row offsets move by at
    // most one row per visit, one way within a layer (else the per-
    // characteristic kernel is used)
    DevBuf nl_planes;
    bool os_gs = false;  // the current step's OS sweeps are Gauss-Seidel (set from its options)
    int nl_np[2] = {0, 0};
    bool nl_rows = false;
    // the stencil of an ALI step runs on a side stream beside its formal solutions
    hipStream_t nl_side = nullptr;
    hipEvent_t nl_fork = nullptr, nl_join = nullptr;
    int span_max = 0;   // largest per-layer row extent of any template
    bool band = false;  // the box sweep uses band tiles (see fs_box.hip)
    bool layer_ok = false;  // whole-layer tiles fit (and were not excluded by RT_F_BAND_TILES)
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
    // the state the per-state scratch above belongs to (its array pointers
    // and batch size), whether its double anchor (FP32 grids) and its
    // nearest-neighbour stencil (nl_st) are in place
    const void *own[8] = {};
    bool anchor_ok = false, nl_ok = false;
    bool owned_by(const rt_state *st) const
    {
        const void *k[8] = {st->chi, st->eps, st->B, st->I_bc, st->J, st->S, st->lstar,
                            reinterpret_cast<const void *>((intptr_t)st->n_lambda)};
        return std::equal(k, k + 8, own);
    }
    void take_ownership(const rt_state *st)
    {
        const void *k[8] = {st->chi, st->eps, st->B, st->I_bc, st->J, st->S, st->lstar,
                            reinterpret_cast<const void *>((intptr_t)st->n_lambda)};
        std::copy(k, k + 8, own);
        anchor_ok = nl_ok = false;
        chi_src = nullptr;
    }
    void release_ownership()
    {
        std::fill(own, own + 8, nullptr);
        anchor_ok = nl_ok = false;
        chi_src = nullptr;
        hist_count = 0;
    }
    // captured plain ALI steps, keyed by batch, ring slot and state pointers
    // Captured plain ALI steps.  With the measurement hooks on, the sweep of
    // a captured step is bracketed by two wall-clock stamp kernels writing
    // into the graph's own `stamps` (two uint64); the time of a replay is
    // collected before the next replay of the same graph and by
    // rt_profile_read.
    struct GraphStep {
        hipGraphExec_t exec = nullptr;
        hipStream_t stream = nullptr;
        std::shared_ptr<DevBuf> stamps;
        int64_t points = 0;
        bool pending = false;
    };
    std::map<std::string, GraphStep> graphs;
    // stamps to write around the next box sweep of a capture, and its points
    unsigned long long *cap_stamps = nullptr;
    int64_t cap_points = 0;
    int wall_khz = 0;  // device wall-clock rate
    double prof_graph_ms = 0.0;
    int32_t prof_graph_launches = 0;
    // BiCGStab vectors and reduction scratch
    DevBuf kvec, kblk, kout, kc;
    // learned ALI correction
    UNetDev *net = nullptr;
    DevBuf net_r, net_f, net_out, J_save, resid;
    // rt_formal_solution_noalloc: this device's copy of the fixed scratch
    // array, the schedules planned for it (host copies, kept for the
    // asynchronous uploads) and the batch indices 0 .. n_lambda_max-1
    void *na_scratch = nullptr;
    std::map<std::string, std::unique_ptr<Schedule>> na_sched;
    std::vector<int32_t> iota_lams;
    // measurement hooks
    bool prof = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_events;
    int64_t prof_points = 0;
    void drop_graphs()
    {
        for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second.exec);
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

inline Variant &variant(rt_grid *g, bool dbl, bool wj, bool wl) { return g->var[dbl][wj][wl]; }

// ---------------------------------------------------------------------------
// functions shared between the modules
// ---------------------------------------------------------------------------
// launch shapes and schedules (api_launch.cpp)
// Adds the sweep time of a profiled graph replay (waits for it).
rt_status collect_graph_time(rt_grid *g, rt_grid::GraphStep &gs);

// ok = false for shapes that cannot hold a bundle's rays, whose tiles do not
// fit, or (unless allow_spill) whose kernel spills registers
Variant make_variant(rt_grid *g, bool dbl, bool wj, bool wl, int lb, int R, int occ = 1, bool band = false,
                     bool allow_spill = false);
void setup_variant(rt_grid *g, bool dbl, bool wj, bool wl);
rt_status get_schedule(rt_grid *g, int n_wg, const std::vector<int32_t> &lambdas, DevSchedule **out,
                       const std::vector<int32_t> *subset = nullptr, const Variant *v = nullptr);
rt_status run_fs_with(rt_grid *g, const Variant &v, const std::vector<int32_t> &lambdas, const void *fld,
                      const void *I_bc, DevBuf &partJ, DevBuf &partL, DevSchedule **sched_out, hipStream_t st,
                      const std::vector<int32_t> *subset = nullptr);
rt_status run_fs(rt_grid *g, bool dbl, bool wj, bool wl, const std::vector<int32_t> &lambdas, const void *fld,
                 const void *I_bc, DevBuf &partJ, DevBuf &partL, DevSchedule **sched_out, hipStream_t st,
                 const std::vector<int32_t> *subset = nullptr);
rt_status formal_solution(rt_grid *g, int32_t n_lambda, const void *chi, const void *S, const void *I_bc,
                          void *J_out, void *lstar_out, void *stream, const std::vector<int32_t> *subset);

// nearest-neighbour Lambda* (api_stencil.cpp)
// Device pointers of a chunk (stage: its staging copy for host-resident chunks, else null).
ChunkPtrs chunk_ptrs(const SphereChunkDev &ch, const void *stage);
rt_status accumulate_stencil(rt_grid *g, const void *chi, int n_lambda, int nb, const int32_t *lambda_of,
                             bool skip_centre, hipStream_t st);
rt_status finish_stencil(rt_grid *g, int nb, const int32_t *lambda_of, const void *centre, void *out,
                         bool out_double, hipStream_t st);
rt_status compute_stencil(rt_grid *g, const void *chi, int n_lambda, int nb, const int32_t *lambda_of, void *out,
                          bool out_double, hipStream_t st);

// device address of this device's copy of the no-allocation scratch array,
// looked up once per device (api_noalloc.hip)
rt_status noalloc_scratch_setup(int device, void **out);

// ALI state (api_ali.cpp) and the Krylov solver (api_krylov.cpp)
rt_status check_state(rt_grid *g, const rt_state *s);
rt_status check_opts(const rt_solve_opts *o);
rt_status ensure_state_buffers(rt_grid *g);
rt_status solve_bicgstab(rt_grid *g, rt_state *s, const rt_solve_opts *o, rt_solve_report *rep, hipStream_t st);
