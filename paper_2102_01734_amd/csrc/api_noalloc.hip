// api_noalloc.hip -- rt_formal_solution_noalloc: the box formal solution with
// every scratch buffer (work schedule, padded (chi, S) input, partial sums) in
// one fixed device array, for callers that cannot allocate device memory.
//
// The array below is a file-scope device variable: each GPU the library runs
// on holds its own copy until the process ends.  Host code never names it
// except to look up its device address (hipGetSymbolAddress, once per device,
// at grid creation); kernels and copies only ever see that address.
#include <mutex>

#include "rt_host.hpp"

static constexpr size_t kNoAllocScratchBytes = size_t(RT_NOALLOC_SCRATCH_BYTES);

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mu;
static std::map<int, void *> g_scratch_ptr;  // device -> that device's copy of scratch

static size_t align256(size_t n) { return (n + 255) / 256 * 256; }

rt_status noalloc_scratch_setup(int device, void **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it == g_scratch_ptr.end()) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return fail(RT_E_HIP, "scratch lookup on device %d: %s", device, hipGetErrorString(e));
        it = g_scratch_ptr.emplace(device, p).first;
    }
    *out = it->second;
    return RT_OK;
}

namespace {

// One sweep of the no-allocation path: its launch shape, schedule (host copy,
// kept in the grid so that the asynchronous upload always reads live memory)
// and where its arrays sit in the scratch.
struct NoAllocPass {
    const Variant *v = nullptr;
    const Schedule *sc = nullptr;
    size_t off_wg = 0, off_items = 0, off_sb = 0, off_si = 0, off_lo = 0, off_part = 0, end = 0;
};

size_t schedule_bytes(size_t n_wg, size_t n_items, size_t n_lambda, size_t n_slots)
{
    return align256((n_wg + 1) * 4) + align256(n_items * sizeof(WorkItem)) + align256((n_lambda + 1) * 4) +
           align256(n_slots * 4) + align256(n_lambda * 4);
}

// Fewest-constraint plan: the largest workgroup count (at most the shape's
// resident count, a multiple of its bundle count) whose partial sums fit the
// scratch behind the padded input.
rt_status plan_pass(rt_grid *g, const Variant &v, int n_lambda, size_t base, int nout, NoAllocPass &p)
{
    const size_t esz = g->dbl ? 8 : 4;
    const size_t slot_bytes = (size_t)g->n_vox * esz * nout;
    const size_t n_items_max = (size_t)n_lambda * g->n_dir * v.nb;
    const int nb = v.nb;
    int n_wg = v.n_wg - v.n_wg % nb;
    auto need = [&](int w) {
        const size_t slots = (size_t)w + n_lambda;
        return base + schedule_bytes(w, n_items_max, n_lambda, slots) + slots * slot_bytes;
    };
    while (n_wg >= nb && need(n_wg) > kNoAllocScratchBytes) n_wg -= nb;
    if (n_wg < nb)
        return fail(RT_E_INVALID,
                    "formal solution of %d wavelengths on %lld voxels needs %zu bytes of scratch with a single "
                    "workgroup per ray bundle; the no-allocation scratch holds %zu",
                    n_lambda, (long long)g->n_vox, need(nb), kNoAllocScratchBytes);
    char key[96];
    snprintf(key, sizeof key, "%d/%d/%d/%d", n_wg, nb, v.band ? 1 : 0, n_lambda);
    auto it = g->na_sched.find(key);
    if (it == g->na_sched.end()) {
        auto sc = std::make_unique<Schedule>();
        std::vector<int32_t> lams(n_lambda);
        for (int i = 0; i < n_lambda; ++i) lams[i] = i;
        build_schedule(g->geo, lams, n_wg, *sc, nullptr, nb);
        it = g->na_sched.emplace(key, std::move(sc)).first;
    }
    p.v = &v;
    p.sc = it->second.get();
    const Schedule &s = *p.sc;
    p.off_wg = base;
    p.off_items = p.off_wg + align256((s.wg_begin.size()) * 4);
    p.off_sb = p.off_items + align256(s.items.size() * sizeof(WorkItem));
    p.off_si = p.off_sb + align256(s.slot_begin.size() * 4);
    p.off_lo = p.off_si + align256(s.slot_ids.size() * 4);
    p.off_part = p.off_lo + align256((size_t)n_lambda * 4);
    p.end = p.off_part + (size_t)s.n_slots * slot_bytes;
    if (p.end > kNoAllocScratchBytes)
        return fail(RT_E_INVALID, "formal solution needs %zu bytes of scratch; the no-allocation scratch holds %zu",
                    p.end, kNoAllocScratchBytes);
    return RT_OK;
}

}  // namespace

extern "C" rt_status rt_formal_solution_noalloc(rt_grid_t g, int32_t n_lambda, const void *chi, const void *S,
                                                const void *I_bc, void *J_out, void *lstar_out, void *stream)
{
    if (!g) return fail(RT_E_INVALID, "grid is NULL");
    if (g->sphere) return fail(RT_E_UNSUPPORTED, "the no-allocation formal solution serves box grids");
    if (n_lambda < 0 || n_lambda > g->desc.n_lambda_max)
        return fail(RT_E_INVALID, "n_lambda %d outside [0, %d]", n_lambda, g->desc.n_lambda_max);
    if (n_lambda == 0) return RT_OK;
    if (!chi || !S || !J_out) return fail(RT_E_INVALID, "chi, S and J_out must not be NULL");
    if (!g->na_scratch) return fail(RT_E_HIP, "no-allocation scratch not set up on device %d", g->device);
    hipStream_t st = (hipStream_t)stream;
    const bool dbl = g->dbl;
    const size_t esz = dbl ? 8 : 4;
    char *base = static_cast<char *>(g->na_scratch);
    // the padded (chi, S) input of all wavelengths, then the schedule and partial sums of one sweep
    const size_t fld_bytes = align256((size_t)8 * n_lambda * g->n_vox * esz);
    if (fld_bytes > kNoAllocScratchBytes)
        return fail(RT_E_INVALID, "padded input of %d wavelengths (%zu bytes) exceeds the no-allocation scratch (%zu)",
                    n_lambda, fld_bytes, kNoAllocScratchBytes);
    const bool wl = lstar_out != nullptr;
    const bool joint = wl && variant(g, dbl, true, true).ok;
    struct Out { bool wj, wl; };
    std::vector<Out> outs;
    if (joint) outs.push_back({true, true});
    else {
        if (wl) outs.push_back({false, true});
        outs.push_back({true, false});
    }
    // validate every sweep before anything is enqueued
    std::vector<NoAllocPass> passes(outs.size());
    for (size_t i = 0; i < outs.size(); ++i) {
        const Variant &v = variant(g, dbl, outs[i].wj, outs[i].wl);
        if (!v.ok) return fail(RT_E_UNSUPPORTED, "no kernel configuration fits this grid");
        rt_status rs = plan_pass(g, v, n_lambda, fld_bytes, (outs[i].wj ? 1 : 0) + (outs[i].wl ? 1 : 0), passes[i]);
        if (rs != RT_OK) return rs;
    }
    const int Nx = g->lx, Ny = g->ly, Nz = g->lz;
    if (dbl) {
        HIPCHK(pad_field<double, double>((const double *)chi, nullptr, (double *)base, Nx, Ny, Nz, n_lambda, 0, st));
        HIPCHK(pad_field<double, double>((const double *)S, nullptr, (double *)base, Nx, Ny, Nz, n_lambda, 1, st));
    } else {
        HIPCHK(pad_field<float, float>((const float *)chi, nullptr, (float *)base, Nx, Ny, Nz, n_lambda, 0, st));
        HIPCHK(pad_field<float, float>((const float *)S, nullptr, (float *)base, Nx, Ny, Nz, n_lambda, 1, st));
    }
    for (size_t i = 0; i < passes.size(); ++i) {
        const NoAllocPass &p = passes[i];
        const Variant &v = *p.v;
        const Schedule &sc = *p.sc;
        // schedule into the scratch (host copies live in the grid until it is destroyed)
        HIPCHK(hipMemcpyAsync(base + p.off_wg, sc.wg_begin.data(), sc.wg_begin.size() * 4, hipMemcpyHostToDevice, st));
        if (!sc.items.empty())
            HIPCHK(hipMemcpyAsync(base + p.off_items, sc.items.data(), sc.items.size() * sizeof(WorkItem),
                                  hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(base + p.off_sb, sc.slot_begin.data(), sc.slot_begin.size() * 4, hipMemcpyHostToDevice,
                              st));
        if (!sc.slot_ids.empty())
            HIPCHK(hipMemcpyAsync(base + p.off_si, sc.slot_ids.data(), sc.slot_ids.size() * 4, hipMemcpyHostToDevice,
                                  st));
        HIPCHK(hipMemcpyAsync(base + p.off_lo, g->iota_lams.data(), (size_t)n_lambda * 4, hipMemcpyHostToDevice,
                              st));
        const size_t slot_elems = (size_t)sc.n_slots * g->n_vox;
        void *partJ = outs[i].wj ? base + p.off_part : nullptr;
        void *partL = outs[i].wl ? base + p.off_part + (outs[i].wj ? slot_elems * esz : 0) : nullptr;
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
        a.wg_begin = reinterpret_cast<const int32_t *>(base + p.off_wg);
        a.items = reinterpret_cast<const WorkItem *>(base + p.off_items);
        a.field = base;
        a.pad_stride = 4 * g->n_vox;
        a.I_bc = I_bc;
        a.partJ = partJ;
        a.partL = partL;
        a.n_bundles = v.nb;
        a.bundle_rays = v.Q;
        a.tile_words = v.tile_words;
        a.brow = g->brow.as<int32_t>();
        a.dir_span = g->span.as<int32_t>();
        if (sc.n_wg > 0)
            HIPCHK(fs_box_launch(a, dbl, outs[i].wj, outs[i].wl, g->para, v.band, v.lb, v.R, sc.n_wg, v.nthr, v.lds,
                                 st));
        const int32_t *sb = reinterpret_cast<const int32_t *>(base + p.off_sb);
        const int32_t *si = reinterpret_cast<const int32_t *>(base + p.off_si);
        const int32_t *lo = reinterpret_cast<const int32_t *>(base + p.off_lo);
        if (dbl) {
            if (partJ)
                HIPCHK(reduce_partials<double, double>((const double *)partJ, sb, si, lo, n_lambda, (double *)J_out,
                                                       g->n_vox, st));
            if (partL)
                HIPCHK(reduce_partials<double, double>((const double *)partL, sb, si, lo, n_lambda,
                                                       (double *)lstar_out, g->n_vox, st));
        } else {
            if (partJ)
                HIPCHK(reduce_partials<float, float>((const float *)partJ, sb, si, lo, n_lambda, (float *)J_out,
                                                     g->n_vox, st));
            if (partL)
                HIPCHK(reduce_partials<float, float>((const float *)partL, sb, si, lo, n_lambda, (float *)lstar_out,
                                                     g->n_vox, st));
        }
    }
    return RT_OK;
}
