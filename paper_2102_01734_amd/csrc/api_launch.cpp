// api_launch.cpp -- launch shapes of the box sweep (variants, autotuner),
// persistent-workgroup schedules, the formal-solution launch sequence (box and
// sphere) and the kernel-timing hooks.
#include "rt_host.hpp"

using namespace rt3d;

ChunkPtrs chunk_ptrs(const SphereChunkDev &ch, const void *stage)
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
// Resident-workgroup count and LDS size of one launch shape; ok = false when
// the shape cannot hold all rays of a bundle or its tiles do not fit.
Variant make_variant(rt_grid *g, bool dbl, bool wj, bool wl, int lb, int R, int occ, bool band, bool allow_spill)
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
            // single-precision band tiles of single-output sweeps are two layer
            // rows wide (no column wrap)
            const int tw = (H + span + 1) * Nx * (dbl || nout > 1 ? 1 : 2);
            if ((size_t)(tw + nthr) * esz * nout * (size_t)occ > g->max_lds) continue;
            v.nb = nb; v.Q = (int)Q; v.nthr = nthr; v.tile_words = tw;
            found = true;
        }
        if (!found) return v;
    }
    v.lds = (size_t)(v.tile_words + v.nthr) * esz * nout;
    if (v.lds > g->max_lds) return v;
    int res = fs_box_occupancy(dbl, wj, wl, g->para, band, lb, R, v.nthr, v.lds);
    if (res < 0) {
        // the kernel keeps part of its state in scratch memory: only when asked
        if (!allow_spill) return v;
        res = -res;
        v.spill = true;
    }
    if (res <= 0) return v;
    v.n_wg = res * g->n_cu;
    v.n_wg -= v.n_wg % v.nb;  // equal classes of workgroups per bundle
    if (v.n_wg < v.nb) return v;
    v.ok = true;
    return v;
}

// Default shape among those compiled for every output combination: shapes
// whose kernels keep everything in registers first (any that spill only if
// none fits).  Layer tiles: the widest workgroups, then the fewest rays per
// thread.  Band tiles: the fewest bundles (widest bands, least flush traffic
// per ray), then the widest workgroups, then the fewest rays per thread.
void setup_variant(rt_grid *g, bool dbl, bool wj, bool wl)
{
    const FsShape *sh = nullptr;
    const int n = fs_box_shapes(&sh);
    Variant &best = variant(g, dbl, wj, wl);
    best = Variant();
    for (int pass = 0; pass < 2 && !best.ok; ++pass) {
        for (int i = 0; i < n; ++i) {
            if (!sh[i].full || sh[i].band != g->band) continue;
            Variant v = make_variant(g, dbl, wj, wl, sh[i].lb, sh[i].R, sh[i].occ, sh[i].band, pass == 1);
            if (!v.ok) continue;
            bool better = !best.ok;
            if (!better && g->band && v.nb != best.nb) better = v.nb < best.nb;
            else if (!better && v.lb != best.lb) better = v.lb > best.lb;
            else if (!better) better = v.R < best.R;
            if (better) best = v;
        }
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
rt_status get_schedule(rt_grid *g, int n_wg, const std::vector<int32_t> &lambdas, DevSchedule **out,
                              const std::vector<int32_t> *subset, const Variant *v)
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

rt_status run_fs_with(rt_grid *g, const Variant &v, const std::vector<int32_t> &lambdas, const void *fld,
                             const void *I_bc, DevBuf &partJ, DevBuf &partL, DevSchedule **sched_out,
                             hipStream_t st, const std::vector<int32_t> *subset)
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
    } else if (g->cap_stamps) {
        // inside the capture of a profiled ALI step: wall-clock stamps around the sweep
        HIPCHK(wall_stamp(g->cap_stamps, st));
        HIPCHK(fs_box_launch(a, dbl, wj, wl, g->para, v.band, v.lb, v.R, sc->n_wg, v.nthr, v.lds, st));
        HIPCHK(wall_stamp(g->cap_stamps + 1, st));
        g->cap_points += sc->points;
        g->cap_stamps = nullptr;
    } else {
        HIPCHK(fs_box_launch(a, dbl, wj, wl, g->para, v.band, v.lb, v.R, sc->n_wg, v.nthr, v.lds, st));
    }
    *sched_out = sc;
    return RT_OK;
}

rt_status collect_graph_time(rt_grid *g, rt_grid::GraphStep &gs)
{
    if (!gs.pending) return RT_OK;
    gs.pending = false;
    unsigned long long ts[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(ts, gs.stamps->p, sizeof ts, hipMemcpyDeviceToHost, gs.stream));
    HIPCHK(hipStreamSynchronize(gs.stream));
    g->prof_graph_ms += (double)(ts[1] - ts[0]) / (double)g->wall_khz;
    g->prof_graph_launches++;
    g->prof_points += gs.points;
    return RT_OK;
}

rt_status run_fs(rt_grid *g, bool dbl, bool wj, bool wl, const std::vector<int32_t> &lambdas,
                        const void *fld, const void *I_bc, DevBuf &partJ, DevBuf &partL, DevSchedule **sched_out,
                        hipStream_t st, const std::vector<int32_t> *subset)
{
    return run_fs_with(g, variant(g, dbl, wj, wl), lambdas, fld, I_bc, partJ, partL, sched_out, st, subset);
}
extern "C" {
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
        // bundle reaches); layer tiles wherever they fit
        if (!g->layer_ok && !sh[i].band) continue;
        const Variant v = make_variant(g, dbl, true, false, sh[i].lb, sh[i].R, sh[i].occ, sh[i].band, false);
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
            if (!g->layer_ok && !sh[i].band) continue;
            const Variant v = make_variant(g, dbl, true, false, threads, rays, sh[i].occ, sh[i].band, true);
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
    for (auto &kv : g->graphs) {
        rt_status rs = collect_graph_time(g, kv.second);
        if (rs != RT_OK) return rs;
    }
    if (fs_ms) *fs_ms = ms + g->prof_graph_ms;
    if (fs_launches) *fs_launches = (int32_t)g->prof_events.size() + g->prof_graph_launches;
    if (fs_points) *fs_points = g->prof_points;
    g->prof_events.clear();
    g->prof_points = 0;
    g->prof_graph_ms = 0.0;
    g->prof_graph_launches = 0;
    return RT_OK;
}

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
rt_status formal_solution(rt_grid *g, int32_t n_lambda, const void *chi, const void *S, const void *I_bc,
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
