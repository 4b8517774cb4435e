// api_ali.cpp -- the operator-splitting (ALI) iteration: state checks, per-state
// buffers, the plain step (eager or as a captured HIP graph), Ng, anchors,
// the non-local OS update, learned proposals and the solve loop.
#include "rt_host.hpp"

using namespace rt3d;

// ---------------------------------------------------------------------------
// ALI
// ---------------------------------------------------------------------------
rt_status check_state(rt_grid *g, const rt_state *s)
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

rt_status check_opts(const rt_solve_opts *o)
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
    if (o->os_method != RT_OS_JACOBI && o->os_method != RT_OS_GAUSS_SEIDEL)
        return fail(RT_E_INVALID, "unknown operator-splitting method %d", o->os_method);
    return RT_OK;
}

// Allocates the per-state buffers (sized for n_lambda_max) once.
rt_status ensure_state_buffers(rt_grid *g)
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
// The operator-splitting update.  Diagonal Lambda*: the fused pointwise
// kernel.  Nearest-neighbour Lambda*: J_fs - J_old, `sweeps` Jacobi (or, when
// the step's options ask for it, colour Gauss-Seidel) sweeps of
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
    if (g->sphere) {  // x = r, y = theta (bounded), z = phi (periodic)
        ja.Nx = g->desc.n[0]; ja.Ny = g->desc.n[1]; ja.Nz = g->desc.n[2];
        ja.per[0] = 0; ja.per[1] = 0; ja.per[2] = 1;
    } else {          // x, y periodic, z bounded
        ja.Nx = g->geo.Nx; ja.Ny = g->geo.Ny; ja.Nz = g->geo.Nz;
        ja.per[0] = 1; ja.per[1] = 1; ja.per[2] = 0;
    }
    ja.n_vox = g->n_vox;
    ja.lambda_of = ua.lambda_of;
    ja.st = g->nl_st.p;
    ja.eps = ua.eps;
    ja.r = g->os_r.as<double>();
    double *x[2] = {g->os_x0.as<double>(), g->os_x1.as<double>()};
    ja.x_in = nullptr;
    ja.x_out = x[0];
    HIPCHK(os_jacobi_sweep(ja, g->dbl, true, nb, st));
    if (g->os_gs) {
        for (int k = 0; k < sweeps; ++k) HIPCHK(os_gs_sweep(ja, g->dbl, nb, st));
    } else {
        for (int k = 0; k < sweeps; ++k) {
            ja.x_in = x[k % 2];
            ja.x_out = x[(k + 1) % 2];
            HIPCHK(os_jacobi_sweep(ja, g->dbl, false, nb, st));
        }
    }
    ua.rfs_in = g->os_r.as<double>();
    ua.dJ = g->os_gs ? x[0] : x[sweeps % 2];
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
             g->net ? g->net_r.p : nullptr, g->resid.p, s->n_lambda, v.lb, v.R,
             g->nonlocal ? (g->os_gs ? 1000000 + sweeps : sweeps) : -1);
    std::string key(buf);
    for (int l : lams) key += std::to_string(l) + ",";
    const bool prof = g->prof;
    if (prof) key += "|timed";
    auto it = g->graphs.find(key);
    if (it == g->graphs.end()) {
        if (g->graphs.size() > 32) g->drop_graphs();
        rt_grid::GraphStep gs;
        gs.stream = st;
        if (prof) {  // wall-clock stamps around the sweep (see run_fs_with)
            if (!g->wall_khz) HIPCHK(hipDeviceGetAttribute(&g->wall_khz, hipDeviceAttributeWallClockRate, g->device));
            if (g->wall_khz <= 0) return fail(RT_E_HIP, "device reports no wall-clock rate");
            gs.stamps = std::make_shared<DevBuf>();
            HIPCHK(gs.stamps->ensure(2 * sizeof(unsigned long long)));
            g->cap_stamps = gs.stamps->as<unsigned long long>();
            g->cap_points = 0;
        }
        g->prof = false;
        hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) rs = plain_step_launches(g, s, lams, lambda_of, st, sweeps);
        hipGraph_t graph = nullptr;
        if (e == hipSuccess) e = hipStreamEndCapture(st, &graph);
        g->prof = prof;
        gs.points = g->cap_points;
        g->cap_stamps = nullptr;
        hipGraphExec_t exec = nullptr;
        if (e == hipSuccess && rs == RT_OK) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (rs != RT_OK) return rs;
        HIPCHK(e);
        gs.exec = exec;
        it = g->graphs.emplace(key, gs).first;
    } else {
        rs = collect_graph_time(g, it->second);  // the previous replay's sweep time
        if (rs != RT_OK) return rs;
    }
    HIPCHK(hipGraphLaunch(it->second.exec, st));
    if (it->second.stamps) it->second.pending = true;
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
    g->os_gs = o->os_method == RT_OS_GAUSS_SEIDEL;
    DevSchedule *lam_sc = nullptr;  // for lambda_of of the batch
    rs = get_schedule(g, variant(g, g->dbl, true, false).n_wg, lams, &lam_sc);
    if (rs != RT_OK) return rs;
    const int32_t *lambda_of = lam_sc->lambda_of.as<int32_t>();

    // The grid's per-state scratch (padded inputs, Ng history, double
    // anchor, nearest-neighbour stencil) belongs to the state stepped last;
    // a different state starts all of it afresh from its own arrays.
    const bool switched = !g->owned_by(s);
    if (switched) {
        g->take_ownership(s);
        g->hist_count = 0;
    }
    // (re)initialisation: padded opacity, S from J, fresh Ng history
    if (s->iter == 0 || switched || s->chi != g->chi_src) {
        if (g->dbl) {
            HIPCHK(pad_field<double, double>((const double *)s->chi, nullptr, g->fld.as<double>(), Nx, Ny, Nz, nl, 0, st));
        } else {
            HIPCHK(pad_field<float, float>((const float *)s->chi, nullptr, g->fld.as<float>(), Nx, Ny, Nz, nl, 0, st));
            HIPCHK(pad_field<float, double>((const float *)s->chi, nullptr, g->fld64.as<double>(), Nx, Ny, Nz, nl, 0, st));
        }
        g->chi_src = s->chi;
    }
    if (s->iter == 0 || switched) {
        g->hist_count = 0;
        if (g->dbl)
            HIPCHK(source_update<double, double>(s->J, (const double *)s->eps, (const double *)s->B, s->S, nullptr,
                                                 g->fld.as<double>(), Nx, Ny, nv, lambda_of, nb, st));
        anchor = true;
    }
    if (!g->dbl && !g->anchor_ok) anchor = true;
    const bool want_l = s->lstar_valid == 0;
    // A state whose Lambda* is already known (from BiCGStab, or set by the
    // caller) but whose stencil this grid has not built: build it here, in
    // full, before the step.
    if (g->nonlocal && !want_l && !g->nl_ok) {
        rs = accumulate_stencil(g, s->chi, nl, nb, lambda_of, false, st);
        if (rs != RT_OK) return rs;
        rs = finish_stencil(g, nb, lambda_of, nullptr, g->nl_st.p, g->dbl, st);
        if (rs != RT_OK) return rs;
        g->nl_ok = true;
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
        // box: the centre is the sweep's diagonal Lambda* (no other point of a
        // characteristic within the stencil window lies in the same voxel);
        // sphere: built here, since a characteristic can leave and re-enter a voxel
        rt_status r = accumulate_stencil(g, s->chi, nl, nb, lambda_of, !g->sphere, g->nl_side);
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
        return finish_stencil(g, nb, lambda_of, g->sphere ? nullptr : s->lstar, g->nl_st.p, g->dbl, st);
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
    if (g->nonlocal && want_l) g->nl_ok = true;
    if (anchor) g->anchor_ok = true;
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
    clear_error();
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
