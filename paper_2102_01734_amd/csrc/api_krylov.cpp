// api_krylov.cpp -- BiCGStab outer solver on the full system (rt_solve with
// RT_SOLVER_BICGSTAB).
#include "rt_host.hpp"

using namespace rt3d;

// BiCGStab on A S = b (A = 1 - diag(1-eps) Lambda, b = (1-eps) Lambda_bc + eps B),
// right-preconditioned by M = 1 - (1-eps) Lambda*; every formal solution in
// double precision (single-precision grids use their double anchor input).
rt_status solve_bicgstab(rt_grid *g, rt_state *s, const rt_solve_opts *o, rt_solve_report *rep, hipStream_t st)
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
    // BiCGStab uses the padded inputs as scratch: the next ALI step, of any
    // state, starts its per-state scratch afresh
    g->release_ownership();
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
    clear_error();
    return RT_OK;
}
