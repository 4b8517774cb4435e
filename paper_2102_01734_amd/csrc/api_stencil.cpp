// api_stencil.cpp -- the nearest-neighbour Lambda* (27-point stencil) of box
// grids: fixed-point accumulation and conversion.
#include "rt_host.hpp"

using namespace rt3d;

// Nearest-neighbour Lambda* of the batch from the caller's opacity, in two
// parts: clear the fixed-point sums and accumulate every characteristic
// (without the centre component when skip_centre), then convert into `out`
// ([lambda][27][vox], double or float), the centre taken from `centre` (the
// diagonal Lambda* of the same operator, [lambda][vox]) when given.
rt_status accumulate_stencil(rt_grid *g, const void *chi, int n_lambda, int nb, const int32_t *lambda_of,
                                    bool skip_centre, hipStream_t st)
{
    const int64_t per = (int64_t)kStencil * g->n_vox;
    HIPCHK(g->nl_acc.ensure((size_t)n_lambda * per * 8));
    for (int64_t off = 0; off < (int64_t)n_lambda * per; off += (int64_t)1 << 30) {
        const int64_t cnt = std::min<int64_t>((int64_t)1 << 30, (int64_t)n_lambda * per - off);
        HIPCHK(fill_u64(g->nl_acc.as<unsigned long long>() + off, 0ull, (int)cnt, st));
    }
    if (g->sphere) {
        for (const auto &chp : g->sph_chunks) {
            const SphereChunkDev &ch = *chp;
            if (ch.host)
                return fail(RT_E_UNSUPPORTED, "the nearest-neighbour Lambda* needs the geometry cache in device memory");
            const ChunkPtrs cp = chunk_ptrs(ch, nullptr);
            SphereStencilArgs a{};
            a.Nr = g->desc.n[0]; a.Nt = g->desc.n[1]; a.Np = g->desc.n[2];
            a.n_vox = g->n_vox;
            a.n_bundles = ch.n_bundles;
            a.bundle_begin = cp.bundle_begin;
            a.char_len = cp.char_len;
            a.vox = cp.vox;
            a.s = cp.s;
            a.w = cp.w;
            a.chi = chi;
            a.lambda_of = lambda_of;
            a.n_batch = nb;
            a.acc = g->nl_acc.as<unsigned long long>();
            a.skip_centre = skip_centre ? 1 : 0;
            HIPCHK(lstar_stencil_sphere_accumulate(a, g->dbl, g->sph_gdouble, g->para, st));
        }
        return RT_OK;
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
    if (g->nl_rows) {
        a.brow = g->brow.as<int32_t>();
        a.dir_plane = g->nl_planes.as<int32_t>() + (size_t)(skip_centre ? 1 : 0) * g->n_dir * kPlaneStride;
        a.planes = g->nl_np[skip_centre ? 1 : 0];
    }
    HIPCHK(lstar_stencil_accumulate(a, g->dbl, g->para, g->n_dir, nb, g->max_lds, st));
    return RT_OK;
}

rt_status finish_stencil(rt_grid *g, int nb, const int32_t *lambda_of, const void *centre, void *out,
                                bool out_double, hipStream_t st)
{
    HIPCHK(lstar_stencil_finish(g->nl_acc.as<unsigned long long>(), lambda_of, g->n_vox, nb, centre, out, out_double,
                                st));
    return RT_OK;
}

rt_status compute_stencil(rt_grid *g, const void *chi, int n_lambda, int nb, const int32_t *lambda_of,
                                 void *out, bool out_double, hipStream_t st)
{
    rt_status rs = accumulate_stencil(g, chi, n_lambda, nb, lambda_of, false, st);
    if (rs != RT_OK) return rs;
    return finish_stencil(g, nb, lambda_of, nullptr, out, out_double, st);
}
extern "C" {
rt_status rt_lstar_stencil(rt_grid_t g, int32_t n_lambda, const void *chi, void *out, void *stream)
{
    if (!g) return fail(RT_E_INVALID, "grid is NULL");
    if (n_lambda == 0) return RT_OK;
    if (n_lambda < 0 || n_lambda > g->desc.n_lambda_max)
        return fail(RT_E_INVALID, "n_lambda %d outside [0, %d]", n_lambda, g->desc.n_lambda_max);
    if (!chi || !out) return fail(RT_E_INVALID, "chi and out must not be NULL");
    if (g->sphere && g->desc.n[2] < 3)
        return fail(RT_E_INVALID, "the spherical nearest-neighbour Lambda* needs Nphi >= 3");
    std::vector<int32_t> lams(n_lambda);
    for (int i = 0; i < n_lambda; ++i) lams[i] = i;
    DevSchedule *sc = nullptr;
    rt_status rs = get_schedule(g, g->sphere ? 0 : variant(g, g->dbl, true, false).n_wg, lams, &sc);
    if (rs != RT_OK) return rs;
    return compute_stencil(g, chi, n_lambda, n_lambda, sc->lambda_of.as<int32_t>(), out, g->dbl,
                           (hipStream_t)stream);
}
}  // extern "C"
