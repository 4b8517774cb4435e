// api_grid.cpp -- grid handles: descriptor validation, the box templates and the
// spherical geometry cache (traced on host threads, uploaded or kept in pinned
// host memory), grid facts, and the library's error text.
#include "rt_host.hpp"

using namespace rt3d;

static thread_local std::string g_err;

rt_status fail(rt_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

void clear_error() { g_err.clear(); }

rt_status hip_fail(hipError_t e, const char *file, int line)
{
    const rt_status st = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? RT_E_NOMEM : RT_E_HIP;
    return fail(st, "HIP error %s at %s:%d", hipGetErrorString(e), file, line);
}

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

// Device bytes a box grid uses at most for its geometry, the partial sums
// of a formal solution with J and Lambda* of n_lambda_max wavelengths (a
// schedule opens at most n_wg + n_lambda slots), both padded-input copies,
// the ALI state (Ng ring, double anchors and their sweep on FP32 grids) and
// the nearest-neighbour stencil.
static int64_t box_device_bytes(rt_grid *g)
{
    const int64_t nl = g->desc.n_lambda_max, nv = g->n_vox, nvis = g->n_visits, nd = g->n_dir;
    const int64_t esz = g->dbl ? 8 : 4;
    int64_t nwg = 0;
    for (int j = 0; j < 2; ++j)
        for (int l = 0; l < 2; ++l) nwg = std::max<int64_t>(nwg, variant(g, g->dbl, j, l).n_wg);
    int64_t b = nvis * (4 + 4 + 8 + 4 + 4) + nd * (8 + 4 + 8 + 8 + 4);
    b += 2 * (nwg + nl) * nv * esz;   // J and Lambda* slots
    b += 2 * 8 * nl * nv * esz;       // padded (chi, S) inputs: formal solution and ALI
    b += 4 * nl * nv * 8;             // Ng ring
    if (!g->dbl) {
        int64_t nwg64 = variant(g, true, true, false).n_wg;
        b += (nwg64 + nl) * nv * 8 + 8 * nl * nv * 8 + 2 * nl * nv * 8;  // anchor sweep, its input, S_a, J_a
    }
    if (g->nonlocal) b += 27 * nl * nv * (esz + 8) + 3 * nl * nv * 8;
    return b;
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
    if (desc->geom == RT_GEOM_SPHERICAL && (desc->flags & RT_F_BAND_TILES))
        return fail(RT_E_INVALID, "RT_F_BAND_TILES applies to box grids only");
    if (desc->geom == RT_GEOM_SPHERICAL && (desc->flags & RT_F_LSTAR_NONLOCAL) && desc->n[2] < 3)
        return fail(RT_E_INVALID, "RT_F_LSTAR_NONLOCAL on a spherical grid needs Nphi >= 3");
    if (desc->geom == RT_GEOM_SPHERICAL && (desc->flags & RT_F_LSTAR_NONLOCAL) && (desc->flags & RT_F_HOST_CACHE))
        return fail(RT_E_INVALID, "RT_F_LSTAR_NONLOCAL needs the geometry cache in device memory (no RT_F_HOST_CACHE)");
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
        g->nonlocal = (desc->flags & RT_F_LSTAR_NONLOCAL) != 0;
        rt_status rs = build_sphere_grid(g.get(), desc);
        if (rs != RT_OK) return rs;
        if (g->nonlocal && g->sph_streaming)
            return fail(RT_E_NOMEM, "RT_F_LSTAR_NONLOCAL needs the whole geometry cache in device memory");
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
        clear_error();
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
    {
        rt_status rs = noalloc_scratch_setup(g->device, &g->na_scratch);
        if (rs != RT_OK) return rs;
    }
    g->iota_lams.resize((size_t)desc->n_lambda_max);
    for (int i = 0; i < desc->n_lambda_max; ++i) g->iota_lams[(size_t)i] = i;

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

    // stencil components and LDS planes of the row-window Lambda* kernel
    std::vector<int32_t> planes((size_t)2 * g->n_dir * kPlaneStride, -1);
    g->nl_rows = true;
    for (int d = 0; d < g->n_dir; ++d) {
        const Direction &dir = g->geo.dirs[d];
        bool used[kStencil] = {};
        int step = 0;
        for (int m = 0; m < dir.M; ++m) {
            const size_t i = (size_t)(dir.vbegin + m);
            const uint32_t packed = g->geo.comp[i];
            for (int j = g->para ? 0 : 1; j < 5; ++j) {
                const uint32_t c = (packed >> (6 * j)) & 63u;
                if (c != kNoComp) used[c] = true;
            }
            if (g->geo.dxy[i] & kLayerEnd) {
                step = 0;
                continue;
            }
            const int db = g->geo.brow[i + 1] - g->geo.brow[i];
            if (db < -1 || db > 1 || (db != 0 && step != 0 && db != step)) g->nl_rows = false;
            if (db != 0) step = db;
        }
        for (int skip = 0; skip < 2; ++skip) {
            int32_t *tab = planes.data() + ((size_t)skip * g->n_dir + d) * kPlaneStride;
            int p = 0;
            for (int c = 0; c < kStencil; ++c) {
                if (!used[c] || (skip && c == kStencilCentre)) continue;
                tab[c] = p;
                tab[32 + p] = c;
                ++p;
            }
            g->nl_np[skip] = std::max(g->nl_np[skip], p);
        }
    }
    if (const char *e = std::getenv("RT3D_STENCIL_PER_CHARACTERISTIC"))
        if (e[0] == '1') g->nl_rows = false;

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
    auto spills = [&]() {
        for (int d = 0; d < 2; ++d)
            for (int j = 0; j < 2; ++j)
                for (int l = 0; l < 2; ++l) {
                    const Variant &v = variant(g.get(), d, j, l);
                    if ((j || l) && v.ok && v.spill) return true;
                }
        return false;
    };
    g->band = (desc->flags & RT_F_BAND_TILES) != 0;
    bool ok = setup_all();
    g->layer_ok = !g->band && ok;
    if (!g->band && (!ok || spills())) {
        // layer tiles that do not fit, or fit only with kernels that spill
        // registers: band tiles instead where they fit without spilling
        g->band = true;
        const bool ok_band = setup_all();
        if (ok_band && (!ok || !spills())) {
            ok = true;
        } else {
            g->band = false;
            ok = setup_all();
        }
    }
    if (!ok)
        return fail(RT_E_UNSUPPORTED,
                    "layer of %d x %d voxels (row span %d per layer) fits neither a layer tile nor a band tile in "
                    "%zu bytes of LDS",
                    g->geo.Nx, g->geo.Ny, g->span_max, g->max_lds);
    // refuse, before anything is allocated, a grid whose working set cannot fit
    const int64_t need = box_device_bytes(g.get());
    size_t free_b = 0, total_b = 0;
    HIPCHK(hipMemGetInfo(&free_b, &total_b));
    if (need > (int64_t)free_b)
        return fail(RT_E_NOMEM,
                    "grid needs about %.1f GB of device memory (geometry, partial sums, padded inputs and ALI state "
                    "for %d wavelengths); %.1f GB free",
                    need * 1e-9, desc->n_lambda_max, (double)free_b * 1e-9);

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
    HIPCHK(g->nl_planes.ensure(planes.size() * 4));
    HIPCHK(hipMemcpy(g->nl_planes.p, planes.data(), planes.size() * 4, hipMemcpyHostToDevice));

    *out = g.release();
    clear_error();
    return RT_OK;
}

rt_status rt_destroy_grid(rt_grid_t grid)
{
    if (!grid) return fail(RT_E_INVALID, "grid is NULL");
    (void)hipDeviceSynchronize();
    delete grid;
    return RT_OK;
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
rt_status rt_grid_info(rt_grid_t g, int64_t *n_vox, int32_t *n_dir, int64_t *n_visits_total, int32_t *n_wg)
{
    if (!g) return fail(RT_E_INVALID, "grid is NULL");
    if (n_vox) *n_vox = g->n_vox;
    if (n_dir) *n_dir = g->n_dir;
    if (n_visits_total) *n_visits_total = g->n_visits;
    if (n_wg) *n_wg = g->sphere ? (int32_t)g->sph_chunks.size() : variant(g, g->dbl, true, false).n_wg;
    return RT_OK;
}
}  // extern "C"
