// sanitize_host.cpp -- drives the host-only parts of the rt3d library (box
// tracker and templates, work schedule, direction shards, spherical tracker
// and irradiation factor) under AddressSanitizer / UndefinedBehaviorSanitizer,
// built with g++ on the CPU.  Exits non-zero on a failed invariant; the
// sanitizers abort on any memory or undefined-behaviour error.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <numeric>
#include <vector>

#include "rt_internal.hpp"

using namespace rt3d;

static int g_fail = 0;
static long g_checks = 0;
#define CHECK(c)                                                            \
    do {                                                                    \
        ++g_checks;                                                         \
        if (!(c)) {                                                         \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            ++g_fail;                                                       \
        }                                                                   \
    } while (0)

static void box_case(int Nx, int Ny, int Nz, int n_mu, int n_phi)
{
    BoxGeometry g;
    const std::string err = build_box_geometry(Nx, Ny, Nz, n_mu, n_phi, g);
    CHECK(err.empty());
    if (!err.empty()) return;
    CHECK((int)g.dirs.size() == n_mu * n_phi);
    for (const Direction &d : g.dirs) {
        // path lengths through the slab sum to Nz / |mu| (unit voxels)
        double sum = 0.0;
        for (int m = 0; m < d.M; ++m) sum += g.s[(size_t)(d.vbegin + m)];
        CHECK(std::fabs(sum - Nz / std::fabs(d.mu)) < 1e-9 * (Nz / std::fabs(d.mu)));
        CHECK(d.span >= 0 && d.span < 4 * (Nx + Ny + Nz) / std::fabs(d.mu) + 4);
    }
    // schedules: every (lambda, direction, bundle) item exactly once per bundle class
    for (int n_lambda : {1, 3, 7}) {
        std::vector<int32_t> lams(n_lambda);
        std::iota(lams.begin(), lams.end(), 0);
        for (int n_wg : {1, 4, 8, 13, 64}) {
            for (int nb : {1, 2, 4}) {
                if (n_wg % nb) continue;
                Schedule sc;
                build_schedule(g, lams, n_wg, sc, nullptr, nb);
                CHECK(sc.n_wg == n_wg);
                CHECK((int)sc.wg_begin.size() == n_wg + 1);
                std::vector<int> seen((size_t)nb * n_lambda * g.dirs.size(), 0);
                for (int w = 0; w < sc.n_wg; ++w)
                    for (int k = sc.wg_begin[w]; k < sc.wg_begin[w + 1]; ++k) {
                        const WorkItem &it = sc.items[(size_t)k];
                        CHECK(it.lambda >= 0 && it.lambda < n_lambda);
                        CHECK(it.dir >= 0 && it.dir < (int)g.dirs.size());
                        CHECK(it.slot >= 0 && it.slot < sc.n_slots);
                        ++seen[((size_t)(w % nb) * n_lambda + it.lambda) * g.dirs.size() + it.dir];
                    }
                for (int s : seen) CHECK(s == 1);
            }
        }
    }
    // a subset schedule and the direction shards
    std::vector<int32_t> sub;
    for (int d = 0; d < (int)g.dirs.size(); d += 3) sub.push_back(d);
    Schedule sc;
    build_schedule(g, {0}, 8, sc, &sub, 1);
    CHECK((int)sc.items.size() == (int)sub.size());
    std::vector<int> count(g.dirs.size(), 0);
    for (int s = 0; s < 3; ++s)
        for (int d : shard_directions(g, 3, s)) ++count[(size_t)d];
    for (int c : count) CHECK(c == 1);
}

static void sphere_case(int Nr, int Nt, int Np, double rc, double ro, double dsrc, int n_mu, int n_phi)
{
    SphereSpec sp;
    sp.Nr = Nr; sp.Nt = Nt; sp.Np = Np; sp.rc = rc; sp.ro = ro; sp.dsrc = dsrc; sp.n_mu = n_mu; sp.n_phi = n_phi;
    CHECK(check_sphere_spec(sp).empty());
    const double h = sphere_spacing(sp);
    CHECK(h > 0.0 && h < ro);
    std::vector<Direction> dirs;
    for (int i = 0; i < n_mu; ++i)
        for (int j = 0; j < n_phi; ++j) dirs.push_back(quadrature_direction(i, j, n_mu, n_phi));
    const int64_t n_vox = (int64_t)Nr * Nt * Np;
    for (int d = 0; d < (int)dirs.size(); ++d) {
        SphereTracks tr;
        trace_sphere_direction(sp, h, dirs[d].n, tr);
        const size_t nc = tr.kind.size();
        CHECK(tr.begin.size() == nc + 1);
        CHECK(tr.p.size() == 3 * nc && tr.ta.size() == nc && tr.tb.size() == nc);
        CHECK(tr.vox.size() == tr.s.size() && (int64_t)tr.vox.size() == tr.begin[nc]);
        std::vector<char> hit((size_t)n_vox, 0);
        for (size_t c = 0; c < nc; ++c) {
            double len = 0.0;
            for (int64_t i = tr.begin[c]; i < tr.begin[c + 1]; ++i) {
                CHECK(tr.vox[(size_t)i] >= 0 && tr.vox[(size_t)i] < n_vox);
                CHECK(tr.s[(size_t)i] > 0.0);
                len += tr.s[(size_t)i];
                hit[(size_t)tr.vox[(size_t)i]] = 1;
            }
            CHECK(std::fabs(len - (tr.tb[c] - tr.ta[c])) < 1e-9 * (1.0 + ro));
            if (tr.kind[c] == 0) {
                const double x[3] = {tr.p[3 * c] + tr.ta[c] * dirs[d].n[0], tr.p[3 * c + 1] + tr.ta[c] * dirs[d].n[1],
                                     tr.p[3 * c + 2] + tr.ta[c] * dirs[d].n[2]};
                CHECK(sphere_irradiation(sp, dirs, d, x) >= 0.0);
            }
        }
        // every voxel is crossed by some characteristic of every direction
        for (char v : hit) CHECK(v == 1);
    }
}

int main()
{
    box_case(1, 1, 1, 2, 1);
    box_case(7, 5, 6, 4, 8);
    box_case(9, 9, 1, 2, 4);
    box_case(17, 13, 9, 4, 8);
    box_case(33, 33, 12, 8, 16);
    BoxGeometry bad;
    CHECK(!build_box_geometry(0, 4, 4, 2, 1, bad).empty());
    CHECK(!build_box_geometry(4, 4, 4, 3, 1, bad).empty());
    CHECK(!build_box_geometry(40000, 4, 4, 2, 1, bad).empty());
    sphere_case(6, 5, 8, 1.0, 3.0, 0.0, 4, 4);
    sphere_case(5, 4, 6, 0.5, 2.0, 4.0, 2, 4);
    SphereSpec sp;
    CHECK(!check_sphere_spec(sp).empty());
    if (g_fail) {
        std::fprintf(stderr, "%d checks failed\n", g_fail);
        return 1;
    }
    std::printf("%ld host checks passed\n", g_checks);
    return 0;
}
