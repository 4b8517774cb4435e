// sphere_geometry.cpp -- tracker of the spherical grid (host, double).
//
// Spherical voxels (Sec. 3.2 of the paper: r, theta, phi cells around an
// opaque core) are bounded by spheres, cones and half-planes.  Directions are
// global (fixed in the Cartesian frame), so each direction needs its own set
// of characteristics:
//   * a square lattice of foot points on the plane through the origin normal
//     to n, with axes e1 = normalise(z x n) (x if n is along z) and
//     e2 = n x e1, spacing h = median cube root of the voxel volumes, points
//     with |p| < ro;
//   * then, in voxel-index order, one characteristic through the centre of
//     every voxel that none has visited yet (small voxels near the poles and
//     the core).
// A line that meets the core gives two characteristics: inward, ending on
// the core, and outward, starting on it.  Along a line p + t n the crossings
// with all voxel boundaries are collected, sorted, and crossings closer than
// 1e-12 (|t| + 1) to the previous segment end are merged; each segment is
// assigned to the voxel containing its midpoint.
//
// The geometry is computed once per grid and reused by every wavelength and
// iteration (the geometry cache of Sec. 4.1).
#include <algorithm>
#include <cmath>

#include "rt_internal.hpp"

namespace rt3d {

static constexpr double kTie = 1e-12;

namespace {

// Boundary tables and the crossing / location primitives of one grid.
struct Shells {
    const SphereSpec &g;
    std::vector<double> r;        // r_i, i = 1..Nr-1
    std::vector<double> cth;      // cos(theta_k), k = 1..Nt-1
    std::vector<int> equator;     // 1 where 2k == Nt (the plane z = 0)
    std::vector<double> cph, sph; // cos, sin of phi_j, j = 0..Np-1

    explicit Shells(const SphereSpec &spec) : g(spec)
    {
        for (int i = 1; i < g.Nr; ++i) r.push_back(g.rc + i * (g.ro - g.rc) / g.Nr);
        for (int k = 1; k < g.Nt; ++k) {
            cth.push_back(std::cos(k * M_PI / g.Nt));
            equator.push_back(2 * k == g.Nt ? 1 : 0);
        }
        for (int j = 0; j < g.Np; ++j) {
            const double ph = 2.0 * M_PI * j / g.Np;
            cph.push_back(std::cos(ph));
            sph.push_back(std::sin(ph));
        }
    }

    // crossing parameters strictly inside (t0, t1)
    void crossings(const double p[3], const double n[3], double t0, double t1, std::vector<double> &tc) const
    {
        tc.clear();
        auto keep = [&](double t) {
            if (t > t0 && t < t1) tc.push_back(t);
        };
        const double pp = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
        for (double ri : r) {
            const double q = ri * ri - pp;
            if (q > 0.0) {
                const double w = std::sqrt(q);
                keep(-w);
                keep(w);
            }
        }
        for (size_t k = 0; k < cth.size(); ++k) {
            if (equator[k]) {
                if (n[2] != 0.0) keep(-p[2] / n[2]);
                continue;
            }
            // (p_z + t n_z)^2 = cos^2(theta) |p + t n|^2 with |n| = 1 and p.n = 0
            const double c = cth[k], c2 = c * c;
            const double A = n[2] * n[2] - c2, Bq = 2.0 * p[2] * n[2], C = p[2] * p[2] - c2 * pp;
            double t[2];
            int nt = 0;
            if (std::fabs(A) < 1e-300) {
                if (Bq != 0.0) t[nt++] = -C / Bq;
            } else {
                const double disc = Bq * Bq - 4.0 * A * C;
                if (disc >= 0.0) {
                    const double w = std::sqrt(disc);
                    t[nt++] = (-Bq - w) / (2.0 * A);
                    t[nt++] = (-Bq + w) / (2.0 * A);
                }
            }
            for (int i = 0; i < nt; ++i) {
                const double z = p[2] + t[i] * n[2];
                if ((z > 0.0) == (c > 0.0)) keep(t[i]);  // only the cone's own nappe
            }
        }
        for (size_t j = 0; j < cph.size(); ++j) {
            // plane through the z axis with normal (-sin phi, cos phi, 0)
            const double cs = cph[j], sn = sph[j];
            const double den = -sn * n[0] + cs * n[1];
            if (den == 0.0) continue;
            const double t = (sn * p[0] - cs * p[1]) / den;
            const double x = p[0] + t * n[0], y = p[1] + t * n[1];
            if (cs * x + sn * y > 0.0) keep(t);  // the half-plane, not its mirror image
        }
        std::sort(tc.begin(), tc.end());
    }

    int32_t locate(const double x[3]) const
    {
        const double rr = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        const double th = std::acos(std::fmax(-1.0, std::fmin(1.0, x[2] / rr)));
        double ph = std::atan2(x[1], x[0]);
        if (ph < 0.0) ph += 2.0 * M_PI;
        const int ir = std::clamp((int)std::floor((rr - g.rc) / (g.ro - g.rc) * g.Nr), 0, g.Nr - 1);
        const int it = std::clamp((int)std::floor(th / M_PI * g.Nt), 0, g.Nt - 1);
        const int ip = std::clamp((int)std::floor(ph / (2.0 * M_PI) * g.Np), 0, g.Np - 1);
        return (int32_t)((ip * g.Nt + it) * g.Nr + ir);
    }

    // segments of p + t n for t in [ta, tb], appended to out; returns their count
    int segments(const double p[3], const double n[3], double ta, double tb, std::vector<double> &tc,
                 SphereTracks &out) const
    {
        crossings(p, n, ta, tb, tc);
        double prev = ta;
        int cnt = 0;
        for (size_t i = 0; i <= tc.size(); ++i) {
            const double t = i < tc.size() ? tc[i] : tb;
            if (!(t - prev > kTie * (std::fabs(prev) + 1.0))) continue;
            const double tm = 0.5 * (prev + t);
            const double x[3] = {p[0] + tm * n[0], p[1] + tm * n[1], p[2] + tm * n[2]};
            out.vox.push_back(locate(x));
            out.s.push_back(t - prev);
            prev = t;
            ++cnt;
        }
        return cnt;
    }
};

}  // namespace

std::string check_sphere_spec(const SphereSpec &g)
{
    if (g.Nr < 1 || g.Nt < 1 || g.Np < 1) return "spherical grid sizes must be >= 1";
    if ((int64_t)g.Nr * g.Nt * g.Np > ((int64_t)1 << 30)) return "spherical grid too large";
    if (!(g.rc > 0.0) || !(g.ro > g.rc) || !std::isfinite(g.ro)) return "need 0 < r_core < r_out";
    if (!(g.dsrc == 0.0 || (g.dsrc > 1.0 && std::isfinite(g.dsrc))))
        return "source distance (in units of r_out) must be 0 (none) or > 1";
    if (g.n_mu < 2 || (g.n_mu % 2) != 0) return "n_mu must be even and >= 2";
    if (g.n_phi < 1) return "n_phi must be >= 1";
    return "";
}

double sphere_spacing(const SphereSpec &g)
{
    std::vector<double> v;
    v.reserve((size_t)g.Nr * g.Nt);
    for (int it = 0; it < g.Nt; ++it)
        for (int ir = 0; ir < g.Nr; ++ir) {
            const double r0 = g.rc + ir * (g.ro - g.rc) / g.Nr, r1 = g.rc + (ir + 1) * (g.ro - g.rc) / g.Nr;
            const double c0 = std::cos(it * M_PI / g.Nt), c1 = std::cos((it + 1) * M_PI / g.Nt);
            v.push_back(std::cbrt((r1 * r1 * r1 - r0 * r0 * r0) / 3.0 * (c0 - c1) * (2.0 * M_PI / g.Np)));
        }
    std::sort(v.begin(), v.end());
    const size_t n = v.size();
    return (n % 2) ? v[n / 2] : 0.5 * (v[n / 2 - 1] + v[n / 2]);
}

void trace_sphere_direction(const SphereSpec &g, double h, const double n[3], SphereTracks &out)
{
    out = SphereTracks();
    out.begin.push_back(0);
    const Shells sh(g);
    const int64_t nvox = (int64_t)g.Nr * g.Nt * g.Np;
    std::vector<uint8_t> seen((size_t)nvox, 0);
    std::vector<double> tc;
    tc.reserve(2 * (g.Nr + g.Nt + g.Np) + 8);

    // frame of the foot-point plane
    double e1[3] = {-n[1], n[0], 0.0};
    double l = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1]);
    if (l < 1e-12) { e1[0] = 1.0; e1[1] = 0.0; l = 1.0; }
    e1[0] /= l; e1[1] /= l;
    const double e2[3] = {n[1] * e1[2] - n[2] * e1[1], n[2] * e1[0] - n[0] * e1[2], n[0] * e1[1] - n[1] * e1[0]};

    auto line = [&](const double p[3]) {
        const double pp = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
        if (!(pp < g.ro * g.ro)) return;
        const double to = std::sqrt(g.ro * g.ro - pp);
        double ta[2], tb[2];
        int8_t kind[2];
        int k = 0;
        if (pp < g.rc * g.rc) {
            const double ti = std::sqrt(g.rc * g.rc - pp);
            ta[k] = -to; tb[k] = -ti; kind[k++] = 0;
            ta[k] = ti; tb[k] = to; kind[k++] = 1;
        } else {
            ta[k] = -to; tb[k] = to; kind[k++] = 0;
        }
        for (int c = 0; c < k; ++c) {
            const size_t v0 = out.vox.size();
            const int M = sh.segments(p, n, ta[c], tb[c], tc, out);
            if (M <= 0) continue;
            for (size_t m = v0; m < out.vox.size(); ++m) seen[(size_t)out.vox[m]] = 1;
            out.begin.push_back((int64_t)out.vox.size());
            out.p.insert(out.p.end(), {p[0], p[1], p[2]});
            out.ta.push_back(ta[c]);
            out.tb.push_back(tb[c]);
            out.kind.push_back(kind[c]);
        }
    };

    const int K = (int)std::ceil(g.ro / h) + 1;
    for (int a = -K; a <= K; ++a)
        for (int b = -K; b <= K; ++b) {
            double p[3];
            for (int q = 0; q < 3; ++q) p[q] = a * h * e1[q] + b * h * e2[q];
            line(p);
        }
    for (int64_t v = 0; v < nvox; ++v) {
        if (seen[(size_t)v]) continue;
        const int ir = (int)(v % g.Nr), it = (int)((v / g.Nr) % g.Nt), ip = (int)(v / ((int64_t)g.Nr * g.Nt));
        const double r = g.rc + (ir + 0.5) * (g.ro - g.rc) / g.Nr;
        const double th = (it + 0.5) * M_PI / g.Nt, ph = (ip + 0.5) * 2.0 * M_PI / g.Np;
        const double c[3] = {r * std::sin(th) * std::cos(ph), r * std::sin(th) * std::sin(ph), r * std::cos(th)};
        const double cn = c[0] * n[0] + c[1] * n[1] + c[2] * n[2];
        const double p[3] = {c[0] - cn * n[0], c[1] - cn * n[1], c[2] - cn * n[2]};
        line(p);
    }
}

double sphere_irradiation(const SphereSpec &g, const std::vector<Direction> &dirs, int d, const double x[3])
{
    if (!(g.dsrc > 1.0)) return 0.0;
    const double zs = g.dsrc * g.ro;
    double u[3] = {x[0], x[1], x[2] - zs};
    const double L = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    for (double &c : u) c /= L;
    if (u[0] * x[0] + u[1] * x[1] + u[2] * x[2] >= 0.0) return 0.0;  // the source is below the horizon
    // is d the closest quadrature direction (ties to the lower index)?
    auto dot = [&](int q) { return dirs[q].n[0] * u[0] + dirs[q].n[1] * u[1] + dirs[q].n[2] * u[2]; };
    const double dd = dot(d);
    for (int q = 0; q < (int)dirs.size(); ++q) {
        if (q == d) continue;
        const double o = dot(q);
        if (o > dd || (o == dd && q < d)) return 0.0;
    }
    const double a = g.ro * (g.dsrc - 1.0);
    return a * a / (L * L) / dirs[d].w;
}

}  // namespace rt3d
