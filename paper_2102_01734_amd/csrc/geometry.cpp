// geometry.cpp -- angle quadrature and the box tracker (host, double).
//
// The tracker computes the geometric path of every characteristic once; the
// result is reused for every wavelength and every iteration (Sec. 4.1 of the
// paper: geometry cache built once, accessed by all later formal solutions).
// On the periodic box every characteristic of a direction is an integer
// translate of the one entering through the centre of the inflow face of
// column (0,0), so a single template per direction is the whole cache.
//
// Traversal: a 3D digital differential analyser.  From the entry point the
// ray advances to the nearest of the next x-, y- and z-plane crossings,
// whose parameters are (i + 1/2)/|n_x|, (j + 1/2)/|n_y| and k/|n_z| (each a
// single correctly rounded division).  A crossing that follows the previous
// recorded one by at most 1e-12 (t + 1) closes no segment: the voxel index
// steps but no zero-length piece is stored.  The ray ends at the far face.
#include <algorithm>
#include <cmath>
#include <limits>

#include "rt_internal.hpp"

namespace rt3d {

static constexpr double kTie = 1e-12;

int trace_box_ray(int Nz, const double n[3], std::vector<int32_t> &di, std::vector<int32_t> &dj,
                  std::vector<int32_t> &kk, std::vector<double> &s)
{
    di.clear(); dj.clear(); kk.clear(); s.clear();
    const double ax = std::fabs(n[0]), ay = std::fabs(n[1]), az = std::fabs(n[2]);
    if (!(az > 0.0) || Nz <= 0) return -1;
    const int sx = n[0] >= 0.0 ? 1 : -1, sy = n[1] >= 0.0 ? 1 : -1;
    const bool down = n[2] < 0.0;
    const double inf = std::numeric_limits<double>::infinity();
    long cx = 0, cy = 0;      // crossings taken in x and y
    int cz = 1;               // index of the next z plane (1..Nz, Nz = exit)
    int ix = 0, iy = 0, depth = 0;
    double prev = 0.0;
    for (;;) {
        const double tx = ax > 0.0 ? (cx + 0.5) / ax : inf;
        const double ty = ay > 0.0 ? (cy + 0.5) / ay : inf;
        const double tz = cz / az;
        double t = tx < ty ? tx : ty;
        if (tz < t) t = tz;
        if (t - prev > kTie * (prev + 1.0)) {
            di.push_back(ix);
            dj.push_back(iy);
            kk.push_back(down ? depth : Nz - 1 - depth);
            s.push_back(t - prev);
            prev = t;
        }
        bool exit_now = false;
        if (tx == t) { ++cx; ix += sx; }
        if (ty == t) { ++cy; iy += sy; }
        if (tz == t) {
            if (cz == Nz) exit_now = true;
            else { ++cz; ++depth; }
        }
        if (exit_now) break;
    }
    return (int)s.size();
}

Direction quadrature_direction(int i, int j, int n_mu, int n_phi)
{
    Direction d;
    d.mu = -1.0 + (2.0 * i + 1.0) / n_mu;
    d.phi = 2.0 * M_PI * (j + 0.5) / n_phi;
    d.w = 1.0 / ((double)n_mu * (double)n_phi);
    const double st = std::sqrt(1.0 - d.mu * d.mu);
    d.n[0] = st * std::cos(d.phi);
    d.n[1] = st * std::sin(d.phi);
    d.n[2] = d.mu;
    return d;
}

std::string build_box_geometry(int Nx, int Ny, int Nz, int n_mu, int n_phi, BoxGeometry &g)
{
    if (Nx < 1 || Ny < 1 || Nz < 1) return "grid sizes must be >= 1";
    if (Nx >= kMaxSide || Ny >= kMaxSide) return "Nx and Ny must be < 32768";
    if (n_mu < 2 || (n_mu % 2) != 0) return "n_mu must be even and >= 2 (mu = 0 is never a direction)";
    if (n_phi < 1) return "n_phi must be >= 1";
    g = BoxGeometry();
    g.Nx = Nx; g.Ny = Ny; g.Nz = Nz; g.n_mu = n_mu; g.n_phi = n_phi;
    const int ndir = n_mu * n_phi;
    g.dirs.resize(ndir);
    std::vector<int32_t> di, dj, kk;
    std::vector<double> s;
    const int64_t plane = 4LL * Nx * Ny;       // padded layer: 2Ny rows of 2Nx
    for (int i = 0; i < n_mu; ++i) {
        for (int j = 0; j < n_phi; ++j) {
            Direction &d = g.dirs[i * n_phi + j];
            d = quadrature_direction(i, j, n_mu, n_phi);
            int M = trace_box_ray(Nz, d.n, di, dj, kk, s);
            if (M <= 0) return "tracker failed";
            // the sweep kernel advances its layer counter at every layer end:
            // layers must be contiguous, monotone in the direction of travel,
            // and all Nz of them must be visited
            int ends = 0;
            for (int m = 0; m < M; ++m) {
                if (m + 1 < M && kk[m + 1] != kk[m] && kk[m + 1] != kk[m] + (d.mu < 0.0 ? 1 : -1))
                    return "tracker produced a non-contiguous layer sequence";
                if (m == M - 1 || kk[m + 1] != kk[m]) ++ends;
            }
            if (ends != Nz || kk[0] != (d.mu < 0.0 ? 0 : Nz - 1))
                return "tracker did not visit every layer once";
            d.vbegin = (int64_t)g.s.size();
            d.M = M;
            // row of each visit relative to the lowest row the template reaches in
            // the same layer (the layer-band tiles of the sweep index by it)
            std::vector<int32_t> rel((size_t)M);
            d.span = 0;
            for (int m0 = 0; m0 < M;) {
                int m1 = m0;
                int jlo = dj[m0], jhi = dj[m0];
                while (m1 + 1 < M && kk[m1 + 1] == kk[m0]) {
                    ++m1;
                    jlo = std::min(jlo, dj[m1]);
                    jhi = std::max(jhi, dj[m1]);
                }
                for (int m = m0; m <= m1; ++m) rel[(size_t)m] = dj[m] - jlo;
                d.span = std::max(d.span, jhi - jlo);
                m0 = m1 + 1;
            }
            for (int m = 0; m < M; ++m) {
                int a = di[m] % Nx; if (a < 0) a += Nx;
                int b = dj[m] % Ny; if (b < 0) b += Ny;
                int64_t off = kk[m] * plane + (int64_t)b * (2 * Nx) + a;
                if (off > 0x7fffffffLL) return "grid too large for 32-bit visit offsets";
                uint32_t w = (uint32_t)a | ((uint32_t)b << kOffBits);
                if (m == M - 1 || kk[m + 1] != kk[m]) w |= kLayerEnd;
                g.goff.push_back((int32_t)off);
                g.dxy.push_back(w);
                g.s.push_back(s[m]);
                g.brow.push_back(rel[(size_t)m]);
                uint32_t packed = 0;
                for (int j = -1; j <= 3; ++j) {
                    const int u = m - j;
                    uint32_t c = kNoComp;
                    if (u >= 0 && u < M) {
                        const int dx = di[u] - di[m], dy = dj[u] - dj[m], dz = kk[u] - kk[m];
                        if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1)
                            c = (uint32_t)((dz + 1) * 9 + (dy + 1) * 3 + (dx + 1));
                    }
                    packed |= c << (6 * (j + 1));
                }
                g.comp.push_back(packed);
                g.di.push_back(di[m]);
                g.dj.push_back(dj[m]);
                g.kk.push_back(kk[m]);
            }
        }
    }
    return std::string();
}

}  // namespace rt3d
