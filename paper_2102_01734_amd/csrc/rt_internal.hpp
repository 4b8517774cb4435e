// rt_internal.hpp -- internal types of the rt3d library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "rt3d.h"

namespace rt3d {

// Per-visit flags packed into the high bits of the horizontal offset word.
constexpr uint32_t kLayerEnd = 0x80000000u;
constexpr int kOffBits = 15;                    // di', dj' each < 2^15
constexpr uint32_t kOffMask = (1u << kOffBits) - 1u;
constexpr int kMaxSide = 1 << kOffBits;
// Per-visit stencil components of the nearest-neighbour Lambda*: 6 bits per
// point m+1, m, m-1, m-2, m-3 (component (dz+1)*9 + (dy+1)*3 + (dx+1) of
// that point's voxel seen from the voxel of point m), kNoComp if none.
constexpr uint32_t kNoComp = 63;

// One direction of the angle quadrature and its characteristic template.
struct Direction {
    double mu = 0, phi = 0, w = 0;
    double n[3] = {0, 0, 0};
    int64_t vbegin = 0;  // first visit of the template in the visit table
    int32_t M = 0;       // number of visits (segments) of every ray
    int32_t span = 0;    // largest row extent (max dj - min dj) of the template within one layer
};

// Characteristic templates of all directions (the geometry cache).  All rays
// of a direction are integer translates of its template, so one visit list
// per direction describes every characteristic of the box.
struct BoxGeometry {
    int Nx = 0, Ny = 0, Nz = 0, n_mu = 0, n_phi = 0;
    std::vector<Direction> dirs;
    // visit table, structure of arrays, directions back to back
    std::vector<int32_t> goff;   // offset in the doubly periodic padded field
    std::vector<uint32_t> dxy;   // di mod Nx | (dj mod Ny) << 15 | layer-end flag
    std::vector<double> s;       // path length inside the voxel
    std::vector<int32_t> brow;   // dj - (smallest dj of the visits in the same layer)
    std::vector<uint32_t> comp;  // stencil components of the points m+1 .. m-3 (kNoComp: none)
    std::vector<int32_t> di, dj, kk;  // unwrapped offsets and layer (tests, tools)
};

// Direction (i, j) of the midpoint quadrature: mu_i = -1 + (2i+1)/n_mu,
// phi_j = 2 pi (j + 1/2)/n_phi, equal weights 1/(n_mu n_phi).
Direction quadrature_direction(int i, int j, int n_mu, int n_phi);

// Builds directions and templates.  Returns an empty string on success.
std::string build_box_geometry(int Nx, int Ny, int Nz, int n_mu, int n_phi, BoxGeometry &g);

// Traces one characteristic from the centre of the inflow face of column
// (0,0); returns the number of segments or -1.
int trace_box_ray(int Nz, const double n[3], std::vector<int32_t> &di, std::vector<int32_t> &dj,
                  std::vector<int32_t> &kk, std::vector<double> &s);

// Work item of the formal-solution kernel: one wavelength and one direction,
// accumulated into partial-sum slot `slot`.
struct WorkItem {
    int32_t lambda, dir, slot, first;  // first != 0: first item of its slot
};

struct Schedule {
    int n_wg = 0;
    std::vector<int32_t> wg_begin;     // n_wg+1 offsets into items
    std::vector<WorkItem> items;
    int n_slots = 0;
    std::vector<int32_t> slot_begin;   // per lambda (in batch order): offsets into slot_ids
    std::vector<int32_t> slot_ids;
};

// Distributes (lambda, direction) items over n_wg persistent workgroups so
// that their summed visit counts balance; see schedule.cpp.
// subset: the directions to schedule (all when null).
void build_schedule(const BoxGeometry &g, const std::vector<int32_t> &lambdas, int n_wg, Schedule &out,
                    const std::vector<int32_t> *subset = nullptr, int n_bundles = 1);

// Splits the directions into n_shards sets of nearly equal visit count
// (longest first to the lightest shard); returns shard `shard` sorted.
std::vector<int32_t> shard_directions(const BoxGeometry &g, int n_shards, int shard);

// ---------------------------------------------------------------------------
// Spherical grid: voxels bounded by the spheres r_i = rc + i (ro - rc)/Nr,
// the cones theta_k = k pi/Nt and the half-planes phi_j = 2 pi j/Np; voxel
// index v = (ip Nt + it) Nr + ir.  See sphere_geometry.cpp.
// ---------------------------------------------------------------------------
struct SphereSpec {
    int Nr = 0, Nt = 0, Np = 0;
    double rc = 0, ro = 0;
    double dsrc = 0;  // point source on +z at dsrc * ro (0: none)
    int n_mu = 0, n_phi = 0;
};

// Characteristics of one direction in trace order.  Characteristic c covers
// visits [begin[c], begin[c+1]) and has foot point p (p.n = 0), parameter
// range [ta, tb] along n and kind 0 (enters from outside) or 1 (leaves the
// core).
struct SphereTracks {
    std::vector<int64_t> begin;
    std::vector<double> p, ta, tb;   // p: 3 per characteristic
    std::vector<int8_t> kind;
    std::vector<int32_t> vox;
    std::vector<double> s;
};

std::string check_sphere_spec(const SphereSpec &g);
// Lattice spacing of the ray set: median over voxels of the cube root of the voxel volume.
double sphere_spacing(const SphereSpec &g);
// Traces every characteristic of direction n (lattice rays, then fill-in rays).
void trace_sphere_direction(const SphereSpec &g, double h, const double n[3], SphereTracks &out);
// Irradiation factor of an outer characteristic of direction d entering at x:
// (ro (dsrc - 1))^2 / |x - x_src|^2 / w_d when x is lit and d is the inward
// quadrature direction closest to the light's direction, else 0.
double sphere_irradiation(const SphereSpec &g, const std::vector<Direction> &dirs, int d, const double x[3]);

// The spherical geometry cache: the characteristics of all directions, in
// chunks of consecutive directions.  Per visit: voxel, path length s and
// averaging weight w_d s / (sum of s over the visits of that voxel in that
// direction).  Per characteristic: the boundary factor (>= 0: outer entry,
// irradiation factor; < 0: core start).  Per chunk: a voxel -> visit index
// (CSR) for the fixed-order gather of J.
struct SphereChunk {
    int dir_begin = 0, dir_end = 0;
    int64_t char_begin = 0, char_end = 0;   // global characteristic range
    int64_t visit_begin = 0, visit_end = 0;  // global visit range
    int max_len = 0;
};

struct SphereCache {
    SphereSpec spec;
    double h = 0;
    std::vector<Direction> dirs;
    std::vector<SphereChunk> chunks;
    int64_t n_chars = 0, n_visits = 0;
    int64_t max_chunk_visits = 0;
};

}  // namespace rt3d
