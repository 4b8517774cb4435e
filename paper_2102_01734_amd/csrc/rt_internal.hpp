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

// One direction of the angle quadrature and its characteristic template.
struct Direction {
    double mu = 0, phi = 0, w = 0;
    double n[3] = {0, 0, 0};
    int64_t vbegin = 0;  // first visit of the template in the visit table
    int32_t M = 0;       // number of visits (segments) of every ray
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
    std::vector<int32_t> di, dj, kk;  // unwrapped offsets and layer (tests, tools)
};

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
void build_schedule(const BoxGeometry &g, const std::vector<int32_t> &lambdas, int n_wg, Schedule &out);

}  // namespace rt3d
