// fs_box.hpp -- launch interface of the box formal-solution kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "rt_internal.hpp"

namespace rt3d {

struct FsBoxArgs {
    int Nx, Ny, Nz;
    int64_t n_vox;
    // visit table (directions back to back) and per-direction data
    const int32_t *goff;
    const uint32_t *dxy;
    const double *s;
    const int64_t *dir_vbegin;
    const int32_t *dir_M;
    const double *dir_wmu;  // w_d |mu_d|
    const double *dir_mu;
    // schedule
    const int32_t *wg_begin;
    const WorkItem *items;
    // (chi, S) pairs, doubly periodic padded [lambda][Nz][2Ny][2Nx][2],
    // element type = kernel type; pad_stride = pairs per wavelength
    const void *field;
    int64_t pad_stride;
    const void *I_bc;  // [lambda][2] or null
    // ray bundles, b = w mod n_bundles for workgroup w.  Layer tiles: workgroup
    // w sweeps rays [b Q, min((b+1) Q, NxNy)), Q = bundle_rays, into a tile of
    // the whole layer.  Band tiles: it sweeps the ray rows
    // [b Ny / n_bundles, (b+1) Ny / n_bundles) into a tile of the rows that
    // those rays reach within one layer (see fs_box.hip)
    int n_bundles, bundle_rays;
    int tile_words;           // words of one tile (NxNy for layer tiles)
    const int32_t *brow;      // per visit: row relative to the layer's lowest template row
    const int32_t *dir_span;  // per direction: largest such relative row
    // partial sums [slot][n_vox]
    void *partJ;
    void *partL;
};

// A compiled launch shape: workgroup size bound `lb`, rays per thread `R`;
// `full`: available for every output combination (else J-only); `occ`: see
// fs_box.hip; `band`: band tiles instead of layer tiles.
struct FsShape {
    int lb, R;
    bool full;
    int occ;  // workgroups per CU the shape is compiled for (layer tiles: = ray bundles per direction)
    bool band;
};
int fs_box_shapes(const FsShape **out);

hipError_t fs_box_launch(const FsBoxArgs &a, bool is_double, bool want_j, bool want_l, bool parabolic_lstar,
                         bool band, int lb, int R, int n_wg, int nthr, size_t lds_bytes, hipStream_t stream);

// Resident workgroups per CU of a shape; negative if its kernel spills
// registers (the magnitude is then still the occupancy).
int fs_box_occupancy(bool is_double, bool want_j, bool want_l, bool parabolic_lstar, bool band, int lb, int R,
                     int nthr, size_t lds_bytes);

}  // namespace rt3d
