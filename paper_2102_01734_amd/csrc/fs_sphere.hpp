// fs_sphere.hpp -- launch interface of the spherical formal-solution kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rt3d {

struct FsSphereArgs {
    int64_t n_vox;
    // characteristics [char0, char0 + n_chars) of one chunk; visit offsets are global
    int64_t char0, n_chars;
    int64_t visit0;              // first visit of the chunk
    const int64_t *char_begin;   // visit range of characteristic c: [char_begin[c], char_begin[c+1])
    const double *char_g;        // boundary factor: >= 0 outer entry (irradiation factor), < 0 core start
    const int32_t *vox;          // per visit: voxel
    const void *s, *w;           // per visit: path length, averaging weight (geometry type)
    const int32_t *lambda_of;    // batch entry -> wavelength
    const void *field;           // (chi, S) pairs [lambda][voxel][2], kernel type
    const void *I_bc;            // [lambda][3]: I_out, I_core, J_sub (kernel type), or null (all zero)
    void *outJ, *outL;           // per batch entry and chunk visit: w I, w Lambda*_point (kernel type)
    int64_t out_stride;          // elements per batch entry in outJ / outL
};

// T: arithmetic and field type; geometry in float (gdouble = false) or double.
hipError_t fs_sphere_launch(const FsSphereArgs &a, bool is_double, bool gdouble, bool want_j, bool want_l,
                            bool parabolic_lstar, int n_batch, hipStream_t st);

// dst[b][v] (=, or += when accumulate) sum over the chunk's visits k of voxel v,
// in CSR order, of src[b][k] (double accumulation).
hipError_t sphere_gather(const void *src, bool src_double, int64_t src_stride, const int32_t *row, const int32_t *idx,
                         int64_t n_vox, int n_batch, void *dst, bool dst_double, bool accumulate, hipStream_t st);

}  // namespace rt3d
