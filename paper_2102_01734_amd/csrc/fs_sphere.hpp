// fs_sphere.hpp -- launch interface of the spherical formal-solution kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rt3d {

// One chunk of the spherical geometry cache in bundle-major form: the
// chunk's characteristics, longest first, in bundles of 64; entry
// e = bundle_begin[b] + m * 64 + c holds visit m of characteristic c of
// bundle b (padding past a characteristic's length is never read).
struct FsSphereArgs {
    int64_t n_bundles;
    const int64_t *bundle_begin;  // [n_bundles]
    const int32_t *char_len;      // [n_bundles * 64]: visits (0 for padding lanes)
    const double *char_g;         // [n_bundles * 64]: >= 0 outer entry (irradiation factor), < 0 core start
    const int32_t *vox;           // per entry: voxel
    const void *s, *w;            // per entry: path length, averaging weight (geometry type)
    const int32_t *lambda_of;     // batch entry -> wavelength
    int n_batch;                  // batch entries (stride of the outputs)
    int lam_stride;               // wavelengths per voxel in the field
    int L;                        // lanes (batch entries) per characteristic: 1, 2, 4, 8 or 16
    const void *field;            // (chi, S) pairs [voxel][lam_stride][2], kernel type
    const void *I_bc;             // [lambda][3]: I_out, I_core, J_sub (kernel type), or null (all zero)
    void *outJ, *outL;            // [entry][n_batch]: w I, w Lambda*-term (kernel type)
};

// T: arithmetic and field type; geometry in float (gdouble = false) or double.
hipError_t fs_sphere_launch(const FsSphereArgs &a, bool is_double, bool gdouble, bool want_j, bool want_l,
                            bool parabolic_lstar, hipStream_t st);

// dst[b][v] (=, or += when accumulate) sum over the chunk's entries k of voxel
// v, in CSR order, of src[k][b] (double accumulation).
hipError_t sphere_gather(const void *src, bool src_double, const int32_t *row, const int32_t *idx, int64_t n_vox,
                         int n_batch, void *dst, bool dst_double, bool accumulate, hipStream_t st);

}  // namespace rt3d
