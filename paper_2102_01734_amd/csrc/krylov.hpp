// krylov.hpp -- vector kernels of the BiCGStab outer solver (see krylov.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rt3d {

// up to four dot products per wavelength: out[4*l + k] = (a_k, b_k) over wavelength l's voxels
struct KDots {
    int n;
    const double *a[4];
    const double *b[4];
};

hipError_t krylov_dots(const KDots &d, int64_t n_vox, int n_lambda, double *blk, int nblk, double *out,
                       hipStream_t st);

enum { KOP_RHS = 0, KOP_P, KOP_AV, KOP_S, KOP_AT, KOP_X, KOP_XH, KOP_J };

// All vectors double [lambda][voxel]; eps, B, lstar in grid precision; c per-wavelength scalars [lambda][4].
struct KVec {
    const void *eps, *B, *lstar;
    const double *c;
    double *x, *y, *u, *b, *r, *rh, *p, *v, *ph, *s, *sh, *t, *J;
};

hipError_t krylov_vec(const KVec &a, int op, int64_t n_vox, int n_lambda, bool grid_double, hipStream_t st);

}  // namespace rt3d
