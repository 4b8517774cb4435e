// krylov.hip -- vector kernels of the BiCGStab outer solver (gfx950).
//
// BiCGStab (van der Vorst 1992) on the operator-splitting system
//   A S = b,  A = 1 - diag(1 - eps) Lambda,  b = (1 - eps) Lambda_bc + eps B,
// the Krylov solver the paper lists next to Jacobi and Gauss-Seidel for the
// OS system (Sec. 4), right-preconditioned by the diagonal
// M = 1 - (1 - eps) Lambda*.  Vectors are double, [lambda][voxel]; per-
// wavelength scalars come from the host.  Dot products are summed per block
// and then over blocks in a fixed order, so iterates are reproducible.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ali.hpp"
#include "krylov.hpp"

namespace rt3d {

// up to four dot products (a_k, b_k) per wavelength, per-block partials
__global__ void __launch_bounds__(256) kdot_kernel(KDots d, int64_t n_vox, double *__restrict__ blk, int nblk)
{
    const int l = blockIdx.y;
    double acc[4] = {0, 0, 0, 0};
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n_vox; v += (int64_t)nblk * blockDim.x) {
        const int64_t i = (int64_t)l * n_vox + v;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < d.n) acc[k] += d.a[k][i] * d.b[k][i];
    }
    __shared__ double red[4][4];
    const int w = threadIdx.x / 64, ln = threadIdx.x % 64;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double x = acc[k];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        if (ln == 0) red[k][w] = x;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int k = threadIdx.x;
        blk[((int64_t)l * nblk + blockIdx.x) * 4 + k] = red[k][0] + red[k][1] + red[k][2] + red[k][3];
    }
}

__global__ void kdot_sum_kernel(const double *__restrict__ blk, int nblk, double *__restrict__ out)
{
    const int l = blockIdx.x;
    const int k = threadIdx.x;
    if (k >= 4) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += blk[((int64_t)l * nblk + b) * 4 + k];
    out[4 * l + k] = s;
}

hipError_t krylov_dots(const KDots &d, int64_t n_vox, int n_lambda, double *blk, int nblk, double *out,
                       hipStream_t st)
{
    if (n_lambda == 0) return hipSuccess;
    hipLaunchKernelGGL(kdot_kernel, dim3(nblk, n_lambda), dim3(256), 0, st, d, n_vox, blk, nblk);
    hipLaunchKernelGGL(kdot_sum_kernel, dim3(n_lambda), dim3(64), 0, st, blk, nblk, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// elementwise steps; c[4*l + k] are the per-wavelength scalars
// ---------------------------------------------------------------------------
template <typename G>
__device__ __forceinline__ double precond(const KVec &a, int64_t i)
{
    const double e = (double)reinterpret_cast<const G *>(a.eps)[i];
    const double L = (double)reinterpret_cast<const G *>(a.lstar)[i];
    const double m = 1.0 - (1.0 - e) * L;
    return m < os_den_min<G>() ? os_den_min<G>() : m;
}

template <typename G>
__global__ void __launch_bounds__(256) kvec_kernel(KVec a, int op, int64_t n_vox)
{
    const int l = blockIdx.y;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n_vox) return;
    const int64_t i = (int64_t)l * n_vox + v;
    const double *c = a.c + 4 * l;
    const double e = (double)reinterpret_cast<const G *>(a.eps)[i];
    switch (op) {
    case KOP_RHS:  // b = (1-eps) J_bc + eps B;  r = b - (x - (1-eps) Lambda x) with Lambda x in y
    {
        const double B = (double)reinterpret_cast<const G *>(a.B)[i];
        const double b = (1.0 - e) * a.u[i] + e * B;
        a.b[i] = b;
        const double r = b - (a.x[i] - (1.0 - e) * a.y[i]);
        a.r[i] = r;
        a.rh[i] = r;
        a.p[i] = 0.0;
        a.v[i] = 0.0;
        break;
    }
    case KOP_P:  // p = r + beta (p - omega v);  phat = p / M
    {
        const double p = a.r[i] + c[0] * (a.p[i] - c[1] * a.v[i]);
        a.p[i] = p;
        a.ph[i] = p / precond<G>(a, i);
        break;
    }
    case KOP_AV:  // v = phat - (1-eps) Lambda phat (Lambda phat in y)
        a.v[i] = a.ph[i] - (1.0 - e) * a.y[i];
        break;
    case KOP_S:  // s = r - alpha v;  shat = s / M
    {
        const double s = a.r[i] - c[0] * a.v[i];
        a.s[i] = s;
        a.sh[i] = s / precond<G>(a, i);
        break;
    }
    case KOP_AT:  // t = shat - (1-eps) Lambda shat (Lambda shat in y)
        a.t[i] = a.sh[i] - (1.0 - e) * a.y[i];
        break;
    case KOP_X:  // x += alpha phat + omega shat;  r = s - omega t   (c = alpha, omega)
        a.x[i] += c[0] * a.ph[i] + c[1] * a.sh[i];
        a.r[i] = a.s[i] - c[1] * a.t[i];
        break;
    case KOP_XH:  // x += alpha phat (converged on s)
        a.x[i] += c[0] * a.ph[i];
        break;
    case KOP_J:  // J = J_bc + Lambda x (Lambda x in y)
        a.J[i] = a.u[i] + a.y[i];
        break;
    default:
        break;
    }
}

template <typename G>
static hipError_t kvec_t(const KVec &a, int op, int64_t n_vox, int n_lambda, hipStream_t st)
{
    dim3 grid((unsigned)((n_vox + 255) / 256), (unsigned)n_lambda);
    hipLaunchKernelGGL((kvec_kernel<G>), grid, dim3(256), 0, st, a, op, n_vox);
    return hipGetLastError();
}

hipError_t krylov_vec(const KVec &a, int op, int64_t n_vox, int n_lambda, bool grid_double, hipStream_t st)
{
    if (n_lambda == 0 || n_vox == 0) return hipSuccess;
    return grid_double ? kvec_t<double>(a, op, n_vox, n_lambda, st) : kvec_t<float>(a, op, n_vox, n_lambda, st);
}

}  // namespace rt3d
