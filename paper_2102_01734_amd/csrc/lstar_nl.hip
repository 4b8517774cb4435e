// lstar_nl.hip -- nearest-neighbour Lambda* of the box (gfx950) and the
// Jacobi sweeps of the operator-splitting system it defines.
//
// The paper's production runs use a non-local Lambda* (Sec. 2, Sec. 3: the
// nearest-neighbour operator, built in the first iteration, with the OS
// system [1 - Lambda*(1-eps)] J_new = J_fs - Lambda*(1-eps) J_old solved by
// Jacobi, Gauss-Seidel or BiCGStab).  Here Lambda* is the exact restriction
// of an operator (the linear-interpolation operator by default, or the
// formal solution itself) to the 27 neighbours of each voxel, as far as a
// characteristic carries it directly from the neighbour to the voxel.
//
// Along one characteristic the intensity is linear in S:
//   I_m = I_{m-1} ex_m + a_m S_{m-1} + b_m S_m + g_m S_{m+1}.
// The derivatives G_j = dI_m / dS(point m - j), j = -1..3, obey
//   G_-1 = g_m,  G_0 = ex_m G_-1' + b_m,  G_1 = ex_m G_0' + a_m,
//   G_2 = ex_m G_1',  G_3 = ex_m G_2'           (' = values at point m - 1),
// and a voxel more than three points upstream cannot be a neighbour of the
// voxel of point m (each step of a straight ray moves some coordinate by
// one and never back), so these five numbers give every neighbour's
// element; G_0 is the local diagonal of the diagonal Lambda*.  Each point
// adds w_d |mu_d| s_m G_j to component c_j of its voxel (the path-length
// weighted mean over the voxel's visits, sum of s = 1/|mu_d|).
//
// One thread follows one characteristic (there is no tile: the sums go to
// HBM).  The sums are fixed-point integers (2^-52 units) added with 64-bit
// integer atomics: integer addition is associative, so the result is bitwise
// independent of the order in which characteristics arrive.  |sum| <= 1 per
// element, so 2^52 leaves ample headroom below 2^63.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ali.hpp"
#include "fs_point.hpp"
#include "lstar_nl.hpp"
#include "rt_internal.hpp"

namespace rt3d {

template <typename G, bool PARA>
__global__ void __launch_bounds__(256) lstar_stencil_kernel(StencilArgs a)
{
    const int Nx = a.Nx, Ny = a.Ny;
    const int NxNy = Nx * Ny;
    const int q = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (q >= NxNy) return;
    const int d = blockIdx.y;
    const int lam = a.lambda_of[blockIdx.z];
    const int y0 = q / Nx, x0 = q - y0 * Nx;
    const G *__restrict__ chi = reinterpret_cast<const G *>(a.chi) + (int64_t)lam * a.n_vox;
    unsigned long long *__restrict__ acc = a.acc + (int64_t)lam * kStencil * a.n_vox;
    const int64_t vb = a.dir_vbegin[d];
    const int M = a.dir_M[d];
    const double wmu = a.dir_wmu[d];
    const int dl = a.dir_mu[d] < 0.0 ? 1 : -1;
    const uint32_t *__restrict__ dxy = a.dxy + vb;
    const double *__restrict__ sv = a.s + vb;
    const uint32_t *__restrict__ comp = a.comp + vb;

    auto voxel = [&](uint32_t w, int k) -> int64_t {
        int x = x0 + (int)(w & kOffMask);
        if (x >= Nx) x -= Nx;
        int y = y0 + (int)((w >> kOffBits) & kOffMask);
        if (y >= Ny) y -= Ny;
        return (int64_t)k * NxNy + (int64_t)y * Nx + x;
    };
    // adds w |mu| s_m G_j to component c_j of voxel v (j = -1..3)
    auto add = [&](int64_t v, double cw, uint32_t comps, const double (&Gv)[5]) {
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            if (!PARA && j == 0) continue;  // no downwind weight in the linear operator
            const uint32_t c = (comps >> (6 * j)) & 63u;
            if (c == kNoComp || (a.skip_centre && c == (uint32_t)kStencilCentre)) continue;
            const long long f = __double2ll_rn(cw * Gv[j] * 0x1p52);
            if (f != 0) atomicAdd(&acc[(int64_t)c * a.n_vox + v], (unsigned long long)f);
        }
    };

    // visit 0 and the look-ahead to visit 1; the layer advances after each layer-end visit
    int k_cur = dl > 0 ? 0 : a.Nz - 1;
    uint32_t w_cur = dxy[0];
    int64_t v_cur = voxel(w_cur, k_cur);
    double t_cur = seg_depth((double)chi[v_cur], sv[0]);
    int k_nxt = k_cur + ((w_cur & kLayerEnd) ? dl : 0);
    uint32_t w_nxt = 0;
    int64_t v_nxt = 0;
    double t_nxt = 0.0;
    if (M > 1) {
        w_nxt = dxy[1];
        v_nxt = voxel(w_nxt, k_nxt);
        t_nxt = seg_depth((double)chi[v_nxt], sv[1]);
    }
    double Gv[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // G_-1, G_0, G_1, G_2, G_3
    {
        double ex0, e00;
        entry_weights<double>(0.5 * t_cur, ex0, e00);
        Gv[1] = e00;
        add(v_cur, wmu * sv[0], comp[0], Gv);
    }
    for (int m = 1; m < M; ++m) {
        const double t_prev = t_cur;
        w_cur = w_nxt;
        v_cur = v_nxt;
        t_cur = t_nxt;
        k_cur = k_nxt;
        k_nxt = k_cur + ((w_cur & kLayerEnd) ? dl : 0);
        const bool last = m + 1 == M;
        if (!last) {
            w_nxt = dxy[m + 1];
            v_nxt = voxel(w_nxt, k_nxt);
            t_nxt = seg_depth((double)chi[v_nxt], sv[m + 1]);
        }
        const double D = half_sum(t_prev, t_cur);
        const double Dp = last ? 0.0 : half_sum(t_cur, t_nxt);
        double ex, wa, wb, wg;
        if (PARA) {
            const PointW<double> pw = point_weights<double>(D, Dp, last);  // full double series
            ex = pw.ex; wa = pw.a; wb = pw.b; wg = pw.g;
        } else {
            // single-precision grids keep the stencil in float: the shorter
            // moment series of the float sweep suffices there
            const double Dv = D < kMinStep ? kMinStep : D;
            double e0, e1, e2;
            kernel_moments<sizeof(G) == 8>(Dv, ex, e0, e1, e2);
            wb = e1 * rcp_f64(Dv);
            wa = e0 - wb;
            wg = 0.0;
        }
        Gv[4] = ex * Gv[3];
        Gv[3] = ex * Gv[2];
        Gv[2] = ex * Gv[1] + wa;
        Gv[1] = ex * Gv[0] + wb;
        Gv[0] = wg;
        add(v_cur, wmu * sv[m], comp[m], Gv);
    }
}

hipError_t lstar_stencil_accumulate(const StencilArgs &a, bool grid_double, bool parabolic, int n_dir, int n_batch,
                                    hipStream_t st)
{
    if (n_dir <= 0 || n_batch <= 0) return hipSuccess;
    const int NxNy = a.Nx * a.Ny;
    dim3 grid((unsigned)((NxNy + 255) / 256), (unsigned)n_dir, (unsigned)n_batch);
    if (grid_double) {
        if (parabolic) hipLaunchKernelGGL((lstar_stencil_kernel<double, true>), grid, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((lstar_stencil_kernel<double, false>), grid, dim3(256), 0, st, a);
    } else {
        if (parabolic) hipLaunchKernelGGL((lstar_stencil_kernel<float, true>), grid, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((lstar_stencil_kernel<float, false>), grid, dim3(256), 0, st, a);
    }
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(256) stencil_finish_kernel(const unsigned long long *__restrict__ acc,
                                                             const int32_t *__restrict__ lambda_of, int64_t n_vox,
                                                             const T *__restrict__ centre, T *__restrict__ out)
{
    const int64_t n = (int64_t)kStencil * n_vox;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t lam = lambda_of[blockIdx.y];
    const int64_t base = lam * n;
    const int64_t c0 = (int64_t)kStencilCentre * n_vox;
    if (centre && i >= c0 && i < c0 + n_vox)
        out[base + i] = centre[lam * n_vox + (i - c0)];
    else
        out[base + i] = (T)((double)(long long)acc[base + i] * 0x1p-52);
}

hipError_t lstar_stencil_finish(const unsigned long long *acc, const int32_t *lambda_of, int64_t n_vox, int n_batch,
                                const void *centre, void *out, bool out_double, hipStream_t st)
{
    if (n_vox <= 0 || n_batch <= 0) return hipSuccess;
    const int64_t n = (int64_t)kStencil * n_vox;
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)n_batch);
    if (out_double)
        hipLaunchKernelGGL((stencil_finish_kernel<double>), grid, dim3(256), 0, st, acc, lambda_of, n_vox,
                           reinterpret_cast<const double *>(centre), reinterpret_cast<double *>(out));
    else
        hipLaunchKernelGGL((stencil_finish_kernel<float>), grid, dim3(256), 0, st, acc, lambda_of, n_vox,
                           reinterpret_cast<const float *>(centre), reinterpret_cast<float *>(out));
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Jacobi sweep: x_v <- (r_v + sum_{c != centre} L_c(v) (1 - eps_u) x_u) / (1 - L_centre(v) (1 - eps_v)),
// neighbours u in component order (a fixed order: reproducible)
// ---------------------------------------------------------------------------
template <typename G>
__global__ void __launch_bounds__(256) os_jacobi_kernel(OsJacobiArgs a, int first)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= a.n_vox) return;
    const int64_t n = a.n_vox;
    const int64_t base = (int64_t)a.lambda_of[blockIdx.y] * n;
    const G *__restrict__ st = reinterpret_cast<const G *>(a.st) + base * kStencil;
    const G *__restrict__ eps = reinterpret_cast<const G *>(a.eps) + base;
    double den = 1.0 - (double)st[kStencilCentre * n + v] * (1.0 - (double)eps[v]);
    den = den < os_den_min<G>() ? os_den_min<G>() : den;
    double acc = a.r[base + v];
    if (!first) {
        const int Nx = a.Nx, Ny = a.Ny;
        const int64_t NxNy = (int64_t)Nx * Ny;
        const int k = (int)(v / NxNy);
        const int rem = (int)(v - (int64_t)k * NxNy);
        const int y = rem / Nx, x = rem - y * Nx;
        for (int c = 0; c < kStencil; ++c) {
            if (c == kStencilCentre) continue;
            const double L = (double)st[(int64_t)c * n + v];
            if (L == 0.0) continue;
            const int ku = k + c / 9 - 1;
            if (ku < 0 || ku >= a.Nz) continue;
            int yu = y + (c / 3) % 3 - 1;
            yu = yu < 0 ? yu + Ny : (yu >= Ny ? yu - Ny : yu);
            int xu = x + c % 3 - 1;
            xu = xu < 0 ? xu + Nx : (xu >= Nx ? xu - Nx : xu);
            const int64_t u = (int64_t)ku * NxNy + (int64_t)yu * Nx + xu;
            acc += L * (1.0 - (double)eps[u]) * a.x_in[base + u];
        }
    }
    a.x_out[base + v] = acc / den;
}

hipError_t os_jacobi_sweep(const OsJacobiArgs &a, bool grid_double, bool first, int n_batch, hipStream_t st)
{
    if (a.n_vox <= 0 || n_batch <= 0) return hipSuccess;
    dim3 grid((unsigned)((a.n_vox + 255) / 256), (unsigned)n_batch);
    if (grid_double)
        hipLaunchKernelGGL((os_jacobi_kernel<double>), grid, dim3(256), 0, st, a, first ? 1 : 0);
    else
        hipLaunchKernelGGL((os_jacobi_kernel<float>), grid, dim3(256), 0, st, a, first ? 1 : 0);
    return hipGetLastError();
}

}  // namespace rt3d
