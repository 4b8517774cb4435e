// unet.hip -- inference of the learned ALI correction network (gfx950).
//
// The 3^3 convolutions between feature maps of 16, 32 or 64 channels are
// implicit GEMMs on the matrix cores (v_mfma_f32_16x16x32_bf16): the
// reduction index k runs over (tap, input channel), 27 CI values padded to a
// multiple of 32, and one wavefront computes T tiles of 16 consecutive
// output voxels (in flattened z, y, x order) times all output channels.  Per
// 32-wide k chunk a lane loads 8 consecutive input channels of one tap for
// its voxel (A, 16 bytes, channels last; zero for the padding taps and for
// taps beyond the top or bottom layer) and 8 weights of one output channel
// (B, 16 bytes); products accumulate in fp32.  Bias, ReLU and the U-Net skip
// addition are fused into the store.  The small layers (3 input features,
// the 1-channel head) and the upsampling are plain VALU kernels.
// Activations never leave HBM between layers; at 129^3 with 16 channels a
// level-0 map is 68 MB.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <memory>

#include "unet.hpp"

namespace rt3d {

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t f2bf(float f)
{
    // round to nearest even (finite inputs)
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

static uint16_t f2bf_host(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

struct Vol {
    int nx, ny, nz;
    __host__ __device__ int64_t n() const { return (int64_t)nx * ny * nz; }
};

// ---------------------------------------------------------------------------
// 3^3 convolution on the matrix cores
// ---------------------------------------------------------------------------
struct ConvArgs {
    const uint16_t *in;
    Vol vi, vo;
    int stride;
    const uint16_t *w;     // [27][CO][CI] bf16
    const float *bias;     // [CO]
    const uint16_t *skip;  // [vo][CO] bf16 added after the ReLU, or null
    uint16_t *out;         // [vo][CO]
};

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v8bf load8(const uint16_t *p, bool ok)
{
    v4u u = ok ? *reinterpret_cast<const v4u *>(p) : v4u{0u, 0u, 0u, 0u};
    return __builtin_bit_cast(v8bf, u);
}

constexpr int kConvTiles = 2;  // 16-voxel tiles per wavefront

template <int CI, int CO>
__global__ void __launch_bounds__(256) conv_mfma_kernel(ConvArgs a)
{
    constexpr int T = kConvTiles;
    constexpr int NB = CO / 16;
    constexpr int NK = (27 * CI + 31) / 32;  // 32-wide chunks of (tap, channel)
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t nvo = a.vo.n();
    const int64_t v0 = wave * (16 * T);
    if (v0 >= nvo) return;  // uniform per wavefront
    const int i = lane & 15;       // A row (voxel) / B column (output channel)
    const int kq = (lane >> 4) * 8;  // first of the 8 k values of this lane in a chunk
    const int S = a.stride;
    int xs[T], ys[T], zs[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        int64_t v = v0 + 16 * t + i;
        v = v < nvo ? v : nvo - 1;  // loads of the tail tile repeat the last voxel; its stores are masked
        const int64_t r = v / a.vo.nx;
        xs[t] = (int)(v - r * a.vo.nx) * S - 1;
        ys[t] = (int)(r % a.vo.ny) * S - 1;
        zs[t] = (int)(r / a.vo.ny) * S - 1;
    }
    v4f acc[T][NB];
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
        for (int c = 0; c < NB; ++c) acc[t][c] = v4f{0.f, 0.f, 0.f, 0.f};

    for (int j = 0; j < NK; ++j) {
        const int k = j * 32 + kq;
        const int tap = k / CI, c0 = k % CI;  // CI is a power of two
        const bool tap_ok = tap < 27;
        const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
        v8bf B[NB];
#pragma unroll
        for (int cb = 0; cb < NB; ++cb)
            B[cb] = load8(a.w + ((int64_t)(tap_ok ? tap : 0) * CO + cb * 16 + i) * CI + c0, tap_ok);
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const int zi = zs[t] + dz;
            const bool ok = tap_ok && zi >= 0 && zi < a.vi.nz;
            const int yi = wrap(ys[t] + dy, a.vi.ny);
            const int xi = wrap(xs[t] + dx, a.vi.nx);
            const v8bf A = load8(a.in + (((int64_t)(ok ? zi : 0) * a.vi.ny + yi) * a.vi.nx + xi) * CI + c0, ok);
#pragma unroll
            for (int cb = 0; cb < NB; ++cb) acc[t][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B[cb], acc[t][cb], 0, 0, 0);
        }
    }
    // D layout: lane holds rows kq/2 .. kq/2 + 3 (voxels) of column i (output channel)
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) {
            const int co = cb * 16 + i;
            const float b = a.bias[co];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t v = v0 + 16 * t + (lane >> 4) * 4 + r;
                if (v >= nvo) continue;
                float val = fmaxf(acc[t][cb][r] + b, 0.f);
                if (a.skip) val += bf2f(a.skip[v * CO + co]);
                a.out[v * CO + co] = f2bf(val);
            }
        }
}

template <int CI, int CO>
static hipError_t conv_t(const ConvArgs &a, hipStream_t st)
{
    const int64_t waves = (a.vo.n() + 16 * kConvTiles - 1) / (16 * kConvTiles);
    hipLaunchKernelGGL((conv_mfma_kernel<CI, CO>), dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, a);
    return hipGetLastError();
}

static hipError_t conv_mfma(const ConvArgs &a, int ci, int co, hipStream_t st)
{
#define RT_CONV_CASE(I, O) \
    if (ci == I && co == O) return conv_t<I, O>(a, st);
    RT_CONV_CASE(16, 16) RT_CONV_CASE(16, 32) RT_CONV_CASE(16, 64)
    RT_CONV_CASE(32, 16) RT_CONV_CASE(32, 32) RT_CONV_CASE(32, 64)
    RT_CONV_CASE(64, 16) RT_CONV_CASE(64, 32) RT_CONV_CASE(64, 64)
#undef RT_CONV_CASE
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// input layer (3 features -> C channels) and head (C -> 1), fp32 VALU
// ---------------------------------------------------------------------------
template <int CO>
__global__ void __launch_bounds__(256) conv_in_kernel(const float *__restrict__ f, Vol v, const float *__restrict__ w,
                                                      const float *__restrict__ bias, uint16_t *__restrict__ out)
{
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= v.n()) return;
    const int x = (int)(id % v.nx);
    const int64_t r = id / v.nx;
    const int y = (int)(r % v.ny);
    const int z = (int)(r / v.ny);
    float acc[CO];
#pragma unroll
    for (int c = 0; c < CO; ++c) acc[c] = bias[c];
    for (int dz = 0; dz < 3; ++dz) {
        const int zi = z + dz - 1;
        if (zi < 0 || zi >= v.nz) continue;
        for (int dy = 0; dy < 3; ++dy) {
            const int yi = wrap(y + dy - 1, v.ny);
            for (int dx = 0; dx < 3; ++dx) {
                const int xi = wrap(x + dx - 1, v.nx);
                const float *fp = f + (((int64_t)zi * v.ny + yi) * v.nx + xi) * 3;
                const float f0 = fp[0], f1 = fp[1], f2 = fp[2];
                const float *wt = w + ((dz * 3 + dy) * 3 + dx) * CO * 3;
#pragma unroll
                for (int c = 0; c < CO; ++c) acc[c] += wt[3 * c] * f0 + wt[3 * c + 1] * f1 + wt[3 * c + 2] * f2;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < CO; ++c) out[id * CO + c] = f2bf(fmaxf(acc[c], 0.f));
}

template <int C>
__global__ void __launch_bounds__(256) head_kernel(const uint16_t *__restrict__ h, int64_t n, const float *__restrict__ w,
                                                   const float *__restrict__ bias, float *__restrict__ out)
{
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n) return;
    float acc = bias[0];
#pragma unroll
    for (int c = 0; c < C; ++c) acc += w[c] * bf2f(h[id * C + c]);
    out[id] = acc;
}

// linear upsampling by 2 (align corners): fine index o takes the coarse
// point o/2 (o even) or the mean of (o-1)/2 and (o+1)/2 (o odd); the upper
// neighbour wraps in x, y and is clamped in z.  One thread per fine voxel
// and 8 channels (16-byte loads and stores; C is a multiple of 16).
__global__ void __launch_bounds__(256) upsample_kernel(const uint16_t *__restrict__ in, Vol vc, uint16_t *__restrict__ out,
                                                       Vol vf, int C)
{
    const int groups = C / 8;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= vf.n() * groups) return;
    const int c0 = (int)(id % groups) * 8;
    const int64_t v = id / groups;
    const int x = (int)(v % vf.nx);
    const int64_t r = v / vf.nx;
    const int y = (int)(r % vf.ny);
    const int z = (int)(r / vf.ny);
    int xs[2], ys[2], zs[2];
    xs[0] = x >> 1; xs[1] = (x & 1) ? wrap((x + 1) >> 1, vc.nx) : xs[0];
    ys[0] = y >> 1; ys[1] = (y & 1) ? wrap((y + 1) >> 1, vc.ny) : ys[0];
    zs[0] = z >> 1; zs[1] = (z & 1) ? min((z + 1) >> 1, vc.nz - 1) : zs[0];
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                const v4u q = *reinterpret_cast<const v4u *>(
                    in + (((int64_t)zs[a] * vc.ny + ys[b]) * vc.nx + xs[d]) * C + c0);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    acc[2 * e] += __uint_as_float(q[e] << 16);
                    acc[2 * e + 1] += __uint_as_float(q[e] & 0xffff0000u);
                }
            }
    v4u o;
#pragma unroll
    for (int e = 0; e < 4; ++e)
        o[e] = (uint32_t)f2bf(0.125f * acc[2 * e]) | ((uint32_t)f2bf(0.125f * acc[2 * e + 1]) << 16);
    *reinterpret_cast<v4u *>(out + v * C + c0) = o;
}

// ---------------------------------------------------------------------------
// features and application of the correction
// ---------------------------------------------------------------------------
template <typename G>
__global__ void __launch_bounds__(256) features_kernel(const float *__restrict__ r, float inv_scale,
                                                       const G *__restrict__ chi, const G *__restrict__ eps, int64_t n,
                                                       float *__restrict__ f)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const float c = fmaxf((float)chi[v], 1e-30f), e = fmaxf((float)eps[v], 1e-30f);
    f[3 * v] = r[v] * inv_scale;
    f[3 * v + 1] = log10f(c) * 0.25f;
    f[3 * v + 2] = log10f(e) * (1.0f / 3.0f) + 1.0f;
}

template <typename G>
hipError_t unet_features(const float *r, double scale, const G *chi, const G *eps, int64_t n, float *features,
                         hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const float inv = scale > 0.0 ? (float)(1.0 / scale) : 0.f;
    hipLaunchKernelGGL((features_kernel<G>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, r, inv, chi, eps, n,
                       features);
    return hipGetLastError();
}
template hipError_t unet_features<float>(const float *, double, const float *, const float *, int64_t, float *,
                                         hipStream_t);
template hipError_t unet_features<double>(const float *, double, const double *, const double *, int64_t, float *,
                                          hipStream_t);

__global__ void __launch_bounds__(256) apply_kernel(const float *__restrict__ out, double scale, double *__restrict__ J,
                                                    int64_t n)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    double d = scale * (double)out[v];
    d = d < -0.5 ? -0.5 : (d > 1.0 ? 1.0 : d);
    J[v] *= 1.0 + d;
}

hipError_t unet_apply(const float *out, double scale, double *J, int64_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(apply_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, out, scale, J, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
std::string parse_unet(const void *blob, size_t bytes, UNetSpec &out)
{
    out = UNetSpec();
    const unsigned char *p = static_cast<const unsigned char *>(blob);
    size_t off = 0;
    auto u32 = [&](uint32_t &v) {
        if (off + 4 > bytes) return false;
        std::memcpy(&v, p + off, 4);
        off += 4;
        return true;
    };
    if (bytes < 12 || std::memcmp(p, "RTUN", 4) != 0) return "not a network blob (magic)";
    off = 4;
    uint32_t ver = 0, L = 0;
    if (!u32(ver) || ver != 1) return "unsupported network blob version";
    if (!u32(L) || L < 1 || L > 6) return "number of levels must be 1..6";
    out.L = (int)L;
    for (uint32_t l = 0; l < L; ++l) {
        uint32_t c = 0;
        if (!u32(c) || (c != 16 && c != 32 && c != 64)) return "channel counts must be 16, 32 or 64";
        out.C.push_back((int)c);
    }
    auto conv = [&](int ci, int co, int taps) {
        UNetSpec::Conv cv;
        cv.ci = ci; cv.co = co; cv.taps = taps;
        const size_t nw = (size_t)taps * co * ci;
        if (off + 4 * (nw + co) > bytes) return false;
        cv.w.resize(nw);
        cv.b.resize(co);
        std::memcpy(cv.w.data(), p + off, 4 * nw);
        off += 4 * nw;
        std::memcpy(cv.b.data(), p + off, 4 * (size_t)co);
        off += 4 * (size_t)co;
        out.convs.push_back(std::move(cv));
        return true;
    };
    const auto &C = out.C;
    if (!conv(3, C[0], 27) || !conv(C[0], C[0], 27)) return "truncated blob";
    for (int l = 1; l < out.L; ++l)
        if (!conv(C[l - 1], C[l], 27) || !conv(C[l], C[l], 27)) return "truncated blob";
    for (int l = out.L - 1; l >= 1; --l)
        if (!conv(C[l], C[l - 1], 27) || !conv(C[l - 1], C[l - 1], 27)) return "truncated blob";
    if (!conv(C[0], 1, 1)) return "truncated blob";
    if (off != bytes) return "trailing bytes after the last layer";
    for (const auto &cv : out.convs)
        for (float x : cv.w)
            if (!std::isfinite(x)) return "non-finite weight";
    return "";
}

struct DevMem {
    void *p = nullptr;
    ~DevMem() { if (p) (void)hipFree(p); }
};

struct UNetDev {
    UNetSpec spec;
    std::vector<Vol> lv;                       // volume of each level
    std::vector<std::unique_ptr<DevMem>> mem;  // every allocation
    std::vector<const void *> w, b;            // per conv: weights (bf16 or fp32), biases (fp32)
    std::vector<uint16_t *> h, t;              // per level activations
    uint16_t *up = nullptr;                    // upsampled map (largest)
};

static hipError_t dev_alloc(UNetDev *u, size_t bytes, void **out)
{
    auto m = std::make_unique<DevMem>();
    hipError_t e = hipMalloc(&m->p, bytes > 0 ? bytes : 16);
    if (e != hipSuccess) return e;
    *out = m->p;
    u->mem.push_back(std::move(m));
    return hipSuccess;
}

UNetDev *unet_create(const UNetSpec &spec, int nx, int ny, int nz, std::string &err)
{
    auto u = std::make_unique<UNetDev>();
    u->spec = spec;
    Vol v{nx, ny, nz};
    for (int l = 0; l < spec.L; ++l) {
        if (l > 0) v = Vol{(v.nx + 1) / 2, (v.ny + 1) / 2, (v.nz + 1) / 2};
        u->lv.push_back(v);
    }
    hipError_t e = hipSuccess;
    for (size_t k = 0; k < spec.convs.size() && e == hipSuccess; ++k) {
        const auto &cv = spec.convs[k];
        const bool mfma = cv.taps == 27 && cv.ci >= 16;
        void *wp = nullptr, *bp = nullptr;
        if (mfma) {
            std::vector<uint16_t> wb(cv.w.size());
            for (size_t i = 0; i < wb.size(); ++i) wb[i] = f2bf_host(cv.w[i]);
            if ((e = dev_alloc(u.get(), wb.size() * 2, &wp)) == hipSuccess)
                e = hipMemcpy(wp, wb.data(), wb.size() * 2, hipMemcpyHostToDevice);
        } else {
            if ((e = dev_alloc(u.get(), cv.w.size() * 4, &wp)) == hipSuccess)
                e = hipMemcpy(wp, cv.w.data(), cv.w.size() * 4, hipMemcpyHostToDevice);
        }
        if (e == hipSuccess && (e = dev_alloc(u.get(), cv.b.size() * 4, &bp)) == hipSuccess)
            e = hipMemcpy(bp, cv.b.data(), cv.b.size() * 4, hipMemcpyHostToDevice);
        u->w.push_back(wp);
        u->b.push_back(bp);
    }
    size_t up_bytes = 0;
    for (int l = 0; l < spec.L && e == hipSuccess; ++l) {
        void *hp = nullptr, *tp = nullptr;
        const size_t bytes = (size_t)u->lv[l].n() * spec.C[l] * 2;
        if ((e = dev_alloc(u.get(), bytes, &hp)) == hipSuccess) e = dev_alloc(u.get(), bytes, &tp);
        u->h.push_back((uint16_t *)hp);
        u->t.push_back((uint16_t *)tp);
        if (l > 0) up_bytes = std::max(up_bytes, (size_t)u->lv[l - 1].n() * spec.C[l] * 2);
    }
    if (e == hipSuccess && spec.L > 1) {
        void *p = nullptr;
        e = dev_alloc(u.get(), up_bytes, &p);
        u->up = (uint16_t *)p;
    }
    if (e != hipSuccess) {
        err = std::string("network buffers: ") + hipGetErrorString(e);
        return nullptr;
    }
    return u.release();
}

void unet_destroy(UNetDev *u) { delete u; }

template <int C>
static hipError_t conv_in_t(const float *f, Vol v, const float *w, const float *b, uint16_t *out, hipStream_t st)
{
    hipLaunchKernelGGL((conv_in_kernel<C>), dim3((unsigned)((v.n() + 255) / 256)), dim3(256), 0, st, f, v, w, b, out);
    return hipGetLastError();
}

template <int C>
static hipError_t head_t(const uint16_t *h, int64_t n, const float *w, const float *b, float *out, hipStream_t st)
{
    hipLaunchKernelGGL((head_kernel<C>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, h, n, w, b, out);
    return hipGetLastError();
}

hipError_t unet_forward(UNetDev *u, const float *features, float *out, hipStream_t st)
{
    const UNetSpec &s = u->spec;
    const auto &C = s.C;
    size_t k = 0;  // conv index in blob order
    hipError_t e;
    auto conv = [&](const uint16_t *in, Vol vi, Vol vo, int stride, int ci, int co, const uint16_t *skip,
                    uint16_t *o) {
        ConvArgs a{in, vi, vo, stride, (const uint16_t *)u->w[k], (const float *)u->b[k], skip, o};
        ++k;
        return conv_mfma(a, ci, co, st);
    };
    // level 0 input layer
    const Vol v0 = u->lv[0];
    switch (C[0]) {
    case 16: e = conv_in_t<16>(features, v0, (const float *)u->w[0], (const float *)u->b[0], u->t[0], st); break;
    case 32: e = conv_in_t<32>(features, v0, (const float *)u->w[0], (const float *)u->b[0], u->t[0], st); break;
    default: e = conv_in_t<64>(features, v0, (const float *)u->w[0], (const float *)u->b[0], u->t[0], st); break;
    }
    if (e != hipSuccess) return e;
    k = 1;
    if ((e = conv(u->t[0], v0, v0, 1, C[0], C[0], nullptr, u->h[0])) != hipSuccess) return e;
    for (int l = 1; l < s.L; ++l) {
        if ((e = conv(u->h[l - 1], u->lv[l - 1], u->lv[l], 2, C[l - 1], C[l], nullptr, u->t[l])) != hipSuccess)
            return e;
        if ((e = conv(u->t[l], u->lv[l], u->lv[l], 1, C[l], C[l], nullptr, u->h[l])) != hipSuccess) return e;
    }
    for (int l = s.L - 1; l >= 1; --l) {
        const Vol vc = u->lv[l], vf = u->lv[l - 1];
        const int64_t nup = vf.n() * (C[l] / 8);
        hipLaunchKernelGGL(upsample_kernel, dim3((unsigned)((nup + 255) / 256)), dim3(256), 0, st, u->h[l], vc, u->up,
                           vf, C[l]);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = conv(u->up, vf, vf, 1, C[l], C[l - 1], u->h[l - 1], u->t[l - 1])) != hipSuccess) return e;
        if ((e = conv(u->t[l - 1], vf, vf, 1, C[l - 1], C[l - 1], nullptr, u->h[l - 1])) != hipSuccess) return e;
    }
    const float *hw = (const float *)u->w[k], *hb = (const float *)u->b[k];
    switch (C[0]) {
    case 16: return head_t<16>(u->h[0], v0.n(), hw, hb, out, st);
    case 32: return head_t<32>(u->h[0], v0.n(), hw, hb, out, st);
    default: return head_t<64>(u->h[0], v0.n(), hw, hb, out, st);
    }
}

}  // namespace rt3d
