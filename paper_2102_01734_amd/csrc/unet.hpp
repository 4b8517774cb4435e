// unet.hpp -- the learned ALI correction network (3D U-Net) on the box grid.
//
// Architecture (levels l = 0 .. L-1, channels C_l in {16, 32, 64}, level l
// has n_l = (n_{l-1} + 1) / 2 points per axis, level 0 the grid itself):
//   h_0 = relu(conv_0b(relu(conv_in(f))))              f: 3 input features
//   h_l = relu(conv_lb(relu(down_l(h_{l-1}))))          down: stride-2 3^3 conv
//   for l = L-1 .. 1:
//     h_{l-1} = relu(dec_{l-1}(relu(up_l(lin2(h_l))) + h_{l-1}))
//   out = head . h_0                                     1x1 conv to 1 channel
// Every conv is 3x3x3, periodic in x and y, zero-padded in z; lin2 is
// linear (align-corners) upsampling by 2.  The 3^3 convolutions with
// C_in, C_out >= 16 run as implicit GEMMs on the bf16 matrix cores with
// fp32 accumulation; activations are bf16, channels last.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace rt3d {

// Parsed network (host copy of the weights, float32).
struct UNetSpec {
    int L = 0;
    std::vector<int> C;
    // conv weights [tap][co][ci] and biases, in blob order
    struct Conv {
        int ci = 0, co = 0, taps = 27;
        std::vector<float> w, b;
    };
    std::vector<Conv> convs;  // in, 0b, (down_l, lb) for l>=1, (up_l, dec_{l-1}) for l=L-1..1, head (taps = 1)
};

// Parses a weight blob: "RTUN", u32 version (1), u32 L, u32 C[L], then for
// every conv in the order above its weights [taps][co][ci] and biases [co]
// as little-endian float32.  Returns "" on success.
std::string parse_unet(const void *blob, size_t bytes, UNetSpec &out);

struct UNetDev;  // device weights and activations (unet.hip)

UNetDev *unet_create(const UNetSpec &spec, int nx, int ny, int nz, std::string &err);
void unet_destroy(UNetDev *u);

// out[v] = network(features) for one volume; features [v][3] float, out [v] float.
hipError_t unet_forward(UNetDev *u, const float *features, float *out, hipStream_t st);

// features[v] = ( r[v] / scale, log10(chi[v]) / 4, log10(eps[v]) / 3 + 1 ), r = (J_fs - J)/J
// from the single-precision residual ratio r; chi and eps in grid precision G.
template <typename G>
hipError_t unet_features(const float *r, double scale, const G *chi, const G *eps, int64_t n, float *features,
                         hipStream_t st);

// J[v] *= 1 + clamp(scale * out[v], -0.5, 1)
hipError_t unet_apply(const float *out, double scale, double *J, int64_t n, hipStream_t st);

}  // namespace rt3d
