// nn_plan.h -- arguments of the surrogate's kernels (k_nn.hip), shared with
// the host-side C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace inim {
namespace nn {

// One convolution layer over `imgs` images of H x W pixels (NHWC, P pixels).
struct ConvArgs {
    const uint16_t* x;   // [P][Cin] BF16 input (forward, weight gradient)
    const uint16_t* w;   // [Cout][ks*ks][Cin] BF16 (forward)
    const uint16_t* wT;  // [Cin][ks*ks][Cout] BF16 (input gradient)
    const float* bias;   // [Cout] or null (forward)
    const uint16_t* dy;  // [P][Cout] BF16 output gradient (backward)
    uint16_t* y16;       // [P][Cout] BF16 output or null
    float* y32;          // [P][Cout] FP32 output or null
    float* dx;           // [P][Cin] FP32 input gradient
    float* dw;           // weight-gradient partials [slices][Cout][ks*ks][Cin]
    int H, W, P, Cin, Cout, ks, relu;
};

struct AdamArgs {
    float lr, b1, b2, eps;
    float c1, c2;  // 1 / (1 - b1^t), 1 / (1 - b2^t)
};

}  // namespace nn
}  // namespace inim
