// launch.h -- host-side launchers of the gfx950 kernels (used by the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "inim_plan.h"

namespace inim {

constexpr int kMaxRadius = 32;

struct BlurTaps {
    int r;
    float w[2 * kMaxRadius + 1];
};

// Integral images of `img` in two steps, sharing the buffers in `scratch`
// (inim_scratch_bytes): the tile partial sums and band carries, then the final
// pass, which writes the planes in `mask` -- or, when field != nullptr, the
// deformation with background d0 -- and, when marg != nullptr, the marginals.
// Accumulators: uint32 for uint32 rasters; for float rasters unsigned
// __int128 (exact 128-bit fixed point) or double.
template <typename Tin, typename Acc>
hipError_t launch_inim_carries(const Tin* img, const Geom& g, void* scratch, const int* status, hipStream_t st);
template <typename Tin, typename Acc>
hipError_t launch_inim_final(const Tin* img, const Geom& g, void* scratch, uint32_t mask, Tin* planes, float2* field,
                             double d0, double* marg, const int* status, hipStream_t st);

hipError_t launch_deform_planes(const void* alpha, const void* alpha_t, int dt, const double* marg, int N, double d0,
                                float2* field, hipStream_t st);

hipError_t launch_fill(uint32_t* counts, size_t count, int* status, bool clear_status, hipStream_t st);
hipError_t launch_splat(const float2* xy, int64_t n, int N, uint32_t* counts, int* status, hipStream_t st);
hipError_t launch_blur(const uint32_t* counts, float* out, int N, const BlurTaps& taps, const int* status,
                       hipStream_t st);
hipError_t launch_validate(const float2* xy, int64_t n, int* status, hipStream_t st);
hipError_t launch_advect(const float2* field, int N, float2* xy, int64_t n, const int* status, hipStream_t st);

}  // namespace inim
