// blur_tile.h -- the separable Gaussian of Sec. 4.1 on one 64 x 16 output tile
// (shared by the stand-alone blur and the blur fused with the integral-image
// aggregate pass).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.h"

namespace inim {

constexpr int kBX = 64, kBY = 16;

// Half-sample symmetric continuation: index -1-t reads t, N+t reads N-1-t
// (period 2N).  Indices within one raster width of the border are reflected
// with compares only; the modulo is needed only when the kernel is wider
// than the raster.
__device__ __forceinline__ int mirror(int k, int N) {
    if (k >= 0 && k < N) return k;
    if (k < 0 && k >= -N) return -1 - k;
    if (k >= N && k < 2 * N) return 2 * N - 1 - k;
    const int P = 2 * N;
    int m = k % P;
    if (m < 0) m += P;
    return m >= N ? P - 1 - m : m;
}

__host__ __device__ inline size_t blur_smem_floats(int r) {
    return (size_t)(kBY + 2 * r) * (kBX + 2 * r) + (size_t)(kBY + 2 * r) * kBX;
}

// Blurs the output tile at (ox, oy) with a block of 256 threads: the
// (16+2r) x (64+2r) window of counts is staged in `lds` as float, filtered
// along x into a second LDS buffer, then along y; emit(row, col, value) is
// called once for every output texel of the tile inside the raster.
// R > 0 fixes the radius at compile time (window sizes are constants, the
// taps sit in registers and the tap loops unroll); R == 0 takes taps.r.
template <int R, typename Emit>
__device__ __forceinline__ void blur_tile_r(const uint32_t* __restrict__ counts, int N, const BlurTaps& taps, int ox,
                                            int oy, float* lds, Emit emit) {
    const int r = R > 0 ? R : taps.r;
    const int IW = kBX + 2 * r, IH = kBY + 2 * r;
    float* in = lds;             // IH x IW
    float* mid = lds + IH * IW;  // IH x kBX
    constexpr int NW = R > 0 ? 2 * R + 1 : 1;
    float w[NW];
    if constexpr (R > 0) {
#pragma unroll
        for (int m = 0; m < NW; ++m) w[m] = taps.w[m];
    }
    for (int k = threadIdx.x; k < IH * IW; k += blockDim.x) {
        const int row = k / IW, cc = k - row * IW;
        const int gj = mirror(oy + row - r, N), gi = mirror(ox + cc - r, N);
        in[k] = (float)counts[(size_t)gj * N + gi];
    }
    __syncthreads();
    for (int k = threadIdx.x; k < IH * kBX; k += blockDim.x) {
        const int row = k / kBX, cc = k - row * kBX;
        const float* s = in + row * IW + cc;
        float a = 0.0f;
        if constexpr (R > 0) {
#pragma unroll
            for (int m = 0; m < NW; ++m) a = fmaf(w[m], s[m], a);
        } else {
            for (int m = 0; m <= 2 * r; ++m) a = fmaf(taps.w[m], s[m], a);
        }
        mid[k] = a;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kBY * kBX; k += blockDim.x) {
        const int row = k / kBX, cc = k - row * kBX;
        if (ox + cc >= N || oy + row >= N) continue;
        const float* s = mid + row * kBX + cc;
        float a = 0.0f;
        if constexpr (R > 0) {
#pragma unroll
            for (int m = 0; m < NW; ++m) a = fmaf(w[m], s[m * kBX], a);
        } else {
            for (int m = 0; m <= 2 * r; ++m) a = fmaf(taps.w[m], s[m * kBX], a);
        }
        emit(row, cc, a);
    }
}

// The blur with the radius dispatched to a compile-time copy for the common
// radii (the same sums in the same order, so the results are identical).
template <typename Emit>
__device__ __forceinline__ void blur_tile(const uint32_t* __restrict__ counts, int N, const BlurTaps& taps, int ox,
                                          int oy, float* lds, Emit emit) {
    switch (taps.r) {
        case 2: blur_tile_r<2>(counts, N, taps, ox, oy, lds, emit); break;
        case 4: blur_tile_r<4>(counts, N, taps, ox, oy, lds, emit); break;
        case 8: blur_tile_r<8>(counts, N, taps, ox, oy, lds, emit); break;
        case 16: blur_tile_r<16>(counts, N, taps, ox, oy, lds, emit); break;
        default: blur_tile_r<0>(counts, N, taps, ox, oy, lds, emit); break;
    }
}

}  // namespace inim
