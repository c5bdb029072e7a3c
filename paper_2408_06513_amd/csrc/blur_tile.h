// blur_tile.h -- the separable Gaussian of Sec. 4.1 on one 64 x 16 output tile
// (shared by the stand-alone blur and the blur fused with the integral-image
// aggregate pass).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.h"

namespace inim {

constexpr int kBX = 64, kBY = 16;
constexpr int kBlurThreads = 256;  // threads of every block that blurs a tile

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

// Blurs the output tile at (ox, oy) with a block of kBlurThreads threads: the
// (16+2r) x (64+2r) window of counts is staged in `lds` as float, filtered
// along x into a second LDS buffer, then along y; emit(row, col, value) is
// called once for every output texel of the tile inside the raster.
// R > 0 fixes the radius at compile time: the window sizes are constants (for
// R a multiple of 4 the window is loaded in 16-byte chunks), the
// taps sit in registers, and each thread computes four neighbouring outputs
// from one register window (4 + 2R values read once: as float4 along x,
// column-wise along y) instead of reading 2R + 1 values per output.  Every
// output is the same fmaf chain over the taps in the same order as with
// R == 0, which takes taps.r and one output per thread.
template <int R, typename Emit>
__device__ __forceinline__ void blur_tile_r(const uint32_t* __restrict__ counts, int N, const BlurTaps& taps, int ox,
                                            int oy, float* lds, Emit emit) {
    const int r = R > 0 ? R : taps.r;
    const int IW = kBX + 2 * r, IH = kBY + 2 * r;
    float* in = lds;             // IH x IW
    float* mid = lds + IH * IW;  // IH x kBX
    // the window in chunks of 4 columns: a chunk inside the raster is one
    // 16-byte load (its first column, ox - R + 4q, is a multiple of 4; the
    // raster's base must be 16-byte aligned, else every chunk takes the other
    // path), a chunk over the border takes its 4 mirrored columns one by one.
    // Each thread loads all its chunks before storing any, so the window costs
    // one round of memory latency (a thread past the last chunk reloads the
    // last one and stores nothing).
    const bool vec = (reinterpret_cast<uintptr_t>(counts) & 15u) == 0u;
    if (R > 0 && R % 4 == 0 && vec) {
        constexpr int IWc = kBX + 2 * R, IHc = kBY + 2 * R, CW = IWc / 4, ITEMS = IHc * CW;
        constexpr int PER = (ITEMS + kBlurThreads - 1) / kBlurThreads;
        uint4 u[PER];
#pragma unroll
        for (int t = 0; t < PER; ++t) {
            const int k0 = (int)threadIdx.x + t * kBlurThreads, k = k0 < ITEMS ? k0 : ITEMS - 1;
            const int row = k / CW, q = k - row * CW;
            const int gj = mirror(oy + row - R, N);
            const int c0 = ox - R + 4 * q;
            const uint32_t* src = counts + (size_t)gj * N;
            if (c0 >= 0 && c0 + 3 < N)
                u[t] = *reinterpret_cast<const uint4*>(src + c0);
            else
                u[t] = make_uint4(src[mirror(c0, N)], src[mirror(c0 + 1, N)], src[mirror(c0 + 2, N)],
                                  src[mirror(c0 + 3, N)]);
        }
#pragma unroll
        for (int t = 0; t < PER; ++t) {
            const int k = (int)threadIdx.x + t * kBlurThreads;
            if (k < ITEMS) {
                const int row = k / CW, q = k - row * CW;
                *reinterpret_cast<float4*>(in + row * IWc + 4 * q) =
                    make_float4((float)u[t].x, (float)u[t].y, (float)u[t].z, (float)u[t].w);
            }
        }
    } else {
        for (int k = threadIdx.x; k < IH * IW; k += blockDim.x) {
            const int row = k / IW, cc = k - row * IW;
            const int gj = mirror(oy + row - r, N), gi = mirror(ox + cc - r, N);
            in[k] = (float)counts[(size_t)gj * N + gi];
        }
    }
    __syncthreads();
    if constexpr (R > 0) {
        static_assert(R % 2 == 0, "window rows of whole float4s");
        constexpr int NW = 2 * R + 1, WIN = 4 + 2 * R;
        float w[NW];
#pragma unroll
        for (int m = 0; m < NW; ++m) w[m] = taps.w[m];
        constexpr int IWc = kBX + 2 * R, IHc = kBY + 2 * R;
        for (int k = threadIdx.x; k < IHc * (kBX / 4); k += blockDim.x) {
            const int row = k / (kBX / 4), c4 = (k - row * (kBX / 4)) * 4;
            const float* s = in + row * IWc + c4;
            float x[WIN];
#pragma unroll
            for (int q = 0; q < WIN / 4; ++q) {
                const float4 t = *reinterpret_cast<const float4*>(s + 4 * q);
                x[4 * q] = t.x; x[4 * q + 1] = t.y; x[4 * q + 2] = t.z; x[4 * q + 3] = t.w;
            }
            float a[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int m = 0; m < NW; ++m)
#pragma unroll
                for (int e = 0; e < 4; ++e) a[e] = fmaf(w[m], x[m + e], a[e]);
            *reinterpret_cast<float4*>(mid + row * kBX + c4) = make_float4(a[0], a[1], a[2], a[3]);
        }
        __syncthreads();
        for (int k = threadIdx.x; k < (kBY / 4) * kBX; k += blockDim.x) {
            const int r4 = (k / kBX) * 4, cc = k - (k / kBX) * kBX;
            const float* s = mid + r4 * kBX + cc;
            float y[WIN];
#pragma unroll
            for (int q = 0; q < WIN; ++q) y[q] = s[q * kBX];
            float a[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int m = 0; m < NW; ++m)
#pragma unroll
                for (int e = 0; e < 4; ++e) a[e] = fmaf(w[m], y[m + e], a[e]);
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (ox + cc < N && oy + r4 + e < N) emit(r4 + e, cc, a[e]);
        }
    } else {
        for (int k = threadIdx.x; k < IH * kBX; k += blockDim.x) {
            const int row = k / kBX, cc = k - row * kBX;
            const float* s = in + row * IW + cc;
            float a = 0.0f;
            for (int m = 0; m <= 2 * r; ++m) a = fmaf(taps.w[m], s[m], a);
            mid[k] = a;
        }
        __syncthreads();
        for (int k = threadIdx.x; k < kBY * kBX; k += blockDim.x) {
            const int row = k / kBX, cc = k - row * kBX;
            if (ox + cc >= N || oy + row >= N) continue;
            const float* s = mid + row * kBX + cc;
            float a = 0.0f;
            for (int m = 0; m <= 2 * r; ++m) a = fmaf(taps.w[m], s[m * kBX], a);
            emit(row, cc, a);
        }
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
