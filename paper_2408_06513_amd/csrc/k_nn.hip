// k_nn.hip -- the kernels of the learned surrogate on gfx950: 3x3 (and 1x1)
// convolutions as implicit GEMMs on the BF16 matrix cores with FP32
// accumulation (forward, gradient of the input, gradient of the weights), and
// the element-wise layers around them (average pooling, nearest upsampling,
// channel concatenation, ReLU masks, mean-squared error, Adam).
//
// Layouts: activations are NHWC (pixel-major, channels contiguous), BF16 as
// uint16 bit patterns or FP32; weights are [Cout][taps][Cin] with taps =
// ks*ks in row-major (ky, kx) order; their transpose for the input gradient is
// [Cin][taps][Cout].
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>

#include "inim.h"
#include "inim_nn.h"
#include "nn_plan.h"

namespace inim {
namespace nn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// Round to nearest even; NaN stays NaN.
__device__ __forceinline__ uint16_t f2bf(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x40u);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// ------------------------------------------------------------------ implicit GEMM
// C[m][n] = sum_k A[m][k] B[k][n] over one BM x BN block tile, K in steps of
// 32 staged through LDS as [row][k] for A and [col][k] for B, so that every
// lane reads its 8 consecutive k of one row (A) or one column (B) as one
// 16-byte LDS read.  Four waves of 32 x 32 x 16 BF16 MFMA tiles: 2 x 2 waves
// of 64 x 64 for the square 128 x 128 tile; for narrow outputs (N <= 64,
// where a 128-wide tile would leave most matrix-core columns idle) 4 x 1
// waves of 64 x BN over a 256-row tile.  MFMA lane layout (gfx950,
// 32x32x16): lane l holds A[l%32][8(l/32)+j] and B[8(l/32)+j][l%32] for j < 8;
// result register i of lane l is C[8(i/4) + 4(l/32) + i%4][l%32].
constexpr int kBK = 32, kPad = 8;

template <int BM, int BN>
struct Tile {
    static constexpr int wavesN = BN >= 128 ? 2 : 1, wavesM = 4 / wavesN;
    static constexpr int WM = BM / wavesM, WN = BN / wavesN;  // one wave's part
    static constexpr int TI = WM / 32, TJ = WN / 32;          // its MFMA tiles
    static constexpr int AC = BM * kBK / 8 / 256;             // A chunks per thread
    static constexpr int BC = (BN * kBK / 8 + 255) / 256;     // B chunks per thread (at most)
    static_assert(WM == 64 && WN % 32 == 0 && TJ >= 1, "tile shape");
};

template <int BM, int BN>
struct GemmLdsT {
    uint16_t a[BM][kBK + kPad];
    uint16_t b[BN][kBK + kPad];
};
using GemmLds = GemmLdsT<128, 128>;

// Element source of one operand: 8 consecutive k of row (A) or column (B) `r`.
// Conv geometry: pixel p = (img, y, x) of an H x W image, taps t = (ky, kx).
struct ConvGeom {
    int H, W, P;  // P = images * H * W
    int ks, taps, half;
    __device__ __forceinline__ bool shift(int p, int t, int sign, int& q) const {
        const int x = p % W, yy = p / W, y = yy % H;
        const int dy = (t / ks - half) * sign, dx = (t % ks - half) * sign;
        const int ny = y + dy, nx = x + dx;
        if (ny < 0 || ny >= H || nx < 0 || nx >= W) return false;
        q = p + dy * W + dx;
        return true;
    }
};

__device__ __forceinline__ u16x8 zero8() { return u16x8{0, 0, 0, 0, 0, 0, 0, 0}; }

// Forward: A[p][(t, ci)] = x[p + off_t][ci]; B[(t, ci)][co] = w[co][t][ci].
// Input gradient: A[q][(t, co)] = dy[q - off_t][co]; B[(t, co)][ci] = wT[ci][t][co].
// Both read 8 channels of one pixel (C % 8 == 0) as one 16-byte load.
struct RowShiftLoader {  // A of forward / input gradient
    const uint16_t* src;
    int C;      // channels of src
    int sign;   // +1 forward, -1 input gradient
    int M, K;   // K = taps * C
    ConvGeom g;
    __device__ __forceinline__ u16x8 load8(int m, int k) const {
        if (m >= M || k >= K) return zero8();
        const int t = k / C, c = k - t * C;
        int q;
        if (!g.shift(m, t, sign, q)) return zero8();
        return *reinterpret_cast<const u16x8*>(src + (size_t)q * C + c);
    }
};
struct WeightLoader {  // B of forward / input gradient: rows of [N][K] contiguous in k
    const uint16_t* w;
    int N, K;
    __device__ __forceinline__ u16x8 load8(int n, int k) const {
        if (n >= N || k >= K) return zero8();
        return *reinterpret_cast<const u16x8*>(w + (size_t)n * K + k);
    }
};

// One K step of 32 in flight: the 8-element chunks this thread moves, loaded
// from global memory into registers while the matrix cores work on the
// previous step, then written to LDS.
template <int AC, int BC>
struct ChunksT {
    u16x8 a[AC], b[BC];
};
using Chunks = ChunksT<2, 2>;

// BM rows x 32 k of A and BN rows x 32 k of B in chunks of 8 consecutive k:
// chunk e is row e / 4, k offset 8 (e % 4).
template <int BM, int BN, class LA, class LB>
__device__ __forceinline__ void load_vec(ChunksT<Tile<BM, BN>::AC, Tile<BM, BN>::BC>& c, const LA& la, const LB& lb,
                                         int bm, int bn, int k0) {
#pragma unroll
    for (int h = 0; h < Tile<BM, BN>::AC; ++h) {
        const int e = threadIdx.x + 256 * h;
        c.a[h] = la.load8(bm + (e >> 2), k0 + (e & 3) * 8);
    }
#pragma unroll
    for (int h = 0; h < Tile<BM, BN>::BC; ++h) {
        const int e = threadIdx.x + 256 * h;
        if (e < BN * 4) c.b[h] = lb.load8(bn + (e >> 2), k0 + (e & 3) * 8);
    }
}

template <int BM, int BN>
__device__ __forceinline__ void store_vec(const ChunksT<Tile<BM, BN>::AC, Tile<BM, BN>::BC>& c,
                                          GemmLdsT<BM, BN>& s) {
#pragma unroll
    for (int h = 0; h < Tile<BM, BN>::AC; ++h) {
        const int e = threadIdx.x + 256 * h;
        *reinterpret_cast<u16x8*>(&s.a[e >> 2][(e & 3) * 8]) = c.a[h];
    }
#pragma unroll
    for (int h = 0; h < Tile<BM, BN>::BC; ++h) {
        const int e = threadIdx.x + 256 * h;
        if (e < BN * 4) *reinterpret_cast<u16x8*>(&s.b[e >> 2][(e & 3) * 8]) = c.b[h];
    }
}

// Weight gradient: dW[co][(t, ci)] = sum_p dy[p][co] x[p + off_t][ci], i.e.
// A[co][p] = dy[p][co] and B[p][(t, ci)] = x[p + off_t][ci].  Each load is 8
// channels of one pixel (16 bytes; Cout and Cin multiples of 8, so a chunk of
// (t, ci) stays in one tap).  Eight consecutive lanes load the same 8
// channels of 8 consecutive pixels, transpose the 8 x 8 block among
// themselves (three lane exchanges), and each stores 8 pixels of one channel
// as one 16-byte row segment of the [row][k] LDS layout.
// With `ones`, column N of B is 1 at every pixel, so that column of the
// product is the bias gradient sum_p dy[p][co].
struct WgradSrc {
    const uint16_t* dy;  // [P][Cout]
    const uint16_t* x;   // [P][Cin]
    int Cout, Cin, N;    // N = taps * Cin
    bool ones;
    ConvGeom g;
};

// The value of lane (lane ^ J): DPP quad permutes for J = 1, 2, the swizzle
// xor mode for J = 4.  All 64 lanes take part.
template <int J>
__device__ __forceinline__ uint32_t xlane(uint32_t v) {
    if constexpr (J == 1) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);  // [1,0,3,2]
    else if constexpr (J == 2) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);  // [2,3,0,1]
    else return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1F | (J << 10));
}

// 8 x 8 transpose of 16-bit values among the 8 lanes of each aligned group:
// lane i ends with element i of lanes 0..7 of its group.  Each stage s = 4,
// 2, 1 swaps the elements whose index bit s differs from the lane's bit s
// with lane ^ s (which swaps those bits of lane and index).
__device__ __forceinline__ u16x8 transpose8(u16x8 v, int lane) {
    uint32_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = (uint32_t)v[2 * k] | ((uint32_t)v[2 * k + 1] << 16);
    const bool b4 = lane & 4, b2 = lane & 2, b1 = lane & 1;
    {
        const uint32_t y0 = xlane<4>(b4 ? w[0] : w[2]), y1 = xlane<4>(b4 ? w[1] : w[3]);
        if (b4) { w[0] = y0; w[1] = y1; } else { w[2] = y0; w[3] = y1; }
    }
    {
        const uint32_t y0 = xlane<2>(b2 ? w[0] : w[1]), y1 = xlane<2>(b2 ? w[2] : w[3]);
        if (b2) { w[0] = y0; w[2] = y1; } else { w[1] = y0; w[3] = y1; }
    }
    {
        const uint32_t s0 = b1 ? ((w[0] & 0xFFFFu) | (w[1] << 16)) : ((w[0] >> 16) | (w[1] & 0xFFFF0000u));
        const uint32_t s1 = b1 ? ((w[2] & 0xFFFFu) | (w[3] << 16)) : ((w[2] >> 16) | (w[3] & 0xFFFF0000u));
        const uint32_t r0 = xlane<1>(s0), r1 = xlane<1>(s1);
        if (b1) {
            w[0] = (w[0] & 0xFFFF0000u) | (r0 & 0xFFFFu);
            w[1] = (w[1] & 0xFFFF0000u) | (r0 >> 16);
            w[2] = (w[2] & 0xFFFF0000u) | (r1 & 0xFFFFu);
            w[3] = (w[3] & 0xFFFF0000u) | (r1 >> 16);
        } else {
            w[0] = (w[0] & 0xFFFFu) | (r0 << 16);
            w[1] = (w[1] & 0xFFFFu) | (r0 & 0xFFFF0000u);
            w[2] = (w[2] & 0xFFFFu) | (r1 << 16);
            w[3] = (w[3] & 0xFFFFu) | (r1 & 0xFFFF0000u);
        }
    }
    u16x8 o;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        o[2 * k] = (uint16_t)(w[k] & 0xFFFFu);
        o[2 * k + 1] = (uint16_t)(w[k] >> 16);
    }
    return o;
}

// Chunk e (0..511) of a K step: pixel kk = e % 8 + 8 ((e / 128) % 4) of the
// step's 32, rows 8 ((e / 8) % 16) .. + 7 of the tile; lanes 8g .. 8g+7 hold
// 8 consecutive pixels of the same rows.
__device__ __forceinline__ int wg_pixel(int e) { return (e & 7) | (((e >> 7) & 3) << 3); }
__device__ __forceinline__ int wg_rows(int e) { return ((e >> 3) & 15) * 8; }

__device__ __forceinline__ void load_wgrad(Chunks& c, const WgradSrc& w, int bm, int bn, int k0) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int e = threadIdx.x + 256 * h;
        const int kk = wg_pixel(e), rc = wg_rows(e);  // pixel k0 + kk; rows rc .. rc + 7 of the tile
        const int p = k0 + kk;
        const int co = bm + rc;
        c.a[h] = (p < w.g.P && co < w.Cout) ? *reinterpret_cast<const u16x8*>(w.dy + (size_t)p * w.Cout + co) : zero8();
        const int n = bn + rc;
        u16x8 v = zero8();
        if (p < w.g.P && n < w.N) {
            const int t = n / w.Cin, ci = n - t * w.Cin;
            int q;
            if (w.g.shift(p, t, 1, q)) v = *reinterpret_cast<const u16x8*>(w.x + (size_t)q * w.Cin + ci);
        } else if (w.ones && p < w.g.P && n == w.N) {
            v[0] = 0x3F80u;  // 1.0 in bfloat16
        }
        c.b[h] = v;
    }
}

__device__ __forceinline__ void store_wgrad(const Chunks& c, GemmLds& s) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int e = threadIdx.x + 256 * h;
        const int k8 = wg_pixel(e) & ~7, row = wg_rows(e) + (lane & 7);
        *reinterpret_cast<u16x8*>(&s.a[row][k8]) = transpose8(c.a[h], lane);
        *reinterpret_cast<u16x8*>(&s.b[row][k8]) = transpose8(c.b[h], lane);
    }
}

// The MFMA part of one K step of 32 for this wave's WM x WN.
template <int BM, int BN>
__device__ __forceinline__ void mma_step(const GemmLdsT<BM, BN>& s, f32x16 (&acc)[Tile<BM, BN>::TI][Tile<BM, BN>::TJ],
                                         int wm, int wn, int lane) {
    using T = Tile<BM, BN>;
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 16) {
        bf16x8 a[T::TI], b[T::TJ];
#pragma unroll
        for (int i = 0; i < T::TI; ++i) {
            const u16x8 va = *reinterpret_cast<const u16x8*>(&s.a[wm * T::WM + i * 32 + (lane & 31)][kk + 8 * (lane >> 5)]);
            a[i] = __builtin_bit_cast(bf16x8, va);
        }
#pragma unroll
        for (int j = 0; j < T::TJ; ++j) {
            const u16x8 vb = *reinterpret_cast<const u16x8*>(&s.b[wn * T::WN + j * 32 + (lane & 31)][kk + 8 * (lane >> 5)]);
            b[j] = __builtin_bit_cast(bf16x8, vb);
        }
#pragma unroll
        for (int i = 0; i < T::TI; ++i)
#pragma unroll
            for (int j = 0; j < T::TJ; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
}

// The K loop over [kbeg, kend) with two LDS buffers: the global loads of
// step i+1 are issued before the MFMAs of step i and written to the other
// buffer after them; one barrier per step.  s points to the two buffers; C is
// the chunk type the load and store callbacks move.
template <int BM, int BN, class C, class Load, class Store>
__device__ __forceinline__ void gemm_loop(GemmLdsT<BM, BN>* s, f32x16 (&acc)[Tile<BM, BN>::TI][Tile<BM, BN>::TJ],
                                          int kbeg, int kend, Load load, Store store) {
    using T = Tile<BM, BN>;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, wm = wave / T::wavesN, wn = wave % T::wavesN;
    C c;
    if (kbeg >= kend) return;
    load(c, kbeg);
    store(c, s[0]);
    __syncthreads();
    int cur = 0;
    for (int k0 = kbeg; k0 < kend; k0 += kBK) {
        const bool more = k0 + kBK < kend;
        if (more) load(c, k0 + kBK);
        mma_step<BM, BN>(s[cur], acc, wm, wn, lane);
        if (more) store(c, s[cur ^ 1]);
        __syncthreads();
        cur ^= 1;
    }
}

// Epilogue over this wave's results: f(m, n, value).
template <int BM, int BN, class F>
__device__ __forceinline__ void for_each_result(const f32x16 (&acc)[Tile<BM, BN>::TI][Tile<BM, BN>::TJ], int bm,
                                                int bn, F f) {
    using T = Tile<BM, BN>;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, wm = wave / T::wavesN, wn = wave % T::wavesN;
#pragma unroll
    for (int i = 0; i < T::TI; ++i)
#pragma unroll
        for (int j = 0; j < T::TJ; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int m = bm + wm * T::WM + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int n = bn + wn * T::WN + j * 32 + (lane & 31);
                f(m, n, acc[i][j][r]);
            }
}

// K range of split slice z (slices of `kslice`, a multiple of 32).
__device__ __forceinline__ void k_range(int K, int kslice, int& kbeg, int& kend) {
    kbeg = blockIdx.z * kslice;
    kend = min(K, kbeg + kslice);
}

// Forward convolution.  With gridDim.z == 1 the epilogue writes
// y = act(b + sum x w) as BF16 (y16) and/or FP32 (y32); with gridDim.z > 1
// slice z of the K range writes its FP32 partial sums to part[z][p][co] and
// k_conv_finish completes the layer.
template <int BM, int BN>
__global__ __launch_bounds__(256) void k_conv_fwd(ConvArgs a, int kslice, float* part) {
    using T = Tile<BM, BN>;
    using C = ChunksT<T::AC, T::BC>;
    __shared__ GemmLdsT<BM, BN> s[2];
    const int bm = blockIdx.x * BM, bn = blockIdx.y * BN;
    const ConvGeom g{a.H, a.W, a.P, a.ks, a.ks * a.ks, a.ks / 2};
    const int K = g.taps * a.Cin;
    const RowShiftLoader la{a.x, a.Cin, 1, a.P, K, g};
    const WeightLoader lb{a.w, a.Cout, K};
    int kbeg, kend;
    k_range(K, kslice, kbeg, kend);
    f32x16 acc[T::TI][T::TJ] = {};
    gemm_loop<BM, BN, C>(s, acc, kbeg, kend, [&](C& c, int k0) { load_vec<BM, BN>(c, la, lb, bm, bn, k0); },
                         [&](const C& c, GemmLdsT<BM, BN>& l) { store_vec<BM, BN>(c, l); });
    if (gridDim.z > 1) {
        float* out = part + (size_t)blockIdx.z * a.P * a.Cout;
        for_each_result<BM, BN>(acc, bm, bn, [&](int m, int n, float v) {
            if (m < a.P && n < a.Cout) out[(size_t)m * a.Cout + n] = v;
        });
        return;
    }
    for_each_result<BM, BN>(acc, bm, bn, [&](int m, int n, float v) {
        if (m >= a.P || n >= a.Cout) return;
        v += a.bias ? a.bias[n] : 0.0f;
        if (a.relu) v = v > 0.0f ? v : 0.0f;
        const size_t o = (size_t)m * a.Cout + n;
        if (a.y16) a.y16[o] = f2bf(v);
        if (a.y32) a.y32[o] = v;
    });
}

// Completion of a split forward convolution: sum of the slices in order,
// bias, ReLU, stores.
__global__ __launch_bounds__(256) void k_conv_finish(ConvArgs a, int slices, const float* __restrict__ part) {
    const size_t n = (size_t)a.P * a.Cout;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        float v = 0.0f;
        for (int z = 0; z < slices; ++z) v += part[(size_t)z * n + i];
        v += a.bias ? a.bias[i % a.Cout] : 0.0f;
        if (a.relu) v = v > 0.0f ? v : 0.0f;
        if (a.y16) a.y16[i] = f2bf(v);
        if (a.y32) a.y32[i] = v;
    }
}

// Input gradient: dx[q][ci] = sum_{t, co} dy[q - off_t][co] wT[ci][t][co],
// FP32; split slices write part[z] and k_sum_parts adds them.
template <int BM, int BN>
__global__ __launch_bounds__(256) void k_conv_dgrad(ConvArgs a, int kslice, float* part) {
    using T = Tile<BM, BN>;
    using C = ChunksT<T::AC, T::BC>;
    __shared__ GemmLdsT<BM, BN> s[2];
    const int bm = blockIdx.x * BM, bn = blockIdx.y * BN;
    const ConvGeom g{a.H, a.W, a.P, a.ks, a.ks * a.ks, a.ks / 2};
    const int K = g.taps * a.Cout;
    const RowShiftLoader la{a.dy, a.Cout, -1, a.P, K, g};
    const WeightLoader lb{a.wT, a.Cin, K};
    int kbeg, kend;
    k_range(K, kslice, kbeg, kend);
    f32x16 acc[T::TI][T::TJ] = {};
    gemm_loop<BM, BN, C>(s, acc, kbeg, kend, [&](C& c, int k0) { load_vec<BM, BN>(c, la, lb, bm, bn, k0); },
                         [&](const C& c, GemmLdsT<BM, BN>& l) { store_vec<BM, BN>(c, l); });
    float* out = gridDim.z > 1 ? part + (size_t)blockIdx.z * a.P * a.Cin : a.dx;
    for_each_result<BM, BN>(acc, bm, bn, [&](int m, int n, float v) {
        if (m < a.P && n < a.Cin) out[(size_t)m * a.Cin + n] = v;
    });
}

// Weight gradient, FP32 [Cout][taps][Cin]; K (pixels) split over gridDim.z
// slices of `kslice` pixels, each slice writing its own partial [slice][...];
// with bias_part != null, also the bias-gradient partials [slice][Cout]
// (the column of ones).
__global__ __launch_bounds__(256) void k_conv_wgrad(ConvArgs a, int kslice, float* bias_part) {
    __shared__ GemmLds s[2];
    const int bm = blockIdx.x * 128, bn = blockIdx.y * 128;
    const ConvGeom g{a.H, a.W, a.P, a.ks, a.ks * a.ks, a.ks / 2};
    const int N = g.taps * a.Cin;
    const WgradSrc src{a.dy, a.x, a.Cout, a.Cin, N, bias_part != nullptr, g};
    int kbeg, kend;
    k_range(a.P, kslice, kbeg, kend);
    f32x16 acc[2][2] = {};
    gemm_loop<128, 128, Chunks>(s, acc, kbeg, kend, [&](Chunks& c, int k0) { load_wgrad(c, src, bm, bn, k0); },
                                [&](const Chunks& c, GemmLds& l) { store_wgrad(c, l); });
    float* out = a.dw + (size_t)blockIdx.z * a.Cout * N;
    for_each_result<128, 128>(acc, bm, bn, [&](int m, int n, float v) {
        if (m >= a.Cout) return;
        if (n < N) out[(size_t)m * N + n] = v;
        else if (n == N && bias_part) bias_part[(size_t)blockIdx.z * a.Cout + m] = v;
    });
}

// Channel-major copies for the weight gradient: out[c][p] = in[p][c] for two
// tensors of the same pixels in one launch (blockIdx.y below the first
// tensor's channel blocks: the first), one block per 64 pixels x 64 channels
// through LDS (C and P multiples of 8).  Loads: 8 lanes read 64 channels (128
// contiguous bytes) of one pixel; stores: 8 lanes write 64 pixels of one
// channel.
struct CmajorSeg {
    const uint16_t* in;  // [P][C]
    int C;
    uint16_t* out;       // [C][P]
};

__global__ __launch_bounds__(256) void k_cmajor(CmajorSeg s0, CmajorSeg s1, int64_t P) {
    __shared__ uint16_t t[64][64 + kPad];
    const int cb0 = (s0.C + 63) / 64;
    const bool first = (int)blockIdx.y < cb0;
    const uint16_t* __restrict__ in = first ? s0.in : s1.in;
    uint16_t* __restrict__ out = first ? s0.out : s1.out;
    const int C = first ? s0.C : s1.C;
    const int64_t p0 = (int64_t)blockIdx.x * 64;
    const int c0 = (first ? (int)blockIdx.y : (int)blockIdx.y - cb0) * 64;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int e = threadIdx.x + 256 * h;
        const int cc = (e & 7) * 8, px = e >> 3;
        if (p0 + px < P && c0 + cc < C) {
            const u16x8 v = *reinterpret_cast<const u16x8*>(in + (size_t)(p0 + px) * C + c0 + cc);
#pragma unroll
            for (int j = 0; j < 8; ++j) t[cc + j][px] = v[j];
        }
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int e = threadIdx.x + 256 * h;
        const int pp = (e & 7) * 8, c = e >> 3;
        if (c0 + c < C && p0 + pp < P)
            *reinterpret_cast<u16x8*>(out + (size_t)(c0 + c) * P + p0 + pp) = *reinterpret_cast<const u16x8*>(&t[c][pp]);
    }
}

// Weight gradient from channel-major operands dyT [Cout][P] and xT [Cin][P]
// (images with power-of-two sides, W a multiple of 8): every 8-element chunk
// of a K step is 8 consecutive pixels of one image row, so A and B chunks are
// plain 16-byte loads stored to LDS as they are, with no lane transposes.
// A tap's column shift kx = +-1 moves the chunk by one element: the
// neighbouring chunk of the same row supplies the element that enters (zero
// past the row's end).  The K order (pixel k0 + k at LDS column k) is that of
// k_conv_wgrad, so both give the same sums.
// Without SWAP the block tile is Cout rows (A = dyT) by (tap, ci) columns
// (B = xT); with SWAP (narrow Cout) it is (tap, ci) rows (A = xT) by Cout
// columns (B = dyT) on a 256 x BN tile, so that a 32- or 64-channel layer
// does not leave three quarters of a 128-row tile empty.
struct WgradRow {
    const uint16_t* src;  // dyT or xT row
    int ky, kx;
    int kind;             // 0 zero, 1 plain, 2 tap-shifted, 3 the column of ones
};

__device__ __forceinline__ u16x8 ones8() {
    const uint16_t o = 0x3F80u;  // 1.0 in bfloat16
    return u16x8{o, o, o, o, o, o, o, o};
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ u16x8 shifted8(const uint16_t* row, int p, int ky, int kx, int wlog, int wmask,
                                          int hmask) {
    const int x = p & wmask, y = (p >> wlog) & hmask;
    const int ny = y + ky;
    if (ny < 0 || ny > hmask) return zero8();
    const uint16_t* src = row + p + ky * (wmask + 1);
    const u32x4 v = __builtin_bit_cast(u32x4, *reinterpret_cast<const u16x8*>(src));
    if (kx == 0) return __builtin_bit_cast(u16x8, v);
    u32x4 o;
    if (kx > 0) {  // element j is pixel j + 1; the last enters from the next chunk
        const uint32_t nb = x + 8 <= wmask ? *reinterpret_cast<const uint32_t*>(src + 8) : 0u;
        o[0] = (v[0] >> 16) | (v[1] << 16);
        o[1] = (v[1] >> 16) | (v[2] << 16);
        o[2] = (v[2] >> 16) | (v[3] << 16);
        o[3] = (v[3] >> 16) | (nb << 16);
    } else {  // element j is pixel j - 1; the first enters from the previous chunk
        const uint32_t pb = x > 0 ? *reinterpret_cast<const uint32_t*>(src - 2) : 0u;
        o[0] = (pb >> 16) | (v[0] << 16);
        o[1] = (v[0] >> 16) | (v[1] << 16);
        o[2] = (v[1] >> 16) | (v[2] << 16);
        o[3] = (v[2] >> 16) | (v[3] << 16);
    }
    return __builtin_bit_cast(u16x8, o);
}

struct WgradGeo {
    int wlog, wmask, hmask;
};

__device__ __forceinline__ u16x8 wgrad_chunk(const WgradRow& r, int p, bool in, const WgradGeo& g) {
    if (!in || r.kind == 0) return zero8();
    if (r.kind == 1) return *reinterpret_cast<const u16x8*>(r.src + p);
    if (r.kind == 2) return shifted8(r.src, p, r.ky, r.kx, g.wlog, g.wmask, g.hmask);
    return ones8();
}

// Row n of the (tap, ci) side: a tap-shifted xT row, the column of ones, or zero.
__device__ __forceinline__ WgradRow xrow(const ConvArgs& a, const uint16_t* xT, int n, int N, bool ones) {
    WgradRow r{xT, 0, 0, 0};
    if (n < N) {
        const int t = n / a.Cin, ci = n - t * a.Cin, half = a.ks / 2;
        r.src = xT + (size_t)ci * a.P;
        r.ky = t / a.ks - half;
        r.kx = t % a.ks - half;
        r.kind = a.ks == 1 ? 1 : 2;
    } else if (ones && n == N) {
        r.kind = 3;
    }
    return r;
}

__device__ __forceinline__ WgradRow dyrow(const ConvArgs& a, const uint16_t* dyT, int co) {
    return WgradRow{co < a.Cout ? dyT + (size_t)co * a.P : dyT, 0, 0, co < a.Cout ? 1 : 0};
}

template <int BM, int BN, bool SWAP>
__global__ __launch_bounds__(256) void k_conv_wgrad_t(ConvArgs a, const uint16_t* __restrict__ dyT,
                                                      const uint16_t* __restrict__ xT, int wlog, int kslice,
                                                      float* bias_part) {
    using T = Tile<BM, BN>;
    using C = ChunksT<T::AC, T::BC>;
    __shared__ GemmLdsT<BM, BN> s[2];
    const int bm = blockIdx.x * BM, bn = blockIdx.y * BN;
    const int N = a.ks * a.ks * a.Cin;
    const bool ones = bias_part != nullptr;
    const WgradGeo geo{wlog, a.W - 1, a.H - 1};
    WgradRow ra[T::AC], rb[T::BC];
#pragma unroll
    for (int h = 0; h < T::AC; ++h) {
        const int row = bm + (int)(threadIdx.x >> 2) + 64 * h;
        ra[h] = SWAP ? xrow(a, xT, row, N, ones) : dyrow(a, dyT, row);
    }
#pragma unroll
    for (int h = 0; h < T::BC; ++h) {
        const int e = threadIdx.x + 256 * h;
        const int row = bn + (e >> 2);
        rb[h] = e < BN * 4 ? (SWAP ? dyrow(a, dyT, row) : xrow(a, xT, row, N, ones)) : WgradRow{xT, 0, 0, 0};
    }
    int kbeg, kend;
    k_range(a.P, kslice, kbeg, kend);
    f32x16 acc[T::TI][T::TJ] = {};
    gemm_loop<BM, BN, C>(
        s, acc, kbeg, kend,
        [&](C& c, int k0) {
            const int p = k0 + (int)(threadIdx.x & 3) * 8;
            const bool in = p < kend;
#pragma unroll
            for (int h = 0; h < T::AC; ++h) c.a[h] = wgrad_chunk(ra[h], p, in, geo);
#pragma unroll
            for (int h = 0; h < T::BC; ++h) c.b[h] = wgrad_chunk(rb[h], p, in, geo);
        },
        [&](const C& c, GemmLdsT<BM, BN>& l) { store_vec<BM, BN>(c, l); });
    float* out = a.dw + (size_t)blockIdx.z * a.Cout * N;
    for_each_result<BM, BN>(acc, bm, bn, [&](int m, int n, float v) {
        const int co = SWAP ? n : m, k = SWAP ? m : n;
        if (co >= a.Cout) return;
        if (k < N) out[(size_t)co * N + k] = v;
        else if (k == N && bias_part) bias_part[(size_t)blockIdx.z * a.Cout + co] = v;
    });
}

// Sums of split partials, out[i] = sum over q of part[q][i], for one or two
// arrays (the weight and bias gradients) in one launch.  A block takes 64
// consecutive elements, one per lane; its four waves sum consecutive quarters
// of the parts in order (eight loads in flight), and the quarters are added
// in order through LDS, so the result does not depend on timing.
struct SumSeg {
    const float* part;  // [parts][len]
    size_t len;
    float* out;
};

__global__ __launch_bounds__(256) void k_sum_parts(SumSeg s0, SumSeg s1, int parts) {
    __shared__ float qs[4][64];
    const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
    const size_t blocks0 = (s0.len + 63) / 64, blocks = blocks0 + (s1.len + 63) / 64;
    const int per = (parts + 3) / 4;
    const int q0 = min(parts, wave * per), q1 = min(parts, q0 + per);
    for (size_t blk = blockIdx.x; blk < blocks; blk += gridDim.x) {
        const bool first = blk < blocks0;
        const float* __restrict__ part = first ? s0.part : s1.part;
        const size_t len = first ? s0.len : s1.len;
        const size_t i = (first ? blk : blk - blocks0) * 64 + lane;
        float acc = 0.0f;
        if (i < len) {
            int q = q0;
            for (; q + 8 <= q1; q += 8) {
                float v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(q + u) * len + i];
#pragma unroll
                for (int u = 0; u < 8; ++u) acc += v[u];
            }
            for (; q < q1; ++q) acc += part[(size_t)q * len + i];
        }
        qs[wave][lane] = acc;
        __syncthreads();
        if (wave == 0 && i < len) (first ? s0.out : s1.out)[i] = ((qs[0][lane] + qs[1][lane]) + qs[2][lane]) + qs[3][lane];
        __syncthreads();
    }
}

// The same sums one element per thread, the parts in order (for few parts or
// long arrays).
__global__ __launch_bounds__(256) void k_sum_parts_flat(SumSeg s0, SumSeg s1, int parts) {
    const size_t len = s0.len + s1.len;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < len; t += (size_t)gridDim.x * blockDim.x) {
        const bool first = t < s0.len;
        const float* __restrict__ part = first ? s0.part : s1.part;
        const size_t n = first ? s0.len : s1.len, i = first ? t : t - s0.len;
        float acc = 0.0f;
        int q = 0;
        for (; q + 8 <= parts; q += 8) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(q + u) * n + i];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += v[u];
        }
        for (; q < parts; ++q) acc += part[(size_t)q * n + i];
        (first ? s0.out : s1.out)[i] = acc;
    }
}

// wT[ci][t][co] = w[co][t][ci]
__global__ __launch_bounds__(256) void k_wtrans(const uint16_t* __restrict__ w, int Cout, int taps, int Cin,
                                                uint16_t* __restrict__ wT) {
    const size_t n = (size_t)Cout * taps * Cin;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int ci = (int)(i % Cin);
        const size_t r = i / Cin;
        const int t = (int)(r % taps), co = (int)(r / taps);
        wT[((size_t)ci * taps + t) * Cout + co] = w[i];
    }
}

// ------------------------------------------------------------------ element-wise layers
__global__ __launch_bounds__(256) void k_f32_to_bf16(const float* __restrict__ a, size_t n, uint16_t* __restrict__ b) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        b[i] = f2bf(a[i]);
}

// 2x2 average pooling, NHWC: y[img][y][x][c] of an (H/2) x (W/2) image.
__global__ __launch_bounds__(256) void k_pool2(const uint16_t* __restrict__ x, int imgs, int H, int W, int C,
                                               uint16_t* __restrict__ y) {
    const int h = H / 2, w = W / 2;
    const size_t n = (size_t)imgs * h * w * C;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        size_t r = i / C;
        const int xx = (int)(r % w);
        r /= w;
        const int yy = (int)(r % h);
        const size_t img = r / h;
        const size_t b = ((img * H + 2 * yy) * W + 2 * xx) * C + c;
        const float s = bf2f(x[b]) + bf2f(x[b + C]) + bf2f(x[b + (size_t)W * C]) + bf2f(x[b + (size_t)W * C + C]);
        y[i] = f2bf(0.25f * s);
    }
}

// Gradient of the pooling: dx[img][y][x][c] = dy[img][y/2][x/2][c] / 4, added
// to dx (FP32) when accumulate != 0.
__global__ __launch_bounds__(256) void k_pool2_back(const float* __restrict__ dy, int imgs, int H, int W, int C,
                                                    float* __restrict__ dx, int accumulate) {
    const size_t n = (size_t)imgs * H * W * C;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        size_t r = i / C;
        const int xx = (int)(r % W);
        r /= W;
        const int yy = (int)(r % H);
        const size_t img = r / H;
        const float v = 0.25f * dy[((img * (H / 2) + yy / 2) * (W / 2) + xx / 2) * C + c];
        dx[i] = accumulate ? dx[i] + v : v;
    }
}

// Nearest 2x upsampling into channels [c0, c0 + C) of a Ct-channel tensor:
// y[img][y][x][c0 + c] = x[img][y/2][x/2][c] (x is h x w, y is 2h x 2w).
__global__ __launch_bounds__(256) void k_up2_into(const uint16_t* __restrict__ x, int imgs, int h, int w, int C,
                                                  uint16_t* __restrict__ y, int Ct, int c0) {
    const size_t n = (size_t)imgs * 4 * h * w * C;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        size_t r = i / C;
        const int xx = (int)(r % (2 * w));
        r /= 2 * w;
        const int yy = (int)(r % (2 * h));
        const size_t img = r / (2 * h);
        y[((img * 2 * h + yy) * 2 * w + xx) * Ct + c0 + c] = x[((img * h + yy / 2) * w + xx / 2) * C + c];
    }
}

// Copy into channels [c0, c0 + C) of a Ct-channel tensor (the skip half of a concatenation).
__global__ __launch_bounds__(256) void k_copy_into(const uint16_t* __restrict__ x, size_t pixels, int C,
                                                   uint16_t* __restrict__ y, int Ct, int c0) {
    const size_t n = pixels * C;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const size_t p = i / C;
        y[p * Ct + c0 + (i - p * C)] = x[i];
    }
}

// The concatenation [up(a) | b] in one pass over its elements: channels
// [0, Ca) from the 2 x 2 upsampled a (imgs x h x w x Ca), [Ca, Ca + Cb) from b
// (imgs x 2h x 2w x Cb).
__global__ __launch_bounds__(256) void k_concat_up2(const uint16_t* __restrict__ a, int imgs, int h, int w, int Ca,
                                                    const uint16_t* __restrict__ b, int Cb, uint16_t* __restrict__ y) {
    const int Ct = Ca + Cb;
    const size_t n = (size_t)imgs * 4 * h * w * Ct;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % Ct);
        const size_t p = i / Ct;  // output pixel
        if (c >= Ca) {
            y[i] = b[p * Cb + (c - Ca)];
        } else {
            const int xx = (int)(p % (2 * w));
            const size_t r = p / (2 * w);
            const int yy = (int)(r % (2 * h));
            const size_t img = r / (2 * h);
            y[i] = a[((img * h + yy / 2) * w + xx / 2) * Ca + c];
        }
    }
}

// Gradients through a concatenation [up(a) | b]: da[img][y][x][c] = sum of
// the 2 x 2 block of dy[...][c] (channels [0, Ca)); db (channels [Ca, Ca+Cb))
// is added to db_acc (FP32) when accumulate != 0, else stored.
__global__ __launch_bounds__(256) void k_up2_back(const float* __restrict__ dy, int imgs, int h, int w, int Ct,
                                                  int Ca, float* __restrict__ da) {
    const size_t n = (size_t)imgs * h * w * Ca;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % Ca);
        size_t r = i / Ca;
        const int xx = (int)(r % w);
        r /= w;
        const int yy = (int)(r % h);
        const size_t img = r / h;
        const size_t b = ((img * 2 * h + 2 * yy) * 2 * w + 2 * xx) * Ct + c;
        const size_t row = (size_t)2 * w * Ct;
        da[i] = dy[b] + dy[b + Ct] + dy[b + row] + dy[b + row + Ct];
    }
}

__global__ __launch_bounds__(256) void k_take_channels(const float* __restrict__ dy, size_t pixels, int Ct, int c0,
                                                       int C, float* __restrict__ out, int accumulate) {
    const size_t n = pixels * C;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const size_t p = i / C;
        const float v = dy[p * Ct + c0 + (i - p * C)];
        out[i] = accumulate ? out[i] + v : v;
    }
}

// ReLU gradient and BF16 cast: g16[i] = bf16(g[i] * (act[i] > 0)) (act = the
// layer's ReLU output); act == nullptr: no mask.
__global__ __launch_bounds__(256) void k_relu_back(const float* __restrict__ g, const uint16_t* __restrict__ act, size_t n,
                                                   uint16_t* __restrict__ g16) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        float v = g[i];
        if (act && !(bf2f(act[i]) > 0.0f)) v = 0.0f;
        g16[i] = f2bf(v);
    }
}

// Mean-squared error of the first Ct of Cp predicted channels against the
// target [P][Ct]: loss_part[block] = sum of (pred - target)^2 over the
// block's elements; grad[p][c] = 2 (pred - target) / (P Ct) as BF16 for
// c < Ct and 0 for the other channels (grad may be null).
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ pred, int Cp, const float* __restrict__ target,
                                             int Ct, size_t P, float* __restrict__ loss_part,
                                             uint16_t* __restrict__ grad) {
    __shared__ float red[256];
    float s = 0.0f;
    const size_t n = P * Cp;
    const float sc = 2.0f / (float)(P * Ct);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const size_t p = i / Cp;
        const int c = (int)(i - p * Cp);
        float d = 0.0f;
        if (c < Ct) d = pred[i] - target[p * Ct + c];
        s += d * d;
        if (grad) grad[i] = f2bf(sc * d);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// Adam (bias-corrected) on FP32 master weights; also writes their BF16 copy.
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, size_t n, AdamArgs a, uint16_t* __restrict__ w16) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = a.b1 * m[i] + (1.0f - a.b1) * gi;
        const float vi = a.b2 * v[i] + (1.0f - a.b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float wi = w[i] - a.lr * (mi * a.c1) / (sqrtf(vi * a.c2) + a.eps);
        w[i] = wi;
        if (w16) w16[i] = f2bf(wi);
    }
}

// ------------------------------------------------------------------ surrogate input, target and output
// Network input: channel 0 = density * scale (the density relative to its
// mean), channels 1..C-1 = 0.
__global__ __launch_bounds__(256) void k_pack_density(const float* __restrict__ d, size_t pixels, float scale, int C,
                                                      uint16_t* __restrict__ x) {
    const size_t n = pixels * C;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const size_t p = i / C;
        x[i] = (i - p * C) == 0 ? f2bf(d[p] * scale) : (uint16_t)0;
    }
}

// The same for a stack of rasters, raster z (blockIdx.y) with scale[z].
constexpr int kMaxScales = 64;
struct Scales {
    float v[kMaxScales];
};

// Density in channel 0 and, from a deformation field f (texel positions,
// [z][res][res][2]), its displacement from the texel centres times 64 in
// channels 1 and 2; other channels 0.  Raster z = blockIdx.y.
__global__ __launch_bounds__(256) void k_pack_input_many(const float* __restrict__ d, const float* __restrict__ f,
                                                         int res, Scales sc, int C, uint16_t* __restrict__ x) {
    const size_t px = (size_t)res * res, n = px * C, z = blockIdx.y;
    const float* dz = d + z * px;
    const float* fz = f + z * px * 2;
    uint16_t* xz = x + z * n;
    const float inv = 1.0f / (float)res;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const size_t p = i / C;
        const int c = (int)(i - p * C);
        float v = 0.0f;
        if (c == 0) {
            v = dz[p] * sc.v[z];
        } else if (c <= 2) {
            const int ix = (int)(p % res), iy = (int)(p / res);
            const float centre = ((c == 1 ? ix : iy) + 0.5f) * inv;
            v = (fz[2 * p + (c - 1)] - centre) * 64.0f;
        }
        xz[i] = c <= 2 ? f2bf(v) : (uint16_t)0;
    }
}

__global__ __launch_bounds__(256) void k_pack_density_many(const float* __restrict__ d, size_t pixels, Scales sc,
                                                           int C, uint16_t* __restrict__ x) {
    const int z = blockIdx.y;
    const float scale = sc.v[z];
    d += (size_t)z * pixels;
    x += (size_t)z * pixels * C;
    const size_t n = pixels * C;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const size_t p = i / C;
        x[i] = (i - p * C) == 0 ? f2bf(d[p] * scale) : (uint16_t)0;
    }
}

// Displacements are expressed in units of 1/64 of the unit square, so that
// targets of every raster size have the same scale.
constexpr float kDispUnit = 64.0f;

// Training target: out[p][c] = (probe[p][c] - texel centre) * 64, p = j N + i.
__global__ __launch_bounds__(256) void k_displacement(const float2* __restrict__ probe, int N, float* __restrict__ out) {
    const size_t n = (size_t)N * N;
    for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (size_t)gridDim.x * blockDim.x) {
        const int j = (int)(p / N), i = (int)(p - (size_t)j * N);
        const float2 q = probe[p];
        out[2 * p] = (q.x - ((float)i + 0.5f) / (float)N) * kDispUnit;
        out[2 * p + 1] = (q.y - ((float)j + 0.5f) / (float)N) * kDispUnit;
    }
}

// The deformation field of the network's output: field[p] = texel centre +
// (smoothed output[p][0..1]) / 64, the output convolved along x, then along
// y, with the normalised taps w[0..2r] (indices clamped at the border); the
// x pass goes to tmp [N][N][2].  Channels beyond the first two are ignored.
// blockIdx.y selects the output of a stack (y [N][N][C], tmp and field
// [N][N][2] per output).
struct FieldTaps {
    int r;
    float w[33];
};

__global__ __launch_bounds__(256) void k_field_smooth_x(const float* __restrict__ y, int C, int N, FieldTaps t,
                                                        float2* __restrict__ tmp) {
    const size_t n = (size_t)N * N;
    y += (size_t)blockIdx.y * n * C;
    tmp += (size_t)blockIdx.y * n;
    for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (size_t)gridDim.x * blockDim.x) {
        const int j = (int)(p / N), i = (int)(p - (size_t)j * N);
        float ax = 0.0f, ay = 0.0f;
        for (int d = -t.r; d <= t.r; ++d) {
            const size_t q = ((size_t)j * N + min(max(i + d, 0), N - 1)) * C;
            ax += t.w[d + t.r] * y[q];
            ay += t.w[d + t.r] * y[q + 1];
        }
        tmp[p] = make_float2(ax, ay);
    }
}

__global__ __launch_bounds__(256) void k_field_smooth_y(const float2* __restrict__ tmp, int N, FieldTaps t,
                                                        float2* __restrict__ field) {
    const size_t n = (size_t)N * N;
    tmp += (size_t)blockIdx.y * n;
    field += (size_t)blockIdx.y * n;
    for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (size_t)gridDim.x * blockDim.x) {
        const int j = (int)(p / N), i = (int)(p - (size_t)j * N);
        float ax = 0.0f, ay = 0.0f;
        for (int d = -t.r; d <= t.r; ++d) {
            const float2 v = tmp[(size_t)min(max(j + d, 0), N - 1) * N + i];
            ax += t.w[d + t.r] * v.x;
            ay += t.w[d + t.r] * v.y;
        }
        field[p] = make_float2(((float)i + 0.5f) / (float)N + ax / kDispUnit, ((float)j + 0.5f) / (float)N + ay / kDispUnit);
    }
}

// Orientation check of a deformed lattice (field[j][i] = image of texel
// centre (i, j)): counts the triangles (two per cell) whose signed area is not
// positive, i.e. folds.  One atomic add per block.
__global__ __launch_bounds__(256) void k_count_folds(const float2* __restrict__ f, int N, unsigned* __restrict__ count) {
    __shared__ unsigned red[256];
    unsigned c = 0;
    const size_t cells = (size_t)(N - 1) * (N - 1);
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < cells; k += (size_t)gridDim.x * blockDim.x) {
        const int j = (int)(k / (N - 1)), i = (int)(k - (size_t)j * (N - 1));
        const float2 a = f[(size_t)j * N + i], b = f[(size_t)j * N + i + 1];
        const float2 cc = f[(size_t)(j + 1) * N + i], d = f[(size_t)(j + 1) * N + i + 1];
        const double c1 = ((double)b.x - a.x) * ((double)cc.y - a.y) - ((double)b.y - a.y) * ((double)cc.x - a.x);
        const double c2 = ((double)cc.x - d.x) * ((double)b.y - d.y) - ((double)cc.y - d.y) * ((double)b.x - d.x);
        c += (c1 <= 0.0) + (c2 <= 0.0);
    }
    red[threadIdx.x] = c;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0]) atomicAdd(count, red[0]);
}

// Sums of the counts of bin x bin texel blocks and of their squares (for the
// standard deviation of the per-bin counts), as two doubles.  One atomic pair
// per block.
__global__ __launch_bounds__(256) void k_bin_moments(const uint32_t* __restrict__ counts, int N, int bin,
                                                     double* __restrict__ out) {
    __shared__ double r1[256], r2[256];
    const int nb = N / bin;
    double s1 = 0.0, s2 = 0.0;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nb * nb; k += gridDim.x * blockDim.x) {
        const int by = k / nb, bx = k - by * nb;
        double s = 0.0;
        for (int y = 0; y < bin; ++y)
            for (int x = 0; x < bin; ++x) s += counts[(size_t)(by * bin + y) * N + bx * bin + x];
        s1 += s;
        s2 += s * s;
    }
    r1[threadIdx.x] = s1;
    r2[threadIdx.x] = s2;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            r1[threadIdx.x] += r1[threadIdx.x + o];
            r2[threadIdx.x] += r2[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicAdd(out, r1[0]);
        atomicAdd(out + 1, r2[0]);
    }
}

}  // namespace nn
}  // namespace inim

// ------------------------------------------------------------------ C ABI (inim_nn.h)
using namespace inim::nn;

namespace {

thread_local std::string g_nn_error;

int nfail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int nfail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_nn_error = buf;
    return code;
}

int launched(const char* what) {
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? INIM_OK : nfail(INIM_EHIP, "%s: %s", what, hipGetErrorString(e));
}

unsigned grid_1d(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    return (unsigned)(g > 8192 ? 8192 : g);
}

constexpr int kTile = 128, kStepK = 32, kMsePartials = 256;

int check_conv(int32_t imgs, int32_t h, int32_t w, int32_t cin, int32_t cout, int32_t ks) {
    if (imgs < 1 || h < 1 || w < 1) return nfail(INIM_EINVAL, "empty image batch %d x %d x %d", imgs, h, w);
    if ((int64_t)imgs * h * w >= ((int64_t)1 << 31)) return nfail(INIM_ERANGE, "too many pixels");
    if (ks != 1 && ks != 3) return nfail(INIM_EINVAL, "kernel size %d is not 1 or 3", ks);
    if (cin < 8 || cin % 8 || cout < 8 || cout % 8)
        return nfail(INIM_EINVAL, "channels %d -> %d must be positive multiples of 8", cin, cout);
    return INIM_OK;
}

// Slices of a K range of `klen` for an M x N tile grid: enough blocks to
// fill the chip (512), each slice at least 4 steps of 32.
// Block tile of a forward or input-gradient GEMM with n output columns:
// 256 x 32 or 256 x 64 when the outputs are that narrow, else 128 x 128.
struct TileShape {
    int bm, bn;
};
TileShape conv_tile(int64_t n) {
    if (n <= 32) return {256, 32};
    if (n <= 64) return {256, 64};
    return {kTile, kTile};
}

int split_slices(int64_t rows, int64_t cols, int64_t klen, TileShape t = {kTile, kTile}, int blocks = 512,
                 int min_steps = 4) {
    const int64_t tiles = ((rows + t.bm - 1) / t.bm) * ((cols + t.bn - 1) / t.bn);
    int64_t s = (blocks + tiles - 1) / tiles;
    const int64_t steps = (klen + kStepK - 1) / kStepK;
    if (s > steps / min_steps) s = steps / min_steps;
    return (int)(s < 1 ? 1 : s);
}

int slice_len(int64_t klen, int slices) {
    const int64_t steps = (klen + kStepK - 1) / kStepK;
    return (int)((steps + slices - 1) / slices) * kStepK;
}

// The weight gradient reads channel-major copies of its operands when the
// images have power-of-two sides and rows of whole 8-pixel chunks; then
// layers of at most 64 output channels take the swapped 256 x BN tile.
struct WgradPlan {
    bool cmajor, swap;
    int bn, slices;
};
WgradPlan wgrad_plan(int h, int w, int64_t P, int cout, int cin, int ks) {
    WgradPlan p;
    p.cmajor = (h & (h - 1)) == 0 && (w & (w - 1)) == 0 && w % 8 == 0;
    p.swap = p.cmajor && cout <= 64;
    p.bn = cout <= 32 ? 32 : 64;
    const int64_t ncols = (int64_t)ks * ks * cin + 1;
    // 512 blocks, at least 4 K steps each (a sweep of 256 to 1536 blocks on
    // the surrogate's layers found no better count overall)
    p.slices = p.swap ? split_slices(ncols, cout, P, TileShape{256, p.bn}) : split_slices(cout, ncols, P);
    return p;
}
size_t align_up256(size_t b) { return (b + 255) & ~(size_t)255; }

// The completion of split sums: few long partials (one thread per element)
// or many short ones (four waves per 64 elements).
void launch_sum_parts(const SumSeg& s0, const SumSeg& s1, int parts, hipStream_t stream) {
    const size_t len = s0.len + s1.len;
    if (parts <= 16 || len >= ((size_t)1 << 18)) {
        hipLaunchKernelGGL(k_sum_parts_flat, dim3(grid_1d((int64_t)len)), dim3(256), 0, stream, s0, s1, parts);
    } else {
        size_t b = (s0.len + 63) / 64 + (s1.len + 63) / 64;
        b = b < 1 ? 1 : (b > 8192 ? 8192 : b);
        hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)b), dim3(256), 0, stream, s0, s1, parts);
    }
}
int fwd_slices(int64_t P, int cin, int cout, int ks) {
    return split_slices(P, cout, (int64_t)ks * ks * cin, conv_tile(cout));
}
int dgrad_slices(int64_t P, int cin, int cout, int ks) {
    return split_slices(P, cin, (int64_t)ks * ks * cout, conv_tile(cin));
}

// Launches k_conv_fwd or k_conv_dgrad with the block tile for n output columns.
template <template <int, int> class Kern>
void launch_conv_gemm(int64_t P, int64_t n, int slices, hipStream_t stream, const ConvArgs& a, int kslice,
                      float* part);
template <int BM, int BN>
struct FwdKernel {
    static void launch(dim3 grd, hipStream_t st, const ConvArgs& a, int kslice, float* part) {
        hipLaunchKernelGGL((k_conv_fwd<BM, BN>), grd, dim3(256), 0, st, a, kslice, part);
    }
};
template <int BM, int BN>
struct DgradKernel {
    static void launch(dim3 grd, hipStream_t st, const ConvArgs& a, int kslice, float* part) {
        hipLaunchKernelGGL((k_conv_dgrad<BM, BN>), grd, dim3(256), 0, st, a, kslice, part);
    }
};
template <template <int, int> class Kern>
void launch_conv_gemm(int64_t P, int64_t n, int slices, hipStream_t stream, const ConvArgs& a, int kslice,
                      float* part) {
    const TileShape t = conv_tile(n);
    const dim3 grd((unsigned)((P + t.bm - 1) / t.bm), (unsigned)((n + t.bn - 1) / t.bn), slices);
    if (t.bn == 32) Kern<256, 32>::launch(grd, stream, a, kslice, part);
    else if (t.bn == 64) Kern<256, 64>::launch(grd, stream, a, kslice, part);
    else Kern<128, 128>::launch(grd, stream, a, kslice, part);
}

}  // namespace

extern "C" {

const char* inim_nn_last_error(void) { return g_nn_error.c_str(); }

int inim_conv_workspace(int32_t imgs, int32_t h, int32_t w, int32_t cin, int32_t cout, int32_t ks, size_t* bytes) {
    int s = check_conv(imgs, h, w, cin, cout, ks);
    if (s != INIM_OK) return s;
    if (!bytes) return nfail(INIM_EINVAL, "bytes NULL");
    const int64_t P = (int64_t)imgs * h * w;
    const size_t wlen = (size_t)cout * ks * ks * cin;
    const WgradPlan wp = wgrad_plan(h, w, P, cout, cin, ks);
    size_t need = (size_t)wp.slices * (wlen + cout);
    const int fs = fwd_slices(P, cin, cout, ks), ds = dgrad_slices(P, cin, cout, ks);
    if (fs > 1 && (size_t)fs * P * cout > need) need = (size_t)fs * P * cout;
    if (ds > 1 && (size_t)ds * P * cin > need) need = (size_t)ds * P * cin;
    *bytes = align_up256(need * sizeof(float));
    if (wp.cmajor) *bytes += align_up256((size_t)P * cin * 2) + align_up256((size_t)P * cout * 2);
    return INIM_OK;
}

int inim_conv_forward(const inim_bf16* x, int32_t imgs, int32_t h, int32_t w, int32_t cin, const inim_bf16* weight,
                      const float* bias, int32_t cout, int32_t ks, int32_t relu, inim_bf16* y16, float* y32, void* work,
                      size_t work_bytes, hipStream_t stream) {
    int s = check_conv(imgs, h, w, cin, cout, ks);
    if (s != INIM_OK) return s;
    if (!x || !weight || (!y16 && !y32)) return nfail(INIM_EINVAL, "x, weight or both outputs NULL");
    ConvArgs a{};
    a.x = x; a.w = weight; a.bias = bias; a.y16 = y16; a.y32 = y32;
    a.H = h; a.W = w; a.P = imgs * h * w; a.Cin = cin; a.Cout = cout; a.ks = ks; a.relu = relu ? 1 : 0;
    const int K = ks * ks * cin;
    int slices = fwd_slices(a.P, cin, cout, ks);
    if (!work || work_bytes < (size_t)slices * a.P * cout * sizeof(float)) slices = 1;  // no room: one slice
    launch_conv_gemm<FwdKernel>(a.P, cout, slices, stream, a, slices > 1 ? slice_len(K, slices) : K,
                                static_cast<float*>(work));
    if (slices > 1)
        hipLaunchKernelGGL(k_conv_finish, dim3(grid_1d((int64_t)a.P * cout)), dim3(256), 0, stream, a, slices,
                           static_cast<const float*>(work));
    return launched("conv forward");
}

int inim_conv_backward_data(const inim_bf16* dy, int32_t imgs, int32_t h, int32_t w, int32_t cin,
                            const inim_bf16* weight_t, int32_t cout, int32_t ks, float* dx, void* work,
                            size_t work_bytes, hipStream_t stream) {
    int s = check_conv(imgs, h, w, cin, cout, ks);
    if (s != INIM_OK) return s;
    if (!dy || !weight_t || !dx) return nfail(INIM_EINVAL, "dy, weight_t or dx NULL");
    ConvArgs a{};
    a.dy = dy; a.wT = weight_t; a.dx = dx;
    a.H = h; a.W = w; a.P = imgs * h * w; a.Cin = cin; a.Cout = cout; a.ks = ks;
    const int K = ks * ks * cout;
    int slices = dgrad_slices(a.P, cin, cout, ks);
    if (!work || work_bytes < (size_t)slices * a.P * cin * sizeof(float)) slices = 1;
    launch_conv_gemm<DgradKernel>(a.P, cin, slices, stream, a, slices > 1 ? slice_len(K, slices) : K,
                                  static_cast<float*>(work));
    if (slices > 1)
        launch_sum_parts(SumSeg{static_cast<const float*>(work), (size_t)a.P * cin, dx}, SumSeg{nullptr, 0, nullptr},
                         slices, stream);
    return launched("conv input gradient");
}

int inim_conv_backward_weight(const inim_bf16* dy, const inim_bf16* x, int32_t imgs, int32_t h, int32_t w, int32_t cin,
                              int32_t cout, int32_t ks, float* dweight, float* dbias, void* work, size_t work_bytes,
                              hipStream_t stream) {
    size_t need;
    int s = inim_conv_workspace(imgs, h, w, cin, cout, ks, &need);
    if (s != INIM_OK) return s;
    if (!dy || !x || !dweight) return nfail(INIM_EINVAL, "dy, x or dweight NULL");
    if (!work || work_bytes < need) return nfail(INIM_EWORKSPACE, "work has %zu bytes, needs %zu", work_bytes, need);
    ConvArgs a{};
    a.dy = dy; a.x = x;
    a.H = h; a.W = w; a.P = imgs * h * w; a.Cin = cin; a.Cout = cout; a.ks = ks;
    const WgradPlan wp = wgrad_plan(h, w, a.P, cout, cin, ks);
    const int slices = wp.slices;
    const int kslice = slice_len(a.P, slices);
    const size_t wlen = (size_t)cout * ks * ks * cin;
    a.dw = static_cast<float*>(work);
    float* bp = dbias ? a.dw + (size_t)slices * wlen : nullptr;  // [slices][cout]
    const int ncols = ks * ks * cin + (dbias ? 1 : 0);               // the bias gradient is the column of ones
    const dim3 grd((cout + kTile - 1) / kTile, (unsigned)((ncols + kTile - 1) / kTile), slices);
    if (wp.cmajor) {
        // partials, then the channel-major copies of x and dy (sizes as in inim_conv_workspace)
        size_t parts = (size_t)slices * (wlen + cout);
        const int fs = fwd_slices(a.P, cin, cout, ks), ds = dgrad_slices(a.P, cin, cout, ks);
        if (fs > 1 && (size_t)fs * a.P * cout > parts) parts = (size_t)fs * a.P * cout;
        if (ds > 1 && (size_t)ds * a.P * cin > parts) parts = (size_t)ds * a.P * cin;
        uint16_t* xT = reinterpret_cast<uint16_t*>(static_cast<char*>(work) + align_up256(parts * sizeof(float)));
        uint16_t* dyT = xT + align_up256((size_t)a.P * cin * 2) / 2;
        int wlog = 0;
        while ((1 << wlog) < w) ++wlog;
        hipLaunchKernelGGL(k_cmajor, dim3((unsigned)((a.P + 63) / 64), (unsigned)((cin + 63) / 64 + (cout + 63) / 64)),
                           dim3(256), 0, stream, CmajorSeg{x, cin, xT}, CmajorSeg{dy, cout, dyT}, (int64_t)a.P);
        if (wp.swap) {
            const dim3 gs((unsigned)((ncols + 255) / 256), (unsigned)((cout + wp.bn - 1) / wp.bn), slices);
            if (wp.bn == 32)
                hipLaunchKernelGGL((k_conv_wgrad_t<256, 32, true>), gs, dim3(256), 0, stream, a, dyT, xT, wlog, kslice,
                                   bp);
            else
                hipLaunchKernelGGL((k_conv_wgrad_t<256, 64, true>), gs, dim3(256), 0, stream, a, dyT, xT, wlog, kslice,
                                   bp);
        } else {
            hipLaunchKernelGGL((k_conv_wgrad_t<128, 128, false>), grd, dim3(256), 0, stream, a, dyT, xT, wlog, kslice,
                               bp);
        }
    } else {
        hipLaunchKernelGGL(k_conv_wgrad, grd, dim3(256), 0, stream, a, kslice, bp);
    }
    launch_sum_parts(SumSeg{a.dw, wlen, dweight}, SumSeg{bp, dbias ? (size_t)cout : 0, dbias}, slices, stream);
    return launched("conv weight gradient");
}

int inim_weight_transpose(const inim_bf16* weight, int32_t cout, int32_t ks, int32_t cin, inim_bf16* weight_t,
                          hipStream_t stream) {
    if (!weight || !weight_t || cout < 1 || cin < 1 || (ks != 1 && ks != 3))
        return nfail(INIM_EINVAL, "bad weight transpose arguments");
    hipLaunchKernelGGL(k_wtrans, dim3(grid_1d((int64_t)cout * ks * ks * cin)), dim3(256), 0, stream, weight, cout,
                       ks * ks, cin, weight_t);
    return launched("weight transpose");
}

int inim_f32_to_bf16(const float* a, int64_t n, inim_bf16* b, hipStream_t stream) {
    if (n < 0 || (n > 0 && (!a || !b))) return nfail(INIM_EINVAL, "bad cast arguments");
    if (n == 0) return INIM_OK;
    hipLaunchKernelGGL(k_f32_to_bf16, dim3(grid_1d(n)), dim3(256), 0, stream, a, (size_t)n, b);
    return launched("cast");
}

int inim_pool2(const inim_bf16* x, int32_t imgs, int32_t h, int32_t w, int32_t c, inim_bf16* y, hipStream_t stream) {
    if (!x || !y || imgs < 1 || h < 2 || w < 2 || h % 2 || w % 2 || c < 1)
        return nfail(INIM_EINVAL, "bad pooling arguments");
    hipLaunchKernelGGL(k_pool2, dim3(grid_1d((int64_t)imgs * (h / 2) * (w / 2) * c)), dim3(256), 0, stream, x, imgs, h, w,
                       c, y);
    return launched("pool");
}

int inim_pool2_backward(const float* dy, int32_t imgs, int32_t h, int32_t w, int32_t c, float* dx, int32_t accumulate,
                        hipStream_t stream) {
    if (!dy || !dx || imgs < 1 || h < 2 || w < 2 || h % 2 || w % 2 || c < 1)
        return nfail(INIM_EINVAL, "bad pooling-gradient arguments");
    hipLaunchKernelGGL(k_pool2_back, dim3(grid_1d((int64_t)imgs * h * w * c)), dim3(256), 0, stream, dy, imgs, h, w, c, dx,
                       accumulate ? 1 : 0);
    return launched("pool gradient");
}

int inim_upsample2_into(const inim_bf16* x, int32_t imgs, int32_t h, int32_t w, int32_t c, inim_bf16* y, int32_t ct,
                        int32_t c0, hipStream_t stream) {
    if (!x || !y || imgs < 1 || h < 1 || w < 1 || c < 1 || c0 < 0 || c0 + c > ct)
        return nfail(INIM_EINVAL, "bad upsampling arguments");
    hipLaunchKernelGGL(k_up2_into, dim3(grid_1d((int64_t)imgs * 4 * h * w * c)), dim3(256), 0, stream, x, imgs, h, w, c, y,
                       ct, c0);
    return launched("upsample");
}

int inim_concat_up2(const inim_bf16* a, int32_t imgs, int32_t h, int32_t w, int32_t ca, const inim_bf16* b,
                    int32_t cb, inim_bf16* y, hipStream_t stream) {
    if (!a || !b || !y || imgs < 1 || h < 1 || w < 1 || ca < 1 || cb < 1) return nfail(INIM_EINVAL, "bad concat arguments");
    hipLaunchKernelGGL(k_concat_up2, dim3(grid_1d((int64_t)imgs * 4 * h * w * (ca + cb))), dim3(256), 0, stream, a, imgs,
                       h, w, ca, b, cb, y);
    return launched("concat");
}

int inim_copy_channels_into(const inim_bf16* x, int64_t pixels, int32_t c, inim_bf16* y, int32_t ct, int32_t c0,
                            hipStream_t stream) {
    if (!x || !y || pixels < 1 || c < 1 || c0 < 0 || c0 + c > ct) return nfail(INIM_EINVAL, "bad channel copy arguments");
    hipLaunchKernelGGL(k_copy_into, dim3(grid_1d(pixels * c)), dim3(256), 0, stream, x, (size_t)pixels, c, y, ct, c0);
    return launched("channel copy");
}

int inim_upsample2_backward(const float* dy, int32_t imgs, int32_t h, int32_t w, int32_t ct, int32_t ca, float* da,
                            hipStream_t stream) {
    if (!dy || !da || imgs < 1 || h < 1 || w < 1 || ca < 1 || ca > ct)
        return nfail(INIM_EINVAL, "bad upsampling-gradient arguments");
    hipLaunchKernelGGL(k_up2_back, dim3(grid_1d((int64_t)imgs * h * w * ca)), dim3(256), 0, stream, dy, imgs, h, w, ct, ca,
                       da);
    return launched("upsample gradient");
}

int inim_take_channels(const float* dy, int64_t pixels, int32_t ct, int32_t c0, int32_t c, float* out,
                       int32_t accumulate, hipStream_t stream) {
    if (!dy || !out || pixels < 1 || c < 1 || c0 < 0 || c0 + c > ct) return nfail(INIM_EINVAL, "bad channel arguments");
    hipLaunchKernelGGL(k_take_channels, dim3(grid_1d(pixels * c)), dim3(256), 0, stream, dy, (size_t)pixels, ct, c0, c,
                       out, accumulate ? 1 : 0);
    return launched("channel gradient");
}

int inim_relu_backward(const float* g, const inim_bf16* act, int64_t n, inim_bf16* g16, hipStream_t stream) {
    if (!g || !g16 || n < 1) return nfail(INIM_EINVAL, "bad ReLU-gradient arguments");
    hipLaunchKernelGGL(k_relu_back, dim3(grid_1d(n)), dim3(256), 0, stream, g, act, (size_t)n, g16);
    return launched("ReLU gradient");
}

int inim_mse(const float* pred, int32_t cp, const float* target, int32_t ct, int64_t pixels, float* loss,
             inim_bf16* grad, void* work, size_t work_bytes, hipStream_t stream) {
    if (!pred || !target || !loss || pixels < 1 || ct < 1 || ct > cp) return nfail(INIM_EINVAL, "bad loss arguments");
    if (!work || work_bytes < kMsePartials * sizeof(float)) return nfail(INIM_EWORKSPACE, "loss work too small");
    float* parts = static_cast<float*>(work);
    hipLaunchKernelGGL(k_mse, dim3(kMsePartials), dim3(256), 0, stream, pred, cp, target, ct, (size_t)pixels, parts, grad);
    launch_sum_parts(SumSeg{parts, 1, loss}, SumSeg{nullptr, 0, nullptr}, kMsePartials, stream);
    return launched("loss");
}

int inim_nn_pack_density(const float* density, int32_t res, float scale, int32_t c, inim_bf16* x, hipStream_t stream) {
    if (!density || !x || res < 2 || c < 1) return nfail(INIM_EINVAL, "bad input-packing arguments");
    const size_t px = (size_t)res * res;
    hipLaunchKernelGGL(k_pack_density, dim3(grid_1d((int64_t)(px * c))), dim3(256), 0, stream, density, px, scale, c, x);
    return launched("pack density");
}

int inim_nn_pack_density_many(const float* density, int32_t count, int32_t res, const float* scale, int32_t c,
                              inim_bf16* x, hipStream_t stream) {
    if (!density || !x || !scale || res < 2 || c < 1 || count < 1 || count > kMaxScales)
        return nfail(INIM_EINVAL, "bad input-packing arguments");
    Scales sc{};
    for (int q = 0; q < count; ++q) sc.v[q] = scale[q];
    const size_t px = (size_t)res * res;
    hipLaunchKernelGGL(k_pack_density_many, dim3(grid_1d((int64_t)(px * c)), count), dim3(256), 0, stream, density, px,
                       sc, c, x);
    return launched("pack density");
}

int inim_nn_pack_input_many(const float* density, const float* field, int32_t count, int32_t res, const float* scale,
                            int32_t c, inim_bf16* x, hipStream_t stream) {
    if (!density || !field || !x || !scale || res < 2 || c < 3 || count < 1 || count > kMaxScales)
        return nfail(INIM_EINVAL, "bad input-packing arguments");
    Scales sc{};
    for (int q = 0; q < count; ++q) sc.v[q] = scale[q];
    const size_t px = (size_t)res * res;
    hipLaunchKernelGGL(k_pack_input_many, dim3(grid_1d((int64_t)(px * c)), count), dim3(256), 0, stream, density, field,
                       res, sc, c, x);
    return launched("pack input");
}

int inim_nn_displacement(const float* probe, int32_t res, float* out, hipStream_t stream) {
    if (!probe || !out || res < 2) return nfail(INIM_EINVAL, "bad displacement arguments");
    hipLaunchKernelGGL(k_displacement, dim3(grid_1d((int64_t)res * res)), dim3(256), 0, stream,
                       reinterpret_cast<const float2*>(probe), res, out);
    return launched("displacement");
}

static hipError_t launch_field(const float* y, int c, int res, int radius, int k, float* field, float* work,
                               hipStream_t stream) {
    FieldTaps t{};
    t.r = radius;
    double w[33], s = 0.0;
    for (int m = -radius; m <= radius; ++m) {  // exp(-m^2 / (2 (r/2)^2)), normalised
        w[m + radius] = radius ? std::exp(-2.0 * m * m / ((double)radius * radius)) : 1.0;
        s += w[m + radius];
    }
    for (int q = 0; q <= 2 * radius; ++q) t.w[q] = (float)(w[q] / s);
    const dim3 g(grid_1d((int64_t)res * res), k);
    hipLaunchKernelGGL(k_field_smooth_x, g, dim3(256), 0, stream, y, c, res, t, reinterpret_cast<float2*>(work));
    hipLaunchKernelGGL(k_field_smooth_y, g, dim3(256), 0, stream, reinterpret_cast<const float2*>(work), res, t,
                       reinterpret_cast<float2*>(field));
    return hipGetLastError();
}

int inim_nn_field(const float* y, int32_t c, int32_t res, int32_t radius, float* field, float* work,
                  hipStream_t stream) {
    if (!y || !field || !work || res < 2 || c < 2 || radius < 0 || radius > 16)
        return nfail(INIM_EINVAL, "bad field arguments");
    (void)launch_field(y, c, res, radius, 1, field, work, stream);
    return launched("field");
}

int inim_nn_field_many(const float* y, int32_t count, int32_t c, int32_t res, int32_t radius, float* field, float* work,
                       hipStream_t stream) {
    if (!y || !field || !work || res < 2 || c < 2 || radius < 0 || radius > 16 || count < 1 || count > 65535)
        return nfail(INIM_EINVAL, "bad field arguments");
    (void)launch_field(y, c, res, radius, count, field, work, stream);
    return launched("field");
}

int inim_nn_count_folds(const float* field, int32_t res, uint32_t* count, hipStream_t stream) {
    if (!field || !count || res < 2) return nfail(INIM_EINVAL, "bad fold-count arguments");
    hipLaunchKernelGGL(k_count_folds, dim3(grid_1d((int64_t)(res - 1) * (res - 1))), dim3(256), 0, stream,
                       reinterpret_cast<const float2*>(field), res, count);
    return launched("fold count");
}

int inim_nn_bin_moments(const uint32_t* counts, int32_t res, int32_t bin, double* out, hipStream_t stream) {
    if (!counts || !out || res < 2 || bin < 1 || res % bin) return nfail(INIM_EINVAL, "bad bin-moment arguments");
    const int64_t nb = (int64_t)(res / bin) * (res / bin);
    hipLaunchKernelGGL(k_bin_moments, dim3(grid_1d(nb)), dim3(256), 0, stream, counts, res, bin, out);
    return launched("bin moments");
}

int inim_adam(float* weight, const float* grad, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
              int32_t step, inim_bf16* weight16, hipStream_t stream) {
    if (!weight || !grad || !m || !v || n < 1 || step < 1) return nfail(INIM_EINVAL, "bad Adam arguments");
    AdamArgs a{lr, b1, b2, eps, 1.0f / (1.0f - powf(b1, (float)step)), 1.0f / (1.0f - powf(b2, (float)step))};
    hipLaunchKernelGGL(k_adam, dim3(grid_1d(n)), dim3(256), 0, stream, weight, grad, m, v, (size_t)n, a, weight16);
    return launched("Adam");
}

}  // extern "C"
