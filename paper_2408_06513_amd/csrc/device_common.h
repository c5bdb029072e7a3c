// device_common.h -- device helpers shared by the gfx950 kernels of libinim:
// wave64 scans, uniform broadcasts, vector loads/stores, the closed-form
// integral images of a constant raster and the per-texel deformation map.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "inim.h"

namespace inim {

constexpr int kWave = 64;

// ---------------------------------------------------------------- fixed point
// Float rasters are summed exactly in 128-bit two's-complement fixed point with
// 64 fractional bits: every float32 whose magnitude is at least 2^-64 and
// below 2^62 converts without error (smaller magnitudes are truncated toward
// zero, an error below 2^-64 each), integer addition is exact and associative,
// so any sum, difference and complement of region sums is exact while the
// total stays below 2^63 in magnitude.  Results are rounded once on output.
typedef unsigned __int128 u128;

__device__ __forceinline__ u128 fx_from_float(float f) {
    const uint32_t bits = __float_as_uint(f);
    const uint32_t ex = (bits >> 23) & 0xFFu;
    uint64_t m = bits & 0x7FFFFFu;
    int e;  // |f| = m * 2^e
    if (ex == 0) {
        e = -149;
    } else {
        m |= 0x800000u;
        e = (int)ex - 150;
    }
    const int sh = e + 64;  // fixed = m * 2^(e + 64)
    u128 v;
    if (sh >= 0) v = (u128)m << sh;
    else if (sh > -64) v = (u128)(m >> (-sh));
    else v = 0;
    return (bits >> 31) ? (u128)0 - v : v;
}

__device__ __forceinline__ double fx_to_double(u128 v) {
    const bool neg = (int64_t)(uint64_t)(v >> 64) < 0;
    if (neg) v = (u128)0 - v;
    const uint64_t hi = (uint64_t)(v >> 64), lo = (uint64_t)v;
    const double d = (double)hi + (double)lo * 0x1p-64;
    return neg ? -d : d;
}

// The fixed-point value as a float, correctly rounded (to nearest, ties to
// even) in one step: the 24 bits below the leading one, then the round bit
// and a sticky bit of everything further down.  |value| >= 2^-64 always
// gives a normal float.
__device__ __noinline__ float fx_to_float_exact(u128 v) {
    const bool neg = (int64_t)(uint64_t)(v >> 64) < 0;
    if (neg) v = (u128)0 - v;
    const uint64_t hi = (uint64_t)(v >> 64), lo = (uint64_t)v;
    if ((hi | lo) == 0) return 0.0f;
    uint64_t top;  // the magnitude shifted so that its leading one is bit 63
    bool sticky;   // a one below the 64 bits of `top`
    int e;         // the leading one's weight is 2^e
    if (hi != 0) {
        const int lz = __clzll((long long)hi);
        top = lz ? (hi << lz) | (lo >> (64 - lz)) : hi;
        sticky = (lz ? (lo << lz) : lo) != 0;
        e = 63 - lz;
    } else {
        const int lz = __clzll((long long)lo);
        top = lo << lz;
        sticky = false;
        e = -1 - lz;
    }
    uint32_t mant = (uint32_t)(top >> 40);  // 24 bits, leading one included
    const uint64_t rest = top & ((1ull << 40) - 1), half = 1ull << 39;
    if (rest > half || (rest == half && (sticky || (mant & 1u)))) {
        if (++mant == (1u << 24)) {
            mant >>= 1;
            ++e;
        }
    }
    const uint32_t bits = ((uint32_t)neg << 31) | ((uint32_t)(e + 127) << 23) | (mant & 0x7FFFFFu);
    return __uint_as_float(bits);
}

// The same result, mostly without the bit scan: for a non-negative value the
// sum of its two halves converted to double is within 1.5 units in the last
// place of double of the exact value, so its float rounding is the correct
// one unless it lies that close to a midpoint between two floats (whose
// double has 0x10000000 in the 29 bits below the float's mantissa); negative
// values and those near a midpoint take the exact conversion.
__device__ __forceinline__ float fx_to_float(u128 v) {
    const uint64_t hi = (uint64_t)(v >> 64), lo = (uint64_t)v;
    const double d = (double)hi + (double)lo * 0x1p-64;
    const uint32_t low = (uint32_t)(uint64_t)__double_as_longlong(d) & 0x1FFFFFFFu;
    if ((int64_t)hi < 0 || low - 0x0FFFFFFEu <= 4u) return fx_to_float_exact(v);
    return (float)d;
}

// ---------------------------------------------------------------- accumulators
// uint32 rasters accumulate modulo 2^32 (exact below 2^32); float rasters in
// the 128-bit fixed point above where exact planes are required, or in double
// where the sums only feed the deformation.

template <typename Acc, typename Tin> __device__ __forceinline__ Acc to_acc(Tin v);
template <> __device__ __forceinline__ uint32_t to_acc<uint32_t, uint32_t>(uint32_t v) { return v; }
template <> __device__ __forceinline__ u128 to_acc<u128, float>(float v) { return fx_from_float(v); }
template <> __device__ __forceinline__ double to_acc<double, float>(float v) { return (double)v; }

__device__ __forceinline__ double to_f64(uint32_t a) { return (double)a; }
__device__ __forceinline__ double to_f64(u128 a) { return fx_to_double(a); }
__device__ __forceinline__ double to_f64(double a) { return a; }

template <typename Tout, typename Acc> __device__ __forceinline__ Tout narrow(Acc a);
template <> __device__ __forceinline__ uint32_t narrow<uint32_t, uint32_t>(uint32_t a) { return a; }
template <> __device__ __forceinline__ float narrow<float, u128>(u128 a) { return fx_to_float(a); }
template <> __device__ __forceinline__ float narrow<float, double>(double a) { return (float)a; }

// ---------------------------------------------------------------- wave64 ops
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t shfl_up(uint32_t v, int d) { return __shfl_up(v, d, kWave); }
__device__ __forceinline__ uint32_t shfl_down(uint32_t v, int d) { return __shfl_down(v, d, kWave); }
__device__ __forceinline__ uint32_t shfl_xor(uint32_t v, int d) { return __shfl_xor(v, d, kWave); }
__device__ __forceinline__ double shfl_up(double v, int d) { return __shfl_up(v, d, kWave); }
__device__ __forceinline__ double shfl_down(double v, int d) { return __shfl_down(v, d, kWave); }
__device__ __forceinline__ double shfl_xor(double v, int d) { return __shfl_xor(v, d, kWave); }
__device__ __forceinline__ u128 join(unsigned long long lo, unsigned long long hi) {
    return ((u128)hi << 64) | (u128)lo;
}
__device__ __forceinline__ u128 shfl_up(u128 v, int d) {
    return join(__shfl_up((unsigned long long)(uint64_t)v, d, kWave), __shfl_up((unsigned long long)(uint64_t)(v >> 64), d, kWave));
}
__device__ __forceinline__ u128 shfl_down(u128 v, int d) {
    return join(__shfl_down((unsigned long long)(uint64_t)v, d, kWave),
                __shfl_down((unsigned long long)(uint64_t)(v >> 64), d, kWave));
}
__device__ __forceinline__ u128 shfl_xor(u128 v, int d) {
    return join(__shfl_xor((unsigned long long)(uint64_t)v, d, kWave),
                __shfl_xor((unsigned long long)(uint64_t)(v >> 64), d, kWave));
}

// Lane moves through the DPP crossbar (GFX9 encodings), applied to each
// 32-bit word of a value.  A lane whose source lies outside the pattern, or
// whose 16-lane row is not in ROWS, receives 0 (the identity of every sum
// below).  All 64 lanes must be active.
enum : int {
    kDppRowShr1 = 0x111,
    kDppRowShr2 = 0x112,
    kDppRowShr4 = 0x114,
    kDppRowShr8 = 0x118,
    kDppWaveShl1 = 0x130,   // lane l reads lane l+1
    kDppWaveShr1 = 0x138,   // lane l reads lane l-1
    kDppRowBcast15 = 0x142, // lane 15 of each row to the next row
    kDppRowBcast31 = 0x143  // lane 31 to rows 2 and 3
};
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF, true);
}
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ uint32_t dpp(uint32_t v) { return dpp32<CTRL, ROWS>(v); }
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint64_t lo = dpp32<CTRL, ROWS>((uint32_t)b), hi = dpp32<CTRL, ROWS>((uint32_t)(b >> 32));
    return __longlong_as_double((long long)((hi << 32) | lo));
}
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ u128 dpp(u128 v) {
    u128 r = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) r |= (u128)dpp32<CTRL, ROWS>((uint32_t)(v >> (32 * k))) << (32 * k);
    return r;
}

// Value of lane l-1 (0 in lane 0) and of lane l+1 (0 in lane 63).
template <typename T>
__device__ __forceinline__ T shfl_up1(T v) { return dpp<kDppWaveShr1>(v); }
template <typename T>
__device__ __forceinline__ T shfl_down1(T v) { return dpp<kDppWaveShl1>(v); }

// Inclusive scan over the 64 lanes: Hillis-Steele steps 1, 2, 4, 8 inside
// each 16-lane row, then the totals of rows 0 and 2 into rows 1 and 3, then
// the total of rows 0-1 into rows 2 and 3.
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
    v += dpp<kDppRowShr1>(v);
    v += dpp<kDppRowShr2>(v);
    v += dpp<kDppRowShr4>(v);
    v += dpp<kDppRowShr8>(v);
    v += dpp<kDppRowBcast15, 0xA>(v);
    v += dpp<kDppRowBcast31, 0xC>(v);
    return v;
}

// Value of v in lane `src` (src uniform across the wave).
__device__ __forceinline__ uint32_t bcast(uint32_t v, int src) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, src);
}
__device__ __forceinline__ double bcast(double v, int src) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, src);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), src);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ u128 bcast(u128 v, int src) {
    uint32_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> (32 * k)), src);
    return ((u128)w[3] << 96) | ((u128)w[2] << 64) | ((u128)w[1] << 32) | (u128)w[0];
}

// ---------------------------------------------------------------- vector IO
// Q adjacent 4-byte values of one lane, moved as 16-byte (or smaller) vectors.
template <typename T, int Q>
struct VecT {
    typedef T type __attribute__((ext_vector_type(Q)));
};
template <typename T>
struct VecT<T, 1> {
    typedef T type;
};

template <typename T, int Q>
__device__ __forceinline__ void load_row(const T* __restrict__ p, T (&out)[Q]) {
    constexpr int V = (Q * sizeof(T) <= 16) ? Q : (int)(16 / sizeof(T));
    typedef typename VecT<T, V>::type vt;
#pragma unroll
    for (int h = 0; h < Q; h += V) {
        vt t = *reinterpret_cast<const vt*>(p + h);
        if constexpr (V == 1) {
            out[h] = t;
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) out[h + e] = t[e];
        }
    }
}

template <typename T, int Q>
__device__ __forceinline__ void store_row_nt(T* __restrict__ p, const T (&in)[Q]) {
    constexpr int V = (Q * sizeof(T) <= 16) ? Q : (int)(16 / sizeof(T));
    typedef typename VecT<T, V>::type vt;
#pragma unroll
    for (int h = 0; h < Q; h += V) {
        vt t;
        if constexpr (V == 1) {
            t = in[h];
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) t[e] = in[h + e];
        }
        __builtin_nontemporal_store(t, reinterpret_cast<vt*>(p + h));
    }
}

// Q float2 texels as interleaved floats.
template <int Q>
__device__ __forceinline__ void store_field_nt(float2* __restrict__ p, const float2 (&in)[Q]) {
    float f[2 * Q];
#pragma unroll
    for (int e = 0; e < Q; ++e) { f[2 * e] = in[e].x; f[2 * e + 1] = in[e].y; }
    store_row_nt<float, 2 * Q>(reinterpret_cast<float*>(p), f);
}

// Element r (uniform) of a per-lane pair holding rows lane and lane+64.
template <typename T>
__device__ __forceinline__ T pick_row(const T (&v)[2], int r) { return (r < 64) ? v[0] : v[1]; }

// ---------------------------------------------------------------- status word
__device__ __forceinline__ bool failed(const int* status) {
    return status != nullptr && __builtin_nontemporal_load(status) != 0;
}

// ---------------------------------------------------------------- constant raster
// Integral images of the all-ones res x res raster at texel (i, j), counted
// combinatorially; exact integers (at most res^2 <= 2^28) held in double, so
// every product and sum below is exact.
struct Planes8 {
    double a, b, g, d, at, bt, gt, dt;
};

__device__ __forceinline__ Planes8 ones_planes(int i, int j, int N) {
    Planes8 p;
    const double I = i, J = j, n = N, nn = n * n;
    p.a = (I + 1.0) * (J + 1.0);
    p.b = (I + 1.0) * (n - 1.0 - J);
    p.g = (n - 1.0 - I) * (n - 1.0 - J);
    p.d = (n - 1.0 - I) * (J + 1.0);
    // alpha_t: the wedge j' <= j - |i' - i| counted column by column.
    const double m = J + 1.0;
    const double kl = fmin(I, m), kr = fmin(n - 1.0 - I, m);
    const double at = m + (kl * m - 0.5 * kl * (kl + 1.0)) + (kr * m - 0.5 * kr * (kr + 1.0));
    const double u = I + J, v = I - J;
    const double U = (u <= n - 1.0) ? 0.5 * (u + 1.0) * (u + 2.0) : nn - 0.5 * (2.0 * n - 2.0 - u) * (2.0 * n - 1.0 - u);
    const double V = (v >= 0.0) ? 0.5 * (n - v) * (n - v + 1.0) : nn - 0.5 * (n + v - 1.0) * (n + v);
    p.at = at;
    p.bt = U - at;
    p.dt = V - at;
    p.gt = nn - U - V + at;
    return p;
}

// ---------------------------------------------------------------- map
// Weighted sum S of eq. (map) at the point (x, y): the anchors q1..q4 of the
// Molchanov-Linsen map, alpha_t paired with (x,1), beta_t with (1,y), gamma_t
// with (x,0) and delta_t with (0,y).  t = S / (2C).
__device__ __forceinline__ void map_sum(const Planes8& P, double x, double y, double& sx, double& sy) {
    double q1x, q1y, q2x, q2y, q3x, q3y, q4x, q4y;
    if (y < x) { q1x = 1.0; q1y = 1.0 + y - x; q3x = x - y; q3y = 0.0; }
    else       { q1x = 1.0 - y + x; q1y = 1.0; q3x = 0.0; q3y = y - x; }
    if (x + y < 1.0) { q2x = x + y; q2y = 0.0; q4x = 0.0; q4y = x + y; }
    else             { q2x = 1.0; q2y = x + y - 1.0; q4x = x + y - 1.0; q4y = 1.0; }
    sx = P.a * q1x + P.b * q2x + P.g * q3x + P.d * q4x + (P.at + P.gt) * x + P.bt;
    sy = P.a * q1y + P.b * q2y + P.g * q3y + P.d * q4y + P.at + (P.bt + P.dt) * y;
}

// t(p; 1), the map of the constant raster, at the centre of texel (i, j): the
// defect that the deformation removes (Sec. 4.2), as floats.
__device__ __forceinline__ float2 defect_texel(int i, int j, int N) {
    const double invN = 1.0 / (double)N;
    const double x = ((double)i + 0.5) * invN, y = ((double)j + 0.5) * invN;
    double sx, sy;
    map_sum(ones_planes(i, j, N), x, y, sx, sy);
    const double s = 1.0 / (2.0 * (double)N * (double)N);
    return make_float2((float)(sx * s), (float)(sy * s));
}

// Scale factors of the deformation: 1 / (2 C_d) with C_d = C_r + d0 res^2 the
// total of d = d_r + d0, and 1 / (2 res^2) for the constant raster.
// omk = 1 - d0 res^2 / C_d, the weight of the defect once the constant part of
// d is folded in (see deform_texel_defect).
struct MapScale {
    double d0, inv2Cd, inv2NN, omk, invN;
};

__device__ __forceinline__ MapScale map_scale(double Cr, int N, double d0) {
    const double NN = (double)N * (double)N;
    const double Cd = Cr + d0 * NN;
    MapScale s;
    s.d0 = d0;
    s.inv2Cd = 1.0 / (2.0 * Cd);
    s.inv2NN = 1.0 / (2.0 * NN);
    s.omk = Cr / Cd;
    s.invN = 1.0 / (double)N;
    return s;
}

// Deformation at texel (i, j), eq. (map_res): T = p + t(p; d_r + d0) - t(p; d0).
// `R` holds the eight planes of d_r; the planes of the constant part are d0
// times the closed forms, and t(p; d0) = t(p; 1).
__device__ __forceinline__ float2 deform_texel(const Planes8& R, const MapScale& ms, int i, int j, int N) {
    const double x = ((double)i + 0.5) / (double)N;
    const double y = ((double)j + 0.5) / (double)N;
    const Planes8 O = ones_planes(i, j, N);
    const double d0 = ms.d0;
    Planes8 D;
    D.a = R.a + d0 * O.a; D.b = R.b + d0 * O.b; D.g = R.g + d0 * O.g; D.d = R.d + d0 * O.d;
    D.at = R.at + d0 * O.at; D.bt = R.bt + d0 * O.bt; D.gt = R.gt + d0 * O.gt; D.dt = R.dt + d0 * O.dt;
    double sdx, sdy, s1x, s1y;
    map_sum(D, x, y, sdx, sdy);
    map_sum(O, x, y, s1x, s1y);
    const double tx = sdx * ms.inv2Cd - s1x * ms.inv2NN;
    const double ty = sdy * ms.inv2Cd - s1y * ms.inv2NN;
    return make_float2((float)(x + tx), (float)(y + ty));
}

// The same deformation with the defect field t1 = t(p; 1) precomputed: the map
// is linear in the planes, S(d) = S(d_r) + d0 S(1) and 2 C_d t(p; d0) / (2 C_d)
// = t1, so T = p + S(d_r) / (2 C_d) - (1 - d0 res^2 / C_d) t1.
__device__ __forceinline__ float2 deform_texel_defect(const Planes8& R, const MapScale& ms, int i, int j, float2 t1) {
    const double x = ((double)i + 0.5) * ms.invN;
    const double y = ((double)j + 0.5) * ms.invN;
    double sx, sy;
    map_sum(R, x, y, sx, sy);
    const double tx = sx * ms.inv2Cd - ms.omk * (double)t1.x;
    const double ty = sy * ms.inv2Cd - ms.omk * (double)t1.y;
    return make_float2((float)(x + tx), (float)(y + ty));
}

// The six complementary planes from alpha, alpha_t and the marginals
// (partitions of Sec. 3.1), in the accumulation type.  Regions that are empty
// by construction (beta on the last row, delta on the last column, gamma on
// either, beta_t on the first column, gamma_t on the last row, delta_t on the
// last column) come out exactly zero from the integer accumulators (both
// terms are exact sums of the same texels); in double they are set to zero.
template <typename Acc>
struct Compl {
    Acc b, g, d, bt, gt, dt;
};

template <typename Acc>
__device__ __forceinline__ Compl<Acc> complements(Acc al, Acc at, Acc X, Acc Y, Acc U, Acc V, Acc C,
                                                  int i, int j, int N) {
    Compl<Acc> o;
    o.b = X - al;
    o.d = Y - al;
    o.g = (C - X) - Y + al;
    o.bt = U - at;
    o.dt = V - at;
    o.gt = (C - U) - V + at;
    if constexpr (__is_same(Acc, double)) {
        if (j == N - 1) { o.b = 0.0; o.gt = 0.0; }
        if (i == N - 1) { o.d = 0.0; o.dt = 0.0; }
        if (i == N - 1 || j == N - 1) o.g = 0.0;
        if (i == 0) o.bt = 0.0;
    }
    return o;
}

}  // namespace inim
