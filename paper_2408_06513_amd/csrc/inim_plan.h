// inim_plan.h -- tiling of the integral-image pass and the device buffers it
// uses; shared by the kernels and the host-side C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace inim {

// Exact 128-bit fixed-point accumulator of float rasters (see device_common.h).
typedef unsigned __int128 u128;

// A res x res raster is cut into bands of H rows and tiles of W = 64*Q columns;
// one wave64 streams one tile top to bottom, Q adjacent columns per lane.
struct Geom {
    int N;         // raster side
    int Q;         // columns per lane
    int W;         // tile width  (<= N, multiple of Q; >= H; >= 64 unless N < 64)
    int H;         // tile height (rows per band)
    int T;         // tiles per band, N / W
    int B;         // bands, N / H
    int lastLane;  // W / Q - 1
};

// Per-tile partial sums written by the aggregate kernel.
//   colsum[b][i]  column sum of band b
//   tcsp[b][i]    prefix of colsum within the tile (inclusive)
//   tLend, tRend  tile-local up-left / up-right diagonal sums of the band's
//                 column prefixes, at the band's last row
//   tLedge[b][c][r]  tile-local up-left diagonal sum ending on the tile's last column, row r
//   tRedge[b][c][r]  tile-local up-right diagonal sum ending on the tile's first column, row r
//   trow[b][c][r]    sum over the tile's columns of the band-local column prefix at row r
template <typename Acc>
struct Agg {
    Acc *colsum, *tcsp, *tLend, *tRend;
    Acc *tLedge, *tRedge, *trow;
};

// Carries at the row above band b (b = 0..B; row B is the state after the last row):
//   cpin[b][i] column prefix, ain[b][i] alpha, Lin[b][i] / Rin[b][i] the
//   up-left / up-right diagonal sums of column prefixes;
// per band row: AC[b][c][r] = alpha(cW-1, bH+r) for c = 0..T (c = T gives
// the row marginal Y(bH+r) = alpha(N-1, bH+r)); and the diagonal marginals
// U[u] = sum over i'+j' <= u, V[v+N-1] = sum over i'-j' >= v (2N-1 each).
template <typename Acc>
struct Carry {
    Acc *cpin, *ain, *Lin, *Rin, *AC, *U, *V;
};

__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// acc_bytes: 4 for uint32 rasters, 8 or 16 for float rasters (wider
// accumulators need more registers per column, so float tiles are narrower).
__host__ __device__ inline Geom make_geom(int N, int acc_bytes = 4, int q_hint = 0, int h_hint = 0) {
    Geom g;
    g.N = N;
    int Q, H;
    if (N < 64) {
        Q = 1;
        H = N < 16 ? N : 16;
    } else if (N <= 2048) {
        Q = 1;
        H = 16;
    } else if (N <= 4096) {
        Q = 1;
        H = 64;
    } else {
        Q = acc_bytes > 4 ? 2 : 4;
        H = N / 256 > 32 ? N / 256 : 32;  // 32-row bands, at most 256 of them
    }
    if (q_hint > 0) Q = q_hint > 4 ? 4 : q_hint;
    if (h_hint > 0) H = h_hint;
    int W = 64 * Q;
    if (W > N) {
        W = N;
        if (Q > W) Q = W;
        while (Q > 1 && (W % Q != 0 || W / Q > 64)) Q >>= 1;
    }
    if (H > W) H = W;
    if (H > 128) H = 128;
    if (H > N) H = N;
    while (N / H > 256) H <<= 1;  // at most 256 bands (carry scans)
    g.Q = Q;
    g.W = W;
    g.H = H;
    g.T = N / W;
    g.B = N / H;
    g.lastLane = W / Q - 1;
    return g;
}

__host__ __device__ inline bool geom_ok(const Geom& g) {
    return g.W >= g.H && g.B <= 256 && g.W % g.Q == 0 && g.W / g.Q <= 64 && g.N % g.W == 0 &&
           g.N % g.H == 0 && g.H <= 128 && (g.Q == 1 || g.Q == 2 || g.Q == 4);
}

// Bytes of the aggregate and carry arrays for accumulator size `acc`
// (4 for uint32 rasters; 8 (double) or 16 (128-bit fixed point) for float rasters).
__host__ __device__ inline size_t inim_scratch_bytes(const Geom& g, size_t acc) {
    const size_t N = (size_t)g.N;
    size_t s = 0;
    s += 4 * align256((size_t)g.B * N * acc);                 // colsum tcsp tLend tRend
    s += 3 * align256((size_t)g.B * g.T * g.H * acc);         // tLedge tRedge trow
    s += 4 * align256((size_t)(g.B + 1) * N * acc);           // cpin ain Lin Rin
    s += align256((size_t)g.B * (g.T + 1) * g.H * acc);       // AC
    s += 2 * align256((size_t)(2 * N) * acc);                 // U V
    return s;
}

template <typename Acc>
__host__ __device__ inline void carve(const Geom& g, char* base, Agg<Acc>& A, Carry<Acc>& K) {
    const size_t N = (size_t)g.N;
    const size_t col = align256((size_t)g.B * N * sizeof(Acc));
    const size_t edge = align256((size_t)g.B * g.T * g.H * sizeof(Acc));
    const size_t car = align256((size_t)(g.B + 1) * N * sizeof(Acc));
    const size_t acb = align256((size_t)g.B * (g.T + 1) * g.H * sizeof(Acc));
    const size_t uvb = align256((size_t)(2 * N) * sizeof(Acc));
    char* p = base;
    A.colsum = (Acc*)p; p += col;
    A.tcsp = (Acc*)p; p += col;
    A.tLend = (Acc*)p; p += col;
    A.tRend = (Acc*)p; p += col;
    A.tLedge = (Acc*)p; p += edge;
    A.tRedge = (Acc*)p; p += edge;
    A.trow = (Acc*)p; p += edge;
    K.cpin = (Acc*)p; p += car;
    K.ain = (Acc*)p; p += car;
    K.Lin = (Acc*)p; p += car;
    K.Rin = (Acc*)p; p += car;
    K.AC = (Acc*)p; p += acb;
    K.U = (Acc*)p; p += uvb;
    K.V = (Acc*)p; p += uvb;
}

}  // namespace inim
