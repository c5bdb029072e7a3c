// k_inim.hip -- integral images of Sec. 3.1 on gfx950.
//
// Decomposition (sums exact in uint32 or 128-bit fixed point; in double where
// they only feed the deformation):
//   cp(i,j)  column prefix   sum over j' <= j of d(i,j')
//   alpha    row prefix of cp
//   L(i,j)   sum of cp along the up-left diagonal,  L(i,j) = cp(i,j) + L(i-1,j-1)
//   R(i,j)   sum of cp along the up-right diagonal, R(i,j) = cp(i,j) + R(i+1,j-1)
//   alpha_t = L + R - cp  (the wedge j' <= j - |i'-i| split into its left and
//            right halves; these are the paper's "triangle integrals" of Sec. 4.4)
// The other six planes follow from the partitions of Sec. 3.1 and marginals.
//
// Four passes, all fully parallel (no inter-workgroup waiting):
//   1. aggregate  one wave per H x W tile: tile-local column prefixes, diagonal
//                 sums and row sums;
//   2. scan_col   per column, a prefix over bands: column-prefix and alpha carries;
//   3. scan_diag  per diagonal, a prefix over bands: the L and R carries; per
//                 band row, a prefix over tiles: alpha at every tile's left edge;
//   4. final      one wave per tile again: rebuilds cp, alpha, L, R with the
//                 carries (boundary values of the neighbouring tiles come from
//                 the partial sums) and writes the requested planes, or the
//                 deformation of Sec. 4.2 directly.
#include <hip/hip_runtime.h>

#include "batch_plan.h"
#include "blur_tile.h"
#include "device_common.h"
#include "inim_plan.h"
#include "launch.h"
#include "tile_agg.h"

namespace inim {

constexpr int kWavesPerBlock = 4;

// skip_exact (float input, may be null) is cleared when a value is negative
// or not finite: the double sums then need the exact path.
template <typename Tin>
__device__ __forceinline__ bool needs_exact(Tin v) {
    if constexpr (__is_same(Tin, float)) return !(v >= 0.0f && v < __builtin_inff());
    return false;
}

template <int Q, typename Tin, typename Acc>
__global__ __launch_bounds__(256) void k_inim_aggregate(const Tin* __restrict__ img, Geom g, Agg<Acc> A,
                                                        const int* status, int* skip_exact) {
    if (failed(status)) return;
    const int lane = lane_id();
    const int tile = blockIdx.x * kWavesPerBlock + (int)(threadIdx.x >> 6);
    if (tile >= g.B * g.T) return;
    const int b = tile / g.T, c = tile - (tile / g.T) * g.T;
    const int x0 = lane * Q;
    const bool act = lane <= g.lastLane;
    const size_t N = (size_t)g.N;
    const int col = c * g.W + x0;
    const Tin* src = img + (size_t)b * g.H * N + col;
    const size_t ebase = ((size_t)b * g.T + c) * g.H;

    TileAgg<Q, Acc> st;
    st.init();
    constexpr int PF = prefetch_rows<Q, Tin>();
    Tin buf[PF][Q];
#pragma unroll
    for (int p = 0; p < PF; ++p)
        if (p < g.H) load_tile_row<Tin, Q>(src + (size_t)p * N, act, buf[p]);

    bool odd = false;
    for (int r0 = 0; r0 < g.H; r0 += PF) {
#pragma unroll
        for (int p = 0; p < PF; ++p) {
            const int r = r0 + p;
            if (r < g.H) {
                Tin v[Q];
#pragma unroll
                for (int e = 0; e < Q; ++e) {
                    v[e] = buf[p][e];
                    if (skip_exact != nullptr) odd |= needs_exact(v[e]);
                }
                if (r + PF < g.H) load_tile_row<Tin, Q>(src + (size_t)(r + PF) * N, act, buf[p]);
                st.step(v, r, lane, g.lastLane);
            }
        }
    }
    if (skip_exact != nullptr && __any(odd) && lane == 0) *skip_exact = 0;
    st.finish(lane, act, g.H, A, ebase, (size_t)b * N + col);
}

// Blur fused with pass 1 for 64 x 16 tiles (g.W == 64, g.H == 16, N >= 64):
// the block blurs one tile of counts (blur_tile.h), writes the density and
// keeps the tile in LDS, optionally zeroes the same texels of the next
// iteration's count raster, then its first wave runs the aggregate over the
// tile rows from LDS.
// Kernel bodies take their block coordinates explicitly: the single-raster
// kernels pass blockIdx, the batched kernels of a scatterplot matrix pass the
// block's place among the blocks of its plot.
template <typename Acc>
__device__ __forceinline__ void blur_aggregate_body(const uint32_t* __restrict__ counts, float* __restrict__ density,
                                                    uint32_t* __restrict__ zero_next, const BlurTaps& taps,
                                                    const Geom& g, const Agg<Acc>& A, float* lds,
                                                    float (&tile)[kBY][kBX], int bx, int by) {
    const int N = g.N;
    const int ox = bx * kBX, oy = by * kBY;
    blur_tile(counts, N, taps, ox, oy, lds, [&](int row, int cc, float v) {
        const size_t k = (size_t)(oy + row) * N + ox + cc;
        density[k] = v;
        tile[row][cc] = v;
        if (zero_next != nullptr) zero_next[k] = 0u;
    });
    __syncthreads();
    const int lane = lane_id(), wave = (int)(threadIdx.x >> 6);
    const int b = by, c = bx;
    const size_t ebase = ((size_t)b * g.T + c) * g.H;
    const size_t o = (size_t)b * N + ox + lane;
    if (wave == 0) {
        // column prefixes and the up-left diagonal sums, row by row; the edge
        // value of row r is parked in lane r and stored once at the end
        Acc cp = Acc(0), L = Acc(0), eL = Acc(0);
#pragma unroll
        for (int r = 0; r < kBY; ++r) {
            cp += (Acc)tile[r][lane];
            Acc upL = shfl_up1(L);
            if (lane == 0) upL = Acc(0);
            L = cp + upL;
            const Acc l63 = bcast(L, 63);
            if (lane == r) eL = l63;
        }
        if (lane < kBY) A.tLedge[ebase + lane] = eL;
        const Acc incl = wave_inclusive_scan(cp);
        A.colsum[o] = cp;
        A.tcsp[o] = incl;
        A.tLend[o] = L;
    } else if (wave == 2) {
        // the same column prefixes and the up-right diagonal sums
        Acc cp = Acc(0), R = Acc(0), eR = Acc(0);
#pragma unroll
        for (int r = 0; r < kBY; ++r) {
            cp += (Acc)tile[r][lane];
            Acc dnR = shfl_down1(R);
            if (lane == 63) dnR = Acc(0);
            R = cp + dnR;
            const Acc r0 = bcast(R, 0);
            if (lane == r) eR = r0;
        }
        if (lane < kBY) A.tRedge[ebase + lane] = eR;
        A.tRend[o] = R;
    } else if (wave == 1) {
        // trow(r) = sum over the tile of the band-local column prefix at row r,
        // i.e. the prefix over rows of the tile's row sums
        Acc rs = Acc(0);
        if (lane < kBY)
            for (int x = 0; x < kBX; ++x) rs += (Acc)tile[lane][(x + lane) & (kBX - 1)];
        const Acc tr = wave_inclusive_scan(rs);
        if (lane < kBY) A.trow[ebase + lane] = tr;
    }
}

template <typename Acc>
__global__ __launch_bounds__(256) void k_blur_aggregate(const uint32_t* __restrict__ counts, float* __restrict__ density,
                                                        uint32_t* __restrict__ zero_next, BlurTaps taps, Geom g,
                                                        Agg<Acc> A, const int* status) {
    extern __shared__ __align__(16) float lds[];  // read as float4 by the blur
    __shared__ float tile[kBY][kBX];
    if (failed(status)) return;
    blur_aggregate_body<Acc>(counts, density, zero_next, taps, g, A, lds, tile, blockIdx.x, blockIdx.y);
}

// ------------------------------------------------------------------ passes 2 and 3
// The carries are prefix sums over bands.  Each workgroup takes 64 chains
// (one per lane) and spreads the B bands over its waves, kScanWaves at most,
// P = ceil(B / waves) consecutive bands per wave: every wave loads its terms
// at once, sums them in registers, publishes its total in LDS, and adds the
// totals of the waves above it.  One round of loads, one barrier.
constexpr int kScanWaves = 16;
constexpr int kScanMaxP = 16;  // B <= kScanWaves * kScanMaxP = 256

__host__ __device__ inline int scan_waves(int B) { return B < kScanWaves ? B : kScanWaves; }
__host__ __device__ inline int scan_per_wave(int B) { return (B + scan_waves(B) - 1) / scan_waves(B); }

// Pass 2, per column i: cpin[b][i] = column prefix above band b,
// ain[b][i] = alpha(i, bH-1), which grows per band by the full-row prefix of
// the band's column sums: the in-tile prefix tcsp plus the totals of the tiles
// to the left (a wave-wide sum; tiles are at least 64 columns wide, so all
// lanes of a wave lie in one tile, or N < 64 and there is one tile).
// Blocks of 64 * waves threads, waves >= scan_waves(g.B); extra waves only
// take part in the barriers.
template <typename Acc>
__device__ __forceinline__ void scan_col_body(const Geom& g, const Agg<Acc>& A, const Carry<Acc>& K, Acc* tot,
                                              Acc* left, int bx) {
    const int lane = lane_id();
    const int wave = (int)(threadIdx.x >> 6);
    const int nw = scan_waves(g.B), P = scan_per_wave(g.B);
    const int i = bx * 64 + lane;
    const bool valid = i < g.N;
    const int ii = valid ? i : 0;
    const int c = (bx * 64) / g.W;  // the block's 64 columns lie in one tile
    const size_t N = (size_t)g.N;
    // the wave's column terms are loaded first, so that their latency overlaps
    // the tile-total phase below (for 128-bit accumulators they are loaded in
    // rounds further down)
    constexpr int PL = sizeof(Acc) <= 8 ? kScanMaxP : 1;
    Acc cs[PL], tc[PL];
    if constexpr (sizeof(Acc) <= 8) {
        const int b0 = wave * P;
#pragma unroll
        for (int k = 0; k < PL; ++k) {
            cs[k] = Acc(0);
            tc[k] = Acc(0);
            const int b = b0 + k;
            if (k < P && b < g.B && valid) {
                cs[k] = A.colsum[(size_t)b * N + ii];
                tc[k] = A.tcsp[(size_t)b * N + ii];
            }
        }
    }
    // left[b]: the totals of the tiles left of c in band b, one (band, tile)
    // pair per thread (tiles q, q + 16, ... in 16-lane row slot q), summed
    // over each 16-lane row by row shifts; the loop is uniform over the block,
    // so every lane takes part in the lane moves
    for (int base = 0; base < g.B * 16; base += blockDim.x) {
        const int e = base + (int)threadIdx.x;
        const int b = e >> 4, q = e & 15;
        Acc t = Acc(0);
        if (b < g.B) {
            const Acc* tr = A.trow + (size_t)b * g.T * g.H + (g.H - 1);
            for (int cc = q; cc < c; cc += 16) t += tr[(size_t)cc * g.H];
        }
        t += dpp<kDppRowShr1>(t);
        t += dpp<kDppRowShr2>(t);
        t += dpp<kDppRowShr4>(t);
        t += dpp<kDppRowShr8>(t);
        if (q == 15 && b < g.B) left[b] = t;
    }
    __syncthreads();

    if constexpr (sizeof(Acc) <= 8) {
        // all P bands of the wave at once: wave w holds bands [w P, w P + P)
        const int b0 = wave * P;
        Acc da[kScanMaxP];
#pragma unroll
        for (int k = 0; k < kScanMaxP; ++k) {
            const int b = b0 + k;
            da[k] = (k < P && b < g.B && valid) ? tc[k] + left[b] : Acc(0);
        }
        Acc rc = Acc(0), ra = Acc(0);
#pragma unroll
        for (int k = 0; k < kScanMaxP; ++k) { rc += cs[k]; ra += da[k]; }
        tot[(wave * 2 + 0) * 64 + lane] = rc;
        tot[(wave * 2 + 1) * 64 + lane] = ra;
        __syncthreads();
        Acc oc = Acc(0), oa = Acc(0);
        for (int w = 0; w < wave; ++w) {
            oc += tot[(w * 2 + 0) * 64 + lane];
            oa += tot[(w * 2 + 1) * 64 + lane];
        }
        if (!valid) return;
#pragma unroll
        for (int k = 0; k < kScanMaxP; ++k) {
            const int b = b0 + k;
            if (k < P && b < g.B) {
                K.cpin[(size_t)b * N + ii] = oc;
                K.ain[(size_t)b * N + ii] = oa;
                oc += cs[k];
                oa += da[k];
            }
        }
        if (wave == nw - 1) {
            K.cpin[(size_t)g.B * N + ii] = oc;
            K.ain[(size_t)g.B * N + ii] = oa;
        }
        return;
    }
    // 128-bit accumulators: the bands in rounds of nw * pc, 8 per wave and
    // round so that the terms stay in registers; in round q wave w holds the
    // pc bands from (q nw + w) pc, after the running totals of the earlier
    // rounds (exact integers: the grouping does not change the sums).
    constexpr int PC = 8;
    const int pc = P < PC ? P : PC, rounds = (P + pc - 1) / pc;
    Acc carry_c = Acc(0), carry_a = Acc(0);  // totals of the earlier rounds
    Acc oc = Acc(0), oa = Acc(0);
    for (int q = 0; q < rounds; ++q) {
        const int b0 = (q * nw + wave) * pc;
        Acc cs[PC], da[PC];
#pragma unroll
        for (int k = 0; k < PC; ++k) {
            cs[k] = Acc(0);
            da[k] = Acc(0);
            const int b = b0 + k;
            if (k < pc && b < g.B && valid) {
                cs[k] = A.colsum[(size_t)b * N + ii];
                da[k] = A.tcsp[(size_t)b * N + ii] + left[b];
            }
        }
        Acc rc = Acc(0), ra = Acc(0);
#pragma unroll
        for (int k = 0; k < PC; ++k) { rc += cs[k]; ra += da[k]; }
        tot[(wave * 2 + 0) * 64 + lane] = rc;
        tot[(wave * 2 + 1) * 64 + lane] = ra;
        __syncthreads();
        oc = carry_c;
        oa = carry_a;
        for (int w = 0; w < wave; ++w) {
            oc += tot[(w * 2 + 0) * 64 + lane];
            oa += tot[(w * 2 + 1) * 64 + lane];
        }
        if (rounds > 1) {
            for (int w = 0; w < nw; ++w) {
                carry_c += tot[(w * 2 + 0) * 64 + lane];
                carry_a += tot[(w * 2 + 1) * 64 + lane];
            }
            __syncthreads();  // tot is rewritten by the next round
        }
#pragma unroll
        for (int k = 0; k < PC; ++k) {
            const int b = b0 + k;
            if (k < pc && b < g.B) {
                if (valid) {
                    K.cpin[(size_t)b * N + ii] = oc;
                    K.ain[(size_t)b * N + ii] = oa;
                }
                oc += cs[k];
                oa += da[k];
            }
        }
    }
    // the last wave's running sums after the last round are the column totals
    if (valid && wave == nw - 1) {
        K.cpin[(size_t)g.B * N + ii] = oc;
        K.ain[(size_t)g.B * N + ii] = oa;
    }
}

template <typename Acc>
__global__ __launch_bounds__(1024) void k_inim_scan_col(Geom g, Agg<Acc> A, Carry<Acc> K, const int* status) {
    extern __shared__ unsigned char smem_raw[];
    __shared__ Acc left[kScanWaves * kScanMaxP];  // per band: totals of the tiles left of c
    if (failed(status)) return;
    scan_col_body<Acc>(g, A, K, reinterpret_cast<Acc*>(smem_raw), left, blockIdx.x);
}

// Pass 3.  blockIdx.y = 0 follows the up-left chains s = t - N (columns
// i = s + (b+1)H), blockIdx.y = 1 the up-right chains s = t (columns
// i = s - (b+1)H), t = 0..2N:
//   Lin[b+1][i] = sum_{k<H} cp(i-k, bH+H-1-k) + Lin[b][i-H]
//   Rin[b+1][i] = sum_{k<H} cp(i+k, bH+H-1-k) + Rin[b][i+H]
// Inside band b, cp = cpin[b] + the band-local prefix: the cpin part is a
// window of cpin (a difference of ain), the band-local part is tLend / tRend
// plus, near a tile edge, the neighbouring tile's edge sum.  Positions of a
// chain outside the raster contribute zero, so the chain value is a plain
// prefix sum over b.
// blockIdx.y = 2: one thread per raster row j = bH + r accumulates over the
// tiles of its band AC[b][c][r] = alpha(cW-1, j) = ain[b][cW-1] + sum over
// c' < c of trow[b][c'][r], for c = 0..T.
template <typename Acc>
__device__ __forceinline__ void scan_diag_body(const Geom& g, const Agg<Acc>& A, const Carry<Acc>& K, Acc* tot,
                                               int bx, int by) {
    const int N = g.N, H = g.H, W = g.W, T = g.T;
    if (by == 2) {
        // S consecutive lanes per raster row j, each taking GT tiles: the lane
        // loads its tiles' terms at once (one round of memory latency; the
        // stores could alias the loads as far as the compiler knows, so a
        // load-add-store loop would wait for memory once per tile), then adds
        // the totals of the row's earlier segments (a scan over the S lanes)
        // before storing.  GT = 32 / sizeof(Acc) x 4 keeps the terms in
        // registers; S = T / GT is a power of two of at most 64.
        constexpr int GT = sizeof(Acc) >= 16 ? 4 : (sizeof(Acc) == 8 ? 8 : 16);
        const int S = (T + GT - 1) / GT;
        const int lane = lane_id();
        const int64_t pairs = (int64_t)N * S;
        const int64_t stride = (int64_t)((2 * N + 1 + 63) / 64) * blockDim.x;  // this raster's blocks of the slice
        // every lane of a wave runs the same trips (the scan moves data between lanes)
        for (int64_t base = (int64_t)bx * blockDim.x + (threadIdx.x & ~63u); base < pairs; base += stride) {
            const int64_t t = base + lane;
            const bool live = t < pairs;
            const int j = live ? (int)(t / S) : 0, seg = live ? (int)(t - (int64_t)j * S) : 0;
            const int b = j / H, r = j - b * H;
            const Acc* ainb = K.ain + (size_t)b * N;
            const Acc* tr = A.trow + (size_t)b * T * H + r;
            Acc* ac = K.AC + (size_t)b * (T + 1) * H + r;
            const int c0 = 1 + seg * GT;
            Acc tv[GT], av[GT];
            Acc tot = Acc(0);
#pragma unroll
            for (int k = 0; k < GT; ++k) {
                const int c = c0 + k;
                const bool in = live && c <= T;
                const int cc = in ? c : 1;  // loads at a valid index, used only where `in`
                const Acc t_ = tr[(size_t)(cc - 1) * H], a_ = ainb[cc * W - 1];
                tv[k] = in ? t_ : Acc(0);
                av[k] = in ? a_ : Acc(0);
            }
#pragma unroll
            for (int k = 0; k < GT; ++k) tot += tv[k];
            Acc incl = tot;  // inclusive scan of the segment totals over the row's S lanes
            for (int d = 1; d < S; d <<= 1) {
                const Acc o = shfl_up(incl, d);
                if (seg >= d) incl += o;
            }
            Acc run = incl - tot;
            if (live) {
                if (seg == 0) ac[0] = Acc(0);
#pragma unroll
                for (int k = 0; k < GT; ++k) {
                    const int c = c0 + k;
                    if (c <= T) {
                        run += tv[k];
                        ac[(size_t)c * H] = av[k] + run;
                    }
                }
            }
        }
        return;
    }
    const int lane = lane_id();
    const int wave = (int)(threadIdx.x >> 6);
    const int nw = scan_waves(g.B), P = scan_per_wave(g.B);
    const int t = bx * 64 + lane;
    const bool left_chain = by == 0;
    const bool tval = t <= 2 * N;
    const int s = left_chain ? t - N : t;
    Acc* out = left_chain ? K.Lin : K.Rin;
    if (wave == 0 && tval && t < N) out[t] = Acc(0);

    // 128-bit accumulators: bands in rounds as in the column scan (8 per wave
    // and round); the others take all P at once (wave w: bands [w P, w P + P))
    constexpr int PC = sizeof(Acc) > 8 ? 8 : kScanMaxP;
    const int pc = sizeof(Acc) > 8 && P > PC ? PC : P;
    const int rounds = sizeof(Acc) > 8 ? (P + pc - 1) / pc : 1;
    Acc carry = Acc(0);  // the chain's sum over the earlier rounds
    for (int q = 0; q < rounds; ++q) {
    const int b0 = (q * nw + wave) * pc;
    Acc term[PC];
    int col[PC];
    if constexpr (sizeof(Acc) <= 8) {
        // the four loads of every term of a group of 4 bands are issued at
        // clamped (always valid) indices before any is used, so the wave
        // waits for memory once per group (once at most rasters), not once
        // per band; then the terms are formed as below
        constexpr int KG = 4;
#pragma unroll
        for (int kc = 0; kc < PC; kc += KG) {
            if (kc >= pc) {  // uniform: the wave's bands end here
#pragma unroll
                for (int u = 0; u < KG; ++u) {
                    term[kc + u] = Acc(0);
                    col[kc + u] = -1;
                }
                continue;
            }
            // keeps the next group's loads behind this group's use of its own
            // (so that only one group's terms are held in registers)
            asm volatile("" ::: "memory");
            Acc a1[KG], a2[KG], lt[KG], ed[KG];
            bool has2[KG], hasE[KG];
#pragma unroll
            for (int u = 0; u < KG; ++u) {
                const int k = kc + u, b = b0 + k;
                const int i = left_chain ? s + (b + 1) * H : s - (b + 1) * H;
                const bool ok = tval && k < pc && b < g.B && i >= 0 && i < N;
                col[k] = ok ? i : -1;
                const int ii = ok ? i : 0, bb = ok ? b : 0;
                const int c = ii / W, x = ii - c * W;
                const Acc* ainb = K.ain + (size_t)bb * N;
                int i1, i2, ie;
                if (left_chain) {
                    i1 = ii;
                    has2[u] = ii >= H;
                    i2 = has2[u] ? ii - H : 0;
                    hasE[u] = x < H - 1 && c > 0;
                    ie = hasE[u] ? (int)(((size_t)bb * T + (c - 1)) * H + (H - 2 - x)) : 0;
                } else {
                    i1 = (ii + H - 1 < N - 1) ? ii + H - 1 : N - 1;
                    has2[u] = ii >= 1;
                    i2 = has2[u] ? ii - 1 : 0;
                    hasE[u] = x > W - H && c < T - 1;
                    ie = hasE[u] ? (int)(((size_t)bb * T + (c + 1)) * H + (H - 2 - (W - 1 - x))) : 0;
                }
                a1[u] = ainb[i1];
                a2[u] = ainb[i2];
                lt[u] = (left_chain ? A.tLend : A.tRend)[(size_t)bb * N + ii];
                ed[u] = (left_chain ? A.tLedge : A.tRedge)[ie];
            }
#pragma unroll
            for (int u = 0; u < KG; ++u) {
                Acc v = a1[u] - (has2[u] ? a2[u] : Acc(0));
                v += lt[u];
                if (hasE[u]) v += ed[u];
                term[kc + u] = col[kc + u] >= 0 ? v : Acc(0);
            }
        }
    } else {
#pragma unroll
    for (int k = 0; k < PC; ++k) {
        term[k] = Acc(0);
        col[k] = -1;
        const int b = b0 + k;
        if (!(tval && k < pc && b < g.B)) continue;
        const int i = left_chain ? s + (b + 1) * H : s - (b + 1) * H;
        if (i < 0 || i >= N) continue;
        col[k] = i;
        const Acc* ainb = K.ain + (size_t)b * N;
        const int c = i / W, x = i - c * W;
        Acc v;
        if (left_chain) {
            v = ainb[i] - (i >= H ? ainb[i - H] : Acc(0));
            v += A.tLend[(size_t)b * N + i];
            if (x < H - 1 && c > 0) v += A.tLedge[((size_t)b * T + (c - 1)) * H + (H - 2 - x)];
        } else {
            const int hi = (i + H - 1 < N - 1) ? i + H - 1 : N - 1;
            v = ainb[hi] - (i >= 1 ? ainb[i - 1] : Acc(0));
            v += A.tRend[(size_t)b * N + i];
            if (x > W - H && c < T - 1) v += A.tRedge[((size_t)b * T + (c + 1)) * H + (H - 2 - (W - 1 - x))];
        }
        term[k] = v;
    }
    }
    Acc run = Acc(0);
#pragma unroll
    for (int k = 0; k < PC; ++k) run += term[k];
    tot[wave * 64 + lane] = run;
    __syncthreads();
    Acc off = carry;
    for (int w = 0; w < wave; ++w) off += tot[w * 64 + lane];
    if (rounds > 1) {
        for (int w = 0; w < nw; ++w) carry += tot[w * 64 + lane];
        __syncthreads();  // tot is rewritten by the next round
    }
#pragma unroll
    for (int k = 0; k < PC; ++k) {
        off += term[k];
        if (col[k] >= 0) out[(size_t)(b0 + k + 1) * N + col[k]] = off;
    }
    }
}

template <typename Acc>
__global__ __launch_bounds__(1024) void k_inim_scan_diag(Geom g, Agg<Acc> A, Carry<Acc> K, const int* status) {
    extern __shared__ unsigned char smem_raw[];
    if (failed(status)) return;
    scan_diag_body<Acc>(g, A, K, reinterpret_cast<Acc*>(smem_raw), blockIdx.x, blockIdx.y);
}

// ------------------------------------------------------------------ marginals
// Both cases of each marginal read their terms from the same few arrays; the
// loads are issued at clamped (always valid) indices before the case is
// chosen, so that one marginal costs one round of memory latency, and the
// terms are then added in the same order as the case's formula.
// U(u) = sum over i'+j' <= u:  for u < N it is R(0, u); beyond, R(u-N+1, N-1)
// misses exactly the columns left of u-N+1, i.e. X(u-N).
template <typename Acc>
__device__ __forceinline__ Acc marg_U(const Geom& g, const Agg<Acc>& A, const Carry<Acc>& K, int u) {
    const int N = g.N;
    const bool lo = u <= N - 1;
    const int b = lo ? u / g.H : g.B, r = lo ? u - (u / g.H) * g.H : 0;
    const int ia = lo ? r : u - N;           // column of the alpha carry
    const int ir = lo ? r + 1 : u - N + 1;   // column of the up-right carry
    const bool has_r = !lo || r + 1 < N;
    const Acc a = K.ain[(size_t)b * N + ia];
    const Acc rin = K.Rin[(size_t)b * N + (has_r ? ir : 0)];
    const Acc e = A.tRedge[((size_t)(lo ? b : 0) * g.T) * g.H + r];
    if (lo) {
        Acc v = a + e;
        if (has_r) v += rin;
        return v;
    }
    return rin + a;
}

// V(v) = sum over i'-j' >= v:  for v >= 0 it is L(N-1, N-1-v); below, L(N-1+v, N-1)
// misses exactly the columns right of N-1+v, i.e. C - X(N-1+v).
template <typename Acc>
__device__ __forceinline__ Acc marg_V(const Geom& g, const Agg<Acc>& A, const Carry<Acc>& K, int v) {
    const int N = g.N;
    const bool lo = v >= 0;
    const int j = lo ? N - 1 - v : 0;
    const int b = lo ? j / g.H : g.B, r = lo ? j - (j / g.H) * g.H : 0;
    const int m = lo ? N - 2 - r : N - 1 + v;  // column of the second alpha term and the up-left carry
    const Acc* ainb = K.ain + (size_t)b * N;
    const Acc a1 = ainb[N - 1];
    const Acc a2 = ainb[m >= 0 ? m : 0];
    const Acc lin = K.Lin[(size_t)b * N + (m >= 0 ? m : 0)];
    const Acc e = A.tLedge[((size_t)(lo ? b : 0) * g.T + (g.T - 1)) * g.H + r];
    if (lo) {
        Acc val = a1 - (m >= 0 ? a2 : Acc(0));
        val += e;
        if (m >= 0) val += lin;
        return val;
    }
    return lin + (a1 - a2);
}

// Y(j) = alpha(N-1, j), the last entry of the band row's alpha carries.
template <typename Acc>
__device__ __forceinline__ Acc marg_Y(const Geom& g, const Carry<Acc>& K, int j) {
    const int b = j / g.H, r = j - b * g.H;
    return K.AC[((size_t)b * (g.T + 1) + g.T) * g.H + r];
}

// The diagonal marginals U and V into the carry arrays (used by the final
// pass), and, when `marg` is not null, all marginals as doubles.
template <typename Acc>
__device__ __forceinline__ void marg_body(const Geom& g, const Agg<Acc>& A, const Carry<Acc>& K, double* marg, int bx) {
    const int o = bx * blockDim.x + threadIdx.x;
    const int N = g.N, M = 2 * N - 1;
    if (o >= 2 * N + 2 * M + 1) return;
    Acc v;
    if (o < N) {
        v = K.ain[(size_t)g.B * N + o];
    } else if (o < 2 * N) {
        v = marg_Y(g, K, o - N);
    } else if (o < 2 * N + M) {
        v = marg_U(g, A, K, o - 2 * N);
        K.U[o - 2 * N] = v;
    } else if (o < 2 * N + 2 * M) {
        v = marg_V(g, A, K, (o - 2 * N - M) - (N - 1));
        K.V[o - 2 * N - M] = v;
    } else {
        v = K.ain[(size_t)g.B * N + (N - 1)];
    }
    if (marg != nullptr) marg[o] = to_f64(v);
}

template <typename Acc>
__global__ __launch_bounds__(256) void k_inim_marg(Geom g, Agg<Acc> A, Carry<Acc> K, double* marg, const int* status) {
    if (failed(status)) return;
    marg_body<Acc>(g, A, K, marg, blockIdx.x);
}

// ------------------------------------------------------------------ pass 4
enum { kModePlanes = 0, kModeDeform = 1 };

// FIXMASK != 0 fixes the plane mask at compile time; FULL promises that all
// 64 lanes are active (W == 64 Q) and that H is a multiple of the prefetch
// depth, so the row loop has no per-row or per-plane branches.
template <int Q, typename Tin, typename Acc, int MODE, uint32_t FIXMASK = 0, bool FULL = false>
__global__ __launch_bounds__(256) void k_inim_final(const Tin* __restrict__ img, Geom g, Agg<Acc> A, Carry<Acc> K,
                                                    uint32_t mask_arg, Tin* __restrict__ planes,
                                                    float2* __restrict__ field, const float2* __restrict__ t1,
                                                    double d0, const int* status) {
    extern __shared__ unsigned char smem_raw[];
    if (failed(status)) return;
    const int lane = lane_id();
    const int wave = (int)(threadIdx.x >> 6);
    const int tile = blockIdx.x * kWavesPerBlock + wave;
    if (tile >= g.B * g.T) return;
    const int N = g.N, H = g.H, W = g.W, T = g.T;
    // planes: bands bottom-up, the reverse of the aggregate pass, so that the
    // first rows read again are the ones the aggregate pass read last (still
    // in the last-level cache when the raster is larger than it)
    const int b = MODE == kModePlanes ? (g.B - 1) - tile / T : tile / T;
    const int c = tile - (tile / T) * T;
    const int x0 = lane * Q;
    const bool act = FULL || lane <= g.lastLane;
    const uint32_t mask = FIXMASK ? FIXMASK : mask_arg;
    const int cW = c * W;
    const int col = cW + x0;
    const size_t NN = (size_t)N * (size_t)N;
    const Acc* ainb = K.ain + (size_t)b * N;
    const Acc* Linb = K.Lin + (size_t)b * N;
    const Acc* Rinb = K.Rin + (size_t)b * N;

    const bool needUV = (MODE == kModeDeform) || (mask & (INIM_BETA_T | INIM_GAMMA_T | INIM_DELTA_T));
    const bool needY = (MODE == kModeDeform) || (mask & (INIM_GAMMA | INIM_DELTA));

    // Per-row boundary values, row r held by lane r % 64 in slot r / 64:
    //   LB(r) = L(cW-1, bH+r), RB(r) = R(cW+W, bH+r), AC(r) = alpha(cW-1, bH+r),
    //   YV(r) = alpha(N-1, bH+r).
    Acc LBv[2], RBv[2], ACv[2], YVv[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int r = lane + 64 * k;
        Acc lb = Acc(0), rb = Acc(0), ac = Acc(0), yv = Acc(0);
        if (r < H) {
            const size_t eb = (size_t)b * T * H;
            const Acc* acb = K.AC + (size_t)b * (T + 1) * H + r;
            ac = acb[(size_t)c * H];
            if (needY) yv = acb[(size_t)T * H];
            if (c > 0) {
                const int m = cW - 2 - r;
                lb = ainb[cW - 1] - (m >= 0 ? ainb[m] : Acc(0));
                lb += A.tLedge[eb + (size_t)(c - 1) * H + r];
                if (m >= 0) lb += Linb[m];
            }
            if (c < T - 1) {
                const int m = cW + W + r;
                rb = ainb[m] - ainb[cW + W - 1];
                rb += A.tRedge[eb + (size_t)(c + 1) * H + r];
                if (m + 1 < N) rb += Rinb[m + 1];
            }
        }
        LBv[k] = lb; RBv[k] = rb; ACv[k] = ac; YVv[k] = yv;
    }

    // U and V over the tile's anti-diagonals u0..u0+S-1 and diagonals
    // v0..v0+S-1, staged in LDS from the marginal arrays.
    const int S = W + H - 1;
    const int u0 = cW + b * H;
    const int v0 = cW - b * H - (H - 1);
    Acc* Uw = reinterpret_cast<Acc*>(smem_raw) + (size_t)wave * 2 * S;
    Acc* Vw = Uw + S;
    if (needUV) {
        for (int k = lane; k < S; k += 64) {
            Uw[k] = K.U[u0 + k];
            Vw[k] = K.V[v0 + k + N - 1];
        }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");

    const Acc Ctot = K.ain[(size_t)g.B * N + (N - 1)];
    Acc Xv[Q], cp[Q], L[Q], R[Q];
#pragma unroll
    for (int e = 0; e < Q; ++e) {
        Xv[e] = Acc(0); cp[e] = L[e] = R[e] = Acc(0);
        if (act) {
            Xv[e] = K.ain[(size_t)g.B * N + col + e];
            cp[e] = K.cpin[(size_t)b * N + col + e];
            L[e] = Linb[col + e];
            R[e] = Rinb[col + e];
        }
    }
    Acc Lleft = (c > 0) ? Linb[cW - 1] : Acc(0);
    Acc Rright = (cW + W < N) ? Rinb[cW + W] : Acc(0);
    MapScale ms{};
    if constexpr (MODE == kModeDeform) ms = map_scale(to_f64(Ctot), N, d0);

    // output slots of the requested planes
    int slot[8];
    {
        int s = 0;
#pragma unroll
        for (int p = 0; p < 8; ++p) { slot[p] = s; s += (mask >> p) & 1u; }
    }

    const Tin* src = img + (size_t)b * H * N + col;
    constexpr int PF = prefetch_rows<Q, Tin>();
    Tin buf[PF][Q];
#pragma unroll
    for (int p = 0; p < PF; ++p)
        if (p < H) load_tile_row<Tin, Q>(src + (size_t)p * N, act, buf[p]);

    for (int r0 = 0; r0 < H; r0 += PF) {
#pragma unroll
        for (int p = 0; p < PF; ++p) {
            const int r = r0 + p;
            if (FULL || r < H) {
                Tin v[Q];
#pragma unroll
                for (int e = 0; e < Q; ++e) v[e] = buf[p][e];
                if (r + PF < H) {
                    if constexpr (FULL) load_row<Tin, Q>(src + (size_t)(r + PF) * N, buf[p]);
                    else load_tile_row<Tin, Q>(src + (size_t)(r + PF) * N, act, buf[p]);
                }
                const int j = b * H + r;

#pragma unroll
                for (int e = 0; e < Q; ++e) cp[e] += to_acc<Acc, Tin>(v[e]);
                // alpha: row prefix of cp across the tile plus the carry from the left
                Acc pre[Q];
                Acc run = Acc(0);
#pragma unroll
                for (int e = 0; e < Q; ++e) { run += cp[e]; pre[e] = run; }
                Acc incl = wave_inclusive_scan(run);
                Acc ex = shfl_up1(incl);
                if (lane == 0) ex = Acc(0);
                const Acc acr = bcast(pick_row(ACv, r), r & 63);
                Acc al[Q];
#pragma unroll
                for (int e = 0; e < Q; ++e) al[e] = acr + (ex + pre[e]);

                // diagonal sums
                Acc upL = shfl_up1(L[Q - 1]);
                Acc dnR = shfl_down1(R[0]);
                if (lane == 0) upL = Lleft;
                if (lane == g.lastLane) dnR = Rright;
#pragma unroll
                for (int e = Q - 1; e >= 1; --e) L[e] = cp[e] + L[e - 1];
                L[0] = cp[0] + upL;
#pragma unroll
                for (int e = 0; e < Q - 1; ++e) R[e] = cp[e] + R[e + 1];
                R[Q - 1] = cp[Q - 1] + dnR;
                Lleft = bcast(pick_row(LBv, r), r & 63);
                Rright = bcast(pick_row(RBv, r), r & 63);

                Acc at[Q];
#pragma unroll
                for (int e = 0; e < Q; ++e) at[e] = (L[e] + R[e]) - cp[e];

                Acc Yr = Acc(0);
                if (needY) Yr = bcast(pick_row(YVv, r), r & 63);

                if (!act) continue;
                if constexpr (MODE == kModePlanes) {
                    Tin* rowp = planes + (size_t)j * N + col;
                    if (mask & INIM_ALPHA) {
                        Tin o[Q];
#pragma unroll
                        for (int e = 0; e < Q; ++e) o[e] = narrow<Tin, Acc>(al[e]);
                        store_row_nt<Tin, Q>(rowp + slot[0] * NN, o);
                    }
                    if (mask & INIM_ALPHA_T) {
                        Tin o[Q];
#pragma unroll
                        for (int e = 0; e < Q; ++e) o[e] = narrow<Tin, Acc>(at[e]);
                        store_row_nt<Tin, Q>(rowp + slot[4] * NN, o);
                    }
                    if (mask & (INIM_ALL & ~INIM_MIN)) {
                        Tin ob[Q], og[Q], od[Q], obt[Q], ogt[Q], odt[Q];
#pragma unroll
                        for (int e = 0; e < Q; ++e) {
                            const int x = x0 + e;
                            Acc U = Acc(0), V = Acc(0);
                            if (needUV) { U = Uw[x + r]; V = Vw[x - r + H - 1]; }
                            const Compl<Acc> cm = complements<Acc>(al[e], at[e], Xv[e], Yr, U, V, Ctot, cW + x, j, N);
                            ob[e] = narrow<Tin, Acc>(cm.b); og[e] = narrow<Tin, Acc>(cm.g); od[e] = narrow<Tin, Acc>(cm.d);
                            obt[e] = narrow<Tin, Acc>(cm.bt); ogt[e] = narrow<Tin, Acc>(cm.gt); odt[e] = narrow<Tin, Acc>(cm.dt);
                        }
                        if (mask & INIM_BETA) store_row_nt<Tin, Q>(rowp + slot[1] * NN, ob);
                        if (mask & INIM_GAMMA) store_row_nt<Tin, Q>(rowp + slot[2] * NN, og);
                        if (mask & INIM_DELTA) store_row_nt<Tin, Q>(rowp + slot[3] * NN, od);
                        if (mask & INIM_BETA_T) store_row_nt<Tin, Q>(rowp + slot[5] * NN, obt);
                        if (mask & INIM_GAMMA_T) store_row_nt<Tin, Q>(rowp + slot[6] * NN, ogt);
                        if (mask & INIM_DELTA_T) store_row_nt<Tin, Q>(rowp + slot[7] * NN, odt);
                    }
                } else {
                    float2 o[Q], d1[Q];
                    load_row<float, 2 * Q>(reinterpret_cast<const float*>(t1 + (size_t)j * N + col),
                                           reinterpret_cast<float(&)[2 * Q]>(d1));
#pragma unroll
                    for (int e = 0; e < Q; ++e) {
                        const int x = x0 + e;
                        const Acc U = Uw[x + r], V = Vw[x - r + H - 1];
                        const Compl<Acc> cm = complements<Acc>(al[e], at[e], Xv[e], Yr, U, V, Ctot, cW + x, j, N);
                        Planes8 P;
                        P.a = to_f64(al[e]); P.b = to_f64(cm.b); P.g = to_f64(cm.g); P.d = to_f64(cm.d);
                        P.at = to_f64(at[e]); P.bt = to_f64(cm.bt); P.gt = to_f64(cm.gt); P.dt = to_f64(cm.dt);
                        o[e] = deform_texel_defect(P, ms, cW + x, j, d1[e]);
                    }
                    store_field_nt<Q>(field + (size_t)j * N + col, o);
                }
            }
        }
    }
}

// ------------------------------------------------------------------ pass 4, deformation, 64 x 16 tiles
// The final pass of the regularisation for the common tiling (W = 64, Q = 1,
// H = 16, N >= 64, so every lane is active): all 16 input rows and defect
// values are loaded up front and the row loop is fully unrolled without
// branches, so the per-texel map of row r overlaps the scans of row r+1.
// One wave per tile: `tile` is the wave's tile, `wave` its slot in the block's
// LDS (2 (W + H - 1) accumulators per wave).  R0, R1: the wave maps rows
// [R0, R1) of the tile; rows before R0 are only replayed for the column
// prefix and the diagonal chains (the same operations in the same order, so
// splitting a tile over waves gives the same field).
template <typename Tin, typename Acc, int R0 = 0, int R1 = 16>
__device__ __forceinline__ void deform16_body(const Tin* __restrict__ img, const Geom& g, const Agg<Acc>& A,
                                              const Carry<Acc>& K, float2* __restrict__ field,
                                              const float2* __restrict__ t1, double d0, unsigned char* smem_raw,
                                              int tile, int wave) {
    constexpr int H = 16, W = 64;
    const int lane = lane_id();
    if (tile >= g.B * g.T) return;
    const int N = g.N, T = g.T;
    const int b = tile / T, c = tile - (tile / T) * T;
    const int cW = c * W;
    const int col = cW + lane;
    const Acc* ainb = K.ain + (size_t)b * N;
    const Acc* Linb = K.Lin + (size_t)b * N;
    const Acc* Rinb = K.Rin + (size_t)b * N;

    // inputs and defect values of the tile's 16 rows
    Tin v[H];
    float2 d1[H];
    const Tin* src = img + (size_t)b * H * N + col;
    const float2* t1p = t1 + (size_t)b * H * N + col;
#pragma unroll
    for (int r = 0; r < R1; ++r) {
        v[r] = src[(size_t)r * N];
        if (r >= R0) d1[r] = t1p[(size_t)r * N];
    }
    // carries into the tile's columns (loaded together with the rows)
    const Acc Ctot = K.ain[(size_t)g.B * N + (N - 1)];
    const Acc X = K.ain[(size_t)g.B * N + col];
    Acc cp = K.cpin[(size_t)b * N + col];
    Acc L = Linb[col], R = Rinb[col];
    Acc Lleft = (c > 0) ? Linb[cW - 1] : Acc(0);
    Acc Rright = (cW + W < N) ? Rinb[cW + W] : Acc(0);

    // per-row boundary values (lane r holds row r)
    Acc lb = Acc(0), rb = Acc(0), ac = Acc(0), yv = Acc(0);
    if (lane < H) {
        const int r = lane;
        const size_t eb = (size_t)b * T * H;
        const Acc* acb = K.AC + (size_t)b * (T + 1) * H + r;
        ac = acb[(size_t)c * H];
        yv = acb[(size_t)T * H];
        if (c > 0) {
            const int m = cW - 2 - r;
            lb = ainb[cW - 1] - (m >= 0 ? ainb[m] : Acc(0));
            lb += A.tLedge[eb + (size_t)(c - 1) * H + r];
            if (m >= 0) lb += Linb[m];
        }
        if (c < T - 1) {
            const int m = cW + W + r;
            rb = ainb[m] - ainb[cW + W - 1];
            rb += A.tRedge[eb + (size_t)(c + 1) * H + r];
            if (m + 1 < N) rb += Rinb[m + 1];
        }
    }

    // U and V over the tile's anti-diagonals and diagonals, evaluated here from
    // the carries (a few loads each) rather than read from a marginals pass,
    // and staged in LDS
    constexpr int S = W + H - 1;
    const int u0 = cW + b * H;
    const int v0 = cW - b * H - (H - 1);
    Acc* Uw = reinterpret_cast<Acc*>(smem_raw) + (size_t)wave * 2 * S;
    Acc* Vw = Uw + S;
    for (int k = lane; k < S; k += 64) {
        Uw[k] = marg_U(g, A, K, u0 + k);
        Vw[k] = marg_V(g, A, K, v0 + k);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");

    const MapScale ms = map_scale(to_f64(Ctot), N, d0);

#pragma unroll
    for (int r = 0; r < R1; ++r) {
        const int j = b * H + r;
        cp += to_acc<Acc, Tin>(v[r]);
        if (r < R0) {  // replayed row: the chains only
            Acc upL = shfl_up1(L), dnR = shfl_down1(R);
            if (lane == 0) upL = Lleft;
            if (lane == 63) dnR = Rright;
            L = cp + upL;
            R = cp + dnR;
            Lleft = bcast(lb, r);
            Rright = bcast(rb, r);
            continue;
        }
        const Acc incl = wave_inclusive_scan(cp);
        const Acc al = bcast(ac, r) + incl;
        Acc upL = shfl_up1(L), dnR = shfl_down1(R);
        if (lane == 0) upL = Lleft;
        if (lane == 63) dnR = Rright;
        L = cp + upL;
        R = cp + dnR;
        Lleft = bcast(lb, r);
        Rright = bcast(rb, r);
        const Acc at = (L + R) - cp;
        const Acc U = Uw[lane + r], V = Vw[lane - r + H - 1];
        const Compl<Acc> cm = complements<Acc>(al, at, X, bcast(yv, r), U, V, Ctot, col, j, N);
        Planes8 P;
        P.a = to_f64(al); P.b = to_f64(cm.b); P.g = to_f64(cm.g); P.d = to_f64(cm.d);
        P.at = to_f64(at); P.bt = to_f64(cm.bt); P.gt = to_f64(cm.gt); P.dt = to_f64(cm.dt);
        const float2 o[1] = {deform_texel_defect(P, ms, col, j, d1[r])};
        store_field_nt<1>(field + (size_t)j * N + col, o);
    }
}

template <typename Tin, typename Acc>
__global__ __launch_bounds__(256) void k_inim_deform16(const Tin* __restrict__ img, Geom g, Agg<Acc> A, Carry<Acc> K,
                                                       float2* __restrict__ field, const float2* __restrict__ t1,
                                                       double d0, const int* status) {
    extern __shared__ unsigned char smem_raw[];
    if (failed(status)) return;
    const int wave = (int)(threadIdx.x >> 6);
    deform16_body<Tin, Acc>(img, g, A, K, field, t1, d0, smem_raw, blockIdx.x * kWavesPerBlock + wave, wave);
}

// Two waves per tile: the even wave maps rows 0-7, the odd one replays them
// and maps rows 8-15 (twice the waves of k_inim_deform16 for the same field).
template <typename Tin, typename Acc>
__global__ __launch_bounds__(256) void k_inim_deform16x2(const Tin* __restrict__ img, Geom g, Agg<Acc> A,
                                                         Carry<Acc> K, float2* __restrict__ field,
                                                         const float2* __restrict__ t1, double d0, const int* status) {
    extern __shared__ unsigned char smem_raw[];
    if (failed(status)) return;
    const int wave = (int)(threadIdx.x >> 6);
    const int tile = (blockIdx.x * kWavesPerBlock + wave) >> 1;
    if (wave & 1)
        deform16_body<Tin, Acc, 8, 16>(img, g, A, K, field, t1, d0, smem_raw, tile, wave);
    else
        deform16_body<Tin, Acc, 0, 8>(img, g, A, K, field, t1, d0, smem_raw, tile, wave);
}

// ------------------------------------------------------------------ defect field
// t(p; 1) of the constant raster at every texel centre (Sec. 4.2: the defect
// does not depend on the density, so it is computed once per call).
__device__ __forceinline__ void defect_body(int N, float2* __restrict__ t1, int64_t bid) {
    const size_t k = (size_t)bid * blockDim.x + threadIdx.x;
    const size_t NN = (size_t)N * N;
    if (k >= NN) return;
    const int j = (int)(k / N), i = (int)(k - (size_t)j * N);
    t1[k] = defect_texel(i, j, N);
}

__global__ __launch_bounds__(256) void k_defect_field(int N, float2* __restrict__ t1) { defect_body(N, t1, blockIdx.x); }

// ------------------------------------------------------------------ deform from stored planes
template <typename Tin>
__global__ __launch_bounds__(256) void k_deform_planes(const Tin* __restrict__ alpha, const Tin* __restrict__ alpha_t,
                                                       const double* __restrict__ marg, int N, double d0,
                                                       float2* __restrict__ field) {
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t NN = (size_t)N * N;
    if (k >= NN) return;
    const int j = (int)(k / N), i = (int)(k - (size_t)j * N);
    const int M = 2 * N - 1;
    const double al = (double)alpha[k], at = (double)alpha_t[k];
    const double X = marg[i], Y = marg[N + j], U = marg[2 * N + i + j];
    const double V = marg[2 * N + M + (i - j + N - 1)], C = marg[2 * N + 2 * M];
    const Compl<double> cm = complements<double>(al, at, X, Y, U, V, C, i, j, N);
    Planes8 P;
    P.a = al; P.b = cm.b; P.g = cm.g; P.d = cm.d; P.at = at; P.bt = cm.bt; P.gt = cm.gt; P.dt = cm.dt;
    field[k] = deform_texel(P, map_scale(C, N, d0), i, j, N);
}

// ------------------------------------------------------------------ launchers
template <typename Acc>
hipError_t launch_inim_scans(const Geom& g, void* scratch, const int* status, hipStream_t st) {
    Agg<Acc> A;
    Carry<Acc> K;
    carve<Acc>(g, (char*)scratch, A, K);
    const int nw = scan_waves(g.B);
    launch_kernel((k_inim_scan_col<Acc>), dim3((g.N + 63) / 64), dim3(64 * nw), (size_t)nw * 2 * 64 * sizeof(Acc),
                       st, g, A, K, status);
    launch_kernel((k_inim_scan_diag<Acc>), dim3((2 * g.N + 1 + 63) / 64, 3), dim3(64 * nw),
                       (size_t)nw * 64 * sizeof(Acc), st, g, A, K, status);
    return hipGetLastError();
}

bool blur_aggregate_fits(const Geom& g) { return g.W == kBX && g.H == kBY && g.Q == 1 && g.N >= kBX; }

hipError_t launch_blur_aggregate(const uint32_t* counts, float* density, uint32_t* zero_next, int N,
                                 const BlurTaps& taps, const Geom& g, void* scratch, const int* status,
                                 hipStream_t st) {
    if (!blur_aggregate_fits(g) || N != g.N) return hipErrorInvalidValue;
    Agg<double> A;
    Carry<double> K;
    carve<double>(g, (char*)scratch, A, K);
    const size_t smem = sizeof(float) * blur_smem_floats(taps.r);
    launch_kernel((k_blur_aggregate<double>), dim3(N / kBX, N / kBY), dim3(256), smem, st, counts, density,
                       zero_next, taps, g, A, status);
    return hipGetLastError();
}

template <typename Tin, typename Acc, int Q>
static hipError_t launch_aggregate_q(const Tin* img, const Geom& g, void* scratch, const int* status, hipStream_t st,
                                     int* skip_exact) {
    Agg<Acc> A;
    Carry<Acc> K;
    carve<Acc>(g, (char*)scratch, A, K);
    const int tiles = g.B * g.T;
    const dim3 grd((tiles + kWavesPerBlock - 1) / kWavesPerBlock);
    launch_kernel((k_inim_aggregate<Q, Tin, Acc>), grd, dim3(64 * kWavesPerBlock), 0, st, img, g, A, status,
                  skip_exact);
    return hipGetLastError();
}

template <typename Tin, typename Acc>
hipError_t launch_inim_aggregate(const Tin* img, const Geom& g, void* scratch, const int* status, hipStream_t st,
                                 int* skip_exact) {
    switch (g.Q) {
        case 1: return launch_aggregate_q<Tin, Acc, 1>(img, g, scratch, status, st, skip_exact);
        case 2: return launch_aggregate_q<Tin, Acc, 2>(img, g, scratch, status, st, skip_exact);
        case 4: return launch_aggregate_q<Tin, Acc, 4>(img, g, scratch, status, st, skip_exact);
    }
    return hipErrorInvalidValue;
}

__global__ void k_set_word(int* w, int v) { *w = v; }

hipError_t launch_set_word(int* w, int v, hipStream_t st) {
    launch_kernel(k_set_word, dim3(1), dim3(1), 0, st, w, v);
    return hipGetLastError();
}

template <typename Tin, typename Acc>
hipError_t launch_inim_carries(const Tin* img, const Geom& g, void* scratch, const int* status, hipStream_t st) {
    hipError_t e = launch_inim_aggregate<Tin, Acc>(img, g, scratch, status, st);
    if (e == hipSuccess) e = launch_inim_scans<Acc>(g, scratch, status, st);
    return e;
}

template <typename Tin, typename Acc, int Q>
static hipError_t launch_final_q(const Tin* img, const Geom& g, void* scratch, uint32_t mask, Tin* planes,
                                 float2* field, const float2* t1, double d0, double* marg, const int* status,
                                 hipStream_t st) {
    Agg<Acc> A;
    Carry<Acc> K;
    carve<Acc>(g, (char*)scratch, A, K);
    const int tiles = g.B * g.T;
    const dim3 blk(64 * kWavesPerBlock);
    const dim3 grd((tiles + kWavesPerBlock - 1) / kWavesPerBlock);
    const int M = 6 * g.N - 1;
    const bool deform16 = field != nullptr && Q == 1 && g.W == 64 && g.H == 16 && g.N >= 64;
    // the 64 x 16 deformation pass evaluates its own diagonal marginals
    if (!deform16 || marg != nullptr)
        launch_kernel((k_inim_marg<Acc>), dim3((M + 255) / 256), dim3(256), 0, st, g, A, K, marg, status);
    const size_t smem = (size_t)kWavesPerBlock * 2 * (g.W + g.H - 1) * sizeof(Acc);
    if (deform16) {
        const dim3 grd2((2 * tiles + kWavesPerBlock - 1) / kWavesPerBlock);
        launch_kernel((k_inim_deform16x2<Tin, Acc>), grd2, blk, smem, st, img, g, A, K, field, t1, d0, status);
    } else if (field != nullptr) {
        launch_kernel((k_inim_final<Q, Tin, Acc, kModeDeform>), grd, blk, smem, st, img, g, A, K, 0u,
                           (Tin*)nullptr, field, t1, d0, status);
    } else if (mask != 0) {
        const bool needUV = (mask & (INIM_BETA_T | INIM_GAMMA_T | INIM_DELTA_T)) != 0;
        const bool full = g.W == 64 * Q && g.H % prefetch_rows<Q, Tin>() == 0;
        if (full && mask == INIM_ALL)
            launch_kernel((k_inim_final<Q, Tin, Acc, kModePlanes, INIM_ALL, true>), grd, blk, smem, st, img, g, A,
                               K, mask, planes, (float2*)nullptr, (const float2*)nullptr, 0.0, status);
        else if (full && mask == INIM_MIN)
            launch_kernel((k_inim_final<Q, Tin, Acc, kModePlanes, INIM_MIN, true>), grd, blk, 0, st, img, g, A, K,
                               mask, planes, (float2*)nullptr, (const float2*)nullptr, 0.0, status);
        else
            launch_kernel((k_inim_final<Q, Tin, Acc, kModePlanes>), grd, blk, needUV ? smem : 0, st, img, g, A,
                               K, mask, planes, (float2*)nullptr, (const float2*)nullptr, 0.0, status);
    }
    return hipGetLastError();
}

template <typename Tin, typename Acc>
hipError_t launch_inim_final(const Tin* img, const Geom& g, void* scratch, uint32_t mask, Tin* planes, float2* field,
                             const float2* t1, double d0, double* marg, const int* status, hipStream_t st) {
    if (field != nullptr && t1 == nullptr) return hipErrorInvalidValue;
    switch (g.Q) {
        case 1: return launch_final_q<Tin, Acc, 1>(img, g, scratch, mask, planes, field, t1, d0, marg, status, st);
        case 2: return launch_final_q<Tin, Acc, 2>(img, g, scratch, mask, planes, field, t1, d0, marg, status, st);
        case 4: return launch_final_q<Tin, Acc, 4>(img, g, scratch, mask, planes, field, t1, d0, marg, status, st);
    }
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ batched (scatterplot matrix)
// Inclusive sum over lanes 0..lane of a wave (64 lanes, one value each).
template <typename T>
__device__ __forceinline__ T lane_prefix(T v) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const T o = __shfl_up(v, d, 64);
        if (lane_id() >= d) v += o;
    }
    return v;
}

// The plot table, built by one wave with one lane per plot (count <= 64):
// workspace offsets and the first block of every plot in every stage are
// prefix sums over the lanes.
__global__ __launch_bounds__(64) void kb_init(BatchArgs a, BatchTable* __restrict__ T) {
    static_assert(kMaxBatch <= 64, "one lane per plot");
    __shared__ bool own[kMaxBatch];
    const int k = threadIdx.x;
    const bool live = k < a.count;
    const BatchInput in = live ? a.in[k] : BatchInput{nullptr, 0, 2, 0};
    const RegLayout L = reg_layout(in.N, in.n, a.radius);
    const size_t size = live ? L.total : 0;
    const size_t base_off = kStatusBytes + align256(sizeof(BatchTable)) + lane_prefix(size) - size;
    int owner = k;  // the first plot of this raster size holds its defect field
    for (int q = 0; q < k && live; ++q)
        if (a.in[q].N == in.N) { owner = q; break; }
    own[k] = owner == k;
    const size_t owner_off = __shfl(base_off, owner, 64);  // the owner's workspace offset
    if (live) {
        char* base = a.ws + base_off;
        BatchPlot P;
        P.xy = reinterpret_cast<float2*>(in.xy);
        P.n = in.n;
        P.N = in.N;
        P.d0 = a.d0 < 0.0 ? (double)in.n / ((double)in.N * (double)in.N) : a.d0;
        P.g = L.g;
        P.counts[0] = reinterpret_cast<uint32_t*>(base + L.counts[0]);
        P.counts[1] = reinterpret_cast<uint32_t*>(base + L.counts[1]);
        P.density = reinterpret_cast<float*>(base + L.density);
        P.field = reinterpret_cast<float2*>(base + L.field);
        P.defect = reinterpret_cast<float2*>(a.ws + owner_off + L.defect);
        P.defect_owner = owner == k;
        P.sxy = reinterpret_cast<float2*>(base + L.sxy);
        P.stage = reinterpret_cast<float2*>(base + L.stage);
        P.idx = reinterpret_cast<uint32_t*>(base + L.idx);
        P.rank = reinterpret_cast<uint32_t*>(base + L.rank);
        P.partial = reinterpret_cast<uint32_t*>(base + L.partial);
        carve<double>(L.g, base + L.scratch, P.A, P.K);
        T->plot[k] = P;
        T->order[k] = a.order[k];
    }
    if (k == 0) {
        T->count = a.count;
        T->wpb = a.wpb;
    }
    __syncthreads();
    // stage tables in launch order: lane q holds plot order[q]
    const int p = live ? a.order[k] : 0;
    const BatchInput ip = a.in[p];
    for (int s = 0; s < kBStages; ++s) {
        const uint32_t b = live ? batch_stage_blocks(s, ip.N, ip.n, a.wpb, own[p]) : 0u;
        const uint32_t incl = lane_prefix(b);
        if (live) T->first[s][k] = incl - b;
        if (k == a.count - 1) T->first[s][a.count] = incl;
    }
}

__global__ __launch_bounds__(256) void kb_defect(const BatchTable* __restrict__ T) {
    int64_t bid, nblk;
    const BatchPlot& P = batch_locate(T, kBDefect, blockIdx.x, bid, nblk);
    defect_body(P.N, P.defect, bid);
}

__global__ __launch_bounds__(256) void kb_blur_agg(const BatchTable* __restrict__ T, BlurTaps taps, int it, int iters,
                                                   const int* status) {
    extern __shared__ __align__(16) float lds[];  // read as float4 by the blur
    __shared__ float tile[kBY][kBX];
    if (failed(status)) return;
    int64_t bid, nblk;
    const BatchPlot& P = batch_locate(T, kBBlurAgg, blockIdx.x, bid, nblk);
    const int tx = P.N / kBX;
    uint32_t* nxt = (it + 1 < iters) ? P.counts[(it + 1) & 1] : nullptr;
    blur_aggregate_body<double>(P.counts[it & 1], P.density, nxt, taps, P.g, P.A, lds, tile, (int)(bid % tx),
                                (int)(bid / tx));
}

__global__ __launch_bounds__(1024) void kb_scan_col(const BatchTable* __restrict__ T, const int* status) {
    __shared__ double tot[kScanWaves * 2 * 64];
    __shared__ double left[kScanWaves * kScanMaxP];
    if (failed(status)) return;
    int64_t bid, nblk;
    const BatchPlot& P = batch_locate(T, kBScanCol, blockIdx.x, bid, nblk);
    scan_col_body<double>(P.g, P.A, P.K, tot, left, (int)bid);
}

__global__ __launch_bounds__(1024) void kb_scan_diag(const BatchTable* __restrict__ T, const int* status) {
    __shared__ double tot[kScanWaves * 64];
    if (failed(status)) return;
    int64_t bid, nblk;
    const BatchPlot& P = batch_locate(T, kBScanDiag, blockIdx.x, bid, nblk);
    const int tx = (2 * P.N + 1 + 63) / 64;
    scan_diag_body<double>(P.g, P.A, P.K, tot, (int)(bid % tx), (int)(bid / tx));
}

__global__ __launch_bounds__(512) void kb_deform(const BatchTable* __restrict__ T, const int* status) {
    extern __shared__ unsigned char smem_raw[];
    if (failed(status)) return;
    int64_t bid, nblk;
    const BatchPlot& P = batch_locate(T, kBDeform, blockIdx.x, bid, nblk);
    const int wave = (int)(threadIdx.x >> 6);
    deform16_body<float, double>(P.density, P.g, P.A, P.K, P.field, P.defect, P.d0, smem_raw,
                                 (int)bid * T->wpb + wave, wave);
}

hipError_t launch_batch_init(const BatchArgs& a, BatchTable* T, hipStream_t st) {
    hipLaunchKernelGGL(kb_init, dim3(1), dim3(64), 0, st, a, T);
    return hipGetLastError();
}

hipError_t launch_batch_inim(int stage, const BatchTable* T, unsigned blocks, int wpb, const BlurTaps& taps, int it,
                             int iters, const int* status, hipStream_t st) {
    if (blocks == 0) return hipSuccess;
    switch (stage) {
        case kBDefect: hipLaunchKernelGGL(kb_defect, dim3(blocks), dim3(256), 0, st, T); break;
        case kBBlurAgg:
            hipLaunchKernelGGL(kb_blur_agg, dim3(blocks), dim3(256), sizeof(float) * blur_smem_floats(taps.r), st, T,
                               taps, it, iters, status);
            break;
        case kBScanCol: hipLaunchKernelGGL(kb_scan_col, dim3(blocks), dim3(1024), 0, st, T, status); break;
        case kBScanDiag: hipLaunchKernelGGL(kb_scan_diag, dim3(blocks), dim3(1024), 0, st, T, status); break;
        case kBDeform:
            if (wpb < 1 || wpb > 8) return hipErrorInvalidValue;
            hipLaunchKernelGGL(kb_deform, dim3(blocks), dim3(64 * wpb), (size_t)wpb * 2 * (64 + 16 - 1) * sizeof(double),
                               st, T, status);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

#define INIM_INSTANTIATE(TIN, ACC)                                                                                    \
    template hipError_t launch_inim_carries<TIN, ACC>(const TIN*, const Geom&, void*, const int*, hipStream_t);      \
    template hipError_t launch_inim_aggregate<TIN, ACC>(const TIN*, const Geom&, void*, const int*, hipStream_t, int*); \
    template hipError_t launch_inim_scans<ACC>(const Geom&, void*, const int*, hipStream_t);                         \
    template hipError_t launch_inim_final<TIN, ACC>(const TIN*, const Geom&, void*, uint32_t, TIN*, float2*,        \
                                                    const float2*, double, double*, const int*, hipStream_t);
INIM_INSTANTIATE(uint32_t, uint32_t)
INIM_INSTANTIATE(float, u128)
INIM_INSTANTIATE(float, double)
#undef INIM_INSTANTIATE

hipError_t launch_defect_field(int N, float2* t1, hipStream_t st) {
    const size_t NN = (size_t)N * N;
    hipLaunchKernelGGL(k_defect_field, dim3((unsigned)((NN + 255) / 256)), dim3(256), 0, st, N, t1);
    return hipGetLastError();
}

hipError_t launch_deform_planes(const void* alpha, const void* alpha_t, int dt, const double* marg, int N, double d0,
                                float2* field, hipStream_t st) {
    const size_t NN = (size_t)N * N;
    const dim3 grd((unsigned)((NN + 255) / 256));
    if (dt == INIM_U32)
        hipLaunchKernelGGL((k_deform_planes<uint32_t>), grd, dim3(256), 0, st, (const uint32_t*)alpha,
                           (const uint32_t*)alpha_t, marg, N, d0, field);
    else
        hipLaunchKernelGGL((k_deform_planes<float>), grd, dim3(256), 0, st, (const float*)alpha, (const float*)alpha_t,
                           marg, N, d0, field);
    return hipGetLastError();
}

}  // namespace inim
