// tile_agg.h -- the tile-local sums of the integral-image pass: one wave
// streams an H x W tile top to bottom (Q adjacent columns per lane) and keeps
// per column the band-local column prefix and its up-left / up-right
// diagonal sums (zero inflow at the tile's edges), and per row the edge
// values and the tile's row-sum prefix (the aggregate pass of k_inim.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "device_common.h"
#include "inim_plan.h"

namespace inim {

template <typename Tin, int Q>
__device__ __forceinline__ void load_tile_row(const Tin* __restrict__ p, bool act, Tin (&v)[Q]) {
    if (act) {
        load_row<Tin, Q>(p, v);
    } else {
#pragma unroll
        for (int e = 0; e < Q; ++e) v[e] = Tin(0);
    }
}

// ------------------------------------------------------------------ pass 1
// Tile-local state of the aggregate pass for one wave: per column, the band-
// local column prefix and the up-left / up-right diagonal sums of it, with
// zero outside the tile.  step() consumes one row of the tile.
template <int Q, typename Acc>
struct TileAgg {
    Acc cp[Q], L[Q], R[Q];
    // per-row outputs parked in lane r % 64, slot r / 64 (H <= 128)
    Acc pk_row[2], pk_le[2], pk_re[2];

    __device__ __forceinline__ void init() {
#pragma unroll
        for (int e = 0; e < Q; ++e) cp[e] = L[e] = R[e] = Acc(0);
#pragma unroll
        for (int k = 0; k < 2; ++k) pk_row[k] = pk_le[k] = pk_re[k] = Acc(0);
    }

    template <typename Tin>
    __device__ __forceinline__ void step(const Tin (&v)[Q], int r, int lane, int lastLane) {
#pragma unroll
        for (int e = 0; e < Q; ++e) cp[e] += to_acc<Acc, Tin>(v[e]);
        Acc upL = shfl_up1(L[Q - 1]);
        Acc dnR = shfl_down1(R[0]);
        if (lane == 0) upL = Acc(0);
        if (lane >= lastLane) dnR = Acc(0);
#pragma unroll
        for (int e = Q - 1; e >= 1; --e) L[e] = cp[e] + L[e - 1];
        L[0] = cp[0] + upL;
#pragma unroll
        for (int e = 0; e < Q - 1; ++e) R[e] = cp[e] + R[e + 1];
        R[Q - 1] = cp[Q - 1] + dnR;
        Acc s = Acc(0);
#pragma unroll
        for (int e = 0; e < Q; ++e) s += cp[e];
        s = bcast(wave_inclusive_scan(s), 63);
        const Acc le = bcast(L[Q - 1], lastLane), re = bcast(R[0], 0);
        if (lane == (r & 63)) {
            if (r < 64) { pk_row[0] = s; pk_le[0] = le; pk_re[0] = re; }
            else        { pk_row[1] = s; pk_le[1] = le; pk_re[1] = re; }
        }
    }

    // per-row edge sums and row sums of the tile, then the band-level outputs:
    // column sums, their in-tile prefix, diagonal sums
    __device__ __forceinline__ void finish(int lane, bool act, int H, const Agg<Acc>& A, size_t ebase, size_t o) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int r = lane + 64 * k;
            if (r < H) {
                A.trow[ebase + r] = pk_row[k];
                A.tLedge[ebase + r] = pk_le[k];
                A.tRedge[ebase + r] = pk_re[k];
            }
        }
        Acc pre[Q];
        Acc run = Acc(0);
#pragma unroll
        for (int e = 0; e < Q; ++e) { run += cp[e]; pre[e] = run; }
        Acc incl = wave_inclusive_scan(run);
        Acc ex = shfl_up1(incl);
        if (lane == 0) ex = Acc(0);
        if (act) {
#pragma unroll
            for (int e = 0; e < Q; ++e) {
                A.colsum[o + e] = cp[e];
                A.tcsp[o + e] = ex + pre[e];
                A.tLend[o + e] = L[e];
                A.tRend[o + e] = R[e];
            }
        }
    }
};

// Rows prefetched ahead: deeper for 16-byte rows per lane.
template <int Q, typename Tin>
constexpr int prefetch_rows() { return Q * sizeof(Tin) >= 16 ? 8 : 4; }

}  // namespace inim
