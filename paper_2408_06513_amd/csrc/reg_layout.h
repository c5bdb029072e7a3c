// reg_layout.h -- the regularisation workspace: its regions and their
// offsets, computed identically on the host (sizes, carving) and on the
// device (the plot table of a batched call).
#pragma once

#include "inim_plan.h"

namespace inim {

constexpr size_t kStatusBytes = 256;
constexpr int kScanThreads = 256, kScanBlock = 4 * kScanThreads;

// The texel sort by rows (rasters with row_sort_fits(N)): kRowTiles sample
// tiles, per-row and per-column LDS counters of at most kRowSortMaxN entries,
// kScanRows rows per block of the tile-count scan.
constexpr int kRowTiles = 256, kRowSortMaxN = 4096, kScanRows = 8;
__host__ __device__ inline bool row_sort_fits(int N) { return N >= 256 && N <= kRowSortMaxN; }
// Rows per block of the per-row sort: consecutive rows are one row-major run
// of texels, so a block takes a group of them, at most 1024 samples on
// average and at most kRowSortMaxN texels (a power of two that divides N).
// Larger groups leave dense rows to fewer, longer blocks.
__host__ __device__ inline int row_group(int64_t n, int N) {
    const int64_t mean = n / N;
    int g = 1;
    while (2 * g * N <= kRowSortMaxN && 2 * g * mean <= 1024) g *= 2;
    return g;
}

// Blocks of the per-block partial sums of an exclusive scan over m words.
__host__ __device__ inline size_t scan_partials(size_t m) { return (m + kScanBlock - 1) / kScanBlock; }

// Byte offsets of the regions of one plot's regularisation workspace.
struct RegLayout {
    // sxy: the samples in texel order, iterated in place; rank: the map
    // between the caller's order and sxy (per sample its rank in its texel,
    // then its slot; or per slot its sample); stage / idx: the samples
    // bucketed by texel row and their indices (row sort only).
    size_t status, counts[2], density, field, defect, scratch, sxy, stage, idx, rank, partial, total;
    Geom g;
    bool f32;  // integral images of the float density in double (radius > 0), or of the counts
};

__host__ __device__ inline RegLayout reg_layout(int32_t res, int64_t n, int radius) {
    RegLayout L;
    const size_t NN = (size_t)res * (size_t)res;
    const size_t nn = n > 0 ? (size_t)n : 0;
    L.f32 = radius > 0;
    L.g = make_geom(res, L.f32 ? 8 : 4);
    size_t o = 0;
    L.status = o; o += kStatusBytes;
    L.counts[0] = o; o += align256(NN * 4);
    L.counts[1] = o; o += align256(NN * 4);
    L.density = o; o += align256(NN * 4);
    L.field = o; o += align256(NN * 8);
    L.defect = o; o += align256(NN * 8);
    L.scratch = o; o += inim_scratch_bytes(L.g, L.f32 ? 8 : 4);
    L.sxy = o; o += align256(nn * 8);
    L.stage = o; o += align256(nn * 8);
    L.idx = o; o += align256(nn * 4);
    L.rank = o; o += align256(nn * 4);
    L.partial = o; o += align256(scan_partials(NN) * 4);
    L.total = o;
    return L;
}

}  // namespace inim
