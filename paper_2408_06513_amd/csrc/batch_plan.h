// batch_plan.h -- one regularisation of many scatterplots at once (the plots
// of a scatterplot matrix, each with its own samples and raster size): every
// stage of the iteration is a single launch whose blocks are divided among
// the plots.  Each plot is processed by exactly the same kernel bodies and
// the same per-plot block decomposition as a call for that plot alone.
#pragma once

#include "reg_layout.h"

namespace inim {

constexpr int kMaxBatch = 64;

enum BatchStage : int {
    kBFill = 0,
    kBSplatRank,
    kBScanReduce,
    kBScanPartials,
    kBScanDown,
    kBScatter,
    kBRowHist,
    kBRowScan,
    kBRowBucket,
    kBRowSort,
    kBDefect,
    kBBlurAgg,
    kBScanCol,
    kBScanDiag,
    kBDeform,
    kBAdvect,
    kBUnpermute,
    kBStages
};

// Blocks of a grid-stride launch over n items, at most `cap`.
__host__ __device__ inline unsigned grid_blocks(int64_t n, int per_block = 256, unsigned cap = 8192) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    return (unsigned)(g > (int64_t)cap ? (int64_t)cap : g);
}

// Blocks of stage s for one plot (the same counts as the single-plot
// launches; the deformation stage with wpb tiles per block).
__host__ __device__ inline unsigned batch_stage_blocks(int s, int N, int64_t n, int wpb, bool defect_owner) {
    const size_t NN = (size_t)N * (size_t)N;
    const bool rows = row_sort_fits(N);  // texel sort by rows (else by global ranks)
    switch (s) {
        case kBFill: return rows ? 1u : grid_blocks((int64_t)(NN / 4 + 1), 256, 2048);
        case kBSplatRank:
        case kBScatter: return rows ? 0u : grid_blocks(n);
        case kBAdvect:
        case kBUnpermute: return grid_blocks(n);
        case kBScanReduce:
        case kBScanDown: return rows ? 0u : (unsigned)scan_partials(NN);
        case kBScanPartials: return rows ? 0u : 1u;
        case kBRowHist:
        case kBRowBucket: return rows ? (unsigned)kRowTiles : 0u;
        case kBRowScan: return rows ? (unsigned)(N / kScanRows) : 0u;
        case kBRowSort: return rows ? (unsigned)(N / row_group(n, N)) : 0u;
        case kBDefect: return defect_owner && !rows ? (unsigned)((NN + 255) / 256) : 0u;
        case kBBlurAgg: return (unsigned)((N / 64) * (N / 16));
        case kBScanCol: return (unsigned)((N + 63) / 64);
        case kBScanDiag: return (unsigned)(((2 * N + 1 + 63) / 64) * 3);
        case kBDeform: return (unsigned)(((N / 16) * (N / 64) + wpb - 1) / wpb);
    }
    return 0;
}

// Per plot: its samples, raster, background and workspace regions.
struct BatchPlot {
    float2* xy;
    int64_t n;
    int N;
    double d0;
    Geom g;
    uint32_t* counts[2];
    float* density;
    float2* field;
    float2* defect;  // t(p; 1), shared by the plots of one raster size
    bool defect_owner;
    float2* sxy;
    float2* stage;  // row sort: the row-bucketed samples and their indices
    uint32_t* idx;
    uint32_t* rank;
    uint32_t* partial;
    Agg<double> A;
    Carry<double> K;
};

// Built on the device at the start of every batched call.  first[s][k] is
// the first block of the k-th plot in launch order (plot order[k]) in the
// launch of stage s; first[s][count] is that launch's block count.
struct BatchTable {
    int count;
    int wpb;  // waves (tiles) per block of the deformation stage
    int order[kMaxBatch];
    uint32_t first[kBStages][kMaxBatch + 1];
    BatchPlot plot[kMaxBatch];
};

// Launch argument of the table-building kernel (passed by value).
struct BatchInput {
    float* xy;
    int64_t n;
    int32_t N;
    int32_t pad;
};
struct BatchArgs {
    char* ws;
    int count;
    int wpb;
    int radius;
    double d0;  // < 0: n / N^2 per plot
    int order[kMaxBatch];
    BatchInput in[kMaxBatch];
};

// Workspace of a batched call: status word, the table, then one
// regularisation workspace per plot (reg_layout) in input order.
__host__ __device__ inline size_t batch_table_offset() { return kStatusBytes; }
__host__ __device__ inline size_t batch_plot_offset(int k, const BatchInput* in, int radius) {
    size_t o = kStatusBytes + align256(sizeof(BatchTable));
    for (int q = 0; q < k; ++q) o += reg_layout(in[q].N, in[q].n, radius).total;
    return o;
}

// The plot and block of a batched launch: finds the k with
// first[s][k] <= blk < first[s][k+1] (uniform across the block).
__device__ __forceinline__ const BatchPlot& batch_locate(const BatchTable* __restrict__ T, int s, uint32_t blk,
                                                        int64_t& bid, int64_t& nblk) {
    int lo = 0, hi = T->count;  // first[s][lo] <= blk < first[s][hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (T->first[s][mid] <= blk) lo = mid;
        else hi = mid;
    }
    bid = (int64_t)(blk - T->first[s][lo]);
    nblk = (int64_t)(T->first[s][lo + 1] - T->first[s][lo]);
    return T->plot[T->order[lo]];
}

}  // namespace inim
