// launch.h -- host-side launchers of the gfx950 kernels (used by the C ABI).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "batch_plan.h"
#include "inim_plan.h"

namespace inim {

constexpr int kMaxRadius = 32;

// Stage timing: while a StageClock is armed on this thread, launches made
// through launch_kernel() go through hipExtLaunchKernelGGL, the first one
// recording `start` when it begins and every one recording `stop` when it
// ends, so the pair brackets exactly the kernels of a stage (no launch
// gaps).  Disarmed (the default), launch_kernel is a plain launch.
struct StageClock {
    hipEvent_t start = nullptr, stop = nullptr;
    bool started = false;
};
StageClock*& stage_clock();

template <typename K, typename... A>
inline void launch_kernel(K kernel, dim3 grid, dim3 block, size_t smem, hipStream_t st, A... args) {
    StageClock* c = stage_clock();
    if (c == nullptr) {
        hipLaunchKernelGGL(kernel, grid, block, smem, st, args...);
        return;
    }
    hipEvent_t s = c->started ? nullptr : c->start;
    c->started = true;
    hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)smem, st, s, c->stop, 0, args...);
}

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
// The two halves of launch_inim_carries: the tile partial sums, then the band scans.
// skip_exact (float rasters, may be null): set to 0 when the raster holds a
// negative or non-finite value.
template <typename Tin, typename Acc>
hipError_t launch_inim_aggregate(const Tin* img, const Geom& g, void* scratch, const int* status, hipStream_t st,
                                 int* skip_exact = nullptr);
// *w = v (one word, on the stream).
hipError_t launch_set_word(int* w, int v, hipStream_t st);
template <typename Acc>
hipError_t launch_inim_scans(const Geom& g, void* scratch, const int* status, hipStream_t st);
// field != nullptr needs t1, the defect field of launch_defect_field.
template <typename Tin, typename Acc>
hipError_t launch_inim_final(const Tin* img, const Geom& g, void* scratch, uint32_t mask, Tin* planes, float2* field,
                             const float2* t1, double d0, double* marg, const int* status, hipStream_t st);
// t1[j*N+i] = t(p; 1), the map of the constant raster at texel (i, j), as floats.
hipError_t launch_defect_field(int N, float2* t1, hipStream_t st);

hipError_t launch_deform_planes(const void* alpha, const void* alpha_t, int dt, const double* marg, int N, double d0,
                                float2* field, hipStream_t st);

hipError_t launch_fill(uint32_t* counts, size_t count, int* status, bool clear_status, hipStream_t st);

// Several sample sets in one launch (passed by value): set q has n[q] samples
// at xy[q]; its raster or field is the q-th of a stack of N x N ones.
constexpr int kMaxSets = 64;
struct SetTable {
    int count;
    float2* xy[kMaxSets];
    int64_t n[kMaxSets];
};
hipError_t launch_splat_many(const SetTable& t, int N, uint32_t* counts, int* status, hipStream_t st);
hipError_t launch_blur_many(const uint32_t* counts, float* out, int N, int k, const BlurTaps& taps, const int* status,
                            hipStream_t st);
// Flags invalid samples of any set, then (if none) moves every set through its field.
hipError_t launch_advect_many(const SetTable& t, const float2* field, int N, int* status, hipStream_t st);
hipError_t launch_splat(const float2* xy, int64_t n, int N, uint32_t* counts, int* status, hipStream_t st);
hipError_t launch_blur(const uint32_t* counts, float* out, int N, const BlurTaps& taps, const int* status,
                       hipStream_t st);
hipError_t launch_validate(const float2* xy, int64_t n, int* status, hipStream_t st);

// Counting sort of the samples by texel (row-major) into sxy: clears the
// status word (then set for invalid samples) and writes the texel counts of
// the input to `counts` and the defect field t(p; 1) to t1 (N x N).  When
// row_sort_fits(N) (a row-bucketed pass, then one sort per row in LDS), map[q]
// is the index of the sample in slot q, and `stage` (n samples) and `idx`
// (n words) are scratch; otherwise (ranks by global atomics) map[p] is the
// slot of sample p.  `offsets` (N * N words), `partial` (scan_partials(N * N)
// words) and `rows` (2 N words) are scratch.
hipError_t launch_sort_by_texel(const float2* xy, int64_t n, int N, uint32_t* counts, uint32_t* map,
                                uint32_t* offsets, uint32_t* partial, uint32_t* rows, float2* sxy, float2* stage,
                                uint32_t* idx, float2* t1, int* status, hipStream_t st);
// The samples of sxy back to the caller's order through the map that
// launch_sort_by_texel wrote for this N.
hipError_t launch_unpermute(const float2* sxy, const uint32_t* map, int64_t n, int N, float2* xy, const int* status,
                            hipStream_t st);
// counts_next != nullptr: also splat the moved samples into it (must be zero).
hipError_t launch_advect(const float2* field, int N, float2* xy, int64_t n, uint32_t* counts_next, const int* status,
                         hipStream_t st);
// Blur of `counts` into `density` fused with the integral-image aggregate pass
// of the double-accumulated deformation path (tiles of 64 x 16); zeroes
// `zero_next` (N x N) when it is not null.  Only when blur_aggregate_fits(g).
bool blur_aggregate_fits(const Geom& g);
hipError_t launch_blur_aggregate(const uint32_t* counts, float* density, uint32_t* zero_next, int N,
                                 const BlurTaps& taps, const Geom& g, void* scratch, const int* status, hipStream_t st);

// Batched regularisation of several plots (batch_plan.h): the table-building
// launch, then one launch per stage with `blocks` = first[stage][count].
hipError_t launch_batch_init(const BatchArgs& a, BatchTable* T, hipStream_t st);
hipError_t launch_batch_raster(int stage, const BatchTable* T, unsigned blocks, int it, int iters, int* status,
                               hipStream_t st);
hipError_t launch_batch_inim(int stage, const BatchTable* T, unsigned blocks, int wpb, const BlurTaps& taps, int it,
                             int iters, const int* status, hipStream_t st);

}  // namespace inim
