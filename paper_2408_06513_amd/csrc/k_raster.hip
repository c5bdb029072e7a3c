// k_raster.hip -- per-sample and per-texel kernels of the regularisation on
// gfx950: the single-pixel splat and the separable Gaussian of Sec. 4.1,
// bilinear advection of Sec. 4.2, input validation and fills.
#include <hip/hip_runtime.h>

#include "blur_tile.h"
#include "device_common.h"
#include "batch_plan.h"
#include "launch.h"
#include "reg_layout.h"

namespace inim {

// Sets the status word when a sample is NaN or outside [0,1]^2.
__device__ __forceinline__ bool in_unit_square(float2 p) {
    return p.x >= 0.0f && p.x <= 1.0f && p.y >= 0.0f && p.y <= 1.0f;  // false for NaN
}

__device__ __forceinline__ void flag_domain(int* status) {
    __hip_atomic_store(status, (int)INIM_EDOMAIN, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------------ fill
// Kernel bodies take their block index and block count explicitly: the
// single-raster kernels pass blockIdx.x and gridDim.x, the batched kernels
// of a scatterplot matrix pass the block's place among the plot's blocks.
__device__ __forceinline__ void fill_body(uint32_t* __restrict__ counts, size_t count, int* status, int clear,
                                          int64_t bid, int64_t nblk) {
    const size_t t = (size_t)bid * blockDim.x + threadIdx.x;
    if (clear && t == 0) *status = 0;
    typedef uint32_t u4 __attribute__((ext_vector_type(4)));
    const size_t n4 = count / 4;
    const size_t stride = (size_t)nblk * blockDim.x;
    const u4 z = {0u, 0u, 0u, 0u};
    for (size_t k = t; k < n4; k += stride) reinterpret_cast<u4*>(counts)[k] = z;
    for (size_t k = n4 * 4 + t; k < count; k += stride) counts[k] = 0u;
}

__global__ __launch_bounds__(256) void k_fill(uint32_t* __restrict__ counts, size_t count, int* status, int clear) {
    fill_body(counts, count, status, clear, blockIdx.x, gridDim.x);
}

// ------------------------------------------------------------------ splat
// Texel of a coordinate: floor(x * N) (exact: N is a power of two), with the
// right/bottom edge x = 1 mapped to N - 1.
__device__ __forceinline__ int texel_of(float x, int N) {
    int k = (int)floorf(x * (float)N);
    return k > N - 1 ? N - 1 : k;
}

__global__ __launch_bounds__(256) void k_splat(const float2* __restrict__ xy, int64_t n, int N,
                                               uint32_t* __restrict__ counts, int* status) {
    if (failed(status)) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        const float2 q = xy[p];
        if (!in_unit_square(q)) {
            flag_domain(status);
            continue;
        }
        const int i = texel_of(q.x, N), j = texel_of(q.y, N);
        __hip_atomic_fetch_add(counts + (size_t)j * N + i, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Rasters of at most kLdsSplatTexels texels: each block counts its samples
// in an LDS copy of the raster, then adds its non-zero counts to the raster
// (where many samples share few texels, per-sample atomics on the same words
// serialise).  At most kLdsSplatBlocks blocks per sample set.
constexpr int kLdsSplatTexels = 16384;
constexpr unsigned kLdsSplatBlocks = 64;

__device__ __forceinline__ void splat_lds_body(const float2* __restrict__ xy, int64_t n, int N,
                                               uint32_t* __restrict__ counts, int* status, int64_t bid, int64_t nblk,
                                               uint32_t* bins) {
    const int NN = N * N;
    for (int k = threadIdx.x; k < NN; k += blockDim.x) bins[k] = 0u;
    __syncthreads();
    const int64_t stride = nblk * blockDim.x;
    for (int64_t p = bid * blockDim.x + threadIdx.x; p < n; p += stride) {
        const float2 q = xy[p];
        if (!in_unit_square(q)) {
            flag_domain(status);
            continue;
        }
        atomicAdd(&bins[texel_of(q.y, N) * N + texel_of(q.x, N)], 1u);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < NN; k += blockDim.x) {
        const uint32_t c = bins[k];
        if (c != 0u) __hip_atomic_fetch_add(counts + k, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ __launch_bounds__(256) void k_splat_lds(const float2* __restrict__ xy, int64_t n, int N,
                                                   uint32_t* __restrict__ counts, int* status) {
    extern __shared__ uint32_t bins[];
    if (failed(status)) return;
    splat_lds_body(xy, n, N, counts, status, blockIdx.x, gridDim.x, bins);
}

__global__ __launch_bounds__(256) void k_validate(const float2* __restrict__ xy, int64_t n, int* status) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride)
        if (!in_unit_square(xy[p])) flag_domain(status);
}

// ------------------------------------------------------------------ blur
// One 64 x 16 output tile per 256-thread block (blur_tile.h); blockIdx.z
// selects the raster of a stack of N x N rasters.
__global__ __launch_bounds__(256) void k_blur(const uint32_t* __restrict__ counts, float* __restrict__ out, int N,
                                              BlurTaps taps, const int* status) {
    extern __shared__ __align__(16) float lds[];  // read as float4 by the blur
    if (failed(status)) return;
    counts += (size_t)blockIdx.z * N * N;
    out += (size_t)blockIdx.z * N * N;
    const int ox = blockIdx.x * kBX, oy = blockIdx.y * kBY;
    blur_tile(counts, N, taps, ox, oy, lds,
              [&](int row, int cc, float v) { out[(size_t)(oy + row) * N + ox + cc] = v; });
}

// ------------------------------------------------------------------ advect
// Bilinear interpolation of the texel-centred field at each sample: cell index
// clamped to [0, N-2], fraction unclamped (linear extrapolation in the border
// half-texels), result clamped to [0,1]; arithmetic in double.
__device__ __forceinline__ void cell_of(float x, int N, int& k0, double& f) {
    const double s = (double)x * (double)N - 0.5;
    int k = (int)floor(s);
    k = k < 0 ? 0 : (k > N - 2 ? N - 2 : k);
    k0 = k;
    f = s - (double)k;
}

__device__ __forceinline__ float clamp01(double v) { return (float)(v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v)); }

__device__ __forceinline__ float2 advect_point(const float2* __restrict__ field, int N, float2 q) {
    int i0, j0;
    double fx, fy;
    cell_of(q.x, N, i0, fx);
    cell_of(q.y, N, j0, fy);
    const float2* r0 = field + (size_t)j0 * N + i0;
    const float2* r1 = r0 + N;
    const float2 a = r0[0], b = r0[1], c = r1[0], d = r1[1];
    const double w00 = (1.0 - fx) * (1.0 - fy), w10 = fx * (1.0 - fy), w01 = (1.0 - fx) * fy, w11 = fx * fy;
    const double nx = w00 * a.x + w10 * b.x + w01 * c.x + w11 * d.x;
    const double ny = w00 * a.y + w10 * b.y + w01 * c.y + w11 * d.y;
    return make_float2(clamp01(nx), clamp01(ny));
}

// Adds 1 at `key` for every lane holding a key below 0xFFFFFFFF: the 64 keys of
// the wave are sorted (bitonic network over lane shuffles) and only the first
// lane of every run of equal keys issues one atomic with the run length.  With
// samples in texel order most lanes of a wave share a few texels.
// The key of lane (lane ^ J): DPP quad permutes for J = 1, 2, the swizzle
// xor mode (within 32 lanes) for J = 4, 8, 16, a permute for J = 32.
template <int J>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v) {
    if constexpr (J == 1) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);  // [1,0,3,2]
    else if constexpr (J == 2) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);  // [2,3,0,1]
    else if constexpr (J <= 16) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1F | (J << 10));
    else return (uint32_t)__shfl_xor((int)v, J, 64);
}

template <int K, int J>
__device__ __forceinline__ uint32_t bitonic_step(uint32_t key, int lane) {
    const uint32_t o = lane_xor<J>(key);
    const bool keep_min = ((lane & K) == 0) == ((lane & J) == 0);
    return keep_min ? min(key, o) : max(key, o);
}

template <int K>
__device__ __forceinline__ uint32_t bitonic_merge(uint32_t key, int lane) {
    if constexpr (K >= 64) key = bitonic_step<K, 32>(key, lane);
    if constexpr (K >= 32) key = bitonic_step<K, 16>(key, lane);
    if constexpr (K >= 16) key = bitonic_step<K, 8>(key, lane);
    if constexpr (K >= 8) key = bitonic_step<K, 4>(key, lane);
    if constexpr (K >= 4) key = bitonic_step<K, 2>(key, lane);
    return bitonic_step<K, 1>(key, lane);
}

__device__ __forceinline__ void wave_count(uint32_t* __restrict__ counts, uint32_t key) {
    const int lane = lane_id();
    key = bitonic_merge<2>(key, lane);
    key = bitonic_merge<4>(key, lane);
    key = bitonic_merge<8>(key, lane);
    key = bitonic_merge<16>(key, lane);
    key = bitonic_merge<32>(key, lane);
    key = bitonic_merge<64>(key, lane);
    const uint32_t prev = (uint32_t)__shfl_up((int)key, 1, 64);
    const bool head = lane == 0 || prev != key;
    const unsigned long long heads = __ballot(head);
    if (head && key != 0xFFFFFFFFu) {
        const unsigned long long rest = lane == 63 ? 0ull : heads >> (lane + 1);
        const int next = rest ? lane + __ffsll((long long)rest) : 64;
        __hip_atomic_fetch_add(counts + key, (uint32_t)(next - lane), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// counts_next (optional): each moved sample is also splatted into it, the
// count raster of the next iteration (Sec. 4.3, step 1 of the next round).
// Every wave runs the same number of loop trips so that wave_count sees all
// 64 lanes.
__device__ __forceinline__ void advect_body(const float2* __restrict__ field, int N, float2* __restrict__ xy, int64_t n,
                                            uint32_t* __restrict__ counts_next, int64_t bid, int64_t nblk) {
    const int64_t stride = (int64_t)nblk * blockDim.x;
    const int64_t first = (int64_t)bid * blockDim.x + (threadIdx.x & ~63u);
    for (int64_t base = first; base < n; base += stride) {
        const int64_t p = base + lane_id();
        uint32_t key = 0xFFFFFFFFu;
        if (p < n) {
            const float2 o = advect_point(field, N, xy[p]);
            xy[p] = o;
            key = (uint32_t)(texel_of(o.y, N) * N + texel_of(o.x, N));
        }
        if (counts_next != nullptr) wave_count(counts_next, key);
    }
}

__global__ __launch_bounds__(256) void k_advect(const float2* __restrict__ field, int N, float2* __restrict__ xy,
                                                int64_t n, uint32_t* __restrict__ counts_next, const int* status) {
    if (failed(status)) return;
    advect_body(field, N, xy, n, counts_next, blockIdx.x, gridDim.x);
}

// ------------------------------------------------------------------ texel order
// Splat that also returns each sample's rank among the samples of its texel
// (the value of the count before its own increment); flags invalid samples.
__device__ __forceinline__ void splat_rank_body(const float2* __restrict__ xy, int64_t n, int N,
                                                uint32_t* __restrict__ counts, uint32_t* __restrict__ rank, int* status,
                                                int64_t bid, int64_t nblk) {
    const int64_t stride = (int64_t)nblk * blockDim.x;
    for (int64_t p = (int64_t)bid * blockDim.x + threadIdx.x; p < n; p += stride) {
        const float2 q = xy[p];
        if (!in_unit_square(q)) {
            flag_domain(status);
            continue;
        }
        const int i = texel_of(q.x, N), j = texel_of(q.y, N);
        rank[p] = __hip_atomic_fetch_add(counts + (size_t)j * N + i, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ __launch_bounds__(256) void k_splat_rank(const float2* __restrict__ xy, int64_t n, int N,
                                                    uint32_t* __restrict__ counts, uint32_t* __restrict__ rank,
                                                    int* status) {
    if (failed(status)) return;
    splat_rank_body(xy, n, N, counts, rank, status, blockIdx.x, gridDim.x);
}

// Exclusive prefix of a uint32 array (length a multiple of 4) in three passes:
// per-block sums, a scan of the block sums by one block, and the scan within
// each block.  A block of 256 threads covers 1024 consecutive words, four per
// thread as one 16-byte vector.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* lds_wave, uint32_t& total) {
    const int lane = lane_id(), wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const uint32_t incl = wave_inclusive_scan(v);
    if (lane == 63) lds_wave[wave] = incl;
    __syncthreads();
    if (wave == 0) {
        const uint32_t t = lane < nw ? lds_wave[lane] : 0u;
        const uint32_t ti = wave_inclusive_scan(t);
        if (lane < nw) lds_wave[lane] = ti - t;
        if (lane == nw - 1) lds_wave[32] = ti;
    }
    __syncthreads();
    total = lds_wave[32];
    return lds_wave[wave] + incl - v;
}

__device__ __forceinline__ void scan_reduce_body(const uint32_t* __restrict__ a, uint32_t* __restrict__ partial,
                                                 uint32_t* lw, int64_t bid) {
    const u32x4 v = reinterpret_cast<const u32x4*>(a)[(size_t)bid * kScanThreads + threadIdx.x];
    uint32_t total;
    (void)block_exclusive_scan(v.x + v.y + v.z + v.w, lw, total);
    if (threadIdx.x == 0) partial[bid] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t* __restrict__ a,
                                                              uint32_t* __restrict__ partial, const int* status) {
    __shared__ uint32_t lw[33];
    if (failed(status)) return;
    scan_reduce_body(a, partial, lw, blockIdx.x);
}

__device__ __forceinline__ void scan_partials_body(uint32_t* __restrict__ partial, int nb, uint32_t* lw) {
    const int per = (nb + (int)blockDim.x - 1) / (int)blockDim.x;
    const int b0 = threadIdx.x * per;
    uint32_t s = 0;
    for (int k = 0; k < per; ++k)
        if (b0 + k < nb) s += partial[b0 + k];
    uint32_t total;
    uint32_t run = block_exclusive_scan(s, lw, total);
    for (int k = 0; k < per; ++k)
        if (b0 + k < nb) {
            const uint32_t v = partial[b0 + k];
            partial[b0 + k] = run;
            run += v;
        }
}

__global__ __launch_bounds__(1024) void k_scan_partials(uint32_t* __restrict__ partial, int nb, const int* status) {
    __shared__ uint32_t lw[33];
    if (failed(status)) return;
    scan_partials_body(partial, nb, lw);
}

__device__ __forceinline__ void scan_down_body(const uint32_t* __restrict__ a, const uint32_t* __restrict__ partial,
                                               uint32_t* __restrict__ out, uint32_t* lw, int64_t bid) {
    const size_t k = (size_t)bid * kScanThreads + threadIdx.x;
    const u32x4 v = reinterpret_cast<const u32x4*>(a)[k];
    uint32_t total;
    const uint32_t run = partial[bid] + block_exclusive_scan(v.x + v.y + v.z + v.w, lw, total);
    u32x4 o;
    o.x = run;
    o.y = run + v.x;
    o.z = o.y + v.y;
    o.w = o.z + v.z;
    reinterpret_cast<u32x4*>(out)[k] = o;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(const uint32_t* __restrict__ a,
                                                            const uint32_t* __restrict__ partial,
                                                            uint32_t* __restrict__ out, const int* status) {
    __shared__ uint32_t lw[33];
    if (failed(status)) return;
    scan_down_body(a, partial, out, lw, blockIdx.x);
}

// Exclusive prefix of at most 1024 words by one block.
__global__ __launch_bounds__(1024) void k_scan_small(const uint32_t* __restrict__ a, int m,
                                                     uint32_t* __restrict__ out, const int* status) {
    __shared__ uint32_t lw[33];
    if (failed(status)) return;
    const int t = threadIdx.x;
    const uint32_t v = t < m ? a[t] : 0u;
    uint32_t total;
    const uint32_t ex = block_exclusive_scan(v, lw, total);
    if (t < m) out[t] = ex;
}

// Moves every sample to slot offset[texel] + rank: texel (row-major) order.
// The slot replaces the rank, so that the results can be gathered back.
__device__ __forceinline__ void scatter_sorted_body(const float2* __restrict__ xy, int64_t n, int N,
                                                    uint32_t* __restrict__ rank, const uint32_t* __restrict__ offset,
                                                    float2* __restrict__ sxy, int64_t bid, int64_t nblk) {
    const int64_t stride = (int64_t)nblk * blockDim.x;
    for (int64_t p = (int64_t)bid * blockDim.x + threadIdx.x; p < n; p += stride) {
        const float2 q = xy[p];
        const int i = texel_of(q.x, N), j = texel_of(q.y, N);
        const uint32_t slot = offset[(size_t)j * N + i] + rank[p];
        sxy[slot] = q;
        rank[p] = slot;
    }
}

__global__ __launch_bounds__(256) void k_scatter_sorted(const float2* __restrict__ xy, int64_t n, int N,
                                                        uint32_t* __restrict__ rank,
                                                        const uint32_t* __restrict__ offset, float2* __restrict__ sxy,
                                                        const int* status) {
    if (failed(status)) return;
    scatter_sorted_body(xy, n, N, rank, offset, sxy, blockIdx.x, gridDim.x);
}

// Back to the caller's order, from the slot of every sample (xy[p] =
// sxy[slot[p]]: xy read and written in order, sxy gathered) or from the
// sample of every slot (xy[perm[q]] = sxy[q]: xy scattered).
__device__ __forceinline__ void unpermute_body(const float2* __restrict__ sxy, const uint32_t* __restrict__ slot,
                                               int64_t n, float2* __restrict__ xy, int64_t bid, int64_t nblk) {
    const int64_t stride = (int64_t)nblk * blockDim.x;
    for (int64_t p = (int64_t)bid * blockDim.x + threadIdx.x; p < n; p += stride) xy[p] = sxy[slot[p]];
}

__global__ __launch_bounds__(256) void k_unpermute(const float2* __restrict__ sxy, const uint32_t* __restrict__ slot,
                                                   int64_t n, float2* __restrict__ xy, const int* status) {
    if (failed(status)) return;
    unpermute_body(sxy, slot, n, xy, blockIdx.x, gridDim.x);
}

__device__ __forceinline__ void unpermute_scatter_body(const float2* __restrict__ sxy,
                                                       const uint32_t* __restrict__ perm, int64_t n,
                                                       float2* __restrict__ xy, int64_t bid, int64_t nblk) {
    const int64_t stride = (int64_t)nblk * blockDim.x;
    for (int64_t q = (int64_t)bid * blockDim.x + threadIdx.x; q < n; q += stride) xy[perm[q]] = sxy[q];
}

__global__ __launch_bounds__(256) void k_unpermute_scatter(const float2* __restrict__ sxy,
                                                           const uint32_t* __restrict__ perm, int64_t n,
                                                           float2* __restrict__ xy, const int* status) {
    if (failed(status)) return;
    unpermute_scatter_body(sxy, perm, n, xy, blockIdx.x, gridDim.x);
}

// Texel order in two levels with no per-sample global atomics (those run at a
// few tens of billions per second whatever the address pattern, which at 1M
// samples costs more than every other step of the sort together).
//  1. Row buckets: kRowTiles blocks, each over one contiguous tile of samples,
//     count their samples per texel row in LDS (row_hist, flagging invalid
//     samples) and store them tile-major, hist[b * N + j]; row_scan turns
//     every row's counts over the tiles into prefixes (same layout) and row
//     totals; row_bucket scans the row totals into the first slot of every
//     row (rowstart) and moves every sample to rowstart[j] plus its tile's
//     prefix in row j plus its place in that run (an LDS counter), together
//     with its index.
//  2. One block per group of row_group(n, N) consecutive rows (row_sort)
//     counts the group's samples per texel in LDS, writes those rows of the
//     count raster, scans the counts and moves every sample to its slot in
//     texel order, recording its index by slot (writes that stay within the
//     group's range of slots).
// The order within a texel is arbitrary: nothing computed from it depends
// on it.  Rasters with row_sort_fits(N) (LDS counters per row and column).
// Each body takes its block's index among the blocks of its plot.
constexpr int kRowThreads = 1024;
// row_bucket moves the samples of its tile in chunks of CHUNK samples, each
// first ordered by row in LDS, so that consecutive lanes write consecutive
// slots: chunks of 4096 for tiles of more than 2048 samples (longer runs),
// else 2048 (56 KB of LDS: two blocks per CU).
constexpr int kRowChunkSmall = 2048, kRowChunkLarge = 4096;
// row_scan: a block of 256 threads takes kScanRows rows; their counts over
// all tiles go through LDS (loads and stores of kScanRows consecutive words
// per tile), kScanParts threads scan a row, kScanTiles tiles each.
constexpr int kScanParts = 256 / kScanRows, kScanTiles = kRowTiles / kScanParts;
// row_sort: groups of up to kSortThreads * kSortHeld samples are read once
// and held in registers between the count and the move; larger ones are read
// twice.
constexpr int kSortThreads = 512, kSortHeld = 8;

__device__ __forceinline__ int64_t row_tile(int64_t n) { return n > 0 ? (n + kRowTiles - 1) / kRowTiles : 1; }

__device__ __forceinline__ void row_hist_body(const float2* __restrict__ xy, int64_t n, int N,
                                              uint32_t* __restrict__ hist, int* status, int64_t b, uint32_t* bins) {
    for (int j = threadIdx.x; j < N; j += kRowThreads) bins[j] = 0u;
    __syncthreads();
    const int64_t tile = row_tile(n), p0 = b * tile, p1 = min(n, p0 + tile);
    // kHistPer samples per thread and round, all loaded before any is counted
    // (a thread past p1 reloads sample p0 and discards it)
    constexpr int kHistPer = 8;
    for (int64_t base = p0; base < p1; base += (int64_t)kRowThreads * kHistPer) {
        float2 q[kHistPer];
#pragma unroll
        for (int k = 0; k < kHistPer; ++k) {
            if (base + (int64_t)k * kRowThreads >= p1) break;  // uniform: no sample left for any thread
            const int64_t p = base + threadIdx.x + (int64_t)k * kRowThreads;
            q[k] = xy[p < p1 ? p : p0];
        }
#pragma unroll
        for (int k = 0; k < kHistPer; ++k) {
            const int64_t p = base + threadIdx.x + (int64_t)k * kRowThreads;
            if (p >= p1) continue;
            if (!in_unit_square(q[k])) {
                flag_domain(status);
                continue;
            }
            atomicAdd(&bins[texel_of(q[k].y, N)], 1u);
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < N; j += kRowThreads) hist[(size_t)b * N + j] = bins[j];
}

__global__ __launch_bounds__(kRowThreads) void k_row_hist(const float2* __restrict__ xy, int64_t n, int N,
                                                           uint32_t* __restrict__ hist, int* status) {
    __shared__ uint32_t bins[kRowSortMaxN];
    row_hist_body(xy, n, N, hist, status, blockIdx.x, bins);
}

// prefix[b * N + j] = sum of hist[b' * N + j] over b' < b; rowtot[j] = the sum
// over all tiles; rows [kScanRows blk, kScanRows blk + kScanRows).
struct RowScanLds {
    uint32_t h[kRowTiles][kScanRows + 1];
};

__device__ __forceinline__ void row_scan_body(const uint32_t* __restrict__ hist, int N, uint32_t* __restrict__ prefix,
                                              uint32_t* __restrict__ rowtot, int64_t blk, RowScanLds& L) {
    static_assert(kRowTiles == 256 && kScanParts <= 64, "a row's parts within one wave");
    const int j0 = (int)blk * kScanRows, t = threadIdx.x;
    const int r = t % kScanRows, b0 = t / kScanRows;  // loads: row r, tiles b0 + kScanParts k
    {
        uint32_t v[kScanTiles];  // every load in flight before the first store
#pragma unroll
        for (int k = 0; k < kScanTiles; ++k) v[k] = hist[(size_t)(b0 + kScanParts * k) * N + j0 + r];
#pragma unroll
        for (int k = 0; k < kScanTiles; ++k) L.h[b0 + kScanParts * k][r] = v[k];
    }
    __syncthreads();
    const int row = t / kScanParts, part = t % kScanParts;  // scan: tiles [kScanTiles part, +kScanTiles)
    uint32_t c[kScanTiles];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kScanTiles; ++k) {
        c[k] = L.h[part * kScanTiles + k][row];
        sum += c[k];
    }
    uint32_t incl = sum;  // inclusive scan over the row's parts (consecutive lanes)
#pragma unroll
    for (int d = 1; d < kScanParts; d <<= 1) {
        const uint32_t o = (uint32_t)__shfl_up((int)incl, d, kScanParts);
        if (part >= d) incl += o;
    }
    uint32_t run = incl - sum;
#pragma unroll
    for (int k = 0; k < kScanTiles; ++k) {
        L.h[part * kScanTiles + k][row] = run;
        run += c[k];
    }
    if (part == kScanParts - 1) rowtot[j0 + row] = run;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanTiles; ++k)
        prefix[(size_t)(b0 + kScanParts * k) * N + j0 + r] = L.h[b0 + kScanParts * k][r];
}

__global__ __launch_bounds__(256) void k_row_scan(const uint32_t* __restrict__ hist, int N,
                                                  uint32_t* __restrict__ prefix, uint32_t* __restrict__ rowtot,
                                                  const int* status) {
    __shared__ RowScanLds L;
    if (failed(status)) return;
    row_scan_body(hist, N, prefix, rowtot, blockIdx.x, L);
}

// Tile b's samples to their row runs; the block of tile 0 also stores
// rowstart for row_sort.  Every sample is in the unit square here (callers
// run it only when the status word is clear).
template <int CHUNK>
struct RowBucketLds {
    uint32_t cnt[kRowSortMaxN];   // per row: count in the chunk, its first LDS slot, then stage minus LDS slot
    uint32_t next[kRowSortMaxN];  // per row: the tile's next slot in `stage`
    float2 lxy[CHUNK];
    uint32_t lidx[CHUNK];
    uint32_t lw[33];
};

template <int CHUNK>
__device__ __forceinline__ void row_bucket_body(const float2* __restrict__ xy, int64_t n, int N,
                                                const uint32_t* __restrict__ prefix,
                                                const uint32_t* __restrict__ rowtot, uint32_t* __restrict__ rowstart,
                                                float2* __restrict__ stage, uint32_t* __restrict__ idx, int64_t b,
                                                RowBucketLds<CHUNK>& L) {
    constexpr int kPer = CHUNK / kRowThreads, kRowsPer = kRowSortMaxN / kRowThreads;
    const int per = (N + kRowThreads - 1) / kRowThreads, r0 = threadIdx.x * per;
    {
        // the row totals and this tile's prefixes are loaded together (one
        // round of memory latency) at valid indices, the unused ones discarded
        uint32_t v[kRowsPer], pf[kRowsPer];
        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k < kRowsPer; ++k) {
            const bool in = k < per && r0 + k < N;
            const int j = in ? r0 + k : 0;
            const uint32_t t_ = rowtot[j];
            pf[k] = prefix[(size_t)b * N + j];
            v[k] = in ? t_ : 0u;
            sum += v[k];
        }
        uint32_t total;
        uint32_t run = block_exclusive_scan(sum, L.lw, total);
#pragma unroll
        for (int k = 0; k < kRowsPer; ++k)
            if (k < per && r0 + k < N) {
                const int j = r0 + k;
                L.next[j] = run + pf[k];
                if (b == 0) rowstart[j] = run;
                run += v[k];
            }
    }
    const int64_t tile = row_tile(n), p0 = b * tile, p1 = min(n, p0 + tile);
    for (int64_t c0 = p0; c0 < p1; c0 += CHUNK) {
        const int m = (int)min((int64_t)CHUNK, p1 - c0);
        for (int j = threadIdx.x; j < N; j += kRowThreads) L.cnt[j] = 0u;
        __syncthreads();
        // the chunk's samples are all loaded before any is counted (one round
        // of memory latency; a thread past m reloads sample c0 and discards it)
        float2 q[kPer];
        uint32_t row[kPer], rk[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            if (k * kRowThreads >= m) break;  // uniform: no sample left for any thread
            const int s = threadIdx.x + k * kRowThreads;
            q[k] = xy[c0 + (s < m ? s : 0)];
        }
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int s = threadIdx.x + k * kRowThreads;
            if (s < m) {
                row[k] = (uint32_t)texel_of(q[k].y, N);
                rk[k] = atomicAdd(&L.cnt[row[k]], 1u);
            }
        }
        __syncthreads();
        // rows [r0, r0 + per) of this thread: first LDS slot, stage offset
        uint32_t v[kRowsPer];
        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k < kRowsPer; ++k) {
            v[k] = (k < per && r0 + k < N) ? L.cnt[r0 + k] : 0u;
            sum += v[k];
        }
        uint32_t total;
        uint32_t run = block_exclusive_scan(sum, L.lw, total);
#pragma unroll
        for (int k = 0; k < kRowsPer; ++k)
            if (k < per && r0 + k < N) {
                L.cnt[r0 + k] = run;
                run += v[k];
            }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int s = threadIdx.x + k * kRowThreads;
            if (s < m) {
                const uint32_t at = L.cnt[row[k]] + rk[k];
                L.lxy[at] = q[k];
                L.lidx[at] = (uint32_t)(c0 + s);
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kRowsPer; ++k)
            if (k < per && r0 + k < N) {
                const int j = r0 + k;
                L.cnt[j] = L.next[j] - L.cnt[j];
                L.next[j] += v[k];
            }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int s = threadIdx.x + k * kRowThreads;
            if (s < m) {
                const float2 w = L.lxy[s];
                const uint32_t at = L.cnt[texel_of(w.y, N)] + (uint32_t)s;
                stage[at] = w;
                idx[at] = L.lidx[s];
            }
        }
        __syncthreads();
    }
}

template <int CHUNK>
__global__ __launch_bounds__(kRowThreads) void k_row_bucket(const float2* __restrict__ xy, int64_t n, int N,
                                                             const uint32_t* __restrict__ prefix,
                                                             const uint32_t* __restrict__ rowtot,
                                                             uint32_t* __restrict__ rowstart,
                                                             float2* __restrict__ stage, uint32_t* __restrict__ idx,
                                                             const int* status) {
    __shared__ RowBucketLds<CHUNK> L;
    if (failed(status)) return;
    row_bucket_body<CHUNK>(xy, n, N, prefix, rowtot, rowstart, stage, idx, blockIdx.x, L);
}

// Rows [g blk, g blk + g) to texel order, g = row_group(n, N); also those
// rows of the defect field when t1 is not null.
struct RowSortLds {
    uint32_t bins[kRowSortMaxN];
    uint32_t lw[33];
};

__device__ __forceinline__ void row_sort_body(const float2* __restrict__ stage, const uint32_t* __restrict__ idx,
                                              const uint32_t* __restrict__ rowstart, int64_t n, int N,
                                              uint32_t* __restrict__ counts, float2* __restrict__ sxy,
                                              uint32_t* __restrict__ perm, float2* __restrict__ t1, int blk,
                                              RowSortLds& L) {
    constexpr int kColsPer = kRowSortMaxN / kSortThreads;
    const int t = threadIdx.x;
    const int g = row_group(n, N), j0 = blk * g, K = g * N;  // K texels, row-major from (0, j0)
    const int64_t q0 = rowstart[j0];
    const int64_t q1 = j0 + g < N ? (int64_t)rowstart[j0 + g] : n;
    const bool held = q1 - q0 <= (int64_t)kSortThreads * kSortHeld;
    // the texel of a sample of these rows, relative to (0, j0)
    auto key = [&](float2 p) { return (uint32_t)((texel_of(p.y, N) - j0) * N + texel_of(p.x, N)); };
    for (int i = t; i < K; i += kSortThreads) L.bins[i] = 0u;
    __syncthreads();
    float2 v[kSortHeld];
    uint32_t col[kSortHeld], from[kSortHeld];
    if (held) {
        // every held sample's loads first (one round of memory latency; a
        // lane past q1 reloads sample q0 and discards it), then the counts
#pragma unroll
        for (int k = 0; k < kSortHeld; ++k) {
            if (q0 + k * kSortThreads >= q1) break;  // uniform: no sample left for any lane
            const int64_t q = q0 + t + k * kSortThreads, qq = q < q1 ? q : q0;
            v[k] = stage[qq];
            from[k] = idx[qq];
        }
#pragma unroll
        for (int k = 0; k < kSortHeld; ++k) {
            const int64_t q = q0 + t + k * kSortThreads;
            if (q < q1) {
                col[k] = key(v[k]);
                atomicAdd(&L.bins[col[k]], 1u);
            }
        }
    } else {
        for (int64_t q = q0 + t; q < q1; q += kSortThreads) atomicAdd(&L.bins[key(stage[q])], 1u);
    }
    __syncthreads();
    // these rows of the count raster, then the exclusive scan of the counts
    // (thread t holds entries [t * per, t * per + per))
    const int per = (K + kSortThreads - 1) / kSortThreads;
    const int i0 = t * per;
    uint32_t c[kColsPer];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kColsPer; ++k) {
        c[k] = (k < per && i0 + k < K) ? L.bins[i0 + k] : 0u;
        sum += c[k];
    }
    for (int i = t; i < K; i += kSortThreads) counts[(size_t)j0 * N + i] = L.bins[i];
    uint32_t total;
    uint32_t run = (uint32_t)q0 + block_exclusive_scan(sum, L.lw, total);
#pragma unroll
    for (int k = 0; k < kColsPer; ++k)
        if (k < per && i0 + k < K) {
            L.bins[i0 + k] = run;
            run += c[k];
        }
    __syncthreads();
    if (held) {
#pragma unroll
        for (int k = 0; k < kSortHeld; ++k) {
            const int64_t q = q0 + t + k * kSortThreads;
            if (q < q1) {
                const uint32_t slot = atomicAdd(&L.bins[col[k]], 1u);
                sxy[slot] = v[k];
                perm[slot] = from[k];
            }
        }
    } else {
        for (int64_t q = q0 + t; q < q1; q += kSortThreads) {
            const float2 p = stage[q];
            const uint32_t slot = atomicAdd(&L.bins[key(p)], 1u);
            sxy[slot] = p;
            perm[slot] = idx[q];
        }
    }
    if (t1 != nullptr)
        for (int i = t; i < K; i += kSortThreads) t1[(size_t)j0 * N + i] = defect_texel(i % N, j0 + i / N, N);
}

__global__ __launch_bounds__(kSortThreads) void k_row_sort(const float2* __restrict__ stage,
                                                            const uint32_t* __restrict__ idx,
                                                            const uint32_t* __restrict__ rowstart, int64_t n, int N,
                                                            uint32_t* __restrict__ counts, float2* __restrict__ sxy,
                                                            uint32_t* __restrict__ perm, float2* __restrict__ t1,
                                                            const int* status) {
    __shared__ RowSortLds L;
    if (failed(status)) return;
    row_sort_body(stage, idx, rowstart, n, N, counts, sxy, perm, t1, blockIdx.x, L);
}

// ------------------------------------------------------------------ several sample sets
// One launch for the sets of a SetTable: blockIdx.y is the set, blockIdx.x
// strides over its samples; raster q is the q-th of a stack of N x N rasters.
__global__ __launch_bounds__(256) void k_splat_many(SetTable t, int N, uint32_t* __restrict__ counts, int* status) {
    const int q = blockIdx.y;
    const float2* __restrict__ xy = t.xy[q];
    uint32_t* c = counts + (size_t)q * N * N;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < t.n[q]; p += stride) {
        const float2 v = xy[p];
        if (!in_unit_square(v)) {
            flag_domain(status);
            continue;
        }
        __hip_atomic_fetch_add(c + (size_t)texel_of(v.y, N) * N + texel_of(v.x, N), 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ __launch_bounds__(256) void k_splat_many_lds(SetTable t, int N, uint32_t* __restrict__ counts, int* status) {
    extern __shared__ uint32_t bins[];
    const int q = blockIdx.y;
    splat_lds_body(t.xy[q], t.n[q], N, counts + (size_t)q * N * N, status, blockIdx.x, gridDim.x, bins);
}

__global__ __launch_bounds__(256) void k_validate_many(SetTable t, int* status) {
    const int q = blockIdx.y;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < t.n[q]; p += stride)
        if (!in_unit_square(t.xy[q][p])) flag_domain(status);
}

__global__ __launch_bounds__(256) void k_advect_many(SetTable t, const float2* __restrict__ field, int N,
                                                     const int* status) {
    if (failed(status)) return;
    const int q = blockIdx.y;
    float2* __restrict__ xy = t.xy[q];
    const float2* f = field + (size_t)q * N * N;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < t.n[q]; p += stride)
        xy[p] = advect_point(f, N, xy[p]);
}

// ------------------------------------------------------------------ launchers
static unsigned grid_for(int64_t n, int per_block = 256, unsigned cap = 8192) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    return (unsigned)(g > cap ? cap : g);
}

StageClock*& stage_clock() {
    thread_local StageClock* c = nullptr;
    return c;
}

hipError_t launch_fill(uint32_t* counts, size_t count, int* status, bool clear_status, hipStream_t st) {
    launch_kernel(k_fill, dim3(grid_for((int64_t)(count / 4 + 1), 256, 2048)), dim3(256), 0, st, counts, count,
                       status, clear_status ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_splat(const float2* xy, int64_t n, int N, uint32_t* counts, int* status, hipStream_t st) {
    if ((int64_t)N * N <= kLdsSplatTexels)
        hipLaunchKernelGGL(k_splat_lds, dim3(grid_for(n, 256, kLdsSplatBlocks)), dim3(256), sizeof(uint32_t) * N * N,
                           st, xy, n, N, counts, status);
    else
        hipLaunchKernelGGL(k_splat, dim3(grid_for(n)), dim3(256), 0, st, xy, n, N, counts, status);
    return hipGetLastError();
}

hipError_t launch_validate(const float2* xy, int64_t n, int* status, hipStream_t st) {
    hipLaunchKernelGGL(k_validate, dim3(grid_for(n)), dim3(256), 0, st, xy, n, status);
    return hipGetLastError();
}

hipError_t launch_blur(const uint32_t* counts, float* out, int N, const BlurTaps& taps, const int* status,
                       hipStream_t st) {
    const size_t smem = sizeof(float) * blur_smem_floats(taps.r);
    const dim3 grd((N + kBX - 1) / kBX, (N + kBY - 1) / kBY);
    launch_kernel(k_blur, grd, dim3(256), smem, st, counts, out, N, taps, status);
    return hipGetLastError();
}

static unsigned grid_for_sets(const SetTable& t) {
    int64_t m = 0;
    for (int q = 0; q < t.count; ++q) m = t.n[q] > m ? t.n[q] : m;
    return grid_for(m);
}

hipError_t launch_blur_many(const uint32_t* counts, float* out, int N, int k, const BlurTaps& taps, const int* status,
                            hipStream_t st) {
    const size_t smem = sizeof(float) * blur_smem_floats(taps.r);
    const dim3 grd((N + kBX - 1) / kBX, (N + kBY - 1) / kBY, k);
    launch_kernel(k_blur, grd, dim3(256), smem, st, counts, out, N, taps, status);
    return hipGetLastError();
}

hipError_t launch_splat_many(const SetTable& t, int N, uint32_t* counts, int* status, hipStream_t st) {
    if ((int64_t)N * N <= kLdsSplatTexels) {
        const unsigned g = grid_for_sets(t);
        hipLaunchKernelGGL(k_splat_many_lds, dim3(g < kLdsSplatBlocks ? g : kLdsSplatBlocks, t.count), dim3(256),
                           sizeof(uint32_t) * N * N, st, t, N, counts, status);
    } else {
        hipLaunchKernelGGL(k_splat_many, dim3(grid_for_sets(t), t.count), dim3(256), 0, st, t, N, counts, status);
    }
    return hipGetLastError();
}

hipError_t launch_advect_many(const SetTable& t, const float2* field, int N, int* status, hipStream_t st) {
    hipLaunchKernelGGL(k_validate_many, dim3(grid_for_sets(t), t.count), dim3(256), 0, st, t, status);
    hipLaunchKernelGGL(k_advect_many, dim3(grid_for_sets(t), t.count), dim3(256), 0, st, t, field, N, status);
    return hipGetLastError();
}

hipError_t launch_advect(const float2* field, int N, float2* xy, int64_t n, uint32_t* counts_next, const int* status,
                         hipStream_t st) {
    launch_kernel(k_advect, dim3(grid_for(n)), dim3(256), 0, st, field, N, xy, n, counts_next, status);
    return hipGetLastError();
}

}  // namespace inim

namespace inim {

static void launch_scan(const uint32_t* a, size_t m, uint32_t* partial, uint32_t* out, const int* status,
                        hipStream_t st) {
    if (m % kScanBlock == 0) {
        const int nb = (int)scan_partials(m);
        hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanThreads), 0, st, a, partial, status);
        hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, st, partial, nb, status);
        hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(kScanThreads), 0, st, a, partial, out, status);
    } else {  // fewer than 1024 words: one block
        hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, a, (int)m, out, status);
    }
}

hipError_t launch_sort_by_texel(const float2* xy, int64_t n, int N, uint32_t* counts, uint32_t* map,
                                uint32_t* offsets, uint32_t* partial, uint32_t* rows, float2* sxy, float2* stage,
                                uint32_t* idx, float2* t1, int* status, hipStream_t st) {
    if (row_sort_fits(N)) {
        // N * kRowTiles <= N * N words of tile counts and offsets
        // tile counts in `counts` (whose rows k_row_sort rewrites), their
        // prefixes in `offsets`, row totals and row starts in `rows`
        uint32_t *rowtot = rows, *rowstart = rows + N;
        hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, st, counts, (size_t)0, status, 1);
        hipLaunchKernelGGL(k_row_hist, dim3(kRowTiles), dim3(kRowThreads), 0, st, xy, n, N, counts, status);
        hipLaunchKernelGGL(k_row_scan, dim3(N / kScanRows), dim3(256), 0, st, counts, N, offsets, rowtot, status);
        const int64_t tile = n > 0 ? (n + kRowTiles - 1) / kRowTiles : 1;  // as row_tile(n)
        if (tile > kRowChunkSmall)
            hipLaunchKernelGGL(k_row_bucket<kRowChunkLarge>, dim3(kRowTiles), dim3(kRowThreads), 0, st, xy, n, N,
                               offsets, rowtot, rowstart, stage, idx, status);
        else
            hipLaunchKernelGGL(k_row_bucket<kRowChunkSmall>, dim3(kRowTiles), dim3(kRowThreads), 0, st, xy, n, N,
                               offsets, rowtot, rowstart, stage, idx, status);
        hipLaunchKernelGGL(k_row_sort, dim3(N / row_group(n, N)), dim3(kSortThreads), 0, st, stage, idx, rowstart,
                           n, N, counts, sxy, map, t1, status);
        return hipGetLastError();
    }
    const size_t m = (size_t)N * N;  // a multiple of 4 (N >= 2, a power of two)
    hipLaunchKernelGGL(k_fill, dim3(grid_for((int64_t)(m / 4 + 1), 256, 2048)), dim3(256), 0, st, counts, m, status, 1);
    hipLaunchKernelGGL(k_splat_rank, dim3(grid_for(n)), dim3(256), 0, st, xy, n, N, counts, map, status);
    launch_scan(counts, m, partial, offsets, status, st);
    hipLaunchKernelGGL(k_scatter_sorted, dim3(grid_for(n)), dim3(256), 0, st, xy, n, N, map, offsets, sxy, status);
    const hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : launch_defect_field(N, t1, st);
}

// ------------------------------------------------------------------ batched (scatterplot matrix)
// One launch per stage for all plots of a BatchTable; each block runs the
// single-plot body for its plot with its block index among that plot's.
// Block 0 of the launch clears the status word; plots sorted by rows get one
// block and nothing to fill.
__global__ __launch_bounds__(256) void kb_fill(const BatchTable* __restrict__ T, int* status) {
    int64_t bid, nblk;
    const BatchPlot& P = batch_locate(T, kBFill, blockIdx.x, bid, nblk);
    const size_t count = row_sort_fits(P.N) ? 0 : (size_t)P.N * P.N;
    fill_body(P.counts[0], count, status, blockIdx.x == 0 ? 1 : 0, bid, nblk);
}

__global__ __launch_bounds__(256) void kb_splat_rank(const BatchTable* __restrict__ T, int* status) {
    if (failed(status)) return;
    int64_t bid, nblk;
    const BatchPlot& P = batch_locate(T, kBSplatRank, blockIdx.x, bid, nblk);
    splat_rank_body(reinterpret_cast<const float2*>(P.xy), P.n, P.N, P.counts[0], P.rank, status, bid, nblk);
}

__global__ __launch_bounds__(kScanThreads) void kb_scan_reduce(const BatchTable* __restrict__ T, const int* status) {
    __shared__ uint32_t lw[33];
    if (failed(status)) return;
    int64_t bid, nblk;
    const BatchPlot& P = batch_locate(T, kBScanReduce, blockIdx.x, bid, nblk);
    scan_reduce_body(P.counts[0], P.partial, lw, bid);
}

__global__ __launch_bounds__(1024) void kb_scan_partials(const BatchTable* __restrict__ T, const int* status) {
    __shared__ uint32_t lw[33];
    if (failed(status)) return;
    int64_t bid, nblk;
    const BatchPlot& P = batch_locate(T, kBScanPartials, blockIdx.x, bid, nblk);
    scan_partials_body(P.partial, (int)scan_partials((size_t)P.N * P.N), lw);
}

__global__ __launch_bounds__(kScanThreads) void kb_scan_down(const BatchTable* __restrict__ T, const int* status) {
    __shared__ uint32_t lw[33];
    if (failed(status)) return;
    int64_t bid, nblk;
    const BatchPlot& P = batch_locate(T, kBScanDown, blockIdx.x, bid, nblk);
    scan_down_body(P.counts[0], P.partial, P.counts[1], lw, bid);
}

__global__ __launch_bounds__(256) void kb_scatter(const BatchTable* __restrict__ T, const int* status) {
    if (failed(status)) return;
    int64_t bid, nblk;
    const BatchPlot& P = batch_locate(T, kBScatter, blockIdx.x, bid, nblk);
    scatter_sorted_body(reinterpret_cast<const float2*>(P.xy), P.n, P.N, P.rank, P.counts[1], P.sxy, bid, nblk);
}

// The row sort of every plot with row_sort_fits(N): tile counts in counts[0],
// prefixes in counts[1], row totals and starts in the density raster (free
// until the first smoothing), as in the single-plot call.
__global__ __launch_bounds__(kRowThreads) void kb_row_hist(const BatchTable* __restrict__ T, int* status) {
    __shared__ uint32_t bins[kRowSortMaxN];
    int64_t bid, nblk;
    const BatchPlot& P = batch_locate(T, kBRowHist, blockIdx.x, bid, nblk);
    row_hist_body(reinterpret_cast<const float2*>(P.xy), P.n, P.N, P.counts[0], status, bid, bins);
}

__global__ __launch_bounds__(256) void kb_row_scan(const BatchTable* __restrict__ T, const int* status) {
    __shared__ RowScanLds L;
    if (failed(status)) return;
    int64_t bid, nblk;
    const BatchPlot& P = batch_locate(T, kBRowScan, blockIdx.x, bid, nblk);
    row_scan_body(P.counts[0], P.N, P.counts[1], reinterpret_cast<uint32_t*>(P.density), bid, L);
}

__global__ __launch_bounds__(kRowThreads) void kb_row_bucket(const BatchTable* __restrict__ T, const int* status) {
    __shared__ RowBucketLds<kRowChunkSmall> L;
    if (failed(status)) return;
    int64_t bid, nblk;
    const BatchPlot& P = batch_locate(T, kBRowBucket, blockIdx.x, bid, nblk);
    uint32_t* rows = reinterpret_cast<uint32_t*>(P.density);
    row_bucket_body<kRowChunkSmall>(reinterpret_cast<const float2*>(P.xy), P.n, P.N, P.counts[1], rows, rows + P.N,
                                    P.stage, P.idx, bid, L);
}

__global__ __launch_bounds__(kSortThreads) void kb_row_sort(const BatchTable* __restrict__ T, const int* status) {
    __shared__ RowSortLds L;
    if (failed(status)) return;
    int64_t bid, nblk;
    const BatchPlot& P = batch_locate(T, kBRowSort, blockIdx.x, bid, nblk);
    const uint32_t* rowstart = reinterpret_cast<const uint32_t*>(P.density) + P.N;
    row_sort_body(P.stage, P.idx, rowstart, P.n, P.N, P.counts[0], P.sxy, P.rank, P.defect_owner ? P.defect : nullptr,
                  (int)bid, L);
}

__global__ __launch_bounds__(256) void kb_advect(const BatchTable* __restrict__ T, int it, int iters,
                                                 const int* status) {
    if (failed(status)) return;
    int64_t bid, nblk;
    const BatchPlot& P = batch_locate(T, kBAdvect, blockIdx.x, bid, nblk);
    uint32_t* nxt = (it + 1 < iters) ? P.counts[(it + 1) & 1] : nullptr;
    advect_body(P.field, P.N, P.sxy, P.n, nxt, bid, nblk);
}

__global__ __launch_bounds__(256) void kb_unpermute(const BatchTable* __restrict__ T, const int* status) {
    if (failed(status)) return;
    int64_t bid, nblk;
    const BatchPlot& P = batch_locate(T, kBUnpermute, blockIdx.x, bid, nblk);
    if (row_sort_fits(P.N))  // rank holds the sample of every slot
        unpermute_scatter_body(P.sxy, P.rank, P.n, reinterpret_cast<float2*>(P.xy), bid, nblk);
    else  // rank holds the slot of every sample
        unpermute_body(P.sxy, P.rank, P.n, reinterpret_cast<float2*>(P.xy), bid, nblk);
}

hipError_t launch_batch_raster(int stage, const BatchTable* T, unsigned blocks, int it, int iters, int* status,
                               hipStream_t st) {
    if (blocks == 0) return hipSuccess;
    switch (stage) {
        case kBFill: hipLaunchKernelGGL(kb_fill, dim3(blocks), dim3(256), 0, st, T, status); break;
        case kBSplatRank: hipLaunchKernelGGL(kb_splat_rank, dim3(blocks), dim3(256), 0, st, T, status); break;
        case kBScanReduce:
            hipLaunchKernelGGL(kb_scan_reduce, dim3(blocks), dim3(kScanThreads), 0, st, T, status);
            break;
        case kBScanPartials: hipLaunchKernelGGL(kb_scan_partials, dim3(blocks), dim3(1024), 0, st, T, status); break;
        case kBScanDown: hipLaunchKernelGGL(kb_scan_down, dim3(blocks), dim3(kScanThreads), 0, st, T, status); break;
        case kBScatter: hipLaunchKernelGGL(kb_scatter, dim3(blocks), dim3(256), 0, st, T, status); break;
        case kBRowHist: hipLaunchKernelGGL(kb_row_hist, dim3(blocks), dim3(kRowThreads), 0, st, T, status); break;
        case kBRowScan: hipLaunchKernelGGL(kb_row_scan, dim3(blocks), dim3(256), 0, st, T, status); break;
        case kBRowBucket: hipLaunchKernelGGL(kb_row_bucket, dim3(blocks), dim3(kRowThreads), 0, st, T, status); break;
        case kBRowSort: hipLaunchKernelGGL(kb_row_sort, dim3(blocks), dim3(kSortThreads), 0, st, T, status); break;
        case kBAdvect: hipLaunchKernelGGL(kb_advect, dim3(blocks), dim3(256), 0, st, T, it, iters, status); break;
        case kBUnpermute: hipLaunchKernelGGL(kb_unpermute, dim3(blocks), dim3(256), 0, st, T, status); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_unpermute(const float2* sxy, const uint32_t* map, int64_t n, int N, float2* xy, const int* status,
                            hipStream_t st) {
    if (row_sort_fits(N))
        hipLaunchKernelGGL(k_unpermute_scatter, dim3(grid_for(n)), dim3(256), 0, st, sxy, map, n, xy, status);
    else
        hipLaunchKernelGGL(k_unpermute, dim3(grid_for(n)), dim3(256), 0, st, sxy, map, n, xy, status);
    return hipGetLastError();
}

}  // namespace inim
