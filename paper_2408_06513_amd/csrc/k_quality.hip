// k_quality.hip -- layout quality measures of a regularised scatterplot
// (Sec. 6, numerical tests) on gfx950: per-bin sample counts and occupied
// texels, orthogonal ordering, trustworthiness.  All results are exact
// integer sums gathered per block and added with 64-bit integer atomics, so
// they do not depend on the order of the additions.
//
// The pair measures are O(n^2) over a sample of the layout: the positions
// (8 bytes each) stay in L2 and every block sweeps them, so these kernels
// are bound by their ALU work, not by HBM.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>

#include "inim.h"
#include "inim_quality.h"

namespace {

constexpr int kThreads = 256, kWave = 64, kWaves = kThreads / kWave;
typedef unsigned long long u64;

__device__ __forceinline__ u64 wave_sum(u64 v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Adds the block's totals of up to three counters into out[0..C-1].
template <int C>
__device__ __forceinline__ void block_add(u64 (&v)[C], u64* out) {
    __shared__ u64 part[C][kWaves];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const u64 s = wave_sum(v[c]);
        if (lane == 0) part[c][wave] = s;
    }
    __syncthreads();
    if (threadIdx.x < C) {
        u64 s = 0;
        for (int w = 0; w < kWaves; ++w) s += part[threadIdx.x][w];
        if (s) atomicAdd(out + threadIdx.x, s);
    }
}

// ------------------------------------------------------------------ bins
// One thread per bin x bin block: rows of `bin` contiguous texels, so
// neighbouring threads read neighbouring segments of a raster row.
__global__ __launch_bounds__(kThreads) void k_bins(const uint32_t* __restrict__ counts, int N, int bin,
                                                   u64* __restrict__ stats) {
    const int nb = N / bin;
    const int64_t total = (int64_t)nb * nb;
    u64 v[3] = {0, 0, 0};  // occupied texels, samples, squared bin counts
    for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < total; q += (int64_t)gridDim.x * kThreads) {
        const int by = (int)(q / nb), bx = (int)(q - (int64_t)by * nb);
        const uint32_t* row = counts + (size_t)by * bin * N + (size_t)bx * bin;
        u64 s = 0;
        for (int y = 0; y < bin; ++y, row += N)
            for (int x = 0; x < bin; ++x) {
                const uint32_t c = row[x];
                s += c;
                v[0] += c != 0;
            }
        v[1] += s;
        v[2] += s * s;
    }
    block_add<3>(v, stats);
}

// ------------------------------------------------------------------ ordering
__device__ __forceinline__ int sgn(float d_hi, float d_lo) { return (d_hi > d_lo) - (d_hi < d_lo); }

// Rows i of the pair triangle, strided over the blocks; the threads of a
// block sweep j > i.
__global__ __launch_bounds__(kThreads) void k_ordering(const float2* __restrict__ a, const float2* __restrict__ b,
                                                       int n, u64* __restrict__ kept) {
    u64 v[3] = {0, 0, 0};
    for (int i = blockIdx.x; i < n - 1; i += gridDim.x) {
        const float2 ai = a[i], bi = b[i];
        for (int j = i + 1 + (int)threadIdx.x; j < n; j += kThreads) {
            const float2 aj = a[j], bj = b[j];
            const bool kx = sgn(aj.x, ai.x) == sgn(bj.x, bi.x);
            const bool ky = sgn(aj.y, ai.y) == sgn(bj.y, bi.y);
            v[0] += kx;
            v[1] += ky;
            v[2] += kx && ky;
        }
    }
    block_add<3>(v, kept);
}

// ------------------------------------------------------------------ trust
// Squared distance in float64 with each operation rounded on its own: no
// fused multiply-add, so the neighbour order is that of the plain formula.
__device__ __forceinline__ double sq_dist(float2 p, float2 q) {
#pragma clang fp contract(off)
    const double dx = (double)q.x - (double)p.x;
    const double dy = (double)q.y - (double)p.y;
    return dx * dx + dy * dy;
}

// Neighbour order of a sample: by squared distance, ties by index.
__device__ __forceinline__ bool before(double d1, int j1, double d2, int j2) {
    return d1 < d2 || (d1 == d2 && j1 < j2);
}

// One block per sample i (strided).  The k nearest neighbours of i in b are
// found one at a time, each the nearest after the previous one in the
// neighbour order, by a block-wide arg-min; each one's rank in a is one plus
// the number of samples before it in a's order, a block-wide count.
__global__ __launch_bounds__(kThreads) void k_trust(const float2* __restrict__ a, const float2* __restrict__ b,
                                                    int n, int k, u64* __restrict__ penalty) {
    __shared__ double best_d[2][kWaves];
    __shared__ int best_j[2][kWaves];
    __shared__ int below[2][kWaves];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    u64 pen = 0;
    int slot = 0;  // the shared slots alternate, so one barrier per reduction suffices
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const float2 ai = a[i], bi = b[i];
        double prev_d = -1.0;
        int prev_j = -1;
        for (int t = 0; t < k; ++t, slot ^= 1) {
            double bd = INFINITY;
            int bj = INT_MAX;
            for (int j = threadIdx.x; j < n; j += kThreads) {
                if (j == i) continue;
                const double d = sq_dist(bi, b[j]);
                if (before(prev_d, prev_j, d, j) && before(d, j, bd, bj)) {
                    bd = d;
                    bj = j;
                }
            }
            for (int o = kWave / 2; o > 0; o >>= 1) {
                const double od = __shfl_xor(bd, o, kWave);
                const int oj = __shfl_xor(bj, o, kWave);
                if (before(od, oj, bd, bj)) {
                    bd = od;
                    bj = oj;
                }
            }
            if (lane == 0) {
                best_d[slot][wave] = bd;
                best_j[slot][wave] = bj;
            }
            __syncthreads();
            bd = best_d[slot][0];
            bj = best_j[slot][0];
            for (int w = 1; w < kWaves; ++w)
                if (before(best_d[slot][w], best_j[slot][w], bd, bj)) {
                    bd = best_d[slot][w];
                    bj = best_j[slot][w];
                }
            if (bj >= n) break;  // unreachable for k < n - 1; keeps a[bj] in bounds
            prev_d = bd;
            prev_j = bj;
            const double dj = sq_dist(ai, a[bj]);
            int c = 0;
            for (int m = threadIdx.x; m < n; m += kThreads)
                if (m != i) c += before(sq_dist(ai, a[m]), m, dj, bj);
            for (int o = kWave / 2; o > 0; o >>= 1) c += __shfl_xor(c, o, kWave);
            if (lane == 0) below[slot][wave] = c;
            __syncthreads();
            int rank = 1;
            for (int w = 0; w < kWaves; ++w) rank += below[slot][w];
            if (rank > k) pen += (u64)(rank - k);
        }
    }
    if (threadIdx.x == 0 && pen) atomicAdd(penalty, pen);
}

// k <= 16: one pass per space.  Output space: every wave keeps the k nearest
// of its share of the samples as a sorted list with one entry per lane
// (lanes k..63 hold entries pushed past the k-th), updated only by the
// candidates that beat its current k-th entry; the four lists are merged by
// rank in LDS.  Input space: one pass counts, for each of the k neighbours,
// the samples before it in the neighbour order; only samples before the last
// of the k can count.  Same order, ties and sums as k_trust.
constexpr int kTrustFastK = 16;

__global__ __launch_bounds__(kThreads) void k_trust_fast(const float2* __restrict__ a, const float2* __restrict__ b,
                                                         int n, int k, u64* __restrict__ penalty) {
    __shared__ double cand_d[kWaves][kTrustFastK];
    __shared__ int cand_j[kWaves][kTrustFastK];
    __shared__ double top_d[kTrustFastK];  // input-space distance of the output neighbours
    __shared__ int top_j[kTrustFastK];
    __shared__ int below[kTrustFastK];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    u64 pen = 0;
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const float2 ai = a[i], bi = b[i];
        double Ld = INFINITY, thr_d = INFINITY;
        int Lj = INT_MAX, thr_j = INT_MAX;  // the lane's list entry; the wave's k-th entry
        for (int base = wave * kWave; base < n; base += kThreads) {
            const int j = base + lane;
            double d = INFINITY;
            int jj = INT_MAX;
            if (j < n && j != i) {
                d = sq_dist(bi, b[j]);
                jj = j;
            }
            u64 m = __ballot(before(d, jj, thr_d, thr_j));
            while (m) {
                const int src = __ffsll((long long)m) - 1;
                m &= m - 1;
                const double cd = __shfl(d, src, kWave);
                const int cj = __shfl(jj, src, kWave);
                if (!before(cd, cj, thr_d, thr_j)) continue;  // the k-th entry moved past it
                const double ud = __shfl_up(Ld, 1, kWave);
                const int uj = __shfl_up(Lj, 1, kWave);
                if (before(cd, cj, Ld, Lj)) {
                    if (lane == 0 || before(ud, uj, cd, cj)) {
                        Ld = cd;  // the candidate's place
                        Lj = cj;
                    } else {
                        Ld = ud;  // entries after it move one lane on
                        Lj = uj;
                    }
                }
                thr_d = __shfl(Ld, k - 1, kWave);
                thr_j = __shfl(Lj, k - 1, kWave);
            }
        }
        if (lane < k) {
            cand_d[wave][lane] = Ld;
            cand_j[wave][lane] = Lj;
        }
        if (threadIdx.x < kTrustFastK) below[threadIdx.x] = 0;
        __syncthreads();
        // the k nearest of the (distinct) candidates: their rank among them
        if (threadIdx.x < kWaves * kTrustFastK) {
            const int w = threadIdx.x / kTrustFastK, t = threadIdx.x % kTrustFastK;
            if (t < k && cand_j[w][t] < n) {
                const double d = cand_d[w][t];
                const int j = cand_j[w][t];
                int r = 0;
                for (int w2 = 0; w2 < kWaves; ++w2)
                    for (int t2 = 0; t2 < k; ++t2)
                        r += cand_j[w2][t2] < n && before(cand_d[w2][t2], cand_j[w2][t2], d, j);
                if (r < k) {
                    top_j[r] = j;
                    top_d[r] = sq_dist(ai, a[j]);
                }
            }
        }
        __syncthreads();
        double last_d = -1.0;
        int last_j = -1;
        for (int t = 0; t < k; ++t)
            if (before(last_d, last_j, top_d[t], top_j[t])) {
                last_d = top_d[t];
                last_j = top_j[t];
            }
        for (int m = threadIdx.x; m < n; m += kThreads) {
            if (m == i) continue;
            const double d = sq_dist(ai, a[m]);
            if (!before(d, m, last_d, last_j)) continue;
            for (int t = 0; t < k; ++t)
                if (before(d, m, top_d[t], top_j[t])) atomicAdd(&below[t], 1);
        }
        __syncthreads();
        if (threadIdx.x == 0)
            for (int t = 0; t < k; ++t) {
                const int rank = 1 + below[t];
                if (rank > k) pen += (u64)(rank - k);
            }
        __syncthreads();  // the shared lists are rewritten for the next sample
    }
    if (threadIdx.x == 0 && pen) atomicAdd(penalty, pen);
}

// ------------------------------------------------------------------ host
thread_local std::string g_quality_error;

int qfail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int qfail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_quality_error = buf;
    return code;
}

int launched(const char* what) {
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? INIM_OK : qfail(INIM_EHIP, "%s: %s", what, hipGetErrorString(e));
}

unsigned capped(int64_t blocks, int64_t cap) {
    if (blocks < 1) blocks = 1;
    return (unsigned)(blocks < cap ? blocks : cap);
}

}  // namespace

extern "C" {

const char* inim_quality_last_error(void) { return g_quality_error.c_str(); }

int inim_quality_bins(const uint32_t* counts, int32_t res, int32_t bin, uint64_t* stats, hipStream_t stream) {
    if (!counts || !stats) return qfail(INIM_EINVAL, "counts and stats must not be NULL");
    if (res < 1 || res > 65536 || bin < 1 || res % bin)
        return qfail(INIM_EINVAL, "bins of %d texels do not tile a %d x %d raster", bin, res, res);
    const int64_t nb = res / bin;
    hipLaunchKernelGGL(k_bins, dim3(capped((nb * nb + kThreads - 1) / kThreads, 4096)), dim3(kThreads), 0, stream,
                       counts, res, bin, (u64*)stats);
    return launched("bin counts");
}

int inim_quality_ordering(const float* a, const float* b, int32_t n, uint64_t* kept, hipStream_t stream) {
    if (!kept || n < 0 || (n > 0 && (!a || !b))) return qfail(INIM_EINVAL, "bad ordering arguments (n = %d)", n);
    if (n < 2) return INIM_OK;
    hipLaunchKernelGGL(k_ordering, dim3(capped(n - 1, 16384)), dim3(kThreads), 0, stream, (const float2*)a,
                       (const float2*)b, n, (u64*)kept);
    return launched("orthogonal ordering");
}

int inim_quality_trust(const float* a, const float* b, int32_t n, int32_t k, uint64_t* penalty,
                       hipStream_t stream) {
    if (!a || !b || !penalty) return qfail(INIM_EINVAL, "a, b and penalty must not be NULL");
    if (k < 1 || 2 * (int64_t)k >= n) return qfail(INIM_EINVAL, "need 1 <= k and 2k < n (k = %d, n = %d)", k, n);
    if (k <= kTrustFastK)
        hipLaunchKernelGGL(k_trust_fast, dim3(capped(n, 1 << 20)), dim3(kThreads), 0, stream, (const float2*)a,
                           (const float2*)b, n, k, (u64*)penalty);
    else
        hipLaunchKernelGGL(k_trust, dim3(capped(n, 1 << 20)), dim3(kThreads), 0, stream, (const float2*)a,
                           (const float2*)b, n, k, (u64*)penalty);
    return launched("trustworthiness");
}

}  // extern "C"
