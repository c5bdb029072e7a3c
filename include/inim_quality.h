/*
 * inim_quality.h -- C ABI of the layout quality measures that rate a
 * regularised scatterplot (Sec. 6, numerical tests): the sample counts per
 * 4 x 4-texel bin and the occupied texels behind the regularity measure and
 * overplotting, and the two neighbourhood measures the paper reports against
 * other layouts, trustworthiness (Venna and Kaski) and orthogonal ordering
 * (Misue et al.).
 *
 * Every call returns exact integer sums, added into device uint64 counters
 * that the caller clears; the measures are simple functions of them:
 *   bin std       = sqrt(S2 / B - (S1 / B)^2), B = (res / bin)^2 bins
 *   overplotting  = (n - occupied) / n
 *   trust         = 1 - 2 P / (n k (2n - 3k - 1))
 *   ordering      = kept_both / (n (n - 1) / 2)
 * Integer atomics make the sums independent of the order of the additions,
 * so results are deterministic and bit-identical to any exact evaluation.
 *
 * Positions are device float [n][2] (x, y), finite.  Work is enqueued on
 * `stream`; nothing is allocated or synchronised.  Return INIM_OK,
 * INIM_EINVAL (NULL pointer or bad size) or INIM_EHIP; the text of the last
 * error of this thread is inim_quality_last_error().
 */
#ifndef INIM_QUALITY_H
#define INIM_QUALITY_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

const char* inim_quality_last_error(void);

/* From a res x res raster of per-texel sample counts (inim_rasterize with
 * radius 0) split into bin x bin texel blocks: adds to stats[0] the number of
 * texels with a non-zero count, to stats[1] the sum of the block counts
 * (the number of samples) and to stats[2] the sum of the squared block
 * counts.  1 <= bin, res % bin == 0, res <= 65536. */
int inim_quality_bins(const uint32_t* counts, int32_t res, int32_t bin, uint64_t* stats, hipStream_t stream);

/* Orthogonal ordering of the mapping a -> b of n samples: over the unordered
 * pairs (i, j), a pair is kept along x when the sign (-1, 0, +1) of
 * x_j - x_i is the same in a and b, likewise along y.  Adds to kept[0],
 * kept[1], kept[2] the pairs kept along x, along y, along both.  n < 2 adds
 * nothing. */
int inim_quality_ordering(const float* a, const float* b, int32_t n, uint64_t* kept, hipStream_t stream);

/* Trustworthiness penalty of the mapping a -> b of n samples with k
 * neighbours: adds to *penalty the sum over samples i of r(i, j) - k over the
 * j among the k nearest neighbours of i in b that are not among its k nearest
 * in a, r(i, j) being the rank of j in a (1 = nearest).  Neighbours are
 * ordered by squared distance dx*dx + dy*dy in float64 with every operation
 * rounded (dx the difference of the float32 coordinates taken as float64),
 * ties by sample index.  1 <= k and 2k < n. */
int inim_quality_trust(const float* a, const float* b, int32_t n, int32_t k, uint64_t* penalty,
                       hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* INIM_QUALITY_H */
