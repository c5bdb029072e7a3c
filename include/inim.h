/*
 * inim.h -- C ABI of the MI355X (gfx950) scatterplot regulariser built on
 * integral images, after Rave, Molchanov and Linsen, "De-cluttering
 * Scatterplots with Integral Images" (IEEE TVCG; arXiv 2408.06513).
 *
 * Conventions shared by every entry point
 *   - A raster has res x res texels, res = 2^k with 2 <= res <= 16384 (the
 *     paper's 2^k x 2^k textures, Sec. 3.2 and Sec. 4.1).  It is stored
 *     row-major: texel (i, j) -- column i (x), row j (y), origin top-left
 *     (Sec. 4.1) -- lives at index j * res + i.
 *   - Samples are float32 pairs (x, y) in [0, 1]^2 (Sec. 4.1), array [n][2].
 *   - Texel (i, j) stands for the point ((i + 1/2) / res, (j + 1/2) / res).
 *   - Every pointer argument named as device memory is HIP device memory
 *     owned by the caller.  The library never allocates, frees or synchronises
 *     device memory; all work is enqueued on `stream` (0 = the null stream)
 *     and runs asynchronously.  Only inim_sync_status synchronises.
 *   - Scratch memory is the caller's `ws` buffer (device memory, 256-byte
 *     aligned, at least the size the matching *_workspace_size call reports).
 *     Its first 256 bytes hold a status word that the kernels of one call set
 *     when they meet invalid data; each call clears it when it starts.  Calls
 *     that share a workspace must not overlap in time.
 *   - Errors found on the host are returned synchronously before anything is
 *     enqueued; the text of the last one is available from inim_last_error()
 *     (thread-local).
 *
 * Plane bits (Sec. 3.1), in this order wherever several planes are stored:
 *   alpha   sum over i' <= i, j' <= j          beta    i' <= i, j' >  j
 *   gamma   i' >  i, j' >  j                   delta   i' >  i, j' <= j
 *   alpha_t i'+j' <= i+j, i'-j' >= i-j         beta_t  i'+j' <= i+j, i'-j' <  i-j
 *   gamma_t i'+j' >  i+j, i'-j' <  i-j         delta_t i'+j' >  i+j, i'-j' >= i-j
 *
 * Marginals (double, device memory), layout
 *   X[res] | Y[res] | U[2res-1] | V[2res-1] | C
 *   X(i) = sum over i' <= i;  Y(j) = sum over j' <= j;  U(u) = sum over
 *   i'+j' <= u;  V[k] = sum over i'-j' >= k-(res-1);  C = total (Sec. 3.1).
 */
#ifndef INIM_H
#define INIM_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    INIM_OK = 0,
    INIM_EINVAL = 1,     /* bad argument (size, pointer, mask, parameter) */
    INIM_EDOMAIN = 2,    /* a sample is NaN or outside [0,1]^2 (reported by inim_sync_status) */
    INIM_ERANGE = 3,     /* n >= 2^32 where counts are 32-bit */
    INIM_EWORKSPACE = 4, /* ws is NULL, misaligned or smaller than required */
    INIM_EHIP = 5        /* a HIP call failed; see inim_last_error() */
} inim_status;

enum {
    INIM_ALPHA = 1u << 0,
    INIM_BETA = 1u << 1,
    INIM_GAMMA = 1u << 2,
    INIM_DELTA = 1u << 3,
    INIM_ALPHA_T = 1u << 4,
    INIM_BETA_T = 1u << 5,
    INIM_GAMMA_T = 1u << 6,
    INIM_DELTA_T = 1u << 7,
    INIM_MIN = INIM_ALPHA | INIM_ALPHA_T,
    INIM_ALL = 0xFFu
};

typedef enum { INIM_U32 = 0, INIM_F32 = 1 } inim_dtype;

/*
 * Smoothing and background parameters (Sec. 4.1, eq. (dr) and eq. (d0)).
 *   radius  Gaussian taps |m| <= radius along each axis, 0 <= radius <= 32;
 *           0 means no smoothing (the count raster itself is the density).
 *   sigma   Gaussian standard deviation in texels; <= 0 selects radius / 2.
 *   d0      background density added to every texel; < 0 selects the paper's
 *           choice n / res^2 (average samples per texel).
 * Defaults (inim_default_params): radius 8, sigma 0 (unset: radius / 2 of the
 * radius in force when the call runs, so a caller who only raises the radius
 * gets the matching sigma), d0 = -1.
 */
typedef struct {
    int32_t radius;
    float sigma;
    double d0;
} inim_params;

void inim_default_params(inim_params* p);

/* Static description of a status code; never NULL. */
const char* inim_strerror(int status);

/* Thread-local text of the last host-side error of this thread ("" if none). */
const char* inim_last_error(void);

/*
 * Workspace for inim_rasterize, inim_advect and inim_regularize at this size:
 * status word, two count rasters, density raster, deformation field, the
 * integral-image carries, a texel-ordered copy of the samples and the
 * buffers that sort them (24 bytes per sample).  `p` may be NULL (defaults).  EINVAL on bad sizes.
 */
int inim_workspace_size(int32_t res, int64_t n, const inim_params* p, size_t* bytes);

/* Workspace for inim_inim_u32 / inim_inim_f32 at this size and type. */
int inim_inim_workspace_size(int32_t res, inim_dtype dt, size_t* bytes);

/*
 * Step 1 of the algorithm (Sec. 4.3; density field of Sec. 4.1): every sample
 * adds one to texel (min(floor(x res), res-1), min(floor(y res), res-1));
 * then the counts are convolved with the normalised separable Gaussian of
 * `p`, the raster continued across its border by half-sample symmetric
 * reflection (... c b a | a b c ...).
 *   xy       device, float [n][2], read only.
 *   counts   device, uint32 [res*res], written (exact sample counts).
 *   density  device, float [res*res], written with the smoothed counts; may be
 *            NULL.  With radius 0 it receives the counts as floats.
 * A NaN or out-of-range sample sets the status word (EDOMAIN); the counts are
 * then incomplete.  ERANGE if n >= 2^32.
 */
int inim_rasterize(const float* xy, int64_t n, int32_t res, const inim_params* p,
                   uint32_t* counts, float* density, void* ws, size_t ws_bytes,
                   hipStream_t stream);

/*
 * Step 2 (Sec. 3.1 and Sec. 4.4): the integral images selected by `mask` of a
 * res x res raster, plus all marginals.
 *   img      device, uint32 or float [res*res], read only.
 *   planes   device, [popcount(mask)][res*res] of the input's type, planes in
 *            bit order; written.  May be NULL when mask == 0.
 *   marg     device, double [6 res - 1], the marginals above; may be NULL.
 * uint32: planes and marginals are exact modulo 2^32 (exact when the total is
 * below 2^32).  float: every input is taken exactly as a 128-bit fixed-point
 * number with 64 fractional bits (exact for magnitudes in [2^-64, 2^62); a
 * smaller magnitude is truncated toward zero), all sums and complements are
 * formed exactly in that integer format, and each output is rounded once to
 * float (planes) or double (marginals).  Hence every plane element is the
 * correctly rounded region sum, within one float rounding, and regions that
 * are empty are exactly 0, provided the total magnitude stays below 2^63.
 * When mask selects at most alpha and alpha_t (no complement), a float
 * raster is summed in double: for non-negative values (sums without
 * cancellation) every element is then within about 1e-12 relative of the
 * exact sum before its rounding to float.  If the raster holds a negative or
 * non-finite value, the exact path above runs instead, decided on the device
 * within the same call.
 * EINVAL for a bad size, an unknown mask bit or a NULL plane pointer with a
 * non-zero mask; EWORKSPACE if ws is too small.
 */
int inim_inim_u32(const uint32_t* img, int32_t res, uint32_t mask, uint32_t* planes,
                  double* marg, void* ws, size_t ws_bytes, hipStream_t stream);
int inim_inim_f32(const float* img, int32_t res, uint32_t mask, float* planes,
                  double* marg, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Step 3, per texel (Sec. 4.2 eq. (map_res) built on Sec. 3.2 eq. (map)):
 *   T(p) = p + t(p; d_r + d0) - t(p; d0)
 * where the eight planes of d_r are rebuilt from alpha, alpha_t and the
 * marginals, and those of the constant d0 are exact closed forms (the defect
 * t(p; d0) does not depend on the value of d0 > 0).
 *   alpha, alpha_t  device planes of d_r (inim_inim_* output, type `dt`).
 *   marg            device marginals of d_r (inim_inim_* output).
 *   d0              background density, >= 0.
 *   field           device, float [res*res][2] (x, y per texel); written.
 */
int inim_deform(const void* alpha, const void* alpha_t, inim_dtype dt, const double* marg,
                int32_t res, double d0, float* field, hipStream_t stream);

/*
 * Steps 2 and 3 of one iteration on a given density (Sec. 4.2 eq. (map_res),
 * Sec. 3.1 planes): the field T(p) at every texel centre of the res x res
 * float density d_r with background d0, by the kernels of one iteration of
 * inim_regularize after its smoothing: the integral images accumulated in
 * double and the map evaluated in their last pass, so alpha and alpha_t never
 * reach memory (res >= 64; smaller rasters take a separate marginals pass).
 * The defect t(p; 1) is recomputed into the workspace by every call.
 *   density   device, float [res*res], row-major; meant for non-negative
 *             densities (a smoothed count raster): sums of mixed signs are
 *             only as exact as double arithmetic makes them.
 *   d0        background density, finite, >= 0 (the method uses n / res^2).
 *   field     device, float [res*res][2]; written.
 *   ws        device workspace of inim_deform_density_workspace_size(res)
 *             bytes, 256-byte aligned; owned by the caller.
 * Returns EINVAL for bad arguments, EWORKSPACE for a small ws, before
 * anything is enqueued.
 */
int inim_deform_density_workspace_size(int32_t res, size_t* bytes);
int inim_deform_density(const float* density, int32_t res, double d0, float* field, void* ws,
                        size_t ws_bytes, hipStream_t stream);

/*
 * Step 3, per sample (Sec. 4.2): each sample takes the bilinear interpolation
 * of `field` from the four nearest texel centres.  The cell index is clamped
 * to [0, res-2] and the fraction is not, so border samples extrapolate
 * linearly; the result is clamped to [0,1]^2.
 *   field  device, float [res*res][2], read only.
 *   xy     device, float [n][2], updated in place.
 * If any sample is NaN or outside [0,1]^2 the status word is set (EDOMAIN) and
 * no sample is modified.
 */
int inim_advect(const float* field, int32_t res, float* xy, int64_t n, void* ws,
                size_t ws_bytes, hipStream_t stream);

/*
 * inim_rasterize for `count` sample sets in shared launches (the surrogate's
 * input for a batch of scatterplots): set q has n[q] samples at xy[q] (host
 * arrays of device pointers and sizes, 1 <= count <= 64), and its counts and
 * density are the q-th res x res raster of `counts` (uint32 [count][res][res])
 * and `density` (float [count][res][res], may be NULL).  Each raster is the
 * one inim_rasterize gives for that set; a NaN or out-of-range sample in any
 * set sets the one status word (EDOMAIN).  ws: at least 256 bytes.
 */
int inim_rasterize_many(float* const* xy, const int64_t* n, int32_t count, int32_t res, const inim_params* p,
                        uint32_t* counts, float* density, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * inim_advect for `count` sample sets in shared launches: set q (n[q]
 * samples at xy[q], host arrays as in inim_rasterize_many) moves through the
 * q-th field of `field` (float [count][res][res][2]), in place.  If any sample
 * of any set is NaN or outside [0,1]^2 the status word is set (EDOMAIN) and
 * no sample is modified.  ws: at least 256 bytes.
 */
int inim_advect_many(const float* field, int32_t res, float* const* xy, const int64_t* n, int32_t count, void* ws,
                     size_t ws_bytes, hipStream_t stream);

/*
 * The whole algorithm (Sec. 4.3): `iters` times splat + smooth, integral
 * images, per-texel deformation and bilinear advection, in place on xy.
 *   xy     device, float [n][2], updated in place.
 *   n == 0 or iters == 0 is a no-op returning INIM_OK.
 * Device-side errors (EDOMAIN) leave xy unchanged and are reported by
 * inim_sync_status.  ERANGE if n >= 2^32.
 */
int inim_regularize(float* xy, int64_t n, int32_t res, int32_t iters, const inim_params* p,
                    void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * inim_regularize with probe points (Sec. 4.3; the deformed grid of Sec. 5
 * without its rendering): the m points of `probe` are moved by the same
 * per-texel deformation as the samples in every iteration, but are never
 * splatted, so they do not change the density or the samples' results.
 * Started at the texel centres, the probes end up holding the composite map
 * T_iters o ... o T_1 of all iterations on the texel lattice.
 *   probe  device, float [m][2] in [0,1]^2, updated in place; may be NULL
 *          when m == 0.
 * xy, n, res, iters, p, ws as for inim_regularize (same workspace size).
 * n == 0 or iters == 0 is a no-op that leaves the probes unchanged.  A NaN or
 * out-of-range probe is reported like an invalid sample (EDOMAIN from
 * inim_sync_status; samples and probes unchanged).  EINVAL if m < 0 or probe
 * is NULL with m > 0.
 */
int inim_regularize_probes(float* xy, int64_t n, float* probe, int64_t m, int32_t res, int32_t iters,
                           const inim_params* p, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * inim_regularize instrumented for measurement: records HIP events on
 * `stream` -- around the per-call sort and unsort, and for each per-iteration
 * stage at the start of its first kernel and the end of its last kernel
 * (the launch-gap-free kernel span) -- synchronises after each iteration,
 * and adds the elapsed milliseconds into stage_ms[0..5]:
 *   0 once per call: sorting the samples by texel (count raster cleared,
 *     every sample splatted with its rank, counts scanned, samples moved),
 *     and moving the results back to the caller's order at the end
 *   1 smoothing + tile partial sums of the integral images (per iteration)
 *   2 integral-image carries, the band scans (per iteration)
 *   3 integral images + per-texel deformation (per iteration)
 *   4 advection, which also splats the moved samples for the next iteration
 *   5 the whole call.
 * stage_ms is host memory and is not cleared.  Same results as inim_regularize.
 */
int inim_regularize_timed(float* xy, int64_t n, int32_t res, int32_t iters, const inim_params* p,
                          void* ws, size_t ws_bytes, hipStream_t stream, double* stage_ms);

/*
 * Graph replay of inim_regularize for callers that repeat the same call
 * (Sec. 4.3 run many times, e.g. every frame of an interactive view).
 * inim_graph_create makes an empty handle (host memory owned by the caller,
 * released with inim_graph_destroy).  inim_regularize_graph behaves exactly
 * like inim_regularize with the same arguments; the first call with a given
 * (xy, n, res, iters, params, ws, ws_bytes) captures the whole launch
 * sequence into a HIP graph on a private stream, and this and every later
 * call with the same arguments launch that graph on `stream`.  Different
 * arguments re-capture.  A handle must not be used by two threads at once.
 * EHIP if capture or instantiation fails.
 */
int inim_graph_create(void** graph);
int inim_graph_destroy(void* graph);
int inim_regularize_graph(float* xy, int64_t n, int32_t res, int32_t iters, const inim_params* p,
                          void* ws, size_t ws_bytes, void* graph, hipStream_t stream);

/*
 * Several plots in one call (Sec. 4.3 for each plot of a scatterplot matrix,
 * Sec. 6): `count` plots, plot k with its own samples xy[k] (device, float
 * [n[k]][2], updated in place) on its own res[k] x res[k] raster, all with
 * the same iteration count and parameters (d0 < 0 selects n[k] / res[k]^2 per
 * plot).  Every stage of the iteration is one launch over the tiles and
 * samples of all plots, so small plots fill the GPU together.  Each plot gets
 * exactly the result of inim_regularize for it alone (bit for bit).
 *   xy, n, res  host arrays of `count` entries; 0 <= count <= 64;
 *               64 <= res[k] <= 2048 (powers of two); plots with n[k] == 0
 *               are left alone.
 *   p           radius >= 1 (the smoothed-density path).
 *   cfg         launch shape, NULL for the default (see inim_batch_config);
 *               every shape gives the same results.
 *   ws          device workspace of inim_batch_workspace_size bytes.
 *   graph       NULL: plain launches; or a handle of inim_graph_create: the
 *               launch sequence is captured once per distinct argument set
 *               and replayed as one HIP graph.
 * A NaN or out-of-range sample in any plot makes the whole call a no-op
 * reported as EDOMAIN by inim_sync_status.  EINVAL for a bad count, size,
 * pointer or configuration.
 */
typedef struct {
    int32_t waves_per_block; /* tiles per block of the deformation stage: 1, 2, 4 or 8; 0 = 4 */
    int32_t order;           /* 0: plots in input order; 1: larger rasters first */
} inim_batch_config;

int inim_batch_workspace_size(float* const* xy, const int64_t* n, const int32_t* res, int32_t count,
                              const inim_params* p, size_t* bytes);
int inim_regularize_batch(float* const* xy, const int64_t* n, const int32_t* res, int32_t count, int32_t iters,
                          const inim_params* p, const inim_batch_config* cfg, void* ws, size_t ws_bytes, void* graph,
                          hipStream_t stream);

/*
 * Picks the fastest launch shape of inim_regularize_batch for these plots by
 * timing each candidate (waves_per_block 1, 2, 4, 8 x both orders) on the
 * device with the caller's data: every candidate runs the whole iteration
 * but leaves its results in the workspace, so xy is not modified.
 * Synchronises `stream`.  best (host) receives the winner, best_ms (host, may
 * be NULL) its time in milliseconds.  iters >= 1.
 */
int inim_batch_autotune(float* const* xy, const int64_t* n, const int32_t* res, int32_t count, int32_t iters,
                        const inim_params* p, void* ws, size_t ws_bytes, hipStream_t stream,
                        inim_batch_config* best, double* best_ms);

/*
 * inim_regularize without a caller workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  It runs the same kernels, on a static
 * scratch array of 64 MiB that the library holds on each GPU it runs on until
 * the process ends; nothing is allocated or freed.  The call fits when
 * inim_workspace_size(res, n, p) is at most 64 MiB: 1M samples at 1024^2
 * (55.5 MiB) or 2.4M samples at 512^2, for example; larger calls return
 * EWORKSPACE before anything is enqueued.
 *   xy, n, res, iters, p  as for inim_regularize; the results are identical.
 *   status  device, int; may be NULL.  When given, the call's status word is
 *           kept there (it is cleared when the call starts) and
 *           inim_sync_status(status, stream) reports EDOMAIN for NaN or
 *           out-of-range samples; with NULL such a call leaves xy unchanged
 *           and the error is not reported.
 * The current device must be the device of `stream` (EINVAL otherwise).  The
 * scratch is looked up once per device.  All calls on one GPU share its
 * scratch, which keeps the last call's contents: two calls that overlap in
 * time on one GPU (other streams, other host threads) race and give wrong
 * results.
 */
int inim_regularize_noalloc(float* xy, int64_t n, int32_t res, int32_t iters, const inim_params* p, int* status,
                            hipStream_t stream);

/*
 * Waits for `stream`, returns the status word of the last call that used ws
 * (INIM_OK or INIM_EDOMAIN) and clears it.  EHIP if the synchronisation fails.
 */
int inim_sync_status(void* ws, hipStream_t stream);


#ifdef __cplusplus
}
#endif

#endif /* INIM_H */
