// k_raster.hip -- per-sample and per-texel kernels of the regularisation on
// gfx950: the single-pixel splat and the separable Gaussian of Sec. 4.1,
// bilinear advection of Sec. 4.2, input validation and fills.
#include <hip/hip_runtime.h>

#include "blur_tile.h"
#include "device_common.h"
#include "launch.h"

namespace inim {

// Sets the status word when a sample is NaN or outside [0,1]^2.
__device__ __forceinline__ bool in_unit_square(float2 p) {
    return p.x >= 0.0f && p.x <= 1.0f && p.y >= 0.0f && p.y <= 1.0f;  // false for NaN
}

__device__ __forceinline__ void flag_domain(int* status) {
    __hip_atomic_store(status, (int)INIM_EDOMAIN, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------------ fill
__global__ __launch_bounds__(256) void k_fill(uint32_t* __restrict__ counts, size_t count, int* status, int clear) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (clear && t == 0) *status = 0;
    typedef uint32_t u4 __attribute__((ext_vector_type(4)));
    const size_t n4 = count / 4;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const u4 z = {0u, 0u, 0u, 0u};
    for (size_t k = t; k < n4; k += stride) reinterpret_cast<u4*>(counts)[k] = z;
    for (size_t k = n4 * 4 + t; k < count; k += stride) counts[k] = 0u;
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

__global__ __launch_bounds__(256) void k_validate(const float2* __restrict__ xy, int64_t n, int* status) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride)
        if (!in_unit_square(xy[p])) flag_domain(status);
}

// ------------------------------------------------------------------ blur
// One 64 x 16 output tile per 256-thread block (blur_tile.h).
__global__ __launch_bounds__(256) void k_blur(const uint32_t* __restrict__ counts, float* __restrict__ out, int N,
                                              BlurTaps taps, const int* status) {
    extern __shared__ float lds[];
    if (failed(status)) return;
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

// counts_next (optional): each moved sample is also splatted into it, the
// count raster of the next iteration (Sec. 4.3, step 1 of the next round).
__global__ __launch_bounds__(256) void k_advect(const float2* __restrict__ field, int N, float2* __restrict__ xy,
                                                int64_t n, uint32_t* __restrict__ counts_next, const int* status) {
    if (failed(status)) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        const float2 q = xy[p];
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
        const float2 o = make_float2(clamp01(nx), clamp01(ny));
        xy[p] = o;
        if (counts_next != nullptr)
            __hip_atomic_fetch_add(counts_next + (size_t)texel_of(o.y, N) * N + texel_of(o.x, N), 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ------------------------------------------------------------------ launchers
static unsigned grid_for(int64_t n, int per_block = 256, unsigned cap = 8192) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    return (unsigned)(g > cap ? cap : g);
}

hipError_t launch_fill(uint32_t* counts, size_t count, int* status, bool clear_status, hipStream_t st) {
    hipLaunchKernelGGL(k_fill, dim3(grid_for((int64_t)(count / 4 + 1), 256, 2048)), dim3(256), 0, st, counts, count,
                       status, clear_status ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_splat(const float2* xy, int64_t n, int N, uint32_t* counts, int* status, hipStream_t st) {
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
    hipLaunchKernelGGL(k_blur, grd, dim3(256), smem, st, counts, out, N, taps, status);
    return hipGetLastError();
}

hipError_t launch_advect(const float2* field, int N, float2* xy, int64_t n, uint32_t* counts_next, const int* status,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_advect, dim3(grid_for(n)), dim3(256), 0, st, field, N, xy, n, counts_next, status);
    return hipGetLastError();
}

}  // namespace inim
