// k_inim.hip -- integral images of Sec. 3.1 on gfx950.
//
// Decomposition (all sums exact in uint32, or in double for float rasters):
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
//   2. chain_col  per column, over bands: the column-prefix and alpha carries;
//   3. chain_diag per diagonal, over bands: the L and R carries;
//   4. final      one wave per tile again: rebuilds cp, alpha, L, R with the
//                 carries (boundary values of the neighbouring tiles come from
//                 the partial sums) and writes the requested planes, or the
//                 deformation of Sec. 4.2 directly.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "inim_plan.h"
#include "launch.h"

namespace inim {

constexpr int kWavesPerBlock = 4;
constexpr int kPF = 4;  // rows prefetched ahead

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
template <int Q, typename Tin>
__global__ __launch_bounds__(256) void k_inim_aggregate(const Tin* __restrict__ img, Geom g,
                                                        Agg<typename AccOf<Tin>::type> A,
                                                        const int* status) {
    using Acc = typename AccOf<Tin>::type;
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

    Acc cp[Q], L[Q], R[Q];
#pragma unroll
    for (int e = 0; e < Q; ++e) cp[e] = L[e] = R[e] = Acc(0);

    Tin buf[kPF][Q];
#pragma unroll
    for (int p = 0; p < kPF; ++p)
        if (p < g.H) load_tile_row<Tin, Q>(src + (size_t)p * N, act, buf[p]);

    for (int r0 = 0; r0 < g.H; r0 += kPF) {
#pragma unroll
        for (int p = 0; p < kPF; ++p) {
            const int r = r0 + p;
            if (r < g.H) {
                Tin v[Q];
#pragma unroll
                for (int e = 0; e < Q; ++e) v[e] = buf[p][e];
                if (r + kPF < g.H) load_tile_row<Tin, Q>(src + (size_t)(r + kPF) * N, act, buf[p]);

#pragma unroll
                for (int e = 0; e < Q; ++e) cp[e] += to_acc<Acc, Tin>(v[e]);
                Acc upL = shfl_up1(L[Q - 1]);
                Acc dnR = shfl_down1(R[0]);
                if (lane == 0) upL = Acc(0);
                if (lane >= g.lastLane) dnR = Acc(0);
#pragma unroll
                for (int e = Q - 1; e >= 1; --e) L[e] = cp[e] + L[e - 1];
                L[0] = cp[0] + upL;
#pragma unroll
                for (int e = 0; e < Q - 1; ++e) R[e] = cp[e] + R[e + 1];
                R[Q - 1] = cp[Q - 1] + dnR;

                Acc s = Acc(0);
#pragma unroll
                for (int e = 0; e < Q; ++e) s += cp[e];
                s = wave_sum(s);
                if (lane == 0) {
                    A.trow[ebase + r] = s;
                    A.tRedge[ebase + r] = R[0];
                }
                if (lane == g.lastLane) A.tLedge[ebase + r] = L[Q - 1];
            }
        }
    }

    // band-level outputs: column sums, their in-tile prefix, diagonal sums
    Acc pre[Q];
    Acc run = Acc(0);
#pragma unroll
    for (int e = 0; e < Q; ++e) { run += cp[e]; pre[e] = run; }
    Acc incl = wave_inclusive_scan(run);
    Acc ex = shfl_up1(incl);
    if (lane == 0) ex = Acc(0);
    if (act) {
        const size_t o = (size_t)b * N + col;
#pragma unroll
        for (int e = 0; e < Q; ++e) {
            A.colsum[o + e] = cp[e];
            A.tcsp[o + e] = ex + pre[e];
            A.tLend[o + e] = L[e];
            A.tRend[o + e] = R[e];
        }
    }
}

// ------------------------------------------------------------------ pass 2
// One thread per column i: cpin[b][i] and ain[b][i] = alpha(i, bH-1).
// alpha grows per band by the full-row prefix of the band's column sums:
// the in-tile prefix plus the totals of the tiles to the left (a wave-wide sum;
// tiles are at least 64 columns wide, so every lane of a wave lies in the same
// tile, or N < 64 and there is a single tile).
template <typename Acc>
__global__ __launch_bounds__(256) void k_inim_chain_col(Geom g, Agg<Acc> A, Carry<Acc> K,
                                                        const int* status) {
    if (failed(status)) return;
    const int lane = lane_id();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < g.N;
    const int ii = valid ? i : 0;
    const int c = ii / g.W;
    const size_t N = (size_t)g.N;
    Acc cp = Acc(0), a = Acc(0);
    for (int b = 0; b < g.B; ++b) {
        Acc cs = Acc(0), ts = Acc(0), t = Acc(0);
        if (valid) {
            cs = A.colsum[(size_t)b * N + ii];
            ts = A.tcsp[(size_t)b * N + ii];
        }
        for (int c0 = 0; c0 < c; c0 += 64)
            if (c0 + lane < c) t += A.trow[((size_t)b * g.T + c0 + lane) * g.H + (g.H - 1)];
        const Acc left = wave_sum(t);
        if (valid) {
            K.cpin[(size_t)b * N + ii] = cp;
            K.ain[(size_t)b * N + ii] = a;
        }
        cp += cs;
        a += left + ts;
    }
    if (valid) {
        K.cpin[(size_t)g.B * N + ii] = cp;
        K.ain[(size_t)g.B * N + ii] = a;
    }
}

// ------------------------------------------------------------------ pass 3
// 2N+1 threads; thread t follows the up-left chain s = t - N, i.e. texel
// columns i = s + (b+1)H at band boundaries b+1, and the up-right chain
// s' = t, columns i = s' - (b+1)H.
//   Lin[b+1][i] = sum_{k<H} cp(i-k, bH+H-1-k) + Lin[b][i-H]
//   Rin[b+1][i] = sum_{k<H} cp(i+k, bH+H-1-k) + Rin[b][i+H]
// where inside band b, cp = cpin[b] + band-local prefix: the cpin part is a
// window of cpin (a difference of ain), the band-local part is tLend/tRend
// plus, near a tile edge, the neighbouring tile's edge sum.
template <typename Acc>
__global__ __launch_bounds__(256) void k_inim_chain_diag(Geom g, Agg<Acc> A, Carry<Acc> K,
                                                         const int* status) {
    if (failed(status)) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int N = g.N, H = g.H, W = g.W, T = g.T;
    if (t > 2 * N) return;
    if (t < N) {
        K.Lin[t] = Acc(0);
        K.Rin[t] = Acc(0);
    }
    // up-left chain
    {
        const int s = t - N;
        // valid b: 0 <= s + (b+1)H <= N-1
        int blo = 0;
        if (s < 0) blo = (-s + H - 1) / H - 1;
        int bhi = (N - 1 - s) / H - 1;
        if (bhi > g.B - 1) bhi = g.B - 1;
        Acc prev = Acc(0);
        for (int b = blo; b <= bhi; ++b) {
            const int i = s + (b + 1) * H;
            const Acc* ainb = K.ain + (size_t)b * N;
            const Acc win = ainb[i] - (i >= H ? ainb[i - H] : Acc(0));
            const int c = i / W, x = i - c * W;
            Acc bl = A.tLend[(size_t)b * N + i];
            if (x < H - 1 && c > 0) bl += A.tLedge[((size_t)b * T + (c - 1)) * H + (H - 2 - x)];
            prev = win + bl + prev;
            K.Lin[(size_t)(b + 1) * N + i] = prev;
        }
    }
    // up-right chain
    {
        const int s = t;
        // valid b: 0 <= s - (b+1)H <= N-1
        int blo = 0;
        if (s - H > N - 1) blo = (s - (N - 1) + H - 1) / H - 1;
        int bhi = s / H - 1;
        if (bhi > g.B - 1) bhi = g.B - 1;
        Acc prev = Acc(0);
        for (int b = blo; b <= bhi; ++b) {
            const int i = s - (b + 1) * H;
            const Acc* ainb = K.ain + (size_t)b * N;
            const int hi = (i + H - 1 < N - 1) ? i + H - 1 : N - 1;
            const Acc win = ainb[hi] - (i >= 1 ? ainb[i - 1] : Acc(0));
            const int c = i / W, x = i - c * W;
            Acc br = A.tRend[(size_t)b * N + i];
            if (x > W - H && c < T - 1) br += A.tRedge[((size_t)b * T + (c + 1)) * H + (H - 2 - (W - 1 - x))];
            prev = win + br + prev;
            K.Rin[(size_t)(b + 1) * N + i] = prev;
        }
    }
}

// ------------------------------------------------------------------ marginals
// U(u) = sum over i'+j' <= u:  for u < N it is R(0, u); beyond, R(u-N+1, N-1)
// misses exactly the columns left of u-N+1, i.e. X(u-N).
template <typename Acc>
__device__ __forceinline__ Acc marg_U(const Geom& g, const Agg<Acc>& A, const Carry<Acc>& K, int u) {
    const int N = g.N;
    if (u <= N - 1) {
        const int b = u / g.H, r = u - b * g.H;
        Acc v = K.ain[(size_t)b * N + r] + A.tRedge[((size_t)b * g.T) * g.H + r];
        if (r + 1 < N) v += K.Rin[(size_t)b * N + r + 1];
        return v;
    }
    return K.Rin[(size_t)g.B * N + (u - N + 1)] + K.ain[(size_t)g.B * N + (u - N)];
}

// V(v) = sum over i'-j' >= v:  for v >= 0 it is L(N-1, N-1-v); below, L(N-1+v, N-1)
// misses exactly the columns right of N-1+v, i.e. C - X(N-1+v).
template <typename Acc>
__device__ __forceinline__ Acc marg_V(const Geom& g, const Agg<Acc>& A, const Carry<Acc>& K, int v) {
    const int N = g.N;
    if (v >= 0) {
        const int j = N - 1 - v;
        const int b = j / g.H, r = j - b * g.H;
        const int m = N - 2 - r;
        const Acc* ainb = K.ain + (size_t)b * N;
        Acc val = ainb[N - 1] - (m >= 0 ? ainb[m] : Acc(0));
        val += A.tLedge[((size_t)b * g.T + (g.T - 1)) * g.H + r];
        if (m >= 0) val += K.Lin[(size_t)b * N + m];
        return val;
    }
    const Acc* ainB = K.ain + (size_t)g.B * N;
    return K.Lin[(size_t)g.B * N + (N - 1 + v)] + (ainB[N - 1] - ainB[N - 1 + v]);
}

// Y(j) = alpha(N-1, j) = ain[b][N-1] + sum over all tiles of trow.
template <typename Acc>
__device__ __forceinline__ Acc marg_Y(const Geom& g, const Agg<Acc>& A, const Carry<Acc>& K, int j) {
    const int b = j / g.H, r = j - b * g.H;
    Acc y = K.ain[(size_t)b * g.N + (g.N - 1)];
    for (int c = 0; c < g.T; ++c) y += A.trow[((size_t)b * g.T + c) * g.H + r];
    return y;
}

template <typename Acc>
__global__ __launch_bounds__(256) void k_inim_marg(Geom g, Agg<Acc> A, Carry<Acc> K, double* marg) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    const int N = g.N, M = 2 * N - 1;
    if (o >= 2 * N + 2 * M + 1) return;
    Acc v;
    if (o < N) v = K.ain[(size_t)g.B * N + o];
    else if (o < 2 * N) v = marg_Y(g, A, K, o - N);
    else if (o < 2 * N + M) v = marg_U(g, A, K, o - 2 * N);
    else if (o < 2 * N + 2 * M) v = marg_V(g, A, K, (o - 2 * N - M) - (N - 1));
    else v = K.ain[(size_t)g.B * N + (N - 1)];
    marg[o] = to_f64(v);
}

// ------------------------------------------------------------------ pass 4
enum { kModePlanes = 0, kModeDeform = 1 };

template <int Q, typename Tin, int MODE>
__global__ __launch_bounds__(256) void k_inim_final(const Tin* __restrict__ img, Geom g,
                                                    Agg<typename AccOf<Tin>::type> A,
                                                    Carry<typename AccOf<Tin>::type> K, uint32_t mask,
                                                    Tin* __restrict__ planes, float2* __restrict__ field,
                                                    double d0, const int* status) {
    using Acc = typename AccOf<Tin>::type;
    extern __shared__ unsigned char smem_raw[];
    if (failed(status)) return;
    const int lane = lane_id();
    const int wave = (int)(threadIdx.x >> 6);
    const int tile = blockIdx.x * kWavesPerBlock + wave;
    if (tile >= g.B * g.T) return;
    const int N = g.N, H = g.H, W = g.W, T = g.T;
    const int b = tile / T, c = tile - (tile / T) * T;
    const int x0 = lane * Q;
    const bool act = lane <= g.lastLane;
    const int cW = c * W;
    const int col = cW + x0;
    const size_t NN = (size_t)N * (size_t)N;
    const Acc* ainb = K.ain + (size_t)b * N;
    const Acc* Linb = K.Lin + (size_t)b * N;
    const Acc* Rinb = K.Rin + (size_t)b * N;

    const bool needUV = (MODE == kModeDeform) || (mask & (INIM_BETA_T | INIM_GAMMA_T | INIM_DELTA_T));
    const bool needXY = (MODE == kModeDeform) || (mask & (INIM_BETA | INIM_GAMMA | INIM_DELTA | INIM_GAMMA_T));

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
            if (c > 0) {
                const int m = cW - 2 - r;
                lb = ainb[cW - 1] - (m >= 0 ? ainb[m] : Acc(0));
                lb += A.tLedge[eb + (size_t)(c - 1) * H + r];
                if (m >= 0) lb += Linb[m];
                ac = ainb[cW - 1];
                for (int cc = 0; cc < c; ++cc) ac += A.trow[eb + (size_t)cc * H + r];
            }
            if (c < T - 1) {
                const int m = cW + W + r;
                rb = ainb[m] - ainb[cW + W - 1];
                rb += A.tRedge[eb + (size_t)(c + 1) * H + r];
                if (m + 1 < N) rb += Rinb[m + 1];
            }
            if (needXY) yv = marg_Y(g, A, K, b * H + r);
        }
        LBv[k] = lb; RBv[k] = rb; ACv[k] = ac; YVv[k] = yv;
    }

    // U and V over the tile's anti-diagonals u0..u0+S-1 and diagonals v0..v0+S-1.
    const int S = W + H - 1;
    const int u0 = cW + b * H;
    const int v0 = cW - b * H - (H - 1);
    Acc* Uw = reinterpret_cast<Acc*>(smem_raw) + (size_t)wave * 2 * S;
    Acc* Vw = Uw + S;
    if (needUV) {
        for (int k = lane; k < S; k += 64) {
            Uw[k] = marg_U(g, A, K, u0 + k);
            Vw[k] = marg_V(g, A, K, v0 + k);
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

    // output slots of the requested planes
    int slot[8];
    {
        int s = 0;
#pragma unroll
        for (int p = 0; p < 8; ++p) { slot[p] = s; s += (mask >> p) & 1u; }
    }

    const Tin* src = img + (size_t)b * H * N + col;
    Tin buf[kPF][Q];
#pragma unroll
    for (int p = 0; p < kPF; ++p)
        if (p < H) load_tile_row<Tin, Q>(src + (size_t)p * N, act, buf[p]);

    for (int r0 = 0; r0 < H; r0 += kPF) {
#pragma unroll
        for (int p = 0; p < kPF; ++p) {
            const int r = r0 + p;
            if (r < H) {
                Tin v[Q];
#pragma unroll
                for (int e = 0; e < Q; ++e) v[e] = buf[p][e];
                if (r + kPF < H) load_tile_row<Tin, Q>(src + (size_t)(r + kPF) * N, act, buf[p]);
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
                if (needXY) Yr = bcast(pick_row(YVv, r), r & 63);

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
                    float2 o[Q];
#pragma unroll
                    for (int e = 0; e < Q; ++e) {
                        const int x = x0 + e;
                        const Acc U = Uw[x + r], V = Vw[x - r + H - 1];
                        const Compl<Acc> cm = complements<Acc>(al[e], at[e], Xv[e], Yr, U, V, Ctot, cW + x, j, N);
                        Planes8 P;
                        P.a = to_f64(al[e]); P.b = to_f64(cm.b); P.g = to_f64(cm.g); P.d = to_f64(cm.d);
                        P.at = to_f64(at[e]); P.bt = to_f64(cm.bt); P.gt = to_f64(cm.gt); P.dt = to_f64(cm.dt);
                        o[e] = deform_texel(P, to_f64(Ctot), cW + x, j, N, d0);
                    }
                    store_field_nt<Q>(field + (size_t)j * N + col, o);
                }
            }
        }
    }
}

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
    field[k] = deform_texel(P, C, i, j, N, d0);
}

// ------------------------------------------------------------------ launchers
template <typename Tin>
static size_t final_smem(const Geom& g, bool needUV) {
    using Acc = typename AccOf<Tin>::type;
    return needUV ? (size_t)kWavesPerBlock * 2 * (g.W + g.H - 1) * sizeof(Acc) : 0;
}

template <typename Tin, int Q>
static hipError_t launch_carries_q(const Tin* img, const Geom& g, void* scratch, const int* status, hipStream_t st) {
    using Acc = typename AccOf<Tin>::type;
    Agg<Acc> A;
    Carry<Acc> K;
    carve<Acc>(g, (char*)scratch, A, K);
    const int tiles = g.B * g.T;
    const dim3 grd((tiles + kWavesPerBlock - 1) / kWavesPerBlock);
    hipLaunchKernelGGL((k_inim_aggregate<Q, Tin>), grd, dim3(64 * kWavesPerBlock), 0, st, img, g, A, status);
    hipLaunchKernelGGL((k_inim_chain_col<Acc>), dim3((g.N + 255) / 256), dim3(256), 0, st, g, A, K, status);
    hipLaunchKernelGGL((k_inim_chain_diag<Acc>), dim3((2 * g.N + 1 + 255) / 256), dim3(256), 0, st, g, A, K, status);
    return hipGetLastError();
}

template <typename Tin, int Q>
static hipError_t launch_final_q(const Tin* img, const Geom& g, void* scratch, uint32_t mask, Tin* planes,
                                 float2* field, double d0, double* marg, const int* status, hipStream_t st) {
    using Acc = typename AccOf<Tin>::type;
    Agg<Acc> A;
    Carry<Acc> K;
    carve<Acc>(g, (char*)scratch, A, K);
    const int tiles = g.B * g.T;
    const dim3 blk(64 * kWavesPerBlock);
    const dim3 grd((tiles + kWavesPerBlock - 1) / kWavesPerBlock);
    if (field != nullptr) {
        hipLaunchKernelGGL((k_inim_final<Q, Tin, kModeDeform>), grd, blk, final_smem<Tin>(g, true), st, img, g, A, K,
                           0u, (Tin*)nullptr, field, d0, status);
    } else if (mask != 0) {
        const bool needUV = (mask & (INIM_BETA_T | INIM_GAMMA_T | INIM_DELTA_T)) != 0;
        hipLaunchKernelGGL((k_inim_final<Q, Tin, kModePlanes>), grd, blk, final_smem<Tin>(g, needUV), st, img, g, A, K,
                           mask, planes, (float2*)nullptr, 0.0, status);
    }
    if (marg != nullptr) {
        const int M = 6 * g.N - 1;
        hipLaunchKernelGGL((k_inim_marg<Acc>), dim3((M + 255) / 256), dim3(256), 0, st, g, A, K, marg);
    }
    return hipGetLastError();
}

template <typename Tin>
hipError_t launch_inim_carries(const Tin* img, const Geom& g, void* scratch, const int* status, hipStream_t st) {
    switch (g.Q) {
        case 1: return launch_carries_q<Tin, 1>(img, g, scratch, status, st);
        case 2: return launch_carries_q<Tin, 2>(img, g, scratch, status, st);
        case 4: return launch_carries_q<Tin, 4>(img, g, scratch, status, st);
        case 8: return launch_carries_q<Tin, 8>(img, g, scratch, status, st);
    }
    return hipErrorInvalidValue;
}

template <typename Tin>
hipError_t launch_inim_final(const Tin* img, const Geom& g, void* scratch, uint32_t mask, Tin* planes, float2* field,
                             double d0, double* marg, const int* status, hipStream_t st) {
    switch (g.Q) {
        case 1: return launch_final_q<Tin, 1>(img, g, scratch, mask, planes, field, d0, marg, status, st);
        case 2: return launch_final_q<Tin, 2>(img, g, scratch, mask, planes, field, d0, marg, status, st);
        case 4: return launch_final_q<Tin, 4>(img, g, scratch, mask, planes, field, d0, marg, status, st);
        case 8: return launch_final_q<Tin, 8>(img, g, scratch, mask, planes, field, d0, marg, status, st);
    }
    return hipErrorInvalidValue;
}

template hipError_t launch_inim_carries<uint32_t>(const uint32_t*, const Geom&, void*, const int*, hipStream_t);
template hipError_t launch_inim_carries<float>(const float*, const Geom&, void*, const int*, hipStream_t);
template hipError_t launch_inim_final<uint32_t>(const uint32_t*, const Geom&, void*, uint32_t, uint32_t*, float2*,
                                                double, double*, const int*, hipStream_t);
template hipError_t launch_inim_final<float>(const float*, const Geom&, void*, uint32_t, float*, float2*, double,
                                             double*, const int*, hipStream_t);

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
