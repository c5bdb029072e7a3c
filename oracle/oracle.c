/*
 * oracle.c -- plain, slow, FP64 CPU oracle for the scatterplot regularisation of
 * Rave, Molchanov and Linsen, "De-cluttering Scatterplots with Integral Images"
 * (IEEE TVCG; arXiv 2408.06513).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header,
 * table or constant with the HIP path and is written from the paper's
 * definitions, step by step, in the order the paper gives them:
 *
 *   counts   Sec. 4.1 (density field): every sample adds one to a single pixel.
 *   blur     Sec. 4.1, eq. (dr): convolution with a discrete Gaussian kernel.
 *   planes   Sec. 3.1: the four axis-aligned and the four 45-degree tilted
 *            integral images, each summed directly from its own inequalities.
 *   map      Sec. 3.2, eq. (map): the Molchanov-Linsen mapping t(x,y;d).
 *   deform   Sec. 4.1 eq. (d0) and Sec. 4.2 eq. (map_res): d = d_r + d0 and
 *            T = p + t(p;d) - t(p;d0), the defect t(p;d0) being the mapping of a
 *            constant raster.
 *   advect   Sec. 4.2: bilinear interpolation of T from the four nearest texels.
 *   regularize  Sec. 4.3 (the algorithm): steps 1-3 repeated a fixed number of
 *            times; the defect is computed once before the loop.
 *
 * Readings where the paper is silent or ambiguous (all fixed in this file):
 *   texel position   pixel (i,j) stands for the point ((i+1/2)/N, (j+1/2)/N);
 *   splat            pixel index floor(x*N), with x = 1 mapped to N-1;
 *   kernel           taps |m| <= r, weights exp(-m^2/(2 sigma^2)) normalised to
 *                    sum 1, sigma = r/2 by default, r = 0 meaning no smoothing;
 *   blur border      half-sample symmetric extension (... c b a | a b c ...);
 *   inequalities     the printed ones of Sec. 3.1 (<= for alpha, strict for the
 *                    complementary regions), which make both partitions hold;
 *   anchors          the printed tie rules (y >= x, x + y >= 1);
 *   defect, d0 = 0   t(.;c) does not depend on the constant c > 0, so with
 *                    d0 = 0 the defect is taken from the constant-1 raster;
 *   interpolation    cell index clamped to [0, N-2], fraction not clamped (the
 *                    border cells extrapolate linearly), result clamped to [0,1];
 *   inputs           N a power of two in [2, 16384]; every coordinate finite and
 *                    inside [0,1] (else status 2, positions untouched); n = 0 is a
 *                    no-op.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared oracle.c -o liboracle.so -lm
 * All arithmetic is IEEE double, round to nearest, no contraction.
 *
 * Threads (OpenMP, optional): only loops whose iterations are independent run
 * in parallel -- the rows of each blur pass, the eight planes (each swept by
 * one thread, as written), the texels of the map, the samples of the advection
 * and row bands of the splat (each thread counts the samples of its own rows).
 * Every value is computed by the same operations in the same order whatever
 * the thread count, so results are bit-identical for any thread count.
 * oracle_set_threads(k) picks k threads (k <= 0: one); without -fopenmp the
 * file builds as a single-threaded program.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int oracle_threads = 1;

/* Number of OpenMP threads of the parallel loops (1 without OpenMP). */
int oracle_set_threads(int k) {
#ifdef _OPENMP
    oracle_threads = k > 0 ? k : 1;
#else
    (void)k;
    oracle_threads = 1;
#endif
    return oracle_threads;
}

#define ORACLE_OK 0
#define ORACLE_EINVAL 1
#define ORACLE_EDOMAIN 2
#define ORACLE_ENOMEM 6

/* plane bits, in the order alpha beta gamma delta alpha_t beta_t gamma_t delta_t */
#define P_ALPHA 0
#define P_BETA 1
#define P_GAMMA 2
#define P_DELTA 3
#define P_ALPHA_T 4
#define P_BETA_T 5
#define P_GAMMA_T 6
#define P_DELTA_T 7

static int valid_res(int N) {
    if (N < 2 || N > 16384) return 0;
    return (N & (N - 1)) == 0;
}

/* ------------------------------------------------------------------------ */
/* Sec. 4.1: single-pixel splat into an accumulation raster.                */
/* ------------------------------------------------------------------------ */
static int pixel_of(double x, int N) {
    int k = (int)floor(x * (double)N);
    if (k > N - 1) k = N - 1; /* x == 1 belongs to the last pixel */
    return k;
}

int oracle_check_points(const double* xy, int64_t n) {
    for (int64_t p = 0; p < n; ++p) {
        double x = xy[2 * p], y = xy[2 * p + 1];
        if (!(x >= 0.0 && x <= 1.0 && y >= 0.0 && y <= 1.0)) return ORACLE_EDOMAIN;
    }
    return ORACLE_OK;
}

int oracle_counts(const double* xy, int64_t n, int N, double* counts) {
    if (!valid_res(N) || n < 0) return ORACLE_EINVAL;
    if (oracle_check_points(xy, n)) return ORACLE_EDOMAIN;
    memset(counts, 0, sizeof(double) * (size_t)N * (size_t)N);
    /* thread t counts the samples whose row lies in its band [j0, j1): every
     * texel is written by one thread, and counts are exact integers */
#pragma omp parallel num_threads(oracle_threads)
    {
        int nt = 1, t = 0;
#ifdef _OPENMP
        nt = omp_get_num_threads();
        t = omp_get_thread_num();
#endif
        int j0 = (int)((int64_t)N * t / nt), j1 = (int)((int64_t)N * (t + 1) / nt);
        for (int64_t p = 0; p < n; ++p) {
            int j = pixel_of(xy[2 * p + 1], N);
            if (j < j0 || j >= j1) continue;
            int i = pixel_of(xy[2 * p], N);
            counts[(size_t)j * N + i] += 1.0;
        }
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* Sec. 4.1 eq. (dr): separable Gaussian smoothing of the splat raster.      */
/* ------------------------------------------------------------------------ */
/* Half-sample symmetric extension: the raster continues as its mirror image,
 * i.e. index -1-t reads t and N+t reads N-1-t (period 2N). */
static int mirror(int k, int N) {
    int m = k % (2 * N);
    if (m < 0) m += 2 * N;
    if (m >= N) m = 2 * N - 1 - m;
    return m;
}

int oracle_blur(const double* c, int N, int r, double sigma, double* out) {
    if (!valid_res(N) || r < 0) return ORACLE_EINVAL;
    size_t NN = (size_t)N * (size_t)N;
    if (r == 0) {
        memcpy(out, c, sizeof(double) * NN);
        return ORACLE_OK;
    }
    if (!(sigma > 0.0)) sigma = 0.5 * (double)r;
    double* g = (double*)malloc(sizeof(double) * (size_t)(2 * r + 1));
    double* tmp = (double*)malloc(sizeof(double) * NN);
    if (!g || !tmp) { free(g); free(tmp); return ORACLE_ENOMEM; }
    double sum = 0.0;
    for (int m = -r; m <= r; ++m) {
        g[m + r] = exp(-(double)(m * m) / (2.0 * sigma * sigma));
        sum += g[m + r];
    }
    for (int m = 0; m <= 2 * r; ++m) g[m] /= sum;
    /* along x (within each row) */
#pragma omp parallel for num_threads(oracle_threads) schedule(static)
    for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i) {
            double a = 0.0;
            for (int m = -r; m <= r; ++m) a += g[m + r] * c[(size_t)j * N + mirror(i + m, N)];
            tmp[(size_t)j * N + i] = a;
        }
    /* along y (within each column) */
#pragma omp parallel for num_threads(oracle_threads) schedule(static)
    for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i) {
            double a = 0.0;
            for (int m = -r; m <= r; ++m) a += g[m + r] * tmp[(size_t)mirror(j + m, N) * N + i];
            out[(size_t)j * N + i] = a;
        }
    free(g);
    free(tmp);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* Sec. 3.1: integral images, each from its own inequalities.                */
/* ------------------------------------------------------------------------ */
/*
 * Axis-aligned planes: pixel (i,j) collects d(i',j') over
 *   alpha: i' <= i, j' <= j      beta:  i' <= i, j' >  j
 *   gamma: i' >  i, j' >  j      delta: i' >  i, j' <= j
 * The raster is swept row by row in the order the j'-condition needs
 * (downwards for "<=", upwards for ">"); acc[i] holds, per column, the sum of
 * the rows already admitted; the i'-condition is then a running sum across the
 * row taken from the left ("<=") or from the right (">").
 */
static void axis_plane(const double* d, int N, int rows_below, int cols_right, double* out) {
    double* acc = (double*)calloc((size_t)N, sizeof(double));
    for (int t = 0; t < N; ++t) {
        int j = rows_below ? (N - 1 - t) : t;
        if (!rows_below) /* j' <= j: admit row j before evaluating it */
            for (int i = 0; i < N; ++i) acc[i] += d[(size_t)j * N + i];
        if (!cols_right) {
            double run = 0.0; /* i' <= i */
            for (int i = 0; i < N; ++i) { run += acc[i]; out[(size_t)j * N + i] = run; }
        } else {
            double run = 0.0; /* i' > i */
            for (int i = N - 1; i >= 0; --i) { out[(size_t)j * N + i] = run; run += acc[i]; }
        }
        if (rows_below) /* j' > j: admit row j only after evaluating it */
            for (int i = 0; i < N; ++i) acc[i] += d[(size_t)j * N + i];
    }
    free(acc);
}

/*
 * Tilted planes, with u = i+j and v = i-j: pixel (i,j) collects d(i',j') over
 *   alpha_t: u' <= u, v' >= v     beta_t:  u' <= u, v' <  v
 *   gamma_t: u' >  u, v' <  v     delta_t: u' >  u, v' >= v
 * The same sweep on the 45-degree rotated lattice: anti-diagonals u are
 * admitted in the order the u-condition needs, acc[v] holds per diagonal v the
 * admitted mass, and the v-condition is a running sum over v.  Index v is stored
 * shifted by N-1 so that it runs over 0..2N-2.
 */
static void tilted_plane(const double* d, int N, int u_after, int v_below, double* out) {
    int M = 2 * N - 1;
    double* acc = (double*)calloc((size_t)M, sizeof(double));
    double* run = (double*)malloc(sizeof(double) * (size_t)M);
    for (int t = 0; t < M; ++t) {
        int u = u_after ? (M - 1 - t) : t;
        int i_lo = u - (N - 1) > 0 ? u - (N - 1) : 0;
        int i_hi = u < N - 1 ? u : N - 1;
        if (!u_after)
            for (int i = i_lo; i <= i_hi; ++i) acc[(i - (u - i)) + N - 1] += d[(size_t)(u - i) * N + i];
        if (!v_below) {
            double s = 0.0; /* v' >= v */
            for (int k = M - 1; k >= 0; --k) { s += acc[k]; run[k] = s; }
        } else {
            double s = 0.0; /* v' < v */
            for (int k = 0; k < M; ++k) { run[k] = s; s += acc[k]; }
        }
        for (int i = i_lo; i <= i_hi; ++i) {
            int j = u - i;
            out[(size_t)j * N + i] = run[(i - j) + N - 1];
        }
        if (u_after)
            for (int i = i_lo; i <= i_hi; ++i) acc[(i - (u - i)) + N - 1] += d[(size_t)(u - i) * N + i];
    }
    free(acc);
    free(run);
}

static void one_plane(const double* d, int N, int which, double* out) {
    switch (which) {
        case P_ALPHA: axis_plane(d, N, 0, 0, out); break;
        case P_BETA: axis_plane(d, N, 1, 0, out); break;
        case P_GAMMA: axis_plane(d, N, 1, 1, out); break;
        case P_DELTA: axis_plane(d, N, 0, 1, out); break;
        case P_ALPHA_T: tilted_plane(d, N, 0, 0, out); break;
        case P_BETA_T: tilted_plane(d, N, 0, 1, out); break;
        case P_GAMMA_T: tilted_plane(d, N, 1, 1, out); break;
        case P_DELTA_T: tilted_plane(d, N, 1, 0, out); break;
    }
}

/*
 * Marginal sums, each straight from its definition:
 *   X(i) = sum over i' <= i (all rows)      Y(j) = sum over j' <= j (all columns)
 *   U(u) = sum over i'+j' <= u               V(v) = sum over i'-j' >= v
 *   C    = sum of all pixels (Sec. 3.1).
 * Layout: X[N] | Y[N] | U[2N-1] | V[2N-1] (V[k] is v = k-(N-1)) | C.
 */
static void marginals(const double* d, int N, double* marg) {
    int M = 2 * N - 1;
    double *X = marg, *Y = marg + N, *U = marg + 2 * N, *V = marg + 2 * N + M, *C = marg + 2 * N + 2 * M;
    double* col = (double*)calloc((size_t)N, sizeof(double));
    double* row = (double*)calloc((size_t)N, sizeof(double));
    double* adiag = (double*)calloc((size_t)M, sizeof(double));
    double* diag = (double*)calloc((size_t)M, sizeof(double));
    double total = 0.0;
    for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i) {
            double a = d[(size_t)j * N + i];
            col[i] += a;
            row[j] += a;
            adiag[i + j] += a;
            diag[i - j + N - 1] += a;
            total += a;
        }
    double s = 0.0;
    for (int i = 0; i < N; ++i) { s += col[i]; X[i] = s; }
    s = 0.0;
    for (int j = 0; j < N; ++j) { s += row[j]; Y[j] = s; }
    s = 0.0;
    for (int u = 0; u < M; ++u) { s += adiag[u]; U[u] = s; }
    s = 0.0;
    for (int k = M - 1; k >= 0; --k) { s += diag[k]; V[k] = s; }
    *C = total;
    free(col); free(row); free(adiag); free(diag);
}

/* planes: popcount(mask) planes of N*N in bit order; marg may be NULL */
int oracle_planes(const double* d, int N, unsigned mask, double* planes, double* marg) {
    if (!valid_res(N) || (mask & ~0xFFu)) return ORACLE_EINVAL;
    size_t NN = (size_t)N * (size_t)N;
    double* out[8] = {0};
    double* o = planes;
    for (int b = 0; b < 8; ++b)
        if (mask & (1u << b)) { out[b] = o; o += NN; }
    /* the planes are independent: one thread sweeps each */
#pragma omp parallel for num_threads(oracle_threads) schedule(dynamic, 1)
    for (int b = 0; b < 8; ++b)
        if (out[b]) one_plane(d, N, b, out[b]);
    if (marg) marginals(d, N, marg);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* Sec. 3.2 eq. (map): t(x,y;d) from the eight planes.                       */
/* ------------------------------------------------------------------------ */
static void anchors(double x, double y, double q[4][2]) {
    if (y < x) { q[0][0] = 1.0; q[0][1] = 1.0 + y - x; q[2][0] = x - y; q[2][1] = 0.0; }
    else       { q[0][0] = 1.0 - y + x; q[0][1] = 1.0; q[2][0] = 0.0; q[2][1] = y - x; }
    if (x + y < 1.0) { q[1][0] = x + y; q[1][1] = 0.0; q[3][0] = 0.0; q[3][1] = x + y; }
    else             { q[1][0] = 1.0; q[1][1] = x + y - 1.0; q[3][0] = x + y - 1.0; q[3][1] = 1.0; }
}

static double texel_pos(int k, int N) { return ((double)k + 0.5) / (double)N; }

/* t: N*N*2 (x,y interleaved); planes8: the 8 planes of d in bit order; C = sum d */
static void molchanov_linsen_map(const double* P, int N, double C, double* t) {
    size_t NN = (size_t)N * (size_t)N;
#pragma omp parallel for num_threads(oracle_threads) schedule(static)
    for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i) {
            size_t k = (size_t)j * N + i;
            double x = texel_pos(i, N), y = texel_pos(j, N);
            double q[4][2];
            anchors(x, y, q);
            double al = P[0 * NN + k], be = P[1 * NN + k], ga = P[2 * NN + k], de = P[3 * NN + k];
            double at = P[4 * NN + k], bt = P[5 * NN + k], gt = P[6 * NN + k], dt = P[7 * NN + k];
            double sx = al * q[0][0] + be * q[1][0] + ga * q[2][0] + de * q[3][0]
                      + at * x + bt * 1.0 + gt * x + dt * 0.0;
            double sy = al * q[0][1] + be * q[1][1] + ga * q[2][1] + de * q[3][1]
                      + at * 1.0 + bt * y + gt * 0.0 + dt * y;
            t[2 * k] = sx / (2.0 * C);
            t[2 * k + 1] = sy / (2.0 * C);
        }
}

/* t(p;d) for an arbitrary raster d (the eight planes are built here) */
int oracle_map(const double* d, int N, double* t) {
    if (!valid_res(N)) return ORACLE_EINVAL;
    size_t NN = (size_t)N * (size_t)N;
    double* P = (double*)malloc(sizeof(double) * 8 * NN);
    if (!P) return ORACLE_ENOMEM;
    double C = 0.0;
    for (size_t k = 0; k < NN; ++k) C += d[k];
    oracle_planes(d, N, 0xFFu, P, NULL);
    molchanov_linsen_map(P, N, C, t);
    free(P);
    return ORACLE_OK;
}

/* Sec. 4.2: the defect t(p;d0), the map of a constant raster (computed once). */
int oracle_defect(int N, double d0, double* t) {
    if (!valid_res(N)) return ORACLE_EINVAL;
    size_t NN = (size_t)N * (size_t)N;
    double* c = (double*)malloc(sizeof(double) * NN);
    if (!c) return ORACLE_ENOMEM;
    double value = d0 > 0.0 ? d0 : 1.0;
    for (size_t k = 0; k < NN; ++k) c[k] = value;
    int st = oracle_map(c, N, t);
    free(c);
    return st;
}

/* eq. (d0) + eq. (map_res) given a precomputed defect */
static int deform_with_defect(const double* dr, int N, double d0, const double* defect, double* field) {
    size_t NN = (size_t)N * (size_t)N;
    double* d = (double*)malloc(sizeof(double) * NN);
    double* t = (double*)malloc(sizeof(double) * 2 * NN);
    if (!d || !t) { free(d); free(t); return ORACLE_ENOMEM; }
    for (size_t k = 0; k < NN; ++k) d[k] = dr[k] + d0; /* eq. (d0) */
    int st = oracle_map(d, N, t);
    if (st == ORACLE_OK)
#pragma omp parallel for num_threads(oracle_threads) schedule(static)
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                size_t k = (size_t)j * N + i;
                field[2 * k] = texel_pos(i, N) + t[2 * k] - defect[2 * k];
                field[2 * k + 1] = texel_pos(j, N) + t[2 * k + 1] - defect[2 * k + 1];
            }
    free(d);
    free(t);
    return st;
}

int oracle_deform(const double* dr, int N, double d0, double* field) {
    if (!valid_res(N) || d0 < 0.0) return ORACLE_EINVAL;
    size_t NN = (size_t)N * (size_t)N;
    double* defect = (double*)malloc(sizeof(double) * 2 * NN);
    if (!defect) return ORACLE_ENOMEM;
    int st = oracle_defect(N, d0, defect);
    if (st == ORACLE_OK) st = deform_with_defect(dr, N, d0, defect, field);
    free(defect);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Sec. 4.2: bilinear interpolation of the deformation at every sample.      */
/* ------------------------------------------------------------------------ */
static void cell(double x, int N, int* k0, double* f) {
    double s = x * (double)N - 0.5; /* continuous texel coordinate */
    double fl = floor(s);
    int k = (int)fl;
    if (k < 0) k = 0;
    if (k > N - 2) k = N - 2;
    *k0 = k;
    *f = s - (double)k; /* not clamped: the border cells extrapolate */
}

static double clamp01(double v) { return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v); }

int oracle_advect(const double* field, int N, double* xy, int64_t n) {
    if (!valid_res(N) || n < 0) return ORACLE_EINVAL;
    if (oracle_check_points(xy, n)) return ORACLE_EDOMAIN;
#pragma omp parallel for num_threads(oracle_threads) schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        int i0, j0;
        double fx, fy;
        cell(xy[2 * p], N, &i0, &fx);
        cell(xy[2 * p + 1], N, &j0, &fy);
        const double* a = field + 2 * ((size_t)j0 * N + i0);
        const double* b = field + 2 * ((size_t)j0 * N + i0 + 1);
        const double* c = field + 2 * ((size_t)(j0 + 1) * N + i0);
        const double* e = field + 2 * ((size_t)(j0 + 1) * N + i0 + 1);
        for (int comp = 0; comp < 2; ++comp) {
            double v = (1.0 - fx) * (1.0 - fy) * a[comp] + fx * (1.0 - fy) * b[comp]
                     + (1.0 - fx) * fy * c[comp] + fx * fy * e[comp];
            xy[2 * p + comp] = clamp01(v);
        }
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* Sec. 4.3: the iteration.                                                   */
/* ------------------------------------------------------------------------ */
/* d0 < 0 selects the paper's choice n / N^2; sigma <= 0 selects r/2.
 * The m probe points (may be 0) are moved by the same deformation as the
 * samples in every iteration but take no part in the density: they sample
 * the composite map of all iterations (the deformed grid of Sec. 5). */
static int regularize(double* xy, int64_t n, double* probe, int64_t m, int N, int iters, int r, double sigma,
                      double d0) {
    if (!valid_res(N) || n < 0 || m < 0 || iters < 0 || r < 0) return ORACLE_EINVAL;
    if (oracle_check_points(xy, n)) return ORACLE_EDOMAIN;
    if (n == 0 || iters == 0) return ORACLE_OK; /* no density: nothing moves */
    if (oracle_check_points(probe, m)) return ORACLE_EDOMAIN;
    size_t NN = (size_t)N * (size_t)N;
    if (d0 < 0.0) d0 = (double)n / (double)NN;
    double* cnt = (double*)malloc(sizeof(double) * NN);
    double* dr = (double*)malloc(sizeof(double) * NN);
    double* field = (double*)malloc(sizeof(double) * 2 * NN);
    double* defect = (double*)malloc(sizeof(double) * 2 * NN);
    int st = ORACLE_ENOMEM;
    if (cnt && dr && field && defect) {
        st = oracle_defect(N, d0, defect); /* once, reused by every iteration */
        for (int it = 0; it < iters && st == ORACLE_OK; ++it) {
            st = oracle_counts(xy, n, N, cnt);                           /* step 1 */
            if (st == ORACLE_OK) st = oracle_blur(cnt, N, r, sigma, dr); /* step 1 */
            if (st == ORACLE_OK) st = deform_with_defect(dr, N, d0, defect, field); /* steps 2-3 */
            if (st == ORACLE_OK) st = oracle_advect(field, N, xy, n);   /* step 3 */
            if (st == ORACLE_OK && m > 0) st = oracle_advect(field, N, probe, m);
        }
    }
    free(cnt); free(dr); free(field); free(defect);
    return st;
}

int oracle_regularize(double* xy, int64_t n, int N, int iters, int r, double sigma, double d0) {
    return regularize(xy, n, NULL, 0, N, iters, r, sigma, d0);
}

int oracle_regularize_probes(double* xy, int64_t n, double* probe, int64_t m, int N, int iters, int r,
                             double sigma, double d0) {
    if (m > 0 && probe == NULL) return ORACLE_EINVAL;
    return regularize(xy, n, probe, m, N, iters, r, sigma, d0);
}
