/*
 * CPU oracle for the exact k-NN scan over multi-dimensional time series
 * (Bachmann & Freytag, "An Analytical Approach to Improving Time Warping on
 * Multidimensional Time Series", arXiv 1811.11076).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library; both sides receive the same
 * seeded inputs and nothing else.
 *
 * Plain, slow, obviously-correct code.  Conventions:
 *   - A series is float32 AoS [len][d]; indices are 0-based.
 *   - S is the query (rows i = 0..m-1), T the candidate (columns j = 0..n-1).
 *   - "w < 0" means no Sakoe-Chiba band.
 *   - DTW is the sum of squared Euclidean point distances along the best
 *     warping path, with no final square root (Sec. 2.1, DTW recursion).
 *   - DK is evaluated in the squared domain (max of squared point distances);
 *     sqrt is monotone so the optimal path is the same (Sec. 2.1, DK
 *     recursion); callers take sqrtf of the squared value.
 *
 * Readings of passages where the paper is silent or garbled (each is listed
 * in the design notes as well):
 *   R-cost  point cost in fp32: e_k = fl(s_k - t_k); acc = e_0*e_0, then
 *           acc = fmaf(e_k, e_k, acc) for k = 1..d-1 (no other contraction).
 *   R-prefix the DP runs bottom-left to top-right (Sec. 2.1, matrix text) with
 *           D(-1,-1) = 0 and every other out-of-matrix cell = +inf.
 *   R-band  band for lengths m, n: cell (i,j) allowed iff
 *           |i(n-1) - j(m-1)| (L-1) <= w (m-1)(n-1), L = max(m,n); every cell
 *           is allowed when m == 1 or n == 1.  For m == n this is |i-j| <= w
 *           (Sec. 2.2).  Windows are clipped to the series (Sec. 2.3 text runs
 *           past the ends).
 *   R-gdk   Alg. 1 loops until (m-1, n-1) is reached (the printed loop test
 *           would stop on the last row OR column and never reach the corner);
 *           ties go to the first of (i+1,j), (i+1,j+1), (i,j+1); moves off the
 *           matrix or out of band count as +inf; no move left -> +inf.
 *   R-sdk0  Alg. 3's first cell gets a virtual predecessor of 0 (with all of
 *           D and E at +inf the printed recurrence never starts).
 *   R-sdkend Alg. 3 returns +inf (not eps) once the active set is empty, and
 *           returns the last computed column's top cell (the printed return
 *           reads D after it was reset).
 *   R-lb    LB terms are summed sequentially, in series order, in fp32.
 *   R-knn   k-NN order is (key, id) ascending; the k-NN threshold for DK is
 *           the k-th smallest greedy bound (Sec. 4.3 states the 1-NN case).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads of the OpenMP loops over queries (for timing the oracle on one
 * core or on all); returns the previous setting. */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    int old = omp_get_max_threads();
    if (n > 0)
        omp_set_num_threads(n);
    return old;
#else
    (void)n;
    return 1;
#endif
}

#define ORC_INF INFINITY
/* longest series the envelope cache of orc_knn_verify keys by length */
#define ORC_MAX_LEN 4096

#if defined(__x86_64__)
#define ORC_CLONES __attribute__((target_clones("fma", "default")))
#else
#define ORC_CLONES
#endif

/* ---------------------------------------------------------------- point cost
 * Sec. 3: d(s,t) = ||s - t||_2; DTW uses d^2 (Sec. 2.1) and so does the
 * squared-domain DK.  Reading R-cost fixes the fp32 operation order. */
ORC_CLONES
float orc_cost_f32(const float *s, const float *t, int d)
{
    float e = s[0] - t[0];
    float acc = e * e;
    for (int k = 1; k < d; ++k) {
        e = s[k] - t[k];
        acc = fmaf(e, e, acc);
    }
    return acc;
}

ORC_CLONES
double orc_cost_f64(const float *s, const float *t, int d)
{
    double acc = 0.0;
    for (int k = 0; k < d; ++k) {
        double e = (double)s[k] - (double)t[k];
        acc = fma(e, e, acc);
    }
    return acc;
}

/* ---------------------------------------------------------------- band (R-band) */
int orc_band_ok(int64_t i, int64_t j, int64_t m, int64_t n, int64_t w)
{
    if (w < 0 || m == 1 || n == 1)
        return 1;
    int64_t L = m > n ? m : n;
    int64_t a = i * (n - 1) - j * (m - 1);
    if (a < 0)
        a = -a;
    return a * (L - 1) <= w * (m - 1) * (n - 1);
}

/* w from a fractional band, identical rule on every side: floor(frac * L). */
int64_t orc_band_w_frac(float frac, int64_t m, int64_t n)
{
    int64_t L = m > n ? m : n;
    return (int64_t)floor((double)frac * (double)L);
}

static float fmin3f(float a, float b, float c)
{
    float x = a < b ? a : b;
    return x < c ? x : c;
}

static double fmin3d(double a, double b, double c)
{
    double x = a < b ? a : b;
    return x < c ? x : c;
}

/* ---------------------------------------------------------------- DTW
 * Sec. 2.1: DTW recursion; evaluated as the quadratic DP of the "distance
 * matrix / warping matrix" paragraph: each cell = its cost plus the smallest
 * of the left, lower and lower-left neighbours.  fp32 "mirror" version. */
ORC_CLONES
float orc_dtw_f32(const float *S, int64_t m, const float *T, int64_t n, int d, int64_t w)
{
    if (m <= 0 || n <= 0)
        return ORC_INF;
    float *prev = malloc(sizeof(float) * n), *cur = malloc(sizeof(float) * n);
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            if (!orc_band_ok(i, j, m, n, w)) {
                cur[j] = ORC_INF;
                continue;
            }
            float best;
            if (i == 0 && j == 0)
                best = 0.0f;
            else
                best = fmin3f((i > 0 && j > 0) ? prev[j - 1] : ORC_INF,
                              (i > 0) ? prev[j] : ORC_INF,
                              (j > 0) ? cur[j - 1] : ORC_INF);
            float c = orc_cost_f32(S + i * d, T + j * d, d);
            cur[j] = c + best;
        }
        float *tmp = prev; prev = cur; cur = tmp;
    }
    float r = prev[n - 1];
    free(prev); free(cur);
    return r;
}

/* The same DP in fp64 from the fp32 inputs ("reference"). */
ORC_CLONES
double orc_dtw_f64(const float *S, int64_t m, const float *T, int64_t n, int d, int64_t w)
{
    if (m <= 0 || n <= 0)
        return ORC_INF;
    double *prev = malloc(sizeof(double) * n), *cur = malloc(sizeof(double) * n);
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            if (!orc_band_ok(i, j, m, n, w)) {
                cur[j] = ORC_INF;
                continue;
            }
            double best;
            if (i == 0 && j == 0)
                best = 0.0;
            else
                best = fmin3d((i > 0 && j > 0) ? prev[j - 1] : ORC_INF,
                              (i > 0) ? prev[j] : ORC_INF,
                              (j > 0) ? cur[j - 1] : ORC_INF);
            cur[j] = orc_cost_f64(S + i * d, T + j * d, d) + best;
        }
        double *tmp = prev; prev = cur; cur = tmp;
    }
    double r = prev[n - 1];
    free(prev); free(cur);
    return r;
}

/* ---------------------------------------------------------------- DK
 * Sec. 2.1: DK recursion (maximum along the path instead of the sum), as the
 * same quadratic DP; squared domain, so the result is exact in fp32 (max and
 * min only select among fp32 cell costs). */
ORC_CLONES
float orc_dk_sq_f32(const float *S, int64_t m, const float *T, int64_t n, int d, int64_t w)
{
    if (m <= 0 || n <= 0)
        return ORC_INF;
    float *prev = malloc(sizeof(float) * n), *cur = malloc(sizeof(float) * n);
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            if (!orc_band_ok(i, j, m, n, w)) {
                cur[j] = ORC_INF;
                continue;
            }
            float best;
            if (i == 0 && j == 0)
                best = 0.0f;
            else
                best = fmin3f((i > 0 && j > 0) ? prev[j - 1] : ORC_INF,
                              (i > 0) ? prev[j] : ORC_INF,
                              (j > 0) ? cur[j - 1] : ORC_INF);
            float c = orc_cost_f32(S + i * d, T + j * d, d);
            cur[j] = c > best ? c : best;
        }
        float *tmp = prev; prev = cur; cur = tmp;
    }
    float r = prev[n - 1];
    free(prev); free(cur);
    return r;
}

/* DK on unsquared cell values (sqrtf per cell); used to check that the
 * squared-domain evaluation followed by one sqrtf gives the same number. */
float orc_dk_unsq_f32(const float *S, int64_t m, const float *T, int64_t n, int d, int64_t w)
{
    if (m <= 0 || n <= 0)
        return ORC_INF;
    float *prev = malloc(sizeof(float) * n), *cur = malloc(sizeof(float) * n);
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            if (!orc_band_ok(i, j, m, n, w)) {
                cur[j] = ORC_INF;
                continue;
            }
            float best;
            if (i == 0 && j == 0)
                best = 0.0f;
            else
                best = fmin3f((i > 0 && j > 0) ? prev[j - 1] : ORC_INF,
                              (i > 0) ? prev[j] : ORC_INF,
                              (j > 0) ? cur[j - 1] : ORC_INF);
            float c = sqrtf(orc_cost_f32(S + i * d, T + j * d, d));
            cur[j] = c > best ? c : best;
        }
        float *tmp = prev; prev = cur; cur = tmp;
    }
    float r = prev[n - 1];
    free(prev); free(cur);
    return r;
}

/* ---------------------------------------------------------------- path enumeration
 * Brute force over every monotone warping path (steps (1,0), (0,1), (1,1))
 * from (0,0) to (m-1,n-1) inside the band: the definitions of Sec. 2.1
 * applied to each path separately.  Outputs
 *   out[0] = min over paths of the fp64 sum of costs,
 *   out[1] = min over paths of the fp32 sum accumulated in path order
 *            (acc = fl(cost + acc)), i.e. what the fp32 recurrence rounds,
 *   out[2] = min over paths of the max of fp32 costs (squared DK),
 *   out[3] = number of paths.
 * Exponential; meant for m, n <= 9. */
struct orc_enum {
    const float *S, *T;
    int64_t m, n, w;
    int d;
    double best_sum64;
    float best_sum32, best_max;
    double count;
};

static void orc_enum_rec(struct orc_enum *E, int64_t i, int64_t j, double s64, float s32, float mx)
{
    if (!orc_band_ok(i, j, E->m, E->n, E->w))
        return;
    float c = orc_cost_f32(E->S + i * E->d, E->T + j * E->d, E->d);
    double c64 = orc_cost_f64(E->S + i * E->d, E->T + j * E->d, E->d);
    s64 += c64;
    s32 = c + s32;
    mx = c > mx ? c : mx;
    if (i == E->m - 1 && j == E->n - 1) {
        if (s64 < E->best_sum64) E->best_sum64 = s64;
        if (s32 < E->best_sum32) E->best_sum32 = s32;
        if (mx < E->best_max) E->best_max = mx;
        E->count += 1.0;
        return;
    }
    if (i + 1 < E->m)
        orc_enum_rec(E, i + 1, j, s64, s32, mx);
    if (i + 1 < E->m && j + 1 < E->n)
        orc_enum_rec(E, i + 1, j + 1, s64, s32, mx);
    if (j + 1 < E->n)
        orc_enum_rec(E, i, j + 1, s64, s32, mx);
}

void orc_enumerate_paths(const float *S, int64_t m, const float *T, int64_t n, int d,
                         int64_t w, double *out)
{
    struct orc_enum E = {S, T, m, n, w, d, ORC_INF, ORC_INF, ORC_INF, 0.0};
    if (m > 0 && n > 0)
        orc_enum_rec(&E, 0, 0, 0.0, 0.0f, 0.0f);
    out[0] = E.best_sum64;
    out[1] = E.best_sum32;
    out[2] = E.best_max;
    out[3] = E.count;
}

/* ---------------------------------------------------------------- envelopes
 * Sec. 2.3 / Sec. 3: the box B_i of row i of S is the per-dimension
 * [min, max] of the points of T that the band lets row i align with.
 * Brute-force windowed min/max (the paper uses Lemire's streaming algorithm
 * for the same numbers).  lo, hi: [m][d].  An empty window gives lo = +inf,
 * hi = -inf. */
void orc_envelope(const float *T, int64_t n, int64_t m, int d, int64_t w, float *lo, float *hi)
{
    for (int64_t i = 0; i < m; ++i) {
        for (int k = 0; k < d; ++k) {
            lo[i * d + k] = ORC_INF;
            hi[i * d + k] = -ORC_INF;
        }
        for (int64_t j = 0; j < n; ++j) {
            if (!orc_band_ok(i, j, m, n, w))
                continue;
            for (int k = 0; k < d; ++k) {
                float v = T[j * d + k];
                if (v < lo[i * d + k]) lo[i * d + k] = v;
                if (v > hi[i * d + k]) hi[i * d + k] = v;
            }
        }
    }
}

/* Squared distance of point x to the box [lo, hi] (Sec. 3: the sum over the
 * dimensions of the squared 1-D interval distances), same fp32 order as the
 * point cost.  An empty box (lo > hi) gives +inf. */
ORC_CLONES
float orc_box_term_f32(const float *x, const float *lo, const float *hi, int d)
{
    float acc = 0.0f;
    for (int k = 0; k < d; ++k) {
        if (lo[k] > hi[k])
            return ORC_INF;
        float e = 0.0f;
        if (x[k] < lo[k]) e = lo[k] - x[k];
        else if (x[k] > hi[k]) e = x[k] - hi[k];
        acc = (k == 0) ? e * e : fmaf(e, e, acc);
    }
    return acc;
}

/* LB_Box(S, T), eq. (1): sum over the rows i of S of d(s_i, B_i)^2 with the
 * boxes built over T; fp32, summed in row order (R-lb). */
ORC_CLONES
float orc_lb_box_f32(const float *S, int64_t m, const float *T, int64_t n, int d, int64_t w)
{
    float *lo = malloc(sizeof(float) * m * d), *hi = malloc(sizeof(float) * m * d);
    orc_envelope(T, n, m, d, w, lo, hi);
    float acc = 0.0f;
    for (int64_t i = 0; i < m; ++i)
        acc = orc_box_term_f32(S + i * d, lo + i * d, hi + i * d, d) + acc;
    free(lo); free(hi);
    return acc;
}

/* LB_Box in fp64 (for the exact identities of eq. (1)). */
double orc_lb_box_f64(const float *S, int64_t m, const float *T, int64_t n, int d, int64_t w)
{
    float *lo = malloc(sizeof(float) * m * d), *hi = malloc(sizeof(float) * m * d);
    orc_envelope(T, n, m, d, w, lo, hi);
    double acc = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        for (int k = 0; k < d; ++k) {
            double x = S[i * d + k], l = lo[i * d + k], u = hi[i * d + k], e = 0.0;
            if (l > u) { acc = ORC_INF; continue; }
            if (x < l) e = l - x;
            else if (x > u) e = x - u;
            acc += e * e;
        }
    }
    free(lo); free(hi);
    return acc;
}

/* LB_Keogh of one dimension k (Sec. 2.3), fp64: sum over rows of the squared
 * distance of s_{i,k} to [l_{i,k}, u_{i,k}]. */
double orc_lb_keogh_f64(const float *S, int64_t m, const float *T, int64_t n, int d, int64_t w, int k)
{
    double acc = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double l = ORC_INF, u = -ORC_INF;
        for (int64_t j = 0; j < n; ++j) {
            if (!orc_band_ok(i, j, m, n, w))
                continue;
            double v = T[j * d + k];
            if (v < l) l = v;
            if (v > u) u = v;
        }
        if (l > u) return ORC_INF;
        double x = S[i * d + k], e = 0.0;
        if (x < l) e = l - x;
        else if (x > u) e = x - u;
        acc += e * e;
    }
    return acc;
}

/* LB_Sigma-min (Sec. 3): sum over rows of the smallest squared distance to
 * any point of T inside the row's window; fp64. */
double orc_lb_sigmamin_f64(const float *S, int64_t m, const float *T, int64_t n, int d, int64_t w)
{
    double acc = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double best = ORC_INF;
        for (int64_t j = 0; j < n; ++j) {
            if (!orc_band_ok(i, j, m, n, w))
                continue;
            double c = orc_cost_f64(S + i * d, T + j * d, d);
            if (c < best) best = c;
        }
        acc += best;
    }
    return acc;
}

/* ---------------------------------------------------------------- greedy DK (Alg. 1)
 * Sec. 4.1, Alg. 1 with reading R-gdk, squared domain.  Starts at (0,0),
 * repeatedly steps to the cheapest of the three successor cells, keeps the
 * running maximum g and returns it as soon as g > eps.  Without an early
 * return the value is the maximum along one warping path, hence an upper
 * bound on squared DK.  *steps (nullable) receives the number of moves. */
ORC_CLONES
float orc_gdk_sq_f32(const float *S, int64_t m, const float *T, int64_t n, int d, int64_t w,
                     float eps, int64_t *steps)
{
    int64_t i = 0, j = 0, st = 0;
    if (m <= 0 || n <= 0) {
        if (steps) *steps = 0;
        return ORC_INF;
    }
    float g = orc_cost_f32(S, T, d);
    if (g > eps) {
        if (steps) *steps = 0;
        return g;
    }
    while (!(i == m - 1 && j == n - 1)) {
        float c_dn = ORC_INF, c_dg = ORC_INF, c_rt = ORC_INF; /* (i+1,j) (i+1,j+1) (i,j+1) */
        if (i + 1 < m && orc_band_ok(i + 1, j, m, n, w))
            c_dn = orc_cost_f32(S + (i + 1) * d, T + j * d, d);
        if (i + 1 < m && j + 1 < n && orc_band_ok(i + 1, j + 1, m, n, w))
            c_dg = orc_cost_f32(S + (i + 1) * d, T + (j + 1) * d, d);
        if (j + 1 < n && orc_band_ok(i, j + 1, m, n, w))
            c_rt = orc_cost_f32(S + i * d, T + (j + 1) * d, d);
        float c;
        if (c_dn <= c_dg && c_dn <= c_rt) { c = c_dn; i += 1; }
        else if (c_dg <= c_rt) { c = c_dg; i += 1; j += 1; }
        else { c = c_rt; j += 1; }
        ++st;
        if (c == ORC_INF) { g = ORC_INF; break; } /* no move inside the band */
        if (c > g) g = c;
        if (g > eps) break;
    }
    if (steps) *steps = st;
    return g;
}

/* Greedy path with the DTW sum (an extension used only to seed the DTW
 * threshold): the walk of Alg. 1 (same moves, same tie order), but the value
 * is the fp32 sum of the costs along the path in path order, acc = fl(cost +
 * acc).  Any warping path's sum is >= DTW, and with monotone rounding the
 * fp32 path-order sum is >= the fp32 DP value, so this is an upper bound of
 * the fp32 DTW.  Early return once the sum exceeds eps. */
ORC_CLONES
float orc_greedy_sum_f32(const float *S, int64_t m, const float *T, int64_t n, int d, int64_t w,
                         float eps, int64_t *steps)
{
    int64_t i = 0, j = 0, st = 0;
    if (m <= 0 || n <= 0) {
        if (steps) *steps = 0;
        return ORC_INF;
    }
    float g = orc_cost_f32(S, T, d);
    if (g > eps) {
        if (steps) *steps = 0;
        return g;
    }
    while (!(i == m - 1 && j == n - 1)) {
        float c_dn = ORC_INF, c_dg = ORC_INF, c_rt = ORC_INF;
        if (i + 1 < m && orc_band_ok(i + 1, j, m, n, w))
            c_dn = orc_cost_f32(S + (i + 1) * d, T + j * d, d);
        if (i + 1 < m && j + 1 < n && orc_band_ok(i + 1, j + 1, m, n, w))
            c_dg = orc_cost_f32(S + (i + 1) * d, T + (j + 1) * d, d);
        if (j + 1 < n && orc_band_ok(i, j + 1, m, n, w))
            c_rt = orc_cost_f32(S + i * d, T + (j + 1) * d, d);
        float c;
        if (c_dn <= c_dg && c_dn <= c_rt) { c = c_dn; i += 1; }
        else if (c_dg <= c_rt) { c = c_dg; i += 1; j += 1; }
        else { c = c_rt; j += 1; }
        ++st;
        if (c == ORC_INF) { g = ORC_INF; break; }
        g = c + g;
        if (g > eps) break;
    }
    if (steps) *steps = st;
    return g;
}

/* ---------------------------------------------------------------- sparse DK (Alg. 3)
 * Sec. 4.2, Alg. 3, whole matching (SUB = false), squared domain, written as
 * the thresholded recurrence the algorithm evaluates.  A cell (i, j) is live
 * when its cost is <= eps and one of its predecessors (i-1, j), (i, j-1),
 * (i-1, j-1) is live; the start (0, 0) has the virtual predecessor 0
 * (R-sdk0).  A live cell holds max(cost, smallest live predecessor); every
 * other cell counts as +inf.  With [lo, hi] the live rows of column j-1, a
 * live cell of column j lies in rows lo .. hi+1 or is reached from the live
 * cell below it in its own column, so each column is evaluated from row lo
 * upward, through row hi+1 and on while the cell below is live.  A column
 * with no live cell ends the scan (R-sdkend): squared DK > eps, +inf.
 * Returns squared DK if it is <= eps, else +inf.  *cells (nullable)
 * receives the number of evaluated in-band cells.  The band, if any,
 * restricts the cells. */
ORC_CLONES
float orc_sparse_dk_sq_f32(const float *S, int64_t m, const float *T, int64_t n, int d,
                           int64_t w, float eps, int64_t *cells)
{
    if (m <= 0 || n <= 0) {
        if (cells) *cells = 0;
        return ORC_INF;
    }
    /* two columns; each remembers the rows it wrote, reset before reuse */
    float *col[2] = {malloc(sizeof(float) * m), malloc(sizeof(float) * m)};
    int64_t wlo[2] = {0, 0}, whi[2] = {m - 1, m - 1};
    for (int64_t i = 0; i < m; ++i) col[0][i] = col[1][i] = ORC_INF;
    int64_t lo = 0, hi = -1; /* live rows of the previous column (none yet) */
    int64_t visited = 0;
    float result = ORC_INF;
    for (int64_t j = 0; j < n; ++j) {
        float *prev = col[(j + 1) & 1], *cur = col[j & 1];
        const int c = (int)(j & 1);
        for (int64_t i = wlo[c]; i <= whi[c]; ++i) cur[i] = ORC_INF;
        const int64_t first = j == 0 ? 0 : lo;
        const int64_t reach = j == 0 ? 0 : hi + 1; /* last row fed by column j-1 */
        int64_t nlo = -1, nhi = -1, last = first - 1;
        for (int64_t i = first; i < m; ++i) {
            const float below = i > 0 ? cur[i - 1] : ORC_INF;
            if (i > reach && !(below <= eps))
                break; /* no live predecessor above this row */
            last = i;
            float pred;
            if (i == 0 && j == 0)
                pred = 0.0f;
            else
                pred = fmin3f(below, prev[i], i > 0 ? prev[i - 1] : ORC_INF);
            float v = ORC_INF;
            if (orc_band_ok(i, j, m, n, w)) {
                ++visited;
                const float cost = orc_cost_f32(S + i * d, T + j * d, d);
                if (cost <= eps && pred <= eps)
                    v = cost > pred ? cost : pred;
            }
            cur[i] = v;
            if (v != ORC_INF) {
                if (nlo < 0) nlo = i;
                nhi = i;
            }
        }
        wlo[c] = first;
        whi[c] = last;
        if (j == n - 1) {
            result = cur[m - 1];
            break;
        }
        if (nlo < 0)
            break; /* R-sdkend: no live cell left -> DK > eps */
        lo = nlo;
        hi = nhi;
    }
    free(col[0]); free(col[1]);
    if (cells) *cells = visited;
    return result;
}

/* ---------------------------------------------------------------- k-NN helpers */
typedef struct { float key; int64_t id; } orc_kv;

static int orc_kv_less(orc_kv a, orc_kv b)
{
    /* keys are >= 0 or +inf; order (key, id) ascending */
    if (a.key < b.key) return 1;
    if (a.key > b.key) return 0;
    return a.id < b.id;
}

static int orc_kv_cmp(const void *pa, const void *pb)
{
    orc_kv a = *(const orc_kv *)pa, b = *(const orc_kv *)pb;
    return orc_kv_less(a, b) ? -1 : (orc_kv_less(b, a) ? 1 : 0);
}

/* Keep the k smallest (key, id) in a sorted array; returns 1 if inserted. */
static int orc_topk_insert(orc_kv *top, int64_t *cnt, int64_t k, orc_kv x)
{
    if (*cnt == k && !orc_kv_less(x, top[k - 1]))
        return 0;
    int64_t p = (*cnt < k) ? (*cnt)++ : k - 1;
    while (p > 0 && orc_kv_less(x, top[p - 1])) {
        top[p] = top[p - 1];
        --p;
    }
    top[p] = x;
    return 1;
}

/* dist: 0 = DTW, 1 = DK.  band_mode: 0 none, 1 absolute w = band_r,
 * 2 fractional w = floor(band_frac * max(m, n)). */
static int64_t orc_pair_w(int band_mode, int64_t band_r, float band_frac, int64_t m, int64_t n)
{
    if (band_mode == 1) return band_r;
    if (band_mode == 2) return orc_band_w_frac(band_frac, m, n);
    return -1;
}

static float orc_pair_key(int dist, const float *S, int64_t m, const float *T, int64_t n, int d, int64_t w)
{
    return dist == 0 ? orc_dtw_f32(S, m, T, n, d, w) : orc_dk_sq_f32(S, m, T, n, d, w);
}

/* Plain definition of the k-NN query (Sec. 1: the k most similar series):
 * the full DP for every (query, candidate) pair, then a (key, id) sort.
 * Outputs [nq][k]: ids (-1 padding), keys (squared for DK; +inf padding).
 * Queries run in parallel when OpenMP is on. */
void orc_knn_brute(const float *db, const int64_t *db_off, int64_t N,
                   const float *qs, const int64_t *q_off, int64_t nq, int d,
                   int64_t k, int dist, int band_mode, int64_t band_r, float band_frac,
                   int64_t *out_ids, float *out_keys)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < nq; ++q) {
        const float *S = qs + q_off[q] * d;
        int64_t m = q_off[q + 1] - q_off[q];
        orc_kv *all = malloc(sizeof(orc_kv) * (N > 0 ? N : 1));
        for (int64_t c = 0; c < N; ++c) {
            int64_t n = db_off[c + 1] - db_off[c];
            int64_t w = orc_pair_w(band_mode, band_r, band_frac, m, n);
            all[c].key = orc_pair_key(dist, S, m, db + db_off[c] * d, n, d, w);
            all[c].id = c;
        }
        qsort(all, N, sizeof(orc_kv), orc_kv_cmp);
        for (int64_t r = 0; r < k; ++r) {
            if (r < N && all[r].key != ORC_INF) {
                out_ids[q * k + r] = all[r].id;
                out_keys[q * k + r] = all[r].key;
            } else {
                out_ids[q * k + r] = -1;
                out_keys[q * k + r] = ORC_INF;
            }
        }
        free(all);
    }
}

/* All-pairs keys [nq][N] by the full DP (for sampled checks and statistics). */
void orc_pair_keys(const float *db, const int64_t *db_off, int64_t N,
                   const float *qs, const int64_t *q_off, int64_t nq, int d,
                   int dist, int band_mode, int64_t band_r, float band_frac, float *out)
{
#pragma omp parallel for collapse(2) schedule(dynamic, 16)
    for (int64_t q = 0; q < nq; ++q)
        for (int64_t c = 0; c < N; ++c) {
            int64_t m = q_off[q + 1] - q_off[q], n = db_off[c + 1] - db_off[c];
            int64_t w = orc_pair_w(band_mode, band_r, band_frac, m, n);
            out[q * N + c] = orc_pair_key(dist, qs + q_off[q] * d, m, db + db_off[c] * d, n, d, w);
        }
}

/* DTW with early abandoning on a full row of the band whose minimum already
 * exceeds tau (Sec. 4, first paragraph: the minimum of a row is a lower bound
 * of the final value).  Returns DTW (fp32 mirror arithmetic) or +inf. */
static float orc_dtw_abandon_f32(const float *S, int64_t m, const float *T, int64_t n, int d,
                                 int64_t w, float tau, int64_t *cells)
{
    float *prev = malloc(sizeof(float) * n), *cur = malloc(sizeof(float) * n);
    int64_t cnt = 0;
    float r = ORC_INF;
    int dead = 0;
    for (int64_t i = 0; i < m && !dead; ++i) {
        float rowmin = ORC_INF;
        for (int64_t j = 0; j < n; ++j) {
            if (!orc_band_ok(i, j, m, n, w)) {
                cur[j] = ORC_INF;
                continue;
            }
            ++cnt;
            float best = (i == 0 && j == 0) ? 0.0f
                         : fmin3f((i > 0 && j > 0) ? prev[j - 1] : ORC_INF,
                                  (i > 0) ? prev[j] : ORC_INF,
                                  (j > 0) ? cur[j - 1] : ORC_INF);
            cur[j] = orc_cost_f32(S + i * d, T + j * d, d) + best;
            if (cur[j] < rowmin) rowmin = cur[j];
        }
        if (rowmin > tau) dead = 1;
        float *tmp = prev; prev = cur; cur = tmp;
    }
    if (!dead) r = prev[n - 1];
    if (r > tau) r = ORC_INF;
    free(prev); free(cur);
    if (cells) *cells += cnt;
    return r;
}

/* Envelope of the query S (m rows) for the columns of a candidate of length
 * n: for column j, the per-dimension [min, max] of the rows i that the band
 * lets j align with (the transposed band test of Sec. 2.3's windows).
 * lo, hi: [n][d]; an empty window gives lo = +inf, hi = -inf. */
void orc_qenv(const float *S, int64_t m, int64_t n, int d, int64_t w, float *lo, float *hi)
{
    for (int64_t j = 0; j < n; ++j) {
        for (int k = 0; k < d; ++k) { lo[j * d + k] = ORC_INF; hi[j * d + k] = -ORC_INF; }
        for (int64_t i = 0; i < m; ++i) {
            if (!orc_band_ok(i, j, m, n, w)) continue;
            for (int k = 0; k < d; ++k) {
                float v = S[i * d + k];
                if (v < lo[j * d + k]) lo[j * d + k] = v;
                if (v > hi[j * d + k]) hi[j * d + k] = v;
            }
        }
    }
}

/* Sum over the candidate's points t_j of the squared distance to the query
 * envelope's box of column j (lo, hi from orc_qenv), fp32 in candidate order
 * (R-lb). */
static float orc_lb_box_qenv_sum_f32(const float *T, int64_t n, int d, const float *lo,
                                     const float *hi)
{
    float acc = 0.0f;
    for (int64_t j = 0; j < n; ++j)
        acc = orc_box_term_f32(T + j * d, lo + j * d, hi + j * d, d) + acc;
    return acc;
}

/* LB_Box with the envelope of the query S around each point of the
 * candidate T: sum over the candidate's points t_j of the squared distance to
 * the box of S over the rows i that the band lets column j align with.  This
 * is LB_Box(T, S) of eq. (1) with the roles of the series exchanged; fp32 in
 * candidate order (R-lb). */
float orc_lb_box_qenv_f32(const float *S, int64_t m, const float *T, int64_t n, int d, int64_t w)
{
    float *lo = malloc(sizeof(float) * n * d), *hi = malloc(sizeof(float) * n * d);
    orc_qenv(S, m, n, d, w, lo, hi);
    float acc = orc_lb_box_qenv_sum_f32(T, n, d, lo, hi);
    free(lo); free(hi);
    return acc;
}

/* DK lower bound from the boxes of Sec. 3.  DK^2 is the largest point cost
 * on the best warping path (Sec. 2.1), and every path aligns each row i of S
 * with some column of its band window, at a cost no smaller than the squared
 * distance of s_i to the box B_i of T over that window.  So the largest of
 * these box distances bounds DK^2 from below: eq. (1)'s construction with a
 * maximum in place of the sum.  fp32 box terms in the point cost's order
 * (each at most the fp32 cost of any cell of its window, by monotone
 * rounding); a maximum rounds nothing.  An empty window gives +inf. */
float orc_lb_dk_box_f32(const float *S, int64_t m, const float *T, int64_t n, int d, int64_t w)
{
    float *lo = malloc(sizeof(float) * m * d), *hi = malloc(sizeof(float) * m * d);
    orc_envelope(T, n, m, d, w, lo, hi);
    float best = 0.0f;
    for (int64_t i = 0; i < m; ++i) {
        float t = orc_box_term_f32(S + i * d, lo + i * d, hi + i * d, d);
        if (t > best) best = t;
    }
    free(lo); free(hi);
    return best;
}

/* The same bound with the roles of the series exchanged: boxes of the query
 * S over the rows each column j of T may align with (orc_qenv), the largest
 * box distance over the candidate's points t_j. */
float orc_lb_dk_box_qenv_f32(const float *S, int64_t m, const float *T, int64_t n, int d,
                             int64_t w)
{
    float *lo = malloc(sizeof(float) * n * d), *hi = malloc(sizeof(float) * n * d);
    orc_qenv(S, m, n, d, w, lo, hi);
    float best = 0.0f;
    for (int64_t j = 0; j < n; ++j) {
        float t = orc_box_term_f32(T + j * d, lo + j * d, hi + j * d, d);
        if (t > best) best = t;
    }
    free(lo); free(hi);
    return best;
}

/* Paper-faithful pruned scan, one query at a time in candidate-id order.
 *   DK  (Sec. 4.3): a first pass computes the greedy bound (Alg. 1) of every
 *       candidate with early return against the running k-th smallest bound;
 *       its k-th smallest value is the threshold; a second pass runs the
 *       sparse DK (Alg. 3) of every candidate against the current threshold,
 *       which is lowered whenever k exact values below it are known.
 *   DTW (Sec. 1 and Sec. 5.1): threshold starts at +inf; each candidate is
 *       pruned when LB_Box > threshold, else DTW with row-minimum early
 *       abandoning runs and the k best are kept.
 * Output as orc_knn_brute.  stats (nullable, 4 int64 per query):
 *   [pruned by the bound, DP started, DP completed (finite), cells visited]. */
static void orc_knn_scan_impl(const float *db, const int64_t *db_off, int64_t N,
                              const float *qs, const int64_t *q_off, int64_t nq, int d,
                              int64_t k, int dist, int band_mode, int64_t band_r,
                              float band_frac, int64_t *out_ids, float *out_keys,
                              int64_t *stats, int keep_env)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < nq; ++q) {
        const float *S = qs + q_off[q] * d;
        int64_t m = q_off[q + 1] - q_off[q];
        /* keep_env: the query's envelope for a candidate length, built on
         * first use and kept (index = length) instead of rebuilt per pair */
        float **env = keep_env ? calloc(ORC_MAX_LEN + 1, sizeof(float *)) : NULL;
        orc_kv *top = malloc(sizeof(orc_kv) * k);
        int64_t cnt = 0, pruned = 0, started = 0, completed = 0, cells = 0;
        float tau = ORC_INF;
        if (dist == 1) {
            orc_kv *ub = malloc(sizeof(orc_kv) * k);
            int64_t nub = 0;
            for (int64_t c = 0; c < N; ++c) {
                int64_t n = db_off[c + 1] - db_off[c];
                int64_t w = orc_pair_w(band_mode, band_r, band_frac, m, n);
                float eps = (nub == k) ? ub[k - 1].key : ORC_INF;
                float g = orc_gdk_sq_f32(S, m, db + db_off[c] * d, n, d, w, eps, NULL);
                if (g <= eps && g != ORC_INF) {
                    orc_kv x = {g, c};
                    orc_topk_insert(ub, &nub, k, x);
                }
            }
            tau = (nub == k) ? ub[k - 1].key : ORC_INF;
            free(ub);
            for (int64_t c = 0; c < N; ++c) {
                int64_t n = db_off[c + 1] - db_off[c];
                int64_t w = orc_pair_w(band_mode, band_r, band_frac, m, n);
                int64_t vis = 0;
                ++started;
                float v = orc_sparse_dk_sq_f32(S, m, db + db_off[c] * d, n, d, w, tau, &vis);
                cells += vis;
                if (v != ORC_INF) {
                    ++completed;
                    orc_kv x = {v, c};
                    orc_topk_insert(top, &cnt, k, x);
                    if (cnt == k && top[k - 1].key < tau) tau = top[k - 1].key;
                }
            }
        } else {
            for (int64_t c = 0; c < N; ++c) {
                int64_t n = db_off[c + 1] - db_off[c];
                int64_t w = orc_pair_w(band_mode, band_r, band_frac, m, n);
                const float *T = db + db_off[c] * d;
                float lb;
                if (env && n <= ORC_MAX_LEN) {
                    if (!env[n]) {
                        env[n] = malloc(sizeof(float) * 2 * n * d);
                        orc_qenv(S, m, n, d, w, env[n], env[n] + n * d);
                    }
                    lb = orc_lb_box_qenv_sum_f32(T, n, d, env[n], env[n] + n * d);
                } else {
                    lb = orc_lb_box_qenv_f32(S, m, T, n, d, w);
                }
                if (lb > tau) { ++pruned; continue; }
                ++started;
                float v = orc_dtw_abandon_f32(S, m, T, n, d, w, tau, &cells);
                if (v != ORC_INF) {
                    ++completed;
                    orc_kv x = {v, c};
                    orc_topk_insert(top, &cnt, k, x);
                    if (cnt == k && top[k - 1].key < tau) tau = top[k - 1].key;
                }
            }
        }
        for (int64_t r = 0; r < k; ++r) {
            if (r < cnt) { out_ids[q * k + r] = top[r].id; out_keys[q * k + r] = top[r].key; }
            else { out_ids[q * k + r] = -1; out_keys[q * k + r] = ORC_INF; }
        }
        if (stats) {
            stats[q * 4 + 0] = pruned; stats[q * 4 + 1] = started;
            stats[q * 4 + 2] = completed; stats[q * 4 + 3] = cells;
        }
        free(top);
        if (env) {
            for (int64_t L = 0; L <= ORC_MAX_LEN; ++L) free(env[L]);
            free(env);
        }
    }
}

void orc_knn_scan(const float *db, const int64_t *db_off, int64_t N,
                  const float *qs, const int64_t *q_off, int64_t nq, int d,
                  int64_t k, int dist, int band_mode, int64_t band_r, float band_frac,
                  int64_t *out_ids, float *out_keys, int64_t *stats)
{
    orc_knn_scan_impl(db, db_off, N, qs, q_off, nq, d, k, dist, band_mode, band_r, band_frac,
                      out_ids, out_keys, stats, 0);
}

/* The same scan with each query's envelope built once per candidate length
 * (the DTW bound's values are unchanged: the same envelope, the same sums).
 * Used to check full-size results, where rebuilding the envelope for every
 * pair would take hours. */
void orc_knn_verify(const float *db, const int64_t *db_off, int64_t N,
                    const float *qs, const int64_t *q_off, int64_t nq, int d,
                    int64_t k, int dist, int band_mode, int64_t band_r, float band_frac,
                    int64_t *out_ids, float *out_keys, int64_t *stats)
{
    orc_knn_scan_impl(db, db_off, N, qs, q_off, nq, d, k, dist, band_mode, band_r, band_frac,
                      out_ids, out_keys, stats, 1);
}

/* Full-DP keys of a list of (query, candidate) pairs: out[p] = key of
 * (qi[p], ci[p]) (DTW sum or squared DK), in parallel over the list. */
void orc_pair_list_keys(const float *db, const int64_t *db_off, const float *qs,
                        const int64_t *q_off, int d, int64_t n_pairs, const int64_t *qi,
                        const int64_t *ci, int dist, int band_mode, int64_t band_r,
                        float band_frac, float *out)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t p = 0; p < n_pairs; ++p) {
        const int64_t q = qi[p], c = ci[p];
        int64_t m = q_off[q + 1] - q_off[q], n = db_off[c + 1] - db_off[c];
        int64_t w = orc_pair_w(band_mode, band_r, band_frac, m, n);
        out[p] = orc_pair_key(dist, qs + q_off[q] * d, m, db + db_off[c] * d, n, d, w);
    }
}

/* ================================================================ subsequence search
 * Sec. 4.1-4.2: a match may start and end anywhere in the long series T
 * (the query S is matched against a contiguous part T[a..b]).  The
 * subsequence DK of (S, T) is min over 0 <= a <= b < n of DK(S, T[a..b]);
 * its end is the first column b at which that minimum is reached, its start
 * the latest a <= b with DK(S, T[a..b]) equal to it (the shortest match
 * ending at b).  Squared domain as everywhere else.
 *
 * Readings (listed in the design notes too):
 *   R-sub0   in SUB mode row 0 has a virtual predecessor of -inf in every
 *            column (a match may start in any column), so D(0,k) = c(0,k);
 *            the printed vectors start at +inf and would never start.
 *   R-subd   the running minimum d of Alg. 3 is set to +inf once, before the
 *            column loop (the listing resets it inside the loop, which would
 *            keep only the last column's value).
 *   R-sgdk   Alg. 2's walk starts at the first j minimising c(s_0, t_j) and
 *            stops once the last row is reached; a move past the last column
 *            counts as +inf; ties as in Alg. 1. */

/* Plain SUB DP (Alg. 3 with SUB, every cell visited): columns of T in
 * order, D(i,k) = max(c(i,k), min(D(i-1,k), D(i,k-1), D(i-1,k-1))) with
 * D(0,k) = c(0,k).  Returns min_k D(m-1,k); *end = first such k. */
ORC_CLONES
float orc_subseq_dk_sq_f32(const float *S, int64_t m, const float *T, int64_t n, int d,
                           int64_t *end)
{
    if (end) *end = -1;
    if (m <= 0 || n <= 0)
        return ORC_INF;
    float *E = malloc(sizeof(float) * m), *D = malloc(sizeof(float) * m);
    for (int64_t i = 0; i < m; ++i) E[i] = ORC_INF;
    float best = ORC_INF;
    for (int64_t k = 0; k < n; ++k) {
        for (int64_t i = 0; i < m; ++i) {
            float c = orc_cost_f32(S + i * d, T + k * d, d);
            if (i == 0) {
                D[0] = c; /* R-sub0 */
            } else {
                float pred = fmin3f(D[i - 1], E[i], E[i - 1]);
                D[i] = c > pred ? c : pred;
            }
        }
        if (D[m - 1] < best) {
            best = D[m - 1];
            if (end) *end = k;
        }
        float *t = E; E = D; D = t;
    }
    free(E); free(D);
    return best;
}

/* The latest start a <= e with DK(S, T[a..e]) == key (whole-match DK of the
 * sub-series, Sec. 2.1), or -1 if there is none. */
int64_t orc_subseq_start(const float *S, int64_t m, const float *T, int64_t e, int d, float key)
{
    for (int64_t a = e; a >= 0; --a)
        if (orc_dk_sq_f32(S, m, T + a * d, e - a + 1, d, -1) == key)
            return a;
    return -1;
}

/* Definition by brute force: DK(S, T[a..b]) for every a <= b (tiny inputs
 * only).  Returns the minimum; *end = first b reaching it, *start = latest
 * a for that b. */
float orc_subseq_brute_f32(const float *S, int64_t m, const float *T, int64_t n, int d,
                           int64_t *end, int64_t *start)
{
    float best = ORC_INF;
    int64_t be = -1, bs = -1;
    for (int64_t b = 0; b < n; ++b)
        for (int64_t a = b; a >= 0; --a) {
            float v = orc_dk_sq_f32(S, m, T + a * d, b - a + 1, d, -1);
            if (v < best) { best = v; be = b; bs = a; }
        }
    if (end) *end = be;
    if (start) *start = bs;
    return best;
}

/* Alg. 2 (greedy DK for subsequence search), reading R-sgdk; early return
 * once the running max exceeds eps.  *steps = moves made. */
ORC_CLONES
float orc_sub_gdk_sq_f32(const float *S, int64_t m, const float *T, int64_t n, int d, float eps,
                         int64_t *steps)
{
    int64_t st = 0;
    if (steps) *steps = 0;
    if (m <= 0 || n <= 0)
        return ORC_INF;
    int64_t j = 0;
    float g = orc_cost_f32(S, T, d);
    for (int64_t jj = 1; jj < n; ++jj) {
        float c = orc_cost_f32(S, T + jj * d, d);
        if (c < g) { g = c; j = jj; }
    }
    int64_t i = 0;
    if (g > eps) return g;
    while (i != m - 1) {
        float c_dn = orc_cost_f32(S + (i + 1) * d, T + j * d, d);
        float c_dg = j + 1 < n ? orc_cost_f32(S + (i + 1) * d, T + (j + 1) * d, d) : ORC_INF;
        float c_rt = j + 1 < n ? orc_cost_f32(S + i * d, T + (j + 1) * d, d) : ORC_INF;
        float c;
        if (c_dn <= c_dg && c_dn <= c_rt) { c = c_dn; i += 1; }
        else if (c_dg <= c_rt) { c = c_dg; i += 1; j += 1; }
        else { c = c_rt; j += 1; }
        ++st;
        if (c > g) g = c;
        if (g > eps) break;
    }
    if (steps) *steps = st;
    return g;
}

/* Alg. 3 with SUB = true: the sparse column sweep that only visits a cell
 * whose own cost is <= eps, its visits of the next column coming from the
 * live cells of this one, plus row 0 in every column (any column may start
 * a match).  Returns the subsequence DK if it is <= eps, else +inf; *end =
 * first column reaching it; *cells = visited cells. */
ORC_CLONES
float orc_sparse_dk_sub_sq_f32(const float *S, int64_t m, const float *T, int64_t n, int d,
                               float eps, int64_t *end, int64_t *cells)
{
    if (end) *end = -1;
    if (cells) *cells = 0;
    if (m <= 0 || n <= 0)
        return ORC_INF;
    float *D = malloc(sizeof(float) * m), *E = malloc(sizeof(float) * m);
    char *inI = calloc(m + 1, 1), *inJ = calloc(m + 1, 1);
    for (int64_t i = 0; i < m; ++i) D[i] = E[i] = ORC_INF;
    float dmin = ORC_INF; /* R-subd */
    int64_t visited = 0;
    inI[0] = 1;
    for (int64_t k = 0; k < n; ++k) {
        /* rows in ascending order; visiting a live row adds the next row of
         * this column (I = I + {i+1}) and rows i, i+1 of the next (J) */
        for (int64_t i = 0; i < m; ++i) {
            if (!inI[i])
                continue;
            ++visited;
            float c = orc_cost_f32(S + i * d, T + k * d, d);
            if (c <= eps) {
                float pred = i == 0 ? -ORC_INF /* R-sub0 */
                                    : fmin3f(D[i - 1], E[i], E[i - 1]);
                D[i] = c > pred ? c : pred;
                inI[i + 1] = 1;
                inJ[i] = 1;
                inJ[i + 1] = 1;
            }
        }
        if (D[m - 1] < dmin) {
            dmin = D[m - 1];
            if (end) *end = k;
        }
        /* E = D; D = +inf; I = J + {0}; J = {} */
        for (int64_t i = 0; i < m; ++i) { E[i] = D[i]; D[i] = ORC_INF; }
        for (int64_t i = 0; i <= m; ++i) { inI[i] = inJ[i]; inJ[i] = 0; }
        inI[0] = 1;
    }
    free(D); free(E); free(inI); free(inJ);
    if (cells) *cells = visited;
    if (dmin > eps) {
        if (end) *end = -1;
        return ORC_INF;
    }
    return dmin;
}

/* Plain definition of the subsequence k-NN query: for every (query, series)
 * the subsequence DK by the plain SUB DP, then a (key, id) sort.  Outputs
 * [nq][k]: ids, keys (squared), end and start columns of each match (-1,
 * +inf, -1, -1 padding).  Queries in parallel under OpenMP. */
void orc_subseq_knn(const float *ser, const int64_t *s_off, int64_t N, const float *qs,
                    const int64_t *q_off, int64_t nq, int d, int64_t k, int64_t *out_ids,
                    float *out_keys, int64_t *out_end, int64_t *out_start)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < nq; ++q) {
        const float *S = qs + q_off[q] * d;
        int64_t m = q_off[q + 1] - q_off[q];
        orc_kv *all = malloc(sizeof(orc_kv) * (N > 0 ? N : 1));
        int64_t *ends = malloc(sizeof(int64_t) * (N > 0 ? N : 1));
        for (int64_t c = 0; c < N; ++c) {
            all[c].key = orc_subseq_dk_sq_f32(S, m, ser + s_off[c] * d, s_off[c + 1] - s_off[c], d,
                                              &ends[c]);
            all[c].id = c;
        }
        qsort(all, N, sizeof(orc_kv), orc_kv_cmp);
        for (int64_t r = 0; r < k; ++r) {
            int64_t o = q * k + r;
            if (r < N && all[r].key != ORC_INF) {
                int64_t c = all[r].id, e = ends[c];
                out_ids[o] = c;
                out_keys[o] = all[r].key;
                out_end[o] = e;
                out_start[o] = orc_subseq_start(S, m, ser + s_off[c] * d, e, d, all[r].key);
            } else {
                out_ids[o] = -1; out_keys[o] = ORC_INF; out_end[o] = -1; out_start[o] = -1;
            }
        }
        free(all); free(ends);
    }
}

/* The paper's pruned subsequence scan (Sec. 4.3 with the SUB variants):
 * threshold = k-th smallest Alg. 2 bound over the series, then Alg. 3 with
 * SUB per series in id order, the threshold falling to the k-th best value
 * found.  Same outputs as orc_subseq_knn; stats[q] = visited cells. */
void orc_subseq_scan(const float *ser, const int64_t *s_off, int64_t N, const float *qs,
                     const int64_t *q_off, int64_t nq, int d, int64_t k, int64_t *out_ids,
                     float *out_keys, int64_t *out_end, int64_t *out_start, int64_t *stats)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < nq; ++q) {
        const float *S = qs + q_off[q] * d;
        int64_t m = q_off[q + 1] - q_off[q];
        orc_kv *ub = malloc(sizeof(orc_kv) * k), *top = malloc(sizeof(orc_kv) * k);
        int64_t *tend = malloc(sizeof(int64_t) * k);
        int64_t nub = 0, cnt = 0, cells = 0;
        for (int64_t c = 0; c < N; ++c) {
            float eps = (nub == k) ? ub[k - 1].key : ORC_INF;
            float g = orc_sub_gdk_sq_f32(S, m, ser + s_off[c] * d, s_off[c + 1] - s_off[c], d, eps,
                                         NULL);
            if (g <= eps && g != ORC_INF) {
                orc_kv x = {g, c};
                orc_topk_insert(ub, &nub, k, x);
            }
        }
        float tau = (nub == k) ? ub[k - 1].key : ORC_INF;
        for (int64_t c = 0; c < N; ++c) {
            int64_t e = -1, vis = 0;
            float v = orc_sparse_dk_sub_sq_f32(S, m, ser + s_off[c] * d, s_off[c + 1] - s_off[c],
                                               d, tau, &e, &vis);
            cells += vis;
            if (v != ORC_INF) {
                orc_kv x = {v, c};
                /* keep each kept entry's end column beside it */
                if (orc_topk_insert(top, &cnt, k, x)) {
                    int64_t p = 0;
                    while (top[p].id != c) ++p;
                    for (int64_t r = cnt - 1; r > p; --r) tend[r] = tend[r - 1];
                    tend[p] = e;
                }
                if (cnt == k && top[k - 1].key < tau) tau = top[k - 1].key;
            }
        }
        for (int64_t r = 0; r < k; ++r) {
            int64_t o = q * k + r;
            if (r < cnt) {
                int64_t c = top[r].id;
                out_ids[o] = c;
                out_keys[o] = top[r].key;
                out_end[o] = tend[r];
                out_start[o] = orc_subseq_start(S, m, ser + s_off[c] * d, tend[r], d, top[r].key);
            } else {
                out_ids[o] = -1; out_keys[o] = ORC_INF; out_end[o] = -1; out_start[o] = -1;
            }
        }
        if (stats) stats[q] = cells;
        free(ub); free(top); free(tend);
    }
}
