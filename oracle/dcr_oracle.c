/*
 * dcr_oracle.c -- plain CPU reference ("oracle") for multinomial resampling with
 * the divide-and-conquer inverse-CMF map of A. A. Popov, "A divide and conquer
 * strategy for multinomial particle filter resampling".
 *
 * TEST INFRASTRUCTURE ONLY.  The test-suite, the smoke check and the benchmark's
 * CPU-baseline leg are the only users of this file.  The GPU library neither
 * links nor calls it, and the two share no code, header, table or constant.
 *
 * Conventions
 *   - Indices are 0-based: the paper's index i is i-1 here.
 *   - All arithmetic is IEEE binary64, round-to-nearest; no fused contractions
 *     (built with -ffp-contract=off) except the explicit fma() in dd_quotient.
 *   - Sums that define the cumulative weights (Sec. I, Eq. 3) and the
 *     exponential-spacings sum (Sec. II, Alg. 1) are carried as double-double
 *     (TwoSum, Knuth / Dekker) so that the oracle is more accurate than any
 *     blocked binary64 summation it is compared with; the normalised value is
 *     the double nearest to the double-double quotient.
 *
 * Readings of the paper taken here (each is also listed in the design notes):
 *   R1  Alg. 1 divides every Z_i by the last partial sum Z_{N+1} (the printed
 *       Z_{i+1} would give unsorted, non-uniform values).
 *   R2  rand on [0,1] is replaced by the open-interval variate
 *       v = (2k+1) 2^-53, k a 52-bit integer from Philox4x32-10, so that -log v
 *       is finite and positive.
 *   R3  The random generator is Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
 *       SC'11).  Draw i (0..N) uses counter (i/2 low, i/2 high, stream low,
 *       stream high) and key (seed low, seed high); even i takes output words
 *       (x0, x1), odd i takes (x2, x3); k = (x_hi << 20) | (x_lo >> 12).
 *   R4  Eq. 3 prints "i = 1..N" for the cumulative weights; the range is 1..M.
 *   R5  The inverse CMF is clamped to the last bin (Alg. 2 starts with b = M),
 *       so r_i = #{ j in [0, M-2] : W_j < u_i }.
 *   R6  The last cumulative weight is set to exactly 1.
 *
 * parity unpinned: nothing.  Every function below is pinned by a test that does
 * not re-type its formula (exact rational arithmetic, brute force, the Fig. 1
 * worked example, a separately written library Philox, and distribution laws).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define DCRO_OK 0
#define DCRO_BAD_WEIGHTS 6
#define DCRO_INVALID 1

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 from its published definition (Salmon et al., SC'11):        */
/* ten rounds of two 32x32->64 multiplications and a key schedule that adds   */
/* the Weyl constants between rounds.                                         */
/* ------------------------------------------------------------------------- */
void dcro_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Reading R2/R3: the i-th open-interval uniform variate of (seed, stream). */
double dcro_uniform_open(uint64_t seed, uint64_t stream, uint64_t i)
{
    uint64_t pair = i >> 1;
    uint32_t ctr[4] = {(uint32_t)pair, (uint32_t)(pair >> 32),
                       (uint32_t)stream, (uint32_t)(stream >> 32)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    dcro_philox4x32_10(ctr, key, x);
    uint32_t lo = (i & 1) ? x[2] : x[0];
    uint32_t hi = (i & 1) ? x[3] : x[1];
    uint64_t k = ((uint64_t)hi << 20) | (uint64_t)(lo >> 12);
    return (double)(2 * k + 1) * 0x1p-53;
}

/* ------------------------------------------------------------------------- */
/* double-double helpers                                                      */
/* ------------------------------------------------------------------------- */
typedef struct { double hi, lo; } dd_t;

static dd_t dd_add(dd_t a, double b)
{
    double s = a.hi + b;
    double bb = s - a.hi;
    double err = (a.hi - (s - bb)) + (b - bb); /* TwoSum: a.hi + b = s + err */
    err += a.lo;
    double h = s + err;                          /* renormalise */
    double l = err - (h - s);
    dd_t r = {h, l};
    return r;
}

/* The double nearest to (a.hi + a.lo) / (b.hi + b.lo): q = a.hi / b.hi, its
 * exact remainder by fma, then one correction step.  It can differ from the
 * correctly rounded quotient only when that quotient lies within ~2^-100
 * (relative) of a rounding midpoint. */
static double dd_quotient(dd_t a, dd_t b)
{
    double q = a.hi / b.hi;
    double rem = fma(-q, b.hi, a.hi);
    rem += a.lo;
    rem -= q * b.lo;
    return q + rem / b.hi;
}

/* ------------------------------------------------------------------------- */
/* Sec. I, Eq. 3: cumulative weights W_j = sum_{k<=j} w_k / sum_k w_k.          */
/* ------------------------------------------------------------------------- */
static double load_weight(const void* w, int is_f32, int64_t j)
{
    return is_f32 ? (double)((const float*)w)[j] : ((const double*)w)[j];
}

static int cumulative_weights_impl(const void* w, int is_f32, int64_t M, double* W,
                                   double* total_out)
{
    if (M < 1) return DCRO_INVALID;
    dd_t T = {0.0, 0.0};
    for (int64_t j = 0; j < M; ++j) {
        double x = load_weight(w, is_f32, j);
        if (!(x >= 0.0) || isinf(x)) return DCRO_BAD_WEIGHTS;
        T = dd_add(T, x);
    }
    if (!(T.hi > 0.0) || isinf(T.hi)) return DCRO_BAD_WEIGHTS;
    if (total_out) *total_out = T.hi + T.lo;
    if (W) {
        dd_t S = {0.0, 0.0};
        for (int64_t j = 0; j < M - 1; ++j) {
            S = dd_add(S, load_weight(w, is_f32, j));
            W[j] = dd_quotient(S, T);
        }
        W[M - 1] = 1.0; /* reading R6 */
    }
    return DCRO_OK;
}

int dcro_cumulative_weights(const double* w, int64_t M, double* W, double* total)
{
    return cumulative_weights_impl(w, 0, M, W, total);
}

/* Same definition applied to binary32 weights promoted exactly to binary64. */
int dcro_cumulative_weights_f32(const float* w, int64_t M, double* W, double* total)
{
    return cumulative_weights_impl(w, 1, M, W, total);
}

/* ------------------------------------------------------------------------- */
/* Sec. II, Alg. 1: sorted uniforms from exponential spacings.                */
/*   z_i = -log v_i (i = 0..N), Z_i = z_0 + ... + z_i, u_i = Z_i / Z_N.        */
/* zkind 0: z in binary64 (the reference form).                               */
/* zkind 1: z = -logf(fl32(v)) promoted to binary64 (the binary32 form).       */
/* ------------------------------------------------------------------------- */
static double spacing(uint64_t seed, uint64_t stream, uint64_t i, int zkind)
{
    double v = dcro_uniform_open(seed, stream, i);
    if (zkind == 1) return (double)(-logf((float)v));
    return -log(v);
}

void dcro_exponential_spacings(int64_t N, uint64_t seed, uint64_t stream, int zkind, double* z)
{
    for (int64_t i = 0; i <= N; ++i) z[i] = spacing(seed, stream, (uint64_t)i, zkind);
}

/* Writes u[0..N-1]; if Z_total is not NULL it receives the last partial sum. */
void dcro_sorted_uniforms(int64_t N, uint64_t seed, uint64_t stream, int zkind, double* u,
                          double* Z_total)
{
    if (N < 0) return;
    dd_t T = {0.0, 0.0};
    for (int64_t i = 0; i <= N; ++i) T = dd_add(T, spacing(seed, stream, (uint64_t)i, zkind));
    if (Z_total) *Z_total = T.hi + T.lo;
    dd_t Z = {0.0, 0.0};
    for (int64_t i = 0; i < N; ++i) {
        Z = dd_add(Z, spacing(seed, stream, (uint64_t)i, zkind));
        u[i] = dd_quotient(Z, T); /* reading R1 */
    }
}

/* ------------------------------------------------------------------------- */
/* Sec. I, Eq. 3 written out: the inverse CMF of u is the number of bin edges  */
/* W_0..W_{M-2} lying strictly below u (reading R5).                           */
/* ------------------------------------------------------------------------- */
int32_t dcro_inverse_cmf_one(const double* W, int64_t M, double u)
{
    int64_t c = 0;
    for (int64_t j = 0; j + 1 < M; ++j)
        if (W[j] < u) ++c;
    return (int32_t)c;
}

void dcro_inverse_cmf_count(const double* W, int64_t M, const double* u, int64_t N, int32_t* r)
{
    for (int64_t i = 0; i < N; ++i) r[i] = dcro_inverse_cmf_one(W, M, u[i]);
}

/* ------------------------------------------------------------------------- */
/* Sec. II, Alg. 2 (the search the samplers share): over the inclusive range  */
/* Z[a..b] of a non-decreasing list, the first index m with Z_m >= X, or b    */
/* when no index before b qualifies (the clamp of reading R5).                */
/*                                                                           */
/* Written from that definition: the indices in [a, b) whose value is below X */
/* form a prefix of the range (Z is non-decreasing), so the answer is a plus  */
/* the length of that prefix.  The length is assembled from its binary digits,*/
/* largest first: a candidate step s is kept when the element s past the      */
/* prefix found so far is still below X.  Each probe is one comparison, which */
/* ncmp counts (about log2 of the range length per search, as Table I states  */
/* for the binary sampler).                                                   */
/* ------------------------------------------------------------------------- */
int64_t dcro_binary_search(const double* Z, int64_t a, int64_t b, double X, int64_t* ncmp)
{
    const int64_t n = b - a; /* candidates a .. b-1; b is the fall-back */
    int64_t top = 1;
    while (top <= n / 2) top *= 2;
    int64_t below = 0; /* length of the prefix of [a, b) known to lie below X */
    for (int64_t s = (n > 0) ? top : 0; s > 0; s /= 2) {
        if (below + s > n) continue;
        if (ncmp) ++*ncmp;
        if (Z[a + below + s - 1] < X) below += s;
    }
    return a + below;
}

/* Sec. II, Alg. 3 with the uniforms supplied: one full-range search each. */
void dcro_binary_sampler(const double* W, int64_t M, const double* u, int64_t N, int32_t* r,
                         int64_t* ncmp)
{
    for (int64_t i = 0; i < N; ++i) r[i] = (int32_t)dcro_binary_search(W, 0, M - 1, u[i], ncmp);
}

/* Sec. II, Alg. 4 (CCF) with sorted uniforms supplied; the scan stops at the
 * last bin (reading R5). */
void dcro_ccf(const double* W, int64_t M, const double* u, int64_t N, int32_t* r, int64_t* ncmp)
{
    int64_t j = 0;
    for (int64_t i = 0; i < N; ++i) {
        while (j < M - 1) {
            if (ncmp) ++*ncmp;
            if (W[j] < u[i])
                ++j;
            else
                break;
        }
        r[i] = (int32_t)j;
    }
}

/* ------------------------------------------------------------------------- */
/* Sec. III, Alg. 5: divide and conquer.  The sorted uniforms are located by  */
/* narrowing, for a contiguous run of them, the stretch of W their answers    */
/* must lie in.  A pending task is a run of uniforms U[iu0..iu1] together with */
/* a stretch W[jw0..jw1] known to contain every answer of the run.  Handling a */
/* task: if its stretch is a single bin, that bin is every answer; otherwise  */
/* its middle uniform (the lower middle of an even run, reading R11) is       */
/* located in the stretch with the search above, and the uniforms before it   */
/* become a task whose stretch ends at that answer while those after it       */
/* become a task whose stretch starts there (the uniforms are sorted, so      */
/* neither side can leave its part).  Tasks are handled in the order they are */
/* made (a first-in first-out list), so every depth of the splitting is done  */
/* before the next; the optional trace lists each located uniform as          */
/* (depth, uniform index, weight index) in that order.                         */
/* ------------------------------------------------------------------------- */
typedef struct {
    int64_t iu0, iu1, jw0, jw1, depth;
} dac_task;

/* Returns the trace length written (0 if no trace buffer). */
int64_t dcro_dac(const double* W, int64_t M, const double* u, int64_t N, int32_t* r,
                 int64_t* ncmp, int64_t* trace, int64_t trace_cap)
{
    if (N <= 0 || M <= 0) return 0;
    /* every task either settles all its uniforms or locates one and makes at
     * most two new tasks, so at most 2N + 1 tasks are ever made */
    dac_task* list = (dac_task*)malloc(sizeof(dac_task) * (size_t)(2 * N + 1));
    if (!list) return 0;
    int64_t made = 0, next = 0, traced = 0;
    dac_task first = {0, N - 1, 0, M - 1, 0};
    list[made++] = first;
    while (next < made) {
        const dac_task t = list[next++];
        if (t.jw0 == t.jw1) {
            for (int64_t i = t.iu0; i <= t.iu1; ++i) r[i] = (int32_t)t.jw0;
            continue;
        }
        const int64_t mid = t.iu0 + (t.iu1 - t.iu0) / 2;
        const int64_t at = dcro_binary_search(W, t.jw0, t.jw1, u[mid], ncmp);
        r[mid] = (int32_t)at;
        if (trace && traced < trace_cap) {
            trace[3 * traced + 0] = t.depth;
            trace[3 * traced + 1] = mid;
            trace[3 * traced + 2] = at;
            ++traced;
        }
        if (mid > t.iu0) {
            dac_task left = {t.iu0, mid - 1, t.jw0, at, t.depth + 1};
            list[made++] = left;
        }
        if (mid < t.iu1) {
            dac_task right = {mid + 1, t.iu1, at, t.jw1, t.depth + 1};
            list[made++] = right;
        }
    }
    free(list);
    return traced;
}

/* ------------------------------------------------------------------------- */
/* End to end (Sec. III, Alg. 5 "DaCSampler"): W from w, N sorted uniforms,    */
/* then the divide-and-conquer map.  W_out / u_out may be NULL.                */
/* ------------------------------------------------------------------------- */
static int resample_impl(const void* w, int is_f32, int64_t M, int64_t N, uint64_t seed,
                         uint64_t stream, int zkind, int32_t* r, double* W_out, double* u_out)
{
    if (M < 1 || N < 0) return DCRO_INVALID;
    double* W = W_out ? W_out : (double*)malloc(sizeof(double) * (size_t)M);
    double* u = u_out ? u_out : (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    int st = cumulative_weights_impl(w, is_f32, M, W, NULL);
    if (st == DCRO_OK && N > 0) {
        dcro_sorted_uniforms(N, seed, stream, zkind, u, NULL);
        dcro_dac(W, M, u, N, r, NULL, NULL, 0);
    }
    if (!W_out) free(W);
    if (!u_out) free(u);
    return st;
}

int dcro_resample(const double* w, int64_t M, int64_t N, uint64_t seed, uint64_t stream,
                  int32_t* r, double* W_out, double* u_out)
{
    return resample_impl(w, 0, M, N, seed, stream, 0, r, W_out, u_out);
}

/* binary64 weights with a chosen spacings form (zkind 1: the binary32 form,
 * as used when binary32 factors give exact binary64 product weights). */
int dcro_resample_z(const double* w, int64_t M, int64_t N, uint64_t seed, uint64_t stream,
                    int zkind, int32_t* r, double* W_out, double* u_out)
{
    return resample_impl(w, 0, M, N, seed, stream, zkind, r, W_out, u_out);
}

int dcro_resample_f32(const float* w, int64_t M, int64_t N, uint64_t seed, uint64_t stream,
                      int zkind, int32_t* r, double* W_out, double* u_out)
{
    return resample_impl(w, 1, M, N, seed, stream, zkind, r, W_out, u_out);
}

/* ------------------------------------------------------------------------- */
/* Other resampling schemes through the same inverse-CMF map.  Sec. V says the */
/* divide-and-conquer map carries over to other kinds of resampling without    */
/* giving an algorithm; the sorted uniforms here are the textbook ones:        */
/*   stratified  u_i = (i + v_i) / N   (one variate in each stratum);          */
/*   systematic  u_i = (i + v_0) / N   (one variate shared by all strata);     */
/* with v_i the variate of draw i of (seed, stream) (readings R2, R3).  Both   */
/* are non-decreasing in i and lie in (0, 1].  scheme 0 is Alg. 1.            */
/* ------------------------------------------------------------------------- */
#define DCRO_SCHEME_MULTINOMIAL 0
#define DCRO_SCHEME_STRATIFIED 1
#define DCRO_SCHEME_SYSTEMATIC 2

int dcro_scheme_uniforms(int64_t N, uint64_t seed, uint64_t stream, int scheme, double* u)
{
    if (N < 0) return DCRO_INVALID;
    if (scheme == DCRO_SCHEME_MULTINOMIAL) {
        if (N > 0) dcro_sorted_uniforms(N, seed, stream, 0, u, NULL);
        return DCRO_OK;
    }
    if (scheme != DCRO_SCHEME_STRATIFIED && scheme != DCRO_SCHEME_SYSTEMATIC) return DCRO_INVALID;
    const double v0 = dcro_uniform_open(seed, stream, 0);
    for (int64_t i = 0; i < N; ++i) {
        const double v = (scheme == DCRO_SCHEME_STRATIFIED) ? dcro_uniform_open(seed, stream, (uint64_t)i)
                                                           : v0;
        u[i] = ((double)i + v) / (double)N;
    }
    return DCRO_OK;
}

/* End to end with the scheme's uniforms (binary32 weights promoted exactly;
 * the multinomial scheme uses the binary32 spacings for them, as
 * dcro_resample_f32 with zkind 1). */
int dcro_resample_scheme(const void* w, int is_f32, int64_t M, int64_t N, uint64_t seed,
                         uint64_t stream, int scheme, int32_t* r, double* W_out, double* u_out)
{
    if (M < 1 || N < 0) return DCRO_INVALID;
    if (scheme == DCRO_SCHEME_MULTINOMIAL)
        return resample_impl(w, is_f32, M, N, seed, stream, is_f32 ? 1 : 0, r, W_out, u_out);
    if (scheme != DCRO_SCHEME_STRATIFIED && scheme != DCRO_SCHEME_SYSTEMATIC) return DCRO_INVALID;
    double* W = W_out ? W_out : (double*)malloc(sizeof(double) * (size_t)M);
    double* u = u_out ? u_out : (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    int st = cumulative_weights_impl(w, is_f32, M, W, NULL);
    if (st == DCRO_OK && N > 0) {
        dcro_scheme_uniforms(N, seed, stream, scheme, u);
        dcro_dac(W, M, u, N, r, NULL, NULL, 0);
    }
    if (!W_out) free(W);
    if (!u_out) free(u);
    return st;
}

/* Many independent resamples of one distribution with consecutive seeds, for
 * the statistical tests: r is [R][N]. */
int dcro_resample_repeat(const double* w, int64_t M, int64_t N, uint64_t seed0, int64_t R,
                         int32_t* r)
{
    double* W = (double*)malloc(sizeof(double) * (size_t)M);
    double* u = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    int st = cumulative_weights_impl(w, 0, M, W, NULL);
    for (int64_t k = 0; st == DCRO_OK && k < R && N > 0; ++k) {
        dcro_sorted_uniforms(N, seed0 + (uint64_t)k, 0, 0, u, NULL);
        dcro_dac(W, M, u, N, r + k * N, NULL, NULL, 0);
    }
    free(W);
    free(u);
    return st;
}

/* Batched form: filter b resamples its own segment w[w_off[b] .. w_off[b+1])
 * into r[n_off[b] .. n_off[b+1]) with stream id b; indices are local to the
 * segment.  Returns the first failing filter's status. */
static int resample_filter(const void* w, int is_f32, const int64_t* w_off, const int64_t* n_off,
                           int64_t b, uint64_t seed, int zkind, int32_t* r)
{
    int64_t M = w_off[b + 1] - w_off[b];
    int64_t N = n_off[b + 1] - n_off[b];
    const void* wb = is_f32 ? (const void*)((const float*)w + w_off[b])
                            : (const void*)((const double*)w + w_off[b]);
    return resample_impl(wb, is_f32, M, N, seed, (uint64_t)b, zkind, r + n_off[b], NULL, NULL);
}

int dcro_resample_batched(const void* w, int is_f32, const int64_t* w_off, const int64_t* n_off,
                          int64_t B, uint64_t seed, int zkind, int32_t* r)
{
    int st_all = DCRO_OK;
    for (int64_t b = 0; b < B; ++b) {
        int st = resample_filter(w, is_f32, w_off, n_off, b, seed, zkind, r);
        if (st != DCRO_OK && st_all == DCRO_OK) st_all = st;
    }
    return st_all;
}

/* The same with the filters spread over `nthreads` OpenMP threads (each
 * filter's arithmetic is unchanged, so the result equals the loop above).
 * Returns the status of the lowest-numbered failing filter; *threads_used
 * (if not NULL) receives the team size. */
int dcro_resample_batched_par(const void* w, int is_f32, const int64_t* w_off,
                              const int64_t* n_off, int64_t B, uint64_t seed, int zkind,
                              int nthreads, int32_t* r, int* threads_used)
{
    int64_t first_bad = B;
    int st_bad = DCRO_OK;
    int team = 1;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
#pragma omp single
        team = omp_get_num_threads();
#pragma omp for schedule(dynamic, 1)
        for (int64_t b = 0; b < B; ++b) {
            int st = resample_filter(w, is_f32, w_off, n_off, b, seed, zkind, r);
            if (st != DCRO_OK) {
#pragma omp critical
                if (b < first_bad) {
                    first_bad = b;
                    st_bad = st;
                }
            }
        }
    }
    if (threads_used) *threads_used = team;
    return st_bad;
}
