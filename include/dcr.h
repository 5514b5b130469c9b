/*
 * dcr.h -- C ABI of libdcr: multinomial resampling on AMD Instinct MI355X
 * (gfx950) by the divide-and-conquer inverse-CMF map of A. A. Popov,
 * "A divide and conquer strategy for multinomial particle filter resampling".
 *
 * The problem (Sec. I, Eqs. 1-3): given M non-negative weights w_j, draw N
 * indices r_i = P^{-1}(u_i), where P^{-1}(u) is the first bin j whose
 * normalised cumulative weight W_j = (w_0 + ... + w_j) / (w_0 + ... + w_{M-1})
 * is >= u, and u_0 <= ... <= u_{N-1} are sorted uniforms (Sec. II, Alg. 1).
 * Indices are 0-based here (the paper's index i is i-1 here).
 *
 * Conventions shared by every entry point
 *   - Memory: every array argument is a caller-owned DEVICE pointer (for
 *     example a torch tensor's data_ptr()).  The library allocates and frees
 *     device memory only in dcr_plan_create_batched / dcr_plan_destroy; the
 *     other calls use the caller's workspace `ws` of `ws_bytes` bytes, sized
 *     by dcr_workspace_bytes() and 256-byte aligned (dcr_resample_noalloc a
 *     static device array).
 *   - Streams: calls enqueue kernels on `stream` and return without
 *     synchronising; results are valid once the stream has reached them.
 *     Calls on different streams must not share a workspace.
 *   - Errors: problems visible on the host (NULL pointers with a non-zero
 *     size, sizes out of range, an unknown precision, a small workspace) return
 *     an error before anything is enqueued.  Problems in the data (a weight
 *     that is negative, NaN or infinite, or a zero / infinite total) are found
 *     on the device: then `*dev_status` (if not NULL) receives
 *     DCR_ERR_BAD_WEIGHTS, every r_i is set to -1 and W is not meaningful;
 *     otherwise `*dev_status` receives DCR_OK.  A failed HIP launch returns
 *     DCR_ERR_HIP (the status of the library's own launches, not an earlier,
 *     unrelated HIP error).
 *   - Sizes: 1 <= M <= 2^31 - 1 and 0 <= N <= 2^31 - 2; N = 0 draws nothing.
 *     N > M is allowed.
 *   - Randomness: draw i of (seed, stream_id) comes from Philox4x32-10
 *     (Salmon et al., SC'11), so every call is reproducible and streams are
 *     independent; a particle filter may use its time step as stream_id.
 */
#ifndef DCR_H
#define DCR_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum dcr_status {
    DCR_OK = 0,
    DCR_ERR_INVALID_ARGUMENT = 1,
    DCR_ERR_UNSUPPORTED = 2,
    DCR_ERR_WORKSPACE_TOO_SMALL = 3,
    DCR_ERR_CAPACITY_EXCEEDED = 4,
    DCR_ERR_HIP = 5,
    DCR_ERR_BAD_WEIGHTS = 6,
    DCR_ERR_INTERNAL = 7
} dcr_status;

/* Precision form.
 *   DCR_FP64:      w is binary64; z = -log v in binary64.
 *   DCR_FP32_COMP: w is binary32 (promoted exactly, sums carried in binary64);
 *                  z = -logf(fl32(v)) in binary32, sums carried in binary64.
 * In both forms W and u are returned as binary64. */
typedef enum dcr_precision {
    DCR_FP64 = 0,
    DCR_FP32_COMP = 1
} dcr_precision;

/* Sorted-uniform scheme of an end-to-end call.
 *   DCR_MULTINOMIAL: Sec. II, Alg. 1 (exponential spacings): multinomial
 *                    resampling, the paper's case.
 *   DCR_STRATIFIED:  u_i = (i + v_i) / N, one variate per stratum.
 *   DCR_SYSTEMATIC:  u_i = (i + v_0) / N, one variate for all strata.
 * v_d is the open-interval variate of draw d of (seed, stream_id), the same
 * Philox4x32-10 draw the spacings use.  Sec. V names the extension of the
 * divide-and-conquer map to such schemes; the map is unchanged. */
typedef enum dcr_scheme {
    DCR_MULTINOMIAL = 0,
    DCR_STRATIFIED = 1,
    DCR_SYSTEMATIC = 2
} dcr_scheme;

/* Human-readable name of a status code (static string, never NULL). */
const char* dcr_status_string(dcr_status s);

/* Workspace bytes needed by any single-distribution call below with sizes
 * (M, N) and precision p.  Host only; enqueues nothing.
 * Errors: DCR_ERR_INVALID_ARGUMENT for sizes out of range or bytes == NULL,
 * DCR_ERR_UNSUPPORTED for an unknown precision. */
dcr_status dcr_workspace_bytes(int64_t M, int64_t N, dcr_precision p, size_t* bytes);

/* Stage 1 -- Sec. I, Eq. 3: normalised cumulative weights.
 *   w        [M] binary64 (DCR_FP64) or binary32 (DCR_FP32_COMP), contiguous.
 *   W        [M] binary64 out: non-decreasing, W[M-1] == 1 exactly.
 *   total    [1] binary64 out (may be NULL): the sum the weights are divided by.
 *   dev_status [1] int32 out (may be NULL): DCR_OK or DCR_ERR_BAD_WEIGHTS.
 * The summation order is fixed (blocked, sequential within every level), so
 * repeated calls return identical bits. */
dcr_status dcr_cumulative_weights(const void* w, int64_t M, dcr_precision p, double* W,
                                  double* total, int32_t* dev_status, void* ws,
                                  size_t ws_bytes, hipStream_t stream);

/* Stage 2 -- Sec. II, Alg. 1: N sorted uniforms by exponential spacings.
 *   z_i = -log v_i for i = 0..N, Z_i = z_0 + ... + z_i, u_i = Z_i / Z_N.
 *   u        [N] binary64 out: non-decreasing, in (0, 1]. */
dcr_status dcr_sorted_uniforms(int64_t N, uint64_t seed, uint64_t stream_id, dcr_precision p,
                               double* u, void* ws, size_t ws_bytes, hipStream_t stream);

/* Stage 3 -- Sec. III, Alg. 5 (with Alg. 2 and Alg. 4 as its base cases): the
 * inverse CMF of sorted uniforms.
 *   W        [M] binary64, non-decreasing (precondition, not checked).
 *   u        [N] binary64, non-decreasing (precondition, not checked).
 *   r        [N] int32 out: r_i = #{ j in [0, M-2] : W_j < u_i }, i.e. the first
 *            j with W_j >= u_i, clamped to M-1.  The result is exact: it does
 *            not depend on how the search is organised. */
dcr_status dcr_inverse_cmf(const double* W, int64_t M, const double* u, int64_t N, int32_t* r,
                           void* ws, size_t ws_bytes, hipStream_t stream);

/* End to end -- Sec. III, Alg. 5 "DaCSampler": stage 1, stage 2 and stage 3.
 *   w, M, p      as in dcr_cumulative_weights.
 *   N, seed, stream_id  as in dcr_sorted_uniforms.
 *   r        [N] int32 out, non-decreasing.
 *   W_opt    [M] binary64 out or NULL (then W is never written to memory).
 *   u_opt    [N] binary64 out or NULL.
 *   dev_status [1] int32 out or NULL.
 * r equals dcr_inverse_cmf applied to the W of dcr_cumulative_weights and the u
 * of dcr_sorted_uniforms with the same arguments, bit for bit. */
dcr_status dcr_resample(const void* w, int64_t M, int64_t N, uint64_t seed, uint64_t stream_id,
                        dcr_precision p, int32_t* r, double* W_opt, double* u_opt,
                        int32_t* dev_status, void* ws, size_t ws_bytes, hipStream_t stream);

/* Batched form: B independent filters in one call (one filter = one
 * single-distribution problem of Sec. I-III, Alg. 5 on its own weights).
 * Filter b owns weights w[w_off[b] .. w_off[b+1]) and draws
 * r[n_off[b] .. n_off[b+1]); it uses Philox stream id b, so its indices equal
 * those of dcr_resample(w + w_off[b], M_b, N_b, seed, b, p, ...) bit for bit.
 *
 * dcr_batched_workspace_bytes: workspace for up to B filters with at most
 * sumM_max weights and sumN_max draws in total.  Host only.
 *   Errors: DCR_ERR_INVALID_ARGUMENT for B < 1, B > 2^24, sumM_max < B,
 *   sumM_max or sumN_max above 2^40 or negative, bytes == NULL;
 *   DCR_ERR_UNSUPPORTED for an unknown precision. */
dcr_status dcr_batched_workspace_bytes(int32_t B, int64_t sumM_max, int64_t sumN_max,
                                       dcr_precision p, size_t* bytes);

/* dcr_resample_batched:
 *   w        concatenated weights, binary64 or binary32 as p says; a filter
 *            may start at any element (no alignment needed).
 *   w_off    [B+1] int64 DEVICE array, non-decreasing, w_off[0] == 0,
 *            1 <= M_b = w_off[b+1] - w_off[b] <= 2^31 - 1, w_off[B] <= sumM_max.
 *            The device checks the offsets against sumM_max only, so w must
 *            hold at least sumM_max weights (the Python binding checks this).
 *   n_off    [B+1] int64 DEVICE array, n_off[0] == 0,
 *            0 <= N_b = n_off[b+1] - n_off[b] <= 2^31 - 2, n_off[B] <= sumN_max.
 *   r        [n_off[B]] int32 out: indices local to each filter (0..M_b-1),
 *            non-decreasing within a filter.
 *   seg_status [B] int32 out or NULL: DCR_OK or DCR_ERR_BAD_WEIGHTS per filter
 *            (a bad filter's indices are -1; the others are unaffected).
 *   dev_status [1] int32 out or NULL: DCR_OK; DCR_ERR_BAD_WEIGHTS if any filter
 *            is bad; DCR_ERR_INVALID_ARGUMENT if the offsets break the rules
 *            above; DCR_ERR_CAPACITY_EXCEEDED if the totals exceed sumM_max /
 *            sumN_max.  In the last two cases nothing else is written.
 *   ws       workspace of dcr_batched_workspace_bytes(B, sumM_max, sumN_max, p)
 *            bytes, 256-byte aligned.
 * The offsets are read on the device, so the call never synchronises with the
 * host.  Host-visible errors are those of dcr_batched_workspace_bytes, NULL
 * pointers, a misaligned or small workspace. */
dcr_status dcr_resample_batched(const void* w, const int64_t* w_off, const int64_t* n_off,
                                int32_t B, int64_t sumM_max, int64_t sumN_max, uint64_t seed,
                                dcr_precision p, int32_t* r, int32_t* seg_status,
                                int32_t* dev_status, void* ws, size_t ws_bytes,
                                hipStream_t stream);

/* End to end with a chosen scheme (Sec. V): as dcr_resample, whose call is
 * dcr_resample_scheme(..., DCR_MULTINOMIAL, ...).  The workspace of
 * dcr_workspace_bytes(M, N, p) suffices for every scheme.  u_opt receives the
 * scheme's uniforms.  Errors: as dcr_resample; DCR_ERR_UNSUPPORTED for an
 * unknown scheme. */
dcr_status dcr_resample_scheme(const void* w, int64_t M, int64_t N, uint64_t seed,
                               uint64_t stream_id, dcr_precision p, dcr_scheme scheme, int32_t* r,
                               double* W_opt, double* u_opt, int32_t* dev_status, void* ws,
                               size_t ws_bytes, hipStream_t stream);

/* End to end on structured weights (the ensemble Gaussian mixture filter of
 * Sec. IV: particle i, likelihood component k): M = Na * P weights
 *   w_{i*P + k} = a[i] * b[k],   i < Na, k < P,
 * formed on the fly as binary64 products (exact for DCR_FP32_COMP, whose a and
 * b are binary32) and never read from memory.  Everything else is as
 * dcr_resample_scheme on the weight array w: the same W, u and r as that call
 * on the materialised products with the same precision form.
 *   a [Na], b [P]   device arrays of the precision's type, non-negative.
 *   ws              dcr_workspace_bytes(Na * P, N, p) bytes.
 * Errors: as dcr_resample_scheme; DCR_ERR_INVALID_ARGUMENT for Na < 1, P < 1,
 * Na * P > 2^31 - 1 or NULL a, b. */
dcr_status dcr_resample_outer(const void* a, int64_t Na, const void* b, int64_t P, int64_t N,
                              uint64_t seed, uint64_t stream_id, dcr_precision p,
                              dcr_scheme scheme, int32_t* r, double* W_opt, double* u_opt,
                              int32_t* dev_status, void* ws, size_t ws_bytes,
                              hipStream_t stream);

/* The uniforms of the stratified or systematic scheme alone:
 *   u        [N] binary64 out, non-decreasing, in (0, 1]; needs no workspace.
 * Errors: DCR_ERR_INVALID_ARGUMENT (N out of range, u NULL with N > 0),
 * DCR_ERR_UNSUPPORTED for DCR_MULTINOMIAL (use dcr_sorted_uniforms) or an
 * unknown scheme. */
dcr_status dcr_scheme_uniforms(int64_t N, uint64_t seed, uint64_t stream_id, dcr_scheme scheme,
                               double* u, hipStream_t stream);

/* dcr_resample_batched with a chosen map tile: `chunk` draws of one filter
 * per map workgroup, 256, 512 or 1024 (0: the default, 512).  The indices do
 * not depend on it; only the speed does.  Errors: as dcr_resample_batched;
 * DCR_ERR_UNSUPPORTED for another chunk. */
dcr_status dcr_resample_batched_ex(const void* w, const int64_t* w_off, const int64_t* n_off,
                                   int32_t B, int64_t sumM_max, int64_t sumN_max, uint64_t seed,
                                   dcr_precision p, int32_t chunk, int32_t* r,
                                   int32_t* seg_status, int32_t* dev_status, void* ws,
                                   size_t ws_bytes, hipStream_t stream);

/* Autotuner of the batched form: runs dcr_resample_batched_ex on the caller's
 * batch with each chunk size (one untimed and three timed calls each, with HIP
 * events on `stream`) and stores the fastest in *best_chunk (and its
 * milliseconds per call in *best_ms if not NULL).  If `cache_path` is not NULL,
 * a line "B sumM_max sumN_max precision chunk ms" of that file with the same
 * shape answers without timing (*best_ms = -1), and a new result is appended.
 * Arguments as dcr_resample_batched; r and ws are overwritten.  Unlike the
 * other calls this one waits for the stream. */
dcr_status dcr_batched_autotune(const void* w, const int64_t* w_off, const int64_t* n_off,
                                int32_t B, int64_t sumM_max, int64_t sumN_max, uint64_t seed,
                                dcr_precision p, int32_t* r, void* ws, size_t ws_bytes,
                                const char* cache_path, int32_t* best_chunk, float* best_ms,
                                hipStream_t stream);

/* Batched plans (the batched form above with its resources held between
 * calls): a plan owns a device workspace for up to B_max filters with at most
 * sumM_max weights and sumN_max draws in total, the map tile for that shape,
 * and a HIP graph of the four batched launches.  Filter b of a call is, as in
 * dcr_resample_batched, an independent problem of Sec. I-III with Philox
 * stream id b, resampled by Alg. 5 on its own weights.
 *
 * dcr_plan_create_batched: allocates the workspace (the only entry point
 *   besides dcr_plan_destroy that allocates or frees device memory) on the
 *   current device.  tune_cache: NULL, or the path of the autotuner's text
 *   cache; a line "B_max sumM_max sumN_max precision chunk ms" with the
 *   plan's shape sets the map tile, else it is the default (512) until
 *   dcr_plan_autotune.  *out receives the plan (NULL on error).
 *   Errors: those of dcr_batched_workspace_bytes; DCR_ERR_HIP if the
 *   allocation fails. */
typedef struct dcr_plan_s* dcr_plan;
dcr_status dcr_plan_create_batched(int32_t B_max, int64_t sumM_max, int64_t sumN_max,
                                   dcr_precision p, const char* tune_cache, dcr_plan* out);

/* dcr_plan_resample_batched: dcr_resample_batched with the plan's workspace and
 * map tile, launched as the plan's graph.  Arguments as dcr_resample_batched
 * with 1 <= B <= B_max and the plan's precision and capacities (offsets whose
 * totals exceed them give DCR_ERR_CAPACITY_EXCEEDED in *dev_status, as
 * there); the indices equal that call's bit for bit.  The first call builds
 * the graph; later calls write their arguments (pointers, B, seed) into its
 * kernel nodes and launch it, so pointers may change from call to call.  The
 * call is asynchronous on `stream`; it waits on the host only when the caller
 * is more than one call of this plan ahead of the device.  A plan serves one
 * caller at a time: calls on it must not overlap (different threads or
 * streams), and it must be used on the device it was created on
 * (DCR_ERR_INVALID_ARGUMENT otherwise). */
dcr_status dcr_plan_resample_batched(dcr_plan plan, const void* w, const int64_t* w_off,
                                     const int64_t* n_off, int32_t B, uint64_t seed, int32_t* r,
                                     int32_t* seg_status, int32_t* dev_status,
                                     hipStream_t stream);

/* dcr_plan_autotune: times the map tiles on the caller's batch
 * (dcr_batched_autotune with the plan's workspace; r is overwritten), keeps
 * the fastest in the plan and appends it to the plan's tune cache, if any.
 * Waits for the stream.  *best_ms (may be NULL) receives its milliseconds per
 * call.  dcr_plan_map_chunk reports the plan's current map tile. */
dcr_status dcr_plan_autotune(dcr_plan plan, const void* w, const int64_t* w_off,
                             const int64_t* n_off, int32_t B, uint64_t seed, int32_t* r,
                             float* best_ms, hipStream_t stream);
dcr_status dcr_plan_map_chunk(dcr_plan plan, int32_t* chunk);

/* dcr_plan_destroy: waits for the plan's launches, then frees its graph and
 * workspace.  DCR_ERR_INVALID_ARGUMENT for NULL. */
dcr_status dcr_plan_destroy(dcr_plan plan);

/* Allocation-free end to end, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): dcr_resample_scheme without the workspace argument.  Its scratch
 * space is a static device array of DCR_NOALLOC_SCRATCH_BYTES held by every
 * GPU the library runs on until the process ends; the call itself allocates
 * nothing.  The caller still owns w, r and the optional W_opt, u_opt and
 * dev_status, with the meaning of dcr_resample_scheme, and the results equal
 * that call's bit for bit.
 *   Limit: the workspace dcr_workspace_bytes(M, N, p) would need must fit the
 *   array (for example M = 2^27 with N = 2^20, or M = N = 2^21); otherwise
 *   DCR_ERR_CAPACITY_EXCEEDED is returned before anything is enqueued.
 *   Sharing: every call on one GPU uses that GPU's one array, so calls that
 *   overlap on a GPU (concurrent streams, or threads) race and must be
 *   serialised by the caller; calls in order on one stream are safe.  Nothing
 *   in the array needs to start at zero: a call writes every word it reads.
 * Errors: those of dcr_resample_scheme (except the workspace ones), plus
 * DCR_ERR_CAPACITY_EXCEEDED, and DCR_ERR_HIP if the array's device address
 * cannot be obtained on the current device. */
#define DCR_NOALLOC_SCRATCH_BYTES (32u << 20)
dcr_status dcr_resample_noalloc(const void* w, int64_t M, int64_t N, uint64_t seed,
                                uint64_t stream_id, dcr_precision p, dcr_scheme scheme,
                                int32_t* r, double* W_opt, double* u_opt, int32_t* dev_status,
                                hipStream_t stream);

/* Kernel timing for measurement (not part of the sampling contract).
 * dcr_profile_begin(cap) creates HIP events for up to `cap` kernel launches;
 * every later launch records its own start and end into the next pair
 * (hipExtLaunchKernel), so an interval covers the kernel alone.
 * dcr_profile_end() waits for the device, stops recording and, for each
 * kernel kind k (see dcr_profile_kind_name), stores
 * the launch count in counts[k] and the summed milliseconds in ms[k]
 * (arrays of n_kinds entries, host memory).  Kinds beyond n_kinds are dropped.
 * Profiling is per host thread: it records the launches made by the thread that
 * called dcr_profile_begin, and other threads' calls are neither recorded nor
 * affected. */
dcr_status dcr_profile_begin(int32_t cap);
dcr_status dcr_profile_end(int32_t n_kinds, int64_t* counts, double* ms);
int32_t dcr_profile_kind_count(void);
const char* dcr_profile_kind_name(int32_t kind);

/* Bandwidth reference for measurement (not part of the sampling contract):
 * kind 0 streams `bytes` from src (coalesced 16-byte loads, `unroll` = 4, 8
 * or 16 in flight per thread, grid-stride) and writes one float partial sum
 * per workgroup to dst (grid floats); kind 2 does the same with one contiguous
 * run of src per workgroup and non-temporal loads (the access pattern of the
 * weight stream); kind 1 copies `bytes` from src to dst.  `grid`
 * workgroups of 256 threads.  src and dst 16-byte aligned, bytes a positive
 * multiple of 16; otherwise DCR_ERR_INVALID_ARGUMENT.  Asynchronous on
 * `stream`. */
dcr_status dcr_stream_probe(int32_t kind, int32_t unroll, const void* src, void* dst,
                            size_t bytes, int32_t grid, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* DCR_H */
