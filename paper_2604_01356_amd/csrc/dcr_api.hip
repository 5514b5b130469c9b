// dcr_api.hip -- host side of the libdcr C ABI (declared in include/dcr.h):
// argument validation, workspace layout and kernel enqueueing.  Nothing here
// allocates device memory; scratch space is the caller's workspace, or for
// dcr_resample_noalloc a static device array.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "dcr.h"
#include "dcr_internal.hpp"
#include "dcr_launch.hpp"

namespace dcr {
thread_local LaunchEvents g_launch_events;
}

namespace {

using dcr::SharedArgs;
using dcr::WArgs;
using dcr::ZArgs;

constexpr int64_t kMaxM = 2147483647LL;   // r is int32
constexpr int64_t kMaxN = 2147483646LL;   // N + 1 draws must stay below 2^31
constexpr int64_t kWBlock = 32768;
constexpr int64_t kWSubPerBlock = 128;
constexpr int64_t kZBlock = 4096;
constexpr int64_t kDenseMinPerWG = 256;   // fewest uniforms per workgroup of the dense map

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

struct Layout {
    int64_t nwb = 0, nzb = 0;
    size_t status = 0, totals = 0;
    size_t w_tot = 0, w_beta = 0, w_sub = 0;
    size_t z_tot = 0, z_beta = 0, z_buf = 0;
    size_t span = 0;
    size_t bytes = 0;
};

// Workspace layout: [header][weight side][spacing side][dense-map chunk spans];
// the stratified and systematic schemes have no spacing side.
Layout make_layout(int64_t M, int64_t N, int scheme = dcr::kSchemeMultinomial) {
    Layout L;
    size_t off = 0;
    L.status = off;
    off += 256;
    L.totals = off;
    off += 256;
    if (M > 0) {
        L.nwb = (M + kWBlock - 1) / kWBlock;
        L.w_tot = off;
        off = align256(off + sizeof(double) * L.nwb);
        L.w_beta = off;
        off = align256(off + sizeof(double) * L.nwb);
        L.w_sub = off;
        off = align256(off + sizeof(double) * L.nwb * kWSubPerBlock);
    }
    if (N > 0 && scheme == dcr::kSchemeMultinomial) {
        L.nzb = (N + 1 + kZBlock - 1) / kZBlock;
        L.z_tot = off;
        off = align256(off + sizeof(double) * L.nzb);
        L.z_beta = off;
        off = align256(off + sizeof(double) * L.nzb);
        L.z_buf = off;
        off = align256(off + sizeof(double) * L.nzb * kZBlock);
    }
    if (N > 0) {
        const size_t chunks = (N + kDenseMinPerWG - 1) / kDenseMinPerWG;
        L.span = off;
        off = align256(off + 2 * sizeof(int64_t) * chunks);
    }
    L.bytes = off;
    return L;
}

template <typename T>
T* at(void* ws, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

bool valid_prec(dcr_precision p) { return p == DCR_FP64 || p == DCR_FP32_COMP; }
int prec_code(dcr_precision p) { return p == DCR_FP32_COMP ? dcr::kPrecFP32 : dcr::kPrecFP64; }
bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

WArgs w_args(const Layout& L, void* ws, int64_t M) {
    WArgs a{};
    a.M = M;
    a.nb = L.nwb;
    a.blk_tot = at<double>(ws, L.w_tot);
    a.beta = at<double>(ws, L.w_beta);
    a.sub_end = at<double>(ws, L.w_sub);
    return a;
}

ZArgs z_args(const Layout& L, void* ws, int64_t N, uint64_t seed, uint64_t stream,
             int scheme = dcr::kSchemeMultinomial) {
    ZArgs a{};
    a.N = N;
    a.nb = L.nzb;
    a.seed = seed;
    a.stream = stream;
    a.scheme = scheme;
    a.zrel = at<double>(ws, L.z_buf);
    a.blk_tot = at<double>(ws, L.z_tot);
    a.beta = at<double>(ws, L.z_beta);
    return a;
}

SharedArgs shared_args(const Layout& L, void* ws) {
    SharedArgs s{};
    s.status = at<int32_t>(ws, L.status);
    s.totals = at<double>(ws, L.totals);
    return s;
}

// ---------------------------------------------------------------------------
// Optional kernel timing (dcr_profile_*).
// ---------------------------------------------------------------------------
enum Kind {
    kKReduce = 0, kKCarries, kKMatW, kKMatU, kKMapFused, kKMapW, kKFinish, kKMapDense, kKMapSpan,
    kKBatchPlan, kKBatchReduce, kKBatchCarries, kKBatchMap, kNumKinds
};
const char* const kKindNames[kNumKinds] = {"reduce",   "carries", "materialize_w", "materialize_u",
                                           "map_fused", "map_w",  "finish",        "map_dense",
                                           "map_span",  "batch_plan", "batch_reduce",
                                           "batch_carries", "batch_map"};

struct Profiler {
    bool on = false;
    int cap = 0;
    int used = 0;
    std::vector<hipEvent_t> ev;
    std::vector<int> kind;
};
thread_local Profiler g_prof;   // each host thread profiles its own launches

// Runs one launcher; while profiling, its kernel records its own start and
// end into the next pair of events (a launcher that launches nothing, e.g. for
// N = 0, uses no slot).
template <class F>
hipError_t timed(int kind, hipStream_t s, F&& launch) {
    (void)s;
    if (!g_prof.on || g_prof.used >= g_prof.cap) return launch();
    const int slot = g_prof.used;
    dcr::g_launch_events.start = g_prof.ev[2 * slot];
    dcr::g_launch_events.stop = g_prof.ev[2 * slot + 1];
    const int64_t before = dcr::g_launch_events.launches;
    const hipError_t e = launch();
    dcr::g_launch_events.start = nullptr;
    dcr::g_launch_events.stop = nullptr;
    if (dcr::g_launch_events.launches != before) {
        g_prof.kind[slot] = kind;
        ++g_prof.used;
    }
    return e;
}

dcr_status hip_status(hipError_t e) { return e == hipSuccess ? DCR_OK : DCR_ERR_HIP; }

}  // namespace

// ---------------------------------------------------------------------------
// Batched form
// ---------------------------------------------------------------------------
namespace {

constexpr int64_t kMaxBatch = 1 << 24;
constexpr int64_t kMaxSum = 1LL << 40;
constexpr int kMinChunk = 256;
constexpr int kChunks[3] = {256, 512, 1024};   // draws per map workgroup the library is built for

struct BatchLayout {
    int64_t wt_cap = 0, zt_cap = 0, mc_cap = 0;
    size_t head = 0, wt_base = 0, zt_base = 0, mc_base = 0, mc_seg = 0, seg_status = 0,
           seg_totals = 0;
    size_t wt_tot = 0, wt_beta = 0, wt_sub = 0, wt_chunk = 0, zt_tot = 0, zt_beta = 0, zrel = 0;
    size_t bytes = 0;
};

BatchLayout make_batch_layout(int64_t B, int64_t sumM, int64_t sumN) {
    BatchLayout L;
    L.wt_cap = (sumM + dcr::kBatchWBlock - 1) / dcr::kBatchWBlock + B;
    L.zt_cap = (sumN + B + dcr::kBatchZBlock - 1) / dcr::kBatchZBlock + B;
    L.mc_cap = (sumN + kMinChunk - 1) / kMinChunk + B;   // the most map workgroups of any chunk
    size_t off = 0;
    auto take = [&](size_t n) {
        const size_t at_ = off;
        off = align256(off + n);
        return at_;
    };
    L.head = take(256);
    L.wt_base = take(sizeof(int64_t) * (B + 1));
    L.zt_base = take(sizeof(int64_t) * (B + 1));
    L.mc_base = take(sizeof(int64_t) * (B + 1));
    L.mc_seg = take(sizeof(int32_t) * L.mc_cap);
    L.seg_status = take(sizeof(int32_t) * B);
    L.seg_totals = take(sizeof(double) * 2 * B);
    L.wt_tot = take(sizeof(double) * L.wt_cap);
    L.wt_beta = take(sizeof(double) * L.wt_cap);
    L.wt_sub = take(sizeof(double) * L.wt_cap * kWSubPerBlock);
    L.wt_chunk = take(sizeof(double) * L.wt_cap * kWSubPerBlock * 16);
    L.zt_tot = take(sizeof(double) * L.zt_cap);
    L.zt_beta = take(sizeof(double) * L.zt_cap);
    L.zrel = take(sizeof(double) * (sumN + B));
    L.bytes = off;
    return L;
}

// Argument block of the batched launches.  The layout is sized for B_layout
// filters (B itself for a stateless call, a plan's B_max), of which the call
// uses B.
dcr::BatchArgs batch_args(const BatchLayout& L, void* ws, const int64_t* w_off,
                          const int64_t* n_off, int32_t B, int64_t B_layout, int32_t chunk,
                          uint64_t seed, int64_t sumM_max, int64_t sumN_max,
                          int32_t* seg_status) {
    dcr::BatchArgs ba{};
    ba.w_off = w_off;
    ba.n_off = n_off;
    ba.B = B;
    ba.chunk = chunk;
    ba.seed = seed;
    ba.wt_cap = L.wt_cap;
    ba.zt_cap = L.zt_cap;
    ba.mc_cap = (sumN_max + chunk - 1) / chunk + B_layout;
    ba.sumM_cap = sumM_max;
    ba.sumN_cap = sumN_max;
    ba.wt_base = at<int64_t>(ws, L.wt_base);
    ba.zt_base = at<int64_t>(ws, L.zt_base);
    ba.mc_base = at<int64_t>(ws, L.mc_base);
    ba.mc_seg = at<int32_t>(ws, L.mc_seg);
    ba.head = at<int32_t>(ws, L.head);
    ba.wt_tot = at<double>(ws, L.wt_tot);
    ba.wt_beta = at<double>(ws, L.wt_beta);
    ba.wt_sub = at<double>(ws, L.wt_sub);
    ba.wt_chunk = at<double>(ws, L.wt_chunk);
    ba.zt_tot = at<double>(ws, L.zt_tot);
    ba.zt_beta = at<double>(ws, L.zt_beta);
    ba.zrel = at<double>(ws, L.zrel);
    ba.seg_status = seg_status ? seg_status : at<int32_t>(ws, L.seg_status);
    ba.seg_totals = at<double>(ws, L.seg_totals);
    return ba;
}

bool batch_sizes_ok(int64_t B, int64_t sumM, int64_t sumN) {
    if (B < 1 || B > kMaxBatch || sumM < B || sumM > kMaxSum || sumN < 0 || sumN > kMaxSum)
        return false;
    const BatchLayout L = make_batch_layout(B, sumM, sumN);
    return L.wt_cap + L.zt_cap <= 0x7FFFFFFF && L.mc_cap <= 0x7FFFFFFF;
}

}  // namespace

// ---------------------------------------------------------------------------
// Autotuner for the batched map: times each built chunk size on the caller's
// batch and keeps the fastest, optionally cached in a text file of lines
// "B sumM sumN precision chunk milliseconds".
// ---------------------------------------------------------------------------
namespace {

bool cache_lookup(const char* path, int64_t B, int64_t sumM, int64_t sumN, int p, int32_t* chunk) {
    if (!path) return false;
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    long long b, m, n;
    int pp, c;
    double ms;
    bool found = false;
    while (std::fscanf(f, "%lld %lld %lld %d %d %lf", &b, &m, &n, &pp, &c, &ms) == 6) {
        if (b == B && m == sumM && n == sumN && pp == p &&
            (c == 256 || c == 512 || c == 1024)) {
            *chunk = c;   // the last entry for the key wins
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const char* path, int64_t B, int64_t sumM, int64_t sumN, int p, int32_t chunk,
                 float ms) {
    if (!path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%lld %lld %lld %d %d %.6f\n", static_cast<long long>(B),
                 static_cast<long long>(sumM), static_cast<long long>(sumN), p, chunk, ms);
    std::fclose(f);
}

}  // namespace

namespace {
dcr_status resample_from(const dcr::WSource& src, int64_t M, int64_t N, uint64_t seed,
                         uint64_t stream_id, dcr_precision p, dcr_scheme scheme, int32_t* r,
                         double* W_opt, double* u_opt, int32_t* dev_status, void* ws,
                         size_t ws_bytes, hipStream_t stream);
bool valid_scheme(dcr_scheme s);
}  // namespace

extern "C" {

const char* dcr_status_string(dcr_status s) {
    switch (s) {
        case DCR_OK: return "ok";
        case DCR_ERR_INVALID_ARGUMENT: return "invalid argument";
        case DCR_ERR_UNSUPPORTED: return "unsupported precision or option";
        case DCR_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
        case DCR_ERR_CAPACITY_EXCEEDED: return "capacity exceeded";
        case DCR_ERR_HIP: return "HIP runtime error";
        case DCR_ERR_BAD_WEIGHTS: return "bad weights (negative, NaN, infinite or zero total)";
        case DCR_ERR_INTERNAL: return "internal error";
    }
    return "unknown status";
}

dcr_status dcr_workspace_bytes(int64_t M, int64_t N, dcr_precision p, size_t* bytes) {
    if (!bytes || M < 1 || M > kMaxM || N < 0 || N > kMaxN) return DCR_ERR_INVALID_ARGUMENT;
    if (!valid_prec(p)) return DCR_ERR_UNSUPPORTED;
    *bytes = make_layout(M, N).bytes;
    return DCR_OK;
}

dcr_status dcr_cumulative_weights(const void* w, int64_t M, dcr_precision p, double* W,
                                  double* total, int32_t* dev_status, void* ws, size_t ws_bytes,
                                  hipStream_t stream) {
    if (M < 1 || M > kMaxM || !w || !W || !ws) return DCR_ERR_INVALID_ARGUMENT;
    if (!valid_prec(p)) return DCR_ERR_UNSUPPORTED;
    if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0) return DCR_ERR_INVALID_ARGUMENT;
    const Layout L = make_layout(M, 0);
    if (ws_bytes < L.bytes) return DCR_ERR_WORKSPACE_TOO_SMALL;
    const WArgs wa = w_args(L, ws, M);
    ZArgs za{};
    const SharedArgs sh = shared_args(L, ws);
    const int prec = prec_code(p);
    const int vec = (aligned16(w) ? 1 : 0) | (aligned16(W) ? 2 : 0);
    dcr::WSource src;
    src.w = w;
    hipError_t e = timed(kKReduce, stream, [&] { return dcr::launch_reduce(prec, src, wa, za, vec, stream); });
    if (e == hipSuccess)
        e = timed(kKCarries, stream,
                  [&] { return dcr::launch_carries(wa, za, sh, dev_status, total, stream); });
    if (e == hipSuccess)
        e = timed(kKMatW, stream,
                  [&] { return dcr::launch_materialize_w(prec, src, wa, sh, W, vec, stream); });
    return hip_status(e);
}

dcr_status dcr_sorted_uniforms(int64_t N, uint64_t seed, uint64_t stream_id, dcr_precision p,
                               double* u, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (N < 0 || N > kMaxN) return DCR_ERR_INVALID_ARGUMENT;
    if (!valid_prec(p)) return DCR_ERR_UNSUPPORTED;
    if (N == 0) return DCR_OK;
    if (!u || !ws || (reinterpret_cast<uintptr_t>(ws) & 255u) != 0) return DCR_ERR_INVALID_ARGUMENT;
    const Layout L = make_layout(0, N);
    if (ws_bytes < L.bytes) return DCR_ERR_WORKSPACE_TOO_SMALL;
    WArgs wa{};
    const ZArgs za = z_args(L, ws, N, seed, stream_id);
    const SharedArgs sh = shared_args(L, ws);
    const int prec = prec_code(p);
    hipError_t e = timed(kKReduce, stream,
                         [&] { return dcr::launch_reduce(prec, dcr::WSource{}, wa, za, 0, stream); });
    if (e == hipSuccess)
        e = timed(kKCarries, stream,
                  [&] { return dcr::launch_carries(wa, za, sh, nullptr, nullptr, stream); });
    if (e == hipSuccess)
        e = timed(kKMatU, stream, [&] { return dcr::launch_materialize_u(za, sh, u, stream); });
    return hip_status(e);
}

dcr_status dcr_inverse_cmf(const double* W, int64_t M, const double* u, int64_t N, int32_t* r,
                           void* ws, size_t ws_bytes, hipStream_t stream) {
    (void)ws;
    (void)ws_bytes;
    if (M < 1 || M > kMaxM || N < 0 || N > kMaxN) return DCR_ERR_INVALID_ARGUMENT;
    if (N == 0) return DCR_OK;
    if (!W || !u || !r) return DCR_ERR_INVALID_ARGUMENT;
    const hipError_t e =
        timed(kKMapW, stream, [&] { return dcr::launch_map_w(W, M, u, N, r, stream); });
    return hip_status(e);
}

}  // extern "C"

namespace {
bool valid_scheme(dcr_scheme s) {
    return s == DCR_MULTINOMIAL || s == DCR_STRATIFIED || s == DCR_SYSTEMATIC;
}
}  // namespace

extern "C" {

dcr_status dcr_scheme_uniforms(int64_t N, uint64_t seed, uint64_t stream_id, dcr_scheme scheme,
                               double* u, hipStream_t stream) {
    if (N < 0 || N > kMaxN) return DCR_ERR_INVALID_ARGUMENT;
    if (scheme != DCR_STRATIFIED && scheme != DCR_SYSTEMATIC) return DCR_ERR_UNSUPPORTED;
    if (N == 0) return DCR_OK;
    if (!u) return DCR_ERR_INVALID_ARGUMENT;
    const Layout L = make_layout(0, N, scheme);
    const ZArgs za = z_args(L, nullptr, N, seed, stream_id, scheme);
    const SharedArgs sh{};
    const hipError_t e =
        timed(kKMatU, stream, [&] { return dcr::launch_materialize_u(za, sh, u, stream); });
    return hip_status(e);
}

dcr_status dcr_resample(const void* w, int64_t M, int64_t N, uint64_t seed, uint64_t stream_id,
                        dcr_precision p, int32_t* r, double* W_opt, double* u_opt,
                        int32_t* dev_status, void* ws, size_t ws_bytes, hipStream_t stream) {
    return dcr_resample_scheme(w, M, N, seed, stream_id, p, DCR_MULTINOMIAL, r, W_opt, u_opt,
                               dev_status, ws, ws_bytes, stream);
}

dcr_status dcr_resample_scheme(const void* w, int64_t M, int64_t N, uint64_t seed,
                               uint64_t stream_id, dcr_precision p, dcr_scheme scheme, int32_t* r,
                               double* W_opt, double* u_opt, int32_t* dev_status, void* ws,
                               size_t ws_bytes, hipStream_t stream) {
    if (!w) return DCR_ERR_INVALID_ARGUMENT;
    dcr::WSource src;
    src.w = w;
    return resample_from(src, M, N, seed, stream_id, p, scheme, r, W_opt, u_opt, dev_status, ws,
                         ws_bytes, stream);
}

dcr_status dcr_resample_outer(const void* a, int64_t Na, const void* b, int64_t P, int64_t N,
                              uint64_t seed, uint64_t stream_id, dcr_precision p,
                              dcr_scheme scheme, int32_t* r, double* W_opt, double* u_opt,
                              int32_t* dev_status, void* ws, size_t ws_bytes,
                              hipStream_t stream) {
    if (!a || !b || Na < 1 || P < 1 || Na > kMaxM / P) return DCR_ERR_INVALID_ARGUMENT;
    dcr::WSource src;
    src.a = a;
    src.b = b;
    src.P = P;
    return resample_from(src, Na * P, N, seed, stream_id, p, scheme, r, W_opt, u_opt, dev_status,
                         ws, ws_bytes, stream);
}

}  // extern "C"

namespace {

dcr_status resample_from(const dcr::WSource& src, int64_t M, int64_t N, uint64_t seed,
                         uint64_t stream_id, dcr_precision p, dcr_scheme scheme, int32_t* r,
                         double* W_opt, double* u_opt, int32_t* dev_status, void* ws,
                         size_t ws_bytes, hipStream_t stream) {
    if (M < 1 || M > kMaxM || N < 0 || N > kMaxN || !ws) return DCR_ERR_INVALID_ARGUMENT;
    if (N > 0 && !r) return DCR_ERR_INVALID_ARGUMENT;
    if (!valid_prec(p) || !valid_scheme(scheme)) return DCR_ERR_UNSUPPORTED;
    if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0) return DCR_ERR_INVALID_ARGUMENT;
    const Layout L = make_layout(M, N, scheme);
    if (ws_bytes < L.bytes) return DCR_ERR_WORKSPACE_TOO_SMALL;
    const WArgs wa = w_args(L, ws, M);
    const ZArgs za = z_args(L, ws, N, seed, stream_id, scheme);
    const SharedArgs sh = shared_args(L, ws);
    const int prec = prec_code(p);
    // an outer product has no alignment to honour
    const int vec = ((src.outer() || aligned16(src.w)) ? 1 : 0) | (aligned16(W_opt) ? 2 : 0);
    int64_t* span = at<int64_t>(ws, L.span);
    // a few weight blocks: 1024 threads per block, the same sums
    hipError_t e = timed(kKReduce, stream, [&] {
        return dcr::small_fits(wa, za) ? dcr::launch_reduce_small(prec, src, wa, za, stream)
                                       : dcr::launch_reduce(prec, src, wa, za, vec, stream);
    });
    if (dcr::finish_fits(wa, za)) {
        // block scans, uniforms and map in one launch
        if (e == hipSuccess)
            e = timed(kKFinish, stream, [&] {
                return dcr::launch_finish(prec, src, wa, za, sh, dev_status, u_opt, r, vec, stream);
            });
        if (e == hipSuccess && W_opt)
            e = timed(kKMatW, stream,
                      [&] { return dcr::launch_materialize_w(prec, src, wa, sh, W_opt, vec, stream); });
        return hip_status(e);
    }
    if (e == hipSuccess)
        e = timed(kKCarries, stream,
                  [&] { return dcr::launch_carries(wa, za, sh, dev_status, nullptr, stream); });
    if (e == hipSuccess && W_opt)
        e = timed(kKMatW, stream,
                  [&] { return dcr::launch_materialize_w(prec, src, wa, sh, W_opt, vec, stream); });
    if (e == hipSuccess && N > 0) {
        if (dcr::map_is_dense(M, N)) {
            e = timed(kKMapSpan, stream,
                      [&] { return dcr::launch_dense_span(wa, za, sh, span, stream); });
            if (e == hipSuccess)
                e = timed(kKMapDense, stream, [&] {
                    return dcr::launch_map_dense(prec, src, wa, za, sh, span, u_opt, r, vec, stream);
                });
        } else
            e = timed(kKMapFused, stream, [&] {
                return dcr::launch_map_fused(prec, src, wa, za, sh, u_opt, r, vec, stream);
            });
    }
    return hip_status(e);
}

}  // namespace

extern "C" {


dcr_status dcr_batched_workspace_bytes(int32_t B, int64_t sumM_max, int64_t sumN_max,
                                       dcr_precision p, size_t* bytes) {
    if (!bytes || !batch_sizes_ok(B, sumM_max, sumN_max)) return DCR_ERR_INVALID_ARGUMENT;
    if (!valid_prec(p)) return DCR_ERR_UNSUPPORTED;
    *bytes = make_batch_layout(B, sumM_max, sumN_max).bytes;
    return DCR_OK;
}

dcr_status dcr_resample_batched(const void* w, const int64_t* w_off, const int64_t* n_off,
                                int32_t B, int64_t sumM_max, int64_t sumN_max, uint64_t seed,
                                dcr_precision p, int32_t* r, int32_t* seg_status,
                                int32_t* dev_status, void* ws, size_t ws_bytes,
                                hipStream_t stream) {
    return dcr_resample_batched_ex(w, w_off, n_off, B, sumM_max, sumN_max, seed, p, 0, r,
                                   seg_status, dev_status, ws, ws_bytes, stream);
}

dcr_status dcr_resample_batched_ex(const void* w, const int64_t* w_off, const int64_t* n_off,
                                   int32_t B, int64_t sumM_max, int64_t sumN_max, uint64_t seed,
                                   dcr_precision p, int32_t chunk, int32_t* r,
                                   int32_t* seg_status, int32_t* dev_status, void* ws,
                                   size_t ws_bytes, hipStream_t stream) {
    if (chunk == 0) chunk = dcr::kBatchChunkDefault;
    if (chunk != 256 && chunk != 512 && chunk != 1024) return DCR_ERR_UNSUPPORTED;
    if (!batch_sizes_ok(B, sumM_max, sumN_max)) return DCR_ERR_INVALID_ARGUMENT;
    if (!w || !w_off || !n_off || !ws || (sumN_max > 0 && !r)) return DCR_ERR_INVALID_ARGUMENT;
    if (!valid_prec(p)) return DCR_ERR_UNSUPPORTED;
    if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0) return DCR_ERR_INVALID_ARGUMENT;
    const BatchLayout L = make_batch_layout(B, sumM_max, sumN_max);
    if (ws_bytes < L.bytes) return DCR_ERR_WORKSPACE_TOO_SMALL;
    const dcr::BatchArgs ba =
        batch_args(L, ws, w_off, n_off, B, B, chunk, seed, sumM_max, sumN_max, seg_status);
    const int prec = prec_code(p);
    hipError_t e = timed(kKBatchPlan, stream, [&] { return dcr::launch_batch_plan(ba, dev_status, stream); });
    if (e == hipSuccess)
        e = timed(kKBatchReduce, stream,
                  [&] { return dcr::launch_reduce_batched(prec, w, ba, stream); });
    if (e == hipSuccess)
        e = timed(kKBatchCarries, stream, [&] { return dcr::launch_carries_batched(ba, stream); });
    if (e == hipSuccess)
        e = timed(kKBatchMap, stream,
                  [&] { return dcr::launch_map_batched(prec, w, ba, r, dev_status, stream); });
    return hip_status(e);
}


dcr_status dcr_batched_autotune(const void* w, const int64_t* w_off, const int64_t* n_off,
                                int32_t B, int64_t sumM_max, int64_t sumN_max, uint64_t seed,
                                dcr_precision p, int32_t* r, void* ws, size_t ws_bytes,
                                const char* cache_path, int32_t* best_chunk, float* best_ms,
                                hipStream_t stream) {
    if (!best_chunk) return DCR_ERR_INVALID_ARGUMENT;
    if (cache_lookup(cache_path, B, sumM_max, sumN_max, static_cast<int>(p), best_chunk)) {
        if (best_ms) *best_ms = -1.0f;
        return DCR_OK;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return DCR_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return DCR_ERR_HIP;
    }
    dcr_status st = DCR_OK;
    float best = -1.0f;
    int32_t pick = dcr::kBatchChunkDefault;
    constexpr int kReps = 3;
    for (int c : kChunks) {
        // one untimed call (also reports argument errors), then kReps timed
        st = dcr_resample_batched_ex(w, w_off, n_off, B, sumM_max, sumN_max, seed, p, c, r,
                                     nullptr, nullptr, ws, ws_bytes, stream);
        if (st != DCR_OK) break;
        if (hipEventRecord(e0, stream) != hipSuccess) { st = DCR_ERR_HIP; break; }
        for (int k = 0; k < kReps && st == DCR_OK; ++k)
            st = dcr_resample_batched_ex(w, w_off, n_off, B, sumM_max, sumN_max, seed, p, c, r,
                                         nullptr, nullptr, ws, ws_bytes, stream);
        if (st != DCR_OK) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            st = DCR_ERR_HIP;
            break;
        }
        ms /= kReps;
        if (best < 0.0f || ms < best) {
            best = ms;
            pick = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != DCR_OK) return st;
    *best_chunk = pick;
    if (best_ms) *best_ms = best;
    cache_store(cache_path, B, sumM_max, sumN_max, static_cast<int>(p), pick, best);
    return DCR_OK;
}

dcr_status dcr_profile_begin(int32_t cap) {
    if (cap < 1 || g_prof.on) return DCR_ERR_INVALID_ARGUMENT;
    g_prof.ev.assign(2 * static_cast<size_t>(cap), nullptr);
    g_prof.kind.assign(cap, -1);
    for (auto& ev : g_prof.ev) {
        if (hipEventCreateWithFlags(&ev, hipEventDisableSystemFence) != hipSuccess) {
            ev = nullptr;
            for (auto& made : g_prof.ev)   // release what was created
                if (made) (void)hipEventDestroy(made);
            g_prof.ev.clear();
            g_prof.kind.clear();
            return DCR_ERR_HIP;
        }
    }
    g_prof.cap = cap;
    g_prof.used = 0;
    g_prof.on = true;
    return DCR_OK;
}

dcr_status dcr_profile_end(int32_t n_kinds, int64_t* counts, double* ms) {
    if (!g_prof.on) return DCR_ERR_INVALID_ARGUMENT;
    g_prof.on = false;
    dcr_status st = DCR_OK;
    for (int k = 0; k < n_kinds; ++k) {
        if (counts) counts[k] = 0;
        if (ms) ms[k] = 0.0;
    }
    // the events carry no memory fence; a device-wide wait orders the reads
    if (g_prof.used > 0 && hipDeviceSynchronize() != hipSuccess) st = DCR_ERR_HIP;
    for (int i = 0; i < g_prof.used && st == DCR_OK; ++i) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, g_prof.ev[2 * i], g_prof.ev[2 * i + 1]) != hipSuccess) {
            st = DCR_ERR_HIP;
            break;
        }
        const int k = g_prof.kind[i];
        if (k >= 0 && k < n_kinds) {
            if (counts) counts[k] += 1;
            if (ms) ms[k] += t;
        }
    }
    for (auto& ev : g_prof.ev)
        if (ev) (void)hipEventDestroy(ev);
    g_prof.ev.clear();
    g_prof.kind.clear();
    g_prof.used = 0;
    g_prof.cap = 0;
    return st;
}

dcr_status dcr_stream_probe(int32_t kind, int32_t unroll, const void* src, void* dst,
                            size_t bytes, int32_t grid, hipStream_t stream) {
    if (kind < 0 || kind > 2 || !src || !dst || bytes == 0 || (bytes & 15) != 0 || grid < 1)
        return DCR_ERR_INVALID_ARGUMENT;
    if (unroll != 4 && unroll != 8 && unroll != 16) return DCR_ERR_INVALID_ARGUMENT;
    if (((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15) != 0)
        return DCR_ERR_INVALID_ARGUMENT;
    return hip_status(dcr::launch_stream_probe(kind, unroll, src, dst,
                                               static_cast<int64_t>(bytes / 16), grid, stream));
}

int32_t dcr_profile_kind_count(void) { return kNumKinds; }

const char* dcr_profile_kind_name(int32_t kind) {
    return (kind >= 0 && kind < kNumKinds) ? kKindNames[kind] : "";
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched plans: a device workspace sized once, the map tile from the tune
// cache (or the autotuner), and a HIP graph of the four batched launches built
// node by node.  Each call writes its arguments (pointers, B, seed) into the
// kernel nodes of an instantiated graph and launches it.  Two instances
// alternate, each with an event recorded after its last launch: before an
// instance's nodes are rewritten, the event is waited on, so a launch still
// in flight never sees the next call's arguments (a wait happens only when a
// caller runs more than one call ahead of the device).
// ---------------------------------------------------------------------------
struct dcr_plan_s {
    int32_t B_max = 0;
    int64_t sumM_max = 0, sumN_max = 0;
    dcr_precision p = DCR_FP64;
    int32_t chunk = dcr::kBatchChunkDefault;
    int device = -1;
    std::string cache_path;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    struct Instance {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipGraphNode_t nodes[4] = {};
        hipEvent_t done = nullptr;
        int32_t chunk = 0;   // the map tile the graph was built for
        bool launched = false;
    };
    Instance inst[2];
    int next = 0;
};

namespace {

void release_instance(dcr_plan_s::Instance& in) {
    if (in.exec) (void)hipGraphExecDestroy(in.exec);
    if (in.graph) (void)hipGraphDestroy(in.graph);
    if (in.done) (void)hipEventDestroy(in.done);
    in = dcr_plan_s::Instance{};
}

// Builds (or rebuilds, after a change of map tile) an instance's graph from
// the call's arguments.
dcr_status build_instance(dcr_plan_s& pl, dcr_plan_s::Instance& in, dcr::BatchNodeArgs& a) {
    release_instance(in);
    hipKernelNodeParams kp[4];
    if (dcr::batched_node_params(prec_code(pl.p), a, pl.B_max, kp) != hipSuccess)
        return DCR_ERR_INTERNAL;
    if (hipEventCreateWithFlags(&in.done, hipEventDisableTiming) != hipSuccess ||
        hipGraphCreate(&in.graph, 0) != hipSuccess) {
        release_instance(in);
        return DCR_ERR_HIP;
    }
    for (int k = 0; k < 4; ++k) {
        const hipGraphNode_t* dep = (k == 0) ? nullptr : &in.nodes[k - 1];
        if (hipGraphAddKernelNode(&in.nodes[k], in.graph, dep, k == 0 ? 0 : 1, &kp[k]) !=
            hipSuccess) {
            release_instance(in);
            return DCR_ERR_HIP;
        }
    }
    if (hipGraphInstantiate(&in.exec, in.graph, nullptr, nullptr, 0) != hipSuccess) {
        release_instance(in);
        return DCR_ERR_HIP;
    }
    in.chunk = a.ba.chunk;
    return DCR_OK;
}

}  // namespace

extern "C" {

dcr_status dcr_plan_create_batched(int32_t B_max, int64_t sumM_max, int64_t sumN_max,
                                   dcr_precision p, const char* tune_cache, dcr_plan* out) {
    if (!out) return DCR_ERR_INVALID_ARGUMENT;
    *out = nullptr;
    if (!batch_sizes_ok(B_max, sumM_max, sumN_max)) return DCR_ERR_INVALID_ARGUMENT;
    if (!valid_prec(p)) return DCR_ERR_UNSUPPORTED;
    dcr_plan_s* pl = new (std::nothrow) dcr_plan_s();
    if (!pl) return DCR_ERR_INTERNAL;
    pl->B_max = B_max;
    pl->sumM_max = sumM_max;
    pl->sumN_max = sumN_max;
    pl->p = p;
    if (tune_cache) pl->cache_path = tune_cache;
    int32_t cached = 0;
    if (cache_lookup(tune_cache, B_max, sumM_max, sumN_max, static_cast<int>(p), &cached))
        pl->chunk = cached;
    pl->ws_bytes = make_batch_layout(B_max, sumM_max, sumN_max).bytes;
    if (hipGetDevice(&pl->device) != hipSuccess || hipMalloc(&pl->ws, pl->ws_bytes) != hipSuccess) {
        delete pl;
        return DCR_ERR_HIP;
    }
    *out = pl;
    return DCR_OK;
}

dcr_status dcr_plan_destroy(dcr_plan plan) {
    if (!plan) return DCR_ERR_INVALID_ARGUMENT;
    dcr_status st = DCR_OK;
    for (auto& in : plan->inst)
        if (in.done && in.launched && hipEventSynchronize(in.done) != hipSuccess) st = DCR_ERR_HIP;
    for (auto& in : plan->inst) release_instance(in);
    if (plan->ws && hipFree(plan->ws) != hipSuccess) st = DCR_ERR_HIP;
    delete plan;
    return st;
}

dcr_status dcr_plan_map_chunk(dcr_plan plan, int32_t* chunk) {
    if (!plan || !chunk) return DCR_ERR_INVALID_ARGUMENT;
    *chunk = plan->chunk;
    return DCR_OK;
}

dcr_status dcr_plan_resample_batched(dcr_plan plan, const void* w, const int64_t* w_off,
                                     const int64_t* n_off, int32_t B, uint64_t seed, int32_t* r,
                                     int32_t* seg_status, int32_t* dev_status,
                                     hipStream_t stream) {
    if (!plan || !w || !w_off || !n_off || B < 1 || B > plan->B_max ||
        (plan->sumN_max > 0 && !r))
        return DCR_ERR_INVALID_ARGUMENT;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return DCR_ERR_HIP;
    if (dev != plan->device) return DCR_ERR_INVALID_ARGUMENT;
    const BatchLayout L = make_batch_layout(plan->B_max, plan->sumM_max, plan->sumN_max);
    dcr::BatchNodeArgs a{};
    a.ba = batch_args(L, plan->ws, w_off, n_off, B, plan->B_max, plan->chunk, seed,
                      plan->sumM_max, plan->sumN_max, seg_status);
    a.w = w;
    a.r = r;
    a.dev_status = dev_status;
    dcr_plan_s::Instance& in = plan->inst[plan->next];
    if (!in.exec || in.chunk != plan->chunk) {
        if (in.launched && hipEventSynchronize(in.done) != hipSuccess) return DCR_ERR_HIP;
        const dcr_status st = build_instance(*plan, in, a);
        if (st != DCR_OK) return st;
    } else {
        // the previous launch of this instance has read its arguments
        if (in.launched && hipEventSynchronize(in.done) != hipSuccess) return DCR_ERR_HIP;
        hipKernelNodeParams kp[4];
        if (dcr::batched_node_params(prec_code(plan->p), a, plan->B_max, kp) != hipSuccess)
            return DCR_ERR_INTERNAL;
        for (int k = 0; k < 4; ++k)
            if (hipGraphExecKernelNodeSetParams(in.exec, in.nodes[k], &kp[k]) != hipSuccess)
                return DCR_ERR_HIP;
    }
    if (hipGraphLaunch(in.exec, stream) != hipSuccess) return DCR_ERR_HIP;
    if (hipEventRecord(in.done, stream) != hipSuccess) return DCR_ERR_HIP;
    in.launched = true;
    plan->next ^= 1;
    return DCR_OK;
}

dcr_status dcr_plan_autotune(dcr_plan plan, const void* w, const int64_t* w_off,
                             const int64_t* n_off, int32_t B, uint64_t seed, int32_t* r,
                             float* best_ms, hipStream_t stream) {
    if (!plan) return DCR_ERR_INVALID_ARGUMENT;
    if (B < 1 || B > plan->B_max) return DCR_ERR_INVALID_ARGUMENT;
    // the plan's graphs may still be reading the workspace
    for (auto& in : plan->inst)
        if (in.launched && hipEventSynchronize(in.done) != hipSuccess) return DCR_ERR_HIP;
    int32_t best = 0;
    float ms = 0.0f;
    const dcr_status st =
        dcr_batched_autotune(w, w_off, n_off, B, plan->sumM_max, plan->sumN_max, seed, plan->p,
                             r, plan->ws, plan->ws_bytes, nullptr, &best, &ms, stream);
    if (st != DCR_OK) return st;
    plan->chunk = best;   // the graphs are rebuilt for it on their next use
    if (best_ms) *best_ms = ms;
    cache_store(plan->cache_path.empty() ? nullptr : plan->cache_path.c_str(), plan->B_max,
                plan->sumM_max, plan->sumN_max, static_cast<int>(plan->p), best, ms);
    return DCR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// dcr_resample_noalloc: the end-to-end call with its scratch space in a static
// device array instead of a caller's workspace, for callers that cannot
// allocate.  Every GPU the library runs on holds its own copy of `scratch`
// (DCR_NOALLOC_SCRATCH_BYTES) until the process ends.  On the host, `scratch`
// names a host-side stand-in, never the device memory: the device address is
// taken once per device with hipGetSymbolAddress and only that address is
// handed to the kernels.  No scratch word is read before the call has written
// it, so the array needs no clearing between calls.
// ---------------------------------------------------------------------------
namespace {

static __device__ __align__(256) unsigned char scratch[DCR_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 256;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, taken on its first
// use there.
dcr_status scratch_for_current_device(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return DCR_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
            return DCR_ERR_HIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return DCR_OK;
}

}  // namespace

extern "C" dcr_status dcr_resample_noalloc(const void* w, int64_t M, int64_t N, uint64_t seed,
                                           uint64_t stream_id, dcr_precision p,
                                           dcr_scheme scheme, int32_t* r, double* W_opt,
                                           double* u_opt, int32_t* dev_status,
                                           hipStream_t stream) {
    // every host-visible error is reported before the first HIP call
    if (!w || M < 1 || M > kMaxM || N < 0 || N > kMaxN || (N > 0 && !r))
        return DCR_ERR_INVALID_ARGUMENT;
    if (!valid_prec(p) || !valid_scheme(scheme)) return DCR_ERR_UNSUPPORTED;
    if (make_layout(M, N, scheme).bytes > DCR_NOALLOC_SCRATCH_BYTES)
        return DCR_ERR_CAPACITY_EXCEEDED;
    void* ws = nullptr;
    const dcr_status st = scratch_for_current_device(&ws);
    if (st != DCR_OK) return st;
    dcr::WSource src;
    src.w = w;
    return resample_from(src, M, N, seed, stream_id, p, scheme, r, W_opt, u_opt, dev_status, ws,
                         DCR_NOALLOC_SCRATCH_BYTES, stream);
}
