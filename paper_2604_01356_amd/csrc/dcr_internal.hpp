// dcr_internal.hpp -- argument blocks and constants shared by the host API and
// the kernels of libdcr (the launchers are in dcr_launch.hpp).  Not part of
// the public C ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace dcr {


constexpr int kPrecFP64 = 0;
constexpr int kPrecFP32 = 1;

constexpr int kStatusOk = 0;
constexpr int kStatusBadWeights = 6;

// Weights given as an outer product: w_j = a[j / P] * b[j % P] (binary64
// product of the two factors, exact for binary32 factors).
template <typename T>
struct Outer {
    const T* a;
    const T* b;
    int64_t P;
};

// Weight side: M weights in nb blocks of 32768.
struct WArgs {
    int64_t M;
    int64_t nb;
    double* blk_tot;   // [nb]   block totals (NaN: the block holds an inadmissible weight)
    double* beta;      // [nb]   block ends beta_1..beta_nb (monotone scan)
    double* sub_end;   // [nb*128] in-block sub-tile ends sigma_1..sigma_128
    double* chunk_tot; // [nb*2048] lane-chunk totals, or null (kept only by the batched form)
};

// Sorted-uniform schemes: Alg. 1 (exponential spacings), stratified
// (i + v_i) / N and systematic (i + v_0) / N.
constexpr int kSchemeMultinomial = 0;
constexpr int kSchemeStratified = 1;
constexpr int kSchemeSystematic = 2;

// Spacing side: draws 0..N in nb blocks of 4096 (nb = 0 for the stratified
// and systematic schemes, whose uniforms need no scan).
struct ZArgs {
    int64_t N;
    int64_t nb;
    uint64_t seed;
    uint64_t stream;
    int32_t scheme;
    double* zrel;      // [N+1] in-block prefix sums of the spacings
    double* blk_tot;   // [nb]
    double* beta;      // [nb]
};

struct SharedArgs {
    int32_t* status;   // [1] device status of the last scan
    double* totals;    // [2] weight total, spacing total
};

// k_finish handles up to 4096 weight blocks (M <= 2^27) and this many
// spacing blocks (N + 1 <= 2^18).
constexpr int kFinishMaxZBlocks = 64;

// Problems of at most this many weight blocks (M <= 2^18) that k_finish
// takes run k_reduce_small in place of k_reduce.
constexpr int kSmallBlocks = 8;

// N * kDenseRatio >= M: several uniforms per sub-tile on average, mapped by
// the windowed linear merge (k_map_dense) instead of one search per uniform.
constexpr int64_t kDenseRatio = 4;

// Batched form: B independent filters over concatenated arrays.  Filter b
// owns weights [w_off[b], w_off[b+1]) and draws [n_off[b], n_off[b+1]); its
// blocks, scans and draws follow the single-distribution structure relative
// to its own start, with Philox stream id b, so each filter's result equals a
// single call on its weights.
struct BatchArgs {
    const int64_t* w_off;   // [B+1] caller's weight offsets (w_off[0] == 0)
    const int64_t* n_off;   // [B+1] caller's draw offsets (n_off[0] == 0)
    int32_t B;
    int32_t chunk;          // draws per map workgroup: 256, 512 or 1024
    uint64_t seed;
    int64_t wt_cap, zt_cap, mc_cap;   // launch sizes: weight blocks, spacing blocks, map chunks
    int64_t sumM_cap, sumN_cap;
    int64_t* wt_base;       // [B+1] first weight block of each filter (k_batch_plan)
    int64_t* zt_base;       // [B+1] first spacing block
    int64_t* mc_base;       // [B+1] first map chunk (`chunk` draws)
    int32_t* mc_seg;        // [mc_cap] filter of each map chunk (k_carries_batched)
    int32_t* head;          // [0] plan status, [1] batch status
    double* wt_tot;         // [wt_cap] weight-block totals
    double* wt_beta;        // [wt_cap] weight-block ends (per filter)
    double* wt_sub;         // [wt_cap * 128] sub-tile ends
    double* wt_chunk;       // [wt_cap * 2048] lane-chunk totals
    double* zt_tot;         // [zt_cap]
    double* zt_beta;        // [zt_cap]
    double* zrel;           // [sumN + B] in-block spacing prefixes, filter b at n_off[b] + b
    int32_t* seg_status;    // [B]
    double* seg_totals;     // [2B] weight total, spacing total
};
constexpr int kPlanThreads = 1024;
constexpr int64_t kBatchWBlock = 32768;
constexpr int64_t kBatchZBlock = 4096;
constexpr int kBatchChunkDefault = 512;
}  // namespace dcr
