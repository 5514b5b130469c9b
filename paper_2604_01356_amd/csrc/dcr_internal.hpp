// dcr_internal.hpp -- argument blocks and launchers shared by the host API and
// the kernels of libdcr.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace dcr {

constexpr int kPrecFP64 = 0;
constexpr int kPrecFP32 = 1;

constexpr int kStatusOk = 0;
constexpr int kStatusBadWeights = 6;

// Weight side: M weights in nb blocks of 32768.
struct WArgs {
    int64_t M;
    int64_t nb;
    double* blk_tot;   // [nb]   block totals (NaN: the block holds an inadmissible weight)
    double* beta;      // [nb]   block ends beta_1..beta_nb (monotone scan)
    double* sub_end;   // [nb*128] in-block sub-tile ends sigma_1..sigma_128
};

// Spacing side: draws 0..N in nb blocks of 4096.
struct ZArgs {
    int64_t N;
    int64_t nb;
    uint64_t seed;
    uint64_t stream;
    double* zrel;      // [N+1] in-block prefix sums of the spacings
    double* blk_tot;   // [nb]
    double* beta;      // [nb]
};

struct SharedArgs {
    int32_t* status;   // [1] device status of the last scan
    double* totals;    // [2] weight total, spacing total
};

hipError_t launch_reduce(int prec, const void* w, const WArgs& wa, const ZArgs& za, int vec_ok,
                         hipStream_t s);
// k_finish handles up to 4096 weight blocks (M <= 2^27) and this many
// spacing blocks (N + 1 <= 2^18).
constexpr int kFinishMaxZBlocks = 64;
bool finish_fits(const WArgs& wa, const ZArgs& za);

// N * kDenseRatio >= M: several uniforms per sub-tile on average, mapped by
// the windowed linear merge (k_map_dense) instead of one search per uniform.
constexpr int64_t kDenseRatio = 4;
bool map_is_dense(int64_t M, int64_t N);
int64_t dense_chunks(int64_t N);
// Runs k_map_dense and then k_map_wide for the chunks it flags in `wide`
// (dense_chunks(N) int32 flags, written before they are read).
hipError_t launch_map_dense(int prec, const void* w, const WArgs& wa, const ZArgs& za,
                            const SharedArgs& sh, double* u_out, int32_t* r, int32_t* wide,
                            int vec_ok, hipStream_t s);

hipError_t launch_carries(const WArgs& wa, const ZArgs& za, const SharedArgs& sh,
                          int32_t* dev_status, double* total_out, hipStream_t s);
hipError_t launch_finish(int prec, const void* w, const WArgs& wa, const ZArgs& za,
                         const SharedArgs& sh, int32_t* dev_status, double* u_out, int32_t* r,
                         int vec_ok, hipStream_t s);
hipError_t launch_materialize_w(int prec, const void* w, const WArgs& wa, const SharedArgs& sh,
                                double* W, int vec_ok, hipStream_t s);
hipError_t launch_materialize_u(const ZArgs& za, const SharedArgs& sh, double* u, hipStream_t s);
hipError_t launch_map_fused(int prec, const void* w, const WArgs& wa, const ZArgs& za,
                            const SharedArgs& sh, double* u_out, int32_t* r, int vec_ok,
                            hipStream_t s);
hipError_t launch_map_w(const double* W, int64_t M, const double* u, int64_t N, int32_t* r,
                        hipStream_t s);

}  // namespace dcr
