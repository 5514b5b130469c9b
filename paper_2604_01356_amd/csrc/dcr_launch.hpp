// dcr_launch.hpp -- host-side launchers of the libdcr kernels and the optional
// per-launch timing hook.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "dcr_internal.hpp"

namespace dcr {

// Optional timing of the next kernel launch: when `start` and `stop` are set,
// the launch records its own start and end into them (hipExtLaunchKernel), so
// the interval is the kernel alone.  `launches` counts every launch made.  One
// instance per host thread: calls from different threads share no state.
struct LaunchEvents {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
    int64_t launches = 0;
};
extern thread_local LaunchEvents g_launch_events;

// Where the weights come from: an array `w` of the precision's type, or
// (P > 0) the outer product w_j = a[j / P] * b[j % P] of two such arrays.
struct WSource {
    const void* w = nullptr;
    const void* a = nullptr;
    const void* b = nullptr;
    int64_t P = 0;
    bool outer() const { return P > 0; }
    template <typename T>
    Outer<T> outer_as() const {
        return Outer<T>{static_cast<const T*>(a), static_cast<const T*>(b), P};
    }
};

hipError_t launch_reduce(int prec, const WSource& src, const WArgs& wa, const ZArgs& za, int vec_ok,
                         hipStream_t s);
bool finish_fits(const WArgs& wa, const ZArgs& za);

bool map_is_dense(int64_t M, int64_t N);
int64_t dense_chunks(int64_t M, int64_t N);   // at most ceil(N / 256)
// k_dense_span: the first and last sub-tile of each chunk of draws of the
// dense map, 2 * dense_chunks(M, N) int64 values in `span`.
hipError_t launch_dense_span(const WArgs& wa, const ZArgs& za, const SharedArgs& sh, int64_t* span,
                             hipStream_t s);
// k_map_dense: merges each chunk of draws within its span (chunks whose span
// is too wide to merge take one quad search per draw in the same launch).
hipError_t launch_map_dense(int prec, const WSource& src, const WArgs& wa, const ZArgs& za,
                            const SharedArgs& sh, const int64_t* span, double* u_out, int32_t* r,
                            int vec_ok, hipStream_t s);

hipError_t launch_carries(const WArgs& wa, const ZArgs& za, const SharedArgs& sh,
                          int32_t* dev_status, double* total_out, hipStream_t s);
hipError_t launch_finish(int prec, const WSource& src, const WArgs& wa, const ZArgs& za,
                         const SharedArgs& sh, int32_t* dev_status, double* u_out, int32_t* r,
                         int vec_ok, hipStream_t s);
// Problems of at most 8 weight blocks that the finishing launch takes:
// k_reduce_small (1024 threads per block) in place of k_reduce.
bool small_fits(const WArgs& wa, const ZArgs& za);
hipError_t launch_reduce_small(int prec, const WSource& src, const WArgs& wa, const ZArgs& za,
                               hipStream_t s);
hipError_t launch_materialize_w(int prec, const WSource& src, const WArgs& wa, const SharedArgs& sh,
                                double* W, int vec_ok, hipStream_t s);
hipError_t launch_materialize_u(const ZArgs& za, const SharedArgs& sh, double* u, hipStream_t s);
hipError_t launch_map_fused(int prec, const WSource& src, const WArgs& wa, const ZArgs& za,
                            const SharedArgs& sh, double* u_out, int32_t* r, int vec_ok,
                            hipStream_t s);
hipError_t launch_map_w(const double* W, int64_t M, const double* u, int64_t N, int32_t* r,
                        hipStream_t s);

// Streaming read (kind 0: grid-stride, one float partial sum per workgroup
// into dst), copy (kind 1), or read of one contiguous run per workgroup with
// non-temporal loads (kind 2) of `pieces` 16-byte pieces, `unroll` (4, 8, 16)
// loads in flight per thread, for bandwidth reference.
hipError_t launch_stream_probe(int kind, int unroll, const void* src, void* dst, int64_t pieces,
                               int grid, hipStream_t s);

// The batched launches, in order: plan, reduce, carries, map.
hipError_t launch_batch_plan(const BatchArgs& ba, int32_t* dev_status, hipStream_t s);
hipError_t launch_reduce_batched(int prec, const void* w, const BatchArgs& ba, hipStream_t s);
hipError_t launch_carries_batched(const BatchArgs& ba, hipStream_t s);
hipError_t launch_map_batched(int prec, const void* w, const BatchArgs& ba, int32_t* r,
                              int32_t* dev_status, hipStream_t s);

// The same four launches as kernel nodes of a graph (batched plans).  The
// argument blocks point into BatchNodeArgs, which the caller keeps alive while
// it adds or updates the nodes.
struct BatchNodeArgs {
    BatchArgs ba;
    const void* w;
    int32_t* r;
    int32_t* dev_status;
    void* argv[4][4];
};
hipError_t batched_node_params(int prec, BatchNodeArgs& a, int carry_wgs,
                               hipKernelNodeParams (&out)[4]);

}  // namespace dcr
