// dcr_kernels.hip -- HIP kernels for gfx950 (MI355X) implementing the three
// stages of divide-and-conquer multinomial resampling (Popov, Secs. I-III):
//   k_reduce            weight-block totals (Eq. 3) and spacing-block totals
//                       (Alg. 1), one launch, two kinds of workgroups
//                       interleaved (tile_role)
//   k_carries           monotone scans of the block totals, totals, validity
//   k_materialize_w     normalised cumulative weights W (stage 1 output)
//   k_materialize_u     sorted uniforms u (stage 2 output)
//   k_finish            block scans + uniforms + map in one launch (the common
//                       end-to-end case)
//   k_reduce_small      k_reduce for at most 8 weight blocks: 1024 threads per
//                       block, so its 8 rounds of loads are in flight at once
//   k_map_fused         inverse CMF of u against the cumulative weights kept
//                       implicit (block bases + sub-tile bases + a rescan of one
//                       256-weight sub-tile), the divide-and-conquer map of
//                       Alg. 5 laid onto the block / sub-tile / element levels
//   k_map_dense         inverse CMF when N >= M/4: the linear merge of Alg. 4
//   k_dense_span        the span of sub-tiles of every chunk of the dense map
//   k_map_w, k_map_w_dense
//                       inverse CMF against a given W (stage 3 alone)
// Every kernel that reads weights has an `_outer` twin for weights given as
// an outer product a[i] * b[k], formed in registers (never read from memory).
//   k_batch_plan, k_reduce_batched, k_carries_batched, k_map_batched
//                       the batched form: many filters in one call
// The summation structure that fixes the bits of W and u is described in
// dcr_device.hpp.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <tuple>
#include <type_traits>

#include "dcr_device.hpp"
#include "dcr_internal.hpp"
#include "dcr_launch.hpp"

namespace dcr {

__device__ __forceinline__ int clamp_count(int64_t remaining, int cap) {
    return remaining <= 0 ? 0 : (remaining >= cap ? cap : static_cast<int>(remaining));
}

// ---------------------------------------------------------------------------
// k_reduce: blocks [0, za.nb) draw spacings, blocks [za.nb, za.nb + wa.nb)
// reduce weights.
//
// Binary32 weights in a full block stream through LDS: each wave's 4 KB round
// (its 4 sub-tiles, 64 lanes x 16 consecutive weights) is fetched with
// coalesced direct-to-LDS loads two rounds ahead, then every lane reads its own
// 16 consecutive weights back.  Lane-strided global loads of the same bytes
// reach only ~85% of the coalesced bandwidth on this chip.
// ---------------------------------------------------------------------------
constexpr int kStreamDepth = 2;                     // rounds in flight beyond the current
constexpr int kWaveRoundF32 = 64 * kLane;           // floats per wave per round (4 KB)
constexpr int kWaves = kThreads / 64;

// Three separate LDS objects hold the stream buffers (separate objects let
// the compiler see that reading one buffer need not wait for the loads still
// in flight into another); the block epilogue reuses the first one.
template <typename Tin>
struct ReduceSmem {
    static constexpr int kBuf = (sizeof(Tin) == 4) ? kWaves * kWaveRoundF32 * 4 : 16;
    // the epilogue: lane totals in rows of 16 padded to 17, then sub-tile totals and ends
    static constexpr int kEpi = (kWIters * (kThreads + kThreads / kRowLanes) + 2 * kWSubPerBlock) * 8;
    // binary64: one round of weights staged per wave (4 waves x 8 KB)
    static constexpr int kStage = (sizeof(Tin) == 8) ? kThreads * kLane * 8 : 0;
    static constexpr int kBuf0a = kBuf > kEpi ? kBuf : kEpi;
    static constexpr int kBuf0 = kBuf0a > kStage ? kBuf0a : kStage;
};

// s_waitcnt lgkmcnt(0) with vmcnt and expcnt left at their maxima
constexpr int kWaitLdsOnly = 0xC07F;

__device__ __forceinline__ void wait_vm(int outstanding) {
    // s_waitcnt with vmcnt = outstanding (0..15), expcnt and lgkmcnt left at max
    __builtin_amdgcn_sched_barrier(0);
    if (outstanding >= 8)
        __builtin_amdgcn_s_waitcnt(0x0F78);
    else if (outstanding >= 4)
        __builtin_amdgcn_s_waitcnt(0x0F74);
    else
        __builtin_amdgcn_s_waitcnt(0x0F70);
    __builtin_amdgcn_sched_barrier(0);
}

// Spacing block g of za: z_i = -log v_i (Alg. 1) for its draws, their
// in-block prefix sums (stored) and the block total.  All threads call it.
template <int P>
__device__ __forceinline__ void reduce_z_block(const ZArgs& za, int64_t g, double* lane_tot,
                                               double* sub_tot) {
    const int t = threadIdx.x;
    const int row = t / kRowLanes;
    const int lane = t % kRowLanes;
    {
        const int64_t i0 = g * kZBlock + static_cast<int64_t>(t) * kLane;
        const int nv = clamp_count(za.N + 1 - i0, kLane);
        double p[kLane];
#pragma unroll
        for (int k = 0; k < kLane; k += 2) {
            double ze = 0.0, zo = 0.0;
            if (k < nv) spacing_pair<P>(static_cast<uint64_t>(i0 + k) >> 1, za.seed, za.stream, ze, zo);
            p[k] = (k < nv) ? ze : 0.0;
            p[k + 1] = (k + 1 < nv) ? zo : 0.0;
        }
#pragma unroll
        for (int k = 1; k < kLane; ++k) p[k] = p[k - 1] + p[k];
        lane_tot[t] = p[kLane - 1];
        lds_barrier();
        double lv[kRowLanes];
#pragma unroll
        for (int k = 0; k < kRowLanes; ++k) lv[k] = lane_tot[row * kRowLanes + k];
        double c = 0.0;
#pragma unroll
        for (int k = 0; k < kRowLanes; ++k)
            if (k < lane) c = c + lv[k];
        if (lane == kRowLanes - 1) sub_tot[row] = c + lv[kRowLanes - 1];
        lds_barrier();
        double rv[kRows];
#pragma unroll
        for (int k = 0; k < kRows; ++k) rv[k] = sub_tot[k];
        double sigma = 0.0, total = 0.0;
#pragma unroll
        for (int k = 0; k < kRows; ++k) {
            if (k < row) sigma = sigma + rv[k];
            total = total + rv[k];
        }
        double zr[kLane];
#pragma unroll
        for (int k = 0; k < kLane; ++k) zr[k] = sigma + (c + p[k]);
        // the block's prefixes leave through LDS, half a block (8 rows) at a
        // time, as coalesced 16-byte pieces with the non-temporal policy; a
        // thread's 16 values sit 17 doubles apart there (fewer bank conflicts)
        constexpr int kHalfThreads = kThreads / 2;
        constexpr int kPad = kLane + 1;
        double* stage = lane_tot;   // kHalfThreads * kPad doubles
        const int64_t blk = g * kZBlock;
        const int64_t lim = (za.N + 1 - blk < kZBlock) ? za.N + 1 - blk : kZBlock;   // prefixes of the block
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            lds_barrier();   // every read of the region before it is done
            if (t / kHalfThreads == h) {
                const int tl = t % kHalfThreads;
#pragma unroll
                for (int k = 0; k < kLane; ++k) stage[tl * kPad + k] = zr[k];
            }
            lds_barrier();
#pragma unroll
            for (int m = 0; m < kHalfThreads * kLane / 2 / kThreads; ++m) {
                const int pc = t + m * kThreads;          // piece of the half
                const int e = 2 * pc;                     // its first value in the half
                const int at = (e / kLane) * kPad + (e % kLane);
                const int64_t j = static_cast<int64_t>(h) * kHalfThreads * kLane + e;   // in the block
                const double a = stage[at], b = stage[at + 1];
                if (j + 1 < lim) {
                    __builtin_nontemporal_store(f64x2{a, b}, reinterpret_cast<f64x2*>(za.zrel + blk + j));
                } else if (j < lim) {
                    za.zrel[blk + j] = a;
                }
            }
        }
        if (t == 0) za.blk_tot[g] = total;
    }
}

// Weight block b of wa: lane-chunk totals, sub-tile totals, the stored
// sub-tile ends and the block total (NaN for an inadmissible block).  The
// three LDS buffers stream binary32 weights; sb0 is also the epilogue's
// scratch.  All threads call it.
// The end of a weight block, whatever its load path: the lane-chunk totals
// lt (round it = sub-tile 16 it + row) become the sub-tile totals, the stored
// sub-tile ends and the block total.  sb0 is at least ReduceSmem<>::kEpi bytes.
__device__ __forceinline__ void reduce_w_epilogue(const double (&lt)[kWIters], int bad,
                                                  const WArgs& wa, int64_t b, unsigned char* sb0) {
    // lane totals: round it, thread t at it * kEpiRow + 17 * row + lane (a
    // sub-tile's 16 totals are read by one thread; rows of 16 doubles put the
    // 64 readers of a wave in one bank)
    constexpr int kEpiRow = kThreads + kThreads / kRowLanes;
    double* lane_tot = reinterpret_cast<double*>(sb0);   // [kWIters][kEpiRow]
    double* sub_tot = lane_tot + kWIters * kEpiRow;       // [kWSubPerBlock]
    double* sub_end = sub_tot + kWSubPerBlock;            // [kWSubPerBlock]
    const int t = threadIdx.x;
    if (wa.chunk_tot) {
        // lane chunk (sub-tile 16 it + row, lane) of the block: coalesced per
        // round, and non-temporal (the map reads them much later; whole lines
        // go out together).  The lane-strided spacing prefixes are not: there
        // every 16-byte piece would go to memory on its own
        double* ct = wa.chunk_tot + b * (kWSubPerBlock * kRowLanes);
#pragma unroll
        for (int it = 0; it < kWIters; ++it) __builtin_nontemporal_store(lt[it], &ct[it * kThreads + t]);
    }
    lds_barrier();   // the first stream buffer becomes the epilogue's scratch
#pragma unroll
    for (int it = 0; it < kWIters; ++it) lane_tot[it * kEpiRow + t + t / kRowLanes] = lt[it];
    bad = block_any(bad);
    if (t < kWSubPerBlock) {
        const int it = t / kRows;
        const int r = t % kRows;
        const double* p = lane_tot + it * kEpiRow + r * (kRowLanes + 1);
        double lv[kRowLanes];
#pragma unroll
        for (int l = 0; l < kRowLanes; ++l) lv[l] = p[l];
        double c = lv[0];
#pragma unroll
        for (int l = 1; l < kRowLanes; ++l) c = c + lv[l];
        sub_tot[t] = c;
    }
    lds_barrier();
    if (t == 0) {
        double s = 0.0;
#pragma unroll 16
        for (int q = 0; q < kWSubPerBlock; ++q) {
            s = s + sub_tot[q];
            sub_end[q] = s;
        }
    }
    lds_barrier();
    if (t < kWSubPerBlock) wa.sub_end[b * kWSubPerBlock + t] = sub_end[t];
    if (t == 0) {
        // an inadmissible block (negative weight, NaN, infinity or overflow)
        // publishes a NaN total, which every scan of the totals detects
        const double tot = sub_end[kWSubPerBlock - 1];
        wa.blk_tot[b] = (bad || !(tot < __builtin_huge_val())) ? __builtin_nan("") : tot;
    }
}

template <typename Tin, int DEPTH = kStreamDepth>
__device__ __forceinline__ void reduce_w_block(const Tin* __restrict__ w, const WArgs& wa, int64_t b,
                                               int vec_ok, unsigned char* sb0, unsigned char* sb1,
                                               unsigned char* sb2) {
    static_assert(DEPTH == 1 || DEPTH == 2, "one or two rounds in flight");
    constexpr int kBufs = DEPTH + 1;
    const int t = threadIdx.x;
    const int row = t / kRowLanes;
    const int lane = t % kRowLanes;
    const int64_t blk0 = b * kWBlock;
    int bad = 0;
    double lt[kWIters];
    const bool full = blk0 + kWBlock <= wa.M;
    const bool aligned = (vec_ok & 1) != 0;
    if constexpr (sizeof(Tin) == 4) {
        if (full && aligned) {
            float* const bufs[3] = {reinterpret_cast<float*>(sb0), reinterpret_cast<float*>(sb1),
                                    reinterpret_cast<float*>(sb2)};
            const int wv = t >> 6;
            const int l64 = t & 63;
            // the wave's rows 4wv..4wv+3 of round `it` are kWaveRoundF32 consecutive weights
            const float* src = reinterpret_cast<const float*>(w) + blk0 + wv * kWaveRoundF32;
            auto issue = [&](int it) {
                float* dst = bufs[it % kBufs] + wv * kWaveRoundF32;
                const float* g0 = src + it * (kWaves * kWaveRoundF32);
#pragma unroll
                for (int k = 0; k < kLane / 4; ++k)
                    __builtin_amdgcn_global_load_lds(g0 + k * 256 + l64 * 4, dst + k * 256, 16, 0,
                                                     kCachePolicyNT);
            };
            float mn = 0.0f;
#pragma unroll
            for (int it = 0; it < DEPTH; ++it) issue(it);
#pragma unroll
            for (int it = 0; it < kWIters; ++it) {
                if (it + DEPTH < kWIters) {
                    issue(it + DEPTH);
                    wait_vm(DEPTH * (kLane / 4));
                } else {
                    wait_vm((kWIters - 1 - it) * (kLane / 4));
                }
                __builtin_amdgcn_wave_barrier();
                const f32x4* mine = reinterpret_cast<const f32x4*>(
                    bufs[it % kBufs] + wv * kWaveRoundF32 + l64 * kLane);
                RawChunk<float> rc;
#pragma unroll
                for (int k = 0; k < kLane / 4; ++k) rc.v[k] = mine[k];
                if (it == 0) mn = rc.raw(0);
                lt[it] = raw_sum<float>(rc, mn);
                __builtin_amdgcn_sched_barrier(0);
                __builtin_amdgcn_wave_barrier();
            }
            // NaN and +inf reach the block total (checked below); negatives the minimum
            bad = (mn < 0.0f) ? 1 : 0;
        } else if (full) {
            // a block that starts off a 16-byte boundary (a filter of a batch
            // may start at any element): each wave loads its round as
            // coalesced 16-byte pieces of element-aligned addresses, two
            // rounds ahead in registers, and passes them through its own LDS
            // region into the lane-chunk layout of the path above
            const int wv = t >> 6;
            const int l64 = t & 63;
            const float* src = reinterpret_cast<const float*>(w) + blk0 + wv * kWaveRoundF32;
            float* const region = reinterpret_cast<float*>(sb0) + wv * kWaveRoundF32;
            f32x4 ring[DEPTH + 1][kLane / 4];
            auto fetch = [&](int it, f32x4 (&dst)[kLane / 4]) {
                const float* g0 = src + it * (kWaves * kWaveRoundF32);
#pragma unroll
                for (int k = 0; k < kLane / 4; ++k)
                    dst[k] = __builtin_nontemporal_load(
                        reinterpret_cast<const f32x4_ea*>(g0 + k * 256 + l64 * 4));
            };
#pragma unroll
            for (int it = 0; it < DEPTH; ++it) fetch(it, ring[it]);
            float mn = 0.0f;
#pragma unroll
            for (int it = 0; it < kWIters; ++it) {
                if (it + DEPTH < kWIters) fetch(it + DEPTH, ring[(it + DEPTH) % (DEPTH + 1)]);
#pragma unroll
                for (int k = 0; k < kLane / 4; ++k)
                    *reinterpret_cast<f32x4*>(region + k * 256 + l64 * 4) = ring[it % (DEPTH + 1)][k];
                __builtin_amdgcn_s_waitcnt(kWaitLdsOnly);   // the wave's writes are done
                __builtin_amdgcn_wave_barrier();
                const f32x4* mine = reinterpret_cast<const f32x4*>(region + l64 * kLane);
                RawChunk<float> rc;
#pragma unroll
                for (int k = 0; k < kLane / 4; ++k) rc.v[k] = mine[k];
                if (it == 0) mn = rc.raw(0);
                lt[it] = raw_sum<float>(rc, mn);
                __builtin_amdgcn_wave_barrier();
            }
            bad = (mn < 0.0f) ? 1 : 0;
        }
    }
    if constexpr (sizeof(Tin) == 8) {
        if (full) {
            // binary64: each wave loads its quarter of a round (1024 weights,
            // its four rows) as coalesced 16-byte non-temporal pieces of
            // element-aligned addresses, one round ahead in registers, and
            // passes them through its own 8 KB of LDS into the lane-chunk
            // layout.  Piece j of lane chunk c sits at slot j ^ (c & 7) of the
            // chunk's 128 bytes, so that neither the wave's writes (eight
            // lanes per chunk) nor its reads (one chunk per lane) meet in a
            // bank.  (Cached lane-strided loads, each lane reading its own
            // line, streamed at about 5.4 TB/s; non-temporal, each 16-byte
            // piece went to memory on its own.)
            constexpr int kWaveRound = kRows / kWaves * kSub;   // 1024 weights
            constexpr int kPieces = kWaveRound / 2 / 64;         // 16-byte pieces per lane
            constexpr int kDepth = 1;
            const int wv = t >> 6;
            const int l64 = t & 63;
            const double* src = reinterpret_cast<const double*>(w) + blk0 + wv * kWaveRound;
            f64x2* const region = reinterpret_cast<f64x2*>(sb0) + wv * (kWaveRound / 2);
            f64x2 ring[kDepth + 1][kPieces];
            auto fetch = [&](int it, f64x2 (&dst)[kPieces]) {
                const double* g0 = src + it * (kWaves * kWaveRound);
#pragma unroll
                for (int k = 0; k < kPieces; ++k)
                    dst[k] = __builtin_nontemporal_load(
                        reinterpret_cast<const f64x2_ea*>(g0 + 2 * (k * 64 + l64)));
            };
#pragma unroll
            for (int it = 0; it < kDepth; ++it) fetch(it, ring[it]);
            double mn = 0.0;
#pragma unroll
            for (int it = 0; it < kWIters; ++it) {
                if (it + kDepth < kWIters) fetch(it + kDepth, ring[(it + kDepth) % (kDepth + 1)]);
#pragma unroll
                for (int k = 0; k < kPieces; ++k) {
                    const int pc = k * 64 + l64;   // piece of the wave's round
                    const int c = pc >> 3, j = pc & 7;
                    region[c * 8 + (j ^ (c & 7))] = ring[it % (kDepth + 1)][k];
                }
                __builtin_amdgcn_s_waitcnt(kWaitLdsOnly);   // the wave's writes are done
                __builtin_amdgcn_wave_barrier();
                RawChunk<double> rc;   // lane l64 holds chunk l64 of the wave's round
#pragma unroll
                for (int j = 0; j < kLane / 2; ++j) rc.v[j] = region[l64 * 8 + (j ^ (l64 & 7))];
                if (it == 0) mn = rc.raw(0);
                lt[it] = raw_sum<double>(rc, mn);
                __builtin_amdgcn_wave_barrier();   // the region is rewritten next round
            }
            bad = (mn < 0.0) ? 1 : 0;
        }
    }
    if (!full) {
        // the array's ragged last block: the same lane-strided loop, each chunk
        // zero-padded beyond the weights that exist (a NaN or infinity still
        // reaches the block total, a negative weight the minimum)
        // (kept rolled: only one block of an array takes this path)
        const int64_t j00 = blk0 + row * kSub + lane * kLane;
        const Tin* base = w + j00;
        Tin mn = static_cast<Tin>(0);
        RawChunk<Tin> cur = load_raw_n<Tin>(base, clamp_count(wa.M - j00, kLane));
#pragma unroll 1
        for (int it = 0; it < kWIters; ++it) {
            const int64_t jn = j00 + static_cast<int64_t>(it + 1) * kRows * kSub;
            const int nn = (it + 1 < kWIters) ? clamp_count(wa.M - jn, kLane) : 0;
            const RawChunk<Tin> nxt = load_raw_n<Tin>(base + (nn > 0 ? (it + 1) * kRows * kSub : 0), nn);
            const double ct = raw_sum<Tin>(cur, mn);
#pragma unroll
            for (int q = 0; q < kWIters; ++q)
                if (q == it) lt[q] = ct;
            cur = nxt;
        }
        bad = (mn < static_cast<Tin>(0)) ? 1 : 0;
    }
    reduce_w_epilogue(lt, bad, wa, b, sb0);
}

// Weight block b of an outer-product source: each lane forms its chunks'
// products (nothing of length M is read), then the common epilogue.
template <typename T>
__device__ __forceinline__ void reduce_w_block_outer(const Outer<T>& o, const WArgs& wa, int64_t b,
                                                     unsigned char* sb0) {
    const int t = threadIdx.x;
    const int row = t / kRowLanes;
    const int lane = t % kRowLanes;
    const int64_t j00 = b * kWBlock + row * kSub + lane * kLane;
    double lt[kWIters];
    double mn = 0.0;
    if (o.P >= kLane) {
        // the factors of kU chunks are loaded before any product is summed
        constexpr int kU = (sizeof(T) == 4) ? kWIters : kWIters / 4;
#pragma unroll 1
        for (int h = 0; h < kWIters; h += kU) {
            OuterRaw<T> raw[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int64_t j0 = j00 + static_cast<int64_t>(h + u) * kRows * kSub;
                raw[u] = outer_load(o, j0, clamp_count(wa.M - j0, kLane));
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const double ct = raw_sum<double>(outer_products(raw[u]), mn);
#pragma unroll
                for (int q = 0; q < kWIters; ++q)
                    if (q == h + u) lt[q] = ct;
            }
        }
    } else {
#pragma unroll 1
        for (int it = 0; it < kWIters; ++it) {
            const int64_t j0 = j00 + static_cast<int64_t>(it) * kRows * kSub;
            const RawChunk<double> rc = src_raw_n(o, j0, clamp_count(wa.M - j0, kLane));
            const double ct = raw_sum<double>(rc, mn);
#pragma unroll
            for (int q = 0; q < kWIters; ++q)
                if (q == it) lt[q] = ct;
        }
    }
    reduce_w_epilogue(lt, (mn < 0.0) ? 1 : 0, wa, b, sb0);
}

// Workgroup order of the reduce launches.  Of nz spacing tiles and nw weight
// tiles, the kind with fewer tiles is spread among the other, one in every p
// workgroups, so that each CU mixes the ALU-bound spacing work with the
// HBM-bound weight stream instead of running the two one after the other.
// p is odd, so that consecutive tiles of the spread kind land on different
// XCDs (workgroups go to the 8 XCDs in turn).  Spacing tiles that fit at one
// per CU go first instead: spread to the end of the launch, a slow (binary64)
// spacing tile would become its tail.
// Workgroup i maps to exactly one tile: is_z tells the kind, idx its index.
struct TileRole {
    bool is_z;
    int64_t idx;
};
constexpr int64_t kTileFirstMax = 256;   // compute units of the chip

__device__ __forceinline__ TileRole tile_role(int64_t i, int64_t nz, int64_t nw) {
    const bool z_minor = nz <= nw;
    const int64_t nminor = z_minor ? nz : nw;
    if (nminor == 0) return TileRole{nz > 0, i};
    const int64_t spread = (nz + nw) / nminor;   // >= 2
    const int64_t p = (z_minor && nz <= kTileFirstMax) ? 1 : spread - (1 - (spread & 1));
    const int64_t k = i / p;
    if (i % p == p - 1 && k < nminor) return TileRole{z_minor, k};
    return TileRole{!z_minor, i - (k < nminor ? k : nminor)};
}

template <typename T, int P>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_reduce_outer(Outer<T> o, WArgs wa, ZArgs za) {
    __shared__ __attribute__((aligned(16))) unsigned char sb0[ReduceSmem<double>::kBuf0];
    const TileRole role = tile_role(blockIdx.x, za.nb, wa.nb);
    if (role.is_z) {
        double* lane_tot = reinterpret_cast<double*>(sb0);
        reduce_z_block<P>(za, role.idx, lane_tot, lane_tot + kThreads);
        return;
    }
    reduce_w_block_outer<T>(o, wa, role.idx, sb0);
}

template <typename Tin, int P>
__global__ __launch_bounds__(kThreads) void k_reduce(const Tin* __restrict__ w, WArgs wa, ZArgs za,
                                                     int vec_ok) {
    __shared__ __attribute__((aligned(16))) unsigned char sb0[ReduceSmem<Tin>::kBuf0];
    __shared__ __attribute__((aligned(16))) unsigned char sb1[ReduceSmem<Tin>::kBuf];
    __shared__ __attribute__((aligned(16))) unsigned char sb2[ReduceSmem<Tin>::kBuf];
    const TileRole role = tile_role(blockIdx.x, za.nb, wa.nb);
    if (role.is_z) {
        double* lane_tot = reinterpret_cast<double*>(sb0);
        reduce_z_block<P>(za, role.idx, lane_tot, lane_tot + kThreads);
        return;
    }
    reduce_w_block<Tin>(w, wa, role.idx, vec_ok, sb0, sb1, sb2);
}

// ---------------------------------------------------------------------------
// Monotone scans of block totals by the 256 threads of one workgroup, two at a
// time (weights and spacings share the barriers).  The same code runs in
// every kernel that needs a scan, so the results agree bit for bit.
// For one sequence of n totals: thread t owns a contiguous range and sums it
// left to right (p_j); the thread bases gamma_t are an exclusive scan of the
// thread totals (DPP wave scans, then the 4 wave totals left to right) made
// non-decreasing by a running maximum; then
//     out_j = min(gamma_t + p_j, gamma_{t+1}),
// which is non-decreasing for non-negative input.  Zero totals keep the
// output exactly where it was (a bin of weight zero gets an empty interval):
// the outputs of a thread whose running sum has reached its total (unless it
// ends the sequence) are gamma_{t+1} itself, and the base that follows a
// thread with a zero total does not enter the running maximum, so
// gamma_{t+1} = gamma_t there; zeros inside a thread's range add nothing to p.  A NaN or infinite total (an inadmissible block)
// sets the sequence's `bad` flag.
// ---------------------------------------------------------------------------
constexpr int kScanThreads = kThreads;
constexpr int kScanWaves = kScanThreads / 64;
constexpr int kScanRegs = 16;   // ranges up to this length stay in registers
constexpr int kBatchScanRegs = 4;
constexpr int kCarryScanRegs = 32;   // k_carries: one workgroup, so registers are plentiful
constexpr int kScanBatch = 16;  // loads in flight per thread when the ranges are longer

// Per-thread inputs of a scan, loaded ahead of the computation so that the
// loads of both scans (and of other data) are in flight together.
template <int R = kScanRegs>
struct ScanIn {
    static constexpr int kRegs = R;
    int64_t a, e;
    bool in_regs;
    int per;   // elements per thread when in registers (workgroup-uniform), else 0
    double v[R];
};

struct ScanOut {
    const double* in;   // the totals (re-read when they do not fit in registers)
    int64_t n;
    double* out_lds;    // may be null
    double* out_gl;     // may be null
};

struct ScanLds {
    double wtot[2][kScanWaves];
    double wmax[2][kScanWaves];
    int wbad[2][kScanWaves];
    int wlastz[2][kScanWaves];   // the wave's last thread has a zero total
    double last[2];
    double spare[2];   // receives the unused outputs of a thread's last registers
};

template <int R>
__device__ __forceinline__ void scan_load(const double* __restrict__ in, int64_t n, ScanIn<R>& si) {
    const int t = threadIdx.x;
    const int64_t per = (n + kScanThreads - 1) / kScanThreads;
    si.a = (static_cast<int64_t>(t) * per < n) ? static_cast<int64_t>(t) * per : n;
    si.e = (si.a + per < n) ? si.a + per : n;
    si.in_regs = per <= R;
    si.per = si.in_regs ? static_cast<int>(per) : 0;
    if (si.in_regs) {
#pragma unroll
        for (int k = 0; k < R; ++k)
            si.v[k] = (k < si.per && si.a + k < si.e) ? in[si.a + k] : 0.0;
    }
}

// Computes both scans; total[k] = out[n-1] of sequence k (0 if n == 0).
template <int R>
__device__ void scan_pair(const ScanIn<R> (&si)[2], const ScanOut (&so)[2], ScanLds& L,
                          double (&total)[2], int (&bad)[2]) {
    const int t = threadIdx.x;
    const int lane64 = t & 63;
    const int wid = t >> 6;
    double excl[2], wmx[2], wb[2];
    // the thread's running sums, kept for the outputs, and its total
    double pre[2][R], thr[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        double tt = 0.0;
        int nonfinite = 0;
        if (si[q].in_regs) {
#pragma unroll
            for (int k = 0; k < R; ++k) {
                tt = tt + si[q].v[k];   // + 0.0 past the range is exact
                pre[q][k] = tt;
                nonfinite |= !(si[q].v[k] < __builtin_huge_val());
            }
        } else {   // batches of loads in flight together, then their sums
            for (int64_t j0 = si[q].a; j0 < si[q].e; j0 += kScanBatch) {
                double x[kScanBatch];
#pragma unroll
                for (int k = 0; k < kScanBatch; ++k)
                    x[k] = (j0 + k < si[q].e) ? so[q].in[j0 + k] : 0.0;
#pragma unroll
                for (int k = 0; k < kScanBatch; ++k) {
                    tt = tt + x[k];   // + 0.0 past the range is exact
                    nonfinite |= !(x[k] < __builtin_huge_val());
                }
            }
        }
        thr[q] = tt;
        const double incl = wave_incl_add(tt);
        excl[q] = wave_shift_up1(incl);
        const bool wave_bad = __builtin_amdgcn_ballot_w64(nonfinite != 0) != 0;
        if (lane64 == 63) {
            L.wtot[q][wid] = incl;
            L.wlastz[q][wid] = (tt == 0.0) ? 1 : 0;
        }
        if (lane64 == 0) L.wbad[q][wid] = wave_bad ? 1 : 0;
    }
    lds_barrier();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        double w4[kScanWaves];
        int b4 = 0;
#pragma unroll
        for (int k = 0; k < kScanWaves; ++k) {
            w4[k] = L.wtot[q][k];
            b4 |= L.wbad[q][k];
        }
        bad[q] = b4;
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < kScanWaves; ++k)
            if (k < wid) s = s + w4[k];
        wb[q] = s;
        // the previous thread's total is zero: this base stays out of the
        // running maximum (0 is its identity for non-negative values)
        const double prev_thr = wave_shift_up1(thr[q]);
        int prev_zero = 0;
#pragma unroll
        for (int k = 0; k < kScanWaves; ++k)
            if (k + 1 == wid) prev_zero = L.wlastz[q][k];
        prev_zero = (lane64 == 0) ? prev_zero : (prev_thr == 0.0 ? 1 : 0);
        wmx[q] = wave_incl_max(prev_zero ? 0.0 : s + excl[q]);
        if (lane64 == 63) L.wmax[q][wid] = wmx[q];
    }
    lds_barrier();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        double m4[kScanWaves], w4[kScanWaves];
#pragma unroll
        for (int k = 0; k < kScanWaves; ++k) {
            m4[k] = L.wmax[q][k];
            w4[k] = L.wtot[q][k];
        }
        double prev = 0.0, prev_next = 0.0;
#pragma unroll
        for (int k = 0; k < kScanWaves; ++k) {
            if (k < wid) prev = fmax(prev, m4[k]);
            if (k <= wid) prev_next = fmax(prev_next, m4[k]);
        }
        const double gamma = fmax(wmx[q], prev);
        // base of the next thread: the next lane's, or for lane 63 the base of
        // the next wave's lane 0, fmax(wave base, running maximum so far)
        double gnext = wave_shift_down1(gamma);
        if (lane64 == 63) {
            double wbn = wb[q];
#pragma unroll
            for (int k = 0; k < kScanWaves; ++k)
                if (k == wid) wbn = wbn + w4[k];
            if (thr[q] == 0.0) wbn = 0.0;   // kept out of the running maximum
            gnext = (wid == kScanWaves - 1) ? __builtin_huge_val() : fmax(wbn, prev_next);
        }
        // once a thread's running sum has reached its total (its last positive
        // total and the zeros after it), the output is the next base itself,
        // unless the thread ends the sequence (a thread whose total is zero
        // has gnext == gamma already)
        const bool pin = thr[q] > 0.0 && si[q].e < so[q].n;
        const int64_t a = si[q].a, e = si[q].e, n = so[q].n;
        double p = 0.0;
        if (si[q].in_regs) {
            // outputs from the running sums of the first pass, for the
            // workgroup-uniform count per thread (a scalar branch); past the
            // range they repeat the thread's total and go to a spare LDS slot,
            // so that only the addresses depend on the range
            const int cnt = static_cast<int>(e - a);   // 0 .. per
            double* const dst = so[q].out_lds ? so[q].out_lds + a : nullptr;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                if (k < si[q].per) {
                    const double o = (pin && pre[q][k] == thr[q]) ? gnext : fmin(gamma + pre[q][k], gnext);
                    if (so[q].out_lds) *((k < cnt) ? dst + k : &L.spare[q]) = o;
                    if (so[q].out_gl && k < cnt) so[q].out_gl[a + k] = o;
                }
            }
            // the last output is the one of the thread's total (the sums repeat
            // it past the range)
            if (a <= n - 1 && n - 1 < e) L.last[q] = fmin(gamma + thr[q], gnext);
        } else {
            for (int64_t j0 = a; j0 < e; j0 += kScanBatch) {
                double x[kScanBatch];
#pragma unroll
                for (int k = 0; k < kScanBatch; ++k) x[k] = (j0 + k < e) ? so[q].in[j0 + k] : 0.0;
#pragma unroll
                for (int k = 0; k < kScanBatch; ++k) {
                    const int64_t j = j0 + k;
                    if (j < e) {
                        p = p + x[k];
                        const double o = (pin && p == thr[q]) ? gnext : fmin(gamma + p, gnext);
                        if (so[q].out_lds) so[q].out_lds[j] = o;
                        if (so[q].out_gl) so[q].out_gl[j] = o;
                        if (j == n - 1) L.last[q] = o;
                    }
                }
            }
        }
        if (n == 0 && t == 0) L.last[q] = 0.0;
    }
    lds_barrier();
    total[0] = L.last[0];
    total[1] = L.last[1];
}

// ---------------------------------------------------------------------------
// Sorted uniforms from the stored in-block prefixes: for draw i in spacing
// block g,  Z_i = min(beta_g + Zrel_i, beta_{g+1})  (Z_i = beta_{g+1} at the
// block's last draw) and  u_i = Z_i / Z_N.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double uniform_of(double zrel, int64_t i, int64_t N, double beta_g,
                                             double beta_n, double ztot) {
    const int64_t g = i / kZBlock;
    const int64_t ilast = (g * kZBlock + kZBlock - 1 < N) ? g * kZBlock + kZBlock - 1 : N;
    const double Z = (i == ilast) ? beta_n : fmin(beta_g + zrel, beta_n);
    return Z / ztot;
}

// Uniform i of the stratified, (i + v_i) / N, or systematic, (i + v_0) / N,
// scheme, with v_d the open-interval variate of draw d of (seed, stream).
__device__ __forceinline__ double scheme_uniform(const ZArgs& za, int64_t i) {
    const uint64_t d = (za.scheme == kSchemeSystematic) ? 0 : static_cast<uint64_t>(i);
    const uint64_t pair = d >> 1;
    const Words4 x = philox4x32_10(static_cast<uint32_t>(pair), static_cast<uint32_t>(pair >> 32),
                                   static_cast<uint32_t>(za.stream),
                                   static_cast<uint32_t>(za.stream >> 32),
                                   static_cast<uint32_t>(za.seed),
                                   static_cast<uint32_t>(za.seed >> 32));
    const double v = (d & 1) ? variate_from_words(x.w2, x.w3) : variate_from_words(x.w0, x.w1);
    return (static_cast<double>(i) + v) / static_cast<double>(za.N);
}

// Uniform i formed from the stored in-block spacing prefix and the scanned
// spacing-block ends (the same values k_materialize_u writes), or by the
// scheme's formula.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double uniform_at(const ZArgs& za, double ztot, int64_t i) {
    if (za.scheme != kSchemeMultinomial) return scheme_uniform(za, i);
    const int64_t g = i / kZBlock;
    const double beta_g = (g == 0) ? 0.0 : za.beta[g - 1];
    return uniform_of(za.zrel[i], i, za.N, beta_g, za.beta[g], ztot);
}

__device__ __forceinline__ void store_uniforms(double* __restrict__ u, int64_t i0, int nout,
                                               const double (&out)[kLane], int vec_out) {
    if (nout == kLane && vec_out) {
        f64x2* q = reinterpret_cast<f64x2*>(u + i0);
#pragma unroll
        for (int v = 0; v < kLane / 2; ++v) q[v] = f64x2{out[2 * v], out[2 * v + 1]};
    } else {
        for (int k = 0; k < nout; ++k) u[i0 + k] = out[k];
    }
}

// ---------------------------------------------------------------------------
// k_carries: block-total scans (weights and spacings), totals and validity.
// ---------------------------------------------------------------------------
template <int R = kScanRegs>
__device__ __forceinline__ void carries_body(const WArgs& wa, const ZArgs& za, const SharedArgs& sh,
                                             int32_t* dev_status, double* total_out, ScanLds& L) {
    const int t = threadIdx.x;
    ScanIn<R> si[2];
    scan_load(wa.blk_tot, wa.nb, si[0]);
    scan_load(za.blk_tot, za.nb, si[1]);
    const ScanOut so[2] = {{wa.blk_tot, wa.nb, nullptr, wa.beta}, {za.blk_tot, za.nb, nullptr, za.beta}};
    double tot[2];
    int bad[2];
    scan_pair(si, so, L, tot, bad);
    if (t == 0) {
        int status = kStatusOk;
        if (wa.nb > 0) {
            if (bad[0] || !(tot[0] > 0.0) || !(tot[0] < __builtin_huge_val()))
                status = kStatusBadWeights;
            sh.totals[0] = tot[0];
            if (total_out) *total_out = tot[0];
        }
        if (za.nb > 0) sh.totals[1] = tot[1];
        sh.status[0] = status;
        if (dev_status) *dev_status = status;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_carries(WArgs wa, ZArgs za, SharedArgs sh,
                                                          int32_t* dev_status, double* total_out) {
    __shared__ ScanLds L;
    carries_body<kCarryScanRegs>(wa, za, sh, dev_status, total_out, L);
}

// ---------------------------------------------------------------------------
// k_materialize_w: one workgroup per (weight block, round of 16 sub-tiles).
// ---------------------------------------------------------------------------
template <typename Src>
__device__ __forceinline__ void k_materialize_w_body(Src w, WArgs wa, SharedArgs sh, double* __restrict__ W, int vec_ok) {
    using Elem = typename SrcElem<Src>::type;
    __shared__ double lane_tot[kThreads];
    // a full round passes through LDS twice: its weights, loaded as coalesced
    // 16-byte pieces, into the lane-chunk layout, then its outputs back out
    // as coalesced 16-byte stores
    __shared__ __attribute__((aligned(16))) double stage[kThreads * kLane];
    const int t = threadIdx.x;
    const int row = t / kRowLanes;
    const int lane = t % kRowLanes;
    const int64_t b = blockIdx.x / kWIters;
    const int it = blockIdx.x % kWIters;
    const int s = it * kRows + row;
    const int64_t blk0 = b * kWBlock;
    const int64_t round0 = blk0 + static_cast<int64_t>(it) * kRows * kSub;   // j0 = round0 + 16t
    const int64_t j0 = blk0 + static_cast<int64_t>(s) * kSub + lane * kLane;
    const int nv = clamp_count(wa.M - j0, kLane);
    const bool full = round0 + kThreads * kLane <= wa.M;   // workgroup-uniform
    // the weights and every base they need in one round trip (the indices
    // are in range whatever the status says)
    double x[kLane];
    if constexpr (std::is_pointer<Src>::value) {
        if (full && (vec_ok & 1)) {
            constexpr int kPer = 16 / sizeof(Elem);            // elements per 16-byte piece
            constexpr int kPieces = kLane / kPer;              // pieces per thread
            typedef Elem piece_t __attribute__((ext_vector_type(kPer)));
            const piece_t* src = reinterpret_cast<const piece_t*>(w + round0);
            piece_t v[kPieces];
#pragma unroll
            for (int m = 0; m < kPieces; ++m) v[m] = src[t + m * kThreads];
            Elem* st = reinterpret_cast<Elem*>(stage);
#pragma unroll
            for (int m = 0; m < kPieces; ++m)
                *reinterpret_cast<piece_t*>(st + (t + m * kThreads) * kPer) = v[m];
            lds_barrier();
#pragma unroll
            for (int k = 0; k < kLane; ++k) x[k] = static_cast<double>(st[t * kLane + k]);
        } else {
            src_chunk(w, j0, nv, (vec_ok & 1) != 0, x);
        }
    } else {
        src_chunk(w, j0, nv, (vec_ok & 1) != 0, x);
    }
    const int status = sh.status[0];
    const double total = sh.totals[0];
    const double sigma = (s == 0) ? 0.0 : wa.sub_end[b * kWSubPerBlock + s - 1];
    const double X = wa.sub_end[b * kWSubPerBlock + kWSubPerBlock - 1];
    const double beta_b = (b == 0) ? 0.0 : wa.beta[b - 1];
    const double beta_n = wa.beta[b];
    double p[kLane];
    p[0] = x[0];
#pragma unroll
    for (int k = 1; k < kLane; ++k) p[k] = p[k - 1] + x[k];
    lane_tot[t] = p[kLane - 1];
    lds_barrier();   // also: every thread has read its weights from the stage
    double lv[kRowLanes];
#pragma unroll
    for (int k = 0; k < kRowLanes; ++k) lv[k] = lane_tot[row * kRowLanes + k];
    double c = 0.0;
#pragma unroll
    for (int k = 0; k < kRowLanes; ++k)
        if (k < lane) c = c + lv[k];
    if (status != kStatusOk) return;   // workgroup-uniform
    double out[kLane];
#pragma unroll
    for (int k = 0; k < kLane; ++k) out[k] = block_end_at(sigma + (c + p[k]), X, beta_b, beta_n) / total;
    if (full && (vec_ok & 2)) {
#pragma unroll
        for (int k = 0; k < kLane; ++k) stage[t * kLane + k] = out[k];
        lds_barrier();
        const f64x2* st = reinterpret_cast<const f64x2*>(stage);
        f64x2* q = reinterpret_cast<f64x2*>(W + round0);
#pragma unroll
        for (int m = 0; m < kLane / 2; ++m) __builtin_nontemporal_store(st[t + m * kThreads], &q[t + m * kThreads]);
    } else {
        for (int k = 0; k < nv; ++k) W[j0 + k] = out[k];
    }
}

template <typename Tin>
__global__ __launch_bounds__(kThreads) void k_materialize_w(const Tin* __restrict__ w, WArgs wa, SharedArgs sh, double* __restrict__ W, int vec_ok) {
    k_materialize_w_body<const Tin*>(w, wa, sh, W, vec_ok);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_materialize_w_outer(Outer<T> w, WArgs wa, SharedArgs sh, double* __restrict__ W, int vec_ok) {
    k_materialize_w_body<Outer<T>>(w, wa, sh, W, vec_ok);
}

// ---------------------------------------------------------------------------
// k_materialize_u: one workgroup per spacing block of 4096 draws, 16 per thread.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_materialize_u(ZArgs za, SharedArgs sh,
                                                            double* __restrict__ u, int vec_out) {
    const int64_t g = blockIdx.x;
    if (za.scheme != kSchemeMultinomial) {
        const int64_t j0 = g * kZBlock + static_cast<int64_t>(threadIdx.x) * kLane;
        const int nj = clamp_count(za.N - j0, kLane);
        double o[kLane];
#pragma unroll
        for (int k = 0; k < kLane; ++k) o[k] = (k < nj) ? scheme_uniform(za, j0 + k) : 0.0;
        store_uniforms(u, j0, nj, o, vec_out);
        return;
    }
    const double beta_g = (g == 0) ? 0.0 : za.beta[g - 1];
    const double beta_n = za.beta[g];
    const double ztot = sh.totals[1];
    const int64_t i0 = g * kZBlock + static_cast<int64_t>(threadIdx.x) * kLane;
    const int nout = clamp_count(za.N - i0, kLane);   // draws i < N are output
    double zr[kLane];
    if (nout == kLane) {
        const f64x2* q = reinterpret_cast<const f64x2*>(za.zrel + i0);
#pragma unroll
        for (int v = 0; v < kLane / 2; ++v) {
            const f64x2 d = q[v];
            zr[2 * v] = d.x;
            zr[2 * v + 1] = d.y;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kLane; ++k) zr[k] = (k < nout) ? za.zrel[i0 + k] : 0.0;
    }
    double out[kLane];
#pragma unroll
    for (int k = 0; k < kLane; ++k) out[k] = uniform_of(zr[k], i0 + k, za.N, beta_g, beta_n, ztot);
    store_uniforms(u, i0, nout, out, vec_out);
}

// ---------------------------------------------------------------------------
// Inverse CMF against implicit cumulative weights, one uniform per quad of 4
// lanes.  The threshold x (S >= x  <=>  W >= u) is located level by level, as
// the divide-and-conquer sampler narrows its ranges (Alg. 5): the block
// (search of the block ends held in LDS, `sbeta`, every kstride-th end), the
// sub-tile (each lane of the quad reads a quarter of the block's stored
// sub-tile ends), the lane chunk (each lane re-sums a quarter of the one
// 256-weight sub-tile with the left-to-right rule of k_reduce) and the element.
// Each level costs one round trip to memory.
// ---------------------------------------------------------------------------
constexpr int kBetaLds = 4096;
constexpr int kQuad = 4;
constexpr int kUPerWG = kThreads / kQuad;
constexpr int kFinishMaxUPQ = 4;          // draws per quad in k_finish, at most
constexpr int64_t kFinishResident = 512;  // k_finish workgroups the chip holds at once (2 per CU)

// Location of the sub-tile that holds the first weight whose cumulative sum
// reaches x (the block and sub-tile levels of the search), for one quad.
struct SubtileLoc {
    int64_t b, blk0, jlast;
    int s, nsub;
    double beta_b, beta_n, sigma, X;   // X: the block's total (its last sub-tile end)
};

__device__ SubtileLoc locate_subtile(const WArgs& wa, const double* sbeta, int64_t kstride,
                                     int ns, double x, int qi) {
    const int64_t nb = wa.nb;
    // ---- block level: first b with beta_{b+1} >= x ----
    int qlo = 0, qhi = ns - 1;
    while (qlo < qhi) {
        const int mid = (qlo + qhi) >> 1;
        if (sbeta[mid] < x)
            qlo = mid + 1;
        else
            qhi = mid;
    }
    int64_t lo = static_cast<int64_t>(qlo) * kstride;
    int64_t hi = ((static_cast<int64_t>(qlo) + 1) * kstride < nb ? (qlo + 1) * kstride : nb) - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (wa.beta[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    SubtileLoc L;
    const int64_t b = lo;
    L.b = b;
    L.beta_b = (b == 0) ? 0.0 : ((b % kstride == 0) ? sbeta[b / kstride - 1] : wa.beta[b - 1]);
    L.beta_n = (kstride == 1) ? sbeta[b] : wa.beta[b];
    const double beta_b = L.beta_b, beta_n = L.beta_n;
    L.blk0 = b * kWBlock;
    const int64_t blen = (wa.M - L.blk0 < kWBlock) ? wa.M - L.blk0 : kWBlock;
    L.jlast = L.blk0 + blen - 1;
    const int nsub = static_cast<int>((blen + kSub - 1) / kSub);
    L.nsub = nsub;
    const double* se = wa.sub_end + b * kWSubPerBlock;
    // ---- sub-tile level: first s with end(s) >= x, where
    //      end(s) = min(beta_b + sigma_{s+1}, beta_{b+1}) and end(nsub-1) = beta_{b+1};
    //      the quad reads the block's 128 stored ends 64 contiguous bytes per
    //      load (lane qi the 16-byte pieces qi, qi + 4, ...: one cache line per
    //      quad and load, where a lane-per-quarter split touches four) and
    //      counts those below x.  The whole row lies in the workspace; entries
    //      past the block's last sub-tile are read but not counted. ----
    constexpr int kPerLane = kWSubPerBlock / kQuad;
    double e[kPerLane];   // e[k] = end of sub-tile se_index(k)
    {
        const f64x2* q = reinterpret_cast<const f64x2*>(se) + qi;
#pragma unroll
        for (int v = 0; v < kPerLane / 2; ++v) {
            const f64x2 d = q[kQuad * v];
            e[2 * v] = d.x;
            e[2 * v + 1] = d.y;
        }
    }
    auto se_index = [qi](int k) { return 2 * kQuad * (k >> 1) + 2 * qi + (k & 1); };
    // the block total: the last stored end, held by lane 3 of the quad
    const double X = quad_bcast(e[kPerLane - 1], kQuad - 1);
    L.X = X;
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < kPerLane; ++k)
        cnt += (se_index(k) < nsub - 1 && block_end_at(e[k], X, beta_b, beta_n) < x) ? 1 : 0;
    const int s = quad_sum(cnt);
    L.s = s;
    // sigma_s = stored end of sub-tile s-1, taken from the lane that read it
    double sig = 0.0;
#pragma unroll
    for (int k = 0; k < kPerLane; ++k)
        if (se_index(k) == s - 1) sig = e[k];
    L.sigma = (s == 0) ? 0.0 : quad_bcast(sig, ((s - 1) % (2 * kQuad)) >> 1);
    return L;
}

// The global sub-tile index alone (block * 128 + sub-tile) of the same
// search, reading the block's sub-tile ends eight at a time (few registers).
__device__ int64_t locate_subtile_index(const WArgs& wa, const double* sbeta, int64_t kstride,
                                        int ns, double x, int qi) {
    const int64_t nb = wa.nb;
    int qlo = 0, qhi = ns - 1;
    while (qlo < qhi) {
        const int mid = (qlo + qhi) >> 1;
        if (sbeta[mid] < x)
            qlo = mid + 1;
        else
            qhi = mid;
    }
    int64_t lo = static_cast<int64_t>(qlo) * kstride;
    int64_t hi = ((static_cast<int64_t>(qlo) + 1) * kstride < nb ? (qlo + 1) * kstride : nb) - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (wa.beta[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    const int64_t b = lo;
    const double beta_b = (b == 0) ? 0.0 : wa.beta[b - 1];
    const double beta_n = wa.beta[b];
    const int64_t blen = (wa.M - b * kWBlock < kWBlock) ? wa.M - b * kWBlock : kWBlock;
    const int nsub = static_cast<int>((blen + kSub - 1) / kSub);
    // the block's 128 stored ends, read as in locate_subtile: lane qi takes
    // the 16-byte pieces qi, qi + 4, ..., four at a time
    const f64x2* se = reinterpret_cast<const f64x2*>(wa.sub_end + b * kWSubPerBlock) + qi;
    const double X = wa.sub_end[b * kWSubPerBlock + kWSubPerBlock - 1];   // the block total
    constexpr int kPieces = kWSubPerBlock / (2 * kQuad);   // per lane
    int cnt = 0;
    for (int v4 = 0; v4 < kPieces; v4 += 4) {
#pragma unroll
        for (int v = v4; v < v4 + 4; ++v) {
            const f64x2 d = se[kQuad * v];
            const int s0 = 2 * kQuad * v + 2 * qi;
            cnt += (s0 < nsub - 1 && block_end_at(d.x, X, beta_b, beta_n) < x) ? 1 : 0;
            cnt += (s0 + 1 < nsub - 1 && block_end_at(d.y, X, beta_b, beta_n) < x) ? 1 : 0;
        }
    }
    return b * kWSubPerBlock + quad_sum(cnt);
}

// locate_subtile's result from locate_subtile_index and four loads of the
// sub-tile's bases: the same search and predicate with few registers.
__device__ SubtileLoc locate_subtile_lean(const WArgs& wa, const double* sbeta, int64_t kstride,
                                          int ns, double x, int qi) {
    const int64_t g = locate_subtile_index(wa, sbeta, kstride, ns, x, qi);
    SubtileLoc L;
    L.b = g / kWSubPerBlock;
    L.s = static_cast<int>(g % kWSubPerBlock);
    L.beta_b = (L.b == 0) ? 0.0 : wa.beta[L.b - 1];
    L.beta_n = wa.beta[L.b];
    L.blk0 = L.b * kWBlock;
    const int64_t blen = (wa.M - L.blk0 < kWBlock) ? wa.M - L.blk0 : kWBlock;
    L.jlast = L.blk0 + blen - 1;
    L.nsub = static_cast<int>((blen + kSub - 1) / kSub);
    L.X = wa.sub_end[L.b * kWSubPerBlock + kWSubPerBlock - 1];
    L.sigma = (L.s == 0) ? 0.0 : wa.sub_end[L.b * kWSubPerBlock + L.s - 1];
    return L;
}

// kLean: for a caller at its register limit (the dense map's wide chunks):
// the lean sub-tile location, and chunk totals summed one chunk at a time, the
// chosen chunk loaded again for the element level.  Same sums, same index.
template <typename Src, bool kLean = false>
__device__ void map_quad(Src w, const WArgs& wa, const double* sbeta, int64_t kstride, int ns,
                         double x, int64_t i, int qi, int32_t* __restrict__ r, int vec_ok) {
    using Elem = typename SrcElem<Src>::type;
    SubtileLoc loc;
    if constexpr (kLean)
        loc = locate_subtile_lean(wa, sbeta, kstride, ns, x, qi);
    else
        loc = locate_subtile(wa, sbeta, kstride, ns, x, qi);
    const int64_t blk0 = loc.blk0, jlast = loc.jlast;
    const int s = loc.s;
    const double beta_b = loc.beta_b, beta_n = loc.beta_n, sigma = loc.sigma, X = loc.X;
    const int64_t sub0 = blk0 + static_cast<int64_t>(s) * kSub;
    const int slen = static_cast<int>((jlast - sub0 + 1 < kSub) ? jlast - sub0 + 1 : kSub);
    const int nl = (slen + kLane - 1) / kLane;
    // ---- lane-chunk level: lane qi sums chunks qi, qi + 4, qi + 8, qi + 12,
    //      so that a load of the quad spans 64 contiguous bytes per chunk row
    //      (two cache lines of binary32 weights where consecutive chunks per
    //      lane span four) ----
    constexpr int kChunks = kRowLanes / kQuad;
    static_assert(kQuad == 4 && kChunks == 4, "four lanes per quad, four chunks per lane");
    double tl[kChunks];   // tl[q] = total of chunk qi + 4q
    const bool full_sub = !kLean && (slen == kSub) && (vec_ok & 1);
    RawChunk<Elem> rc[kChunks];
    if constexpr (kLean) {
#pragma unroll 1
        for (int q = 0; q < kChunks; ++q) {
            const int l = qi + kQuad * q;
            const int nv = (l < nl) ? ((slen - l * kLane < kLane) ? slen - l * kLane : kLane) : 0;
            double xx[kLane];
            src_chunk(w, sub0 + l * kLane, nv, (vec_ok & 1) != 0, xx);
            const double ts = chunk_sum(xx);
#pragma unroll
            for (int qq = 0; qq < kChunks; ++qq)
                if (qq == q) tl[qq] = ts;
        }
    } else if (full_sub) {
#pragma unroll
        for (int q = 0; q < kChunks; ++q)
            rc[q] = src_raw(w, sub0 + (qi + kQuad * q) * kLane);
#pragma unroll
        for (int q = 0; q < kChunks; ++q) {
            Elem mn = static_cast<Elem>(0);
            tl[q] = raw_sum<Elem>(rc[q], mn);
        }
    } else {
#pragma unroll
        for (int q = 0; q < kChunks; ++q) {
            const int l = qi + kQuad * q;
            const int nv = (l < nl) ? ((slen - l * kLane < kLane) ? slen - l * kLane : kLane) : 0;
            double xx[kLane];
            src_chunk(w, sub0 + l * kLane, nv, (vec_ok & 1) != 0, xx);
            tl[q] = chunk_sum(xx);
        }
    }
    // left-to-right chunk starts c_l: c_{l+1} = c_l + (total of chunk l),
    // added by the lane that holds chunk l and passed to the whole quad, so
    // the sums are the same additions in the same order as one lane running
    // over all 16 chunks; cb[q] = start of chunk qi + 4q
    double cb[kChunks];
    {
        double run = 0.0;   // c_l, the same in every lane of the quad
#pragma unroll
        for (int q = 0; q < kChunks; ++q) {
            cb[q] = (qi == 0) ? run : 0.0;
            run = dpp_f64<kDppQuadBcast(0)>(run + tl[q]);
            cb[q] = (qi == 1) ? run : cb[q];
            run = dpp_f64<kDppQuadBcast(1)>(run + tl[q]);
            cb[q] = (qi == 2) ? run : cb[q];
            run = dpp_f64<kDppQuadBcast(2)>(run + tl[q]);
            cb[q] = (qi == 3) ? run : cb[q];
            run = dpp_f64<kDppQuadBcast(3)>(run + tl[q]);
        }
    }
    // each lane finds the first of its chunks ending at >= x; the quad's
    // first such chunk (the ends are non-decreasing) is the smallest of these
    // and its lane takes the element level
    constexpr int kNone = kRowLanes;
    int lmine = kNone;
#pragma unroll
    for (int q = kChunks - 1; q >= 0; --q) {
        const int l = qi + kQuad * q;
        const double en = block_end_at(sigma + (cb[q] + tl[q]), X, beta_b, beta_n);
        lmine = (l < nl && en >= x) ? l : lmine;
    }
    int lf = min(lmine, dpp_i32<kDppQuadSwap1>(lmine));
    lf = min(lf, dpp_i32<kDppQuadSwap2>(lf));
    if (lf == kNone) lf = nl - 1;   // unreachable: the sub-tile's end is >= x by the search above
    const int owner = lf % kQuad;
    double cf = cb[0];   // start of chunk lf, in its lane
#pragma unroll
    for (int q = 1; q < kChunks; ++q) cf = (q == lf / kQuad) ? cb[q] : cf;
    if (qi != owner) return;
    // ---- element level, by the lane that summed chunk lf ----
    const int64_t l0 = sub0 + static_cast<int64_t>(lf) * kLane;
    const int nv = (slen - lf * kLane < kLane) ? slen - lf * kLane : kLane;
    double xx[kLane];
    if (full_sub) {   // the chunk is still in registers
        RawChunk<Elem> sel = rc[0];
#pragma unroll
        for (int q = 1; q < kChunks; ++q)
            if (q == lf / kQuad) sel = rc[q];
#pragma unroll
        for (int k = 0; k < kLane; ++k) xx[k] = sel.at(k);
    } else {
        src_chunk(w, l0, nv, (vec_ok & 1) != 0, xx);
    }
    // the running sum is the only dependent chain: every element's end is
    // formed and compared (independent work), and the first one reaching x
    // is taken from a bit mask rather than by leaving the loop
    double pk = 0.0;
    unsigned hit = 0;
#pragma unroll
    for (int k = 0; k < kLane; ++k) {
        pk = pk + xx[k];
        const double en = block_end_at(sigma + (cf + pk), X, beta_b, beta_n);
        hit |= (k < nv && en >= x) ? (1u << k) : 0u;
    }
    const int64_t jr = hit ? l0 + __builtin_ctz(hit) : l0 + nv - 1;
    r[i] = static_cast<int32_t>(jr);
}

// Map of draws 64c .. 64c+63 with the scanned block ends read from memory
// (after k_carries).  All threads call it; sbeta is kBetaLds doubles of LDS.
template <typename Src>
__device__ __forceinline__ void map_chunk(Src w, const WArgs& wa, const ZArgs& za,
                                          const SharedArgs& sh, double* __restrict__ u_out,
                                          int32_t* __restrict__ r, int vec_ok, int64_t c,
                                          double* sbeta) {
    const int64_t N = za.N;
    const int t = threadIdx.x;
    const int64_t nb = wa.nb;
    const int64_t kstride = (nb + kBetaLds - 1) / kBetaLds;
    const int ns = static_cast<int>((nb + kstride - 1) / kstride);
    for (int q = t; q < ns; q += kThreads) {
        const int64_t b = (static_cast<int64_t>(q) + 1) * kstride - 1;
        sbeta[q] = wa.beta[b < nb ? b : nb - 1];
    }
    const int64_t i = c * kUPerWG + (t / kQuad);
    const bool ok = sh.status[0] == kStatusOk;
    double x = 0.0;
    if (i < N) {
        const double uu = uniform_at(za, sh.totals[1], i);
        if (u_out && (t & (kQuad - 1)) == 0) u_out[i] = uu;
        if (ok) x = threshold_for(uu, sh.totals[0]);
    }
    lds_barrier();
    if (i >= N) return;   // the four lanes of a quad share i
    if (!ok) {
        if ((t & (kQuad - 1)) == 0) r[i] = -1;
        return;
    }
    map_quad<Src>(w, wa, sbeta, kstride, ns, x, i, t & (kQuad - 1), r, vec_ok);
}

template <typename Tin>
__global__ __launch_bounds__(kThreads) void k_map_fused(const Tin* __restrict__ w, WArgs wa, ZArgs za,
                                                        SharedArgs sh, double* __restrict__ u_out,
                                                        int32_t* __restrict__ r, int vec_ok) {
    __shared__ double sbeta[kBetaLds];
    map_chunk<const Tin*>(w, wa, za, sh, u_out, r, vec_ok, blockIdx.x, sbeta);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_map_fused_outer(Outer<T> w, WArgs wa, ZArgs za,
                                                              SharedArgs sh, double* __restrict__ u_out,
                                                              int32_t* __restrict__ r) {
    __shared__ double sbeta[kBetaLds];
    map_chunk<Outer<T>>(w, wa, za, sh, u_out, r, 1, blockIdx.x, sbeta);
}

// ---------------------------------------------------------------------------
// Inverse CMF in the dense regime (several uniforms per sub-tile: the
// linear-merge limit of Alg. 5, where it behaves like Alg. 4).  A workgroup
// takes `per_wg` consecutive uniforms (16 per thread), chosen so that their
// span of weights usually fits one window of 16 sub-tiles; the first and the
// last are located by the quad search, which bounds the sub-tiles all of
// them fall in (the split of Alg. 5).  The span is re-summed a window at a
// time into LDS as normalised cumulative weights (the values of
// k_materialize_w); then every thread places its own 16 sorted uniforms that
// end in the window (the merge of Alg. 4, one run of uniforms per thread):
// a table of the window's value buckets narrows each uniform's search to a
// few entries, and the short bisections of several uniforms run
// interleaved, so no thread waits on a long chain of LDS reads.  A chunk whose
// span is wider than 64 sub-tiles takes one quad search per uniform instead.
// ---------------------------------------------------------------------------
constexpr int kDenseU = 4096;                 // most uniforms per workgroup
constexpr int kDensePer = kDenseU / kThreads;  // per thread
constexpr int kWinSub = 16;
constexpr int kWinLen = kWinSub * kSub;       // weights per window (= kThreads * kLane)
constexpr int kMaxWin = 4;
static_assert(kWinLen <= kBetaLds, "the window reuses the block-end stage");

// LDS slot of window entry i: within each group of 16 entries (the 16 a
// thread writes when it fills the window) the slots are rotated by the group's
// index, so that the 64 lanes of a wave writing their k-th entries spread over
// the banks instead of meeting in one.  Unsigned arithmetic (i >= 0): the
// searches compute this for every probe, and a signed quotient costs three
// more instructions each time.
__device__ __forceinline__ int win_slot(int i) {
    const unsigned u = static_cast<unsigned>(i);
    return static_cast<int>(u ^ ((u / kLane) & (kLane - 1)));
}

// Bucket index of a window of non-decreasing values: with lo the first value
// and hi the last, bucket(x) = floor((x - lo) * kBuckets / (hi - lo)) clamped
// to 0..kBuckets-1 (0 everywhere when the window has no width).  Every step
// (the subtraction, the product with a non-negative factor, the truncation
// and the clamp) is monotone in x, so bucket(sw[i]) < bucket(v) implies
// sw[i] < v, and bucket(sw[i]) > bucket(v) implies sw[i] > v.
constexpr int kBuckets = 2048;
constexpr int kPlaceGroup = 5;   // draws whose searches are interleaved (groups of 5, 5, 5, 1)

struct WinBuckets {
    double lo;
    double scale;
    __device__ __forceinline__ int of(double x) const {
        const double d = (x - lo) * scale;
        if (d >= static_cast<double>(kBuckets - 1)) return kBuckets - 1;
        return d > 0.0 ? static_cast<int>(d) : 0;
    }
};

// Fills tb[0..kBuckets] (16-bit entries; tbw is (kBuckets + 2) / 2 words of
// LDS whose first kBuckets / 2 words are zero and visible to every thread when
// this is called): tb[b] is the count of the window's first n = nwin-1
// entries whose bucket is below b.  Along the window the buckets do not
// decrease, so that count is the first entry whose bucket is >= b (n if none).
// Each entry adds one to its bucket's counter (two 16-bit counters per word,
// an entry count stays below 2^16), then the counters are scanned: thread t
// takes buckets 8t .. 8t+7.  Every tb[b] lies in 0..n whatever the values.
// Called by every thread of the workgroup.
__device__ __forceinline__ WinBuckets build_buckets(const double* sw, int nwin, uint32_t* tbw) {
    constexpr int kPerT = kBuckets / kThreads;
    static_assert(kBuckets % kThreads == 0 && kPerT % 2 == 0, "bucket words per thread");
    __shared__ int wtot[kThreads / 64];
    WinBuckets bm;
    bm.lo = sw[win_slot(0)];
    const double width = sw[win_slot(nwin - 1)] - bm.lo;
    double sc = (width > 0.0) ? static_cast<double>(kBuckets) / width : 0.0;
    if (!(sc <= 1.0e300)) sc = 0.0;
    bm.scale = sc;
    const int n = nwin - 1;
    const int t = threadIdx.x;
    for (int i = t; i < n; i += kThreads) {
        const int bi = bm.of(sw[win_slot(i)]);
        atomicAdd(&tbw[bi >> 1], (bi & 1) ? 0x10000u : 1u);
    }
    lds_barrier();
    uint32_t wv[kPerT / 2];
#pragma unroll
    for (int j = 0; j < kPerT / 2; ++j) wv[j] = tbw[t * (kPerT / 2) + j];
    int tot = 0;
#pragma unroll
    for (int j = 0; j < kPerT / 2; ++j) tot += static_cast<int>((wv[j] & 0xffffu) + (wv[j] >> 16));
    const int lane64 = t & 63;
    int incl = tot;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int v = __shfl_up(incl, d, 64);
        if (lane64 >= d) incl += v;
    }
    if (lane64 == 63) wtot[t >> 6] = incl;
    lds_barrier();
    int run = incl - tot;
    for (int q = 0; q < (t >> 6); ++q) run += wtot[q];
#pragma unroll
    for (int j = 0; j < kPerT / 2; ++j) {
        const uint32_t lo = static_cast<uint32_t>(run);
        run += static_cast<int>(wv[j] & 0xffffu);
        const uint32_t hi = static_cast<uint32_t>(run);
        run += static_cast<int>(wv[j] >> 16);
        tbw[t * (kPerT / 2) + j] = lo | (hi << 16);
    }
    if (t == kThreads - 1) reinterpret_cast<uint16_t*>(tbw)[kBuckets] = static_cast<uint16_t>(run);
    lds_barrier();
    return bm;
}

// Clears the bucket counters of tbw (before the barrier that precedes
// place_in_window).  Called by every thread of the workgroup.
__device__ __forceinline__ void clear_buckets(uint32_t* tbw) {
    static_assert(kBuckets / 2 == kThreads * 4, "one 16-byte store per thread");
    reinterpret_cast<uint4*>(tbw)[threadIdx.x] = make_uint4(0u, 0u, 0u, 0u);
}

// Places this thread's sorted values x[next..nmine) that end in a window of
// nwin non-decreasing values (entry i at sw[win_slot(i)]; those not above the
// window's last value, or
// all that remain in the final window): each one's position is the count of
// window entries below it among the first nwin-1.  For a value v in bucket b
// that count lies in [tb[b], tb[b+1]] (the monotone bucket map), and a
// bisection of that range finds it; the ranges of kPlaceGroup values are
// bisected together, so their LDS reads are in flight at once.
// res[q] = base + position; next moves past the values placed.  Called by
// every thread of the workgroup (the table is built here, in tbw: see
// build_buckets, its counters cleared by clear_buckets before the barrier
// that precedes this call).
__device__ __forceinline__ void place_in_window(const double* sw, uint32_t* tbw, int nwin,
                                                bool final_window,
                                                const double (&x)[kDensePer], int nmine,
                                                int64_t base, int& next,
                                                int32_t (&res)[kDensePer]) {
    const WinBuckets bm = build_buckets(sw, nwin, tbw);
    const uint16_t* tb = reinterpret_cast<const uint16_t*>(tbw);
    const double wend = sw[win_slot(nwin - 1)];
    int nxt = next;
#pragma unroll
    for (int g = 0; g < kDensePer; g += kPlaceGroup) {
        if (g < nmine) {
            // the position lies in [a, e]; slots past the thread's kDensePer
            // values (the last group) stay empty, removed once unrolled
            int a[kPlaceGroup], e[kPlaceGroup];
#pragma unroll
            for (int k = 0; k < kPlaceGroup; ++k) {
                const int q = g + k;
                a[k] = 0;
                e[k] = 0;
                if (q < kDensePer) {
                    const bool act = q >= next && q < nmine && (final_window || x[q] <= wend);
                    const int b = bm.of(x[q]);
                    const int ta = tb[b];
                    const int te = tb[b + 1];
                    a[k] = act ? ta : 0;
                    e[k] = act ? te : 0;
                    if (act) nxt = q + 1;
                }
            }
            // a and e stay in 0..nwin-1, so every probe reads inside the window
            for (;;) {
                int m[kPlaceGroup];
                double sv[kPlaceGroup];
#pragma unroll
                for (int k = 0; k < kPlaceGroup; ++k) m[k] = (a[k] + e[k]) >> 1;
#pragma unroll
                for (int k = 0; k < kPlaceGroup; ++k)
                    if (g + k < kDensePer) sv[k] = sw[win_slot(m[k])];
                bool more = false;
#pragma unroll
                for (int k = 0; k < kPlaceGroup; ++k) {
                    if (g + k < kDensePer) {
                        const bool go = a[k] < e[k];
                        const bool below = sv[k] < x[g + k];
                        a[k] = (go && below) ? m[k] + 1 : a[k];
                        e[k] = (go && !below) ? m[k] : e[k];
                        more = more || a[k] < e[k];
                    }
                }
                if (!more) break;
            }
#pragma unroll
            for (int k = 0; k < kPlaceGroup; ++k) {
                const int q = g + k;
                if (q < kDensePer && q >= next && q < nxt) res[q] = static_cast<int32_t>(base + a[k]);
            }
        }
    }
    next = nxt;
}

// Spans of the dense-map chunks: chunk c (uniforms c*per_wg .. c1-1) covers
// the sub-tiles from that of its first uniform to that of its last (the split
// of Alg. 5).  One quad locates each end, 32 chunks per workgroup;
// span[2c] and span[2c+1] receive the global sub-tile ids.  Nothing is
// written when the status is not ok (the map then writes -1 without reading
// the spans).
__global__ __launch_bounds__(kThreads) void k_dense_span(WArgs wa, ZArgs za, SharedArgs sh,
                                                         int64_t* __restrict__ span, int per_wg,
                                                         int64_t nchunks) {
    __shared__ double sbeta[kBetaLds];
    const int t = threadIdx.x;
    const int64_t nb = wa.nb;
    const int64_t kstride = (nb + kBetaLds - 1) / kBetaLds;
    const int ns = static_cast<int>((nb + kstride - 1) / kstride);
    for (int q = t; q < ns; q += kThreads) {
        const int64_t b = (static_cast<int64_t>(q) + 1) * kstride - 1;
        sbeta[q] = wa.beta[b < nb ? b : nb - 1];
    }
    const bool ok = sh.status[0] == kStatusOk;
    const int64_t e = static_cast<int64_t>(blockIdx.x) * (kThreads / kQuad) + t / kQuad;
    const int64_t c = e >> 1;
    const bool mine = ok && c < nchunks;   // the same for the four lanes of a quad
    double x = 0.0;
    if (mine) {
        const int64_t c0 = c * per_wg;
        const int64_t c1 = (c0 + per_wg < za.N) ? c0 + per_wg : za.N;
        x = threshold_for(uniform_at(za, sh.totals[1], (e & 1) ? c1 - 1 : c0), sh.totals[0]);
    }
    lds_barrier();   // the block ends are in LDS
    if (!mine) return;
    const int64_t g = locate_subtile_index(wa, sbeta, kstride, ns, x, t & (kQuad - 1));
    if ((t & (kQuad - 1)) == 0) span[e] = g;
}

// The loads one thread makes for a window row: its lane chunk of global
// sub-tile ws0 + row and the bases that chunk's cumulative values need.
template <typename Elem>
struct WinRowLoad {
    RawChunk<Elem> rc;
    double sigma, X, beta_b, beta_n;
    int nv;
};

template <typename Src>
__device__ __forceinline__ WinRowLoad<typename SrcElem<Src>::type> window_row_load(
    Src w, const WArgs& wa, int64_t ws0, int64_t gs1, int row, int lane) {
    WinRowLoad<typename SrcElem<Src>::type> L;
    const int nw = static_cast<int>((gs1 - ws0 + 1 < kWinSub) ? gs1 - ws0 + 1 : kWinSub);
    const int64_t gs = ws0 + row;
    const int64_t b = gs / kWSubPerBlock;
    const int sb = static_cast<int>(gs % kWSubPerBlock);
    const int64_t j0 = b * kWBlock + static_cast<int64_t>(sb) * kSub + lane * kLane;
    L.nv = (row < nw) ? clamp_count(wa.M - j0, kLane) : 0;
    L.sigma = 0.0;
    L.X = 0.0;
    L.beta_b = 0.0;
    L.beta_n = 0.0;
    if (L.nv > 0) {
        L.sigma = (sb == 0) ? 0.0 : wa.sub_end[b * kWSubPerBlock + sb - 1];
        L.X = wa.sub_end[b * kWSubPerBlock + kWSubPerBlock - 1];
        L.beta_b = (b == 0) ? 0.0 : wa.beta[b - 1];
        L.beta_n = wa.beta[b];
    }
    L.rc = src_raw_n(w, j0, L.nv);
    return L;
}

// A chunk whose span is too wide for the windows: one quad search per
// uniform, with the block ends staged in sbeta (kBetaLds doubles of LDS).
// Called by every thread of the workgroup.
template <typename Src>
__device__ __forceinline__ void map_wide_chunk(Src w, const WArgs& wa, const ZArgs& za, double total,
                                               double ztot, int64_t c0, int64_t c1,
                                               int32_t* __restrict__ r, int vec_ok, double* sbeta) {
    const int t = threadIdx.x;
    const int64_t nb = wa.nb;
    const int64_t kstride = (nb + kBetaLds - 1) / kBetaLds;
    const int ns = static_cast<int>((nb + kstride - 1) / kstride);
    for (int q = t; q < ns; q += kThreads) {
        const int64_t b = (static_cast<int64_t>(q) + 1) * kstride - 1;
        sbeta[q] = wa.beta[b < nb ? b : nb - 1];
    }
    lds_barrier();
    for (int64_t i = c0 + t / kQuad; i < c1; i += kUPerWG) {
        const double x = threshold_for(uniform_at(za, ztot, i), total);
        map_quad<Src, true>(w, wa, sbeta, kstride, ns, x, i, t & (kQuad - 1), r, vec_ok);
    }
}

template <typename Src>
__device__ __forceinline__ void k_map_dense_body(Src w, WArgs wa, ZArgs za, SharedArgs sh, const int64_t* __restrict__ span, double* __restrict__ u_out, int32_t* __restrict__ r, int vec_ok, int per_wg) {
    using Elem = typename SrcElem<Src>::type;
    // a window of normalised cumulative weights, its bucket table and the
    // lane-chunk totals of its rows
    __shared__ double sw[kWinLen];
    __shared__ double ltot[kThreads];
    __shared__ __attribute__((aligned(16))) uint32_t tbw[(kBuckets + 2) / 2];
    const int t = threadIdx.x;
    const int64_t N = za.N;
    const int64_t c0 = static_cast<int64_t>(blockIdx.x) * per_wg;
    const int64_t c1 = (c0 + per_wg < N) ? c0 + per_wg : N;
    const int64_t iu0 = c0 + static_cast<int64_t>(t) * kDensePer;
    const int nmine = clamp_count(c1 - iu0, kDensePer);
    // every load whose address is known at the start goes out together: the
    // status, the totals, the chunk's span, and this thread's in-block spacing
    // prefixes and spacing block ends (its 16 draws lie in one spacing block:
    // 16 divides 4096 and per_wg).  All lie in the workspace whatever the
    // status says; nothing is used before the status is checked.
    const int status = sh.status[0];
    const double total = sh.totals[0];
    const double ztot = sh.totals[1];
    const int64_t gs0 = span[2 * static_cast<int64_t>(blockIdx.x)];
    const int64_t gs1 = span[2 * static_cast<int64_t>(blockIdx.x) + 1];
    const bool spacings = za.scheme == kSchemeMultinomial;
    double us[kDensePer];
    double zb = 0.0, zn = 0.0;
    if (spacings) {
        if (nmine == kDensePer) {
            const f64x2* q2 = reinterpret_cast<const f64x2*>(za.zrel + iu0);
#pragma unroll
            for (int v = 0; v < kDensePer / 2; ++v) {
                const f64x2 d = q2[v];
                us[2 * v] = d.x;
                us[2 * v + 1] = d.y;
            }
        } else {
#pragma unroll
            for (int q = 0; q < kDensePer; ++q) us[q] = (q < nmine) ? za.zrel[iu0 + q] : 0.0;
        }
        const int64_t gz = iu0 / kZBlock;
        zb = (gz == 0) ? 0.0 : za.beta[gz - 1];
        zn = za.beta[gz < za.nb ? gz : za.nb - 1];
    }
    if (status != kStatusOk) {
        for (int q = 0; q < nmine; ++q) r[iu0 + q] = -1;
        return;
    }
    // a span wider than kMaxWin windows takes one quad search per uniform
    // instead (map_wide_chunk)
    const bool is_wide = gs1 - gs0 + 1 > static_cast<int64_t>(kWinSub) * kMaxWin;
    const int row = t / kRowLanes;
    const int lane = t % kRowLanes;
    // the first window's loads go out before the uniforms are formed
    WinRowLoad<Elem> cur{};
    if (!is_wide) cur = window_row_load(w, wa, gs0, gs1, row, lane);
    if (!spacings) {
#pragma unroll
        for (int q = 0; q < kDensePer; ++q) us[q] = (q < nmine) ? scheme_uniform(za, iu0 + q) : 0.0;
    } else {
#pragma unroll
        for (int q = 0; q < kDensePer; ++q) us[q] = uniform_of(us[q], iu0 + q, N, zb, zn, ztot);
    }
    if (u_out) store_uniforms(u_out, iu0, nmine, us, (reinterpret_cast<uintptr_t>(u_out) & 15) == 0);
    if (is_wide) {   // workgroup-uniform
        map_wide_chunk<Src>(w, wa, za, total, ztot, c0, c1, r, vec_ok, sw);
        return;
    }
    int32_t res[kDensePer];
    int next = 0;   // this thread's first draw not placed yet (the draws are sorted)
#pragma unroll
    for (int q = 0; q < kDensePer; ++q) res[q] = 0;
    // one window: row r holds global sub-tile ws0 + r, so thread t writes
    // window entries 16t .. 16t+15, then the draws that end in it are placed
    auto window = [&](const WinRowLoad<Elem>& L, int64_t ws0) {
        const int nw = static_cast<int>((gs1 - ws0 + 1 < kWinSub) ? gs1 - ws0 + 1 : kWinSub);
        clear_buckets(tbw);
        {
            double pt = L.rc.at(0);
#pragma unroll
            for (int k = 1; k < kLane; ++k) pt = pt + L.rc.at(k);
            ltot[t] = pt;
        }
        lds_barrier();
        double c = 0.0;
        for (int k = 0; k < lane; ++k) c = c + ltot[row * kRowLanes + k];
        // normalised cumulative weights (the in-chunk prefixes summed again
        // from the raw values, same order); entries past the weights read +inf
        double pk = 0.0;
#pragma unroll
        for (int k = 0; k < kLane; ++k) {
            pk = (k == 0) ? L.rc.at(0) : pk + L.rc.at(k);
            const double S = block_end_at(L.sigma + (c + pk), L.X, L.beta_b, L.beta_n);
            sw[win_slot(t * kLane + k)] = (k < L.nv) ? S / total : __builtin_huge_val();
        }
        lds_barrier();
        // entries of the window that exist
        const int64_t wlen64 = wa.M - ws0 * kSub;
        const int nwin = (nw * kSub < wlen64) ? nw * kSub : static_cast<int>(wlen64);
        place_in_window(sw, tbw, nwin, false, us, nmine, ws0 * kSub, next, res);
        lds_barrier();   // ltot, the window and its table are rewritten by the next window
    };
    window(cur, gs0);   // the loads made before the uniforms
    for (int64_t ws0 = gs0 + kWinSub; ws0 <= gs1; ws0 += kWinSub)
        window(window_row_load(w, wa, ws0, gs1, row, lane), ws0);
    if (nmine == kDensePer && (reinterpret_cast<uintptr_t>(r + iu0) & 15) == 0) {
        int4* dst = reinterpret_cast<int4*>(r + iu0);
#pragma unroll
        for (int v = 0; v < kDensePer / 4; ++v)
            dst[v] = make_int4(res[4 * v], res[4 * v + 1], res[4 * v + 2], res[4 * v + 3]);
    } else {
#pragma unroll
        for (int q = 0; q < kDensePer; ++q)
            if (q < nmine) r[iu0 + q] = res[q];
    }
}

template <typename Tin>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_map_dense(const Tin* __restrict__ w, WArgs wa, ZArgs za, SharedArgs sh, const int64_t* __restrict__ span, double* __restrict__ u_out, int32_t* __restrict__ r, int vec_ok, int per_wg) {
    k_map_dense_body<const Tin*>(w, wa, za, sh, span, u_out, r, vec_ok, per_wg);
}

template <typename T>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_map_dense_outer(Outer<T> w, WArgs wa, ZArgs za, SharedArgs sh, const int64_t* __restrict__ span, double* __restrict__ u_out, int32_t* __restrict__ r, int vec_ok, int per_wg) {
    k_map_dense_body<Outer<T>>(w, wa, za, sh, span, u_out, r, vec_ok, per_wg);
}

// ---------------------------------------------------------------------------
// k_finish: everything after k_reduce in one launch, for up to 4096 weight
// blocks and 64 spacing blocks.  Every workgroup scans the block totals itself
// (the same scan as k_carries, so the same bits), forms the uniforms of its 64
// draws and maps them; workgroup 0 also publishes the scans, totals and status.
// ---------------------------------------------------------------------------
template <typename Src, int UPQ>
__device__ __forceinline__ void k_finish_body(Src w, WArgs wa, ZArgs za, SharedArgs sh, int32_t* dev_status, double* __restrict__ u_out, int32_t* __restrict__ r, int vec_ok) {
    static_assert(UPQ >= 1 && UPQ <= kFinishMaxUPQ, "draws per quad");
    __shared__ double sbeta[kBetaLds];
    __shared__ double szbeta[kFinishMaxZBlocks];
    __shared__ ScanLds L;
    const int t = threadIdx.x;
    const int qi = t & (kQuad - 1);
    const bool lead = blockIdx.x == 0;
    // the workgroup's draws: UPQ rounds of 64, quad t/4 taking draw
    // i0 + 64k + t/4 in round k
    const int64_t i0 = static_cast<int64_t>(blockIdx.x) * kUPerWG * UPQ + (t / kQuad);
    // every independent load first: the block totals of both scans and the
    // in-block spacing prefixes of this quad's draws
    ScanIn<> si[2];
    scan_load(wa.blk_tot, wa.nb, si[0]);
    scan_load(za.blk_tot, za.nb, si[1]);
    const bool spacings = za.scheme == kSchemeMultinomial;
    double zrel[UPQ];
#pragma unroll
    for (int k = 0; k < UPQ; ++k) {
        const int64_t i = i0 + static_cast<int64_t>(k) * kUPerWG;
        zrel[k] = (spacings && i < za.N) ? za.zrel[i] : 0.0;
    }
    const ScanOut so[2] = {{wa.blk_tot, wa.nb, sbeta, nullptr}, {za.blk_tot, za.nb, szbeta, nullptr}};
    double tt[2];
    int bad[2];
    scan_pair(si, so, L, tt, bad);
    if (lead) {   // publish the scans, from LDS, with coalesced stores
        for (int64_t j = t; j < wa.nb; j += kThreads) wa.beta[j] = sbeta[j];
        for (int64_t j = t; j < za.nb; j += kThreads) za.beta[j] = szbeta[j];
    }
    const double tot = tt[0], ztot = tt[1];
    const int status =
        (bad[0] || !(tot > 0.0) || !(tot < __builtin_huge_val())) ? kStatusBadWeights : kStatusOk;
    if (lead && t == 0) {
        sh.status[0] = status;
        sh.totals[0] = tot;
        sh.totals[1] = ztot;
        if (dev_status) *dev_status = status;
    }
    // draw i (spacing prefix zk) of this quad
    auto one = [&](int64_t i, double zk) {
        const int64_t g = i / kZBlock;
        const double uu = spacings ? uniform_of(zk, i, za.N, (g == 0) ? 0.0 : szbeta[g - 1],
                                                szbeta[g], ztot)
                                   : scheme_uniform(za, i);
        if (u_out && qi == 0) u_out[i] = uu;
        if (status != kStatusOk) {
            if (qi == 0) r[i] = -1;
            return;
        }
        const double x = threshold_for(uu, tot);
        map_quad<Src>(w, wa, sbeta, 1, static_cast<int>(wa.nb), x, i, qi, r, vec_ok);
    };
    if constexpr (UPQ == 1) {
        if (i0 < za.N) one(i0, zrel[0]);   // the four lanes of a quad share i
    } else {
#pragma unroll 1
        for (int k = 0; k < UPQ; ++k) {
            const int64_t i = i0 + static_cast<int64_t>(k) * kUPerWG;
            if (i >= za.N) break;
            double zk = zrel[0];   // zrel[k], selected without indexing registers
#pragma unroll
            for (int q = 1; q < UPQ; ++q) zk = (k == q) ? zrel[q] : zk;
            one(i, zk);
        }
    }
}

template <typename Tin, int UPQ>
__global__ __launch_bounds__(kThreads) void k_finish(const Tin* __restrict__ w, WArgs wa, ZArgs za, SharedArgs sh, int32_t* dev_status, double* __restrict__ u_out, int32_t* __restrict__ r, int vec_ok) {
    k_finish_body<const Tin*, UPQ>(w, wa, za, sh, dev_status, u_out, r, vec_ok);
}

template <typename T, int UPQ>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_finish_outer(Outer<T> w, WArgs wa, ZArgs za, SharedArgs sh, int32_t* dev_status, double* __restrict__ u_out, int32_t* __restrict__ r, int vec_ok) {
    k_finish_body<Outer<T>, UPQ>(w, wa, za, sh, dev_status, u_out, r, vec_ok);
}

// ---------------------------------------------------------------------------
// Small problems (at most kSmallBlocks weight blocks): k_reduce_small, with
// the sums of k_reduce.  A weight block reduced by 256 threads takes 8
// dependent rounds of loads, and a spacing block 16 dependent draws per
// thread; with only a few blocks that is the whole time of the reduce.  With
// 1024 threads a weight block has all its loads in flight at once (two lane
// chunks per thread), and a spacing block four lanes per 16-draw chunk.
// ---------------------------------------------------------------------------
constexpr int kSmallThreads = 1024;                   // threads of a k_reduce_small workgroup
constexpr int kSmallRounds = kSmallThreads / kThreads;  // weight rounds per workgroup

// Spacing block g by 1024 threads (reduce_z_block's sums, four times the
// threads): lane qi of quad c takes draws 4qi .. 4qi+3 of lane chunk c, and
// the chunk's running sum passes from lane to lane in draw order, so every
// prefix is the same left-to-right sum.  All threads call it.
template <int P>
__device__ __forceinline__ void reduce_z_block_quads(const ZArgs& za, int64_t g, double* lane_tot,
                                                     double* sub_tot) {
    const int t = threadIdx.x;
    const int c = t >> 2;   // lane chunk of the block (the thread of the 256-thread layout)
    const int qi = t & (kQuad - 1);
    const int row = c / kRowLanes;
    const int lane = c % kRowLanes;
    const int64_t i0 = g * kZBlock + static_cast<int64_t>(c) * kLane + 4 * qi;
    const int nv = clamp_count(za.N + 1 - i0, 4);
    double x[4];
#pragma unroll
    for (int k = 0; k < 4; k += 2) {
        double ze = 0.0, zo = 0.0;
        if (k < nv) spacing_pair<P>(static_cast<uint64_t>(i0 + k) >> 1, za.seed, za.stream, ze, zo);
        x[k] = (k < nv) ? ze : 0.0;
        x[k + 1] = (k + 1 < nv) ? zo : 0.0;
    }
    double p[4];
    double run = 0.0;   // the chunk's sum before lane ph's draws, in every lane
#pragma unroll
    for (int ph = 0; ph < kQuad; ++ph) {
        double a[4];
        a[0] = (ph == 0) ? x[0] : run + x[0];
#pragma unroll
        for (int k = 1; k < 4; ++k) a[k] = a[k - 1] + x[k];
        if (qi == ph) {
#pragma unroll
            for (int k = 0; k < 4; ++k) p[k] = a[k];
        }
        run = quad_bcast(a[3], ph);
    }
    if (qi == 0) lane_tot[c] = run;   // the chunk total
    lds_barrier();
    double lv[kRowLanes];
#pragma unroll
    for (int k = 0; k < kRowLanes; ++k) lv[k] = lane_tot[row * kRowLanes + k];
    double cb = 0.0;
#pragma unroll
    for (int k = 0; k < kRowLanes; ++k)
        if (k < lane) cb = cb + lv[k];
    if (lane == kRowLanes - 1 && qi == 0) sub_tot[row] = cb + lv[kRowLanes - 1];
    lds_barrier();
    double rv[kRows];
#pragma unroll
    for (int k = 0; k < kRows; ++k) rv[k] = sub_tot[k];
    double sigma = 0.0, total = 0.0;
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        if (k < row) sigma = sigma + rv[k];
        total = total + rv[k];
    }
    double zr[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) zr[k] = sigma + (cb + p[k]);
    if (nv == 4) {
        f64x2* q = reinterpret_cast<f64x2*>(za.zrel + i0);
        q[0] = f64x2{zr[0], zr[1]};
        q[1] = f64x2{zr[2], zr[3]};
    } else {
        for (int k = 0; k < nv; ++k) za.zrel[i0 + k] = zr[k];
    }
    if (t == 0) za.blk_tot[g] = total;
}

// Weight block b by 1024 threads: thread (q, row, lane) of the 256-thread
// layout q = t / 256 sums the lane chunks of rounds q and q + 4, both loaded
// at once; then k_reduce's epilogue (sub-tile totals, the chain of sub-tile
// ends, the block total; NaN for a block holding an inadmissible weight).
// All threads call it; lds holds kSmallLds doubles.
constexpr int kSmallLds = kSmallThreads / 64 * 256;   // 2 KB of staging per wave
static_assert(kSmallLds >= kWIters * kThreads + 2 * kWSubPerBlock, "the epilogue's LDS");

// Lane chunks of two 1024-weight ranges of a block (the wave's chunks of two
// rounds; range r holds n[r] weights, the rest read as zeros), for the 64
// lanes of a wave: every piece is loaded first, as
// coalesced 16-byte pieces of element-aligned addresses (a lane-strided load
// touches 64 cache lines per instruction, and one CU issues them all), then a
// quarter (binary64) or half (binary32) of a range at a time passes through
// the wave's 2 KB of LDS to the lanes owning its chunks, each chunk's pieces
// rotated by the chunk's index against bank conflicts.  tsum[r] = the left-
// to-right sum of the lane's chunk of range r; mn (0 on entry) falls to the
// smallest weight seen when one is negative.
template <typename Elem>
__device__ __forceinline__ void wide_chunk_sums(const Elem* __restrict__ r0, const Elem* __restrict__ r1,
                                                const int (&n)[2], double* stage, double (&tsum)[2],
                                                Elem& mn) {
    typedef Elem piece_t __attribute__((ext_vector_type(16 / sizeof(Elem))));
    typedef Elem piece_ea __attribute__((ext_vector_type(16 / sizeof(Elem)), aligned(sizeof(Elem))));
    constexpr int kPer = 16 / sizeof(Elem);          // elements per piece
    constexpr int kCP = kLane / kPer;                // pieces per chunk (8 or 4)
    constexpr int kLoads = kLane * 64 / kPer / 64;   // pieces per lane per range (8 or 4)
    constexpr int kStep = 2;                         // loads per pass through LDS (128 pieces)
    constexpr int kOwners = kStep * 64 / kCP;        // lanes served per pass (16 or 32)
    const int l64 = threadIdx.x & 63;
    piece_t pc[2][kLoads];
    const Elem* const rr[2] = {r0, r1};
#pragma unroll
    for (int rg = 0; rg < 2; ++rg) {
#pragma unroll
        for (int k = 0; k < kLoads; ++k) {
            const int e0 = (k * 64 + l64) * kPer;   // the piece's first element
            if (e0 + kPer <= n[rg]) {
                pc[rg][k] = *reinterpret_cast<const piece_ea*>(rr[rg] + e0);
            } else {
                piece_t v = {};
#pragma unroll
                for (int i = 0; i < kPer; ++i)
                    if (e0 + i < n[rg]) v[i] = rr[rg][e0 + i];
                pc[rg][k] = v;
            }
        }
    }
    piece_t* const st = reinterpret_cast<piece_t*>(stage);   // 128 pieces
#pragma unroll
    for (int rg = 0; rg < 2; ++rg) {
#pragma unroll
        for (int s0 = 0; s0 < kLoads; s0 += kStep) {
#pragma unroll
            for (int k = s0; k < s0 + kStep; ++k) {
                const int pl = (k - s0) * 64 + l64;   // piece of this pass
                const int c = pl / kCP, j = pl % kCP;
                st[c * kCP + (j ^ (c & (kCP - 1)))] = pc[rg][k];
            }
            __builtin_amdgcn_s_waitcnt(kWaitLdsOnly);   // the wave's writes are done
            __builtin_amdgcn_wave_barrier();
            const int c = l64 - (s0 / kStep) * kOwners;   // this lane's chunk in the pass
            if (c >= 0 && c < kOwners) {
                RawChunk<Elem> rc;
#pragma unroll
                for (int j = 0; j < kCP; ++j) rc.v[j] = st[c * kCP + (j ^ (c & (kCP - 1)))];
                tsum[rg] = raw_sum<Elem>(rc, mn);
            }
            __builtin_amdgcn_wave_barrier();   // the slot is rewritten by the next pass
        }
    }
}

template <typename Src>
__device__ __forceinline__ void reduce_w_block_wide(Src w, const WArgs& wa, int64_t b,
                                                    double* lds) {
    using Elem = typename SrcElem<Src>::type;
    double* lane_tot = lds;                              // [8][256]
    double* sub_tot = lds + kWIters * kThreads;          // [128]
    double* sub_end = sub_tot + kWSubPerBlock;           // [128]
    const int t = threadIdx.x;
    const int tr = t % kThreads;
    const int q = t / kThreads;
    const int row = tr / kRowLanes;
    const int lane = tr % kRowLanes;
    double t0 = 0.0, t1 = 0.0;
    Elem mn = static_cast<Elem>(0);
    if constexpr (std::is_pointer<Src>::value && sizeof(Elem) == 8) {
        // binary64 (a lane chunk is a whole cache line): the wave's chunks of
        // rounds q and q + 4, 1024 consecutive weights each, of which those
        // before M exist
        const int wv = t >> 6;
        const int64_t o0 = b * kWBlock + static_cast<int64_t>(q) * kRows * kSub +
                           static_cast<int64_t>(wv % (kThreads / 64)) * 64 * kLane;
        const int64_t o1 = o0 + static_cast<int64_t>(kSmallRounds) * kRows * kSub;
        const int n[2] = {clamp_count(wa.M - o0, 64 * kLane), clamp_count(wa.M - o1, 64 * kLane)};
        double ts[2] = {0.0, 0.0};
        wide_chunk_sums<Elem>(w + (n[0] > 0 ? o0 : 0), w + (n[1] > 0 ? o1 : 0), n, lds + wv * 256,
                              ts, mn);
        t0 = ts[0];
        t1 = ts[1];
        lds_barrier();   // the staging slots become the epilogue's
    } else {
        // binary32 chunks (two per cache line) and outer products: lane-strided
        const int64_t j0 = b * kWBlock + static_cast<int64_t>(q * kRows + row) * kSub + lane * kLane;
        const int64_t j1 = j0 + static_cast<int64_t>(kSmallRounds) * kRows * kSub;
        const RawChunk<Elem> r0 = src_raw_n(w, j0, clamp_count(wa.M - j0, kLane));
        const RawChunk<Elem> r1 = src_raw_n(w, j1, clamp_count(wa.M - j1, kLane));
        mn = r0.raw(0);
        t0 = raw_sum<Elem>(r0, mn);
        t1 = raw_sum<Elem>(r1, mn);
    }
    const int bad = block_any((mn < static_cast<Elem>(0)) ? 1 : 0);
    lane_tot[q * kThreads + tr] = t0;
    lane_tot[(q + kSmallRounds) * kThreads + tr] = t1;
    lds_barrier();
    if (t < kWSubPerBlock) {   // sub-tile 16 it + r: the 16 lane totals left to right
        const int it = t / kRows;
        const int r = t % kRows;
        const double* p = lane_tot + it * kThreads + r * kRowLanes;
        double lv[kRowLanes];
#pragma unroll
        for (int l = 0; l < kRowLanes; ++l) lv[l] = p[l];
        double c = lv[0];
#pragma unroll
        for (int l = 1; l < kRowLanes; ++l) c = c + lv[l];
        sub_tot[t] = c;
    }
    lds_barrier();
    if (t == 0) {
        double c = 0.0;
        for (int q0 = 0; q0 < kWSubPerBlock; q0 += 16) {
            double v[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) v[k] = sub_tot[q0 + k];
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                c = c + v[k];
                sub_end[q0 + k] = c;
            }
        }
    }
    lds_barrier();
    if (t < kWSubPerBlock) wa.sub_end[b * kWSubPerBlock + t] = sub_end[t];
    if (t == 0) {
        const double tot = sub_end[kWSubPerBlock - 1];
        wa.blk_tot[b] = (bad || !(tot < __builtin_huge_val())) ? __builtin_nan("") : tot;
    }
}

template <typename T, int P>
__global__ __launch_bounds__(kSmallThreads) void k_reduce_small(const T* __restrict__ w, WArgs wa,
                                                               ZArgs za) {
    __shared__ __attribute__((aligned(16))) double lds[kSmallLds];
    if (static_cast<int64_t>(blockIdx.x) < za.nb) {
        reduce_z_block_quads<P>(za, blockIdx.x, lds, lds + kSmallThreads);
        return;
    }
    reduce_w_block_wide<const T*>(w, wa, blockIdx.x - za.nb, lds);
}

template <typename T, int P>
__global__ __launch_bounds__(kSmallThreads) void k_reduce_small_outer(Outer<T> w, WArgs wa, ZArgs za) {
    __shared__ double lds[kWIters * kThreads + 2 * kWSubPerBlock];
    if (static_cast<int64_t>(blockIdx.x) < za.nb) {
        reduce_z_block_quads<P>(za, blockIdx.x, lds, lds + kSmallThreads);
        return;
    }
    reduce_w_block_wide<Outer<T>>(w, wa, blockIdx.x - za.nb, lds);
}

// ---------------------------------------------------------------------------
// Stage 3 alone: inverse CMF of sorted u against a given non-decreasing W.
// Each workgroup takes consecutive uniforms; its first and last uniform are
// located in the whole of W (a 64-ary search of one wave each, Alg. 2 with a
// wider split), which bounds the range every other uniform of the workgroup
// can fall in (the split of Alg. 5); each uniform is then located inside that
// range, from LDS when the range is short.  k_map_w takes 256 uniforms, one
// per thread; k_map_w_dense (N * 4 >= M) takes the dense map's runs of 16.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t lower_bound_clamped(const double* __restrict__ W, int64_t a,
                                                       int64_t b, double X) {
    while (a < b) {
        const int64_t m = (a + b) >> 1;
        if (W[m] < X)
            a = m + 1;
        else
            b = m;
    }
    return b;
}

// #{j in [0, M-1) : W_j < x} for non-decreasing W (= lower_bound_clamped(W,
// 0, M-1, x)) by a 64-ary search of one wave: each step probes 64 evenly
// spaced positions and keeps the stride between the last one below x and the
// next.  Every lane of the wave must call it; all return the same value.
__device__ __forceinline__ int64_t lower_bound_wave(const double* __restrict__ W, int64_t M,
                                                    double x) {
    const int lane = threadIdx.x & 63;
    int64_t lo = 0, hi = M - 1;   // the count lies in [lo, hi]
    while (lo < hi) {
        const int64_t stride = (hi - lo + 63) / 64;
        const int64_t j = lo + lane * stride;
        const bool below = j < hi && W[j] < x;
        const int k = __popcll(__ballot(below));
        if (k == 0) {
            hi = lo;
        } else {
            const int64_t nlo = lo + (k - 1) * stride + 1;
            const int64_t nhi = lo + k * stride;
            lo = nlo;
            hi = (nhi < hi) ? nhi : hi;
        }
    }
    return lo;
}

constexpr int kMapWStage = 4096;   // W entries a workgroup stages in LDS

__global__ __launch_bounds__(kThreads) void k_map_w(const double* __restrict__ W, int64_t M,
                                                    const double* __restrict__ u, int64_t N,
                                                    int32_t* __restrict__ r) {
    __shared__ double sw[kMapWStage];
    __shared__ int64_t range[2];
    const int t = threadIdx.x;
    const int64_t first = static_cast<int64_t>(blockIdx.x) * kThreads;
    const int64_t last = (first + kThreads < N ? first + kThreads : N) - 1;
    const int64_t i = first + t;
    const double x = (i <= last) ? u[i] : 0.0;
    // the range of the workgroup's uniforms: waves 0 and 1 locate the first
    // and the last one (the split of Alg. 5)
    if (t < 128) {
        const int64_t j = lower_bound_wave(W, M, u[(t < 64) ? first : last]);
        if ((t & 63) == 0) range[t >> 6] = j;
    }
    lds_barrier();
    const int64_t lo = range[0], hi = range[1];
    const int64_t len = hi - lo + 1;
    if (len <= kMapWStage) {
        // a short range (several uniforms per weight): W[lo..hi] into LDS,
        // each uniform located there
        for (int64_t q = t; q < len; q += kThreads) sw[q] = W[lo + q];
        lds_barrier();
        if (i <= last) {
            int a = 0, b = static_cast<int>(len) - 1;
            while (a < b) {
                const int m = (a + b) >> 1;
                if (sw[m] < x)
                    a = m + 1;
                else
                    b = m;
            }
            r[i] = static_cast<int32_t>(lo + b);
        }
    } else if (i <= last) {
        r[i] = static_cast<int32_t>(lower_bound_clamped(W, lo, hi, x));
    }
}

// Stage 3 in the dense regime (N * 4 >= M): per_wg consecutive uniforms per
// workgroup, 16 per thread, as in k_map_dense.  Waves 0 and 1 locate the
// first and the last uniform; the range of W between them is staged a window
// of kWinLen values at a time, and every thread places its own uniforms in
// it (place_in_window), the last window taking all that remain (the clamp).
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_map_w_dense(
    const double* __restrict__ W, int64_t M, const double* __restrict__ u, int64_t N,
    int32_t* __restrict__ r, int per_wg) {
    __shared__ double sw[kWinLen];
    __shared__ __attribute__((aligned(16))) uint32_t tbw[(kBuckets + 2) / 2];
    __shared__ int64_t range[2];
    const int t = threadIdx.x;
    const int64_t c0 = static_cast<int64_t>(blockIdx.x) * per_wg;
    const int64_t c1 = (c0 + per_wg < N) ? c0 + per_wg : N;
    const int64_t iu0 = c0 + static_cast<int64_t>(t) * kDensePer;
    const int nmine = clamp_count(c1 - iu0, kDensePer);
    double x[kDensePer];
#pragma unroll
    for (int q = 0; q < kDensePer; ++q) x[q] = (q < nmine) ? u[iu0 + q] : 0.0;
    if (t < 128) {
        const int64_t j = lower_bound_wave(W, M, u[(t < 64) ? c0 : c1 - 1]);
        if ((t & 63) == 0) range[t >> 6] = j;
    }
    lds_barrier();
    const int64_t lo = range[0], hi = range[1];
    int32_t res[kDensePer];
#pragma unroll
    for (int q = 0; q < kDensePer; ++q) res[q] = 0;
    int next = 0;
    for (int64_t ws0 = lo; ws0 <= hi; ws0 += kWinLen) {
        const int nwin = static_cast<int>((hi + 1 - ws0 < kWinLen) ? hi + 1 - ws0 : kWinLen);
        for (int k = t; k < nwin; k += kThreads) sw[win_slot(k)] = W[ws0 + k];
        clear_buckets(tbw);
        lds_barrier();
        place_in_window(sw, tbw, nwin, ws0 + kWinLen > hi, x, nmine, ws0, next, res);
        lds_barrier();   // the window is rewritten next
    }
    if (nmine == kDensePer && (reinterpret_cast<uintptr_t>(r + iu0) & 15) == 0) {
        int4* dst = reinterpret_cast<int4*>(r + iu0);
#pragma unroll
        for (int v = 0; v < kDensePer / 4; ++v)
            dst[v] = make_int4(res[4 * v], res[4 * v + 1], res[4 * v + 2], res[4 * v + 3]);
    } else {
#pragma unroll
        for (int q = 0; q < kDensePer; ++q)
            if (q < nmine) r[iu0 + q] = res[q];
    }
}

// ---------------------------------------------------------------------------
// Batched form.  k_batch_plan counts each filter's weight blocks, spacing
// blocks and map chunks and scans the counts into per-filter bases; the other
// kernels are launched over capacity-sized grids and map their workgroup to a
// filter by a search of those bases.  Each then runs the single-distribution
// block code on the filter's own view of the arrays.
// ---------------------------------------------------------------------------
static_assert(kBatchWBlock == kWBlock && kBatchZBlock == kZBlock, "block sizes");
constexpr int kStatusInvalid = 1;
constexpr int kStatusCapacity = 4;
constexpr int64_t kMaxSegM = 2147483647LL;
constexpr int64_t kMaxSegN = 2147483646LL;

__global__ __launch_bounds__(kPlanThreads) void k_batch_plan(BatchArgs ba, int32_t* dev_status) {
    constexpr int kPlanWaves = kPlanThreads / 64;
    __shared__ int64_t wtot[3][kPlanWaves];
    __shared__ int err;
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wid = t >> 6;
    if (t == 0) err = (ba.w_off[0] != 0 || ba.n_off[0] != 0) ? kStatusInvalid : kStatusOk;
    __syncthreads();
    // thread t takes filters [b0, b1): their counts of weight blocks, spacing
    // blocks and map chunks, summed
    const int64_t B = ba.B;
    const int64_t per = (B + kPlanThreads - 1) / kPlanThreads;
    const int64_t b0 = (static_cast<int64_t>(t) * per < B) ? static_cast<int64_t>(t) * per : B;
    const int64_t b1 = (b0 + per < B) ? b0 + per : B;
    auto counts = [&](int64_t b, int64_t (&c)[3]) {
        const int64_t M = ba.w_off[b + 1] - ba.w_off[b];
        const int64_t N = ba.n_off[b + 1] - ba.n_off[b];
        if (M < 1 || M > kMaxSegM || N < 0 || N > kMaxSegN) {
            err = kStatusInvalid;
            c[0] = c[1] = c[2] = 0;
        } else {
            c[0] = (M + kBatchWBlock - 1) / kBatchWBlock;
            c[1] = (N > 0) ? (N + 1 + kBatchZBlock - 1) / kBatchZBlock : 0;
            c[2] = (N + ba.chunk - 1) / ba.chunk;
        }
    };
    int64_t sum[3] = {0, 0, 0};
    for (int64_t b = b0; b < b1; ++b) {
        int64_t c[3];
        counts(b, c);
#pragma unroll
        for (int k = 0; k < 3; ++k) sum[k] += c[k];
    }
    // exclusive scan of the thread sums: within the wave by shuffles, then
    // the wave totals
    int64_t incl[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        incl[k] = sum[k];
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int64_t v = __shfl_up(incl[k], d, 64);
            if (lane >= d) incl[k] += v;
        }
        if (lane == 63) wtot[k][wid] = incl[k];
    }
    __syncthreads();
    int64_t base[3], total[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        int64_t before = 0, all = 0;
#pragma unroll
        for (int q = 0; q < kPlanWaves; ++q) {
            const int64_t v = wtot[k][q];
            before += (q < wid) ? v : 0;
            all += v;
        }
        base[k] = before + incl[k] - sum[k];
        total[k] = all;
    }
    for (int64_t b = b0; b < b1; ++b) {
        ba.wt_base[b] = base[0];
        ba.zt_base[b] = base[1];
        ba.mc_base[b] = base[2];
        int64_t c[3];
        counts(b, c);
#pragma unroll
        for (int k = 0; k < 3; ++k) base[k] += c[k];
    }
    __syncthreads();   // every thread's error report is in
    if (t == 0) {
        ba.wt_base[B] = total[0];
        ba.zt_base[B] = total[1];
        ba.mc_base[B] = total[2];
        int st = err;
        if (st == kStatusOk &&
            (total[0] > ba.wt_cap || total[1] > ba.zt_cap || total[2] > ba.mc_cap ||
             ba.w_off[B] > ba.sumM_cap || ba.n_off[B] > ba.sumN_cap))
            st = kStatusCapacity;
        ba.head[0] = st;
        ba.head[1] = st;
        if (dev_status) *dev_status = st;
    }
}

// Largest b in [0, B) with base[b] <= x, for non-decreasing base with
// base[0] = 0 <= x: a 64-ary search, one element per lane per step.  Every
// lane of the wave must call it.
__device__ __forceinline__ int find_segment(const int64_t* __restrict__ base, int B, int64_t x) {
    const int lane = threadIdx.x & 63;
    int lo = 0, hi = B;
    while (hi - lo > 1) {
        const int stride = (hi - lo + 63) / 64;
        const int idx = lo + lane * stride;
        const bool le = idx < hi && base[idx] <= x;
        const int k = __popcll(__ballot(le));   // a prefix of the lanes, k >= 1
        lo = lo + (k - 1) * stride;
        hi = (lo + stride < hi) ? lo + stride : hi;
    }
    return lo;
}

__device__ __forceinline__ WArgs seg_wargs(const BatchArgs& ba, int b) {
    WArgs a;
    const int64_t t0 = ba.wt_base[b];
    a.M = ba.w_off[b + 1] - ba.w_off[b];
    a.nb = ba.wt_base[b + 1] - t0;
    a.blk_tot = ba.wt_tot + t0;
    a.beta = ba.wt_beta + t0;
    a.sub_end = ba.wt_sub + t0 * kWSubPerBlock;
    a.chunk_tot = ba.wt_chunk + t0 * (kWSubPerBlock * kRowLanes);
    return a;
}

__device__ __forceinline__ ZArgs seg_zargs(const BatchArgs& ba, int b) {
    ZArgs a;
    const int64_t t0 = ba.zt_base[b];
    a.N = ba.n_off[b + 1] - ba.n_off[b];
    a.nb = ba.zt_base[b + 1] - t0;
    a.seed = ba.seed;
    a.stream = static_cast<uint64_t>(b);
    a.scheme = kSchemeMultinomial;
    a.zrel = ba.zrel + ba.n_off[b] + b;
    a.blk_tot = ba.zt_tot + t0;
    a.beta = ba.zt_beta + t0;
    return a;
}

__device__ __forceinline__ SharedArgs seg_shared(const BatchArgs& ba, int b) {
    SharedArgs a;
    a.status = ba.seg_status + b;
    a.totals = ba.seg_totals + 2 * static_cast<int64_t>(b);
    return a;
}

__device__ __forceinline__ int aligned16_flag(const void* p) {
    return (reinterpret_cast<uintptr_t>(p) & 15) == 0 ? 1 : 0;
}

// zt_cap workgroups draw spacing blocks and wt_cap reduce weight blocks,
// interleaved by tile_role.
template <typename Tin, int P>
__global__ __launch_bounds__(kThreads) void k_reduce_batched(const Tin* __restrict__ w, BatchArgs ba) {
    __shared__ __attribute__((aligned(16))) unsigned char sb0[ReduceSmem<Tin>::kBuf0];
    __shared__ __attribute__((aligned(16))) unsigned char sb1[ReduceSmem<Tin>::kBuf];
    __shared__ __attribute__((aligned(16))) unsigned char sb2[ReduceSmem<Tin>::kBuf];
    // the plan's status, the tile count and the tile's filter are looked up
    // together (the plan writes every base, so the search stays in range even
    // when it failed); nothing found is used before the status is checked
    const TileRole role = tile_role(blockIdx.x, ba.zt_cap, ba.wt_cap);
    const int64_t tile = role.idx;
    const int plan = ba.head[0];
    const int64_t* base = role.is_z ? ba.zt_base : ba.wt_base;
    const int64_t ntiles = base[ba.B];
    const int b = find_segment(base, ba.B, tile);
    const int64_t first = base[b];
    if (plan != kStatusOk || tile >= ntiles) return;
    if (role.is_z) {
        const ZArgs za = seg_zargs(ba, b);
        double* lane_tot = reinterpret_cast<double*>(sb0);
        reduce_z_block<P>(za, tile - first, lane_tot, lane_tot + kThreads);
        return;
    }
    const WArgs wa = seg_wargs(ba, b);
    const Tin* ws = w + ba.w_off[b];
    reduce_w_block<Tin>(ws, wa, tile - first, aligned16_flag(ws), sb0, sb1, sb2);
}

// One workgroup per filter: its block-total scans, totals and status.
__global__ __launch_bounds__(kScanThreads) void k_carries_batched(BatchArgs ba) {
    __shared__ ScanLds L;
    // a plan's graph launches one workgroup per filter it can hold; those
    // beyond the call's B have nothing to do
    if (ba.head[0] != kStatusOk || static_cast<int>(blockIdx.x) >= ba.B) return;
    const int b = blockIdx.x;
    const SharedArgs sh = seg_shared(ba, b);
    // a filter's few block totals: fewer of them held in registers (the
    // others are read again), so that more filters are resident at once;
    // the sums are the same either way
    carries_body<kBatchScanRegs>(seg_wargs(ba, b), seg_zargs(ba, b), sh, nullptr, nullptr, L);
    if (threadIdx.x == 0 && sh.status[0] != kStatusOk) atomicMax(ba.head + 1, kStatusBadWeights);
    // the filter of each of its map chunks, for the map's lookup
    const int64_t m0 = ba.mc_base[b], m1 = ba.mc_base[b + 1];
    for (int64_t c = m0 + threadIdx.x; c < m1; c += kScanThreads) ba.mc_seg[c] = b;
}

// ---------------------------------------------------------------------------
// Map of a chunk of kSegU consecutive draws with the sub-tiles shared between
// draws (the batched filters draw on average one index per 40 weights, and
// several draws fall in most touched sub-tiles).  The divide-and-conquer
// levels of Alg. 5, per workgroup:
//   block     every draw's block by a search of the block ends in LDS;
//   sub-tile  the sub-tile ends of the chunk's blocks staged in LDS once,
//             then a search per draw (a global search when the chunk spans
//             more blocks than the stage holds);
//   split     the distinct sub-tiles are compacted in draw order;
//   chunk     the 16 lane-chunk totals of every touched sub-tile (one load
//             per chunk, all in flight together), their left-to-right running
//             sums, then a search of the 16 chunk ends per draw;
//   element   each draw re-reads its chunk's 16 weights (just fetched, so
//             from cache) and counts the partial sums below its threshold.
// Comparisons are of unnormalised partial sums S_j with the threshold x of
// each draw (S_j >= x  <=>  W_j >= u).  Sums follow k_reduce's order.
// ---------------------------------------------------------------------------
// The draws per workgroup (kSegU: 256, 512 or 1024) and the touched
// sub-tiles per chunk pass are template parameters; the autotuner picks the
// draws per workgroup for a batch (the result does not depend on it).
constexpr int kSegBetaLds = 128;             // block ends kept in LDS (sampled beyond)
constexpr int kSegSubBlocks = 4;             // blocks whose sub-tile ends are staged
constexpr int kSegDraws = 1;                 // draws per thread in flight at the element level

// A touched sub-tile's 16 chunk values in LDS take 17 slots: with a row of
// exactly 16 doubles every thread of a wave walking its own row met the
// others in the same bank.
constexpr int kCrunStride = kRowLanes + 1;

template <int kSegU, int kSegPass>
struct SegLds {
    double sx[kSegU];                                  // thresholds, in draw order
    double sbeta[kSegBetaLds];
    double ssub[kSegSubBlocks * kWSubPerBlock];
    double crun[kSegPass * kCrunStride];               // chunk totals, then running sums
    int32_t sid[kSegU];                                // sub-tile of each draw, then r
    int16_t srank[kSegU];                              // rank of each draw's sub-tile
    int32_t lsub[kSegU];                               // touched sub-tiles
    int32_t lstart[kSegU + 1];                         // first draw of each
    int32_t wsum[kThreads / 64];
    int32_t span[2];
};

// First block b (0..nb-1) with beta_b >= x (beta_b = end of block b).
__device__ __forceinline__ int64_t seg_block_of(const WArgs& wa, const double* sbeta, int64_t kstride,
                                                int ns, double x) {
    int lo = 0, hi = ns - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (sbeta[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    int64_t blo = static_cast<int64_t>(lo) * kstride;
    int64_t bhi = ((static_cast<int64_t>(lo) + 1) * kstride < wa.nb ? (lo + 1) * kstride : wa.nb) - 1;
    while (blo < bhi) {
        const int64_t mid = (blo + bhi) >> 1;
        if (wa.beta[mid] < x)
            blo = mid + 1;
        else
            bhi = mid;
    }
    return blo;
}

template <typename Tin, int kSegU, int kSegPass>
__device__ void map_seg_chunk(const Tin* __restrict__ w, const WArgs& wa, const ZArgs& za,
                              const SharedArgs& sh, int32_t* __restrict__ r, int64_t c,
                              SegLds<kSegU, kSegPass>& L) {
    constexpr int kSegPer = kSegU / kThreads;
    const int t = threadIdx.x;
    const int64_t N = za.N;
    const int64_t i0 = c * kSegU;
    const int nu = static_cast<int>((N - i0 < kSegU) ? N - i0 : kSegU);   // >= 1
    // the filter's status and totals, and the spacing prefixes and spacing
    // block ends of the chunk's draws, in one round trip: every address is in
    // range whatever the status says
    const int status = sh.status[0];
    const double total = sh.totals[0];
    const double ztot = sh.totals[1];
    double zr[kSegPer], zlo[kSegPer], zhi[kSegPer];
#pragma unroll
    for (int k = 0; k < kSegPer; ++k) {
        const int pos = t + k * kThreads;
        const int64_t i = i0 + ((pos < nu) ? pos : nu - 1);
        const int64_t g = i / kZBlock;
        zr[k] = za.zrel[i];
        zlo[k] = (g == 0) ? 0.0 : za.beta[g - 1];
        zhi[k] = za.beta[g];
    }
    // the block ends in the same round trip (in range whatever the status)
    const int64_t nb = wa.nb;
    const int64_t kstride = (nb + kSegBetaLds - 1) / kSegBetaLds;
    const int ns = static_cast<int>((nb + kstride - 1) / kstride);
    for (int q = t; q < ns; q += kThreads) {
        const int64_t b = (static_cast<int64_t>(q) + 1) * kstride - 1;
        L.sbeta[q] = wa.beta[b < nb ? b : nb - 1];
    }
    if (status != kStatusOk) {
        for (int k = 0; k < kSegPer; ++k) {
            const int pos = t + k * kThreads;
            if (pos < nu) r[i0 + pos] = -1;
        }
        return;
    }
    // block end beta_b and the previous end, from LDS when every end is there
    auto beta_end = [&](int64_t b) { return (kstride == 1) ? L.sbeta[b] : wa.beta[b]; };
    // ---- thresholds of the chunk's draws (coalesced: position t + 256k) ----
    double xs[kSegPer];
#pragma unroll
    for (int k = 0; k < kSegPer; ++k) {
        const int pos = t + k * kThreads;
        xs[k] = __builtin_huge_val();
        if (pos < nu)
            xs[k] = threshold_for(uniform_of(zr[k], i0 + pos, N, zlo[k], zhi[k], ztot), total);
        L.sx[pos] = xs[k];
    }
    lds_barrier();
    // ---- block level, and the blocks spanned by the chunk ----
    int64_t bk[kSegPer];
    if (kstride == 1) {
        // count of block ends below x among the first ns-1, for the draws in
        // lock step (the last end is the total, never below x)
        int cnt[kSegPer] = {};
        for (int step = kSegBetaLds / 2; step >= 1; step >>= 1) {
#pragma unroll
            for (int k = 0; k < kSegPer; ++k)
                if (cnt[k] + step <= ns - 1 && L.sbeta[cnt[k] + step - 1] < xs[k]) cnt[k] += step;
        }
#pragma unroll
        for (int k = 0; k < kSegPer; ++k) bk[k] = cnt[k];
    } else {
#pragma unroll
        for (int k = 0; k < kSegPer; ++k)
            bk[k] = (t + k * kThreads < nu) ? seg_block_of(wa, L.sbeta, kstride, ns, xs[k]) : 0;
    }
#pragma unroll
    for (int k = 0; k < kSegPer; ++k) {
        const int pos = t + k * kThreads;
        if (pos >= nu) bk[k] = 0;
        if (pos == 0) L.span[0] = static_cast<int32_t>(bk[k]);
        if (pos == nu - 1) L.span[1] = static_cast<int32_t>(bk[k]);
    }
    lds_barrier();
    const int64_t bfirst = L.span[0], blast = L.span[1];
    const bool staged = blast - bfirst + 1 <= kSegSubBlocks;
    if (staged) {
        const int64_t n = (blast - bfirst + 1) * kWSubPerBlock;
        const double* src = wa.sub_end + bfirst * kWSubPerBlock;
        for (int q = t; q < n; q += kThreads) L.ssub[q] = src[q];
    }
    lds_barrier();
    // sigma_s of block b (stored end of sub-tile s-1; 0 for s = 0)
    auto sigma_of = [&](int64_t b, int s) {
        if (s == 0) return 0.0;
        return staged ? L.ssub[(b - bfirst) * kWSubPerBlock + s - 1]
                      : wa.sub_end[b * kWSubPerBlock + s - 1];
    };
    // ---- sub-tile level: first s with end(s) >= x, where
    //      end(s) = min(beta_{b-1} + sigma_{s+1}, beta_b), end(nsub-1) = beta_b ----
    {
        double bb[kSegPer], bn[kSegPer], bx[kSegPer];
        int nsub[kSegPer], cnt[kSegPer];
#pragma unroll
        for (int k = 0; k < kSegPer; ++k) {
            // unused positions search the first staged block (in range)
            if (t + k * kThreads >= nu) bk[k] = bfirst;
            const int64_t b = bk[k];
            bb[k] = (b == 0) ? 0.0 : beta_end(b - 1);
            bn[k] = beta_end(b);
            bx[k] = sigma_of(b, kWSubPerBlock);   // the block total
            const int64_t blen = (wa.M - b * kWBlock < kWBlock) ? wa.M - b * kWBlock : kWBlock;
            nsub[k] = static_cast<int>((blen + kSub - 1) / kSub);
            cnt[k] = 0;
        }
        // count of sub-tile ends below x among the first nsub-1, in lock step:
        // a bisection in LDS when the chunk's blocks are staged; otherwise two
        // rounds of independent loads from memory (the last end of each group
        // of 16 sub-tiles, then the 16 ends of the group holding the answer)
        if (staged) {
            for (int step = kWSubPerBlock / 2; step >= 1; step >>= 1) {
#pragma unroll
                for (int k = 0; k < kSegPer; ++k)
                    if (cnt[k] + step <= nsub[k] - 1 &&
                        block_end_at(sigma_of(bk[k], cnt[k] + step), bx[k], bb[k], bn[k]) < xs[k])
                        cnt[k] += step;
            }
        } else {
            constexpr int kGroup = 16;
            constexpr int kGroups = kWSubPerBlock / kGroup;
#pragma unroll 1
            for (int k = 0; k < kSegPer; ++k) {   // one draw at a time (few registers)
                const double* se = wa.sub_end + bk[k] * kWSubPerBlock;
                double e[kGroups];
#pragma unroll
                for (int g = 0; g < kGroups; ++g) e[g] = se[g * kGroup + kGroup - 1];
                int c1 = 0;
#pragma unroll
                for (int g = 0; g < kGroups; ++g)
                    c1 += (g * kGroup + kGroup - 1 < nsub[k] - 1 &&
                           block_end_at(e[g], bx[k], bb[k], bn[k]) < xs[k]) ? 1 : 0;
                const int g0 = (c1 < kGroups) ? c1 : kGroups - 1;
                double f[kGroup];
#pragma unroll
                for (int q = 0; q < kGroup; ++q) f[q] = se[g0 * kGroup + q];
                int c2 = 0;
#pragma unroll
                for (int q = 0; q < kGroup; ++q)
                    c2 += (c1 * kGroup + q < nsub[k] - 1 &&
                           block_end_at(f[q], bx[k], bb[k], bn[k]) < xs[k]) ? 1 : 0;
                cnt[k] = c1 * kGroup + ((c1 < kGroups) ? c2 : 0);
            }
        }
#pragma unroll
        for (int k = 0; k < kSegPer; ++k) {
            const int pos = t + k * kThreads;
            if (pos < nu) L.sid[pos] = static_cast<int32_t>(bk[k] * kWSubPerBlock + cnt[k]);
        }
    }
    lds_barrier();
    // ---- split: distinct sub-tiles in draw order (thread t owns positions
    //      4t..4t+3) ----
    int heads = 0;
    int hmask = 0;
#pragma unroll
    for (int k = 0; k < kSegPer; ++k) {
        const int pos = kSegPer * t + k;
        const bool h = pos < nu && (pos == 0 || L.sid[pos] != L.sid[pos - 1]);
        hmask |= h ? (1 << k) : 0;
        heads += h ? 1 : 0;
    }
    const int lane64 = t & 63;
    int incl = heads;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int v = __shfl_up(incl, d, 64);
        if (lane64 >= d) incl += v;
    }
    if (lane64 == 63) L.wsum[t >> 6] = incl;
    lds_barrier();
    int wbase = 0;
    for (int q = 0; q < (t >> 6); ++q) wbase += L.wsum[q];
    const int ntouched = L.wsum[0] + L.wsum[1] + L.wsum[2] + L.wsum[3];
    int rank = wbase + incl - heads - 1;
#pragma unroll
    for (int k = 0; k < kSegPer; ++k) {
        const int pos = kSegPer * t + k;
        if (hmask & (1 << k)) {
            ++rank;
            L.lsub[rank] = L.sid[pos];
            L.lstart[rank] = pos;
        }
        if (pos < nu) L.srank[pos] = static_cast<int16_t>(rank);
    }
    if (t == 0) L.lstart[ntouched] = nu;
    lds_barrier();
    // ---- chunk and element levels, kSegPass touched sub-tiles at a time ----
    const int row = t / kRowLanes;
    const int lane = t % kRowLanes;
    for (int p0 = 0; p0 < ntouched; p0 += kSegPass) {
        const int p1 = (p0 + kSegPass < ntouched) ? p0 + kSegPass : ntouched;
        // chunk totals: thread (row, lane) takes chunk `lane` of sub-tiles
        // p0+row+16m, stored by the reduce when it kept them, else re-summed
        if (wa.chunk_tot) {
#pragma unroll 4
            for (int k = p0 + row; k < p1; k += kRows)
                L.crun[(k - p0) * kCrunStride + lane] =
                    wa.chunk_tot[static_cast<int64_t>(L.lsub[k]) * kRowLanes + lane];
        } else {
#pragma unroll 4
        for (int k = p0 + row; k < p1; k += kRows) {
            const int32_t g = L.lsub[k];
            const int64_t b = g / kWSubPerBlock;
            const int64_t j0 = b * kWBlock + static_cast<int64_t>(g % kWSubPerBlock) * kSub +
                               lane * kLane;
            const int nv = clamp_count(wa.M - j0, kLane);
            const int64_t bend = b * kWBlock + kWBlock;
            const int nvb = (j0 + nv <= bend) ? nv : static_cast<int>(bend - j0);
            const RawChunk<Tin> rc = load_raw_n<Tin>(w + (nvb > 0 ? j0 : 0), nvb > 0 ? nvb : 0);
            // left to right from the first value, as k_reduce sums a chunk
            double cs = rc.at(0);
#pragma unroll
            for (int q = 1; q < kLane; ++q) cs = cs + rc.at(q);
            L.crun[(k - p0) * kCrunStride + lane] = cs;
        }
        }
        lds_barrier();
        // running sums c_{l+1} = c_l + t_l, left to right
        if (t < p1 - p0) {
            double run = 0.0;
#pragma unroll
            for (int l = 0; l < kRowLanes; ++l) {
                run = run + L.crun[t * kCrunStride + l];
                L.crun[t * kCrunStride + l] = run;
            }
        }
        lds_barrier();
        // draws of these sub-tiles, kSegDraws per thread at a time: chunk
        // searches in lock step, then all chunk loads, then the counts
        const int d0 = L.lstart[p0], d1 = L.lstart[p1];
        for (int pb = d0; pb < d1; pb += kSegDraws * kThreads) {
            int lc[kSegDraws], nv[kSegDraws], nl[kSegDraws];
            int64_t j0[kSegDraws];
            double bb[kSegDraws], bn[kSegDraws], sg[kSegDraws], cl[kSegDraws], xx[kSegDraws];
            double bx[kSegDraws];
            const double* cr[kSegDraws];
#pragma unroll
            for (int m = 0; m < kSegDraws; ++m) {
                const int pos = pb + t + m * kThreads;
                const bool v = pos < d1;
                const int k = v ? L.srank[pos] : p0;
                // sub-tile ids are not negative: unsigned quotients are shifts
                const uint32_t g = static_cast<uint32_t>(L.lsub[k]);
                const int64_t b = g / kWSubPerBlock;
                const int s = static_cast<int>(g % kWSubPerBlock);
                xx[m] = v ? L.sx[pos] : -__builtin_huge_val();
                const int64_t blk0 = b * kWBlock;
                const int64_t jlast = ((blk0 + kWBlock < wa.M) ? blk0 + kWBlock : wa.M) - 1;
                const int64_t sub0 = blk0 + static_cast<int64_t>(s) * kSub;
                const int slen = static_cast<int>((jlast - sub0 + 1 < kSub) ? jlast - sub0 + 1 : kSub);
                nl[m] = static_cast<int>(static_cast<unsigned>(slen + kLane - 1) / kLane);
                bb[m] = (b == 0) ? 0.0 : beta_end(b - 1);
                bn[m] = beta_end(b);
                sg[m] = sigma_of(b, s);
                bx[m] = sigma_of(b, kWSubPerBlock);   // the block total
                cr[m] = L.crun + (k - p0) * kCrunStride;
                j0[m] = sub0;
                nv[m] = slen;
                lc[m] = 0;
            }
            // first chunk whose end reaches x (the last chunk's end is end(s) >= x)
#pragma unroll
            for (int step = kRowLanes / 2; step >= 1; step >>= 1) {
#pragma unroll
                for (int m = 0; m < kSegDraws; ++m)
                    if (lc[m] + step <= nl[m] - 1 &&
                        block_end_at(sg[m] + cr[m][lc[m] + step - 1], bx[m], bb[m], bn[m]) <
                            xx[m])
                        lc[m] += step;
            }
            RawChunk<Tin> xv[kSegDraws];
#pragma unroll
            for (int m = 0; m < kSegDraws; ++m) {
                cl[m] = (lc[m] == 0) ? 0.0 : cr[m][lc[m] - 1];
                const int slen = nv[m];
                nv[m] = (pb + t + m * kThreads < d1)
                            ? ((slen - lc[m] * kLane < kLane) ? slen - lc[m] * kLane : kLane)
                            : 0;
                j0[m] += lc[m] * kLane;
                xv[m] = load_raw_n<Tin>(w + (nv[m] > 0 ? j0[m] : 0), nv[m]);
            }
#pragma unroll
            for (int m = 0; m < kSegDraws; ++m) {
                const int pos = pb + t + m * kThreads;
                if (pos >= d1) continue;
                double pk = 0.0;
                int cnt = 0;
#pragma unroll
                for (int q = 0; q < kLane; ++q) {
                    pk = pk + xv[m].at(q);
                    const double S = block_end_at(sg[m] + (cl[m] + pk), bx[m], bb[m], bn[m]);
                    cnt += (q < nv[m] && S < xx[m]) ? 1 : 0;
                }
                L.sid[pos] = static_cast<int32_t>(j0[m] + cnt);
            }
        }
        lds_barrier();   // crun is rewritten by the next pass
    }
    // ---- coalesced index store ----
#pragma unroll
    for (int k = 0; k < kSegPer; ++k) {
        const int pos = t + k * kThreads;
        if (pos < nu) r[i0 + pos] = L.sid[pos];
    }
}

// kSegU draws of one filter per workgroup; indices are local to the filter.
template <typename Tin, int kSegU, int kSegPass>
__global__ __launch_bounds__(kThreads) void k_map_batched(const Tin* __restrict__ w, BatchArgs ba,
                                                          int32_t* __restrict__ r,
                                                          int32_t* dev_status) {
    __shared__ SegLds<kSegU, kSegPass> L;
    // the plan's status, the chunk count and the chunk's filter are looked up
    // together (the plan writes every base, so the search stays in range even
    // when it failed); nothing found is used before the status is checked
    const int plan = ba.head[0];
    const int64_t nchunks = ba.mc_base[ba.B];
    const int64_t c = blockIdx.x;
    // written by k_carries_batched for every chunk when the plan succeeded;
    // read only then, and only for c < nchunks
    const int b = ba.mc_seg[c < ba.mc_cap ? c : 0];
    if (blockIdx.x == 0 && threadIdx.x == 0 && dev_status)
        *dev_status = (plan != kStatusOk) ? plan : ba.head[1];
    if (plan != kStatusOk) return;
    if (c >= nchunks) return;
    const Tin* ws = w + ba.w_off[b];
    map_seg_chunk<Tin, kSegU, kSegPass>(ws, seg_wargs(ba, b), seg_zargs(ba, b), seg_shared(ba, b),
                       r + ba.n_off[b], c - ba.mc_base[b], L);
}

// ---------------------------------------------------------------------------
// Bandwidth reference for measurement (not part of the method): a streaming
// read of n 16-byte pieces (summed, one partial sum per workgroup) and a
// streaming copy, each thread keeping U coalesced 16-byte loads in flight,
// the access pattern the weight stream of k_reduce aims at.
// ---------------------------------------------------------------------------
template <int U>
__global__ __launch_bounds__(kThreads) void k_stream_read(const f32x4* __restrict__ src, int64_t n,
                                                          float* __restrict__ part) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
    int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (; i + (U - 1) * stride < n; i += U * stride) {
        f32x4 v[U];
#pragma unroll
        for (int k = 0; k < U; ++k) v[k] = src[i + k * stride];
#pragma unroll
        for (int k = 0; k < U; ++k) acc += v[k];
    }
    for (; i < n; i += stride) acc += src[i];
    __shared__ float red[kThreads];
    red[threadIdx.x] = acc.x + acc.y + acc.z + acc.w;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int k = 0; k < kThreads; ++k) t += red[k];
        part[blockIdx.x] = t;
    }
}

// The pattern of the reduce: every workgroup reads its own contiguous run of
// `per` pieces (the last one what remains of the n) with non-temporal loads,
// U in flight per thread.
template <int U>
__global__ __launch_bounds__(kThreads) void k_stream_read_blocks(const f32x4* __restrict__ src,
                                                                int64_t n, int64_t per,
                                                                float* __restrict__ part) {
    const int64_t first = static_cast<int64_t>(blockIdx.x) * per;
    const int64_t lim = (first + per < n) ? per : ((n > first) ? n - first : 0);
    const f32x4* p = src + first;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int64_t i = threadIdx.x; i < lim; i += static_cast<int64_t>(kThreads) * U) {
        f32x4 v[U];
#pragma unroll
        for (int k = 0; k < U; ++k)
            v[k] = (i + k * kThreads < lim) ? __builtin_nontemporal_load(p + i + k * kThreads)
                                            : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < U; ++k) acc += v[k];
    }
    __shared__ float red[kThreads];
    red[threadIdx.x] = acc.x + acc.y + acc.z + acc.w;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int k = 0; k < kThreads; ++k) t += red[k];
        part[blockIdx.x] = t;
    }
}

template <int U>
__global__ __launch_bounds__(kThreads) void k_stream_copy(const f32x4* __restrict__ src, int64_t n,
                                                          f32x4* __restrict__ dst) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
    int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    for (; i + (U - 1) * stride < n; i += U * stride) {
        f32x4 v[U];
#pragma unroll
        for (int k = 0; k < U; ++k) v[k] = src[i + k * stride];
#pragma unroll
        for (int k = 0; k < U; ++k) dst[i + k * stride] = v[k];
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
// Every kernel launch of the library goes through here: the launch records
// its own start and end into the timing events when they are set.  The status
// of the launch itself (not an earlier, unrelated HIP error) is kept for the
// launcher to return: the first failure since the last take_launch_status().
thread_local hipError_t g_launch_status = hipSuccess;

template <typename... P, typename... A>
static void launch(void (*kernel)(P...), dim3 grid, dim3 block, uint32_t shmem, hipStream_t s,
                   A... args) {
    static_assert(sizeof...(P) == sizeof...(A), "one value per kernel parameter");
    std::tuple<P...> vals(args...);   // each value as the parameter's own type
    void* argv[sizeof...(P)];
    std::apply([&argv](auto&... v) {
        int k = 0;
        ((argv[k++] = static_cast<void*>(&v)), ...);
    }, vals);
    const hipError_t e =
        hipExtLaunchKernel(reinterpret_cast<const void*>(kernel), grid, block, argv, shmem, s,
                           g_launch_events.start, g_launch_events.stop, 0);
    if (e != hipSuccess && g_launch_status == hipSuccess) g_launch_status = e;
    ++g_launch_events.launches;
}

static hipError_t take_launch_status() {
    const hipError_t e = g_launch_status;
    g_launch_status = hipSuccess;
    return e;
}

template <typename Tin, int P>
static hipError_t launch_reduce_t(const void* w, const WArgs& wa, const ZArgs& za, int vec_ok,
                                  hipStream_t s) {
    const int64_t grid = wa.nb + za.nb;
    if (grid <= 0) return hipSuccess;
    launch((k_reduce<Tin, P>), dim3(static_cast<unsigned>(grid)), dim3(kThreads), 0, s,
                       static_cast<const Tin*>(w), wa, za, vec_ok);
    return take_launch_status();
}

hipError_t launch_reduce(int prec, const WSource& src, const WArgs& wa, const ZArgs& za, int vec_ok,
                         hipStream_t s) {
    if (src.outer()) {
        const int64_t grid = wa.nb + za.nb;
        if (grid <= 0) return hipSuccess;
        if (prec == kPrecFP32)
            launch(k_reduce_outer<float, kPrecFP32>, dim3(static_cast<unsigned>(grid)),
                   dim3(kThreads), 0, s, src.outer_as<float>(), wa, za);
        else
            launch(k_reduce_outer<double, kPrecFP64>, dim3(static_cast<unsigned>(grid)),
                   dim3(kThreads), 0, s, src.outer_as<double>(), wa, za);
        return take_launch_status();
    }
    if (prec == kPrecFP32) return launch_reduce_t<float, kPrecFP32>(src.w, wa, za, vec_ok, s);
    return launch_reduce_t<double, kPrecFP64>(src.w, wa, za, vec_ok, s);
}

hipError_t launch_carries(const WArgs& wa, const ZArgs& za, const SharedArgs& sh,
                          int32_t* dev_status, double* total_out, hipStream_t s) {
    launch(k_carries, dim3(1), dim3(kScanThreads), 0, s, wa, za, sh, dev_status,
                       total_out);
    return take_launch_status();
}

hipError_t launch_materialize_w(int prec, const WSource& src, const WArgs& wa, const SharedArgs& sh,
                                double* W, int vec_ok, hipStream_t s) {
    const int64_t grid = wa.nb * kWIters;
    if (grid <= 0) return hipSuccess;
    const void* w = src.w;
    if (src.outer()) {
        if (prec == kPrecFP32)
            launch(k_materialize_w_outer<float>, dim3(static_cast<unsigned>(grid)), dim3(kThreads),
                   0, s, src.outer_as<float>(), wa, sh, W, 1);
        else
            launch(k_materialize_w_outer<double>, dim3(static_cast<unsigned>(grid)), dim3(kThreads),
                   0, s, src.outer_as<double>(), wa, sh, W, 1);
    } else if (prec == kPrecFP32)
        launch(k_materialize_w<float>, dim3(static_cast<unsigned>(grid)), dim3(kThreads),
                           0, s, static_cast<const float*>(w), wa, sh, W, vec_ok);
    else
        launch(k_materialize_w<double>, dim3(static_cast<unsigned>(grid)),
                           dim3(kThreads), 0, s, static_cast<const double*>(w), wa, sh, W, vec_ok);
    return take_launch_status();
}

hipError_t launch_materialize_u(const ZArgs& za, const SharedArgs& sh, double* u, hipStream_t s) {
    if (za.N <= 0) return hipSuccess;
    const int64_t grid = (za.scheme != kSchemeMultinomial) ? (za.N + kZBlock - 1) / kZBlock : za.nb;
    if (grid <= 0) return hipSuccess;
    const int vec_out = (reinterpret_cast<uintptr_t>(u) % 16) == 0 ? 1 : 0;
    launch(k_materialize_u, dim3(static_cast<unsigned>(grid)), dim3(kThreads), 0, s, za, sh, u,
           vec_out);
    return take_launch_status();
}

hipError_t launch_map_fused(int prec, const WSource& src, const WArgs& wa, const ZArgs& za,
                            const SharedArgs& sh, double* u_out, int32_t* r, int vec_ok,
                            hipStream_t s) {
    if (za.N <= 0) return hipSuccess;
    const int64_t grid = (za.N + kUPerWG - 1) / kUPerWG;
    const void* w = src.w;
    if (src.outer()) {
        if (prec == kPrecFP32)
            launch(k_map_fused_outer<float>, dim3(static_cast<unsigned>(grid)), dim3(kThreads), 0,
                   s, src.outer_as<float>(), wa, za, sh, u_out, r);
        else
            launch(k_map_fused_outer<double>, dim3(static_cast<unsigned>(grid)), dim3(kThreads), 0,
                   s, src.outer_as<double>(), wa, za, sh, u_out, r);
    } else if (prec == kPrecFP32)
        launch(k_map_fused<float>, dim3(static_cast<unsigned>(grid)), dim3(kThreads), 0,
                           s, static_cast<const float*>(w), wa, za, sh, u_out, r, vec_ok);
    else
        launch(k_map_fused<double>, dim3(static_cast<unsigned>(grid)), dim3(kThreads),
                           0, s, static_cast<const double*>(w), wa, za, sh, u_out, r, vec_ok);
    return take_launch_status();
}

// Uniforms per dense-map workgroup: about 13/16 of a window's weights' worth
// (per_wg * M / N), a multiple of 256 in [256, 4096].
int dense_per_wg(int64_t M, int64_t N) {
    const double want = static_cast<double>(kWinLen) * 13.0 / 16.0 * static_cast<double>(N) /
                        static_cast<double>(M);
    int64_t q = static_cast<int64_t>(want) / kThreads * kThreads;
    if (q < kThreads) q = kThreads;
    if (q > kDenseU) q = kDenseU;
    return static_cast<int>(q);
}

int64_t dense_chunks(int64_t M, int64_t N) {
    const int per = dense_per_wg(M, N);
    return (N + per - 1) / per;
}

hipError_t launch_dense_span(const WArgs& wa, const ZArgs& za, const SharedArgs& sh, int64_t* span,
                             hipStream_t s) {
    if (za.N <= 0) return hipSuccess;
    const int per = dense_per_wg(wa.M, za.N);
    const int64_t chunks = dense_chunks(wa.M, za.N);
    constexpr int64_t kEndsPerWG = kThreads / kQuad;
    const int64_t grid = (2 * chunks + kEndsPerWG - 1) / kEndsPerWG;
    launch(k_dense_span, dim3(static_cast<unsigned>(grid)), dim3(kThreads), 0, s, wa, za, sh, span,
           per, chunks);
    return take_launch_status();
}

hipError_t launch_map_dense(int prec, const WSource& src, const WArgs& wa, const ZArgs& za,
                            const SharedArgs& sh, const int64_t* span, double* u_out, int32_t* r,
                            int vec_ok, hipStream_t s) {
    if (za.N <= 0) return hipSuccess;
    const int per = dense_per_wg(wa.M, za.N);
    const int64_t grid = dense_chunks(wa.M, za.N);
    const void* w = src.w;
    if (src.outer()) {
        if (prec == kPrecFP32)
            launch(k_map_dense_outer<float>, dim3(static_cast<unsigned>(grid)), dim3(kThreads), 0, s,
                   src.outer_as<float>(), wa, za, sh, span, u_out, r, vec_ok, per);
        else
            launch(k_map_dense_outer<double>, dim3(static_cast<unsigned>(grid)), dim3(kThreads), 0,
                   s, src.outer_as<double>(), wa, za, sh, span, u_out, r, vec_ok, per);
    } else if (prec == kPrecFP32)
        launch(k_map_dense<float>, dim3(static_cast<unsigned>(grid)), dim3(kThreads), 0, s,
               static_cast<const float*>(w), wa, za, sh, span, u_out, r, vec_ok, per);
    else
        launch(k_map_dense<double>, dim3(static_cast<unsigned>(grid)), dim3(kThreads), 0, s,
               static_cast<const double*>(w), wa, za, sh, span, u_out, r, vec_ok, per);
    return take_launch_status();
}

bool map_is_dense(int64_t M, int64_t N) { return N * kDenseRatio >= M; }

bool finish_fits(const WArgs& wa, const ZArgs& za) {
    if (map_is_dense(wa.M, za.N)) return false;
    return za.N > 0 && wa.nb >= 1 && wa.nb <= kBetaLds &&
           (za.nb >= 1 || za.scheme != kSchemeMultinomial) && za.nb <= kFinishMaxZBlocks;
}

hipError_t launch_finish(int prec, const WSource& src, const WArgs& wa, const ZArgs& za,
                         const SharedArgs& sh, int32_t* dev_status, double* u_out, int32_t* r,
                         int vec_ok, hipStream_t s) {
    // draws per quad: more than one once the workgroups of one draw per quad
    // would exceed what the chip holds at once, so that the block scans of
    // each workgroup serve several draws and every workgroup is resident
    const int64_t rounds = (za.N + kUPerWG * kFinishResident - 1) / (kUPerWG * kFinishResident);
    const int upq = (rounds <= 1) ? 1 : (rounds <= 2 ? 2 : kFinishMaxUPQ);
    const int64_t per_wg = static_cast<int64_t>(kUPerWG) * upq;
    const dim3 grid(static_cast<unsigned>((za.N + per_wg - 1) / per_wg));
    const dim3 block(kThreads);
    const void* w = src.w;
    auto go = [&](auto k1, auto k2, auto k4, auto wsrc, int vec) {
        if (upq == 1)
            launch(k1, grid, block, 0, s, wsrc, wa, za, sh, dev_status, u_out, r, vec);
        else if (upq == 2)
            launch(k2, grid, block, 0, s, wsrc, wa, za, sh, dev_status, u_out, r, vec);
        else
            launch(k4, grid, block, 0, s, wsrc, wa, za, sh, dev_status, u_out, r, vec);
    };
    if (src.outer()) {
        if (prec == kPrecFP32)
            go(k_finish_outer<float, 1>, k_finish_outer<float, 2>, k_finish_outer<float, 4>,
               src.outer_as<float>(), 1);
        else
            go(k_finish_outer<double, 1>, k_finish_outer<double, 2>, k_finish_outer<double, 4>,
               src.outer_as<double>(), 1);
    } else if (prec == kPrecFP32) {
        go(k_finish<float, 1>, k_finish<float, 2>, k_finish<float, 4>,
           static_cast<const float*>(w), vec_ok);
    } else {
        go(k_finish<double, 1>, k_finish<double, 2>, k_finish<double, 4>,
           static_cast<const double*>(w), vec_ok);
    }
    return take_launch_status();
}

bool small_fits(const WArgs& wa, const ZArgs& za) {
    return finish_fits(wa, za) && wa.nb <= kSmallBlocks;
}

hipError_t launch_reduce_small(int prec, const WSource& src, const WArgs& wa, const ZArgs& za,
                               hipStream_t s) {
    const dim3 grid(static_cast<unsigned>(za.nb + wa.nb));
    const dim3 block(kSmallThreads);
    if (src.outer()) {
        if (prec == kPrecFP32)
            launch(k_reduce_small_outer<float, kPrecFP32>, grid, block, 0, s,
                   src.outer_as<float>(), wa, za);
        else
            launch(k_reduce_small_outer<double, kPrecFP64>, grid, block, 0, s,
                   src.outer_as<double>(), wa, za);
    } else if (prec == kPrecFP32) {
        launch(k_reduce_small<float, kPrecFP32>, grid, block, 0, s,
               static_cast<const float*>(src.w), wa, za);
    } else {
        launch(k_reduce_small<double, kPrecFP64>, grid, block, 0, s,
               static_cast<const double*>(src.w), wa, za);
    }
    return take_launch_status();
}

hipError_t launch_map_w(const double* W, int64_t M, const double* u, int64_t N, int32_t* r,
                        hipStream_t s) {
    if (N <= 0) return hipSuccess;
    if (map_is_dense(M, N)) {
        launch(k_map_w_dense, dim3(static_cast<unsigned>(dense_chunks(M, N))), dim3(kThreads), 0,
               s, W, M, u, N, r, dense_per_wg(M, N));
        return take_launch_status();
    }
    const int64_t grid = (N + kThreads - 1) / kThreads;
    launch(k_map_w, dim3(static_cast<unsigned>(grid)), dim3(kThreads), 0, s, W, M, u, N, r);
    return take_launch_status();
}


template <int U>
static void launch_stream_probe_t(int kind, const void* src, void* dst, int64_t pieces, int grid,
                                  hipStream_t s) {
    if (kind == 0)
        launch(k_stream_read<U>, dim3(static_cast<unsigned>(grid)), dim3(kThreads), 0, s,
               static_cast<const f32x4*>(src), pieces, static_cast<float*>(dst));
    else if (kind == 1)
        launch(k_stream_copy<U>, dim3(static_cast<unsigned>(grid)), dim3(kThreads), 0, s,
               static_cast<const f32x4*>(src), pieces, static_cast<f32x4*>(dst));
    else
        launch(k_stream_read_blocks<U>, dim3(static_cast<unsigned>(grid)), dim3(kThreads), 0, s,
               static_cast<const f32x4*>(src), pieces, (pieces + grid - 1) / grid,
               static_cast<float*>(dst));
}

hipError_t launch_stream_probe(int kind, int unroll, const void* src, void* dst, int64_t pieces,
                               int grid, hipStream_t s) {
    if (unroll == 16)
        launch_stream_probe_t<16>(kind, src, dst, pieces, grid, s);
    else if (unroll == 8)
        launch_stream_probe_t<8>(kind, src, dst, pieces, grid, s);
    else
        launch_stream_probe_t<4>(kind, src, dst, pieces, grid, s);
    return take_launch_status();
}

hipError_t launch_batch_plan(const BatchArgs& ba, int32_t* dev_status, hipStream_t s) {
    launch(k_batch_plan, dim3(1), dim3(kPlanThreads), 0, s, ba, dev_status);
    return take_launch_status();
}

hipError_t launch_reduce_batched(int prec, const void* w, const BatchArgs& ba, hipStream_t s) {
    const unsigned grid = static_cast<unsigned>(ba.zt_cap + ba.wt_cap);
    if (prec == kPrecFP32)
        launch(k_reduce_batched<float, kPrecFP32>, dim3(grid), dim3(kThreads), 0, s,
               static_cast<const float*>(w), ba);
    else
        launch(k_reduce_batched<double, kPrecFP64>, dim3(grid), dim3(kThreads), 0, s,
               static_cast<const double*>(w), ba);
    return take_launch_status();
}

hipError_t launch_carries_batched(const BatchArgs& ba, hipStream_t s) {
    launch(k_carries_batched, dim3(static_cast<unsigned>(ba.B)), dim3(kScanThreads), 0, s, ba);
    return take_launch_status();
}

template <typename Tin>
static void launch_map_batched_t(const Tin* w, const BatchArgs& ba, int32_t* r, int32_t* dev_status,
                                 hipStream_t s) {
    const unsigned grid = static_cast<unsigned>(ba.mc_cap);
    if (ba.chunk == 256)
        launch(k_map_batched<Tin, 256, 32>, dim3(grid), dim3(kThreads), 0, s, w, ba, r, dev_status);
    else if (ba.chunk == 1024)
        launch(k_map_batched<Tin, 1024, 64>, dim3(grid), dim3(kThreads), 0, s, w, ba, r, dev_status);
    else
        launch(k_map_batched<Tin, 512, 64>, dim3(grid), dim3(kThreads), 0, s, w, ba, r, dev_status);
}

// The four batched launches as kernel nodes of a HIP graph (the order of
// launch_batch_plan .. launch_map_batched, with the same grids; carries takes
// `carry_wgs` workgroups, at least ba.B).  The argument blocks of `out` point
// into `a`, which must outlive the use of `out`.
hipError_t batched_node_params(int prec, BatchNodeArgs& a, int carry_wgs,
                               hipKernelNodeParams (&out)[4]) {
    const BatchArgs& ba = a.ba;
    if (ba.chunk != 256 && ba.chunk != 512 && ba.chunk != 1024) return hipErrorInvalidValue;
    a.argv[0][0] = &a.ba;
    a.argv[0][1] = &a.dev_status;
    a.argv[1][0] = &a.w;
    a.argv[1][1] = &a.ba;
    a.argv[2][0] = &a.ba;
    a.argv[3][0] = &a.w;
    a.argv[3][1] = &a.ba;
    a.argv[3][2] = &a.r;
    a.argv[3][3] = &a.dev_status;
    const bool f32 = prec == kPrecFP32;
    void* map = nullptr;
    if (ba.chunk == 256)
        map = f32 ? reinterpret_cast<void*>(&k_map_batched<float, 256, 32>)
                  : reinterpret_cast<void*>(&k_map_batched<double, 256, 32>);
    else if (ba.chunk == 1024)
        map = f32 ? reinterpret_cast<void*>(&k_map_batched<float, 1024, 64>)
                  : reinterpret_cast<void*>(&k_map_batched<double, 1024, 64>);
    else
        map = f32 ? reinterpret_cast<void*>(&k_map_batched<float, 512, 64>)
                  : reinterpret_cast<void*>(&k_map_batched<double, 512, 64>);
    void* const funcs[4] = {
        reinterpret_cast<void*>(&k_batch_plan),
        f32 ? reinterpret_cast<void*>(&k_reduce_batched<float, kPrecFP32>)
            : reinterpret_cast<void*>(&k_reduce_batched<double, kPrecFP64>),
        reinterpret_cast<void*>(&k_carries_batched), map};
    const dim3 grids[4] = {dim3(1), dim3(static_cast<unsigned>(ba.zt_cap + ba.wt_cap)),
                           dim3(static_cast<unsigned>(carry_wgs)),
                           dim3(static_cast<unsigned>(ba.mc_cap))};
    const dim3 blocks[4] = {dim3(kPlanThreads), dim3(kThreads), dim3(kScanThreads),
                            dim3(kThreads)};
    for (int k = 0; k < 4; ++k) {
        out[k] = hipKernelNodeParams{};
        out[k].func = funcs[k];
        out[k].gridDim = grids[k];
        out[k].blockDim = blocks[k];
        out[k].sharedMemBytes = 0;
        out[k].kernelParams = a.argv[k];
        out[k].extra = nullptr;
    }
    return hipSuccess;
}

hipError_t launch_map_batched(int prec, const void* w, const BatchArgs& ba, int32_t* r,
                              int32_t* dev_status, hipStream_t s) {
    if (ba.chunk != 256 && ba.chunk != 512 && ba.chunk != 1024) return hipErrorInvalidValue;
    if (prec == kPrecFP32)
        launch_map_batched_t(static_cast<const float*>(w), ba, r, dev_status, s);
    else
        launch_map_batched_t(static_cast<const double*>(w), ba, r, dev_status, s);
    return take_launch_status();
}

}  // namespace dcr
