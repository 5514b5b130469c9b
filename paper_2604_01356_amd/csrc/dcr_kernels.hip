// dcr_kernels.hip -- HIP kernels for gfx950 (MI355X) implementing the three
// stages of divide-and-conquer multinomial resampling (Popov, Secs. I-III):
//   k_reduce            weight-block totals (Eq. 3) and spacing-block totals
//                       (Alg. 1), one launch, two kinds of workgroups
//   k_carries           monotone scans of the block totals, totals, validity
//   k_materialize_w     normalised cumulative weights W (stage 1 output)
//   k_materialize_u     sorted uniforms u (stage 2 output)
//   k_map_fused         inverse CMF of u against the cumulative weights kept
//                       implicit (block bases + sub-tile bases + a rescan of one
//                       256-weight sub-tile), the divide-and-conquer map of
//                       Alg. 5 laid onto the block / sub-tile / element levels
//   k_map_w             inverse CMF against a given W (stage 3 alone)
// The summation structure that fixes the bits of W and u is described in
// dcr_device.hpp.
#include "dcr_device.hpp"
#include "dcr_internal.hpp"

namespace dcr {

__device__ __forceinline__ int clamp_count(int64_t remaining, int cap) {
    return remaining <= 0 ? 0 : (remaining >= cap ? cap : static_cast<int>(remaining));
}

// ---------------------------------------------------------------------------
// k_reduce: blocks [0, za.nb) draw spacings, blocks [za.nb, za.nb + wa.nb)
// reduce weights.
// ---------------------------------------------------------------------------
template <typename Tin, int P>
__global__ __launch_bounds__(kThreads) void k_reduce(const Tin* __restrict__ w, WArgs wa, ZArgs za,
                                                     int vec_ok) {
    __shared__ double lane_tot[kWIters * kThreads];
    __shared__ double sub_tot[kWSubPerBlock];
    __shared__ double sub_end[kWSubPerBlock];
    const int t = threadIdx.x;
    const int row = t / kRowLanes;
    const int lane = t % kRowLanes;

    if (static_cast<int64_t>(blockIdx.x) < za.nb) {
        // ---- exponential spacings z_i = -log v_i, i = 0..N (Alg. 1) ----
        const int64_t g = blockIdx.x;
        const int64_t i0 = g * kZBlock + static_cast<int64_t>(t) * kLane;
        const int nv = clamp_count(za.N + 1 - i0, kLane);
        double z[kLane];
#pragma unroll
        for (int k = 0; k < kLane; k += 2) {
            double ze = 0.0, zo = 0.0;
            if (k < nv) spacing_pair<P>(static_cast<uint64_t>(i0 + k) >> 1, za.seed, za.stream, ze, zo);
            z[k] = (k < nv) ? ze : 0.0;
            z[k + 1] = (k + 1 < nv) ? zo : 0.0;
        }
        if (nv == kLane) {
            f64x2* q = reinterpret_cast<f64x2*>(za.zbuf + i0);
#pragma unroll
            for (int v = 0; v < kLane / 2; ++v) q[v] = f64x2{z[2 * v], z[2 * v + 1]};
        } else {
            for (int k = 0; k < nv; ++k) za.zbuf[i0 + k] = z[k];
        }
        lane_tot[t] = chunk_sum(z);
        __syncthreads();
        if (t < kRows) {
            double c = lane_tot[t * kRowLanes];
            for (int l = 1; l < kRowLanes; ++l) c = c + lane_tot[t * kRowLanes + l];
            sub_tot[t] = c;
        }
        __syncthreads();
        if (t == 0) {
            double s = 0.0;
            for (int r = 0; r < kRows; ++r) s = s + sub_tot[r];
            za.blk_tot[g] = s;
        }
        return;
    }

    // ---- weights: lane-chunk totals, sub-tile totals, sub-tile ends ----
    const int64_t b = static_cast<int64_t>(blockIdx.x) - za.nb;
    const int64_t blk0 = b * kWBlock;
    int bad = 0;
    // two rounds of loads in flight per wave keeps the register count low
    // enough for several waves per SIMD
#pragma unroll 2
    for (int it = 0; it < kWIters; ++it) {
        const int64_t j0 = blk0 + static_cast<int64_t>(it * kRows + row) * kSub + lane * kLane;
        const int nv = clamp_count(wa.M - j0, kLane);
        double x[kLane];
        load_chunk<Tin>(w + (nv > 0 ? j0 : 0), nv, (vec_ok & 1) != 0, x);
#pragma unroll
        for (int k = 0; k < kLane; ++k) bad |= bad_weight(x[k]) ? 1 : 0;
        lane_tot[it * kThreads + t] = chunk_sum(x);
    }
    bad = block_any(bad);
    if (t < kWSubPerBlock) {
        const int it = t / kRows;
        const int r = t % kRows;
        const double* p = lane_tot + it * kThreads + r * kRowLanes;
        double c = p[0];
        for (int l = 1; l < kRowLanes; ++l) c = c + p[l];
        sub_tot[t] = c;
    }
    __syncthreads();
    if (t == 0) {
        double s = 0.0;
        for (int q = 0; q < kWSubPerBlock; ++q) {
            s = s + sub_tot[q];
            sub_end[q] = s;
        }
    }
    __syncthreads();
    if (t < kWSubPerBlock) wa.sub_end[b * kWSubPerBlock + t] = sub_end[t];
    if (t == 0) {
        wa.blk_tot[b] = sub_end[kWSubPerBlock - 1];
        wa.blk_bad[b] = bad;
    }
}

// ---------------------------------------------------------------------------
// Monotone two-level scan run by a whole 1024-thread workgroup:
//   thread t owns a contiguous range, sums it left to right (p), group-of-32
//   exclusive bases h are left-to-right sums of thread totals, group bases G
//   are left-to-right sums of group totals, gamma_t = G + h, and
//   out_j = min(gamma_t + p_j, gamma_{t+1}).
// out is non-decreasing for non-negative input.  Returns out[n-1] to every
// thread (0 for n == 0).
// ---------------------------------------------------------------------------
__device__ double monotone_scan(const double* __restrict__ in, int64_t n, double* __restrict__ out,
                                double* T, double* GT, double* gam, double* bcast) {
    const int t = threadIdx.x;
    const int64_t per = (n + kCarryThreads - 1) / kCarryThreads;
    const int64_t a = (static_cast<int64_t>(t) * per < n) ? static_cast<int64_t>(t) * per : n;
    const int64_t e = (a + per < n) ? a + per : n;
    double tt = 0.0;
    for (int64_t j = a; j < e; ++j) tt = tt + in[j];
    T[t] = tt;
    __syncthreads();
    const int g = t / 32;
    const int q = t % 32;
    double h = 0.0;
    for (int k = 0; k < q; ++k) h = h + T[g * 32 + k];
    if (q == 31) GT[g] = h + T[t];
    __syncthreads();
    double G = 0.0;
    for (int k = 0; k < g; ++k) G = G + GT[k];
    const double gamma = G + h;
    gam[t] = gamma;
    if (t == 0) gam[kCarryThreads] = __builtin_huge_val();
    __syncthreads();
    const double gnext = gam[t + 1];
    double p = 0.0;
    for (int64_t j = a; j < e; ++j) {
        p = p + in[j];
        const double v = fmin(gamma + p, gnext);
        out[j] = v;
        if (j == n - 1) *bcast = v;
    }
    if (n == 0 && t == 0) *bcast = 0.0;
    __syncthreads();
    const double r = *bcast;
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kCarryThreads) void k_carries(WArgs wa, ZArgs za, SharedArgs sh,
                                                           int32_t* dev_status, double* total_out) {
    __shared__ double T[kCarryThreads];
    __shared__ double GT[kCarryThreads / 32];
    __shared__ double gam[kCarryThreads + 1];
    __shared__ double bcast;
    const int t = threadIdx.x;
    int status = kStatusOk;
    if (wa.nb > 0) {
        int bad = 0;
        for (int64_t b = t; b < wa.nb; b += kCarryThreads) bad |= wa.blk_bad[b];
        bad = block_any(bad);
        const double tot = monotone_scan(wa.blk_tot, wa.nb, wa.beta, T, GT, gam, &bcast);
        if (bad || !(tot > 0.0) || tot == __builtin_huge_val()) status = kStatusBadWeights;
        if (t == 0) {
            sh.totals[0] = tot;
            if (total_out) *total_out = tot;
        }
    }
    if (za.nb > 0) {
        const double ztot = monotone_scan(za.blk_tot, za.nb, za.beta, T, GT, gam, &bcast);
        if (t == 0) sh.totals[1] = ztot;
    }
    if (t == 0) {
        sh.status[0] = status;
        if (dev_status) *dev_status = status;
    }
}

// ---------------------------------------------------------------------------
// k_materialize_w: one workgroup per (weight block, round of 16 sub-tiles).
// ---------------------------------------------------------------------------
template <typename Tin>
__global__ __launch_bounds__(kThreads) void k_materialize_w(const Tin* __restrict__ w, WArgs wa,
                                                            SharedArgs sh, double* __restrict__ W,
                                                            int vec_ok) {
    __shared__ double lane_tot[kThreads];
    const int t = threadIdx.x;
    const int row = t / kRowLanes;
    const int lane = t % kRowLanes;
    const int64_t b = blockIdx.x / kWIters;
    const int it = blockIdx.x % kWIters;
    const int s = it * kRows + row;
    const int64_t blk0 = b * kWBlock;
    const int64_t j0 = blk0 + static_cast<int64_t>(s) * kSub + lane * kLane;
    const int nv = clamp_count(wa.M - j0, kLane);
    double x[kLane];
    load_chunk<Tin>(w + (nv > 0 ? j0 : 0), nv, (vec_ok & 1) != 0, x);
    double p[kLane];
    p[0] = x[0];
#pragma unroll
    for (int k = 1; k < kLane; ++k) p[k] = p[k - 1] + x[k];
    lane_tot[t] = p[kLane - 1];
    __syncthreads();
    double c = 0.0;
    for (int l = 0; l < lane; ++l) c = c + lane_tot[row * kRowLanes + l];
    if (nv == 0 || sh.status[0] != kStatusOk) return;
    const double sigma = (s == 0) ? 0.0 : wa.sub_end[b * kWSubPerBlock + s - 1];
    const double beta_b = (b == 0) ? 0.0 : wa.beta[b - 1];
    const double beta_n = wa.beta[b];
    const int64_t jlast = ((blk0 + kWBlock < wa.M) ? blk0 + kWBlock : wa.M) - 1;
    const double total = sh.totals[0];
    double out[kLane];
#pragma unroll
    for (int k = 0; k < kLane; ++k) {
        const double S = (j0 + k == jlast) ? beta_n : fmin(beta_b + (sigma + (c + p[k])), beta_n);
        out[k] = S / total;
    }
    if (nv == kLane && (vec_ok & 2)) {
        f64x2* q = reinterpret_cast<f64x2*>(W + j0);
#pragma unroll
        for (int v = 0; v < kLane / 2; ++v) q[v] = f64x2{out[2 * v], out[2 * v + 1]};
    } else {
        for (int k = 0; k < nv; ++k) W[j0 + k] = out[k];
    }
}

// ---------------------------------------------------------------------------
// k_materialize_u: one workgroup per spacing block of 4096 draws.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_materialize_u(ZArgs za, SharedArgs sh,
                                                            double* __restrict__ u, int vec_out) {
    __shared__ double lane_tot[kThreads];
    __shared__ double row_tot[kRows];
    const int t = threadIdx.x;
    const int row = t / kRowLanes;
    const int lane = t % kRowLanes;
    const int64_t g = blockIdx.x;
    const int64_t i0 = g * kZBlock + static_cast<int64_t>(t) * kLane;
    const int nv = clamp_count(za.N + 1 - i0, kLane);
    double p[kLane];
    if (nv == kLane) {
        const f64x2* q = reinterpret_cast<const f64x2*>(za.zbuf + i0);
#pragma unroll
        for (int v = 0; v < kLane / 2; ++v) {
            const f64x2 d = q[v];
            p[2 * v] = d.x;
            p[2 * v + 1] = d.y;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kLane; ++k) p[k] = (k < nv) ? za.zbuf[i0 + k] : 0.0;
    }
#pragma unroll
    for (int k = 1; k < kLane; ++k) p[k] = p[k - 1] + p[k];
    lane_tot[t] = p[kLane - 1];
    __syncthreads();
    double c = 0.0;
    for (int l = 0; l < lane; ++l) c = c + lane_tot[row * kRowLanes + l];
    if (lane == kRowLanes - 1) row_tot[row] = c + lane_tot[t];
    __syncthreads();
    double sigma = 0.0;
    for (int r = 0; r < row; ++r) sigma = sigma + row_tot[r];
    const double beta_g = (g == 0) ? 0.0 : za.beta[g - 1];
    const double beta_n = za.beta[g];
    const int64_t ilast = (g * kZBlock + kZBlock - 1 < za.N) ? g * kZBlock + kZBlock - 1 : za.N;
    const double ztot = sh.totals[1];
    const int nout = clamp_count(za.N - i0, kLane);   // draws i < N are output
    double out[kLane];
#pragma unroll
    for (int k = 0; k < kLane; ++k) {
        const double Z = (i0 + k == ilast) ? beta_n : fmin(beta_g + (sigma + (c + p[k])), beta_n);
        out[k] = Z / ztot;
    }
    if (nout == kLane && vec_out) {
        f64x2* q = reinterpret_cast<f64x2*>(u + i0);
#pragma unroll
        for (int v = 0; v < kLane / 2; ++v) q[v] = f64x2{out[2 * v], out[2 * v + 1]};
    } else {
        for (int k = 0; k < nout; ++k) u[i0 + k] = out[k];
    }
}

// ---------------------------------------------------------------------------
// Inverse CMF against implicit cumulative weights.  For each uniform u the
// threshold x (S >= x  <=>  W >= u) is located level by level, as the
// divide-and-conquer sampler narrows its ranges (Alg. 5): first the block
// (search of the block ends beta), then the sub-tile (search of the stored
// sub-tile ends), then the lane chunk and the element by re-summing the one
// 256-weight sub-tile with the same left-to-right rule as k_reduce.
// ---------------------------------------------------------------------------
template <typename Tin>
__global__ __launch_bounds__(kThreads) void k_map_fused(const Tin* __restrict__ w, WArgs wa,
                                                        SharedArgs sh, const double* __restrict__ u,
                                                        int64_t N, int32_t* __restrict__ r,
                                                        int vec_ok) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= N) return;
    if (sh.status[0] != kStatusOk) {
        r[i] = -1;
        return;
    }
    const double total = sh.totals[0];
    const double x = threshold_for(u[i], total);
    // block level: first b with beta_{b+1} >= x
    int64_t lo = 0, hi = wa.nb - 1;
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
    const int64_t blk0 = b * kWBlock;
    const int64_t blen = (wa.M - blk0 < kWBlock) ? wa.M - blk0 : kWBlock;
    const int64_t jlast = blk0 + blen - 1;
    const int nsub = static_cast<int>((blen + kSub - 1) / kSub);
    const double* se = wa.sub_end + b * kWSubPerBlock;
    // sub-tile level: first s with end(s) >= x
    int slo = 0, shi = nsub - 1;
    while (slo < shi) {
        const int mid = (slo + shi) >> 1;
        const double e = fmin(beta_b + se[mid], beta_n);
        if (e < x)
            slo = mid + 1;
        else
            shi = mid;
    }
    const int s = slo;
    const double sigma = (s == 0) ? 0.0 : se[s - 1];
    const int64_t sub0 = blk0 + static_cast<int64_t>(s) * kSub;
    const int slen = static_cast<int>((jlast - sub0 + 1 < kSub) ? jlast - sub0 + 1 : kSub);
    const int nl = (slen + kLane - 1) / kLane;
    // lane level: lane-chunk totals, left to right, four chunks in flight
    const bool last_sub = (s == nsub - 1);   // its last chunk ends at beta_{b+1}
    int lf = -1;
    double c = 0.0, cf = 0.0, cprev = 0.0;
    for (int l4 = 0; l4 < nl && lf < 0; l4 += 4) {
        double lt[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int l = l4 + q;
            const int nv = (l < nl) ? ((slen - l * kLane < kLane) ? slen - l * kLane : kLane) : 0;
            double xx[kLane];
            load_chunk<Tin>(w + (nv > 0 ? sub0 + l * kLane : 0), nv, (vec_ok & 1) != 0, xx);
            lt[q] = chunk_sum(xx);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int l = l4 + q;
            if (l < nl && lf < 0) {
                const double cn = c + lt[q];
                const double e =
                    (last_sub && l == nl - 1) ? beta_n : fmin(beta_b + (sigma + cn), beta_n);
                if (e >= x) {
                    lf = l;
                    cf = c;
                }
                cprev = c;
                c = cn;
            }
        }
    }
    if (lf < 0) {  // unreachable: the sub-tile's end is >= x by the search above
        lf = nl - 1;
        cf = cprev;
    }
    // element level
    const int64_t l0 = sub0 + static_cast<int64_t>(lf) * kLane;
    const int nv = (slen - lf * kLane < kLane) ? slen - lf * kLane : kLane;
    double xx[kLane];
    load_chunk<Tin>(w + l0, nv, (vec_ok & 1) != 0, xx);
    double pk = 0.0;
    int64_t jr = l0 + nv - 1;
    for (int k = 0; k < nv; ++k) {
        pk = pk + xx[k];
        const int64_t j = l0 + k;
        const double e = (j == jlast) ? beta_n : fmin(beta_b + (sigma + (cf + pk)), beta_n);
        if (e >= x) {
            jr = j;
            break;
        }
    }
    r[i] = static_cast<int32_t>(jr);
}

// ---------------------------------------------------------------------------
// Stage 3 alone: inverse CMF of sorted u against a given non-decreasing W.
// Each workgroup takes 256 consecutive uniforms; its first and last uniform
// are located in the whole of W (Alg. 2), which bounds the range every other
// uniform of the workgroup can fall in (the split of Alg. 5); each uniform is
// then located inside that range.
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

__global__ __launch_bounds__(kThreads) void k_map_w(const double* __restrict__ W, int64_t M,
                                                    const double* __restrict__ u, int64_t N,
                                                    int32_t* __restrict__ r) {
    __shared__ int64_t range[2];
    const int t = threadIdx.x;
    const int64_t first = static_cast<int64_t>(blockIdx.x) * kThreads;
    const int64_t last = (first + kThreads < N ? first + kThreads : N) - 1;
    if (t == 0) range[0] = lower_bound_clamped(W, 0, M - 1, u[first]);
    if (t == 1) range[1] = lower_bound_clamped(W, 0, M - 1, u[last]);
    __syncthreads();
    const int64_t i = first + t;
    if (i <= last) r[i] = static_cast<int32_t>(lower_bound_clamped(W, range[0], range[1], u[i]));
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
template <typename Tin, int P>
static hipError_t launch_reduce_t(const void* w, const WArgs& wa, const ZArgs& za, int vec_ok,
                                  hipStream_t s) {
    const int64_t grid = wa.nb + za.nb;
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_reduce<Tin, P>), dim3(static_cast<unsigned>(grid)), dim3(kThreads), 0, s,
                       static_cast<const Tin*>(w), wa, za, vec_ok);
    return hipGetLastError();
}

hipError_t launch_reduce(int prec, const void* w, const WArgs& wa, const ZArgs& za, int vec_ok,
                         hipStream_t s) {
    if (prec == kPrecFP32) return launch_reduce_t<float, kPrecFP32>(w, wa, za, vec_ok, s);
    return launch_reduce_t<double, kPrecFP64>(w, wa, za, vec_ok, s);
}

hipError_t launch_carries(const WArgs& wa, const ZArgs& za, const SharedArgs& sh,
                          int32_t* dev_status, double* total_out, hipStream_t s) {
    hipLaunchKernelGGL(k_carries, dim3(1), dim3(kCarryThreads), 0, s, wa, za, sh, dev_status,
                       total_out);
    return hipGetLastError();
}

hipError_t launch_materialize_w(int prec, const void* w, const WArgs& wa, const SharedArgs& sh,
                                double* W, int vec_ok, hipStream_t s) {
    const int64_t grid = wa.nb * kWIters;
    if (grid <= 0) return hipSuccess;
    if (prec == kPrecFP32)
        hipLaunchKernelGGL(k_materialize_w<float>, dim3(static_cast<unsigned>(grid)), dim3(kThreads),
                           0, s, static_cast<const float*>(w), wa, sh, W, vec_ok);
    else
        hipLaunchKernelGGL(k_materialize_w<double>, dim3(static_cast<unsigned>(grid)),
                           dim3(kThreads), 0, s, static_cast<const double*>(w), wa, sh, W, vec_ok);
    return hipGetLastError();
}

hipError_t launch_materialize_u(const ZArgs& za, const SharedArgs& sh, double* u, hipStream_t s) {
    if (za.nb <= 0 || za.N <= 0) return hipSuccess;
    const int vec_out = (reinterpret_cast<uintptr_t>(u) % 16) == 0 ? 1 : 0;
    hipLaunchKernelGGL(k_materialize_u, dim3(static_cast<unsigned>(za.nb)), dim3(kThreads), 0, s, za,
                       sh, u, vec_out);
    return hipGetLastError();
}

hipError_t launch_map_fused(int prec, const void* w, const WArgs& wa, const SharedArgs& sh,
                            const double* u, int64_t N, int32_t* r, int vec_ok, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    const int64_t grid = (N + kThreads - 1) / kThreads;
    if (prec == kPrecFP32)
        hipLaunchKernelGGL(k_map_fused<float>, dim3(static_cast<unsigned>(grid)), dim3(kThreads), 0,
                           s, static_cast<const float*>(w), wa, sh, u, N, r, vec_ok);
    else
        hipLaunchKernelGGL(k_map_fused<double>, dim3(static_cast<unsigned>(grid)), dim3(kThreads),
                           0, s, static_cast<const double*>(w), wa, sh, u, N, r, vec_ok);
    return hipGetLastError();
}

hipError_t launch_map_w(const double* W, int64_t M, const double* u, int64_t N, int32_t* r,
                        hipStream_t s) {
    if (N <= 0) return hipSuccess;
    const int64_t grid = (N + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_map_w, dim3(static_cast<unsigned>(grid)), dim3(kThreads), 0, s, W, M, u, N,
                       r);
    return hipGetLastError();
}

}  // namespace dcr
