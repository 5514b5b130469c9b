// dcr_device.hpp -- device-side building blocks shared by the libdcr kernels.
//
// Summation structure (defines the bits of W and u; every kernel that forms a
// partial sum goes through the helpers below, so the bits agree everywhere):
//
//   lane chunk  16 consecutive elements, summed left to right:
//               p(k) = (((x0 + x1) + x2) ... + xk)
//   sub-tile    16 lane chunks = 256 elements; lane-chunk totals t_l combined
//               left to right: c_0 = 0, c_{l+1} = c_l + t_l;
//               in-sub-tile prefix q = c_l + p(k)  (equals c_{l+1} at k = 15)
//   block       NS sub-tiles; sub-tile totals tau_s combined left to right:
//               sigma_0 = 0, sigma_{s+1} = sigma_s + tau_s;
//               in-block prefix S_blk = sigma_s + q  (equals sigma_{s+1} at the
//               end of sub-tile s)
//   array       block totals scanned by a monotone two-level scan (carries)
//               into beta_1..beta_nb (beta_0 = 0, beta_nb = total);
//               S_j = min(beta_b + S_blk, beta_{b+1}), and S_j = beta_{b+1}
//               once S_blk has reached the block total (block_end_at; always
//               at the block's last element).  A weight of zero therefore
//               ends exactly where the previous weight does, also across
//               lane-chunk, sub-tile and block boundaries (the scan keeps a
//               zero block total's end at the previous end).
//
// Every level either adds a non-negative local prefix to a base computed by
// the same left-to-right rule (monotone because round-to-nearest is monotone)
// or clamps to the next base, so S is non-decreasing and the end of every
// segment equals the base of the next one.  Normalisation: W_j = S_j / total
// (correctly rounded binary64 division; W_{M-1} = total / total = 1).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dcr_internal.hpp"

namespace dcr {

constexpr int kLane = 16;                 // elements per lane chunk
constexpr int kRowLanes = 16;             // lane chunks per sub-tile
constexpr int kSub = kLane * kRowLanes;   // 256 elements per sub-tile
constexpr int kThreads = 256;             // threads per workgroup (16 rows)
constexpr int kRows = kThreads / kRowLanes;
constexpr int kWSubPerBlock = 128;        // sub-tiles per weight block
constexpr int kWBlock = kWSubPerBlock * kSub;   // 32768 weights per block
constexpr int kWIters = kWSubPerBlock / kRows;  // 8 sub-tile rounds per block
constexpr int kZBlock = kThreads * kLane;       // 4096 spacings per block
constexpr int kCarryThreads = 1024;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of
// (x0,x1,x2,x3) -> (hi(B*x2)^x1^k0, lo(B*x2), hi(A*x0)^x3^k1, lo(A*x0)) with
// A = 0xD2511F53, B = 0xCD9E8D57 and the key advanced by the Weyl constants
// 0x9E3779B9, 0xBB67AE85 between rounds.
// ---------------------------------------------------------------------------
struct Words4 {
    uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        // each product's two halves from one 32 x 32 -> 64 multiply
        const uint64_t pa = static_cast<uint64_t>(0xD2511F53u) * c0;
        const uint64_t pb = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        const uint32_t lo_a = static_cast<uint32_t>(pa);
        const uint32_t hi_a = static_cast<uint32_t>(pa >> 32);
        const uint32_t lo_b = static_cast<uint32_t>(pb);
        const uint32_t hi_b = static_cast<uint32_t>(pb >> 32);
        const uint32_t n0 = hi_b ^ c1 ^ k0;
        const uint32_t n2 = hi_a ^ c3 ^ k1;
        c0 = n0;
        c1 = lo_b;
        c2 = n2;
        c3 = lo_a;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Words4{c0, c1, c2, c3};
}

// Open-interval variate from 52 random bits: v = (2k + 1) * 2^-53, exact in
// binary64 and inside [2^-53, 1 - 2^-53], so -log v is finite and positive.
__device__ __forceinline__ double variate_from_words(uint32_t lo, uint32_t hi) {
    const uint64_t k = (static_cast<uint64_t>(hi) << 20) | static_cast<uint64_t>(lo >> 12);
    return static_cast<double>(2 * k + 1) * 0x1p-53;
}

// Exponential spacing z = -log v in the precision form P.
template <int P>
__device__ __forceinline__ double spacing_from_variate(double v) {
    if constexpr (P == kPrecFP32) {
        return static_cast<double>(-logf(static_cast<float>(v)));
    } else {
        return -log(v);
    }
}

// Draws (2*pair, 2*pair + 1) of (seed, stream): one Philox block, words
// (w0, w1) for the even draw and (w2, w3) for the odd draw.
template <int P>
__device__ __forceinline__ void spacing_pair(uint64_t pair, uint64_t seed, uint64_t stream,
                                             double& z_even, double& z_odd) {
    const Words4 x = philox4x32_10(static_cast<uint32_t>(pair), static_cast<uint32_t>(pair >> 32),
                                   static_cast<uint32_t>(stream),
                                   static_cast<uint32_t>(stream >> 32),
                                   static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
    z_even = spacing_from_variate<P>(variate_from_words(x.w0, x.w1));
    z_odd = spacing_from_variate<P>(variate_from_words(x.w2, x.w3));
}

// ---------------------------------------------------------------------------
// Loading one lane chunk of weights as binary64 (binary32 promoted exactly).
// `n_valid` elements are real (0..16); the rest read as 0.  `vec_ok` allows
// 16-byte vector loads (chunk fully valid and base pointer 16-byte aligned).
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <typename Tin>
__device__ __forceinline__ void load_chunk(const Tin* __restrict__ p, int n_valid, bool vec_ok,
                                           double (&x)[kLane]) {
    if (vec_ok && n_valid == kLane) {
        if constexpr (sizeof(Tin) == 4) {
            const f32x4* q = reinterpret_cast<const f32x4*>(p);
            f32x4 f[kLane / 4];
#pragma unroll
            for (int v = 0; v < kLane / 4; ++v) f[v] = q[v];
#pragma unroll
            for (int v = 0; v < kLane / 4; ++v) {
                x[4 * v + 0] = f[v].x;
                x[4 * v + 1] = f[v].y;
                x[4 * v + 2] = f[v].z;
                x[4 * v + 3] = f[v].w;
            }
        } else {
            const f64x2* q = reinterpret_cast<const f64x2*>(p);
            f64x2 d[kLane / 2];
#pragma unroll
            for (int v = 0; v < kLane / 2; ++v) d[v] = q[v];
#pragma unroll
            for (int v = 0; v < kLane / 2; ++v) {
                x[2 * v + 0] = d[v].x;
                x[2 * v + 1] = d[v].y;
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < kLane; ++k) x[k] = (k < n_valid) ? static_cast<double>(p[k]) : 0.0;
    }
}

// A full, 16-byte aligned lane chunk kept unconverted in registers between
// its load and its use, so that loads of later chunks can be issued first.
template <typename Tin>
struct RawChunk;

template <>
struct RawChunk<float> {
    f32x4 v[kLane / 4];
    __device__ __forceinline__ double at(int k) const { return static_cast<double>(v[k >> 2][k & 3]); }
    __device__ __forceinline__ float raw(int k) const { return v[k >> 2][k & 3]; }
};

template <>
struct RawChunk<double> {
    f64x2 v[kLane / 2];
    __device__ __forceinline__ double at(int k) const { return v[k >> 1][k & 1]; }
    __device__ __forceinline__ double raw(int k) const { return v[k >> 1][k & 1]; }
};

template <typename Tin>
__device__ __forceinline__ RawChunk<Tin> load_raw(const Tin* __restrict__ p) {
    RawChunk<Tin> r;
    if constexpr (sizeof(Tin) == 4) {
        const f32x4* q = reinterpret_cast<const f32x4*>(p);
#pragma unroll
        for (int v = 0; v < kLane / 4; ++v) r.v[v] = q[v];
    } else {
        const f64x2* q = reinterpret_cast<const f64x2*>(p);
#pragma unroll
        for (int v = 0; v < kLane / 2; ++v) r.v[v] = q[v];
    }
    return r;
}

// The same from an address aligned only to the element size (a segment of a
// concatenated batch may start anywhere): vector loads of element-aligned
// addresses, which global memory accepts on this chip.
template <typename Tin>
__device__ __forceinline__ RawChunk<Tin> load_raw_any(const Tin* __restrict__ p) {
    RawChunk<Tin> r;
    if constexpr (sizeof(Tin) == 4) {
#pragma unroll
        for (int v = 0; v < kLane / 4; ++v) __builtin_memcpy(&r.v[v], p + 4 * v, sizeof(f32x4));
    } else {
#pragma unroll
        for (int v = 0; v < kLane / 2; ++v) __builtin_memcpy(&r.v[v], p + 2 * v, sizeof(f64x2));
    }
    return r;
}

// Streamed loads: data read once (the weight stream of a reduce) is loaded
// with the non-temporal cache policy where every wave's load covers whole
// cache lines (coalesced 16-byte pieces), so it does not displace reused data;
// on this chip the streaming read rate rises from about 6.2 to 7.0 TB/s.  The
// vector type has element alignment: a filter of a batch may start at any
// element, and global memory accepts element-aligned vector loads here.
typedef float f32x4_ea __attribute__((ext_vector_type(4), aligned(4)));
typedef double f64x2_ea __attribute__((ext_vector_type(2), aligned(8)));
constexpr int kCachePolicyNT = 2;   // non-temporal bit of the cache-policy operand

// A chunk of which only the first n values exist (n <= 0: none; nothing is
// read beyond them), zero-padded; full chunks are vector-loaded.
template <typename Tin>
__device__ __forceinline__ RawChunk<Tin> load_raw_n(const Tin* __restrict__ p, int n) {
    if (n >= kLane) return load_raw_any<Tin>(p);
    RawChunk<Tin> rc;
    constexpr int kPer = (sizeof(Tin) == 4) ? 4 : 2;
#pragma unroll
    for (int q = 0; q < kLane; ++q) rc.v[q / kPer][q % kPer] = (q < n) ? p[q] : static_cast<Tin>(0);
    return rc;
}

// ---------------------------------------------------------------------------
// Weight sources.  The kernels read weights either from an array (`const T*`)
// or from an outer product, w_j = a[j / P] * b[j % P] (the weights of an
// ensemble Gaussian mixture step: particle i, likelihood component k), formed
// in binary64 (exact for binary32 factors), so that the M weights are never
// read from memory.  src_* (source, element offset, count) return a chunk.
// ---------------------------------------------------------------------------
template <typename W>
struct SrcElem;
template <typename T>
struct SrcElem<const T*> {
    using type = T;
};
template <typename T>
struct SrcElem<Outer<T>> {
    using type = double;
};

template <typename T>
__device__ __forceinline__ RawChunk<T> src_raw(const T* __restrict__ w, int64_t j) {
    return load_raw<T>(w + j);
}
template <typename T>
__device__ __forceinline__ RawChunk<T> src_raw_any(const T* __restrict__ w, int64_t j) {
    return load_raw_any<T>(w + j);
}
template <typename T>
__device__ __forceinline__ RawChunk<T> src_raw_n(const T* __restrict__ w, int64_t j, int n) {
    return load_raw_n<T>(w + (n > 0 ? j : 0), n);
}
template <typename T>
__device__ __forceinline__ void src_chunk(const T* __restrict__ w, int64_t j, int n, bool vec_ok,
                                          double (&x)[kLane]) {
    load_chunk<T>(w + (n > 0 ? j : 0), n, vec_ok, x);
}

// Outer product.  j = i P + k with 0 <= k < P, from a binary64 quotient and
// an integer correction (exact for j < 2^52).
template <typename T>
__device__ __forceinline__ void outer_split(const Outer<T>& o, int64_t j, int64_t& i, int64_t& k) {
    i = static_cast<int64_t>(static_cast<double>(j) / static_cast<double>(o.P));
    k = j - i * o.P;
    while (k < 0) {
        --i;
        k += o.P;
    }
    while (k >= o.P) {
        ++i;
        k -= o.P;
    }
}

// The factors of one lane chunk of products, loaded ahead of their use (rows
// of at least kLane products, so a chunk meets at most one row end): products
// q < wq are a0 * b[k + q], the rest a1 * b[k + q - P]; products q >= n do
// not exist and read 0.
template <typename T>
struct OuterRaw {
    T a0, a1;
    int wq, n;
    RawChunk<T> b;
    __device__ __forceinline__ double at(int q) const {
        const double x = static_cast<double>(q < wq ? a0 : a1) * static_cast<double>(b.raw(q));
        return (q < n) ? x : 0.0;
    }
};

template <typename T>
__device__ __forceinline__ OuterRaw<T> outer_load(const Outer<T>& o, int64_t j, int n) {
    OuterRaw<T> r;
    int64_t i = 0, k = 0;
    if (n > 0) outer_split(o, j, i, k);
    const int64_t room = o.P - k;
    r.wq = (room < kLane) ? static_cast<int>(room) : kLane;
    r.n = n;
    // every load reads a valid element (the first product's factors stand in
    // for what does not exist), and no loaded value is used before the sum,
    // so the loads of several chunks stay in flight together
    r.a0 = o.a[i];
    r.a1 = o.a[(r.wq < n) ? i + 1 : i];
    if (n == kLane && r.wq == kLane) {
        r.b = load_raw_any<T>(o.b + k);
    } else {
        constexpr int kPer = (sizeof(T) == 4) ? 4 : 2;
#pragma unroll
        for (int q = 0; q < kLane; ++q) {
            const int64_t kq = (q >= n) ? k : ((q < r.wq) ? k + q : k + q - o.P);
            r.b.v[q / kPer][q % kPer] = o.b[kq];
        }
    }
    return r;
}

template <typename T>
__device__ __forceinline__ RawChunk<double> outer_products(const OuterRaw<T>& r) {
    RawChunk<double> rc;
#pragma unroll
    for (int q = 0; q < kLane; ++q) rc.v[q / 2][q % 2] = r.at(q);
    return rc;
}

// Products j .. j+n-1 (n <= 0: none), zero-padded to a chunk.
template <typename T>
__device__ __forceinline__ RawChunk<double> src_raw_n(const Outer<T>& o, int64_t j, int n) {
    if (o.P >= kLane) return outer_products(outer_load(o, j, n));
    // rows shorter than a chunk: product q is a[i + (k+q) / P] * b[(k+q) % P];
    // every load reads a valid element (the first product's for q >= n)
    RawChunk<double> rc;
    int64_t i = 0, k = 0;
    if (n > 0) outer_split(o, j, i, k);
    const uint32_t P = static_cast<uint32_t>(o.P);
#pragma unroll
    for (int q = 0; q < kLane; ++q) {
        const uint32_t kq = (q < n) ? static_cast<uint32_t>(k) + q : static_cast<uint32_t>(k);
        const uint32_t di = kq / P;
        const double x = static_cast<double>(o.a[i + di]) * static_cast<double>(o.b[kq - di * P]);
        rc.v[q / 2][q % 2] = (q < n) ? x : 0.0;
    }
    return rc;
}
template <typename T>
__device__ __forceinline__ RawChunk<double> src_raw(const Outer<T>& o, int64_t j) {
    return src_raw_n(o, j, kLane);
}
template <typename T>
__device__ __forceinline__ RawChunk<double> src_raw_any(const Outer<T>& o, int64_t j) {
    return src_raw_n(o, j, kLane);
}
template <typename T>
__device__ __forceinline__ void src_chunk(const Outer<T>& o, int64_t j, int n, bool,
                                          double (&x)[kLane]) {
    const RawChunk<double> rc = src_raw_n(o, j, n);
#pragma unroll
    for (int q = 0; q < kLane; ++q) x[q] = rc.at(q);
}

// Left-to-right binary64 sum of a raw chunk; also folds its elements into a
// running minimum (in the input precision) used to detect negative weights.
template <typename Tin>
__device__ __forceinline__ double raw_sum(const RawChunk<Tin>& r, Tin& mn) {
    double s = r.at(0);
    mn = fmin(mn, r.raw(0));
#pragma unroll
    for (int k = 1; k < kLane; ++k) {
        s = s + r.at(k);
        mn = fmin(mn, r.raw(k));
    }
    return s;
}

// Unnormalised cumulative weight at the end of an element of block b (or of a
// lane chunk or sub-tile, at its last element): y is its in-block prefix, X
// the block's total (its last stored sub-tile end), beta_b and beta_n the
// scanned ends of blocks b-1 and b.  A prefix that has reached the block total
// is the block end itself, so the weights of zero after a block's last
// positive weight end exactly where it does (an empty interval: never drawn);
// the prefix of the block's last element always equals X.
__device__ __forceinline__ double block_end_at(double y, double X, double beta_b, double beta_n) {
    return (y == X) ? beta_n : fmin(beta_b + y, beta_n);
}

// A weight is admissible iff it is finite and >= 0 (NaN fails both tests).
__device__ __forceinline__ bool bad_weight(double x) { return !(x >= 0.0) || x == __builtin_huge_val(); }

// Left-to-right sum of one lane chunk.
__device__ __forceinline__ double chunk_sum(const double (&x)[kLane]) {
    double s = x[0];
#pragma unroll
    for (int k = 1; k < kLane; ++k) s = s + x[k];
    return s;
}

// ---------------------------------------------------------------------------
// Normalisation threshold: the smallest binary64 x >= 0 with
// fl(x / total) >= u, for 0 < u <= 1 and 0 < total < inf.  Because
// x -> fl(x / total) is non-decreasing, fl(S / total) >= u  <=>  S >= x, so
// every comparison of a normalised cumulative weight with u becomes a
// comparison of an unnormalised partial sum with x.  fl(u * total) is within
// two units in the last place of the answer, so the loops below take at most
// a few steps; their bound only guards against misuse.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double next_up_nonneg(double x) {
    return __longlong_as_double(__double_as_longlong(x) + 1);
}
__device__ __forceinline__ double next_down_pos(double x) {
    return __longlong_as_double(__double_as_longlong(x) - 1);
}

__device__ __forceinline__ double threshold_for(double u, double total) {
    double x = u * total;
    if (x / total >= u) {
        for (int it = 0; it < 64 && x > 0.0; ++it) {
            const double d = next_down_pos(x);
            if (d / total >= u)
                x = d;
            else
                break;
        }
    } else {
        for (int it = 0; it < 64; ++it) {
            x = next_up_nonneg(x);
            if (x / total >= u) break;
        }
    }
    return x;
}

// ---------------------------------------------------------------------------
// Cross-lane moves with DPP (register speed, no LDS round trip).  Lanes whose
// source lies outside the pattern receive 0, the identity of the sums and of
// the maxima of non-negative values used here.
// ---------------------------------------------------------------------------
template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xF, false);
    return __hiloint2double(hi, lo);
}

template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143, kDppWaveShr1 = 0x138;
constexpr int kDppQuadSwap1 = 0xB1;   // quad_perm [1,0,3,2]
constexpr int kDppQuadSwap2 = 0x4E;   // quad_perm [2,3,0,1]
constexpr int kDppQuadBcast(int k) { return k * 0x55; }   // quad_perm [k,k,k,k]

// Inclusive scans over the 64 lanes of a wave (rows of 16 by doubling shifts,
// then the row carries by broadcast of lanes 15 and 31).
__device__ __forceinline__ double wave_incl_add(double v) {
    v = v + dpp_f64<kDppRowShr1>(v);
    v = v + dpp_f64<kDppRowShr2>(v);
    v = v + dpp_f64<kDppRowShr4>(v);
    v = v + dpp_f64<kDppRowShr8>(v);
    v = v + dpp_f64<kDppRowBcast15, 0xA>(v);
    v = v + dpp_f64<kDppRowBcast31, 0xC>(v);
    return v;
}

__device__ __forceinline__ double wave_incl_max(double v) {
    v = fmax(v, dpp_f64<kDppRowShr1>(v));
    v = fmax(v, dpp_f64<kDppRowShr2>(v));
    v = fmax(v, dpp_f64<kDppRowShr4>(v));
    v = fmax(v, dpp_f64<kDppRowShr8>(v));
    v = fmax(v, dpp_f64<kDppRowBcast15, 0xA>(v));
    v = fmax(v, dpp_f64<kDppRowBcast31, 0xC>(v));
    return v;
}

// The value of the previous lane (0 in lane 0).
__device__ __forceinline__ double wave_shift_up1(double v) { return dpp_f64<kDppWaveShr1>(v); }

// Value of lane k of this lane's quad, for a quad-uniform k in 0..3.
__device__ __forceinline__ double quad_bcast(double v, int k) {
    const double v0 = dpp_f64<kDppQuadBcast(0)>(v);
    const double v1 = dpp_f64<kDppQuadBcast(1)>(v);
    const double v2 = dpp_f64<kDppQuadBcast(2)>(v);
    const double v3 = dpp_f64<kDppQuadBcast(3)>(v);
    return k == 0 ? v0 : (k == 1 ? v1 : (k == 2 ? v2 : v3));
}

// Sum of an integer over the 4 lanes of a quad.
__device__ __forceinline__ int quad_sum(int v) {
    v += dpp_i32<kDppQuadSwap1>(v);
    v += dpp_i32<kDppQuadSwap2>(v);
    return v;
}

// Workgroup-wide logical OR (all threads must call it).
__device__ __forceinline__ int block_any(int pred) { return __syncthreads_or(pred); }

// Workgroup barrier that orders LDS accesses only: outstanding global loads
// and stores stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

constexpr int kDppWaveShl1 = 0x130;
// The value of the next lane (0 in lane 63).
__device__ __forceinline__ double wave_shift_down1(double v) { return dpp_f64<kDppWaveShl1>(v); }

}  // namespace dcr
