// Read-only sweeps over the state: norm, Pauli-string and dense-observable
// expectations, measurement probabilities and the sampler (Table I:
// expectation, measurement, sampler; Sec. II: outcomes from the numerically
// computed probability distribution), plus the write sweeps set-basis,
// scale, collapse and Pauli rotation.
//
// Every reduction accumulates in FP64 in an order that depends only on n
// (never on the grid size or on other work on the device): a fixed partition
// into blocks, a fixed per-thread order inside a block, a fixed LDS tree, and
// a fixed final pass.  Results are therefore bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <thread>
#include <vector>

#include "sv_internal.h"

namespace sv {
namespace {

template <typename R>
struct Cx;
template <>
struct Cx<float> {
    using T = float2;
};
template <>
struct Cx<double> {
    using T = double2;
};

constexpr int kThreads = 256;

// v with a zero bit inserted at each of the n ascending positions pos.
__device__ __forceinline__ uint64_t insert_bits0(uint64_t v, const int32_t* pos, int n)
{
    for (int j = 0; j < n; ++j) {
        const int p = pos[j];
        v = ((v >> p) << (p + 1)) | (v & ((uint64_t(1) << p) - 1));
    }
    return v;
}

// |a|^2 in FP64 with a fixed rounding sequence (no contraction freedom):
// complex64 components square exactly in FP64.
template <typename T2>
__device__ __forceinline__ double prob(const T2 a)
{
    const double re = double(a.x), im = double(a.y);
    return fma(re, re, __dmul_rn(im, im));
}

// Fixed-shape LDS tree over kThreads values; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* lds)
{
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (int(threadIdx.x) < s) lds[threadIdx.x] = __dadd_rn(lds[threadIdx.x], lds[threadIdx.x + s]);
        __syncthreads();
    }
    const double r = lds[0];
    __syncthreads();
    return r;
}

// ------------------------------------------------------------ write sweeps

template <typename T2>
__global__ __launch_bounds__(kThreads) void k_set_basis(T2* __restrict__ psi, uint64_t dim, uint64_t x)
{
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < dim; i += stride) {
        T2 v;
        v.x = (i == x) ? 1 : 0;
        v.y = 0;
        psi[i] = v;
    }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_scale(typename Cx<R>::T* __restrict__ psi, uint64_t dim,
                                                   R f)
{
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < dim; i += stride) {
        auto v = psi[i];
        v.x *= f;
        v.y *= f;
        psi[i] = v;
    }
}

unsigned grid_for(sv_handle_s* h, uint64_t items)
{
    uint64_t b = (items + kThreads - 1) / kThreads;
    const uint64_t cap = uint64_t(h->cu_count) * 16;
    return unsigned(std::max<uint64_t>(1, std::min(b, cap)));
}

// ------------------------------------------------------------ norm / expect

// Partition of `items` work items into `nb` blocks of `per` items (powers of
// two), a function of the item count only.
struct Partition {
    uint64_t nb, per;
};

Partition partition(uint64_t items)
{
    uint64_t nb = items / 2048;
    if (nb < 1) nb = 1;
    if (nb > 8192) nb = 8192;
    return {nb, items / nb};
}

constexpr int kMaxTermsPerSweep = 32;
constexpr int kMaxActive = 16;     // Z-type terms that need per-item work in one sweep
constexpr int kExpectUnroll = 4;   // items loaded per thread per round

struct ExpectArgs {
    uint64_t per;        // items per block
    uint64_t x;          // common X/Y mask of the terms
    int32_t hbit;        // highest bit of x (pair sweeps)
    int32_t n_terms;
    int32_t n_active;    // x == 0: terms [0, n_active) meet the varying bits
    uint64_t z[kMaxTermsPerSweep];
    int32_t ny[kMaxTermsPerSweep];
};

// Fixed-order sum over the 64 lanes of a wave (butterfly), valid in every lane.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = __dadd_rn(v, __shfl_xor(v, o, 64));
    return v;
}

// Block partials of terms [0, n) and of the norm: part[t * nb + block]
// (t = n is the norm).  Each value is summed over its wave by a butterfly,
// then the four wave sums in order.
__device__ __forceinline__ void write_partials(const double* val, double norm, int n, double* part,
                                               double (*wsum)[kThreads / 64])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int t = 0; t <= kMaxTermsPerSweep; ++t) {
        if (t <= n) {
            const double w = wave_sum(t == n ? norm : val[t < kMaxTermsPerSweep ? t : 0]);
            if (lane == 0) wsum[t][wave] = w;
        }
    }
    __syncthreads();
    if (int(threadIdx.x) <= n) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) s = __dadd_rn(s, wsum[threadIdx.x][w]);
        part[uint64_t(threadIdx.x) * gridDim.x + blockIdx.x] = s;
    }
}

// x == 0 sweeps (Z-type terms and the norm).  Item i contributes
// |psi_i|^2 * (-1)^popcount(i & z).  Block b covers items
// [b * per, (b + 1) * per); thread tid takes items it0 + u * 256 + tid.
// Only the bits of `it` above the thread index vary inside a thread
// ("vary"); a term whose Z mask misses them has a constant sign per thread
// and shares the plain sum (the norm).  The others (the first n_active,
// arranged by the host) need per-item work, done per round of four items:
// those differ only in bits 8-9 of `it`, so a term's sign over the round is
// (-1)^parity(it0 & z & vary) * (-1)^parity(u & m), m = bits 8-9 of
// z & vary, and the round adds +-h[m], h the Walsh-Hadamard transform of the
// round's four probabilities.  The next round's loads are in flight while a
// round is summed.
template <typename R>
__device__ __forceinline__ void expect_z_body(const typename Cx<R>::T* __restrict__ psi, const ExpectArgs a,
                                              double* __restrict__ part)
{
    using T2 = typename Cx<R>::T;
    static_assert(kExpectUnroll == 4 && kThreads == 256, "a round spans bits 8-9 of it");
    __shared__ double wsum[kMaxTermsPerSweep + 1][kThreads / 64];
    constexpr uint64_t kRound = uint64_t(kExpectUnroll) * kThreads;
    const uint64_t first = uint64_t(blockIdx.x) * a.per;
    const uint64_t vary = (a.per - 1) & ~uint64_t(kThreads - 1);
    double acc[kMaxActive];
#pragma unroll
    for (int t = 0; t < kMaxActive; ++t) acc[t] = 0.0;
    double norm = 0.0;
    // two register buffers in turn: while one round is summed the next
    // one's loads are in flight (no copy between them, which would wait)
    T2 va[kExpectUnroll] = {}, vb[kExpectUnroll] = {};
    // items past the block's end (per < 1024) load a valid amplitude and are
    // not summed: unconditional loads keep the wait counts exact
    auto load = [&](T2 (&v)[kExpectUnroll], uint64_t it0) {
#pragma unroll
        for (int u = 0; u < kExpectUnroll; ++u) {
            const uint64_t it = it0 + uint64_t(u) * kThreads + threadIdx.x;
            v[u] = psi[first + (it < a.per ? it : a.per - 1)];
        }
    };
    auto sum_round = [&](const T2 (&v)[kExpectUnroll], uint64_t it0) {
        double pr[kExpectUnroll];
#pragma unroll
        for (int u = 0; u < kExpectUnroll; ++u)
            pr[u] = (it0 + uint64_t(u) * kThreads + threadIdx.x < a.per) ? prob(v[u]) : 0.0;
        const double s01 = __dadd_rn(pr[0], pr[1]), d01 = __dsub_rn(pr[0], pr[1]);
        const double s23 = __dadd_rn(pr[2], pr[3]), d23 = __dsub_rn(pr[2], pr[3]);
        const double h0 = __dadd_rn(s01, s23), h1 = __dadd_rn(d01, d23);
        const double h2 = __dsub_rn(s01, s23), h3 = __dsub_rn(d01, d23);
        norm = __dadd_rn(norm, h0);
#pragma unroll
        for (int t = 0; t < kMaxActive; ++t) {
            if (t < a.n_active) {
                const uint64_t zv = a.z[t] & vary;
                const uint32_t m = uint32_t(zv >> 8);
                const double lo = (m & 1) ? h1 : h0;
                const double hi = (m & 1) ? h3 : h2;
                const double hv = (m & 2) ? hi : lo;
                const double sg = (__popcll(it0 & zv) & 1) ? -1.0 : 1.0;
                acc[t] = fma(hv, sg, acc[t]);  // exact sign, one rounding
            }
        }
    };
    // the prefetch is unconditional (past the end it re-reads the block's
    // last amplitude), so the compiler can wait for the older round only
    load(va, 0);
    for (uint64_t it0 = 0; it0 < a.per; it0 += 2 * kRound) {
        load(vb, it0 + kRound);
        sum_round(va, it0);
        if (it0 + kRound >= a.per) break;
        load(va, it0 + 2 * kRound);
        sum_round(vb, it0 + kRound);
    }
    // constant signs: (-1)^parity((first | tid) & z)
    const uint64_t fixed = first | threadIdx.x;
    double val[kMaxTermsPerSweep];
#pragma unroll
    for (int t = 0; t < kMaxTermsPerSweep; ++t) {
        if (t < a.n_terms) {
            const double x = (t < kMaxActive && t < a.n_active) ? acc[t < kMaxActive ? t : 0] : norm;
            val[t] = (__popcll(fixed & a.z[t]) & 1) ? -x : x;
        } else {
            val[t] = 0.0;
        }
    }
    write_partials(val, norm, a.n_terms, part, wsum);
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_expect_z(const typename Cx<R>::T* __restrict__ psi,
                                                      ExpectArgs a, double* __restrict__ part)
{
    expect_z_body<R>(psi, a, part);
}

// Several x == 0 sweeps in one launch (small states, where a launch costs
// more than its sweep): sweep y takes args[y] and part + y * stride.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_expect_z_group(const typename Cx<R>::T* __restrict__ psi,
                                                            const ExpectArgs* __restrict__ args,
                                                            double* __restrict__ part, uint64_t stride)
{
    expect_z_body<R>(psi, args[blockIdx.y], part + blockIdx.y * stride);
}

// Pair sweeps for terms sharing one X/Y mask x != 0: item q is the pair
// (i, j = i ^ x), i = q with a zero inserted at bit hbit (the highest bit
// of x).  With w = conj(psi_j) psi_i the pair contributes
// 2 Re(w * i^ny) * (-1)^popcount(i & z), because P|i> = ph(i)|j> and
// ph(j) = conj(ph(i)) for a Hermitian Pauli string.
template <typename R>
__device__ __forceinline__ void expect_xy_body(const typename Cx<R>::T* __restrict__ psi, const ExpectArgs a,
                                               double* __restrict__ part)
{
    using T2 = typename Cx<R>::T;
    __shared__ double wsum[kMaxTermsPerSweep + 1][kThreads / 64];
    constexpr uint64_t kRound = uint64_t(kExpectUnroll) * kThreads;
    const uint64_t first = uint64_t(blockIdx.x) * a.per;
    const uint64_t lomask = (uint64_t(1) << a.hbit) - 1;
    double acc[kMaxTermsPerSweep];
#pragma unroll
    for (int t = 0; t < kMaxTermsPerSweep; ++t) acc[t] = 0.0;
    double norm = 0.0;
    auto index = [&](uint64_t it) {
        const uint64_t q = first + it;
        return ((q >> a.hbit) << (a.hbit + 1)) | (q & lomask);
    };
    T2 ai[kExpectUnroll] = {}, aj[kExpectUnroll] = {}, bi[kExpectUnroll] = {}, bj[kExpectUnroll] = {};
    auto load = [&](T2 (&vi)[kExpectUnroll], T2 (&vj)[kExpectUnroll], uint64_t it0) {
#pragma unroll
        for (int u = 0; u < kExpectUnroll; ++u) {
            const uint64_t it = it0 + uint64_t(u) * kThreads + threadIdx.x;
            const uint64_t i = index(it < a.per ? it : a.per - 1);
            vi[u] = psi[i];
            vj[u] = psi[i ^ a.x];
        }
    };
    auto sum_round = [&](const T2 (&vi)[kExpectUnroll], const T2 (&vj)[kExpectUnroll], uint64_t it0) {
#pragma unroll
        for (int u = 0; u < kExpectUnroll; ++u) {
            const uint64_t it = it0 + uint64_t(u) * kThreads + threadIdx.x;
            if (it >= a.per) continue;
            const uint64_t i = index(it);
            const double ir = double(vi[u].x), im = double(vi[u].y), jr = double(vj[u].x), jm = double(vj[u].y);
            // w = conj(a_j) * a_i
            const double wr = fma(jr, ir, __dmul_rn(jm, im));
            const double wi = fma(jr, im, -__dmul_rn(jm, ir));
            norm = __dadd_rn(norm, __dadd_rn(prob(vi[u]), prob(vj[u])));
#pragma unroll
            for (int t = 0; t < kMaxTermsPerSweep; ++t) {
                if (t < a.n_terms) {
                    const int m = a.ny[t] & 3;
                    double w = (m & 1) ? wi : wr;
                    if (m == 1 || m == 2) w = -w;
                    w = 2.0 * w;
                    if (__popcll(i & a.z[t]) & 1) w = -w;
                    acc[t] = __dadd_rn(acc[t], w);
                }
            }
        }
    };
    load(ai, aj, 0);
    for (uint64_t it0 = 0; it0 < a.per; it0 += 2 * kRound) {
        load(bi, bj, it0 + kRound);
        sum_round(ai, aj, it0);
        if (it0 + kRound >= a.per) break;
        load(ai, aj, it0 + 2 * kRound);
        sum_round(bi, bj, it0 + kRound);
    }
    write_partials(acc, norm, a.n_terms, part, wsum);
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_expect_xy(const typename Cx<R>::T* __restrict__ psi,
                                                       ExpectArgs a, double* __restrict__ part)
{
    expect_xy_body<R>(psi, a, part);
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_expect_xy_group(const typename Cx<R>::T* __restrict__ psi,
                                                             const ExpectArgs* __restrict__ args,
                                                             double* __restrict__ part, uint64_t stride)
{
    expect_xy_body<R>(psi, args[blockIdx.y], part + blockIdx.y * stride);
}

// out[t] = sum over blocks of part[t * nb + b], fixed order.  One block per t.
__global__ __launch_bounds__(kThreads) void k_finish_sums(const double* __restrict__ part, uint64_t nb,
                                                         double* __restrict__ out)
{
    __shared__ double lds[kThreads];
    const double* p = part + uint64_t(blockIdx.x) * nb;
    double acc = 0.0;
    for (uint64_t b = threadIdx.x; b < nb; b += kThreads) acc = __dadd_rn(acc, p[b]);
    const double s = block_sum(acc, lds);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// k_finish_sums for a group of sweeps: block (t, y) finishes term t of
// sweep y (its partials at part + y * stride, nb_z blocks for the first
// n_z sweeps, nb_xy for the others) into out[y * slot + t], in the same
// order as k_finish_sums.
__global__ __launch_bounds__(kThreads) void k_finish_group(const double* __restrict__ part, uint64_t stride,
                                                          const ExpectArgs* __restrict__ args, uint32_t n_z,
                                                          uint64_t nb_z, uint64_t nb_xy, double* __restrict__ out,
                                                          uint32_t slot)
{
    __shared__ double lds[kThreads];
    const uint32_t y = blockIdx.y;
    if (int(blockIdx.x) > args[y].n_terms) return;
    const uint64_t nb = y < n_z ? nb_z : nb_xy;
    const double* p = part + y * stride + uint64_t(blockIdx.x) * nb;
    double acc = 0.0;
    for (uint64_t b = threadIdx.x; b < nb; b += kThreads) acc = __dadd_rn(acc, p[b]);
    const double s = block_sum(acc, lds);
    if (threadIdx.x == 0) out[uint64_t(y) * slot + blockIdx.x] = s;
}

// ----------------------------------------------------------------- sampler
//
// Three-level inverse CDF whose boundaries are monotone bit for bit, so the
// search is always consistent and never lands on a zero-probability index.
// The state splits into nc chunks of cs amplitudes, each chunk into blocks
// of W = 64 amplitudes (W = dim below 64):
//   block sums: the sequential FP64 sum of a block's probabilities in index
//     order;
//   block prefixes C: inside a chunk, the sequential running sum of its
//     block sums (C[b] = C[b-1] + sum_b); the chunk total S[c] is its last C;
//   chunk boundaries B[0..nc] from S by per-thread sequential prefixes plus a
//     sequential pass over thread totals (B[c+1] == B[c] whenever S[c] == 0);
//   for a shot, r = u * B[nc]; chunk c = smallest c with r < B[c+1]; block
//     b = smallest b with r < B[c] + C[b]; inside the block, the outcome is
//     the smallest i with r < B[c] + (E + l_i), where E = C[b-1] (0 for the
//     first block) and l_i the sequential running sum of the block's
//     probabilities.  Its last value equals the block sum bit for bit, so
//     E + l_last == C[b] and the boundaries join up exactly.
// A zero-probability amplitude repeats the previous boundary exactly (inside
// a block, across blocks, and at the start of a chunk, which only a shot with
// r >= B[c] reaches), so it can never be the first index whose boundary
// exceeds r.
//
// Only the block prefixes need the whole state: one coalesced read sweep.
// Each shot then reads one block of W amplitudes, so a sample costs about one
// state read plus W amplitudes per shot, at any number of shots.

struct SampleLayout {
    uint64_t nc;     // chunks
    uint64_t cs;     // amplitudes per chunk
    int w;           // amplitudes per block
    uint64_t nbk;    // blocks per chunk
};

constexpr int kBlk = 64;         // amplitudes per block (states of >= 64 amplitudes)
constexpr uint64_t kSub = 4096;  // amplitudes per LDS sub-tile of the prefix sweep

SampleLayout sample_layout(int n)
{
    const uint64_t dim = uint64_t(1) << n;
    uint64_t nc = dim / (4 * kSub);
    if (nc < 1) nc = 1;
    if (nc > 65536) nc = 65536;
    const uint64_t cs = dim / nc;
    const int w = int(std::min<uint64_t>(kBlk, cs));
    return {nc, cs, w, cs / uint64_t(w)};
}

__device__ __forceinline__ double readlane_f64(double v, int lane)
{
    const uint64_t b = uint64_t(__double_as_longlong(v));
    const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(b)), lane));
    const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(b >> 32)), lane));
    return __longlong_as_double((long long)((uint64_t(hi) << 32) | lo));
}

// Block prefixes C and chunk totals S.  One workgroup per chunk (grid-
// stride); a chunk is read in sub-tiles of up to kSub amplitudes, coalesced,
// whose probabilities go to LDS as rows of one block each (padded by one
// slot).  Lane l of wave 0 then sums row l in index order, and the wave
// extends the chunk's running prefix over the rows in order, lane by lane,
// with the running value held identically in every lane.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_block_prefix(const typename Cx<R>::T* __restrict__ psi,
                                                          SampleLayout L, double* __restrict__ C,
                                                          double* __restrict__ S)
{
    using T2 = typename Cx<R>::T;
    constexpr int kRow = kBlk + 1;
    constexpr int kPer = int(kSub) / kThreads;
    __shared__ double p[(kSub / kBlk) * kRow];
    const int tid = threadIdx.x, lane = tid & 63;
    if (blockIdx.x >= L.nc) return;
    const uint64_t sub_len = L.cs < kSub ? L.cs : kSub;
    const uint64_t nsub = L.cs / sub_len;
    const int rows = int(sub_len / uint64_t(L.w));
    const int wshift = __ffs(L.w) - 1;
    // this workgroup's sub-tiles in order: step k is sub-tile k % nsub of
    // chunk blockIdx.x + (k / nsub) * gridDim.x
    const uint64_t steps = ((L.nc - blockIdx.x + gridDim.x - 1) / gridDim.x) * nsub;
    auto src_of = [&](uint64_t k) {
        return psi + (blockIdx.x + (k / nsub) * gridDim.x) * L.cs + (k % nsub) * sub_len;
    };
    const bool full = sub_len == kSub;
    T2 v[kPer];
    if (full) {
        const T2* src = src_of(0);
#pragma unroll
        for (int u = 0; u < kPer; ++u) v[u] = src[u * kThreads + tid];
    }
    double carry = 0.0;
    for (uint64_t k = 0; k < steps; ++k) {
        const uint64_t c = blockIdx.x + (k / nsub) * gridDim.x, sb = k % nsub;
        if (sb == 0) carry = 0.0;
        if (full) {
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                const int i = u * kThreads + tid;
                p[(i >> wshift) * kRow + (i & (L.w - 1))] = prob(v[u]);
            }
        } else {
            const T2* src = src_of(k);
            for (int i = tid; i < int(sub_len); i += kThreads)
                p[(i >> wshift) * kRow + (i & (L.w - 1))] = prob(src[i]);
        }
        __syncthreads();
        // the next sub-tile streams in while wave 0 sums this one
        if (full && k + 1 < steps) {
            const T2* src = src_of(k + 1);
#pragma unroll
            for (int u = 0; u < kPer; ++u) v[u] = src[u * kThreads + tid];
        }
        if (tid < 64) {
            double sum = 0.0;
            if (lane < rows) {
                if (L.w == kBlk) {
                    // the row's loads issued kQ at a time, then summed in order
                    constexpr int kQ = sizeof(R) == 4 ? 16 : 8;
                    for (int j0 = 0; j0 < kBlk; j0 += kQ) {
                        double q[kQ];
#pragma unroll
                        for (int j = 0; j < kQ; ++j) q[j] = p[lane * kRow + j0 + j];
#pragma unroll
                        for (int j = 0; j < kQ; ++j) sum = __dadd_rn(sum, q[j]);
                    }
                } else {
                    for (int j = 0; j < L.w; ++j) sum = __dadd_rn(sum, p[lane * kRow + j]);
                }
            }
            double mine = 0.0;
            for (int l = 0; l < rows; ++l) {
                carry = __dadd_rn(carry, readlane_f64(sum, l));
                if (lane == l) mine = carry;
            }
            if (lane < rows) C[c * L.nbk + sb * uint64_t(rows) + lane] = mine;
            if (tid == 0 && sb == nsub - 1) S[c] = carry;
        }
        __syncthreads();
    }
}

// Block prefixes C and chunk totals S for chunks of whole segments of
// kSegBlocks blocks of kBlk amplitudes (complex64 states of >= 14 qubits):
// one workgroup per chunk, one block per thread.  Each thread sums its block's
// probabilities in index order straight from its loads (no LDS staging),
// then the waves extend the chunk's running prefix over their blocks in
// order, lane by lane, wave after wave, segment after segment: the same
// sums in the same order as k_block_prefix, so C and S are bitwise the same.
constexpr int kSegBlocks = kThreads;  // blocks per segment (one per thread)

template <typename R>
__global__ __launch_bounds__(kThreads) void k_block_prefix_rows(const typename Cx<R>::T* __restrict__ psi,
                                                               SampleLayout L, double* __restrict__ C,
                                                               double* __restrict__ S)
{
    using T2 = typename Cx<R>::T;
    constexpr int kQ = sizeof(R) == 4 ? 16 : 8;  // amplitudes loaded at a time
    __shared__ double carry_out;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t c = blockIdx.x;
    const uint64_t nseg = L.nbk / kSegBlocks;
    double carry = 0.0;  // the chunk's running prefix (uniform)
    for (uint64_t sg = 0; sg < nseg; ++sg) {
        const uint64_t b = sg * kSegBlocks + uint64_t(tid);
        const T2* blk = psi + c * L.cs + b * kBlk;
        double sum = 0.0;
        for (int j0 = 0; j0 < kBlk; j0 += kQ) {
            T2 v[kQ];
#pragma unroll
            for (int j = 0; j < kQ; ++j) v[j] = blk[j0 + j];
#pragma unroll
            for (int j = 0; j < kQ; ++j) sum = __dadd_rn(sum, prob(v[j]));
        }
        // wave w extends the prefix over its 64 blocks once waves 0..w-1 have
        for (int w = 0; w < kSegBlocks / 64; ++w) {
            if (wave == w) {
                if (w > 0) carry = carry_out;
                double mine = 0.0;
                for (int l = 0; l < 64; ++l) {
                    carry = __dadd_rn(carry, readlane_f64(sum, l));
                    if (lane == l) mine = carry;
                }
                C[c * L.nbk + b] = mine;
                if (lane == 0) carry_out = carry;
            }
            __syncthreads();
        }
        carry = carry_out;
        __syncthreads();
    }
    if (tid == 0) S[c] = carry;
}

constexpr int kScanThreads = 1024;
constexpr int kScanRound = 8192;                      // chunk totals staged in LDS per round
constexpr int kScanPad = kScanRound + kScanRound / 64;  // one pad slot per 64

__device__ __forceinline__ int scan_slot(int i) { return i + (i >> 6); }

// B[0..nc] from S[0..nc-1] (single workgroup).  Thread t owns the chunks
// [t * per, (t + 1) * per): its local prefix is the sequential sum of their
// totals, the offsets o_t of the threads are the sequential sum of the
// thread totals in thread order, and B[c + 1] = o_t + local_c.  Since
// local_last == tot_t and o_{t+1} = o_t + tot_t with the same rounding, the
// boundaries are monotone across threads and B[c + 1] == B[c] whenever
// S[c] == 0.  S and B move between HBM and LDS in coalesced rounds of
// kScanRound chunks (per divides kScanRound), the owners of a round's
// chunks walk them in LDS, and the chain over the thread totals runs in
// wave 0 from registers.
__global__ __launch_bounds__(kScanThreads) void k_scan_chunks(const double* __restrict__ S, uint64_t nc,
                                                             double* __restrict__ B)
{
    __shared__ double stage[kScanPad];
    __shared__ double tot[kScanThreads];
    __shared__ double off[kScanThreads];
    const int t = threadIdx.x;
    const uint64_t per = (nc + kScanThreads - 1) / kScanThreads;
    const uint64_t lo = std::min<uint64_t>(nc, t * per);
    const uint64_t hi = std::min<uint64_t>(nc, lo + per);
    double run = 0.0;
    for (uint64_t r0 = 0; r0 < nc; r0 += kScanRound) {
        const int len = int(std::min<uint64_t>(kScanRound, nc - r0));
        for (int i = t; i < len; i += kScanThreads) stage[scan_slot(i)] = S[r0 + i];
        __syncthreads();
        if (lo >= r0 && lo < r0 + uint64_t(len)) {
            const int b0 = int(lo - r0), cnt = int(hi - lo);
            int i = 0;
            for (; i + 16 <= cnt; i += 16) {
                double q[16];
#pragma unroll
                for (int j = 0; j < 16; ++j) q[j] = stage[scan_slot(b0 + i + j)];
#pragma unroll
                for (int j = 0; j < 16; ++j) run = __dadd_rn(run, q[j]);
            }
            for (; i < cnt; ++i) run = __dadd_rn(run, stage[scan_slot(b0 + i)]);
        }
        __syncthreads();
    }
    tot[t] = run;
    __syncthreads();
    if (t < 64) {
        // lane l holds the totals of threads 16 l .. 16 l + 15
        constexpr int kPerLane = kScanThreads / 64;
        double v[kPerLane], mine[kPerLane];
#pragma unroll
        for (int j = 0; j < kPerLane; ++j) {
            v[j] = tot[t * kPerLane + j];
            mine[j] = 0.0;
        }
        double o = 0.0;
        for (int l = 0; l < 64; ++l) {
#pragma unroll
            for (int j = 0; j < kPerLane; ++j) {
                if (t == l) mine[j] = o;
                o = __dadd_rn(o, readlane_f64(v[j], l));
            }
        }
#pragma unroll
        for (int j = 0; j < kPerLane; ++j) off[t * kPerLane + j] = mine[j];
    }
    __syncthreads();
    const double o = off[t];
    run = 0.0;
    for (uint64_t r0 = 0; r0 < nc; r0 += kScanRound) {
        const int len = int(std::min<uint64_t>(kScanRound, nc - r0));
        for (int i = t; i < len; i += kScanThreads) stage[scan_slot(i)] = S[r0 + i];
        __syncthreads();
        if (lo >= r0 && lo < r0 + uint64_t(len)) {
            const int b0 = int(lo - r0), cnt = int(hi - lo);
            int i = 0;
            for (; i + 16 <= cnt; i += 16) {
                double q[16];
#pragma unroll
                for (int j = 0; j < 16; ++j) q[j] = stage[scan_slot(b0 + i + j)];
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    run = __dadd_rn(run, q[j]);
                    q[j] = __dadd_rn(o, run);
                }
#pragma unroll
                for (int j = 0; j < 16; ++j) stage[scan_slot(b0 + i + j)] = q[j];
            }
            for (; i < cnt; ++i) {
                const int k = scan_slot(b0 + i);
                run = __dadd_rn(run, stage[k]);
                stage[k] = __dadd_rn(o, run);
            }
        }
        __syncthreads();
        for (int i = t; i < len; i += kScanThreads) B[r0 + i + 1] = stage[scan_slot(i)];
        __syncthreads();
    }
    if (t == 0) B[0] = 0.0;
}

__device__ __forceinline__ double shot_r(double u, double total)
{
    double r = __dmul_rn(u, total);
    if (!(r < total)) r = nextafter(total, 0.0);
    return r;
}

// ------------------------------------------------------- shot buckets
//
// The shots of a batch are resolved in chunk order.  A first pass finds
// each shot's chunk (a binary search over B inside the range a guide table
// gives) and its rank among the shots of that chunk (one atomic counter per
// chunk); an exclusive scan of the counters gives the buckets' offsets; a
// second pass puts each shot (its chunk and index, and r) at its bucket's
// offset plus its rank; the resolver then takes the buckets in order, one
// shot per thread, so the shots of one chunk run in the same workgroup and
// share the lines of the chunk's block prefixes and of the blocks they land
// in, instead of each shot fetching its own.  Ranks follow the order of the
// atomic additions and may differ between runs; each outcome depends only
// on its shot's r, so the outputs do not.
//
// counts[nc] is a flag that the first pass sets when a uniform lies outside
// [0, 1) (or is NaN); such a shot is resolved as u = 0.

// Smallest chunk c in [lo, hi] with r < B[c+1], or hi if there is none.
__device__ __forceinline__ uint32_t chunk_in(const double* __restrict__ B, uint64_t lo, uint64_t hi, double r)
{
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (r < B[mid + 1])
            hi = mid;
        else
            lo = mid + 1;
    }
    return uint32_t(lo);
}

__device__ __forceinline__ double checked_uniform(double u, bool* bad)
{
    if (u >= 0.0 && u < 1.0) return u;
    *bad = true;
    return 0.0;
}

// Guide table of the chunk search (a cutpoint table): G[k] is the chunk of
// the point u = k / 2^g, for k = 0 .. 2^g.  Since r = u * N and the chunk
// are monotone in u, a shot with k / 2^g <= u < (k + 1) / 2^g has its chunk
// in [G[k], G[k+1]], a range of one or two chunks unless many chunks hold
// little probability between two cutpoints.
__global__ __launch_bounds__(kThreads) void k_chunk_guide(SampleLayout L, const double* __restrict__ B, int g,
                                                         uint32_t* __restrict__ G)
{
    const uint64_t k = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k > (uint64_t(1) << g)) return;
    G[k] = chunk_in(B, 0, L.nc - 1, shot_r(ldexp(double(k), -g), B[L.nc]));
}

// Lanes of a wave that add to the same counter form a group: the group's
// lowest lane adds the group's size once, and every lane gets the counter's
// old value plus its rank in the group (lanes in lane order).  All lanes of
// the wave take part; inactive lanes add nothing.
__device__ __forceinline__ uint32_t wave_claim(uint32_t* __restrict__ ctr, uint32_t c, bool act)
{
    const int lane = threadIdx.x & 63;
    uint64_t todo = __ballot(act);
    uint64_t peers = 0;
    while (todo) {
        const int l = __ffsll((unsigned long long)todo) - 1;
        const uint32_t cl = uint32_t(__builtin_amdgcn_readlane(int(c), l));
        const uint64_t m = __ballot(act && c == cl);
        if (act && c == cl) peers = m;
        todo &= ~m;
    }
    const int leader = act ? __ffsll((unsigned long long)peers) - 1 : lane;
    uint32_t base = 0;
    if (act && lane == leader) base = atomicAdd(ctr + c, uint32_t(__popcll(peers)));
    base = uint32_t(__shfl(int(base), leader, 64));
    return base + uint32_t(__popcll(peers & ((uint64_t(1) << lane) - 1)));
}

__global__ __launch_bounds__(kThreads) void k_fill_u32(uint32_t* __restrict__ p, uint64_t n)
{
    const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Each shot's chunk (through the guide table) and its rank among the shots
// of that chunk.
__global__ __launch_bounds__(kThreads) void k_shot_chunks(SampleLayout L, const double* __restrict__ B,
                                                         const uint32_t* __restrict__ G, int g,
                                                         const double* __restrict__ u, uint64_t ns,
                                                         uint32_t* __restrict__ key, uint32_t* __restrict__ rank,
                                                         uint32_t* __restrict__ counts)
{
    const uint64_t s = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool act = s < ns;
    uint32_t c = 0;
    if (act) {
        bool bad = false;
        const double us = checked_uniform(u[s], &bad);
        if (bad) counts[L.nc] = 1u;
        const uint64_t k = uint64_t(ldexp(us, g));  // < 2^g
        c = chunk_in(B, G[k], G[k + 1], shot_r(us, B[L.nc]));
        key[s] = c;
    }
    const uint32_t rk = wave_claim(counts, c, act);
    if (act) rank[s] = rk;
}

constexpr int kCountThreads = 1024;
constexpr int kCountTiles = 64;  // counts per thread: nc <= kCountThreads * kCountTiles

// Exclusive scan of counts[0..nc) into off[0..nc] (single workgroup).
// Element e = j * 1024 + t is thread t's item of tile j (coalesced loads and
// stores).  A first pass takes every wave's total of every tile, those are
// scanned in LDS (over the waves of a tile, then over the tiles), and a
// second pass scans each tile inside its waves and adds the two offsets.
__global__ __launch_bounds__(kCountThreads) void k_scan_counts(const uint32_t* __restrict__ counts, uint64_t nc,
                                                              uint32_t* __restrict__ off)
{
    __shared__ uint32_t wtot[kCountThreads / 64][kCountTiles];
    __shared__ uint32_t jtot[kCountTiles + 1];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int J = int((nc + kCountThreads - 1) / kCountThreads);
#pragma unroll 8
    for (int j = 0; j < J; ++j) {
        const uint64_t e = uint64_t(j) * kCountThreads + t;
        uint32_t x = e < nc ? counts[e] : 0u;
        for (int d = 32; d > 0; d >>= 1) x += uint32_t(__shfl_xor(int(x), d, 64));
        if (lane == 0) wtot[w][j] = x;
    }
    __syncthreads();
    if (t < J) {  // column t: exclusive prefix over the waves, and the tile total
        uint32_t run = 0;
        for (int ww = 0; ww < kCountThreads / 64; ++ww) {
            const uint32_t x = wtot[ww][t];
            wtot[ww][t] = run;
            run += x;
        }
        jtot[t] = run;
    }
    __syncthreads();
    if (t == 0) {
        uint32_t run = 0;
        for (int j = 0; j < J; ++j) {
            const uint32_t x = jtot[j];
            jtot[j] = run;
            run += x;
        }
        jtot[kCountTiles] = run;
    }
    __syncthreads();
#pragma unroll 8
    for (int j = 0; j < J; ++j) {
        const uint64_t e = uint64_t(j) * kCountThreads + t;
        const uint32_t x = e < nc ? counts[e] : 0u;
        uint32_t incl = x;
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = uint32_t(__shfl_up(int(incl), d, 64));
            if (lane >= d) incl += y;
        }
        if (e < nc) off[e] = jtot[j] + wtot[w][j] + (incl - x);
    }
    if (t == 0) off[nc] = jtot[kCountTiles];
}

// Places each shot in its chunk's bucket: sorted[pos] = chunk << 32 | shot,
// rs[pos] = r, pos = the bucket's offset plus the shot's rank in it.
__global__ __launch_bounds__(kThreads) void k_shot_place(SampleLayout L, const double* __restrict__ B,
                                                        const double* __restrict__ u, uint64_t ns,
                                                        const uint32_t* __restrict__ key,
                                                        const uint32_t* __restrict__ rank,
                                                        const uint32_t* __restrict__ off,
                                                        uint64_t* __restrict__ sorted, double* __restrict__ rs)
{
    const uint64_t s = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= ns) return;
    const uint32_t c = key[s];
    if (c >= L.nc) return;
    bool bad = false;
    const double us = checked_uniform(u[s], &bad);
    const uint64_t pos = uint64_t(off[c]) + rank[s];
    if (pos < ns) {
        sorted[pos] = (uint64_t(c) << 32) | uint64_t(uint32_t(s));
        rs[pos] = shot_r(us, B[L.nc]);
    }
}

// One thread per placed shot, in bucket order: block by binary search over
// the chunk's C, then the block's amplitudes in order.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_resolve(const typename Cx<R>::T* __restrict__ psi,
                                                     SampleLayout L, const double* __restrict__ B,
                                                     const double* __restrict__ C,
                                                     const uint64_t* __restrict__ sorted,
                                                     const double* __restrict__ rs, uint64_t ns,
                                                     uint64_t* __restrict__ idx_out)
{
    using T2 = typename Cx<R>::T;
    const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= ns) return;
    const uint64_t e0 = sorted[i];
    const uint64_t c = e0 >> 32, s = e0 & 0xffffffffu;
    if (c >= L.nc || s >= ns) return;
    if (!(B[L.nc] > 0.0)) {  // a zero state: the call reports the error
        idx_out[s] = 0;
        return;
    }
    const double r = rs[i];
    const double base = B[c];
    const double* cc = C + c * L.nbk;
    const T2* chunk = psi + c * L.cs;
    uint64_t found = ~uint64_t(0);
    if (r < __dadd_rn(base, cc[L.nbk - 1])) {
        uint64_t b0 = 0, b1 = L.nbk - 1;  // smallest b with r < base + C[b]
        while (b0 < b1) {
            const uint64_t mid = b0 + (b1 - b0) / 2;
            if (r < __dadd_rn(base, cc[mid]))
                b1 = mid;
            else
                b0 = mid + 1;
        }
        const double e = b0 ? cc[b0 - 1] : 0.0;
        const T2* blk = chunk + b0 * uint64_t(L.w);
        double run = 0.0;
        constexpr int kAhead = 16;
        for (int j0 = 0; j0 < L.w && found == ~uint64_t(0); j0 += kAhead) {
            T2 v[kAhead];
#pragma unroll
            for (int j = 0; j < kAhead; ++j)
                if (j0 + j < L.w) v[j] = blk[j0 + j];
#pragma unroll
            for (int j = 0; j < kAhead; ++j) {
                if (j0 + j < L.w && found == ~uint64_t(0)) {
                    run = __dadd_rn(run, prob(v[j]));
                    if (r < __dadd_rn(base, __dadd_rn(e, run))) found = c * L.cs + b0 * uint64_t(L.w) + uint64_t(j0 + j);
                }
            }
        }
    }
    if (found == ~uint64_t(0)) {
        // rounding left r at or past B[c] + C[last] (B[c+1] comes from a
        // different summation order): take the chunk's last amplitude with
        // non-zero probability (the chunk has one, since S[c] > 0 whenever
        // the chunk can be chosen)
        found = c * L.cs;
        for (uint64_t k = L.cs; k-- > 0;) {
            if (prob(chunk[k]) > 0.0) {
                found = c * L.cs + k;
                break;
            }
        }
    }
    idx_out[s] = found;
}

struct BitArgs {
    int32_t n_bits;
    int32_t bits[SV_MAX_QUBITS];
};

__global__ __launch_bounds__(kThreads) void k_extract_bits(uint64_t* __restrict__ idx, uint64_t ns, BitArgs a)
{
    const uint64_t s = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= ns) return;
    const uint64_t v = idx[s];
    uint64_t o = 0;
    for (int b = 0; b < a.n_bits; ++b) o |= ((v >> a.bits[b]) & 1u) << b;
    idx[s] = o;
}

template <typename R>
double run_norm_t(sv_handle_s* h, const void* psi_v, int n)
{
    using T2 = typename Cx<R>::T;
    const T2* psi = static_cast<const T2*>(psi_v);
    const uint64_t dim = uint64_t(1) << n;
    const Partition P = partition(dim);
    double* part = reinterpret_cast<double*>(h->ws + kMatRingBytes);
    double* res = part + P.nb;
    ExpectArgs a{};
    a.per = P.per;
    a.n_terms = 0;
    a.n_active = 0;
    hipLaunchKernelGGL((k_expect_z<R>), dim3(unsigned(P.nb)), dim3(kThreads), 0, h->stream, psi, a, part);
    SV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_finish_sums, dim3(1), dim3(kThreads), 0, h->stream, part, P.nb, res);
    SV_HIP(hipGetLastError());
    double out = 0.0;
    SV_HIP(hipMemcpyAsync(&out, res, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    SV_HIP(hipStreamSynchronize(h->stream));
    return out;
}

int highest_bit(uint64_t v)
{
    int b = -1;
    while (v) {
        v >>= 1;
        ++b;
    }
    return b;
}

template <typename R>
void run_expect_t(sv_handle_s* h, const void* psi_v, int n, const PauliMasks* terms, int n_terms, double* out)
{
    using T2 = typename Cx<R>::T;
    const T2* psi = static_cast<const T2*>(psi_v);
    const uint64_t dim = uint64_t(1) << n;
    // Sweeps: one per distinct X/Y mask and per kMaxTermsPerSweep terms.
    // Z-type terms (x == 0) whose mask meets the bits that vary inside a
    // thread need per-item work: at most kMaxActive of them per sweep, placed
    // first; the others only flip the sign of the plain sum.
    std::vector<int> order(n_terms);
    for (int t = 0; t < n_terms; ++t) order[t] = t;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return terms[a].x < terms[b].x; });
    double* part = reinterpret_cast<double*>(h->ws + kMatRingBytes);
    std::vector<double> sums(n_terms, 0.0);
    double norm = -1.0;
    struct Launch {
        std::vector<int> idx;  // term indices, active ones first
        int n_active;
    };
    std::vector<Launch> launches;
    const uint64_t zvary = (partition(dim).per - 1) & ~uint64_t(kThreads - 1);
    for (int i = 0; i < n_terms;) {
        int j = i;
        while (j < n_terms && terms[order[j]].x == terms[order[i]].x) ++j;
        if (terms[order[i]].x == 0) {
            std::vector<int> act, pas;
            for (int k = i; k < j; ++k) ((terms[order[k]].z & zvary) ? act : pas).push_back(order[k]);
            size_t ia = 0, ip = 0;
            while (ia < act.size() || ip < pas.size()) {
                Launch L;
                while (ia < act.size() && L.idx.size() < size_t(kMaxActive)) L.idx.push_back(act[ia++]);
                L.n_active = int(L.idx.size());
                while (ip < pas.size() && L.idx.size() < size_t(kMaxTermsPerSweep)) L.idx.push_back(pas[ip++]);
                launches.push_back(std::move(L));
            }
        } else {
            for (int k = i; k < j; k += kMaxTermsPerSweep) {
                Launch L;
                for (int m = k; m < std::min(j, k + kMaxTermsPerSweep); ++m) L.idx.push_back(order[m]);
                L.n_active = int(L.idx.size());
                launches.push_back(std::move(L));
            }
        }
        i = j;
    }
    // Sweeps in groups of up to kGroup, read back once per group: each
    // sweep's finished sums go to its own slot of the results area.  A large
    // state's sweeps are launched one by one and reuse the partials after
    // the results area (each finish consumes them before the next sweep
    // writes them: one stream).  A small state's group takes one launch per
    // kind (its Z-type sweeps, which come first, then its pair sweeps) and
    // one finish, each sweep with partials of its own.
    constexpr size_t kGroup = 64, kSlot = kMaxTermsPerSweep + 1;
    constexpr int kGroupedQubits = 22;
    auto make_args = [&](const Launch& L) {
        const uint64_t x = terms[L.idx[0]].x;
        ExpectArgs a{};
        a.per = partition(x != 0 ? dim / 2 : dim).per;
        a.x = x;
        a.hbit = x != 0 ? highest_bit(x) : 0;
        a.n_terms = int(L.idx.size());
        a.n_active = L.n_active;
        for (int t = 0; t < a.n_terms; ++t) {
            a.z[t] = terms[L.idx[t]].z;
            a.ny[t] = terms[L.idx[t]].ny;
        }
        return a;
    };
    const bool grouped = n <= kGroupedQubits;
    const Partition Pz = partition(dim), Pxy = partition(dim > 1 ? dim / 2 : 1);
    const uint64_t stride = kSlot * Pz.nb;  // one sweep's partials (pair sweeps have fewer blocks)
    double* res_dev = part;
    double* parts = part + kGroup * kSlot;
    size_t group = kGroup;
    if (grouped) {
        const size_t room = (h->ws_bytes - kMatRingBytes) / sizeof(double) - kGroup * kSlot;
        group = std::max<size_t>(1, std::min<size_t>(kGroup, room / stride));
    }
    std::vector<double> host(kGroup * kSlot);
    std::vector<ExpectArgs> ga;
    for (size_t g0 = 0; g0 < launches.size(); g0 += group) {
        const size_t g1 = std::min(launches.size(), g0 + group);
        if (grouped) {
            ga.clear();
            uint32_t n_z = 0;
            for (size_t li = g0; li < g1; ++li) {
                ga.push_back(make_args(launches[li]));
                if (ga.back().x == 0) ++n_z;
            }
            const uint32_t n_all = uint32_t(ga.size());
            const ExpectArgs* dargs =
                static_cast<const ExpectArgs*>(stage_matrix(h, ga.data(), sizeof(ExpectArgs) * ga.size()));
            if (n_z > 0)
                hipLaunchKernelGGL((k_expect_z_group<R>), dim3(unsigned(Pz.nb), n_z), dim3(kThreads), 0, h->stream,
                                   psi, dargs, parts, stride);
            if (n_all > n_z)
                hipLaunchKernelGGL((k_expect_xy_group<R>), dim3(unsigned(Pxy.nb), n_all - n_z), dim3(kThreads), 0,
                                   h->stream, psi, dargs + n_z, parts + n_z * stride, stride);
            SV_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_finish_group, dim3(unsigned(kSlot), n_all), dim3(kThreads), 0, h->stream, parts,
                               stride, dargs, n_z, Pz.nb, Pxy.nb, res_dev, uint32_t(kSlot));
            SV_HIP(hipGetLastError());
        } else {
            for (size_t li = g0; li < g1; ++li) {
                const ExpectArgs a = make_args(launches[li]);
                const Partition P = partition(a.x != 0 ? dim / 2 : dim);
                if (a.x != 0)
                    hipLaunchKernelGGL((k_expect_xy<R>), dim3(unsigned(P.nb)), dim3(kThreads), 0, h->stream, psi, a,
                                       parts);
                else
                    hipLaunchKernelGGL((k_expect_z<R>), dim3(unsigned(P.nb)), dim3(kThreads), 0, h->stream, psi, a,
                                       parts);
                SV_HIP(hipGetLastError());
                hipLaunchKernelGGL(k_finish_sums, dim3(unsigned(a.n_terms + 1)), dim3(kThreads), 0, h->stream,
                                   parts, P.nb, res_dev + (li - g0) * kSlot);
                SV_HIP(hipGetLastError());
            }
        }
        SV_HIP(hipMemcpyAsync(host.data(), res_dev, sizeof(double) * kSlot * (g1 - g0), hipMemcpyDeviceToHost,
                              h->stream));
        SV_HIP(hipStreamSynchronize(h->stream));
        for (size_t li = g0; li < g1; ++li) {
            const Launch& L = launches[li];
            const int nt = int(L.idx.size());
            const double* r = host.data() + (li - g0) * kSlot;
            for (int t = 0; t < nt; ++t) sums[L.idx[t]] = r[t];
            if (norm < 0.0) norm = r[nt];
        }
    }
    if (!(norm > 0.0)) throw Error{SV_ERR_INVALID_VALUE, "state has zero norm"};
    for (int t = 0; t < n_terms; ++t) out[t] = sums[t] / norm;
}

// Device buffers of one sampling call: block prefixes C (nc * nbk
// doubles), chunk totals S (nc), chunk boundaries B (nc + 1), bucket counts
// (nc + 1: the last is the flag for uniforms outside [0, 1)) and offsets
// (nc + 1), and per shot of a batch its chunk, its bucket entry and its r;
// with host uniforms and outputs also a batch of uniforms and indices.
struct SampleBuffers {
    double* C;
    double* S;
    double* B;
    uint32_t* counts;
    uint32_t* off;
    uint32_t* guide;
    uint32_t* key;
    uint32_t* rank;
    uint64_t* sorted;
    double* rs;
    double* du;
    uint64_t* didx;
    int64_t batch;
};

constexpr int kGuideMaxBits = 16;
constexpr size_t kShotBytes = 2 * sizeof(uint32_t) + sizeof(uint64_t) + sizeof(double);  // key, rank, sorted, rs
constexpr size_t kHostShotBytes = sizeof(double) + sizeof(uint64_t);                    // du, didx
constexpr size_t kCarveAlign = 256;

constexpr size_t carve_size(size_t bytes) { return (bytes + kCarveAlign - 1) & ~(kCarveAlign - 1); }

// Bytes of the per-call part of SampleBuffers (everything but C).
constexpr size_t sample_fixed_bytes(uint64_t nc)
{
    return carve_size(sizeof(double) * nc) + carve_size(sizeof(double) * (nc + 1)) +
           2 * carve_size(sizeof(uint32_t) * (nc + 1)) + carve_size(sizeof(uint32_t) * ((size_t(1) << kGuideMaxBits) + 1));
}

// Bytes of a shot batch.
constexpr size_t sample_batch_bytes(int64_t batch, bool host_io)
{
    const size_t b = size_t(batch);
    size_t t = 2 * carve_size(sizeof(uint32_t) * b) + carve_size(sizeof(uint64_t) * b) + carve_size(sizeof(double) * b);
    if (host_io) t += carve_size(sizeof(double) * b) + carve_size(sizeof(uint64_t) * b);
    return t;
}

// Lays SampleBuffers (all but C) out from w.
void carve_sample_buffers(char* w, uint64_t nc, int64_t batch, bool host_io, SampleBuffers& sb)
{
    auto take = [&](size_t bytes) {
        char* p = w;
        w += carve_size(bytes);
        return p;
    };
    sb.S = reinterpret_cast<double*>(take(sizeof(double) * nc));
    sb.B = reinterpret_cast<double*>(take(sizeof(double) * (nc + 1)));
    sb.counts = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * (nc + 1)));
    sb.off = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * (nc + 1)));
    sb.guide = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * ((size_t(1) << kGuideMaxBits) + 1)));
    const size_t b = size_t(batch);
    sb.key = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * b));
    sb.rank = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * b));
    sb.sorted = reinterpret_cast<uint64_t*>(take(sizeof(uint64_t) * b));
    sb.rs = reinterpret_cast<double*>(take(sizeof(double) * b));
    sb.du = host_io ? reinterpret_cast<double*>(take(sizeof(double) * b)) : nullptr;
    sb.didx = host_io ? reinterpret_cast<uint64_t*>(take(sizeof(uint64_t) * b)) : nullptr;
    sb.batch = batch;
}

// Bits of the guide table for a batch of ns shots on nc chunks: about one
// cutpoint per 16 shots, at most four per chunk and 2^16 in all.
int guide_bits(uint64_t ns, uint64_t nc)
{
    int g = 0;
    while (g < kGuideMaxBits && (uint64_t(16) << (g + 1)) <= ns && (uint64_t(1) << (g + 1)) <= 4 * nc) ++g;
    return g;
}

// The sampler's launches.  With host_io, u and out are host arrays (each
// batch's uniforms go to the device and its outcomes come back); otherwise
// they are device arrays that the kernels read and write directly.  Blocks
// until the outcomes are written; the norm and the uniforms are checked at
// the end (on an error the outputs are unspecified).
template <typename R>
void sample_core(hipStream_t stream, int cu_count, const void* psi_v, int n, const double* u, int64_t n_shots,
                 const int32_t* bit_ordering, int n_bits, uint64_t* out, const SampleBuffers& sb, bool host_io)
{
    using T2 = typename Cx<R>::T;
    const T2* psi = static_cast<const T2*>(psi_v);
    const SampleLayout L = sample_layout(n);
    // complex64 rows (512 B per thread) stream well from the threads'
    // own loads; complex128 rows (1 KB) lose lines to eviction before
    // their threads have read them (1.46x the bytes in the HBM counters)
    // and take the LDS-staged sweep
    if (sizeof(R) == 4 && L.w == kBlk && L.nbk % kSegBlocks == 0)
        hipLaunchKernelGGL((k_block_prefix_rows<R>), dim3(unsigned(L.nc)), dim3(kThreads), 0, stream, psi, L, sb.C,
                           sb.S);
    else
        hipLaunchKernelGGL((k_block_prefix<R>), dim3(unsigned(std::min<uint64_t>(L.nc, uint64_t(cu_count) * 8))),
                           dim3(kThreads), 0, stream, psi, L, sb.C, sb.S);
    SV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_scan_chunks, dim3(1), dim3(kScanThreads), 0, stream, sb.S, L.nc, sb.B);
    SV_HIP(hipGetLastError());

    if (L.nc > uint64_t(kCountThreads) * kCountTiles) throw Error{SV_ERR_INTERNAL, "sampler chunk count"};
    BitArgs ba{};
    ba.n_bits = n_bits;
    for (int b = 0; b < n_bits; ++b) ba.bits[b] = bit_ordering[b];
    int g_built = -1;  // bits of the guide table in sb.guide
    for (int64_t s0 = 0; s0 < n_shots; s0 += sb.batch) {
        const uint64_t ns = uint64_t(std::min<int64_t>(sb.batch, n_shots - s0));
        const double* du = u + s0;
        uint64_t* dout = out + s0;
        if (host_io) {
            SV_HIP(hipMemcpyAsync(sb.du, u + s0, sizeof(double) * ns, hipMemcpyHostToDevice, stream));
            du = sb.du;
            dout = sb.didx;
        }
        // the first batch also clears the uniforms flag
        const uint64_t nclear = s0 == 0 ? L.nc + 1 : L.nc;
        hipLaunchKernelGGL(k_fill_u32, dim3(unsigned((nclear + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                           stream, sb.counts, nclear);
        SV_HIP(hipGetLastError());
        const int g = guide_bits(ns, L.nc);
        if (g != g_built) {
            const uint64_t ng = (uint64_t(1) << g) + 1;
            hipLaunchKernelGGL(k_chunk_guide, dim3(unsigned((ng + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                               stream, L, sb.B, g, sb.guide);
            SV_HIP(hipGetLastError());
            g_built = g;
        }
        const unsigned sg = unsigned((ns + kThreads - 1) / kThreads);
        hipLaunchKernelGGL(k_shot_chunks, dim3(sg), dim3(kThreads), 0, stream, L, sb.B, sb.guide, g, du, ns, sb.key,
                           sb.rank, sb.counts);
        SV_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(kCountThreads), 0, stream, sb.counts, L.nc, sb.off);
        SV_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_shot_place, dim3(sg), dim3(kThreads), 0, stream, L, sb.B, du, ns, sb.key, sb.rank,
                           sb.off, sb.sorted, sb.rs);
        SV_HIP(hipGetLastError());
        hipLaunchKernelGGL((k_resolve<R>), dim3(sg), dim3(kThreads), 0, stream, psi, L, sb.B, sb.C, sb.sorted, sb.rs,
                           ns, dout);
        SV_HIP(hipGetLastError());
        if (n_bits > 0) {
            hipLaunchKernelGGL(k_extract_bits, dim3(sg), dim3(kThreads), 0, stream, dout, ns, ba);
            SV_HIP(hipGetLastError());
        }
        if (host_io) {
            SV_HIP(hipMemcpyAsync(out + s0, sb.didx, sizeof(uint64_t) * ns, hipMemcpyDeviceToHost, stream));
            SV_HIP(hipStreamSynchronize(stream));
        }
    }
    double total = 0.0;
    uint32_t bad = 0;
    SV_HIP(hipMemcpyAsync(&total, sb.B + L.nc, sizeof(double), hipMemcpyDeviceToHost, stream));
    SV_HIP(hipMemcpyAsync(&bad, sb.counts + L.nc, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
    SV_HIP(hipStreamSynchronize(stream));
    if (!(total > 0.0)) throw Error{SV_ERR_INVALID_VALUE, "state has zero norm"};
    if (bad) throw Error{SV_ERR_INVALID_VALUE, "uniforms must lie in [0, 1)"};
}

// The handle's sampler: block prefixes in the handle's growable scratch,
// everything else in its workspace.
template <typename R>
void run_sample_t(sv_handle_s* h, const void* psi_v, int n, const double* u, int64_t n_shots,
                  const int32_t* bit_ordering, int n_bits, uint64_t* out, bool host_io)
{
    const SampleLayout L = sample_layout(n);
    SampleBuffers sb{};
    sb.C = reinterpret_cast<double*>(ensure_aux(h, sizeof(double) * L.nc * L.nbk));
    const size_t used = kMatRingBytes + sample_fixed_bytes(L.nc);
    if (used >= h->ws_bytes) throw Error{SV_ERR_OUT_OF_MEMORY, "workspace too small for the sampler"};
    const size_t per_shot = kShotBytes + (host_io ? kHostShotBytes : 0);
    int64_t batch = int64_t((h->ws_bytes - used) / per_shot) - int64_t(kCarveAlign);
    if (batch > (int64_t(1) << 22)) batch = int64_t(1) << 22;
    if (batch < 1) throw Error{SV_ERR_OUT_OF_MEMORY, "workspace too small for the sampler"};
    if (used + sample_batch_bytes(batch, host_io) > h->ws_bytes)
        throw Error{SV_ERR_INTERNAL, "sampler workspace layout"};
    carve_sample_buffers(h->ws + kMatRingBytes, L.nc, batch, host_io, sb);
    sample_core<R>(h->stream, h->cu_count, psi_v, n, u, n_shots, bit_ordering, n_bits, out, sb, host_io);
}

// ------------------------------------------- allocation-free sampler scratch
//
// The sampler variant for callers that cannot allocate device memory keeps
// all of its scratch in this fixed array (one copy per GPU, held until the
// process ends): block prefixes for states of up to SV_SAMPLE_NOALLOC_MAX_QUBITS
// qubits, chunk totals and boundaries, and one shot batch.  In host code the
// array's name is not a device address: its address on each device comes
// from hipGetSymbolAddress, looked up once per device and kept.

constexpr size_t kNoAllocPrefixBytes = (size_t(1) << SV_SAMPLE_NOALLOC_MAX_QUBITS) / kBlk * sizeof(double);
constexpr uint64_t kNoAllocMaxChunks = (uint64_t(1) << SV_SAMPLE_NOALLOC_MAX_QUBITS) / (4 * kSub);
constexpr int kMaxScratchDevices = 64;
constexpr int64_t kNoAllocShotBatch = int64_t(1) << 16;
static_assert(kNoAllocPrefixBytes + sample_fixed_bytes(kNoAllocMaxChunks) + sample_batch_bytes(kNoAllocShotBatch, true) <=
                  SV_SAMPLE_NOALLOC_SCRATCH_BYTES,
              "allocation-free sampler scratch too small");

}  // namespace
}  // namespace sv

static __device__ __align__(256) char scratch[SV_SAMPLE_NOALLOC_SCRATCH_BYTES];

namespace sv {
namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of `scratch` on `device` (looked up once, with that
// device current).
char* noalloc_scratch(int device)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    SV_CHECK(device >= 0 && device < kMaxScratchDevices, "device index out of range");
    if (!g_scratch_ptr[device]) {
        int cur = 0;
        SV_HIP(hipGetDevice(&cur));
        if (cur != device) SV_HIP(hipSetDevice(device));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        SV_HIP(e);
        SV_CHECK(p != nullptr, "hipGetSymbolAddress returned no address for the sampler scratch");
        g_scratch_ptr[device] = p;
    }
    return static_cast<char*>(g_scratch_ptr[device]);
}

template <typename R>
void run_sample_noalloc_t(sv_handle_s* h, const void* psi_v, int n, const double* u, int64_t n_shots,
                          const int32_t* bit_ordering, int n_bits, uint64_t* out)
{
    const SampleLayout L = sample_layout(n);
    if (sizeof(double) * L.nc * L.nbk > kNoAllocPrefixBytes || L.nc > kNoAllocMaxChunks)
        throw Error{SV_ERR_INTERNAL, "allocation-free sampler layout"};
    char* w = noalloc_scratch(h->device);
    SampleBuffers sb{};
    sb.C = reinterpret_cast<double*>(w);
    carve_sample_buffers(w + kNoAllocPrefixBytes, L.nc, kNoAllocShotBatch, true, sb);
    sample_core<R>(h->stream, h->cu_count, psi_v, n, u, n_shots, bit_ordering, n_bits, out, sb, true);
}

// --------------------------------------------------------- measurement
//
// Probabilities (Table I: measurement; probability computation and collapse
// as separate steps).  Outcome bins of m measured qubits: bin b holds the
// indices whose bits at the measured qubits spell b.  Its sum runs over the
// 2^(n-m) indices of that bin (the measured bits inserted as b), split into
// a fixed partition of blocks, so every bin's sum has a fixed order; one
// launch covers all bins (grid = bins x blocks per bin).  Z-product parity:
// two accumulators per thread (even, odd) over a fixed partition of the
// whole state.

struct BinArgs {
    uint64_t per;                  // compressed items per block
    uint64_t nbp;                  // blocks per bin
    int32_t m;
    int32_t qpos[SV_MAX_TARGETS];  // measured qubit of outcome bit a
    int32_t qsorted[SV_MAX_TARGETS];
};

__device__ __forceinline__ double block_wave_sum(double v, double* wsum)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const double w = wave_sum(v);
    if (lane == 0) wsum[wave] = w;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kThreads / 64; ++i) s = __dadd_rn(s, wsum[i]);
    __syncthreads();
    return s;
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_bin_probs(const typename Cx<R>::T* __restrict__ psi, BinArgs a,
                                                        double* __restrict__ part)
{
    __shared__ double wsum[kThreads / 64];
    const uint64_t bin = blockIdx.x / a.nbp, blk = blockIdx.x % a.nbp;
    uint64_t obits = 0;
    for (int b = 0; b < a.m; ++b) obits |= ((bin >> b) & 1) << a.qpos[b];
    const uint64_t j0 = blk * a.per;
    double acc = 0.0;
    for (uint64_t j = threadIdx.x; j < a.per; j += kThreads)
        acc = __dadd_rn(acc, prob(psi[insert_bits0(j0 + j, a.qsorted, a.m) | obits]));
    const double s = block_wave_sum(acc, wsum);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Streams a block's items [first, first + per) in rounds of kExpectUnroll
// items per thread, two register buffers in turn (one round's loads in
// flight while the other is summed), calling f(item, amplitude) for each
// item in the order of a plain per-thread loop (it = tid, tid + 256, ...).
// Past the end a round re-reads the block's last amplitude and skips it, so
// every load is unconditional and the compiler waits for the older round
// only.
template <typename T2, typename F>
__device__ __forceinline__ void stream_items(const T2* __restrict__ psi, uint64_t first, uint64_t per, F&& f)
{
    constexpr uint64_t kRound = uint64_t(kExpectUnroll) * kThreads;
    T2 va[kExpectUnroll] = {}, vb[kExpectUnroll] = {};
    auto load = [&](T2 (&v)[kExpectUnroll], uint64_t it0) {
#pragma unroll
        for (int u = 0; u < kExpectUnroll; ++u) {
            const uint64_t it = it0 + uint64_t(u) * kThreads + threadIdx.x;
            v[u] = psi[first + (it < per ? it : per - 1)];
        }
    };
    auto visit = [&](const T2 (&v)[kExpectUnroll], uint64_t it0) {
#pragma unroll
        for (int u = 0; u < kExpectUnroll; ++u) {
            const uint64_t it = it0 + uint64_t(u) * kThreads + threadIdx.x;
            if (it < per) f(first + it, v[u]);
        }
    };
    load(va, 0);
    for (uint64_t it0 = 0; it0 < per; it0 += 2 * kRound) {
        load(vb, it0 + kRound);
        visit(va, it0);
        if (it0 + kRound >= per) break;
        load(va, it0 + 2 * kRound);
        visit(vb, it0 + kRound);
    }
}

// Outcome probabilities of M <= 4 qubits: a fixed partition of the whole
// state, one accumulator per outcome in registers (every item adds to all of
// them, 0 to all but its own: exact), then a fixed block reduction per
// outcome into part[b * gridDim.x + block].
template <typename R, int M>
__global__ __launch_bounds__(kThreads) void k_bin_probs_small(const typename Cx<R>::T* __restrict__ psi, uint64_t per,
                                                              BinArgs a, double* __restrict__ part)
{
    __shared__ double wsum[kThreads / 64];
    double acc[1 << M];
#pragma unroll
    for (int b = 0; b < (1 << M); ++b) acc[b] = 0.0;
    stream_items(psi, uint64_t(blockIdx.x) * per, per, [&](uint64_t i, const typename Cx<R>::T& v) {
        int bin = 0;
#pragma unroll
        for (int q = 0; q < M; ++q) bin |= int((i >> a.qpos[q]) & 1) << q;
        const double p = prob(v);
#pragma unroll
        for (int b = 0; b < (1 << M); ++b) acc[b] = __dadd_rn(acc[b], bin == b ? p : 0.0);
    });
#pragma unroll
    for (int b = 0; b < (1 << M); ++b) {
        const double v = block_wave_sum(acc[b], wsum);
        if (threadIdx.x == 0) part[uint64_t(b) * gridDim.x + blockIdx.x] = v;
    }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_parity_probs(const typename Cx<R>::T* __restrict__ psi, uint64_t per,
                                                           uint64_t mask, double* __restrict__ part)
{
    __shared__ double wsum[kThreads / 64];
    double acc[2] = {0.0, 0.0};
    stream_items(psi, uint64_t(blockIdx.x) * per, per, [&](uint64_t i, const typename Cx<R>::T& v) {
        const int par = __popcll(i & mask) & 1;
        const double p = prob(v);
        acc[0] = __dadd_rn(acc[0], par ? 0.0 : p);
        acc[1] = __dadd_rn(acc[1], par ? p : 0.0);
    });
    const double e = block_wave_sum(acc[0], wsum);
    const double o = block_wave_sum(acc[1], wsum);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = e;
        part[gridDim.x + blockIdx.x] = o;
    }
}

// Collapse: kept amplitudes (bits at the measured qubits == obits, or the
// parity of i & mask == parity when parity >= 0) times scale, all others 0.
// A vector with nothing kept is written without being read.
struct CollapseArgs {
    uint64_t n_vecs;
    uint64_t qmask, obits, mask;
    int32_t parity;
    double scale;
};

constexpr int kColUnits = 8;

template <typename R>
__global__ __launch_bounds__(kThreads) void k_collapse(typename Cx<R>::T* __restrict__ psi, CollapseArgs a)
{
    using T = typename Cx<R>::T;
    constexpr int APV = sizeof(T) == 8 ? 2 : 1;  // amplitudes per 16-byte vector
    using V = typename std::conditional<APV == 2, float4, double2>::type;
    const R sc = R(a.scale);
    const uint64_t v0 = uint64_t(blockIdx.x) * (kThreads * kColUnits) + threadIdx.x;
    V x[kColUnits];
    int keep[kColUnits];  // bit e: amplitude e of the vector is kept
#pragma unroll
    for (int u = 0; u < kColUnits; ++u) {
        const uint64_t v = v0 + uint64_t(u) * kThreads;
        keep[u] = 0;
        if (v >= a.n_vecs) continue;
#pragma unroll
        for (int e = 0; e < APV; ++e) {
            const uint64_t ie = v * APV + e;
            const bool k = a.parity >= 0 ? int(__popcll(ie & a.mask) & 1) == a.parity : (ie & a.qmask) == a.obits;
            keep[u] |= int(k) << e;
        }
        if (keep[u]) x[u] = *reinterpret_cast<const V*>(psi + v * APV);
    }
#pragma unroll
    for (int u = 0; u < kColUnits; ++u) {
        const uint64_t v = v0 + uint64_t(u) * kThreads;
        if (v >= a.n_vecs) continue;
        V y{};
        if (keep[u]) {
            if constexpr (APV == 2) {
                y = float4{(keep[u] & 1) ? x[u].x * sc : 0.f, (keep[u] & 1) ? x[u].y * sc : 0.f,
                           (keep[u] & 2) ? x[u].z * sc : 0.f, (keep[u] & 2) ? x[u].w * sc : 0.f};
            } else {
                y = V{x[u].x * sc, x[u].y * sc};
            }
        }
        *reinterpret_cast<V*>(psi + v * APV) = y;
    }
}

// --------------------------------------------------------- Pauli rotation
//
// psi <- exp(i theta P) psi = cos(theta) psi + i sin(theta) P psi (Table I:
// rotation by a Pauli string), P|k> = i^ny (-1)^popcount(k & z) |k ^ x>.
// x == 0: a phase per amplitude.  x != 0: amplitudes i and j = i ^ x form a
// pair (i has bit h = highest bit of x clear) updated together:
//   new[i] = c psi[i] + i s i^ny (-1)^popcount(j & z) psi[j], and likewise
// for j.  Items run over the control-satisfying pairs (bit h and the
// controls inserted).

struct RotArgs {
    uint64_t items;
    uint64_t x, z, cval;
    int32_t ny;                       // number of Y factors, mod 4
    int32_t n_ins;                    // inserted bits (h if x != 0, then the controls), ascending
    int32_t ins[SV_MAX_QUBITS + 1];
    double c, s;
};

template <typename T, typename R>
__device__ __forceinline__ T mul_i_pow(const T v, int e)
{
    switch (e & 3) {
        case 0: return v;
        case 1: return T{-v.y, v.x};
        case 2: return T{-v.x, -v.y};
        default: return T{v.y, -v.x};
    }
}

// exp(i theta (+-1)) v = (c +- i s) v, the sign from the parity of i & z
template <typename T, typename R>
__device__ __forceinline__ T rot_phase(const T v, uint64_t i, const RotArgs& a, R c, R s)
{
    const R sg = (__popcll(i & a.z) & 1) ? -s : s;
    return T{c * v.x - sg * v.y, c * v.y + sg * v.x};
}

// the pair (i, j = i ^ x): new[i] = c v_i + i^(ny+1) s (-1)^popcount(j & z) v_j, and likewise for j
template <typename T, typename R>
__device__ __forceinline__ void rot_pair(T& vi, T& vj, uint64_t i, uint64_t j, const RotArgs& a, R c, R s)
{
    const R si = (__popcll(j & a.z) & 1) ? -s : s;
    const R sj = (__popcll(i & a.z) & 1) ? -s : s;
    const T pi = mul_i_pow<T, R>(T{si * vj.x, si * vj.y}, a.ny + 1);
    const T pj = mul_i_pow<T, R>(T{sj * vi.x, sj * vi.y}, a.ny + 1);
    vi = T{c * vi.x + pi.x, c * vi.y + pi.y};
    vj = T{c * vj.x + pj.x, c * vj.y + pj.y};
}

// PAIRED (complex64 with bit 0 neither in x nor a control): items 2u and
// 2u + 1 are the neighbours i, i + 1 and their partners j, j + 1, so both
// move as 16-byte vectors.
// One-shot grid: each thread takes kRotUnits units kThreads apart and
// issues all their loads before any arithmetic.
constexpr int kRotUnits = 4;

template <typename R, bool PAIRED>
__global__ __launch_bounds__(kThreads) void k_pauli_rotation(typename Cx<R>::T* __restrict__ psi, RotArgs a)
{
    using T = typename Cx<R>::T;
    using V = typename std::conditional<PAIRED, float4, T>::type;  // one or two amplitudes
    const R c = R(a.c), s = R(a.s);
    const uint64_t units = PAIRED ? a.items / 2 : a.items;
    const uint64_t t0 = uint64_t(blockIdx.x) * (kThreads * kRotUnits) + threadIdx.x;
    uint64_t ii[kRotUnits];
    V vi[kRotUnits], vj[kRotUnits];
#pragma unroll
    for (int u = 0; u < kRotUnits; ++u) {
        const uint64_t t = t0 + uint64_t(u) * kThreads;
        ii[u] = t < units ? (insert_bits0(PAIRED ? 2 * t : t, a.ins, a.n_ins) | a.cval) : ~uint64_t(0);
        if (ii[u] == ~uint64_t(0)) continue;
        vi[u] = *reinterpret_cast<const V*>(psi + ii[u]);
        if (a.x != 0) vj[u] = *reinterpret_cast<const V*>(psi + (ii[u] ^ a.x));
    }
#pragma unroll
    for (int u = 0; u < kRotUnits; ++u) {
        const uint64_t i = ii[u];
        if (i == ~uint64_t(0)) continue;
        if constexpr (PAIRED) {
            T v0{vi[u].x, vi[u].y}, v1{vi[u].z, vi[u].w};
            if (a.x == 0) {
                v0 = rot_phase(v0, i, a, c, s);
                v1 = rot_phase(v1, i + 1, a, c, s);
            } else {
                const uint64_t j = i ^ a.x;
                T u0{vj[u].x, vj[u].y}, u1{vj[u].z, vj[u].w};
                rot_pair(v0, u0, i, j, a, c, s);
                rot_pair(v1, u1, i + 1, j + 1, a, c, s);
                *reinterpret_cast<float4*>(psi + j) = float4{u0.x, u0.y, u1.x, u1.y};
            }
            *reinterpret_cast<float4*>(psi + i) = float4{v0.x, v0.y, v1.x, v1.y};
        } else {
            if (a.x == 0) {
                psi[i] = rot_phase(vi[u], i, a, c, s);
                continue;
            }
            const uint64_t j = i ^ a.x;
            T x = vi[u], y = vj[u];
            rot_pair(x, y, i, j, a, c, s);
            psi[i] = x;
            psi[j] = y;
        }
    }
}

// ------------------------------------------- dense-observable expectation
//
// <psi|M|psi> = sum over groups g of sum_r conj(x_r) (M x)_r, x the group's
// 2^K amplitudes (Table I: expectation with a dense matrix observable).
// One thread per group, M (complex128) in LDS, FP64 arithmetic for both
// precisions, per-thread sums over a fixed partition of the groups; block
// partials of (re, im, norm).

struct ObsArgs {
    uint64_t per;                 // groups per block
    int32_t k;
    uint64_t off[1 << 5];         // group offset of matrix index r
    int32_t tsorted[5];
};

template <typename R, int K>
__global__ __launch_bounds__(kThreads) void k_expect_matrix(const typename Cx<R>::T* __restrict__ psi,
                                                            const double2* __restrict__ mat, ObsArgs a,
                                                            double* __restrict__ part)
{
    constexpr int D = 1 << K;
    __shared__ double2 M[D * D];
    __shared__ double wsum[kThreads / 64];
    for (int e = threadIdx.x; e < D * D; e += kThreads) M[e] = mat[e];
    __syncthreads();
    const uint64_t g0 = uint64_t(blockIdx.x) * a.per;
    double re = 0.0, im = 0.0, nrm = 0.0;
    using T = typename Cx<R>::T;
    // adds group g's conj(x_r) (M x)_r and |x_r|^2 over the rows r
    auto group = [&](const T (&x)[D], uint64_t g) {
        const uint64_t b = insert_bits0(g0 + g, a.tsorted, K);
        // K <= 3: rows and columns unrolled, x_r straight from the
        // registers (a compiler barrier per row keeps M's entries from being
        // hoisted into registers all at once).  K > 3: rows one at a time;
        // x_r is read again (a cache hit), since indexing the register
        // array with a run-time row would put it in scratch memory.
#pragma unroll
        for (int rr = 0; rr < (K <= 3 ? D : 1); ++rr)
#pragma unroll 1
        for (int r2 = 0; r2 < (K <= 3 ? 1 : D); ++r2) {
            const int r = K <= 3 ? rr : r2;
            asm volatile("" ::: "memory");
            double yr = 0.0, yi = 0.0;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                // K <= 3: the row straight from memory (a uniform address:
                // scalar loads, no LDS traffic per group)
                const double2 m = K <= 3 ? mat[r * D + c] : M[r * D + c];
                const double mx = m.x, my = m.y;
                yr = fma(mx, double(x[c].x), fma(-my, double(x[c].y), yr));
                yi = fma(mx, double(x[c].y), fma(my, double(x[c].x), yi));
            }
            const T v = K <= 3 ? x[rr] : psi[b + a.off[r]];
            const double vr = double(v.x), vi = double(v.y);
            // conj(x_r) y
            re = fma(vr, yr, fma(vi, yi, re));
            im = fma(vr, yi, fma(-vi, yr, im));
            nrm = fma(vr, vr, fma(vi, vi, nrm));
        }
    };
    // group g's amplitudes; past the block's end the last group is read
    // again (and not summed), so every load is unconditional
    auto load = [&](T (&x)[D], uint64_t g) {
        const uint64_t b = insert_bits0(g0 + (g < a.per ? g : a.per - 1), a.tsorted, K);
#pragma unroll
        for (int c = 0; c < D; ++c) x[c] = psi[b + a.off[c]];
    };
    if constexpr (K <= 3) {
        // two register buffers in turn: one group's loads in flight while
        // the other is summed (groups in the order of a plain loop)
        T xa[D] = {}, xb[D] = {};
        load(xa, threadIdx.x);
        for (uint64_t g = threadIdx.x; g < a.per; g += 2 * kThreads) {
            load(xb, g + kThreads);
            group(xa, g);
            if (g + kThreads >= a.per) break;
            load(xa, g + 2 * kThreads);
            group(xb, g + kThreads);
        }
    } else {
        for (uint64_t g = threadIdx.x; g < a.per; g += kThreads) {
            T x[D];
            load(x, g);
            group(x, g);
        }
    }
    const double s0 = block_wave_sum(re, wsum);
    const double s1 = block_wave_sum(im, wsum);
    const double s2 = block_wave_sum(nrm, wsum);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = s0;
        part[gridDim.x + blockIdx.x] = s1;
        part[2 * gridDim.x + blockIdx.x] = s2;
    }
}

template <typename R>
void run_bin_probs_t(sv_handle_s* h, const void* psi_v, int n, const int32_t* qubits, int m, double* out)
{
    using T2 = typename Cx<R>::T;
    BinArgs a{};
    a.m = m;
    for (int b = 0; b < m; ++b) a.qpos[b] = a.qsorted[b] = qubits[b];
    std::sort(a.qsorted, a.qsorted + m);
    const uint64_t bins = uint64_t(1) << m;
    if (m <= 4) {
        // few outcomes: per-thread accumulators over one contiguous sweep
        const Partition P = partition(uint64_t(1) << n);
        double* part = reinterpret_cast<double*>(h->ws + kMatRingBytes);
        double* res = part + bins * P.nb;
        const T2* psi = static_cast<const T2*>(psi_v);
        if (m == 1)
            hipLaunchKernelGGL((k_bin_probs_small<R, 1>), dim3(unsigned(P.nb)), dim3(kThreads), 0, h->stream, psi, P.per, a, part);
        else if (m == 2)
            hipLaunchKernelGGL((k_bin_probs_small<R, 2>), dim3(unsigned(P.nb)), dim3(kThreads), 0, h->stream, psi, P.per, a, part);
        else if (m == 3)
            hipLaunchKernelGGL((k_bin_probs_small<R, 3>), dim3(unsigned(P.nb)), dim3(kThreads), 0, h->stream, psi, P.per, a, part);
        else
            hipLaunchKernelGGL((k_bin_probs_small<R, 4>), dim3(unsigned(P.nb)), dim3(kThreads), 0, h->stream, psi, P.per, a, part);
        SV_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_finish_sums, dim3(unsigned(bins)), dim3(kThreads), 0, h->stream, part, P.nb, res);
        SV_HIP(hipGetLastError());
        SV_HIP(hipMemcpyAsync(out, res, sizeof(double) * bins, hipMemcpyDeviceToHost, h->stream));
        SV_HIP(hipStreamSynchronize(h->stream));
        return;
    }
    const uint64_t items = uint64_t(1) << (n - m);
    uint64_t nbp = std::max<uint64_t>(1, std::min<uint64_t>(items / 2048, std::max<uint64_t>(1, 8192 / bins)));
    a.nbp = nbp;
    a.per = items / nbp;
    double* part = reinterpret_cast<double*>(h->ws + kMatRingBytes);
    double* res = part + bins * nbp;
    hipLaunchKernelGGL((k_bin_probs<R>), dim3(unsigned(bins * nbp)), dim3(kThreads), 0, h->stream,
                       static_cast<const T2*>(psi_v), a, part);
    SV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_finish_sums, dim3(unsigned(bins)), dim3(kThreads), 0, h->stream, part, nbp, res);
    SV_HIP(hipGetLastError());
    SV_HIP(hipMemcpyAsync(out, res, sizeof(double) * bins, hipMemcpyDeviceToHost, h->stream));
    SV_HIP(hipStreamSynchronize(h->stream));
}

template <typename R>
void run_parity_probs_t(sv_handle_s* h, const void* psi_v, int n, uint64_t mask, double* out)
{
    using T2 = typename Cx<R>::T;
    const Partition P = partition(uint64_t(1) << n);
    double* part = reinterpret_cast<double*>(h->ws + kMatRingBytes);
    double* res = part + 2 * P.nb;
    hipLaunchKernelGGL((k_parity_probs<R>), dim3(unsigned(P.nb)), dim3(kThreads), 0, h->stream,
                       static_cast<const T2*>(psi_v), P.per, mask, part);
    SV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_finish_sums, dim3(2), dim3(kThreads), 0, h->stream, part, P.nb, res);
    SV_HIP(hipGetLastError());
    SV_HIP(hipMemcpyAsync(out, res, sizeof(double) * 2, hipMemcpyDeviceToHost, h->stream));
    SV_HIP(hipStreamSynchronize(h->stream));
}

template <typename R, int K>
void launch_expect_matrix_k(sv_handle_s* h, const void* psi_v, const double2* mat, const ObsArgs& a, unsigned nb,
                            double* part)
{
    hipLaunchKernelGGL((k_expect_matrix<R, K>), dim3(nb), dim3(kThreads), 0, h->stream,
                       static_cast<const typename Cx<R>::T*>(psi_v), mat, a, part);
}

template <typename R>
void run_expect_matrix_t(sv_handle_s* h, const void* psi_v, int n, const double* m, const int32_t* targets, int k,
                         double* out)
{
    ObsArgs a{};
    a.k = k;
    for (int r = 0; r < (1 << k); ++r) {
        uint64_t o = 0;
        for (int b = 0; b < k; ++b)
            if ((r >> b) & 1) o |= uint64_t(1) << targets[b];
        a.off[r] = o;
    }
    for (int b = 0; b < k; ++b) a.tsorted[b] = targets[b];
    std::sort(a.tsorted, a.tsorted + k);
    const Partition P = partition(uint64_t(1) << (n - k));
    const double2* dm = static_cast<const double2*>(stage_matrix(h, m, sizeof(double2) << (2 * k)));
    double* part = reinterpret_cast<double*>(h->ws + kMatRingBytes);
    double* res = part + 3 * P.nb;
    a.per = P.per;
    const unsigned nb = unsigned(P.nb);
    switch (k) {
        case 1: launch_expect_matrix_k<R, 1>(h, psi_v, dm, a, nb, part); break;
        case 2: launch_expect_matrix_k<R, 2>(h, psi_v, dm, a, nb, part); break;
        case 3: launch_expect_matrix_k<R, 3>(h, psi_v, dm, a, nb, part); break;
        case 4: launch_expect_matrix_k<R, 4>(h, psi_v, dm, a, nb, part); break;
        default: launch_expect_matrix_k<R, 5>(h, psi_v, dm, a, nb, part); break;
    }
    SV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_finish_sums, dim3(3), dim3(kThreads), 0, h->stream, part, P.nb, res);
    SV_HIP(hipGetLastError());
    SV_HIP(hipMemcpyAsync(out, res, sizeof(double) * 3, hipMemcpyDeviceToHost, h->stream));
    SV_HIP(hipStreamSynchronize(h->stream));
}

// -------------------------------------------- index bit swap, accessor
//
// Index bit swap (Table I): the amplitude at i moves to pi(i), pi exchanging
// bits a_p and b_p of every pair (all distinct), for the indices whose mask
// bits hold the mask values.  pi is an involution, so each moved pair (i,
// pi(i)) is swapped once, by the thread of the smaller index; fixed points
// are not touched.

struct SwapArgs {
    uint64_t items;                  // mask-compressed indices
    uint64_t mval;
    int32_t n_pairs;
    int32_t a[SV_MAX_QUBITS / 2], b[SV_MAX_QUBITS / 2];
    int32_t n_mask;
    int32_t msorted[SV_MAX_QUBITS];
};

constexpr int kSwapUnits = 4;

// One-shot grid, kSwapUnits indices per thread kThreads apart, every load
// issued before the stores.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_swap_bits(typename Cx<R>::T* __restrict__ psi, SwapArgs a)
{
    using T = typename Cx<R>::T;
    const uint64_t t0 = uint64_t(blockIdx.x) * (kThreads * kSwapUnits) + threadIdx.x;
    uint64_t ii[kSwapUnits], jj[kSwapUnits];
    T x[kSwapUnits], y[kSwapUnits];
#pragma unroll
    for (int u = 0; u < kSwapUnits; ++u) {
        const uint64_t t = t0 + uint64_t(u) * kThreads;
        ii[u] = jj[u] = 0;
        x[u] = y[u] = T{};
        if (t >= a.items) continue;
        const uint64_t i = insert_bits0(t, a.msorted, a.n_mask) | a.mval;
        uint64_t j = i;
        for (int p = 0; p < a.n_pairs; ++p) {
            const uint64_t d = ((i >> a.a[p]) ^ (i >> a.b[p])) & 1;
            j ^= (d << a.a[p]) | (d << a.b[p]);
        }
        if (j > i) {
            ii[u] = i;
            jj[u] = j;
            x[u] = psi[i];
            y[u] = psi[j];
        }
    }
#pragma unroll
    for (int u = 0; u < kSwapUnits; ++u) {
        if (jj[u] > ii[u]) {
            psi[ii[u]] = y[u];
            psi[jj[u]] = x[u];
        }
    }
}

// Accessor (Table I: copy between host and device while reordering the
// qubits): element k of a chunk is the amplitude whose bit ordering[a] is bit
// a of (first + k) and whose mask bits hold the mask values.  Gather into a
// contiguous device buffer (then one copy to the host), or scatter from one.
struct AccessArgs {
    uint64_t first, count, mval;
    int32_t n_bits;
    int32_t ordering[SV_MAX_QUBITS];
};

__device__ __forceinline__ uint64_t access_index(uint64_t k, const AccessArgs& a)
{
    uint64_t i = a.mval;
    for (int b = 0; b < a.n_bits; ++b) i |= ((k >> b) & 1) << a.ordering[b];
    return i;
}

template <typename R, bool SET>
__global__ __launch_bounds__(kThreads) void k_access(typename Cx<R>::T* __restrict__ psi,
                                                     typename Cx<R>::T* __restrict__ buf, AccessArgs a)
{
    for (uint64_t k = uint64_t(blockIdx.x) * kThreads + threadIdx.x; k < a.count; k += uint64_t(gridDim.x) * kThreads) {
        const uint64_t i = access_index(a.first + k, a);
        if (SET)
            psi[i] = buf[k];
        else
            buf[k] = psi[i];
    }
}

}  // namespace

void launch_set_basis(sv_handle_s* h, sv_dtype_t dt, void* psi, int n, uint64_t x)
{
    const uint64_t dim = uint64_t(1) << n;
    if (dt == SV_C64)
        hipLaunchKernelGGL(k_set_basis<float2>, dim3(grid_for(h, dim)), dim3(kThreads), 0, h->stream,
                           static_cast<float2*>(psi), dim, x);
    else
        hipLaunchKernelGGL(k_set_basis<double2>, dim3(grid_for(h, dim)), dim3(kThreads), 0, h->stream,
                           static_cast<double2*>(psi), dim, x);
    SV_HIP(hipGetLastError());
}

void launch_scale(sv_handle_s* h, sv_dtype_t dt, void* psi, int n, double f)
{
    const uint64_t dim = uint64_t(1) << n;
    if (dt == SV_C64)
        hipLaunchKernelGGL(k_scale<float>, dim3(grid_for(h, dim)), dim3(kThreads), 0, h->stream,
                           static_cast<float2*>(psi), dim, float(f));
    else
        hipLaunchKernelGGL(k_scale<double>, dim3(grid_for(h, dim)), dim3(kThreads), 0, h->stream,
                           static_cast<double2*>(psi), dim, f);
    SV_HIP(hipGetLastError());
}

double run_norm(sv_handle_s* h, sv_dtype_t dt, const void* psi, int n)
{
    return dt == SV_C64 ? run_norm_t<float>(h, psi, n) : run_norm_t<double>(h, psi, n);
}

void run_expect(sv_handle_s* h, sv_dtype_t dt, const void* psi, int n, const PauliMasks* terms, int n_terms,
                double* out)
{
    if (dt == SV_C64)
        run_expect_t<float>(h, psi, n, terms, n_terms, out);
    else
        run_expect_t<double>(h, psi, n, terms, n_terms, out);
}

void run_sample(sv_handle_s* h, sv_dtype_t dt, const void* psi, int n, const double* u, int64_t n_shots,
                const int32_t* bit_ordering, int n_bits, uint64_t* out, bool host_io)
{
    if (dt == SV_C64)
        run_sample_t<float>(h, psi, n, u, n_shots, bit_ordering, n_bits, out, host_io);
    else
        run_sample_t<double>(h, psi, n, u, n_shots, bit_ordering, n_bits, out, host_io);
}

void run_sample_noalloc(sv_handle_s* h, sv_dtype_t dt, const void* psi, int n, const double* u, int64_t n_shots,
                        const int32_t* bit_ordering, int n_bits, uint64_t* out)
{
    if (n > SV_SAMPLE_NOALLOC_MAX_QUBITS)
        throw Error{SV_ERR_INVALID_VALUE, "state too large for sv_sample_noalloc (at most " +
                                              std::to_string(SV_SAMPLE_NOALLOC_MAX_QUBITS) + " qubits)"};
    if (dt == SV_C64)
        run_sample_noalloc_t<float>(h, psi, n, u, n_shots, bit_ordering, n_bits, out);
    else
        run_sample_noalloc_t<double>(h, psi, n, u, n_shots, bit_ordering, n_bits, out);
}


void run_measure_probs(sv_handle_s* h, sv_dtype_t dt, const void* psi, int n, const int32_t* qubits, int m,
                       double* out)
{
    if (dt == SV_C64)
        run_bin_probs_t<float>(h, psi, n, qubits, m, out);
    else
        run_bin_probs_t<double>(h, psi, n, qubits, m, out);
}

void run_parity_probs(sv_handle_s* h, sv_dtype_t dt, const void* psi, int n, uint64_t mask, double* out)
{
    if (dt == SV_C64)
        run_parity_probs_t<float>(h, psi, n, mask, out);
    else
        run_parity_probs_t<double>(h, psi, n, mask, out);
}

void launch_collapse(sv_handle_s* h, sv_dtype_t dt, void* psi, int n, uint64_t qmask, uint64_t obits,
                     uint64_t parity_mask, int parity, double scale)
{
    CollapseArgs a{};
    const uint64_t dim = uint64_t(1) << n;
    a.qmask = qmask;
    a.obits = obits;
    a.mask = parity_mask;
    a.parity = parity;
    a.scale = scale;
    a.n_vecs = dt == SV_C64 ? dim / 2 : dim;
    const uint64_t blocks = (a.n_vecs + kThreads * kColUnits - 1) / (kThreads * kColUnits);
    SV_CHECK(blocks <= 0x7fffffffu, "state too large for one launch");
    if (dt == SV_C64)
        hipLaunchKernelGGL(k_collapse<float>, dim3(unsigned(blocks)), dim3(kThreads), 0, h->stream,
                           static_cast<float2*>(psi), a);
    else
        hipLaunchKernelGGL(k_collapse<double>, dim3(unsigned(blocks)), dim3(kThreads), 0, h->stream,
                           static_cast<double2*>(psi), a);
    SV_HIP(hipGetLastError());
}

void launch_pauli_rotation(sv_handle_s* h, sv_dtype_t dt, void* psi, int n, const PauliMasks& pm, double theta,
                           const int32_t* controls, const int32_t* cvals, int n_controls)
{
    RotArgs a{};
    a.x = pm.x;
    a.z = pm.z;
    a.ny = pm.ny & 3;
    a.c = std::cos(theta);
    a.s = std::sin(theta);
    std::vector<int32_t> ins;
    if (pm.x) ins.push_back(63 - __builtin_clzll(pm.x));
    for (int b = 0; b < n_controls; ++b) {
        ins.push_back(controls[b]);
        if (!cvals || cvals[b]) a.cval |= uint64_t(1) << controls[b];
    }
    std::sort(ins.begin(), ins.end());
    a.n_ins = int(ins.size());
    for (size_t b = 0; b < ins.size(); ++b) a.ins[b] = ins[b];
    a.items = uint64_t(1) << (n - a.n_ins);
    const bool bit0_free = (a.n_ins == 0 || a.ins[0] != 0) && !(pm.x & 1);
    auto blocks = [](uint64_t units) {
        const uint64_t b = (units + kThreads * kRotUnits - 1) / (kThreads * kRotUnits);
        SV_CHECK(b <= 0x7fffffffu, "state too large for one launch");
        return unsigned(b);
    };
    if (dt == SV_C64 && bit0_free)
        hipLaunchKernelGGL((k_pauli_rotation<float, true>), dim3(blocks(a.items / 2)), dim3(kThreads), 0,
                           h->stream, static_cast<float2*>(psi), a);
    else if (dt == SV_C64)
        hipLaunchKernelGGL((k_pauli_rotation<float, false>), dim3(blocks(a.items)), dim3(kThreads), 0,
                           h->stream, static_cast<float2*>(psi), a);
    else
        hipLaunchKernelGGL((k_pauli_rotation<double, false>), dim3(blocks(a.items)), dim3(kThreads), 0,
                           h->stream, static_cast<double2*>(psi), a);
    SV_HIP(hipGetLastError());
}

void run_expect_matrix(sv_handle_s* h, sv_dtype_t dt, const void* psi, int n, const double* m,
                       const int32_t* targets, int k, double* out)
{
    if (dt == SV_C64)
        run_expect_matrix_t<float>(h, psi, n, m, targets, k, out);
    else
        run_expect_matrix_t<double>(h, psi, n, m, targets, k, out);
}


void launch_swap_bits(sv_handle_s* h, sv_dtype_t dt, void* psi, int n, const int32_t* pairs, int n_pairs,
                      const int32_t* mask_bits, const int32_t* mask_values, int n_mask)
{
    SwapArgs a{};
    a.n_pairs = n_pairs;
    for (int p = 0; p < n_pairs; ++p) {
        a.a[p] = pairs[2 * p];
        a.b[p] = pairs[2 * p + 1];
    }
    a.n_mask = n_mask;
    for (int m = 0; m < n_mask; ++m) {
        a.msorted[m] = mask_bits[m];
        if (mask_values[m]) a.mval |= uint64_t(1) << mask_bits[m];
    }
    std::sort(a.msorted, a.msorted + n_mask);
    a.items = uint64_t(1) << (n - n_mask);
    const uint64_t blocks = (a.items + kThreads * kSwapUnits - 1) / (kThreads * kSwapUnits);
    SV_CHECK(blocks <= 0x7fffffffu, "state too large for one launch");
    if (dt == SV_C64)
        hipLaunchKernelGGL(k_swap_bits<float>, dim3(unsigned(blocks)), dim3(kThreads), 0, h->stream,
                           static_cast<float2*>(psi), a);
    else
        hipLaunchKernelGGL(k_swap_bits<double>, dim3(unsigned(blocks)), dim3(kThreads), 0, h->stream,
                           static_cast<double2*>(psi), a);
    SV_HIP(hipGetLastError());
}

namespace {

// memcpy on up to 8 host threads for large copies (the caller's pages are
// often touched for the first time here, and page faults then dominate a
// single-threaded copy).
void host_copy(char* dst, const char* src, size_t bytes)
{
    constexpr size_t kPart = size_t(4) << 20;
    unsigned nt = std::min(8u, std::max(1u, std::thread::hardware_concurrency()));
    nt = unsigned(std::min<size_t>(nt, bytes / kPart));
    if (nt < 2) {
        std::memcpy(dst, src, bytes);
        return;
    }
    const size_t per = ((bytes + nt - 1) / nt + 4095) & ~size_t(4095);
    std::vector<std::thread> th;
    th.reserve(nt);
    for (unsigned t = 0; t < nt; ++t) {
        const size_t lo = std::min(bytes, size_t(t) * per), hi = std::min(bytes, lo + per);
        if (hi > lo) th.emplace_back([=] { std::memcpy(dst + lo, src + lo, hi - lo); });
    }
    for (auto& x : th) x.join();
}

template <typename R>
void launch_access(sv_handle_s* h, void* psi, char* stage, const AccessArgs& a, bool set)
{
    using T2 = typename Cx<R>::T;
    if (set)
        hipLaunchKernelGGL((k_access<R, true>), dim3(grid_for(h, a.count)), dim3(kThreads), 0, h->stream,
                           static_cast<T2*>(psi), reinterpret_cast<T2*>(stage), a);
    else
        hipLaunchKernelGGL((k_access<R, false>), dim3(grid_for(h, a.count)), dim3(kThreads), 0, h->stream,
                           static_cast<T2*>(psi), reinterpret_cast<T2*>(stage), a);
    SV_HIP(hipGetLastError());
}

}  // namespace

// The accessor moves its elements in chunks through two device staging
// regions of the workspace and two pinned host buffers of the handle, so
// that the device gathers (or scatters) one chunk and the host link carries
// it while host threads copy the previous chunk to (or from) the caller's
// memory.
void run_accessor(sv_handle_s* h, sv_dtype_t dt, void* psi, int n, const int32_t* ordering, int n_bits,
                  const int32_t* mask_bits, const int32_t* mask_values, int n_mask, void* host, int64_t begin,
                  int64_t end, bool set)
{
    (void)n;
    AccessArgs a{};
    a.n_bits = n_bits;
    for (int b = 0; b < n_bits; ++b) a.ordering[b] = ordering[b];
    for (int m = 0; m < n_mask; ++m)
        if (mask_values[m]) a.mval |= uint64_t(1) << mask_bits[m];
    const size_t amp = dt == SV_C64 ? 8 : 16;
    const size_t avail = h->ws_bytes - kMatRingBytes;
    const uint64_t chunk = std::min<size_t>(avail / 2, size_t(16) << 20) / amp;
    const size_t stage_bytes = chunk * amp;
    if (h->acc_pinned_bytes < 2 * stage_bytes) {
        if (h->acc_pinned) SV_HIP(hipHostFree(h->acc_pinned));
        h->acc_pinned = nullptr;
        h->acc_pinned_bytes = 0;
        SV_HIP(hipHostMalloc(reinterpret_cast<void**>(&h->acc_pinned), 2 * stage_bytes, hipHostMallocDefault));
        h->acc_pinned_bytes = 2 * stage_bytes;
    }
    for (hipEvent_t& ev : h->acc_event)
        if (!ev) SV_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    char* dstage[2] = {h->ws + kMatRingBytes, h->ws + kMatRingBytes + stage_bytes};
    char* hstage[2] = {h->acc_pinned, h->acc_pinned + stage_bytes};
    char* hb = static_cast<char*>(host);
    const uint64_t total = uint64_t(end - begin);
    const uint64_t n_chunks = (total + chunk - 1) / chunk;
    auto args_of = [&](uint64_t i) {
        AccessArgs c = a;
        c.first = uint64_t(begin) + i * chunk;
        c.count = std::min<uint64_t>(chunk, total - i * chunk);
        return c;
    };
    auto launch = [&](char* stage, const AccessArgs& c) {
        if (dt == SV_C64)
            launch_access<float>(h, psi, stage, c, set);
        else
            launch_access<double>(h, psi, stage, c, set);
    };
    if (!set) {
        // chunk i: gather into dstage, copy to hstage, event; the host copies
        // chunk i out of hstage while chunk i + 1 is on the device
        auto issue = [&](uint64_t i) {
            const int sl = int(i & 1);
            const AccessArgs c = args_of(i);
            launch(dstage[sl], c);
            SV_HIP(hipMemcpyAsync(hstage[sl], dstage[sl], c.count * amp, hipMemcpyDeviceToHost, h->stream));
            SV_HIP(hipEventRecord(h->acc_event[sl], h->stream));
        };
        for (uint64_t i = 0; i < std::min<uint64_t>(2, n_chunks); ++i) issue(i);
        for (uint64_t i = 0; i < n_chunks; ++i) {
            const int sl = int(i & 1);
            SV_HIP(hipEventSynchronize(h->acc_event[sl]));
            const AccessArgs c = args_of(i);
            host_copy(hb + i * chunk * amp, hstage[sl], c.count * amp);
            if (i + 2 < n_chunks) issue(i + 2);
        }
    } else {
        // chunk i: the host fills hstage (once its previous copy to the
        // device is done), then copy to dstage, event, scatter
        for (uint64_t i = 0; i < n_chunks; ++i) {
            const int sl = int(i & 1);
            if (i >= 2) SV_HIP(hipEventSynchronize(h->acc_event[sl]));
            const AccessArgs c = args_of(i);
            host_copy(hstage[sl], hb + i * chunk * amp, c.count * amp);
            SV_HIP(hipMemcpyAsync(dstage[sl], hstage[sl], c.count * amp, hipMemcpyHostToDevice, h->stream));
            SV_HIP(hipEventRecord(h->acc_event[sl], h->stream));
            launch(dstage[sl], c);
        }
    }
    SV_HIP(hipStreamSynchronize(h->stream));
}

}  // namespace sv
