// Read-only sweeps over the state: norm, Pauli-string expectations and the
// sampler (Table I: expectation, sampler; Sec. II: outcomes from the
// numerically computed probability distribution, without collapse), plus the
// two write sweeps set-basis and scale.
//
// Every reduction accumulates in FP64 in an order that depends only on n
// (never on the grid size or on other work on the device): a fixed partition
// into blocks, a fixed per-thread order inside a block, a fixed LDS tree, and
// a fixed final pass.  Results are therefore bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
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
constexpr int kExpectUnroll = 4;  // items loaded ahead per thread

struct ExpectArgs {
    uint64_t per;        // items per block
    uint64_t x;          // common X/Y mask of the terms
    int32_t hbit;        // highest bit of x (pair sweeps)
    int32_t n_terms;
    uint64_t z[kMaxTermsPerSweep];
    int32_t ny[kMaxTermsPerSweep];
};

// Per block: FP64 partials of every term and of the norm, written to
// part[t * nb + block] (t = n_terms is the norm).
//
// x == 0: item i contributes |psi_i|^2 * (-1)^popcount(i & z).
// x != 0: item q is the pair (i, j = i ^ x) with bit hbit of i clear; with
//         w = conj(psi_j) psi_i the pair contributes
//         2 Re(w * i^ny) * (-1)^popcount(i & z), because P|i> = ph(i)|j> and
//         ph(j) = conj(ph(i)) for a Hermitian Pauli string.
template <typename R, bool kPairs>
__global__ __launch_bounds__(kThreads) void k_expect(const typename Cx<R>::T* __restrict__ psi,
                                                    ExpectArgs a, double* __restrict__ part)
{
    __shared__ double lds[kThreads];
    double acc[kMaxTermsPerSweep + 1];
#pragma unroll
    for (int t = 0; t <= kMaxTermsPerSweep; ++t) acc[t] = 0.0;
    const uint64_t first = uint64_t(blockIdx.x) * a.per;
    // index bits that change across one thread's items (x == 0 sweeps)
    const uint64_t vary = (a.per - 1) & ~uint64_t(kThreads - 1);
    using T2 = typename Cx<R>::T;
    // items it0 + u * kThreads + tid, u < kExpectUnroll: all loads of a
    // round are issued before any arithmetic, so each thread keeps several
    // HBM requests in flight
    for (uint64_t it0 = 0; it0 < a.per; it0 += uint64_t(kExpectUnroll) * kThreads) {
        T2 vi[kExpectUnroll] = {}, vj[kExpectUnroll] = {};
        uint64_t ii[kExpectUnroll] = {};
#pragma unroll
        for (int u = 0; u < kExpectUnroll; ++u) {
            const uint64_t it = it0 + uint64_t(u) * kThreads + threadIdx.x;
            const uint64_t q = first + it;
            if (!kPairs) {
                if (it < a.per) vi[u] = psi[q];
            } else {
                const uint64_t lo = q & ((uint64_t(1) << a.hbit) - 1);
                ii[u] = ((q >> a.hbit) << (a.hbit + 1)) | lo;
                if (it < a.per) {
                    vi[u] = psi[ii[u]];
                    vj[u] = psi[ii[u] ^ a.x];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kExpectUnroll; ++u) {
            const uint64_t it = it0 + uint64_t(u) * kThreads + threadIdx.x;
            if (it >= a.per) continue;
            if (!kPairs) {
                // q = first | tid | (it - tid): only the bits of `it` above
                // the thread index vary inside the loop.  A term whose Z
                // mask misses them has a constant sign per thread and shares
                // the plain sum (the norm slot); the others flip with
                // parity(it & vary & z).
                const double p = prob(vi[u]);
                acc[kMaxTermsPerSweep] = __dadd_rn(acc[kMaxTermsPerSweep], p);
#pragma unroll
                for (int t = 0; t < kMaxTermsPerSweep; ++t) {
                    if (t < a.n_terms && (a.z[t] & vary) != 0) {
                        const double sg = (__popcll(it & vary & a.z[t]) & 1) ? -p : p;
                        acc[t] = __dadd_rn(acc[t], sg);
                    }
                }
            } else {
                const T2 ai = vi[u], aj = vj[u];
                const double ir = double(ai.x), im = double(ai.y), jr = double(aj.x), jm = double(aj.y);
                // w = conj(a_j) * a_i
                const double wr = fma(jr, ir, __dmul_rn(jm, im));
                const double wi = fma(jr, im, -__dmul_rn(jm, ir));
                acc[kMaxTermsPerSweep] = __dadd_rn(acc[kMaxTermsPerSweep], __dadd_rn(prob(ai), prob(aj)));
#pragma unroll
                for (int t = 0; t < kMaxTermsPerSweep; ++t) {
                    if (t < a.n_terms) {
                        const int m = a.ny[t] & 3;
                        double v = (m == 0) ? wr : (m == 1) ? -wi : (m == 2) ? -wr : wi;
                        v = 2.0 * v;
                        if (__popcll(ii[u] & a.z[t]) & 1) v = -v;
                        acc[t] = __dadd_rn(acc[t], v);
                    }
                }
            }
        }
    }
    if (!kPairs) {
        // apply the per-thread constant signs: a term that misses the
        // varying bits takes the plain sum with the sign of
        // parity((first | tid) & z); a term that hits them accumulated the
        // varying part of its sign, and the constant part flips the total
        const uint64_t fixed = first | threadIdx.x;
#pragma unroll
        for (int t = 0; t < kMaxTermsPerSweep; ++t) {
            if (t < a.n_terms) {
                const bool neg = (__popcll(fixed & a.z[t]) & 1) != 0;
                const double v = ((a.z[t] & vary) != 0) ? acc[t] : acc[kMaxTermsPerSweep];
                acc[t] = neg ? -v : v;
            }
        }
    }
#pragma unroll
    for (int t = 0; t <= kMaxTermsPerSweep; ++t) {
        if (t < a.n_terms || t == kMaxTermsPerSweep) {
            const double s = block_sum(acc[t], lds);
            const int slot = (t == kMaxTermsPerSweep) ? a.n_terms : t;
            if (threadIdx.x == 0) part[uint64_t(slot) * gridDim.x + blockIdx.x] = s;
        }
    }
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
    __shared__ double p[(kSub / kBlk) * kRow];
    const int tid = threadIdx.x, lane = tid & 63;
    const uint64_t sub_len = L.cs < kSub ? L.cs : kSub;
    const uint64_t nsub = L.cs / sub_len;
    const int rows = int(sub_len / uint64_t(L.w));
    const int wshift = __ffs(L.w) - 1;
    for (uint64_t c = blockIdx.x; c < L.nc; c += gridDim.x) {
        double carry = 0.0;
        for (uint64_t sb = 0; sb < nsub; ++sb) {
            const T2* src = psi + c * L.cs + sb * sub_len;
            if (sub_len == kSub) {
                constexpr int kPer = int(kSub) / kThreads;
                T2 v[kPer];
#pragma unroll
                for (int u = 0; u < kPer; ++u) v[u] = src[u * kThreads + tid];
#pragma unroll
                for (int u = 0; u < kPer; ++u) {
                    const int i = u * kThreads + tid;
                    p[(i >> wshift) * kRow + (i & (L.w - 1))] = prob(v[u]);
                }
            } else {
                for (int i = tid; i < int(sub_len); i += kThreads)
                    p[(i >> wshift) * kRow + (i & (L.w - 1))] = prob(src[i]);
            }
            __syncthreads();
            if (tid < 64) {
                double sum = 0.0;
                if (lane < rows)
                    for (int j = 0; j < L.w; ++j) sum = __dadd_rn(sum, p[lane * kRow + j]);
                double mine = 0.0;
                for (int l = 0; l < rows; ++l) {
                    carry = __dadd_rn(carry, readlane_f64(sum, l));
                    if (lane == l) mine = carry;
                }
                if (lane < rows) C[c * L.nbk + sb * uint64_t(rows) + lane] = mine;
            }
            __syncthreads();
        }
        if (tid == 0) S[c] = carry;
    }
}

constexpr int kScanThreads = 1024;

// B[0..nc] from S[0..nc-1] (single block).
__global__ __launch_bounds__(kScanThreads) void k_scan_chunks(const double* __restrict__ S, uint64_t nc,
                                                             double* __restrict__ B)
{
    __shared__ double tot[kScanThreads];
    __shared__ double off[kScanThreads];
    const uint64_t per = (nc + kScanThreads - 1) / kScanThreads;
    const uint64_t lo = std::min<uint64_t>(nc, threadIdx.x * per);
    const uint64_t hi = std::min<uint64_t>(nc, lo + per);
    double run = 0.0;
    for (uint64_t c = lo; c < hi; ++c) {
        run = __dadd_rn(run, S[c]);
        B[c + 1] = run;  // local inclusive prefix for now
    }
    tot[threadIdx.x] = run;
    __syncthreads();
    if (threadIdx.x == 0) {
        double o = 0.0;
        for (int t = 0; t < kScanThreads; ++t) {
            off[t] = o;
            o = __dadd_rn(o, tot[t]);
        }
    }
    __syncthreads();
    const double o = off[threadIdx.x];
    for (uint64_t c = lo; c < hi; ++c) B[c + 1] = __dadd_rn(o, B[c + 1]);
    if (threadIdx.x == 0) B[0] = 0.0;
}

__device__ __forceinline__ double shot_r(double u, double total)
{
    double r = __dmul_rn(u, total);
    if (!(r < total)) r = nextafter(total, 0.0);
    return r;
}

// One thread per shot: chunk by binary search over B, block by binary search
// over the chunk's C, then the block's amplitudes in order.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_resolve(const typename Cx<R>::T* __restrict__ psi,
                                                     SampleLayout L, const double* __restrict__ B,
                                                     const double* __restrict__ C,
                                                     const double* __restrict__ u, uint64_t ns,
                                                     uint64_t* __restrict__ idx_out)
{
    using T2 = typename Cx<R>::T;
    const uint64_t s = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= ns) return;
    const double r = shot_r(u[s], B[L.nc]);
    uint64_t lo = 0, hi = L.nc - 1;  // smallest c with r < B[c+1]
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (r < B[mid + 1])
            hi = mid;
        else
            lo = mid + 1;
    }
    const uint64_t c = lo;
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
        for (uint64_t i = L.cs; i-- > 0;) {
            if (prob(chunk[i]) > 0.0) {
                found = c * L.cs + i;
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
    hipLaunchKernelGGL((k_expect<R, false>), dim3(unsigned(P.nb)), dim3(kThreads), 0, h->stream, psi, a, part);
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
    // group terms by their X/Y mask: one sweep per distinct mask and per
    // kMaxTermsPerSweep terms
    std::vector<int> order(n_terms);
    for (int t = 0; t < n_terms; ++t) order[t] = t;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return terms[a].x < terms[b].x; });
    double* part = reinterpret_cast<double*>(h->ws + kMatRingBytes);
    std::vector<double> sums(n_terms, 0.0);
    double norm = -1.0;
    std::vector<std::pair<int, int>> launches;  // (first index into order, count)
    for (int i = 0; i < n_terms;) {
        int j = i;
        while (j < n_terms && terms[order[j]].x == terms[order[i]].x && j - i < kMaxTermsPerSweep) ++j;
        launches.push_back({i, j - i});
        i = j;
    }
    double* res_dev = part;  // reused per launch after the partials are consumed
    for (auto& L : launches) {
        const uint64_t x = terms[order[L.first]].x;
        const bool pairs = x != 0;
        const uint64_t items = pairs ? dim / 2 : dim;
        const Partition P = partition(items);
        double* p = part + 64;  // first 64 doubles hold the finished sums
        ExpectArgs a{};
        a.per = P.per;
        a.x = x;
        a.hbit = pairs ? highest_bit(x) : 0;
        a.n_terms = L.second;
        for (int t = 0; t < L.second; ++t) {
            a.z[t] = terms[order[L.first + t]].z;
            a.ny[t] = terms[order[L.first + t]].ny;
        }
        if (pairs)
            hipLaunchKernelGGL((k_expect<R, true>), dim3(unsigned(P.nb)), dim3(kThreads), 0, h->stream, psi, a, p);
        else
            hipLaunchKernelGGL((k_expect<R, false>), dim3(unsigned(P.nb)), dim3(kThreads), 0, h->stream, psi, a, p);
        SV_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_finish_sums, dim3(unsigned(L.second + 1)), dim3(kThreads), 0, h->stream, p, P.nb,
                           res_dev);
        SV_HIP(hipGetLastError());
        double host[kMaxTermsPerSweep + 1];
        SV_HIP(hipMemcpyAsync(host, res_dev, sizeof(double) * (L.second + 1), hipMemcpyDeviceToHost, h->stream));
        SV_HIP(hipStreamSynchronize(h->stream));
        for (int t = 0; t < L.second; ++t) sums[order[L.first + t]] = host[t];
        if (norm < 0.0) norm = host[L.second];
    }
    if (!(norm > 0.0)) throw Error{SV_ERR_INVALID_VALUE, "state has zero norm"};
    for (int t = 0; t < n_terms; ++t) out[t] = sums[t] / norm;
}

template <typename R>
void run_sample_t(sv_handle_s* h, const void* psi_v, int n, const double* u, int64_t n_shots,
                  const int32_t* bit_ordering, int n_bits, uint64_t* out)
{
    using T2 = typename Cx<R>::T;
    const T2* psi = static_cast<const T2*>(psi_v);
    const SampleLayout L = sample_layout(n);
    double* C = reinterpret_cast<double*>(ensure_aux(h, sizeof(double) * L.nc * L.nbk));
    char* w = h->ws + kMatRingBytes;
    auto take = [&](size_t bytes) {
        char* p = w;
        w += (bytes + 255) & ~size_t(255);
        return p;
    };
    double* S = reinterpret_cast<double*>(take(sizeof(double) * L.nc));
    double* B = reinterpret_cast<double*>(take(sizeof(double) * (L.nc + 1)));
    const size_t used = size_t(w - h->ws);
    if (used >= h->ws_bytes) throw Error{SV_ERR_OUT_OF_MEMORY, "workspace too small for the sampler"};
    const size_t per_shot = sizeof(double) + sizeof(uint64_t);
    int64_t batch = int64_t((h->ws_bytes - used) / per_shot) - 1024;
    if (batch > (int64_t(1) << 22)) batch = int64_t(1) << 22;
    if (batch < 1) throw Error{SV_ERR_OUT_OF_MEMORY, "workspace too small for the sampler"};
    double* du = reinterpret_cast<double*>(take(sizeof(double) * batch));
    uint64_t* didx = reinterpret_cast<uint64_t*>(take(sizeof(uint64_t) * batch));
    if (size_t(w - h->ws) > h->ws_bytes) throw Error{SV_ERR_INTERNAL, "sampler workspace layout"};

    hipLaunchKernelGGL((k_block_prefix<R>), dim3(unsigned(std::min<uint64_t>(L.nc, uint64_t(h->cu_count) * 8))),
                       dim3(kThreads), 0, h->stream, psi, L, C, S);
    SV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_scan_chunks, dim3(1), dim3(kScanThreads), 0, h->stream, S, L.nc, B);
    SV_HIP(hipGetLastError());
    double total = 0.0;
    SV_HIP(hipMemcpyAsync(&total, B + L.nc, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    SV_HIP(hipStreamSynchronize(h->stream));
    if (!(total > 0.0)) throw Error{SV_ERR_INVALID_VALUE, "state has zero norm"};

    BitArgs ba{};
    ba.n_bits = n_bits;
    for (int b = 0; b < n_bits; ++b) ba.bits[b] = bit_ordering[b];
    for (int64_t s0 = 0; s0 < n_shots; s0 += batch) {
        const uint64_t ns = uint64_t(std::min<int64_t>(batch, n_shots - s0));
        SV_HIP(hipMemcpyAsync(du, u + s0, sizeof(double) * ns, hipMemcpyHostToDevice, h->stream));
        const unsigned sg = unsigned((ns + kThreads - 1) / kThreads);
        hipLaunchKernelGGL((k_resolve<R>), dim3(sg), dim3(kThreads), 0, h->stream, psi, L, B, C, du, ns, didx);
        SV_HIP(hipGetLastError());
        if (n_bits > 0) {
            hipLaunchKernelGGL(k_extract_bits, dim3(sg), dim3(kThreads), 0, h->stream, didx, ns, ba);
            SV_HIP(hipGetLastError());
        }
        SV_HIP(hipMemcpyAsync(out + s0, didx, sizeof(uint64_t) * ns, hipMemcpyDeviceToHost, h->stream));
        SV_HIP(hipStreamSynchronize(h->stream));
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
                const int32_t* bit_ordering, int n_bits, uint64_t* out)
{
    if (dt == SV_C64)
        run_sample_t<float>(h, psi, n, u, n_shots, bit_ordering, n_bits, out);
    else
        run_sample_t<double>(h, psi, n, u, n_shots, bit_ordering, n_bits, out);
}

}  // namespace sv
