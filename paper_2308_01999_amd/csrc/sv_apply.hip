// Dense k-qubit gate sweeps on gfx950 (Table I: gate application with a dense
// matrix; Sec. II-B: the dominant, memory-bound operation).
//
// The state is one contiguous vector of interleaved complex amplitudes.  A
// sweep visits 2^(n-k-c) groups; group g owns the 2^k amplitudes whose index
// is g with zero bits inserted at the (sorted) target and control positions,
// the control bits then set to their values, plus off(r) = sum of the target
// bits set in r.  Each group is read once and written once, so the sweep
// moves 2 * 2^(n-c) amplitudes through HBM: the kernel is bandwidth-bound up
// to k = 5 on MI355X and its job is to keep the loads wide and coalesced.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "sv_tile.h"

namespace sv {
namespace {

using namespace tile;

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

constexpr int kMaxUnrolledK = 6;

struct ApplyArgs {
    uint64_t n_groups;
    uint64_t cval;
    int32_t n_fixed;
    int32_t fixed[SV_MAX_QUBITS];
    uint64_t off[1 << kMaxUnrolledK];
};

__device__ __forceinline__ uint64_t group_base(uint64_t g, const ApplyArgs& a)
{
    uint64_t base = g;
    for (int j = 0; j < a.n_fixed; ++j) {
        const int p = a.fixed[j];
        const uint64_t lo = base & ((uint64_t(1) << p) - 1);
        base = ((base >> p) << (p + 1)) | lo;
    }
    return base | a.cval;
}

// One group per thread (no grid-stride loop: a loop would let the compiler
// hoist the whole matrix into scalar registers and spill them).  Consecutive lanes take consecutive
// groups, so when no target sits in the low index bits each of the 2^k loads
// of a wave covers 64 consecutive amplitudes (512 B for complex64, 1 KiB for
// complex128).  The matrix index is compile-time after unrolling and the
// matrix pointer is uniform, so its entries come in through scalar loads and
// feed the FMAs as scalar operands.  All 2^k inputs are in registers before
// the first store, which makes the in-place update safe.
template <typename R, int K>
__global__ __launch_bounds__(256) void k_apply_dense(typename Cx<R>::T* __restrict__ psi,
                                                     const typename Cx<R>::T* __restrict__ mat,
                                                     ApplyArgs a)
{
    using T2 = typename Cx<R>::T;
    constexpr int D = 1 << K;
    const uint64_t blk = uint64_t(blockIdx.y) * gridDim.x + blockIdx.x;
    const uint64_t g = blk * blockDim.x + threadIdx.x;
    if (g >= a.n_groups) return;
    const uint64_t base = group_base(g, a);
    T2 v[D];
#pragma unroll
    for (int c = 0; c < D; ++c) v[c] = psi[base + a.off[c]];
#pragma unroll
    for (int r = 0; r < D; ++r) {
        R re = 0, im = 0;
#pragma unroll
        for (int c = 0; c < D; ++c) {
            const T2 m = mat[r * D + c];
            re = fma(m.x, v[c].x, re);
            re = fma(-m.y, v[c].y, re);
            im = fma(m.x, v[c].y, im);
            im = fma(m.y, v[c].x, im);
        }
        psi[base + a.off[r]] = T2{re, im};
    }
}

// ------------------------------------------------------------------ MFMA
//
// For complex64 with k = 4, 5 and complex128 with k = 5, the update of many
// groups at once is the complex GEMM Y = M X, with one group per column of X.
// It runs on the matrix cores as three real GEMMs (Gauss's product: three
// real products per complex product instead of four):
//     P1 = Re M Re X,  P2 = Im M Im X,  P3 = (Re M + Im M)(Re X + Im X),
//     Re Y = P1 - P2,  Im Y = P3 - P1 - P2.
// The host packs the three real matrices A_0 = Re M, A_1 = Im M,
// A_2 = Re M + Im M in the order each lane consumes its A-operand slices, so
// a lane loads its slice with a few 16-byte loads (pack_matrix below).
//
// Lane layouts (measured on gfx950):
//   v_mfma_f32_32x32x2_f32: A[i][k] lane i + 32k; B[k][j] lane j + 32k;
//     D[i][j] lane j + 32((i/4)%2), register 4(i/8) + i%4.
//   v_mfma_f32_16x16x4_f32: A[i][k] lane i + 16k; B[k][j] lane j + 16k;
//     D[i][j] lane j + 16(i/4), register i%4.
//   v_mfma_f64_16x16x4_f64: A[i][k] lane i + 16k; B[k][j] lane j + 16k;
//     D[i][j] lane j + 16(i%4), register i/4.

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// c64, k = 5: 16 floats of each A_g per lane (k index 2j + half)
__device__ __forceinline__ void load_a_c64k5(const float4* __restrict__ m4, int lane, float* ar, float* ai,
                                             float* as)
{
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        float4 v = m4[(0 * 64 + lane) * 4 + q];
        ar[4 * q] = v.x; ar[4 * q + 1] = v.y; ar[4 * q + 2] = v.z; ar[4 * q + 3] = v.w;
        v = m4[(1 * 64 + lane) * 4 + q];
        ai[4 * q] = v.x; ai[4 * q + 1] = v.y; ai[4 * q + 2] = v.z; ai[4 * q + 3] = v.w;
        v = m4[(2 * 64 + lane) * 4 + q];
        as[4 * q] = v.x; as[4 * q + 1] = v.y; as[4 * q + 2] = v.z; as[4 * q + 3] = v.w;
    }
}

// c64, k = 4: 4 floats of each A_g per lane (k index 4s + q)
__device__ __forceinline__ void load_a_c64k4(const float4* __restrict__ m4, int lane, float* ar, float* ai,
                                             float* as)
{
    float4 v = m4[0 * 64 + lane];
    ar[0] = v.x; ar[1] = v.y; ar[2] = v.z; ar[3] = v.w;
    v = m4[1 * 64 + lane];
    ai[0] = v.x; ai[1] = v.y; ai[2] = v.z; ai[3] = v.w;
    v = m4[2 * 64 + lane];
    as[0] = v.x; as[1] = v.y; as[2] = v.z; as[3] = v.w;
}

__device__ __forceinline__ void mfma_c64k5(const float* ar, const float* ai, const float* as, const float2* x,
                                           f32x16& p1, f32x16& p2, f32x16& p3)
{
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        p1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[j], x[j].x, p1, 0, 0, 0);
        p2 = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[j], x[j].y, p2, 0, 0, 0);
        p3 = __builtin_amdgcn_mfma_f32_32x32x2f32(as[j], x[j].x + x[j].y, p3, 0, 0, 0);
    }
}

__device__ __forceinline__ void mfma_c64k4(const float* ar, const float* ai, const float* as, const float2* x,
                                           f32x4& p1, f32x4& p2, f32x4& p3)
{
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
        p1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[s4], x[s4].x, p1, 0, 0, 0);
        p2 = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[s4], x[s4].y, p2, 0, 0, 0);
        p3 = __builtin_amdgcn_mfma_f32_16x16x4f32(as[s4], x[s4].x + x[s4].y, p3, 0, 0, 0);
    }
}

// Direct MFMA kernels: used when the LDS-tiled kernels below do not apply
// (gates with controls, states of fewer than 12 qubits).  One wave takes 32
// (k = 5) or 16 (k = 4) consecutive groups per step of a grid-stride loop;
// the A operands stay in registers for the whole kernel.
__global__ __launch_bounds__(256) void k_apply_mfma_c64_k5(float2* __restrict__ psi,
                                                          const float4* __restrict__ mats, ApplyArgs a,
                                                          uint64_t n_tiles)
{
    const int lane = threadIdx.x & 63;
    const int col = lane & 31;
    const int half = lane >> 5;
    float ar[16], ai[16], as[16];
    load_a_c64k5(mats, lane, ar, ai, as);
    // The lane loads matrix index 2j + half and stores row 8(r/4) + 4 half +
    // r%4: the lane-dependent part is bit 0 (loads) or bit 2 (stores) of the
    // matrix index, i.e. target 0 or target 2; the rest of each offset is
    // uniform across the wave.
    const uint64_t lane_in = half ? a.off[1] : 0;
    const uint64_t lane_out = half ? a.off[4] : 0;
    const uint64_t n_waves = uint64_t(gridDim.x) * (blockDim.x >> 6);
    for (uint64_t t = uint64_t(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6); t < n_tiles; t += n_waves) {
        const uint64_t g = t * 32 + col;
        const bool valid = g < a.n_groups;
        const uint64_t base = valid ? group_base(g, a) : 0;
        float2 x[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) x[j] = valid ? psi[base + lane_in + a.off[2 * j]] : float2{0.f, 0.f};
        f32x16 p1 = {0}, p2 = {0}, p3 = {0};
        mfma_c64k5(ar, ai, as, x, p1, p2, p3);
        if (valid) {
#pragma unroll
            for (int r = 0; r < 16; ++r)
                psi[base + lane_out + a.off[8 * (r / 4) + (r % 4)]] = float2{p1[r] - p2[r], p3[r] - p1[r] - p2[r]};
        }
    }
}

__global__ __launch_bounds__(256) void k_apply_mfma_c64_k4(float2* __restrict__ psi,
                                                          const float4* __restrict__ mats, ApplyArgs a,
                                                          uint64_t n_tiles)
{
    const int lane = threadIdx.x & 63;
    const int col = lane & 15;
    const int q = lane >> 4;
    float ar[4], ai[4], as[4];
    load_a_c64k4(mats, lane, ar, ai, as);
    // loads use matrix index 4 s4 + q, stores row 4 q + r: the lane part is
    // bits 0-1 (targets 0, 1) for loads and bits 2-3 (targets 2, 3) for stores
    const uint64_t lane_in = ((q & 1) ? a.off[1] : 0) + ((q & 2) ? a.off[2] : 0);
    const uint64_t lane_out = ((q & 1) ? a.off[4] : 0) + ((q & 2) ? a.off[8] : 0);
    const uint64_t n_waves = uint64_t(gridDim.x) * (blockDim.x >> 6);
    for (uint64_t t = uint64_t(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6); t < n_tiles; t += n_waves) {
        const uint64_t g = t * 16 + col;
        const bool valid = g < a.n_groups;
        const uint64_t base = valid ? group_base(g, a) : 0;
        float2 x[4];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) x[s4] = valid ? psi[base + lane_in + a.off[4 * s4]] : float2{0.f, 0.f};
        f32x4 p1 = {0}, p2 = {0}, p3 = {0};
        mfma_c64k4(ar, ai, as, x, p1, p2, p3);
        if (valid) {
#pragma unroll
            for (int r = 0; r < 4; ++r) psi[base + lane_out + a.off[r]] = float2{p1[r] - p2[r], p3[r] - p1[r] - p2[r]};
        }
    }
}

// ------------------------------------------------------- LDS-staged tiles
//
// The main sweep for uncontrolled gates on states of >= 12 (complex64) or
// >= 11 (complex128) qubits.  A tile is the 2^12 (complex64) or 2^11
// (complex128) amplitudes = 32 KiB whose index bits outside {0..L-1} and
// the targets >= L are fixed, with L the smallest width that leaves 2^(TB-k)
// whole groups in the tile.  The tile is 2^(k_hi) contiguous runs of 2^L
// amplitudes (one run per setting of the high targets), so every global
// access is a coalesced 16-byte load or store over runs of >= 1 KiB,
// whatever the targets are; the gather of each group's 2^k amplitudes
// happens in LDS.  A workgroup sweeps `tiles_per_wg` consecutive tiles,
// loading its A operands once and prefetching tile t+1 into registers while
// tile t is in LDS.  Each wave owns whole groups, so the in-place update in
// LDS needs no synchronisation beyond the three barriers per tile.

// The wide shape of the complex64 k = 5 sweep: 64 KiB tiles in 512-thread
// workgroups (8 waves, 256 groups), so every run of a tile is 2 KiB long
// instead of 1 KiB.  Which shape runs is chosen per handle (tile_shape).
constexpr int kK5Threads = 512;
constexpr int kK5TileBits = 13;

// 512-thread workgroups: two per CU (LDS), so four waves per SIMD must fit
// the register file (<= 128 VGPRs)
#ifndef SV_K5_WIDE_WAVES
#define SV_K5_WIDE_WAVES 2
#endif
template <int NT>
__global__ __launch_bounds__(NT, NT == 512 ? SV_K5_WIDE_WAVES : 1) void k_tile_c64_k5(float2* __restrict__ psi,
                                                             const float4* __restrict__ mats, TileArgs a)
{
    __shared__ float4 lds[NT * kTileVecs];
    // the packed A operands (same for every wave): 3 x 64 lanes x 4 float4,
    // read back four k-steps at a time so only 12 of them are live at once
    __shared__ float4 amat[kK5AStaged * 64 * 4];
    tile_c64_k5_sweep<NT, false>(psi, mats, a, blockIdx.x, lds, amat, ZSums{nullptr, -1, nullptr, nullptr});
}

// The same sweep for a block of coupled fusion: each group's inputs are first
// multiplied by the block's phase coupling (CoupleDev).
template <int NT>
__global__ __launch_bounds__(NT, NT == 512 ? SV_K5_WIDE_WAVES : 3) void k_tile_c64_k5c(
    float2* __restrict__ psi, const float4* __restrict__ mats, TileArgs a, const CoupleDev* __restrict__ cp)
{
    __shared__ float4 lds[NT * kTileVecs];
    __shared__ float4 amat[kK5AStaged * 64 * 4];
    tile_c64_k5_sweep<NT, false, true>(psi, mats, a, blockIdx.x, lds, amat, ZSums{nullptr, -1, nullptr, nullptr},
                                       cp);
}

__global__ __launch_bounds__(kTileThreads) void k_tile_c64_k4(float2* __restrict__ psi,
                                                             const float4* __restrict__ mats, TileArgs a)
{
    __shared__ float4 lds[kTileThreads * kTileVecs];
    const uint64_t t0 = uint64_t(blockIdx.x) * a.tiles_per_wg;
    if (t0 >= a.n_tiles) return;
    const uint64_t t1 = (a.n_tiles - t0 < a.tiles_per_wg) ? a.n_tiles : t0 + a.tiles_per_wg;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, col = lane & 15, q = lane >> 4;
    float ar[4], ai[4], as[4];
    load_a_c64k4(mats, lane, ar, ai, as);
    uint64_t roff[kTileVecs];
    uint32_t poff[kTileVecs];
    tile_offsets<2>(a, roff, poff);
    // each wave owns 4 column tiles of 16 groups: 256 groups per tile
    const int lin = ((q & 1) ? a.lds_off[1] : 0) + ((q & 2) ? a.lds_off[2] : 0);
    const int lout = ((q & 1) ? a.lds_off[4] : 0) + ((q & 2) ? a.lds_off[8] : 0);
    int pb[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) pb[ct] = int(insert_zero_bits(uint64_t(wave * 64 + ct * 16 + col), a.lo_pos, a.n_lo));
    float2* lds2 = reinterpret_cast<float2*>(lds);
#define SV_DECL(u) float4 buf##u;
    SV_REP8(SV_DECL)
#undef SV_DECL
    uint64_t base = tile_base(t0, a);
#define SV_LOAD(u) buf##u = gload(reinterpret_cast<const float4*>(psi + base + roff[u] + poff[u]));
    SV_REP8(SV_LOAD)
#undef SV_LOAD
    for (uint64_t t = t0; t < t1; ++t) {
#define SV_STAGE(u)                                                                        \
    {                                                                                      \
        const int i = (u * kTileThreads + tid) * 2;                                        \
        *reinterpret_cast<float4*>(lds2 + pair_slot(i)) = swap_pair(buf##u, pair_swapped(i)); \
    }
        SV_REP8(SV_STAGE)
#undef SV_STAGE
        __syncthreads();
        uint64_t nbase = 0;
        if (t + 1 < t1) {
            nbase = tile_base(t + 1, a);
#define SV_PREFETCH(u) buf##u = gload(reinterpret_cast<const float4*>(psi + nbase + roff[u] + poff[u]));
            SV_REP8(SV_PREFETCH)
#undef SV_PREFETCH
        }
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            float2 x[4];
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) x[s4] = lds2[lds_swz(pb[ct] + lin + a.lds_off[4 * s4])];
            f32x4 p1 = {0}, p2 = {0}, p3 = {0};
            mfma_c64k4(ar, ai, as, x, p1, p2, p3);
#pragma unroll
            for (int r = 0; r < 4; ++r)
                lds2[lds_swz(pb[ct] + lout + a.lds_off[r])] = float2{p1[r] - p2[r], p3[r] - p1[r] - p2[r]};
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kTileVecs; ++u) {
            const int i = (u * kTileThreads + tid) * 2;
            gstore(reinterpret_cast<float4*>(psi + base + roff[u] + poff[u]),
                   swap_pair(*reinterpret_cast<const float4*>(lds2 + pair_slot(i)), pair_swapped(i)));
        }
        base = nbase;
        __syncthreads();
    }
}

// complex128, k = 5 on v_mfma_f64_16x16x4_f64: 64 groups per tile, one
// 16-column tile per wave; two 16-row tiles cover the 32 output amplitudes.
// Re M and Im M are staged in LDS, lane-contiguous (16 KiB), and summed at
// use for the third product, which keeps 48 doubles per lane out of the
// registers: three workgroups per CU instead of two.
// NT = 256: 32 KiB tiles (2048 amplitudes); NT = 512: 64 KiB tiles (the
// wide shape), eight waves.
template <int NT, bool COUPLED>
__global__ __launch_bounds__(NT) void k_tile_c128_k5(double2* __restrict__ psi,
                                                              const double2* __restrict__ mats, TileArgs a,
                                                              const CoupleDev* __restrict__ cp)
{
    __shared__ double2 lds[NT * kTileVecs];
    __shared__ double amat[2 * 16 * 64];
    const uint64_t t0 = uint64_t(blockIdx.x) * a.tiles_per_wg;
    if (t0 >= a.n_tiles) return;
    const uint64_t t1 = (a.n_tiles - t0 < a.tiles_per_wg) ? a.n_tiles : t0 + a.tiles_per_wg;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, col = lane & 15, q = lane >> 4;
    {
        // packed A_g: lane l holds its 16 doubles contiguously; LDS: [g][j][l]
        const double* m1 = reinterpret_cast<const double*>(mats);
        for (int e = tid; e < 2 * 16 * 64; e += NT) {
            const int g = e >> 10, j = (e >> 6) & 15, l = e & 63;
            amat[e] = m1[(g * 64 + l) * 16 + j];
        }
    }
    uint64_t roff[kTileVecs];
    uint32_t poff[kTileVecs];
    tile_offsets<1, NT>(a, roff, poff);
    const int pb = int(insert_zero_bits(uint64_t(wave * 16 + col), a.lo_pos, a.n_lo));
    // loads: matrix index 4s + q; stores: row 16 rt + 4 v + q: bits 0-1 = q
    const int pq = pb + ((q & 1) ? a.lds_off[1] : 0) + ((q & 2) ? a.lds_off[2] : 0);
#define SV_DECL(u) double2 buf##u;
    SV_REP8(SV_DECL)
#undef SV_DECL
    uint64_t base = tile_base(t0, a);
#define SV_LOAD(u) buf##u = gload(psi + base + roff[u] + poff[u]);
    SV_REP8(SV_LOAD)
#undef SV_LOAD
    for (uint64_t t = t0; t < t1; ++t) {
#define SV_STAGE(u) lds[lds_swz(u * NT + tid)] = buf##u;
        SV_REP8(SV_STAGE)
#undef SV_STAGE
        __syncthreads();
        uint64_t nbase = 0;
        if (t + 1 < t1) {
            nbase = tile_base(t + 1, a);
#define SV_PREFETCH(u) buf##u = gload(psi + nbase + roff[u] + poff[u]);
            SV_REP8(SV_PREFETCH)
#undef SV_PREFETCH
        }
        double2 x[8];
#pragma unroll
        for (int s8 = 0; s8 < 8; ++s8) x[s8] = lds[lds_swz(pq + a.lds_off[4 * s8])];
        if constexpr (COUPLED) {
            // the block's phase coupling on this lane's group (tile-local base
            // pb); its amplitude s8 is matrix column 4 s8 + q, walked in
            // Gray-code order of s8
            auto cmul = [](const double2 u, const double2 w) {
                return double2{u.x * w.x - u.y * w.y, u.x * w.y + u.y * w.x};
            };
            auto cmulc = [](const double2 u, const double2 w) {
                return double2{u.x * w.x + u.y * w.y, u.y * w.x - u.x * w.y};
            };
            const uint64_t g = base + deposit_bits(uint32_t(pb >> a.L), a.hi_pos, a.n_hi) +
                               uint64_t(pb & ((1 << a.L) - 1));
            double L[5];
            couple_terms(cp, g, L);
            double2 e[5];
#pragma unroll
            for (int b = 0; b < 5; ++b) {
                double sn, cs;
                sincospi(L[b], &sn, &cs);
                e[b] = double2{cs, sn};
            }
            double2 v = double2{1.0, 0.0};
            if (q & 1) v = e[0];
            if (q & 2) v = cmul(v, e[1]);
            x[0] = cmul(x[0], v);
#pragma unroll
            for (int st = 1; st < 8; ++st) {
                const int j = st ^ (st >> 1), b = __builtin_ctz(st);
                v = ((j >> b) & 1) ? cmul(v, e[b + 2]) : cmulc(v, e[b + 2]);
                x[j] = cmul(x[j], v);
            }
        }
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
            f64x4 p1 = {0}, p2 = {0}, p3 = {0};
#pragma unroll
            for (int s8 = 0; s8 < 8; ++s8) {
                const double a0 = amat[(0 * 16 + rt * 8 + s8) * 64 + lane];
                const double a1 = amat[(1 * 16 + rt * 8 + s8) * 64 + lane];
                const double a2 = a0 + a1;
                p1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, x[s8].x, p1, 0, 0, 0);
                p2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, x[s8].y, p2, 0, 0, 0);
                p3 = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, x[s8].x + x[s8].y, p3, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v)
                lds[lds_swz(pq + a.lds_off[16 * rt + 4 * v])] = double2{p1[v] - p2[v], p3[v] - p1[v] - p2[v]};
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kTileVecs; ++u)
            gstore(psi + base + roff[u] + poff[u], lds[lds_swz(u * NT + tid)]);
        base = nbase;
        __syncthreads();
    }
}

// ----------------------------------------------------------- k = 6 tiles
//
// Six-qubit blocks on the matrix cores: a 64 x 64 complex matrix per group,
// three real GEMMs (Gauss).  64 KiB tiles in 512-thread workgroups (eight
// waves); the A operands are staged once per workgroup in LDS.  Every wave
// reads all inputs of its groups, so the outputs are written back only after
// a barrier.  One workgroup fits a CU (LDS), so the next tile's loads are in
// flight while a tile is transformed, as in the k = 5 sweep.
constexpr int kK6Threads = 512;

// complex64: v_mfma_f32_32x32x2_f32.  Wave w takes 32 groups (column tile
// w & 3) and 32 output rows (row tile w >> 2), K = 64 in 32 steps of 2.
// A_g (g = Re, Im, Re + Im) per lane l = i + 32 half, row tile rt:
// amat[((g * 2 + rt) * 64 + l) * 8 + s4] = A_g[32 rt + i][2 (4 s4 + j) + half], j = 0..3.
__global__ __launch_bounds__(kK6Threads, 2) void k_tile_c64_k6(float2* __restrict__ psi,
                                                              const float4* __restrict__ mats, TileArgs a)
{
    constexpr int NT = kK6Threads;
    __shared__ float4 lds[NT * kTileVecs];
    __shared__ float4 amat[3 * 2 * 64 * 8];
    const uint64_t t0 = uint64_t(blockIdx.x) * a.tiles_per_wg;
    if (t0 >= a.n_tiles) return;
    const uint64_t t1 = (a.n_tiles - t0 < a.tiles_per_wg) ? a.n_tiles : t0 + a.tiles_per_wg;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, col = lane & 31, half = lane >> 5;
    const int ct = wave & 3, rt = wave >> 2;
    for (int e = tid; e < 3 * 2 * 64 * 8; e += NT) amat[e] = mats[e];
    uint64_t roff[kTileVecs];
    uint32_t poff[kTileVecs];
    tile_offsets<2, NT>(a, roff, poff);
    const int pb = int(insert_zero_bits(uint64_t(ct * 32 + col), a.lo_pos, a.n_lo));
    const int pin = pb + (half ? a.lds_off[1] : 0);
    const int pout = pb + (half ? a.lds_off[4] : 0) + (rt ? a.lds_off[32] : 0);
    float2* lds2 = reinterpret_cast<float2*>(lds);
#define SV_DECL(u) float4 buf##u;
    SV_REP8(SV_DECL)
#undef SV_DECL
    uint64_t base = tile_base(t0, a);
#define SV_LOAD(u) buf##u = gload(reinterpret_cast<const float4*>(psi + base + roff[u] + poff[u]));
    SV_REP8(SV_LOAD)
#undef SV_LOAD
    for (uint64_t t = t0; t < t1; ++t) {
#define SV_STAGE(u)                                                                        \
    {                                                                                      \
        const int i = (u * NT + tid) * 2;                                                  \
        *reinterpret_cast<float4*>(lds2 + pair_slot(i)) = swap_pair(buf##u, pair_swapped(i)); \
    }
        SV_REP8(SV_STAGE)
#undef SV_STAGE
        __syncthreads();
        uint64_t nbase = 0;
        if (t + 1 < t1) {
            nbase = tile_base(t + 1, a);
#define SV_PREFETCH(u) buf##u = gload(reinterpret_cast<const float4*>(psi + nbase + roff[u] + poff[u]));
            SV_REP8(SV_PREFETCH)
#undef SV_PREFETCH
        }
        float2 x[32];
#pragma unroll
        for (int s2 = 0; s2 < 32; ++s2) x[s2] = lds2[lds_swz(pin + a.lds_off[2 * s2])];
        f32x16 p1 = {0}, p2 = {0}, p3 = {0};
#pragma unroll
        for (int s4 = 0; s4 < 8; ++s4) {
            const float4 vr = amat[((0 * 2 + rt) * 64 + lane) * 8 + s4];
            const float4 vi = amat[((1 * 2 + rt) * 64 + lane) * 8 + s4];
            const float4 vs = amat[((2 * 2 + rt) * 64 + lane) * 8 + s4];
            const float ar[4] = {vr.x, vr.y, vr.z, vr.w};
            const float ai[4] = {vi.x, vi.y, vi.z, vi.w};
            const float as[4] = {vs.x, vs.y, vs.z, vs.w};
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const float2 xv = x[4 * s4 + jj];
                p1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[jj], xv.x, p1, 0, 0, 0);
                p2 = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[jj], xv.y, p2, 0, 0, 0);
                p3 = __builtin_amdgcn_mfma_f32_32x32x2f32(as[jj], xv.x + xv.y, p3, 0, 0, 0);
            }
        }
        __syncthreads();  // every wave has read its inputs
#pragma unroll
        for (int r = 0; r < 16; ++r)
            lds2[lds_swz(pout + a.lds_off[8 * (r / 4) + (r % 4)])] = float2{p1[r] - p2[r], p3[r] - p1[r] - p2[r]};
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kTileVecs; ++u) {
            const int i = (u * NT + tid) * 2;
            gstore(reinterpret_cast<float4*>(psi + base + roff[u] + poff[u]),
                   swap_pair(*reinterpret_cast<const float4*>(lds2 + pair_slot(i)), pair_swapped(i)));
        }
        base = nbase;
        __syncthreads();
    }
}

// complex128: v_mfma_f64_16x16x4_f64.  Wave w takes 16 groups (column tile
// w & 3) and 32 output rows (row tiles 2 (w >> 2) and 2 (w >> 2) + 1), K = 64
// in 16 steps of 4.  A_g (g = Re, Im; Re + Im is summed here) per lane
// l = i + 16 q, row tile rt: amat[((g * 4 + rt) * 16 + s) * 64 + l] = A_g[16 rt + i][4 s + q].
__global__ __launch_bounds__(kK6Threads, 2) void k_tile_c128_k6(double2* __restrict__ psi,
                                                               const double* __restrict__ mats, TileArgs a)
{
    constexpr int NT = kK6Threads;
    __shared__ double2 lds[NT * kTileVecs];
    __shared__ double amat[2 * 4 * 16 * 64];
    const uint64_t t0 = uint64_t(blockIdx.x) * a.tiles_per_wg;
    if (t0 >= a.n_tiles) return;
    const uint64_t t1 = (a.n_tiles - t0 < a.tiles_per_wg) ? a.n_tiles : t0 + a.tiles_per_wg;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, col = lane & 15, q = lane >> 4;
    const int ct = wave & 3, rh = wave >> 2;
    for (int e = tid; e < 2 * 4 * 16 * 64; e += NT) amat[e] = mats[e];
    uint64_t roff[kTileVecs];
    uint32_t poff[kTileVecs];
    tile_offsets<1, NT>(a, roff, poff);
    const int pb = int(insert_zero_bits(uint64_t(ct * 16 + col), a.lo_pos, a.n_lo));
    // inputs: matrix index 4 s + q; outputs: row 16 rt + 4 v + q: bits 0-1 = q
    const int pq = pb + ((q & 1) ? a.lds_off[1] : 0) + ((q & 2) ? a.lds_off[2] : 0);
#define SV_DECL(u) double2 buf##u;
    SV_REP8(SV_DECL)
#undef SV_DECL
    uint64_t base = tile_base(t0, a);
#define SV_LOAD(u) buf##u = gload(psi + base + roff[u] + poff[u]);
    SV_REP8(SV_LOAD)
#undef SV_LOAD
    for (uint64_t t = t0; t < t1; ++t) {
#define SV_STAGE(u) lds[lds_swz(u * NT + tid)] = buf##u;
        SV_REP8(SV_STAGE)
#undef SV_STAGE
        __syncthreads();
        uint64_t nbase = 0;
        if (t + 1 < t1) {
            nbase = tile_base(t + 1, a);
#define SV_PREFETCH(u) buf##u = gload(psi + nbase + roff[u] + poff[u]);
            SV_REP8(SV_PREFETCH)
#undef SV_PREFETCH
        }
        double2 x[16];
#pragma unroll
        for (int s = 0; s < 16; ++s) x[s] = lds[lds_swz(pq + a.lds_off[4 * s])];
        f64x4 p1[2], p2[2], p3[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int rt = 2 * rh + h;
            p1[h] = f64x4{0, 0, 0, 0};
            p2[h] = f64x4{0, 0, 0, 0};
            p3[h] = f64x4{0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                const double ar = amat[((0 * 4 + rt) * 16 + s) * 64 + lane];
                const double ai = amat[((1 * 4 + rt) * 16 + s) * 64 + lane];
                p1[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, x[s].x, p1[h], 0, 0, 0);
                p2[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, x[s].y, p2[h], 0, 0, 0);
                p3[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar + ai, x[s].x + x[s].y, p3[h], 0, 0, 0);
            }
        }
        __syncthreads();  // every wave has read its inputs
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int rt = 2 * rh + h;
#pragma unroll
            for (int v = 0; v < 4; ++v)
                lds[lds_swz(pq + a.lds_off[16 * rt + 4 * v])] =
                    double2{p1[h][v] - p2[h][v], p3[h][v] - p1[h][v] - p2[h][v]};
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kTileVecs; ++u)
            gstore(psi + base + roff[u] + poff[u], lds[lds_swz(u * NT + tid)]);
        base = nbase;
        __syncthreads();
    }
}

// Large gates (k = 7..10, compute-bound): one workgroup per group.  The
// group's 2^k amplitudes are staged in LDS; each thread forms whole rows.
struct ApplyArgsLarge {
    uint64_t n_groups;
    uint64_t cval;
    int32_t n_fixed;
    int32_t fixed[SV_MAX_QUBITS];
    int32_t k;
    uint64_t tbit[SV_MAX_TARGETS];
};

template <typename R>
__global__ __launch_bounds__(256) void k_apply_large(typename Cx<R>::T* __restrict__ psi,
                                                     const typename Cx<R>::T* __restrict__ mat,
                                                     ApplyArgsLarge a)
{
    using T2 = typename Cx<R>::T;
    extern __shared__ unsigned char smem_raw[];
    T2* v = reinterpret_cast<T2*>(smem_raw);
    const int D = 1 << a.k;
    for (uint64_t g = blockIdx.x; g < a.n_groups; g += gridDim.x) {
        uint64_t base = g;
        for (int j = 0; j < a.n_fixed; ++j) {
            const int p = a.fixed[j];
            const uint64_t lo = base & ((uint64_t(1) << p) - 1);
            base = ((base >> p) << (p + 1)) | lo;
        }
        base |= a.cval;
        for (int c = threadIdx.x; c < D; c += blockDim.x) {
            uint64_t off = 0;
            for (int b = 0; b < a.k; ++b)
                if ((c >> b) & 1) off |= a.tbit[b];
            v[c] = psi[base + off];
        }
        __syncthreads();
        for (int r = threadIdx.x; r < D; r += blockDim.x) {
            R re = 0, im = 0;
            for (int c = 0; c < D; ++c) {
                const T2 m = mat[size_t(r) * D + c];
                re = fma(m.x, v[c].x, re);
                re = fma(-m.y, v[c].y, re);
                im = fma(m.x, v[c].y, im);
                im = fma(m.y, v[c].x, im);
            }
            uint64_t off = 0;
            for (int b = 0; b < a.k; ++b)
                if ((r >> b) & 1) off |= a.tbit[b];
            psi[base + off] = T2{re, im};
        }
        __syncthreads();
    }
}

enum class Path { kValu, kLarge, kMfmaC64K5, kMfmaC64K4, kTileC64K5, kTileC64K4, kTileC128K5, kTileC64K6, kTileC128K6 };

Path choose(sv_dtype_t dt, int n, int k, int n_controls)
{
    if (k > kMaxUnrolledK) return Path::kLarge;
    const bool tile_ok = n_controls == 0;
    if (dt == SV_C64 && k == 5) return (tile_ok && n >= 12) ? Path::kTileC64K5 : Path::kMfmaC64K5;
    if (dt == SV_C64 && k == 4) return (tile_ok && n >= 12) ? Path::kTileC64K4 : Path::kMfmaC64K4;
    if (dt == SV_C128 && k == 5 && tile_ok && n >= 11) return Path::kTileC128K5;
    if (dt == SV_C64 && k == 6 && tile_ok && n >= 13) return Path::kTileC64K6;
    if (dt == SV_C128 && k == 6 && tile_ok && n >= 12) return Path::kTileC128K6;
    return Path::kValu;
}

void fill_args(ApplyArgs& a, const GateDesc& d)
{
    a.n_groups = d.n_groups;
    a.cval = d.cval;
    a.n_fixed = d.n_fixed;
    for (int j = 0; j < d.n_fixed; ++j) a.fixed[j] = d.fixed_sorted[j];
    for (int r = 0; r < (1 << d.k); ++r) {
        uint64_t off = 0;
        for (int b = 0; b < d.k; ++b)
            if ((r >> b) & 1) off |= d.tbit[b];
        a.off[r] = off;
    }
}

void launch_mfma_c64(sv_handle_s* h, float2* psi, const float4* mats, const GateDesc& d)
{
    ApplyArgs a{};
    fill_args(a, d);
    const uint64_t cols = d.k == 5 ? 32 : 16;
    const uint64_t n_tiles = (d.n_groups + cols - 1) / cols;
    const uint64_t waves_per_block = 4;
    uint64_t blocks = (n_tiles + waves_per_block - 1) / waves_per_block;
    const uint64_t cap = uint64_t(h->cu_count) * 8;
    if (blocks > cap) blocks = cap;
    if (d.k == 5)
        hipLaunchKernelGGL(k_apply_mfma_c64_k5, dim3(unsigned(blocks)), dim3(256), 0, h->stream, psi, mats, a,
                           n_tiles);
    else
        hipLaunchKernelGGL(k_apply_mfma_c64_k4, dim3(unsigned(blocks)), dim3(256), 0, h->stream, psi, mats, a,
                           n_tiles);
    SV_HIP(hipGetLastError());
}

// Tile geometry for a gate with targets d.tbit (matrix order) on n qubits;
// tb = log2 of the tile's amplitude count.  The tile is the low L index
// bits plus the bit set H (hi_pos): by default L is the smallest width that
// leaves 2^(tb-k) groups in the tile and H the targets >= L.  With
// spread_lo > 0 (and a target below tb - k) the runs are 2^(tb-k)
// amplitudes and each target below them is matched by a free bit at or
// above spread_lo in H, so the tile's runs are spread out in memory.
// lo_pos lists the targets' positions inside the tile (bits < L as is, H's
// bits at L + their rank in H).  strided: workgroups take their tiles
// n_tiles / tiles_per_wg apart (tile_base) instead of consecutively.
}  // namespace

TileArgs make_tile_args(const GateDesc& d, int n, int tb, int cu_count, int spread_lo, bool strided)
{
    int tq[SV_MAX_TARGETS];
    bool is_target[64] = {};
    for (int a = 0; a < d.k; ++a) {
        int q = 0;
        while ((uint64_t(1) << q) != d.tbit[a]) ++q;
        tq[a] = q;
        is_target[q] = true;
    }
    const int gbits = tb - d.k;  // log2 groups per tile
    int L = gbits;
    for (;;) {
        int klo = 0;
        for (int a = 0; a < d.k; ++a) klo += tq[a] < L;
        if (L - klo >= gbits) break;
        ++L;
    }
    bool extra[64] = {};
    if (spread_lo > 0) {
        int klo = 0;
        for (int a = 0; a < d.k; ++a) klo += tq[a] < gbits;
        int found = 0;
        bool pick[64] = {};
        for (int q = std::max(gbits, spread_lo); q < n && found < klo; ++q)
            if (!is_target[q]) {
                pick[q] = true;
                ++found;
            }
        if (klo > 0 && found == klo) {
            L = gbits;
            for (int q = 0; q < 64; ++q) extra[q] = pick[q];
        }
    }
    TileArgs t{};
    t.L = L;
    int nh = 0;
    for (int q = L; q < n; ++q)
        if (is_target[q] || extra[q]) t.hi_pos[nh++] = q;
    t.n_hi = nh;
    int local[SV_MAX_TARGETS];
    for (int a = 0; a < d.k; ++a) {
        if (tq[a] < L) {
            local[a] = tq[a];
        } else {
            int rank = 0;
            while (t.hi_pos[rank] != tq[a]) ++rank;
            local[a] = L + rank;
        }
    }
    int nl = 0;
    for (int p = 0; p < tb; ++p)
        for (int a = 0; a < d.k; ++a)
            if (local[a] == p) t.lo_pos[nl++] = p;
    t.n_lo = nl;
    for (int c = 0; c < (1 << d.k); ++c) {
        int off = 0;
        for (int a = 0; a < d.k; ++a)
            if ((c >> a) & 1) off |= 1 << local[a];
        t.lds_off[c] = off;
    }
    t.n_tiles = uint64_t(1) << (n - tb);
    // about 32 workgroups per CU over the sweep, each on consecutive tiles
    const uint64_t target_wgs = uint64_t(cu_count) * SV_TILE_WGS_PER_CU;
    uint64_t per = t.n_tiles / target_wgs;
    if (per < 1) per = 1;
    const uint64_t cap = d.k >= 5 ? SV_TILES_PER_WG_MAX_K5 : SV_TILES_PER_WG_MAX;
    if (per > cap) per = cap;
    t.tiles_per_wg = per;
    t.lg_tiles = n - tb;
    if (strided && (per & (per - 1)) == 0)
        while ((uint64_t(1) << t.trot) < per) ++t.trot;
    return t;
}

namespace {

// ------------------------------------------------- tile shape autotuning

hipEvent_t tuner_event(TileTuner& T)
{
    if (!T.pool.empty()) {
        hipEvent_t e = T.pool.back();
        T.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    SV_HIP(hipEventCreate(&e));
    return e;
}

// Folds finished trials into their entries, oldest first, up to the first
// one still running (trials finish in launch order on the handle's stream;
// one per launch query while the device runs behind the host).
void tuner_poll(TileTuner& T)
{
    while (!T.pending.empty()) {
        TileTrial& tr = T.pending.front();
        const hipError_t q = hipEventQuery(tr.e1);
        if (q == hipErrorNotReady) return;
        TileTuneEntry& e = T.entries[tr.key];
        float ms = 0.f;
        if (q == hipSuccess && hipEventElapsedTime(&ms, tr.e0, tr.e1) == hipSuccess) {
            e.sum_ms[tr.shape] += ms;
            ++e.measured[tr.shape];
        } else {
            (void)hipGetLastError();
            e.unusable[tr.shape] = true;  // no timing: never chosen, not tried again
        }
        --e.in_flight[tr.shape];
        T.pool.push_back(tr.e0);
        T.pool.push_back(tr.e1);
        T.pending.pop_front();
    }
}

// Variants of the k = 5 sweeps (complex64 and complex128) the handle chooses
// among: narrow 32 KiB tiles, wide 64 KiB tiles, and narrow tiles with the
// spread layout (free bits from 12 up in place of the low targets) taken in
// strided order.  Which is fastest depends on the target set: in-circuit on
// 30 qubits, the spread variant wins for windows of low or high targets, the
// plain narrow one for targets around bits 10-13, the wide one where the
// targets sit right above the 1 KiB runs.
struct TileVariant {
    bool wide;
    int spread_lo;
    bool strided;
};
// Index 0 is the default: the variant that runs before any timing (and for
// target sets seen too rarely to be timed), the best single variant in-circuit.
constexpr TileVariant kTileVariants[kTileShapes] = {{false, 12, true}, {false, 0, false}, {true, 0, false}};
constexpr int kVariantSpread = 0, kVariantNarrow = 1, kVariantWide = 2;
constexpr TileVariant kPlainTiles = {false, 0, false};  // the sweeps without variants (k = 4, 6)

uint64_t tune_key(Path p, const GateDesc& d)
{
    uint64_t key = (uint64_t(d.n) << 40) | (uint64_t(p == Path::kTileC128K5) << 48);
    for (int a = 0; a < d.k; ++a) key |= d.tbit[a];
    return key;
}

// Tile bits of the wide shape: complex64 64 KiB = 2^13 amplitudes,
// complex128 64 KiB = 2^12.
int wide_tile_bits(Path p) { return p == Path::kTileC128K5 ? 12 : kK5TileBits; }

// Variant for a k = 5 tile sweep (index into kTileVariants).  *trial is set
// when this launch is to be timed.
int tile_shape(sv_handle_s* h, Path p, const GateDesc& d, bool* trial, bool allow_trial)
{
    *trial = false;
    if (d.n < wide_tile_bits(p)) return kVariantNarrow;
    if (h->tile_mode == SV_TILE_NARROW) return kVariantNarrow;
    if (h->tile_mode == SV_TILE_WIDE) return kVariantWide;
    if (h->tile_mode == SV_TILE_SPREAD) return kVariantSpread;
    // a small state sweeps from the caches in a few microseconds, bound by
    // the launch more than by any tile shape: the default, untimed
    if (d.n < SV_TILE_TUNE_MIN_QUBITS) return kVariantSpread;
    TileTuner& T = *h->tuner;
    const uint64_t key = tune_key(p, d);
    // while the stream is being recorded into a graph: no event queries and
    // no timed trials, only the choice made so far
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    const bool capturing = hipStreamIsCapturing(h->stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
    if (capturing) (void)hipGetLastError();
    if (!capturing) tuner_poll(T);
    TileTuneEntry& e = T.entries[key];
    auto done = [&](int c) { return e.unusable[c] || e.measured[c] + e.in_flight[c] >= kTileTrials; };
    if (!capturing && allow_trial && T.sweeps++ >= uint64_t(kTileWarmSweeps)) {
        // trial j (counted over all variants) of this key belongs to round
        // j / kTileShapes, which visits the variants starting from the
        // round's number, so each variant takes every place in the order
        int j = 0;
        for (int c = 0; c < kTileShapes; ++c) j += e.measured[c] + e.in_flight[c];
        int s = -1;
        for (int i = 0; i < kTileShapes && s < 0; ++i) {
            const int c = (j / kTileShapes + j % kTileShapes + i) % kTileShapes;
            if (!done(c)) s = c;
        }
        if (s >= 0) {
            *trial = true;
            return s;
        }
    }
    int best = -1;
    for (int c = 0; c < kTileShapes; ++c) {
        if (e.unusable[c] || e.measured[c] == 0) continue;
        if (best < 0 || e.sum_ms[c] * e.measured[best] < e.sum_ms[best] * e.measured[c]) best = c;
    }
    return best < 0 ? kVariantSpread : best;
}

void launch_tile(sv_handle_s* h, Path p, void* psi, const void* mats, const GateDesc& d,
                 const CoupleDev* cpl = nullptr)
{
    bool trial = false;
    const bool tuned = p == Path::kTileC64K5 || p == Path::kTileC128K5;
    // coupled sweeps do more arithmetic per group than the plain ones:
    // they take the variant the plain sweeps chose, without timed trials
    const int variant = tuned ? tile_shape(h, p, d, &trial, cpl == nullptr) : 0;
    const bool wide = tuned && kTileVariants[variant].wide;
    TileTrial tr{};
    if (trial) {
        tr.key = tune_key(p, d);
        tr.shape = variant;
        tr.e0 = tuner_event(*h->tuner);
        tr.e1 = tuner_event(*h->tuner);
        SV_HIP(hipEventRecord(tr.e0, h->stream));
    }
    const int tb = (p == Path::kTileC128K5)   ? (wide ? 12 : 11)
                   : (p == Path::kTileC64K6) ? 13
                   : (p == Path::kTileC128K6) ? 12
                   : wide                     ? kK5TileBits
                                              : 12;
    const TileVariant& v = tuned ? kTileVariants[variant] : kPlainTiles;
    const TileArgs t = make_tile_args(d, d.n, tb, h->cu_count, v.spread_lo, v.strided);
    const uint64_t blocks = (t.n_tiles + t.tiles_per_wg - 1) / t.tiles_per_wg;
    switch (p) {
        case Path::kTileC64K5:
            if (cpl && wide)
                hipLaunchKernelGGL(k_tile_c64_k5c<kK5Threads>, dim3(unsigned(blocks)), dim3(kK5Threads), 0,
                                   h->stream, static_cast<float2*>(psi), static_cast<const float4*>(mats), t, cpl);
            else if (cpl)
                hipLaunchKernelGGL(k_tile_c64_k5c<kTileThreads>, dim3(unsigned(blocks)), dim3(kTileThreads), 0,
                                   h->stream, static_cast<float2*>(psi), static_cast<const float4*>(mats), t, cpl);
            else if (wide)
                hipLaunchKernelGGL(k_tile_c64_k5<kK5Threads>, dim3(unsigned(blocks)), dim3(kK5Threads), 0,
                                   h->stream, static_cast<float2*>(psi), static_cast<const float4*>(mats), t);
            else
                hipLaunchKernelGGL(k_tile_c64_k5<kTileThreads>, dim3(unsigned(blocks)), dim3(kTileThreads), 0,
                                   h->stream, static_cast<float2*>(psi), static_cast<const float4*>(mats), t);
            break;
        case Path::kTileC64K4:
            hipLaunchKernelGGL(k_tile_c64_k4, dim3(unsigned(blocks)), dim3(kTileThreads), 0, h->stream,
                               static_cast<float2*>(psi), static_cast<const float4*>(mats), t);
            break;
        case Path::kTileC128K5:
            if (cpl && wide)
                hipLaunchKernelGGL((k_tile_c128_k5<512, true>), dim3(unsigned(blocks)), dim3(512), 0, h->stream,
                                   static_cast<double2*>(psi), static_cast<const double2*>(mats), t, cpl);
            else if (cpl)
                hipLaunchKernelGGL((k_tile_c128_k5<kTileThreads, true>), dim3(unsigned(blocks)), dim3(kTileThreads),
                                   0, h->stream, static_cast<double2*>(psi), static_cast<const double2*>(mats), t, cpl);
            else if (wide)
                hipLaunchKernelGGL((k_tile_c128_k5<512, false>), dim3(unsigned(blocks)), dim3(512), 0, h->stream,
                                   static_cast<double2*>(psi), static_cast<const double2*>(mats), t, nullptr);
            else
                hipLaunchKernelGGL((k_tile_c128_k5<kTileThreads, false>), dim3(unsigned(blocks)), dim3(kTileThreads),
                                   0, h->stream, static_cast<double2*>(psi), static_cast<const double2*>(mats), t,
                                   nullptr);
            break;
        case Path::kTileC64K6:
            hipLaunchKernelGGL(k_tile_c64_k6, dim3(unsigned(blocks)), dim3(kK6Threads), 0, h->stream,
                               static_cast<float2*>(psi), static_cast<const float4*>(mats), t);
            break;
        case Path::kTileC128K6:
            hipLaunchKernelGGL(k_tile_c128_k6, dim3(unsigned(blocks)), dim3(kK6Threads), 0, h->stream,
                               static_cast<double2*>(psi), static_cast<const double*>(mats), t);
            break;
        default:
            throw Error{SV_ERR_INTERNAL, "not a tile path"};
    }
    SV_HIP(hipGetLastError());
    if (trial) {
        SV_HIP(hipEventRecord(tr.e1, h->stream));
        h->tuner->entries[tr.key].in_flight[tr.shape]++;
        h->tuner->pending.push_back(tr);
    }
}

template <typename R>
void launch_apply_t(sv_handle_s* h, void* psi_v, const void* mat_v, const GateDesc& d)
{
    using T2 = typename Cx<R>::T;
    T2* psi = static_cast<T2*>(psi_v);
    const T2* mat = static_cast<const T2*>(mat_v);
    if (d.k <= kMaxUnrolledK) {
        ApplyArgs a{};
        fill_args(a, d);
        // a dispatch counts at most 2^32 - 1 work-items per grid dimension:
        // spread the blocks over x and y
        const uint64_t threads = 256;
        const uint64_t blocks = (d.n_groups + threads - 1) / threads;
        const uint64_t bx = blocks < (uint64_t(1) << 20) ? blocks : (uint64_t(1) << 20);
        const uint64_t by = (blocks + bx - 1) / bx;
        const dim3 grid{unsigned(bx), unsigned(by), 1u};
        switch (d.k) {
#define SV_CASE(K)                                                                            \
    case K:                                                                                   \
        hipLaunchKernelGGL((k_apply_dense<R, K>), grid, dim3(threads), 0, h->stream, psi, mat, a); \
        break;
            SV_CASE(1)
            SV_CASE(2)
            SV_CASE(3)
            SV_CASE(4)
            SV_CASE(5)
            SV_CASE(6)
#undef SV_CASE
            default:
                throw Error{SV_ERR_INTERNAL, "unreachable gate size"};
        }
    } else {
        ApplyArgsLarge a{};
        a.n_groups = d.n_groups;
        a.cval = d.cval;
        a.n_fixed = d.n_fixed;
        for (int j = 0; j < d.n_fixed; ++j) a.fixed[j] = d.fixed_sorted[j];
        a.k = d.k;
        for (int b = 0; b < d.k; ++b) a.tbit[b] = d.tbit[b];
        uint64_t blocks = d.n_groups;
        const uint64_t cap = uint64_t(h->cu_count) * 8;
        if (blocks > cap) blocks = cap;
        const size_t lds = sizeof(T2) << d.k;  // <= 16 KiB
        hipLaunchKernelGGL((k_apply_large<R>), dim3(unsigned(blocks)), dim3(256), lds, h->stream,
                           psi, mat, a);
    }
    SV_HIP(hipGetLastError());
}

// ------------------------------------------- generalized permutation gates
//
// G = D P on k targets (Table I: gate application with a generalized
// permutation matrix; Sec. II-D: diagonal gates and diagonal gate fusion):
// in every group, the amplitude at offset r becomes diag[r] times the one
// at offset perm[r].  A diagonal (no permutation) touches each amplitude on
// its own: one coalesced streaming pass with the 2^k-entry table in LDS,
// over the control-satisfying amplitudes only.  A true permutation moves
// amplitudes inside their group: the tile geometry of the dense sweeps
// (whole groups per 32 KiB tile) with the permutation done in LDS.

struct DiagArgs {
    uint64_t n_vecs;                   // vectors in the control-compressed index space
    int32_t k;
    int32_t tpos[SV_MAX_TARGETS];      // index bit of matrix bit a
    int32_t n_ctrl;
    int32_t cpos[SV_MAX_QUBITS];       // control bits, ascending
    uint64_t cval;
};

constexpr int kDiagThreads = 256;
constexpr int kDiagVecs = 8;

template <typename T>
__device__ __forceinline__ T cmul(const T a, const T b)
{
    return T{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

__device__ __forceinline__ int diag_row(uint64_t i, const DiagArgs& a)
{
    int r = 0;
    for (int b = 0; b < a.k; ++b) r |= int((i >> a.tpos[b]) & 1) << b;
    return r;
}

// APV complex amplitudes per 16-byte vector: 2 for complex64 (pairs i, i+1
// with bit 0 free), 1 for complex128.  NARROW: complex64 one amplitude per
// 8-byte access (bit 0 is a control).
template <typename R, bool NARROW>
__global__ __launch_bounds__(kDiagThreads) void k_apply_diag(typename Cx<R>::T* __restrict__ psi,
                                                             const typename Cx<R>::T* __restrict__ table, DiagArgs a)
{
    using T = typename Cx<R>::T;
    constexpr int APV = (sizeof(T) == 8 && !NARROW) ? 2 : 1;
    __shared__ T tab[1 << SV_MAX_TARGETS];
    for (int e = threadIdx.x; e < (1 << a.k); e += kDiagThreads) tab[e] = table[e];
    __syncthreads();
    const uint64_t v0 = uint64_t(blockIdx.x) * (kDiagThreads * kDiagVecs) + threadIdx.x;
    T x[kDiagVecs][APV];
    uint64_t at[kDiagVecs];
#pragma unroll
    for (int u = 0; u < kDiagVecs; ++u) {
        const uint64_t v = v0 + uint64_t(u) * kDiagThreads;
        at[u] = v < a.n_vecs ? (insert_zero_bits(v * APV, a.cpos, a.n_ctrl) | a.cval) : ~uint64_t(0);
        if (at[u] != ~uint64_t(0)) {
            if constexpr (APV == 2) {
                const float4 w = gload(reinterpret_cast<const float4*>(psi + at[u]));
                x[u][0] = T{w.x, w.y};
                x[u][APV - 1] = T{w.z, w.w};
            } else if constexpr (sizeof(T) == 16) {
                x[u][0] = gload(psi + at[u]);
            } else {
                x[u][0] = psi[at[u]];
            }
        }
    }
#pragma unroll
    for (int u = 0; u < kDiagVecs; ++u) {
        if (at[u] == ~uint64_t(0)) continue;
#pragma unroll
        for (int e = 0; e < APV; ++e) x[u][e] = cmul(tab[diag_row(at[u] + e, a)], x[u][e]);
        if constexpr (APV == 2) {
            gstore(reinterpret_cast<float4*>(psi + at[u]), float4{x[u][0].x, x[u][0].y, x[u][APV - 1].x, x[u][APV - 1].y});
        } else if constexpr (sizeof(T) == 16) {
            gstore(psi + at[u], x[u][0]);
        } else {
            psi[at[u]] = x[u][0];
        }
    }
}

// One 32 KiB tile per workgroup (whole groups: 2^tb amplitudes), loaded to
// LDS, then every output read from its permuted source in LDS.  diag: 2^k
// entries in the state's precision, perm: 2^k ints (k <= 6).
template <typename R>
__global__ __launch_bounds__(kTileThreads) void k_tile_gperm(typename Cx<R>::T* __restrict__ psi,
                                                             const typename Cx<R>::T* __restrict__ diag,
                                                             const int32_t* __restrict__ perm, TileArgs a, int k)
{
    using T = typename Cx<R>::T;
    constexpr int kAmps = 32768 / int(sizeof(T));
    __shared__ T lds[kAmps];
    __shared__ T dtab[64];
    __shared__ int32_t ptab[64];
    __shared__ int32_t lpos[SV_MAX_TARGETS];
    const int tid = threadIdx.x;
    if (tid < (1 << k)) {
        dtab[tid] = diag[tid];
        ptab[tid] = perm[tid];
    }
    if (tid < k) lpos[tid] = 31 - __clz(a.lds_off[1 << tid]);
    const uint64_t base = tile_base(blockIdx.x, a);
    const uint64_t mask = (uint64_t(1) << a.L) - 1;
    // 16-byte accesses: amplitude pairs (e, e + 1), e even, for complex64
    // (the runs are at least 2^6 amplitudes long, so a pair never straddles
    // two runs), single amplitudes for complex128
    constexpr int APV = sizeof(T) == 8 ? 2 : 1;
    constexpr int kVecs = kAmps / APV / kTileThreads;
    auto glob = [&](int e) { return base + deposit_bits(uint32_t(e >> a.L), a.hi_pos, a.n_hi) + (uint64_t(e) & mask); };
    using V = typename std::conditional<APV == 2, float4, double2>::type;
    V v[kVecs];
#pragma unroll
    for (int u = 0; u < kVecs; ++u) v[u] = gload(reinterpret_cast<const V*>(psi + glob((u * kTileThreads + tid) * APV)));
#pragma unroll
    for (int u = 0; u < kVecs; ++u) reinterpret_cast<V*>(lds)[u * kTileThreads + tid] = v[u];
    __syncthreads();
    const int full = a.lds_off[(1 << k) - 1];
    auto out = [&](int e) {
        int r = 0;
        for (int b = 0; b < k; ++b) r |= ((e >> lpos[b]) & 1) << b;
        return cmul(dtab[r], lds[(e & ~full) + a.lds_off[ptab[r]]]);
    };
#pragma unroll
    for (int u = 0; u < kVecs; ++u) {
        const int e = (u * kTileThreads + tid) * APV;
        if constexpr (APV == 2) {
            const T lo = out(e), hi = out(e + 1);
            v[u] = V{lo.x, lo.y, hi.x, hi.y};
        } else {
            v[u] = out(e);
        }
    }
#pragma unroll
    for (int u = 0; u < kVecs; ++u)
        gstore(reinterpret_cast<V*>(psi + glob((u * kTileThreads + tid) * APV)), v[u]);
}

// Phase coupling on its own (blocks of coupled fusion whose dense part does
// not run on the five-qubit tiles): one thread per amplitude, which is
// rewritten only if its phase is not zero.
template <typename R>
__global__ __launch_bounds__(256) void k_couple(typename Cx<R>::T* __restrict__ psi, uint64_t dim,
                                                const CoupleDev* __restrict__ cp)
{
    using T = typename Cx<R>::T;
    const uint64_t i = uint64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= dim) return;
    double th = 0.0;
    for (int a = 0; a < cp->k; ++a) {
        if (!((i >> cp->t[a]) & 1)) continue;
        for (int c = 0; c < cp->n; ++c) th = fma(double((i >> cp->q[c]) & 1), cp->phase[a * SV_MAX_QUBITS + c], th);
    }
    if (th == 0.0) return;
    th -= 2.0 * rint(0.5 * th);
    double sn, cs;
    sincospi(th, &sn, &cs);
    const T v = psi[i];
    const double re = double(v.x), im = double(v.y);
    psi[i] = T{R(re * cs - im * sn), R(re * sn + im * cs)};
}

}  // namespace

void launch_apply_coupled(sv_handle_s* h, sv_dtype_t dt, void* psi, const void* mat, const void* couple,
                          const GateDesc& d)
{
    const CoupleDev* cp = static_cast<const CoupleDev*>(couple);
    const Path p = choose(dt, d.n, d.k, d.n_controls);
    if (p == Path::kTileC64K5 || p == Path::kTileC128K5) {
        launch_tile(h, p, psi, mat, d, cp);
        return;
    }
    const uint64_t dim = uint64_t(1) << d.n;
    const unsigned blocks = unsigned((dim + 255) / 256);
    if (dt == SV_C64)
        hipLaunchKernelGGL(k_couple<float>, dim3(blocks), dim3(256), 0, h->stream, static_cast<float2*>(psi), dim, cp);
    else
        hipLaunchKernelGGL(k_couple<double>, dim3(blocks), dim3(256), 0, h->stream, static_cast<double2*>(psi), dim,
                           cp);
    SV_HIP(hipGetLastError());
    launch_apply(h, dt, psi, mat, d);
}

size_t packed_matrix_bytes(sv_dtype_t dt, int n, int k, int n_controls)
{
    const size_t d2 = size_t(1) << (2 * k);
    switch (choose(dt, n, k, n_controls)) {
        case Path::kMfmaC64K4:
        case Path::kMfmaC64K5:
        case Path::kTileC64K4:
        case Path::kTileC64K5:
            return 3 * d2 * sizeof(float);
        case Path::kTileC128K5:
            return 3 * d2 * sizeof(double);
        case Path::kTileC64K6:
            return 3 * d2 * sizeof(float);
        case Path::kTileC128K6:
            return 2 * d2 * sizeof(double);
        default:
            return d2 * (dt == SV_C64 ? 8 : 16);
    }
}

void pack_matrix(sv_dtype_t dt, int n, int k, int n_controls, const double* m, int adjoint, void* dst)
{
    const int d = 1 << k;
    // A_g[i][c] with g = 0: Re M, 1: Im M, 2: Re M + Im M (of M or M^dagger)
    auto A = [&](int g, int i, int c) {
        const int src = adjoint ? (c * d + i) : (i * d + c);
        const double re = m[2 * src];
        const double im = adjoint ? -m[2 * src + 1] : m[2 * src + 1];
        return g == 0 ? re : g == 1 ? im : re + im;
    };
    const Path p = choose(dt, n, k, n_controls);
    if (p == Path::kMfmaC64K5 || p == Path::kTileC64K5) {
        // lane l = col + 32 half: 16 floats A_g[col][2j + half], j = 0..15
        float* o = static_cast<float*>(dst);
        for (int g = 0; g < 3; ++g)
            for (int l = 0; l < 64; ++l)
                for (int j = 0; j < 16; ++j) o[(g * 64 + l) * 16 + j] = float(A(g, l & 31, 2 * j + (l >> 5)));
        return;
    }
    if (p == Path::kMfmaC64K4 || p == Path::kTileC64K4) {
        // lane l = col + 16 q: 4 floats A_g[col][4s + q], s = 0..3
        float* o = static_cast<float*>(dst);
        for (int g = 0; g < 3; ++g)
            for (int l = 0; l < 64; ++l)
                for (int s4 = 0; s4 < 4; ++s4) o[(g * 64 + l) * 4 + s4] = float(A(g, l & 15, 4 * s4 + (l >> 4)));
        return;
    }
    if (p == Path::kTileC128K5) {
        // lane l = i0 + 16 q: 16 doubles A_g[i0 + 16 rt][4s + q], (rt, s)
        double* o = static_cast<double*>(dst);
        for (int g = 0; g < 3; ++g)
            for (int l = 0; l < 64; ++l)
                for (int rt = 0; rt < 2; ++rt)
                    for (int s8 = 0; s8 < 8; ++s8)
                        o[(g * 64 + l) * 16 + rt * 8 + s8] = A(g, (l & 15) + 16 * rt, 4 * s8 + (l >> 4));
        return;
    }
    if (p == Path::kTileC64K6) {
        // lane l = i + 32 half, row tile rt: 32 floats A_g[32 rt + i][2 s + half], s = 0..31
        float* o = static_cast<float*>(dst);
        for (int g = 0; g < 3; ++g)
            for (int rt = 0; rt < 2; ++rt)
                for (int l = 0; l < 64; ++l)
                    for (int s2 = 0; s2 < 32; ++s2)
                        o[((g * 2 + rt) * 64 + l) * 32 + s2] = float(A(g, 32 * rt + (l & 31), 2 * s2 + (l >> 5)));
        return;
    }
    if (p == Path::kTileC128K6) {
        // [g][rt][s][lane]: A_g[16 rt + i][4 s + q] at lane i + 16 q (g = Re, Im)
        double* o = static_cast<double*>(dst);
        for (int g = 0; g < 2; ++g)
            for (int rt = 0; rt < 4; ++rt)
                for (int s4 = 0; s4 < 16; ++s4)
                    for (int l = 0; l < 64; ++l)
                        o[((g * 4 + rt) * 16 + s4) * 64 + l] = A(g, 16 * rt + (l & 15), 4 * s4 + (l >> 4));
        return;
    }
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
            const double re = A(0, r, c), im = A(1, r, c);
            if (dt == SV_C64) {
                float* o = static_cast<float*>(dst);
                o[2 * (r * d + c)] = float(re);
                o[2 * (r * d + c) + 1] = float(im);
            } else {
                double* o = static_cast<double*>(dst);
                o[2 * (r * d + c)] = re;
                o[2 * (r * d + c) + 1] = im;
            }
        }
}

void launch_apply(sv_handle_s* h, sv_dtype_t dt, void* psi, const void* mat, const GateDesc& d)
{
    const Path p = choose(dt, d.n, d.k, d.n_controls);
    switch (p) {
        case Path::kMfmaC64K4:
        case Path::kMfmaC64K5:
            launch_mfma_c64(h, static_cast<float2*>(psi), static_cast<const float4*>(mat), d);
            break;
        case Path::kTileC64K4:
        case Path::kTileC64K5:
        case Path::kTileC128K5:
        case Path::kTileC64K6:
        case Path::kTileC128K6:
            launch_tile(h, p, psi, mat, d);
            break;
        default:
            if (dt == SV_C64)
                launch_apply_t<float>(h, psi, mat, d);
            else
                launch_apply_t<double>(h, psi, mat, d);
    }
}


// ------------------------------------------- generalized permutation gates

size_t gperm_table_bytes(sv_dtype_t dt, int k, bool has_perm)
{
    return (size_t(1) << k) * (dt == SV_C64 ? 8 : 16) + (has_perm ? (size_t(1) << k) * 4 : 0);
}

// Device table: diag' (2^k complex in the state's precision), then perm' (2^k
// int32) if has_perm, where (perm', diag') is G or, for adjoint, G^dagger =
// P^T D^*: output q of G^dagger takes input r = perm^-1(q) times conj(diag[r]).
void pack_gperm(sv_dtype_t dt, int k, const int64_t* perm, const double* diag, int adjoint, void* dst)
{
    const int d = 1 << k;
    std::vector<int32_t> p(d), src(d);
    for (int r = 0; r < d; ++r) p[r] = perm ? int32_t(perm[r]) : r;
    for (int r = 0; r < d; ++r) src[r] = r;
    if (adjoint)
        for (int r = 0; r < d; ++r) src[p[r]] = r;  // src = perm^-1
    char* o = static_cast<char*>(dst);
    for (int q = 0; q < d; ++q) {
        const int r = src[q];
        const double re = diag[2 * r], im = adjoint ? -diag[2 * r + 1] : diag[2 * r + 1];
        if (dt == SV_C64) {
            reinterpret_cast<float*>(o)[2 * q] = float(re);
            reinterpret_cast<float*>(o)[2 * q + 1] = float(im);
        } else {
            reinterpret_cast<double*>(o)[2 * q] = re;
            reinterpret_cast<double*>(o)[2 * q + 1] = im;
        }
    }
    if (perm) {
        int32_t* po = reinterpret_cast<int32_t*>(o + size_t(d) * (dt == SV_C64 ? 8 : 16));
        for (int q = 0; q < d; ++q) po[q] = adjoint ? src[q] : p[q];
    }
}

void launch_gperm(sv_handle_s* h, sv_dtype_t dt, void* psi, const void* table, const GateDesc& d, bool has_perm)
{
    const size_t tab_bytes = (size_t(1) << d.k) * (dt == SV_C64 ? 8 : 16);
    if (!has_perm) {
        DiagArgs a{};
        a.k = d.k;
        for (int b = 0; b < d.k; ++b) {
            int q = 0;
            while ((uint64_t(1) << q) != d.tbit[b]) ++q;
            a.tpos[b] = q;
        }
        uint64_t cmask = 0;
        for (int j = 0; j < d.n_fixed; ++j) {
            const uint64_t bit = uint64_t(1) << d.fixed_sorted[j];
            bool is_t = false;
            for (int b = 0; b < d.k; ++b) is_t |= d.tbit[b] == bit;
            if (!is_t) {
                a.cpos[a.n_ctrl++] = d.fixed_sorted[j];
                cmask |= bit;
            }
        }
        a.cval = d.cval;
        const uint64_t amps = uint64_t(1) << (d.n - a.n_ctrl);
        const bool narrow = dt == SV_C64 && ((cmask & 1) || d.n - a.n_ctrl < 1);
        const int apv = (dt == SV_C64 && !narrow) ? 2 : 1;
        a.n_vecs = amps / apv;
        const uint64_t per_block = uint64_t(kDiagThreads) * kDiagVecs;
        const uint64_t blocks = (a.n_vecs + per_block - 1) / per_block;
        SV_CHECK(blocks <= 0x7fffffffu, "state too large for one launch");
        if (dt == SV_C64) {
            if (narrow)
                hipLaunchKernelGGL((k_apply_diag<float, true>), dim3(unsigned(blocks)), dim3(kDiagThreads), 0, h->stream,
                                   static_cast<float2*>(psi), static_cast<const float2*>(table), a);
            else
                hipLaunchKernelGGL((k_apply_diag<float, false>), dim3(unsigned(blocks)), dim3(kDiagThreads), 0,
                                   h->stream, static_cast<float2*>(psi), static_cast<const float2*>(table), a);
        } else {
            hipLaunchKernelGGL((k_apply_diag<double, false>), dim3(unsigned(blocks)), dim3(kDiagThreads), 0, h->stream,
                               static_cast<double2*>(psi), static_cast<const double2*>(table), a);
        }
        SV_HIP(hipGetLastError());
        return;
    }
    SV_CHECK(d.n_controls == 0 && d.k <= 6, "a permutation takes at most 6 qubits, controls included");
    const int tb = dt == SV_C64 ? 12 : 11;
    SV_CHECK(d.n >= tb, "internal: small states take the dense path");
    TileArgs t = make_tile_args(d, d.n, tb, h->cu_count, 0, false);
    t.tiles_per_wg = 1;
    const char* tab = static_cast<const char*>(table);
    if (dt == SV_C64)
        hipLaunchKernelGGL(k_tile_gperm<float>, dim3(unsigned(t.n_tiles)), dim3(kTileThreads), 0, h->stream,
                           static_cast<float2*>(psi), reinterpret_cast<const float2*>(tab),
                           reinterpret_cast<const int32_t*>(tab + tab_bytes), t, d.k);
    else
        hipLaunchKernelGGL(k_tile_gperm<double>, dim3(unsigned(t.n_tiles)), dim3(kTileThreads), 0, h->stream,
                           static_cast<double2*>(psi), reinterpret_cast<const double2*>(tab),
                           reinterpret_cast<const int32_t*>(tab + tab_bytes), t, d.k);
    SV_HIP(hipGetLastError());
}

}  // namespace sv
