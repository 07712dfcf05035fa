// Batched execution of many independent circuits (complex64) in one
// recorded run.  Circuits below the level path's qubit count go to one
// persistent launch: each workgroup takes circuits from a device queue (in
// the order the host chose) and runs a circuit's whole fused program, then
// its Z-type Pauli expectations:
//   - states of <= 12 qubits stay in LDS from |0..0> to the end, and are
//     written to HBM once;
//   - larger states are swept block by block through 4096-amplitude tiles
//     staged in LDS, the same tiling as the single-state sweep.
// Larger circuits run on the level path: launch l applies block l of every
// such circuit that has one, each block through the single-state
// five-qubit tile sweep (many workgroups per state, so the streamed states
// move at the single-state sweep's rate), and a circuit's expectations are
// taken on a side stream right after its last level.
// k = 4, 5 blocks run as three real GEMMs on the matrix cores (Gauss's
// product), k <= 3 on the vector ALUs.  The workgroup records its
// circuit's completion on the device wall clock.  Every workgroup exits
// once the queue is empty; no workgroup waits on another.
//
// A workgroup reads back only what it wrote itself (its circuit's state),
// so the workgroup-scope fences of its barriers order all of its memory
// traffic; a device-scope fence would also write back and invalidate the
// L2 at every block.  Block descriptors and matrices are staged in LDS once
// per block, so that the tile loop's only vector-memory waits are those on
// the state's own tiles.
#include <hip/hip_runtime.h>

#include "sv_batch.h"

namespace sv {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kRegion = 4096;  // amplitudes in LDS (resident state or tile)

__device__ __forceinline__ uint64_t insert_zeros(uint64_t v, const int8_t* pos, int n)
{
    for (int j = 0; j < n; ++j) {
        const int p = pos[j];
        const uint64_t lo = v & ((uint64_t(1) << p) - 1);
        v = ((v >> p) << (p + 1)) | lo;
    }
    return v;
}

// LDS slot of region amplitude a: its low five bits XOR bits 5-9, so that
// the group gathers (consecutive groups 2^m amplitudes apart when the low
// bits are targets) spread over the LDS banks.  Bijective on aligned blocks
// of 1024 amplitudes and the identity below 32, so a resident state of any
// size stays inside its own 2^n slots.
__device__ __forceinline__ int swz(int a) { return a ^ ((a >> 5) & 31); }

// Block descriptor fields as wave-uniform scalars, read once per region
// (re-reading them from memory inside the lanes' loops would put a memory
// wait in front of every gather).
struct RegionGeom {
    int n_lo;
    int lo_pos[kBatchMaxK];
    int off[32];
};

__device__ __forceinline__ void region_geom(const BatchBlock& b, int n_off, RegionGeom& g)
{
    g.n_lo = __builtin_amdgcn_readfirstlane(b.n_lo);
#pragma unroll
    for (int j = 0; j < kBatchMaxK; ++j) g.lo_pos[j] = __builtin_amdgcn_readfirstlane(b.lo_pos[j]);
#pragma unroll
    for (int j = 0; j < 32; ++j) g.off[j] = j < n_off ? __builtin_amdgcn_readfirstlane(int(b.lds_off[j])) : 0;
}

// v with zeros inserted at the region's low target positions
__device__ __forceinline__ int spread_lo(int v, const RegionGeom& g)
{
#pragma unroll
    for (int j = 0; j < kBatchMaxK; ++j) {
        if (j < g.n_lo) {
            const int p = g.lo_pos[j];
            v = ((v >> p) << (p + 1)) | (v & ((1 << p) - 1));
        }
    }
    return v;
}

// LDS operand block for k = 4, 5: Re M, Im M, Re M + Im M in the per-lane
// order of the MFMA A operand (k = 5: 4 float4 per lane each; k = 4: 1).
constexpr int kAmat = 3 * 64 * 4;

// ---------------------------------------------------------- block kernels

// v_mfma_f32_32x32x2_f32: A[i][k] lane i + 32k, B[k][j] lane j + 32k,
// D[i][j] lane j + 32((i/4)%2), register 4(i/8) + i%4.
__device__ __forceinline__ void region_mfma5(float2* lds, const BatchBlock& b, const float4* amat)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, col = lane & 31, half = lane >> 5;
    RegionGeom g;
    region_geom(b, 32, g);
    const int groups = 1 << (__builtin_amdgcn_readfirstlane(b.L) - g.n_lo);
    for (int ct = wave; ct * 32 < groups; ct += kThreads / 64) {
        const int gl = ct * 32 + col;
        const bool valid = gl < groups;
        // lanes past the last group read group 0 and feed zeros
        const int pb = spread_lo(valid ? gl : 0, g);
        const int pin = pb + (half ? g.off[1] : 0);
        const int pout = pb + (half ? g.off[4] : 0);
        f32x16 p1 = {0}, p2 = {0}, p3 = {0};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            // one quarter of the B operands live at a time (the compiler
            // would otherwise load all 16 up front, 32 more registers)
            asm volatile("" ::: "memory");
            float2 x[4];
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const float2 v = lds[swz(pin + g.off[2 * (4 * q + jj)])];
                x[jj] = valid ? v : float2{0.f, 0.f};
            }
            const float4 vr = amat[(0 * 64 + lane) * 4 + q];
            const float4 vi = amat[(1 * 64 + lane) * 4 + q];
            const float4 vs = amat[(2 * 64 + lane) * 4 + q];
            const float ar[4] = {vr.x, vr.y, vr.z, vr.w};
            const float ai[4] = {vi.x, vi.y, vi.z, vi.w};
            const float as[4] = {vs.x, vs.y, vs.z, vs.w};
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const float2 xv = x[jj];
                p1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[jj], xv.x, p1, 0, 0, 0);
                p2 = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[jj], xv.y, p2, 0, 0, 0);
                p3 = __builtin_amdgcn_mfma_f32_32x32x2f32(as[jj], xv.x + xv.y, p3, 0, 0, 0);
            }
        }
        if (valid) {
#pragma unroll
            for (int r = 0; r < 16; ++r)
                lds[swz(pout + g.off[8 * (r / 4) + (r % 4)])] = float2{p1[r] - p2[r], p3[r] - p1[r] - p2[r]};
        }
    }
}

// v_mfma_f32_16x16x4_f32: A[i][k] lane i + 16k, B[k][j] lane j + 16k,
// D[i][j] lane j + 16(i/4), register i%4.
__device__ __forceinline__ void region_mfma4(float2* lds, const BatchBlock& b, const float4* amat)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, col = lane & 15, q = lane >> 4;
    const float4 vr = amat[0 * 64 + lane], vi = amat[1 * 64 + lane], vs = amat[2 * 64 + lane];
    const float ar[4] = {vr.x, vr.y, vr.z, vr.w};
    const float ai[4] = {vi.x, vi.y, vi.z, vi.w};
    const float as[4] = {vs.x, vs.y, vs.z, vs.w};
    RegionGeom g;
    region_geom(b, 16, g);
    const int groups = 1 << (__builtin_amdgcn_readfirstlane(b.L) - g.n_lo);
    const int lin = ((q & 1) ? g.off[1] : 0) + ((q & 2) ? g.off[2] : 0);
    const int lout = ((q & 1) ? g.off[4] : 0) + ((q & 2) ? g.off[8] : 0);
    for (int ct = wave; ct * 16 < groups; ct += kThreads / 64) {
        const int gl = ct * 16 + col;
        const bool valid = gl < groups;
        const int pb = spread_lo(valid ? gl : 0, g);
        float2 x[4];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const float2 v = lds[swz(pb + lin + g.off[4 * s4])];
            x[s4] = valid ? v : float2{0.f, 0.f};
        }
        f32x4 p1 = {0}, p2 = {0}, p3 = {0};
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            p1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[s4], x[s4].x, p1, 0, 0, 0);
            p2 = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[s4], x[s4].y, p2, 0, 0, 0);
            p3 = __builtin_amdgcn_mfma_f32_16x16x4f32(as[s4], x[s4].x + x[s4].y, p3, 0, 0, 0);
        }
        if (valid) {
#pragma unroll
            for (int r = 0; r < 4; ++r) lds[swz(pb + lout + g.off[r])] = float2{p1[r] - p2[r], p3[r] - p1[r] - p2[r]};
        }
    }
}

// k <= 3 on the vector ALUs: one group per thread per step; the matrix
// (complex64, row-major) is read with wave-uniform addresses.
template <int K>
__device__ __forceinline__ void region_valu(float2* lds, const BatchBlock& b, const float2* __restrict__ m)
{
    constexpr int D = 1 << K;
    RegionGeom g;
    region_geom(b, D, g);
    const int groups = 1 << (__builtin_amdgcn_readfirstlane(b.L) - g.n_lo);
    for (int gl = threadIdx.x; gl < groups; gl += kThreads) {
        // keeps the matrix loads inside the loop (hoisting all 2^(2K) entries
        // out of it would exhaust the scalar registers)
        asm volatile("" ::: "memory");
        const int pb = spread_lo(gl, g);
        float2 v[D];
#pragma unroll
        for (int c = 0; c < D; ++c) v[c] = lds[swz(pb + g.off[c])];
#pragma unroll
        for (int r = 0; r < D; ++r) {
            float re = 0.f, im = 0.f;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                const float2 e = m[r * D + c];
                re = fmaf(e.x, v[c].x, re);
                re = fmaf(-e.y, v[c].y, re);
                im = fmaf(e.x, v[c].y, im);
                im = fmaf(e.y, v[c].x, im);
            }
            lds[swz(pb + g.off[r])] = float2{re, im};
        }
    }
}

// Copies block b's matrix to LDS: the packed A operands for k = 4, 5, the
// complex64 matrix for k <= 3.  The caller synchronises before it is read.
__device__ __forceinline__ void stage_matrix(const float* __restrict__ mats, const BatchBlock& b, float4* amat)
{
    const int k = __builtin_amdgcn_readfirstlane(b.k);
    if (k >= 4) {
        const float4* m4 = reinterpret_cast<const float4*>(mats + b.mat_off);
        const int n4 = k == 5 ? kAmat : 3 * 64;
        for (int e = threadIdx.x; e < n4; e += kThreads) amat[e] = m4[e];
    } else {
        const float2* m2 = reinterpret_cast<const float2*>(mats + b.mat_off);
        float2* d2 = reinterpret_cast<float2*>(amat);
        for (int e = threadIdx.x; e < (1 << (2 * k)); e += kThreads) d2[e] = m2[e];
    }
}

// Applies block b to the region in LDS (descriptor and matrix already
// staged in LDS).  Callers synchronise before and after.
__device__ __forceinline__ void apply_region(float2* lds, const BatchBlock& b, const float4* amat)
{
    const float2* m2 = reinterpret_cast<const float2*>(amat);
    switch (__builtin_amdgcn_readfirstlane(b.k)) {
        case 5: region_mfma5(lds, b, amat); break;
        case 4: region_mfma4(lds, b, amat); break;
        case 3: region_valu<3>(lds, b, m2); break;
        case 2: region_valu<2>(lds, b, m2); break;
        default: region_valu<1>(lds, b, m2); break;
    }
}

// Fixed-shape tree over the block; result valid in every thread.
__device__ __forceinline__ double block_sum(double v, double* red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (int(threadIdx.x) < s) red[threadIdx.x] = __dadd_rn(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double prob(const float2 a)
{
    const double re = double(a.x), im = double(a.y);
    return fma(re, re, __dmul_rn(im, im));
}

// Z-type expectations over a state held in LDS or in HBM; FP64, fixed
// per-thread order and fixed tree.  Terms go in passes of kTermsPerPass;
// every pass also sums the norm (identically), and each result is divided
// by it.
constexpr int kTermsPerPass = 8;

template <bool kInLds>
__device__ __forceinline__ void expectations(const float2* src, uint64_t dim, const uint64_t* __restrict__ zm,
                                             int n_terms, double* red, double* __restrict__ out)
{
    for (int t0 = 0; t0 < n_terms; t0 += kTermsPerPass) {
        double acc[kTermsPerPass + 1];
#pragma unroll
        for (int t = 0; t <= kTermsPerPass; ++t) acc[t] = 0.0;
        for (uint64_t i = threadIdx.x; i < dim; i += kThreads) {
            const double p = prob(src[kInLds ? uint64_t(swz(int(i))) : i]);
            acc[kTermsPerPass] = __dadd_rn(acc[kTermsPerPass], p);
#pragma unroll
            for (int t = 0; t < kTermsPerPass; ++t)
                if (t0 + t < n_terms) acc[t] = __dadd_rn(acc[t], (__popcll(i & zm[t0 + t]) & 1) ? -p : p);
        }
        const double nrm = block_sum(acc[kTermsPerPass], red);
#pragma unroll
        for (int t = 0; t < kTermsPerPass; ++t) {
            if (t0 + t < n_terms) {
                const double s = block_sum(acc[t], red);
                if (threadIdx.x == 0) out[t0 + t] = s / nrm;
            }
        }
    }
}

// complex64 pairs (i, i + 1), i even, move as one 16-byte slot; the slot's
// two halves are swapped when bit 0 of the XOR is set
__device__ __forceinline__ int pair_slot(int i) { return i ^ ((i >> 5) & 30); }
__device__ __forceinline__ float4 swap_pair(const float4 v, int i)
{
    return ((i >> 5) & 1) ? float4{v.z, v.w, v.x, v.y} : v;
}

#define SV_REP8(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7)

__global__ __launch_bounds__(kThreads) void k_batch(BatchArgs A)
{
    __shared__ float2 lds[kRegion];
    __shared__ float4 amat[kAmat];
    __shared__ BatchBlock blk;
    static_assert(sizeof(BatchBlock) % 4 == 0, "the block descriptor is copied as words");
    __shared__ double red[kThreads];
    __shared__ uint32_t next;
    float2* states = static_cast<float2*>(A.states);
    const int tid = threadIdx.x;
    if (tid == 0) {
        next = atomicAdd(A.queue, 1u);
    }
    __syncthreads();
    // uniform across the workgroup: descriptors below load as scalars.  The
    // queue is read again only at the bottom of the loop, so the loop's one
    // exit is this uniform test (a thread-0 branch at the top of the loop
    // let the compiler give thread 0 a loop of its own around the barriers)
    uint32_t slot = __builtin_amdgcn_readfirstlane(next);
    __syncthreads();
    while (slot < A.n_queue) {
        const uint32_t ci = A.order[slot];
        const BatchCircuit c = A.circuits[ci];
        float2* psi = states + c.state_off;
        const uint64_t dim = uint64_t(1) << c.n;
        const bool resident = c.n <= 12;
        // |0..0> (slot 0 is amplitude 0 under the swizzle)
        if (resident) {
            for (int i = tid; i < int(dim); i += kThreads) lds[i] = float2{i == 0 ? 1.f : 0.f, 0.f};
        } else {
            float4* p4 = reinterpret_cast<float4*>(psi);
            for (uint64_t i = tid; i < dim / 2; i += kThreads) p4[i] = float4{i == 0 ? 1.f : 0.f, 0.f, 0.f, 0.f};
        }
        // resident: one region (the state, kept in LDS); streaming: the
        // state's 4096-amplitude tiles, loaded and stored around each block,
        // the next tile's loads in flight while one is transformed
        const uint64_t n_regions = resident ? 1 : (dim >> 12);
        for (uint32_t bi = 0; bi < c.n_blocks; ++bi) {
            __syncthreads();
            // the block's descriptor and matrix are staged in LDS once: the
            // tile loop then reads no global memory but the state, and a wait
            // for a descriptor load (vector loads complete in order) cannot
            // also wait for the tiles prefetched before it
            if (tid < int(sizeof(BatchBlock) / 4))
                reinterpret_cast<uint32_t*>(&blk)[tid] =
                    reinterpret_cast<const uint32_t*>(A.blocks + c.block0 + bi)[tid];
            __syncthreads();
            const BatchBlock& b = blk;
            stage_matrix(A.mats, b, amat);
            // streaming tiles: run index i >> L of the thread's vector u and
            // the offset inside the run (unused for a resident state)
            uint32_t goff[8];
            const int mask = (1 << b.L) - 1;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = (u * kThreads + tid) * 2;
                const uint32_t r = uint32_t(i >> b.L);
                uint32_t o = 0;
                for (int j = 0; j < b.n_hi; ++j) o |= ((r >> j) & 1u) << b.hi_pos[j];
                goff[u] = o + uint32_t(i & mask);
            }
#define SV_DECL(u) float4 buf##u = {};
            SV_REP8(SV_DECL)
#undef SV_DECL
#define SV_LOAD(u) buf##u = *reinterpret_cast<const float4*>(psi + base + goff[u]);
            uint64_t base = 0;
            if (!resident) {
                base = insert_zeros(0, b.hi_pos, b.n_hi);
                SV_REP8(SV_LOAD)
            }
            // one apply site for both kinds of state
            for (uint64_t t = 0; t < n_regions; ++t) {
                const uint64_t cur = base;
                if (!resident) {
#define SV_STAGE(u)                                                                       \
    {                                                                                     \
        const int i = (u * kThreads + tid) * 2;                                           \
        *reinterpret_cast<float4*>(lds + pair_slot(i)) = swap_pair(buf##u, i);            \
    }
                    SV_REP8(SV_STAGE)
#undef SV_STAGE
                }
                __syncthreads();
                if (!resident && t + 1 < n_regions) {
                    base = insert_zeros((t + 1) << b.L, b.hi_pos, b.n_hi);
                    SV_REP8(SV_LOAD)
                }
                apply_region(lds, b, amat);
                __syncthreads();
                if (!resident) {
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int i = (u * kThreads + tid) * 2;
                        *reinterpret_cast<float4*>(psi + cur + goff[u]) =
                            swap_pair(*reinterpret_cast<const float4*>(lds + pair_slot(i)), i);
                    }
                    __syncthreads();
                }
            }
#undef SV_LOAD
        }
        __syncthreads();
        if (resident) {
            for (int i = tid; i < int(dim); i += kThreads) psi[i] = lds[swz(i)];
            expectations<true>(lds, dim, A.z_masks + c.term0, int(c.n_terms), red, A.expect + c.term0);
        } else {
            expectations<false>(psi, dim, A.z_masks + c.term0, int(c.n_terms), red, A.expect + c.term0);
        }
        __syncthreads();
        if (tid == 0) {
            A.t_done[ci] = wall_clock64();
            next = atomicAdd(A.queue, 1u);
        }
        __syncthreads();
        slot = __builtin_amdgcn_readfirstlane(next);
        __syncthreads();
    }
}

__global__ void k_batch_reset(uint32_t* queue, uint64_t* t_start)
{
    *queue = 0;
    *t_start = wall_clock64();
}

// Level path: workgroup w sweeps its tiles of one block of one circuit; on a
// circuit's last block it also leaves the Z-type sums of its tiles.
template <bool FIRST>
__global__ __launch_bounds__(tile::kTileThreads, 3) void k_batch_level(float2* __restrict__ states,
                                                                    const BatchTileDesc* __restrict__ descs,
                                                                    const BatchLevelEntry* __restrict__ entries,
                                                                    const float4* __restrict__ mats,
                                                                    const uint64_t* __restrict__ z_masks,
                                                                    double* __restrict__ partials)
{
    __shared__ float4 lds[tile::kTileThreads * tile::kTileVecs];
    __shared__ float4 amat[tile::kK5AStaged * 64 * 4];
    __shared__ double zacc[(tile::kTileThreads / 64) * (tile::kZSumsMax + 1)];
    const BatchLevelEntry e = entries[blockIdx.x];
    const BatchTileDesc& d = descs[e.desc];
    const tile::ZSums zs{z_masks + d.term0, d.n_terms,
                         partials + d.red_off + uint64_t(e.wg) * uint64_t(d.n_terms + 1), zacc};
    tile::tile_c64_k5_sweep<tile::kTileThreads, FIRST>(states + d.state_off, mats + d.mat_off, d.t, e.wg, lds,
                                                       amat, zs);
}

// Level path: a finished circuit's expectations from its workgroups' sums,
// then its completion time.  Thread (g, c) of G = kThreads / S groups of S =
// n_terms + 1 columns (the norm last) adds the rows g, g + G, ... of column
// c; the groups' sums are then added in group order: a fixed order for a
// given workgroup count.
__global__ __launch_bounds__(kThreads) void k_batch_finish(BatchArgs A, const BatchFinish* __restrict__ fin)
{
    __shared__ double part[kThreads];
    __shared__ double nrm;
    const BatchFinish f = fin[blockIdx.x];
    const BatchCircuit c = A.circuits[f.circuit];
    const int nt = int(c.n_terms), S = nt + 1, G = kThreads / S;
    const int tid = int(threadIdx.x), g = tid / S, col = tid - g * S;
    double v = 0.0;
    if (g < G) {
        const double* p = A.partials + f.red_off + col;
#pragma unroll 4
        for (uint32_t w = uint32_t(g); w < f.n_wg; w += uint32_t(G)) v = __dadd_rn(v, p[uint64_t(w) * S]);
    }
    part[tid] = v;
    __syncthreads();
    if (tid < S) {
        double s = 0.0;
        for (int q = 0; q < G; ++q) s = __dadd_rn(s, part[q * S + tid]);
        v = s;
        if (tid == nt) nrm = s;
    }
    __syncthreads();
    if (tid < nt) A.expect[c.term0 + tid] = v / nrm;
    __syncthreads();
    if (tid == 0) A.t_done[f.circuit] = wall_clock64();
}

}  // namespace

void launch_batch_reset(hipStream_t stream, const BatchArgs& a)
{
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, stream, a.queue, a.t_start);
    SV_HIP(hipGetLastError());
}

void launch_batch_level(hipStream_t stream, const BatchArgs& a, uint64_t first, uint32_t n_entries, bool first_level)
{
    float2* states = static_cast<float2*>(a.states);
    if (first_level)
        hipLaunchKernelGGL(k_batch_level<true>, dim3(n_entries), dim3(tile::kTileThreads), 0, stream, states, a.tdescs,
                           a.entries + first, a.tmats, a.z_masks, a.partials);
    else
        hipLaunchKernelGGL(k_batch_level<false>, dim3(n_entries), dim3(tile::kTileThreads), 0, stream, states,
                           a.tdescs, a.entries + first, a.tmats, a.z_masks, a.partials);
    SV_HIP(hipGetLastError());
}

void launch_batch_finish(hipStream_t stream, const BatchArgs& a, uint64_t first, uint32_t n)
{
    hipLaunchKernelGGL(k_batch_finish, dim3(n), dim3(kThreads), 0, stream, a, a.finish + first);
    SV_HIP(hipGetLastError());
}

void launch_batch(hipStream_t stream, int cu_count, const BatchArgs& a)
{
    // as many workgroups as fit on the device at once; each exits when the
    // queue is empty
    int per_cu = 0;
    SV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch, kThreads, 0));
    if (per_cu < 1) per_cu = 1;
    const unsigned blocks = unsigned(cu_count) * unsigned(per_cu);
    hipLaunchKernelGGL(k_batch, dim3(blocks), dim3(kThreads), 0, stream, a);
    SV_HIP(hipGetLastError());
}

}  // namespace sv
