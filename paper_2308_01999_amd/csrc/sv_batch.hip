// Batched execution of many independent small circuits in one persistent
// launch (complex64).  Each workgroup takes circuits from a device queue
// (largest first) and runs a circuit's whole fused program, then its
// Z-type Pauli expectations:
//   - states of <= 12 qubits stay in LDS from |0..0> to the end, and are
//     written to HBM once;
//   - larger states are swept block by block through 4096-amplitude tiles
//     staged in LDS, the same tiling as the single-state sweep.
// k = 4, 5 blocks run as three real GEMMs on the matrix cores (Gauss's
// product), k <= 3 on the vector ALUs.  The workgroup records its
// circuit's completion on the device wall clock.  Every workgroup exits
// once the queue is empty; no workgroup waits on another.
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

// ---------------------------------------------------------- block kernels

// v_mfma_f32_32x32x2_f32: A[i][k] lane i + 32k, B[k][j] lane j + 32k,
// D[i][j] lane j + 32((i/4)%2), register 4(i/8) + i%4.
__device__ __forceinline__ void region_mfma5(float2* lds, const BatchBlock& b, const float* ar, const float* ai,
                                             const float* as)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, col = lane & 31, half = lane >> 5;
    const int groups = 1 << (b.L - b.n_lo);
    for (int ct = wave; ct * 32 < groups; ct += kThreads / 64) {
        const int gl = ct * 32 + col;
        const bool valid = gl < groups;
        const int pb = valid ? int(insert_zeros(uint64_t(gl), b.lo_pos, b.n_lo)) : 0;
        const int pin = pb + (half ? b.lds_off[1] : 0);
        const int pout = pb + (half ? b.lds_off[4] : 0);
        float2 x[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) x[j] = valid ? lds[pin + b.lds_off[2 * j]] : float2{0.f, 0.f};
        f32x16 p1 = {0}, p2 = {0}, p3 = {0};
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            p1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[j], x[j].x, p1, 0, 0, 0);
            p2 = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[j], x[j].y, p2, 0, 0, 0);
            p3 = __builtin_amdgcn_mfma_f32_32x32x2f32(as[j], x[j].x + x[j].y, p3, 0, 0, 0);
        }
        if (valid) {
#pragma unroll
            for (int r = 0; r < 16; ++r)
                lds[pout + b.lds_off[8 * (r / 4) + (r % 4)]] = float2{p1[r] - p2[r], p3[r] - p1[r] - p2[r]};
        }
    }
}

// v_mfma_f32_16x16x4_f32: A[i][k] lane i + 16k, B[k][j] lane j + 16k,
// D[i][j] lane j + 16(i/4), register i%4.
__device__ __forceinline__ void region_mfma4(float2* lds, const BatchBlock& b, const float* ar, const float* ai,
                                             const float* as)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, col = lane & 15, q = lane >> 4;
    const int groups = 1 << (b.L - b.n_lo);
    const int lin = ((q & 1) ? b.lds_off[1] : 0) + ((q & 2) ? b.lds_off[2] : 0);
    const int lout = ((q & 1) ? b.lds_off[4] : 0) + ((q & 2) ? b.lds_off[8] : 0);
    for (int ct = wave; ct * 16 < groups; ct += kThreads / 64) {
        const int gl = ct * 16 + col;
        const bool valid = gl < groups;
        const int pb = valid ? int(insert_zeros(uint64_t(gl), b.lo_pos, b.n_lo)) : 0;
        float2 x[4];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) x[s4] = valid ? lds[pb + lin + b.lds_off[4 * s4]] : float2{0.f, 0.f};
        f32x4 p1 = {0}, p2 = {0}, p3 = {0};
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            p1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[s4], x[s4].x, p1, 0, 0, 0);
            p2 = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[s4], x[s4].y, p2, 0, 0, 0);
            p3 = __builtin_amdgcn_mfma_f32_16x16x4f32(as[s4], x[s4].x + x[s4].y, p3, 0, 0, 0);
        }
        if (valid) {
#pragma unroll
            for (int r = 0; r < 4; ++r) lds[pb + lout + b.lds_off[r]] = float2{p1[r] - p2[r], p3[r] - p1[r] - p2[r]};
        }
    }
}

// k <= 3 on the vector ALUs: one group per thread per step; the matrix
// (complex64, row-major) is read with wave-uniform addresses.
template <int K>
__device__ __forceinline__ void region_valu(float2* lds, const BatchBlock& b, const float2* __restrict__ m)
{
    constexpr int D = 1 << K;
    const int groups = 1 << (b.L - b.n_lo);
    for (int gl = threadIdx.x; gl < groups; gl += kThreads) {
        // keeps the matrix loads inside the loop (hoisting all 2^(2K) entries
        // out of it would exhaust the scalar registers)
        asm volatile("" ::: "memory");
        const int pb = int(insert_zeros(uint64_t(gl), b.lo_pos, b.n_lo));
        float2 v[D];
#pragma unroll
        for (int c = 0; c < D; ++c) v[c] = lds[pb + b.lds_off[c]];
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
            lds[pb + b.lds_off[r]] = float2{re, im};
        }
    }
}

__device__ __forceinline__ void load_a(const float* __restrict__ mats, const BatchBlock& b, float* ar, float* ai,
                                       float* as)
{
    const int lane = threadIdx.x & 63;
    const float4* m4 = reinterpret_cast<const float4*>(mats + b.mat_off);
    if (b.k == 5) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float4 v = m4[(0 * 64 + lane) * 4 + q];
            ar[4 * q] = v.x; ar[4 * q + 1] = v.y; ar[4 * q + 2] = v.z; ar[4 * q + 3] = v.w;
            v = m4[(1 * 64 + lane) * 4 + q];
            ai[4 * q] = v.x; ai[4 * q + 1] = v.y; ai[4 * q + 2] = v.z; ai[4 * q + 3] = v.w;
            v = m4[(2 * 64 + lane) * 4 + q];
            as[4 * q] = v.x; as[4 * q + 1] = v.y; as[4 * q + 2] = v.z; as[4 * q + 3] = v.w;
        }
    } else if (b.k == 4) {
        float4 v = m4[0 * 64 + lane];
        ar[0] = v.x; ar[1] = v.y; ar[2] = v.z; ar[3] = v.w;
        v = m4[1 * 64 + lane];
        ai[0] = v.x; ai[1] = v.y; ai[2] = v.z; ai[3] = v.w;
        v = m4[2 * 64 + lane];
        as[0] = v.x; as[1] = v.y; as[2] = v.z; as[3] = v.w;
    }
}

// Applies block b to the region in LDS (A operands already in registers
// for k = 4, 5).  Callers synchronise before and after.
__device__ __forceinline__ void apply_region(float2* lds, const BatchBlock& b, const float* __restrict__ mats,
                                             const float* ar, const float* ai, const float* as)
{
    switch (b.k) {
        case 5: region_mfma5(lds, b, ar, ai, as); break;
        case 4: region_mfma4(lds, b, ar, ai, as); break;
        case 3: region_valu<3>(lds, b, reinterpret_cast<const float2*>(mats + b.mat_off)); break;
        case 2: region_valu<2>(lds, b, reinterpret_cast<const float2*>(mats + b.mat_off)); break;
        default: region_valu<1>(lds, b, reinterpret_cast<const float2*>(mats + b.mat_off)); break;
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

__device__ __forceinline__ void expectations(const float2* src, uint64_t dim, const uint64_t* __restrict__ zm,
                                             int n_terms, double* red, double* __restrict__ out)
{
    for (int t0 = 0; t0 < n_terms; t0 += kTermsPerPass) {
        double acc[kTermsPerPass + 1];
#pragma unroll
        for (int t = 0; t <= kTermsPerPass; ++t) acc[t] = 0.0;
        for (uint64_t i = threadIdx.x; i < dim; i += kThreads) {
            const double p = prob(src[i]);
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

__global__ __launch_bounds__(kThreads) void k_batch(BatchArgs A)
{
    __shared__ float2 lds[kRegion];
    __shared__ double red[kThreads];
    __shared__ uint32_t next;
    float2* states = static_cast<float2*>(A.states);
    float4* l4 = reinterpret_cast<float4*>(lds);
    if (threadIdx.x == 0) atomicMin(reinterpret_cast<unsigned long long*>(A.t_start),
                                    static_cast<unsigned long long>(wall_clock64()));
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(A.queue, 1u);
        __syncthreads();
        // uniform across the workgroup: descriptors below load as scalars
        const uint32_t slot = __builtin_amdgcn_readfirstlane(next);
        __syncthreads();
        if (slot >= A.n_circuits) break;
        const uint32_t ci = A.order[slot];
        const BatchCircuit c = A.circuits[ci];
        float2* psi = states + c.state_off;
        const uint64_t dim = uint64_t(1) << c.n;
        const bool resident = c.n <= 12;
        if (resident) {
            for (int i = threadIdx.x; i < int(dim); i += kThreads) lds[i] = float2{i == 0 ? 1.f : 0.f, 0.f};
        } else {
            float4* p4 = reinterpret_cast<float4*>(psi);
            for (uint64_t i = threadIdx.x; i < dim / 2; i += kThreads)
                p4[i] = float4{i == 0 ? 1.f : 0.f, 0.f, 0.f, 0.f};
        }
        // resident: one region (the state, kept in LDS); streaming: the
        // state's 4096-amplitude tiles, loaded and stored around each block
        const uint64_t n_regions = resident ? 1 : (dim >> 12);
        float ar[16], ai[16], as[16];
        for (uint32_t bi = 0; bi < c.n_blocks; ++bi) {
            __threadfence();
            __syncthreads();
            const BatchBlock& b = A.blocks[c.block0 + bi];
            load_a(A.mats, b, ar, ai, as);
            const int mask = (1 << b.L) - 1;
            uint64_t goff[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = (u * kThreads + int(threadIdx.x)) * 2;
                const uint32_t r = uint32_t(i >> b.L);
                uint64_t o = 0;
                for (int j = 0; j < b.n_hi; ++j) o |= uint64_t((r >> j) & 1u) << b.hi_pos[j];
                goff[u] = o + uint64_t(i & mask);
            }
            for (uint64_t t = 0; t < n_regions; ++t) {
                uint64_t base = 0;
                if (!resident) {
                    base = insert_zeros(t << b.L, b.hi_pos, b.n_hi);
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        l4[u * kThreads + threadIdx.x] = *reinterpret_cast<const float4*>(psi + base + goff[u]);
                    __syncthreads();
                }
                apply_region(lds, b, A.mats, ar, ai, as);
                __syncthreads();
                if (!resident) {
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        *reinterpret_cast<float4*>(psi + base + goff[u]) = l4[u * kThreads + threadIdx.x];
                    __syncthreads();
                }
            }
        }
        __threadfence();
        __syncthreads();
        if (resident) {
            for (int i = threadIdx.x; i < int(dim); i += kThreads) psi[i] = lds[i];
            expectations(lds, dim, A.z_masks + c.term0, int(c.n_terms), red, A.expect + c.term0);
        } else {
            expectations(psi, dim, A.z_masks + c.term0, int(c.n_terms), red, A.expect + c.term0);
        }
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) A.t_done[ci] = wall_clock64();
    }
}

__global__ void k_batch_reset(uint32_t* queue, uint64_t* t_start)
{
    *queue = 0;
    *t_start = ~uint64_t(0);
}

}  // namespace

void launch_batch_reset(hipStream_t stream, const BatchArgs& a)
{
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, stream, a.queue, a.t_start);
    SV_HIP(hipGetLastError());
}

void launch_batch(hipStream_t stream, int cu_count, const BatchArgs& a)
{
    // enough workgroups to fill the device; each exits when the queue is empty
    const unsigned blocks = unsigned(cu_count) * 4;
    hipLaunchKernelGGL(k_batch, dim3(blocks), dim3(kThreads), 0, stream, a);
    SV_HIP(hipGetLastError());
}

}  // namespace sv
