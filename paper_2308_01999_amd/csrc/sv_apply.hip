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

template <typename R>
void launch_apply_t(sv_handle_s* h, void* psi_v, const void* mat_v, const GateDesc& d)
{
    using T2 = typename Cx<R>::T;
    T2* psi = static_cast<T2*>(psi_v);
    const T2* mat = static_cast<const T2*>(mat_v);
    if (d.k <= kMaxUnrolledK) {
        ApplyArgs a{};
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

}  // namespace

void launch_apply(sv_handle_s* h, sv_dtype_t dt, void* psi, const void* mat, const GateDesc& d)
{
    if (dt == SV_C64)
        launch_apply_t<float>(h, psi, mat, d);
    else
        launch_apply_t<double>(h, psi, mat, d);
}

}  // namespace sv
