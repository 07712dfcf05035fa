// Tile geometry of the LDS-staged sweeps and the complex64 five-qubit tile
// transform, shared by the single-state sweep and the batched level sweep.
//
// A tile is 2^TB amplitudes (32 KiB) whose index bits outside {0..L-1} and
// the targets >= L are fixed: 2^n_hi contiguous runs of 2^L amplitudes, so
// every global access is a coalesced 16-byte load or store over runs of
// >= 1 KiB whatever the targets are, and each group's 2^k amplitudes are
// gathered in LDS.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "sv_internal.h"

namespace sv {

struct TileArgs {
    uint64_t n_tiles;
    uint64_t tiles_per_wg;
    int32_t L;
    int32_t n_hi;
    int32_t hi_pos[SV_MAX_TARGETS];
    int32_t n_lo;
    int32_t lo_pos[SV_MAX_TARGETS];
    int32_t lds_off[64];  // matrix index -> LDS offset from the group's base
    int32_t trot;         // tile order: tile index rotated right by trot bits over lg_tiles bits
    int32_t lg_tiles;     // log2 n_tiles
};

// Geometry of a tile sweep of the gate d on n qubits with 2^tb-amplitude
// tiles: spread_lo > 0 swaps each target below the run boundary for a free
// index bit from spread_lo up (the spread layout); strided makes workgroups
// take tiles far apart.  Host only.
TileArgs make_tile_args(const GateDesc& d, int n, int tb, int cu_count, int spread_lo, bool strided);

// Phase coupling of a block (coupled fusion): before the block's
// matrix, the amplitude at index i is multiplied by exp(i pi theta(i)),
// theta(i) = sum over the block's matrix bits a set in i of
// sum over the coupled qubits c set in i of phase[a][c] (in units of pi).
// A group's amplitudes share every bit outside the block, so per group
// theta is a sum of per-bit terms L_a: the amplitude at matrix column col
// gets exp(i pi sum_{a in col} L_a).
struct CoupleDev {
    int32_t n;                                     // coupled qubits
    int32_t k;                                     // the block's targets
    int32_t q[SV_MAX_QUBITS];                      // coupled index bits
    int32_t t[SV_MAX_TARGETS];                     // target index bits (matrix bit order)
    double phase[SV_MAX_TARGETS * SV_MAX_QUBITS];  // [a * SV_MAX_QUBITS + c], units of pi
};

namespace tile {

typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint64_t insert_zero_bits(uint64_t v, const int32_t* pos, int n)
{
    for (int j = 0; j < n; ++j) {
        const int p = pos[j];
        const uint64_t lo = v & ((uint64_t(1) << p) - 1);
        v = ((v >> p) << (p + 1)) | lo;
    }
    return v;
}

__device__ __forceinline__ uint64_t deposit_bits(uint32_t r, const int32_t* pos, int n)
{
    uint64_t o = 0;
    for (int b = 0; b < n; ++b) o |= uint64_t((r >> b) & 1u) << pos[b];
    return o;
}

constexpr int kTileThreads = 256;
constexpr int kTileVecs = 8;  // 16-byte vectors per thread per tile (32 KiB / 256 / 16)

#ifndef SV_TILE_NT
#define SV_TILE_NT 1
#endif
#ifndef SV_TILE_WGS_PER_CU
#define SV_TILE_WGS_PER_CU 32
#endif
#ifndef SV_TILES_PER_WG_MAX
#define SV_TILES_PER_WG_MAX 64
#endif
#ifndef SV_TILES_PER_WG_MAX_K5
#define SV_TILES_PER_WG_MAX_K5 4
#endif


typedef float nf4 __attribute__((ext_vector_type(4)));
typedef double nd2 __attribute__((ext_vector_type(2)));

template <typename V>
__device__ __forceinline__ V gload(const V* p)
{
    if (SV_TILE_NT) {
        if constexpr (sizeof(V) == 16 && std::is_same<V, float4>::value) {
            const nf4 v = __builtin_nontemporal_load(reinterpret_cast<const nf4*>(p));
            return V{v.x, v.y, v.z, v.w};
        } else {
            const nd2 v = __builtin_nontemporal_load(reinterpret_cast<const nd2*>(p));
            return V{v.x, v.y};
        }
    }
    return *p;
}

template <typename V>
__device__ __forceinline__ void gstore(V* p, const V v)
{
    if (SV_TILE_NT) {
        if constexpr (std::is_same<V, float4>::value) {
            __builtin_nontemporal_store(nf4{v.x, v.y, v.z, v.w}, reinterpret_cast<nf4*>(p));
        } else {
            __builtin_nontemporal_store(nd2{v.x, v.y}, reinterpret_cast<nd2*>(p));
        }
        return;
    }
    *p = v;
}

// The 8 per-thread vectors live in named registers (an array carried across
// the tile loop would be placed in scratch memory by the compiler).
#define SV_REP8(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7)

// Offsets (relative to a tile's base) of the thread's 8 vectors; vector u
// of thread tid holds tile-local amplitudes starting at
// i = (u * 256 + tid) * amps_per_vec, which is also its LDS position.  Its
// run index i >> L is the same for the whole wave (L >= 6 for complex128 and
// >= 7 for complex64, so the lane bits of tid stay below L), so the 64-bit
// run offset is a scalar and only the 32-bit offset inside the run is
// per lane.
template <int APV, int NT = kTileThreads>
__device__ __forceinline__ void tile_offsets(const TileArgs& a, uint64_t* roff, uint32_t* poff)
{
    const int mask = (1 << a.L) - 1;
#pragma unroll
    for (int u = 0; u < kTileVecs; ++u) {
        const int i = (u * NT + int(threadIdx.x)) * APV;
        const uint32_t r = uint32_t(__builtin_amdgcn_readfirstlane(i >> a.L));
        roff[u] = deposit_bits(r, a.hi_pos, a.n_hi);
        poff[u] = uint32_t(i & mask);
    }
}

// Global index of tile t's first amplitude.  With a.trot > 0 the tile index
// is first rotated right by trot bits: workgroup w, which sweeps its
// tiles_per_wg = 2^trot tiles t = w * 2^trot + j, then touches tiles
// w + j * (n_tiles / 2^trot), so at any moment the workgroups in flight work
// on neighbouring tiles instead of tiles 2^trot apart.
__device__ __forceinline__ uint64_t tile_base(uint64_t t, const TileArgs& a)
{
    if (a.trot > 0) t = ((t & ((uint64_t(1) << a.trot) - 1)) << (a.lg_tiles - a.trot)) | (t >> a.trot);
    return insert_zero_bits(t << a.L, a.hi_pos, a.n_hi);
}

// LDS slot of tile-local amplitude a: its low five bits are XORed with bits
// 5-9.  The gathers read, per instruction, the amplitudes of consecutive
// groups; when the low target bits spread those groups 2^m amplitudes apart
// (m <= 5), they would all map to one LDS bank without this.  Bijective on
// every aligned block of 1024 amplitudes, so it only permutes a tile.
__device__ __forceinline__ int lds_swz(int a) { return a ^ ((a >> 5) & 31); }

// complex64 staging moves pairs (i, i + 1), i even: both land in one aligned
// 16-byte slot, in swapped order when bit 0 of the XOR is set.
__device__ __forceinline__ int pair_slot(int i) { return i ^ ((i >> 5) & 30); }
__device__ __forceinline__ bool pair_swapped(int i) { return ((i >> 5) & 1) != 0; }
__device__ __forceinline__ float4 swap_pair(const float4 v, bool sw)
{
    return sw ? float4{v.z, v.w, v.x, v.y} : v;
}

// The three A operands (Re M, Im M, Re M + Im M) of the complex64 k = 5
// sweep, kept in LDS (44 KiB per workgroup with the tile: three per CU).
constexpr int kK5AParts = 3;
// Of those, the parts a sweep stages in LDS: Re M and Im M (Re M + Im M is
// formed as they are read), so that a 32 KiB tile and its operands take
// 40 KiB: four workgroups per CU.
constexpr int kK5AStaged = 2;


// Z-type expectation sums of the state a sweep leaves behind, taken from the
// tiles in LDS (no extra read of the state): for a workgroup, out[t] =
// sum over its amplitudes i of |psi_i|^2 (-1)^popcount(i & zm[t]) for
// t < n_terms, and out[n_terms] = sum |psi_i|^2, all FP64 in a fixed order
// (per thread by a Walsh-Hadamard transform, per wave by a butterfly, waves
// and tiles in order).  acc: LDS of 4 x (kZSumsMax + 1) doubles.
// n_terms < 0: no sums.
constexpr int kZSumsMax = 32;
struct ZSums {
    const uint64_t* zm;
    int n_terms;
    double* out;
    double* acc;
};

// A double's bits as two floats and back (for LDS that the sweep accesses as
// floats).
__device__ __forceinline__ float2 f64_as_f32x2(double d)
{
    const uint64_t b = uint64_t(__double_as_longlong(d));
    return float2{__uint_as_float(uint32_t(b)), __uint_as_float(uint32_t(b >> 32))};
}
__device__ __forceinline__ double f32x2_as_f64(float2 f)
{
    return __longlong_as_double(
        static_cast<long long>(uint64_t(__float_as_uint(f.x)) | (uint64_t(__float_as_uint(f.y)) << 32)));
}

// L_a (units of pi, reduced to [-1, 1]) of the group whose base index (block
// bits zero) is g.  Sums in a fixed order, exact selection of terms.
__device__ __forceinline__ void couple_terms(const CoupleDev* __restrict__ cp, uint64_t g, double* L)
{
#pragma unroll
    for (int a = 0; a < 5; ++a) L[a] = 0.0;
    const int n = cp->n;
    for (int c = 0; c < n; ++c) {
        const double b = double((g >> cp->q[c]) & 1);
#pragma unroll
        for (int a = 0; a < 5; ++a) L[a] = fma(b, cp->phase[a * SV_MAX_QUBITS + c], L[a]);
    }
#pragma unroll
    for (int a = 0; a < 5; ++a) L[a] -= 2.0 * rint(0.5 * L[a]);
}

__device__ __forceinline__ float2 cmulf(const float2 x, const float2 y)
{
    return float2{x.x * y.x - x.y * y.y, x.x * y.y + x.y * y.x};
}

__device__ __forceinline__ float2 cmulf_conj(const float2 x, const float2 y)
{
    return float2{x.x * y.x + x.y * y.y, x.y * y.x - x.x * y.y};
}

// complex64 pair (i, i + 1) of the state |0..0> starting at global index i// complex64 pair (i, i + 1) of the state |0..0> starting at global index i
__device__ __forceinline__ float4 basis0_pair(uint64_t i) { return i == 0 ? float4{1.f, 0.f, 0.f, 0.f} : float4{}; }

// The complex64 five-qubit tile sweep of workgroup `wg` (its tiles_per_wg
// tiles from wg * tiles_per_wg): a tile is staged in LDS, each wave gathers
// 32 groups of 32 amplitudes through the swizzle and multiplies them by the
// matrix as three real GEMMs on the matrix cores (Gauss's product: Re = A_0
// Re x - A_1 Im x, Im = A_2 (Re x + Im x) - A_0 Re x - A_1 Im x with A_0 =
// Re M, A_1 = Im M, A_2 = Re M + Im M), the next tile's loads in flight
// meanwhile.  mats: the packed A operands (3 x 64 lanes x 4 float4); lds:
// NT * kTileVecs float4 of LDS; amat: kK5AStaged * 64 * 4 float4 of LDS.
// FIRST: the input is the basis state |0..0>, which is not read.  COUPLED:
// the block's phase coupling cp multiplies each group's inputs first.
template <int NT, bool FIRST, bool COUPLED = false>
__device__ __forceinline__ void tile_c64_k5_sweep(float2* __restrict__ psi, const float4* __restrict__ mats,
                                                  const TileArgs& a, uint64_t wg, float4* lds, float4* amat,
                                                  const ZSums& zs, const CoupleDev* __restrict__ cp = nullptr)
{
    const uint64_t t0 = wg * a.tiles_per_wg;
    if (t0 >= a.n_tiles) return;
    const uint64_t t1 = (a.n_tiles - t0 < a.tiles_per_wg) ? a.n_tiles : t0 + a.tiles_per_wg;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, col = lane & 31, half = lane >> 5;
    // (from |0..0> only the workgroup with tile 0 multiplies; see below)
    if (!FIRST || t0 == 0)
        for (int e = tid; e < kK5AStaged * 64 * 4; e += NT) amat[e] = mats[e];
    if (zs.n_terms >= 0 && lane <= kZSumsMax) zs.acc[wave * (kZSumsMax + 1) + lane] = 0.0;
    uint64_t roff[kTileVecs];
    uint32_t poff[kTileVecs];
    tile_offsets<2, NT>(a, roff, poff);
    const int pb = int(insert_zero_bits(uint64_t(wave * 32 + col), a.lo_pos, a.n_lo));
    const int pin = pb + (half ? a.lds_off[1] : 0);
    const int pout = pb + (half ? a.lds_off[4] : 0);
    float2* lds2 = reinterpret_cast<float2*>(lds);
#define SV_DECL(u) float4 buf##u;
    SV_REP8(SV_DECL)
#undef SV_DECL
    uint64_t base = tile_base(t0, a);
#define SV_LOAD(u)                                                                              \
    buf##u = FIRST ? basis0_pair(base + roff[u] + poff[u])                                      \
                   : gload(reinterpret_cast<const float4*>(psi + base + roff[u] + poff[u]));
    SV_REP8(SV_LOAD)
#undef SV_LOAD
    for (uint64_t t = t0; t < t1; ++t) {
        if constexpr (FIRST) {
            // |0..0> is zero on every tile but tile 0 (the one holding index
            // 0), and so is the gate's image of it there: such a tile is
            // only written
            if (base != 0) {
#pragma unroll
                for (int u = 0; u < kTileVecs; ++u)
                    gstore(reinterpret_cast<float4*>(psi + base + roff[u] + poff[u]), float4{0.f, 0.f, 0.f, 0.f});
                if (t + 1 < t1) {
                    base = tile_base(t + 1, a);
#define SV_LOAD(u) buf##u = basis0_pair(base + roff[u] + poff[u]);
                    SV_REP8(SV_LOAD)
#undef SV_LOAD
                }
                continue;
            }
        }
#define SV_STAGE(u)                                                                        \
    {                                                                                      \
        const int i = (u * NT + tid) * 2;                                        \
        *reinterpret_cast<float4*>(lds2 + pair_slot(i)) = swap_pair(buf##u, pair_swapped(i)); \
    }
        SV_REP8(SV_STAGE)
#undef SV_STAGE
        __syncthreads();
        if constexpr (COUPLED) {
            // the phase coupling, in LDS on the 16 amplitudes this lane will
            // gather (so no barrier is needed), before the next tile's loads
            // are issued (fewer live registers): lane (col, half) owns columns 2j + half of its
            // group, whose tile-local base is pb.  The factors walk j in
            // Gray-code order, one multiplication (or division) per step.
            const uint64_t g = base + deposit_bits(uint32_t(pb >> a.L), a.hi_pos, a.n_hi) +
                               uint64_t(pb & ((1 << a.L) - 1));
            double L[5];
            couple_terms(cp, g, L);
            float2 e[5];
#pragma unroll
            for (int b = 0; b < 5; ++b) {
                float sn, cs;
                sincospif(float(L[b]), &sn, &cs);
                e[b] = float2{cs, sn};
            }
            float2 v = half ? e[0] : float2{1.f, 0.f};
            float2* y = &lds2[lds_swz(pin)];
            *y = cmulf(*y, v);
#pragma unroll
            for (int s = 1; s < 16; ++s) {
                const int j = s ^ (s >> 1), b = __builtin_ctz(s);
                v = ((j >> b) & 1) ? cmulf(v, e[b + 1]) : cmulf_conj(v, e[b + 1]);
                y = &lds2[lds_swz(pin + a.lds_off[2 * j])];
                *y = cmulf(*y, v);
            }
        }
        uint64_t nbase = 0;
        if (t + 1 < t1) {
            nbase = tile_base(t + 1, a);
#define SV_PREFETCH(u)                                                                          \
    buf##u = FIRST ? basis0_pair(nbase + roff[u] + poff[u])                                     \
                   : gload(reinterpret_cast<const float4*>(psi + nbase + roff[u] + poff[u]));
            SV_REP8(SV_PREFETCH)
#undef SV_PREFETCH
        }
        float2 x[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) x[j] = lds2[lds_swz(pin + a.lds_off[2 * j])];
        f32x16 p1 = {0}, p2 = {0}, p3 = {0};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 vr = amat[(0 * 64 + lane) * 4 + q];
            const float4 vi = amat[(1 * 64 + lane) * 4 + q];
            const float4 vs = float4{vr.x + vi.x, vr.y + vi.y, vr.z + vi.z, vr.w + vi.w};
            const float ar[4] = {vr.x, vr.y, vr.z, vr.w};
            const float ai[4] = {vi.x, vi.y, vi.z, vi.w};
            const float as[4] = {vs.x, vs.y, vs.z, vs.w};
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const float2 xv = x[4 * q + jj];
                p1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[jj], xv.x, p1, 0, 0, 0);
                p2 = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[jj], xv.y, p2, 0, 0, 0);
                p3 = __builtin_amdgcn_mfma_f32_32x32x2f32(as[jj], xv.x + xv.y, p3, 0, 0, 0);
            }
        }
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
        if (zs.n_terms >= 0) {
            // The tile is still in LDS.  A thread's 16 amplitudes differ in
            // the tile-local bits 0 and kUBit..kUBit+2 (amplitude j = e + 2u
            // is element e of vector u) and share all others, so a term's
            // sum over them is s * c[k]: c the Walsh-Hadamard transform of
            // their probabilities over j, c[k] = sum_j p_j (-1)^popcount(j & k),
            // k the term mask's bits at those four index bits, s its parity
            // over the bits the 16 share.  The norm is the term of mask 0.
            constexpr int kUBit = 1 + __builtin_ctz(NT);
            static_assert(kTileVecs == 8, "the transform spans one pair bit and three vector bits");
            double c[16];
#pragma unroll
            for (int u = 0; u < kTileVecs; ++u) {
                const int i = (u * NT + tid) * 2;
                const float4 v = swap_pair(*reinterpret_cast<const float4*>(lds2 + pair_slot(i)), pair_swapped(i));
                c[2 * u] = fma(double(v.x), double(v.x), __dmul_rn(double(v.y), double(v.y)));
                c[2 * u + 1] = fma(double(v.z), double(v.z), __dmul_rn(double(v.w), double(v.w)));
            }
#pragma unroll
            for (int h = 1; h < 16; h <<= 1) {
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    if (j & h) continue;
                    const double x = c[j], y = c[j | h];
                    c[j] = __dadd_rn(x, y);
                    c[j | h] = __dsub_rn(x, y);
                }
            }
            // the coefficients take the thread's own slots (its amplitudes
            // are read; no other thread reads these slots before the next
            // barrier): c[2u], c[2u + 1] in vector u's slot, their bits
            // moved as floats, the slots' type
#pragma unroll
            for (int u = 0; u < kTileVecs; ++u) {
                float2* slot = lds2 + pair_slot((u * NT + tid) * 2);
                slot[0] = f64_as_f32x2(c[2 * u]);
                slot[1] = f64_as_f32x2(c[2 * u + 1]);
            }
            // global index of the thread's amplitude j = 0, and the global
            // positions of the tile-local bits 0 and kUBit..kUBit+2
            const int mask = (1 << a.L) - 1;
            const uint64_t gt =
                base + deposit_bits(uint32_t((tid * 2) >> a.L), a.hi_pos, a.n_hi) + uint64_t((tid * 2) & mask);
            int jpos[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int b = q == 0 ? 0 : kUBit + q - 1;
                jpos[q] = b < a.L ? b : a.hi_pos[b - a.L];
            }
            // terms (the norm last, as term n_terms) in passes of eight; a
            // pass's wave sums by a reduce-scatter butterfly: after the
            // exchanges over lane bits 5, 4, 3 a lane holds one term, term
            // (lane >> 3) & 7 of the pass, summed over 8 lanes, and three
            // more exchanges sum the rest
            double* row = zs.acc + wave * (kZSumsMax + 1);
            const bool b5 = (lane & 32) != 0, b4 = (lane & 16) != 0, b3 = (lane & 8) != 0;
            for (int p0 = 0; p0 <= zs.n_terms; p0 += 8) {
                double v[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const int tt = p0 + t;
                    const uint64_t m = tt < zs.n_terms ? zs.zm[tt] : 0;
                    const int k = int((m >> jpos[0]) & 1) | int(((m >> jpos[1]) & 1) << 1) |
                                  int(((m >> jpos[2]) & 1) << 2) | int(((m >> jpos[3]) & 1) << 3);
                    const double x = f32x2_as_f64(lds2[pair_slot(((k >> 1) * NT + tid) * 2) + (k & 1)]);
                    v[t] = tt > zs.n_terms ? 0.0 : ((__popcll(gt & m) & 1) ? -x : x);
                }
                double w4[4];
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    w4[j] = __dadd_rn(b5 ? v[j + 4] : v[j], __shfl_xor(b5 ? v[j] : v[j + 4], 32, 64));
                double w2[2];
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    w2[j] = __dadd_rn(b4 ? w4[j + 2] : w4[j], __shfl_xor(b4 ? w4[j] : w4[j + 2], 16, 64));
                double w = __dadd_rn(b3 ? w2[1] : w2[0], __shfl_xor(b3 ? w2[0] : w2[1], 8, 64));
                w = __dadd_rn(w, __shfl_xor(w, 4, 64));
                w = __dadd_rn(w, __shfl_xor(w, 2, 64));
                w = __dadd_rn(w, __shfl_xor(w, 1, 64));
                const int tt = p0 + ((lane >> 3) & 7);
                if ((lane & 7) == 0 && tt <= zs.n_terms) {
                    const int r = tt == zs.n_terms ? kZSumsMax : tt;
                    row[r] = __dadd_rn(row[r], w);
                }
            }
        }
        base = nbase;
        __syncthreads();
    }
    if (zs.n_terms >= 0 && tid <= zs.n_terms) {
        // the waves' rows in order; the norm last
        const int c = tid == zs.n_terms ? kZSumsMax : tid;
        double v = 0.0;
        for (int w = 0; w < NT / 64; ++w) v = __dadd_rn(v, zs.acc[w * (kZSumsMax + 1) + c]);
        zs.out[tid] = v;
    }
}


}  // namespace tile
}  // namespace sv
