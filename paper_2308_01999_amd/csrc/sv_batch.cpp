// Host side of the batched path: fuses every circuit of a batch (in
// parallel host threads), chooses the fusion width per qubit count (fixed,
// or measured by the autotuner), lays out the states, packs block
// descriptors and matrices, uploads them once, and runs the persistent batch
// kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "sv_batch.h"
#include "sv_tune_cache.h"

namespace sv {

sv_fused_s* fuse_gate_list(const int32_t* codes, const int32_t* qubits, const double* params, int n_gates,
                           int kmax, int kdiag, bool coupled = false);

// One level of the level path: its workgroup entries and the circuits whose
// expectations follow it.
struct BatchLevel {
    uint64_t entry0 = 0;
    uint32_t n_entries = 0;
    uint64_t finish0 = 0;
    uint32_t n_finish = 0;
};

// Level-path tile shape of one qubit count.
struct LevelShape {
    int tiles_per_wg = 4;  // tiles per workgroup, taken in strided order
    int spread = 1;        // 1: spread tile layout, 0: plain
};

// How a batch runs the circuits of one qubit count.
struct SizePlan {
    int kmax = kBatchMaxK;  // fusion width on the persistent kernel
    bool level = false;     // true: the level path (fused at min(5, n))
    LevelShape shape;       // the level path's tile shape
    bool tuned = false;     // chosen by the autotuner (measured or from its cache)
};

struct BatchHost {
    std::vector<BatchCircuit> circuits;
    std::vector<uint32_t> order;  // the persistent kernel's queue
    std::vector<BatchBlock> blocks;
    std::vector<float> mats;
    std::vector<uint64_t> z_masks;
    uint64_t state_amps = 0;
    // level path
    std::vector<BatchTileDesc> tdescs;
    std::vector<float4> tmats;
    std::vector<BatchLevelEntry> entries;
    std::vector<BatchFinish> finish;
    std::vector<BatchLevel> levels;
    uint64_t n_partials = 0;
};

}  // namespace sv

struct sv_batch_s {
    sv_handle_s* h = nullptr;
    int n_circuits = 0;
    int total_terms = 0;
    std::vector<int> n;
    std::vector<uint64_t> state_off;  // amplitudes
    uint64_t state_amps = 0;
    std::map<int, sv::SizePlan> plans;  // per qubit count
    double tune_s = 0.0;                // host time in the autotuner
    double build_s = 0.0;               // host time fusing, packing and uploading the batch
    std::vector<sv::BatchLevel> levels;
    std::vector<int> blocks_per_circuit;
    char* dev = nullptr;  // one arena for all device-side descriptors
    size_t dev_bytes = 0;
    sv::BatchArgs args{};
    double tick_hz = 1e8;
    // the run (queue reset + persistent kernel), recorded once per states
    // buffer into a HIP graph and replayed by every later run
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void* graph_states = nullptr;
};

namespace sv {
namespace {

// Region geometry of a block with sorted targets tq on n qubits: the whole
// state when n <= 12, else a 4096-amplitude tile.
void block_geometry(BatchBlock& b, const int* tq, int k, int n)
{
    b.k = k;
    int L;
    if (n <= 12) {
        L = n;
    } else {
        const int gbits = 12 - k;
        L = gbits;
        for (;;) {
            int klo = 0;
            for (int a = 0; a < k; ++a) klo += tq[a] < L;
            if (L - klo >= gbits) break;
            ++L;
        }
    }
    b.L = L;
    int nh = 0, nl = 0;
    int hi[8], lo[8];
    for (int a = 0; a < k; ++a) {
        if (tq[a] < L)
            lo[nl++] = tq[a];
        else
            hi[nh++] = tq[a];
    }
    b.n_hi = nh;
    b.n_lo = nl;
    for (int j = 0; j < 8; ++j) {
        b.hi_pos[j] = int8_t(j < nh ? hi[j] : 0);
        b.lo_pos[j] = int8_t(j < nl ? lo[j] : 0);
    }
    for (int c = 0; c < 32; ++c) {
        if (c >= (1 << k)) {
            b.lds_off[c] = 0;
            continue;
        }
        int run = 0, low = 0;
        for (int a = 0; a < k; ++a) {
            if (!((c >> a) & 1)) continue;
            if (tq[a] < L) {
                low |= 1 << tq[a];
            } else {
                int rank = 0;
                while (hi[rank] != tq[a]) ++rank;
                run |= 1 << rank;
            }
        }
        b.lds_off[c] = int16_t((run << L) + low);
    }
}

// Packs block matrix m (complex128, row-major, 2^k x 2^k) for the batch
// kernel: the per-lane A-operand layout of the matrix-core path for k = 4,
// 5, plain complex64 for k <= 3.  Returns the number of floats appended.
size_t pack_batch_matrix(const double* m, int k, std::vector<float>& out)
{
    const int d = 1 << k;
    auto A = [&](int g, int i, int c) {
        const double re = m[2 * (i * d + c)], im = m[2 * (i * d + c) + 1];
        return float(g == 0 ? re : g == 1 ? im : re + im);
    };
    const size_t start = out.size();
    if (k == 5) {
        for (int g = 0; g < 3; ++g)
            for (int l = 0; l < 64; ++l)
                for (int j = 0; j < 16; ++j) out.push_back(A(g, l & 31, 2 * j + (l >> 5)));
    } else if (k == 4) {
        for (int g = 0; g < 3; ++g)
            for (int l = 0; l < 64; ++l)
                for (int s4 = 0; s4 < 4; ++s4) out.push_back(A(g, l & 15, 4 * s4 + (l >> 4)));
    } else {
        for (int e = 0; e < d * d; ++e) {
            out.push_back(float(m[2 * e]));
            out.push_back(float(m[2 * e + 1]));
        }
    }
    while (out.size() % 4) out.push_back(0.f);  // keep 16-byte alignment
    return out.size() - start;
}

struct CircuitInput {
    int n;
    const int32_t* codes;
    const int32_t* qubits;
    const double* params;
    int n_gates;
};

// Fuses all circuits with the given per-circuit widths on host threads.
std::vector<sv_fused_s*> fuse_all(const std::vector<CircuitInput>& in, const std::vector<int>& kmax)
{
    std::vector<sv_fused_s*> out(in.size(), nullptr);
    std::atomic<size_t> next{0};
    std::mutex err_mu;
    std::string err;
    sv_status_t err_status = SV_OK;
    unsigned nt = std::thread::hardware_concurrency();
    if (nt == 0) nt = 4;
    nt = std::min<unsigned>(nt, 16);
    auto work = [&] {
        for (;;) {
            const size_t i = next.fetch_add(1);
            if (i >= in.size()) return;
            try {
                out[i] = fuse_gate_list(in[i].codes, in[i].qubits, in[i].params, in[i].n_gates, kmax[i], 0);
            } catch (const Error& e) {
                std::lock_guard<std::mutex> g(err_mu);
                if (err.empty()) {
                    err = "circuit " + std::to_string(i) + ": " + e.msg;
                    err_status = e.status;
                }
            }
        }
    };
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t) th.emplace_back(work);
    for (auto& t : th) t.join();
    if (!err.empty()) {
        for (auto* f : out) {
            if (f) {
                delete[] f->blocks;
                delete[] f->storage;
                delete f;
            }
        }
        throw Error{err_status, err};
    }
    return out;
}

void free_fused(sv_fused_s* f)
{
    if (!f) return;
    delete[] f->blocks;
    delete[] f->storage;
    delete f;
}

// Builds the device-side descriptors for circuits `sel` with widths kmax.
// Block b (k targets tq, 2^k x 2^k complex128 m) as a five-qubit gate: the
// targets, then free qubits below the lowest target and above the highest as
// the high matrix bits, the matrix M (x) I (32 x 32 complex128).
void pad_block_to_five(int n, int k, const int* tq, const double* m, int32_t* out_t, std::vector<double>& out_m)
{
    uint64_t used = 0;
    int lo = n, hi = -1;
    for (int a = 0; a < k; ++a) {
        out_t[a] = tq[a];
        used |= uint64_t(1) << tq[a];
        lo = std::min(lo, tq[a]);
        hi = std::max(hi, tq[a]);
    }
    int kk = k;
    for (int q = lo - 1; q >= 0 && kk < 5; --q)
        if (!((used >> q) & 1)) out_t[kk++] = q;
    for (int q = hi + 1; q < n && kk < 5; ++q)
        if (!((used >> q) & 1)) out_t[kk++] = q;
    if (kk < 5) throw Error{SV_ERR_INTERNAL, "level path: no free qubits to pad a block"};
    const int d = 1 << k, D = 32;
    out_m.assign(size_t(2) * D * D, 0.0);
    for (int e = 0; e < D / d; ++e)
        for (int r = 0; r < d; ++r)
            for (int c = 0; c < d; ++c) {
                const size_t dst = size_t(e * d + r) * D + size_t(e * d + c);
                out_m[2 * dst] = m[2 * (size_t(r) * d + c)];
                out_m[2 * dst + 1] = m[2 * (size_t(r) * d + c) + 1];
            }
}

// Level-path descriptors of circuit j (state at c.state_off, fused blocks f):
// one tile-sweep descriptor and packed matrix per block, in tile shape s.
// Returns the index of its first descriptor.
uint32_t add_level_circuit(BatchHost& H, const BatchCircuit& c, const sv_fused_s* f, int cu_count,
                           const LevelShape& s)
{
    const uint32_t first = uint32_t(H.tdescs.size());
    const size_t mat_bytes = packed_matrix_bytes(SV_C64, c.n, 5, 0);
    std::vector<double> pm;
    for (int bi = 0; bi < f->n_blocks; ++bi) {
        const FusedBlock& fb = f->blocks[bi];
        int32_t t5[5];
        const double* m5 = fb.m;
        if (fb.k < 5) {
            pad_block_to_five(c.n, fb.k, fb.targets, fb.m, t5, pm);
            m5 = pm.data();
        } else {
            for (int a = 0; a < 5; ++a) t5[a] = fb.targets[a];
        }
        GateDesc d{};
        d.n = c.n;
        d.k = 5;
        for (int a = 0; a < 5; ++a) d.tbit[a] = uint64_t(1) << t5[a];
        BatchTileDesc td{};
        // the single-state sweep's narrow tiles, in the spread or the plain
        // layout; a workgroup takes tiles_per_wg tiles in strided order.
        // The last block also takes the Z-type sums (its partial sums are
        // placed once the level schedule is fixed).
        td.t = make_tile_args(d, c.n, 12, cu_count, s.spread ? 12 : 0, false);
        td.t.tiles_per_wg = std::min<uint64_t>(uint64_t(s.tiles_per_wg), td.t.n_tiles);
        td.t.trot = 0;
        while ((uint64_t(1) << td.t.trot) < td.t.tiles_per_wg) ++td.t.trot;
        td.state_off = c.state_off;
        td.term0 = c.term0;
        td.n_terms = bi + 1 == f->n_blocks ? int32_t(c.n_terms) : -1;
        td.red_off = 0;
        td.mat_off = H.tmats.size();
        H.tmats.resize(H.tmats.size() + mat_bytes / sizeof(float4));
        pack_matrix(SV_C64, c.n, 5, 0, m5, 0, H.tmats.data() + td.mat_off);
        H.tdescs.push_back(td);
    }
    return first;
}

// Fused programs of circuits (input index -> program) that a caller keeps
// across several builds; build_host neither fuses nor frees them.
using Prefused = std::map<int, sv_fused_s*>;

BatchHost build_host(const std::vector<CircuitInput>& in, const std::vector<int>& sel,
                     const std::map<int, SizePlan>& plans, const std::vector<int>& term0,
                     const std::vector<int>& nterms, const uint64_t* z_masks, std::vector<int>* blocks_out,
                     int cu_count, const Prefused* prefused = nullptr)
{
    // each distinct circuit is fused once (a tuning sample repeats circuits)
    auto plan_of = [&](int n) -> const SizePlan& { return plans.at(n); };
    std::vector<CircuitInput> sub;
    std::vector<int> ks;
    std::map<int, size_t> uniq;
    std::vector<size_t> slot(sel.size());
    std::vector<sv_fused_s*> fused(sel.size());
    std::vector<sv_fused_s*> fused_u;  // fused here, freed here
    if (prefused) {
        for (size_t j = 0; j < sel.size(); ++j) fused[j] = prefused->at(sel[j]);
    } else {
        for (size_t j = 0; j < sel.size(); ++j) {
            const int i = sel[j];
            auto it = uniq.find(i);
            if (it == uniq.end()) {
                const SizePlan& pl = plan_of(in[i].n);
                it = uniq.emplace(i, sub.size()).first;
                sub.push_back(in[i]);
                ks.push_back(pl.level ? std::min(kBatchMaxK, in[i].n) : pl.kmax);
            }
            slot[j] = it->second;
        }
        fused_u = fuse_all(sub, ks);
        for (size_t j = 0; j < sel.size(); ++j) fused[j] = fused_u[slot[j]];
    }
    BatchHost H;
    H.circuits.resize(sel.size());
    std::vector<uint32_t> level_circuits, level_first;
    uint64_t off = 0;
    for (size_t j = 0; j < sel.size(); ++j) {
        const int i = sel[j];
        BatchCircuit& c = H.circuits[j];
        c.n = in[i].n;
        c.block0 = uint32_t(H.blocks.size());
        c.n_blocks = uint32_t(fused[j]->n_blocks);
        c.term0 = uint32_t(H.z_masks.size());
        c.n_terms = uint32_t(nterms[i]);
        for (int t = 0; t < nterms[i]; ++t) H.z_masks.push_back(z_masks[term0[i] + t]);
        c.state_off = off;
        off += std::max<uint64_t>(uint64_t(1) << c.n, 32);  // 256-byte aligned starts
        const SizePlan& pl = plan_of(c.n);
        if (pl.level && fused[j]->n_blocks > 0) {
            level_circuits.push_back(uint32_t(j));
            level_first.push_back(add_level_circuit(H, c, fused[j], cu_count, pl.shape));
            if (blocks_out) (*blocks_out)[i] = fused[j]->n_blocks;
            continue;
        }
        for (int bidx = 0; bidx < fused[j]->n_blocks; ++bidx) {
            const FusedBlock& fb = fused[j]->blocks[bidx];
            BatchBlock b{};
            block_geometry(b, fb.targets, fb.k, c.n);
            b.mat_off = uint32_t(H.mats.size());
            pack_batch_matrix(fb.m, fb.k, H.mats);
            H.blocks.push_back(b);
        }
        if (blocks_out) (*blocks_out)[i] = fused[j]->n_blocks;
    }
    H.state_amps = off;
    for (auto* f : fused_u) free_fused(f);
    // Queue order.  The cheapest circuits, up to kShortShare of the batch's
    // work, go first (smallest first): they are done within that share of
    // the launch instead of after every large state.  The rest follow
    // largest first, so the long circuits start early and none starts late.
    // A circuit's work is its state size times its sweeps.
    constexpr double kShortShare = 0.05;
    for (uint32_t j = 0; j < uint32_t(sel.size()); ++j)
        if (std::find(level_circuits.begin(), level_circuits.end(), j) == level_circuits.end()) H.order.push_back(j);
    auto work = [&](uint32_t c) { return double(uint64_t(1) << H.circuits[c].n) * (H.circuits[c].n_blocks + 1); };
    std::stable_sort(H.order.begin(), H.order.end(), [&](uint32_t a, uint32_t b) { return work(a) < work(b); });
    double total = 0.0;
    for (uint32_t c : H.order) total += work(c);
    size_t n_short = 0;
    for (double cum = 0.0; n_short < H.order.size(); ++n_short) {
        cum += work(H.order[n_short]);
        if (cum > kShortShare * total) break;
    }
    std::reverse(H.order.begin() + std::ptrdiff_t(n_short), H.order.end());
    // Level path: launch l sweeps block l of every circuit that has one;
    // after it, the circuits whose last block it was are reduced.  In a
    // launch, the circuits that end there come first (their tiles also take
    // the Z-type sums, so they should not be the launch's last
    // workgroups), then the others, most blocks first.
    std::vector<size_t> lorder(level_circuits.size());
    std::iota(lorder.begin(), lorder.end(), size_t(0));
    std::stable_sort(lorder.begin(), lorder.end(), [&](size_t a, size_t b) {
        return H.circuits[level_circuits[a]].n_blocks > H.circuits[level_circuits[b]].n_blocks;
    });
    uint32_t depth = 0;
    for (uint32_t j : level_circuits) depth = std::max(depth, H.circuits[j].n_blocks);
    // A level with few tiles (the last levels, where a few deep circuits are
    // left) takes fewer tiles per workgroup, so that it still has about four
    // rounds of workgroups for the device: at most its tiles / (4 x the
    // workgroups that fit at once, three per CU), a power of two.  Not a
    // circuit's last block: the order of its Z-type sums follows its tiles
    // per workgroup, which thus stays the plan's, whatever the rest of the
    // batch.  The last block gets room for its workgroups' sums.
    {
        std::vector<uint64_t> level_tiles(depth, 0);
        for (size_t q = 0; q < level_circuits.size(); ++q) {
            const BatchCircuit& c = H.circuits[level_circuits[q]];
            for (uint32_t l = 0; l < c.n_blocks; ++l) level_tiles[l] += H.tdescs[level_first[q] + l].t.n_tiles;
        }
        const uint64_t fill = uint64_t(cu_count) * 3 * 4;
        for (size_t q = 0; q < level_circuits.size(); ++q) {
            const BatchCircuit& c = H.circuits[level_circuits[q]];
            for (uint32_t l = 0; l < c.n_blocks; ++l) {
                BatchTileDesc& td = H.tdescs[level_first[q] + l];
                TileArgs& t = td.t;
                uint64_t cap = 1;
                while (cap * 2 * fill <= level_tiles[l]) cap *= 2;
                if (l + 1 < c.n_blocks && t.tiles_per_wg > cap) {
                    t.tiles_per_wg = cap;
                    t.trot = 0;
                    while ((uint64_t(1) << t.trot) < t.tiles_per_wg) ++t.trot;
                }
                if (l + 1 == c.n_blocks) {
                    td.red_off = H.n_partials;
                    H.n_partials += (t.n_tiles + t.tiles_per_wg - 1) / t.tiles_per_wg * (c.n_terms + 1);
                }
            }
        }
    }
    for (uint32_t l = 0; l < depth; ++l) {
        BatchLevel L;
        L.entry0 = H.entries.size();
        L.finish0 = H.finish.size();
        std::vector<size_t> here;
        for (size_t q : lorder)
            if (H.circuits[level_circuits[q]].n_blocks == l + 1) here.push_back(q);
        for (size_t q : lorder)
            if (H.circuits[level_circuits[q]].n_blocks > l + 1) here.push_back(q);
        for (size_t q : here) {
            const BatchCircuit& c = H.circuits[level_circuits[q]];
            const uint32_t di = level_first[q] + l;
            const TileArgs& t = H.tdescs[di].t;
            const uint64_t n_wg = (t.n_tiles + t.tiles_per_wg - 1) / t.tiles_per_wg;
            for (uint64_t w = 0; w < n_wg; ++w) H.entries.push_back({di, uint32_t(w)});
            if (c.n_blocks == l + 1) H.finish.push_back({level_circuits[q], uint32_t(n_wg), H.tdescs[di].red_off});
        }
        L.n_entries = uint32_t(H.entries.size() - L.entry0);
        L.n_finish = uint32_t(H.finish.size() - L.finish0);
        H.levels.push_back(L);
    }
    return H;
}

template <typename T>
size_t align_up(size_t v)
{
    return (v + 255) & ~size_t(255);
}

// Uploads H into one device arena and fills args (states excluded).
char* upload(const BatchHost& H, BatchArgs& a, hipStream_t stream, size_t* dev_bytes)
{
    struct Part {
        const void* src;
        size_t bytes;
        size_t room;
    };
    auto part = [](const void* src, size_t bytes) { return Part{src, bytes, align_up<int>(std::max<size_t>(bytes, 1))}; };
    const size_t n_terms = std::max<size_t>(1, H.z_masks.size());
    Part parts[] = {
        part(H.circuits.data(), H.circuits.size() * sizeof(BatchCircuit)),
        part(H.order.data(), H.order.size() * sizeof(uint32_t)),
        part(H.blocks.data(), H.blocks.size() * sizeof(BatchBlock)),
        part(H.mats.data(), H.mats.size() * sizeof(float)),
        part(H.z_masks.data(), H.z_masks.size() * sizeof(uint64_t)),
        part(nullptr, n_terms * sizeof(double)),                   // expectations
        part(nullptr, H.circuits.size() * sizeof(uint64_t)),       // completion times
        part(nullptr, 256),                                        // run start
        part(nullptr, 256),                                        // queue
        part(H.tdescs.data(), H.tdescs.size() * sizeof(BatchTileDesc)),
        part(H.tmats.data(), H.tmats.size() * sizeof(float4)),
        part(H.entries.data(), H.entries.size() * sizeof(BatchLevelEntry)),
        part(H.finish.data(), H.finish.size() * sizeof(BatchFinish)),
        part(nullptr, H.n_partials * sizeof(double)),             // last levels' sums
    };
    size_t total = 0;
    for (const Part& q : parts) total += q.room;
    char* dev = static_cast<char*>(dev_alloc(total, "batch descriptors"));
    if (dev_bytes) *dev_bytes = total;
    char* where[sizeof(parts) / sizeof(parts[0])];
    char* p = dev;
    for (size_t i = 0; i < sizeof(parts) / sizeof(parts[0]); ++i) {
        where[i] = p;
        if (parts[i].src && parts[i].bytes) {
            const hipError_t e = hipMemcpyAsync(p, parts[i].src, parts[i].bytes, hipMemcpyHostToDevice, stream);
            if (e != hipSuccess) {
                (void)hipStreamSynchronize(stream);
                dev_free(dev, total);
                throw Error{SV_ERR_DEVICE, std::string("hipMemcpyAsync: ") + hipGetErrorString(e)};
            }
        }
        p += parts[i].room;
    }
    a.circuits = reinterpret_cast<const BatchCircuit*>(where[0]);
    a.order = reinterpret_cast<const uint32_t*>(where[1]);
    a.blocks = reinterpret_cast<const BatchBlock*>(where[2]);
    a.mats = reinterpret_cast<const float*>(where[3]);
    a.z_masks = reinterpret_cast<const uint64_t*>(where[4]);
    a.expect = reinterpret_cast<double*>(where[5]);
    a.t_done = reinterpret_cast<uint64_t*>(where[6]);
    a.t_start = reinterpret_cast<uint64_t*>(where[7]);
    a.queue = reinterpret_cast<uint32_t*>(where[8]);
    a.tdescs = reinterpret_cast<const BatchTileDesc*>(where[9]);
    a.tmats = reinterpret_cast<const float4*>(where[10]);
    a.entries = reinterpret_cast<const BatchLevelEntry*>(where[11]);
    a.finish = reinterpret_cast<const BatchFinish*>(where[12]);
    a.partials = reinterpret_cast<double*>(where[13]);
    a.n_queue = uint32_t(H.order.size());
    const hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        dev_free(dev, total);
        throw Error{SV_ERR_DEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(e)};
    }
    return dev;
}

// Runs the level path's launches of args on a stream: level l, then the
// expectations of the circuits it finishes.
void launch_levels(hipStream_t stream, const BatchArgs& a, const std::vector<BatchLevel>& levels)
{
    for (size_t l = 0; l < levels.size(); ++l) {
        const BatchLevel& L = levels[l];
        launch_batch_level(stream, a, L.entry0, L.n_entries, l == 0);
        if (L.n_finish > 0) launch_batch_finish(stream, a, L.finish0, L.n_finish);
    }
}

// ------------------------------------------------------------ autotuner
//
// For each qubit count of a batch the autotuner times, on a sample of the
// batch's own circuits of that size (up to 64, repeated until they fill the
// device), the persistent kernel at fusion widths 3, 4 and 5, and the level
// path in each tile shape (1, 2, 4 or 8 tiles per workgroup; spread or plain
// layout), as far as the size may take each path, and keeps the fastest
// width and shape; where both paths are open to the size it keeps the
// faster path.  Results are kept for the process and, when the environment
// variable SV_AUTOTUNE_CACHE names a file, in that JSON file, keyed by the
// device's architecture, the state type and the qubit count, so that later
// processes skip the timing.

using tunecache::Records;
using tunecache::TuneRecord;

std::mutex g_tune_mu;
Records g_tuned;  // (arch, n)
std::map<int, std::string> g_arch;                           // device -> architecture name

std::string device_arch(int device)
{
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_arch.find(device);
    if (it != g_arch.end()) return it->second;
    hipDeviceProp_t prop{};
    SV_HIP(hipGetDeviceProperties(&prop, device));
    std::string a(prop.gcnArchName);
    for (char& ch : a)
        if (ch == '"' || ch == '\\' || uint8_t(ch) < 0x20) ch = '_';
    g_arch[device] = a;
    return a;
}

std::string tune_cache_path()
{
    const char* p = std::getenv("SV_AUTOTUNE_CACHE");
    return p ? std::string(p) : std::string();
}

// The tuned record of (arch, n), from the process or the cache file;
// missing parts stay -1.
TuneRecord lookup_tuned(const std::string& arch, int n)
{
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tuned.find({arch, n});
    TuneRecord r = it == g_tuned.end() ? TuneRecord{} : it->second;
    const std::string path = tune_cache_path();
    if ((r.kmax == -1 || r.tiles_per_wg == -1) && !path.empty()) {
        const auto file = tunecache::read_tune_file(path);
        auto f = file.find({arch, n});
        if (f != file.end()) {
            if (r.kmax == -1 && f->second.kmax != -1) {
                r.kmax = f->second.kmax;
                r.persistent_ms = f->second.persistent_ms;
            }
            if (r.tiles_per_wg == -1 && f->second.tiles_per_wg != -1) {
                r.tiles_per_wg = f->second.tiles_per_wg;
                r.spread = f->second.spread;
                r.level_ms = f->second.level_ms;
            }
            g_tuned[{arch, n}] = r;
        }
    }
    return r;
}

void store_tuned(const std::string& arch, int n, const TuneRecord& r)
{
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tuned[{arch, n}] = r;
    const std::string path = tune_cache_path();
    if (!path.empty()) tunecache::write_tune_file(path, {{{arch, n}, r}});
}

// Times one plan of the sample: an untimed run, then a timed one; returns
// the timed run's milliseconds, or a negative value if its memory could not
// be had.
float time_plan(sv_handle_s* h, const std::vector<CircuitInput>& in, const std::vector<int>& sample,
                const std::map<int, SizePlan>& plans, const std::vector<int>& term0, const std::vector<int>& nterms,
                const uint64_t* z_masks, hipEvent_t e0, hipEvent_t e1, const Prefused* prefused = nullptr,
                int timed_runs = 1)
{
    BatchHost H = build_host(in, sample, plans, term0, nterms, z_masks, nullptr, h->cu_count, prefused);
    BatchArgs a{};
    size_t dev_bytes = 0;
    char* dev = upload(H, a, h->stream, &dev_bytes);
    const size_t st_bytes = H.state_amps * sizeof(float) * 2;
    void* states = nullptr;
    try {
        states = dev_alloc(st_bytes, "autotuner states");
    } catch (...) {
        dev_free(dev, dev_bytes);
        return -1.f;
    }
    a.states = states;
    float ms = 0.f;
    try {
        // an untimed run, then the fastest of timed_runs
        for (int rep = 0; rep <= timed_runs; ++rep) {
            if (rep > 0) SV_HIP(hipEventRecord(e0, h->stream));
            launch_batch_reset(h->stream, a);
            if (a.n_queue > 0) launch_batch(h->stream, h->cu_count, a);
            launch_levels(h->stream, a, H.levels);
            if (rep > 0) {
                SV_HIP(hipEventRecord(e1, h->stream));
                SV_HIP(hipEventSynchronize(e1));
                float t = 0.f;
                SV_HIP(hipEventElapsedTime(&t, e0, e1));
                ms = rep == 1 ? t : std::min(ms, t);
            }
        }
    } catch (...) {
        dev_free(states, st_bytes);
        dev_free(dev, dev_bytes);
        throw;
    }
    dev_free(states, st_bytes);
    dev_free(dev, dev_bytes);
    return ms;
}

// The persistent kernel's fusion width for circuits idx of n qubits: each
// width 3..5 timed on up to 64 of them, repeated to two workgroups' worth
// per CU.  Fills rec.kmax and rec.persistent_ms (per circuit).
void tune_width(sv_handle_s* h, const std::vector<CircuitInput>& in, const std::vector<int>& idx, int n,
                const std::vector<int>& term0, const std::vector<int>& nterms, const uint64_t* z_masks,
                TuneRecord& rec)
{
    std::vector<int> sel;
    for (int i : idx)
        if (int(sel.size()) < 64) sel.push_back(i);
    std::vector<int> sample;
    const size_t want = std::max<size_t>(sel.size(), size_t(h->cu_count) * 2);
    while (sample.size() < want) sample.push_back(sel[sample.size() % sel.size()]);
    hipEvent_t e0, e1;
    SV_HIP(hipEventCreate(&e0));
    SV_HIP(hipEventCreate(&e1));
    try {
        for (int k = 3; k <= std::min(kBatchMaxK, n); ++k) {
            SizePlan p;
            p.kmax = k;
            const float ms = time_plan(h, in, sample, {{n, p}}, term0, nterms, z_masks, e0, e1);
            if (ms < 0.f) break;
            const double per = double(ms) / double(sample.size());
            if (rec.kmax == -1 || per < rec.persistent_ms) {
                rec.kmax = k;
                rec.persistent_ms = per;
            }
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rec.kmax == -1) {  // no room to time: the widest width
        rec.kmax = std::min(kBatchMaxK, n);
        rec.persistent_ms = 0.0;
    }
}

// The level path's tile shape for a batch whose level-path circuits are
// by_n (qubit count -> circuits): every circuit of the level path shares
// its launches, so the shapes are timed on one mixed sample, up to 256
// circuits and 320 MiB of states of each size (fused once for all shapes),
// repeated until every level holds twelve tiles per CU, at most 2 GiB of
// states in all; the fastest of
// two timed runs per shape.  The default shape (4 tiles per workgroup,
// spread) stays unless another is at least kShapeMargin faster.  Returns the
// chosen shape and its time per circuit of the sample.
constexpr double kShapeMargin = 0.02;

LevelShape tune_level_shape(sv_handle_s* h, const std::vector<CircuitInput>& in,
                            const std::map<int, std::vector<int>>& by_n, const std::vector<int>& term0,
                            const std::vector<int>& nterms, const uint64_t* z_masks, double* ms_per_circuit)
{
    std::vector<int> sel;
    uint64_t tiles = 0, bytes = 0;
    int min_n = kBatchMaxQubits;
    for (const auto& kv : by_n) {
        min_n = std::min(min_n, kv.first);
        // at most 256 circuits and 320 MiB of states per size
        const size_t cap = std::min<size_t>(256, std::max<size_t>(1, (size_t(320) << 20) >> (kv.first + 3)));
        for (size_t j = 0; j < kv.second.size() && j < cap; ++j) {
            sel.push_back(kv.second[j]);
            tiles += uint64_t(1) << (kv.first - 12);
            bytes += uint64_t(8) << kv.first;
        }
    }
    std::vector<int> sample = sel;
    while (tiles * (sample.size() / sel.size()) < uint64_t(h->cu_count) * 12 &&
           bytes * (sample.size() / sel.size() + 1) <= (uint64_t(2) << 30))
        sample.insert(sample.end(), sel.begin(), sel.end());
    // fused once, at the level path's width
    Prefused pre;
    {
        std::vector<CircuitInput> sub;
        std::vector<int> ks;
        for (int i : sel) {
            sub.push_back(in[i]);
            ks.push_back(std::min(kBatchMaxK, in[i].n));
        }
        auto f = fuse_all(sub, ks);
        for (size_t j = 0; j < sel.size(); ++j) pre[sel[j]] = f[j];
    }
    const LevelShape dflt;
    LevelShape best = dflt;
    double best_ms = -1.0, dflt_ms = -1.0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    try {
        SV_HIP(hipEventCreate(&e0));
        SV_HIP(hipEventCreate(&e1));
        for (int tpw = 1; tpw <= 8 && uint64_t(tpw) <= (uint64_t(1) << (min_n - 12)); tpw *= 2) {
            for (int spread = 1; spread >= 0; --spread) {
                std::map<int, SizePlan> plans;
                for (const auto& kv : by_n) {
                    SizePlan p;
                    p.level = true;
                    p.shape.tiles_per_wg = tpw;
                    p.shape.spread = spread;
                    plans[kv.first] = p;
                }
                const float ms = time_plan(h, in, sample, plans, term0, nterms, z_masks, e0, e1, &pre, 2);
                if (ms < 0.f) continue;
                const double per = double(ms) / double(sample.size());
                if (tpw == dflt.tiles_per_wg && spread == dflt.spread) dflt_ms = per;
                if (best_ms < 0.0 || per < best_ms) {
                    best_ms = per;
                    best.tiles_per_wg = tpw;
                    best.spread = spread;
                }
            }
        }
    } catch (...) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        for (auto& kv : pre) free_fused(kv.second);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (auto& kv : pre) free_fused(kv.second);
    if (dflt_ms > 0.0 && best_ms > dflt_ms * (1.0 - kShapeMargin)) {
        best = dflt;
        best_ms = dflt_ms;
    }
    *ms_per_circuit = best_ms < 0.0 ? 0.0 : best_ms;
    return best;
}

}  // namespace
}  // namespace sv

using namespace sv;

namespace sv {

sv_batch_s* batch_create(sv_handle_s* h, int n_circuits, const int32_t* n_qubits, const int32_t* gate_offsets,
                         const int32_t* codes, const int32_t* qubits, const double* params,
                         const int32_t* term_offsets, const uint64_t* z_masks, int max_fused_qubits)
{
    SV_CHECK(h != nullptr, "handle is NULL");
    SV_CHECK(n_circuits >= 1, "n_circuits must be positive");
    SV_CHECK(n_qubits && gate_offsets && term_offsets, "NULL batch arrays");
    SV_CHECK(max_fused_qubits >= 0 && max_fused_qubits <= kBatchMaxK, "max_fused_qubits must be in [0, 5]");
    const int total_gates = gate_offsets[n_circuits];
    const int total_terms = term_offsets[n_circuits];
    SV_CHECK(gate_offsets[0] == 0 && term_offsets[0] == 0, "offsets must start at 0");
    SV_CHECK(total_gates == 0 || (codes && qubits && params), "NULL gate arrays");
    SV_CHECK(total_terms == 0 || z_masks, "NULL z_masks");
    std::vector<CircuitInput> in(n_circuits);
    std::vector<int> term0(n_circuits), nterms(n_circuits);
    for (int i = 0; i < n_circuits; ++i) {
        const int n = n_qubits[i];
        SV_CHECK(n >= 1 && n <= kBatchMaxQubits, "batch circuits must have 1..30 qubits");
        SV_CHECK(gate_offsets[i + 1] >= gate_offsets[i], "gate offsets must not decrease");
        SV_CHECK(term_offsets[i + 1] >= term_offsets[i], "term offsets must not decrease");
        const int nt = term_offsets[i + 1] - term_offsets[i];
        SV_CHECK(nt <= kBatchMaxTerms, "at most 32 Z-type terms per circuit");
        for (int t = 0; t < nt; ++t)
            SV_CHECK(n == 64 || (z_masks[term_offsets[i] + t] >> n) == 0, "Z mask names a qubit outside the circuit");
        in[i] = {n, codes + gate_offsets[i], qubits + 2 * size_t(gate_offsets[i]), params + 3 * size_t(gate_offsets[i]),
                 gate_offsets[i + 1] - gate_offsets[i]};
        for (int g = 0; g < in[i].n_gates; ++g) {
            const int code = in[i].codes[g] & ~int(SV_GATE_ADJOINT);
            const int q0 = in[i].qubits[2 * g], q1 = in[i].qubits[2 * g + 1];
            const bool two = code == SV_GATE_CX || code == SV_GATE_CZ || code == SV_GATE_CP || code == SV_GATE_SWAP;
            SV_CHECK(q0 >= 0 && q0 < n && (!two || (q1 >= 0 && q1 < n && q1 != q0)),
                     "circuit " + std::to_string(i) + ": gate qubit out of range");
        }
        term0[i] = term_offsets[i];
        nterms[i] = nt;
    }
    // fusion width per qubit count
    std::map<int, std::vector<int>> by_n;
    for (int i = 0; i < n_circuits; ++i) by_n[n_qubits[i]].push_back(i);
    auto* b = new sv_batch_s;
    try {
        b->h = h;
        b->n_circuits = n_circuits;
        b->total_terms = total_terms;
        b->n.assign(n_qubits, n_qubits + n_circuits);
        using clock = std::chrono::steady_clock;
        std::string arch;
        std::map<int, std::vector<int>> level_untuned;  // level sizes without a tuned shape
        for (auto& kv : by_n) {
            const int n = kv.first;
            SizePlan p;
            // the handle's level-path size decides the path
            p.level = n >= h->batch_level_qubits;
            if (max_fused_qubits > 0) {
                // a fixed width and no timing: the level path's default shape
                p.kmax = p.level ? std::min(kBatchMaxK, n) : std::min(max_fused_qubits, n);
            } else {
                if (arch.empty()) arch = device_arch(h->device);
                TuneRecord rec = lookup_tuned(arch, n);
                p.tuned = true;
                if (p.level) {
                    p.kmax = std::min(kBatchMaxK, n);
                    if (rec.tiles_per_wg != -1) {
                        p.shape.tiles_per_wg = int(std::min<uint64_t>(uint64_t(rec.tiles_per_wg), uint64_t(1) << (n - 12)));
                        p.shape.spread = rec.spread;
                    } else {
                        level_untuned[n] = kv.second;
                    }
                } else {
                    if (rec.kmax == -1) {
                        const auto t0 = clock::now();
                        tune_width(h, in, kv.second, n, term0, nterms, z_masks, rec);
                        store_tuned(arch, n, rec);
                        b->tune_s += std::chrono::duration<double>(clock::now() - t0).count();
                    }
                    p.kmax = rec.kmax;
                }
            }
            b->plans[n] = p;
        }
        if (!level_untuned.empty()) {
            // one shape for the level sizes not tuned yet, timed on a mix of
            // them, kept for each of those sizes
            const auto t0 = clock::now();
            double ms = 0.0;
            const LevelShape sh = tune_level_shape(h, in, level_untuned, term0, nterms, z_masks, &ms);
            for (const auto& kv : level_untuned) {
                TuneRecord rec = lookup_tuned(arch, kv.first);
                rec.tiles_per_wg = sh.tiles_per_wg;
                rec.spread = sh.spread;
                rec.level_ms = ms;
                store_tuned(arch, kv.first, rec);
                SizePlan& p = b->plans[kv.first];
                p.shape.tiles_per_wg = int(std::min<uint64_t>(uint64_t(sh.tiles_per_wg), uint64_t(1) << (kv.first - 12)));
                p.shape.spread = sh.spread;
            }
            b->tune_s += std::chrono::duration<double>(clock::now() - t0).count();
        }
        const auto t_build = clock::now();
        std::vector<int> all(n_circuits);
        std::iota(all.begin(), all.end(), 0);
        b->blocks_per_circuit.assign(n_circuits, 0);
        BatchHost H = build_host(in, all, b->plans, term0, nterms, z_masks, &b->blocks_per_circuit, h->cu_count);
        b->levels = H.levels;
        b->state_off.resize(n_circuits);
        for (int i = 0; i < n_circuits; ++i) b->state_off[i] = H.circuits[i].state_off;
        b->state_amps = H.state_amps;
        b->dev = upload(H, b->args, h->stream, &b->dev_bytes);
        b->build_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_build).count();
        int khz = 0;
        SV_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, h->device));
        b->tick_hz = khz > 0 ? double(khz) * 1e3 : 1e8;
    } catch (...) {
        delete b;
        throw;
    }
    return b;
}

static void drop_graph(sv_batch_s* b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_states = nullptr;
}

// Records the run for b->args.states on a private stream (the handle's may
// be the null stream, which cannot be captured): the queue reset, the
// persistent kernel (if any circuit takes it), then every level of the
// level path, each followed by the expectations of the circuits it
// finishes.  Kernel nodes only.
static void record_run(sv_batch_s* b)
{
    sv_handle_s* h = b->h;
    SV_HIP(hipStreamSynchronize(h->stream));
    drop_graph(b);
    hipStream_t cap = nullptr;
    SV_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    try {
        SV_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed));
        try {
            launch_batch_reset(cap, b->args);
            if (b->args.n_queue > 0) launch_batch(cap, h->cu_count, b->args);
            launch_levels(cap, b->args, b->levels);
        } catch (...) {
            hipGraph_t dropped = nullptr;
            (void)hipStreamEndCapture(cap, &dropped);
            if (dropped) (void)hipGraphDestroy(dropped);
            throw;
        }
        SV_HIP(hipStreamEndCapture(cap, &b->graph));
        SV_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        b->graph_states = b->args.states;
    } catch (...) {
        (void)hipStreamDestroy(cap);
        drop_graph(b);
        throw;
    }
    SV_HIP(hipStreamDestroy(cap));
}

void batch_run(sv_batch_s* b, void* states, double* expect_out, double* latency_s, double* kernel_s)
{
    SV_CHECK(b != nullptr, "batch is NULL");
    SV_CHECK(states != nullptr && (reinterpret_cast<uintptr_t>(states) & 255) == 0,
             "states must be a 256-byte aligned device buffer");
    sv_handle_s* h = b->h;
    b->args.states = states;
    hipEvent_t e0, e1;
    SV_HIP(hipEventCreate(&e0));
    SV_HIP(hipEventCreate(&e1));
    float ms = 0.f;
    std::vector<uint64_t> done(b->n_circuits);
    uint64_t t0 = 0;
    try {
        if (!b->exec || b->graph_states != states) record_run(b);
        SV_HIP(hipEventRecord(e0, h->stream));
        SV_HIP(hipGraphLaunch(b->exec, h->stream));
        SV_HIP(hipEventRecord(e1, h->stream));
        if (expect_out && b->total_terms > 0)
            SV_HIP(hipMemcpyAsync(expect_out, b->args.expect, sizeof(double) * b->total_terms,
                                  hipMemcpyDeviceToHost, h->stream));
        SV_HIP(hipMemcpyAsync(done.data(), b->args.t_done, sizeof(uint64_t) * b->n_circuits, hipMemcpyDeviceToHost,
                              h->stream));
        SV_HIP(hipMemcpyAsync(&t0, b->args.t_start, sizeof(uint64_t), hipMemcpyDeviceToHost, h->stream));
        SV_HIP(hipStreamSynchronize(h->stream));
        SV_HIP(hipEventElapsedTime(&ms, e0, e1));
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (latency_s)
        for (int i = 0; i < b->n_circuits; ++i) latency_s[i] = double(done[i] - t0) / b->tick_hz;
    if (kernel_s) *kernel_s = double(ms) * 1e-3;
}

void batch_layout(sv_batch_s* b, uint64_t* state_bytes, uint64_t* byte_offsets)
{
    *state_bytes = b->state_amps * 8;
    if (byte_offsets)
        for (int i = 0; i < b->n_circuits; ++i) byte_offsets[i] = b->state_off[i] * 8;
}

void batch_info(sv_batch_s* b, int n_qubits, int32_t* kmax, int32_t* blocks)
{
    auto it = b->plans.find(n_qubits);
    *kmax = it == b->plans.end() ? 0 : it->second.kmax;
    if (blocks)
        for (int i = 0; i < b->n_circuits; ++i) blocks[i] = b->blocks_per_circuit[i];
}

void batch_plan(sv_batch_s* b, int n_qubits, sv_batch_size_plan_t* out)
{
    *out = sv_batch_size_plan_t{};
    auto it = b->plans.find(n_qubits);
    if (it == b->plans.end()) return;
    const SizePlan& p = it->second;
    out->max_fused_qubits = p.kmax;
    out->level_path = p.level ? 1 : 0;
    out->tiles_per_wg = p.level ? p.shape.tiles_per_wg : 0;
    out->spread = p.level ? p.shape.spread : 0;
    out->tuned = p.tuned ? 1 : 0;
}

void batch_host_times(sv_batch_s* b, double* tune_s, double* build_s)
{
    if (tune_s) *tune_s = b->tune_s;
    if (build_s) *build_s = b->build_s;
}

void batch_destroy(sv_batch_s* b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->h->stream);
    drop_graph(b);
    dev_free(b->dev, b->dev_bytes);
    delete b;
}

}  // namespace sv
