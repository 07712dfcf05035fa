// Internal declarations shared by the host side of libsv and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <deque>
#include <unordered_map>
#include <vector>

#include <cstddef>
#include <cstdint>
#include <string>

#include "sv.h"

namespace sv {

// ------------------------------------------------------------------ errors

void set_error(const std::string& msg);

struct Error {
    sv_status_t status;
    std::string msg;
};

#define SV_HIP(call)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            throw ::sv::Error{e_ == hipErrorOutOfMemory ? SV_ERR_OUT_OF_MEMORY : SV_ERR_DEVICE, \
                              std::string(#call) + ": " + hipGetErrorString(e_)};        \
    } while (0)

#define SV_CHECK(cond, msg)                                                              \
    do {                                                                                 \
        if (!(cond)) throw ::sv::Error{SV_ERR_INVALID_VALUE, (msg)};                     \
    } while (0)

// ------------------------------------------------------ device memory

// Every device allocation libsv makes for itself (handle workspaces,
// scratch, states it owns, recorded programs, batch descriptors) goes
// through dev_alloc / dev_free, which keep a process-wide count against an
// optional cap: the environment variable SV_HBM_BUDGET_BYTES (a decimal byte
// count, read at the first allocation) or sv_set_hbm_budget.  A request
// beyond the cap throws SV_ERR_OUT_OF_MEMORY before any HIP call; memory the
// caller lends (borrowed state pointers) is not counted.
void budget_reserve(size_t bytes, const char* what);
void budget_release(size_t bytes);
void* dev_alloc(size_t bytes, const char* what);
void dev_free(void* p, size_t bytes);

// ------------------------------------------------------------- workspace

// Layout of the handle's device workspace (bytes from its start).  The
// matrix ring sits at the front; the rest is scratch for one blocking
// reduction at a time (reductions never overlap on one handle).
constexpr size_t kMatRingBytes = 4u << 20;     // gate matrices (device copy)
constexpr int kMatRingSegments = 4;            // host staging reuse granularity
constexpr size_t kDefaultWorkspace = 64u << 20;
constexpr size_t kMinWorkspace = 12u << 20;

}  // namespace sv

// Online choice among the k = 5 tile variants (complex64 and complex128):
// after the handle's first kTileWarmSweeps tuned sweeps (untimed, on the
// default variant, while clocks and caches settle), per key (dtype, n, target mask) kTileTrials
// timings of each variant, taken in rotating round-robin order so that every
// variant meets the same mix of neighbouring work, then the variant with
// the lowest mean.  States below SV_TILE_TUNE_MIN_QUBITS are not tuned.
namespace sv {
constexpr int kTileShapes = 3;
constexpr int kTileTrials = 3;
constexpr int kTileWarmSweeps = SV_TILE_WARM_SWEEPS;
struct TileTuneEntry {
    float sum_ms[kTileShapes] = {};
    int measured[kTileShapes] = {};
    int in_flight[kTileShapes] = {};
    bool unusable[kTileShapes] = {};
};
struct TileTrial {
    uint64_t key;
    int shape;
    hipEvent_t e0, e1;
};
struct TileTuner {
    std::unordered_map<uint64_t, TileTuneEntry> entries;
    std::deque<TileTrial> pending;  // in launch order
    std::vector<hipEvent_t> pool;
    uint64_t sweeps = 0;  // tuned sweeps launched (warm-up count)
};
}  // namespace sv

struct sv_handle_s {
    hipStream_t stream = nullptr;
    int device = 0;
    int cu_count = 256;
    char* ws = nullptr;             // device workspace
    size_t ws_bytes = 0;
    char* pinned = nullptr;         // pinned host staging: matrix ring + result readback
    size_t pinned_bytes = 0;
    size_t ring_pos = 0;            // next free byte of the matrix ring
    int ring_seg = 0;               // segment the ring is writing into
    hipEvent_t seg_event[sv::kMatRingSegments] = {};
    bool seg_event_live[sv::kMatRingSegments] = {};
    char* aux = nullptr;            // device scratch that grows with the state (sampler prefixes)
    size_t aux_bytes = 0;
    char* acc_pinned = nullptr;     // pinned host staging of the accessor (two chunks), on first use
    size_t acc_pinned_bytes = 0;
    hipEvent_t acc_event[2] = {};
    int tile_mode = 0;              // sv_tile_mode_t
    int batch_level_qubits = SV_BATCH_LEVEL_DEFAULT;  // batches: circuits of >= this many qubits take the level path
    sv::TileTuner* tuner = nullptr;
};

struct sv_state_s {
    sv_handle_s* h = nullptr;
    int n = 0;
    sv_dtype_t dt = SV_C64;
    void* d = nullptr;
    bool owned = false;
};

struct FusedBlock {
    int k = 0;
    int targets[SV_MAX_TARGETS] = {};
    // dense: 2^k x 2^k complex128, row-major, interleaved; diagonal: the 2^k
    // diagonal entries
    double* m = nullptr;
    bool diagonal = false;
    // Phase coupling applied before m (dense blocks of coupled fusion): the
    // amplitude at index i is first multiplied by exp(i theta), theta = sum
    // over targets a with bit targets[a] of i set, and coupled qubits c with
    // bit couple_q[c] of i set, of couple[a * n_couple + c].
    int n_couple = 0;
    int couple_q[SV_MAX_QUBITS] = {};
    double* couple = nullptr;
};

struct sv_fused_s {
    int n_blocks = 0;
    FusedBlock* blocks = nullptr;
    double* storage = nullptr;
};

namespace sv {

// --------------------------------------------------- device-side launchers

// Arguments of one dense gate sweep, prepared on the host.
struct GateDesc {
    int n = 0;                     // qubits of the state
    int k = 0;                     // number of targets
    int n_controls = 0;
    int n_fixed = 0;               // targets + controls
    int fixed_sorted[SV_MAX_QUBITS] = {};  // ascending positions of targets and controls
    uint64_t cval = 0;             // control bits that must be set
    uint64_t n_groups = 0;         // 2^(n - k - n_controls)
    uint64_t tbit[SV_MAX_TARGETS] = {};    // 1 << targets[a], matrix bit order
    int min_target = 0;
};

// Device format of a gate matrix for the sweep kernel chosen for (dt, n, k,
// controls):
// its size, and packing of a complex128 row-major matrix (or its adjoint)
// into it on the host.
size_t packed_matrix_bytes(sv_dtype_t dt, int n, int k, int n_controls);
void pack_matrix(sv_dtype_t dt, int n, int k, int n_controls, const double* m, int adjoint, void* dst);

// psi: amplitudes; mat: device copy of the packed matrix; desc: the sweep.
void launch_apply(sv_handle_s* h, sv_dtype_t dt, void* psi, const void* mat, const GateDesc& desc);
// The same for a block of coupled fusion: couple is the device copy of its
// phase coupling (a CoupleDev, sv_tile.h), applied before the matrix.
void launch_apply_coupled(sv_handle_s* h, sv_dtype_t dt, void* psi, const void* mat, const void* couple,
                          const GateDesc& desc);

// Generalized permutation gate G = D P (diagonal when has_perm is false):
// device table size and packing (adjoint folded in), and the sweep.
size_t gperm_table_bytes(sv_dtype_t dt, int k, bool has_perm);
void pack_gperm(sv_dtype_t dt, int k, const int64_t* perm, const double* diag, int adjoint, void* dst);
void launch_gperm(sv_handle_s* h, sv_dtype_t dt, void* psi, const void* table, const GateDesc& desc, bool has_perm);

void launch_set_basis(sv_handle_s* h, sv_dtype_t dt, void* psi, int n, uint64_t x);
void launch_scale(sv_handle_s* h, sv_dtype_t dt, void* psi, int n, double factor);

// Device scratch of at least `bytes` owned by the handle, grown on demand
// (the stream is synchronised before an old buffer is freed).
char* ensure_aux(sv_handle_s* h, size_t bytes);

// Blocking reductions; results land in host memory.
double run_norm(sv_handle_s* h, sv_dtype_t dt, const void* psi, int n);

struct PauliMasks {
    uint64_t x = 0, z = 0;
    int ny = 0;
};
void run_expect(sv_handle_s* h, sv_dtype_t dt, const void* psi, int n, const PauliMasks* terms,
                int n_terms, double* out);

// host_io: u and out are host arrays; otherwise device arrays.
void run_sample(sv_handle_s* h, sv_dtype_t dt, const void* psi, int n, const double* u,
                int64_t n_shots, const int32_t* bit_ordering, int n_bits, uint64_t* out, bool host_io);
// The same sampler with every device buffer in a fixed per-GPU array of
// SV_SAMPLE_NOALLOC_SCRATCH_BYTES (no allocation; n <= SV_SAMPLE_NOALLOC_MAX_QUBITS).
void run_sample_noalloc(sv_handle_s* h, sv_dtype_t dt, const void* psi, int n, const double* u,
                        int64_t n_shots, const int32_t* bit_ordering, int n_bits, uint64_t* out);

// Measurement: unnormalised probabilities of the 2^m outcomes of qubits
// (m <= SV_MAX_TARGETS) or of the two parities of the bits in mask; collapse
// (keep (i & qmask) == obits, or parity(i & parity_mask) == parity when
// parity >= 0, times scale; zero the rest).
void run_measure_probs(sv_handle_s* h, sv_dtype_t dt, const void* psi, int n, const int32_t* qubits, int m,
                       double* out);
void run_parity_probs(sv_handle_s* h, sv_dtype_t dt, const void* psi, int n, uint64_t mask, double* out);
void launch_collapse(sv_handle_s* h, sv_dtype_t dt, void* psi, int n, uint64_t qmask, uint64_t obits,
                     uint64_t parity_mask, int parity, double scale);

// psi <- exp(i theta P) psi on the indices whose controls hold their values.
void launch_pauli_rotation(sv_handle_s* h, sv_dtype_t dt, void* psi, int n, const PauliMasks& pm, double theta,
                           const int32_t* controls, const int32_t* cvals, int n_controls);

// Index bit swap of disjoint bit pairs on the mask-selected indices (async),
// and the reordering accessor (blocking; host memory in the state's dtype).
void launch_swap_bits(sv_handle_s* h, sv_dtype_t dt, void* psi, int n, const int32_t* pairs, int n_pairs,
                      const int32_t* mask_bits, const int32_t* mask_values, int n_mask);
void run_accessor(sv_handle_s* h, sv_dtype_t dt, void* psi, int n, const int32_t* ordering, int n_bits,
                  const int32_t* mask_bits, const int32_t* mask_values, int n_mask, void* host, int64_t begin,
                  int64_t end, bool set);

// out = (Re, Im of sum conj(psi) M psi, sum |psi|^2) for M on targets (k <= 5).
void run_expect_matrix(sv_handle_s* h, sv_dtype_t dt, const void* psi, int n, const double* m,
                       const int32_t* targets, int k, double* out);

// Copies `bytes` of host data into the matrix ring and returns the device
// address (stream-ordered before any later launch on the handle).
const void* stage_matrix(sv_handle_s* h, const void* host, size_t bytes);

}  // namespace sv
