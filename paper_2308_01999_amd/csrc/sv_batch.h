// Device-side descriptors of a batch of independent circuits (complex64),
// shared by the host builder and the persistent batch kernel.
#pragma once

#include <cstdint>

#include "sv_tile.h"

namespace sv {

constexpr int kBatchMaxTerms = 32;  // Z-type terms per circuit
constexpr int kBatchMaxQubits = 30;
constexpr int kBatchMaxK = 5;

// One fused block.  Its groups are enumerated inside an LDS region of
// 2^(L + n_hi) amplitudes: the whole state when it has <= 12 qubits
// (L = n, n_hi = 0), else a 4096-amplitude tile.  Group g of the region
// starts at g with zeros inserted at lo_pos; amplitude c of a group sits at
// that start + lds_off[c].
struct BatchBlock {
    int32_t k;
    int32_t L;
    int32_t n_hi;
    int32_t n_lo;
    uint32_t mat_off;  // float offset of the packed matrix
    int8_t hi_pos[8];
    int8_t lo_pos[8];
    int16_t lds_off[32];
};

struct BatchCircuit {
    int32_t n;
    uint32_t n_blocks;
    uint32_t block0;
    uint32_t term0;
    uint32_t n_terms;
    uint32_t pad;
    uint64_t state_off;  // amplitude offset in the states buffer
};

// One block of a circuit on the level path (states of at least the level
// path's qubit count): the block as a five-qubit gate (smaller blocks padded
// with free qubits) in the single-state tile sweep's geometry, and where the
// circuit's state and the block's packed matrix live.
struct BatchTileDesc {
    TileArgs t;
    uint64_t state_off;  // amplitude offset of the circuit's state
    uint64_t mat_off;    // float4 offset of the packed A operands
    // the circuit's last block: its Z-type sums go to partials[red_off +
    // wg * (n_terms + 1) ...] (terms, then the norm); n_terms = -1 otherwise
    uint64_t red_off;
    uint32_t term0;
    int32_t n_terms;
};

// A circuit whose last level is done: its n_wg workgroup sums at red_off.
struct BatchFinish {
    uint32_t circuit;
    uint32_t n_wg;
    uint64_t red_off;
};

// Workgroup w of a level launch sweeps tiles of block desc[entries[w].x],
// as workgroup entries[w].y of that block's single-state sweep.
struct BatchLevelEntry {
    uint32_t desc;
    uint32_t wg;
};

struct BatchArgs {
    void* states;
    const BatchCircuit* circuits;
    const uint32_t* order;  // circuit indices in queue order (short first, then largest first)
    const BatchBlock* blocks;
    const float* mats;
    const uint64_t* z_masks;
    double* expect;
    uint64_t* t_done;   // device wall clock at each circuit's completion
    uint64_t* t_start;  // device wall clock at the run's start (the reset kernel)
    uint32_t* queue;
    uint32_t n_queue;  // circuits the persistent kernel takes (order[0 .. n_queue))
    const BatchTileDesc* tdescs;     // level path
    const float4* tmats;
    const BatchLevelEntry* entries;
    const BatchFinish* finish;       // circuits whose last level is done, per level
    double* partials;                // per-workgroup Z-type sums of the last levels
};

void launch_batch(hipStream_t stream, int cu_count, const BatchArgs& a);
void launch_batch_reset(hipStream_t stream, const BatchArgs& a);
// One level of the level path: n_entries workgroups from entries + first;
// first_level: the states are |0..0> and are not read.
void launch_batch_level(hipStream_t stream, const BatchArgs& a, uint64_t first, uint32_t n_entries, bool first_level);
// Z-type expectations and completion times of the n circuits finish[first ..]
// from the sums their last level left (one workgroup each).
void launch_batch_finish(hipStream_t stream, const BatchArgs& a, uint64_t first, uint32_t n);

}  // namespace sv
