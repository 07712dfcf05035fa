// Device-side descriptors of a batch of independent circuits (complex64),
// shared by the host builder and the persistent batch kernel.
#pragma once

#include <cstdint>

#include "sv_internal.h"

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

struct BatchArgs {
    void* states;
    const BatchCircuit* circuits;
    const uint32_t* order;  // circuit indices in queue order (short first, then largest first)
    const BatchBlock* blocks;
    const float* mats;
    const uint64_t* z_masks;
    double* expect;
    uint64_t* t_done;   // device wall clock at each circuit's completion
    uint64_t* t_start;  // earliest workgroup start (atomic min)
    uint32_t* queue;
    uint32_t n_circuits;
};

void launch_batch(hipStream_t stream, int cu_count, const BatchArgs& a);
void launch_batch_reset(hipStream_t stream, const BatchArgs& a);

}  // namespace sv
