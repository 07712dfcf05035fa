/*
 * sv.h -- C ABI of libsv, an MI355X (gfx950) state-vector simulation core.
 *
 * The problem statement follows the cuQuantum SDK paper, Sec. II: a state of
 * n qubits is a complex vector of 2^n amplitudes held in GPU memory; gates are
 * applied to it in place; measurement outcomes are sampled from the
 * probability distribution without collapsing it; expectation values of
 * Pauli strings are computed from it; a library handle owns a small
 * workspace (a few tens of MB, Table I "resource management").
 *
 * Conventions used by every entry point:
 *   - Qubit j is bit j of the amplitude index (qubit 0 is the least
 *     significant bit); the paper maps each qubit to one index bit (Sec. II-C).
 *   - Amplitudes are interleaved (re, im): 8 bytes per amplitude for
 *     SV_C64 (two floats), 16 bytes for SV_C128 (two doubles).
 *   - A k-qubit gate matrix is passed as 2^k x 2^k complex128, row-major,
 *     interleaved (re, im) doubles; bit a of its row/column index is the
 *     state of targets[a] (targets[0] is the matrix least-significant bit).
 *     For SV_C64 states the library rounds it once to complex64.
 *   - Control values default to 1.
 *   - Every call validates all arguments before any device work; invalid
 *     input returns SV_ERR_INVALID_VALUE and leaves the state untouched.
 *   - Host arrays passed in are copied before the call returns; the caller
 *     may free them immediately.
 *   - sv_apply_* calls are asynchronous on the handle's stream; sv_norm,
 *     sv_expect_pauli, sv_sample, sv_copy_* and sv_sync block until their
 *     results are in host memory.
 *   - HIP runtime errors map to SV_ERR_DEVICE; allocation failure maps to
 *     SV_ERR_OUT_OF_MEMORY.  sv_last_error() returns a thread-local message
 *     for the last non-OK status.  No C++ exception crosses this ABI.
 *   - A handle may be used by one host thread at a time; different handles
 *     may be used concurrently from different threads.
 */
#ifndef SV_H
#define SV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SV_OK = 0,
    SV_ERR_INVALID_VALUE = 1,
    SV_ERR_OUT_OF_MEMORY = 2,
    SV_ERR_NOT_SUPPORTED = 3,
    SV_ERR_DEVICE = 4,
    SV_ERR_INTERNAL = 5
} sv_status_t;

typedef enum { SV_C64 = 0, SV_C128 = 1 } sv_dtype_t;

/* Largest qubit count of one state (2^36 complex64 amplitudes = 512 GiB is
 * beyond one MI355X; 34 qubits complex64 / 33 complex128 = 128 GiB fit). */
#define SV_MAX_QUBITS 36
/* Largest number of targets of one dense gate or fused block. */
#define SV_MAX_TARGETS 10

typedef struct sv_handle_s* sv_handle_t;
typedef struct sv_state_s* sv_state_t;
typedef struct sv_fused_s* sv_fused_t;

/* One gate of a circuit, as input to gate fusion.  `matrix` is
 * 2^n_targets x 2^n_targets complex128 (see conventions); with adjoint != 0
 * the gate is its conjugate transpose (as the adjoint flag of
 * sv_apply_matrix), so a circuit and its inverse share their matrices. */
typedef struct {
    int32_t n_targets;
    const int32_t* targets;
    const double* matrix;
    int32_t n_controls;
    const int32_t* controls;
    const int32_t* control_values; /* NULL: all 1 */
    int32_t adjoint;               /* 0: matrix; else its conjugate transpose */
} sv_gate_t;

/* A Pauli string: ops[a] in {'I','X','Y','Z'} acts on qubits[a]. */
typedef struct {
    int32_t n_ops;
    const int32_t* qubits;
    const char* ops;
} sv_pauli_term_t;

/* ---------------------------------------------------------------- handles */

/* Creates a handle bound to `hip_stream` (a hipStream_t; NULL means the null
 * stream) on the current device, with a device workspace of
 * `workspace_bytes` (0: 64 MiB; minimum 12 MiB) used for reduction partials,
 * sampler tables and gate matrices (Table I: the handle holds a few tens of
 * MB of GPU memory).  The stream is borrowed, never destroyed by libsv. */
sv_status_t sv_handle_create(sv_handle_t* out, void* hip_stream, size_t workspace_bytes);

/* Waits for the handle's stream, then frees the workspace and the handle. */
sv_status_t sv_handle_destroy(sv_handle_t h);

/* Rebinds the handle to another stream (the caller synchronises the switch). */
sv_status_t sv_handle_set_stream(sv_handle_t h, void* hip_stream);

/* Tile variant of the five-qubit sweeps (the fused-gate hot path, Sec.
 * II-B: gate fusion makes k = 5 the common case), complex64 and complex128.
 * All variants do the same arithmetic on every amplitude group, so results
 * are bitwise the same whichever runs; they differ in tile shape (256-thread
 * workgroups on 32 KiB tiles of 1 KiB runs, or 512-thread workgroups on
 * 64 KiB tiles with twice as long runs), in which index bits besides the
 * targets a tile spans, and in the order workgroups take tiles.  Which one
 * moves HBM fastest depends on the target bits.
 *   SV_TILE_AUTO (default): after the handle's first SV_TILE_WARM_SWEEPS
 *     five-qubit sweeps (untimed, spread), it times each variant three
 *     times, in rotating order, on the sweeps of every (dtype, state size,
 *     target set) it sees, with HIP events on its stream, then keeps the
 *     variant with the lowest mean (no timing while the stream is being
 *     captured; the spread variant until a target set has timings).
 *     States of fewer than SV_TILE_TUNE_MIN_QUBITS qubits, whose sweeps
 *     are bound by the launch rather than by the tile shape, always take
 *     the spread variant, untimed;
 *   SV_TILE_NARROW / SV_TILE_WIDE: always that shape, each workgroup on
 *     consecutive tiles (wide needs n >= 13 for complex64 and n >= 12 for
 *     complex128; smaller states use the narrow one);
 *   SV_TILE_SPREAD: narrow tiles whose runs are always 1 KiB, with each
 *     target below the run boundary swapped for a free index bit from 12
 *     up, and workgroups taking tiles far apart (needs n >= 13 for
 *     complex64 and n >= 12 for complex128, and enough free bits; otherwise
 *     the narrow shape).
 * Returns SV_ERR_INVALID_VALUE for any other mode. */
typedef enum { SV_TILE_AUTO = 0, SV_TILE_NARROW = 1, SV_TILE_WIDE = 2, SV_TILE_SPREAD = 3 } sv_tile_mode_t;
/* Untimed five-qubit sweeps an SV_TILE_AUTO handle runs before its first
 * timed trial. */
#define SV_TILE_WARM_SWEEPS 64
/* Smallest state an SV_TILE_AUTO handle times tile variants on. */
#define SV_TILE_TUNE_MIN_QUBITS 22
sv_status_t sv_handle_set_tile_mode(sv_handle_t h, int32_t mode);

/* Blocks until all work issued on the handle's stream has finished. */
sv_status_t sv_sync(sv_handle_t h);

/* ----------------------------------------------------------------- states */

/* Creates a state of n_qubits in [1, SV_MAX_QUBITS] and the given dtype.
 * device_ptr == NULL: libsv allocates 2^n amplitudes and sets |0..0>.
 * Otherwise the state borrows device_ptr, which must hold 2^n amplitudes of
 * the dtype, be 256-byte aligned and outlive the state; its contents are
 * left as they are (the relaxed memory model of Sec. II-A: the vector only
 * has to live in GPU memory).  The state is used with handle h. */
sv_status_t sv_create(sv_handle_t h, int32_t n_qubits, sv_dtype_t dtype, void* device_ptr,
                      sv_state_t* out);

/* Frees the state (and its amplitudes if libsv allocated them). */
sv_status_t sv_destroy(sv_state_t s);

/* Device address of the amplitudes. */
sv_status_t sv_state_device_ptr(sv_state_t s, void** out);

/* Sets the state to the computational basis state |x>, x < 2^n (async). */
sv_status_t sv_set_basis_state(sv_state_t s, uint64_t x);

/* ------------------------------------------------------- gate application */

/*
 * Applies a dense k-qubit gate in place (Table I: gate application with a
 * dense matrix; Sec. II-B: gate application is the most time-consuming
 * operation).  For every index i whose target bits are 0 and whose control
 * bits equal the control values, the 2^k amplitudes psi[i + off(c)], with
 * off(c) = sum over set bits a of c of 2^targets[a], are replaced by
 * M (or M^dagger if adjoint != 0) times them; all other amplitudes are
 * unchanged.  1 <= k <= min(n, SV_MAX_TARGETS); targets and controls are
 * distinct and in [0, n); control_values may be NULL (all 1) or hold 0/1.
 * Asynchronous on the handle's stream.
 */
sv_status_t sv_apply_matrix(sv_state_t s, const double* matrix, const int32_t* targets, int32_t k,
                            const int32_t* controls, const int32_t* control_values,
                            int32_t n_controls, int32_t adjoint);

/*
 * Generalized permutation gate (Table I: gate application with a
 * generalized permutation matrix; Sec. II-D: diagonal gates, e.g. CZ, cost
 * one sweep whatever their size): G = D P on k targets, where row r of G
 * has its only non-zero entry diag[r] in column perm[r].  In every group
 * (as for sv_apply_matrix, targets[0] = bit 0 of r, controls as there) the
 * amplitude at offset r becomes diag[r] times the one at offset perm[r].
 *   perm: 2^k int64, a permutation of 0 .. 2^k - 1, host memory, or NULL
 *     for the identity (G is then the diagonal matrix diag);
 *   diag: 2^k complex128 (re, im interleaved), host memory, finite;
 *   adjoint != 0 applies G^dagger.
 * A diagonal gate takes 1 <= k <= min(n, SV_MAX_TARGETS) and any controls,
 * and moves only the 2^(n - n_controls) amplitudes its controls select (one
 * read and one write each).  A gate with a permutation takes
 * k + n_controls <= 6.  Host arrays are copied before return.
 * SV_ERR_INVALID_VALUE for bad sizes, repeated or out-of-range qubits, a
 * perm that is not a permutation, or non-finite entries.  Asynchronous on
 * the handle's stream.
 */
sv_status_t sv_apply_gen_permutation(sv_state_t s, const int64_t* perm, const double* diag, const int32_t* targets,
                                     int32_t k, const int32_t* controls, const int32_t* control_values,
                                     int32_t n_controls, int32_t adjoint);

/*
 * Named standard gates (host only).  Writes the target matrix of `name`
 * into matrix_out (room for 16 complex128), its number of targets into
 * *n_targets and its number of leading control qubits into *n_controls.
 * Names: "u3" (theta, phi, lambda; OpenQASM convention), "h", "x", "y",
 * "z", "cx", "cz", "cp" (phi), "swap"; a "_dg" suffix yields the adjoint.
 * For the controlled gates the first qubit of a gate is its control.
 */
sv_status_t sv_gate_matrix(const char* name, const double* params, int32_t n_params,
                           double* matrix_out, int32_t* n_targets, int32_t* n_controls);

/* ------------------------------------------------------------ gate fusion */

/*
 * Gate fusion (Sec. II-B, after qHiPSTER; the fused-gate-size option of
 * Sec. II-D): groups consecutive gates into blocks of at most
 * max_fused_qubits (1..SV_MAX_TARGETS) qubits, each block one dense unitary
 * equal to the ordered product of its gates embedded on the block's qubits
 * (controls become dense qubits of the block).  Host only; FP64 products.
 * Applying the blocks in order equals applying the gates in order.
 */
sv_status_t sv_fuse_gates(const sv_gate_t* gates, int32_t n_gates, int32_t max_fused_qubits,
                          sv_fused_t* out);

/* Codes of the named gates for sv_fuse_gate_list (the matrices of
 * sv_gate_matrix); SV_GATE_ADJOINT may be or-ed into a code to ask for the
 * adjoint. */
typedef enum {
    SV_GATE_U3 = 0,
    SV_GATE_H = 1,
    SV_GATE_X = 2,
    SV_GATE_Y = 3,
    SV_GATE_Z = 4,
    SV_GATE_CX = 5,
    SV_GATE_CZ = 6,
    SV_GATE_CP = 7,
    SV_GATE_SWAP = 8,
    SV_GATE_ADJOINT = 256
} sv_gate_code_t;

/*
 * Gate fusion of a circuit of named gates given as flat arrays (host only):
 * gate g has code codes[g], qubits qubits[2g] (and qubits[2g + 1] for the
 * two-qubit gates; for CX and CP the first is the control) and parameters
 * params[3g .. 3g + 2] (theta, phi, lambda for U3; phi for CP; ignored
 * otherwise).  Equivalent to sv_fuse_gates over the matrices of
 * sv_gate_matrix, without building them on the caller's side.
 */
sv_status_t sv_fuse_gate_list(const int32_t* codes, const int32_t* qubits, const double* params,
                              int32_t n_gates, int32_t max_fused_qubits, sv_fused_t* out);

/*
 * Dense and diagonal gate fusion (Sec. II-D: diagonal gates such as CZ and
 * CP cost one sweep whatever their size, so they are fused into diagonal
 * blocks of up to max_fused_diagonal_qubits qubits, beside the dense blocks
 * of up to max_fused_qubits).  A gate counts as diagonal when every
 * off-diagonal entry of its target matrix is exactly zero (controls keep
 * it diagonal).  Diagonal gates commute with each other, so a diagonal
 * block may gather diagonal gates from across the circuit as long as no
 * non-diagonal gate on a shared qubit lies between them; a dense block may
 * still absorb diagonal gates.  max_fused_diagonal_qubits in
 * [0, SV_MAX_TARGETS]; 0 gives exactly sv_fuse_gates / sv_fuse_gate_list.
 * Applying the blocks in order equals applying the gates in order.  Host
 * only; FP64 products.
 */
sv_status_t sv_fuse_gates_diag(const sv_gate_t* gates, int32_t n_gates, int32_t max_fused_qubits,
                               int32_t max_fused_diagonal_qubits, sv_fused_t* out);
sv_status_t sv_fuse_gate_list_diag(const int32_t* codes, const int32_t* qubits, const double* params,
                                   int32_t n_gates, int32_t max_fused_qubits, int32_t max_fused_diagonal_qubits,
                                   sv_fused_t* out);

/*
 * Coupled fusion: dense fusion (blocks of up to max_fused_qubits qubits)
 * that also lets diagonal phase gates pass (Sec. II-D: diagonal gates are
 * cheap to fuse; Table II fuses the QFT's 577 gates into 18).  A diagonal
 * gate on at most two qubits whose entries all have modulus one (CZ, CP, Z,
 * phase gates) touching a block's qubits and a qubit outside it is not
 * forced into a block of its own: it commutes with everything up to the
 * next non-diagonal gate on its qubits, so it is deferred and applied at
 * the start of the next block that contains one of its qubits.  There its
 * parts inside the block join the block's matrix, and a part coupling a
 * block qubit a to an outside qubit b becomes a phase coupling of the
 * block: before the matrix, the amplitude at index i is multiplied by
 * exp(i phi) when bits a and b of i are both set (sv_fused_block_coupling).
 * Phases still deferred at the end form blocks without gates.  Blocks are
 * dense (never diagonal blocks).  Applying the blocks in order (each:
 * coupling, then matrix) equals applying the gates in order.  Host only;
 * FP64 products.
 */
sv_status_t sv_fuse_gates_coupled(const sv_gate_t* gates, int32_t n_gates, int32_t max_fused_qubits,
                                  sv_fused_t* out);
sv_status_t sv_fuse_gate_list_coupled(const int32_t* codes, const int32_t* qubits, const double* params,
                                      int32_t n_gates, int32_t max_fused_qubits, sv_fused_t* out);

/* Phase coupling of block i: *n_coupled qubits outside the block (ascending
 * into coupled_qubits, room for SV_MAX_QUBITS, may be NULL) and, if phases
 * is not NULL, phases[a * n_coupled + c] (k x n_coupled doubles): the
 * amplitude at index i is multiplied by exp(i sum of phases[a * n_coupled +
 * c] over the a with bit targets[a] of i set and the c with bit
 * coupled_qubits[c] of i set) before the block's matrix.  0 coupled qubits
 * for blocks of the other fusion modes. */
sv_status_t sv_fused_block_coupling(sv_fused_t f, int32_t i, int32_t* n_coupled, int32_t* coupled_qubits,
                                    double* phases);

/* Number of blocks. */
sv_status_t sv_fused_count(sv_fused_t f, int32_t* n_blocks);

/* Block i: its qubit count into *k, its ascending targets into targets
 * (room for SV_MAX_TARGETS), and, if matrix != NULL, its 2^k x 2^k
 * complex128 matrix, or for a diagonal block its 2^k diagonal entries. */
sv_status_t sv_fused_block(sv_fused_t f, int32_t i, int32_t* k, int32_t* targets, double* matrix);

/* *diagonal = 1 if block i is a diagonal block, else 0. */
sv_status_t sv_fused_block_is_diagonal(sv_fused_t f, int32_t i, int32_t* diagonal);

sv_status_t sv_fused_free(sv_fused_t f);

/* Applies all blocks of f in order (async).  Block matrices are uploaded in
 * batches of up to 1 MiB, one host-to-device copy per batch. */
sv_status_t sv_apply_fused(sv_state_t s, sv_fused_t f);

/* Applies blocks [first, first + count) of f in order (async), so a caller
 * can interleave its own work (timing events, measurements) between blocks.
 * Requires 0 <= first and first + count <= the block count. */
sv_status_t sv_apply_fused_range(sv_state_t s, sv_fused_t f, int32_t first, int32_t count);

/* A fused program recorded once into a HIP graph for repeated runs (Sec.
 * II-B: fusion leaves few, large sweeps; for small states each sweep is far
 * shorter than a kernel launch, so replaying a recorded graph removes the
 * per-launch host cost).  sv_graph_create packs and uploads all block
 * matrices of f into device memory owned by the graph (synchronously), then
 * records the block sweeps for state s into a graph on a private stream;
 * the k = 5 tile variants are the handle's current choices.  f may be freed
 * afterwards.  The graph contains kernels only (no memory set or copy
 * nodes).
 * sv_graph_launch runs the recorded sweeps on s in place on the handle's
 * current stream (async), exactly like sv_apply_fused(s, f) would; s must
 * still exist and keep its device memory.  sv_graph_destroy waits for the
 * handle's stream and frees the graph and its matrices.
 * Errors: SV_ERR_INVALID_VALUE for NULL arguments; SV_ERR_OUT_OF_MEMORY if
 * the matrices do not fit; SV_ERR_DEVICE for HIP failures. */
typedef struct sv_graph_s* sv_graph_t;
sv_status_t sv_graph_create(sv_state_t s, sv_fused_t f, sv_graph_t* out);
sv_status_t sv_graph_launch(sv_graph_t g);
sv_status_t sv_graph_destroy(sv_graph_t g);

/* --------------------------------------------------------- Pauli rotation */

/*
 * Rotation by a Pauli string (Table I): psi <- exp(i theta P) psi
 * = cos(theta) psi + i sin(theta) P psi, P the product of the term's
 * single-qubit Paulis ('I', 'X', 'Y', 'Z'; identity elsewhere), applied to
 * the amplitudes whose controls (distinct, disjoint from the term's qubits)
 * hold their values (NULL: all 1); all other amplitudes are unchanged.  One
 * sweep: X/Y factors pair amplitude i with i XOR x, a Z-only string is a
 * phase per amplitude.  Asynchronous.  SV_ERR_INVALID_VALUE for bad qubits,
 * operators or controls, or a non-finite theta.
 */
sv_status_t sv_apply_pauli_rotation(sv_state_t s, double theta, const sv_pauli_term_t* term, const int32_t* controls,
                                    const int32_t* control_values, int32_t n_controls);

/* ------------------------------------------------------------ measurement */

/*
 * Measurement (Table I: on a Z-product basis and batched single-qubit
 * measurement, with probability computation and collapse as separate
 * steps).  Outcome b of measuring qubits[0..m-1] has bit a equal to the
 * value of qubits[a].  Probabilities are unnormalised sums of |psi_i|^2 in
 * FP64, in a fixed order (bitwise reproducible); the calls that return them
 * block.
 *   sv_measure_probabilities: probs[b] for the 2^m outcomes,
 *     1 <= m <= SV_MAX_TARGETS;
 *   sv_zbasis_probabilities: the sums over indices whose measured bits have
 *     even / odd parity (eigenvalue +1 / -1 of the Z-product), any m <= n;
 *   sv_collapse: keeps the amplitudes of outcome `outcome`, divided by
 *     sqrt(norm), sets every other to 0 (norm > 0: the outcome's
 *     probability makes the result a unit vector);
 *   sv_collapse_zbasis: the same for the amplitudes of parity `parity`;
 *   sv_measure_zbasis: parity 0 if randnum * (p_even + p_odd) < p_even,
 *     else 1, into *parity; collapses onto it if collapse != 0;
 *   sv_batch_measure: the first outcome b (in outcome order) whose running
 *     sum of probabilities exceeds randnum times their total, into
 *     *outcome (never a zero-probability outcome); collapses onto it if
 *     collapse != 0.
 * randnum in [0, 1).  Collapse is one write sweep that reads only vectors
 * holding a kept amplitude (asynchronous on its own).
 */
sv_status_t sv_measure_probabilities(sv_state_t s, const int32_t* qubits, int32_t m, double* probs);
sv_status_t sv_zbasis_probabilities(sv_state_t s, const int32_t* qubits, int32_t m, double* p_even, double* p_odd);
sv_status_t sv_collapse(sv_state_t s, const int32_t* qubits, int32_t m, uint64_t outcome, double norm);
sv_status_t sv_collapse_zbasis(sv_state_t s, const int32_t* qubits, int32_t m, int32_t parity, double norm);
sv_status_t sv_measure_zbasis(sv_state_t s, const int32_t* qubits, int32_t m, double randnum, int32_t collapse,
                              int32_t* parity);
sv_status_t sv_batch_measure(sv_state_t s, const int32_t* qubits, int32_t m, double randnum, int32_t collapse,
                             uint64_t* outcome);

/* ---------------------------------------------- index bit swap, accessor */

/*
 * Index bit swap (Table I; the single-GPU building block of the paper's
 * qubit reordering, Sec. II-C): for every index whose mask bits equal
 * mask_values, the amplitude moves to the index with bits pairs[2p] and
 * pairs[2p + 1] exchanged for every pair p.  All bits of the pairs and the
 * mask must be distinct.  Up to 6 bits in all (pairs and mask), on states of
 * at least 12 (complex64) / 11 (complex128) qubits: one sweep that reads and
 * writes every amplitude once in LDS tiles; otherwise each moved amplitude
 * is read and written once and amplitudes the swap leaves in place are not
 * touched.  Asynchronous.
 */
sv_status_t sv_swap_index_bits(sv_state_t s, const int32_t* pairs, int32_t n_pairs, const int32_t* mask_bits,
                               const int32_t* mask_values, int32_t n_mask);

/*
 * Accessor (Table I: copy between host and device while changing the qubit
 * order): host element k - begin, k in [begin, end), is the amplitude whose
 * bit ordering[a] equals bit a of k (a < n_bits) and whose mask bits hold
 * mask_values; n_bits + n_mask must equal n, all bits distinct; end <=
 * 2^n_bits.  Host buffers hold amplitudes in the state's dtype (interleaved
 * re, im; complex64 or complex128).  get reads the state, set writes it.
 * Gathered / scattered on the device through the handle's workspace in
 * chunks of up to 32 MiB, one host copy per chunk.  Both block.
 */
sv_status_t sv_accessor_get(sv_state_t s, const int32_t* ordering, int32_t n_bits, const int32_t* mask_bits,
                            const int32_t* mask_values, int32_t n_mask, void* dst, int64_t begin, int64_t end);
sv_status_t sv_accessor_set(sv_state_t s, const int32_t* ordering, int32_t n_bits, const int32_t* mask_bits,
                            const int32_t* mask_values, int32_t n_mask, const void* src, int64_t begin, int64_t end);

/* ------------------------------------------------------------- reductions */

/* The total of the probability distribution that measurement outcomes are
 * drawn from (Sec. II: the probability distribution is computed
 * numerically): *out = sum_i |psi_i|^2 accumulated in FP64 in a fixed order
 * (bitwise reproducible for a given state).  Blocks.  SV_ERR_INVALID_VALUE
 * for a NULL state or out. */
sv_status_t sv_norm(sv_state_t s, double* out);

/*
 * Expectation of a dense observable (Table I: expectation with a dense matrix
 * observable): out[0] + i out[1] = <psi| M |psi> / <psi|psi> for the
 * 2^k x 2^k complex128 row-major M on targets (targets[0] = matrix LSB),
 * 1 <= k <= 5.  One read sweep, FP64 arithmetic and sums in a fixed order.
 * Blocks.
 */
sv_status_t sv_expect_matrix(sv_state_t s, const double* matrix, const int32_t* targets, int32_t k, double* out);

/* Renormalisation of the state whose probability distribution (Sec. II)
 * no longer sums to one (for example after rounding in complex64 or a
 * collapse by the caller): scales the state by 1/sqrt(norm), the norm as
 * sv_norm computes it and the scale applied in the state's precision.
 * *norm_out (may be NULL) receives the norm before scaling.  Blocks until
 * the norm is known; the scaling sweep is asynchronous.
 * SV_ERR_INVALID_VALUE when the norm is zero or not finite (the state is
 * then left as it is). */
sv_status_t sv_renormalize(sv_state_t s, double* norm_out);

/*
 * Expectation values of Pauli strings (Table I: expectation value with
 * Pauli strings): out[t] = <psi|P_t|psi> / <psi|psi>, FP64 accumulation in a
 * fixed order.  A term may not name a qubit twice.  Blocks.
 */
sv_status_t sv_expect_pauli(sv_state_t s, const sv_pauli_term_t* terms, int32_t n_terms,
                            double* out);

/*
 * Sampler (Table I: bit strings as measurement outcomes without collapsing
 * the state; Sec. II: from the numerically computed probability
 * distribution).  For each uniform u in [0, 1), the outcome is the
 * smallest index i with u * N < C_i, C_i the FP64 cumulative sum of
 * |psi_j|^2 over j <= i and N its total; zero-probability indices are never
 * returned.  With bit_ordering (q_0 .. q_{m-1}, distinct), bit a of each
 * output is bit q_a of the outcome; NULL returns the full index.  Outputs
 * are in the order of the uniforms.  A uniform outside [0, 1) is rejected
 * (SV_ERR_INVALID_VALUE) before any device work; a state of zero norm is
 * reported (SV_ERR_INVALID_VALUE) once the sampler has run, and out's
 * contents are then unspecified.  Blocks.
 */
sv_status_t sv_sample(sv_state_t s, const double* uniforms, int64_t n_shots,
                      const int32_t* bit_ordering, int32_t n_bits, uint64_t* out);

/*
 * The sampler of sv_sample with the uniforms and the outcomes in device
 * memory of the state's GPU (for uniforms drawn on the device and outcomes
 * consumed there: no transfer over the host link).  uniforms: n_shots
 * doubles in [0, 1); out: n_shots uint64 outcomes, in the order of the
 * uniforms, bitwise the same as sv_sample's for the same uniforms;
 * bit_ordering stays a host array.  Both device ranges must lie inside
 * allocations on the handle's device (SV_ERR_INVALID_VALUE otherwise).  A
 * uniform outside [0, 1) or NaN cannot be seen before the kernels run: the
 * call then returns SV_ERR_INVALID_VALUE, as for a state of zero norm, and
 * the contents of out are unspecified.  The sampler's work runs on the
 * handle's stream after the work already queued there; blocks until the
 * outcomes are written.
 */
sv_status_t sv_sample_device(sv_state_t s, const double* uniforms, int64_t n_shots,
                             const int32_t* bit_ordering, int32_t n_bits, uint64_t* out);

/*
 * The sampler of sv_sample for callers that cannot allocate device memory
 * (code that must not call hipMalloc: tight serving loops, harnesses that
 * forbid allocation).  Same arguments, outputs and errors as sv_sample, and
 * the same kernels, so the outcomes are identical.  sv_sample keeps its block
 * prefixes in a handle buffer that grows with the state (a device
 * allocation on first use); this call allocates nothing: all of its device
 * scratch lives in one fixed array of SV_SAMPLE_NOALLOC_SCRATCH_BYTES per
 * GPU, part of libsv's code object and held until the process ends, and it
 * does not touch the handle's workspace.  States of more than
 * SV_SAMPLE_NOALLOC_MAX_QUBITS qubits are rejected with
 * SV_ERR_INVALID_VALUE before any device work.  Every call on one GPU shares
 * that GPU's array (each call rewrites what it reads), so calls that overlap
 * on one GPU, from different handles or threads, race: the caller must
 * serialise them.  Blocks.
 */
#define SV_SAMPLE_NOALLOC_MAX_QUBITS 28
#define SV_SAMPLE_NOALLOC_SCRATCH_BYTES (37u << 20)
sv_status_t sv_sample_noalloc(sv_state_t s, const double* uniforms, int64_t n_shots,
                              const int32_t* bit_ordering, int32_t n_bits, uint64_t* out);

/* ------------------------------------------------------------------ copies */

/* Copies amplitudes [first, first + count) to / from host memory (Table I:
 * accessor, here without reordering).  Blocks. */
sv_status_t sv_copy_to_host(sv_state_t s, void* dst, uint64_t first, uint64_t count);
sv_status_t sv_copy_from_host(sv_state_t s, const void* src, uint64_t first, uint64_t count);

/* ------------------------------------------------------ batched circuits */

typedef struct sv_batch_s* sv_batch_t;

/*
 * A batch of independent complex64 circuits run together in one recorded
 * run (the batched execution of many small states; the paper's fused-gate
 * path of Sec. II-B applied to each).  Circuit i has n_qubits[i]
 * in [1, 30] qubits, starts from |0..0>, and is the named-gate list
 * [gate_offsets[i], gate_offsets[i+1]) of the flat arrays codes, qubits
 * (2 per gate) and params (3 per gate), coded as for sv_fuse_gate_list.
 * Its observables are the Z-type Pauli strings z_masks[term_offsets[i] ..
 * term_offsets[i+1]) (bit q set = Z on qubit q), at most 32 per circuit;
 * each result is <psi|Z..Z|psi> / <psi|psi> accumulated in FP64.
 * Two paths run the circuits.  The persistent kernel: one launch, one
 * workgroup per circuit at a time, the circuit fused at a width of 1..5
 * qubits.  The level path: circuits fused into blocks of up to five
 * qubits, each block swept as a five-qubit gate by the single-state tile
 * sweep (narrow tiles in a spread or plain layout, 1..8 tiles per
 * workgroup), block l of all of them in launch l.
 * Circuits below the handle's level-path qubit count
 * (sv_handle_set_batch_level_qubits, default SV_BATCH_LEVEL_DEFAULT) take
 * the persistent kernel, the others the level path.  max_fused_qubits in
 * [1, 5] fixes the persistent kernel's width, and the level path runs in
 * its default shape (spread layout, 4 tiles per workgroup).
 * max_fused_qubits = 0 lets the autotuner choose: per qubit count of the
 * persistent kernel, the fastest width of 3..5 on the batch's own circuits
 * of that size; for the level path, whose circuits share its launches, the
 * fastest tile shape on a mix of the batch's level-path circuits of the
 * sizes not tuned yet.  Tuned choices are kept for the process
 * and, if the environment variable SV_AUTOTUNE_CACHE names a file, in that
 * JSON file (keyed by device architecture, state type and qubit count;
 * entries of other keys are kept, unreadable lines skipped, and a file that
 * cannot be written is no error), so that later processes reuse them
 * without timing.  A circuit's results depend only on the circuit itself,
 * the handle's settings and the plan of its size (sv_batch_plan), never on
 * the rest of the batch.  Circuits are fused on host threads and their
 * descriptors uploaded once.  Host arrays may be freed on return.
 */
sv_status_t sv_batch_create(sv_handle_t h, int32_t n_circuits, const int32_t* n_qubits,
                            const int32_t* gate_offsets, const int32_t* codes, const int32_t* qubits,
                            const double* params, const int32_t* term_offsets, const uint64_t* z_masks,
                            int32_t max_fused_qubits, sv_batch_t* out);

/* Qubit count from which circuits of batches created later on handle h run on
 * the level path (default SV_BATCH_LEVEL_DEFAULT); SV_BATCH_LEVEL_NONE keeps
 * every circuit on the persistent kernel.  Range [SV_BATCH_LEVEL_MIN_QUBITS,
 * SV_BATCH_LEVEL_NONE]; SV_ERR_INVALID_VALUE otherwise. */
#define SV_BATCH_LEVEL_MIN_QUBITS 13
#define SV_BATCH_LEVEL_DEFAULT 15
#define SV_BATCH_LEVEL_NONE 31
sv_status_t sv_handle_set_batch_level_qubits(sv_handle_t h, int32_t n_qubits);

/* Bytes of device memory the batch's states need (*state_bytes) and, if
 * byte_offsets is not NULL, the byte offset of each circuit's state. */
sv_status_t sv_batch_state_layout(sv_batch_t b, uint64_t* state_bytes, uint64_t* byte_offsets);

/* Fusion width used for circuits of n_qubits (0 if the batch has none) and
 * the fused block count of every circuit (blocks_per_circuit may be NULL). */
sv_status_t sv_batch_info(sv_batch_t b, int32_t n_qubits, int32_t* max_fused_qubits, int32_t* blocks_per_circuit);

/* The plan of the batch's circuits of n_qubits: fusion width, path (1: the
 * level path), the level path's tile shape (tiles per workgroup, 1 for the
 * spread layout, 0 for plain; both 0 on the persistent kernel), and whether
 * the autotuner chose it.  All zero if the batch has no circuit of that
 * size. */
typedef struct {
    int32_t max_fused_qubits;
    int32_t level_path;
    int32_t tiles_per_wg;
    int32_t spread;
    int32_t tuned;
} sv_batch_size_plan_t;
sv_status_t sv_batch_plan(sv_batch_t b, int32_t n_qubits, sv_batch_size_plan_t* out);

/* Host seconds that sv_batch_create spent in the autotuner (*tune_s, 0 when
 * every choice came from its process or file cache) and fusing, packing and
 * uploading the batch itself (*build_s).  Either pointer may be NULL. */
sv_status_t sv_batch_host_times(sv_batch_t b, double* tune_s, double* build_s);

/*
 * Runs the whole batch on the handle's stream and blocks.  The run (queue
 * reset, the persistent kernel, the level path's launches) is recorded into
 * a HIP graph on the first call for a given states buffer and replayed by
 * later calls with the same buffer.
 * states: device buffer of sv_batch_state_layout bytes, 256-byte aligned; on
 * return it holds every circuit's final state.  expect_out (host, may be
 * NULL): all term results in term order.  latency_s (host, may be NULL):
 * per circuit, the device wall-clock time from the run's start to that
 * circuit's completion (its state and expectations written).  kernel_s
 * (may be NULL): the event time of the graph launch.
 */
sv_status_t sv_batch_run(sv_batch_t b, void* states, double* expect_out, double* latency_s, double* kernel_s);

sv_status_t sv_batch_destroy(sv_batch_t b);

/* ---------------------------------------------------- device memory budget */

/*
 * Cap on the device memory libsv allocates itself (Table I: resource
 * management; Sec. II-A: the caller may keep states in memory of its own, so
 * only libsv's own allocations count: handle workspaces and scratch, states
 * created without a device pointer, recorded programs and batch
 * descriptors).  The cap starts as the environment variable
 * SV_HBM_BUDGET_BYTES (a decimal byte count, read at the first allocation;
 * unset or unparsable: no cap).  sv_set_hbm_budget replaces it (0: no cap).
 * An allocation that would take the total past the cap fails with
 * SV_ERR_OUT_OF_MEMORY before any device work, and the call that needed it
 * has no effect.  sv_hbm_usage reports the bytes in use and the cap (0: no
 * cap); either pointer may be NULL.  Both are host-only.
 */
sv_status_t sv_set_hbm_budget(uint64_t bytes);
sv_status_t sv_hbm_usage(uint64_t* used_bytes, uint64_t* budget_bytes);

/* ------------------------------------------------------------------ errors */

/* Thread-local text for the last non-OK status of this thread. */
const char* sv_last_error(void);

/* Library version string. */
const char* sv_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SV_H */
