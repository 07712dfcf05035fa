// The C ABI of libsv (declared in include/sv.h): argument validation, handle
// and state bookkeeping, matrix staging, and dispatch to the HIP kernels.
// No exception crosses the ABI: every entry point catches and maps to a
// status code with a thread-local message.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "sv_batch.h"
#include "sv_internal.h"
#include "sv_tile.h"

namespace sv {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

// ------------------------------------------------- device memory budget

namespace {

std::atomic<uint64_t> g_hbm_used{0};
std::atomic<uint64_t> g_hbm_budget{0};  // 0: no cap
std::once_flag g_budget_env_once;

void read_budget_env()
{
    std::call_once(g_budget_env_once, [] {
        const char* v = std::getenv("SV_HBM_BUDGET_BYTES");
        if (v == nullptr || *v == 0) return;
        char* end = nullptr;
        const unsigned long long b = std::strtoull(v, &end, 10);
        if (end != nullptr && *end == 0) g_hbm_budget.store(b);
    });
}

}  // namespace

void budget_reserve(size_t bytes, const char* what)
{
    read_budget_env();
    const uint64_t cap = g_hbm_budget.load();
    uint64_t used = g_hbm_used.load();
    for (;;) {
        if (cap != 0 && (bytes > cap || used > cap - bytes))
            throw Error{SV_ERR_OUT_OF_MEMORY, std::string(what) + ": " + std::to_string(bytes) +
                                                  " B would exceed the HBM budget of " + std::to_string(cap) +
                                                  " B (" + std::to_string(used) + " B in use)"};
        if (g_hbm_used.compare_exchange_weak(used, used + bytes)) return;
    }
}

void budget_release(size_t bytes) { g_hbm_used.fetch_sub(bytes); }

void* dev_alloc(size_t bytes, const char* what)
{
    budget_reserve(bytes, what);
    void* p = nullptr;
    const hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        budget_release(bytes);
        (void)hipGetLastError();
        throw Error{e == hipErrorOutOfMemory ? SV_ERR_OUT_OF_MEMORY : SV_ERR_DEVICE,
                    std::string(what) + ": hipMalloc of " + std::to_string(bytes) + " B failed: " +
                        hipGetErrorString(e)};
    }
    return p;
}

void dev_free(void* p, size_t bytes)
{
    if (p == nullptr) return;
    (void)hipFree(p);
    budget_release(bytes);
}

sv_batch_s* batch_create(sv_handle_s* h, int n_circuits, const int32_t* n_qubits, const int32_t* gate_offsets,
                         const int32_t* codes, const int32_t* qubits, const double* params,
                         const int32_t* term_offsets, const uint64_t* z_masks, int max_fused_qubits);
void batch_run(sv_batch_s* b, void* states, double* expect_out, double* latency_s, double* kernel_s);
void batch_destroy(sv_batch_s* b);
void batch_layout(sv_batch_s* b, uint64_t* state_bytes, uint64_t* byte_offsets);
void batch_info(sv_batch_s* b, int n_qubits, int32_t* kmax, int32_t* blocks);
void batch_plan(sv_batch_s* b, int n_qubits, sv_batch_size_plan_t* out);
void batch_host_times(sv_batch_s* b, double* tune_s, double* build_s);
sv_fused_s* fuse(const sv_gate_t* gates, int n_gates, int kmax, int kdiag, bool coupled = false);
sv_fused_s* fuse_gate_list(const int32_t* codes, const int32_t* qubits, const double* params, int n_gates,
                           int kmax, int kdiag, bool coupled = false);
void gate_matrix(const char* name, const double* params, int n_params, double* out, int* n_targets,
                 int* n_controls);

namespace {

size_t amp_bytes(sv_dtype_t dt) { return dt == SV_C64 ? 8 : 16; }

template <typename F>
sv_status_t guarded(F&& f)
{
    try {
        f();
        return SV_OK;
    } catch (const Error& e) {
        set_error(e.msg);
        return e.status;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return SV_ERR_OUT_OF_MEMORY;
    } catch (...) {
        set_error("internal error");
        return SV_ERR_INTERNAL;
    }
}

void check_state(const sv_state_s* s)
{
    SV_CHECK(s != nullptr && s->h != nullptr && s->d != nullptr, "invalid state");
}

// Validates targets/controls of one gate on an n-qubit state and fills the
// sweep descriptor.
GateDesc make_desc(int n, const int32_t* targets, int k, const int32_t* controls, const int32_t* cvals,
                   int n_controls)
{
    SV_CHECK(k >= 1 && k <= SV_MAX_TARGETS, "k must be in [1, 10]");
    SV_CHECK(k <= n, "more targets than qubits");
    SV_CHECK(targets != nullptr, "targets is NULL");
    SV_CHECK(n_controls >= 0, "n_controls is negative");
    SV_CHECK(n_controls == 0 || controls != nullptr, "controls is NULL");
    SV_CHECK(k + n_controls <= n, "targets plus controls exceed the qubit count");
    GateDesc d;
    d.n = n;
    d.k = k;
    d.n_controls = n_controls;
    uint64_t used = 0;
    int minq = n;
    for (int a = 0; a < k; ++a) {
        const int q = targets[a];
        SV_CHECK(q >= 0 && q < n, "target out of range");
        SV_CHECK(!((used >> q) & 1), "repeated target");
        used |= uint64_t(1) << q;
        d.tbit[a] = uint64_t(1) << q;
        minq = std::min(minq, q);
    }
    d.min_target = minq;
    for (int a = 0; a < n_controls; ++a) {
        const int q = controls[a];
        SV_CHECK(q >= 0 && q < n, "control out of range");
        SV_CHECK(!((used >> q) & 1), "control repeats a target or another control");
        used |= uint64_t(1) << q;
        const int v = cvals ? cvals[a] : 1;
        SV_CHECK(v == 0 || v == 1, "control values must be 0 or 1");
        if (v) d.cval |= uint64_t(1) << q;
    }
    d.n_fixed = 0;
    for (int q = 0; q < n; ++q)
        if ((used >> q) & 1) d.fixed_sorted[d.n_fixed++] = q;
    d.n_groups = uint64_t(1) << (n - k - n_controls);
    return d;
}

// Dense uncontrolled gates on 2-4 qubits of a state of >= 14 qubits run as
// five-qubit gates M (x) I on their targets plus free qubits next to them
// (below the lowest target first, then above the highest): the five-qubit
// tile sweep, with its tuned variants, moves the state faster than the
// smaller gates' own kernels, and the result is the same gate.  The extra
// qubits are the high matrix bits; out_m is the 32 x 32 complex128 matrix.
bool pad_to_five(int n, int k, int n_controls, const int32_t* targets, const double* m, int32_t* out_t,
                 std::vector<double>& out_m)
{
    if (n_controls != 0 || k < 2 || k > 4 || n < 14) return false;
    uint64_t used = 0;
    int lo = n, hi = -1;
    for (int a = 0; a < k; ++a) {
        out_t[a] = targets[a];
        used |= uint64_t(1) << targets[a];
        lo = std::min(lo, int(targets[a]));
        hi = std::max(hi, int(targets[a]));
    }
    int kk = k;
    for (int q = lo - 1; q >= 0 && kk < 5; --q)
        if (!((used >> q) & 1)) out_t[kk++] = q;
    for (int q = hi + 1; q < n && kk < 5; ++q)
        if (!((used >> q) & 1)) out_t[kk++] = q;
    if (kk < 5) return false;
    const int d = 1 << k, D = 32;
    out_m.assign(size_t(2) * D * D, 0.0);
    for (int e = 0; e < D / d; ++e)
        for (int r = 0; r < d; ++r)
            for (int c = 0; c < d; ++c) {
                const size_t dst = size_t(e * d + r) * D + size_t(e * d + c);
                out_m[2 * dst] = m[2 * (size_t(r) * d + c)];
                out_m[2 * dst + 1] = m[2 * (size_t(r) * d + c) + 1];
            }
    return true;
}

void check_matrix_finite(const double* m, int k)
{
    SV_CHECK(m != nullptr, "matrix is NULL");
    const size_t n = size_t(2) << (2 * k);
    for (size_t i = 0; i < n; ++i) SV_CHECK(std::isfinite(m[i]), "matrix entry is not finite");
}

}  // namespace

// Matrix ring: the device region [0, kMatRingBytes) of the workspace mirrors
// the pinned host region of the same size, in kMatRingSegments segments.
// Before host bytes of a segment are rewritten, the copies that last read
// that segment must have completed: an event is recorded when the ring
// leaves a segment and waited on when it comes back to it.  On the device
// side, stream order puts every later copy after the kernels that read the
// earlier contents.
const void* stage_matrix(sv_handle_s* h, const void* host, size_t bytes)
{
    const size_t seg = kMatRingBytes / kMatRingSegments;
    bytes = (bytes + 255) & ~size_t(255);
    if (bytes > seg) {
        // large gates (k >= 9): copy into the scratch part of the workspace
        // and wait, so that the host buffer may be released on return
        SV_CHECK(kMatRingBytes + bytes <= h->ws_bytes, "matrix larger than the handle's workspace");
        char* dst = h->ws + kMatRingBytes;
        SV_HIP(hipMemcpyAsync(dst, host, bytes, hipMemcpyHostToDevice, h->stream));
        SV_HIP(hipStreamSynchronize(h->stream));
        return dst;
    }
    size_t pos = h->ring_pos;
    if ((pos % seg) + bytes > seg) pos = (pos / seg + 1) * seg;  // does not fit: next segment
    if (pos >= kMatRingBytes) pos = 0;
    const int new_seg = int(pos / seg);
    if (new_seg != h->ring_seg) {
        // leaving ring_seg: mark its last use; entering new_seg: wait for its last use
        SV_HIP(hipEventRecord(h->seg_event[h->ring_seg], h->stream));
        h->seg_event_live[h->ring_seg] = true;
        if (h->seg_event_live[new_seg]) {
            SV_HIP(hipEventSynchronize(h->seg_event[new_seg]));
            h->seg_event_live[new_seg] = false;
        }
        h->ring_seg = new_seg;
    }
    std::memcpy(h->pinned + pos, host, bytes);
    SV_HIP(hipMemcpyAsync(h->ws + pos, h->pinned + pos, bytes, hipMemcpyHostToDevice, h->stream));
    h->ring_pos = pos + bytes;
    return h->ws + pos;
}

char* ensure_aux(sv_handle_s* h, size_t bytes)
{
    bytes = (bytes + 255) & ~size_t(255);
    if (bytes <= h->aux_bytes) return h->aux;
    SV_HIP(hipStreamSynchronize(h->stream));
    if (h->aux) {
        dev_free(h->aux, h->aux_bytes);
        h->aux = nullptr;
        h->aux_bytes = 0;
    }
    h->aux = static_cast<char*>(dev_alloc(bytes, "sampler scratch"));
    h->aux_bytes = bytes;
    return h->aux;
}

}  // namespace sv

using namespace sv;

extern "C" {

const char* sv_last_error(void) { return g_last_error.c_str(); }

sv_status_t sv_set_hbm_budget(uint64_t bytes)
{
    return guarded([&] {
        read_budget_env();
        g_hbm_budget.store(bytes);
    });
}

sv_status_t sv_hbm_usage(uint64_t* used_bytes, uint64_t* budget_bytes)
{
    return guarded([&] {
        read_budget_env();
        if (used_bytes) *used_bytes = g_hbm_used.load();
        if (budget_bytes) *budget_bytes = g_hbm_budget.load();
    });
}

const char* sv_version(void) { return "libsv 0.1 (gfx950)"; }

sv_status_t sv_handle_create(sv_handle_t* out, void* hip_stream, size_t workspace_bytes)
{
    return guarded([&] {
        SV_CHECK(out != nullptr, "out is NULL");
        *out = nullptr;
        if (workspace_bytes == 0) workspace_bytes = kDefaultWorkspace;
        SV_CHECK(workspace_bytes >= kMinWorkspace, "workspace must be at least 12 MiB");
        // the budget is a host-side limit: checked before any device work
        budget_reserve(workspace_bytes, "handle workspace");
        budget_release(workspace_bytes);
        auto* h = new sv_handle_s;
        try {
            h->stream = static_cast<hipStream_t>(hip_stream);
            SV_HIP(hipGetDevice(&h->device));
            SV_HIP(hipDeviceGetAttribute(&h->cu_count, hipDeviceAttributeMultiprocessorCount, h->device));
            h->ws = static_cast<char*>(dev_alloc(workspace_bytes, "handle workspace"));
            h->ws_bytes = workspace_bytes;
            SV_HIP(hipHostMalloc(&h->pinned, kMatRingBytes, hipHostMallocDefault));
            h->pinned_bytes = kMatRingBytes;
            for (int i = 0; i < kMatRingSegments; ++i)
                SV_HIP(hipEventCreateWithFlags(&h->seg_event[i], hipEventDisableTiming));
            h->tuner = new TileTuner;
        } catch (...) {
            delete h->tuner;
            for (int i = 0; i < kMatRingSegments; ++i)
                if (h->seg_event[i]) (void)hipEventDestroy(h->seg_event[i]);
            if (h->pinned) (void)hipHostFree(h->pinned);
            dev_free(h->ws, h->ws_bytes);
            delete h;
            throw;
        }
        *out = h;
    });
}

sv_status_t sv_handle_destroy(sv_handle_t h)
{
    return guarded([&] {
        SV_CHECK(h != nullptr, "handle is NULL");
        const hipError_t e = hipStreamSynchronize(h->stream);
        for (int i = 0; i < kMatRingSegments; ++i)
            if (h->seg_event[i]) (void)hipEventDestroy(h->seg_event[i]);
        if (h->pinned) (void)hipHostFree(h->pinned);
        if (h->acc_pinned) (void)hipHostFree(h->acc_pinned);
        for (hipEvent_t ev : h->acc_event)
            if (ev) (void)hipEventDestroy(ev);
        dev_free(h->ws, h->ws_bytes);
        dev_free(h->aux, h->aux_bytes);
        if (h->tuner) {
            for (auto& t : h->tuner->pending) {
                (void)hipEventDestroy(t.e0);
                (void)hipEventDestroy(t.e1);
            }
            for (hipEvent_t ev : h->tuner->pool) (void)hipEventDestroy(ev);
            delete h->tuner;
        }
        delete h;
        SV_HIP(e);
    });
}

sv_status_t sv_handle_set_stream(sv_handle_t h, void* hip_stream)
{
    return guarded([&] {
        SV_CHECK(h != nullptr, "handle is NULL");
        h->stream = static_cast<hipStream_t>(hip_stream);
    });
}

sv_status_t sv_handle_set_tile_mode(sv_handle_t h, int32_t mode)
{
    return guarded([&] {
        SV_CHECK(h != nullptr, "handle is NULL");
        SV_CHECK(mode == SV_TILE_AUTO || mode == SV_TILE_NARROW || mode == SV_TILE_WIDE || mode == SV_TILE_SPREAD,
                 "tile mode must be SV_TILE_AUTO, SV_TILE_NARROW, SV_TILE_WIDE or SV_TILE_SPREAD");
        h->tile_mode = mode;
    });
}

sv_status_t sv_handle_set_batch_level_qubits(sv_handle_t h, int32_t n_qubits)
{
    return guarded([&] {
        SV_CHECK(h != nullptr, "handle is NULL");
        SV_CHECK(n_qubits >= SV_BATCH_LEVEL_MIN_QUBITS && n_qubits <= SV_BATCH_LEVEL_NONE,
                 "level-path qubit count must be in [SV_BATCH_LEVEL_MIN_QUBITS, SV_BATCH_LEVEL_NONE]");
        h->batch_level_qubits = n_qubits;
    });
}

sv_status_t sv_sync(sv_handle_t h)
{
    return guarded([&] {
        SV_CHECK(h != nullptr, "handle is NULL");
        SV_HIP(hipStreamSynchronize(h->stream));
    });
}

sv_status_t sv_create(sv_handle_t h, int32_t n_qubits, sv_dtype_t dtype, void* device_ptr, sv_state_t* out)
{
    return guarded([&] {
        SV_CHECK(out != nullptr, "out is NULL");
        *out = nullptr;
        SV_CHECK(h != nullptr, "handle is NULL");
        SV_CHECK(n_qubits >= 1 && n_qubits <= SV_MAX_QUBITS, "n_qubits must be in [1, 36]");
        SV_CHECK(dtype == SV_C64 || dtype == SV_C128, "dtype must be SV_C64 or SV_C128");
        SV_CHECK(device_ptr == nullptr || (reinterpret_cast<uintptr_t>(device_ptr) & 255) == 0,
                 "device_ptr must be 256-byte aligned");
        auto* s = new sv_state_s;
        s->h = h;
        s->n = n_qubits;
        s->dt = dtype;
        if (device_ptr) {
            s->d = device_ptr;
            s->owned = false;
        } else {
            const size_t bytes = amp_bytes(dtype) << n_qubits;
            try {
                s->d = dev_alloc(bytes, "state");
            } catch (...) {
                delete s;
                throw;
            }
            s->owned = true;
            try {
                launch_set_basis(h, dtype, s->d, n_qubits, 0);
            } catch (...) {
                dev_free(s->d, bytes);
                delete s;
                throw;
            }
        }
        *out = s;
    });
}

sv_status_t sv_destroy(sv_state_t s)
{
    return guarded([&] {
        SV_CHECK(s != nullptr, "state is NULL");
        hipError_t e = hipSuccess;
        if (s->owned) {
            e = hipStreamSynchronize(s->h->stream);
            dev_free(s->d, amp_bytes(s->dt) << s->n);
        }
        delete s;
        SV_HIP(e);
    });
}

sv_status_t sv_state_device_ptr(sv_state_t s, void** out)
{
    return guarded([&] {
        check_state(s);
        SV_CHECK(out != nullptr, "out is NULL");
        *out = s->d;
    });
}

sv_status_t sv_set_basis_state(sv_state_t s, uint64_t x)
{
    return guarded([&] {
        check_state(s);
        SV_CHECK(x < (uint64_t(1) << s->n), "basis index out of range");
        launch_set_basis(s->h, s->dt, s->d, s->n, x);
    });
}

sv_status_t sv_apply_matrix(sv_state_t s, const double* matrix, const int32_t* targets, int32_t k,
                            const int32_t* controls, const int32_t* control_values, int32_t n_controls,
                            int32_t adjoint)
{
    return guarded([&] {
        check_state(s);
        GateDesc d = make_desc(s->n, targets, k, controls, control_values, n_controls);
        check_matrix_finite(matrix, k);
        int32_t pt[SV_MAX_TARGETS];
        std::vector<double> pm;
        if (pad_to_five(s->n, k, n_controls, targets, matrix, pt, pm)) {
            d = make_desc(s->n, pt, 5, nullptr, nullptr, 0);
            matrix = pm.data();
            k = 5;
        }
        const size_t bytes = packed_matrix_bytes(s->dt, s->n, k, n_controls);
        std::vector<char> tmp(bytes);
        pack_matrix(s->dt, s->n, k, n_controls, matrix, adjoint, tmp.data());
        const void* dm = stage_matrix(s->h, tmp.data(), bytes);
        launch_apply(s->h, s->dt, s->d, dm, d);
    });
}

sv_status_t sv_apply_gen_permutation(sv_state_t s, const int64_t* perm, const double* diag, const int32_t* targets,
                                     int32_t k, const int32_t* controls, const int32_t* control_values,
                                     int32_t n_controls, int32_t adjoint)
{
    return guarded([&] {
        check_state(s);
        GateDesc d = make_desc(s->n, targets, k, controls, control_values, n_controls);
        SV_CHECK(diag != nullptr, "diag is NULL");
        const int dim = 1 << k;
        for (int i = 0; i < 2 * dim; ++i) SV_CHECK(std::isfinite(diag[i]), "diag entry is not finite");
        bool identity = true;
        if (perm != nullptr) {
            std::vector<char> seen(dim, 0);
            for (int r = 0; r < dim; ++r) {
                SV_CHECK(perm[r] >= 0 && perm[r] < dim && !seen[perm[r]], "perm is not a permutation of 0..2^k-1");
                seen[perm[r]] = 1;
                identity &= perm[r] == r;
            }
        }
        if (identity) {
            // a diagonal gate: one streaming pass over the control-satisfying amplitudes
            std::vector<char> tmp(gperm_table_bytes(s->dt, k, false));
            pack_gperm(s->dt, k, nullptr, diag, adjoint, tmp.data());
            const void* dt_ = stage_matrix(s->h, tmp.data(), tmp.size());
            launch_gperm(s->h, s->dt, s->d, dt_, d, false);
            return;
        }
        SV_CHECK(k + n_controls <= 6, "a permutation gate takes at most 6 qubits, controls included");
        // controls become the top matrix bits of an uncontrolled permutation
        // that leaves the rows with other control values alone
        const int kk = k + n_controls;
        const int dd = 1 << kk;
        std::vector<int64_t> p(dd);
        std::vector<double> dg(2 * dd);
        std::vector<int32_t> tg(kk);
        int want = 0;
        for (int a = 0; a < k; ++a) tg[a] = targets[a];
        for (int a = 0; a < n_controls; ++a) {
            tg[k + a] = controls[a];
            if (!control_values || control_values[a]) want |= 1 << a;
        }
        for (int r = 0; r < dd; ++r) {
            const int cb = r >> k, lo = r & (dim - 1);
            const bool on = cb == want;
            p[r] = on ? ((int64_t(cb) << k) | perm[lo]) : r;
            dg[2 * r] = on ? diag[2 * lo] : 1.0;
            dg[2 * r + 1] = on ? diag[2 * lo + 1] : 0.0;
        }
        d = make_desc(s->n, tg.data(), kk, nullptr, nullptr, 0);
        if (s->n < (s->dt == SV_C64 ? 12 : 11)) {
            // small states: the dense sweep with G written out
            std::vector<double> m(size_t(2) * dd * dd, 0.0);
            for (int r = 0; r < dd; ++r) {
                m[2 * (size_t(r) * dd + p[r])] = dg[2 * r];
                m[2 * (size_t(r) * dd + p[r]) + 1] = dg[2 * r + 1];
            }
            const size_t bytes = packed_matrix_bytes(s->dt, s->n, kk, 0);
            std::vector<char> tmp(bytes);
            pack_matrix(s->dt, s->n, kk, 0, m.data(), adjoint, tmp.data());
            launch_apply(s->h, s->dt, s->d, stage_matrix(s->h, tmp.data(), bytes), d);
            return;
        }
        std::vector<char> tmp(gperm_table_bytes(s->dt, kk, true));
        pack_gperm(s->dt, kk, p.data(), dg.data(), adjoint, tmp.data());
        launch_gperm(s->h, s->dt, s->d, stage_matrix(s->h, tmp.data(), tmp.size()), d, true);
    });
}

sv_status_t sv_gate_matrix(const char* name, const double* params, int32_t n_params, double* matrix_out,
                           int32_t* n_targets, int32_t* n_controls)
{
    return guarded([&] {
        int nt = 0, nc = 0;
        gate_matrix(name, params, n_params, matrix_out, &nt, &nc);
        if (n_targets) *n_targets = nt;
        if (n_controls) *n_controls = nc;
    });
}

sv_status_t sv_fuse_gates(const sv_gate_t* gates, int32_t n_gates, int32_t max_fused_qubits, sv_fused_t* out)
{
    return guarded([&] {
        SV_CHECK(out != nullptr, "out is NULL");
        *out = nullptr;
        *out = fuse(gates, n_gates, max_fused_qubits, 0);
    });
}

sv_status_t sv_fuse_gates_diag(const sv_gate_t* gates, int32_t n_gates, int32_t max_fused_qubits,
                               int32_t max_fused_diagonal_qubits, sv_fused_t* out)
{
    return guarded([&] {
        SV_CHECK(out != nullptr, "out is NULL");
        *out = nullptr;
        *out = fuse(gates, n_gates, max_fused_qubits, max_fused_diagonal_qubits);
    });
}

sv_status_t sv_fuse_gate_list(const int32_t* codes, const int32_t* qubits, const double* params, int32_t n_gates,
                              int32_t max_fused_qubits, sv_fused_t* out)
{
    return guarded([&] {
        SV_CHECK(out != nullptr, "out is NULL");
        *out = nullptr;
        *out = fuse_gate_list(codes, qubits, params, n_gates, max_fused_qubits, 0);
    });
}

sv_status_t sv_fuse_gate_list_diag(const int32_t* codes, const int32_t* qubits, const double* params,
                                   int32_t n_gates, int32_t max_fused_qubits, int32_t max_fused_diagonal_qubits,
                                   sv_fused_t* out)
{
    return guarded([&] {
        SV_CHECK(out != nullptr, "out is NULL");
        *out = nullptr;
        *out = fuse_gate_list(codes, qubits, params, n_gates, max_fused_qubits, max_fused_diagonal_qubits);
    });
}

sv_status_t sv_fuse_gates_coupled(const sv_gate_t* gates, int32_t n_gates, int32_t max_fused_qubits, sv_fused_t* out)
{
    return guarded([&] {
        SV_CHECK(out != nullptr, "out is NULL");
        *out = nullptr;
        *out = fuse(gates, n_gates, max_fused_qubits, 0, true);
    });
}

sv_status_t sv_fuse_gate_list_coupled(const int32_t* codes, const int32_t* qubits, const double* params,
                                      int32_t n_gates, int32_t max_fused_qubits, sv_fused_t* out)
{
    return guarded([&] {
        SV_CHECK(out != nullptr, "out is NULL");
        *out = nullptr;
        *out = fuse_gate_list(codes, qubits, params, n_gates, max_fused_qubits, 0, true);
    });
}

sv_status_t sv_fused_block_coupling(sv_fused_t f, int32_t i, int32_t* n_coupled, int32_t* coupled_qubits,
                                    double* phases)
{
    return guarded([&] {
        SV_CHECK(f != nullptr && n_coupled != nullptr, "NULL argument");
        SV_CHECK(i >= 0 && i < f->n_blocks, "block index out of range");
        const FusedBlock& b = f->blocks[i];
        *n_coupled = b.n_couple;
        if (coupled_qubits)
            for (int c = 0; c < b.n_couple; ++c) coupled_qubits[c] = b.couple_q[c];
        if (phases && b.n_couple > 0) std::memcpy(phases, b.couple, sizeof(double) * size_t(b.k) * b.n_couple);
    });
}

sv_status_t sv_fused_count(sv_fused_t f, int32_t* n_blocks)
{
    return guarded([&] {
        SV_CHECK(f != nullptr && n_blocks != nullptr, "NULL argument");
        *n_blocks = f->n_blocks;
    });
}

sv_status_t sv_fused_block(sv_fused_t f, int32_t i, int32_t* k, int32_t* targets, double* matrix)
{
    return guarded([&] {
        SV_CHECK(f != nullptr && k != nullptr && targets != nullptr, "NULL argument");
        SV_CHECK(i >= 0 && i < f->n_blocks, "block index out of range");
        const FusedBlock& b = f->blocks[i];
        *k = b.k;
        for (int a = 0; a < b.k; ++a) targets[a] = b.targets[a];
        if (matrix) std::memcpy(matrix, b.m, sizeof(double) * (size_t(2) << (b.diagonal ? b.k : 2 * b.k)));
    });
}

sv_status_t sv_fused_block_is_diagonal(sv_fused_t f, int32_t i, int32_t* diagonal)
{
    return guarded([&] {
        SV_CHECK(f != nullptr && diagonal != nullptr, "NULL argument");
        SV_CHECK(i >= 0 && i < f->n_blocks, "block index out of range");
        *diagonal = f->blocks[i].diagonal ? 1 : 0;
    });
}

sv_status_t sv_fused_free(sv_fused_t f)
{
    return guarded([&] {
        if (!f) return;
        delete[] f->blocks;
        delete[] f->storage;
        delete f;
    });
}

}  // extern "C"

namespace sv {
namespace {

// A block of coupled fusion on 1-4 qubits of a state of >= 14 qubits as a
// five-qubit block: pad qubits as pad_to_five takes them, the matrix
// M (x) I, and a coupling term of a block qubit with a pad qubit becomes a
// phase inside the block (its columns with both bits set scaled, since the
// coupling acts before M); the other coupled qubits stay coupled.
bool pad_coupled_to_five(int n, const FusedBlock& b, FusedBlock& out, std::vector<double>& mstore,
                         std::vector<double>& cstore)
{
    if (b.k < 1 || b.k >= 5 || n < 14) return false;
    uint64_t used = 0;
    int lo = n, hi = -1;
    int t[5];
    for (int a = 0; a < b.k; ++a) {
        t[a] = b.targets[a];
        used |= uint64_t(1) << t[a];
        lo = std::min(lo, t[a]);
        hi = std::max(hi, t[a]);
    }
    int kk = b.k;
    for (int q = lo - 1; q >= 0 && kk < 5; --q)
        if (!((used >> q) & 1)) t[kk++] = q;
    for (int q = hi + 1; q < n && kk < 5; ++q)
        if (!((used >> q) & 1)) t[kk++] = q;
    if (kk < 5) return false;
    const int d = 1 << b.k, D = 32;
    mstore.assign(size_t(2) * D * D, 0.0);
    for (int e = 0; e < D / d; ++e)
        for (int r = 0; r < d; ++r)
            for (int c = 0; c < d; ++c) {
                const size_t dst = size_t(e * d + r) * D + size_t(e * d + c);
                mstore[2 * dst] = b.m[2 * (size_t(r) * d + c)];
                mstore[2 * dst + 1] = b.m[2 * (size_t(r) * d + c) + 1];
            }
    out = b;
    out.k = 5;
    for (int a = 0; a < 5; ++a) out.targets[a] = t[a];
    out.m = mstore.data();
    std::vector<int> keep;
    for (int c = 0; c < b.n_couple; ++c) {
        int pad = -1;
        for (int a = b.k; a < 5; ++a)
            if (t[a] == b.couple_q[c]) pad = a;
        if (pad < 0) {
            keep.push_back(c);
            continue;
        }
        for (int a = 0; a < b.k; ++a) {
            const double ph = b.couple[size_t(a) * b.n_couple + c];
            if (ph == 0.0) continue;
            const double er = std::cos(ph), ei = std::sin(ph);
            for (int col = 0; col < D; ++col) {
                if (!((col >> a) & 1) || !((col >> pad) & 1)) continue;
                for (int row = 0; row < D; ++row) {
                    double* u = &mstore[2 * (size_t(row) * D + col)];
                    const double ur = u[0], ui = u[1];
                    u[0] = ur * er - ui * ei;
                    u[1] = ur * ei + ui * er;
                }
            }
        }
    }
    out.n_couple = int(keep.size());
    cstore.assign(size_t(5) * keep.size(), 0.0);
    for (size_t j = 0; j < keep.size(); ++j) {
        out.couple_q[j] = b.couple_q[keep[j]];
        for (int a = 0; a < b.k; ++a) cstore[size_t(a) * keep.size() + j] = b.couple[size_t(a) * b.n_couple + keep[j]];
    }
    out.couple = cstore.data();
    return true;
}

// The blocks as launched: dense blocks on 2-4 qubits of a large state padded
// to five qubits (pad_to_five; blocks of coupled fusion from 1 qubit up,
// pad_coupled_to_five), all others as they are.
void effective_blocks(int n, const sv_fused_s* f, int first, int end, std::vector<FusedBlock>& eff,
                      std::vector<std::vector<double>>& padm, std::vector<std::vector<double>>& padc)
{
    eff.assign(f->blocks, f->blocks + f->n_blocks);
    padm.resize(f->n_blocks);
    padc.resize(f->n_blocks);
    for (int b = first; b < end; ++b) {
        FusedBlock& blk = eff[b];
        if (blk.diagonal) continue;
        if (blk.n_couple > 0) {
            FusedBlock out;
            if (pad_coupled_to_five(n, blk, out, padm[b], padc[b])) blk = out;
            continue;
        }
        int32_t pt[SV_MAX_TARGETS];
        int32_t t[SV_MAX_TARGETS];
        for (int a = 0; a < blk.k; ++a) t[a] = blk.targets[a];
        if (pad_to_five(n, blk.k, 0, t, blk.m, pt, padm[b])) {
            blk.k = 5;
            for (int a = 0; a < 5; ++a) blk.targets[a] = pt[a];
            blk.m = padm[b].data();
        }
    }
}

// A fused block's device form and sweep: the dense sweep, or for a diagonal
// block the diagonal sweep; a block with a phase coupling carries it (a
// CoupleDev) after its matrix, 256-byte aligned.
size_t matrix_part_bytes(const sv_state_s* s, const FusedBlock& b)
{
    return b.diagonal ? gperm_table_bytes(s->dt, b.k, false) : packed_matrix_bytes(s->dt, s->n, b.k, 0);
}

size_t block_bytes(const sv_state_s* s, const FusedBlock& b)
{
    const size_t m = matrix_part_bytes(s, b);
    return b.n_couple > 0 ? ((m + 255) & ~size_t(255)) + sizeof(CoupleDev) : m;
}

void pack_block(const sv_state_s* s, const FusedBlock& b, void* dst)
{
    if (b.diagonal)
        pack_gperm(s->dt, b.k, nullptr, b.m, 0, dst);
    else
        pack_matrix(s->dt, s->n, b.k, 0, b.m, 0, dst);
    if (b.n_couple > 0) {
        CoupleDev cd{};
        cd.n = b.n_couple;
        cd.k = b.k;
        for (int c = 0; c < b.n_couple; ++c) cd.q[c] = b.couple_q[c];
        for (int a = 0; a < b.k; ++a) cd.t[a] = b.targets[a];
        for (int a = 0; a < b.k; ++a)
            for (int c = 0; c < b.n_couple; ++c)
                cd.phase[a * SV_MAX_QUBITS + c] = b.couple[size_t(a) * b.n_couple + c] / M_PI;
        const size_t off = (matrix_part_bytes(s, b) + 255) & ~size_t(255);
        std::memcpy(static_cast<char*>(dst) + off, &cd, sizeof(cd));
    }
}

void launch_block(sv_handle_s* h, const sv_state_s* s, const FusedBlock& b, const void* dm, const GateDesc& d)
{
    if (b.diagonal)
        launch_gperm(h, s->dt, s->d, dm, d, false);
    else if (b.n_couple > 0)
        launch_apply_coupled(h, s->dt, s->d, dm,
                             static_cast<const char*>(dm) + ((matrix_part_bytes(s, b) + 255) & ~size_t(255)), d);
    else
        launch_apply(h, s->dt, s->d, dm, d);
}

void apply_fused_blocks(sv_state_s* s, sv_fused_s* f, int first, int count)
{
    check_state(s);
    SV_CHECK(f != nullptr, "fused gates are NULL");
    SV_CHECK(first >= 0 && count >= 0 && first <= f->n_blocks && count <= f->n_blocks - first,
             "block range out of bounds");
    const int end = first + count;
    std::vector<GateDesc> descs(f->n_blocks);
    std::vector<std::vector<double>> padm, padc;
    std::vector<FusedBlock> eff;
    effective_blocks(s->n, f, first, end, eff, padm, padc);
    for (int b = first; b < end; ++b) {
        const FusedBlock& blk = eff[b];
        descs[b] = make_desc(s->n, blk.targets, blk.k, nullptr, nullptr, 0);
    }
    {
        // stage in segment-sized batches: one copy per batch of blocks
        const size_t seg = kMatRingBytes / kMatRingSegments;
        int b = first;
        while (b < end) {
            std::vector<size_t> offs;
            size_t bytes = 0;
            int e = b;
            while (e < end) {
                const size_t mb = (block_bytes(s, eff[e]) + 255) & ~size_t(255);
                if (bytes + mb > seg) break;
                offs.push_back(bytes);
                bytes += mb;
                ++e;
            }
            if (e == b) {
                // one block larger than a ring segment: stage it on its own
                const size_t mb = block_bytes(s, eff[b]);
                std::vector<char> one(mb);
                pack_block(s, eff[b], one.data());
                launch_block(s->h, s, eff[b], stage_matrix(s->h, one.data(), mb), descs[b]);
                ++b;
                continue;
            }
            std::vector<char> tmp(bytes);
            for (int j = b; j < e; ++j) pack_block(s, eff[j], tmp.data() + offs[j - b]);
            const char* dm = static_cast<const char*>(stage_matrix(s->h, tmp.data(), bytes));
            for (int j = b; j < e; ++j) launch_block(s->h, s, eff[j], dm + offs[j - b], descs[j]);
            b = e;
        }
    }
}

}  // namespace
}  // namespace sv

extern "C" {

sv_status_t sv_apply_fused(sv_state_t s, sv_fused_t f)
{
    return guarded([&] {
        SV_CHECK(f != nullptr, "fused gates are NULL");
        apply_fused_blocks(s, f, 0, f->n_blocks);
    });
}

sv_status_t sv_apply_fused_range(sv_state_t s, sv_fused_t f, int32_t first, int32_t count)
{
    return guarded([&] { apply_fused_blocks(s, f, first, count); });
}

struct sv_graph_s {
    sv_state_s* s = nullptr;
    char* mats = nullptr;  // packed block matrices, device
    size_t mats_bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

sv_status_t sv_graph_create(sv_state_t s, sv_fused_t f, sv_graph_t* out)
{
    return guarded([&] {
        SV_CHECK(out != nullptr, "out is NULL");
        *out = nullptr;
        check_state(s);
        SV_CHECK(f != nullptr, "fused gates are NULL");
        sv_handle_s* h = s->h;
        std::vector<GateDesc> descs(f->n_blocks);
        std::vector<size_t> offs(f->n_blocks);
        std::vector<std::vector<double>> padm, padc;
        std::vector<FusedBlock> eff;
        effective_blocks(s->n, f, 0, f->n_blocks, eff, padm, padc);
        size_t bytes = 0;
        for (int b = 0; b < f->n_blocks; ++b) {
            const FusedBlock& blk = eff[b];
            descs[b] = make_desc(s->n, blk.targets, blk.k, nullptr, nullptr, 0);
            offs[b] = bytes;
            bytes += (block_bytes(s, blk) + 255) & ~size_t(255);
        }
        std::vector<char> host(bytes ? bytes : 1);
        for (int b = 0; b < f->n_blocks; ++b) pack_block(s, eff[b], host.data() + offs[b]);
        auto* g = new sv_graph_s;
        g->s = s;
        hipStream_t cap = nullptr;
        hipStream_t saved = h->stream;
        try {
            g->mats = static_cast<char*>(dev_alloc(host.size(), "recorded program matrices"));
            g->mats_bytes = host.size();
            SV_HIP(hipMemcpy(g->mats, host.data(), host.size(), hipMemcpyHostToDevice));
            // record on a private stream: the handle's own stream may be the
            // null stream, which cannot be captured
            SV_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
            h->stream = cap;
            SV_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed));
            try {
                for (int b = 0; b < f->n_blocks; ++b) launch_block(h, s, eff[b], g->mats + offs[b], descs[b]);
            } catch (...) {
                hipGraph_t dropped = nullptr;
                (void)hipStreamEndCapture(cap, &dropped);
                if (dropped) (void)hipGraphDestroy(dropped);
                throw;
            }
            SV_HIP(hipStreamEndCapture(cap, &g->graph));
            h->stream = saved;
            SV_HIP(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
            SV_HIP(hipStreamDestroy(cap));
            cap = nullptr;
        } catch (...) {
            h->stream = saved;
            if (cap) (void)hipStreamDestroy(cap);
            if (g->exec) (void)hipGraphExecDestroy(g->exec);
            if (g->graph) (void)hipGraphDestroy(g->graph);
            dev_free(g->mats, g->mats_bytes);
            delete g;
            throw;
        }
        *out = g;
    });
}

sv_status_t sv_graph_launch(sv_graph_t g)
{
    return guarded([&] {
        SV_CHECK(g != nullptr, "graph is NULL");
        check_state(g->s);
        SV_HIP(hipGraphLaunch(g->exec, g->s->h->stream));
    });
}

sv_status_t sv_graph_destroy(sv_graph_t g)
{
    return guarded([&] {
        SV_CHECK(g != nullptr, "graph is NULL");
        const hipError_t e = hipStreamSynchronize(g->s->h->stream);
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        dev_free(g->mats, g->mats_bytes);
        delete g;
        SV_HIP(e);
    });
}

sv_status_t sv_norm(sv_state_t s, double* out)
{
    return guarded([&] {
        check_state(s);
        SV_CHECK(out != nullptr, "out is NULL");
        *out = run_norm(s->h, s->dt, s->d, s->n);
    });
}

sv_status_t sv_renormalize(sv_state_t s, double* norm_out)
{
    return guarded([&] {
        check_state(s);
        const double nrm = run_norm(s->h, s->dt, s->d, s->n);
        SV_CHECK(nrm > 0.0 && std::isfinite(nrm), "state norm is zero or not finite");
        launch_scale(s->h, s->dt, s->d, s->n, 1.0 / std::sqrt(nrm));
        if (norm_out) *norm_out = nrm;
    });
}

sv_status_t sv_expect_pauli(sv_state_t s, const sv_pauli_term_t* terms, int32_t n_terms, double* out)
{
    return guarded([&] {
        check_state(s);
        SV_CHECK(n_terms >= 0, "n_terms is negative");
        SV_CHECK(n_terms == 0 || (terms != nullptr && out != nullptr), "NULL argument");
        std::vector<PauliMasks> pm(n_terms);
        for (int t = 0; t < n_terms; ++t) {
            const sv_pauli_term_t& T = terms[t];
            SV_CHECK(T.n_ops >= 0 && T.n_ops <= s->n, "term has a bad number of operators");
            SV_CHECK(T.n_ops == 0 || (T.qubits && T.ops), "term has NULL arrays");
            uint64_t seen = 0;
            for (int a = 0; a < T.n_ops; ++a) {
                const int q = T.qubits[a];
                SV_CHECK(q >= 0 && q < s->n, "Pauli qubit out of range");
                SV_CHECK(!((seen >> q) & 1), "Pauli term names a qubit twice");
                seen |= uint64_t(1) << q;
                const uint64_t b = uint64_t(1) << q;
                switch (T.ops[a]) {
                    case 'I': break;
                    case 'X': pm[t].x |= b; break;
                    case 'Y': pm[t].x |= b; pm[t].z |= b; pm[t].ny++; break;
                    case 'Z': pm[t].z |= b; break;
                    default: SV_CHECK(false, "Pauli operator must be one of I, X, Y, Z");
                }
            }
        }
        if (n_terms > 0) run_expect(s->h, s->dt, s->d, s->n, pm.data(), n_terms, out);
    });
}

}  // extern "C"

namespace sv {
namespace {

// Distinct measured qubits of a state: their mask.
uint64_t measured_mask(const sv_state_s* s, const int32_t* qubits, int m, int max_m)
{
    SV_CHECK(m >= 1 && m <= max_m && m <= s->n, "bad number of measured qubits");
    SV_CHECK(qubits != nullptr, "qubits is NULL");
    uint64_t mask = 0;
    for (int a = 0; a < m; ++a) {
        SV_CHECK(qubits[a] >= 0 && qubits[a] < s->n, "measured qubit out of range");
        SV_CHECK(!((mask >> qubits[a]) & 1), "measured qubit repeated");
        mask |= uint64_t(1) << qubits[a];
    }
    return mask;
}

uint64_t outcome_bits(const int32_t* qubits, int m, uint64_t outcome)
{
    uint64_t o = 0;
    for (int a = 0; a < m; ++a)
        if ((outcome >> a) & 1) o |= uint64_t(1) << qubits[a];
    return o;
}

PauliMasks pauli_masks(const sv_state_s* s, const sv_pauli_term_t& T, uint64_t* used)
{
    PauliMasks pm;
    SV_CHECK(T.n_ops >= 0 && T.n_ops <= s->n, "term has a bad number of operators");
    SV_CHECK(T.n_ops == 0 || (T.qubits && T.ops), "term has NULL arrays");
    for (int a = 0; a < T.n_ops; ++a) {
        const int q = T.qubits[a];
        SV_CHECK(q >= 0 && q < s->n, "Pauli qubit out of range");
        SV_CHECK(!((*used >> q) & 1), "Pauli term names a qubit twice");
        *used |= uint64_t(1) << q;
        const uint64_t b = uint64_t(1) << q;
        switch (T.ops[a]) {
            case 'I': break;
            case 'X': pm.x |= b; break;
            case 'Y': pm.x |= b; pm.z |= b; pm.ny++; break;
            case 'Z': pm.z |= b; break;
            default: SV_CHECK(false, "Pauli operator must be one of I, X, Y, Z");
        }
    }
    return pm;
}

}  // namespace
}  // namespace sv

extern "C" {

sv_status_t sv_apply_pauli_rotation(sv_state_t s, double theta, const sv_pauli_term_t* term, const int32_t* controls,
                                    const int32_t* control_values, int32_t n_controls)
{
    return guarded([&] {
        check_state(s);
        SV_CHECK(term != nullptr, "term is NULL");
        SV_CHECK(std::isfinite(theta), "theta is not finite");
        uint64_t used = 0;
        const PauliMasks pm = pauli_masks(s, *term, &used);
        SV_CHECK(n_controls >= 0 && (n_controls == 0 || controls != nullptr), "bad controls");
        for (int a = 0; a < n_controls; ++a) {
            const int q = controls[a];
            SV_CHECK(q >= 0 && q < s->n, "control out of range");
            SV_CHECK(!((used >> q) & 1), "control repeats a Pauli qubit or another control");
            used |= uint64_t(1) << q;
            const int v = control_values ? control_values[a] : 1;
            SV_CHECK(v == 0 || v == 1, "control values must be 0 or 1");
        }
        launch_pauli_rotation(s->h, s->dt, s->d, s->n, pm, theta, controls, control_values, n_controls);
    });
}

sv_status_t sv_measure_probabilities(sv_state_t s, const int32_t* qubits, int32_t m, double* probs)
{
    return guarded([&] {
        check_state(s);
        measured_mask(s, qubits, m, SV_MAX_TARGETS);
        SV_CHECK(probs != nullptr, "probs is NULL");
        run_measure_probs(s->h, s->dt, s->d, s->n, qubits, m, probs);
    });
}

sv_status_t sv_zbasis_probabilities(sv_state_t s, const int32_t* qubits, int32_t m, double* p_even, double* p_odd)
{
    return guarded([&] {
        check_state(s);
        const uint64_t mask = measured_mask(s, qubits, m, s->n);
        SV_CHECK(p_even != nullptr && p_odd != nullptr, "NULL output");
        double r[2];
        run_parity_probs(s->h, s->dt, s->d, s->n, mask, r);
        *p_even = r[0];
        *p_odd = r[1];
    });
}

sv_status_t sv_collapse(sv_state_t s, const int32_t* qubits, int32_t m, uint64_t outcome, double norm)
{
    return guarded([&] {
        check_state(s);
        const uint64_t mask = measured_mask(s, qubits, m, s->n);
        SV_CHECK(m >= 64 || outcome < (uint64_t(1) << m), "outcome has bits beyond the measured qubits");
        SV_CHECK(norm > 0.0 && std::isfinite(norm), "norm must be positive and finite");
        launch_collapse(s->h, s->dt, s->d, s->n, mask, outcome_bits(qubits, m, outcome), 0, -1, 1.0 / std::sqrt(norm));
    });
}

sv_status_t sv_collapse_zbasis(sv_state_t s, const int32_t* qubits, int32_t m, int32_t parity, double norm)
{
    return guarded([&] {
        check_state(s);
        const uint64_t mask = measured_mask(s, qubits, m, s->n);
        SV_CHECK(parity == 0 || parity == 1, "parity must be 0 or 1");
        SV_CHECK(norm > 0.0 && std::isfinite(norm), "norm must be positive and finite");
        launch_collapse(s->h, s->dt, s->d, s->n, 0, 0, mask, parity, 1.0 / std::sqrt(norm));
    });
}

sv_status_t sv_measure_zbasis(sv_state_t s, const int32_t* qubits, int32_t m, double randnum, int32_t collapse,
                              int32_t* parity)
{
    return guarded([&] {
        check_state(s);
        const uint64_t mask = measured_mask(s, qubits, m, s->n);
        SV_CHECK(parity != nullptr, "parity is NULL");
        SV_CHECK(randnum >= 0.0 && randnum < 1.0, "randnum must lie in [0, 1)");
        double r[2];
        run_parity_probs(s->h, s->dt, s->d, s->n, mask, r);
        const double total = r[0] + r[1];
        SV_CHECK(total > 0.0 && std::isfinite(total), "state norm is zero or not finite");
        const int par = randnum * total < r[0] ? 0 : 1;
        *parity = par;
        if (collapse) launch_collapse(s->h, s->dt, s->d, s->n, 0, 0, mask, par, 1.0 / std::sqrt(r[par]));
    });
}

sv_status_t sv_batch_measure(sv_state_t s, const int32_t* qubits, int32_t m, double randnum, int32_t collapse,
                             uint64_t* outcome)
{
    return guarded([&] {
        check_state(s);
        const uint64_t mask = measured_mask(s, qubits, m, SV_MAX_TARGETS);
        SV_CHECK(outcome != nullptr, "outcome is NULL");
        SV_CHECK(randnum >= 0.0 && randnum < 1.0, "randnum must lie in [0, 1)");
        std::vector<double> p(size_t(1) << m);
        run_measure_probs(s->h, s->dt, s->d, s->n, qubits, m, p.data());
        // running sums in outcome order; the outcome is the first whose
        // running sum exceeds randnum times the total
        std::vector<double> c(p.size());
        double acc = 0.0;
        for (size_t b = 0; b < p.size(); ++b) c[b] = acc = acc + p[b];
        SV_CHECK(acc > 0.0 && std::isfinite(acc), "state norm is zero or not finite");
        const double r = randnum * acc;
        size_t b = 0;
        while (b + 1 < c.size() && !(r < c[b])) ++b;
        *outcome = b;
        if (collapse) launch_collapse(s->h, s->dt, s->d, s->n, mask, outcome_bits(qubits, m, b), 0, -1, 1.0 / std::sqrt(p[b]));
    });
}

sv_status_t sv_swap_index_bits(sv_state_t s, const int32_t* pairs, int32_t n_pairs, const int32_t* mask_bits,
                               const int32_t* mask_values, int32_t n_mask)
{
    return guarded([&] {
        check_state(s);
        SV_CHECK(n_pairs >= 0 && n_mask >= 0, "negative count");
        SV_CHECK(n_pairs == 0 || pairs != nullptr, "pairs is NULL");
        SV_CHECK(n_mask == 0 || (mask_bits != nullptr && mask_values != nullptr), "mask arrays are NULL");
        SV_CHECK(2 * n_pairs + n_mask <= s->n, "more bits than qubits");
        uint64_t used = 0;
        for (int a = 0; a < 2 * n_pairs; ++a) {
            SV_CHECK(pairs[a] >= 0 && pairs[a] < s->n, "swapped bit out of range");
            SV_CHECK(!((used >> pairs[a]) & 1), "a bit appears twice among the pairs");
            used |= uint64_t(1) << pairs[a];
        }
        for (int a = 0; a < n_mask; ++a) {
            SV_CHECK(mask_bits[a] >= 0 && mask_bits[a] < s->n, "mask bit out of range");
            SV_CHECK(!((used >> mask_bits[a]) & 1), "mask bit repeats a swapped or mask bit");
            used |= uint64_t(1) << mask_bits[a];
            SV_CHECK(mask_values[a] == 0 || mask_values[a] == 1, "mask values must be 0 or 1");
        }
        if (n_pairs == 0) return;
        const int kk = 2 * n_pairs + n_mask;
        if (kk <= 6 && s->n >= (s->dt == SV_C64 ? 12 : 11)) {
            // up to 6 bits: the swap is a permutation gate on the pair bits
            // (matrix bits 2p, 2p + 1) and the mask bits (the bits above),
            // run by the LDS-tile permutation sweep: every amplitude read and
            // written once in 16-byte vectors, instead of scattered 8-byte
            // moves of the amplitudes that change place
            const int dd = 1 << kk;
            std::vector<int32_t> tg(kk);
            for (int a = 0; a < 2 * n_pairs; ++a) tg[a] = pairs[a];
            int want = 0;
            for (int a = 0; a < n_mask; ++a) {
                tg[2 * n_pairs + a] = mask_bits[a];
                want |= mask_values[a] << a;
            }
            std::vector<int64_t> perm(dd);
            std::vector<double> diag(2 * size_t(dd), 0.0);
            for (int r = 0; r < dd; ++r) {
                int q = r;
                if ((r >> (2 * n_pairs)) == want)
                    for (int p = 0; p < n_pairs; ++p) {
                        const int x = (r >> (2 * p)) & 1, y = (r >> (2 * p + 1)) & 1;
                        q = (q & ~(3 << (2 * p))) | (y << (2 * p)) | (x << (2 * p + 1));
                    }
                perm[r] = q;  // an involution: output r takes input q
                diag[2 * r] = 1.0;
            }
            const GateDesc d = make_desc(s->n, tg.data(), kk, nullptr, nullptr, 0);
            std::vector<char> tmp(gperm_table_bytes(s->dt, kk, true));
            pack_gperm(s->dt, kk, perm.data(), diag.data(), 0, tmp.data());
            launch_gperm(s->h, s->dt, s->d, stage_matrix(s->h, tmp.data(), tmp.size()), d, true);
            return;
        }
        launch_swap_bits(s->h, s->dt, s->d, s->n, pairs, n_pairs, mask_bits, mask_values, n_mask);
    });
}

namespace {
void check_access(const sv_state_s* s, const int32_t* ordering, int32_t n_bits, const int32_t* mask_bits,
                  const int32_t* mask_values, int32_t n_mask, const void* host, int64_t begin, int64_t end)
{
    SV_CHECK(n_bits >= 0 && n_mask >= 0 && n_bits + n_mask == s->n, "ordering plus mask bits must cover every qubit");
    SV_CHECK(n_bits == 0 || ordering != nullptr, "ordering is NULL");
    SV_CHECK(n_mask == 0 || (mask_bits != nullptr && mask_values != nullptr), "mask arrays are NULL");
    uint64_t used = 0;
    for (int a = 0; a < n_bits; ++a) {
        SV_CHECK(ordering[a] >= 0 && ordering[a] < s->n, "ordering bit out of range");
        SV_CHECK(!((used >> ordering[a]) & 1), "ordering repeats a bit");
        used |= uint64_t(1) << ordering[a];
    }
    for (int a = 0; a < n_mask; ++a) {
        SV_CHECK(mask_bits[a] >= 0 && mask_bits[a] < s->n, "mask bit out of range");
        SV_CHECK(!((used >> mask_bits[a]) & 1), "mask bit repeats a bit");
        used |= uint64_t(1) << mask_bits[a];
        SV_CHECK(mask_values[a] == 0 || mask_values[a] == 1, "mask values must be 0 or 1");
    }
    SV_CHECK(begin >= 0 && begin <= end && uint64_t(end) <= (uint64_t(1) << n_bits), "range out of bounds");
    SV_CHECK(begin == end || host != nullptr, "host buffer is NULL");
}
}  // namespace

sv_status_t sv_accessor_get(sv_state_t s, const int32_t* ordering, int32_t n_bits, const int32_t* mask_bits,
                            const int32_t* mask_values, int32_t n_mask, void* dst, int64_t begin, int64_t end)
{
    return guarded([&] {
        check_state(s);
        check_access(s, ordering, n_bits, mask_bits, mask_values, n_mask, dst, begin, end);
        if (begin < end)
            run_accessor(s->h, s->dt, s->d, s->n, ordering, n_bits, mask_bits, mask_values, n_mask, dst, begin, end,
                         false);
    });
}

sv_status_t sv_accessor_set(sv_state_t s, const int32_t* ordering, int32_t n_bits, const int32_t* mask_bits,
                            const int32_t* mask_values, int32_t n_mask, const void* src, int64_t begin, int64_t end)
{
    return guarded([&] {
        check_state(s);
        check_access(s, ordering, n_bits, mask_bits, mask_values, n_mask, src, begin, end);
        if (begin < end)
            run_accessor(s->h, s->dt, s->d, s->n, ordering, n_bits, mask_bits, mask_values, n_mask,
                         const_cast<void*>(src), begin, end, true);
    });
}

sv_status_t sv_expect_matrix(sv_state_t s, const double* matrix, const int32_t* targets, int32_t k, double* out)
{
    return guarded([&] {
        check_state(s);
        SV_CHECK(k >= 1 && k <= 5, "a dense observable takes 1 to 5 qubits");
        const GateDesc d = make_desc(s->n, targets, k, nullptr, nullptr, 0);
        (void)d;
        check_matrix_finite(matrix, k);
        SV_CHECK(out != nullptr, "out is NULL");
        double r[3];
        run_expect_matrix(s->h, s->dt, s->d, s->n, matrix, targets, k, r);
        SV_CHECK(r[2] > 0.0 && std::isfinite(r[2]), "state norm is zero or not finite");
        out[0] = r[0] / r[2];
        out[1] = r[1] / r[2];
    });
}

}  // extern "C"

namespace {

// A device range [p, p + bytes) passed by the caller: it must lie inside one
// allocation of device memory on the handle's device.
void check_device_range(const sv_handle_s* h, const void* p, uint64_t bytes, const char* what)
{
    hipPointerAttribute_t at{};
    const hipError_t e = hipPointerGetAttributes(&at, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error{SV_ERR_INVALID_VALUE, std::string(what) + " is not device memory"};
    }
    if (at.type != hipMemoryTypeDevice || at.device != h->device)
        throw Error{SV_ERR_INVALID_VALUE, std::string(what) + " is not device memory of the handle's device"};
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, hipDeviceptr_t(p)) != hipSuccess) {
        (void)hipGetLastError();
        throw Error{SV_ERR_INVALID_VALUE, std::string(what) + " is not device memory"};
    }
    const uintptr_t b = uintptr_t(base), q = uintptr_t(p);
    if (q < b || bytes > size || q - b > size - bytes)
        throw Error{SV_ERR_INVALID_VALUE, std::string(what) + " extends past its device allocation"};
}

// Arguments of a sampling call; returns false when there is nothing to do.
bool check_sample_args(const sv_state_s* s, const double* uniforms, int64_t n_shots, const int32_t* bit_ordering,
                       int32_t* n_bits, uint64_t* out, bool host_io = true)
{
    check_state(s);
    SV_CHECK(n_shots >= 0, "n_shots is negative");
    if (n_shots == 0) return false;
    SV_CHECK(uniforms != nullptr && out != nullptr, "NULL argument");
    if (host_io) {
        for (int64_t i = 0; i < n_shots; ++i)
            SV_CHECK(uniforms[i] >= 0.0 && uniforms[i] < 1.0, "uniforms must lie in [0, 1)");
    } else {
        SV_CHECK(n_shots <= (int64_t(1) << 40), "n_shots too large");
        check_device_range(s->h, uniforms, sizeof(double) * uint64_t(n_shots), "uniforms");
        check_device_range(s->h, out, sizeof(uint64_t) * uint64_t(n_shots), "out");
    }
    if (bit_ordering) {
        SV_CHECK(*n_bits >= 1 && *n_bits <= s->n, "n_bits must be in [1, n]");
        uint64_t seen = 0;
        for (int b = 0; b < *n_bits; ++b) {
            const int q = bit_ordering[b];
            SV_CHECK(q >= 0 && q < s->n, "bit_ordering entry out of range");
            SV_CHECK(!((seen >> q) & 1), "bit_ordering repeats a qubit");
            seen |= uint64_t(1) << q;
        }
    } else {
        *n_bits = 0;
    }
    return true;
}

}  // namespace

extern "C" {

sv_status_t sv_sample(sv_state_t s, const double* uniforms, int64_t n_shots, const int32_t* bit_ordering,
                      int32_t n_bits, uint64_t* out)
{
    return guarded([&] {
        if (!check_sample_args(s, uniforms, n_shots, bit_ordering, &n_bits, out)) return;
        run_sample(s->h, s->dt, s->d, s->n, uniforms, n_shots, bit_ordering, n_bits, out, true);
    });
}

sv_status_t sv_sample_device(sv_state_t s, const double* uniforms, int64_t n_shots, const int32_t* bit_ordering,
                             int32_t n_bits, uint64_t* out)
{
    return guarded([&] {
        if (!check_sample_args(s, uniforms, n_shots, bit_ordering, &n_bits, out, false)) return;
        run_sample(s->h, s->dt, s->d, s->n, uniforms, n_shots, bit_ordering, n_bits, out, false);
    });
}

sv_status_t sv_sample_noalloc(sv_state_t s, const double* uniforms, int64_t n_shots, const int32_t* bit_ordering,
                              int32_t n_bits, uint64_t* out)
{
    return guarded([&] {
        if (!check_sample_args(s, uniforms, n_shots, bit_ordering, &n_bits, out)) return;
        run_sample_noalloc(s->h, s->dt, s->d, s->n, uniforms, n_shots, bit_ordering, n_bits, out);
    });
}

sv_status_t sv_copy_to_host(sv_state_t s, void* dst, uint64_t first, uint64_t count)
{
    return guarded([&] {
        check_state(s);
        const uint64_t dim = uint64_t(1) << s->n;
        SV_CHECK(first <= dim && count <= dim - first, "range out of bounds");
        if (count == 0) return;
        SV_CHECK(dst != nullptr, "dst is NULL");
        const size_t ab = amp_bytes(s->dt);
        SV_HIP(hipMemcpyAsync(dst, static_cast<char*>(s->d) + first * ab, count * ab, hipMemcpyDeviceToHost,
                              s->h->stream));
        SV_HIP(hipStreamSynchronize(s->h->stream));
    });
}

sv_status_t sv_copy_from_host(sv_state_t s, const void* src, uint64_t first, uint64_t count)
{
    return guarded([&] {
        check_state(s);
        const uint64_t dim = uint64_t(1) << s->n;
        SV_CHECK(first <= dim && count <= dim - first, "range out of bounds");
        if (count == 0) return;
        SV_CHECK(src != nullptr, "src is NULL");
        const size_t ab = amp_bytes(s->dt);
        SV_HIP(hipMemcpyAsync(static_cast<char*>(s->d) + first * ab, src, count * ab, hipMemcpyHostToDevice,
                              s->h->stream));
        SV_HIP(hipStreamSynchronize(s->h->stream));
    });
}

sv_status_t sv_batch_create(sv_handle_t h, int32_t n_circuits, const int32_t* n_qubits, const int32_t* gate_offsets,
                            const int32_t* codes, const int32_t* qubits, const double* params,
                            const int32_t* term_offsets, const uint64_t* z_masks, int32_t max_fused_qubits,
                            sv_batch_t* out)
{
    return guarded([&] {
        SV_CHECK(out != nullptr, "out is NULL");
        *out = nullptr;
        *out = batch_create(h, n_circuits, n_qubits, gate_offsets, codes, qubits, params, term_offsets, z_masks,
                            max_fused_qubits);
    });
}

sv_status_t sv_batch_state_layout(sv_batch_t b, uint64_t* state_bytes, uint64_t* byte_offsets)
{
    return guarded([&] {
        SV_CHECK(b != nullptr && state_bytes != nullptr, "NULL argument");
        batch_layout(b, state_bytes, byte_offsets);
    });
}

sv_status_t sv_batch_info(sv_batch_t b, int32_t n_qubits, int32_t* max_fused_qubits, int32_t* blocks_per_circuit)
{
    return guarded([&] {
        SV_CHECK(b != nullptr && max_fused_qubits != nullptr, "NULL argument");
        batch_info(b, n_qubits, max_fused_qubits, blocks_per_circuit);
    });
}

sv_status_t sv_batch_plan(sv_batch_t b, int32_t n_qubits, sv_batch_size_plan_t* out)
{
    return guarded([&] {
        SV_CHECK(b != nullptr && out != nullptr, "NULL argument");
        batch_plan(b, n_qubits, out);
    });
}

sv_status_t sv_batch_host_times(sv_batch_t b, double* tune_s, double* build_s)
{
    return guarded([&] {
        SV_CHECK(b != nullptr, "batch is NULL");
        batch_host_times(b, tune_s, build_s);
    });
}

sv_status_t sv_batch_run(sv_batch_t b, void* states, double* expect_out, double* latency_s, double* kernel_s)
{
    return guarded([&] { batch_run(b, states, expect_out, latency_s, kernel_s); });
}

sv_status_t sv_batch_destroy(sv_batch_t b)
{
    return guarded([&] { batch_destroy(b); });
}

}  // extern "C"
