// Host side: the standard gate table and gate fusion.
//
// Gate fusion follows the idea the paper takes from qHiPSTER (Sec. II-B):
// many small gates are multiplied into one multi-qubit matrix so that the
// state is swept once per fused block instead of once per gate; the block
// size is capped by a "max fused gate size" option (Sec. II-D).  The paper
// does not give the fusion algorithm; this one is our own (see fuse_blocks).
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "sv_internal.h"

namespace sv {

using cd = std::complex<double>;

// ------------------------------------------------------------- gate table

namespace {

struct NamedGate {
    const char* name;
    int n_params;
    int n_targets;
    int n_controls;
};

const NamedGate kGates[] = {
    {"u3", 3, 1, 0}, {"h", 0, 1, 0},  {"x", 0, 1, 0},  {"y", 0, 1, 0},    {"z", 0, 1, 0},
    {"cx", 0, 1, 1}, {"cz", 0, 1, 1}, {"cp", 1, 1, 1}, {"swap", 0, 2, 0},
};

// Target matrix of gate kGates[gi], row-major, in std::complex.
void named_matrix(int gi, const double* p, cd* m)
{
    const cd I(0.0, 1.0);
    switch (gi) {
    case 0: {  // u3
        // OpenQASM U3: [[cos, -e^{i lambda} sin], [e^{i phi} sin, e^{i(phi+lambda)} cos]]
        const double c = std::cos(0.5 * p[0]), s = std::sin(0.5 * p[0]);
        m[0] = c;
        m[1] = -std::polar(1.0, p[2]) * s;
        m[2] = std::polar(1.0, p[1]) * s;
        m[3] = std::polar(1.0, p[1] + p[2]) * c;
        break;
    }
    case 1: {  // h
        const double r = 1.0 / std::sqrt(2.0);
        m[0] = r; m[1] = r; m[2] = r; m[3] = -r;
        break;
    }
    case 2:  // x
    case 5:  // cx
        m[0] = 0; m[1] = 1; m[2] = 1; m[3] = 0;
        break;
    case 3:  // y
        m[0] = 0; m[1] = -I; m[2] = I; m[3] = 0;
        break;
    case 4:  // z
    case 6:  // cz
        m[0] = 1; m[1] = 0; m[2] = 0; m[3] = -1;
        break;
    case 7:  // cp
        m[0] = 1; m[1] = 0; m[2] = 0; m[3] = std::polar(1.0, p[0]);
        break;
    case 8:  // swap; basis |b1 b0>: swaps |01> and |10>
        for (int i = 0; i < 16; ++i) m[i] = 0;
        m[0] = 1; m[1 * 4 + 2] = 1; m[2 * 4 + 1] = 1; m[3 * 4 + 3] = 1;
        break;
    }
}

// The matrix of gate kGates[gi] (its adjoint if adj), complex128
// interleaved, row-major.
void code_matrix(int gi, bool adj, const double* params, double* out)
{
    cd m[16];
    named_matrix(gi, params, m);
    const int d = 1 << kGates[gi].n_targets;
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
            const cd v = adj ? std::conj(m[c * d + r]) : m[r * d + c];
            out[2 * (r * d + c)] = v.real();
            out[2 * (r * d + c) + 1] = v.imag();
        }
}

}  // namespace

void gate_matrix(const char* name_c, const double* params, int n_params, double* out, int* n_targets,
                 int* n_controls)
{
    SV_CHECK(name_c != nullptr, "gate name is NULL");
    std::string name(name_c);
    bool adj = false;
    if (name.size() > 3 && name.compare(name.size() - 3, 3, "_dg") == 0) {
        adj = true;
        name.resize(name.size() - 3);
    }
    int gi = -1;
    for (int e = 0; e < int(sizeof(kGates) / sizeof(kGates[0])); ++e)
        if (name == kGates[e].name) gi = e;
    SV_CHECK(gi >= 0, "unknown gate name '" + std::string(name_c) + "'");
    const NamedGate* g = &kGates[gi];
    SV_CHECK(n_params == g->n_params, "gate '" + name + "' takes " + std::to_string(g->n_params) + " parameters");
    SV_CHECK(g->n_params == 0 || params != nullptr, "gate parameters are NULL");
    for (int i = 0; i < n_params; ++i) SV_CHECK(std::isfinite(params[i]), "gate parameter is not finite");
    SV_CHECK(out != nullptr, "matrix output is NULL");
    code_matrix(gi, adj, params, out);
    if (n_targets) *n_targets = g->n_targets;
    if (n_controls) *n_controls = g->n_controls;
}

// ------------------------------------------------------------------ fusion

namespace {

// At most SV_MAX_TARGETS qubit indices (or control values), kept inline.
struct QubitList {
    int v[SV_MAX_TARGETS];
    int n = 0;
    void push_back(int x) { v[n++] = x; }
    size_t size() const { return size_t(n); }
    int operator[](size_t i) const { return v[i]; }
    const int* begin() const { return v; }
    const int* end() const { return v + n; }
};

struct HostGate {
    QubitList targets, controls, cvals;
    uint64_t qmask = 0;  // targets | controls
    bool diagonal = false;  // every off-diagonal entry of the matrix is exactly 0
    // the 2^k x 2^k target matrix, row-major: inline up to two targets
    cd m_small[16];
    std::vector<cd> m_big;
    cd* set_size(int d)
    {
        if (d * d <= 16) return m_small;
        m_big.resize(size_t(d) * d);
        return m_big.data();
    }
    const cd* mat() const { return m_big.empty() ? m_small : m_big.data(); }
};

// A selected block: its gates (circuit order) and whether it is a diagonal
// block (all its gates diagonal, applied as one diagonal sweep).
struct Selected {
    std::vector<int> gates;
    bool diagonal = false;
};

// A block matrix under construction: 2^m x 2^m, row-major, its real and
// imaginary parts in separate arrays, starting as the identity.
struct BlockMatrix {
    int m;
    uint64_t dim;
    std::vector<double> re, im;
    explicit BlockMatrix(int m_) : m(m_), dim(uint64_t(1) << m_), re(dim * dim, 0.0), im(dim * dim, 0.0)
    {
        for (uint64_t i = 0; i < dim; ++i) re[i * dim + i] = 1.0;
    }
    // interleaved (re, im), row-major
    void store(double* out) const
    {
        for (size_t e = 0; e < size_t(dim * dim); ++e) {
            out[2 * e] = re[e];
            out[2 * e + 1] = im[e];
        }
    }
};

// U <- G * U where G acts on positions pos_t (matrix bit order) with
// controls at positions pos_c having values cv.  Each column of U is
// updated like a state of m qubits; the 2^k rows of a group are combined
// element by element along their (contiguous) columns, real and imaginary
// parts apart, so the inner loop is plain multiply-adds on contiguous
// doubles.  No std::complex products: those would go through the C99
// special-value path.
__attribute__((always_inline)) inline void left_multiply_body(BlockMatrix& U, const HostGate& g,
                                                              const QubitList& pos_t, const QubitList& pos_c)
{
    const int k = int(pos_t.size());
    const int d = 1 << k;
    const uint64_t dim = U.dim;
    uint64_t tmask = 0, cmask = 0, cset = 0;
    for (int p : pos_t) tmask |= uint64_t(1) << p;
    for (size_t a = 0; a < pos_c.size(); ++a) {
        cmask |= uint64_t(1) << pos_c[a];
        if (g.cvals[a]) cset |= uint64_t(1) << pos_c[a];
    }
    uint64_t off[1 << SV_MAX_TARGETS];
    for (int r = 0; r < d; ++r) {
        uint64_t o = 0;
        for (int a = 0; a < k; ++a)
            if ((r >> a) & 1) o |= uint64_t(1) << pos_t[a];
        off[r] = o;
    }
    if (k <= 2) {
        // one and two targets (nearly every named gate): the group's rows
        // are combined in registers, column by column, with no staging
        double mr[16], mi[16];
        for (int e = 0; e < d * d; ++e) {
            mr[e] = g.mat()[e].real();
            mi[e] = g.mat()[e].imag();
        }
        for (uint64_t row = 0; row < dim; ++row) {
            if ((row & tmask) || (row & cmask) != cset) continue;
            double* __restrict pr[4];
            double* __restrict pi[4];
            for (int r = 0; r < d; ++r) {
                pr[r] = &U.re[(row + off[r]) * dim];
                pi[r] = &U.im[(row + off[r]) * dim];
            }
            if (k == 1) {
                for (uint64_t col = 0; col < dim; ++col) {
                    const double x0r = pr[0][col], x0i = pi[0][col], x1r = pr[1][col], x1i = pi[1][col];
                    pr[0][col] = mr[0] * x0r - mi[0] * x0i + (mr[1] * x1r - mi[1] * x1i);
                    pi[0][col] = mr[0] * x0i + mi[0] * x0r + (mr[1] * x1i + mi[1] * x1r);
                    pr[1][col] = mr[2] * x0r - mi[2] * x0i + (mr[3] * x1r - mi[3] * x1i);
                    pi[1][col] = mr[2] * x0i + mi[2] * x0r + (mr[3] * x1i + mi[3] * x1r);
                }
            } else {
                for (uint64_t col = 0; col < dim; ++col) {
                    double xr[4], xi[4];
                    for (int c = 0; c < 4; ++c) {
                        xr[c] = pr[c][col];
                        xi[c] = pi[c][col];
                    }
                    for (int r = 0; r < 4; ++r) {
                        double yr = 0.0, yi = 0.0;
                        for (int c = 0; c < 4; ++c) {
                            yr += mr[4 * r + c] * xr[c] - mi[4 * r + c] * xi[c];
                            yi += mr[4 * r + c] * xi[c] + mi[4 * r + c] * xr[c];
                        }
                        pr[r][col] = yr;
                        pi[r][col] = yi;
                    }
                }
            }
        }
        return;
    }
    thread_local std::vector<double> in_re, in_im;
    in_re.resize(size_t(d) * dim);
    in_im.resize(size_t(d) * dim);
    for (uint64_t row = 0; row < dim; ++row) {
        if ((row & tmask) || (row & cmask) != cset) continue;
        for (int c = 0; c < d; ++c) {
            std::memcpy(&in_re[c * dim], &U.re[(row + off[c]) * dim], sizeof(double) * dim);
            std::memcpy(&in_im[c * dim], &U.im[(row + off[c]) * dim], sizeof(double) * dim);
        }
        for (int r = 0; r < d; ++r) {
            double* __restrict ore = &U.re[(row + off[r]) * dim];
            double* __restrict oim = &U.im[(row + off[r]) * dim];
            for (uint64_t col = 0; col < dim; ++col) ore[col] = oim[col] = 0.0;
            for (int c = 0; c < d; ++c) {
                const cd e = g.mat()[size_t(r) * d + c];
                const double mr = e.real(), mi = e.imag();
                if (mr == 0.0 && mi == 0.0) continue;
                const double* __restrict xr = &in_re[c * dim];
                const double* __restrict xi = &in_im[c * dim];
                for (uint64_t col = 0; col < dim; ++col) {
                    ore[col] += mr * xr[col] - mi * xi[col];
                    oim[col] += mr * xi[col] + mi * xr[col];
                }
            }
        }
    }
}

// The same, built for AVX2 (four doubles per vector instruction; the same
// operations in the same order, so the same results), taken where the CPU
// has it.
__attribute__((target("avx2"))) void left_multiply_avx2(BlockMatrix& U, const HostGate& g, const QubitList& pos_t,
                                                        const QubitList& pos_c)
{
    left_multiply_body(U, g, pos_t, pos_c);
}

void left_multiply_base(BlockMatrix& U, const HostGate& g, const QubitList& pos_t, const QubitList& pos_c)
{
    left_multiply_body(U, g, pos_t, pos_c);
}

void left_multiply(BlockMatrix& U, const HostGate& g, const QubitList& pos_t, const QubitList& pos_c)
{
    static const bool avx2 = __builtin_cpu_supports("avx2");
    if (avx2)
        left_multiply_avx2(U, g, pos_t, pos_c);
    else
        left_multiply_base(U, g, pos_t, pos_c);
}

int popcount64(uint64_t v) { return __builtin_popcountll(v); }

// Block selection's absorb count (see select_blocks) for several qubit sets
// at once, over the gate masks m[0, n): one scan with one independent chain
// per set (the chains overlap in the CPU where one set's scan would wait on
// each step).  A set whose qubits are all blocked takes no further gate (a
// gate inside it touches a blocked qubit), so scanning on past that point
// changes none of its counts.  At most 64 sets.
__attribute__((always_inline)) inline void count_absorbed_many_body(const uint64_t* m, size_t n,
                                                                    const uint64_t* sets, int n_sets, int* counts)
{
    uint64_t blocked[64];
    for (int c = 0; c < n_sets; ++c) {
        blocked[c] = 0;
        counts[c] = 0;
    }
    for (size_t j0 = 0; j0 < n; j0 += 8) {
        const size_t j1 = std::min(n, j0 + 8);
        for (size_t j = j0; j < j1; ++j) {
            const uint64_t Q = m[j];
            for (int c = 0; c < n_sets; ++c) {
                const bool ok = (Q & (blocked[c] | ~sets[c])) == 0;
                counts[c] += ok;
                blocked[c] |= ok ? uint64_t(0) : Q;
            }
        }
        bool open = false;
        for (int c = 0; c < n_sets; ++c) open |= (sets[c] & ~blocked[c]) != 0;
        if (!open) break;
    }
}

__attribute__((target("avx2"))) void count_absorbed_many_avx2(const uint64_t* m, size_t n, const uint64_t* sets,
                                                              int n_sets, int* counts)
{
    count_absorbed_many_body(m, n, sets, n_sets, counts);
}

void count_absorbed_many_base(const uint64_t* m, size_t n, const uint64_t* sets, int n_sets, int* counts)
{
    count_absorbed_many_body(m, n, sets, n_sets, counts);
}

void count_absorbed_many(const uint64_t* m, size_t n, const uint64_t* sets, int n_sets, int* counts)
{
    static const bool avx2 = __builtin_cpu_supports("avx2");
    if (avx2)
        count_absorbed_many_avx2(m, n, sets, n_sets, counts);
    else
        count_absorbed_many_base(m, n, sets, n_sets, counts);
}

// Block selection over the gate dependency order.
//
// Absorbing into a qubit set S: scan the remaining gates in circuit order
// and take a gate when its qubits lie in S and none of them is blocked;
// otherwise block its qubits (every later gate on them must wait).  Taken
// gates never depend on a skipped gate, so the block they form can be
// emitted before all remaining gates.
//
// While gates remain, for every "ready" gate (no remaining predecessor on
// any of its qubits) grow a qubit set from the seed's qubits one qubit at a
// time, up to kmax: the candidates are the qubits of the near-future gates
// that touch the set, and the one whose addition lets the most gates be
// absorbed wins (lowest qubit on ties).  The seed whose grown set absorbs
// the most gates becomes the next block.
//
// With kdiag > 0, diagonal blocks compete as well: absorbing into a
// diagonal set takes diagonal gates only, and since diagonal gates commute
// with one another, a skipped diagonal gate does not block later ones; only
// skipped non-diagonal gates block their qubits.  A diagonal set grows up to
// kdiag qubits from the qubits of near-future diagonal gates.  Every round
// takes the dense or diagonal block that absorbs the most gates (dense on
// ties).
std::vector<Selected> select_blocks(const std::vector<HostGate>& gates, int kmax, int kdiag)
{
    std::vector<int> live(gates.size());
    std::vector<uint64_t> mask(gates.size());
    std::vector<char> diag(gates.size());
    for (size_t i = 0; i < gates.size(); ++i) {
        live[i] = int(i);
        mask[i] = gates[i].qmask;
        diag[i] = gates[i].diagonal;
    }
    std::vector<Selected> blocks;
    std::vector<int> ready;
    std::vector<char> take;
    constexpr size_t kWindow = 256;  // gates looked at for candidate qubits
    auto absorb = [&](uint64_t S, bool mark) {
        uint64_t blocked = 0;
        int count = 0;
        const uint64_t* m = mask.data();
        for (size_t j = 0, n = live.size(); j < n; ++j) {
            // taken: inside S and on no blocked qubit (no branch on it)
            const uint64_t Q = m[j];
            const bool ok = (Q & (blocked | ~S)) == 0;
            count += ok;
            if (mark) take[j] = ok;
            blocked |= ok ? uint64_t(0) : Q;
            if ((S & ~blocked) == 0) break;  // every qubit of S is blocked
        }
        return count;
    };
    auto absorb_many = [&](const uint64_t* sets, int n_sets, int* counts) {
        count_absorbed_many(mask.data(), live.size(), sets, n_sets, counts);
    };
    auto absorb_diag = [&](uint64_t S, bool mark) {
        uint64_t blocked = 0;
        int count = 0;
        for (size_t j = 0; j < live.size(); ++j) {
            const uint64_t Q = mask[j];
            if (diag[j] && (Q & blocked) == 0 && (Q & ~S) == 0) {
                ++count;
                if (mark) take[j] = 1;
            } else if (!diag[j]) {
                blocked |= Q;
            }
            if ((S & ~blocked) == 0) break;
        }
        return count;
    };
    auto grow_diag = [&](uint64_t S) {
        while (popcount64(S) < kdiag) {
            uint64_t cand = 0, blocked = 0;
            const size_t lim = std::min(live.size(), kWindow);
            for (size_t j = 0; j < lim; ++j) {
                if (diag[j] && (mask[j] & S) && !(mask[j] & blocked)) cand |= mask[j] & ~S;
                if (!diag[j]) blocked |= mask[j];
            }
            if (!cand) break;
            int best_q = -1, best_c = -1;
            for (int q = 0; q < 64; ++q) {
                if (!((cand >> q) & 1)) continue;
                const int c = absorb_diag(S | (uint64_t(1) << q), false);
                if (c > best_c) {
                    best_c = c;
                    best_q = q;
                }
            }
            S |= uint64_t(1) << best_q;
        }
        return S;
    };
    // per round, for every qubit q: the qubits of the window's gates that
    // touch q (a set's candidates are then those of its qubits)
    uint64_t nbr[64];
    auto grow = [&](uint64_t S) {
        while (popcount64(S) < kmax) {
            uint64_t cand = 0;
            for (uint64_t r = S; r; r &= r - 1) cand |= nbr[__builtin_ctzll(r)];
            cand &= ~S;
            if (!cand) break;
            // every candidate qubit's set, lowest qubit first; the first
            // that absorbs the most wins
            uint64_t sets[64];
            int counts[64], n_sets = 0;
            for (uint64_t r = cand; r; r &= r - 1) sets[n_sets++] = S | (uint64_t(1) << __builtin_ctzll(r));
            absorb_many(sets, n_sets, counts);
            int best = 0;
            for (int c = 1; c < n_sets; ++c)
                if (counts[c] > counts[best]) best = c;
            S = sets[best];
        }
        return S;
    };
    while (!live.empty()) {
        std::fill(std::begin(nbr), std::end(nbr), uint64_t(0));
        for (size_t j = 0, lim = std::min(live.size(), kWindow); j < lim; ++j)
            for (uint64_t r = mask[j]; r; r &= r - 1) nbr[__builtin_ctzll(r)] |= mask[j];
        ready.clear();
        uint64_t seen = 0;
        for (size_t j = 0; j < live.size(); ++j) {
            if ((mask[j] & seen) == 0) ready.push_back(int(j));
            seen |= mask[j];
        }
        uint64_t best_S = 0;
        int best_count = -1;
        bool best_diag = false;
        for (int pos : ready) {
            const uint64_t S = grow(mask[size_t(pos)]);
            const int c = absorb(S, false);
            if (c > best_count) {
                best_count = c;
                best_S = S;
            }
        }
        if (kdiag > 0) {
            // seeds: the diagonal gates not blocked by an earlier non-diagonal one
            uint64_t blocked = 0;
            const size_t lim = std::min(live.size(), kWindow);
            for (size_t j = 0; j < lim; ++j) {
                if (diag[j] && !(mask[j] & blocked) && popcount64(mask[j]) <= kdiag) {
                    const uint64_t S = grow_diag(mask[j]);
                    const int c = absorb_diag(S, false);
                    if (c > best_count) {
                        best_count = c;
                        best_S = S;
                        best_diag = true;
                    }
                }
                if (!diag[j]) blocked |= mask[j];
            }
        }
        SV_CHECK(best_count > 0, "internal: fusion found no block");
        take.assign(live.size(), 0);
        if (best_diag)
            absorb_diag(best_S, true);
        else
            absorb(best_S, true);
        std::vector<int> blk;
        size_t w = 0;
        for (size_t j = 0; j < live.size(); ++j) {
            if (take[j]) {
                blk.push_back(live[j]);
            } else {
                live[w] = live[j];
                mask[w] = mask[j];
                ++w;
            }
        }
        live.resize(w);
        mask.resize(w);
        size_t w2 = 0;
        for (size_t j = 0; j < take.size(); ++j)
            if (!take[j]) diag[w2++] = diag[j];
        diag.resize(w2);
        Selected sel;
        sel.gates = std::move(blk);
        sel.diagonal = best_diag;
        blocks.push_back(std::move(sel));
    }
    return blocks;
}

// ------------------------------------------------------- coupled fusion
//
// Diagonal gates whose entries all have modulus one and that act on at most
// two qubits (CZ, CP, Z, phase gates) are phases: such a gate multiplies the
// amplitude at index i by exp(i theta(i)) with theta = c + s_a b_a + s_b b_b
// + p b_a b_b (b_q the bit of qubit q in i).  Coupled fusion does not force
// them into blocks: a dense block on qubit set S takes the gates inside S as
// usual, and a phase gate that touches S but also a qubit outside it is
// deferred: it commutes with every later gate on its qubits up to the next
// non-diagonal one, so it can be applied at the start of the next block
// that contains one of its qubits.  There the deferred terms are flushed:
// constant, singles and pairs inside the block's qubits are folded into the
// block's matrix, and a pair (a, b) with a in the block and b outside
// becomes a phase coupling: the block's input amplitude is multiplied by
// exp(i phi_ab) when both bits are set, which depends on the amplitude's
// index outside the block and so is applied in the sweep itself.  A
// deferred gate blocks later non-diagonal gates on its qubits from joining
// the block being built (they have to wait for the flush).

struct PhasePoly {
    double constant = 0.0;
    double single[64] = {};
    uint64_t single_mask = 0;
    std::map<std::pair<int, int>, double> pair;  // (a, b), a < b
};

// The phase terms of gate g if it is a deferrable phase gate.
bool phase_terms(const HostGate& g, PhasePoly& out)
{
    if (!g.diagonal || popcount64(g.qmask) > 2) return false;
    int qs[2] = {-1, -1}, nq = 0;
    for (int q = 0; q < 64; ++q)
        if ((g.qmask >> q) & 1) qs[nq++] = q;
    const int d = 1 << g.targets.size();
    double th[4] = {};
    for (int x = 0; x < (1 << nq); ++x) {
        // the gate's diagonal entry for bits x of its (ascending) qubits
        auto bit = [&](int q) {
            for (int a = 0; a < nq; ++a)
                if (qs[a] == q) return (x >> a) & 1;
            return 0;
        };
        bool on = true;
        for (size_t a = 0; a < g.controls.size(); ++a) on &= bit(g.controls[a]) == g.cvals[a];
        cd e(1.0, 0.0);
        if (on) {
            int r = 0;
            for (size_t a = 0; a < g.targets.size(); ++a) r |= bit(g.targets[a]) << a;
            e = g.mat()[size_t(r) * d + r];
        }
        if (std::fabs(std::abs(e) - 1.0) > 1e-12) return false;
        th[x] = std::arg(e);
    }
    // zero terms are left out (a CP has no single-qubit part)
    auto single = [&](int q, double v) {
        if (v == 0.0) return;
        out.single[q] += v;
        out.single_mask |= uint64_t(1) << q;
    };
    out.constant += th[0];
    if (nq == 1) {
        single(qs[0], th[1] - th[0]);
    } else {
        single(qs[0], th[1] - th[0]);
        single(qs[1], th[2] - th[0]);
        const double p = th[3] - th[2] - th[1] + th[0];
        if (p != 0.0) out.pair[{qs[0], qs[1]}] += p;
    }
    return true;
}

void add_terms(PhasePoly& to, const PhasePoly& from)
{
    to.constant += from.constant;
    for (int q = 0; q < 64; ++q)
        if ((from.single_mask >> q) & 1) to.single[q] += from.single[q];
    to.single_mask |= from.single_mask;
    for (const auto& kv : from.pair) to.pair[kv.first] += kv.second;
}

// Moves the terms of `from` that touch S (and its constant) into `to`.
void flush_terms(PhasePoly& from, uint64_t S, PhasePoly& to)
{
    to.constant += from.constant;
    from.constant = 0.0;
    for (int q = 0; q < 64; ++q) {
        if (((from.single_mask & S) >> q) & 1) {
            to.single[q] += from.single[q];
            to.single_mask |= uint64_t(1) << q;
            from.single[q] = 0.0;
        }
    }
    from.single_mask &= ~S;
    for (auto it = from.pair.begin(); it != from.pair.end();) {
        const uint64_t m = (uint64_t(1) << it->first.first) | (uint64_t(1) << it->first.second);
        if (m & S) {
            to.pair[it->first] += it->second;
            it = from.pair.erase(it);
        } else {
            ++it;
        }
    }
}

struct CoupledSel {
    std::vector<int> gates;  // taken, in circuit order
    uint64_t S = 0;
    PhasePoly flushed;       // applied before the gates
};

std::vector<CoupledSel> select_blocks_coupled(const std::vector<HostGate>& gates, int kmax)
{
    const size_t G = gates.size();
    std::vector<int> live(G);
    std::vector<uint64_t> mask(G);
    std::vector<char> diag(G), deferrable(G);
    std::vector<PhasePoly> terms(G);
    for (size_t i = 0; i < G; ++i) {
        live[i] = int(i);
        mask[i] = gates[i].qmask;
        diag[i] = gates[i].diagonal;
        deferrable[i] = phase_terms(gates[i], terms[i]);
    }
    std::vector<CoupledSel> blocks;
    PhasePoly pending;
    std::vector<char> take;  // 1 taken, 2 deferred
    constexpr size_t kWindow = 256;
    // Gates S takes (inside S) and defers (phases touching S) in one scan.
    auto absorb = [&](uint64_t S, bool mark) {
        uint64_t blocked_all = 0, blocked_nd = 0;
        int count = 0;
        for (size_t j = 0; j < live.size(); ++j) {
            const uint64_t Q = mask[j];
            const int li = live[j];
            if (Q & blocked_all) {
                if (diag[li])
                    blocked_nd |= Q;
                else
                    blocked_all |= Q;
            } else if (!diag[li]) {
                if ((Q & ~S) == 0 && (Q & blocked_nd) == 0) {
                    ++count;
                    if (mark) take[j] = 1;
                } else {
                    blocked_all |= Q;
                }
            } else if ((Q & ~S) == 0) {
                ++count;
                if (mark) take[j] = 1;
            } else if ((Q & S) && deferrable[li]) {
                ++count;
                if (mark) take[j] = 2;
                blocked_nd |= Q;
            } else {
                blocked_nd |= Q;
            }
            if ((S & ~blocked_all) == 0) break;
        }
        return count;
    };
    std::vector<int> ready;
    // Grows S one qubit at a time from the qubits of near-future gates that
    // touch it; when none is left, by all qubits of a ready gate disjoint
    // from S that fits (independent gates side by side in one block), the
    // one that lets the most gates be absorbed.
    auto grow = [&](uint64_t S) {
        while (popcount64(S) < kmax) {
            uint64_t cand = 0;
            const size_t lim = std::min(live.size(), kWindow);
            for (size_t j = 0; j < lim; ++j)
                if (mask[j] & S) cand |= mask[j] & ~S;
            if (cand) {
                int best_q = -1, best_c = -1;
                for (int q = 0; q < 64; ++q) {
                    if (!((cand >> q) & 1)) continue;
                    const int c = absorb(S | (uint64_t(1) << q), false);
                    if (c > best_c) {
                        best_c = c;
                        best_q = q;
                    }
                }
                S |= uint64_t(1) << best_q;
                continue;
            }
            const int here = absorb(S, false);
            uint64_t best_m = 0;
            int best_c = here;
            for (int pos : ready) {
                const uint64_t m = mask[size_t(pos)];
                if ((m & S) || popcount64(S | m) > kmax) continue;
                const int c = absorb(S | m, false);
                if (c > best_c) {
                    best_c = c;
                    best_m = m;
                }
            }
            if (!best_m) break;
            S |= best_m;
        }
        return S;
    };
    while (!live.empty()) {
        ready.clear();
        uint64_t seen = 0;
        for (size_t j = 0; j < live.size(); ++j) {
            if ((mask[j] & seen) == 0) ready.push_back(int(j));
            seen |= mask[j];
        }
        uint64_t best_S = 0;
        int best_count = -1;
        for (int pos : ready) {
            const uint64_t S = grow(mask[size_t(pos)]);
            const int c = absorb(S, false);
            if (c > best_count) {
                best_count = c;
                best_S = S;
            }
        }
        SV_CHECK(best_count > 0, "internal: coupled fusion found no block");
        CoupledSel sel;
        sel.S = best_S;
        // the phases deferred so far that touch the block precede its gates
        flush_terms(pending, best_S, sel.flushed);
        take.assign(live.size(), 0);
        absorb(best_S, true);
        size_t w = 0;
        for (size_t j = 0; j < live.size(); ++j) {
            if (take[j] == 1) {
                sel.gates.push_back(live[j]);
            } else if (take[j] == 2) {
                add_terms(pending, terms[size_t(live[j])]);
            } else {
                live[w] = live[j];
                mask[w] = mask[j];
                ++w;
            }
        }
        live.resize(w);
        mask.resize(w);
        blocks.push_back(std::move(sel));
    }
    // phases still deferred at the end: blocks without gates, each on up to
    // kmax qubits chosen greedily to cover the most remaining terms
    while (pending.single_mask || !pending.pair.empty()) {
        uint64_t S = 0;
        while (popcount64(S) < kmax) {
            int score[64] = {};
            for (int q = 0; q < 64; ++q)
                if (((pending.single_mask & ~S) >> q) & 1) ++score[q];
            for (const auto& kv : pending.pair) {
                const int a = kv.first.first, b = kv.first.second;
                if (((S >> a) & 1) || ((S >> b) & 1)) continue;
                ++score[a];
                ++score[b];
            }
            int best = -1;
            for (int q = 0; q < 64; ++q)
                if (score[q] > 0 && (best < 0 || score[q] > score[best])) best = q;
            if (best < 0) break;
            S |= uint64_t(1) << best;
        }
        CoupledSel sel;
        sel.S = S;
        flush_terms(pending, S, sel.flushed);
        blocks.push_back(std::move(sel));
    }
    if (pending.constant != 0.0) {
        // a global phase left over: the last block carries it (or a block of
        // its own on qubit 0 when there is none)
        if (blocks.empty()) {
            CoupledSel sel;
            sel.S = 1;
            blocks.push_back(std::move(sel));
        }
        blocks.back().flushed.constant += pending.constant;
    }
    return blocks;
}

}  // namespace

sv_fused_s* fuse(const sv_gate_t* gates, int n_gates, int kmax, int kdiag, bool coupled);

sv_fused_s* fuse_gate_list(const int32_t* codes, const int32_t* qubits, const double* params, int n_gates,
                           int kmax, int kdiag, bool coupled)
{
    SV_CHECK(n_gates >= 0, "n_gates is negative");
    SV_CHECK(n_gates == 0 || (codes && qubits && params), "NULL gate arrays");
    std::vector<sv_gate_t> gates(n_gates);
    std::vector<double> mats(size_t(n_gates) * 32);
    std::vector<int32_t> qs(size_t(n_gates) * 2);
    for (int g = 0; g < n_gates; ++g) {
        const int code = codes[g] & ~int(SV_GATE_ADJOINT);
        const bool adj = (codes[g] & SV_GATE_ADJOINT) != 0;
        SV_CHECK(code >= SV_GATE_U3 && code <= SV_GATE_SWAP, "gate " + std::to_string(g) + ": unknown code");
        // the gate codes follow the gate table's order
        const NamedGate& ng = kGates[code];
        const double* p = params + 3 * size_t(g);
        for (int i = 0; i < ng.n_params; ++i)
            SV_CHECK(std::isfinite(p[i]), "gate " + std::to_string(g) + ": parameter is not finite");
        code_matrix(code, adj, p, &mats[size_t(g) * 32]);
        const int nt = ng.n_targets, nc = ng.n_controls;
        // qubit order: controls first, then targets
        qs[2 * g] = qubits[2 * g];
        qs[2 * g + 1] = qubits[2 * g + 1];
        sv_gate_t& e = gates[g];
        e.n_controls = nc;
        e.controls = nc ? &qs[2 * g] : nullptr;
        e.control_values = nullptr;
        e.n_targets = nt;
        e.targets = &qs[2 * g + nc];
        e.matrix = &mats[size_t(g) * 32];
        e.adjoint = 0;  // the adjoint code is already in the matrix
    }
    return fuse(gates.data(), n_gates, kmax, kdiag, coupled);
}

namespace {

// Blocks of coupled fusion: each block's matrix is the product of its gates
// times the diagonal of its flushed phases inside its qubits (applied
// first), and its coupling holds the flushed pairs with one qubit outside.
sv_fused_s* build_coupled(const std::vector<HostGate>& hg, const std::vector<CoupledSel>& sel)
{
    struct Plan {
        std::vector<int> qs;      // targets, ascending
        std::vector<int> cq;      // coupled qubits, ascending
    };
    std::vector<Plan> plan(sel.size());
    size_t total = 0;
    for (size_t b = 0; b < sel.size(); ++b) {
        const CoupledSel& c = sel[b];
        uint64_t T = 0;
        for (int i : c.gates) T |= hg[i].qmask;
        T |= c.flushed.single_mask & c.S;
        uint64_t C = 0;
        for (const auto& kv : c.flushed.pair) {
            const uint64_t ma = uint64_t(1) << kv.first.first, mb = uint64_t(1) << kv.first.second;
            T |= (ma | mb) & c.S;
            C |= (ma | mb) & ~c.S;
        }
        if (T == 0) T = c.S & (~c.S + 1);  // a block holding only a global phase
        for (int q = 0; q < 64; ++q) {
            if ((T >> q) & 1) plan[b].qs.push_back(q);
            if ((C >> q) & 1) plan[b].cq.push_back(q);
        }
        SV_CHECK(plan[b].qs.size() <= size_t(SV_MAX_TARGETS), "internal: coupled block too wide");
        SV_CHECK(plan[b].cq.size() <= size_t(SV_MAX_QUBITS), "coupled fusion: too many coupled qubits");
        const size_t d = size_t(1) << plan[b].qs.size();
        total += 2 * d * d + plan[b].qs.size() * plan[b].cq.size();
    }
    auto* f = new sv_fused_s;
    f->n_blocks = int(sel.size());
    f->blocks = new FusedBlock[sel.size()];
    f->storage = new double[std::max<size_t>(total, 1)];
    size_t at = 0;
    for (size_t b = 0; b < sel.size(); ++b) {
        const CoupledSel& c = sel[b];
        const std::vector<int>& qs = plan[b].qs;
        const std::vector<int>& cq = plan[b].cq;
        const int m = int(qs.size());
        const uint64_t dim = uint64_t(1) << m;
        auto pos = [&](int q) { return int(std::lower_bound(qs.begin(), qs.end(), q) - qs.begin()); };
        FusedBlock& blk = f->blocks[b];
        blk.k = m;
        for (int a = 0; a < m; ++a) blk.targets[a] = qs[a];
        BlockMatrix U(m);
        for (int gi : c.gates) {
            const HostGate& g = hg[gi];
            QubitList pt, pc;
            for (int q : g.targets) pt.push_back(pos(q));
            for (int q : g.controls) pc.push_back(pos(q));
            left_multiply(U, g, pt, pc);
        }
        // flushed phases inside the block: U <- U diag(exp(i theta(col)))
        for (uint64_t col = 0; col < dim; ++col) {
            double th = c.flushed.constant;
            for (int a = 0; a < m; ++a)
                if (((col >> a) & 1) && ((c.flushed.single_mask >> qs[a]) & 1)) th += c.flushed.single[qs[a]];
            for (const auto& kv : c.flushed.pair) {
                const int x = kv.first.first, y = kv.first.second;
                if (((c.S >> x) & 1) && ((c.S >> y) & 1) && ((col >> pos(x)) & 1) && ((col >> pos(y)) & 1))
                    th += kv.second;
            }
            if (th == 0.0) continue;
            const double er = std::cos(th), ei = std::sin(th);
            for (uint64_t row = 0; row < dim; ++row) {
                const double ur = U.re[row * dim + col], ui = U.im[row * dim + col];
                U.re[row * dim + col] = ur * er - ui * ei;
                U.im[row * dim + col] = ur * ei + ui * er;
            }
        }
        blk.m = f->storage + at;
        U.store(blk.m);
        at += 2 * dim * dim;
        blk.n_couple = int(cq.size());
        for (size_t j = 0; j < cq.size(); ++j) blk.couple_q[j] = cq[j];
        blk.couple = f->storage + at;
        for (size_t e = 0; e < size_t(m) * cq.size(); ++e) blk.couple[e] = 0.0;
        for (const auto& kv : c.flushed.pair) {
            const int x = kv.first.first, y = kv.first.second;
            const bool xin = (c.S >> x) & 1, yin = (c.S >> y) & 1;
            if (xin == yin) continue;
            const int a = pos(xin ? x : y), o = xin ? y : x;
            const size_t ci = size_t(std::lower_bound(cq.begin(), cq.end(), o) - cq.begin());
            blk.couple[size_t(a) * cq.size() + ci] += kv.second;
        }
        at += size_t(m) * cq.size();
    }
    return f;
}

}  // namespace

sv_fused_s* fuse(const sv_gate_t* gates, int n_gates, int kmax, int kdiag, bool coupled)
{
    SV_CHECK(n_gates >= 0, "n_gates is negative");
    SV_CHECK(n_gates == 0 || gates != nullptr, "gates is NULL");
    SV_CHECK(kmax >= 1 && kmax <= SV_MAX_TARGETS, "max_fused_qubits must be in [1, 10]");
    SV_CHECK(kdiag >= 0 && kdiag <= SV_MAX_TARGETS, "max_fused_diagonal_qubits must be in [0, 10]");
    std::vector<HostGate> hg(n_gates);
    for (int i = 0; i < n_gates; ++i) {
        const sv_gate_t& g = gates[i];
        SV_CHECK(g.n_targets >= 1 && g.n_targets <= SV_MAX_TARGETS, "gate " + std::to_string(i) + ": bad n_targets");
        SV_CHECK(g.n_controls >= 0 && g.n_targets + g.n_controls <= SV_MAX_TARGETS,
                 "gate " + std::to_string(i) + ": more than 10 qubits with controls");
        SV_CHECK(g.targets && g.matrix, "gate " + std::to_string(i) + ": NULL targets or matrix");
        SV_CHECK(g.n_controls == 0 || g.controls, "gate " + std::to_string(i) + ": NULL controls");
        HostGate& h = hg[i];
        for (int a = 0; a < g.n_targets; ++a) {
            const int q = g.targets[a];
            SV_CHECK(q >= 0 && q < 64 && !((h.qmask >> q) & 1), "gate " + std::to_string(i) + ": bad or repeated qubit");
            h.qmask |= uint64_t(1) << q;
            h.targets.push_back(q);
        }
        for (int a = 0; a < g.n_controls; ++a) {
            const int q = g.controls[a];
            SV_CHECK(q >= 0 && q < 64 && !((h.qmask >> q) & 1), "gate " + std::to_string(i) + ": bad or repeated qubit");
            h.qmask |= uint64_t(1) << q;
            h.controls.push_back(q);
            const int cv = g.control_values ? g.control_values[a] : 1;
            SV_CHECK(cv == 0 || cv == 1, "control values must be 0 or 1");
            h.cvals.push_back(cv);
        }
        const int d = 1 << g.n_targets;
        cd* hm = h.set_size(d);
        h.diagonal = true;
        for (int e = 0; e < d * d; ++e) {
            SV_CHECK(std::isfinite(g.matrix[2 * e]) && std::isfinite(g.matrix[2 * e + 1]),
                     "gate " + std::to_string(i) + ": matrix entry is not finite");
            // the adjoint's entry (r, c) is the conjugate of entry (c, r)
            const int src = g.adjoint ? (e % d) * d + e / d : e;
            const double im = g.matrix[2 * src + 1];
            hm[e] = cd(g.matrix[2 * src], g.adjoint ? -im : im);
            if (e / d != e % d && hm[e] != cd(0.0, 0.0)) h.diagonal = false;
        }
    }
    if (coupled) return build_coupled(hg, select_blocks_coupled(hg, kmax));
    const auto sel = select_blocks(hg, kmax, kdiag);
    // build matrices
    std::vector<std::vector<int>> qs(sel.size());
    size_t total = 0;
    for (size_t b = 0; b < sel.size(); ++b) {
        uint64_t S = 0;
        for (int i : sel[b].gates) S |= hg[i].qmask;
        for (int q = 0; q < 64; ++q)
            if ((S >> q) & 1) qs[b].push_back(q);
        const size_t d = size_t(1) << qs[b].size();
        total += sel[b].diagonal ? d : d * d;
    }
    auto* f = new sv_fused_s;
    f->n_blocks = int(sel.size());
    f->blocks = new FusedBlock[sel.size()];
    f->storage = new double[2 * std::max<size_t>(total, 1)];
    size_t at = 0;
    for (size_t b = 0; b < sel.size(); ++b) {
        const int m = int(qs[b].size());
        const uint64_t dim = uint64_t(1) << m;
        auto pos = [&](int q) { return int(std::lower_bound(qs[b].begin(), qs[b].end(), q) - qs[b].begin()); };
        FusedBlock& blk = f->blocks[b];
        blk.k = m;
        for (int a = 0; a < m; ++a) blk.targets[a] = qs[b][a];
        blk.m = f->storage + 2 * at;
        if (sel[b].diagonal) {
            // the product of the gates' diagonals: entry i gets, from every
            // gate whose control bits in i match, the diagonal element of the
            // row that i's bits at the gate's targets select
            blk.diagonal = true;
            std::vector<cd> D(dim, cd(1.0, 0.0));
            for (int gi : sel[b].gates) {
                const HostGate& g = hg[gi];
                const int d = 1 << g.targets.size();
                for (uint64_t i = 0; i < dim; ++i) {
                    bool on = true;
                    for (size_t a = 0; a < g.controls.size(); ++a)
                        on &= int((i >> pos(g.controls[a])) & 1) == g.cvals[a];
                    if (!on) continue;
                    int r = 0;
                    for (size_t a = 0; a < g.targets.size(); ++a) r |= int((i >> pos(g.targets[a])) & 1) << a;
                    const cd e = g.mat()[size_t(r) * d + r];
                    D[i] = cd(D[i].real() * e.real() - D[i].imag() * e.imag(),
                              D[i].real() * e.imag() + D[i].imag() * e.real());
                }
            }
            for (uint64_t i = 0; i < dim; ++i) {
                blk.m[2 * i] = D[i].real();
                blk.m[2 * i + 1] = D[i].imag();
            }
            at += dim;
            continue;
        }
        BlockMatrix U(m);
        for (int gi : sel[b].gates) {
            const HostGate& g = hg[gi];
            QubitList pt, pc;
            for (int q : g.targets) pt.push_back(pos(q));
            for (int q : g.controls) pc.push_back(pos(q));
            left_multiply(U, g, pt, pc);
        }
        U.store(blk.m);
        at += dim * dim;
    }
    return f;
}

}  // namespace sv
