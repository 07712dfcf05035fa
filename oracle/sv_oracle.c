/*
 * CPU oracle for state-vector circuit simulation.  TEST INFRASTRUCTURE ONLY:
 * nothing in the product library calls, links or loads this file; only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg do.
 *
 * Plain, slow, obviously-correct complex128 code that follows the
 * definitions of the operations, written independently of the GPU library
 * (it has its own gate table and its own index loops).  Every floating-point
 * operation is in IEEE double; build with -ffp-contract=off so that no FMA
 * contraction changes the rounding, and -fcx-limited-range so that complex
 * multiplication is the textbook (ac-bd) + i(ad+bc).
 *
 * Conventions (the paper only says that each index bit of the state vector
 * corresponds to one qubit, Sec. II-C):
 *   - qubit j is bit j of the amplitude index (qubit 0 = least significant);
 *   - a k-qubit gate matrix is 2^k x 2^k, row-major, and bit a of its row /
 *     column index is the state of targets[a] (targets[0] = matrix LSB);
 *   - control values default to 1.
 *
 * Every function here is pinned by the CPU test suite against brute-force
 * Kronecker-product unitaries, closed forms or exact enumerations.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double _Complex cplx;

#define ORC_OK 0
#define ORC_BAD 1

/* ------------------------------------------------------------------------ */
/* Gate table.  The paper defines no gates; these are the standard textbook  */
/* matrices (U3 in the OpenQASM convention, global phase included because   */
/* amplitudes are compared directly).                                        */
/* ------------------------------------------------------------------------ */

static void set2(cplx* m, cplx a, cplx b, cplx c, cplx d)
{
    m[0] = a; m[1] = b; m[2] = c; m[3] = d;
}

/*
 * Writes the target matrix of a named gate into `out` (row-major complex,
 * interleaved re/im doubles), the number of target qubits into *k_out and the
 * number of leading control qubits into *nctrl_out.  A gate named
 * "<name>_dg" yields the conjugate transpose of "<name>".  Returns 0 or 1
 * (unknown name / wrong parameter count).
 */
int orc_gate_matrix(const char* name_in, const double* p, int np, double* out,
                    int* k_out, int* nctrl_out)
{
    char name[32];
    size_t len = strlen(name_in);
    int adj = 0;
    if (len >= sizeof(name)) return ORC_BAD;
    memcpy(name, name_in, len + 1);
    if (len > 3 && strcmp(name + len - 3, "_dg") == 0) {
        adj = 1;
        name[len - 3] = '\0';
    }
    cplx m[16];
    int k = 1, nc = 0;
    const double r2 = 1.0 / sqrt(2.0);
    if (strcmp(name, "u3") == 0) {
        if (np != 3) return ORC_BAD;
        double c = cos(p[0] / 2.0), s = sin(p[0] / 2.0);
        cplx el = cexp(I * p[2]), ep = cexp(I * p[1]), epl = cexp(I * (p[1] + p[2]));
        set2(m, c, -el * s, ep * s, epl * c);
    } else if (strcmp(name, "h") == 0) {
        set2(m, r2, r2, r2, -r2);
    } else if (strcmp(name, "x") == 0) {
        set2(m, 0, 1, 1, 0);
    } else if (strcmp(name, "y") == 0) {
        set2(m, 0, -I, I, 0);
    } else if (strcmp(name, "z") == 0) {
        set2(m, 1, 0, 0, -1);
    } else if (strcmp(name, "cx") == 0) {
        set2(m, 0, 1, 1, 0);
        nc = 1;
    } else if (strcmp(name, "cz") == 0) {
        set2(m, 1, 0, 0, -1);
        nc = 1;
    } else if (strcmp(name, "cp") == 0) {
        if (np != 1) return ORC_BAD;
        set2(m, 1, 0, 0, cexp(I * p[0]));
        nc = 1;
    } else if (strcmp(name, "swap") == 0) {
        k = 2;
        for (int i = 0; i < 16; ++i) m[i] = 0;
        m[0 * 4 + 0] = 1; m[1 * 4 + 2] = 1; m[2 * 4 + 1] = 1; m[3 * 4 + 3] = 1;
    } else {
        return ORC_BAD;
    }
    if (adj && strcmp(name, "u3") != 0 && strcmp(name, "cp") != 0 && strcmp(name, "y") != 0) {
        /* h, x, z, cx, cz, swap are real symmetric: their own adjoints */
        adj = 0;
    }
    int d = 1 << k;
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
            cplx v = adj ? conj(m[c * d + r]) : m[r * d + c];
            out[2 * (r * d + c)] = creal(v);
            out[2 * (r * d + c) + 1] = cimag(v);
        }
    *k_out = k;
    *nctrl_out = nc;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Gate application (Table I: gate application with a dense matrix; the     */
/* state is updated in place, Sec. II-A).                                     */
/*                                                                          */
/* For every index i whose target bits are all 0 and whose control bits      */
/* equal the control values, the 2^k amplitudes psi[i + off(c)], where      */
/* off(c) sets bit targets[a] for each set bit a of c, are replaced by       */
/* M times them.  Every other amplitude is unchanged.  The loop visits all   */
/* indices and skips those that are not group bases.                         */
/* ------------------------------------------------------------------------ */

int orc_apply(double* psi_ri, int n, const double* m_ri, const int* targets, int k,
              const int* controls, const int* cvals, int nc)
{
    if (n < 1 || n > 40 || k < 1 || k > 10 || nc < 0 || k + nc > n) return ORC_BAD;
    cplx* psi = (cplx*)psi_ri;
    const cplx* m = (const cplx*)m_ri;
    int64_t dim = (int64_t)1 << n;
    int d = 1 << k;
    uint64_t tmask = 0, cmask = 0, cval = 0;
    for (int a = 0; a < k; ++a) {
        if (targets[a] < 0 || targets[a] >= n || (tmask >> targets[a] & 1)) return ORC_BAD;
        tmask |= (uint64_t)1 << targets[a];
    }
    for (int a = 0; a < nc; ++a) {
        uint64_t b = (uint64_t)1 << controls[a];
        if (controls[a] < 0 || controls[a] >= n || (tmask & b) || (cmask & b)) return ORC_BAD;
        cmask |= b;
        if (cvals == NULL || cvals[a]) cval |= b;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < dim; ++i) {
        if (((uint64_t)i & tmask) != 0 || ((uint64_t)i & cmask) != cval) continue;
        uint64_t idx[1024];
        cplx v[1024];
        for (int c = 0; c < d; ++c) {
            uint64_t j = (uint64_t)i;
            for (int a = 0; a < k; ++a)
                if ((c >> a) & 1) j |= (uint64_t)1 << targets[a];
            idx[c] = j;
            v[c] = psi[j];
        }
        for (int r = 0; r < d; ++r) {
            cplx acc = 0;
            for (int c = 0; c < d; ++c) acc += m[r * d + c] * v[c];
            psi[idx[r]] = acc;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Generalized permutation gate (Table I: gate application with a            */
/* generalized permutation matrix; Sec. II-D: diagonal gates and their       */
/* fusion).  G = D P on k targets: row r of G has its one non-zero entry     */
/* diag[r] in column perm[r] (perm == NULL: the identity, so G is the        */
/* diagonal matrix diag).  For every group base i (as in orc_apply) the      */
/* new amplitude at i + off(r) is diag[r] times the old one at               */
/* i + off(perm[r]).  perm must be a permutation of 0 .. 2^k - 1.           */
/* ------------------------------------------------------------------------ */

int orc_apply_gperm(double* psi_ri, int n, const int64_t* perm, const double* diag_ri, const int* targets,
                    int k, const int* controls, const int* cvals, int nc)
{
    if (n < 1 || n > 40 || k < 1 || k > 12 || nc < 0 || k + nc > n) return ORC_BAD;
    cplx* psi = (cplx*)psi_ri;
    const cplx* dg = (const cplx*)diag_ri;
    int64_t dim = (int64_t)1 << n;
    int d = 1 << k;
    uint64_t tmask = 0, cmask = 0, cval = 0;
    for (int a = 0; a < k; ++a) {
        if (targets[a] < 0 || targets[a] >= n || (tmask >> targets[a] & 1)) return ORC_BAD;
        tmask |= (uint64_t)1 << targets[a];
    }
    for (int a = 0; a < nc; ++a) {
        uint64_t b = (uint64_t)1 << controls[a];
        if (controls[a] < 0 || controls[a] >= n || (tmask & b) || (cmask & b)) return ORC_BAD;
        cmask |= b;
        if (cvals == NULL || cvals[a]) cval |= b;
    }
    if (perm != NULL) {
        char seen[4096];
        memset(seen, 0, sizeof(seen));
        for (int r = 0; r < d; ++r) {
            if (perm[r] < 0 || perm[r] >= d || seen[perm[r]]) return ORC_BAD;
            seen[perm[r]] = 1;
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < dim; ++i) {
        if (((uint64_t)i & tmask) != 0 || ((uint64_t)i & cmask) != cval) continue;
        uint64_t idx[4096];
        cplx v[4096];
        for (int c = 0; c < d; ++c) {
            uint64_t j = (uint64_t)i;
            for (int a = 0; a < k; ++a)
                if ((c >> a) & 1) j |= (uint64_t)1 << targets[a];
            idx[c] = j;
            v[c] = psi[j];
        }
        for (int r = 0; r < d; ++r) psi[idx[r]] = dg[r] * v[perm ? perm[r] : r];
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Index bit swap (Table I: swap index bit pairs of the state vector).  For  */
/* every index i whose mask bits equal the mask values, the amplitude moves  */
/* to the index with bits a_p and b_p exchanged for every pair p (all bits  */
/* of all pairs distinct, none a mask bit); other amplitudes stay.           */
/* ------------------------------------------------------------------------ */

int orc_swap_index_bits(double* psi_ri, int n, const int* pairs, int npairs, const int* mbits, const int* mvals,
                        int nmask)
{
    if (n < 1 || n > 40 || npairs < 0 || nmask < 0) return ORC_BAD;
    uint64_t used = 0, mmask = 0, mval = 0;
    for (int a = 0; a < 2 * npairs; ++a) {
        if (pairs[a] < 0 || pairs[a] >= n || (used >> pairs[a] & 1)) return ORC_BAD;
        used |= (uint64_t)1 << pairs[a];
    }
    for (int a = 0; a < nmask; ++a) {
        uint64_t b = (uint64_t)1 << mbits[a];
        if (mbits[a] < 0 || mbits[a] >= n || (used & b)) return ORC_BAD;
        used |= b;
        mmask |= b;
        if (mvals[a]) mval |= b;
    }
    int64_t dim = (int64_t)1 << n;
    cplx* psi = (cplx*)psi_ri;
    cplx* out = (cplx*)malloc(sizeof(cplx) * (size_t)dim);
    if (!out) return ORC_BAD;
    memcpy(out, psi, sizeof(cplx) * (size_t)dim);
    for (int64_t i = 0; i < dim; ++i) {
        if (((uint64_t)i & mmask) != mval) continue;
        uint64_t j = (uint64_t)i;
        for (int p = 0; p < npairs; ++p) {
            const uint64_t ba = ((uint64_t)i >> pairs[2 * p]) & 1, bb = ((uint64_t)i >> pairs[2 * p + 1]) & 1;
            j &= ~(((uint64_t)1 << pairs[2 * p]) | ((uint64_t)1 << pairs[2 * p + 1]));
            j |= (bb << pairs[2 * p]) | (ba << pairs[2 * p + 1]);
        }
        out[j] = psi[i];
    }
    memcpy(psi, out, sizeof(cplx) * (size_t)dim);
    free(out);
    return ORC_OK;
}

/* Accessor with reordering (Table I: copy the state between host and device */
/* while changing the qubit order): element k - begin of buf is the          */
/* amplitude whose bit ordering[a] is bit a of k (a < nbits) and whose mask  */
/* bits hold the mask values; nbits + nmask == n, all bits distinct.         */
/* set != 0 writes buf into the state instead of reading.                    */
int orc_accessor(double* psi_ri, int n, const int* ordering, int nbits, const int* mbits, const int* mvals,
                 int nmask, double* buf_ri, int64_t begin, int64_t end, int set)
{
    if (n < 1 || n > 40 || nbits < 0 || nmask < 0 || nbits + nmask != n) return ORC_BAD;
    uint64_t used = 0, mval = 0;
    for (int a = 0; a < nbits; ++a) {
        if (ordering[a] < 0 || ordering[a] >= n || (used >> ordering[a] & 1)) return ORC_BAD;
        used |= (uint64_t)1 << ordering[a];
    }
    for (int a = 0; a < nmask; ++a) {
        if (mbits[a] < 0 || mbits[a] >= n || (used >> mbits[a] & 1)) return ORC_BAD;
        used |= (uint64_t)1 << mbits[a];
        if (mvals[a]) mval |= (uint64_t)1 << mbits[a];
    }
    if (begin < 0 || end < begin || end > ((int64_t)1 << nbits)) return ORC_BAD;
    cplx* psi = (cplx*)psi_ri;
    cplx* buf = (cplx*)buf_ri;
    for (int64_t k = begin; k < end; ++k) {
        uint64_t i = mval;
        for (int a = 0; a < nbits; ++a) i |= (((uint64_t)k >> a) & 1) << ordering[a];
        if (set)
            psi[i] = buf[k - begin];
        else
            buf[k - begin] = psi[i];
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Reductions.  Sums are Neumaier-compensated and run in index order, so the */
/* result is the exact sum rounded to within a few ulps.                     */
/* ------------------------------------------------------------------------ */

typedef struct { double s, c; } ksum;

static void ks_add(ksum* k, double x)
{
    double t = k->s + x;
    if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x;
    else k->c += (x - t) + k->s;
    k->s = t;
}

static double ks_val(const ksum* k) { return k->s + k->c; }

/* Squared norm sum_i |psi_i|^2: the total of the probability distribution
 * that measurement without collapse is computed from (Sec. II). */
double orc_norm(const double* psi_ri, int n)
{
    int64_t dim = (int64_t)1 << n;
    ksum k = {0.0, 0.0};
    for (int64_t i = 0; i < dim; ++i) {
        double re = psi_ri[2 * i], im = psi_ri[2 * i + 1];
        ks_add(&k, re * re);
        ks_add(&k, im * im);
    }
    return ks_val(&k);
}

/* <psi|phi> with compensated sums of the real and imaginary parts. */
static void inner(const cplx* a, const cplx* b, int64_t dim, double* re, double* im)
{
    ksum kr = {0.0, 0.0}, ki = {0.0, 0.0};
    for (int64_t i = 0; i < dim; ++i) {
        double ar = creal(a[i]), ai = cimag(a[i]), br = creal(b[i]), bi = cimag(b[i]);
        /* conj(a) * b = (ar br + ai bi) + i (ar bi - ai br) */
        ks_add(&kr, ar * br);
        ks_add(&kr, ai * bi);
        ks_add(&ki, ar * bi);
        ks_add(&ki, -(ai * br));
    }
    *re = ks_val(&kr);
    *im = ks_val(&ki);
}

/*
 * Expectation value of a Pauli string (Table I: expectation with Pauli
 * strings): <psi|P|psi> / <psi|psi>.  P|psi> is formed the plain way, by
 * applying each single-qubit Pauli matrix of the string to a copy of the
 * state with orc_apply.  ops[a] is 'X', 'Y', 'Z' or 'I' acting on qubits[a].
 * out[0] = real part, out[1] = imaginary part (zero up to rounding, P being
 * Hermitian), out[2] = <psi|psi>.
 */
int orc_expect_pauli(const double* psi_ri, int n, const int* qubits, const char* ops,
                     int nops, double* out)
{
    static const double X[8] = {0, 0, 1, 0, 1, 0, 0, 0};
    static const double Y[8] = {0, 0, 0, -1, 0, 1, 0, 0};
    static const double Z[8] = {1, 0, 0, 0, 0, 0, -1, 0};
    int64_t dim = (int64_t)1 << n;
    double* phi = (double*)malloc(sizeof(cplx) * (size_t)dim);
    if (!phi) return ORC_BAD;
    memcpy(phi, psi_ri, sizeof(cplx) * (size_t)dim);
    for (int a = 0; a < nops; ++a) {
        const double* m = NULL;
        if (ops[a] == 'X') m = X;
        else if (ops[a] == 'Y') m = Y;
        else if (ops[a] == 'Z') m = Z;
        else if (ops[a] == 'I') continue;
        else { free(phi); return ORC_BAD; }
        if (orc_apply(phi, n, m, &qubits[a], 1, NULL, NULL, 0) != ORC_OK) {
            free(phi);
            return ORC_BAD;
        }
    }
    double re, im;
    inner((const cplx*)psi_ri, (const cplx*)phi, dim, &re, &im);
    double nrm = orc_norm(psi_ri, n);
    free(phi);
    out[0] = re / nrm;
    out[1] = im / nrm;
    out[2] = nrm;
    return ORC_OK;
}

/*
 * Sampler (Table I: sampling bit strings as measurement outcomes without
 * collapsing the state).  p_i = |psi_i|^2, C_i = sum_{j<=i} p_j (compensated,
 * in index order), r = u * C_{2^n - 1}; the outcome is the smallest i with
 * r < C_i, so zero-probability indices are never returned.  With a bit
 * ordering (q_0 .. q_{m-1}), output bit a is bit q_a of that index;
 * bit_ordering == NULL returns the full index.  `cdf_out`, if not NULL,
 * receives C (2^n doubles).
 */
/* ------------------------------------------------------------------------ */
/* Pauli rotation (Table I: rotation of the state vector by a Pauli string): */
/* psi <- exp(i theta P) psi = cos(theta) psi + i sin(theta) P psi, with P   */
/* the product of the single-qubit Paulis of the string (the identity on    */
/* every other qubit), applied to the indices whose control bits equal the  */
/* control values; every other amplitude is unchanged.                      */
/* ------------------------------------------------------------------------ */

int orc_apply_pauli_rotation(double* psi_ri, int n, double theta, const int* qubits, const char* ops, int nops,
                             const int* controls, const int* cvals, int nc)
{
    static const double X[8] = {0, 0, 1, 0, 1, 0, 0, 0};
    static const double Y[8] = {0, 0, 0, -1, 0, 1, 0, 0};
    static const double Z[8] = {1, 0, 0, 0, 0, 0, -1, 0};
    if (n < 1 || n > 40 || nops < 0 || nc < 0) return ORC_BAD;
    uint64_t used = 0, cmask = 0, cval = 0;
    for (int a = 0; a < nops; ++a) {
        if (qubits[a] < 0 || qubits[a] >= n || (used >> qubits[a] & 1)) return ORC_BAD;
        used |= (uint64_t)1 << qubits[a];
    }
    for (int a = 0; a < nc; ++a) {
        uint64_t b = (uint64_t)1 << controls[a];
        if (controls[a] < 0 || controls[a] >= n || (used & b)) return ORC_BAD;
        used |= b;
        cmask |= b;
        if (cvals == NULL || cvals[a]) cval |= b;
    }
    int64_t dim = (int64_t)1 << n;
    cplx* psi = (cplx*)psi_ri;
    cplx* phi = (cplx*)malloc(sizeof(cplx) * (size_t)dim);
    if (!phi) return ORC_BAD;
    memcpy(phi, psi, sizeof(cplx) * (size_t)dim);
    for (int a = 0; a < nops; ++a) {
        const double* m = NULL;
        if (ops[a] == 'X') m = X;
        else if (ops[a] == 'Y') m = Y;
        else if (ops[a] == 'Z') m = Z;
        else if (ops[a] == 'I') continue;
        else { free(phi); return ORC_BAD; }
        orc_apply((double*)phi, n, m, &qubits[a], 1, NULL, NULL, 0);
    }
    const double c = cos(theta), sn = sin(theta);
    for (int64_t i = 0; i < dim; ++i) {
        if (((uint64_t)i & cmask) != cval) continue;
        psi[i] = c * psi[i] + (I * sn) * phi[i];
    }
    free(phi);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Measurement (Table I: measurement on a Z-product basis and batched        */
/* single-qubit measurement, with probability and collapse as separate     */
/* steps).  probs[b] = sum of |psi_i|^2 over the indices i whose bits at    */
/* qubits[0..m-1] spell b (bit a of b = bit qubits[a] of i), unnormalised,  */
/* each bin a compensated sum in index order.                               */
/* ------------------------------------------------------------------------ */

int orc_measure_probs(const double* psi_ri, int n, const int* qubits, int m, double* probs)
{
    if (n < 1 || n > 40 || m < 1 || m > 20 || m > n) return ORC_BAD;
    uint64_t used = 0;
    for (int a = 0; a < m; ++a) {
        if (qubits[a] < 0 || qubits[a] >= n || (used >> qubits[a] & 1)) return ORC_BAD;
        used |= (uint64_t)1 << qubits[a];
    }
    const cplx* psi = (const cplx*)psi_ri;
    int64_t dim = (int64_t)1 << n;
    int64_t bins = (int64_t)1 << m;
    ksum* acc = (ksum*)calloc((size_t)bins, sizeof(ksum));
    if (!acc) return ORC_BAD;
    for (int64_t i = 0; i < dim; ++i) {
        int64_t b = 0;
        for (int a = 0; a < m; ++a) b |= (int64_t)((i >> qubits[a]) & 1) << a;
        const double re = creal(psi[i]), im = cimag(psi[i]);
        ks_add(&acc[b], re * re + im * im);
    }
    for (int64_t b = 0; b < bins; ++b) probs[b] = ks_val(&acc[b]);
    free(acc);
    return ORC_OK;
}

/* Collapse onto one outcome: amplitudes whose bits at qubits spell outcome  */
/* (parity < 0), or whose bits at qubits have that parity (parity 0 or 1),  */
/* are divided by sqrt(norm); all others become 0.                          */
int orc_collapse(double* psi_ri, int n, const int* qubits, int m, uint64_t outcome, int parity, double norm)
{
    if (n < 1 || n > 40 || m < 1 || m > n || !(norm > 0.0)) return ORC_BAD;
    uint64_t used = 0;
    for (int a = 0; a < m; ++a) {
        if (qubits[a] < 0 || qubits[a] >= n || (used >> qubits[a] & 1)) return ORC_BAD;
        used |= (uint64_t)1 << qubits[a];
    }
    cplx* psi = (cplx*)psi_ri;
    int64_t dim = (int64_t)1 << n;
    const double s = 1.0 / sqrt(norm);
    for (int64_t i = 0; i < dim; ++i) {
        uint64_t b = 0;
        int par = 0;
        for (int a = 0; a < m; ++a) {
            const int bit = (int)((i >> qubits[a]) & 1);
            b |= (uint64_t)bit << a;
            par ^= bit;
        }
        const int keep = parity < 0 ? (b == outcome) : (par == parity);
        psi[i] = keep ? s * psi[i] : 0.0;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Expectation of a dense k-qubit observable M (Table I: expectation with a  */
/* dense matrix observable): <psi| M |psi> / <psi|psi>, complex, with M on  */
/* targets (targets[0] = matrix LSB).  out = (re, im, <psi|psi>).           */
/* ------------------------------------------------------------------------ */

int orc_expect_matrix(const double* psi_ri, int n, const double* m_ri, const int* targets, int k, double* out)
{
    int64_t dim = (int64_t)1 << n;
    double* phi = (double*)malloc(sizeof(cplx) * (size_t)dim);
    if (!phi) return ORC_BAD;
    memcpy(phi, psi_ri, sizeof(cplx) * (size_t)dim);
    if (orc_apply(phi, n, m_ri, targets, k, NULL, NULL, 0) != ORC_OK) {
        free(phi);
        return ORC_BAD;
    }
    double re, im;
    inner((const cplx*)psi_ri, (const cplx*)phi, dim, &re, &im);
    double nrm = orc_norm(psi_ri, n);
    free(phi);
    out[0] = re / nrm;
    out[1] = im / nrm;
    out[2] = nrm;
    return ORC_OK;
}

int orc_sample(const double* psi_ri, int n, const double* u, int64_t nshots,
               const int* bit_ordering, int nbits, uint64_t* out, double* cdf_out)
{
    int64_t dim = (int64_t)1 << n;
    double* cdf = cdf_out ? cdf_out : (double*)malloc(sizeof(double) * (size_t)dim);
    if (!cdf) return ORC_BAD;
    ksum k = {0.0, 0.0};
    for (int64_t i = 0; i < dim; ++i) {
        double re = psi_ri[2 * i], im = psi_ri[2 * i + 1];
        ks_add(&k, re * re);
        ks_add(&k, im * im);
        cdf[i] = ks_val(&k);
    }
    double total = cdf[dim - 1];
    for (int64_t s = 0; s < nshots; ++s) {
        if (!(u[s] >= 0.0 && u[s] < 1.0)) {
            if (!cdf_out) free(cdf);
            return ORC_BAD;
        }
        double r = u[s] * total;
        /* smallest i with r < cdf[i]; cdf is non-decreasing and r < cdf[dim-1] */
        int64_t lo = 0, hi = dim - 1;
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if (r < cdf[mid]) hi = mid;
            else lo = mid + 1;
        }
        uint64_t idx = (uint64_t)lo;
        if (bit_ordering) {
            uint64_t v = 0;
            for (int a = 0; a < nbits; ++a) v |= ((idx >> bit_ordering[a]) & 1u) << a;
            idx = v;
        }
        out[s] = idx;
    }
    if (!cdf_out) free(cdf);
    return ORC_OK;
}

/* Number of OpenMP threads the oracle's parallel loops use. */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the number of OpenMP threads of the parallel loops (n >= 1). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* |0..0> or |x> */
void orc_set_basis(double* psi_ri, int n, uint64_t x)
{
    int64_t dim = (int64_t)1 << n;
    memset(psi_ri, 0, sizeof(cplx) * (size_t)dim);
    psi_ri[2 * x] = 1.0;
}
