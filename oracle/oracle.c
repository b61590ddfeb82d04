/*
 * FP64 CPU oracle for dense state-vector simulation — TEST INFRASTRUCTURE.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code, header, table or
 * helper with the GPU library: the two are written independently so that
 * one can check the other.
 *
 * Everything here is the plain definition from QCLAB (Keip, Camps,
 * Van Beeumen 2025), written out one output element at a time, in double
 * precision, with no blocking or reordering:
 *
 *  - Gate application (section 3.2, "Application of Gates"): the register
 *    operator is U = I_l (x) U' (x) I_r.  Row i of that Kronecker product
 *    has the entries U'[r(i), t] at the columns that agree with i outside
 *    the gate's qubits and carry local index t on them, so
 *        (U psi)_i = sum_t U'[r(i), t] psi_{i with local index t}.
 *    For gates on non-adjacent or reordered qubits the same formula holds
 *    with the local index read from those qubits (qubit list order: first
 *    listed = most significant bit of the local index).  A controlled gate
 *    is Pc (x) U' + (I - Pc) (x) I with Pc the projector on the control
 *    values (section 2 and the MCX gates of section 5.4): rows whose control
 *    bits differ from the control values are copied.
 *  - Measurement probabilities (section 3.3): P(s) is the sum of |psi_i|^2
 *    over the indices whose measured bits equal s.
 *  - Collapse (section 3.3): keep the amplitudes of the outcome, divide by
 *    sqrt(P(outcome)), zero the others.
 *  - Pauli expectation <psi|P|psi> = sum_i conj(psi_i) (P psi)_i, where row
 *    i of the Kronecker product P = s_0 (x) ... (x) s_{n-1} has its single
 *    non-zero entry at column j (j differs from i exactly on the qubits with
 *    an X or Y) and equals the product of the 2x2 Pauli matrix entries
 *    s_q[i_q][j_q].  This is the Pauli form behind the tomography
 *    coefficients S1..S3 of section 5.2.
 *
 * Index convention (sections 3.1 and 5.1: the teleportation input
 * kron(v, bell) puts v on qubit 0): qubit q is bit n-1-q of the amplitude
 * index, so qubit 0 is the most significant bit.
 *
 * Sums of squares use Neumaier compensated summation so that the oracle's
 * own rounding error stays near one ulp even for 2^28 terms.
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fcx-limited-range -fPIC -shared
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* value (0/1) of qubit q in index i */
static inline int qubit_value(uint64_t i, int n, int q) {
    return (int)((i >> (n - 1 - q)) & 1u);
}

/* local index of i on the listed qubits; qubits[0] is the most significant */
static inline uint64_t read_local(uint64_t i, int n, int k, const int *qubits) {
    uint64_t r = 0;
    for (int j = 0; j < k; ++j) r = (r << 1) | (uint64_t)qubit_value(i, n, qubits[j]);
    return r;
}

/* i with the listed qubits overwritten by local index r */
static inline uint64_t write_local(uint64_t i, int n, int k, const int *qubits, uint64_t r) {
    for (int j = 0; j < k; ++j) {
        uint64_t bit = (r >> (k - 1 - j)) & 1u;
        uint64_t m = (uint64_t)1 << (n - 1 - qubits[j]);
        i = bit ? (i | m) : (i & ~m);
    }
    return i;
}

/* Neumaier compensated accumulator */
typedef struct { double s, c; } csum_t;
static inline void csum_add(csum_t *a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static inline double csum_value(const csum_t *a) { return a->s + a->c; }

int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/*
 * out = U psi for U = (controlled) I_l (x) u (x) I_r on the listed qubits.
 * in/out: 2^n complex doubles (out must not alias in).
 * u: 2^k x 2^k complex, row-major (u[r*d + t] = U'[r][t]).
 * ctrl/ctrl_val: nc control qubits and their required values (0 or 1).
 * Returns 0, or -1 on invalid arguments.
 */
int oracle_apply(const cplx *in, cplx *out, int n, int k, const int *qubits,
                 const cplx *u, int nc, const int *ctrl, const int *ctrl_val) {
    if (n < 1 || n > 40 || k < 0 || k > n || nc < 0 || k + nc > n) return -1;
    for (int a = 0; a < k; ++a) {
        if (qubits[a] < 0 || qubits[a] >= n) return -1;
        for (int b = 0; b < a; ++b) if (qubits[a] == qubits[b]) return -1;
    }
    for (int a = 0; a < nc; ++a) {
        if (ctrl[a] < 0 || ctrl[a] >= n) return -1;
        for (int b = 0; b < k; ++b) if (ctrl[a] == qubits[b]) return -1;
        for (int b = 0; b < a; ++b) if (ctrl[a] == ctrl[b]) return -1;
    }
    const uint64_t dim = (uint64_t)1 << n;
    const uint64_t d = (uint64_t)1 << k;
#pragma omp parallel for schedule(static)
    for (int64_t ii = 0; ii < (int64_t)dim; ++ii) {
        uint64_t i = (uint64_t)ii;
        int active = 1;
        for (int a = 0; a < nc; ++a)
            if (qubit_value(i, n, ctrl[a]) != (ctrl_val[a] ? 1 : 0)) active = 0;
        if (!active) { out[i] = in[i]; continue; }
        uint64_t r = read_local(i, n, k, qubits);
        cplx acc = 0.0;
        for (uint64_t t = 0; t < d; ++t)
            acc += u[r * d + t] * in[write_local(i, n, k, qubits, t)];
        out[i] = acc;
    }
    return 0;
}

/* P(s) for s in [0, 2^m): sum of |psi_i|^2 over i whose listed qubits read s.
 * With m == n and qubits 0..n-1 this is the full distribution. */
int oracle_probs(const cplx *psi, int n, int m, const int *qubits, double *out) {
    if (n < 1 || n > 40 || m < 0 || m > n || (m != n && m > 24)) return -1;
    for (int a = 0; a < m; ++a) {
        if (qubits[a] < 0 || qubits[a] >= n) return -1;
        for (int b = 0; b < a; ++b) if (qubits[a] == qubits[b]) return -1;
    }
    const uint64_t dim = (uint64_t)1 << n;
    const uint64_t bins = (uint64_t)1 << m;
    if (m == n) {
        /* every bin holds exactly one amplitude */
#pragma omp parallel for schedule(static)
        for (int64_t ii = 0; ii < (int64_t)dim; ++ii) {
            uint64_t i = (uint64_t)ii;
            double a = creal(psi[i]), b = cimag(psi[i]);
            out[read_local(i, n, m, qubits)] = a * a + b * b;
        }
        return 0;
    }
    int nt = oracle_threads();
    csum_t *part = (csum_t *)calloc((size_t)nt * bins, sizeof(csum_t));
    if (!part) return -1;
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        csum_t *mine = part + (size_t)tid * bins;
#pragma omp for schedule(static)
        for (int64_t ii = 0; ii < (int64_t)dim; ++ii) {
            uint64_t i = (uint64_t)ii;
            double a = creal(psi[i]), b = cimag(psi[i]);
            csum_add(&mine[read_local(i, n, m, qubits)], a * a + b * b);
        }
    }
    for (uint64_t s = 0; s < bins; ++s) {
        csum_t acc = {0.0, 0.0};
        for (int t = 0; t < nt; ++t) {
            csum_add(&acc, part[(size_t)t * bins + s].s);
            csum_add(&acc, part[(size_t)t * bins + s].c);
        }
        out[s] = csum_value(&acc);
    }
    free(part);
    return 0;
}

/* Pauli matrix entry sigma[row][col] for sigma in {I,X,Y,Z}. */
static cplx pauli_entry(char s, int row, int col) {
    switch (s) {
    case 'I': return row == col ? 1.0 : 0.0;
    case 'X': return row != col ? 1.0 : 0.0;
    case 'Y': return row == col ? 0.0 : (row == 0 ? -I : I);
    case 'Z': return row == col ? (row == 0 ? 1.0 : -1.0) : 0.0;
    default: return NAN;
    }
}

/* <psi|P|psi> for the Pauli string p (n characters; character q acts on
 * qubit q).  Writes the real and imaginary parts. */
int oracle_expect_pauli(const cplx *psi, int n, const char *p, double *re, double *im) {
    if (n < 1 || n > 40) return -1;
    int nz = 0;
    int idx[64];
    for (int q = 0; q < n; ++q) {
        char c = p[q];
        if (c != 'I' && c != 'X' && c != 'Y' && c != 'Z') return -1;
        if (c != 'I') idx[nz++] = q;       /* identity factors contribute 1 */
    }
    const uint64_t dim = (uint64_t)1 << n;
    int nt = oracle_threads();
    csum_t *part = (csum_t *)calloc((size_t)nt * 2, sizeof(csum_t));
    if (!part) return -1;
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        csum_t *mine = part + (size_t)tid * 2;
#pragma omp for schedule(static)
        for (int64_t ii = 0; ii < (int64_t)dim; ++ii) {
            uint64_t i = (uint64_t)ii;
            uint64_t j = i;
            cplx coef = 1.0;
            for (int a = 0; a < nz; ++a) {
                int q = idx[a];
                int iq = qubit_value(i, n, q);
                int jq = (p[q] == 'X' || p[q] == 'Y') ? 1 - iq : iq;
                uint64_t m = (uint64_t)1 << (n - 1 - q);
                j = jq ? (j | m) : (j & ~m);
                coef *= pauli_entry(p[q], iq, jq);
            }
            cplx term = conj(psi[i]) * coef * psi[j];
            csum_add(&mine[0], creal(term));
            csum_add(&mine[1], cimag(term));
        }
    }
    csum_t r = {0, 0}, m = {0, 0};
    for (int t = 0; t < nt; ++t) {
        csum_add(&r, part[2 * t].s); csum_add(&r, part[2 * t].c);
        csum_add(&m, part[2 * t + 1].s); csum_add(&m, part[2 * t + 1].c);
    }
    *re = csum_value(&r);
    *im = csum_value(&m);
    free(part);
    return 0;
}

/* Collapse psi (in place) onto outcome b of qubit q and renormalise.
 * Writes P(outcome).  If P(outcome) is zero the state is left unchanged and
 * 1 is returned. */
int oracle_collapse(cplx *psi, int n, int q, int b, double *prob) {
    if (n < 1 || n > 40 || q < 0 || q >= n || (b != 0 && b != 1)) return -1;
    int qs[1] = {q};
    double pr[2];
    if (oracle_probs(psi, n, 1, qs, pr) != 0) return -1;
    *prob = pr[b];
    if (pr[b] == 0.0) return 1;
    const double scale = 1.0 / sqrt(pr[b]);
    const uint64_t dim = (uint64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t ii = 0; ii < (int64_t)dim; ++ii) {
        uint64_t i = (uint64_t)ii;
        psi[i] = (qubit_value(i, n, q) == b) ? psi[i] * scale : 0.0;
    }
    return 0;
}
