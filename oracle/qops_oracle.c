/*
 * FP64 CPU oracle for full-state (Schroedinger-style) circuit simulation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or table with the GPU simulator and is deliberately plain: one pass
 * over the state per gate, in list order, no fusion, no reordering, no layout
 * tricks, parallelised only by an OpenMP loop over independent amplitude
 * groups.
 *
 * What it computes (paper Sec. II-B, "Quantum Simulator"): a full-state
 * simulation keeps all 2^n complex amplitudes and updates them gate by gate;
 * it can report the final probability distribution.  Expectation values of
 * Z (Sec. IV-E, repeated QAOA runs build expectation values) are sums of
 * probabilities weighted by +-1.
 *
 * Conventions: qubit q is bit q of the basis index; a gate on ordered qubits
 * (q_0..q_{k-1}) has a 2^k x 2^k matrix whose index bit j belongs to q_j;
 * controls must all be 1 for the gate to act.  Amplitudes are stored
 * interleaved (re, im) in double precision.
 *
 * Gate matrices are the textbook ones (Nielsen & Chuang, the reference the
 * paper cites for its single-qubit merging), with U3 in the OpenQASM-3 form
 *   U3(t,p,l) = [[cos(t/2), -e^{il} sin(t/2)], [e^{ip} sin(t/2), e^{i(p+l)} cos(t/2)]].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum {
    ORC_H = 0, ORC_X, ORC_Y, ORC_Z, ORC_S, ORC_SDG, ORC_T, ORC_TDG, ORC_SX,
    ORC_RX, ORC_RY, ORC_RZ, ORC_P, ORC_U3,
    ORC_CX, ORC_CZ, ORC_CP, ORC_SWAP, ORC_RZZ, ORC_DENSE
};

#define ORC_MAXK 8

static void set(double* m, int dim, int r, int c, double re, double im)
{
    m[2 * (r * dim + c)] = re;
    m[2 * (r * dim + c) + 1] = im;
}

/* Number of target qubits of a kind (DENSE: given by the caller). */
int orc_kind_arity(int kind)
{
    if (kind <= ORC_U3) return 1;
    if (kind <= ORC_RZZ) return 2;
    return -1;
}

/* Writes the 2^k x 2^k matrix of a gate (interleaved complex, row-major). */
int orc_gate_matrix(int kind, const double* prm, int k, const double* dense, double* out)
{
    int dim;
    const double r2 = 1.0 / sqrt(2.0);
    if (kind == ORC_DENSE) {
        if (k < 1 || k > ORC_MAXK) return -1;
        dim = 1 << k;
        memcpy(out, dense, sizeof(double) * 2 * (size_t)dim * dim);
        return 0;
    }
    k = orc_kind_arity(kind);
    if (k < 0) return -1;
    dim = 1 << k;
    memset(out, 0, sizeof(double) * 2 * (size_t)dim * dim);
    double c, s;
    switch (kind) {
    case ORC_H: set(out, 2, 0, 0, r2, 0); set(out, 2, 0, 1, r2, 0);
                set(out, 2, 1, 0, r2, 0); set(out, 2, 1, 1, -r2, 0); break;
    case ORC_X: set(out, 2, 0, 1, 1, 0); set(out, 2, 1, 0, 1, 0); break;
    case ORC_Y: set(out, 2, 0, 1, 0, -1); set(out, 2, 1, 0, 0, 1); break;
    case ORC_Z: set(out, 2, 0, 0, 1, 0); set(out, 2, 1, 1, -1, 0); break;
    case ORC_S: set(out, 2, 0, 0, 1, 0); set(out, 2, 1, 1, 0, 1); break;
    case ORC_SDG: set(out, 2, 0, 0, 1, 0); set(out, 2, 1, 1, 0, -1); break;
    case ORC_T: set(out, 2, 0, 0, 1, 0); set(out, 2, 1, 1, r2, r2); break;
    case ORC_TDG: set(out, 2, 0, 0, 1, 0); set(out, 2, 1, 1, r2, -r2); break;
    case ORC_SX: set(out, 2, 0, 0, 0.5, 0.5); set(out, 2, 0, 1, 0.5, -0.5);
                 set(out, 2, 1, 0, 0.5, -0.5); set(out, 2, 1, 1, 0.5, 0.5); break;
    case ORC_RX: c = cos(prm[0] / 2); s = sin(prm[0] / 2);
                 set(out, 2, 0, 0, c, 0); set(out, 2, 0, 1, 0, -s);
                 set(out, 2, 1, 0, 0, -s); set(out, 2, 1, 1, c, 0); break;
    case ORC_RY: c = cos(prm[0] / 2); s = sin(prm[0] / 2);
                 set(out, 2, 0, 0, c, 0); set(out, 2, 0, 1, -s, 0);
                 set(out, 2, 1, 0, s, 0); set(out, 2, 1, 1, c, 0); break;
    case ORC_RZ: set(out, 2, 0, 0, cos(prm[0] / 2), -sin(prm[0] / 2));
                 set(out, 2, 1, 1, cos(prm[0] / 2), sin(prm[0] / 2)); break;
    case ORC_P: set(out, 2, 0, 0, 1, 0); set(out, 2, 1, 1, cos(prm[0]), sin(prm[0])); break;
    case ORC_U3: {
        double t = prm[0], p = prm[1], l = prm[2];
        c = cos(t / 2); s = sin(t / 2);
        set(out, 2, 0, 0, c, 0);
        set(out, 2, 0, 1, -cos(l) * s, -sin(l) * s);
        set(out, 2, 1, 0, cos(p) * s, sin(p) * s);
        set(out, 2, 1, 1, cos(p + l) * c, sin(p + l) * c);
        break;
    }
    /* two-qubit kinds: index bit 0 <-> q_0, bit 1 <-> q_1 */
    case ORC_CX: /* q_0 control, q_1 target: |1,t> -> |1,1-t> */
        set(out, 4, 0, 0, 1, 0); set(out, 4, 2, 2, 1, 0);
        set(out, 4, 1, 3, 1, 0); set(out, 4, 3, 1, 1, 0); break;
    case ORC_CZ:
        set(out, 4, 0, 0, 1, 0); set(out, 4, 1, 1, 1, 0);
        set(out, 4, 2, 2, 1, 0); set(out, 4, 3, 3, -1, 0); break;
    case ORC_CP:
        set(out, 4, 0, 0, 1, 0); set(out, 4, 1, 1, 1, 0);
        set(out, 4, 2, 2, 1, 0); set(out, 4, 3, 3, cos(prm[0]), sin(prm[0])); break;
    case ORC_SWAP:
        set(out, 4, 0, 0, 1, 0); set(out, 4, 1, 2, 1, 0);
        set(out, 4, 2, 1, 1, 0); set(out, 4, 3, 3, 1, 0); break;
    case ORC_RZZ: {
        double cc = cos(prm[0] / 2), ss = sin(prm[0] / 2);
        set(out, 4, 0, 0, cc, -ss); set(out, 4, 1, 1, cc, ss);
        set(out, 4, 2, 2, cc, ss); set(out, 4, 3, 3, cc, -ss); break;
    }
    default: return -1;
    }
    return 0;
}

/* Basis index with the bits of g placed, in order, into the positions that
 * are NOT listed in sorted_pos[0..m-1] (ascending). */
static uint64_t spread_around(uint64_t g, const int* sorted_pos, int m)
{
    uint64_t x = g;
    for (int i = 0; i < m; ++i) {
        uint64_t low = x & ((1ull << sorted_pos[i]) - 1);
        x = ((x >> sorted_pos[i]) << (sorted_pos[i] + 1)) | low;
    }
    return x;
}

/*
 * Applies the 2^k x 2^k matrix `u` to ordered qubits q[0..k-1] under controls
 * c[0..nc-1]:  for every x whose target bits are 0 and whose control bits are
 * 1, gather a_r = psi[x + sum_j r_j 2^{q_j}], write psi[...] = sum_s u[r][s] a_s.
 */
int orc_apply_matrix(int n, double* psi, int k, const int* q, int nc, const int* c, const double* u)
{
    if (k < 1 || k > ORC_MAXK || k > n) return -1;
    int sorted[ORC_MAXK];
    uint64_t cmask = 0;
    for (int j = 0; j < k; ++j) {
        if (q[j] < 0 || q[j] >= n) return -2;
        sorted[j] = q[j];
    }
    for (int j = 0; j < nc; ++j) {
        if (c[j] < 0 || c[j] >= n) return -2;
        cmask |= 1ull << c[j];
    }
    for (int a = 0; a < k; ++a)            /* insertion sort, k is tiny */
        for (int b = a + 1; b < k; ++b)
            if (sorted[b] < sorted[a]) { int t = sorted[a]; sorted[a] = sorted[b]; sorted[b] = t; }
    for (int a = 0; a + 1 < k; ++a)
        if (sorted[a] == sorted[a + 1]) return -3;
    for (int j = 0; j < k; ++j)
        if (cmask & (1ull << q[j])) return -3;

    const int dim = 1 << k;
    uint64_t off[1 << ORC_MAXK];
    for (int r = 0; r < dim; ++r) {
        uint64_t o = 0;
        for (int j = 0; j < k; ++j)
            if (r & (1 << j)) o |= 1ull << q[j];
        off[r] = o;
    }
    const int64_t ngroups = (int64_t)1 << (n - k);
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < ngroups; ++g) {
        uint64_t x = spread_around((uint64_t)g, sorted, k);
        if ((x & cmask) != cmask) continue;
        double a[2 << ORC_MAXK];
        for (int s = 0; s < dim; ++s) {
            a[2 * s] = psi[2 * (x + off[s])];
            a[2 * s + 1] = psi[2 * (x + off[s]) + 1];
        }
        for (int r = 0; r < dim; ++r) {
            double re = 0.0, im = 0.0;
            for (int s = 0; s < dim; ++s) {
                double ur = u[2 * (r * dim + s)], ui = u[2 * (r * dim + s) + 1];
                re += ur * a[2 * s] - ui * a[2 * s + 1];
                im += ur * a[2 * s + 1] + ui * a[2 * s];
            }
            psi[2 * (x + off[r])] = re;
            psi[2 * (x + off[r]) + 1] = im;
        }
    }
    return 0;
}

/*
 * Runs a gate list in order.  Gate i: kind[i]; its k targets are
 * qubits[i*8 .. i*8+k-1]; its controls ctrls[i*8 .. i*8+nctrl[i]-1]; its
 * parameters params[i*3 ..]; a DENSE gate's matrix starts at
 * mats + mat_off[i] (interleaved complex doubles) and has k = nq[i].
 * Returns 0, or -(1 + index of the failing gate).
 */
int orc_run(int n, double* psi, int ngates, const int* kind, const int* nq, const int* qubits,
            const int* nctrl, const int* ctrls, const double* params, const double* mats,
            const int64_t* mat_off)
{
    double u[2 << (2 * ORC_MAXK)];
    for (int i = 0; i < ngates; ++i) {
        int k = kind[i] == ORC_DENSE ? nq[i] : orc_kind_arity(kind[i]);
        if (k < 1 || k > ORC_MAXK) return -(1 + i);
        const double* dm = kind[i] == ORC_DENSE ? mats + mat_off[i] : NULL;
        if (orc_gate_matrix(kind[i], params + 3 * i, k, dm, u) != 0) return -(1 + i);
        if (orc_apply_matrix(n, psi, k, qubits + 8 * i, nctrl[i], ctrls + 8 * i, u) != 0) return -(1 + i);
    }
    return 0;
}

/* Threads the OpenMP loops use. */
int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the threads of later OpenMP loops (timing at one thread and at all
 * host cores); no effect on the arithmetic or its order within a group. */
void orc_set_num_threads(int t)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* |x0>: all zero except amplitude x0 = 1. */
void orc_basis(int n, double* psi, uint64_t x0)
{
    memset(psi, 0, sizeof(double) * 2 * ((size_t)1 << n));
    psi[2 * x0] = 1.0;
}

/* Sum over x of |psi_x|^2, in index order. */
double orc_norm(int n, const double* psi)
{
    double s = 0.0;
    const uint64_t N = 1ull << n;
    for (uint64_t x = 0; x < N; ++x) s += psi[2 * x] * psi[2 * x] + psi[2 * x + 1] * psi[2 * x + 1];
    return s;
}

/* Marginal distribution of qubits q[0..m-1]: out[y] = sum of |psi_x|^2 over x
 * whose bit q_j equals bit j of y; summed in index order. */
void orc_probabilities(int n, const double* psi, int m, const int* q, double* out)
{
    memset(out, 0, sizeof(double) * ((size_t)1 << m));
    const uint64_t N = 1ull << n;
    for (uint64_t x = 0; x < N; ++x) {
        uint64_t y = 0;
        for (int j = 0; j < m; ++j) y |= ((x >> q[j]) & 1ull) << j;
        out[y] += psi[2 * x] * psi[2 * x] + psi[2 * x + 1] * psi[2 * x + 1];
    }
}

/* <Z_a Z_b> = sum_x |psi_x|^2 (-1)^(b_a(x) + b_b(x)) for each pair (a, b) =
 * (pairs[2i], pairs[2i+1]); the two-qubit correlators a diagonal cost
 * Hamiltonian such as Max-Cut's is built from (repeated QAOA runs, paper
 * Sec. IV-E).  Plain sequential sum over x. */
void orc_expect_zz(int n, const double* psi, const int* pairs, int npairs, double* out)
{
    for (int i = 0; i < npairs; ++i) out[i] = 0.0;
    const uint64_t N = 1ull << n;
    for (uint64_t x = 0; x < N; ++x) {
        double p = psi[2 * x] * psi[2 * x] + psi[2 * x + 1] * psi[2 * x + 1];
        for (int i = 0; i < npairs; ++i) {
            const uint64_t s = ((x >> pairs[2 * i]) ^ (x >> pairs[2 * i + 1])) & 1ull;
            out[i] += s ? -p : p;
        }
    }
}

/* <Z_q> = sum_x |psi_x|^2 (1 - 2 b_q(x)) for every qubit q, in index order. */
void orc_expect_z(int n, const double* psi, double* out)
{
    for (int q = 0; q < n; ++q) out[q] = 0.0;
    const uint64_t N = 1ull << n;
    for (uint64_t x = 0; x < N; ++x) {
        double p = psi[2 * x] * psi[2 * x] + psi[2 * x + 1] * psi[2 * x + 1];
        for (int q = 0; q < n; ++q) out[q] += ((x >> q) & 1ull) ? -p : p;
    }
}
