/*
 * FP64 CPU oracle for the Schroedinger-Feynman path sum.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or helper with the GPU library; both only read the
 * same gate records and input arrays.
 *
 * What it computes (arXiv:1807.10749):
 *   O1  full state vector: |0...0> evolved gate by gate in list order
 *       (Section 1: the circuits start with H on every qubit and interleave
 *       CZ layers with one-qubit gates).
 *   O2  Schroedinger-Feynman path sum (Section 2, Eq. (CZ); Section 3, the
 *       path expansion |psi> = sum_j |phi_j>): the qubits are split into
 *       block A (holding qubit 0) and block B; every CZ that crosses the cut
 *       is written P0 (x) I + P1 (x) Z, each path picks one term per crossing
 *       CZ, both blocks are evolved separately, and requested amplitudes are
 *       accumulated as sum_p psiA_p(x_A) * psiB_p(x_B) ("Final-state
 *       amplitudes", end of Section 2).
 *   Path selection for fidelity f (Section 3, Eq. (fid)): ceil(f 2^k)
 *   distinct path ids drawn with Floyd's algorithm over SplitMix64.
 *   Two-qubit gates (section on harder benchmarks through two-qubit gates):
 *   iSWAP inside a block is applied as a 4x4 matrix; a crossing two-qubit
 *   gate G is split as in Eq. (4way), sum_{i,j} |i><j| (x) G_ij with the
 *   block-A endpoint first, term r = 2i + j from two path bits (a crossing
 *   CZ keeps the Section 2 split with one bit).
 *   Rejection sampling of bitstrings from a batch of output probabilities
 *   (Section "Frugal rejection sampling", Algorithms 1 and 2): candidate
 *   bitstrings, acceptance and the per-batch sampling-error estimate.
 *
 * Readings of points the paper leaves open (kept identical in the GPU path
 * by definition, never by shared code):
 *   - gate matrices: H = [[1,1],[1,-1]]/sqrt2, X^1/2 = [[1+i,1-i],[1-i,1+i]]/2,
 *     Y^1/2 = [[1+i,-1-i],[1+i,1+i]]/2, T = diag(1, e^{i pi/4});
 *   - bitstring bit q is the value of qubit q; local index of a qubit inside
 *     its block is its rank among the block's qubits;
 *   - crossing gates are ordered by (cycle, smaller qubit id); the first
 *     takes the highest path bits (one for a CZ, two for an iSWAP), so in a
 *     CZ-only circuit crossing CZ j is decided by bit (k-1-j); the projector
 *     goes on the block-A endpoint and Z on the block-B endpoint.
 *
 * Everything is plain loops in double precision.  OpenMP is used only to
 * spread independent loop iterations over host cores.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    uint8_t kind;   /* 0 H, 1 X^1/2, 2 Y^1/2, 3 T, 4 CZ */
    uint8_t pad;
    uint16_t cycle;
    uint16_t q0, q1;
} or_gate;

enum { OR_H = 0, OR_XH = 1, OR_YH = 2, OR_T = 3, OR_CZ = 4, OR_ISWAP = 5 };

/* Two-qubit gate matrices, row-major 4x4 in the basis |x_q0 x_q1> (index 2 x_q0 + x_q1).
 * iSWAP (section on two-qubit gates): |00> -> |00>, |01> -> i|10>, |10> -> i|01>, |11> -> |11>. */
static int gate_matrix2(int kind, double complex m[16])
{
    for (int i = 0; i < 16; ++i) m[i] = 0.0;
    if (kind == OR_CZ) {
        m[0] = 1.0; m[5] = 1.0; m[10] = 1.0; m[15] = -1.0;
        return 0;
    }
    if (kind == OR_ISWAP) {
        m[0] = 1.0; m[6] = I; m[9] = I; m[15] = 1.0;
        return 0;
    }
    return -1;
}

int or_gate_matrix2(int kind, double *out)
{
    double complex m[16];
    if (gate_matrix2(kind, m)) return -1;
    for (int i = 0; i < 16; ++i) { out[2 * i] = creal(m[i]); out[2 * i + 1] = cimag(m[i]); }
    return 0;
}

/* Section on two-qubit gates, Eq. (4way): a two-qubit gate G whose first qubit sits in block A
 * is  sum_{i,j} |i><j| (x) G_ij  with G_ij the 2x2 block of rows 2i.. and columns 2j..; term
 * r = 2i + j.  A CZ has only the diagonal terms, which are the Section 2 branches
 * P0 (x) I + P1 (x) Z; it keeps one path bit, with r = 3 s (s = 0: P0 (x) I, s = 1: P1 (x) Z). */
static void branch_ops(int kind, int r, double complex ea[4], double complex gb[4])
{
    double complex m[16];
    gate_matrix2(kind, m);
    const int i = r >> 1, j = r & 1;
    for (int t = 0; t < 4; ++t) ea[t] = 0.0;
    ea[2 * i + j] = 1.0;                                   /* |i><j| */
    for (int s = 0; s < 2; ++s)
        for (int t = 0; t < 2; ++t) gb[2 * s + t] = m[(2 * i + s) * 4 + (2 * j + t)];
}

int or_branch_ops(int kind, int r, double *ea_out, double *gb_out)
{
    if ((kind != OR_CZ && kind != OR_ISWAP) || r < 0 || r > 3) return -1;
    double complex ea[4], gb[4];
    branch_ops(kind, r, ea, gb);
    for (int t = 0; t < 4; ++t) {
        ea_out[2 * t] = creal(ea[t]); ea_out[2 * t + 1] = cimag(ea[t]);
        gb_out[2 * t] = creal(gb[t]); gb_out[2 * t + 1] = cimag(gb[t]);
    }
    return 0;
}

/* path bits a crossing two-qubit gate takes: 1 for CZ (two terms), 2 for iSWAP (four) */
static int branch_bits(int kind) { return kind == OR_ISWAP ? 2 : 1; }

/* ------------------------------------------------------------------ */
/* Gate matrices, row-major m[0]=u00 m[1]=u01 m[2]=u10 m[3]=u11.        */
/* ------------------------------------------------------------------ */
static int gate_matrix(int kind, double complex m[4])
{
    const double r = 1.0 / sqrt(2.0);
    switch (kind) {
    case OR_H:
        m[0] = r; m[1] = r; m[2] = r; m[3] = -r;
        return 0;
    case OR_XH:
        m[0] = 0.5 * (1.0 + I); m[1] = 0.5 * (1.0 - I);
        m[2] = 0.5 * (1.0 - I); m[3] = 0.5 * (1.0 + I);
        return 0;
    case OR_YH:
        m[0] = 0.5 * (1.0 + I); m[1] = 0.5 * (-1.0 - I);
        m[2] = 0.5 * (1.0 + I); m[3] = 0.5 * (1.0 + I);
        return 0;
    case OR_T:
        m[0] = 1.0; m[1] = 0.0; m[2] = 0.0; m[3] = cexp(I * M_PI / 4.0);
        return 0;
    default:
        return -1;
    }
}

/* Exported copy of the matrices for the tests: out = 8 doubles (re, im). */
int or_gate_matrix(int kind, double *out)
{
    double complex m[4];
    if (gate_matrix(kind, m)) return -1;
    for (int i = 0; i < 4; ++i) { out[2 * i] = creal(m[i]); out[2 * i + 1] = cimag(m[i]); }
    return 0;
}

/* Apply a one-qubit matrix on bit t of a 2^n vector. */
static void apply_1q(double complex *psi, int n, int t, const double complex m[4])
{
    const int64_t half = (int64_t)1 << (n - 1);
    const uint64_t low = ((uint64_t)1 << t) - 1;
#pragma omp parallel for schedule(static) if (n > 14)
    for (int64_t i = 0; i < half; ++i) {
        uint64_t i0 = (((uint64_t)i & ~low) << 1) | ((uint64_t)i & low);
        uint64_t i1 = i0 | ((uint64_t)1 << t);
        double complex a = psi[i0], b = psi[i1];
        psi[i0] = m[0] * a + m[1] * b;
        psi[i1] = m[2] * a + m[3] * b;
    }
}

/* Two-qubit matrix on bits a (first) and b of a 2^n vector. */
static void apply_2q(double complex *psi, int n, int a, int b, const double complex m[16])
{
    const int64_t quarter = (int64_t)1 << (n - 2);
    const int lo = a < b ? a : b, hi = a < b ? b : a;
#pragma omp parallel for schedule(static) if (n > 14)
    for (int64_t i = 0; i < quarter; ++i) {
        uint64_t x = (uint64_t)i;
        x = ((x >> lo) << (lo + 1)) | (x & (((uint64_t)1 << lo) - 1));
        x = ((x >> hi) << (hi + 1)) | (x & (((uint64_t)1 << hi) - 1));
        uint64_t idx[4];
        double complex v[4];
        for (int r = 0; r < 4; ++r) {
            idx[r] = x | ((uint64_t)(r >> 1) << a) | ((uint64_t)(r & 1) << b);
            v[r] = psi[idx[r]];
        }
        for (int r = 0; r < 4; ++r)
            psi[idx[r]] = m[4 * r] * v[0] + m[4 * r + 1] * v[1] + m[4 * r + 2] * v[2] + m[4 * r + 3] * v[3];
    }
}

/* CZ on bits a, b: negate amplitudes whose bits a and b are both 1. */
static void apply_cz(double complex *psi, int n, int a, int b)
{
    const int64_t size = (int64_t)1 << n;
#pragma omp parallel for schedule(static) if (n > 14)
    for (int64_t i = 0; i < size; ++i)
        if ((((uint64_t)i >> a) & 1) && (((uint64_t)i >> b) & 1)) psi[i] = -psi[i];
}

/* Projector P_s on bit a: zero amplitudes whose bit a differs from s. */
static void apply_projector(double complex *psi, int n, int a, int s)
{
    const int64_t size = (int64_t)1 << n;
#pragma omp parallel for schedule(static) if (n > 14)
    for (int64_t i = 0; i < size; ++i)
        if ((int)(((uint64_t)i >> a) & 1) != s) psi[i] = 0.0;
}

/* Pauli Z on bit b: negate amplitudes whose bit b is 1. */
static void apply_z(double complex *psi, int n, int b)
{
    const int64_t size = (int64_t)1 << n;
#pragma omp parallel for schedule(static) if (n > 14)
    for (int64_t i = 0; i < size; ++i)
        if (((uint64_t)i >> b) & 1) psi[i] = -psi[i];
}

static int is_2q(int kind) { return kind == OR_CZ || kind == OR_ISWAP; }

static int check_gates(int n, const or_gate *g, size_t ng)
{
    for (size_t i = 0; i < ng; ++i) {
        if (g[i].kind > OR_ISWAP || g[i].q0 >= n) return -1;
        if (is_2q(g[i].kind) && (g[i].q1 >= n || g[i].q1 == g[i].q0)) return -1;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* O1: full state vector.  psi_out holds 2^n complex (re, im) doubles. */
/* ------------------------------------------------------------------ */
int or_full_state(int n, const or_gate *gates, size_t ng, double *psi_out)
{
    if (n < 1 || n > 34 || check_gates(n, gates, ng)) return -1;
    double complex *psi = (double complex *)psi_out;
    const int64_t size = (int64_t)1 << n;
#pragma omp parallel for schedule(static) if (n > 14)
    for (int64_t i = 0; i < size; ++i) psi[i] = 0.0;
    psi[0] = 1.0;
    for (size_t i = 0; i < ng; ++i) {
        if (gates[i].kind == OR_CZ) {
            apply_cz(psi, n, gates[i].q0, gates[i].q1);
        } else if (gates[i].kind == OR_ISWAP) {
            double complex m[16];
            gate_matrix2(OR_ISWAP, m);
            apply_2q(psi, n, gates[i].q0, gates[i].q1, m);
        } else {
            double complex m[4];
            gate_matrix(gates[i].kind, m);
            apply_1q(psi, n, gates[i].q0, m);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Bit helpers                                                         */
/* ------------------------------------------------------------------ */
uint64_t or_pext(uint64_t x, uint64_t mask)
{
    uint64_t out = 0;
    int j = 0;
    for (int q = 0; q < 64; ++q)
        if ((mask >> q) & 1) { out |= ((x >> q) & 1) << j; ++j; }
    return out;
}

static int popcount64(uint64_t x)
{
    int c = 0;
    while (x) { x &= x - 1; ++c; }
    return c;
}

/* Local index of qubit q inside the block given by mask = its rank. */
static int local_index(uint64_t mask, int q)
{
    return popcount64(mask & (((uint64_t)1 << q) - 1));
}

/* Crossing two-qubit gates ordered by (cycle, smaller qubit); returns their number or -1.
 * idx_out (capacity cap) receives gate indices in path-bit order. */
int or_cut_gates(int n, const or_gate *gates, size_t ng, uint64_t mask_a,
                 int64_t *idx_out, int cap)
{
    if (check_gates(n, gates, ng)) return -1;
    int k = 0;
    for (size_t i = 0; i < ng; ++i) {
        if (!is_2q(gates[i].kind)) continue;
        int ina = (int)((mask_a >> gates[i].q0) & 1), inb = (int)((mask_a >> gates[i].q1) & 1);
        if (ina == inb) continue;
        if (k < cap && idx_out) idx_out[k] = (int64_t)i;
        ++k;
    }
    if (k > cap || !idx_out) return k;
    /* insertion sort on (cycle, min qubit) keeps equal keys in list order */
    for (int a = 1; a < k; ++a) {
        int64_t v = idx_out[a];
        int cv = gates[v].cycle;
        int mv = gates[v].q0 < gates[v].q1 ? gates[v].q0 : gates[v].q1;
        int b = a - 1;
        while (b >= 0) {
            int64_t w = idx_out[b];
            int cw = gates[w].cycle;
            int mw = gates[w].q0 < gates[w].q1 ? gates[w].q0 : gates[w].q1;
            if (cw < cv || (cw == cv && mw <= mv)) break;
            idx_out[b + 1] = w;
            --b;
        }
        idx_out[b + 1] = v;
    }
    return k;
}

/* ------------------------------------------------------------------ */
/* O2: Schroedinger-Feynman path sum.                                  */
/* ------------------------------------------------------------------ */
typedef struct {
    int n, qa, qb, k;
    uint64_t mask_a, mask_b;
    const or_gate *gates;
    size_t ng;
    int *bit_of_gate;   /* per gate: lowest path bit of the term index deciding it, or -1 */
} or_cut_info;

/* Evolve both blocks for one path id.  psiA has 2^qa entries, psiB 2^qb. */
static void evolve_path(const or_cut_info *c, uint64_t path,
                        double complex *psiA, double complex *psiB)
{
    const int64_t sa = (int64_t)1 << c->qa, sb = (int64_t)1 << c->qb;
    for (int64_t i = 0; i < sa; ++i) psiA[i] = 0.0;
    for (int64_t i = 0; i < sb; ++i) psiB[i] = 0.0;
    psiA[0] = 1.0;
    psiB[0] = 1.0;
    for (size_t g = 0; g < c->ng; ++g) {
        const or_gate *G = &c->gates[g];
        int q0 = G->q0;
        int a0 = (int)((c->mask_a >> q0) & 1);
        if (!is_2q(G->kind)) {
            double complex m[4];
            gate_matrix(G->kind, m);
            if (a0) apply_1q(psiA, c->qa, local_index(c->mask_a, q0), m);
            else    apply_1q(psiB, c->qb, local_index(c->mask_b, q0), m);
            continue;
        }
        int q1 = G->q1;
        int a1 = (int)((c->mask_a >> q1) & 1);
        if (a0 == a1) {
            double complex *psi = a0 ? psiA : psiB;
            const int nq = a0 ? c->qa : c->qb;
            const uint64_t mk = a0 ? c->mask_a : c->mask_b;
            if (G->kind == OR_CZ) {
                apply_cz(psi, nq, local_index(mk, q0), local_index(mk, q1));
            } else {
                double complex m[16];
                gate_matrix2(G->kind, m);
                apply_2q(psi, nq, local_index(mk, q0), local_index(mk, q1), m);
            }
        } else if (G->kind == OR_CZ) {
            /* crossing CZ = P0 (x) I + P1 (x) Z; this path takes term s */
            int s = (int)((path >> c->bit_of_gate[g]) & 1);
            int qa_ = a0 ? q0 : q1, qb_ = a0 ? q1 : q0;
            apply_projector(psiA, c->qa, local_index(c->mask_a, qa_), s);
            if (s) apply_z(psiB, c->qb, local_index(c->mask_b, qb_));
        } else {
            /* Eq. (4way) with the block-A endpoint as the first qubit (a symmetric gate such as
             * iSWAP reads the same either way); this path takes term r = 2i + j */
            int r = (int)((path >> c->bit_of_gate[g]) & 3);
            int qa_ = a0 ? q0 : q1, qb_ = a0 ? q1 : q0;
            double complex ea[4], gb[4];
            branch_ops(G->kind, r, ea, gb);
            apply_1q(psiA, c->qa, local_index(c->mask_a, qa_), ea);
            apply_1q(psiB, c->qb, local_index(c->mask_b, qb_), gb);
        }
    }
}

static int make_cut_info(int n, const or_gate *gates, size_t ng, uint64_t mask_a, or_cut_info *c)
{
    if (n < 2 || n > 64 || check_gates(n, gates, ng)) return -1;
    uint64_t all = n == 64 ? ~(uint64_t)0 : (((uint64_t)1 << n) - 1);
    if (!(mask_a & 1) || (mask_a & ~all) || (mask_a == all)) return -1;
    c->n = n;
    c->mask_a = mask_a;
    c->mask_b = all & ~mask_a;
    c->qa = popcount64(c->mask_a);
    c->qb = popcount64(c->mask_b);
    c->gates = gates;
    c->ng = ng;
    if (c->qa > 30 || c->qb > 30) return -1;
    int nc = or_cut_gates(n, gates, ng, mask_a, NULL, 0);
    if (nc < 0) return -1;
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (nc ? nc : 1));
    c->bit_of_gate = (int *)malloc(sizeof(int) * (ng ? ng : 1));
    for (size_t i = 0; i < ng; ++i) c->bit_of_gate[i] = -1;
    or_cut_gates(n, gates, ng, mask_a, idx, nc);
    /* the first crossing gate takes the highest path bits: crossing gate j's term index sits
     * right below the bits of the gates before it */
    int k = 0;
    for (int j = 0; j < nc; ++j) k += branch_bits(gates[idx[j]].kind);
    if (k > 63) { free(idx); free(c->bit_of_gate); return -1; }
    int top = k;
    for (int j = 0; j < nc; ++j) {
        top -= branch_bits(gates[idx[j]].kind);
        c->bit_of_gate[idx[j]] = top;
    }
    free(idx);
    c->k = k;
    return 0;
}

/*
 * amps_out: 2*nbits doubles (re, im), overwritten with
 *   sum over the listed paths (in the listed order) of psiA_p(x_A) psiB_p(x_B).
 * normsA_out / normsB_out (optional, npaths doubles): ||psiA_p||^2, ||psiB_p||^2.
 */
int or_path_sum(int n, const or_gate *gates, size_t ng, uint64_t mask_a,
                const uint64_t *paths, int64_t npaths,
                const uint64_t *bits, int64_t nbits, double *amps_out,
                double *normsA_out, double *normsB_out)
{
    or_cut_info c;
    if (make_cut_info(n, gates, ng, mask_a, &c)) return -1;
    for (int64_t p = 0; p < npaths; ++p)
        if (c.k < 64 && (paths[p] >> c.k) != 0) { free(c.bit_of_gate); return -1; }
    uint64_t all = n == 64 ? ~(uint64_t)0 : (((uint64_t)1 << n) - 1);
    for (int64_t j = 0; j < nbits; ++j)
        if (bits[j] & ~all) { free(c.bit_of_gate); return -1; }

    const int64_t sa = (int64_t)1 << c.qa, sb = (int64_t)1 << c.qb;
    uint64_t *xa = (uint64_t *)malloc(sizeof(uint64_t) * (nbits ? nbits : 1));
    uint64_t *xb = (uint64_t *)malloc(sizeof(uint64_t) * (nbits ? nbits : 1));
    for (int64_t j = 0; j < nbits; ++j) {
        xa[j] = or_pext(bits[j], c.mask_a);
        xb[j] = or_pext(bits[j], c.mask_b);
    }
    double complex *amps = (double complex *)amps_out;
    for (int64_t j = 0; j < nbits; ++j) amps[j] = 0.0;

    /* Large blocks: one path at a time, amplitude loops spread over cores.
     * Small blocks: paths spread over cores, each core summing its own
     * contiguous run of paths; the per-core sums are added in core order. */
    const int per_path_parallel = (c.qa > 16 || c.qb > 16);
    if (per_path_parallel) {
        double complex *A = (double complex *)malloc(sizeof(double complex) * sa);
        double complex *B = (double complex *)malloc(sizeof(double complex) * sb);
        for (int64_t p = 0; p < npaths; ++p) {
            evolve_path(&c, paths[p], A, B);
            for (int64_t j = 0; j < nbits; ++j) amps[j] += A[xa[j]] * B[xb[j]];
            if (normsA_out) { double s = 0; for (int64_t i = 0; i < sa; ++i) s += creal(A[i] * conj(A[i])); normsA_out[p] = s; }
            if (normsB_out) { double s = 0; for (int64_t i = 0; i < sb; ++i) s += creal(B[i] * conj(B[i])); normsB_out[p] = s; }
        }
        free(A); free(B);
    } else {
        int nt = 1;
#ifdef _OPENMP
        nt = omp_get_max_threads();
#endif
        if (nt > npaths && npaths > 0) nt = (int)npaths;
        if (nt < 1) nt = 1;
        double complex *part = (double complex *)calloc((size_t)nt * (nbits ? nbits : 1), sizeof(double complex));
#pragma omp parallel num_threads(nt)
        {
            int t = 0;
#ifdef _OPENMP
            t = omp_get_thread_num();
#endif
            int64_t lo = npaths * t / nt, hi = npaths * (t + 1) / nt;
            double complex *A = (double complex *)malloc(sizeof(double complex) * sa);
            double complex *B = (double complex *)malloc(sizeof(double complex) * sb);
            double complex *acc = part + (size_t)t * (nbits ? nbits : 1);
            for (int64_t p = lo; p < hi; ++p) {
                evolve_path(&c, paths[p], A, B);
                for (int64_t j = 0; j < nbits; ++j) acc[j] += A[xa[j]] * B[xb[j]];
                if (normsA_out) { double s = 0; for (int64_t i = 0; i < sa; ++i) s += creal(A[i] * conj(A[i])); normsA_out[p] = s; }
                if (normsB_out) { double s = 0; for (int64_t i = 0; i < sb; ++i) s += creal(B[i] * conj(B[i])); normsB_out[p] = s; }
            }
            free(A); free(B);
        }
        for (int t = 0; t < nt; ++t)
            for (int64_t j = 0; j < nbits; ++j) amps[j] += part[(size_t)t * nbits + j];
        free(part);
    }
    free(xa); free(xb); free(c.bit_of_gate);
    return 0;
}

/* Number of path bits k for a cut (one per crossing CZ, two per crossing iSWAP), or -1. */
int or_num_cut(int n, const or_gate *gates, size_t ng, uint64_t mask_a)
{
    const int nc = or_cut_gates(n, gates, ng, mask_a, NULL, 0);
    if (nc <= 0) return nc;
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * nc);
    or_cut_gates(n, gates, ng, mask_a, idx, nc);
    int k = 0;
    for (int j = 0; j < nc; ++j) k += branch_bits(gates[idx[j]].kind);
    free(idx);
    return k;
}

/* ------------------------------------------------------------------ */
/* Path selection: ceil(f 2^k) distinct ids, Floyd's algorithm          */
/* (Bentley and Floyd, "A sample of brilliance", CACM 1987) driven by   */
/* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014); a bounded draw in   */
/* [0, m) is floor(r * m / 2^64) for a 64-bit output r.                */
/* ------------------------------------------------------------------ */
static uint64_t splitmix_next(uint64_t *state)
{
    *state += 0x9E3779B97F4A7C15ULL;
    uint64_t z = *state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : (x > y);
}

/* Open-addressing set of uint64 (key + 1 stored, 0 = empty). */
typedef struct { uint64_t *slot; uint64_t cap; } u64set;

static int set_insert(u64set *s, uint64_t key)   /* 1 if inserted, 0 if present */
{
    uint64_t h = key * 0x9E3779B97F4A7C15ULL;
    uint64_t i = h & (s->cap - 1);
    for (;;) {
        if (s->slot[i] == 0) { s->slot[i] = key + 1; return 1; }
        if (s->slot[i] == key + 1) return 0;
        i = (i + 1) & (s->cap - 1);
    }
}

int64_t or_num_paths(int k, double f)
{
    if (k < 0 || k > 62 || !(f > 0.0) || f > 1.0) return -1;
    return (int64_t)ceil(ldexp(f, k));
}

int or_sample_paths(int k, double f, uint64_t seed, uint64_t *out, int64_t cap, int64_t *n_out)
{
    int64_t m = or_num_paths(k, f);
    if (m < 0 || m > cap) return -1;
    const uint64_t N = (uint64_t)1 << k;
    u64set s;
    s.cap = 1;
    while (s.cap < 2 * (uint64_t)m + 2) s.cap <<= 1;
    s.slot = (uint64_t *)calloc(s.cap, sizeof(uint64_t));
    uint64_t st = seed;
    int64_t filled = 0;
    for (uint64_t j = N - (uint64_t)m; j < N; ++j) {
        uint64_t r = splitmix_next(&st);
        uint64_t t = (uint64_t)(((unsigned __int128)r * (unsigned __int128)(j + 1)) >> 64);
        if (set_insert(&s, t)) out[filled++] = t;
        else { set_insert(&s, j); out[filled++] = j; }
    }
    free(s.slot);
    qsort(out, (size_t)m, sizeof(uint64_t), cmp_u64);
    *n_out = m;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Rejection sampling from a batch of output probabilities            */
/* (Section "Frugal rejection sampling" and its figure: Algorithm 1,   */
/* basic; Algorithm 2, frugal).                                        */
/*                                                                     */
/* Step 2 (candidates): count distinct uniform n-qubit bitstrings;     */
/* draw i is output i of SplitMix64(seed) masked to n bits, repeats    */
/* are skipped, the kept draws stay in draw order.                     */
/* Step 4 (acceptance) for candidate j with amplitude a_j:             */
/*   p_j = re^2 + im^2 (two products and a sum, each rounded),         */
/*   t_j = p_j * s with s = 2^n / M (N p_j / M),                       */
/*   u_j = (output j of SplitMix64(seed_u) >> 11) * 2^-53;             */
/*   Algorithm 2 accepts when u_j < t_j, i.e. with probability         */
/*   min{1, p_j N / M'}; Algorithm 1 first removes candidates with     */
/*   p_j > M / N (t_j > 1) and accepts the rest when u_j < t_j.        */
/* The batch's sampling error (the probability mass above M/N, which   */
/* the paper computes per batch when Porter-Thomas statistics are not  */
/* assumed) is estimated from the uniform candidates as                */
/*   (N / n) * sum_{j : t_j > 1} p_j.                                  */
/* ------------------------------------------------------------------ */
int or_sample_bitstrings(int n_qubits, uint64_t count, uint64_t seed, uint64_t *out)
{
    if (n_qubits < 1 || n_qubits > 64) return -1;
    if (n_qubits < 64 && count > ((uint64_t)1 << n_qubits)) return -1;
    const uint64_t mask = n_qubits == 64 ? ~(uint64_t)0 : (((uint64_t)1 << n_qubits) - 1);
    u64set s;
    s.cap = 1;
    while (s.cap < 2 * count + 2) s.cap <<= 1;
    s.slot = (uint64_t *)calloc(s.cap, sizeof(uint64_t));
    if (!s.slot) return -1;
    uint64_t st = seed, got = 0;
    while (got < count) {
        const uint64_t x = splitmix_next(&st) & mask;
        if (set_insert(&s, x)) out[got++] = x;
    }
    free(s.slot);
    return 0;
}

/* output j (0-based) of SplitMix64(seed) */
uint64_t or_splitmix64_at(uint64_t seed, uint64_t j)
{
    uint64_t st = seed + j * 0x9E3779B97F4A7C15ULL;
    return splitmix_next(&st);
}

int or_rejection_accept(const double *amps, int64_t n, int n_qubits, double m, uint64_t seed_u,
                        int basic, uint8_t *accept, double *err_est)
{
    if (n < 0 || n_qubits < 1 || n_qubits > 64 || !(m > 0.0)) return -1;
    const double s = ldexp(1.0, n_qubits) / m;
    double excess = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        const double re = amps[2 * j], im = amps[2 * j + 1];
        const double rr = re * re;
        const double ii = im * im;
        const double p = rr + ii;
        const double t = p * s;
        const double u = (double)(or_splitmix64_at(seed_u, (uint64_t)j) >> 11) * 0x1p-53;
        int acc;
        if (basic) acc = (t <= 1.0) && (u < t);
        else acc = u < t;
        accept[j] = (uint8_t)acc;
        if (t > 1.0) excess += p;
    }
    *err_est = n ? excess * ldexp(1.0, n_qubits) / (double)n : 0.0;
    return 0;
}
