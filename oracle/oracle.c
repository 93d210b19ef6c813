/*
 * CPU oracle for the state-vector simulator -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * use this file.  It shares no code with the GPU library: it has its own gate
 * matrices, its own index arithmetic and its own reductions.  Everything is
 * complex double precision and every gate is applied on its own, in the order
 * given, with no fusion, as the paper states the method (Section 3.2).
 *
 * Conventions (readings of the paper, stated once here):
 *  - qubit q is bit q of the amplitude index (Eq. 1q-op pairs s with s + 2^q);
 *  - a gate record on qubits (q[0], ..., q[k-1]) defines its matrix on the
 *    local index r = sum_j bit(q[j]) * 2^j; for controlled gates the controls
 *    come first and the target last;
 *  - rotations are R_P(theta) = exp(-i theta P / 2); no global-phase variants.
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* Gate record, 56 bytes: the input format written by the seeded generators. */
typedef struct {
    uint16_t kind;
    uint16_t nq;
    int32_t q[5];
    int32_t slot;
    uint32_t mat_off;
    double theta[3];
} orc_gate;

typedef struct {
    double coeff;
    uint64_t xmask;
    uint64_t zmask;
} orc_pauli;

enum {
    G_ID = 0, G_H = 1, G_X = 2, G_Y = 3, G_Z = 4, G_S = 5, G_SDG = 6, G_T = 7,
    G_TDG = 8, G_SX = 9, G_RX = 10, G_RY = 11, G_RZ = 12, G_U1 = 13,
    G_U2 = 14, G_U3 = 15,
    G_CX = 20, G_CY = 21, G_CZ = 22, G_CH = 23, G_SWAP = 24, G_CRX = 25,
    G_CRY = 26, G_CRZ = 27, G_CU1 = 28, G_CU3 = 29, G_RXX = 30, G_RZZ = 31,
    G_CCX = 40, G_CSWAP = 41, G_RCCX = 42, G_RC3X = 43, G_C3X = 44, G_C3XSQRTX = 45, G_C4X = 46,
    G_MAT = 50,
    G_BARRIER = 60, G_MEASURE = 61, G_RESET = 62, G_ASSERT0 = 63
};

enum { ORC_OK = 0, ORC_E_ARG = -1, ORC_E_QUBIT = -2, ORC_E_ZERO_PROB = -4,
       ORC_E_NOT_DEFINITE = -5 };

/* ------------------------------------------------------------ 1-qubit gates */
static void u3_matrix(double th, double ph, double la, cplx m[4]) {
    /* OpenQASM U3 (Table 3 of the paper): the general single-qubit rotation */
    m[0] = cos(th / 2);
    m[1] = -cexp(I * la) * sin(th / 2);
    m[2] = cexp(I * ph) * sin(th / 2);
    m[3] = cexp(I * (ph + la)) * cos(th / 2);
}

/* 2x2 matrix of a single-qubit kind, row-major.  Returns 0 if not 1-qubit. */
static int one_qubit_matrix(int kind, const double *t, cplx m[4]) {
    const double r = 1.0 / sqrt(2.0);
    m[0] = 1; m[1] = 0; m[2] = 0; m[3] = 1;
    switch (kind) {
    case G_ID: return 1;
    case G_H: m[0] = r; m[1] = r; m[2] = r; m[3] = -r; return 1;
    case G_X: m[0] = 0; m[1] = 1; m[2] = 1; m[3] = 0; return 1;
    case G_Y: m[0] = 0; m[1] = -I; m[2] = I; m[3] = 0; return 1;
    case G_Z: m[3] = -1; return 1;
    case G_S: m[3] = I; return 1;
    case G_SDG: m[3] = -I; return 1;
    case G_T: m[3] = cexp(I * M_PI / 4); return 1;
    case G_TDG: m[3] = cexp(-I * M_PI / 4); return 1;
    case G_SX:
        m[0] = 0.5 * (1 + I); m[1] = 0.5 * (1 - I);
        m[2] = 0.5 * (1 - I); m[3] = 0.5 * (1 + I); return 1;
    case G_RX:
        m[0] = cos(t[0] / 2); m[1] = -I * sin(t[0] / 2);
        m[2] = -I * sin(t[0] / 2); m[3] = cos(t[0] / 2); return 1;
    case G_RY:
        m[0] = cos(t[0] / 2); m[1] = -sin(t[0] / 2);
        m[2] = sin(t[0] / 2); m[3] = cos(t[0] / 2); return 1;
    case G_RZ: m[0] = cexp(-I * t[0] / 2); m[3] = cexp(I * t[0] / 2); return 1;
    case G_U1: m[3] = cexp(I * t[0]); return 1;
    case G_U2: u3_matrix(M_PI / 2, t[0], t[1], m); return 1;
    case G_U3: u3_matrix(t[0], t[1], t[2], m); return 1;
    default: return 0;
    }
}

/* The relative-phase Toffolis of OpenQASM's standard library are defined
 * there as gate sequences on the target (the last local bit) and the
 * controls; each step below is (kind, qubit) for a single-qubit gate, or
 * (G_CX, control) for a CNOT onto the target.  u2(0, pi) is H and u1(+-pi/4)
 * is T / T^dagger. */
typedef struct { int kind, q; } seq_step;
static const seq_step RCCX_SEQ[] = {
    {G_H, 2}, {G_T, 2}, {G_CX, 1}, {G_TDG, 2}, {G_CX, 0}, {G_T, 2}, {G_CX, 1}, {G_TDG, 2}, {G_H, 2}};
static const seq_step RC3X_SEQ[] = {
    {G_H, 3}, {G_T, 3}, {G_CX, 2}, {G_TDG, 3}, {G_H, 3}, {G_CX, 0}, {G_T, 3}, {G_CX, 1}, {G_TDG, 3},
    {G_CX, 0}, {G_T, 3}, {G_CX, 1}, {G_TDG, 3}, {G_H, 3}, {G_T, 3}, {G_CX, 2}, {G_TDG, 3}, {G_H, 3}};

/* m = S_last ... S_1 for the steps of a sequence on k local bits (target =
 * local bit k-1): every column of the identity is pushed through the steps. */
static void sequence_matrix(const seq_step *seq, int ns, int k, cplx *m) {
    const int dim = 1 << k, tgt = k - 1;
    cplx col[32], nxt[32];
    for (int c = 0; c < dim; c++) {
        for (int r = 0; r < dim; r++) col[r] = (r == c) ? 1 : 0;
        for (int s = 0; s < ns; s++) {
            for (int r = 0; r < dim; r++) nxt[r] = 0;
            if (seq[s].kind == G_CX) {
                for (int r = 0; r < dim; r++)
                    nxt[((r >> seq[s].q) & 1) ? (r ^ (1 << tgt)) : r] += col[r];
            } else {
                cplx u[4];
                one_qubit_matrix(seq[s].kind, NULL, u);
                const int b = seq[s].q;
                for (int r = 0; r < dim; r++) {
                    const int bit = (r >> b) & 1;
                    nxt[r & ~(1 << b)] += u[0 * 2 + bit] * col[r];   /* row 0 of u, column bit */
                    nxt[r | (1 << b)] += u[1 * 2 + bit] * col[r];    /* row 1 of u */
                }
            }
            for (int r = 0; r < dim; r++) col[r] = nxt[r];
        }
        for (int r = 0; r < dim; r++) m[r * dim + c] = col[r];
    }
}

/* Dense 2^k x 2^k matrix (row-major) of a k-qubit kind in the record's qubit
 * order.  `m` must hold 32*32 entries.  Returns k, or 0 for unknown kinds. */
static int gate_matrix(const orc_gate *g, const double *theta, cplx *m) {
    int k = g->nq;
    int dim = 1 << k;
    for (int i = 0; i < dim * dim; i++) m[i] = 0;
    cplx u[4];
    if (k == 1) return one_qubit_matrix(g->kind, theta, m) ? 1 : 0;
    /* controlled single-qubit gates: control = q[0] (local bit 0),
     * target = q[1] (local bit 1) */
    int ctrl_kind = -1;
    switch (g->kind) {
    case G_CX: ctrl_kind = G_X; break;
    case G_CY: ctrl_kind = G_Y; break;
    case G_CZ: ctrl_kind = G_Z; break;
    case G_CH: ctrl_kind = G_H; break;
    case G_CRX: ctrl_kind = G_RX; break;
    case G_CRY: ctrl_kind = G_RY; break;
    case G_CRZ: ctrl_kind = G_RZ; break;
    case G_CU1: ctrl_kind = G_U1; break;
    case G_CU3: ctrl_kind = G_U3; break;
    default: break;
    }
    if (k == 2 && ctrl_kind >= 0) {
        one_qubit_matrix(ctrl_kind, theta, u);
        for (int r = 0; r < 4; r++) {
            for (int c = 0; c < 4; c++) {
                int rc = r & 1, rt = r >> 1, cc = c & 1, ct = c >> 1;
                if (rc != cc) continue;
                if (rc == 0) m[r * 4 + c] = (rt == ct) ? 1 : 0;
                else m[r * 4 + c] = u[rt * 2 + ct];
            }
        }
        return 2;
    }
    if (k == 2 && g->kind == G_SWAP) {
        m[0 * 4 + 0] = 1; m[1 * 4 + 2] = 1; m[2 * 4 + 1] = 1; m[3 * 4 + 3] = 1;
        return 2;
    }
    if (k == 2 && (g->kind == G_RXX || g->kind == G_RZZ)) {
        /* exp(-i theta P/2) = cos(theta/2) I - i sin(theta/2) P, P = XX or ZZ */
        double c = cos(theta[0] / 2), s = sin(theta[0] / 2);
        for (int r = 0; r < 4; r++) {
            m[r * 4 + r] += c;
            if (g->kind == G_RXX) m[r * 4 + (r ^ 3)] += -I * s;
            else {
                int par = ((r & 1) ^ (r >> 1)) ? -1 : 1;
                m[r * 4 + r] += -I * s * par;
            }
        }
        return 2;
    }
    /* multi-controlled gates: all local bits but the last are controls */
    int base = -1;
    switch (g->kind) {
    case G_CCX: if (k == 3) base = G_X; break;
    case G_C3X: if (k == 4) base = G_X; break;
    case G_C4X: if (k == 5) base = G_X; break;
    case G_C3XSQRTX: if (k == 4) base = G_SX; break;
    default: break;
    }
    if (base >= 0) {
        one_qubit_matrix(base, theta, u);
        int cmask = (1 << (k - 1)) - 1;
        for (int r = 0; r < dim; r++) {
            for (int c = 0; c < dim; c++) {
                if ((r & cmask) != (c & cmask)) continue;
                int rt = r >> (k - 1), ct = c >> (k - 1);
                if ((r & cmask) == cmask) m[r * dim + c] = u[rt * 2 + ct];
                else m[r * dim + c] = (rt == ct) ? 1 : 0;
            }
        }
        return k;
    }
    if (k == 3 && g->kind == G_RCCX) {
        sequence_matrix(RCCX_SEQ, (int)(sizeof(RCCX_SEQ) / sizeof(RCCX_SEQ[0])), 3, m);
        return 3;
    }
    if (k == 4 && g->kind == G_RC3X) {
        sequence_matrix(RC3X_SEQ, (int)(sizeof(RC3X_SEQ) / sizeof(RC3X_SEQ[0])), 4, m);
        return 4;
    }
    if (k == 3 && g->kind == G_CSWAP) {
        /* control = local bit 0; swap local bits 1 and 2 when it is set */
        for (int c = 0; c < 8; c++) {
            int r = c;
            if (c & 1) r = (c & 1) | ((c >> 1) & 1) << 2 | ((c >> 2) & 1) << 1;
            m[r * 8 + c] = 1;
        }
        return 3;
    }
    return 0;
}

/* ---------------------------------------------------- the update equations */

/* Eq. (1q-op): for every i in [0, 2^(n-1)), s_i = floor(i/2^q) 2^(q+1)
 * + (i mod 2^q), and (a[s_i], a[s_i + 2^q]) <- U (a[s_i], a[s_i + 2^q]). */
static void apply_1q(int n, cplx *a, int q, const cplx u[4]) {
    const int64_t half = (int64_t)1 << (n - 1);
    const int64_t bq = (int64_t)1 << q;
#pragma omp parallel for if (n >= 16) schedule(static)
    for (int64_t i = 0; i < half; i++) {
        int64_t s = (i / bq) * (bq << 1) + (i % bq);
        cplx x0 = a[s], x1 = a[s + bq];
        a[s] = u[0] * x0 + u[1] * x1;
        a[s + bq] = u[2] * x0 + u[3] * x1;
    }
}

/* Eq. (2q-op), p < q: s_i = floor(floor(i/2^p)/2^(q-p-1)) 2^(q+1)
 * + (floor(i/2^p) mod 2^(q-p-1)) 2^(p+1) + (i mod 2^p), and the four
 * amplitudes (s, s+2^p, s+2^q, s+2^p+2^q) are multiplied by U (4x4). */
static void apply_2q(int n, cplx *a, int p, int q, const cplx *u) {
    const int64_t quarter = (int64_t)1 << (n - 2);
    const int64_t bp = (int64_t)1 << p, bq = (int64_t)1 << q;
    const int64_t span = (int64_t)1 << (q - p - 1);
#pragma omp parallel for if (n >= 16) schedule(static)
    for (int64_t i = 0; i < quarter; i++) {
        int64_t ip = i / bp;
        int64_t s = (ip / span) * (bq << 1) + (ip % span) * (bp << 1) + (i % bp);
        cplx x[4] = {a[s], a[s + bp], a[s + bq], a[s + bp + bq]};
        for (int r = 0; r < 4; r++) {
            cplx acc = 0;
            for (int c = 0; c < 4; c++) acc += u[r * 4 + c] * x[c];
            a[s + (r & 1 ? bp : 0) + (r & 2 ? bq : 0)] = acc;
        }
    }
}

/* The same update for k >= 3 qubits (the paper states only k <= 2): the
 * group base is i with zero bits inserted at the sorted qubit positions, and
 * the 2^k amplitudes are gathered in the record's qubit order. */
static void apply_kq(int n, cplx *a, const int *qs, int k, const cplx *u) {
    int sorted[5];
    for (int j = 0; j < k; j++) sorted[j] = qs[j];
    for (int i = 0; i < k; i++)
        for (int j = i + 1; j < k; j++)
            if (sorted[j] < sorted[i]) { int t = sorted[i]; sorted[i] = sorted[j]; sorted[j] = t; }
    const int dim = 1 << k;
    const int64_t groups = (int64_t)1 << (n - k);
#pragma omp parallel for if (n >= 16) schedule(static)
    for (int64_t i = 0; i < groups; i++) {
        int64_t s = i;
        for (int j = 0; j < k; j++) {
            int64_t low = s & (((int64_t)1 << sorted[j]) - 1);
            s = ((s >> sorted[j]) << (sorted[j] + 1)) | low;
        }
        cplx x[32], y[32];
        for (int c = 0; c < dim; c++) {
            int64_t idx = s;
            for (int j = 0; j < k; j++) if (c >> j & 1) idx += (int64_t)1 << qs[j];
            x[c] = a[idx];
        }
        for (int r = 0; r < dim; r++) {
            cplx acc = 0;
            for (int c = 0; c < dim; c++) acc += u[r * dim + c] * x[c];
            y[r] = acc;
        }
        for (int r = 0; r < dim; r++) {
            int64_t idx = s;
            for (int j = 0; j < k; j++) if (r >> j & 1) idx += (int64_t)1 << qs[j];
            a[idx] = y[r];
        }
    }
}

/* Apply one matrix on the record's qubits.  For two qubits with q[0] > q[1]
 * the matrix is conjugated by SWAP so that Eq. (2q-op) sees p < q, as the
 * paper does before fusing (U(b,a) -> SWAP U(a,b) SWAP, Section 4.2). */
static void apply_matrix(int n, cplx *a, const int *qs, int k, const cplx *u) {
    if (k == 1) {
        apply_1q(n, a, qs[0], u);
    } else if (k == 2) {
        if (qs[0] < qs[1]) {
            apply_2q(n, a, qs[0], qs[1], u);
        } else {
            static const int sw[4] = {0, 2, 1, 3};
            cplx v[16];
            for (int r = 0; r < 4; r++)
                for (int c = 0; c < 4; c++) v[sw[r] * 4 + sw[c]] = u[r * 4 + c];
            apply_2q(n, a, qs[1], qs[0], v);
        }
    } else {
        apply_kq(n, a, qs, k, u);
    }
}

/* ----------------------------------------------------- measurement helpers */
static void half_weights(int n, const cplx *a, int q, double *p0, double *p1) {
    double s0 = 0, s1 = 0;
    const int64_t dim = (int64_t)1 << n;
    for (int64_t x = 0; x < dim; x++) {
        double w = creal(a[x]) * creal(a[x]) + cimag(a[x]) * cimag(a[x]);
        if ((x >> q) & 1) s1 += w; else s0 += w;
    }
    *p0 = s0;
    *p1 = s1;
}

/* Keep the half where bit q equals `keep`, zero the other, and scale by
 * 1/sqrt(weight of the kept half) so the result has unit norm. */
static void collapse(int n, cplx *a, int q, int keep, double kept_weight) {
    const double scale = 1.0 / sqrt(kept_weight);
    const int64_t dim = (int64_t)1 << n;
    for (int64_t x = 0; x < dim; x++) {
        if ((int)((x >> q) & 1) == keep) a[x] *= scale;
        else a[x] = 0;
    }
}

/* ================================================================ public API */

int orc_gate_matrix(const orc_gate *g, const double *theta_override,
                    double *out_interleaved) {
    cplx m[1024];
    const double *t = theta_override ? theta_override : g->theta;
    int k = gate_matrix(g, t, m);
    if (!k) return ORC_E_ARG;
    int dim = 1 << k;
    for (int i = 0; i < dim * dim; i++) {
        out_interleaved[2 * i] = creal(m[i]);
        out_interleaved[2 * i + 1] = cimag(m[i]);
    }
    return k;
}

/* Born-rule measurement of qubit q with the uniform draw u in [0,1):
 * p0 = P0/(P0+P1); outcome 0 iff u < p0; the state is projected and
 * renormalised.  Writes the outcome and its probability. */
int orc_measure(int n, double *psi, int q, double u, int *outcome, double *prob) {
    if (q < 0 || q >= n) return ORC_E_QUBIT;
    if (!(u >= 0.0 && u < 1.0)) return ORC_E_ARG;
    cplx *a = (cplx *)psi;
    double P0, P1;
    half_weights(n, a, q, &P0, &P1);
    double p0 = P0 / (P0 + P1);
    int o = (u < p0) ? 0 : 1;
    collapse(n, a, q, o, o ? P1 : P0);
    *outcome = o;
    *prob = o ? P1 / (P0 + P1) : p0;
    return ORC_OK;
}

/* Measurement assertion (Section 4.3): if P(q = 0) > 0 the outcome is taken
 * to be 0, the state is projected and renormalised and P(q = 0) is returned;
 * otherwise the state is untouched and the call fails. */
int orc_assert0(int n, double *psi, int q, double *prob) {
    if (q < 0 || q >= n) return ORC_E_QUBIT;
    cplx *a = (cplx *)psi;
    double P0, P1;
    half_weights(n, a, q, &P0, &P1);
    if (!(P0 > 0.0)) return ORC_E_ZERO_PROB;
    collapse(n, a, q, 0, P0);
    *prob = P0 / (P0 + P1);
    return ORC_OK;
}

/* Reset of a definite qubit: identity if it is |0>, X if it is |1>. */
int orc_reset(int n, double *psi, int q) {
    if (q < 0 || q >= n) return ORC_E_QUBIT;
    cplx *a = (cplx *)psi;
    double P0, P1;
    half_weights(n, a, q, &P0, &P1);
    if (P1 == 0.0) return ORC_OK;
    if (P0 != 0.0) return ORC_E_NOT_DEFINITE;
    static const cplx x[4] = {0, 1, 1, 0};
    apply_1q(n, a, q, x);
    return ORC_OK;
}

/* Apply a gate list, one record at a time.  MEASURE / ASSERT0 / RESET records
 * are executed in place: a MEASURE record with slot s draws uniforms[s] unless
 * forced[s] >= 0 names the outcome; outcomes[s] and probs[s] receive the
 * result.  Returns 0, or a negative error code and the index of the failing
 * record in *fail_at. */
int orc_run(int n, double *psi, const orc_gate *g, int64_t ng,
            const double *mats, const double *params, const double *uniforms,
            const int *forced, int *outcomes, double *probs, int64_t *fail_at) {
    cplx *a = (cplx *)psi;
    cplx m[1024];
    for (int64_t i = 0; i < ng; i++) {
        const orc_gate *gi = &g[i];
        int k = gi->nq;
        if (fail_at) *fail_at = i;
        if (gi->kind == G_BARRIER) continue;
        if (k < 1 || k > 5) return ORC_E_ARG;
        for (int j = 0; j < k; j++) {
            if (gi->q[j] < 0 || gi->q[j] >= n) return ORC_E_QUBIT;
            for (int l = 0; l < j; l++) if (gi->q[l] == gi->q[j]) return ORC_E_QUBIT;
        }
        if (gi->kind == G_MEASURE || gi->kind == G_ASSERT0) {
            int s = gi->slot, o, rc;
            double p;
            if (gi->kind == G_ASSERT0) {
                rc = orc_assert0(n, psi, gi->q[0], &p);
                o = 0;
            } else if (forced && forced[s] >= 0) {
                double P0, P1;
                half_weights(n, a, gi->q[0], &P0, &P1);
                o = forced[s];
                if ((o ? P1 : P0) <= 0.0) return ORC_E_ZERO_PROB;
                collapse(n, a, gi->q[0], o, o ? P1 : P0);
                p = (o ? P1 : P0) / (P0 + P1);
                rc = ORC_OK;
            } else {
                if (!uniforms) return ORC_E_ARG;
                rc = orc_measure(n, psi, gi->q[0], uniforms[s], &o, &p);
            }
            if (rc) return rc;
            if (outcomes) outcomes[s] = o;
            if (probs) probs[s] = p;
            continue;
        }
        if (gi->kind == G_RESET) {
            int rc = orc_reset(n, psi, gi->q[0]);
            if (rc) return rc;
            continue;
        }
        double th[3] = {gi->theta[0], gi->theta[1], gi->theta[2]};
        if (gi->slot >= 0 && params) th[0] = params[gi->slot];
        if (gi->kind == G_MAT) {
            int dim = 1 << k;
            const double *src = mats + 2 * (size_t)gi->mat_off;
            for (int e = 0; e < dim * dim; e++) m[e] = src[2 * e] + I * src[2 * e + 1];
        } else if (gate_matrix(gi, th, m) != k) {
            return ORC_E_ARG;
        }
        apply_matrix(n, a, gi->q, k, m);
    }
    if (fail_at) *fail_at = -1;
    return ORC_OK;
}

double orc_norm(int n, const double *psi) {
    const cplx *a = (const cplx *)psi;
    double s = 0;
    const int64_t dim = (int64_t)1 << n;
    for (int64_t x = 0; x < dim; x++)
        s += creal(a[x]) * creal(a[x]) + cimag(a[x]) * cimag(a[x]);
    return s;
}

/* Marginal probabilities of the qubits qs[0..nqs-1]: out[j] with
 * j = sum_i bit(qs[i]) 2^i, divided by the total weight. */
int orc_probs(int n, const double *psi, const int *qs, int nqs, double *out) {
    const cplx *a = (const cplx *)psi;
    for (int j = 0; j < (1 << nqs); j++) out[j] = 0;
    double tot = 0;
    const int64_t dim = (int64_t)1 << n;
    for (int64_t x = 0; x < dim; x++) {
        int j = 0;
        for (int i = 0; i < nqs; i++) j |= (int)((x >> qs[i]) & 1) << i;
        double w = creal(a[x]) * creal(a[x]) + cimag(a[x]) * cimag(a[x]);
        out[j] += w;
        tot += w;
    }
    for (int j = 0; j < (1 << nqs); j++) out[j] /= tot;
    return ORC_OK;
}

/* <psi|H|psi> / <psi|psi> for H = sum_k c_k P_k, with
 * P|x> = i^{#Y} (-1)^{popcount(x & zmask)} |x ^ xmask>. */
double orc_expval(int n, const double *psi, const orc_pauli *t, int64_t nt) {
    const cplx *a = (const cplx *)psi;
    const int64_t dim = (int64_t)1 << n;
    double total = 0;
    for (int64_t k = 0; k < nt; k++) {
        uint64_t xm = t[k].xmask, zm = t[k].zmask;
        int ny = __builtin_popcountll(xm & zm);
        cplx iy = 1;
        for (int j = 0; j < ny % 4; j++) iy *= I;
        cplx acc = 0;
        for (int64_t x = 0; x < dim; x++) {
            double sign = (__builtin_popcountll((uint64_t)x & zm) & 1) ? -1.0 : 1.0;
            acc += conj(a[x ^ (int64_t)xm]) * iy * sign * a[x];
        }
        total += t[k].coeff * creal(acc);
    }
    return total / orc_norm(n, psi);
}

/* Threads used by the amplitude loops (timing runs only: every loop sums in
 * a fixed order per amplitude, so the results do not depend on it).  Returns
 * the number now in effect. */
int orc_set_threads(int k) {
    if (k > 0) omp_set_num_threads(k);
    return omp_get_max_threads();
}
