// Gate lowering: gate records -> FP64 operators on ascending qubits.
//
// The gate set is the OpenQASM 2.0 table of the paper (Section 4.1, Table 3)
// plus a general matrix record.  Rotations follow R_P(theta) =
// exp(-i theta P / 2) = cos(theta/2) I - i sin(theta/2) P.  A record's matrix
// is defined on its own qubit order (local bit j <-> q[j]); lowering permutes
// it to ascending qubit order, which is the paper's normalisation of every
// two-qubit gate to first index < second index, U(b,a) -> SWAP U(a,b) SWAP
// (Section 4.2), done as a relabelling of matrix indices and never as a
// state sweep.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <new>
#include <thread>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "host.h"

namespace qs {

double now_seconds() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

TraceRange::TraceRange(const char *name) { roctxRangePushA(name); }
TraceRange::~TraceRange() { roctxRangePop(); }

namespace {

const cd kI(0.0, 1.0);

// Pauli letters as 2x2 row-major matrices.
void pauli2(char p, cd out[4]) {
    switch (p) {
    case 'X': out[0] = 0; out[1] = 1; out[2] = 1; out[3] = 0; break;
    case 'Y': out[0] = 0; out[1] = -kI; out[2] = kI; out[3] = 0; break;
    case 'Z': out[0] = 1; out[1] = 0; out[2] = 0; out[3] = -1; break;
    default: out[0] = 1; out[1] = 0; out[2] = 0; out[3] = 1; break;
    }
}

// Pauli string on `k` local qubits, letters[j] on local bit j.
void pauli_string(const char *letters, int k, std::vector<cd> *out) {
    int d = 1 << k;
    out->assign(size_t(d) * d, cd(0));
    for (int c = 0; c < d; c++) {
        // P|c> = prod_j sigma_j |c_j>: each letter maps a bit to one bit with a phase
        int r = 0;
        cd ph = 1;
        for (int j = 0; j < k; j++) {
            cd s[4];
            pauli2(letters[j], s);
            int b = (c >> j) & 1;
            int nb = (s[(0) * 2 + b] != cd(0)) ? 0 : 1;
            ph *= s[nb * 2 + b];
            r |= nb << j;
        }
        (*out)[size_t(r) * d + c] = ph;
    }
}

// exp(-i theta P / 2) for a Pauli string P.
void pauli_rotation(const char *letters, int k, double theta, std::vector<cd> *out) {
    std::vector<cd> p;
    pauli_string(letters, k, &p);
    int d = 1 << k;
    out->assign(size_t(d) * d, cd(0));
    double c = std::cos(theta / 2), s = std::sin(theta / 2);
    for (int i = 0; i < d * d; i++) (*out)[i] = -kI * s * p[i];
    for (int i = 0; i < d; i++) (*out)[size_t(i) * d + i] += c;
}

void one_qubit(int kind, const double *t, cd u[4]) {
    const double h = std::sqrt(0.5);
    std::vector<cd> tmp;
    auto from = [&](const std::vector<cd> &v) { for (int i = 0; i < 4; i++) u[i] = v[i]; };
    u[0] = 1; u[1] = 0; u[2] = 0; u[3] = 1;
    switch (kind) {
    case QSIM_G_ID: break;
    case QSIM_G_H: u[0] = h; u[1] = h; u[2] = h; u[3] = -h; break;
    case QSIM_G_X: pauli2('X', u); break;
    case QSIM_G_Y: pauli2('Y', u); break;
    case QSIM_G_Z: pauli2('Z', u); break;
    case QSIM_G_S: u[3] = kI; break;
    case QSIM_G_SDG: u[3] = -kI; break;
    case QSIM_G_T: u[3] = std::polar(1.0, M_PI / 4); break;
    case QSIM_G_TDG: u[3] = std::polar(1.0, -M_PI / 4); break;
    case QSIM_G_SX: u[0] = u[3] = cd(0.5, 0.5); u[1] = u[2] = cd(0.5, -0.5); break;
    case QSIM_G_RX: pauli_rotation("X", 1, t[0], &tmp); from(tmp); break;
    case QSIM_G_RY: pauli_rotation("Y", 1, t[0], &tmp); from(tmp); break;
    case QSIM_G_RZ: pauli_rotation("Z", 1, t[0], &tmp); from(tmp); break;
    case QSIM_G_U1: u[3] = std::polar(1.0, t[0]); break;
    case QSIM_G_U2:
    case QSIM_G_U3: {
        double th = kind == QSIM_G_U2 ? M_PI / 2 : t[0];
        double ph = kind == QSIM_G_U2 ? t[0] : t[1];
        double la = kind == QSIM_G_U2 ? t[1] : t[2];
        u[0] = std::cos(th / 2);
        u[1] = -std::polar(1.0, la) * std::sin(th / 2);
        u[2] = std::polar(1.0, ph) * std::sin(th / 2);
        u[3] = std::polar(1.0, ph + la) * std::cos(th / 2);
        break;
    }
    default: break;
    }
}

bool is_one_qubit(int kind) { return kind >= QSIM_G_ID && kind <= QSIM_G_U3; }

// |0><0| (x) I + |1><1| (x) U with `nc` control bits (local bits 0..nc-1, all
// required set) and the target on local bit nc.
void controlled(const cd u[4], int nc, std::vector<cd> *out) {
    int k = nc + 1, d = 1 << k, all = (1 << nc) - 1;
    out->assign(size_t(d) * d, cd(0));
    for (int c = 0; c < d; c++) {
        if ((c & all) != all) { (*out)[size_t(c) * d + c] = 1; continue; }
        int tb = c >> nc;
        for (int rt = 0; rt < 2; rt++) {
            int r = (c & all) | (rt << nc);
            (*out)[size_t(r) * d + c] = u[rt * 2 + tb];
        }
    }
}

int kind_arity(int kind) {
    if (is_one_qubit(kind)) return 1;
    switch (kind) {
    case QSIM_G_CX: case QSIM_G_CY: case QSIM_G_CZ: case QSIM_G_CH: case QSIM_G_SWAP:
    case QSIM_G_CRX: case QSIM_G_CRY: case QSIM_G_CRZ: case QSIM_G_CU1: case QSIM_G_CU3:
    case QSIM_G_RXX: case QSIM_G_RZZ: return 2;
    case QSIM_G_CCX: case QSIM_G_CSWAP: case QSIM_G_RCCX: return 3;
    case QSIM_G_C3X: case QSIM_G_C3XSQRTX: case QSIM_G_RC3X: return 4;
    case QSIM_G_C4X: return 5;
    default: return 0;
    }
}

// Rotation kinds whose matrix is cos(theta/2) A + sin(theta/2) B.  (Controlled
// rotations are affine, not linear, in these: their control-off block is
// constant.)
bool is_half_angle_linear(int kind) {
    switch (kind) {
    case QSIM_G_RX: case QSIM_G_RY: case QSIM_G_RZ: case QSIM_G_RXX: case QSIM_G_RZZ: return true;
    default: return false;
    }
}

// A gate given as a circuit on its k local bits (the relative-phase Toffolis
// of OpenQASM's standard library): the product of the steps, last step
// leftmost, built by multiplying each step's k-bit operator onto the
// accumulated matrix.  A step is a single-qubit kind on local bit `a`, or a
// CNOT from local bit `a` to local bit `b` (kind QSIM_G_CX).
struct Step {
    int kind, a, b;
};

void circuit_matrix(const Step *steps, int ns, int k, std::vector<cd> *m) {
    const int d = 1 << k;
    m->assign(size_t(d) * d, cd(0));
    for (int i = 0; i < d; i++) (*m)[size_t(i) * d + i] = 1;
    std::vector<cd> g(size_t(d) * d), acc(size_t(d) * d);
    for (int s = 0; s < ns; s++) {
        std::fill(g.begin(), g.end(), cd(0));
        if (steps[s].kind == QSIM_G_CX) {
            for (int c = 0; c < d; c++) {
                const int r = ((c >> steps[s].a) & 1) ? (c ^ (1 << steps[s].b)) : c;
                g[size_t(r) * d + c] = 1;
            }
        } else {
            cd u[4];
            one_qubit(steps[s].kind, nullptr, u);
            const int a = steps[s].a;
            for (int c = 0; c < d; c++)
                for (int rb = 0; rb < 2; rb++) {
                    const int r = (c & ~(1 << a)) | (rb << a);
                    g[size_t(r) * d + c] = u[rb * 2 + ((c >> a) & 1)];
                }
        }
        for (int r = 0; r < d; r++)
            for (int c = 0; c < d; c++) {
                cd v = 0;
                for (int x = 0; x < d; x++) v += g[size_t(r) * d + x] * (*m)[size_t(x) * d + c];
                acc[size_t(r) * d + c] = v;
            }
        m->swap(acc);
    }
}

// OpenQASM's rccx a, b, c and rc3x a, b, c, d (controls first, target last)
const Step kRccx[] = {{QSIM_G_H, 2, 0},   {QSIM_G_T, 2, 0},  {QSIM_G_CX, 1, 2}, {QSIM_G_TDG, 2, 0},
                      {QSIM_G_CX, 0, 2},  {QSIM_G_T, 2, 0},  {QSIM_G_CX, 1, 2}, {QSIM_G_TDG, 2, 0},
                      {QSIM_G_H, 2, 0}};
const Step kRc3x[] = {{QSIM_G_H, 3, 0},   {QSIM_G_T, 3, 0},   {QSIM_G_CX, 2, 3}, {QSIM_G_TDG, 3, 0},
                      {QSIM_G_H, 3, 0},   {QSIM_G_CX, 0, 3},  {QSIM_G_T, 3, 0},  {QSIM_G_CX, 1, 3},
                      {QSIM_G_TDG, 3, 0}, {QSIM_G_CX, 0, 3},  {QSIM_G_T, 3, 0},  {QSIM_G_CX, 1, 3},
                      {QSIM_G_TDG, 3, 0}, {QSIM_G_H, 3, 0},   {QSIM_G_T, 3, 0},  {QSIM_G_CX, 2, 3},
                      {QSIM_G_TDG, 3, 0}, {QSIM_G_H, 3, 0}};

}  // namespace

int gate_matrix(const qsim_gate &g, const double *t, std::vector<cd> *m) {
    int kind = g.kind;
    cd u[4];
    if (is_one_qubit(kind)) {
        one_qubit(kind, t, u);
        m->assign(u, u + 4);
        return QSIM_OK;
    }
    switch (kind) {
    case QSIM_G_CX: one_qubit(QSIM_G_X, t, u); controlled(u, 1, m); return QSIM_OK;
    case QSIM_G_CY: one_qubit(QSIM_G_Y, t, u); controlled(u, 1, m); return QSIM_OK;
    case QSIM_G_CZ: one_qubit(QSIM_G_Z, t, u); controlled(u, 1, m); return QSIM_OK;
    case QSIM_G_CH: one_qubit(QSIM_G_H, t, u); controlled(u, 1, m); return QSIM_OK;
    case QSIM_G_CRX: one_qubit(QSIM_G_RX, t, u); controlled(u, 1, m); return QSIM_OK;
    case QSIM_G_CRY: one_qubit(QSIM_G_RY, t, u); controlled(u, 1, m); return QSIM_OK;
    case QSIM_G_CRZ: one_qubit(QSIM_G_RZ, t, u); controlled(u, 1, m); return QSIM_OK;
    case QSIM_G_CU1: one_qubit(QSIM_G_U1, t, u); controlled(u, 1, m); return QSIM_OK;
    case QSIM_G_CU3: one_qubit(QSIM_G_U3, t, u); controlled(u, 1, m); return QSIM_OK;
    case QSIM_G_CCX: one_qubit(QSIM_G_X, t, u); controlled(u, 2, m); return QSIM_OK;
    case QSIM_G_C3X: one_qubit(QSIM_G_X, t, u); controlled(u, 3, m); return QSIM_OK;
    case QSIM_G_C4X: one_qubit(QSIM_G_X, t, u); controlled(u, 4, m); return QSIM_OK;
    case QSIM_G_C3XSQRTX: one_qubit(QSIM_G_SX, t, u); controlled(u, 3, m); return QSIM_OK;
    case QSIM_G_RCCX: circuit_matrix(kRccx, int(sizeof(kRccx) / sizeof(kRccx[0])), 3, m); return QSIM_OK;
    case QSIM_G_RC3X: circuit_matrix(kRc3x, int(sizeof(kRc3x) / sizeof(kRc3x[0])), 4, m); return QSIM_OK;
    case QSIM_G_RXX: pauli_rotation("XX", 2, t[0], m); return QSIM_OK;
    case QSIM_G_RZZ: pauli_rotation("ZZ", 2, t[0], m); return QSIM_OK;
    case QSIM_G_SWAP:
        m->assign(16, cd(0));
        for (int c = 0; c < 4; c++) (*m)[size_t(((c & 1) << 1) | (c >> 1)) * 4 + c] = 1;
        return QSIM_OK;
    case QSIM_G_CSWAP:
        m->assign(64, cd(0));
        for (int c = 0; c < 8; c++) {
            int r = c;
            if (c & 1) r = 1 | ((c & 2) << 1) | ((c & 4) >> 1);
            (*m)[size_t(r) * 8 + c] = 1;
        }
        return QSIM_OK;
    default: return QSIM_E_UNSUPPORTED;
    }
}

namespace {

// Relabel a matrix given on record order qs[0..k-1] to ascending qubit order.
void to_sorted(const int *qs, int k, const cd *src, int nblocks, Op *op) {
    int order[kMaxK];
    for (int j = 0; j < k; j++) order[j] = j;
    std::sort(order, order + k, [&](int a, int b) { return qs[a] < qs[b]; });
    int rank[kMaxK];
    for (int j = 0; j < k; j++) rank[order[j]] = j;
    op->k = k;
    for (int j = 0; j < k; j++) op->q[j] = qs[order[j]];
    int d = 1 << k;
    std::vector<int> map(d);
    for (int r = 0; r < d; r++) {
        int s = 0;
        for (int j = 0; j < k; j++) s |= ((r >> j) & 1) << rank[j];
        map[r] = s;
    }
    op->m.assign(size_t(nblocks) * d * d, cd(0));
    for (int b = 0; b < nblocks; b++)
        for (int r = 0; r < d; r++)
            for (int c = 0; c < d; c++)
                op->m[size_t(b) * d * d + size_t(map[r]) * d + map[c]] =
                    src[size_t(b) * d * d + size_t(r) * d + c];
}

}  // namespace

namespace {

// One gate record (not a barrier or a measurement record) -> its operator.
// Returns QSIM_OK or the record's error.
int lower_gate(int n, const qsim_gate &gi, const GateInputs &in, bool keep_params, Op *out,
               std::vector<cd> &m, std::vector<cd> &m2) {
    int k = gi.nq;
    if (k < 1 || k > kMaxK) return QSIM_E_ARG;
    if (gi.kind != QSIM_G_MAT && kind_arity(gi.kind) != k)
        return kind_arity(gi.kind) ? QSIM_E_ARG : QSIM_E_UNSUPPORTED;
    for (int j = 0; j < k; j++) {
        if (gi.q[j] < 0 || gi.q[j] >= n) return QSIM_E_QUBIT;
        for (int l = 0; l < j; l++)
            if (gi.q[l] == gi.q[j]) return QSIM_E_QUBIT;
    }
    double th[3] = {gi.theta[0], gi.theta[1], gi.theta[2]};
    bool symbolic = false;
    if (gi.slot >= 0) {
        if (keep_params) {
            if (!is_half_angle_linear(gi.kind)) return QSIM_E_UNSUPPORTED;
            if (size_t(gi.slot) >= in.n_params) return QSIM_E_ARG;
            symbolic = true;
        } else {
            if (!in.params || size_t(gi.slot) >= in.n_params) return QSIM_E_ARG;
            th[0] = in.params[gi.slot];
        }
    }
    for (double v : th)
        if (!std::isfinite(v)) return QSIM_E_ARG;
    Op op;
    op.src_kind = gi.kind;
    op.orient = (k == 2 && gi.q[0] > gi.q[1]) ? 1 : 0;
    int d = 1 << k;
    if (gi.kind == QSIM_G_MAT) {
        if (!in.mats || size_t(gi.mat_off) + size_t(d) * d > in.n_mats) return QSIM_E_ARG;
        const double *mats = in.mats;
        m.resize(size_t(d) * d);
        const double *src = mats + 2 * size_t(gi.mat_off);
        for (int e = 0; e < d * d; e++) {
            m[e] = cd(src[2 * e], src[2 * e + 1]);
            if (!std::isfinite(m[e].real()) || !std::isfinite(m[e].imag())) return QSIM_E_ARG;
        }
        to_sorted(gi.q, k, m.data(), 1, &op);
    } else if (symbolic) {
        // basis blocks: theta = 0 gives the cos(theta/2) block, theta = pi the sin block
        double t0[3] = {0.0, th[1], th[2]}, t1[3] = {M_PI, th[1], th[2]};
        int rc = gate_matrix(gi, t0, &m);
        if (rc) return rc;
        rc = gate_matrix(gi, t1, &m2);
        if (rc) return rc;
        m.insert(m.end(), m2.begin(), m2.end());
        to_sorted(gi.q, k, m.data(), 2, &op);
        op.np = 1;
        op.slot[0] = gi.slot;
    } else {
        int rc = gate_matrix(gi, th, &m);
        if (rc) return rc;
        to_sorted(gi.q, k, m.data(), 1, &op);
    }
    *out = std::move(op);
    return QSIM_OK;
}

}  // namespace

int lower(int n, const qsim_gate *g, size_t ng, const GateInputs &in, bool keep_params,
          bool allow_meas, Lowered *out) {
    out->ops.clear();
    out->op_epoch.clear();
    out->meas.clear();
    out->input_gates = 0;
    // First, in record order: epochs, measurement records and the gate
    // record of every operator.  Then the operators themselves, which are
    // independent, on several threads.  The first failing record in
    // program order decides the error.
    std::vector<size_t> op_gate;
    op_gate.reserve(ng);
    int epoch = 0;
    int first_rc = QSIM_OK;
    size_t first_at = ng;
    // Records out->meas[run_begin ..] follow each other with no operator or
    // barrier between them.  Non-unitary steps on different qubits commute,
    // and after a measurement, an assertion or a reset the qubit is definite,
    // so a reset that meets an earlier record of its qubit in the same run
    // either joins a measurement (one record that collapses the state and
    // moves the outcome to |0>) or is a no-op and is dropped; each such
    // reset saves a reduction and a rewrite of the state (QSIM_FOLD_RESETS=0
    // keeps every record as written).
    const char *fv = std::getenv("QSIM_FOLD_RESETS");
    const bool fold_resets = !(fv && *fv && std::atoi(fv) == 0);
    size_t run_begin = 0;
    for (size_t i = 0; i < ng && first_at == ng; i++) {
        const qsim_gate &gi = g[i];
        if (gi.kind == QSIM_G_BARRIER) {
            epoch++;
            run_begin = out->meas.size();
            continue;
        }
        if (gi.kind == QSIM_G_MEASURE || gi.kind == QSIM_G_RESET || gi.kind == QSIM_G_ASSERT0) {
            int rc = QSIM_OK;
            if (!allow_meas) rc = QSIM_E_UNSUPPORTED;
            else if (gi.nq != 1) rc = QSIM_E_ARG;
            else if (gi.q[0] < 0 || gi.q[0] >= n) rc = QSIM_E_QUBIT;
            else if (gi.kind != QSIM_G_RESET && gi.slot < 0) rc = QSIM_E_ARG;
            if (rc) {
                first_rc = rc;
                first_at = i;
                break;
            }
            if (gi.kind == QSIM_G_RESET && fold_resets) {
                bool folded = false;
                for (size_t j = out->meas.size(); j > run_begin; j--) {
                    MeasRec &prev = out->meas[j - 1];
                    if (prev.q != gi.q[0]) continue;
                    if (prev.kind == DEVOP_MEASURE) prev.kind = DEVOP_MEASURE_RESET;
                    folded = true;
                    break;
                }
                if (folded) continue;
            }
            MeasRec r;
            r.epoch = epoch;
            r.kind = gi.kind == QSIM_G_MEASURE ? DEVOP_MEASURE
                     : gi.kind == QSIM_G_ASSERT0 ? DEVOP_ASSERT0 : DEVOP_RESET;
            r.q = gi.q[0];
            r.slot = gi.kind == QSIM_G_RESET ? 0 : gi.slot;
            out->meas.push_back(r);
            epoch++;
            continue;
        }
        op_gate.push_back(i);
        out->op_epoch.push_back(epoch);
        run_begin = out->meas.size();
    }
    // the operators, in contiguous ranges; each range keeps its first error
    const size_t nops = op_gate.size();
    out->ops.resize(nops);
    const size_t kPerThread = 16384;
    const int nth = int(std::min<size_t>(size_t(std::max(1, std::min(16, int(std::thread::hardware_concurrency())))),
                                         (nops + kPerThread - 1) / kPerThread));
    std::vector<int> rcs(size_t(std::max(nth, 1)), QSIM_OK);
    std::vector<size_t> at(size_t(std::max(nth, 1)), ng);
    std::vector<char> oom(size_t(std::max(nth, 1)), 0);
    auto work = [&](int w) {
        try {
            std::vector<cd> m, m2;
            for (size_t j = nops * size_t(w) / size_t(nth); j < nops * size_t(w + 1) / size_t(nth); j++) {
                const int rc = lower_gate(n, g[op_gate[j]], in, keep_params, &out->ops[j], m, m2);
                if (rc) {
                    rcs[size_t(w)] = rc;
                    at[size_t(w)] = op_gate[j];
                    return;
                }
            }
        } catch (const std::bad_alloc &) {
            oom[size_t(w)] = 1;
        }
    };
    if (nth > 1) {
        std::vector<std::thread> th;
        for (int w = 1; w < nth; w++) th.emplace_back(work, w);
        work(0);
        for (auto &x : th) x.join();
    } else if (nth == 1) {
        work(0);
    }
    for (char f : oom)
        if (f) throw std::bad_alloc();
    for (size_t w = 0; w < rcs.size(); w++)
        if (rcs[w] && at[w] < first_at) {
            first_at = at[w];
            first_rc = rcs[w];
        }
    if (first_rc) return first_rc;
    out->input_gates = int64_t(nops);
    out->n_epochs = epoch + 1;
    return QSIM_OK;
}

}  // namespace qs
