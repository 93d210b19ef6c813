// Gate fusion (Section 4.2, Figs. 3-4), applied in the paper's order:
//   F1  consecutive 1-qubit gates on one wire merge into one C1 operator;
//   F3  a 2-qubit operator absorbs the adjacent 1-qubit operator on each of
//       its wires, forward (the 1q gate comes first) before backward;
//   SWAP normalisation: every 2-qubit operator is expressed on ascending
//       qubits (done once, in lowering, as an index relabelling);
//   F2  consecutive 2-qubit operators on the same pair merge into one C2.
// "Consecutive" is read along each wire (circuit DAG), not along the list.
//
// Level 5 goes beyond the paper: a greedy, cost-driven merge into operators
// of up to `max_width` qubits.  The cost of an operator is the number of its
// nonzero XOR-shift diagonals (complex MACs per amplitude in the sweep
// kernels) plus a fixed cost per operator (one more LDS round trip); a merge
// is kept when it does not raise the total.  Because fused matrices keep the
// sparsity of their factors (a Pauli-string exponential has two nonzero
// diagonals whatever its width), this recovers the gate specialisation the
// paper gave up under fusion (Section 4.1).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <thread>

#include "host.h"

namespace qs {

double max_abs(const cd *m, size_t n) {
    // the largest squared modulus, one square root at the end
    double r2 = 0;
    for (size_t i = 0; i < n; i++) {
        const double a = m[i].real(), b = m[i].imag();
        r2 = std::max(r2, a * a + b * b);
    }
    return std::sqrt(r2);
}

// Bit m of *present is set when some row r has M[r][r ^ m] above tol.
// Returns the number of set bits.
int xor_terms(const cd *m, int k, double tol, uint32_t *present) {
    int d = 1 << k;
    uint32_t p = 0;
    for (int s = 0; s < d; s++) {
        for (int r = 0; r < d; r++) {
            const cd v = m[size_t(r) * d + (r ^ s)];
            if (std::fabs(v.real()) > tol || std::fabs(v.imag()) > tol) { p |= 1u << s; break; }
        }
    }
    *present = p;
    return __builtin_popcount(p);
}

namespace {

// Positions of `sub` qubits inside the ascending list `uq`.
void positions(const Op &sub, const int *uq, int uk, int *pos) {
    for (int j = 0; j < sub.k; j++)
        for (int i = 0; i < uk; i++)
            if (uq[i] == sub.q[j]) pos[j] = i;
}

// Offsets of the 2^k members of a group for ascending positions pos[].
void member_offsets(const int *pos, int k, int *off) {
    off[0] = 0;
    for (int r = 1; r < (1 << k); r++) {
        int j = __builtin_ctz(r);
        off[r] = off[r & (r - 1)] + (1 << pos[j]);
    }
}

int insert_zeros(int g, const int *pos, int k) {
    for (int j = 0; j < k; j++) {
        int p = pos[j];
        g = ((g >> p) << (p + 1)) | (g & ((1 << p) - 1));
    }
    return g;
}

int op_terms(const Op &o, double rel_tol) {
    int d = o.dim();
    size_t blk = size_t(d) * d;
    uint32_t all = 0;
    double mx = max_abs(o.m.data(), o.m.size());
    for (int b = 0; b < (1 << o.np); b++) {
        uint32_t p;
        xor_terms(o.m.data() + b * blk, o.k, rel_tol * mx, &p);
        all |= p;
    }
    return __builtin_popcount(all);
}

}  // namespace

// Expand basis block `basis` of `a` onto the ascending union qubits uq.
void embed(const Op &a, const int *uq, int uk, std::vector<cd> *out, int basis) {
    int pos[kMaxK], off[1 << kMaxK];
    positions(a, uq, uk, pos);
    member_offsets(pos, a.k, off);
    int D = 1 << uk, d = a.dim();
    const cd *am = a.m.data() + size_t(basis) * d * d;
    out->assign(size_t(D) * D, cd(0));
    for (int g = 0; g < (D >> a.k); g++) {
        int base = insert_zeros(g, pos, a.k);
        for (int r = 0; r < d; r++)
            for (int c = 0; c < d; c++)
                (*out)[size_t(base + off[r]) * D + base + off[c]] = am[size_t(r) * d + c];
    }
}

namespace {

// Expand every basis block of `a` onto qubits uq.
Op expand(const Op &a, const int *uq, int uk) {
    if (uk == a.k) return a;
    Op r;
    r.k = uk;
    for (int j = 0; j < uk; j++) r.q[j] = uq[j];
    r.np = a.np;
    std::copy(a.slot, a.slot + 3, r.slot);
    int D = 1 << uk;
    r.m.resize(size_t(1 << a.np) * D * D);
    std::vector<cd> tmp;
    for (int b = 0; b < (1 << a.np); b++) {
        embed(a, uq, uk, &tmp, b);
        std::copy(tmp.begin(), tmp.end(), r.m.begin() + size_t(b) * D * D);
    }
    return r;
}

// big := E(small) * big  (left == true: small applied after big)
// big := big * E(small)  (left == false: small applied before big)
// small's qubits must be a subset of big's.  Angle slots concatenate.
void mul_small(Op *big, const Op &small, bool left) {
    int pos[kMaxK], off[1 << kMaxK];
    positions(small, big->q, big->k, pos);
    member_offsets(pos, small.k, off);
    const int D = big->dim(), d = small.dim();
    const size_t BB = size_t(D) * D, sb = size_t(d) * d;
    const int nb_big = 1 << big->np, nb_small = 1 << small.np;
    std::vector<cd> res(BB * nb_big * nb_small);
    // the small factor's nonzero entries, as (row, col, re, im); complex
    // products are written out (std::complex's operator* takes the
    // NaN-checking library path)
    struct Nz { int i, j; double re, im; };
    for (int bs = 0; bs < nb_small; bs++) {
        const cd *S = small.m.data() + bs * sb;
        Nz nz[(1 << kMaxK) * (1 << kMaxK)];
        int nnz = 0;
        for (int i = 0; i < d; i++)
            for (int j = 0; j < d; j++) {
                const cd v = S[size_t(i) * d + j];
                if (v.real() != 0.0 || v.imag() != 0.0) nz[nnz++] = {i, j, v.real(), v.imag()};
            }
        for (int bb = 0; bb < nb_big; bb++) {
            const double *M = reinterpret_cast<const double *>(big->m.data() + bb * BB);
            double *R = reinterpret_cast<double *>(res.data() + (size_t(bb) + size_t(bs) * nb_big) * BB);
            for (int g = 0; g < (D >> small.k); g++) {
                const int base = insert_zeros(g, pos, small.k);
                if (left) {
                    // R[base+off[i]][c] = sum_j S[i][j] M[base+off[j]][c]
                    for (int e = 0; e < nnz; e++) {
                        const double *src = M + 2 * size_t(base + off[nz[e].j]) * D;
                        double *dst = R + 2 * size_t(base + off[nz[e].i]) * D;
                        const double sr = nz[e].re, si = nz[e].im;
                        for (int c = 0; c < D; c++) {
                            const double mr = src[2 * c], mi = src[2 * c + 1];
                            dst[2 * c] += sr * mr - si * mi;
                            dst[2 * c + 1] += sr * mi + si * mr;
                        }
                    }
                } else {
                    // R[r][base+off[i]] = sum_j M[r][base+off[j]] S[j][i]
                    for (int r = 0; r < D; r++) {
                        const double *src = M + 2 * size_t(r) * D;
                        double *dst = R + 2 * size_t(r) * D;
                        for (int e = 0; e < nnz; e++) {
                            const double mr = src[2 * (base + off[nz[e].i])], mi = src[2 * (base + off[nz[e].i]) + 1];
                            const double sr = nz[e].re, si = nz[e].im;
                            dst[2 * (base + off[nz[e].j])] += mr * sr - mi * si;
                            dst[2 * (base + off[nz[e].j]) + 1] += mr * si + mi * sr;
                        }
                    }
                }
            }
        }
    }
    for (int j = 0; j < small.np; j++) big->slot[big->np + j] = small.slot[j];
    big->np += small.np;
    big->m.swap(res);
}

int union_qubits(const Op &a, const Op &b, int *uq) {
    int n = 0, i = 0, j = 0;
    while (i < a.k || j < b.k) {
        int x = (j >= b.k || (i < a.k && a.q[i] < b.q[j])) ? a.q[i++] : b.q[j];
        if (n == 0 || uq[n - 1] != x) uq[n++] = x;
        if (j < b.k && b.q[j] == x) j++;
        if (n > kMaxK) return n;
    }
    return n;
}

void compact(Lowered *L) {
    std::vector<Op> ops;
    std::vector<int> nep;
    ops.reserve(L->ops.size());
    nep.reserve(L->ops.size());
    for (size_t i = 0; i < L->ops.size(); i++) {
        if (L->ops[i].dead) continue;
        nep.push_back(L->op_epoch[i]);
        ops.push_back(std::move(L->ops[i]));
    }
    L->ops.swap(ops);
    L->op_epoch.swap(nep);
}

// F1: merge wire-consecutive 1-qubit operators.
void fuse_f1(int n, Lowered *L, const FuseConfig &cfg) {
    const std::vector<int> *ep = &L->op_epoch;
    std::vector<int> last(n, -1);
    for (size_t i = 0; i < L->ops.size(); i++) {
        Op &o = L->ops[i];
        if (o.k == 1) {
            int j = last[o.q[0]];
            if (j >= 0 && L->ops[j].k == 1 && (*ep)[j] == (*ep)[i] &&
                L->ops[j].np + o.np <= cfg.max_params) {
                mul_small(&L->ops[j], o, true);
                o.dead = true;
                continue;
            }
        }
        for (int t = 0; t < o.k; t++) last[o.q[t]] = int(i);
    }
    compact(L);
}

// F3: 2-qubit operators absorb the adjacent 1-qubit operator of each wire.
void fuse_f3(int n, Lowered *L, const FuseConfig &cfg) {
    const std::vector<int> *ep = &L->op_epoch;
    const size_t N = L->ops.size();
    // previous / next operator on the wire of each 1-qubit operator
    std::vector<int> prev(N, -1), next(N, -1), last(n, -1);
    for (size_t i = 0; i < N; i++) {
        const Op &o = L->ops[i];
        for (int t = 0; t < o.k; t++) {
            int j = last[o.q[t]];
            if (o.k == 1) prev[i] = j;
            if (j >= 0 && L->ops[j].k == 1) next[j] = int(i);
            last[o.q[t]] = int(i);
        }
    }
    for (size_t i = 0; i < N; i++) {
        Op &u = L->ops[i];
        if (u.k != 1) continue;
        int f = next[i], b = prev[i];
        if (f >= 0 && L->ops[f].k == 2 && (*ep)[f] == (*ep)[i] &&
            L->ops[f].np + u.np <= cfg.max_params) {
            mul_small(&L->ops[f], u, false);    // G' = G (u (x) I)
            u.dead = true;
        } else if (b >= 0 && !L->ops[b].dead && L->ops[b].k == 2 && (*ep)[b] == (*ep)[i] &&
                   L->ops[b].np + u.np <= cfg.max_params) {
            mul_small(&L->ops[b], u, true);     // G' = (u (x) I) G
            u.dead = true;
        }
    }
    compact(L);
}

// F2: merge wire-consecutive 2-qubit operators on the same pair.  Without
// normalisation (`ordered`), only operators whose gates named the pair in the
// same order merge.
void fuse_f2(int n, Lowered *L, const FuseConfig &cfg, bool ordered,
             const std::vector<int> &orient) {
    const std::vector<int> *ep = &L->op_epoch;
    std::vector<int> last(n, -1);
    for (size_t i = 0; i < L->ops.size(); i++) {
        Op &o = L->ops[i];
        if (o.k == 2) {
            int j = last[o.q[0]];
            if (j >= 0 && j == last[o.q[1]] && L->ops[j].k == 2 && (*ep)[j] == (*ep)[i] &&
                L->ops[j].np + o.np <= cfg.max_params &&
                (!ordered || orient[j] == orient[i])) {
                mul_small(&L->ops[j], o, true);
                o.dead = true;
                continue;
            }
        }
        for (int t = 0; t < o.k; t++) last[o.q[t]] = int(i);
    }
}

// Level 5: cost-driven merge into operators of up to max_width qubits.
// Returns the cost of the resulting list: the sum, in list order, of each
// operator's terms (op_terms; 2^k when not sparse) plus lds_cost.
double fuse_width(int n, Lowered *L, const FuseConfig &cfg) {
    const std::vector<int> *ep = &L->op_epoch;
    const double tol = 1e-14;
    std::vector<Op> out;
    std::vector<int> out_terms, out_ep;
    std::vector<int> owner(n, -1);
    int closed_before = 0;
    const int kWindow = 4;
    out.reserve(L->ops.size());
    for (size_t i = 0; i < L->ops.size(); i++) {
        Op &o = L->ops[i];
        if (!out.empty() && out_ep.back() != (*ep)[i]) closed_before = int(out.size());
        int gmin = closed_before;
        for (int t = 0; t < o.k; t++) gmin = std::max(gmin, owner[o.q[t]]);
        int o_terms = cfg.sparse ? op_terms(o, tol) : (1 << o.k);
        int best = -1, best_terms = 0;
        double best_gain = -1e30;
        Op best_op;
        int lo = std::max(gmin, int(out.size()) - kWindow);
        for (int c = int(out.size()) - 1; c >= lo; c--) {
            int uq[2 * kMaxK];
            int uk = union_qubits(out[c], o, uq);
            if (uk > cfg.max_width) continue;
            if (out[c].np + o.np > cfg.max_params) continue;
            Op merged = expand(out[c], uq, uk);
            mul_small(&merged, o, true);
            int mt = cfg.sparse ? op_terms(merged, tol) : (1 << uk);
            double gain = out_terms[c] + o_terms + cfg.lds_cost - mt;
            if (gain >= 0 && gain > best_gain) {
                best_gain = gain;
                best = c;
                best_terms = mt;
                best_op = std::move(merged);
            }
        }
        if (best >= 0) {
            out[best] = std::move(best_op);
            out_terms[best] = best_terms;
            for (int t = 0; t < o.k; t++) owner[o.q[t]] = best;
        } else {
            for (int t = 0; t < o.k; t++) owner[o.q[t]] = int(out.size());
            out.push_back(std::move(o));
            out_terms.push_back(o_terms);
            out_ep.push_back((*ep)[i]);
        }
    }
    L->ops.swap(out);
    L->op_epoch.swap(out_ep);
    // out_terms holds each operator's terms as op_terms counts them
    double c = 0;
    for (int t : out_terms) c += t + cfg.lds_cost;
    return c;
}

// An operator of at most kMaxK qubits in XOR-shift form,
//   y[r] = sum over m in present of d[m][r] * x[r ^ m],
// used to evaluate the products of many candidate runs cheaply: a gate with
// few terms multiplies in (its terms x our terms x 2^k) MACs.  Only the rows
// d[m] of present m are meaningful.
struct XOp {
    int k = 0;
    int q[kMaxK] = {0, 0, 0, 0, 0};
    uint32_t present = 0;
    cd d[1 << kMaxK][1 << kMaxK];
};

inline int gather_bits(int r, const int *sel, int k) {
    int out = 0;
    for (int j = 0; j < k; j++) out |= ((r >> sel[j]) & 1) << j;
    return out;
}
inline int scatter_bits(int m, const int *sel, int k) {
    int out = 0;
    for (int j = 0; j < k; j++) out |= ((m >> j) & 1) << sel[j];
    return out;
}

// Bit m set when M[r][r ^ m] != 0 for some r (exact zeros only).
uint32_t exact_present(const Op &o) {
    const int D = o.dim();
    uint32_t p = 0;
    for (int m = 0; m < D; m++)
        for (int r = 0; r < D; r++)
            if (o.m[size_t(r) * D + (r ^ m)] != cd(0)) { p |= 1u << m; break; }
    return p;
}

void xop_from(const Op &o, uint32_t present, XOp *x) {
    x->k = o.k;
    for (int j = 0; j < o.k; j++) x->q[j] = o.q[j];
    x->present = present;
    const int D = o.dim();
    for (uint32_t pm = present; pm; pm &= pm - 1) {
        const int m = __builtin_ctz(pm);
        for (int r = 0; r < D; r++) x->d[m][r] = o.m[size_t(r) * D + (r ^ m)];
    }
}

// `a` re-expressed on the ascending qubit list uq (a superset of its own).
void xop_expand(const XOp &a, const int *uq, int uk, XOp *out) {
    int sel[kMaxK];
    for (int j = 0; j < a.k; j++)
        for (int i = 0; i < uk; i++)
            if (uq[i] == a.q[j]) sel[j] = i;
    out->k = uk;
    for (int i = 0; i < uk; i++) out->q[i] = uq[i];
    out->present = 0;
    const int D = 1 << uk;
    int gi[1 << kMaxK];
    for (int r = 0; r < D; r++) gi[r] = gather_bits(r, sel, a.k);
    for (uint32_t pm = a.present; pm; pm &= pm - 1) {
        const int m = __builtin_ctz(pm);
        const int mm = scatter_bits(m, sel, a.k);
        out->present |= 1u << mm;
        for (int r = 0; r < D; r++) out->d[mm][r] = a.d[m][gi[r]];
    }
}

// out := G * cur with G = gate o (present terms gp) on a subset of cur's
// qubits:  (G M)[r][r^g^m] += G[r][r^g] M_m[r^g].
void xop_left_mul(const Op &o, uint32_t gp, const XOp &cur, XOp *out) {
    const int D = 1 << cur.k, Do = o.dim();
    int sel[kMaxK];
    for (int j = 0; j < o.k; j++)
        for (int i = 0; i < cur.k; i++)
            if (cur.q[i] == o.q[j]) sel[j] = i;
    int gi[1 << kMaxK];
    for (int r = 0; r < D; r++) gi[r] = gather_bits(r, sel, o.k);
    out->k = cur.k;
    std::copy(cur.q, cur.q + kMaxK, out->q);
    uint32_t present = 0;
    for (uint32_t pg = gp; pg; pg &= pg - 1) {
        const int gm = __builtin_ctz(pg);
        const int gmm = scatter_bits(gm, sel, o.k);
        double gre[1 << kMaxK], gim[1 << kMaxK];
        for (int r = 0; r < D; r++) {
            const cd v = o.m[size_t(gi[r]) * Do + (gi[r] ^ gm)];
            gre[r] = v.real();
            gim[r] = v.imag();
        }
        for (uint32_t pm = cur.present; pm; pm &= pm - 1) {
            const int m = __builtin_ctz(pm);
            const int t = gmm ^ m;
            const cd *src = cur.d[m];
            cd *dst = out->d[t];
            if (!(present & (1u << t))) {
                // first contribution to row t
                present |= 1u << t;
                for (int r = 0; r < D; r++) {
                    const cd b = src[r ^ gmm];
                    dst[r] = cd(gre[r] * b.real() - gim[r] * b.imag(), gre[r] * b.imag() + gim[r] * b.real());
                }
            } else {
                for (int r = 0; r < D; r++) {
                    const cd b = src[r ^ gmm];
                    dst[r] += cd(gre[r] * b.real() - gim[r] * b.imag(), gre[r] * b.imag() + gim[r] * b.real());
                }
            }
        }
    }
    out->present = present;
}

// Terms above rel_tol times the largest entry (as op_terms counts them).
int xop_terms(const XOp &x, double rel_tol) {
    const int D = 1 << x.k;
    double rmax[1 << kMaxK];
    double mx = 0;
    int nt = 0;
    for (uint32_t pm = x.present; pm; pm &= pm - 1) {
        const cd *row = x.d[__builtin_ctz(pm)];
        double v = 0;
        for (int r = 0; r < D; r++) v = std::max(v, std::max(std::fabs(row[r].real()), std::fabs(row[r].imag())));
        rmax[nt++] = v;
        mx = std::max(mx, v);
    }
    const double tol = rel_tol * mx;
    int n = 0;
    for (int i = 0; i < nt; i++) n += rmax[i] > tol;
    return n;
}

// Ascending union of two ascending qubit lists (stops past kMaxK).
int union_lists(const int *a, int ka, const int *b, int kb, int *uq) {
    int n = 0, i = 0, j = 0;
    while (i < ka || j < kb) {
        int x;
        if (j >= kb || (i < ka && a[i] < b[j])) x = a[i++];
        else if (i >= ka || b[j] < a[i]) x = b[j++];
        else { x = a[i++]; j++; }
        uq[n++] = x;
        if (n > kMaxK) return n;
    }
    return n;
}

// Level 5, second candidate: the cheapest partition of the operator list into
// runs of consecutive operators, each run merged into one operator of at most
// max_width qubits (dynamic programming over run ends, same cost model).  A
// run's partial products may be dense -- half of a CNOT ladder -- while the
// whole run is sparse -- the Pauli-string exponential the ladder implements
// -- which a merge judged one step at a time does not reach.
// The runs that start at one operator: for e = s + 1 .. s + n, the terms and
// width of the product of operators s .. e - 1.
constexpr int kMaxRun = 64;
struct RunTable {
    uint8_t n = 0;
    uint8_t terms[kMaxRun];
    uint8_t k[kMaxRun];
};

// Reads `in` only; returns the cost of the chosen list, summed as
// fuse_width sums its own.
double fuse_runs(const Lowered &in, const FuseConfig &cfg, Lowered *out) {
    const double tol = 1e-14;
    const Lowered *L = &in;
    const size_t N = L->ops.size();
    std::vector<double> best(N + 1, 1e300);
    std::vector<int> from(N + 1, -1);
    best[0] = 0;
    bool any_params = false;
    for (const Op &o : L->ops) any_params = any_params || o.np > 0;
    std::vector<uint32_t> gp;
    if (!any_params) {
        gp.resize(N);
        for (size_t i = 0; i < N; i++) gp[i] = exact_present(L->ops[i]);
    }
    // the products of the runs from s (independent of the cost so far)
    auto table = [&](size_t s, XOp *b0, XOp *b1, RunTable *t) {
        t->n = 0;
        auto put = [&](int terms, int k) {
            t->terms[t->n] = uint8_t(terms);
            t->k[t->n] = uint8_t(k);
            t->n++;
        };
        if (!any_params) {
            // products in XOR-shift form (no angle slots to carry)
            XOp *cur = b0, *nxt = b1;
            xop_from(L->ops[s], gp[s], cur);
            put(xop_terms(*cur, tol), cur->k);
            for (size_t e = s + 2; e <= N && int(e - s) <= kMaxRun; e++) {
                const Op &o = L->ops[e - 1];
                if (L->op_epoch[e - 1] != L->op_epoch[s]) break;
                int uq[2 * kMaxK];
                const int uk = union_lists(cur->q, cur->k, o.q, o.k, uq);
                if (uk > cfg.max_width) break;
                if (uk != cur->k) {
                    xop_expand(*cur, uq, uk, nxt);
                    std::swap(cur, nxt);
                }
                xop_left_mul(o, gp[e - 1], *cur, nxt);
                std::swap(cur, nxt);
                put(xop_terms(*cur, tol), cur->k);
            }
        } else {
            Op cur = L->ops[s];
            for (size_t e = s + 1; e <= N && int(e - s) <= kMaxRun; e++) {
                if (e > s + 1) {
                    const Op &o = L->ops[e - 1];
                    if (L->op_epoch[e - 1] != L->op_epoch[s]) break;
                    if (cur.np + o.np > cfg.max_params) break;
                    int uq[2 * kMaxK];
                    const int uk = union_qubits(cur, o, uq);
                    if (uk > cfg.max_width) break;
                    cur = expand(cur, uq, uk);
                    mul_small(&cur, o, true);
                }
                put(cfg.sparse ? op_terms(cur, tol) : 0, cur.k);
            }
        }
    };
    // blocks of starts: their tables on several threads, then the dynamic
    // programme over the block in order
    const size_t kBlock = 8192;
    const int nth = std::max(1, std::min(16, int(std::thread::hardware_concurrency())));
    std::vector<RunTable> tab(std::min(kBlock, N));
    for (size_t b0 = 0; b0 < N; b0 += kBlock) {
        const size_t nb = std::min(kBlock, N - b0);
        const int use = int(std::min<size_t>(size_t(nth), (nb + 255) / 256));
        std::vector<char> failed(size_t(use), 0);
        auto work = [&](int w) {
            try {
                std::unique_ptr<XOp> x0(new XOp), x1(new XOp);
                for (size_t i = size_t(w); i < nb; i += size_t(use)) table(b0 + i, x0.get(), x1.get(), &tab[i]);
            } catch (const std::bad_alloc &) {
                failed[size_t(w)] = 1;
            }
        };
        std::vector<std::thread> th;
        for (int w = 1; w < use; w++) th.emplace_back(work, w);
        work(0);
        for (auto &x : th) x.join();
        for (char f : failed)
            if (f) throw std::bad_alloc();
        for (size_t i = 0; i < nb; i++) {
            const size_t s = b0 + i;
            for (int j = 0; j < tab[i].n; j++) {
                const size_t e = s + 1 + size_t(j);
                const double c = best[s] + (cfg.sparse ? tab[i].terms[j] : (1 << tab[i].k[j])) + cfg.lds_cost;
                if (c < best[e]) {
                    best[e] = c;
                    from[e] = int(s);
                }
            }
        }
    }
    // rebuild the chosen runs, last to first
    std::vector<std::pair<int, int>> runs;
    for (int e = int(N); e > 0; e = from[e]) runs.push_back({from[e], e});
    std::reverse(runs.begin(), runs.end());
    // each run's dense product (independent of the others: several threads,
    // each on a contiguous range of runs)
    std::vector<Op> fused(runs.size());
    std::vector<int> out_ep(runs.size());
    std::vector<int> terms(runs.size());
    const size_t nr = runs.size();
    const int use = int(std::min<size_t>(size_t(nth), (nr + 1023) / 1024));
    std::vector<char> failed(size_t(std::max(use, 1)), 0);
    auto rebuild = [&](int w) {
        try {
            for (size_t j = nr * size_t(w) / size_t(use); j < nr * size_t(w + 1) / size_t(use); j++) {
                const auto &r = runs[j];
                Op cur = L->ops[size_t(r.first)];
                for (int i = r.first + 1; i < r.second; i++) {
                    int uq[2 * kMaxK];
                    const int uk = union_qubits(cur, L->ops[size_t(i)], uq);
                    cur = expand(cur, uq, uk);
                    mul_small(&cur, L->ops[size_t(i)], true);
                }
                out_ep[j] = L->op_epoch[size_t(r.first)];
                terms[j] = cfg.sparse ? op_terms(cur, tol) : (1 << cur.k);
                fused[j] = std::move(cur);
            }
        } catch (const std::bad_alloc &) {
            failed[size_t(w)] = 1;
        }
    };
    if (use > 0) {
        std::vector<std::thread> th;
        for (int w = 1; w < use; w++) th.emplace_back(rebuild, w);
        rebuild(0);
        for (auto &x : th) x.join();
        for (char f : failed)
            if (f) throw std::bad_alloc();
    }
    out->ops.swap(fused);
    out->op_epoch.swap(out_ep);
    double c = 0;
    for (int t : terms) c += t + cfg.lds_cost;
    return c;
}

// The paper's passes, levels 1-4 (level 5 starts from level 4's list).
void fuse_paper(int n, Lowered *L, const FuseConfig &cfg, int64_t counts[6]) {
    if (cfg.level >= 1) { fuse_f1(n, L, cfg); counts[1] = int64_t(L->ops.size()); }
    if (cfg.level >= 2) { fuse_f3(n, L, cfg); counts[2] = int64_t(L->ops.size()); }
    if (cfg.level == 3) {
        // without SWAP normalisation a pair merges only with a pair that the
        // gates named in the same order
        std::vector<int> orient(L->ops.size(), 0);
        for (size_t i = 0; i < L->ops.size(); i++) orient[i] = L->ops[i].orient;
        fuse_f2(n, L, cfg, true, orient);
        compact(L);
        counts[3] = int64_t(L->ops.size());
    }
    if (cfg.level >= 4) {
        std::vector<int> none;
        fuse_f2(n, L, cfg, false, none);
        compact(L);
        counts[3] = counts[4] = int64_t(L->ops.size());
    }
}

}  // namespace

void fuse(int n, Lowered *L, const FuseConfig &cfg, int64_t counts[6]) {
    for (int l = 0; l < 6; l++) counts[l] = -1;
    counts[0] = int64_t(L->ops.size());
    if (cfg.level < 5) {
        fuse_paper(n, L, cfg, counts);
        return;
    }
    {
        // Two candidates, the cheaper under the cost model wins: the greedy
        // merge of the F1-F4 operators (any that commute into place) and the
        // best partition of the unfused gate list into runs of consecutive
        // gates.  They are independent: the partition starts at once on its
        // own thread, reading *L, while this thread runs F1-F4 and the greedy
        // merge on a copy.
        Lowered runs, mine;
        double runs_cost = 0, width_cost = 0;
        bool runs_ok = true;
        std::thread th([L, &runs, &cfg, &runs_ok, &runs_cost] {
            try {
                runs_cost = fuse_runs(*L, cfg, &runs);
            } catch (const std::bad_alloc &) {
                runs_ok = false;
            }
        });
        try {
            mine = *L;
            fuse_paper(n, &mine, cfg, counts);
            width_cost = fuse_width(n, &mine, cfg);
        } catch (...) {
            th.join();
            throw;
        }
        th.join();
        Lowered &win = (runs_ok && runs_cost < width_cost) ? runs : mine;
        L->ops.swap(win.ops);
        L->op_epoch.swap(win.op_epoch);
        counts[5] = int64_t(L->ops.size());
    }
}

}  // namespace qs
