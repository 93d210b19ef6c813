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

#include "host.h"

namespace qs {

double max_abs(const cd *m, size_t n) {
    double r = 0;
    for (size_t i = 0; i < n; i++) r = std::max(r, std::abs(m[i]));
    return r;
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
void fuse_width(int n, Lowered *L, const FuseConfig &cfg) {
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
}

}  // namespace

void fuse(int n, Lowered *L, const FuseConfig &cfg, int64_t counts[6]) {
    for (int l = 0; l < 6; l++) counts[l] = -1;
    counts[0] = int64_t(L->ops.size());
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
    if (cfg.level >= 5) { fuse_width(n, L, cfg); counts[5] = int64_t(L->ops.size()); }
}

}  // namespace qs
