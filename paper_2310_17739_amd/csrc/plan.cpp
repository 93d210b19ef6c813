// Pass planning and packing of fused operators into device tables.
//
// A pass reads every amplitude once and writes it once.  A tiled pass stages
// tiles of 2^t amplitudes in LDS: a tile spans a qubit set T that always
// contains the low c qubits (so that each tile is made of contiguous 2^c
// amplitude chunks) and t - c further qubits chosen for the pass; every
// operator whose qubits lie in T is applied to the tile in LDS before it is
// written back.  The paper instead runs one gate per device-wide
// synchronisation inside a single kernel (Section 4.1); grouping operators
// into passes is what lets several fused operators share one trip through
// HBM.
//
// Operators commute when they touch disjoint qubits, so a pass may take an
// operator from further down the list as long as no skipped operator before
// it shares one of its qubits.  Operators that share qubits may commute as
// well: two functions of one Pauli string each (a I + b P, the fused
// exponentials of the benchmark circuits) commute exactly when their strings
// do, and diagonal operators commute with each other and with any such
// operator whose string moves none of their qubits.  The planner lets an
// operator pass skipped ones it commutes with in this sense (QSIM_PLAN_COMMUTE=0
// turns it off).
//
// A qubit on which an operator is diagonal (no XOR shift of it moves that
// qubit: Z letters of a Pauli string, the phase of a controlled phase) need
// not be in the tile.  Every amplitude of a tile has the same value of that
// qubit, read from the tile's base index, and it selects which block of the
// operator's coefficients the tile uses.  Only the moved qubits then count
// against the tile's width.
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "host.h"

namespace qs {

namespace {

// Commutation class of an operator: a function a I + b X^x Z^z of one Pauli
// string (x, z over the circuit's qubits), a diagonal, or neither.  Entries
// are compared to 1e-13 of the operator's largest one.
struct OpClass {
    int kind = 0;   // 0 neither, 1 diagonal, 2 Pauli function
    uint64_t q = 0, x = 0, z = 0;
};

OpClass op_class(const Op &o) {
    OpClass c;
    c.q = o.mask();
    if (o.np > 0 || o.m.empty()) return c;
    const int d = o.dim();
    // moduli compared through their squares: |v| > tol  <=>  |v|^2 > tol^2
    auto n2 = [](cd v) { return v.real() * v.real() + v.imag() * v.imag(); };
    double mx2 = 0.0;
    for (const cd &v : o.m) mx2 = std::max(mx2, n2(v));
    const double tol2 = 1e-26 * mx2;   // (1e-13 times the largest modulus)^2
    auto at = [&](int r, int col) { return o.m[size_t(r) * d + size_t(col)]; };
    uint32_t present = 0;
    for (int s = 0; s < d; s++)
        for (int r = 0; r < d; r++)
            if (n2(at(r, r ^ s)) > tol2) { present |= 1u << s; break; }
    if (present == 1u) {
        c.kind = 1;
        return c;
    }
    // at most the main diagonal (constant) and one shift X
    const uint32_t others = present & ~1u;
    if (__builtin_popcount(others) != 1) return c;
    const int X = __builtin_ctz(others);
    if (present & 1u)
        for (int r = 1; r < d; r++)
            if (n2(at(r, r) - at(0, 0)) > tol2) return c;
    // the shift's entries: a common value times the signs (-1)^popcount(r & z)
    const cd d0 = at(0, X);
    int zl = 0;
    for (int j = 0; j < o.k; j++) {
        const cd v = at(1 << j, (1 << j) ^ X);
        if (n2(v + d0) <= tol2) zl |= 1 << j;
        else if (n2(v - d0) > tol2) return c;
    }
    for (int r = 0; r < d; r++) {
        const double sg = (__builtin_popcount(r & zl) & 1) ? -1.0 : 1.0;
        if (n2(at(r, r ^ X) - sg * d0) > tol2) return c;
    }
    c.kind = 2;
    for (int j = 0; j < o.k; j++) {
        if ((X >> j) & 1) c.x |= uint64_t(1) << o.q[j];
        if ((zl >> j) & 1) c.z |= uint64_t(1) << o.q[j];
    }
    return c;
}

bool commute(const OpClass &a, const OpClass &b) {
    if (!(a.q & b.q)) return true;
    if (a.kind == 2 && b.kind == 2)
        return ((__builtin_popcountll(a.x & b.z) + __builtin_popcountll(a.z & b.x)) & 1) == 0;
    if (a.kind == 1 && b.kind == 1) return true;
    if (a.kind == 1 && b.kind == 2) return (b.x & a.q) == 0;
    if (a.kind == 2 && b.kind == 1) return (a.x & b.q) == 0;
    return false;
}

// Operators scanned after every qubit is blocked by a skipped operator: only
// commuting ones can still join the pass, and a longer tail finds none more
// on the benchmark circuits.
constexpr int kCommuteTail = 64;

}  // namespace

void plan_passes(int n, const Lowered &L, const std::vector<uint32_t> &meta_bytes,
                 const std::vector<uint64_t> &need, const PlanConfig &cfg, std::vector<Pass> *passes) {
    passes->clear();
    const std::vector<Op> &ops = L.ops;
    const int N = int(ops.size());
    const int t = std::min(cfg.tile_qubits, n);
    const int c = std::min(cfg.low_qubits, t);
    const uint64_t all = (n >= 64) ? ~uint64_t(0) : ((uint64_t(1) << n) - 1);
    const uint64_t low = (uint64_t(1) << c) - 1;
    constexpr uint32_t kMeasBytes = sizeof(DevOp);   // a measurement record, no coefficients

    // operators of epoch e: [ep_begin[e], ep_begin[e + 1])
    std::vector<int> ep_begin(L.n_epochs + 1, N);
    for (int i = N - 1; i >= 0; i--) ep_begin[L.op_epoch[i]] = i;
    for (int e = L.n_epochs - 1; e >= 0; e--)
        if (ep_begin[e] > ep_begin[e + 1]) ep_begin[e] = ep_begin[e + 1];
    // measurement records after epoch e: [mb[e], mb[e + 1])
    std::vector<int> mb(L.n_epochs + 1, int(L.meas.size()));
    for (int i = int(L.meas.size()) - 1; i >= 0; i--) mb[L.meas[i].epoch] = i;
    for (int e = L.n_epochs - 1; e >= 0; e--)
        if (mb[e] > mb[e + 1]) mb[e] = mb[e + 1];

    auto tile_pass = [&](uint64_t T) {
        Pass p;
        p.kind = Pass::TILE;
        // pad the tile to exactly t qubits with the lowest unused qubits
        for (int q = 0; q < n && __builtin_popcountll(T) < t; q++) T |= uint64_t(1) << q;
        p.t = t;
        p.c = c;
        p.tile_mask = T;
        for (int q = c; q < n; q++)
            if ((T >> q) & 1) p.hi[p.nhi++] = q;
        int j = 0;
        for (int q = 0; q < n && j < 16; q++)
            if ((T >> q) & 1) p.tq[j++] = uint8_t(q);
        return p;
    };
    auto strided = [&](int i) {
        Pass p;
        p.kind = Pass::STRIDED;
        p.strided = true;
        p.ops = {i};
        passes->push_back(std::move(p));
    };

    if (cfg.one_op_per_pass) {
        for (int e = 0; e < L.n_epochs; e++) {
            for (int i = ep_begin[e]; i < ep_begin[e + 1]; i++) strided(i);
            for (int m = mb[e]; m < mb[e + 1]; m++) {
                Pass p;
                p.kind = Pass::MEASURE;
                p.meas = L.meas[m];
                passes->push_back(std::move(p));
            }
        }
        return;
    }

    if (t >= n) {
        // The whole state is one tile: resident passes run operators and
        // measurement records in program order, split where the records and
        // coefficients outgrow the LDS budget; operators too wide for the
        // tile kernel run as sweeps of their own.
        Pass cur = tile_pass(all);
        size_t meta = 0;
        auto flush = [&]() {
            if (!cur.seq.empty()) passes->push_back(std::move(cur));
            cur = tile_pass(all);
            meta = 0;
        };
        for (int e = 0; e < L.n_epochs; e++) {
            for (int i = ep_begin[e]; i < ep_begin[e + 1]; i++) {
                if (ops[i].k > cfg.max_tile_k) {
                    flush();
                    strided(i);
                    continue;
                }
                if (!cur.seq.empty() && meta + meta_bytes[i] > cfg.meta_budget) flush();
                cur.ops.push_back(i);
                cur.seq.push_back(i);
                meta += meta_bytes[i];
            }
            for (int m = mb[e]; m < mb[e + 1]; m++) {
                if (!cur.seq.empty() && meta + kMeasBytes > cfg.meta_budget) flush();
                cur.seq.push_back(~int(cur.inline_meas.size()));
                cur.inline_meas.push_back(L.meas[m]);
                meta += kMeasBytes;
            }
        }
        flush();
        return;
    }

    const char *cv = std::getenv("QSIM_PLAN_COMMUTE");
    const bool use_commute = !(cv && *cv && std::atoi(cv) == 0);
    std::vector<OpClass> cls;
    if (use_commute) {
        cls.resize(size_t(N));
        for (int i = 0; i < N; i++) cls[size_t(i)] = op_class(ops[i]);
    }
    std::vector<OpClass> skipped;   // classes of the operators a pass skipped, in order
    // doubly linked list of pending operators of one epoch
    std::vector<int> nxt(N + 1), prv(N + 1);
    const int head = N;
    for (int e = 0; e < L.n_epochs; e++) {
        const int b = ep_begin[e], en = ep_begin[e + 1];
        nxt[head] = b < en ? b : head;
        prv[head] = en - 1 >= b ? en - 1 : head;
        for (int i = b; i < en; i++) {
            nxt[i] = (i + 1 < en) ? i + 1 : head;
            prv[i] = (i > b) ? i - 1 : head;
        }
        while (nxt[head] != head) {
            const int first = nxt[head];
            if (ops[first].k > cfg.max_tile_k) {
                // too wide for the tile kernel at this precision: its own sweep
                nxt[head] = nxt[first];
                prv[nxt[first]] = head;
                strided(first);
                continue;
            }
            uint64_t T = low, blocked = 0;
            std::vector<int> sel;
            skipped.clear();
            size_t meta = 0;
            int scanned = 0, all_blocked_at = -1;
            for (int i = nxt[head]; i != head && scanned < cfg.window; i = nxt[i], scanned++) {
                const uint64_t qm = ops[i].mask();
                // may the operator run before every skipped one?
                bool free = !(qm & blocked);
                if (!free && use_commute) {
                    free = true;
                    const OpClass &ci = cls[size_t(i)];
                    for (const OpClass &s : skipped)
                        if (!commute(s, ci)) {
                            free = false;
                            break;
                        }
                }
                if (free && ops[i].k <= cfg.max_tile_k && (sel.empty() || meta + meta_bytes[i] <= cfg.meta_budget) &&
                    __builtin_popcountll(T | need[i]) <= t) {
                    T |= need[i];
                    sel.push_back(i);
                    meta += meta_bytes[i];
                } else {
                    blocked |= qm;
                    if (use_commute) skipped.push_back(cls[size_t(i)]);
                }
                if (blocked == all) {
                    if (!use_commute) break;
                    if (all_blocked_at < 0) all_blocked_at = scanned;
                    else if (scanned - all_blocked_at >= kCommuteTail) break;
                }
            }
            for (int i : sel) {
                nxt[prv[i]] = nxt[i];
                prv[nxt[i]] = prv[i];
            }
            Pass p = tile_pass(T);
            p.ops = std::move(sel);
            p.seq = p.ops;
            passes->push_back(std::move(p));
        }
        for (int m = mb[e]; m < mb[e + 1]; m++) {
            Pass p;
            p.kind = Pass::MEASURE;
            p.meas = L.meas[m];
            passes->push_back(std::move(p));
        }
    }
}

void place_xcd_qubits(int n, std::vector<Pass> *passes) {
    const uint64_t all = (n >= 64) ? ~uint64_t(0) : ((uint64_t(1) << n) - 1);
    const size_t np = passes->size();
    // for every qubit, the passes whose tile holds it
    std::vector<std::vector<int>> in_tile(static_cast<size_t>(n));
    for (size_t i = 0; i < np; i++) {
        const Pass &p = (*passes)[i];
        const bool tiled = p.kind == Pass::TILE && !p.strided;
        for (int q = 0; q < n; q++)
            if (!tiled || ((p.tile_mask >> q) & 1)) in_tile[size_t(q)].push_back(int(i));
    }
    auto next_in = [&](int q, int after) {
        const auto &v = in_tile[size_t(q)];
        auto it = std::upper_bound(v.begin(), v.end(), after);
        return it == v.end() ? int(np) : *it;
    };
    int prev[3] = {-1, -1, -1};
    for (size_t i = 0; i < np; i++) {
        Pass &p = (*passes)[i];
        if (p.kind != Pass::TILE || p.strided || p.tile_mask == all) {
            prev[0] = prev[1] = prev[2] = -1;
            continue;
        }
        const uint64_t rest = all & ~p.tile_mask;
        const int nx = std::min(3, __builtin_popcountll(rest));
        uint64_t used = 0;
        int cur[3] = {-1, -1, -1};
        for (int j = 0; j < nx; j++)
            if (prev[j] >= 0 && ((rest >> prev[j]) & 1)) {
                cur[j] = prev[j];
                used |= uint64_t(1) << prev[j];
            }
        for (int j = 0; j < nx; j++) {
            if (cur[j] >= 0) continue;
            int best = -1, best_next = -1;
            for (int q = 0; q < n; q++) {
                if (!((rest >> q) & 1) || ((used >> q) & 1)) continue;
                const int nx2 = next_in(q, int(i));
                if (nx2 > best_next) {
                    best_next = nx2;
                    best = q;
                }
            }
            cur[j] = best;
            used |= uint64_t(1) << best;
        }
        p.nxcd = nx;
        for (int j = 0; j < 3; j++) {
            p.xcd_q[j] = uint8_t(j < nx ? cur[j] : 0);
            prev[j] = j < nx ? cur[j] : -1;
        }
    }
}

uint32_t op_present(const Op &o, bool sparse) {
    const int d = o.dim();
    if (!sparse) return (d >= 32) ? 0xffffffffu : ((1u << d) - 1);
    const size_t blk = size_t(d) * d;
    const double tol = 1e-14 * max_abs(o.m.data(), o.m.size());
    uint32_t present = 0;
    for (int b = 0; b < (1 << o.np); b++) {
        uint32_t pb;
        xor_terms(o.m.data() + b * blk, o.k, tol, &pb);
        present |= pb;
    }
    return present ? present : 1u;   // the zero operator keeps one (zero) diagonal
}

void place_positions(int n, const std::vector<Op> &ops, int logt, int max_k, bool first_in_regs,
                     std::vector<Pass> *passes) {
    const uint64_t all = (n >= 64) ? ~uint64_t(0) : ((uint64_t(1) << n) - 1);
    for (Pass &p : *passes) {
        if (!first_in_regs || p.reg || p.kind != Pass::TILE || p.strided || p.tile_mask == all ||
            p.t <= logt || p.ops.empty())
            continue;
        const uint64_t low = (uint64_t(1) << p.c) - 1;
        const int le = std::min(p.t - logt, 4);
        auto tile_qubits = [&](int idx) { return ops[idx].mask() & p.tile_mask; };
        auto fits = [&](int idx, int off) {
            const uint64_t in = tile_qubits(idx);
            return !(in & low) && __builtin_popcountll(in) <= max_k && off + __builtin_popcountll(in) <= le;
        };
        // the first operator: one that commutes with every operator before it
        uint64_t before = 0;
        int pick = -1;
        for (size_t x = 0; x < p.ops.size(); x++) {
            const Op &o = ops[p.ops[x]];
            if (!(o.mask() & before) && fits(p.ops[x], 0)) {
                pick = int(x);
                break;
            }
            before |= o.mask();
        }
        uint64_t first_in = 0;
        int k1 = 0;
        if (pick >= 0) {
            const int idx = p.ops[size_t(pick)];
            p.ops.erase(p.ops.begin() + pick);
            p.ops.insert(p.ops.begin(), idx);
            first_in = tile_qubits(idx);
            k1 = __builtin_popcountll(first_in);
            p.first_in_regs = true;
        }
        // the last operator: one that commutes with every operator after it,
        // its tile qubits disjoint from the first one's
        uint64_t after = 0;
        int lpick = -1;
        for (int x = int(p.ops.size()) - 1; x >= (p.first_in_regs ? 1 : 0); x--) {
            const Op &o = ops[p.ops[size_t(x)]];
            if (!(o.mask() & after) && !(tile_qubits(p.ops[size_t(x)]) & first_in) && fits(p.ops[size_t(x)], k1)) {
                lpick = x;
                break;
            }
            after |= o.mask();
        }
        uint64_t last_in = 0;
        if (lpick >= 0) {
            const int idx = p.ops[size_t(lpick)];
            p.ops.erase(p.ops.begin() + lpick);
            p.ops.push_back(idx);
            last_in = tile_qubits(idx);
            p.last_in_regs = true;
            p.last_off = k1;
        }
        if (!p.first_in_regs && !p.last_in_regs) continue;
        p.seq = p.ops;
        // positions 0..c-1: low qubits; logt..: the first operator's tile
        // qubits, then the last one's; the other tile qubits fill the
        // remaining positions in ascending order
        const int k2 = __builtin_popcountll(last_in);
        int fill[16], nf = 0;
        for (int q = 0; q < n; q++)
            if (((p.tile_mask >> q) & 1) && !((low | first_in | last_in) >> q & 1)) fill[nf++] = q;
        int f = 0, r1 = 0, r2 = 0;
        for (int pos = 0; pos < p.t; pos++) {
            if (pos < p.c) p.tq[pos] = uint8_t(pos);
            else if (pos >= logt && pos < logt + k1) {
                while (!((first_in >> r1) & 1)) r1++;
                p.tq[pos] = uint8_t(r1++);
            } else if (pos >= logt + k1 && pos < logt + k1 + k2) {
                while (!((last_in >> r2) & 1)) r2++;
                p.tq[pos] = uint8_t(r2++);
            } else p.tq[pos] = uint8_t(fill[f++]);
        }
    }
}

uint64_t op_moved_qubits(const Op &o, uint32_t present) {
    uint32_t bits = 0;
    for (int m = 1; m < o.dim(); m++)
        if ((present >> m) & 1) bits |= uint32_t(m);
    uint64_t r = 0;
    for (int j = 0; j < o.k; j++)
        if ((bits >> j) & 1) r |= uint64_t(1) << o.q[j];
    return r;
}

int pack_plan(const std::vector<Op> &ops, const std::vector<uint32_t> &present_of,
              std::vector<Pass> &passes, const PlanConfig &cfg, PackedPlan *out) {
    out->ops.clear();
    out->pass_begin.clear();
    out->coef_begin.clear();
    out->coefs.clear();
    out->op_np.clear();
    out->op_slots.clear();
    out->terms = 0;
    for (Pass &p : passes) {
        out->pass_begin.push_back(uint32_t(out->ops.size()));
        out->coef_begin.push_back(uint32_t(out->coefs.size()));
        if (p.reg) {
            const int rc = pack_reg_pass(ops, present_of, p, cfg.reg_coalesce, out);
            if (rc) return rc;
            continue;
        }
        const std::vector<int> &items = p.seq.empty() ? p.ops : p.seq;
        for (int idx : items) {
            if (idx < 0) {
                const MeasRec &mr = p.inline_meas[~idx];
                DevOp r{};
                r.coef = uint32_t(mr.slot);
                r.present = 0;
                r.k = 1;
                r.pos[0] = uint8_t(mr.q);
                r.kind = uint8_t(mr.kind);
                out->ops.push_back(r);
                out->op_np.push_back(0);
                for (int j = 0; j < 3; j++) out->op_slots.push_back(-1);
                continue;
            }
            const Op &o = ops[idx];
            const int d = o.dim();
            const size_t blk = size_t(d) * d;
            const int nb = 1 << o.np;
            const uint32_t present = present_of[idx];
            // Local bit order of the record: the positions addressed (every
            // qubit for a strided sweep; the tile's qubits in a tiled pass,
            // by ascending tile position), then the block qubits.
            // perm[j'] = the operator's bit at new bit j'.
            int tpos[kMaxK];
            for (int j = 0; j < o.k; j++) {
                tpos[j] = -1;
                if (p.strided) tpos[j] = o.q[j];
                else
                    for (int x = 0; x < p.t && x < 16; x++)
                        if (p.tq[x] == o.q[j]) tpos[j] = x;
            }
            int perm[kMaxK], kin = 0, kx = 0;
            for (int j = 0; j < o.k; j++)
                if (tpos[j] >= 0) perm[kin++] = j;
            for (int a = 1; a < kin; a++)
                for (int b = a; b > 0 && tpos[perm[b]] < tpos[perm[b - 1]]; b--) std::swap(perm[b], perm[b - 1]);
            for (int j = 0; j < o.k; j++)
                if (tpos[j] < 0) perm[kin + kx++] = j;
            auto old_index = [&](int rn) {
                int ro = 0;
                for (int j = 0; j < o.k; j++)
                    if ((rn >> j) & 1) ro |= 1 << perm[j];
                return ro;
            };
            // present shifts in the new order; a shift that moves a block qubit
            // cannot be applied from outside the tile
            uint32_t pres = 0;
            for (int mn = 0; mn < d; mn++) {
                if (!((present >> old_index(mn)) & 1)) continue;
                if (mn >> kin) return QSIM_E_ARG;
                pres |= 1u << mn;
            }
            DevOp r{};
            r.coef = uint32_t(out->coefs.size());
            r.present = pres;
            r.k = uint8_t(kin);
            r.kx = uint8_t(kx);
            r.kind = DEVOP_MAT;
            for (int j = 0; j < kin; j++) r.pos[j] = uint8_t(tpos[perm[j]]);
            for (int j = 0; j < kx; j++) r.xq[j] = uint8_t(o.q[perm[kin + j]]);
            // coefficients: for each basis block b, each block e of the block
            // qubits, each present shift m (ascending), the 2^kin diagonal
            // entries M[r][r ^ m] with r = r_in + 2^kin e
            const int din = 1 << kin;
            for (int b = 0; b < nb; b++)
                for (int e = 0; e < (1 << kx); e++)
                    for (int mn = 0; mn < din; mn++) {
                        if (!((pres >> mn) & 1)) continue;
                        for (int ri = 0; ri < din; ri++) {
                            const int rn = ri | (e << kin);
                            out->coefs.push_back(o.m[b * blk + size_t(old_index(rn)) * d + old_index(rn ^ mn)]);
                        }
                    }
            out->terms += __builtin_popcount(pres);
            out->ops.push_back(r);
            out->op_np.push_back(int8_t(o.np));
            for (int j = 0; j < 3; j++) out->op_slots.push_back(o.slot[j]);
        }
    }
    out->pass_begin.push_back(uint32_t(out->ops.size()));
    out->coef_begin.push_back(uint32_t(out->coefs.size()));
    return QSIM_OK;
}

}  // namespace qs
