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
// it shares one of its qubits.
#include <algorithm>
#include <cmath>

#include "host.h"

namespace qs {

void plan_passes(int n, const std::vector<Op> &ops, const std::vector<int> &fence_after,
                 const std::vector<uint32_t> &meta_bytes, const PlanConfig &cfg,
                 std::vector<Pass> *passes) {
    passes->clear();
    const int N = int(ops.size());
    if (N == 0) return;
    const int t = std::min(cfg.tile_qubits, n);
    const int c = std::min(cfg.low_qubits, t);
    const uint64_t all = (n >= 64) ? ~uint64_t(0) : ((uint64_t(1) << n) - 1);
    const uint64_t low = (uint64_t(1) << c) - 1;

    // fences split the list into independent segments
    std::vector<int> seg_end;
    {
        std::vector<int> f = fence_after;
        std::sort(f.begin(), f.end());
        for (int x : f)
            if (x >= 0 && x < N - 1 && (seg_end.empty() || seg_end.back() != x + 1)) seg_end.push_back(x + 1);
        seg_end.push_back(N);
    }

    auto finish = [&](uint64_t T, std::vector<int> &&sel, bool strided) {
        Pass p;
        p.strided = strided;
        if (!strided) {
            // pad the tile to exactly t qubits with the lowest unused qubits
            for (int q = 0; q < n && __builtin_popcountll(T) < t; q++) T |= uint64_t(1) << q;
            p.t = t;
            p.c = c;
            p.tile_mask = T;
            for (int q = c; q < n; q++)
                if ((T >> q) & 1) p.hi[p.nhi++] = q;
        }
        p.ops = std::move(sel);
        passes->push_back(std::move(p));
    };

    if (cfg.one_op_per_pass) {
        for (int i = 0; i < N; i++) finish(0, {i}, true);
        return;
    }
    if (t >= n) {
        // the whole state fits one tile: one pass per segment, with operators
        // too wide for the tile kernel as sweeps of their own
        int b = 0;
        for (int e : seg_end) {
            std::vector<int> sel;
            size_t meta = 0;
            for (int i = b; i < e; i++) {
                if (ops[i].k > cfg.max_tile_k) {
                    if (!sel.empty()) finish(all, std::move(sel), false);
                    sel.clear();
                    meta = 0;
                    finish(0, {i}, true);
                    continue;
                }
                if (!sel.empty() && meta + meta_bytes[i] > cfg.meta_budget) {
                    finish(all, std::move(sel), false);
                    sel.clear();
                    meta = 0;
                }
                sel.push_back(i);
                meta += meta_bytes[i];
            }
            if (!sel.empty()) finish(all, std::move(sel), false);
            b = e;
        }
        return;
    }

    // doubly linked list of pending operators
    std::vector<int> nxt(N + 1), prv(N + 1);
    int seg_begin = 0;
    for (int e : seg_end) {
        // list over [seg_begin, e): head sentinel = N
        int head = N;
        nxt[head] = seg_begin < e ? seg_begin : head;
        prv[head] = e - 1 >= seg_begin ? e - 1 : head;
        for (int i = seg_begin; i < e; i++) {
            nxt[i] = (i + 1 < e) ? i + 1 : head;
            prv[i] = (i > seg_begin) ? i - 1 : head;
        }
        while (nxt[head] != head) {
            const int first = nxt[head];
            if (ops[first].k > cfg.max_tile_k) {
                // too wide for the tile kernel at this precision: its own sweep
                nxt[head] = nxt[first];
                prv[nxt[first]] = head;
                finish(0, {first}, true);
                continue;
            }
            uint64_t T = low, blocked = 0;
            std::vector<int> sel;
            size_t meta = 0;
            int scanned = 0;
            for (int i = nxt[head]; i != head && scanned < cfg.window; i = nxt[i], scanned++) {
                uint64_t qm = ops[i].mask();
                if ((qm & blocked) || ops[i].k > cfg.max_tile_k ||
                    (!sel.empty() && meta + meta_bytes[i] > cfg.meta_budget)) {
                    blocked |= qm;
                } else if (__builtin_popcountll(T | qm) <= t) {
                    T |= qm;
                    sel.push_back(i);
                    meta += meta_bytes[i];
                } else {
                    blocked |= qm;
                }
                if (blocked == all) break;
            }
            for (int i : sel) {
                nxt[prv[i]] = nxt[i];
                prv[nxt[i]] = prv[i];
            }
            finish(T, std::move(sel), false);
        }
        seg_begin = e;
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

void pack_plan(const std::vector<Op> &ops, const std::vector<uint32_t> &present_of,
               const std::vector<Pass> &passes, PackedPlan *out) {
    out->ops.clear();
    out->pass_begin.clear();
    out->coef_begin.clear();
    out->coefs.clear();
    out->terms = 0;
    for (const Pass &p : passes) {
        out->pass_begin.push_back(uint32_t(out->ops.size()));
        out->coef_begin.push_back(uint32_t(out->coefs.size()));
        for (int idx : p.ops) {
            const Op &o = ops[idx];
            const int d = o.dim();
            const size_t blk = size_t(d) * d;
            const int nb = 1 << o.np;
            const uint32_t present = present_of[idx];
            DevOp r{};
            r.coef = uint32_t(out->coefs.size());
            r.present = present;
            r.k = uint8_t(o.k);
            r.kind = DEVOP_MAT;
            for (int j = 0; j < o.k; j++) {
                int pos = o.q[j];
                if (!p.strided) {
                    // rank of qubit q[j] among the tile qubits
                    if (pos >= p.c) {
                        int rnk = p.c;
                        for (int h = 0; h < p.nhi && p.hi[h] < o.q[j]; h++) rnk++;
                        pos = rnk;
                    }
                }
                r.pos[j] = uint8_t(pos);
            }
            // coefficients: for each basis block, for each present shift m (ascending),
            // the 2^k diagonal entries M[r][r ^ m], r = 0..2^k-1
            for (int b = 0; b < nb; b++)
                for (int m = 0; m < d; m++) {
                    if (!((present >> m) & 1)) continue;
                    for (int row = 0; row < d; row++)
                        out->coefs.push_back(o.m[b * blk + size_t(row) * d + (row ^ m)]);
                }
            out->terms += __builtin_popcount(present);
            out->ops.push_back(r);
        }
    }
    out->pass_begin.push_back(uint32_t(out->ops.size()));
    out->coef_begin.push_back(uint32_t(out->coefs.size()));
}

}  // namespace qs
