// Register programs of tiled passes.
//
// In a register-resident pass each of the 2^(t-4) threads of a workgroup
// holds 16 amplitudes of the tile in registers.  An element of the tile is
// named by its position bits: lane bits 0..5 (the thread's lane), wave bits
// 6..logt-1 (its wave) and register bits logt..logt+3 (which of its 16
// registers).  A layout says which tile qubit each position bit carries.
// An operator is applied where all of its tile qubits are on register bits:
// a thread then holds whole groups of it, and the update of Eq. (1q-op) /
// Eq. (2q-op), generalised to k qubits, runs on registers without any data
// exchange.  Between operators the layout changes in two ways:
//
// * a qubit on lane bit 4 or 5 trades places with a register bit through
//   v_permlane16_swap / v_permlane32_swap: two registers exchange half of
//   their lanes, one instruction per 32-bit word;
// * otherwise the tile goes through LDS once (write in the old layout, read
//   in a new one), and the new layout puts on the register bits the qubits
//   of the operator at hand and then those used soonest after it, on lane
//   bits 4 and 5 the next ones, and the low qubits back on the low lane bits
//   (coalesced global loads and stores).
//
// A qubit an operator is diagonal on may stay outside the tile (a block
// qubit): the tile's base index selects that operator's coefficient block,
// as in the LDS-tiled passes.
#include <algorithm>
#include <cstring>

#include "host.h"

namespace qs {

namespace {

struct Layout {
    int t = 0;
    uint8_t pc[16] = {0};   // canonical tile bit at position p
    uint8_t cp[16] = {0};   // position of canonical bit c
    void set(int p, int c) {
        pc[p] = uint8_t(c);
        cp[c] = uint8_t(p);
    }
};

}  // namespace

int pack_reg_pass(const std::vector<Op> &ops, const std::vector<uint32_t> &present_of, Pass &p,
                  bool coalesce, PackedPlan *out) {
    const int t = p.t;
    const int L = kRegBits;
    const int logt = t - L;
    const int c = p.c;
    if (reg_threads_for(t) == 0 || c > 4 || p.strided || p.kind != Pass::TILE) return QSIM_E_ARG;
    p.reg_logt = logt;
    // canonical bit of each tile qubit (ascending qubits; low qubits 0..c-1
    // are canonical 0..c-1)
    int canon_of[kMaxQubits];
    int qubit_of[16];
    {
        int j = 0;
        for (int q = 0; q < kMaxQubits; q++) {
            canon_of[q] = -1;
            if ((p.tile_mask >> q) & 1) {
                if (j >= 16) return QSIM_E_ARG;
                canon_of[q] = j;
                qubit_of[j++] = q;
            }
        }
        if (j != t) return QSIM_E_ARG;
        for (int q = 0; q < c; q++)
            if (canon_of[q] != q) return QSIM_E_ARG;
    }
    const std::vector<int> &seq = p.ops;
    const size_t N = seq.size();
    std::vector<uint32_t> need(N);
    for (size_t i = 0; i < N; i++) {
        const Op &o = ops[seq[i]];
        uint32_t m = 0;
        for (int j = 0; j < o.k; j++)
            if (canon_of[o.q[j]] >= 0) m |= 1u << canon_of[o.q[j]];
        if (__builtin_popcount(m) > L) return QSIM_E_ARG;
        need[i] = m;
    }
    // uses[c]: ascending operator indices that need canonical bit c
    std::vector<std::vector<int>> uses(t);
    for (size_t i = 0; i < N; i++)
        for (int b = 0; b < t; b++)
            if ((need[i] >> b) & 1) uses[b].push_back(int(i));
    auto next_use = [&](int b, size_t after) {
        auto it = std::upper_bound(uses[b].begin(), uses[b].end(), int(after) - 1);
        return it == uses[b].end() ? int(N) + 1 : *it;
    };
    const uint32_t lowmask = (1u << c) - 1;
    const int near[2] = {4, 5};

    // A layout for the operators from i on: `must` on register bits, then
    // the tile qubits (other than the low ones) used soonest; lane bits 4, 5
    // next; the low qubits not on register bits on their own lane bits.
    auto build = [&](size_t i, uint32_t must) {
        Layout l;
        l.t = t;
        uint32_t placed = 0;
        bool pos_used[16] = {false};
        std::vector<std::pair<int, int>> cand;
        for (int b = 0; b < t; b++)
            if (!((must >> b) & 1) && !((lowmask >> b) & 1)) cand.push_back({next_use(b, i), b});
        std::stable_sort(cand.begin(), cand.end());
        size_t ci = 0;
        uint32_t regset = must;
        while (__builtin_popcount(regset) < L && ci < cand.size()) regset |= 1u << cand[ci++].second;
        int rp = logt;
        for (int b = 0; b < t; b++)
            if ((regset >> b) & 1) {
                l.set(rp, b);
                pos_used[rp++] = true;
                placed |= 1u << b;
            }
        for (int k = 0; k < 2 && ci < cand.size(); k++) {
            const int b = cand[ci++].second;
            l.set(near[k], b);
            pos_used[near[k]] = true;
            placed |= 1u << b;
        }
        for (int b = 0; b < c; b++)
            if (!((placed >> b) & 1) && !pos_used[b]) {
                l.set(b, b);
                pos_used[b] = true;
                placed |= 1u << b;
            }
        int pp = 0;
        for (int b = 0; b < t; b++) {
            if ((placed >> b) & 1) continue;
            while (pos_used[pp]) pp++;
            l.set(pp, b);
            pos_used[pp] = true;
            placed |= 1u << b;
        }
        return l;
    };
    auto coalesced = [&](const Layout &l) {
        for (int b = 0; b < c; b++)
            if (l.pc[b] != b) return false;
        return true;
    };
    auto push_rec = [&](const DevOp &r) {
        out->ops.push_back(r);
        out->op_np.push_back(0);
        for (int j = 0; j < 3; j++) out->op_slots.push_back(-1);
    };
    auto push_xpose = [&](const Layout &from, const Layout &to) {
        DevOp a{}, b{};
        unsigned char *pa = reinterpret_cast<unsigned char *>(&a);
        unsigned char *pb = reinterpret_cast<unsigned char *>(&b);
        for (int x = 0; x < t; x++) {
            pa[x] = from.pc[x];
            pb[x] = to.pc[x];
        }
        a.kind = DEVOP_XPOSE;
        b.kind = DEVOP_XPOSE2;
        push_rec(a);
        push_rec(b);
        p.reg_xposes++;
    };
    auto is_reg = [&](int pos) { return pos >= logt; };

    Layout cur = build(0, N ? (need[0] & ~lowmask) : 0);
    for (int x = 0; x < t; x++) p.load_pos[x] = cur.pc[x];
    for (size_t i = 0; i < N; i++) {
        uint32_t miss = 0;
        for (int b = 0; b < t; b++)
            if (((need[i] >> b) & 1) && !is_reg(cur.cp[b])) miss |= 1u << b;
        if (miss) {
            bool swappable = true;
            for (int b = 0; b < t; b++)
                if (((miss >> b) & 1) && cur.cp[b] != 4 && cur.cp[b] != 5) swappable = false;
            if (swappable) {
                for (int b = 0; b < t; b++) {
                    if (!((miss >> b) & 1)) continue;
                    // victim: the register qubit not needed now whose next use is furthest
                    int vic = -1, best = -1;
                    for (int rp = logt; rp < t; rp++) {
                        const int vb = cur.pc[rp];
                        if ((need[i] >> vb) & 1) continue;
                        const int nu = next_use(vb, i + 1);
                        if (nu > best) {
                            best = nu;
                            vic = rp;
                        }
                    }
                    if (vic < 0) return QSIM_E_ARG;
                    const int lp = cur.cp[b], vb = cur.pc[vic];
                    cur.set(lp, vb);
                    cur.set(vic, b);
                    DevOp r{};
                    r.kind = DEVOP_SWAP;
                    r.pos[0] = uint8_t(lp);
                    r.pos[1] = uint8_t(vic - logt);
                    push_rec(r);
                    p.reg_swaps++;
                }
            } else {
                const Layout nl = build(i, need[i]);
                push_xpose(cur, nl);
                cur = nl;
            }
        }
        // the operator on the register bits of the current layout
        const Op &o = ops[seq[i]];
        const uint32_t present = present_of[seq[i]];
        const int d = o.dim();
        int rb[kMaxK], kin = 0, kx = 0, tile_j[kMaxK], blk_j[kMaxK];
        for (int j = 0; j < o.k; j++) {
            const int cb = canon_of[o.q[j]];
            if (cb >= 0) {
                if (!is_reg(cur.cp[cb])) return QSIM_E_ARG;
                tile_j[kin] = j;
                rb[kin++] = cur.cp[cb] - logt;
            } else {
                blk_j[kx++] = j;
            }
        }
        // compact shifts must not move block qubits; map each to its
        // register shift
        uint32_t pres_r = 0;
        int m_of_M[1 << kRegBits];
        for (int M = 0; M < (1 << L); M++) m_of_M[M] = -1;
        for (int m = 0; m < d; m++) {
            if (!((present >> m) & 1)) continue;
            int M = 0;
            for (int x = 0; x < kx; x++)
                if ((m >> blk_j[x]) & 1) return QSIM_E_ARG;
            for (int x = 0; x < kin; x++)
                if ((m >> tile_j[x]) & 1) M |= 1 << rb[x];
            pres_r |= 1u << M;
            m_of_M[M] = m;
        }
        DevOp r{};
        r.kind = DEVOP_RMAT;
        r.coef = uint32_t(out->coefs.size());
        r.present = pres_r;
        r.k = uint8_t(L);
        r.kx = uint8_t(kx);
        for (int x = 0; x < kx; x++) r.xq[x] = uint8_t(o.q[blk_j[x]]);
        const size_t blk = size_t(d) * d;
        for (int b = 0; b < (1 << o.np); b++)
            for (int e = 0; e < (1 << kx); e++)
                for (int M = 0; M < (1 << L); M++) {
                    if (!((pres_r >> M) & 1)) continue;
                    const int m = m_of_M[M];
                    for (int rr = 0; rr < (1 << L); rr++) {
                        int rl = 0;
                        for (int x = 0; x < kin; x++)
                            if ((rr >> rb[x]) & 1) rl |= 1 << tile_j[x];
                        for (int x = 0; x < kx; x++)
                            if ((e >> x) & 1) rl |= 1 << blk_j[x];
                        out->coefs.push_back(o.m[b * blk + size_t(rl) * d + size_t(rl ^ m)]);
                    }
                }
        out->terms += __builtin_popcount(pres_r);
        out->ops.push_back(r);
        out->op_np.push_back(int8_t(o.np));
        for (int j = 0; j < 3; j++) out->op_slots.push_back(o.slot[j]);
    }
    if (coalesce && !coalesced(cur)) {
        Layout nl = build(N, 0);
        push_xpose(cur, nl);
        cur = nl;
    }
    for (int x = 0; x < t; x++) p.store_pos[x] = cur.pc[x];
    for (int x = 0; x < 16; x++) p.tq[x] = x < t ? uint8_t(qubit_of[x]) : 0;
    return QSIM_OK;
}

}  // namespace qs
