// C ABI of the simulator (include/qsim.h): state handles, the compile ->
// upload -> launch path of qsim_apply, and the measurement / observable
// calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <new>

#include "host.h"
#include "launch.h"
#include "runtime.h"
#include "swizzle.h"

using namespace qs;

namespace {
thread_local char g_last_error[256] = "";
}

namespace qk {
int note_hip(hipError_t e, const char *where) {
    if (e == hipSuccess) return QSIM_OK;
    std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s (%d)", where, hipGetErrorString(e), int(e));
    return QSIM_E_HIP;
}
}  // namespace qk

namespace qs {

std::atomic<int> g_alloc_countdown{-1};

bool alloc_fault() {
    int v = g_alloc_countdown.load();
    while (v >= 0) {
        if (g_alloc_countdown.compare_exchange_weak(v, v - 1)) return v == 0;
    }
    return false;
}

}  // namespace qs

namespace qs {

size_t elem_bytes(int dtype) { return dtype == QSIM_C64 ? 8 : 16; }

int env_int(const char *name, int dflt) {
    const char *v = std::getenv(name);
    return (v && *v) ? std::atoi(v) : dflt;
}

int resident_max(int dtype) {
    // the whole state in one workgroup's LDS (128 KiB of the 160 KiB)
    return dtype == QSIM_C64 ? 14 : 13;
}

// 12-qubit tiles while a pass gives each CU at most a few of them; complex64
// passes with many tiles (2,048 or more 12-qubit tiles over all the states
// the pass covers: one state of 23+ qubits, or a batch of smaller ones) take
// 13-qubit tiles: several tiles are then queued per CU, so loads, operators
// and stores of different tiles overlap, and the larger tiles carry more
// operators per pass
int default_tile_qubits(int n, int dtype, uint64_t nstates) {
    const bool many = dtype == QSIM_C64 && n > 12 && (nstates << (n - 12)) >= 2048;
    return env_int("QSIM_TILE_QUBITS", many ? 13 : 12);
}

void default_configs(int n, int dtype, const qsim_fuse_opts *opt, FuseConfig *fc, PlanConfig *pc) {
    fc->level = 5;
    fc->max_width = 4;
    fc->sparse = true;
    fc->max_params = 0;
    pc->one_op_per_pass = false;
    pc->tile_qubits = default_tile_qubits(n, dtype, 1);
    pc->low_qubits = env_int("QSIM_LOW_QUBITS", dtype == QSIM_C64 ? 4 : 3);
    pc->window = env_int("QSIM_PLAN_WINDOW", 1024);
    pc->max_tile_k = 4;
    // complex64 tiles use 512 threads; complex128 tiles 256, whose groups of
    // 16 outputs then fit the registers without chunking
    pc->threads = env_int("QSIM_TILE_THREADS", dtype == QSIM_C64 ? 512 : 256) == 256 ? 256 : 512;
    pc->first_in_regs = env_int("QSIM_FIRST_IN_REGS", 1) != 0;
    pc->reg_engine = env_int("QSIM_REG_ENGINE", 0) != 0;
    pc->reg_coalesce = env_int("QSIM_REG_COALESCE", 1) != 0;
    pc->xcd_order = env_int("QSIM_XCD_ORDER", 1) != 0;
    if (opt) {
        if (opt->level >= 0 && opt->level <= 5) fc->level = opt->level;
        if (opt->max_width > 0) fc->max_width = opt->max_width;
        if (opt->tile_qubits > 0) pc->tile_qubits = opt->tile_qubits;
        if (opt->low_qubits > 0) pc->low_qubits = opt->low_qubits;
        pc->one_op_per_pass = (opt->flags & QSIM_F_ONE_OP_PER_PASS) != 0;
        fc->sparse = (opt->flags & QSIM_F_NO_SPARSE) == 0;
        pc->full_support = (opt->flags & QSIM_F_FULL_SUPPORT) != 0;
        if (opt->flags & QSIM_F_REG_ENGINE) pc->reg_engine = true;
    }
    if (dtype == QSIM_C128) fc->max_width = std::min(fc->max_width, 4);
    fc->max_width = std::max(1, std::min(fc->max_width, kMaxK));
    fc->lds_cost = pc->one_op_per_pass ? 64.0 : 3.0;
    if (const char *v = std::getenv("QSIM_LDS_COST")) fc->lds_cost = std::atof(v);
    if (opt && opt->op_cost > 0.0f) fc->lds_cost = opt->op_cost;
    if (!opt || opt->max_width <= 0) fc->max_width = env_int("QSIM_MAX_WIDTH", fc->max_width);
    if (dtype == QSIM_C128) fc->max_width = std::min(fc->max_width, 4);
    fc->max_width = std::max(1, std::min(fc->max_width, kMaxK));
    pc->tile_qubits = std::max(6, std::min(pc->tile_qubits, resident_max(dtype)));
    if (n <= resident_max(dtype)) pc->tile_qubits = n;
    if (pc->tile_qubits > n) pc->tile_qubits = n;
    pc->low_qubits = std::max(0, std::min(pc->low_qubits, pc->tile_qubits - 1));
    // LDS behind the tile (and its reduction scratch) for a pass's records and
    // coefficients: as much as fits without lowering the number of workgroups
    // a CU holds at once, which the tile's LDS and the tile kernel's
    // registers set (two workgroups; four for complex64 tiles of 256
    // threads).  QSIM_META_BUDGET caps it.
    const size_t tile_bytes = (size_t(1) << pc->tile_qubits) * elem_bytes(dtype) + qk::kTileRedBytes;
    const size_t lds = qk::max_lds_bytes();
    const size_t by_regs = (dtype == QSIM_C64 && pc->threads == 256) ? 4 : 2;
    const size_t per_cu = std::max<size_t>(1, std::min(tile_bytes <= lds ? lds / tile_bytes : 0, by_regs));
    const size_t room = lds / per_cu > tile_bytes ? lds / per_cu - tile_bytes : 0;
    pc->meta_budget = std::min(room, size_t(std::max(1024, env_int("QSIM_META_BUDGET", 1 << 30))));
}

// The XCD-order qubits of a tiled pass: distinct qubits outside the tile.
bool xcd_ok(uint64_t rest, int nx, const uint8_t *xq) {
    if (nx < 0 || nx > 3 || nx > __builtin_popcountll(rest)) return false;
    uint64_t seen = 0;
    for (int j = 0; j < nx; j++) {
        if (xq[j] >= 64 || !((rest >> xq[j]) & 1) || ((seen >> xq[j]) & 1)) return false;
        seen |= uint64_t(1) << xq[j];
    }
    return true;
}

// A register-resident pass: tile qubits partition the n qubits, layouts are
// permutations of the tile positions, every record is well formed, the
// re-layout records name the layout the swaps and re-layouts before them
// leave (so the kernel's LDS writes are a permutation of the tile), and
// coefficient ranges lie inside the pass's share of the table.
int validate_reg_pass(int n, int dtype, const Compiled &c, size_t i) {
    const PackedPlan &p = c.plan;
    const PassInfo &pi = c.passes[i];
    const qk::RegArgs &ra = pi.ra;
    const int t = ra.t;
    const uint64_t all = (n >= 64) ? ~uint64_t(0) : ((uint64_t(1) << n) - 1);
    if (pi.strided || pi.kind != Pass::TILE || ra.n != n || reg_threads_for(t) == 0 || t >= n || n - t > 31)
        return QSIM_E_ARG;
    const uint32_t nrec = p.pass_begin[i + 1] - p.pass_begin[i];
    bool any_xpose = false;
    for (uint32_t j = p.pass_begin[i]; j < p.pass_begin[i + 1] && j < p.ops.size(); j++)
        any_xpose |= p.ops[j].kind == DEVOP_XPOSE;
    if (size_t(ra.lds_bytes) != qk::reg_lds_bytes(elem_bytes(dtype), t, any_xpose, nrec) ||
        ra.lds_bytes > qk::max_lds_bytes())
        return QSIM_E_ARG;
    if (ra.flags & ~uint32_t(qk::RF_NONTEMPORAL)) return QSIM_E_ARG;
    uint64_t tile = 0;
    for (int j = 0; j < t; j++) {
        if (ra.tq[j] >= n || (j && ra.tq[j] <= ra.tq[j - 1])) return QSIM_E_ARG;
        tile |= uint64_t(1) << ra.tq[j];
    }
    if ((tile & ra.rest_mask) || ((tile | ra.rest_mask) != all)) return QSIM_E_ARG;
    if (!xcd_ok(ra.rest_mask, ra.nxcd, ra.xcd_q)) return QSIM_E_ARG;
    auto is_perm = [&](const uint8_t *pos) {
        uint32_t seen = 0;
        for (int x = 0; x < t; x++) {
            if (pos[x] >= t || ((seen >> pos[x]) & 1)) return false;
            seen |= 1u << pos[x];
        }
        return true;
    };
    if (!is_perm(ra.load_pos) || !is_perm(ra.store_pos)) return QSIM_E_ARG;
    const uint32_t rb = p.pass_begin[i], re = p.pass_begin[i + 1];
    if (rb > re || re > p.ops.size() || p.coef_begin[i] > p.coef_begin[i + 1] ||
        p.coef_begin[i + 1] > p.coefs.size())
        return QSIM_E_ARG;
    const int logt = t - kRegBits;
    uint8_t cur[16];
    std::memcpy(cur, ra.load_pos, 16);
    for (uint32_t j = rb; j < re; j++) {
        const DevOp &o = p.ops[j];
        if (o.kind == DEVOP_RMAT) {
            if (o.k != kRegBits || o.kx > kMaxK || !o.present || (o.present >> (1 << kRegBits))) return QSIM_E_ARG;
            for (int a = 0; a < o.kx; a++) {
                if (o.xq[a] >= n || ((tile >> o.xq[a]) & 1)) return QSIM_E_ARG;
                if (a && o.xq[a] <= o.xq[a - 1]) return QSIM_E_ARG;
            }
            if (p.op_np[j] < 0 || p.op_np[j] > 3) return QSIM_E_ARG;
            const size_t need = size_t(o.coef) + size_t(devop_coefs(o)) * (size_t(1) << p.op_np[j]);
            if (o.coef < p.coef_begin[i] || need > p.coef_begin[i + 1]) return QSIM_E_ARG;
        } else if (o.kind == DEVOP_SWAP) {
            if ((o.pos[0] != 4 && o.pos[0] != 5) || o.pos[1] >= kRegBits) return QSIM_E_ARG;
            std::swap(cur[o.pos[0]], cur[logt + o.pos[1]]);
        } else if (o.kind == DEVOP_XPOSE) {
            if (j + 1 >= re || p.ops[j + 1].kind != DEVOP_XPOSE2) return QSIM_E_ARG;
            const uint8_t *from = reinterpret_cast<const uint8_t *>(&o);
            const uint8_t *to = reinterpret_cast<const uint8_t *>(&p.ops[j + 1]);
            if (!is_perm(from) || !is_perm(to) || std::memcmp(from, cur, size_t(t)) != 0) return QSIM_E_ARG;
            std::memcpy(cur, to, size_t(t));
            j++;
        } else {
            return QSIM_E_ARG;
        }
    }
    if (std::memcmp(cur, ra.store_pos, size_t(t)) != 0) return QSIM_E_ARG;
    return QSIM_OK;
}

// Check, before anything is launched, that every device record stays inside
// the buffers and tiles the kernels will index: tile qubits partition the n
// qubits, operator positions are ascending and inside the tile (or the
// state), and coefficient ranges lie inside the coefficient table.
int validate_plan(int n, int dtype, const Compiled &c) {
    const PackedPlan &p = c.plan;
    if (p.pass_begin.size() != c.passes.size() + 1 || p.coef_begin.size() != c.passes.size() + 1)
        return QSIM_E_ARG;
    const uint64_t all = (n >= 64) ? ~uint64_t(0) : ((uint64_t(1) << n) - 1);
    for (size_t i = 0; i < c.passes.size(); i++) {
        const PassInfo &pi = c.passes[i];
        int width = n;
        if (pi.reg) {
            const int rc = validate_reg_pass(n, dtype, c, i);
            if (rc) return rc;
            continue;
        }
        if (pi.kind == Pass::MEASURE) {
            if (p.pass_begin[i] != p.pass_begin[i + 1] || pi.meas.q < 0 || pi.meas.q >= n ||
                !devop_is_record(pi.meas.kind))
                return QSIM_E_ARG;
            continue;
        }
        if (!pi.strided) {
            const qk::TileArgs &ta = pi.ta;
            if (ta.n != n || ta.t < 1 || ta.t > n || ta.t > resident_max(dtype) || ta.c < 0 ||
                ta.c > ta.t || ta.nhi != ta.t - ta.c || n - ta.t > 31)
                return QSIM_E_ARG;
            uint64_t m = (uint64_t(1) << ta.c) - 1;
            int prev = ta.c - 1;
            for (int h = 0; h < ta.nhi; h++) {
                if (ta.hi[h] <= prev || ta.hi[h] >= n) return QSIM_E_ARG;
                prev = ta.hi[h];
                m |= uint64_t(1) << ta.hi[h];
            }
            if ((m & ta.rest_mask) || ((m | ta.rest_mask) != all) || m != ta.tile_mask) return QSIM_E_ARG;
            if (!xcd_ok(ta.rest_mask, ta.nxcd, ta.xcd_q)) return QSIM_E_ARG;
            // tile positions: the low qubits first, then every other tile
            // qubit once
            uint64_t mq = 0;
            for (int j = 0; j < ta.t; j++) {
                if (j < ta.c && ta.tq[j] != j) return QSIM_E_ARG;
                if (ta.tq[j] >= n || ((mq >> ta.tq[j]) & 1)) return QSIM_E_ARG;
                mq |= uint64_t(1) << ta.tq[j];
            }
            if (mq != ta.tile_mask) return QSIM_E_ARG;
            if (ta.regs) {
                // operators run on a thread's registers: their tile positions
                // are consecutive register-index bits (log2(threads) + off + j)
                const int logt = ta.threads == 512 ? 9 : 8;
                const uint32_t rb = p.pass_begin[i], re = p.pass_begin[i + 1];
                const int first = ta.regs & 1, last = (ta.regs >> 1) & 1, off = (ta.regs >> 2) & 7;
                if ((ta.regs >> 5) || ta.t <= logt || ta.t >= n || re - rb < uint32_t(first + last)) return QSIM_E_ARG;
                const int le = std::min(ta.t - logt, 4);
                auto check_regs = [&](const DevOp &o, int at) {
                    if (o.kind != DEVOP_MAT || o.k > first_regs_max_k(dtype) || at + o.k > le) return false;
                    for (int a2 = 0; a2 < o.k; a2++)
                        if (o.pos[a2] != logt + at + a2) return false;
                    return true;
                };
                if (first && !check_regs(p.ops[rb], 0)) return QSIM_E_ARG;
                if (last && (!check_regs(p.ops[re - 1], off) || off != (first ? int(p.ops[rb].k) : 0)))
                    return QSIM_E_ARG;
                if (!last && off) return QSIM_E_ARG;
            }
            width = ta.t;
        }
        if (p.pass_begin[i] > p.pass_begin[i + 1] || p.pass_begin[i + 1] > p.ops.size()) return QSIM_E_ARG;
        if (p.coef_begin[i] > p.coef_begin[i + 1] || p.coef_begin[i + 1] > p.coefs.size()) return QSIM_E_ARG;
        if (!pi.strided &&
            qk::tile_lds_bytes(elem_bytes(dtype), pi.ta.t, p.pass_begin[i + 1] - p.pass_begin[i],
                               p.coef_begin[i + 1] - p.coef_begin[i]) > qk::max_lds_bytes())
            return QSIM_E_ARG;
        for (uint32_t j = p.pass_begin[i]; j < p.pass_begin[i + 1]; j++) {
            const DevOp &o = p.ops[j];
            if (o.kind != DEVOP_MAT) {
                // measurement records run only inside resident (whole-state) passes
                if (pi.strided || pi.ta.t != n || o.pos[0] >= n || !devop_is_record(o.kind)) return QSIM_E_ARG;
                continue;
            }
            // tiled passes may hold operators with block qubits (kx > 0),
            // which must lie outside the tile; k = 0 then is an operator
            // diagonal on all its qubits
            if (pi.strided ? (o.kx != 0 || o.k < 1) : (o.k + o.kx < 1)) return QSIM_E_ARG;
            if (o.k > width || o.k + o.kx > kMaxK) return QSIM_E_ARG;
            if (!pi.strided && o.k > 4) return QSIM_E_ARG;
            for (int a = 0; a < o.k; a++) {
                if (o.pos[a] >= width) return QSIM_E_ARG;
                if (a && o.pos[a] <= o.pos[a - 1]) return QSIM_E_ARG;
                if (!pi.strided && o.slot[a] != lds_slot(int(elem_bytes(dtype)), 1 << o.pos[a])) return QSIM_E_ARG;
            }
            for (int a = 0; a < o.kx; a++) {
                if (o.xq[a] >= n || ((pi.ta.tile_mask >> o.xq[a]) & 1)) return QSIM_E_ARG;
                if (a && o.xq[a] <= o.xq[a - 1]) return QSIM_E_ARG;
            }
            const uint32_t d = 1u << o.k;
            const uint32_t mask = (d >= 32) ? 0xffffffffu : ((1u << d) - 1);
            if (!o.present || (o.present & ~mask)) return QSIM_E_ARG;
            const size_t need = size_t(o.coef) + size_t(devop_coefs(o)) * (size_t(1) << p.op_np[j]);
            if (need > p.coefs.size()) return QSIM_E_ARG;
            if (!pi.strided && (o.coef < p.coef_begin[i] || need > p.coef_begin[i + 1])) return QSIM_E_ARG;
            if (p.op_np[j] < 0 || p.op_np[j] > 3) return QSIM_E_ARG;
        }
    }
    return QSIM_OK;
}

int compile_circuit(int n, int dtype, const qsim_gate *g, size_t ng, const GateInputs &in,
                    const qsim_fuse_opts *opt, Compiled *out) {
    return compile_program(n, dtype, g, ng, in, false, false, 0, opt, out);
}

int compile_program(int n, int dtype, const qsim_gate *g, size_t ng, const GateInputs &in,
                    bool keep_params, bool allow_meas, int max_params,
                    const qsim_fuse_opts *opt, Compiled *out) {
    TraceRange range("qsim.compile");
    double t0 = now_seconds();
    if (alloc_fault()) throw std::bad_alloc();
    FuseConfig fc;
    PlanConfig pc;
    default_configs(n, dtype, opt, &fc, &pc);
    fc.max_params = keep_params ? std::max(1, std::min(max_params, 3)) : 0;
    Lowered L;
    int rc;
    {
        TraceRange r("qsim.lower");
        rc = lower(n, g, ng, in, keep_params, allow_meas, &L);
    }
    if (rc) return rc;
    int64_t counts[6];
    {
        TraceRange r("qsim.fuse");
        fuse(n, &L, fc, counts);
    }
    TraceRange plan_range("qsim.plan");
    std::vector<uint32_t> present(L.ops.size()), meta(L.ops.size());
    for (size_t i = 0; i < L.ops.size(); i++) {
        present[i] = op_present(L.ops[i], fc.sparse);
        // LDS holds the bound (per-state) coefficients: no cos/sin blocks
        meta[i] = uint32_t(sizeof(DevOp) + size_t(__builtin_popcount(present[i])) *
                                               L.ops[i].dim() * elem_bytes(dtype));
    }
    std::vector<uint64_t> need(L.ops.size());
    for (size_t i = 0; i < L.ops.size(); i++)
        need[i] = pc.full_support ? L.ops[i].mask() : op_moved_qubits(L.ops[i], present[i]);
    std::vector<Pass> passes;
    plan_passes(n, L, meta, need, pc, &passes);
    // tiled passes of 10..13 qubits (not whole-state ones, which may hold
    // measurement records) run register-resident
    for (Pass &p : passes)
        p.reg = pc.reg_engine && p.kind == Pass::TILE && !p.strided && p.t < n && reg_threads_for(p.t) > 0 &&
                p.c <= 4 && p.inline_meas.empty();
    place_positions(n, L.ops, pc.threads == 512 ? 9 : 8, first_regs_max_k(dtype), pc.first_in_regs, &passes);
    if (pc.xcd_order) place_xcd_qubits(n, &passes);
    rc = pack_plan(L.ops, present, passes, pc, &out->plan);
    if (rc) return rc;
    // LDS slot offsets of the tile positions (the tile kernel's layout)
    for (size_t i = 0; i < passes.size(); i++) {
        if (passes[i].strided || passes[i].kind != Pass::TILE) continue;
        for (uint32_t j = out->plan.pass_begin[i]; j < out->plan.pass_begin[i + 1]; j++) {
            DevOp &o = out->plan.ops[j];
            if (o.kind != DEVOP_MAT) continue;
            for (int a = 0; a < o.k; a++) o.slot[a] = uint16_t(lds_slot(int(elem_bytes(dtype)), 1 << o.pos[a]));
        }
    }
    out->passes.clear();
    out->passes.reserve(passes.size());
    for (const Pass &p : passes) {
        PassInfo pi;
        pi.kind = p.kind;
        pi.meas = p.meas;
        pi.strided = p.strided;
        pi.ta.n = n;
        pi.ta.t = p.t;
        pi.ta.c = p.c;
        pi.ta.nhi = p.nhi;
        uint64_t all = (n >= 64) ? ~uint64_t(0) : ((uint64_t(1) << n) - 1);
        pi.ta.rest_mask = all & ~p.tile_mask;
        pi.ta.tile_mask = p.tile_mask;
        pi.ta.threads = pc.threads;
        pi.ta.regs = (p.first_in_regs ? 1 : 0) | (p.last_in_regs ? 2 : 0) | (p.last_off << 2);
        for (int h = 0; h < p.nhi; h++) pi.ta.hi[h] = uint8_t(p.hi[h]);
        for (int j = 0; j < 16; j++) pi.ta.tq[j] = p.tq[j];
        pi.ta.nxcd = p.nxcd;
        for (int j = 0; j < 4; j++) pi.ta.xcd_q[j] = p.xcd_q[j];
        if (p.reg) {
            pi.ra.nxcd = p.nxcd;
            for (int j = 0; j < 4; j++) pi.ra.xcd_q[j] = p.xcd_q[j];
            pi.reg = true;
            pi.ra.rest_mask = pi.ta.rest_mask;
            pi.ra.n = n;
            pi.ra.t = p.t;
            pi.ra.lds_bytes = uint32_t(qk::reg_lds_bytes(elem_bytes(dtype), p.t, p.reg_xposes > 0,
                                                         out->plan.pass_begin[out->passes.size() + 1] -
                                                             out->plan.pass_begin[out->passes.size()]));
            // states beyond the 256 MB Infinity Cache stream from HBM:
            // non-temporal loads and stores there
            pi.ra.flags = ((elem_bytes(dtype) << n) > (size_t(256) << 20)) ? qk::RF_NONTEMPORAL : 0u;
            for (int j = 0; j < 16; j++) {
                pi.ra.tq[j] = p.tq[j];
                pi.ra.load_pos[j] = p.load_pos[j];
                pi.ra.store_pos[j] = p.store_pos[j];
            }
            out->stats_reg_swaps += p.reg_swaps;
            out->stats_reg_xposes += p.reg_xposes;
        }
        out->passes.push_back(pi);
    }
    qsim_apply_stats &s = out->stats;
    std::memset(&s, 0, sizeof(s));
    s.input_gates = L.input_gates;
    for (int l = 0; l < 6; l++) s.ops_after[l] = counts[l];
    s.fused_ops = int64_t(L.ops.size());
    out->records = int64_t(L.meas.size());
    s.passes = int64_t(passes.size());
    s.terms = out->plan.terms;
    s.bytes_moved = int64_t(passes.size()) * 2 * (int64_t(1) << n) * int64_t(elem_bytes(dtype));
    s.tile_qubits = pc.one_op_per_pass ? 0 : pc.tile_qubits;
    s.max_width = fc.max_width;
    for (const PassInfo &pi : out->passes) s.reg_passes += pi.reg ? 1 : 0;
    s.reg_swaps = out->stats_reg_swaps;
    s.reg_relayouts = out->stats_reg_xposes;
    s.compile_seconds = now_seconds() - t0;
    // parameterised templates are validated after their coefficient layout
    // is bound (qsim_batch_create)
    return keep_params ? QSIM_OK : validate_plan(n, dtype, *out);
}

}  // namespace qs

// ------------------------------------------------------------- handles
namespace {

int hip_rc(hipError_t e) { return qk::note_hip(e, "runtime call"); }

int grow(void **ptr, size_t *cap, size_t need, hipStream_t st) {
    if (need <= *cap) return QSIM_OK;
    if (qs::alloc_fault()) return QSIM_E_NOMEM;   // before anything is freed
    if (*ptr) {
        (void)hipStreamSynchronize(st);
        (void)hipFree(*ptr);
        *ptr = nullptr;
        *cap = 0;
    }
    size_t sz = std::max(need, size_t(4096));
    sz = (sz + sz / 4 + 255) & ~size_t(255);
    hipError_t e = hipMalloc(ptr, sz);
    if (e != hipSuccess) { qk::note_hip(e, "hipMalloc"); *ptr = nullptr; return QSIM_E_NOMEM; }
    *cap = sz;
    return QSIM_OK;
}

int grow_host(void **ptr, size_t *cap, size_t need) {
    if (need <= *cap) return QSIM_OK;
    if (qs::alloc_fault()) return QSIM_E_NOMEM;
    if (*ptr) (void)hipHostFree(*ptr);
    *ptr = nullptr;
    *cap = 0;
    size_t sz = std::max(need, size_t(4096));
    sz = (sz + sz / 4 + 255) & ~size_t(255);
    hipError_t e = hipHostMalloc(ptr, sz, hipHostMallocDefault);
    if (e != hipSuccess) { qk::note_hip(e, "hipHostMalloc"); *ptr = nullptr; return QSIM_E_NOMEM; }
    *cap = sz;
    return QSIM_OK;
}

}  // namespace

namespace qs {

// Copy the packed plan to pinned staging (coefficients cast to the state
// precision) and then to the device, asynchronously on `st`.
int upload_plan(DeviceTables *dt, int dtype, const PackedPlan &plan, hipStream_t st) {
    const size_t ops_bytes = plan.ops.size() * sizeof(DevOp);
    const size_t coef_bytes = plan.coefs.size() * elem_bytes(dtype);
    const size_t ops_pad = (ops_bytes + 255) & ~size_t(255);
    if (dt->stage_ev_valid) {
        (void)hipEventSynchronize(dt->stage_ev);   // previous upload has left the staging buffer
        dt->stage_ev_valid = false;
    }
    int rc = grow_host(&dt->h_stage, &dt->cap_stage, ops_pad + coef_bytes + 256);
    if (rc) return rc;
    rc = grow((void **)&dt->d_ops, &dt->cap_ops, ops_pad + 256, st);
    if (rc) return rc;
    rc = grow(&dt->d_coefs, &dt->cap_coefs, coef_bytes + 256, st);
    if (rc) return rc;
    unsigned char *h = (unsigned char *)dt->h_stage;
    if (ops_bytes) std::memcpy(h, plan.ops.data(), ops_bytes);
    if (dtype == QSIM_C64) {
        float *c = (float *)(h + ops_pad);
        for (size_t i = 0; i < plan.coefs.size(); i++) {
            c[2 * i] = float(plan.coefs[i].real());
            c[2 * i + 1] = float(plan.coefs[i].imag());
        }
    } else if (coef_bytes) {
        std::memcpy(h + ops_pad, plan.coefs.data(), coef_bytes);
    }
    if (ops_bytes && hipMemcpyAsync(dt->d_ops, h, ops_bytes, hipMemcpyHostToDevice, st) != hipSuccess)
        return QSIM_E_HIP;
    if (coef_bytes &&
        hipMemcpyAsync(dt->d_coefs, h + ops_pad, coef_bytes, hipMemcpyHostToDevice, st) != hipSuccess)
        return QSIM_E_HIP;
    if (!dt->stage_ev) {
        if (hipEventCreateWithFlags(&dt->stage_ev, hipEventDisableTiming) != hipSuccess) return QSIM_E_HIP;
    }
    if (hipEventRecord(dt->stage_ev, st) != hipSuccess) return QSIM_E_HIP;
    dt->stage_ev_valid = true;
    return QSIM_OK;
}

void free_tables(DeviceTables *dt) {
    if (dt->stage_ev_valid) (void)hipEventSynchronize(dt->stage_ev);
    if (dt->stage_ev) (void)hipEventDestroy(dt->stage_ev);
    if (dt->d_ops) (void)hipFree(dt->d_ops);
    if (dt->d_coefs) (void)hipFree(dt->d_coefs);
    if (dt->h_stage) (void)hipHostFree(dt->h_stage);
    *dt = DeviceTables{};
}

int enqueue_passes(const Compiled &c, const DeviceTables &dt, int dtype, void *state,
                   hipStream_t st, bool init_zero_first, uint64_t sstride, uint32_t nstates) {
    const PackedPlan &p = c.plan;
    for (size_t i = 0; i < c.passes.size(); i++) {
        const PassInfo &pi = c.passes[i];
        const uint32_t ob = p.pass_begin[i], oe = p.pass_begin[i + 1];
        int rc;
        if (pi.kind == Pass::MEASURE) return QSIM_E_UNSUPPORTED;
        if (pi.strided) {
            for (uint32_t j = ob; j < oe; j++) {
                rc = qk::launch_sweep(dtype, state, sstride, nstates, pi.ta.n, p.ops[j], dt.d_coefs, st);
                if (rc) return rc;
            }
        } else if (pi.reg) {
            uint32_t flags = (init_zero_first && i == 0) ? qk::TF_INIT_ZERO : 0u;
            rc = qk::launch_reg(dtype, state, sstride, nstates, pi.ra, dt.d_ops, ob, oe, dt.d_coefs,
                                p.coef_begin[i], p.coef_begin[i + 1], 0, nullptr, flags, st);
            if (rc) return rc;
        } else {
            uint32_t flags = (init_zero_first && i == 0) ? qk::TF_INIT_ZERO : 0u;
            rc = qk::launch_tile(dtype, state, sstride, nstates, pi.ta, dt.d_ops, ob, oe, dt.d_coefs,
                                 p.coef_begin[i], p.coef_begin[i + 1], 0, nullptr, flags, st);
            if (rc) return rc;
        }
    }
    return QSIM_OK;
}

}  // namespace qs

struct qsim_state {
    int n = 0;
    int dtype = 0;
    void *buf = nullptr;
    hipStream_t stream = nullptr;
    DeviceTables tables;
    void *d_red = nullptr;     // reduction partials and outputs
    size_t cap_red = 0;
    void *d_small = nullptr;   // constant coefficients (the X operator)
    size_t cap_small = 0;
    void *d_masks = nullptr;   // Pauli masks of qsim_expval
    size_t cap_masks = 0;
    void *d_scan = nullptr;    // sampling: prefix sums, block sums, shots
    size_t cap_scan = 0;
    double *h_out = nullptr;   // pinned readback
    size_t cap_out = 0;
    qsim_apply_stats last{};
};

struct qsim_program {
    int n = 0;
    int dtype = 0;
    Compiled c;
    DeviceTables dt;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    void *graph_buf = nullptr;
    std::vector<hipEvent_t> events;
    size_t timed_passes = 0;
};

namespace {

int reduce_buffers(qsim_h h, size_t partial_doubles, size_t out_doubles, double **partials,
                   double **out) {
    size_t need = (partial_doubles + out_doubles) * sizeof(double) + 512;
    int rc = grow(&h->d_red, &h->cap_red, need, h->stream);
    if (rc) return rc;
    *partials = (double *)h->d_red;
    *out = (double *)h->d_red + ((partial_doubles + 31) & ~size_t(31));
    if (h->cap_out < out_doubles * sizeof(double)) {
        void *p = h->h_out;
        size_t cap = h->cap_out;
        rc = grow_host(&p, &cap, out_doubles * sizeof(double));
        if (rc) return rc;
        h->h_out = (double *)p;
        h->cap_out = cap;
    }
    return QSIM_OK;
}

// Marginal weights of qubits qs (unnormalised), into h->h_out[0 .. 2^nqs).
int marginal(qsim_h h, const int *qs, int nqs) {
    const uint32_t nch = qk::marginal_chunks(h->n, nqs);
    double *part, *out;
    int rc = reduce_buffers(h, size_t(nch) << nqs, size_t(1) << nqs, &part, &out);
    if (rc) return rc;
    rc = qk::launch_marginal(h->dtype, h->buf, 0, 1, h->n, qs, nqs, part, out, h->stream);
    if (rc) return rc;
    if (hipMemcpyAsync(h->h_out, out, (size_t(1) << nqs) * sizeof(double), hipMemcpyDeviceToHost,
                       h->stream) != hipSuccess)
        return QSIM_E_HIP;
    return hip_rc(hipStreamSynchronize(h->stream));
}

int weights01(qsim_h h, int q, double *P0, double *P1) {
    int rc = marginal(h, &q, 1);
    if (rc) return rc;
    *P0 = h->h_out[0];
    *P1 = h->h_out[1];
    return QSIM_OK;
}

}  // namespace

extern "C" {

int qsim_version(void) { return 1; }

int qsim_debug_fail_alloc(int after) {
    if (after < -1) return QSIM_E_ARG;
    qs::g_alloc_countdown.store(after);
    return QSIM_OK;
}

const char *qsim_last_error(void) { return g_last_error; }

const char *qsim_strerror(int s) {
    switch (s) {
    case QSIM_OK: return "ok";
    case QSIM_E_ARG: return "invalid argument";
    case QSIM_E_QUBIT: return "qubit out of range or repeated";
    case QSIM_E_NOMEM: return "out of memory";
    case QSIM_E_ZERO_PROB: return "asserted outcome has zero probability";
    case QSIM_E_NOT_DEFINITE: return "qubit is not in a definite state";
    case QSIM_E_HIP: return "HIP runtime error";
    case QSIM_E_CAPACITY: return "capacity exceeded";
    case QSIM_E_UNSUPPORTED: return "unsupported gate or option";
    default: return "unknown status";
    }
}

int qsim_create(int n, int dtype, void *dev_buf, size_t buf_bytes, void *hip_stream, qsim_h *out) {
    if (!out || n < 1 || n > kMaxQubits || (dtype != QSIM_C64 && dtype != QSIM_C128) || !dev_buf)
        return QSIM_E_ARG;
    if (buf_bytes < (size_t(1) << n) * elem_bytes(dtype)) return QSIM_E_CAPACITY;
    int rc = qk::init_kernels();
    if (rc) return rc;
    qsim_state *h = new (std::nothrow) qsim_state;
    if (!h) return QSIM_E_NOMEM;
    h->n = n;
    h->dtype = dtype;
    h->buf = dev_buf;
    h->stream = (hipStream_t)hip_stream;
    // constants: the X operator as one XOR-shift-1 diagonal (1, 1)
    rc = grow(&h->d_small, &h->cap_small, 4096, h->stream);
    if (rc) { delete h; return rc; }
    if (dtype == QSIM_C64) {
        float x[4] = {1, 0, 1, 0};
        rc = hip_rc(hipMemcpy(h->d_small, x, sizeof(x), hipMemcpyHostToDevice));
    } else {
        double x[4] = {1, 0, 1, 0};
        rc = hip_rc(hipMemcpy(h->d_small, x, sizeof(x), hipMemcpyHostToDevice));
    }
    if (!rc) rc = qk::launch_init_zero(dtype, dev_buf, 0, 1, n, h->stream);
    if (!rc) rc = hip_rc(hipStreamSynchronize(h->stream));
    if (rc) { qsim_destroy(h); return rc; }
    *out = h;
    return QSIM_OK;
}

int qsim_destroy(qsim_h h) {
    if (!h) return QSIM_E_ARG;
    (void)hipStreamSynchronize(h->stream);
    free_tables(&h->tables);
    if (h->d_red) (void)hipFree(h->d_red);
    if (h->d_small) (void)hipFree(h->d_small);
    if (h->d_masks) (void)hipFree(h->d_masks);
    if (h->d_scan) (void)hipFree(h->d_scan);
    if (h->h_out) (void)hipHostFree(h->h_out);
    delete h;
    return QSIM_OK;
}

int qsim_set_stream(qsim_h h, void *st) {
    if (!h) return QSIM_E_ARG;
    (void)hipStreamSynchronize(h->stream);
    h->stream = (hipStream_t)st;
    return QSIM_OK;
}

int qsim_stream_copy(void *dst, const void *src, size_t bytes, int flags, uint32_t rotate,
                     void *hip_stream) {
    if (!dst || !src || bytes % 16 || (flags & ~1)) return QSIM_E_ARG;
    return qk::launch_stream_copy(dst, src, bytes, (flags & 1) != 0, rotate, (hipStream_t)hip_stream);
}

int qsim_init_zero(qsim_h h) {
    if (!h) return QSIM_E_ARG;
    return qk::launch_init_zero(h->dtype, h->buf, 0, 1, h->n, h->stream);
}

int qsim_apply(qsim_h h, const qsim_gate *g, size_t ng, const double *mats, size_t n_mats,
               const double *params, size_t n_params, const qsim_fuse_opts *opt) {
    if (!h || (ng && !g)) return QSIM_E_ARG;
    TraceRange range("qsim_apply");
    Compiled c;
    int rc;
    try {
        rc = compile_circuit(h->n, h->dtype, g, ng, GateInputs{mats, n_mats, params, n_params}, opt, &c);
    } catch (const std::bad_alloc &) {
        return QSIM_E_NOMEM;
    }
    if (rc) return rc;
    if (c.plan.ops.empty()) { h->last = c.stats; return QSIM_OK; }
    rc = upload_plan(&h->tables, h->dtype, c.plan, h->stream);
    if (rc) return rc;
    rc = enqueue_passes(c, h->tables, h->dtype, h->buf, h->stream, false);
    h->last = c.stats;
    return rc;
}

int qsim_compile(int n, int dtype, const qsim_gate *g, size_t ng, const double *mats,
                 size_t n_mats, const double *params, size_t n_params, const qsim_fuse_opts *opt,
                 qsim_prog *out) {
    if (!out || n < 1 || n > kMaxQubits || (dtype != QSIM_C64 && dtype != QSIM_C128) || (ng && !g))
        return QSIM_E_ARG;
    int rc = qk::init_kernels();
    if (rc) return rc;
    qsim_program *p = new (std::nothrow) qsim_program;
    if (!p) return QSIM_E_NOMEM;
    p->n = n;
    p->dtype = dtype;
    try {
        rc = compile_circuit(n, dtype, g, ng, GateInputs{mats, n_mats, params, n_params}, opt, &p->c);
    } catch (const std::bad_alloc &) {
        rc = QSIM_E_NOMEM;
    }
    if (!rc && !p->c.plan.ops.empty()) {
        rc = upload_plan(&p->dt, dtype, p->c.plan, nullptr);
        if (!rc) rc = hip_rc(hipStreamSynchronize(nullptr));
    }
    if (rc) { qsim_program_destroy(p); return rc; }
    *out = p;
    return QSIM_OK;
}

int qsim_run(qsim_h h, qsim_prog p) {
    if (!h || !p || h->n != p->n || h->dtype != p->dtype) return QSIM_E_ARG;
    TraceRange range("qsim_run");
    if (p->c.plan.ops.empty()) return QSIM_OK;
    if (p->graph_exec && p->graph_buf == h->buf) {
        return hip_rc(hipGraphLaunch(p->graph_exec, h->stream));
    }
    return enqueue_passes(p->c, p->dt, p->dtype, h->buf, h->stream, false);
}

int qsim_program_graph(qsim_prog p, qsim_h h, int enable) {
    if (!p || !h || h->n != p->n || h->dtype != p->dtype) return QSIM_E_ARG;
    if (p->graph_exec) { (void)hipGraphExecDestroy(p->graph_exec); p->graph_exec = nullptr; }
    if (p->graph) { (void)hipGraphDestroy(p->graph); p->graph = nullptr; }
    p->graph_buf = nullptr;
    if (!enable || p->c.plan.ops.empty()) return QSIM_OK;
    hipStream_t cs;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return QSIM_E_HIP;
    int rc = hip_rc(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    if (!rc) {
        int erc = enqueue_passes(p->c, p->dt, p->dtype, h->buf, cs, false);
        hipGraph_t g = nullptr;
        rc = hip_rc(hipStreamEndCapture(cs, &g));
        if (!rc && erc) rc = erc;
        if (!rc) {
            p->graph = g;
            rc = hip_rc(hipGraphInstantiate(&p->graph_exec, g, nullptr, nullptr, 0));
        } else if (g) {
            (void)hipGraphDestroy(g);
        }
    }
    (void)hipStreamDestroy(cs);
    if (!rc) p->graph_buf = h->buf;
    return rc;
}

int qsim_run_timed(qsim_h h, qsim_prog p) {
    if (!h || !p || h->n != p->n || h->dtype != p->dtype) return QSIM_E_ARG;
    const size_t np = p->c.passes.size();
    if (p->events.size() < 2 * np) {
        for (size_t i = p->events.size(); i < 2 * np; i++) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return QSIM_E_HIP;
            p->events.push_back(e);
        }
    }
    const PackedPlan &pl = p->c.plan;
    for (size_t i = 0; i < np; i++) {
        const PassInfo &pi = p->c.passes[i];
        if (hipEventRecord(p->events[2 * i], h->stream) != hipSuccess) return QSIM_E_HIP;
        int rc;
        if (pi.strided) {
            rc = QSIM_OK;
            for (uint32_t j = pl.pass_begin[i]; j < pl.pass_begin[i + 1] && !rc; j++)
                rc = qk::launch_sweep(p->dtype, h->buf, 0, 1, p->n, pl.ops[j], p->dt.d_coefs, h->stream);
        } else if (pi.reg) {
            rc = qk::launch_reg(p->dtype, h->buf, 0, 1, pi.ra, p->dt.d_ops, pl.pass_begin[i], pl.pass_begin[i + 1],
                                p->dt.d_coefs, pl.coef_begin[i], pl.coef_begin[i + 1], 0, nullptr, 0, h->stream);
        } else {
            rc = qk::launch_tile(p->dtype, h->buf, 0, 1, pi.ta, p->dt.d_ops, pl.pass_begin[i],
                                 pl.pass_begin[i + 1], p->dt.d_coefs, pl.coef_begin[i],
                                 pl.coef_begin[i + 1], 0, nullptr, 0, h->stream);
        }
        if (rc) return rc;
        if (hipEventRecord(p->events[2 * i + 1], h->stream) != hipSuccess) return QSIM_E_HIP;
    }
    p->timed_passes = np;
    return QSIM_OK;
}

int qsim_program_kernel_ms(qsim_prog p, double *ms, int64_t *launches) {
    if (!p || !ms || !launches) return QSIM_E_ARG;
    double tot = 0;
    for (size_t i = 0; i < p->timed_passes; i++) {
        if (hipEventSynchronize(p->events[2 * i + 1]) != hipSuccess) return QSIM_E_HIP;
        float f = 0;
        if (hipEventElapsedTime(&f, p->events[2 * i], p->events[2 * i + 1]) != hipSuccess) return QSIM_E_HIP;
        tot += f;
    }
    *ms = tot;
    *launches = int64_t(p->timed_passes);
    return QSIM_OK;
}

int qsim_program_stats(qsim_prog p, qsim_apply_stats *out) {
    if (!p || !out) return QSIM_E_ARG;
    *out = p->c.stats;
    return QSIM_OK;
}

int qsim_program_destroy(qsim_prog p) {
    if (!p) return QSIM_E_ARG;
    (void)hipDeviceSynchronize();
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    for (hipEvent_t e : p->events) (void)hipEventDestroy(e);
    free_tables(&p->dt);
    delete p;
    return QSIM_OK;
}

int qsim_last_stats(qsim_h h, qsim_apply_stats *out) {
    if (!h || !out) return QSIM_E_ARG;
    *out = h->last;
    return QSIM_OK;
}

int qsim_measure(qsim_h h, int q, double u, int *outcome, double *p_outcome) {
    if (!h || !outcome || !p_outcome) return QSIM_E_ARG;
    if (q < 0 || q >= h->n) return QSIM_E_QUBIT;
    if (!(u >= 0.0 && u < 1.0)) return QSIM_E_ARG;
    TraceRange range("qsim_measure");
    double P0, P1;
    int rc = weights01(h, q, &P0, &P1);
    if (rc) return rc;
    if (!(P0 + P1 > 0.0)) return QSIM_E_ZERO_PROB;
    const double p0 = P0 / (P0 + P1);
    const int o = (u < p0) ? 0 : 1;
    const double kept = o ? P1 : P0;
    rc = qk::launch_collapse(h->dtype, h->buf, h->n, q, o, 1.0 / std::sqrt(kept), h->stream);
    if (rc) return rc;
    *outcome = o;
    *p_outcome = kept / (P0 + P1);
    return QSIM_OK;
}

int qsim_measure_assert(qsim_h h, int q, int want, double *p_want) {
    if (!h || !p_want || (want != 0 && want != 1)) return QSIM_E_ARG;
    if (q < 0 || q >= h->n) return QSIM_E_QUBIT;
    TraceRange range("qsim_measure_assert");
    double P0, P1;
    int rc = weights01(h, q, &P0, &P1);
    if (rc) return rc;
    const double kept = want ? P1 : P0;
    if (!(kept > 0.0)) return QSIM_E_ZERO_PROB;
    rc = qk::launch_collapse(h->dtype, h->buf, h->n, q, want, 1.0 / std::sqrt(kept), h->stream);
    if (rc) return rc;
    *p_want = kept / (P0 + P1);
    return QSIM_OK;
}

int qsim_reset(qsim_h h, int q) {
    if (!h) return QSIM_E_ARG;
    if (q < 0 || q >= h->n) return QSIM_E_QUBIT;
    double P0, P1;
    int rc = weights01(h, q, &P0, &P1);
    if (rc) return rc;
    if (P1 == 0.0) return QSIM_OK;
    if (P0 != 0.0) return QSIM_E_NOT_DEFINITE;
    DevOp x{};
    x.coef = 0;
    x.present = 2u;   // shift 1: (X psi)[r] = psi[r ^ 1]
    x.k = 1;
    x.pos[0] = uint8_t(q);
    x.kind = DEVOP_MAT;
    return qk::launch_sweep(h->dtype, h->buf, 0, 1, h->n, x, h->d_small, h->stream);
}

int qsim_probs_noalloc(qsim_h h, const int *qs, int nqs, double *dev_out) {
    if (!h || !dev_out || nqs < 0 || nqs > 12 || (nqs && !qs)) return QSIM_E_ARG;
    int local[12];
    for (int i = 0; i < nqs; i++) {
        if (qs[i] < 0 || qs[i] >= h->n) return QSIM_E_QUBIT;
        for (int j = 0; j < i; j++)
            if (qs[j] == qs[i]) return QSIM_E_QUBIT;
        local[i] = qs[i];
    }
    return qk::launch_probs_noalloc(h->dtype, h->buf, h->n, local, nqs, dev_out, h->stream);
}

int qsim_norm(qsim_h h, double *out) {
    if (!h || !out) return QSIM_E_ARG;
    int rc = marginal(h, nullptr, 0);
    if (rc) return rc;
    *out = h->h_out[0];
    return QSIM_OK;
}

int qsim_probs(qsim_h h, const int *qs, int nqs, double *out) {
    if (!h || !out || nqs < 0 || nqs > 12 || (nqs && !qs)) return QSIM_E_ARG;
    for (int i = 0; i < nqs; i++) {
        if (qs[i] < 0 || qs[i] >= h->n) return QSIM_E_QUBIT;
        for (int j = 0; j < i; j++)
            if (qs[j] == qs[i]) return QSIM_E_QUBIT;
    }
    int rc = marginal(h, qs, nqs);
    if (rc) return rc;
    double tot = 0;
    for (int j = 0; j < (1 << nqs); j++) tot += h->h_out[j];
    if (!(tot > 0)) return QSIM_E_ZERO_PROB;
    for (int j = 0; j < (1 << nqs); j++) out[j] = h->h_out[j] / tot;
    return QSIM_OK;
}

int qsim_expval(qsim_h h, const qsim_pauli *t, size_t nt, double *out) {
    if (!h || !out || (nt && !t)) return QSIM_E_ARG;
    const uint64_t lim = (h->n >= 64) ? ~uint64_t(0) : ((uint64_t(1) << h->n) - 1);
    for (size_t k = 0; k < nt; k++) {
        if ((t[k].xmask & ~lim) || (t[k].zmask & ~lim) || !std::isfinite(t[k].coeff)) return QSIM_E_ARG;
    }
    TraceRange range("qsim_expval");
    double nrm;
    int rc = qsim_norm(h, &nrm);
    if (rc) return rc;
    if (!(nrm > 0)) return QSIM_E_ZERO_PROB;
    if (nt == 0) { *out = 0.0; return QSIM_OK; }
    std::vector<uint64_t> table;
    const qk::PauliRows nrows = qk::pauli_rows(t, nt, &table);
    rc = grow(&h->d_masks, &h->cap_masks, 8 * table.size(), h->stream);
    if (rc) return rc;
    uint64_t *dm = (uint64_t *)h->d_masks;
    // pageable source: the copy has left `table` when the call returns
    if (hipMemcpyAsync(dm, table.data(), 8 * table.size(), hipMemcpyHostToDevice, h->stream) != hipSuccess)
        return QSIM_E_HIP;
    const uint32_t nch = qk::pauli_chunks(h->n);
    double *part, *dout;
    rc = reduce_buffers(h, size_t(nch) * 2 * nt, 2 * nt, &part, &dout);
    if (rc) return rc;
    rc = qk::launch_pauli(h->dtype, h->buf, 0, 1, h->n, dm, int(nt), nrows, part, dout, h->stream);
    if (rc) return rc;
    if (hipMemcpyAsync(h->h_out, dout, 2 * nt * sizeof(double), hipMemcpyDeviceToHost, h->stream) !=
        hipSuccess)
        return QSIM_E_HIP;
    rc = hip_rc(hipStreamSynchronize(h->stream));
    if (rc) return rc;
    double total = 0;
    for (size_t k = 0; k < nt; k++) {
        const double re = h->h_out[2 * k], im = h->h_out[2 * k + 1];
        // <P> = Re(i^{#Y} S), S = sum_x (-1)^{popcount(x & z)} conj(a[x ^ x_mask]) a[x]
        double v;
        switch (__builtin_popcountll(t[k].xmask & t[k].zmask) & 3) {
        case 0: v = re; break;
        case 1: v = -im; break;
        case 2: v = -re; break;
        default: v = im; break;
        }
        total += t[k].coeff * v;
    }
    *out = total / nrm;
    return QSIM_OK;
}

int qsim_sample(qsim_h h, const double *u, size_t m, uint64_t *out) {
    if (!h || (m && (!u || !out))) return QSIM_E_ARG;
    for (size_t s = 0; s < m; s++)
        if (!(u[s] >= 0.0 && u[s] < 1.0)) return QSIM_E_ARG;
    TraceRange range("qsim_sample");
    const uint64_t len = uint64_t(1) << h->n;
    const uint64_t nb = qk::scan_blocks(h->n);
    // layout: cum[len] | bsum[nb] | boff[nb] | u[m] | shots[m]
    const size_t need = (len + 2 * nb + 2 * m) * 8 + 1024;
    int rc = grow(&h->d_scan, &h->cap_scan, need, h->stream);
    if (rc) return rc;
    double *cum = (double *)h->d_scan, *bsum = cum + len, *boff = bsum + nb, *du = boff + nb;
    uint64_t *dshot = (uint64_t *)(du + m);
    if ((rc = qk::launch_blockscan(h->dtype, h->buf, h->n, cum, bsum, h->stream))) return rc;
    std::vector<double> bs(nb);
    if ((rc = hip_rc(hipMemcpyAsync(bs.data(), bsum, nb * 8, hipMemcpyDeviceToHost, h->stream)))) return rc;
    if ((rc = hip_rc(hipStreamSynchronize(h->stream)))) return rc;
    double acc = 0.0;
    for (uint64_t b = 0; b < nb; b++) {   // exclusive prefix of block totals, in order
        const double v = bs[b];
        bs[b] = acc;
        acc += v;
    }
    if (!(acc > 0.0)) return QSIM_E_ZERO_PROB;
    if ((rc = hip_rc(hipMemcpyAsync(boff, bs.data(), nb * 8, hipMemcpyHostToDevice, h->stream)))) return rc;
    if (m && (rc = hip_rc(hipMemcpyAsync(du, u, m * 8, hipMemcpyHostToDevice, h->stream)))) return rc;
    if ((rc = qk::launch_addoff_search(cum, h->n, boff, du, m, dshot, h->stream))) return rc;
    if (m && (rc = hip_rc(hipMemcpyAsync(out, dshot, m * 8, hipMemcpyDeviceToHost, h->stream)))) return rc;
    return hip_rc(hipStreamSynchronize(h->stream));
}

int qsim_get_state(qsim_h h, void *dst) {
    if (!h || !dst) return QSIM_E_ARG;
    size_t bytes = (size_t(1) << h->n) * elem_bytes(h->dtype);
    if (hipMemcpyAsync(dst, h->buf, bytes, hipMemcpyDeviceToHost, h->stream) != hipSuccess) return QSIM_E_HIP;
    return hip_rc(hipStreamSynchronize(h->stream));
}

int qsim_set_state(qsim_h h, const void *src) {
    if (!h || !src) return QSIM_E_ARG;
    size_t bytes = (size_t(1) << h->n) * elem_bytes(h->dtype);
    if (hipMemcpyAsync(h->buf, src, bytes, hipMemcpyHostToDevice, h->stream) != hipSuccess) return QSIM_E_HIP;
    return hip_rc(hipStreamSynchronize(h->stream));
}

int qsim_autotune(qsim_h h, const qsim_gate *g, size_t ng, const double *mats, size_t n_mats,
                  const double *params, size_t n_params, size_t prefix_gates, qsim_fuse_opts *best,
                  double *ns_per_gate) {
    if (!h || !best || (ng && !g)) return QSIM_E_ARG;
    if (prefix_gates == 0) prefix_gates = 20000;
    // the prefix ends at a whole number of records; barriers are kept
    const size_t np = std::min(ng, prefix_gates);
    std::vector<qsim_fuse_opts> cands;
    const int tdef = (h->dtype == QSIM_C64 && h->n >= 23) ? 13 : 12;
    const int ldef = h->dtype == QSIM_C64 ? 4 : 3;
    const int wmax = h->dtype == QSIM_C64 ? 5 : 4;
    for (int t : {tdef - 1, tdef, tdef + 1}) {
        if (t > resident_max(h->dtype)) continue;
        for (int w = 2; w <= wmax; w++)
            for (float cost : {2.0f, 4.0f, 8.0f})
                for (int low : {ldef - 1, ldef}) {
                    qsim_fuse_opts o{};
                    o.level = 5;
                    o.max_width = w;
                    o.tile_qubits = t;
                    o.op_cost = cost;
                    o.low_qubits = low;
                    cands.push_back(o);
                }
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return QSIM_E_HIP;
    double best_ns = 1e300;
    int rc = QSIM_OK;
    DeviceTables dt;
    for (const qsim_fuse_opts &o : cands) {
        Compiled c;
        try {
            rc = compile_circuit(h->n, h->dtype, g, np, GateInputs{mats, n_mats, params, n_params}, &o, &c);
        } catch (const std::bad_alloc &) {
            rc = QSIM_E_NOMEM;
        }
        if (rc) break;
        if (c.plan.ops.empty()) continue;
        if ((rc = upload_plan(&dt, h->dtype, c.plan, h->stream))) break;
        // warm, then time one run
        if ((rc = enqueue_passes(c, dt, h->dtype, h->buf, h->stream, false))) break;
        (void)hipEventRecord(e0, h->stream);
        if ((rc = enqueue_passes(c, dt, h->dtype, h->buf, h->stream, false))) break;
        (void)hipEventRecord(e1, h->stream);
        if ((rc = hip_rc(hipEventSynchronize(e1)))) break;
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        const double ns = 1e6 * double(ms) / double(std::max<int64_t>(1, c.stats.input_gates));
        if (ns < best_ns) {
            best_ns = ns;
            *best = o;
        }
    }
    free_tables(&dt);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!rc) rc = qk::launch_init_zero(h->dtype, h->buf, 0, 1, h->n, h->stream);
    if (!rc) rc = hip_rc(hipStreamSynchronize(h->stream));
    if (ns_per_gate) *ns_per_gate = best_ns;
    return rc;
}

}  // extern "C"

namespace qs {

int tune_width(int n, int dtype, const qsim_gate *g, size_t ng, const GateInputs &in,
               const qsim_fuse_opts *base, int *best_w, double *best_ns) {
    const int wmax = dtype == QSIM_C64 ? 5 : 4;
    const size_t bytes = elem_bytes(dtype) << n;
    void *buf = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = hip_rc(hipMalloc(&buf, bytes));
    if (rc) return QSIM_E_NOMEM;
    if (!rc) rc = hip_rc(hipStreamCreate(&st));
    if (!rc) rc = hip_rc(hipEventCreate(&e0));
    if (!rc) rc = hip_rc(hipEventCreate(&e1));
    DeviceTables dt;
    *best_w = 0;
    *best_ns = 1e300;
    for (int w = 2; w <= wmax && !rc; w++) {
        qsim_fuse_opts o{};
        if (base) o = *base;
        o.level = 5;
        o.max_width = w;
        Compiled c;
        try {
            rc = compile_circuit(n, dtype, g, ng, in, &o, &c);
        } catch (const std::bad_alloc &) {
            rc = QSIM_E_NOMEM;
        }
        if (rc) break;
        if (c.plan.ops.empty()) {
            *best_w = w;
            *best_ns = 0.0;
            break;
        }
        if ((rc = upload_plan(&dt, dtype, c.plan, st))) break;
        // warm, then the best of three timed runs
        if ((rc = enqueue_passes(c, dt, dtype, buf, st, true))) break;
        double best_run = 1e300;
        for (int rep = 0; rep < 3 && !rc; rep++) {
            (void)hipEventRecord(e0, st);
            if ((rc = enqueue_passes(c, dt, dtype, buf, st, true))) break;
            (void)hipEventRecord(e1, st);
            if ((rc = hip_rc(hipEventSynchronize(e1)))) break;
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            best_run = std::min(best_run, double(ms));
        }
        const double ns = 1e6 * best_run / double(std::max<int64_t>(1, c.stats.input_gates));
        if (!rc && ns < *best_ns) {
            *best_ns = ns;
            *best_w = w;
        }
    }
    if (st) (void)hipStreamSynchronize(st);
    free_tables(&dt);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    (void)hipFree(buf);
    return rc;
}

int tune_tile_batch(int n, int dtype, const qsim_gate *g, size_t ng, const GateInputs &in,
                    const qsim_fuse_opts &base, uint32_t nstates, int *best_t) {
    *best_t = base.tile_qubits;
    if (n <= resident_max(dtype) || nstates == 0) return QSIM_OK;
    // enough states for 4,096 12-qubit tiles (16 per CU), within 1 GiB
    const size_t state_bytes = elem_bytes(dtype) << n;
    uint64_t sample = std::max<uint64_t>(1, uint64_t(4096) >> std::min(n - 12, 12));
    sample = std::min<uint64_t>(sample, nstates);
    sample = std::max<uint64_t>(1, std::min<uint64_t>(sample, (uint64_t(1) << 30) / state_bytes));
    void *buf = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (alloc_fault() || hipMalloc(&buf, state_bytes * sample) != hipSuccess) {
        (void)hipGetLastError();
        return QSIM_E_NOMEM;
    }
    int rc = hip_rc(hipStreamCreate(&st));
    if (!rc) rc = hip_rc(hipEventCreate(&e0));
    if (!rc) rc = hip_rc(hipEventCreate(&e1));
    DeviceTables dt;
    double best_ms = 1e300;
    for (int t = 12; t <= 13 && !rc; t++) {
        qsim_fuse_opts o = base;
        o.tile_qubits = t;
        Compiled c;
        try {
            rc = compile_circuit(n, dtype, g, ng, in, &o, &c);
        } catch (const std::bad_alloc &) {
            rc = QSIM_E_NOMEM;
        }
        if (rc) break;
        if (c.plan.ops.empty()) break;
        if ((rc = upload_plan(&dt, dtype, c.plan, st))) break;
        const uint64_t sstride = uint64_t(1) << n;
        // warm, then the best of three timed runs
        if ((rc = enqueue_passes(c, dt, dtype, buf, st, true, sstride, uint32_t(sample)))) break;
        double run_ms = 1e300;
        for (int rep = 0; rep < 3 && !rc; rep++) {
            (void)hipEventRecord(e0, st);
            if ((rc = enqueue_passes(c, dt, dtype, buf, st, true, sstride, uint32_t(sample)))) break;
            (void)hipEventRecord(e1, st);
            if ((rc = hip_rc(hipEventSynchronize(e1)))) break;
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            run_ms = std::min(run_ms, double(ms));
        }
        if (!rc && run_ms < best_ms) {
            best_ms = run_ms;
            *best_t = t;
        }
    }
    if (st) (void)hipStreamSynchronize(st);
    free_tables(&dt);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    (void)hipFree(buf);
    return rc;
}

}  // namespace qs

extern "C" {

int qsim_debug_fuse(int n, const qsim_gate *g, size_t ng, const double *mats, size_t n_mats,
                    const double *params, size_t n_params, const qsim_fuse_opts *opt, int32_t *out_k, int32_t *out_qubits,
                    double *out_mats, size_t cap_ops, size_t cap_doubles, size_t *n_ops,
                    int64_t *counts) {
    if (n < 1 || n > kMaxQubits || (ng && !g) || !n_ops) return QSIM_E_ARG;
    FuseConfig fc;
    PlanConfig pc;
    default_configs(n, QSIM_C128, opt, &fc, &pc);
    if (opt && opt->max_width > 0) fc.max_width = std::max(1, std::min(opt->max_width, kMaxK));
    Lowered L;
    int rc;
    int64_t cnt[6];
    try {
        if (alloc_fault()) throw std::bad_alloc();
        rc = lower(n, g, ng, GateInputs{mats, n_mats, params, n_params}, false, false, &L);
        if (rc) return rc;
        fuse(n, &L, fc, cnt);
    } catch (const std::bad_alloc &) {
        return QSIM_E_NOMEM;
    }
    if (counts)
        for (int l = 0; l < 6; l++) counts[l] = cnt[l];
    *n_ops = L.ops.size();
    size_t need = 0;
    for (const Op &o : L.ops) need += 2 * size_t(o.dim()) * o.dim();
    if (L.ops.size() > cap_ops || need > cap_doubles) return QSIM_E_CAPACITY;
    size_t pos = 0;
    for (size_t i = 0; i < L.ops.size(); i++) {
        const Op &o = L.ops[i];
        out_k[i] = o.k;
        for (int j = 0; j < kMaxK; j++) out_qubits[5 * i + j] = j < o.k ? o.q[j] : -1;
        for (size_t e = 0; e < size_t(o.dim()) * o.dim(); e++) {
            out_mats[pos++] = o.m[e].real();
            out_mats[pos++] = o.m[e].imag();
        }
    }
    return QSIM_OK;
}

int qsim_parse_qasm(const char *text, size_t len, qsim_gate *out, size_t cap, size_t *n_out,
                    int32_t *n_qubits, int32_t *n_clbits) {
    if ((!text && len) || !n_out) return QSIM_E_ARG;
    std::vector<qsim_gate> g;
    int nq = 0, nc = 0;
    std::string err;
    int rc;
    try {
        rc = parse_qasm(text ? text : "", len, &g, &nq, &nc, &err);
    } catch (const std::bad_alloc &) {
        return QSIM_E_NOMEM;
    }
    if (rc) {
        std::snprintf(g_last_error, sizeof(g_last_error), "%s", err.c_str());
        return rc;
    }
    *n_out = g.size();
    if (n_qubits) *n_qubits = nq;
    if (n_clbits) *n_clbits = nc;
    if (g.size() > cap || (!out && !g.empty())) return QSIM_E_CAPACITY;
    if (!g.empty()) std::memcpy(out, g.data(), g.size() * sizeof(qsim_gate));
    return QSIM_OK;
}

int qsim_debug_emulate(int n, int dtype, const qsim_gate *g, size_t ng, const double *mats,
                       size_t n_mats, const double *params, size_t n_params,
                       const qsim_fuse_opts *opt, double *psi) {
    if (n < 1 || n > 24 || (dtype != QSIM_C64 && dtype != QSIM_C128) || !psi) return QSIM_E_ARG;
    Compiled c;
    int rc;
    try {
        rc = compile_circuit(n, dtype, g, ng, GateInputs{mats, n_mats, params, n_params}, opt, &c);
    } catch (const std::bad_alloc &) {
        return QSIM_E_NOMEM;
    }
    if (rc) return rc;
    const PackedPlan &p = c.plan;
    cd *st = reinterpret_cast<cd *>(psi);
    // y[r] = sum over present shifts (ascending) of cf[term * 2^k + r] x[r ^ m]
    // on the 2^k members of every group of a width-w array addressed by pos[]
    auto apply = [&](cd *v, int w, const DevOp &o, const cd *cf) {
        const int k = o.k, d = 1 << k;
        std::vector<cd> x(d), y(d);
        for (uint64_t grp = 0; grp < (uint64_t(1) << (w - k)); grp++) {
            uint64_t b0 = grp;
            for (int j = 0; j < k; j++)
                b0 = ((b0 >> o.pos[j]) << (o.pos[j] + 1)) | (b0 & ((uint64_t(1) << o.pos[j]) - 1));
            auto at = [&](int r) {
                uint64_t a = b0;
                for (int j = 0; j < k; j++)
                    if ((r >> j) & 1) a |= uint64_t(1) << o.pos[j];
                return a;
            };
            for (int r = 0; r < d; r++) x[r] = v[at(r)];
            for (int r = 0; r < d; r++) {
                cd acc = 0;
                int term = 0;
                for (int m = 0; m < d; m++)
                    if ((o.present >> m) & 1) acc += cf[size_t(term++) * d + r] * x[r ^ m];
                y[r] = acc;
            }
            for (int r = 0; r < d; r++) v[at(r)] = y[r];
        }
    };
    for (size_t i = 0; i < c.passes.size(); i++) {
        const PassInfo &pi = c.passes[i];
        if (pi.kind == Pass::MEASURE) return QSIM_E_ARG;
        if (pi.strided) {
            for (uint32_t j = p.pass_begin[i]; j < p.pass_begin[i + 1]; j++) {
                const DevOp &o = p.ops[j];
                if (o.kind != DEVOP_MAT || o.kx) return QSIM_E_ARG;
                apply(st, n, o, p.coefs.data() + o.coef);
            }
            continue;
        }
        if (pi.reg) {
            // register-resident pass: elements indexed by position bits
            // (thread bits, then register bits), moved as the kernel moves them
            const qk::RegArgs &ra = pi.ra;
            const int t = ra.t, logt = t - kRegBits;
            std::vector<cd> v(size_t(1) << t), w(v.size());
            for (uint64_t tile = 0; tile < (uint64_t(1) << (n - t)); tile++) {
                const uint64_t base = qk::tile_base(tile, ra.rest_mask, ra.nxcd, ra.xcd_q);
                auto addr = [&](uint64_t P, const uint8_t *pos) {
                    uint64_t a = base;
                    for (int b = 0; b < t; b++)
                        if ((P >> b) & 1) a |= uint64_t(1) << ra.tq[pos[b]];
                    return a;
                };
                uint8_t cur[16];
                std::memcpy(cur, ra.load_pos, 16);
                for (uint64_t P = 0; P < v.size(); P++) v[P] = st[addr(P, ra.load_pos)];
                for (uint32_t j = p.pass_begin[i]; j < p.pass_begin[i + 1]; j++) {
                    const DevOp &o = p.ops[j];
                    if (o.kind == DEVOP_RMAT) {
                        uint32_t e = 0;
                        for (int x = 0; x < o.kx; x++) e |= uint32_t((base >> o.xq[x]) & 1) << x;
                        const cd *cf = p.coefs.data() + o.coef + (size_t(e) * __builtin_popcount(o.present) << 4);
                        for (uint64_t tid = 0; tid < (uint64_t(1) << logt); tid++) {
                            cd x[16], y[16];
                            for (int r = 0; r < 16; r++) x[r] = v[tid | (uint64_t(r) << logt)];
                            for (int r = 0; r < 16; r++) {
                                cd acc = 0;
                                int term = 0;
                                for (int M = 0; M < 16; M++)
                                    if ((o.present >> M) & 1) acc += cf[size_t(term++) * 16 + r] * x[r ^ M];
                                y[r] = acc;
                            }
                            for (int r = 0; r < 16; r++) v[tid | (uint64_t(r) << logt)] = y[r];
                        }
                    } else if (o.kind == DEVOP_SWAP) {
                        const int a = o.pos[0], b = logt + o.pos[1];
                        for (uint64_t P = 0; P < v.size(); P++) {
                            const uint64_t ba = (P >> a) & 1, bb = (P >> b) & 1;
                            uint64_t Q = P & ~((uint64_t(1) << a) | (uint64_t(1) << b));
                            Q |= (ba << b) | (bb << a);
                            w[Q] = v[P];
                        }
                        std::swap(v, w);
                        std::swap(cur[a], cur[b]);
                    } else if (o.kind == DEVOP_XPOSE && j + 1 < p.pass_begin[i + 1]) {
                        const uint8_t *from = reinterpret_cast<const uint8_t *>(&o);
                        const uint8_t *to = reinterpret_cast<const uint8_t *>(&p.ops[j + 1]);
                        if (std::memcmp(from, cur, size_t(t)) != 0) return QSIM_E_ARG;
                        int to_pos[16];
                        for (int b = 0; b < t; b++) to_pos[to[b]] = b;
                        for (uint64_t P = 0; P < v.size(); P++) {
                            uint64_t Q = 0;
                            for (int b = 0; b < t; b++)
                                if ((P >> b) & 1) Q |= uint64_t(1) << to_pos[from[b]];
                            w[Q] = v[P];
                        }
                        std::swap(v, w);
                        std::memcpy(cur, to, size_t(t));
                        j++;
                    } else {
                        return QSIM_E_ARG;
                    }
                }
                if (std::memcmp(cur, ra.store_pos, size_t(t)) != 0) return QSIM_E_ARG;
                for (uint64_t P = 0; P < v.size(); P++) st[addr(P, ra.store_pos)] = v[P];
            }
            continue;
        }
        const qk::TileArgs &ta = pi.ta;
        const int t = ta.t;
        std::vector<cd> v(size_t(1) << t);
        for (uint64_t tile = 0; tile < (uint64_t(1) << (n - t)); tile++) {
            // the workgroup's tile in the kernel's order
            const uint64_t base = qk::tile_base(tile, ta.rest_mask, ta.nxcd, ta.xcd_q);
            auto addr = [&](uint64_t jpos) {
                uint64_t a = base;
                for (int b = 0; b < t; b++)
                    if ((jpos >> b) & 1) a |= uint64_t(1) << ta.tq[b];
                return a;
            };
            for (uint64_t jpos = 0; jpos < v.size(); jpos++) v[jpos] = st[addr(jpos)];
            for (uint32_t j = p.pass_begin[i]; j < p.pass_begin[i + 1]; j++) {
                const DevOp &o = p.ops[j];
                if (o.kind != DEVOP_MAT) return QSIM_E_ARG;
                uint32_t e = 0;
                for (int x = 0; x < o.kx; x++) e |= uint32_t((base >> o.xq[x]) & 1) << x;
                apply(v.data(), t, o,
                      p.coefs.data() + o.coef + size_t(e) * (size_t(__builtin_popcount(o.present)) << o.k));
            }
            for (uint64_t jpos = 0; jpos < v.size(); jpos++) st[addr(jpos)] = v[jpos];
        }
    }
    return QSIM_OK;
}

int qsim_debug_plan(int n, int dtype, const qsim_gate *g, size_t ng, const double *mats,
                    size_t n_mats, const double *params, size_t n_params,
                    const qsim_fuse_opts *opt, qsim_apply_stats *out) {
    if (n < 1 || n > kMaxQubits || (dtype != QSIM_C64 && dtype != QSIM_C128) || !out) return QSIM_E_ARG;
    Compiled c;
    int rc;
    try {
        rc = compile_circuit(n, dtype, g, ng, GateInputs{mats, n_mats, params, n_params}, opt, &c);
    } catch (const std::bad_alloc &) {
        return QSIM_E_NOMEM;
    }
    if (rc) return rc;
    *out = c.stats;
    return QSIM_OK;
}

}  // extern "C"
