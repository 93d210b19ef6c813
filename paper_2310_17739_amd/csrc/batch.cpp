// Batched programs (qsim_batch_*): many states of one width share a compiled
// program; several widths form one batch.  The whole run -- angle binding,
// the program's passes and device-side measurement decisions, FP64 norms and
// Pauli overlaps -- is enqueued without host round trips and can be recorded
// once as a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "host.h"
#include "launch.h"
#include "runtime.h"

using namespace qs;

namespace {

int hip_ok(hipError_t e, const char *where) { return qk::note_hip(e, where); }

template <typename P>
int dalloc(P **p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) return QSIM_OK;
    if (alloc_fault()) return QSIM_E_NOMEM;
    void *v = nullptr;
    hipError_t e = hipMalloc(&v, bytes);
    if (e != hipSuccess) { qk::note_hip(e, "hipMalloc (batch)"); return QSIM_E_NOMEM; }
    *p = static_cast<P *>(v);
    return QSIM_OK;
}

template <typename P>
void dfree(P *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

struct Group {
    int n = 0, nstates = 0, nparams = 0, nslots = 0;
    size_t nterms = 0;
    uint64_t sstride = 0;          // elements between states
    bool own_states = false;
    void *d_states = nullptr;
    Compiled c;
    std::vector<qsim_pauli> terms;
    // device tables
    DevOp *d_ops = nullptr;
    void *d_coefs = nullptr;       // bound coefficients (per state when parameterised)
    uint64_t cstride = 0;          // elements between states' coefficient arrays
    double *d_tmpl = nullptr;      // FP64 template coefficients (parameterised)
    qk::BindEntry *d_bind = nullptr;
    uint32_t nbind = 0, max_count = 0;
    double *d_params = nullptr;
    double *d_uniforms = nullptr;
    int32_t *d_forced = nullptr;
    int32_t *d_outcomes = nullptr;
    double *d_probs = nullptr;
    int32_t *d_status = nullptr;
    int32_t *d_fail_at = nullptr;
    double *d_part = nullptr;      // reduction partials
    size_t part_doubles = 0;
    double *d_p01 = nullptr;       // [nstates][2]
    double *d_norm = nullptr;      // [nstates]
    uint64_t *d_masks = nullptr;   // [2][nterms]
    double *d_pauli = nullptr;     // [nstates][nterms][2]
    uint32_t pauli_chunks = 0, norm_chunks = 0;
    qk::PauliRows pauli_rows;
    int64_t coef_bytes = 0;
    int tuned_width = 0;           // fusion width the autotuner chose (0: not tuned)
    double tune_seconds = 0.0;
};

void free_group(Group &g) {
    if (g.own_states) dfree(g.d_states);
    dfree(g.d_ops);
    dfree(g.d_coefs);
    dfree(g.d_tmpl);
    dfree(g.d_bind);
    dfree(g.d_params);
    dfree(g.d_uniforms);
    dfree(g.d_forced);
    dfree(g.d_outcomes);
    dfree(g.d_probs);
    dfree(g.d_status);
    dfree(g.d_fail_at);
    dfree(g.d_part);
    dfree(g.d_p01);
    dfree(g.d_norm);
    dfree(g.d_masks);
    dfree(g.d_pauli);
}

uint32_t pow2_floor(uint64_t x) {
    uint32_t r = 1;
    while (uint64_t(r) * 2 <= x && r < (1u << 30)) r *= 2;
    return r;
}

}  // namespace

struct qsim_batch {
    int dtype = QSIM_C64;
    bool use_graph = false;
    std::vector<Group> groups;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    qsim_batch_info info{};
};

namespace {

// Rewrite a parameterised plan from its template layout (2^np cos/sin blocks
// per operator) to the bound layout (one block per operator, per state) and
// collect the bind entries.  Returns the bound coefficient count.
size_t bind_layout(Compiled *c, std::vector<qk::BindEntry> *ents, uint32_t *max_count) {
    PackedPlan &p = c->plan;
    size_t bound = 0;
    *max_count = 0;
    for (size_t j = 0; j < p.ops.size(); j++) {
        DevOp &o = p.ops[j];
        if (!devop_is_mat(o.kind)) continue;
        const uint32_t count = devop_coefs(o);
        qk::BindEntry e{};
        e.bound_off = uint32_t(bound);
        e.count = count;
        e.tmpl_off = o.coef;
        e.np = p.op_np[j];
        for (int s = 0; s < 3; s++) e.slot[s] = p.op_slots[3 * j + s];
        ents->push_back(e);
        *max_count = std::max(*max_count, count);
        o.coef = uint32_t(bound);
        bound += count;
    }
    // pass coefficient ranges in the bound layout
    std::vector<uint32_t> new_begin(p.coef_begin.size());
    size_t run = 0;
    for (size_t i = 0; i + 1 < p.pass_begin.size(); i++) {
        new_begin[i] = uint32_t(run);
        for (uint32_t j = p.pass_begin[i]; j < p.pass_begin[i + 1]; j++)
            if (devop_is_mat(p.ops[j].kind)) run += devop_coefs(p.ops[j]);
    }
    new_begin.back() = uint32_t(run);
    p.coef_begin = new_begin;
    for (auto &x : p.op_np) x = 0;
    return bound;
}

int setup_group(Group &G, const qsim_batch_group &in, int dtype, const qsim_batch_opts &opt) {
    G.n = in.n;
    G.nstates = in.n_states;
    G.nparams = in.params ? in.n_params : 0;
    G.nslots = in.n_slots;
    G.nterms = in.terms ? in.n_terms : 0;
    G.sstride = uint64_t(1) << in.n;
    const size_t elem = elem_bytes(dtype);
    const bool param = in.params != nullptr && in.n_params > 0;
    // the group's passes cover all its states: its default tile width
    // follows their total tile count
    qsim_fuse_opts base{};
    if (opt.fuse.level > 0) base = opt.fuse;
    else base.level = 5;
    if (base.tile_qubits <= 0) base.tile_qubits = default_tile_qubits(in.n, dtype, uint64_t(in.n_states));
    const qsim_fuse_opts *fo = &base;
    qsim_fuse_opts tuned{};
    if (opt.autotune) {
        // the template's fusion width, timed on its first instance (angles of
        // state 0 bound on the host), then (unless `opt.fuse` fixes it) its
        // tile width, timed over a sample of states run together as the batch
        // runs them; measurement records are left out of the timed circuit,
        // and the low-qubit choice stays that of `opt.fuse`
        std::vector<qsim_gate> timed;
        timed.reserve(in.ng);
        for (size_t i = 0; i < in.ng; i++)
            if (in.g[i].kind != QSIM_G_MEASURE && in.g[i].kind != QSIM_G_ASSERT0 && in.g[i].kind != QSIM_G_RESET)
                timed.push_back(in.g[i]);
        int w = 0;
        double ns = 0.0;
        const double t0 = now_seconds();
        int rc = tune_width(in.n, dtype, timed.data(), timed.size(),
                            GateInputs{in.mats, in.mats ? in.n_mats : 0, param ? in.params : nullptr,
                                       param ? size_t(in.n_params) : 0},
                            fo, &w, &ns);
        if (rc) return rc;
        tuned = *fo;
        tuned.level = 5;
        tuned.max_width = w;
        if (!(opt.fuse.level > 0 && opt.fuse.tile_qubits > 0) && !std::getenv("QSIM_TILE_QUBITS")) {
            int t = tuned.tile_qubits;
            rc = tune_tile_batch(in.n, dtype, timed.data(), timed.size(),
                                 GateInputs{in.mats, in.mats ? in.n_mats : 0, param ? in.params : nullptr,
                                            param ? size_t(in.n_params) : 0},
                                 tuned, uint32_t(in.n_states), &t);
            if (rc) return rc;
            tuned.tile_qubits = t;
        }
        G.tune_seconds = now_seconds() - t0;
        fo = &tuned;
        G.tuned_width = w;
    }
    int rc = compile_program(in.n, dtype, in.g, in.ng,
                             GateInputs{in.mats, in.mats ? in.n_mats : 0, nullptr,
                                        param ? size_t(in.n_params) : 0},
                             param, true,
                             opt.max_params > 0 ? opt.max_params : 2, fo, &G.c);
    if (rc) return rc;
    // every parameter slot and measurement slot must be inside its vector
    for (size_t i = 0; i < in.ng; i++) {
        const qsim_gate &g = in.g[i];
        if ((g.kind == QSIM_G_MEASURE || g.kind == QSIM_G_ASSERT0) && (g.slot < 0 || g.slot >= in.n_slots))
            return QSIM_E_ARG;
        if (g.kind == QSIM_G_MEASURE && !in.uniforms) return QSIM_E_ARG;
        if (g.kind < QSIM_G_MAT && g.slot >= 0 && (!param || g.slot >= in.n_params)) return QSIM_E_ARG;
    }
    std::vector<qk::BindEntry> ents;
    size_t ncoef = G.c.plan.coefs.size();
    if (param) {
        ncoef = bind_layout(&G.c, &ents, &G.max_count);
        G.nbind = uint32_t(ents.size());
        G.cstride = ncoef;
    }
    rc = validate_plan(G.n, dtype, G.c);
    if (rc) return rc;
    const PackedPlan &p = G.c.plan;
    // device tables
    if ((rc = dalloc(&G.d_ops, p.ops.size() * sizeof(DevOp)))) return rc;
    if (!p.ops.empty() && (rc = hip_ok(hipMemcpy(G.d_ops, p.ops.data(), p.ops.size() * sizeof(DevOp),
                                                hipMemcpyHostToDevice), "upload ops")))
        return rc;
    const size_t nstate_coef = param ? size_t(G.nstates) : 1;
    G.coef_bytes = int64_t(ncoef * nstate_coef * elem);
    if ((rc = dalloc((char **)&G.d_coefs, std::max<size_t>(ncoef * nstate_coef * elem, 16)))) return rc;
    if (param) {
        if ((rc = dalloc(&G.d_tmpl, p.coefs.size() * 16))) return rc;
        if (!p.coefs.empty() && (rc = hip_ok(hipMemcpy(G.d_tmpl, p.coefs.data(), p.coefs.size() * 16,
                                                      hipMemcpyHostToDevice), "upload template")))
            return rc;
        if ((rc = dalloc(&G.d_bind, ents.size() * sizeof(qk::BindEntry)))) return rc;
        if (!ents.empty() && (rc = hip_ok(hipMemcpy(G.d_bind, ents.data(), ents.size() * sizeof(qk::BindEntry),
                                                   hipMemcpyHostToDevice), "upload bind table")))
            return rc;
        const size_t pb = size_t(G.nstates) * G.nparams * sizeof(double);
        if ((rc = dalloc(&G.d_params, pb))) return rc;
        if ((rc = hip_ok(hipMemcpy(G.d_params, in.params, pb, hipMemcpyHostToDevice), "upload params"))) return rc;
    } else if (ncoef) {
        std::vector<char> host(ncoef * elem);
        if (dtype == QSIM_C64) {
            float *f = (float *)host.data();
            for (size_t i = 0; i < ncoef; i++) { f[2 * i] = float(p.coefs[i].real()); f[2 * i + 1] = float(p.coefs[i].imag()); }
        } else {
            std::memcpy(host.data(), p.coefs.data(), ncoef * elem);
        }
        if ((rc = hip_ok(hipMemcpy(G.d_coefs, host.data(), host.size(), hipMemcpyHostToDevice), "upload coefs")))
            return rc;
    }
    // states
    if (in.dev_states) {
        G.d_states = in.dev_states;
    } else {
        G.own_states = true;
        if ((rc = dalloc((char **)&G.d_states, size_t(G.nstates) * G.sstride * elem))) return rc;
    }
    // measurement I/O
    const size_t ns = size_t(G.nstates) * std::max(G.nslots, 0);
    if (ns) {
        if ((rc = dalloc(&G.d_outcomes, ns * 4))) return rc;
        if ((rc = dalloc(&G.d_probs, ns * 8))) return rc;
        if (in.uniforms) {
            if ((rc = dalloc(&G.d_uniforms, ns * 8))) return rc;
            if ((rc = hip_ok(hipMemcpy(G.d_uniforms, in.uniforms, ns * 8, hipMemcpyHostToDevice), "uniforms"))) return rc;
        }
        if (in.forced) {
            if ((rc = dalloc(&G.d_forced, ns * 4))) return rc;
            if ((rc = hip_ok(hipMemcpy(G.d_forced, in.forced, ns * 4, hipMemcpyHostToDevice), "forced"))) return rc;
        }
    }
    if ((rc = dalloc(&G.d_status, size_t(G.nstates) * 4))) return rc;
    if ((rc = dalloc(&G.d_fail_at, size_t(G.nstates) * 4))) return rc;
    // reductions: chunk counts keep the partial buffers small for big batches
    G.norm_chunks = std::max<uint32_t>(1, std::min<uint32_t>(qk::marginal_chunks(G.n, 0),
                                                           pow2_floor((1u << 22) / uint64_t(G.nstates) / 2)));
    size_t part = size_t(G.nstates) * 2 * G.norm_chunks;
    if (G.nterms) {
        G.pauli_chunks = std::max<uint32_t>(1, std::min<uint32_t>(qk::pauli_chunks(G.n),
                                                                pow2_floor((1u << 22) / (uint64_t(G.nstates) * G.nterms * 2))));
        part = std::max(part, size_t(G.nstates) * G.nterms * 2 * G.pauli_chunks);
        G.terms.assign(in.terms, in.terms + G.nterms);
        const uint64_t lim = (uint64_t(1) << G.n) - 1;
        for (size_t k = 0; k < G.nterms; k++)
            if ((in.terms[k].xmask & ~lim) || (in.terms[k].zmask & ~lim)) return QSIM_E_ARG;
        std::vector<uint64_t> masks;
        G.pauli_rows = qk::pauli_rows(in.terms, G.nterms, &masks);
        if ((rc = dalloc(&G.d_masks, masks.size() * 8))) return rc;
        if ((rc = hip_ok(hipMemcpy(G.d_masks, masks.data(), masks.size() * 8, hipMemcpyHostToDevice), "masks"))) return rc;
        if ((rc = dalloc(&G.d_pauli, size_t(G.nstates) * G.nterms * 2 * 8))) return rc;
    }
    G.part_doubles = part;
    if ((rc = dalloc(&G.d_part, part * 8))) return rc;
    if ((rc = dalloc(&G.d_p01, size_t(G.nstates) * 2 * 8))) return rc;
    if ((rc = dalloc(&G.d_norm, size_t(G.nstates) * 8))) return rc;
    return QSIM_OK;
}

int enqueue_group(const Group &G, int dtype, hipStream_t st) {
    int rc;
    if ((rc = qk::launch_fill_i32(G.d_status, 0, uint64_t(G.nstates), st))) return rc;
    if ((rc = qk::launch_fill_i32(G.d_fail_at, -1, uint64_t(G.nstates), st))) return rc;
    if (G.nbind) {
        rc = qk::launch_bind(dtype, G.d_tmpl, G.d_bind, G.nbind, G.d_params, G.nparams, G.d_coefs,
                             G.cstride, uint32_t(G.nstates), G.max_count, st);
        if (rc) return rc;
    }
    const PackedPlan &p = G.c.plan;
    qk::MeasArgs ma{};
    ma.uniforms = G.d_uniforms;
    ma.forced = G.d_forced;
    ma.outcomes = G.d_outcomes;
    ma.probs = G.d_probs;
    ma.status = G.d_status;
    ma.fail_at = G.d_fail_at;
    ma.nslots = G.nslots;
    const bool first_tile = !G.c.passes.empty() && G.c.passes[0].kind == Pass::TILE;
    if (!first_tile) {
        if ((rc = qk::launch_init_zero(dtype, G.d_states, G.sstride, uint32_t(G.nstates), G.n, st))) return rc;
    }
    for (size_t i = 0; i < G.c.passes.size(); i++) {
        const PassInfo &pi = G.c.passes[i];
        if (pi.kind == Pass::MEASURE) {
            int q = pi.meas.q;
            rc = qk::launch_marginal(dtype, G.d_states, G.sstride, uint32_t(G.nstates), G.n, &q, 1,
                                     G.d_part, G.d_p01, st, G.norm_chunks);
            if (!rc)
                rc = qk::launch_decide(dtype, G.d_states, G.sstride, uint32_t(G.nstates), G.n, q,
                                       pi.meas.kind, pi.meas.slot, G.d_p01, ma, st);
        } else if (pi.strided) {
            rc = QSIM_OK;
            for (uint32_t j = p.pass_begin[i]; j < p.pass_begin[i + 1] && !rc; j++)
                rc = qk::launch_sweep(dtype, G.d_states, G.sstride, uint32_t(G.nstates), G.n, p.ops[j],
                                      G.d_coefs, st, G.cstride, G.d_status);
        } else if (pi.reg) {
            const uint32_t flags = (i == 0 && first_tile) ? qk::TF_INIT_ZERO : 0u;
            rc = qk::launch_reg(dtype, G.d_states, G.sstride, uint32_t(G.nstates), pi.ra, G.d_ops,
                                p.pass_begin[i], p.pass_begin[i + 1], G.d_coefs, p.coef_begin[i],
                                p.coef_begin[i + 1], G.cstride, G.d_status, flags, st);
        } else {
            const uint32_t flags = (i == 0 && first_tile) ? qk::TF_INIT_ZERO : 0u;
            rc = qk::launch_tile(dtype, G.d_states, G.sstride, uint32_t(G.nstates), pi.ta, G.d_ops,
                                 p.pass_begin[i], p.pass_begin[i + 1], G.d_coefs, p.coef_begin[i],
                                 p.coef_begin[i + 1], G.cstride, &ma, flags, st);
        }
        if (rc) return rc;
    }
    if (G.c.passes.empty()) {
        if ((rc = qk::launch_init_zero(dtype, G.d_states, G.sstride, uint32_t(G.nstates), G.n, st))) return rc;
    }
    rc = qk::launch_marginal(dtype, G.d_states, G.sstride, uint32_t(G.nstates), G.n, nullptr, 0, G.d_part,
                             G.d_norm, st, G.norm_chunks);
    if (rc) return rc;
    if (G.nterms) {
        rc = qk::launch_pauli(dtype, G.d_states, G.sstride, uint32_t(G.nstates), G.n, G.d_masks,
                              int(G.nterms), G.pauli_rows, G.d_part, G.d_pauli, st, G.pauli_chunks);
        if (rc) return rc;
    }
    return QSIM_OK;
}

int enqueue_all(qsim_batch *b, hipStream_t st) {
    for (const Group &G : b->groups) {
        int rc = enqueue_group(G, b->dtype, st);
        if (rc) return rc;
    }
    return QSIM_OK;
}

}  // namespace

extern "C" {

int qsim_batch_create(const qsim_batch_group *groups, int n_groups, const qsim_batch_opts *opt,
                      qsim_batch_h *out) {
    if (!groups || n_groups <= 0 || !out) return QSIM_E_ARG;
    qsim_batch_opts o{};
    o.dtype = QSIM_C64;
    if (opt) o = *opt;
    if (o.dtype != QSIM_C64 && o.dtype != QSIM_C128) return QSIM_E_ARG;
    for (int i = 0; i < n_groups; i++) {
        const qsim_batch_group &g = groups[i];
        if (g.n < 1 || g.n > kMaxQubits || g.n_states < 1 || (g.ng && !g.g) || g.n_slots < 0 ||
            (g.params && g.n_params < 1))
            return QSIM_E_ARG;
        if (g.n_states > 65535) return QSIM_E_CAPACITY;
    }
    int rc = qk::init_kernels();
    if (rc) return rc;
    qsim_batch *b = new (std::nothrow) qsim_batch;
    if (!b) return QSIM_E_NOMEM;
    b->dtype = o.dtype;
    b->use_graph = o.use_graph != 0;
    TraceRange range("qsim_batch_create");
    const double t0 = now_seconds();
    try {
        b->groups.resize(size_t(n_groups));
        for (int i = 0; i < n_groups && !rc; i++) {
            rc = setup_group(b->groups[size_t(i)], groups[i], o.dtype, o);
            if (!rc) {
                const Group &G = b->groups[size_t(i)];
                b->info.states += G.nstates;
                b->info.input_gates += G.c.stats.input_gates * G.nstates;
                b->info.fused_ops += G.c.stats.fused_ops;
                b->info.passes += G.c.stats.passes;
                b->info.records += G.c.records;
                b->info.tune_seconds += G.tune_seconds;
                b->info.state_bytes += int64_t(G.nstates) * int64_t(G.sstride * elem_bytes(o.dtype));
                b->info.coef_bytes += G.coef_bytes;
            }
        }
    } catch (const std::bad_alloc &) {
        rc = QSIM_E_NOMEM;
    }
    b->info.compile_seconds = now_seconds() - t0;
    if (rc) { qsim_batch_destroy(b); return rc; }
    *out = b;
    return QSIM_OK;
}

int qsim_batch_run(qsim_batch_h b, void *hip_stream) {
    if (!b) return QSIM_E_ARG;
    TraceRange range("qsim_batch_run");
    hipStream_t st = (hipStream_t)hip_stream;
    if (!b->use_graph) return enqueue_all(b, st);
    if (!b->graph_exec) {
        hipStream_t cs;
        int rc = hip_ok(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "stream for capture");
        if (rc) return rc;
        rc = hip_ok(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
        if (!rc) {
            int erc = enqueue_all(b, cs);
            hipGraph_t g = nullptr;
            rc = hip_ok(hipStreamEndCapture(cs, &g), "end capture");
            if (!rc && erc) rc = erc;
            if (!rc) {
                b->graph = g;
                rc = hip_ok(hipGraphInstantiate(&b->graph_exec, g, nullptr, nullptr, 0), "graph instantiate");
            } else if (g) {
                (void)hipGraphDestroy(g);
            }
        }
        (void)hipStreamDestroy(cs);
        if (rc) return rc;
    }
    return hip_ok(hipGraphLaunch(b->graph_exec, st), "graph launch");
}

int qsim_batch_results(qsim_batch_h b, int group, int32_t *outcomes, double *probs, double *expvals,
                       double *norms, int32_t *status) {
    if (!b || group < 0 || group >= int(b->groups.size())) return QSIM_E_ARG;
    int rc = hip_ok(hipDeviceSynchronize(), "batch sync");
    if (rc) return rc;
    const Group &G = b->groups[size_t(group)];
    const size_t ns = size_t(G.nstates) * G.nslots;
    if (outcomes && ns && (rc = hip_ok(hipMemcpy(outcomes, G.d_outcomes, ns * 4, hipMemcpyDeviceToHost), "outcomes")))
        return rc;
    if (probs && ns && (rc = hip_ok(hipMemcpy(probs, G.d_probs, ns * 8, hipMemcpyDeviceToHost), "probs")))
        return rc;
    if (status && (rc = hip_ok(hipMemcpy(status, G.d_status, size_t(G.nstates) * 4, hipMemcpyDeviceToHost), "status")))
        return rc;
    std::vector<double> nrm(size_t(G.nstates));
    if ((rc = hip_ok(hipMemcpy(nrm.data(), G.d_norm, nrm.size() * 8, hipMemcpyDeviceToHost), "norms"))) return rc;
    if (norms) std::copy(nrm.begin(), nrm.end(), norms);
    if (expvals) {
        if (!G.nterms) {
            std::fill(expvals, expvals + G.nstates, 0.0);
        } else {
            std::vector<double> s(size_t(G.nstates) * G.nterms * 2);
            if ((rc = hip_ok(hipMemcpy(s.data(), G.d_pauli, s.size() * 8, hipMemcpyDeviceToHost), "pauli"))) return rc;
            for (int bb = 0; bb < G.nstates; bb++) {
                double total = 0;
                for (size_t k = 0; k < G.nterms; k++) {
                    const double re = s[(size_t(bb) * G.nterms + k) * 2], im = s[(size_t(bb) * G.nterms + k) * 2 + 1];
                    double v;
                    switch (__builtin_popcountll(G.terms[k].xmask & G.terms[k].zmask) & 3) {
                    case 0: v = re; break;
                    case 1: v = -im; break;
                    case 2: v = -re; break;
                    default: v = im; break;
                    }
                    total += G.terms[k].coeff * v;
                }
                expvals[bb] = total / nrm[size_t(bb)];
            }
        }
    }
    return QSIM_OK;
}

int qsim_batch_get_state(qsim_batch_h b, int group, int index, void *dst) {
    if (!b || !dst || group < 0 || group >= int(b->groups.size())) return QSIM_E_ARG;
    const Group &G = b->groups[size_t(group)];
    if (index < 0 || index >= G.nstates) return QSIM_E_ARG;
    int rc = hip_ok(hipDeviceSynchronize(), "batch sync");
    if (rc) return rc;
    const size_t e = elem_bytes(b->dtype);
    return hip_ok(hipMemcpy(dst, (char *)G.d_states + size_t(index) * G.sstride * e, G.sstride * e,
                            hipMemcpyDeviceToHost),
                  "get state");
}

int qsim_batch_group_stats(qsim_batch_h b, int group, qsim_apply_stats *out, int32_t *tuned_width) {
    if (!b || !out || group < 0 || size_t(group) >= b->groups.size()) return QSIM_E_ARG;
    *out = b->groups[size_t(group)].c.stats;
    if (tuned_width) *tuned_width = b->groups[size_t(group)].tuned_width;
    return QSIM_OK;
}

int qsim_batch_info_get(qsim_batch_h b, qsim_batch_info *out) {
    if (!b || !out) return QSIM_E_ARG;
    *out = b->info;
    return QSIM_OK;
}

int qsim_batch_destroy(qsim_batch_h b) {
    if (!b) return QSIM_E_ARG;
    (void)hipDeviceSynchronize();
    if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (Group &G : b->groups) free_group(G);
    delete b;
    return QSIM_OK;
}

}  // extern "C"
