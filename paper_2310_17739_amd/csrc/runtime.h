// Compiled circuits and their device tables (shared by the single-state
// calls, the batched form and the server).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "host.h"
#include "launch.h"

namespace qs {

struct PassInfo {
    int kind = Pass::TILE;      // Pass::TILE, STRIDED or MEASURE
    bool strided = false;
    qk::TileArgs ta{};
    bool reg = false;           // register-resident tiled pass (k_reg)
    qk::RegArgs ra{};
    MeasRec meas;               // MEASURE passes
};

struct Compiled {
    PackedPlan plan;
    std::vector<PassInfo> passes;
    qsim_apply_stats stats{};
    int64_t stats_reg_swaps = 0, stats_reg_xposes = 0;   // register-resident passes
    int64_t records = 0;   // measurement, assertion and reset records after folding
};

// Device copies of a packed plan with a pinned staging buffer.
struct DeviceTables {
    DevOp *d_ops = nullptr;
    size_t cap_ops = 0;
    void *d_coefs = nullptr;
    size_t cap_coefs = 0;
    void *h_stage = nullptr;
    size_t cap_stage = 0;
    hipEvent_t stage_ev = nullptr;
    bool stage_ev_valid = false;
};

size_t elem_bytes(int dtype);
int env_int(const char *name, int dflt);
int resident_max(int dtype);
// Default tile width for passes over `nstates` states of n qubits
// (QSIM_TILE_QUBITS overrides it).
int default_tile_qubits(int n, int dtype, uint64_t nstates);
void default_configs(int n, int dtype, const qsim_fuse_opts *opt, FuseConfig *fc, PlanConfig *pc);
int compile_circuit(int n, int dtype, const qsim_gate *g, size_t ng, const GateInputs &in,
                    const qsim_fuse_opts *opt, Compiled *out);
// General form: keep_params keeps slot >= 0 angles symbolic (cos/sin basis
// blocks, at most max_params per fused operator); allow_meas accepts
// MEASURE / ASSERT0 / RESET records.
int compile_program(int n, int dtype, const qsim_gate *g, size_t ng, const GateInputs &in,
                    bool keep_params, bool allow_meas, int max_params,
                    const qsim_fuse_opts *opt, Compiled *out);
int validate_plan(int n, int dtype, const Compiled &c);
// Time fusion widths 2..5 (complex128: 2..4) for this circuit on a scratch
// state of width n (allocated and freed here), each compiled with `base`
// otherwise; writes the fastest width and its time per input gate.
int tune_width(int n, int dtype, const qsim_gate *g, size_t ng, const GateInputs &in,
               const qsim_fuse_opts *base, int *best_w, double *best_ns);
// Time tile widths 12 and 13 for a batch group's template (the other options
// from `base`, fusion width included) over a sample of up to `nstates` states
// run together, as the batch runs them; writes the faster width (base's tile
// width for groups whose states fit one tile, which are not timed).
int tune_tile_batch(int n, int dtype, const qsim_gate *g, size_t ng, const GateInputs &in,
                    const qsim_fuse_opts &base, uint32_t nstates, int *best_t);
int upload_plan(DeviceTables *dt, int dtype, const PackedPlan &plan, hipStream_t st);
void free_tables(DeviceTables *dt);
// (sstride, nstates: the same passes over nstates states laid out every
// sstride elements, all with the plan's coefficients)
int enqueue_passes(const Compiled &c, const DeviceTables &dt, int dtype, void *state,
                   hipStream_t st, bool init_zero_first, uint64_t sstride = 0, uint32_t nstates = 1);

}  // namespace qs
