// Internal host-side types of the simulator library: lowered and fused
// operators, pass plans and the packed device tables.
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "qsim.h"

namespace qs {

using cd = std::complex<double>;

constexpr int kMaxK = 5;          // widest operator (2^5 x 2^5)
constexpr int kMaxQubits = 40;

// A k-qubit operator on ascending qubits q[0] < ... < q[k-1].  The matrix is
// 2^k x 2^k row-major with local index bit j <-> qubit q[j].
//
// Parameterised operators (templates for batched runs) carry `np` angle
// slots.  Every rotation R_P(theta) = cos(theta/2) I - i sin(theta/2) P is
// linear in (cos theta/2, sin theta/2), so an operator holding np rotations
// is a sum over s in {0,1}^np of prod_j (s_j ? sin : cos)(theta_j / 2) times
// a fixed matrix; `m` then stores the 2^np basis matrices one after another.
struct Op {
    int k = 0;
    int q[kMaxK] = {0, 0, 0, 0, 0};
    int np = 0;                 // number of angle slots
    int slot[3] = {-1, -1, -1}; // parameter-vector indices
    std::vector<cd> m;          // (1 << np) * 4^k entries
    int src_kind = -1;          // originating gate kind for unfused ops
    int orient = 0;             // 2-qubit gates: 1 if the record named the pair descending
    bool dead = false;

    int dim() const { return 1 << k; }
    uint64_t mask() const {
        uint64_t r = 0;
        for (int j = 0; j < k; j++) r |= uint64_t(1) << q[j];
        return r;
    }
};

// A measurement, assertion or reset record of a program: it runs after the
// operators of epoch `epoch` and before those of epoch + 1.
struct MeasRec {
    int epoch = 0;
    int kind = 0;   // DEVOP_MEASURE, DEVOP_ASSERT0, DEVOP_RESET or DEVOP_MEASURE_RESET
    int q = 0;
    int slot = 0;
};

// A lowered circuit: operators in order, each with its epoch (barriers and
// measurement records start a new epoch; fusion never crosses epochs).
struct Lowered {
    std::vector<Op> ops;
    std::vector<int> op_epoch;
    std::vector<MeasRec> meas;
    int n_epochs = 1;
    int64_t input_gates = 0;
};

struct FuseConfig {
    int level = 5;
    int max_width = 4;
    double lds_cost = 3.0;     // cost of one extra operator, in complex MACs per amplitude
    int max_params = 2;        // angle slots per fused operator (templates)
    bool sparse = true;
};

// ---- OpenQASM 2.0 frontend (qasm.cpp)
// Parses the program into gate records; on error returns the status and a
// message naming the line in *err.
int parse_qasm(const char *text, size_t len, std::vector<qsim_gate> *out, int *n_qubits, int *n_clbits,
               std::string *err);

// ---- lowering (gates.cpp)
// Returns QSIM_OK or an error; fills `out`.  Gate matrices are built in FP64.
// Measurement records are accepted only with `allow_meas`.
// The caller's matrix pool and parameter vector with their lengths: a MAT
// record needs mat_off + 4^k <= n_mats (complex entries), a record with
// slot >= 0 needs slot < n_params.
struct GateInputs {
    const double *mats = nullptr;
    size_t n_mats = 0;
    const double *params = nullptr;
    size_t n_params = 0;
};
int lower(int n, const qsim_gate *g, size_t ng, const GateInputs &in, bool keep_params,
          bool allow_meas, Lowered *out);
// Dense matrix of one gate record on its own qubits in record order.
int gate_matrix(const qsim_gate &g, const double *theta, std::vector<cd> *m);

// ---- fusion (fuse.cpp)
// Applies the fusion levels in place; counts[l] = operator count after
// level l (for l <= cfg.level).
void fuse(int n, Lowered *L, const FuseConfig &cfg, int64_t counts[6]);
// Helpers shared by fusion and packing.
void embed(const Op &a, const int *uq, int uk, std::vector<cd> *out, int basis);
int xor_terms(const cd *m, int k, double tol, uint32_t *present);
double max_abs(const cd *m, size_t n);

// ---- planning (plan.cpp)
struct Pass {
    enum Kind { TILE = 0, STRIDED = 1, MEASURE = 2 };
    int kind = TILE;
    MeasRec meas;                 // MEASURE passes (tiled programs)
    std::vector<MeasRec> inline_meas;   // resident passes: records after ops[inline_at[i]] ...
    std::vector<int> seq;         // resident passes: order of items, >= 0 op index, < 0 ~meas index
    int t = 0;                    // tile qubits
    int c = 0;                    // contiguous low qubits (0..c-1) in the tile
    uint64_t tile_mask = 0;       // all tile qubits
    int nhi = 0;
    int hi[kMaxQubits] = {0};     // tile qubits >= c, ascending
    std::vector<int> ops;         // operator indices (into the fused list)
    bool strided = false;         // one operator applied by the strided sweep
    uint8_t tq[16] = {0};         // tiled passes: qubit at tile position j
    bool first_in_regs = false;   // the first operator runs on the loaded registers
    bool last_in_regs = false;    // the last operator runs on the registers stored
    int last_off = 0;             // its first register-index bit
    // register-resident passes (see pack_reg_pass): the tile lives in the
    // threads' registers; position p of an element index (lane bits 0..5,
    // wave bits 6..logt-1, register bits logt..t-1) holds canonical tile
    // bit load_pos[p] as loaded and store_pos[p] as stored (canonical bit c
    // is the c-th smallest tile qubit)
    bool reg = false;
    int reg_logt = 0;
    uint8_t load_pos[16] = {0};
    uint8_t store_pos[16] = {0};
    int reg_swaps = 0, reg_xposes = 0;
    int nxcd = 0;                 // XCD-aware tile order (see qk::TileArgs)
    uint8_t xcd_q[4] = {0};
};

struct PlanConfig {
    int tile_qubits = 12;
    int low_qubits = 3;
    int window = 1024;            // lookahead when filling a pass
    int max_tile_k = 5;           // widest operator the tile kernel applies
    size_t meta_budget = 16384;   // bytes of a pass's operator records and coefficients
    int threads = 512;            // tile kernel workgroup size (256 or 512)
    bool one_op_per_pass = false;
    bool full_support = false;    // every qubit of an operator in its tile
    bool first_in_regs = true;    // apply a pass's first operator before the tile reaches LDS
    bool reg_engine = false;      // tiled passes of 10..13 qubits run register-resident
    bool reg_coalesce = true;     // restore the low qubits to lane bits 0..c-1 before the store
    bool xcd_order = true;        // XCD-aware tile order across passes
};

// Choose, for every tiled pass, the outside qubits that name a tile's XCD
// (Pass::xcd_q): those of the previous pass while they stay outside the
// tile, otherwise the outside qubits that stay outside longest.
void place_xcd_qubits(int n, std::vector<Pass> *passes);

// Register bits of a register-resident pass: each thread holds 2^kRegBits
// amplitudes, so a tile of t qubits takes 2^(t - kRegBits) threads.
constexpr int kRegBits = 4;
inline int reg_threads_for(int t) { return (t >= 10 && t <= 13) ? (1 << (t - kRegBits)) : 0; }

// meta_bytes[i]: LDS bytes operator i needs in a tiled pass (record +
// coefficients at the state precision); need[i]: the qubits operator i must
// have inside its tile (all of its qubits, or only those some XOR shift of it
// moves).  Measurement records of L.meas are placed between epochs: inside
// resident passes (t == n) as records, as passes of their own otherwise.
void plan_passes(int n, const Lowered &L, const std::vector<uint32_t> &meta_bytes,
                 const std::vector<uint64_t> &need, const PlanConfig &cfg, std::vector<Pass> *passes);

// Tile positions of the tiled passes (t < n).  Positions ascend by qubit
// (the low c qubits at 0..c-1).  With `first_in_regs`, a tiled pass whose
// tile spans more than 2^logt elements gets a first operator that the tile
// kernel applies to a thread's registers as loaded: an operator of the pass
// that commutes with every operator before it, touches no low qubit and has
// at most min(t - logt, max_k) qubits in the tile moves to the front, and its
// tile qubits take positions logt, logt + 1, ... (the bits of a thread's
// register index).  Likewise an operator that commutes with every operator
// after it moves to the end, its tile qubits (disjoint from the first one's)
// on the next register-index bits: the kernel applies it to the tile as it
// leaves LDS.
void place_positions(int n, const std::vector<Op> &ops, int logt, int max_k, bool first_in_regs,
                     std::vector<Pass> *passes);

// Widest operator the tile kernel applies to a thread's registers (also
// bounded by the register-index bits of the tile, t - log2(threads)).
inline int first_regs_max_k(int) { return 4; }

// ---- packing into device tables (plan.cpp)
// Device operator record (32 bytes, read as eight scalar words): see kernels.hip.
struct DevOp {
    uint32_t coef;     // offset of the first coefficient (complex elements)
    uint32_t present;  // bit m set: the XOR-shift-m diagonal over the k positions is nonzero
    uint8_t k;         // qubits addressed by position (tile-local in tiled passes, global in strided)
    uint8_t pos[5];    // their positions, ascending
    uint8_t kind;      // DEVOP_*
    uint8_t kx;        // tiled passes: further qubits, outside the tile, on which the operator is diagonal
    uint16_t slot[5];  // tiled passes: LDS slot offset of position j's bit, lds_slot(1 << pos[j])
    uint8_t xq[5];     // their qubit numbers, ascending; bit j of the tile's base index is bit k + j
                       // of the operator's local index and selects the coefficient block
    uint8_t pad;
};
static_assert(sizeof(DevOp) == 32, "DevOp layout");

// Coefficients of one record: for each of the 2^kx blocks, each present
// shift's 2^k diagonal entries.
inline uint32_t devop_coefs(const DevOp &o) { return uint32_t(__builtin_popcount(o.present)) << (o.k + o.kx); }

enum { DEVOP_MAT = 0, DEVOP_MEASURE = 1, DEVOP_ASSERT0 = 2, DEVOP_RESET = 3,
       // register-resident passes:
       DEVOP_RMAT = 4,    // operator on the kRegBits register bits: present = register XOR
                          // shifts, k = kRegBits, coefficients 2^k per shift, kx / xq block qubits
       DEVOP_SWAP = 5,    // pos[0] = lane bit (4 or 5), pos[1] = register bit: exchange them
       DEVOP_XPOSE = 6,   // LDS re-layout; bytes 0..13 = canonical bit per position before,
       DEVOP_XPOSE2 = 7,  // and, in the record that follows, after
       DEVOP_MEASURE_RESET = 8   // a measurement followed by a reset of the same qubit
};
inline bool devop_is_mat(int kind) { return kind == DEVOP_MAT || kind == DEVOP_RMAT; }
inline bool devop_is_record(int kind) {
    return kind == DEVOP_MEASURE || kind == DEVOP_ASSERT0 || kind == DEVOP_RESET || kind == DEVOP_MEASURE_RESET;
}

struct PackedPlan {
    std::vector<DevOp> ops;             // in pass order
    std::vector<uint32_t> pass_begin;   // op range of pass i: [pass_begin[i], pass_begin[i+1])
    std::vector<uint32_t> coef_begin;   // coefficient range of pass i, likewise
    std::vector<cd> coefs;              // FP64 coefficients; cast on upload
    std::vector<int8_t> op_np;          // per record: angle slots of its operator
    std::vector<int32_t> op_slots;      // per record: 3 slot indices
    int64_t terms = 0;
};

// Shifts m whose XOR diagonal M[r][r ^ m] is nonzero in some basis block
// (all shifts when `sparse` is false).
uint32_t op_present(const Op &o, bool sparse);

// Qubits of `o` that some present XOR shift moves (its off-diagonal support).
uint64_t op_moved_qubits(const Op &o, uint32_t present);

// Pack fused ops into device records following `passes`.  In a tiled pass an
// operator's qubits outside the tile become its block qubits (kx, xq), which
// requires it to be diagonal on them.  For parameterised ops the coefficient
// layout holds the 2^np basis blocks (a bind step combines them).  Returns
// QSIM_OK, or QSIM_E_ARG if a tiled pass leaves a moved qubit outside its tile.
int pack_plan(const std::vector<Op> &ops, const std::vector<uint32_t> &present,
              std::vector<Pass> &passes, const PlanConfig &cfg, PackedPlan *out);

// Register program of one tiled pass (regplan.cpp): appends the pass's
// records and coefficients to `out` and sets p.load_pos / p.store_pos.
// Every operator runs on the register bits: before it, qubits it needs that
// sit on lane bits 4 or 5 are swapped in (DEVOP_SWAP), others are brought in
// by an LDS re-layout (DEVOP_XPOSE pair), which also chooses the qubits the
// next operators need (furthest next use leaves first).  Returns QSIM_OK or
// QSIM_E_ARG for an operator the pass cannot hold.
int pack_reg_pass(const std::vector<Op> &ops, const std::vector<uint32_t> &present, Pass &p,
                  bool coalesce, PackedPlan *out);

double now_seconds();

// A named host range for profilers (roctx; `rocprofv3 --marker-trace` lists
// them): pushed when constructed, popped when it leaves scope.  Ranges nest
// per thread.  With no profiler attached a push and a pop cost a few tens of
// nanoseconds, so they mark library calls and compile stages, not launches.
struct TraceRange {
    explicit TraceRange(const char *name);
    ~TraceRange();
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

// Allocation-failure injection for tests (qsim_debug_fail_alloc): true when
// this allocation attempt is the one set to fail.  Every device and pinned
// allocation of the library, and the start of every compile (standing for
// its host allocations), asks once.
bool alloc_fault();

}  // namespace qs
