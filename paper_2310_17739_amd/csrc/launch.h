// Host-callable launchers of the gfx950 kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "host.h"

namespace qk {

// Record a failed HIP call (error string and the call site) for
// qsim_last_error; returns QSIM_OK for hipSuccess, else QSIM_E_HIP.
int note_hip(hipError_t e, const char *where);

// Tile of a pass: the qubits outside the tile enumerate the tiles
// (blockIdx.x); tile position j holds qubit tq[j].  The low c qubits sit at
// positions 0..c-1 (contiguous chunks in memory); hi[] lists the other tile
// qubits in ascending order.  Positions ascend by qubit, except that an
// operator run on a thread's registers (`regs`) has its qubits at positions
// log2(threads) + off + j, the bits of the register index: the first one is
// applied to the tile as loaded, the last one as the tile leaves LDS.
struct TileArgs {
    uint64_t rest_mask;   // qubits not in the tile
    uint64_t tile_mask;   // qubits in the tile (j bit b <-> b-th lowest of them)
    int32_t n, t, c, nhi;
    int32_t threads;      // workgroup size of the tile kernel: 256 or 512
    int32_t regs;         // bit 0: the first record runs on the loaded registers; bit 1: the
                          // last one on the registers stored; bits 2-4: its register-bit offset
    uint8_t tq[16];       // qubit at tile position j
    uint8_t hi[48];
    // XCD-aware tile order: workgroup b takes the tile whose qubits xcd_q[j]
    // (outside the tile) equal bit j of b for j < nxcd, the other bits of b
    // going to the remaining outside qubits in ascending order.  Workgroups
    // are handed to the XCDs round-robin, so these qubits name the XCD (and
    // its L2) that processes an amplitude; keeping them from pass to pass
    // keeps amplitudes in one XCD's L2.
    int32_t nxcd;
    uint8_t xcd_q[4];
};

// Base index of the tile of workgroup bx (see TileArgs::xcd_q).
__host__ __device__ inline uint64_t tile_base(uint64_t bx, uint64_t rest_mask, int nxcd, const uint8_t *xcd_q) {
    uint64_t lo = 0, lomask = 0;
    for (int j = 0; j < nxcd; j++) {
        lomask |= uint64_t(1) << xcd_q[j];
        if ((bx >> j) & 1) lo |= uint64_t(1) << xcd_q[j];
    }
    uint64_t m = rest_mask & ~lomask, x = bx >> nxcd, r = 0;
    while (m && x) {
        const uint64_t low = m & (~m + 1);
        if (x & 1) r |= low;
        x >>= 1;
        m &= m - 1;
    }
    return lo | r;
}

// Measurement inputs / outputs of a batched program (per state b, slot s:
// index b * nslots + s).
struct MeasArgs {
    const double *uniforms;   // draws in [0,1)
    const int32_t *forced;    // >= 0: force this outcome (may be null)
    int32_t *outcomes;
    double *probs;            // probability of the recorded outcome
    int32_t *status;          // per state: 0, or a negative QSIM_E_* code
    int32_t *fail_at;         // per state: instruction index of the failure
    int32_t nslots;
};

enum : uint32_t { TF_INIT_ZERO = 1, TF_NO_STORE = 2 };

// Register-resident pass (records DEVOP_RMAT / SWAP / XPOSE): canonical tile
// bit c is qubit tq[c]; position p of an element index (lane bits 0..5, wave
// bits 6..logt-1, register bits logt..logt+3) holds canonical bit
// load_pos[p] as loaded and store_pos[p] as stored.  The workgroup has
// 2^(t-4) threads.  LDS: the tile (2^t elements, only for a pass with LDS
// re-layouts) and then the pass's records: lds_bytes = reg_lds_bytes(...).
struct RegArgs {
    uint64_t rest_mask;
    int32_t n, t;
    uint32_t lds_bytes;
    uint32_t flags;          // RF_NONTEMPORAL: stream the state past the caches
    uint8_t tq[16];
    uint8_t load_pos[16];
    uint8_t store_pos[16];
    int32_t nxcd;            // XCD-aware tile order, as in TileArgs
    uint8_t xcd_q[4];
};
enum : uint32_t { RF_NONTEMPORAL = 1 };

// One register-resident pass over `nstates` states spaced `sstride` apart;
// records [ob, oe) of `ops`, coefficients of state b at coefs + b * cstride;
// states whose status is nonzero are skipped; flags: TF_INIT_ZERO.
// Records [ob, oe), coefficient range [cb, ce) of
// the pass (elements; touched once at the start so that scalar reads hit L2).
size_t reg_lds_bytes(size_t elem, int t, bool relayouts, uint32_t nrec);
int launch_reg(int dtype, void *state, uint64_t sstride, uint32_t nstates, const RegArgs &ra,
               const qs::DevOp *ops, uint32_t ob, uint32_t oe, const void *coefs, uint32_t cb, uint32_t ce,
               uint64_t cstride, const int32_t *status, uint32_t flags, hipStream_t st);

// Enable > 64 KiB of dynamic LDS for the tile kernels.  Idempotent.
int init_kernels();
size_t max_lds_bytes();

// LDS bytes of a tile pass: the tile, the workgroup-reduction scratch of
// in-tile measurements (2 values x up to 8 waves, FP64), the pass's operator
// records and its coefficients.
constexpr size_t kTileRedBytes = 2 * 8 * sizeof(double);
size_t tile_lds_bytes(size_t elem, int t, uint32_t nrec, uint32_t ncoef);

// One tiled pass (or a whole resident program when t == n) over `nstates`
// states spaced `sstride` elements apart: operator records [ob, oe) whose
// coefficients occupy [cb, ce) (elements of the state dtype); the
// coefficients of state b are read at coefs + b * cstride.
int launch_tile(int dtype, void *state, uint64_t sstride, uint32_t nstates, const TileArgs &ta,
                const qs::DevOp *ops, uint32_t ob, uint32_t oe, const void *coefs, uint32_t cb,
                uint32_t ce, uint64_t cstride, const MeasArgs *ma, uint32_t flags,
                hipStream_t st);

// Whether launch_sweep applies `op` with the FP32 matrix cores (dense 4- or
// 5-qubit operators on complex64 states of at least k + 5 qubits;
// QSIM_MFMA=0 turns it off).
bool dense_mfma_ok(int dtype, int n, const qs::DevOp &op);

// One operator over the whole state (positions are global qubits); the
// coefficients of state b start at coefs + b * cstride; states whose status
// is nonzero are skipped.
int launch_sweep(int dtype, void *state, uint64_t sstride, uint32_t nstates, int n,
                 const qs::DevOp &op, const void *coefs, hipStream_t st, uint64_t cstride = 0,
                 const int32_t *status = nullptr);

// Measurement / assertion / reset / measurement-then-reset of qubit q in
// every state of a batch from per-state weights p01[2b], p01[2b+1] (a
// marginal reduction), decided on the device (kind: qs::DEVOP_*).
int launch_decide(int dtype, void *state, uint64_t sstride, uint32_t nstates, int n, int q,
                  int kind, int slot, const double *p01, const MeasArgs &ma, hipStream_t st);

// Binding of parameterised operator coefficients (see k_bind).
struct BindEntry {
    uint32_t bound_off;   // offset in a state's bound coefficient array (elements)
    uint32_t count;       // coefficients of the operator (terms * 2^k)
    uint32_t tmpl_off;    // offset of block 0 in the FP64 template (complex elements)
    int32_t np;           // angle slots (0..3)
    int32_t slot[3];
    int32_t pad;
};
int launch_bind(int dtype, const double *tmpl, const BindEntry *ents, uint32_t nents,
                const double *params, int nparams, void *out, uint64_t cstride, uint32_t nstates,
                uint32_t max_count, hipStream_t st);

int launch_fill_i32(int32_t *p, int32_t v, uint64_t n, hipStream_t st);

// Sampling: per-block inclusive prefix sums of |a_x|^2 into cum[2^n] and
// block totals into bsum[scan_blocks(n)]; then, with boff the exclusive
// prefix of the block totals, finish the sums and search each shot.
uint64_t scan_blocks(int n);
int launch_blockscan(int dtype, const void *state, int n, double *cum, double *bsum, hipStream_t st);
int launch_addoff_search(double *cum, int n, const double *boff, const double *u, uint64_t m,
                         uint64_t *out, hipStream_t st);

// Streaming copy of `bytes` (a multiple of 16) from src to dst (dst == src
// allowed) in 64 KiB blocks, one workgroup each, block b handled by
// workgroup (b - rotate) mod blocks; plain or non-temporal loads and stores.
int launch_stream_copy(void *dst, const void *src, uint64_t bytes, bool nontemporal, uint32_t rotate,
                       hipStream_t st);

// |0...0> in every state of a batch.
int launch_init_zero(int dtype, void *state, uint64_t sstride, uint32_t nstates, int n,
                     hipStream_t st);

// Marginal weights: for every bin j of the qubits qs[0..nqs-1] (j = sum_i
// bit(qs[i]) 2^i), sum of |a_x|^2 over x with those bits; FP64, fixed order.
// Writes partial sums to `partials` ([nstates][2^nqs][nchunks]) and the
// final sums to `out` ([nstates][2^nqs]).
int launch_marginal(int dtype, const void *state, uint64_t sstride, uint32_t nstates, int n,
                    const int *qs, int nqs, double *partials, double *out, hipStream_t st,
                    uint32_t nchunks = 0);
uint32_t marginal_chunks(int n, int nqs);

// The marginal of qubits qs[0..nqs-1] normalised by its total, written to
// device memory dev_out (2^nqs doubles), with the reduction partials in a
// fixed per-device scratch array instead of an allocated buffer (at most
// 2^17 partials: for nqs > 8 the state is cut into fewer chunks than
// launch_marginal would use).  Calls that overlap on one device race on the
// scratch.
int launch_probs_noalloc(int dtype, const void *state, int n, const int *qs, int nqs, double *dev_out,
                         hipStream_t st);

// Pauli-term overlaps S_k = sum_x (-1)^{popcount(x & z_k)} conj(a[x ^ x_k]) a[x]
// (complex, FP64), written as out[(b * nterms + k) * 2 + {0,1}].  Terms that
// share an X mask share one read of the state: pauli_rows builds the device
// table (the zmask of every term, then rows of up to kPauliRow terms with a
// common X mask: xmask, count, term indices).  Rows are ordered by the
// kernel width that serves them (5-8 terms, 3-4, 2, 1), so that a row pays
// only for the accumulators it uses; `bucket` holds the row count of each.
constexpr int kPauliRow = 8;
struct PauliRows {
    uint32_t rows = 0;
    uint32_t bucket[4] = {0, 0, 0, 0};   // rows served by widths 8, 4, 2, 1
};
PauliRows pauli_rows(const qsim_pauli *t, size_t nt, std::vector<uint64_t> *table);
int launch_pauli(int dtype, const void *state, uint64_t sstride, uint32_t nstates, int n,
                 const uint64_t *table, int nterms, const PauliRows &rows, double *partials,
                 double *out, hipStream_t st, uint32_t nchunks = 0);
uint32_t pauli_chunks(int n);

// Keep the half with bit q == outcome, scale it by `scale`, zero the other.
int launch_collapse(int dtype, void *state, int n, int q, int outcome, double scale,
                    hipStream_t st);

}  // namespace qk
