/*
 * qsim.h -- C ABI of the MI355X state-vector simulator.
 *
 * The library applies long sequences of 1- and 2-qubit gates (and k <= 5
 * qubit gates) to a 2^n-amplitude complex state held in device memory, with
 * gate fusion, simulated mid-circuit measurement and measurement assertion,
 * and FP64 observables.  Section numbers below are those of the paper
 * "Deep Quantum Circuit Simulations of Low-energy Nuclear States"
 * (arXiv:2310.17739).
 *
 * General rules
 *  - Every call returns an int status: QSIM_OK (0) or a negative QSIM_E_*.
 *    No C++ exception crosses this boundary.  On error the state is left as
 *    it was before the call (batched and served runs report per-state
 *    status instead).
 *  - A state handle is not thread-safe; distinct handles may be used from
 *    distinct threads.
 *  - Host arrays passed in (gates, matrices, parameters, terms) are owned by
 *    the caller and are copied before the call returns.
 *  - Device buffers passed in (the state) are owned by the caller (in the
 *    Python binding: a torch tensor) and must outlive the handle.
 *  - qsim_apply is asynchronous on the handle's stream.  Calls that return
 *    host values (measure, reset, expval, probs, norm, get_state) synchronise
 *    that stream.
 *
 * Conventions
 *  - Amplitude index i = sum_q b_q 2^q: qubit q is bit q (Section 3.2,
 *    Eq. (1q-op) pairs a[s] with a[s + 2^q]).
 *  - State storage is interleaved (re, im): complex64 (2 x float) or
 *    complex128 (2 x double), contiguous, 2^n elements.
 *  - A gate record on qubits (q[0], ..., q[k-1]) defines its matrix on the
 *    local index r = sum_j bit(q[j]) 2^j.  Controlled gates list their
 *    controls first and their target last.  R_P(theta) = exp(-i theta P/2).
 */
#ifndef QSIM_H
#define QSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qsim_state *qsim_h;

/* state storage precision */
enum { QSIM_C64 = 1, QSIM_C128 = 2 };

/* status codes */
enum {
    QSIM_OK = 0,
    QSIM_E_ARG = -1,          /* bad argument (non-finite angle, u outside [0,1), mask >= 2^n ...) */
    QSIM_E_QUBIT = -2,        /* qubit >= n, or repeated inside one gate */
    QSIM_E_NOMEM = -3,        /* device or host allocation failed */
    QSIM_E_ZERO_PROB = -4,    /* assertion of an outcome whose probability is exactly 0 */
    QSIM_E_NOT_DEFINITE = -5, /* reset of a qubit that is in superposition */
    QSIM_E_HIP = -6,          /* HIP runtime error */
    QSIM_E_CAPACITY = -7,     /* state or request larger than the buffer / pool */
    QSIM_E_UNSUPPORTED = -8   /* gate kind or option not supported */
};

/* Gate kinds: the OpenQASM 2.0 table of Section 4.1 (Table 3), a general
 * matrix record, and the non-unitary records of Listing 1 (Section 4.3). */
enum {
    QSIM_G_ID = 0, QSIM_G_H = 1, QSIM_G_X = 2, QSIM_G_Y = 3, QSIM_G_Z = 4,
    QSIM_G_S = 5, QSIM_G_SDG = 6, QSIM_G_T = 7, QSIM_G_TDG = 8, QSIM_G_SX = 9,
    QSIM_G_RX = 10, QSIM_G_RY = 11, QSIM_G_RZ = 12, QSIM_G_U1 = 13,
    QSIM_G_U2 = 14, QSIM_G_U3 = 15,
    QSIM_G_CX = 20, QSIM_G_CY = 21, QSIM_G_CZ = 22, QSIM_G_CH = 23,
    QSIM_G_SWAP = 24, QSIM_G_CRX = 25, QSIM_G_CRY = 26, QSIM_G_CRZ = 27,
    QSIM_G_CU1 = 28, QSIM_G_CU3 = 29, QSIM_G_RXX = 30, QSIM_G_RZZ = 31,
    QSIM_G_CCX = 40, QSIM_G_CSWAP = 41,
    QSIM_G_RCCX = 42,     /* relative-phase Toffoli (OpenQASM rccx): CCX up to a diagonal */
    QSIM_G_RC3X = 43,     /* relative-phase 3-controlled X (OpenQASM rc3x) */
    QSIM_G_C3X = 44, QSIM_G_C3XSQRTX = 45,
    QSIM_G_C4X = 46,
    QSIM_G_MAT = 50,      /* 2^nq x 2^nq complex128 matrix from the pool */
    QSIM_G_BARRIER = 60,  /* fusion fence */
    QSIM_G_MEASURE = 61,  /* Born-rule measurement (batched programs only) */
    QSIM_G_RESET = 62,    /* reset of a definite qubit (batched programs only) */
    QSIM_G_ASSERT0 = 63   /* measurement assertion of outcome 0 (batched programs only) */
};

/* One gate record (56 bytes). */
typedef struct qsim_gate {
    uint16_t kind;     /* QSIM_G_* */
    uint16_t nq;       /* qubits named in q[] (1..5) */
    int32_t q[5];      /* qubits: controls first, target last */
    int32_t slot;      /* -1: theta[] literal.  >= 0 on a rotation: theta[0]
                          is read from the per-circuit parameter vector at
                          this index.  On MEASURE / ASSERT0: the measurement
                          slot (index of its uniform draw and its outputs). */
    uint32_t mat_off;  /* MAT: offset, in complex entries, into the pool */
    double theta[3];   /* angles in radians */
} qsim_gate;

/* One Pauli-sum term: letter on qubit j is I (x=0,z=0), X (1,0), Z (0,1)
 * or Y (1,1) for the bits j of xmask and zmask. */
typedef struct qsim_pauli {
    double coeff;
    uint64_t xmask;
    uint64_t zmask;
} qsim_pauli;

/* Fusion and pass-planning options.  NULL selects the tuned defaults. */
typedef struct qsim_fuse_opts {
    int32_t level;       /* 0 none; 1 F1 (1q+1q); 2 F1+F3 (2q absorbs 1q);
                            3 = 2 + F2 on identically ordered pairs;
                            4 = 2 + SWAP normalisation + F2 (the paper's
                            strategy, Section 4.2, Fig. 4);
                            5 = 4 + cost-driven fusion into k <= max_width
                            qubit operators (default) */
    int32_t max_width;   /* 2..5 (complex128 is limited to 4); 0 = default */
    int32_t tile_qubits; /* qubits per LDS tile; 0 = default for n and dtype */
    int32_t flags;       /* QSIM_F_* */
    float op_cost;       /* fusion cost of one more operator, in complex MACs
                            per amplitude; 0 = default (3) */
    int32_t low_qubits;  /* contiguous low qubits in every tile; 0 = default
                            (4 for complex64, 3 for complex128) */
} qsim_fuse_opts;

enum {
    QSIM_F_ONE_OP_PER_PASS = 1,  /* every fused operator is its own full-state sweep */
    QSIM_F_NO_SPARSE = 2,        /* treat fused operators as dense (no zero skipping) */
    QSIM_F_FULL_SUPPORT = 4,     /* keep every qubit of an operator in its LDS tile
                                    (default: qubits on which the operator is
                                    diagonal may stay outside the tile) */
    QSIM_F_REG_ENGINE = 8        /* tiled passes of 10..13 qubits keep the tile in
                                    registers: operators run on a thread's register
                                    bits, qubits reach those bits through lane
                                    exchanges (v_permlane16/32_swap) or LDS
                                    re-layouts (also: QSIM_REG_ENGINE=1) */
};

/* Counters of the last qsim_apply (host-side compile and device plan). */
typedef struct qsim_apply_stats {
    int64_t input_gates;      /* gate records, barriers excluded */
    int64_t ops_after[6];     /* operators after fusion level 0..5 (those computed) */
    int64_t fused_ops;        /* operators executed */
    int64_t passes;           /* full-state read+write passes enqueued */
    int64_t terms;            /* sum over operators of their nonzero XOR diagonals */
    int64_t bytes_moved;      /* algorithmic HBM bytes of the passes: passes * 2 * 2^n * elem */
    double compile_seconds;   /* host time spent lowering, fusing, planning, packing */
    int32_t tile_qubits;      /* tile size used */
    int32_t max_width;        /* fusion width used */
    int64_t reg_passes;       /* passes whose tile stays in registers */
    int64_t reg_swaps;        /* lane/register exchanges in those passes */
    int64_t reg_relayouts;    /* LDS re-layouts in those passes */
} qsim_apply_stats;

/* ------------------------------------------------------------------ core */

/* Bind a state to a caller-owned device buffer of at least 2^n elements
 * (8 bytes each for QSIM_C64, 16 for QSIM_C128) and set it to |0...0>.
 * `hip_stream` is a hipStream_t (NULL = default stream).  1 <= n <= 40.
 * Errors: QSIM_E_ARG, QSIM_E_CAPACITY (buffer too small), QSIM_E_NOMEM. */
int qsim_create(int n, int dtype, void *dev_buf, size_t buf_bytes,
                void *hip_stream, qsim_h *out);
int qsim_destroy(qsim_h h);
int qsim_set_stream(qsim_h h, void *hip_stream);
int qsim_init_zero(qsim_h h);   /* |0...0>, asynchronous */

/* Apply U_{m-1} ... U_0 (Section 3.2) given as gate records.  MAT records
 * read their matrices from `mats` (interleaved complex128, n_mats complex
 * entries; a k-qubit record needs mat_off + 4^k <= n_mats); records with
 * slot >= 0 read theta[0] from `params` (slot < n_params).  Both arrays stay
 * the caller's and are read before the call returns.  BARRIER records fence
 * fusion.
 * MEASURE / RESET / ASSERT0 records are rejected (QSIM_E_UNSUPPORTED): use
 * the calls below, or qsim_batch_* for programs with device-side decisions.
 * Errors: QSIM_E_QUBIT, QSIM_E_ARG, QSIM_E_UNSUPPORTED, QSIM_E_NOMEM,
 * QSIM_E_HIP.  Asynchronous. */
int qsim_apply(qsim_h h, const qsim_gate *g, size_t ng, const double *mats, size_t n_mats,
               const double *params, size_t n_params, const qsim_fuse_opts *opt);
int qsim_last_stats(qsim_h h, qsim_apply_stats *out);

/* Born-rule measurement of qubit q (Section 4.3): P0, P1 are reduced in
 * FP64, p0 = P0/(P0+P1), outcome = (u < p0) ? 0 : 1, the state is projected
 * and renormalised to unit norm (scale computed in FP64).  u in [0,1).
 * Writes the outcome and its probability.  Synchronous. */
int qsim_measure(qsim_h h, int q, double u, int *outcome, double *p_outcome);

/* Measurement assertion (Section 4.3).  The paper asserts that the
 * ancilla reads 0 (want = 0); want = 1 asserts the other outcome, as a
 * filter step that keeps the |1> branch would.  If P(q = want) > 0 the
 * outcome is taken as `want`, the state is projected and renormalised (FP64
 * scale) and P(q = want) / (P0 + P1) is written to *p_want; otherwise
 * QSIM_E_ZERO_PROB and the state is untouched.  want not in {0, 1}:
 * QSIM_E_ARG.  Synchronous. */
int qsim_measure_assert(qsim_h h, int q, int want, double *p_want);

/* Reset (Listing 1): identity if qubit q is |0>, X if it is |1>;
 * QSIM_E_NOT_DEFINITE (state untouched) if it is in superposition. */
int qsim_reset(qsim_h h, int q);

/* Energy of a Hamiltonian given as a Pauli sum: the energies of Table 7 are
 * such expectation values of the state the circuit prepares (Section 2:
 * H written as a sum of Pauli strings).  Computes <psi|H|psi> / <psi|psi>
 * for H = sum_k coeff_k P_k with P|x> = i^{#Y} (-1)^{popcount(x & zmask)}
 * |x ^ xmask> (a Y on qubit q sets both mask bits), accumulated in FP64 with
 * a fixed reduction order.  t: nt caller-owned terms; masks must be < 2^n
 * and coefficients finite (QSIM_E_ARG).  Writes one double.  Synchronous. */
int qsim_expval(qsim_h h, const qsim_pauli *t, size_t nt, double *out);

/* Born-rule marginal distribution of a qubit subset (Section 4.3: after
 * the assertions, the final state's probabilities are what the shots are
 * drawn from).  out[j], j = sum_i bit(qs[i]) 2^i, is the weight of the
 * basis states with those bits, normalised by <psi|psi> and reduced in FP64.
 * qs: nqs distinct qubits (0 <= nqs <= 12; QSIM_E_QUBIT otherwise); out:
 * 2^nqs caller-owned doubles.  QSIM_E_ZERO_PROB for the zero vector.
 * Synchronous. */
int qsim_probs(qsim_h h, const int *qs, int nqs, double *out);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): qsim_probs without any
 * allocation and without host synchronisation.  Same inputs and checks as
 * qsim_probs; the 2^nqs probabilities go to `dev_out`, caller-owned device
 * memory, asynchronously on the handle's stream (read them after that stream
 * is synchronised).  The reduction partials live in a fixed device array of
 * 2^17 + 4096 doubles (about 1 MiB), one per GPU, held until the process
 * ends; up to 8 qubits the reduction order, and so every bit of the result,
 * equals qsim_probs, and above 8 the state is cut into fewer chunks.  All
 * calls on one GPU share that array: calls that overlap on a GPU (other
 * streams, other threads) race and must be serialised by the caller.  The
 * zero vector gives NaN entries (0/0) instead of QSIM_E_ZERO_PROB.  Errors:
 * QSIM_E_ARG, QSIM_E_QUBIT, QSIM_E_HIP. */
int qsim_probs_noalloc(qsim_h h, const int *qs, int nqs, double *dev_out);

/* <psi|psi> in FP64: the squared norm that renormalisation after a
 * projective measurement divides by (Section 4.3); for complex64 states it
 * also shows the rounding drift of the sweeps.  Synchronous. */
int qsim_norm(qsim_h h, double *out);

/* Copy the 2^n amplitudes of the state vector (Section 3.2: amplitude i
 * holds the coefficient of basis state i, qubit q being bit q of i) to or
 * from host memory: 2^n caller-owned elements of the state dtype
 * (interleaved re, im).  Synchronous. */
int qsim_get_state(qsim_h h, void *host_dst);
int qsim_set_state(qsim_h h, const void *host_src);

/* ------------------------------------------------- compiled programs */

/* A circuit compiled once (lowering, fusion, pass plan) with its operator
 * tables resident in device memory, replayable on any state of the same
 * width and dtype.  qsim_apply is compile + run + free. */
typedef struct qsim_program *qsim_prog;

/* Compile and upload (synchronous).  Same inputs and errors as qsim_apply. */
int qsim_compile(int n, int dtype, const qsim_gate *g, size_t ng, const double *mats,
                 size_t n_mats, const double *params, size_t n_params,
                 const qsim_fuse_opts *opt, qsim_prog *out);
/* Enqueue the program's passes on the handle's stream (asynchronous).
 * QSIM_E_ARG if the width or dtype differ from the handle's. */
int qsim_run(qsim_h h, qsim_prog p);
/* Capture the program's launches on `h` into a HIP graph (enable = 1) so that
 * qsim_run replays the graph; enable = 0 drops the graph.  The graph is tied
 * to h's state buffer. */
int qsim_program_graph(qsim_prog p, qsim_h h, int enable);
/* Enqueue the passes with a HIP event pair around every launch; after the
 * stream is synchronised, qsim_program_kernel_ms returns the summed
 * kernel time (ms) of the last timed run and the number of launches. */
int qsim_run_timed(qsim_h h, qsim_prog p);
int qsim_program_kernel_ms(qsim_prog p, double *ms, int64_t *launches);
int qsim_program_stats(qsim_prog p, qsim_apply_stats *out);
int qsim_program_destroy(qsim_prog p);

/* -------------------------------------------------- batched programs */

/* Many states run the same program in one device-side schedule: the
 * trajectories of a circuit with mid-circuit measurements (Section 4.3:
 * without measurement assertion every shot is its own run), or many
 * parameter sets of one circuit template.  A group is a set of states of
 * one width sharing a program; a batch holds several groups.  Programs may
 * contain MEASURE, ASSERT0 and RESET records: the decision is taken on the
 * device from the group's uniform draws, so no host round trip is needed.
 * All results are accumulated in FP64 and read back by qsim_batch_results. */
typedef struct qsim_batch *qsim_batch_h;

typedef struct qsim_batch_group {
    int32_t n;               /* state width (qubits) */
    int32_t n_states;        /* states in the group (<= 65535) */
    const qsim_gate *g;      /* the shared program */
    size_t ng;
    const double *mats;      /* MAT pool (complex128), or NULL */
    size_t n_mats;           /* complex entries in the pool */
    const double *params;    /* n_states x n_params angles read by records with
                                slot >= 0 (RX, RY, RZ, RXX, RZZ), or NULL */
    int32_t n_params;
    const double *uniforms;  /* n_states x n_slots draws in [0,1), or NULL (then the
                                program may hold no MEASURE record: QSIM_E_ARG) */
    const int32_t *forced;   /* n_states x n_slots outcomes to force (-1: draw), or NULL */
    int32_t n_slots;         /* measurement slots per state */
    const qsim_pauli *terms; /* observable evaluated at the end, or NULL */
    size_t n_terms;
    void *dev_states;        /* caller-owned device buffer of n_states * 2^n
                                elements (state b at offset b * 2^n), or NULL
                                to let the batch allocate it */
} qsim_batch_group;

typedef struct qsim_batch_opts {
    int32_t dtype;           /* QSIM_C64 or QSIM_C128 */
    int32_t use_graph;       /* 1: record the whole run once as a HIP graph and replay it */
    int32_t max_params;      /* angle slots per fused operator (0 = 2) */
    int32_t autotune;        /* 1: per group, time fusion widths 2..5 (complex128: 2..4) on
                                the template with state 0's angles bound, on a scratch
                                state allocated for the purpose, and compile the group
                                with the fastest; the other fields of `fuse` are kept */
    qsim_fuse_opts fuse;     /* level 0 selects the default (5) */
} qsim_batch_opts;

typedef struct qsim_batch_info {
    int64_t states;
    int64_t input_gates;     /* summed over groups, per state */
    int64_t fused_ops;
    int64_t passes;          /* summed over groups */
    int64_t state_bytes;
    int64_t coef_bytes;
    double compile_seconds;  /* includes tune_seconds */
    double tune_seconds;     /* time spent by the autotuner (0 without it) */
    int64_t records;         /* summed over groups: measurement, assertion and reset
                                records run per state, after a reset that follows a
                                record of its qubit with no gate between has been
                                joined to it or dropped (QSIM_FOLD_RESETS=0 keeps all) */
} qsim_batch_info;

/* Compile every group once (lowering, fusion, plan; angle-dependent
 * operators keep their cos/sin basis blocks) and allocate device memory.
 * Errors as qsim_compile, plus QSIM_E_CAPACITY (n_states > 65535) and
 * QSIM_E_ARG for a MEASURE record in a group without uniforms. */
int qsim_batch_create(const qsim_batch_group *groups, int n_groups, const qsim_batch_opts *opt,
                      qsim_batch_h *out);
/* Run every group from |0...0> (asynchronous on hip_stream): bind angles,
 * apply the program, decide measurements on the device, reduce norms and
 * Pauli overlaps. */
int qsim_batch_run(qsim_batch_h b, void *hip_stream);
/* Synchronise and read one group's results (NULL to skip an output):
 * outcomes / probs: n_states x n_slots (outcome, probability of it);
 * expvals: <H>/<psi|psi> per state; norms: <psi|psi> per state;
 * status: 0, or the QSIM_E_* code of a failed assertion / reset. */
int qsim_batch_results(qsim_batch_h b, int group, int32_t *outcomes, double *probs,
                       double *expvals, double *norms, int32_t *status);
int qsim_batch_get_state(qsim_batch_h b, int group, int index, void *host_dst);
int qsim_batch_info_get(qsim_batch_h b, qsim_batch_info *out);
/* Compile statistics of one group (fused operators, passes, fusion width
 * used) and the width the autotuner chose for it (0 if not tuned). */
int qsim_batch_group_stats(qsim_batch_h b, int group, qsim_apply_stats *out, int32_t *tuned_width);
int qsim_batch_destroy(qsim_batch_h b);

/* ----------------------------------------------------------- serving */

/* A request loop with continuous batching: requests (circuits of any width)
 * are compiled by host worker threads as they arrive and admitted, in
 * arrival order, as soon as a slot (a HIP stream) and enough pool memory
 * (2^n state elements) are free; admitted requests run concurrently on the
 * device.  Each request's plan and kernels do not depend on what else is
 * resident, so its result is the same alone and in any mix.  The server
 * owns one device pool, allocated at creation. */
typedef struct qsim_server *qsim_server_h;

typedef struct qsim_server_opts {
    int32_t dtype;            /* QSIM_C64 or QSIM_C128 */
    int32_t slots;            /* requests resident at once (streams), 1..64 */
    int32_t compile_threads;  /* host compile workers, 1..64 */
    int32_t pad;
    size_t pool_bytes;        /* device pool for states (admission budget) */
    qsim_fuse_opts fuse;      /* level 0 selects the default */
} qsim_server_opts;

typedef struct qsim_request {
    int32_t n;                /* width */
    int32_t pad;
    const qsim_gate *g;       /* copied at submit */
    size_t ng;
    const double *mats;       /* MAT pool, copied; `n_mats` complex entries */
    size_t n_mats;
    const qsim_pauli *terms;  /* observable, copied; may be NULL */
    size_t n_terms;
    void *host_state_out;     /* if not NULL, receives the final state (2^n
                                 elements) before the result is reported; the
                                 caller keeps it valid until then */
} qsim_request;

typedef struct qsim_result {
    int64_t id;
    int32_t status;           /* QSIM_OK or the request's error */
    int32_t n;
    double expval;            /* <H>/<psi|psi> (0 without terms) */
    double norm;              /* <psi|psi> */
    double t_submit, t_admit, t_done;   /* seconds, server clock (qsim_server_clock) */
    int64_t passes;
} qsim_result;

typedef struct qsim_server_stats {
    int64_t submitted, completed, rejected, in_flight, waiting;
    size_t pool_bytes, pool_in_use, pool_peak;
    int64_t peak_in_flight;   /* most requests admitted (resident on the device) at once */
} qsim_server_stats;

/* Errors: QSIM_E_ARG, QSIM_E_NOMEM (pool allocation), QSIM_E_HIP. */
int qsim_server_create(const qsim_server_opts *opt, qsim_server_h *out);
/* Copy the request and queue it; writes its id.  QSIM_E_CAPACITY if the
 * state can never fit the pool, QSIM_E_ARG for a bad width or list. */
int qsim_server_submit(qsim_server_h s, const qsim_request *r, int64_t *id);
/* Move up to `max` finished results into `out`; writes how many.  With
 * wait_ms > 0, blocks up to that long for at least one. */
int qsim_server_poll(qsim_server_h s, qsim_result *out, int max, int *n_out, int wait_ms);
int qsim_server_get_stats(qsim_server_h s, qsim_server_stats *out);
/* Seconds on the server clock (steady clock), for arrival bookkeeping. */
double qsim_server_clock(void);
/* Finish everything in flight, then free the server. */
int qsim_server_destroy(qsim_server_h s);

/* ----------------------------------------------------------- sampling */

/* Draw m shots of all n qubits at once from the current state (Section
 * 4.3: after measurement assertion the final state is sampled for all m
 * shots together).  Shot s is the smallest basis index x with
 * C(x) > u[s] * C(2^n - 1), where C is the FP64 inclusive prefix sum of
 * |a_x|^2 in index order; u[s] in [0,1).  out[s] receives x.  Synchronous;
 * uses 8 * 2^n bytes of device scratch, allocated on first use. */
int qsim_sample(qsim_h h, const double *uniforms, size_t m, uint64_t *out);

/* ------------------------------------------------------ copy ceiling */

/* Not a step of the method: the same-footprint memory ceiling that the
 * benchmark sets beside a tile pass.  Copies `bytes` (a multiple of 16)
 * from src to dst, both device pointers; dst == src is allowed and makes an
 * in-place pass that reads and writes every byte once, the traffic of one
 * tile pass over a state of that size.  Workgroups of 256 threads each move
 * a 64 KiB block (16 loads of 16 bytes per thread in flight, then 16
 * stores), the tile kernel's shape for complex128.  flags bit 0: non-temporal
 * loads and stores.  `rotate` offsets the block a workgroup takes; changing
 * it between calls moves every block to another workgroup and XCD, as a tile
 * pass over a new qubit set does.  Asynchronous on hip_stream.  Errors:
 * QSIM_E_ARG (null pointer, size not a multiple of 16, unknown flag). */
int qsim_stream_copy(void *dst, const void *src, size_t bytes, int flags, uint32_t rotate,
                     void *hip_stream);

/* ----------------------------------------------------------- autotune */

/* Pick fusion width, per-operator cost, tile qubits and contiguous low
 * qubits for this circuit on this device: each candidate compiles a prefix
 * of the circuit (up to `prefix_gates` records, 0 = 20000) and runs it on
 * h's state, timed with HIP events; the fastest per input gate wins.  The
 * state is left as |0...0>.  Writes the chosen options (level 5) and their
 * time per input gate in ns.  Synchronous. */
int qsim_autotune(qsim_h h, const qsim_gate *g, size_t ng, const double *mats, size_t n_mats,
                  const double *params, size_t n_params, size_t prefix_gates,
                  qsim_fuse_opts *best, double *ns_per_gate);

/* ------------------------------------------------------- host-only tools */

/* Run lowering and fusion only (no device): writes the fused operators as
 * (k, qubits, matrix) so that a checker can apply them.  For each operator
 * i: out_k[i], out_qubits[5*i .. 5*i+k-1] (ascending), and its 4^k complex
 * entries (row-major, local index bit j = j-th smallest qubit) appended to
 * out_mats (interleaved doubles).  Capacities in operators / doubles;
 * QSIM_E_CAPACITY if too small.  `counts` (6 entries, may be NULL) receives
 * the operator count after each fusion level. */
int qsim_debug_fuse(int n, const qsim_gate *g, size_t ng, const double *mats, size_t n_mats,
                    const double *params, size_t n_params, const qsim_fuse_opts *opt,
                    int32_t *out_k, int32_t *out_qubits, double *out_mats,
                    size_t cap_ops, size_t cap_doubles, size_t *n_ops,
                    int64_t *counts);

/* Parse an OpenQASM 2.0 program into gate records (host only; the paper
 * ingests its circuits as QASM text, Section 4.1, with the gate set of its
 * Table 3).
 *
 * text, len: the program (not necessarily NUL-terminated).  Qubits and
 * classical bits are numbered across their registers in declaration order
 * (n_qubits, n_clbits receive the totals; either may be NULL).  Accepted: the
 * OPENQASM header; include lines (the standard gates are built in: id h x y z
 * s sdg t tdg sx rx ry rz u1 p u2 u3 u U cx CX cy cz ch swap crx cry crz cu1
 * cp cu3 rxx rzz ccx cswap c3x c3sqrtx c4x); qreg / creg; gate definitions
 * with parameters (expanded at each call); calls on qubits or whole registers
 * (broadcast over equal sizes); measure (record MEASURE, slot = classical bit
 * index), reset, barrier; parameter expressions with pi, + - * / ^, unary
 * minus, parentheses, sin cos tan exp ln sqrt.
 *
 * out: caller array of cap records (may be NULL with cap 0 to size the
 * output); *n_out always receives the number of records of the program.
 * Errors: QSIM_E_CAPACITY when cap < *n_out (nothing written); QSIM_E_ARG on
 * a syntax error or a wrong operand count, QSIM_E_QUBIT on an out-of-range
 * index or a repeated qubit, QSIM_E_UNSUPPORTED on if, opaque or an unknown
 * gate -- qsim_last_error() then names the line. */
int qsim_parse_qasm(const char *text, size_t len, qsim_gate *out, size_t cap, size_t *n_out,
                    int32_t *n_qubits, int32_t *n_clbits);

/* Host-only: applies the circuit to psi exactly as the device tables of its
 * compiled plan describe (the same lowering, fusion, pass plan and packing as
 * qsim_compile for n and dtype), in FP64 on the host: tiled passes gather each
 * tile through its position table, apply every operator record with the
 * coefficient block its block qubits select, and scatter the tile back;
 * strided passes apply their operator on global positions.  For tests of the
 * planner and the packer without a GPU.
 *
 * psi: 2^n interleaved complex128 values, updated in place (caller-owned).
 * Errors: as qsim_compile, and QSIM_E_ARG for n > 24 or psi == NULL. */
int qsim_debug_emulate(int n, int dtype, const qsim_gate *g, size_t ng, const double *mats,
                       size_t n_mats, const double *params, size_t n_params,
                       const qsim_fuse_opts *opt, double *psi);

/* Host-only: number of full-state passes the planner makes for the fused
 * circuit (same inputs as qsim_debug_fuse), for n qubits and dtype. */
int qsim_debug_plan(int n, int dtype, const qsim_gate *g, size_t ng,
                    const double *mats, size_t n_mats, const double *params,
                    size_t n_params, const qsim_fuse_opts *opt, qsim_apply_stats *out);

/* Test hook for the out-of-memory paths: the allocation attempt `after`
 * attempts from now (0 = the next one) fails as if the device or host were
 * out of memory, once; -1 disarms.  Counted attempts: every device and
 * pinned-host allocation the library makes and the start of every compile
 * (standing for its host allocations).  The failing call returns
 * QSIM_E_NOMEM and leaves the state and the handle as they were. */
int qsim_debug_fail_alloc(int after);

const char *qsim_strerror(int status);
/* Text of the last failed HIP call on this thread (empty if none). */
const char *qsim_last_error(void);
int qsim_version(void);

#ifdef __cplusplus
}
#endif
#endif /* QSIM_H */
