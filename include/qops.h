/*
 * qops.h -- C ABI of libqops, a full-state quantum circuit simulator for
 * AMD Instinct MI355X (gfx950) with profile-guided gate fusion and virtual
 * swaps.
 *
 * Method (paper: QOPS, profile-guided optimisation of quantum circuit
 * simulation):
 *   - Sec. II-B: a Schroedinger-style (full-state) simulation keeps all 2^n
 *     complex amplitudes of an n-qubit register and updates them gate by
 *     gate; it can report the final probability distribution.
 *   - Sec. II-B / Fig. 4: index bits that are cheap to reach (the "chunk
 *     segment") make gates fast; here the cheap tier is a work-group tile
 *     held in registers and LDS, the expensive tier a strided sweep of HBM.
 *   - Sec. III-C: a profiling run records per-gate counters (gate kind x
 *     qubit) and a timestamped gate sequence; the results of that run are
 *     still valid simulation results (Sec. IV-A).
 *   - Sec. III-D: virtual swap turns a SWAP into a relabelling of where a
 *     logical qubit lives instead of moving amplitudes; single-qubit gate
 *     merging fuses runs of one-qubit gates into one unitary.
 *   - Sec. IV-E: the same circuit is simulated many times with new
 *     parameters; expectation values are read out after each run.
 *
 * Conventions (all calls):
 *   - Logical qubit q is bit q of a logical basis index (qubit 0 = LSB).
 *   - A gate on ordered qubits (q_0..q_{k-1}) has a 2^k x 2^k matrix whose
 *     row/column index bit j belongs to q_j.  Controls are all on |1>.
 *   - Amplitudes are interleaved (re, im): complex64 (QOPS_C64, 8 bytes) or
 *     complex128 (QOPS_C128, 16 bytes).
 *   - The device state is stored in PHYSICAL order: logical qubit q lives in
 *     physical index bit l2p[q].  Readout calls map back to logical order.
 *   - Every call returns an int32_t status (QOPS_OK = 0 or a negative code);
 *     qops_last_error() returns a thread-local description of the last
 *     failure.  No call throws.
 *   - Work is enqueued on the HIP stream given at creation.  Calls marked
 *     "blocking" synchronise that stream before returning; the others are
 *     asynchronous with respect to the host.
 */
#ifndef QOPS_C_ABI_H_
#define QOPS_C_ABI_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status ---- */
enum qops_status {
    QOPS_OK = 0,
    QOPS_INVALID_ARG = -1,      /* null pointer, bad enum, bad size          */
    QOPS_QUBIT_RANGE = -2,      /* qubit index outside [0, n)                */
    QOPS_DUPLICATE_QUBIT = -3,  /* a qubit listed twice in one gate          */
    QOPS_UNSUPPORTED = -4,      /* k > 6, > 4 controls, n outside [1, 34]    */
    QOPS_OUT_OF_MEMORY = -5,    /* device or host allocation failed          */
    QOPS_HIP_ERROR = -6,        /* a HIP runtime call failed                 */
    QOPS_BAD_STATE = -7,        /* handle / plan / precision mismatch        */
    QOPS_NOT_UNITARY = -8       /* opt-in unitarity check failed             */
};

/* Thread-local, NUL-terminated description of the last failing call.
 * (Library plumbing; no passage of the paper.) */
const char* qops_last_error(void);
/* Library version as 10000*major + 100*minor + patch. */
int32_t qops_version(void);

/* --------------------------------------------------------- gate list ---- */
enum qops_precision { QOPS_C64 = 0, QOPS_C128 = 1 };

/* Gate kinds.  Matrices (c = cos(t/2), s = sin(t/2)):
 *   H, X, Y, Z, S=diag(1,i), SDG, T=diag(1,e^{i pi/4}), TDG, SX=sqrt(X);
 *   RX(t)=[[c,-is],[-is,c]], RY(t)=[[c,-s],[s,c]], RZ(t)=diag(e^{-it/2},e^{it/2}),
 *   P(l)=diag(1,e^{il}), U3(t,p,l)=[[c,-e^{il}s],[e^{ip}s,e^{i(p+l)}c]];
 *   CX(q0 control, q1 target), CZ, CP(l) (phase e^{il} on |11>), SWAP,
 *   RZZ(t) (e^{-it/2} when the two bits agree, e^{+it/2} otherwise);
 *   DENSE: the 2^k x 2^k matrix given in `mat`. */
enum qops_kind {
    QOPS_H = 0, QOPS_X, QOPS_Y, QOPS_Z, QOPS_S, QOPS_SDG, QOPS_T, QOPS_TDG, QOPS_SX,
    QOPS_RX, QOPS_RY, QOPS_RZ, QOPS_P, QOPS_U3,
    QOPS_CX, QOPS_CZ, QOPS_CP, QOPS_SWAP, QOPS_RZZ,
    QOPS_DENSE,
    QOPS_NUM_KINDS
};

#define QOPS_MAX_K 6
#define QOPS_MAX_CTRL 4
#define QOPS_MAX_QUBITS 34

typedef struct qops_gate {
    uint16_t kind;        /* enum qops_kind                                   */
    uint8_t k;            /* number of targets (must match the kind; 1..6 for
                             DENSE)                                          */
    uint8_t n_ctrl;       /* extra controls, 0..4 (not allowed on SWAP)       */
    int32_t q[6];         /* targets, logical qubits                          */
    int32_t ctrl[4];      /* controls, logical qubits                         */
    double param[3];      /* angles in radians (RX/RY/RZ/P/CP/RZZ: param[0];
                             U3: theta, phi, lambda)                          */
    const double* mat;    /* DENSE only: 2^k x 2^k complex128 row-major,
                             interleaved (re, im); read during the call and
                             never retained                                  */
} qops_gate;

/* ------------------------------------------------------------ handle ---- */
typedef struct qops_sim qops_sim;

/* Paper Sec. II-B: a full-state simulation of n qubits holds all 2^n complex
 * amplitudes in memory; this handle owns (or borrows) that array on the GPU.
 * Creates a simulator of n qubits (1 <= n <= 34).  If dev_state is non-null
 * the handle BORROWS that device buffer (bytes >= 2^n * amplitude size; the
 * caller keeps it alive until qops_destroy); otherwise the library allocates
 * and owns it.  `stream` is a hipStream_t (null = default stream).  The state
 * is NOT initialised: call qops_init_basis or qops_init_amplitudes. */
int32_t qops_create(int32_t n, int32_t precision, void* dev_state, size_t bytes, void* stream,
                    qops_sim** out);
/* Frees library-owned memory and plans.  Null is accepted.  (Plumbing.) */
int32_t qops_destroy(qops_sim* h);
/* Caps the work-groups of every state pass this handle launches (register
 * and LDS tile passes, gate-wise sweeps, bit exchanges); 0 (the default)
 * restores each kernel's own grid: one work-group per tile for register
 * tiles, as many as fit on the chip for LDS tiles, up to 16384 for sweeps.
 * The kernels walk the remaining tiles or groups in grid-stride loops, so
 * the results do not depend on the cap; a small cap makes each work-group
 * process many tiles (the persistent path a full-size state takes).
 * QOPS_INVALID_ARG for a negative value. */
int32_t qops_set_launch_limit(qops_sim* h, int32_t max_workgroups);
/* Device pointer of the state (physical order, Sec. III-D: the layout the
 * virtual swaps leave) and its size in bytes.  The pointer stays owned by
 * the handle (or by the caller that lent it). */
int32_t qops_state_pointer(qops_sim* h, void** dev_ptr, size_t* bytes);

/* Paper Sec. II-B: the simulation starts from a basis state.  Sets |x> (x in
 * logical order, x < 2^n, else QOPS_INVALID_ARG) and resets the layout to
 * the identity.  Asynchronous. */
int32_t qops_init_basis(qops_sim* h, uint64_t x);
/* Paper Sec. II-B: an arbitrary initial state vector.  Copies 2^n amplitudes
 * (precision of the handle, logical order; the caller keeps `host`) from
 * host memory and resets the layout to the identity.  Blocking. */
int32_t qops_init_amplitudes(qops_sim* h, const void* host);

/* ------------------------------------------------------------- plans ---- */
/* Plan modes:
 *   GATEWISE  one HBM sweep per gate, no fusion (the unoptimised simulator;
 *             the gate-by-gate baseline)
 *   FUSED     single-qubit merging, diagonal riding and tile packing with
 *             built-in heuristics
 *   PROFILED  like FUSED, but every candidate plan is priced with the cost
 *             table measured by a profiling run (opts.profile)
 *   LEARNED   like PROFILED, priced by a trained cost model (opts.model);
 *             falls back to PROFILED pricing when no model is given */
enum qops_plan_mode { QOPS_PLAN_GATEWISE = 0, QOPS_PLAN_FUSED = 1, QOPS_PLAN_PROFILED = 2,
                      QOPS_PLAN_LEARNED = 3 };
enum qops_swap_mode { QOPS_SWAP_VIRTUAL = 0, QOPS_SWAP_PHYSICAL = 1 };

typedef struct qops_profile qops_profile;
typedef struct qops_model qops_model;
typedef struct qops_plan qops_plan;

typedef struct qops_plan_opts {
    int32_t mode;          /* enum qops_plan_mode (default FUSED)             */
    int32_t swap_mode;     /* enum qops_swap_mode (default VIRTUAL)           */
    int32_t tile_upper;    /* upper tile qubits per pass beyond the 6 lane
                              qubits; 0 = choose automatically                */
    int32_t max_fuse_k;    /* widest dense block (<= 6 qubits) the planner
                              may build by composing gates whose bits fit a
                              common set (1 = only 1q merging); 0 = 1 in FUSED
                              mode, chosen among 1..4 by PROFILED / LEARNED   */
    int32_t use_mfma;      /* 1 = matrix cores for dense blocks with k >= 3
                              (default), 0 = vector ALU where it can         */
    int32_t check_unitary; /* 1 = reject non-unitary DENSE input (1e-9)       */
    int32_t remap;         /* 1 = before the gates, move the six qubits that
                              non-diagonal gates target most often into
                              physical bits 0..5 (held by every tile pass),
                              by physical bit exchanges; PROFILED / LEARNED
                              modes decide this themselves                    */
    const qops_profile* profile;  /* PROFILED / LEARNED pricing input         */
    const qops_model* model;      /* LEARNED pricing input                    */
    int32_t fold_rotations;        /* rotation folding (paper Sec. III-D):
                                      diagonal phases on equal parities of the
                                      path variables merge across CNOT / X /
                                      SWAP; 1 = on, -1 = off, 0 = the paper's
                                      rule (on when T gates exceed 10% of the
                                      gates).  Exact, global phase included.  */
    int32_t merge_blocks;          /* priced merging of dense blocks (the
                                      two-qubit block merging of the paper's
                                      all-on configuration, Sec. IV,
                                      generalised to <= 6 qubits and priced
                                      as in Sec. III-C/D): two uncontrolled
                                      dense blocks that commute past the operations
                                      between them become one block on the
                                      union of their qubits (<= 6) when the
                                      measured per-block cost of the union is
                                      below the sum of theirs (a per-width
                                      cost table for each precision).  1 or
                                      0 (the default) = on, -1 = off.        */
} qops_plan_opts;

/* Fills opts with the defaults listed above (Sec. III-D: which optimisations
 * the optimisation run switches on).  QOPS_INVALID_ARG for null. */
int32_t qops_plan_opts_default(qops_plan_opts* opts);

/* Paper Sec. III-D (the optimisation run): applies the switched-on
 * optimisations -- virtual swaps, single-qubit gate merging, rotation
 * folding, profile-guided remapping -- and packs the gates into passes.
 * Builds an execution plan for `gates` (n_gates entries) on an n-qubit
 * register of the given precision, starting from layout l2p_in (n entries;
 * null = identity).  Gates and DENSE matrices are copied; the plan is
 * independent of any handle and owned by the caller until qops_plan_free.
 * FP64 unitary composition happens here.  Errors: QOPS_QUBIT_RANGE,
 * QOPS_DUPLICATE_QUBIT, QOPS_UNSUPPORTED (k > 6, > 4 controls),
 * QOPS_NOT_UNITARY (opt-in), QOPS_INVALID_ARG (bad mode or pointer). */
int32_t qops_plan_build(int32_t n, int32_t precision, const int32_t* l2p_in, const qops_gate* gates,
                        size_t n_gates, const qops_plan_opts* opts, qops_plan** out);
/* Frees a plan and its device image (null accepted). */
int32_t qops_plan_free(qops_plan* p);

/* Plan statistics: the passes, gates and swaps the optimisations produced
 * and the planning time (the paper's compile time, Sec. IV-B). */
typedef struct qops_plan_stats {
    int32_t n_passes;          /* kernel launches over the state              */
    int32_t n_tile_passes;     /* of which fused tile passes                  */
    int32_t n_permute_passes;  /* of which physical bit-permutation passes    */
    int32_t n_ops;             /* fused operations after merging              */
    int32_t n_gates_in;        /* gates given                                 */
    int32_t n_virtual_swaps;   /* SWAPs turned into layout updates            */
    int32_t tile_upper;        /* chosen upper tile width                     */
    int32_t max_fuse_k;        /* chosen fusion width                         */
    double bytes_alg;          /* algorithmic HBM bytes of all passes         */
    double predicted_s;        /* cost-model prediction (0 if not priced)     */
    double plan_seconds;       /* host time spent building the plan           */
    int32_t n_folded;          /* phase gates removed by rotation folding     */
} qops_plan_stats;
int32_t qops_plan_stats_get(const qops_plan* p, qops_plan_stats* out);
/* The layout (l2p, n int32 written to caller memory) the plan leaves
 * behind: Sec. III-D, virtual swaps relabel where a logical qubit lives. */
int32_t qops_plan_final_layout(const qops_plan* p, int32_t* l2p);

/* Plan introspection (host only; no GPU needed), the optimisation run's
 * result of Sec. III-D (merged and virtually swapped gates).  Lowered
 * operations act on
 * PHYSICAL bits after virtual swaps, single-qubit merging and diagonal
 * fusion.  kind: 0 = one-qubit (2x2 on t[0]), 1 = diagonal table over bits
 * t[0..k-1], 2 = dense 2^k x 2^k on t[0..k-1] (matrix bit order), 3 =
 * physical bit exchange of t[0], t[1].  `mat` (nullable) receives the
 * matrix (2*4^k doubles) or diagonal table (2*2^k doubles), interleaved. */
typedef struct qops_op_info {
    int32_t kind;
    int32_t k;
    int32_t t[10];
    uint64_t cmask;        /* physical control bits                           */
    int32_t pass;          /* index of the pass that executes the operation   */
    int32_t n_merged;      /* input gates folded into this operation          */
} qops_op_info;
/* Number of lowered operations; operation i (QOPS_INVALID_ARG if i is out
 * of range). */
int32_t qops_plan_num_ops(const qops_plan* p, size_t* n);
int32_t qops_plan_op(const qops_plan* p, size_t i, qops_op_info* info, double* mat);

/* Pass types: 0 register tile, 1 LDS tile (dense blocks), 2 whole state in
 * one work-group's LDS, 3 gate-wise HBM sweep, 4 physical bit exchange. */
typedef struct qops_pass_info {
    int32_t type;
    int32_t tile_bits;     /* L: the pass touches tiles of 2^L amplitudes     */
    int32_t n_upper;       /* upper tile bits (beyond physical bits 0..5)     */
    int32_t upper[8];      /* those physical bits                             */
    int32_t n_ops;         /* lowered operations in the pass                  */
    int32_t n_remaps;      /* register/LDS remaps inside the pass             */
    int32_t n_mfma;        /* dense blocks on matrix cores                    */
    double bytes_alg;      /* algorithmic HBM bytes                           */
    double flops;          /* algorithmic floating-point operations           */
} qops_pass_info;
/* Pass i of the plan (QOPS_INVALID_ARG past the last pass). */
int32_t qops_plan_pass_info(const qops_plan* p, size_t i, qops_pass_info* info);

/* Paper Sec. II-B: gate-by-gate update of the full state, here pass by pass.
 * Runs a plan on the handle (n, precision and the handle's current layout
 * must equal the plan's; otherwise QOPS_BAD_STATE).  The plan stays owned
 * by the caller and must outlive the queued work.  Asynchronous. */
int32_t qops_run_plan(qops_sim* h, const qops_plan* p);
/* Paper Sec. IV-E (repeated runs of one circuit with new parameters).
 * Re-binds the angles / dense matrices of a plan to a new gate list with the
 * same structure (same kinds, qubits and controls): the planner runs again on
 * the new parameters with the plan's options, so fused blocks are re-composed
 * in FP64 and the pass structure is kept; the device buffers of the plan are
 * reused.  For repeated runs with new parameters (QAOA angle sweeps).
 * QOPS_BAD_STATE if the structure differs. */
int32_t qops_plan_update(qops_plan* p, const qops_gate* gates, size_t n_gates);

/* Paper Sec. II-B + III-D: plans (opts may be null = defaults) and runs a
 * gate list on the handle in one call; the plan is kept by the handle until
 * the next apply or destroy.  Errors as qops_plan_build.  Asynchronous. */
int32_t qops_apply(qops_sim* h, const qops_gate* gates, size_t n_gates, const qops_plan_opts* opts);

/* --------------------------------------------------------- profiling ---- */
/* A profiling run (paper Sec. III-C) executes a plan exactly like
 * qops_run_plan -- the state it leaves is the normal result -- while timing
 * every pass with HIP events on the handle's stream (the context record:
 * which pass, which operations, start/end time) and counting gates per kind
 * and qubit (the counter record).  Blocking.  The profile is library-owned
 * until qops_profile_free. */
typedef struct qops_pass_record {
    int32_t pass;          /* index in the plan                               */
    int32_t type;          /* pass type (see qops_pass_info)                  */
    int32_t n_ops;         /* lowered operations                              */
    int32_t n_gates;       /* input gates folded into them                    */
    int32_t tile_bits;
    int32_t n_mfma;
    int32_t max_k;
    int32_t n_remaps;
    double t_begin;        /* seconds since the first pass started            */
    double seconds;        /* device time of the pass                         */
    double bytes_alg;      /* algorithmic HBM bytes                           */
    double flops;
    uint64_t phys_mask;    /* physical bits targeted by the pass              */
} qops_pass_record;

int32_t qops_profile_run(qops_sim* h, const qops_plan* p, qops_profile** out);
/* Sec. III-C context records: number of pass records, and record i. */
int32_t qops_profile_num_passes(const qops_profile* pr, size_t* n);
int32_t qops_profile_pass(const qops_profile* pr, size_t i, qops_pass_record* rec);
/* Sec. III-C counter records: counts[kind * n + q] for logical qubit q
 * (targets and controls; QOPS_NUM_KINDS * n int32 each, caller memory,
 * either may be null), and the same per physical bit at the time of the
 * gate. */
int32_t qops_profile_counts(const qops_profile* pr, int32_t* logical, int32_t* physical);
/* Sum of pass times (Sec. III-C timestamps), and the plan's qubit count. */
int32_t qops_profile_total(const qops_profile* pr, double* seconds, int32_t* n);
/* Cost-model features of every pass (64 floats per pass, pass order, into
 * caller memory): what the profile-guided pricing of Sec. III-D reads. */
int32_t qops_profile_features(const qops_profile* pr, float* out);
/* Sec. III-C: the profile is dumped to a file (counters, pass records) as
 * JSON.  QOPS_INVALID_ARG if the file cannot be written. */
int32_t qops_profile_dump(const qops_profile* pr, const char* path);
/* Writes the profile as a Chrome trace-event file (the JSON that
 * chrome://tracing and Perfetto open): one complete event per pass on a
 * "passes" track (start, duration, kernel kind, tile bits, operations, gates,
 * algorithmic bytes and flops, achieved GB/s), and per logical qubit a
 * counter track of the gates that touch it (the per-qubit hotspot view of
 * the paper's performance-debug use, Sec. IV-D). */
int32_t qops_profile_trace(const qops_profile* pr, const char* path);
/* Merges the pass records of `src` into `dst` (a cost table built from many
 * profiling runs, Sec. III-C); `src` is unchanged. */
int32_t qops_profile_merge(qops_profile* dst, const qops_profile* src);
/* Frees a profile (null accepted). */
int32_t qops_profile_free(qops_profile* pr);

/* ------------------------------------------------------ cost model ---- */
/* A 3-layer perceptron, 64 -> 128 -> 128 -> 1 with ReLU, predicting from the
 * 64 pass features of qops_profile_features the natural log of a pass's run
 * time (seconds) scaled to 30 qubits: ln(t) - (n - 30) ln 2 for an n-qubit
 * state (plan pricing adds the (n - 30) ln 2 back, so the per-amplitude cost
 * it learns carries over to other sizes).  Parameters (float) in this order: W1 [128 x 64]
 * row-major, b1 [128], W2 [128 x 128], b2 [128], W3 [1 x 128], b3 [1];
 * inputs are standardised with per-feature mean/sd before the first layer.
 * Training runs on the GPU (forward, backward of the mean squared error,
 * Adam) with fixed summation orders.  Prices candidate plans in LEARNED mode
 * (the choice of which optimisation to switch on, paper Sec. III-D). */
/* Number of network parameters (W1..b3). */
int32_t qops_mlp_num_params(size_t* n);
/* params may be null (all zero) or hold qops_mlp_num_params floats (copied).
 * The model is owned by the caller until qops_model_free. */
int32_t qops_mlp_create(const float* params, size_t n, qops_model** out);
/* Per-feature standardisation (64 means, 64 positive deviations; copied). */
int32_t qops_mlp_set_normalization(qops_model* m, const float* mu, const float* sd);
/* Copies parameters, means and deviations out; any output may be null. */
int32_t qops_mlp_get_params(const qops_model* m, float* params, float* mu, float* sd);
/* Loss (1/rows) sum (y - t)^2 and its gradient w.r.t. every parameter, on
 * the GPU (host arrays in and out: X rows x 64, t rows, grads
 * qops_mlp_num_params floats).  Blocking. */
int32_t qops_mlp_grad(qops_model* m, const float* X, const float* t, int32_t rows, float* grads, float* loss);
/* Trains with Adam (beta 0.9/0.999, eps 1e-8) for `epochs` passes over the
 * rows in batches of `batch`, reshuffled each epoch from `seed`.  Blocking. */
int32_t qops_mlp_train(qops_model* m, const float* X, const float* t, int32_t rows, int32_t epochs, int32_t batch,
                       float lr, uint64_t seed, float* final_loss);
/* out[r] = the network's output for row r (on the GPU).  Blocking. */
int32_t qops_mlp_predict(qops_model* m, const float* X, int32_t rows, float* out);
/* Binary save / load of a model (QOPS_INVALID_ARG on an unreadable or
 * mismatched file); free accepts null. */
int32_t qops_model_save(const qops_model* m, const char* path);
int32_t qops_model_load(const char* path, qops_model** out);
int32_t qops_model_free(qops_model* m);

/* Sec. III-D (profile-guided choice of optimisations).
 * Predicted run time of a plan under the pricing of `opts` (PROFILED: the
 * plain cost table of opts->profile -- per pass shape (kernel kind, tile
 * width, register/wave split, widest dense block, operation count) the
 * median measured time per amplitude, falling back to coarser shapes;
 * LEARNED: opts->model). */
int32_t qops_plan_predict(const qops_plan* p, const qops_plan_opts* opts, double* seconds);
/* Predicted time of every pass recorded in `pr` (held-out evaluation of a
 * cost model), out: one double per pass. */
int32_t qops_profile_predict_passes(const qops_profile* pr, const qops_plan_opts* opts, double* out);
/* Binary save / load of a profile (pass records, features, counters), the
 * corpus a plain cost table is fitted to (Sec. III-C dumps).  Load returns a
 * library-owned profile (qops_profile_free). */
int32_t qops_profile_save(const qops_profile* pr, const char* path);
int32_t qops_profile_load(const char* path, qops_profile** out);
/* A compact profile that prices like `src` under the plain table: per pass
 * shape (kernel kind, tile width, register/wave split, widest dense block,
 * operation count) it keeps the passes at the 10/30/50/70/90th percentiles of
 * time per amplitude (all of them for shapes with at most five).  For
 * shipping a table fitted to a large corpus.  Library-owned result. */
int32_t qops_profile_compact(const qops_profile* src, qops_profile** out);
/* An empty profile of n qubits to merge runs into. */
int32_t qops_profile_create(int32_t n, qops_profile** out);

/* --------------------------------------------------- batched runs ---- */
/* Many small, uneven circuits (a parameter sweep, paper Sec. IV-E: the same
 * ansatz simulated again and again with new angles) run as ONE graph launch:
 * circuits of up to small_max_n qubits each run start to finish in one
 * work-group's LDS; the larger ones are planned into tile passes (register
 * or LDS tiles) and the graph nodes of step p run pass p of every circuit
 * that has one, one node per kernel kind.  Every circuit starts in
 * |0..0>; the outputs are <Z_q> of every logical qubit of every circuit
 * (FP64, deterministic), concatenated in circuit order (sum of n_i doubles).
 * SWAP gates are handled virtually. */
typedef struct qops_batch {
    int32_t count;                 /* circuits                                  */
    const int32_t* n;              /* qubits of each circuit (1..26)            */
    const qops_gate* const* gates; /* gate list of each circuit                 */
    const size_t* n_gates;
    int32_t precision;             /* QOPS_C64 / QOPS_C128                      */
    void* stream;                  /* hipStream_t; null = a private stream      */
    int32_t small_max_n;           /* whole-state-in-LDS limit (0 = 13 / 12)    */
    int32_t tile_bits;             /* tile size 2^tile_bits of the larger ones
                                      (0 = 13 / 12)                             */
    int32_t max_fuse_k;            /* block fusion width (as in qops_plan_opts;
                                      0 = 1)                                    */
} qops_batch;
typedef struct qops_batch_exec qops_batch_exec;
typedef struct qops_batch_stats {
    int32_t small_circuits;
    int32_t tile_circuits;
    int32_t graph_nodes;
    int32_t small_max_n;
    int32_t tile_bits;
    int32_t max_fuse_k;
    int64_t outputs;
    double state_bytes;            /* device memory of the tile-pass states     */
} qops_batch_stats;
/* Sec. IV-E: plans every circuit, lays out the device program, runs the
 * batch once and captures it as a graph.  Gate lists are copied; the
 * executor is owned by the caller until qops_batch_free.  Errors as
 * qops_plan_build for any circuit, QOPS_UNSUPPORTED for n outside 1..26. */
int32_t qops_batch_create(const qops_batch* b, qops_batch_exec** out);
/* One graph launch (asynchronous). */
int32_t qops_batch_launch(qops_batch_exec* e);
/* Waits and copies the <Z> outputs (sum of n_i doubles). */
int32_t qops_batch_results(qops_batch_exec* e, double* out_expz);
/* Mean device time of `reps` back-to-back graph launches (blocking). */
int32_t qops_batch_time(qops_batch_exec* e, int32_t reps, double* seconds);
/* New angles / matrices for every circuit (same structure): re-composes the
 * fused operations in FP64 and replaces the coefficients the graph reads;
 * QOPS_BAD_STATE if the structure changed. */
int32_t qops_batch_update(qops_batch_exec* e, const qops_gate* const* gates, const size_t* n_gates);
/* Shape the executor chose; frees an executor (null accepted). */
int32_t qops_batch_info(const qops_batch_exec* e, qops_batch_stats* s);
int32_t qops_batch_free(qops_batch_exec* e);
/* Sec. III-D's profile-then-choose idea applied to launch shapes.
 * Autotuner: times the batch for every (small_max_n, tile_bits, max_fuse_k)
 * candidate and returns the fastest; results are cached in a text file keyed
 * by the batch's precision, size and qubit-count histogram (cache_path
 * nullable).  b's own shape fields are ignored. */
int32_t qops_batch_autotune(const qops_batch* b, const char* cache_path, int32_t* best_small_max_n,
                            int32_t* best_tile_bits, int32_t* best_fuse_k, double* best_seconds);

/* -------------------------------------------- host-memory state tier ---- */
/* Paper Sec. II-B (storage-based simulation: the top index bits, the "file
 * segment", select a state file; the rest index inside it) and Sec. III-D
 * (virtual swap keeps the hot qubits out of the file segment).  Here the top
 * g physical bits select one of 2^g segments of a state kept in pinned host
 * memory, for states beyond device memory.  A run streams the state through
 * the device in stages: a stage may hold up to max_active global bits as
 * device-local bits (its "active" bits), so gates targeting them run; every
 * other gate's controls and diagonal phases on global bits are resolved per
 * group of segments.  Profile-guided placement (opts.remap = 1): the gate
 * counters choose which qubits start in the segment bits (for a basis state
 * set by qops_tier_init_basis), and when a stage activates a global bit it
 * exchanges it on the device with the local bit whose qubit is next needed
 * latest.  The device holds two group slots of 2^(n-g+max_active)
 * amplitudes; transfers run on two copy streams of the handle, overlapped
 * with the group plans on the caller's stream. */
typedef struct qops_tier qops_tier;
typedef struct qops_tier_opts {
    int32_t remap;          /* 1 = profile-guided placement and exchanges
                               (default), 0 = keep the layout               */
    int32_t reserved;
    qops_plan_opts plan;    /* options of the per-group plans (mode FUSED or
                               GATEWISE, fusion width, swap mode); priced
                               modes fall back to FUSED                      */
} qops_tier_opts;
typedef struct qops_tier_stats {
    int32_t stages;         /* streams of the whole state through the device */
    int32_t groups;         /* device groups over all stages                 */
    int32_t exchanges;      /* global<->local bit exchanges inserted         */
    int32_t virtual_swaps;  /* SWAP gates turned into layout updates         */
    int32_t gpu_passes;     /* kernel passes over all groups                 */
    int32_t reserved;
    double h2d_bytes;       /* host-to-device bytes of the run               */
    double d2h_bytes;       /* device-to-host bytes of the run               */
    double seconds;         /* wall time of the run (qops_tier_run)          */
    double plan_seconds;    /* host time of staging and group planning       */
} qops_tier_stats;
/* Fills opts: remap = 1, plan = qops_plan_opts_default. */
int32_t qops_tier_opts_default(qops_tier_opts* opts);
/* n qubits (2..34), g = global_bits segment bits (1..min(8, n-1)),
 * max_active in 1..g.  host_state: caller's PINNED buffer of >= 2^n
 * amplitudes (kept alive until destroy), or null for library-owned pinned
 * memory, one hipHostMalloc block per segment.  stream: the caller's stream for the group plans.
 * Errors: QOPS_UNSUPPORTED / QOPS_INVALID_ARG for shapes, QOPS_OUT_OF_MEMORY
 * or QOPS_HIP_ERROR for allocations.  The state is not initialised. */
int32_t qops_tier_create(int32_t n, int32_t precision, int32_t global_bits, int32_t max_active, void* host_state,
                         size_t bytes, void* stream, qops_tier** out);
int32_t qops_tier_destroy(qops_tier* t);
/* Host pointer and size in bytes of segment s (0 <= s < 2^g): physical
 * amplitudes s * 2^(n-g) .. (s+1) * 2^(n-g) - 1.  A library-owned state has
 * one pinned allocation per segment (the paper's one file per segment). */
int32_t qops_tier_segment_pointer(qops_tier* t, int32_t segment, void** host, size_t* bytes);
/* |x> in logical order, identity layout.  Blocking (host writes). */
int32_t qops_tier_init_basis(qops_tier* t, uint64_t x);
/* Runs a gate list (opts null = defaults); stats may be null.  Blocking.
 * QOPS_UNSUPPORTED if one gate targets more global bits than max_active. */
int32_t qops_tier_run(qops_tier* t, const qops_gate* gates, size_t n_gates, const qops_tier_opts* opts,
                      qops_tier_stats* stats);
/* Host-only staging of a gate list (no GPU): the stages, groups and
 * exchanges qops_tier_run would use from layout l2p_in (null = identity, or
 * with remap the profile-guided placement); l2p_out (nullable, n int32)
 * receives the final layout.  Byte counts are left 0. */
int32_t qops_tier_plan(int32_t n, int32_t global_bits, int32_t max_active, const int32_t* l2p_in,
                       const qops_gate* gates, size_t n_gates, int32_t remap, qops_tier_stats* stats, int32_t* l2p_out);
/* The layout (n int32): logical qubit q lives in physical bit l2p[q]. */
int32_t qops_tier_get_layout(qops_tier* t, int32_t* l2p);
/* <Z_q> of every logical qubit (n doubles), FP64: the segments stream
 * through the device once.  Blocking. */
int32_t qops_tier_expect_z(qops_tier* t, double* out);
/* Copies the state to host memory (2^n amplitudes, caller-owned) in logical
 * or physical order.  Blocking. */
int32_t qops_tier_read_state(qops_tier* t, void* host, int32_t order);

/* ------------------------------------------------------------ layout ---- */
/* Paper Sec. III-D, virtual swap: a SWAP becomes a relabelling of where the
 * two logical qubits live.  SWAP of logical qubits a and b.  VIRTUAL:
 * exchange l2p[a] and l2p[b], move no amplitude.  PHYSICAL: one
 * bit-exchange pass over the state (asynchronous).  QOPS_QUBIT_RANGE,
 * QOPS_DUPLICATE_QUBIT (a == b), QOPS_INVALID_ARG (bad mode). */
int32_t qops_swap(qops_sim* h, int32_t a, int32_t b, int32_t mode);
/* Sec. III-D: copies the logical-to-physical map (n int32, caller memory). */
int32_t qops_get_layout(qops_sim* h, int32_t* l2p);
/* Sec. II-B / III-D: moving a qubit into the cheap index bits (the chunk
 * segment).  Moves amplitudes so that logical qubit q lives in physical bit
 * l2p[q] (a permutation of 0..n-1, else QOPS_INVALID_ARG), by bit-exchange
 * passes.  Asynchronous. */
int32_t qops_set_layout(qops_sim* h, const int32_t* l2p);

/* ----------------------------------------------------------- readout ---- */
enum qops_order { QOPS_ORDER_LOGICAL = 0, QOPS_ORDER_PHYSICAL = 1 };
/* Paper Sec. II-B: full-state simulation exposes the intermediate and final
 * states.  Copies the 2^n amplitudes to host memory (caller-owned, 2^n *
 * amplitude size bytes) in logical or physical order.  Blocking. */
int32_t qops_read_state(qops_sim* h, void* host, int32_t order);
/* Sec. II-B (the probability distribution sums to one): sum_x |psi_x|^2,
 * FP64 accumulation, deterministic order.  Blocking. */
int32_t qops_norm(qops_sim* h, double* out);
/* Paper Sec. II-B: the final probability distribution.
 * Marginal distribution of logical qubits q[0..m-1] (1 <= m <= n):
 * out[y] (2^m doubles) = sum of |psi_x|^2 over x whose bit q_j equals bit j
 * of y.  FP64, deterministic.  Blocking. */
int32_t qops_probabilities(qops_sim* h, const int32_t* qubits, int32_t m, double* out);
/* Paper Sec. IV-E: expectation values read out after each run.
 * <Z_q> = sum_x |psi_x|^2 (1 - 2 b_q(x)) for every logical qubit (n
 * doubles, caller host memory).  FP64, deterministic.  Blocking. */
int32_t qops_expect_z(qops_sim* h, double* out);
/* <Z_a Z_b> = sum_x |psi_x|^2 (-1)^(b_a(x) + b_b(x)) for each pair of logical
 * qubits (a, b) = (pairs[2i], pairs[2i+1]), i < npairs: the correlators a
 * diagonal cost Hamiltonian such as weighted Max-Cut's,
 * C = sum_e w_e (1 - Z_a Z_b) / 2, is evaluated from in repeated QAOA runs
 * (paper Sec. IV-E).  out holds npairs doubles.  FP64, deterministic; one
 * read of the state per eight pairs.  QOPS_QUBIT_RANGE for a qubit outside
 * [0, n).  Blocking. */
int32_t qops_expect_zz(qops_sim* h, const int32_t* pairs, int32_t npairs, double* out);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * <Z_q> as qops_expect_z, written to DEVICE memory out_dev (n doubles,
 * logical order, caller-owned), asynchronously on the handle's stream, with
 * no allocation of any kind.  The partial sums live in one fixed 576 KiB
 * device array per GPU (held until the process ends) instead of the handle's
 * growable scratch buffer; every n up to 34 fits it (QOPS_UNSUPPORTED
 * otherwise).  Every call on a GPU shares that array: calls that overlap in
 * time on one GPU (other streams, other handles, other threads) race, so
 * order them on one stream.  The summation order is fixed; for n <= 27 it
 * is the one qops_expect_z uses. */
int32_t qops_expect_z_noalloc(qops_sim* h, double* out_dev);
/* Waits for all work enqueued on the handle's stream.  (Plumbing.) */
int32_t qops_synchronize(qops_sim* h);

#ifdef __cplusplus
}
#endif
#endif /* QOPS_C_ABI_H_ */
