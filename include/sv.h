/*
 * sv.h -- C ABI of the MI355X (gfx950) state-vector library `libsv.so`.
 *
 * Scope: the dense state-vector hot path of the paper's simulator -- apply
 * layers of (parameterised) gates to a 2^n-amplitude state and reduce Pauli
 * expectation values -- plus adjoint gradients, terminal sampling and a
 * ragged multi-circuit batch.  The paper's backend contract names the
 * operations (Appendix A.5: zeros_state, apply_unitary, expectation_sv,
 * measure_probs, sample, cast, to_numpy); the circuit model is the paper's
 * typed operation with targets first, then controls and optional control
 * states (Section 4.2); fusion width follows the paper's `fuse` option
 * (Section 4.3: 0 disables fusion, a positive width must be at least 2).
 *
 * Conventions
 *   - Qubit q is bit q of the basis index (little-endian).
 *   - A k-target gate's local matrix index is j = sum_i bit(targets[i]) 2^i.
 *   - Rotations are exp(-i theta P / 2) (paper Section 9.1).
 *   - The state is two planes (re, im) of 2^n elements each, FP64 for
 *     SV_C128 and FP32 for SV_C64 (paper Section 5.2: paired real tensors;
 *     matrices are always built in FP64 and narrowed at the boundary).
 *
 * Ownership and memory
 *   - State planes and the workspace are DEVICE memory owned by the caller
 *     (e.g. torch tensors).  A handle borrows them until sv_free and never
 *     frees them.  Host arrays (ops, params, terms) are read during the call
 *     and not kept.  Output arrays are caller-owned HOST memory unless the
 *     function name ends in _device.
 *
 * Synchronisation
 *   - Every call enqueues work on the handle's HIP stream.  sv_apply_layer
 *     and sv_reset return without waiting.  Calls that return host values
 *     (expect, adjoint, sample, copy) wait for that stream.
 *
 * Errors
 *   - Every call returns an sv_status.  All argument checks run before any
 *     device work is enqueued (nothing is narrowed or defaulted silently);
 *     on error the state is unchanged and sv_last_error() describes it.
 */
#ifndef LIBSV_PUBLIC_SV_H_
#define LIBSV_PUBLIC_SV_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sv_state sv_state;

typedef enum { SV_C128 = 0, SV_C64 = 1 } sv_dtype;

typedef enum {
  SV_OK = 0,
  SV_EINVAL = -1,        /* bad qubit, duplicate qubit, bad width, mask >= 2^n ... */
  SV_EDTYPE = -2,        /* unsupported dtype */
  SV_EUNBOUND = -3,      /* parameter index out of range or non-finite parameter */
  SV_ENOMEM = -4,        /* workspace too small / allocation failed */
  SV_EUNSUPPORTED = -5,  /* valid request this path does not implement */
  SV_EDEVICE = -6        /* a HIP runtime call failed */
} sv_status;

/* Gate kinds (paper Section 4.2 gate table).  Controlled gates are a base
 * kind plus controls: CX = SV_X with one control, CZ = SV_Z with one control,
 * Toffoli = SV_X with two controls, CP = SV_P with one control, etc. */
typedef enum {
  SV_I = 0, SV_X, SV_Y, SV_Z, SV_H, SV_S, SV_SDG, SV_T, SV_TDG, SV_SX,
  SV_RX, SV_RY, SV_RZ,     /* exp(-i theta P/2), 1 parameter */
  SV_P,                    /* diag(1, e^{i lambda}), 1 parameter */
  SV_U2,                   /* U3(pi/2, phi, lambda), 2 parameters */
  SV_U3,                   /* [[c, -e^{il}s], [e^{if}s, e^{i(f+l)}c]], 3 parameters */
  SV_SWAP,                 /* 2 targets */
  SV_RXX, SV_RYY, SV_RZZ,  /* exp(-i theta P(x)P/2), 2 targets, 1 parameter */
  SV_GIVENS,               /* rotation [[c,-s],[s,c]] on local |1>,|2>, 2 targets */
  SV_DEXC,                 /* rotation [[c,-s],[s,c]] on local |3>,|12>, 4 targets */
  SV_UNITARY,              /* user matrix on 1..3 targets (4..5: SV_EUNSUPPORTED) */
  SV_NKINDS
} sv_gate_kind;

#define SV_MAX_TARGETS 5
#define SV_MAX_CONTROLS 5

/* One typed operation (paper Section 4.2 circuit model). */
typedef struct {
  int32_t kind;                        /* sv_gate_kind */
  int32_t n_targets;                   /* must equal the kind's arity (1..3 for SV_UNITARY) */
  int32_t targets[SV_MAX_TARGETS];     /* targets first */
  int32_t n_controls;                  /* 0..SV_MAX_CONTROLS */
  int32_t controls[SV_MAX_CONTROLS];
  uint32_t control_states;             /* bit i = 1: control i fires on |1>; 0: on |0> */
  int32_t param_index[3];              /* into params[]; unused slots ignored */
  const double *matrix;                /* SV_UNITARY only: HOST row-major 2^k x 2^k,
                                          interleaved (re, im) complex128 */
} sv_op;

/* One Pauli term (paper Section 4.4 Pauli action): x_mask marks X or Y,
 * z_mask marks Z or Y (a Y is a bit set in both). */
typedef struct {
  uint64_t x_mask;
  uint64_t z_mask;
  double coeff;
} sv_pauli_term;

/* Special fuse_width values (besides 0 and 2..5, the paper's semantics). */
#define SV_FUSE_AUTO (-1)   /* LDS tile clustering: many <=5-qubit blocks per sweep */

/* Workspace flags. */
#define SV_WS_ADJOINT 1u    /* room for the adjoint's second state and partial sums */

/* Bytes of device workspace a handle needs.  Always >= the forward path's
 * needs; SV_WS_ADJOINT adds a second state (lambda) and gradient partials.
 * 0 for n outside 1..32 or an unknown dtype. */
size_t sv_workspace_bytes(int32_t n_qubits, sv_dtype dtype, uint32_t flags);

/* Wrap caller-owned device planes re/im (2^n elements each, 16-byte aligned)
 * and a 256-byte aligned workspace into a handle, bound to `hip_stream`
 * (NULL = default stream), and set the state to |0...0>.  n is 1..32 (32
 * qubits: 64 GiB of FP64 planes).  Errors: SV_EINVAL (n outside 1..32, null or
 * misaligned planes or workspace), SV_EDTYPE, SV_ENOMEM (ws_bytes <
 * sv_workspace_bytes). */
sv_status sv_alloc(int32_t n_qubits, sv_dtype dtype, void *re, void *im, void *workspace,
                   size_t ws_bytes, void *hip_stream, sv_state **out);

/* Release the handle (never the borrowed memory). */
sv_status sv_free(sv_state *st);

/* Re-bind the handle to another stream. */
sv_status sv_set_stream(sv_state *st, void *hip_stream);

/* State <- |0...0> (async). */
sv_status sv_reset(sv_state *st);

/* Apply ops[0..n_ops) in order (paper Section 5.3 gate application:
 * gather the amplitudes that differ only on the targets, multiply, scatter),
 * binding parameters from params[0..n_params).  fuse_width: 0 = one sweep per
 * gate; 2..5 = greedy in-order blocks of at most that many qubits, one sweep
 * per block (paper Section 4.3 `fuse`); SV_FUSE_AUTO = LDS-tiled clusters of
 * <=5-qubit blocks.  Async on the handle's stream.  Errors: SV_EINVAL (qubit
 * out of range, repeated qubit, bad arity/kind/width), SV_EUNBOUND (parameter
 * index out of range or a non-finite parameter), SV_ENOMEM. */
sv_status sv_apply_layer(sv_state *st, const sv_op *ops, int32_t n_ops, const double *params,
                         int32_t n_params, int32_t fuse_width);

/* <P_j> for every term (paper Section 4.4, matrix-free Pauli action) and
 * sum_j coeff_j <P_j>.  Either output may be NULL.  Accumulates in FP64 for
 * both dtypes.  Waits for the stream.  Errors: SV_EINVAL (mask >= 2^n). */
sv_status sv_expect_pauli(sv_state *st, const sv_pauli_term *terms, int32_t n_terms,
                          double *out_terms, double *out_sum);

/* As sv_expect_pauli, for callers that cannot allocate device memory (code
 * under HIP graph capture aside: this call waits for the stream; tight serving
 * loops; harnesses that forbid hipMalloc).  It allocates nothing: the partial
 * sums live in a fixed device array of SV_NOALLOC_SCRATCH_BYTES per GPU,
 * which the library holds until the process ends.  Calls on one GPU share
 * that array, so calls that overlap on one GPU (other streams, other threads)
 * race.  SV_ENOMEM, before any device work, when the terms' partial sums do
 * not fit (about 1000 terms with 256 compute units); other errors as
 * sv_expect_pauli. */
#define SV_NOALLOC_SCRATCH_BYTES (4u << 20)
sv_status sv_expect_pauli_noalloc(sv_state *st, const sv_pauli_term *terms, int32_t n_terms,
                                  double *out_terms, double *out_sum);

/* Adjoint gradient of E(theta) = <0|U^dag(theta) H U(theta)|0> (paper
 * Section 4.2 objective).  On entry *st holds the INITIAL state (normally
 * |0...0>); on return it holds U(theta)|initial>.  grad has n_params entries
 * (a parameter read by several gates sums their contributions).  n_evals
 * (may be NULL) receives 1 (one forward and one backward pass).  Needs a
 * workspace allocated with SV_WS_ADJOINT.  Every parameterised kind is
 * differentiated, with or without controls: Pauli rotations and phases by
 * their generator, U2 / U3 as P(phi) RY(theta) P(lambda) under the same
 * controls, single and double excitations by the Pauli-Y generator of their
 * rotated pair of basis patterns.  Errors: as sv_apply_layer, plus
 * SV_EUNSUPPORTED for an op on more than 4 qubits (targets and controls
 * together; the backward sweeps hold 4-qubit register groups), SV_ENOMEM. */
sv_status sv_adjoint_grad(sv_state *st, const sv_op *ops, int32_t n_ops, const double *params,
                          int32_t n_params, const sv_pauli_term *terms, int32_t n_terms,
                          double *energy, double *grad, int32_t *n_evals);

/* As sv_adjoint_grad but asynchronous: energy then grad (1 + n_params FP64)
 * are written to DEVICE memory d_out on the handle's stream.  The energy is
 * summed on the device in the library's term order (it may differ from
 * sv_adjoint_grad's host sum in the last bits).  The first call for a circuit
 * structure on a handle may allocate (plan, scratch) and synchronise the
 * handle's stream; later calls enqueue only. */
sv_status sv_adjoint_grad_device(sv_state *st, const sv_op *ops, int32_t n_ops,
                                 const double *params, int32_t n_params,
                                 const sv_pauli_term *terms, int32_t n_terms, double *d_out);

/* Terminal Z-basis sampling (paper Section 5.3 measurement path) by a fixed
 * order of floating-point operations, so equal states give equal bits:
 * p_b = fma(x,x,y*y) in FP64; chunk sums over 2^min(n,10) indices by pairwise
 * tree; prefix over chunks in blocks of 2^10 chunks (local prefixes left to
 * right, block totals prefixed left to right, P_k = block offset + local
 * prefix); u_s = (splitmix64(seed, s) >> 11) 2^-53;
 * inverse-CDF search with a strict '>' (see DESIGN notes for the fallbacks).
 * out[s] packs bit qubits[i] of the drawn index into bit i.  Waits. */
sv_status sv_sample(sv_state *st, uint64_t seed, int64_t shots, const int32_t *qubits,
                    int32_t n_measured, uint64_t *out);

/* Terminal readout counts (paper Section 4.4: terminal readout returns
 * bit-string counts): draws `shots` samples of the n_measured qubits exactly
 * as sv_sample does and writes the HOST array counts[2^n_measured], counts[b]
 * = number of draws whose packed bits (bit i = qubit qubits[i]) equal b.
 * n_measured <= SV_COUNTS_MAX_QUBITS.  Waits. */
#define SV_COUNTS_MAX_QUBITS 24
sv_status sv_sample_counts(sv_state *st, uint64_t seed, int64_t shots, const int32_t *qubits,
                           int32_t n_measured, uint64_t *counts);

/* Shot-based estimate of sum_j c_j <P_j> (paper Section 4.4 shot estimator:
 * Pauli terms rotated into their measurement bases, qubit-wise commuting
 * terms grouped, a shot budget split over the groups).  Fixed readings:
 * terms in order join the first group whose basis agrees on every shared
 * qubit (identity terms join none and are exact, value 1); group g of G gets
 * floor(shots/G) draws, one more if g < shots mod G, sampled with seed + g
 * from a copy of the state rotated by H (X qubits) or S^dagger then H (Y
 * qubits; applied as Z or S, then RY(pi/2)), reading the group's qubits in increasing order.  values[j] =
 * (N - 2*odd_j)/N with odd_j the draws of odd parity on term j's qubits;
 * *energy = sum_j c_j values[j] in term order; *variance = sum over groups of
 * sum_{j,k} c_j c_k (v_jk - v_j v_k) / N (v_jk: parity over the symmetric
 * difference of the two terms' qubits), the variance of the energy estimate.
 * The state is not modified; the first call allocates a second pair of
 * planes for the rotated copy.  shots >= number of groups; a group holds at
 * most SV_SHOT_GROUP_MAX_TERMS terms (SV_EUNSUPPORTED beyond).  Waits. */
#define SV_SHOT_GROUP_MAX_TERMS 1024
sv_status sv_shot_estimate(sv_state *st, uint64_t seed, int64_t shots, const sv_pauli_term *terms,
                           int32_t n_terms, double *values, double *energy, double *variance,
                           int32_t *n_groups);

/* ---------------------------------------------------- density matrices
 * (paper Section 4.1 density-matrix state; Section 5.3 runs rho as a vector
 * of twice the qubits.)  A handle of 2n qubits holds rho of n qubits as
 * vec(rho): rho_{rc} at index r 2^n + c, row bits on qubits n..2n-1.
 * sv_reset gives |0><0|.  Each call waits like the state-vector call it
 * builds on; errors as there, plus SV_EINVAL when the handle does not hold
 * 2n qubits. */

/* rho <- U rho U^dagger for the circuit (same op model and parameters as
 * sv_apply_layer): applied as U on the row qubits and conj(U) on the column
 * qubits (conjugated angles take negated copies of the parameters). */
sv_status sv_dm_apply(sv_state *st, int32_t n, const sv_op *ops, int32_t n_ops,
                      const double *params, int32_t n_params);

/* rho <- sum_k K_k rho K_k^dagger on each of the n_qubits distinct qubits
 * (streaming passes of the vector, up to four qubits per pass); kraus holds n_kraus HOST
 * 2x2 matrices, row-major, interleaved (re, im) complex128.  Trace
 * preservation (sum_k K_k^dagger K_k = I) is the caller's. */
sv_status sv_dm_apply_kraus(sv_state *st, int32_t n, const int32_t *qubits, int32_t n_qubits,
                            const double *kraus, int32_t n_kraus);

/* rho <- sum_k K_k rho K_k^dagger for a channel on the qubit pair (q0, q1);
 * kraus holds n_kraus HOST 4x4 matrices, row-major, interleaved (re, im),
 * local index bit(q0) + 2 bit(q1).  One streaming pass of the vector. */
sv_status sv_dm_apply_kraus2(sv_state *st, int32_t n, int32_t q0, int32_t q1, const double *kraus,
                             int32_t n_kraus);

/* out_terms[j] = Tr(rho P_j) (real part), *out_sum = sum_j c_j Tr(rho P_j),
 * summed in fixed orders. */
sv_status sv_dm_expect_pauli(sv_state *st, int32_t n, const sv_pauli_term *terms, int32_t n_terms,
                             double *out_terms, double *out_sum);

/* Copy amplitudes [offset, offset+count) of both planes to HOST buffers of
 * the state's element type (the paper's explicit to_numpy exit).  Waits. */
sv_status sv_copy_to_host(const sv_state *st, void *re, void *im, uint64_t offset,
                          uint64_t count);

/* Copy HOST amplitudes into [offset, offset+count) (checkpoint reload).  Waits. */
sv_status sv_copy_from_host(sv_state *st, const void *re, const void *im, uint64_t offset,
                            uint64_t count);

/* Thread-local message of the last failing call on this thread. */
const char *sv_last_error(void);

/* ------------------------------------------------------------ batching
 * A ragged batch of independent circuits (paper Section 4.1 batched state
 * vector, generalised to mixed qubit counts), run as ONE persistent launch
 * over a device work queue of (circuit, sweep, tile-range) units.  The plan
 * is built once per batch structure; sv_batch_run may be captured in a HIP
 * graph by the caller; parameters are read from device memory so replays
 * with new angles need no re-plan. */
typedef struct sv_batch sv_batch;

typedef struct {
  int32_t n_qubits;
  int32_t n_ops;
  const sv_op *ops;
  int32_t n_params;         /* parameters of this circuit (its own index space) */
  int32_t n_terms;          /* observable: sum of Pauli terms, reported per circuit */
  const sv_pauli_term *terms;
} sv_circuit_desc;

/* Plan a batch.  Every circuit gets its own tile plan (the planner of
 * sv_apply_layer with SV_FUSE_AUTO); its state starts at |0..0>.
 *   tile_bits   qubits per LDS tile (0 = 13, the only compiled value)
 *   low_bits    contiguous low qubits per tile (0 = 5)
 *   group_bits  qubits per register group (0 = the narrowest compiled width
 *               >= 3 that holds the widest op: 3 or 5)
 * Ops, terms and user matrices are read during the call and not kept (user
 * matrices are copied: later changes to them are not seen).  All device
 * memory (states, plan, queue) is allocated here with hipMalloc and released
 * by sv_batch_free.  Each circuit's observable must have every term's X/Y
 * support inside one 13-qubit tile (SV_EUNSUPPORTED otherwise).
 * Errors: SV_EINVAL (bad sizes, qubits, tiling), SV_EUNBOUND (parameter index
 * >= the circuit's n_params), SV_EDTYPE, SV_EUNSUPPORTED, SV_EDEVICE. */
sv_status sv_batch_plan(const sv_circuit_desc *circuits, int32_t n_circuits, sv_dtype dtype,
                        int32_t tile_bits, int32_t low_bits, int32_t group_bits, sv_batch **out);

/* Copy new angles into the batch: `params` is host memory holding every
 * circuit's parameters concatenated in circuit order (count = sum of
 * n_params).  Synchronous.  SV_EUNBOUND on a non-finite value. */
sv_status sv_batch_upload_params(sv_batch *b, const double *params, int64_t count);

/* Device pointer of the parameter vector; circuit c's parameters start at
 * element param_offset(c) (param_offset(n_circuits) = total length).  A
 * caller may write angles there directly, e.g. from another kernel. */
double *sv_batch_params_device(sv_batch *b);
int64_t sv_batch_param_offset(const sv_batch *b, int32_t circuit);

/* Enqueue the whole batch on `hip_stream`: reset the queue (a small kernel,
 * no memset), build gate coefficients from the device parameters, run the
 * persistent kernel, reduce each circuit's observable into the device array
 * returned by sv_batch_results_device (n_circuits FP64, sum_j c_j <P_j>).
 * Asynchronous; allocates nothing, so the caller may capture it in a graph.
 * Overlapping runs of one batch race. */
sv_status sv_batch_run(sv_batch *b, void *hip_stream);
double *sv_batch_results_device(sv_batch *b);

/* Same work as sv_batch_run, as a HIP graph that the library captures on its
 * first call (on a stream of its own) and launches on `hip_stream`. */
sv_status sv_batch_graph_launch(sv_batch *b, void *hip_stream);

/* Synchronise `hip_stream`, then SV_EDEVICE if a unit's bounded dependency
 * wait expired in the last run (its results are then invalid). */
sv_status sv_batch_check(sv_batch *b, void *hip_stream);

/* Polls of a dependency wait before it expires (default 1048576, about a second).  A
 * negative value skips every dependency wait and flags it as expired, so the
 * next sv_batch_check reports the error (tests of the error path). */
sv_status sv_batch_set_spin_limit(sv_batch *b, int32_t polls);

/* Device pointers to circuit c's state planes (valid until sv_batch_free). */
sv_status sv_batch_state(sv_batch *b, int32_t circuit, void **re, void **im);

/* Synchronous copies to host memory, ordered after the work on `hip_stream`:
 * the n_circuits observables, or circuit c's planes (2^n elements each, FP64
 * for SV_C128, FP32 for SV_C64). */
sv_status sv_batch_copy_results(sv_batch *b, double *out, void *hip_stream);
sv_status sv_batch_copy_state(sv_batch *b, int32_t circuit, void *re, void *im, void *hip_stream);

/* Statistics: work units in the queue, total sweeps, the sum over circuits
 * of n_ops * 2^n (gate-amplitude updates), and the algorithmic HBM bytes of
 * one run (each sweep reads and writes both planes, the first only writes;
 * each Pauli pass reads both planes).  Any output may be NULL. */
sv_status sv_batch_stats(const sv_batch *b, int64_t *units, int64_t *sweeps, double *updates,
                         double *bytes);

/* Wait for the device, then release the batch and its device memory. */
sv_status sv_batch_free(sv_batch *b);

/* Autotuner: plans the batch with every compiled tiling (register-group
 * width >= the widest op, contiguous low bits 2..5), times `reps` runs of each
 * on `hip_stream` with HIP events after one warm-up run, and returns the
 * fastest tiling (for sv_batch_plan) and its mean time in milliseconds.
 * `params` (concatenated, as for sv_batch_upload_params) may be NULL: all
 * angles 0.  Allocates and frees a batch per candidate; synchronous. */
sv_status sv_batch_autotune(const sv_circuit_desc *circuits, int32_t n_circuits, sv_dtype dtype,
                            const double *params, int32_t reps, void *hip_stream,
                            int32_t *tile_bits, int32_t *low_bits, int32_t *group_bits,
                            double *best_ms);

/* --------------------------------------------------------------- serving
 * Small adjoint requests (paper Section 4.1 batched state vector, with one
 * request per state; Section 6.3 task-parallel queues): each request is an
 * independent circuit with its own qubit count, angles and observable, and
 * asks for E = <psi|H|psi> and dE/dtheta by the adjoint method.  A submission
 * is one persistent launch over a device queue of requests; one workgroup
 * takes one request and runs all of it -- forward sweeps, lambda = H|psi>,
 * backward sweeps with the gradient terms, the gather into dE/dtheta -- with
 * the request's planes held in the L2 and last-level caches.  Results are bitwise independent
 * of the other requests in the submission (one workgroup, fixed order).
 * Requests must have 3 <= n_qubits <= sv_serve_max_qubits() (16), ops on at
 * most 3 qubits (targets and controls) and no user matrices; FP64 only.
 * Plans are built on first sight of a request structure (qubits, ops,
 * parameter count) and cached in the handle. */
typedef struct sv_serve sv_serve;

/* Handle; host-only until the first submission, which binds it to the
 * current device and allocates its device buffers there. */
sv_status sv_serve_create(sv_serve **out);
int32_t sv_serve_max_qubits(void);

/* SV_OK if the serving kernel takes this request (its plans are then built
 * and cached on the host); SV_EUNSUPPORTED (message says why) if it must run
 * through sv_adjoint_grad instead; SV_EINVAL for an invalid request.
 * Host-only: no device call. */
sv_status sv_serve_check(sv_serve *s, const sv_circuit_desc *request);

/* Enqueue `n_requests` (1..65535) requests on `hip_stream`.  `params` (host) holds every
 * request's n_params angles concatenated in request order; `d_out` (device,
 * FP64) receives, per request in order, 1 + n_params values: E, then
 * dE/dtheta_0 .. dE/dtheta_{n_params-1}.  Asynchronous: returns after the
 * host-to-device copy of one staging block and two kernel launches are
 * queued; `d_out` must stay valid until the stream passes them.  Up to four
 * submissions may be queued; a fifth waits for the oldest to finish.
 * Device buffers grow with hipMalloc when a submission needs more than the
 * largest so far.  Every request is checked before any device work; the
 * first refusal returns its status with the request index in the message.
 * Errors: SV_EINVAL, SV_EUNBOUND (bad parameter index or non-finite angle),
 * SV_EUNSUPPORTED, SV_EDEVICE. */
sv_status sv_serve_submit(sv_serve *s, const sv_circuit_desc *requests, int32_t n_requests,
                          const double *params, double *d_out, void *hip_stream);

/* Wait for queued submissions, then release the handle and its buffers. */
sv_status sv_serve_free(sv_serve *s);

/* ------------------------------------------------------- plan inspection
 * Number of full-state sweeps and register blocks sv_apply_layer would use
 * for this circuit with these settings (host-only; for tests and tuning). */
sv_status sv_plan_stats(int32_t n_qubits, const sv_op *ops, int32_t n_ops, int32_t fuse_width,
                        int32_t tile_bits, int32_t low_bits, int32_t group_bits,
                        int32_t *n_sweeps, int32_t *n_blocks);

/* Backward program sv_adjoint_grad would run for this circuit (FP64; 0 for a
 * setting = the default backward tiling): its tile sweeps, register stages
 * and gradient slots (host-only; for tests and tuning).  Errors as for
 * sv_adjoint_grad's op checks. */
sv_status sv_adjoint_plan_stats(int32_t n_qubits, const sv_op *ops, int32_t n_ops, int32_t n_params,
                                int32_t tile_bits, int32_t low_bits, int32_t group_bits,
                                int32_t *n_sweeps, int32_t *n_stages, int32_t *n_gslots);

/* Default tiling of sv_apply_layer (backward = 0) or of the backward sweeps
 * of sv_adjoint_grad (backward = 1) for an n_qubits state of this dtype, as
 * used by a handle without sv_set_tiling / sv_set_adjoint_tiling (host-only).
 * Writes the three values (see sv_set_tiling); SV_EINVAL on a bad dtype or
 * null output. */
sv_status sv_default_tiling(int32_t n_qubits, sv_dtype dtype, int32_t backward,
                            int32_t *tile_bits, int32_t *low_bits, int32_t *group_bits);

/* Tiling used by SV_FUSE_AUTO for a handle (0 = keep the default): tile_bits =
 * qubits per LDS tile, low_bits = contiguous low qubits in every tile (rows of
 * 2^low_bits elements in HBM), group_bits = qubits per register block.  A
 * combination without a compiled kernel is SV_EINVAL. */
sv_status sv_set_tiling(sv_state *st, int32_t tile_bits, int32_t low_bits, int32_t group_bits);

/* The same for the backward sweeps of sv_adjoint_grad (two states per tile). */
sv_status sv_set_adjoint_tiling(sv_state *st, int32_t tile_bits, int32_t low_bits,
                                int32_t group_bits);

/* Greedy in-order fusion (paper Section 9.2 ablation planner): block id per
 * op into block_of (host array of n_ops), returns the block count in *n_blocks. */
sv_status sv_fuse_blocks(const sv_op *ops, int32_t n_ops, int32_t width, int32_t *block_of,
                         int32_t *n_blocks);

/* Kernel-time instrumentation (for benchmarks).  While enabled, every tile
 * sweep launched for this handle is bracketed by HIP events recorded on the
 * handle's stream.  sv_timing_read waits for the stream and returns the summed
 * event time of those launches in milliseconds, their count, and their
 * algorithmic HBM bytes (read + write of both planes; write only for a sweep
 * that synthesises |0...0>), then clears the log. */
sv_status sv_timing_enable(sv_state *st, int32_t on);
sv_status sv_timing_read(sv_state *st, double *sweep_ms, int64_t *launches, double *bytes);

/* Library build identification (gfx target, compile flags). */
const char *sv_version(void);

#ifdef __cplusplus
}
#endif
#endif
