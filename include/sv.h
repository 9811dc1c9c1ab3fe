/*
 * sv.h -- C ABI of the MI355X state-vector sweep library (libsvmi.so).
 *
 * The library applies a quantum circuit to a 2^n complex amplitude vector in
 * place, Schroedinger style: every gate updates the 2^{n-k} disjoint sets of
 * 2^k amplitudes whose indices agree outside the gate's k qubits (Sec. 3,
 * "Fast Schroedinger simulation").  It starts from the basis vector
 * (1,0,...,0) (Sec. 2) and keeps every amplitude ("strong simulation").
 *
 * Conventions
 *   - Qubit q is bit q of the amplitude index (little-endian), as in the
 *     paper's bitmask examples (Sec. 4.3, Fig. reorder).
 *   - A gate's local index is l = sum_t bit(j, q[t]) * 2^t, so q[0] is the
 *     least significant bit of its matrix index.  CNOT: q[0] control,
 *     q[1] target (defined by action, Sec. 2).
 *   - Amplitudes are interleaved (re, im): SV_C64 = two floats (8 bytes),
 *     SV_C128 = two doubles (16 bytes), the layout of torch.complex64 /
 *     torch.complex128.
 *   - A context may hold a batch of B states of the same width stored back
 *     to back (state b at element offset b * 2^n); one circuit is applied to
 *     all of them, with per-state parameter vectors.
 *
 * Ownership
 *   - Device buffers (states, adjoint scratch) belong to the caller.  The
 *     library borrows the raw device pointers, never frees them, and needs
 *     them to stay valid for the lifetime of the context.
 *   - The library owns the context, its plan cache and its device work
 *     areas (plans, reduction partials, sampling trees), released by
 *     sv_destroy.
 *   - Host arrays passed to a call are read during the call only.
 *
 * Errors
 *   - Every entry point validates its arguments synchronously and returns a
 *     non-SV_OK status with a message (sv_last_error) without touching the
 *     state when validation fails.
 *   - Kernels run asynchronously on the context's HIP stream.  A device
 *     fault surfaces as SV_EDEVICE from the next call that synchronises
 *     (sv_expect, sv_norm, sv_apply_circuit_norm, sv_sample, sv_amplitudes,
 *     sv_adjoint_grad, sv_sync, sv_apply_batch).
 *   - No C++ exception crosses this boundary.  A context is not thread-safe;
 *     separate contexts are independent.
 */
#ifndef SV_H_
#define SV_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SV_OK = 0,
    SV_EINVAL = 1,        /* bad argument (qubit range, sizes, alignment, op code, ...) */
    SV_ENOMEM = 2,        /* device or host allocation failed */
    SV_EDEVICE = 3,       /* HIP runtime / kernel error */
    SV_EUNSUPPORTED = 4   /* valid request the library does not support */
} sv_status;

typedef enum { SV_C64 = 1, SV_C128 = 2 } sv_dtype;

/* Gate vocabulary.  Sec. 2 defines NOT (X), H, Z, CNOT, CZ, P = Z^(1/2) (S),
 * X^(1/2), Y^(1/2) and T; Sec. 4.3 adds P = T^2, Z = T^4.  sqrt(Y) is the
 * principal square root (it squares to Y).  Rotations are exp(-i theta P/2),
 * SV_OP_P is diag(1, e^{i theta}), SV_OP_CP is diag(1,1,1,e^{i theta}).
 * SV_OP_MAT is an explicit 2^nq x 2^nq matrix (nq <= 6) from sv_circuit.mats;
 * SV_OP_DIAG an explicit diagonal of 2^nq entries (a diagonal gate of
 * Sec. 4.3 with arbitrary phases or magnitudes), also from mats. */
typedef enum {
    SV_OP_I = 0, SV_OP_H = 1, SV_OP_X = 2, SV_OP_Y = 3, SV_OP_Z = 4,
    SV_OP_S = 5, SV_OP_SDG = 6, SV_OP_T = 7, SV_OP_TDG = 8,
    SV_OP_SQRTX = 9, SV_OP_SQRTY = 10, SV_OP_SQRTW = 11,
    SV_OP_SQRTXDG = 12, SV_OP_SQRTYDG = 13, SV_OP_SQRTWDG = 14,
    SV_OP_RX = 15, SV_OP_RY = 16, SV_OP_RZ = 17, SV_OP_P = 18,
    SV_OP_CZ = 19, SV_OP_CNOT = 20, SV_OP_SWAP = 21, SV_OP_CP = 22,
    SV_OP_MAT = 23, SV_OP_DIAG = 24,
    SV_OP_COUNT_ = 25
} sv_op;

/* One gate.  nq: number of qubits (1..6).  param: index into the parameter
 * vector for angle gates (theta used when param < 0).  mat: offset, in
 * doubles, of the gate's matrix in sv_circuit.mats (SV_OP_MAT: row-major,
 * interleaved complex, 2^nq x 2^nq; SV_OP_DIAG: 2^nq interleaved complex
 * diagonal entries). */
typedef struct {
    int32_t op;
    int32_t nq;
    int32_t q[6];
    int32_t param;
    int32_t mat;
    double theta;
} sv_gate;

typedef struct {
    int32_t n_qubits;
    int32_t n_gates;
    const sv_gate* gates;
    int64_t n_mat_doubles;
    const double* mats;
    int32_t n_params;
} sv_circuit;

/* Observable sum_k coeff[k] * P_k with P_k = i^{|x&z|} X^x Z^z (Y = iXZ on a
 * qubit whose x and z bits are both set).  Host arrays of n_terms entries. */
typedef struct {
    int32_t n_terms;
    const double* coeff;
    const uint64_t* x_mask;
    const uint64_t* z_mask;
} sv_pauli_sum;

typedef struct {
    int32_t max_fuse_k;    /* structured = 0: gates are fused into dense blocks of at most this many
                              qubits, 1..6 (default 4); blocks of 5-6 qubits run as plain kernels */
    int32_t tile_bits;     /* local qubits per tile pass, 0 = default */
    int32_t low_bits;      /* contiguous low bits per tile segment, 0 = default */
    int32_t plain;         /* 1 = one kernel per gate, no reordering or fusion */
    int32_t threads;       /* workgroup size of tile passes, 0 = default */
    int32_t product_init;  /* 1 = fold leading one-qubit gates into the init of |0..0> */
    int32_t structured;    /* 1 = H, sqrt(X), sqrt(Y), sqrt(W) and inverses as multiply-free H'
                              butterflies with the diagonal phases applied lazily (default) */
    int32_t timing;        /* 1 = time every tile-pass launch with HIP events (sv_timing) */
    int32_t jit;           /* run-time specialised tile passes: 0 auto (batch * 2^n >= 2^24),
                              1 always, -1 never */
    int32_t max_work_mib;  /* cap, in MiB, on the device memory the library allocates for a context
                              (plans, pools, reduction and sampling scratch) or a batch call's work
                              area; 0 = no cap.  A call that would exceed it returns SV_ENOMEM */
    int32_t batch_tuned;   /* sv_apply_batch: 1 = items of every width that sv_tune_batch has tuned
                              (same dtype and direction) use its fusion mode and tile geometry */
    int32_t paper;         /* sv_apply_circuit: the paper's own plan instead of tile passes, for
                              ablations: 1 = kind clusters (Sec. 4.2, 4.5) with one pass per
                              diagonal cluster (bitmask phases, Gray-code CZ, Sec. 4.3) and per pair
                              of one-qubit gates (multiply-free unnormalised products, scale and
                              phase counters with rescale passes, Sec. 4.1, 4.4); 2 = the same with
                              the recursive transform of Sec. 5.1 (a layer's low-qubit gates on
                              LDS-staged chunks); 0 = tile passes (default) */
    int32_t plan_beam;     /* tile-pass planner (Sec. 4.5 reordering): width of the beam search
                              over the sequence of the passes' local qubit sets, 1..64; 1 = the
                              greedy set of each pass alone.  0 = default: 8, or 16 for SV_C128
                              contexts.  Any width gives the same state up to rounding; a wider
                              search costs host planning time (about 0.1 s at width 8 for 1 900
                              gates on 33 qubits, about 1.7x the greedy planning of a batch item;
                              plans are cached by circuit structure) and never yields more
                              passes than width 1 */
} sv_opts;

typedef struct {
    int32_t gates_in;       /* gates in the circuit */
    int32_t passes;         /* full-state read+write sweeps (tile passes + plain kernels) */
    int32_t phases;         /* LDS register phases over all passes */
    int32_t dense_ops;      /* dense blocks applied */
    int32_t diag_ops;       /* diagonal (phase/sign) ops applied */
    int32_t launches;       /* kernel launches */
    int32_t folded_init;    /* gates folded into the product-state init */
    int32_t reserved;
    double plan_ms;         /* host planning time (0 on a plan-cache hit) */
    double hbm_bytes;       /* algorithmic HBM bytes moved by the sweep */
    double flops;           /* algorithmic floating-point operations (an FMA counts 2) */
    double alu_ops;         /* algorithmic vector arithmetic instructions per lane of the
                               tile passes (an FMA counts 1): the ALU-side roofline.
                               sv_adjoint_grad counts the forward and backward sweeps
                               (gradient terms included), sv_apply_batch all items */
} sv_stats;

typedef struct sv_ctx_s* sv_ctx;

enum { SV_INIT_ZERO = 0, SV_INIT_BASIS = 1, SV_INIT_UNIFORM = 2, SV_INIT_ZERO_DEFERRED = 3 };

/* Fill *opts with the defaults. */
void sv_opts_default(sv_opts* opts);

/* Create a context over caller-owned device memory holding the state of
 * Sec. 2: n qubits described by 2^n complex amplitudes, amplitude j at
 * element j (qubit q = bit q of j), stored in place and kept whole for the
 * lifetime of the context (the strong simulation of Sec. 3).
 *   n_qubits   1..34 (SV_C64) or 1..33 (SV_C128)
 *   batch      number of states (>= 1, <= 65535) stored back to back in d_state
 *   d_state    device pointer, 16-byte aligned; borrowed, never freed
 *   state_bytes must equal batch * 2^n * bytes-per-amplitude
 *   hip_stream hipStream_t to launch on (NULL = default stream)
 *   opts       NULL = defaults (copied)
 * The context itself is host memory owned by the library (sv_destroy).
 * Errors: SV_EINVAL for a NULL out or d_state, n or batch out of range, a
 * wrong state_bytes, misalignment or out-of-range options (nothing is
 * created); SV_ENOMEM; SV_EDEVICE when the device cannot be configured. */
sv_status sv_create(sv_ctx* out, int32_t n_qubits, sv_dtype dtype, int32_t batch,
                    void* d_state, size_t state_bytes, void* hip_stream, const sv_opts* opts);
sv_status sv_destroy(sv_ctx ctx);
sv_status sv_set_stream(sv_ctx ctx, void* hip_stream);
sv_status sv_set_opts(sv_ctx ctx, const sv_opts* opts);

/* Initialise every state of the batch: SV_INIT_ZERO (|0..0>), SV_INIT_BASIS
 * (|basis_index>), SV_INIT_UNIFORM (all amplitudes 2^{-n/2}, the result of a
 * Hadamard layer on |0..0>, Sec. 4.5 footnote).  SV_INIT_ZERO_DEFERRED
 * records |0..0> without writing it: the next library call that reads the
 * state writes it first, unless the next sweep starts with one-qubit gates
 * that are folded into a product-state initialisation (then the state is
 * written once).  Reading the buffer directly before such a call sees stale
 * data, and a caller's write to it in between is ignored.  After every other
 * kind the buffer's content is the input of the next sweep, caller writes
 * included (no folding). */
sv_status sv_init(sv_ctx ctx, int32_t kind, uint64_t basis_index);

/* Apply a circuit to every state of the batch, in place: psi <- U_G ... U_1
 * psi, where each gate updates every one of the 2^{n-k} disjoint sets of
 * 2^k amplitudes whose indices differ only in the gate's k qubits (Sec. 3,
 * fast Schroedinger simulation).  Gates are reordered only where they
 * commute and clustered into tile passes (Sec. 4.2, 4.5), diagonal phases
 * are consolidated (Sec. 4.3) and the H / sqrt(X) / sqrt(Y) family runs as
 * multiply-free butterflies (Sec. 4.4); the result differs from the gate by
 * gate product only by rounding.
 *   circuit  host, read during the call; n_qubits must equal the context's
 *   params   host FP64, batch * n_params values (row b = state b); may be
 *            NULL when no gate is parameterised
 *   stats    host, may be NULL: passes, launches, plan time, algorithmic
 *            bytes, flops and ALU instructions
 * Asynchronous on the context's stream (plans are uploaded synchronously).
 * Errors (before any kernel, state untouched): SV_EINVAL for an unknown op,
 * nq outside 1..6 or not the op's arity, a qubit out of range or repeated,
 * param >= n_params, a matrix offset outside mats, NULL or non-finite
 * params; SV_ENOMEM when a work area cannot be allocated (or exceeds
 * max_work_mib); SV_EUNSUPPORTED when planning fails. */
sv_status sv_apply_circuit(sv_ctx ctx, const sv_circuit* circuit, const double* params,
                           sv_stats* stats);

/* sv_apply_circuit followed by the norm check of Sec. 4.1 in the same
 * sweep: norm2_out (host, batch doubles) receives ||psi_b||^2 in FP64.
 * When the plan ends with a tile pass, that pass sums |psi_j|^2 of every
 * tile as it writes it (fixed order: lanes, waves, then the tiles in two
 * fixed-order steps), so the norm costs no extra read of the state;
 * otherwise a separate FP64 reduction runs.  Synchronises.
 * Errors: those of sv_apply_circuit, and SV_EINVAL for a NULL norm2_out. */
sv_status sv_apply_circuit_norm(sv_ctx ctx, const sv_circuit* circuit, const double* params,
                                double* norm2_out, sv_stats* stats);

/* Expectation of a Pauli sum: out[b] = sum_k coeff_k Re <psi_b|P_k|psi_b>.
 * Every amplitude product is formed and summed in FP64 on the device
 * (the FP64 accumulation the norm check of Sec. 4.1 calls for a float
 * state), over a fixed grid and a fixed tree, so results repeat bit for
 * bit.  Terms that share an x mask share one read of the state.
 *   obs  host arrays of n_terms entries; masks must lie inside the register
 *   out  host, batch doubles
 * Synchronises the stream.  Errors: SV_EINVAL for NULL pointers, masks
 * outside the register or a non-finite coefficient (nothing launched);
 * SV_ENOMEM; SV_EDEVICE from earlier asynchronous work. */
sv_status sv_expect(sv_ctx ctx, const sv_pauli_sum* obs, double* out);

/* sv_expect for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same result as sv_expect, bit for bit, but the
 * library allocates nothing.  Its Pauli tables, block partials and results
 * live in a fixed per-device work area of 4 MiB (a file-scope device array
 * that each GPU holds until the process ends); a call needs about
 * 24 bytes per Pauli term + 8 * batch * min(8192, 2^n / 2048) + 8 * batch
 * bytes of it and fails with SV_EINVAL, before any device work, when that
 * exceeds 4 MiB.  Every call on one GPU shares that area and leaves its
 * contents behind: calls that overlap on one GPU (other streams, other
 * threads) race and must be serialised by the caller.  Synchronises the
 * stream.  Errors: those of sv_expect, and SV_EINVAL when the work area is
 * too small. */
sv_status sv_expect_noalloc(sv_ctx ctx, const sv_pauli_sum* obs, double* out);

/* Copies the states of src into dst (a snapshot, or a branch point for two
 * continuations of one simulation).  Both contexts must have the same
 * width, dtype and batch, and disjoint state buffers.  Enqueued on dst's
 * stream; when src uses another stream, the call first waits for it.  A
 * pending deferred |0..0> in src is passed on without a copy.  The copy
 * streams 16-byte words with several loads in flight per thread.
 * Errors: SV_EINVAL for NULL or mismatched contexts or overlapping buffers. */
sv_status sv_copy_state(sv_ctx dst, sv_ctx src);

/* out[b] = ||psi_b||^2 in FP64 (norm check of Sec. 4.1).  Synchronises. */
sv_status sv_norm(sv_ctx ctx, double* out);

/* Measurement of every qubit in the computational basis (Sec. 2: the state
 * vector gives the probability |psi_j|^2 of every output bit string j), by
 * inverse-CDF sampling with the caller's random numbers:
 *   uniforms  host, batch * count values in [0, 1) (row b = state b)
 *   out       host, batch * count indices: out[b * count + k] is the
 *             smallest j with sum_{i <= j} |psi_b[i]|^2 > u * ||psi_b||^2,
 *             u = uniforms[b * count + k].
 * The prefix sums are FP64 and taken over a 64-ary tree of probability
 * masses (node = sum of 64 children) built on the device in one pass over
 * the state; every sample then descends the tree on the device.  A target
 * that rounding puts at or past the end of a subtree maps to its last
 * amplitude of nonzero probability.  Device memory: about 1/64 of the state
 * in FP64 tree nodes plus 16 bytes per sample, kept by the context.
 * Synchronises.
 * Errors: SV_EINVAL for NULL pointers, uniforms outside [0, 1), more than
 * 2^32 samples (batch * count) in one call, or a state of zero or
 * non-finite norm (out is then unspecified). */
sv_status sv_sample(sv_ctx ctx, int64_t count, const double* uniforms, uint64_t* out);

/* Amplitude readout: out[2 * (b * count + k)] and out[2 * (b * count + k) + 1]
 * are the real and imaginary parts of psi_b[indices[k]] (host arrays; indices
 * must be < 2^n, batch * count at most 2^32).  Synchronises.
 * Errors: SV_EINVAL for NULL pointers, an index out of range or too many
 * values. */
sv_status sv_amplitudes(sv_ctx ctx, int64_t count, const uint64_t* indices, double* out);

/* Adjoint gradient of E_b = <psi_b|H|psi_b> with psi_b = U(theta_b) psi_b^in,
 * where psi_b^in is the current state.  Not in the paper: this is the
 * published adjoint-differentiation method for expectation values (Jones and
 * Gacon, 2020, arXiv:2009.02823) built on the paper's sweep.  Runs the
 * forward sweep (as sv_apply_circuit), forms lambda = H psi in d_scratch,
 * then sweeps back through the gates, un-computing both vectors with the
 * inverse gates instead of storing intermediate states, and accumulates
 * grad[p] = sum over gates l using p of Im <lambda_l|G_l|psi_l> (G_l the
 * generator of exp(-i theta G_l / 2)) with FP64 reductions.
 *   d_scratch   device, caller-owned, >= state_bytes, 16-byte aligned: lambda
 *   energy_out  host, batch values
 *   grad_out    host, batch * n_params values (row b = state b)
 * On return the state holds U^dagger U psi^in (psi^in up to rounding).
 * Synchronises.  Errors: those of sv_apply_circuit and sv_expect, and
 * SV_EINVAL for a NULL or too small d_scratch or NULL outputs. */
sv_status sv_adjoint_grad(sv_ctx ctx, const sv_circuit* circuit, const double* params,
                          const sv_pauli_sum* obs, void* d_scratch, size_t scratch_bytes,
                          double* energy_out, double* grad_out, sv_stats* stats);

/* One item of a heterogeneous batch (circuits of different widths). */
typedef struct {
    const sv_circuit* circuit;
    const double* params;        /* host, circuit->n_params values (may be NULL) */
    void* d_state;               /* device, 2^n amplitudes of dtype, holds the input state */
    void* d_lambda;              /* device scratch of the same size (gradients only) */
    const sv_pauli_sum* observable;
} sv_batch_item;

enum { SV_BATCH_FORWARD = 1, SV_BATCH_GRAD = 2, SV_BATCH_INIT_ZERO = 4, SV_BATCH_ENERGY = 8 };

/* Heterogeneous batch: many circuits of different widths, each swept as by
 * sv_apply_circuit (Sec. 3 with the planning of Sec. 4) and, with
 * SV_BATCH_GRAD, differentiated as by sv_adjoint_grad (adjoint method of
 * Jones and Gacon, arXiv:2009.02823).  Not in the paper: one persistent
 * kernel launch per direction runs every item -- resident workgroups pull
 * (item, pass, tile) work from per-XCD device queues, and a tile waits only
 * for the tiles of its own item's previous pass.  Circuits of at most 12
 * qubits are one tile (the whole state in LDS for the whole circuit).
 *   items     host, count entries; states and lambdas device, 16-byte aligned
 *   dtype     of every state
 *   flags     SV_BATCH_FORWARD or SV_BATCH_GRAD, | SV_BATCH_INIT_ZERO to start
 *             every state at |0..0> (else the buffers hold the inputs)
 *   energies  host, count values (needs observables)
 *   grads     host, concatenation of every item's n_params gradients (may be
 *             NULL without SV_BATCH_GRAD)
 *   opts      tile geometry and fusion; NULL = defaults
 * The library keeps two grow-only device work areas per device across calls
 * (one per launch) and a side stream of default priority for uploads.  The
 * backward plans are built on the host while the forward launch runs (not
 * with max_work_mib, where everything is planned first); stats->plan_ms is
 * the host work before the first launch.  Batches with gates of more than 4
 * qubits, or dense fusion beyond 4 qubits, run item by item.
 * Synchronises the stream.  Errors: SV_EINVAL for a NULL or invalid item
 * (as sv_apply_circuit), SV_ENOMEM (including max_work_mib), SV_EDEVICE;
 * after an error the states are unspecified. */
sv_status sv_apply_batch(int32_t count, const sv_batch_item* items, sv_dtype dtype,
                         void* hip_stream, int32_t flags, double* energies, double* grads,
                         const sv_opts* opts, sv_stats* stats);

typedef struct sv_batch_job_s* sv_batch_job;

/* sv_apply_batch in two halves, so that a caller can prepare its next batch
 * while the GPU runs the current one (not in the paper).  sv_apply_batch_async
 * validates, plans, uploads and queues every launch of the batch on the
 * stream, then returns without waiting; *job receives a handle.  The items,
 * circuits, parameters and observables may be released on return; the
 * device states and lambdas must stay until the job is finished.  Energies
 * are computed with SV_BATCH_GRAD, or in a forward batch with
 * SV_BATCH_ENERGY (every item then needs an observable).  Two jobs may be in
 * flight per device (each holds one of the device's two work-area slots); a
 * third call, asynchronous or not, fails with SV_EINVAL until one is
 * finished.  Work queued on the same stream runs in order, so consecutive
 * jobs on the same states are safe.  Errors: those of sv_apply_batch, found
 * before anything is queued; a failed call returns no job. */
sv_status sv_apply_batch_async(int32_t count, const sv_batch_item* items, sv_dtype dtype,
                               void* hip_stream, int32_t flags, const sv_opts* opts, sv_batch_job* job);

/* Waits for a job of sv_apply_batch_async, writes its results and releases
 * it (the handle is invalid afterwards, also on error).
 *   energies  host, count values (NULL if the job computed none)
 *   grads     host, the items' n_params gradients concatenated (NULL without
 *             SV_BATCH_GRAD)
 *   stats     may be NULL; plan_ms is the host work before the first launch
 * Errors: SV_EINVAL for a NULL job or missing outputs (the job is still
 * waited for and released), SV_EDEVICE for a device error or a dependency
 * wait that exceeded its time budget. */
sv_status sv_batch_finish(sv_batch_job job, double* energies, double* grads, sv_stats* stats);

/* Autotuner of the batched launch (the block-size choice of Sec. 5.1 made by
 * measurement, and the fusion width): for every width among the items, times
 * one persistent launch of that width's items under candidate fusion modes
 * (butterflies with lazily applied phases; dense blocks of 2, 3 or 4
 * qubits), then 2^T-amplitude tiles from T = 11 up to the default size (a
 * larger tile for one width would raise the LDS of every workgroup of a
 * mixed launch) and 2^L-amplitude segments (L = 3..5) around the best,
 * keeping a change only when it is more than
 * 3 % faster.  The choices are remembered per (dtype, direction, width) in
 * the process and in $SVMI_BATCH_TUNE_CACHE (default
 * /tmp/svmi-batch-tune.txt); sv_apply_batch uses them when opts.batch_tuned
 * is set.  flags as for sv_apply_batch (SV_BATCH_GRAD tunes the gradient
 * direction).  The items' states (and lambdas) are overwritten: initialise
 * them afterwards.  widths_tuned (may be NULL) receives the number of widths
 * tuned.  Errors: those of sv_apply_batch. */
sv_status sv_tune_batch(int32_t count, const sv_batch_item* items, sv_dtype dtype, void* hip_stream, int32_t flags,
                        const sv_opts* opts, int32_t* widths_tuned);

/* The remembered choice of sv_tune_batch for one width: out->structured,
 * max_fuse_k, tile_bits and low_bits (0 = default).  Host only.
 * Errors: SV_EINVAL when that width has not been tuned. */
sv_status sv_batch_tuning(sv_dtype dtype, int32_t grad, int32_t n_qubits, sv_opts* out);

/* Accumulated tile-pass kernel time since the last call (needs opts.timing):
 * total milliseconds, number of launches and the algorithmic HBM bytes of
 * those launches (one read and one write of every amplitude per launch).
 * Synchronises the stream and resets the counters. */
sv_status sv_timing(sv_ctx ctx, double* tile_ms, int64_t* tile_launches, double* tile_bytes);

/* Tile-geometry autotuner (the block-size choice of Sec. 5.1, made by
 * measurement): applies `circuit` once per candidate geometry -- 2^T-amplitude
 * tiles for T in {12, 13, 14} (c64; 14 from 14 qubits on, one 128 KiB workgroup
 * per CU) or {11, 12} (c128), 2^L-amplitude contiguous segments for L in
 * {4, 5} -- to the context's state, times the second of two
 * sweeps with HIP events, and keeps the fastest in the context's options
 * (tile_bits, low_bits, threads).  The state's content is destroyed:
 * initialise it afterwards.  Results are remembered per (width, dtype, batch,
 * circuit structure, options) in the process and in a text file
 * ($SVMI_TUNE_CACHE, default /tmp/svmi-tune.txt); a remembered result is
 * applied without running (best_ms = -1).  chosen, best_ms may be NULL. */
sv_status sv_tune(sv_ctx ctx, const sv_circuit* circuit, const double* params, sv_opts* chosen, double* best_ms);

/* Plan a circuit on the host only (no device work) and report its shape in
 * *stats (passes, phases, dense/diagonal ops, plan time, algorithmic bytes
 * and flops for one state).  `adjoint` = 1 plans the backward sweep.
 * Usable without a GPU. */
sv_status sv_plan_info(const sv_circuit* circuit, sv_dtype dtype, int32_t adjoint, const sv_opts* opts,
                       sv_stats* stats);

/* Host-only trace of the fused plan of `circuit` (parameters of one state in
 * `params`, NULL when n_params == 0): the operations the tile passes apply,
 * in order, in global-qubit terms (Sec. 4.3 phase forms, Sec. 4.4 butterflies,
 * dense and diagonal blocks, scales).  One text line per operation:
 *   PASS q...            local qubits of a tile pass
 *   PHASE q0 q1 q2 q3    qubits of a register phase
 *   BF q m p...          (x, y) <- (x + t y, x - t y) on qubit q, y = bit set,
 *                        t = e^{i pi m/4} (-1)^(sum of the bits of qubits p)
 *   FORM c aQ:v... bA,B:v...  multiply amplitude j by e^{i pi e(j)/4},
 *                        e = c + sum v j_Q + sum v j_A j_B
 *   DENSE k q... (re im)...   row-major 2^k x 2^k matrix, local bit t = qubit q[t]
 *   DENSE1 1 q (re im)x4 [| p...]  (x, y) <- (u00 x + s u01 y, u10 x + s u11 y) on qubit q,
 *                        s = (-1)^(sum of the bits of qubits p)
 *   DIAG k q... (re im)...    2^k diagonal entries
 *   SCALE s              multiply every amplitude by s
 *   GRAD p gen s q...    adjoint plans: parameter p gains s * Im<lambda|G|psi>, G = X, Y,
 *                        Z (gen 1, 2, 3) on q or -2|11><11| (gen 4) on q0 q1
 * Product-state folding of leading gates is off for the trace.  With
 * opts.paper set, the trace is the paper's plan instead, one line per kind
 * cluster:
 *   DIAG e8 b0 b1 b2 cz k:m... | g...   8th-root phase exponent bit-planes
 *                        and the one-sided CZ masks m_k (partners below k),
 *                        binary with qubit n-1 first
 *   LAYER op m | g...    one-qubit gates of kind op on the qubits of mask m
 *   GATES | g...         gates applied one by one
 * where g... are the circuit's gate indices in the order applied.  Writes at
 * most cap-1 bytes plus a NUL to buf and the full length to *len.  Usable
 * without a GPU. */
sv_status sv_plan_trace(const sv_circuit* circuit, const double* params, sv_dtype dtype, int32_t adjoint,
                        const sv_opts* opts, char* buf, size_t cap, size_t* len);

/* ---- Schroedinger-Feynman mode (Sec. 1, Sec. 6: the paper's second mode,
 * whose Schroedinger sweeps it accelerates; built here from the path sum).
 * The register is cut into half A (the qubits set in half_mask) and half B.
 * Every gate across the cut (CZ, CP or CNOT; any other is SV_EUNSUPPORTED)
 * is the sum of two products of one-half operators, |0><0| (x) I +
 * |1><1| (x) U, so the circuit is a sum over 2^c paths (c = cross gates) of
 * products of half-width states: psi[j] = sum_s A_s[jA] B_s[jB], where jA
 * and jB gather the bits of j on each half in qubit order.  Both halves
 * start at |0..0>.  Path bits are carried as extra high qubits of each
 * half's buffer, added at their cross gates (so a gate before a cross gate
 * is applied once for all the paths that share it); when the work area
 * cannot hold them all, the last cross gates are enumerated one assignment
 * at a time from a checkpoint.  The path sum of each requested amplitude is
 * accumulated in FP64. */
typedef struct sv_sf_s* sv_sf;

typedef struct {
    int32_t n_qubits, n_a, n_b;   /* register and half widths */
    int32_t n_cross;              /* gates across the cut = path bits */
    int32_t n_inner;              /* path bits held in memory for the given work size (-1: none fits) */
    int32_t n_outer;              /* path bits enumerated one assignment at a time */
    double paths;                 /* 2^n_cross */
    size_t work_bytes_all_inner;  /* device work bytes to hold every path bit */
    size_t work_bytes_min;        /* device work bytes with every path bit enumerated */
} sv_sf_info;

/* Host only: cut statistics and work sizes for `work_bytes` of device work
 * area.  Errors: SV_EINVAL (bad circuit, dtype), SV_EUNSUPPORTED (a gate
 * across the cut other than CZ, CP, CNOT; an empty half). */
sv_status sv_sf_plan(const sv_circuit* circuit, uint64_t half_mask, sv_dtype dtype, size_t work_bytes,
                     sv_sf_info* info);

/* Create a Schroedinger-Feynman simulator of `circuit` (copied) over a
 * caller-owned device work area (256-byte aligned, borrowed for the life of
 * the object): the two half buffers and, when path bits are enumerated,
 * their checkpoints.  Errors: those of sv_sf_plan, SV_EINVAL when the work
 * area holds no split, SV_ENOMEM, SV_EDEVICE. */
sv_status sv_sf_create(sv_sf* out, const sv_circuit* circuit, uint64_t half_mask, sv_dtype dtype, void* d_work,
                       size_t work_bytes, void* hip_stream, const sv_opts* opts);
sv_status sv_sf_destroy(sv_sf sf);

/* Amplitudes psi[indices[k]] of U(params)|0..0>, k < count: out[2k], out[2k+1]
 * (host FP64) = real and imaginary part.  params: host, n_params values (may
 * be NULL without parameters).  The first call plans (and compiles) every
 * half-width sweep.  stats (may be NULL): passes, launches and algorithmic
 * bytes of the sweeps, copies and path contractions.  Synchronises.
 * Errors: SV_EINVAL for NULL pointers, indices >= 2^n, NULL or non-finite
 * params; SV_ENOMEM; SV_EDEVICE. */
sv_status sv_sf_amplitudes(sv_sf sf, const double* params, int64_t count, const uint64_t* indices, double* out,
                           sv_stats* stats);

/* Wait for the context's stream and report any device error. */
sv_status sv_sync(sv_ctx ctx);

/* Thread-local description of the last non-OK status ("" if none). */
const char* sv_last_error(void);

/* Library version string. */
const char* sv_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SV_H_ */
