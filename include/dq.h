/*
 * dq.h -- C ABI of libdq, a gfx950 (MI355X) state-vector engine for batched
 * parameterised qubit circuits: gate application, Pauli-sum expectation
 * values and adjoint-method gradients.
 *
 * The operations follow the paper's qubit simulator (DeepQuantum, arXiv
 * 2512.18995):
 *   - a circuit is an ordered list of gates on wires, applied to a start
 *     state:  |psi_M> = U_M ... U_1 |psi_0>           (section 4.1, eq. of
 *     pure-state evolution; section 4.2, QubitCircuit API);
 *   - gate angles are trainable parameters or encoded data
 *     (section 4.2, listing code:qubitcircuit, "encode=True");
 *   - observables are Pauli strings, one expectation per observable and per
 *     batch sample, [batch, n_obs]             (section 4.2, expectation());
 *   - gradients come from the adjoint differentiation method behind a
 *     custom autograd Function               (section 7.2, distributed sim.);
 *   - samples are processed as a batch       (section 4.3, batch processing).
 *
 * Conventions
 *   - state layout: [batch][2^n] complex, (re, im) interleaved, complex64
 *     (float2) or complex128 (double2), contiguous; sample b starts at
 *     b * 2^n amplitudes.  Flat index j = sum_w bit_w * 2^(n-1-w): wire 0 is
 *     the most significant bit (the leftmost ket factor);
 *   - RX/RY/RZ(t) = exp(-i t P / 2), RZZ(t) = exp(-i t Z(x)Z / 2),
 *     CP(t) = diag(1, 1, 1, e^{i t}) on (control, target), CNOT flips the
 *     target where the control is 1, CZ negates |11>, H = (X + Z)/sqrt 2;
 *   - a gate angle is  scale * value  with value = params[idx] (per sample
 *     row when params_bstride != 0), data[idx] (per sample row when
 *     data_bstride != 0), or 1 for fixed gates;
 *   - params, data, expectations, gradient weights and gradients are float64
 *     device arrays for both state types.  Gate matrices are formed in
 *     double on the device and rounded once to the state's precision.
 *
 * Ownership and memory
 *   - every device buffer passed in (state, params, data, outputs,
 *     workspace) belongs to the caller; libdq never frees them;
 *   - a plan / observable owns copies of the host arrays given at creation
 *     and a small device buffer (op tables, fixed matrices) that it
 *     allocates on its first use on a device and frees in *_destroy;
 *   - nothing else is allocated: all scratch space is the caller's
 *     workspace, sized by dq_workspace_size.
 *
 * Errors and asynchrony
 *   - every call validates its arguments on the host before enqueueing any
 *     work; on failure nothing is enqueued, the status is returned and
 *     dq_last_error() describes it (thread-local, valid until the next call
 *     on the same thread);
 *   - device work is asynchronous on `stream` (a hipStream_t; NULL = the
 *     null stream).  Faults of earlier device work surface as DQ_ERR_HIP on
 *     a later call or at the caller's synchronisation;
 *   - the functions are re-entrant for distinct plans; concurrent calls on
 *     one plan are safe once it has been used once on each device.
 */
#ifndef DQ_H
#define DQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DQ_VERSION 1
#define DQ_MAX_QUBITS 34          /* 2^34 complex64 amplitudes = 137 GB */
#define DQ_MAX_GATE_QUBITS 5

typedef enum {
    DQ_OK = 0,
    DQ_ERR_INVALID_ARG = 1,    /* null pointer, bad wire, bad index, bad size */
    DQ_ERR_UNSUPPORTED = 2,    /* op / dtype / combination not implemented */
    DQ_ERR_WORKSPACE = 3,      /* ws_bytes smaller than dq_workspace_size */
    DQ_ERR_OUT_OF_RANGE = 4,   /* qubit count or batch beyond the limits */
    DQ_ERR_HIP = 5,            /* a HIP runtime call failed */
    DQ_ERR_INTERNAL = 6
} dq_status;

typedef enum { DQ_C64 = 0, DQ_C128 = 1 } dq_dtype;

typedef enum {
    DQ_OP_H = 0, DQ_OP_X = 1, DQ_OP_Y = 2, DQ_OP_Z = 3,
    DQ_OP_RX = 4, DQ_OP_RY = 5, DQ_OP_RZ = 6,
    DQ_OP_CNOT = 7, DQ_OP_CZ = 8, DQ_OP_SWAP = 9,
    DQ_OP_CP = 10, DQ_OP_RZZ = 11,
    DQ_OP_UNITARY = 12,         /* dense 2^nq x 2^nq matrix, nq = 1..5 */
    DQ_OP_RXX = 13,             /* exp(-i t X(x)X / 2) and exp(-i t Y(x)Y / 2): the two-qubit */
    DQ_OP_RYY = 14,             /* rotations of the paper's gate set beside RZZ (section 4) */
    DQ_OP_U3 = 15,              /* U3(theta, phi, lambda) = [[cos(theta/2), -e^{i lambda} sin(theta/2)],
                                   [e^{i phi} sin(theta/2), e^{i(phi+lambda)} cos(theta/2)]], the
                                   general one-qubit gate of the paper's QResNet (section 4.3); its
                                   three angles are scale * source[idx + k], k = 0, 1, 2 (scale for
                                   each when the source is DQ_SRC_NONE) */
    DQ_OP_CRX = 16,             /* controlled rotations on (control, target): the identity where */
    DQ_OP_CRY = 17,             /* the control is 0, RX / RY / RZ(t) where it is 1 (the pooling  */
    DQ_OP_CRZ = 18              /* gate of the QCNN and the controlled encoding of the QResNet,
                                   section 4.3) */
} dq_op;

typedef enum { DQ_SRC_NONE = 0, DQ_SRC_PARAM = 1, DQ_SRC_DATA = 2 } dq_src;

/* One gate of a circuit.  wires: (control, target) for CNOT / CZ / CP; for
 * DQ_OP_UNITARY wires[0] is the most significant bit of the matrix index.
 * matrix (UNITARY only): host pointer to 2^nq x 2^nq complex entries,
 * row-major, (re, im) interleaved doubles; copied by dq_plan_create. */
typedef struct {
    int32_t op;
    int32_t nq;
    int32_t wires[DQ_MAX_GATE_QUBITS];
    int32_t src;
    int64_t idx;
    double scale;
    const double *matrix;
} dq_gate;

/* One Pauli string with a real coefficient: P = i^{|x&z|} X^x Z^z, i.e.
 * bit w of xmask / zmask selects X / Z on wire w, both bits select Y. */
typedef struct {
    double coef;
    uint64_t xmask;
    uint64_t zmask;
} dq_pauli_term;

/* Planner options (NULL = defaults). */
typedef struct {
    int32_t fusion;       /* 1 (default): register-tile passes that apply many gates per
                             state sweep; 0: the plain path, one kernel launch per gate */
    int32_t tile_bits;    /* register-resident wires per tile: 0 = auto (5 for complex64,
                             4 for complex128; with jit 6 and 5); 1..6 (complex128: 1..5;
                             6 only with jit, else 5 is used) */
    int32_t fold_init;    /* 1 (default): fold the leading one-qubit gates of every wire into
                             the initial product-state write when applying from |0..0> */
    int32_t dense_fuse;   /* 0 (default): register tiles; 4 or 5: the forward sweep groups gates
                             into dense blocks on k wires (product of the gate matrices, formed
                             on the device in double) applied on the matrix cores (MFMA) */
    int32_t jit;          /* 0 (default): register-tile passes read their operation list at run
                             time; 1: each distinct pass is compiled (hipRTC, at the plan's first
                             use on a device; code objects cached in DQ_JIT_CACHE, default
                             $HOME/.cache/dq_jit) into straight-line code with every operand
                             position a compile-time constant; the planner keeps passes
                             within 2048 operations x amplitudes per lane (a longer pass
                             with up to 32 amplitudes per lane would stay interpreted) */
    int32_t adj_tile_bits; /* register-resident wires per tile of the adjoint sweep, which holds
                             two states: 0 = auto (min(tile bits, 4) for complex64, 3 for
                             complex128; with jit 5 and 4); 1..5 (complex128: 1..4) */
    int32_t low_bits;     /* states of 128 MiB and more: physical bits 3.. that every tile
                             includes, so that each wave reads runs of 2^(3+k) amplitudes:
                             0 = auto (bits 3 and 4), 1 = none, 2 = bit 3, 3 = bits 3 and 4 */
    int32_t layout;       /* 0 (default): for states of 128 MiB and more, try relabelling physical
                             bits 1..4 with wires spread over the register (transpositions,
                             undone by swaps appended to the circuit, so states keep the
                             canonical order) and keep the plan with the fewest sweeps;
                             1: canonical bit order only */
    int32_t arith64;      /* 0 (default): tile passes compute in the state's precision;
                             1 (complex64 plans with jit = 1, fusion = 1, dense_fuse = 0 only;
                             else DQ_ERR_UNSUPPORTED): complex64 states swept with float64
                             arithmetic and float64 gate matrices, each amplitude rounded to
                             complex64 once per pass (about 8x smaller gradient error against
                             complex128 on deep circuits); tiles hold one register bit less
                             (as for complex128), so passes are more numerous; dense UNITARY
                             gates of two or more wires (which run as per-gate sweeps) are not
                             supported in such plans (DQ_ERR_UNSUPPORTED) */
} dq_options;

typedef struct dq_plan_s *dq_plan;
typedef struct dq_obs_s *dq_obs;

/* Plan statistics, for tests and benchmarks. */
typedef struct {
    int32_t nqubits;
    int32_t dtype;
    int64_t ngates;
    int64_t fwd_steps;        /* kernel sweeps of the state in dq_apply_circuit */
    int64_t fwd_tile_passes;  /* of which register-tile passes */
    int64_t fwd_dense_blocks; /* of which matrix-core dense blocks */
    int64_t adj_steps;        /* sweeps of the (state, adjoint) pair in dq_adjoint_grad */
    int64_t folded_gates;     /* gates folded into the initial product state */
    int64_t grad_gates;       /* gate occurrences that carry a gradient */
    int32_t tile_bits;        /* register bits of the forward tiles */
    int32_t adj_tile_bits;    /* register bits of the adjoint tiles */
    int32_t layout_swaps;     /* transpositions of the chosen qubit layout (0: canonical) */
    int32_t pad;
    /* register-tile operations of the forward program (index 0) and the
     * adjoint program (index 1) by kind: 0 dense 2x2, 1 diagonal 2x2, 2 CNOT,
     * 3 CZ, 4 two-qubit diagonal, 5 swap, 6 real 2x2, 7 RX form; [.][0][k]
     * counts operations whose target is a lane bit (cross-lane exchange),
     * [.][1][k] those on register bits */
    int64_t tile_ops[2][2][8];
} dq_plan_stats;

/* Build a plan for an n-qubit circuit (host only; no device work).
 * nparams / ndata: row lengths of params / data that gate idx refer to.
 * Errors: DQ_ERR_INVALID_ARG for a bad gate (unknown op, wrong nq, wire out
 * of range or repeated, idx out of range, NULL matrix), DQ_ERR_OUT_OF_RANGE
 * for nqubits outside 1..DQ_MAX_QUBITS. */
dq_status dq_plan_create(dq_plan *out, int32_t nqubits, const dq_gate *gates, int64_t ngates,
                         int64_t nparams, int64_t ndata, dq_dtype dtype, const dq_options *opt);
void dq_plan_destroy(dq_plan plan);
dq_status dq_plan_get_stats(dq_plan plan, dq_plan_stats *out);
/* Text description of the forward and adjoint programs, one line per step:
 * "<fwd|adj> <index> tile R=.. lbits=.. rbits=.. ops=kind:q0:q1:gen:slot:lslot;..."
 * for register-tile passes (q = tile-local bit: < 6 lane, else register
 * q - 6), "<fwd|adj> <index> sweep kind=.. k=.. bits=.. slot=.. gen=.. gslot=.."
 * for whole-state sweeps.  Writes at most cap bytes including the
 * terminating NUL; *needed (nullable) receives the full size.  Host only. */
dq_status dq_plan_describe(dq_plan plan, char *buf, size_t cap, size_t *needed);
/* Plans created with jit = 1: *count (nullable) receives the number of
 * distinct compiled pass kernels; for 0 <= index < count, the kernel's source
 * (it includes "tile_dev.h") is written as by dq_plan_describe.  index < 0
 * only sets *count.  Host only. */
dq_status dq_plan_jit_source(dq_plan plan, int32_t index, char *buf, size_t cap, size_t *needed, int32_t *count);

/* Observables: nobs Pauli sums over the terms [obs_offsets[o], obs_offsets[o+1]).
 * Host only; masks must not touch wires >= nqubits. */
dq_status dq_obs_create(dq_obs *out, int32_t nqubits, const dq_pauli_term *terms,
                        const int64_t *obs_offsets, int32_t nobs);
void dq_obs_destroy(dq_obs obs);

/* Workspace bytes needed by dq_apply_circuit / dq_expval (grad = 0) or
 * dq_adjoint_grad (grad = 1; grad = 2 with preserve_state = 1) for this
 * batch; per_sample = 1 when params or data differ per sample.  obs may be NULL when grad = 0 and no expval is
 * taken.  The workspace is a caller-owned device buffer, 256-byte aligned. */
dq_status dq_workspace_size(dq_plan plan, dq_obs obs, int64_t batch, int32_t per_sample,
                            int32_t grad, size_t *bytes);

/* state[b] = init (a device array of 2^n amplitudes) for every sample, or
 * |0...0> when init is NULL. */
dq_status dq_state_init(dq_plan plan, void *state, int64_t batch, const void *init, void *stream);

/* Apply the plan's circuit to every sample of `state` in place (paper 4.1).
 * from_zero = 1: the input contents are ignored and the circuit is applied
 * to |0...0>, with the leading one-qubit gates of each wire folded into the
 * first write of the state.  params: [P] (params_bstride = 0) or rows of
 * params_bstride doubles per sample; data likewise.  ws: workspace of at
 * least dq_workspace_size(plan, NULL, batch, per_sample, 0) bytes. */
dq_status dq_apply_circuit(dq_plan plan, void *state, int64_t batch, const double *params,
                           int64_t params_bstride, const double *data, int64_t data_bstride,
                           int32_t from_zero, void *ws, size_t ws_bytes, void *stream);

/* dq_apply_circuit without a workspace and without any allocation, for
 * callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation.  Same arguments
 * and results as dq_apply_circuit; the per-sample gate-matrix blocks go to
 * a library-owned device scratch array of DQ_NOALLOC_SCRATCH_BYTES (16 MiB)
 * per device, held until the process ends.  Preconditions: the plan has
 * been used on the current device by dq_apply_circuit (which uploads its
 * tables and loads its compiled passes; this call uploads, compiles and
 * allocates nothing), and the matrix blocks (dq_workspace_size with grad =
 * 0) fit the scratch.  Errors, with nothing enqueued: DQ_ERR_INVALID_ARG
 * (as dq_apply_circuit, or a plan not yet resident on the device),
 * DQ_ERR_OUT_OF_RANGE (matrix blocks beyond the scratch).  All calls on one
 * device share its scratch: calls that overlap on one device (concurrent
 * streams or threads) race and must be serialised by the caller; calls in
 * one stream are ordered.  No timing events are recorded. */
#define DQ_NOALLOC_SCRATCH_BYTES (16u << 20)
dq_status dq_apply_circuit_noalloc(dq_plan plan, void *state, int64_t batch, const double *params,
                                   int64_t params_bstride, const double *data, int64_t data_bstride, int32_t from_zero,
                                   void *stream);

/* out[b][o] = sum_k coef_k <psi_b| P_k |psi_b> over the terms of observable
 * o (paper 4.2, expectation()).  out: device [batch][nobs] float64.
 * Reductions are deterministic (fixed order, float64 across blocks). */
dq_status dq_expval(dq_plan plan, dq_obs obs, const void *state, int64_t batch, double *out,
                    void *ws, size_t ws_bytes, void *stream);

/* Marginal probabilities of a computational-basis measurement of the wires
 * wires[0..nwires) (paper 4.2: measurement of a circuit with its
 * probabilities; 4.1: the Born rule): out[b][m] = sum of |psi_b[j]|^2 over
 * the basis states j whose measured wires read m, wires[0] being the most
 * significant bit of m.  nwires 1..12 distinct wires below n; batch at most
 * 65535; out: device [batch][2^nwires] float64; ws: caller-owned device
 * buffer of at least dq_probs_workspace_size(plan, batch, nwires) bytes.
 * One read of the state; deterministic (fixed-order float64 sums).  Invalid
 * arguments are rejected on the host before any device work
 * (DQ_ERR_INVALID_ARG, DQ_ERR_WORKSPACE, DQ_ERR_OUT_OF_RANGE). */
dq_status dq_probs_workspace_size(dq_plan plan, int64_t batch, int32_t nwires, size_t *bytes);
dq_status dq_probs(dq_plan plan, const void *state, int64_t batch, const int32_t *wires, int32_t nwires,
                   double *out, void *ws, size_t ws_bytes, void *stream);

/* Measurement shots by inversion of the cumulative distribution (paper
 * 4.2: sampling a circuit's measurement): out[b][s] = the smallest outcome m
 * with u[b][s] < p[b][0] + ... + p[b][m] (summed in this order in float64),
 * or the last outcome of nonzero probability when u[b][s] is not below the
 * total (rounding); 0 when every probability is 0.  p: device
 * [batch][nout] float64 (dq_probs's output, or any distribution), nout
 * 1..2^20; u: device [batch][shots] float64 uniforms in [0, 1) drawn by the
 * caller; out: device [batch][shots] int64.  No workspace; host validation
 * as above. */
dq_status dq_sample(const double *p, int64_t batch, int32_t nout, const double *u, int32_t shots, int64_t *out,
                    void *stream);

/* Adjoint gradient (paper 7.2) of L = sum_{b,o} grad_out[b][o] E[b][o]
 * where E is dq_expval of the final state.  `state` must hold the final
 * states produced by dq_apply_circuit with the same params / data; it is
 * overwritten (un-applied back towards the start state) unless
 * preserve_state = 1, which keeps it at the cost of one more state of
 * workspace.  grad_params: [P] when params_bstride = 0 (summed over the
 * batch) or [batch][P]; grad_data (nullable): [D] when data_bstride = 0 or
 * [batch][D].  Both are overwritten. */
dq_status dq_adjoint_grad(dq_plan plan, dq_obs obs, void *state, int64_t batch,
                          const double *params, int64_t params_bstride, const double *data,
                          int64_t data_bstride, const double *grad_out, double *grad_params,
                          double *grad_data, int32_t preserve_state, void *ws, size_t ws_bytes,
                          void *stream);

/* Hessian (paper 3.1, the second-order gradient benchmark) of
 * L = sum_o weights[o] E_o for one sample with shared parameters:
 * hess[p][q] = d^2 L / dparams[p] dparams[q], row-major [P][P] float64,
 * overwritten.  params: device [P]; data: device [D] (one sample's row;
 * NULL when the circuit reads no data; data angles are held fixed);
 * weights: device [nobs] float64.  Method: every gate angle that reads a
 * parameter ("occurrence", K of them: U3 has three, a controlled rotation
 * two, other rotations one) is shifted by +pi/2 and -pi/2 in a batch of 2K
 * circuits; one batched forward and adjoint sweep gives the gradient with
 * respect to every occurrence angle of each shifted circuit, and
 * H_ab = (g_a(+b) - g_a(-b)) / 2 is exact for the planned gates (the
 * two-term shift rule of generators with eigenvalues a distance 1 apart);
 * H[p][q] sums H_ab times both chain factors (scales) over the
 * occurrences of p and q.  max_shifts: occurrences per batch (0 = all K;
 * fewer bound the workspace at 2 * max_shifts states); batches run in
 * order and the result is deterministic.  ws: caller-owned device buffer of
 * at least dq_hessian_workspace_size bytes.  The first call builds a
 * derived plan (host) that the plan keeps until dq_plan_destroy.
 * Errors: DQ_ERR_INVALID_ARG (NULL pointer, a plan without parameters, a
 * negative max_shifts), DQ_ERR_OUT_OF_RANGE (2 * max_shifts states beyond
 * the batch or memory limit), DQ_ERR_WORKSPACE; nothing is enqueued then. */
dq_status dq_hessian_workspace_size(dq_plan plan, dq_obs obs, int32_t max_shifts, size_t *bytes);
dq_status dq_hessian(dq_plan plan, dq_obs obs, const double *params, const double *data, const double *weights,
                     double *hess, int32_t max_shifts, void *ws, size_t ws_bytes, void *stream);

/* Kernel timing for benchmarks.  While enabled on a plan, every kernel
 * launch made for it (apply, expval, adjoint) is bracketed by a pair of
 * hipEvents recorded on the launch's stream.  dq_profile_read waits for the
 * recorded events and returns, per kernel family, the number of launches,
 * the summed event time and the summed algorithmic bytes (what the launch
 * must read plus write: 2 states for a forward sweep, 4 for an adjoint
 * sweep, half / a quarter of a state for CNOT / CZ, ...).  reset = 1
 * clears the counters.  Events are created on first need and kept by the
 * plan; profiling adds two event records per launch and nothing else. */
enum {
    DQ_PROF_FWD_TILE = 0,   /* register-tile forward pass */
    DQ_PROF_ADJ_TILE = 1,   /* register-tile adjoint pass over (psi, lambda) */
    DQ_PROF_GATE = 2,       /* one-gate sweep of the plain path */
    DQ_PROF_GRAD_GATE = 3,  /* one-gate gradient reduction of the plain adjoint */
    DQ_PROF_EXPVAL = 4,     /* Pauli-sum expectation reduction */
    DQ_PROF_LAMBDA = 5,     /* adjoint seed lambda = sum w H psi */
    DQ_PROF_INIT = 6,       /* state initialisation / product-state write */
    DQ_PROF_OTHER = 7,      /* matrix preparation, final gradient reduction, copies */
    DQ_PROF_DENSE = 8,      /* dense 4- or 5-qubit block on the matrix cores */
    DQ_PROF_KINDS = 9
};
typedef struct {
    int64_t launches[DQ_PROF_KINDS];
    double ms[DQ_PROF_KINDS];
    double bytes[DQ_PROF_KINDS];
    double flops[DQ_PROF_KINDS];   /* algorithmic real floating-point operations: per
                                      amplitude, 14 for a dense 2x2 complex matrix, 6 for a
                                      real, RX-form or diagonal one, 6 for a two-qubit
                                      diagonal, 3 for a gradient term, 0 for permutations */
} dq_profile;
dq_status dq_profile_enable(dq_plan plan, int32_t on);
dq_status dq_profile_read(dq_plan plan, dq_profile *out, int32_t reset);

/* Uneven batches (paper 4.3, batched processing), several circuits of
 * different sizes at once.  A multi-plan binds nplans plans of one dtype and
 * one observable handle per circuit.  Circuit c has one sample: its state is
 * the 2^{n_c} amplitudes at packed offset state_off[c] of one state buffer,
 * its parameters the nparams_c doubles at param_off[c] of one parameter
 * buffer (dq_multi_layout fills both offset arrays; circuits are packed in
 * order, each state 256-byte aligned).  Register-tile passes of equal depth
 * of all circuits run as one kernel launch over every circuit's tiles, so a
 * step needs as many tile launches as the deepest circuit has passes, not
 * their sum; plans whose programs are not pure tile passes of the common
 * tile shape run through the single-plan path inside the same calls.  All
 * per-circuit offsets are fixed at creation, so the launch sequence can be
 * captured in a HIP graph and replayed.  Data-encoded gates are not
 * supported here (ndata must be 0). */
typedef struct dq_multi_s *dq_multi;
dq_status dq_multi_create(dq_multi *out, const dq_plan *plans, const dq_obs *obs, int32_t nplans);
void dq_multi_destroy(dq_multi m);
/* total packed state amplitudes / parameters / expectation outputs, and the
 * per-circuit offsets (arrays of nplans, each nullable) */
dq_status dq_multi_layout(dq_multi m, int64_t *state_amps, int64_t *param_count, int64_t *nout,
                          int64_t *state_off, int64_t *param_off, int64_t *out_off);
dq_status dq_multi_workspace_size(dq_multi m, size_t *bytes);
/* batched[c] (nplans entries, caller-owned) = 1 if circuit c runs inside the
 * shared tile launches, 0 if it takes the single-plan path; *count (nullable)
 * = number of batched circuits.  Host only, no device work. */
dq_status dq_multi_batched(dq_multi m, int32_t *batched, int32_t *count);
/* every circuit from |0...0> (leading one-qubit gates folded) */
dq_status dq_multi_apply(dq_multi m, void *states, const double *params, void *ws, size_t ws_bytes, void *stream);
/* out[out_off[c] + o] = expectation of observable o of circuit c (float64, device) */
dq_status dq_multi_expval(dq_multi m, const void *states, double *out, void *ws, size_t ws_bytes, void *stream);
/* adjoint gradients of sum_c sum_o grad_out[out_off[c] + o] E_c,o; the states
 * are consumed; grad_params packed like params */
dq_status dq_multi_adjoint_grad(dq_multi m, void *states, const double *params, const double *grad_out,
                                double *grad_params, void *ws, size_t ws_bytes, void *stream);

/* Description of the last error on this thread ("" after success). */
const char *dq_last_error(void);
int32_t dq_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DQ_H */
