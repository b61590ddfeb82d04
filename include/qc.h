/*
 * qc.h — C ABI of libqc.so, a dense state-vector simulator for AMD MI355X
 * (gfx950).
 *
 * The operations follow the circuit model of QCLAB (Keip, Camps,
 * Van Beeumen, "QCLAB: A Matlab Toolbox for Quantum Computing", 2025):
 * a register of n qubits holds 2^n complex amplitudes, gates act as
 * I_l (x) U' (x) I_r (section 3.2), measurement probabilities are sums of
 * |amplitude|^2 over the indices of an outcome (section 3.3).
 *
 * Conventions used by every call
 * ------------------------------
 * - Qubit labels are the paper's: qubit 0 is the leftmost Kronecker factor,
 *   i.e. bit n-1 of the amplitude index; qubit q is bit n-1-q (section 3.1,
 *   and the teleportation input kron(v, bell) of section 5.1).
 * - A state is a caller-owned, contiguous device buffer of 2^n amplitudes,
 *   interleaved (re, im): float pairs for QC_C64, double pairs for QC_C128.
 *   The library borrows it for the duration of the enqueued work; it never
 *   allocates, frees or resizes a state.
 * - Gate matrices are HOST arrays of FP64, row-major, interleaved:
 *   u[2*(r*d + c)] and u[2*(r*d + c) + 1] are the real and imaginary parts
 *   of U[r][c], d = 2^k.  The local basis index r takes its most significant
 *   bit from the first listed qubit.  Matrices are consumed (converted and
 *   staged) before the call returns; the caller may reuse them at once.
 *   The library does not check unitarity.
 * - Reduction outputs are DEVICE FP64 buffers owned by the caller; their
 *   values are valid once `stream` reaches the call.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   Every call is asynchronous with respect to the host, except where noted.
 * - Every call returns a status (QC_OK = 0 or a negative QC_ERR_* code).
 *   Arguments are validated on the host before anything is enqueued: a call
 *   that fails validation enqueues nothing and leaves the state untouched.
 *   qc_last_error() gives a human-readable reason (per host thread).
 *   No C++ exception crosses this interface.
 * - The library owns a small per-device workspace (reduction partials) and a
 *   64 MiB staging ring (pinned host memory copied to device memory on the
 *   call's stream) for matrices and op lists, both allocated on first use.
 *   Every call takes its own ring slot, so gate and circuit calls issued
 *   from one host thread may run on different streams at once.  Calls that
 *   use the reduction workspace (qc_probs, qc_expect_pauli, qc_state_diff,
 *   qc_sample, qc_collapse, qc_adjoint_grad) must not run concurrently on
 *   different streams of the same device.  Concurrent calls from several
 *   host threads are not supported.
 * - HIP graph capture.  Gate, circuit, reduction and measurement calls
 *   may be captured into a HIP graph: they enqueue no allocation, memset
 *   or host synchronisation while their stream is capturing.  Call
 *   qc_reserve before the capture (it allocates the workspace and empties
 *   the staging ring).  The ring slots a capture takes (its matrices and op
 *   lists, copied again by every replay) are protected: later calls skip
 *   them, until the next qc_reserve, after which graphs captured earlier
 *   must not be replayed.  A call whose staging would not fit in the rest
 *   of the ring during a capture fails with QC_ERR_UNSUPPORTED and
 *   enqueues nothing.  Kernel timing (qc_timing_enable) records nothing for
 *   launches made while their stream is capturing.
 */
#ifndef QC_H_
#define QC_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- element types -------------------------------------------------- */
#define QC_C64  1   /* complex64: two float32 per amplitude  */
#define QC_C128 2   /* complex128: two float64 per amplitude */

/* ---- status codes --------------------------------------------------- */
#define QC_OK               0
#define QC_ERR_ARG         -1   /* malformed argument (null pointer, size) */
#define QC_ERR_QUBIT       -2   /* qubit label out of range or repeated    */
#define QC_ERR_DTYPE       -3   /* unknown or mismatched element type      */
#define QC_ERR_UNSUPPORTED -4   /* valid request the library does not serve */
#define QC_ERR_HIP         -5   /* HIP runtime error (see qc_last_error)   */
#define QC_ERR_NOMEM       -6   /* workspace allocation failed             */

/* Largest register the library accepts (2^36 amplitudes). */
#define QC_MAX_QUBITS 36
/* Largest gate handled by the fused path (2^5 x 2^5 matrices). */
#define QC_MAX_FUSED 5
/* Most control qubits on one gate. */
#define QC_MAX_CTRLS 16
/* Most selector qubits of a multiplexed block (qc_apply_multiplexed). */
#define QC_MAX_SEL 2

/* A borrowed view of a caller-owned state vector. */
typedef struct {
    void   *amp;    /* device pointer, 2^n interleaved complex amplitudes */
    int32_t n;      /* number of qubits, 1..QC_MAX_QUBITS                 */
    int32_t dtype;  /* QC_C64 or QC_C128                                  */
} qc_state_t;

/* One gate of a circuit handed to qc_apply_circuit / qc_fuse_plan.
 * Register operator: Pc (x) U + (I - Pc) (x) I, with U on `targets`
 * (targets[0] = most significant bit of U's local index) and Pc the
 * projector onto ctrls[j] == ctrl_vals[j] for all j (a value of 0 is an
 * "open" control, as in the MCX gates of section 5.4). */
typedef struct {
    int32_t n_targets;                 /* 1..QC_MAX_FUSED                */
    int32_t n_ctrls;                   /* 0..QC_MAX_CTRLS                */
    int32_t targets[QC_MAX_FUSED];
    int32_t ctrls[QC_MAX_CTRLS];
    int32_t ctrl_vals[QC_MAX_CTRLS];   /* 0 or 1                         */
    const double *matrix;              /* host, 2^n_targets square, FP64 */
} qc_gate_t;

/* Execution strategies for qc_apply_circuit. */
#define QC_EXEC_UNFUSED 0   /* one launch (one state sweep) per gate          */
#define QC_EXEC_FUSED   1   /* fuse into <= fuse_k-qubit blocks (FP64 products),
                               one sweep per block                            */
#define QC_EXEC_TILED   2   /* group gates into runs whose non-diagonal
                               targets fit one LDS tile of 2^12 (complex128)
                               or 2^13 (complex64) amplitudes; one sweep per
                               run, gates applied one by one inside LDS      */

/* Counters filled by qc_apply_circuit (may be NULL). */
typedef struct {
    int64_t gates;          /* gates in the input list                      */
    int64_t launches;       /* kernels enqueued                             */
    int64_t sweeps;         /* full passes over the state                   */
    int64_t fused_blocks;   /* dense blocks applied (QC_EXEC_FUSED)         */
    double  state_bytes;    /* algorithmic HBM bytes of all sweeps          */
} qc_exec_stats_t;

/* Gate kinds of a parametrised program (qc_adjoint_grad). */
#define QC_OP_RX   1    /* exp(-i t X / 2) on q0, t = theta[param]        */
#define QC_OP_RY   2    /* exp(-i t Y / 2) on q0                          */
#define QC_OP_RZ   3    /* exp(-i t Z / 2) on q0                          */
#define QC_OP_H    4    /* Hadamard on q0                                 */
#define QC_OP_X    5
#define QC_OP_Y    6
#define QC_OP_Z    7
#define QC_OP_CZ   8    /* controlled Z on (q0, q1)                       */
#define QC_OP_CNOT 9    /* control q0, target q1                          */

typedef struct {
    int32_t kind;   /* QC_OP_*                                          */
    int32_t q0;     /* first qubit                                      */
    int32_t q1;     /* second qubit (two-qubit kinds), else ignored     */
    int32_t param;  /* index into theta for RX/RY/RZ, else ignored      */
} qc_op_t;

/* ---- diagnostics ---------------------------------------------------- */

/* Static string for a status code. */
const char *qc_status_string(int status);
/* Reason for the last failing call on this host thread ("" if none). */
const char *qc_last_error(void);
/* Library version as major*10000 + minor*100 + patch. */
int qc_version(void);

/* Allocate the device's workspace and staging ring if needed, wait for
 * the device, and empty the ring (releasing the slots of graphs captured
 * earlier).  Host-synchronous; call it before capturing a HIP graph.
 * QC_ERR_UNSUPPORTED when `stream` is itself being captured. */
int qc_reserve(void *stream);

/* ---- state preparation (section 3.1 "Initialization") --------------- */

/* s := |basis_index>, the basis state whose index bits are the qubit
 * values (qubit 0 = most significant).  QC_ERR_ARG if
 * basis_index >= 2^n. */
int qc_state_init(qc_state_t s, uint64_t basis_index, void *stream);

/* dst := src, converting precision when the element types differ (FP64 ->
 * FP32 rounds to nearest).  Both states must have the same n and must not
 * overlap. */
int qc_state_copy(qc_state_t dst, qc_state_t src, void *stream);

/* Error report of a against a reference b (same n, any element types):
 * out_dev[0] = sum |a_i - b_i|^2, out_dev[1] = sum |b_i|^2,
 * out_dev[2] = max_i |a_i - b_i|, all accumulated in FP64.  Deterministic. */
int qc_state_diff(qc_state_t a, qc_state_t b, double *out_dev, void *stream);

/* ---- gate application (section 3.2 "Application of Gates") ---------- */

/* psi := (I_l (x) U (x) I_r) psi for a 2x2 U on qubit q (u: 8 doubles). */
int qc_apply_1q(qc_state_t s, int q, const double *u, void *stream);

/* Two-qubit gate: U (4x4, 32 doubles) on qubits (qa, qb), any two distinct
 * qubits in either order; qa is the most significant bit of U's index. */
int qc_apply_2q(qc_state_t s, int qa, int qb, const double *u, void *stream);

/* Multi-controlled one-qubit gate: U acts on `target` in the subspace where
 * every ctrl[j] equals ctrl_val[j] (0 or 1; 0 = open control), identity
 * elsewhere.  This covers CNOT, CZ, CP and the MCX gates of section 5.4.
 * A diagonal U with U[0][0] == 1 only rescales the target-1 part of the
 * control subspace and touches no other amplitude. */
int qc_apply_controlled(qc_state_t s, int n_ctrl, const int *ctrl, const int *ctrl_val,
                        int target, const double *u, void *stream);

/* Dense k-qubit gate, 1 <= k <= QC_MAX_FUSED: U (2^k x 2^k) on the listed
 * qubits (qubits[0] = most significant bit of U's index).  For QC_C64 with
 * k == 5 and n >= 12 the product runs on the FP32 matrix cores (MFMA); on
 * the vector units otherwise (FP32 for QC_C64, FP64 for QC_C128). */
int qc_apply_fused_k(qc_state_t s, int k, const int *qubits, const double *u, void *stream);

/* Multiplexed k-qubit gate (a k-qubit gate whose matrix depends on the
 * values of n_sel other qubits): psi := sum_v P_v (x) U_v psi, where P_v
 * projects the selector qubits onto the value v (sel_qubits[0] = most
 * significant bit of v) and U_v (2^k x 2^k) acts on `qubits` as in
 * qc_apply_fused_k.  This is the block form of the controlled gates of
 * section 3.2 (Pc (x) U + (I - Pc) (x) I is the case U_v = I for every v
 * but one).  u holds the 2^n_sel matrices one after the other, each
 * 2^k x 2^k row-major interleaved FP64 (matrix v starts at
 * u + v * 2 * 4^k); it is consumed before the call returns.  1 <= k <=
 * QC_MAX_FUSED, 0 <= n_sel <= QC_MAX_SEL, all k + n_sel labels distinct.
 * Same precision and kernels as qc_apply_fused_k (matrix cores need
 * n >= 12 + n_sel). */
int qc_apply_multiplexed(qc_state_t s, int k, const int *qubits, int n_sel,
                         const int *sel_qubits, const double *u, void *stream);

/* Relabel the qubits (the permutation gates of section 5.4 taken
 * together): qubit q of the register becomes qubit perm[q], i.e. the
 * amplitude at basis state x moves to the basis state whose bit for label
 * perm[q] is x's bit for label q.  perm must hold a permutation of 0..n-1
 * (QC_ERR_QUBIT otherwise, QC_ERR_ARG if NULL).  One sweep over the state when the relabelling is
 * its own inverse (any set of disjoint SWAPs), two otherwise; none for the
 * identity.  In place; the state's size and precision are unchanged. */
int qc_permute_qubits(qc_state_t s, const int *perm, void *stream);

/* Apply a gate list in order.  mode QC_EXEC_UNFUSED launches one kernel per
 * gate; QC_EXEC_FUSED first groups the gates into blocks (host FP64 matrix
 * products, see qc_fuse_plan) and applies each block with one
 * qc_apply_multiplexed sweep; QC_EXEC_TILED applies runs of gates in LDS
 * tiles (fuse_k is ignored).  fuse_k must be 1..QC_MAX_FUSED and is capped
 * at n.  A gate is moved ahead of another only when the two commute (no
 * shared qubit, or every shared qubit is one on which both act diagonally:
 * a control, or a target of a diagonal matrix), so the result is the
 * ordered product.  In the fused and tiled modes a SWAP gate (two targets,
 * no controls, exactly the 4 x 4 permutation matrix of section 5.4) moves
 * no data: the later gates are applied with its two qubits exchanged, and
 * the relabelling of all such SWAPs is applied at the end with
 * qc_permute_qubits (counted in stats).  stats may be NULL. */
int qc_apply_circuit(qc_state_t s, int n_gates, const qc_gate_t *gates, int mode,
                     int fuse_k, qc_exec_stats_t *stats, void *stream);

/* Host-only planning step of QC_EXEC_FUSED (no device work): partition the
 * gate list into blocks applied in block order.  A block acts
 * non-diagonally on at most fuse_k qubits (its block qubits) and may touch
 * up to QC_MAX_SEL more qubits on which all its gates act diagonally (its
 * selector qubits, making the block a multiplexed gate); a gate wider than
 * that forms a block of its own.  Moving every gate of a block ahead of the
 * gates of later blocks only swaps commuting gates (see qc_apply_circuit).
 * block_of[g] receives the block index of gate g; *n_blocks the number of
 * blocks.  block_of must hold n_gates entries.  SWAP gates are planned here
 * like any other gate; qc_apply_circuit first takes them out of the list
 * and relabels the gates after them (see there), and plans that list. */
int qc_fuse_plan(int n, int n_gates, const qc_gate_t *gates, int fuse_k,
                 int *block_of, int *n_blocks);

/* The FP64 matrices the fuser builds for one multiplexed block (host only:
 * no device work).  A run of gates on k qubits is one 2^k x 2^k unitary,
 * the product of the gates' register operators in circuit order (section
 * 3.2, the Kronecker extension P_c (x) U + (I - P_c) (x) I of each gate);
 * with n_sel selector qubits the product splits into one such matrix per
 * selector value v (sel_qubits[0] = most significant bit of v).  Every gate
 * target must be one of `qubits`, or a selector qubit if the gate's matrix
 * is diagonal; every control one of the k + n_sel labels (QC_ERR_QUBIT
 * otherwise).  out receives 2^n_sel matrices of 2^k x 2^k, row-major,
 * interleaved FP64 (matrix v at out + v * 2 * 4^k), in the layout
 * qc_apply_multiplexed takes.  Limits as for qc_apply_multiplexed. */
int qc_block_matrices(int n_gates, const qc_gate_t *gates, int k, const int *qubits, int n_sel,
                      const int *sel_qubits, double *out);

/* ---- measurement and reductions (section 3.3 "Measurement") --------- */

/* Marginal outcome distribution over the m listed qubits:
 * out_dev[s] = sum of |psi_i|^2 over the indices i whose listed qubits read
 * s (qubits[0] = most significant bit of s), FP64, 2^m entries.  With
 * m == n this is the full distribution.  m in [1, n]; m <= 24 unless m == n. */
int qc_probs(qc_state_t s, int m, const int *qubits, double *out_dev, void *stream);

/* qc_probs for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, result and kernels, but no allocation of any kind -
 * no workspace, no staging ring, no hipMalloc/hipFree, and no qc_reserve
 * needed.  Its partial sums live in a static device array of
 * QC_PROBS_NOALLOC_SCRATCH doubles (64 KiB) that each GPU holds until the
 * process ends; every call on a GPU shares that GPU's array, so calls that
 * overlap on one GPU (concurrent streams or host threads) race.  The array
 * needs no clearing: each call writes every partial it reads.  A marginal
 * whose partial sums would not fit returns QC_ERR_UNSUPPORTED (none does
 * with the current launch shapes: fewer than 8192 partials, or none when
 * every bin is one block). */
#define QC_PROBS_NOALLOC_SCRATCH 8192
int qc_probs_noalloc(qc_state_t s, int m, const int *qubits, double *out_dev, void *stream);

/* Pauli-string expectation values <psi|P|psi>, the coefficients
 * S_i = <sigma_i> of the tomography example (section 5.2), for tensor
 * products of I, X, Y, Z.  paulis holds n_terms strings of n
 * characters from {I,X,Y,Z} back to back (character q acts on qubit q);
 * coeff holds n_terms FP64 coefficients (host).
 * out_dev[0] = sum_t coeff[t] * Re <psi|P_t|psi>; if per_term != 0,
 * out_dev[1 + t] = Re <psi|P_t|psi> as well.  FP64 accumulation,
 * deterministic order.  The state is not renormalised. */
int qc_expect_pauli(qc_state_t s, int n_terms, const char *paulis, const double *coeff,
                    int per_term, double *out_dev, void *stream);

/* Collapse onto outcome `outcome` (0 or 1) of qubit q and renormalise
 * (section 3.3): with P = sum over indices whose qubit q reads `outcome`
 * of |psi_i|^2 (FP64), those amplitudes are divided by sqrt(P) and every
 * other amplitude is set to 0.  prob_dev[0] receives P (device FP64; may be
 * NULL).  If P == 0 the state is left unchanged (an impossible outcome). */
int qc_collapse(qc_state_t s, int q, int outcome, double *prob_dev, void *stream);

/* One branch of a qubit reset (the "qubit resets" of section 3.3): qubit q
 * is measured and set back to |0>.  With P = sum over indices whose qubit q
 * reads `outcome` of |psi_i|^2 (FP64), the amplitude pair (psi_i0, psi_i1),
 * i1 = i0 with qubit q set, becomes (psi_i_outcome / sqrt(P), 0): the
 * outcome's collapse of qc_collapse followed, for outcome 1, by X on q.
 * prob_dev[0] receives P (device FP64; may be NULL).  If P == 0 the state
 * is left unchanged (an impossible outcome).  A full reset splits a state
 * into the branches of both outcomes, as a measurement does. */
int qc_reset(qc_state_t s, int q, int outcome, double *prob_dev, void *stream);

/* State of the unlisted qubits when the m listed qubits hold `values`
 * (0/1 each), the reducedStatevector of section 5.1: dst (n - m qubits, the
 * same element type, remaining qubits in their original order) receives
 * the amplitudes of src whose listed qubits read `values`, without
 * renormalisation.  1 <= m < n. */
int qc_reduced_state(qc_state_t src, int m, const int *qubits, const int *values, qc_state_t dst,
                     void *stream);

/* Shot sampling from the measurement distribution of all qubits (the
 * counts of section 5.2).  u_dev holds `shots` caller-supplied uniforms in
 * [0, 1) (device FP64); out_dev[k] (device int64) receives the first basis
 * index whose cumulative weight, in index order, exceeds u_dev[k] times
 * the total weight.  The cumulative weights are FP64 (per chunk of up to
 * 4096 amplitudes for n <= 33, larger chunks above). */
int qc_sample(qc_state_t s, int shots, const double *u_dev, int64_t *out_dev, void *stream);

/* Shot counts over the m listed qubits (the counts of section 5.2): each
 * of the `shots` uniforms u_dev[k] in [0, 1) (device FP64) draws one basis
 * index as qc_sample does, and counts_dev[s] (device int64, 2^m entries,
 * overwritten) receives the number of shots whose listed qubits read s
 * (qubits[0] = most significant bit of s).  1 <= m <= min(n,
 * QC_MAX_COUNT_QUBITS); 0 <= shots <= QC_MAX_COUNT_SHOTS. */
#define QC_MAX_COUNT_QUBITS 24
#define QC_MAX_COUNT_SHOTS (1 << 21)
int qc_counts(qc_state_t s, int m, const int *qubits, int shots, const double *u_dev,
              int64_t *counts_dev, void *stream);

/* ---- differentiation ------------------------------------------------ */

/* Adjoint-method gradient of E(theta) = <phi|H|phi>, phi = U_L..U_1 psi_in,
 * H = sum_t coeff[t] P_t (Pauli strings as in qc_expect_pauli).
 * psi holds psi_in on entry; lam is a caller-owned state of the same n and
 * type used as the adjoint vector.  On return psi holds psi_in again up to
 * rounding (the backward pass un-computes the forward pass).
 * energy_dev[0] = E; grad_dev[p] = dE/dtheta[p] (FP64, n_params entries;
 * a parameter used by several gates gets the sum).  theta is a host FP64
 * array.  Method: Jones & Gacon, arXiv:2009.02823 (the paper has none). */
int qc_adjoint_grad(qc_state_t psi, qc_state_t lam, const qc_op_t *ops, int n_ops,
                    const double *theta, int n_params, int n_terms, const char *paulis,
                    const double *coeff, double *energy_dev, double *grad_dev, void *stream);

/* ---- batched persistent launch --------------------------------------- */

/* One circuit of a batch: it starts from |0...0>, applies its gates (one or
 * two targets each, any controls) and ends with the energy
 * <H> = sum_t coeff[t] <psi|P_t|psi> (Pauli strings as in qc_expect_pauli).
 * All host arrays are read during qc_batch_create only. */
typedef struct {
    int32_t n;                 /* qubits, 1..30                                */
    int32_t n_gates;
    const qc_gate_t *gates;    /* n_targets 1 or 2                             */
    int32_t n_terms;
    const char *paulis;        /* n_terms * n characters                       */
    const double *coeff;       /* n_terms                                      */
} qc_circuit_t;

typedef struct qc_batch qc_batch_t;   /* opaque, owns a device-resident program */

/* Plan a batch and upload its device program (host-synchronous; allocates
 * device memory).  Circuits whose state fits one LDS tile (n <= 13 for
 * QC_C64, n <= 12 for QC_C128) run entirely inside one workgroup; larger
 * ones run on a group of 8 co-resident workgroups over a state kept in the
 * arena.  keep_states != 0 also writes every final state to the arena. */
int qc_batch_create(int n_circuits, const qc_circuit_t *circuits, int dtype, int keep_states,
                    qc_batch_t **out);
/* Bytes of caller-owned device memory qc_run_batch needs as its arena, the
 * persistent grid size and the number of phases in the program. */
int qc_batch_info(const qc_batch_t *b, uint64_t *arena_bytes, int *grid, int *phases);
/* Run every circuit of the batch in ONE persistent kernel launch (plus a
 * tiny kernel that clears the barrier counters).  energy_dev receives one
 * FP64 energy per circuit.  No allocation, no host synchronisation and no
 * memset: the call may be captured in a HIP graph.  Concurrent runs of the
 * same batch object race on its barrier counters. */
int qc_run_batch(qc_batch_t *b, void *arena_dev, double *energy_dev, void *stream);
/* View of circuit i's final state inside the arena (keep_states, or
 * circuits too large for one tile). */
int qc_batch_state(const qc_batch_t *b, void *arena_dev, int i, qc_state_t *view);
/* Device error flags of the last run (host-synchronous): bit 0 is set when
 * a group barrier timed out (the energies of that run are then invalid). */
int qc_batch_status(qc_batch_t *b, int *flags);
int qc_batch_destroy(qc_batch_t *b);

/* ---- autotuning ----------------------------------------------------- */

/* Launch-shape knobs (process-wide; the defaults suit MI355X). */
#define QC_KNOB_MFMA_WG_PER_CU 1   /* fused MFMA kernel: 32 KiB tile slots per CU (1..5; a 64 KiB workgroup takes two) */
#define QC_KNOB_TILE_WG_PER_CU 2   /* workgroups per CU, LDS tile-run kernel (1..16)        */
#define QC_KNOB_FUSE_LOOKAHEAD 3   /* fuser: candidates scored with a one-step lookahead
                                      (0..256; 0 or 1 = plain greedy; default 16)          */
#define QC_KNOB_MFMA_TILE_BITS 4   /* fused MFMA kernel tile: 13 = 32 x 256 amplitudes (2 KiB
                                      contiguous runs, used when n >= 13 + outer selector
                                      qubits), 12 = 32 x 128 (1 KiB runs); default 13      */
#define QC_KNOB_TILE_BITS 5        /* QC_EXEC_TILED tile size cap, 2^value amplitudes (6..13;
                                      complex128 tiles stop at 12; default 13)             */
#define QC_KNOB_TILE_ENGINE 6      /* QC_EXEC_TILED engine: 1 = register-resident tiles
                                      (amplitudes in registers, LDS only to exchange index
                                      bits; default), 0 = LDS-resident tiles               */
#define QC_KNOB_WIDE_MIN_TILES 7   /* complex128 register tiles of 2^13 amplitudes (16 per
                                      thread, one workgroup per CU) when the register holds
                                      at least 2^value such tiles, else 2^12 (8..30;
                                      default 12)                                          */
int qc_set_knob(int knob, int value);
int qc_get_knob(int knob, int *value);

typedef struct {
    int32_t mode;            /* QC_EXEC_*                          */
    int32_t fuse_k;          /* block width for QC_EXEC_FUSED      */
    int32_t mfma_wg_per_cu;  /* knob value used                    */
    int32_t sweeps;          /* state sweeps of the strategy       */
    float   ms;              /* median time of one run             */
    int32_t mfma_tile_bits;  /* QC_KNOB_MFMA_TILE_BITS value used  */
    int32_t tile_bits;       /* QC_KNOB_TILE_BITS value used       */
} qc_tune_entry_t;

/* Time every execution strategy for this gate list on `scratch` (its
 * contents are overwritten: each run starts from |0...0>), `reps` timed
 * runs after one warm-up each, and report them fastest first.  Strategies:
 * unfused, LDS tile runs at three tile sizes (QC_KNOB_TILE_BITS), fused
 * k = 2..5, and for complex64 k = 5 every matrix-core tile shape
 * (QC_KNOB_MFMA_TILE_BITS) with its workgroup counts
 * (QC_KNOB_MFMA_WG_PER_CU).  Writes at most max_entries entries,
 * their count to *n_entries; the knobs are left at the fastest entry's
 * values.  Host-synchronous. */
int qc_autotune(qc_state_t scratch, int n_gates, const qc_gate_t *gates, int reps,
                qc_tune_entry_t *entries, int max_entries, int *n_entries, void *stream);

/* ---- kernel timing (for roofline reports) ---------------------------- */

/* Start (on != 0) or stop recording HIP events around every kernel the
 * library launches.  Starting clears earlier records. */
int qc_timing_enable(int on);
/* Synchronise on the recorded events and report, for the kernel family
 * `name` (for example "fused_mfma_c64"), the number of launches and their
 * total duration in milliseconds.  Blocks the host. */
int qc_timing_query(const char *name, int64_t *count, double *total_ms);

#ifdef __cplusplus
}
#endif
#endif /* QC_H_ */
