/*
 * qsv.h -- C ABI of the gfx950 state-vector library (libqsv.so).
 *
 * The calls follow the paper's statement of the problem (section III, the
 * hardware-abstraction layer of a quantum virtual machine; section IV.A, the
 * XACC accelerator / buffer / instruction model; section V.B, its program
 * listing): a host program allocates a qubit buffer, executes gate
 * instructions (name, qubits, parameters) in program order, and reads back
 * expectation values of Hamiltonian terms or measurement samples.  Here the
 * buffer is an exact 2^n-amplitude state vector resident in GPU memory
 * (the "brute-force" representation of section I) and the instructions are
 * applied in place by hand-written HIP kernels.
 *
 * Conventions that hold for every call:
 *   - Amplitudes are stored contiguously as interleaved (re, im) pairs:
 *     complex64 (8 bytes) or complex128 (16 bytes) -- the memory layout of
 *     torch.complex64 / torch.complex128.  Qubit q is bit q of the index.
 *   - For a k-qubit operation on qubits (q[0], ..., q[k-1]) the local matrix
 *     index is m = sum_j bit(q[j]) * 2^j, i.e. the FIRST listed qubit is the
 *     least-significant bit.  CNOT and CPHASE list (control, target).
 *   - Rotations are R_P(theta) = exp(-i theta P / 2).
 *   - Matrices are passed in complex128 (row-major, interleaved re, im) and
 *     rounded once to the state's precision inside the library.
 *   - Reductions (norm, expectation values, sampling prefix sums) accumulate
 *     in FP64 in a fixed order, so repeated calls give identical results.
 *   - No state is ever renormalised.
 *   - Every function returns a qsv_status; none throws, aborts or exits.
 *     On failure the thread-local message from qsv_last_error() says why.
 *
 * Threading and streams: all work on one state is issued to the HIP stream
 * given at allocation.  Different states may be used concurrently from
 * different threads.  Concurrent calls on the same state are a caller error
 * (detected best-effort, QSV_ERR_STATE).  Calls that return host results
 * (norm, expval, sample, copies) synchronise that stream before returning;
 * calls that only apply gates are stream-ordered and return immediately.
 */
#ifndef LIBQSV_ABI_H_
#define LIBQSV_ABI_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QSV_OK = 0,
  QSV_ERR_ARG = -1,          /* invalid argument (range, duplicate qubit, NaN, size) */
  QSV_ERR_OOM = -2,          /* device allocation failed */
  QSV_ERR_HIP = -3,          /* HIP runtime error (text in qsv_last_error) */
  QSV_ERR_UNSUPPORTED = -4,  /* valid request the library does not implement */
  QSV_ERR_STATE = -5         /* bad or freed handle, or concurrent use of one state */
} qsv_status;

typedef enum { QSV_C64 = 1, QSV_C128 = 2 } qsv_dtype;

/* Gate identifiers.  Matrices (FP64, then rounded):
 *   I, X, Y, Z (Pauli), H = [[1,1],[1,-1]]/sqrt2, S = diag(1,i), SDG = S^dag,
 *   T = diag(1,e^{i pi/4}), TDG = T^dag,
 *   RX/RY/RZ(theta) = exp(-i theta P/2) (params[0] = theta),
 *   CNOT(control, target), CZ = diag(1,1,1,-1),
 *   CPHASE(control, target; params[0] = phi) = diag(1,1,1,e^{i phi}),
 *   SWAP, and QSV_MAT: an explicit 2^k x 2^k matrix (qsv_op.mat). */
typedef enum {
  QSV_I = 0, QSV_X = 1, QSV_Y = 2, QSV_Z = 3, QSV_H = 4, QSV_S = 5, QSV_SDG = 6,
  QSV_T = 7, QSV_TDG = 8, QSV_RX = 9, QSV_RY = 10, QSV_RZ = 11, QSV_CNOT = 12,
  QSV_CZ = 13, QSV_CPHASE = 14, QSV_SWAP = 15, QSV_MAT = 16
} qsv_gate;

/* Largest registers accepted by qsv_alloc_state: 2^35 complex64 or 2^34
 * complex128 amplitudes (256 GiB, what one GPU's HBM holds); every launch
 * stays within the dispatch limits up to these sizes. */
#define QSV_MAX_QUBITS 35
#define QSV_MAX_QUBITS_C128 34
#define QSV_MAX_K 6         /* widest explicit matrix (2^6 x 2^6) */

/* Opaque handle of one device-resident state vector. */
typedef struct qsv_state qsv_state;

/* One instruction of a gate list (paper section IV.A: an instruction is a
 * name plus the qubits it acts on; section V.B: with angle parameters).
 * 64 bytes, no padding. */
typedef struct qsv_op {
  int32_t gate;        /* qsv_gate */
  int32_t nq;          /* number of qubits: 1 or 2 for named gates, 1..QSV_MAX_K for QSV_MAT */
  int32_t q[6];        /* qubits; q[0] is the least-significant bit of the local index */
  double p[3];         /* angles: RX/RY/RZ/CPHASE read p[0] */
  const double* mat;   /* QSV_MAT only: 2^nq x 2^nq complex128, row-major, re/im interleaved */
} qsv_op;

/* Execution strategy of qsv_apply_circuit.
 *   mode 0 = automatic (fused tile passes; the per-gate form when the
 *   environment has QSV_FORCE_PERGATE=1, read at first use), 1 = one
 *   kernel per gate ("plain per-gate form"), 2 = fused tile passes, 3 =
 *   fused tile passes with the tile shape (tile qubits, and the contiguous
 *   segment qubits every tile keeps) chosen by an autotuner: the first call
 *   of a gate structure times the candidate plans' passes on a copy of the
 *   state (allocating a second state-sized buffer) and keeps the fastest,
 *   per structure in the process and in the QSV_AUTOTUNE_CACHE file if the
 *   environment names one (see qsv_batch_create); tile_qubits > 0 skips the
 *   tuning.
 *   tile_qubits: qubits per LDS tile in fused mode (0 = library choice).
 *   state_is_output (qsv_adjoint only, 0 or 1): 1 = the state already holds
 *   the circuit's output (an earlier qsv_apply_circuit of the same ops), so
 *   qsv_adjoint starts from it instead of applying the ops first; other
 *   calls require 0.
 *   graph (qsv_apply_circuit in a fused mode only, 0 or 1): 1 = launch the
 *   plan's tile passes as one hipGraph.  The state keeps one graph, captured
 *   on the state's stream (which must not be the null stream) the first time
 *   and again whenever the plan's structure, tile width or the state's
 *   program buffer changes; other calls upload this call's program words
 *   (the angles) and replay it.  Plans with steps that run as their own
 *   kernels (matrices on more than two qubits, registers narrower than one
 *   register group) are launched without a graph.  Calls with graph = 1 on
 *   one state must not overlap a capture of its stream by the caller.
 *   race_check (qsv_apply_circuit in a fused mode without graph, 0 or 1): 1
 *   = debug mode that checks every tile and permutation pass for races:
 *   the pass runs first out of place, from the state into a second
 *   state-sized buffer filled with a poison pattern, then in place as
 *   usual; an amplitude the out-of-place run left unwritten or that differs
 *   bitwise from the in-place result fails the call with QSV_ERR_STATE
 *   (the state then holds the plan's result up to that pass).  Synchronous
 *   per pass; allocates the second buffer.
 *   Other fields are reserved and must be zero. */
typedef struct qsv_plan_opts {
  int32_t mode;
  int32_t tile_qubits;
  int32_t state_is_output;
  int32_t graph;
  int32_t race_check;
  int32_t reserved[3];
} qsv_plan_opts;

/* Allocate a state of n_qubits (1..QSV_MAX_QUBITS) initialised to |0...0>.
 * ext_dev_ptr == NULL: the library allocates (hipMalloc) and owns the memory.
 * ext_dev_ptr != NULL: the state borrows caller memory of ext_bytes bytes
 *   (>= 2^n * bytes-per-amplitude, 256-byte aligned, e.g. a torch tensor's
 *   storage); the caller keeps it alive until qsv_free_state.
 * stream: hipStream_t for all work on this state (NULL = default stream).
 * Paper section III: host-managed buffer of the virtual machine.
 * Errors: QSV_ERR_ARG (n, dtype, size/alignment), QSV_ERR_OOM, QSV_ERR_HIP. */
qsv_status qsv_alloc_state(int n_qubits, qsv_dtype dtype, void* ext_dev_ptr, size_t ext_bytes,
                           void* stream, qsv_state** out);

/* Release the handle (and the memory, if the library owns it).  Waits for
 * the state's pending work.  NULL is accepted and ignored.  Paper section
 * III: the host manages the buffers of the virtual machine.
 * Errors: QSV_ERR_STATE (freed or foreign handle), QSV_ERR_HIP. */
qsv_status qsv_free_state(qsv_state* s);

/* Query n, dtype and the device pointer of the amplitudes (any output may
 * be NULL).  Plumbing: no passage of the paper.  Errors: QSV_ERR_STATE. */
qsv_status qsv_state_info(const qsv_state* s, int* n_qubits, int* dtype, void** dev_ptr);

/* Reset to the computational basis state |x> (x < 2^n), stream-ordered.
 * Paper section V.B: a buffer is created in |0...0> before the program runs
 * (createBuffer); a basis state other than 0 is the QFT workload's input.
 * Errors: QSV_ERR_ARG (x >= 2^n), QSV_ERR_STATE, QSV_ERR_HIP. */
qsv_status qsv_set_basis(qsv_state* s, uint64_t x);

/* Apply one named gate in place (paper section IV.A: one instruction visit).
 * qubits: nq distinct qubits in [0, n); params: np angles (np must equal the
 * gate's parameter count).  QSV_MAT is not accepted here (use
 * qsv_apply_fused).  One HBM pass (or less for diagonal / permutation gates).
 * Errors: QSV_ERR_ARG. */
qsv_status qsv_apply_gate(qsv_state* s, int gate, const int32_t* qubits, int nq,
                          const double* params, int np);

/* Apply an explicit 2^k x 2^k matrix (a fused super-gate, paper section II:
 * gates grouped into aggregates acting as a whole) to k distinct qubits,
 * 1 <= k <= QSV_MAX_K.  mat: complex128 row-major interleaved, read during
 * the call only.  k >= 4 runs on the matrix cores.  Errors: QSV_ERR_ARG. */
qsv_status qsv_apply_fused(qsv_state* s, const int32_t* qubits, int k, const double* mat);

/* Execute a whole gate list in program order (paper section IV.A: the
 * accelerator's execute() on an IR function).  opts may be NULL (automatic).
 * The fused mode groups gates into LDS tile passes (paper section II: SWAP
 * augmentation and super-gate aggregation, done on the index space); the
 * mathematical result equals per-gate application up to rounding.
 * Errors: QSV_ERR_ARG for any invalid op (nothing is applied then). */
qsv_status qsv_apply_circuit(qsv_state* s, const qsv_op* ops, int n_ops,
                             const qsv_plan_opts* opts);

/* Diagnostics of the fused planner (host only; the device is not touched):
 * the number of HBM tile passes and of ops executed by separate kernels that
 * qsv_apply_circuit in fused mode would use for this gate list on a register
 * of n_qubits of the given dtype (tile_qubits 0 = library choice).
 * Errors: QSV_ERR_ARG (invalid ops, n or tile size). */
qsv_status qsv_plan_info(int n_qubits, qsv_dtype dtype, const qsv_op* ops, int n_ops,
                         int tile_qubits, int* passes, int* separate_ops);

/* Expectation value of sum_t coeff[t] * P_t (paper section V.B: one
 * expectation value per Hamiltonian term).  Each Pauli string P_t is given
 * by bit masks: qubit q carries X if only xmask bit q is set, Z if only zmask
 * bit q is set, Y if both.  out_total (host, may be NULL) receives the sum;
 * out_terms (host, may be NULL, n_terms doubles) receives coeff[t] * <P_t>.
 * Accumulation in FP64.  Errors: QSV_ERR_ARG (masks beyond n, NaN coeff). */
qsv_status qsv_expval(qsv_state* s, const uint64_t* xmask, const uint64_t* zmask,
                      const double* coeff, int n_terms, double* out_total, double* out_terms);

/* qsv_expval without any device allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  amps_dev: the caller's device
 * array of 2^n_qubits amplitudes (interleaved re/im of dtype, 16-byte
 * aligned, on the current device); it is read only.  Terms and outputs as
 * for qsv_expval (host arrays; the call synchronises hip_stream, NULL = the
 * null stream).  The reduction partials live in a fixed scratch array of
 * QSV_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends; at most QSV_NOALLOC_MAX_TERMS terms per call.
 * Calls that overlap on one GPU share that array and race: the caller
 * serialises them.  Errors: QSV_ERR_ARG (NULL or misaligned amps_dev, n,
 * dtype, masks beyond n, NaN coefficients, too many terms), QSV_ERR_HIP. */
#define QSV_NOALLOC_SCRATCH_BYTES (512u * 1024u)
#define QSV_NOALLOC_MAX_TERMS 32768
qsv_status qsv_expval_noalloc(const void* amps_dev, int n_qubits, qsv_dtype dtype,
                              const uint64_t* xmask, const uint64_t* zmask, const double* coeff,
                              int n_terms, void* hip_stream, double* out_total, double* out_terms);

/* Gradient of E(theta) = <psi_L| H |psi_L>, psi_L = U_L ... U_1 psi_0, with
 * respect to the angle of every RX / RY / RZ op (R_P(theta) = exp(-i theta P/2)),
 * by one adjoint (reverse) sweep: dE/dtheta_k = Im <lambda_k| P |psi_k> with
 * lambda_k = U_{k+1}^dag ... U_L^dag H psi_L.  psi_0 is the state's current
 * content (or, with opts->state_is_output = 1, the content is psi_L and psi_0
 * is what the sweep recomputes); the ops are applied as by
 * qsv_apply_circuit(opts), E is computed
 * as by qsv_expval, then a second state-sized device buffer (allocated on
 * first use, kept with the state) holds lambda while every op is undone in
 * reverse on both vectors, each rotation's gradient and both inverse updates
 * sharing one kernel.  energy (host, may be NULL) receives E; grad (host,
 * n_ops doubles) receives dE/dtheta per op, 0 for ops that are not rotations.
 * On return the state holds psi_0 again (recomputed by the sweep, up to
 * rounding).  Gradients accumulate in FP64.  (A parameter-gradient of the
 * paper's section V.B variational use case; not a computation of the paper.)
 * Errors: QSV_ERR_ARG (ops, masks, coefficients), QSV_ERR_OOM. */
qsv_status qsv_adjoint(qsv_state* s, const qsv_op* ops, int n_ops, const uint64_t* xmask,
                       const uint64_t* zmask, const double* coeff, int n_terms,
                       const qsv_plan_opts* opts, double* energy, double* grad);

/* sum_i |psi_i|^2 in FP64 (host result; synchronises the state's stream).
 * Paper section V.B: MEASURE reads the probabilities |psi_i|^2, whose sum is
 * 1 for a normalised state; the path never renormalises, so this reports
 * the drift.  Errors: QSV_ERR_ARG (out NULL), QSV_ERR_STATE, QSV_ERR_HIP. */
qsv_status qsv_norm(qsv_state* s, double* out);

/* Measurement samples of the full register without collapse (paper section
 * V.B, MEASURE).  For each caller-supplied uniform u in [0, 1) returns the
 * smallest index i with C_i > u * C_{N-1}, C the FP64 inclusive prefix sum of
 * |psi_i|^2 (bit q of the index = outcome of qubit q).  uniforms and out are
 * host arrays of n_shots entries.  Errors: QSV_ERR_ARG (u outside [0,1),
 * n_shots < 0). */
qsv_status qsv_sample(qsv_state* s, const double* uniforms, int n_shots, uint64_t* out);

/* ---------------------------------------------------------------- batches
 * Many independent circuits (each from |0...0>, uneven widths) evaluated in
 * one persistent kernel launch that a HIP graph replays.  Circuit i has
 * widths[i] qubits (1..30), ops[op_offsets[i] .. op_offsets[i+1]) (gates on
 * at most 2 qubits) and the diagonal Hamiltonian sum_t coeff[t] Z(zmask[t])
 * over terms [term_offsets[i], term_offsets[i+1]) (Z-strings only).  Each
 * workgroup pulls the next circuit (largest first) from a device counter and
 * runs it alone: circuits that fit one LDS tile never touch HBM, wider ones
 * stream tile passes through a scratch region owned by the batch.  Energies
 * accumulate in FP64.  tile_qubits 0 lets the autotuner time the candidate
 * tile widths on this batch and keep the fastest (cached per structure in
 * the process; with QSV_AUTOTUNE_CACHE naming a file in the environment, the
 * cache is read from that file at the first tuning and new results are
 * appended to it, one line "<structure hash, hex> <tile qubits>" each).
 * The parameter-sweep loop of the paper's VQE listing (section V.B) is the
 * use case.  Creation allocates all device memory; runs allocate nothing.
 * Errors: QSV_ERR_ARG, QSV_ERR_UNSUPPORTED (wider gates), QSV_ERR_OOM. */
typedef struct qsv_batch qsv_batch;
qsv_status qsv_batch_create(qsv_dtype dtype, int n_circuits, const int32_t* widths,
                            const int32_t* op_offsets, const qsv_op* ops,
                            const int32_t* term_offsets, const uint64_t* zmask, const double* coeff,
                            int tile_qubits, qsv_batch** out);
/* New parameter values (angles, matrices) for the same gate structure
 * (the same gates on the same qubits; an angle of 0 is a structure like any
 * other angle).  ops: host array of all circuits' ops, read during the call.
 * Paper section V.B: the optimiser's next point of the parameter sweep.
 * When the new programs outgrow the device program buffer or need the full
 * tile body, the buffer grows and the launch is captured again (the only
 * case in which an update allocates).
 * Errors: QSV_ERR_ARG (a different structure), QSV_ERR_STATE (freed handle),
 * QSV_ERR_OOM / QSV_ERR_HIP (the buffer could not grow: the batch then
 * refuses runs). */
qsv_status qsv_batch_update(qsv_batch* b, const qsv_op* ops);
/* Launch the captured graph; energies (host, n_circuits doubles, may be
 * NULL) on return.  Paper section V.B: one energy per point of the sweep.
 * Errors: QSV_ERR_STATE, QSV_ERR_HIP. */
qsv_status qsv_batch_run(qsv_batch* b, double* energies);
/* Chosen tile width, total tile passes over all circuits, scratch bytes
 * (outputs may be NULL).  Plumbing: no passage.  Errors: QSV_ERR_STATE. */
qsv_status qsv_batch_info(const qsv_batch* b, int* tile_qubits, int* total_passes,
                          int64_t* scratch_bytes);
/* Release a batch and its device memory; NULL is accepted.  Plumbing.
 * Errors: QSV_ERR_STATE (freed or foreign handle). */
qsv_status qsv_batch_free(qsv_batch* b);

/* ---------------------------------------------------------------------
 * Matrix-product-state path (paper section III, gate application on an MPS
 * by contraction and SVD; section IV.B, the MPS visitor with its cutoff on
 * singular values).  The register is n site tensors B_l (chi_l x 2 x chi_l+1,
 * complex128, right-canonical) and n+1 bond vectors of Schmidt coefficients
 * on the device; qubit q lives at site q.  A two-qubit gate on adjacent sites
 * contracts the two site tensors, applies the 4x4 gate, scales the rows by the
 * left bond's coefficients and splits the (2 chi_l) x (2 chi_l+2) block by a
 * one-sided Jacobi SVD (in LDS while the three bonds of the update are at
 * most 32, else in a per-update device workspace of about 0.8 MB that the
 * library allocates for MPSs with chi_max above 32); singular values not above `cutoff`, or not above
 * 1e-12 of the largest, are dropped, and at most chi_max are kept (at least
 * one); the state is not renormalised.  Gates on distant qubits are routed by
 * SWAP updates that bring the higher qubit next to the lower one and back.
 * One-qubit gates are folded into the next two-qubit update of their qubit.
 * Updates on disjoint sites run in one launch (one workgroup each).
 * ------------------------------------------------------------------- */
#define QSV_MPS_MAX_CHI 64      /* largest bond dimension (slot stride of the site tensors) */
#define QSV_MPS_MAX_QUBITS 1024

typedef struct qsv_mps qsv_mps;

/* |0...0> on n_qubits (1..QSV_MPS_MAX_QUBITS); chi_max in 1..QSV_MPS_MAX_CHI;
 * cutoff >= 0 (the paper's default is 1e-4).  hip_stream NULL = the null
 * stream.  The library owns all device memory: n_qubits slots of
 * 2 * QSV_MPS_MAX_CHI^2 complex128 entries (128 KiB each), whatever chi_max.  Errors: QSV_ERR_ARG,
 * QSV_ERR_OOM. */
qsv_status qsv_mps_alloc(int n_qubits, int chi_max, double cutoff, void* hip_stream,
                         qsv_mps** out);
/* Release an MPS (waits for its stream); NULL is accepted and ignored.
 * Errors: QSV_ERR_STATE (freed or foreign handle). */
qsv_status qsv_mps_free(qsv_mps* m);

/* Apply one- and two-qubit instructions in program order (qsv_op as for
 * states; QSV_MAT with nq <= 2).  Stream-ordered; host arrays are read during
 * the call.  Errors: QSV_ERR_ARG (qubits, parameters), QSV_ERR_UNSUPPORTED
 * (instructions on three or more qubits). */
qsv_status qsv_mps_apply_circuit(qsv_mps* m, const qsv_op* ops, int n_ops);

/* Amplitudes <x|psi> for host indices idx[0..count) (bit q = qubit q), written
 * as complex128 pairs to the host array out (2 * count doubles).  Synchronous.
 * Errors: QSV_ERR_ARG (index >= 2^n), QSV_ERR_UNSUPPORTED (n > 63). */
qsv_status qsv_mps_amplitudes(qsv_mps* m, const uint64_t* idx, int64_t count, double* out);

/* Bond dimensions (host, n+1 ints; dims[0] = dims[n] = 1) and, if schmidt is
 * not NULL, the Schmidt coefficients (host, (n+1) rows of QSV_MPS_MAX_CHI
 * doubles; row b holds dims[b] values in descending order, zeros after).
 * Synchronous. */
qsv_status qsv_mps_bonds(qsv_mps* m, int32_t* dims, double* schmidt);

/* Two-site updates and kernel launches issued since allocation. */
qsv_status qsv_mps_info(const qsv_mps* m, int64_t* bond_updates, int64_t* launches);

/* Copy the raw amplitudes to / from host memory (bytes must equal the state
 * size; interleaved re/im of the state's dtype).  Synchronous.  Paper
 * section III: hybrid programs transfer memory buffers between the host and
 * the accelerator.  Errors: QSV_ERR_ARG (size, NULL), QSV_ERR_STATE,
 * QSV_ERR_HIP. */
qsv_status qsv_copy_to_host(qsv_state* s, void* dst, size_t bytes);
qsv_status qsv_copy_from_host(qsv_state* s, const void* src, size_t bytes);

/* Wait for all work issued on the state's stream.  Paper section IV.A:
 * XACC follows the co-processor model of OpenCL / CUDA, where the host waits
 * for the work it offloaded.  Errors: QSV_ERR_STATE, QSV_ERR_HIP. */
qsv_status qsv_synchronize(qsv_state* s);

/* Human-readable description of the last failure on this thread (valid until
 * the next call on this thread; never NULL).  Plumbing: no passage. */
const char* qsv_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LIBQSV_ABI_H_ */
