// plan.hpp -- host-side execution entry points shared by the ABI layer and
// the circuit executor (per-gate dispatch, fused tile passes, dense blocks).
#pragma once
#include <complex>
#include <vector>

#include "internal.hpp"

namespace qsv {

int gate_matrix(int g, const double* p, std::complex<double>* m);
bool gate_is_diagonal(int g);
int gate_arity(int g);
int gate_nparams(int g);
qsv_status validate_op(const qsv_state* s, const qsv_op& o);

// one instruction through the per-gate kernels (matrix staging at ws_off)
qsv_status apply_op_pergate(qsv_state* s, const qsv_op& o, size_t ws_off);
size_t dense_ws_bytes();

// real embedding of a 2^k x 2^k matrix in MFMA operand order
template <typename T>
void dense_mfma_fragments(int k, const std::complex<double>* mat, std::vector<T>& frag);

// inverse of one instruction applied to an arbitrary buffer of the state's shape
qsv_status apply_op_inverse(qsv_state* s, void* data, const qsv_op& o, size_t ws_off);

// expectation value of a Pauli sum on an arbitrary buffer (host results)
qsv_status expval_impl(qsv_state* s, const void* data, const uint64_t* xmask, const uint64_t* zmask,
                       const double* coeff, int n_terms, double* out_total, double* out_terms);

// explicit k-qubit matrix (qsv_apply_fused)
qsv_status apply_fused_block(qsv_state* s, const qsv_op& o);

// whole gate list (qsv_apply_circuit); ops already validated
qsv_status run_circuit(qsv_state* s, const qsv_op* ops, int n_ops, const qsv_plan_opts& opts);

// passes / fallback ops the fused planner would use (diagnostics)
qsv_status plan_passes(const qsv_state* s, const qsv_op* ops, int n_ops, int tile_qubits,
                       int* passes, int* fallback_ops);

qsv_status plan_program(const qsv_state* s, const qsv_op* ops, int n_ops, int tile_qubits,
                        std::vector<int32_t>& prog, std::vector<int64_t>& steps);

// The gate list the adjoint sweep's planner works on: each CNOT(c, t) as
// H_t CZ(c, t) H_t, other ops unchanged; origin (if given) receives each
// op's index in the input list.
void expand_cnots(const qsv_op* ops, int n_ops, std::vector<qsv_op>& out, std::vector<int>* origin = nullptr);

// Reverse sweep of the adjoint gradient as tile passes: ops[n_ops-1] .. ops[0]
// taken as their inverses (the same structure), grouped by the fused
// planner.  A step is either a tile pass over qubits S with the original op
// indices in a valid application order, or one op that no tile takes.
struct AdjStep {
  bool tile = true;
  int op = -1;
  std::vector<int> S;
  std::vector<int> ops;
};
void plan_adjoint(const qsv_op* ops, int n_ops, int n, int t, int c, int RB, std::vector<AdjStep>& steps);

}  // namespace qsv
