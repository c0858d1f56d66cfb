// internal.hpp -- host-side internals of libqsv (state object, error
// plumbing, kernel launcher declarations).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/qsv.h"
#include "common.hpp"

namespace qsv {

constexpr uint32_t kStateMagic = 0x31565351u;  // "QSV1"
constexpr uint32_t kDeadMagic = 0xDEADBEEFu;

void set_error(const std::string& msg);
const char* get_error();

// Status helper: records a message and returns the code.
qsv_status fail(qsv_status code, const std::string& msg);
qsv_status hip_fail(hipError_t e, const char* where);

#define QSV_HIP(call)                                      \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return ::qsv::hip_fail(e_, #call); \
  } while (0)

// Bytes a device program buffer holds beyond its last word: the tile
// kernels' layer loop reads the record after the current one before that
// record is known to exist, so up to one record (24 words) past the
// program's end is read.
constexpr int kProgSlackBytes = 256;

inline int max_qubits(qsv_dtype dt) { return dt == QSV_C128 ? QSV_MAX_QUBITS_C128 : QSV_MAX_QUBITS; }

}  // namespace qsv

struct qsv_state {
  uint32_t magic = qsv::kStateMagic;
  int n = 0;
  qsv_dtype dt = QSV_C64;
  uint64_t N = 0;           // 2^n amplitudes
  size_t amp_bytes = 8;     // 8 (complex64) or 16 (complex128)
  size_t bytes = 0;         // N * amp_bytes
  void* psi = nullptr;      // device amplitudes
  bool owns = false;
  hipStream_t stream = nullptr;
  // device workspace (reduction partials, staged matrices, sampler scratch)
  void* ws = nullptr;
  size_t ws_bytes = 0;
  // device copy of the current fused program (int32 words + matrix data)
  void* pbuf = nullptr;
  size_t pbuf_bytes = 0;
  std::vector<int32_t> hprog;     // host image kept alive across the async upload
  // second state-sized buffer (adjoint sweep: lambda)
  void* aux = nullptr;
  size_t aux_bytes = 0;
  // device copy of the adjoint sweep's tile programs and its host image
  void* apbuf = nullptr;
  size_t apbuf_bytes = 0;
  std::vector<int32_t> ahprog;
  void* hpbuf = nullptr;  // programs of lambda = H psi by tile passes
  size_t hpbuf_bytes = 0;
  std::vector<int32_t> hhprog;
  // graph of the last fused plan launched with plan option graph = 1, and
  // what its launches were made from (dtype, n, psi, program buffer, stream,
  // then per pass: word offset, body, tile and segment bits)
  hipGraph_t fg_graph = nullptr;
  hipGraphExec_t fg_exec = nullptr;
  std::vector<uint64_t> fg_sig;
  std::atomic<int> busy{0};
};

namespace qsv {

// Grow the state's device workspace to at least `bytes` (stream-ordered:
// waits for the stream before freeing a smaller buffer).
qsv_status ensure_workspace(qsv_state* s, size_t bytes);
// Grow the second state-sized buffer s->aux to the state's size.
qsv_status ensure_aux(qsv_state* s, const char* what);
// Race check helpers (gates.hip): fill nvec 16-byte vectors with the poison
// pattern; count, over nvec vectors, the 4-byte words of b that still hold
// the poison (counts[0]) and those that differ from a (counts[1]), adding to
// counts (two zeroed unsigned 64-bit counters).
hipError_t launch_poison(void* a, uint64_t nvec, hipStream_t st);
hipError_t launch_race_compare(const void* a, const void* b, uint64_t nvec, unsigned long long* counts,
                               hipStream_t st);

// ---------------------------------------------------------------- launchers
template <typename T>
hipError_t launch_init_basis(cpx<T>* psi, uint64_t N, uint64_t x, hipStream_t st);
template <typename T>
hipError_t launch_gate1(cpx<T>* psi, int n, int q, const M2<T>& U, hipStream_t st);
template <typename T>
hipError_t launch_diag1(cpx<T>* psi, int n, int q, cpx<T> d0, cpx<T> d1, hipStream_t st);
template <typename T>
hipError_t launch_gate2(cpx<T>* psi, int n, int qa, int qb, const M4<T>& U, hipStream_t st);
template <typename T>
hipError_t launch_cnot(cpx<T>* psi, int n, int c, int t, hipStream_t st);
template <typename T>
hipError_t launch_swap(cpx<T>* psi, int n, int a, int b, hipStream_t st);
template <typename T>
hipError_t launch_cphase(cpx<T>* psi, int n, int a, int b, cpx<T> ph, hipStream_t st);
// dense k-qubit matrix (1 <= k <= 6) staged in device memory (row-major
// 2^k x 2^k, state precision); qubits in listed order.
template <typename T>
hipError_t launch_dense(cpx<T>* psi, int n, int k, const int* qubits, const cpx<T>* mat_dev,
                        hipStream_t st);

// dense k-qubit block (k = 4..6) on the matrix cores; frag_dev holds the
// real embedding of the matrix in MFMA operand order (dense_mfma_fragments)
template <typename T>
hipError_t launch_dense_mfma(cpx<T>* psi, int n, int k, const int* qubits, const T* frag_dev,
                             hipStream_t st);

// adjoint: lambda = H psi, and one reverse step of a rotation (gradient into out_dev)
template <typename T>
hipError_t launch_hpsi(const cpx<T>* psi, cpx<T>* lam, int n, const uint64_t* x, const uint64_t* z,
                       const double* wr, const double* wi, int nt, hipStream_t st);
template <typename T>
hipError_t launch_adj_rot(cpx<T>* psi, cpx<T>* lam, int n, int q, const M2<T>& V, const M2<double>& G,
                          double* part, double* out_dev, hipStream_t st);
size_t adjoint_partials();
// lambda = H psi by tile passes (adjoint.hip): one pass of the program at
// prog_dev (host copy prog_host); the pass with the energy flag writes
// <psi|H|psi> to *energy_dev (part: adjoint_partials() doubles)
template <typename T>
hipError_t launch_hpsi_tile(const cpx<T>* psi, cpx<T>* lam, int n, const int32_t* prog_dev,
                            const int32_t* prog_host, double* part, double* energy_dev, hipStream_t st);
template <typename T>
int hpsi_tile_bits();
int hpsi_term_words();
// fused reverse sweep (adjoint.hip): one tile pass of the program at
// prog_dev (host copy prog_host); part holds n_grad * 1024 doubles
template <typename T>
hipError_t launch_adj_tile(cpx<T>* psi, cpx<T>* lam, int n, const int32_t* prog_dev, const int32_t* prog_host,
                           double* part, double* out_dev, hipStream_t st);
template <typename T>
int adj_tile_bits();
int adj_max_grad();
int adj_rec_words();
int adj_gate_words();
template <typename T>
int adj_round_bits();

// reductions: FP64 partials written to ws, final values to out_dev (doubles)
template <typename T>
hipError_t launch_norm(const cpx<T>* psi, uint64_t N, double* ws, double* out_dev, hipStream_t st);
// nt terms sharing one xmask; zmask[t] and the phase class of each term
// (n_y mod 4) given; out_dev[t] = Re( i^{ny_t} sum_i conj(psi_{i^x}) (-1)^{|i&z_t|} psi_i )
template <typename T>
hipError_t launch_expval_group(const cpx<T>* psi, int n, uint64_t xmask, int nt,
                               const uint64_t* zmask_host, const int* ny_host, double* ws,
                               double* out_dev, hipStream_t st);
size_t expval_ws_doubles(int n, int nt);
// nt <= 32 Z-only terms from one read: out_dev[t] = sum_i (-1)^{|i & z_t|} |psi_i|^2;
// needs n >= zreg_min_qubits<T>()
template <typename T>
hipError_t launch_expval_zreg(const cpx<T>* psi, int n, const uint64_t* zmask, int nt, double* ws,
                              double* out_dev, hipStream_t st);
template <typename T>
int zreg_min_qubits();
// nt <= 16 terms whose X masks lie in the tile qubits S (ascending, t of
// them, S[0..c) = 0..c-1): out_dev[k] as launch_expval_group gives for term k
template <typename T>
hipError_t launch_expval_tile(const cpx<T>* psi, int n, const int* S, int t, int c,
                              const uint64_t* xmask, const uint64_t* zmask, const int* ny, int nt,
                              double* ws, double* out_dev, hipStream_t st);
// the same for nt <= 16 one-qubit X / Y terms on distinct tile qubits, all
// with the same Y parity, none with Z on its register round's bits, by
// register rounds; hipErrorInvalidValue (nothing launched) otherwise
template <typename T>
hipError_t launch_expval_xreg(const cpx<T>* psi, int n, const int* S, int t, int c,
                              const uint64_t* xmask, const uint64_t* zmask, const int* ny, int nt,
                              double* ws, double* out_dev, hipStream_t st);
template <typename T>
int xtile_max_bits();
template <typename T>
int xtile_low_bits();

// sampler: returns indices into out_dev (uint64) for uniforms_dev
template <typename T>
hipError_t launch_sample(const cpx<T>* psi, int n, const double* uniforms_dev, int shots,
                         double* ws, uint64_t* out_dev, hipStream_t st);
size_t sample_ws_doubles(int n);

}  // namespace qsv
