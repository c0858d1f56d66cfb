/*
 * oracle.c -- plain complex128 state-vector reference simulator.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no source with the GPU
 * library: gate matrices, index arithmetic, reductions and sampling are all
 * written out here again from their definitions.
 *
 * What it computes (paper: section I, "brute-force" simulation in the full
 * 2^n Hilbert space; section II, the wave-function as a rank-n tensor whose
 * index bits are the qubits; section IV.A, execution of the instruction list
 * in program (pre-order) order; section V.B, per-term expectation values of
 * a Pauli-sum Hamiltonian and MEASURE):
 *
 *   O1  psi = e_x, N = 2^n amplitudes, qubit q = bit q of the index.
 *   O2  each gate's matrix is built in FP64 from its name and angles.
 *   O3  a k-qubit gate on qubits (q_0..q_{k-1}) (q_0 = least significant bit
 *       of the local index) acts, for every base index b with all listed bits
 *       clear, on the 2^k-vector v_m = psi[b + sum_j m_j 2^{q_j}]: v <- U v.
 *   O4  <P> for a Pauli string = <psi| (P psi) >, computed by applying the
 *       Pauli factors as gates to a copy and taking the inner product.
 *   O5  norm = sum |psi_i|^2.
 *   O6  sample(u) = smallest i with C_i > u * C_{N-1}, C the sequential
 *       inclusive prefix sum of |psi_i|^2 (last index with nonzero
 *       probability if rounding leaves none).
 *
 * All sums over the state use pairwise (recursive halving) summation.
 * Loops may run under OpenMP; the arithmetic per element is unchanged by it.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* gate identifiers of the oracle's own table (mapped from names in oracle.py) */
enum {
  O_I = 0, O_X, O_Y, O_Z, O_H, O_S, O_SDG, O_T, O_TDG, O_RX, O_RY, O_RZ,
  O_CNOT, O_CZ, O_CPHASE, O_SWAP, O_U
};

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

/* O2: gate matrix (row-major, dim x dim) for a named gate.  Returns the
 * number of qubits, or -1 for an unknown gate.  Rotations follow
 * R_P(theta) = exp(-i theta P / 2) = cos(theta/2) I - i sin(theta/2) P. */
int orc_gate_matrix(int gate, const double* p, cplx* out) {
  const double r2 = 1.0 / sqrt(2.0);
  double c, s;
  memset(out, 0, 16 * sizeof(cplx));
  switch (gate) {
    case O_I: out[0] = 1; out[3] = 1; return 1;
    case O_X: out[1] = 1; out[2] = 1; return 1;
    case O_Y: out[1] = -I; out[2] = I; return 1;
    case O_Z: out[0] = 1; out[3] = -1; return 1;
    case O_H: out[0] = r2; out[1] = r2; out[2] = r2; out[3] = -r2; return 1;
    case O_S: out[0] = 1; out[3] = I; return 1;
    case O_SDG: out[0] = 1; out[3] = -I; return 1;
    case O_T: out[0] = 1; out[3] = cexp(I * M_PI / 4.0); return 1;
    case O_TDG: out[0] = 1; out[3] = cexp(-I * M_PI / 4.0); return 1;
    case O_RX:
      c = cos(p[0] / 2.0); s = sin(p[0] / 2.0);
      out[0] = c; out[1] = -I * s; out[2] = -I * s; out[3] = c; return 1;
    case O_RY:
      c = cos(p[0] / 2.0); s = sin(p[0] / 2.0);
      out[0] = c; out[1] = -s; out[2] = s; out[3] = c; return 1;
    case O_RZ:
      out[0] = cexp(-I * p[0] / 2.0); out[3] = cexp(I * p[0] / 2.0); return 1;
    /* two-qubit gates: local index m = bit(first qubit) + 2*bit(second) */
    case O_CNOT: /* (control, target): flips target where control = 1 */
      out[0 * 4 + 0] = 1; out[2 * 4 + 2] = 1;
      out[3 * 4 + 1] = 1; out[1 * 4 + 3] = 1; return 2;
    case O_CZ:
      out[0] = 1; out[5] = 1; out[10] = 1; out[15] = -1; return 2;
    case O_CPHASE:
      out[0] = 1; out[5] = 1; out[10] = 1; out[15] = cexp(I * p[0]); return 2;
    case O_SWAP:
      out[0] = 1; out[2 * 4 + 1] = 1; out[1 * 4 + 2] = 1; out[15] = 1; return 2;
    default: return -1;
  }
}

/* O1 */
void orc_init_basis(cplx* psi, int n, uint64_t x) {
  uint64_t N = 1ull << n;
  for (uint64_t i = 0; i < N; ++i) psi[i] = 0;
  psi[x] = 1;
}

/* O3: apply a dense 2^k x 2^k matrix U (row-major) to qubits q[0..k-1]. */
int orc_apply_matrix(cplx* psi, int n, int k, const int* q, const cplx* U) {
  if (k < 1 || k > 10) return -1;
  uint64_t mask = 0;
  for (int j = 0; j < k; ++j) {
    if (q[j] < 0 || q[j] >= n) return -1;
    if (mask & (1ull << q[j])) return -1;
    mask |= 1ull << q[j];
  }
  const int64_t N = (int64_t)1 << n;
  const int D = 1 << k;
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < N; ++b) {
    if ((uint64_t)b & mask) continue;
    uint64_t idx[1024];
    cplx v[1024];
    for (int m = 0; m < D; ++m) {
      uint64_t i = (uint64_t)b;
      for (int j = 0; j < k; ++j)
        if ((m >> j) & 1) i |= 1ull << q[j];
      idx[m] = i;
      v[m] = psi[i];
    }
    for (int r = 0; r < D; ++r) {
      cplx acc = 0;
      for (int c = 0; c < D; ++c) acc += U[(size_t)r * D + c] * v[c];
      psi[idx[r]] = acc;
    }
  }
  return 0;
}

/* O2 + O3 for one gate record.  mat (interleaved re,im, row-major) is used
 * only for O_U with nq qubits. */
int orc_apply_op(cplx* psi, int n, int gate, int nq, const int* q, const double* p,
                 const double* mat) {
  if (gate == O_U) {
    if (nq < 1 || nq > 10 || !mat) return -1;
    return orc_apply_matrix(psi, n, nq, q, (const cplx*)mat);
  }
  cplx U[16];
  int k = orc_gate_matrix(gate, p, U);
  if (k < 0 || k != nq) return -1;
  return orc_apply_matrix(psi, n, k, q, U);
}

/* ---- pairwise sums ---------------------------------------------------- */

static double pw_norm(const cplx* a, uint64_t n) {
  if (n <= 16) {
    double s = 0;
    for (uint64_t i = 0; i < n; ++i) s += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    return s;
  }
  uint64_t h = n / 2;
  return pw_norm(a, h) + pw_norm(a + h, n - h);
}

static cplx pw_dot(const cplx* a, const cplx* b, uint64_t n) {
  if (n <= 16) {
    cplx s = 0;
    for (uint64_t i = 0; i < n; ++i) s += conj(a[i]) * b[i];
    return s;
  }
  uint64_t h = n / 2;
  return pw_dot(a, b, h) + pw_dot(a + h, b + h, n - h);
}

/* O5 */
double orc_norm(const cplx* psi, int n) {
  uint64_t N = 1ull << n;
  /* split the top of the recursion across threads; each half is pairwise */
  if (n >= 12) {
    const int P = 64;
    double part[64];
#pragma omp parallel for schedule(static)
    for (int t = 0; t < P; ++t) part[t] = pw_norm(psi + (N / P) * t, N / P);
    /* combine the 64 partials pairwise in a fixed order */
    for (int w = 1; w < P; w *= 2)
      for (int t = 0; t + w < P; t += 2 * w) part[t] += part[t + w];
    return part[0];
  }
  return pw_norm(psi, N);
}

/* <a|b> = sum conj(a_i) b_i */
void orc_inner(const cplx* a, const cplx* b, int n, double* out_re_im) {
  uint64_t N = 1ull << n;
  cplx r;
  if (n >= 12) {
    const int P = 64;
    cplx part[64];
#pragma omp parallel for schedule(static)
    for (int t = 0; t < P; ++t) part[t] = pw_dot(a + (N / P) * t, b + (N / P) * t, N / P);
    for (int w = 1; w < P; w *= 2)
      for (int t = 0; t + w < P; t += 2 * w) part[t] += part[t + w];
    r = part[0];
  } else {
    r = pw_dot(a, b, N);
  }
  out_re_im[0] = creal(r);
  out_re_im[1] = cimag(r);
}

/* O4: <psi|P|psi> for P = prod_j paulis[j] on qubits[j] (paulis: 1=X 2=Y 3=Z).
 * work must hold 2^n amplitudes.  Returns 0 or -1. */
int orc_pauli_expval(const cplx* psi, int n, int w, const int* paulis, const int* qubits,
                     cplx* work, double* out_re_im) {
  uint64_t N = 1ull << n;
  memcpy(work, psi, N * sizeof(cplx));
  for (int j = 0; j < w; ++j) {
    int g = paulis[j] == 1 ? O_X : paulis[j] == 2 ? O_Y : paulis[j] == 3 ? O_Z : -1;
    if (g < 0) return -1;
    double p0 = 0;
    if (orc_apply_op(work, n, g, 1, &qubits[j], &p0, NULL)) return -1;
  }
  orc_inner(psi, work, n, out_re_im);
  return 0;
}

/* O6: inverse-CDF sampling with the caller's uniforms in [0, 1). */
int orc_sample(const cplx* psi, int n, const double* u, int shots, uint64_t* out) {
  uint64_t N = 1ull << n;
  double* C = (double*)malloc(N * sizeof(double));
  if (!C) return -1;
  double acc = 0;
  uint64_t last_nz = 0;
  for (uint64_t i = 0; i < N; ++i) {
    double p = creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]);
    acc += p;
    C[i] = acc;
    if (p > 0) last_nz = i;
  }
  const double total = C[N - 1];
  for (int s = 0; s < shots; ++s) {
    if (!(u[s] >= 0.0 && u[s] < 1.0)) { free(C); return -1; }
    double t = u[s] * total;
    /* smallest i with C[i] > t (C is non-decreasing) */
    uint64_t lo = 0, hi = N;
    while (lo < hi) {
      uint64_t mid = lo + (hi - lo) / 2;
      if (C[mid] > t) hi = mid; else lo = mid + 1;
    }
    out[s] = lo < N ? lo : last_nz;
  }
  free(C);
  return 0;
}
