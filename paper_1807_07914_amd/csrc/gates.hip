// gates.hip -- per-gate state-vector kernels for gfx950 (one HBM pass per gate).
//
// The paper's section I: each 1- or 2-qubit gate is a sparse matrix-vector
// product over the full 2^n amplitude array with low arithmetic intensity,
// so these kernels are pure streaming kernels: every thread owns a few
// amplitude pairs/quartets, loads them with 16-byte vector loads where the
// partner layout allows, applies the small matrix in registers and stores
// back in place.  No amplitude is touched by two threads of one launch.
#include <algorithm>

#include "internal.hpp"

namespace qsv {

constexpr int kBlock = 256;
constexpr int kGate1Items = 2, kDiag1Items = 4, kGate2Items = 2, kPerm2Items = 4;

// Workgroups each per-gate launch covers (grid_for turns them into a grid).
template <typename T>
static uint64_t init_blocks(uint64_t N) {
  return (N / VecInfo<T>::A + kBlock - 1) / kBlock;
}
template <typename T>
static uint64_t gate1_blocks(int n) {
  const uint64_t items = (1ull << n) / (2 * VecInfo<T>::A);
  return (items + kBlock * kGate1Items - 1) / (kBlock * kGate1Items);
}
template <typename T>
static uint64_t diag1_blocks(int n) {
  const uint64_t nvec = (1ull << n) / VecInfo<T>::A;
  return (nvec + kBlock * kDiag1Items - 1) / (kBlock * kDiag1Items);
}
static uint64_t gate2_blocks(int n) {
  return ((1ull << n) / 4 + kBlock * kGate2Items - 1) / (kBlock * kGate2Items);
}
static uint64_t perm2_blocks(int n) {
  return ((1ull << n) / 4 + kBlock * kPerm2Items - 1) / (kBlock * kPerm2Items);
}
static uint64_t dense_blocks(int n, int k) {
  const uint64_t G = kBlock >> k;
  return (((1ull << n) >> k) + G - 1) / G;
}

// ---------------------------------------------------------------- init
template <typename T>
__global__ __launch_bounds__(kBlock) void k_init_basis(vec16<T>* __restrict__ v, uint64_t nvec,
                                                        uint64_t x) {
  constexpr int A = VecInfo<T>::A;
  const uint64_t i = block_index() * kBlock + threadIdx.x;
  if (i >= nvec) return;
  vec16<T> z;
#pragma unroll
  for (int e = 0; e < A; ++e) {
    z.a[e].x = (i * A + e == x) ? T(1) : T(0);
    z.a[e].y = T(0);
  }
  v[i] = z;
}

template <typename T>
hipError_t launch_init_basis(cpx<T>* psi, uint64_t N, uint64_t x, hipStream_t st) {
  constexpr int A = VecInfo<T>::A;
  const uint64_t nvec = N / A;
  hipLaunchKernelGGL(k_init_basis<T>, grid_for(init_blocks<T>(N)), dim3(kBlock), 0, st,
                     reinterpret_cast<vec16<T>*>(psi), nvec, x);
  return hipGetLastError();
}

// ------------------------------------------------------ 1-qubit, general
// Work item = two 16-byte vectors.  For q >= log2(A) the vectors hold the
// bit-q = 0 and bit-q = 1 partners of A pairs; for complex64 and q = 0 the
// item is two adjacent vectors, each holding one whole pair.
template <typename T, int IPT>
__global__ __launch_bounds__(kBlock) void k_gate1(vec16<T>* __restrict__ v, uint64_t items, int q,
                                                   M2<T> U) {
  constexpr int A = VecInfo<T>::A;
  constexpr int LA = VecInfo<T>::LOG_A;
  const uint64_t base = block_index() * (kBlock * IPT) + threadIdx.x;
  vec16<T> lo[IPT], hi[IPT];
  uint64_t il[IPT], ih[IPT];
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const uint64_t it = base + (uint64_t)j * kBlock;
    if (q >= LA) {
      const uint64_t a = insert0(it * A, q);
      il[j] = a / A;
      ih[j] = (a + (1ull << q)) / A;
    } else {
      il[j] = 2 * it;
      ih[j] = 2 * it + 1;
    }
    if (it < items) {
      lo[j] = v[il[j]];
      hi[j] = v[ih[j]];
    }
  }
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const uint64_t it = base + (uint64_t)j * kBlock;
    if (it >= items) continue;
    if (q >= LA) {
#pragma unroll
      for (int e = 0; e < A; ++e) apply2(U, lo[j].a[e], hi[j].a[e]);
    } else {
      apply2(U, lo[j].a[0], lo[j].a[A - 1]);
      apply2(U, hi[j].a[0], hi[j].a[A - 1]);
    }
    v[il[j]] = lo[j];
    v[ih[j]] = hi[j];
  }
}

// scalar fallback for registers smaller than one work item
template <typename T>
__global__ void k_gate1_scalar(cpx<T>* __restrict__ psi, uint64_t pairs, int q, M2<T> U) {
  const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= pairs) return;
  const uint64_t i0 = insert0(k, q), i1 = i0 | (1ull << q);
  cpx<T> a = psi[i0], b = psi[i1];
  apply2(U, a, b);
  psi[i0] = a;
  psi[i1] = b;
}

template <typename T>
hipError_t launch_gate1(cpx<T>* psi, int n, int q, const M2<T>& U, hipStream_t st) {
  constexpr int A = VecInfo<T>::A;
  constexpr int IPT = kGate1Items;
  const uint64_t N = 1ull << n;
  if (N < 4 * (uint64_t)A) {
    hipLaunchKernelGGL(k_gate1_scalar<T>, dim3(1), dim3(64), 0, st, psi, N / 2, q, U);
    return hipGetLastError();
  }
  const uint64_t items = N / (2 * A);
  hipLaunchKernelGGL((k_gate1<T, IPT>), grid_for(gate1_blocks<T>(n)), dim3(kBlock), 0, st,
                     reinterpret_cast<vec16<T>*>(psi), items, q, U);
  return hipGetLastError();
}

// ----------------------------------------------------- 1-qubit, diagonal
template <typename T, int IPT>
__global__ __launch_bounds__(kBlock) void k_diag1(vec16<T>* __restrict__ v, uint64_t nvec, int q,
                                                   cpx<T> d0, cpx<T> d1) {
  constexpr int A = VecInfo<T>::A;
  const uint64_t base = block_index() * (kBlock * IPT) + threadIdx.x;
  vec16<T> x[IPT];
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const uint64_t it = base + (uint64_t)j * kBlock;
    if (it < nvec) x[j] = v[it];
  }
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const uint64_t it = base + (uint64_t)j * kBlock;
    if (it >= nvec) continue;
#pragma unroll
    for (int e = 0; e < A; ++e) {
      const uint64_t i = it * A + e;
      x[j].a[e] = cmul(((i >> q) & 1ull) ? d1 : d0, x[j].a[e]);
    }
    v[it] = x[j];
  }
}

template <typename T>
hipError_t launch_diag1(cpx<T>* psi, int n, int q, cpx<T> d0, cpx<T> d1, hipStream_t st) {
  constexpr int A = VecInfo<T>::A;
  constexpr int IPT = kDiag1Items;
  const uint64_t nvec = (1ull << n) / A;
  hipLaunchKernelGGL((k_diag1<T, IPT>), grid_for(diag1_blocks<T>(n)), dim3(kBlock), 0, st,
                     reinterpret_cast<vec16<T>*>(psi), nvec, q, d0, d1);
  return hipGetLastError();
}

// ------------------------------------------------------ 2-qubit, general
// Quartet (i0, i0|2^qa, i0|2^qb, i0|2^qa|2^qb), qa < qb; U is indexed with
// qa as the least-significant local bit.
template <typename T, int IPT>
__global__ __launch_bounds__(kBlock) void k_gate2(cpx<T>* __restrict__ psi, uint64_t items, int qa,
                                                   int qb, M4<T> U) {
  const uint64_t base = block_index() * (kBlock * IPT) + threadIdx.x;
  const uint64_t A = 1ull << qa, B = 1ull << qb;
  cpx<T> x[IPT][4];
  uint64_t i0[IPT];
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const uint64_t it = base + (uint64_t)j * kBlock;
    i0[j] = insert00(it, qa, qb);
    if (it < items) {
      x[j][0] = psi[i0[j]];
      x[j][1] = psi[i0[j] | A];
      x[j][2] = psi[i0[j] | B];
      x[j][3] = psi[i0[j] | A | B];
    }
  }
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const uint64_t it = base + (uint64_t)j * kBlock;
    if (it >= items) continue;
    cpx<T> y[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      cpx<T> acc = cmul(U.m[r * 4 + 0], x[j][0]);
      acc = cfma(U.m[r * 4 + 1], x[j][1], acc);
      acc = cfma(U.m[r * 4 + 2], x[j][2], acc);
      acc = cfma(U.m[r * 4 + 3], x[j][3], acc);
      y[r] = acc;
    }
    psi[i0[j]] = y[0];
    psi[i0[j] | A] = y[1];
    psi[i0[j] | B] = y[2];
    psi[i0[j] | A | B] = y[3];
  }
}

template <typename T>
hipError_t launch_gate2(cpx<T>* psi, int n, int qa, int qb, const M4<T>& U, hipStream_t st) {
  constexpr int IPT = kGate2Items;
  const uint64_t items = (1ull << n) / 4;
  hipLaunchKernelGGL((k_gate2<T, IPT>), grid_for(gate2_blocks(n)), dim3(kBlock), 0, st, psi, items, qa,
                     qb, U);
  return hipGetLastError();
}

// ------------------------------------------- 2-qubit permutations / phase
// mode 0: CNOT (swap i|C <-> i|C|T), 1: SWAP (i|A <-> i|B), 2: phase on i|A|B
template <typename T, int MODE, int IPT>
__global__ __launch_bounds__(kBlock) void k_perm2(cpx<T>* __restrict__ psi, uint64_t items, int lo,
                                                   int hi, uint64_t P, uint64_t Q, cpx<T> ph) {
  const uint64_t base = block_index() * (kBlock * IPT) + threadIdx.x;
  cpx<T> a[IPT], b[IPT];
  uint64_t ia[IPT], ib[IPT];
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const uint64_t it = base + (uint64_t)j * kBlock;
    const uint64_t i0 = insert00(it, lo, hi);
    ia[j] = i0 | P;
    ib[j] = i0 | Q;
    if (it < items) {
      a[j] = psi[ia[j]];
      if (MODE != 2) b[j] = psi[ib[j]];
    }
  }
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const uint64_t it = base + (uint64_t)j * kBlock;
    if (it >= items) continue;
    if (MODE == 2) {
      psi[ia[j]] = cmul(ph, a[j]);
    } else {
      psi[ia[j]] = b[j];
      psi[ib[j]] = a[j];
    }
  }
}

template <typename T, int MODE>
static hipError_t launch_perm2(cpx<T>* psi, int n, int a, int b, uint64_t P, uint64_t Q, cpx<T> ph,
                               hipStream_t st) {
  constexpr int IPT = kPerm2Items;
  const int lo = a < b ? a : b, hi = a < b ? b : a;
  const uint64_t items = (1ull << n) / 4;
  hipLaunchKernelGGL((k_perm2<T, MODE, IPT>), grid_for(perm2_blocks(n)), dim3(kBlock), 0, st, psi, items,
                     lo, hi, P, Q, ph);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cnot(cpx<T>* psi, int n, int c, int t, hipStream_t st) {
  const uint64_t C = 1ull << c, Tm = 1ull << t;
  return launch_perm2<T, 0>(psi, n, c, t, C, C | Tm, cpx<T>{T(1), T(0)}, st);
}

template <typename T>
hipError_t launch_swap(cpx<T>* psi, int n, int a, int b, hipStream_t st) {
  return launch_perm2<T, 1>(psi, n, a, b, 1ull << a, 1ull << b, cpx<T>{T(1), T(0)}, st);
}

template <typename T>
hipError_t launch_cphase(cpx<T>* psi, int n, int a, int b, cpx<T> ph, hipStream_t st) {
  const uint64_t P = (1ull << a) | (1ull << b);
  return launch_perm2<T, 2>(psi, n, a, b, P, P, ph, st);
}

// ---------------------------------------------------- dense k-qubit (VALU)
// Generic fallback for an explicit 2^k x 2^k matrix: a workgroup stages
// 256 / 2^k groups of 2^k amplitudes in LDS; thread (group, row) computes one
// output amplitude from the staged group and the transposed matrix in LDS.
struct QList {
  int q[6];       // listed order: q[0] = least-significant local bit
  int sorted[6];  // ascending, for base-index insertion
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_dense(cpx<T>* __restrict__ psi, int k, QList ql,
                                                   const cpx<T>* __restrict__ mat, uint64_t groups,
                                                   int lds_mat) {
  extern __shared__ unsigned char smem_raw[];
  const int D = 1 << k;
  const int G = kBlock / D;  // groups per workgroup (D <= 64 so G >= 4)
  // matrix transposed in LDS (sUt[c*D + r]) when it fits, else read from
  // global memory (L2-resident) in row-major order
  cpx<T>* sx = reinterpret_cast<cpx<T>*>(smem_raw);   // G*D staged inputs
  cpx<T>* sUt = sx + G * D;
  if (lds_mat)
    for (int e = threadIdx.x; e < D * D; e += kBlock) {
      const int r = e / D, c = e % D;
      sUt[c * D + r] = mat[e];
    }
  const int gl = threadIdx.x / D, r = threadIdx.x % D;
  const uint64_t g = block_index() * G + gl;
  const bool ok = g < groups;
  uint64_t b = g;
  for (int j = 0; j < k; ++j) b = insert0(b, ql.sorted[j]);
  uint64_t idx = b;
  for (int j = 0; j < k; ++j)
    if ((r >> j) & 1) idx |= 1ull << ql.q[j];
  if (ok) sx[gl * D + r] = psi[idx];
  __syncthreads();
  if (!ok) return;
  cpx<T> acc{T(0), T(0)};
  const cpx<T>* xg = sx + gl * D;
  if (lds_mat)
    for (int c = 0; c < D; ++c) acc = cfma(sUt[c * D + r], xg[c], acc);
  else
    for (int c = 0; c < D; ++c) acc = cfma(mat[r * D + c], xg[c], acc);
  psi[idx] = acc;
}

template <typename T>
hipError_t launch_dense(cpx<T>* psi, int n, int k, const int* qubits, const cpx<T>* mat_dev,
                        hipStream_t st) {
  QList ql{};
  for (int j = 0; j < k; ++j) ql.q[j] = ql.sorted[j] = qubits[j];
  for (int a = 0; a < k; ++a)
    for (int b = a + 1; b < k; ++b)
      if (ql.sorted[b] < ql.sorted[a]) {
        int t = ql.sorted[a];
        ql.sorted[a] = ql.sorted[b];
        ql.sorted[b] = t;
      }
  const int D = 1 << k;
  const int G = kBlock / D;
  const uint64_t groups = (1ull << n) >> k;
  const int lds_mat = (size_t)D * D * sizeof(cpx<T>) <= 32768;
  const size_t shmem = (size_t)((lds_mat ? D * D : 0) + G * D) * sizeof(cpx<T>);
  hipLaunchKernelGGL(k_dense<T>, grid_for(dense_blocks(n, k)), dim3(kBlock), shmem, st, psi, k, ql, mat_dev,
                     groups, lds_mat);
  return hipGetLastError();
}

// ------------------------------------------------------ instantiations
#define QSV_INST(T)                                                                          \
  template hipError_t launch_init_basis<T>(cpx<T>*, uint64_t, uint64_t, hipStream_t);       \
  template hipError_t launch_gate1<T>(cpx<T>*, int, int, const M2<T>&, hipStream_t);        \
  template hipError_t launch_diag1<T>(cpx<T>*, int, int, cpx<T>, cpx<T>, hipStream_t);      \
  template hipError_t launch_gate2<T>(cpx<T>*, int, int, int, const M4<T>&, hipStream_t);   \
  template hipError_t launch_cnot<T>(cpx<T>*, int, int, int, hipStream_t);                  \
  template hipError_t launch_swap<T>(cpx<T>*, int, int, int, hipStream_t);                  \
  template hipError_t launch_cphase<T>(cpx<T>*, int, int, int, cpx<T>, hipStream_t);        \
  template hipError_t launch_dense<T>(cpx<T>*, int, int, const int*, const cpx<T>*, hipStream_t);
QSV_INST(float)
QSV_INST(double)

// ---------------------------------------------------------- race check
// A 4-byte word pattern that no pass writes by chance (a float NaN, and two
// of them a double NaN).
constexpr uint32_t kPoison = 0x7FBADBADu;

__global__ __launch_bounds__(kBlock) void k_poison(uint4* __restrict__ a, uint64_t nvec) {
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < nvec; i += stride)
    a[i] = uint4{kPoison, kPoison, kPoison, kPoison};
}

__global__ __launch_bounds__(kBlock) void k_race_compare(const uint4* __restrict__ a, const uint4* __restrict__ b,
                                                         uint64_t nvec, unsigned long long* __restrict__ counts) {
  unsigned long long unwritten = 0, differ = 0;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < nvec; i += stride) {
    const uint4 x = a[i], y = b[i];
    unwritten += (y.x == kPoison) + (y.y == kPoison) + (y.z == kPoison) + (y.w == kPoison);
    differ += (x.x != y.x) + (x.y != y.y) + (x.z != y.z) + (x.w != y.w);
  }
  // integer sums: the order of the additions does not matter
  for (int o = 32; o > 0; o >>= 1) {
    unwritten += __shfl_xor(unwritten, o);
    differ += __shfl_xor(differ, o);
  }
  if ((threadIdx.x & 63) == 0 && (unwritten | differ)) {
    atomicAdd(&counts[0], unwritten);
    atomicAdd(&counts[1], differ);
  }
}

static unsigned race_grid(uint64_t nvec) {
  return (unsigned)std::min<uint64_t>((nvec + kBlock - 1) / kBlock, 4096);
}

hipError_t launch_poison(void* a, uint64_t nvec, hipStream_t st) {
  if (nvec == 0) return hipSuccess;
  hipLaunchKernelGGL(k_poison, dim3(race_grid(nvec)), dim3(kBlock), 0, st, static_cast<uint4*>(a), nvec);
  return hipGetLastError();
}

hipError_t launch_race_compare(const void* a, const void* b, uint64_t nvec, unsigned long long* counts,
                               hipStream_t st) {
  if (nvec == 0) return hipSuccess;
  hipLaunchKernelGGL(k_race_compare, dim3(race_grid(nvec)), dim3(kBlock), 0, st, static_cast<const uint4*>(a),
                     static_cast<const uint4*>(b), nvec, counts);
  return hipGetLastError();
}

}  // namespace qsv

// Host-only debug export (not in the public header): the launch shapes the
// per-gate kernels use on an n-qubit register, one row of four int64 per
// kernel (grid x, grid y, threads per workgroup, workgroups the range needs)
// in the order init, 1-qubit, diagonal, 2-qubit, permutation / phase, dense
// k = 1..6 (11 rows), for checks of the geometry on the CPU.
extern "C" qsv_status qsv_debug_launch_dims(qsv_dtype dt, int n, int64_t* out) {
  using namespace qsv;
  if (dt != QSV_C64 && dt != QSV_C128) return fail(QSV_ERR_ARG, "bad dtype");
  if (n < 7 || n > max_qubits(dt)) return fail(QSV_ERR_ARG, "n out of range");
  if (!out) return fail(QSV_ERR_ARG, "out is NULL");
  const bool f = dt == QSV_C64;
  const uint64_t nb[11] = {f ? init_blocks<float>(1ull << n) : init_blocks<double>(1ull << n),
                           f ? gate1_blocks<float>(n) : gate1_blocks<double>(n),
                           f ? diag1_blocks<float>(n) : diag1_blocks<double>(n),
                           gate2_blocks(n), perm2_blocks(n),
                           dense_blocks(n, 1), dense_blocks(n, 2), dense_blocks(n, 3),
                           dense_blocks(n, 4), dense_blocks(n, 5), dense_blocks(n, 6)};
  for (int r = 0; r < 11; ++r) {
    const dim3 g = grid_for(nb[r]);
    out[4 * r] = g.x;
    out[4 * r + 1] = g.y;
    out[4 * r + 2] = kBlock;
    out[4 * r + 3] = (int64_t)nb[r];
  }
  return QSV_OK;
}
