// dense_mfma.hip -- explicit k-qubit blocks (k = 4..6) on the matrix cores.
//
// A fused super-gate (paper section II: gates aggregated into one operator
// that acts as a whole) on k qubits is a dense 2^k x 2^k complex matrix U.
// For every group of 2^k amplitudes that differ only in the block's qubits,
// y = U x.  Over all groups this is the real matrix product
//     [Y_re; Y_im] = [[U_re, -U_im], [U_im, U_re]] [X_re; X_im]
// (rows and columns interleaved re/im), i.e. a (2^(k+1) x 2^(k+1)) x
// (2^(k+1) x groups) GEMM, which runs on MFMA:
//   complex64  : v_mfma_f32_32x32x2_f32, 32 groups per wavefront
//   complex128 : v_mfma_f64_16x16x4_f64, 16 groups per wavefront
// A workgroup stages a tile -- the block qubits plus the lowest other qubits,
// so that global access is in contiguous segments -- in LDS (XOR-swizzled),
// each wavefront multiplies its groups, and the tile is written back.  The
// embedded matrix is precomputed by the host in MFMA operand order.
#include <complex>
#include <vector>

#include "internal.hpp"
#include "tile.hpp"

namespace qsv {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mf;
template <>
struct Mf<float> {
  static constexpr int M = 32;     // rows per instruction (and groups per wavefront)
  static constexpr int KK = 2;     // reduction depth per instruction
  static constexpr int NACC = 16;  // accumulator registers per lane
  static constexpr int SB = 5;     // LDS swizzle bits
  using acc_t = floatx16;
  __device__ static acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
  // D[i][j]: j = lane % 32, i = (v % 4) + 8 (v / 4) + 4 (lane / 32) (measured on gfx950)
  __device__ static int drow(int lane, int v) { return (v & 3) + 8 * (v >> 2) + 4 * (lane >> 5); }
};
template <>
struct Mf<double> {
  static constexpr int M = 16;
  static constexpr int KK = 4;
  static constexpr int NACC = 4;
  static constexpr int SB = 4;
  using acc_t = doublex4;
  __device__ static acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // D[i][j]: j = lane % 16, i = 4 v + lane / 16 (measured on gfx950)
  __device__ static int drow(int lane, int v) { return 4 * v + (lane >> 4); }
};
// A[i][k] and B[k][j] sit in lane (i or j) + M * k for both instructions.

struct DenseDesc {
  int t, c, k, nns;
  int S[16];      // tile qubits, ascending
  int nonS[40];   // other qubits, ascending
  int bpos[6];    // local position of listed block qubit j
  int gpos[8];    // local positions of the group bits, ascending
};

constexpr int kDenseThreads = 256;

template <typename T, int K>
__global__ __launch_bounds__(kDenseThreads) void k_dense_mfma(cpx<T>* __restrict__ psi, DenseDesc d,
                                                               const T* __restrict__ frag,
                                                               uint64_t ntiles) {
  using F = Mf<T>;
  constexpr int D = 1 << K;        // complex dimension
  constexpr int R2 = 2 * D;        // real dimension
  constexpr int MT = R2 / F::M;    // M tiles
  constexpr int KS = R2 / F::KK;   // reduction steps
  constexpr int A = VecInfo<T>::A;
  constexpr int TMAX = K + (sizeof(T) == 4 ? 7 : 6);
  __shared__ cpx<T> tile[1 << TMAX];
  __shared__ uint64_t segoff[1 << (TMAX - 4 > 0 ? TMAX - 4 : 1)];
  __shared__ uint32_t moff[D];
  __shared__ uint32_t goff[1 << (TMAX - K)];

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int t = d.t, c = d.c;
  const int ng = 1 << (t - K);
  for (int m = threadIdx.x; m < D; m += kDenseThreads) {
    uint32_t o = 0;
    for (int j = 0; j < K; ++j)
      if ((m >> j) & 1) o |= 1u << d.bpos[j];
    moff[m] = o;
  }
  for (int g = threadIdx.x; g < ng; g += kDenseThreads) {
    uint32_t o = 0;
    for (int j = 0; j < t - K; ++j)
      if ((g >> j) & 1) o |= 1u << d.gpos[j];
    goff[g] = o;
  }
  const int nseg = 1 << (t - c);
  for (int h = threadIdx.x; h < nseg; h += kDenseThreads) {
    uint64_t o = 0;
    for (int j = 0; j < t - c; ++j)
      if ((h >> j) & 1) o |= 1ull << d.S[c + j];
    segoff[h] = o;
  }
  __syncthreads();

  vec16<T>* gv = reinterpret_cast<vec16<T>*>(psi);
  const int nvec = (1 << t) / A;
  const uint32_t cmask = (1u << c) - 1u;
  // this wavefront's groups: n = wave * M + (lane % M)
  const int n = wave * F::M + (lane % F::M);
  const bool live = n < ng;
  const uint32_t gsw = live ? tile_swizzle(goff[n], F::SB) : 0u;
  const int kq = lane / F::M;  // reduction index within an instruction

  for (uint64_t tid = blockIdx.x; tid < ntiles; tid += gridDim.x) {
    uint64_t base = 0;
    for (int i = 0; i < d.nns; ++i) base |= ((tid >> i) & 1ull) << d.nonS[i];
    for (int i = threadIdx.x; i < nvec; i += kDenseThreads) {
      const uint32_t l = (uint32_t)i * A;
      const uint64_t g = base | segoff[l >> c] | (l & cmask);
      const vec16<T> x = gv[g / A];
#pragma unroll
      for (int e = 0; e < A; ++e) tile[tile_swizzle(l + e, F::SB)] = x.a[e];
    }
    __syncthreads();

    typename F::acc_t acc[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int v = 0; v < F::NACC; ++v) acc[mt][v] = T(0);
    const T* fr = frag + lane;
    for (int s = 0; s < KS; ++s) {
      // B[kk][n]: real column rc = KK s + kk -> complex column rc / 2, part rc % 2
      const int rc = F::KK * s + kq;
      T b = T(0);
      if (live) {
        const cpx<T> x = tile[gsw ^ tile_swizzle(moff[rc >> 1], F::SB)];
        b = (rc & 1) ? x.y : x.x;
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt] = F::mma(fr[(size_t)(mt * KS + s) * 64], b, acc[mt]);
    }
    __syncthreads();  // every group's inputs are read before any output is written
    if (live) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int v = 0; v < F::NACC; ++v) {
          const int r = mt * F::M + F::drow(lane, v);  // real output row
          cpx<T>& dst = tile[gsw ^ tile_swizzle(moff[r >> 1], F::SB)];
          if (r & 1) dst.y = acc[mt][v];
          else dst.x = acc[mt][v];
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nvec; i += kDenseThreads) {
      const uint32_t l = (uint32_t)i * A;
      vec16<T> x;
#pragma unroll
      for (int e = 0; e < A; ++e) x.a[e] = tile[tile_swizzle(l + e, F::SB)];
      const uint64_t g = base | segoff[l >> c] | (l & cmask);
      gv[g / A] = x;
    }
    __syncthreads();
  }
}

// Host: the real embedding of U in MFMA A-operand order,
// frag[(mt * KS + s) * 64 + lane] = A[M mt + lane % M][KK s + lane / M].
template <typename T>
void dense_mfma_fragments(int k, const std::complex<double>* mat, std::vector<T>& frag) {
  const int Mr = sizeof(T) == 4 ? 32 : 16, KK = sizeof(T) == 4 ? 2 : 4;
  const int D = 1 << k, R2 = 2 * D, MT = R2 / Mr, KS = R2 / KK;
  frag.assign((size_t)MT * KS * 64, T(0));
  for (int mt = 0; mt < MT; ++mt)
    for (int s = 0; s < KS; ++s)
      for (int l = 0; l < 64; ++l) {
        const int r = Mr * mt + l % Mr, rc = KK * s + l / Mr;
        const int p = r >> 1, q = rc >> 1;
        const double ur = mat[p * D + q].real(), ui = mat[p * D + q].imag();
        double v;
        if (!(r & 1)) v = (rc & 1) ? -ui : ur;
        else v = (rc & 1) ? ur : ui;
        frag[((size_t)mt * KS + s) * 64 + l] = (T)v;
      }
}

size_t dense_mfma_frag_count(int k, bool f32) {
  const int Mr = f32 ? 32 : 16, KK = f32 ? 2 : 4;
  const int R2 = 2 << k;
  return (size_t)(R2 / Mr) * (R2 / KK) * 64;
}

template <typename T>
hipError_t launch_dense_mfma(cpx<T>* psi, int n, int k, const int* qubits, const T* frag_dev,
                             hipStream_t st) {
  DenseDesc d{};
  const int gbits = sizeof(T) == 4 ? 7 : 6;
  int t = k + gbits;
  if (t > n) t = n;
  d.t = t;
  d.k = k;
  // tile = block qubits + the lowest t - k other qubits
  uint64_t Smask = 0;
  for (int j = 0; j < k; ++j) Smask |= 1ull << qubits[j];
  int need = t - k;
  for (int q = 0; q < n && need > 0; ++q)
    if (!((Smask >> q) & 1)) {
      Smask |= 1ull << q;
      --need;
    }
  int ns = 0, nn = 0;
  for (int q = 0; q < n; ++q) {
    if ((Smask >> q) & 1) d.S[ns++] = q;
    else d.nonS[nn++] = q;
  }
  d.nns = nn;
  int c = 0;
  while (c < t && d.S[c] == c) ++c;
  // S holds the lowest t - k non-block qubits, so c >= t - k: every segment is
  // at least one 16-byte vector and 2^(t-c) <= 2^k fits the segment table
  if (c < VecInfo<T>::LOG_A || t - c > k) return hipErrorInvalidValue;
  d.c = c;
  int gi = 0;
  for (int j = 0; j < t; ++j) {
    bool blk = false;
    for (int b = 0; b < k; ++b)
      if (d.S[j] == qubits[b]) {
        d.bpos[b] = j;
        blk = true;
      }
    if (!blk) d.gpos[gi++] = j;
  }
  const uint64_t ntiles = 1ull << (n - t);
  const unsigned grid = (unsigned)(ntiles < 2048 ? ntiles : 2048);
  switch (k) {
#define QSV_DK(KV)                                                                               \
  case KV:                                                                                       \
    hipLaunchKernelGGL((k_dense_mfma<T, KV>), dim3(grid), dim3(kDenseThreads), 0, st, psi, d,    \
                       frag_dev, ntiles);                                                        \
    break;
    QSV_DK(4)
    QSV_DK(5)
    QSV_DK(6)
#undef QSV_DK
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template void dense_mfma_fragments<float>(int, const std::complex<double>*, std::vector<float>&);
template void dense_mfma_fragments<double>(int, const std::complex<double>*, std::vector<double>&);
template hipError_t launch_dense_mfma<float>(cpx<float>*, int, int, const int*, const float*,
                                             hipStream_t);
template hipError_t launch_dense_mfma<double>(cpx<double>*, int, int, const int*, const double*,
                                              hipStream_t);

}  // namespace qsv
