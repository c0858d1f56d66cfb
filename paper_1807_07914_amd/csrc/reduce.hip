// reduce.hip -- FP64 reductions over the amplitude array: norm, Pauli-string
// expectation values and inverse-CDF sampling.
//
// Paper section V.B computes one expectation value per Hamiltonian term and
// uses MEASURE on the register; here both are exact reductions of the state
// vector.  Every reduction is two-stage and deterministic: a fixed grid of
// workgroups writes one FP64 partial per (workgroup, term) in a fixed
// per-thread order and a fixed LDS tree, and a single workgroup combines the
// partials in a fixed tree.  No floating-point atomics are used.
#include <algorithm>
#include <vector>

#include "internal.hpp"
#include "tile.hpp"

namespace qsv {

constexpr int kRB = 256;         // reduction workgroup size
constexpr int kMaxPartials = 1024;

static inline unsigned reduce_grid(uint64_t units) {
  // enough workgroups to fill the chip, but a fixed function of the size
  uint64_t g = (units + kRB * 16 - 1) / (kRB * 16);
  if (g < 1) g = 1;
  if (g > kMaxPartials) g = kMaxPartials;
  return (unsigned)g;
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = kRB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// Final stage: out[t] = sum_b part[b * nt + t], one workgroup, fixed tree.
__global__ __launch_bounds__(kRB) void k_final(const double* __restrict__ part, int nb, int nt,
                                               double* __restrict__ out) {
  __shared__ double sh[kRB];
  for (int t = 0; t < nt; ++t) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += kRB) acc += part[(size_t)b * nt + t];
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) out[t] = s;
  }
}

// ---------------------------------------------------------------- norm
template <typename T>
__global__ __launch_bounds__(kRB) void k_norm_part(const vec16<T>* __restrict__ v, uint64_t nvec,
                                                   uint64_t chunk, double* __restrict__ part) {
  constexpr int A = VecInfo<T>::A;
  __shared__ double sh[kRB];
  const uint64_t lo = (uint64_t)blockIdx.x * chunk;
  const uint64_t hi = lo + chunk < nvec ? lo + chunk : nvec;
  double acc = 0.0;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += kRB) {
    const vec16<T> x = v[i];
#pragma unroll
    for (int e = 0; e < A; ++e) {
      const double re = (double)x.a[e].x, im = (double)x.a[e].y;
      acc = fma(re, re, fma(im, im, acc));
    }
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

template <typename T>
hipError_t launch_norm(const cpx<T>* psi, uint64_t N, double* ws, double* out_dev, hipStream_t st) {
  constexpr int A = VecInfo<T>::A;
  const uint64_t nvec = N / A;
  const unsigned g = reduce_grid(nvec);
  const uint64_t chunk = (nvec + g - 1) / g;
  hipLaunchKernelGGL(k_norm_part<T>, dim3(g), dim3(kRB), 0, st,
                     reinterpret_cast<const vec16<T>*>(psi), nvec, chunk, ws);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kRB), 0, st, ws, (int)g, 1, out_dev);
  return hipGetLastError();
}

// ------------------------------------------------------ expectation values
// Terms of one launch share the X-mask x.  With n_y = |x & z| (the Y count),
// <P> = Re( i^{n_y} sum_i conj(psi_{i^x}) (-1)^{|i & z|} psi_i ).
//  x == 0: accumulate (-1)^{|i&z|} |psi_i|^2.
//  x != 0: visit each pair (i, j = i^x) once (i has x's top bit clear); with
//          w = conj(psi_j) psi_i the pair contributes s_i (w + (-1)^{n_y} conj w),
//          i.e. 2 s_i Re w (n_y even) or 2i s_i Im w (n_y odd); the host applies
//          the factor 2 * Re(i^{n_y}) or 2 * Re(i^{n_y + 1}).
constexpr int kMaxTermsPerLaunch = 16;
struct ZTerms {
  uint64_t z[kMaxTermsPerLaunch];
  int odd[kMaxTermsPerLaunch];  // n_y odd -> accumulate Im w
};

template <typename T, bool XZERO>
__global__ __launch_bounds__(kRB) void k_expval_part(const cpx<T>* __restrict__ psi, uint64_t units,
                                                     uint64_t chunk, uint64_t x, int top, int nt,
                                                     ZTerms zt, double* __restrict__ part) {
  __shared__ double sh[kRB];
  double acc[kMaxTermsPerLaunch];
#pragma unroll
  for (int t = 0; t < kMaxTermsPerLaunch; ++t) acc[t] = 0.0;
  const uint64_t lo = (uint64_t)blockIdx.x * chunk;
  const uint64_t hi = lo + chunk < units ? lo + chunk : units;
  for (uint64_t u = lo + threadIdx.x; u < hi; u += kRB) {
    if (XZERO) {
      const cpx<T> a = psi[u];
      const double p = fma((double)a.x, (double)a.x, (double)a.y * (double)a.y);
#pragma unroll
      for (int t = 0; t < kMaxTermsPerLaunch; ++t)
        if (t < nt) acc[t] += (__popcll(u & zt.z[t]) & 1) ? -p : p;
    } else {
      const uint64_t i = insert0(u, top);
      const uint64_t j = i ^ x;
      const cpx<T> a = psi[i], b = psi[j];
      // w = conj(b) * a
      const double wr = fma((double)b.x, (double)a.x, (double)b.y * (double)a.y);
      const double wi = fma((double)b.x, (double)a.y, -(double)b.y * (double)a.x);
#pragma unroll
      for (int t = 0; t < kMaxTermsPerLaunch; ++t)
        if (t < nt) {
          const double w = zt.odd[t] ? wi : wr;
          acc[t] += (__popcll(i & zt.z[t]) & 1) ? -w : w;
        }
    }
  }
  for (int t = 0; t < nt; ++t) {
    const double s = block_sum(acc[t], sh);
    if (threadIdx.x == 0) part[(size_t)blockIdx.x * nt + t] = s;
  }
}

// ------------------------------------------------- X-mask terms by tiles
// Terms whose X masks lie in a set S of at most TB qubits (the low c qubits
// always included, so that the tile is read as contiguous segments) are
// reduced from one read of the state: each workgroup stages a tile (the 2^t
// amplitudes with fixed non-S bits) in LDS and evaluates every term on it.
// Per term this is the same sum as k_expval_part over i with bit top(x) = 0
// of (-1)^{|i & z|} conj(psi_{i^x}) psi_i (real or imaginary part), taken
// tile by tile; the sign splits into the tile's outside bits and its local
// bits.
struct XTileDesc {
  int t, c, nns;
  int S[16];      // tile qubits, ascending (S[j] = local bit j)
  int nonS[48];   // other qubits, ascending
};
struct XTileTerms {
  uint64_t z[kMaxTermsPerLaunch];     // global Z masks (outside bits give the tile parity)
  uint32_t x[kMaxTermsPerLaunch];     // local X masks
  uint32_t zloc[kMaxTermsPerLaunch];  // local Z masks
  int top[kMaxTermsPerLaunch];        // local position of the highest X bit
  int odd[kMaxTermsPerLaunch];        // imaginary part (odd number of Y)
};

template <typename T, int TB>
__global__ __launch_bounds__(kRB) void k_expval_tile(const cpx<T>* __restrict__ psi, XTileDesc d,
                                                     XTileTerms tt, int nt, uint64_t ntiles,
                                                     double* __restrict__ part) {
  __shared__ cpx<T> tile[1 << TB];
  __shared__ uint64_t segoff[256];
  __shared__ double sh[kRB];
  constexpr int A = VecInfo<T>::A;
  const int t = d.t, c = d.c;
  const int nseg = 1 << (t - c);
  for (int h = threadIdx.x; h < nseg; h += kRB) {
    uint64_t o = 0;
    for (int j = 0; j < t - c; ++j)
      if ((h >> j) & 1) o |= 1ull << d.S[c + j];
    segoff[h] = o;
  }
  double acc[kMaxTermsPerLaunch];
#pragma unroll
  for (int k = 0; k < kMaxTermsPerLaunch; ++k) acc[k] = 0.0;
  const vec16<T>* gv = reinterpret_cast<const vec16<T>*>(psi);
  const int nvec = (1 << t) / A;
  const uint32_t cmask = (1u << c) - 1u;
  const int half = 1 << (t - 1);
  __syncthreads();
  for (uint64_t tid = blockIdx.x; tid < ntiles; tid += gridDim.x) {
    uint64_t base = 0;
    for (int i = 0; i < d.nns; ++i) base |= ((tid >> i) & 1ull) << d.nonS[i];
    for (int i = threadIdx.x; i < nvec; i += kRB) {
      const uint32_t l = (uint32_t)i * A;
      const uint64_t g = base | segoff[l >> c] | (l & cmask);
      const vec16<T> x = gv[g / A];
#pragma unroll
      for (int e = 0; e < A; ++e) tile[l + e] = x.a[e];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kMaxTermsPerLaunch; ++k) {
      if (k < nt) {
        const int pb = __popcll(base & tt.z[k]) & 1;
        const uint32_t xm = tt.x[k], zl = tt.zloc[k];
        const int top = tt.top[k];
        const uint32_t lowm = (1u << top) - 1u;
        for (int u = threadIdx.x; u < half; u += kRB) {
          const uint32_t l = (((uint32_t)u >> top) << (top + 1)) | ((uint32_t)u & lowm);
          const cpx<T> a = tile[l], b = tile[l ^ xm];
          const double wr = fma((double)b.x, (double)a.x, (double)b.y * (double)a.y);
          const double wi = fma((double)b.x, (double)a.y, -(double)b.y * (double)a.x);
          const double w = tt.odd[k] ? wi : wr;
          acc[k] += ((__popc(l & zl) ^ pb) & 1) ? -w : w;
        }
      }
    }
    __syncthreads();
  }
  for (int k = 0; k < nt; ++k) {
    const double r = block_sum(acc[k], sh);
    if (threadIdx.x == 0) part[(size_t)blockIdx.x * nt + k] = r;
  }
}

template <typename T>
int xtile_max_bits();

// ------------------------------- one-qubit X / Y terms by register rounds
// Terms whose X mask is a single tile qubit (X_q or Y_q times any Z string,
// the common shape of a Hamiltonian's transverse terms) are evaluated on
// register groups, like the rounds of a tile pass: the tile is staged in LDS
// (XOR-swizzled), and in round r every thread gathers the 2^RB amplitudes
// that differ in the round's register bits (one XOR per amplitude, Gray
// order).  A term on register bit j then sums its 2^(RB-1) pairs
// w = conj(psi_{i^x}) psi_i (real or imaginary part) from registers; its Z
// string may not touch the round's register bits, so the sign
// (-1)^{|i & z|} is the parity of the group's free bits times that of the
// tile's outside qubits.  The pair products of one group are summed in the
// state's precision (2^(RB-1) of them), the groups in FP64.
constexpr int kMaxXRounds = 4;
constexpr int kMaxXSlots = kMaxXRounds * 5;  // one term per (round, register bit)
struct XRegDesc {
  int t, c, nns, nrounds;
  int S[16];
  int nonS[48];
  uint32_t free_mask[kMaxXRounds];
  uint32_t bofs[kMaxXRounds][5];  // swizzled LDS byte offsets of the register bits
};
struct XRegTerms {                   // per slot r * RB + j (X on register bit j of round r)
  uint64_t zout[kMaxXSlots];         // Z mask on the qubits outside the tile
  uint32_t zloc[kMaxXSlots];         // Z mask on the tile's free bits of the round (a parity)
  int term[kMaxXSlots];              // output index, -1 for an empty slot
};

template <typename T, int RB, int J, bool ODD>
__device__ __forceinline__ T pair_sum(const cpx<T> (&a)[1 << RB]) {
  T s = T(0);
#pragma unroll
  for (int l = 0; l < (1 << RB); ++l) {
    if ((l >> J) & 1) continue;
    const cpx<T> x = a[l], b = a[l | (1 << J)];
    s += ODD ? fma(b.x, x.y, -b.y * x.x) : fma(b.x, x.x, b.y * x.y);
  }
  return s;
}

// rounds unrolled (at most kMaxXRounds) so that every slot index is static;
// ODD: every term of the launch takes the imaginary part (one Y)
template <typename T, int RB, bool ODD, int R>
__device__ __forceinline__ void xreg_round(const char* __restrict__ tb, const XRegDesc& d,
                                           const XRegTerms& tt, uint64_t base, double (&acc)[kMaxXSlots]) {
  constexpr int NR = 1 << RB;
  constexpr int SB = sizeof(T) == 4 ? 5 : 4;
  if (R >= d.nrounds) return;
  const int ng = 1 << (d.t - RB);
  const uint32_t free_mask = d.free_mask[R];
  for (int gi = threadIdx.x; gi < ng; gi += kRB) {
    uint32_t lg = 0, fm = free_mask;
    for (int bit = 0; fm; ++bit) {
      const uint32_t low = fm & (0u - fm);
      if ((gi >> bit) & 1) lg |= low;
      fm ^= low;
    }
    cpx<T> a[NR];
    uint32_t ad = tile_swizzle(lg, SB) * (uint32_t)sizeof(cpx<T>);
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      if (i > 0) ad ^= d.bofs[R][__builtin_ctz(i)];
      a[i ^ (i >> 1)] = *reinterpret_cast<const cpx<T>*>(tb + ad);
    }
#define QSV_XSLOT(J)                                                                         \
  if ((J) < RB && tt.term[R * RB + (J)] >= 0) {                                              \
    constexpr int JJ = (J) < RB ? (J) : 0;                                                    \
    const int k = R * RB + JJ;                                                               \
    const T s = pair_sum<T, RB, JJ, ODD>(a);                                                 \
    const int par = (__popc(lg & tt.zloc[k]) + __popcll(base & tt.zout[k])) & 1;             \
    acc[k] += par ? -(double)s : (double)s;                                                  \
  }
    QSV_XSLOT(0)
    QSV_XSLOT(1)
    QSV_XSLOT(2)
    QSV_XSLOT(3)
    QSV_XSLOT(4)
#undef QSV_XSLOT
  }
}

__device__ __forceinline__ uint64_t xreg_tile_base(const XRegDesc& d, uint64_t id) {
  uint64_t b = 0;
  for (int i = 0; i < d.nns; ++i) b |= ((id >> i) & 1ull) << d.nonS[i];
  return b;
}

// this thread's vectors of the tile with base index b, into registers
template <typename T, int NV>
__device__ __forceinline__ void xreg_fetch(vec16<T> (&stage)[NV], const vec16<T>* __restrict__ gv, uint64_t b,
                                           const uint64_t* segoff, int c, uint32_t cmask, int nvec) {
  constexpr int A = VecInfo<T>::A;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int i = (int)threadIdx.x + v * kRB;
    if (i < nvec) {
      const uint32_t l = (uint32_t)i * A;
      stage[v] = gv[(b | segoff[l >> c] | (l & cmask)) / A];
    }
  }
}

template <typename T, int TB, int RB, bool ODD>
__global__ __launch_bounds__(kRB) void k_expval_xreg(const cpx<T>* __restrict__ psi, XRegDesc d,
                                                     XRegTerms tt, int nt, uint64_t ntiles,
                                                     double* __restrict__ part) {
  constexpr int A = VecInfo<T>::A;
  constexpr int SB = sizeof(T) == 4 ? 5 : 4;
  __shared__ cpx<T> tile[1 << TB];
  __shared__ uint64_t segoff[256];
  __shared__ double sh[kRB];
  const int t = d.t, c = d.c;
  const int nseg = 1 << (t - c);
  for (int h = threadIdx.x; h < nseg; h += kRB) {
    uint64_t o = 0;
    for (int j = 0; j < t - c; ++j)
      if ((h >> j) & 1) o |= 1ull << d.S[c + j];
    segoff[h] = o;
  }
  double acc[kMaxXSlots];
#pragma unroll
  for (int k = 0; k < kMaxXSlots; ++k) acc[k] = 0.0;
  const vec16<T>* gv = reinterpret_cast<const vec16<T>*>(psi);
  const int nvec = (1 << t) / A;
  const uint32_t cmask = (1u << c) - 1u;
  const char* tb = reinterpret_cast<const char*>(tile);
  __syncthreads();
  // Software pipeline: the next tile's vectors are loaded into registers
  // while the rounds of the current one run, so HBM reads overlap the math
  // (complex64 only: the complex128 variant's staging array went to scratch)
  constexpr bool PIPE = sizeof(T) == 4;
  constexpr int NV = PIPE ? (1 << TB) / A / kRB : 1;  // vectors per thread of a full tile
  vec16<T> stage[NV];
  if (PIPE && (uint64_t)blockIdx.x < ntiles)
    xreg_fetch<T, NV>(stage, gv, xreg_tile_base(d, blockIdx.x), segoff, c, cmask, nvec);
  for (uint64_t tid = blockIdx.x; tid < ntiles; tid += gridDim.x) {
    const uint64_t base = xreg_tile_base(d, tid);
    if constexpr (PIPE) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int i = (int)threadIdx.x + v * kRB;
        if (i < nvec) {
          const uint32_t l = (uint32_t)i * A;
#pragma unroll
          for (int e = 0; e < A; ++e) tile[tile_swizzle(l + e, SB)] = stage[v].a[e];
        }
      }
    } else {
      for (int i = threadIdx.x; i < nvec; i += kRB) {
        const uint32_t l = (uint32_t)i * A;
        const vec16<T> x = gv[(base | segoff[l >> c] | (l & cmask)) / A];
#pragma unroll
        for (int e = 0; e < A; ++e) tile[tile_swizzle(l + e, SB)] = x.a[e];
      }
    }
    __syncthreads();
    if (PIPE && tid + gridDim.x < ntiles)
      xreg_fetch<T, NV>(stage, gv, xreg_tile_base(d, tid + gridDim.x), segoff, c, cmask, nvec);
    // (the empty asm keeps the compiler from hoisting the LDS gathers of all
    // rounds together, which would hold every round's amplitudes at once)
    xreg_round<T, RB, ODD, 0>(tb, d, tt, base, acc);
    asm volatile("" ::: "memory");
    xreg_round<T, RB, ODD, 1>(tb, d, tt, base, acc);
    asm volatile("" ::: "memory");
    xreg_round<T, RB, ODD, 2>(tb, d, tt, base, acc);
    asm volatile("" ::: "memory");
    xreg_round<T, RB, ODD, 3>(tb, d, tt, base, acc);
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < kMaxXSlots; ++k) {
    if (k < kMaxXRounds * RB && tt.term[k] >= 0) {
      const double v = block_sum(acc[k], sh);
      if (threadIdx.x == 0) part[(size_t)blockIdx.x * nt + tt.term[k]] = v;
    }
  }
}

// The same values as launch_expval_tile for nt <= 16 terms whose X masks are
// distinct single qubits of the tile S, all with an even or all with an odd
// number of Y: rounds of RB register bits cover the terms' X qubits (filled
// up with other tile qubits), at most kMaxXRounds.  Returns
// hipErrorInvalidValue, launching nothing, for terms outside that shape
// (or with Z on a register bit of their round).
template <typename T>
hipError_t launch_expval_xreg(const cpx<T>* psi, int n, const int* S, int t, int c, const uint64_t* xmask,
                              const uint64_t* zmask, const int* ny, int nt, double* ws, double* out_dev,
                              hipStream_t st) {
  constexpr int RB = sizeof(T) == 4 ? 5 : 4;
  constexpr int NR = 1 << RB;
  constexpr int SB = sizeof(T) == 4 ? 5 : 4;
  if (nt < 1 || nt > kMaxTermsPerLaunch || t < RB || t > xtile_max_bits<T>() || c > t || t - c > 8 ||
      (1 << c) < VecInfo<T>::A)
    return hipErrorInvalidValue;
  XRegDesc d{};
  d.t = t;
  d.c = c;
  int pos[64];
  for (int q = 0; q < 64; ++q) pos[q] = -1;
  uint64_t Smask = 0;
  for (int j = 0; j < t; ++j) {
    d.S[j] = S[j];
    pos[S[j]] = j;
    Smask |= 1ull << S[j];
  }
  for (int q = 0; q < n; ++q)
    if (!((Smask >> q) & 1)) d.nonS[d.nns++] = q;
  // rounds: the distinct X bits (local positions), RB to a round, filled up
  std::vector<int> xb;
  for (int k = 0; k < nt; ++k) {
    if (xmask[k] == 0 || (xmask[k] & (xmask[k] - 1)) || (xmask[k] & ~Smask)) return hipErrorInvalidValue;
    const int p = pos[__builtin_ctzll(xmask[k])];
    if (std::find(xb.begin(), xb.end(), p) == xb.end()) xb.push_back(p);
  }
  d.nrounds = (int)((xb.size() + RB - 1) / RB);
  if (d.nrounds > kMaxXRounds) return hipErrorInvalidValue;
  std::vector<std::vector<int>> R(d.nrounds);
  for (size_t i = 0; i < xb.size(); ++i) R[i / RB].push_back(xb[i]);
  for (auto& reg : R) {
    for (int p = 0; p < t && (int)reg.size() < RB; ++p)
      if (std::find(reg.begin(), reg.end(), p) == reg.end()) reg.push_back(p);
    std::sort(reg.begin(), reg.end());
  }
  const uint32_t tmask = (1u << t) - 1u;
  for (int r = 0; r < d.nrounds; ++r) {
    uint32_t rm = 0;
    for (int k = 0; k < RB; ++k) {
      rm |= 1u << R[r][k];
      d.bofs[r][k] = tile_swizzle(1u << R[r][k], SB) * (uint32_t)sizeof(cpx<T>);
    }
    d.free_mask[r] = tmask & ~rm;
  }
  XRegTerms tt{};
  for (int k = 0; k < kMaxXSlots; ++k) tt.term[k] = -1;
  for (int k = 0; k < nt; ++k) {
    const int p = pos[__builtin_ctzll(xmask[k])];
    int slot = -1, rr = 0;
    for (int r = 0; r < d.nrounds; ++r)
      for (int j = 0; j < RB; ++j)
        if (R[r][j] == p) {
          slot = r * RB + j;
          rr = r;
        }
    if (slot < 0 || tt.term[slot] >= 0) return hipErrorInvalidValue;  // one term per qubit
    uint32_t zl = 0;
    for (int q = 0; q < n; ++q)
      if (((zmask[k] >> q) & 1) && pos[q] >= 0) zl |= 1u << pos[q];
    uint32_t rm = 0;
    for (int j = 0; j < RB; ++j) rm |= 1u << R[rr][j];
    if (zl & rm) return hipErrorInvalidValue;                      // Z on a register bit of its round
    if ((ny[k] & 1) != (ny[0] & 1)) return hipErrorInvalidValue;  // one parity of Y per launch
    tt.term[slot] = k;
    tt.zout[slot] = zmask[k] & ~Smask;
    tt.zloc[slot] = zl;
  }
  const uint64_t ntiles = 1ull << (n - t);
  const unsigned g = (unsigned)(ntiles < (uint64_t)kMaxPartials ? ntiles : (uint64_t)kMaxPartials);
  constexpr int TB = sizeof(T) == 4 ? 13 : 12;
  if (ny[0] & 1)
    hipLaunchKernelGGL((k_expval_xreg<T, TB, RB, true>), dim3(g), dim3(kRB), 0, st, psi, d, tt, nt, ntiles, ws);
  else
    hipLaunchKernelGGL((k_expval_xreg<T, TB, RB, false>), dim3(g), dim3(kRB), 0, st, psi, d, tt, nt, ntiles, ws);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kRB), 0, st, ws, (int)g, nt, out_dev);
  return hipGetLastError();
}

template <typename T>
int xtile_max_bits() {
  return sizeof(T) == 4 ? 13 : 12;
}
template <typename T>
int xtile_low_bits() {
  return sizeof(T) == 4 ? 5 : 4;
}

// out_dev[k] for terms k < nt (nt <= kMaxTermsPerLaunch) whose X masks lie in
// the tile qubits S (ascending, S[0..c) = 0..c-1); same values as
// launch_expval_group for each term.
template <typename T>
hipError_t launch_expval_tile(const cpx<T>* psi, int n, const int* S, int t, int c,
                              const uint64_t* xmask, const uint64_t* zmask, const int* ny, int nt,
                              double* ws, double* out_dev, hipStream_t st) {
  if (nt < 1 || nt > kMaxTermsPerLaunch || t < 1 || t > xtile_max_bits<T>() || c > t || t - c > 8 ||
      (1 << c) < VecInfo<T>::A)
    return hipErrorInvalidValue;
  XTileDesc d{};
  d.t = t;
  d.c = c;
  int pos[64];
  for (int q = 0; q < 64; ++q) pos[q] = -1;
  uint64_t Smask = 0;
  for (int j = 0; j < t; ++j) {
    d.S[j] = S[j];
    pos[S[j]] = j;
    Smask |= 1ull << S[j];
  }
  for (int q = 0; q < n; ++q)
    if (!((Smask >> q) & 1)) d.nonS[d.nns++] = q;
  XTileTerms tt{};
  auto compress = [&](uint64_t m) {
    uint32_t r = 0;
    for (int q = 0; q < n; ++q)
      if (((m >> q) & 1) && pos[q] >= 0) r |= 1u << pos[q];
    return r;
  };
  for (int k = 0; k < nt; ++k) {
    if (xmask[k] == 0 || (xmask[k] & ~Smask)) return hipErrorInvalidValue;
    tt.x[k] = compress(xmask[k]);
    tt.zloc[k] = compress(zmask[k]);
    tt.z[k] = zmask[k] & ~Smask;
    tt.top[k] = 31 - __builtin_clz(tt.x[k]);
    tt.odd[k] = ny[k] & 1;
  }
  const uint64_t ntiles = 1ull << (n - t);
  const unsigned g = (unsigned)(ntiles < (uint64_t)kMaxPartials ? ntiles : (uint64_t)kMaxPartials);
  if (sizeof(T) == 4)
    hipLaunchKernelGGL((k_expval_tile<T, 13>), dim3(g), dim3(kRB), 0, st, psi, d, tt, nt, ntiles, ws);
  else
    hipLaunchKernelGGL((k_expval_tile<T, 12>), dim3(g), dim3(kRB), 0, st, psi, d, tt, nt, ntiles, ws);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kRB), 0, st, ws, (int)g, nt, out_dev);
  return hipGetLastError();
}

size_t expval_ws_doubles(int n, int nt) {
  (void)n;
  return (size_t)kMaxPartials * (nt < 1 ? 1 : nt);
}

template <typename T>
hipError_t launch_expval_group(const cpx<T>* psi, int n, uint64_t xmask, int nt,
                               const uint64_t* zmask_host, const int* ny_host, double* ws,
                               double* out_dev, hipStream_t st) {
  for (int t0 = 0; t0 < nt; t0 += kMaxTermsPerLaunch) {
    const int cnt = nt - t0 < kMaxTermsPerLaunch ? nt - t0 : kMaxTermsPerLaunch;
    ZTerms zt{};
    for (int t = 0; t < cnt; ++t) {
      zt.z[t] = zmask_host[t0 + t];
      zt.odd[t] = ny_host[t0 + t] & 1;
    }
    const uint64_t N = 1ull << n;
    if (xmask == 0) {
      const unsigned g = reduce_grid(N);
      const uint64_t chunk = (N + g - 1) / g;
      hipLaunchKernelGGL((k_expval_part<T, true>), dim3(g), dim3(kRB), 0, st, psi, N, chunk,
                         xmask, 0, cnt, zt, ws);
      hipLaunchKernelGGL(k_final, dim3(1), dim3(kRB), 0, st, ws, (int)g, cnt, out_dev + t0);
    } else {
      const int top = 63 - __builtin_clzll(xmask);
      const uint64_t units = N / 2;
      const unsigned g = reduce_grid(units);
      const uint64_t chunk = (units + g - 1) / g;
      hipLaunchKernelGGL((k_expval_part<T, false>), dim3(g), dim3(kRB), 0, st, psi, units, chunk,
                         xmask, top, cnt, zt, ws);
      hipLaunchKernelGGL(k_final, dim3(1), dim3(kRB), 0, st, ws, (int)g, cnt, out_dev + t0);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ------------------------------------------- Z-only terms, register sums
// All Z strings of one launch from one read of the state.  A wavefront reads
// a unit of 64 x 16 coalesced 16-byte vectors; lane l takes vectors
// l + 64 k (k < 16), so the NR = 16 A amplitudes a thread holds differ
// exactly in the index bits {0} + {7..10} (complex64, A = 2) or {6..9}
// (complex128, A = 1), the register bits.  The sign of a term with Z mask z
// splits into (-1)^{|r & z_r|} for register combination r (z_r: z on the
// register bits) and (-1)^{|i0 & z_hi|} for the thread's index i0 with the
// register bits clear.  With the probabilities p_r in FP64, their
// Walsh-Hadamard transform W_s = sum_r (-1)^{|r & s|} p_r (NR log NR adds)
// gives every term's register sum at once: a term costs one read of
// W_{z_r} and one signed add per thread.
constexpr int kMaxZTerms = 32;
struct ZRegTerms {
  uint64_t zhi[kMaxZTerms];
  int zr[kMaxZTerms];        // z on the register bits, as a register combination
};

template <typename T>
struct ZRegCfg;
template <>
struct ZRegCfg<float> {
  static constexpr int NR = 32;                  // amplitudes per thread
  static constexpr uint64_t RMASK = 0x781ull;    // index bits {0, 7, 8, 9, 10}
  static constexpr int UNIT_BITS = 11;           // amplitudes per wavefront unit: 2^11
};
template <>
struct ZRegCfg<double> {
  static constexpr int NR = 16;
  static constexpr uint64_t RMASK = 0x3c0ull;    // index bits {6, 7, 8, 9}
  static constexpr int UNIT_BITS = 10;
};

template <typename T>
__global__ __launch_bounds__(kRB) void k_expval_zreg(const vec16<T>* __restrict__ v, uint64_t nunits,
                                                      ZRegTerms wt, int nt, double* __restrict__ part) {
  constexpr int A = VecInfo<T>::A;
  constexpr int NR = ZRegCfg<T>::NR;
  constexpr int VPT = NR / A;  // 16 vectors per thread
  __shared__ double sh[kRB];
  __shared__ double wcol[NR * kRB];  // thread-private columns: [s][thread], conflict-free
  double acc[kMaxZTerms];
#pragma unroll
  for (int t = 0; t < kMaxZTerms; ++t) acc[t] = 0.0;
  const int lane = threadIdx.x & 63;
  const uint64_t wid = ((uint64_t)blockIdx.x * kRB + threadIdx.x) >> 6;
  const uint64_t nw = ((uint64_t)gridDim.x * kRB) >> 6;
  for (uint64_t u = wid; u < nunits; u += nw) {
    const uint64_t v0 = u * 64 * VPT + lane;
    double p[NR];
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
      const vec16<T> x = v[v0 + 64 * k];
#pragma unroll
      for (int e = 0; e < A; ++e) {
        const double re = (double)x.a[e].x, im = (double)x.a[e].y;
        p[e + A * k] = fma(re, re, im * im);
      }
    }
    // Walsh-Hadamard transform in registers: p[s] = sum_r (-1)^{|r & s|} p_r
#pragma unroll
    for (int h = 1; h < NR; h <<= 1)
#pragma unroll
      for (int r = 0; r < NR; ++r)
        if (!(r & h)) {
          const double x = p[r], y = p[r | h];
          p[r] = x + y;
          p[r | h] = x - y;
        }
    // each term needs the coefficient at its own (uniform) register mask: a
    // dynamic index, taken from this thread's column in LDS rather than from
    // registers (which would put the array in scratch memory)
#pragma unroll
    for (int s = 0; s < NR; ++s) wcol[s * kRB + threadIdx.x] = p[s];
    const uint64_t i0 = v0 * A;  // index of (lane, k = 0, e = 0): register bits clear
#pragma unroll
    for (int t = 0; t < kMaxZTerms; ++t) {
      if (t < nt) {
        const double w = wcol[wt.zr[t] * kRB + threadIdx.x];
        acc[t] += (__popcll(i0 & wt.zhi[t]) & 1) ? -w : w;
      }
    }
  }
#pragma unroll
  for (int t = 0; t < kMaxZTerms; ++t) {
    if (t < nt) {  // static indices keep acc in registers
      const double s = block_sum(acc[t], sh);
      if (threadIdx.x == 0) part[(size_t)blockIdx.x * nt + t] = s;
    }
  }
}

template <typename T>
int zreg_min_qubits() {
  return ZRegCfg<T>::UNIT_BITS;
}

// out_dev[t] = sum_i (-1)^{|i & z_t|} |psi_i|^2 for nt <= kMaxZTerms Z masks;
// needs 2^n >= one unit (n >= 11 complex64, n >= 10 complex128).
template <typename T>
hipError_t launch_expval_zreg(const cpx<T>* psi, int n, const uint64_t* zmask, int nt, double* ws,
                               double* out_dev, hipStream_t st) {
  constexpr uint64_t RM = ZRegCfg<T>::RMASK;
  if (nt < 1 || nt > kMaxZTerms || n < ZRegCfg<T>::UNIT_BITS || n > 62) return hipErrorInvalidValue;
  ZRegTerms wt{};
  for (int t = 0; t < nt; ++t) {
    wt.zhi[t] = zmask[t] & ~RM;
    int zr = 0, k = 0;
    for (int q = 0; q < 64; ++q)
      if ((RM >> q) & 1) {
        if ((zmask[t] >> q) & 1) zr |= 1 << k;
        ++k;
      }
    wt.zr[t] = zr;
  }
  const uint64_t nunits = 1ull << (n - ZRegCfg<T>::UNIT_BITS);
  uint64_t g = (nunits + 3) / 4;  // four wavefronts per workgroup
  if (g > kMaxPartials) g = kMaxPartials;
  hipLaunchKernelGGL(k_expval_zreg<T>, dim3((unsigned)g), dim3(kRB), 0, st,
                     reinterpret_cast<const vec16<T>*>(psi), nunits, wt, nt, ws);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kRB), 0, st, ws, (int)g, nt, out_dev);
  return hipGetLastError();
}

// ---------------------------------------------------------------- sampling
// Block sums of |psi_i|^2 over blocks of kSB amplitudes, their inclusive
// prefix, then one wavefront per shot: binary search over the block prefix
// for the first block whose inclusive prefix exceeds t = u * total, and an
// in-block scan (64 lanes x kSB/64 consecutive amplitudes).
constexpr int kSB = 4096;

template <typename T>
__global__ __launch_bounds__(kRB) void k_block_sums(const cpx<T>* __restrict__ psi, uint64_t N,
                                                    double* __restrict__ bsum) {
  // block b = amplitudes [b kSB, (b + 1) kSB), read as coalesced 16-byte
  // vectors (thread t takes vectors t, t + kRB, ...); the order of the sum
  // inside a block is free: the shot rescan recomputes its own running sum
  __shared__ double sh[kRB];
  constexpr int A = VecInfo<T>::A;
  const vec16<T>* v = reinterpret_cast<const vec16<T>*>(psi);
  const uint64_t nvec = N / A, v0 = (uint64_t)blockIdx.x * (kSB / A);
  double acc = 0.0;
#pragma unroll
  for (int e = 0; e < kSB / A / kRB; ++e) {
    const uint64_t i = v0 + (uint64_t)e * kRB + threadIdx.x;
    if (i < nvec) {
      const vec16<T> x = v[i];
#pragma unroll
      for (int q = 0; q < A; ++q)
        acc += fma((double)x.a[q].x, (double)x.a[q].x, (double)x.a[q].y * (double)x.a[q].y);
    }
  }
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) bsum[blockIdx.x] = r;
}

// inclusive prefix of nb block sums, one workgroup: contiguous chunks per
// thread, sequential within the chunk, then a sequential pass over chunk totals
__global__ __launch_bounds__(kRB) void k_block_prefix(const double* __restrict__ bsum, uint64_t nb,
                                                      double* __restrict__ pref) {
  __shared__ double tot[kRB];
  const uint64_t per = (nb + kRB - 1) / kRB;
  const uint64_t lo = threadIdx.x * per;
  const uint64_t hi = lo + per < nb ? lo + per : nb;
  double acc = 0.0;
  for (uint64_t b = lo; b < hi; ++b) acc += bsum[b];
  tot[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double run = 0.0;
    for (int t = 0; t < kRB; ++t) {
      const double v = tot[t];
      tot[t] = run;
      run += v;
    }
  }
  __syncthreads();
  double run = tot[threadIdx.x];
  for (uint64_t b = lo; b < hi; ++b) {
    run += bsum[b];
    pref[b] = run;
  }
}

template <typename T>
__global__ __launch_bounds__(kRB) void k_sample_shots(const cpx<T>* __restrict__ psi, uint64_t N,
                                                      const double* __restrict__ bsum,
                                                      const double* __restrict__ pref, uint64_t nb,
                                                      const double* __restrict__ uni, int shots,
                                                      uint64_t* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int shot = blockIdx.x * (kRB / 64) + (threadIdx.x >> 6);
  if (shot >= shots) return;  // whole wavefront exits together
  const double total = pref[nb - 1];
  const double t = uni[shot] * total;
  // smallest block b with pref[b] > t
  uint64_t lo = 0, hi = nb;
  while (lo < hi) {
    const uint64_t mid = lo + (hi - lo) / 2;
    if (pref[mid] > t) hi = mid; else lo = mid + 1;
  }
  bool clamp = false;
  uint64_t b = lo;
  if (b >= nb) {  // rounding left no block above t: last block with mass
    clamp = true;
    b = nb - 1;
    while (b > 0 && !(bsum[b] > 0.0)) --b;
  }
  const double base = b == 0 ? 0.0 : pref[b - 1];
  constexpr int per = kSB / 64;
  const uint64_t s = b * (uint64_t)kSB + (uint64_t)lane * per;
  double ls = 0.0;
  for (int e = 0; e < per; ++e) {
    const uint64_t i = s + e;
    if (i < N) {
      const cpx<T> a = psi[i];
      ls += fma((double)a.x, (double)a.x, (double)a.y * (double)a.y);
    }
  }
  // inclusive scan over lanes
  double inc = ls;
  for (int d = 1; d < 64; d <<= 1) {
    const double o = __shfl_up(inc, d, 64);
    if (lane >= d) inc += o;
  }
  const double exc = inc - ls;
  const uint64_t hit = clamp ? 0ull : (uint64_t)__ballot(base + inc > t);
  // last index with nonzero probability in this block (clamp fallback)
  uint64_t lastnz = 0;
  bool any = false;
  for (int e = 0; e < per; ++e) {
    const uint64_t i = s + e;
    if (i < N) {
      const cpx<T> a = psi[i];
      if (a.x != T(0) || a.y != T(0)) { lastnz = i; any = true; }
    }
  }
  const uint64_t nzmask = (uint64_t)__ballot(any);
  uint64_t res;
  if (hit) {
    const int L = __ffsll((unsigned long long)hit) - 1;
    // lane L walks its run sequentially
    uint64_t found = ~0ull;
    if (lane == L) {
      double run = base + exc;
      for (int e = 0; e < per; ++e) {
        const uint64_t i = s + e;
        if (i >= N) break;
        const cpx<T> a = psi[i];
        run += fma((double)a.x, (double)a.x, (double)a.y * (double)a.y);
        if (run > t) { found = i; break; }
      }
      if (found == ~0ull) found = any ? lastnz : s;
    }
    res = __shfl(found, L, 64);
  } else {
    const int L = nzmask ? 63 - __clzll((long long)nzmask) : 0;
    res = __shfl(lastnz, L, 64);
  }
  if (lane == 0) out[shot] = res;
}

size_t sample_ws_doubles(int n) {
  const uint64_t N = 1ull << n;
  const uint64_t nb = (N + kSB - 1) / kSB;
  return 2 * nb;
}

template <typename T>
hipError_t launch_sample(const cpx<T>* psi, int n, const double* uniforms_dev, int shots,
                         double* ws, uint64_t* out_dev, hipStream_t st) {
  const uint64_t N = 1ull << n;
  const uint64_t nb = (N + kSB - 1) / kSB;
  double* bsum = ws;
  double* pref = ws + nb;
  hipLaunchKernelGGL(k_block_sums<T>, dim3((unsigned)nb), dim3(kRB), 0, st, psi, N, bsum);
  hipLaunchKernelGGL(k_block_prefix, dim3(1), dim3(kRB), 0, st, bsum, nb, pref);
  if (shots > 0) {
    const unsigned g = (unsigned)((shots + (kRB / 64) - 1) / (kRB / 64));
    hipLaunchKernelGGL(k_sample_shots<T>, dim3(g), dim3(kRB), 0, st, psi, N, bsum, pref, nb,
                       uniforms_dev, shots, out_dev);
  }
  return hipGetLastError();
}

#define QSV_RINST(T)                                                                          \
  template hipError_t launch_norm<T>(const cpx<T>*, uint64_t, double*, double*, hipStream_t); \
  template hipError_t launch_expval_group<T>(const cpx<T>*, int, uint64_t, int, const uint64_t*, \
                                             const int*, double*, double*, hipStream_t);      \
  template hipError_t launch_sample<T>(const cpx<T>*, int, const double*, int, double*,       \
                                       uint64_t*, hipStream_t);                                   \
  template hipError_t launch_expval_zreg<T>(const cpx<T>*, int, const uint64_t*, int, double*,   \
                                            double*, hipStream_t);                                \
  template int zreg_min_qubits<T>();                                                             \
  template hipError_t launch_expval_xreg<T>(const cpx<T>*, int, const int*, int, int,             \
                                            const uint64_t*, const uint64_t*, const int*, int,    \
                                            double*, double*, hipStream_t);                       \
  template hipError_t launch_expval_tile<T>(const cpx<T>*, int, const int*, int, int,             \
                                            const uint64_t*, const uint64_t*, const int*, int,    \
                                            double*, double*, hipStream_t);                       \
  template int xtile_max_bits<T>();                                                              \
  template int xtile_low_bits<T>();
QSV_RINST(float)
QSV_RINST(double)

}  // namespace qsv
