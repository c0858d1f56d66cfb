// adjoint.hip -- reverse-mode gradients of <psi(theta)|H|psi(theta)>.
//
// For psi_L = U_L ... U_1 psi_0 and E = <psi_L|H|psi_L>, with every
// parameterised gate a rotation R_P(theta) = exp(-i theta P / 2), the
// derivative with respect to the angle of gate k is
//     dE/dtheta_k = Im <lambda_k| P |psi_k>,
// psi_k = U_k ... U_1 psi_0 and lambda_k = U_{k+1}^dag ... U_L^dag H psi_L.
// One reverse sweep yields every derivative: start from psi_L and
// lambda = H psi_L, and for k = L .. 1 accumulate the gradient of gate k,
// then apply U_k^dag to both states.  Here lambda = H psi is formed by tile
// passes (or by gathers for X masks wider than a tile), and the sweep runs
// as tile passes over both states in LDS that apply each pass's inverse
// gates and take every rotation's term on the way (states below five qubits
// use one kernel per rotation).  Gradients are accumulated in FP64 in a
// fixed order (no floating-point atomics).  (Not part of the paper, whose
// gradients are taken over tensor-network factors; it is the
// parameter-gradient of its VQE use case.)
#include <algorithm>

#include "internal.hpp"

namespace qsv {

constexpr int kAB = 256;
constexpr int kMaxAdjPartials = 1024;

__device__ __forceinline__ double block_sum_d(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = kAB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// ---------------------------------------------------------- lambda = H psi
// lambda_j = sum_t w_t (-1)^{|(j ^ x_t) & z_t|} psi_{j ^ x_t},  w_t = c_t i^{n_y}
constexpr int kMaxHTerms = 64;
struct HTerms {
  uint64_t x[kMaxHTerms];
  uint64_t z[kMaxHTerms];
  double wr[kMaxHTerms], wi[kMaxHTerms];
  int nt;
};

template <typename T>
__global__ __launch_bounds__(kAB) void k_hpsi(const cpx<T>* __restrict__ psi, cpx<T>* __restrict__ lam,
                                              uint64_t N, HTerms h, int accumulate) {
  const uint64_t j = block_index() * kAB + threadIdx.x;
  if (j >= N) return;
  double ar = 0.0, ai = 0.0;
  if (accumulate) {
    const cpx<T> l = lam[j];
    ar = (double)l.x;
    ai = (double)l.y;
  }
  int t = 0;
  while (t < h.nt) {
    const uint64_t x = h.x[t];
    const cpx<T> p = psi[j ^ x];
    const double pr = (double)p.x, pi = (double)p.y;
    for (; t < h.nt && h.x[t] == x; ++t) {
      const double s = (__popcll((j ^ x) & h.z[t]) & 1) ? -1.0 : 1.0;
      const double wr = s * h.wr[t], wi = s * h.wi[t];
      ar = fma(wr, pr, fma(-wi, pi, ar));
      ai = fma(wr, pi, fma(wi, pr, ai));
    }
  }
  lam[j] = cpx<T>{(T)ar, (T)ai};
}

// -------------------------------------- rotation: gradient + inverse update
// Per pair (i0, i1) on qubit q:  g += Im( conj(l0) (G00 p0 + G01 p1)
//                                        + conj(l1) (G10 p0 + G11 p1) )
// then (p0, p1) <- V (p0, p1), (l0, l1) <- V (l0, l1) with V = U^dag.
template <typename T>
__global__ __launch_bounds__(kAB) void k_adj_rot(cpx<T>* __restrict__ psi, cpx<T>* __restrict__ lam,
                                                 uint64_t pairs, uint64_t chunk, int q, M2<T> V,
                                                 M2<double> G, double* __restrict__ part) {
  __shared__ double sh[kAB];
  const uint64_t lo = (uint64_t)blockIdx.x * chunk;
  const uint64_t hi = lo + chunk < pairs ? lo + chunk : pairs;
  double acc = 0.0;
  for (uint64_t k = lo + threadIdx.x; k < hi; k += kAB) {
    const uint64_t i0 = insert0(k, q), i1 = i0 | (1ull << q);
    cpx<T> p0 = psi[i0], p1 = psi[i1], l0 = lam[i0], l1 = lam[i1];
    const cpx<double> P0{(double)p0.x, (double)p0.y}, P1{(double)p1.x, (double)p1.y};
    const cpx<double> g0 = cfma(G.m[1], P1, cmul(G.m[0], P0));
    const cpx<double> g1 = cfma(G.m[3], P1, cmul(G.m[2], P0));
    // Im(conj(l) g) = l.x g.y - l.y g.x
    acc += (double)l0.x * g0.y - (double)l0.y * g0.x + (double)l1.x * g1.y - (double)l1.y * g1.x;
    apply2(V, p0, p1);
    apply2(V, l0, l1);
    psi[i0] = p0;
    psi[i1] = p1;
    lam[i0] = l0;
    lam[i1] = l1;
  }
  const double s = block_sum_d(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kAB) void k_adj_final(const double* __restrict__ part, int nb,
                                                   double* __restrict__ out) {
  __shared__ double sh[kAB];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += kAB) acc += part[b];
  const double s = block_sum_d(acc, sh);
  if (threadIdx.x == 0) *out = s;
}

// ------------------------------------------ fused reverse sweep, by tiles
// The reverse sweep as tile passes: a workgroup stages the tile of both psi
// and lambda in LDS (the 2^t amplitudes with fixed non-S bits), applies
// every inverse gate of the pass to both in order, and at each rotation adds
// the tile's share of Im <lambda| P |psi> before applying the inverse.  A
// wavefront reduces its share (DPP steps) and adds it to its own LDS slot
// per rotation (no atomics: the order of every addition is fixed); at the
// end each workgroup writes its per-rotation sums, which one workgroup per
// rotation then adds in a fixed tree.  One HBM read and write of both
// states per pass instead of one per rotation.
//
// Program (int32 words): [0] t, [1] c, [2] n_nonS, [3] n_ops, [4] n_grad,
// [5] offset of the op records, [6] offset of the gradient map (the
// circuit's op index of each gradient slot), [7] the number of type-7
// records, S[t] from word 8, nonS after.
// Op record (kAdjRec words): [0] type, [1] a, [2] b, [3] gradient slot or
// -1, [4] generator (0 X, 1 Y, 2 Z), then complex doubles (re, im) from
// word 8:
//   1 U1  : 2x2 on local bit a (row-major)
//   2 DIAG: factor d[bit_a + 2 bit_b] per amplitude; operands a, b are
//           kind << 8 | value (kind 0: local bit, 2: qubit outside the tile),
//           b = -1 for one qubit (d[0], d[1]); a gradient slot takes Z on a
//   3 U2  : 4x4 on local bits a < b (a = LSB of the row index)
//   5 SIGNS: a run of CZ and Z gates as one sign pattern; [1] n_dist,
//           [2] n_lo, [3] n_oo, then from word 8: n_dist pairs (d, M),
//           n_lo pairs (local bit, outside qubit or -1), n_oo pairs of
//           outside qubits.  Amplitude l of the tile changes sign when
//           sum_d popc(l & (l >> d) & M) + popc(l & Mo) + c is odd, with Mo
//           the local bits whose partner is -1 or a qubit set in the tile's
//           base index and c the parity of the outside pairs with both
//           qubits set (a Z outside the tile is the pair (q, q))
//   6 ROUND: one-qubit gates on K local qubits applied in registers: each
//           thread holds the 2^K amplitudes of both states that differ in
//           those bits and applies every gate of the record to them in turn
//           (gates on different qubits commute, gates on one qubit keep
//           their order), taking each rotation's term first.  [2] the gate
//           count of each register bit, 8 bits per bit j from bit 8 j,
//           [1] 0, or the offset from the record of a sign block (a type-5
//           record of 8 + 2 (n_dist + n_lo + n_oo) words, padded to a
//           multiple of 8) applied to the amplitudes as they are loaded,
//           before the gates: a sign run that precedes the round,
//           [3] record length in words, [4 + j] local bit j (ascending),
//           gates from word 8 ordered by bit, kAdjGate words each:
//           [0] j | shape << 4 | generator << 8, [1] gradient slot or -1,
//           from word 4 the matrix (m00, m01, m10, m11 as re, im) in the
//           state's precision
//   7 TILE PHASE: a diagonal unitary diag(d[0], d[1]) on the qubit a
//           outside the tile (named gates only): one phase for the whole
//           tile, applied to both states by the tile's store; a gradient
//           slot takes Z on a (+-Im<lambda|psi> over the tile)
// Records of types 1-5 and 7 are kAdjRec words long.
constexpr int kAdjRec = 72;
constexpr int kAdjGate = 20;

// A 16-byte vector of amplitudes as a native vector type (kept in registers
// where an array of structs of amplitudes went to scratch memory).
template <typename T>
struct AdjVec;
template <>
struct AdjVec<float> {
  using V = float4;
  __device__ static cpx<float> at(const V& v, int e) { return e ? cpx<float>{v.z, v.w} : cpx<float>{v.x, v.y}; }
};
template <>
struct AdjVec<double> {
  using V = double2;
  __device__ static cpx<double> at(const V& v, int) { return cpx<double>{v.x, v.y}; }
};

template <typename T>
struct AdjRound {
  static constexpr int K = sizeof(T) == 4 ? 4 : 3;  // register bits per round
};
constexpr int kMaxAdjGrad = 256;

template <typename T>
__device__ __forceinline__ cpx<T> cpx_at(const int32_t* w, int e) {
  const double re = __hiloint2double(w[4 * e + 1], w[4 * e]);
  const double im = __hiloint2double(w[4 * e + 3], w[4 * e + 2]);
  return cpx<T>{(T)re, (T)im};
}

template <typename T>
__device__ __forceinline__ cpx<T> rec_cpx(const int32_t* r, int e) {
  return cpx_at<T>(r + 8, e);
}

// One DPP step of a sum: v + v taken from the lane that CTRL selects (both
// 32-bit halves moved with the same pattern)
template <int CTRL>
__device__ __forceinline__ double dpp_add(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return v + __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_d(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}

// Sum over the 64 lanes, the same in every lane (all lanes active): lane
// pairs, quads, then rows of 16 by DPP, and the four row sums in a fixed order
__device__ __forceinline__ double wave_sum_d(double v) {
  v = dpp_add<0xB1>(v);   // quad_perm [1,0,3,2]
  v = dpp_add<0x4E>(v);   // quad_perm [2,3,0,1]
  v = dpp_add<0x124>(v);  // row_ror 4
  v = dpp_add<0x128>(v);  // row_ror 8
  return (lane_d(v, 0) + lane_d(v, 16)) + (lane_d(v, 32) + lane_d(v, 48));
}

// Im( conj(l0) (G p)_0 + conj(l1) (G p)_1 ) for G = X, Y or Z: one pair's
// term, formed in the amplitudes' own precision and handed to the FP64 sums
template <typename T>
__device__ __forceinline__ double grad_pair(int gen, cpx<T> p0, cpx<T> p1, cpx<T> l0, cpx<T> l1) {
  T v;
  if (gen == 0)  // X: Im(conj(l0) p1 + conj(l1) p0)
    v = (l0.x * p1.y - l0.y * p1.x) + (l1.x * p0.y - l1.y * p0.x);
  else if (gen == 1)  // Y: -Re(conj(l0) p1) + Re(conj(l1) p0)
    v = (l1.x * p0.x + l1.y * p0.y) - (l0.x * p1.x + l0.y * p1.y);
  else  // Z
    v = (l0.x * p0.y - l0.y * p0.x) - (l1.x * p1.y - l1.y * p1.x);
  return (double)v;
}

// 2x2 on the pair (a0, a1) of psi and the pair (b0, b1) of lambda by the
// matrix's shape, in place: m holds the uniform entries (m00, m01, m10, m11
// as re, im).  Shape 1 diagonal, 2 real, 3 real diagonal with imaginary
// off-diagonal (RX, Y), 0 general.  One asm block per pair of both states
// whose results land in the amplitudes' own registers, so that the shapes'
// code paths leave the register arrays where they were (left to itself the
// compiler ties results to temporaries and copies arrays back at merges).
#define QSV_F32_DIAG(X, Y)            \
  "v_mul_f32 %[t0], %[m01], " Y "\n\t"  \
  "v_mul_f32 " Y ", %[m00], " Y "\n\t"  \
  "v_fmac_f32 " Y ", %[m01], " X "\n\t" \
  "v_fma_f32 " X ", %[m00], " X ", -%[t0]\n\t"
#define QSV_F32_REAL(A, B)            \
  "v_mul_f32 %[t0], %[m01], " B "\n\t"  \
  "v_mul_f32 " B ", %[m11], " B "\n\t"  \
  "v_fmac_f32 " B ", %[m10], " A "\n\t" \
  "v_fma_f32 " A ", %[m00], " A ", %[t0]\n\t"
#define QSV_F32_RX(AX, AY, BX, BY)        \
  "v_mul_f32 %[t0], %[m01], " BY "\n\t"     \
  "v_mul_f32 %[t1], %[m10], " AY "\n\t"     \
  "v_mul_f32 " AY ", %[m00], " AY "\n\t"    \
  "v_fmac_f32 " AY ", %[m01], " BX "\n\t"   \
  "v_mul_f32 " BY ", %[m11], " BY "\n\t"    \
  "v_fmac_f32 " BY ", %[m10], " AX "\n\t"   \
  "v_fma_f32 " AX ", %[m00], " AX ", -%[t0]\n\t" \
  "v_fma_f32 " BX ", %[m11], " BX ", -%[t1]\n\t"
#define QSV_F64_DIAG(X, Y)                  \
  "v_mul_f64 %[t0], %[m01], " Y "\n\t"        \
  "v_mul_f64 " Y ", %[m00], " Y "\n\t"        \
  "v_fma_f64 " Y ", %[m01], " X ", " Y "\n\t" \
  "v_fma_f64 " X ", %[m00], " X ", -%[t0]\n\t"
#define QSV_F64_REAL(A, B)                  \
  "v_mul_f64 %[t0], %[m01], " B "\n\t"        \
  "v_mul_f64 " B ", %[m11], " B "\n\t"        \
  "v_fma_f64 " B ", %[m10], " A ", " B "\n\t" \
  "v_fma_f64 " A ", %[m00], " A ", %[t0]\n\t"
#define QSV_F64_RX(AX, AY, BX, BY)                \
  "v_mul_f64 %[t0], %[m01], " BY "\n\t"             \
  "v_mul_f64 %[t1], %[m10], " AY "\n\t"             \
  "v_mul_f64 " AY ", %[m00], " AY "\n\t"            \
  "v_fma_f64 " AY ", %[m01], " BX ", " AY "\n\t"    \
  "v_mul_f64 " BY ", %[m11], " BY "\n\t"            \
  "v_fma_f64 " BY ", %[m10], " AX ", " BY "\n\t"    \
  "v_fma_f64 " AX ", %[m00], " AX ", -%[t0]\n\t"    \
  "v_fma_f64 " BX ", %[m11], " BX ", -%[t1]\n\t"

template <int F, typename T>
__device__ __forceinline__ void form_apply2(const T* m, cpx<T>& a0, cpx<T>& a1, cpx<T>& b0, cpx<T>& b1) {
  constexpr bool D = sizeof(T) == 8;
  T t0, t1;
  if (F == 1) {  // a0 *= m00, a1 *= m11 (complex), the same for b
    if (D) {
      asm(QSV_F64_DIAG("%[a0x]", "%[a0y]") QSV_F64_DIAG("%[b0x]", "%[b0y]")
          : [a0x] "+v"(a0.x), [a0y] "+v"(a0.y), [b0x] "+v"(b0.x), [b0y] "+v"(b0.y), [t0] "=&v"(t0)
          : [m00] "s"(m[0]), [m01] "s"(m[1]));
      asm(QSV_F64_DIAG("%[a1x]", "%[a1y]") QSV_F64_DIAG("%[b1x]", "%[b1y]")
          : [a1x] "+v"(a1.x), [a1y] "+v"(a1.y), [b1x] "+v"(b1.x), [b1y] "+v"(b1.y), [t0] "=&v"(t0)
          : [m00] "s"(m[6]), [m01] "s"(m[7]));
    } else {
      asm(QSV_F32_DIAG("%[a0x]", "%[a0y]") QSV_F32_DIAG("%[b0x]", "%[b0y]")
          : [a0x] "+v"(a0.x), [a0y] "+v"(a0.y), [b0x] "+v"(b0.x), [b0y] "+v"(b0.y), [t0] "=&v"(t0)
          : [m00] "s"(m[0]), [m01] "s"(m[1]));
      asm(QSV_F32_DIAG("%[a1x]", "%[a1y]") QSV_F32_DIAG("%[b1x]", "%[b1y]")
          : [a1x] "+v"(a1.x), [a1y] "+v"(a1.y), [b1x] "+v"(b1.x), [b1y] "+v"(b1.y), [t0] "=&v"(t0)
          : [m00] "s"(m[6]), [m01] "s"(m[7]));
    }
  } else if (F == 2) {  // real entries: each component of (a0, a1) by the real 2x2
    if (D)
      asm(QSV_F64_REAL("%[a0x]", "%[a1x]") QSV_F64_REAL("%[a0y]", "%[a1y]")
          QSV_F64_REAL("%[b0x]", "%[b1x]") QSV_F64_REAL("%[b0y]", "%[b1y]")
          : [a0x] "+v"(a0.x), [a0y] "+v"(a0.y), [a1x] "+v"(a1.x), [a1y] "+v"(a1.y), [b0x] "+v"(b0.x),
            [b0y] "+v"(b0.y), [b1x] "+v"(b1.x), [b1y] "+v"(b1.y), [t0] "=&v"(t0)
          : [m00] "s"(m[0]), [m01] "s"(m[2]), [m10] "s"(m[4]), [m11] "s"(m[6]));
    else
      asm(QSV_F32_REAL("%[a0x]", "%[a1x]") QSV_F32_REAL("%[a0y]", "%[a1y]")
          QSV_F32_REAL("%[b0x]", "%[b1x]") QSV_F32_REAL("%[b0y]", "%[b1y]")
          : [a0x] "+v"(a0.x), [a0y] "+v"(a0.y), [a1x] "+v"(a1.x), [a1y] "+v"(a1.y), [b0x] "+v"(b0.x),
            [b0y] "+v"(b0.y), [b1x] "+v"(b1.x), [b1y] "+v"(b1.y), [t0] "=&v"(t0)
          : [m00] "s"(m[0]), [m01] "s"(m[2]), [m10] "s"(m[4]), [m11] "s"(m[6]));
  } else if (F == 3) {  // real diagonal (m00, m11), imaginary off-diagonal (m01, m10)
    if (D)
      asm(QSV_F64_RX("%[a0x]", "%[a0y]", "%[a1x]", "%[a1y]") QSV_F64_RX("%[b0x]", "%[b0y]", "%[b1x]", "%[b1y]")
          : [a0x] "+v"(a0.x), [a0y] "+v"(a0.y), [a1x] "+v"(a1.x), [a1y] "+v"(a1.y), [b0x] "+v"(b0.x),
            [b0y] "+v"(b0.y), [b1x] "+v"(b1.x), [b1y] "+v"(b1.y), [t0] "=&v"(t0), [t1] "=&v"(t1)
          : [m00] "s"(m[0]), [m01] "s"(m[3]), [m10] "s"(m[5]), [m11] "s"(m[6]));
    else
      asm(QSV_F32_RX("%[a0x]", "%[a0y]", "%[a1x]", "%[a1y]") QSV_F32_RX("%[b0x]", "%[b0y]", "%[b1x]", "%[b1y]")
          : [a0x] "+v"(a0.x), [a0y] "+v"(a0.y), [a1x] "+v"(a1.x), [a1y] "+v"(a1.y), [b0x] "+v"(b0.x),
            [b0y] "+v"(b0.y), [b1x] "+v"(b1.x), [b1y] "+v"(b1.y), [t0] "=&v"(t0), [t1] "=&v"(t1)
          : [m00] "s"(m[0]), [m01] "s"(m[3]), [m10] "s"(m[5]), [m11] "s"(m[6]));
  } else {  // general: rare (explicit one-qubit matrices), plain code
    M2<T> V;
#pragma unroll
    for (int f = 0; f < 4; ++f) V.m[f] = cpx<T>{m[2 * f], m[2 * f + 1]};
    apply2(V, a0, a1);
    apply2(V, b0, b1);
  }
}
#undef QSV_F32_DIAG
#undef QSV_F32_REAL
#undef QSV_F32_RX
#undef QSV_F64_DIAG
#undef QSV_F64_REAL
#undef QSV_F64_RX

// LDS position of tile amplitude l: the bits that select a 256-byte row are
// XORed into the position within the row, so lanes whose amplitudes differ
// only above the row (register groups over low qubits) fall in distinct banks
template <typename T>
__device__ __forceinline__ uint32_t swz(uint32_t l) {
  constexpr int SB = sizeof(T) == 4 ? 5 : 4;
  return l ^ ((l >> SB) & ((1u << SB) - 1u));
}

// A ROUND gate on register bit J of the 2^K amplitudes x (psi) and y
// (lambda) that one thread holds: the rotation's term over its pairs (before
// the gate), then the gate; shape and generator are template arguments so
// the pair loops carry no branches
template <typename T, int K, int J, int G>
__device__ __forceinline__ double round_grad(const cpx<T>* x, const cpx<T>* y) {
  double g = 0.0;
#pragma unroll
  for (int q = 0; q < (1 << (K - 1)); ++q) {
    const int i0 = ((q >> J) << (J + 1)) | (q & ((1 << J) - 1)), i1 = i0 | (1 << J);
    g += grad_pair<T>(G, x[i0], x[i1], y[i0], y[i1]);
  }
  return g;
}

template <typename T, int K, int J, int F>
__device__ __forceinline__ void round_apply(const T* m, cpx<T>* x, cpx<T>* y) {
#pragma unroll
  for (int q = 0; q < (1 << (K - 1)); ++q) {
    const int i0 = ((q >> J) << (J + 1)) | (q & ((1 << J) - 1)), i1 = i0 | (1 << J);
    form_apply2<F>(m, x[i0], x[i1], y[i0], y[i1]);
  }
}

template <typename T, int K, int J>
__device__ __forceinline__ double round_gate(int form, int gen, bool grad, const T* V, cpx<T>* x, cpx<T>* y) {
  double g = 0.0;
  if (grad) {
    if (gen == 0)
      g = round_grad<T, K, J, 0>(x, y);
    else if (gen == 1)
      g = round_grad<T, K, J, 1>(x, y);
    else
      g = round_grad<T, K, J, 2>(x, y);
  }
  // one if per shape, each opaque to the others (an if-else chain over the
  // shapes makes the compiler copy the register arrays at every merge)
  asm volatile("" : "+s"(form));
  if (form == 1) round_apply<T, K, J, 1>(V, x, y);
  asm volatile("" : "+s"(form));
  if (form == 2) round_apply<T, K, J, 2>(V, x, y);
  asm volatile("" : "+s"(form));
  if (form == 3) round_apply<T, K, J, 3>(V, x, y);
  asm volatile("" : "+s"(form));
  if (form == 0) round_apply<T, K, J, 0>(V, x, y);
  return g;
}

// The gates of a round on register bit J (cnt of them, at gw, which moves
// past them), each with its rotation's wave sum added to its slot
// The parts of a sign run (type-5 layout at rec) fixed by the tile's base
// index: the local bits Mo whose sign pattern is linear in this tile, and
// the parity cpar of the outside pairs.
__device__ __forceinline__ void sign_tile_terms(const int32_t* rec, uint64_t base, uint32_t& Mo, int& cpar) {
  const int nd = rec[1], nlo = rec[2], noo = rec[3];
  const int32_t* w = rec + 8;
  for (int i = 0; i < nlo; ++i) {
    const int oq = w[2 * nd + 2 * i + 1];
    if (oq < 0 || ((base >> oq) & 1ull)) Mo ^= 1u << w[2 * nd + 2 * i];
  }
  for (int i = 0; i < noo; ++i) {
    const int32_t* pq = w + 2 * (nd + nlo + i);
    cpar ^= (int)((base >> pq[0]) & (base >> pq[1]) & 1ull);
  }
}

template <typename T, int K, int J>
__device__ __forceinline__ void round_bit(int cnt, const int32_t*& gw, cpx<T>* x, cpx<T>* y, double* gacc,
                                          int wave, int lane) {
  for (int e = 0; e < cnt; ++e, gw += kAdjGate) {
    const int info = gw[0], gslot = gw[1];
    const int form = (info >> 4) & 3, gn = (info >> 8) & 3;
    T V[8];
    const T* gm = reinterpret_cast<const T*>(gw + 4);
#pragma unroll
    for (int f = 0; f < 8; ++f) V[f] = gm[f];
    double gv = round_gate<T, K, J>(form, gn, gslot >= 0, V, x, y);
    if (gslot >= 0) {
      gv = wave_sum_d(gv);
      if (lane == 0) gacc[gslot * (kAB / 64) + wave] += gv;
    }
  }
}

template <typename T, int TB>
__global__ __launch_bounds__(kAB) void k_adj_tile(cpx<T>* __restrict__ psi, cpx<T>* __restrict__ lam,
                                                  const int32_t* __restrict__ prog, uint64_t ntiles,
                                                  double* __restrict__ part) {
  constexpr int A = VecInfo<T>::A;
  __shared__ cpx<T> tp[1 << TB];
  __shared__ cpx<T> tl[1 << TB];
  __shared__ double gacc[kMaxAdjGrad * (kAB / 64)];
  __shared__ uint64_t segoff[256];
  const int t = prog[0], c = prog[1], nns = prog[2], nops = prog[3], ngrad = prog[4];
  const int ntph = prog[7];  // records of tile phases (type 7)
  const int32_t* S = prog + 8;
  const int32_t* nonS = S + t;
  const int32_t* recs = prog + prog[5];
  const int nseg = 1 << (t - c);
  for (int h = threadIdx.x; h < nseg; h += kAB) {
    uint64_t o = 0;
    for (int j = 0; j < t - c; ++j)
      if ((h >> j) & 1) o |= 1ull << S[c + j];
    segoff[h] = o;
  }
  for (int i = threadIdx.x; i < ngrad * (kAB / 64); i += kAB) gacc[i] = 0.0;
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  vec16<T>* gp = reinterpret_cast<vec16<T>*>(psi);
  vec16<T>* gl = reinterpret_cast<vec16<T>*>(lam);
  const int nvec = (1 << t) / A;
  const uint32_t cmask = (1u << c) - 1u;
  const int half = 1 << (t - 1), full = 1 << t;
  // Each thread's share of the next tile of both states is loaded into
  // registers while the gates of the current one run.  Every lane issues
  // every load (an index past a smaller tile repeats one of its vectors,
  // whose value is not used), so that the loads go out back to back.
  constexpr int VPT = (1 << TB) / A / kAB;
  using V = typename AdjVec<T>::V;
  const V* __restrict__ vp = reinterpret_cast<const V*>(psi);
  const V* __restrict__ vl = reinterpret_cast<const V*>(lam);
  V xs[VPT], ys[VPT];
  auto tile_base = [&](uint64_t id) {
    uint64_t b = 0;
    for (int i = 0; i < nns; ++i) b |= ((id >> i) & 1ull) << nonS[i];
    return b;
  };
#define QSV_ADJ_LOAD_TILE(B)                                                  \
  _Pragma("unroll") for (int k = 0; k < VPT; ++k) {                           \
    const int i = threadIdx.x + k * kAB;                                      \
    const uint32_t l = (uint32_t)(i < nvec ? i : (i & (nvec - 1))) * A;       \
    const uint64_t g = ((B) | segoff[l >> c] | (l & cmask)) / A;              \
    xs[k] = vp[g];                                                            \
    ys[k] = vl[g];                                                            \
  }
  if (blockIdx.x < ntiles) {
    const uint64_t b0 = tile_base(blockIdx.x);
    QSV_ADJ_LOAD_TILE(b0)
  }
  for (uint64_t tid = blockIdx.x; tid < ntiles; tid += gridDim.x) {
    const uint64_t base = tile_base(tid);
    // A diagonal unitary on a qubit outside the tile is one phase for the
    // whole tile, the same on both states: it is multiplied into tph and
    // applied by the store.  Its gradient term is +-Im<lambda|psi> over the
    // tile, which the tile's other records (unitaries applied to both
    // states) leave unchanged: the thread's share s_im is taken at the load.
    cpx<T> tph{T(1), T(0)};
    double s_im = 0.0;
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
      const int i = threadIdx.x + k * kAB;
      if (i < nvec) {
        const uint32_t l = (uint32_t)i * A;
#pragma unroll
        for (int e = 0; e < A; ++e) {
          const cpx<T> p = AdjVec<T>::at(xs[k], e), q = AdjVec<T>::at(ys[k], e);
          tp[swz<T>(l + e)] = p;
          tl[swz<T>(l + e)] = q;
          if (ntph > 0) s_im += (double)q.x * (double)p.y - (double)q.y * (double)p.x;
        }
      }
    }
    __syncthreads();
    if (tid + gridDim.x < ntiles) {
      const uint64_t bn = tile_base(tid + gridDim.x);
      QSV_ADJ_LOAD_TILE(bn)
    }
#undef QSV_ADJ_LOAD_TILE
    const int32_t* r = recs;
    for (int o = 0; o < nops; ++o, r += r[0] == 6 ? r[3] : kAdjRec) {
      const int type = r[0], ra = r[1], rb = r[2], slot = (type < 4 || type == 7) ? r[3] : -1, gen = r[4];
      double g = 0.0;
      if (type == 1) {
        M2<T> V;
#pragma unroll
        for (int e = 0; e < 4; ++e) V.m[e] = rec_cpx<T>(r, e);
        const uint32_t lowm = (1u << ra) - 1u;
        for (int u = threadIdx.x; u < half; u += kAB) {
          const uint32_t i0 = (((uint32_t)u >> ra) << (ra + 1)) | ((uint32_t)u & lowm), i1 = i0 | (1u << ra);
          cpx<T> p0 = tp[swz<T>(i0)], p1 = tp[swz<T>(i1)], l0 = tl[swz<T>(i0)], l1 = tl[swz<T>(i1)];
          if (slot >= 0) g += grad_pair<T>(gen, p0, p1, l0, l1);
          apply2(V, p0, p1);
          apply2(V, l0, l1);
          tp[swz<T>(i0)] = p0;
          tp[swz<T>(i1)] = p1;
          tl[swz<T>(i0)] = l0;
          tl[swz<T>(i1)] = l1;
        }
      } else if (type == 7) {
        const bool one = ((base >> ra) & 1ull) != 0;  // the outside qubit's value in this tile
        tph = cmul(one ? rec_cpx<T>(r, 1) : rec_cpx<T>(r, 0), tph);
        if (slot >= 0) g = one ? -s_im : s_im;
      } else if (type == 2) {
        const cpx<T> d0 = rec_cpx<T>(r, 0), d1 = rec_cpx<T>(r, 1), d2 = rec_cpx<T>(r, 2), d3 = rec_cpx<T>(r, 3);
        const int ka = ra >> 8, va = ra & 255;
        const int kb = rb < 0 ? -1 : (rb >> 8), vb = rb < 0 ? 0 : (rb & 255);
        const int oa = ka == 0 ? -1 : (int)((base >> va) & 1ull);  // outside operands: one bit per tile
        const int ob = kb < 0 ? 0 : kb == 0 ? -1 : (int)((base >> vb) & 1ull);
        for (int l = threadIdx.x; l < full; l += kAB) {
          const int bA = oa >= 0 ? oa : (l >> va) & 1;
          const int bB = ob >= 0 ? ob : (l >> vb) & 1;
          const cpx<T> dd = bB ? (bA ? d3 : d2) : (bA ? d1 : d0);
          const cpx<T> p = tp[swz<T>(l)], q = tl[swz<T>(l)];
          if (slot >= 0) {
            const double im = (double)q.x * (double)p.y - (double)q.y * (double)p.x;
            g += bA ? -im : im;
          }
          tp[swz<T>(l)] = cmul(dd, p);
          tl[swz<T>(l)] = cmul(dd, q);
        }
      } else if (type == 6) {
        constexpr int K = AdjRound<T>::K, NR = 1 << K;
        const int ngate = rb;
        uint32_t off[NR];
        off[0] = 0;
#pragma unroll
        for (int m = 1; m < NR; ++m) off[m] = off[m & (m - 1)] | (1u << r[4 + __builtin_ctz(m)]);
        const int ngroups = full >> K;
        const int32_t* sr = r[1] ? r + r[1] : nullptr;  // a sign run applied at the load
        uint32_t Mo = 0;
        int cpar = 0;
        if (sr) sign_tile_terms(sr, base, Mo, cpar);
        for (int g0 = 0; g0 < ngroups; g0 += kAB) {  // every lane runs every group step (shuffles below)
          const int gi = g0 + (int)threadIdx.x;
          const bool valid = gi < ngroups;
          uint32_t b = (uint32_t)gi;
#pragma unroll
          for (int j = 0; j < K; ++j) {
            const int bj = r[4 + j];
            b = ((b >> bj) << (bj + 1)) | (b & ((1u << bj) - 1u));
          }
          cpx<T> x[NR], y[NR];
#pragma unroll
          for (int m = 0; m < NR; ++m) {
            x[m] = valid ? tp[swz<T>(b | off[m])] : cpx<T>{0, 0};
            y[m] = valid ? tl[swz<T>(b | off[m])] : cpx<T>{0, 0};
          }
          if (sr) {
            const int nd = sr[1];
            const int32_t* w = sr + 8;
#pragma unroll
            for (int m = 0; m < NR; ++m) {
              const uint32_t l = b | off[m];
              int par = cpar + __popc(l & Mo);
              for (int i = 0; i < nd; ++i) par += __popc(l & (l >> w[2 * i]) & (uint32_t)w[2 * i + 1]);
              if (par & 1) {
                x[m] = cpx<T>{-x[m].x, -x[m].y};
                y[m] = cpx<T>{-y[m].x, -y[m].y};
              }
            }
          }
          const int32_t* gw = r + 8;
          round_bit<T, K, 0>((ngate >> 0) & 255, gw, x, y, gacc, wave, lane);
          round_bit<T, K, 1>((ngate >> 8) & 255, gw, x, y, gacc, wave, lane);
          round_bit<T, K, 2>((ngate >> 16) & 255, gw, x, y, gacc, wave, lane);
          if (K > 3) round_bit<T, K, (K > 3 ? 3 : 2)>((ngate >> 24) & 255, gw, x, y, gacc, wave, lane);
          if (valid) {
#pragma unroll
            for (int m = 0; m < NR; ++m) {
              tp[swz<T>(b | off[m])] = x[m];
              tl[swz<T>(b | off[m])] = y[m];
            }
          }
        }
      } else if (type == 5) {
        const int nd = ra;
        const int32_t* w = r + 8;
        uint32_t Mo = 0;
        int cpar = 0;
        sign_tile_terms(r, base, Mo, cpar);
        for (int l = threadIdx.x; l < full; l += kAB) {
          int par = cpar + __popc((uint32_t)l & Mo);
          for (int i = 0; i < nd; ++i) par += __popc((uint32_t)l & ((uint32_t)l >> w[2 * i]) & (uint32_t)w[2 * i + 1]);
          if (par & 1) {
            const cpx<T> p = tp[swz<T>(l)], q = tl[swz<T>(l)];
            tp[swz<T>(l)] = cpx<T>{-p.x, -p.y};
            tl[swz<T>(l)] = cpx<T>{-q.x, -q.y};
          }
        }
      } else {
        M4<T> U;
#pragma unroll
        for (int e = 0; e < 16; ++e) U.m[e] = rec_cpx<T>(r, e);
        const int j0 = ra, j1 = rb;
        for (int u = threadIdx.x; u < (full >> 2); u += kAB) {
          uint32_t i = (uint32_t)u;
          i = ((i >> j0) << (j0 + 1)) | (i & ((1u << j0) - 1u));
          i = ((i >> j1) << (j1 + 1)) | (i & ((1u << j1) - 1u));
          const uint32_t ix[4] = {i, i | (1u << j0), i | (1u << j1), i | (1u << j0) | (1u << j1)};
          cpx<T> x[4], y[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            x[e] = tp[swz<T>(ix[e])];
            y[e] = tl[swz<T>(ix[e])];
          }
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            cpx<T> ax = cmul(U.m[4 * rr], x[0]), ay = cmul(U.m[4 * rr], y[0]);
#pragma unroll
            for (int cc = 1; cc < 4; ++cc) {
              ax = cfma(U.m[4 * rr + cc], x[cc], ax);
              ay = cfma(U.m[4 * rr + cc], y[cc], ay);
            }
            tp[swz<T>(ix[rr])] = ax;
            tl[swz<T>(ix[rr])] = ay;
          }
        }
      }
      if (slot >= 0) {
        g = wave_sum_d(g);
        if (lane == 0) gacc[slot * (kAB / 64) + wave] += g;
      }
      __syncthreads();
    }
    for (int i = threadIdx.x; i < nvec; i += kAB) {
      const uint32_t l = (uint32_t)i * A;
      const uint64_t g = (base | segoff[l >> c] | (l & cmask)) / A;
      vec16<T> x, y;
#pragma unroll
      for (int e = 0; e < A; ++e) {
        x.a[e] = tp[swz<T>(l + e)];
        y.a[e] = tl[swz<T>(l + e)];
        if (ntph > 0) {
          x.a[e] = cmul(tph, x.a[e]);
          y.a[e] = cmul(tph, y.a[e]);
        }
      }
      gp[g] = x;
      gl[g] = y;
    }
    __syncthreads();
  }
  for (int sl = threadIdx.x; sl < ngrad; sl += kAB) {
    double v = 0.0;
    for (int w = 0; w < kAB / 64; ++w) v += gacc[sl * (kAB / 64) + w];
    part[(size_t)sl * gridDim.x + blockIdx.x] = v;
  }
}

// out[map[s]] = sum_b part[s * nb + b], one workgroup per gradient slot
__global__ __launch_bounds__(kAB) void k_adj_gsum(const double* __restrict__ part, int nb,
                                                  const int32_t* __restrict__ map, double* __restrict__ out) {
  __shared__ double sh[kAB];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += kAB) acc += part[(size_t)blockIdx.x * nb + b];
  const double s = block_sum_d(acc, sh);
  if (threadIdx.x == 0) out[map[blockIdx.x]] = s;
}

template <typename T>
int adj_tile_bits() {
  return sizeof(T) == 4 ? 12 : 11;
}
int adj_max_grad() { return kMaxAdjGrad; }
int adj_rec_words() { return kAdjRec; }
int adj_gate_words() { return kAdjGate; }
template <typename T>
int adj_round_bits() {
  return AdjRound<T>::K;
}
template int adj_round_bits<float>();
template int adj_round_bits<double>();

// Workgroups of the sweep kernel resident at once (cached per device).
template <typename T>
static int adj_grid() {
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (cache[dev] == 0) {
    int per_cu = 0, ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_adj_tile<T, (sizeof(T) == 4 ? 12 : 11)>, kAB, 0) !=
            hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return 0;
    cache[dev] = per_cu * ncu;
  }
  return cache[dev];
}

// One tile pass of the sweep (program at prog_dev, header in prog_host);
// part needs n_grad * adj_max_grid() doubles; gradients go to out_dev[map].
template <typename T>
hipError_t launch_adj_tile(cpx<T>* psi, cpx<T>* lam, int n, const int32_t* prog_dev, const int32_t* prog_host,
                           double* part, double* out_dev, hipStream_t st) {
  constexpr int TB = sizeof(T) == 4 ? 12 : 11;
  const int t = prog_host[0], ngrad = prog_host[4];
  if (t > TB || ngrad > kMaxAdjGrad || t - prog_host[1] > 8) return hipErrorInvalidValue;
  const uint64_t ntiles = 1ull << (n - t);
  int resident = adj_grid<T>();
  if (resident <= 0) return hipErrorInvalidValue;
  const unsigned grid = (unsigned)std::min<uint64_t>(ntiles, (uint64_t)std::min(resident, kMaxAdjPartials));
  hipLaunchKernelGGL((k_adj_tile<T, TB>), dim3(grid), dim3(kAB), 0, st, psi, lam, prog_dev, ntiles, part);
  if (ngrad > 0)
    hipLaunchKernelGGL(k_adj_gsum, dim3(ngrad), dim3(kAB), 0, st, part, (int)grid, prog_dev + prog_host[6],
                       out_dev);
  return hipGetLastError();
}

size_t adjoint_partials() { return kMaxAdjPartials; }

template <typename T>
hipError_t launch_hpsi(const cpx<T>* psi, cpx<T>* lam, int n, const uint64_t* x, const uint64_t* z,
                       const double* wr, const double* wi, int nt, hipStream_t st) {
  const uint64_t N = 1ull << n;
  const dim3 grid = grid_for((N + kAB - 1) / kAB);
  for (int t0 = 0; t0 < nt || t0 == 0; t0 += kMaxHTerms) {
    HTerms h{};
    h.nt = nt - t0 < kMaxHTerms ? nt - t0 : kMaxHTerms;
    for (int t = 0; t < h.nt; ++t) {
      h.x[t] = x[t0 + t];
      h.z[t] = z[t0 + t];
      h.wr[t] = wr[t0 + t];
      h.wi[t] = wi[t0 + t];
    }
    hipLaunchKernelGGL(k_hpsi<T>, grid, dim3(kAB), 0, st, psi, lam, N, h, t0 > 0 ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (nt == 0) break;
  }
  return hipSuccess;
}

// ------------------------------------------- lambda = H psi by tile passes
// Terms whose X mask lies in a tile's qubit set S are applied by one pass
// over the tiles of S: the psi tile is staged in LDS (swizzled), and each
// thread forms lambda_j = sum_t w_t (-1)^{|(j ^ x_t) & z_t|} psi_{j ^ x_t}
// for its amplitudes in FP64 registers, term by term, adding to the lambda
// already stored when the pass is not the first.  With j = base | loc(l)
// the sign's parity splits into parity(l & zl_t) over the tile's local bits
// and parity(base & z_t) ^ parity(x_t & z_t), uniform per tile.  The last
// pass also sums Re(conj(psi_j) lambda_j) = <psi|H|psi> from the FP64 values.
//
// Program (int32 words): [0] t, [1] c, [2] n_nonS, [3] n_terms, [4] add to
// lambda, [5] sum the energy, [6] offset of the terms, S[t] from word 8,
// nonS after.  Term (kHTermWords words): [0] local X mask, [1] local Z mask,
// [2..3] Z mask, [4] parity(x & z), [6..7] weight re, [8..9] weight im
// (w = c i^{n_y}).
constexpr int kHTermWords = 10;

// One term on a thread's amplitudes l = threadIdx.x + i * kAB: partner from
// registers (X-free) or LDS, the sign (-1)^{|l & zl|} flipped into the
// weight's sign bit, two FMAs for a real weight and four otherwise
template <typename T, int PER, bool LDSX, bool REAL>
__device__ __forceinline__ void hpsi_term(const cpx<T>* tp, const cpx<T>* own, uint32_t xl, uint32_t zl, double wr,
                                          double wi, int full, double* ar, double* ai) {
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const uint32_t l = threadIdx.x + (uint32_t)i * kAB;
    if (LDSX && (int)l >= full) continue;
    const cpx<T> p = LDSX ? tp[swz<T>(l ^ xl)] : own[i];
    const double pr = (double)p.x, pi = (double)p.y;
    const int sb = (__popc(l & zl) & 1) << 31;
    const double sr = __hiloint2double(__double2hiint(wr) ^ sb, __double2loint(wr));
    if (REAL) {
      ar[i] = fma(sr, pr, ar[i]);
      ai[i] = fma(sr, pi, ai[i]);
    } else {
      const double si = __hiloint2double(__double2hiint(wi) ^ sb, __double2loint(wi));
      ar[i] = fma(sr, pr, fma(-si, pi, ar[i]));
      ai[i] = fma(sr, pi, fma(si, pr, ai[i]));
    }
  }
}

template <typename T, int TB>
__global__ __launch_bounds__(kAB) void k_hpsi_tile(const cpx<T>* __restrict__ psi, cpx<T>* __restrict__ lam,
                                                   const int32_t* __restrict__ prog, uint64_t ntiles,
                                                   double* __restrict__ part) {
  constexpr int A = VecInfo<T>::A;
  constexpr int PER = (1 << TB) / kAB;  // amplitudes per thread in a full tile
  __shared__ cpx<T> tp[1 << TB];
  __shared__ uint64_t segoff[256];
  __shared__ double sh[kAB];
  const int t = prog[0], c = prog[1], nns = prog[2], nterms = prog[3], add = prog[4], energy = prog[5];
  const int32_t* S = prog + 8;
  const int32_t* nonS = S + t;
  const int32_t* terms = prog + prog[6];
  const int nseg = 1 << (t - c);
  for (int h = threadIdx.x; h < nseg; h += kAB) {
    uint64_t o = 0;
    for (int j = 0; j < t - c; ++j)
      if ((h >> j) & 1) o |= 1ull << S[c + j];
    segoff[h] = o;
  }
  __syncthreads();
  const vec16<T>* gp = reinterpret_cast<const vec16<T>*>(psi);
  const int nvec = (1 << t) / A, full = 1 << t;
  const uint32_t cmask = (1u << c) - 1u;
  double eacc = 0.0;
  for (uint64_t tid = blockIdx.x; tid < ntiles; tid += gridDim.x) {
    uint64_t base = 0;
    for (int i = 0; i < nns; ++i) base |= ((tid >> i) & 1ull) << nonS[i];
    for (int i = threadIdx.x; i < nvec; i += kAB) {
      const uint32_t l = (uint32_t)i * A;
      const vec16<T> x = gp[(base | segoff[l >> c] | (l & cmask)) / A];
#pragma unroll
      for (int e = 0; e < A; ++e) tp[swz<T>(l + e)] = x.a[e];
    }
    __syncthreads();
    double ar[PER], ai[PER];
    cpx<T> own[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const uint32_t l = threadIdx.x + (uint32_t)i * kAB;
      ar[i] = 0.0;
      ai[i] = 0.0;
      own[i] = cpx<T>{0, 0};
      if ((int)l < full) {
        own[i] = tp[swz<T>(l)];
        if (add) {
          const cpx<T> v = lam[base | segoff[l >> c] | (l & cmask)];
          ar[i] = (double)v.x;
          ai[i] = (double)v.y;
        }
      }
    }
    for (int k = 0; k < nterms; ++k) {
      const int32_t* w = terms + k * kHTermWords;
      const uint32_t xl = (uint32_t)w[0], zl = (uint32_t)w[1];
      const uint64_t zg = ((uint64_t)(uint32_t)w[3] << 32) | (uint32_t)w[2];
      const int ts = (__popcll(base & zg) + w[4]) & 1;
      const double wr0 = __hiloint2double(w[7], w[6]), wi0 = __hiloint2double(w[9], w[8]);
      const double wr = ts ? -wr0 : wr0, wi = ts ? -wi0 : wi0;
      // X-free terms use the amplitudes held in registers, the others read
      // their partners from LDS; real weights take two FMAs.  One opaque if
      // per case (an if-else would have the compiler copy the accumulators
      // at the merge)
      uint32_t xo = xl;
      const int real = (w[8] | (w[9] & 0x7fffffff)) == 0;  // wi == +-0 from its bits (scalar)
      int kind = __builtin_amdgcn_readfirstlane((xo != 0) * 2 + real);  // uniform
      asm volatile("" : "+s"(kind));
      if (kind == 1) hpsi_term<T, PER, false, true>(tp, own, xo, zl, wr, wi, full, ar, ai);
      asm volatile("" : "+s"(kind));
      if (kind == 0) hpsi_term<T, PER, false, false>(tp, own, xo, zl, wr, wi, full, ar, ai);
      asm volatile("" : "+s"(kind));
      if (kind == 3) hpsi_term<T, PER, true, true>(tp, own, xo, zl, wr, wi, full, ar, ai);
      asm volatile("" : "+s"(kind));
      if (kind == 2) hpsi_term<T, PER, true, false>(tp, own, xo, zl, wr, wi, full, ar, ai);
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const uint32_t l = threadIdx.x + (uint32_t)i * kAB;
      if ((int)l < full) {
        if (energy) eacc = fma((double)own[i].x, ar[i], fma((double)own[i].y, ai[i], eacc));
        lam[base | segoff[l >> c] | (l & cmask)] = cpx<T>{(T)ar[i], (T)ai[i]};
      }
    }
    __syncthreads();
  }
  if (energy) {
    const double v = block_sum_d(eacc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
  }
}

template <typename T>
int hpsi_tile_bits() {
  return sizeof(T) == 4 ? 12 : 11;
}
int hpsi_term_words() { return kHTermWords; }

// One pass of lambda = H psi (program at prog_dev, header in prog_host); with
// the energy flag set, *energy_dev receives <psi|H|psi> (part holds one
// double per workgroup, adjoint_partials() of them)
template <typename T>
hipError_t launch_hpsi_tile(const cpx<T>* psi, cpx<T>* lam, int n, const int32_t* prog_dev,
                            const int32_t* prog_host, double* part, double* energy_dev, hipStream_t st) {
  constexpr int TB = sizeof(T) == 4 ? 12 : 11;
  const int t = prog_host[0];
  if (t > TB || t - prog_host[1] > 8 || t > n) return hipErrorInvalidValue;
  const uint64_t ntiles = 1ull << (n - t);
  const unsigned grid = (unsigned)std::min<uint64_t>(ntiles, (uint64_t)kMaxAdjPartials);
  hipLaunchKernelGGL((k_hpsi_tile<T, TB>), dim3(grid), dim3(kAB), 0, st, psi, lam, prog_dev, ntiles, part);
  if (prog_host[5]) hipLaunchKernelGGL(k_adj_final, dim3(1), dim3(kAB), 0, st, part, (int)grid, energy_dev);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_rot(cpx<T>* psi, cpx<T>* lam, int n, int q, const M2<T>& V, const M2<double>& G,
                          double* part, double* out_dev, hipStream_t st) {
  const uint64_t pairs = (1ull << n) / 2;
  uint64_t g = (pairs + kAB * 8 - 1) / (kAB * 8);
  if (g < 1) g = 1;
  if (g > kMaxAdjPartials) g = kMaxAdjPartials;
  const uint64_t chunk = (pairs + g - 1) / g;
  hipLaunchKernelGGL(k_adj_rot<T>, dim3((unsigned)g), dim3(kAB), 0, st, psi, lam, pairs, chunk, q, V,
                     G, part);
  hipLaunchKernelGGL(k_adj_final, dim3(1), dim3(kAB), 0, st, part, (int)g, out_dev);
  return hipGetLastError();
}

#define QSV_AINST(T)                                                                              \
  template int adj_tile_bits<T>();                                                                \
  template int hpsi_tile_bits<T>();                                                               \
  template hipError_t launch_hpsi_tile<T>(const cpx<T>*, cpx<T>*, int, const int32_t*,             \
                                          const int32_t*, double*, double*, hipStream_t);          \
  template hipError_t launch_adj_tile<T>(cpx<T>*, cpx<T>*, int, const int32_t*, const int32_t*,    \
                                         double*, double*, hipStream_t);                          \
  template hipError_t launch_hpsi<T>(const cpx<T>*, cpx<T>*, int, const uint64_t*, const uint64_t*, \
                                     const double*, const double*, int, hipStream_t);             \
  template hipError_t launch_adj_rot<T>(cpx<T>*, cpx<T>*, int, int, const M2<T>&,                  \
                                        const M2<double>&, double*, double*, hipStream_t);
QSV_AINST(float)
QSV_AINST(double)

}  // namespace qsv
