// adjoint.hip -- reverse-mode gradients of <psi(theta)|H|psi(theta)>.
//
// For psi_L = U_L ... U_1 psi_0 and E = <psi_L|H|psi_L>, with every
// parameterised gate a rotation R_P(theta) = exp(-i theta P / 2), the
// derivative with respect to the angle of gate k is
//     dE/dtheta_k = Im <lambda_k| P |psi_k>,
// psi_k = U_k ... U_1 psi_0 and lambda_k = U_{k+1}^dag ... U_L^dag H psi_L.
// One reverse sweep yields every derivative: start from psi_L and
// lambda = H psi_L, and for k = L .. 1 accumulate the gradient of gate k,
// then apply U_k^dag to both states.  A rotation's gradient and both inverse
// updates share one kernel and one HBM pass over the two states; the
// gradient is accumulated in FP64 with the fixed two-stage tree used by all
// reductions.  (Not part of the paper, whose gradients are taken over
// tensor-network factors; it is the parameter-gradient of its VQE use case.)
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
  const uint64_t j = (uint64_t)blockIdx.x * kAB + threadIdx.x;
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

size_t adjoint_partials() { return kMaxAdjPartials; }

template <typename T>
hipError_t launch_hpsi(const cpx<T>* psi, cpx<T>* lam, int n, const uint64_t* x, const uint64_t* z,
                       const double* wr, const double* wi, int nt, hipStream_t st) {
  const uint64_t N = 1ull << n;
  const unsigned grid = (unsigned)((N + kAB - 1) / kAB);
  for (int t0 = 0; t0 < nt || t0 == 0; t0 += kMaxHTerms) {
    HTerms h{};
    h.nt = nt - t0 < kMaxHTerms ? nt - t0 : kMaxHTerms;
    for (int t = 0; t < h.nt; ++t) {
      h.x[t] = x[t0 + t];
      h.z[t] = z[t0 + t];
      h.wr[t] = wr[t0 + t];
      h.wi[t] = wi[t0 + t];
    }
    hipLaunchKernelGGL(k_hpsi<T>, dim3(grid), dim3(kAB), 0, st, psi, lam, N, h, t0 > 0 ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (nt == 0) break;
  }
  return hipSuccess;
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
  template hipError_t launch_hpsi<T>(const cpx<T>*, cpx<T>*, int, const uint64_t*, const uint64_t*, \
                                     const double*, const double*, int, hipStream_t);             \
  template hipError_t launch_adj_rot<T>(cpx<T>*, cpx<T>*, int, int, const M2<T>&,                  \
                                        const M2<double>&, double*, double*, hipStream_t);
QSV_AINST(float)
QSV_AINST(double)

}  // namespace qsv
