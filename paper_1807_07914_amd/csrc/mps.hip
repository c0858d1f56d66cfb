// mps.hip -- matrix-product-state gate application on gfx950.
//
// Paper section III (the figure on applying a two-body gate to adjacent MPS
// tensors: contract the gate with the two site tensors, then split the result
// by an SVD) and section IV.B (the MPS visitor: canonical form of n rank-3
// tensors and n-1 diagonal bond matrices; singular values below a cutoff
// epsilon, 1e-4 by default, are truncated).
//
// Storage (complex128): site l holds B_l[a][s][b] = Gamma_l Lambda_l+1, the
// right-canonical tensor, at sites[l * kSlot + (2a + s) * kChi + b]; bond b
// (between sites b-1 and b) holds its Schmidt coefficients at lam[b * kChi];
// dims[b] is its dimension.  Every slot has the fixed stride kChi, so an
// update never moves other sites.
//
// One two-site update (one workgroup of 512 threads; T' and M in LDS while
// the update's three bonds are at most 32, else in a global workspace that
// stays in the caches):
//   T'[(a,s'), (t',c)] = sum_{s,t} G[s'+2t', s+2t] sum_m B_l[a,s,m] B_l+1[m,t,c]
//   M = diag(Lambda_l) T'  -- the two-site block in mixed-canonical form
//   one-sided Jacobi on the rows of M: a unitary from the left makes the rows
//   orthogonal; row norms are the singular values S and the normalised rows
//   the right singular vectors V^H (no left vectors are formed)
//   B_l+1' = rows of V^H (kept), B_l' = T' V, Lambda_l+1' = S (kept)
// The left site needs no division by a bond coefficient because T' carries
// no Lambda_l: T' V = Lambda_l^-1 U S = Gamma_l' Lambda_l+1'.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_set>
#include <vector>

#include "internal.hpp"
#include "plan.hpp"

struct qsv_mps;

namespace qsv {
namespace {

constexpr int kChi = QSV_MPS_MAX_CHI;         // slot stride and largest bond
constexpr int kChiL = 32;                     // largest bond of an update staged in LDS
constexpr int kRowsL = 2 * kChiL;             // row stride of T' and M in LDS
constexpr int kRowsG = 2 * kChi;              // row stride of T' and M in global memory
constexpr int kSlot = 2 * kChi * kChi;        // complex entries per site slot
constexpr int kThreads = 512;
constexpr int kPairLanes = 16;                // lanes per Jacobi row pair (one DPP row)
constexpr int kGroups = kThreads / kPairLanes;  // row pairs in flight per step
constexpr int kMaxSweeps = 48;                // bound on Jacobi sweeps
constexpr double kOrthTol = 1e-14;            // rotate while |<r_p,r_q>| > tol |r_p||r_q|
constexpr double kZeroRel = 1e-12;            // numerical-zero rule for singular values
constexpr double kZeroRow = 1e-13;            // rows below this fraction of |M|_F are not rotated
constexpr uint32_t kMpsMagic = 0x5053514du;   // "MQSP"

static_assert(kGroups >= kRowsL / 2, "one lane group per row pair in the LDS path");
static_assert(kPairLanes == 16, "the DPP group sum spans one 16-lane row");

struct z2 {
  double x, y;
};

// One update: the site index and, for two-site updates, a 4x4 gate with local
// index (bit of site) + 2 (bit of site+1); for one-site updates a 2x2 in g[0..8).
struct MpsJob {
  int32_t site;
  int32_t pad;
  double g[32];
};

__device__ __forceinline__ z2 zmul(z2 a, z2 b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ void zfma(z2& acc, z2 a, z2 b) {
  acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
  acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
}
// acc += a * conj(b)
__device__ __forceinline__ void zfmac(z2& acc, z2 a, z2 b) {
  acc.x = fma(a.x, b.x, fma(a.y, b.y, acc.x));
  acc.y = fma(a.y, b.x, fma(-a.x, b.y, acc.y));
}

// Sum over each 16-lane DPP row (xor 1, xor 2, half-row mirror, row
// mirror).  Every lane of a row ends with the bitwise-same value: at each
// stage the two partners add the same two numbers, in either order.
template <int CTRL>
__device__ __forceinline__ double dpp_sum(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return v + __hiloint2double(hi, lo);
}
// 1/sqrt(x) and 1/x for positive normal x: the hardware estimates refined
// by two Newton steps each (the estimate's error squares per step), in
// place of the library forms that also handle zeros, infinities and
// denormals, which cannot occur here.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = fma(y, fma(-h * y, y, 0.5), y);
  y = fma(y, fma(-h * y, y, 0.5), y);
  return y;
}
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(y, fma(-x, y, 1.0), y);
  y = fma(y, fma(-x, y, 1.0), y);
  return y;
}
__device__ __forceinline__ double group_sum(double v) {
  return dpp_sum<0x140>(dpp_sum<0x141>(dpp_sum<0x4E>(dpp_sum<0xB1>(v))));
}

__global__ void k_mps_init(z2* __restrict__ sites, double* __restrict__ lam, int* __restrict__ dims,
                           int* __restrict__ err, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) sites[(size_t)i * kSlot] = z2{1.0, 0.0};
  if (i <= n) {
    lam[(size_t)i * kChi] = 1.0;
    dims[i] = 1;
  }
  if (i == 0) err[0] = 0;
}

// One two-site update by the workgroup, with T' and M at row stride ROWS in
// tp and mr and the site tensors staged at sa and sb: LDS arrays for bonds up
// to kChiL (ROWS = kRowsL), a slice of global memory (L2-resident) for larger
// ones (ROWS = kRowsG).  The steps are the same either way.
template <int ROWS>
__device__ __forceinline__ void bond_update(z2* __restrict__ sites, double* __restrict__ lam, int* __restrict__ dims,
                                            const MpsJob& jb, int cl, int cm, int cr, int chi_max, double cutoff,
                                            z2* sa, z2* sb, z2* tp, z2* mr, double* sv, int* order, int* flags,
                                            int* keep_s, double* red) {
  const int l = jb.site;
  const int tid = threadIdx.x;
  const int R = 2 * cl, L = 2 * cr;
  z2* A = sites + (size_t)l * kSlot;
  z2* B = A + kSlot;

  // stage B_l as [(2a+s) * cm + m] and B_l+1 as [(2m+t) * cr + c]
  for (int i = tid; i < 2 * cl * cm; i += kThreads) {
    const int r = i / cm, m = i - r * cm;
    sa[i] = A[r * kChi + m];
  }
  for (int i = tid; i < 2 * cm * cr; i += kThreads) {
    const int r = i / cr, c = i - r * cr;
    sb[i] = B[r * kChi + c];
  }
  for (int i = tid; i < kMaxSweeps; i += kThreads) flags[i] = 0;
  __syncthreads();

  // contract the two sites and apply the gate
  const z2* G = reinterpret_cast<const z2*>(jb.g);
  for (int i = tid; i < cl * cr; i += kThreads) {
    const int a = i / cr, c = i - a * cr;
    z2 th[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};   // index s + 2t
    for (int m = 0; m < cm; ++m) {
      const z2 a0 = sa[(2 * a) * cm + m], a1 = sa[(2 * a + 1) * cm + m];
      const z2 b0 = sb[(2 * m) * cr + c], b1 = sb[(2 * m + 1) * cr + c];
      zfma(th[0], a0, b0);
      zfma(th[1], a1, b0);
      zfma(th[2], a0, b1);
      zfma(th[3], a1, b1);
    }
    for (int o = 0; o < 4; ++o) {
      z2 acc{0, 0};
      for (int k = 0; k < 4; ++k) zfma(acc, G[o * 4 + k], th[k]);
      tp[(2 * a + (o & 1)) * ROWS + (o >> 1) * cr + c] = acc;
    }
  }
  __syncthreads();

  // M: rows scaled by the left bond's Schmidt coefficients
  const double* lam_l = lam + (size_t)l * kChi;
  double part = 0;
  for (int i = tid; i < R * L; i += kThreads) {
    const int r = i / L, col = i - r * L;
    const double w = lam_l[r >> 1];
    const z2 v = tp[r * ROWS + col];
    const z2 u{w * v.x, w * v.y};
    mr[r * ROWS + col] = u;
    part = fma(u.x, u.x, fma(u.y, u.y, part));
  }
  red[tid] = part;
  __syncthreads();
  if (tid == 0) {
    double f = 0;
    for (int i = 0; i < kThreads; ++i) f += red[i];
    red[0] = f;
  }
  __syncthreads();
  // rows below 1e-13 of |M|_F are numerical zeros: they are never rotated
  // (orthogonalising rounding noise does not converge) and are always below
  // the kept-value threshold
  const double zthr = kZeroRow * kZeroRow * red[0];

  // one-sided Jacobi on the rows of M, round-robin pairing: in each step
  // every row belongs to one pair; a sweep of R-1 steps meets every pair once.
  // A lane group takes pairs grp, grp + kGroups, ... (one pair each in LDS).
  const int grp = tid / kPairLanes, lane = tid % kPairLanes;
  const int npairs = R / 2;
  for (int sw = 0; sw < kMaxSweeps; ++sw) {
    for (int step = 0; step < R - 1; ++step) {
      for (int pr = grp; pr < npairs; pr += kGroups) {
        int p, q;
        if (pr == 0) {
          p = R - 1;
          q = step;
        } else {
          p = (step + pr) % (R - 1);
          q = (step - pr + R - 1) % (R - 1);
        }
        z2* rp = mr + p * ROWS;
        z2* rq = mr + q * ROWS;
        constexpr int kCols = ROWS / kPairLanes;   // columns per lane at most
        z2 xs[kCols], ys[kCols];
        double al = 0, be = 0, gr = 0, gi = 0;   // |r_p|^2, |r_q|^2, sum r_p conj(r_q)
#pragma unroll
        for (int k = 0; k < kCols; ++k) {
          const int c = lane + k * kPairLanes;
          xs[k] = c < L ? rp[c] : z2{0, 0};
          ys[k] = c < L ? rq[c] : z2{0, 0};
          const z2 x = xs[k], y = ys[k];
          al = fma(x.x, x.x, fma(x.y, x.y, al));
          be = fma(y.x, y.x, fma(y.y, y.y, be));
          gr = fma(x.x, y.x, fma(x.y, y.y, gr));
          gi = fma(x.y, y.x, fma(-x.x, y.y, gi));
        }
        // all lanes of the pair get bitwise-equal sums, so they take one decision
        al = group_sum(al);
        be = group_sum(be);
        gr = group_sum(gr);
        gi = group_sum(gi);
        const double g2 = gr * gr + gi * gi;
        if (al >= zthr && be >= zthr && g2 > kOrthTol * kOrthTol * al * be) {
          // y = e^{i arg g} r_q makes the pair's Gram matrix real; then the
          // symmetric 2x2 Jacobi rotation with the smaller angle.  The row
          // floor zthr bounds |tau| by about 5e39, so tau^2 cannot overflow.
          // The test is relative only: kept rows of small norm must still come
          // out orthonormal to the others, or the right site loses its
          // canonical form.
          const double iag = rsqrt_nr(g2);
          const double tau = 0.5 * (be - al) * iag;
          const double u = fma(tau, tau, 1.0);
          const double t = copysign(rcp_nr(fabs(tau) + u * rsqrt_nr(u)), tau);
          const double cs = rsqrt_nr(fma(t, t, 1.0)), sn = cs * t;
          const double er = gr * iag, ei = gi * iag;
#pragma unroll
          for (int k = 0; k < kCols; ++k) {
            const int c = lane + k * kPairLanes;
            if (c < L) {
              const z2 x = xs[k], y0 = ys[k];
              const z2 y{er * y0.x - ei * y0.y, er * y0.y + ei * y0.x};
              rp[c] = z2{cs * x.x - sn * y.x, cs * x.y - sn * y.y};
              rq[c] = z2{sn * x.x + cs * y.x, sn * x.y + cs * y.y};
            }
          }
          if (lane == 0) flags[sw] = 1;
        }
      }
      // global-memory rows: the barrier also orders this step's writes
      // before the next step's reads within the workgroup
      if (ROWS == kRowsG) __threadfence_block();
      __syncthreads();
    }
    if (!flags[sw]) break;   // every thread reads the same value after the barrier
  }

  // singular values, descending order (ties by row), kept count
  for (int r = tid; r < R; r += kThreads) {
    double s2 = 0;
    for (int c = 0; c < L; ++c) {
      const z2 v = mr[r * ROWS + c];
      s2 = fma(v.x, v.x, fma(v.y, v.y, s2));
    }
    sv[r] = sqrt(s2);
  }
  __syncthreads();
  if (tid < R) {
    const double me = sv[tid];
    int rank = 0;
    for (int j = 0; j < R; ++j) rank += (sv[j] > me) || (sv[j] == me && j < tid);
    order[rank] = tid;
  }
  if (tid == 0) {
    double top = 0;
    for (int j = 0; j < R; ++j) top = fmax(top, sv[j]);
    int cnt = 0;
    for (int j = 0; j < R; ++j) cnt += (sv[j] > cutoff) && (sv[j] > kZeroRel * top);
    *keep_s = max(1, min(cnt, min(chi_max, min(R, L))));
  }
  __syncthreads();
  const int k = *keep_s;

  // B_l+1'[j][t][c] = V^H[j][(t,c)]
  for (int i = tid; i < k * L; i += kThreads) {
    const int j = i / L, col = i - j * L;
    const int r = order[j];
    const double inv = sv[r] > 0 ? 1.0 / sv[r] : 0.0;
    const z2 v = mr[r * ROWS + col];
    const int t = col / cr, c = col - t * cr;
    B[(2 * j + t) * kChi + c] = z2{v.x * inv, v.y * inv};
  }
  // B_l'[(a,s)][j] = sum_col T'[(a,s), col] conj(V^H[j][col])
  for (int i = tid; i < R * k; i += kThreads) {
    const int r = i / k, j = i - r * k;
    const int rr = order[j];
    z2 acc{0, 0};
    for (int col = 0; col < L; ++col) zfmac(acc, tp[r * ROWS + col], mr[rr * ROWS + col]);
    const double inv = sv[rr] > 0 ? 1.0 / sv[rr] : 0.0;
    A[r * kChi + j] = z2{acc.x * inv, acc.y * inv};
  }
  double* lam_m = lam + (size_t)(l + 1) * kChi;
  for (int j = tid; j < kChi; j += kThreads) lam_m[j] = j < k ? sv[order[j]] : 0.0;
  if (tid == 0) dims[l + 1] = k;
}

// Global-memory workspace of one update (complex entries): the staged site
// tensors, T' and M at row stride kRowsG.
constexpr size_t kBondWsEntries = (size_t)4 * kChi * kChi + (size_t)2 * kRowsG * kRowsG;

// Two-site updates, one per workgroup; the jobs of one launch act on disjoint
// sites.  Updates whose three bonds are at most kChiL run in LDS; larger ones
// use the job's slice of gws (kBondWsEntries entries; NULL when the MPS's
// bond cap is at most kChiL, which keeps every bond there).
__global__ __launch_bounds__(kThreads) void k_mps_bond(z2* __restrict__ sites, double* __restrict__ lam,
                                                        int* __restrict__ dims, const MpsJob* __restrict__ jobs,
                                                        int chi_max, double cutoff, int* __restrict__ err,
                                                        z2* __restrict__ gws) {
  __shared__ z2 ltp[kRowsL * kRowsL];   // T' in LDS (rows (a,s), columns (t,c))
  __shared__ z2 lmr[kRowsL * kRowsL];   // first the staged site tensors, then M
  __shared__ double sv[kRowsG];
  __shared__ int order[kRowsG];
  __shared__ int flags[kMaxSweeps];
  __shared__ int keep_s;
  __shared__ double red[kThreads];

  const MpsJob& jb = jobs[blockIdx.x];
  const int l = jb.site;
  const int cl = dims[l], cm = dims[l + 1], cr = dims[l + 2];
  if (cl < 1 || cm < 1 || cr < 1 || cl > kChi || cm > kChi || cr > kChi) {  // uniform
    if (threadIdx.x == 0) err[0] = 1;
    return;
  }
  if (cl <= kChiL && cm <= kChiL && cr <= kChiL) {  // uniform
    bond_update<kRowsL>(sites, lam, dims, jb, cl, cm, cr, chi_max, cutoff, lmr, lmr + kRowsL * kRowsL / 2, ltp,
                        lmr, sv, order, flags, &keep_s, red);
  } else if (gws) {
    z2* w = gws + (size_t)blockIdx.x * kBondWsEntries;
    z2* sa = w;
    z2* sb = sa + (size_t)2 * kChi * kChi;
    z2* tp = sb + (size_t)2 * kChi * kChi;
    z2* mr = tp + (size_t)kRowsG * kRowsG;
    bond_update<kRowsG>(sites, lam, dims, jb, cl, cm, cr, chi_max, cutoff, sa, sb, tp, mr, sv, order, flags,
                        &keep_s, red);
  } else if (threadIdx.x == 0) {
    err[0] = 1;
  }
}

// One-site gates: B'[a][s'][b] = sum_s U[s'][s] B[a][s][b].
__global__ __launch_bounds__(kThreads) void k_mps_site(z2* __restrict__ sites, const int* __restrict__ dims,
                                                        const MpsJob* __restrict__ jobs) {
  const MpsJob& jb = jobs[blockIdx.x];
  const int l = jb.site;
  const int cl = min(dims[l], kChi), cr = min(dims[l + 1], kChi);
  const z2* U = reinterpret_cast<const z2*>(jb.g);
  z2* S = sites + (size_t)l * kSlot;
  for (int i = threadIdx.x; i < cl * cr; i += kThreads) {
    const int a = i / cr, b = i - a * cr;
    const z2 x0 = S[(2 * a) * kChi + b], x1 = S[(2 * a + 1) * kChi + b];
    z2 y0 = zmul(U[0], x0), y1 = zmul(U[2], x0);
    zfma(y0, U[1], x1);
    zfma(y1, U[3], x1);
    S[(2 * a) * kChi + b] = y0;
    S[(2 * a + 1) * kChi + b] = y1;
  }
}

// Amplitudes: one wavefront per index walks the sites left to right,
// v <- v B_l[:, bit l, :], with v (at most kChi entries) in LDS.
constexpr int kAmpWaves = 4;
__global__ __launch_bounds__(64 * kAmpWaves) void k_mps_amp(const z2* __restrict__ sites,
                                                            const int* __restrict__ dims, int n,
                                                            const uint64_t* __restrict__ idx, int64_t count,
                                                            z2* __restrict__ out) {
  __shared__ z2 v[kAmpWaves][2][kChi];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * kAmpWaves + w;
  const uint64_t x = i < count ? idx[i] : 0;
  if (lane < kChi) v[w][0][lane] = z2{lane == 0 ? 1.0 : 0.0, 0.0};
  __syncthreads();
  int cur = 0;
  for (int l = 0; l < n; ++l) {
    const int cl = min(dims[l], kChi), cr = min(dims[l + 1], kChi);
    const int s = (int)((x >> l) & 1);
    const z2* Bs = sites + (size_t)l * kSlot;
    if (lane < cr) {
      z2 acc{0, 0};
      for (int b = 0; b < cl; ++b) zfma(acc, v[w][cur][b], Bs[(2 * b + s) * kChi + lane]);
      v[w][cur ^ 1][lane] = acc;
    }
    __syncthreads();
    cur ^= 1;
  }
  if (i < count && lane == 0) out[i] = v[w][cur][0];
}

}  // namespace
}  // namespace qsv

struct qsv_mps {
  uint32_t magic;
  int n, chi_max;
  double cutoff;
  hipStream_t stream;
  qsv::z2* sites;
  double* lam;
  int* dims;
  int* err;
  qsv::MpsJob* jobs_dev;
  size_t jobs_cap;
  qsv::z2* gws;       // workspaces of updates with bonds above the LDS limit
  size_t gws_jobs;    // updates the workspace holds
  std::vector<qsv::MpsJob> jobs_host;   // source of the last upload, kept until the stream passes it
  uint64_t* idx_dev;
  qsv::z2* amp_dev;
  size_t amp_cap;
  int64_t bond_updates, launches;
  std::atomic<int> busy;
};

namespace qsv {
namespace {

using cd = std::complex<double>;

std::mutex g_mps_mu;
std::unordered_set<const qsv_mps*> g_mps_live;

bool mps_live(const qsv_mps* m) {
  std::lock_guard<std::mutex> lk(g_mps_mu);
  return m && g_mps_live.count(m) && m->magic == kMpsMagic;
}

struct MpsBusy {
  qsv_mps* m;
  bool ok;
  explicit MpsBusy(qsv_mps* mm) : m(mm) {
    int expect = 0;
    ok = m->busy.compare_exchange_strong(expect, 1);
  }
  ~MpsBusy() {
    if (ok) m->busy.store(0);
  }
};

#define QSV_MPS_ENTER(m)                                                                     \
  if (!::qsv::mps_live(m)) return ::qsv::fail(QSV_ERR_STATE, "invalid or freed MPS handle"); \
  ::qsv::MpsBusy busy_guard_(m);                                                             \
  if (!busy_guard_.ok) return ::qsv::fail(QSV_ERR_STATE, "MPS is in use by another call");

void release(qsv_mps* m) {
  (void)hipFree(m->sites);
  (void)hipFree(m->lam);
  (void)hipFree(m->dims);
  (void)hipFree(m->err);
  (void)hipFree(m->jobs_dev);
  (void)hipFree(m->gws);
  (void)hipFree(m->idx_dev);
  (void)hipFree(m->amp_dev);
}

// 4x4 index of a gate whose first operand is the high site: swap the bit roles
int swap_bits(int r) { return ((r & 1) << 1) | (r >> 1); }

MpsJob make_job(int site, const cd* g, int dim) {
  MpsJob j{};
  j.site = site;
  for (int e = 0; e < dim * dim; ++e) {
    j.g[2 * e] = g[e].real();
    j.g[2 * e + 1] = g[e].imag();
  }
  return j;
}

const cd kSwap[16] = {1, 0, 0, 0, 0, 0, 1, 0, 0, 1, 0, 0, 0, 0, 0, 1};

qsv_status check_mps_op(int n, const qsv_op& o) {
  const int k = o.gate == QSV_MAT ? o.nq : gate_arity(o.gate);
  if (o.gate != QSV_MAT && k < 0) return fail(QSV_ERR_ARG, "unknown gate id " + std::to_string(o.gate));
  if (o.gate == QSV_MAT && (o.nq < 1 || o.nq > QSV_MAX_K)) return fail(QSV_ERR_ARG, "matrix op: nq out of range");
  if (o.nq != k) return fail(QSV_ERR_ARG, "wrong qubit count for gate");
  if (k > 2) return fail(QSV_ERR_UNSUPPORTED, "the MPS path takes one- and two-qubit instructions");
  for (int j = 0; j < k; ++j)
    if (o.q[j] < 0 || o.q[j] >= n)
      return fail(QSV_ERR_ARG, "qubit " + std::to_string(o.q[j]) + " outside [0, " + std::to_string(n) + ")");
  if (k == 2 && o.q[0] == o.q[1]) return fail(QSV_ERR_ARG, "duplicate qubit " + std::to_string(o.q[0]));
  if (o.gate == QSV_MAT) {
    if (!o.mat) return fail(QSV_ERR_ARG, "matrix op without matrix");
    const int D = 1 << k;
    for (int e = 0; e < 2 * D * D; ++e)
      if (!std::isfinite(o.mat[e])) return fail(QSV_ERR_ARG, "non-finite matrix entry");
  } else {
    for (int e = 0; e < gate_nparams(o.gate); ++e)
      if (!std::isfinite(o.p[e])) return fail(QSV_ERR_ARG, "non-finite gate parameter");
  }
  return QSV_OK;
}

// Host encoder: the job list and its launches for one instruction list (ops
// already validated).  launches hold (offset, count); a negative count marks
// the one-site launch.
void encode_mps(int n, const qsv_op* ops, int n_ops, std::vector<MpsJob>& jobs,
                std::vector<std::pair<size_t, int>>& launches) {
  // pending one-qubit products per qubit (folded into the next two-site update)
  std::vector<std::array<cd, 4>> pend(n, std::array<cd, 4>{1, 0, 0, 1});
  std::vector<char> has(n, 0);
  // two-site jobs with their ASAP level: a job waits for the last job on either site
  std::vector<std::pair<int, MpsJob>> bond;
  std::vector<int> last(n, 0);
  auto push = [&](int site, const cd* g) {
    const int lv = std::max(last[site], last[site + 1]) + 1;
    last[site] = last[site + 1] = lv;
    bond.emplace_back(lv, make_job(site, g, 4));
  };
  cd mat[64];
  for (int i = 0; i < n_ops; ++i) {
    const qsv_op& o = ops[i];
    const int k = o.gate == QSV_MAT ? o.nq : gate_arity(o.gate);
    if (o.gate == QSV_MAT) {
      for (int e = 0; e < (1 << (2 * k)); ++e) mat[e] = cd(o.mat[2 * e], o.mat[2 * e + 1]);
    } else {
      gate_matrix(o.gate, o.p, mat);
    }
    if (k == 1) {
      const int q = o.q[0];
      const std::array<cd, 4> P = pend[q];
      for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) pend[q][2 * r + c] = mat[2 * r] * P[c] + mat[2 * r + 1] * P[2 + c];
      has[q] = 1;
      continue;
    }
    const int q0 = o.q[0], q1 = o.q[1];
    // G (K), K = pending one-qubit products, index bit(q0) + 2 bit(q1)
    cd G[16];
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c) {
        cd acc = 0;
        for (int x = 0; x < 4; ++x)
          acc += mat[4 * r + x] * pend[q0][2 * (x & 1) + (c & 1)] * pend[q1][2 * (x >> 1) + (c >> 1)];
        G[4 * r + c] = acc;
      }
    pend[q0] = pend[q1] = std::array<cd, 4>{1, 0, 0, 1};
    has[q0] = has[q1] = 0;
    const int lo = std::min(q0, q1), hi = std::max(q0, q1);
    if (q0 != lo) {
      cd Gs[16];
      for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) Gs[4 * r + c] = G[4 * swap_bits(r) + swap_bits(c)];
      std::copy(Gs, Gs + 16, G);
    }
    for (int b = hi - 1; b > lo; --b) push(b, kSwap);   // bring qubit hi next to lo
    push(lo, G);
    for (int b = lo + 1; b < hi; ++b) push(b, kSwap);   // and back
  }
  std::stable_sort(bond.begin(), bond.end(),
                   [](const std::pair<int, MpsJob>& a, const std::pair<int, MpsJob>& b) { return a.first < b.first; });
  // launches: one per level of two-site jobs, then one for the leftover one-site gates
  jobs.clear();
  launches.clear();
  for (size_t i = 0; i < bond.size();) {
    size_t j = i;
    while (j < bond.size() && bond[j].first == bond[i].first) jobs.push_back(bond[j++].second);
    launches.emplace_back(i, (int)(j - i));
    i = j;
  }
  const size_t n_bond = jobs.size();
  int n_site = 0;
  for (int q = 0; q < n; ++q)
    if (has[q]) {
      jobs.push_back(make_job(q, pend[q].data(), 2));
      ++n_site;
    }
  if (n_site) launches.emplace_back(n_bond, -n_site);
}

}  // namespace
}  // namespace qsv

using namespace qsv;

extern "C" qsv_status qsv_mps_alloc(int n_qubits, int chi_max, double cutoff, void* hip_stream,
                                    qsv_mps** out) {
  if (!out) return fail(QSV_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (n_qubits < 1 || n_qubits > QSV_MPS_MAX_QUBITS) return fail(QSV_ERR_ARG, "n_qubits out of range");
  if (chi_max < 1 || chi_max > QSV_MPS_MAX_CHI) return fail(QSV_ERR_ARG, "chi_max out of range");
  if (!(cutoff >= 0) || !std::isfinite(cutoff)) return fail(QSV_ERR_ARG, "cutoff must be finite and >= 0");
  qsv_mps* m = new qsv_mps();
  m->magic = kMpsMagic;
  m->n = n_qubits;
  m->chi_max = chi_max;
  m->cutoff = cutoff;
  m->stream = (hipStream_t)hip_stream;
  const size_t nb = (size_t)n_qubits + 1;
  hipError_t e = hipMalloc(&m->sites, (size_t)n_qubits * kSlot * sizeof(z2));
  if (e == hipSuccess) e = hipMalloc(&m->lam, nb * kChi * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&m->dims, nb * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&m->err, 256);
  if (e == hipSuccess) e = hipMemsetAsync(m->sites, 0, (size_t)n_qubits * kSlot * sizeof(z2), m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(m->lam, 0, nb * kChi * sizeof(double), m->stream);
  if (e == hipSuccess) {
    k_mps_init<<<(unsigned)((nb + 255) / 256), 256, 0, m->stream>>>(m->sites, m->lam, m->dims, m->err, n_qubits);
    e = hipGetLastError();
  }
  if (e != hipSuccess) {
    release(m);
    delete m;
    return hip_fail(e, "qsv_mps_alloc");
  }
  {
    std::lock_guard<std::mutex> lk(g_mps_mu);
    g_mps_live.insert(m);
  }
  *out = m;
  return QSV_OK;
}

extern "C" qsv_status qsv_mps_free(qsv_mps* m) {
  if (!m) return QSV_OK;
  if (!mps_live(m)) return fail(QSV_ERR_STATE, "invalid or freed MPS handle");
  {
    std::lock_guard<std::mutex> lk(g_mps_mu);
    g_mps_live.erase(m);
  }
  (void)hipStreamSynchronize(m->stream);
  release(m);
  m->magic = kDeadMagic;
  delete m;
  return QSV_OK;
}

extern "C" qsv_status qsv_mps_apply_circuit(qsv_mps* m, const qsv_op* ops, int n_ops) {
  QSV_MPS_ENTER(m);
  if (n_ops < 0 || (n_ops > 0 && !ops)) return fail(QSV_ERR_ARG, "bad op list");
  for (int i = 0; i < n_ops; ++i) {
    qsv_status st = check_mps_op(m->n, ops[i]);
    if (st) return fail(st, "op " + std::to_string(i) + ": " + get_error());
  }
  std::vector<std::pair<size_t, int>> launches;   // (offset, count), negative count = one-site
  QSV_HIP(hipStreamSynchronize(m->stream));       // the previous upload's source is reused
  encode_mps(m->n, ops, n_ops, m->jobs_host, launches);
  if (m->jobs_host.empty()) return QSV_OK;
  if (m->jobs_host.size() > m->jobs_cap) {
    (void)hipFree(m->jobs_dev);
    m->jobs_dev = nullptr;
    m->jobs_cap = 0;
    const size_t cap = std::max<size_t>(1024, m->jobs_host.size() * 2);
    QSV_HIP(hipMalloc(&m->jobs_dev, cap * sizeof(MpsJob)));
    m->jobs_cap = cap;
  }
  QSV_HIP(hipMemcpyAsync(m->jobs_dev, m->jobs_host.data(), m->jobs_host.size() * sizeof(MpsJob),
                         hipMemcpyHostToDevice, m->stream));
  if (m->chi_max > kChiL) {  // bonds may outgrow LDS: one global workspace per update of a launch
    size_t most = 0;
    for (const auto& lc : launches) most = std::max<size_t>(most, lc.second > 0 ? (size_t)lc.second : 0);
    if (most > m->gws_jobs) {
      QSV_HIP(hipStreamSynchronize(m->stream));
      (void)hipFree(m->gws);
      m->gws = nullptr;
      m->gws_jobs = 0;
      QSV_HIP(hipMalloc(&m->gws, most * kBondWsEntries * sizeof(z2)));
      m->gws_jobs = most;
    }
  }
  for (const auto& lc : launches) {
    if (lc.second > 0) {
      k_mps_bond<<<lc.second, kThreads, 0, m->stream>>>(m->sites, m->lam, m->dims, m->jobs_dev + lc.first,
                                                        m->chi_max, m->cutoff, m->err, m->gws);
      m->bond_updates += lc.second;
    } else {
      k_mps_site<<<-lc.second, kThreads, 0, m->stream>>>(m->sites, m->dims, m->jobs_dev + lc.first);
    }
    QSV_HIP(hipGetLastError());
    ++m->launches;
  }
  return QSV_OK;
}

static qsv_status mps_check_err(qsv_mps* m) {
  int err = 0;
  QSV_HIP(hipMemcpyAsync(&err, m->err, sizeof(int), hipMemcpyDeviceToHost, m->stream));
  QSV_HIP(hipStreamSynchronize(m->stream));
  if (err) return fail(QSV_ERR_STATE, "MPS bond dimension outside the kernel's range");
  return QSV_OK;
}

extern "C" qsv_status qsv_mps_amplitudes(qsv_mps* m, const uint64_t* idx, int64_t count, double* out) {
  QSV_MPS_ENTER(m);
  if (count < 0 || (count > 0 && (!idx || !out))) return fail(QSV_ERR_ARG, "bad index or output array");
  if (m->n > 63) return fail(QSV_ERR_UNSUPPORTED, "amplitudes need n <= 63 (64-bit indices)");
  for (int64_t i = 0; i < count; ++i)
    if (idx[i] >> m->n) return fail(QSV_ERR_ARG, "index " + std::to_string(idx[i]) + " outside the register");
  if (count == 0) return mps_check_err(m);
  if ((size_t)count > m->amp_cap) {
    QSV_HIP(hipStreamSynchronize(m->stream));
    (void)hipFree(m->idx_dev);
    (void)hipFree(m->amp_dev);
    m->idx_dev = nullptr;
    m->amp_dev = nullptr;
    m->amp_cap = 0;
    QSV_HIP(hipMalloc(&m->idx_dev, (size_t)count * sizeof(uint64_t)));
    QSV_HIP(hipMalloc(&m->amp_dev, (size_t)count * sizeof(z2)));
    m->amp_cap = (size_t)count;
  }
  QSV_HIP(hipMemcpyAsync(m->idx_dev, idx, (size_t)count * sizeof(uint64_t), hipMemcpyHostToDevice, m->stream));
  const int64_t blocks = (count + kAmpWaves - 1) / kAmpWaves;
  k_mps_amp<<<(unsigned)blocks, 64 * kAmpWaves, 0, m->stream>>>(m->sites, m->dims, m->n, m->idx_dev, count,
                                                                m->amp_dev);
  QSV_HIP(hipGetLastError());
  QSV_HIP(hipMemcpyAsync(out, m->amp_dev, (size_t)count * sizeof(z2), hipMemcpyDeviceToHost, m->stream));
  return mps_check_err(m);
}

extern "C" qsv_status qsv_mps_bonds(qsv_mps* m, int32_t* dims, double* schmidt) {
  QSV_MPS_ENTER(m);
  if (!dims) return fail(QSV_ERR_ARG, "dims is NULL");
  const size_t nb = (size_t)m->n + 1;
  QSV_HIP(hipMemcpyAsync(dims, m->dims, nb * sizeof(int), hipMemcpyDeviceToHost, m->stream));
  if (schmidt)
    QSV_HIP(hipMemcpyAsync(schmidt, m->lam, nb * kChi * sizeof(double), hipMemcpyDeviceToHost, m->stream));
  return mps_check_err(m);
}

extern "C" qsv_status qsv_mps_info(const qsv_mps* m, int64_t* bond_updates, int64_t* launches) {
  if (!mps_live(m)) return fail(QSV_ERR_STATE, "invalid or freed MPS handle");
  if (bond_updates) *bond_updates = m->bond_updates;
  if (launches) *launches = m->launches;
  return QSV_OK;
}

// Host-only debug export (not in the public header): the encoder's job list
// for an instruction list, for the CPU emulator in the tests.  Arrays are
// filled when their capacity suffices; the counts are always reported.
// gates holds 32 doubles per job (a 4x4, or a 2x2 in the first 8, complex).
extern "C" qsv_status qsv_debug_mps_program(int n, const qsv_op* ops, int n_ops, int32_t* sites,
                                            double* gates, int64_t cap_jobs, int64_t* n_jobs,
                                            int32_t* launch_counts, int64_t cap_launches,
                                            int64_t* n_launches) {
  if (n < 1 || n > QSV_MPS_MAX_QUBITS) return fail(QSV_ERR_ARG, "n out of range");
  if (n_ops < 0 || (n_ops > 0 && !ops)) return fail(QSV_ERR_ARG, "bad op list");
  for (int i = 0; i < n_ops; ++i) {
    qsv_status st = check_mps_op(n, ops[i]);
    if (st) return st;
  }
  std::vector<MpsJob> jobs;
  std::vector<std::pair<size_t, int>> launches;
  encode_mps(n, ops, n_ops, jobs, launches);
  if (n_jobs) *n_jobs = (int64_t)jobs.size();
  if (n_launches) *n_launches = (int64_t)launches.size();
  if (sites && gates && (int64_t)jobs.size() <= cap_jobs)
    for (size_t j = 0; j < jobs.size(); ++j) {
      sites[j] = jobs[j].site;
      std::memcpy(gates + 32 * j, jobs[j].g, sizeof(jobs[j].g));
    }
  if (launch_counts && (int64_t)launches.size() <= cap_launches)
    for (size_t j = 0; j < launches.size(); ++j) launch_counts[j] = launches[j].second;
  return QSV_OK;
}
