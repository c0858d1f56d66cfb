// tile.hip -- fused tile-pass kernel: one HBM read and one HBM write of the
// state per pass, with many gates applied in between.
//
// The paper's section II groups gates into super-gates that act as a whole
// and adds SWAPs so that more gates can be applied in an accelerated way;
// on a state vector the analogue is to pick a set S of t qubits, stream the
// state through LDS one tile (all 2^t amplitudes with fixed non-S bits) at a
// time, and apply every gate whose support lies in S -- plus every diagonal
// gate, whose factor is computable from the index alone -- before writing the
// tile back.  The host planner (circuit.hip) chooses S and the gate order.
//
// gfx950 mapping: 256 threads per workgroup, tile of up to 2^13 complex64 /
// 2^12 complex128 amplitudes (64 KiB LDS).  Global loads and stores are
// 16-byte vectors over contiguous segments of 2^c amplitudes.  LDS uses an
// XOR swizzle of the amplitude index so that power-of-two strides between
// the lanes of a round do not hit one bank.  Within a round each thread holds
// 2^RB amplitudes in registers and applies 1- and 2-qubit matrices on the
// round's register bits with fully unrolled code.  The round's program (ops,
// matrices, LDS offsets) is one 256-word block that every wavefront loads
// into four VGPRs one round ahead and reads with v_readlane, so the op
// stream never waits on memory.
#include "internal.hpp"
#include "tile.hpp"

namespace qsv {

template <typename T>
struct SwzBits;
template <>
struct SwzBits<float> {
  static constexpr int B = 5;
};
template <>
struct SwzBits<double> {
  static constexpr int B = 4;
};

__device__ __forceinline__ int rl(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

// matrix entries stored in round blocks: one word per float, two per double
template <typename T>
struct WordsPer {
  static constexpr int W = sizeof(T) / 4;
};

// Round block held in four VGPRs (64 words each), written under a full exec
// mask.  Every read is a v_readlane of one of these four registers with the
// line chosen on the scalar side: the op loop may run with some lanes off
// (fewer groups than threads), and a VGPR computed there would hold stale
// values in the lanes that readlane addresses.
struct Blk {
  int l0, l1, l2, l3;
  __device__ __forceinline__ int word(int k) const {
    const int i = k & 63, ln = k >> 6;
    if (ln == 0) return rl(l0, i);
    if (ln == 1) return rl(l1, i);
    if (ln == 2) return rl(l2, i);
    return rl(l3, i);
  }
  // C consecutive words of one line (the encoder never splits such a run)
  template <int C>
  __device__ __forceinline__ void readn(int k, int (&o)[C]) const {
    const int i = k & 63, ln = k >> 6;
    if (ln == 0) {
#pragma unroll
      for (int c = 0; c < C; ++c) o[c] = rl(l0, i + c);
    } else if (ln == 1) {
#pragma unroll
      for (int c = 0; c < C; ++c) o[c] = rl(l1, i + c);
    } else if (ln == 2) {
#pragma unroll
      for (int c = 0; c < C; ++c) o[c] = rl(l2, i + c);
    } else {
#pragma unroll
      for (int c = 0; c < C; ++c) o[c] = rl(l3, i + c);
    }
  }
  template <typename T>
  __device__ __forceinline__ T real(int k) const;
};
template <>
__device__ __forceinline__ float Blk::real<float>(int k) const {
  return __int_as_float(word(k));
}
template <>
__device__ __forceinline__ double Blk::real<double>(int k) const {
  return __hiloint2double(word(k + 1), word(k));
}

template <typename T>
__device__ __forceinline__ T word_real(const int* w);
template <>
__device__ __forceinline__ float word_real<float>(const int* w) {
  return __int_as_float(w[0]);
}
template <>
__device__ __forceinline__ double word_real<double>(const int* w) {
  return __hiloint2double(w[1], w[0]);
}

template <typename T, int RB, int J>
__device__ __forceinline__ void u1(cpx<T> (&a)[1 << RB], const M2<T>& U) {
#pragma unroll
  for (int m = 0; m < (1 << RB); ++m)
    if (!((m >> J) & 1)) apply2(U, a[m], a[m | (1 << J)]);
}

template <typename T, int RB, int J0, int J1>
__device__ __forceinline__ void u2(cpx<T> (&a)[1 << RB], const M4<T>& U) {
#pragma unroll
  for (int m = 0; m < (1 << RB); ++m) {
    if (((m >> J0) & 1) || ((m >> J1) & 1)) continue;
    const int i0 = m, i1 = m | (1 << J0), i2 = m | (1 << J1), i3 = m | (1 << J0) | (1 << J1);
    const cpx<T> x0 = a[i0], x1 = a[i1], x2 = a[i2], x3 = a[i3];
    cpx<T> y[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      cpx<T> acc = cmul(U.m[4 * r + 0], x0);
      acc = cfma(U.m[4 * r + 1], x1, acc);
      acc = cfma(U.m[4 * r + 2], x2, acc);
      acc = cfma(U.m[4 * r + 3], x3, acc);
      y[r] = acc;
    }
    a[i0] = y[0];
    a[i1] = y[1];
    a[i2] = y[2];
    a[i3] = y[3];
  }
}

template <typename T, int RB>
__device__ __forceinline__ void dispatch_u1(cpx<T> (&a)[1 << RB], int j, const M2<T>& U) {
  switch (j) {
    case 0: u1<T, RB, 0>(a, U); break;
    case 1: u1<T, RB, 1>(a, U); break;
    case 2: u1<T, RB, 2>(a, U); break;
    case 3: u1<T, RB, 3>(a, U); break;
    default:
      if constexpr (RB > 4) u1<T, RB, (RB > 4 ? 4 : 0)>(a, U);
      break;
  }
}

template <typename T, int RB>
__device__ __forceinline__ void dispatch_u2(cpx<T> (&a)[1 << RB], int j0, int j1, const M4<T>& U) {
  const int key = j0 * 8 + j1;
  switch (key) {
    case 0 * 8 + 1: u2<T, RB, 0, 1>(a, U); break;
    case 0 * 8 + 2: u2<T, RB, 0, 2>(a, U); break;
    case 0 * 8 + 3: u2<T, RB, 0, 3>(a, U); break;
    case 1 * 8 + 2: u2<T, RB, 1, 2>(a, U); break;
    case 1 * 8 + 3: u2<T, RB, 1, 3>(a, U); break;
    case 2 * 8 + 3: u2<T, RB, 2, 3>(a, U); break;
    default:
      if constexpr (RB > 4) {
        constexpr int H = RB > 4 ? 4 : 3;
        switch (key) {
          case 0 * 8 + H: u2<T, RB, 0, H>(a, U); break;
          case 1 * 8 + H: u2<T, RB, 1, H>(a, U); break;
          case 2 * 8 + H: u2<T, RB, 2, H>(a, U); break;
          case 3 * 8 + H: u2<T, RB, 3, H>(a, U); break;
          default: break;
        }
      }
      break;
  }
}

// CNOT / SWAP on register bits: pure register renaming
template <typename T, int RB, int J0, int J1, int CODE>
__device__ __forceinline__ void perm2(cpx<T> (&a)[1 << RB]) {
#pragma unroll
  for (int m = 0; m < (1 << RB); ++m) {
    if (((m >> J0) & 1) || ((m >> J1) & 1)) continue;
    const int i1 = m | (1 << J0), i2 = m | (1 << J1), i3 = m | (1 << J0) | (1 << J1);
    if (CODE == 0) {
      const cpx<T> x = a[i1];
      a[i1] = a[i3];
      a[i3] = x;
    } else if (CODE == 1) {
      const cpx<T> x = a[i2];
      a[i2] = a[i3];
      a[i3] = x;
    } else {
      const cpx<T> x = a[i1];
      a[i1] = a[i2];
      a[i2] = x;
    }
  }
}

template <typename T, int RB, int J0, int J1>
__device__ __forceinline__ void perm2_code(cpx<T> (&a)[1 << RB], int code) {
  if (code == 0) perm2<T, RB, J0, J1, 0>(a);
  else if (code == 1) perm2<T, RB, J0, J1, 1>(a);
  else perm2<T, RB, J0, J1, 2>(a);
}

template <typename T, int RB>
__device__ __forceinline__ void dispatch_perm2(cpx<T> (&a)[1 << RB], int j0, int j1, int code) {
  const int key = j0 * 8 + j1;
  switch (key) {
    case 0 * 8 + 1: perm2_code<T, RB, 0, 1>(a, code); break;
    case 0 * 8 + 2: perm2_code<T, RB, 0, 2>(a, code); break;
    case 0 * 8 + 3: perm2_code<T, RB, 0, 3>(a, code); break;
    case 1 * 8 + 2: perm2_code<T, RB, 1, 2>(a, code); break;
    case 1 * 8 + 3: perm2_code<T, RB, 1, 3>(a, code); break;
    case 2 * 8 + 3: perm2_code<T, RB, 2, 3>(a, code); break;
    default:
      if constexpr (RB > 4) {
        constexpr int H = RB > 4 ? 4 : 3;
        switch (key) {
          case 0 * 8 + H: perm2_code<T, RB, 0, H>(a, code); break;
          case 1 * 8 + H: perm2_code<T, RB, 1, H>(a, code); break;
          case 2 * 8 + H: perm2_code<T, RB, 2, H>(a, code); break;
          case 3 * 8 + H: perm2_code<T, RB, 3, H>(a, code); break;
          default: break;
        }
      }
      break;
  }
}

// value of a diagonal operand bit that does not depend on m (free / outside)
__device__ __forceinline__ int const_bit(int kind, int val, uint32_t lg, uint64_t base) {
  return kind == TK_FREE ? (int)((lg >> val) & 1u) : (int)((base >> val) & 1ull);
}

// What one call of the tile body does around the rounds: take the tile from
// the state (or build |0...0> in it), write it back, and/or accumulate the
// FP64 value of sum_t c_t <Z-string_t> over the tile's amplitudes.
struct TileIO {
  int init;             // tile starts as the part of |0...0> (no load)
  int store;            // write the tile back to the state
  int reduce;           // accumulate the Z-string sum
  const uint64_t* z;    // Z masks of the terms (reduce)
  const double* coef;   // coefficients (reduce)
  int nt;
};

// One fused tile pass over tile `tid` of the pass program `prog`; returns the
// thread's partial of the Z-string sum (0 unless io.reduce).  Ends with a
// barrier so that the caller can start another tile at once.
template <typename T, int TBMAX, int RB>
__device__ __forceinline__ double tile_body(cpx<T>* __restrict__ psi, const int32_t* __restrict__ prog,
                                            uint64_t tid, const TileIO& io) {
  constexpr int A = VecInfo<T>::A;
  constexpr int NR = 1 << RB;
  constexpr int VPT = (1 << TBMAX) / A / kTileThreads;  // 16-byte vectors per thread
  constexpr int SB = SwzBits<T>::B;
  constexpr int WT = WordsPer<T>::W;                      // words per real
  __shared__ cpx<T> tile[1 << TBMAX];
  __shared__ uint64_t segoff[1 << (TBMAX - 4)];
  const int lane = threadIdx.x & 63;

  const int t = prog[0], c = prog[1], nns = prog[2], nrounds = prog[3];
  const int32_t* S = prog + 4;
  const int32_t* nonS = S + t;
  const int32_t* blocks = prog + ((4 + t + nns + 63) & ~63);
  uint64_t base = 0;
  for (int i = 0; i < nns; ++i) base |= ((tid >> i) & 1ull) << nonS[i];
  const int nseg = 1 << (t - c);
  for (int h = threadIdx.x; h < nseg; h += kTileThreads) {
    uint64_t o = 0;
    for (int j = 0; j < t - c; ++j)
      if ((h >> j) & 1) o |= 1ull << S[c + j];
    segoff[h] = o;
  }
  // first round block (prefetched while the tile loads)
  Blk nb{0, 0, 0, 0};
  if (nrounds > 0) {
    nb.l0 = blocks[lane];
    nb.l1 = blocks[64 + lane];
    nb.l2 = blocks[128 + lane];
    nb.l3 = blocks[192 + lane];
  }
  __syncthreads();

  // ---- load the tile (coalesced 16-byte vectors) into LDS
  vec16<T>* gv = reinterpret_cast<vec16<T>*>(psi);
  const int nvec = (1 << t) / A;
  const uint32_t cmask = (1u << c) - 1u;
  if (io.init) {
    for (int i = threadIdx.x; i < nvec; i += kTileThreads) {
      const uint32_t l = (uint32_t)i * A;
      const uint64_t g = base | segoff[l >> c] | (l & cmask);
#pragma unroll
      for (int e = 0; e < A; ++e)
        tile[tile_swizzle(l + e, SB)] = cpx<T>{(g + e == 0) ? T(1) : T(0), T(0)};
    }
  } else {
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
      const int i = threadIdx.x + k * kTileThreads;
      if (i < nvec) {
        const uint32_t l = (uint32_t)i * A;
        const uint64_t g = base | segoff[l >> c] | (l & cmask);
        const vec16<T> x = gv[g / A];
#pragma unroll
        for (int e = 0; e < A; ++e) tile[tile_swizzle(l + e, SB)] = x.a[e];
      }
    }
  }
  __syncthreads();

  // ---- rounds
  const int ng = 1 << (t - RB);
  for (int r = 0; r < nrounds; ++r) {
    const Blk b = nb;
    if (r + 1 < nrounds) {  // prefetch the next round's block
      const int32_t* nbp = blocks + (size_t)(r + 1) * kRoundWords;
      nb.l0 = nbp[lane];
      nb.l1 = nbp[64 + lane];
      nb.l2 = nbp[128 + lane];
      nb.l3 = nbp[192 + lane];
    }
    const int nops = rl(b.l0, 0);
    const uint32_t free_mask = (uint32_t)rl(b.l0, 1);
    for (int gi = threadIdx.x; gi < ng; gi += kTileThreads) {
      // deposit gi into the free local bits
      uint32_t lg = 0, fm = free_mask;
      for (int bit = 0; fm; ++bit) {
        const uint32_t low = fm & (0u - fm);
        if ((gi >> bit) & 1) lg |= low;
        fm ^= low;
      }
      const uint32_t sg = tile_swizzle(lg, SB);
      cpx<T> a[NR];
#pragma unroll
      for (int m = 0; m < NR; ++m) a[m] = tile[sg ^ (uint32_t)rl(b.l0, 2 + m)];

      int k = 2 + NR;
      for (int o = 0; o < nops; ++o) {
        const int type = b.word(k), len = b.word(k + 1);
        if (type == TOP_U1) {
          int wv[1 + 8 * WT];
          b.readn<1 + 8 * WT>(k + 2, wv);
          M2<T> U;
#pragma unroll
          for (int e = 0; e < 4; ++e)
            U.m[e] = cpx<T>{word_real<T>(wv + 1 + 2 * e * WT), word_real<T>(wv + 1 + (2 * e + 1) * WT)};
          dispatch_u1<T, RB>(a, wv[0], U);
        } else if (type == TOP_U2) {
          const int j0 = b.word(k + 2), j1 = b.word(k + 3);
          M4<T> U;
#pragma unroll
          for (int e = 0; e < 16; ++e)
            U.m[e] = cpx<T>{b.real<T>(k + 4 + 2 * e * WT), b.real<T>(k + 4 + (2 * e + 1) * WT)};
          dispatch_u2<T, RB>(a, j0, j1, U);
        } else if (type == TOP_PERM2) {
          int wv[3];
          b.readn<3>(k + 2, wv);
          dispatch_perm2<T, RB>(a, wv[0], wv[1], wv[2]);
        } else if (type == TOP_SIGN) {
          int p = k + 2;
          uint32_t neg = (uint32_t)b.word(p++);
          const int nf = b.word(p++);
          for (int q = 0; q < nf; ++q, p += 2)
            if ((lg >> b.word(p)) & 1u) neg ^= (uint32_t)b.word(p + 1);
          const int nd = b.word(p++);
          int par = 0;
          for (int q = 0; q < nd; ++q, p += 2)
            par ^= __popc(lg & (lg >> b.word(p)) & (uint32_t)b.word(p + 1));
          par ^= __popc(lg & (uint32_t)b.word(p++));
          const int nrc = b.word(p++);
          for (int q = 0; q < nrc; ++q, p += 2)
            if ((base >> b.word(p)) & 1ull) neg ^= (uint32_t)b.word(p + 1);
          const int nfc = b.word(p++);
          for (int q = 0; q < nfc; ++q, p += 2)
            par ^= (int)(((base >> b.word(p)) & 1ull) & ((lg >> b.word(p + 1)) & 1u));
          const int ncc = b.word(p++);
          for (int q = 0; q < ncc; ++q, p += 2)
            par ^= (int)((base >> b.word(p)) & (base >> b.word(p + 1)) & 1ull);
          if (par & 1) neg = ~neg;
#pragma unroll
          for (int m = 0; m < NR; ++m)
            if ((neg >> m) & 1u) a[m] = cpx<T>{-a[m].x, -a[m].y};
        } else if (type == TOP_PHASE1) {
          int wv[2 + 4 * WT];
          b.readn<2 + 4 * WT>(k + 2, wv);
          const int kind = wv[0], val = wv[1];
          const cpx<T> d0{word_real<T>(wv + 2), word_real<T>(wv + 2 + WT)};
          const cpx<T> d1{word_real<T>(wv + 2 + 2 * WT), word_real<T>(wv + 2 + 3 * WT)};
          if (kind == TK_REG) {
#pragma unroll
            for (int m = 0; m < NR; ++m) a[m] = cmul(((val >> m) & 1) ? d1 : d0, a[m]);
          } else {
            const cpx<T> d = const_bit(kind, val, lg, base) ? d1 : d0;
#pragma unroll
            for (int m = 0; m < NR; ++m) a[m] = cmul(d, a[m]);
          }
        } else if (type == TOP_DIAG2) {
          const int ka = b.word(k + 2), va = b.word(k + 3), kb = b.word(k + 4), vb = b.word(k + 5);
          cpx<T> d[4];
#pragma unroll
          for (int e = 0; e < 4; ++e)
            d[e] = cpx<T>{b.real<T>(k + 6 + 2 * e * WT), b.real<T>(k + 6 + (2 * e + 1) * WT)};
          const uint32_t ma = ka == TK_REG ? (uint32_t)va : (const_bit(ka, va, lg, base) ? ~0u : 0u);
          const uint32_t mb = kb == TK_REG ? (uint32_t)vb : (const_bit(kb, vb, lg, base) ? ~0u : 0u);
#pragma unroll
          for (int m = 0; m < NR; ++m) {
            const int ba = (ma >> m) & 1, bb = (mb >> m) & 1;
            const cpx<T> f = bb ? (ba ? d[3] : d[2]) : (ba ? d[1] : d[0]);
            a[m] = cmul(f, a[m]);
          }
        }
        k += len;
      }
#pragma unroll
      for (int m = 0; m < NR; ++m) tile[sg ^ (uint32_t)rl(b.l0, 2 + m)] = a[m];
    }
    __syncthreads();
  }

  // ---- Z-string sum over the tile (FP64)
  double acc = 0.0;
  if (io.reduce) {
    for (int l = threadIdx.x; l < (1 << t); l += kTileThreads) {
      const uint64_t g = base | segoff[(uint32_t)l >> c] | ((uint32_t)l & cmask);
      const cpx<T> x = tile[tile_swizzle((uint32_t)l, SB)];
      const double pr = fma((double)x.x, (double)x.x, (double)x.y * (double)x.y);
      double f = 0.0;
      for (int q = 0; q < io.nt; ++q) f += (__popcll(g & io.z[q]) & 1) ? -io.coef[q] : io.coef[q];
      acc = fma(pr, f, acc);
    }
  }

  // ---- store the tile back
  if (io.store) {
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
      const int i = threadIdx.x + k * kTileThreads;
      if (i < nvec) {
        const uint32_t l = (uint32_t)i * A;
        vec16<T> x;
#pragma unroll
        for (int e = 0; e < A; ++e) x.a[e] = tile[tile_swizzle(l + e, SB)];
        const uint64_t g = base | segoff[l >> c] | (l & cmask);
        gv[g / A] = x;
      }
    }
  }
  __syncthreads();
  return acc;
}

template <typename T, int TBMAX, int RB>
__global__ __launch_bounds__(kTileThreads) void k_tile(cpx<T>* __restrict__ psi,
                                                        const int32_t* __restrict__ prog) {
  const TileIO io{0, 1, 0, nullptr, nullptr, 0};
  (void)tile_body<T, TBMAX, RB>(psi, prog, blockIdx.x, io);
}

// ------------------------------------------------------------ batches
// Persistent kernel over many independent circuits.  Each workgroup takes
// the next job from an atomic counter (jobs are sorted largest first) and
// runs the whole circuit by itself: every pass of its plan, every tile of a
// pass in turn.  A circuit that fits one tile lives only in LDS (built as
// |0...0>, transformed, reduced); wider circuits keep their state in a
// scratch region of HBM between passes.  The last pass accumulates the
// circuit's Z-string energy instead of storing the state.
// Job record (int64 x 8): width, n_passes, first pass index, scratch offset
// (amplitudes), first term, n_terms, output slot, unused.
constexpr int kJobWords = 8;

__global__ void k_batch_reset(int* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

template <typename T, int TBMAX, int RB>
__global__ __launch_bounds__(kTileThreads) void k_batch(cpx<T>* __restrict__ scratch,
                                                         const int32_t* __restrict__ progs,
                                                         const int64_t* __restrict__ passoff,
                                                         const int64_t* __restrict__ jobs,
                                                         const uint64_t* __restrict__ zt,
                                                         const double* __restrict__ ct,
                                                         double* __restrict__ out,
                                                         int* __restrict__ counter, int njobs) {
  __shared__ int jid;
  __shared__ double red[kTileThreads];
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) jid = atomicAdd(counter, 1);
    __syncthreads();
    // The job index must be a scalar: with a per-lane copy the compiler takes
    // the exit test for divergent and may nest the loop so that lane 0 (the
    // only lane that fetches new jobs) leaves while the others spin on the
    // stale index.
    const int j = __builtin_amdgcn_readfirstlane(jid);
    if (j >= njobs) break;
    const int64_t* J = jobs + (size_t)kJobWords * j;
    const int w = (int)J[0], np = (int)J[1];
    const int64_t p0 = J[2], soff = J[3], t0 = J[4], nt = J[5], outi = J[6];
    double acc = 0.0;
    for (int p = 0; p < np; ++p) {
      const int32_t* prog = progs + passoff[p0 + p];
      const int t = prog[0];
      const uint64_t ntiles = 1ull << (w - t);
      const TileIO io{p == 0, p + 1 < np, p + 1 == np, zt + t0, ct + t0, (int)nt};
      for (uint64_t tid = 0; tid < ntiles; ++tid)
        acc += tile_body<T, TBMAX, RB>(scratch + soff, prog, tid, io);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s2 = kTileThreads / 2; s2 > 0; s2 >>= 1) {
      if ((int)threadIdx.x < s2) red[threadIdx.x] += red[threadIdx.x + s2];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[outi] = red[0];
  }
}

template <typename T>
struct TileCfg;
template <>
struct TileCfg<float> {
  static constexpr int TBMAX = 13, RB = 5;
};
template <>
struct TileCfg<double> {
  static constexpr int TBMAX = 12, RB = 4;
};

template <typename T>
int tile_max_bits() {
  return TileCfg<T>::TBMAX;
}
template <typename T>
int tile_reg_bits() {
  return TileCfg<T>::RB;
}
template <typename T>
int tile_swizzle_bits() {
  return SwzBits<T>::B;
}

template <typename T>
hipError_t launch_tile_pass(cpx<T>* psi, int n, int t, const int32_t* prog_dev, hipStream_t st) {
  const uint64_t ntiles = 1ull << (n - t);
  hipLaunchKernelGGL((k_tile<T, TileCfg<T>::TBMAX, TileCfg<T>::RB>), dim3((unsigned)ntiles),
                     dim3(kTileThreads), 0, st, psi, prog_dev);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_batch(cpx<T>* scratch, const int32_t* progs, const int64_t* passoff,
                        const int64_t* jobs, const uint64_t* zt, const double* ct, double* out,
                        int* counter, int njobs, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, st, counter);
  hipLaunchKernelGGL((k_batch<T, TileCfg<T>::TBMAX, TileCfg<T>::RB>), dim3(grid), dim3(kTileThreads),
                     0, st, scratch, progs, passoff, jobs, zt, ct, out, counter, njobs);
  return hipGetLastError();
}
template hipError_t launch_batch<float>(cpx<float>*, const int32_t*, const int64_t*, const int64_t*,
                                        const uint64_t*, const double*, double*, int*, int, int,
                                        hipStream_t);
template hipError_t launch_batch<double>(cpx<double>*, const int32_t*, const int64_t*,
                                         const int64_t*, const uint64_t*, const double*, double*,
                                         int*, int, int, hipStream_t);

template int tile_max_bits<float>();
template int tile_max_bits<double>();
template int tile_reg_bits<float>();
template int tile_reg_bits<double>();
template int tile_swizzle_bits<float>();
template int tile_swizzle_bits<double>();
template hipError_t launch_tile_pass<float>(cpx<float>*, int, int, const int32_t*, hipStream_t);
template hipError_t launch_tile_pass<double>(cpx<double>*, int, int, const int32_t*, hipStream_t);

}  // namespace qsv
