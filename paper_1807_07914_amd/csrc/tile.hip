// tile.hip -- fused tile-pass kernel: one HBM read and one HBM write of the
// state per pass, with many gates applied in between.
//
// The paper's section II groups gates into super-gates that act as a whole
// and adds SWAPs so that more gates can be applied in an accelerated way;
// on a state vector the analogue is to pick a set S of t qubits, stream the
// state through LDS one tile (all 2^t amplitudes with fixed non-S bits) at a
// time, and apply every gate whose support lies in S -- plus every diagonal
// gate, whose factor is computable from the index alone -- before writing the
// tile back.  The host planner (circuit.hip) chooses S and the gate order,
// and rewrites the gates into real rotations and diagonal factors applied in
// bulk (see the layer encoding in tile.hpp).
//
// gfx950 mapping: 256 threads per workgroup, tile of up to 2^13 complex64 /
// 2^12 complex128 amplitudes (64 KiB LDS).  Global loads and stores are
// 16-byte vectors over contiguous segments of 2^c amplitudes.  LDS uses an
// XOR swizzle of the amplitude index so that power-of-two strides between
// the lanes of a round do not hit one bank.  Within a round each thread holds
// 2^RB amplitudes in registers and applies the round's layers with fully
// unrolled code.  The round's program (header, one fixed-layout record per
// layer, aux words and tables) is read with scalar loads: the addresses are
// uniform, and every field lands in a scalar register.
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


// words per real: one per float, two per double
template <typename T>
struct WordsPer {
  static constexpr int W = sizeof(T) / 4;
};

// x <- (1 + c) x, in place (c = -2 negates, c = 0 leaves x as it is)
template <typename T>
__device__ __forceinline__ void scale1(cpx<T>& x, T c) {
  x.x = fma(c, x.x, x.x);
  x.y = fma(c, x.y, x.y);
}

// x <- z x for the complex factor z = (zr, zi), in place: four ALU ops and
// one temporary.  Written as one asm block so that the products land in the
// amplitude's own registers (left to itself the compiler ties the last FMA
// to the temporary and copies every amplitude back).
__device__ __forceinline__ void cmul(cpx<float>& x, float zr, float zi) {
  float t;
  asm("v_mul_f32 %2, %4, %1\n\t"
      "v_mul_f32 %1, %3, %1\n\t"
      "v_fmac_f32 %1, %4, %0\n\t"
      "v_fma_f32 %0, %3, %0, -%2"
      : "+v"(x.x), "+v"(x.y), "=&v"(t)
      : "s"(zr), "s"(zi));
}
__device__ __forceinline__ void cmul(cpx<double>& x, double zr, double zi) {
  double t;
  asm("v_mul_f64 %2, %4, %1\n\t"
      "v_mul_f64 %1, %3, %1\n\t"
      "v_fma_f64 %1, %4, %0, %1\n\t"
      "v_fma_f64 %0, %3, %0, -%2"
      : "+v"(x.x), "+v"(x.y), "=&v"(t)
      : "s"(zr), "s"(zi));
}

// 1 / sqrt(x): the hardware reciprocal square root in single precision
// (about one ulp, the precision of the complex64 state), an exact division
// and square root in double precision.
__device__ __forceinline__ float inv_sqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double inv_sqrt(double x) { return 1.0 / sqrt(x); }

// The same product for a factor that differs between lanes (VGPR operands).
__device__ __forceinline__ void cmul_lane(cpx<float>& x, float zr, float zi) {
  float t;
  asm("v_mul_f32 %2, %4, %1\n\t"
      "v_mul_f32 %1, %3, %1\n\t"
      "v_fmac_f32 %1, %4, %0\n\t"
      "v_fma_f32 %0, %3, %0, -%2"
      : "+v"(x.x), "+v"(x.y), "=&v"(t)
      : "v"(zr), "v"(zi));
}
__device__ __forceinline__ void cmul_lane(cpx<double>& x, double zr, double zi) {
  double t;
  asm("v_mul_f64 %2, %4, %1\n\t"
      "v_mul_f64 %1, %3, %1\n\t"
      "v_fma_f64 %1, %4, %0, %1\n\t"
      "v_fma_f64 %0, %3, %0, -%2"
      : "+v"(x.x), "+v"(x.y), "=&v"(t)
      : "v"(zr), "v"(zi));
}

// x <- exp(i phi) x as three shears of (re, im): p = -tan(phi/2), q = sin(phi)
template <typename T>
__device__ __forceinline__ void phase_shears(cpx<T>& x, T p, T q) {
  x.x = fma(p, x.y, x.x);
  x.y = fma(q, x.x, x.y);
  x.x = fma(p, x.y, x.x);
}

// Real rotation on register bit J as in-place shears (bounded coefficients):
// x0 += p x1; x1 += q x0; and x0 += p x1 again when three.
template <typename T, int RB, int J>
__device__ __forceinline__ void shears(cpx<T> (&a)[1 << RB], T p, T q, bool three) {
#pragma unroll
  for (int m = 0; m < (1 << RB); ++m) {
    if ((m >> J) & 1) continue;
    cpx<T>& x0 = a[m];
    cpx<T>& x1 = a[m | (1 << J)];
    x0.x = fma(p, x1.x, x0.x);
    x0.y = fma(p, x1.y, x0.y);
    x1.x = fma(q, x0.x, x1.x);
    x1.y = fma(q, x0.y, x1.y);
  }
  if (three) {
#pragma unroll
    for (int m = 0; m < (1 << RB); ++m) {
      if ((m >> J) & 1) continue;
      cpx<T>& x0 = a[m];
      const cpx<T> x1 = a[m | (1 << J)];
      x0.x = fma(p, x1.x, x0.x);
      x0.y = fma(p, x1.y, x0.y);
    }
  }
}

// Table step: amplitude m times sign(m) exp(i phi_m); (p_m, q_m) at entries
// 2m, 2m + 1 of the table line tp (a line of the round block in memory), the
// sign as bit m of sm.  The entries are uniform: scalar loads bring them into
// SGPRs, with no vector instruction per entry.
template <typename T, int RB>
__device__ __forceinline__ void table_step(cpx<T> (&a)[1 << RB], const int32_t* __restrict__ tp) {
  constexpr int W = WordsPer<T>::W;
#pragma unroll
  for (int m = 0; m < (1 << RB); ++m) {
    T zr, zi;
    if constexpr (W == 1) {
      zr = __int_as_float(tp[2 * m]);
      zi = __int_as_float(tp[2 * m + 1]);
    } else {
      // through readfirstlane: left to itself the compiler read the real
      // parts with vector loads, whose waits covered the next tile's prefetch
      zr = __hiloint2double(__builtin_amdgcn_readfirstlane(tp[4 * m + 1]),
                            __builtin_amdgcn_readfirstlane(tp[4 * m]));
      zi = __hiloint2double(__builtin_amdgcn_readfirstlane(tp[4 * m + 3]),
                            __builtin_amdgcn_readfirstlane(tp[4 * m + 2]));
    }
    cmul(a[m], zr, zi);
  }
}

// 2x2 and 4x4 matrices (general, rare): accumulated column by column.
template <typename T, int RB, int J>
__device__ __forceinline__ void u1(cpx<T> (&a)[1 << RB], const M2<T>& U) {
#pragma unroll
  for (int m = 0; m < (1 << RB); ++m) {
    if ((m >> J) & 1) continue;
    cpx<T>& x0 = a[m];
    cpx<T>& x1 = a[m | (1 << J)];
    const cpx<T> t0 = cmul(U.m[0], x0), t1 = cmul(U.m[2], x0);
    x0 = cfma(U.m[1], x1, t0);
    x1 = cfma(U.m[3], x1, t1);
  }
}

template <typename T, int RB, int J0, int J1>
__device__ __forceinline__ void u2(cpx<T> (&a)[1 << RB], const M4<T>& U) {
#pragma unroll
  for (int m = 0; m < (1 << RB); ++m) {
    if (((m >> J0) & 1) || ((m >> J1) & 1)) continue;
    const int i[4] = {m, m | (1 << J0), m | (1 << J1), m | (1 << J0) | (1 << J1)};
    cpx<T> acc[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = cmul(U.m[4 * r], a[i[0]]);
#pragma unroll
    for (int c = 1; c < 4; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] = cfma(U.m[4 * r + c], a[i[c]], acc[r]);
#pragma unroll
    for (int r = 0; r < 4; ++r) a[i[r]] = acc[r];
  }
}

// LDS offsets of the images of the register bits under a CNOT / SWAP of
// register bits j0 < j1 (code as in LT_PERM2; code < 0: the identity): the
// register index map is linear, so the offset of P m is the XOR of these
// over the bits of m.
template <int RB>
__device__ __forceinline__ void perm_images(const uint32_t (&bofs)[RB], int code, int j0, int j1,
                                            uint32_t (&out)[RB]) {
#pragma unroll
  for (int j = 0; j < RB; ++j) {
    uint32_t v = bofs[j];
    if (code == 2) {  // SWAP: the two bits trade places
      if (j == j0) v = bofs[j1];
      if (j == j1) v = bofs[j0];
    } else if (code == 0) {  // CNOT, control j0: e_j0 -> e_j0 + e_j1
      if (j == j0) v = bofs[j0] ^ bofs[j1];
    } else if (code == 1) {  // CNOT, control j1
      if (j == j1) v = bofs[j1] ^ bofs[j0];
    }
    out[j] = v;
  }
}

// CZ between register bits J and K: the amplitudes with both bits set change sign
template <typename T, int RB, int J, int K>
__device__ __forceinline__ void cz_pair(cpx<T> (&a)[1 << RB]) {
#pragma unroll
  for (int m = 0; m < (1 << RB); ++m)
    if (((m >> J) & 1) && ((m >> K) & 1)) scale1(a[m], T(-2));
}
// x <- (1 + c) x for the amplitudes with register bit J set (c = -2 or 0)
template <typename T, int RB, int J>
__device__ __forceinline__ void cond_z(cpx<T> (&a)[1 << RB], T c) {
#pragma unroll
  for (int m = 0; m < (1 << RB); ++m)
    if ((m >> J) & 1) scale1(a[m], c);
}
template <typename T, int RB>
__device__ __forceinline__ void dispatch_u1(cpx<T> (&a)[1 << RB], int j, const M2<T>& U) {
  if (j == 0) u1<T, RB, 0>(a, U);
  if (j == 1) u1<T, RB, 1>(a, U);
  if (j == 2) u1<T, RB, 2>(a, U);
  if (j == 3) u1<T, RB, 3>(a, U);
  if constexpr (RB > 4) {
    if (j == 4) u1<T, RB, (RB > 4 ? 4 : 3)>(a, U);
  }
}

template <typename T, int RB>
__device__ __forceinline__ void dispatch_u2(cpx<T> (&a)[1 << RB], int j0, int j1, const M4<T>& U) {
  constexpr int H = RB > 4 ? 4 : 3;
  const int key = j0 * 8 + j1;
  if (key == 0 * 8 + 1) u2<T, RB, 0, 1>(a, U);
  if (key == 0 * 8 + 2) u2<T, RB, 0, 2>(a, U);
  if (key == 0 * 8 + 3) u2<T, RB, 0, 3>(a, U);
  if (key == 1 * 8 + 2) u2<T, RB, 1, 2>(a, U);
  if (key == 1 * 8 + 3) u2<T, RB, 1, 3>(a, U);
  if (key == 2 * 8 + 3) u2<T, RB, 2, 3>(a, U);
  if constexpr (RB > 4) {
    if (key == 0 * 8 + H) u2<T, RB, 0, H>(a, U);
    if (key == 1 * 8 + H) u2<T, RB, 1, H>(a, U);
    if (key == 2 * 8 + H) u2<T, RB, 2, H>(a, U);
    if (key == 3 * 8 + H) u2<T, RB, 3, H>(a, U);
  }
}


// value of a diagonal operand bit that does not depend on m (free / outside)
__device__ __forceinline__ int const_bit(int kind, int val, uint32_t lg, uint64_t base) {
  return kind == TK_FREE ? (int)((lg >> val) & 1u) : (int)((base >> val) & 1ull);
}

// Real k of a layer record held in scalar registers (one word per float,
// two per double).
template <typename T>
__device__ __forceinline__ T rec_real(const int32_t* w, int k);
template <>
__device__ __forceinline__ float rec_real<float>(const int32_t* w, int k) {
  return __int_as_float(w[k]);
}
template <>
__device__ __forceinline__ double rec_real<double>(const int32_t* w, int k) {
  return __hiloint2double(w[k + 1], w[k]);
}
template <typename T>
__device__ __forceinline__ T aux_real(const int32_t* __restrict__ ap, int k);
template <>
__device__ __forceinline__ float aux_real<float>(const int32_t* __restrict__ ap, int k) {
  return __int_as_float(ap[k]);
}
template <>
__device__ __forceinline__ double aux_real<double>(const int32_t* __restrict__ ap, int k) {
  return __hiloint2double(ap[k + 1], ap[k]);
}

// The rounds of one tile pass (program `pass`, layout in tile.hpp) over the
// tile held in LDS at `tb`.  Round headers, layer records, aux words and
// tables are read with scalar loads (the addresses are uniform), so every
// field lands in a scalar register.  Every round ends with a barrier.
// Copy a pass's lane table (see tile.hpp) into LDS; the caller's next
// barrier publishes it.  Called before the first tile of the pass, while no
// load of a tile is in flight (vector loads complete in order).
template <typename T>
__device__ __forceinline__ void stage_lane_table(const int32_t* __restrict__ pass, cpx<T>* __restrict__ lt) {
  constexpr int WT = WordsPer<T>::W;
  const int t = pass[0], nns = pass[2], nrounds = pass[3];
  if (nrounds <= 0) return;
  const int32_t* rb0 = pass + pass[4 + t + nns];
  const int ne = rb0[kHdrLaneTabN];
  const int32_t* e = pass + rb0[kHdrLaneTab];
  for (int i = threadIdx.x; i < ne; i += kTileThreads)
    lt[i] = cpx<T>{aux_real<T>(e, 2 * i * WT), aux_real<T>(e, (2 * i + 1) * WT)};
}

template <typename T>
struct LaneTab {
  static constexpr int N = kLaneTabBytes / (int)sizeof(cpx<T>);
};

template <typename T, int TBMAX, int RB, int BODY>
__device__ __forceinline__ void run_rounds(char* __restrict__ tb, const int32_t* __restrict__ pass, int t,
                                           int nns, uint64_t base, const cpx<T>* __restrict__ lt) {
  constexpr int NR = 1 << RB;
  constexpr int SB = SwzBits<T>::B;
  constexpr int WT = WordsPer<T>::W;
  constexpr int LR = LayerRec<T>::W;
  const int ng = 1 << (t - RB);
  const int nrounds = pass[3];
  const int32_t* roff = pass + 4 + t + nns;
  // the tile's factors of the per-group phase steps that depend on the tile
  // only, once per tile: wave w takes slots w, w + 4, ...  A slot index that
  // is uniform over the wave keeps every program read a scalar load: a vector
  // load here would have to wait for the next tile's prefetch (loads and
  // stores complete in order) and end the overlap of memory and arithmetic.
  __shared__ cpx<T> tfac[kMaxTileFactors];
  if (nrounds > 0) {
    const int32_t* rb0 = pass + roff[0];
    const int nk = rb0[kHdrTileFac + 1];
    if (nk > 0) {
      const int32_t* lst = pass + rb0[kHdrTileFac];
      const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
      for (int k = wave; k < nk; k += kTileThreads / 64) {
        const int32_t* e = lst + __builtin_amdgcn_readfirstlane(lst[k]);
        const int nt = __builtin_amdgcn_readfirstlane(e[0]);
        cpx<T> w{T(1), T(0)};
        for (int q = 0; q < nt; ++q) {
          const int32_t* tm = e + 1 + q * (2 + 2 * WT);
          const uint32_t olo = (uint32_t)__builtin_amdgcn_readfirstlane(tm[0]);
          const uint32_t ohi = (uint32_t)__builtin_amdgcn_readfirstlane(tm[1]);
          const uint64_t om = ((uint64_t)ohi << 32) | olo;
          const cpx<T> rr{aux_real<T>(tm, 2), aux_real<T>(tm, 2 + WT)};
          const cpx<T> wn = cmul(rr, w);
          const bool on = (base & om) == om;  // uniform condition
          w.x = on ? wn.x : w.x;
          w.y = on ? wn.y : w.y;
        }
        if ((threadIdx.x & 63) == 0) tfac[k] = w;
      }
      __syncthreads();
    }
  }
  for (int r = 0; r < nrounds; ++r) {
    const int32_t* rb = pass + roff[r];
    const int nlayers = rb[0];
    const uint32_t free_mask = (uint32_t)rb[1];
    // The LDS offset of combination m is the XOR of the offsets of its
    // register bits (deposit and swizzle are XOR-linear): walking m in
    // Gray-code order takes one XOR per amplitude.
    uint32_t bofs[RB];
#pragma unroll
    for (int j = 0; j < RB; ++j) bofs[j] = (uint32_t)rb[2 + j];
    // A store map moves amplitudes between register groups, so every
    // group's load comes before any store.
    const int moff = rb[kHdrMap];
    static_assert((1 << (TBMAX - RB)) <= kTileThreads, "at most one register group per thread");
    const int gi = threadIdx.x;
    cpx<T> a[NR];
    uint32_t sgb = 0;  // LDS offset of the group's combination 0
    if (gi < ng) {
      // deposit gi into the free local bits
      uint32_t lg = 0, fm = free_mask;
      for (int bit = 0; fm; ++bit) {
        const uint32_t low = fm & (0u - fm);
        if ((gi >> bit) & 1) lg |= low;
        fm ^= low;
      }
      sgb = tile_swizzle(lg, SB) * (uint32_t)sizeof(cpx<T>);
      {
        uint32_t ad = sgb;
#pragma unroll
        for (int i = 0; i < NR; ++i) {
          if (i > 0) ad ^= bofs[__builtin_ctz(i)];
          a[i ^ (i >> 1)] = *reinterpret_cast<const cpx<T>*>(tb + ad);
        }
      }


      // A record's table follows it, so that its address does not wait for
      // a word of the record.
      const int32_t* __restrict__ rec = rb + kRoundHeader;
      int32_t wn[LR];
#pragma unroll
      for (int i = 0; i < LR; ++i) wn[i] = rec[i];
      for (int o = 0; o < nlayers; ++o) {
        int32_t w[LR];
#pragma unroll
        for (int i = 0; i < LR; ++i) w[i] = wn[i];
        const int flags = w[0];
        const int32_t* __restrict__ tab = rec + LR;
        rec += LR + ((flags & LT_TAB) ? kTableWords : 0);
        // The next record's words are loaded while this layer runs.  After
        // the last layer they are the round's aux words, the next block or
        // the buffer's slack past the program's end (kProgSlackBytes), and
        // are not used.
#pragma unroll
        for (int i = 0; i < LR; ++i) wn[i] = rec[i];
        const int32_t* __restrict__ ap = rb + w[3];  // aux words of the record
        int p = 0;
        if (flags & LT_TAB) table_step<T, RB>(a, tab);
        if (flags & LT_CZR) {
          const uint32_t pairs = (uint32_t)w[2];
#define QSV_CZR(J, K) \
  if ((K) < RB && ((pairs >> cz_pair_index(J, K)) & 1u)) cz_pair<T, RB, J, ((K) < RB ? (K) : (J) + 1)>(a);
          QSV_CZR(0, 1)
          QSV_CZR(0, 2)
          QSV_CZR(1, 2)
          QSV_CZR(0, 3)
          QSV_CZR(1, 3)
          QSV_CZR(2, 3)
          QSV_CZR(0, 4)
          QSV_CZR(1, 4)
          QSV_CZR(2, 4)
          QSV_CZR(3, 4)
#undef QSV_CZR
        }
        if (flags & LT_CZF) {
          // per-lane parity of the conditions for each register bit first,
          // then one pass over the amplitudes per bit that has entries
          const int ne = ap[p++];
          uint32_t zm = 0, jm = 0;
          for (int e = 0; e < ne; ++e) {
            const int ew = ap[p++];
            const int j = ew & 15, val = ew >> 8;
            const uint32_t on = ((ew >> 4) & 15) == TK_FREE ? (lg >> val) & 1u : (uint32_t)((base >> val) & 1ull);
            zm ^= on << j;
            jm |= 1u << j;
          }
#define QSV_CZF(J) \
  if ((J) < RB && ((jm >> (J)) & 1u)) cond_z<T, RB, ((J) < RB ? (J) : 0)>(a, ((zm >> (J)) & 1u) ? T(-2) : T(0));
          QSV_CZF(0)
          QSV_CZF(1)
          QSV_CZF(2)
          QSV_CZF(3)
          QSV_CZF(4)
#undef QSV_CZF
        }
        if (flags & LT_SIGN) {
          int par = 0;
          const int nd = ap[p++];
          for (int q = 0; q < nd; ++q, p += 2)
            par ^= __popc(lg & (lg >> ap[p]) & (uint32_t)ap[p + 1]);
          const int nfc = ap[p++];
          for (int q = 0; q < nfc; ++q, p += 2)
            par ^= (int)(((base >> ap[p]) & 1ull) & ((lg >> ap[p + 1]) & 1u));
          const int ncc = ap[p++];
          for (int q = 0; q < ncc; ++q, p += 2)
            par ^= (int)((base >> ap[p]) & (base >> ap[p + 1]) & 1ull);
          const T cg = (par & 1) ? T(-2) : T(0);  // per lane
#pragma unroll
          for (int m = 0; m < NR; ++m) scale1(a[m], cg);
        }
        if (flags & LT_PHASEL) {
          {
            const int j = ap[p], slot = ap[p + 1], unit = ap[p + 2], nt = ap[p + 3];
            p += 4;
            cpx<T> w{T(1), T(0)};
            if (slot >= 0) w = tfac[slot];  // uniform address: one broadcast read
            if (nt < 0) {
              // lane-table form: the group's terms as two table entries
              const int e0 = ap[p++];
              const cpx<T> f = cmul(lt[e0 + (gi & 15)], lt[e0 + 16 + ((gi >> 4) & 15)]);
              w = cmul(f, w);
            }
            for (int q = 0; q < nt; ++q, p += 3 + 2 * WT) {
              // every word read before the lane condition (scalar loads; a
              // read inside the divergent branch became a vector load that
              // waited for the next tile's prefetch), then a select
              const uint32_t lgm = (uint32_t)ap[p];
              const uint64_t om = ((uint64_t)(uint32_t)ap[p + 2] << 32) | (uint32_t)ap[p + 1];
              const cpx<T> rr{aux_real<T>(ap, p + 3), aux_real<T>(ap, p + 3 + WT)};
              const bool on = ((lg & lgm) == lgm) & ((base & om) == om);
              const cpx<T> wn = cmul(rr, w);
              w.x = on ? wn.x : w.x;
              w.y = on ? wn.y : w.y;
            }
            // one in-place complex product per amplitude (a single body: two
            // alternative bodies made the compiler keep a second copy of the
            // amplitudes); a pure phase is renormalised first, so that the
            // rounding of the factor product cannot change the norm
            T zr = w.x, zi = w.y;
            if (unit) {
              const T inv = inv_sqrt(w.x * w.x + w.y * w.y);
              zr *= inv;
              zi *= inv;
            }
#pragma unroll
            for (int m = 0; m < NR; ++m)
              if (j < 0 || ((m >> j) & 1)) cmul_lane(a[m], zr, zi);
          }
        }
        if (BODY == kBodyFull && (flags & LT_RAWD)) {
          // a diagonal factor d = (1 + c) exp(i phi) per operand value, as
          // (p, q, c) triples: PHASE1 two (by the qubit's bit), DIAG2 four
          const int type = ap[p], ka = ap[p + 1], va = ap[p + 2];
          const int kb = type == RAW_DIAG2 ? ap[p + 3] : TK_REG;
          const int vb = type == RAW_DIAG2 ? ap[p + 4] : 0;
          const int f0 = p + (type == RAW_DIAG2 ? 5 : 3);
          const uint32_t ma = ka == TK_REG ? (uint32_t)va : (const_bit(ka, va, lg, base) ? ~0u : 0u);
          const uint32_t mb = kb == TK_REG ? (uint32_t)vb : (const_bit(kb, vb, lg, base) ? ~0u : 0u);
          const int nfac = type == RAW_DIAG2 ? 4 : 2;
          p = f0 + 3 * nfac * WT;
          T fp[4], fq[4], fc[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int at = f0 + 3 * (e < nfac ? e : 0) * WT;
            fp[e] = aux_real<T>(ap, at);
            fq[e] = aux_real<T>(ap, at + WT);
            fc[e] = aux_real<T>(ap, at + 2 * WT);
          }
#pragma unroll
          for (int m = 0; m < NR; ++m) {
            const int sel = (int)((ma >> m) & 1u) + 2 * (int)((mb >> m) & 1u);  // per lane
            const T pm = sel == 0 ? fp[0] : sel == 1 ? fp[1] : sel == 2 ? fp[2] : fp[3];
            const T qm = sel == 0 ? fq[0] : sel == 1 ? fq[1] : sel == 2 ? fq[2] : fq[3];
            const T cm = sel == 0 ? fc[0] : sel == 1 ? fc[1] : sel == 2 ? fc[2] : fc[3];
            phase_shears(a[m], pm, qm);
            scale1(a[m], cm);
          }
        }
        // rotations on register bits, ascending
#define QSV_ROT(J)                                                                    \
  if ((J) < RB && (flags & (LT_ROT0 << (J)))) {                                       \
    const T pj = rec_real<T>(w, kRecRot + 2 * (J) * WT);                              \
    const T qj = rec_real<T>(w, kRecRot + (2 * (J) + 1) * WT);                        \
    shears<T, RB, ((J) < RB ? (J) : 0)>(a, pj, qj, (flags & (LT_SHEAR3 << (J))) != 0); \
  }
        QSV_ROT(0)
        QSV_ROT(1)
        QSV_ROT(2)
        QSV_ROT(3)
        QSV_ROT(4)
#undef QSV_ROT
        if (BODY >= kBodyPerm && (flags & LT_PERM2)) {
          // A CNOT or SWAP of two register bits is a linear map m -> P m of
          // the register index.  Each amplitude goes through the group's own
          // LDS slots (no other thread touches them during the round): a[m]
          // is written to the slot of P m, whose address walks the images of
          // the register bits, then every slot is read back in order.  Static
          // register indices only: a runtime choice among register
          // permutations made the compiler keep a second copy of the group.
          const int j0 = ap[p], j1 = ap[p + 1], code = ap[p + 2];
          p += 3;
          {
            uint32_t pb[RB];
            perm_images<RB>(bofs, code, j0, j1, pb);
            uint32_t ad = sgb;
            asm volatile("" : "+v"(ad));
#pragma unroll
            for (int i = 0; i < NR; ++i) {
              if (i > 0) ad ^= pb[__builtin_ctz(i)];
              *reinterpret_cast<cpx<T>*>(tb + ad) = a[i ^ (i >> 1)];
            }
            ad = sgb;
            asm volatile("" : "+v"(ad));
#pragma unroll
            for (int i = 0; i < NR; ++i) {
              if (i > 0) ad ^= bofs[__builtin_ctz(i)];
              a[i ^ (i >> 1)] = *reinterpret_cast<const cpx<T>*>(tb + ad);
            }
          }
        }
        if (BODY == kBodyFull && (flags & LT_U2)) {
          const int j0 = ap[p], j1 = ap[p + 1];
          M4<T> U;
#pragma unroll
          for (int e = 0; e < 16; ++e)
            U.m[e] = cpx<T>{aux_real<T>(ap, p + 2 + 2 * e * WT), aux_real<T>(ap, p + 2 + (2 * e + 1) * WT)};
          p += 2 + 32 * WT;
          dispatch_u2<T, RB>(a, j0, j1, U);
        }
        if (BODY == kBodyFull && (flags & LT_U1)) {
          const int j = ap[p];
          M2<T> U;
#pragma unroll
          for (int e = 0; e < 4; ++e)
            U.m[e] = cpx<T>{aux_real<T>(ap, p + 1 + 2 * e * WT), aux_real<T>(ap, p + 1 + (2 * e + 1) * WT)};
          dispatch_u1<T, RB>(a, j, U);
        }
      }
    }
    if (moff) __syncthreads();
    if (gi < ng) {
      // the store's offset of the group's combination 0: as loaded, or its
      // image under the store map (the XOR of the images of the group's
      // free bits and of the tile's outside bits)
      uint32_t sgs = sgb;
      if (moff) {
        sgs = 0;
        const int32_t* __restrict__ mp = rb + moff;
        const int nf = __popc(free_mask);
        for (int i = 0; i < nf; ++i)
          if ((gi >> i) & 1) sgs ^= (uint32_t)mp[i];
        const int32_t* __restrict__ ob = mp + nf;
        const int no = ob[0];
        for (int k = 0; k < no; ++k)
          if ((base >> ob[1 + 2 * k]) & 1ull) sgs ^= (uint32_t)ob[2 + 2 * k];
      }
      // recomputed rather than kept from the load walk: 2^RB live
      // addresses would cost as many registers
      // the store's offsets (the header's; a permutation that ends the
      // round is folded into them)
      uint32_t sofs[RB];
#pragma unroll
      for (int j = 0; j < RB; ++j) sofs[j] = (uint32_t)rb[kHdrStore + j];
      uint32_t ad = sgs;
      asm volatile("" : "+v"(ad));
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        if (i > 0) ad ^= sofs[__builtin_ctz(i)];
        *reinterpret_cast<cpx<T>*>(tb + ad) = a[i ^ (i >> 1)];
      }
    }
    __syncthreads();
  }

}

// What one call of the tile body does around the rounds: take the tile from
// the state (or build |0...0> in it), write it back, and/or accumulate the
// FP64 value of sum_t c_t <Z-string_t> over the tile's amplitudes.
struct TileIO {
  int init;             // tile starts as the part of |0...0> (no load)
  int store;            // write the tile back to the state
  int reduce;           // accumulate the Z-string sum
  const uint64_t* z;    // Z masks of the terms (reduce)
  const uint32_t* zl;   // the same over the pass's local bits (bit j: qubit S[j])
  const double* coef;   // coefficients (reduce)
  int nt;
};

// A 16-byte vector of amplitudes (two complex64 or one complex128) as a
// native vector type, moved between registers and the swizzled LDS tile.
template <typename T>
struct StageVec;
template <>
struct StageVec<float> {
  using V = float4;
  __device__ static void put(cpx<float>* tile, int sb, uint32_t l, const V& v) {
    tile[tile_swizzle(l, sb)] = cpx<float>{v.x, v.y};
    tile[tile_swizzle(l + 1, sb)] = cpx<float>{v.z, v.w};
  }
  __device__ static V get(const cpx<float>* tile, int sb, uint32_t l) {
    const cpx<float> a = tile[tile_swizzle(l, sb)], b = tile[tile_swizzle(l + 1, sb)];
    return V{a.x, a.y, b.x, b.y};
  }
};
template <>
struct StageVec<double> {
  using V = double2;
  __device__ static void put(cpx<double>* tile, int sb, uint32_t l, const V& v) {
    tile[tile_swizzle(l, sb)] = cpx<double>{v.x, v.y};
  }
  __device__ static V get(const cpx<double>* tile, int sb, uint32_t l) {
    const cpx<double> a = tile[tile_swizzle(l, sb)];
    return V{a.x, a.y};
  }
};

// Z-string sum over one tile, sum_x |psi_x|^2 sum_q coef_q (-1)^popc(x & z_q),
// in FP64, for a pass whose tile is not stored afterwards (its LDS slots are
// reused).  Thread j owns the local indices l = j + 256 k.  The parity of
// x & z_q splits into the tile's outside bits (uniform), the bits of j and
// those of k, so after an in-place Walsh-Hadamard transform of the thread's
// probabilities over k, H[m] = sum_k P[k] (-1)^popc(k & m), every term costs
// one LDS read: coef_q * (+-1) * H[(local mask of z_q) >> 8].  Returns the
// thread's partial.
template <typename T, int TBMAX>
__device__ __forceinline__ double tile_zsum(cpx<T>* __restrict__ tile, int t, uint64_t base, const TileIO& io) {
  constexpr int SB = SwzBits<T>::B;
  constexpr int KMAX = (1 << TBMAX) / kTileThreads;  // slots per thread: 32 (c64), 16 (c128)
  constexpr int KL = 8;                               // transform bits done in registers at once
  static_assert(KMAX % KL == 0, "whole register blocks per thread");
  const uint32_t j = threadIdx.x;
  const int kn = t > 8 ? 1 << (t - 8) : 1;  // amplitudes per thread
  if (j >= (1u << t)) return 0.0;          // tiles under 256 amplitudes
  auto slot = [&](int k) -> double* {
    return reinterpret_cast<double*>(&tile[tile_swizzle(j + (uint32_t)k * kTileThreads, SB)]);
  };
  // the transform over the low 3 bits of k, from the amplitudes (slots past
  // kn hold zeros, so the full-size transform gives H[m] for m < kn) ...
#pragma unroll 1
  for (int kh = 0; kh < KMAX / KL; ++kh) {
    double h[KL];
#pragma unroll
    for (int e = 0; e < KL; ++e) {
      const int k = kh * KL + e;
      h[e] = 0.0;
      if (k < kn) {
        const cpx<T> x = tile[tile_swizzle(j + (uint32_t)k * kTileThreads, SB)];
        h[e] = fma((double)x.x, (double)x.x, (double)x.y * (double)x.y);
      }
    }
#pragma unroll
    for (int b = 1; b < KL; b <<= 1)
#pragma unroll
      for (int e = 0; e < KL; ++e)
        if (!(e & b)) {
          const double u = h[e], v = h[e | b];
          h[e] = u + v;
          h[e | b] = u - v;
        }
#pragma unroll
    for (int e = 0; e < KL; ++e) *slot(kh * KL + e) = h[e];
  }
  // ... then over the high bits, column by column
  if constexpr (KMAX > KL) {
#pragma unroll 1
    for (int e = 0; e < KL; ++e) {
      double h[KMAX / KL];
#pragma unroll
      for (int kh = 0; kh < KMAX / KL; ++kh) h[kh] = *slot(kh * KL + e);
#pragma unroll
      for (int b = 1; b < KMAX / KL; b <<= 1)
#pragma unroll
        for (int kh = 0; kh < KMAX / KL; ++kh)
          if (!(kh & b)) {
            const double u = h[kh], v = h[kh | b];
            h[kh] = u + v;
            h[kh | b] = u - v;
          }
#pragma unroll
      for (int kh = 0; kh < KMAX / KL; ++kh) *slot(kh * KL + e) = h[kh];
    }
  }
  double acc = 0.0;
  for (int q = 0; q < io.nt; ++q) {
    const uint32_t zl = io.zl[q];
    const int par = (__popcll(base & io.z[q]) + __popc(j & zl & 255u)) & 1;
    acc = fma(par ? -io.coef[q] : io.coef[q], *slot((int)(zl >> 8)), acc);
  }
  return acc;
}

// One fused tile pass over tile `tid` of the pass program `prog`; returns the
// thread's partial of the Z-string sum (0 unless io.reduce).  Ends with a
// barrier so that the caller can start another tile at once.  BODY selects
// the steps compiled in (kBodyLean: tables, magnitudes, signs, per-group
// phases and rotations; kBodyPerm: those and register permutations;
// kBodyFull: every step): the host picks the smallest body a pass needs,
// since fewer registers let more workgroups share a compute unit and the
// full body spills.
template <typename T, int TBMAX, int RB, int BODY, bool GROUPED = true>
__device__ __forceinline__ double tile_body(const cpx<T>* src, cpx<T>* dst, const int32_t* __restrict__ prog,
                                            uint64_t tid, const TileIO& io) {
  constexpr int A = VecInfo<T>::A;
  constexpr int NR = 1 << RB;
  constexpr int VPT = (1 << TBMAX) / A / kTileThreads;  // 16-byte vectors per thread
  constexpr int SB = SwzBits<T>::B;
  constexpr int WT = WordsPer<T>::W;                      // words per real
  __shared__ cpx<T> tile[1 << TBMAX];
  __shared__ uint64_t segoff[1 << (TBMAX - 4)];
  const int t = prog[0], c = prog[1], nns = prog[2];
  const int32_t* S = prog + 4;
  const int32_t* nonS = S + t;
  uint64_t base = 0;
  for (int i = 0; i < nns; ++i) base |= ((tid >> i) & 1ull) << nonS[i];
  const int nseg = 1 << (t - c);
  for (int h = threadIdx.x; h < nseg; h += kTileThreads) {
    uint64_t o = 0;
    for (int j = 0; j < t - c; ++j)
      if ((h >> j) & 1) o |= 1ull << S[c + j];
    segoff[h] = o;
  }
  __shared__ cpx<T> ltab[LaneTab<T>::N];
  stage_lane_table<T>(prog, ltab);
  __syncthreads();

  // ---- load the tile (coalesced 16-byte vectors) into LDS
  const vec16<T>* gv = reinterpret_cast<const vec16<T>*>(src);
  vec16<T>* gw = reinterpret_cast<vec16<T>*>(dst);
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
    // GROUPED: every load in flight before the first LDS write.  Every lane
    // issues every load (an index past a smaller tile repeats one of its
    // vectors, whose value is not used), so the compiler does not wait after
    // each.  The batch kernel's full body has no registers to spare for a
    // group and loads one vector at a time.
    using V = typename StageVec<T>::V;
    const V* __restrict__ gq = reinterpret_cast<const V*>(src);
    constexpr int G = GROUPED ? VPT : 1;
#pragma unroll
    for (int k0 = 0; k0 < VPT; k0 += G) {
      V xs[G];
#pragma unroll
      for (int k = 0; k < G; ++k) {
        const int i = threadIdx.x + (k0 + k) * kTileThreads;
        const uint32_t l = (uint32_t)(i < nvec ? i : (i & (nvec - 1))) * A;
        xs[k] = gq[(base | segoff[l >> c] | (l & cmask)) / A];
      }
#pragma unroll
      for (int k = 0; k < G; ++k) {
        const int i = threadIdx.x + (k0 + k) * kTileThreads;
        if (i < nvec) StageVec<T>::put(tile, SB, (uint32_t)i * A, xs[k]);
      }
    }
  }
  __syncthreads();

  // ---- rounds
  run_rounds<T, TBMAX, RB, BODY>(reinterpret_cast<char*>(tile), prog, t, nns, base, ltab);

  // ---- Z-string sum over the tile (FP64)
  double acc = 0.0;
  if (io.reduce) acc = tile_zsum<T, TBMAX>(tile, t, base, io);  // no store follows a reduce

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
        gw[g / A] = x;
      }
    }
  }
  __syncthreads();
  return acc;
}

// One workgroup per tile, reading the tile from src and writing it to dst:
// the same pointer for a pass in place; distinct buffers for the race check
// of the fused plans (plan option race_check), which runs each pass out of
// place first and compares.
template <typename T, int TBMAX, int RB, int BODY, int MINWG>
__global__ __launch_bounds__(kTileThreads, MINWG) void k_tile(const cpx<T>* src, cpx<T>* dst,
                                                              const int32_t* __restrict__ prog) {
  const TileIO io{0, 1, 0, nullptr, nullptr, nullptr, 0};
  (void)tile_body<T, TBMAX, RB, BODY>(src, dst, prog, blockIdx.x, io);
}

// Pipelined tile pass for one state.  A persistent workgroup walks the tiles
// blockIdx.x, blockIdx.x + gridDim.x, ...  While the rounds of one tile run,
// each thread already has
// its share of the next tile in flight from HBM into registers (VPT 16-byte
// vectors: 64 VGPRs for a 64 KiB tile), so that HBM traffic overlaps the
// arithmetic instead of alternating with it.  The rounds read their program
// with scalar loads only, so no wait inside them covers those vector loads
// (which complete in order).  Used for lean passes over tiles of exactly
// 2^TBMAX amplitudes.
template <typename T, int TBMAX, int RB, int BODY, int MINWG>
__global__ __launch_bounds__(kTileThreads, MINWG) void k_tile_pipe(cpx<T>* __restrict__ psi,
                                                                   const int32_t* __restrict__ prog,
                                                                   uint64_t ntiles) {
  constexpr int A = VecInfo<T>::A;
  constexpr int VPT = (1 << TBMAX) / A / kTileThreads;
  constexpr int SB = SwzBits<T>::B;
  constexpr int CMIN = 4;  // every pass keeps at least the low 4 qubits contiguous (128- or 256-byte segments)
  __shared__ cpx<T> tile[1 << TBMAX];
  __shared__ uint64_t segoff[1 << (TBMAX - CMIN)];
  const int t = prog[0], c = prog[1], nns = prog[2];
  const int32_t* S = prog + 4;
  const int32_t* nonS = S + t;
  const int nseg = 1 << (t - c);
  for (int h = threadIdx.x; h < nseg; h += kTileThreads) {
    uint64_t o = 0;
    for (int j = 0; j < t - c; ++j)
      if ((h >> j) & 1) o |= 1ull << S[c + j];
    segoff[h] = o;
  }
  __shared__ cpx<T> ltab[LaneTab<T>::N];
  stage_lane_table<T>(prog, ltab);
  __syncthreads();

  // 16-byte vectors as native vector types (kept in registers)
  using V = typename StageVec<T>::V;
  const V* gv = reinterpret_cast<const V*>(psi);
  V* gw = reinterpret_cast<V*>(psi);
  const uint32_t cmask = (1u << c) - 1u;
  auto tile_base = [&](uint64_t tid) {
    uint64_t base = 0;
    for (int i = 0; i < nns; ++i) base |= ((tid >> i) & 1ull) << nonS[i];
    return base;
  };
  V stage[VPT];
  auto fetch = [&](uint64_t tid) {
    const uint64_t base = tile_base(tid);
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
      const uint32_t l = (uint32_t)(threadIdx.x + k * kTileThreads) * A;
      stage[k] = gv[(base | segoff[l >> c] | (l & cmask)) / A];
    }
  };

  auto put = [&]() {
#pragma unroll
    for (int k = 0; k < VPT; ++k)
      StageVec<T>::put(tile, SB, (uint32_t)(threadIdx.x + k * kTileThreads) * A, stage[k]);
  };
  // The loop is rotated so that every iteration issues the next tile's loads
  // before this tile's stores: waiting for the loads then never waits for
  // the stores (memory operations are counted in issue order).
  uint64_t tid = blockIdx.x;
  if (tid >= ntiles) return;
  fetch(tid);
  put();
  __syncthreads();
  if (tid + gridDim.x < ntiles) fetch(tid + gridDim.x);
  for (;;) {
    const uint64_t base = tile_base(tid);
    run_rounds<T, TBMAX, RB, BODY>(reinterpret_cast<char*>(tile), prog, t, nns, base, ltab);
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
      const uint32_t l = (uint32_t)(threadIdx.x + k * kTileThreads) * A;
      gw[(base | segoff[l >> c] | (l & cmask)) / A] = StageVec<T>::get(tile, SB, l);
    }
    __syncthreads();
    tid += gridDim.x;
    if (tid >= ntiles) break;
    put();
    __syncthreads();
    if (tid + gridDim.x < ntiles) fetch(tid + gridDim.x);  // in flight during the rounds
  }
}

// ------------------------------------------------------ qubit permutation
// One HBM pass that relabels qubits by an involution sigma of the index bits:
// out[y] = in[sigma(y)], where sigma(y) moves bit q of y to bit sigma(q).
// The pass's qubit set S (t qubits) holds the low c qubits and is closed
// under sigma, so sigma maps the tile (S, b) onto the tile (S, sigma(b)) and
// local index l onto pi(l).  The pair of tiles {tid, sigma(tid)} belongs to
// the smaller id of the two (a tile that sigma fixes is taken alone): the
// workgroup reads both into LDS, then writes each into the other's place
// with its local index permuted.  Every amplitude is read and written once,
// and no other workgroup touches the pair.  Workgroups are persistent (one
// launch of resident workgroups walks the tile ids), so the half of the ids
// that are not pair leaders cost a test, not a workgroup dispatch.  Small
// tiles (16 KiB per pair) let eight workgroups share a compute unit; that
// concurrency, not prefetching within a workgroup, keeps HBM busy (a
// variant that loaded the next pair into registers during the stores ran
// 25% slower: its joins made the compiler wait for the loads early).
template <typename T>
__global__ __launch_bounds__(kTileThreads) void k_qperm(const cpx<T>* src, cpx<T>* dst,
                                                        const int32_t* __restrict__ prog) {
  constexpr int A = VecInfo<T>::A;
  constexpr int TP = QpermCfg<T>::TP;
  constexpr int SB = SwzBits<T>::B;
  constexpr int VPT = (1 << TP) / A / kTileThreads;
  __shared__ cpx<T> lds[2][1 << TP];
  __shared__ uint64_t segoff[1 << (TP - 4)];
  __shared__ uint32_t pl[2][64];
  const int t = prog[0], c = prog[1], nns = prog[2];
  const int32_t* S = prog + 4;
  const int32_t* nonS = S + t;
  const int32_t* pil = nonS + nns;
  const int32_t* pin = pil + t;
  const int nseg = 1 << (t - c);
  for (int h = threadIdx.x; h < nseg; h += kTileThreads) {
    uint64_t o = 0;
    for (int j = 0; j < t - c; ++j)
      if ((h >> j) & 1) o |= 1ull << S[c + j];
    segoff[h] = o;
  }
  // pi(l) = pl[0][l & 63] ^ pl[1][l >> 6] (a bit permutation is XOR-linear)
  for (int v = threadIdx.x; v < 128; v += kTileThreads) {
    const int half = v >> 6, x = v & 63;
    uint32_t o = 0;
    for (int k = 0; k < 6; ++k) {
      const int b = 6 * half + k;
      if (((x >> k) & 1) && b < t) o |= 1u << pil[b];
    }
    pl[half][x] = o;
  }
  __syncthreads();
  const uint32_t cmask = (1u << c) - 1u;
  const int nvec = (1 << t) / A;
  const vec16<T>* gv = reinterpret_cast<const vec16<T>*>(src);
  vec16<T>* gw = reinterpret_cast<vec16<T>*>(dst);
  const uint64_t ntiles = 1ull << nns;
  for (uint64_t tid = blockIdx.x; tid < ntiles; tid += gridDim.x) {
    uint64_t tid2 = 0;
    for (int i = 0; i < nns; ++i) tid2 |= ((tid >> i) & 1ull) << pin[i];
    if (tid2 < tid) continue;  // uniform: the partner's workgroup takes the pair
    uint64_t base = 0, base2 = 0;
    for (int i = 0; i < nns; ++i) {
      base |= ((tid >> i) & 1ull) << nonS[i];
      base2 |= ((tid2 >> i) & 1ull) << nonS[i];
    }
    const bool pair = tid2 != tid;
    // all of the thread's loads in flight before the first LDS write; every
    // lane issues every load (an index past a smaller tile repeats one of its
    // vectors, whose value is not used), so the compiler does not wait after
    // each
    using V = typename StageVec<T>::V;
    const V* __restrict__ gq = reinterpret_cast<const V*>(src);
    V xs[VPT], ys[VPT];
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
      const int i = threadIdx.x + k * kTileThreads;
      const uint32_t l = (uint32_t)(i < nvec ? i : (i & (nvec - 1))) * A;
      const uint64_t off = segoff[l >> c] | (l & cmask);
      xs[k] = gq[(base | off) / A];
      if (pair) ys[k] = gq[(base2 | off) / A];
    }
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
      const int i = threadIdx.x + k * kTileThreads;
      if (i < nvec) {
        StageVec<T>::put(lds[0], SB, (uint32_t)i * A, xs[k]);
        if (pair) StageVec<T>::put(lds[1], SB, (uint32_t)i * A, ys[k]);
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nvec; i += kTileThreads) {
      const uint32_t l = (uint32_t)i * A;
      const uint64_t off = segoff[l >> c] | (l & cmask);
      vec16<T> x, y;
#pragma unroll
      for (int e = 0; e < A; ++e) {
        const uint32_t src = tile_swizzle(pl[0][(l + e) & 63] ^ pl[1][(l + e) >> 6], SB);
        x.a[e] = lds[0][src];
        if (pair) y.a[e] = lds[1][src];
      }
      // the partner tile takes this tile's amplitudes (a fixed tile its own)
      gw[(base2 | off) / A] = x;
      if (pair) gw[(base | off) / A] = y;
    }
    __syncthreads();  // the LDS is reused by the next pair
  }
}

// Workgroups of k_qperm that fit the device at once (cached per device).
template <typename T>
static int qperm_grid() {
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (cache[dev] == 0) {
    int per_cu = 0, ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_qperm<T>, kTileThreads, 0) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return 0;
    cache[dev] = std::max(1, per_cu * ncu);
  }
  return cache[dev];
}

// ------------------------------------------------------------ batches
// Every tile of one pass of one batched circuit (state at psi), lean body,
// by one workgroup: the segment table once per pass, and each thread's share
// of the next tile loading into registers while the current tile's rounds
// run (a batch often has about one workgroup per compute unit, so other
// workgroups do not hide the load latency).  The first pass builds |0...0> in the tile
// instead of loading; the last reduces the Z-string sum instead of storing.
// Returns the thread's partial of that sum.
template <typename T, int TBMAX, int RB>
__device__ __forceinline__ double batch_pass(cpx<T>* __restrict__ psi, const int32_t* __restrict__ prog,
                                             uint64_t ntiles, const TileIO& io) {
  constexpr int A = VecInfo<T>::A;
  constexpr int VPT = (1 << TBMAX) / A / kTileThreads;  // 16-byte vectors per thread
  constexpr int PF = VPT;                               // of which prefetched
  constexpr int SB = SwzBits<T>::B;
  using V = typename StageVec<T>::V;
  __shared__ cpx<T> tile[1 << TBMAX];
  __shared__ uint64_t segoff[1 << (TBMAX - 4)];
  const int t = prog[0], c = prog[1], nns = prog[2];
  const int32_t* S = prog + 4;
  const int32_t* nonS = S + t;
  const int nseg = 1 << (t - c);
  for (int h = threadIdx.x; h < nseg; h += kTileThreads) {
    uint64_t o = 0;
    for (int j = 0; j < t - c; ++j)
      if ((h >> j) & 1) o |= 1ull << S[c + j];
    segoff[h] = o;
  }
  __shared__ cpx<T> ltab[LaneTab<T>::N];
  stage_lane_table<T>(prog, ltab);
  __syncthreads();
  V* gv = reinterpret_cast<V*>(psi);
  const int nvec = (1 << t) / A;
  const uint32_t cmask = (1u << c) - 1u;
  V stage[PF];
  double acc = 0.0;
  // Every lane issues every load of the tile whose base index is b0: an
  // index past a smaller tile repeats one of its vectors, whose value is not
  // used.  (With the loads inside per-lane branches the compiler waited for
  // every earlier memory operation, the previous tile's stores included,
  // before each load, and the prefetch ran one load at a time.)
  auto vload = [&](uint64_t b0, int k) -> V {
    const int i = threadIdx.x + k * kTileThreads;
    const uint32_t l = (uint32_t)(i < nvec ? i : (i & (nvec - 1))) * A;
    return gv[(b0 | segoff[l >> c] | (l & cmask)) / A];
  };
  if (!io.init) {
#pragma unroll
    for (int k = 0; k < PF; ++k) stage[k] = vload(0, k);
  }
  for (uint64_t tid = 0; tid < ntiles; ++tid) {
    uint64_t base = 0;
    for (int i = 0; i < nns; ++i) base |= ((tid >> i) & 1ull) << nonS[i];
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
      for (int k = 0; k < PF; ++k) {
        const int i = threadIdx.x + k * kTileThreads;
        if (i < nvec) StageVec<T>::put(tile, SB, (uint32_t)i * A, stage[k]);
      }
    }
    __syncthreads();
    if (!io.init && tid + 1 < ntiles) {  // the next tile, in flight during the rounds
      uint64_t nb = 0;
      for (int i = 0; i < nns; ++i) nb |= (((tid + 1) >> i) & 1ull) << nonS[i];
#pragma unroll
      for (int k = 0; k < PF; ++k) stage[k] = vload(nb, k);
    }
    run_rounds<T, TBMAX, RB, kBodyLean>(reinterpret_cast<char*>(tile), prog, t, nns, base, ltab);
    if (io.reduce) acc += tile_zsum<T, TBMAX>(tile, t, base, io);  // no store follows a reduce
    if (io.store) {
#pragma unroll
      for (int k = 0; k < VPT; ++k) {
        const int i = threadIdx.x + k * kTileThreads;
        if (i < nvec) {
          const uint32_t l = (uint32_t)i * A;
          gv[(base | segoff[l >> c] | (l & cmask)) / A] = StageVec<T>::get(tile, SB, l);
        }
      }
    }
    __syncthreads();
  }
  return acc;
}

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

template <typename T, int TBMAX, int RB, bool FULL>
__global__ __launch_bounds__(kTileThreads, 2) void k_batch(cpx<T>* __restrict__ scratch,
                                                         const int32_t* __restrict__ progs,
                                                         const int64_t* __restrict__ passoff,
                                                         const int64_t* __restrict__ jobs,
                                                         const uint64_t* __restrict__ zt,
                                                         const uint32_t* __restrict__ zlt,
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
      const TileIO io{p == 0, p + 1 < np, p + 1 == np, zt + t0, zlt + t0, ct + t0, (int)nt};
      if constexpr (FULL) {
        for (uint64_t tid = 0; tid < ntiles; ++tid)
          acc += tile_body<T, TBMAX, RB, kBodyFull, false>(scratch + soff, scratch + soff, prog, tid, io);
      } else {
        acc += batch_pass<T, TBMAX, RB>(scratch + soff, prog, ntiles, io);
      }
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

// Tiles of up to 2^12 complex64 / 2^11 complex128 amplitudes use a half-size
// LDS buffer; with the lean body three workgroups then share a compute unit.

// Workgroups of a kernel that fit the device at once (cached per device).
template <typename T, int TB, int RB, int BODY, int MINWG>
static int pipe_grid() {
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (cache[dev] == 0) {
    int per_cu = 0, ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_tile_pipe<T, TB, RB, BODY, MINWG>, kTileThreads, 0) !=
            hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return 0;
    cache[dev] = per_cu * ncu;
  }
  return cache[dev];
}

template <typename T, int TB, int RB, int BODY, int MINWG>
static hipError_t launch_pass(cpx<T>* psi, const int32_t* prog_dev, uint64_t ntiles, bool pipe, hipStream_t st) {
  if constexpr (TB == TileCfg<T>::TBMAX && (BODY != kBodyFull || sizeof(T) == 4)) {
    const int resident = pipe ? pipe_grid<T, TB, RB, BODY, MINWG>() : 0;
    if (resident > 0) {
      const unsigned grid = (unsigned)std::min<uint64_t>(ntiles, (uint64_t)resident);
      hipLaunchKernelGGL((k_tile_pipe<T, TB, RB, BODY, MINWG>), dim3(grid), dim3(kTileThreads), 0, st, psi,
                         prog_dev, ntiles);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((k_tile<T, TB, RB, BODY, MINWG>), dim3((unsigned)ntiles), dim3(kTileThreads), 0, st, psi, psi,
                     prog_dev);
  return hipGetLastError();
}

// The same pass out of place (src to dst), always one workgroup per tile.
template <typename T, int TB, int RB, int BODY, int MINWG>
static hipError_t launch_pass_oop(const cpx<T>* src, cpx<T>* dst, const int32_t* prog_dev, uint64_t ntiles,
                                  hipStream_t st) {
  hipLaunchKernelGGL((k_tile<T, TB, RB, BODY, MINWG>), dim3((unsigned)ntiles), dim3(kTileThreads), 0, st, src, dst,
                     prog_dev);
  return hipGetLastError();
}

// One fused tile pass.  `prog_host` is the host copy of the pass program
// (its header is read here); body is the smallest body its steps need.
template <typename T>
hipError_t launch_tile_pass(cpx<T>* psi, int n, const int32_t* prog_dev, const int32_t* prog_host, int body,
                            hipStream_t st) {
  constexpr int TB = TileCfg<T>::TBMAX, RB = TileCfg<T>::RB;
  const int t = prog_host[0], c = prog_host[1];
  const uint64_t ntiles = 1ull << (n - t);
  const bool small = t <= TB - 1;
  const int tbits = small ? TB - 1 : TB;
  // The pipelined kernel holds the next tile in registers: passes over
  // full-size tiles only (for half-size tiles the extra registers and LDS
  // cost a workgroup per compute unit, more than the overlap gains); full
  // body only for complex64 (the complex128 one would spill heavily).
  const bool pipe = (body != kBodyFull || sizeof(T) == 4) && !small && t - c <= tbits - 4;
  if (small) {
    if (body == kBodyFull) return launch_pass<T, TB - 1, RB, kBodyFull, 2>(psi, prog_dev, ntiles, pipe, st);
    if (body == kBodyPerm) return launch_pass<T, TB - 1, RB, kBodyPerm, 3>(psi, prog_dev, ntiles, pipe, st);
    return launch_pass<T, TB - 1, RB, kBodyLean, 3>(psi, prog_dev, ntiles, pipe, st);
  }
  if (body == kBodyFull) return launch_pass<T, TB, RB, kBodyFull, 2>(psi, prog_dev, ntiles, pipe, st);
  if (body == kBodyPerm) return launch_pass<T, TB, RB, kBodyPerm, 2>(psi, prog_dev, ntiles, pipe, st);
  return launch_pass<T, TB, RB, kBodyLean, 2>(psi, prog_dev, ntiles, pipe, st);
}

// One fused tile pass out of place (src to dst, for the race check).
template <typename T>
hipError_t launch_tile_pass_oop(const cpx<T>* src, cpx<T>* dst, int n, const int32_t* prog_dev,
                                const int32_t* prog_host, int body, hipStream_t st) {
  constexpr int TB = TileCfg<T>::TBMAX, RB = TileCfg<T>::RB;
  const int t = prog_host[0];
  const uint64_t ntiles = 1ull << (n - t);
  if (t <= TB - 1) {
    if (body == kBodyFull) return launch_pass_oop<T, TB - 1, RB, kBodyFull, 2>(src, dst, prog_dev, ntiles, st);
    if (body == kBodyPerm) return launch_pass_oop<T, TB - 1, RB, kBodyPerm, 3>(src, dst, prog_dev, ntiles, st);
    return launch_pass_oop<T, TB - 1, RB, kBodyLean, 3>(src, dst, prog_dev, ntiles, st);
  }
  if (body == kBodyFull) return launch_pass_oop<T, TB, RB, kBodyFull, 2>(src, dst, prog_dev, ntiles, st);
  if (body == kBodyPerm) return launch_pass_oop<T, TB, RB, kBodyPerm, 2>(src, dst, prog_dev, ntiles, st);
  return launch_pass_oop<T, TB, RB, kBodyLean, 2>(src, dst, prog_dev, ntiles, st);
}
template hipError_t launch_tile_pass_oop<float>(const cpx<float>*, cpx<float>*, int, const int32_t*, const int32_t*,
                                                int, hipStream_t);
template hipError_t launch_tile_pass_oop<double>(const cpx<double>*, cpx<double>*, int, const int32_t*,
                                                 const int32_t*, int, hipStream_t);

// One qubit-permutation pass (program: see tile.hpp, kind kPassQperm).
// src == dst for the pass in place; distinct buffers for the race check.
template <typename T>
hipError_t launch_qperm(const cpx<T>* src, cpx<T>* dst, int n, const int32_t* prog_dev, const int32_t* prog_host,
                        hipStream_t st) {
  const uint64_t ntiles = 1ull << (n - prog_host[0]);
  const int resident = qperm_grid<T>();
  const unsigned grid = (unsigned)std::min<uint64_t>(ntiles, (uint64_t)(resident > 0 ? resident : 1024));
  hipLaunchKernelGGL(k_qperm<T>, dim3(grid), dim3(kTileThreads), 0, st, src, dst, prog_dev);
  return hipGetLastError();
}
template hipError_t launch_qperm<float>(const cpx<float>*, cpx<float>*, int, const int32_t*, const int32_t*,
                                        hipStream_t);
template hipError_t launch_qperm<double>(const cpx<double>*, cpx<double>*, int, const int32_t*, const int32_t*,
                                         hipStream_t);

template <typename T>
hipError_t launch_batch(cpx<T>* scratch, const int32_t* progs, const int64_t* passoff,
                        const int64_t* jobs, const uint64_t* zt, const uint32_t* zlt, const double* ct,
                        double* out, int* counter, int njobs, int grid, bool full, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, st, counter);
  if (full)
    hipLaunchKernelGGL((k_batch<T, TileCfg<T>::TBMAX, TileCfg<T>::RB, true>), dim3(grid), dim3(kTileThreads),
                       0, st, scratch, progs, passoff, jobs, zt, zlt, ct, out, counter, njobs);
  else  // every program of the batch uses only the lean steps
    hipLaunchKernelGGL((k_batch<T, TileCfg<T>::TBMAX, TileCfg<T>::RB, false>), dim3(grid), dim3(kTileThreads),
                       0, st, scratch, progs, passoff, jobs, zt, zlt, ct, out, counter, njobs);
  return hipGetLastError();
}
template hipError_t launch_batch<float>(cpx<float>*, const int32_t*, const int64_t*, const int64_t*,
                                        const uint64_t*, const uint32_t*, const double*, double*, int*, int,
                                        int, bool, hipStream_t);
template hipError_t launch_batch<double>(cpx<double>*, const int32_t*, const int64_t*,
                                         const int64_t*, const uint64_t*, const uint32_t*, const double*,
                                         double*, int*, int, int, bool, hipStream_t);

template int tile_max_bits<float>();
template int tile_max_bits<double>();
template int tile_reg_bits<float>();
template int tile_reg_bits<double>();
template int tile_swizzle_bits<float>();
template int tile_swizzle_bits<double>();
template hipError_t launch_tile_pass<float>(cpx<float>*, int, const int32_t*, const int32_t*, int, hipStream_t);
template hipError_t launch_tile_pass<double>(cpx<double>*, int, const int32_t*, const int32_t*, int, hipStream_t);

}  // namespace qsv
