// tile.hpp -- encoding of fused tile passes shared by the host planner and
// the tile kernel.
//
// A pass covers a set S of t qubits (the tile).  Each workgroup owns one
// tile: the 2^t amplitudes whose non-S index bits equal the workgroup's tile
// id.  The low c qubits 0..c-1 are always in S so that a tile is made of
// 2^(t-c) contiguous segments of 2^c amplitudes (coalesced HBM access).
// Local index bit j of the tile corresponds to global qubit S[j] (S sorted).
//
// The pass body is a sequence of rounds.  In a round every thread takes
// groups of 2^RB amplitudes that differ only in the round's RB "register"
// local bits, applies the round's layers to them in registers and writes
// them back to LDS.  The other t - RB local bits ("free" bits) select the
// group.  Diagonal work may involve any qubit: a register bit varies over
// the amplitudes of a group, a free bit is constant per group, and a qubit
// outside S is constant per tile (read from the tile base index).
//
// Program layout (int32 words):
//   pass header : t, c, n_nonS, n_rounds, S[t], nonS[n_nonS],
//                 round_off[n_rounds] (word offset of each round block from
//                 the start of the pass), padded to a multiple of 16 words.
//   round block : a header of kRoundHeader words: [0] n_layers, [1] free-bit
//                 mask, [2 + j] the swizzled LDS byte offset of register bit
//                 j (the offset of register combination m is the XOR of
//                 those of its bits), and in the first round block only
//                 [kHdrTileFac] the word offset (from the start of the pass)
//                 of the pass's tile-factor list, 0 if it has none, and
//                 [kHdrTileFac + 1] its number of slots K; in every round
//                 block [kHdrStore + j] the LDS byte offset the round's
//                 store uses for register bit j: the same as [2 + j], or,
//                 when a CNOT / SWAP of register bits ends the round, the
//                 offset of that bit's image, so that the store writes
//                 register combination m to the slot of P m at no cost;
//                 [kHdrMap] the word offset (from the start of the round
//                 block) of the round's store map, 0 if it has none (see
//                 below); then the n_layers layer records of
//                 LayerRec<T>::W words, each followed by its table (64 words)
//                 if it has LT_TAB; then the aux words of the records.
//                 Offsets in a record count words from the start of its round
//                 block.
//   store map   : the CNOTs that end a round (targets in the tile, controls
//                 anywhere) as one affine map of the local index, applied by
//                 the round's store: local index x of a tile with outside
//                 bits o goes to the slot of A x + B o over GF(2).  [kHdrStore
//                 + j] hold the swizzled offsets of A's columns for the
//                 register bits; the map block holds them for the free bits,
//                 one word per bit of the free-bit mask from the lowest, then
//                 n_out and n_out pairs (outside qubit, offset of B's column).
//                 Amplitudes move between register groups, so the kernel
//                 waits for every group's load before any store.
//   layer record: [0] flags, [1] unused, [2] CZ pair set
//                 (LT_CZR), [3] aux offset: the payloads of the steps LT_CZF,
//                 LT_SIGN, LT_PHASEL, LT_RAWD and LT_PERM2 / LT_U2 / LT_U1
//                 that are present follow one another from there, in this
//                 order; [kRecRot + 2 j W] p_j and [kRecRot + (2 j + 1) W] q_j
//                 of the rotation on register bit j (W words per real).  Every
//                 field has a fixed position, so the kernel reads a record
//                 with scalar loads straight into scalar registers.
//   steps, in the order a layer applies them (all optional):
//     LT_TAB    : amplitude m is multiplied by the complex factor
//                 z_m = (re, im) at entry m of the table (two words per entry
//                 for float, four for double): phases, signs and magnitudes
//                 of diagonal factors on register bits.
//     LT_CZR    : pair set P (record word 2).  For every CZ pair (j, k) in P (bit
//                 cz_pair_index(j, k)), amplitudes with register bits j and
//                 k both set change sign.
//     LT_CZF    : aux n, then n words j | kind << 4 | val << 8.  Amplitudes
//                 with register bit j set change sign when the operand
//                 (kind 1: free local bit val of the group, kind 2: outside
//                 qubit val of the tile) is 1: a CZ between a register
//                 qubit and a qubit that is constant over the group.
//     LT_SIGN   : aux nd, (d, M)*nd, nfc, (q, f)*nfc, ncc, (qa, qb)*ncc.
//                 Every amplitude of the group changes sign when the group
//                 parity sum_d popcount(lg & (lg >> d) & M)
//                 + sum_(q,f) bit(q) bit(lg, f) + sum_(qa,qb) bit(qa) bit(qb)
//                 is odd (CZs among free bits and outside qubits).
//     LT_PHASEL : aux j, slot, unit, nt, (lgmask, omask_lo, omask_hi, r)*nt:
//                 per-group factor w = f_slot (1 if slot < 0) times the
//                 product of r over the terms whose free bits lgmask are all
//                 set in the group and whose outside qubits omask are all set
//                 in the tile, applied to the amplitudes with register bit j
//                 set (every amplitude if j < 0).  unit = 1: every factor has
//                 modulus 1, so w is applied as a pure phase.  Lane-table
//                 form (nt = -1): aux j, slot, unit, -1, e: every term
//                 is on one free bit and no outside qubit, and the product
//                 over the group's terms is L[e + (g & 15)] L[e + 16 + (g >> 4)]
//                 with g the group's index over the free bits (bit k of g is
//                 the k-th free local bit, ascending) and L the pass's lane
//                 table.
//   lane table (one per pass, optional): complex entries (r) at the word
//                 offset in the first round's header word kHdrLaneTab (from
//                 the pass start), their number in word kHdrLaneTabN; the
//                 kernel copies them to LDS before its first tile, so a
//                 per-group phase step costs two LDS reads instead of a loop
//                 over its terms.
//   tile-factor list (one per pass, optional): K word offsets of the entries
//                 (from the list's start), then each entry nt,
//                 (omask_lo, omask_hi, r)*nt.  At the start of every tile,
//                 f_k = product of r over the terms of entry k whose outside
//                 qubits omask are all set in the tile: the factors of a
//                 per-group phase step that depend only on the tile, taken
//                 once per tile (K <= kMaxTileFactors) instead of once per
//                 register group.
//     LT_RAWD   : aux type, payload, for diagonal factors that may be zero:
//                 RAW_PHASE1 : kind, val, f[2]          factor f[bit of the qubit]
//                 RAW_DIAG2  : kindA, valA, kindB, valB, f[4]  factor f[bitA + 2 bitB]
//                 each factor (1 + c) exp(i phi) stored as p, q, c
//                 (p = -tan(phi / 2), q = sin(phi), |phi| <= pi/2)
//     rotations : for every flagged register bit j, ascending: p_j, q_j.
//                 In-place shears x0 += p x1, x1 += q x0 on the amplitude
//                 pairs of bit j, and a third x0 += p x1 when the three-shear
//                 flag of j is set.  Three shears with p = -tan(theta / 2),
//                 q = sin(theta) are the rotation by theta; two shears with
//                 p = -tan(theta), q = sin(theta) cos(theta) are
//                 diag(1 / cos(theta), cos(theta)) applied after that
//                 rotation, a scale the planner takes out in a later table.
//     LT_PERM2  : aux j0, j1, code  CNOT / SWAP as a register permutation on
//                 bits j0 < j1 (m = b0 + 2 b1): code 0 swaps m = 1 <-> 3
//                 (CNOT, control j0), 1 swaps 2 <-> 3 (CNOT, control j1),
//                 2 swaps 1 <-> 2 (SWAP)
//     LT_U2     : aux j0, j1, U[4x4]  4x4 on register bits j0 < j1 (j0 = LSB)
//     LT_U1     : aux j, U[2x2]       2x2 on register bit j
//   Operand kinds: 0 register (val = mask over m), 1 free (val = local bit),
//   2 outside (val = global qubit).  Reals are stored in the state's
//   precision, one word per float, two words (low, high) per double.
//
// Qubit-permutation pass (n_rounds word = kPassQperm): relabels qubits by an
// involution sigma of the qubits, out[y] = in[sigma(y)] (sigma(y) moves bit
// q of y to bit sigma(q)), in one read and one write of the state.  S holds
// the low c qubits and is closed under sigma; t is at most QpermCfg<T>::TP.
//   t, c, n_nonS, kPassQperm, S[t] (ascending), nonS[n_nonS] (the qubit of
//   each tile-id bit, in any order), pi[t] (sigma(S[k]) = S[pi[k]]),
//   pin[n_nonS] (sigma(nonS[i]) = nonS[pin[i]]), padded to a multiple of 16
//   words.
//
// Every step except the rare LT_RAWD / LT_U2 / LT_U1 updates the amplitudes
// in place with FMAs whose addend is the amplitude itself.  A layer is a
// fixed sequence of optional steps rather than one of several op kinds:
// merging several mutually exclusive op bodies made the register allocator
// keep a second copy of all amplitudes and copy them on every op.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qsv {

enum LayerFlag : int32_t {
  LT_TAB = 1 << 0,
  LT_CZR = 1 << 1,
  LT_SIGN = 1 << 2,
  LT_PHASEL = 1 << 3,
  LT_RAWD = 1 << 4,
  LT_CZF = 1 << 5,
  LT_ROT0 = 1 << 8,     // rotation on register bit j: LT_ROT0 << j
  LT_SHEAR3 = 1 << 16,  // three shears on bit j: LT_SHEAR3 << j
  LT_PERM2 = 1 << 24,
  LT_U2 = 1 << 25,
  LT_U1 = 1 << 26,
};

enum RawDiagType : int32_t { RAW_PHASE1 = 4, RAW_DIAG2 = 5 };

enum TileOperandKind : int32_t { TK_REG = 0, TK_FREE = 1, TK_OUT = 2 };

constexpr int kTileThreads = 256;
// tile-kernel bodies: the steps compiled into a kernel variant
constexpr int kBodyLean = 0;  // tables, CZ signs, group parities, per-group phases, rotations
constexpr int kBodyPerm = 1;  // those and register permutations (LT_PERM2)
constexpr int kBodyFull = 2;  // every step
constexpr int kRoundHeader = 32;  // words of a round block header
constexpr int kRecRot = 4;        // first rotation word of a layer record
constexpr int kTableWords = 64;   // words of a table
constexpr int kHdrTileFac = 8;    // round-header word of the tile-factor list offset
constexpr int kHdrStore = 10;     // round-header words of the store's register-bit offsets
constexpr int kHdrMap = 16;       // round-header word of the store map's offset (0: none)
constexpr int kMaxTileFactors = 128;  // tile-factor slots of one pass
constexpr int kHdrLaneTab = 7;        // first round's header word of the lane-table offset
constexpr int kHdrLaneTabN = 15;      // first round's header word of the lane-table entry count
constexpr int kLaneTabBytes = 8192;   // LDS of a pass's lane tables (1024 complex64 / 512 complex128)
constexpr int kPassQperm = -1;        // n_rounds word of a qubit-permutation pass

// Largest tile of a qubit-permutation pass: a pair of tiles takes 16 KiB of
// LDS, so that eight workgroups share a compute unit (the low c qubits and
// their images need at most 2c bits: 10 for complex64, 8 for complex128).
template <typename T>
struct QpermCfg {
  static constexpr int TP = sizeof(T) == 4 ? 10 : 9;
};

// words of a layer record: 4 + 2 * RB reals (RB = 5 floats, RB = 4 doubles)
template <typename T>
struct LayerRec;
template <>
struct LayerRec<float> {
  static constexpr int W = 16;
};
template <>
struct LayerRec<double> {
  static constexpr int W = 24;
};

// Index of the CZ between register bits j != k in an LT_CZR pair set:
// (0,1)=0, (0,2)=1, (1,2)=2, (0,3)=3, ... (pairs ordered by the larger bit).
__host__ __device__ constexpr int cz_pair_index(int j, int k) {
  return j < k ? k * (k - 1) / 2 + j : j * (j - 1) / 2 + k;
}
// Whether register combination m changes sign under the CZ pair set `pairs`.
__host__ __device__ inline bool cz_pairs_negate(uint32_t pairs, int m) {
  int par = 0;
  for (int k = 1; k < 8; ++k)
    for (int j = 0; j < k; ++j)
      if (((pairs >> cz_pair_index(j, k)) & 1u) && ((m >> j) & 1) && ((m >> k) & 1)) par ^= 1;
  return par != 0;
}

// XOR-linear bijection on tile-local amplitude indices that spreads
// power-of-two strides over the LDS banks: B = 5 for 8-byte amplitudes
// (32 per 256-byte bank row), B = 4 for 16-byte amplitudes.
__host__ __device__ inline uint32_t tile_swizzle(uint32_t l, int B) {
  const uint32_t M = (1u << B) - 1u;
  return l ^ ((l >> B) & M) ^ ((l >> (2 * B)) & M);
}

}  // namespace qsv
