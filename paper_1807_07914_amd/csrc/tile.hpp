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
// local bits, applies the round's ops to them in registers and writes them
// back to LDS.  The other t - RB local bits ("free" bits) select the group.
// Diagonal ops may act on any qubit: for a register bit their value is a
// mask over the register index m, for a free bit it is a per-group constant,
// and for a qubit outside S it is constant over the tile (read from the tile
// base index).
//
// Program layout (int32 words):
//   pass header : t, c, n_nonS, n_rounds, S[t], nonS[n_nonS], padded to a
//                 multiple of 64 words
//   round block : exactly kRoundWords words (read by each wavefront into
//                 registers, 64 words per VGPR, and accessed with readlane):
//                 [0] n_ops  [1] free-bit mask  [2 .. 2+2^RB) swizzled LDS
//                 offsets of the register combinations m, then the ops.
//                 An op never straddles a 64-word line unless it is longer
//                 than a line.
//   op          : type, n_words, payload...
//     U1     : j, U[2x2]                     2x2 on register bit j
//     U2     : j0, j1, U[4x4]                4x4 on register bits j0 < j1 (j0 = LSB)
//     PHASE1 : kind, val, d0, d1             factor d0 / d1 by the qubit's bit
//     DIAG2  : kindA, valA, kindB, valB, d[4]  factor d[bitA + 2 bitB]
//     PERM2  : j0, j1, code                 CNOT / SWAP as a register permutation
//     SIGN   : Mrr, nf, (f, mask)*nf, nd, (d, M)*nd, zfree,
//              nrc, (q, mask)*nrc, nfc, (q, f)*nfc, ncc, (qa, qb)*ncc
//              negation pattern over m:  Mrr ^ [mask for every free bit f
//              set in the group] ^ [mask for every outside qubit q set in
//              the tile], complemented when the group parity
//              popcount(lg & zfree) + sum_d popcount(lg & (lg >> d) & M)
//              + sum_(q,f) bit(q) bit(lg, f) + sum_(qa,qb) bit(qa) bit(qb) is odd.
//   Operand kinds: 0 register (val = mask over m), 1 free (val = local bit),
//   2 outside (val = global qubit).  Matrix entries are stored in the
//   state's precision, one word per float, two words per double.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qsv {

enum TileOpType : int32_t {
  TOP_U1 = 1,
  TOP_U2 = 2,
  TOP_SIGN = 3,
  TOP_PHASE1 = 4,
  TOP_DIAG2 = 5,
  TOP_PERM2 = 6,  // j0, j1, code: register permutation on bits j0 < j1 (m = b0 + 2 b1):
                  // code 0 swaps m = 1 <-> 3 (CNOT, control j0), 1 swaps 2 <-> 3
                  // (CNOT, control j1), 2 swaps 1 <-> 2 (SWAP)
};

enum TileOperandKind : int32_t { TK_REG = 0, TK_FREE = 1, TK_OUT = 2 };

constexpr int kTileThreads = 256;
constexpr int kRoundLines = 4;                 // VGPRs per lane holding a round block
constexpr int kRoundWords = 64 * kRoundLines;  // words per round block

// XOR-linear bijection on tile-local amplitude indices that spreads
// power-of-two strides over the LDS banks: B = 5 for 8-byte amplitudes
// (32 per 256-byte bank row), B = 4 for 16-byte amplitudes.
__host__ __device__ inline uint32_t tile_swizzle(uint32_t l, int B) {
  const uint32_t M = (1u << B) - 1u;
  return l ^ ((l >> B) & M) ^ ((l >> (2 * B)) & M);
}

}  // namespace qsv
