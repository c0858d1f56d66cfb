// circuit.hip -- execution of whole gate lists (qsv_apply_circuit): the
// fusion planner and the host side of the tile-pass kernel.
//
// The paper's general algorithm (section II) optionally augments the circuit
// with SWAPs to maximise accelerated gate applications and groups gates into
// ordered super-gates that are applied as a whole; the ExaTENSOR visitor
// (section IV.B.2) caches instructions lazily and evaluates them in bulk.
// On the state vector this becomes: queue the instruction list, then
// repeatedly choose a tile qubit set S and apply, in one HBM pass, every
// queued gate that (a) acts only on S, or is diagonal, and (b) does not need
// a gate that stays queued.  Gates commute when they share no qubit, and
// diagonal gates commute with each other, which the dependency scan uses.
// Schedules depend only on the circuit's structure and are cached by a hash
// of it; matrices are filled in for every call.
#include <algorithm>
#include <atomic>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <cmath>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "plan.hpp"
#include "tile.hpp"

namespace qsv {

template <typename T>
int tile_max_bits();
// Default tile width of a single-state plan: the full LDS tile, whose lean
// passes run on the pipelined kernel (HBM traffic of the next tile overlaps
// the rounds of the current one).
template <typename T>
static int default_tile_bits() {
  return tile_max_bits<T>();
}
template <typename T>
int tile_reg_bits();
template <typename T>
hipError_t launch_tile_pass(cpx<T>* psi, int n, const int32_t* prog_dev, const int32_t* prog_host, int body,
                            hipStream_t st);
template <typename T>
hipError_t launch_qperm(const cpx<T>* src, cpx<T>* dst, int n, const int32_t* prog_dev, const int32_t* prog_host,
                        hipStream_t st);
template <typename T>
hipError_t launch_tile_pass_oop(const cpx<T>* src, cpx<T>* dst, int n, const int32_t* prog_dev,
                                const int32_t* prog_host, int body, hipStream_t st);

using cd = std::complex<double>;

qsv_status apply_fused_block(qsv_state* s, const qsv_op& o) { return apply_op_pergate(s, o, 0); }

// ------------------------------------------------------------ op classes
enum PKind { PK_U1 = 0, PK_U2 = 1, PK_D1 = 2, PK_D2 = 3, PK_OTHER = 4, PK_NOOP = 5, PK_CX = 6 };

struct POp {
  int kind = PK_OTHER;
  int nq = 0;
  int q[6] = {0, 0, 0, 0, 0, 0};
  bool sign = false;  // Z (D1) or CZ (D2): a pure sign pattern
  cd m[16];           // U1: 2x2, U2: 4x4 (listed order), D1: d0,d1, D2: d[4]
  uint64_t qmask = 0;
  bool nondiag() const { return kind == PK_U1 || kind == PK_U2 || kind == PK_OTHER || kind == PK_CX; }
};

static bool is_zero(cd z) { return z.real() == 0.0 && z.imag() == 0.0; }
static bool is_one(cd z) { return z.real() == 1.0 && z.imag() == 0.0; }
static bool is_mone(cd z) { return z.real() == -1.0 && z.imag() == 0.0; }

// CNOT(c, t) as H_t CZ(c, t) H_t: the Hadamards become rotations (merged
// with the target's neighbouring one-qubit gates) and the CZ a sign step.
// The adjoint sweep plans CNOTs this way; the forward tile passes apply them
// as store maps instead (classify_tile).  Other ops are kept as they are.
void expand_cnots(const qsv_op* ops, int n_ops, std::vector<qsv_op>& out, std::vector<int>* origin) {
  out.clear();
  out.reserve((size_t)n_ops);
  if (origin) origin->clear();
  for (int i = 0; i < n_ops; ++i) {
    const qsv_op& o = ops[i];
    if (o.gate != QSV_CNOT) {
      out.push_back(o);
      if (origin) origin->push_back(i);
      continue;
    }
    if (origin) origin->insert(origin->end(), 3, i);
    qsv_op h{};
    h.gate = QSV_H;
    h.nq = 1;
    h.q[0] = o.q[1];
    qsv_op cz{};
    cz.gate = QSV_CZ;
    cz.nq = 2;
    cz.q[0] = o.q[0];
    cz.q[1] = o.q[1];
    out.push_back(h);
    out.push_back(cz);
    out.push_back(h);
  }
}

// Parameterised gates are classified by their gate, not by the value of the
// angle: RX / RY stay two-by-two rotations and RZ / CPHASE diagonal phases
// at every angle, 0 included.  A plan (and a batch's captured structure)
// then does not change when only the angles do, and the adjoint sweep keeps
// a slot for every rotation (a rotation at angle 0 is the identity, but its
// derivative is not zero).
static POp classify(const qsv_op& o) {
  POp p;
  p.nq = o.nq;
  for (int j = 0; j < o.nq; ++j) {
    p.q[j] = o.q[j];
    p.qmask |= 1ull << o.q[j];
  }
  cd m[16];
  const double zero[3] = {0, 0, 0};
  if (o.gate == QSV_RX || o.gate == QSV_RY || o.gate == QSV_RZ || o.gate == QSV_CPHASE) {
    gate_matrix(o.gate, o.p ? o.p : zero, m);
    if (o.gate == QSV_CPHASE) {
      p.kind = PK_D2;
      for (int i = 0; i < 4; ++i) p.m[i] = m[i * 5];
    } else if (o.gate == QSV_RZ) {
      p.kind = PK_D1;
      p.m[0] = m[0];
      p.m[1] = m[3];
    } else {
      p.kind = PK_U1;
      for (int i = 0; i < 4; ++i) p.m[i] = m[i];
    }
    return p;
  }
  if (o.gate == QSV_MAT) {
    if (o.nq > 2) {
      p.kind = PK_OTHER;
      return p;
    }
    const int D = 1 << o.nq;
    for (int i = 0; i < D * D; ++i) m[i] = cd(o.mat[2 * i], o.mat[2 * i + 1]);
  } else {
    gate_matrix(o.gate, o.p ? o.p : zero, m);
  }
  if (o.nq == 1) {
    if (is_zero(m[1]) && is_zero(m[2])) {
      if (is_one(m[0]) && is_one(m[3])) {
        p.kind = PK_NOOP;
        return p;
      }
      p.kind = PK_D1;
      p.m[0] = m[0];
      p.m[1] = m[3];
      p.sign = is_one(m[0]) && is_mone(m[3]);
    } else {
      p.kind = PK_U1;
      for (int i = 0; i < 4; ++i) p.m[i] = m[i];
    }
    return p;
  }
  bool diag = true;
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c)
      if (r != c && !is_zero(m[r * 4 + c])) diag = false;
  if (diag) {
    p.kind = PK_D2;
    for (int i = 0; i < 4; ++i) p.m[i] = m[i * 5];
    p.sign = is_one(m[0]) && is_one(m[5]) && is_one(m[10]) && is_mone(m[15]);
  } else {
    p.kind = PK_U2;
    for (int i = 0; i < 16; ++i) p.m[i] = m[i];
  }
  return p;
}

// The class of an op in a forward tile-pass plan: a CNOT is a permutation
// of basis states, x_t ^= x_c.  The CNOTs that end a round (target in the
// tile, control anywhere) compose into one affine map of the tile's local
// index, which the round's store applies by writing each amplitude to the
// slot of its image: no arithmetic, and a ladder of CNOTs takes no layers.
static POp classify_tile(const qsv_op& o) {
  if (o.gate != QSV_CNOT) return classify(o);
  POp p;
  p.kind = PK_CX;
  p.nq = 2;
  p.q[0] = o.q[0];  // control
  p.q[1] = o.q[1];  // target
  p.qmask = (1ull << o.q[0]) | (1ull << o.q[1]);
  return p;
}

// kinds of the planner's per-round work items
enum WorkType { TOP_U1 = 1, TOP_U2, TOP_SIGN, TOP_PHASE1, TOP_DIAG2, TOP_PERM2, TOP_GIVENS };

// ------------------------------------------------------------- schedule
struct Round {
  int R[8];                 // register local bits (exactly RB entries)
  std::vector<int> ops;     // op indices in application order
};
struct Step {
  bool tile = true;
  int op = -1;              // fallback op (tile == false)
  std::vector<int> inv;     // qubit-permutation pass: the involution (empty otherwise)
  std::vector<int> S;       // sorted tile qubits
  std::vector<Round> rounds;
};
struct Schedule {
  int n = 0, t = 0, c = 0, RB = 0;
  std::vector<uint32_t> key;  // exact structure (guards against hash collisions)
  std::vector<Step> steps;
  int passes = 0;
  bool relabeled = false;     // the steps apply the op list with its SWAPs relabeled away
};

// Dependency scan: the ops a pass over tile set S (or a round over register
// set S) can apply, in program order.  A CNOT needs its target in Tmask (the
// tile).  In a round (round = true) a CNOT runs at the round's store, after
// everything else, so later ops on its qubits other than CNOTs wait for the
// next round.  Returns the weighted count of non-diagonal ops taken.
static int scan(const std::vector<POp>& P, const std::vector<int>& pending, uint64_t Smask,
                uint64_t allq, std::vector<int>* take, uint64_t Tmask, bool round) {
  uint64_t bnd = 0, bd = 0, pm = 0;
  int score = 0;
  for (int i : pending) {
    const POp& o = P[i];
    const bool nd = o.nondiag();
    const bool cx = o.kind == PK_CX;
    const bool blocked = (o.qmask & bnd) || (nd && (o.qmask & bd)) || (!cx && (o.qmask & pm));
    if (!blocked) {
      const bool exe = !nd || ((o.kind == PK_U1 || o.kind == PK_U2) && (o.qmask & ~Smask) == 0) ||
                       (cx && ((Tmask >> o.q[1]) & 1ull));
      if (exe) {
        if (take) take->push_back(i);
        if (nd) score += o.nq;
        if (cx && round) pm |= o.qmask;
        continue;
      }
    }
    if (nd)
      bnd |= o.qmask;
    else
      bd |= o.qmask;
    if (bnd == allq) break;
  }
  return score;
}

static std::shared_ptr<Schedule> build_schedule(const std::vector<POp>& P, int n, int t, int c,
                                                int RB) {
  auto sch = std::make_shared<Schedule>();
  sch->n = n;
  sch->t = t;
  sch->c = c;
  sch->RB = RB;
  const uint64_t allq = n >= 64 ? ~0ull : ((1ull << n) - 1);
  std::vector<int> pending;
  for (int i = 0; i < (int)P.size(); ++i)
    if (P[i].kind != PK_NOOP) pending.push_back(i);
  std::vector<char> done(P.size(), 0);
  while (!pending.empty()) {
    const POp& f0 = P[pending[0]];
    if (f0.kind == PK_OTHER) {
      Step st;
      st.tile = false;
      st.op = pending[0];
      sch->steps.push_back(st);
      pending.erase(pending.begin());
      continue;
    }
    // choose S: low c qubits + first queued non-diagonal op + greedy growth
    uint64_t Smask = c >= 64 ? ~0ull : ((1ull << c) - 1);
    if (n <= t) {
      Smask = allq;
    } else {
      for (int i : pending)
        if (P[i].kind == PK_U1 || P[i].kind == PK_U2) {
          Smask |= P[i].qmask;
          break;
        } else if (P[i].kind == PK_CX) {
          Smask |= 1ull << P[i].q[1];
          break;
        } else if (P[i].kind == PK_OTHER) {
          break;
        }
      // first queued non-diagonal op position per qubit (tie-break)
      std::vector<int> firstpos(n, 1 << 30);
      for (int k = 0; k < (int)pending.size(); ++k) {
        const POp& o = P[pending[k]];
        if (!o.nondiag()) continue;
        for (int j = 0; j < o.nq; ++j) firstpos[o.q[j]] = std::min(firstpos[o.q[j]], k);
      }
      while (__builtin_popcountll(Smask) < t) {
        int best = -1, bs = -1, bpos = 1 << 30;
        for (int q = 0; q < n; ++q) {
          if ((Smask >> q) & 1) continue;
          const int sc = scan(P, pending, Smask | (1ull << q), allq, nullptr, Smask | (1ull << q), false);
          if (sc > bs || (sc == bs && firstpos[q] < bpos)) {
            best = q;
            bs = sc;
            bpos = firstpos[q];
          }
        }
        Smask |= 1ull << best;
      }
    }
    std::vector<int> take;
    scan(P, pending, Smask, allq, &take, Smask, false);
    if (take.empty()) {  // cannot happen: the first queued op is executable
      Step st;
      st.tile = false;
      st.op = pending[0];
      sch->steps.push_back(st);
      pending.erase(pending.begin());
      continue;
    }
    Step st;
    for (int q = 0; q < n; ++q)
      if ((Smask >> q) & 1) st.S.push_back(q);
    std::vector<int> lpos(n, -1);
    for (int j = 0; j < (int)st.S.size(); ++j) lpos[st.S[j]] = j;
    // Rounds are chosen like passes, one level down: a register set of RB
    // tile qubits (starting from the first queued non-diagonal op, grown
    // greedily by the number of ops the dependency scan can then apply),
    // and every op the scan admits for it, in program order.  Diagonal ops
    // run in whichever round reaches them.  Taking every admissible op,
    // rather than cutting rounds in program order, lets a round apply
    // several layers of gates and merge runs of 2x2 gates on one qubit.
    {
      std::vector<int> rem(take);
      while (!rem.empty()) {
        uint64_t Rg = 0;  // register qubits (global mask)
        bool gates = false;
        for (int i : rem)
          if (P[i].kind == PK_U1 || P[i].kind == PK_U2) {
            Rg = P[i].qmask;
            gates = true;
            break;
          } else if (P[i].kind == PK_OTHER) {
            break;
          }
        bool cxs = false;
        for (int i : rem) cxs = cxs || P[i].kind == PK_CX;
        if (!gates && !cxs) {  // only diagonal ops left: one round takes them all
          Round cur;
          for (int k = 0; k < 8; ++k) cur.R[k] = -1;
          cur.ops = rem;
          st.rounds.push_back(cur);
          break;
        }
        const int want = std::min(RB, (int)st.S.size());
        while (__builtin_popcountll(Rg) < want) {
          int best = -1, bs = -1;
          for (int q : st.S) {
            if ((Rg >> q) & 1) continue;
            const int sc = scan(P, rem, Rg | (1ull << q), allq, nullptr, Smask, true);
            if (sc > bs) {
              best = q;
              bs = sc;
            }
          }
          Rg |= 1ull << best;
        }
        Round cur;
        scan(P, rem, Rg, allq, &cur.ops, Smask, true);
        int k = 0;
        for (int j = 0; j < (int)st.S.size() && k < 8; ++j)
          if ((Rg >> st.S[j]) & 1) cur.R[k++] = j;
        for (; k < 8; ++k) cur.R[k] = -1;
        std::vector<char> in(P.size(), 0);
        for (int i : cur.ops) in[i] = 1;
        std::vector<int> left;
        for (int i : rem)
          if (!in[i]) left.push_back(i);
        rem.swap(left);
        st.rounds.push_back(std::move(cur));
      }
      for (int i : take) done[i] = 1;
    }
    // pad every round's register set to exactly RB distinct local bits
    for (Round& r : st.rounds) {
      uint64_t used = 0;
      int k = 0;
      for (; k < 8 && r.R[k] >= 0; ++k) used |= 1ull << r.R[k];
      for (int b = 0; k < RB && b < (int)st.S.size(); ++b)
        if (!((used >> b) & 1)) {
          r.R[k++] = b;
          used |= 1ull << b;
        }
    }
    sch->steps.push_back(std::move(st));
    sch->passes++;
    std::vector<int> rest;
    for (int i : pending)
      if (!done[i]) rest.push_back(i);
    pending.swap(rest);
  }
  return sch;
}

// Contiguous low qubits of every tile (the HBM segment of c qubits): 5 for
// complex64 (256-byte segments), 4 for complex128.  Every tile spends them,
// so for complex64 the plan with 128-byte segments (one more qubit free per
// tile) is taken when it needs fewer passes.  QSV_SEGMENT_QUBITS=4 or 5 in
// the environment fixes the choice (read at first use, and again after
// qsv_debug_reload_env; for measurement).
static std::atomic<int> g_env_segment{-1};
static int env_segment_qubits() {
  int v = g_env_segment.load();
  if (v < 0) {
    const char* e = std::getenv("QSV_SEGMENT_QUBITS");
    v = (e && (e[0] == '4' || e[0] == '5') && e[1] == 0) ? e[0] - '0' : 0;
    g_env_segment.store(v);
  }
  return v;
}
static std::shared_ptr<Schedule> plan_tile_passes(const std::vector<POp>& P, int n, int t, bool f32, int RB,
                                                  int force_c) {
  const int forced = force_c > 0 ? force_c : env_segment_qubits();
  int c = forced ? forced : (f32 ? 5 : 4);
  if (!f32) c = 4;
  if (c > t) c = t;
  auto sch = build_schedule(P, n, t, c, RB);
  if (f32 && !forced && c == 5) {
    auto alt = build_schedule(P, n, t, 4, RB);
    if (alt->passes < sch->passes) sch = alt;
  }
  return sch;
}

// SWAP relabeling.  A SWAP exchanges which physical bit holds which logical
// qubit instead of moving amplitudes: lab[q] is the bit that holds logical
// qubit q, every other op is rewritten onto lab of its qubits, and the state
// is put back in order at the end by one permutation of the index bits,
// out[x] = in[sigma(x)] with sigma(q) = lab[q].  Returns false when the list
// has no SWAP.
static bool relabel_swaps(const std::vector<qsv_op>& ops, int n, std::vector<qsv_op>& out, std::vector<int>& lab) {
  lab.resize(n);
  for (int q = 0; q < n; ++q) lab[q] = q;
  out.clear();
  bool any = false;
  for (const qsv_op& o : ops) {
    if (o.gate == QSV_SWAP) {
      std::swap(lab[o.q[0]], lab[o.q[1]]);
      any = true;
      continue;
    }
    qsv_op r = o;
    for (int j = 0; j < r.nq && j < 6; ++j) r.q[j] = lab[o.q[j]];
    out.push_back(r);
  }
  return any;
}

// sigma as at most two involutions applied as passes, first a then b.  The
// pass for v maps in to out[x] = in[v(x)], so the two give
// out[x] = in[a(b(x))] and need a(b(q)) = sigma(q): on each cycle
// c_0 -> c_1 -> ... of sigma, b(c_i) = c_(-i) and a(c_j) = c_(1-j) (both
// reflections of the cycle).  An involution sigma is one pass; the identity
// none.
static std::vector<std::vector<int>> involution_passes(const std::vector<int>& sigma) {
  const int n = (int)sigma.size();
  bool ident = true, invol = true;
  for (int q = 0; q < n; ++q) {
    ident = ident && sigma[q] == q;
    invol = invol && sigma[sigma[q]] == q;
  }
  if (ident) return {};
  if (invol) return {sigma};
  std::vector<int> a(n), b(n);
  std::vector<char> seen(n, 0);
  for (int q0 = 0; q0 < n; ++q0) {
    if (seen[q0]) continue;
    std::vector<int> cyc;
    for (int q = q0; !seen[q]; q = sigma[q]) {
      seen[q] = 1;
      cyc.push_back(q);
    }
    const int k = (int)cyc.size();
    for (int i = 0; i < k; ++i) {
      b[cyc[i]] = cyc[(k - i) % k];
      a[cyc[i]] = cyc[((1 - i) % k + k) % k];
    }
  }
  return {a, b};
}

// The fused plan of a gate list (CNOTs expanded): tile passes and per-gate
// steps, and, when the list has SWAPs and relabeling them away needs fewer
// passes in all, the plan of the relabeled list followed by its
// qubit-permutation passes.
static std::shared_ptr<Schedule> plan_schedule(const std::vector<qsv_op>& xops, int n, int t, bool f32, int RB,
                                               int force_c = 0) {
  std::vector<POp> P(xops.size());
  for (size_t i = 0; i < xops.size(); ++i) P[i] = classify_tile(xops[i]);
  auto sch = plan_tile_passes(P, n, t, f32, RB, force_c);
  std::vector<qsv_op> rops;
  std::vector<int> lab;
  if (!relabel_swaps(xops, n, rops, lab)) return sch;
  std::vector<POp> R(rops.size());
  for (size_t i = 0; i < rops.size(); ++i) R[i] = classify_tile(rops[i]);
  auto alt = plan_tile_passes(R, n, t, f32, RB, force_c);
  const std::vector<std::vector<int>> inv = involution_passes(lab);
  if (alt->passes + (int)inv.size() >= sch->passes) return sch;
  for (const std::vector<int>& v : inv) {
    Step st;
    st.tile = false;
    st.inv = v;
    alt->steps.push_back(std::move(st));
  }
  alt->passes += (int)inv.size();
  alt->relabeled = true;
  return alt;
}

// The op list a schedule's steps index: the list itself, or with its SWAPs
// relabeled away.
static const std::vector<qsv_op>& step_ops(const Schedule& sch, const std::vector<qsv_op>& xops, int n,
                                           std::vector<qsv_op>& buf) {
  if (!sch.relabeled) return xops;
  std::vector<int> lab;
  relabel_swaps(xops, n, buf, lab);
  return buf;
}

// Program of a qubit-permutation pass for the involution v (layout in
// tile.hpp): S = the low c qubits, closed under v, then more of v's fixed
// qubits and pairs, lowest first, up to QpermCfg<T>::TP qubits; the other
// qubits in tile-id order.
template <typename T>
static void emit_qperm(const std::vector<int>& v, int n, std::vector<int32_t>& prog) {
  int t = std::min(QpermCfg<T>::TP, n);
  int c = std::min(sizeof(T) == 4 ? 5 : 4, t);
  std::vector<char> in(n, 0);
  int cnt = 0;
  for (int q = 0; q < c; ++q)
    for (int r : {q, v[q]})
      if (!in[r]) {
        in[r] = 1;
        ++cnt;
      }
  for (int q = 0; q < n && cnt < t; ++q) {
    if (in[q]) continue;
    const int need = v[q] == q ? 1 : 2;
    if (cnt + need > t) continue;
    in[q] = in[v[q]] = 1;
    cnt += need;
  }
  t = cnt;
  // nonS in the order of the tile id's bits: each of the lowest outside
  // qubits next to its image, so that the tiles in flight at one time (low
  // id bits) read and write nearby segments on both sides of the pass
  std::vector<int> S, nonS, pos(n, -1);
  std::vector<char> taken(n, 0);
  for (int q = 0; q < n; ++q) {
    if (in[q]) {
      S.push_back(q);
    } else if (!taken[q]) {
      nonS.push_back(q);
      taken[q] = 1;
      if (!taken[v[q]]) {
        nonS.push_back(v[q]);
        taken[v[q]] = 1;
      }
    }
  }
  for (int k = 0; k < t; ++k) pos[S[k]] = k;
  for (int i = 0; i < (int)nonS.size(); ++i) pos[nonS[i]] = i;
  const size_t base = prog.size();
  prog.push_back(t);
  prog.push_back(c);
  prog.push_back((int32_t)nonS.size());
  prog.push_back(kPassQperm);
  for (int q : S) prog.push_back(q);
  for (int q : nonS) prog.push_back(q);
  for (int q : S) prog.push_back(pos[v[q]]);
  for (int q : nonS) prog.push_back(pos[v[q]]);
  while ((prog.size() - base) % 16) prog.push_back(0);
}

// ------------------------------------------------------- schedule cache
static std::mutex g_cache_mu;
static std::unordered_map<uint64_t, std::shared_ptr<Schedule>> g_cache;

static uint64_t mix(uint64_t h, uint64_t v) {
  h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
  return h;
}

static std::vector<uint32_t> structure_key(const std::vector<POp>& P, int n, int t, int c, int RB) {
  std::vector<uint32_t> k = {(uint32_t)n, (uint32_t)t, (uint32_t)c, (uint32_t)RB, (uint32_t)P.size()};
  for (const POp& o : P) {
    k.push_back((uint32_t)o.kind | ((uint32_t)o.sign << 8) | ((uint32_t)o.nq << 16));
    for (int j = 0; j < o.nq; ++j) k.push_back((uint32_t)o.q[j]);
  }
  return k;
}

static uint64_t key_hash(const std::vector<uint32_t>& k) {
  uint64_t h = 0x51535631ull;
  for (uint32_t v : k) h = mix(h, v);
  return h;
}

// ------------------------------------------------------- materialisation
// Reals in the state's precision: one word per float, two (low, high) per
// double.
template <typename T>
struct RealWords {
  static void put(double v, std::vector<int32_t>& out) {
    if (sizeof(T) == 4) {
      float f = (float)v;
      int32_t w;
      std::memcpy(&w, &f, 4);
      out.push_back(w);
    } else {
      int64_t w;
      std::memcpy(&w, &v, 8);
      out.push_back((int32_t)(w & 0xffffffff));
      out.push_back((int32_t)(w >> 32));
    }
  }
};

template <typename T>
int tile_swizzle_bits();

// ---------------------------------------------------- gate algebra (host)
// A 2x2 that is a unitary times a positive scale k factors as
//     U = diag(l0, l1) . k R . diag(1, r1),   |l0| = |l1| = |r1| = 1,
// with R a real rotation by theta in [0, pi/2] (cos = c/k, sin = s/k, c and s
// the moduli of the diagonal and off-diagonal entries).  R runs as in-place
// shears (GIVENS op), either two with a deferred scale,
//     [[1, 0], [sin cos, 1]] . [[1, -tan], [0, 1]] = diag(1/cos, cos) . R,
// the scale joining the factor carried for the qubit (when cos >= 0.3), or
// three that give R exactly,
//     R = [[1, -h], [0, 1]] . [[1, 0], [sin, 1]] . [[1, -h], [0, 1]],
//     h = tan(theta / 2) in [0, 1], sin in [0, 1].
// Diagonal factors commute with all other diagonal gates and with gates on
// other qubits, so a tile pass carries them per qubit and applies them in
// bulk: one 2^RB-entry table per layer of rotations (complex entries: phase,
// sign and magnitude at once), and a per-group factor for qubits that are
// not register bits.
struct Split {
  int kind;         // 0 diagonal (d0, d1 carry the whole gate), 1 rotation, -1 no factorisation
  int form;         // 0: two shears and a carried scale, 1: three shears
  double p, q;      // shear coefficients
  cd d0, d1;        // diagonal factor after the rotation (carried)
  cd r1;            // diagonal factor diag(1, r1) before the rotation
};

static cd unit_phase(cd z) { return z / std::abs(z); }

// Smallest cos(theta) of a rotation applied as two shears: the carried scale
// and the first shear's coefficient stay within a factor 1 / 0.3 of 1.
constexpr double kTwoShearMinCos = 0.3;

static Split split_u1(const cd* u) {
  Split sp{-1, 0, 0.0, 0.0, cd(1.0), cd(1.0), cd(1.0)};
  const double a00 = std::abs(u[0]), a01 = std::abs(u[1]), a10 = std::abs(u[2]), a11 = std::abs(u[3]);
  const double k2 = 0.5 * (a00 * a00 + a01 * a01 + a10 * a10 + a11 * a11);
  if (!(k2 > 0.0) || !std::isfinite(k2)) return sp;
  if (a01 == 0.0 && a10 == 0.0) {
    if (a00 == 0.0 || a11 == 0.0) return sp;  // singular: kept as a 2x2
    sp.kind = 0;
    sp.d0 = u[0];
    sp.d1 = u[3];
    return sp;
  }
  // a scaled unitary has orthogonal columns of equal norm
  if (std::abs(a00 * a00 + a10 * a10 - k2) > 1e-12 * k2 || std::abs(a01 * a01 + a11 * a11 - k2) > 1e-12 * k2 ||
      std::abs(std::conj(u[0]) * u[1] + std::conj(u[2]) * u[3]) > 1e-12 * k2 || a10 == 0.0 || a01 == 0.0)
    return sp;
  const double c = 0.5 * (a00 + a11), s = 0.5 * (a01 + a10), kap = std::sqrt(c * c + s * s);
  const cd l1 = unit_phase(u[2]);
  cd l0, r1;
  if (a00 > 0.0 && a11 > 0.0) {
    l0 = unit_phase(u[0]);
    r1 = unit_phase(u[3]) / l1;
  } else {
    l0 = -unit_phase(u[1]);
    r1 = 1.0;
  }
  // accept only an exact factorisation (to rounding)
  const cd v[4] = {l0 * c, -l0 * s * r1, l1 * s, l1 * c * r1};
  for (int e = 0; e < 4; ++e)
    if (std::abs(v[e] - u[e]) > 1e-12 * std::sqrt(k2)) return sp;
  sp.kind = 1;
  sp.r1 = r1;
  // Unit rotation by theta in [0, pi/2].  Two shears (p = -tan(theta),
  // q = sin(theta) cos(theta)) give it up to the scale diag(1/cos, cos)
  // applied after it, which joins the carried factor; when cos(theta) is
  // small that scale and p grow, and three shears (p = -tan(theta / 2),
  // q = sin(theta)) give the rotation exactly.
  if (c >= kTwoShearMinCos * kap) {
    sp.form = 0;
    sp.p = -s / c;
    sp.q = c * s / (kap * kap);
    sp.d0 = c * l0;
    sp.d1 = (kap * kap / c) * l1;
  } else {
    sp.form = 1;
    sp.p = -s / (kap + c);
    sp.q = s / kap;
    sp.d0 = kap * l0;
    sp.d1 = kap * l1;
  }
  return sp;
}

// Writes the program of one tile pass (layout in tile.hpp).  Returns false
// if a sign mask is not made of single register bits (the planner builds
// none such; checked so that no wrong program is written).
template <typename T>
static bool emit_pass(const Step& st, const std::vector<POp>& P, int n, int c, int RB,
                      std::vector<int32_t>& prog) {
  const int t = (int)st.S.size();
  const int NR = 1 << RB;
  const int SB = tile_swizzle_bits<T>();
  const int WT = sizeof(T) == 4 ? 1 : 2;
  std::vector<int> lpos(n, -1);
  for (int j = 0; j < t; ++j) lpos[st.S[j]] = j;
  std::vector<int> nonS;
  for (int q = 0; q < n; ++q)
    if (lpos[q] < 0) nonS.push_back(q);
  const size_t h0 = prog.size();
  prog.push_back(t);
  prog.push_back(c);
  prog.push_back((int32_t)nonS.size());
  prog.push_back((int32_t)st.rounds.size());
  for (int q : st.S) prog.push_back(q);
  for (int q : nonS) prog.push_back(q);
  const size_t roff0 = prog.size();  // round offsets, filled in as the rounds are written
  prog.resize(prog.size() + st.rounds.size(), 0);
  while ((prog.size() - h0) % 16) prog.push_back(0);

  // Diagonal factors not yet applied, per tile-local qubit (diag(pd0, pd1)),
  // and a scalar for the whole tile.
  std::vector<cd> pd0(t, cd(1.0)), pd1(t, cd(1.0));
  cd gscale = 1.0;

  struct PhTerm {
    uint32_t lgm;
    uint64_t om;
    cd r;
  };
  std::vector<std::vector<PhTerm>> tfac;  // the pass's tile-factor slots
  std::vector<cd> ltab;                   // the pass's lane table
  const size_t kLaneTab = kLaneTabBytes / (2 * sizeof(T));
  // diagonal work that runs between two non-diagonal ops of a round
  struct DGroup {
    bool tab = false;
    cd tb[32];
    uint32_t pairs = 0;                                  // CZ between register bits: pair index set
    std::vector<std::pair<int, uint32_t>> fmix, rcmix;  // (free pos | outside q, mask over m)
    uint32_t Md[32] = {0};
    std::vector<int32_t> fc, cc;
    std::vector<std::pair<int, std::vector<PhTerm>>> phl;  // register bit (-1: every m) -> terms
    std::vector<int> raw;                                  // PHASE1 / DIAG2 ops kept as they are
  };
  struct NdItem {
    int type = 0;
    int j0 = -1, j1 = -1;
    cd m[16];
    int jf = 0;
    double p = 0.0, q = 0.0;
    int code = 0;
  };
  struct RPlan {
    int R[8];
    int regof[64];
    std::vector<NdItem> nd;
    std::vector<DGroup> g;  // g[i] runs before nd[i], g.back() after the last one
    int last[8];            // first group after the last non-diagonal op on register bit j
    std::vector<int> cx;    // CNOTs applied by the round's store, in program order
  };
  std::vector<RPlan> plans;

  auto mbit = [&](int j) {
    uint32_t mk = 0;
    for (int m = 0; m < NR; ++m)
      if ((m >> j) & 1) mk |= 1u << m;
    return mk;
  };
  auto table_of = [&](DGroup& g) -> cd* {
    if (!g.tab) {
      for (int m = 0; m < NR; ++m) g.tb[m] = 1.0;
      g.tab = true;
    }
    return g.tb;
  };
  auto has_sign = [](const DGroup& g) {
    if (g.pairs || !g.fmix.empty() || !g.rcmix.empty() || !g.fc.empty() || !g.cc.empty()) return true;
    for (int d = 0; d < 32; ++d)
      if (g.Md[d]) return true;
    return false;
  };
  auto has_key = [](const DGroup& g, int key) {
    for (auto& e : g.phl)
      if (e.first == key) return true;
    return false;
  };
  // Diagonal work may run anywhere after the last non-diagonal op on its
  // register bits (group lo) up to the current point (the last group): take
  // the latest group that already holds work of the same kind, else the last.
  auto pick = [](RPlan& rp, int lo, auto pred) -> DGroup& {
    const int hi = (int)rp.g.size() - 1;
    for (int gi = hi; gi >= lo; --gi)
      if (pred(rp.g[gi])) return rp.g[gi];
    return rp.g[hi];
  };
  // diag(e0, e1) on register bit j
  auto tab_bit = [&](RPlan& rp, int j, cd e0, cd e1) {
    if (e0 == cd(1.0) && e1 == cd(1.0)) return;
    cd* tbl = table_of(pick(rp, rp.last[j], [](const DGroup& g) { return g.tab; }));
    for (int m = 0; m < NR; ++m) tbl[m] *= ((m >> j) & 1) ? e1 : e0;
  };
  auto add_term = [&](DGroup& g, int key, uint32_t lgm, uint64_t om, cd rr) {
    for (auto& e : g.phl)
      if (e.first == key) {
        for (auto& tm : e.second)
          if (tm.lgm == lgm && tm.om == om) {
            tm.r *= rr;
            return;
          }
        e.second.push_back({lgm, om, rr});
        return;
      }
    g.phl.push_back({key, {{lgm, om, rr}}});
  };
  auto add_mask = [](std::vector<std::pair<int, uint32_t>>& v, int key, uint32_t mk) {
    for (auto& e : v)
      if (e.first == key) {
        e.second ^= mk;
        return;
      }
    v.push_back({key, mk});
  };
  // operand kind/value of a qubit for the ops kept as they are
  auto operand = [&](const RPlan& rp, int q, int& kind, int& val) {
    const int p = lpos[q];
    if (p < 0) {
      kind = TK_OUT;
      val = q;
    } else if (rp.regof[p] >= 0) {
      kind = TK_REG;
      val = (int)mbit(rp.regof[p]);
    } else {
      kind = TK_FREE;
      val = p;
    }
  };

  for (const Round& r : st.rounds) {
    plans.emplace_back();
    RPlan& rp = plans.back();
    for (int b = 0; b < 64; ++b) rp.regof[b] = -1;
    for (int k = 0; k < RB; ++k) {
      rp.R[k] = r.R[k];
      rp.regof[r.R[k]] = k;
      rp.last[k] = 0;
    }
    rp.g.emplace_back();
    const int* regof = rp.regof;

    // diag(e0, e1) on qubit q: carried while q is in the tile, else a factor
    // per tile
    auto phase1 = [&](int q, cd e0, cd e1) {
      const int p = lpos[q];
      if (p >= 0) {
        pd0[p] *= e0;
        pd1[p] *= e1;
      } else {
        gscale *= e0;
        if (e1 != e0) add_term(pick(rp, 0, [&](const DGroup& g) { return has_key(g, -1); }), -1, 0u, 1ull << q, e1 / e0);
      }
    };
    // factor rr where both qubits are 1
    auto interaction = [&](int qa, int qb, cd rr) {
      if (rr == cd(1.0)) return;
      int pa = lpos[qa], pb = lpos[qb];
      int ja = pa >= 0 ? regof[pa] : -1, jb = pb >= 0 ? regof[pb] : -1;
      if (ja >= 0 && jb >= 0) {
        cd* tbl = table_of(pick(rp, std::max(rp.last[ja], rp.last[jb]), [](const DGroup& g) { return g.tab; }));
        for (int m = 0; m < NR; ++m)
          if (((m >> ja) & 1) && ((m >> jb) & 1)) tbl[m] *= rr;
        return;
      }
      if (ja < 0 && jb >= 0) {
        std::swap(qa, qb);
        std::swap(pa, pb);
        std::swap(ja, jb);
      }
      uint32_t lgm = 0;
      uint64_t om = 0;
      auto other = [&](int q, int p) {
        if (p >= 0) lgm |= 1u << p;
        else om |= 1ull << q;
      };
      if (ja >= 0) {
        other(qb, pb);
        add_term(pick(rp, rp.last[ja], [&](const DGroup& g) { return has_key(g, ja); }), ja, lgm, om, rr);
      } else {
        other(qa, pa);
        other(qb, pb);
        add_term(pick(rp, 0, [&](const DGroup& g) { return has_key(g, -1); }), -1, lgm, om, rr);
      }
    };
    // CZ as a sign pattern
    auto cz = [&](int qa, int qb) {
      int pa = lpos[qa], pb = lpos[qb];
      int ja = pa >= 0 ? regof[pa] : -1, jb = pb >= 0 ? regof[pb] : -1;
      if (ja < 0 && jb >= 0) {
        std::swap(qa, qb);
        std::swap(pa, pb);
        std::swap(ja, jb);
      }
      auto sg = [&](const DGroup& g) { return has_sign(g) || g.tab; };
      if (ja >= 0 && jb >= 0) {
        pick(rp, std::max(rp.last[ja], rp.last[jb]), sg).pairs ^= 1u << cz_pair_index(ja, jb);
      } else if (ja >= 0 && pb >= 0) {
        add_mask(pick(rp, rp.last[ja], has_sign).fmix, pb, mbit(ja));
      } else if (ja >= 0) {
        add_mask(pick(rp, rp.last[ja], has_sign).rcmix, qb, mbit(ja));
      } else {
        DGroup& g = pick(rp, 0, has_sign);
        if (pa >= 0 && pb >= 0) {
          const int lo = std::min(pa, pb), hi = std::max(pa, pb);
          g.Md[hi - lo] ^= 1u << lo;
        } else if (pa >= 0 || pb >= 0) {
          if (pa >= 0) g.fc.insert(g.fc.end(), {qb, pa});
          else g.fc.insert(g.fc.end(), {qa, pb});
        } else {
          g.cc.insert(g.cc.end(), {qa, qb});
        }
      }
    };
    // an op kept as it is: after the last non-diagonal op on its register bits
    auto raw = [&](int i) {
      const POp& o = P[i];
      int gi = 0;
      for (int j = 0; j < o.nq; ++j) {
        const int p = lpos[o.q[j]];
        if (p >= 0 && regof[p] >= 0) gi = std::max(gi, rp.last[regof[p]]);
      }
      rp.g[gi].raw.push_back(i);
    };
    auto push_nd = [&](const NdItem& it, int ja, int jb) {
      rp.nd.push_back(it);
      rp.g.emplace_back();
      rp.last[ja] = (int)rp.nd.size();
      if (jb >= 0) rp.last[jb] = (int)rp.nd.size();
    };

    // working list: fold single-qubit chains and batch sign ops
    struct W {
      int type;
      int j0, j1;
      cd m[16];
      int op;
      std::vector<int> signs;
    };
    std::vector<W> work;
    int last_u1[64];
    for (int b = 0; b < 64; ++b) last_u1[b] = -1;
    for (int i : r.ops) {
      const POp& o = P[i];
      if (o.kind == PK_CX) {  // to the store map; nothing later in the round touches its qubits
        rp.cx.push_back(i);
        for (int j = 0; j < 2; ++j)
          if (lpos[o.q[j]] >= 0) last_u1[lpos[o.q[j]]] = -1;
        continue;
      }
      if (o.kind == PK_U1) {
        const int p = lpos[o.q[0]];
        if (last_u1[p] >= 0) {  // U <- U_new * U_old
          W& w = work[last_u1[p]];
          cd nm[4];
          for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) nm[a * 2 + b] = o.m[a * 2 + 0] * w.m[b] + o.m[a * 2 + 1] * w.m[2 + b];
          for (int e = 0; e < 4; ++e) w.m[e] = nm[e];
          continue;
        }
        W w;
        w.type = TOP_U1;
        w.j0 = regof[p];
        w.j1 = -1;
        for (int e = 0; e < 4; ++e) w.m[e] = o.m[e];
        w.op = i;
        work.push_back(w);
        last_u1[p] = (int)work.size() - 1;
        continue;
      }
      if (o.kind == PK_D1 && lpos[o.q[0]] >= 0 && last_u1[lpos[o.q[0]]] >= 0) {
        W& w = work[last_u1[lpos[o.q[0]]]];  // diag(d0, d1) * U
        w.m[0] *= o.m[0];
        w.m[1] *= o.m[0];
        w.m[2] *= o.m[1];
        w.m[3] *= o.m[1];
        continue;
      }
      for (int j = 0; j < o.nq; ++j)
        if (lpos[o.q[j]] >= 0) last_u1[lpos[o.q[j]]] = -1;
      if (o.kind == PK_U2) {
        W w;
        w.type = TOP_U2;
        int ja = regof[lpos[o.q[0]]], jb = regof[lpos[o.q[1]]];
        if (ja < jb) {
          for (int e = 0; e < 16; ++e) w.m[e] = o.m[e];
        } else {
          auto sw = [](int m) { return ((m & 1) << 1) | ((m >> 1) & 1); };
          for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) w.m[sw(a) * 4 + sw(b)] = o.m[a * 4 + b];
          std::swap(ja, jb);
        }
        w.j0 = ja;
        w.j1 = jb;
        w.op = i;
        // CNOT / SWAP patterns become register permutations
        static const int pats[3][4] = {{0, 3, 2, 1}, {0, 1, 3, 2}, {0, 2, 1, 3}};
        for (int code = 0; code < 3; ++code) {
          bool ok = true;
          for (int r = 0; r < 4 && ok; ++r)
            for (int c2 = 0; c2 < 4 && ok; ++c2) {
              const cd want = (c2 == pats[code][r]) ? cd(1.0, 0.0) : cd(0.0, 0.0);
              if (w.m[r * 4 + c2] != want) ok = false;
            }
          if (ok) {
            w.type = TOP_PERM2;
            w.m[0] = cd((double)code, 0.0);
            break;
          }
        }
        work.push_back(w);
      } else if (o.sign) {
        W w;
        w.type = TOP_SIGN;
        w.op = i;
        w.signs.push_back(i);
        work.push_back(w);
      } else {
        W w;
        w.type = o.kind == PK_D1 ? TOP_PHASE1 : TOP_DIAG2;
        w.op = i;
        work.push_back(w);
      }
    }

    // Order the work by depth: a non-diagonal item runs one level after the
    // latest item on its register bits, a diagonal item in the gap right
    // after the last non-diagonal item on its register bits.  Items on
    // different qubits commute and each qubit keeps its own order, so the
    // result is unchanged, while a layer can now hold every rotation of one
    // level instead of breaking at each diagonal op in between.
    {
      int lastN[8] = {0}, lastD[8] = {0};
      std::vector<int> key(work.size()), ord(work.size());
      for (size_t k = 0; k < work.size(); ++k) {
        const W& w = work[k];
        ord[k] = (int)k;
        if (w.type == TOP_U1 || w.type == TOP_U2 || w.type == TOP_PERM2) {
          int L = 0;
          for (int j : {w.j0, w.j1})
            if (j >= 0) L = std::max(L, std::max(lastN[j], lastD[j]));
          ++L;
          for (int j : {w.j0, w.j1})
            if (j >= 0) lastN[j] = L;
          key[k] = 2 * L;
        } else {
          const POp& o = P[w.op];
          int gap = 0;
          for (int e = 0; e < o.nq; ++e) {
            const int p = lpos[o.q[e]];
            if (p >= 0 && regof[p] >= 0) gap = std::max(gap, lastN[regof[p]]);
          }
          for (int e = 0; e < o.nq; ++e) {
            const int p = lpos[o.q[e]];
            if (p >= 0 && regof[p] >= 0) lastD[regof[p]] = std::max(lastD[regof[p]], gap);
          }
          key[k] = 2 * gap + 1;
        }
      }
      std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return key[a] < key[b]; });
      std::vector<W> sorted;
      sorted.reserve(work.size());
      for (int k : ord) sorted.push_back(std::move(work[k]));
      work.swap(sorted);
    }

    for (const W& w : work) {
      if (w.type == TOP_U1) {
        const int j = w.j0, p = rp.R[j];
        // the carried factor's moduli are applied first (real table entries:
        // every scale stays close to 1 rather than piling up in one scalar);
        // its phases go into the gate, which keeps a unitary gate unitary
        const double mu0 = std::abs(pd0[p]), mu1 = std::abs(pd1[p]);
        cd e0 = pd0[p], e1 = pd1[p];
        if (mu0 > 0.0 && mu1 > 0.0 && std::isfinite(mu0) && std::isfinite(mu1)) {
          tab_bit(rp, j, cd(mu0), cd(mu1));
          e0 /= mu0;
          e1 /= mu1;
        }
        const cd U[4] = {w.m[0] * e0, w.m[1] * e1, w.m[2] * e0, w.m[3] * e1};
        const Split sp = split_u1(U);
        if (sp.kind == 0) {
          pd0[p] = sp.d0;
          pd1[p] = sp.d1;
          continue;
        }
        NdItem it;
        it.j0 = j;
        if (sp.kind == 1) {
          tab_bit(rp, j, cd(1.0), sp.r1);
          it.type = TOP_GIVENS;
          it.jf = j | (sp.form << 8);
          it.p = sp.p;
          it.q = sp.q;
          pd0[p] = sp.d0;
          pd1[p] = sp.d1;
        } else {
          it.type = TOP_U1;
          for (int e = 0; e < 4; ++e) it.m[e] = U[e];
          pd0[p] = pd1[p] = 1.0;
        }
        push_nd(it, j, -1);
      } else if (w.type == TOP_U2) {
        const int p0 = rp.R[w.j0], p1 = rp.R[w.j1];
        NdItem it;
        it.type = TOP_U2;
        it.j0 = w.j0;
        it.j1 = w.j1;
        for (int a = 0; a < 4; ++a)
          for (int b = 0; b < 4; ++b)
            it.m[a * 4 + b] = w.m[a * 4 + b] * ((b & 1) ? pd1[p0] : pd0[p0]) * ((b >> 1) ? pd1[p1] : pd0[p1]);
        pd0[p0] = pd1[p0] = pd0[p1] = pd1[p1] = 1.0;
        push_nd(it, w.j0, w.j1);
      } else if (w.type == TOP_PERM2) {
        const int p0 = rp.R[w.j0], p1 = rp.R[w.j1];
        const int code = (int)w.m[0].real();
        if (code == 0) {  // CNOT, control j0: the control's factor commutes
          tab_bit(rp, w.j1, pd0[p1], pd1[p1]);
          pd0[p1] = pd1[p1] = 1.0;
        } else if (code == 1) {
          tab_bit(rp, w.j0, pd0[p0], pd1[p0]);
          pd0[p0] = pd1[p0] = 1.0;
        } else {  // SWAP exchanges the carried factors
          std::swap(pd0[p0], pd0[p1]);
          std::swap(pd1[p0], pd1[p1]);
        }
        NdItem it;
        it.type = TOP_PERM2;
        it.j0 = w.j0;
        it.j1 = w.j1;
        it.code = code;
        push_nd(it, w.j0, w.j1);
      } else if (w.type == TOP_PHASE1) {
        const POp& o = P[w.op];
        if (!is_zero(o.m[0]) && !is_zero(o.m[1])) phase1(o.q[0], o.m[0], o.m[1]);
        else raw(w.op);
      } else if (w.type == TOP_DIAG2) {
        const POp& o = P[w.op];
        const cd* d = o.m;
        if (!is_zero(d[0]) && !is_zero(d[1]) && !is_zero(d[2]) && !is_zero(d[3])) {
          // d(a, b) = d0 ra^a rb^b rab^(ab)
          gscale *= d[0];
          phase1(o.q[0], cd(1.0), d[1] / d[0]);
          phase1(o.q[1], cd(1.0), d[2] / d[0]);
          interaction(o.q[0], o.q[1], d[3] * d[0] / (d[1] * d[2]));
        } else {
          raw(w.op);
        }
      } else {  // TOP_SIGN
        for (int i : w.signs) {
          const POp& o = P[i];
          if (o.kind == PK_D1) phase1(o.q[0], cd(1.0), cd(-1.0));
          else cz(o.q[0], o.q[1]);
        }
      }
    }
    // A CNOT target's carried factor does not commute with the store map:
    // it is applied in this round.  A control's commutes and stays carried.
    for (int i : rp.cx) {
      const int p = lpos[P[i].q[1]];
      if (pd0[p] == cd(1.0) && pd1[p] == cd(1.0)) continue;
      const int j = regof[p];
      if (j >= 0) {
        tab_bit(rp, j, pd0[p], pd1[p]);
      } else {
        gscale *= pd0[p];
        const cd rr = pd1[p] / pd0[p];
        if (rr != cd(1.0)) add_term(pick(rp, 0, [&](const DGroup& g) { return has_key(g, -1); }), -1, 1u << p, 0ull, rr);
      }
      pd0[p] = pd1[p] = 1.0;
    }
  }

  // every carried factor is applied by the end of the pass
  if (!plans.empty()) {
    RPlan& rp = plans.back();
    for (int p = 0; p < t; ++p) {
      if (pd0[p] == cd(1.0) && pd1[p] == cd(1.0)) continue;
      const int j = rp.regof[p];
      if (j >= 0) {
        tab_bit(rp, j, pd0[p], pd1[p]);
      } else {
        gscale *= pd0[p];
        const cd rr = pd1[p] / pd0[p];
        if (rr != cd(1.0)) add_term(pick(rp, 0, [&](const DGroup& g) { return has_key(g, -1); }), -1, 1u << p, 0ull, rr);
      }
    }
    if (gscale != cd(1.0)) {
      cd* tbl = table_of(pick(rp, 0, [](const DGroup& g) { return g.tab; }));
      for (int m = 0; m < NR; ++m) tbl[m] *= gscale;
    }
  }

  // (p, q, c) of a diagonal factor d = (1 + c) exp(i phi), |phi| <= pi/2:
  // p = -tan(phi / 2), q = sin(phi); a negative real part goes into c
  auto factor_pqc = [](cd d, double& fp, double& fq, double& fc) {
    const double r = std::abs(d);
    if (r == 0.0) {
      fp = fq = 0.0;
      fc = -1.0;
      return;
    }
    cd u = d / r;
    double sg = 1.0;
    if (u.real() < 0.0) {
      u = -u;
      sg = -1.0;
    }
    fp = -u.imag() / (1.0 + u.real());
    fq = u.imag();
    fc = sg * r - 1.0;
  };
  constexpr int LR = LayerRec<T>::W;
  for (size_t ri = 0; ri < plans.size(); ++ri) {
    RPlan& rp = plans[ri];
    uint32_t rmask = 0;
    for (int k = 0; k < RB; ++k) rmask |= 1u << rp.R[k];
    const uint32_t tmask = t >= 32 ? ~0u : ((1u << t) - 1u);
    // records of the round: fixed fields, aux words, table index
    struct Rec {
      int32_t flags = 0;
      int tab = -1;
      int32_t pairs = 0;
      std::vector<int32_t> aux;
      std::vector<int32_t> rot = std::vector<int32_t>(LR - kRecRot, 0);
    };
    std::vector<Rec> recs;
    std::vector<std::vector<int32_t>> tables;

    // layers: the diagonal work of a group, then rotations on distinct
    // register bits with nothing diagonal between them, then at most one
    // permutation or general matrix
    struct Layer {
      int group = -1;
      std::vector<int> rots;
      int tail = -1;
    };
    auto group_empty = [&](const DGroup& g) { return !g.tab && !has_sign(g) && g.phl.empty() && g.raw.empty(); };
    std::vector<Layer> layers;
    Layer cur;
    cur.group = 0;
    uint32_t used = 0;
    auto flush = [&]() {
      const bool diag = cur.group >= 0 && !group_empty(rp.g[cur.group]);
      if (diag || !cur.rots.empty() || cur.tail >= 0) layers.push_back(cur);
      cur = Layer();
      used = 0;
    };
    for (size_t i = 0; i < rp.nd.size(); ++i) {
      const NdItem& it = rp.nd[i];
      if (it.type == TOP_GIVENS) {
        if (cur.tail >= 0 || ((used >> it.j0) & 1u)) flush();
        cur.rots.push_back((int)i);
        used |= 1u << it.j0;
      } else {
        if (cur.tail >= 0) flush();
        cur.tail = (int)i;
      }
      if (!group_empty(rp.g[i + 1])) {
        flush();
        cur.group = (int)i + 1;
      } else if (cur.tail >= 0) {
        flush();
      }
    }
    flush();

    for (const Layer& L : layers) {
      DGroup empty_group;
      DGroup& g = L.group >= 0 ? rp.g[L.group] : empty_group;
      // the diagonal table: one complex factor per register combination
      bool tab = false;
      std::vector<int32_t> tline;
      if (g.tab) {
        for (int m = 0; m < NR; ++m)
          if (cz_pairs_negate(g.pairs, m)) g.tb[m] = -g.tb[m];
        g.pairs = 0;
        bool ident = true;
        for (int m = 0; m < NR; ++m)
          if (g.tb[m] != cd(1.0)) ident = false;
        if (!ident) {
          tab = true;
          for (int m = 0; m < NR; ++m) {
            RealWords<T>::put(g.tb[m].real(), tline);
            RealWords<T>::put(g.tb[m].imag(), tline);
          }
        }
      }
      std::vector<int32_t> loc;
      for (int d = 1; d < 32; ++d)
        if (g.Md[d]) loc.insert(loc.end(), {d, (int32_t)g.Md[d]});
      const bool sign = !loc.empty() || !g.fc.empty() || !g.cc.empty();
      // extra per-group phases and raw diagonals run as diagonal-only layers first
      struct Extra {
        int kind;  // 0 phasel, 1 raw
        int idx;
      };
      std::vector<Extra> extras;
      // per-group phase steps: all terms of one register bit (or of every
      // amplitude) in one step, applied once
      std::vector<std::pair<int, std::vector<PhTerm>>> phl;
      for (auto& e : g.phl) {
        std::vector<PhTerm> terms;
        for (auto& tm : e.second)
          if (tm.r != cd(1.0)) terms.push_back(tm);
        if (!terms.empty()) phl.push_back({e.first, terms});
      }
      for (size_t e = 0; e < phl.size(); ++e) extras.push_back({0, (int)e});
      for (size_t e = 0; e < g.raw.size(); ++e) extras.push_back({1, (int)e});
      auto phasel_words = [&](std::vector<int32_t>& w, int e) {
        // terms on outside qubits only depend on the tile: their product is
        // taken once per tile into a slot of the pass's tile-factor list
        std::vector<PhTerm> terms, outside;
        bool unit = true;
        for (const PhTerm& tm : phl[e].second) {
          if (std::abs(std::abs(tm.r) - 1.0) > 1e-12) unit = false;
          (tm.lgm == 0 ? outside : terms).push_back(tm);
        }
        int slot = -1;
        if (!outside.empty() && tfac.size() < (size_t)kMaxTileFactors) {
          slot = (int)tfac.size();
          tfac.push_back(outside);
        } else {
          terms.insert(terms.end(), outside.begin(), outside.end());
        }
        // lane-table form: every term on one free bit, none on an outside
        // qubit; the product over the group's terms is one entry of each of
        // two 16-entry tables indexed by the group's compact free bits
        bool table = !terms.empty() && ltab.size() + 32 <= kLaneTab;
        cd rk[8] = {1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0};
        const uint32_t fm = tmask & ~rmask;
        for (const PhTerm& tm : terms) {
          if (!table) break;
          if (tm.om != 0 || __builtin_popcount(tm.lgm) != 1 || !(tm.lgm & fm)) {
            table = false;
            break;
          }
          const int k = __builtin_popcount(fm & (tm.lgm - 1u));
          if (k >= 8) {
            table = false;
            break;
          }
          rk[k] *= tm.r;
        }
        w.push_back(phl[e].first);
        w.push_back(slot);
        w.push_back(unit ? 1 : 0);
        if (table) {
          w.push_back(-1);
          w.push_back((int32_t)ltab.size());
          for (int half = 0; half < 2; ++half)
            for (int v = 0; v < 16; ++v) {
              cd f = 1.0;
              for (int k = 0; k < 4; ++k)
                if ((v >> k) & 1) f *= rk[4 * half + k];
              ltab.push_back(f);
            }
          return;
        }
        w.push_back((int32_t)terms.size());
        for (auto& tm : terms) {
          w.push_back((int32_t)tm.lgm);
          w.push_back((int32_t)(tm.om & 0xffffffffull));
          w.push_back((int32_t)(tm.om >> 32));
          RealWords<T>::put(tm.r.real(), w);
          RealWords<T>::put(tm.r.imag(), w);
        }
      };
      auto raw_words = [&](std::vector<int32_t>& w, int e) {
        const POp& o = P[g.raw[e]];
        int ka, va;
        operand(rp, o.q[0], ka, va);
        const int nfac = o.kind == PK_D1 ? 2 : 4;
        if (o.kind == PK_D1) {
          w.insert(w.end(), {RAW_PHASE1, ka, va});
        } else {
          int kb, vb;
          operand(rp, o.q[1], kb, vb);
          w.insert(w.end(), {RAW_DIAG2, ka, va, kb, vb});
        }
        for (int f = 0; f < nfac; ++f) {
          double fp, fq, fc;
          factor_pqc(o.m[f], fp, fq, fc);
          RealWords<T>::put(fp, w);
          RealWords<T>::put(fq, w);
          RealWords<T>::put(fc, w);
        }
      };
      // Steps in the order a layer applies them, each as (flag, payload
      // words); consecutive steps become one layer record, one step of each
      // kind per record.
      struct Blob {
        int32_t flag;
        std::vector<int32_t> w;
      };
      std::vector<Blob> blobs;
      if (tab) blobs.push_back({LT_TAB, {0}});  // line filled in at packing
      if (g.pairs) blobs.push_back({LT_CZR, {(int32_t)g.pairs}});
      {
        // conditional Z on register bit j: every register bit of a mask
        // (an XOR of single-bit masks) with its free / outside qubit
        std::vector<int32_t> ent;
        bool bad_mask = false;
        auto add_entries = [&](const std::vector<std::pair<int, uint32_t>>& v, int kind) {
          for (auto& e : v) {
            uint32_t rest = e.second;
            for (int j = 0; j < RB; ++j)
              if ((e.second >> (1u << j)) & 1u) {
                ent.push_back(j | (kind << 4) | (e.first << 8));
                rest ^= mbit(j);
              }
            if (rest) bad_mask = true;
          }
        };
        add_entries(g.fmix, TK_FREE);
        add_entries(g.rcmix, TK_OUT);
        if (bad_mask) return false;  // masks are built from single register bits only
        constexpr size_t kEntries = 16;  // entries per step
        for (size_t e0 = 0; e0 < ent.size(); e0 += kEntries) {
          const size_t ne = std::min(kEntries, ent.size() - e0);
          std::vector<int32_t> w = {(int32_t)ne};
          w.insert(w.end(), ent.begin() + e0, ent.begin() + e0 + ne);
          blobs.push_back({LT_CZF, w});
        }
      }
      if (sign) {
        // group parity terms compose by XOR: long lists are split over steps
        std::vector<int32_t> lc = loc, fcl = g.fc, ccl = g.cc;
        constexpr size_t kPairs = 12;  // list entries per sign step
        do {
          std::vector<int32_t> w;
          auto take_flat = [&](std::vector<int32_t>& v) {
            const size_t n = std::min(v.size() / 2, kPairs);
            w.push_back((int32_t)n);
            w.insert(w.end(), v.begin(), v.begin() + 2 * n);
            v.erase(v.begin(), v.begin() + 2 * n);
          };
          take_flat(lc);
          take_flat(fcl);
          take_flat(ccl);
          blobs.push_back({LT_SIGN, w});
        } while (!fcl.empty() || !lc.empty() || !ccl.empty());
      }
      for (const Extra& E : extras) {
        std::vector<int32_t> w;
        if (E.kind == 0) phasel_words(w, E.idx);
        else raw_words(w, E.idx);
        blobs.push_back({E.kind == 0 ? LT_PHASEL : LT_RAWD, w});
      }
      {
        std::vector<int> rots(L.rots);
        std::sort(rots.begin(), rots.end(), [&](int x, int y) { return rp.nd[x].j0 < rp.nd[y].j0; });
        for (int i : rots) {
          const NdItem& it = rp.nd[i];
          Blob bl{LT_ROT0 << it.j0, {}};
          if (it.jf >> 8) bl.flag |= LT_SHEAR3 << it.j0;
          RealWords<T>::put(it.p, bl.w);
          RealWords<T>::put(it.q, bl.w);
          blobs.push_back(bl);
        }
      }
      if (L.tail >= 0) {
        const NdItem& it = rp.nd[L.tail];
        Blob bl{0, {}};
        if (it.type == TOP_PERM2) {
          bl.flag = LT_PERM2;
          bl.w = {it.j0, it.j1, it.code};
        } else if (it.type == TOP_U2) {
          bl.flag = LT_U2;
          bl.w = {it.j0, it.j1};
          for (int e = 0; e < 16; ++e) {
            RealWords<T>::put(it.m[e].real(), bl.w);
            RealWords<T>::put(it.m[e].imag(), bl.w);
          }
        } else {
          bl.flag = LT_U1;
          bl.w = {it.j0};
          for (int e = 0; e < 4; ++e) {
            RealWords<T>::put(it.m[e].real(), bl.w);
            RealWords<T>::put(it.m[e].imag(), bl.w);
          }
        }
        blobs.push_back(bl);
      }
      // step kinds in application order (rotations: one kind per register bit)
      auto order = [](int32_t flag) {
        if (flag & LT_TAB) return 0;
        if (flag & LT_CZR) return 1;
        if (flag & LT_CZF) return 2;
        if (flag & LT_SIGN) return 3;
        if (flag & LT_PHASEL) return 4;
        if (flag & LT_RAWD) return 5;
        for (int j = 0; j < 8; ++j)
          if (flag & (LT_ROT0 << j)) return 6 + j;
        return 14;
      };
      // consecutive steps go into one record, one step of each kind per record
      int last = 1 << 30;
      for (const Blob& bl : blobs) {
        const int ord = order(bl.flag);
        if (ord <= last) recs.emplace_back();
        last = ord;
        Rec& rc = recs.back();
        rc.flags |= bl.flag;
        if (bl.flag & LT_TAB) {
          rc.tab = (int)tables.size();
          tables.push_back(tline);
        } else if (bl.flag & LT_CZR) {
          rc.pairs = bl.w[0];
        } else if (ord >= 6 && ord < 6 + RB) {
          const int j = ord - 6;
          for (int e = 0; e < 2 * WT; ++e) rc.rot[2 * j * WT + e] = bl.w[e];
        } else {
          rc.aux.insert(rc.aux.end(), bl.w.begin(), bl.w.end());
        }
      }
    }

    // A permutation that ends the round moves to the round header: the
    // round's store applies it by writing each register combination to the
    // slot of its image (the payload is the last aux segment of its record).
    std::vector<int32_t> hdr(kRoundHeader, 0);
    for (int k = 0; k < RB; ++k) {
      hdr[2 + k] = (int32_t)(tile_swizzle(1u << rp.R[k], SB) * (uint32_t)(2 * sizeof(T)));
      hdr[kHdrStore + k] = hdr[2 + k];
    }
    // The store map of the round's CNOTs: local index x of a tile with
    // outside bits o goes to A x + B o.  Row r of A (B) says which local
    // (outside) bits local bit r of the image is the XOR of; CNOT(c, q)
    // adds row c to row q (or outside bit c, for a control outside the tile).
    std::vector<int32_t> mapw;
    if (!rp.cx.empty()) {
      std::vector<uint32_t> rowA(t);
      std::vector<uint64_t> rowB(t, 0);
      for (int p = 0; p < t; ++p) rowA[p] = 1u << p;
      for (int i : rp.cx) {
        const int pc = lpos[P[i].q[0]], pt = lpos[P[i].q[1]];
        if (pc >= 0) {
          rowA[pt] ^= rowA[pc];
          rowB[pt] ^= rowB[pc];
        } else {
          rowB[pt] ^= 1ull << P[i].q[0];
        }
      }
      auto col_ofs = [&](auto bitof) {  // swizzled LDS offset of a column
        uint32_t v = 0;
        for (int r = 0; r < t; ++r)
          if (bitof(r)) v |= 1u << r;
        return (int32_t)(tile_swizzle(v, SB) * (uint32_t)(2 * sizeof(T)));
      };
      for (int k = 0; k < RB; ++k) {
        const int b = rp.R[k];
        hdr[kHdrStore + k] = col_ofs([&](int r) { return (rowA[r] >> b) & 1u; });
      }
      const uint32_t fm = tmask & ~rmask;
      for (int b = 0; b < t; ++b)
        if ((fm >> b) & 1u) mapw.push_back(col_ofs([&](int r) { return (rowA[r] >> b) & 1u; }));
      uint64_t outs = 0;
      for (int r = 0; r < t; ++r) outs |= rowB[r];
      mapw.push_back(__builtin_popcountll(outs));
      for (int q = 0; q < 64; ++q)
        if ((outs >> q) & 1ull) {
          mapw.push_back(q);
          mapw.push_back(col_ofs([&](int r) { return (rowB[r] >> q) & 1ull; }));
        }
    }
    if (rp.cx.empty() && !recs.empty() && (recs.back().flags & LT_PERM2)) {
      Rec& lr = recs.back();
      const size_t na = lr.aux.size();
      const int j0 = lr.aux[na - 3], j1 = lr.aux[na - 2], code = lr.aux[na - 1];
      if (code == 2) {  // SWAP: the two bits trade offsets
        hdr[kHdrStore + j0] = hdr[2 + j1];
        hdr[kHdrStore + j1] = hdr[2 + j0];
      } else if (code == 0) {  // CNOT, control j0: e_j0 -> e_j0 + e_j1
        hdr[kHdrStore + j0] = hdr[2 + j0] ^ hdr[2 + j1];
      } else {  // CNOT, control j1
        hdr[kHdrStore + j1] = hdr[2 + j1] ^ hdr[2 + j0];
      }
      lr.aux.resize(na - 3);
      lr.flags &= ~LT_PERM2;
      if (lr.flags == 0 && lr.tab < 0) recs.pop_back();
    }
    // round block: header, records, aux words, tables
    const size_t b0 = prog.size();
    prog[roff0 + ri] = (int32_t)(b0 - h0);
    hdr[0] = (int32_t)recs.size();
    hdr[1] = (int32_t)(tmask & ~rmask);
    prog.insert(prog.end(), hdr.begin(), hdr.end());
    std::vector<size_t> at(recs.size());
    for (size_t i = 0; i < recs.size(); ++i) {
      at[i] = prog.size();
      prog.resize(at[i] + LR, 0);
      int32_t* w = prog.data() + at[i];
      w[0] = recs[i].flags;
      w[2] = recs[i].pairs;
      for (int e = 0; e < LR - kRecRot; ++e) w[kRecRot + e] = recs[i].rot[e];
      if (recs[i].tab >= 0) {
        const std::vector<int32_t>& tl = tables[recs[i].tab];
        prog.insert(prog.end(), tl.begin(), tl.end());
      }
    }
    for (size_t i = 0; i < recs.size(); ++i) {
      if (recs[i].aux.empty()) continue;
      prog[at[i] + 3] = (int32_t)(prog.size() - b0);
      prog.insert(prog.end(), recs[i].aux.begin(), recs[i].aux.end());
    }
    if (!mapw.empty()) {
      prog[b0 + kHdrMap] = (int32_t)(prog.size() - b0);
      prog.insert(prog.end(), mapw.begin(), mapw.end());
    }
    while ((prog.size() - b0) % 16) prog.push_back(0);
  }
  if (!tfac.empty()) {
    // the tile-factor list after the round blocks; the first round's header
    // points to it
    const size_t l0 = prog.size();
    const size_t K = tfac.size();
    prog.resize(l0 + K, 0);
    for (size_t k = 0; k < K; ++k) {
      prog[l0 + k] = (int32_t)(prog.size() - l0);
      prog.push_back((int32_t)tfac[k].size());
      for (const PhTerm& tm : tfac[k]) {
        prog.push_back((int32_t)(tm.om & 0xffffffffull));
        prog.push_back((int32_t)(tm.om >> 32));
        RealWords<T>::put(tm.r.real(), prog);
        RealWords<T>::put(tm.r.imag(), prog);
      }
    }
    const size_t rb0 = h0 + (size_t)prog[roff0];
    prog[rb0 + kHdrTileFac] = (int32_t)(l0 - h0);
    prog[rb0 + kHdrTileFac + 1] = (int32_t)K;
    while ((prog.size() - h0) % 16) prog.push_back(0);
  }
  if (!ltab.empty()) {
    // the lane table after the round blocks (and the tile-factor list)
    const size_t l1 = prog.size();
    for (const cd& f : ltab) {
      RealWords<T>::put(f.real(), prog);
      RealWords<T>::put(f.imag(), prog);
    }
    const size_t rb0 = h0 + (size_t)prog[roff0];
    prog[rb0 + kHdrLaneTab] = (int32_t)(l1 - h0);
    prog[rb0 + kHdrLaneTabN] = (int32_t)ltab.size();
    while ((prog.size() - h0) % 16) prog.push_back(0);
  }
  return true;
}

// The smallest tile-kernel body whose steps cover a pass program.
template <typename T>
static int program_body(const int32_t* pass) {
  const int t = pass[0], nns = pass[2], nrounds = pass[3];
  const int32_t* roff = pass + 4 + t + nns;
  int body = kBodyLean;
  for (int r = 0; r < nrounds; ++r) {
    const int32_t* b = pass + roff[r];
    const int32_t* rec = b + kRoundHeader;
    for (int l = 0; l < b[0]; ++l) {
      if (rec[0] & (LT_RAWD | LT_U2 | LT_U1)) return kBodyFull;
      if (rec[0] & LT_PERM2) body = kBodyPerm;
      rec += LayerRec<T>::W + ((rec[0] & LT_TAB) ? kTableWords : 0);
    }
  }
  return body;
}

// Whether a pass program uses steps beyond the lean tile body (tables, CZ
// signs, group parities, per-group phases, rotations).
template <typename T>
static bool program_needs_full(const int32_t* pass) {
  const int t = pass[0], nns = pass[2], nrounds = pass[3];
  const int32_t* roff = pass + 4 + t + nns;
  for (int r = 0; r < nrounds; ++r) {
    const int32_t* b = pass + roff[r];
    const int32_t* rec = b + kRoundHeader;
    for (int l = 0; l < b[0]; ++l) {
      if (rec[0] & (LT_RAWD | LT_PERM2 | LT_U2 | LT_U1)) return true;
      rec += LayerRec<T>::W + ((rec[0] & LT_TAB) ? kTableWords : 0);
    }
  }
  return false;
}

// ------------------------------------------------------------- driver
// ------------------------------------------------------ autotuner cache
// Choices of the autotuners by structure hash: tile qubits for a batch;
// 100 * tile qubits + segment qubits for a single-state plan (mode 3; its
// hashes are kept apart from the batches' by a constant mixed in).  They
// persist across processes when QSV_AUTOTUNE_CACHE names a file: it is read
// once, at the first tuning of the process, and every new result is
// appended as a line "<structure hash, hex> <value>".  Unreadable lines end
// the read; a value outside the dtype's range is ignored when it is looked
// up.  Callers hold g_tune_mu.
static std::mutex g_tune_mu;
static std::unordered_map<uint64_t, int> g_tuned;
static const char* tune_cache_path() {
  const char* p = std::getenv("QSV_AUTOTUNE_CACHE");
  return (p && *p) ? p : nullptr;
}
static bool g_tune_loaded = false;
static void tuned_load_once() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = tune_cache_path();
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  unsigned long long h = 0;
  int t = 0;
  while (std::fscanf(f, "%llx %d", &h, &t) == 2) g_tuned[(uint64_t)h] = t;
  std::fclose(f);
}
static void tuned_store(uint64_t h, int t) {
  g_tuned[h] = t;
  const char* path = tune_cache_path();
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%016llx %d\n", (unsigned long long)h, t);
  std::fclose(f);
}

// Single-state autotuner (plan mode 3): the candidate shapes (tile qubits
// TBMAX and TBMAX - 1; segment qubits 5 and 4 for complex64, 4 for
// complex128) are planned, and the tile and permutation passes of each are
// timed once on a copy of the state in the second state-sized buffer (the
// per-gate steps are the same in every candidate); the fastest shape is kept
// for the structure.  Returns the tile and segment qubits to plan with.
template <typename T>
static qsv_status tuned_shape(qsv_state* s, const std::vector<qsv_op>& xops, int* t_out, int* c_out) {
  const int RB = tile_reg_bits<T>(), TBMAX = tile_max_bits<T>();
  const int n = s->n;
  const bool f32 = sizeof(T) == 4;
  std::vector<POp> P(xops.size());
  for (size_t i = 0; i < xops.size(); ++i) P[i] = classify_tile(xops[i]);
  const uint64_t h = mix(key_hash(structure_key(P, n, 0, f32 ? -1 : -2, RB)), 0x53494e474c45ull);  // "SINGLE"
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tuned_load_once();
    auto it = g_tuned.find(h);
    if (it != g_tuned.end()) {
      const int tt = it->second / 100, cc = it->second % 100;
      if (tt >= RB && tt <= std::min(TBMAX, n) && cc >= 1 && cc <= tt && n - tt <= 23) {
        *t_out = tt;
        *c_out = cc;
        return QSV_OK;
      }
    }
  }
  qsv_status st = ensure_aux(s, "hipMalloc(autotuner buffer)");
  if (st) return st;
  cpx<T>* scratch = static_cast<cpx<T>*>(s->aux);
  QSV_HIP(hipMemcpyAsync(scratch, s->psi, s->bytes, hipMemcpyDeviceToDevice, s->stream));
  hipEvent_t e0, e1;
  QSV_HIP(hipEventCreate(&e0));
  QSV_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  int best_t = std::min(TBMAX, n), best_c = 0;
  std::vector<int32_t> prog;
  qsv_status rc = QSV_OK;
  for (int tt = std::min(TBMAX, n); tt >= std::max(RB, std::min(TBMAX, n) - 1) && !rc; --tt) {
    if (n - tt > 23) continue;
    for (int cc : (f32 ? std::vector<int>{5, 4} : std::vector<int>{4})) {
      if (cc > tt) continue;
      auto sch = plan_schedule(xops, n, tt, f32, RB, cc);
      std::vector<qsv_op> rbuf;
      const std::vector<qsv_op>& sops = step_ops(*sch, xops, n, rbuf);
      std::vector<POp> SP(sops.size());
      for (size_t i = 0; i < sops.size(); ++i) SP[i] = classify_tile(sops[i]);
      prog.clear();
      std::vector<size_t> offs;
      bool ok = true;
      for (const Step& stp : sch->steps) {
        offs.push_back(prog.size());
        if (!stp.inv.empty()) emit_qperm<T>(stp.inv, n, prog);
        if (stp.tile) ok = ok && emit_pass<T>(stp, SP, n, sch->c, RB, prog);
      }
      if (!ok) continue;
      const size_t need = prog.size() * sizeof(int32_t) + kProgSlackBytes;
      if (s->pbuf_bytes < need) {
        QSV_HIP(hipStreamSynchronize(s->stream));
        if (s->pbuf) QSV_HIP(hipFree(s->pbuf));
        s->pbuf = nullptr;
        s->pbuf_bytes = 0;
        QSV_HIP(hipMalloc(&s->pbuf, need * 2));
        s->pbuf_bytes = need * 2;
      }
      int32_t* dprog = static_cast<int32_t*>(s->pbuf);
      if (!prog.empty())
        QSV_HIP(hipMemcpyAsync(dprog, prog.data(), prog.size() * sizeof(int32_t), hipMemcpyHostToDevice, s->stream));
      QSV_HIP(hipEventRecord(e0, s->stream));
      for (size_t k = 0; k < sch->steps.size(); ++k) {
        const Step& stp = sch->steps[k];
        const int32_t* ph = prog.data() + offs[k];
        if (!stp.inv.empty())
          QSV_HIP(launch_qperm<T>(scratch, scratch, n, dprog + offs[k], ph, s->stream));
        else if (stp.tile)
          QSV_HIP(launch_tile_pass<T>(scratch, n, dprog + offs[k], ph, program_body<T>(ph), s->stream));
      }
      QSV_HIP(hipEventRecord(e1, s->stream));
      QSV_HIP(hipEventSynchronize(e1));  // also keeps prog alive for the upload
      float ms = 0;
      QSV_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) {
        best = ms;
        best_t = tt;
        best_c = sch->c;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (best_c == 0) best_c = std::min(f32 ? 5 : 4, best_t);  // no candidate could be encoded
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tuned_store(h, 100 * best_t + best_c);
  }
  *t_out = best_t;
  *c_out = best_c;
  return QSV_OK;
}

// Launch a plan whose steps are all tile passes through the state's graph:
// capture the passes once for what their launches depend on (the signature
// below), replay afterwards.  The program words were uploaded to dprog on
// the same stream just before, so a replay runs this call's angles.
template <typename T>
static qsv_status launch_fused_graph(qsv_state* s, const Schedule& sch, const std::vector<int32_t>& prog,
                                     const std::vector<size_t>& offs, const int32_t* dprog) {
  std::vector<uint64_t> sig = {sizeof(T), (uint64_t)s->n, (uint64_t)(uintptr_t)s->psi, (uint64_t)(uintptr_t)dprog,
                               (uint64_t)(uintptr_t)s->stream};
  std::vector<int> body(sch.steps.size());
  for (size_t k = 0; k < sch.steps.size(); ++k) {
    const int32_t* ph = prog.data() + offs[k];
    body[k] = sch.steps[k].tile ? program_body<T>(ph) : -1;   // -1: qubit-permutation pass
    sig.insert(sig.end(), {(uint64_t)offs[k], (uint64_t)(int64_t)body[k], (uint64_t)ph[0], (uint64_t)ph[1]});
  }
  if (!s->fg_exec || sig != s->fg_sig) {
    if (s->fg_exec) (void)hipGraphExecDestroy(s->fg_exec);
    if (s->fg_graph) (void)hipGraphDestroy(s->fg_graph);
    s->fg_exec = nullptr;
    s->fg_graph = nullptr;
    s->fg_sig.clear();
    QSV_HIP(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (size_t k = 0; k < sch.steps.size() && e == hipSuccess; ++k)
      e = body[k] < 0 ? launch_qperm<T>(static_cast<cpx<T>*>(s->psi), static_cast<cpx<T>*>(s->psi), s->n,
                                        dprog + offs[k], prog.data() + offs[k], s->stream)
                      : launch_tile_pass<T>(static_cast<cpx<T>*>(s->psi), s->n, dprog + offs[k],
                                            prog.data() + offs[k], body[k], s->stream);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(s->stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return hip_fail(e != hipSuccess ? e : e2, "fused plan capture");
    }
    hipGraphExec_t x = nullptr;
    const hipError_t e3 = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e3 != hipSuccess) {
      (void)hipGraphDestroy(g);
      return hip_fail(e3, "hipGraphInstantiate(fused plan)");
    }
    s->fg_graph = g;
    s->fg_exec = x;
    s->fg_sig = std::move(sig);
  }
  QSV_HIP(hipGraphLaunch(s->fg_exec, s->stream));
  return QSV_OK;
}

// The race check of a fused plan (plan option race_check): every tile and
// permutation pass runs first out of place, from the state into the second
// state-sized buffer filled with a poison pattern, then in place as usual.
// In place is race-free when every amplitude belongs to exactly one
// workgroup and is read before it is written: the out-of-place run must
// then write every amplitude (no poison left) and produce the in-place
// result bit for bit (the same arithmetic; a read of an amplitude that
// another workgroup had already updated would differ).  The per-gate steps
// run as usual.  Synchronous per pass.
template <typename T>
static qsv_status run_race_checked(qsv_state* s, const Schedule& sch, const std::vector<qsv_op>& sops,
                                   const std::vector<int32_t>& prog, const std::vector<size_t>& offs,
                                   const int32_t* dprog) {
  qsv_status st0 = ensure_aux(s, "hipMalloc(race check buffer)");
  if (st0) return st0;
  st0 = ensure_workspace(s, std::max(dense_ws_bytes(), (size_t)256));
  if (st0) return st0;
  cpx<T>* psi = static_cast<cpx<T>*>(s->psi);
  cpx<T>* out = static_cast<cpx<T>*>(s->aux);
  const uint64_t nvec = s->bytes / 16;
  for (size_t k = 0; k < sch.steps.size(); ++k) {
    const Step& st = sch.steps[k];
    if (!st.tile && st.inv.empty()) {
      qsv_status e = apply_op_pergate(s, sops[st.op], 0);
      if (e) return e;
      continue;
    }
    const int32_t* ph = prog.data() + offs[k];
    // the workspace is free between steps: the counters live at its start
    unsigned long long* counts = static_cast<unsigned long long*>(s->ws);
    QSV_HIP(hipMemsetAsync(counts, 0, 2 * sizeof(unsigned long long), s->stream));
    QSV_HIP(launch_poison(out, nvec, s->stream));
    if (st.tile) {
      const int body = program_body<T>(ph);
      QSV_HIP(launch_tile_pass_oop<T>(psi, out, s->n, dprog + offs[k], ph, body, s->stream));
      QSV_HIP(launch_tile_pass<T>(psi, s->n, dprog + offs[k], ph, body, s->stream));
    } else {
      QSV_HIP(launch_qperm<T>(psi, out, s->n, dprog + offs[k], ph, s->stream));
      QSV_HIP(launch_qperm<T>(psi, psi, s->n, dprog + offs[k], ph, s->stream));
    }
    QSV_HIP(launch_race_compare(psi, out, nvec, counts, s->stream));
    unsigned long long h[2] = {0, 0};
    QSV_HIP(hipMemcpyAsync(h, counts, sizeof(h), hipMemcpyDeviceToHost, s->stream));
    QSV_HIP(hipStreamSynchronize(s->stream));
    if (h[0] || h[1])
      return fail(QSV_ERR_STATE, "race check: pass " + std::to_string(k) + " (" + (st.tile ? "tile" : "permutation") +
                                     ") left " + std::to_string(h[0]) + " words unwritten and " +
                                     std::to_string(h[1]) + " words different out of place");
  }
  return QSV_OK;
}

template <typename T>
static qsv_status run_fused_T(qsv_state* s, const qsv_op* ops, int n_ops, const qsv_plan_opts& opts) {
  const int RB = tile_reg_bits<T>();
  const int TBMAX = tile_max_bits<T>();
  const int n = s->n;
  if (n < RB) {  // register smaller than one register group: per-gate kernels
    qsv_status sw = ensure_workspace(s, dense_ws_bytes());  // dense blocks stage their matrix there
    if (sw) return sw;
    for (int i = 0; i < n_ops; ++i) {
      qsv_status st = apply_op_pergate(s, ops[i], 0);
      if (st) return st;
    }
    return QSV_OK;
  }
  std::vector<qsv_op> xops(ops, ops + n_ops);  // the list the plan and its per-gate steps refer to
  ops = xops.data();
  n_ops = (int)xops.size();
  int t = opts.tile_qubits > 0 ? opts.tile_qubits : default_tile_bits<T>();
  if (t > TBMAX) return fail(QSV_ERR_UNSUPPORTED, "tile_qubits exceeds the LDS tile capacity");
  if (t < RB) return fail(QSV_ERR_ARG, "tile_qubits smaller than the register group");
  if (t > n) t = n;
  // one workgroup per tile in the non-persistent tile kernel: the launch's
  // work-items (2^(n-t) * 256) must stay below 2^32
  if (n - t > 23) return fail(QSV_ERR_UNSUPPORTED, "tile_qubits too small for this register (over 2^23 tiles)");
  int force_c = 0;  // segment qubits chosen by the autotuner (0: by the planner)
  if (opts.mode == 3 && opts.tile_qubits == 0) {
    qsv_status st = tuned_shape<T>(s, xops, &t, &force_c);
    if (st) return st;
  }
  std::vector<POp> P(n_ops);
  for (int i = 0; i < n_ops; ++i) P[i] = classify_tile(ops[i]);
  // the key carries the dtype in place of the segment width when the
  // planner chooses it (the cached schedule holds the width it chose)
  std::vector<uint32_t> key = structure_key(P, n, t, force_c ? force_c : (sizeof(T) == 4 ? -1 : -2), RB);
  const uint64_t h = key_hash(key);
  std::shared_ptr<Schedule> sch;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_cache.find(h);
    if (it != g_cache.end() && it->second->key == key) sch = it->second;
  }
  if (!sch) {
    sch = plan_schedule(xops, n, t, sizeof(T) == 4, RB, force_c);
    sch->key = std::move(key);
    std::lock_guard<std::mutex> lk(g_cache_mu);
    if (g_cache.size() > 256) g_cache.clear();
    g_cache[h] = sch;
  }
  // the ops the steps index (SWAPs relabeled away when the plan chose so)
  std::vector<qsv_op> rbuf;
  const std::vector<qsv_op>& sops = step_ops(*sch, xops, n, rbuf);
  if (sch->relabeled) {
    P.resize(sops.size());
    for (size_t i = 0; i < sops.size(); ++i) P[i] = classify_tile(sops[i]);
  }
  // materialise programs for all tile and permutation steps
  std::vector<int32_t>& prog = s->hprog;
  prog.clear();
  std::vector<size_t> offs;
  for (const Step& st : sch->steps) {
    offs.push_back(prog.size());
    if (!st.inv.empty()) emit_qperm<T>(st.inv, n, prog);
    if (st.tile && !emit_pass<T>(st, P, n, sch->c, RB, prog)) return fail(QSV_ERR_UNSUPPORTED, "a fused tile pass could not be encoded");
  }
  const size_t need = prog.size() * sizeof(int32_t) + kProgSlackBytes;
  if (s->pbuf_bytes < need) {
    if (s->pbuf) {
      QSV_HIP(hipStreamSynchronize(s->stream));
      QSV_HIP(hipFree(s->pbuf));
      s->pbuf = nullptr;
      s->pbuf_bytes = 0;
    }
    const size_t want = need < (1u << 20) ? (1u << 20) : need * 2;
    QSV_HIP(hipMalloc(&s->pbuf, want));
    s->pbuf_bytes = want;
  }
  int32_t* dprog = static_cast<int32_t*>(s->pbuf);
  if (!prog.empty())
    QSV_HIP(hipMemcpyAsync(dprog, prog.data(), prog.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                           s->stream));
  qsv_status st0 = ensure_workspace(s, dense_ws_bytes());
  if (st0) return st0;
  bool all_tile = true;
  for (const Step& st : sch->steps) all_tile = all_tile && (st.tile || !st.inv.empty());
  if (opts.graph && all_tile) return launch_fused_graph<T>(s, *sch, prog, offs, dprog);
  if (opts.race_check) return run_race_checked<T>(s, *sch, sops, prog, offs, dprog);
  for (size_t k = 0; k < sch->steps.size(); ++k) {
    const Step& st = sch->steps[k];
    if (!st.inv.empty()) {
      QSV_HIP(launch_qperm<T>(static_cast<cpx<T>*>(s->psi), static_cast<cpx<T>*>(s->psi), n, dprog + offs[k],
                              prog.data() + offs[k], s->stream));
      continue;
    }
    if (!st.tile) {
      qsv_status e = apply_op_pergate(s, sops[st.op], 0);
      if (e) return e;
      continue;
    }
    QSV_HIP(launch_tile_pass<T>(static_cast<cpx<T>*>(s->psi), n, dprog + offs[k], prog.data() + offs[k],
                                program_body<T>(prog.data() + offs[k]), s->stream));
  }
  return QSV_OK;
}

void plan_adjoint(const qsv_op* ops, int n_ops, int n, int t, int c, int RB, std::vector<AdjStep>& steps) {
  std::vector<POp> P;
  std::vector<int> orig;
  for (int k = n_ops - 1; k >= 0; --k) {
    P.push_back(classify(ops[k]));
    orig.push_back(k);
  }
  auto sch = build_schedule(P, n, t, c, RB);
  steps.clear();
  for (const Step& st : sch->steps) {
    AdjStep a;
    a.tile = st.tile;
    a.S = st.S;
    if (!st.tile) a.op = orig[st.op];
    for (const Round& r : st.rounds)
      for (int i : r.ops) a.ops.push_back(orig[i]);
    steps.push_back(std::move(a));
  }
}

// QSV_FORCE_PERGATE=1 in the environment turns the automatic mode into the
// per-gate form (read at first use, and again after qsv_debug_reload_env): a
// switch for comparing the two forms, or for isolating a planner problem,
// without changing the caller.
static std::atomic<int> g_env_pergate{-1};
static bool force_pergate() {
  int v = g_env_pergate.load();
  if (v < 0) {
    const char* e = std::getenv("QSV_FORCE_PERGATE");
    v = (e && e[0] == '1' && e[1] == 0) ? 1 : 0;
    g_env_pergate.store(v);
  }
  return v != 0;
}

qsv_status run_circuit(qsv_state* s, const qsv_op* ops, int n_ops, const qsv_plan_opts& opts) {
  if (opts.mode == 1 || (opts.mode == 0 && force_pergate())) {
    qsv_status st = ensure_workspace(s, dense_ws_bytes());
    if (st) return st;
    for (int i = 0; i < n_ops; ++i) {
      st = apply_op_pergate(s, ops[i], 0);
      if (st) return st;
    }
    return QSV_OK;
  }
  return s->dt == QSV_C64 ? run_fused_T<float>(s, ops, n_ops, opts)
                          : run_fused_T<double>(s, ops, n_ops, opts);
}

// Program image of the fused plan (diagnostics and host-side emulation):
// the int32 words of every tile pass concatenated, and per step either the
// word offset of its pass or -(1 + op index) for an op run by its own kernel.
qsv_status plan_program(const qsv_state* s, const qsv_op* ops, int n_ops, int tile_qubits,
                        std::vector<int32_t>& prog, std::vector<int64_t>& steps) {
  const bool f = s->dt == QSV_C64;
  const int RB = f ? tile_reg_bits<float>() : tile_reg_bits<double>();
  const int TBMAX = f ? tile_max_bits<float>() : tile_max_bits<double>();
  int t = tile_qubits > 0 ? tile_qubits : (f ? default_tile_bits<float>() : default_tile_bits<double>());
  if (t > TBMAX || t < RB) return fail(QSV_ERR_ARG, "bad tile_qubits");
  const int n = s->n;
  if (n < RB) return fail(QSV_ERR_UNSUPPORTED, "register smaller than the register group");
  if (t > n) t = n;
  // per-gate steps index this list (SWAPs relabeled away when the plan ends
  // in qubit-permutation passes)
  std::vector<qsv_op> xops(ops, ops + n_ops);
  auto sch = plan_schedule(xops, n, t, f, RB);
  std::vector<qsv_op> rbuf;
  const std::vector<qsv_op>& sops = step_ops(*sch, xops, n, rbuf);
  std::vector<POp> P(sops.size());
  for (size_t i = 0; i < sops.size(); ++i) P[i] = classify_tile(sops[i]);
  const int c = sch->c;
  prog.clear();
  steps.clear();
  for (const Step& st : sch->steps) {
    if (!st.inv.empty()) {
      steps.push_back((int64_t)prog.size());
      if (f)
        emit_qperm<float>(st.inv, n, prog);
      else
        emit_qperm<double>(st.inv, n, prog);
      continue;
    }
    if (!st.tile) {
      steps.push_back(-(int64_t)(1 + st.op));
      continue;
    }
    steps.push_back((int64_t)prog.size());
    const bool ok = f ? emit_pass<float>(st, P, n, c, RB, prog) : emit_pass<double>(st, P, n, c, RB, prog);
    if (!ok) return fail(QSV_ERR_UNSUPPORTED, "a fused tile pass could not be encoded");
  }
  return QSV_OK;
}

// Number of HBM passes the fused planner uses for a gate list (diagnostics).
qsv_status plan_passes(const qsv_state* s, const qsv_op* ops, int n_ops, int tile_qubits,
                       int* passes, int* fallback_ops) {
  const bool f = s->dt == QSV_C64;
  const int RB = f ? tile_reg_bits<float>() : tile_reg_bits<double>();
  const int TBMAX = f ? tile_max_bits<float>() : tile_max_bits<double>();
  int t = tile_qubits > 0 ? tile_qubits : (f ? default_tile_bits<float>() : default_tile_bits<double>());
  if (t > TBMAX || t < RB) return fail(QSV_ERR_ARG, "bad tile_qubits");
  const int n = s->n;
  if (t > n) t = n;
  std::vector<qsv_op> xops(ops, ops + n_ops);
  auto sch = plan_schedule(xops, n, t, f, RB);
  int fb = 0;
  for (const Step& st : sch->steps) fb += (st.tile || !st.inv.empty()) ? 0 : 1;
  if (passes) *passes = sch->passes;
  if (fallback_ops) *fallback_ops = fb;
  return QSV_OK;
}

}  // namespace qsv

// ====================================================================
// Batches of independent circuits: one persistent launch, captured as a
// hipGraph, with the tile width chosen by timing (autotuner).
// ====================================================================
namespace qsv {

template <typename T>
hipError_t launch_batch(cpx<T>* scratch, const int32_t* progs, const int64_t* passoff,
                        const int64_t* jobs, const uint64_t* zt, const uint32_t* zlt, const double* ct,
                        double* out, int* counter, int njobs, int grid, bool full, hipStream_t st);

}  // namespace qsv

struct qsv_batch {
  uint32_t magic = 0x48544142u;  // "BATH"
  qsv_dtype dt = QSV_C64;
  hipStream_t stream = nullptr;
  int ncirc = 0;
  std::vector<int> width, op_off, term_off;
  std::vector<qsv_op> ops;                 // structure copy (matrix pointers cleared)
  std::vector<uint64_t> op_sig;            // per-op class and qubits (update checks)
  std::vector<uint32_t> key;               // exact structure of all circuits
  int tile_bits = 0;
  bool full = false;  // the captured kernel has the full tile body
  int grid = 0;
  int njobs = 0;
  int total_passes = 0;
  size_t scratch_amps = 0;
  std::vector<int64_t> job_words, passoff;
  std::vector<int32_t> hprog;
  std::vector<uint64_t> hz;
  std::vector<double> hc;
  std::vector<uint32_t> hzl;  // per term: its Z mask over the local bits of the circuit's last pass
  // device buffers
  int32_t* d_prog = nullptr;
  size_t prog_cap = 0;  // words allocated for d_prog (updates may change the size)
  int64_t* d_passoff = nullptr;
  int64_t* d_jobs = nullptr;
  uint64_t* d_z = nullptr;
  uint32_t* d_zl = nullptr;
  double* d_c = nullptr;
  void* d_scratch = nullptr;
  double* d_out = nullptr;
  int* d_counter = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace qsv {

static std::mutex g_batch_mu;
static std::unordered_set<const qsv_batch*> g_batches;

static void batch_release_device(qsv_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  void* ptrs[] = {b->d_prog, b->d_passoff, b->d_jobs, b->d_z, b->d_zl, b->d_c, b->d_scratch, b->d_out,
                  b->d_counter};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  b->d_prog = nullptr;
  b->d_passoff = nullptr;
  b->d_jobs = nullptr;
  b->d_z = nullptr;
  b->d_zl = nullptr;
  b->d_c = nullptr;
  b->d_scratch = nullptr;
  b->d_out = nullptr;
  b->d_counter = nullptr;
}

// Programs of every circuit for tile width t (host images only).
template <typename T>
static qsv_status batch_materialise(qsv_batch* b, int t, bool check_only_structure) {
  const int RB = tile_reg_bits<T>();
  b->hprog.clear();
  b->passoff.clear();
  b->hzl.assign(b->hz.size(), 0u);
  std::vector<int64_t> first(b->ncirc), npass(b->ncirc);
  std::vector<int> neff(b->ncirc);
  for (int ci = 0; ci < b->ncirc; ++ci) {
    const int n = std::max(b->width[ci], RB);
    neff[ci] = n;
    const int tc = std::min(t, n);
    int c = sizeof(T) == 4 ? 5 : 4;
    if (c > tc) c = tc;
    const int o0 = b->op_off[ci], o1 = b->op_off[ci + 1];
    std::vector<qsv_op> xops(b->ops.data() + o0, b->ops.data() + o1);
    // A circuit held in one register group (n <= RB) applies its CNOTs in
    // registers as H CZ H: there a store map would only add rounds.
    const bool maps = n > RB;
    if (!maps) {
      std::vector<qsv_op> e;
      expand_cnots(xops.data(), (int)xops.size(), e);
      xops.swap(e);
    }
    std::vector<POp> P(xops.size());
    for (size_t i = 0; i < xops.size(); ++i) P[i] = maps ? classify_tile(xops[i]) : classify(xops[i]);
    auto plan_c = [&](int cc) {
      std::vector<uint32_t> key = structure_key(P, n, tc, cc, RB);
      const uint64_t h = key_hash(key);
      std::shared_ptr<Schedule> found;
      {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto it = g_cache.find(h);
        if (it != g_cache.end() && it->second->key == key) found = it->second;
      }
      if (!found) {
        found = build_schedule(P, n, tc, cc, RB);
        found->key = std::move(key);
        std::lock_guard<std::mutex> lk(g_cache_mu);
        if (g_cache.size() > 4096) g_cache.clear();
        g_cache[h] = found;
      }
      return found;
    };
    std::shared_ptr<Schedule> sch = plan_c(c);
    // complex64 over several tiles: 128-byte segments leave each tile one
    // more qubit of its own, kept when that needs fewer passes (as for
    // single states; the 19- and 20-qubit HEA circuits: 8 -> 6 and 7)
    if (sizeof(T) == 4 && n > tc && c == 5) {
      std::shared_ptr<Schedule> alt = plan_c(4);
      if (alt->passes < sch->passes) {
        sch = alt;
        c = 4;
      }
    }
    first[ci] = (int64_t)b->passoff.size();
    int np = 0;
    for (const Step& st : sch->steps) {
      if (!st.tile)
        return fail(QSV_ERR_UNSUPPORTED,
                    "batched circuits support gates on at most 2 qubits (circuit " +
                        std::to_string(ci) + ")");
      b->passoff.push_back((int64_t)b->hprog.size());
      if (!emit_pass<T>(st, P, n, c, RB, b->hprog)) return fail(QSV_ERR_UNSUPPORTED, "a fused tile pass could not be encoded");
      ++np;
    }
    if (np == 0) {  // empty circuit: one pass with no rounds still builds and reduces the state
      Step st;
      for (int q = 0; q < tc; ++q) st.S.push_back(q);
      b->passoff.push_back((int64_t)b->hprog.size());
      if (!emit_pass<T>(st, P, n, c, RB, b->hprog)) return fail(QSV_ERR_UNSUPPORTED, "a fused tile pass could not be encoded");
      np = 1;
    }
    npass[ci] = np;
    // the terms' Z masks over the local bits of the last pass (it reduces)
    std::vector<int> S0;
    const std::vector<int>* Sl = &S0;
    if (!sch->steps.empty()) {
      Sl = &sch->steps.back().S;
    } else {
      for (int q = 0; q < tc; ++q) S0.push_back(q);
    }
    for (int64_t k = b->term_off[ci]; k < b->term_off[ci + 1] && (size_t)k < b->hz.size(); ++k)
      for (size_t j = 0; j < Sl->size(); ++j)
        if ((b->hz[(size_t)k] >> (*Sl)[j]) & 1ull) b->hzl[(size_t)k] |= 1u << j;
  }
  if (check_only_structure) return QSV_OK;
  // jobs, largest first
  std::vector<int> order(b->ncirc);
  for (int i = 0; i < b->ncirc; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    const double cx = std::ldexp((double)(b->op_off[x + 1] - b->op_off[x] + 1), neff[x]);
    const double cy = std::ldexp((double)(b->op_off[y + 1] - b->op_off[y] + 1), neff[y]);
    return cx > cy;
  });
  b->job_words.assign((size_t)b->ncirc * 8, 0);
  b->scratch_amps = 0;
  b->total_passes = 0;
  for (int k = 0; k < b->ncirc; ++k) {
    const int ci = order[k];
    int64_t* J = &b->job_words[(size_t)k * 8];
    J[0] = neff[ci];
    J[1] = npass[ci];
    J[2] = first[ci];
    J[3] = (int64_t)b->scratch_amps;
    J[4] = b->term_off[ci];
    J[5] = b->term_off[ci + 1] - b->term_off[ci];
    J[6] = ci;
    if (npass[ci] > 1) b->scratch_amps += (size_t)1 << neff[ci];
    b->total_passes += (int)npass[ci];
  }
  b->njobs = b->ncirc;
  return QSV_OK;
}

template <typename T>
static qsv_status batch_capture(qsv_batch* b);

template <typename T>
static qsv_status batch_build(qsv_batch* b, int t) {
  batch_release_device(b);
  qsv_status st = batch_materialise<T>(b, t, false);
  if (st) return st;
  b->tile_bits = t;
  auto dalloc = [&](void** p, size_t bytes) -> qsv_status {
    hipError_t e = hipMalloc(p, bytes < 256 ? 256 : bytes);
    if (e != hipSuccess) {
      *p = nullptr;
      return hip_fail(e, "hipMalloc(batch)");
    }
    return QSV_OK;
  };
  // Tables and per-group phases that come out as identities are left out,
  // so new angles can change the program size: keep room for updates.
  b->prog_cap = b->hprog.size() * 2 + 4096;
  if ((st = dalloc((void**)&b->d_prog, b->prog_cap * 4))) return st;
  if ((st = dalloc((void**)&b->d_passoff, b->passoff.size() * 8))) return st;
  if ((st = dalloc((void**)&b->d_jobs, b->job_words.size() * 8))) return st;
  if ((st = dalloc((void**)&b->d_z, b->hz.size() * 8))) return st;
  if ((st = dalloc((void**)&b->d_zl, b->hzl.size() * 4))) return st;
  if ((st = dalloc((void**)&b->d_c, b->hc.size() * 8))) return st;
  if ((st = dalloc(&b->d_scratch, b->scratch_amps * sizeof(cpx<T>)))) return st;
  if ((st = dalloc((void**)&b->d_out, (size_t)b->ncirc * 8))) return st;
  if ((st = dalloc((void**)&b->d_counter, 256))) return st;
  QSV_HIP(hipMemcpy(b->d_prog, b->hprog.data(), b->hprog.size() * 4, hipMemcpyHostToDevice));
  QSV_HIP(hipMemcpy(b->d_passoff, b->passoff.data(), b->passoff.size() * 8, hipMemcpyHostToDevice));
  QSV_HIP(hipMemcpy(b->d_jobs, b->job_words.data(), b->job_words.size() * 8, hipMemcpyHostToDevice));
  if (!b->hz.empty()) {
    QSV_HIP(hipMemcpy(b->d_z, b->hz.data(), b->hz.size() * 8, hipMemcpyHostToDevice));
    QSV_HIP(hipMemcpy(b->d_zl, b->hzl.data(), b->hzl.size() * 4, hipMemcpyHostToDevice));
    QSV_HIP(hipMemcpy(b->d_c, b->hc.data(), b->hc.size() * 8, hipMemcpyHostToDevice));
  }
  int dev = 0, cus = 0;
  QSV_HIP(hipGetDevice(&dev));
  QSV_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  b->grid = std::max(1, std::min(b->njobs, 2 * cus));  // two 64 KiB-LDS workgroups per CU
  return batch_capture<T>(b);
}

// Captures the counter reset and the persistent kernel (lean, or full when a
// program needs it) into the batch's graph; runs replay it.
template <typename T>
static qsv_status batch_capture(qsv_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  QSV_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  bool full = false;  // the lean kernel unless some pass needs the full tile body
  for (int64_t off : b->passoff) full = full || program_needs_full<T>(b->hprog.data() + off);
  b->full = full;
  hipError_t e = launch_batch<T>(static_cast<cpx<T>*>(b->d_scratch), b->d_prog, b->d_passoff,
                                 b->d_jobs, b->d_z, b->d_zl, b->d_c, b->d_out, b->d_counter, b->njobs,
                                 b->grid, full, b->stream);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(b->stream, &g);
  if (e != hipSuccess) return hip_fail(e, "batch launch capture");
  if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
  b->graph = g;
  QSV_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  return QSV_OK;
}

static qsv_status batch_time(qsv_batch* b, float* ms) {
  hipEvent_t e0, e1;
  QSV_HIP(hipEventCreate(&e0));
  QSV_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  for (int r = 0; r < 2; ++r) {
    QSV_HIP(hipEventRecord(e0, b->stream));
    QSV_HIP(hipGraphLaunch(b->exec, b->stream));
    QSV_HIP(hipEventRecord(e1, b->stream));
    QSV_HIP(hipEventSynchronize(e1));
    float t = 0;
    QSV_HIP(hipEventElapsedTime(&t, e0, e1));
    if (r > 0 || true) best = std::min(best, t);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = best;
  return QSV_OK;
}

template <typename T>
static qsv_status batch_create_T(qsv_batch* b, int tile_qubits) {
  const int TBMAX = tile_max_bits<T>(), RB = tile_reg_bits<T>();
  if (tile_qubits > 0) {
    if (tile_qubits > TBMAX || tile_qubits < RB)
      return fail(QSV_ERR_ARG, "tile_qubits outside [register group, LDS capacity]");
    return batch_build<T>(b, tile_qubits);
  }
  // autotuner: candidate tile widths timed on the real batch, cached by structure
  const uint64_t h = key_hash(b->key);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tuned_load_once();
    auto it = g_tuned.find(h);
    if (it != g_tuned.end() && it->second >= RB && it->second <= TBMAX) return batch_build<T>(b, it->second);
  }
  int maxw = 0;
  for (int w : b->width) maxw = std::max(maxw, w);
  std::vector<int> cands;
  for (int t = TBMAX; t >= std::max(RB, TBMAX - 2); --t) cands.push_back(t);
  if (maxw <= TBMAX - 2) cands = {TBMAX};  // every circuit fits one tile at any candidate
  int best_t = cands[0];
  float best_ms = 1e30f;
  for (int t : cands) {
    qsv_status st = batch_build<T>(b, t);
    if (st) return st;
    float ms = 0;
    st = batch_time(b, &ms);
    if (st) return st;
    if (ms < best_ms) {
      best_ms = ms;
      best_t = t;
    }
  }
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tuned_store(h, best_t);
  }
  if (best_t != b->tile_bits) return batch_build<T>(b, best_t);
  return QSV_OK;
}

}  // namespace qsv

using namespace qsv;

extern "C" {

qsv_status qsv_batch_create(qsv_dtype dtype, int n_circuits, const int32_t* widths,
                            const int32_t* op_offsets, const qsv_op* ops,
                            const int32_t* term_offsets, const uint64_t* zmask, const double* coeff,
                            int tile_qubits, qsv_batch** out) {
  if (!out) return fail(QSV_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (dtype != QSV_C64 && dtype != QSV_C128) return fail(QSV_ERR_ARG, "bad dtype");
  if (n_circuits < 1 || !widths || !op_offsets || !term_offsets)
    return fail(QSV_ERR_ARG, "need at least one circuit and its offsets");
  if (op_offsets[0] != 0 || term_offsets[0] != 0) return fail(QSV_ERR_ARG, "offsets must start at 0");
  for (int i = 0; i < n_circuits; ++i) {
    if (widths[i] < 1 || widths[i] > 30) return fail(QSV_ERR_ARG, "batch widths must be in [1, 30]");
    if (op_offsets[i + 1] < op_offsets[i] || term_offsets[i + 1] < term_offsets[i])
      return fail(QSV_ERR_ARG, "offsets must be non-decreasing");
  }
  const int nops = op_offsets[n_circuits], nterms = term_offsets[n_circuits];
  if (nops > 0 && !ops) return fail(QSV_ERR_ARG, "ops is NULL");
  if (nterms > 0 && (!zmask || !coeff)) return fail(QSV_ERR_ARG, "term arrays are NULL");
  std::unique_ptr<qsv_batch> b(new qsv_batch());
  b->dt = dtype;
  b->ncirc = n_circuits;
  b->width.assign(widths, widths + n_circuits);
  b->op_off.assign(op_offsets, op_offsets + n_circuits + 1);
  b->term_off.assign(term_offsets, term_offsets + n_circuits + 1);
  for (int ci = 0; ci < n_circuits; ++ci) {
    qsv_state tmp;
    tmp.n = widths[ci];
    tmp.dt = dtype;
    tmp.N = 1ull << widths[ci];
    for (int i = op_offsets[ci]; i < op_offsets[ci + 1]; ++i) {
      qsv_status st = validate_op(&tmp, ops[i]);
      if (st) return fail(st, "circuit " + std::to_string(ci) + " op " + std::to_string(i) + ": " + get_error());
    }
    const uint64_t lim = (1ull << widths[ci]) - 1;
    for (int t = term_offsets[ci]; t < term_offsets[ci + 1]; ++t) {
      if (zmask[t] & ~lim) return fail(QSV_ERR_ARG, "Z mask names a qubit beyond the circuit width");
      if (!std::isfinite(coeff[t])) return fail(QSV_ERR_ARG, "non-finite coefficient");
    }
  }
  b->ops.assign(ops, ops + nops);
  b->hz.assign(zmask, zmask + nterms);
  b->hc.assign(coeff, coeff + nterms);
  // per-op structural signature, and the exact structure of the whole batch
  // (autotuner cache key)
  auto sig = [](const POp& p) {
    uint64_t v = (uint64_t)p.kind | ((uint64_t)p.sign << 4) | ((uint64_t)p.nq << 5);
    for (int j = 0; j < p.nq && j < 6; ++j) v |= (uint64_t)(p.q[j] & 63) << (8 + 6 * j);
    return v;
  };
  b->op_sig.resize(nops);
  for (int i = 0; i < nops; ++i) b->op_sig[i] = sig(classify(ops[i]));
  b->key = {(uint32_t)dtype, (uint32_t)n_circuits};
  for (int ci = 0; ci < n_circuits; ++ci) {
    b->key.push_back((uint32_t)widths[ci]);
    for (int i = op_offsets[ci]; i < op_offsets[ci + 1]; ++i) {
      const POp p = classify(ops[i]);
      b->key.push_back((uint32_t)p.kind | ((uint32_t)p.sign << 8) | ((uint32_t)p.nq << 16));
      for (int j = 0; j < p.nq; ++j) b->key.push_back((uint32_t)p.q[j]);
    }
  }
  hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "hipStreamCreate(batch)");
  // matrices are copied into the programs; keep only the structure afterwards
  qsv_status st = dtype == QSV_C64 ? batch_create_T<float>(b.get(), tile_qubits)
                                   : batch_create_T<double>(b.get(), tile_qubits);
  for (qsv_op& o : b->ops) o.mat = nullptr;
  if (st) {
    batch_release_device(b.get());
    (void)hipStreamDestroy(b->stream);
    return st;
  }
  {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    g_batches.insert(b.get());
  }
  *out = b.release();
  return QSV_OK;
}

static bool batch_live(const qsv_batch* b) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  return b && g_batches.count(b);
}

qsv_status qsv_batch_update(qsv_batch* b, const qsv_op* ops) {
  if (!batch_live(b)) return fail(QSV_ERR_STATE, "invalid or freed batch handle");
  const int nops = b->op_off[b->ncirc];
  if (nops > 0 && !ops) return fail(QSV_ERR_ARG, "ops is NULL");
  for (int ci = 0; ci < b->ncirc; ++ci) {
    qsv_state tmp;
    tmp.n = b->width[ci];
    tmp.dt = b->dt;
    tmp.N = 1ull << b->width[ci];
    for (int i = b->op_off[ci]; i < b->op_off[ci + 1]; ++i) {
      qsv_status st = validate_op(&tmp, ops[i]);
      if (st) return st;
      const POp a = classify(ops[i]);
      uint64_t v = (uint64_t)a.kind | ((uint64_t)a.sign << 4) | ((uint64_t)a.nq << 5);
      for (int j = 0; j < a.nq && j < 6; ++j) v |= (uint64_t)(a.q[j] & 63) << (8 + 6 * j);
      if (v != b->op_sig[i])
        return fail(QSV_ERR_ARG, "op " + std::to_string(i) + " changes the batch structure");
    }
  }
  std::vector<qsv_op> keep = b->ops;
  std::vector<int32_t> keep_prog = b->hprog;
  std::vector<int64_t> keep_off = b->passoff;
  b->ops.assign(ops, ops + nops);
  const size_t npass = b->passoff.size();
  qsv_status st = b->dt == QSV_C64 ? batch_materialise<float>(b, b->tile_bits, true)
                                   : batch_materialise<double>(b, b->tile_bits, true);
  b->ops = keep;
  if (!st && b->passoff.size() != npass)
    st = fail(QSV_ERR_STATE, "the updated programs changed the batch's pass structure");
  if (st) {  // the batch keeps its previous programs
    b->hprog.swap(keep_prog);
    b->passoff.swap(keep_off);
    return st;
  }
  // Angles change which tables and phases are identities, so the programs
  // can outgrow the buffer (a batch built at angle 0 is nearly empty), and
  // new matrices can need the full tile body: then the buffer grows and the
  // launch is captured again.
  bool need_full = false;
  for (int64_t off : b->passoff)
    need_full = need_full || (b->dt == QSV_C64 ? program_needs_full<float>(b->hprog.data() + off)
                                               : program_needs_full<double>(b->hprog.data() + off));
  const bool grow = b->hprog.size() + kProgSlackBytes / 4 > b->prog_cap;
  QSV_HIP(hipStreamSynchronize(b->stream));
  if (grow) {
    QSV_HIP(hipFree(b->d_prog));
    b->d_prog = nullptr;
    b->prog_cap = b->hprog.size() * 2 + 4096;
    hipError_t e = hipMalloc((void**)&b->d_prog, b->prog_cap * 4);
    if (e != hipSuccess) {
      b->d_prog = nullptr;
      b->prog_cap = 0;
      if (b->exec) (void)hipGraphExecDestroy(b->exec);
      if (b->graph) (void)hipGraphDestroy(b->graph);
      b->exec = nullptr;
      b->graph = nullptr;
      return hip_fail(e, "hipMalloc(batch programs)");
    }
  }
  QSV_HIP(hipMemcpyAsync(b->d_prog, b->hprog.data(), b->hprog.size() * 4, hipMemcpyHostToDevice, b->stream));
  QSV_HIP(hipMemcpyAsync(b->d_passoff, b->passoff.data(), npass * 8, hipMemcpyHostToDevice, b->stream));
  QSV_HIP(hipStreamSynchronize(b->stream));
  if (grow || (need_full && !b->full)) {
    qsv_status cs = b->dt == QSV_C64 ? batch_capture<float>(b) : batch_capture<double>(b);
    if (cs) return cs;
  }
  return QSV_OK;
}

qsv_status qsv_batch_run(qsv_batch* b, double* energies) {
  if (!batch_live(b)) return fail(QSV_ERR_STATE, "invalid or freed batch handle");
  if (!b->exec) return fail(QSV_ERR_STATE, "the batch lost its launch in a failed update; create a new batch");
  QSV_HIP(hipGraphLaunch(b->exec, b->stream));
  if (energies)
    QSV_HIP(hipMemcpyAsync(energies, b->d_out, (size_t)b->ncirc * 8, hipMemcpyDeviceToHost,
                           b->stream));
  QSV_HIP(hipStreamSynchronize(b->stream));
  return QSV_OK;
}

qsv_status qsv_batch_info(const qsv_batch* b, int* tile_qubits, int* total_passes,
                          int64_t* scratch_bytes) {
  if (!batch_live(b)) return fail(QSV_ERR_STATE, "invalid or freed batch handle");
  if (tile_qubits) *tile_qubits = b->tile_bits;
  if (total_passes) *total_passes = b->total_passes;
  if (scratch_bytes) *scratch_bytes = (int64_t)(b->scratch_amps * (b->dt == QSV_C64 ? 8 : 16));
  return QSV_OK;
}

qsv_status qsv_batch_free(qsv_batch* b) {
  if (!b) return QSV_OK;
  {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    if (!g_batches.count(b)) return fail(QSV_ERR_STATE, "invalid or freed batch handle");
    g_batches.erase(b);
  }
  (void)hipStreamSynchronize(b->stream);
  batch_release_device(b);
  (void)hipStreamDestroy(b->stream);
  b->magic = 0;
  delete b;
  return QSV_OK;
}

}  // extern "C"

extern "C" {

// Host-only debug export (not in the public header): the environment
// switches (QSV_FORCE_PERGATE, QSV_SEGMENT_QUBITS, QSV_AUTOTUNE_CACHE) are
// read again at their next use, as in a new process: the autotuners' choices
// and the schedule cache are dropped.  For tests that change the environment
// within one process.  Not safe while another thread plans or tunes.
qsv_status qsv_debug_reload_env() {
  g_env_segment.store(-1);
  g_env_pergate.store(-1);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned.clear();
    g_tune_loaded = false;
  }
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_cache.clear();
  }
  return QSV_OK;
}

// Host-only debug export (not in the public header): the program image, pass
// offsets and job table qsv_batch_create would upload for tile width
// tile_qubits, for emulation and checks on the CPU.  Sizes are returned in
// n_words / n_passes; buffers may be NULL for a size query.
qsv_status qsv_debug_batch_program(qsv_dtype dtype, int n_circuits, const int32_t* widths,
                                   const int32_t* op_offsets, const qsv_op* ops,
                                   const int32_t* term_offsets, int tile_qubits, int32_t* words,
                                   int64_t cap_words, int64_t* n_words, int64_t* passoff,
                                   int64_t cap_passes, int64_t* n_passes, int64_t* jobs) {
  if (dtype != QSV_C64 && dtype != QSV_C128) return fail(QSV_ERR_ARG, "bad dtype");
  if (n_circuits < 1) return fail(QSV_ERR_ARG, "no circuits");
  qsv_batch b;
  b.dt = dtype;
  b.ncirc = n_circuits;
  b.width.assign(widths, widths + n_circuits);
  b.op_off.assign(op_offsets, op_offsets + n_circuits + 1);
  b.term_off.assign(term_offsets, term_offsets + n_circuits + 1);
  b.ops.assign(ops, ops + op_offsets[n_circuits]);
  for (int ci = 0; ci < n_circuits; ++ci) {
    qsv_state tmp;
    tmp.n = widths[ci];
    tmp.dt = dtype;
    tmp.N = 1ull << widths[ci];
    for (int i = op_offsets[ci]; i < op_offsets[ci + 1]; ++i) {
      qsv_status st = validate_op(&tmp, ops[i]);
      if (st) return st;
    }
  }
  const int t = tile_qubits > 0 ? tile_qubits : (dtype == QSV_C64 ? 13 : 12);
  qsv_status st = dtype == QSV_C64 ? batch_materialise<float>(&b, t, false)
                                   : batch_materialise<double>(&b, t, false);
  if (st) return st;
  if (n_words) *n_words = (int64_t)b.hprog.size();
  if (n_passes) *n_passes = (int64_t)b.passoff.size();
  for (int64_t i = 0; words && i < cap_words && i < (int64_t)b.hprog.size(); ++i) words[i] = b.hprog[i];
  for (int64_t i = 0; passoff && i < cap_passes && i < (int64_t)b.passoff.size(); ++i)
    passoff[i] = b.passoff[i];
  if (jobs)
    for (size_t i = 0; i < b.job_words.size(); ++i) jobs[i] = b.job_words[i];
  return QSV_OK;
}

}  // extern "C"
