// Device side for gfx950 (CDNA4, wave64): batched unit propagation and the
// bit-sliced exhaustive leaf evaluator.
//
// Unit propagation kernel: one workgroup per cube (persistent: workgroups
// pull cube indices from a counter).  The assignment lives in LDS as two
// bitmaps (variable true / variable false).  Each round every lane scans a
// slice of the query's clauses; a clause with one open literal sets it with
// an atomic OR (a variable set both ways is a conflict); rounds repeat until
// nothing changes.  The fixpoint is unique, so the order does not matter.
// Then the active variables (unassigned and in an unsatisfied clause) get
// slots 0..f-1 in increasing variable order and every unsatisfied clause is
// compiled, in clause order, into a 32-byte record (two uint4):
//   [0].x,y : 64-bit word, OR of the literal patterns of slots 0..5
//   [0].z,w : 64-bit lane mask, the lanes where a literal of slots 6..11
//             is true (the same patterns over the lane id)
//   [1].x   : positive literals of slots 12..37 (26 bits)
//   [1].y   : all literals of slots 12..37 (positive or negative)
//   [1].z   : the residual clause's length |c| (open literals)
//   [1].w   : 2^20 + |c| + 1, the leaf kernel's packed counter increment
//
// Leaf kernel: assignment index a = 4096*block + 64*lane + bit.  Slot j < 6
// is bit j of `bit` (a constant 64-bit pattern), slot 6..11 is bit j-6 of
// the lane id, slot >= 12 is bit j-12 of the block (the same for the whole
// wave).  A wave evaluates one block (64 lanes x 64 bits) per step, reading
// the records with wave-uniform loads: a clause satisfied by a block-level
// literal is skipped with a scalar test (such a literal holds where the block
// bits equal the positive mask: ~(H ^ [1].x) & [1].y != 0); else a lane in the clause's lane
// mask keeps its word and the other lanes AND the clause's pattern word
// in.  A block dies when every lane's word is 0.
// DECIDE takes the smallest (cube, index) witness per query with atomicMin
// and lets later work of that query stop early; COUNT sums popcounts.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <list>
#include <map>
#include <mutex>
#include <string>

#include "common.hpp"
#include "device.hpp"
#include "parallel.hpp"

namespace scuba {

#define HIP_OK(x)                                                                       \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess) fail(SCUBA_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace {

constexpr int kBlock = 256;          // threads per workgroup (4 waves)
// A record's packed counter: clauses in bits 20..31, |c| + 1 summed in bits
// 0..19.  Within 4096 records neither field overflows (|c| <= 38).
constexpr uint32_t kRecCount = 1u << 20;
constexpr uint32_t kRecRun = 4096;
// leaf_kernel: blocks evaluated together per pass over a leaf's records
constexpr uint32_t kPass = 8;
constexpr uint32_t kHighMask = (1u << 26) - 1;

__device__ __forceinline__ uint64_t slot_pattern(uint32_t j) {
  switch (j) {
    case 0: return 0xAAAAAAAAAAAAAAAAull;
    case 1: return 0xCCCCCCCCCCCCCCCCull;
    case 2: return 0xF0F0F0F0F0F0F0F0ull;
    case 3: return 0xFF00FF00FF00FF00ull;
    case 4: return 0xFFFF0000FFFF0000ull;
    default: return 0xFFFFFFFF00000000ull;
  }
}

// wave-uniform copy of a 32-bit value (the builtin returns a signed int:
// widen through uint32_t so that 64-bit values are zero-extended)
__device__ __forceinline__ uint32_t uniform_u32(uint32_t x) {
  return uint32_t(__builtin_amdgcn_readfirstlane(int(x)));
}
__device__ __forceinline__ uint64_t uniform_u64(uint64_t x) {
  return (uint64_t(uniform_u32(uint32_t(x >> 32))) << 32) | uniform_u32(uint32_t(x));
}

// Clause access for the propagation kernel: the query's CNF either read
// from global memory (DIMACS literals, 32-bit offsets) or staged in LDS as
// 16-bit literals (variable << 1 | negated) with 16-bit offsets.
struct GlobalCnf {
  const uint32_t* co;
  const int32_t* L;
  __device__ __forceinline__ uint32_t beg(uint32_t c) const { return co[c]; }
  __device__ __forceinline__ uint32_t end(uint32_t c) const { return co[c + 1]; }
  __device__ __forceinline__ void lit(uint32_t i, uint32_t* v, bool* neg) const {
    const int32_t l = L[i];
    *v = uint32_t(l > 0 ? l : -l);
    *neg = l < 0;
  }
};
struct LdsCnf {
  const uint16_t* co;
  const uint16_t* L;
  __device__ __forceinline__ uint32_t beg(uint32_t c) const { return co[c]; }
  __device__ __forceinline__ uint32_t end(uint32_t c) const { return co[c + 1]; }
  __device__ __forceinline__ void lit(uint32_t i, uint32_t* v, bool* neg) const {
    const uint32_t x = L[i];
    *v = x >> 1;
    *neg = x & 1;
  }
};

template <class Cnf>
__device__ __forceinline__ bool clause_satisfied(const Cnf& cnf, uint32_t c, const uint32_t* T, const uint32_t* F) {
  for (uint32_t i = cnf.beg(c), e = cnf.end(c); i < e; i++) {
    uint32_t v;
    bool neg;
    cnf.lit(i, &v, &neg);
    if ((neg ? F[v >> 5] : T[v >> 5]) & (1u << (v & 31))) return true;
  }
  return false;
}

// Per-team state of the propagation kernel (one cube per team).
struct UpShared {
  uint32_t conflict, error;
  // frontier length, overflow and "something newly set" of round r in set
  // r % 3: a set is read in the round after it is written and cleared in
  // the round after that, so one barrier per round separates all three
  uint32_t qn[3], ovf[3], chg[3];
  uint32_t scan[2][16];            // per wave (teams of up to 16), alternating: one barrier per scan
};

constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint32_t kStageUnroll = 8;   // CNF staging: loads in flight per thread
static_assert(kUpWaves == kBlock / 64, "a workgroup holds kUpWaves waves");

// Makes LDS writes of the wave visible to all its lanes, and keeps the
// compiler from moving LDS accesses across it.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// exclusive scan of one value per lane over the wave: inclusive scans of
// the four 16-lane rows by DPP row shifts, then the row totals (read into
// scalar registers) added to the rows above them
__device__ __forceinline__ uint32_t wave_exclusive_scan(uint32_t v, uint32_t* total) {
  const uint32_t lane = threadIdx.x & 63;
  int x = int(v);
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);   // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);   // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);   // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);   // row_shr:8
  const uint32_t r0 = uint32_t(__builtin_amdgcn_readlane(x, 15)), r1 = uint32_t(__builtin_amdgcn_readlane(x, 31)),
                 r2 = uint32_t(__builtin_amdgcn_readlane(x, 47)), r3 = uint32_t(__builtin_amdgcn_readlane(x, 63));
  const uint32_t row = lane >> 4;
  uint32_t y = uint32_t(x);
  if (row >= 1) y += r0;
  if (row >= 2) y += r1;
  if (row >= 3) y += r2;
  *total = r0 + r1 + r2 + r3;
  return y - v;
}

// inclusive maximum over the lanes 0..lane (values below 2^31), by the same
// DPP row shifts and row totals as the scan above
__device__ __forceinline__ uint32_t wave_inclusive_max(uint32_t v) {
  const uint32_t lane = threadIdx.x & 63;
  int x = int(v);
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false));   // row_shr:1
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false));   // row_shr:2
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false));   // row_shr:4
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false));   // row_shr:8
  const int r0 = __builtin_amdgcn_readlane(x, 15), r1 = __builtin_amdgcn_readlane(x, 31),
            r2 = __builtin_amdgcn_readlane(x, 47);
  const uint32_t row = lane >> 4;
  if (row >= 1) x = max(x, r0);
  if (row >= 2) x = max(x, r1);
  if (row >= 3) x = max(x, r2);
  return uint32_t(x);
}

// The threads that propagate one cube: one wave (TW = 1, four cubes per
// workgroup) or the whole workgroup (TW = 4, for rounds with few cubes).
template <int TW>
struct Team {
  static constexpr uint32_t kSize = 64 * TW;
  static constexpr uint32_t kQueue = kUpQueue * TW;   // frontier entries per buffer
  UpShared& sh;
  uint32_t par = 0;   // scan buffer of the next scan (every thread keeps its own copy)
  __device__ __forceinline__ uint32_t lane() const { return TW == 1 ? (threadIdx.x & 63) : threadIdx.x; }
  __device__ __forceinline__ void sync() const {
    if (TW == 1) wave_sync();
    else __syncthreads();
  }
  // exclusive scan of one value per thread over the team
  __device__ __forceinline__ uint32_t scan(uint32_t v, uint32_t* total) {
    if (TW == 1) return wave_exclusive_scan(v, total);
    const uint32_t l = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t wtot;
    const uint32_t x = wave_exclusive_scan(v, &wtot) + v;   // inclusive within the wave
    // consecutive scans alternate buffers: a thread writing scan i+1 has
    // passed scan i's barrier, and every thread reads scan i-1's buffer
    // before it reaches that barrier, so one barrier per scan suffices
    if (l == 63) sh.scan[par][wv] = wtot;
    __syncthreads();
    uint32_t base = 0, tot = 0;
    for (uint32_t w = 0; w < uint32_t(TW); w++) {
      if (w < wv) base += sh.scan[par][w];
      tot += sh.scan[par][w];
    }
    par ^= 1;
    *total = tot;
    return base + x - v;
  }
};

// Per-literal occurrence lists (literal index 2*v + negative -> clauses),
// in HBM (32-bit) or staged in LDS (16-bit).
struct GlobalOcc {
  const uint32_t* off;
  const uint32_t* occ;
  __device__ __forceinline__ uint32_t beg(uint32_t li) const { return off[li]; }
  __device__ __forceinline__ uint32_t end(uint32_t li) const { return off[li + 1]; }
  __device__ __forceinline__ uint32_t at(uint32_t k) const { return occ[k]; }
};
struct LdsOcc {
  const uint16_t* off;
  const uint16_t* occ;
  __device__ __forceinline__ uint32_t beg(uint32_t li) const { return off[li]; }
  __device__ __forceinline__ uint32_t end(uint32_t li) const { return off[li + 1]; }
  __device__ __forceinline__ uint32_t at(uint32_t k) const { return occ[k]; }
};

// One clause against the current assignment: a conflict is flagged; a unit
// literal is set, and when it is new its entry (variable << 1 | value) is
// returned (kNone otherwise).
template <class Cnf>
__device__ __forceinline__ uint32_t visit_clause(const Cnf& cnf, uint32_t c, uint32_t* T, uint32_t* F,
                                                 uint32_t w, UpShared& sh) {
  bool sat = false;
  uint32_t open = 0, last_v = 0;
  bool last_neg = false;
  const uint32_t b = cnf.beg(c), e = cnf.end(c);
  if (e - b <= 4) {
    // short clauses (the gate clauses): the literals, then their
    // assignment words, are loaded independently of each other
    uint32_t v[4], t[4], f[4];
    bool neg[4];
#pragma unroll
    for (uint32_t u = 0; u < 4; u++) {
      v[u] = 0;
      neg[u] = false;
      if (b + u < e) cnf.lit(b + u, &v[u], &neg[u]);
    }
#pragma unroll
    for (uint32_t u = 0; u < 4; u++) {
      t[u] = b + u < e ? T[v[u] >> 5] : 0u;
      f[u] = b + u < e ? F[v[u] >> 5] : 0u;
    }
#pragma unroll
    for (uint32_t u = 0; u < 4; u++) {
      if (b + u >= e) break;
      const uint32_t bit = 1u << (v[u] & 31);
      const uint32_t tu = t[u] & bit, fu = f[u] & bit;
      if (neg[u] ? fu : tu) sat = true;
      if (!(tu | fu)) { open++; last_v = v[u]; last_neg = neg[u]; }
    }
  } else {
    for (uint32_t i = b; i < e; i++) {
      uint32_t v;
      bool neg;
      cnf.lit(i, &v, &neg);
      const uint32_t bit = 1u << (v & 31);
      const uint32_t t = T[v >> 5] & bit, f = F[v >> 5] & bit;
      if (neg ? f : t) { sat = true; break; }
      if (!(t | f)) { open++; last_v = v; last_neg = neg; }
    }
  }
  if (sat) return kNone;
  if (open == 0) {
    sh.conflict = 1;
  } else if (open == 1) {
    const uint32_t bit = 1u << (last_v & 31);
    const uint32_t old = atomicOr(last_neg ? &F[last_v >> 5] : &T[last_v >> 5], bit);
    if (!(old & bit)) {
      sh.chg[w] = 1;
      return (last_v << 1) | (last_neg ? 0u : 1u);
    }
  }
  return kNone;
}

// Queue a new assignment for the next round (an overflow makes that round
// scan every clause).
// The active lanes of a wave that have an entry take consecutive slots with
// one atomic per wave (ranked by the ballot of the lanes that push).
__device__ __forceinline__ void push(uint32_t e, uint32_t* next, uint32_t cap, uint32_t w, UpShared& sh) {
  const uint64_t m = __ballot(e != kNone);
  if (!m) return;
  const uint32_t leader = uint32_t(__builtin_ctzll(m));
  uint32_t base = 0;
  if ((threadIdx.x & 63) == leader) base = atomicAdd(&sh.qn[w], uint32_t(__popcll(m)));
  base = uint32_t(__builtin_amdgcn_readlane(int(base), int(leader)));
  if (e == kNone) return;
  const uint32_t rank = __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
  const uint32_t slot = base + rank;
  if (slot < cap) next[slot] = e;
  else sh.ovf[w] = 1;
}

// Pieces of the unit propagation of one cube by one team.  Every thread of
// the team calls each of them (uniform control flow within the team).  The
// assignment is two LDS bitmaps, T (variable true) and F (variable false),
// over variables 0..nv; A marks the active variables (unassigned, in an
// unsatisfied clause) and P holds, per bitmap word, the slot of its first
// active variable.

// Clears the bitmaps, the owner marks and the counters.
template <int TW>
__device__ __forceinline__ void up_clear(Team<TW>& tm, uint32_t nw, uint32_t* T, uint32_t* F, uint32_t* A,
                                         uint32_t* X, UpShared& sh) {
  constexpr uint32_t S = Team<TW>::kSize;
  const uint32_t lane = tm.lane();
  for (uint32_t w = lane; w < nw; w += S) { T[w] = 0; F[w] = 0; A[w] = 0; }
  for (uint32_t t = lane; t < S; t += S) X[2 * (t & ~63u) + 64 + (t & 63)] = 0;   // the owner marks
  if (lane == 0) {
    sh.conflict = 0;
    sh.error = 0;
    for (uint32_t k = 0; k < 3; k++) { sh.qn[k] = 0; sh.ovf[k] = 0; sh.chg[k] = 0; }
  }
}

// The first frontier: every literal that holds before propagation, as if a
// round -1 had set it (queue 1, counter set 2).  From a literal list (a
// cube's literals, or one decision on top of a fixpoint):
template <int TW>
__device__ __forceinline__ void up_seed_lits(Team<TW>& tm, const int32_t* __restrict__ lits, uint32_t n_lits,
                                             uint32_t nv, uint32_t* T, uint32_t* F, uint32_t* Q, UpShared& sh) {
  constexpr uint32_t S = Team<TW>::kSize, QC = Team<TW>::kQueue;
  const uint32_t lane = tm.lane();
  uint32_t* seed = Q + QC;
  for (uint32_t j = lane; j < n_lits; j += S) {
    const int32_t l = lits[j];
    const uint32_t v = uint32_t(l > 0 ? l : -l);
    if (v == 0 || v > nv) { sh.error = 1; continue; }
    const uint32_t bit = 1u << (v & 31);
    const uint32_t old = atomicOr(l > 0 ? &T[v >> 5] : &F[v >> 5], bit);
    if (!(old & bit)) push((v << 1) | (l > 0 ? 1u : 0u), seed, QC, 2, sh);
  }
}
// ... and from the unit clauses of the CNF (an empty clause is a conflict).
template <int TW, class Cnf>
__device__ __forceinline__ void up_seed_units(Team<TW>& tm, const Cnf& cnf, uint32_t nc, uint32_t* T, uint32_t* F,
                                              uint32_t* Q, UpShared& sh) {
  constexpr uint32_t S = Team<TW>::kSize, QC = Team<TW>::kQueue;
  const uint32_t lane = tm.lane();
  uint32_t* seed = Q + QC;
  for (uint32_t c = lane; c < nc; c += S) {
    const uint32_t b = cnf.beg(c), e = cnf.end(c);
    if (e == b) { sh.conflict = 1; continue; }
    if (e - b != 1) continue;
    uint32_t v;
    bool neg;
    cnf.lit(b, &v, &neg);
    const uint32_t bit = 1u << (v & 31);
    const uint32_t old = atomicOr(neg ? &F[v >> 5] : &T[v >> 5], bit);
    if (!(old & bit)) push((v << 1) | (neg ? 0u : 1u), seed, QC, 2, sh);
  }
}

// Propagation rounds from the first frontier to the fixpoint, then the
// conflict test over the bitmaps (sh.conflict / sh.error on return).
// Round r visits the clauses of the literals that round r-1 made false (its
// frontier); when that frontier overflowed its queue, round r scans every
// clause instead.  A round that sets nothing new ends at the fixpoint:
// every clause has been visited after its last false literal was assigned.
// Every changing round sets a new bit, so at most 2*(nv+1) rounds change
// something.  Each wave takes every TW-th frontier entry and spreads the
// (entry, occurrence) pairs of up to 64 entries at a time over its lanes: a
// wave scan of the occurrence counts gives each entry's first pair, and a
// lane finds the entry of its pair: among up to four entries by comparisons
// with their offsets held in scalar registers, else from marks that each
// entry writes at its first pair of a 64-pair chunk (Xw[64..127] in LDS)
// and a wave max-scan over them.  The only team-wide barrier of a round is
// at its end.
template <int TW, class Cnf, class Occ>
__device__ __forceinline__ void up_rounds(Team<TW>& tm, const Cnf& cnf, const Occ& occ, uint32_t nv, uint32_t nc,
                                          uint32_t* T, uint32_t* F, uint32_t* Q, uint32_t* X, UpShared& sh) {
  constexpr uint32_t S = Team<TW>::kSize, QC = Team<TW>::kQueue;
  const uint32_t lane = tm.lane();
  const uint32_t nw = (nv >> 5) + 1;
  const uint32_t wl = threadIdx.x & 63, wv = TW == 1 ? 0u : uniform_u32(lane >> 6);
  uint32_t* Xw = X + wv * 128;
  uint32_t mark_tag = 0;   // tags of the owner marks; 0 (the cleared marks) never matches
  const uint32_t occ_total = occ.end(2 * nv + 1);
  const uint32_t max_rounds = 2 * nv + 4;
  for (uint32_t r = 0;; r++) {
    const uint32_t k = r % 3, kp = (r + 2) % 3, kn = (r + 1) % 3;
    const uint32_t* cur = Q + ((r + 1) & 1) * QC;
    uint32_t* next = Q + (r & 1) * QC;
    if (lane == 0) { sh.qn[kn] = 0; sh.ovf[kn] = 0; sh.chg[kn] = 0; }
    // both counters of the previous round are read at once
    const uint32_t ovf_p = uniform_u32(sh.ovf[kp]), qn_p = uniform_u32(sh.qn[kp]);
    if (ovf_p) {
      for (uint32_t c = lane; c < nc; c += S) push(visit_clause(cnf, c, T, F, k, sh), next, QC, k, sh);
    } else {
      const uint32_t n = min(qn_p, QC);
      for (uint32_t base = 0; wv + TW * base < n; base += 64) {
        const uint32_t j = wv + TW * (base + wl);
        uint32_t cnt = 0, start = 0;
        if (j < n) {
          const uint32_t e = cur[j];
          const uint32_t v = e >> 1, val = e & 1;
          const uint32_t bit = 1u << (v & 31);
          // the literal of v that is now false is the negative one iff v = 1;
          // its list bounds are loaded alongside the conflict test
          const uint32_t li = 2 * v + val;
          const uint32_t b = occ.beg(li), en = occ.end(li);
          if (T[v >> 5] & F[v >> 5] & bit) {
            sh.conflict = 1;
          } else {
            start = b;
            cnt = en - b;
          }
        }
        uint32_t total;
        const uint32_t off = wave_exclusive_scan(cnt, &total);
        // pair q of an entry reads occurrence q + (start - off) of its list
        const uint32_t d = start - off;
        const uint32_t m = min(64u, (n - (wv + TW * base) + TW - 1) / TW);   // lanes with an entry
        if (m <= 4) {
          // few entries: a pair's entry is the last one whose offset is at
          // or below it, among the offsets of lanes 0..3 read into scalar
          // registers (no LDS round trip; a lane without an entry has
          // offset = total, above every pair)
          const uint32_t d0 = uint32_t(__builtin_amdgcn_readlane(int(d), 0)),
                         d1 = uint32_t(__builtin_amdgcn_readlane(int(d), 1)),
                         d2 = uint32_t(__builtin_amdgcn_readlane(int(d), 2)),
                         d3 = uint32_t(__builtin_amdgcn_readlane(int(d), 3)),
                         o1 = uint32_t(__builtin_amdgcn_readlane(int(off), 1)),
                         o2 = uint32_t(__builtin_amdgcn_readlane(int(off), 2)),
                         o3 = uint32_t(__builtin_amdgcn_readlane(int(off), 3));
          for (uint32_t q = wl; q < total; q += 64) {
            const uint32_t p = q + (q >= o3 ? d3 : q >= o2 ? d2 : q >= o1 ? d1 : d0);
            push(visit_clause(cnf, occ.at(p), T, F, k, sh), next, QC, k, sh);
          }
          continue;
        }
        Xw[wl] = d;
        uint32_t carry = 0;   // owner (lane + 1) of the previous chunk's last pair
        for (uint32_t q0 = 0; q0 < total; q0 += 64) {
          // each entry marks the position of its first pair in this chunk;
          // a lane's owner is the last mark at or before it (a max-scan of
          // the tagged marks), else the previous chunk's last owner
          const uint32_t tag = ++mark_tag % 0xFFFFFFu + 1;   // 1 .. 2^24 - 1
          if (cnt && off >= q0 && off - q0 < 64) Xw[64 + (off - q0)] = (tag << 8) | (wl + 1);
          wave_sync();
          const uint32_t mk = Xw[64 + wl];
          const uint32_t own = max(wave_inclusive_max((mk >> 8) == tag ? (mk & 0xFFu) : 0u), carry);
          carry = uint32_t(__builtin_amdgcn_readlane(int(own), 63));
          const uint32_t q = q0 + wl;
          uint32_t e = kNone;
          if (q < total && own != 0) {
            const uint32_t oi = q + Xw[own - 1];
            if (oi < occ_total) e = visit_clause(cnf, occ.at(oi), T, F, k, sh);
          }
          push(e, next, QC, k, sh);
          wave_sync();   // the marks are rewritten by the next chunk
        }
        wave_sync();   // Xw is rewritten by the next entries
      }
    }
    tm.sync();
    const uint32_t changed = uniform_u32(sh.chg[k]), conflict = uniform_u32(sh.conflict);
    if (conflict || !changed) break;
    if (r >= max_rounds) {   // cannot happen: every changing round sets a new bit
      if (lane == 0) sh.error = 1;
      break;
    }
  }
  tm.sync();
  for (uint32_t w = lane; w < nw; w += S)
    if (T[w] & F[w]) sh.conflict = 1;
  tm.sync();
}

// Active variables into A, over contiguous clauses per lane.  A lane with
// at most 64 clauses keeps which of them are unsatisfied, in a register
// mask that also serves the residual records.
struct ActiveScan {
  uint32_t c0, c1, my_unsat;
  bool keep;
  uint64_t unsat;
};
template <int TW, class Cnf>
__device__ __forceinline__ ActiveScan up_active(Team<TW>& tm, const Cnf& cnf, uint32_t nc, const uint32_t* T,
                                                const uint32_t* F, uint32_t* A) {
  constexpr uint32_t S = Team<TW>::kSize;
  const uint32_t lane = tm.lane();
  ActiveScan as;
  const uint32_t cpl = (nc + S - 1) / S;
  as.c0 = min(nc, lane * cpl);
  as.c1 = min(nc, as.c0 + cpl);
  as.keep = cpl <= 64;
  as.unsat = 0;
  as.my_unsat = 0;
  for (uint32_t c = as.c0; c < as.c1; c++) {
    if (clause_satisfied(cnf, c, T, F)) continue;
    as.my_unsat++;
    if (as.keep) as.unsat |= uint64_t(1) << (c - as.c0);
    for (uint32_t i = cnf.beg(c), e = cnf.end(c); i < e; i++) {
      uint32_t v;
      bool neg;
      cnf.lit(i, &v, &neg);
      const uint32_t bit = 1u << (v & 31);
      if (!((T[v >> 5] | F[v >> 5]) & bit)) atomicOr(&A[v >> 5], bit);
    }
  }
  return as;
}

// The bits of bitmap word w that are variables 1..nv.
__device__ __forceinline__ uint32_t var_mask(uint32_t w, uint32_t nv) {
  uint32_t valid = 0xFFFFFFFFu;
  if (w == 0) valid &= ~1u;   // no variable 0
  if (w == (nv >> 5)) valid &= (nv & 31) == 31 ? 0xFFFFFFFFu : ((2u << (nv & 31)) - 1);
  return valid;
}

// Slot prefix per bitmap word (contiguous words per lane) into P, and the
// team totals of active (f) and unassigned variables.  A must be complete
// (a team barrier after up_active).
template <int TW>
__device__ __forceinline__ void up_prefix(Team<TW>& tm, uint32_t nv, const uint32_t* T, const uint32_t* F,
                                          const uint32_t* A, uint32_t* P, uint32_t* f_total, uint32_t* free_total) {
  constexpr uint32_t S = Team<TW>::kSize;
  const uint32_t lane = tm.lane();
  const uint32_t nw = (nv >> 5) + 1;
  const uint32_t wpl = (nw + S - 1) / S;
  const uint32_t w0 = min(nw, lane * wpl), w1 = min(nw, w0 + wpl);
  uint32_t my_act = 0, my_free = 0;
  for (uint32_t w = w0; w < w1; w++) {
    my_act += __popc(A[w]);
    my_free += __popc(~(T[w] | F[w]) & var_mask(w, nv));
  }
  uint32_t base = tm.scan(my_act, f_total);
  tm.scan(my_free, free_total);
  for (uint32_t w = w0; w < w1; w++) { P[w] = base; base += __popc(A[w]); }
}

// The residual record of unsatisfied clause c (slots from A and P) at
// record index rec.  Its last word is the leaf kernel's counter increment
// for one evaluated clause: kRecCount (one clause) plus |c| + 1 (its word
// operations per 64-bit word).
template <class Cnf>
__device__ __forceinline__ void up_record(const Cnf& cnf, uint32_t c, const uint32_t* T, const uint32_t* F,
                                          const uint32_t* A, const uint32_t* P, uint4* __restrict__ res,
                                          uint64_t rec) {
  uint64_t low = 0, lm = 0;
  uint32_t hp = 0, hn = 0, len = 0;
  for (uint32_t i = cnf.beg(c), e = cnf.end(c); i < e; i++) {
    uint32_t v;
    bool neg;
    cnf.lit(i, &v, &neg);
    const uint32_t bit = 1u << (v & 31);
    if ((T[v >> 5] | F[v >> 5]) & bit) continue;     // false literal
    len++;
    const uint32_t slot = P[v >> 5] + __popc(A[v >> 5] & (bit - 1));
    if (slot < 6) low |= neg ? ~slot_pattern(slot) : slot_pattern(slot);
    else if (slot < 12) lm |= neg ? ~slot_pattern(slot - 6) : slot_pattern(slot - 6);
    else (neg ? hn : hp) |= 1u << (slot - 12);
  }
  res[2 * rec] = make_uint4(uint32_t(low), uint32_t(low >> 32), uint32_t(lm), uint32_t(lm >> 32));
  res[2 * rec + 1] = make_uint4(hp, hp | hn, len, kRecCount | (len + 1));
}

// The residual records of the lane's unsatisfied clauses, in clause order,
// at records res_base + pos.. (pos: the team scan of my_unsat).  P must be
// complete (a team barrier after up_prefix).
template <class Cnf>
__device__ __forceinline__ void up_records(const Cnf& cnf, const ActiveScan& as, const uint32_t* T,
                                           const uint32_t* F, const uint32_t* A, const uint32_t* P,
                                           uint4* __restrict__ res, uint64_t res_base, uint32_t pos) {
  for (uint32_t c = as.c0; c < as.c1; c++) {
    if (as.keep ? !((as.unsat >> (c - as.c0)) & 1) : clause_satisfied(cnf, c, T, F)) continue;
    up_record(cnf, c, T, F, A, P, res, res_base + pos);
    pos++;
  }
}

// A host fixpoint in one pass over the clauses in HBM.  The pass confirms
// that no clause is unit or empty under the assignment, marks the active
// variables in A and lists the unsatisfied clauses.  Wave wv of the team
// takes the clauses [c0, c1) of fix_range, 64 at a time with lane j on
// clause base + j, so consecutive lanes read consecutive clause offsets and
// literals, fix_unroll chunks at a time (the first four literals of a
// clause with the chunk, longer clauses' rest when evaluated).  The wave's unsatisfied clauses go to list[]
// in clause order (ballot ranks), the first cap of them.  Returns the
// wave's count of unsatisfied clauses; *bad is set (wave-uniform) when a
// clause is unit or empty, so the assignment is not a fixpoint.
// Chunks per group: two for the eight-wave teams, whose registers then
// fit three workgroups per CU (more teams in flight per CU beat deeper
// pipelines per wave there), three for the others.
template <int TW>
constexpr uint32_t fix_unroll() { return TW == 8 ? 2 : 3; }
constexpr uint32_t kFixList = 512;   // listed unsatisfied clauses per wave
constexpr uint64_t kFixWideClauses = 16384;

// Element i of a 32-bit array whose indexes stay below 2^30: the byte
// offset is a 32-bit value, so a uniform base takes the scalar-base form of
// the load.
template <class T>
__device__ __forceinline__ T ld32(const T* base, uint32_t i) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (i << 2));
}

template <int TW>
__device__ __forceinline__ void fix_range(uint32_t nc, uint32_t wv, uint32_t* c0, uint32_t* c1) {
  const uint32_t per = ((nc + TW - 1) / TW + 63) & ~63u;
  *c0 = min(nc, wv * per);
  *c1 = min(nc, *c0 + per);
}

__device__ __forceinline__ void fix_lit(int32_t l, const uint32_t* T, const uint32_t* F, bool* sat, uint32_t* open) {
  const uint32_t v = uint32_t(l > 0 ? l : -l), bit = 1u << (v & 31);
  const uint32_t t = T[v >> 5], f = F[v >> 5];
  if (((l > 0) ? t : f) & bit) *sat = true;
  else if (!((t | f) & bit)) (*open)++;
}
__device__ __forceinline__ void fix_mark(int32_t l, const uint32_t* T, const uint32_t* F, uint32_t* A) {
  const uint32_t v = uint32_t(l > 0 ? l : -l), bit = 1u << (v & 31);
  if (!((T[v >> 5] | F[v >> 5]) & bit)) atomicOr(&A[v >> 5], bit);
}

template <int TW, bool kTF = false>
__device__ __forceinline__ uint32_t fix_scan(const GlobalCnf& cnf, uint32_t nc, uint32_t wv, const uint32_t* T,
                                             const uint32_t* F, uint32_t* A, uint32_t* list, uint32_t cap,
                                             uint32_t* bad, const uint2* TF = nullptr) {
  constexpr uint32_t kFixUnroll = fix_unroll<TW>();
  constexpr uint32_t G = 64 * kFixUnroll;   // clauses per group
  const uint32_t wl = threadIdx.x & 63;
  uint32_t c0, c1;
  fix_range<TW>(nc, wv, &c0, &c1);
  uint32_t n = 0;
  bool wrong = false;
  // Software pipeline over groups of kFixUnroll chunks: while group g is
  // evaluated, the literals of group g + 1 and the clause starts of group
  // g + 2 are in flight.  A clause's end is the next lane's start, the
  // next chunk's first start, or the group's end offset (one uniform
  // load); a lane past the range gets an empty clause.  Literals come four
  // at a time in one 16-byte load from the clause's start (what lies past
  // a shorter clause is read, within the CNF's regions, and ignored).
  auto starts = [&](uint32_t base, uint32_t* bb, uint32_t* last) {
#pragma unroll
    for (uint32_t u = 0; u < kFixUnroll; u++) {
      const uint32_t c = base + 64 * u + wl;
      bb[u] = c < c1 ? ld32(cnf.co, c) : 0u;
    }
    *last = base < c1 ? ld32(cnf.co, min(base + G, c1)) : 0u;
  };
  auto ends = [&](uint32_t base, const uint32_t* bb, uint32_t last, uint32_t* ee) {
#pragma unroll
    for (uint32_t u = 0; u < kFixUnroll; u++) {
      const uint32_t nx = u + 1 < kFixUnroll ? uint32_t(__builtin_amdgcn_readlane(int(bb[u + 1]), 0)) : last;
      const uint32_t dn = uint32_t(__shfl_down(int(bb[u]), 1));
      const uint32_t c = base + 64 * u + wl;
      ee[u] = c >= c1 ? 0u : c + 1 == c1 ? last : (wl < 63 ? dn : nx);
    }
  };
  auto lits = [&](const uint32_t* bb, const uint32_t* ee, int4* xx) {
#pragma unroll
    for (uint32_t u = 0; u < kFixUnroll; u++) {
      xx[u] = make_int4(0, 0, 0, 0);
      if (bb[u] < ee[u]) __builtin_memcpy(&xx[u], reinterpret_cast<const char*>(cnf.L) + (bb[u] << 2), 16);
    }
  };
  uint32_t b[kFixUnroll], e[kFixUnroll], nb[kFixUnroll], last, nlast;
  int4 x[kFixUnroll];
  starts(c0, b, &last);
  ends(c0, b, last, e);
  lits(b, e, x);
  starts(c0 + G, nb, &nlast);
  for (uint32_t base = c0; base < c1; base += G) {
    uint32_t ne[kFixUnroll], bb[kFixUnroll], blast;
    int4 nx[kFixUnroll];
    ends(base + G, nb, nlast, ne);
    lits(nb, ne, nx);                  // group g + 1
    starts(base + 2 * G, bb, &blast);  // group g + 2
#pragma unroll
    for (uint32_t u = 0; u < kFixUnroll; u++) {
      const uint32_t c = base + 64 * u + wl;
      const int32_t xs[4] = {x[u].x, x[u].y, x[u].z, x[u].w};
      // branch-free over the four loaded literals: one past the clause's end
      // reads variable 0 (never assigned) and is masked out; the bitmap
      // words of all four are read before any is used (one 64-bit read
      // each from the interleaved copy, when there is one)
      uint32_t bit4[4], t4[4], f4[4];
      bool ok4[4], pos4[4];
#pragma unroll
      for (uint32_t j = 0; j < 4; j++) {
        ok4[j] = b[u] + j < e[u];
        const int32_t l = ok4[j] ? xs[j] : 0;
        const uint32_t v = uint32_t(l > 0 ? l : -l);
        pos4[j] = l > 0;
        bit4[j] = 1u << (v & 31);
        if (kTF) {
          const uint2 tf = TF[v >> 5];
          t4[j] = tf.x;
          f4[j] = tf.y;
        } else {
          t4[j] = T[v >> 5];
          f4[j] = F[v >> 5];
        }
      }
      bool sat = false;
      uint32_t open = 0;
#pragma unroll
      for (uint32_t j = 0; j < 4; j++) {
        sat |= ok4[j] && ((pos4[j] ? t4[j] : f4[j]) & bit4[j]) != 0;
        open += (ok4[j] && !((t4[j] | f4[j]) & bit4[j])) ? 1u : 0u;
      }
      for (uint32_t i = b[u] + 4; i < e[u]; i++) fix_lit(ld32(cnf.L, i), T, F, &sat, &open);
      const bool unsat = c < c1 && !sat;
      if (unsat) {
        wrong |= open < 2;
#pragma unroll
        for (uint32_t j = 0; j < 4; j++)
          if (b[u] + j < e[u]) fix_mark(xs[j], T, F, A);
        for (uint32_t i = b[u] + 4; i < e[u]; i++) fix_mark(ld32(cnf.L, i), T, F, A);
      }
      const uint64_t m = __ballot(unsat);
      if (unsat) {
        const uint32_t r = n + __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
        if (r < cap) list[r] = c;
      }
      n += uint32_t(__popcll(m));
    }
#pragma unroll
    for (uint32_t u = 0; u < kFixUnroll; u++) {
      b[u] = nb[u];
      e[u] = ne[u];
      x[u] = nx[u];
      nb[u] = bb[u];
    }
    nlast = blast;
  }
  *bad = __ballot(wrong) != 0;
  return n;
}

// Records of the wave's unsatisfied clauses at res_base + pos.., in clause
// order: from the wave's list when it holds them all, else by a second pass
// over the wave's clauses.
template <int TW>
__device__ __forceinline__ void fix_records(const GlobalCnf& cnf, uint32_t nc, uint32_t wv, uint32_t n,
                                            const uint32_t* list, uint32_t cap, const uint32_t* T,
                                            const uint32_t* F, const uint32_t* A, const uint32_t* P,
                                            uint4* __restrict__ res, uint64_t res_base, uint32_t pos) {
  const uint32_t wl = threadIdx.x & 63;
  if (n <= cap) {
    for (uint32_t i = wl; i < n; i += 64) up_record(cnf, list[i], T, F, A, P, res, res_base + pos + i);
    return;
  }
  uint32_t c0, c1;
  fix_range<TW>(nc, wv, &c0, &c1);
  for (uint32_t base = c0; base < c1; base += 64) {
    const uint32_t c = base + wl;
    const bool unsat = c < c1 && !clause_satisfied(cnf, c, T, F);
    const uint64_t m = __ballot(unsat);
    if (unsat)
      up_record(cnf, c, T, F, A, P, res,
                res_base + pos + __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u)));
    pos += uint32_t(__popcll(m));
  }
}

// A cube that carries the host's fixpoint, from the CNF in HBM: the
// bitmaps from the cube's record, one pass (fix_scan), then slots and
// records.  The host's fixpoint is the unit-propagation fixpoint of the
// same clauses, so a clause that is unit or empty under it (or a variable
// set both ways) means the two sides disagree: the cube's status is 2, an
// error the host reports.
template <int TW>
__device__ void fix_cube(Team<TW>& tm, const GlobalCnf& cnf, const DevCubeDesc& cd, uint32_t ci, uint32_t nv,
                         uint32_t nc, const int32_t* __restrict__ cube_lits, DevCubeOut* __restrict__ out,
                         uint4* __restrict__ res, uint32_t* T, uint32_t* F, uint32_t* A, uint32_t* P,
                         uint2* TF, uint32_t* lists) {
  constexpr uint32_t S = Team<TW>::kSize;
  const uint32_t lane = tm.lane(), wv = TW == 1 ? 0u : uniform_u32(lane >> 6);
  const uint32_t nw = (nv >> 5) + 1;
  const uint32_t* fw = reinterpret_cast<const uint32_t*>(cube_lits + cd.lit_off);
  uint32_t clash = 0;
  for (uint32_t w = lane; w < nw; w += S) {
    const uint32_t t = fw[w], f = fw[nw + w];
    T[w] = t;
    F[w] = f;
    TF[w] = make_uint2(t, f);
    A[w] = 0;
    clash |= t & f;
  }
  tm.sync();
  uint32_t* list = lists + wv * kFixList;
  uint32_t bad;
  const uint32_t n = fix_scan<TW, true>(cnf, nc, wv, T, F, A, list, kFixList, &bad, TF);
  bad |= __ballot(clash != 0) != 0;
  const bool lead = (threadIdx.x & 63) == 0;
  uint32_t n_bad, n_unsat;
  tm.scan(lead ? bad : 0u, &n_bad);
  // lane 0 of a wave holds the count of the waves before it
  const uint32_t pos = uniform_u32(tm.scan(lead ? n : 0u, &n_unsat));
  tm.sync();
  if (n_bad) {
    if (lane == 0) {
      out[ci].status = 2;
      out[ci].f = out[ci].m = out[ci].nres = 0;
    }
    tm.sync();
    return;
  }
  uint32_t f_total, free_total;
  up_prefix<TW>(tm, nv, T, F, A, P, &f_total, &free_total);
  tm.sync();
  const bool f_ok = (cd.f_expect < 0 || uint32_t(cd.f_expect) == f_total) && f_total <= kMaxLeafVars;
  const bool cap_ok = n_unsat <= cd.nres_cap;
  if (f_ok && cap_ok) fix_records<TW>(cnf, nc, wv, n, list, kFixList, T, F, A, P, res, cd.res_base, pos);
  if (lane == 0) {
    out[ci].status = !f_ok ? 2 : (!cap_ok ? 3 : 0);
    out[ci].f = int32_t(f_total);
    out[ci].m = int32_t(free_total - f_total);
    out[ci].nres = int32_t(n_unsat);
  }
  tm.sync();
}

// Unit propagation of one cube by one team from the empty assignment (the
// cube's literals and the unit clauses), then its active variables, slots
// and residual records.
template <int TW, class Cnf, class Occ>
__device__ void propagate_cube(const Cnf& cnf, const Occ& occ, const DevCubeDesc& cd, uint32_t ci, uint32_t nv,
                               uint32_t nc, const int32_t* __restrict__ cube_lits, DevCubeOut* __restrict__ out,
                               uint4* __restrict__ res, uint32_t* T, uint32_t* F, uint32_t* A, uint32_t* P,
                               uint32_t* Q, uint32_t* X, UpShared& sh) {
  Team<TW> tm{sh};
  const uint32_t lane = tm.lane();
  const uint32_t nw = (nv >> 5) + 1;   // bits 0..nv
  up_clear<TW>(tm, nw, T, F, A, X, sh);
  tm.sync();
  if (cd.n_lits & kCubeFixpoint) {
    // the host's fixpoint: round 0 visits every clause (as after a queue
    // overflow), which confirms it or propagates on from it
    const uint32_t* fw = reinterpret_cast<const uint32_t*>(cube_lits + cd.lit_off);
    for (uint32_t w = lane; w < nw; w += Team<TW>::kSize) { T[w] = fw[w]; F[w] = fw[nw + w]; }
    if (lane == 0) sh.ovf[2] = 1;
  } else {
    up_seed_lits<TW>(tm, cube_lits + cd.lit_off, cd.n_lits, nv, T, F, Q, sh);
    up_seed_units<TW>(tm, cnf, nc, T, F, Q, sh);
  }
  tm.sync();
  up_rounds<TW>(tm, cnf, occ, nv, nc, T, F, Q, X, sh);
  if (uniform_u32(sh.conflict) || uniform_u32(sh.error)) {
    if (lane == 0) {
      out[ci].status = sh.error ? 2 : 1;
      out[ci].f = out[ci].m = out[ci].nres = 0;
    }
    tm.sync();
    return;
  }
  const ActiveScan as = up_active<TW>(tm, cnf, nc, T, F, A);
  tm.sync();
  uint32_t f_total, free_total;
  up_prefix<TW>(tm, nv, T, F, A, P, &f_total, &free_total);
  tm.sync();

  const bool f_ok = (cd.f_expect < 0 || uint32_t(cd.f_expect) == f_total) && f_total <= kMaxLeafVars;
  uint32_t n_unsat;
  const uint32_t pos = tm.scan(as.my_unsat, &n_unsat);
  const bool cap_ok = n_unsat <= cd.nres_cap;
  if (f_ok && cap_ok) up_records(cnf, as, T, F, A, P, res, cd.res_base, pos);
  if (lane == 0) {
    out[ci].status = !f_ok ? 2 : (!cap_ok ? 3 : 0);
    out[ci].f = int32_t(f_total);
    out[ci].m = int32_t(free_total - f_total);
    out[ci].nres = int32_t(n_unsat);
  }
  tm.sync();
}

// Persistent propagation kernel.  A workgroup takes a group of up to
// kUpWaves / TW consecutive cubes of one query; a query whose CNF fits the
// LDS budget is staged once (16-bit clause offsets, literals, occurrence
// offsets and occurrence lists) and shared by the group's teams; each team
// then propagates one cube on its own bitmaps and frontier queues.
template <int TW>
__global__ __launch_bounds__(kBlock) void up_kernel(const DevQueryDesc* __restrict__ qd,
                                                   const uint32_t* __restrict__ coff,
                                                   const int32_t* __restrict__ lits,
                                                   const uint32_t* __restrict__ occ_offs,
                                                   const uint32_t* __restrict__ occs,
                                                   const DevCubeDesc* __restrict__ cubes,
                                                   const int32_t* __restrict__ cube_lits,
                                                   const uint2* __restrict__ groups, uint32_t n_groups,
                                                   DevCubeOut* __restrict__ out, uint4* __restrict__ res,
                                                   uint32_t* head, uint32_t nw_max) {
  // LDS: per team four bitmaps of nw_max words, two frontier queues and
  // the scan space, then the staged CNF
  constexpr uint32_t kTeams = kUpWaves / TW;
  extern __shared__ uint32_t smem[];
  __shared__ UpShared sh[kTeams];
  __shared__ uint32_t s_group;
  const uint32_t tid = threadIdx.x, team = (tid >> 6) / TW;
  const size_t per_team = size_t(nw_max) * 4 + 2 * Team<TW>::kQueue + 2 * Team<TW>::kSize;
  uint32_t* T = smem + team * per_team;
  uint32_t* F = T + nw_max;
  uint32_t* A = F + nw_max;
  uint32_t* P = A + nw_max;
  uint32_t* Q = P + nw_max;
  uint32_t* X = Q + 2 * Team<TW>::kQueue;
  uint16_t* stage = reinterpret_cast<uint16_t*>(smem + kTeams * per_team);

  for (;;) {
    if (tid == 0) s_group = atomicAdd(head, 1u);
    __syncthreads();
    const uint32_t gi = s_group;
    __syncthreads();
    if (gi >= n_groups) break;

    const uint2 g = groups[gi];                  // (first cube, count)
    const DevQueryDesc q = qd[cubes[g.x].qid];
    const uint32_t* co = coff + q.coff_base;
    const int32_t* L = lits + q.lit_base;
    const uint32_t* oo = occ_offs + q.occ_off_base;
    const uint32_t* oc = occs + q.occ_base;
    if (q.staged) {
      const uint32_t nl = co[q.n_clauses];
      const uint32_t nli = 2 * (q.n_vars + 1);
      uint16_t* sco = stage;
      uint16_t* sl = sco + q.n_clauses + 1;
      uint16_t* soo = sl + nl;
      uint16_t* soc = soo + nli + 1;
      // kStageUnroll loads in flight per thread and array
      for (uint32_t b = tid; b <= q.n_clauses; b += kStageUnroll * kBlock) {
        uint32_t x[kStageUnroll];
#pragma unroll
        for (uint32_t u = 0; u < kStageUnroll; u++) {
          const uint32_t c = b + u * kBlock;
          x[u] = c <= q.n_clauses ? co[c] : 0u;
        }
#pragma unroll
        for (uint32_t u = 0; u < kStageUnroll; u++) {
          const uint32_t c = b + u * kBlock;
          if (c <= q.n_clauses) sco[c] = uint16_t(x[u]);
        }
      }
      for (uint32_t b = tid; b < nl; b += kStageUnroll * kBlock) {
        int32_t x[kStageUnroll];
        uint32_t y[kStageUnroll];
#pragma unroll
        for (uint32_t u = 0; u < kStageUnroll; u++) {
          const uint32_t i = b + u * kBlock;
          x[u] = i < nl ? L[i] : 0;
          y[u] = i < nl ? oc[i] : 0u;
        }
#pragma unroll
        for (uint32_t u = 0; u < kStageUnroll; u++) {
          const uint32_t i = b + u * kBlock;
          if (i < nl) {
            sl[i] = uint16_t((uint32_t(x[u] > 0 ? x[u] : -x[u]) << 1) | (x[u] < 0 ? 1u : 0u));
            soc[i] = uint16_t(y[u]);
          }
        }
      }
      for (uint32_t b = tid; b <= nli; b += kStageUnroll * kBlock) {
        uint32_t x[kStageUnroll];
#pragma unroll
        for (uint32_t u = 0; u < kStageUnroll; u++) {
          const uint32_t i = b + u * kBlock;
          x[u] = i <= nli ? oo[i] : 0u;
        }
#pragma unroll
        for (uint32_t u = 0; u < kStageUnroll; u++) {
          const uint32_t i = b + u * kBlock;
          if (i <= nli) soo[i] = uint16_t(x[u]);
        }
      }
      __syncthreads();
      if (team < g.y) {
        const uint32_t ci = g.x + team;
        propagate_cube<TW>(LdsCnf{sco, sl}, LdsOcc{soo, soc}, cubes[ci], ci, q.n_vars, q.n_clauses, cube_lits,
                           out, res, T, F, A, P, Q, X, sh[team]);
      }
    } else if (team < g.y) {
      const uint32_t ci = g.x + team;
      propagate_cube<TW>(GlobalCnf{co, L}, GlobalOcc{oo, oc}, cubes[ci], ci, q.n_vars, q.n_clauses, cube_lits,
                         out, res, T, F, A, P, Q, X, sh[team]);
    }
    __syncthreads();   // the staged CNF is replaced by the next group
  }
}

// Persistent kernel for launches whose cubes all carry the host's
// fixpoint.  A workgroup takes a group of cubes of one query (up to four
// one-wave teams, else one cube), as up_kernel does, and each team checks
// one cube with fix_cube.  Nothing is staged: the one pass reads the CNF
// from HBM, and the launch asks only for the teams' bitmaps and lists, so
// more workgroups share a CU than with staging.  TW = 8 (workgroups of
// 512 threads, one cube each, three per CU) is for rounds with large CNFs:
// eight waves finish a large cube about twice as soon as four, and while
// one workgroup of a CU waits on the loads that start its next cube (the
// group claim, the descriptors, the fixpoint), the others stream clauses.
template <int TW>
constexpr int fix_threads() { return TW == 8 ? 512 : kBlock; }
template <int TW>
__global__ __launch_bounds__(fix_threads<TW>())
__attribute__((amdgpu_waves_per_eu(TW == 1 ? 5 : 6))) void fix_kernel(const DevQueryDesc* __restrict__ qd,
                                                    const uint32_t* __restrict__ coff,
                                                    const int32_t* __restrict__ lits,
                                                    const DevCubeDesc* __restrict__ cubes,
                                                    const int32_t* __restrict__ cube_lits,
                                                    const uint2* __restrict__ groups, uint32_t n_groups,
                                                    DevCubeOut* __restrict__ out, uint4* __restrict__ res,
                                                    uint32_t* head, uint32_t nw_max) {
  // LDS per team: T, F, A, P of nw_max words, T and F interleaved (2 nw_max
  // words), then kFixList per wave
  constexpr uint32_t kTeams = fix_threads<TW>() / 64 / TW;
  extern __shared__ uint32_t smem[];
  __shared__ UpShared sh[kTeams];
  __shared__ uint32_t s_group;
  // the group, the cube and its query are wave-uniform (scalar loads, and
  // CNF bases in scalar registers)
  const uint32_t tid = threadIdx.x, team = uniform_u32((tid >> 6) / TW);
  uint32_t* T = smem + team * (size_t(nw_max) * 6 + TW * kFixList);
  uint32_t* F = T + nw_max;
  uint32_t* A = F + nw_max;
  uint32_t* P = A + nw_max;
  uint2* TF = reinterpret_cast<uint2*>(P + nw_max);
  uint32_t* lists = P + 3 * size_t(nw_max);
  for (;;) {
    if (tid == 0) s_group = atomicAdd(head, 1u);
    __syncthreads();
    const uint32_t gi = uniform_u32(s_group);
    __syncthreads();
    if (gi >= n_groups) break;
    const uint2 g = groups[gi];
    if (team < g.y) {
      const uint32_t ci = g.x + team;
      const DevQueryDesc q = qd[cubes[ci].qid];
      Team<TW> tm{sh[team]};
      fix_cube<TW>(tm, GlobalCnf{coff + q.coff_base, lits + q.lit_base}, cubes[ci], ci, q.n_vars, q.n_clauses,
                   cube_lits, out, res, T, F, A, P, TF, lists);
    }
  }
}

// acc AND a clause's satisfaction word: lanes in the clause's lane mask (a
// literal of slots 6..11 holds there) keep acc, the others AND in the OR of
// the slot-0..5 literal patterns.  The uniform lane mask serves directly as
// the per-lane condition of the select (its only scalar operand).
__device__ __forceinline__ uint64_t clause_and(uint64_t acc, const uint4& r) {
  const uint64_t lanes = (uint64_t(r.w) << 32) | r.z;
  const uint32_t alo = uint32_t(acc), ahi = uint32_t(acc >> 32);
  const uint32_t tlo = alo & r.x, thi = ahi & r.y;
  uint32_t nlo, nhi;
  asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(nlo) : "v"(tlo), "v"(alo), "s"(lanes));
  asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(nhi) : "v"(thi), "v"(ahi), "s"(lanes));
  return (uint64_t(nhi) << 32) | nlo;
}

__global__ __launch_bounds__(kBlock) void leaf_kernel(const DevItem* __restrict__ items,
                                                     uint32_t n_items,
                                                     const DevCubeDesc* __restrict__ cubes,
                                                     DevCubeOut* __restrict__ out,
                                                     const uint4* __restrict__ res,
                                                     unsigned long long* __restrict__ qkey,
                                                     uint32_t* head, uint32_t mode,
                                                     const uint32_t* __restrict__ n_items_dev) {
  __shared__ uint32_t s_base, s_skip;
  // the item count from device memory when the host does not know it
  if (n_items_dev) n_items = *n_items_dev;
  // the wave index is the same for all lanes of a wave: make that explicit so
  // that block indices, the skip tests and the clause loop stay scalar
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = uniform_u32(tid >> 6);
  constexpr uint32_t kWaves = kBlock / 64;
  constexpr uint32_t kClaim = 8;   // items taken per claim

  for (;;) {
    // the first wave claims kClaim consecutive items and decides, one lane
    // per item, which are still useful (not a device-refuted leaf, and in
    // DECIDE mode not preceded by a witness already found for the query)
    if (wave == 0) {
      uint32_t base = 0;
      if (lane == 0) base = atomicAdd(head + 1, kClaim);
      base = uniform_u32(__shfl(base, 0, 64));
      bool skip = true;
      const uint32_t i = base + lane;
      if (lane < kClaim && i < n_items) {
        const DevItem it0 = items[i];
        skip = out[it0.cube].status != 0;
        if (!skip && mode == SCUBA_MODE_DECIDE) {
          const DevCubeDesc c0 = cubes[it0.cube];
          const uint64_t k = __hip_atomic_load(&qkey[c0.qid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          skip = k <= (uint64_t(c0.seq) << 38) + (uint64_t(it0.it_lo) << 12);
        }
      }
      const uint64_t mask = __ballot(skip);
      if (lane == 0) {
        s_base = base;
        s_skip = uint32_t(mask);
      }
    }
    __syncthreads();
    const uint32_t base = s_base, skip_mask = s_skip;
    __syncthreads();
    if (base >= n_items) break;
    for (uint32_t t = 0; t < kClaim; t++) {
      const uint32_t item = base + t;
      if (item >= n_items) break;
      if ((skip_mask >> t) & 1) continue;

      const DevItem it = items[item];
      const DevCubeDesc cd = cubes[it.cube];
      const uint32_t f = uniform_u32(uint32_t(out[it.cube].f));
      const uint32_t nres = uniform_u32(uint32_t(out[it.cube].nres));
      const uint64_t key_base = uint64_t(cd.seq) << 38;
      // the leaf's records, read with wave-uniform (scalar) loads
      const uint4* __restrict__ rec = res + 2 * uniform_u64(cd.res_base);

      uint64_t valid;
      if (f >= 12) valid = ~0ull;
      else if (f >= 6) valid = lane < (1u << (f - 6)) ? ~0ull : 0ull;
      else valid = lane == 0 ? ((2ull << ((1u << f) - 1)) - 1) : 0ull;

      uint64_t count = 0, blocks = 0, evals = 0, word_ops = 0, first = ~0ull;
      uint32_t steps = 0;
      bool stop = false;
      // kPass blocks per pass over the records (blk, blk + kWaves, ..., the
      // wave's next kPass): one set of record loads, kPass independent
      // dependency chains.  Each block keeps its own clause sequence and
      // dead-block test (after every group of four records), exactly as if
      // it were evaluated alone.
      for (uint32_t blk = it.it_lo + wave; blk < it.it_hi && !stop; blk += kPass * kWaves) {
        if (mode == SCUBA_MODE_DECIDE && (steps++ & 3) == 0) {
          const uint64_t k = uniform_u64(
              __hip_atomic_load(&qkey[cd.qid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
          if (k <= key_base + (uint64_t(blk) << 12)) break;
        }
        uint32_t H[kPass], live[kPass], done[kPass], lits[kPass];
        uint64_t acc[kPass];
        uint32_t n_in = 0, any = 0;
#pragma unroll
        for (uint32_t p = 0; p < kPass; p++) {
          const uint32_t b = blk + p * kWaves;
          const bool in = b < it.it_hi;
          H[p] = b & kHighMask;
          acc[p] = in ? valid : 0ull;
          live[p] = in ? 1u : 0u;   // wave-uniform 0 / 1 (a plain scalar)
          done[p] = lits[p] = 0;
          n_in += in;
          any |= live[p];
        }
        // runs of at most kRecRun records: an evaluated clause adds its
        // record's packed counter (one scalar add), unpacked after each run
        for (uint32_t c0 = 0; c0 < nres && any; c0 += kRecRun) {
          const uint32_t cend = min(nres, c0 + kRecRun);
          uint32_t pk[kPass];
#pragma unroll
          for (uint32_t p = 0; p < kPass; p++) pk[p] = 0;
          // four clauses per step: their records are loaded together (the
          // record region is padded so that reading past nres stays inside
          // it); full groups first, then the last partial group
          uint32_t c = c0;
          for (; c + 4 <= cend; c += 4) {
            const uint4 r0 = rec[2 * c], r1 = rec[2 * c + 1], r2 = rec[2 * c + 2], r3 = rec[2 * c + 3];
            const uint4 r4 = rec[2 * c + 4], r5 = rec[2 * c + 5], r6 = rec[2 * c + 6], r7 = rec[2 * c + 7];
            // the four skip masks are needed first; the length words are
            // named too, so that each record pair stays one 32-byte load
            asm volatile("" :: "s"(r1.x), "s"(r1.y), "s"(r3.x), "s"(r3.y), "s"(r5.x), "s"(r5.y), "s"(r7.x), "s"(r7.y));
            asm volatile("" :: "s"(r1.z), "s"(r3.z), "s"(r5.z), "s"(r7.z));
            any = 0;
#pragma unroll
            for (uint32_t p = 0; p < kPass; p++) {
              if (live[p]) {
                const uint32_t h = H[p];
                if (!(~(h ^ r1.x) & r1.y)) { acc[p] = clause_and(acc[p], r0); pk[p] += r1.w; }
                if (!(~(h ^ r3.x) & r3.y)) { acc[p] = clause_and(acc[p], r2); pk[p] += r3.w; }
                if (!(~(h ^ r5.x) & r5.y)) { acc[p] = clause_and(acc[p], r4); pk[p] += r5.w; }
                if (!(~(h ^ r7.x) & r7.y)) { acc[p] = clause_and(acc[p], r6); pk[p] += r7.w; }
                live[p] = uint32_t(__any(acc[p] != 0));
              }
              any |= live[p];
            }
            if (!any) break;
          }
          if (c < cend && any) {
            const uint4 r0 = rec[2 * c], r1 = rec[2 * c + 1], r2 = rec[2 * c + 2], r3 = rec[2 * c + 3];
            const uint4 r4 = rec[2 * c + 4], r5 = rec[2 * c + 5];
            const uint32_t left = cend - c;   // 1..3
            any = 0;
#pragma unroll
            for (uint32_t p = 0; p < kPass; p++) {
              if (live[p]) {
                const uint32_t h = H[p];
                if (!(~(h ^ r1.x) & r1.y)) { acc[p] = clause_and(acc[p], r0); pk[p] += r1.w; }
                if (left > 1 && !(~(h ^ r3.x) & r3.y)) { acc[p] = clause_and(acc[p], r2); pk[p] += r3.w; }
                if (left > 2 && !(~(h ^ r5.x) & r5.y)) { acc[p] = clause_and(acc[p], r4); pk[p] += r5.w; }
                live[p] = uint32_t(__any(acc[p] != 0));
              }
              any |= live[p];
            }
          }
#pragma unroll
          for (uint32_t p = 0; p < kPass; p++) {
            done[p] += pk[p] >> 20;
            lits[p] += pk[p] & (kRecCount - 1);
          }
        }
        blocks += n_in;
#pragma unroll
        for (uint32_t p = 0; p < kPass; p++) {
          evals += done[p];
          word_ops += uint64_t(lits[p]) * 64;   // (|c| + 1) per clause and 64-bit word
          if (mode == SCUBA_MODE_COUNT) count += __popcll(acc[p]);
        }
        // satisfying assignments, the earlier block first
        for (uint32_t h = 0; h < n_in; h++) {
          uint64_t a_acc = acc[0];
#pragma unroll
          for (uint32_t p = 1; p < kPass; p++)
            if (h == p) a_acc = acc[p];
          const uint64_t hit = __ballot(a_acc != 0);
          if (!hit) continue;
          const uint32_t fl = __builtin_ctzll(hit);
          const uint64_t acc_fl = __shfl(a_acc, int(fl), 64);
          const uint64_t a = (uint64_t(blk + h * kWaves) << 12) | (uint64_t(fl) << 6) |
                             uint64_t(__builtin_ctzll(acc_fl));
          if (lane == 0) {
            if (a < first) first = a;
            if (mode == SCUBA_MODE_DECIDE) atomicMin(&qkey[cd.qid], (unsigned long long)(key_base | a));
          }
          if (mode == SCUBA_MODE_DECIDE) {
            stop = true;
            break;
          }
        }
      }
      // wave totals
      for (uint32_t d = 32; d >= 1; d >>= 1) count += __shfl_xor(count, int(d), 64);
      if (lane == 0) {
        if (mode == SCUBA_MODE_COUNT && count) atomicAdd((unsigned long long*)&out[it.cube].count, (unsigned long long)count);
        if (first != ~0ull) atomicMin((unsigned long long*)&out[it.cube].first, (unsigned long long)first);
        atomicAdd((unsigned long long*)&out[it.cube].blocks, (unsigned long long)blocks);
        atomicAdd((unsigned long long*)&out[it.cube].clause_blocks, (unsigned long long)evals);
        atomicAdd((unsigned long long*)&out[it.cube].word_ops, (unsigned long long)word_ops);
      }
    }
  }
}


// The same evaluation with the skip test on the vector unit.  Per block,
// a wave takes the leaf's clauses 64 at a time, lane i holding the record
// of clause g + i: one vector test per lane finds the clauses that no
// block-level literal satisfies, a ballot collects them, and each of those
// is broadcast to the wave (v_readlane of its pattern word and lane mask)
// and ANDed in as above.  A clause satisfied at block level costs no scalar
// instruction.  The word-operation counters are per-lane sums (corrected
// for the clauses a dead block did not reach), so they count exactly the
// clauses evaluated.  kLds: a work item's records are first staged in LDS
// by the whole workgroup (coalesced 16-byte loads) when they fit
// lds_records; else every wave reads them from memory.
template <bool kLds>
__global__ __launch_bounds__(kBlock) void leaf_kernel_v(const DevItem* __restrict__ items, uint32_t n_items,
                                                       const DevCubeDesc* __restrict__ cubes,
                                                       DevCubeOut* __restrict__ out,
                                                       const uint4* __restrict__ res,
                                                       unsigned long long* __restrict__ qkey, uint32_t* head,
                                                       uint32_t mode, const uint32_t* __restrict__ n_items_dev,
                                                       uint32_t lds_records) {
  extern __shared__ uint4 tile[];
  __shared__ uint32_t s_base, s_skip;
  if (n_items_dev) n_items = *n_items_dev;
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = uniform_u32(tid >> 6);
  constexpr uint32_t kWaves = kBlock / 64;
  constexpr uint32_t kClaim = 8;
  for (;;) {
    if (wave == 0) {
      uint32_t base = 0;
      if (lane == 0) base = atomicAdd(head + 1, kClaim);
      base = uniform_u32(__shfl(base, 0, 64));
      bool skip = true;
      const uint32_t i = base + lane;
      if (lane < kClaim && i < n_items) {
        const DevItem it0 = items[i];
        skip = out[it0.cube].status != 0;
        if (!skip && mode == SCUBA_MODE_DECIDE) {
          const DevCubeDesc c0 = cubes[it0.cube];
          const uint64_t k = __hip_atomic_load(&qkey[c0.qid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          skip = k <= (uint64_t(c0.seq) << 38) + (uint64_t(it0.it_lo) << 12);
        }
      }
      const uint64_t mask = __ballot(skip);
      if (lane == 0) {
        s_base = base;
        s_skip = uint32_t(mask);
      }
    }
    __syncthreads();
    const uint32_t base = uniform_u32(s_base), skip_mask = uniform_u32(s_skip);
    __syncthreads();
    if (base >= n_items) break;
    for (uint32_t t = 0; t < kClaim; t++) {
      const uint32_t item = base + t;
      if (item >= n_items) break;
      if ((skip_mask >> t) & 1) continue;
      const DevItem it = items[item];
      const DevCubeDesc cd = cubes[it.cube];
      const uint32_t f = uniform_u32(uint32_t(out[it.cube].f));
      const uint32_t nres = uniform_u32(uint32_t(out[it.cube].nres));
      const uint64_t key_base = uint64_t(cd.seq) << 38;
      const uint4* __restrict__ src = res + 2 * uniform_u64(cd.res_base);
      const bool staged = kLds && nres <= lds_records;
      if (kLds) {
        __syncthreads();   // the previous item's tile is no longer read
        if (staged)
          for (uint32_t x = tid; x < 2 * nres; x += kBlock) tile[x] = src[x];
        __syncthreads();
      }
      uint64_t valid;
      if (f >= 12) valid = ~0ull;
      else if (f >= 6) valid = lane < (1u << (f - 6)) ? ~0ull : 0ull;
      else valid = lane == 0 ? ((2ull << ((1u << f) - 1)) - 1) : 0ull;

      uint64_t count = 0, first = ~0ull;
      uint32_t blocks = 0, evals = 0, word_lanes = 0, steps = 0;
      for (uint32_t blk = it.it_lo + wave; blk < it.it_hi; blk += kWaves) {
        if (mode == SCUBA_MODE_DECIDE && (steps++ & 7) == 0) {
          const uint64_t k = uniform_u64(
              __hip_atomic_load(&qkey[cd.qid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
          if (k <= key_base + (uint64_t(blk) << 12)) break;
        }
        const uint32_t H = blk & kHighMask;
        uint64_t acc = valid;
        for (uint32_t g = 0; g < nres; g += 64) {
          const uint32_t c = g + lane;
          uint4 r0 = make_uint4(0u, 0u, 0u, 0u), r1 = make_uint4(0u, 0u, 0u, 0u);
          if (c < nres) {
            if (staged) {
              r0 = tile[2 * c];
              r1 = tile[2 * c + 1];
            } else {
              r0 = src[2 * c];
              r1 = src[2 * c + 1];
            }
          }
          const bool ap = c < nres && !(~(H ^ r1.x) & r1.y);
          uint64_t m = __ballot(ap);
          const uint32_t n_ap = uint32_t(__popcll(m));
          evals += n_ap;
          if (ap) word_lanes += r1.z + 1;
          uint32_t n_done = 0;
          while (m) {
            const uint32_t j = uint32_t(__builtin_ctzll(m));
            m &= m - 1;
            const uint4 r = make_uint4(uint32_t(__builtin_amdgcn_readlane(int(r0.x), int(j))),
                                       uint32_t(__builtin_amdgcn_readlane(int(r0.y), int(j))),
                                       uint32_t(__builtin_amdgcn_readlane(int(r0.z), int(j))),
                                       uint32_t(__builtin_amdgcn_readlane(int(r0.w), int(j))));
            acc = clause_and(acc, r);
            if ((++n_done & 3) == 0 && m && !__any(acc != 0)) break;
          }
          if (m) {
            // the block died before the clauses still in m: not evaluated
            evals -= uint32_t(__popcll(m));
            if (ap && ((m >> lane) & 1)) word_lanes -= r1.z + 1;
          }
          if (!__any(acc != 0)) break;
        }
        blocks++;
        if (mode == SCUBA_MODE_COUNT) count += __popcll(acc);
        const uint64_t hit = __ballot(acc != 0);
        if (hit) {
          const uint32_t fl = __builtin_ctzll(hit);
          const uint64_t acc_fl = __shfl(acc, int(fl), 64);
          const uint64_t a = (uint64_t(blk) << 12) | (uint64_t(fl) << 6) | uint64_t(__builtin_ctzll(acc_fl));
          if (lane == 0) {
            if (a < first) first = a;
            if (mode == SCUBA_MODE_DECIDE) atomicMin(&qkey[cd.qid], (unsigned long long)(key_base | a));
          }
          if (mode == SCUBA_MODE_DECIDE) break;
        }
      }
      uint64_t wl = word_lanes;
      for (uint32_t d = 32; d >= 1; d >>= 1) {
        count += __shfl_xor(count, int(d), 64);
        wl += __shfl_xor(wl, int(d), 64);
      }
      if (lane == 0) {
        if (mode == SCUBA_MODE_COUNT && count) atomicAdd((unsigned long long*)&out[it.cube].count, (unsigned long long)count);
        if (first != ~0ull) atomicMin((unsigned long long*)&out[it.cube].first, (unsigned long long)first);
        atomicAdd((unsigned long long*)&out[it.cube].blocks, (unsigned long long)blocks);
        atomicAdd((unsigned long long*)&out[it.cube].clause_blocks, (unsigned long long)evals);
        atomicAdd((unsigned long long*)&out[it.cube].word_ops, (unsigned long long)(wl * 64));
      }
    }
  }
}

// ---------------------------------------------------------------- device split
// Counters of the split loop (u32 words of one 256-byte block).
constexpr uint32_t kSpExpandHead = 0;   // expansion: next popped node
constexpr uint32_t kSpChildren = 1;     // children pushed by this step
constexpr uint32_t kSpLeaves = 2;       // leaves emitted by this step
constexpr uint32_t kSpRes = 3;          // their residual records
constexpr uint32_t kSpItems = 4;        // their work items
constexpr uint32_t kSpError = 5;        // a propagation error (a broken invariant)
constexpr uint32_t kSpLeafHead = 6;     // leaf kernel's head (it claims at head + 1)

// Work items of a leaf with f active variables: blocks of 4096 assignments
// in chunks of 2^chunk_log2 blocks, at most kSplitItemsPerLeaf chunks.
__device__ __forceinline__ uint32_t split_items_of(int32_t f, uint32_t chunk_log2, uint32_t* chunk) {
  const uint32_t blocks = f >= 12 ? (1u << (f - 12)) : 1u;
  uint32_t c = chunk_log2 >= 26 ? (1u << 26) : (1u << chunk_log2);
  const uint32_t need = (blocks + kSplitItemsPerLeaf - 1) / kSplitItemsPerLeaf;
  if (c < need) c = need;
  *chunk = c;
  return (blocks + c - 1) / c;
}

// One popped node per wave: the parent's fixpoint plus the decision literal
// (or a start node from the empty assignment), propagation to the new
// fixpoint, then: a conflict is a refuted cube; at most k active variables
// and at most max_res unsatisfied clauses make a leaf; else the first
// active variable of the query's branch order is the branching variable
// (its negative literal is the branch explored first).  The fixpoint of a
// leaf or branching node goes to fix_out.  Nodes of queries already decided
// or out of budget are dropped.
__global__ __launch_bounds__(kBlock) void split_expand_kernel(
    const DevQueryDesc* __restrict__ qd, const uint32_t* __restrict__ coff, const int32_t* __restrict__ lits,
    const uint32_t* __restrict__ occ_offs, const uint32_t* __restrict__ occs,
    const unsigned long long* __restrict__ order_off, const uint32_t* __restrict__ order,
    const DevSplitNode* __restrict__ nodes, const uint32_t* __restrict__ node_fix, uint32_t first, uint32_t b,
    const int32_t* __restrict__ start_lits, const unsigned long long* __restrict__ qkey,
    DevSplitStat* __restrict__ stats, DevSplitOut* __restrict__ sout, uint32_t* __restrict__ fix_out,
    uint32_t* __restrict__ ctr, uint32_t nw_max, uint32_t k, uint32_t max_res, unsigned long long max_cubes) {
  extern __shared__ uint32_t smem[];
  __shared__ UpShared sh[kUpWaves];
  __shared__ uint32_t s_claim[kUpWaves];
  const uint32_t lane = threadIdx.x & 63, wave = uniform_u32(threadIdx.x >> 6);
  const size_t per_team = size_t(nw_max) * 4 + 2 * Team<1>::kQueue + 2 * Team<1>::kSize;
  uint32_t* T = smem + wave * per_team;
  uint32_t* F = T + nw_max;
  uint32_t* A = F + nw_max;
  uint32_t* P = A + nw_max;
  uint32_t* Q = P + nw_max;
  uint32_t* X = Q + 2 * Team<1>::kQueue;
  Team<1> tm{sh[wave]};
  for (;;) {
    // the claimed node index goes through LDS: a value that only lane 0
    // sets and a readfirstlane broadcasts lets the compiler fold the other
    // lanes' placeholder into a constant on a path of its own, after which
    // those lanes work on another node than lane 0
    if (lane == 0) s_claim[wave] = atomicAdd(&ctr[kSpExpandHead], 1u);
    wave_sync();
    const uint32_t i = uniform_u32(s_claim[wave]);
    wave_sync();
    if (i >= b) break;
    const DevSplitNode nd = nodes[first + i];
    const uint32_t qid = uniform_u32(nd.qid);
    DevSplitOut so{};
    so.qid = qid;
    // both read once for the wave, so that the drop is a uniform branch
    const unsigned long long key =
        uniform_u64(__hip_atomic_load(&qkey[qid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    const unsigned long long spent =
        uniform_u64(__hip_atomic_load(&stats[qid].cubes, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (key != ~0ull || spent >= max_cubes) {
      if (lane == 0) {
        if (key == ~0ull) stats[qid].budget = 1;
        sout[i] = so;   // kind 0: dropped
      }
      // every path back to the claim passes a wave barrier after its lane-0
      // stores: without one here the compiler sends lanes 1..63 back to the
      // loop head on a path of their own, around lane 0's claim
      tm.sync();
      continue;
    }
    const DevQueryDesc q = qd[qid];
    const uint32_t nv = q.n_vars, nc = q.n_clauses, nw = (nv >> 5) + 1;
    const GlobalCnf cnf{coff + q.coff_base, lits + q.lit_base};
    const GlobalOcc occ{occ_offs + q.occ_off_base, occs + q.occ_base};
    up_clear<1>(tm, nw, T, F, A, X, sh[wave]);
    tm.sync();
    const bool start = nd.lit == 0;
    if (!start) {
      const uint32_t* fx = node_fix + size_t(first + i) * 2 * nw_max;
      for (uint32_t w = lane; w < nw; w += 64) { T[w] = fx[w]; F[w] = fx[nw_max + w]; }
      tm.sync();
      up_seed_lits<1>(tm, &nodes[first + i].lit, 1, nv, T, F, Q, sh[wave]);
    } else {
      up_seed_lits<1>(tm, start_lits + nd.lit_off, nd.n_lits, nv, T, F, Q, sh[wave]);
      up_seed_units<1>(tm, cnf, nc, T, F, Q, sh[wave]);
    }
    tm.sync();
    up_rounds<1>(tm, cnf, occ, nv, nc, T, F, Q, X, sh[wave]);
    if (uniform_u32(sh[wave].conflict) || uniform_u32(sh[wave].error)) {
      if (lane == 0) {
        if (sh[wave].error) ctr[kSpError] = 1;
        atomicAdd(&stats[qid].cubes, 1ull);
        atomicAdd(&stats[qid].refuted, 1ull);
        so.kind = kSplitRefuted;
        sout[i] = so;
      }
      tm.sync();
      continue;
    }
    // A query of kSplitWideClauses clauses or more takes its unassigned
    // variables as the node's slots (m = 0), counted from the bitmaps; the
    // unsatisfied clauses are counted by a pass over the clauses only when
    // that could make a leaf.  Smaller queries count the active variables
    // (unassigned, in an unsatisfied clause) exactly.
    const bool wide = nc >= kSplitWideClauses;
    uint32_t f_total, free_total, n_unsat = 0;
    if (wide) {
      uint32_t my_free = 0;
      for (uint32_t w = lane; w < nw; w += 64) my_free += __popc(~(T[w] | F[w]) & var_mask(w, nv));
      tm.scan(my_free, &free_total);
      f_total = free_total;
      if (f_total <= k && f_total > 0) {
        uint32_t bad;
        n_unsat = fix_scan<1>(cnf, nc, 0, T, F, A, nullptr, 0, &bad);
      }
    } else {
      const ActiveScan as = up_active<1>(tm, cnf, nc, T, F, A);
      tm.sync();
      up_prefix<1>(tm, nv, T, F, A, P, &f_total, &free_total);
      tm.scan(as.my_unsat, &n_unsat);
    }
    so.f = int32_t(f_total);
    so.m = int32_t(free_total - f_total);
    so.nres = n_unsat;
    if (f_total <= k && n_unsat <= max_res) {
      so.kind = kSplitLeaf;
      if (lane == 0) atomicAdd(&stats[qid].cubes, 1ull);
    } else {
      // the first variable of the branch order that is active (unassigned
      // for a wide query), 64 candidates at a time
      const uint32_t* ord = order + order_off[qid];
      uint32_t v = 0;
      for (uint32_t j0 = 0; j0 < nv; j0 += 64) {
        const uint32_t j = j0 + lane;
        const uint32_t x = j < nv ? ord[j] : 0u;
        const uint32_t bit = 1u << (x & 31);
        const bool act = x != 0 && x <= nv &&
                         (wide ? !((T[x >> 5] | F[x >> 5]) & bit) : ((A[x >> 5] & bit) != 0));
        const uint64_t m = __ballot(act);
        if (m) {
          v = uint32_t(__builtin_amdgcn_readlane(int(x), int(__builtin_ctzll(m))));
          break;
        }
      }
      if (v == 0) {   // f > 0 has an active variable: cannot happen
        if (lane == 0) ctr[kSpError] = 1;
        so.kind = kSplitDropped;
      } else {
        so.kind = kSplitBranch;
        so.lit = -int32_t(v);
      }
    }
    uint32_t* fo = fix_out + size_t(i) * 2 * nw_max;
    for (uint32_t w = lane; w < nw; w += 64) { fo[w] = T[w]; fo[nw_max + w] = F[w]; }
    if (lane == 0) sout[i] = so;
    tm.sync();
  }
}

// Exclusive scan over the workgroup (1024 threads) of one value per thread.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* total, uint32_t* part) {
  const uint32_t wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
  uint32_t wt;
  const uint32_t x = wave_exclusive_scan(v, &wt);
  if ((threadIdx.x & 63) == 0) part[wv] = wt;
  __syncthreads();
  uint32_t base = 0, tot = 0;
  for (uint32_t w = 0; w < nwv; w++) {
    if (w < wv) base += part[w];
    tot += part[w];
  }
  __syncthreads();   // part is rewritten by the next scan
  *total = tot;
  return base + x;
}

// One workgroup: positions of this step's children, leaves, residual
// records and work items (exclusive scans over the popped nodes, in their
// order, so the layout is deterministic), the step totals, and the heads
// of the next kernels reset.
__global__ __launch_bounds__(1024) void split_scan_kernel(const DevSplitOut* __restrict__ sout, uint32_t b,
                                                          uint32_t chunk_log2, uint32_t* __restrict__ child_off,
                                                          uint32_t* __restrict__ leaf_idx,
                                                          uint32_t* __restrict__ res_off,
                                                          uint32_t* __restrict__ item_off,
                                                          uint32_t* __restrict__ ctr) {
  __shared__ uint32_t part[16];
  const uint32_t per = (b + blockDim.x - 1) / blockDim.x;
  const uint32_t i0 = min(b, threadIdx.x * per), i1 = min(b, i0 + per);
  uint32_t c = 0, l = 0, r = 0, it = 0;
  for (uint32_t i = i0; i < i1; i++) {
    const DevSplitOut so = sout[i];
    uint32_t ch;
    c += so.kind == kSplitBranch ? 2u : 0u;
    if (so.kind == kSplitLeaf) {
      l++;
      r += so.nres;
      it += split_items_of(so.f, chunk_log2, &ch);
    }
  }
  uint32_t tc, tl, tr, ti;
  uint32_t bc = block_exclusive_scan(c, &tc, part);
  uint32_t bl = block_exclusive_scan(l, &tl, part);
  uint32_t br = block_exclusive_scan(r, &tr, part);
  uint32_t bi = block_exclusive_scan(it, &ti, part);
  for (uint32_t i = i0; i < i1; i++) {
    const DevSplitOut so = sout[i];
    uint32_t ch;
    child_off[i] = bc;
    leaf_idx[i] = bl;
    res_off[i] = br;
    item_off[i] = bi;
    bc += so.kind == kSplitBranch ? 2u : 0u;
    if (so.kind == kSplitLeaf) {
      bl++;
      br += so.nres;
      bi += split_items_of(so.f, chunk_log2, &ch);
    }
  }
  if (threadIdx.x == 0) {
    ctr[kSpChildren] = tc;
    ctr[kSpLeaves] = tl;
    ctr[kSpRes] = tr;
    ctr[kSpItems] = ti;
    ctr[kSpExpandHead] = 0;
    ctr[kSpLeafHead + 1] = 0;
  }
}

// One popped node per wave.  A branching node of rank r among the step's
// nb branching nodes pushes its second branch at r and its first branch at
// nb + r, each with a copy of the node's fixpoint: the first branches of
// the whole step lie on top, so a step of nb nodes continues every query's
// walk depth-first.  A leaf gets its cube descriptor, initial results,
// residual records (rebuilt from its fixpoint, as the propagation kernels
// build them) and work items.
__global__ __launch_bounds__(kBlock) void split_scatter_kernel(
    const DevQueryDesc* __restrict__ qd, const uint32_t* __restrict__ coff, const int32_t* __restrict__ lits,
    const DevSplitOut* __restrict__ sout, const uint32_t* __restrict__ fix_out, uint32_t first, uint32_t b,
    const uint32_t* __restrict__ child_off, const uint32_t* __restrict__ leaf_idx,
    const uint32_t* __restrict__ res_off, const uint32_t* __restrict__ item_off, DevSplitNode* __restrict__ nodes,
    uint32_t* __restrict__ node_fix, DevCubeDesc* __restrict__ descs, DevCubeOut* __restrict__ louts,
    uint32_t* __restrict__ leaf_src, DevItem* __restrict__ items, uint4* __restrict__ res, uint32_t seq_base,
    uint32_t nw_max, uint32_t chunk_log2, const uint32_t* __restrict__ ctr) {
  extern __shared__ uint32_t smem[];
  __shared__ UpShared sh[kUpWaves];
  const uint32_t lane = threadIdx.x & 63, wave = uniform_u32(threadIdx.x >> 6);
  uint32_t* T = smem + wave * (size_t(nw_max) * 4 + kFixList);
  uint32_t* F = T + nw_max;
  uint32_t* A = F + nw_max;
  uint32_t* P = A + nw_max;
  uint32_t* list = P + nw_max;
  const uint32_t nb = ctr[kSpChildren] / 2;   // branching nodes of this step
  Team<1> tm{sh[wave]};
  for (uint32_t i = blockIdx.x * kUpWaves + wave; i < b; i += gridDim.x * kUpWaves) {
    const DevSplitOut so = sout[i];
    const uint32_t kind = uniform_u32(so.kind);
    const uint32_t* fx = fix_out + size_t(i) * 2 * nw_max;
    if (kind == kSplitBranch) {
      const uint32_t r = child_off[i] / 2;
      const uint32_t s0 = first + r, s1 = first + nb + r;
      if (lane == 0) {
        nodes[s0] = DevSplitNode{so.qid, -so.lit, 0u, 0u};
        nodes[s1] = DevSplitNode{so.qid, so.lit, 0u, 0u};
      }
      uint32_t* d0 = node_fix + size_t(s0) * 2 * nw_max;
      uint32_t* d1 = node_fix + size_t(s1) * 2 * nw_max;
      const uint32_t nw = (qd[so.qid].n_vars >> 5) + 1;
      for (uint32_t w = lane; w < nw; w += 64) {
        const uint32_t t = fx[w], f = fx[nw_max + w];
        d0[w] = t;
        d0[nw_max + w] = f;
        d1[w] = t;
        d1[nw_max + w] = f;
      }
      tm.sync();   // the whole wave reaches the next node together
    } else if (kind == kSplitLeaf) {
      const uint32_t j = leaf_idx[i];
      const DevQueryDesc q = qd[so.qid];
      const uint32_t nv = q.n_vars, nc = q.n_clauses, nw = (nv >> 5) + 1;
      const GlobalCnf cnf{coff + q.coff_base, lits + q.lit_base};
      const bool wide = nc >= kSplitWideClauses;
      // a wide query's slots are its unassigned variables
      for (uint32_t w = lane; w < nw; w += 64) {
        const uint32_t t = fx[w], f = fx[nw_max + w];
        T[w] = t;
        F[w] = f;
        A[w] = wide ? ~(t | f) & var_mask(w, nv) : 0u;
      }
      tm.sync();
      uint32_t f_total, free_total, n_unsat = 0;
      if (wide) {
        // the listing pass only when the leaf has unsatisfied clauses (its
        // marks fall on variables that A already holds)
        uint32_t n = 0, bad = 0;
        if (so.nres) n = fix_scan<1>(cnf, nc, 0, T, F, A, list, kFixList, &bad);
        tm.sync();
        up_prefix<1>(tm, nv, T, F, A, P, &f_total, &free_total);
        tm.sync();
        if (n) fix_records<1>(cnf, nc, 0, n, list, kFixList, T, F, A, P, res, res_off[i], 0);
        n_unsat = n;
      } else {
        const ActiveScan as = up_active<1>(tm, cnf, nc, T, F, A);
        tm.sync();
        up_prefix<1>(tm, nv, T, F, A, P, &f_total, &free_total);
        tm.sync();
        const uint32_t pos = tm.scan(as.my_unsat, &n_unsat);
        up_records(cnf, as, T, F, A, P, res, res_off[i], pos);
      }
      uint32_t chunk;
      const uint32_t n_it = split_items_of(so.f, chunk_log2, &chunk);
      const uint32_t blocks = so.f >= 12 ? (1u << (so.f - 12)) : 1u;
      for (uint32_t t = lane; t < n_it; t += 64) {
        const uint32_t lo = t * chunk;
        items[item_off[i] + t] = DevItem{j, lo, min(blocks, lo + chunk), 0u};
      }
      if (lane == 0) {
        DevCubeDesc d{};
        d.qid = so.qid;
        d.seq = seq_base + j;
        d.f_expect = so.f;
        d.nres_cap = so.nres;
        d.res_base = res_off[i];
        descs[j] = d;
        DevCubeOut o{};
        // a rebuilt fixpoint that disagrees with the expansion is a mismatch
        o.status = (f_total == uint32_t(so.f) && n_unsat == so.nres) ? 0 : 2;
        o.f = so.f;
        o.m = so.m;
        o.nres = int32_t(so.nres);
        o.first = ~0ull;
        louts[j] = o;
        leaf_src[j] = i;
      }
      tm.sync();
    }
  }
}

// After the leaf kernel: per-query counters from this step's leaves, and
// the fixpoint of the leaf that holds a query's witness key (DECIDE).
__global__ __launch_bounds__(kBlock) void split_capture_kernel(
    const DevCubeDesc* __restrict__ descs, const DevCubeOut* __restrict__ louts,
    const uint32_t* __restrict__ leaf_src, const uint32_t* __restrict__ fix_out,
    uint32_t* __restrict__ ctr, const unsigned long long* __restrict__ qkey,
    DevSplitStat* __restrict__ stats, uint32_t* __restrict__ wit, uint32_t nw_max, uint32_t mode) {
  const uint32_t n = ctr[kSpLeaves];
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    const DevCubeDesc d = descs[j];
    const DevCubeOut o = louts[j];
    if (o.status != 0) atomicOr(&ctr[kSpError], 2u);
    atomicAdd(&stats[d.qid].leaves, 1ull);
    atomicAdd(&stats[d.qid].blocks, (unsigned long long)o.blocks);
    atomicAdd(&stats[d.qid].clause_blocks, (unsigned long long)o.clause_blocks);
    atomicAdd(&stats[d.qid].word_ops, (unsigned long long)o.word_ops);
    if (mode == SCUBA_MODE_DECIDE) {
      const unsigned long long key = qkey[d.qid];
      if (key != ~0ull && uint32_t(key >> 38) == d.seq) {
        const uint32_t* fx = fix_out + size_t(leaf_src[j]) * 2 * nw_max;
        uint32_t* wq = wit + size_t(d.qid) * 2 * nw_max;
        for (uint32_t w = 0; w < 2 * nw_max; w++) wq[w] = fx[w];
      }
    }
  }
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

// Device scratch of the allocation-free decide entry point: one copy per
// GPU that the library runs on, held until the process ends.  Host code
// never uses this name as an address: dev_init looks up its device address
// once per device and every user takes that pointer.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

struct CnfLayout {
  size_t q, coff, lits, occ_off, occ, qkey, end;
};
CnfLayout cnf_layout(const CnfHost& c) {
  CnfLayout l;
  l.q = 0;
  l.coff = align256(l.q + c.q.size() * sizeof(DevQueryDesc));
  l.lits = align256(l.coff + c.n_coff * 4);
  // the witness keys, then the occurrence lists last: an upload for
  // host-fixpoint rounds only stops before them
  l.qkey = align256(l.lits + c.n_lits * 4);
  l.occ_off = align256(l.qkey + c.q.size() * 8);
  l.occ = align256(l.occ_off + c.n_occ_off * 4);
  l.end = align256(l.occ + c.n_occ * 4);
  return l;
}
struct RoundLayout {
  size_t head, cubes, groups, lits, items, outs, res, end;
};
RoundLayout round_layout(size_t base, size_t n_cubes, size_t n_lits, size_t n_items, uint64_t nres) {
  RoundLayout l;
  l.head = base;
  l.cubes = align256(l.head + 256);
  l.groups = align256(l.cubes + n_cubes * sizeof(DevCubeDesc));   // at most one group per cube
  l.lits = align256(l.groups + n_cubes * sizeof(uint2));
  l.items = align256(l.lits + n_lits * 4);
  l.outs = align256(l.items + n_items * sizeof(DevItem));
  l.res = align256(l.outs + n_cubes * sizeof(DevCubeOut));
  l.end = align256(l.res + (size_t(nres) + 4) * 32);   // + look-ahead of the leaf kernel
  return l;
}

struct SplitLayout {
  size_t order_off, order, ctr, stats, wit, nodes, node_fix, sout, fix_out, child_off, leaf_idx, res_off, item_off,
      descs, louts, leaf_src, items, res, end;
};
SplitLayout split_layout(size_t base, size_t nq, size_t n_order, const SplitRun& r) {
  const size_t B = r.batch, N = r.stack_cap, fw = 2 * size_t(r.nw_max) * 4;
  SplitLayout l;
  l.order_off = base;
  l.order = align256(l.order_off + nq * 8);
  l.ctr = align256(l.order + n_order * 4);
  l.stats = align256(l.ctr + 256);
  l.wit = align256(l.stats + nq * sizeof(DevSplitStat));
  l.nodes = align256(l.wit + nq * fw);
  l.node_fix = align256(l.nodes + N * sizeof(DevSplitNode));
  l.sout = align256(l.node_fix + N * fw);
  l.fix_out = align256(l.sout + B * sizeof(DevSplitOut));
  l.child_off = align256(l.fix_out + B * fw);
  l.leaf_idx = align256(l.child_off + B * 4);
  l.res_off = align256(l.leaf_idx + B * 4);
  l.item_off = align256(l.res_off + B * 4);
  l.descs = align256(l.item_off + B * 4);
  l.louts = align256(l.descs + B * sizeof(DevCubeDesc));
  l.leaf_src = align256(l.louts + B * sizeof(DevCubeOut));
  l.items = align256(l.leaf_src + B * 4);
  l.res = align256(l.items + B * kSplitItemsPerLeaf * sizeof(DevItem));
  l.end = align256(l.res + (B * size_t(r.nres_max) + 4) * 32);   // + look-ahead of the leaf kernel
  return l;
}
// dynamic LDS of the split kernels
size_t split_expand_lds(uint32_t nw_max) {
  return kUpWaves * (size_t(nw_max) * 4 + 2 * Team<1>::kQueue + 2 * Team<1>::kSize) * 4;
}
size_t split_scatter_lds(uint32_t nw_max) { return kUpWaves * (size_t(nw_max) * 4 + kFixList) * 4; }

}  // namespace

void score_stream_init(int device);

void dev_init(DeviceInfo* info, int device) {
  int n = 0;
  HIP_OK(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) fail(SCUBA_E_DEVICE, "no such HIP device");
  HIP_OK(hipSetDevice(device));
  hipDeviceProp_t p;
  HIP_OK(hipGetDeviceProperties(&p, device));
  info->device = device;
  info->cus = p.multiProcessorCount;
  score_stream_init(device);
  std::snprintf(info->arch, sizeof(info->arch), "%s", p.gcnArchName);
  {
    // the scratch array's address on this device, looked up once per
    // device with that device current
    static std::mutex mu;
    static std::map<int, void*> addr;
    std::lock_guard<std::mutex> g(mu);
    auto it = addr.find(device);
    if (it == addr.end()) {
      void* ptr = nullptr;
      HIP_OK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
      if (!ptr) fail(SCUBA_E_DEVICE, "no device address for the scratch array");
      it = addr.emplace(device, ptr).first;
    }
    info->scratch = it->second;
    info->scratch_bytes = kScratchBytes;
  }
  info->max_lds = p.sharedMemPerBlock;
  info->up_lds_max = info->max_lds;
  info->leaf_lds_max = info->max_lds;
  // the propagation kernel stages whole CNFs: let it use the opt-in LDS
  // size of the device when that is larger (160 KB per CU on gfx950)
  int optin = 0;
  if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, device) == hipSuccess &&
      size_t(optin) > info->max_lds) {
    const size_t want = size_t(optin) - 1024;   // static LDS of the kernel
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&up_kernel<1>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(want)) == hipSuccess &&
        hipFuncSetAttribute(reinterpret_cast<const void*>(&up_kernel<4>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(want)) == hipSuccess &&
        hipFuncSetAttribute(reinterpret_cast<const void*>(&fix_kernel<1>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(want)) == hipSuccess &&
        hipFuncSetAttribute(reinterpret_cast<const void*>(&fix_kernel<4>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(want)) == hipSuccess &&
        hipFuncSetAttribute(reinterpret_cast<const void*>(&fix_kernel<8>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(want)) == hipSuccess &&
        hipFuncSetAttribute(reinterpret_cast<const void*>(&split_expand_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(want)) == hipSuccess &&
        hipFuncSetAttribute(reinterpret_cast<const void*>(&split_scatter_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(want)) == hipSuccess)
      info->up_lds_max = want;
    else
      (void)hipGetLastError();
    // and the leaf kernel whose records are staged in LDS
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&leaf_kernel_v<true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(want)) == hipSuccess)
      info->leaf_lds_max = want;
    else
      (void)hipGetLastError();
  } else {
    (void)hipGetLastError();
  }
}

void dev_copy_h2d(void* dst, const void* src, size_t bytes, void* stream) {
  HIP_OK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, static_cast<hipStream_t>(stream)));
}
void dev_copy_d2h(void* dst, const void* src, size_t bytes, void* stream) {
  HIP_OK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, static_cast<hipStream_t>(stream)));
}
void dev_sync(void* stream) { HIP_OK(hipStreamSynchronize(static_cast<hipStream_t>(stream))); }

void* dev_pinned(size_t bytes) {
  void* p = nullptr;
  HIP_OK(hipHostMalloc(&p, bytes, hipHostMallocDefault));
  return p;
}
void dev_pinned_free(void* p) {
  if (p) (void)hipHostFree(p);
}

size_t dev_cnf_bytes(const CnfHost& cnf) { return cnf_layout(cnf).end; }
size_t dev_round_bytes(size_t n_cubes, size_t n_cube_lits, size_t n_items, uint64_t res_records) {
  return round_layout(0, n_cubes, n_cube_lits, n_items, res_records).end;
}

void dev_upload_cnf(const DeviceInfo& info, void* ws, size_t ws_bytes, const CnfHost& cnf, void* stream,
                    void* staging, size_t staging_bytes, bool wait, bool with_occ) {
  HIP_OK(hipSetDevice(info.device));
  CnfLayout l = cnf_layout(cnf);
  if (l.end > ws_bytes) fail(SCUBA_E_CAPACITY, "workspace too small for the CNF batch");
  if (l.end > staging_bytes) fail(SCUBA_E_INTERNAL, "staging too small");
  char* s = static_cast<char*>(staging);
  std::memcpy(s + l.q, cnf.q.data(), cnf.q.size() * sizeof(DevQueryDesc));
  uint32_t* coff = reinterpret_cast<uint32_t*>(s + l.coff);
  int32_t* lits = reinterpret_cast<int32_t*>(s + l.lits);
  uint32_t* occ_off = reinterpret_cast<uint32_t*>(s + l.occ_off);
  uint32_t* occ = reinterpret_cast<uint32_t*>(s + l.occ);
  // each query's arrays, written in place: clause offsets (query-relative),
  // literals, and its occurrence lists (literal index 2*v + (l < 0), clauses
  // in increasing order) by a counting sort
  parallel_for(cnf.q.size(), [&](size_t qi) {
    const CnfQuery& q = cnf.src->q[qi];
    const DevQueryDesc& d = cnf.q[qi];
    if (cnf.skip_root_unsat && q.root_unsat) return;   // an empty descriptor
    for (size_t c = 0; c < q.off.size(); c++) coff[d.coff_base + c] = uint32_t(q.off[c]);
    std::memcpy(lits + d.lit_base, q.lits.data(), q.lits.size() * 4);
    if (!with_occ) return;
    uint32_t* oo = occ_off + d.occ_off_base;
    const size_t nli = 2 * (size_t(q.n_vars) + 1);
    uint32_t* oc = occ + d.occ_base;
    if (q.has_occurrences()) {   // built with the CNF
      std::memcpy(oo, q.occ_off.data(), (nli + 1) * 4);
      std::memcpy(oc, q.occ.data(), q.occ.size() * 4);
      return;
    }
    std::memset(oo, 0, (nli + 1) * 4);
    for (int32_t x : q.lits) oo[2 * size_t(x > 0 ? x : -x) + (x < 0) + 1]++;
    for (size_t i = 0; i < nli; i++) oo[i + 1] += oo[i];
    std::vector<uint32_t> fill(oo, oo + nli);
    for (uint64_t c = 0; c < q.n_clauses(); c++)
      for (uint64_t i = q.off[c]; i < q.off[c + 1]; i++) {
        const int32_t x = q.lits[i];
        oc[fill[2 * size_t(x > 0 ? x : -x) + (x < 0)]++] = uint32_t(c);
      }
  });
  std::memset(s + l.qkey, 0xFF, cnf.q.size() * 8);
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_OK(hipMemcpyAsync(ws, s, with_occ ? l.end : l.occ_off, hipMemcpyHostToDevice, st));
  if (wait) HIP_OK(hipStreamSynchronize(st));
}

struct DevGraphs {
  int device = 0;
  hipStream_t stream = nullptr;
  hipEvent_t ready = nullptr;
  std::map<std::vector<uint64_t>, hipGraphExec_t> execs;
  std::list<std::vector<uint64_t>> lru;   // most recent first
  static constexpr size_t kMax = 64;
};

DevGraphs* dev_graphs_create(int device) {
  auto* g = new DevGraphs;
  g->device = device;
  return g;
}

void dev_graphs_destroy(DevGraphs* g) {
  if (!g) return;
  (void)hipSetDevice(g->device);
  for (auto& [k, e] : g->execs) (void)hipGraphExecDestroy(e);
  if (g->ready) (void)hipEventDestroy(g->ready);
  if (g->stream) (void)hipStreamDestroy(g->stream);
  delete g;
}

// One copy stream per device for the eager rounds' uploads (created on
// first use, kept for the process; default priority).
hipStream_t copy_stream(int device) {
  static std::mutex mu;
  static std::map<int, hipStream_t> streams;
  std::lock_guard<std::mutex> g(mu);
  auto it = streams.find(device);
  if (it != streams.end()) return it->second;
  hipStream_t cs;
  HIP_OK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  streams.emplace(device, cs);
  return cs;
}

// The learned scorer's stream and ordering event per device, created by
// dev_init (library set-up), so that taking the stream allocates nothing.
std::mutex score_mu;
std::map<int, std::pair<hipStream_t, hipEvent_t>> score_streams;

void score_stream_init(int device) {
  std::lock_guard<std::mutex> g(score_mu);
  if (score_streams.count(device)) return;
  hipStream_t ss;
  hipEvent_t ev;
  HIP_OK(hipStreamCreateWithFlags(&ss, hipStreamNonBlocking));
  HIP_OK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  score_streams.emplace(device, std::make_pair(ss, ev));
}

// The scoring stream, ordered after the work that `after` (the caller's
// stream) holds so far.  The scoring passes then wait for the caller's
// earlier work (the weights' sync) but not for what the call enqueues on
// `after` later: the CNF upload.
void* dev_score_stream(int device, void* after) {
  std::lock_guard<std::mutex> g(score_mu);
  auto it = score_streams.find(device);
  if (it == score_streams.end()) fail(SCUBA_E_INTERNAL, "scoring stream used before device set-up");
  HIP_OK(hipSetDevice(device));
  HIP_OK(hipEventRecord(it->second.second, static_cast<hipStream_t>(after)));
  HIP_OK(hipStreamWaitEvent(it->second.first, it->second.second, 0));
  return it->second.first;
}

// A kernel launch; with events, the events bracket the dispatch itself (so
// their interval is the kernel's execution), else a plain launch (the form
// that stream capture records).
template <typename K, typename... Args>
void launch(K kernel, dim3 grid, dim3 block, size_t lds, hipStream_t q, hipEvent_t start, hipEvent_t stop,
            Args... args) {
  if (start) hipExtLaunchKernelGGL(kernel, grid, block, uint32_t(lds), q, start, stop, 0u, args...);
  else hipLaunchKernelGGL(kernel, grid, block, lds, q, args...);
}

void dev_round_begin(const DeviceInfo& info, void* ws, size_t ws_bytes, const CnfHost& cnf, const RoundHost& rh,
                     uint32_t mode, uint32_t grid, void* stream, void* staging, size_t staging_bytes,
                     RoundTimes* times, DevGraphs* graphs, DevRoundPending* pend) {
  HIP_OK(hipSetDevice(info.device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  CnfLayout cl = cnf_layout(cnf);
  const size_t nc = rh.cubes.size(), ni = rh.items.size();
  RoundLayout rl = round_layout(cl.end, nc, rh.cube_lits.size(), ni, rh.res_records);
  if (rl.end > ws_bytes) fail(SCUBA_E_CAPACITY, "workspace too small for this round");
  const size_t up_bytes = rl.res - rl.head;
  if (up_bytes > staging_bytes || align256(nc * sizeof(DevCubeOut)) + cnf.q.size() * 8 > staging_bytes)
    fail(SCUBA_E_INTERNAL, "staging too small");
  // host-side checks of what the kernels assume
  // a round with at most one cube per CU, or whose queries mostly send one
  // cube (so that a workgroup of one-wave teams would hold one busy wave),
  // gives each cube a whole workgroup (team of four waves); other rounds
  // give each cube one wave and put up to four cubes of a query in a
  // workgroup, sharing its staged CNF
  uint32_t groups_of_four = 0;
  for (uint32_t i = 0; i < nc;) {
    uint32_t j = i + 1;
    while (j < nc && j - i < kUpWaves && rh.cubes[j].qid == rh.cubes[i].qid) j++;
    groups_of_four++;
    i = j;
  }
  const uint32_t tw_up = (nc <= uint32_t(info.cus) || 2 * groups_of_four > nc) ? 4 : 1;
  // every cube with the host's fixpoint: fix_kernel (one pass from HBM,
  // nothing staged); else up_kernel
  // (its loads take 32-bit byte offsets: clauses and literals below 2^30)
  uint32_t fix_only = nc ? 1u : 0u;
  for (const DevCubeDesc& c : rh.cubes) {
    if (!(c.n_lits & kCubeFixpoint)) fix_only = 0;
    if (c.qid < cnf.q.size() && (cnf.src->q[c.qid].lits.size() >= (size_t(1) << 30) ||
                                 cnf.src->q[c.qid].n_clauses() >= (uint64_t(1) << 30)))
      fix_only = 0;
  }
  if (nc && !fix_only && cnf.no_occ)
    fail(SCUBA_E_INTERNAL, "a propagation round needs occurrence lists that were not uploaded");
  // a fix launch whose largest CNF has kFixWideClauses clauses or more
  // gives each cube eight waves (one 512-thread workgroup)
  uint64_t max_clauses = 0;
  for (const DevCubeDesc& c : rh.cubes)
    if (c.qid < cnf.q.size()) max_clauses = std::max<uint64_t>(max_clauses, cnf.q[c.qid].n_clauses);
  const uint32_t tw = fix_only && max_clauses >= kFixWideClauses ? 8 : tw_up;
  const uint32_t teams = tw >= 8 ? 1 : kUpWaves / tw;
  const uint32_t block = tw >= 8 ? 64 * tw : kBlock;
  const size_t team_bytes = fix_only ? (size_t(rh.nw_max) * 6 + size_t(tw) * kFixList) * 4
                                     : size_t(rh.nw_max) * 4 * 4 + 2 * size_t(kUpQueue) * tw * 4 +
                                           2 * 64 * size_t(tw) * 4;
  const size_t up_lds = teams * team_bytes + (fix_only ? 0 : cnf.stage_bytes);
  // the LDS variant stages a work item's records when the round's largest
  // residual fits the kernel's LDS (else all items read from memory)
  uint32_t lds_records = 0;
  if (rh.leaf_variant == kLeafVectorLds) {
    const size_t cap = (info.leaf_lds_max - 64) / 32;
    lds_records = uint32_t(std::min<size_t>(rh.tile_max, cap));
  }
  const size_t leaf_lds = size_t(lds_records) * 32;
  if (rh.leaf_variant > kLeafVectorLds) fail(SCUBA_E_INTERNAL, "unknown leaf variant");
  if (up_lds > info.up_lds_max) fail(SCUBA_E_CAPACITY, "query too large for the propagation kernel's LDS");

  for (const DevCubeDesc& c : rh.cubes) {
    const bool fix = c.n_lits & kCubeFixpoint;
    const uint32_t n = c.n_lits & ~kCubeFixpoint;
    if (fix && c.qid < cnf.q.size() && n != 2 * ((cnf.q[c.qid].n_vars >> 5) + 1))
      fail(SCUBA_E_INTERNAL, "cube fixpoint of the wrong size");
    if (c.qid >= cnf.q.size() || uint64_t(c.lit_off) + n > rh.cube_lits.size() ||
        c.res_base + c.nres_cap > rh.res_records || c.nres_cap > rh.tile_max ||
        (cnf.q[c.qid].n_vars >> 5) + 1 > rh.nw_max ||
        (cnf.skip_root_unsat && cnf.src->q[c.qid].root_unsat))
      fail(SCUBA_E_INTERNAL, "cube descriptor out of range");
  }
  for (const DevItem& it : rh.items)
    if (it.cube >= nc || it.it_lo >= it.it_hi) fail(SCUBA_E_INTERNAL, "work item out of range");

  char* s = static_cast<char*>(staging);
  const size_t b = rl.head;
  std::memset(s + (rl.head - b), 0, 256);
  std::memcpy(s + (rl.cubes - b), rh.cubes.data(), nc * sizeof(DevCubeDesc));
  // groups of up to kUpWaves consecutive cubes of one query, the largest
  // CNFs first: a group's time grows with its query's clauses and literals,
  // and workgroups take groups in this order, so the long ones do not start
  // last
  uint32_t n_groups = 0;
  {
    uint2* gp = reinterpret_cast<uint2*>(s + (rl.groups - b));
    for (uint32_t i = 0; i < nc;) {
      uint32_t j = i + 1;
      while (j < nc && j - i < teams && rh.cubes[j].qid == rh.cubes[i].qid) j++;
      gp[n_groups++] = make_uint2(i, j - i);
      i = j;
    }
    auto size_of = [&](const uint2& g) {
      const CnfQuery& q = cnf.src->q[rh.cubes[g.x].qid];
      return q.lits.size() + q.off.size();
    };
    std::stable_sort(gp, gp + n_groups, [&](const uint2& x, const uint2& y) { return size_of(x) > size_of(y); });
  }
  std::memcpy(s + (rl.lits - b), rh.cube_lits.data(), rh.cube_lits.size() * 4);
  std::memcpy(s + (rl.items - b), rh.items.data(), ni * sizeof(DevItem));
  DevCubeOut init{};
  init.first = ~0ull;
  for (size_t i = 0; i < nc; i++) std::memcpy(s + (rl.outs - b) + i * sizeof(DevCubeOut), &init, sizeof(init));

  char* w = static_cast<char*>(ws);
  const uint32_t g = grid ? grid : uint32_t(info.cus) * 8;
  const uint32_t gu = n_groups ? std::min<uint32_t>(g, n_groups) : 0;
  const uint32_t gl = ni ? std::min<uint32_t>(g, uint32_t(ni)) : 0;
  // the whole round as one stream sequence: upload (the zeroed head and the
  // initial outputs included, so no memset), kernels, download
  // eager rounds time the two kernels with events that bracket their
  // dispatches (ev[2..3] and ev[4..5]); ev[0..1] and ev[6..7] bracket the
  // copies
  // The eager form uploads on the device's copy stream (ordered after the
  // caller's work by ev[8]) and makes q wait for it, so that the upload's
  // completion is not inside the first kernel's events.
  auto enqueue = [&](hipStream_t q, hipEvent_t* ev) {
    if (ev) {
      hipStream_t cs = copy_stream(info.device);
      HIP_OK(hipEventRecord(ev[8], q));
      HIP_OK(hipStreamWaitEvent(cs, ev[8], 0));
      HIP_OK(hipEventRecord(ev[0], cs));
      HIP_OK(hipMemcpyAsync(w + rl.head, s, up_bytes, hipMemcpyHostToDevice, cs));
      HIP_OK(hipEventRecord(ev[1], cs));
      HIP_OK(hipStreamWaitEvent(q, ev[1], 0));
    } else {
      HIP_OK(hipMemcpyAsync(w + rl.head, s, up_bytes, hipMemcpyHostToDevice, q));
    }
    if (gu && fix_only) {
      launch(tw == 8 ? fix_kernel<8> : tw == 4 ? fix_kernel<4> : fix_kernel<1>, dim3(gu), dim3(block), up_lds,
             q, ev ? ev[2] : nullptr,
             ev ? ev[3] : nullptr, reinterpret_cast<const DevQueryDesc*>(w + cl.q),
             reinterpret_cast<const uint32_t*>(w + cl.coff), reinterpret_cast<const int32_t*>(w + cl.lits),
             reinterpret_cast<const DevCubeDesc*>(w + rl.cubes), reinterpret_cast<const int32_t*>(w + rl.lits),
             reinterpret_cast<const uint2*>(w + rl.groups), n_groups, reinterpret_cast<DevCubeOut*>(w + rl.outs),
             reinterpret_cast<uint4*>(w + rl.res), reinterpret_cast<uint32_t*>(w + rl.head), rh.nw_max);
      HIP_OK(hipGetLastError());
    } else if (gu) {
      launch(tw == 4 ? up_kernel<4> : up_kernel<1>, dim3(gu), dim3(kBlock), up_lds, q,
                            ev ? ev[2] : nullptr, ev ? ev[3] : nullptr,
                            reinterpret_cast<const DevQueryDesc*>(w + cl.q),
                            reinterpret_cast<const uint32_t*>(w + cl.coff),
                            reinterpret_cast<const int32_t*>(w + cl.lits),
                            reinterpret_cast<const uint32_t*>(w + cl.occ_off),
                            reinterpret_cast<const uint32_t*>(w + cl.occ),
                            reinterpret_cast<const DevCubeDesc*>(w + rl.cubes),
                            reinterpret_cast<const int32_t*>(w + rl.lits),
                            reinterpret_cast<const uint2*>(w + rl.groups), n_groups,
                            reinterpret_cast<DevCubeOut*>(w + rl.outs), reinterpret_cast<uint4*>(w + rl.res),
                            reinterpret_cast<uint32_t*>(w + rl.head), rh.nw_max);
      HIP_OK(hipGetLastError());
    }
    if (gl) {
      const auto* items = reinterpret_cast<const DevItem*>(w + rl.items);
      const auto* cubes = reinterpret_cast<const DevCubeDesc*>(w + rl.cubes);
      auto* outs_d = reinterpret_cast<DevCubeOut*>(w + rl.outs);
      const auto* res = reinterpret_cast<const uint4*>(w + rl.res);
      auto* qkey = reinterpret_cast<unsigned long long*>(w + cl.qkey);
      auto* head = reinterpret_cast<uint32_t*>(w + rl.head);
      hipEvent_t e0 = ev ? ev[4] : nullptr, e1 = ev ? ev[5] : nullptr;
      if (rh.leaf_variant == kLeafScalar)
        launch(leaf_kernel, dim3(gl), dim3(kBlock), leaf_lds, q, e0, e1, items, uint32_t(ni), cubes, outs_d, res,
               qkey, head, mode, (const uint32_t*)nullptr);
      else if (rh.leaf_variant == kLeafVector)
        launch(leaf_kernel_v<false>, dim3(gl), dim3(kBlock), leaf_lds, q, e0, e1, items, uint32_t(ni), cubes,
               outs_d, res, qkey, head, mode, (const uint32_t*)nullptr, 0u);
      else
        launch(leaf_kernel_v<true>, dim3(gl), dim3(kBlock), leaf_lds, q, e0, e1, items, uint32_t(ni), cubes,
               outs_d, res, qkey, head, mode, (const uint32_t*)nullptr, lds_records);
      HIP_OK(hipGetLastError());
    }
    if (ev) HIP_OK(hipEventRecord(ev[6], q));
    HIP_OK(hipMemcpyAsync(s, w + rl.outs, nc * sizeof(DevCubeOut), hipMemcpyDeviceToHost, q));
    HIP_OK(hipMemcpyAsync(s + align256(nc * sizeof(DevCubeOut)), w + cl.qkey, cnf.q.size() * 8,
                          hipMemcpyDeviceToHost, q));
    if (ev) HIP_OK(hipEventRecord(ev[7], q));
  };

  times->cubes += nc;
  times->items += ni;
  if (pend->active) fail(SCUBA_E_INTERNAL, "a round is already in flight");
  hipEvent_t* ev = reinterpret_cast<hipEvent_t*>(pend->ev);
  pend->active = true;   // (release destroys whichever events exist)
  pend->sync_stream = st;
  for (int i = 0; i < 9; i++) HIP_OK(hipEventCreate(&ev[i]));
  pend->device = info.device;
  pend->gu = gu;
  pend->gl = gl;
  pend->fix_only = fix_only;
  pend->nc = nc;
  pend->nq = cnf.q.size();
  pend->staging = staging;
  if (!graphs) {
    enqueue(st, ev);
    pend->graph = false;
    pend->sync_stream = st;
  } else {
    if (!graphs->stream) {
      HIP_OK(hipStreamCreateWithFlags(&graphs->stream, hipStreamNonBlocking));
      HIP_OK(hipEventCreateWithFlags(&graphs->ready, hipEventDisableTiming));
    }
    hipStream_t gs = graphs->stream;
    // every value the captured kernels and copies bake in: pointers, the
    // offsets of both layouts, sizes, group count and launch shapes
    std::vector<uint64_t> key = {uint64_t(uintptr_t(ws)), uint64_t(uintptr_t(staging)),
                                 cl.q, cl.coff, cl.lits, cl.occ_off, cl.occ, cl.qkey, cl.end,
                                 rl.head, rl.cubes, rl.groups, rl.lits, rl.items, rl.outs, rl.res, rl.end,
                                 up_bytes, nc, rh.cube_lits.size(), ni, rh.res_records, cnf.q.size(), n_groups,
                                 mode, gu, gl, rh.nw_max, up_lds, leaf_lds, uint64_t(info.device), tw,
                                 fix_only, rh.leaf_variant, lds_records};
    auto it = graphs->execs.find(key);
    if (it == graphs->execs.end()) {
      hipGraph_t graph;
      HIP_OK(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
      enqueue(gs, nullptr);
      HIP_OK(hipStreamEndCapture(gs, &graph));
      hipGraphExec_t exec;
      hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      HIP_OK(e);
      if (graphs->execs.size() >= DevGraphs::kMax) {
        auto old = graphs->execs.find(graphs->lru.back());
        (void)hipGraphExecDestroy(old->second);
        graphs->execs.erase(old);
        graphs->lru.pop_back();
      }
      it = graphs->execs.emplace(key, exec).first;
      graphs->lru.push_front(key);
      times->graph_captures++;
    } else {
      graphs->lru.remove(key);
      graphs->lru.push_front(key);
    }
    // ordered after the caller's work on its stream
    HIP_OK(hipEventRecord(graphs->ready, st));
    HIP_OK(hipStreamWaitEvent(gs, graphs->ready, 0));
    HIP_OK(hipEventRecord(ev[0], gs));
    HIP_OK(hipGraphLaunch(it->second, gs));
    HIP_OK(hipEventRecord(ev[1], gs));
    pend->graph = true;
    pend->sync_stream = gs;
  }
}

void dev_round_end(DevRoundPending* pend, std::vector<DevCubeOut>* outs, std::vector<uint64_t>* qkeys,
                   RoundTimes* times) {
  if (!pend->active) fail(SCUBA_E_INTERNAL, "no round in flight");
  HIP_OK(hipSetDevice(pend->device));
  hipEvent_t* ev = reinterpret_cast<hipEvent_t*>(pend->ev);
  HIP_OK(hipStreamSynchronize(static_cast<hipStream_t>(pend->sync_stream)));
  float ms;
  if (!pend->graph) {
    HIP_OK(hipEventElapsedTime(&ms, ev[0], ev[1])); times->h2d_ms += ms;
    if (pend->gu) { HIP_OK(hipEventElapsedTime(&ms, ev[2], ev[3])); times->up_ms += ms; }
    if (pend->gl) { HIP_OK(hipEventElapsedTime(&ms, ev[4], ev[5])); times->leaf_ms += ms; }
    HIP_OK(hipEventElapsedTime(&ms, ev[6], ev[7])); times->d2h_ms += ms;
    times->up_launches += pend->gu != 0;
    times->fix_launches += pend->gu != 0 && pend->fix_only;
    times->leaf_launches += pend->gl != 0;
  } else {
    HIP_OK(hipEventElapsedTime(&ms, ev[0], ev[1]));
    times->graph_ms += ms;
    times->graph_launches++;
  }
  const char* s = static_cast<const char*>(pend->staging);
  outs->resize(pend->nc);
  std::memcpy(outs->data(), s, pend->nc * sizeof(DevCubeOut));
  qkeys->resize(pend->nq);
  std::memcpy(qkeys->data(), s + align256(pend->nc * sizeof(DevCubeOut)), pend->nq * 8);
  dev_round_release(pend);
}

void dev_round_release(DevRoundPending* pend) {
  if (!pend->active) return;
  pend->active = false;
  (void)hipSetDevice(pend->device);
  (void)hipStreamSynchronize(static_cast<hipStream_t>(pend->sync_stream));
  for (int i = 0; i < 9; i++)
    if (pend->ev[i]) (void)hipEventDestroy(static_cast<hipEvent_t>(pend->ev[i]));
  for (auto& e : pend->ev) e = nullptr;
}

DevRoundPending::~DevRoundPending() { dev_round_release(this); }

void dev_round(const DeviceInfo& info, void* ws, size_t ws_bytes, const CnfHost& cnf, const RoundHost& rh,
               uint32_t mode, uint32_t grid, void* stream, void* staging, size_t staging_bytes,
               std::vector<DevCubeOut>* outs, std::vector<uint64_t>* qkeys, RoundTimes* times,
               DevGraphs* graphs) {
  DevRoundPending pend;
  dev_round_begin(info, ws, ws_bytes, cnf, rh, mode, grid, stream, staging, staging_bytes, times, graphs, &pend);
  dev_round_end(&pend, outs, qkeys, times);
}

size_t dev_split_node_bytes(uint32_t nw_max) { return sizeof(DevSplitNode) + 2 * size_t(nw_max) * 4; }

size_t dev_split_bytes(const CnfHost& cnf, size_t n_order, const SplitRun& r) {
  const CnfLayout cl = cnf_layout(cnf);
  return split_layout(cl.end, cnf.q.size(), n_order, r).end;
}

void dev_split(const DeviceInfo& info, void* ws, size_t ws_bytes, const CnfHost& cnf,
               const std::vector<uint64_t>& order_off, const std::vector<uint32_t>& order,
               const std::vector<uint32_t>& start, const SplitRun& r, void* stream, void* staging,
               size_t staging_bytes, SplitOutput* out) {
  HIP_OK(hipSetDevice(info.device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t nq = cnf.q.size();
  const CnfLayout cl = cnf_layout(cnf);
  const SplitLayout sl = split_layout(cl.end, nq, order.size(), r);
  if (sl.end > ws_bytes) fail(SCUBA_E_CAPACITY, "workspace too small for the device split");
  // host-side checks of what the kernels assume
  if (r.batch == 0 || r.batch > (1u << 20) || r.stack_cap < 2 * size_t(r.batch))
    fail(SCUBA_E_INTERNAL, "device split batch or stack out of range");
  if (start.size() > r.stack_cap) fail(SCUBA_E_CAPACITY, "more start nodes than the device split stack holds");
  if (order_off.size() != nq) fail(SCUBA_E_INTERNAL, "branch orders do not match the batch");
  for (uint32_t q : start) {
    if (q >= nq || (cnf.skip_root_unsat && cnf.src->q[q].root_unsat)) fail(SCUBA_E_INTERNAL, "start node out of range");
    if ((cnf.q[q].n_vars >> 5) + 1 > r.nw_max) fail(SCUBA_E_INTERNAL, "query wider than the split bitmaps");
    if (order_off[q] + cnf.q[q].n_vars > order.size()) fail(SCUBA_E_INTERNAL, "branch order out of range");
    if (cnf.q[q].n_clauses > r.nres_max && r.max_res > r.nres_max)
      fail(SCUBA_E_INTERNAL, "residual bound below a query's clause count");
    // the clause pass of wide queries takes 32-bit byte offsets
    if (cnf.src->q[q].lits.size() >= (size_t(1) << 30) || cnf.q[q].n_clauses >= (uint32_t(1) << 30))
      fail(SCUBA_E_CAPACITY, "a query of 2^30 or more clauses or literals for the device split");
  }
  if (r.k > kMaxLeafVars || r.chunk_log2 > 26) fail(SCUBA_E_INTERNAL, "split options out of range");
  const size_t e_lds = split_expand_lds(r.nw_max), s_lds = split_scatter_lds(r.nw_max);
  if (e_lds > info.up_lds_max || s_lds > info.up_lds_max)
    fail(SCUBA_E_CAPACITY, "query too large for the device split's LDS");
  const size_t B = r.batch;
  const size_t up_b = sl.nodes + start.size() * sizeof(DevSplitNode) - sl.order_off;
  const size_t fin_b = align256(nq * 8) + align256(nq * sizeof(DevSplitStat)) + nq * 2 * size_t(r.nw_max) * 4;
  const size_t cnt_b = align256(B * sizeof(DevCubeDesc)) + B * sizeof(DevCubeOut);
  if (std::max({up_b, fin_b, cnt_b, size_t(256)}) > staging_bytes) fail(SCUBA_E_INTERNAL, "staging too small");

  char* s = static_cast<char*>(staging);
  std::memset(s, 0, up_b);   // counters, statistics and witness fixpoints start at 0
  std::memcpy(s + (sl.order_off - sl.order_off), order_off.data(), nq * 8);
  std::memcpy(s + (sl.order - sl.order_off), order.data(), order.size() * 4);
  DevSplitNode* sn = reinterpret_cast<DevSplitNode*>(s + (sl.nodes - sl.order_off));
  for (size_t i = 0; i < start.size(); i++) sn[i] = DevSplitNode{start[i], 0, 0u, 0u};
  char* w = static_cast<char*>(ws);
  HIP_OK(hipMemcpyAsync(w + sl.order_off, s, up_b, hipMemcpyHostToDevice, st));
  HIP_OK(hipStreamSynchronize(st));   // the staging buffer is reused below

  const auto* qd = reinterpret_cast<const DevQueryDesc*>(w + cl.q);
  const auto* coff = reinterpret_cast<const uint32_t*>(w + cl.coff);
  const auto* lits = reinterpret_cast<const int32_t*>(w + cl.lits);
  const auto* occ_off = reinterpret_cast<const uint32_t*>(w + cl.occ_off);
  const auto* occ = reinterpret_cast<const uint32_t*>(w + cl.occ);
  auto* qkey = reinterpret_cast<unsigned long long*>(w + cl.qkey);
  auto* ctr = reinterpret_cast<uint32_t*>(w + sl.ctr);
  auto* stats = reinterpret_cast<DevSplitStat*>(w + sl.stats);
  auto* nodes = reinterpret_cast<DevSplitNode*>(w + sl.nodes);
  auto* node_fix = reinterpret_cast<uint32_t*>(w + sl.node_fix);
  auto* sout = reinterpret_cast<DevSplitOut*>(w + sl.sout);
  auto* fix_out = reinterpret_cast<uint32_t*>(w + sl.fix_out);
  auto* descs = reinterpret_cast<DevCubeDesc*>(w + sl.descs);
  auto* louts = reinterpret_cast<DevCubeOut*>(w + sl.louts);
  const uint32_t g = r.grid ? r.grid : uint32_t(info.cus) * 8;
  hipEvent_t ev[4];
  for (auto& e : ev) HIP_OK(hipEventCreate(&e));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() { for (int i = 0; i < 4; i++) (void)hipEventDestroy(e[i]); }
  } eg{ev};
  if (r.mode == SCUBA_MODE_COUNT) out->leaves.assign(nq, {});
  // Steps pop at most the headroom above a reserve of (largest variable
  // count + 2) nodes; within the reserve they pop one node.  A one-node step
  // is depth-first: the nodes it leaves above the current stack are at most
  // one per decision of the current path, and a path decides at most every
  // variable once, so the stack never exceeds its capacity.
  uint64_t reserve = 2;
  for (uint32_t q : start) reserve = std::max<uint64_t>(reserve, uint64_t(cnf.q[q].n_vars) + 2);
  if (r.stack_cap < start.size() + reserve)
    fail(SCUBA_E_CAPACITY, "device split stack smaller than the start nodes and one depth-first path");
  uint64_t top = start.size(), seq_base = 0;
  while (top > 0) {
    const uint64_t head = r.stack_cap - top;
    uint64_t b = std::min<uint64_t>({uint64_t(B), top, head > reserve ? head - reserve : 1});
    if (top + b > r.stack_cap) fail(SCUBA_E_INTERNAL, "device split stack bound broken");
    const uint64_t first = top - b;
    const uint32_t gw = uint32_t(std::min<uint64_t>(g, (b + kUpWaves - 1) / kUpWaves));
    launch(split_expand_kernel, dim3(gw), dim3(kBlock), e_lds, st, ev[0], ev[1], qd, coff, lits, occ_off, occ,
           reinterpret_cast<const unsigned long long*>(w + sl.order_off),
           reinterpret_cast<const uint32_t*>(w + sl.order), (const DevSplitNode*)nodes, (const uint32_t*)node_fix,
           uint32_t(first), uint32_t(b), (const int32_t*)nullptr, (const unsigned long long*)qkey, stats, sout,
           fix_out, ctr, r.nw_max, r.k, r.max_res, (unsigned long long)r.max_cubes);
    HIP_OK(hipGetLastError());
    launch(split_scan_kernel, dim3(1), dim3(1024), 0, st, nullptr, nullptr, (const DevSplitOut*)sout, uint32_t(b),
           r.chunk_log2, reinterpret_cast<uint32_t*>(w + sl.child_off), reinterpret_cast<uint32_t*>(w + sl.leaf_idx),
           reinterpret_cast<uint32_t*>(w + sl.res_off), reinterpret_cast<uint32_t*>(w + sl.item_off), ctr);
    HIP_OK(hipGetLastError());
    launch(split_scatter_kernel, dim3(gw), dim3(kBlock), s_lds, st, nullptr, nullptr, qd, coff, lits,
           (const DevSplitOut*)sout, (const uint32_t*)fix_out, uint32_t(first), uint32_t(b),
           reinterpret_cast<const uint32_t*>(w + sl.child_off), reinterpret_cast<const uint32_t*>(w + sl.leaf_idx),
           reinterpret_cast<const uint32_t*>(w + sl.res_off), reinterpret_cast<const uint32_t*>(w + sl.item_off),
           nodes, node_fix, descs, louts, reinterpret_cast<uint32_t*>(w + sl.leaf_src),
           reinterpret_cast<DevItem*>(w + sl.items), reinterpret_cast<uint4*>(w + sl.res), uint32_t(seq_base),
           r.nw_max, r.chunk_log2, (const uint32_t*)ctr);
    HIP_OK(hipGetLastError());
    if (r.leaf_variant == kLeafScalar)
      launch(leaf_kernel, dim3(g), dim3(kBlock), 0, st, ev[2], ev[3], reinterpret_cast<const DevItem*>(w + sl.items),
             0u, (const DevCubeDesc*)descs, louts, reinterpret_cast<const uint4*>(w + sl.res), qkey,
             ctr + kSpLeafHead, r.mode, (const uint32_t*)(ctr + kSpItems));
    else
      launch(leaf_kernel_v<false>, dim3(g), dim3(kBlock), 0, st, ev[2], ev[3],
             reinterpret_cast<const DevItem*>(w + sl.items), 0u, (const DevCubeDesc*)descs, louts,
             reinterpret_cast<const uint4*>(w + sl.res), qkey, ctr + kSpLeafHead, r.mode,
             (const uint32_t*)(ctr + kSpItems), 0u);
    HIP_OK(hipGetLastError());
    launch(split_capture_kernel, dim3(std::min<uint64_t>(g, (b + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
           nullptr, nullptr, (const DevCubeDesc*)descs, (const DevCubeOut*)louts,
           reinterpret_cast<const uint32_t*>(w + sl.leaf_src), (const uint32_t*)fix_out, ctr,
           (const unsigned long long*)qkey, stats, reinterpret_cast<uint32_t*>(w + sl.wit), r.nw_max, r.mode);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(s, ctr, 256, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    uint32_t c[64];
    std::memcpy(c, s, 256);
    if (c[kSpError] & 1) fail(SCUBA_E_DEVICE, "device split: propagation error");
    if (c[kSpError] & 2) fail(SCUBA_E_DEVICE, "device split: a leaf's rebuilt fixpoint disagrees with its expansion");
    if (c[kSpChildren] > 2 * b || c[kSpLeaves] > b) fail(SCUBA_E_DEVICE, "device split: step totals out of range");
    float ms;
    HIP_OK(hipEventElapsedTime(&ms, ev[0], ev[1]));
    out->expand_ms += ms;
    HIP_OK(hipEventElapsedTime(&ms, ev[2], ev[3]));
    out->leaf_ms += ms;
    if (r.mode == SCUBA_MODE_COUNT && c[kSpLeaves]) {
      const size_t nl = c[kSpLeaves];
      HIP_OK(hipMemcpyAsync(s, descs, nl * sizeof(DevCubeDesc), hipMemcpyDeviceToHost, st));
      HIP_OK(hipMemcpyAsync(s + align256(B * sizeof(DevCubeDesc)), louts, nl * sizeof(DevCubeOut),
                            hipMemcpyDeviceToHost, st));
      HIP_OK(hipStreamSynchronize(st));
      const DevCubeDesc* dh = reinterpret_cast<const DevCubeDesc*>(s);
      const DevCubeOut* oh = reinterpret_cast<const DevCubeOut*>(s + align256(B * sizeof(DevCubeDesc)));
      for (size_t j = 0; j < nl; j++) out->leaves[dh[j].qid].push_back(oh[j]);
    }
    top = first + c[kSpChildren];
    seq_base += c[kSpLeaves];
    out->steps++;
    out->nodes += b;
    out->max_stack = std::max<uint64_t>(out->max_stack, top);
    // the witness key holds leaf sequence numbers below 2^26
    if (top > 0 && seq_base + B >= (uint64_t(1) << 26)) {
      out->stopped = true;
      break;
    }
  }
  HIP_OK(hipMemcpyAsync(s, qkey, nq * 8, hipMemcpyDeviceToHost, st));
  HIP_OK(hipMemcpyAsync(s + align256(nq * 8), stats, nq * sizeof(DevSplitStat), hipMemcpyDeviceToHost, st));
  HIP_OK(hipMemcpyAsync(s + align256(nq * 8) + align256(nq * sizeof(DevSplitStat)), w + sl.wit,
                        nq * 2 * size_t(r.nw_max) * 4, hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  out->qkeys.resize(nq);
  std::memcpy(out->qkeys.data(), s, nq * 8);
  out->stats.resize(nq);
  std::memcpy(out->stats.data(), s + align256(nq * 8), nq * sizeof(DevSplitStat));
  out->wit.resize(nq * 2 * size_t(r.nw_max));
  std::memcpy(out->wit.data(), s + align256(nq * 8) + align256(nq * sizeof(DevSplitStat)),
              out->wit.size() * 4);
}

size_t dev_split_staging(const CnfHost& cnf, size_t n_order, size_t n_start, const SplitRun& r) {
  const size_t nq = cnf.q.size();
  const SplitLayout sl = split_layout(0, nq, n_order, r);
  const size_t up_b = sl.nodes + n_start * sizeof(DevSplitNode);
  const size_t fin_b = align256(nq * 8) + align256(nq * sizeof(DevSplitStat)) + nq * 2 * size_t(r.nw_max) * 4;
  const size_t cnt_b = align256(size_t(r.batch) * sizeof(DevCubeDesc)) + size_t(r.batch) * sizeof(DevCubeOut);
  return std::max({up_b, fin_b, cnt_b, size_t(256)});
}

}  // namespace scuba
