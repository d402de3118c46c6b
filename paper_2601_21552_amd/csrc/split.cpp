// Host unit propagation (eager clause counters with a trail and reasons)
// and the resumable depth-first cube splitter with backjumping.
#include "split.hpp"

#include <algorithm>
#include <cmath>

namespace scuba {

Splitter::Splitter(const CnfQuery& q, uint32_t k, uint32_t max_residual, uint64_t max_cubes)
    : q_(q), k_(k), max_res_(max_residual), max_cubes_(max_cubes), n_(q.n_vars) {
  if (q_.lits.size() >= (uint64_t(1) << 32)) throw Error(SCUBA_E_CAPACITY, "query with 2^32 or more literals");
  coff_.assign(q_.off.begin(), q_.off.end());   // 32-bit clause offsets for the propagation loops
  if (q_.has_occurrences()) {
    occ_off_ = q_.occ_off.data();
    occ_ = q_.occ.data();
  } else {   // built here for a query that has none
    CnfQuery tmp;
    tmp.n_vars = q_.n_vars;
    tmp.off = q_.off;
    tmp.lits = q_.lits;
    tmp.build_occurrences();
    own_occ_off_ = std::move(tmp.occ_off);
    own_occ_ = std::move(tmp.occ);
    occ_off_ = own_occ_off_.data();
    occ_ = own_occ_.data();
  }
  // static order: literal occurrences in the original CNF, most first,
  // ties to the lowest variable (a counting sort by occurrences; variables
  // enter their bucket in increasing order)
  occurrences_.assign(size_t(n_) + 1, 0);
  uint32_t most = 0;
  for (uint32_t v = 1; v <= n_; v++) {
    occurrences_[v] = occ_off_[2 * v + 2] - occ_off_[2 * v];
    most = std::max(most, occurrences_[v]);
  }
  std::vector<uint32_t> start(size_t(most) + 2, 0);
  for (uint32_t v = 1; v <= n_; v++) start[most - occurrences_[v] + 1]++;
  for (size_t i = 1; i < start.size(); i++) start[i] += start[i - 1];
  order_.resize(n_);
  for (uint32_t v = 1; v <= n_; v++) order_[start[most - occurrences_[v]]++] = int32_t(v);
  static_rank_.assign(size_t(n_) + 1, 0);
  for (uint32_t i = 0; i < n_; i++) static_rank_[order_[i]] = i;
  // clause counts per variable at the root (copied by every reset); a clause
  // holds a variable at most once, so this is the occurrence count
  act_init_ = occurrences_;
  f_init_ = 0;
  for (uint32_t v = 1; v <= n_; v++) f_init_ += act_init_[v] > 0;
  bit_pos_.assign(size_t(n_) + 1, 0);
  bit_width_.assign(size_t(n_) + 1, 0);
  for (size_t i = 0; i < q_.in_first.size(); i++)
    for (uint32_t b = 0; b < q_.in_width[i]; b++) {
      bit_pos_[q_.in_first[i] + b] = b;
      bit_width_[q_.in_first[i] + b] = q_.in_width[i];
    }
}

void Splitter::set_word_order() {
  word_ = true;
  word_order_.clear();
  // inputs that a root equality defines from the others come last: once
  // the others are fixed, propagation through the equality fixes them
  std::vector<uint8_t> defined(size_t(n_) + 1, 0);
  for (size_t i = 0; i < q_.in_first.size(); i++) {
    const bool d = i < q_.in_defined.size() && q_.in_defined[i];
    for (uint32_t b = 0; b < q_.in_width[i]; b++) defined[q_.in_first[i] + b] = d;
  }
  for (uint32_t v = 1; v <= n_; v++)
    if (bit_width_[v]) word_order_.push_back(int32_t(v));
  std::stable_sort(word_order_.begin(), word_order_.end(), [&](int32_t a, int32_t b) {
    if (defined[a] != defined[b]) return defined[a] < defined[b];
    return bit_pos_[a] > bit_pos_[b];
  });
}

void Splitter::set_learned(uint32_t candidates, uint32_t rescore) {
  learned_ = true;
  words_first_ = true;
  n_cands_ = std::max<uint32_t>(candidates, 1);
  rescore_ = std::max<uint32_t>(rescore, 1);
}

void Splitter::set_trace(uint32_t candidates, uint32_t every, uint32_t depth) {
  trace_ = true;
  n_cands_ = std::max<uint32_t>(candidates, 1);
  trace_every_ = std::max<uint32_t>(every, 1);
  trace_depth_ = depth;
}

// The first m active variables of the static order and the input words'
// top bits; with words_first_, the words alone while one of them is open.
std::vector<int32_t> Splitter::candidates(uint32_t m, std::set<int32_t>* words) const {
  std::vector<int32_t> c;
  // the most significant active bit of each input word (these stand for
  // their words, see choose_learned); with words_first_ and an input bit
  // active, the words are the only candidates
  auto word_tops = [&](size_t n_static) {
    if (words) words->clear();
    for (size_t i = 0; i < q_.in_first.size(); i++)
      for (uint32_t b = q_.in_width[i]; b-- > 0;) {
        const int32_t v = int32_t(q_.in_first[i] + b);
        if (assign_[v] >= 0 || act_cnt_[v] == 0) continue;
        if (std::find(c.begin(), c.begin() + n_static, v) == c.begin() + n_static) {
          c.push_back(v);
          if (words) words->insert(v);
        }
        break;
      }
  };
  if (words_first_) {
    word_tops(0);
    if (!c.empty()) return c;
  }
  for (int32_t v : order_) {
    if (c.size() >= m) break;
    if (assign_[v] < 0 && act_cnt_[v] > 0) c.push_back(v);
  }
  word_tops(c.size());
  return c;
}

// Features of each candidate at the current node (kFeatures per variable):
// positive / negative occurrences in unsatisfied clauses, occurrences in
// unsatisfied clauses with 2, 3 and more open literals, the Jeroslow-Wang
// weight (sum of 2^-open), static occurrences, input-bit flag and relative
// bit position, the node's active count, unsatisfied-clause fraction and
// depth, log occurrences, neighbour count, static rank, and a constant.
void Splitter::features(const std::vector<int32_t>& cands, std::vector<float>* out) const {
  out->assign(cands.size() * kFeatures, 0.f);
  const float nc = float(std::max<uint64_t>(q_.n_clauses(), 1));
  for (size_t r = 0; r < cands.size(); r++) {
    const int32_t v = cands[r];
    float pos = 0, neg = 0, bin = 0, ter = 0, lng = 0, jw = 0, nb = 0;
    for (int side = 0; side < 2; side++) {
      const size_t li = 2 * size_t(v) + side;
      for (uint32_t j = occ_off_[li]; j < occ_off_[li + 1]; j++) {
        const uint32_t c = occ_[j];
        if (ntrue_[c]) continue;
        const uint32_t open = uint32_t(coff_[c + 1] - coff_[c]) - nfalse_[c];
        (side ? neg : pos) += 1;
        if (open == 2) bin += 1;
        else if (open == 3) ter += 1;
        else lng += 1;
        jw += std::ldexp(1.f, -int(std::min<uint32_t>(open, 60)));
        nb += float(open) - 1.f;
      }
    }
    float* f = out->data() + r * kFeatures;
    f[0] = pos / 32.f;
    f[1] = neg / 32.f;
    f[2] = bin / 16.f;
    f[3] = ter / 16.f;
    f[4] = lng / 16.f;
    f[5] = jw;
    f[6] = float(occurrences_[v]) / 64.f;
    f[7] = bit_width_[v] ? 1.f : 0.f;
    f[8] = bit_width_[v] ? (float(bit_pos_[v]) + 0.5f) / float(bit_width_[v]) : 0.f;
    f[9] = float(f_) / 256.f;
    f[10] = float(n_unsat_) / nc;
    f[11] = float(stack_.size()) / 64.f;
    f[12] = std::log2(1.f + pos + neg);
    f[13] = nb / 64.f;
    f[14] = float(r) / float(cands.size());
    f[15] = 1.f;
  }
}

// Width in bits of the value ranges left to the inputs: sum over input
// words of log2(hi - lo + 1), the ranges narrowed by the word-level facts
// when the query has them (0 when they conflict).
float Splitter::input_range_bits() {
  const size_t ni = q_.in_first.size();
  if (ni == 0) return 0.f;
  if (!q_.word_facts.empty()) {
    std::vector<uint32_t> lv;
    if (!word_check(&lv)) return 0.f;
  }
  float bits = 0.f;
  for (size_t a = 0; a < ni; a++) {
    __int128 lo, hi;
    if (!q_.word_facts.empty()) {
      lo = wlo_[a];
      hi = whi_[a];
    } else {
      lo = hi = 0;
      for (uint32_t b = 0; b < q_.in_width[a]; b++) {
        const int8_t x = assign_[q_.in_first[a] + b];
        const __int128 w = (__int128)1 << b;
        if (x == 1) { lo += w; hi += w; }
        else if (x < 0) hi += w;
      }
    }
    bits += std::log2(float(double(hi - lo) + 1.0));
  }
  return bits;
}

// One-step lookahead after propagating v = 0 and v = 1: the reduction of
// the active variable count (a conflicting branch counts as reducing it
// to 0), log2(1 + reduction) summed over the two branches, plus the
// reduction of the inputs' range width in bits (a word-level view of the
// same progress: deciding a high input bit halves that input's range).
float Splitter::lookahead_label(int32_t v) {
  const size_t pos = trail_.size();
  const uint32_t f = f_;
  const float r = input_range_bits();
  float dr = 0.f;
  auto branch = [&](int32_t lit) {
    const bool ok = propagate(lit);
    const uint32_t fb = ok ? f_ : 0;
    dr += r - (ok ? input_range_bits() : 0.f);
    undo_to(pos);
    return fb;
  };
  const uint32_t f0 = branch(-v), f1 = branch(v);
  return std::log2(1.f + float(f - f0)) + std::log2(1.f + float(f - f1)) + dr;
}

void Splitter::provide_scores(const float* scores) {
  ranking_ = req_vars_;
  bool finite = true;
  for (size_t i = 0; i < req_vars_.size(); i++) finite &= std::isfinite(scores[i]);
  if (finite) {
    std::vector<size_t> idx(req_vars_.size());
    for (size_t i = 0; i < idx.size(); i++) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return scores[a] > scores[b]; });
    for (size_t i = 0; i < idx.size(); i++) ranking_[i] = req_vars_[idx[i]];
  }
  have_scores_ = true;
}

// The most significant unassigned active bit of the input word that holds
// variable v, or 0.
int32_t Splitter::word_top_bit(int32_t v) const {
  const uint32_t w = bit_width_[v];
  if (!w) return 0;
  const uint32_t first = uint32_t(v) - bit_pos_[v];
  for (uint32_t b = w; b-- > 0;) {
    const int32_t u = int32_t(first + b);
    if (assign_[u] < 0 && act_cnt_[u] > 0) return u;
  }
  return 0;
}

// The best-ranked candidate while the last ranking applies (the node it was
// made at and `rescore` levels below), else 0.  A candidate that was the top
// active bit of an input word stands for that word: once its bit is
// assigned, the word's next active bit takes its place in the ranking (so a
// ranking that puts input words first descends through their bits the way
// the word ordering does).
int32_t Splitter::choose_learned() {
  if (!rank_valid_ || stack_.size() < rank_depth_ || stack_.size() >= rank_depth_ + rescore_) return 0;
  for (int32_t v : ranking_) {
    if (assign_[v] < 0 && act_cnt_[v] > 0) return v;
    if (rank_words_.count(v)) {
      const int32_t u = word_top_bit(v);
      if (u) return u;
    }
  }
  return 0;
}

void Splitter::reset_state() {
  assign_.assign(size_t(n_) + 1, -1);
  reason_.assign(size_t(n_) + 1, -1);
  level_.assign(size_t(n_) + 1, 0);
  seen_.assign(size_t(n_) + 1, 0);
  seen_stamp_ = 0;
  ntrue_.assign(q_.n_clauses(), 0);
  nfalse_.assign(q_.n_clauses(), 0);
  act_cnt_ = act_init_;
  f_ = f_init_;
  n_unsat_ = q_.n_clauses();
  trail_.clear();
  stack_.clear();
}

// Assign `lit` (reason -1) and everything unit propagation implies.  On a
// conflict, conflict_clause_ holds a clause whose literals are all false
// (-1 when a decision clashes with an earlier assignment).
bool Splitter::propagate(int32_t lit) {
  queue_.clear();
  queue_.push_back({lit, -1});
  conflict_clause_ = -1;
  bool conflict = false;
  const uint32_t lvl = uint32_t(stack_.size());
  for (size_t qi = 0; qi < queue_.size() && !conflict; qi++) {
    const int32_t l = queue_[qi].first, why = queue_[qi].second;
    const int32_t v = std::abs(l);
    const int8_t val = l > 0;
    if (assign_[v] >= 0) {
      if (assign_[v] != val) {
        conflict = true;
        conflict_clause_ = why;   // every literal of the implying clause is now false
      }
      continue;
    }
    if (act_cnt_[v] > 0) f_--;
    assign_[v] = val;
    reason_[v] = why;
    level_[v] = lvl;
    trail_.push_back(v);
    size_t li = 2 * size_t(v) + (val ? 0 : 1), lf = 2 * size_t(v) + (val ? 1 : 0);
    for (uint32_t j = occ_off_[li]; j < occ_off_[li + 1]; j++) {
      uint32_t c = occ_[j];
      if (ntrue_[c]++ == 0) {
        n_unsat_--;
        for (uint64_t i = coff_[c]; i < coff_[c + 1]; i++) {
          int32_t u = std::abs(q_.lits[i]);
          if (--act_cnt_[u] == 0 && assign_[u] < 0) f_--;
        }
      }
    }
    for (uint32_t j = occ_off_[lf]; j < occ_off_[lf + 1]; j++) {
      uint32_t c = occ_[j];
      nfalse_[c]++;
      if (ntrue_[c] != 0) continue;
      uint64_t size = coff_[c + 1] - coff_[c];
      if (nfalse_[c] == size) {
        if (!conflict) conflict_clause_ = int64_t(c);
        conflict = true;
      } else if (nfalse_[c] + 1 == size) {
        for (uint64_t i = coff_[c]; i < coff_[c + 1]; i++)
          if (assign_[std::abs(q_.lits[i])] < 0) { queue_.push_back({q_.lits[i], int32_t(c)}); break; }
      }
    }
  }
  return !conflict;
}

void Splitter::undo_to(size_t pos) {
  while (trail_.size() > pos) {
    int32_t v = trail_.back();
    trail_.pop_back();
    int8_t val = assign_[v];
    size_t li = 2 * size_t(v) + (val ? 0 : 1), lf = 2 * size_t(v) + (val ? 1 : 0);
    for (uint32_t j = occ_off_[lf]; j < occ_off_[lf + 1]; j++) nfalse_[occ_[j]]--;
    for (uint32_t j = occ_off_[li]; j < occ_off_[li + 1]; j++) {
      uint32_t c = occ_[j];
      if (--ntrue_[c] == 0) {
        n_unsat_++;
        for (uint64_t i = coff_[c]; i < coff_[c + 1]; i++) {
          int32_t u = std::abs(q_.lits[i]);
          if (act_cnt_[u]++ == 0 && assign_[u] < 0) f_++;
        }
      }
    }
    assign_[v] = -1;
    reason_[v] = -1;
    if (act_cnt_[v] > 0) f_++;
  }
}

// Decision levels (1-based) that the last conflict depends on: walk the
// implication graph back from the conflicting clause to decisions.
std::vector<uint32_t> Splitter::analyze() {
  if (conflict_clause_ < 0) {   // no clause to blame: depend on every decision
    std::vector<uint32_t> levels;
    for (uint32_t l = 1; l <= stack_.size(); l++) levels.push_back(l);
    return levels;
  }
  std::vector<int32_t> vars;
  for (uint64_t i = coff_[conflict_clause_]; i < coff_[conflict_clause_ + 1]; i++)
    vars.push_back(std::abs(q_.lits[i]));
  return levels_of(vars);
}

// Decision levels behind the assignments of `vars` (through the implying
// clauses).
std::vector<uint32_t> Splitter::levels_of(const std::vector<int32_t>& vars) {
  std::vector<uint32_t> levels;
  if (++seen_stamp_ == 0) { std::fill(seen_.begin(), seen_.end(), 0); seen_stamp_ = 1; }
  std::vector<int32_t> work;
  auto push = [&](int32_t u) {
    if (seen_[u] != seen_stamp_) { seen_[u] = seen_stamp_; work.push_back(u); }
  };
  for (int32_t u : vars) push(u);
  while (!work.empty()) {
    int32_t u = work.back();
    work.pop_back();
    if (assign_[u] < 0 || level_[u] == 0) continue;   // root facts need no decision
    if (reason_[u] < 0) {
      levels.push_back(level_[u]);
      continue;
    }
    const uint64_t c = uint64_t(reason_[u]);
    for (uint64_t i = coff_[c]; i < coff_[c + 1]; i++) push(std::abs(q_.lits[i]));
  }
  std::sort(levels.begin(), levels.end());
  levels.erase(std::unique(levels.begin(), levels.end()), levels.end());
  return levels;
}

namespace {
__int128 floor_div128(__int128 a, __int128 b) {   // b > 0
  __int128 q = a / b;
  if (a % b != 0 && a < 0) q--;
  return q;
}
__int128 ceil_div128(__int128 a, __int128 b) { return -floor_div128(-a, b); }
}  // namespace

// Interval propagation of the root facts over the atom ranges that the
// current assignment of the input bits allows.  Returns false on an empty
// range, with the decision levels it rests on.
bool Splitter::word_check(std::vector<uint32_t>* levels) {
  const size_t na = q_.atom_range.size();
  const size_t ni = q_.in_first.size();
  if (na == 0) return true;
  wlo_.resize(na);
  whi_.resize(na);
  wsrc_.resize(na);
  auto bit_of = [](size_t a) { return a < 63 ? uint64_t(1) << a : uint64_t(1) << 63; };
  for (size_t a = 0; a < na; a++) {
    wlo_[a] = q_.atom_range[a].first;
    whi_[a] = q_.atom_range[a].second;
    wsrc_[a] = 0;
    if (a >= ni) continue;
    __int128 lo = 0, hi = 0;
    bool any = false;
    for (uint32_t b = 0; b < q_.in_width[a]; b++) {
      const int8_t v = assign_[q_.in_first[a] + b];
      const __int128 w = (__int128)1 << b;
      if (v == 1) { lo += w; hi += w; any = true; }
      else if (v == 0) any = true;
      else hi += w;
    }
    if (!any) continue;
    if (lo > wlo_[a]) wlo_[a] = lo;
    if (hi < whi_[a]) whi_[a] = hi;
    wsrc_[a] = bit_of(a);
  }
  uint64_t blame = 0;
  bool conflict = false;
  for (int pass = 0; pass < 8 && !conflict; pass++) {
    bool changed = false;
    for (const WordFact& f : q_.word_facts) {
      for (int sgn = 1; sgn >= -1 && !conflict; sgn -= 2) {
        if (sgn < 0 && !f.eq) break;
        // maximum of the fact's left side, and the atoms it rests on
        __int128 total = sgn * f.c0;
        uint64_t src = 0;
        const size_t nt = f.terms.size();
        __int128 tmax[64];
        if (nt > 64) break;
        for (size_t t = 0; t < nt; t++) {
          const WordTerm& wt = f.terms[t];
          __int128 plo = 1, phi = 1;
          for (uint32_t a : wt.atoms) {
            plo *= wlo_[a];
            phi *= whi_[a];
            src |= wsrc_[a];
          }
          const __int128 c = sgn * wt.coef;
          tmax[t] = c > 0 ? c * phi : c * plo;
          total += tmax[t];
        }
        if (total < 0) { conflict = true; blame = src; break; }
        for (size_t t = 0; t < nt && !conflict; t++) {
          const WordTerm& wt = f.terms[t];
          const __int128 c = sgn * wt.coef;
          const __int128 need = -(total - tmax[t]);   // c * prod >= need
          for (size_t pos = 0; pos < wt.atoms.size(); pos++) {
            const uint32_t a = wt.atoms[pos];
            __int128 olo = 1, ohi = 1;
            for (size_t o = 0; o < wt.atoms.size(); o++)
              if (o != pos) { olo *= wlo_[wt.atoms[o]]; ohi *= whi_[wt.atoms[o]]; }
            if (c > 0) {
              if (need <= 0 || ohi <= 0) continue;   // nothing to learn (or 0 < need: total < 0 next pass)
              const __int128 lo = ceil_div128(ceil_div128(need, c), ohi);
              if (lo > wlo_[a]) { wlo_[a] = lo; wsrc_[a] |= src; changed = true; }
            } else {
              if (olo <= 0) continue;
              const __int128 u = floor_div128(-need, -c);   // prod <= u
              const __int128 hi = u < 0 ? -1 : floor_div128(u, olo);
              if (hi < whi_[a]) { whi_[a] = hi; wsrc_[a] |= src; changed = true; }
            }
            if (wlo_[a] > whi_[a]) { conflict = true; blame = wsrc_[a] | src; break; }
          }
        }
      }
      if (conflict) break;
    }
    if (!changed) break;
  }
  if (!conflict) return true;
  std::vector<int32_t> vars;
  for (size_t a = 0; a < ni; a++) {
    if (!(blame & bit_of(a))) continue;
    for (uint32_t b = 0; b < q_.in_width[a]; b++)
      if (assign_[q_.in_first[a] + b] >= 0) vars.push_back(int32_t(q_.in_first[a] + b));
  }
  *levels = levels_of(vars);
  return false;
}

bool Splitter::root_propagate() {
  for (uint64_t c = 0; c < q_.n_clauses(); c++) {
    uint64_t size = coff_[c + 1] - coff_[c];
    if (size == 0) return false;
    if (size == 1 && !propagate(q_.lits[coff_[c]])) return false;
  }
  return true;
}

int32_t Splitter::choose_word() const {
  for (int32_t v : word_order_)
    if (assign_[v] < 0 && act_cnt_[v] > 0) return v;
  return choose_static();
}

std::vector<int32_t> Splitter::branch_order() const {
  if (!word_) return order_;
  // choose_word takes the first active input bit of word_order_, else the
  // first active variable of the static order, which is then no input bit
  std::vector<int32_t> out = word_order_;
  for (int32_t v : order_)
    if (!bit_width_[v]) out.push_back(v);
  return out;
}

int32_t Splitter::choose_static() const {
  for (int32_t v : order_)
    if (assign_[v] < 0 && act_cnt_[v] > 0) return v;
  return 0;
}

// The branch explored first: v = 0.
int32_t Splitter::first_literal(int32_t v) const { return -v; }

std::vector<int32_t> Splitter::path() const {
  std::vector<int32_t> lits;
  lits.reserve(stack_.size());
  for (const Decision& d : stack_) lits.push_back(d.phase ? -d.lit : d.lit);
  return lits;
}

void Splitter::emit(CubeKind kind, std::vector<int32_t> lits, std::vector<Cube>& out, bool keep) {
  Cube c;
  c.kind = kind;
  c.lits = std::move(lits);
  if (kind != CubeKind::kLeaf) {
    n_refuted_++;
    n_pruned_ += kind == CubeKind::kPruned;
    if (keep) out.push_back(std::move(c));
  } else {
    c.f = int32_t(f_);
    c.nres = uint32_t(n_unsat_);
    if (keep_leaf_state_) {
      c.assign = assign_;
      c.active.reserve(f_);
      for (uint32_t v = 1; v <= n_; v++)
        if (assign_[v] < 0 && act_cnt_[v] > 0) c.active.push_back(int32_t(v));
    }
    n_leaves_++;
    out.push_back(std::move(c));
  }
}

// The current branch of the deepest decision is done and failed as `r`
// (for a leaf: outcome unknown).  Moves to the next branch to walk and
// returns true, or returns false when the tree is exhausted.
bool Splitter::finish_branch(Failure r, std::vector<Cube>& out, bool keep) {
  while (!stack_.empty()) {
    Decision& d = stack_.back();
    const uint32_t lvl = uint32_t(stack_.size());
    undo_to(d.trail_pos);
    const bool depends = r.unknown || std::binary_search(r.levels.begin(), r.levels.end(), lvl);
    d.acc.unknown |= r.unknown;
    for (uint32_t l : r.levels)
      if (l < lvl) d.acc.levels.push_back(l);
    std::sort(d.acc.levels.begin(), d.acc.levels.end());
    d.acc.levels.erase(std::unique(d.acc.levels.begin(), d.acc.levels.end()), d.acc.levels.end());
    if (d.phase == 0) {
      if (!depends) {
        // the 1-branch fails for the same reasons: prune it
        std::vector<int32_t> lits = path();
        lits.back() = -d.lit;
        emit(CubeKind::kPruned, std::move(lits), out, keep);
      } else {
        d.phase = 1;
        if (propagate(-d.lit)) return true;
        Failure f1;
        f1.levels = analyze();
        emit(CubeKind::kRefuted, path(), out, keep);
        r = std::move(f1);
        if (cubes_total() >= max_cubes_) return true;   // the caller stops on the budget
        continue;   // this decision's 1-branch is done too
      }
    }
    r = std::move(d.acc);
    stack_.pop_back();
    if (stack_.size() <= rank_depth_) rank_valid_ = false;   // the ranked node is done
    if (cubes_total() >= max_cubes_ && !stack_.empty()) return true;
  }
  return false;
}

Splitter::State Splitter::next(uint32_t max_leaves, std::vector<Cube>& out, bool keep_refuted) {
  if (state_ != kRunning) return state_;
  if (!awaiting_) produced_ = 0;   // a call that resumes after scores keeps counting
  awaiting_ = false;
  if (!started_) {
    started_ = true;
    reset_state();
    if (!root_propagate()) {
      root_conflict_ = true;
      emit(CubeKind::kRefuted, {}, out, keep_refuted);
      state_ = kExhausted;
      return state_;
    }
    at_fresh_node_ = true;
  }
  if (pending_) {
    pending_ = false;
    if (!finish_branch(std::move(pending_r_), out, keep_refuted)) { state_ = kExhausted; return state_; }
    if (cubes_total() >= max_cubes_) { state_ = kBudget; return state_; }
    at_fresh_node_ = true;
    word_checked_ = false;
  }
  for (;;) {
    Failure r;
    bool leaf = false;
    if (at_fresh_node_ && !stack_.empty() && !q_.word_facts.empty() && !word_checked_) {
      word_checked_ = true;
      if (!word_check(&r.levels)) {
        emit(CubeKind::kPruned, path(), out, keep_refuted);
        at_fresh_node_ = false;
      }
    }
    if (at_fresh_node_) {
      int32_t v = 0;
      if (f_ > k_ || n_unsat_ > max_res_) {
        if (learned_) {
          v = choose_learned();
          if (!v && have_scores_) {   // scores for this node arrived
            have_scores_ = false;
            rank_valid_ = true;
            rank_depth_ = stack_.size();
            v = choose_learned();
          } else if (!v) {
            req_vars_ = candidates(n_cands_, &rank_words_);
            if (req_vars_.size() > 1) {
              features(req_vars_, &req_feats_);
              awaiting_ = true;
              return kNeedScore;
            }
            // one candidate needs no scores: with input words first, it is
            // the top active bit of the one open word
            if (req_vars_.size() == 1) v = req_vars_[0];
          }
        }
        if (!v) v = word_ ? choose_word() : choose_static();
        if (trace_ && stack_.size() < trace_depth_ && decisions_++ % trace_every_ == 0) {
          const std::vector<int32_t> cands = candidates(n_cands_);
          std::vector<float> fe;
          features(cands, &fe);
          tr_feats_.insert(tr_feats_.end(), fe.begin(), fe.end());
          for (int32_t c : cands) {
            tr_labels_.push_back(lookahead_label(c));
            tr_nodes_.push_back(decisions_);
          }
        }
      }
      if (v == 0) {   // a leaf (v == 0 with f > k cannot happen: f > 0 needs an active variable)
        emit(CubeKind::kLeaf, path(), out, keep_refuted);
        produced_++;
        r.unknown = true;
        leaf = true;
      } else {
        const int32_t lit = first_literal(v);
        stack_.push_back({lit, 0, trail_.size(), Failure{}});
        if (propagate(lit)) { word_checked_ = false; continue; }
        r.levels = analyze();
        emit(CubeKind::kRefuted, path(), out, keep_refuted);
      }
      at_fresh_node_ = false;
    }
    if (leaf && produced_ >= max_leaves) {
      pending_r_ = std::move(r);
      pending_ = true;
      return kRunning;
    }
    const bool moved = finish_branch(std::move(r), out, keep_refuted);
    if (!moved) { state_ = kExhausted; return state_; }
    if (cubes_total() >= max_cubes_) { state_ = kBudget; return state_; }
    at_fresh_node_ = true;
    word_checked_ = false;
    if (produced_ >= max_leaves) return kRunning;
  }
}

bool Splitter::leaf_of(const std::vector<int32_t>& cube, std::vector<int8_t>* assign,
                       std::vector<int32_t>* active, uint32_t* nres) {
  started_ = true;
  state_ = kExhausted;
  reset_state();
  bool ok = root_propagate();
  for (size_t i = 0; ok && i < cube.size(); i++) ok = propagate(cube[i]);
  if (!ok) return false;
  *assign = assign_;
  active->clear();
  std::vector<char> act(size_t(n_) + 1, 0);
  uint32_t unsat = 0;
  for (uint64_t c = 0; c < q_.n_clauses(); c++) {
    if (ntrue_[c]) continue;
    unsat++;
    for (uint64_t i = coff_[c]; i < coff_[c + 1]; i++) {
      int32_t v = std::abs(q_.lits[i]);
      if (assign_[v] < 0) act[v] = 1;
    }
  }
  for (uint32_t v = 1; v <= n_; v++)
    if (act[v]) active->push_back(int32_t(v));
  *nres = unsat;
  return true;
}

}  // namespace scuba
