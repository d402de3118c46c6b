// Host unit propagation (eager clause counters with a trail) and the
// resumable depth-first cube splitter.
#include "split.hpp"

#include <algorithm>

namespace scuba {

Splitter::Splitter(const CnfQuery& q, uint32_t k, uint32_t max_residual, uint64_t max_cubes)
    : q_(q), k_(k), max_res_(max_residual), max_cubes_(max_cubes), n_(q.n_vars) {
  std::vector<uint32_t> cnt(2 * (size_t(n_) + 1) + 1, 0);
  for (int32_t l : q_.lits) cnt[2 * size_t(std::abs(l)) + (l < 0)]++;
  occ_off_.assign(cnt.size() + 1, 0);
  for (size_t i = 0; i < cnt.size(); i++) occ_off_[i + 1] = occ_off_[i] + cnt[i];
  occ_.assign(occ_off_.back(), 0);
  std::vector<uint32_t> fill(occ_off_.begin(), occ_off_.end() - 1);
  for (uint64_t c = 0; c < q_.n_clauses(); c++)
    for (uint64_t i = q_.off[c]; i < q_.off[c + 1]; i++) {
      int32_t l = q_.lits[i];
      occ_[fill[2 * size_t(std::abs(l)) + (l < 0)]++] = uint32_t(c);
    }
  // static order: literal occurrences in the original CNF, most first,
  // ties to the lowest variable
  order_.resize(n_);
  for (uint32_t v = 1; v <= n_; v++) order_[v - 1] = int32_t(v);
  auto occurrences = [&](int32_t v) {
    return (occ_off_[2 * v + 1] - occ_off_[2 * v]) + (occ_off_[2 * v + 2] - occ_off_[2 * v + 1]);
  };
  std::stable_sort(order_.begin(), order_.end(), [&](int32_t a, int32_t b) {
    uint32_t oa = occurrences(a), ob = occurrences(b);
    return oa != ob ? oa > ob : a < b;
  });
}

void Splitter::reset_state() {
  assign_.assign(size_t(n_) + 1, -1);
  ntrue_.assign(q_.n_clauses(), 0);
  nfalse_.assign(q_.n_clauses(), 0);
  act_cnt_.assign(size_t(n_) + 1, 0);
  for (int32_t l : q_.lits) act_cnt_[std::abs(l)]++;
  f_ = 0;
  for (uint32_t v = 1; v <= n_; v++) f_ += act_cnt_[v] > 0;
  n_unsat_ = q_.n_clauses();
  trail_.clear();
  stack_.clear();
}

bool Splitter::enqueue_and_propagate(int32_t lit) {
  queue_.clear();
  queue_.push_back(lit);
  bool conflict = false;
  for (size_t qi = 0; qi < queue_.size() && !conflict; qi++) {
    int32_t l = queue_[qi];
    int32_t v = std::abs(l);
    int8_t val = l > 0;
    if (assign_[v] >= 0) {
      if (assign_[v] != val) conflict = true;
      continue;
    }
    if (act_cnt_[v] > 0) f_--;
    assign_[v] = val;
    trail_.push_back(v);
    size_t li = 2 * size_t(v) + (val ? 0 : 1), lf = 2 * size_t(v) + (val ? 1 : 0);
    for (uint32_t j = occ_off_[li]; j < occ_off_[li + 1]; j++) {
      uint32_t c = occ_[j];
      if (ntrue_[c]++ == 0) {
        n_unsat_--;
        for (uint64_t i = q_.off[c]; i < q_.off[c + 1]; i++) {
          int32_t u = std::abs(q_.lits[i]);
          if (--act_cnt_[u] == 0 && assign_[u] < 0) f_--;
        }
      }
    }
    for (uint32_t j = occ_off_[lf]; j < occ_off_[lf + 1]; j++) {
      uint32_t c = occ_[j];
      nfalse_[c]++;
      if (ntrue_[c] != 0) continue;
      uint64_t size = q_.off[c + 1] - q_.off[c];
      if (nfalse_[c] == size) {
        conflict = true;
      } else if (nfalse_[c] + 1 == size) {
        for (uint64_t i = q_.off[c]; i < q_.off[c + 1]; i++)
          if (assign_[std::abs(q_.lits[i])] < 0) { queue_.push_back(q_.lits[i]); break; }
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
        for (uint64_t i = q_.off[c]; i < q_.off[c + 1]; i++) {
          int32_t u = std::abs(q_.lits[i]);
          if (act_cnt_[u]++ == 0 && assign_[u] < 0) f_++;
        }
      }
    }
    assign_[v] = -1;
    if (act_cnt_[v] > 0) f_++;
  }
}

bool Splitter::root_propagate() {
  for (uint64_t c = 0; c < q_.n_clauses(); c++) {
    uint64_t size = q_.off[c + 1] - q_.off[c];
    if (size == 0) return false;
    if (size == 1 && !enqueue_and_propagate(q_.lits[q_.off[c]])) return false;
  }
  return true;
}

int32_t Splitter::choose_static() const {
  for (int32_t v : order_)
    if (assign_[v] < 0 && act_cnt_[v] > 0) return v;
  return 0;
}

void Splitter::emit(bool refuted, std::vector<Cube>& out, bool keep) {
  Cube c;
  c.refuted = refuted;
  c.lits.reserve(stack_.size());
  for (const Decision& d : stack_) c.lits.push_back(d.phase ? d.var : -d.var);
  if (refuted) {
    n_refuted_++;
    if (keep) out.push_back(std::move(c));
  } else {
    c.f = int32_t(f_);
    c.nres = uint32_t(n_unsat_);
    n_leaves_++;
    out.push_back(std::move(c));
  }
}

Splitter::State Splitter::next(uint32_t max_leaves, std::vector<Cube>& out, bool keep_refuted) {
  if (state_ != kRunning) return state_;
  if (!started_) {
    started_ = true;
    reset_state();
    if (!root_propagate()) {
      root_conflict_ = true;
      emit(true, out, keep_refuted);
      state_ = kExhausted;
      return state_;
    }
    at_fresh_node_ = true;
  }
  uint32_t produced = 0;
  for (;;) {
    if (at_fresh_node_) {
      if (f_ <= k_ && n_unsat_ <= max_res_) {
        emit(false, out, keep_refuted);
        produced++;
        at_fresh_node_ = false;
      } else {
        int32_t v = choose_static();
        if (v == 0) {  // no active variable: every clause is satisfied
          emit(false, out, keep_refuted);
          produced++;
          at_fresh_node_ = false;
        } else {
          stack_.push_back({v, 0, trail_.size()});
          if (!enqueue_and_propagate(-v)) {
            emit(true, out, keep_refuted);
            at_fresh_node_ = false;
          }
          if (at_fresh_node_ && cubes_total() < max_cubes_) continue;
        }
      }
    }
    // backtrack to the next unexplored 1-branch
    bool moved = false;
    while (!stack_.empty()) {
      Decision& d = stack_.back();
      undo_to(d.trail_pos);
      if (d.phase == 0) {
        d.phase = 1;
        if (enqueue_and_propagate(d.var)) { moved = true; break; }
        emit(true, out, keep_refuted);
        if (cubes_total() >= max_cubes_) break;
      } else {
        stack_.pop_back();
      }
    }
    if (!moved && stack_.empty()) { state_ = kExhausted; return state_; }
    if (cubes_total() >= max_cubes_) { state_ = kBudget; return state_; }
    at_fresh_node_ = true;
    if (produced >= max_leaves) return kRunning;
  }
}

bool Splitter::leaf_of(const std::vector<int32_t>& cube, std::vector<int8_t>* assign,
                       std::vector<int32_t>* active, uint32_t* nres) {
  started_ = true;
  state_ = kExhausted;
  reset_state();
  bool ok = root_propagate();
  for (size_t i = 0; ok && i < cube.size(); i++) ok = enqueue_and_propagate(cube[i]);
  if (!ok) return false;
  *assign = assign_;
  active->clear();
  std::vector<char> act(size_t(n_) + 1, 0);
  uint32_t unsat = 0;
  for (uint64_t c = 0; c < q_.n_clauses(); c++) {
    if (ntrue_[c]) continue;
    unsat++;
    for (uint64_t i = q_.off[c]; i < q_.off[c + 1]; i++) {
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
