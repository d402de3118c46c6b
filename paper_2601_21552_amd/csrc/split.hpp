// Host unit propagation and the cube splitter.
//
// The splitter walks a DPLL tree in depth-first order (0-branch first).  At
// each node unit propagation runs to its fixpoint; a conflicting node is a
// refuted cube; a node with at most k active variables (unassigned and in
// some clause not yet satisfied) and at most max_residual unsatisfied
// clauses is a leaf for the device; otherwise the scorer picks the branching
// variable.  The walk is resumable, so leaves can be produced lazily.
#pragma once
#include <cstdint>
#include <vector>

#include "common.hpp"

namespace scuba {

struct Cube {
  std::vector<int32_t> lits;  // branching literals, root first
  int32_t f = -1;             // active variables (leaves)
  uint32_t nres = 0;          // unsatisfied clauses at the fixpoint (leaves)
  bool refuted = false;
};

class Splitter {
 public:
  enum State { kRunning = 0, kExhausted = 1, kBudget = 2 };

  Splitter(const CnfQuery& q, uint32_t k, uint32_t max_residual, uint64_t max_cubes);

  // Produce up to max_leaves more leaves, appended to `out` in depth-first
  // order; refuted cubes are counted, and appended too when keep_refuted.
  // Returns the state after the call.
  State next(uint32_t max_leaves, std::vector<Cube>& out, bool keep_refuted);

  State state() const { return state_; }
  uint64_t cubes_total() const { return n_leaves_ + n_refuted_; }
  uint64_t cubes_refuted() const { return n_refuted_; }
  bool root_conflict() const { return root_conflict_; }

  // Propagation fixpoint of (F, cube) from the root: assignment (-1/0/1 per
  // variable, index 0 unused), active variables in increasing order, and the
  // number of unsatisfied clauses.  Returns false on a conflict.  This
  // abandons the depth-first walk (next() returns kExhausted afterwards).
  bool leaf_of(const std::vector<int32_t>& cube, std::vector<int8_t>* assign,
               std::vector<int32_t>* active, uint32_t* nres);

 private:
  bool enqueue_and_propagate(int32_t lit);
  void undo_to(size_t trail_pos);
  int32_t choose_static() const;
  void emit(bool refuted, std::vector<Cube>& out, bool keep);
  void reset_state();
  bool root_propagate();

  const CnfQuery& q_;
  uint32_t k_, max_res_;
  uint64_t max_cubes_;
  uint32_t n_;
  std::vector<uint32_t> occ_off_;   // literal index 2v+neg -> clause list
  std::vector<uint32_t> occ_;
  std::vector<int32_t> order_;      // static order: occurrences desc, index asc
  // search state
  std::vector<int8_t> assign_;
  std::vector<uint32_t> ntrue_, nfalse_;
  std::vector<uint32_t> act_cnt_;
  uint32_t f_ = 0;
  uint64_t n_unsat_ = 0;
  std::vector<int32_t> trail_;
  std::vector<int32_t> queue_;
  struct Decision { int32_t var; int phase; size_t trail_pos; };
  std::vector<Decision> stack_;
  bool started_ = false, root_conflict_ = false, at_fresh_node_ = false;
  State state_ = kRunning;
  uint64_t n_leaves_ = 0, n_refuted_ = 0;
};

}  // namespace scuba
