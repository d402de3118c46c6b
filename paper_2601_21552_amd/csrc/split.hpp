// Host unit propagation and the cube splitter.
//
// The splitter walks a DPLL tree in depth-first order (0-branch first).
// At each node unit propagation runs to its fixpoint; a conflicting node is a
// refuted cube; a node with at most k active variables (unassigned and in
// some clause not yet satisfied) and at most max_residual unsatisfied
// clauses is a leaf for the device; otherwise the scorer picks the branching
// variable.  The walk is resumable, so leaves can be produced lazily.
//
// Word-level bounds: for bit-blasted queries the root facts over the inputs
// are checked at every node against the value ranges the assigned input
// bits leave (interval propagation to a fixpoint).  An empty range proves
// the node has no model; it becomes a pruned cube, blamed on the decisions
// behind the input bits the contradiction used.
//
// Backjumping: every propagation records the clause that implied each
// variable, so a conflict names the decisions it depends on.  When every
// failure below the 0-branch of a decision is a host conflict that does not
// depend on that decision, the 1-branch fails for the same reasons; it is
// emitted as a pruned cube instead of being walked.  Leaves count as
// failures that depend on every decision (their outcome is not known here).
#pragma once
#include <cstdint>
#include <set>
#include <vector>

#include "common.hpp"

namespace scuba {

enum class CubeKind : int32_t { kLeaf = 0, kRefuted = 1, kPruned = 2 };

struct Cube {
  std::vector<int32_t> lits;  // branching literals, root first
  int32_t f = -1;             // active variables (leaves)
  uint32_t nres = 0;          // unsatisfied clauses at the fixpoint (leaves)
  CubeKind kind = CubeKind::kLeaf;
  // the leaf's fixpoint, kept when the splitter is asked to: the assignment
  // (-1 unassigned, 0, 1 per variable) and the active variables, ascending
  std::vector<int8_t> assign;
  std::vector<int32_t> active;
  bool refuted() const { return kind != CubeKind::kLeaf; }
};

constexpr int kFeatures = 16;   // per candidate variable, see features()

class Splitter {
 public:
  // kNeedScore: the walk waits for scores of the candidates in request()
  enum State { kRunning = 0, kExhausted = 1, kBudget = 2, kNeedScore = 3 };

  Splitter(const CnfQuery& q, uint32_t k, uint32_t max_residual, uint64_t max_cubes);

  // Learned ordering: at a decision node the walk stops with kNeedScore and
  // asks for scores of its candidates: while an input word has an active
  // bit, the most significant active bit of each input word (each stands
  // for its word, so a decision halves one input's range); after that, the
  // top `candidates` active variables of the static order.  The ranking by
  // score then orders the decisions of that node and of its descendants up
  // to `rescore` levels below.  Non-finite scores fall back to the static
  // order.
  void set_learned(uint32_t candidates, uint32_t rescore);
  // Word ordering: among active input bits the most significant first (ties
  // to the lowest variable), which halves an input's value range per
  // decision; then the static order for the remaining (auxiliary) variables.
  void set_word_order();
  // The fixed branch order of the static or word ordering: every variable,
  // the one a node branches on being the first of them that is active
  // there (the word ordering's active input bits, then the static order).
  std::vector<int32_t> branch_order() const;
  // Leaves carry their fixpoint (Cube::assign, Cube::active).
  void set_keep_leaf_state() { keep_leaf_state_ = true; }
  // Trace mode (static ordering): at every `every`-th decision node above
  // depth `depth`, record features and one-step lookahead labels of the top
  // `candidates` variables.
  void set_trace(uint32_t candidates, uint32_t every, uint32_t depth);
  const std::vector<int32_t>& request_vars() const { return req_vars_; }
  const std::vector<float>& request_features() const { return req_feats_; }
  void provide_scores(const float* scores);
  // trace rows: features (kFeatures each), label, node number
  const std::vector<float>& trace_features() const { return tr_feats_; }
  const std::vector<float>& trace_labels() const { return tr_labels_; }
  const std::vector<uint32_t>& trace_nodes() const { return tr_nodes_; }

  // Produce up to max_leaves more leaves, appended to `out` in depth-first
  // order; refuted and pruned cubes are counted, and appended too when
  // keep_refuted.  Returns the state after the call.
  State next(uint32_t max_leaves, std::vector<Cube>& out, bool keep_refuted);

  State state() const { return state_; }
  uint64_t cubes_total() const { return n_leaves_ + n_refuted_; }
  uint64_t cubes_refuted() const { return n_refuted_; }
  uint64_t cubes_pruned() const { return n_pruned_; }
  bool root_conflict() const { return root_conflict_; }

  // Propagation fixpoint of (F, cube) from the root: assignment (-1/0/1 per
  // variable, index 0 unused), active variables in increasing order, and the
  // number of unsatisfied clauses.  Returns false on a conflict.  This
  // abandons the depth-first walk (next() returns kExhausted afterwards).
  bool leaf_of(const std::vector<int32_t>& cube, std::vector<int8_t>* assign,
               std::vector<int32_t>* active, uint32_t* nres);

 private:
  struct Failure {
    std::vector<uint32_t> levels;  // decision levels the failure depends on
    bool unknown = false;          // a leaf below: depends on everything
  };
  struct Decision {
    int32_t lit;                   // literal of the branch explored first
    int phase;                     // 0: first branch, 1: its negation
    size_t trail_pos;
    Failure acc;                   // failures of the branches done so far
  };

  bool propagate(int32_t lit);     // a decision (or cube literal)
  void undo_to(size_t trail_pos);
  int32_t choose_static() const;
  int32_t choose_word() const;
  int32_t first_literal(int32_t v) const;
  std::vector<uint32_t> analyze();
  std::vector<uint32_t> levels_of(const std::vector<int32_t>& vars);
  bool word_check(std::vector<uint32_t>* levels);
  void emit(CubeKind kind, std::vector<int32_t> lits, std::vector<Cube>& out, bool keep);
  std::vector<int32_t> path() const;
  bool finish_branch(Failure r, std::vector<Cube>& out, bool keep);
  void reset_state();
  bool root_propagate();
  std::vector<int32_t> candidates(uint32_t m, std::set<int32_t>* words = nullptr) const;
  int32_t word_top_bit(int32_t v) const;
  void features(const std::vector<int32_t>& cands, std::vector<float>* out) const;
  float lookahead_label(int32_t v);
  float input_range_bits();
  int32_t choose_learned();

  const CnfQuery& q_;
  uint32_t k_, max_res_;
  uint64_t max_cubes_;
  uint32_t n_;
  // occurrence lists (literal index 2v+neg -> clause list): the query's own,
  // or built here when the query has none
  std::vector<uint32_t> own_occ_off_, own_occ_;
  std::vector<uint32_t> coff_;   // the query's clause offsets, 32-bit
  const uint32_t* occ_off_ = nullptr;
  const uint32_t* occ_ = nullptr;
  std::vector<int32_t> order_;      // static branching order
  std::vector<int32_t> word_order_; // input bits by significance (word ordering)
  bool word_ = false;
  bool words_first_ = false;   // learned: input words only while one is open
  bool keep_leaf_state_ = false;
  // search state
  std::vector<int8_t> assign_;
  std::vector<int32_t> reason_;     // implying clause, -1 for decisions
  std::vector<uint32_t> level_;     // decision level of the assignment
  std::vector<uint32_t> ntrue_, nfalse_;
  std::vector<uint32_t> act_cnt_, act_init_;
  uint32_t f_ = 0, f_init_ = 0;
  uint64_t n_unsat_ = 0;
  std::vector<int32_t> trail_;
  std::vector<std::pair<int32_t, int32_t>> queue_;   // (literal, reason)
  int64_t conflict_clause_ = -1;
  std::vector<uint32_t> seen_;
  uint32_t seen_stamp_ = 0;
  std::vector<Decision> stack_;
  std::vector<uint32_t> static_rank_;   // position of each variable in order_
  std::vector<uint32_t> occurrences_;
  std::vector<uint32_t> bit_pos_, bit_width_;   // input bits: position and width
  // word-level bounds (per atom: range and the atoms whose bits it rests on)
  std::vector<__int128> wlo_, whi_;
  std::vector<uint64_t> wsrc_;
  bool word_checked_ = false;   // the current node passed the word check
  // learned ordering
  bool learned_ = false, have_scores_ = false, rank_valid_ = false;
  uint32_t n_cands_ = 32, rescore_ = 1;
  std::vector<int32_t> req_vars_, ranking_;
  std::set<int32_t> rank_words_;   // candidates that stand for their input word
  std::vector<float> req_feats_;
  size_t rank_depth_ = 0;
  // traces
  bool trace_ = false;
  uint32_t trace_every_ = 1, trace_depth_ = 0, decisions_ = 0;
  std::vector<float> tr_feats_, tr_labels_;
  std::vector<uint32_t> tr_nodes_;
  uint32_t produced_ = 0;
  bool awaiting_ = false;
  bool started_ = false, root_conflict_ = false, at_fresh_node_ = false;
  // the branch that a call's last leaf ended, finished by the next call
  // (work that a query decided by that leaf never needs)
  bool pending_ = false;
  Failure pending_r_;
  State state_ = kRunning;
  uint64_t n_leaves_ = 0, n_refuted_ = 0, n_pruned_ = 0;
};

}  // namespace scuba
