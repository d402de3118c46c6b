// Shared host-side types of the library (not part of the C ABI).
#pragma once
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/scuba.h"

namespace scuba {

struct Error : std::runtime_error {
  scuba_status code;
  Error(scuba_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(scuba_status c, const std::string& m) { throw Error(c, m); }

// A root fact over atoms for word-level bounds at split nodes:
// sum(coef * prod(atoms)) + c0 >= 0 (or == 0).  Atoms 0 .. inputs-1 are the
// declared inputs; later atoms are quotients / remainders by constants.
struct WordTerm {
  std::vector<uint32_t> atoms;
  __int128 coef;
};
struct WordFact {
  std::vector<WordTerm> terms;
  __int128 c0;
  bool eq;
};

// One query's CNF plus what the result stage needs to decode witnesses.
struct CnfQuery {
  uint32_t n_vars = 0;
  std::vector<uint64_t> off{0};      // clause offsets into lits
  std::vector<int32_t> lits;
  std::vector<uint32_t> in_first;    // declared inputs: first CNF variable
  std::vector<uint32_t> in_width;    //                  width in bits
  std::vector<uint8_t> in_defined;   // 1: a root equality defines the input
                                     //    from the others (decided last)
  bool root_unsat = false;
  uint32_t wrap_bits = 0;             // > 0: machine integers of this width
  // word-level root facts and the value range of every atom (empty when a
  // magnitude would not fit 100 bits: then no word-level check)
  std::vector<WordFact> word_facts;
  std::vector<std::pair<__int128, __int128>> atom_range;
  // original query, kept for the exact integer witness check
  bool has_query = false;
  std::vector<scuba_node> nodes;
  std::vector<uint32_t> roots;

  // Occurrence lists: literal index 2*v + (1 if negative) -> the clauses
  // that hold the literal, in increasing order (occ_off has 2*(n_vars+1)+1
  // entries).  Built with the CNF for every query not decided at the root,
  // and shared by the splitter and the device upload.
  std::vector<uint32_t> occ_off, occ;

  uint64_t n_clauses() const { return off.size() - 1; }
  bool has_occurrences() const {
    return occ_off.size() == 2 * (size_t(n_vars) + 1) + 1 && occ.size() == lits.size();
  }
  void build_occurrences();
};

// Limits shared by host and device code paths.
constexpr uint32_t kMaxLeafVars = 38;       // f <= 38: high slots fit 26 bits
constexpr uint32_t kDefaultMaxResidual = 2048;

// Builds the CNF of one query (normalisation + Tseitin).
CnfQuery bitblast_query(const scuba_node* nodes, uint64_t n_nodes, const uint32_t* roots,
                        uint64_t n_roots, uint32_t flags);

// Exact integer check of a witness against the original query.
bool int_check_query(const CnfQuery& q, const std::vector<uint64_t>& values);

}  // namespace scuba

struct scuba_cnf {
  std::vector<scuba::CnfQuery> q;
};
