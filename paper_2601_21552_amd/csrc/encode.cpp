// Query -> CNF: word-level normalisation and Tseitin encoding.
//
// A query is the constraint set of one memory access (Sec. 4.1 and 5.2):
// kind-1 id bounds, kind-2 "offset >= size", kind-3 definitions and asserts,
// built from expression trees (Sec. 5.1).  Semantics: exact integers, inputs
// unsigned in 0 .. 2^w - 1, satisfiable iff the access can be out of bounds.
//
// Normalisation (verdict- and count-preserving): every integer node becomes
// a polynomial over atoms (inputs; quotients/remainders by constants become
// fresh atoms defined by x = q*k + r, 0 <= r < k).  Every comparison becomes
// a bound on a key polynomial with coprime coefficients and a positive
// leading coefficient, so common additive terms and common positive factors
// cancel and "idx < N" and "idx >= N" meet on one key.  Bounds the roots put
// on the same key are intersected with the key's value range; an empty
// intersection proves UNSAT at the root.
//
// Encoding: every key is computed once in two's complement modulo 2^W,
// where W holds the key's whole value range (modular arithmetic then gives
// the exact value).  Gates are full equivalences with structural hashing, so
// every auxiliary variable is a function of the inputs and the CNF has one
// model per satisfying input tuple.  Root bounds become clauses on the key's
// bits directly (no auxiliary variables).
#include <algorithm>
#include <map>
#include <set>
#include <unordered_map>

#include "bigint.hpp"
#include "common.hpp"

namespace scuba {
namespace {

constexpr int32_t kTrue = 0x7fffffff;
constexpr int32_t kFalse = -kTrue;

using BitVec = std::vector<int32_t>;  // literals, least significant bit first

struct GateKey {
  uint32_t type;
  int32_t a, b, c;
  bool operator==(const GateKey& o) const { return type == o.type && a == o.a && b == o.b && c == o.c; }
};
struct GateKeyHash {
  size_t operator()(const GateKey& k) const {
    uint64_t h = k.type * 0x9E3779B97F4A7C15ull;
    h ^= uint64_t(uint32_t(k.a)) * 0xC2B2AE3D27D4EB4Full + (h << 6) + (h >> 2);
    h ^= uint64_t(uint32_t(k.b)) * 0x165667B19E3779F9ull + (h << 6) + (h >> 2);
    h ^= uint64_t(uint32_t(k.c)) * 0x27D4EB2F165667C5ull + (h << 6) + (h >> 2);
    return size_t(h);
  }
};

// Structural-hashing table of the gate library: open addressing with linear
// probing (keys never leave it); type 0 marks an empty slot.
class GateMap {
 public:
  GateMap() : slots_(1024) {}
  const int32_t* find(const GateKey& k) const {
    for (size_t i = GateKeyHash()(k) & (slots_.size() - 1);; i = (i + 1) & (slots_.size() - 1)) {
      const Slot& s = slots_[i];
      if (s.key.type == 0) return nullptr;
      if (s.key == k) return &s.value;
    }
  }
  void insert(const GateKey& k, int32_t v) {
    if (2 * (used_ + 1) > slots_.size()) grow();
    put(k, v);
    used_++;
  }

 private:
  struct Slot {
    GateKey key{0, 0, 0, 0};
    int32_t value = 0;
  };
  void put(const GateKey& k, int32_t v) {
    size_t i = GateKeyHash()(k) & (slots_.size() - 1);
    while (slots_[i].key.type != 0) i = (i + 1) & (slots_.size() - 1);
    slots_[i].key = k;
    slots_[i].value = v;
  }
  void grow() {
    std::vector<Slot> old(slots_.size() * 2);
    old.swap(slots_);
    for (const Slot& s : old)
      if (s.key.type != 0) put(s.key, s.value);
  }
  std::vector<Slot> slots_;
  size_t used_ = 0;
};

// Clause sink + gate library with constant folding and structural hashing.
class Gates {
 public:
  explicit Gates(CnfQuery& out) : q_(out) {
    q_.lits.reserve(1 << 14);
    q_.off.reserve(1 << 12);
  }

  int32_t fresh() { return int32_t(++q_.n_vars); }

  static void sort3(int32_t* x, int n) {
    for (int i = 1; i < n; i++)
      for (int j = i; j > 0 && x[j - 1] > x[j]; j--) std::swap(x[j - 1], x[j]);
  }

  void clause(std::initializer_list<int32_t> ls) { clause(ls.begin(), ls.size()); }
  void clause(const std::vector<int32_t>& ls) { clause(ls.data(), ls.size()); }
  // Appends the clause after dropping false constants and repeated
  // literals; a true constant or a complementary pair drops the clause.
  void clause(const int32_t* ls, size_t n) {
    const size_t start = q_.lits.size();
    for (size_t i = 0; i < n; i++) {
      int32_t l = ls[i];
      if (l == kTrue) { q_.lits.resize(start); return; }
      if (l == kFalse) continue;
      bool dup = false;
      for (size_t j = start; j < q_.lits.size(); j++) {
        if (q_.lits[j] == l) dup = true;
        if (q_.lits[j] == -l) { q_.lits.resize(start); return; }  // tautology
      }
      if (!dup) q_.lits.push_back(l);
    }
    q_.off.push_back(q_.lits.size());
  }
  // Appends a clause that is known to hold no constant, no repeated variable
  // and no complementary pair (the gate definitions below, after their
  // special cases).
  void gate_clause(std::initializer_list<int32_t> ls) {
    for (int32_t l : ls) q_.lits.push_back(l);
    q_.off.push_back(q_.lits.size());
  }

  int32_t AND(int32_t a, int32_t b) {
    if (a == kFalse || b == kFalse || a == -b) return kFalse;
    if (a == kTrue || a == b) return b;
    if (b == kTrue) return a;
    if (std::abs(a) > std::abs(b)) std::swap(a, b);
    GateKey k{1, a, b, 0};
    if (const int32_t* hit = cache_.find(k)) return *hit;
    int32_t o = fresh();
    gate_clause({-o, a});
    gate_clause({-o, b});
    gate_clause({o, -a, -b});
    cache_.insert(k, o);
    return o;
  }
  int32_t OR(int32_t a, int32_t b) { return -AND(-a, -b); }

  int32_t XOR(int32_t a, int32_t b) {
    bool flip = false;
    auto strip = [&](int32_t& x) {
      if (x == kTrue) { x = kFalse; flip = !flip; }
      else if (x < 0 && x != kFalse) { x = -x; flip = !flip; }
    };
    strip(a);
    strip(b);
    int32_t r;
    if (a == kFalse) r = b;
    else if (b == kFalse) r = a;
    else if (a == b) r = kFalse;
    else {
      if (a > b) std::swap(a, b);
      GateKey k{2, a, b, 0};
      if (const int32_t* hit = cache_.find(k)) r = *hit;
      else {
        int32_t o = fresh();
        gate_clause({-o, a, b});
        gate_clause({-o, -a, -b});
        gate_clause({o, -a, b});
        gate_clause({o, a, -b});
        cache_.insert(k, o);
        r = o;
      }
    }
    return flip ? -r : r;
  }

  int32_t XOR3(int32_t a, int32_t b, int32_t c) {
    bool flip = false;
    int32_t v[3] = {a, b, c};
    for (int32_t& x : v) {
      if (x == kTrue) { x = kFalse; flip = !flip; }
      else if (x < 0 && x != kFalse) { x = -x; flip = !flip; }
    }
    int32_t xs[3];
    int nx = 0;
    for (int32_t x : v) if (x != kFalse) xs[nx++] = x;
    sort3(xs, nx);
    // cancel equal pairs
    int32_t ys[3];
    int ny = 0;
    for (int i = 0; i < nx;) {
      if (i + 1 < nx && xs[i] == xs[i + 1]) { i += 2; continue; }
      ys[ny++] = xs[i++];
    }
    int32_t r;
    if (ny == 0) r = kFalse;
    else if (ny == 1) r = ys[0];
    else if (ny == 2) r = XOR(ys[0], ys[1]);
    else {
      // three-input gates (the full adders' sum and carry) are not looked up
      // in the structural hash: the adders never share them
      int32_t o = fresh();
      for (int m = 0; m < 8; m++) {
        int va = m & 1, vb = (m >> 1) & 1, vc = (m >> 2) & 1;
        int p = va ^ vb ^ vc;
        gate_clause({va ? -ys[0] : ys[0], vb ? -ys[1] : ys[1], vc ? -ys[2] : ys[2], p ? o : -o});
      }
      r = o;
    }
    return flip ? -r : r;
  }

  int32_t MAJ(int32_t a, int32_t b, int32_t c) {
    // constants and repeated inputs
    int32_t v[3] = {a, b, c};
    for (int i = 0; i < 3; i++) {
      if (v[i] == kTrue) { int32_t x = v[(i + 1) % 3], y = v[(i + 2) % 3]; return OR(x, y); }
      if (v[i] == kFalse) { int32_t x = v[(i + 1) % 3], y = v[(i + 2) % 3]; return AND(x, y); }
    }
    for (int i = 0; i < 3; i++)
      for (int j = i + 1; j < 3; j++) {
        if (v[i] == v[j]) return v[i];
        if (v[i] == -v[j]) return v[3 - i - j];
      }
    int neg = (a < 0) + (b < 0) + (c < 0);
    bool flip = false;
    if (neg >= 2) { a = -a; b = -b; c = -c; flip = true; }
    int32_t s[3] = {a, b, c};
    auto by_var = [](int32_t& x, int32_t& y) { if (std::abs(x) > std::abs(y)) std::swap(x, y); };
    by_var(s[0], s[1]);
    by_var(s[1], s[2]);
    by_var(s[0], s[1]);
    const int32_t o = fresh();
    gate_clause({-s[0], -s[1], o});
    gate_clause({-s[0], -s[2], o});
    gate_clause({-s[1], -s[2], o});
    gate_clause({s[0], s[1], -o});
    gate_clause({s[0], s[2], -o});
    gate_clause({s[1], s[2], -o});
    return flip ? -o : o;
  }

  // ---- words (two's complement, modulo 2^W) ----
  static BitVec resize(const BitVec& x, uint32_t w, bool sign_extend) {
    BitVec r(w, kFalse);
    for (uint32_t i = 0; i < w; i++) {
      if (i < x.size()) r[i] = x[i];
      else r[i] = (sign_extend && !x.empty()) ? x.back() : kFalse;
    }
    return r;
  }
  static BitVec constant(const BigInt& v, uint32_t w) {
    BitVec r(w);
    for (uint32_t i = 0; i < w; i++) r[i] = v.tc_bit(i) ? kTrue : kFalse;
    return r;
  }
  BitVec add(const BitVec& x, const BitVec& y, uint32_t w) {  // operands already w bits
    BitVec r(w);
    int32_t carry = kFalse;
    for (uint32_t i = 0; i < w; i++) {
      // a false operand bit with no carry passes the other bit through and
      // carries nothing (what XOR3 and MAJ return there, without the calls)
      if (carry == kFalse && (x[i] == kFalse || y[i] == kFalse)) {
        r[i] = x[i] == kFalse ? y[i] : x[i];
        continue;
      }
      r[i] = XOR3(x[i], y[i], carry);
      if (i + 1 < w) carry = MAJ(x[i], y[i], carry);
    }
    return r;
  }
  BitVec neg(const BitVec& x, uint32_t w) {
    BitVec inv(w), one = constant(BigInt(1), w);
    for (uint32_t i = 0; i < w; i++) inv[i] = -x[i];
    return add(inv, one, w);
  }
  // unsigned x * unsigned y (zero-extended), modulo 2^w
  BitVec mul_u(const BitVec& x, const BitVec& y, uint32_t w) {
    BitVec acc(w, kFalse);
    bool first = true;
    for (uint32_t j = 0; j < y.size() && j < w; j++) {
      if (y[j] == kFalse) continue;
      BitVec row(w, kFalse);
      for (uint32_t i = j; i < w; i++) row[i] = (i - j < x.size()) ? AND(x[i - j], y[j]) : kFalse;
      if (first) { acc = row; first = false; }
      else acc = add(acc, row, w);
    }
    return acc;
  }
  // c * x for a constant c >= 0 and a w-bit word, modulo 2^w
  BitVec mul_const(const BitVec& x, const BigInt& c, uint32_t w) {
    BitVec acc(w, kFalse);
    bool first = true;
    for (uint32_t s = 0; s < w; s++) {
      if (!c.bit(s)) continue;
      BitVec sh(w, kFalse);
      for (uint32_t i = s; i < w; i++) sh[i] = x[i - s];
      if (first) { acc = sh; first = false; }
      else acc = add(acc, sh, w);
    }
    return acc;
  }

  // unsigned comparisons of a word with a constant, as a gate (LSB chain)
  // (constants >= 2^|x| are outside the word's range)
  static bool above(const BitVec& x, const BigInt& c) { return c.bit_length() > x.size(); }
  int32_t ge_const_gate(const BitVec& x, const BigInt& c) {
    if (above(x, c)) return kFalse;
    int32_t g = kTrue;
    for (uint32_t i = 0; i < x.size(); i++) g = c.bit(i) ? AND(x[i], g) : OR(x[i], g);
    return g;
  }
  int32_t eq_const_gate(const BitVec& x, const BigInt& c) {
    if (above(x, c)) return kFalse;
    int32_t g = kTrue;
    for (uint32_t i = 0; i < x.size(); i++) g = AND(g, c.bit(i) ? x[i] : -x[i]);
    return g;
  }
  // unsigned x >= c as clauses: for each 1-bit i of c, x_i or some higher
  // x_j with c_j = 0
  void assert_ge_const(const BitVec& x, const BigInt& c) {
    if (above(x, c)) { clause(std::vector<int32_t>{}); return; }
    for (uint32_t i = 0; i < x.size(); i++) {
      if (!c.bit(i)) continue;
      std::vector<int32_t> cl{x[i]};
      for (uint32_t j = i + 1; j < x.size(); j++)
        if (!c.bit(j)) cl.push_back(x[j]);
      clause(cl);
    }
  }
  // unsigned x <= c: for each 0-bit i of c, not x_i or some higher not x_j
  // with c_j = 1
  void assert_le_const(const BitVec& x, const BigInt& c) {
    if (above(x, c)) return;
    for (uint32_t i = 0; i < x.size(); i++) {
      if (c.bit(i)) continue;
      std::vector<int32_t> cl{-x[i]};
      for (uint32_t j = i + 1; j < x.size(); j++)
        if (c.bit(j)) cl.push_back(-x[j]);
      clause(cl);
    }
  }

 private:
  CnfQuery& q_;
  GateMap cache_;
};

// ---------------------------------------------------------------- validation

enum class Ty { Int, Bool };

std::vector<Ty> validate(const scuba_node* nodes, uint64_t n, const uint32_t* roots, uint64_t nr,
                         uint32_t* n_inputs) {
  std::vector<Ty> ty(n);
  uint32_t nv = 0;
  for (uint64_t i = 0; i < n; i++) {
    const scuba_node& x = nodes[i];
    auto need = [&](uint32_t idx, Ty t) {
      if (idx >= i) fail(SCUBA_E_INVALID, "node " + std::to_string(i) + ": operand is not an earlier node");
      if (ty[idx] != t) fail(SCUBA_E_INVALID, "node " + std::to_string(i) + ": operand type mismatch");
    };
    switch (x.op) {
      case SCUBA_OP_VAR:
        if (x.width < 1 || x.width > 64) fail(SCUBA_E_WIDTH, "node " + std::to_string(i) + ": width outside 1..64");
        if (x.imm != nv) fail(SCUBA_E_INVALID, "node " + std::to_string(i) + ": inputs must be numbered 0,1,2,... in order");
        nv++;
        ty[i] = Ty::Int;
        break;
      case SCUBA_OP_CONST: ty[i] = Ty::Int; break;
      case SCUBA_OP_ADD: case SCUBA_OP_SUB: case SCUBA_OP_MUL:
        need(x.a, Ty::Int); need(x.b, Ty::Int); ty[i] = Ty::Int; break;
      case SCUBA_OP_SHL:
        need(x.a, Ty::Int);
        if (x.imm > 64) fail(SCUBA_E_INVALID, "shift amount above 64");
        ty[i] = Ty::Int; break;
      case SCUBA_OP_UDIV: case SCUBA_OP_UREM:
        need(x.a, Ty::Int);
        if (x.imm == 0) fail(SCUBA_E_INVALID, "division by zero");
        ty[i] = Ty::Int; break;
      case SCUBA_OP_LT: case SCUBA_OP_LE: case SCUBA_OP_GT: case SCUBA_OP_GE:
      case SCUBA_OP_EQ: case SCUBA_OP_NE:
        need(x.a, Ty::Int); need(x.b, Ty::Int); ty[i] = Ty::Bool; break;
      case SCUBA_OP_AND: case SCUBA_OP_OR:
        need(x.a, Ty::Bool); need(x.b, Ty::Bool); ty[i] = Ty::Bool; break;
      case SCUBA_OP_NOT: need(x.a, Ty::Bool); ty[i] = Ty::Bool; break;
      default: fail(SCUBA_E_INVALID, "node " + std::to_string(i) + ": unknown op");
    }
  }
  for (uint64_t r = 0; r < nr; r++)
    if (roots[r] >= n || ty[roots[r]] != Ty::Bool) fail(SCUBA_E_INVALID, "root is not a boolean node");
  *n_inputs = nv;
  return ty;
}

struct Range {
  BigInt lo, hi;
};

Range range_add(const Range& a, const Range& b) { return {a.lo + b.lo, a.hi + b.hi}; }
Range range_mul(const Range& a, const Range& b) {
  BigInt c[4] = {a.lo * b.lo, a.lo * b.hi, a.hi * b.lo, a.hi * b.hi};
  Range r{c[0], c[0]};
  for (auto& v : c) { if (v < r.lo) r.lo = v; if (v > r.hi) r.hi = v; }
  return r;
}
Range range_scale(const Range& a, const BigInt& c) {
  return c >= BigInt(0) ? Range{a.lo * c, a.hi * c} : Range{a.hi * c, a.lo * c};
}

// ---------------------------------------------------------------- polynomials

using Mono = std::vector<uint32_t>;    // sorted atom ids
using Poly = std::map<Mono, BigInt>;   // {} is the constant term

void poly_add_into(Poly& p, const Poly& r, const BigInt& s) {
  for (auto& [m, c] : r) {
    BigInt v = p[m] + c * s;
    if (v.is_zero()) p.erase(m);
    else p[m] = v;
  }
}
Poly poly_mul(const Poly& a, const Poly& b) {
  Poly out;
  for (auto& [m1, c1] : a)
    for (auto& [m2, c2] : b) {
      Mono m = m1;
      m.insert(m.end(), m2.begin(), m2.end());
      std::sort(m.begin(), m.end());
      BigInt v = out[m] + c1 * c2;
      if (v.is_zero()) out.erase(m);
      else out[m] = v;
    }
  return out;
}

struct Atom {
  Range range;
  BitVec bits;         // unsigned magnitude bits
};

// A bound on a key polynomial: lo <= key <= hi (absent side = unbounded).
struct Bound {
  bool has_lo = false, has_hi = false;
  BigInt lo, hi;
  void lower(const BigInt& v) { if (!has_lo || v > lo) { lo = v; has_lo = true; } }
  void upper(const BigInt& v) { if (!has_hi || v < hi) { hi = v; has_hi = true; } }
};

enum class Rel { GE0, EQ0 };

// ---------------------------------------------------------------- relaxation
//
// Rational feasibility of a system of linear constraints over monomials,
// each  dir . m + c >= 0  with dir a primitive integer vector and c a
// reduced fraction.  Fourier-Motzkin elimination decides it exactly; for a
// given direction only the tightest constant is kept.  Every derived
// constraint is a non-negative combination of the inputs, so "infeasible"
// is a proof that the integer system has no solution either.
class Relaxation {
 public:
  static constexpr size_t kCap = 20000;   // constraints; beyond it: undecided

  // dir . m + num/den >= 0 ; returns false on an immediate contradiction
  bool add(Poly dir, BigInt num, BigInt den = BigInt(1)) { return insert(pool_, std::move(dir), num, den); }

  // true: infeasible; false: feasible or undecided (cap)
  bool infeasible() {
    if (contradiction_) return true;
    for (;;) {
      if (pool_.size() > kCap) return false;
      // variable with the fewest new constraints, ties to the smallest
      std::map<Mono, std::pair<size_t, size_t>> occ;
      for (auto& [dir, c] : pool_)
        for (auto& [m, a] : dir) (a.sign() > 0 ? occ[m].first : occ[m].second)++;
      if (occ.empty()) return false;
      const Mono* best = nullptr;
      long long best_cost = 0;
      for (auto& [m, pn] : occ) {
        long long cost = (long long)pn.first * (long long)pn.second - (long long)pn.first - (long long)pn.second;
        if (!best || cost < best_cost) { best = &m; best_cost = cost; }
      }
      const Mono x = *best;
      std::vector<const std::pair<const Poly, Frac>*> pos, neg;
      Pool next;
      for (auto& e : pool_) {
        auto it = e.first.find(x);
        if (it == e.first.end()) next.emplace(e.first, e.second);
        else (it->second.sign() > 0 ? pos : neg).push_back(&e);
      }
      for (auto* p : pos) {
        const BigInt a = p->first.at(x);
        for (auto* q : neg) {
          const BigInt b = -q->first.at(x);
          Poly dir;
          for (auto& [m, c] : p->first) if (m != x) dir[m] = c * b;
          for (auto& [m, c] : q->first) {
            if (m == x) continue;
            BigInt v = dir[m] + c * a;
            if (v.is_zero()) dir.erase(m);
            else dir[m] = v;
          }
          // b*(pn/pd) + a*(qn/qd)
          BigInt num = b * p->second.num * q->second.den + a * q->second.num * p->second.den;
          BigInt den = p->second.den * q->second.den;
          if (!insert(next, std::move(dir), num, den)) return true;
        }
      }
      pool_.swap(next);
    }
  }

 private:
  struct Frac {
    BigInt num, den;   // den > 0, reduced
  };
  using Pool = std::map<Poly, Frac>;

  bool insert(Pool& pool, Poly dir, BigInt num, BigInt den) {
    for (auto it = dir.begin(); it != dir.end();) {
      if (it->second.is_zero()) it = dir.erase(it);
      else ++it;
    }
    if (dir.empty()) {
      if (num.sign() * den.sign() < 0) contradiction_ = true;
      return !contradiction_;
    }
    BigInt g;
    for (auto& [m, c] : dir) g = BigInt::gcd(g, c);
    if (g != BigInt(1)) {
      for (auto& [m, c] : dir) c = BigInt::floor_div(c, g);
      den = den * g;
    }
    if (den.sign() < 0) { num = -num; den = -den; }
    BigInt r = BigInt::gcd(num, den);
    if (!r.is_zero() && r != BigInt(1)) {
      num = BigInt::floor_div(num, r);
      den = BigInt::floor_div(den, r);
    }
    auto it = pool.find(dir);
    if (it == pool.end()) pool.emplace(std::move(dir), Frac{num, den});
    else if (num * it->second.den < it->second.num * den) it->second = Frac{num, den};
    return true;
  }

  Pool pool_;
  bool contradiction_ = false;
};

class Encoder {
 public:
  Encoder(const scuba_node* nodes, uint64_t n, const uint32_t* roots, uint64_t nr, uint32_t flags,
          CnfQuery& out)
      : nodes_(nodes), n_(n), roots_(roots), nr_(nr), flags_(flags), out_(out), g_(out) {}

  void run() {
    uint32_t nv = 0;
    validate(nodes_, n_, roots_, nr_, &nv);
    // inputs get the first variables, LSB first, in declaration order
    for (uint64_t i = 0; i < n_; i++) {
      if (nodes_[i].op != SCUBA_OP_VAR) continue;
      Atom a;
      a.range = {BigInt(0), BigInt::pow2(nodes_[i].width) - BigInt(1)};
      out_.in_first.push_back(out_.n_vars + 1);
      out_.in_width.push_back(nodes_[i].width);
      out_.in_defined.push_back(0);
      for (uint32_t b = 0; b < nodes_[i].width; b++) a.bits.push_back(g_.fresh());
      atoms_.push_back(a);
    }
    const uint32_t wrap = (flags_ >> 8) & 0xFF;
    if (wrap) {
      if (wrap > 64) fail(SCUBA_E_WIDTH, "wrap-around width outside 1..64");
      for (uint64_t i = 0; i < n_; i++)
        if (nodes_[i].op == SCUBA_OP_VAR && nodes_[i].width > wrap)
          fail(SCUBA_E_WIDTH, "node " + std::to_string(i) + ": input wider than the wrap-around width");
      out_.wrap_bits = wrap;
      if (wrap_abstraction_unsat(wrap)) {
        out_.root_unsat = true;
        g_.clause(std::vector<int32_t>{});  // the empty clause
        return;
      }
      run_wrap(wrap);
    } else if (flags_ & SCUBA_BB_NO_REWRITE) {
      run_structural();
    } else {
      run_normalised();
    }
  }

 private:
  // ---------------------------------------------------------- normalised
  void run_normalised() {
    polys_.resize(n_);
    for (uint64_t i = 0; i < n_; i++) {
      const scuba_node& x = nodes_[i];
      switch (x.op) {
        case SCUBA_OP_VAR: polys_[i] = Poly{{Mono{uint32_t(x.imm)}, BigInt(1)}}; break;
        case SCUBA_OP_CONST:
          if (x.imm) polys_[i] = Poly{{Mono{}, BigInt::from_u64(x.imm)}};
          break;
        case SCUBA_OP_ADD: polys_[i] = polys_[x.a]; poly_add_into(polys_[i], polys_[x.b], BigInt(1)); break;
        case SCUBA_OP_SUB: polys_[i] = polys_[x.a]; poly_add_into(polys_[i], polys_[x.b], BigInt(-1)); break;
        case SCUBA_OP_MUL: polys_[i] = poly_mul(polys_[x.a], polys_[x.b]); break;
        case SCUBA_OP_SHL:
          for (auto& [m, c] : polys_[x.a]) polys_[i][m] = c.shl(uint32_t(x.imm));
          break;
        case SCUBA_OP_UDIV: case SCUBA_OP_UREM: polys_[i] = div_atom(i); break;
        default: break;
      }
    }
    // root facts; anything that is not a conjunction of comparisons is
    // kept as a boolean formula and encoded with gates
    std::vector<std::pair<uint32_t, bool>> complex_roots;
    for (uint64_t r = 0; r < nr_; r++) collect(roots_[r], true, complex_roots);
    for (auto& f : div_facts_) facts_.push_back(f);
    // the facts as given are what gets encoded
    for (auto& [p, rel] : facts_) add_fact(bounds_, p, rel);

    // Root equalities that define an atom linearly (coefficient +-1, the atom
    // in no other monomial) eliminate it from every fact; the rewritten facts
    // are implied by the originals and only join the UNSAT check.
    std::map<Poly, Bound> check = bounds_;
    std::vector<std::pair<uint32_t, Poly>> subs;
    for (auto& [p0, rel] : facts_) {
      if (rel != Rel::EQ0) continue;
      Poly p = substitute_all(p0, subs);
      const Mono* pivot = nullptr;
      for (auto& [m, c] : p) {
        if (m.size() != 1 || c.abs() != BigInt(1)) continue;
        bool alone = true;
        for (auto& [m2, c2] : p)
          if (&m2 != &m && std::find(m2.begin(), m2.end(), m[0]) != m2.end()) alone = false;
        if (alone) { pivot = &m; break; }
      }
      if (!pivot) continue;
      const uint32_t atom = (*pivot)[0];
      const BigInt c = p.at(*pivot);
      Poly expr;   // atom = -(p - c*atom)/c = -c*(p - c*atom) since c = +-1
      for (auto& [m, cc] : p)
        if (&m != pivot) expr[m] = -(cc * c);
      for (auto& [a, e] : subs) e = substitute(e, atom, expr);
      subs.push_back({atom, expr});
      if (atom < out_.in_defined.size()) out_.in_defined[atom] = 1;
    }
    if (!subs.empty())
      for (auto& [p, rel] : facts_) add_fact(check, substitute_all(p, subs), rel);

    if (!unsat_) {
      for (auto& [key, b] : check) {
        Range kr = poly_range(key);
        BigInt lo = b.has_lo && b.lo > kr.lo ? b.lo : kr.lo;
        BigInt hi = b.has_hi && b.hi < kr.hi ? b.hi : kr.hi;
        if (lo > hi) { unsat_ = true; break; }
      }
    }
    if (!unsat_) {
      std::vector<std::pair<Poly, Rel>> all = facts_;
      if (!subs.empty())
        for (auto& [p, rel] : facts_) all.push_back({substitute_all(p, subs), rel});
      unsat_ = relaxation_infeasible(all);
    }
    if (unsat_) {
      out_.root_unsat = true;
      g_.clause(std::vector<int32_t>{});  // the empty clause
      return;
    }
    export_word_facts(subs);
    for (auto& [key, b] : bounds_) assert_bound(key, b);
    for (auto& [node, pos] : complex_roots) {
      int32_t l = bool_lit(node);
      g_.clause({pos ? l : -l});
    }
  }

  // Root facts (as given and with the defining equalities substituted)
  // for the splitter's word-level bounds; dropped as a whole when some
  // magnitude could leave 100 bits.
  void export_word_facts(const std::vector<std::pair<uint32_t, Poly>>& subs) {
    std::vector<std::pair<Poly, Rel>> all = facts_;
    if (!subs.empty())
      for (auto& [p, rel] : facts_) all.push_back({substitute_all(p, subs), rel});
    std::vector<std::pair<__int128, __int128>> ranges;
    for (const Atom& a : atoms_) {
      __int128 lo, hi;
      if (!a.range.lo.to_i128(&lo, 64) || !a.range.hi.to_i128(&hi, 64) || lo < 0) return;
      ranges.push_back({lo, hi});
    }
    std::vector<WordFact> out;
    for (auto& [p, rel] : all) {
      WordFact f;
      f.eq = rel == Rel::EQ0;
      f.c0 = 0;
      BigInt mag;   // bound on |sum| over the atom ranges
      for (auto& [m, c] : p) {
        Range r = range_scale(mono_range(m), c);
        mag = mag + (r.hi.abs() > r.lo.abs() ? r.hi.abs() : r.lo.abs());
        if (m.empty()) {
          if (!c.to_i128(&f.c0)) return;
          continue;
        }
        WordTerm t;
        t.atoms = m;
        if (!c.to_i128(&t.coef)) return;
        f.terms.push_back(std::move(t));
      }
      if (mag.bit_length() > 100 || f.terms.empty()) {
        if (mag.bit_length() > 100) return;
        continue;
      }
      out.push_back(std::move(f));
    }
    out_.word_facts = std::move(out);
    out_.atom_range = std::move(ranges);
  }

  // Linear relaxation of the root facts: every fact, its product with each
  // atom when all monomials of the product already occur in the facts
  // (z >= 0 and p >= 0 give z*p >= 0; p == 0 gives z*p == 0), and the value
  // range of every monomial.  Infeasible over the rationals -> UNSAT.
  bool relaxation_infeasible(const std::vector<std::pair<Poly, Rel>>& facts) const {
    std::set<Mono> present;
    for (auto& [p, rel] : facts)
      for (auto& [m, c] : p)
        if (!m.empty()) present.insert(m);
    if (present.empty()) return false;
    std::set<uint32_t> atoms;
    for (const Mono& m : present) atoms.insert(m.begin(), m.end());
    Relaxation lp;
    auto add_row = [&](const Poly& p, Rel rel) {
      Poly dir;
      BigInt c0;
      for (auto& [m, c] : p) {
        if (m.empty()) c0 = c;
        else dir[m] = c;
      }
      bool ok = true;
      if (rel == Rel::EQ0) {
        Poly neg;
        for (auto& [m, c] : dir) neg[m] = -c;
        ok = lp.add(std::move(neg), -c0);
      }
      return lp.add(std::move(dir), c0) && ok;
    };
    for (auto& [p, rel] : facts) {
      if (!add_row(p, rel)) return true;
      for (uint32_t z : atoms) {
        if (atoms_[z].range.lo < BigInt(0)) continue;
        Poly zp;
        bool inside = true;
        for (auto& [m, c] : p) {
          Mono mz = m;
          mz.insert(std::upper_bound(mz.begin(), mz.end(), z), z);
          if (!present.count(mz)) { inside = false; break; }
          zp[mz] = c;
        }
        if (inside && !add_row(zp, rel)) return true;
      }
    }
    for (const Mono& m : present) {
      Range r = mono_range(m);
      if (!lp.add(Poly{{m, BigInt(1)}}, -r.lo)) return true;
      if (!lp.add(Poly{{m, BigInt(-1)}}, r.hi)) return true;
    }
    return lp.infeasible();
  }

  Poly div_atom(uint64_t i) {
    const scuba_node& x = nodes_[i];
    const Poly& px = polys_[x.a];
    auto key = std::make_pair(px, x.imm);
    auto it = div_pairs_.find(key);
    uint32_t qa, ra;
    if (it != div_pairs_.end()) {
      qa = it->second.first;
      ra = it->second.second;
    } else {
      Range rx = poly_range(px);
      if (rx.lo < BigInt(0)) fail(SCUBA_E_INVALID, "node " + std::to_string(i) + ": divides a value that can be negative");
      BigInt k = BigInt::from_u64(x.imm);
      // Fresh bits for q and r.  Their ranges are the full bit domains: the
      // modular encoding of every key that mentions them must hold any value
      // the bits can take, and the defining facts below pin the true values.
      Atom q, r;
      BigInt rmax = k - BigInt(1);
      if (rx.hi < rmax) rmax = rx.hi;
      uint32_t bq = std::max<uint32_t>(1, BigInt::floor_div(rx.hi, k).bit_length());
      uint32_t br = std::max<uint32_t>(1, rmax.bit_length());
      for (uint32_t b = 0; b < bq; b++) q.bits.push_back(g_.fresh());
      for (uint32_t b = 0; b < br; b++) r.bits.push_back(g_.fresh());
      q.range = {BigInt(0), BigInt::pow2(bq) - BigInt(1)};
      r.range = {BigInt(0), BigInt::pow2(br) - BigInt(1)};
      qa = uint32_t(atoms_.size());
      atoms_.push_back(q);
      ra = uint32_t(atoms_.size());
      atoms_.push_back(r);
      div_pairs_[key] = {qa, ra};
      // x - k*q - r = 0  and  r <= k - 1  (and the bit domains of q, r)
      Poly def = px;
      poly_add_into(def, Poly{{Mono{qa}, k}}, BigInt(-1));
      poly_add_into(def, Poly{{Mono{ra}, BigInt(1)}}, BigInt(-1));
      div_facts_.push_back({def, Rel::EQ0});
      Poly rb{{Mono{}, k - BigInt(1)}};
      poly_add_into(rb, Poly{{Mono{ra}, BigInt(1)}}, BigInt(-1));
      div_facts_.push_back({rb, Rel::GE0});
    }
    return Poly{{Mono{x.op == SCUBA_OP_UDIV ? qa : ra}, BigInt(1)}};
  }

  Range mono_range(const Mono& m) const {
    Range r{BigInt(1), BigInt(1)};
    for (uint32_t a : m) r = range_mul(r, atoms_[a].range);
    return r;
  }
  Range poly_range(const Poly& p) const {
    Range r{BigInt(0), BigInt(0)};
    for (auto& [m, c] : p) r = range_add(r, range_scale(mono_range(m), c));
    return r;
  }

  static Poly substitute(const Poly& p, uint32_t atom, const Poly& expr) {
    Poly out;
    for (auto& [m, c] : p) {
      Mono rest;
      size_t k = 0;
      for (uint32_t a : m) {
        if (a == atom) k++;
        else rest.push_back(a);
      }
      Poly term{{rest, c}};
      for (size_t i = 0; i < k; i++) term = poly_mul(term, expr);
      poly_add_into(out, term, BigInt(1));
    }
    return out;
  }
  static Poly substitute_all(Poly p, const std::vector<std::pair<uint32_t, Poly>>& subs) {
    for (auto& [a, e] : subs) p = substitute(p, a, e);
    return p;
  }

  // p >= 0 or p == 0  ->  bound on the canonical key
  void add_fact(std::map<Poly, Bound>& bounds, const Poly& p, Rel rel) {
    BigInt c0;
    Poly rest;
    for (auto& [m, c] : p) {
      if (m.empty()) c0 = c;
      else rest[m] = c;
    }
    if (rest.empty()) {
      if ((rel == Rel::GE0 && c0 < BigInt(0)) || (rel == Rel::EQ0 && !c0.is_zero())) unsat_ = true;
      return;
    }
    BigInt g;
    for (auto& [m, c] : rest) g = BigInt::gcd(g, c);
    int s = rest.begin()->second.sign();
    Poly key;
    for (auto& [m, c] : rest) key[m] = BigInt::floor_div(c, g) * BigInt(s);
    Bound& b = bounds[key];
    // rest = s*g*key ; fact: s*g*key + c0 (>= | ==) 0
    if (rel == Rel::EQ0) {
      BigInt q, r;
      BigInt::floor_divmod(-c0, g, &q, &r);
      if (!r.is_zero()) { unsat_ = true; return; }
      BigInt v = q * BigInt(s);
      b.lower(v);
      b.upper(v);
    } else if (s > 0) {
      b.lower(BigInt::ceil_div(-c0, g));
    } else {
      b.upper(BigInt::floor_div(c0, g));
    }
  }

  // comparison node -> (a - b) with the relation, given polarity
  bool comparison_fact(uint32_t i, bool pos, Poly* p, Rel* rel) {
    const scuba_node& x = nodes_[i];
    auto diff = [&](uint32_t a, uint32_t b, int64_t k) {
      Poly d = polys_[a];
      poly_add_into(d, polys_[b], BigInt(-1));
      if (k) poly_add_into(d, Poly{{Mono{}, BigInt(k)}}, BigInt(1));
      return d;
    };
    switch (x.op) {
      case SCUBA_OP_LT: *p = pos ? diff(x.b, x.a, -1) : diff(x.a, x.b, 0); *rel = Rel::GE0; return true;
      case SCUBA_OP_LE: *p = pos ? diff(x.b, x.a, 0) : diff(x.a, x.b, -1); *rel = Rel::GE0; return true;
      case SCUBA_OP_GT: *p = pos ? diff(x.a, x.b, -1) : diff(x.b, x.a, 0); *rel = Rel::GE0; return true;
      case SCUBA_OP_GE: *p = pos ? diff(x.a, x.b, 0) : diff(x.b, x.a, -1); *rel = Rel::GE0; return true;
      case SCUBA_OP_EQ: if (pos) { *p = diff(x.a, x.b, 0); *rel = Rel::EQ0; return true; } return false;
      case SCUBA_OP_NE: if (!pos) { *p = diff(x.a, x.b, 0); *rel = Rel::EQ0; return true; } return false;
      default: return false;
    }
  }

  void collect(uint32_t i, bool pos, std::vector<std::pair<uint32_t, bool>>& complex_roots) {
    const scuba_node& x = nodes_[i];
    if (x.op == SCUBA_OP_NOT) { collect(x.a, !pos, complex_roots); return; }
    if ((x.op == SCUBA_OP_AND && pos) || (x.op == SCUBA_OP_OR && !pos)) {
      collect(x.a, pos, complex_roots);
      collect(x.b, pos, complex_roots);
      return;
    }
    Poly p;
    Rel rel;
    if (comparison_fact(i, pos, &p, &rel)) { facts_.push_back({p, rel}); return; }
    complex_roots.push_back({i, pos});
  }

  // key polynomial in two's complement modulo 2^W (W holds its range)
  const BitVec& key_bits(const Poly& key, uint32_t* w_out) {
    Range r = poly_range(key);
    uint32_t w = BigInt::tc_width(r.lo, r.hi);
    *w_out = w;
    auto it = key_cache_.find(key);
    if (it != key_cache_.end()) return it->second;
    BitVec acc(w, kFalse);
    bool first = true;
    for (auto& [m, c] : key) {
      BitVec term = mono_bits(m, w);
      BitVec scaled = g_.mul_const(term, c.abs(), w);
      if (c.neg()) scaled = g_.neg(scaled, w);
      if (first) { acc = scaled; first = false; }
      else acc = g_.add(acc, scaled, w);
    }
    return key_cache_.emplace(key, acc).first->second;
  }

  BitVec mono_bits(const Mono& m, uint32_t w) {
    auto ck = std::make_pair(m, w);
    auto it = mono_cache_.find(ck);
    if (it != mono_cache_.end()) return it->second;
    BitVec acc;
    if (m.empty()) acc = Gates::constant(BigInt(1), w);
    else {
      acc = Gates::resize(atoms_[m[0]].bits, w, false);
      for (size_t i = 1; i < m.size(); i++) {
        Mono prefix(m.begin(), m.begin() + i + 1);
        auto pk = std::make_pair(prefix, w);
        auto pit = mono_cache_.find(pk);
        if (pit != mono_cache_.end()) { acc = pit->second; continue; }
        acc = g_.mul_u(acc, atoms_[m[i]].bits, w);
        mono_cache_.emplace(pk, acc);
      }
    }
    mono_cache_.emplace(ck, acc);
    return acc;
  }

  // signed key -> unsigned word with the sign bit flipped (order preserving)
  static BitVec biased(const BitVec& x) {
    BitVec u = x;
    u.back() = -u.back();
    return u;
  }

  void assert_bound(const Poly& key, const Bound& b) {
    Range kr = poly_range(key);
    bool need_lo = b.has_lo && b.lo > kr.lo;
    bool need_hi = b.has_hi && b.hi < kr.hi;
    if (!need_lo && !need_hi) return;
    uint32_t w;
    BitVec x = biased(key_bits(key, &w));
    BigInt bias = BigInt::pow2(w - 1);
    if (need_lo && need_hi && b.lo == b.hi) {
      BigInt v = b.lo + bias;
      for (uint32_t i = 0; i < w; i++) g_.clause({v.bit(i) ? x[i] : -x[i]});
      return;
    }
    if (need_lo) g_.assert_ge_const(x, b.lo + bias);
    if (need_hi) g_.assert_le_const(x, b.hi + bias);
  }

  // literal of a boolean node used inside a formula
  int32_t bool_lit(uint32_t i) {
    auto it = bool_cache_.find(i);
    if (it != bool_cache_.end()) return it->second;
    const scuba_node& x = nodes_[i];
    int32_t l;
    switch (x.op) {
      case SCUBA_OP_NOT: l = -bool_lit(x.a); break;
      case SCUBA_OP_AND: l = g_.AND(bool_lit(x.a), bool_lit(x.b)); break;
      case SCUBA_OP_OR: l = g_.OR(bool_lit(x.a), bool_lit(x.b)); break;
      default: {
        Poly p;
        Rel rel;
        bool negate = false;
        if (!comparison_fact(i, true, &p, &rel)) {   // NE: not EQ
          comparison_fact(i, false, &p, &rel);
          negate = true;
        }
        l = fact_lit(p, rel);
        if (negate) l = -l;
      }
    }
    bool_cache_[i] = l;
    return l;
  }

  int32_t fact_lit(const Poly& p, Rel rel) {
    BigInt c0;
    Poly rest;
    for (auto& [m, c] : p) {
      if (m.empty()) c0 = c;
      else rest[m] = c;
    }
    if (rest.empty()) {
      bool t = rel == Rel::GE0 ? c0 >= BigInt(0) : c0.is_zero();
      return t ? kTrue : kFalse;
    }
    BigInt g;
    for (auto& [m, c] : rest) g = BigInt::gcd(g, c);
    int s = rest.begin()->second.sign();
    Poly key;
    for (auto& [m, c] : rest) key[m] = BigInt::floor_div(c, g) * BigInt(s);
    Range kr = poly_range(key);
    uint32_t w;
    if (rel == Rel::EQ0) {
      BigInt q, r;
      BigInt::floor_divmod(-c0, g, &q, &r);
      if (!r.is_zero()) return kFalse;
      BigInt v = q * BigInt(s);
      if (v < kr.lo || v > kr.hi) return kFalse;
      BitVec x = biased(key_bits(key, &w));
      return g_.eq_const_gate(x, v + BigInt::pow2(w - 1));
    }
    if (s > 0) {  // key >= L
      BigInt L = BigInt::ceil_div(-c0, g);
      if (L <= kr.lo) return kTrue;
      if (L > kr.hi) return kFalse;
      BitVec x = biased(key_bits(key, &w));
      return g_.ge_const_gate(x, L + BigInt::pow2(w - 1));
    }
    BigInt U = BigInt::floor_div(c0, g);  // key <= U  <=>  not (key >= U+1)
    if (U >= kr.hi) return kTrue;
    if (U < kr.lo) return kFalse;
    BitVec x = biased(key_bits(key, &w));
    return -g_.ge_const_gate(x, U + BigInt(1) + BigInt::pow2(w - 1));
  }

  // ---------------------------------------------------------- structural
  // Each node is a circuit of its own (no normalisation): widths from value
  // ranges, comparisons through the sign or zero test of a - b.
  // ---------------------------------------------------------- modular
  // Every integer node is an unsigned m-bit word: ADD, SUB, MUL and SHL are
  // taken modulo 2^m, UDIV / UREM by a constant are the unsigned quotient
  // and remainder, comparisons are unsigned (machine integers of m bits).
  // Machine-integer queries refuted by the exact method.  An arithmetic node
  // whose exact value provably stays in [0, 2^m) computes the same m-bit
  // word as the exact integer (it never wraps); every other arithmetic node
  // is replaced by a fresh m-bit input (its wrapped value is some m-bit
  // word).  The resulting exact-integer query has every behaviour of the
  // machine-integer one (comparisons of values in [0, 2^m) are the unsigned
  // ones), so refuting it at the root (normalisation, bounds, relaxation)
  // refutes the machine-integer query.  Value ranges start from the input
  // widths and are narrowed, to a fixpoint, by the comparisons that the
  // roots assert: a guard idx < N bounds even a wrapping idx, which is what
  // shows that idx * s and N * s cannot wrap.  A root comparison that no
  // value pair can meet refutes the query directly.
  bool wrap_abstraction_unsat(uint32_t m) {
    const BigInt top = BigInt::pow2(m) - BigInt(1);
    const Range full{BigInt(0), top};
    // the comparisons the roots assert (through conjunctions)
    struct Fact { uint32_t op, a, b; };
    std::vector<Fact> facts;
    std::vector<uint32_t> todo(roots_, roots_ + nr_);
    while (!todo.empty()) {
      const uint32_t i = todo.back();
      todo.pop_back();
      const scuba_node& x = nodes_[i];
      if (x.op == SCUBA_OP_AND) { todo.push_back(x.a); todo.push_back(x.b); }
      else if (x.op >= SCUBA_OP_LT && x.op <= SCUBA_OP_EQ) facts.push_back({x.op, x.a, x.b});
    }
    std::vector<Range> nar(n_, full);     // narrowing of each integer node by the facts
    std::vector<Range> r(n_);
    std::vector<char> exact(n_, 1);
    for (uint32_t iter = 0; iter < 16; iter++) {
      for (uint64_t i = 0; i < n_; i++) {
        const scuba_node& x = nodes_[i];
        Range e;
        bool arith = false;
        switch (x.op) {
          case SCUBA_OP_VAR: e = {BigInt(0), BigInt::pow2(x.width) - BigInt(1)}; break;
          case SCUBA_OP_CONST: {
            BigInt c;
            BigInt::floor_divmod(BigInt::from_u64(x.imm), BigInt::pow2(m), nullptr, &c);
            e = {c, c};
            break;
          }
          case SCUBA_OP_ADD: e = range_add(r[x.a], r[x.b]); arith = true; break;
          case SCUBA_OP_SUB: e = {r[x.a].lo - r[x.b].hi, r[x.a].hi - r[x.b].lo}; arith = true; break;
          case SCUBA_OP_MUL: e = range_mul(r[x.a], r[x.b]); arith = true; break;
          case SCUBA_OP_SHL: e = range_scale(r[x.a], BigInt::pow2(uint32_t(x.imm))); arith = true; break;
          case SCUBA_OP_UDIV: {
            const BigInt k = BigInt::from_u64(x.imm);
            BigInt lo, hi;
            BigInt::floor_divmod(r[x.a].lo, k, &lo, nullptr);
            BigInt::floor_divmod(r[x.a].hi, k, &hi, nullptr);
            e = {lo, hi};
            break;
          }
          case SCUBA_OP_UREM: {
            const BigInt k = BigInt::from_u64(x.imm);
            e = r[x.a].hi < k ? r[x.a] : Range{BigInt(0), k - BigInt(1)};
            break;
          }
          default: continue;   // boolean nodes
        }
        exact[i] = !arith || (e.lo >= BigInt(0) && e.hi <= top);
        if (!exact[i]) e = full;
        // the facts' narrowing
        if (nar[i].lo > e.lo) e.lo = nar[i].lo;
        if (nar[i].hi < e.hi) e.hi = nar[i].hi;
        if (e.lo > e.hi) return true;   // no value of this node meets the roots
        r[i] = e;
      }
      bool changed = false;
      auto tighten = [&](uint32_t i, const BigInt* lo, const BigInt* hi) {
        if (lo && *lo > nar[i].lo) { nar[i].lo = *lo; changed = true; }
        if (hi && *hi < nar[i].hi) { nar[i].hi = *hi; changed = true; }
      };
      for (const Fact& f : facts) {
        uint32_t a = f.a, b = f.b;
        uint32_t op = f.op;
        if (op == SCUBA_OP_GT) { std::swap(a, b); op = SCUBA_OP_LT; }
        if (op == SCUBA_OP_GE) { std::swap(a, b); op = SCUBA_OP_LE; }
        const BigInt d = op == SCUBA_OP_LT ? BigInt(1) : BigInt(0);
        if (op == SCUBA_OP_EQ) {
          tighten(a, &r[b].lo, &r[b].hi);
          tighten(b, &r[a].lo, &r[a].hi);
        } else {   // a + d <= b
          const BigInt ahi = r[b].hi - d, blo = r[a].lo + d;
          tighten(a, nullptr, &ahi);
          tighten(b, &blo, nullptr);
        }
      }
      if (!changed) break;
    }
    // the exact-integer query: wrapping nodes become fresh m-bit inputs
    std::vector<scuba_node> nodes(nodes_, nodes_ + n_);
    uint32_t nv = 0;
    bool any_abstract = false;
    for (uint64_t i = 0; i < n_; i++) {
      scuba_node& x = nodes[i];
      if (x.op == SCUBA_OP_VAR) {
        x.imm = nv++;
      } else if (x.op == SCUBA_OP_CONST) {
        x.imm = x.imm & (m == 64 ? ~0ull : ((uint64_t(1) << m) - 1));
      } else if (!exact[i]) {
        x = scuba_node{SCUBA_OP_VAR, 0, 0, m, nv++};
        any_abstract = true;
      }
    }
    (void)any_abstract;
    CnfQuery probe;
    Encoder e(nodes.data(), n_, roots_, nr_, 0, probe);
    e.run();
    return probe.root_unsat;
  }

  void run_wrap(uint32_t m) {
    std::vector<BitVec> bv(n_);
    std::vector<int32_t> bl(n_, kFalse);
    std::map<std::pair<BitVec, BitVec>, std::pair<int32_t, int32_t>> cmp_cache;
    const BigInt mod = BigInt::pow2(m);
    for (uint64_t i = 0; i < n_; i++) {
      const scuba_node& x = nodes_[i];
      switch (x.op) {
        case SCUBA_OP_VAR: bv[i] = Gates::resize(atoms_[x.imm].bits, m, false); break;
        case SCUBA_OP_CONST: {
          BigInt r;
          BigInt::floor_divmod(BigInt::from_u64(x.imm), mod, nullptr, &r);
          bv[i] = Gates::constant(r, m);
          break;
        }
        case SCUBA_OP_ADD: bv[i] = g_.add(bv[x.a], bv[x.b], m); break;
        case SCUBA_OP_SUB: bv[i] = g_.add(bv[x.a], g_.neg(bv[x.b], m), m); break;
        case SCUBA_OP_MUL: bv[i] = g_.mul_u(bv[x.a], bv[x.b], m); break;
        case SCUBA_OP_SHL: {
          BitVec b(std::min<uint64_t>(x.imm, m), kFalse);
          for (uint32_t j = 0; b.size() < m; j++) b.push_back(bv[x.a][j]);
          bv[i] = b;
          break;
        }
        case SCUBA_OP_UDIV: case SCUBA_OP_UREM: {
          const BigInt k = BigInt::from_u64(x.imm);
          if (k >= mod) {   // every m-bit value is below k
            bv[i] = x.op == SCUBA_OP_UDIV ? Gates::constant(BigInt(0), m) : bv[x.a];
            break;
          }
          // fresh q (m bits) and r (< k): a == q*k + r exactly, r < k
          BitVec qb, rb;
          for (uint32_t b = 0; b < m; b++) qb.push_back(g_.fresh());
          const uint32_t rw = std::max<uint32_t>(1, (k - BigInt(1)).bit_length());
          for (uint32_t b = 0; b < rw; b++) rb.push_back(g_.fresh());
          const uint32_t w = m + k.bit_length() + 1;
          BitVec sum = g_.add(g_.mul_const(Gates::resize(qb, w, false), k, w), Gates::resize(rb, w, false), w);
          BitVec xa = Gates::resize(bv[x.a], w, false);
          for (uint32_t b = 0; b < w; b++) g_.clause({-g_.XOR(xa[b], sum[b])});
          g_.clause({-g_.ge_const_gate(rb, k)});
          bv[i] = x.op == SCUBA_OP_UDIV ? qb : Gates::resize(rb, m, false);
          break;
        }
        case SCUBA_OP_LT: case SCUBA_OP_LE: case SCUBA_OP_GT: case SCUBA_OP_GE:
        case SCUBA_OP_EQ: case SCUBA_OP_NE: {
          uint32_t a = x.a, b = x.b;
          if (x.op == SCUBA_OP_GT || x.op == SCUBA_OP_LE) std::swap(a, b);
          // unsigned: the borrow of a - b over m + 1 bits, and equality; one
          // comparator per pair of words (nodes with the same bits share it,
          // so comparing a word with itself twice is one gate)
          auto key = std::make_pair(bv[a], bv[b]);
          auto hit = cmp_cache.find(key);
          if (hit == cmp_cache.end()) {
            BitVec d = g_.add(Gates::resize(bv[a], m + 1, false),
                              g_.neg(Gates::resize(bv[b], m + 1, false), m + 1), m + 1);
            int32_t e = kTrue;
            for (uint32_t j = 0; j < m; j++) e = g_.AND(e, -g_.XOR(bv[a][j], bv[b][j]));
            hit = cmp_cache.emplace(key, std::make_pair(d.back(), e)).first;
          }
          const int32_t lt = hit->second.first, eq = hit->second.second;
          switch (x.op) {
            case SCUBA_OP_LT: case SCUBA_OP_GT: bl[i] = lt; break;
            case SCUBA_OP_LE: case SCUBA_OP_GE: bl[i] = -lt; break;
            case SCUBA_OP_EQ: bl[i] = eq; break;
            default: bl[i] = -eq; break;
          }
          break;
        }
        case SCUBA_OP_AND: bl[i] = g_.AND(bl[x.a], bl[x.b]); break;
        case SCUBA_OP_OR: bl[i] = g_.OR(bl[x.a], bl[x.b]); break;
        case SCUBA_OP_NOT: bl[i] = -bl[x.a]; break;
        default: break;
      }
    }
    for (uint64_t r = 0; r < nr_; r++) g_.clause({bl[roots_[r]]});
  }

  void run_structural() {
    std::vector<Range> rg(n_);
    std::vector<BitVec> bv(n_);
    std::vector<int32_t> bl(n_, kFalse);
    std::vector<std::pair<BitVec, uint32_t>> dummy;
    for (uint64_t i = 0; i < n_; i++) {
      const scuba_node& x = nodes_[i];
      switch (x.op) {
        case SCUBA_OP_VAR: {
          rg[i] = atoms_[x.imm].range;
          bv[i] = atoms_[x.imm].bits;
          bv[i].push_back(kFalse);  // sign bit
          break;
        }
        case SCUBA_OP_CONST: {
          BigInt v = BigInt::from_u64(x.imm);
          rg[i] = {v, v};
          bv[i] = Gates::constant(v, BigInt::tc_width(v, v));
          break;
        }
        case SCUBA_OP_ADD: case SCUBA_OP_SUB: {
          Range rb = rg[x.b];
          if (x.op == SCUBA_OP_SUB) rb = {-rg[x.b].hi, -rg[x.b].lo};
          rg[i] = range_add(rg[x.a], rb);
          uint32_t w = BigInt::tc_width(rg[i].lo, rg[i].hi);
          uint32_t wi = std::max<uint32_t>({w, uint32_t(bv[x.a].size()), uint32_t(bv[x.b].size())}) + 1;
          BitVec a = Gates::resize(bv[x.a], wi, true), b = Gates::resize(bv[x.b], wi, true);
          if (x.op == SCUBA_OP_SUB) b = g_.neg(b, wi);
          bv[i] = Gates::resize(g_.add(a, b, wi), w, true);
          break;
        }
        case SCUBA_OP_MUL: {
          rg[i] = range_mul(rg[x.a], rg[x.b]);
          uint32_t w = BigInt::tc_width(rg[i].lo, rg[i].hi);
          uint32_t wi = std::max<uint32_t>({w, uint32_t(bv[x.a].size()), uint32_t(bv[x.b].size())});
          BitVec a = Gates::resize(bv[x.a], wi, true), b = Gates::resize(bv[x.b], wi, true);
          bv[i] = Gates::resize(g_.mul_u(a, b, wi), w, true);
          break;
        }
        case SCUBA_OP_SHL: {
          rg[i] = {rg[x.a].lo.shl(uint32_t(x.imm)), rg[x.a].hi.shl(uint32_t(x.imm))};
          BitVec b(x.imm, kFalse);
          b.insert(b.end(), bv[x.a].begin(), bv[x.a].end());
          bv[i] = b;
          break;
        }
        case SCUBA_OP_UDIV: case SCUBA_OP_UREM: {
          if (rg[x.a].lo < BigInt(0)) fail(SCUBA_E_INVALID, "node " + std::to_string(i) + ": divides a value that can be negative");
          BigInt k = BigInt::from_u64(x.imm);
          Range rq{BigInt::floor_div(rg[x.a].lo, k), BigInt::floor_div(rg[x.a].hi, k)};
          BigInt rmax = k - BigInt(1);
          if (rg[x.a].hi < rmax) rmax = rg[x.a].hi;
          BitVec qb, rb;
          for (uint32_t b = 0; b < std::max<uint32_t>(1, rq.hi.bit_length()); b++) qb.push_back(g_.fresh());
          for (uint32_t b = 0; b < std::max<uint32_t>(1, rmax.bit_length()); b++) rb.push_back(g_.fresh());
          qb.push_back(kFalse);
          rb.push_back(kFalse);
          // x == q*k + r  and  r < k
          uint32_t w = std::max<uint32_t>(uint32_t(bv[x.a].size()), uint32_t(qb.size()) + k.bit_length() + 1) + 1;
          BitVec prod = g_.mul_const(Gates::resize(qb, w, true), k, w);
          BitVec sum = g_.add(prod, Gates::resize(rb, w, true), w);
          BitVec xa = Gates::resize(bv[x.a], w, true);
          for (uint32_t b = 0; b < w; b++) {
            int32_t e = -g_.XOR(xa[b], sum[b]);
            g_.clause({e});
          }
          BitVec ru = Gates::resize(rb, uint32_t(rb.size()), false);
          g_.clause({-g_.ge_const_gate(ru, k)});
          if (x.op == SCUBA_OP_UDIV) { rg[i] = rq; bv[i] = qb; }
          else { rg[i] = {BigInt(0), rmax}; bv[i] = rb; }
          break;
        }
        case SCUBA_OP_LT: case SCUBA_OP_LE: case SCUBA_OP_GT: case SCUBA_OP_GE:
        case SCUBA_OP_EQ: case SCUBA_OP_NE: {
          uint32_t a = x.a, b = x.b;
          bool swap = x.op == SCUBA_OP_GT || x.op == SCUBA_OP_LE;
          if (swap) std::swap(a, b);
          uint32_t w = std::max<uint32_t>(uint32_t(bv[a].size()), uint32_t(bv[b].size())) + 1;
          BitVec d = g_.add(Gates::resize(bv[a], w, true), g_.neg(Gates::resize(bv[b], w, true), w), w);
          int32_t lt = d.back();  // a - b < 0
          int32_t eq = kTrue;
          for (int32_t l : d) eq = g_.AND(eq, -l);
          switch (x.op) {
            case SCUBA_OP_LT: case SCUBA_OP_GT: bl[i] = lt; break;     // a<b ; b<a
            case SCUBA_OP_LE: case SCUBA_OP_GE: bl[i] = -lt; break;    // !(b<a) ; !(a<b)
            case SCUBA_OP_EQ: bl[i] = eq; break;
            default: bl[i] = -eq; break;
          }
          break;
        }
        case SCUBA_OP_AND: bl[i] = g_.AND(bl[x.a], bl[x.b]); break;
        case SCUBA_OP_OR: bl[i] = g_.OR(bl[x.a], bl[x.b]); break;
        case SCUBA_OP_NOT: bl[i] = -bl[x.a]; break;
        default: break;
      }
    }
    for (uint64_t r = 0; r < nr_; r++) g_.clause({bl[roots_[r]]});
  }

  const scuba_node* nodes_;
  uint64_t n_;
  const uint32_t* roots_;
  uint64_t nr_;
  uint32_t flags_;
  CnfQuery& out_;
  Gates g_;
  std::vector<Atom> atoms_;
  std::vector<Poly> polys_;
  std::map<std::pair<Poly, uint64_t>, std::pair<uint32_t, uint32_t>> div_pairs_;
  std::vector<std::pair<Poly, Rel>> div_facts_;
  std::vector<std::pair<Poly, Rel>> facts_;
  std::map<Poly, Bound> bounds_;
  std::map<Poly, BitVec> key_cache_;
  std::map<std::pair<Mono, uint32_t>, BitVec> mono_cache_;
  std::map<uint32_t, int32_t> bool_cache_;
  bool unsat_ = false;
};

}  // namespace

CnfQuery bitblast_query(const scuba_node* nodes, uint64_t n_nodes, const uint32_t* roots,
                        uint64_t n_roots, uint32_t flags) {
  CnfQuery q;
  Encoder e(nodes, n_nodes, roots, n_roots, flags, q);
  e.run();
  q.has_query = true;
  q.nodes.assign(nodes, nodes + n_nodes);
  q.roots.assign(roots, roots + n_roots);
  if (!q.root_unsat) q.build_occurrences();   // a query decided at the root is not split
  return q;
}

// A counting sort of the literal occurrences by literal index.
void CnfQuery::build_occurrences() {
  const size_t nli = 2 * (size_t(n_vars) + 1);
  occ_off.assign(nli + 1, 0);
  for (int32_t x : lits) occ_off[2 * size_t(x > 0 ? x : -x) + (x < 0) + 1]++;
  for (size_t i = 0; i < nli; i++) occ_off[i + 1] += occ_off[i];
  occ.resize(lits.size());
  std::vector<uint32_t> fill(occ_off.begin(), occ_off.end() - 1);
  const uint64_t nc = n_clauses();
  for (uint64_t c = 0; c < nc; c++)
    for (uint64_t i = off[c]; i < off[c + 1]; i++) {
      const int32_t x = lits[i];
      occ[fill[2 * size_t(x > 0 ? x : -x) + (x < 0)]++] = uint32_t(c);
    }
}

}  // namespace scuba
