// Integer-level witness check: the decoded inputs must satisfy the original
// query (before normalisation) under exact integer arithmetic, i.e. the
// access really is out of bounds for that input (Sec. 5.2: the solver
// provides values that satisfy every constraint).
#include "bigint.hpp"
#include "common.hpp"

namespace scuba {

namespace {
// The same check with machine integers of m bits (every integer node taken
// modulo 2^m, comparisons unsigned).
bool wrap_check_query(const CnfQuery& q, const std::vector<uint64_t>& values, uint32_t m) {
  const uint64_t mask = m >= 64 ? ~uint64_t(0) : (uint64_t(1) << m) - 1;
  std::vector<uint64_t> iv(q.nodes.size(), 0);
  std::vector<char> bv(q.nodes.size(), 0);
  for (size_t i = 0; i < q.nodes.size(); i++) {
    const scuba_node& x = q.nodes[i];
    switch (x.op) {
      case SCUBA_OP_VAR: {
        if (x.imm >= values.size()) return false;
        const uint64_t v = values[x.imm];
        if (x.width < 64 && (v >> x.width)) return false;
        iv[i] = v & mask;
        break;
      }
      case SCUBA_OP_CONST: iv[i] = x.imm & mask; break;
      case SCUBA_OP_ADD: iv[i] = (iv[x.a] + iv[x.b]) & mask; break;
      case SCUBA_OP_SUB: iv[i] = (iv[x.a] - iv[x.b]) & mask; break;
      case SCUBA_OP_MUL: iv[i] = uint64_t((unsigned __int128)iv[x.a] * iv[x.b]) & mask; break;
      case SCUBA_OP_SHL: iv[i] = x.imm >= 64 ? 0 : (iv[x.a] << x.imm) & mask; break;
      case SCUBA_OP_UDIV: iv[i] = iv[x.a] / x.imm; break;
      case SCUBA_OP_UREM: iv[i] = iv[x.a] % x.imm; break;
      case SCUBA_OP_LT: bv[i] = iv[x.a] < iv[x.b]; break;
      case SCUBA_OP_LE: bv[i] = iv[x.a] <= iv[x.b]; break;
      case SCUBA_OP_GT: bv[i] = iv[x.a] > iv[x.b]; break;
      case SCUBA_OP_GE: bv[i] = iv[x.a] >= iv[x.b]; break;
      case SCUBA_OP_EQ: bv[i] = iv[x.a] == iv[x.b]; break;
      case SCUBA_OP_NE: bv[i] = iv[x.a] != iv[x.b]; break;
      case SCUBA_OP_AND: bv[i] = bv[x.a] && bv[x.b]; break;
      case SCUBA_OP_OR: bv[i] = bv[x.a] || bv[x.b]; break;
      case SCUBA_OP_NOT: bv[i] = !bv[x.a]; break;
      default: return false;
    }
  }
  for (uint32_t r : q.roots)
    if (!bv[r]) return false;
  return true;
}
}  // namespace

bool int_check_query(const CnfQuery& q, const std::vector<uint64_t>& values) {
  if (!q.has_query) return true;
  if (q.wrap_bits) return wrap_check_query(q, values, q.wrap_bits);
  std::vector<BigInt> iv(q.nodes.size());
  std::vector<char> bv(q.nodes.size(), 0);
  for (size_t i = 0; i < q.nodes.size(); i++) {
    const scuba_node& x = q.nodes[i];
    switch (x.op) {
      case SCUBA_OP_VAR: {
        if (x.imm >= values.size()) return false;
        uint64_t v = values[x.imm];
        if (x.width < 64 && (v >> x.width)) return false;
        iv[i] = BigInt::from_u64(v);
        break;
      }
      case SCUBA_OP_CONST: iv[i] = BigInt::from_u64(x.imm); break;
      case SCUBA_OP_ADD: iv[i] = iv[x.a] + iv[x.b]; break;
      case SCUBA_OP_SUB: iv[i] = iv[x.a] - iv[x.b]; break;
      case SCUBA_OP_MUL: iv[i] = iv[x.a] * iv[x.b]; break;
      case SCUBA_OP_SHL: iv[i] = iv[x.a].shl(uint32_t(x.imm)); break;
      case SCUBA_OP_UDIV: case SCUBA_OP_UREM: {
        if (iv[x.a] < BigInt(0)) return false;
        BigInt qq, rr;
        BigInt::floor_divmod(iv[x.a], BigInt::from_u64(x.imm), &qq, &rr);
        iv[i] = x.op == SCUBA_OP_UDIV ? qq : rr;
        break;
      }
      case SCUBA_OP_LT: bv[i] = iv[x.a] < iv[x.b]; break;
      case SCUBA_OP_LE: bv[i] = iv[x.a] <= iv[x.b]; break;
      case SCUBA_OP_GT: bv[i] = iv[x.a] > iv[x.b]; break;
      case SCUBA_OP_GE: bv[i] = iv[x.a] >= iv[x.b]; break;
      case SCUBA_OP_EQ: bv[i] = iv[x.a] == iv[x.b]; break;
      case SCUBA_OP_NE: bv[i] = iv[x.a] != iv[x.b]; break;
      case SCUBA_OP_AND: bv[i] = bv[x.a] && bv[x.b]; break;
      case SCUBA_OP_OR: bv[i] = bv[x.a] || bv[x.b]; break;
      case SCUBA_OP_NOT: bv[i] = !bv[x.a]; break;
      default: return false;
    }
  }
  for (uint32_t r : q.roots)
    if (!bv[r]) return false;
  return true;
}

}  // namespace scuba
