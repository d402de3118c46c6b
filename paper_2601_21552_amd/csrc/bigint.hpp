// Small arbitrary-precision signed integer (sign + base-2^32 magnitude).
// Used for exact polynomial coefficients, value ranges and the integer-level
// witness check; every query quantity is an exact integer (no wrap-around).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace scuba {

class BigInt {
 public:
  BigInt() = default;
  BigInt(int64_t v) { set_i64(v); }           // NOLINT (implicit by design)
  static BigInt from_u64(uint64_t v) {
    BigInt r;
    if (v) { r.mag_.push_back(uint32_t(v)); if (v >> 32) r.mag_.push_back(uint32_t(v >> 32)); }
    return r;
  }
  static BigInt pow2(uint32_t e) {
    BigInt r;
    r.mag_.assign(e / 32 + 1, 0);
    r.mag_[e / 32] = 1u << (e % 32);
    return r;
  }

  bool is_zero() const { return mag_.empty(); }
  bool neg() const { return neg_; }
  int sign() const { return is_zero() ? 0 : (neg_ ? -1 : 1); }

  // number of bits of |x| (0 for zero)
  uint32_t bit_length() const {
    if (mag_.empty()) return 0;
    uint32_t top = mag_.back();
    return uint32_t(mag_.size() - 1) * 32 + (32 - __builtin_clz(top));
  }
  bool bit(uint32_t i) const {  // bit i of |x|
    size_t w = i / 32;
    return w < mag_.size() && ((mag_[w] >> (i % 32)) & 1u);
  }
  // bit i of the two's complement representation (infinite sign extension)
  bool tc_bit(uint32_t i) const {
    if (!neg_) return bit(i);
    BigInt t = -(*this) - BigInt(1);  // ~x = -x - 1 ; bit of x = !bit(~x)
    return !t.bit(i);
  }
  bool fits_i64() const { return bit_length() <= 63; }
  // value as a 128-bit integer when |x| < 2^bits (bits <= 126)
  bool to_i128(__int128* out, uint32_t bits = 100) const {
    if (bit_length() > bits) return false;
    unsigned __int128 m = 0;
    for (size_t i = mag_.size(); i-- > 0;) m = (m << 32) | mag_[i];
    *out = neg_ ? -(__int128)m : (__int128)m;
    return true;
  }
  int64_t to_i64() const {
    uint64_t m = 0;
    if (mag_.size() > 0) m |= mag_[0];
    if (mag_.size() > 1) m |= uint64_t(mag_[1]) << 32;
    return neg_ ? -int64_t(m) : int64_t(m);
  }
  uint64_t low_u64() const {  // |x| mod 2^64
    uint64_t m = 0;
    if (mag_.size() > 0) m |= mag_[0];
    if (mag_.size() > 1) m |= uint64_t(mag_[1]) << 32;
    return m;
  }

  BigInt operator-() const { BigInt r = *this; if (!r.is_zero()) r.neg_ = !r.neg_; return r; }
  BigInt abs() const { BigInt r = *this; r.neg_ = false; return r; }

  friend BigInt operator+(const BigInt& a, const BigInt& b) {
    if (a.neg_ == b.neg_) { BigInt r; r.mag_ = add_mag(a.mag_, b.mag_); r.neg_ = a.neg_; r.trim(); return r; }
    int c = cmp_mag(a.mag_, b.mag_);
    if (c == 0) return BigInt();
    BigInt r;
    if (c > 0) { r.mag_ = sub_mag(a.mag_, b.mag_); r.neg_ = a.neg_; }
    else { r.mag_ = sub_mag(b.mag_, a.mag_); r.neg_ = b.neg_; }
    r.trim();
    return r;
  }
  friend BigInt operator-(const BigInt& a, const BigInt& b) { return a + (-b); }
  friend BigInt operator*(const BigInt& a, const BigInt& b) {
    BigInt r;
    if (a.is_zero() || b.is_zero()) return r;
    r.mag_.assign(a.mag_.size() + b.mag_.size(), 0);
    for (size_t i = 0; i < a.mag_.size(); i++) {
      uint64_t carry = 0;
      for (size_t j = 0; j < b.mag_.size(); j++) {
        uint64_t t = uint64_t(a.mag_[i]) * b.mag_[j] + r.mag_[i + j] + carry;
        r.mag_[i + j] = uint32_t(t);
        carry = t >> 32;
      }
      size_t k = i + b.mag_.size();
      while (carry) {
        uint64_t t = uint64_t(r.mag_[k]) + carry;
        r.mag_[k++] = uint32_t(t);
        carry = t >> 32;
      }
    }
    r.neg_ = a.neg_ != b.neg_;
    r.trim();
    return r;
  }
  BigInt shl(uint32_t k) const { return (*this) * pow2(k); }

  // floor division and the matching non-negative remainder (d > 0 required
  // for the remainder to be non-negative; d != 0 always)
  static void floor_divmod(const BigInt& n, const BigInt& d, BigInt* q, BigInt* r) {
    BigInt qa, ra;
    divmod_mag(n.abs(), d.abs(), &qa, &ra);   // |n| = qa*|d| + ra
    // truncated quotient sign
    bool qneg = n.neg_ != d.neg_;
    BigInt tq = qneg ? -qa : qa;
    BigInt tr = n.neg_ ? -ra : ra;            // n = tq*d + tr, sign(tr) = sign(n)
    if (!tr.is_zero() && (tr.neg_ != d.neg_)) { tq = tq - BigInt(1); tr = tr + d; }
    if (q) *q = tq;
    if (r) *r = tr;
  }
  static BigInt floor_div(const BigInt& n, const BigInt& d) { BigInt q; floor_divmod(n, d, &q, nullptr); return q; }
  static BigInt ceil_div(const BigInt& n, const BigInt& d) { return -floor_div(-n, d); }
  static BigInt gcd(BigInt a, BigInt b) {
    a = a.abs(); b = b.abs();
    while (!b.is_zero()) { BigInt r; floor_divmod(a, b, nullptr, &r); a = b; b = r; }
    return a;
  }

  friend int cmp(const BigInt& a, const BigInt& b) {
    if (a.sign() != b.sign()) return a.sign() < b.sign() ? -1 : 1;
    int c = cmp_mag(a.mag_, b.mag_);
    return a.neg_ ? -c : c;
  }
  friend bool operator==(const BigInt& a, const BigInt& b) { return cmp(a, b) == 0; }
  friend bool operator!=(const BigInt& a, const BigInt& b) { return cmp(a, b) != 0; }
  friend bool operator<(const BigInt& a, const BigInt& b) { return cmp(a, b) < 0; }
  friend bool operator<=(const BigInt& a, const BigInt& b) { return cmp(a, b) <= 0; }
  friend bool operator>(const BigInt& a, const BigInt& b) { return cmp(a, b) > 0; }
  friend bool operator>=(const BigInt& a, const BigInt& b) { return cmp(a, b) >= 0; }

  // minimal two's complement width holding every value of [lo, hi]
  static uint32_t tc_width(const BigInt& lo, const BigInt& hi) {
    uint32_t w = 1;
    auto need = [](const BigInt& v) -> uint32_t {
      if (!v.neg_) return v.bit_length() + 1;              // sign bit 0
      BigInt t = (-v) - BigInt(1);                          // -v-1 >= 0
      return t.bit_length() + 1;
    };
    w = std::max(w, need(lo));
    w = std::max(w, need(hi));
    return w;
  }

  std::string str() const {
    if (is_zero()) return "0";
    std::vector<uint32_t> m = mag_;
    std::string s;
    while (!m.empty()) {
      uint64_t rem = 0;
      for (size_t i = m.size(); i-- > 0;) {
        uint64_t cur = (rem << 32) | m[i];
        m[i] = uint32_t(cur / 10);
        rem = cur % 10;
      }
      s.push_back(char('0' + rem));
      while (!m.empty() && m.back() == 0) m.pop_back();
    }
    if (neg_) s.push_back('-');
    return std::string(s.rbegin(), s.rend());
  }

  // ordering for use as a map key
  bool operator_less_key(const BigInt& o) const { return cmp(*this, o) < 0; }

 private:
  void set_i64(int64_t v) {
    mag_.clear();
    neg_ = v < 0;
    uint64_t m = neg_ ? uint64_t(0) - uint64_t(v) : uint64_t(v);
    if (m) { mag_.push_back(uint32_t(m)); if (m >> 32) mag_.push_back(uint32_t(m >> 32)); }
  }
  void trim() { while (!mag_.empty() && mag_.back() == 0) mag_.pop_back(); if (mag_.empty()) neg_ = false; }
  static int cmp_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
    if (a.size() != b.size()) return a.size() < b.size() ? -1 : 1;
    for (size_t i = a.size(); i-- > 0;)
      if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
    return 0;
  }
  static std::vector<uint32_t> add_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
    std::vector<uint32_t> r(std::max(a.size(), b.size()) + 1, 0);
    uint64_t carry = 0;
    for (size_t i = 0; i < r.size(); i++) {
      uint64_t t = carry;
      if (i < a.size()) t += a[i];
      if (i < b.size()) t += b[i];
      r[i] = uint32_t(t);
      carry = t >> 32;
    }
    return r;
  }
  static std::vector<uint32_t> sub_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {  // a >= b
    std::vector<uint32_t> r(a.size(), 0);
    int64_t borrow = 0;
    for (size_t i = 0; i < a.size(); i++) {
      int64_t t = int64_t(a[i]) - borrow - (i < b.size() ? int64_t(b[i]) : 0);
      borrow = t < 0;
      if (t < 0) t += (int64_t(1) << 32);
      r[i] = uint32_t(t);
    }
    return r;
  }
  static void divmod_mag(const BigInt& n, const BigInt& d, BigInt* q, BigInt* r) {  // n, d >= 0, d > 0
    BigInt quo, rem;
    uint32_t nb = n.bit_length();
    quo.mag_.assign(n.mag_.size() + 1, 0);
    for (uint32_t i = nb; i-- > 0;) {
      rem = rem.shl(1);
      if (n.bit(i)) rem = rem + BigInt(1);
      if (rem >= d) { rem = rem - d; quo.mag_[i / 32] |= 1u << (i % 32); }
    }
    quo.trim();
    *q = quo;
    *r = rem;
  }

  std::vector<uint32_t> mag_;
  bool neg_ = false;
};

}  // namespace scuba
