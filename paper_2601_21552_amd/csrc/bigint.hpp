// Small arbitrary-precision signed integer (sign + base-2^32 magnitude).
// Used for exact polynomial coefficients, value ranges and the integer-level
// witness check; every query quantity is an exact integer (no wrap-around).
// Magnitudes of up to four limbs (128 bits, the common case) live inside the
// object; longer ones move to the heap.  Products and quotients of operands
// that fit 128 bits use native 128-bit arithmetic.
#pragma once
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

namespace scuba {

// Limb storage with four inline limbs.
class Limbs {
 public:
  Limbs() = default;
  Limbs(const Limbs& o) { copy_from(o); }
  Limbs(Limbs&& o) noexcept { move_from(o); }
  Limbs& operator=(const Limbs& o) {
    if (this != &o) { release(); copy_from(o); }
    return *this;
  }
  Limbs& operator=(Limbs&& o) noexcept {
    if (this != &o) { release(); move_from(o); }
    return *this;
  }
  ~Limbs() { release(); }

  size_t size() const { return n_; }
  bool empty() const { return n_ == 0; }
  uint32_t* data() { return p_; }
  const uint32_t* data() const { return p_; }
  uint32_t& operator[](size_t i) { return p_[i]; }
  uint32_t operator[](size_t i) const { return p_[i]; }
  uint32_t back() const { return p_[n_ - 1]; }
  void clear() { n_ = 0; }
  void pop_back() { n_--; }
  void push_back(uint32_t v) {
    reserve(n_ + 1);
    p_[n_++] = v;
  }
  void assign(size_t n, uint32_t v) {
    reserve(n);
    std::fill(p_, p_ + n, v);
    n_ = uint32_t(n);
  }

 private:
  void reserve(size_t n) {
    if (n <= cap_) return;
    size_t c = std::max<size_t>(n, 2 * size_t(cap_));
    uint32_t* q = new uint32_t[c];
    std::memcpy(q, p_, n_ * sizeof(uint32_t));
    release();
    p_ = q;
    cap_ = uint32_t(c);
  }
  void release() {
    if (p_ != in_) delete[] p_;
    p_ = in_;
    cap_ = kInline;
  }
  void copy_from(const Limbs& o) {
    n_ = 0;
    reserve(o.n_);
    std::memcpy(p_, o.p_, o.n_ * sizeof(uint32_t));
    n_ = o.n_;
  }
  void move_from(Limbs& o) {
    if (o.p_ == o.in_) {
      std::memcpy(in_, o.in_, o.n_ * sizeof(uint32_t));
      p_ = in_;
      cap_ = kInline;
    } else {
      p_ = o.p_;
      cap_ = o.cap_;
      o.p_ = o.in_;
      o.cap_ = kInline;
    }
    n_ = o.n_;
    o.n_ = 0;
  }

  static constexpr uint32_t kInline = 4;
  uint32_t in_[kInline];
  uint32_t* p_ = in_;
  uint32_t n_ = 0, cap_ = kInline;
};

class BigInt {
 public:
  BigInt() = default;
  BigInt(int64_t v) { set_i64(v); }           // NOLINT (implicit by design)
  static BigInt from_u64(uint64_t v) {
    BigInt r;
    r.set_u128(v);
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
    unsigned __int128 m = mag_u128();
    *out = neg_ ? -(__int128)m : (__int128)m;
    return true;
  }
  int64_t to_i64() const {
    uint64_t m = low_u64();
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
    BigInt r;
    if (a.neg_ == b.neg_) {
      add_mag(a.mag_, b.mag_, &r.mag_);
      r.neg_ = a.neg_;
      r.trim();
      return r;
    }
    int c = cmp_mag(a.mag_, b.mag_);
    if (c == 0) return r;
    if (c > 0) { sub_mag(a.mag_, b.mag_, &r.mag_); r.neg_ = a.neg_; }
    else { sub_mag(b.mag_, a.mag_, &r.mag_); r.neg_ = b.neg_; }
    r.trim();
    return r;
  }
  friend BigInt operator-(const BigInt& a, const BigInt& b) {
    BigInt nb = b;
    if (!nb.is_zero()) nb.neg_ = !nb.neg_;
    return a + nb;
  }
  friend BigInt operator*(const BigInt& a, const BigInt& b) {
    BigInt r;
    if (a.is_zero() || b.is_zero()) return r;
    if (a.mag_.size() <= 2 && b.mag_.size() <= 2) {   // 64 x 64 -> 128 bits
      r.set_u128((unsigned __int128)a.low_u64() * b.low_u64());
    } else {
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
      r.trim();
    }
    r.neg_ = a.neg_ != b.neg_;
    return r;
  }
  // x * 2^k
  BigInt shl(uint32_t k) const {
    BigInt r;
    if (is_zero()) return r;
    const uint32_t w = k / 32, s = k % 32;
    r.mag_.assign(mag_.size() + w + 1, 0);
    for (size_t i = 0; i < mag_.size(); i++) {
      const uint64_t v = uint64_t(mag_[i]) << s;
      r.mag_[i + w] |= uint32_t(v);
      r.mag_[i + w + 1] |= uint32_t(v >> 32);
    }
    r.neg_ = neg_;
    r.trim();
    return r;
  }

  // floor division and the matching non-negative remainder (d > 0 required
  // for the remainder to be non-negative; d != 0 always)
  static void floor_divmod(const BigInt& n, const BigInt& d, BigInt* q, BigInt* r) {
    BigInt qa, ra;
    divmod_mag(n, d, &qa, &ra);               // |n| = qa*|d| + ra
    // truncated quotient sign
    bool qneg = n.neg_ != d.neg_;
    BigInt tq = qneg ? -qa : qa;
    BigInt tr = n.neg_ ? -ra : ra;            // n = tq*d + tr, sign(tr) = sign(n)
    if (!tr.is_zero() && (tr.neg_ != d.neg_)) { tq = tq - BigInt(1); tr = tr + d; }
    if (q) *q = std::move(tq);
    if (r) *r = std::move(tr);
  }
  static BigInt floor_div(const BigInt& n, const BigInt& d) { BigInt q; floor_divmod(n, d, &q, nullptr); return q; }
  static BigInt ceil_div(const BigInt& n, const BigInt& d) { return -floor_div(-n, d); }
  static BigInt gcd(BigInt a, BigInt b) {
    a.neg_ = false;
    b.neg_ = false;
    while (!b.is_zero()) {
      BigInt q, r;
      divmod_mag(a, b, &q, &r);
      a = std::move(b);
      b = std::move(r);
    }
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
    std::vector<uint32_t> m(mag_.data(), mag_.data() + mag_.size());
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
    neg_ = v < 0;
    set_mag(neg_ ? uint64_t(0) - uint64_t(v) : uint64_t(v));
    if (mag_.empty()) neg_ = false;
  }
  // |x| = m (the sign is left as it is)
  void set_mag(unsigned __int128 m) {
    mag_.clear();
    while (m) {
      mag_.push_back(uint32_t(m));
      m >>= 32;
    }
  }
  void set_u128(unsigned __int128 m) {
    set_mag(m);
    neg_ = false;
  }
  unsigned __int128 mag_u128() const {   // |x| when it has at most four limbs
    unsigned __int128 m = 0;
    for (size_t i = mag_.size(); i-- > 0;) m = (m << 32) | mag_[i];
    return m;
  }
  void trim() { while (!mag_.empty() && mag_.back() == 0) mag_.pop_back(); if (mag_.empty()) neg_ = false; }
  static int cmp_mag(const Limbs& a, const Limbs& b) {
    if (a.size() != b.size()) return a.size() < b.size() ? -1 : 1;
    for (size_t i = a.size(); i-- > 0;)
      if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
    return 0;
  }
  static void add_mag(const Limbs& a, const Limbs& b, Limbs* out) {
    Limbs r;
    r.assign(std::max(a.size(), b.size()) + 1, 0);
    uint64_t carry = 0;
    for (size_t i = 0; i < r.size(); i++) {
      uint64_t t = carry;
      if (i < a.size()) t += a[i];
      if (i < b.size()) t += b[i];
      r[i] = uint32_t(t);
      carry = t >> 32;
    }
    *out = std::move(r);
  }
  static void sub_mag(const Limbs& a, const Limbs& b, Limbs* out) {  // |a| >= |b|
    Limbs r;
    r.assign(a.size(), 0);
    int64_t borrow = 0;
    for (size_t i = 0; i < a.size(); i++) {
      int64_t t = int64_t(a[i]) - borrow - (i < b.size() ? int64_t(b[i]) : 0);
      borrow = t < 0;
      if (t < 0) t += (int64_t(1) << 32);
      r[i] = uint32_t(t);
    }
    *out = std::move(r);
  }
  // |n| = q * |d| + r with 0 <= r < |d| (d != 0); q and r non-negative
  static void divmod_mag(const BigInt& n, const BigInt& d, BigInt* q, BigInt* r) {
    if (n.mag_.size() <= 4 && d.mag_.size() <= 4) {
      const unsigned __int128 nm = n.mag_u128(), dm = d.mag_u128();
      q->set_u128(nm / dm);
      r->set_u128(nm % dm);
      return;
    }
    // schoolbook binary long division for longer operands
    BigInt quo, rem;
    uint32_t nb = n.bit_length();
    quo.mag_.assign(n.mag_.size() + 1, 0);
    BigInt dabs = d.abs();
    for (uint32_t i = nb; i-- > 0;) {
      rem = rem.shl(1);
      if (n.bit(i)) rem = rem + BigInt(1);
      if (rem >= dabs) { rem = rem - dabs; quo.mag_[i / 32] |= 1u << (i % 32); }
    }
    quo.trim();
    *q = std::move(quo);
    *r = std::move(rem);
  }

  Limbs mag_;
  bool neg_ = false;
};

}  // namespace scuba
