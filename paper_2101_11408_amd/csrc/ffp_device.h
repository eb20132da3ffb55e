// Device-side building blocks of the parser: format constants, the
// 64x64->128-bit product, Algorithm 1 of the paper, the token lexer and the
// big-integer helpers of the exact fallback.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ffp_internal.h"

// The per-token logic is compiled for the GPU by the kernels and, unchanged,
// for the host by the CPU unit tests of the library.
#define FFP_HD __host__ __device__ __forceinline__

namespace ffp {

// ---------------------------------------------------------------------------
// IEEE formats (Section 2, Table 2) and the constants Algorithm 1 uses for
// each of them (Sections 5 to 10).
// ---------------------------------------------------------------------------
struct F64 {
  using bits_t = uint64_t;
  static constexpr int kMant = 52;         // stored significand bits
  static constexpr int kShift = 9;         // z_hi >> (u + 9) keeps 54 bits
  static constexpr int kMinExp = -1022;    // smallest normal exponent
  static constexpr int kMaxExp = 1023;
  static constexpr int kBias = 1023;
  static constexpr int kTieLo = -4;        // ties only for q in [-4, 23]
  static constexpr int kTieHi = 23;
  static constexpr int kSubExp = -1074;    // exponent of the subnormal quantum
  static constexpr uint64_t kSecondMask = 0x1FFull;  // 64 - 55 low bits
  static constexpr uint64_t kInf = 0x7FF0000000000000ull;
  static constexpr uint64_t kQNaN = 0x7FF8000000000000ull;
  static constexpr uint64_t kSign = 1ull << 63;
};

struct F32 {
  using bits_t = uint32_t;
  static constexpr int kMant = 23;
  static constexpr int kShift = 38;        // z_hi >> (u + 38) keeps 25 bits
  static constexpr int kMinExp = -126;
  static constexpr int kMaxExp = 127;
  static constexpr int kBias = 127;
  static constexpr int kTieLo = -17;       // ties only for q in [-17, 10]
  static constexpr int kTieHi = 10;
  static constexpr int kSubExp = -149;
  static constexpr uint64_t kSecondMask = (1ull << 38) - 1;  // 64 - 26 low bits
  static constexpr uint32_t kInf = 0x7F800000u;
  static constexpr uint32_t kQNaN = 0x7FC00000u;
  static constexpr uint32_t kSign = 1u << 31;
};

constexpr int kQMin = -342;  // table range, Section 5 and Appendix B
constexpr int kQMax = 308;

// ---------------------------------------------------------------------------
// 64 x 64 -> 128-bit product from four 32 x 32 -> 64-bit multiply-adds
// (v_mad_u64_u32 on CDNA); no partial sum overflows 64 bits.
// ---------------------------------------------------------------------------
FFP_HD void mul_64x64(uint64_t a, uint64_t b, uint64_t& hi,
                                          uint64_t& lo) {
  const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
  const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  const uint64_t p00 = (uint64_t)a0 * b0;
  const uint64_t p01 = (uint64_t)a0 * b1 + (p00 >> 32);
  const uint64_t p10 = (uint64_t)a1 * b0 + (uint32_t)p01;
  hi = (uint64_t)a1 * b1 + (p01 >> 32) + (p10 >> 32);
  lo = (p10 << 32) | (uint32_t)p00;
}

// Status codes (public values of include/ffp.h).
constexpr uint32_t kStOk = 0;
constexpr uint32_t kStInvalid = 1;
constexpr uint32_t kStRange = 2;

// ---------------------------------------------------------------------------
// Algorithm 1: nearest binary value of w * 10^q for 0 < w <= 10^19.
//
// thi/tlo is the 128-bit table entry for q.  Sets `abort` when the truncated
// product cannot decide (z mod 2^64 all ones with q outside [-27, 55]), and
// `st` to kStRange for results that overflowed to infinity or underflowed to
// zero.  The sign is applied by the caller.
//
// The second 64-bit product is computed only when the low 9 (binary64) or
// 38 (binary32) bits of the first product's high word are all ones, the
// paper's stopping rule (Sections 7 to 9); otherwise the bits that decide
// the result are already exact.  On the GPU a wavefront executes the second
// product only when one of its lanes needs it.
//
// Subnormal branch: p is the exponent of the leading bit of the 54/25-bit m,
// so the result is subnormal when p < -1022 (-126) and m must lose
// -1022 - p (-126 - p) bits before the final rounding step.  Read literally,
// the printed algorithm uses p <= -1022 and one more bit of shift; that
// disagrees with Section 9.3 (subnormal below 2^-1022) and with the
// exponent of Example 4, and halves every subnormal.
// ---------------------------------------------------------------------------
template <class F>
FFP_HD typename F::bits_t alg1(uint64_t w, int q, uint64_t thi,
                                                   uint64_t tlo, bool& abort,
                                                   uint32_t& st) {
  using B = typename F::bits_t;
  abort = false;
  st = kStOk;
  if (q < kQMin) {  // w * 10^q < 2^-1075 for every w < 2^64
    st = kStRange;
    return 0;
  }
  if (q > kQMax) {  // beyond 2^1024 for every w >= 1
    st = kStRange;
    return F::kInf;
  }
  const int l = __builtin_clzll(w);
  w <<= l;
  uint64_t zh, zl;
  mul_64x64(w, thi, zh, zl);
  if ((zh & F::kSecondMask) == F::kSecondMask) {
    uint64_t ph, pl;
    mul_64x64(w, tlo, ph, pl);
    zl += ph;
    zh += (zl < ph);
  }
  abort = (zl == ~0ull) && (q < -27 || q > 55);
  const int u = (int)(zh >> 63);
  uint64_t m = zh >> (u + F::kShift);
  int p = ((217706 * q) >> 16) + 63 - l + u;  // arithmetic shift = floor
  if (p <= F::kMinExp - 64) {
    st = kStRange;
    return 0;
  }
  if (p < F::kMinExp) {
    m >>= (F::kMinExp - p);
    m = (m + (m & 1)) >> 1;
    if (m == 0) st = kStRange;
    return (B)m;  // exponent field 0; m == 2^kMant encodes the smallest normal
  }
  if (zl <= 1 && (m & 1) && !(m & 2) && q >= F::kTieLo && q <= F::kTieHi &&
      (m << (u + F::kShift)) == zh) {
    m -= 1;  // exact tie with an even lower neighbour: do not round up
  }
  m = (m + (m & 1)) >> 1;
  if (m == (2ull << F::kMant)) {
    m >>= 1;
    p += 1;
  }
  if (p > F::kMaxExp) {
    st = kStRange;
    return F::kInf;
  }
  return ((B)(p + F::kBias) << F::kMant) | ((B)m & (((B)1 << F::kMant) - 1));
}

// ---------------------------------------------------------------------------
// Delimiter classification.
// ---------------------------------------------------------------------------
FFP_HD bool is_delim(const DelimSet& d, uint32_t c) {
  // selects instead of d.bits[c >> 6]: a runtime index would force the set
  // into scratch memory
  const uint32_t h = (c >> 6) & 3;
  const uint64_t word = h == 0 ? d.bits[0] : h == 1 ? d.bits[1] : h == 2 ? d.bits[2] : d.bits[3];
  return (word >> (c & 63)) & 1;
}

FFP_HD bool is_digit(uint32_t c) { return (c - '0') < 10u; }

// ---------------------------------------------------------------------------
// Lexer (Section 4): sign, significand digits with an optional '.', optional
// exponent.  Keeps the first 19 significant digits in w (leading zeros are
// not significant), counts the dropped ones and whether any of them is
// nonzero, and returns q such that w * 10^q is the value truncated to 19
// significant digits.  The source returns a delimiter byte for every
// position past the end of the buffer, so the lexer never needs the token
// length: it consumes the grammar and then requires a delimiter.
// ---------------------------------------------------------------------------
enum LexKind : uint32_t { kLexExact = 0, kLexTruncated = 1, kLexInvalid = 2 };

struct Lexed {
  uint64_t w;
  int32_t q;
  uint32_t neg;
  uint32_t kind;
};

// Exponent digits saturate here; with buffers below 2^47 bytes the digit
// counts cannot bring a saturated exponent back into range.
constexpr int64_t kExpCap = 1ll << 56;

template <class Src>
FFP_HD Lexed lex_token(const Src& src, uint64_t pos, uint32_t flags) {
  Lexed r;
  r.w = 0;
  r.q = 0;
  r.neg = 0;
  r.kind = kLexExact;
  uint32_t c = src(pos);
  if (c == '-') {
    r.neg = 1;
    c = src(++pos);
  } else if (c == '+') {
    if (flags & 1u) r.kind = kLexInvalid;
    c = src(++pos);
  }
  uint32_t nsig = 0;
  int64_t ndig = 0, nfrac = 0, dropped = 0;
  uint32_t nonzero_dropped = 0;
  uint64_t w = 0;
  // integer part
  while (is_digit(c)) {
    const uint32_t d = c - '0';
    ++ndig;
    if (nsig < 19) {
      if (nsig != 0 || d != 0) {
        w = w * 10 + d;
        ++nsig;
      }
    } else {
      ++dropped;
      nonzero_dropped |= d;
    }
    c = src(++pos);
  }
  if (c == '.') {
    c = src(++pos);
    const int64_t before = ndig;
    while (is_digit(c)) {
      const uint32_t d = c - '0';
      ++ndig;
      if (nsig < 19) {
        if (nsig != 0 || d != 0) {
          w = w * 10 + d;
          ++nsig;
        }
      } else {
        ++dropped;
        nonzero_dropped |= d;
      }
      c = src(++pos);
    }
    nfrac = ndig - before;
  }
  if (ndig == 0) r.kind = kLexInvalid;
  int64_t e = 0;
  if ((c | 0x20u) == 'e') {
    c = src(++pos);
    bool eneg = false;
    if (c == '-') {
      eneg = true;
      c = src(++pos);
    } else if (c == '+') {
      c = src(++pos);
    }
    if (!is_digit(c)) r.kind = kLexInvalid;
    while (is_digit(c)) {
      if (e < kExpCap) e = e * 10 + (c - '0');
      c = src(++pos);
    }
    if (eneg) e = -e;
  }
  if (!src.is_end(c)) r.kind = kLexInvalid;
  int64_t q = e - nfrac + dropped;
  q = q < -100000 ? -100000 : (q > 100000 ? 100000 : q);
  r.q = (int32_t)q;
  r.w = w;
  if (r.kind == kLexExact && nonzero_dropped) r.kind = kLexTruncated;
  return r;
}

// Byte sources for the lexer.
struct GlobalSrc {
  const uint8_t* text;
  uint64_t nbytes;
  DelimSet delim;
  FFP_HD uint32_t operator()(uint64_t i) const {
    return i < nbytes ? (uint32_t)text[i] : delim.byte;
  }
  FFP_HD bool is_end(uint32_t c) const { return is_delim(delim, c); }
};

// ---------------------------------------------------------------------------
// Big unsigned integers for the exact fallback: little-endian 32-bit limbs.
// On the GPU they live in LDS with a stride of one wavefront (limb i of lane
// l at base[i * 64 + l]), so that lanes never share a bank.
// ---------------------------------------------------------------------------
struct BigRef {
  uint32_t* base;
  int n;       // limbs in use (no leading zero limb)
  int stride;  // distance between limbs (the wavefront size in LDS)
  FFP_HD uint32_t& operator[](int i) const { return base[i * stride]; }
};

// x = x * m + a; returns false on overflow of kBigLimbs.
FFP_HD bool big_mul_add(BigRef& x, uint32_t m, uint32_t a) {
  uint64_t carry = a;
  for (int i = 0; i < x.n; ++i) {
    const uint64_t t = (uint64_t)x[i] * m + carry;
    x[i] = (uint32_t)t;
    carry = t >> 32;
  }
  if (carry) {
    if (x.n >= kBigLimbs) return false;
    x[x.n] = (uint32_t)carry;
    ++x.n;
  }
  return true;
}

// dst = src * (b1:b0) for a 64-bit multiplier.
FFP_HD bool big_mul_u64(BigRef& dst, const BigRef& src, uint64_t b) {
  const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  if (src.n + 2 > kBigLimbs) return false;
  uint64_t c0 = 0, c1 = 0;
  // two passes of a 1-limb multiply-accumulate
  for (int i = 0; i < src.n; ++i) {
    const uint64_t t = (uint64_t)src[i] * b0 + c0;
    dst[i] = (uint32_t)t;
    c0 = t >> 32;
  }
  dst[src.n] = (uint32_t)c0;
  dst[src.n + 1] = 0;
  if (b1) {
    for (int i = 0; i < src.n; ++i) {
      const uint64_t t = (uint64_t)src[i] * b1 + dst[i + 1] + c1;
      dst[i + 1] = (uint32_t)t;
      c1 = t >> 32;
    }
    dst[src.n + 1] = (uint32_t)c1;
  }
  int n = src.n + 2;
  while (n > 0 && dst[n - 1] == 0) --n;
  dst.n = n;
  return true;
}

// sign(a - (c << s)) for s >= 0, without materialising the shift.
FFP_HD int big_cmp_shl(const BigRef& a, const BigRef& c, int s) {
  const int ws = s >> 5, bs = s & 31;
  const int nc = c.n + ws + 1;
  int top = a.n > nc ? a.n : nc;
  for (int i = top - 1; i >= 0; --i) {
    const uint32_t ai = i < a.n ? a[i] : 0u;
    const int j = i - ws;
    uint32_t ci = 0;
    if (j >= 0 && j < c.n) ci = c[j] << bs;
    if (bs && j - 1 >= 0 && j - 1 < c.n) ci |= c[j - 1] >> (32 - bs);
    if (ai != ci) return ai > ci ? 1 : -1;
  }
  return 0;
}

// sign(a * 2^ea - c * 2^ec)
FFP_HD int big_cmp_pow2(const BigRef& a, int ea, const BigRef& c, int ec) {
  if (ea >= ec) return -big_cmp_shl(c, a, ea - ec);
  return big_cmp_shl(a, c, ec - ea);
}

// ---------------------------------------------------------------------------
// Decision for one lexed token: Algorithm 1 on w (and on w+1 when digits
// beyond the 19th were dropped and not all zero, Section 11).
// ---------------------------------------------------------------------------
template <class F>
struct Decision {
  typename F::bits_t bits;  // sign applied
  uint32_t status;          // kStOk / kStInvalid / kStRange
  uint32_t path;            // Counter index
  bool fallback;            // undecided: needs the exact fallback
};

template <class F>
FFP_HD Decision<F> decide_lexed(const Lexed& L, const unsigned long long* table) {
  Decision<F> d;
  d.fallback = false;
  if (L.kind == kLexInvalid) {
    d.bits = F::kQNaN;
    d.status = kStInvalid;
    d.path = kCntInvalid;
    return d;
  }
  if (L.w == 0) {
    d.bits = L.neg ? F::kSign : 0;
    d.status = kStOk;
    d.path = kCntEarly;
    return d;
  }
  const int qi = L.q < kQMin ? kQMin : (L.q > kQMax ? kQMax : L.q);
  const uint64_t thi = table[2 * (qi - kQMin)];
  const uint64_t tlo = table[2 * (qi - kQMin) + 1];
  bool ab;
  d.bits = alg1<F>(L.w, L.q, thi, tlo, ab, d.status);
  d.fallback = ab;
  d.path = (L.q < kQMin || L.q > kQMax) ? kCntEarly : kCntOne;
  if (L.kind == kLexTruncated) {
    bool ab2;
    uint32_t st2;
    const typename F::bits_t b2 = alg1<F>(L.w + 1, L.q, thi, tlo, ab2, st2);
    d.fallback = d.fallback || ab2 || b2 != d.bits;
    d.path = kCntTwo;
  }
  if (L.neg) d.bits |= F::kSign;
  if (d.fallback) d.path = kCntFallback;
  return d;
}

// ---------------------------------------------------------------------------
// Exact fallback for one token (the paper asks for an exact higher-precision
// method here and leaves the method open, Section 11).
//
// The token's first 769 significant digits form the integer P; a nonzero
// digit beyond them appends a sticky 1, so that v = P * 10^f decides every
// comparison with a midpoint exactly.  A candidate b comes from Algorithm 1
// on the first 19 digits; v is then compared with the halfway points
// (2m+1) * 2^(e-1) between b and its neighbours until b is the nearest value,
// ties to even.  Encodings are used as integers, so "next value up" is
// bits + 1 across binades and into infinity.
//
// limbs points at 3 * kBigLimbs limbs spaced `stride` apart.  Returns false
// if a big integer outgrew kBigLimbs (cannot happen for tokens that reach the
// fallback; reported as an internal error).
// ---------------------------------------------------------------------------
template <class F>
FFP_HD void decode_bits(typename F::bits_t b, uint64_t& m, int& e) {
  const uint32_t field = (uint32_t)(b >> F::kMant);
  const uint64_t frac = (uint64_t)(b & (((typename F::bits_t)1 << F::kMant) - 1));
  if (field == 0) {
    m = frac;
    e = F::kSubExp;
  } else {
    m = frac | (1ull << F::kMant);
    e = (int)field - F::kBias - F::kMant;
  }
}

template <class F>
FFP_HD bool fallback_decide(const GlobalSrc& src, uint64_t pos, const unsigned long long* table,
                            uint32_t* limbs, int stride, typename F::bits_t& out_bits,
                            uint32_t& out_status) {
  using Bits = typename F::bits_t;
  BigRef X{limbs, 0, stride};                          // P, or P * 5^f when f >= 0
  BigRef Y{limbs + kBigLimbs * stride, 0, stride};     // 5^-f when f < 0
  BigRef T{limbs + 2 * kBigLimbs * stride, 0, stride}; // 2m+1 or (2m+1) * 5^-f

  uint32_t c = src(pos);
  bool neg = false;
  if (c == '-') {
    neg = true;
    c = src(++pos);
  } else if (c == '+') {
    c = src(++pos);
  }
  uint64_t w = 0;
  int nw = 0;
  int64_t dropped_w = 0, dropped = 0, nfrac = 0;
  int kept = 0;
  bool sticky = false, in_frac = false;
  uint32_t chunk = 0, chunk_pow = 1;
  bool ok = true;
  for (;;) {
    if (c == '.' && !in_frac) {
      in_frac = true;
      c = src(++pos);
      continue;
    }
    if (!is_digit(c)) break;
    const uint32_t dg = c - '0';
    if (in_frac) ++nfrac;
    if (kept == 0 && dg == 0) {
      c = src(++pos);
      continue;
    }
    if (nw < 19) {
      w = w * 10 + dg;
      ++nw;
    } else {
      ++dropped_w;
    }
    if (kept < kFallbackDigits) {
      chunk = chunk * 10 + dg;
      chunk_pow *= 10;
      ++kept;
      if (chunk_pow == 1000000000u) {
        ok &= big_mul_add(X, chunk_pow, chunk);
        chunk = 0;
        chunk_pow = 1;
      }
    } else {
      ++dropped;
      sticky |= dg != 0;
    }
    c = src(++pos);
  }
  if (chunk_pow > 1) ok &= big_mul_add(X, chunk_pow, chunk);
  int64_t e10 = 0;
  if ((c | 0x20u) == 'e') {
    c = src(++pos);
    bool eneg = false;
    if (c == '-') {
      eneg = true;
      c = src(++pos);
    } else if (c == '+') {
      c = src(++pos);
    }
    while (is_digit(c)) {
      if (e10 < kExpCap) e10 = e10 * 10 + (c - '0');
      c = src(++pos);
    }
    if (eneg) e10 = -e10;
  }
  const int64_t q64 = e10 - nfrac + dropped_w;
  int64_t f64v = e10 - nfrac + dropped;
  if (sticky) {
    ok &= big_mul_add(X, 10, 1);
    f64v -= 1;
  }

  Bits bits;
  uint32_t status = kStOk;
  if (w == 0) {
    bits = 0;
  } else if (q64 < kQMin) {
    bits = 0;
    status = kStRange;
  } else if (q64 > kQMax) {
    bits = F::kInf;
    status = kStRange;
  } else {
    const int q = (int)q64;
    const int f = (int)f64v;  // in [q - 750, q] since at most 769 digits are kept
    bool ab;
    uint32_t st1;
    bits = alg1<F>(w, q, table[2 * (q - kQMin)], table[2 * (q - kQMin) + 1], ab, st1);
    if (f >= 0) {  // X = P * 5^f, v = X * 2^f
      for (int k = 0; k < f; k += 13) {
        const int sh = f - k < 13 ? f - k : 13;
        uint32_t p5 = 1;
        for (int t = 0; t < sh; ++t) p5 *= 5;
        ok &= big_mul_add(X, p5, 0);
      }
    } else {  // Y = 5^-f, v = P * 2^f / Y
      Y[0] = 1;
      Y.n = 1;
      for (int k = 0; k < -f; k += 13) {
        const int sh = -f - k < 13 ? -f - k : 13;
        uint32_t p5 = 1;
        for (int t = 0; t < sh; ++t) p5 *= 5;
        ok &= big_mul_add(Y, p5, 0);
      }
    }
    if (bits == F::kInf) bits = F::kInf - 1;
    for (int iter = 0; iter < 8 && ok; ++iter) {
      if (bits < F::kInf) {
        // sign(v - midpoint(bits, bits + 1))
        uint64_t m;
        int e;
        decode_bits<F>(bits, m, e);
        const uint64_t h = 2 * m + 1;
        if (f >= 0) {
          T[0] = (uint32_t)h;
          T[1] = (uint32_t)(h >> 32);
          T.n = T[1] ? 2 : 1;
        } else {
          ok &= big_mul_u64(T, Y, h);
        }
        const int up = big_cmp_pow2(X, f, T, e - 1);
        if (up > 0 || (up == 0 && (bits & 1))) {
          bits += 1;
          if (bits == F::kInf) break;
          continue;
        }
      }
      if (bits > 0) {
        // sign(v - midpoint(bits - 1, bits))
        uint64_t m;
        int e;
        decode_bits<F>(bits - 1, m, e);
        const uint64_t h = 2 * m + 1;
        if (f >= 0) {
          T[0] = (uint32_t)h;
          T[1] = (uint32_t)(h >> 32);
          T.n = T[1] ? 2 : 1;
        } else {
          ok &= big_mul_u64(T, Y, h);
        }
        const int dn = big_cmp_pow2(X, f, T, e - 1);
        if (dn < 0 || (dn == 0 && ((bits - 1) & 1) == 0)) {
          bits -= 1;
          continue;
        }
      }
      break;
    }
    if (bits == F::kInf || bits == 0) status = kStRange;
  }
  if (neg) bits |= F::kSign;
  out_bits = bits;
  out_status = status;
  return ok;
}

}  // namespace ffp
