// Device-side building blocks of the parser: format constants, the
// 64x64->128-bit product, Algorithm 1 of the paper and the token lexer.
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
  static constexpr bool kTieFallback = false;
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
  static constexpr bool kTieFallback = false;
};

// binary16 and bfloat16 use the same table and steps.  The tie windows and
// the round-half-up subnormal step above rest on the paper's proofs for
// binary64 and binary32 (a short decimal is never an exact midpoint outside
// the windows, nor among subnormals); for binary16 that fails (2^-25 has 18
// significant digits).  For these formats a product that may be an exact
// midpoint (kTieFallback) is decided exactly where that is cheap -- q in
// [0, 27], where the product is exact, and q in [-27, -1] with 5^-q dividing
// w, where the value is (w / 5^-q) * 2^q -- and goes to the exact fallback
// otherwise.
struct F16 {
  using bits_t = uint16_t;
  static constexpr int kMant = 10;
  static constexpr int kShift = 51;        // z_hi >> (u + 51) keeps 12 bits
  static constexpr int kMinExp = -14;
  static constexpr int kMaxExp = 15;
  static constexpr int kBias = 15;
  static constexpr int kTieLo = 0;         // unused (kTieFallback)
  static constexpr int kTieHi = -1;
  static constexpr int kSubExp = -24;
  static constexpr uint64_t kSecondMask = (1ull << 51) - 1;
  static constexpr uint16_t kInf = 0x7C00u;
  static constexpr uint16_t kQNaN = 0x7E00u;
  static constexpr uint16_t kSign = 0x8000u;
  static constexpr bool kTieFallback = true;
};

struct BF16 {
  using bits_t = uint16_t;
  static constexpr int kMant = 7;
  static constexpr int kShift = 54;        // z_hi >> (u + 54) keeps 9 bits
  static constexpr int kMinExp = -126;
  static constexpr int kMaxExp = 127;
  static constexpr int kBias = 127;
  static constexpr int kTieLo = 0;         // unused (kTieFallback)
  static constexpr int kTieHi = -1;
  static constexpr int kSubExp = -133;
  static constexpr uint64_t kSecondMask = (1ull << 54) - 1;
  static constexpr uint16_t kInf = 0x7F80u;
  static constexpr uint16_t kQNaN = 0x7FC0u;
  static constexpr uint16_t kSign = 0x8000u;
  static constexpr bool kTieFallback = true;
};

// The constants of a format as values, so that one inlined copy of
// Algorithm 1 serves every format a kernel may meet (the format of a job is
// the same for all lanes of a wavefront).
struct FormatRT {
  int32_t mant;
  int32_t shift;
  int32_t min_exp;
  int32_t max_exp;
  int32_t bias;
  int32_t tie_lo;
  int32_t tie_hi;
  int32_t tie_fallback;
  uint64_t second_mask;
  uint64_t inf;
};

template <class F>
FFP_HD constexpr FormatRT format_of() {
  return FormatRT{F::kMant,  F::kShift, F::kMinExp,         F::kMaxExp,      F::kBias,
                  F::kTieLo, F::kTieHi, F::kTieFallback ? 1 : 0, F::kSecondMask, F::kInf};
}

// ---------------------------------------------------------------------------
// gfx950 instructions the lexer relies on, and wave-wide votes.  On the GPU
// each is one instruction; the host build of the same logic (the CPU tests)
// computes the same values in plain C, and takes its wave votes from a hook
// the test installs (a single host "lane" stands for a wavefront whose other
// lanes the test chooses).
// ---------------------------------------------------------------------------
FFP_HD uint32_t funnel_bits(uint32_t hi, uint32_t lo, uint32_t s) {  // v_alignbit_b32
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_alignbit(hi, lo, s);
#else
  return (uint32_t)((((uint64_t)hi << 32) | lo) >> (s & 31));
#endif
}

FFP_HD uint32_t funnel_bytes(uint32_t hi, uint32_t lo, uint32_t s) {  // v_alignbyte_b32
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_alignbyte(hi, lo, s);
#else
  return (uint32_t)((((uint64_t)hi << 32) | lo) >> (8 * (s & 3)));
#endif
}

FFP_HD uint32_t dot4_u8(uint32_t a, uint32_t b, uint32_t c) {  // v_dot4_u32_u8
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_udot4(a, b, c, false);
#else
  for (int i = 0; i < 4; ++i) c += ((a >> (8 * i)) & 0xFFu) * ((b >> (8 * i)) & 0xFFu);
  return c;
#endif
}

FFP_HD uint32_t mul_u24(uint32_t a, uint32_t b) {  // v_mul_u32_u24
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul24(a, b);
#else
  return (a & 0xFFFFFFu) * (b & 0xFFFFFFu);
#endif
}

// Host build: the vote of the wavefront a host lane stands for (null: the
// lane alone).  A host variable; device code never reads it.
inline bool (*host_wave_vote)(bool pred, bool all) = nullptr;

FFP_HD bool wave_all(bool p) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __all(p);
#else
  return host_wave_vote ? host_wave_vote(p, true) : p;
#endif
}

FFP_HD bool wave_any(bool p) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __any(p);
#else
  return host_wave_vote ? host_wave_vote(p, false) : p;
#endif
}

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
FFP_HD uint64_t alg1_rt(uint64_t w, int q, uint64_t thi, uint64_t tlo, const FormatRT& F,
                       bool& abort, uint32_t& st) {
  abort = false;
  st = kStOk;
  if (q < kQMin) {  // w * 10^q < 2^-1075 for every w < 2^64
    st = kStRange;
    return 0;
  }
  if (q > kQMax) {  // beyond 2^1024 for every w >= 1
    st = kStRange;
    return F.inf;
  }
  const int l = __builtin_clzll(w);
  w <<= l;
  uint64_t zh, zl;
  mul_64x64(w, thi, zh, zl);
  if ((zh & F.second_mask) == F.second_mask) {
    uint64_t ph, pl;
    mul_64x64(w, tlo, ph, pl);
    zl += ph;
    zh += (zl < ph);
  }
  abort = (zl == ~0ull) && (q < -27 || q > 55);
  const int u = (int)(zh >> 63);
  uint64_t m = zh >> (u + F.shift);
  int p = ((217706 * q) >> 16) + 63 - l + u;  // arithmetic shift = floor
  if (p <= F.min_exp - 64) {
    st = kStRange;
    return 0;
  }
  if (p < F.min_exp) {
    const int s = F.min_exp - p;
    m >>= s;
    if (F.tie_fallback && (m & 1) && zl <= 1 && u + F.shift + s < 64 &&
        (zh & ((1ull << (u + F.shift + s)) - 1)) == 0)
      abort = true;  // may be an exact midpoint between subnormals
    m = (m + (m & 1)) >> 1;
    if (m == 0) st = kStRange;
    return m;  // exponent field 0; m == 2^mant encodes the smallest normal
  }
  // an exact tie needs the low product word at 0 or 1: rare, so waves
  // branch around the rest of the test
  if (__builtin_expect(zl <= 1, 0) && (m & 1) && (m << (u + F.shift)) == zh) {
    if (F.tie_fallback) {
      // For q in [0, 27] the entry is 5^q itself and the product is exact:
      // the bits below the rounding bit decide (all zero: an exact tie).
      // Elsewhere the product only approximates the value; q in [-27, -1]
      // with 5^-q dividing w is decided exactly by the caller, the rest goes
      // to the exact fallback.
      if (q >= 0 && q <= 27) {
        if (zl == 0 && !(m & 2)) m -= 1;
      } else {
        abort = true;
      }
    } else if (!(m & 2) && q >= F.tie_lo && q <= F.tie_hi) {
      m -= 1;  // exact tie with an even lower neighbour: do not round up
    }
  }
  m = (m + (m & 1)) >> 1;
  if (m == (2ull << F.mant)) {
    m >>= 1;
    p += 1;
  }
  if (p > F.max_exp) {
    st = kStRange;
    return F.inf;
  }
  return ((uint64_t)(p + F.bias) << F.mant) | (m & ((1ull << F.mant) - 1));
}

template <class F>
FFP_HD typename F::bits_t alg1(uint64_t w, int q, uint64_t thi, uint64_t tlo, bool& abort,
                               uint32_t& st) {
  constexpr FormatRT fmt = format_of<F>();
  return (typename F::bits_t)alg1_rt(w, q, thi, tlo, fmt, abort, st);
}

// ---------------------------------------------------------------------------
// Directed rounding.  The paper rounds to nearest, ties to even, and notes
// that its approach extends to the other IEEE modes (footnote of Section 6).
// Toward zero, toward +infinity and toward -infinity reduce, once the sign is
// known, to two rules on the magnitude: truncate it, or raise it to the next
// representable value when anything is lost.  Overflow (the IEEE condition:
// the magnitude, rounded with an unbounded exponent, exceeds the largest
// finite value) gives the largest finite value when truncating and infinity
// otherwise; a nonzero value below the smallest subnormal gives zero when
// truncating and the smallest subnormal otherwise.
// ---------------------------------------------------------------------------
enum RoundDir : uint32_t { kDirNearest = 0, kDirTruncate = 1, kDirAway = 2 };

// Rounding-direction field of the flags (public values of include/ffp.h).
constexpr uint32_t kFlagRoundMask = 0x30;
constexpr uint32_t kRoundTowardZero = 0x10;
constexpr uint32_t kRoundUp = 0x20;    // toward +infinity
constexpr uint32_t kRoundDown = 0x30;  // toward -infinity

FFP_HD uint32_t round_dir(uint32_t flags, uint32_t neg) {
  const uint32_t m = flags & kFlagRoundMask;
  if (m == 0) return kDirNearest;
  if (m == kRoundTowardZero) return kDirTruncate;
  return (m == kRoundUp) == (neg == 0) ? kDirAway : kDirTruncate;
}

// Directed rounding of w * 10^q (0 < w < 2^64) with the table entry of q
// (Algorithm 1's product, both halves always).  The value is v = w * 10^q;
// the 128-bit product z approximates it scaled to [2^126, 2^128).  Let Z be
// the exact scaled value.  From the table's construction:
//   q in [0, 27]   the entry is 5^q itself in the high word: z = Z exactly;
//   q in [28, 55]  the entry is exact, the product is truncated: Z in [z, z+1);
//   q > 55         the entry is truncated too: Z in [z, z+2);
//   q < 0          the entry is a rounded-up reciprocal (or the truncation of
//                  one): Z in (z-1, z+2).
// Whether 5^k divides w (1 <= k <= 27), with the quotient in n: n = w times
// the inverse of 5^k modulo 2^64 is the quotient exactly when n * 5^k does
// not overflow and gives back w.
FFP_HD bool exact_div_pow5(uint64_t w, int k, uint64_t& n) {
  uint64_t p5 = 1, inv = 1;
  for (int i = 0; i < k; ++i) {
    p5 *= 5;
    inv *= 0xCCCCCCCCCCCCCCCDull;  // 5^-1 mod 2^64
  }
  n = w * inv;
  uint64_t hi, lo;
  mul_64x64(n, p5, hi, lo);
  return hi == 0 && lo == w;
}

// v is exactly representable only if its odd part, a multiple of 5^q for
// q > 0, has at most 53 bits, so never for q >= 23; for q < 0 only if 5^-q
// divides w.  Let R be the bits of z below the last kept significand bit.
// Outside the exact region the truncation is m (the kept bits) and v is
// inexact unless R sits within the error of 0 or of the next unit (R = 0,
// or R >= 2^r - 2): those products set `abort` (the exact fallback decides),
// except that for q in [-27, -1] a w divisible by 5^-q gives the exact
// value (w / 5^-q) * 2^q, rounded directly.
FFP_HD uint64_t round_exact(uint64_t w, int q, bool sticky, const FormatRT& F, uint32_t dir,
                            uint32_t& st);

FFP_HD uint64_t alg1_dir_rt(uint64_t w, int q, uint64_t thi, uint64_t tlo, const FormatRT& F,
                            bool away, bool& abort, uint32_t& st) {
  abort = false;
  st = kStOk;
  const uint64_t largest = F.inf - 1;
  if (q < kQMin) {  // strictly between 0 and half the smallest subnormal
    if (!away) st = kStRange;
    return away ? 1 : 0;
  }
  if (q > kQMax) {
    st = kStRange;
    return away ? F.inf : largest;
  }
  const uint64_t w0 = w;
  const int l = __builtin_clzll(w);
  w <<= l;
  uint64_t zh, zl, ph, pl;
  mul_64x64(w, thi, zh, zl);
  mul_64x64(w, tlo, ph, pl);
  zl += ph;
  zh += (zl < ph);
  const int u = (int)(zh >> 63);
  int p = ((217706 * q) >> 16) + 63 - l + u;  // exponent of the leading bit
  if (p <= F.min_exp - 64) {
    if (!away) st = kStRange;
    return away ? 1 : 0;
  }
  // rb: bits of zh below the last kept bit (all of zl lies below it too)
  int rb = u + F.shift + 1;
  if (p < F.min_exp) rb += F.min_exp - p;
  const uint64_t mask = rb < 64 ? (1ull << rb) - 1 : ~0ull;
  uint64_t m = rb < 64 ? zh >> rb : 0;
  const uint64_t rh = zh & mask;
  const bool rzero = rh == 0 && zl == 0;
  const bool rtop = rh == mask && zl >= ~1ull;  // R >= 2^r - 2
  bool inexact = true;
  if (q >= 0 && q <= 27) {
    inexact = !rzero;
  } else if (q > 55) {
    abort = rtop;
  } else if (q < 0) {
    uint64_t n;
    if ((rzero || rtop) && q >= -27 && exact_div_pow5(w0, -q, n))
      return round_exact(n, q, false, F, away ? kDirAway : kDirTruncate, st);
    abort = rzero || rtop;
  }
  if (away && inexact) ++m;
  if (p < F.min_exp) {  // subnormal; m == 2^mant encodes the smallest normal
    if (m == 0) st = kStRange;
    return m;
  }
  if (m == (2ull << F.mant)) {
    m >>= 1;
    p += 1;
  }
  if (p > F.max_exp) {
    st = kStRange;
    return away ? F.inf : largest;
  }
  return ((uint64_t)(p + F.bias) << F.mant) | (m & ((1ull << F.mant) - 1));
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
enum LexKind : uint32_t {
  kLexExact = 0,
  kLexTruncated = 1,
  kLexInvalid = 2,
  kLexInf = 3,        // inf / infinity (flag FFP_INFNAN)
  kLexNaN = 4,        // nan (flag FFP_INFNAN)
  kLexHex = 5,        // hexadecimal: value w * 2^q exactly (flag FFP_HEX)
  kLexHexSticky = 6   // hexadecimal: w * 2^q plus nonzero nibbles below it
};

// Grammar flags (public values of include/ffp.h).
constexpr uint32_t kFlagRejectPlus = 1;
constexpr uint32_t kFlagJson = 2;    // JSON number grammar
constexpr uint32_t kFlagInfNan = 4;  // inf, infinity, nan in any case
constexpr uint32_t kFlagHex = 8;     // hexadecimal floating-point tokens
constexpr uint32_t kFlagJsonDoc = 0x40;  // JSON documents: numbers outside strings
constexpr uint32_t kFlagCsv = 0x80;      // CSV: tokens of the selected columns

FFP_HD int hex_value(uint32_t c) {
  if (c - '0' < 10u) return (int)(c - '0');
  const uint32_t l = c | 0x20u;
  return (l - 'a' < 6u) ? (int)(l - 'a' + 10) : -1;
}

// Case-insensitive match of the letters of `word` at pos; returns the
// position after them, or 0 if they do not match.
template <class Src>
FFP_HD uint64_t match_word(const Src& src, uint64_t pos, const char* word) {
  for (; *word; ++word, ++pos)
    if ((src(pos) | 0x20u) != (uint32_t)*word) return 0;
  return pos;
}

struct Lexed {
  uint64_t w;
  int32_t q;
  uint32_t neg;
  uint32_t kind;
};

// Exponent digits saturate here; with buffers below 2^47 bytes the digit
// counts cannot bring a saturated exponent back into range.
constexpr int64_t kExpCap = 1ll << 56;

// Hexadecimal token after its sign (Appendix C): 0x, hexadecimal digits with
// an optional point, an optional binary exponent.  The first 16 significant
// nibbles go to w, the others only set the sticky kind; q = exponent -
// 4 * (fraction nibbles - dropped nibbles).
template <class Src>
FFP_HD Lexed lex_hex(const Src& src, uint64_t pos, Lexed r) {
  pos += 2;
  uint32_t c = src(pos);
  uint64_t w = 0;
  int nsig = 0;
  int64_t ndig = 0, nfrac = 0, dropped = 0;
  bool sticky = false, point = false;
  for (;; c = src(++pos)) {
    const int h = hex_value(c);
    if (h < 0) {
      if (c == '.' && !point) {
        point = true;
        continue;
      }
      break;
    }
    ++ndig;
    nfrac += point;
    if (nsig < 16) {
      if (nsig || h) {
        w = (w << 4) | (uint64_t)h;
        ++nsig;
      }
    } else {
      ++dropped;
      sticky |= h != 0;
    }
  }
  int64_t e = 0;
  bool ok = ndig > 0;
  if ((c | 0x20u) == 'p') {
    c = src(++pos);
    const bool eneg = c == '-';
    if (c == '-' || c == '+') c = src(++pos);
    ok = ok && is_digit(c);
    for (; is_digit(c); c = src(++pos))
      if (e < kExpCap) e = e * 10 + (c - '0');
    if (eneg) e = -e;
  }
  ok = ok && src.is_end(c);
  int64_t q = e - 4 * (nfrac - dropped);
  q = q < -100000 ? -100000 : (q > 100000 ? 100000 : q);
  r.w = w;
  r.q = (int32_t)q;
  if (r.kind != kLexInvalid) r.kind = !ok ? kLexInvalid : (sticky ? kLexHexSticky : kLexHex);
  return r;
}

// kExt: the extensions (hexadecimal tokens, flag FFP_HEX, and directed
// rounding) are compiled in; kernels built without them keep their registers
// for the decimal path.
template <bool kExt = true, class Src>
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
    if (flags & (kFlagRejectPlus | kFlagJson)) r.kind = kLexInvalid;
    c = src(++pos);
  }
  if ((flags & kFlagInfNan) && ((c | 0x20u) == 'i' || (c | 0x20u) == 'n')) {
    uint64_t e = 0;
    uint32_t kind = kLexInvalid;
    if ((e = match_word(src, pos, "infinity")) && src.is_end(src(e))) {
      kind = kLexInf;
    } else if ((e = match_word(src, pos, "inf")) && src.is_end(src(e))) {
      kind = kLexInf;
    } else if ((e = match_word(src, pos, "nan")) && src.is_end(src(e))) {
      kind = kLexNaN;
    }
    if (r.kind != kLexInvalid) r.kind = kind;
    return r;
  }
  if (kExt && (flags & kFlagHex) && c == '0' && (src(pos + 1) | 0x20u) == 'x')
    return lex_hex(src, pos, r);
  const uint32_t first_digit = c;  // for the JSON leading-zero rule
  uint32_t nsig = 0;
  int64_t ndig = 0, nfrac = 0, dropped = 0;
  uint32_t nonzero_dropped = 0;
  uint64_t w = 0;
  int64_t nint = 0;
  // integer part
  while (is_digit(c)) {
    ++nint;
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
    if ((flags & kFlagJson) && nfrac == 0) r.kind = kLexInvalid;  // "1." is not JSON
  }
  if (ndig == 0) r.kind = kLexInvalid;
  if ((flags & kFlagJson) && (nint == 0 || (nint > 1 && first_digit == '0')))
    r.kind = kLexInvalid;  // ".5" and leading zeros are not JSON
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
// Decision for one lexed token: Algorithm 1 on w (and on w+1 when digits
// beyond the 19th were dropped and not all zero, Section 11).
// ---------------------------------------------------------------------------
// Rounding of w * 2^q (plus something below its last bit when `sticky`)
// in direction `dir`: the exact rounding of a hexadecimal token, and of a
// decimal that reduces to an integer times a power of two.
FFP_HD uint64_t round_exact(uint64_t w, int q, bool sticky, const FormatRT& F, uint32_t dir,
                            uint32_t& st) {
  st = kStOk;
  if (w == 0) return 0;
  const uint64_t largest = F.inf - 1;
  const int l = __builtin_clzll(w);
  w <<= l;
  int64_t e = (int64_t)q + 63 - l;  // exponent of the leading bit
  if (e > F.max_exp) {
    st = kStRange;
    return dir == kDirTruncate ? largest : F.inf;
  }
  const int64_t unit = (e < F.min_exp ? F.min_exp : e) - F.mant;  // exponent of the last kept bit
  const int64_t s = 63 + unit - e;  // bits of w below it, >= 63 - mant
  uint64_t m = 0, rem = w;          // rem: the bits below the last kept one
  if (s < 64) {
    m = w >> s;
    rem = w & ((1ull << s) - 1);
  }
  bool up;
  if (dir == kDirNearest) {
    if (s == 64) {  // w is at least half a unit (w >= 2^63); exactly half is a tie to 0
      up = w > (1ull << 63) || sticky;
    } else if (s < 64) {
      const uint64_t half = 1ull << (s - 1);
      up = rem > half || (rem == half && (sticky || (m & 1)));
    } else {
      up = false;  // below half a unit
    }
  } else {
    up = dir == kDirAway && (rem != 0 || sticky);
  }
  if (up) ++m;
  if (e < F.min_exp) {  // subnormal; m == 2^mant encodes the smallest normal
    if (m == 0) st = kStRange;
    return m;
  }
  if (m == (2ull << F.mant)) {
    m >>= 1;
    ++e;
  }
  if (e > F.max_exp) {
    st = kStRange;
    return dir == kDirTruncate ? largest : F.inf;
  }
  return ((uint64_t)(e + F.bias) << F.mant) | (m & ((1ull << F.mant) - 1));
}

// The 128-bit table entry for q, q clamped to the table's range (values
// outside it are decided without the entry).  One 16-byte read: the table
// is 16-byte aligned.
struct TableEntry {
  uint64_t hi, lo;
};

FFP_HD TableEntry table_entry(const unsigned long long* table, int q) {
  const int qi = q < kQMin ? kQMin : (q > kQMax ? kQMax : q);
  struct alignas(16) Entry {
    unsigned long long hi, lo;
  };
  const Entry e = reinterpret_cast<const Entry*>(table)[qi - kQMin];
  return TableEntry{e.hi, e.lo};
}

struct DecisionRT {
  uint64_t bits;      // sign applied (sign_bit = 1 << (format width - 1))
  uint32_t status;    // kStOk / kStInvalid / kStRange
  uint32_t path;      // Counter index
  bool fallback;      // undecided: needs the exact fallback
};

// qnan / sign: the format's canonical quiet NaN and sign bit; flags: the
// rounding direction (with kExt); pre: the table entry for L.q when the
// caller has read it already (else it is read here).
template <bool kExt = true>
FFP_HD DecisionRT decide_lexed_rt(const Lexed& L, const unsigned long long* table,
                                  const FormatRT& fmt, uint64_t qnan, uint64_t sign,
                                  uint32_t flags, const TableEntry* pre = nullptr) {
  DecisionRT d;
  d.fallback = false;
  if (L.kind == kLexInvalid) {
    d.bits = qnan;
    d.status = kStInvalid;
    d.path = kCntInvalid;
    return d;
  }
  if (L.kind == kLexInf || L.kind == kLexNaN) {
    d.bits = (L.kind == kLexInf ? fmt.inf : qnan) | (L.neg ? sign : 0);
    d.status = kStOk;
    d.path = kCntEarly;
    return d;
  }
  const uint32_t dir = kExt ? round_dir(flags, L.neg) : (uint32_t)kDirNearest;
  if (kExt && (L.kind == kLexHex || L.kind == kLexHexSticky)) {
    d.bits = round_exact(L.w, L.q, L.kind == kLexHexSticky, fmt, dir, d.status) |
             (L.neg ? sign : 0);
    d.path = kCntOne;
    return d;
  }
  if (L.w == 0) {
    d.bits = L.neg ? sign : 0;
    d.status = kStOk;
    d.path = kCntEarly;
    return d;
  }
  const TableEntry ent = pre ? *pre : table_entry(table, L.q);
  const uint64_t thi = ent.hi, tlo = ent.lo;
  bool ab;
  d.path = (L.q < kQMin || L.q > kQMax) ? kCntEarly : kCntOne;
  if (kExt && dir != kDirNearest) {
    // w and w+1 bracket a truncated token's value; a monotone rounding that
    // maps both ends to the same result and status maps the value there too
    const bool away = dir == kDirAway;
    d.bits = alg1_dir_rt(L.w, L.q, thi, tlo, fmt, away, ab, d.status);
    d.fallback = ab;
    if (L.kind == kLexTruncated) {
      bool ab2;
      uint32_t st2;
      const uint64_t b2 = alg1_dir_rt(L.w + 1, L.q, thi, tlo, fmt, away, ab2, st2);
      d.fallback = d.fallback || ab2 || b2 != d.bits || st2 != d.status;
      d.path = kCntTwo;
    }
  } else {
    d.bits = alg1_rt(L.w, L.q, thi, tlo, fmt, ab, d.status);
    uint64_t n;
    if (fmt.tie_fallback && ab && L.kind == kLexExact && L.q < 0 && L.q >= -27 &&
        exact_div_pow5(L.w, -L.q, n)) {
      // binary16 / bfloat16: a possible midpoint with w * 10^q = n * 2^q
      // exactly, rounded directly
      d.bits = round_exact(n, L.q, false, fmt, kDirNearest, d.status);
      ab = false;
    }
    d.fallback = ab;
    if (L.kind == kLexTruncated) {
      bool ab2;
      uint32_t st2;
      const uint64_t b2 = alg1_rt(L.w + 1, L.q, thi, tlo, fmt, ab2, st2);
      d.fallback = d.fallback || ab2 || b2 != d.bits;
      d.path = kCntTwo;
    }
  }
  if (L.neg) d.bits |= sign;
  if (d.fallback) d.path = kCntFallback;
  return d;
}

template <class F>
struct Decision {
  typename F::bits_t bits;  // sign applied
  uint32_t status;          // kStOk / kStInvalid / kStRange
  uint32_t path;            // Counter index
  bool fallback;            // undecided: needs the exact fallback
};

template <class F, bool kExt = true>
FFP_HD Decision<F> decide_lexed(const Lexed& L, const unsigned long long* table, uint32_t flags,
                                const TableEntry* pre = nullptr) {
  constexpr FormatRT fmt = format_of<F>();
  const DecisionRT r = decide_lexed_rt<kExt>(L, table, fmt, F::kQNaN, F::kSign, flags, pre);
  Decision<F> d;
  d.bits = (typename F::bits_t)r.bits;
  d.status = r.status;
  d.path = r.path;
  d.fallback = r.fallback;
  return d;
}

// ---------------------------------------------------------------------------
// Significand and binary exponent of an encoding (value = m * 2^e).
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

}  // namespace ffp
