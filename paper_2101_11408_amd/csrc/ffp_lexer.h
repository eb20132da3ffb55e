// The bitmap lexer of the parse kernel and the tile layout it reads: byte
// classes of 16-byte chunks, the LDS tile, and the lexers that turn a token
// start into (w, q, sign) from the tile's digit and delimiter bitmaps
// (Section 4 of the paper; digits converted SWAR-style as in Appendix D).
// Device code of the parse kernel; compiled unchanged for the host by the
// CPU test of the lexers (wave-wide votes then come from the test).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "ffp_device.h"
#include "ffp_internal.h"

namespace ffp {

// High bit of each byte of x set for non-delimiter bytes (a single
// delimiter byte below 0x80, replicated in drep) / for ASCII digits.  The
// low seven bits of each byte, after the xor, plus 0x7F (0x76) carry into
// the byte's high bit when they are nonzero (10 or more); x's own high bit
// marks the bytes at or above 0x80, which are neither the delimiter nor a
// digit.  Exact per byte (no carry crosses a byte); three VALU operations
// per word.
FFP_HD uint32_t nondelim_word(uint32_t x, uint32_t drep) {
  const uint32_t t = ((x ^ drep) & 0x7F7F7F7Fu) + 0x7F7F7F7Fu;
  return (t | x) & 0x80808080u;
}

FFP_HD uint32_t digit_word(uint32_t x) {
  const uint32_t t = ((x ^ 0x30303030u) & 0x7F7F7F7Fu) + 0x76767676u;
  return ~(t | x) & 0x80808080u;
}

FFP_HD uint32_t nondelim_word_lut(uint32_t x, const uint8_t* lut) {
  uint32_t h = 0;
#pragma unroll
  for (int b = 0; b < 4; ++b) h |= (lut[(x >> (8 * b)) & 0xFF] ? 0u : 0x80u) << (8 * b);
  return h;
}

// High bit of each byte of x set where the byte equals c (crep = c repeated
// in the four bytes): y = x ^ crep is zero exactly there; its low seven bits
// plus 0x7F carry into bit 7 when nonzero, and y's own bit 7 covers the rest.
FFP_HD uint32_t byte_eq_word(uint32_t x, uint32_t crep) {
  const uint32_t y = x ^ crep;
  return ~(((y & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | y) & 0x80808080u;
}

// Bit i of the result: parity of bits 0..i of a 16-bit mask.
FFP_HD uint32_t prefix_xor16(uint32_t x) {
  x ^= x << 1;
  x ^= x << 2;
  x ^= x << 4;
  x ^= x << 8;
  return x & 0xFFFFu;
}

// Gather the high bits of the bytes of four words into a 16-bit mask: byte
// dot products with weights 1..128 put bytes 8..15 at bits 7..14 of `hi`;
// shifted up by 8 it is the accumulator of the same for bytes 0..7.
FFP_HD uint32_t pack_high_bits(uint32_t h0, uint32_t h1, uint32_t h2,
                               uint32_t h3) {
  const uint32_t hi = dot4_u8(h3, 0x80402010u, dot4_u8(h2, 0x08040201u, 0u));
  const uint32_t all = dot4_u8(h1, 0x80402010u, dot4_u8(h0, 0x08040201u, hi << 8));
  return all >> 7;
}

// ---------------------------------------------------------------------------
// The parse kernel's LDS tile
// ---------------------------------------------------------------------------
template <int K>
struct TileSmem {
  static constexpr int kBytes = kThreads * kChunk * K;
  static constexpr int kChunks = kThreads * K;
  // The fast lexer reads up to 24 bytes before and 36 bytes after a token
  // start; the pads keep those reads inside the array (their contents are
  // masked off).
  static constexpr int kPadFront = 32;
  static constexpr int kPadBack = 96;
  // The 1 KiB of text after the tile (the first chunks of the next tile, or
  // delimiters past the job's end) is added before the round that decides a
  // token running past the tile's end, so that such a token is lexed from
  // LDS like the others; only a token reaching beyond it reads global memory.
  static constexpr int kExtChunks = kWave;
  static constexpr int kExtBytes = kExtChunks * kChunk;
  // block scan of the per-thread start counts: one 16-bit field per row of
  // 256 chunks (a row holds at most 2048 starts)
  using Packed = typename std::conditional<(K <= 2), uint32_t, uint64_t>::type;
  unsigned long long pow10[20];
  // digit-group masks: entry d keeps the low nibbles of bytes d..7 of an
  // 8-byte window (its last 8 - d bytes), 0 for d >= 8; one LDS read
  // instead of a 64-bit shift and selects per group
  unsigned long long keep8[16];
  alignas(16) uint8_t text[kPadFront + kBytes + kExtBytes + kPadBack];
  // bit i of these bitmaps describes byte i of the tile (16 bits per chunk),
  // then the extension, then 128 zero bits so that 32-bit windows stay in
  // range
  alignas(8) uint16_t nd[kChunks + kExtChunks + 8];  // not a delimiter
  alignas(8) uint16_t dg[kChunks + kExtChunks + 8];  // ASCII digit
  uint8_t delim_lut[256];
  Packed scan[kThreads / kWave];
  uint32_t prev_nd;   // the byte before the tile is a token byte
  uint32_t prev_str;  // JSON documents: the tile begins inside a string
  uint32_t ext_end;  // the extension holds a delimiter
  unsigned long long red_min, red_max, red_count;  // this workgroup's reduction
  unsigned long long red_part[kThreads / kWave];    // per-wave sums of block counts
};

struct LdsSrc {
  const uint8_t* text;  // LDS tile (first byte of the tile)
  uint64_t tile_start;
  const uint8_t* lut;   // LDS delimiter table
  FFP_HD uint32_t operator()(uint64_t i) const {
    return text[i - tile_start];
  }
  FFP_HD bool is_end(uint32_t c) const { return lut[c] != 0; }
};

// 32 bits of a tile bitmap starting at bit s (one funnel shift).
FFP_HD uint32_t bit_window(const uint16_t* bm, uint32_t s) {
  const uint32_t* w = reinterpret_cast<const uint32_t*>(bm);
  const uint32_t i = s >> 5;
  return funnel_bits(w[i + 1], w[i], s & 31);
}

// Value of 4 ASCII digits, the first (most significant) in the low byte:
// (d0*10 + d1) * 100 + (d2*10 + d3) from two byte dot products.
FFP_HD uint32_t value4(uint32_t x) {
  return mul_u24(dot4_u8(x, 0x0000010Au, 0u), 100u) +
         dot4_u8(x, 0x010A0000u, 0u);
}

// Value of the n (0..8) ASCII digits that end just before tile offset `end`
// (SWAR on two 32-bit words; Appendix D of the paper does the same on one
// 64-bit word).  Reads bytes [end-8, end).
template <int K>
FFP_HD uint32_t digits8_before(const TileSmem<K>& sm, int end, int n) {
  const int A = end - 8 + TileSmem<K>::kPadFront;
  const uint32_t* W = reinterpret_cast<const uint32_t*>(sm.text);
  const uint32_t w0 = W[A >> 2], w1 = W[(A >> 2) + 1], w2 = W[(A >> 2) + 2];
  uint32_t lo = funnel_bytes(w1, w0, (uint32_t)A & 3u);
  uint32_t hi = funnel_bytes(w2, w1, (uint32_t)A & 3u);
  const uint64_t keep = sm.keep8[(8 - n) & 15];  // the 8 - n leading bytes dropped
  lo &= (uint32_t)keep;
  hi &= (uint32_t)(keep >> 32);
  return mul_u24(value4(lo), 10000u) + value4(hi);
}

// The 8 ASCII digits that end just before `end`, all 8 of them digits: no
// mask.  value4 of ASCII bytes exceeds that of the digit values by
// '0' * 11 * 101 = 53328 (no byte product carries), so the 8-digit value is
// off by 53328 * 10001, subtracted at the end.
template <int K>
FFP_HD uint32_t digits8_full(const TileSmem<K>& sm, int end) {
  const int A = end - 8 + TileSmem<K>::kPadFront;
  const uint32_t* W = reinterpret_cast<const uint32_t*>(sm.text);
  const uint32_t w0 = W[A >> 2], w1 = W[(A >> 2) + 1], w2 = W[(A >> 2) + 2];
  const uint32_t lo = funnel_bytes(w1, w0, (uint32_t)A & 3u);
  const uint32_t hi = funnel_bytes(w2, w1, (uint32_t)A & 3u);
  return mul_u24(value4(lo), 10000u) + value4(hi) - 533333328u;
}

// Same for n (0..4) digits.  Reads bytes [end-4, end).
template <int K>
FFP_HD uint32_t digits4_before(const TileSmem<K>& sm, int end, int n) {
  const int A = end - 4 + TileSmem<K>::kPadFront;
  const uint32_t* W = reinterpret_cast<const uint32_t*>(sm.text);
  const uint32_t w0 = W[A >> 2], w1 = W[(A >> 2) + 1];
  const uint32_t x = funnel_bytes(w1, w0, (uint32_t)A & 3u);
  const uint32_t keep = (uint32_t)(sm.keep8[(8 - n) & 15] >> 32);
  return value4(x & keep);
}

// Value of the n (0..19) digits ending before `end`; the wave skips groups
// that no lane needs.
template <int K>
FFP_HD uint64_t digits_before(const TileSmem<K>& sm, int end, int n) {
  if (wave_all(n <= 4)) return digits4_before<K>(sm, end, n);
  // groups that are whole in every lane need no mask
  uint64_t v = wave_all(n >= 8) ? digits8_full<K>(sm, end) : digits8_before<K>(sm, end, n < 8 ? n : 8);
  if (wave_any(n > 8)) {
    const int n1 = n > 16 ? 8 : (n > 8 ? n - 8 : 0);
    v += (uint64_t)(wave_all(n >= 16) ? digits8_full<K>(sm, end - 8)
                                   : digits8_before<K>(sm, end - 8, n1)) * 100000000ull;
    if (wave_any(n > 16)) {  // at most 3 more digits (n <= 19)
      const int n2 = n > 16 ? n - 16 : 0;
      v += (uint64_t)digits4_before<K>(sm, end - 16, n2) * 10000000000000000ull;
    }
  }
  return v;
}

constexpr uint32_t kFastOk = 0, kFastInvalid = 1, kFastSlow = 2;

// Lexing modes of the parse kernel's instances (see k_parse).
constexpr int kModePlain = 0, kModeGrammar = 1, kModeExt = 2, kModeDoc = 3, kModeCsv = 4;
// The plain grammar with the full start list of a 16 KiB tile: the twin of
// the plain instance for calls with a block denser than its short list.
constexpr int kModePlainDense = 5;

struct FastLex {
  uint64_t w;
  int32_t q;
  uint32_t neg;
  uint32_t code;
  TableEntry ent;  // kFastOk: the power-of-five table entry for q
};

// Lexer for a token lying wholly inside the tile, from the digit and
// delimiter bitmaps: the runs of the grammar are found with count-trailing-
// zeros on 32-bit windows instead of a loop over bytes, and the digits are
// converted up to eight at a time.  Tokens of 32 bytes or more, with more than
// 19 mantissa digits or more than 8 exponent digits are left to the
// byte-by-byte lexer (kFastSlow); for all others the result equals
// lex_token's.  kGrammar: the grammar flags (FFP_JSON, FFP_INFNAN, FFP_HEX)
// are honoured; without it they must be clear.  A lexed token also gets its
// entry of the power-of-five table, read before the mantissa digits are
// converted so that the read's latency overlaps that work.
template <int K, bool kGrammar>
FFP_HD FastLex fast_lex(const TileSmem<K>& sm, uint32_t s, uint32_t flags,
                        const unsigned long long* table) {
  FastLex r;
  r.w = 0;
  r.q = 0;
  r.neg = 0;
  r.code = kFastSlow;
  const uint8_t* tb = sm.text + TileSmem<K>::kPadFront;
  const uint32_t nd = bit_window(sm.nd, s);
  if (nd == ~0u) return r;
  const uint32_t dg = bit_window(sm.dg, s);
  const int L = __builtin_ctz(~nd);  // token length, < 32
  const uint32_t c0 = tb[s];
  const int a = (c0 == '-' || c0 == '+') ? 1 : 0;
  // bit L of dg is clear (a delimiter is not a digit), so every count below
  // stops at or before L
  const int b = a + __builtin_ctz(~(dg >> a));                // end of integer digits
  const int f1d = b + 1 + __builtin_ctz(~((dg >> b) >> 1));   // end of fraction if '.' at b
  const uint32_t cb = tb[s + b];
  const bool dot = cb == '.';
  const int f0 = dot ? b + 1 : b;
  const int f1 = dot ? f1d : b;
  // the byte after the mantissa (an exponent marker, if any) and the one
  // after it (the exponent's sign): two reads where the mantissa ends
  const uint32_t cx = tb[s + f1], cx1 = tb[s + f1 + 1];
  const bool has_e = f1 < L && (cx | 0x20u) == 'e';
  const bool es = has_e && (cx1 == '-' || cx1 == '+');
  const bool eneg = es && cx1 == '-';
  const int e0 = f1 + 1 + (es ? 1 : 0);
  const int e1 = has_e ? e0 + __builtin_ctz(~(dg >> (e0 & 31))) : e0;
  const int end = has_e ? e1 : f1;
  const int nint = b - a, nfrac = f1 - f0, nexp = e1 - e0;
  r.neg = c0 == '-';
  bool valid = end == L && nint + nfrac > 0 && (!has_e || nexp > 0) &&
               !(c0 == '+' && (flags & (kFlagRejectPlus | kFlagJson)));
  if (kGrammar && (flags & (kFlagJson | kFlagInfNan | kFlagHex))) {  // the same for every lane
    const uint32_t ca = tb[s + a];  // first byte after the sign
    if (flags & kFlagJson)  // no ".5", no "1.", no leading zeros
      valid = valid && nint > 0 && (!dot || nfrac > 0) && !(nint > 1 && ca == '0');
    if (!valid && (flags & kFlagInfNan) && ((ca | 0x20u) == 'i' || (ca | 0x20u) == 'n'))
      return r;  // inf / nan: the byte-by-byte lexer
    if ((flags & kFlagHex) && ca == '0' && (tb[s + a + 1] | 0x20u) == 'x')
      return r;  // hexadecimal: the byte-by-byte lexer
  }
  if (!valid) {
    r.code = kFastInvalid;
    return r;
  }
  // Digits converted: all of them, except that when the integer part is
  // empty or a single '0', up to 8 leading zeros of the fraction are skipped
  // (values below 0.01 printed with 17 significant digits have 20 or more
  // digits, but no more than 19 significant ones).
  int ni = nint, nf = nfrac;
  if (wave_any(nint + nfrac > 19)) {
    if (nint + nfrac > 19 && (nint == 0 || (nint == 1 && tb[s + a] == '0'))) {
      const int A = (int)s + f0 + TileSmem<K>::kPadFront;
      const uint32_t* W = reinterpret_cast<const uint32_t*>(sm.text);
      const uint32_t w0 = W[A >> 2], w1 = W[(A >> 2) + 1], w2 = W[(A >> 2) + 2];
      // the 8 bytes from f0, first byte lowest; a zero byte is a '0'
      const uint64_t x =
          ((uint64_t)funnel_bytes(w2, w1, (uint32_t)A & 3u) << 32 |
           funnel_bytes(w1, w0, (uint32_t)A & 3u)) ^ 0x3030303030303030ull;
      const int zf = x == 0 ? 8 : (int)(__builtin_ctzll(x) >> 3);  // < nfrac: nfrac > 18
      ni = 0;
      nf = nfrac - zf;
    }
  }
  if (ni + nf > 19 || nexp > 8) return r;
  int ev = 0;
  if (wave_any(has_e)) {  // exponents of up to 4 digits in every lane: one 4-digit group
    const int ne = has_e ? nexp : 0;
    ev = wave_all(ne <= 4) ? (int)digits4_before<K>(sm, (int)s + e1, ne)
                        : (int)digits8_before<K>(sm, (int)s + e1, ne);
  }
  r.q = (eneg ? -ev : ev) - nfrac;
  r.ent = table_entry(table, r.q);
  const uint64_t fv = digits_before<K>(sm, (int)s + f1, nf);
  if (wave_all(ni <= 1)) {  // at most one integer digit ("0.5", "7.25", ".5"): read it
    const uint32_t d = ni ? tb[s + b - 1] - '0' : 0u;
    r.w = wave_all(d == 0) ? fv : (uint64_t)d * sm.pow10[nf] + fv;
  } else {
    r.w = digits_before<K>(sm, (int)s + b, ni) * sm.pow10[nf] + fv;
  }
  r.code = kFastOk;
  return r;
}

// First position >= p (a tile offset) whose bit in a tile bitmap is clear;
// the bitmaps end in zero bits, so the scan always stops.
FFP_HD uint32_t run_end(const uint16_t* bm, uint32_t p) {
  for (;;) {
    const uint32_t w = bit_window(bm, p);
    if (w != ~0u) return p + (uint32_t)__builtin_ctz(~w);
    p += 32;
  }
}

// First position in [p, end) of the tile text whose byte is not '0' (all
// bytes there are digits), or end; 16 bytes per LDS read.
template <int K>
FFP_HD uint32_t first_nonzero_digit(const TileSmem<K>& sm, uint32_t p,
                                                        uint32_t end) {
  const uint8_t* tb = sm.text + TileSmem<K>::kPadFront;
  while (p < end) {
    const uint32_t a = p & ~15u;
    const uint4 v = *reinterpret_cast<const uint4*>(tb + a);
    const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t base = a + 4 * i;
      uint32_t x = wd[i] ^ 0x30303030u;  // zero bytes are '0'
      if (base + 4 <= p) x = 0;
      else if (base < p) x &= ~0u << (8 * (p - base));
      if (base >= end) x = 0;
      else if (end - base < 4) x &= (1u << (8 * (end - base))) - 1u;
      if (x) return base + ((uint32_t)__builtin_ctz(x) >> 3);
    }
    p = a + 16;
  }
  return end;
}

// Lexer for a token the bitmap lexer leaves to the byte-by-byte one (32
// bytes or longer, more than 19 significant digits, more than 8 exponent
// digits), when the token lies in the tile (or the text kept after it) and
// no grammar flag other than FFP_REJECT_PLUS is set.  Digit runs are found
// 32 bytes at a time on the bitmaps, leading zeros and nonzero dropped
// digits 16 bytes at a time; the first 19 significant digits are converted
// with the SWAR helpers.  The result equals lex_token's (Section 4's grammar;
// Section 11's w, q and the dropped-digit flag).
template <int K>
FFP_HD Lexed long_lex(const TileSmem<K>& sm, uint32_t s, uint32_t flags) {
  const uint8_t* tb = sm.text + TileSmem<K>::kPadFront;
  Lexed r;
  r.w = 0;
  r.q = 0;
  r.neg = 0;
  r.kind = kLexInvalid;
  const uint32_t end = run_end(sm.nd, s);
  const uint32_t c0 = tb[s];
  uint32_t i0 = s;
  if (c0 == '-' || c0 == '+') {
    r.neg = c0 == '-';
    if (c0 == '+' && (flags & kFlagRejectPlus)) return r;
    ++i0;
  }
  const uint32_t b = run_end(sm.dg, i0);  // end of the integer digits
  uint32_t f0 = b, f1 = b;
  if (tb[b] == '.') {
    f0 = b + 1;
    f1 = run_end(sm.dg, f0);
  }
  const uint32_t nint = b - i0, nfrac = f1 - f0;
  if (nint + nfrac == 0) return r;
  uint32_t p = f1;
  int64_t e = 0;
  if ((tb[p] | 0x20u) == 'e') {
    uint32_t e0 = p + 1;
    const bool eneg = tb[e0] == '-';
    if (tb[e0] == '-' || tb[e0] == '+') ++e0;
    const uint32_t e1 = run_end(sm.dg, e0);
    if (e1 == e0) return r;
    // leading zeros do not count; beyond 17 significant digits the value
    // saturates (lex_token stops growing it past 2^56, and q is clamped)
    const uint32_t z = first_nonzero_digit<K>(sm, e0, e1);
    e = e1 - z > 17 ? kExpCap : (int64_t)digits_before<K>(sm, (int)e1, (int)(e1 - z));
    if (eneg) e = -e;
    p = e1;
  }
  if (p != end) return r;
  // significant digits: from the first nonzero one, the dot skipped
  uint32_t nz = first_nonzero_digit<K>(sm, i0, b);
  const bool in_int = nz < b;
  if (!in_int) nz = first_nonzero_digit<K>(sm, f0, f1);
  uint64_t w = 0;
  int64_t dropped = 0;
  bool nonzero_dropped = false;
  if (in_int || nz < f1) {
    const uint32_t n_int = in_int ? b - nz : 0;               // significant integer digits
    const uint32_t n_frac = in_int ? nfrac : f1 - nz;         // significant fraction digits
    const uint32_t nsig = n_int + n_frac;
    const uint32_t take_int = n_int < 19 ? n_int : 19;
    const uint32_t take_frac = nsig <= 19 ? n_frac : 19 - take_int;
    const uint32_t fs = in_int ? f0 : nz;                     // first significant fraction digit
    if (take_int) w = digits_before<K>(sm, (int)(nz + take_int), (int)take_int);
    if (take_frac)
      w = w * sm.pow10[take_frac] + digits_before<K>(sm, (int)(fs + take_frac), (int)take_frac);
    if (nsig > 19) {
      dropped = nsig - 19;
      // dropped digits: the rest of the integer run, then the fraction run
      if (take_int < n_int)
        nonzero_dropped = first_nonzero_digit<K>(sm, nz + take_int, b) < b;
      if (!nonzero_dropped)
        nonzero_dropped = first_nonzero_digit<K>(sm, fs + take_frac, f1) < f1;
    }
  }
  int64_t q = e - (int64_t)nfrac + dropped;
  q = q < -100000 ? -100000 : (q > 100000 ? 100000 : q);
  r.q = (int32_t)q;
  r.w = w;
  r.kind = nonzero_dropped ? kLexTruncated : kLexExact;
  return r;
}

}  // namespace ffp
