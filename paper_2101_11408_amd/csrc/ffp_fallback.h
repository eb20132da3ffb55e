// Exact fallback, one wavefront per token (device code).
//
// The paper leaves the exact higher-precision method for undecided inputs
// open (Section 11).  Here the 64 lanes of a wavefront cooperate on one
// token:
//   - the token is read in windows of 64 x 16 bytes; ballots find the end,
//     the exponent marker and the decimal point, and a wave-wide prefix sum
//     gives every digit its index, so each lane places its own digits;
//   - the first 769 significant digits (plus a sticky 1 when a nonzero digit
//     follows them) form the integer P, so that v = P * 10^f decides every
//     comparison with a midpoint exactly (a midpoint between neighbouring
//     binary64 values has at most 768 significant digits);
//   - big integers hold one 64-bit limb per lane (numbers below 2^4096, far
//     above the 2^2600 the comparisons need); multiplying by a 64-bit scalar
//     is one 64 x 64 -> 128-bit product per lane, and the carries between
//     limbs are resolved at once from two ballots (generate and propagate
//     masks added as 64-bit integers);
//   - a candidate from Algorithm 1 on the first 19 digits is moved to the
//     nearest encoding by comparing v with the halfway points
//     (2m+1) * 2^(e-1) between neighbouring values, ties to even; encodings
//     are used as integers, so "next value up" crosses binades and reaches
//     infinity (whose encoding reads as the value 2^(emax+1));
//   - under a directed rounding mode the comparisons are with the values
//     m * 2^e themselves: the truncation is the largest encoding not above
//     v, the rounding away from zero the smallest not below it.
// Every branch below depends only on wave-uniform values, so the lanes stay
// converged for the cross-lane operations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ffp_device.h"
#include "ffp_internal.h"
#include "ffp_lexer.h"

namespace ffp {

constexpr int kFbWindow = kWave * 16;  // text bytes per wavefront step
constexpr int kExpKeep = 18;           // significant exponent digits kept

// Per-wavefront LDS of the fallback.
// digits[] is 4-byte aligned with 8 bytes before it, so that the 8-digit
// conversions below may read aligned words on either side of a run.
struct FbLds {
  alignas(4) uint8_t pad[8];
  uint8_t digits[kFallbackDigits + 12];  // significant digits, values 0..9
  uint8_t edigits[kExpKeep + 6];         // significant exponent digits
};

// Value of the n (0..8) digit values d[end - n .. end): two aligned words
// around them, the unwanted leading bytes masked off, then four digits at a
// time by byte dot products (weights 10/1, then 100), the first digit in the
// low byte.
__device__ __forceinline__ uint32_t fb_val4(uint32_t x) {
  return __umul24(__builtin_amdgcn_udot4(x, 0x0000010Au, 0u, false), 100u) +
         __builtin_amdgcn_udot4(x, 0x010A0000u, 0u, false);
}

__device__ __forceinline__ uint32_t fb_val8(const uint8_t* d, int end, int n) {
  if (n <= 0) end = 8;        // nothing kept: any in-range words will do
  const int A = end - 8 + 8;  // byte offset of d[end - 8] from d - 8 (>= 1 for n >= 1)
  const uint32_t* W = reinterpret_cast<const uint32_t*>(d - 8);
  const uint32_t w0 = W[A >> 2], w1 = W[(A >> 2) + 1], w2 = W[(A >> 2) + 2];
  uint32_t lo = __builtin_amdgcn_alignbyte(w1, w0, (uint32_t)A & 3u);
  uint32_t hi = __builtin_amdgcn_alignbyte(w2, w1, (uint32_t)A & 3u);
  const int drop = 8 - n;
  const uint64_t keep = drop >= 8 ? 0ull : (~0ull << (8 * drop));
  lo &= (uint32_t)keep;
  hi &= (uint32_t)(keep >> 32);
  return __umul24(fb_val4(lo), 10000u) + fb_val4(hi);
}

// Value of the digit values d[lo .. hi), hi - lo <= 19.
__device__ __forceinline__ uint64_t fb_digits_value(const uint8_t* d, int lo, int hi) {
  const int n = hi - lo;
  const int n0 = n < 8 ? n : 8;
  const int n1 = n < 16 ? (n > 8 ? n - 8 : 0) : 8;
  const int n2 = n > 16 ? n - 16 : 0;
  return (uint64_t)fb_val8(d, hi, n0) + (uint64_t)fb_val8(d, hi - 8, n1) * 100000000ull +
         (uint64_t)fb_val8(d, hi - 16, n2) * 10000000000000000ull;
}

__device__ __forceinline__ int fb_lane() { return (int)(threadIdx.x & (kWave - 1)); }

// Makes LDS stores of the wavefront's lanes visible to its other lanes.
__device__ __forceinline__ void fb_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t fb_ballot(bool p) { return (uint64_t)__ballot(p); }

__device__ __forceinline__ uint32_t fb_read32(uint32_t v, int lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

__device__ __forceinline__ uint64_t fb_read64(uint64_t v, int lane) {
  return (uint64_t)fb_read32((uint32_t)v, lane) |
         ((uint64_t)fb_read32((uint32_t)(v >> 32), lane) << 32);
}

// Exclusive prefix sum over the wavefront.
__device__ __forceinline__ uint32_t fb_excl_scan(uint32_t v) {
  const int l = fb_lane();
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, kWave);
    if (l >= d) x += y;
  }
  return x - v;
}

// ---------------------------------------------------------------------------
// Big integers: limb i (64 bits) in lane i.
// ---------------------------------------------------------------------------

// x * m + a, a added to limb 0.  The top carry out of lane 63 is dropped
// (callers stay far below 2^4096).
__device__ __forceinline__ uint64_t fbig_mul_add(uint64_t x, uint64_t m, uint64_t a) {
  const int l = fb_lane();
  uint64_t hi, lo;
  mul_64x64(x, m, hi, lo);
  uint64_t h = __shfl_up(hi, 1, kWave);
  h = l == 0 ? a : h;
  const uint64_t s = lo + h;
  // carry out of this limb's sum (g) and "passes a carry on" (p): exclusive,
  // since an overflowing sum of two 64-bit values is at most 2^64 - 2
  const uint64_t G = fb_ballot(s < lo);
  const uint64_t P = fb_ballot(s == ~0ull);
  // carry into lane i = bit i of the carries of (G|P) + G
  const uint64_t C = ((G | P) + G) ^ P;
  return s + ((C >> l) & 1ull);
}

// Index of the highest nonzero limb, -1 for zero.
__device__ __forceinline__ int fbig_top(uint64_t x) {
  const uint64_t B = fb_ballot(x != 0);
  return B ? 63 - __builtin_clzll(B) : -1;
}

// Bit length (0 for zero).
__device__ __forceinline__ int fbig_bits(uint64_t x) {
  const int t = fbig_top(x);
  if (t < 0) return 0;
  const uint64_t v = fb_read64(x, t);
  return 64 * t + 64 - __builtin_clzll(v);
}

// x << s (s >= 0); the caller checks that the result fits 64 limbs.
__device__ __forceinline__ uint64_t fbig_shl(uint64_t x, int s) {
  const int l = fb_lane();
  const int ws = s >> 6, bs = s & 63;
  const int j = l - ws;
  const uint64_t a = __shfl(x, j < 0 ? 0 : j, kWave);
  const uint64_t b = __shfl(x, j - 1 < 0 ? 0 : j - 1, kWave);
  uint64_t r = j >= 0 ? a << bs : 0;
  if (bs != 0 && j - 1 >= 0) r |= b >> (64 - bs);
  return r;
}

// sign(x - y)
__device__ __forceinline__ int fbig_cmp(uint64_t x, uint64_t y) {
  const uint64_t D = fb_ballot(x != y);
  if (D == 0) return 0;
  const int k = 63 - __builtin_clzll(D);
  return fb_read64(x, k) > fb_read64(y, k) ? 1 : -1;
}

// sign(a * 2^ea - c * 2^ec)
__device__ __forceinline__ int fbig_cmp_pow2(uint64_t a, int ea, uint64_t c, int ec) {
  constexpr int kMaxBits = 64 * kWave;
  if (ea >= ec) {
    const int s = ea - ec;
    const int ab = fbig_bits(a);
    if (ab == 0) return fbig_top(c) < 0 ? 0 : -1;
    if (ab + s > kMaxBits - 1) return 1;  // a * 2^s exceeds anything c can hold
    return fbig_cmp(fbig_shl(a, s), c);
  }
  const int s = ec - ea;
  const int cb = fbig_bits(c);
  if (cb == 0) return fbig_top(a) < 0 ? 0 : 1;
  if (cb + s > kMaxBits - 1) return -1;
  return fbig_cmp(a, fbig_shl(c, s));
}

// ---------------------------------------------------------------------------
// Wave-cooperative lexing of a token that the lexer already accepted.
// ---------------------------------------------------------------------------

// Bits [0, p) of a lane's 16 byte positions (window position 16*lane + k).
__device__ __forceinline__ uint32_t fb_mask_lt(int p) {
  const int k = p - 16 * fb_lane();
  return k <= 0 ? 0u : (k >= 16 ? 0xFFFFu : ((1u << k) - 1u));
}

// Lowest window position whose bit is set in some lane's 16-bit mask, or
// kFbWindow.
__device__ __forceinline__ int fb_first(uint32_t m16) {
  const uint64_t B = fb_ballot(m16 != 0);
  if (!B) return kFbWindow;
  const int L = __builtin_ctzll(B);
  return 16 * L + (int)fb_read32((uint32_t)__builtin_ctz(m16 | 0x10000u), L);
}

__device__ __forceinline__ uint32_t fb_byte(const uint32_t (&wd)[4], int k) {
  return (wd[k >> 2] >> (8 * (k & 3))) & 0xFFu;
}

// Byte at window position p (uniform p < kFbWindow).
__device__ __forceinline__ uint32_t fb_byte_at(const uint32_t (&wd)[4], int p) {
  const int k = p & 15;
  const uint32_t w = (k >> 2) == 0 ? wd[0] : (k >> 2) == 1 ? wd[1] : (k >> 2) == 2 ? wd[2] : wd[3];
  return (fb_read32(w, p >> 4) >> (8 * (k & 3))) & 0xFFu;
}

// A run of digits seen window by window: count, index of the first nonzero
// digit, significant digits below `limit` stored to `out`, and whether a
// nonzero digit came after them.
struct FbDigits {
  int64_t n = 0;
  int64_t z = -1;
  bool sticky = false;
};

// pre: the digits of dm in lanes below this one (fb_excl_scan of the
// per-lane counts), total: those of the whole window.
__device__ __forceinline__ void fb_feed(FbDigits& s, uint32_t dm, const uint32_t (&wd)[4],
                                        uint8_t* out, int limit, uint32_t pre, uint32_t total) {
  if (s.z < 0) {
    constexpr uint32_t kZero = '0' * 0x01010101u;
    const uint32_t zm = pack_high_bits(byte_eq_word(wd[0], kZero), byte_eq_word(wd[1], kZero),
                                       byte_eq_word(wd[2], kZero), byte_eq_word(wd[3], kZero));
    const uint32_t nz = dm & ~zm;
    const uint64_t B = fb_ballot(nz != 0);
    if (B) {
      const int L = __builtin_ctzll(B);
      const uint32_t below = __popc(dm & ((nz & (0u - nz)) - 1u));
      s.z = s.n + (int64_t)fb_read32(pre + below, L);
    }
  }
  if (s.z >= 0) {
    // index of the lane's first digit among the significant digits, in 32
    // bits: at least -kFbWindow (the leading zeros of this window), and
    // clamped at `limit` above (which keeps every such digit out of range)
    const int64_t g64 = s.n + (int64_t)pre - s.z;
    const int32_t g0 = g64 > limit ? limit : (int32_t)g64;
    uint32_t r = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      if ((dm >> k) & 1u) {
        const uint32_t si = (uint32_t)(g0 + (int32_t)r);
        if (si < (uint32_t)limit) out[si] = (uint8_t)(fb_byte(wd, k) - '0');
        ++r;
      }
    }
    // a nonzero digit past the kept ones (tokens of more than `limit`
    // significant digits only)
    if (fb_ballot(g0 + (int32_t)__popc(dm) > limit) != 0) {
      bool stick = false;
      uint32_t r2 = 0;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        if ((dm >> k) & 1u) {
          stick |= g0 + (int32_t)r2 >= limit && fb_byte(wd, k) != '0';
          ++r2;
        }
      }
      s.sticky |= fb_ballot(stick) != 0;
    }
  }
  s.n += total;
}

struct FbToken {
  bool neg;
  int64_t nsig;    // significant mantissa digits
  int64_t nfrac;   // digits after the decimal point
  bool sticky;     // a nonzero digit beyond the first kFallbackDigits
  int64_t e10;     // explicit exponent (saturated beyond 18 digits)
};

// Lexes the token starting at `pos` of a job's text; the significant digits
// go to lds->digits.  Text past nbytes reads as a delimiter.
__device__ FbToken fb_lex(const uint8_t* text, uint64_t nbytes, uint64_t pos, FbLds* lds) {
  const int l = fb_lane();
  FbToken t;
  // a leading sign stays in the first window: it is neither a digit nor a
  // '.', an exponent marker or an end byte, so the scans below pass over it
  // (no dependent load of the first byte before the window's loads)
  t.neg = false;
  bool first = true;
  FbDigits mant, expo;
  int64_t nint = -1;  // digits before the point, -1 without a point
  int state = 0;      // 0 mantissa, 1 exponent sign or first digit, 2 exponent digits
  bool eneg = false;
  for (;; pos += kFbWindow) {
    uint32_t wd[4];
    const uint64_t base = pos + 16 * (uint64_t)l;
    // the lane's 16 bytes from the aligned words around them when those lie
    // inside the text; byte by byte otherwise (bytes past the text read as a
    // blank)
    const uint32_t sh = (uint32_t)(((uintptr_t)text + base) & 3u);
    if (base >= sh && base - sh + (sh ? 20u : 16u) <= nbytes) {
      const uint32_t* w = reinterpret_cast<const uint32_t*>(text + (base - sh));
      const uint32_t x0 = w[0], x1 = w[1], x2 = w[2], x3 = w[3], x4 = sh ? w[4] : 0u;
      wd[0] = __builtin_amdgcn_alignbyte(x1, x0, sh);
      wd[1] = __builtin_amdgcn_alignbyte(x2, x1, sh);
      wd[2] = __builtin_amdgcn_alignbyte(x3, x2, sh);
      wd[3] = __builtin_amdgcn_alignbyte(x4, x3, sh);
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        uint32_t w = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const uint64_t i = base + 4 * q + b;
          w |= (i < nbytes ? (uint32_t)text[i] : (uint32_t)' ') << (8 * b);
        }
        wd[q] = w;
      }
    }
    if (first) {
      t.neg = fb_byte_at(wd, 0) == '-';
      first = false;
    }
    // byte classes of the lane's 16 bytes, four at a time (the parse
    // kernel's exact per-byte tests): digits, '.', 'e' or 'E', and the end
    // bytes (anything but those and the signs)
    constexpr uint32_t kDot = '.' * 0x01010101u, kE = 'e' * 0x01010101u;
    constexpr uint32_t kPlus = '+' * 0x01010101u, kMinus = '-' * 0x01010101u;
    const uint32_t dm = pack_high_bits(digit_word(wd[0]), digit_word(wd[1]), digit_word(wd[2]),
                                       digit_word(wd[3]));
    const uint32_t dot = pack_high_bits(byte_eq_word(wd[0], kDot), byte_eq_word(wd[1], kDot),
                                        byte_eq_word(wd[2], kDot), byte_eq_word(wd[3], kDot));
    const uint32_t em = pack_high_bits(
        byte_eq_word(wd[0] | 0x20202020u, kE), byte_eq_word(wd[1] | 0x20202020u, kE),
        byte_eq_word(wd[2] | 0x20202020u, kE), byte_eq_word(wd[3] | 0x20202020u, kE));
    const uint32_t sgn = pack_high_bits(byte_eq_word(wd[0], kPlus) | byte_eq_word(wd[0], kMinus),
                                        byte_eq_word(wd[1], kPlus) | byte_eq_word(wd[1], kMinus),
                                        byte_eq_word(wd[2], kPlus) | byte_eq_word(wd[2], kMinus),
                                        byte_eq_word(wd[3], kPlus) | byte_eq_word(wd[3], kMinus));
    const uint32_t endm = ~(dm | dot | em | sgn) & 0xFFFFu;
    const int endp = fb_first(endm);
    int es = 0;  // start of the exponent part in this window
    if (state == 0) {
      const int ep = fb_first(em & fb_mask_lt(endp));
      const int mend = ep < endp ? ep : endp;
      const uint32_t mdm = dm & fb_mask_lt(mend);
      const uint32_t cnt = __popc(mdm);
      const uint32_t pre = fb_excl_scan(cnt);
      const int dp = fb_first(dot & fb_mask_lt(mend));
      // digits before the point: those of the lanes below its lane, and its
      // lane's own below it
      if (dp < kFbWindow)
        nint = mant.n + (int64_t)fb_read32(pre + __popc(mdm & fb_mask_lt(dp)), dp >> 4);
      fb_feed(mant, mdm, wd, lds->digits, kFallbackDigits, pre,
              fb_read32(pre + cnt, kWave - 1));
      if (ep < endp) {
        state = 1;
        es = ep + 1;
      }
    }
    if (state == 1 && es < kFbWindow) {
      const uint32_t c = fb_byte_at(wd, es);
      if (c == '-' || c == '+') {
        eneg = c == '-';
        ++es;
      }
      state = 2;
    }
    if (state == 2) {
      const uint32_t edm = dm & fb_mask_lt(endp) & ~fb_mask_lt(es);
      const uint32_t cnt = __popc(edm);
      const uint32_t pre = fb_excl_scan(cnt);
      fb_feed(expo, edm, wd, lds->edigits, kExpKeep, pre, fb_read32(pre + cnt, kWave - 1));
    }
    if (endp < kFbWindow) break;
  }
  t.nsig = mant.z < 0 ? 0 : mant.n - mant.z;
  t.nfrac = nint < 0 ? 0 : mant.n - nint;
  t.sticky = mant.sticky;
  fb_wave_sync();
  int64_t e = 0;
  const int64_t esig = expo.z < 0 ? 0 : expo.n - expo.z;
  if (esig > kExpKeep || expo.sticky) {
    e = kExpCap;  // beyond every digit count of a buffer: decides by itself
  } else {
    for (int i = 0; i < (int)esig; ++i) e = e * 10 + lds->edigits[i];
  }
  t.e10 = eneg ? -e : e;
  return t;
}

// ---------------------------------------------------------------------------
// The decision.
// ---------------------------------------------------------------------------
// pow5: 5^(27 i) for i < kPow5Steps, kWave limbs each (lane i holds limb i).
constexpr int kPow5Step = 27;
constexpr int kPow5Steps = 43;

template <class F>
__device__ void fb_decide(const uint8_t* text, uint64_t nbytes, uint64_t pos,
                          const unsigned long long* table, const unsigned long long* pow5,
                          FbLds* lds, uint32_t flags, typename F::bits_t& out_bits,
                          uint32_t& out_status) {
  using Bits = typename F::bits_t;
  const int l = fb_lane();
  const FbToken t = fb_lex(text, nbytes, pos, lds);
  const uint32_t dir = round_dir(flags, t.neg);

  Bits bits = 0;
  uint32_t status = kStOk;
  if (t.nsig > 0) {
    const int nw = t.nsig < 19 ? (int)t.nsig : 19;
    uint64_t w = 0;
    w = fb_digits_value(lds->digits, 0, nw);
    int kept = t.nsig < kFallbackDigits ? (int)t.nsig : kFallbackDigits;
    const int64_t q64 = t.e10 - t.nfrac + (t.nsig - nw);
    int64_t f64v = t.e10 - t.nfrac + (t.nsig - kept);
    if (q64 < kQMin) {  // below half the smallest subnormal
      if (dir == kDirAway) {
        bits = 1;
      } else {
        status = kStRange;
      }
    } else if (q64 > kQMax) {
      bits = dir == kDirTruncate ? F::kInf - 1 : F::kInf;
      status = kStRange;
    } else {
      if (t.sticky) {  // P = 10 * P + 1: strictly between the truncation and the next digit
        if (l == 0) lds->digits[kept] = 1;
        ++kept;
        f64v -= 1;
        fb_wave_sync();
      }
      const int q = (int)q64;
      const int f = (int)f64v;  // in [q - 770, q]
      // P from 19-digit groups counted from the last digit: group j in lane j
      const int ng = (kept + 18) / 19;
      uint64_t grp = 0;
      if (l < ng) {
        const int hi = kept - 19 * l;
        const int lo = hi - 19 > 0 ? hi - 19 : 0;
        grp = fb_digits_value(lds->digits, lo, hi);
      }
      uint64_t X = l == 0 ? fb_read64(grp, ng - 1) : 0;
      for (int j = ng - 2; j >= 0; --j) X = fbig_mul_add(X, 10000000000000000000ull, fb_read64(grp, j));
      uint64_t Y = l == 0 ? 1 : 0;  // 5^-f when f < 0
      constexpr uint64_t k5p27 = 7450580596923828125ull;
      if (f >= 0) {  // X = P * 5^f, v = X * 2^f
        for (int k = f; k > 0; k -= 27) {
          uint64_t p5 = k5p27;
          if (k < 27) {
            p5 = 1;
            for (int i = 0; i < k; ++i) p5 *= 5;
          }
          X = fbig_mul_add(X, p5, 0);
        }
      } else {  // v = P * 2^f / 5^-f: 5^(27 i) from the table, then the rest
        int i = -f / kPow5Step;
        if (i > kPow5Steps - 1) i = kPow5Steps - 1;
        Y = pow5[i * kWave + l];
        for (int k = -f - kPow5Step * i; k > 0; k -= 27) {
          uint64_t p5 = k5p27;
          if (k < 27) {
            p5 = 1;
            for (int r = 0; r < k; ++r) p5 *= 5;
          }
          Y = fbig_mul_add(Y, p5, 0);
        }
      }
      bool ab;
      uint32_t st1;
      bits = alg1<F>(w, q, table[2 * (q - kQMin)], table[2 * (q - kQMin) + 1], ab, st1);
      if (bits == F::kInf) bits = F::kInf - 1;
      // sign(v - (2m+half) * 2^(e-1)): half = 1 for the midpoint above
      // encoding b, 0 for b itself
      auto vs_at = [&](Bits b, uint64_t half) {
        uint64_t m;
        int e;
        decode_bits<F>(b, m, e);
        const uint64_t h = 2 * m + half;
        const uint64_t T = f >= 0 ? (l == 0 ? h : 0) : fbig_mul_add(Y, h, 0);
        return fbig_cmp_pow2(X, f, T, e - 1);
      };
      auto vs_mid = [&](Bits b) { return vs_at(b, 1); };
      if (dir == kDirTruncate) {  // largest b with value(b) <= v
        for (int iter = 0; iter < 8; ++iter) {
          if (bits < F::kInf && vs_at((Bits)(bits + 1), 0) >= 0) {
            bits += 1;
            continue;
          }
          if (bits > 0 && vs_at(bits, 0) < 0) {
            bits -= 1;
            continue;
          }
          break;
        }
      } else if (dir == kDirAway) {  // smallest b with value(b) >= v
        for (int iter = 0; iter < 8; ++iter) {
          if (bits < F::kInf && vs_at(bits, 0) > 0) {
            bits += 1;
            continue;
          }
          if (bits > 0 && vs_at((Bits)(bits - 1), 0) <= 0) {
            bits -= 1;
            continue;
          }
          break;
        }
      }
      for (int iter = 0; iter < 8 && dir == kDirNearest; ++iter) {
        if (bits < F::kInf) {
          const int up = vs_mid(bits);
          if (up > 0 || (up == 0 && (bits & 1))) {
            bits += 1;
            if (bits == F::kInf) break;
            continue;
          }
        }
        if (bits > 0) {
          const int dn = vs_mid(bits - 1);
          if (dn < 0 || (dn == 0 && ((bits - 1) & 1) == 0)) {
            bits -= 1;
            continue;
          }
        }
        break;
      }
      if (bits == F::kInf || bits == 0) status = kStRange;
      if (bits == F::kInf && dir == kDirTruncate) bits = F::kInf - 1;  // overflow: largest finite
    }
  }
  if (t.neg) bits |= F::kSign;
  out_bits = bits;
  out_status = status;
}

}  // namespace ffp
