// Host build of the parse kernel's bitmap lexers (fast_lex, long_lex in
// ffp_lexer.h), checked token by token against the byte-by-byte lexer
// (lex_token in ffp_device.h, which the CPU tests check against the oracle).
// Used only by the CPU unit tests.
//
// Each token is placed at a random offset of a 16 KiB tile (the extension
// after the tile included) whose other bytes are random digits, signs, dots,
// exponent markers and delimiters, so that the masked reads before and after
// the token see arbitrary neighbours; the tile's bitmaps are built with the
// kernel's own byte-class helpers.  Wave-wide votes come from a host hook:
// in the first pass a lane votes alone, in the second the other lanes of its
// wavefront vote at random, so both sides of every uniform branch run.
//
// usage: lexer_check <token file> <flags> <seed>
// prints: tokens, mismatches; then up to 10 mismatching tokens.
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <random>
#include <string>
#include <vector>

#include "ffp_lexer.h"

using namespace ffp;

namespace {

std::mt19937_64 g_rng;

// A stand-in for the power-of-five table: entry i holds (i + 1000, ~i), so
// that the entry the fast lexer reads identifies the q it was read for.
alignas(16) unsigned long long g_table[2 * (kQMax - kQMin + 1)];
bool g_random_wave = false;

bool vote(bool p, bool all) {
  if (!g_random_wave) return p;
  const bool others = (g_rng() & 1) != 0;  // the rest of the wavefront
  return all ? (p && others) : (p || others);
}

constexpr int K = 4;
using S = TileSmem<K>;

struct Tile {
  S sm;
};

void build_bitmaps(S& sm) {
  const uint32_t drep = '\n' * 0x01010101u;
  for (int c = 0; c < S::kChunks + S::kExtChunks; ++c) {
    uint32_t w[4];
    memcpy(w, &sm.text[S::kPadFront + c * kChunk], 16);
    sm.nd[c] = (uint16_t)pack_high_bits(nondelim_word(w[0], drep), nondelim_word(w[1], drep),
                                        nondelim_word(w[2], drep), nondelim_word(w[3], drep));
    sm.dg[c] = (uint16_t)pack_high_bits(digit_word(w[0]), digit_word(w[1]), digit_word(w[2]),
                                        digit_word(w[3]));
  }
  for (int c = S::kChunks + S::kExtChunks; c < S::kChunks + S::kExtChunks + 8; ++c)
    sm.nd[c] = sm.dg[c] = 0;
}

struct BufSrc {
  const std::string* t;
  uint32_t operator()(uint64_t i) const { return i < t->size() ? (uint8_t)(*t)[i] : '\n'; }
  bool is_end(uint32_t c) const { return c == '\n'; }
};

}  // namespace

int main(int argc, char** argv) {
  if (argc < 4) {
    fprintf(stderr, "usage: %s tokens flags seed\n", argv[0]);
    return 2;
  }
  for (int i = 0; i < kQMax - kQMin + 1; ++i) {
    g_table[2 * i] = 1000ull + (unsigned long long)i;
    g_table[2 * i + 1] = ~(unsigned long long)i;
  }
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  std::vector<std::string> toks;
  {
    std::string cur;
    int ch;
    while ((ch = fgetc(f)) != EOF) {
      if (ch == '\n') {
        if (!cur.empty()) toks.push_back(cur);
        cur.clear();
      } else {
        cur.push_back((char)ch);
      }
    }
    if (!cur.empty()) toks.push_back(cur);
  }
  fclose(f);
  const uint32_t flags = (uint32_t)atoi(argv[2]);
  g_rng.seed(strtoull(argv[3], nullptr, 10));
  host_wave_vote = vote;

  Tile* tile = new Tile();
  S& sm = tile->sm;
  for (int i = 0; i < 20; ++i) {
    unsigned long long p = 1;
    for (int k = 0; k < i; ++k) p *= 10;
    sm.pow10[i] = p;
  }
  for (int i = 0; i < 16; ++i)
    sm.keep8[i] = i >= 8 ? 0ull : (~0ull << (8 * i)) & 0x0F0F0F0F0F0F0F0Full;
  for (int i = 0; i < 256; ++i) sm.delim_lut[i] = i == '\n';
  static const char kNoise[] = "0123456789012345678901234567890123456789.-+eE\n\n\n";
  const int span = S::kBytes + S::kExtBytes;
  long bad = 0, n = 0;
  for (int pass = 0; pass < 2; ++pass) {
    g_random_wave = pass == 1;
    for (const std::string& t : toks) {
      if ((int)t.size() + 2 > span) continue;
      uint8_t* text = sm.text;
      for (size_t i = 0; i < sizeof(sm.text); ++i) text[i] = kNoise[g_rng() % (sizeof(kNoise) - 1)];
      const int s = 1 + (int)(g_rng() % (uint64_t)(span - t.size() - 1));
      uint8_t* tb = text + S::kPadFront;
      tb[s - 1] = '\n';
      memcpy(tb + s, t.data(), t.size());
      tb[s + t.size()] = '\n';
      build_bitmaps(sm);
      const std::string ref_text = t;
      const Lexed ref = lex_token(BufSrc{&ref_text}, 0, flags);
      const FastLex fl = fast_lex<K, false>(sm, (uint32_t)s, flags, g_table);
      Lexed got;
      const char* path = "fast";
      if (fl.code == kFastSlow) {
        got = long_lex<K>(sm, (uint32_t)s, flags);
        path = "long";
      } else {
        got.w = fl.w;
        got.q = fl.q;
        got.neg = fl.neg;
        got.kind = fl.code == kFastInvalid ? kLexInvalid : kLexExact;
      }
      // exponents beyond +-100000 decide alike (far outside the table); the
      // byte lexer saturates them there
      auto sat = [](int32_t q) { return q < -100000 ? -100000 : (q > 100000 ? 100000 : q); };
      bool ok = got.kind == ref.kind;
      if (ok && ref.kind != kLexInvalid)
        ok = got.w == ref.w && sat(got.q) == sat(ref.q) && got.neg == ref.neg;
      if (ok && fl.code == kFastOk) {  // the fast lexer's table entry is q's
        const TableEntry e = table_entry(g_table, fl.q);
        ok = fl.ent.hi == e.hi && fl.ent.lo == e.lo;
      }
      ++n;
      if (!ok) {
        if (bad < 10)
          printf("MISMATCH %s pass %d s %d token '%s': got kind %u w %llu q %d neg %u; "
                 "ref kind %u w %llu q %d neg %u\n",
                 path, pass, s, t.c_str(), got.kind, (unsigned long long)got.w, got.q, got.neg,
                 ref.kind, (unsigned long long)ref.w, ref.q, ref.neg);
        ++bad;
      }
    }
  }
  printf("%ld %ld\n", n, bad);
  delete tile;
  return 0;
}
