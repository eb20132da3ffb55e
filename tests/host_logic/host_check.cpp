// Host build of the library's per-token logic (lexer, Algorithm 1 and the
// w / w+1 test from ffp_device.h), used only by the CPU unit tests: it lets
// the oracle check that logic without a GPU.  Tokens that the logic sends to
// the exact fallback (a wavefront-cooperative GPU kernel) are marked with
// status 255; they, the tile scan and every other part of the kernels are
// covered by the GPU tests.
//
// usage: host_check <text file> <f64|f32|f16|bf16> <flags> <out file> [delimiters]
// writes, per token, the encoding zero-extended to 64 bits and a status
// byte; prints the number of tokens and of fallback decisions.
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "ffp_device.h"
#include "ffp_table.inc"

alignas(16) static const unsigned long long kTable[FFP_TABLE_SIZE * 2] = {FFP_TABLE_ENTRIES};

template <class F>
static void run(const std::vector<uint8_t>& buf, const ffp::DelimSet& ds, uint32_t flags,
                FILE* out, long* ntok, long* nfb) {
  const ffp::GlobalSrc src{buf.data(), buf.size(), ds};
  uint64_t i = 0, n = buf.size();
  while (i < n) {
    if (ffp::is_delim(ds, buf[i])) {
      ++i;
      continue;
    }
    const uint64_t start = i;
    while (i < n && !ffp::is_delim(ds, buf[i])) ++i;
    const ffp::Lexed L = ffp::lex_token(src, start, flags);
    ffp::Decision<F> d = ffp::decide_lexed<F>(L, kTable, flags);
    uint64_t bits = d.bits;
    uint8_t st = (uint8_t)d.status;
    if (d.fallback) {
      st = 255;
      ++*nfb;
    }
    fwrite(&bits, 8, 1, out);
    fwrite(&st, 1, 1, out);
    ++*ntok;
  }
}

int main(int argc, char** argv) {
  if (argc < 5) {
    fprintf(stderr, "usage: %s text f64|f32|f16|bf16 flags out [delims]\n", argv[0]);
    return 2;
  }
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  std::vector<uint8_t> buf;
  uint8_t tmp[1 << 16];
  size_t r;
  while ((r = fread(tmp, 1, sizeof(tmp), f)) > 0) buf.insert(buf.end(), tmp, tmp + r);
  fclose(f);
  ffp::DelimSet ds{};
  const char* delims = argc > 5 ? argv[5] : "\n";
  bool first = true;
  for (const char* p = delims; *p; ++p) {
    const unsigned c = (unsigned char)*p;
    ds.bits[c >> 6] |= 1ull << (c & 63);
    if (first) ds.byte = c;
    first = false;
  }
  ds.single = strlen(delims) == 1;
  const uint32_t flags = (uint32_t)atoi(argv[3]);
  FILE* out = fopen(argv[4], "wb");
  if (!out) return 2;
  long ntok = 0, nfb = 0;
  if (strcmp(argv[2], "f64") == 0)
    run<ffp::F64>(buf, ds, flags, out, &ntok, &nfb);
  else if (strcmp(argv[2], "f32") == 0)
    run<ffp::F32>(buf, ds, flags, out, &ntok, &nfb);
  else if (strcmp(argv[2], "f16") == 0)
    run<ffp::F16>(buf, ds, flags, out, &ntok, &nfb);
  else
    run<ffp::BF16>(buf, ds, flags, out, &ntok, &nfb);
  fclose(out);
  printf("%ld %ld\n", ntok, nfb);
  return 0;
}
