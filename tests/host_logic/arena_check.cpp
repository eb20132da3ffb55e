// Randomised check of the request server's arena (ffp_arena.h) against a
// byte-map model: every allocation lands at the lowest offset where a free
// run of that length starts (first fit), no two live ranges overlap, the
// free ranges stay fully coalesced, and the used byte count matches.
// Prints "ok <operations>" or the first failure and exits nonzero.
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <vector>

#include "ffp_arena.h"

static int fail(const char* what, long step) {
  printf("FAIL %s at step %ld\n", what, step);
  return 1;
}

int main(int argc, char** argv) {
  const uint64_t size = argc > 1 ? strtoull(argv[1], nullptr, 10) : 4096;
  const long steps = argc > 2 ? strtol(argv[2], nullptr, 10) : 200000;
  std::mt19937_64 rng(argc > 3 ? strtoull(argv[3], nullptr, 10) : 1);
  ffp::Arena a;
  a.init(size);
  std::vector<uint8_t> used(size, 0);
  struct Live { uint64_t off, n; };
  std::vector<Live> live;
  uint64_t used_bytes = 0, peak = 0;
  for (long step = 0; step < steps; ++step) {
    const bool do_alloc = live.empty() || (rng() % 100) < 55;
    if (do_alloc) {
      const uint64_t n = 1 + rng() % (size >= 16 ? size / 8 : 2);
      // model: lowest start of a free run of n bytes
      uint64_t want = ~0ull, run = 0;
      for (uint64_t i = 0; i < size; ++i) {
        run = used[i] ? 0 : run + 1;
        if (run == n) { want = i + 1 - n; break; }
      }
      uint64_t off = 0;
      const bool ok = a.alloc(n, &off);
      if (ok != (want != ~0ull)) return fail("alloc success differs", step);
      if (!ok) continue;
      if (off != want) return fail("not first fit", step);
      for (uint64_t i = off; i < off + n; ++i) {
        if (used[i]) return fail("overlap", step);
        used[i] = 1;
      }
      live.push_back({off, n});
      used_bytes += n;
      if (used_bytes > peak) peak = used_bytes;
    } else {
      const size_t k = rng() % live.size();
      const Live l = live[k];
      live[k] = live.back();
      live.pop_back();
      a.release(l.off, l.n);
      for (uint64_t i = l.off; i < l.off + l.n; ++i) used[i] = 0;
      used_bytes -= l.n;
    }
    if (a.used() != used_bytes) return fail("used bytes", step);
    if (a.peak() != peak) return fail("peak bytes", step);
    // free ranges: exactly the maximal runs of free bytes
    uint64_t pos = 0;
    for (const auto& fr : a.free_ranges()) {
      if (fr.first < pos) return fail("free ranges out of order", step);
      for (uint64_t i = pos; i < fr.first; ++i)
        if (!used[i]) return fail("free byte outside the free ranges", step);
      for (uint64_t i = fr.first; i < fr.first + fr.second; ++i)
        if (used[i]) return fail("used byte inside a free range", step);
      const uint64_t end = fr.first + fr.second;
      if (end < size && !used[end]) return fail("free ranges not coalesced", step);
      if (fr.first > 0 && !used[fr.first - 1]) return fail("free ranges not coalesced", step);
      pos = end;
    }
    for (uint64_t i = pos; i < size; ++i)
      if (!used[i]) return fail("free byte after the last free range", step);
  }
  printf("ok %ld\n", steps);
  return 0;
}
