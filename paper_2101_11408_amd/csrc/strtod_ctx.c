/* Context measurement beside the GPU parser (not part of it): the C
 * library's strtod / strtof over every newline-separated token of a buffer,
 * on one or more threads, as the paper's experiments time conventional
 * parsers (Section 12).  Built into its own small library; the benchmark
 * calls it through ctypes. */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

struct part {
  const char* begin;
  const char* end;
  int as_float;
  uint64_t tokens;
  double checksum;
};

static void* parse_part(void* arg) {
  struct part* p = (struct part*)arg;
  const char* s = p->begin;
  double sum = 0.0;
  uint64_t n = 0;
  while (s < p->end) {
    if (*s == '\n') {
      ++s;
      continue;
    }
    char* e = NULL;
    if (p->as_float)
      sum += (double)strtof(s, &e);
    else
      sum += strtod(s, &e);
    ++n;
    /* skip whatever the parser did not consume up to the delimiter */
    while (e < p->end && *e != '\n') ++e;
    s = e;
  }
  p->tokens = n;
  p->checksum = sum;
  return NULL;
}

static double now_s(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* Parses buf[0, n) `reps` times with `threads` threads (each a contiguous
 * share cut at newlines) and returns the shortest wall time in seconds;
 * *tokens receives the token count.  Returns a negative value on failure. */
double ffp_ctx_strtod_seconds(const char* buf, uint64_t n, int as_float, int threads, int reps,
                              uint64_t* tokens) {
  if (threads < 1 || threads > 256 || reps < 1) return -1.0;
  char* text = (char*)malloc(n + 1); /* NUL-terminated copy: parsers stop there */
  if (!text) return -1.0;
  memcpy(text, buf, n);
  text[n] = 0;
  struct part parts[256];
  pthread_t tid[256];
  const char* cut = text;
  for (int t = 0; t < threads; ++t) {
    const char* end = t == threads - 1 ? text + n : text + (n * (uint64_t)(t + 1)) / threads;
    if (end < cut) end = cut;
    while (end < text + n && *end != '\n') ++end;
    parts[t].begin = cut;
    parts[t].end = end;
    parts[t].as_float = as_float;
    cut = end;
  }
  double best = 1e30;
  uint64_t total = 0;
  for (int r = 0; r < reps; ++r) {
    const double t0 = now_s();
    for (int t = 0; t < threads; ++t) pthread_create(&tid[t], NULL, parse_part, &parts[t]);
    for (int t = 0; t < threads; ++t) pthread_join(tid[t], NULL);
    const double dt = now_s() - t0;
    if (dt < best) best = dt;
    total = 0;
    for (int t = 0; t < threads; ++t) total += parts[t].tokens;
  }
  free(text);
  *tokens = total;
  return best;
}
