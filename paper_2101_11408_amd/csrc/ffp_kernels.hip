// HIP kernels of the parser (gfx950, wave64).
//
// One parse call runs four kernels on the caller's stream:
//   k_count     streams the text once and counts the tokens starting in each
//               64 KiB block (a token starts at a non-delimiter byte that
//               follows a delimiter or the start of the text);
//   k_scan      one workgroup turns the block counts into the index of each
//               block's first token and writes every job's token count;
//   k_parse     each workgroup walks whole blocks in LDS tiles: 16-byte
//               coalesced loads, digit and delimiter bitmaps, a block scan of
//               token starts, then one lane per token: lexing (Section 4),
//               Algorithm 1 (Sections 5-10) with the power-of-five table read
//               through the caches, and the w / w+1 test for long
//               significands (Section 11).  Undecided tokens go to a queue;
//   k_fallback  exact decision for the queued tokens, one wavefront per
//               token: big-integer comparison with the halfway points
//               between neighbouring binary values.
// No workgroup ever waits for another one.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ffp_device.h"
#include "ffp_fallback.h"
#include "ffp_internal.h"
#include "ffp_kernels.h"
#include "ffp_lexer.h"
#include "ffp_table.inc"

namespace ffp {

alignas(16) __device__ const unsigned long long g_table[FFP_TABLE_SIZE * 2] = {FFP_TABLE_ENTRIES};
// big powers 5^(27 i) for the exact fallback (one 64-bit limb per lane)
static_assert(FFP_POW5_LIMBS == kWave && FFP_POW5_STEPS == kPow5Steps &&
                  FFP_POW5_STEP == kPow5Step, "fallback power table layout");
alignas(16) __device__ const unsigned long long g_pow5[FFP_POW5_STEPS * FFP_POW5_LIMBS] = {
    FFP_POW5_ENTRIES};

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
#define FFP_GLOBAL __attribute__((address_space(1)))

template <class T>
__device__ __forceinline__ T gload(const T* p) {
  return *(const FFP_GLOBAL T*)p;  // address-space cast: a global load
}
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <class T>
__device__ __forceinline__ void gstore(T* p, T v) {
  *(FFP_GLOBAL T*)p = v;  // address-space cast: a global store
}

// Reduction of parsed values: a key whose unsigned order is the numeric
// order of the encodings of a `width`-bit format (-0 before +0).  NaN, and
// tokens whose status is not FFP_OK, are left out: their key is kNoMin for
// the minimum and kNoMax for the maximum.
constexpr uint64_t kNoMin = ~0ull;
constexpr uint64_t kNoMax = 0ull;

__device__ __forceinline__ int dtype_width(uint32_t dtype) {
  return dtype == kF64 ? 64 : dtype == kF32 ? 32 : 16;
}

__device__ __forceinline__ uint64_t dtype_inf(uint32_t dtype) {
  return dtype == kF64 ? F64::kInf : dtype == kF32 ? F32::kInf : dtype == kF16 ? F16::kInf : BF16::kInf;
}

__device__ __forceinline__ bool order_key(uint64_t bits, uint32_t status, uint32_t dtype,
                                          uint64_t& key) {
  const int width = dtype_width(dtype);
  const uint64_t mag = bits & ((1ull << (width - 1)) - 1);
  if (status != kStOk || mag > dtype_inf(dtype)) return false;
  const uint64_t x = bits << (64 - width);
  key = (x >> 63) ? ~x : (x | (1ull << 63));
  return true;
}

__device__ __forceinline__ uint64_t key_to_bits(uint64_t key, uint32_t dtype) {
  const uint64_t x = (key >> 63) ? (key & ~(1ull << 63)) : ~key;
  return x >> (64 - dtype_width(dtype));
}

// An encoding with an order key (status OK, not NaN) as a term of the exact
// sum: value = (-1)^neg * m * 2^(b - 1074), b >= 0; inf for infinities.
// Per format: b = max(field, 1) - bias - (precision - 1) + 1074.
struct SumTerm {
  uint64_t m;
  int b;
  bool neg, inf;
};

__device__ __forceinline__ SumTerm sum_term(uint64_t bits, uint32_t dtype) {
  const int t = dtype == kF64 ? 52 : dtype == kF32 ? 23 : dtype == kF16 ? 10 : 7;
  const int ew = dtype == kF64 ? 11 : dtype == kF16 ? 5 : 8;
  const int bias = (1 << (ew - 1)) - 1;
  const uint32_t field = (uint32_t)(bits >> t) & ((1u << ew) - 1);
  SumTerm r;
  r.neg = (bits >> (t + ew)) & 1;
  r.inf = field == (1u << ew) - 1;
  r.m = (bits & ((1ull << t) - 1)) | (field ? 1ull << t : 0ull);
  r.b = (int)(field ? field : 1u) - bias - t + 1074;
  return r;
}

// Adds a term's magnitude to an accumulator (kSumLimbs words, in LDS or in
// global memory): m << (b mod 32) in three 32-bit pieces.
__device__ __forceinline__ void sum_add(unsigned long long* acc, const SumTerm& x) {
  unsigned long long* a = acc + (x.b >> 5);
  const int r = x.b & 31;
  const uint64_t lo = x.m << r;
  const uint64_t hi = r ? x.m >> (64 - r) : 0ull;
  if (lo & 0xFFFFFFFFull) atomicAdd(a, (unsigned long long)(lo & 0xFFFFFFFFull));
  if (lo >> 32) atomicAdd(a + 1, (unsigned long long)(lo >> 32));
  if (hi) atomicAdd(a + 2, (unsigned long long)hi);
}

__device__ __forceinline__ uint32_t sum_flag_bits(const SumTerm& x) {
  uint32_t f = kSumAny;
  if (x.inf) f |= x.neg ? kSumNegInf : kSumPosInf;
  if (!(x.neg && x.m == 0)) f |= kSumNotNegZero;
  return f;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
  for (int d = 32; d > 0; d >>= 1) {
    const uint64_t o = __shfl_xor(v, d, kWave);
    v = o < v ? o : v;
  }
  return v;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
  for (int d = 32; d > 0; d >>= 1) {
    const uint64_t o = __shfl_xor(v, d, kWave);
    v = o > v ? o : v;
  }
  return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// Exclusive scan over the threads of a block of `nthreads` threads; `total`
// receives the sum.  s_tmp holds nthreads / 64 words and must not be reused
// before the next barrier.
template <int nthreads, class T>
__device__ __forceinline__ T block_excl_scan(T v, T& total, T* s_tmp) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  T x = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const T y = __shfl_up(x, d, kWave);
    if (lane >= d) x += y;
  }
  if (lane == kWave - 1) s_tmp[wid] = x;
  __syncthreads();
  T before = 0, sum = 0;
#pragma unroll
  for (int i = 0; i < nthreads / kWave; ++i) {
    const T t = s_tmp[i];
    before += (i < wid) ? t : 0;
    sum += t;
  }
  total = sum;
  return before + x - v;
}

// Public error codes written into job records (include/ffp.h).
constexpr int32_t kErrArg = -1;       // FFP_E_ARG
constexpr int32_t kErrCapacity = -2;  // FFP_E_CAPACITY
constexpr int32_t kErrQueue = -7;     // FFP_E_QUEUE

// Job that owns global block b.
__device__ __forceinline__ JobDesc job_of_block(const JobSet& js, uint64_t b) {
  if (!js.jobs) return js.single;
  uint32_t lo = 0, hi = js.njobs;  // last job with block_begin <= b
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (js.jobs[mid].block_begin <= b) lo = mid; else hi = mid;
  }
  return js.jobs[lo];
}

__device__ __forceinline__ uint64_t total_blocks_of(const JobSet& js) {
  return js.jobs ? *js.total_blocks_dev : js.total_blocks;
}

// Blocks of a job: its text starts `align` bytes into the first block.
__device__ __forceinline__ uint64_t job_blocks(const JobDesc& job, uint32_t shift) {
  if (job.nbytes == 0) return 0;
  const uint64_t vend = job.nbytes + ((uint64_t)(uintptr_t)job.text & 15u);
  return (vend + (1ull << shift) - 1) >> shift;
}


// 16 bytes of virtual text [off, off+16) of a job: one aligned load inside the
// text; byte by byte at its two ends, where bytes outside the text read as a
// delimiter and no memory outside it is touched.
__device__ __forceinline__ uint4 load_chunk(const uint8_t* vbase, uint64_t off, uint64_t align,
                                            uint64_t vend, uint32_t pad) {
  if (off >= align && off + kChunk <= vend) {
    const u32x4 v = gload(reinterpret_cast<const u32x4*>(vbase + off));
    return make_uint4(v.x, v.y, v.z, v.w);
  }
  uint32_t wds[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    uint32_t word = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const uint64_t o = off + k * 4 + b;
      const uint32_t byte = (o >= align && o < vend) ? (uint32_t)gload(vbase + o) : pad;
      word |= byte << (8 * b);
    }
    wds[k] = word;
  }
  return make_uint4(wds[0], wds[1], wds[2], wds[3]);
}

// High bit of each byte of x set when the byte is not in a set of 2 to 4
// bytes (DelimSet::few): one byte comparison per member.
__device__ __forceinline__ uint32_t nondelim_word_few(uint32_t x, const DelimSet& d) {
  uint32_t eq = byte_eq_word(x, d.few[0]) | byte_eq_word(x, d.few[1]);
  if (d.nfew > 2) eq |= byte_eq_word(x, d.few[2]) | byte_eq_word(x, d.few[3]);
  return ~eq & 0x80808080u;
}

// Non-delimiter bits of 16 bytes: a lone delimiter below 0x80 by the
// three-operation byte test, sets of 2 to 4 such bytes by one comparison per
// member (kFew), larger sets from the LDS table.  Loops over many chunks
// take the kFew decision outside the loop (one branch per loop, not per
// chunk, keeps the registers of the unrolled loop down).
template <bool kSingle, bool kFew = false>
__device__ __forceinline__ uint32_t nondelim_mask16(uint4 v, uint32_t drep, const uint8_t* lut,
                                                    const DelimSet& d) {
  if (kSingle)
    return pack_high_bits(nondelim_word(v.x, drep), nondelim_word(v.y, drep),
                          nondelim_word(v.z, drep), nondelim_word(v.w, drep));
  if (kFew)
    return pack_high_bits(nondelim_word_few(v.x, d), nondelim_word_few(v.y, d),
                          nondelim_word_few(v.z, d), nondelim_word_few(v.w, d));
  return pack_high_bits(nondelim_word_lut(v.x, lut), nondelim_word_lut(v.y, lut),
                        nondelim_word_lut(v.z, lut), nondelim_word_lut(v.w, lut));
}

// The same with the kFew decision taken at run time (single chunks).
template <bool kSingle>
__device__ __forceinline__ uint32_t nondelim_mask16_any(uint4 v, uint32_t drep, const uint8_t* lut,
                                                        const DelimSet& d) {
  return !kSingle && d.nfew ? nondelim_mask16<kSingle, true>(v, drep, lut, d)
                            : nondelim_mask16<kSingle, false>(v, drep, lut, d);
}

// ---------------------------------------------------------------------------
// JSON documents (FFP_JSON_DOCUMENT).  A quote preceded by an odd number of
// consecutive backslashes is escaped; the others open and close strings.
// Token bytes are the non-delimiters (escaped quotes included) outside
// strings, and a token must start with '-' or a digit.
// ---------------------------------------------------------------------------

// Whether the quote at text[pos] is escaped: the backslashes right before it,
// walked back one by one inside the text.
__device__ __forceinline__ bool quote_escaped(const uint8_t* text, uint64_t pos) {
  uint32_t odd = 0;
  while (pos > 0 && gload(text + pos - 1) == '\\') {
    --pos;
    odd ^= 1u;
  }
  return odd != 0;
}

struct DocBits {
  uint32_t uq;  // unescaped quotes
  uint32_t eq;  // escaped quotes (ordinary bytes)
  uint32_t ms;  // bytes a number may start with: '-' and digits
};

// Quote classes of the 16 bytes v whose first byte is text[pos] (pos < 0 for
// padding before the text: padding holds no quote).  dgm: the digit mask.
__device__ __forceinline__ DocBits doc_chunk(uint4 v, uint32_t dgm, const uint8_t* text,
                                             int64_t pos) {
  constexpr uint32_t kQ = '"' * 0x01010101u, kB = '\\' * 0x01010101u, kM = '-' * 0x01010101u;
  const uint32_t qm = pack_high_bits(byte_eq_word(v.x, kQ), byte_eq_word(v.y, kQ),
                                     byte_eq_word(v.z, kQ), byte_eq_word(v.w, kQ));
  DocBits d;
  d.uq = qm;
  d.eq = 0;
  d.ms = dgm | pack_high_bits(byte_eq_word(v.x, kM), byte_eq_word(v.y, kM),
                              byte_eq_word(v.z, kM), byte_eq_word(v.w, kM));
  if (qm) {
    const uint32_t bm = pack_high_bits(byte_eq_word(v.x, kB), byte_eq_word(v.y, kB),
                                       byte_eq_word(v.z, kB), byte_eq_word(v.w, kB));
    // quotes right after a backslash may be escaped
    uint32_t cand = qm & (bm << 1);
    if ((qm & 1u) && pos > 0 && gload(text + pos - 1) == '\\') cand |= 1u;
    while (cand) {
      const int k = __builtin_ctz(cand);
      cand &= cand - 1;
      if (quote_escaped(text, (uint64_t)(pos + k))) {
        d.uq &= ~(1u << k);
        d.eq |= 1u << k;
      }
    }
  }
  return d;
}

// Bytes inside a string among 16 whose unescaped quotes are uq, given the
// state before the first of them (an opening quote is outside, a closing
// one inside).
__device__ __forceinline__ uint32_t doc_in_string(uint32_t uq, uint32_t carry) {
  const uint32_t before = (prefix_xor16(uq) << 1) & 0xFFFFu;
  return carry ? (~before & 0xFFFFu) : before;
}

// Whether the byte before text[pos] is a token byte, for a position whose
// string state is `in_string`.
__device__ __forceinline__ uint32_t doc_prev_token(const uint8_t* text, int64_t pos,
                                                   uint32_t in_string, const DelimSet& d) {
  if (pos <= 0 || in_string) return 0;
  const uint32_t c = gload(text + pos - 1);
  if (c == '"') return quote_escaped(text, (uint64_t)(pos - 1)) ? 1u : 0u;
  return is_delim(d, c) ? 0u : 1u;
}

// Is the byte just before virtual offset off a non-delimiter?
__device__ __forceinline__ uint32_t prev_nondelim(const uint8_t* vbase, uint64_t off,
                                                  uint64_t align, const DelimSet& d) {
  if (off <= align) return 0;  // start of the text
  return is_delim(d, gload(vbase + off - 1)) ? 0u : 1u;
}

// The call's device state starts clean: the parse kernel appends to the
// queue and raises error bits; the reduction starts from its identities.
__device__ __forceinline__ void reset_call_state(DeviceState* st) {
  st->queue_tail = 0;
  st->error = 0;
  st->dense = 0;
  st->red_min = ~0ull;
  st->red_max = 0;
  st->red_count = 0;
  st->sum_flags = 0;
}

// What a call without the count kernel needs clean: its queue and error.
__device__ __forceinline__ void reset_spare_state(DeviceState* st) {
  st->queue_tail = 0;
  st->error = 0;
}

// The exact sum's accumulators, cleared by the threads of one workgroup.
__device__ __forceinline__ void reset_sum_state(DeviceState* st, int tid, int nthreads) {
  for (int i = tid; i < 2 * kSumLimbs; i += nthreads) (&st->sum_acc[0][0])[i] = 0;
}

// ---------------------------------------------------------------------------
// k_count: tokens starting in each block.  Each thread classifies kRows
// chunks of 16 bytes (kRows = block bytes / 4 KiB); the start mask of a chunk
// needs the last bit of the chunk before it, exchanged through LDS.
// ---------------------------------------------------------------------------
// k_count for JSON documents: per block, the tokens starting in it if it
// begins outside a string and if it begins inside one, and the parity of its
// unescaped quotes.  Rows of 256 chunks are scanned one after the other for
// the string state; s_tb (a byte per chunk) passes the last token bit of
// each chunk, for both entry states, to the next chunk's thread.
template <int kRows>
__device__ void count_json_doc(const CountParams& P, const uint8_t* lut, uint32_t* s_scan,
                               uint8_t* s_tb) {
  constexpr uint32_t kShift = kRows == 1 ? 12 : (kRows == 4 ? 14 : 16);
  __shared__ uint32_t s_prev2;
  const int tid = threadIdx.x;
  const uint64_t nblk = total_blocks_of(P.js);
  for (uint64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    const JobDesc job = job_of_block(P.js, b);
    const uint64_t align = (uint64_t)(uintptr_t)job.text & 15u;
    const uint8_t* vbase = job.text - align;
    const uint64_t vend = job.nbytes + align;
    const uint64_t bstart = (b - job.block_begin) << kShift;
    __syncthreads();  // s_tb / s_prev2 / s_scan of the previous block are consumed
    uint32_t t0[kRows], t1[kRows], ms[kRows];
    uint32_t parity = 0;  // unescaped quotes before the row, mod 2
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      const uint64_t off = bstart + (uint64_t)(r * kThreads + tid) * kChunk;
      uint32_t base = 0, uq = 0;
      ms[r] = 0;
      if (off < vend) {
        const uint4 v = load_chunk(vbase, off, align, vend, P.delim.byte);
        const uint32_t dgm = pack_high_bits(digit_word(v.x), digit_word(v.y), digit_word(v.z),
                                            digit_word(v.w));
        const DocBits d = doc_chunk(v, dgm, job.text, (int64_t)off - (int64_t)align);
        base = nondelim_mask16<false>(v, 0u, lut, P.delim) | d.eq;
        uq = d.uq;
        ms[r] = d.ms;
      }
      uint32_t rowq;
      const uint32_t ex = block_excl_scan<kThreads>((uint32_t)__popc(uq), rowq, s_scan);
      const uint32_t in0 = doc_in_string(uq, (parity + ex) & 1u);
      t0[r] = base & ~in0;
      t1[r] = base & in0;
      s_tb[r * kThreads + tid] = (uint8_t)(((t0[r] >> 15) & 1u) | (((t1[r] >> 15) & 1u) << 1));
      parity = (parity + rowq) & 1u;
      __syncthreads();  // s_scan is read before the next row writes it
    }
    if (tid == 0) {
      const int64_t pos = (int64_t)bstart - (int64_t)align;
      s_prev2 = doc_prev_token(job.text, pos, 0u, P.delim) |
                (doc_prev_token(job.text, pos, 1u, P.delim) << 1);
    }
    __syncthreads();
    uint32_t n0 = 0, n1 = 0;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      const int chunk = r * kThreads + tid;
      const uint32_t pb = chunk == 0 ? s_prev2 : (uint32_t)s_tb[chunk - 1];
      n0 += __popc(t0[r] & ~((t0[r] << 1) | (pb & 1u)) & ms[r] & 0xFFFFu);
      n1 += __popc(t1[r] & ~((t1[r] << 1) | (pb >> 1)) & ms[r] & 0xFFFFu);
    }
    uint32_t total;
    (void)block_excl_scan<kThreads>(n0 | (n1 << 16), total, s_scan);
    if (tid == 0)
      P.block_sum[b] = (uint64_t)(total & 0xFFFFu) | ((uint64_t)(total >> 16) << 32) |
                       ((uint64_t)parity << 63);
  }
}

// ---------------------------------------------------------------------------
// CSV number columns (FFP_CSV): rows end at '\n', fields are separated by
// ',', and a token's column is the number of ',' bytes between the last '\n'
// before it (or the text's start) and the token.  The column state is a
// segmented count: a '\n' resets it, a ',' adds one.
// ---------------------------------------------------------------------------
struct CsvBits {
  uint32_t nl, cm;  // '\n' and ',' bytes of 16 (bits outside the text cleared)
};

// The bytes of a chunk at virtual offset off that lie in the text [align, vend).
__device__ __forceinline__ uint32_t text_bits(uint64_t off, uint64_t align, uint64_t vend) {
  uint32_t valid = 0xFFFFu;
  if (off < align) valid &= 0xFFFFu << (uint32_t)(align - off);
  if (off + kChunk > vend) valid &= off >= vend ? 0u : (1u << (uint32_t)(vend - off)) - 1u;
  return valid;
}

__device__ __forceinline__ CsvBits csv_chunk(uint4 v, uint32_t valid) {
  constexpr uint32_t kNl = '\n' * 0x01010101u, kCm = ',' * 0x01010101u;
  CsvBits b;
  b.nl = pack_high_bits(byte_eq_word(v.x, kNl), byte_eq_word(v.y, kNl), byte_eq_word(v.z, kNl),
                        byte_eq_word(v.w, kNl)) & valid;
  b.cm = pack_high_bits(byte_eq_word(v.x, kCm), byte_eq_word(v.y, kCm), byte_eq_word(v.z, kCm),
                        byte_eq_word(v.w, kCm)) & valid;
  return b;
}

// Segment word of a run of bytes: bit 31 set when the run holds a '\n';
// bits 0..30 the ',' bytes after its last '\n' (all of them without one).
constexpr uint32_t kSegNl = 0x80000000u;

__device__ __forceinline__ uint32_t csv_seg(const CsvBits& b) {
  if (b.nl) return kSegNl | (uint32_t)__popc(b.cm >> (31 - __builtin_clz(b.nl)));
  return (uint32_t)__popc(b.cm);
}

// The segment word of run a followed by run b (0 is the empty run).
__device__ __forceinline__ uint32_t csv_seg_then(uint32_t a, uint32_t b) {
  return (b & kSegNl) ? b : (a & kSegNl) | ((a + b) & ~kSegNl);
}

// Exclusive scan of segment words over the kThreads threads of a block (in
// thread order); `total` receives the whole block's word.  s_tmp holds
// kThreads / kWave words and must not be reused before the next barrier.
__device__ __forceinline__ uint32_t block_excl_segscan(uint32_t x, uint32_t& total,
                                                       uint32_t* s_tmp) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  uint32_t inc = x;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t o = __shfl_up(inc, d, kWave);
    if (lane >= d) inc = csv_seg_then(o, inc);
  }
  if (lane == kWave - 1) s_tmp[wid] = inc;
  uint32_t ex = __shfl_up(inc, 1, kWave);
  if (lane == 0) ex = 0;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kThreads / kWave; ++w) {
    if (w < wid) pre = csv_seg_then(pre, s_tmp[w]);
    tot = csv_seg_then(tot, s_tmp[w]);
  }
  total = tot;
  return csv_seg_then(pre, ex);
}

// Column at virtual offset vstart (a multiple of the chunk size) of a job:
// the ',' bytes back to the last '\n' before it, read backwards 4 KiB at a
// time by the whole workgroup (the same value in every thread).
__device__ uint32_t csv_entry_column(const uint8_t* vbase, uint64_t align, uint64_t vend,
                                     uint64_t vstart, uint32_t* s_tmp) {
  const int tid = threadIdx.x;
  uint32_t acc = 0;  // segment word of [window start, vstart)
  uint64_t hi = vstart;
  while (hi > 0) {
    const uint64_t lo = hi > (uint64_t)kThreads * kChunk ? hi - (uint64_t)kThreads * kChunk : 0;
    const uint64_t off = lo + (uint64_t)tid * kChunk;
    uint32_t seg = 0;
    if (off < hi) seg = csv_seg(csv_chunk(load_chunk(vbase, off, align, vend, 0u),
                                          text_bits(off, align, vend)));
    uint32_t tot;
    (void)block_excl_segscan(seg, tot, s_tmp);
    __syncthreads();  // s_tmp is consumed
    acc = csv_seg_then(tot, acc);
    if (acc & kSegNl) break;  // the same in every thread
    hi = lo;
  }
  return acc & ~kSegNl;
}

// The starts among `starts` (bits of one chunk) whose column, given the
// column `entry` at the chunk's first byte, is selected.
__device__ __forceinline__ uint32_t csv_select(uint32_t starts, const CsvBits& b, uint32_t entry,
                                               uint64_t columns) {
  uint32_t keep = 0;
  while (starts) {
    const int k = __builtin_ctz(starts);
    starts &= starts - 1;
    const uint32_t below = (1u << k) - 1u;
    const uint32_t nlb = b.nl & below;
    uint32_t col;
    if (nlb) {
      const uint32_t after = ~((2u << (31 - __builtin_clz(nlb))) - 1u);
      col = (uint32_t)__popc(b.cm & below & after);
    } else {
      col = entry + (uint32_t)__popc(b.cm & below);
    }
    if (col < 64 && ((columns >> col) & 1u)) keep |= 1u << k;
  }
  return keep;
}

// k_count for CSV: per block, the tokens of the selected columns.  The
// column at the block's start comes from a backward read to the last '\n';
// within the block, rows of 256 chunks are scanned one after the other.
template <int kRows>
__device__ void count_csv(const CountParams& P, const uint8_t* lut, uint32_t* s_scan,
                          uint16_t* s_nd) {
  constexpr uint32_t kShift = kRows == 1 ? 12 : (kRows == 4 ? 14 : 16);
  __shared__ uint32_t s_prev;
  const int tid = threadIdx.x;
  const uint64_t nblk = total_blocks_of(P.js);
  for (uint64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    const JobDesc job = job_of_block(P.js, b);
    const uint64_t align = (uint64_t)(uintptr_t)job.text & 15u;
    const uint8_t* vbase = job.text - align;
    const uint64_t vend = job.nbytes + align;
    const uint64_t bstart = (b - job.block_begin) << kShift;
    __syncthreads();  // s_nd / s_prev / s_scan of the previous block are consumed
    uint32_t col = csv_entry_column(vbase, align, vend, bstart, s_scan);
    if (tid == 0) s_prev = prev_nondelim(vbase, bstart, align, P.delim);
    uint32_t n = 0;
    // one row at a time (no per-row arrays: this kernel serves every
    // delimiter set, and its registers bound its occupancy)
#pragma unroll 1
    for (int r = 0; r < kRows; ++r) {
      const int chunk = r * kThreads + tid;
      const uint64_t off = bstart + (uint64_t)chunk * kChunk;
      const uint4 v = load_chunk(vbase, off, align, vend, P.delim.byte);
      const uint32_t m = off < vend ? nondelim_mask16_any<false>(v, 0u, lut, P.delim) : 0u;
      const CsvBits cb = csv_chunk(v, text_bits(off, align, vend));
      s_nd[chunk] = (uint16_t)m;
      uint32_t row;
      // (its barrier also publishes s_nd and s_prev)
      const uint32_t ex = block_excl_segscan(csv_seg(cb), row, s_scan);
      const uint32_t pb = chunk == 0 ? s_prev : ((uint32_t)s_nd[chunk - 1] >> 15);
      const uint32_t entry = (ex & kSegNl) ? (ex & ~kSegNl) : col + ex;
      n += __popc(csv_select(m & ~((m << 1) | pb) & 0xFFFFu, cb, entry, P.csv_columns));
      col = (row & kSegNl) ? (row & ~kSegNl) : col + row;
      __syncthreads();  // s_scan is read before the next row writes it
    }
    uint32_t total;
    (void)block_excl_scan<kThreads>(n, total, s_scan);
    if (tid == 0) P.block_sum[b] = total;
  }
}

template <bool kSingle, int kRows>
__global__ __launch_bounds__(kThreads) void k_count(CountParams P) {
  constexpr int kCountRows = kRows;
  constexpr uint32_t kShift = kRows == 1 ? 12 : (kRows == 4 ? 14 : 16);
  __shared__ uint16_t s_nd[kCountRows * kThreads];
  __shared__ uint8_t s_lut[256];
  __shared__ uint32_t s_scan[kThreads / kWave];
  __shared__ uint32_t s_prev;
  __shared__ uint64_t s_tiles[kThreads / kWave];  // 64 KiB blocks: per-wave tile starts
  const int tid = threadIdx.x;
  if (!kSingle)
    for (int i = tid; i < 256; i += kThreads) s_lut[i] = is_delim(P.delim, (uint32_t)i);
  const uint32_t drep = P.delim.byte * 0x01010101u;
  if (P.reset_state && blockIdx.x == 0) {
    if (tid == 0) {
      reset_call_state(P.st);
      if (P.spare) {
        reset_spare_state(P.spare);
        reset_spare_state(P.spare + 1);
      }
    }
    reset_sum_state(P.st, tid, kThreads);
  }
  const uint64_t nblk = total_blocks_of(P.js);
  if (!kSingle && P.json_doc) {
    count_json_doc<kRows>(P, s_lut, s_scan, reinterpret_cast<uint8_t*>(s_nd));
    return;
  }
  if (!kSingle && P.csv) {
    __syncthreads();  // the delimiter table is written
    count_csv<kRows>(P, s_lut, s_scan, s_nd);
    return;
  }
  for (uint64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    const JobDesc job = job_of_block(P.js, b);
    const uint64_t align = (uint64_t)(uintptr_t)job.text & 15u;
    const uint8_t* vbase = job.text - align;
    const uint64_t vend = job.nbytes + align;
    const uint64_t bstart = (b - job.block_begin) << kShift;
    __syncthreads();  // s_nd / s_prev of the previous block are consumed
    uint32_t m[kCountRows];
    if (!kSingle && P.delim.nfew) {
#pragma unroll
      for (int r = 0; r < kCountRows; ++r) {
        const uint64_t off = bstart + (uint64_t)(r * kThreads + tid) * kChunk;
        m[r] = off < vend ? nondelim_mask16<kSingle, true>(
                                load_chunk(vbase, off, align, vend, P.delim.byte), drep, s_lut,
                                P.delim)
                          : 0u;
        s_nd[r * kThreads + tid] = (uint16_t)m[r];
      }
    } else {
#pragma unroll
      for (int r = 0; r < kCountRows; ++r) {
        const uint64_t off = bstart + (uint64_t)(r * kThreads + tid) * kChunk;
        m[r] = off < vend ? nondelim_mask16<kSingle, false>(
                                load_chunk(vbase, off, align, vend, P.delim.byte), drep, s_lut,
                                P.delim)
                          : 0u;
        s_nd[r * kThreads + tid] = (uint16_t)m[r];
      }
    }
    if (tid == 0) s_prev = prev_nondelim(vbase, bstart, align, P.delim);
    __syncthreads();
    uint32_t n = 0;
    // 64 KiB blocks: the starts of each 16 KiB tile (rows 4t .. 4t+3), one
    // 16-bit field per tile (at most 8192 starts each)
    uint64_t tiles = 0;
#pragma unroll
    for (int r = 0; r < kCountRows; ++r) {
      const int chunk = r * kThreads + tid;
      const uint32_t pb = chunk == 0 ? s_prev : ((uint32_t)s_nd[chunk - 1] >> 15);
      const uint32_t c = __popc(m[r] & ~((m[r] << 1) | pb) & 0xFFFFu);
      n += c;
      if (kCountRows == 16) tiles += (uint64_t)c << (16 * (r / 4));
    }
    if (kCountRows == 16) {
      // the block's total is the sum of its tiles' fields
      tiles = wave_sum_u64(tiles);
      if ((tid & (kWave - 1)) == 0) s_tiles[tid / kWave] = tiles;
      __syncthreads();
      if (tid == 0) {
        uint64_t t = 0;
#pragma unroll
        for (int w = 0; w < kThreads / kWave; ++w) t += s_tiles[w];
        uint64_t word = 0;
        bool dense = false;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          const uint64_t c = (t >> (16 * f)) & 0xFFFFu;
          word += c;
          dense = dense || c > kShortTileStarts;
        }
        // the flag only where the scan kernel runs and masks it off (calls
        // without it, P.reset_state, read these counts as they are)
        if (dense && !P.reset_state) word |= kDenseTileBit;
        P.block_sum[b] = word;
      }
    } else {
      uint32_t total;
      (void)block_excl_scan<kThreads>(n, total, s_scan);
      if (tid == 0) P.block_sum[b] = total;
    }
  }
}

// ---------------------------------------------------------------------------
// k_scan: exclusive prefix of the block counts (in place, one extra entry for
// the grand total), each job's token count, and the per-call reset of the
// fallback queue and the device error word.
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 8;

__global__ __launch_bounds__(kScanThreads) void k_scan(ScanParams P) {
  __shared__ uint32_t s_scan[kScanThreads / kWave];
  __shared__ uint64_t s_carry;
  const int tid = threadIdx.x;
  const uint64_t n = total_blocks_of(P.js);
  __shared__ uint32_t s_parity;  // JSON documents: inside a string before the round
  if (tid == 0) {
    s_carry = 0;
    s_parity = 0;
    reset_call_state(P.st);
    if (P.spare) {
      reset_spare_state(P.spare);
      reset_spare_state(P.spare + 1);
    }
  }
  reset_sum_state(P.st, tid, kScanThreads);
  // a block above P.dense_limit starts, or one with a dense 16 KiB tile
  // (plain counts only)
  bool dense = false;
  for (uint64_t base = 0; base < n; base += (uint64_t)kScanThreads * kScanPer) {
    uint64_t v[kScanPer];
    uint64_t sum = 0;
    uint32_t entry = 0;  // JSON documents: the blocks' string states (bit i)
    if (P.json_doc) {
      // a block begins inside a string when the quotes before it are odd in
      // number; its count is the one for that state
      uint32_t par = 0;
#pragma unroll
      for (int i = 0; i < kScanPer; ++i) {
        const uint64_t k = base + (uint64_t)tid * kScanPer + i;
        v[i] = k < n ? P.block_sum[k] : 0;
        par += (uint32_t)(v[i] >> 63);
      }
      __syncthreads();  // s_parity of the previous round is final
      uint32_t ptotal;
      uint32_t run = s_parity + block_excl_scan<kScanThreads>(par, ptotal, s_scan);
#pragma unroll
      for (int i = 0; i < kScanPer; ++i) {
        const uint32_t in = run & 1u;
        entry |= in << i;
        run += (uint32_t)(v[i] >> 63);
        v[i] = in ? (v[i] >> 32) & 0x7FFFFFFFull : v[i] & 0xFFFFFFFFull;
        sum += v[i];
      }
      __syncthreads();  // s_scan is read before the count scan writes it
      if (tid == 0) s_parity = (s_parity + ptotal) & 1u;
    } else {
#pragma unroll
      for (int i = 0; i < kScanPer; ++i) {
        const uint64_t k = base + (uint64_t)tid * kScanPer + i;
        v[i] = k < n ? P.block_sum[k] : 0;
        dense = dense || (v[i] & kDenseTileBit) ||
                (P.dense_limit && (v[i] & ~kDenseTileBit) > P.dense_limit);
        v[i] &= ~kDenseTileBit;
        sum += v[i];
      }
    }
    __syncthreads();  // s_carry of the previous round is final
    const uint64_t carry = s_carry;
    // a round covers 8192 blocks of 64 KiB with at most 32768 token starts
    // each: its sums fit in 32 bits
    uint32_t total;
    const uint32_t ex = block_excl_scan<kScanThreads>((uint32_t)sum, total, s_scan);
    uint64_t run = carry + ex;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
      const uint64_t k = base + (uint64_t)tid * kScanPer + i;
      if (k < n) P.block_sum[k] = run | ((uint64_t)((entry >> i) & 1u) << 63);
      run += v[i];
    }
    __syncthreads();
    if (tid == 0) s_carry = carry + total;
  }
  // (the barrier also makes s_carry final)
  if (__syncthreads_or(dense) && tid == 0) P.st->dense = 1;
  if (!P.js.jobs) {  // one job: its token count is the total
    if (tid == 0) {
      const uint64_t count = s_carry;
      P.block_sum[n] = count;
      *P.js.single.count_out = count;
      if (P.js.single.err_out && count > P.js.single.capacity) *P.js.single.err_out = kErrCapacity;
    }
    return;
  }
  if (tid == 0) P.block_sum[n] = s_carry;
  __syncthreads();
  // token count of every job: prefix at its end minus prefix at its start
  const uint32_t nj = P.js.njobs;
  for (uint32_t j = tid; j < nj; j += kScanThreads) {
    const JobDesc job = P.js.jobs[j];
    const uint64_t b0 = job.block_begin, b1 = b0 + job_blocks(job, P.js.block_shift);
    const uint64_t count = P.block_sum[b1] - P.block_sum[b0];
    *job.count_out = count;
    if (job.err_out && count > job.capacity) *job.err_out = kErrCapacity;
  }
}

// ---------------------------------------------------------------------------
// k_prep (batched calls): the internal job table, whose block offsets are an
// exclusive scan of the jobs' block counts, zeroed counts and errors, and the
// total block count.  A batch beyond the scratch (more bytes than the
// caller's bound) is turned into empty jobs that report FFP_E_CAPACITY.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kScanThreads) void k_prep(PrepParams P) {
  __shared__ uint64_t s_scan[kScanThreads / kWave];
  __shared__ uint64_t s_carry_blocks, s_carry_bytes;
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_carry_blocks = 0;
    s_carry_bytes = 0;
  }
  for (uint32_t base = 0; base < P.njobs; base += kScanThreads) {
    const uint32_t j = base + tid;
    UserJob u{};
    if (j < P.njobs) u = P.user[j];
    const bool ok = j < P.njobs && u.dtype >= kF64 && u.dtype <= kBF16 &&
                    u.nbytes < kMaxBytes && (u.nbytes == 0 || u.text != nullptr) &&
                    (u.capacity == 0 || (u.values != nullptr && u.status != nullptr));
    const uint64_t nb = ok ? u.nbytes : 0;
    const uint64_t vend = nb ? nb + ((uint64_t)(uintptr_t)u.text & 15u) : 0;
    const uint64_t blocks = (vend + (1ull << P.block_shift) - 1) >> P.block_shift;
    __syncthreads();  // carries of the previous round are final
    const uint64_t cb = s_carry_blocks, cbytes = s_carry_bytes;
    uint64_t tot_blocks, tot_bytes;
    const uint64_t ex_blocks = block_excl_scan<kScanThreads>(blocks, tot_blocks, s_scan);
    __syncthreads();
    (void)block_excl_scan<kScanThreads>(nb, tot_bytes, s_scan);
    if (j < P.njobs) {
      JobDesc d{};
      d.text = u.text;
      d.nbytes = nb;
      d.values = u.values;
      d.status = u.status;
      d.capacity = ok ? u.capacity : 0;
      d.count_out = &P.user[j].count;
      d.err_out = &P.user[j].err;
      d.block_begin = cb + ex_blocks;
      d.dtype = ok ? (uint32_t)u.dtype : kF64;
      d.job_id = j;
      P.jobs[j] = d;
      P.user[j].count = 0;
      P.user[j].err = ok ? 0 : kErrArg;
    }
    __syncthreads();
    if (tid == 0) {
      s_carry_blocks = cb + tot_blocks;
      s_carry_bytes = cbytes + tot_bytes;
    }
  }
  __syncthreads();
  const bool over = s_carry_blocks > P.block_cap || s_carry_bytes > P.max_bytes;
  if (tid == 0) P.st->total_blocks = over ? 0 : s_carry_blocks;
  if (over) {
    for (uint32_t j = tid; j < P.njobs; j += kScanThreads) {
      P.jobs[j].nbytes = 0;
      P.jobs[j].block_begin = 0;
      P.user[j].err = kErrCapacity;
    }
  }
}

// Tokens of a job that start in its first `vbytes` virtual bytes (a multiple
// of the chunk size; virtual byte v is text[v - align]), counted by the
// threads of a workgroup (each returns its share): a start is a token byte
// whose predecessor is a delimiter or lies before the text.
template <bool kSingle>
__device__ uint64_t count_starts_before(const uint8_t* vbase, uint64_t align, uint64_t vend,
                                        uint64_t vbytes, const DelimSet& delim, uint32_t drep,
                                        const uint8_t* lut, int tid) {
  uint64_t n = 0;
  for (uint64_t c = (uint64_t)tid; c * kChunk < vbytes; c += kThreads) {
    const uint64_t off = c * kChunk;
    const uint4 v = load_chunk(vbase, off, align, vend, delim.byte);
    // the byte before the chunk: past the text's first byte for c > 0
    // (off - 1 >= 15 >= align) and before vbytes <= vend
    const uint32_t prev = c ? (lut[gload(vbase + off - 1)] ? 0u : 1u) : 0u;
    const uint32_t m = nondelim_mask16_any<kSingle>(v, drep, lut, delim);
    n += __popc(m & ~((m << 1) | prev) & 0xFFFFu);
  }
  return n;
}

// ---------------------------------------------------------------------------
// The exact fallback on one queued token (fb_decide), by one wavefront: the
// fallback kernel's work, and that of the parse workgroups of small calls.
// ---------------------------------------------------------------------------
constexpr int kFbThreads = 256;
constexpr int kFbWaves = kFbThreads / kWave;

template <class F>
__device__ __forceinline__ void fallback_token(const JobDesc& job, uint64_t pos, uint64_t idx,
                                               FbLds* lds, const FallbackParams& P) {
  typename F::bits_t bits;
  uint32_t status;
  fb_decide<F>(job.text, job.nbytes, pos, g_table, g_pow5, lds, P.flags, bits, status);
  if (fb_lane() == 0) {
    gstore(reinterpret_cast<typename F::bits_t*>(job.values) + idx, bits);
    gstore(job.status + idx, (uint8_t)status);
    uint64_t key;
    const bool in = (P.reduce_out || P.sum_out) && order_key(bits, status, job.dtype, key);
    if (in && P.reduce_out) {
      atomicMin(&P.st->red_min, (unsigned long long)key);
      atomicMax(&P.st->red_max, (unsigned long long)key);
      atomicAdd(&P.st->red_count, 1ull);
    }
    if (in && P.sum_out) {
      const SumTerm x = sum_term(bits, job.dtype);
      if (!x.inf && x.m) sum_add(&P.st->sum_acc[x.neg ? 1 : 0][0], x);
      atomicOr(&P.st->sum_flags, sum_flag_bits(x));
    }
  }
}

// The nq queued tokens of one block of a plain call without a reduction,
// decided by the waves of the calling workgroup in turn (lds: one FbLds per
// wave).  Not inlined: the parse kernel calls it once per block at most, and
// as a call its registers do not add to those of the token loop.
__device__ __noinline__ void decide_queue_segment(const QueueEntry* seg, uint32_t nq,
                                                  const uint8_t* text, uint64_t nbytes,
                                                  void* values, uint8_t* status, uint32_t dtype,
                                                  uint32_t flags, FbLds* lds) {
  JobDesc job{};
  job.text = text;
  job.nbytes = nbytes;
  job.values = values;
  job.status = status;
  job.dtype = dtype;
  FallbackParams F{};
  F.flags = flags;
  const uint32_t wid = threadIdx.x / kWave;
  for (uint32_t i = wid; i < nq; i += kThreads / kWave) {
    const QueueEntry e = seg[i];
    const uint64_t idx = e.index_job & ((1ull << 48) - 1);
    fb_wave_sync();  // the previous token's LDS reads are done
    switch (dtype) {
      case kF64: fallback_token<F64>(job, e.offset, idx, lds + wid, F); break;
      case kF32: fallback_token<F32>(job, e.offset, idx, lds + wid, F); break;
      case kF16: fallback_token<F16>(job, e.offset, idx, lds + wid, F); break;
      default: fallback_token<BF16>(job, e.offset, idx, lds + wid, F); break;
    }
  }
}

// ---------------------------------------------------------------------------
// k_parse (the tile layout and the lexers are in ffp_lexer.h)
// ---------------------------------------------------------------------------

// Algorithm 1 (and w+1 for long significands) on a lexed token, the queue
// append for undecided tokens, and the stores.  Returns the path counter.
// kLocalFb (with ParseParams::fb_local set): the token goes to the block's
// own queue segment, at seg_base plus the workgroup's LDS counter *local_n.
template <class F, bool kExt, bool kLocalFb>
__device__ __forceinline__ int finish_token(const Lexed& L, uint64_t text_pos, const JobDesc& job,
                                            uint64_t first_idx, uint32_t j,
                                            const unsigned long long* table,
                                            const TableEntry* ent,
                                            const ParseParams& P, uint32_t* local_n,
                                            uint64_t seg_base, uint64_t& bits_out,
                                            uint32_t& status_out) {
  Decision<F> d = decide_lexed<F, kExt>(L, table, P.flags, ent);
  bits_out = d.bits;
  status_out = d.fallback ? kPending : d.status;
  uint8_t st = (uint8_t)d.status;
  if (d.fallback) {
    const unsigned long long slot = kLocalFb && P.fb_local
                                        ? seg_base + atomicAdd(local_n, 1u)
                                        : atomicAdd(&P.st->queue_tail, 1ull);
    if (slot < P.queue_cap) {
      QueueEntry e;
      e.offset = text_pos;
      e.index_job = (first_idx + j) | ((uint64_t)job.job_id << 48);
      P.queue[slot] = e;
    } else {
      atomicOr(&P.st->error, (unsigned)kDevQueue);
      if (job.err_out) *job.err_out = kErrQueue;
    }
    st = kPending;
  }
  const uint64_t idx = first_idx + j;
  gstore(reinterpret_cast<typename F::bits_t*>(job.values) + idx, d.bits);
  gstore(job.status + idx, st);
  return (int)d.path;
}

// Registers: within 128 (four waves per SIMD), and within 96 for the plain
// instance without a reduction (five waves per SIMD; at 96 the other
// instances spill to scratch inside the token loop).  Five 16 KiB-tile
// workgroups fit a CU's LDS with the shorter start list of that instance.
// kReduce: the call also keeps the minimum, maximum and count of the
// values.  kMode: kModePlain lexes Section 4's grammar (FFP_REJECT_PLUS
// aside, no grammar flag); kModeGrammar adds the JSON grammar and inf / nan
// (FFP_JSON, FFP_INFNAN); kModeExt adds hexadecimal tokens (FFP_HEX) and the
// directed rounding modes.  Separate instances, so that the plain parse pays
// nothing for either: its register and branch budget is the tightest.
template <int K, bool kSingle, bool kReduce, int kMode>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(kMode == kModePlain && !kReduce ? 5 : 4))) void
k_parse(ParseParams P) {
  constexpr bool kExt = kMode == kModeExt;
  constexpr bool kGrammar = kMode != kModePlain && kMode != kModePlainDense;
  using S = TileSmem<K>;
  using Packed = typename S::Packed;
  __shared__ S sm;
  // the exact sum's accumulators of this workgroup (reduction instances)
  __shared__ unsigned long long s_sum[kReduce ? 2 * kSumLimbs : 1];
  // CSV: the column scans' wave totals
  constexpr bool csv = kMode == kModeCsv;
  __shared__ uint32_t s_seg[csv ? kThreads / kWave : 1];
  // Token starts of a tile (offsets in the tile), in token order.  A tile
  // can hold kBytes / 2 tokens; the plain 16 KiB instance without a
  // reduction keeps a list half that long (its LDS then lets five workgroups
  // share a CU).  It runs when no block of the call has more starts than
  // that (the scan kernel's DeviceState::dense), its twin kModePlainDense
  // with the full list otherwise: both are launched, and the one not
  // needed returns at once.  The JSON document instance also keeps its
  // token bitmaps here until the starts are written.
  constexpr bool kShortStarts = K == 4 && kMode == kModePlain && !kReduce;
  constexpr int kStartsCap = kShortStarts ? S::kBytes / 4 : S::kBytes / 2;
  static_assert(!kShortStarts || kStartsCap == (int)kShortTileStarts, "short start list");
  __shared__ uint16_t s_starts[kStartsCap];
  if (kShortStarts && P.st->dense) return;
  if (kMode == kModePlainDense && !P.st->dense) return;
  __shared__ uint32_t s_sum_flags;
  // Small calls: the block's queued tokens, decided by this workgroup after
  // the block's tile (ParseParams::fb_local).  The fallback's per-wave LDS
  // then lives in the tile's text array, unused until the next tile.
  constexpr bool kLocalFb = K == 1 && !kReduce &&
                            (kMode == kModePlain || kMode == kModeGrammar || kMode == kModeExt);
  __shared__ uint32_t s_fb_n;
  static_assert(!kLocalFb || sizeof(FbLds) * (kThreads / kWave) <= sizeof(sm.text),
                "the fallback's LDS fits the tile text");
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);

  // The power-of-five table is read from the code object's global copy
  // through the L1/L2 caches: keeping its 10,416 bytes out of LDS lets four
  // workgroups share a CU instead of three (13% faster than a per-workgroup
  // LDS copy when measured).
  const unsigned long long* table = g_table;
  for (int i = tid; i < 256; i += kThreads) sm.delim_lut[i] = is_delim(P.delim, (uint32_t)i);
  if (tid < 20) {
    unsigned long long p = 1;
    for (int i = 0; i < tid; ++i) p *= 10;
    sm.pow10[tid] = p;
  }
  if (tid < 16) sm.keep8[tid] = tid >= 8 ? 0ull : (~0ull << (8 * tid)) & 0x0F0F0F0F0F0F0F0Full;
  if (tid < S::kExtChunks + 8) {
    sm.nd[S::kChunks + tid] = 0;
    sm.dg[S::kChunks + tid] = 0;
  }
  if (tid == 0) {
    sm.red_min = kNoMin;
    sm.red_max = kNoMax;
    sm.red_count = 0;
    s_sum_flags = 0;
    s_fb_n = 0;
  }
  if (kReduce)
    for (int i = tid; i < 2 * kSumLimbs; i += kThreads) s_sum[i] = 0;
  const uint32_t drep = P.delim.byte * 0x01010101u;
  const uint64_t nblk = total_blocks_of(P.js);
  // tiles per block (the host keeps blocks at least one tile long)
  const int ntiles = (int)((1u << P.js.block_shift) / S::kBytes);
  // path counters, kept in scalars (a runtime-indexed array would live in
  // scratch memory)
  uint32_t c_tok = 0, c_inv = 0, c_early = 0, c_one = 0, c_two = 0, c_fb = 0;
  // reduction instances: this lane's minimum and maximum order keys and
  // count of the values it decided (wave reductions once, at the end, instead
  // of three per round)
  uint64_t r_min = kNoMin, r_max = kNoMax;
  uint32_t r_cnt = 0;

  for (uint64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const JobDesc job = job_of_block(P.js, blk);
    // Tiles cover the job's text as if it started at the 16-byte boundary
    // below `text`: virtual byte v is text[v - align].
    const uint64_t align = (uint64_t)(uintptr_t)job.text & 15u;
    const uint8_t* vbase = job.text - align;
    const uint64_t nbytes = job.nbytes;
    const uint64_t vend = nbytes + align;
    const uint64_t bstart = (blk - job.block_begin) << P.js.block_shift;
    uint64_t next_idx;
    if (K == 1 && (P.sum_in_parse || P.self_count)) {  // small calls: 4 KiB blocks, one tile each
      // the counts of this job's earlier blocks, summed by the workgroup, or
      // (self_count) the tokens before the block, counted from the text
      uint64_t part = 0;
      if (P.self_count) {
        if (blk == 0 && tid == 0) reset_spare_state(P.other_st);
        __syncthreads();  // the delimiter table is written
        part = count_starts_before<kSingle>(vbase, align, vend, bstart, P.delim,
                                            P.delim.byte * 0x01010101u, sm.delim_lut, tid);
      } else {
        for (uint64_t i = job.block_begin + tid; i < blk; i += kThreads) part += P.block_prefix[i];
      }
      part = wave_sum_u64(part);
      __syncthreads();  // sm.red_part of the previous block is consumed
      if (lane == 0) sm.red_part[tid / kWave] = part;
      __syncthreads();
      next_idx = 0;
#pragma unroll
      for (int w = 0; w < kThreads / kWave; ++w) next_idx += sm.red_part[w];
      if (!P.self_count && tid == 0 &&
          blk + 1 == job.block_begin + job_blocks(job, P.js.block_shift)) {
        // the job's last block: its token count and the capacity check
        const uint64_t count = next_idx + P.block_prefix[blk];
        *job.count_out = count;
        // a queue overflow reported by another workgroup takes precedence
        if (job.err_out && count > job.capacity) atomicCAS(job.err_out, 0, kErrCapacity);
      }
    } else {
      next_idx = (P.block_prefix[blk] & kPrefixMask) - (P.block_prefix[job.block_begin] & kPrefixMask);
    }
    // JSON documents: whether the block begins inside a string
    constexpr bool doc = kMode == kModeDoc;
    const uint32_t block_entry = doc ? (uint32_t)(P.block_prefix[blk] >> 63) : 0u;
    const GlobalSrc gsrc{job.text, nbytes, P.delim};

    // A tile's chunks are loaded at the top of its iteration; the other
    // workgroups on the CU hide the latency.  (Loading the next tile into
    // registers during the token rounds held 4K registers through them and
    // measured no faster.)
    uint4 pre[K];
    // the byte before the block, loaded with the block's first chunks
    const uint32_t block_prev =
        tid != 0 ? 0u
        : doc    ? doc_prev_token(job.text, (int64_t)bstart - (int64_t)align, block_entry, P.delim)
                 : prev_nondelim(vbase, bstart, align, P.delim);
    // CSV: the column at the block's start (then carried from tile to tile;
    // the same value in every thread)
    uint32_t csv_col = 0;
    if (csv) {
      __syncthreads();  // s_seg of the previous block is consumed
      csv_col = csv_entry_column(vbase, align, vend, bstart, s_seg);
    }
    for (int t = 0; t < ntiles; ++t) {
      const uint64_t tile_start = bstart + (uint64_t)t * S::kBytes;  // virtual
      if (tile_start >= vend) break;
      if (tile_start >= align && tile_start + S::kBytes <= vend) {  // the same for every lane
        // the whole tile lies inside the text: plain 16-byte loads
        const uint8_t* tp = vbase + tile_start + (uint32_t)tid * kChunk;
#pragma unroll
        for (int c = 0; c < K; ++c) {
          const u32x4 v = gload(reinterpret_cast<const u32x4*>(tp + c * kThreads * kChunk));
          pre[c] = make_uint4(v.x, v.y, v.z, v.w);
        }
      } else {
#pragma unroll
        for (int c = 0; c < K; ++c)
          pre[c] = load_chunk(vbase, tile_start + (uint64_t)(c * kThreads + tid) * kChunk, align,
                              vend, P.delim.byte);
      }
      __syncthreads();  // LDS of the previous tile is consumed
      // -- store the tile to LDS and classify bytes ---------------------
      uint32_t ndm[K], dgm[K];
      CsvBits cb[csv ? K : 1];
      // (JSON documents: ten delimiters, always the table)
      const bool few = !kSingle && !doc && P.delim.nfew != 0;
#pragma unroll
      for (int c = 0; c < K; ++c) {
        const int chunk = c * kThreads + tid;
        const uint4 v = pre[c];
        *reinterpret_cast<uint4*>(&sm.text[S::kPadFront + chunk * kChunk]) = v;
        ndm[c] = few ? nondelim_mask16<kSingle, true>(v, drep, sm.delim_lut, P.delim)
                     : nondelim_mask16<kSingle, false>(v, drep, sm.delim_lut, P.delim);
        sm.nd[chunk] = (uint16_t)ndm[c];
        dgm[c] = pack_high_bits(digit_word(v.x), digit_word(v.y), digit_word(v.z), digit_word(v.w));
        sm.dg[chunk] = (uint16_t)dgm[c];
        if (csv)
          cb[c] = csv_chunk(v, text_bits(tile_start + (uint64_t)chunk * kChunk, align, vend));
      }
      // CSV: the column at each chunk's first byte, row after row of the tile
      uint32_t csv_entry[csv ? K : 1];
      if (csv) {
#pragma unroll
        for (int c = 0; c < K; ++c) {
          uint32_t row;
          const uint32_t ex = block_excl_segscan(csv_seg(cb[c]), row, s_seg);
          csv_entry[c] = (ex & kSegNl) ? (ex & ~kSegNl) : csv_col + ex;
          csv_col = (row & kSegNl) ? (row & ~kSegNl) : csv_col + row;
          __syncthreads();  // s_seg is read before the next row writes it
        }
      }
      // JSON documents: token bytes are the non-delimiters outside strings;
      // the string state of each chunk comes from a block scan of its
      // unescaped quotes (s_starts holds the token bitmaps until the
      // token starts are written)
      uint32_t tbm[K], msm[K], tile_last_tb = 0, tile_end_str = 0;
      if (doc) {
        uint32_t uq[K];
        Packed pq = 0;
#pragma unroll
        for (int c = 0; c < K; ++c) {
          const int chunk = c * kThreads + tid;
          const DocBits d = doc_chunk(pre[c], dgm[c], job.text,
                                      (int64_t)(tile_start + (uint64_t)chunk * kChunk) - (int64_t)align);
          uq[c] = d.uq;
          tbm[c] = ndm[c] | d.eq;
          msm[c] = d.ms;
          pq |= (Packed)__popc(d.uq) << (16 * c);
        }
        Packed totq;
        const Packed exq = block_excl_scan<kThreads>(pq, totq, sm.scan);
        const uint32_t carry_in = t == 0 ? block_entry : sm.prev_str;
        uint32_t rowq = 0;
#pragma unroll
        for (int c = 0; c < K; ++c) {
          const int chunk = c * kThreads + tid;
          const uint32_t cin = (carry_in + rowq + ((uint32_t)(exq >> (16 * c)) & 0xFFFFu)) & 1u;
          tbm[c] &= ~doc_in_string(uq[c], cin);
          s_starts[chunk] = (uint16_t)tbm[c];
          rowq += (uint32_t)(totq >> (16 * c)) & 0xFFFFu;
        }
        tile_last_tb = (tbm[K - 1] >> 15) & 1u;
        tile_end_str = (carry_in + rowq) & 1u;
      }
      const uint64_t next_start = tile_start + S::kBytes;
      // wave 0 loads the extension (the 1 KiB after the tile: the next
      // tile's first chunks, or delimiters past the text), used if a token
      // runs past the tile
      uint4 ext_v = make_uint4(0, 0, 0, 0);
      if (tid < S::kExtChunks)
        ext_v = load_chunk(vbase, next_start + (uint64_t)tid * kChunk, align, vend, P.delim.byte);
      if (tid == 0 && t == 0) sm.prev_nd = block_prev;
      __syncthreads();

      // -- token starts: non-delimiter byte after a delimiter -----------
      uint32_t startm[K];
      Packed packed = 0;
#pragma unroll
      for (int c = 0; c < K; ++c) {
        const int chunk = c * kThreads + tid;
        const uint32_t prevbit =
            chunk == 0 ? sm.prev_nd
            : doc      ? ((uint32_t)s_starts[chunk - 1] >> 15) & 1u
                       : ((uint32_t)sm.nd[chunk - 1] >> 15) & 1u;
        const uint32_t m = doc ? tbm[c] : ndm[c];
        startm[c] = m & ~((m << 1) | prevbit) & 0xFFFFu;
        if (doc) startm[c] &= msm[c];  // numbers start with '-' or a digit
        if (csv) startm[c] = csv_select(startm[c], cb[c], csv_entry[c], P.csv_columns);
        packed |= (Packed)__popc(startm[c]) << (16 * c);
      }
      Packed total_packed;
      const Packed excl_packed = block_excl_scan<kThreads>(packed, total_packed, sm.scan);
      uint32_t row_off[K];
      uint32_t ntok = 0;
#pragma unroll
      for (int c = 0; c < K; ++c) {
        row_off[c] = ntok;
        ntok += (uint32_t)(total_packed >> (16 * c)) & 0xFFFFu;
      }
      if (K == 1 && P.self_count && tid == 0 &&
          blk + 1 == job.block_begin + job_blocks(job, P.js.block_shift)) {
        // the job's last block (one tile): its token count and the capacity check
        const uint64_t count = next_idx + ntok;
        *job.count_out = count;
        if (job.err_out && count > job.capacity) atomicCAS(job.err_out, 0, kErrCapacity);
      }
      const bool straddle = (sm.nd[S::kChunks - 1] >> 15) & 1u;
      const LdsSrc lsrc{sm.text + S::kPadFront, tile_start, sm.delim_lut};
      // tokens of this tile that fit the caller's capacity
      const uint32_t nfit = next_idx >= job.capacity ? 0u
                            : (job.capacity - next_idx < ntok ? (uint32_t)(job.capacity - next_idx)
                                                              : ntok);
#pragma unroll
      for (int c = 0; c < K; ++c) {
        uint32_t p = row_off[c] + ((uint32_t)(excl_packed >> (16 * c)) & 0xFFFFu);
        uint32_t m = startm[c];
        const uint32_t base = (uint32_t)((c * kThreads + tid) * kChunk);
        while (m) {
          const uint32_t k = __ffs(m) - 1;
          s_starts[p++] = (uint16_t)(base + k);
          m &= m - 1;
        }
      }
      // -- one lane per token -------------------------------------------
      // When the tile's last byte belongs to a token, that token (the last
      // one starting here) continues past the tile: the extension is filled
      // before the rounds (no other token reads it); if the token also runs
      // past the extension it is read from global memory, which returns a
      // delimiter past the text.
      if (straddle && nfit == ntok) {  // the last token is decided here: fill the extension
        if (tid < S::kExtChunks) {  // wave 0: chunk tid of the next tile
          const uint4 v = ext_v;
          *reinterpret_cast<uint4*>(&sm.text[S::kPadFront + S::kBytes + tid * kChunk]) = v;
          const uint32_t m = nondelim_mask16_any<kSingle>(v, drep, sm.delim_lut, P.delim);
          sm.nd[S::kChunks + tid] = (uint16_t)m;
          sm.dg[S::kChunks + tid] = (uint16_t)pack_high_bits(digit_word(v.x), digit_word(v.y),
                                                             digit_word(v.z), digit_word(v.w));
          const uint64_t has_delim = (uint64_t)__ballot(m != 0xFFFFu);
          if (tid == 0) sm.ext_end = has_delim != 0;
        }
      }
      __syncthreads();
      // the token read from global memory, if any (index; ~0: none)
      const uint32_t global_j = straddle && nfit == ntok && !sm.ext_end ? ntok - 1 : ~0u;
      // whole rounds of 256 tokens: lanes without a token in the last round
      // stay in step, so the reduction below sees every lane
      for (uint32_t round = 0; round < nfit; round += kThreads) {
        const uint32_t j = round + tid;
        const bool has_token = j < nfit;
        uint64_t vbits = 0;
        uint32_t vstatus = kStInvalid;
        if (has_token) {
          const uint32_t s = s_starts[j];
          const uint64_t vpos = tile_start + s;  // virtual
          const uint64_t pos = vpos - align;     // offset in the text
          const bool global = j == global_j;
          FastLex fl;
          if (!global) {
            fl = fast_lex<K, kGrammar>(sm, s, P.flags, table);
          } else {
            fl.code = kFastSlow;
          }
          Lexed L;
          TableEntry ent;  // the table entry for L.q (read by the fast lexer)
          if (fl.code == kFastSlow) {
            if (global)
              L = lex_token<kExt>(gsrc, pos, P.flags);
            else if (kGrammar && (P.flags & (kFlagJson | kFlagInfNan | kFlagHex)))
              L = lex_token<kExt>(lsrc, vpos, P.flags);
            else
              L = long_lex<K>(sm, s, P.flags);
            ent = table_entry(table, L.q);
          } else {
            L.w = fl.w;
            L.q = fl.q;
            L.neg = fl.neg;
            L.kind = fl.code == kFastInvalid ? kLexInvalid : kLexExact;
            ent = fl.ent;
          }
          int path;
          switch (job.dtype) {
            case kF64: path = finish_token<F64, kExt, kLocalFb>(L, pos, job, next_idx, j, table, &ent, P, &s_fb_n, blk * kLocalQueueSeg, vbits, vstatus); break;
            case kF32: path = finish_token<F32, kExt, kLocalFb>(L, pos, job, next_idx, j, table, &ent, P, &s_fb_n, blk * kLocalQueueSeg, vbits, vstatus); break;
            case kF16: path = finish_token<F16, kExt, kLocalFb>(L, pos, job, next_idx, j, table, &ent, P, &s_fb_n, blk * kLocalQueueSeg, vbits, vstatus); break;
            default: path = finish_token<BF16, kExt, kLocalFb>(L, pos, job, next_idx, j, table, &ent, P, &s_fb_n, blk * kLocalQueueSeg, vbits, vstatus); break;
          }
          if (P.count_paths) {
            c_tok += 1;
            c_inv += path == kCntInvalid;
            c_early += path == kCntEarly;
            c_one += path == kCntOne;
            c_two += path == kCntTwo;
            c_fb += path == kCntFallback;
          }
        }
        if (kReduce) {
          uint64_t key = 0;
          const bool in = has_token && order_key(vbits, vstatus, job.dtype, key);
          if (in) {  // this lane's running minimum, maximum and count
            r_min = key < r_min ? key : r_min;
            r_max = key > r_max ? key : r_max;
            ++r_cnt;
          }
          if (P.sum_out) {  // the same values, into the exact sum
            const SumTerm x = sum_term(vbits, job.dtype);
            if (in && !x.inf && x.m) sum_add(s_sum + (x.neg ? kSumLimbs : 0), x);
            const uint32_t f = in ? sum_flag_bits(x) : 0u;
            uint32_t fw = 0;
#pragma unroll
            for (uint32_t bit = 1; bit <= kSumAny; bit <<= 1)
              if (__ballot((f & bit) != 0)) fw |= bit;
            if (lane == 0 && fw) atomicOr(&s_sum_flags, fw);
          }
        }
      }
      next_idx += ntok;
      if (doc) {
        if (tid == kThreads - 1) {  // the thread of the tile's last chunk
          sm.prev_nd = tile_last_tb;
          sm.prev_str = tile_end_str;
        }
      } else if (tid == 0) {
        sm.prev_nd = (sm.nd[S::kChunks - 1] >> 15) & 1u;
      }
    }
    if (kLocalFb && P.fb_local) {
      // the block's queued tokens, one wave each (as in k_fallback)
      __syncthreads();  // the block's queue entries and s_fb_n are written
      const uint32_t nq = s_fb_n;
      if (nq) {
        decide_queue_segment(P.queue + blk * kLocalQueueSeg, nq, job.text, job.nbytes, job.values, job.status,
                             job.dtype, P.flags, reinterpret_cast<FbLds*>(sm.text));
        __syncthreads();  // s_fb_n is read and the tile's LDS is free again
        if (tid == 0) s_fb_n = 0;
      }
    }
    if (kReduce && P.sum_out) {
      // the block's sum into the call's accumulators: each word (below
      // 2^47 after a block of at most 2^15 tokens) as two 32-bit pieces
      __syncthreads();
      for (int i = tid; i < 2 * kSumLimbs; i += kThreads) {
        const unsigned long long v = s_sum[i];
        if (v) {
          s_sum[i] = 0;
          unsigned long long* g = &P.st->sum_acc[0][0] + i;
          atomicAdd(g, v & 0xFFFFFFFFull);
          if (v >> 32) atomicAdd(g + 1, v >> 32);
        }
      }
      if (tid == 0 && s_sum_flags) {
        atomicOr(&P.st->sum_flags, s_sum_flags);
        s_sum_flags = 0;
      }
    }
  }

  if (kReduce) {
    // the lanes' running values, reduced once per workgroup
    const uint64_t kmin = wave_min_u64(r_min);
    const uint64_t kmax = wave_max_u64(r_max);
    const uint64_t cnt = wave_sum_u64(r_cnt);
    if (lane == 0 && cnt) {
      atomicMin(&sm.red_min, (unsigned long long)kmin);
      atomicMax(&sm.red_max, (unsigned long long)kmax);
      atomicAdd(&sm.red_count, (unsigned long long)cnt);
    }
    __syncthreads();
    if (tid == 0 && sm.red_count) {
      atomicMin(&P.st->red_min, sm.red_min);
      atomicMax(&P.st->red_max, sm.red_max);
      atomicAdd(&P.st->red_count, sm.red_count);
    }
  }
  if (P.count_paths) {
    const uint32_t cnt[kNumCounters] = {c_tok, c_inv, c_early, c_one, c_two, c_fb};
#pragma unroll
    for (int i = 0; i < kNumCounters; ++i) {
      const uint64_t s = wave_sum_u64(cnt[i]);
      if (lane == 0 && s) atomicAdd(&P.st->counters[i], (unsigned long long)s);
    }
  }
}

// ---------------------------------------------------------------------------
// k_fallback: one wavefront per queued token (fb_decide), wavefronts striding
// over the queue.
// ---------------------------------------------------------------------------
// Compiled for six waves per SIMD (80 registers): a token's decision is a
// chain of dependent cross-lane steps and memory reads, so more resident
// wavefronts beat fewer, wider ones (config 3: 4.88 ms per call at four
// waves per SIMD, 4.67 at six, 4.77 at eight).
__global__ __launch_bounds__(kFbThreads) __attribute__((amdgpu_waves_per_eu(6))) void
k_fallback(FallbackParams P) {
  __shared__ FbLds lds[kFbWaves];
  const unsigned long long tail = P.st->queue_tail;
  const uint64_t n = tail < P.queue_cap ? tail : P.queue_cap;
  const int wid = threadIdx.x / kWave;
  const uint64_t stride = (uint64_t)gridDim.x * kFbWaves;
  for (uint64_t i = (uint64_t)blockIdx.x * kFbWaves + wid; i < n; i += stride) {
    const QueueEntry e = P.queue[i];
    const uint32_t job_id = (uint32_t)(e.index_job >> 48);
    const uint64_t idx = e.index_job & ((1ull << 48) - 1);
    const JobDesc job = P.js.jobs ? P.js.jobs[job_id] : P.js.single;
    fb_wave_sync();  // the previous token's LDS reads are done
    switch (job.dtype) {
      case kF64: fallback_token<F64>(job, e.offset, idx, &lds[wid], P); break;
      case kF32: fallback_token<F32>(job, e.offset, idx, &lds[wid], P); break;
      case kF16: fallback_token<F16>(job, e.offset, idx, &lds[wid], P); break;
      default: fallback_token<BF16>(job, e.offset, idx, &lds[wid], P); break;
    }
  }
}

// ---------------------------------------------------------------------------
// k_reduce_final (plain calls with a reduction): one thread turns the
// call's minimum / maximum keys and count into the caller's three words.
// A kernel of its own: the kernel boundary orders it after every update of
// the parse and fallback kernels (a last-workgroup test inside the fallback
// kernel would need a device-scope fence in every workgroup, which writes
// back the XCD's L2 each time).
// ---------------------------------------------------------------------------
// The exact sum, rounded once to binary64 (nearest, ties to even): the
// accumulators' carries resolved into 32-bit limbs, the smaller magnitude
// subtracted from the larger, the leading 53 bits kept with a guard bit and
// a sticky bit below them.  out[0]: the encoding, out[1]: 1 if the sum is
// exactly representable.  One thread.
__device__ void sum_final(DeviceState* st, uint64_t* out) {
  __shared__ uint32_t mag[2][kSumLimbs];
  for (int side = 0; side < 2; ++side) {
    unsigned long long carry = 0;
    for (int i = 0; i < kSumLimbs; ++i) {
      const unsigned long long t = st->sum_acc[side][i] + carry;
      mag[side][i] = (uint32_t)t;
      carry = t >> 32;
    }
  }
  const uint32_t flags = st->sum_flags;
  uint64_t bits;
  bool exact = true;
  if ((flags & kSumPosInf) && (flags & kSumNegInf)) {
    bits = F64::kQNaN;
    exact = false;
  } else if (flags & (kSumPosInf | kSumNegInf)) {
    bits = F64::kInf | ((flags & kSumNegInf) ? F64::kSign : 0ull);
  } else {
    // sign of the difference: the first limb from the top that differs
    int cmp = 0;
    for (int i = kSumLimbs - 1; i >= 0 && cmp == 0; --i)
      cmp = mag[0][i] > mag[1][i] ? 1 : (mag[0][i] < mag[1][i] ? -1 : 0);
    const int big = cmp >= 0 ? 0 : 1;
    __shared__ uint32_t d[kSumLimbs];
    int64_t borrow = 0;
    int top = -1;  // index of the highest nonzero limb of |difference|
    for (int i = 0; i < kSumLimbs; ++i) {
      const int64_t t = (int64_t)mag[big][i] - (int64_t)mag[1 - big][i] - borrow;
      borrow = t < 0;
      d[i] = (uint32_t)(t + (borrow << 32));
      if (d[i]) top = i;
    }
    const uint64_t sign = big ? F64::kSign : 0ull;
    if (top < 0) {
      // an exact zero: -0 only when every summed value was -0
      bits = ((flags & kSumAny) && !(flags & kSumNotNegZero)) ? F64::kSign : 0ull;
    } else {
      const int t = top * 32 + 31 - __builtin_clz(d[top]);  // leading bit
      if (t <= 52) {
        // below 2^53 units of 2^-1074: the encoding is the integer itself
        bits = sign | ((uint64_t)d[1] << 32 | d[0]);
      } else {
        // bits [t-52, t] of d, then the guard bit t-53 and the sticky rest
        auto bit_at = [&](int i) -> uint64_t { return (d[i >> 5] >> (i & 31)) & 1u; };
        uint64_t m = 0;
        for (int i = t; i >= t - 52; --i) m = (m << 1) | bit_at(i);
        const uint64_t guard = t >= 53 ? bit_at(t - 53) : 0u;
        bool sticky = false;
        for (int i = 0; i < t - 53 && !sticky; ++i) sticky = bit_at(i) != 0;
        exact = !guard && !sticky;
        int e = t;
        if (guard && (sticky || (m & 1))) {
          if (++m == (1ull << 53)) {
            m >>= 1;
            ++e;
          }
        }
        const int field = e - 51;  // 2^t units of 2^-1074 is 2^(t-1074)
        if (field >= 2047) {
          bits = sign | F64::kInf;
          exact = false;
        } else {
          bits = sign | ((uint64_t)field << 52) | (m & ((1ull << 52) - 1));
        }
      }
    }
  }
  gstore(out + 0, bits);
  gstore(out + 1, (uint64_t)(exact ? 1u : 0u));
}

__global__ void k_reduce_final(FallbackParams P) {
  if (threadIdx.x != 0) return;
  if (P.sum_out) sum_final(P.st, P.sum_out);
  if (!P.reduce_out) return;
  const unsigned long long kmin = P.st->red_min;
  const unsigned long long kmax = P.st->red_max;
  const unsigned long long cnt = P.st->red_count;
  const uint32_t dt = P.js.single.dtype;
  const uint64_t nan = dt == kF64 ? F64::kQNaN : dt == kF32 ? F32::kQNaN
                       : dt == kF16 ? F16::kQNaN : BF16::kQNaN;
  gstore(P.reduce_out + 0, cnt ? key_to_bits(kmin, dt) : nan);
  gstore(P.reduce_out + 1, cnt ? key_to_bits(kmax, dt) : nan);
  gstore(P.reduce_out + 2, (uint64_t)cnt);
}

// ---------------------------------------------------------------------------
// Scratch of the entry point that allocates nothing: device state, per-block
// counts and the fallback queue at fixed offsets (ffp_internal.h).  Each GPU
// holds its own copy of the array for the life of the process; host code
// never passes the array's name to a kernel, only the device address
// returned for it below.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(int device, void** ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[device]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != device) return hipErrorInvalidDevice;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[device] = p;
  }
  *ptr = addr[device];
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
int parse_tile_bytes(int k) { return kThreads * kChunk * k; }

template <int K, bool kSingle>
static hipError_t occ_ks(bool wide, int* blocks) {
  return wide ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    blocks, k_parse<K, kSingle, true, kModeExt>, kThreads, 0)
              : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    blocks, k_parse<K, kSingle, false, kModePlain>, kThreads, 0);
}

template <int K>
static hipError_t occ_k(bool single, bool wide, int* blocks) {
  return single ? occ_ks<K, true>(wide, blocks) : occ_ks<K, false>(wide, blocks);
}

hipError_t parse_occupancy(int k, bool single_delim, bool wide, int* blocks_per_cu) {
  switch (k) {
    case 1: return occ_k<1>(single_delim, wide, blocks_per_cu);
    case 2: return occ_k<2>(single_delim, wide, blocks_per_cu);
    case 4: return occ_k<4>(single_delim, wide, blocks_per_cu);
    default: return hipErrorInvalidValue;
  }
}

template <int kRows>
static void launch_count_rows(bool single_delim, const CountParams& P, int grid, hipStream_t s) {
  if (single_delim)
    hipLaunchKernelGGL((k_count<true, kRows>), dim3(grid), dim3(kThreads), 0, s, P);
  else
    hipLaunchKernelGGL((k_count<false, kRows>), dim3(grid), dim3(kThreads), 0, s, P);
}

hipError_t launch_count(bool single_delim, const CountParams& P, int grid, hipStream_t s) {
  switch (P.js.block_shift) {
    case 12: launch_count_rows<1>(single_delim, P, grid, s); break;
    case 14: launch_count_rows<4>(single_delim, P, grid, s); break;
    case 16: launch_count_rows<16>(single_delim, P, grid, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_prep(const PrepParams& P, hipStream_t s) {
  hipLaunchKernelGGL(k_prep, dim3(1), dim3(kScanThreads), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_scan(const ScanParams& P, hipStream_t s) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, s, P);
  return hipGetLastError();
}

template <int K, bool kSingle, bool kReduce>
static void launch_parse_mode(const ParseParams& P, int grid, hipStream_t s) {
  if constexpr (!kSingle) {  // JSON documents and CSV: delimiter sets of many bytes
    if (P.flags & kFlagJsonDoc) {
      hipLaunchKernelGGL((k_parse<K, kSingle, kReduce, kModeDoc>), dim3(grid), dim3(kThreads), 0,
                         s, P);
      return;
    }
    if (P.flags & kFlagCsv) {
      hipLaunchKernelGGL((k_parse<K, kSingle, kReduce, kModeCsv>), dim3(grid), dim3(kThreads), 0,
                         s, P);
      return;
    }
  }
  if (P.flags & (kFlagHex | kFlagRoundMask))
    hipLaunchKernelGGL((k_parse<K, kSingle, kReduce, kModeExt>), dim3(grid), dim3(kThreads), 0, s, P);
  else if (P.flags & (kFlagJson | kFlagInfNan))
    hipLaunchKernelGGL((k_parse<K, kSingle, kReduce, kModeGrammar>), dim3(grid), dim3(kThreads), 0, s,
                       P);
  else {
    hipLaunchKernelGGL((k_parse<K, kSingle, kReduce, kModePlain>), dim3(grid), dim3(kThreads), 0, s,
                       P);
    // the full-list twin for dense calls: its LDS admits four workgroups
    // per CU where the plain instance has five, so it gets four fifths of
    // the grid (one dispatch wave; its block loop strides by the grid)
    if constexpr (K == 4 && !kReduce)
      hipLaunchKernelGGL((k_parse<K, kSingle, kReduce, kModePlainDense>),
                         dim3(grid > 4 ? grid - grid / 5 : grid), dim3(kThreads), 0, s, P);
  }
}

template <int K, bool kSingle>
static hipError_t launch_parse_k(const ParseParams& P, int grid, hipStream_t s) {
  if (P.reduce_out || P.sum_out)
    launch_parse_mode<K, kSingle, true>(P, grid, s);
  else
    launch_parse_mode<K, kSingle, false>(P, grid, s);
  return hipGetLastError();
}

hipError_t launch_parse(int k, bool single_delim, const ParseParams& P, int grid, hipStream_t s) {
  switch (k) {
    case 1: return single_delim ? launch_parse_k<1, true>(P, grid, s) : launch_parse_k<1, false>(P, grid, s);
    case 2: return single_delim ? launch_parse_k<2, true>(P, grid, s) : launch_parse_k<2, false>(P, grid, s);
    case 4: return single_delim ? launch_parse_k<4, true>(P, grid, s) : launch_parse_k<4, false>(P, grid, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fallback(const FallbackParams& P, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_fallback, dim3(grid), dim3(kFbThreads), 0, s, P);
  return launch_reduce_final(P, s);
}

hipError_t launch_reduce_final(const FallbackParams& P, hipStream_t s) {
  if (P.reduce_out || P.sum_out)
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kWave), 0, s, P);
  return hipGetLastError();
}

}  // namespace ffp
