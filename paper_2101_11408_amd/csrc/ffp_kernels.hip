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
#include "ffp_table.inc"

namespace ffp {

alignas(16) __device__ const unsigned long long g_table[FFP_TABLE_SIZE * 2] = {FFP_TABLE_ENTRIES};

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

// High bit of each byte of x set for non-delimiter bytes (a single
// delimiter byte below 0x80, replicated in drep) / for ASCII digits.  The
// low seven bits of each byte, after the xor, plus 0x7F (0x76) carry into
// the byte's high bit when they are nonzero (10 or more); x's own high bit
// marks the bytes at or above 0x80, which are neither the delimiter nor a
// digit.  Exact per byte (no carry crosses a byte); three VALU operations
// per word.
__device__ __forceinline__ uint32_t nondelim_word(uint32_t x, uint32_t drep) {
  const uint32_t t = ((x ^ drep) & 0x7F7F7F7Fu) + 0x7F7F7F7Fu;
  return (t | x) & 0x80808080u;
}

__device__ __forceinline__ uint32_t digit_word(uint32_t x) {
  const uint32_t t = ((x ^ 0x30303030u) & 0x7F7F7F7Fu) + 0x76767676u;
  return ~(t | x) & 0x80808080u;
}

__device__ __forceinline__ uint32_t nondelim_word_lut(uint32_t x, const uint8_t* lut) {
  uint32_t h = 0;
#pragma unroll
  for (int b = 0; b < 4; ++b) h |= (lut[(x >> (8 * b)) & 0xFF] ? 0u : 0x80u) << (8 * b);
  return h;
}

// Gather the high bits of the bytes of four words into a 16-bit mask: byte
// dot products with weights 1..128 put bytes 8..15 at bits 7..14 of `hi`;
// shifted up by 8 it is the accumulator of the same for bytes 0..7.
__device__ __forceinline__ uint32_t pack_high_bits(uint32_t h0, uint32_t h1, uint32_t h2,
                                                   uint32_t h3) {
  const uint32_t hi = __builtin_amdgcn_udot4(
      h3, 0x80402010u, __builtin_amdgcn_udot4(h2, 0x08040201u, 0u, false), false);
  const uint32_t all = __builtin_amdgcn_udot4(
      h1, 0x80402010u, __builtin_amdgcn_udot4(h0, 0x08040201u, hi << 8, false), false);
  return all >> 7;
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

template <bool kSingle>
__device__ __forceinline__ uint32_t nondelim_mask16(uint4 v, uint32_t drep, const uint8_t* lut) {
  if (kSingle)
    return pack_high_bits(nondelim_word(v.x, drep), nondelim_word(v.y, drep),
                          nondelim_word(v.z, drep), nondelim_word(v.w, drep));
  return pack_high_bits(nondelim_word_lut(v.x, lut), nondelim_word_lut(v.y, lut),
                        nondelim_word_lut(v.z, lut), nondelim_word_lut(v.w, lut));
}

// Is the byte just before virtual offset off a non-delimiter?
__device__ __forceinline__ uint32_t prev_nondelim(const uint8_t* vbase, uint64_t off,
                                                  uint64_t align, const DelimSet& d) {
  if (off <= align) return 0;  // start of the text
  return is_delim(d, gload(vbase + off - 1)) ? 0u : 1u;
}

// ---------------------------------------------------------------------------
// k_count: tokens starting in each block.  Each thread classifies kRows
// chunks of 16 bytes (kRows = block bytes / 4 KiB); the start mask of a chunk
// needs the last bit of the chunk before it, exchanged through LDS.
// ---------------------------------------------------------------------------
template <bool kSingle, int kRows>
__global__ __launch_bounds__(kThreads) void k_count(CountParams P) {
  constexpr int kCountRows = kRows;
  constexpr uint32_t kShift = kRows == 1 ? 12 : (kRows == 4 ? 14 : 16);
  __shared__ uint16_t s_nd[kCountRows * kThreads];
  __shared__ uint8_t s_lut[256];
  __shared__ uint32_t s_scan[kThreads / kWave];
  __shared__ uint32_t s_prev;
  const int tid = threadIdx.x;
  if (!kSingle)
    for (int i = tid; i < 256; i += kThreads) s_lut[i] = is_delim(P.delim, (uint32_t)i);
  const uint32_t drep = P.delim.byte * 0x01010101u;
  const uint64_t nblk = total_blocks_of(P.js);
  for (uint64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    const JobDesc job = job_of_block(P.js, b);
    const uint64_t align = (uint64_t)(uintptr_t)job.text & 15u;
    const uint8_t* vbase = job.text - align;
    const uint64_t vend = job.nbytes + align;
    const uint64_t bstart = (b - job.block_begin) << kShift;
    __syncthreads();  // s_nd / s_prev of the previous block are consumed
    uint32_t m[kCountRows];
#pragma unroll
    for (int r = 0; r < kCountRows; ++r) {
      const uint64_t off = bstart + (uint64_t)(r * kThreads + tid) * kChunk;
      m[r] = off < vend ? nondelim_mask16<kSingle>(
                              load_chunk(vbase, off, align, vend, P.delim.byte), drep, s_lut)
                        : 0u;
      s_nd[r * kThreads + tid] = (uint16_t)m[r];
    }
    if (tid == 0) s_prev = prev_nondelim(vbase, bstart, align, P.delim);
    __syncthreads();
    uint32_t n = 0;
#pragma unroll
    for (int r = 0; r < kCountRows; ++r) {
      const int chunk = r * kThreads + tid;
      const uint32_t pb = chunk == 0 ? s_prev : ((uint32_t)s_nd[chunk - 1] >> 15);
      n += __popc(m[r] & ~((m[r] << 1) | pb) & 0xFFFFu);
    }
    uint32_t total;
    (void)block_excl_scan<kThreads>(n, total, s_scan);
    if (tid == 0) P.block_sum[b] = total;
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
  if (tid == 0) {
    s_carry = 0;
    // the call's device state starts clean (the parse kernel appends to the
    // queue and raises error bits; the reduction starts from its identities)
    P.st->queue_tail = 0;
    P.st->error = 0;
    P.st->red_min = ~0ull;
    P.st->red_max = 0;
    P.st->red_count = 0;
  }
  for (uint64_t base = 0; base < n; base += (uint64_t)kScanThreads * kScanPer) {
    uint64_t v[kScanPer];
    uint64_t sum = 0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
      const uint64_t k = base + (uint64_t)tid * kScanPer + i;
      v[i] = k < n ? P.block_sum[k] : 0;
      sum += v[i];
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
      if (k < n) P.block_sum[k] = run;
      run += v[i];
    }
    __syncthreads();
    if (tid == 0) s_carry = carry + total;
  }
  __syncthreads();
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

// ---------------------------------------------------------------------------
// k_parse
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
  uint16_t starts[kBytes / 2];
  // bit i of these bitmaps describes byte i of the tile (16 bits per chunk),
  // then the extension, then 128 zero bits so that 32-bit windows stay in
  // range
  alignas(8) uint16_t nd[kChunks + kExtChunks + 8];  // not a delimiter
  alignas(8) uint16_t dg[kChunks + kExtChunks + 8];  // ASCII digit
  uint8_t delim_lut[256];
  Packed scan[kThreads / kWave];
  uint32_t prev_nd;
  uint32_t ext_end;  // the extension holds a delimiter
  unsigned long long red_min, red_max, red_count;  // this workgroup's reduction
};

struct LdsSrc {
  const uint8_t* text;  // LDS tile (first byte of the tile)
  uint64_t tile_start;
  const uint8_t* lut;   // LDS delimiter table
  __device__ __forceinline__ uint32_t operator()(uint64_t i) const {
    return text[i - tile_start];
  }
  __device__ __forceinline__ bool is_end(uint32_t c) const { return lut[c] != 0; }
};

// 32 bits of a tile bitmap starting at bit s (one funnel shift).
__device__ __forceinline__ uint32_t bit_window(const uint16_t* bm, uint32_t s) {
  const uint32_t* w = reinterpret_cast<const uint32_t*>(bm);
  const uint32_t i = s >> 5;
  return __builtin_amdgcn_alignbit(w[i + 1], w[i], s & 31);
}

// Value of 4 ASCII digits, the first (most significant) in the low byte:
// (d0*10 + d1) * 100 + (d2*10 + d3) from two byte dot products.
__device__ __forceinline__ uint32_t value4(uint32_t x) {
  return __umul24(__builtin_amdgcn_udot4(x, 0x0000010Au, 0u, false), 100u) +
         __builtin_amdgcn_udot4(x, 0x010A0000u, 0u, false);
}

// Value of the n (0..8) ASCII digits that end just before tile offset `end`
// (SWAR on two 32-bit words; Appendix D of the paper does the same on one
// 64-bit word).  Reads bytes [end-8, end).
template <int K>
__device__ __forceinline__ uint32_t digits8_before(const TileSmem<K>& sm, int end, int n) {
  const int A = end - 8 + TileSmem<K>::kPadFront;
  const uint32_t* W = reinterpret_cast<const uint32_t*>(sm.text);
  const uint32_t w0 = W[A >> 2], w1 = W[(A >> 2) + 1], w2 = W[(A >> 2) + 2];
  uint32_t lo = __builtin_amdgcn_alignbyte(w1, w0, (uint32_t)A & 3u);
  uint32_t hi = __builtin_amdgcn_alignbyte(w2, w1, (uint32_t)A & 3u);
  const uint64_t keep = sm.keep8[(8 - n) & 15];  // the 8 - n leading bytes dropped
  lo &= (uint32_t)keep;
  hi &= (uint32_t)(keep >> 32);
  return __umul24(value4(lo), 10000u) + value4(hi);
}

// Same for n (0..4) digits.  Reads bytes [end-4, end).
template <int K>
__device__ __forceinline__ uint32_t digits4_before(const TileSmem<K>& sm, int end, int n) {
  const int A = end - 4 + TileSmem<K>::kPadFront;
  const uint32_t* W = reinterpret_cast<const uint32_t*>(sm.text);
  const uint32_t w0 = W[A >> 2], w1 = W[(A >> 2) + 1];
  const uint32_t x = __builtin_amdgcn_alignbyte(w1, w0, (uint32_t)A & 3u);
  const uint32_t keep = (uint32_t)(sm.keep8[(8 - n) & 15] >> 32);
  return value4(x & keep);
}

// Value of the n (0..19) digits ending before `end`; the wave skips groups
// that no lane needs.
template <int K>
__device__ __forceinline__ uint64_t digits_before(const TileSmem<K>& sm, int end, int n) {
  if (__all(n <= 4)) return digits4_before<K>(sm, end, n);
  uint64_t v = digits8_before<K>(sm, end, n < 8 ? n : 8);
  if (__any(n > 8)) {
    const int n1 = n > 16 ? 8 : (n > 8 ? n - 8 : 0);
    v += (uint64_t)digits8_before<K>(sm, end - 8, n1) * 100000000ull;
    if (__any(n > 16)) {  // at most 3 more digits (n <= 19)
      const int n2 = n > 16 ? n - 16 : 0;
      v += (uint64_t)digits4_before<K>(sm, end - 16, n2) * 10000000000000000ull;
    }
  }
  return v;
}

constexpr uint32_t kFastOk = 0, kFastInvalid = 1, kFastSlow = 2;

// Lexing modes of the parse kernel's instances (see k_parse).
constexpr int kModePlain = 0, kModeGrammar = 1, kModeExt = 2;

struct FastLex {
  uint64_t w;
  int32_t q;
  uint32_t neg;
  uint32_t code;
};

// Lexer for a token lying wholly inside the tile, from the digit and
// delimiter bitmaps: the runs of the grammar are found with count-trailing-
// zeros on 32-bit windows instead of a loop over bytes, and the digits are
// converted up to eight at a time.  Tokens of 32 bytes or more, with more than
// 19 mantissa digits or more than 8 exponent digits are left to the
// byte-by-byte lexer (kFastSlow); for all others the result equals
// lex_token's.  kGrammar: the grammar flags (FFP_JSON, FFP_INFNAN, FFP_HEX)
// are honoured; without it they must be clear.
template <int K, bool kGrammar>
__device__ __forceinline__ FastLex fast_lex(const TileSmem<K>& sm, uint32_t s, uint32_t flags) {
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
  const uint32_t cb = tb[s + b], cb1 = tb[s + b + 1];
  const uint32_t cf = tb[s + f1d], cf1 = tb[s + f1d + 1];
  const bool dot = cb == '.';
  const int f0 = dot ? b + 1 : b;
  const int f1 = dot ? f1d : b;
  const uint32_t cx = dot ? cf : cb, cx1 = dot ? cf1 : cb1;
  const bool has_e = f1 < L && (cx | 0x20u) == 'e';
  const bool es = has_e && (cx1 == '-' || cx1 == '+');
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
  if (__any(nint + nfrac > 19)) {
    if (nint + nfrac > 19 && (nint == 0 || (nint == 1 && tb[s + a] == '0'))) {
      const int A = (int)s + f0 + TileSmem<K>::kPadFront;
      const uint32_t* W = reinterpret_cast<const uint32_t*>(sm.text);
      const uint32_t w0 = W[A >> 2], w1 = W[(A >> 2) + 1], w2 = W[(A >> 2) + 2];
      // the 8 bytes from f0, first byte lowest; a zero byte is a '0'
      const uint64_t x =
          ((uint64_t)__builtin_amdgcn_alignbyte(w2, w1, (uint32_t)A & 3u) << 32 |
           __builtin_amdgcn_alignbyte(w1, w0, (uint32_t)A & 3u)) ^ 0x3030303030303030ull;
      const int zf = x == 0 ? 8 : (int)(__builtin_ctzll(x) >> 3);  // < nfrac: nfrac > 18
      ni = 0;
      nf = nfrac - zf;
    }
  }
  if (ni + nf > 19 || nexp > 8) return r;
  const uint64_t iv = digits_before<K>(sm, (int)s + b, ni);
  const uint64_t fv = digits_before<K>(sm, (int)s + f1, nf);
  r.w = iv * sm.pow10[nf] + fv;
  int ev = 0;
  if (__any(has_e)) {  // exponents of up to 4 digits in every lane: one 4-digit group
    const int ne = has_e ? nexp : 0;
    ev = __all(ne <= 4) ? (int)digits4_before<K>(sm, (int)s + e1, ne)
                        : (int)digits8_before<K>(sm, (int)s + e1, ne);
  }
  r.q = (es && cx1 == '-' ? -ev : ev) - nfrac;
  r.code = kFastOk;
  return r;
}

// First position >= p (a tile offset) whose bit in a tile bitmap is clear;
// the bitmaps end in zero bits, so the scan always stops.
__device__ __forceinline__ uint32_t run_end(const uint16_t* bm, uint32_t p) {
  for (;;) {
    const uint32_t w = bit_window(bm, p);
    if (w != ~0u) return p + (uint32_t)__builtin_ctz(~w);
    p += 32;
  }
}

// First position in [p, end) of the tile text whose byte is not '0' (all
// bytes there are digits), or end; 16 bytes per LDS read.
template <int K>
__device__ __forceinline__ uint32_t first_nonzero_digit(const TileSmem<K>& sm, uint32_t p,
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
__device__ Lexed long_lex(const TileSmem<K>& sm, uint32_t s, uint32_t flags) {
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

// Algorithm 1 (and w+1 for long significands) on a lexed token, the queue
// append for undecided tokens, and the stores.  Returns the path counter.
template <class F, bool kExt>
__device__ __forceinline__ int finish_token(const Lexed& L, uint64_t text_pos, const JobDesc& job,
                                            uint64_t idx, const unsigned long long* table,
                                            const ParseParams& P, uint64_t& bits_out,
                                            uint32_t& status_out) {
  Decision<F> d = decide_lexed<F, kExt>(L, table, P.flags);
  bits_out = d.bits;
  status_out = d.fallback ? kPending : d.status;
  uint8_t st = (uint8_t)d.status;
  if (d.fallback) {
    const unsigned long long slot = atomicAdd(&P.st->queue_tail, 1ull);
    if (slot < P.queue_cap) {
      QueueEntry e;
      e.offset = text_pos;
      e.index_job = idx | ((uint64_t)job.job_id << 48);
      P.queue[slot] = e;
    } else {
      atomicOr(&P.st->error, (unsigned)kDevQueue);
      if (job.err_out) *job.err_out = kErrQueue;
    }
    st = kPending;
  }
  gstore(reinterpret_cast<typename F::bits_t*>(job.values) + idx, d.bits);
  gstore(job.status + idx, st);
  return (int)d.path;
}

// Registers: within 128 (four waves per SIMD; the LDS of a 16 KiB tile
// allows four workgroups per CU), and within 96 for the plain instance
// without a reduction at 8 KiB and smaller tiles (five waves per SIMD; at
// 96 the other instances spill to scratch inside the token loop).
// kReduce: the call also keeps the minimum, maximum and count of the
// values.  kMode: kModePlain lexes Section 4's grammar (FFP_REJECT_PLUS
// aside, no grammar flag); kModeGrammar adds the JSON grammar and inf / nan
// (FFP_JSON, FFP_INFNAN); kModeExt adds hexadecimal tokens (FFP_HEX) and the
// directed rounding modes.  Separate instances, so that the plain parse pays
// nothing for either: its register and branch budget is the tightest.
template <int K, bool kSingle, bool kReduce, int kMode>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(K <= 2 && kMode == kModePlain && !kReduce ? 5 : 4))) void
k_parse(ParseParams P) {
  constexpr bool kExt = kMode == kModeExt;
  constexpr bool kGrammar = kMode != kModePlain;
  using S = TileSmem<K>;
  using Packed = typename S::Packed;
  __shared__ S sm;
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
  }
  const uint32_t drep = P.delim.byte * 0x01010101u;
  const uint64_t nblk = total_blocks_of(P.js);
  // tiles per block (the host keeps blocks at least one tile long)
  const int ntiles = (int)((1u << P.js.block_shift) / S::kBytes);
  // path counters, kept in scalars (a runtime-indexed array would live in
  // scratch memory)
  uint32_t c_tok = 0, c_inv = 0, c_early = 0, c_one = 0, c_two = 0, c_fb = 0;

  for (uint64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const JobDesc job = job_of_block(P.js, blk);
    // Tiles cover the job's text as if it started at the 16-byte boundary
    // below `text`: virtual byte v is text[v - align].
    const uint64_t align = (uint64_t)(uintptr_t)job.text & 15u;
    const uint8_t* vbase = job.text - align;
    const uint64_t nbytes = job.nbytes;
    const uint64_t vend = nbytes + align;
    const uint64_t bstart = (blk - job.block_begin) << P.js.block_shift;
    uint64_t next_idx = P.block_prefix[blk] - P.block_prefix[job.block_begin];
    const GlobalSrc gsrc{job.text, nbytes, P.delim};

    // A tile's chunks are loaded at the top of its iteration; the other
    // workgroups on the CU hide the latency.  (Loading the next tile into
    // registers during the token rounds held 4K registers through them and
    // measured no faster.)
    uint4 pre[K];
    // the byte before the block, loaded with the block's first chunks
    const uint32_t block_prev = tid == 0 ? prev_nondelim(vbase, bstart, align, P.delim) : 0u;
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
      uint32_t ndm[K];
#pragma unroll
      for (int c = 0; c < K; ++c) {
        const int chunk = c * kThreads + tid;
        const uint4 v = pre[c];
        *reinterpret_cast<uint4*>(&sm.text[S::kPadFront + chunk * kChunk]) = v;
        ndm[c] = nondelim_mask16<kSingle>(v, drep, sm.delim_lut);
        sm.nd[chunk] = (uint16_t)ndm[c];
        sm.dg[chunk] = (uint16_t)pack_high_bits(digit_word(v.x), digit_word(v.y),
                                                digit_word(v.z), digit_word(v.w));
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
            chunk == 0 ? sm.prev_nd : ((uint32_t)sm.nd[chunk - 1] >> 15) & 1u;
        const uint32_t m = ndm[c];
        startm[c] = m & ~((m << 1) | prevbit) & 0xFFFFu;
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
#pragma unroll
      for (int c = 0; c < K; ++c) {
        uint32_t p = row_off[c] + ((uint32_t)(excl_packed >> (16 * c)) & 0xFFFFu);
        uint32_t m = startm[c];
        const uint32_t base = (uint32_t)((c * kThreads + tid) * kChunk);
        while (m) {
          const uint32_t k = __ffs(m) - 1;
          sm.starts[p++] = (uint16_t)(base + k);
          m &= m - 1;
        }
      }
      __syncthreads();

      // -- one lane per token -------------------------------------------
      // When the tile's last byte belongs to a token, that token (the last
      // one starting here) continues past the tile: the extension is filled
      // before its round; if the token also runs past the extension it is
      // read from global memory, which returns a delimiter past the text.
      const bool straddle = (sm.nd[S::kChunks - 1] >> 15) & 1u;
      const LdsSrc lsrc{sm.text + S::kPadFront, tile_start, sm.delim_lut};
      // tokens of this tile that fit the caller's capacity
      const uint32_t nfit = next_idx >= job.capacity ? 0u
                            : (job.capacity - next_idx < ntok ? (uint32_t)(job.capacity - next_idx)
                                                              : ntok);
      if (straddle && nfit == ntok) {  // the last token is decided here: fill the extension
        if (tid < S::kExtChunks) {  // wave 0: chunk tid of the next tile
          const uint4 v = ext_v;
          *reinterpret_cast<uint4*>(&sm.text[S::kPadFront + S::kBytes + tid * kChunk]) = v;
          const uint32_t m = nondelim_mask16<kSingle>(v, drep, sm.delim_lut);
          sm.nd[S::kChunks + tid] = (uint16_t)m;
          sm.dg[S::kChunks + tid] = (uint16_t)pack_high_bits(digit_word(v.x), digit_word(v.y),
                                                             digit_word(v.z), digit_word(v.w));
          const uint64_t has_delim = (uint64_t)__ballot(m != 0xFFFFu);
          if (tid == 0) sm.ext_end = has_delim != 0;
        }
        __syncthreads();
      }
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
          const uint64_t idx = next_idx + j;
          const uint32_t s = sm.starts[j];
          const uint64_t vpos = tile_start + s;  // virtual
          const uint64_t pos = vpos - align;     // offset in the text
          const bool global = j == global_j;
          FastLex fl;
          if (!global) {
            fl = fast_lex<K, kGrammar>(sm, s, P.flags);
          } else {
            fl.code = kFastSlow;
          }
          Lexed L;
          if (fl.code == kFastSlow) {
            if (global)
              L = lex_token<kExt>(gsrc, pos, P.flags);
            else if (kGrammar && (P.flags & (kFlagJson | kFlagInfNan | kFlagHex)))
              L = lex_token<kExt>(lsrc, vpos, P.flags);
            else
              L = long_lex<K>(sm, s, P.flags);
          } else {
            L.w = fl.w;
            L.q = fl.q;
            L.neg = fl.neg;
            L.kind = fl.code == kFastInvalid ? kLexInvalid : kLexExact;
          }
          int path;
          switch (job.dtype) {
            case kF64: path = finish_token<F64, kExt>(L, pos, job, idx, table, P, vbits, vstatus); break;
            case kF32: path = finish_token<F32, kExt>(L, pos, job, idx, table, P, vbits, vstatus); break;
            case kF16: path = finish_token<F16, kExt>(L, pos, job, idx, table, P, vbits, vstatus); break;
            default: path = finish_token<BF16, kExt>(L, pos, job, idx, table, P, vbits, vstatus); break;
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
          const uint64_t kmin = wave_min_u64(in ? key : kNoMin);
          const uint64_t kmax = wave_max_u64(in ? key : kNoMax);
          const uint64_t cnt = wave_sum_u64(in ? 1u : 0u);
          if (lane == 0 && cnt) {
            atomicMin(&sm.red_min, (unsigned long long)kmin);
            atomicMax(&sm.red_max, (unsigned long long)kmax);
            atomicAdd(&sm.red_count, (unsigned long long)cnt);
          }
        }
      }
      next_idx += ntok;
      if (tid == 0) sm.prev_nd = (sm.nd[S::kChunks - 1] >> 15) & 1u;
    }
  }

  if (kReduce) {
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
constexpr int kFbThreads = 256;
constexpr int kFbWaves = kFbThreads / kWave;

template <class F>
__device__ __forceinline__ void fallback_token(const JobDesc& job, uint64_t pos, uint64_t idx,
                                               FbLds* lds, const FallbackParams& P) {
  typename F::bits_t bits;
  uint32_t status;
  fb_decide<F>(job.text, job.nbytes, pos, g_table, lds, P.flags, bits, status);
  if (fb_lane() == 0) {
    gstore(reinterpret_cast<typename F::bits_t*>(job.values) + idx, bits);
    gstore(job.status + idx, (uint8_t)status);
    uint64_t key;
    if (P.reduce_out && order_key(bits, status, job.dtype, key)) {
      atomicMin(&P.st->red_min, (unsigned long long)key);
      atomicMax(&P.st->red_max, (unsigned long long)key);
      atomicAdd(&P.st->red_count, 1ull);
    }
  }
}

__global__ __launch_bounds__(kFbThreads) void k_fallback(FallbackParams P) {
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
__global__ void k_reduce_final(FallbackParams P) {
  if (threadIdx.x != 0) return;
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
  if (P.flags & (kFlagHex | kFlagRoundMask))
    hipLaunchKernelGGL((k_parse<K, kSingle, kReduce, kModeExt>), dim3(grid), dim3(kThreads), 0, s, P);
  else if (P.flags & (kFlagJson | kFlagInfNan))
    hipLaunchKernelGGL((k_parse<K, kSingle, kReduce, kModeGrammar>), dim3(grid), dim3(kThreads), 0, s,
                       P);
  else
    hipLaunchKernelGGL((k_parse<K, kSingle, kReduce, kModePlain>), dim3(grid), dim3(kThreads), 0, s,
                       P);
}

template <int K, bool kSingle>
static hipError_t launch_parse_k(const ParseParams& P, int grid, hipStream_t s) {
  if (P.reduce_out)
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
  if (P.reduce_out) hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kWave), 0, s, P);
  return hipGetLastError();
}

}  // namespace ffp
