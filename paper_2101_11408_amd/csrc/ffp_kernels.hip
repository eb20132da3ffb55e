// HIP kernels of the parser (gfx950, wave64).
//
//   k_init      clears the per-call scan state and the token count.
//   k_parse     single pass over the text: 16-byte coalesced loads into an
//               LDS tile, delimiter classification, a block scan of token
//               starts, a decoupled look-back across tiles for the global
//               token index, then one lane per token: lexing (Section 4),
//               Algorithm 1 (Sections 5-10), the w / w+1 test for long
//               significands (Section 11) and the stores.  Tokens that stay
//               undecided are appended to a compact queue.
//   k_fallback  exact decision for the queued tokens by big-integer
//               comparison against the halfway point between two
//               neighbouring binary values.
#include <hip/hip_runtime.h>

#include "ffp_device.h"
#include "ffp_internal.h"
#include "ffp_kernels.h"
#include "ffp_table.inc"

namespace ffp {

__device__ const unsigned long long g_table[FFP_TABLE_SIZE * 2] = {FFP_TABLE_ENTRIES};

// ---------------------------------------------------------------------------
// small wave / block helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// Exclusive scan over the 256 threads of a block; `total` receives the sum.
// s_tmp holds 4 words and must not be reused before the next barrier.
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t v, uint64_t& total,
                                                    uint64_t* s_tmp) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  uint64_t x = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint64_t y = __shfl_up(x, d, kWave);
    if (lane >= d) x += y;
  }
  if (lane == kWave - 1) s_tmp[wid] = x;
  __syncthreads();
  uint64_t before = 0, sum = 0;
#pragma unroll
  for (int i = 0; i < kThreads / kWave; ++i) {
    const uint64_t t = s_tmp[i];
    before += (i < wid) ? t : 0;
    sum += t;
  }
  total = sum;
  return before + x - v;
}

__device__ __forceinline__ uint64_t atomic_load_agent(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_store_agent(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Look-back spin budget: a predecessor publishes its aggregate right after
// counting its own tile, so this is never reached unless the scan state is
// corrupt; the kernel then records an internal error and still exits.
constexpr uint32_t kSpinLimit = 1u << 22;

// ---------------------------------------------------------------------------
// k_init
// ---------------------------------------------------------------------------
__global__ void k_init(uint64_t* tile_state, uint64_t ntiles, DeviceState* st,
                       uint64_t* count_out) {
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = tid; i < ntiles; i += stride) tile_state[i] = 0;
  if (tid == 0) {
    st->tile_counter = 0;
    st->error = 0;
    st->queue_tail = 0;
    if (count_out) *count_out = 0;
  }
}

// ---------------------------------------------------------------------------
// k_parse
// ---------------------------------------------------------------------------
template <int K>
struct TileSmem {
  static constexpr int kBytes = kThreads * kChunk * K;
  static constexpr int kChunks = kThreads * K;
  unsigned long long table[FFP_TABLE_SIZE * 2];
  alignas(16) uint8_t text[kBytes];
  uint16_t starts[kBytes / 2];
  uint16_t nd[kChunks];
  uint8_t delim_lut[256];
  uint64_t scan[kThreads / kWave];
  uint64_t tile;
  uint64_t excl;
  uint32_t prev_nd;
};

struct LdsSrc {
  const uint8_t* text;  // LDS tile
  uint64_t tile_start;
  const uint8_t* lut;   // LDS delimiter table
  __device__ __forceinline__ uint32_t operator()(uint64_t i) const {
    return text[i - tile_start];
  }
  __device__ __forceinline__ bool is_end(uint32_t c) const { return lut[c] != 0; }
};

template <class F>
__device__ __forceinline__ void store_result(const JobDesc& job, uint64_t idx,
                                             typename F::bits_t bits, uint8_t st) {
  reinterpret_cast<typename F::bits_t*>(job.values)[idx] = bits;
  job.status[idx] = st;
}

// Decide one token; src_pos is its first byte in the source's coordinates,
// text_pos its offset in the job's text.  Returns the path counter index.
template <class F, class Src>
__device__ __forceinline__ int decide_token(const Src& src, uint64_t src_pos, uint64_t text_pos,
                                            const JobDesc& job, uint64_t idx,
                                            const unsigned long long* table,
                                            const ParseParams& P) {
  const Lexed L = lex_token(src, src_pos, P.flags);
  Decision<F> d = decide_lexed<F>(L, table);
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
    }
    st = kPending;
  }
  store_result<F>(job, idx, d.bits, st);
  return (int)d.path;
}

template <int K>
__global__ __launch_bounds__(kThreads) void k_parse(ParseParams P) {
  using S = TileSmem<K>;
  __shared__ S sm;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wid = tid / kWave;

  for (int i = tid; i < FFP_TABLE_SIZE * 2; i += kThreads) sm.table[i] = g_table[i];
  for (int i = tid; i < 256; i += kThreads) sm.delim_lut[i] = is_delim(P.delim, (uint32_t)i);

  const uint64_t total_tiles = P.jobs ? *P.total_tiles_dev : P.total_tiles;
  // path counters, kept in scalars (a runtime-indexed array would live in
  // scratch memory)
  uint32_t c_tok = 0, c_inv = 0, c_early = 0, c_one = 0, c_two = 0, c_fb = 0;

  for (;;) {
    if (tid == 0) sm.tile = atomicAdd(&P.st->tile_counter, 1u);
    __syncthreads();
    const uint64_t tile = sm.tile;
    if (tile >= total_tiles) break;

    // -- which job owns this tile --------------------------------------
    JobDesc job;
    if (P.jobs) {
      uint32_t lo = 0, hi = P.njobs;  // last job with tile_begin <= tile
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (P.jobs[mid].tile_begin <= tile) lo = mid; else hi = mid;
      }
      job = P.jobs[lo];
    } else {
      job = P.single;
    }
    // Tiles cover the job's text as if it started at the 16-byte boundary
    // below `text`: virtual byte v is text[v - align].  Chunks wholly inside
    // the text use one aligned 16-byte load; the (at most two) edge chunks
    // of a job load byte by byte and never touch memory outside the text.
    const uint64_t align = (uint64_t)(uintptr_t)job.text & 15u;
    const uint8_t* vbase = job.text - align;
    const uint64_t tile_in_job = tile - job.tile_begin;
    const uint64_t tile_start = tile_in_job * S::kBytes;  // virtual
    const uint64_t nbytes = job.nbytes;
    const uint64_t vend = nbytes + align;

    // -- load the tile and classify bytes ------------------------------
    uint32_t ndm[K];
#pragma unroll
    for (int c = 0; c < K; ++c) {
      const int chunk = c * kThreads + tid;
      const uint64_t off = tile_start + (uint64_t)chunk * kChunk;
      uint4 v;
      if (off >= align && off + kChunk <= vend) {
        v = *reinterpret_cast<const uint4*>(vbase + off);
      } else {
        uint32_t wds[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          uint32_t word = 0;
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const uint64_t o = off + k * 4 + b;
            const uint32_t byte = (o >= align && o < vend) ? vbase[o] : P.delim.byte;
            word |= byte << (8 * b);
          }
          wds[k] = word;
        }
        v = make_uint4(wds[0], wds[1], wds[2], wds[3]);
      }
      *reinterpret_cast<uint4*>(&sm.text[chunk * kChunk]) = v;
      const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
      uint32_t m = 0;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const uint32_t byte = (w4[k >> 2] >> (8 * (k & 3))) & 0xFF;
        const bool nd = P.delim.single ? (byte != P.delim.byte) : !sm.delim_lut[byte];
        m |= (uint32_t)nd << k;
      }
      ndm[c] = m;
      sm.nd[chunk] = (uint16_t)m;
    }
    if (tid == 0) {
      uint32_t prev = 0;
      if (tile_start > align) {
        const uint32_t byte = vbase[tile_start - 1];
        prev = P.delim.single ? (byte != P.delim.byte) : !is_delim(P.delim, byte);
      }
      sm.prev_nd = prev;
    }
    __syncthreads();

    // -- token starts: non-delimiter byte after a delimiter -------------
    uint32_t startm[K];
    uint64_t packed = 0;
#pragma unroll
    for (int c = 0; c < K; ++c) {
      const int chunk = c * kThreads + tid;
      const uint32_t prevbit = chunk == 0 ? sm.prev_nd : ((uint32_t)sm.nd[chunk - 1] >> 15) & 1u;
      const uint32_t m = ndm[c];
      startm[c] = m & ~((m << 1) | prevbit) & 0xFFFFu;
      packed |= (uint64_t)__popc(startm[c]) << (16 * c);
    }
    uint64_t total_packed;
    const uint64_t excl_packed = block_excl_scan(packed, total_packed, sm.scan);
    uint32_t row_off[K];
    uint32_t ntok = 0;
#pragma unroll
    for (int c = 0; c < K; ++c) {
      row_off[c] = ntok;
      ntok += (uint32_t)((total_packed >> (16 * c)) & 0xFFFF);
    }
#pragma unroll
    for (int c = 0; c < K; ++c) {
      uint32_t p = row_off[c] + (uint32_t)((excl_packed >> (16 * c)) & 0xFFFF);
      uint32_t m = startm[c];
      const uint32_t base = (uint32_t)((c * kThreads + tid) * kChunk);
      while (m) {
        const uint32_t k = __ffs(m) - 1;
        sm.starts[p++] = (uint16_t)(base + k);
        m &= m - 1;
      }
    }

    // -- decoupled look-back for the global index of the first token ----
    if (wid == 0) {
      const uint64_t agg = ntok;
      uint64_t excl = 0;
      uint64_t* state = P.tile_state;
      if (tile_in_job == 0) {
        if (lane == 0) atomic_store_agent(&state[tile], kFlagInc | agg);
      } else {
        if (lane == 0) atomic_store_agent(&state[tile], kFlagAgg | agg);
        int64_t look = (int64_t)tile - 1 - lane;
        const int64_t first = (int64_t)job.tile_begin;
        uint32_t spins = 0;
        for (;;) {
          const uint64_t s = look >= first ? atomic_load_agent(&state[look]) : kFlagInc;
          const uint32_t flag = (uint32_t)(s >> 62);
          const uint64_t incm = __ballot(flag == 2);
          const uint64_t window = incm ? (((incm & (~incm + 1)) << 1) - 1) : ~0ull;
          const uint64_t invm = __ballot(flag == 0) & window;
          if (invm) {
            if (++spins > kSpinLimit) {
              if (lane == 0) atomicOr(&P.st->error, (unsigned)kDevInternal);
              break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
          }
          const uint64_t mine = ((window >> lane) & 1ull) ? (s & kValueMask) : 0;
          excl += wave_sum_u64(mine);
          if (incm) break;
          look -= kWave;
        }
        if (lane == 0) atomic_store_agent(&state[tile], kFlagInc | (excl + agg));
      }
      if (lane == 0) {
        sm.excl = excl;
        const uint64_t ntiles_job = (vend + S::kBytes - 1) / S::kBytes;
        if (tile_in_job + 1 == ntiles_job) *job.count_out = excl + agg;
      }
    }
    __syncthreads();
    const uint64_t excl = sm.excl;

    // -- one lane per token ---------------------------------------------
    // When the tile's last byte belongs to a token, that token (the last
    // one starting here) may continue past the tile: it is read from global
    // memory, which returns a delimiter past the end of the buffer.
    const bool straddle = (sm.nd[S::kChunks - 1] >> 15) & 1u;
    LdsSrc lsrc{sm.text, tile_start, sm.delim_lut};
    GlobalSrc gsrc{job.text, nbytes, P.delim};
    for (uint32_t j = tid; j < ntok; j += kThreads) {
      const uint64_t idx = excl + j;
      if (idx >= job.capacity) break;
      const uint64_t vpos = tile_start + sm.starts[j];  // virtual
      const uint64_t pos = vpos - align;                 // offset in the text
      int path;
      const bool global = straddle && j == ntok - 1;
      if (job.dtype == kF64) {
        path = global ? decide_token<F64>(gsrc, pos, pos, job, idx, sm.table, P)
                      : decide_token<F64>(lsrc, vpos, pos, job, idx, sm.table, P);
      } else {
        path = global ? decide_token<F32>(gsrc, pos, pos, job, idx, sm.table, P)
                      : decide_token<F32>(lsrc, vpos, pos, job, idx, sm.table, P);
      }
      c_tok += 1;
      c_inv += path == kCntInvalid;
      c_early += path == kCntEarly;
      c_one += path == kCntOne;
      c_two += path == kCntTwo;
      c_fb += path == kCntFallback;
    }
    __syncthreads();
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
// k_fallback: one lane per queued token (see fallback_decide); each lane keeps
// its three big integers in LDS, limbs one wavefront apart.
// ---------------------------------------------------------------------------
constexpr int kFbThreads = kWave;

template <class F>
__device__ void fallback_token(const JobDesc& job, uint64_t pos, uint64_t idx,
                               const DelimSet& delim, DeviceState* st, uint32_t* lds) {
  typename F::bits_t bits;
  uint32_t status;
  const GlobalSrc src{job.text, job.nbytes, delim};
  if (!fallback_decide<F>(src, pos, g_table, lds, kWave, bits, status))
    atomicOr(&st->error, (unsigned)kDevInternal);
  reinterpret_cast<typename F::bits_t*>(job.values)[idx] = bits;
  job.status[idx] = (uint8_t)status;
}

__global__ __launch_bounds__(kFbThreads) void k_fallback(FallbackParams P) {
  __shared__ uint32_t lds[3 * kBigLimbs * kWave];
  const unsigned long long tail = P.st->queue_tail;
  const uint64_t n = tail < P.queue_cap ? tail : P.queue_cap;
  uint32_t* mine = lds + threadIdx.x;
  for (uint64_t i = (uint64_t)blockIdx.x * kFbThreads + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * kFbThreads) {
    const QueueEntry e = P.queue[i];
    const uint32_t job_id = (uint32_t)(e.index_job >> 48);
    const uint64_t idx = e.index_job & ((1ull << 48) - 1);
    const JobDesc job = P.jobs ? P.jobs[job_id] : P.single;
    if (job.dtype == kF64) {
      fallback_token<F64>(job, e.offset, idx, P.delim, P.st, mine);
    } else {
      fallback_token<F32>(job, e.offset, idx, P.delim, P.st, mine);
    }
  }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
template <int K>
static hipError_t launch_parse_k(const ParseParams& P, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_parse<K>, dim3(grid), dim3(kThreads), 0, s, P);
  return hipGetLastError();
}

int parse_tile_bytes(int k) { return kThreads * kChunk * k; }

hipError_t parse_occupancy(int k, int* blocks_per_cu) {
  switch (k) {
    case 1: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_parse<1>, kThreads, 0);
    case 2: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_parse<2>, kThreads, 0);
    case 4: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_parse<4>, kThreads, 0);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_init(uint64_t* tile_state, uint64_t ntiles, DeviceState* st,
                       uint64_t* count_out, hipStream_t s) {
  uint64_t blocks = (ntiles + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_init, dim3((unsigned)blocks), dim3(256), 0, s, tile_state, ntiles, st,
                     count_out);
  return hipGetLastError();
}

hipError_t launch_parse(int k, const ParseParams& P, int grid, hipStream_t s) {
  switch (k) {
    case 1: return launch_parse_k<1>(P, grid, s);
    case 2: return launch_parse_k<2>(P, grid, s);
    case 4: return launch_parse_k<4>(P, grid, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fallback(const FallbackParams& P, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_fallback, dim3(grid), dim3(kFbThreads), 0, s, P);
  return hipGetLastError();
}

}  // namespace ffp
