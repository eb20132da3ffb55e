// C-ABI of the parsing library: context, scratch, argument checks and the
// launch sequence init -> parse -> fallback on the caller's stream.
#include <hip/hip_runtime.h>

#include <stdlib.h>
#include <string.h>

#include <new>
#include <utility>
#include <vector>

#include "ffp.h"
#include "ffp_internal.h"
#include "ffp_kernels.h"

using ffp::DelimSet;
using ffp::DeviceState;
using ffp::JobDesc;
using ffp::QueueEntry;

struct ffp_ctx {
  int device = 0;
  DelimSet delim{};
  uint32_t flags = 0;
  int num_cus = 0;
  int tile_k = 4;
  int blocks_per_cu = 1;
  int fb_grid = 0;

  uint64_t* d_block_sum = nullptr;  // per-block counts, then their prefix
  uint64_t block_cap = 0;
  QueueEntry* d_queue = nullptr;
  uint64_t queue_cap = 0;
  DeviceState* d_state = nullptr;

  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used, ev_free;
  double timed_ms = 0.0;
  uint64_t timed_launches = 0;

  bool counters = false;
};

namespace {

// Keeps the caller's current device across a call.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

bool is_grammar_byte(int c) {
  return (c >= '0' && c <= '9') || c == '.' || c == 'e' || c == 'E' || c == '+' || c == '-';
}

// Grow the scratch for buffers of up to nbytes.  Old buffers may still be in
// use by queued work, so the device is drained before anything is freed.
int grow(ffp_ctx* ctx, uint64_t nbytes) {
  const uint64_t blocks = (nbytes + 15 + ffp::kBlockBytes - 1) / ffp::kBlockBytes + 1;
  // A token that reaches the fallback through the w / w+1 test has more than
  // 19 significant digits, hence at least 20 bytes plus a delimiter (except
  // the last token): (nbytes + 1) / 21 bounds their number.  The reserve
  // covers the inconclusive-product case of Algorithm 1.
  const uint64_t q = (nbytes + 1) / 21 + ffp::kAbortReserve;
  if ((blocks > ctx->block_cap || q > ctx->queue_cap) && hipDeviceSynchronize() != hipSuccess)
    return FFP_E_HIP;
  if (blocks > ctx->block_cap) {
    if (ctx->d_block_sum) (void)hipFree(ctx->d_block_sum);
    ctx->d_block_sum = nullptr;
    ctx->block_cap = 0;
    if (hipMalloc(&ctx->d_block_sum, blocks * sizeof(uint64_t)) != hipSuccess) return FFP_E_NOMEM;
    ctx->block_cap = blocks;
  }
  if (q > ctx->queue_cap) {
    if (ctx->d_queue) (void)hipFree(ctx->d_queue);
    ctx->d_queue = nullptr;
    ctx->queue_cap = 0;
    if (hipMalloc(&ctx->d_queue, q * sizeof(QueueEntry)) != hipSuccess) return FFP_E_NOMEM;
    ctx->queue_cap = q;
  }
  return FFP_SUCCESS;
}

int launch_jobs(ffp_ctx* ctx, const ffp::JobSet& js, uint64_t nblocks, hipStream_t s) {
  ffp::ScanParams sp{};
  sp.js = js;
  sp.block_sum = ctx->d_block_sum;
  sp.st = ctx->d_state;
  if (nblocks > 0) {
    ffp::CountParams cp{};
    cp.js = js;
    cp.block_sum = ctx->d_block_sum;
    cp.delim = ctx->delim;
    uint64_t grid = (uint64_t)ctx->num_cus * 8;
    if (grid > nblocks) grid = nblocks;
    if (ffp::launch_count(ctx->delim.single != 0, cp, (int)grid, s) != hipSuccess) return FFP_E_HIP;
  }
  if (ffp::launch_scan(sp, s) != hipSuccess) return FFP_E_HIP;
  if (nblocks == 0) return FFP_SUCCESS;

  ffp::ParseParams P{};
  P.js = js;
  P.block_prefix = ctx->d_block_sum;
  P.st = ctx->d_state;
  P.queue = ctx->d_queue;
  P.queue_cap = ctx->queue_cap;
  P.delim = ctx->delim;
  P.flags = ctx->flags;
  P.count_paths = ctx->counters ? 1u : 0u;
  uint64_t grid = (uint64_t)ctx->num_cus * (uint64_t)ctx->blocks_per_cu;
  if (grid > nblocks) grid = nblocks;

  std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
  if (ctx->timing) {
    if (!ctx->ev_free.empty()) {
      ev = ctx->ev_free.back();
      ctx->ev_free.pop_back();
    } else {
      if (hipEventCreate(&ev.first) != hipSuccess || hipEventCreate(&ev.second) != hipSuccess)
        return FFP_E_HIP;
    }
    if (hipEventRecord(ev.first, s) != hipSuccess) return FFP_E_HIP;
  }
  if (ffp::launch_parse(ctx->tile_k, ctx->delim.single != 0, P, (int)grid, s) != hipSuccess)
    return FFP_E_HIP;
  if (ctx->timing) {
    if (hipEventRecord(ev.second, s) != hipSuccess) return FFP_E_HIP;
    ctx->ev_used.push_back(ev);
  }

  ffp::FallbackParams F{};
  F.js = js;
  F.queue = ctx->d_queue;
  F.queue_cap = ctx->queue_cap;
  F.st = ctx->d_state;
  F.delim = ctx->delim;
  if (ffp::launch_fallback(F, ctx->fb_grid, s) != hipSuccess) return FFP_E_HIP;
  return FFP_SUCCESS;
}

int parse_common(ffp_ctx* ctx, uint32_t dtype, const uint8_t* d_text, uint64_t nbytes,
                 void* d_values, uint8_t* d_status, uint64_t capacity, uint64_t* d_count,
                 void* stream) {
  if (!ctx || !d_count) return FFP_E_ARG;
  if (nbytes >= ffp::kMaxBytes) return FFP_E_ARG;
  if (nbytes > 0 && !d_text) return FFP_E_ARG;
  if (capacity > 0 && (!d_values || !d_status)) return FFP_E_ARG;
  DeviceGuard g(ctx->device);
  int rc = grow(ctx, nbytes);
  if (rc != FFP_SUCCESS) return rc;

  JobDesc job{};
  job.text = d_text;
  job.nbytes = nbytes;
  job.values = d_values;
  job.status = d_status;
  job.capacity = capacity;
  job.count_out = d_count;
  job.block_begin = 0;
  job.dtype = dtype;
  job.job_id = 0;
  // blocks start at the 16-byte boundary at or below d_text
  const uint64_t vbytes = nbytes ? nbytes + ((uintptr_t)d_text & 15u) : 0;
  const uint64_t nblocks = (vbytes + ffp::kBlockBytes - 1) / ffp::kBlockBytes;

  ffp::JobSet js{};
  js.single = job;
  js.jobs = nullptr;
  js.njobs = 1;
  js.total_blocks = nblocks;
  js.total_blocks_dev = nullptr;
  return launch_jobs(ctx, js, nblocks, (hipStream_t)stream);
}

int64_t finish_sync(ffp_ctx* ctx, int rc, uint64_t capacity, uint64_t* d_count, void* stream) {
  if (rc != FFP_SUCCESS) return rc;
  DeviceGuard g(ctx->device);
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return FFP_E_HIP;
  uint64_t count = 0;
  unsigned err = 0;
  if (hipMemcpy(&count, d_count, sizeof(count), hipMemcpyDeviceToHost) != hipSuccess) return FFP_E_HIP;
  if (hipMemcpy(&err, &ctx->d_state->error, sizeof(err), hipMemcpyDeviceToHost) != hipSuccess)
    return FFP_E_HIP;
  if (err & ffp::kDevInternal) return FFP_E_INTERNAL;
  if (err & ffp::kDevQueue) return FFP_E_QUEUE;
  if (count > capacity) return FFP_E_CAPACITY;
  return (int64_t)count;
}

}  // namespace

extern "C" {

const char* ffp_strerror(int err) {
  switch (err) {
    case FFP_SUCCESS: return "success";
    case FFP_E_ARG: return "invalid argument";
    case FFP_E_CAPACITY: return "more tokens than the output capacity";
    case FFP_E_HIP: return "HIP runtime error";
    case FFP_E_NOMEM: return "device memory allocation failed";
    case FFP_E_BUDGET: return "request exceeds the HBM budget";
    case FFP_E_BUSY: return "no free slot";
    case FFP_E_QUEUE: return "fallback queue overflow";
    case FFP_E_INTERNAL: return "internal consistency check failed";
    default: return "unknown error";
  }
}

int ffp_create(int hip_device, const ffp_options* opts, ffp_ctx** out) {
  if (!out) return FFP_E_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev)
    return FFP_E_ARG;
  ffp_options o{};
  if (opts) {
    o = *opts;
  } else {
    o.delim_set['\n' >> 6] |= 1ull << ('\n' & 63);
  }
  if (o.flags & ~FFP_REJECT_PLUS) return FFP_E_ARG;
  int members = 0, first = -1;
  for (int c = 0; c < 256; ++c) {
    if ((o.delim_set[c >> 6] >> (c & 63)) & 1) {
      if (is_grammar_byte(c)) return FFP_E_ARG;
      if (first < 0) first = c;
      ++members;
    }
  }
  if (members == 0) return FFP_E_ARG;

  ffp_ctx* ctx = new (std::nothrow) ffp_ctx();
  if (!ctx) return FFP_E_NOMEM;
  ctx->device = hip_device;
  for (int i = 0; i < 4; ++i) ctx->delim.bits[i] = o.delim_set[i];
  ctx->delim.single = members == 1 ? 1u : 0u;
  ctx->delim.byte = (uint32_t)first;
  ctx->flags = o.flags;
  if (const char* k = getenv("FFP_TILE_K")) {
    const int v = atoi(k);
    if (v == 1 || v == 2 || v == 4) ctx->tile_k = v;
  }

  DeviceGuard g(hip_device);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) {
    delete ctx;
    return FFP_E_HIP;
  }
  ctx->num_cus = prop.multiProcessorCount;
  if (ffp::parse_occupancy(ctx->tile_k, ctx->delim.single != 0, &ctx->blocks_per_cu) != hipSuccess ||
      ctx->blocks_per_cu < 1)
    ctx->blocks_per_cu = 1;
  ctx->fb_grid = ctx->num_cus * 2;
  if (hipMalloc(&ctx->d_state, sizeof(DeviceState)) != hipSuccess) {
    delete ctx;
    return FFP_E_NOMEM;
  }
  if (hipMemset(ctx->d_state, 0, sizeof(DeviceState)) != hipSuccess ||
      grow(ctx, 1 << 20) != FFP_SUCCESS) {
    ffp_destroy(ctx);
    return FFP_E_NOMEM;
  }
  *out = ctx;
  return FFP_SUCCESS;
}

void ffp_destroy(ffp_ctx* ctx) {
  if (!ctx) return;
  {
    DeviceGuard g(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto& e : ctx->ev_used) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    for (auto& e : ctx->ev_free) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    if (ctx->d_block_sum) (void)hipFree(ctx->d_block_sum);
    if (ctx->d_queue) (void)hipFree(ctx->d_queue);
    if (ctx->d_state) (void)hipFree(ctx->d_state);
  }
  delete ctx;
}

int ffp_reserve(ffp_ctx* ctx, uint64_t max_nbytes) {
  if (!ctx || max_nbytes >= ffp::kMaxBytes) return FFP_E_ARG;
  DeviceGuard g(ctx->device);
  return grow(ctx, max_nbytes);
}

int ffp_parse_f64(ffp_ctx* ctx, const uint8_t* d_text, uint64_t nbytes, double* d_values,
                  uint8_t* d_status, uint64_t capacity, uint64_t* d_count, void* stream) {
  return parse_common(ctx, ffp::kF64, d_text, nbytes, d_values, d_status, capacity, d_count,
                      stream);
}

int ffp_parse_f32(ffp_ctx* ctx, const uint8_t* d_text, uint64_t nbytes, float* d_values,
                  uint8_t* d_status, uint64_t capacity, uint64_t* d_count, void* stream) {
  return parse_common(ctx, ffp::kF32, d_text, nbytes, d_values, d_status, capacity, d_count,
                      stream);
}

int64_t ffp_parse_f64_sync(ffp_ctx* ctx, const uint8_t* d_text, uint64_t nbytes,
                           double* d_values, uint8_t* d_status, uint64_t capacity,
                           uint64_t* d_count, void* stream) {
  const int rc = parse_common(ctx, ffp::kF64, d_text, nbytes, d_values, d_status, capacity,
                              d_count, stream);
  return finish_sync(ctx, rc, capacity, d_count, stream);
}

int64_t ffp_parse_f32_sync(ffp_ctx* ctx, const uint8_t* d_text, uint64_t nbytes,
                           float* d_values, uint8_t* d_status, uint64_t capacity,
                           uint64_t* d_count, void* stream) {
  const int rc = parse_common(ctx, ffp::kF32, d_text, nbytes, d_values, d_status, capacity,
                              d_count, stream);
  return finish_sync(ctx, rc, capacity, d_count, stream);
}

int ffp_last_device_error(ffp_ctx* ctx) {
  if (!ctx) return FFP_E_ARG;
  DeviceGuard g(ctx->device);
  unsigned err = 0;
  if (hipMemcpy(&err, &ctx->d_state->error, sizeof(err), hipMemcpyDeviceToHost) != hipSuccess)
    return FFP_E_HIP;
  if (err & ffp::kDevInternal) return FFP_E_INTERNAL;
  if (err & ffp::kDevQueue) return FFP_E_QUEUE;
  return FFP_SUCCESS;
}

int ffp_timing_enable(ffp_ctx* ctx, int enable) {
  if (!ctx) return FFP_E_ARG;
  ctx->timing = enable != 0;
  return FFP_SUCCESS;
}

int ffp_timing_read(ffp_ctx* ctx, double* total_ms, uint64_t* launches) {
  if (!ctx || !total_ms || !launches) return FFP_E_ARG;
  DeviceGuard g(ctx->device);
  for (auto& e : ctx->ev_used) {
    if (hipEventSynchronize(e.second) != hipSuccess) return FFP_E_HIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e.first, e.second) != hipSuccess) return FFP_E_HIP;
    ctx->timed_ms += ms;
    ctx->timed_launches += 1;
    ctx->ev_free.push_back(e);
  }
  ctx->ev_used.clear();
  *total_ms = ctx->timed_ms;
  *launches = ctx->timed_launches;
  ctx->timed_ms = 0.0;
  ctx->timed_launches = 0;
  return FFP_SUCCESS;
}

int ffp_counters_enable(ffp_ctx* ctx, int enable) {
  if (!ctx) return FFP_E_ARG;
  ctx->counters = enable != 0;
  return FFP_SUCCESS;
}

int ffp_counters_read(ffp_ctx* ctx, uint64_t counters[6]) {
  if (!ctx || !counters) return FFP_E_ARG;
  DeviceGuard g(ctx->device);
  unsigned long long c[8];
  if (hipDeviceSynchronize() != hipSuccess) return FFP_E_HIP;
  if (hipMemcpy(c, ctx->d_state->counters, sizeof(c), hipMemcpyDeviceToHost) != hipSuccess)
    return FFP_E_HIP;
  if (hipMemset(ctx->d_state->counters, 0, sizeof(c)) != hipSuccess) return FFP_E_HIP;
  for (int i = 0; i < 6; ++i) counters[i] = c[i];
  return FFP_SUCCESS;
}

}  // extern "C"
