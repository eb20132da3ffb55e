// C-ABI of the parsing library: contexts, scratch, argument checks, the
// stream-ordered launch sequences (plain and batched), captured graphs and
// the autotuner.
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "ffp.h"
#include "ffp_context.h"
#include "ffp_internal.h"
#include "ffp_kernels.h"

namespace {

constexpr uint32_t kMaxJobs = 65535;  // job ids travel in 16 bits
constexpr uint64_t kMaxBatchBytes = 1ull << 52;

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

// Bytes a token of the grammar selected by `flags` may contain: such a byte
// cannot be a delimiter (the lexers would read across it).
bool is_grammar_byte(int c, uint32_t flags) {
  if ((c >= '0' && c <= '9') || c == '.' || c == 'e' || c == 'E' || c == '+' || c == '-')
    return true;
  const int l = c | 0x20;
  if ((flags & FFP_HEX) && ((l >= 'a' && l <= 'f') || l == 'x' || l == 'p')) return true;
  if ((flags & FFP_INFNAN) && (l == 'a' || l == 'f' || l == 'i' || l == 'n' || l == 't' || l == 'y'))
    return true;
  return false;
}

template <class T>
int grow_array(T** p, uint64_t* cap, uint64_t need) {
  if (need <= *cap) return FFP_SUCCESS;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *cap = 0;
  if (hipMalloc(p, need * sizeof(T)) != hipSuccess) return FFP_E_NOMEM;
  *cap = need;
  return FFP_SUCCESS;
}

// Grow the scratch for up to `bytes` of text spread over `njobs` jobs.  Old
// buffers may still be in use by queued work, so the device is drained before
// anything is freed.
int grow(ffp_ctx* ctx, uint64_t bytes, uint64_t njobs) {
  // every job may start 15 bytes into its first block and end in a partial
  // block; one more entry holds the grand total
  const uint64_t blocks = ((bytes + 15 * njobs) >> ffp::kMinBlockShift) + 2 * njobs + 1;
  // A token that reaches the fallback through the w / w+1 test has more than
  // 19 significant digits, hence at least 20 bytes plus a delimiter (except
  // the last token of a job): (bytes + njobs) / 21 bounds their number.  The
  // reserve covers the inconclusive-product case of Algorithm 1.
  const uint64_t q = (bytes + njobs) / 21 + ffp::kAbortReserve;
  const bool batch = njobs > 1;
  if (blocks > ctx->block_cap || q > ctx->queue_cap || (batch && njobs > ctx->jobs_cap)) {
    if (hipDeviceSynchronize() != hipSuccess) return FFP_E_HIP;
  }
  int rc = grow_array(&ctx->d_block_sum, &ctx->block_cap, blocks);
  if (rc == FFP_SUCCESS) rc = grow_array(&ctx->d_queue, &ctx->queue_cap, q);
  if (rc == FFP_SUCCESS && batch) rc = grow_array(&ctx->d_jobs, &ctx->jobs_cap, njobs);
  return rc;
}

// Launch shape of one call: block size, tile size and workgroups.
struct CallShape {
  uint32_t block_shift;
  int tile_k;
  int grid;  // parse workgroups before clipping to the block count
};

// Whether a call launches the plain instance of the parse kernel without a
// reduction (no grammar or rounding flag).
bool plain_instance(const ffp_ctx* ctx, bool reduce) {
  return (ctx->flags & (FFP_JSON | FFP_INFNAN | FFP_HEX | FFP_ROUND_MASK)) == 0 && !reduce;
}

// Tile of a call when the context has no fixed schedule: 16 KiB (the plain
// instance without a reduction runs there at five waves per SIMD with its
// shorter start list; the others at four, where the larger tile halves the
// per-tile work).  Measured on 10M mixed numbers: 0.139 against 0.146 ms for
// the plain instance, 0.224 against 0.239 with the reduction, 0.165 against
// 0.181 with the JSON and inf/nan grammar, 0.185 against 0.200 rounding up.
// JSON documents and CSV tables take 8 KiB tiles (their 16 KiB instances
// spill registers).  Small calls get smaller tiles with their smaller
// blocks (call_shape).
int auto_tile_k(const ffp_ctx* ctx) {
  return (ctx->flags & (FFP_JSON_DOCUMENT | FFP_CSV)) ? 2 : 4;
}

// The largest block (64, 16 or 4 KiB) that still gives every parse
// workgroup two blocks; small inputs get small blocks (and tiles no larger
// than a block) so that they spread over many workgroups.
CallShape call_shape(const ffp_ctx* ctx, uint64_t bytes, bool reduce) {
  CallShape cs{};
  int k = ctx->tile_auto ? auto_tile_k(ctx) : ctx->tile_k;
  int bpc = ctx->tile_auto ? 0 : ctx->blocks_per_cu;
  const bool plain = plain_instance(ctx, reduce);
  auto grid_for = [&](int kk, int b) {
    // resident workgroups of the instance this call launches
    const int lim = plain ? ctx->max_bpc[kk] : ctx->max_bpc_wide[kk];
    if (b < 1 || b > lim) b = lim;
    return ctx->num_cus * (b < 1 ? 1 : b);
  };
  uint32_t shift = ffp::kMinBlockShift;
  if (ctx->block_kib) {
    shift = ctx->block_kib == 64 ? 16 : ctx->block_kib == 16 ? 14 : 12;
  } else {
    const uint64_t g = (uint64_t)grid_for(k, bpc);
    for (uint32_t sh = ffp::kMaxBlockShift; sh > ffp::kMinBlockShift; sh -= 2) {
      if ((bytes >> sh) >= 2 * g) {
        shift = sh;
        break;
      }
    }
  }
  while (k > 1 && (4096u * (uint32_t)k) > (1u << shift)) {
    k >>= 1;
    bpc = 0;  // the tuned count belongs to the larger tile
  }
  cs.block_shift = shift;
  cs.tile_k = k;
  cs.grid = grid_for(k, bpc);
  return cs;
}

// The device scratch a call runs on: the context's own (grown as needed) or
// the fixed array of the entry point that allocates nothing.
struct Scratch {
  uint64_t* block_sum;
  QueueEntry* queue;
  uint64_t queue_cap;
  DeviceState* state;
  bool fixed;  // the fixed array: no timing events, no path counters
};

Scratch own_scratch(const ffp_ctx* ctx) {
  return Scratch{ctx->d_block_sum, ctx->d_queue, ctx->queue_cap, ctx->d_state, false};
}

// Calls of at most this many blocks run without the scan kernel: each parse
// workgroup sums the counts of its job's earlier blocks itself (one launch
// less, which is most of a small call's time).
constexpr uint64_t kSumInParseMaxBlocks = 1024;

// Plain calls of at most this many blocks (32 KiB) run without the count
// kernel as well: each parse workgroup counts the tokens before its block
// from the text (at most 28 KiB of cached reads) instead of waiting for a
// kernel launch.  Measured from launch to a synchronised stream: 21.2 us
// against 23.3 us at 4 KiB, 24.1 against 24.7 at 32 KiB; past that the
// counting costs more than the launch (26.5 against 24.9 us at 64 KiB).
constexpr uint64_t kSelfCountMaxBlocks = 8;

// Plain calls of at most this many 4 KiB blocks (128 KiB) run without the
// fallback kernel: each parse workgroup decides the queued tokens of its own
// block after parsing it (ParseParams::fb_local), one wave per token.
// Measured from launch to a synchronised stream on easy text: 20.8 against
// 22.1 us at 4 KiB, 24.4 against 25.7 us at 64 KiB.  A block that queues
// many tokens keeps four waves on them instead of the fallback kernel's
// wider grid, so texts of hard tokens take longer (4 KiB: 52.7 against
// 42.2 us).
constexpr uint64_t kLocalFbMaxBlocks = 32;

// count -> scan -> parse -> fallback for a job set whose block count is
// `nblocks` (plain calls) or on the device (batched calls: nblocks is then
// the scratch's bound and max_blocks the call's); small calls skip the scan,
// the smallest the count kernel, small plain calls the fallback kernel.
int launch_jobs(ffp_ctx* ctx, const Scratch& sc, const ffp::JobSet& js, const CallShape& shape,
                uint64_t nblocks, uint64_t max_blocks, hipStream_t s) {
  // (the parse kernel's 4 KiB-tile instances carry the summation)
  // (JSON documents need the scan: it gives each block its string state)
  const bool json_doc = (ctx->flags & FFP_JSON_DOCUMENT) != 0;
  const bool csv = (ctx->flags & FFP_CSV) != 0;
  uint64_t* const reduce_out = js.jobs ? nullptr : ctx->reduce_out;  // plain calls only
  uint64_t* const sum_out = js.jobs ? nullptr : ctx->sum_out;
  const bool count_paths = ctx->counters && !sc.fixed;
  // (the reductions and the path counters live in the main state)
  const bool self_count = !js.jobs && !sc.fixed && ctx->d_spare && nblocks > 0 &&
                          nblocks <= kSelfCountMaxBlocks && shape.tile_k == 1 &&
                          js.block_shift == ffp::kMinBlockShift && !json_doc && !csv &&
                          !reduce_out && !sum_out && !count_paths;
  const bool sum_in_parse = !self_count && nblocks > 0 && max_blocks <= kSumInParseMaxBlocks &&
                            shape.tile_k == 1 && !json_doc;
  const bool fb_local = !js.jobs && nblocks > 0 && nblocks <= kLocalFbMaxBlocks &&
                        shape.tile_k == 1 && js.block_shift == ffp::kMinBlockShift && !json_doc &&
                        !csv && !reduce_out && !sum_out &&
                        nblocks * ffp::kLocalQueueSeg <= sc.queue_cap;
  // A call without the count kernel runs on the spare state the previous
  // call left clean and cleans the other one; every other call cleans its
  // own state and both spares.
  DeviceState* st = sc.state;
  DeviceState* other = nullptr;
  if (self_count) {
    st = ctx->d_spare + ctx->spare_sel;
    other = ctx->d_spare + (1 - ctx->spare_sel);
    ctx->spare_sel ^= 1;
  }
  DeviceState* const spare = sc.fixed ? nullptr : ctx->d_spare;
  ctx->last_state = st;
  ffp::ScanParams sp{};
  sp.js = js;
  sp.block_sum = sc.block_sum;
  sp.st = st;
  sp.spare = spare;
  sp.json_doc = json_doc ? 1u : 0u;
  // the 16 KiB plain parse keeps at most kShortTileStarts starts per tile:
  // 16 KiB blocks are tiles, so their counts decide; 64 KiB blocks carry a
  // flag for a dense tile from the count kernel (4 KiB blocks never run
  // 16 KiB tiles)
  sp.dense_limit = json_doc || js.block_shift == ffp::kMaxBlockShift ? 0u : ffp::kShortTileStarts;
  if (nblocks > 0 && !self_count) {
    ffp::CountParams cp{};
    cp.js = js;
    cp.block_sum = sc.block_sum;
    cp.delim = ctx->delim;
    cp.st = st;
    cp.spare = spare;
    cp.reset_state = sum_in_parse ? 1u : 0u;
    cp.json_doc = json_doc ? 1u : 0u;
    cp.csv = csv ? 1u : 0u;
    cp.csv_columns = ctx->csv_columns;
    uint64_t grid = (uint64_t)ctx->num_cus * 8;
    if (grid > nblocks) grid = nblocks;
    if (ffp::launch_count(ctx->delim.single != 0, cp, (int)grid, s) != hipSuccess) return FFP_E_HIP;
  }
  if (!sum_in_parse && !self_count && ffp::launch_scan(sp, s) != hipSuccess) return FFP_E_HIP;
  if (nblocks == 0) {  // no token: the reductions of an empty set
    ffp::FallbackParams F{};
    F.st = st;
    F.js = js;
    F.reduce_out = reduce_out;
    F.sum_out = sum_out;
    return ffp::launch_reduce_final(F, s) == hipSuccess ? FFP_SUCCESS : FFP_E_HIP;
  }

  ffp::ParseParams P{};
  P.js = js;
  P.block_prefix = sc.block_sum;
  P.st = st;
  P.queue = sc.queue;
  P.queue_cap = sc.queue_cap;
  P.delim = ctx->delim;
  P.flags = ctx->flags;
  P.count_paths = count_paths ? 1u : 0u;
  P.sum_in_parse = sum_in_parse ? 1u : 0u;
  P.self_count = self_count ? 1u : 0u;
  P.other_st = other;
  P.csv_columns = ctx->csv_columns;
  P.fb_local = fb_local ? 1u : 0u;
  P.reduce_out = reduce_out;
  P.sum_out = sum_out;
  uint64_t grid = (uint64_t)shape.grid;
  if (grid > nblocks) grid = nblocks;

  std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
  const bool timing = ctx->timing && !sc.fixed;
  if (timing) {
    if (!ctx->ev_free.empty()) {
      ev = ctx->ev_free.back();
      ctx->ev_free.pop_back();
    } else {
      // timing-only events: no system-scope fence (cache write-back and
      // invalidation) at the record, which would otherwise slow down the
      // kernels around it
      if (hipEventCreateWithFlags(&ev.first, hipEventDisableSystemFence) != hipSuccess ||
          hipEventCreateWithFlags(&ev.second, hipEventDisableSystemFence) != hipSuccess)
        return FFP_E_HIP;
    }
    if (hipEventRecord(ev.first, s) != hipSuccess) return FFP_E_HIP;
  }
  if (ffp::launch_parse(shape.tile_k, ctx->delim.single != 0, P, (int)grid, s) != hipSuccess)
    return FFP_E_HIP;
  if (timing) {
    if (hipEventRecord(ev.second, s) != hipSuccess) return FFP_E_HIP;
    ctx->ev_used.push_back(ev);
  }
  if (fb_local) return FFP_SUCCESS;  // the parse kernel decided the queued tokens

  ffp::FallbackParams F{};
  F.js = js;
  F.queue = sc.queue;
  F.queue_cap = sc.queue_cap;
  F.st = st;
  F.delim = ctx->delim;
  F.reduce_out = P.reduce_out;
  F.sum_out = P.sum_out;
  F.flags = P.flags;
  // a small plain call queues at most a few hundred tokens per 4 KiB block:
  // a grid to match (launching the full grid of idle workgroups costs more
  // than the usual empty queue's work)
  uint64_t fb_grid = (uint64_t)ctx->fb_grid;
  if (!js.jobs && nblocks <= kSumInParseMaxBlocks) {
    const uint64_t want = nblocks * 8 < 16 ? 16 : nblocks * 8;
    if (want < fb_grid) fb_grid = want;
  }
  if (ffp::launch_fallback(F, (int)fb_grid, s) != hipSuccess) return FFP_E_HIP;
  return FFP_SUCCESS;
}

int parse_common(ffp_ctx* ctx, uint32_t dtype, const uint8_t* d_text, uint64_t nbytes,
                 void* d_values, uint8_t* d_status, uint64_t capacity, uint64_t* d_count,
                 void* stream, int32_t* d_err = nullptr, bool fixed = false) {
  if (!ctx || !d_count) return FFP_E_ARG;
  if (nbytes >= ffp::kMaxBytes) return FFP_E_ARG;
  if (nbytes > 0 && !d_text) return FFP_E_ARG;
  if (capacity > 0 && (!d_values || !d_status)) return FFP_E_ARG;
  if (fixed && nbytes > ffp::kNoAllocMaxBytes) return FFP_E_SIZE;
  if (fixed && !ctx->d_fixed) return FFP_E_HIP;
  DeviceGuard g(ctx->device);
  Scratch sc{};
  if (fixed) {
    // the fixed array: nothing is allocated, grown or freed
    unsigned char* base = ctx->d_fixed;
    sc.state = reinterpret_cast<DeviceState*>(base + ffp::kNoAllocStateOff);
    sc.block_sum = reinterpret_cast<uint64_t*>(base + ffp::kNoAllocBlockOff);
    sc.queue = reinterpret_cast<QueueEntry*>(base + ffp::kNoAllocQueueOff);
    sc.queue_cap = ffp::kNoAllocQueue;
    sc.fixed = true;
  } else {
    const int rc = grow(ctx, nbytes, 1);
    if (rc != FFP_SUCCESS) return rc;
    sc = own_scratch(ctx);
  }

  JobDesc job{};
  job.text = d_text;
  job.nbytes = nbytes;
  job.values = d_values;
  job.status = d_status;
  job.capacity = capacity;
  job.count_out = d_count;
  job.err_out = d_err;
  job.block_begin = 0;
  job.dtype = dtype;
  job.job_id = 0;
  const CallShape shape =
      call_shape(ctx, nbytes, ctx->reduce_out != nullptr || ctx->sum_out != nullptr);
  // blocks start at the 16-byte boundary at or below d_text
  const uint64_t vbytes = nbytes ? nbytes + ((uintptr_t)d_text & 15u) : 0;
  const uint64_t nblocks = (vbytes + (1ull << shape.block_shift) - 1) >> shape.block_shift;

  ffp::JobSet js{};
  js.single = job;
  js.jobs = nullptr;
  js.njobs = 1;
  js.block_shift = shape.block_shift;
  js.total_blocks = nblocks;
  js.total_blocks_dev = nullptr;
  return launch_jobs(ctx, sc, js, shape, nblocks, nblocks, (hipStream_t)stream);
}

int batch_common(ffp_ctx* ctx, ffp_job* d_jobs, uint32_t njobs, uint64_t max_total_bytes,
                 hipStream_t s) {
  if (!ctx || !d_jobs || njobs == 0 || njobs > kMaxJobs) return FFP_E_ARG;
  if (max_total_bytes >= kMaxBatchBytes) return FFP_E_ARG;
  if (ctx->flags & (FFP_JSON_DOCUMENT | FFP_CSV)) return FFP_E_ARG;  // plain calls only
  DeviceGuard g(ctx->device);
  // at least two jobs' worth of job table, so that grow() sizes it
  int rc = grow(ctx, max_total_bytes, njobs < 2 ? 2 : njobs);
  if (rc != FFP_SUCCESS) return rc;
  const CallShape shape = call_shape(ctx, max_total_bytes, false);
  ffp::PrepParams pp{};
  pp.user = reinterpret_cast<ffp::UserJob*>(d_jobs);
  pp.njobs = njobs;
  pp.block_shift = shape.block_shift;
  pp.jobs = ctx->d_jobs;
  pp.st = ctx->d_state;
  pp.block_cap = ctx->block_cap - 1;
  pp.max_bytes = max_total_bytes;
  if (ffp::launch_prep(pp, s) != hipSuccess) return FFP_E_HIP;
  ffp::JobSet js{};
  js.jobs = ctx->d_jobs;
  js.njobs = njobs;
  js.block_shift = shape.block_shift;
  js.total_blocks = 0;
  js.total_blocks_dev = reinterpret_cast<const uint64_t*>(&ctx->d_state->total_blocks);
  // grids are sized for the largest batch the scratch allows; kernels read
  // the true block count on the device
  // the call's bound on its blocks (every job may start 15 bytes into its
  // first block and end in a partial one)
  const uint64_t max_blocks =
      ((max_total_bytes + 15ull * njobs) >> shape.block_shift) + 2ull * njobs;
  return launch_jobs(ctx, own_scratch(ctx), js, shape, ctx->block_cap - 1, max_blocks, s);
}

int64_t finish_sync(ffp_ctx* ctx, int rc, uint64_t capacity, uint64_t* d_count, void* stream) {
  if (rc != FFP_SUCCESS) return rc;
  DeviceGuard g(ctx->device);
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return FFP_E_HIP;
  uint64_t count = 0;
  unsigned err = 0;
  if (hipMemcpy(&count, d_count, sizeof(count), hipMemcpyDeviceToHost) != hipSuccess) return FFP_E_HIP;
  if (hipMemcpy(&err, &ctx->last_state->error, sizeof(err), hipMemcpyDeviceToHost) != hipSuccess)
    return FFP_E_HIP;
  if (err & ffp::kDevInternal) return FFP_E_INTERNAL;
  if (err & ffp::kDevQueue) return FFP_E_QUEUE;
  if (count > capacity) return FFP_E_CAPACITY;
  return (int64_t)count;
}

// --- autotuner cache: a flat JSON object {"key": [tile_k, blocks_per_cu]} --
std::map<std::string, std::pair<int, int>> read_cache(const char* path) {
  std::map<std::string, std::pair<int, int>> out;
  FILE* f = fopen(path, "r");
  if (!f) return out;
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
  fclose(f);
  size_t i = 0;
  while ((i = text.find('"', i)) != std::string::npos) {
    const size_t j = text.find('"', i + 1);
    if (j == std::string::npos) break;
    const std::string key = text.substr(i + 1, j - i - 1);
    int a = 0, b = 0;
    const size_t lb = text.find('[', j);
    if (lb == std::string::npos || sscanf(text.c_str() + lb, "[%d,%d]", &a, &b) != 2) break;
    out[key] = {a, b};
    i = text.find(']', lb);
    if (i == std::string::npos) break;
  }
  return out;
}

void write_cache(const char* path, const std::map<std::string, std::pair<int, int>>& m) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return;
  fprintf(f, "{\n");
  size_t k = 0;
  for (const auto& e : m)
    fprintf(f, "  \"%s\": [%d, %d]%s\n", e.first.c_str(), e.second.first, e.second.second,
            ++k < m.size() ? "," : "");
  fprintf(f, "}\n");
  fclose(f);
  rename(tmp.c_str(), path);
}

std::string tune_key(const ffp_ctx* ctx, uint32_t njobs, uint64_t bytes) {
  int lg = 0;
  while ((1ull << (lg + 1)) <= bytes) ++lg;
  int lj = 0;
  while ((1u << (lj + 1)) <= njobs) ++lj;
  char key[160];
  snprintf(key, sizeof key, "%s|cus=%d|jobs=2^%d|bytes=2^%d|single=%u", ctx->arch.c_str(),
           ctx->num_cus, lj, lg, ctx->delim.single);
  return key;
}

}  // namespace

namespace ffp {

int ctx_grow(ffp_ctx* ctx, uint64_t bytes, uint64_t njobs) {
  DeviceGuard g(ctx->device);
  return grow(ctx, bytes, njobs);
}

int ctx_parse(ffp_ctx* ctx, uint32_t dtype, const uint8_t* d_text, uint64_t nbytes,
              void* d_values, uint8_t* d_status, uint64_t capacity, uint64_t* d_count,
              hipStream_t s, int32_t* d_err) {
  return parse_common(ctx, dtype, d_text, nbytes, d_values, d_status, capacity, d_count, s,
                      d_err);
}

int ctx_batch(ffp_ctx* ctx, ffp_job* d_jobs, uint32_t njobs, uint64_t max_total_bytes,
              hipStream_t s) {
  return batch_common(ctx, d_jobs, njobs, max_total_bytes, s);
}

int ctx_clone(const ffp_ctx* src, ffp_ctx** out) {
  ffp_options o{};
  for (int i = 0; i < 4; ++i) o.delim_set[i] = src->delim.bits[i];
  o.flags = src->flags;
  const int rc = ffp_create(src->device, &o, out);
  if (rc != FFP_SUCCESS) return rc;
  (*out)->tile_auto = src->tile_auto;
  (*out)->tile_k = src->tile_k;
  (*out)->blocks_per_cu = src->blocks_per_cu;
  (*out)->block_kib = src->block_kib;
  return FFP_SUCCESS;
}

int ctx_capture_batch(ffp_ctx* ctx, ffp_job* d_jobs, uint32_t njobs, uint64_t max_total_bytes,
                      hipGraph_t* graph, hipGraphExec_t* exec) {
  DeviceGuard g(ctx->device);
  *graph = nullptr;
  *exec = nullptr;
  hipStream_t cs = nullptr;
  if (hipStreamCreate(&cs) != hipSuccess) return FFP_E_HIP;
  int rc = FFP_SUCCESS;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    rc = FFP_E_HIP;
  } else {
    const int lrc = batch_common(ctx, d_jobs, njobs, max_total_bytes, cs);
    const hipError_t ec = hipStreamEndCapture(cs, graph);
    if (lrc != FFP_SUCCESS) rc = lrc;
    else if (ec != hipSuccess) rc = FFP_E_HIP;
    else if (hipGraphInstantiate(exec, *graph, nullptr, nullptr, 0) != hipSuccess) rc = FFP_E_HIP;
  }
  (void)hipStreamDestroy(cs);
  if (rc != FFP_SUCCESS) {
    if (*exec) (void)hipGraphExecDestroy(*exec);
    if (*graph) (void)hipGraphDestroy(*graph);
    *graph = nullptr;
    *exec = nullptr;
  }
  return rc;
}

uint64_t ctx_scratch_bytes(const ffp_ctx* ctx) {
  return ctx->block_cap * sizeof(uint64_t) + ctx->queue_cap * sizeof(QueueEntry) +
         ctx->jobs_cap * sizeof(JobDesc) + sizeof(DeviceState);
}

}  // namespace ffp

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
    case FFP_E_SIZE: return "input larger than the fixed scratch of ffp_parse_f64_noalloc allows";
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
  if (o.flags & ~(FFP_REJECT_PLUS | FFP_JSON | FFP_INFNAN | FFP_HEX | FFP_ROUND_MASK |
                  FFP_JSON_DOCUMENT | FFP_CSV))
    return FFP_E_ARG;
  if (o.flags & FFP_CSV) {
    // CSV: ',' and '\n' separate fields and rows; hexadecimal tokens,
    // directed rounding and JSON documents do not combine with it
    if (o.flags & (FFP_HEX | FFP_ROUND_MASK | FFP_JSON_DOCUMENT)) return FFP_E_ARG;
    if (!((o.delim_set[0] >> ',') & 1) || !((o.delim_set[0] >> '\n') & 1)) return FFP_E_ARG;
  }
  if (o.flags & FFP_JSON_DOCUMENT) {
    // JSON text: the structural characters, whitespace and the quote delimit
    // the number tokens; the JSON number grammar applies
    o.flags |= FFP_JSON;
    for (int i = 0; i < 4; ++i) o.delim_set[i] = 0;
    for (const char* c = "[]{},: \t\r\n\""; *c; ++c)
      o.delim_set[(unsigned char)*c >> 6] |= 1ull << ((unsigned char)*c & 63);
  }
  int members = 0, first = -1;
  for (int c = 0; c < 256; ++c) {
    if ((o.delim_set[c >> 6] >> (c & 63)) & 1) {
      if (is_grammar_byte(c, o.flags)) return FFP_E_ARG;
      if (first < 0) first = c;
      ++members;
    }
  }
  if (members == 0) return FFP_E_ARG;

  ffp_ctx* ctx = new (std::nothrow) ffp_ctx();
  if (!ctx) return FFP_E_NOMEM;
  ctx->device = hip_device;
  for (int i = 0; i < 4; ++i) ctx->delim.bits[i] = o.delim_set[i];
  // the single-delimiter classification assumes a byte below 0x80; other
  // sets (and a lone byte at or above 0x80) use the 256-entry table
  ctx->delim.single = members == 1 && first < 0x80 ? 1u : 0u;
  ctx->delim.byte = (uint32_t)first;
  // sets of 2 to 4 bytes below 0x80: byte comparisons instead of a table
  ctx->delim.nfew = 0;
  if (members >= 2 && members <= 4) {
    uint32_t k = 0;
    bool low = true;
    for (int c = 0; c < 256; ++c) {
      if ((o.delim_set[c >> 6] >> (c & 63)) & 1) {
        low = low && c < 0x80;
        ctx->delim.few[k++] = (uint32_t)c * 0x01010101u;
      }
    }
    for (; k < 4; ++k) ctx->delim.few[k] = ctx->delim.few[0];
    if (low) ctx->delim.nfew = (uint32_t)members;
  }
  ctx->flags = o.flags;
  ctx->csv_columns = ~0ull;

  DeviceGuard g(hip_device);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) {
    delete ctx;
    return FFP_E_HIP;
  }
  ctx->num_cus = prop.multiProcessorCount;
  ctx->arch = prop.gcnArchName;
  for (int k : {1, 2, 4}) {
    int b = 0;
    if (ffp::parse_occupancy(k, ctx->delim.single != 0, false, &b) != hipSuccess || b < 1) b = 1;
    ctx->max_bpc[k] = b;
    int bw = 0;
    if (ffp::parse_occupancy(k, ctx->delim.single != 0, true, &bw) != hipSuccess || bw < 1) bw = 1;
    ctx->max_bpc_wide[k] = bw < b ? bw : b;
  }
  if (const char* k = getenv("FFP_TILE_K")) {
    const int v = atoi(k);
    if (v == 1 || v == 2 || v == 4) {
      ctx->tile_k = v;
      ctx->tile_auto = false;
    }
  }
  ctx->blocks_per_cu = ctx->max_bpc[ctx->tile_k];
  ctx->fb_grid = ctx->num_cus * 6;  // six workgroups of four waves per CU: six waves per SIMD
  // the main state and the two spares, all clean
  if (hipMalloc(&ctx->d_state, 3 * sizeof(DeviceState)) != hipSuccess) {
    delete ctx;
    return FFP_E_NOMEM;
  }
  ctx->d_spare = ctx->d_state + 1;
  ctx->last_state = ctx->d_state;
  if (hipMemset(ctx->d_state, 0, 3 * sizeof(DeviceState)) != hipSuccess ||
      grow(ctx, 1 << 20, 1) != FFP_SUCCESS) {
    ffp_destroy(ctx);
    return FFP_E_NOMEM;
  }
  // the fixed scratch of ffp_parse_f64_noalloc: its address on this device
  // (looked up once per device, with the device current)
  void* fixed = nullptr;
  if (ffp::noalloc_scratch(hip_device, &fixed) != hipSuccess) {
    ffp_destroy(ctx);
    return FFP_E_HIP;
  }
  ctx->d_fixed = static_cast<unsigned char*>(fixed);
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
    if (ctx->d_jobs) (void)hipFree(ctx->d_jobs);
    if (ctx->d_state) (void)hipFree(ctx->d_state);
  }
  delete ctx;
}

int ffp_reserve(ffp_ctx* ctx, uint64_t max_nbytes) {
  if (!ctx || max_nbytes >= ffp::kMaxBytes) return FFP_E_ARG;
  DeviceGuard g(ctx->device);
  return grow(ctx, max_nbytes, 1);
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

int ffp_parse_f64_noalloc(ffp_ctx* ctx, const uint8_t* d_text, uint64_t nbytes,
                          double* d_values, uint8_t* d_status, uint64_t capacity,
                          uint64_t* d_count, void* stream) {
  return parse_common(ctx, ffp::kF64, d_text, nbytes, d_values, d_status, capacity, d_count,
                      stream, nullptr, true);
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

int ffp_parse_f16(ffp_ctx* ctx, const uint8_t* d_text, uint64_t nbytes, uint16_t* d_values,
                  uint8_t* d_status, uint64_t capacity, uint64_t* d_count, void* stream) {
  return parse_common(ctx, ffp::kF16, d_text, nbytes, d_values, d_status, capacity, d_count,
                      stream);
}

int ffp_parse_bf16(ffp_ctx* ctx, const uint8_t* d_text, uint64_t nbytes, uint16_t* d_values,
                   uint8_t* d_status, uint64_t capacity, uint64_t* d_count, void* stream) {
  return parse_common(ctx, ffp::kBF16, d_text, nbytes, d_values, d_status, capacity, d_count,
                      stream);
}

int64_t ffp_parse_f16_sync(ffp_ctx* ctx, const uint8_t* d_text, uint64_t nbytes,
                           uint16_t* d_values, uint8_t* d_status, uint64_t capacity,
                           uint64_t* d_count, void* stream) {
  const int rc = parse_common(ctx, ffp::kF16, d_text, nbytes, d_values, d_status, capacity,
                              d_count, stream);
  return finish_sync(ctx, rc, capacity, d_count, stream);
}

int64_t ffp_parse_bf16_sync(ffp_ctx* ctx, const uint8_t* d_text, uint64_t nbytes,
                            uint16_t* d_values, uint8_t* d_status, uint64_t capacity,
                            uint64_t* d_count, void* stream) {
  const int rc = parse_common(ctx, ffp::kBF16, d_text, nbytes, d_values, d_status, capacity,
                              d_count, stream);
  return finish_sync(ctx, rc, capacity, d_count, stream);
}

int ffp_parse_batch(ffp_ctx* ctx, ffp_job* d_jobs, uint32_t njobs, uint64_t max_total_bytes,
                    void* stream) {
  return batch_common(ctx, d_jobs, njobs, max_total_bytes, (hipStream_t)stream);
}

int ffp_batch_graph_create(ffp_ctx* ctx, ffp_job* d_jobs, uint32_t njobs,
                           uint64_t max_total_bytes, ffp_graph** out) {
  if (!ctx || !out) return FFP_E_ARG;
  *out = nullptr;
  if (!d_jobs || njobs == 0 || njobs > kMaxJobs || max_total_bytes >= kMaxBatchBytes)
    return FFP_E_ARG;
  ffp_graph* gr = new (std::nothrow) ffp_graph();
  if (!gr) return FFP_E_NOMEM;
  // a private context with the same options and schedule
  int rc = ffp::ctx_clone(ctx, &gr->own);
  if (rc != FFP_SUCCESS) {
    delete gr;
    return rc;
  }
  DeviceGuard g(ctx->device);
  rc = grow(gr->own, max_total_bytes, njobs < 2 ? 2 : njobs);
  if (rc == FFP_SUCCESS)
    rc = ffp::ctx_capture_batch(gr->own, d_jobs, njobs, max_total_bytes, &gr->graph, &gr->exec);
  if (rc != FFP_SUCCESS) {
    ffp_batch_graph_destroy(gr);
    return rc;
  }
  *out = gr;
  return FFP_SUCCESS;
}

int ffp_batch_graph_launch(ffp_graph* gr, void* stream) {
  if (!gr || !gr->exec) return FFP_E_ARG;
  DeviceGuard g(gr->own->device);
  return hipGraphLaunch(gr->exec, (hipStream_t)stream) == hipSuccess ? FFP_SUCCESS : FFP_E_HIP;
}

void ffp_batch_graph_destroy(ffp_graph* gr) {
  if (!gr) return;
  if (gr->own) {
    DeviceGuard g(gr->own->device);
    (void)hipDeviceSynchronize();
    if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
    if (gr->graph) (void)hipGraphDestroy(gr->graph);
    ffp_destroy(gr->own);
  }
  delete gr;
}

int ffp_get_tuning(ffp_ctx* ctx, ffp_tuning* out) {
  if (!ctx || !out) return FFP_E_ARG;
  memset(out, 0, sizeof *out);
  out->tile_k = ctx->tile_auto ? auto_tile_k(ctx) : ctx->tile_k;
  out->blocks_per_cu = ctx->tile_auto ? ctx->max_bpc[out->tile_k] : ctx->blocks_per_cu;
  out->block_kib = ctx->block_kib;
  return FFP_SUCCESS;
}

int ffp_set_tuning(ffp_ctx* ctx, const ffp_tuning* t) {
  if (!ctx || !t) return FFP_E_ARG;
  if (t->tile_k != 1 && t->tile_k != 2 && t->tile_k != 4) return FFP_E_ARG;
  if (t->blocks_per_cu < 0 || t->blocks_per_cu > ctx->max_bpc[t->tile_k]) return FFP_E_ARG;
  if (t->block_kib != 0 && t->block_kib != 4 && t->block_kib != 16 && t->block_kib != 64)
    return FFP_E_ARG;
  ctx->block_kib = t->block_kib;
  ctx->tile_auto = false;
  ctx->tile_k = t->tile_k;
  ctx->blocks_per_cu = t->blocks_per_cu == 0 ? ctx->max_bpc[t->tile_k] : t->blocks_per_cu;
  return FFP_SUCCESS;
}

int ffp_autotune_batch(ffp_ctx* ctx, ffp_job* d_jobs, uint32_t njobs, uint64_t max_total_bytes,
                       void* stream, ffp_tuning* out) {
  if (!ctx || !d_jobs || !out) return FFP_E_ARG;
  DeviceGuard g(ctx->device);
  const char* cache_path = getenv("FFP_TUNE_CACHE");
  const std::string key = tune_key(ctx, njobs, max_total_bytes);
  std::map<std::string, std::pair<int, int>> cache;
  if (cache_path) {
    cache = read_cache(cache_path);
    auto it = cache.find(key);
    if (it != cache.end()) {
      ffp_tuning t{};
      t.tile_k = it->second.first;
      t.blocks_per_cu = it->second.second;
      if (ffp_set_tuning(ctx, &t) == FFP_SUCCESS) return ffp_get_tuning(ctx, out);
    }
  }
  const hipStream_t s = (hipStream_t)stream;
  const bool was_timing = ctx->timing;
  // drop pending measurements of the caller
  double ms0 = 0;
  uint64_t n0 = 0;
  if (was_timing && ffp_timing_read(ctx, &ms0, &n0) != FFP_SUCCESS) return FFP_E_HIP;
  ctx->timing = true;
  double best = 1e30;
  const bool was_auto = ctx->tile_auto;
  const int was_k = ctx->tile_k, was_b = ctx->blocks_per_cu;
  int best_k = ctx->tile_k, best_b = ctx->blocks_per_cu;
  ctx->tile_auto = false;  // the candidates below are fixed schedules
  for (int k : {1, 2, 4}) {
    std::vector<int> cands;
    for (int b = ctx->max_bpc[k]; b >= 1; b = (b > 2 ? b - 1 : b - 1)) cands.push_back(b);
    for (int b : cands) {
      ctx->tile_k = k;
      ctx->blocks_per_cu = b;
      int rc = batch_common(ctx, d_jobs, njobs, max_total_bytes, s);  // warm-up
      double ms = 0;
      uint64_t n = 0;
      if (rc == FFP_SUCCESS) rc = ffp_timing_read(ctx, &ms, &n);
      double t_best = 1e30;
      for (int rep = 0; rep < 3 && rc == FFP_SUCCESS; ++rep) {
        rc = batch_common(ctx, d_jobs, njobs, max_total_bytes, s);
        if (rc == FFP_SUCCESS) rc = ffp_timing_read(ctx, &ms, &n);
        if (rc == FFP_SUCCESS && n > 0 && ms < t_best) t_best = ms;
      }
      if (rc != FFP_SUCCESS) {
        ctx->timing = was_timing;
        ctx->tile_auto = was_auto;
        ctx->tile_k = was_k;
        ctx->blocks_per_cu = was_b;
        return rc;
      }
      if (t_best < best) {
        best = t_best;
        best_k = k;
        best_b = b;
      }
    }
  }
  ctx->timing = was_timing;
  ctx->tile_auto = false;
  ctx->tile_k = best_k;
  ctx->blocks_per_cu = best_b;
  if (cache_path) {
    cache[key] = {best_k, best_b};
    write_cache(cache_path, cache);
  }
  return ffp_get_tuning(ctx, out);
}

int ffp_last_device_error(ffp_ctx* ctx) {
  if (!ctx) return FFP_E_ARG;
  DeviceGuard g(ctx->device);
  unsigned err = 0;
  if (hipMemcpy(&err, &ctx->last_state->error, sizeof(err), hipMemcpyDeviceToHost) != hipSuccess)
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

int ffp_set_reduce(ffp_ctx* ctx, uint64_t* d_out) {
  if (!ctx) return FFP_E_ARG;
  ctx->reduce_out = d_out;
  return FFP_SUCCESS;
}

int ffp_set_csv_columns(ffp_ctx* ctx, uint64_t columns) {
  if (!ctx) return FFP_E_ARG;
  ctx->csv_columns = columns;
  return FFP_SUCCESS;
}

int ffp_set_reduce_sum(ffp_ctx* ctx, uint64_t* d_sum) {
  if (!ctx) return FFP_E_ARG;
  ctx->sum_out = d_sum;
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
