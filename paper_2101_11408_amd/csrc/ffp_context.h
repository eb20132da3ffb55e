// Definition of the parsing context shared by the C-ABI and the server
// (internal; the public handle is opaque).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <utility>
#include <vector>

#include "ffp.h"
#include "ffp_internal.h"

using ffp::DelimSet;
using ffp::DeviceState;
using ffp::JobDesc;
using ffp::QueueEntry;

struct ffp_ctx {
  int device = 0;
  DelimSet delim{};
  uint32_t flags = 0;
  int num_cus = 0;
  std::string arch;
  int tile_k = 4;
  bool tile_auto = true;         // tile_k chosen per call (see call_shape)
  int blocks_per_cu = 1;        // chosen schedule
  int block_kib = 0;            // 0: chosen per call from its size
  int max_bpc[5] = {0, 0, 0, 0, 0};  // occupancy limit per tile_k (plain instance)
  int max_bpc_wide[5] = {0, 0, 0, 0, 0};  // the same for the other instances
  int fb_grid = 0;

  uint64_t* d_block_sum = nullptr;  // per-block counts, then their prefix
  uint64_t block_cap = 0;
  QueueEntry* d_queue = nullptr;
  uint64_t queue_cap = 0;
  JobDesc* d_jobs = nullptr;  // internal job table of batched calls
  uint64_t jobs_cap = 0;
  DeviceState* d_state = nullptr;
  // two more states for the calls that run without the count kernel, used
  // in turn (d_state + 1 and d_state + 2; one allocation)
  DeviceState* d_spare = nullptr;
  int spare_sel = 0;
  // the fixed scratch of ffp_parse_f64_noalloc on this context's device
  unsigned char* d_fixed = nullptr;
  // device state of the last call (d_state, or the fixed scratch's)
  DeviceState* last_state = nullptr;

  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used, ev_free;
  double timed_ms = 0.0;
  uint64_t timed_launches = 0;

  bool counters = false;
  uint64_t* reduce_out = nullptr;  // plain calls: min, max, count of the values
  uint64_t* sum_out = nullptr;     // plain calls: exact sum of the values
  uint64_t csv_columns = ~0ull;    // FFP_CSV: the selected columns
};

struct ffp_graph {
  ffp_ctx* own = nullptr;  // private context: the graph holds its scratch
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace ffp {

// Grow the scratch of ctx for up to `bytes` of text over `njobs` jobs.
int ctx_grow(ffp_ctx* ctx, uint64_t bytes, uint64_t njobs);

// Stream-ordered plain parse of one buffer (the body of ffp_parse_f64/f32).
// d_err (or null) receives the error codes a batched job record would get
// (capacity exceeded, fallback queue overflow).
int ctx_parse(ffp_ctx* ctx, uint32_t dtype, const uint8_t* d_text, uint64_t nbytes,
              void* d_values, uint8_t* d_status, uint64_t capacity, uint64_t* d_count,
              hipStream_t s, int32_t* d_err = nullptr);

// Stream-ordered batched parse (the body of ffp_parse_batch).
int ctx_batch(ffp_ctx* ctx, ffp_job* d_jobs, uint32_t njobs, uint64_t max_total_bytes,
              hipStream_t s);

// A new context with the options and schedule of `src`.
int ctx_clone(const ffp_ctx* src, ffp_ctx** out);

// Capture ctx_batch(ctx, d_jobs, njobs, max_total_bytes) into an
// instantiated graph; ctx's scratch must already fit the batch.
int ctx_capture_batch(ffp_ctx* ctx, ffp_job* d_jobs, uint32_t njobs, uint64_t max_total_bytes,
                      hipGraph_t* graph, hipGraphExec_t* exec);

// Bytes of device scratch held by ctx.
uint64_t ctx_scratch_bytes(const ffp_ctx* ctx);

}  // namespace ffp
