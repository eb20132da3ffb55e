// Shared host/device definitions of the parsing library (not part of the
// public C-ABI; see include/ffp.h for that).
#pragma once

#include <stdint.h>

namespace ffp {

// Parse kernel geometry: 256 threads per workgroup (4 wave64s), each thread
// loads 16-byte chunks; a tile is kThreads * 16 * K bytes.
constexpr int kThreads = 256;
constexpr int kChunk = 16;
constexpr int kWave = 64;

// Internal per-token status for tokens whose exact value is still being
// decided by the fallback kernel; never visible after a completed call.
constexpr uint8_t kPending = 3;

// The text of a job is cut into blocks of 2^block_shift bytes (4, 16 or
// 64 KiB, chosen per call; counted from the 16-byte boundary at or below the
// job's first byte).  The count kernel gives the number of tokens starting in
// each block, a scan turns those into the index of each block's first token,
// and the parse kernel walks a block in tiles of kThreads * kChunk * K bytes.
constexpr int kMinBlockShift = 12;
constexpr int kMaxBlockShift = 16;

// Significant decimal digits kept by the exact fallback.  Any midpoint
// between neighbouring binary64 values needs at most 768 significant digits
// (Section 11), so 769 digits plus a sticky digit decide every comparison.
constexpr int kFallbackDigits = 769;

// Maximum buffer size accepted (keeps saturated exponents exact, see the
// lexer).
constexpr uint64_t kMaxBytes = 1ull << 47;

// Queue entries reserved for the rare inconclusive-product case of
// Algorithm 1 on top of the provable bound for long tokens.
constexpr uint64_t kAbortReserve = 65536;

// Fixed scratch of the entry point that allocates nothing
// (ffp_parse_f64_noalloc): texts of up to kNoAllocMaxBytes; the device
// state, the per-block counts and the fallback queue sized as a regular call
// on such a text sizes them (one job, blocks of at least 4 KiB).
constexpr uint64_t kNoAllocMaxBytes = 8ull << 20;
constexpr uint64_t kNoAllocBlocks = ((kNoAllocMaxBytes + 15) >> kMinBlockShift) + 3;
constexpr uint64_t kNoAllocQueue = (kNoAllocMaxBytes + 1) / 21 + kAbortReserve;
constexpr uint64_t kNoAllocStateOff = 0;
constexpr uint64_t kNoAllocBlockOff = 2048;
constexpr uint64_t kNoAllocQueueOff = kNoAllocBlockOff + ((kNoAllocBlocks * 8 + 255) & ~255ull);
constexpr uint64_t kNoAllocScratchBytes = kNoAllocQueueOff + kNoAllocQueue * 16;

enum DType : uint32_t { kF64 = 0, kF32 = 1, kF16 = 2, kBF16 = 3 };

enum DevError : uint32_t { kDevOk = 0, kDevQueue = 1, kDevInternal = 2 };

// Path counters (same categories as the code-path table of the paper's
// experiments).
enum Counter : int {
  kCntTokens = 0,
  kCntInvalid = 1,
  kCntEarly = 2,
  kCntOne = 3,
  kCntTwo = 4,
  kCntFallback = 5,
  kNumCounters = 6
};

struct JobDesc {
  const uint8_t* text;
  uint64_t nbytes;
  void* values;
  uint8_t* status;
  uint64_t capacity;
  uint64_t* count_out;
  int32_t* err_out;      // batched calls: the job record's err field
  uint64_t block_begin;  // index of this job's first block in the block space
  uint32_t dtype;
  uint32_t job_id;
};

struct QueueEntry {
  uint64_t offset;     // byte offset of the token's first byte in its job
  uint64_t index_job;  // token index | (job id << 48)
};

// Exact sum of the values (ffp_set_reduce_sum): every value of the four
// output formats is an integer multiple of 2^-1074, below 2^1024 in
// magnitude.  The magnitudes of the positive and of the negative values are
// accumulated apart, as fixed-point numbers in units of 2^-1074, in limbs of
// 32 bits held in 64-bit words: additions put pieces below 2^32 into the
// words and the carries they collect in the upper halves are resolved once,
// at the end.  Limbs 0..65 receive the pieces of single values (a 53-bit
// significand shifted by up to 2046 bits spans three limbs), the rest takes
// the carries.
constexpr int kSumLimbs = 68;
// sum_flags bits: a +inf / -inf was summed, a value other than -0 was
// summed, some value was summed
constexpr uint32_t kSumPosInf = 1, kSumNegInf = 2, kSumNotNegZero = 4, kSumAny = 8;

struct DeviceState {
  unsigned int error;
  unsigned int pad;
  unsigned long long queue_tail;
  unsigned long long total_blocks;  // batched calls: blocks of all jobs
  unsigned long long counters[8];
  // min / max of the order keys of the values and their count (reduction)
  unsigned long long red_min, red_max, red_count;
  // exact sum: accumulators of the positive ([0]) and negative ([1]) values
  unsigned long long sum_acc[2][kSumLimbs];
  unsigned int sum_flags;
  // set by the scan kernel when a block of the call holds more token starts
  // than ScanParams::dense_limit (then the 16 KiB plain parse runs with the
  // full start list)
  unsigned int dense;
};

static_assert(sizeof(DeviceState) <= kNoAllocBlockOff, "device state fits its scratch slot");
static_assert(sizeof(QueueEntry) == 16, "queue entry size");

struct DelimSet {
  uint64_t bits[4];
  uint32_t single;     // 1 if the set holds exactly one byte, below 0x80
  uint32_t byte;       // that byte (or any member, used as padding)
  // Sets of 2 to 4 bytes, all below 0x80: their members repeated in the four
  // bytes of a word (unused slots repeat the first), classified by byte
  // comparisons instead of table lookups; nfew = 0 for other sets.
  uint32_t nfew;
  uint32_t few[4];
};

// Jobs: either one job passed by value (plain calls) or a device table
// sorted by block_begin (batched calls).
struct JobSet {
  JobDesc single;
  const JobDesc* jobs;      // null for plain calls
  uint32_t njobs;
  uint32_t block_shift;
  uint64_t total_blocks;             // plain calls
  const uint64_t* total_blocks_dev;  // batched calls
};

// Public job record (include/ffp.h, struct ffp_job), as the kernels see it.
struct UserJob {
  const uint8_t* text;
  uint64_t nbytes;
  void* values;
  uint8_t* status;
  uint64_t capacity;
  uint64_t count;
  int32_t dtype;
  int32_t err;
};

struct PrepParams {
  UserJob* user;
  uint32_t njobs;
  uint32_t block_shift;
  JobDesc* jobs;
  DeviceState* st;
  uint64_t block_cap;  // blocks the scratch can hold
  uint64_t max_bytes;  // the caller's bound on the sum of nbytes
};

struct CountParams {
  JobSet js;
  uint64_t* block_sum;  // per block: tokens starting in it
  DelimSet delim;
  DeviceState* st;      // reset here when the call runs without the scan kernel
  DeviceState* spare;   // with reset_state: the context's two spare states (or null)
  uint32_t reset_state;
  uint32_t json_doc;    // FFP_JSON_DOCUMENT: counts for both entry states
  uint32_t csv;         // FFP_CSV: only tokens of the selected columns count
  uint64_t csv_columns; // FFP_CSV: bit c selects column c (c < 64)
};

// JSON documents: a block's count word holds the tokens starting in it when
// it begins outside a string (bits 0-31) and inside one (bits 32-62), and
// the parity of its unescaped quotes (bit 63); after the scan, the prefix
// (bits 0-62) and whether the block begins inside a string (bit 63).
constexpr uint64_t kPrefixMask = ~0ull >> 1;

// The plain 16 KiB-tile parse keeps at most this many token starts per tile.
// Calls with 64 KiB blocks that run the scan kernel: the count word of a
// block carries kDenseTileBit when one of its four 16 KiB tiles holds more
// (the scan kernel then sets DeviceState::dense and masks the bit off).
constexpr uint32_t kShortTileStarts = 4096;
constexpr uint64_t kDenseTileBit = 1ull << 62;

struct ScanParams {
  JobSet js;
  uint64_t* block_sum;  // in: counts; out: exclusive prefix over all blocks
  DeviceState* st;
  DeviceState* spare;   // the context's two spare states, reset here (or null)
  uint32_t json_doc;    // count words of JSON documents (see kPrefixMask)
  uint32_t dense_limit; // DeviceState::dense: block counts above this (0: never),
                        // or a count word with kDenseTileBit
};

struct ParseParams {
  JobSet js;
  const uint64_t* block_prefix;
  DeviceState* st;
  QueueEntry* queue;
  uint64_t queue_cap;
  DelimSet delim;
  uint32_t flags;           // FFP_REJECT_PLUS ...
  uint32_t count_paths;
  uint64_t* reduce_out;     // plain calls: min, max, count of the values (or null)
  uint64_t* sum_out;        // plain calls: exact sum of the values (or null)
  // Small calls (4 KiB tiles) run without the scan kernel: block_prefix
  // then holds each block's own token count, every workgroup sums the counts
  // of its job's earlier blocks, and the workgroup of a job's last block
  // writes the job's count (and the capacity error).
  uint32_t sum_in_parse;
  // The smallest plain calls run without the count kernel too: each
  // workgroup counts the tokens before its block from the text itself, and
  // st is one of the context's two spare states, clean when the call starts;
  // the call resets the other one (other_st) for the next such call.
  uint32_t self_count;
  DeviceState* other_st;
  uint64_t csv_columns;  // FFP_CSV: bit c selects column c (c < 64)
  // Small calls (4 KiB blocks, no reduction) decide their queued tokens in
  // the parse kernel: block b queues into entries [b * kLocalQueueSeg,
  // (b + 1) * kLocalQueueSeg) of the queue, and the workgroup that parsed
  // the block runs the exact fallback on them (no fallback kernel).
  uint32_t fb_local;
};

// Queue entries per 4 KiB block when a block's workgroup decides its own
// queued tokens: a token starts at a byte whose predecessor is a delimiter,
// so a block holds at most half its bytes in token starts.
constexpr uint64_t kLocalQueueSeg = (1u << kMinBlockShift) / 2;

struct FallbackParams {
  JobSet js;
  const QueueEntry* queue;
  uint64_t queue_cap;
  DeviceState* st;
  DelimSet delim;
  uint64_t* reduce_out;  // as in ParseParams
  uint64_t* sum_out;     // as in ParseParams
  uint32_t flags;        // as in ParseParams (the rounding direction)
};

}  // namespace ffp
