/*
 * ffp.h -- exact decimal -> IEEE-754 binary64 / binary32 parsing on AMD
 * Instinct MI355X (gfx950).
 *
 * The library turns a buffer of delimiter-separated ASCII decimal numbers into
 * the nearest binary64 or binary32 values, ties rounded to even, following
 * Lemire, "Number Parsing at a Gigabyte per Second" (Software: Practice and
 * Experience, 2021):
 *   - strings are explicitly delimited and nothing outside [text, text+nbytes)
 *     is ever read (Section 4);
 *   - up to 19 significant digits go into a 64-bit significand w with a
 *     decimal exponent q (Sections 4 and 11);
 *   - w * 10^q is converted with one or two 64x64->128-bit products against a
 *     128-bit power-of-five table (Algorithm 1, Sections 5 to 10);
 *   - longer numbers try the truncated w and w+1 (Section 11), and whatever
 *     those cannot decide goes to an exact big-integer fallback on the GPU;
 *   - the result is the correctly rounded value in every case.
 *
 * All entry points use plain C types.  Device pointers come from hipMalloc
 * (for instance torch tensors on a ROCm device); `stream` is a hipStream_t
 * (NULL = the default stream).  No entry point throws; every one returns an
 * ffp_error code.  Calls that take a stream are asynchronous and
 * stream-ordered unless their name ends in _sync.
 */
#ifndef FFP_H
#define FFP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------------------
 * Per-token status, one byte per token in the caller's status array.  The
 * paper leaves error reporting to the application (Section 4: a parser may
 * fail on a malformed number); this is the library's contract.  Overflow and
 * underflow follow Algorithm 1's early exits (Section 5: q > 308 is
 * infinite, q < -342 is zero) and its subnormal branch (Section 9.3).
 * ------------------------------------------------------------------------- */
enum ffp_token_status {
    /* The correctly rounded value.  A zero significand gives a signed zero,
     * "-0" gives -0.0, subnormal results are FFP_OK. */
    FFP_OK = 0,
    /* The token does not match the grammar below.  The value is the canonical
     * quiet NaN: 0x7FF8000000000000 (binary64) or 0x7FC00000 (binary32). */
    FFP_INVALID = 1,
    /* A nonzero decimal whose rounded value is +-infinity (overflow) or +-0
     * (total underflow).  The value is that infinity or zero. */
    FFP_OUT_OF_RANGE = 2
};

/* ---------------------------------------------------------------------------
 * Error codes returned by the entry points.
 * ------------------------------------------------------------------------- */
enum ffp_error {
    FFP_SUCCESS = 0,
    FFP_E_ARG = -1,       /* invalid argument (null pointer, bad option, ...) */
    FFP_E_CAPACITY = -2,  /* more tokens than the caller's capacity (_sync) */
    FFP_E_HIP = -3,       /* a HIP runtime call failed */
    FFP_E_NOMEM = -4,     /* device scratch could not be allocated */
    FFP_E_BUDGET = -5,    /* request does not fit the server's HBM budget */
    FFP_E_BUSY = -6,      /* server has no free slot (non-blocking submit) */
    FFP_E_QUEUE = -7,     /* fallback queue overflowed; result incomplete */
    FFP_E_INTERNAL = -8,  /* internal consistency check failed */
    FFP_E_SIZE = -9       /* input larger than ffp_parse_f64_noalloc accepts */
};

/* Reject a leading '+' sign, as JSON does (Section 4). */
#define FFP_REJECT_PLUS 1u
/* JSON numbers: the number grammar of the JSON specification, i.e. the
 * grammar below without '+', without leading zeros ("01") and with digits on
 * both sides of a '.' (".5" and "1." are rejected).  With delimiters such as
 * "[],: \n" the numbers of a JSON document of arrays (the paper's canada
 * test file, Section 12) are its tokens; other tokens come back invalid. */
#define FFP_JSON 2u
/* Accept inf, infinity and nan in any letter case with an optional sign:
 * +-infinity (status FFP_OK) and the canonical quiet NaN with the token's
 * sign (status FFP_OK). */
#define FFP_INFNAN 4u
/* Also accept hexadecimal floating-point tokens (Appendix C):
 * [+-]? 0[xX] ( H+ ('.' H*)? | '.' H+ ) ( [pP] [+-]? D+ )?   H = [0-9a-fA-F],
 * value = hexadecimal significand * 16^-(nibbles after the point) * 2^exponent,
 * rounded in the context's rounding direction (exact; no table, no
 * fallback). */
#define FFP_HEX 8u
/* JSON documents (a structural index of the numbers of a JSON text, the
 * paper's canada file being one, Section 12): the buffer is JSON text; bytes
 * inside strings are skipped, a quote preceded by an odd number of
 * consecutive backslashes is escaped (it neither opens nor closes a string),
 * and the tokens are the runs outside strings of bytes other than the
 * structural characters [ ] { } , : whitespace (space, tab, CR, LF) and
 * unescaped quotes that start with '-' or a digit -- the number literals, in
 * document order (keys, strings, true, false and null get no index).  Each is
 * read with the JSON number grammar (FFP_JSON is implied).  The context's
 * delimiter set is replaced by the structural characters, whitespace and the
 * quote.  Plain calls only: batched calls and servers on such a context
 * return FFP_E_ARG. */
#define FFP_JSON_DOCUMENT 0x40u
/* CSV number columns (structural parsing of a table, named as future work
 * in Section 13): the buffer is a table whose rows end at '\n' and whose
 * fields are separated by ','; a token's column is the number of ',' bytes
 * between the last '\n' before it (or the buffer's start) and the token.
 * Tokens are the runs of non-delimiter bytes as usual (the delimiter set
 * must contain ',' and '\n'; other members, such as ' ' or '\r', delimit
 * tokens without starting a field or a row), and only the tokens of the
 * columns selected by ffp_set_csv_columns get indices, in buffer order; the
 * other flags' grammar applies to them.  Fields are not quoted.  Does not
 * combine with FFP_HEX, a directed rounding mode or FFP_JSON_DOCUMENT
 * (FFP_E_ARG).  Plain calls only: batched calls and servers on such a
 * context return FFP_E_ARG. */
#define FFP_CSV 0x80u
/* Rounding direction, a two-bit field of the flags (IEEE 754 rounding-
 * direction attributes; the paper rounds to nearest and notes that its
 * method extends to the other modes, footnote of Section 6).  0 selects
 * round to nearest, ties to even.  Under a directed mode the result is the
 * representable value next to the token's exact value on the mode's side
 * (the value itself when representable).  Overflow (the magnitude, rounded
 * with an unbounded exponent, exceeds the largest finite value) gives the
 * largest finite value when the mode truncates the magnitude (toward zero;
 * toward -inf for positive values; toward +inf for negative ones) and
 * infinity otherwise, status FFP_OUT_OF_RANGE either way.  A nonzero value
 * below the smallest subnormal gives a signed zero (FFP_OUT_OF_RANGE) when
 * truncating and the smallest subnormal (FFP_OK) otherwise. */
#define FFP_ROUND_MASK 0x30u
#define FFP_ROUND_NEAREST 0x00u
#define FFP_ROUND_TOWARD_ZERO 0x10u
#define FFP_ROUND_UP 0x20u   /* toward +infinity */
#define FFP_ROUND_DOWN 0x30u /* toward -infinity */

/* ---------------------------------------------------------------------------
 * Options.  delim_set is a 256-bit set of delimiter bytes: byte c is a
 * delimiter when bit (c & 63) of delim_set[c >> 6] is set.  It must be
 * non-empty and must not contain any byte of the grammar the flags select:
 * 0-9 . e E + - always, a-f A-F x X p P with FFP_HEX, and the letters of
 * inf, infinity and nan in either case (a f i n t y A F I N T Y) with
 * FFP_INFNAN (FFP_E_ARG otherwise).  Passing NULL for the options selects
 * {'\n'} and flags 0.
 * ------------------------------------------------------------------------- */
typedef struct ffp_options {
    uint64_t delim_set[4];
    uint32_t flags;
    uint32_t reserved;
} ffp_options;

typedef struct ffp_ctx ffp_ctx;

/* ---------------------------------------------------------------------------
 * Tokens and grammar.
 *
 * Tokens are the maximal non-empty runs of non-delimiter bytes, in buffer
 * order; empty runs between delimiters are skipped.  Token i gets values[i]
 * and status[i].  A token is accepted when the whole run matches
 *
 *     [+-]? ( D+ ('.' D*)? | '.' D+ ) ( [eE] [+-]? D+ )?       D = [0-9]
 *
 * over ASCII (Section 4 leaves the grammar to the application; this is the
 * strict from_chars-like choice: no blanks, no inf/nan, no hexadecimal, an
 * exponent marker must be followed by digits).
 * ------------------------------------------------------------------------- */

/* Create a context on HIP device `hip_device`.  The context owns the device
 * scratch (per-block token counts, the fallback queue, the job table of
 * batched calls), its launch schedule and timing events; the 10,416-byte
 * power-of-five table (Appendix B) lives in the library's device image.  Returns FFP_E_ARG for a bad option set,
 * FFP_E_HIP / FFP_E_NOMEM on runtime failures.  *out is NULL on failure. */
int ffp_create(int hip_device, const ffp_options* opts, ffp_ctx** out);

/* Destroy a context; waits for its outstanding work.  NULL is a no-op. */
void ffp_destroy(ffp_ctx* ctx);

/* Human-readable text for an ffp_error code (static storage). */
const char* ffp_strerror(int err);

/* Grow the context's device scratch so that later calls on buffers of up to
 * max_nbytes bytes allocate nothing.  Calls on larger buffers grow the scratch
 * themselves (a hipMalloc outside any kernel).  Returns FFP_E_NOMEM on
 * failure. */
int ffp_reserve(ffp_ctx* ctx, uint64_t max_nbytes);

/* ---------------------------------------------------------------------------
 * Plain parse: one buffer, one stream-ordered launch sequence.
 *
 * Each token (a maximal run of non-delimiter bytes) is read with the grammar
 * of Section 4 (sign, digits with an optional point, optional exponent) and
 * converted as Sections 5-10 describe: the first 19 significant digits w
 * and the decimal exponent q, Algorithm 1 with the 128-bit table entry for
 * q (Section 5, Appendix B), the second product when the first one cannot
 * decide (Sections 7-9), the tie and subnormal rules (Sections 6 and 9)
 * and the binary exponent of Section 10; longer significands are decided
 * from w and w+1 or, when those disagree, by an exact comparison with the
 * halfway points (Section 11).  The result is the nearest binary64
 * (binary32) value, ties to even (Section 2).
 *
 *   d_text    device pointer to nbytes bytes of text (read only; bytes
 *             outside [d_text, d_text+nbytes) are never read).  nbytes may
 *             be 0.  nbytes must be below 2^47.
 *   d_values  device array of `capacity` doubles (or floats) -- written for
 *             tokens 0 .. min(count, capacity)-1 only.
 *   d_status  device array of `capacity` bytes (ffp_token_status).
 *   d_count   device pointer to one uint64_t: receives the true number of
 *             tokens, which may exceed capacity.
 *   stream    hipStream_t; the work is queued and the call returns.
 *
 * Returns FFP_SUCCESS when the work was queued, FFP_E_ARG for bad arguments
 * (null pointers with nonzero sizes, nbytes too large), FFP_E_NOMEM if the
 * scratch could not grow, FFP_E_HIP if a launch failed.  A context serves one
 * stream at a time: calls on one context must be ordered on one stream (or
 * synchronised by the caller); the context is not thread-safe.
 * ------------------------------------------------------------------------- */
int ffp_parse_f64(ffp_ctx* ctx, const uint8_t* d_text, uint64_t nbytes,
                  double* d_values, uint8_t* d_status, uint64_t capacity,
                  uint64_t* d_count, void* stream);
int ffp_parse_f32(ffp_ctx* ctx, const uint8_t* d_text, uint64_t nbytes,
                  float* d_values, uint8_t* d_status, uint64_t capacity,
                  uint64_t* d_count, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * parse as ffp_parse_f64, with the same arguments and results, that calls
 * no hipMalloc, hipFree or other allocating routine.  Its scratch (device
 * state, per-block token counts and the fallback queue, about 7.5 MB) is a
 * fixed array in the library's device image, one per GPU, held until the
 * process ends; its address is looked up once per device by ffp_create.
 * Texts of up to 8 MiB (8388608 bytes) are accepted; a larger nbytes returns
 * FFP_E_SIZE and queues nothing.  Every call on a GPU shares that GPU's
 * array (from any context or thread): calls whose work overlaps on one GPU
 * race and give wrong results, so order them on one stream or synchronise
 * between them.  The array keeps the last call's contents; each call resets
 * what must start at zero on the device, in stream order.  The context's
 * timing events and path counters are not used by this call;
 * ffp_last_device_error reports on it as on any call. */
int ffp_parse_f64_noalloc(ffp_ctx* ctx, const uint8_t* d_text, uint64_t nbytes,
                          double* d_values, uint8_t* d_status, uint64_t capacity,
                          uint64_t* d_count, void* stream);

/* As above, then waits for the stream.  Returns the token count (>= 0), or a
 * negative ffp_error: FFP_E_CAPACITY when count > capacity (the first
 * `capacity` tokens are still written), FFP_E_QUEUE when the fallback queue
 * overflowed, FFP_E_INTERNAL on a failed device-side consistency check.
 * The queue holds every token of more than 19 significant digits the
 * buffer can contain (a token that reaches the fallback through the w / w+1
 * test of Section 11 has at least 20 bytes) plus 65536 others; a token of at
 * most 19 significant digits reaches it only in the inconclusive-product
 * case of Algorithm 1 (Section 8), so an overflow needs more than 65536 such
 * tokens in one call. */
int64_t ffp_parse_f64_sync(ffp_ctx* ctx, const uint8_t* d_text, uint64_t nbytes,
                           double* d_values, uint8_t* d_status, uint64_t capacity,
                           uint64_t* d_count, void* stream);
int64_t ffp_parse_f32_sync(ffp_ctx* ctx, const uint8_t* d_text, uint64_t nbytes,
                           float* d_values, uint8_t* d_status, uint64_t capacity,
                           uint64_t* d_count, void* stream);

/* The same parse with binary16 (IEEE half) or bfloat16 results: the 16-bit
 * encodings, nearest value with ties to even.  The paper names binary16
 * among the standard formats (Section 2) and writes Algorithm 1 for any
 * significand width; these calls use the same table and steps.  The
 * paper's tie windows are derived for binary64 and binary32 only: here a
 * product that may be an exact midpoint is decided exactly when the product
 * is exact (q in [0, 27]) or 5^-q divides w (q in [-27, -1], the value is
 * then (w / 5^-q) * 2^q), and goes to the exact fallback otherwise, which a
 * token of at most 19 significant digits reaches only in the inconclusive-
 * product case. */
int ffp_parse_f16(ffp_ctx* ctx, const uint8_t* d_text, uint64_t nbytes,
                  uint16_t* d_values, uint8_t* d_status, uint64_t capacity,
                  uint64_t* d_count, void* stream);
int ffp_parse_bf16(ffp_ctx* ctx, const uint8_t* d_text, uint64_t nbytes,
                   uint16_t* d_values, uint8_t* d_status, uint64_t capacity,
                   uint64_t* d_count, void* stream);
int64_t ffp_parse_f16_sync(ffp_ctx* ctx, const uint8_t* d_text, uint64_t nbytes,
                           uint16_t* d_values, uint8_t* d_status, uint64_t capacity,
                           uint64_t* d_count, void* stream);
int64_t ffp_parse_bf16_sync(ffp_ctx* ctx, const uint8_t* d_text, uint64_t nbytes,
                            uint16_t* d_values, uint8_t* d_status, uint64_t capacity,
                            uint64_t* d_count, void* stream);

/* Device-side error word of the last call on this context, read after the
 * caller has synchronised its stream: FFP_SUCCESS, FFP_E_QUEUE or
 * FFP_E_INTERNAL.  Blocks on the context's own copy stream. */
int ffp_last_device_error(ffp_ctx* ctx);

/* ---------------------------------------------------------------------------
 * Batched parse: many independent buffers in one launch sequence.
 *
 * d_jobs is a device array of njobs (1 <= njobs <= 65535) ffp_job records.
 * The kernels read text, nbytes, values, status, capacity and dtype from it
 * and write count and err back into it; the caller may rewrite the records
 * on the device between calls (this is what a captured graph replays).
 * Every job is parsed exactly as ffp_parse_f64 / ffp_parse_f32 would parse
 * it alone; all blocks of all jobs share one persistent launch of each
 * kernel.  max_total_bytes bounds the sum of nbytes over the jobs (it sizes
 * the scratch); if the jobs exceed it, every job gets err = FFP_E_CAPACITY
 * and count = 0.  Returns FFP_E_ARG for bad arguments, FFP_E_NOMEM, FFP_E_HIP.
 * ------------------------------------------------------------------------- */
#define FFP_DTYPE_F64 0
#define FFP_DTYPE_F32 1
#define FFP_DTYPE_F16 2   /* binary16, 2-byte values */
#define FFP_DTYPE_BF16 3  /* bfloat16, 2-byte values */

typedef struct ffp_job {
    const uint8_t* text;  /* device text of this job (any alignment) */
    uint64_t nbytes;
    void* values;         /* device: capacity values of the dtype */
    uint8_t* status;      /* device: capacity bytes */
    uint64_t capacity;
    uint64_t count;       /* out: true number of tokens */
    int32_t dtype;        /* FFP_DTYPE_F64, _F32, _F16 or _BF16 */
    int32_t err;          /* out: FFP_SUCCESS, FFP_E_CAPACITY (count >
                             capacity, or max_total_bytes exceeded),
                             FFP_E_ARG (unknown dtype) or FFP_E_QUEUE (the
                             fallback queue overflowed on this job) */
} ffp_job;

int ffp_parse_batch(ffp_ctx* ctx, ffp_job* d_jobs, uint32_t njobs, uint64_t max_total_bytes,
                    void* stream);

/* A batched parse captured once into a HIP graph and replayed: the graph
 * holds the fixed d_jobs pointer, njobs and the scratch sized for
 * max_total_bytes; the records behind d_jobs may change between launches.
 * The context must outlive the graph and must not run other calls
 * concurrently with a launch. */
typedef struct ffp_graph ffp_graph;
int ffp_batch_graph_create(ffp_ctx* ctx, ffp_job* d_jobs, uint32_t njobs,
                           uint64_t max_total_bytes, ffp_graph** out);
int ffp_batch_graph_launch(ffp_graph* g, void* stream);
void ffp_batch_graph_destroy(ffp_graph* g);

/* Launch schedule of the parse kernel: tile bytes per workgroup step
 * (4096 * tile_k, tile_k in {1, 2, 4}), resident workgroups per CU
 * (1 .. the occupancy limit; 0 = the limit) and the block size in KiB
 * (4, 16 or 64; 0 = chosen per call: the largest block that still gives
 * every parse workgroup two blocks, so that small inputs spread over many
 * workgroups).  A call never uses tiles larger than its blocks.  Until a
 * schedule is set (ffp_set_tuning, ffp_autotune_batch or the FFP_TILE_K
 * environment variable) the tile is chosen per call: 16 KiB, 8 KiB for
 * FFP_JSON_DOCUMENT and FFP_CSV contexts (within the block size above);
 * ffp_get_tuning then reports that choice.  The schedule never changes
 * results. */
typedef struct ffp_tuning {
    int32_t tile_k;
    int32_t blocks_per_cu;
    int32_t block_kib;
    int32_t reserved;
} ffp_tuning;

int ffp_get_tuning(ffp_ctx* ctx, ffp_tuning* out);
int ffp_set_tuning(ffp_ctx* ctx, const ffp_tuning* t);

/* Autotuner: runs the given batch (it must be valid input; its outputs are
 * overwritten) under every candidate schedule, times the parse kernel with
 * HIP events, keeps the fastest in the context and returns it.  With the
 * environment variable FFP_TUNE_CACHE naming a file, results are cached
 * there as JSON keyed by GPU architecture, job count and byte-size bucket,
 * and a cached entry is used without measuring.  Synchronises the stream. */
int ffp_autotune_batch(ffp_ctx* ctx, ffp_job* d_jobs, uint32_t njobs, uint64_t max_total_bytes,
                       void* stream, ffp_tuning* out);

/* ---------------------------------------------------------------------------
 * Timing of the dominant kernel.  When enabled, each parse call records HIP
 * events on its stream around the parse kernel (K-parse) only; the totals
 * accumulate until read.  ffp_timing_read synchronises on the last event and
 * returns the summed milliseconds and the number of timed launches.  The
 * events are created without the system-scope fence (timing only, so that
 * recording them does not write back and invalidate the caches between the
 * kernels): waiting on them does not make the call's results visible to the
 * host; synchronise the stream for that.
 * ------------------------------------------------------------------------- */
int ffp_timing_enable(ffp_ctx* ctx, int enable);
int ffp_timing_read(ffp_ctx* ctx, double* total_ms, uint64_t* launches);

/* ---------------------------------------------------------------------------
 * In-kernel reduction (the paper's benchmark keeps the running minimum of
 * the parsed values, Section 12).  With d_out set (a device array of three
 * uint64_t), every later plain parse call on the context also writes, when
 * its last kernel ends: d_out[0] the encoding of the smallest value and
 * d_out[1] of the largest among the tokens with status FFP_OK that are not
 * NaN (-0 orders before +0), zero-extended to 64 bits, and d_out[2] their
 * number; with no such token both encodings are the canonical quiet NaN.
 * NULL turns it off.  Batched calls ignore it.
 * ------------------------------------------------------------------------- */
int ffp_set_reduce(ffp_ctx* ctx, uint64_t* d_out);

/* Columns of a FFP_CSV context whose tokens are parsed: bit c selects column
 * c (columns from 64 on are never selected).  Default: every column below 64.
 * Applies to the calls made after it. */
int ffp_set_csv_columns(ffp_ctx* ctx, uint64_t columns);

/* ---------------------------------------------------------------------------
 * Exact in-kernel sum (an extension of the reduction above; Section 12's
 * benchmark reduces the parsed values, and summing them is the other common
 * reduction).  With d_sum set (a device array of two uint64_t), every later
 * plain parse call on the context also writes, when its last kernel ends:
 *   d_sum[0]  the binary64 encoding of the sum of the values that the
 *             reduction above covers (status FFP_OK, not NaN), computed
 *             exactly and rounded once, to nearest with ties to even, in
 *             binary64 whatever the call's output format; a sum beyond the
 *             binary64 range rounds to an infinity of its sign;
 *   d_sum[1]  1 if that rounding was exact, else 0.
 * Infinities follow IEEE addition (+inf and -inf together give the
 * canonical quiet NaN, with d_sum[1] = 0).  An exact zero is -0 only when
 * every summed value is -0; the empty sum is +0.  The result does not depend
 * on the order of the tokens or on how the call is split into workgroups.
 * Exact for every call that fits in device memory (the accumulators'
 * carries cannot overflow below 2^43 bytes of text).  Independent of
 * ffp_set_reduce; NULL turns it off.  Batched calls ignore it.
 * ------------------------------------------------------------------------- */
int ffp_set_reduce_sum(ffp_ctx* ctx, uint64_t* d_sum);

/* ---------------------------------------------------------------------------
 * Device path counters (Table 5 of the paper reports the same categories on
 * CPUs).  When enabled, the parse kernels count tokens per path; reading
 * synchronises.  counters[0..5]: tokens, invalid, early-exit (zero / out of
 * range before any product), one significand evaluated (up to 19 digits,
 * decided), w and w+1 evaluated (more than 19 digits, decided), sent to the
 * exact fallback.
 * ------------------------------------------------------------------------- */
int ffp_counters_enable(ffp_ctx* ctx, int enable);
int ffp_counters_read(ffp_ctx* ctx, uint64_t counters[6]);

/* ---------------------------------------------------------------------------
 * Serving: a request loop with continuous batching.
 *
 * A server owns a fixed slice of device memory (the HBM budget, allocated
 * once at creation) and a dispatcher thread.  Requests (one text buffer
 * each) are submitted from any host thread and queue in arrival order.  As
 * soon as one of the server's streams is free, the dispatcher admits the
 * requests at the head of the queue whose outputs (and, for host text, a
 * device copy of the text) fit the free part of the budget, and launches
 * them together as one batched parse (ffp_parse_batch) on that stream;
 * requests that arrive while batches are on the GPU go into the next batch,
 * so work of several batches overlaps on the device.  Each request is
 * parsed exactly as ffp_parse_f64 / ffp_parse_f32 would parse it alone.
 * A request's outputs stay in the server's memory until it is released.
 *
 * Times are CLOCK_MONOTONIC nanoseconds (ffp_clock_ns).
 * The server is thread-safe, except that ffp_server_destroy must not run
 * concurrently with any other call on it.
 * ------------------------------------------------------------------------- */
typedef struct ffp_server ffp_server;

#define FFP_SERVE_BATCHED 0 /* continuous batching over `streams` streams */
#define FFP_SERVE_PLAIN 1   /* one plain parse launch per request, in
                               arrival order (the one-buffer-per-launch
                               comparison point) */

typedef struct ffp_server_options {
    uint64_t hbm_budget_bytes; /* device memory of the server: per-stream
                                  scratch plus the request arena (0 = 32 GiB) */
    uint64_t max_batch_bytes;  /* text bytes per batch; sizes each stream's
                                  scratch (0 = 256 MiB); also the largest
                                  request accepted */
    uint32_t max_inflight;     /* requests held at once, queued or running or
                                  done and not yet released (0 = 65536) */
    uint32_t streams;          /* batches in flight, 1..4 (0 = 2) */
    uint32_t max_batch_jobs;   /* requests per batch, 1..65535 (0 = 1024) */
    uint32_t mode;             /* FFP_SERVE_BATCHED or FFP_SERVE_PLAIN */
    uint32_t use_graph;        /* batched mode: replay a captured graph of the
                                  batch launch sequence per batch */
    uint32_t spin_us;          /* an idle dispatcher polls for new requests
                                  this long before it sleeps (0 = it sleeps at
                                  once): a CPU core spent for a shorter path
                                  from submission to launch */
    uint32_t reserved[2];
} ffp_server_options;

typedef struct ffp_result {
    const void* values;      /* device: `count` values of the dtype, owned
                                by the server until ffp_server_release */
    const uint8_t* status;   /* device: `count` ffp_token_status bytes */
    uint64_t count;          /* tokens of the request */
    uint64_t nbytes;         /* text bytes of the request */
    int32_t dtype;           /* FFP_DTYPE_* */
    int32_t err;             /* FFP_SUCCESS, FFP_E_QUEUE, FFP_E_INTERNAL or
                                FFP_E_HIP */
    uint64_t t_arrive_ns;    /* arrival time given at submission */
    uint64_t t_launch_ns;    /* its batch was queued on a stream */
    uint64_t t_done_ns;      /* the dispatcher saw the batch complete */
    uint32_t batch_jobs;     /* requests in that batch */
    uint32_t reserved;
} ffp_result;

typedef struct ffp_server_stats {
    uint64_t submitted, completed, batches, bytes;
    uint64_t arena_bytes;       /* request arena (budget minus scratch) */
    uint64_t arena_peak_bytes;  /* most arena bytes held at once */
    uint64_t scratch_bytes;     /* scratch of all streams */
    uint64_t max_batch_seen;    /* largest batch launched (requests) */
    uint64_t cancelled;         /* released while still queued, never run */
} ffp_server_stats;

/* Current CLOCK_MONOTONIC time in nanoseconds. */
uint64_t ffp_clock_ns(void);

/* Create a server with the options and schedule of `ctx` (delimiters,
 * flags, tuning).  `ctx` is only read; the server makes its own contexts.
 * NULL options select the defaults.  Returns FFP_E_BUDGET when the budget
 * cannot hold the scratch plus the largest request, FFP_E_NOMEM when the
 * budget cannot be allocated, FFP_E_ARG for bad options. */
int ffp_server_create(ffp_ctx* ctx, const ffp_server_options* opts, ffp_server** out);

/* Submit one request.  `text` holds nbytes bytes, in device memory when
 * on_device != 0, else in host memory (preferably pinned, e.g. from
 * hipHostMalloc); either way it must stay valid and unchanged until the
 * request is done.  arrival_ns = 0 means now.  Writes the request's ticket.
 * Returns FFP_E_BUDGET when the request can never fit (larger than
 * max_batch_bytes, or its outputs larger than the arena), FFP_E_BUSY when
 * max_inflight requests are held, FFP_E_ARG for bad arguments. */
int ffp_server_submit(ffp_server* srv, const uint8_t* text, uint64_t nbytes, int on_device,
                      int dtype, uint64_t arrival_ns, uint64_t* ticket);

/* Returns 1 and fills *out when the request is done, 0 while it is queued
 * or running, FFP_E_ARG for an unknown ticket. */
int ffp_server_poll(ffp_server* srv, uint64_t ticket, ffp_result* out);

/* Blocks until the request is done, then fills *out.  FFP_E_ARG for an
 * unknown ticket. */
int ffp_server_wait(ffp_server* srv, uint64_t ticket, ffp_result* out);

/* Copies min(count, max_count) values and status bytes of a done request to
 * dst_values / dst_status (device or pinned host memory; either may be
 * NULL), stream-ordered on `stream`.  FFP_E_BUSY if the request is not done.
 * The request may be released right after this call, without waiting for
 * the stream: the server keeps its memory out of reuse until the copies
 * queued here have completed. */
int ffp_server_copy_result(ffp_server* srv, uint64_t ticket, void* dst_values,
                           uint8_t* dst_status, uint64_t max_count, void* stream);

/* Frees the request's memory.  A request still waiting in the queue is
 * cancelled (never launched, counted in `cancelled`); one that is running is
 * detached: its memory is freed when it completes.  A done request whose
 * results are still being copied (ffp_server_copy_result) keeps its memory
 * until those copies complete.  Either way its ticket is forgotten now. */
int ffp_server_release(ffp_server* srv, uint64_t ticket);

int ffp_server_stats_read(ffp_server* srv, ffp_server_stats* out);

/* Stops admitting, waits for the batches on the GPU, frees everything.
 * Requests still queued are dropped. */
void ffp_server_destroy(ffp_server* srv);

/* Replay of an arrival trace (capacity planning and benchmarks): a
 * submitting thread submits request i at its arrival time (spinning for the
 * last few hundred microseconds; retrying while the server answers
 * FFP_E_BUSY), a collecting thread waits for the requests in submission
 * order, records their timestamps, copies the results of requests that name
 * destinations (ffp_server_copy_result on a stream of its own; others are
 * discarded) and releases them.  Blocks until every request is done and
 * every copy has completed.  Returns FFP_SUCCESS or the first submission
 * error. */
typedef struct ffp_replay_request {
    const uint8_t* text;
    uint64_t nbytes;
    int32_t on_device;
    int32_t dtype;
    uint64_t arrival_ns;  /* CLOCK_MONOTONIC */
    void* dst_values;     /* optional (device or pinned host): the values */
    uint8_t* dst_status;  /* optional: the status bytes */
    uint64_t dst_capacity;  /* tokens the destinations hold */
} ffp_replay_request;

typedef struct ffp_replay_result {
    uint64_t t_arrive_ns, t_launch_ns, t_done_ns;
    uint64_t count;
    int32_t err;
    uint32_t batch_jobs;
} ffp_replay_result;

int ffp_server_replay(ffp_server* srv, const ffp_replay_request* reqs, uint64_t n,
                      ffp_replay_result* out);

#ifdef __cplusplus
}
#endif

#endif /* FFP_H */
