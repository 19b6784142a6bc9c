/*
 * thapi_tally.h -- C ABI of the MI355X trace-tally library.
 *
 * The library turns streams of API entry/exit records into exact per-API
 * tallies on one AMD Instinct MI355X (gfx950).  The problem it solves is the
 * one the paper's Tally view states (THAPI, section 3.4 "Babeltrace2 Analysis
 * Tools", and the worked table of section 4.3): for every function, the
 * number of calls and the summed, minimum and maximum inclusive duration
 * (Time / Calls / Min / Max; Average and Time(%) derive from them), plus the
 * number of hosts, processes and threads.  Intervals come from the start and
 * end events of each call (section 3.3, interval plugins).  Threads are
 * identified by host, process id and thread id (the event record of
 * section 1.1).  This library additionally keeps self time (inclusive time
 * minus the inclusive time of direct children), per-thread and per-process
 * breakdowns and, for variable-length records, summed transfer sizes.
 *
 * All arithmetic is unsigned 64-bit integer nanoseconds; results are
 * bit-exact and independent of how the input is chunked.
 *
 * Every function returns an int status: THAPI_OK (0) or a negative
 * THAPI_E_* code.  No exception crosses the ABI.  A call that fails leaves
 * the handle's state unchanged unless stated otherwise.
 */
#ifndef THAPI_TALLY_H
#define THAPI_TALLY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define THAPI_TALLY_ABI_VERSION 2u

/* ---- status codes ------------------------------------------------------ */
#define THAPI_OK            0
#define THAPI_E_INVAL      -1  /* null argument, bad ABI version, bad config, record bytes not a
                                  multiple of the record size, payload size != sum of payload_len
                                  (device input: reported by the flush; handle is failed) */
#define THAPI_E_NOMEM      -2  /* device allocation failed, or a chunk larger than the whole budget */
#define THAPI_E_AGAIN      -3  /* over the device budget with THAPI_NONBLOCKING: retry later */
#define THAPI_E_DEPTH      -4  /* some thread's call stack exceeded max_depth; handle is failed */
#define THAPI_E_MALFORMED  -5  /* THAPI_STRICT only: an anomaly counter is non-zero after a flush */
#define THAPI_E_DEVICE     -6  /* a HIP call failed; sticky, only read(stats)/close stay valid */
#define THAPI_E_BUFSZ      -7  /* read: capacity too small, *n_rows holds the required count */
#define THAPI_E_CAPACITY   -8  /* more streams or threads than configured (max_streams, max_threads);
                                  handle is failed */
#define THAPI_E_STATE      -9  /* call not valid now (submit after the final flush, use after failure) */

/* ---- record formats (all little-endian) -------------------------------- *
 * THAPI_FMT_FIXED24, 24 bytes per record:
 *   API record    [0,8) ts u64 | [8,12) tid u32 | [12,14) fn u16 | [14] kind u8
 *                 (0 = entry, 1 = exit) | [15] reserved | [16,24) ignored
 *   kernel record [0,8) start u64 | [8,12) queue u32 | [12,14) kernel_id u16 |
 *                 [14] kind = 2 | [15] reserved | [16,24) end u64
 * THAPI_FMT_VAR16, 16-byte header + payload heap:
 *   header        [0,8) ts u64 | [8,12) tid u32 | [12,14) fn u16 | [14] kind u8 |
 *                 [15] payload_len u8 (0..255)
 *   payloads are concatenated in record order in a separate buffer; record i's
 *   payload starts at the sum of payload_len over records before it in the
 *   same chunk.  An entry of a function with fn_has_size[fn] != 0 and
 *   payload_len >= 8 carries its u64 transfer size at payload offset 0 (the
 *   typed "size" argument of the section 1.1 record).  A kernel record carries
 *   its u64 end time at payload offset 0 and needs payload_len >= 8.
 * THAPI_FMT_PACKED, interleaved variable-length records as a trace writer
 *   lays them out (a CTF-like stream, section 3.1): packets one after the
 *   other, each a 16-byte header [0,4) magic 0x4B504854 ("THPK") | [4,8)
 *   packet bytes (header included, a multiple of 8) | [8,12) events |
 *   [12,16) 0, followed by its events, every event a VAR16 header with its
 *   payload inline and padded with zeros to a multiple of 8 bytes; the
 *   events must fill the packet exactly.  submit() takes the packet bytes as
 *   `records` (a multiple of 8 bytes) and, as `payload`, the packet index:
 *   the u64 byte offset of every packet, ascending, the first 0 and each
 *   next packet starting where the previous one ends (the index a trace
 *   reader keeps, which lets packets be decoded in parallel).  A flush
 *   decodes packed chunks on the GPU and tallies their events as VAR16
 *   records (fn_has_size and kernel records as for VAR16); results equal
 *   those of the same events submitted as VAR16.  Host input is checked by
 *   submit (THAPI_E_INVAL); device input by the flush, which fails with
 *   THAPI_E_INVAL and leaves the handle failed.
 * Host and process come from the stream key, not from the record. */
#define THAPI_FMT_FIXED24 1u
#define THAPI_FMT_VAR16   2u
#define THAPI_FMT_PACKED  3u

/* ---- open flags -------------------------------------------------------- */
#define THAPI_DEVICE_INPUT 0x01u /* submit() takes device pointers (e.g. a torch tensor's data_ptr) */
#define THAPI_NONBLOCKING  0x02u /* submit() over budget returns THAPI_E_AGAIN instead of waiting */
#define THAPI_DROP_ON_FULL 0x04u /* submit() over budget drops the chunk and counts its records */
#define THAPI_STRICT       0x08u /* flush() returns THAPI_E_MALFORMED when any anomaly was counted */
#define THAPI_PROFILE      0x10u /* time every kernel with HIP events (see thapi_tally_timings) */
#define THAPI_GRAPH        0x20u /* flush() captures its kernels in a HIP graph once per launch
                                    signature (work-list size, shape, buffers) and replays it */
#define THAPI_SERVICE      0x40u /* streaming form: a library thread tallies chunks as they arrive
                                    (continuous batching, see thapi_tally_ticket_done); cannot be
                                    combined with THAPI_GRAPH (open returns THAPI_E_INVAL) */
#define THAPI_INTERVALS    0x80u /* every flush also keeps the interval of each call it tallies (see
                                    thapi_tally_intervals); not with THAPI_SERVICE */

/* ---- flush / read ------------------------------------------------------ */
#define THAPI_TICKET_ALL  UINT64_MAX
#define THAPI_FLUSH_FINAL 0x1u   /* close every stream: open calls become unclosed_final */

#define THAPI_SCOPE_THREAD  1u   /* one row per (trace, host, pid, tid, fn) */
#define THAPI_SCOPE_PROCESS 2u   /* one row per (trace, host, pid, fn); tid = THAPI_ALL */
#define THAPI_SCOPE_FN      3u   /* one row per (trace, fn); host = pid = tid = THAPI_ALL */
#define THAPI_SCOPE_KERNEL  4u   /* one row per (trace, host, pid, kernel_id); tid = THAPI_ALL */
#define THAPI_ALL 0xFFFFFFFFu

#define THAPI_ROW_API    1u
#define THAPI_ROW_KERNEL 2u

#define THAPI_MAX_DEPTH_LIMIT   64u  /* max_depth may not exceed this */
#define THAPI_MAX_RANGE_THREADS 64u  /* a performance figure, not a limit: the distinct threads of one
                                        stream that one pass over a range holds on chip (1024 / max_depth
                                        when max_depth > 16).  A range meeting more takes one extra pass
                                        per further group of that many of the stream's threads (each
                                        pass reads the range's records again); results are the same */

typedef struct thapi_tally thapi_tally; /* opaque, owned by the library */

typedef struct {
  uint32_t abi_version;         /* must equal THAPI_TALLY_ABI_VERSION */
  uint32_t format;              /* THAPI_FMT_FIXED24, THAPI_FMT_VAR16 or THAPI_FMT_PACKED */
  uint32_t n_fns;               /* API fn ids must be < n_fns (1..65536) */
  uint32_t n_kernel_ids;        /* kernel ids must be < n_kernel_ids (0..65536) */
  uint32_t max_depth;           /* per-thread call-stack limit, 1..64; 0 -> 64 (a smaller limit lets one
                                   pass hold more threads, see THAPI_MAX_RANGE_THREADS) */
  uint32_t max_threads;         /* distinct (stream, tid) over the handle's life; 0 -> 65536 */
  uint32_t max_streams;         /* distinct stream keys over the handle's life; 0 -> 4096 */
  uint32_t flags;               /* THAPI_DEVICE_INPUT | THAPI_NONBLOCKING | ... */
  const uint8_t *fn_has_size;   /* VAR16: n_fns flags, copied at open; may be NULL (no sizes) */
  uint64_t device_budget_bytes; /* bytes of staged chunks admitted at once; 0 -> 16 GiB */
  int32_t device;               /* HIP device ordinal */
  uint32_t reserved;            /* must be 0 */
  void *hip_stream;             /* hipStream_t to launch on (e.g. torch's current stream); NULL = own */
  const char *autotune_cache;   /* path of the launch-shape cache file, or NULL */
} thapi_tally_config;

typedef struct {
  uint32_t trace_id, host_id, pid, reserved; /* reserved must be 0 */
} thapi_stream_key;

typedef struct {                /* 88 bytes, naturally aligned */
  uint32_t trace_id, host_id, pid, tid;
  uint16_t id;                  /* fn id (API rows) or kernel id (kernel rows) */
  uint8_t row_kind;             /* THAPI_ROW_API or THAPI_ROW_KERNEL */
  uint8_t pad;
  uint32_t pad2;
  uint64_t count;
  uint64_t incl_sum, incl_min, incl_max; /* kernel rows: device duration end - start */
  uint64_t self_sum, self_min, self_max; /* kernel rows: 0 */
  uint64_t bytes_sum;                    /* VAR16 transfer sizes of tallied calls */
} thapi_tally_row;

typedef struct {
  uint64_t records;        /* records consumed */
  uint64_t entries, exits; /* valid API entry / exit records */
  uint64_t kernel_records; /* valid kernel records (tallied) */
  uint64_t orphan_exits;   /* exit with an empty stack (skipped) */
  uint64_t fn_mismatch;    /* exit whose fn differs from the popped entry's (not tallied) */
  uint64_t neg_duration;   /* exit earlier than its entry (not tallied) */
  uint64_t self_underflow; /* children longer than the call: self time clamped to 0 */
  uint64_t ts_regress;     /* API record earlier than the thread's previous one */
  uint64_t unclosed_final; /* entries still open at the final flush (not tallied) */
  uint64_t open_now;       /* entries open right now */
  uint64_t depth_overflow; /* threads whose stack ever exceeded max_depth */
  uint64_t bad_records;    /* unknown kind, fn/kernel id out of range, kernel end < start */
  uint64_t dropped_records;/* records of chunks dropped under THAPI_DROP_ON_FULL */
  uint64_t distinct_hosts, distinct_processes, distinct_threads;
} thapi_tally_stats;

/* Opens a handle on cfg->device: the state of an analysis of traces whose
 * calls are tallied per API function (section 3.4, the Tally view of the
 * section 4.3 table).  Allocates all device tables up front
 * (tallies: max_threads * n_fns * 64 B; stacks: max_threads * max_depth * 32 B).
 * *out is set only on success.  Errors: THAPI_E_INVAL (bad config),
 * THAPI_E_NOMEM, THAPI_E_DEVICE. */
int thapi_tally_open(const thapi_tally_config *cfg, thapi_tally **out);

/* Queues one chunk of one stream: events of one (trace, host, process), the
 * context a trace's stream carries (section 3.1; the section 1.1 record holds
 * host, vpid and vtid), in the order they were recorded.  Chunks of one key
 * are applied in submit order; keys are independent (the key is passed by
 * value; its `reserved` word must be 0).  Host input (default) is copied before the
 * call returns, so the caller may reuse its buffers at once; with
 * THAPI_DEVICE_INPUT the pointers are device memory that must stay valid and
 * unmodified until a flush covering the returned ticket has returned.
 * payload/payload_bytes are used by VAR16 only (must be NULL/0 for FIXED24).
 * VAR16 host input whose payload_len sum is not payload_bytes is refused
 * here; device input is not read by submit (no synchronisation), and the
 * flush that tallies such a chunk fails with THAPI_E_INVAL instead, having
 * read no byte outside [payload, payload + payload_bytes).
 * Thread-safe.  Errors: THAPI_E_INVAL, THAPI_E_NOMEM, THAPI_E_AGAIN,
 * THAPI_E_CAPACITY (too many streams), THAPI_E_STATE. */
int thapi_tally_submit(thapi_tally *t, thapi_stream_key key,
                       const void *records, size_t record_bytes,
                       const void *payload, size_t payload_bytes, uint64_t *ticket_out);

/* Runs every queued chunk up to `ticket` (THAPI_TICKET_ALL: all) through the
 * GPU pipeline and waits for it: each entry is matched with its exit per
 * thread (the interval of a call, section 3.3) and the call is added to its
 * (thread, function) tally (section 3.4); calls open at a chunk's end stay on
 * the device until a later chunk closes them, so a trace can be analysed while
 * it is still written (section 6).  THAPI_FLUSH_FINAL also closes all streams:
 * open entries become unclosed_final and no further submit is accepted.
 * Errors: THAPI_E_DEPTH, THAPI_E_CAPACITY, THAPI_E_MALFORMED (STRICT),
 * THAPI_E_INVAL (VAR16 device input with a payload size mismatch),
 * THAPI_E_DEVICE, THAPI_E_STATE. */
int thapi_tally_flush(thapi_tally *t, uint64_t ticket, uint32_t flags);

/* Reads the tally of everything flushed so far (calls, and total, min and
 * max of inclusive and self time per function: the columns of the section
 * 4.3 table, whose header counts hosts, processes and threads) for one scope
 * and trace
 * (THAPI_ALL = all traces), in canonical order (trace, host, pid, tid,
 * row_kind, id).  rows may be NULL when capacity is 0 (size query).
 * *n_rows receives the number of rows of the scope; if it exceeds capacity,
 * nothing is written to rows and THAPI_E_BUFSZ is returned.  stats (may be
 * NULL) receives the counters summed over the selected traces. */
int thapi_tally_read(thapi_tally *t, uint32_t scope, uint32_t trace_id,
                     thapi_tally_row *rows, size_t capacity, size_t *n_rows,
                     thapi_tally_stats *stats);

/* Forgets every tally, stack, stream and counter (device memory is kept) so
 * the handle can start a new trace set.  Not valid while submits are queued
 * (THAPI_E_STATE), except on a THAPI_SERVICE handle that a failure other than
 * THAPI_E_DEVICE stopped: there the chunks still queued are discarded (their
 * tickets never complete) and the service thread is started again.  On a
 * running service handle, reset first waits until every submitted chunk is
 * tallied.  The device tables are cleared by work enqueued on the handle's
 * stream, which later flushes and reads follow; the call does not wait for it.
 * A handle failed with THAPI_E_DEVICE cannot be reset. */
int thapi_tally_reset(thapi_tally *t);

/* Batched form: times the pipeline on the chunks queued right now under each
 * candidate launch shape -- records in the LDS tile region (1024, 2048, and
 * 4096 for FIXED24), LDS tally entries (every entry the LDS holds beyond 2048,
 * 2048, 1024), work-list ranges per CU (1, 2, 4, 8, 16) and the wave
 * schedule (0: all waves build a tile, then walk it; 1: half the waves build
 * the next tile while the other half walks the previous one) -- and keeps the fastest
 * for this workload class (device, format, max_depth, and the log2 buckets of
 * n_fns, chunk count and record count).  The choice is used by every later
 * flush of that class and, when cfg.autotune_cache names a file, written
 * there as text lines "key T E rpc pipe" and read back by later opens.  Each
 * candidate runs reps + 1 times (the first one warms up; the minimum of the
 * rest counts).  The queued chunks stay queued and the tables are re-initialised
 * afterwards, so the handle must not have flushed since open/reset:
 * THAPI_E_STATE otherwise, or when nothing is queued.  chosen (may be NULL)
 * receives {T, E, rpc, pipe}.  Errors: THAPI_E_STATE, THAPI_E_CAPACITY (no candidate
 * could take the work), THAPI_E_DEVICE. */
int thapi_tally_autotune(thapi_tally *t, uint32_t reps, uint32_t *chosen);

/* Measurement helper, not part of the tally: the launch shape the last flush
 * chose, shape[0..3] = {T, E, rpc, pipe} as for thapi_tally_autotune.  The
 * shape is the tuned one of the flush's workload class when there is one.
 * Otherwise it is the one that the environment variable THAPI_TALLY_SHAPE,
 * read at open as "T,E[,rpc[,pipe]]", names, provided that it is a valid
 * shape and fits the LDS (a shape that does not is ignored).  Otherwise it is
 * the default.  Errors: THAPI_E_INVAL (a NULL argument), THAPI_E_STATE (no
 * flush since open). */
int thapi_tally_last_shape(thapi_tally *t, uint32_t *shape);

/* Streaming form (THAPI_SERVICE).  Aggregation on the node while the trace
 * is still being produced (section 3, On-node Processing, builds aggregates
 * from temporarily stored traces; section 6 names tracing and analysis run
 * concurrently as work in progress), as a continuous-batching service: open()
 * starts a worker thread and, for host input, reserves device_budget_bytes of
 * device memory as the admission arena.  submit() waits for arena room (or
 * returns THAPI_E_AGAIN / drops, per the flags), queues the chunk in ticket
 * order, copies the caller's bytes into a pinned staging ring (at most
 * min(device_budget_bytes, 512 MiB), so the caller may reuse its buffer when
 * submit returns) and enqueues the ring -> arena DMA on one of four copy
 * streams, without waiting for it; the worker repeatedly takes every queued
 * chunk, makes its launch wait on the device for those chunks' copies,
 * tallies them all in one pipeline launch while later chunks keep copying,
 * stamps their completion and frees their ring and arena space.  Open calls stay on the device stacks between batches, so results
 * equal those of one flush over the same submissions.  flush(ticket) waits
 * until the worker has covered `ticket`; flush(..., THAPI_FLUSH_FINAL) waits
 * for everything submitted, then closes all streams.  A failure inside the
 * worker (THAPI_E_DEPTH, THAPI_E_CAPACITY, THAPI_E_DEVICE) makes the handle
 * failed and is returned by the next flush.
 *
 * thapi_tally_ticket_done: THAPI_OK and *done_ns (may be NULL) = the
 * CLOCK_MONOTONIC time in ns at which the batch holding `ticket` completed,
 * THAPI_E_AGAIN if it has not yet, THAPI_E_INVAL for a ticket never issued.
 *
 * thapi_tally_service_info: writes min(n, 6) counters {batches, chunks in
 * batches, largest batch (chunks), bytes admitted, chunks queued now, arena
 * bytes in use}; returns the number written. */
int thapi_tally_ticket_done(thapi_tally *t, uint64_t ticket, uint64_t *done_ns);
int thapi_tally_service_info(thapi_tally *t, uint64_t *info, int n);

/* Aggregate export and merge (section 3.7, On-node Processing: the aggregate
 * of a trace, small enough to keep where the trace itself is not, can be
 * replayed into a tally, and the aggregates of many nodes are combined at a
 * global master).
 *
 * thapi_tally_export writes everything flushed so far as one self-describing
 * little-endian byte blob: every stream's key, dropped records and counters;
 * every thread's (stream, tid), open calls (its carried stack), flags and
 * last timestamp; every non-empty (thread, fn) tally and (stream, kernel)
 * tally.  (The payload-role tables -- copy rows and the handle join -- and
 * the intervals of the last flush are not part of it.)  Layout, in order:
 *   header  16 x u32: magic "THTALLY1" (2 words), version 1, format, n_fns,
 *           n_kernel_ids, max_depth, n_streams, n_threads, n_frames, n_rows,
 *           n_krows, finalized (0/1), 3 x 0
 *   streams n_streams x {u32 trace, host, pid, 0; u64 dropped; u64 counters[11]}
 *           (counters: records, entries, exits, kernel records, orphan exits,
 *           fn mismatch, negative durations, self underflow, ts regressions,
 *           unclosed at the final flush, bad records)
 *   threads n_threads x {u32 stream index, tid, open calls, flags (1: has a
 *           timestamp, 2: stack overflowed); u64 last timestamp}
 *   frames  n_frames x {u32 thread index, fn; u64 entry ts, children time,
 *           bytes}, each thread's open calls bottom first, threads in order
 *   rows    n_rows x {u32 thread index, fn; u64 count, incl sum/min/max,
 *           self sum/min/max, bytes}
 *   krows   n_krows x {u32 stream index, kernel id; u64 count, sum, min, max}
 * Two-call pattern: *size receives the blob size; with capacity `cap` too
 * small nothing is written and THAPI_E_BUFSZ is returned (THAPI_OK when buf
 * is NULL and cap is 0).  Errors: THAPI_E_INVAL, THAPI_E_BUFSZ,
 * THAPI_E_STATE (failed handle), THAPI_E_DEVICE.
 *
 * thapi_tally_merge combines a blob into the handle: streams match by key
 * (new keys are registered), threads by (stream key, tid); counts, sums,
 * counters and dropped records add, mins and maxes combine; a blob thread's
 * open calls and last timestamp are installed on the handle's thread, which
 * must have no open call (THAPI_E_STATE otherwise, and nothing changes).  So
 * the merge of the exports of handles that saw disjoint sets of streams
 * equals one handle that saw them all, and a fresh handle that merges an
 * export taken between flushes continues the trace exactly where the
 * exporting handle stopped (checkpoint / resume).  The blob's format, n_fns,
 * n_kernel_ids and max_depth must equal the handle's (THAPI_E_INVAL).  Not
 * valid on a THAPI_SERVICE handle, while chunks are queued or after the final
 * flush (THAPI_E_STATE).  Errors: THAPI_E_INVAL (malformed blob),
 * THAPI_E_CAPACITY (more streams than max_streams: nothing changes; more
 * threads than max_threads: the handle is failed), THAPI_E_STATE,
 * THAPI_E_DEVICE. */
int thapi_tally_export(thapi_tally *t, void *buf, size_t cap, size_t *size);
int thapi_tally_merge(thapi_tally *t, const void *buf, size_t size);

/* For callers that cannot allocate memory (code under stream capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same work as
 * thapi_tally_flush, with the same results and errors, but the flush's device
 * buffers -- the work list and the range summaries -- live in a static device
 * array of THAPI_NOALLOC_SCRATCH_BYTES that each GPU holds for the life of
 * the process, and the call allocates no device or pinned host memory (no
 * hipMalloc, hipFree, hipHostMalloc or graph instantiation).  The kernels
 * are launched directly even on a THAPI_GRAPH handle.  Requires a handle
 * opened with THAPI_DEVICE_INPUT and without THAPI_SERVICE (host input is
 * staged in allocations that a flush frees; the service thread flushes by
 * itself): THAPI_E_INVAL otherwise.  A flush whose summaries do not fit the
 * array (about 68 KiB per range at max_depth 16, 260 KiB at 64; the work is
 * cut into fewer, longer ranges first, and every chunk needs one) returns
 * THAPI_E_NOMEM and leaves every chunk queued.  A flush that meets more
 * threads of one stream within one range than a pass holds
 * (THAPI_MAX_RANGE_THREADS) needs memory for extra passes: it fails the
 * handle with THAPI_E_NOMEM.  Every call on one GPU shares
 * that GPU's array and leaves its contents behind (the work-queue head that
 * must start at zero is re-written by each call); calls that overlapped on
 * one GPU would race on it, so the library serialises them within the
 * process (each process has its own copy of the array). */
#define THAPI_NOALLOC_SCRATCH_BYTES (32u << 20)
int thapi_tally_flush_noalloc(thapi_tally *t, uint64_t ticket, uint32_t flags);

/* Intervals (section 3.3: an interval plugin turns the entry and exit events
 * of a call into one record spanning them; section 3.6 draws them on a
 * timeline), materialised instead of aggregated.  With THAPI_INTERVALS, every
 * flush keeps one record per call it tallies -- the calls completed inside its
 * chunks and those it closed that earlier chunks or flushes opened -- until
 * the next flush or reset: the stream key, tid, fn, depth (1 = top level),
 * entry and exit timestamps, and the entry timestamp and fn of the parent
 * (the call on top of the thread's stack when this one was entered; 0 and
 * THAPI_ALL at the top level).  Calls that are not tallied (anomalies, calls
 * still open) have no interval.  The device holds up to 32 bytes per record
 * of the flush for them.
 * thapi_tally_intervals writes the last flush's intervals, in no particular
 * order (sort by trace, host, pid, tid, start, depth, end, fn, parent for a
 * canonical one), to `out`: host memory, or device memory with
 * THAPI_OUT_DEVICE.  *n receives the count; with capacity `cap` too small
 * nothing is written and THAPI_E_BUFSZ is returned (THAPI_OK when out is
 * NULL and cap is 0).  Errors: THAPI_E_INVAL, THAPI_E_BUFSZ, THAPI_E_STATE
 * (handle opened without THAPI_INTERVALS, or failed), THAPI_E_DEVICE. */
typedef struct {                 /* 56 bytes */
  uint32_t trace_id, host_id, pid, tid;
  uint32_t fn, depth;
  uint64_t start, end;
  uint64_t parent_start;
  uint32_t parent_fn;
  uint32_t pad;
} thapi_tally_interval;
#define THAPI_OUT_DEVICE 0x1u
int thapi_tally_intervals(thapi_tally *t, thapi_tally_interval *out, size_t cap, size_t *n, uint32_t flags);

/* Payload analytics (VAR16 and packed handles).  Functions can be given a
 * role, and every record of such a function that carries the role's payload
 * counts, whether or not its call is tallied (these are per-record counts,
 * made while the records are decoded):
 *   THAPI_ROLE_COPY: an entry with payload_len >= 24 carries a transfer
 *     size (u64 at payload offset 0), its destination (8) and source (16)
 *     pointers.  A pointer whose top byte is 0xff is device memory, any other
 *     host memory (section 1.1 reads a copy's direction from these prefixes).
 *     Per (stream, fn, direction) the entries are counted and the sizes
 *     summed; direction = 2 * (source on device) + (destination on device):
 *     THAPI_DIR_H2H 0, THAPI_DIR_H2D 1, THAPI_DIR_D2H 2, THAPI_DIR_D2D 3.
 *   THAPI_ROLE_CREATE: an exit with payload_len >= 8 returns a handle (u64
 *     at offset 0).  THAPI_ROLE_RELEASE: an entry with payload_len >= 8
 *     takes one.  Creates and releases of a stream are joined by handle value
 *     (the validation of section 4.2, which reports releases that were never
 *     handled): a value created C times and released R times leaves
 *     max(0, C - R) handles unreleased and max(0, R - C) releases that match
 *     no create.  Record order is not considered, and handles persist across
 *     flushes until a reset.
 * thapi_tally_set_roles: roles[fn] in {0, THAPI_ROLE_*} for every fn
 * (n_fns must equal the handle's), and room for max_handles distinct
 * (stream, handle) values.  Valid once, before the first submit after open
 * or reset (THAPI_E_STATE otherwise); a reset clears the tables and keeps
 * the roles.  More distinct handles than that room fail the flush with
 * THAPI_E_CAPACITY.  Errors: THAPI_E_INVAL (FIXED24 handle, bad role),
 * THAPI_E_NOMEM, THAPI_E_STATE, THAPI_E_DEVICE.
 * thapi_tally_copies / thapi_tally_handles: the rows of trace_id (THAPI_ALL:
 * all) in order (trace, host, pid[, fn, dir]): one copy row per (stream, fn,
 * direction) with entries, one handle row per stream with a create or a
 * release.  Two-call pattern as for read (THAPI_E_BUFSZ).  THAPI_E_STATE when
 * no roles were set. */
#define THAPI_ROLE_COPY    1u
#define THAPI_ROLE_CREATE  2u
#define THAPI_ROLE_RELEASE 3u
#define THAPI_DIR_H2H 0u
#define THAPI_DIR_H2D 1u
#define THAPI_DIR_D2H 2u
#define THAPI_DIR_D2D 3u
typedef struct {                 /* 40 bytes */
  uint32_t trace_id, host_id, pid, fn, dir, pad;
  uint64_t count, bytes;
} thapi_copy_row;
typedef struct {                 /* 56 bytes */
  uint32_t trace_id, host_id, pid, pad;
  uint64_t creates, releases, handles, unreleased, unmatched;
} thapi_handle_row;
int thapi_tally_set_roles(thapi_tally *t, const uint8_t *roles, uint32_t n_fns, uint32_t max_handles);
int thapi_tally_copies(thapi_tally *t, uint32_t trace_id, thapi_copy_row *rows, size_t capacity,
                       size_t *n_rows);
int thapi_tally_handles(thapi_tally *t, uint32_t trace_id, thapi_handle_row *rows, size_t capacity,
                        size_t *n_rows);

/* Frees everything.  Queued chunks that were never flushed are discarded. */
int thapi_tally_close(thapi_tally *t);

/* Measurement helper, not part of the tally: the streaming-read bandwidth of
 * `device` in GB/s (1e9 bytes/s), from a plain read kernel (16-byte
 * non-temporal loads, grid-stride, about 16 workgroups per compute unit)
 * over a freshly allocated buffer of `bytes` (rounded down to the kernel's
 * quantum; at least 1 MiB), best of `reps` timed passes after one warm-up.
 * The figure that an HBM-bound kernel's fraction of the published peak can
 * be set against.  Errors: THAPI_E_INVAL, THAPI_E_NOMEM, THAPI_E_DEVICE. */
int thapi_tally_read_bandwidth(int32_t device, uint64_t bytes, uint32_t reps, double *gbs);

/* Static English text for a status code; never NULL. */
const char *thapi_tally_strerror(int code);

/* THAPI_PROFILE only: per-kernel durations (ms) of the last flush and read,
 * measured with HIP events on the launch stream, in the order
 * {prepass, main, combine, final, readout, intervals, decode, payload}
 * (decode: the packed chunks' decode into records; payload: the copy and
 * handle analytics of functions with roles); entries that did not run are 0.  A flush that needed extra passes (THAPI_MAX_RANGE_THREADS)
 * reports its first pass only.
 * Under THAPI_GRAPH, "main" is the whole replayed graph.
 * n: capacity of ms[]; returns the number of entries written. */
int thapi_tally_timings(thapi_tally *t, double *ms, int n);

#ifdef __cplusplus
}
#endif

#endif /* THAPI_TALLY_H */
