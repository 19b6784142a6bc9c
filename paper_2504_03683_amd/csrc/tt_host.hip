// tt_host.hip -- host runtime and C ABI of the tally library (see thapi_tally.h).
//
// The handle owns every device table up front (sized from the config), a
// HIP stream (or borrows the caller's), a queue of submitted chunks in
// ticket order, and grow-only scratch buffers for flushes and reads.  A flush
// turns the queued chunks into a device work list of ranges and launches the
// pipeline: [VAR16 payload pre-pass] -> range kernel -> combine -> [final].
// A read sorts the threads canonically and compacts the tally tables into
// rows on the device, then copies the rows out.
#include <algorithm>
#include <array>
#include <atomic>
#include <condition_variable>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <chrono>
#include <string>
#include <thread>
#include <vector>

#include "thapi_tally.h"
#include "tt_common.h"

namespace tt {
size_t range_lds_bytes(uint32_t T, uint32_t E, uint32_t KL, uint32_t D, int fmt);
hipError_t launch_range(int fmt, uint32_t T, const Seg *segs, const Range *ranges, const uint32_t *order,
                        uint32_t n_ranges, uint32_t *qhead, uint32_t n_wg, const Tables &tb, const Shape &sh,
                        RHdr *rhdr, UItem *ru, OItem *ro, uint32_t *rnslots, uint32_t *rmore,
                        const Range *pranges, uint32_t rid_base, hipStream_t st);
hipError_t prepare_range_kernels(uint32_t max_lds_bytes);
hipError_t prepare_combine_kernel();
hipError_t launch_paylen(const Seg *segs, Range *ranges, uint32_t n_ranges, const uint32_t *seg_first_range,
                         uint32_t n_segs, const uint32_t *slice_first, uint32_t n_slices, uint64_t *paylen,
                         uint32_t *err, hipStream_t st);
hipError_t launch_fill64(uint64_t *p, size_t n, uint64_t v, hipStream_t st);
hipError_t launch_fill32(uint32_t *p, size_t n, uint32_t v, hipStream_t st);
hipError_t launch_init_all(const InitSet &is, hipStream_t st);
hipError_t launch_combine(const uint32_t *spans, uint32_t n_spans, const RHdr *rhdr, const UItem *ru,
                          const OItem *ro, const uint32_t *rnslots, const Tables &tb, const uint32_t *clist,
                          hipStream_t st);
hipError_t launch_final(const Tables &tb, uint32_t max_threads, hipStream_t st);
size_t part_range_bytes(uint32_t n_fns, int fmt);
hipError_t launch_part_merge(int fmt, const uint32_t *spans, uint32_t n_spans, const Tables &tb, hipStream_t st);
hipError_t launch_iv_out(const Tables &tb, const uint64_t *ivbase, const RHdr *rhdr, uint32_t n_ranges,
                         const uint32_t *rnslots, const uint64_t *off, const uint32_t *skeys, void *out,
                         hipStream_t st);
size_t pk_scratch_bytes(uint64_t np);
hipError_t launch_pk_count(const PkChunk *chunks, const uint64_t *first, uint32_t nc, uint64_t np, uint8_t *scr,
                           uint64_t *tot_out, uint32_t *err, hipStream_t st);
hipError_t launch_pk_write(const PkChunk *chunks, const uint64_t *first, uint32_t nc, uint64_t np, uint8_t *scr,
                           uint64_t *hdr, uint64_t *heap, uint32_t *err, hipStream_t st);
hipError_t launch_payload(const Seg *segs, const Range *ranges, uint32_t n_ranges, const uint32_t *slice_first,
                          uint32_t n_slices, const uint64_t *sliceoff, const PayTables &pt, hipStream_t st);
hipError_t launch_handle_stats(const PayTables &pt, unsigned long long *out, uint32_t ns, hipStream_t st);
hipError_t launch_thread_stats(const Tables &tb, uint32_t max_threads, unsigned long long *out, uint32_t ns,
                               uint32_t ns1, hipStream_t st);
hipError_t launch_sort_threads(const Tables &tb, const uint32_t *stream_rank, uint64_t *keys, uint32_t *vals,
                               uint64_t *keys2, uint32_t *vals2, uint32_t n, int rank_bits, hipStream_t st);
hipError_t launch_group_bounds(const uint64_t *keys, uint32_t n, uint32_t *gbeg, uint32_t *gend, uint32_t n_ranks,
                               hipStream_t st);
bool sort_small_fits(uint32_t n);
hipError_t launch_sort_small(const Tables &tb, const uint32_t *stream_rank, uint64_t *keys, uint32_t *vals, uint32_t n,
                             uint32_t *gbeg, uint32_t *gend, uint32_t n_ranks, hipStream_t st);
struct RowCtx {
  int mode;
  uint32_t n_ids;
  const uint64_t *keys;
  const uint32_t *vals;
  const uint32_t *gbeg, *gend;
  const uint32_t *rank_stream;
  const uint32_t *rank_key;
  const uint32_t *trace_span;
};
hipError_t launch_group_rows(const RowCtx &c, const Tables &tb, uint32_t n_groups, uint32_t *cnt, uint64_t *off,
                             uint8_t *out, hipStream_t st);
}  // namespace tt

using namespace tt;

// Device memory of thapi_tally_flush_noalloc: the work list and the range
// summaries of one flush.  In host code this name is only a stand-in for the
// symbol: host code uses the address hipGetSymbolAddress gives for each
// device (scratch_on), never the name.
static __device__ __align__(256) uint8_t scratch[THAPI_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch[MAX_DEVICES] = {};        // the array's address on each device (null: not resolved)
std::mutex g_noalloc_mu[MAX_DEVICES];        // one no-alloc flush at a time per device

// Resolves the scratch array's address on `dev`, which must be the current
// device; once per device (thapi_tally_open calls it).
hipError_t scratch_setup(int dev) {
  if (dev < 0 || dev >= MAX_DEVICES) return hipSuccess;   // (the no-alloc flush then refuses)
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch[dev]) return hipSuccess;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch[dev] = (uint8_t *)p;
  return hipSuccess;
}

uint8_t *scratch_on(int dev) {
  if (dev < 0 || dev >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  return g_scratch[dev];
}


struct DevBuf {
  void *p = nullptr;
  size_t cap = 0;
  hipError_t ensure(size_t bytes) {
    if (bytes <= cap) return hipSuccess;
    if (p) { hipFree(p); p = nullptr; cap = 0; }
    size_t want = std::max<size_t>(bytes, 256);
    want = want + want / 4;
    hipError_t e = hipMalloc(&p, want);
    if (e == hipSuccess) cap = want;
    return e;
  }
  void release() { if (p) hipFree(p); p = nullptr; cap = 0; }
  // grows to `bytes` keeping the first `keep` bytes (copied on `st`, which is
  // synchronised before the old buffer is freed)
  hipError_t ensure_keep(size_t bytes, size_t keep, hipStream_t st) {
    if (bytes <= cap) return hipSuccess;
    DevBuf nb;
    hipError_t e = nb.ensure(bytes);
    if (e == hipSuccess && keep && p) e = hipMemcpyAsync(nb.p, p, std::min(keep, cap), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) { nb.release(); return e; }
    release();
    p = nb.p;
    cap = nb.cap;
    return hipSuccess;
  }
  template <class T> T *as() const { return (T *)p; }
};
// An array inside a packed DevBuf (set by each upload).
struct DevView {
  void *p = nullptr;
  template <class T> T *as() const { return (T *)p; }
};

struct Chunk {
  uint32_t stream;
  const uint8_t *rec;
  const uint8_t *pay;
  uint64_t n_rec;
  uint64_t pay_bytes;
  uint64_t ticket;
  void *owned;       // staged device copy (host input), freed after its flush
  uint64_t owned_bytes;
  bool in_arena;     // service mode: the staged copy lives in the device arena
  bool in_hin;       // host input, no service: the staged copy lives in the host-input arena
  bool in_ring;      // service mode: the bytes went through the pinned staging ring
  bool ready;        // service mode: the copy to the device is enqueued (or complete)
  int ev;            // service mode: event recorded after the copy (index into the pool), or -1
  uint64_t pk_bytes;    // packed chunk not yet decoded: its bytes (rec) and packets (index at pay)
  uint64_t pk_packets;
};

// First-in first-out allocator over [0, cap): allocations are released in the
// order they were made, so free space is the one or two gaps around the live
// span [tail, head).  Used for the device arena and the pinned staging ring
// of the streaming form (chunks are tallied, and so released, in ticket order).
struct Fifo {
  uint64_t cap = 0, head = 0, tail = 0;
  std::deque<std::pair<uint64_t, uint64_t>> live;   // [offset, end) of live allocations, in order
  bool fit(uint64_t n, uint64_t *at) const {
    if (live.empty()) { if (n > cap) return false; *at = 0; return true; }
    if (head > tail) {
      if (cap - head >= n) { *at = head; return true; }
      if (tail > n) { *at = 0; return true; }   // wrap; the end of the buffer stays unused
      return false;
    }
    if (tail - head > n) { *at = head; return true; }
    return false;
  }
  void take(uint64_t at, uint64_t n) {
    if (live.empty()) tail = at;
    head = at + n;
    live.push_back({at, at + n});
  }
  void release_front() {
    if (live.empty()) return;
    live.pop_front();
    if (live.empty()) head = tail = 0;
    else tail = live.front().first;
  }
};
constexpr int N_COPY_STREAMS = 4;
constexpr uint64_t RING_MAX = 512ull << 20;   // pinned staging ring of the streaming form

using SKey = std::array<uint32_t, 3>;

// The device work of one flush: segments (one per chunk), ranges (a stream's
// records cut into pieces of about equal length), per-stream spans of
// consecutive ranges, and the work-list order (longest range first).
struct Plan {
  std::vector<Seg> segs;
  std::vector<Range> ranges;
  std::vector<uint32_t> segfirst, spans, order;
  std::vector<uint32_t> slicefirst;   // VAR16: first payload slice of each range (and the total)
  uint64_t total = 0;
};

// Device addresses of one flush's work list (packed in one upload) and of its
// range summaries: in the handle's grow-only buffers, or in the static
// scratch array given to process_batch.
struct FlushBufs {
  Seg *segs = nullptr;
  Range *ranges = nullptr;
  uint32_t *order = nullptr, *segfirst = nullptr, *spans = nullptr, *qhead = nullptr, *slicefirst = nullptr;
  RHdr *rhdr = nullptr;
  UItem *ru = nullptr;
  OItem *ro = nullptr;
  uint32_t *rnslots = nullptr;
  uint32_t *rmore = nullptr;   // per summary row: threads left to extra passes
  uint64_t *paylen = nullptr;   // VAR16: per payload slice, its bytes and then its offset
};

enum { TM_PREPASS = 0, TM_RANGE, TM_COMBINE, TM_FINAL, TM_READOUT, TM_IVOUT, TM_DECODE, TM_PAYLOAD, TM_N };

}  // namespace

struct thapi_tally {
  thapi_tally_config cfg{};
  std::vector<uint8_t> has_size;
  int dev = 0;
  hipStream_t st = nullptr;
  bool own_stream = false;
  int n_cu = 256;
  size_t lds_limit = 65536;

  std::mutex mu;            // queue, registry, budget
  std::mutex run_mu;        // serialises flush / read / reset / close
  std::condition_variable cv;
  std::map<SKey, uint32_t> stream_idx;
  std::vector<SKey> stream_keys;
  std::vector<uint64_t> dropped;
  std::deque<Chunk> queue;
  uint64_t next_ticket = 1;
  uint64_t budget_used = 0;
  int failed = 0;
  bool finalized = false;

  Tables tb{};
  uint32_t gcap = 0;
  void *d_gkeys = nullptr, *d_gvals = nullptr, *d_ngs = nullptr, *d_ths = nullptr, *d_tht = nullptr,
       *d_tally = nullptr, *d_ktally = nullptr, *d_cstate = nullptr, *d_cstack = nullptr, *d_sstats = nullptr,
       *d_err = nullptr, *d_hs = nullptr, *d_thord = nullptr, *d_snth = nullptr;
  Shape shape{};
  bool shape_forced = false;                          // THAPI_TALLY_SHAPE gave a shape that fits
  uint64_t seen_threads = 0, seen_streams = 0;        // threads and streams at the end of the last flush
  uint32_t e4096 = 0;                                 // FIXED24: most tally entries beside a 4096-record tile (0: none)
  uint32_t last_shape[4] = {0, 0, 0, 0};              // {T, E, rpc, pipe} of the last flush (T = 0: none yet)

  DevBuf rhdr, ru, ro, rnslots, rmore, paylen;
  DevBuf wide_pack;                                   // the extra passes' work list
  // packed chunks decoded into VAR16 for one flush: per-packet counts and
  // offsets, then the headers and kept payload words
  DevBuf pk_scr, pk_hdr, pk_heap;
  // payload roles (thapi_tally_set_roles): the copy and handle tables
  bool roles_on = false;
  PayTables pt{};
  uint32_t hcap = 0;
  void *d_roles = nullptr, *d_copies = nullptr, *d_hk = nullptr, *d_hs2 = nullptr, *d_hc = nullptr, *d_hr = nullptr,
       *d_hx = nullptr, *d_hlk = nullptr, *d_hlm = nullptr, *d_hln = nullptr;
  DevBuf hstat;
  // THAPI_INTERVALS: the current flush's interval buffers (see Tables), the
  // public records of the last intervals() call and its offsets / keys
  DevBuf iv, iv_n, iv_h0, iv_snap, civ, civ_n, ivout, ivaux;
  DevBuf part, part_gslot, part_mask;                  // partial tallies of the current flush (see Tables)
  uint32_t iv_nranges = 0;                            // summary rows of the last flush
  std::vector<uint64_t> iv_bases;                     // their first IvRec
  bool iv_valid = false;                              // the interval buffers hold the last flush's
  DevBuf plan_pack;                                   // the work list, uploaded in one copy
  FlushBufs fb;                                       // the current flush's device addresses
  DevBuf keys, vals, keys2, vals2, gbeg, gend, cnt, off, rows, tstats;
  DevBuf read_pack;                                   // the readout's host tables, uploaded in one copy
  DevView rank_key, trace_span, stream_rank, rstream;
  void *h_pinned = nullptr;  // small pinned staging for results of device->host copies
  size_t h_pinned_cap = 0;
  void *h_plan = nullptr;    // pinned staging of the work list (asynchronous uploads)
  size_t h_plan_cap = 0;

  double timings[TM_N] = {0};
  double dec_ms1 = 0;                                 // packed decode: count and scan (the writes follow)
  bool dec_pending = false;
  hipEvent_t ev[2 * TM_N] = {};

  std::string arch;                                   // gcnArchName of the device
  std::map<std::string, std::array<uint32_t, 4>> tuned;  // autotuned {T, E, rpc, pipe} per workload class
  bool flushed_any = false;
  hipGraphExec_t gexec = nullptr;                     // THAPI_GRAPH: the captured pipeline
  std::array<uint64_t, 26> gsig{};
  uint64_t graph_builds = 0, graph_launches = 0;
  std::string cache_path;

  // THAPI_SERVICE: the continuous-batching worker and the device arena that
  // admits staged chunks (capacity = device_budget_bytes, FIFO reuse)
  std::thread worker;
  bool stop = false;
  std::condition_variable work_cv;                    // worker: chunks ready or stop
  bool worker_running = false;
  hipStream_t cst[N_COPY_STREAMS] = {};               // host -> device copies (chunk k on stream k % N)
  uint8_t *arena = nullptr;                           // device arena, capacity device_budget_bytes
  Fifo afifo;
  uint8_t *ring = nullptr;                            // pinned staging ring, min(budget, RING_MAX) bytes
  Fifo rfifo;
  std::vector<hipEvent_t> ev_pool;                    // copy-completion events
  // host input without the service: chunks are staged one after another in a
  // grow-only device arena that is reused once none of them is live any more
  // (so a steady submit/flush cycle allocates nothing); a chunk that does not
  // fit gets a buffer of its own.  hin_live counts every staged host-input
  // byte, hin_in the arena's, hin_want the most ever live at once.
  uint8_t *hin = nullptr;
  uint64_t hin_cap = 0, hin_top = 0, hin_in = 0, hin_live = 0, hin_want = 0;
  hipStream_t hst = nullptr;                          // its copies
  std::vector<int> ev_free;
  uint64_t done_upto = 0;                             // every ticket <= this one is tallied
  std::vector<uint64_t> done_ns;                      // [ticket] CLOCK_MONOTONIC ns of its batch's completion
  uint64_t n_batches = 0, n_batch_chunks = 0, max_batch_chunks = 0, bytes_admitted = 0;

  // the rows of the last read that did not fit its buffer (the size query of
  // a two-call read), kept until the tallies or streams change
  std::atomic<uint64_t> gen{0};       // bumped by submit, flush and reset
  // export: the blob of a size query, kept for the second call
  std::vector<uint8_t> exp_blob;
  bool exp_valid = false;
  uint64_t exp_gen = 0;
  DevBuf merge_buf;
  bool rc_valid = false;
  uint64_t rc_gen = 0;
  uint32_t rc_scope = 0, rc_trace = 0;
  thapi_tally_row *rc_rows = nullptr;   // pinned, grow-only; rc_n rows valid
  size_t rc_n = 0, rc_cap = 0;
  thapi_tally_stats rc_stats{};
};

namespace {

int hip_fail(thapi_tally *t, hipError_t e) {
  if (e == hipSuccess) return THAPI_OK;
  if (t) t->failed = THAPI_E_DEVICE;
  return THAPI_E_DEVICE;
}
#define HIPCHK(x) do { hipError_t _e = (x); if (_e != hipSuccess) return hip_fail(t, _e); } while (0)

// The record layout the kernels see: packed chunks are turned into VAR16
// before a flush tallies them.
int kfmt(const thapi_tally *t) { return t->cfg.format == THAPI_FMT_FIXED24 ? 1 : 2; }
// Granularity of submitted record bytes (packed chunks: 8-byte words).
uint32_t record_size(const thapi_tally *t) {
  return t->cfg.format == THAPI_FMT_FIXED24 ? 24u : (t->cfg.format == THAPI_FMT_VAR16 ? 16u : 8u);
}

// Resets every table in one launch on the handle's stream; `wait` also
// waits for it (a reset does not: whatever follows on the stream is ordered
// after it).
hipError_t init_tables(thapi_tally *t, bool wait = true) {
  const thapi_tally_config &c = t->cfg;
  hipError_t e;
  // every table in one launch
  InitSet is{};
  is.gkeys = (uint64_t *)t->d_gkeys; is.n_gkeys = t->gcap;
  is.gvals = (uint32_t *)t->d_gvals; is.n_gvals = t->gcap;
  is.ngs = (uint32_t *)t->d_ngs;
  is.err = (uint32_t *)t->d_err;
  is.tally = t->tb.tally; is.n_tally = (size_t)c.max_threads * c.n_fns;
  is.ktally = t->tb.ktally; is.n_ktally = (size_t)c.max_streams * c.n_kernel_ids;
  is.cstate = (uint32_t *)t->d_cstate; is.n_cstate = (size_t)c.max_threads * sizeof(CState) / 4;
  is.sstats = (uint64_t *)t->d_sstats; is.n_sstats = (size_t)c.max_streams * ST_N;
  is.s_nth = (uint32_t *)t->d_snth; is.n_s_nth = c.max_streams;
  if ((e = launch_init_all(is, t->st)) != hipSuccess) return e;
  return wait ? hipStreamSynchronize(t->st) : hipSuccess;
}

void free_all(thapi_tally *t) {
  void *ps[] = {t->d_gkeys, t->d_gvals, t->d_ngs, t->d_ths, t->d_tht, t->d_tally, t->d_ktally,
                t->d_cstate, t->d_cstack, t->d_sstats, t->d_err, t->d_hs, t->d_thord, t->d_snth,
                t->d_roles, t->d_copies, t->d_hk, t->d_hs2, t->d_hc, t->d_hr, t->d_hx,
                t->d_hlk, t->d_hlm, t->d_hln};
  for (void *p : ps) if (p) hipFree(p);
  DevBuf *bs[] = {&t->plan_pack, &t->rhdr, &t->ru, &t->ro, &t->rnslots, &t->rmore, &t->wide_pack, &t->paylen, &t->keys, &t->vals, &t->keys2,
                  &t->vals2, &t->gbeg, &t->gend, &t->cnt, &t->off, &t->read_pack, &t->rows, &t->tstats,
                  &t->merge_buf, &t->iv, &t->iv_n, &t->iv_h0, &t->iv_snap, &t->civ, &t->civ_n, &t->ivout,
                  &t->ivaux, &t->pk_scr, &t->pk_hdr, &t->pk_heap, &t->hstat, &t->part, &t->part_gslot,
                  &t->part_mask};
  for (DevBuf *b : bs) b->release();
  for (auto &c : t->queue) if (c.owned) hipFree(c.owned);
  t->queue.clear();
  if (t->h_pinned) hipHostFree(t->h_pinned);
  if (t->h_plan) hipHostFree(t->h_plan);
  if (t->rc_rows) { hipHostFree(t->rc_rows); t->rc_rows = nullptr; }
  for (auto &e : t->ev) if (e) hipEventDestroy(e);
  if (t->gexec) { hipGraphExecDestroy(t->gexec); t->gexec = nullptr; }
  if (t->arena) { hipFree(t->arena); t->arena = nullptr; }
  if (t->hin) { hipFree(t->hin); t->hin = nullptr; t->hin_cap = 0; }
  if (t->hst) { hipStreamDestroy(t->hst); t->hst = nullptr; }
  if (t->ring) { hipHostFree(t->ring); t->ring = nullptr; }
  for (auto &s : t->cst) if (s) { hipStreamDestroy(s); s = nullptr; }
  for (auto &e : t->ev_pool) if (e) hipEventDestroy(e);
  t->ev_pool.clear();
  if (t->own_stream && t->st) hipStreamDestroy(t->st);
}

// Picks the range kernel's tile and LDS tally size for the format and depth:
// the largest tile and tally that fit the LDS, preferring a full tally (2048
// entries) over a larger tile, then as many more tally entries (in steps of
// 64, up to TALLY_E_MAX) as the rest of the LDS holds: more (thread, fn) keys
// stay in LDS instead of overflowing to the global table.
// THAPI_TALLY_SHAPE="T,E[,rpc[,pipe]]" overrides the choice (used to tune
// the launch shape); one that is not valid or does not fit is ignored, and
// the default then follows the threads per stream as without it.
constexpr uint32_t TALLY_E_MAX = 4096;
uint32_t grow_tally(const thapi_tally *t, uint32_t T, uint32_t E, uint32_t KL) {
  const uint32_t D = t->cfg.max_depth;
  while (E + 64 <= TALLY_E_MAX && range_lds_bytes(T, E + 64, KL, D, kfmt(t)) + 256 <= t->lds_limit) E += 64;
  return E;
}
Shape pick_shape(const thapi_tally *t, bool *forced) {
  Shape s{};
  const uint32_t D = t->cfg.max_depth;
  const int fmt = kfmt(t);
  s.KL = std::min<uint32_t>(t->cfg.n_kernel_ids, KL_MAX);
  s.rpc = 1;
  s.pipe = 1;   // producer and walker waves overlap (the faster schedule on the layered workload)
  *forced = false;
  auto fits = [&](uint32_t T, uint32_t E) {
    size_t b = range_lds_bytes(T, E, s.KL, D, fmt);
    if (b + 256 > t->lds_limit) return false;  // (plus the kernel's static LDS)
    s.T = T; s.E = E; s.lds_bytes = (uint32_t)b;
    return true;
  };
  if (const char *env = getenv("THAPI_TALLY_SHAPE")) {
    unsigned T = 0, E = 0, rpc = 1, pipe = 1;
    const int n = sscanf(env, "%u,%u,%u,%u", &T, &E, &rpc, &pipe);
    const bool t_ok = T == 1024 || T == 2048 || (T == 4096 && fmt == 1);   // (4096: FIXED24 only)
    if (n >= 2 && t_ok && E >= 64 && E % 64 == 0 && rpc >= 1 && rpc <= 64 && pipe <= 1 && fits(T, E)) {
      s.rpc = rpc;
      s.pipe = pipe;
      *forced = true;
      return s;
    }
  }
  const uint32_t cand[][2] = {{2048, 2048}, {1024, 2048}, {2048, 1024}, {1024, 1024},
                              {1024, 512}, {1024, 256}, {1024, 128}, {1024, 64}};
  for (auto &c : cand)
    if (fits(c[0], c[1])) {
      if (c[1] == 2048) fits(c[0], grow_tally(t, c[0], c[1], s.KL));
      return s;
    }
  s.T = 0;
  return s;
}

hipError_t timed_begin(thapi_tally *t, int k) {
  if (!(t->cfg.flags & THAPI_PROFILE)) return hipSuccess;
  return hipEventRecord(t->ev[2 * k], t->st);
}
hipError_t timed_end(thapi_tally *t, int k) {
  if (!(t->cfg.flags & THAPI_PROFILE)) return hipSuccess;
  return hipEventRecord(t->ev[2 * k + 1], t->st);
}
void collect_timing(thapi_tally *t, int k) {
  if (!(t->cfg.flags & THAPI_PROFILE)) return;
  float ms = 0;
  if (hipEventElapsedTime(&ms, t->ev[2 * k], t->ev[2 * k + 1]) == hipSuccess) t->timings[k] = ms;
}

hipError_t ensure_pinned(thapi_tally *t, size_t bytes) {
  if (bytes <= t->h_pinned_cap) return hipSuccess;
  if (t->h_pinned) hipHostFree(t->h_pinned);
  t->h_pinned = nullptr;
  t->h_pinned_cap = 0;
  size_t want = std::max<size_t>(bytes, 4096);
  hipError_t e = hipHostMalloc(&t->h_pinned, want, hipHostMallocDefault);
  if (e == hipSuccess) t->h_pinned_cap = want;
  return e;
}

}  // namespace

extern "C" {

const char *thapi_tally_strerror(int code) {
  switch (code) {
    case THAPI_OK: return "ok";
    case THAPI_E_INVAL: return "invalid argument";
    case THAPI_E_NOMEM: return "out of device memory or chunk larger than the budget";
    case THAPI_E_AGAIN: return "device budget full, retry later";
    case THAPI_E_DEPTH: return "a thread's call stack exceeded max_depth";
    case THAPI_E_MALFORMED: return "anomalies counted (strict mode)";
    case THAPI_E_DEVICE: return "HIP device error";
    case THAPI_E_BUFSZ: return "row buffer too small";
    case THAPI_E_CAPACITY: return "configured capacity exceeded (streams, threads or threads per range)";
    case THAPI_E_STATE: return "call not valid in the handle's state";
    default: return "unknown status";
  }
}

namespace {
void load_tune_cache(thapi_tally *t);
void service_loop(thapi_tally *t);
hipError_t grow_plan_staging(thapi_tally *t, size_t bytes);
hipError_t clear_payload_tables(thapi_tally *t);
}  // namespace

int thapi_tally_open(const thapi_tally_config *cfg, thapi_tally **out) {
  if (!cfg || !out) return THAPI_E_INVAL;
  if (cfg->abi_version != THAPI_TALLY_ABI_VERSION) return THAPI_E_INVAL;
  if (cfg->format != THAPI_FMT_FIXED24 && cfg->format != THAPI_FMT_VAR16 && cfg->format != THAPI_FMT_PACKED)
    return THAPI_E_INVAL;
  if (cfg->n_fns < 1 || cfg->n_fns > 65536 || cfg->n_kernel_ids > 65536) return THAPI_E_INVAL;
  if (cfg->max_depth > THAPI_MAX_DEPTH_LIMIT || cfg->reserved) return THAPI_E_INVAL;
  if (cfg->max_threads > (1u << 30) || cfg->max_streams > (1u << 24)) return THAPI_E_INVAL;
  // the streaming form's batches differ in size from one to the next, so a
  // captured graph would be rebuilt for nearly every batch: not offered
  if ((cfg->flags & THAPI_SERVICE) && (cfg->flags & THAPI_GRAPH)) return THAPI_E_INVAL;
  // intervals are kept per flush; the service flushes on its own schedule
  if ((cfg->flags & THAPI_SERVICE) && (cfg->flags & THAPI_INTERVALS)) return THAPI_E_INVAL;
  thapi_tally *t = new (std::nothrow) thapi_tally();
  if (!t) return THAPI_E_NOMEM;
  t->cfg = *cfg;
  if (!t->cfg.max_depth) t->cfg.max_depth = 64;
  if (!t->cfg.max_threads) t->cfg.max_threads = 65536;
  if (!t->cfg.max_streams) t->cfg.max_streams = 4096;
  if (!t->cfg.device_budget_bytes) t->cfg.device_budget_bytes = 16ull << 30;
  t->cfg.fn_has_size = nullptr;
  if (cfg->autotune_cache) t->cache_path = cfg->autotune_cache;
  t->cfg.autotune_cache = nullptr;
  if (cfg->format != THAPI_FMT_FIXED24 && cfg->fn_has_size)
    t->has_size.assign(cfg->fn_has_size, cfg->fn_has_size + cfg->n_fns);
  const thapi_tally_config &c = t->cfg;
  auto bail = [&](int code) { free_all(t); delete t; return code; };
  t->dev = c.device;
  if (hipSetDevice(c.device) != hipSuccess) return bail(THAPI_E_DEVICE);
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, c.device) == hipSuccess && v > 0) t->n_cu = v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, c.device) == hipSuccess && v > 0)
    t->lds_limit = (size_t)v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeSharedMemPerBlockOptin, c.device) == hipSuccess &&
      (size_t)v > t->lds_limit)
    t->lds_limit = (size_t)v;
  if (c.hip_stream) {
    t->st = (hipStream_t)c.hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&t->st, hipStreamNonBlocking) != hipSuccess) return bail(THAPI_E_DEVICE);
    t->own_stream = true;
  }
  for (auto &e : t->ev)
    if (hipEventCreate(&e) != hipSuccess) return bail(THAPI_E_DEVICE);
  t->gcap = 1;
  while (t->gcap < 2ull * c.max_threads) t->gcap <<= 1;
  const uint32_t D = c.max_depth;
  struct A { void **p; size_t bytes; } allocs[] = {
      {&t->d_gkeys, 8ull * t->gcap},
      {&t->d_gvals, 4ull * t->gcap},
      {&t->d_ngs, 256},
      {&t->d_ths, 4ull * c.max_threads},
      {&t->d_tht, 4ull * c.max_threads},
      {&t->d_tally, sizeof(Tally) * (size_t)c.max_threads * c.n_fns},
      {&t->d_ktally, sizeof(KTally) * (size_t)c.max_streams * std::max<uint32_t>(c.n_kernel_ids, 1)},
      {&t->d_cstate, sizeof(CState) * (size_t)c.max_threads},
      {&t->d_cstack, sizeof(Frame) * (size_t)c.max_threads * D},
      {&t->d_sstats, 8ull * c.max_streams * ST_N},
      {&t->d_err, 256},
      {&t->d_hs, std::max<size_t>(c.n_fns, 1)},
      {&t->d_thord, 4ull * c.max_threads},
      {&t->d_snth, 4ull * c.max_streams},
  };
  for (auto &a : allocs) {
    hipError_t e = hipMalloc(a.p, a.bytes);
    if (e != hipSuccess) { hipGetLastError(); return bail(THAPI_E_NOMEM); }
  }
  Tables &tb = t->tb;
  tb.gkeys = (uint64_t *)t->d_gkeys; tb.gvals = (uint32_t *)t->d_gvals; tb.gmask = t->gcap - 1;
  tb.n_gslots = (uint32_t *)t->d_ngs; tb.max_threads = c.max_threads;
  tb.th_stream = (uint32_t *)t->d_ths; tb.th_tid = (uint32_t *)t->d_tht;
  tb.th_ord = (uint32_t *)t->d_thord; tb.s_nth = (uint32_t *)t->d_snth;
  tb.tally = (Tally *)t->d_tally; tb.n_fns = c.n_fns;
  tb.ktally = (KTally *)t->d_ktally; tb.n_kid = c.n_kernel_ids;
  tb.cstate = (CState *)t->d_cstate; tb.cstack = (Frame *)t->d_cstack; tb.D = D;
  tb.sstats = (unsigned long long *)t->d_sstats; tb.err = (uint32_t *)t->d_err;
  tb.has_size = nullptr;
  if (!t->has_size.empty()) {
    if (hipMemcpy(t->d_hs, t->has_size.data(), c.n_fns, hipMemcpyHostToDevice) != hipSuccess)
      return bail(THAPI_E_DEVICE);
    tb.has_size = (const uint8_t *)t->d_hs;
  }
  t->shape = pick_shape(t, &t->shape_forced);
  if (kfmt(t) == 1 && range_lds_bytes(4096, 1024, t->shape.KL, c.max_depth, 1) + 256 <= t->lds_limit)
    t->e4096 = grow_tally(t, 4096, 1024, t->shape.KL);
  if (!t->shape.T) return bail(THAPI_E_INVAL);
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c.device) == hipSuccess) t->arch = prop.gcnArchName;
    const std::string::size_type colon = t->arch.find(':');
    if (colon != std::string::npos) t->arch.resize(colon);
    if (t->arch.empty()) t->arch = "gpu";
  }
  load_tune_cache(t);
  // pinned staging for the work list and for counters read back, sized up
  // front
  if (grow_plan_staging(t, 1u << 20) != hipSuccess ||
      ensure_pinned(t, 64 + (24 + 8ull * ST_N) * c.max_streams) != hipSuccess)
    return bail(THAPI_E_NOMEM);
  if (prepare_range_kernels((uint32_t)(t->lds_limit - 256)) != hipSuccess) return bail(THAPI_E_DEVICE);
  if (scratch_setup(c.device) != hipSuccess) return bail(THAPI_E_DEVICE);
  if (prepare_combine_kernel() != hipSuccess) return bail(THAPI_E_DEVICE);
  if (c.flags & THAPI_SERVICE) {
    for (auto &s : t->cst)
      if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return bail(THAPI_E_DEVICE);
    if (!(c.flags & THAPI_DEVICE_INPUT)) {
      if (hipMalloc((void **)&t->arena, c.device_budget_bytes) != hipSuccess) {
        hipGetLastError();
        return bail(THAPI_E_NOMEM);
      }
      t->afifo.cap = c.device_budget_bytes;
      const uint64_t rcap = std::min<uint64_t>(c.device_budget_bytes, RING_MAX);
      if (hipHostMalloc((void **)&t->ring, rcap, hipHostMallocDefault) != hipSuccess) {
        hipGetLastError();
        return bail(THAPI_E_NOMEM);
      }
      t->rfifo.cap = rcap;
    }
  }
  if (init_tables(t) != hipSuccess) return bail(THAPI_E_DEVICE);
  if (c.flags & THAPI_SERVICE) {
    t->worker_running = true;
    t->worker = std::thread(service_loop, t);
  }
  *out = t;
  return THAPI_OK;
}

namespace {

// A copy-completion event from the pool (caller holds t->mu); -1 if none
// could be created.
int event_get(thapi_tally *t) {
  if (!t->ev_free.empty()) { const int k = t->ev_free.back(); t->ev_free.pop_back(); return k; }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) { hipGetLastError(); return -1; }
  t->ev_pool.push_back(e);
  return (int)t->ev_pool.size() - 1;
}

// Gives a staged chunk's arena, ring and event back (caller holds t->mu;
// chunks are released in ticket order).
void release_chunk(thapi_tally *t, const Chunk &c) {
  if (c.in_arena) {
    t->afifo.release_front();
    if (c.in_ring) t->rfifo.release_front();
    if (c.ev >= 0) t->ev_free.push_back(c.ev);
    t->budget_used -= c.owned_bytes;
  } else if (c.in_hin) {
    t->budget_used -= c.owned_bytes;
    t->hin_live -= c.owned_bytes;
    t->hin_in -= c.owned_bytes;
    if (!t->hin_in) t->hin_top = 0;
  } else if (c.owned) {
    hipFree(c.owned);
    t->budget_used -= c.owned_bytes;
    t->hin_live -= c.owned_bytes;
  }
}

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

namespace {
// Events of a packed chunk held in host memory, checked the way the decode
// kernels check them (magic, sizes, 8-byte alignment, events filling each
// packet exactly, packets contiguous and covering the chunk); UINT64_MAX
// when it is malformed.
uint64_t packed_events(const uint8_t *buf, uint64_t nbytes, const uint64_t *index, uint64_t n_packets) {
  uint64_t events = 0;
  for (uint64_t k = 0; k < n_packets; k++) {
    const uint64_t off = index[k];
    if (off % 8 || off + 16 > nbytes || (k == 0 && off != 0)) return UINT64_MAX;
    uint32_t h[4];
    memcpy(h, buf + off, 16);
    if (h[0] != 0x4B504854u || h[3] || h[1] < 16 || h[1] % 8 || off + h[1] > nbytes) return UINT64_MAX;
    if ((k + 1 < n_packets ? index[k + 1] : nbytes) != off + h[1]) return UINT64_MAX;
    uint64_t o = 16;
    for (uint32_t e = 0; e < h[2]; e++) {
      if (o + 16 > h[1]) return UINT64_MAX;
      const uint64_t sz = (16 + (uint64_t)buf[off + o + 15] + 7) / 8 * 8;
      if (o + sz > h[1]) return UINT64_MAX;
      o += sz;
    }
    if (o != h[1]) return UINT64_MAX;
    events += h[2];
  }
  return events;
}
}  // namespace

int thapi_tally_submit(thapi_tally *t, thapi_stream_key key, const void *records, size_t record_bytes,
                       const void *payload, size_t payload_bytes, uint64_t *ticket_out) {
  if (!t || key.reserved) return THAPI_E_INVAL;
  const uint32_t rs = record_size(t);
  if (record_bytes % rs) return THAPI_E_INVAL;
  if (record_bytes && !records) return THAPI_E_INVAL;
  const bool var = t->cfg.format == THAPI_FMT_VAR16;
  const bool pk = t->cfg.format == THAPI_FMT_PACKED;
  if (!var && !pk && (payload || payload_bytes)) return THAPI_E_INVAL;
  if (payload_bytes && !payload) return THAPI_E_INVAL;
  // packed: the payload argument is the packet index (u64 offsets), one packet at least
  if (pk && (payload_bytes % 8 || (record_bytes && !payload_bytes) || (!record_bytes && payload_bytes) ||
             payload_bytes / 8 > UINT32_MAX))
    return THAPI_E_INVAL;
  const bool dev_in = (t->cfg.flags & THAPI_DEVICE_INPUT) != 0;
  if (dev_in && ((uintptr_t)records & 7)) return THAPI_E_INVAL;
  const uint64_t n_rec = record_bytes / rs;
  {
    std::lock_guard<std::mutex> g(t->mu);
    if (t->failed) return THAPI_E_STATE;
    if (t->finalized) return THAPI_E_STATE;
  }
  if (hipSetDevice(t->dev) != hipSuccess) return THAPI_E_DEVICE;
  // VAR16: the payload heap must hold exactly the declared payload lengths.
  // Host input is checked here; device input is checked on the GPU by the
  // flush that tallies the chunk (no synchronisation per submit).
  if (var && n_rec && !dev_in) {
    uint64_t sum = 0;
    const uint8_t *r = (const uint8_t *)records;
    for (uint64_t i = 0; i < n_rec; i++) sum += r[i * 16 + 15];
    if (sum != payload_bytes) return THAPI_E_INVAL;
  } else if (var && !n_rec && payload_bytes) {
    return THAPI_E_INVAL;
  }
  uint64_t pk_events = 0;
  if (pk && n_rec && !dev_in) {
    if (((uintptr_t)payload & 7) != 0) return THAPI_E_INVAL;
    pk_events = packed_events((const uint8_t *)records, record_bytes, (const uint64_t *)payload, payload_bytes / 8);
    if (pk_events == UINT64_MAX) return THAPI_E_INVAL;
  }
  if (pk && dev_in && ((uintptr_t)payload & 7)) return THAPI_E_INVAL;
  std::unique_lock<std::mutex> lk(t->mu);
  t->gen++;
  SKey sk{key.trace_id, key.host_id, key.pid};
  auto it = t->stream_idx.find(sk);
  uint32_t sidx;
  if (it == t->stream_idx.end()) {
    if (t->stream_keys.size() >= t->cfg.max_streams) return THAPI_E_CAPACITY;
    sidx = (uint32_t)t->stream_keys.size();
    t->stream_idx[sk] = sidx;
    t->stream_keys.push_back(sk);
    t->dropped.push_back(0);
  } else {
    sidx = it->second;
  }
  Chunk c{};
  c.ev = -1;
  c.stream = sidx;
  c.n_rec = pk ? 0 : n_rec;
  if (pk) { c.pk_bytes = record_bytes; c.pk_packets = payload_bytes / 8; }
  c.pay_bytes = payload_bytes;
  c.ready = true;
  const bool service = (t->cfg.flags & THAPI_SERVICE) != 0;
  if (dev_in) {
    c.rec = (const uint8_t *)records;
    c.pay = (const uint8_t *)payload;
  } else if (n_rec && service) {
    // admission: wait for room in the device arena and the pinned staging
    // ring (both FIFO), queue the chunk in ticket order at once, then -- outside
    // the lock -- copy the caller's bytes into the ring and enqueue the ring ->
    // arena copy on one of the copy streams with an event after it.  The
    // worker's launch waits for that event on the device, so a submit never
    // waits for its own DMA; the caller's buffer is free when submit returns.
    const uint64_t rec_al = (record_bytes + 255) / 256 * 256;
    const uint64_t bytes = rec_al + (payload_bytes + 255) / 256 * 256;
    if (bytes > t->cfg.device_budget_bytes) return THAPI_E_NOMEM;
    const bool via_ring = bytes <= t->rfifo.cap;   // (larger chunks: one synchronous pageable copy)
    uint64_t off = 0, roff = 0;
    for (;;) {
      if (t->failed || t->stop) return THAPI_E_STATE;
      if (t->afifo.fit(bytes, &off) && (!via_ring || t->rfifo.fit(bytes, &roff))) break;
      if (t->cfg.flags & THAPI_DROP_ON_FULL) {
        t->dropped[sidx] += pk ? pk_events : n_rec;
        if (ticket_out) *ticket_out = 0;
        return THAPI_OK;
      }
      if (t->cfg.flags & THAPI_NONBLOCKING) return THAPI_E_AGAIN;
      t->cv.wait(lk);
    }
    const int ev = via_ring ? event_get(t) : -1;
    if (via_ring && ev < 0) return THAPI_E_DEVICE;
    t->afifo.take(off, bytes);
    if (via_ring) t->rfifo.take(roff, bytes);
    t->budget_used += bytes;
    t->bytes_admitted += record_bytes + payload_bytes;
    c.in_arena = true;
    c.in_ring = via_ring;
    c.owned_bytes = bytes;
    c.rec = t->arena + off;
    c.pay = payload_bytes ? t->arena + off + rec_al : nullptr;
    c.ready = false;
    c.ev = ev;
    c.ticket = t->next_ticket++;
    const uint64_t ticket = c.ticket;
    hipStream_t cs = t->cst[ticket % N_COPY_STREAMS];
    t->queue.push_back(c);
    lk.unlock();
    hipError_t e;
    if (via_ring) {
      uint8_t *h = t->ring + roff;
      memcpy(h, records, record_bytes);
      if (payload_bytes) memcpy(h + rec_al, payload, payload_bytes);
      e = hipMemcpyAsync(t->arena + off, h, rec_al + payload_bytes, hipMemcpyHostToDevice, cs);
      if (e == hipSuccess) e = hipEventRecord(t->ev_pool[ev], cs);
    } else {
      e = hipMemcpyAsync(t->arena + off, records, record_bytes, hipMemcpyHostToDevice, cs);
      if (e == hipSuccess && payload_bytes)
        e = hipMemcpyAsync(t->arena + off + rec_al, payload, payload_bytes, hipMemcpyHostToDevice, cs);
      if (e == hipSuccess) e = hipStreamSynchronize(cs);
    }
    lk.lock();
    for (auto it = t->queue.rbegin(); it != t->queue.rend(); ++it)
      if (it->ticket == ticket) { it->ready = true; break; }
    t->cv.notify_all();
    if (e != hipSuccess) {
      t->failed = THAPI_E_DEVICE;
      t->work_cv.notify_all();
      return THAPI_E_DEVICE;
    }
    if (ticket_out) *ticket_out = ticket;
    t->work_cv.notify_all();
    return THAPI_OK;
  } else if (n_rec) {
    const uint64_t bytes = record_bytes + payload_bytes + 64;
    if (bytes > t->cfg.device_budget_bytes) return THAPI_E_NOMEM;
    while (t->budget_used + bytes > t->cfg.device_budget_bytes) {
      if (t->cfg.flags & THAPI_DROP_ON_FULL) {
        t->dropped[sidx] += pk ? pk_events : n_rec;
        if (ticket_out) *ticket_out = 0;
        return THAPI_OK;
      }
      if (t->cfg.flags & THAPI_NONBLOCKING) return THAPI_E_AGAIN;
      t->cv.wait(lk);
      if (t->failed) return THAPI_E_STATE;
    }
    t->budget_used += bytes;
    t->hin_live += bytes;
    t->hin_want = std::max(t->hin_want, t->hin_live);
    hipError_t e = hipSuccess;
    if (!t->hst) e = hipStreamCreateWithFlags(&t->hst, hipStreamNonBlocking);
    if (e == hipSuccess && !t->hin_in && t->hin_cap < t->hin_want) {
      // nothing staged in the arena: grow it to the most host input held at once so far
      if (t->hin) hipFree(t->hin);
      t->hin = nullptr;
      t->hin_cap = 0;
      const uint64_t want = (t->hin_want + (1ull << 20) - 1) & ~((1ull << 20) - 1);
      if (hipMalloc((void **)&t->hin, want) == hipSuccess) t->hin_cap = want;
      else { hipGetLastError(); t->hin = nullptr; }
    }
    void *d = nullptr;
    const uint64_t at = (t->hin_top + 255) & ~255ull;
    if (e == hipSuccess && t->hin && at + bytes <= t->hin_cap) {
      d = t->hin + at;
      t->hin_top = at + bytes;
      t->hin_in += bytes;
      c.in_hin = true;
    }
    lk.unlock();
    if (e == hipSuccess && !d) e = hipMalloc(&d, bytes);
    if (e == hipSuccess) e = hipMemcpyAsync(d, records, record_bytes, hipMemcpyHostToDevice, t->hst);
    if (e == hipSuccess && payload_bytes)
      e = hipMemcpyAsync((uint8_t *)d + ((record_bytes + 15) / 16 * 16), payload, payload_bytes,
                         hipMemcpyHostToDevice, t->hst);
    if (e == hipSuccess) e = hipStreamSynchronize(t->hst);
    lk.lock();
    if (e != hipSuccess) {
      if (c.in_hin) {
        t->hin_in -= bytes;
        if (!t->hin_in) t->hin_top = 0;
      } else if (d) {
        hipFree(d);
      }
      t->budget_used -= bytes;
      t->hin_live -= bytes;
      t->cv.notify_all();
      return e == hipErrorOutOfMemory ? THAPI_E_NOMEM : hip_fail(t, e);
    }
    c.owned = c.in_hin ? nullptr : d;
    c.owned_bytes = bytes;
    c.rec = (const uint8_t *)d;
    c.pay = payload_bytes ? (const uint8_t *)d + ((record_bytes + 15) / 16 * 16) : nullptr;
  }
  c.ticket = t->next_ticket++;
  if (ticket_out) *ticket_out = c.ticket;
  t->queue.push_back(c);
  if (service) t->work_cv.notify_all();
  return THAPI_OK;
}

namespace {


// With max_ranges, the work list holds at most that many ranges (every
// chunk still gets at least one; the caller checks n_seg <= max_ranges).
void plan_work(const thapi_tally *t, const std::vector<Chunk> &work, const Shape &sh, Plan &pl,
               uint64_t max_ranges = 0) {
  pl = Plan();
  for (auto &c : work) pl.total += c.n_rec;
  // The work list holds about rpc * n_cu ranges: with n_seg chunks, ranges of
  // ceil(total / (rpc * n_cu - n_seg)) records give at most rpc * n_cu of
  // them (each chunk adds at most one partial range).  Ranges are never
  // shorter than 4 tiles.  The combine folds one stream's range summaries one
  // after the other, so a stream of N records gets at most about
  // sqrt(N / RANGE_FOLD) ranges: the count that balances the range kernel's
  // time (N / R records per workgroup) against the fold's (R summaries), with
  // RANGE_FOLD the records a workgroup tallies in the time one summary takes
  // to fold (measured: about 4.4 ns per record; about 1.1 us per summary
  // with the U items folded in parallel).
  constexpr double RANGE_FOLD = 250.0;
  uint64_t n_seg = 0;
  std::map<uint32_t, uint64_t> per_stream;
  for (auto &c : work) {
    n_seg += c.n_rec ? 1 : 0;
    per_stream[c.stream] += c.n_rec;
  }
  const uint64_t ncu = std::max<uint64_t>(1, (uint64_t)t->n_cu) * std::max<uint32_t>(1, sh.rpc);
  uint64_t target = ncu > 2 * n_seg ? ncu - n_seg : std::max<uint64_t>(1, ncu / 2);
  // each chunk adds at most one partial range to the total / rlen full ones
  if (max_ranges) target = std::min<uint64_t>(target, max_ranges > n_seg ? max_ranges - n_seg : 1);
  uint64_t rlen = (pl.total + target - 1) / target;
  rlen = std::max<uint64_t>(rlen, 4ull * sh.T);
  rlen = std::min<uint64_t>(rlen, 1ull << 30);
  for (size_t i = 0; i < work.size(); i++) {
    const Chunk &c = work[i];
    if (!c.n_rec) continue;
    Seg sg{};
    sg.rec = c.rec; sg.pay = c.pay; sg.n_rec = c.n_rec; sg.pay_bytes = c.pay_bytes; sg.stream = c.stream;
    pl.segfirst.push_back((uint32_t)pl.ranges.size());
    const uint32_t si = (uint32_t)pl.segs.size();
    pl.segs.push_back(sg);
    const uint64_t ns = per_stream[c.stream];
    const uint64_t rmax = std::max<uint64_t>(1, (uint64_t)std::sqrt((double)ns / RANGE_FOLD));
    const uint64_t rl = std::max<uint64_t>(rlen, (ns + rmax - 1) / rmax);
    const uint64_t nr = (c.n_rec + rl - 1) / rl;
    const uint64_t step = (c.n_rec + nr - 1) / nr;
    for (uint64_t b = 0; b < c.n_rec; b += step) {
      Range r{};
      r.seg = si; r.stream = c.stream; r.begin = b; r.n = std::min<uint64_t>(step, c.n_rec - b); r.pay_begin = 0;
      if (pl.spans.empty() || pl.spans[pl.spans.size() - 3] != c.stream) {
        pl.spans.push_back(c.stream); pl.spans.push_back((uint32_t)pl.ranges.size());
        pl.spans.push_back((uint32_t)pl.ranges.size());
      }
      pl.ranges.push_back(r);
      pl.spans[pl.spans.size() - 1] = (uint32_t)pl.ranges.size();
    }
  }
  pl.segfirst.push_back((uint32_t)pl.ranges.size());
  {
    uint64_t acc = 0;   // intervals: each range may write one per record, from here
    for (auto &r : pl.ranges) { r.iv_base = acc; acc += r.n; }
  }
  {
    uint32_t acc = 0;   // payload slices of each range
    for (auto &r : pl.ranges) { pl.slicefirst.push_back(acc); acc += (uint32_t)((r.n + PAY_SLICE - 1) / PAY_SLICE); }
    pl.slicefirst.push_back(acc);
  }
  // longest first: the persistent workgroups take them in this order, so the
  // short ranges fill in at the end (LPT scheduling)
  pl.order.resize(pl.ranges.size());
  for (uint32_t k = 0; k < pl.order.size(); k++) pl.order[k] = k;
  std::stable_sort(pl.order.begin(), pl.order.end(),
                   [&](uint32_t a, uint32_t b) { return pl.ranges[a].n > pl.ranges[b].n; });
}

// Bytes of a packed upload of n arrays: 256-byte aligned parts of at least
// 256 bytes each.
size_t pack_bytes(const size_t *bytes, int n) {
  size_t tot = 0;
  for (int i = 0; i < n; i++) tot += std::max<size_t>((bytes[i] + 255) & ~(size_t)255, 256);
  return tot;
}

// Grows the pinned staging of packed uploads to `bytes` at least.
hipError_t grow_plan_staging(thapi_tally *t, size_t bytes) {
  if (bytes <= t->h_plan_cap) return hipSuccess;
  if (t->h_plan) hipHostFree(t->h_plan);
  t->h_plan = nullptr;
  t->h_plan_cap = 0;
  const size_t want = std::max<size_t>(bytes, 1 << 16);
  hipError_t e = hipHostMalloc(&t->h_plan, want, hipHostMallocDefault);
  if (e == hipSuccess) t->h_plan_cap = want;
  return e;
}

// Host -> device upload of n host arrays in one asynchronous copy: they are
// packed at 256-byte aligned offsets in the pinned staging buffer (which must
// hold pack_bytes() already) and land at the same offsets of `dev`; *views[i]
// receives the device address of array i.  The staging is reused by the next
// call only, which comes after the work that the copy feeds has completed
// (flushes and reads each end with a synchronisation).
hipError_t stage_h2d(thapi_tally *t, uint8_t *dev, void **const *views, const void *const *src,
                     const size_t *bytes, int n) {
  size_t o = 0, used = 0;
  for (int i = 0; i < n; i++) {
    if (bytes[i]) {
      memcpy((uint8_t *)t->h_plan + o, src[i], bytes[i]);
      used = o + bytes[i];
    }
    *views[i] = dev + o;
    o += std::max<size_t>((bytes[i] + 255) & ~(size_t)255, 256);
  }
  return used ? hipMemcpyAsync(dev, t->h_plan, used, hipMemcpyHostToDevice, t->st) : hipSuccess;
}

// Sizes of one flush's device buffers: the packed work list and the range
// summaries (RHdr per range and slot, U and O items per range, slot and level).
struct PlanSizes {
  size_t part[7];
  size_t pack, rhdr, ru, ro, rnslots, rmore, paylen;
  size_t total() const {
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    return al(pack) + al(rhdr) + al(ru) + al(ro) + al(rnslots) + al(rmore) + al(paylen);
  }
};

PlanSizes plan_sizes(const thapi_tally *t, const Plan &pl) {
  const size_t nR = pl.ranges.size(), nS = pl.segs.size();
  const size_t D = t->cfg.max_depth;
  PlanSizes z{};
  const size_t part[7] = {sizeof(Seg) * nS, sizeof(Range) * nR, 4 * nR, 4 * (nS + 1), 4 * pl.spans.size(), 4,
                          4 * pl.slicefirst.size()};
  for (int i = 0; i < 7; i++) z.part[i] = part[i];
  z.pack = pack_bytes(part, 7);
  z.rhdr = sizeof(RHdr) * nR * S_MAX;
  z.ru = sizeof(UItem) * nR * S_MAX * D;
  z.ro = sizeof(OItem) * nR * S_MAX * D;
  z.rnslots = 4 * std::max<size_t>(nR, 1);
  z.rmore = 4 * std::max<size_t>(nR, 1);
  z.paylen = 8 * std::max<size_t>(pl.slicefirst.empty() ? 1 : pl.slicefirst.back(), 1);
  return z;
}

// Uploads the work list and points t->fb at the flush's buffers: the
// handle's grow-only buffers, or -- with `scratch` -- consecutive 256-byte
// aligned parts of that device array, which the caller has checked is large
// enough (as it has the pinned staging).
constexpr size_t PART_MAX_BYTES = 1ull << 30;   // partial tallies of one flush at most
hipError_t upload_plan(thapi_tally *t, const Plan &pl, uint8_t *scratch = nullptr) {
  const PlanSizes z = plan_sizes(t, pl);
  hipError_t e;
#define UPCHK(x) do { if ((e = (x)) != hipSuccess) return e; } while (0)
  uint8_t *pack;
  FlushBufs &fb = t->fb;
  if (scratch) {
    size_t o = 0;
    auto carve = [&](size_t bytes) { uint8_t *p = scratch + o; o += (bytes + 255) & ~(size_t)255; return p; };
    pack = carve(z.pack);
    fb.rhdr = (RHdr *)carve(z.rhdr);
    fb.ru = (UItem *)carve(z.ru);
    fb.ro = (OItem *)carve(z.ro);
    fb.rnslots = (uint32_t *)carve(z.rnslots);
    fb.rmore = (uint32_t *)carve(z.rmore);
    fb.paylen = (uint64_t *)carve(z.paylen);
    t->tb.part_ranges = 0;   // (the ranges add their tallies with global atomics)
  } else {
    UPCHK(t->rhdr.ensure(z.rhdr));
    UPCHK(t->ru.ensure(z.ru));
    UPCHK(t->ro.ensure(z.ro));
    UPCHK(t->rnslots.ensure(z.rnslots));
    UPCHK(t->rmore.ensure(z.rmore));
    UPCHK(t->paylen.ensure(z.paylen));
    UPCHK(t->plan_pack.ensure(z.pack));
    UPCHK(grow_plan_staging(t, z.pack));
    pack = t->plan_pack.as<uint8_t>();
    fb.rhdr = t->rhdr.as<RHdr>();
    fb.ru = t->ru.as<UItem>();
    fb.ro = t->ro.as<OItem>();
    fb.rnslots = t->rnslots.as<uint32_t>();
    fb.rmore = t->rmore.as<uint32_t>();
    fb.paylen = t->paylen.as<uint64_t>();
    // partial tallies for as many ranges as PART_MAX_BYTES holds
    const size_t per = part_range_bytes(t->cfg.n_fns, kfmt(t));
    const uint64_t np = std::min<uint64_t>(pl.ranges.size(), PART_MAX_BYTES / per);
    t->tb.part_ranges = 0;
    if (np) {
      UPCHK(t->part.ensure(per * np));
      UPCHK(t->part_gslot.ensure(4ull * PART_ORDS * np));
      UPCHK(t->part_mask.ensure(4ull * np));
      t->tb.part = t->part.as<uint8_t>();
      t->tb.part_gslot = t->part_gslot.as<uint32_t>();
      t->tb.part_mask = t->part_mask.as<uint32_t>();
      t->tb.part_ranges = (uint32_t)np;
    }
  }
  // the work queue's head (zero) travels with the work list
  static const uint32_t zero = 0;
  const void *src[7] = {pl.segs.data(), pl.ranges.data(), pl.order.data(), pl.segfirst.data(), pl.spans.data(), &zero,
                        pl.slicefirst.data()};
  void **dst[7] = {(void **)&fb.segs, (void **)&fb.ranges, (void **)&fb.order, (void **)&fb.segfirst,
                   (void **)&fb.spans, (void **)&fb.qhead, (void **)&fb.slicefirst};
  UPCHK(stage_h2d(t, pack, dst, src, z.part, 7));
#undef UPCHK
  return hipSuccess;
}

// THAPI_INTERVALS: sizes the interval buffers for the planned flush and
// points the tables at them (each range may write one IvRec per record; the
// combine at most one interval per U item it folds).
hipError_t prepare_intervals(thapi_tally *t, const Plan &pl) {
  Tables &tb = t->tb;
  if (!(t->cfg.flags & THAPI_INTERVALS)) return hipSuccess;
  const size_t nR = std::max<size_t>(pl.ranges.size(), 1), D = t->cfg.max_depth;
  const size_t pairs = nR * S_MAX;
  const size_t ccap = std::min<size_t>(pairs * D, 0xFFFFFFF0u);
  hipError_t e;
  if ((e = t->iv.ensure(sizeof(IvRec) * std::max<uint64_t>(pl.total, 1))) != hipSuccess) return e;
  if ((e = t->iv_n.ensure(4 * nR)) != hipSuccess) return e;
  if ((e = t->iv_h0.ensure(4 * pairs)) != hipSuccess) return e;
  if ((e = t->iv_snap.ensure(sizeof(IvFrame) * pairs * D)) != hipSuccess) return e;
  if ((e = t->civ.ensure(sizeof(CIval) * ccap)) != hipSuccess) return e;
  if ((e = t->civ_n.ensure(4)) != hipSuccess) return e;
  tb.iv = t->iv.as<IvRec>();
  tb.iv_n = t->iv_n.as<uint32_t>();
  tb.iv_h0 = t->iv_h0.as<uint32_t>();
  tb.iv_snap = t->iv_snap.as<IvFrame>();
  tb.civ = t->civ.as<CIval>();
  tb.civ_n = t->civ_n.as<uint32_t>();
  tb.civ_cap = (uint32_t)ccap;
  t->iv_nranges = (uint32_t)pl.ranges.size();
  t->iv_bases.resize(pl.ranges.size());
  for (size_t i = 0; i < pl.ranges.size(); i++) t->iv_bases[i] = pl.ranges[i].iv_base;
  t->iv_valid = true;
  return hipSuccess;
}

// The kernels of one flush, in stream order.  `timed` records the per-kernel
// events (not used under graph capture).
hipError_t launch_pipeline(thapi_tally *t, const Plan &pl, const Shape &sh, bool final, bool timed) {
  const uint32_t nR = (uint32_t)pl.ranges.size(), nS = (uint32_t)pl.segs.size();
  const uint32_t nSp = (uint32_t)(pl.spans.size() / 3);
  const FlushBufs &fb = t->fb;
  hipError_t e;
#define LPCHK(x) do { if ((e = (x)) != hipSuccess) return e; } while (0)
#define TB(k) do { if (timed) LPCHK(timed_begin(t, k)); } while (0)
#define TE(k) do { if (timed) LPCHK(timed_end(t, k)); } while (0)
  LPCHK(launch_fill32(t->tb.err, 1, 0, t->st));
  if (t->tb.civ_n) LPCHK(launch_fill32(t->tb.civ_n, 1, 0, t->st));
  if (nR) {
    if (kfmt(t) == 2) {
      TB(TM_PREPASS);
      const uint32_t nSl = pl.slicefirst.back();
      LPCHK(launch_paylen(fb.segs, fb.ranges, nR, fb.segfirst, nS, fb.slicefirst, nSl, fb.paylen, t->tb.err, t->st));
      TE(TM_PREPASS);
      if (t->roles_on) {
        TB(TM_PAYLOAD);
        LPCHK(launch_payload(fb.segs, fb.ranges, nR, fb.slicefirst, nSl, fb.paylen, t->pt, t->st));
        TE(TM_PAYLOAD);
      }
    }
    TB(TM_RANGE);
    LPCHK(launch_range(kfmt(t), sh.T, fb.segs, fb.ranges, fb.order, nR, fb.qhead, (uint32_t)t->n_cu, t->tb,
                       sh, fb.rhdr, fb.ru, fb.ro, fb.rnslots, fb.rmore, fb.ranges, 0, t->st));
    TE(TM_RANGE);
    TB(TM_COMBINE);
    LPCHK(launch_combine(fb.spans, nSp, fb.rhdr, fb.ru, fb.ro, fb.rnslots, t->tb, nullptr, t->st));
    LPCHK(launch_part_merge(kfmt(t), fb.spans, nSp, t->tb, t->st));
    TE(TM_COMBINE);
  }
  if (final) {
    TB(TM_FINAL);
    LPCHK(launch_final(t->tb, t->cfg.max_threads, t->st));
    TE(TM_FINAL);
  }
#undef TB
#undef TE
#undef LPCHK
  return hipSuccess;
}

// THAPI_GRAPH: the pipeline is captured once per launch signature (sizes,
// shape, buffers) and replayed while the signature repeats.
hipError_t run_pipeline(thapi_tally *t, const Plan &pl, const Shape &sh, bool final) {
  const bool prof = (t->cfg.flags & THAPI_PROFILE) != 0;
  if (!(t->cfg.flags & THAPI_GRAPH)) return launch_pipeline(t, pl, sh, final, prof);
  const std::array<uint64_t, 26> sig = {pl.slicefirst.empty() ? 0 : pl.slicefirst.back(),
                                        (uint64_t)(uintptr_t)t->fb.slicefirst,
                                        pl.ranges.size(), pl.segs.size(), pl.spans.size(), sh.T, sh.E,
                                        sh.rpc | ((uint64_t)sh.pipe << 32), final ? 1u : 0u,
                                        (uint64_t)(uintptr_t)t->tb.iv, (uint64_t)(uintptr_t)t->tb.civ,
                                        (uint64_t)(uintptr_t)t->tb.iv_n, (uint64_t)(uintptr_t)t->tb.iv_h0,
                                        (uint64_t)(uintptr_t)t->tb.iv_snap, (uint64_t)(uintptr_t)t->tb.civ_n,
                                        (uint64_t)(uintptr_t)t->fb.segs,
                                        (uint64_t)(uintptr_t)t->fb.ranges, (uint64_t)(uintptr_t)t->fb.order,
                                        (uint64_t)(uintptr_t)t->fb.rhdr, (uint64_t)(uintptr_t)t->fb.ru,
                                        (uint64_t)(uintptr_t)t->fb.ro, (uint64_t)(uintptr_t)t->fb.rnslots,
                                        (uint64_t)(uintptr_t)t->fb.spans, (uint64_t)(uintptr_t)t->fb.paylen,
                                        (uint64_t)(uintptr_t)t->tb.part, t->tb.part_ranges};
  hipError_t e;
  if (!t->gexec || sig != t->gsig) {
    if (t->gexec) { hipGraphExecDestroy(t->gexec); t->gexec = nullptr; }
    hipGraph_t g = nullptr;
    if ((e = hipStreamBeginCapture(t->st, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
    const hipError_t le = launch_pipeline(t, pl, sh, final, false);
    e = hipStreamEndCapture(t->st, &g);
    if (le != hipSuccess) { if (g) hipGraphDestroy(g); return le; }
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&t->gexec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) { t->gexec = nullptr; return e; }
    t->gsig = sig;
    t->graph_builds++;
  }
  if (prof && (e = timed_begin(t, TM_RANGE)) != hipSuccess) return e;
  if ((e = hipGraphLaunch(t->gexec, t->st)) != hipSuccess) return e;
  if (prof && (e = timed_end(t, TM_RANGE)) != hipSuccess) return e;
  t->graph_launches++;
  return hipSuccess;
}

// ---- autotune cache: one line per workload class, "key T E rpc pipe"
std::string tune_key(const thapi_tally *t, const std::vector<Chunk> &work) {
  uint64_t total = 0, nseg = 0;
  for (auto &c : work) { total += c.n_rec; nseg += c.n_rec ? 1 : 0; }
  auto lg = [](uint64_t x) { int b = 0; while (x > 1) { x >>= 1; b++; } return b; };
  char k[160];
  snprintf(k, sizeof k, "%s/cu%d/fmt%u/D%u/fns%d/segs%d/recs%d", t->arch.c_str(), t->n_cu, t->cfg.format,
           t->cfg.max_depth, lg(t->cfg.n_fns), lg(nseg), lg(total));
  return k;
}

void load_tune_cache(thapi_tally *t) {
  if (t->cache_path.empty()) return;
  FILE *f = fopen(t->cache_path.c_str(), "r");
  if (!f) return;
  char key[256];
  unsigned T, E, rpc, pipe;
  while (fscanf(f, "%255s %u %u %u %u", key, &T, &E, &rpc, &pipe) == 5) t->tuned[key] = {T, E, rpc, pipe};
  fclose(f);
}

void save_tune_cache(thapi_tally *t) {
  if (t->cache_path.empty()) return;
  FILE *f = fopen(t->cache_path.c_str(), "w");
  if (!f) return;
  for (auto &kv : t->tuned)
    fprintf(f, "%s %u %u %u %u\n", kv.first.c_str(), kv.second[0], kv.second[1], kv.second[2], kv.second[3]);
  fclose(f);
}

// The default schedule for this handle: builders and walkers overlap
// (pipelined) unless the streams it has tallied so far hold more than
// WIDE_STREAM_THREADS threads each on average.  Each thread then brings only
// a few records to a half tile, and its windows run nearly empty, so the
// whole-tile schedule (every wave builds, then every wave walks, with every
// slot's partial window waiting for its next records) is faster (measured:
// pipelined 1.3x faster at 8 threads per stream, 1.3x slower at 12, 2.2x
// slower at 64).
// With the pipelined schedule, FIXED24 streams whose threads (on average, so
// far) all get direct-mapped rows in the largest tally that fits beside a
// tile of 4096 records use that tile: each hand-over between the building
// and the walking waves then moves twice the records (measured on the
// layered workload: range kernel 1.83 -> 1.58 ms).
constexpr uint64_t WIDE_STREAM_THREADS = 10;
Shape default_shape(const thapi_tally *t) {
  Shape s = t->shape;
  if (t->shape_forced || !t->seen_streams) return s;
  if (t->seen_threads > WIDE_STREAM_THREADS * t->seen_streams) {
    s.pipe = 0;
    return s;
  }
  if (kfmt(t) == 1 && s.pipe && t->e4096) {
    const uint64_t tps = (t->seen_threads + t->seen_streams - 1) / t->seen_streams;
    if (tps * t->cfg.n_fns <= t->e4096) {
      s.T = 4096;
      s.E = t->e4096;
      s.lds_bytes = (uint32_t)range_lds_bytes(4096, s.E, s.KL, t->cfg.max_depth, 1);
    }
  }
  return s;
}

// The shape for this work: a tuned entry when one matches, else the default.
Shape shape_for(thapi_tally *t, const std::vector<Chunk> &work) {
  if (t->tuned.empty()) return default_shape(t);
  auto it = t->tuned.find(tune_key(t, work));
  if (it == t->tuned.end()) return default_shape(t);
  Shape s = t->shape;
  const size_t b = range_lds_bytes(it->second[0], it->second[1], s.KL, t->cfg.max_depth, kfmt(t));
  const bool t_ok = it->second[0] == 1024 || it->second[0] == 2048 || (it->second[0] == 4096 && kfmt(t) == 1);
  if (t_ok && it->second[1] >= 64 && b + 256 <= t->lds_limit) {
    s.T = it->second[0]; s.E = it->second[1]; s.lds_bytes = (uint32_t)b;
    s.rpc = std::max<uint32_t>(1, std::min<uint32_t>(it->second[2], 64));
    s.pipe = it->second[3] ? 1u : 0u;
  }
  return s;
}

}  // namespace

namespace {

// Tallies one batch of chunks (taken off the queue by the caller) and, with
// `final`, closes every stream.  Caller holds run_mu.
// Groups the chunks of one batch by stream (each stream's chunks stay in
// ticket order), picks the launch shape and plans the work list.
Shape prepare_batch(thapi_tally *t, std::vector<Chunk> &work, Plan &pl, uint64_t max_ranges = 0) {
  std::stable_sort(work.begin(), work.end(), [](const Chunk &a, const Chunk &b) { return a.stream < b.stream; });
  const Shape sh = shape_for(t, work);
  t->last_shape[0] = sh.T; t->last_shape[1] = sh.E; t->last_shape[2] = sh.rpc; t->last_shape[3] = sh.pipe;
  plan_work(t, work, sh, pl, max_ranges);
  return sh;
}

// After a first pass that left threads to extra passes (ERR_WIDE: some
// range met more threads of its stream than slot_cap holds in LDS; the
// combine and the final flush did nothing): one extra pass over such a
// range per class of slot_cap stream-thread ordinals (the threads the first
// pass took are skipped), each writing summary rows of its own after the
// first pass's; then the combine, whose spans list each range followed by
// its extra passes (threads are disjoint between them, and each thread's
// summaries stay in record order), and the final flush.  *err receives the
// error bits of this second launch.
hipError_t run_extra_passes(thapi_tally *t, const Plan &pl, const Shape &sh, bool final, uint32_t *err) {
  const uint32_t nR = (uint32_t)pl.ranges.size(), D = t->cfg.max_depth, SC = slot_cap(D);
  const size_t nst = t->stream_keys.size();
  hipError_t e;
#define XCHK(x) do { if ((e = (x)) != hipSuccess) return e; } while (0)
  XCHK(ensure_pinned(t, 4ull * (nR + nst) + 64));
  uint32_t *h = (uint32_t *)t->h_pinned;
  XCHK(hipMemcpyAsync(h, t->fb.rmore, 4ull * nR, hipMemcpyDeviceToHost, t->st));
  XCHK(hipMemcpyAsync(h + nR, t->tb.s_nth, 4ull * nst, hipMemcpyDeviceToHost, t->st));
  XCHK(hipStreamSynchronize(t->st));
  std::vector<Range> ex;
  std::vector<uint32_t> clist, spans2;
  uint64_t ivtot = pl.total;
  for (size_t k = 0; k + 2 < pl.spans.size(); k += 3) {
    const uint32_t stream = pl.spans[k], rb = pl.spans[k + 1], re = pl.spans[k + 2];
    spans2.push_back(stream);
    spans2.push_back((uint32_t)clist.size());
    for (uint32_t r = rb; r < re; r++) {
      clist.push_back(r);
      if (!h[r]) continue;
      const uint32_t classes = (h[nR + stream] + SC - 1) / SC;
      for (uint32_t c = 0; c < classes; c++) {
        Range x = pl.ranges[r];
        x.pass = c + 1;
        x.parent = r;
        x.iv_base = ivtot;
        ivtot += x.n;
        clist.push_back(nR + (uint32_t)ex.size());
        ex.push_back(x);
      }
    }
    spans2.push_back((uint32_t)clist.size());
  }
  const uint32_t nE = (uint32_t)ex.size(), nRows = nR + nE;
  std::vector<uint32_t> order2(nE);
  for (uint32_t k = 0; k < nE; k++) order2[k] = k;
  std::stable_sort(order2.begin(), order2.end(), [&](uint32_t a, uint32_t b) { return ex[a].n > ex[b].n; });
  // summary rows for the extra passes, after the first pass's (kept)
  XCHK(t->rhdr.ensure_keep(sizeof(RHdr) * nRows * S_MAX, sizeof(RHdr) * nR * S_MAX, t->st));
  XCHK(t->ru.ensure_keep(sizeof(UItem) * nRows * S_MAX * D, sizeof(UItem) * nR * S_MAX * D, t->st));
  XCHK(t->ro.ensure_keep(sizeof(OItem) * nRows * S_MAX * D, sizeof(OItem) * nR * S_MAX * D, t->st));
  XCHK(t->rnslots.ensure_keep(4ull * nRows, 4ull * nR, t->st));
  XCHK(t->rmore.ensure_keep(4ull * nRows, 4ull * nR, t->st));
  FlushBufs &fb = t->fb;
  fb.rhdr = t->rhdr.as<RHdr>();
  fb.ru = t->ru.as<UItem>();
  fb.ro = t->ro.as<OItem>();
  fb.rnslots = t->rnslots.as<uint32_t>();
  fb.rmore = t->rmore.as<uint32_t>();
  if (t->cfg.flags & THAPI_INTERVALS) {
    // the extra passes' intervals follow the first pass's
    Tables &tb = t->tb;
    const size_t pairs = (size_t)nRows * S_MAX;
    const size_t ccap = std::min<size_t>(pairs * D, 0xFFFFFFF0u);
    XCHK(t->iv.ensure_keep(sizeof(IvRec) * std::max<uint64_t>(ivtot, 1), sizeof(IvRec) * pl.total, t->st));
    XCHK(t->iv_n.ensure_keep(4ull * nRows, 4ull * nR, t->st));
    XCHK(t->iv_h0.ensure(4 * pairs));
    XCHK(t->iv_snap.ensure(sizeof(IvFrame) * pairs * D));
    XCHK(t->civ.ensure(sizeof(CIval) * ccap));
    tb.iv = t->iv.as<IvRec>();
    tb.iv_n = t->iv_n.as<uint32_t>();
    tb.iv_h0 = t->iv_h0.as<uint32_t>();
    tb.iv_snap = t->iv_snap.as<IvFrame>();
    tb.civ = t->civ.as<CIval>();
    tb.civ_cap = (uint32_t)ccap;
    t->iv_nranges = nRows;
    for (auto &x : ex) t->iv_bases.push_back(x.iv_base);
  }
  // the extra work list, its order, the combine's positions and spans, and
  // the work queue's head (zero), up in one copy
  static const uint32_t zero = 0;
  const size_t bytes[5] = {sizeof(Range) * nE, 4ull * nE, 4 * clist.size(), 4 * spans2.size(), 4};
  XCHK(grow_plan_staging(t, pack_bytes(bytes, 5)));
  XCHK(t->wide_pack.ensure(pack_bytes(bytes, 5)));
  Range *d_ex = nullptr;
  uint32_t *d_order = nullptr, *d_clist = nullptr, *d_spans = nullptr, *d_qhead = nullptr;
  void **views[5] = {(void **)&d_ex, (void **)&d_order, (void **)&d_clist, (void **)&d_spans, (void **)&d_qhead};
  const void *src[5] = {ex.data(), order2.data(), clist.data(), spans2.data(), &zero};
  XCHK(stage_h2d(t, t->wide_pack.as<uint8_t>(), views, src, bytes, 5));
  XCHK(launch_fill32(t->tb.err, 1, 0, t->st));
  if (t->tb.civ_n) XCHK(launch_fill32(t->tb.civ_n, 1, 0, t->st));
  Shape sx = sh;
  sx.pipe = 0;   // (extra passes run one schedule: all waves build a tile, then walk it)
  XCHK(launch_range(kfmt(t), sh.T, fb.segs, d_ex, d_order, nE, d_qhead, (uint32_t)t->n_cu, t->tb, sx,
                    fb.rhdr, fb.ru, fb.ro, fb.rnslots, fb.rmore, fb.ranges, nR, t->st));
  XCHK(launch_combine(d_spans, (uint32_t)(spans2.size() / 3), fb.rhdr, fb.ru, fb.ro, fb.rnslots, t->tb, d_clist,
                      t->st));
  if (final) XCHK(launch_final(t->tb, t->cfg.max_threads, t->st));
  XCHK(hipMemcpyAsync(h, t->tb.err, 4, hipMemcpyDeviceToHost, t->st));
  XCHK(hipStreamSynchronize(t->st));
  *err = h[0];
#undef XCHK
  return hipSuccess;
}

// Packed chunks of a batch (taken off the queue by the caller) become VAR16
// chunks in the handle's decode buffers.  All packets of the batch are
// decoded together: one count pass (one lane per packet, the packet index
// giving each lane its start), a scan of the counts, the per-chunk totals
// fetched, then one write pass.  The staged copies stay owned by the
// chunks.  A malformed chunk fails the handle with THAPI_E_INVAL (the batch
// is released untallied).  Caller holds run_mu.
int transcode_packed(thapi_tally *t, std::vector<Chunk> &work) {
  if (t->cfg.format != THAPI_FMT_PACKED) return THAPI_OK;
  std::vector<size_t> which;
  std::vector<PkChunk> desc;
  std::vector<uint64_t> first;
  uint64_t npk = 0;
  for (size_t i = 0; i < work.size(); i++)
    if (work[i].pk_packets) {
      which.push_back(i);
      desc.push_back(PkChunk{work[i].rec, work[i].pk_bytes, (const uint64_t *)work[i].pay, 0});
      first.push_back(npk);
      npk += work[i].pk_packets;
    }
  if (which.empty()) return THAPI_OK;
  first.push_back(npk);
  if (hipSetDevice(t->dev) != hipSuccess) return THAPI_E_DEVICE;
  const uint32_t nc = (uint32_t)which.size();
  // descriptors, packet prefix and the gathered totals after the scan scratch
  const size_t b_scr = (pk_scratch_bytes(npk) + 255) & ~(size_t)255;
  const size_t bytes[2] = {sizeof(PkChunk) * nc, 8ull * (nc + 1)};
  const size_t b_tot = 16ull * (nc + 1);
  HIPCHK(t->pk_scr.ensure(b_scr + pack_bytes(bytes, 2) + b_tot));
  uint8_t *sc = t->pk_scr.as<uint8_t>();
  HIPCHK(grow_plan_staging(t, pack_bytes(bytes, 2)));
  void *d_desc = nullptr, *d_first = nullptr;
  void **views[2] = {&d_desc, &d_first};
  const void *src[2] = {desc.data(), first.data()};
  HIPCHK(stage_h2d(t, sc + b_scr, views, src, bytes, 2));
  uint64_t *d_tot = (uint64_t *)(sc + b_scr + pack_bytes(bytes, 2));
  HIPCHK(launch_fill32(t->tb.err, 1, 0, t->st));
  // streaming form: the decode waits on the device for the chunks' copies
  for (size_t j : which)
    if (work[j].ev >= 0) HIPCHK(hipStreamWaitEvent(t->st, t->ev_pool[work[j].ev], 0));
  HIPCHK(timed_begin(t, TM_DECODE));
  HIPCHK(launch_pk_count((const PkChunk *)d_desc, (const uint64_t *)d_first, nc, npk, sc, d_tot, t->tb.err,
                         t->st));
  HIPCHK(timed_end(t, TM_DECODE));
  HIPCHK(ensure_pinned(t, b_tot + 16));
  uint64_t *h = (uint64_t *)t->h_pinned;
  HIPCHK(hipMemcpyAsync(h, d_tot, b_tot, hipMemcpyDeviceToHost, t->st));
  HIPCHK(hipMemcpyAsync(h + 2 * (nc + 1), t->tb.err, 4, hipMemcpyDeviceToHost, t->st));
  HIPCHK(hipStreamSynchronize(t->st));
  collect_timing(t, TM_DECODE);
  t->dec_ms1 = t->timings[TM_DECODE];
  if ((uint32_t)h[2 * (nc + 1)] & ERR_PAYLOAD) {
    std::lock_guard<std::mutex> g(t->mu);
    for (auto &c : work) release_chunk(t, c);
    work.clear();
    t->failed = THAPI_E_INVAL;
    t->cv.notify_all();
    return THAPI_E_INVAL;
  }
  const uint64_t ne = h[2 * nc], nb = h[2 * nc + 1];
  HIPCHK(t->pk_hdr.ensure(16 * std::max<uint64_t>(ne, 1)));
  HIPCHK(t->pk_heap.ensure(std::max<uint64_t>(nb, 8)));
  uint64_t *hdr = t->pk_hdr.as<uint64_t>(), *heap = t->pk_heap.as<uint64_t>();
  HIPCHK(timed_begin(t, TM_DECODE));
  HIPCHK(launch_pk_write((const PkChunk *)d_desc, (const uint64_t *)d_first, nc, npk, sc, hdr, heap, t->tb.err,
                         t->st));
  HIPCHK(timed_end(t, TM_DECODE));
  for (uint32_t j = 0; j < nc; j++) {
    Chunk &c = work[which[j]];
    c.rec = (const uint8_t *)(hdr + 2 * h[2 * j]);
    c.n_rec = h[2 * j + 2] - h[2 * j];
    c.pay = (const uint8_t *)heap + h[2 * j + 1];
    c.pay_bytes = h[2 * j + 3] - h[2 * j + 1];
    c.pk_packets = 0;
  }
  t->dec_pending = (t->cfg.flags & THAPI_PROFILE) != 0;
  return THAPI_OK;
}

// Tallies one batch of chunks, planned by prepare_batch (`pl`, `sh`) and
// taken off the queue by the caller, and with `final` closes every stream.
// With `scratch` the work list and range summaries go to that device array
// (already checked to be large enough) instead of the handle's buffers.
// Caller holds run_mu.
int process_batch(thapi_tally *t, std::vector<Chunk> &work, bool final, const Plan &pl, const Shape &sh,
                  uint8_t *scratch = nullptr) {
  t->gen++;
  if (hipSetDevice(t->dev) != hipSuccess) return THAPI_E_DEVICE;
  for (int k = 0; k < TM_N; k++) t->timings[k] = 0;
  const uint32_t nR = (uint32_t)pl.ranges.size();
  int rc = THAPI_OK;
  if (nR) HIPCHK(upload_plan(t, pl, scratch));
  HIPCHK(prepare_intervals(t, pl));
  // streaming form: the launch waits on the device for the chunks' copies
  for (auto &c : work)
    if (c.ev >= 0) HIPCHK(hipStreamWaitEvent(t->st, t->ev_pool[c.ev], 0));
  // (the scratch variant replays no graph: instantiating one allocates)
  const bool graph = (t->cfg.flags & THAPI_GRAPH) && !scratch;
  if (graph) HIPCHK(run_pipeline(t, pl, sh, final));
  else HIPCHK(launch_pipeline(t, pl, sh, final, (t->cfg.flags & THAPI_PROFILE) != 0));
  HIPCHK(ensure_pinned(t, 64));
  uint32_t *herr = (uint32_t *)t->h_pinned;
  HIPCHK(hipMemcpyAsync(herr, t->tb.err, 4, hipMemcpyDeviceToHost, t->st));
  HIPCHK(hipMemcpyAsync(herr + 1, t->tb.n_gslots, 4, hipMemcpyDeviceToHost, t->st));   // (threads so far)
  HIPCHK(hipStreamSynchronize(t->st));
  uint32_t err = *herr;
  t->seen_threads = herr[1];
  {
    std::lock_guard<std::mutex> g(t->mu);
    t->seen_streams = t->stream_keys.size();
  }
  bool nomem = false;
  if (err == ERR_WIDE) {
    // threads left to extra passes (their summary rows need memory that the
    // no-alloc flush does not have)
    if (scratch) nomem = true;
    else HIPCHK(run_extra_passes(t, pl, sh, final, &err));
  }
  if (graph) {
    collect_timing(t, TM_RANGE);  // whole graph
  } else {
    if (nR) {
      if (kfmt(t) == 2) collect_timing(t, TM_PREPASS);
      if (kfmt(t) == 2 && t->roles_on) collect_timing(t, TM_PAYLOAD);
      collect_timing(t, TM_RANGE);
      collect_timing(t, TM_COMBINE);
    }
    if (final) collect_timing(t, TM_FINAL);
  }
  if (t->dec_pending) {
    // the packed decode of this batch: its count and scan, then its writes
    collect_timing(t, TM_DECODE);
    t->timings[TM_DECODE] += t->dec_ms1;
    t->dec_pending = false;
  }
  {
    std::lock_guard<std::mutex> g(t->mu);
    for (auto &c : work) release_chunk(t, c);
    t->cv.notify_all();
    if (nomem) { t->failed = THAPI_E_NOMEM; rc = THAPI_E_NOMEM; }
    else if (err & ERR_PIPE) { t->failed = THAPI_E_DEVICE; rc = THAPI_E_DEVICE; }
    else if (err & ERR_PAYLOAD) { t->failed = THAPI_E_INVAL; rc = THAPI_E_INVAL; }
    else if (err & (ERR_CAPACITY | ERR_WIDE)) { t->failed = THAPI_E_CAPACITY; rc = THAPI_E_CAPACITY; }
    else if (err & ERR_DEPTH) { t->failed = THAPI_E_DEPTH; rc = THAPI_E_DEPTH; }
    if (final) t->finalized = true;
    t->flushed_any = true;
  }
  if (rc == THAPI_OK && (t->cfg.flags & THAPI_STRICT)) {
    // strict mode: any anomaly counted so far fails the flush
    const size_t nst = t->stream_keys.size();
    if (nst) {
      HIPCHK(ensure_pinned(t, 8 * nst * ST_N));
      const uint64_t *h = (const uint64_t *)t->h_pinned;
      HIPCHK(hipMemcpyAsync(t->h_pinned, t->tb.sstats, 8 * nst * ST_N, hipMemcpyDeviceToHost, t->st));
      HIPCHK(hipStreamSynchronize(t->st));
      for (size_t i = 0; i < nst; i++) {
        const uint64_t *c = &h[i * ST_N];
        if (c[ST_ORPHAN] || c[ST_MISMATCH] || c[ST_NEGDUR] || c[ST_UNDER] || c[ST_TSREG] || c[ST_UNCLOSED] ||
            c[ST_BAD])
          rc = THAPI_E_MALFORMED;
      }
    }
  }
  return rc;
}

// THAPI_SERVICE worker: the continuous-batching loop.  Each iteration takes
// every chunk whose copy has landed (the ready prefix of the queue, in ticket
// order), tallies them in one pipeline launch, stamps their completion time
// and frees their arena space, which admits waiting submitters.  Chunks that
// arrive meanwhile are copied on their own stream while the kernels run and
// join the next iteration.
void service_loop(thapi_tally *t) {
  hipSetDevice(t->dev);
  for (;;) {
    std::vector<Chunk> work;
    {
      std::unique_lock<std::mutex> lk(t->mu);
      t->work_cv.wait(lk, [&] {
        return t->stop || t->failed || (!t->queue.empty() && t->queue.front().ready);
      });
      if (t->failed) { t->worker_running = false; t->cv.notify_all(); return; }
      if (t->queue.empty() || !t->queue.front().ready) {
        if (t->stop) { t->worker_running = false; return; }
        continue;
      }
      while (!t->queue.empty() && t->queue.front().ready) {
        work.push_back(t->queue.front());
        t->queue.pop_front();
      }
    }
    uint64_t last = 0;
    for (auto &c : work) last = std::max(last, c.ticket);
    const size_t nchunks = work.size();
    int rc;
    {
      std::lock_guard<std::mutex> run(t->run_mu);
      rc = transcode_packed(t, work);
      if (rc == THAPI_OK) {
        Plan pl;
        const Shape sh = prepare_batch(t, work, pl);
        rc = process_batch(t, work, false, pl, sh);
      }
    }
    const uint64_t tdone = now_ns();
    std::lock_guard<std::mutex> g(t->mu);
    if (rc != THAPI_OK && rc != THAPI_E_MALFORMED && !t->failed) t->failed = rc;
    if (t->done_ns.size() <= last) t->done_ns.resize(last + 1, 0);
    for (auto &c : work) t->done_ns[c.ticket] = tdone;
    t->done_upto = std::max(t->done_upto, last);
    t->n_batches++;
    t->n_batch_chunks += nchunks;
    t->max_batch_chunks = std::max<uint64_t>(t->max_batch_chunks, nchunks);
    t->cv.notify_all();
  }
}

}  // namespace

int thapi_tally_flush(thapi_tally *t, uint64_t ticket, uint32_t flags) {
  if (!t) return THAPI_E_INVAL;
  const bool final = (flags & THAPI_FLUSH_FINAL) != 0;
  if (t->cfg.flags & THAPI_SERVICE) {
    // the worker tallies; wait until it has covered `ticket`
    std::unique_lock<std::mutex> lk(t->mu);
    if (t->finalized) return THAPI_E_STATE;
    const uint64_t want = std::min<uint64_t>(ticket, t->next_ticket - 1);
    t->cv.wait(lk, [&] { return t->failed || t->done_upto >= want || (want == 0); });
    if (t->failed) return t->failed == THAPI_E_DEVICE ? THAPI_E_DEVICE : t->failed;
    if (!final) return THAPI_OK;
    if (!t->queue.empty()) return THAPI_E_STATE;  // submits still arriving: finish them first
    lk.unlock();
    std::lock_guard<std::mutex> run(t->run_mu);
    std::vector<Chunk> none;
    Plan pl;
    const Shape sh = prepare_batch(t, none, pl);
    return process_batch(t, none, true, pl, sh);
  }
  std::lock_guard<std::mutex> run(t->run_mu);
  std::vector<Chunk> work;
  {
    std::lock_guard<std::mutex> g(t->mu);
    if (t->failed) return t->failed == THAPI_E_DEVICE ? THAPI_E_DEVICE : THAPI_E_STATE;
    if (t->finalized) return THAPI_E_STATE;
    while (!t->queue.empty() && t->queue.front().ticket <= ticket) {
      work.push_back(t->queue.front());
      t->queue.pop_front();
    }
  }
  const int trc = transcode_packed(t, work);
  if (trc != THAPI_OK) return trc;
  Plan pl;
  const Shape sh = prepare_batch(t, work, pl);
  return process_batch(t, work, final, pl, sh);
}

int thapi_tally_flush_noalloc(thapi_tally *t, uint64_t ticket, uint32_t flags) {
  if (!t) return THAPI_E_INVAL;
  if ((t->cfg.flags & (THAPI_SERVICE | THAPI_INTERVALS)) || !(t->cfg.flags & THAPI_DEVICE_INPUT) ||
      t->cfg.format == THAPI_FMT_PACKED)
    return THAPI_E_INVAL;
  if (t->dev < 0 || t->dev >= MAX_DEVICES) return THAPI_E_INVAL;
  uint8_t *const scr = scratch_on(t->dev);
  if (!scr) return THAPI_E_DEVICE;
  const bool final = (flags & THAPI_FLUSH_FINAL) != 0;
  std::lock_guard<std::mutex> run(t->run_mu);
  // the chunks up to `ticket` are planned first and taken off the queue only
  // when their work fits the array (only flushes, which hold run_mu, take
  // chunks off the queue; submits append)
  std::vector<Chunk> work;
  {
    std::lock_guard<std::mutex> g(t->mu);
    if (t->failed) return t->failed == THAPI_E_DEVICE ? THAPI_E_DEVICE : THAPI_E_STATE;
    if (t->finalized) return THAPI_E_STATE;
    for (auto &c : t->queue) {
      if (c.ticket > ticket) break;
      work.push_back(c);
    }
  }
  const size_t n_take = work.size();
  uint64_t n_seg = 0;
  for (auto &c : work) n_seg += c.n_rec ? 1 : 0;
  // bytes per range of the summaries (header and U / O items per slot) and
  // of its work-list entries; a fixed part covers the segments and the
  // 256-byte alignment of the eleven parts
  const uint64_t D = t->cfg.max_depth;
  const uint64_t per_range = sizeof(RHdr) * S_MAX + (sizeof(UItem) + sizeof(OItem)) * S_MAX * D +
                             sizeof(Range) + 4 * 5 + 8;
  const uint64_t fixed = 11 * 256 + (sizeof(Seg) + 4) * (n_seg + 1) + 12 * (n_seg + 1);
  if (fixed >= THAPI_NOALLOC_SCRATCH_BYTES) return THAPI_E_NOMEM;
  const uint64_t max_ranges = (THAPI_NOALLOC_SCRATCH_BYTES - fixed) / per_range;
  if (n_seg > max_ranges) return THAPI_E_NOMEM;
  Plan pl;
  const Shape sh = prepare_batch(t, work, pl, max_ranges ? max_ranges : 1);
  const PlanSizes z = plan_sizes(t, pl);
  if (z.total() > THAPI_NOALLOC_SCRATCH_BYTES || z.pack > t->h_plan_cap) return THAPI_E_NOMEM;
  {
    std::lock_guard<std::mutex> g(t->mu);
    for (size_t k = 0; k < n_take; k++) t->queue.pop_front();
  }
  std::lock_guard<std::mutex> dev_lock(g_noalloc_mu[t->dev]);
  return process_batch(t, work, final, pl, sh, scr);
}

int thapi_tally_ticket_done(thapi_tally *t, uint64_t ticket, uint64_t *done_ns) {
  if (!t || !ticket) return THAPI_E_INVAL;
  std::lock_guard<std::mutex> g(t->mu);
  if (ticket >= t->next_ticket) return THAPI_E_INVAL;
  if (ticket > t->done_upto || ticket >= t->done_ns.size()) return THAPI_E_AGAIN;
  if (done_ns) *done_ns = t->done_ns[ticket];
  return THAPI_OK;
}

int thapi_tally_service_info(thapi_tally *t, uint64_t *info, int n) {
  if (!t || (n && !info)) return THAPI_E_INVAL;
  std::lock_guard<std::mutex> g(t->mu);
  const uint64_t v[6] = {t->n_batches, t->n_batch_chunks, t->max_batch_chunks, t->bytes_admitted,
                         (uint64_t)t->queue.size(), t->budget_used};
  const int m = std::min(n, 6);
  for (int k = 0; k < m; k++) info[k] = v[k];
  return m;
}

int thapi_tally_last_shape(thapi_tally *t, uint32_t *shape) {
  if (!t || !shape) return THAPI_E_INVAL;
  std::lock_guard<std::mutex> run(t->run_mu);
  if (!t->last_shape[0]) return THAPI_E_STATE;
  for (int k = 0; k < 4; k++) shape[k] = t->last_shape[k];
  return THAPI_OK;
}

int thapi_tally_autotune(thapi_tally *t, uint32_t reps, uint32_t *chosen) {
  if (!t) return THAPI_E_INVAL;
  std::lock_guard<std::mutex> run(t->run_mu);
  std::vector<Chunk> work;
  {
    std::lock_guard<std::mutex> g(t->mu);
    if (t->failed) return t->failed == THAPI_E_DEVICE ? THAPI_E_DEVICE : THAPI_E_STATE;
    if (t->finalized || t->flushed_any || t->queue.empty() || (t->cfg.flags & THAPI_SERVICE) ||
        t->cfg.format == THAPI_FMT_PACKED)
      return THAPI_E_STATE;
    work.assign(t->queue.begin(), t->queue.end());
  }
  if (hipSetDevice(t->dev) != hipSuccess) return THAPI_E_DEVICE;
  std::stable_sort(work.begin(), work.end(), [](const Chunk &a, const Chunk &b) { return a.stream < b.stream; });
  reps = std::max<uint32_t>(1, std::min<uint32_t>(reps, 16));
  const uint32_t D = t->cfg.max_depth;
  const int fmt = kfmt(t);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  float best_ms = -1;
  Shape best = t->shape;
  const uint32_t Ts[] = {4096, 2048, 1024}, Es[] = {0, 2048, 1024}, rpcs[] = {1, 2, 4, 8, 16}, pipes[] = {0, 1};
  int rc = THAPI_OK;
  for (uint32_t T : Ts)
    for (uint32_t E0 : Es)
      for (uint32_t rpc : rpcs)
      for (uint32_t pipe : pipes) {
        if (T == 4096 && fmt != 1) continue;   // (FIXED24 only)
        // (E0 = 0: the most entries beyond 2048 that fit -- beyond 1024 beside
        // 4096-record tiles; skipped when none do)
        const uint32_t base = T == 4096 ? 1024u : 2048u;   // (4096 x 2048 does not fit)
        const uint32_t E = E0 ? E0 : grow_tally(t, T, base, t->shape.KL);
        if (!E0 && E == base) continue;
        Shape sh = t->shape;
        const size_t b = range_lds_bytes(T, E, sh.KL, D, fmt);
        if (b + 256 > t->lds_limit) continue;
        sh.T = T; sh.E = E; sh.rpc = rpc; sh.pipe = pipe; sh.lds_bytes = (uint32_t)b;
        Plan pl;
        plan_work(t, work, sh, pl);
        float ms_min = -1;
        bool ok = true;
        for (uint32_t r = 0; r < reps + 1 && ok; r++) {
          hipError_t e = init_tables(t);
          if (e == hipSuccess) e = upload_plan(t, pl);
          if (e == hipSuccess) e = prepare_intervals(t, pl);
          if (e == hipSuccess) e = hipEventRecord(e0, t->st);
          if (e == hipSuccess) e = launch_pipeline(t, pl, sh, false, false);
          if (e == hipSuccess) e = hipEventRecord(e1, t->st);
          uint32_t herr = 0;
          if (e == hipSuccess) e = hipMemcpyAsync(&herr, t->tb.err, 4, hipMemcpyDeviceToHost, t->st);
          if (e == hipSuccess) e = hipStreamSynchronize(t->st);
          if (e != hipSuccess) { rc = hip_fail(t, e); ok = false; break; }
          if (herr) { ok = false; break; }  // this shape cannot take the work (e.g. threads per range)
          float ms = 0;
          hipEventElapsedTime(&ms, e0, e1);
          if (r > 0 && (ms_min < 0 || ms < ms_min)) ms_min = ms;  // first run warms up
        }
        if (rc != THAPI_OK) break;
        if (ok && ms_min >= 0 && (best_ms < 0 || ms_min < best_ms)) { best_ms = ms_min; best = sh; }
      }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc != THAPI_OK) return rc;
  if (init_tables(t) != hipSuccess) return hip_fail(t, hipErrorUnknown);
  if (best_ms < 0) return THAPI_E_CAPACITY;
  t->tuned[tune_key(t, work)] = {best.T, best.E, best.rpc, best.pipe};
  save_tune_cache(t);
  if (chosen) { chosen[0] = best.T; chosen[1] = best.E; chosen[2] = best.rpc; chosen[3] = best.pipe; }
  return THAPI_OK;
}

int thapi_tally_read(thapi_tally *t, uint32_t scope, uint32_t trace_id, thapi_tally_row *rows, size_t capacity,
                     size_t *n_rows, thapi_tally_stats *stats) {
  if (!t || !n_rows) return THAPI_E_INVAL;
  if (scope < THAPI_SCOPE_THREAD || scope > THAPI_SCOPE_KERNEL) return THAPI_E_INVAL;
  if (capacity && !rows) return THAPI_E_INVAL;
  std::lock_guard<std::mutex> run(t->run_mu);
  if (hipSetDevice(t->dev) != hipSuccess) return THAPI_E_DEVICE;
  std::vector<SKey> keys;
  std::vector<uint64_t> dropped;
  int failed;
  {
    std::lock_guard<std::mutex> g(t->mu);
    keys = t->stream_keys;
    dropped = t->dropped;
    failed = t->failed;
  }
  if (failed == THAPI_E_DEVICE) return THAPI_E_DEVICE;
  const uint64_t gen = t->gen.load();
  if (t->rc_valid && t->rc_gen == gen && t->rc_scope == scope && t->rc_trace == trace_id) {
    *n_rows = t->rc_n;
    if (stats) *stats = t->rc_stats;
    if (t->rc_n > capacity) return capacity == 0 && !rows ? THAPI_OK : THAPI_E_BUFSZ;
    if (t->rc_n) memcpy(rows, t->rc_rows, sizeof(thapi_tally_row) * t->rc_n);
    t->rc_valid = false;
    return THAPI_OK;
  }
  t->rc_valid = false;
  const uint32_t nstreams = (uint32_t)keys.size();
  // canonical order of the selected streams
  std::vector<uint32_t> sel;
  for (uint32_t i = 0; i < nstreams; i++)
    if (trace_id == THAPI_ALL || keys[i][0] == trace_id) sel.push_back(i);
  std::sort(sel.begin(), sel.end(), [&](uint32_t a, uint32_t b) { return keys[a] < keys[b]; });
  const uint32_t nrank = (uint32_t)sel.size();
  std::vector<uint32_t> srank(std::max<uint32_t>(nstreams, 1), 0xFFFFFFFFu), rank_key(3 * std::max<uint32_t>(nrank, 1));
  for (uint32_t r = 0; r < nrank; r++) {
    srank[sel[r]] = r;
    rank_key[3 * r] = keys[sel[r]][0]; rank_key[3 * r + 1] = keys[sel[r]][1]; rank_key[3 * r + 2] = keys[sel[r]][2];
  }
  std::vector<uint32_t> tspan;  // FN scope: [rank_begin, rank_end) per trace
  for (uint32_t r = 0; r < nrank; r++) {
    if (r == 0 || rank_key[3 * r] != rank_key[3 * (r - 1)]) { tspan.push_back(r); tspan.push_back(r + 1); }
    else tspan.back() = r + 1;
  }
  const uint32_t ntrace = (uint32_t)(tspan.size() / 2);
  HIPCHK(timed_begin(t, TM_READOUT));
  // thread count, per-stream thread statistics and counters gathered in one
  // device buffer, then one round trip through pinned memory
  const size_t ns1 = std::max<uint32_t>(nstreams, 1);
  const size_t sbytes = 64 + 24 * ns1 + 8 * ns1 * ST_N;
  HIPCHK(ensure_pinned(t, sbytes));
  const uint32_t *hng = (const uint32_t *)t->h_pinned;   // low word of a u64
  const uint64_t *ts3 = (const uint64_t *)((uint8_t *)t->h_pinned + 64);
  const uint64_t *sst = ts3 + 3 * ns1;
  HIPCHK(t->tstats.ensure(sbytes));
  HIPCHK(launch_fill64(t->tstats.as<uint64_t>() + 8, 3ull * ns1, 0, t->st));
  HIPCHK(launch_thread_stats(t->tb, t->cfg.max_threads, t->tstats.as<unsigned long long>(), nstreams, (uint32_t)ns1,
                             t->st));
  HIPCHK(hipMemcpyAsync(t->h_pinned, t->tstats.p, 64 + 24 * ns1 + 8ull * nstreams * ST_N, hipMemcpyDeviceToHost,
                        t->st));
  HIPCHK(hipStreamSynchronize(t->st));
  const uint32_t ng = std::min<uint32_t>(*hng, t->cfg.max_threads);
  thapi_tally_stats stats_all{};
  {
    thapi_tally_stats s{};
    std::vector<std::array<uint32_t, 2>> hosts;
    for (uint32_t i : sel) {
      const uint64_t *c = &sst[(size_t)i * ST_N];
      s.records += c[ST_RECORDS]; s.entries += c[ST_ENTRIES]; s.exits += c[ST_EXITS];
      s.kernel_records += c[ST_KERNEL]; s.orphan_exits += c[ST_ORPHAN]; s.fn_mismatch += c[ST_MISMATCH];
      s.neg_duration += c[ST_NEGDUR]; s.self_underflow += c[ST_UNDER]; s.ts_regress += c[ST_TSREG];
      s.unclosed_final += c[ST_UNCLOSED]; s.bad_records += c[ST_BAD];
      s.dropped_records += dropped[i];
      s.distinct_threads += ts3[3 * i]; s.open_now += ts3[3 * i + 1]; s.depth_overflow += ts3[3 * i + 2];
      if (c[ST_ENTRIES] + c[ST_EXITS] + c[ST_KERNEL]) {
        s.distinct_processes++;
        hosts.push_back({keys[i][0], keys[i][1]});
      }
    }
    std::sort(hosts.begin(), hosts.end());
    s.distinct_hosts = (uint64_t)(std::unique(hosts.begin(), hosts.end()) - hosts.begin());
    stats_all = s;
    if (stats) *stats = s;
  }
  // threads of the selected streams, sorted canonically
  uint32_t nsel_threads = 0;
  for (uint32_t i : sel) nsel_threads += (uint32_t)ts3[3 * i];
  int rank_bits = 1;
  while ((1u << rank_bits) <= nrank + 1 && rank_bits < 32) rank_bits++;
  HIPCHK(t->keys.ensure(8ull * std::max<uint32_t>(ng, 1)));
  HIPCHK(t->vals.ensure(4ull * std::max<uint32_t>(ng, 1)));
  HIPCHK(t->keys2.ensure(8ull * std::max<uint32_t>(ng, 1)));
  HIPCHK(t->vals2.ensure(4ull * std::max<uint32_t>(ng, 1)));
  HIPCHK(t->gbeg.ensure(4ull * std::max<uint32_t>(nrank, 1)));
  HIPCHK(t->gend.ensure(4ull * std::max<uint32_t>(nrank, 1)));
  const uint32_t maxg = std::max<uint32_t>(std::max<uint32_t>(nsel_threads, nrank), 1);
  HIPCHK(t->cnt.ensure(4ull * maxg));
  HIPCHK(t->off.ensure(8ull * (maxg + 1)));
  std::vector<uint32_t> rank_stream(std::max<uint32_t>(nrank, 1), 0);
  for (uint32_t r = 0; r < nrank; r++) rank_stream[r] = sel[r];
  {
    // host tables of the readout, staged in pinned memory (the work-list
    // staging is free between flushes)
    const void *src[4] = {srank.data(), rank_key.data(), tspan.data(), rank_stream.data()};
    void **dst[4] = {&t->stream_rank.p, &t->rank_key.p, &t->trace_span.p, &t->rstream.p};
    const size_t part[4] = {4ull * srank.size(), 4ull * rank_key.size(), 4ull * tspan.size(), 4ull * rank_stream.size()};
    const size_t tot = pack_bytes(part, 4);
    HIPCHK(t->read_pack.ensure(tot));
    HIPCHK(grow_plan_staging(t, tot));
    HIPCHK(stage_h2d(t, t->read_pack.as<uint8_t>(), dst, src, part, 4));
  }
  if (sort_small_fits(ng)) {
    // keys, sort and group bounds in one launch
    HIPCHK(launch_sort_small(t->tb, t->stream_rank.as<uint32_t>(), t->keys.as<uint64_t>(), t->vals.as<uint32_t>(), ng,
                             t->gbeg.as<uint32_t>(), t->gend.as<uint32_t>(), std::max<uint32_t>(nrank, 1), t->st));
  } else {
    HIPCHK(launch_fill32(t->gbeg.as<uint32_t>(), std::max<uint32_t>(nrank, 1), 0, t->st));
    HIPCHK(launch_fill32(t->gend.as<uint32_t>(), std::max<uint32_t>(nrank, 1), 0, t->st));
    HIPCHK(launch_sort_threads(t->tb, t->stream_rank.as<uint32_t>(), t->keys.as<uint64_t>(), t->vals.as<uint32_t>(),
                               t->keys2.as<uint64_t>(), t->vals2.as<uint32_t>(), ng, rank_bits, t->st));
    HIPCHK(launch_group_bounds(t->keys.as<uint64_t>(), ng, t->gbeg.as<uint32_t>(), t->gend.as<uint32_t>(), nrank,
                               t->st));
  }
  RowCtx rc{};
  rc.mode = (int)scope;
  rc.n_ids = scope == THAPI_SCOPE_KERNEL ? t->cfg.n_kernel_ids : t->cfg.n_fns;
  rc.keys = t->keys.as<uint64_t>(); rc.vals = t->vals.as<uint32_t>();
  rc.gbeg = t->gbeg.as<uint32_t>(); rc.gend = t->gend.as<uint32_t>();
  rc.rank_key = t->rank_key.as<uint32_t>(); rc.trace_span = t->trace_span.as<uint32_t>();
  rc.rank_stream = t->rstream.as<uint32_t>();
  uint32_t ngroups = 0;
  if (scope == THAPI_SCOPE_THREAD) ngroups = ng ? nsel_threads : 0;
  else if (scope == THAPI_SCOPE_PROCESS) ngroups = ng ? nrank : 0;
  else if (scope == THAPI_SCOPE_FN) ngroups = ng ? ntrace : 0;
  else ngroups = t->cfg.n_kernel_ids ? nrank : 0;
  uint64_t total = 0;
  if (ngroups) {
    HIPCHK(launch_group_rows(rc, t->tb, ngroups, t->cnt.as<uint32_t>(), t->off.as<uint64_t>(), nullptr, t->st));
    uint64_t *htot = (uint64_t *)t->h_pinned;
    HIPCHK(hipMemcpyAsync(htot, t->off.as<uint64_t>() + ngroups, 8, hipMemcpyDeviceToHost, t->st));
    HIPCHK(hipStreamSynchronize(t->st));
    total = *htot;
  }
  *n_rows = (size_t)total;
  // rows that do not fit the caller's buffer are kept for the second call of
  // a two-call read
  const bool keep = total > capacity;
  if (keep && total > t->rc_cap) {
    // (pinned, so that the rows arrive in one DMA; not zero-filled)
    if (t->rc_rows) hipHostFree(t->rc_rows);
    t->rc_rows = nullptr;
    t->rc_cap = 0;
    HIPCHK(hipHostMalloc((void **)&t->rc_rows, sizeof(thapi_tally_row) * total, hipHostMallocDefault));
    t->rc_cap = total;
  }
  if (keep) t->rc_n = total;
  thapi_tally_row *dst = keep ? t->rc_rows : rows;
  if (total) {
    HIPCHK(t->rows.ensure(88ull * total));
    HIPCHK(launch_group_rows(rc, t->tb, ngroups, t->cnt.as<uint32_t>(), t->off.as<uint64_t>(), t->rows.as<uint8_t>(),
                             t->st));
    HIPCHK(hipMemcpyAsync(dst, t->rows.p, 88ull * total, hipMemcpyDeviceToHost, t->st));
  }
  HIPCHK(timed_end(t, TM_READOUT));
  HIPCHK(hipStreamSynchronize(t->st));
  collect_timing(t, TM_READOUT);
  if (keep) {
    t->rc_valid = true;
    t->rc_gen = gen;
    t->rc_scope = scope;
    t->rc_trace = trace_id;
    t->rc_stats = stats_all;
    return capacity == 0 && !rows ? THAPI_OK : THAPI_E_BUFSZ;
  }
  return THAPI_OK;
}

int thapi_tally_reset(thapi_tally *t) {
  if (!t) return THAPI_E_INVAL;
  const bool service = (t->cfg.flags & THAPI_SERVICE) != 0;
  if (service) {
    std::unique_lock<std::mutex> lk(t->mu);
    if (t->failed == THAPI_E_DEVICE) return THAPI_E_DEVICE;
    if (t->failed) {
      // the worker stopped at the failure: wait until every queued chunk's
      // copy is enqueued and has landed, then discard what it left queued
      t->cv.wait(lk, [&] {
        for (auto &c : t->queue)
          if (!c.ready) return false;
        return true;
      });
      lk.unlock();
      for (auto &cs : t->cst)
        if (cs && hipStreamSynchronize(cs) != hipSuccess) return hip_fail(t, hipErrorUnknown);
      lk.lock();
      for (auto &c : t->queue) release_chunk(t, c);
      t->queue.clear();
      t->cv.notify_all();
    } else {
      // every submitted chunk must have been tallied (the worker may hold a
      // batch it took off the queue)
      if (!t->queue.empty()) return THAPI_E_STATE;
      t->cv.wait(lk, [&] { return t->failed || t->done_upto + 1 >= t->next_ticket; });
      if (t->failed) return t->failed == THAPI_E_DEVICE ? THAPI_E_DEVICE : THAPI_E_STATE;
    }
  }
  std::lock_guard<std::mutex> run(t->run_mu);
  {
    std::lock_guard<std::mutex> g(t->mu);
    if (!t->queue.empty()) return THAPI_E_STATE;
    if (t->failed == THAPI_E_DEVICE) return THAPI_E_DEVICE;
  }
  if (hipSetDevice(t->dev) != hipSuccess) return THAPI_E_DEVICE;
  t->gen++;
  if (init_tables(t, false) != hipSuccess) return hip_fail(t, hipErrorUnknown);
  if (clear_payload_tables(t) != hipSuccess) return hip_fail(t, hipErrorUnknown);
  std::lock_guard<std::mutex> g(t->mu);
  t->stream_idx.clear();
  t->stream_keys.clear();
  t->dropped.clear();
  t->failed = 0;
  t->finalized = false;
  t->flushed_any = false;
  t->iv_nranges = 0;
  t->iv_valid = false;
  if (service && !t->worker_running) {
    // a failure stopped the worker (it has released the lock for good once
    // worker_running is false): start a new one
    if (t->worker.joinable()) t->worker.join();
    t->stop = false;
    t->worker_running = true;
    t->worker = std::thread(service_loop, t);
  }
  return THAPI_OK;
}

int thapi_tally_close(thapi_tally *t) {
  if (!t) return THAPI_E_INVAL;
  if (t->worker.joinable()) {
    {
      std::lock_guard<std::mutex> g(t->mu);
      t->stop = true;
      t->cv.notify_all();
      t->work_cv.notify_all();
    }
    t->worker.join();
  }
  {
    std::lock_guard<std::mutex> run(t->run_mu);
    hipSetDevice(t->dev);
    if (t->st) hipStreamSynchronize(t->st);
    free_all(t);
  }
  delete t;
  return THAPI_OK;
}

int thapi_tally_intervals(thapi_tally *t, thapi_tally_interval *out, size_t cap, size_t *n, uint32_t flags) {
  if (!t || !n || (cap && !out) || (flags & ~THAPI_OUT_DEVICE)) return THAPI_E_INVAL;
  if (!(t->cfg.flags & THAPI_INTERVALS)) return THAPI_E_STATE;
  std::lock_guard<std::mutex> run(t->run_mu);
  {
    std::lock_guard<std::mutex> g(t->mu);
    if (t->failed == THAPI_E_DEVICE) return THAPI_E_DEVICE;
    if (t->failed) return THAPI_E_STATE;
  }
  *n = 0;
  if (!t->iv_valid) return THAPI_OK;
  if (hipSetDevice(t->dev) != hipSuccess) return THAPI_E_DEVICE;
  const uint32_t nR = t->iv_nranges;
  // interval counts: each range's, then the combine's
  HIPCHK(ensure_pinned(t, 4ull * (nR + 1)));
  uint32_t *hc = (uint32_t *)t->h_pinned;
  if (nR) HIPCHK(hipMemcpyAsync(hc, t->tb.iv_n, 4ull * nR, hipMemcpyDeviceToHost, t->st));
  HIPCHK(hipMemcpyAsync(hc + nR, t->tb.civ_n, 4, hipMemcpyDeviceToHost, t->st));
  HIPCHK(hipStreamSynchronize(t->st));
  std::vector<uint64_t> off(nR + 1);
  uint64_t total = 0;
  for (uint32_t r = 0; r < nR; r++) { off[r] = total; total += hc[r]; }
  off[nR] = total;
  total += std::min<uint32_t>(hc[nR], t->tb.civ_cap);
  *n = total;
  if (!out) return THAPI_OK;
  if (cap < total) return THAPI_E_BUFSZ;
  if (!total) return THAPI_OK;
  // offsets and stream keys up in one copy, then one conversion launch
  std::vector<uint32_t> keys(3 * std::max<size_t>(t->stream_keys.size(), 1));
  for (size_t i = 0; i < t->stream_keys.size(); i++)
    for (int k = 0; k < 3; k++) keys[3 * i + k] = t->stream_keys[i][k];
  const size_t bytes[3] = {8 * off.size(), 4 * keys.size(), 8 * std::max<size_t>(t->iv_bases.size(), 1)};
  HIPCHK(grow_plan_staging(t, pack_bytes(bytes, 3)));
  HIPCHK(t->ivaux.ensure(pack_bytes(bytes, 3)));
  void *d_off = nullptr, *d_keys = nullptr, *d_bases = nullptr;
  void **views[3] = {&d_off, &d_keys, &d_bases};
  const void *src[3] = {off.data(), keys.data(), t->iv_bases.data()};
  HIPCHK(stage_h2d(t, t->ivaux.as<uint8_t>(), views, src, bytes, 3));
  const bool on_dev = (flags & THAPI_OUT_DEVICE) != 0;
  void *dst = out;
  if (!on_dev) {
    HIPCHK(t->ivout.ensure(sizeof(thapi_tally_interval) * total));
    dst = t->ivout.p;
  }
  HIPCHK(timed_begin(t, TM_IVOUT));
  HIPCHK(launch_iv_out(t->tb, (const uint64_t *)d_bases, t->fb.rhdr, nR, t->fb.rnslots, (const uint64_t *)d_off,
                       (const uint32_t *)d_keys, dst, t->st));
  HIPCHK(timed_end(t, TM_IVOUT));
  if (!on_dev) HIPCHK(hipMemcpyAsync(out, dst, sizeof(thapi_tally_interval) * total, hipMemcpyDeviceToHost, t->st));
  HIPCHK(hipStreamSynchronize(t->st));
  collect_timing(t, TM_IVOUT);
  return THAPI_OK;
}

namespace {
// Clears the copy and handle tables (on the handle's stream).
hipError_t clear_payload_tables(thapi_tally *t) {
  if (!t->roles_on) return hipSuccess;
  hipError_t e;
  const size_t nc = (size_t)t->cfg.max_streams * t->cfg.n_fns * 8;
  if ((e = launch_fill64((uint64_t *)t->d_copies, nc, 0, t->st)) != hipSuccess) return e;
  if ((e = launch_fill64((uint64_t *)t->d_hk, t->hcap, EMPTY64, t->st)) != hipSuccess) return e;
  if ((e = launch_fill32((uint32_t *)t->d_hx, 2ull * t->cfg.max_streams, 0, t->st)) != hipSuccess) return e;
  if ((e = launch_fill32((uint32_t *)t->d_hs2, t->hcap, 0, t->st)) != hipSuccess) return e;
  if ((e = launch_fill32((uint32_t *)t->d_hc, t->hcap, 0, t->st)) != hipSuccess) return e;
  return launch_fill32((uint32_t *)t->d_hr, t->hcap, 0, t->st);
}

// Stream indices of the registered streams in canonical (trace, host, pid)
// order, keeping those of trace `trace` (or all).
std::vector<uint32_t> canonical_streams(const thapi_tally *t, uint32_t trace) {
  std::vector<uint32_t> v;
  for (uint32_t i = 0; i < t->stream_keys.size(); i++)
    if (trace == THAPI_ALL || t->stream_keys[i][0] == trace) v.push_back(i);
  std::sort(v.begin(), v.end(), [&](uint32_t a, uint32_t b) { return t->stream_keys[a] < t->stream_keys[b]; });
  return v;
}
}  // namespace

int thapi_tally_set_roles(thapi_tally *t, const uint8_t *roles, uint32_t n_fns, uint32_t max_handles) {
  if (!t || !roles || n_fns != t->cfg.n_fns || t->cfg.format == THAPI_FMT_FIXED24) return THAPI_E_INVAL;
  for (uint32_t i = 0; i < n_fns; i++)
    if (roles[i] > THAPI_ROLE_RELEASE) return THAPI_E_INVAL;
  std::lock_guard<std::mutex> run(t->run_mu);
  {
    std::lock_guard<std::mutex> g(t->mu);
    if (t->failed) return t->failed == THAPI_E_DEVICE ? THAPI_E_DEVICE : THAPI_E_STATE;
    if (t->roles_on || t->flushed_any || !t->queue.empty()) return THAPI_E_STATE;
  }
  if (hipSetDevice(t->dev) != hipSuccess) return THAPI_E_DEVICE;
  uint32_t cap = 64;
  while (cap < 2ull * std::max<uint32_t>(max_handles, 1)) {
    if (cap >= (1u << 30)) return THAPI_E_INVAL;
    cap <<= 1;
  }
  struct A { void **p; size_t bytes; } allocs[] = {
      {&t->d_roles, n_fns},
      {&t->d_copies, 16ull * 4 * t->cfg.max_streams * n_fns},
      {&t->d_hk, 8ull * cap},
      {&t->d_hs2, 4ull * cap},
      {&t->d_hc, 4ull * cap},
      {&t->d_hr, 4ull * cap},
      {&t->d_hx, 8ull * t->cfg.max_streams},
      {&t->d_hlk, 8ull * cap},
      {&t->d_hlm, 4ull * cap},
      {&t->d_hln, 4},
  };
  for (auto &a : allocs) {
    if (hipMalloc(a.p, a.bytes) != hipSuccess) {
      hipGetLastError();
      for (auto &b : allocs) if (*b.p) { hipFree(*b.p); *b.p = nullptr; }
      return THAPI_E_NOMEM;
    }
  }
  HIPCHK(hipMemcpy(t->d_roles, roles, n_fns, hipMemcpyHostToDevice));
  t->hcap = cap;
  PayTables &pt = t->pt;
  pt.roles = (const uint8_t *)t->d_roles;
  pt.copies = (uint64_t *)t->d_copies;
  pt.hk = (uint64_t *)t->d_hk;
  pt.hs = (uint32_t *)t->d_hs2;
  pt.hc = (uint32_t *)t->d_hc;
  pt.hr = (uint32_t *)t->d_hr;
  pt.hx = (uint32_t *)t->d_hx;
  pt.hl_key = (uint64_t *)t->d_hlk;
  pt.hl_meta = (uint32_t *)t->d_hlm;
  pt.hl_n = (uint32_t *)t->d_hln;
  pt.hl_cap = cap;
  pt.n_streams = t->cfg.max_streams;
  pt.hmask = cap - 1;
  pt.n_fns = n_fns;
  pt.err = t->tb.err;
  t->roles_on = true;
  HIPCHK(clear_payload_tables(t));
  HIPCHK(hipStreamSynchronize(t->st));
  return THAPI_OK;
}

int thapi_tally_copies(thapi_tally *t, uint32_t trace_id, thapi_copy_row *rows, size_t capacity, size_t *n_rows) {
  if (!t || !n_rows || (capacity && !rows)) return THAPI_E_INVAL;
  std::lock_guard<std::mutex> run(t->run_mu);
  if (!t->roles_on) return THAPI_E_STATE;
  {
    std::lock_guard<std::mutex> g(t->mu);
    if (t->failed == THAPI_E_DEVICE) return THAPI_E_DEVICE;
  }
  if (hipSetDevice(t->dev) != hipSuccess) return THAPI_E_DEVICE;
  const size_t ns = t->stream_keys.size(), nf = t->cfg.n_fns;
  std::vector<uint64_t> h(std::max<size_t>(ns * nf * 8, 1));
  if (ns) {
    HIPCHK(hipMemcpyAsync(h.data(), t->d_copies, 8 * ns * nf * 8, hipMemcpyDeviceToHost, t->st));
    HIPCHK(hipStreamSynchronize(t->st));
  }
  std::vector<thapi_copy_row> out;
  for (uint32_t s : canonical_streams(t, trace_id))
    for (uint32_t f = 0; f < nf; f++)
      for (uint32_t d = 0; d < 4; d++) {
        const uint64_t *c = &h[((size_t)s * nf + f) * 8 + 2 * d];
        if (!c[0]) continue;
        thapi_copy_row r{};
        r.trace_id = t->stream_keys[s][0]; r.host_id = t->stream_keys[s][1]; r.pid = t->stream_keys[s][2];
        r.fn = f; r.dir = d; r.count = c[0]; r.bytes = c[1];
        out.push_back(r);
      }
  *n_rows = out.size();
  if (!rows && !capacity) return THAPI_OK;
  if (capacity < out.size()) return THAPI_E_BUFSZ;
  if (!out.empty()) memcpy(rows, out.data(), out.size() * sizeof(thapi_copy_row));
  return THAPI_OK;
}

int thapi_tally_handles(thapi_tally *t, uint32_t trace_id, thapi_handle_row *rows, size_t capacity,
                        size_t *n_rows) {
  if (!t || !n_rows || (capacity && !rows)) return THAPI_E_INVAL;
  std::lock_guard<std::mutex> run(t->run_mu);
  if (!t->roles_on) return THAPI_E_STATE;
  {
    std::lock_guard<std::mutex> g(t->mu);
    if (t->failed == THAPI_E_DEVICE) return THAPI_E_DEVICE;
  }
  if (hipSetDevice(t->dev) != hipSuccess) return THAPI_E_DEVICE;
  const size_t ns = t->stream_keys.size();
  std::vector<uint64_t> h(std::max<size_t>(5 * ns, 1));
  if (ns) {
    HIPCHK(t->hstat.ensure(40 * ns));
    HIPCHK(launch_fill64(t->hstat.as<uint64_t>(), 5 * ns, 0, t->st));
    HIPCHK(launch_handle_stats(t->pt, t->hstat.as<unsigned long long>(), (uint32_t)ns, t->st));
    HIPCHK(hipMemcpyAsync(h.data(), t->hstat.p, 40 * ns, hipMemcpyDeviceToHost, t->st));
    HIPCHK(hipStreamSynchronize(t->st));
  }
  std::vector<thapi_handle_row> out;
  for (uint32_t s : canonical_streams(t, trace_id)) {
    const uint64_t *c = &h[5 * (size_t)s];
    if (!c[0] && !c[1]) continue;
    thapi_handle_row r{};
    r.trace_id = t->stream_keys[s][0]; r.host_id = t->stream_keys[s][1]; r.pid = t->stream_keys[s][2];
    r.creates = c[0]; r.releases = c[1]; r.handles = c[2]; r.unreleased = c[3]; r.unmatched = c[4];
    out.push_back(r);
  }
  *n_rows = out.size();
  if (!rows && !capacity) return THAPI_OK;
  if (capacity < out.size()) return THAPI_E_BUFSZ;
  if (!out.empty()) memcpy(rows, out.data(), out.size() * sizeof(thapi_handle_row));
  return THAPI_OK;
}

int thapi_tally_timings(thapi_tally *t, double *ms, int n) {
  if (!t || (n && !ms)) return THAPI_E_INVAL;
  int k = std::min<int>(n, TM_N);
  for (int i = 0; i < k; i++) ms[i] = t->timings[i];
  return k;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Aggregate export and merge.  Blob layout (little-endian), in this order:
//   header   16 x u32: magic "THTALLY1" (2 words), version 1, format, n_fns,
//            n_kernel_ids, max_depth, n_streams, n_threads, n_frames, n_rows,
//            n_krows, finalized, 3 x 0
//   streams  n_streams x {u32 trace, host, pid, 0; u64 dropped; u64 counters[11]}
//   threads  n_threads x {u32 stream index, tid, open calls h, flags; u64 last ts}
//   frames   n_frames  x {u32 thread index, fn; u64 ts, children time, bytes}
//            (each thread's h open calls, bottom first, threads in order)
//   rows     n_rows    x {u32 thread index, fn; u64 count, incl sum/min/max,
//                         self sum/min/max, bytes}
//   krows    n_krows   x {u32 stream index, kernel id; u64 count, sum, min, max}
// Counters in stream order: records, entries, exits, kernel records, orphan
// exits, fn mismatch, negative durations, self underflow, ts regressions,
// unclosed at the final flush, bad records.  Thread flags: 1 = has a
// timestamp, 2 = its stack overflowed max_depth.
namespace {

constexpr uint32_t BLOB_MAGIC0 = 0x4C415448u, BLOB_MAGIC1 = 0x31594C4Cu;   // "THTALLY1"
constexpr size_t BLOB_HDR = 64, BLOB_STREAM = 112, BLOB_THREAD = 24, BLOB_FRAME = 32, BLOB_ROW = 72,
                 BLOB_KROW = 40;

struct Writer {
  uint8_t *p;
  void u32(uint32_t v) { memcpy(p, &v, 4); p += 4; }
  void u64(uint64_t v) { memcpy(p, &v, 8); p += 8; }
};
struct Reader {
  const uint8_t *p;
  uint32_t u32() { uint32_t v; memcpy(&v, p, 4); p += 4; return v; }
  uint64_t u64() { uint64_t v; memcpy(&v, p, 8); p += 8; return v; }
};

// Builds the blob of everything flushed so far into t->exp_blob.  Caller
// holds run_mu.
int build_export(thapi_tally *t) {
  const uint32_t D = t->cfg.max_depth, nf = t->cfg.n_fns, nk = t->cfg.n_kernel_ids;
  std::vector<SKey> keys;
  std::vector<uint64_t> dropped;
  bool finalized;
  {
    std::lock_guard<std::mutex> g(t->mu);
    keys = t->stream_keys;
    dropped = t->dropped;
    finalized = t->finalized;
  }
  const size_t ns = keys.size();
  uint32_t ng = 0;
  HIPCHK(hipStreamSynchronize(t->st));   // (a reset's table initialisation may still be queued)
  HIPCHK(hipMemcpyAsync(t->h_pinned, t->tb.n_gslots, 4, hipMemcpyDeviceToHost, t->st));
  HIPCHK(hipStreamSynchronize(t->st));
  ng = std::min<uint32_t>(*(const uint32_t *)t->h_pinned, t->cfg.max_threads);
  std::vector<uint32_t> ths(ng), tht(ng);
  std::vector<CState> cs(ng);
  std::vector<Frame> fr((size_t)ng * D);
  std::vector<Tally> tal((size_t)ng * nf);
  std::vector<KTally> kt(ns * nk);
  std::vector<uint64_t> sst(ns * ST_N);
  if (ng) {
    HIPCHK(hipMemcpy(ths.data(), t->tb.th_stream, 4ull * ng, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(tht.data(), t->tb.th_tid, 4ull * ng, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(cs.data(), t->tb.cstate, sizeof(CState) * ng, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(fr.data(), t->tb.cstack, sizeof(Frame) * fr.size(), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(tal.data(), t->tb.tally, sizeof(Tally) * tal.size(), hipMemcpyDeviceToHost));
  }
  if (!kt.empty()) HIPCHK(hipMemcpy(kt.data(), t->tb.ktally, sizeof(KTally) * kt.size(), hipMemcpyDeviceToHost));
  if (!sst.empty()) HIPCHK(hipMemcpy(sst.data(), t->tb.sstats, 8 * sst.size(), hipMemcpyDeviceToHost));
  size_t n_frames = 0, n_rows = 0, n_krows = 0;
  for (uint32_t g = 0; g < ng; g++) n_frames += std::min<uint32_t>(cs[g].h, D);
  for (auto &v : tal) n_rows += v.count != 0;
  for (auto &v : kt) n_krows += v.count != 0;
  const size_t bytes = BLOB_HDR + BLOB_STREAM * ns + BLOB_THREAD * ng + BLOB_FRAME * n_frames + BLOB_ROW * n_rows +
                       BLOB_KROW * n_krows;
  t->exp_blob.assign(bytes, 0);
  Writer w{t->exp_blob.data()};
  const uint32_t hdr[16] = {BLOB_MAGIC0, BLOB_MAGIC1, 1u, t->cfg.format, nf, nk, D, (uint32_t)ns, ng,
                            (uint32_t)n_frames, (uint32_t)n_rows, (uint32_t)n_krows, finalized ? 1u : 0u, 0, 0, 0};
  for (uint32_t v : hdr) w.u32(v);
  for (size_t i = 0; i < ns; i++) {
    w.u32(keys[i][0]); w.u32(keys[i][1]); w.u32(keys[i][2]); w.u32(0);
    w.u64(dropped[i]);
    for (int k = 0; k < ST_N; k++) w.u64(sst[i * ST_N + k]);
  }
  for (uint32_t g = 0; g < ng; g++) {
    w.u32(ths[g]); w.u32(tht[g]); w.u32(std::min<uint32_t>(cs[g].h, D)); w.u32(cs[g].flags);
    w.u64(cs[g].last_ts);
  }
  for (uint32_t g = 0; g < ng; g++)
    for (uint32_t k = 0; k < std::min<uint32_t>(cs[g].h, D); k++) {
      const Frame &f = fr[(size_t)g * D + k];
      w.u32(g); w.u32(f.fn); w.u64(f.ts); w.u64(f.child); w.u64(f.bytes);
    }
  for (uint32_t g = 0; g < ng; g++)
    for (uint32_t f = 0; f < nf; f++) {
      const Tally &v = tal[(size_t)g * nf + f];
      if (!v.count) continue;
      w.u32(g); w.u32(f);
      w.u64(v.count); w.u64(v.incl_sum); w.u64(v.incl_min); w.u64(v.incl_max);
      w.u64(v.self_sum); w.u64(v.self_min); w.u64(v.self_max); w.u64(v.bytes_sum);
    }
  for (size_t s = 0; s < ns; s++)
    for (uint32_t k = 0; k < nk; k++) {
      const KTally &v = kt[s * nk + k];
      if (!v.count) continue;
      w.u32((uint32_t)s); w.u32(k);
      w.u64(v.count); w.u64(v.sum); w.u64(v.min); w.u64(v.max);
    }
  t->exp_gen = t->gen.load();
  t->exp_valid = true;
  return THAPI_OK;
}

}  // namespace

namespace tt {
hipError_t launch_merge(const Tables &tb, const MThread *th, uint32_t n_th, const Frame *frames, uint32_t *gmap,
                        const MRow *rows, uint32_t n_rows, const MKRow *krows, uint32_t n_krows, const uint64_t *scnt,
                        const uint32_t *sidx, uint32_t n_streams, uint32_t *conflict, bool check_only,
                        hipStream_t st);
}  // namespace tt

extern "C" {

int thapi_tally_export(thapi_tally *t, void *buf, size_t cap, size_t *size) {
  if (!t || !size || (cap && !buf)) return THAPI_E_INVAL;
  std::lock_guard<std::mutex> run(t->run_mu);
  {
    std::lock_guard<std::mutex> g(t->mu);
    if (t->failed) return t->failed == THAPI_E_DEVICE ? THAPI_E_DEVICE : THAPI_E_STATE;
  }
  if (hipSetDevice(t->dev) != hipSuccess) return THAPI_E_DEVICE;
  // the blob of a size query is kept for the second call while nothing changed
  if (!t->exp_valid || t->exp_gen != t->gen.load()) {
    const int rc = build_export(t);
    if (rc != THAPI_OK) return rc;
  }
  *size = t->exp_blob.size();
  if (t->exp_blob.size() > cap) return !buf && !cap ? THAPI_OK : THAPI_E_BUFSZ;
  memcpy(buf, t->exp_blob.data(), t->exp_blob.size());
  t->exp_valid = false;
  return THAPI_OK;
}

int thapi_tally_merge(thapi_tally *t, const void *buf, size_t size) {
  if (!t || (!buf && size)) return THAPI_E_INVAL;
  if (size < BLOB_HDR) return THAPI_E_INVAL;
  const uint8_t *b = (const uint8_t *)buf;
  Reader r{b};
  uint32_t h[16];
  for (auto &v : h) v = r.u32();
  if (h[0] != BLOB_MAGIC0 || h[1] != BLOB_MAGIC1 || h[2] != 1u) return THAPI_E_INVAL;
  if (h[3] != t->cfg.format || h[4] != t->cfg.n_fns || h[5] != t->cfg.n_kernel_ids || h[6] != t->cfg.max_depth)
    return THAPI_E_INVAL;
  const uint64_t ns = h[7], nth = h[8], nfr = h[9], nrow = h[10], nkr = h[11];
  const uint64_t want = BLOB_HDR + BLOB_STREAM * ns + BLOB_THREAD * nth + BLOB_FRAME * nfr + BLOB_ROW * nrow +
                        BLOB_KROW * nkr;
  if (want != size) return THAPI_E_INVAL;
  const uint32_t D = t->cfg.max_depth, nf = t->cfg.n_fns, nk = t->cfg.n_kernel_ids;
  // parse and validate everything before any change
  std::vector<SKey> skeys(ns);
  std::vector<uint64_t> sdrop(ns), scnt(ns * ST_N);
  std::map<SKey, uint32_t> seen;
  for (uint64_t i = 0; i < ns; i++) {
    skeys[i] = {r.u32(), r.u32(), r.u32()};
    if (r.u32() != 0) return THAPI_E_INVAL;
    sdrop[i] = r.u64();
    for (int k = 0; k < ST_N; k++) scnt[i * ST_N + k] = r.u64();
    if (!seen.emplace(skeys[i], (uint32_t)i).second) return THAPI_E_INVAL;
  }
  std::vector<MThread> th(nth);
  std::set<std::pair<uint32_t, uint32_t>> tkeys;
  uint64_t frames_needed = 0;
  for (uint64_t i = 0; i < nth; i++) {
    MThread &m = th[i];
    m.stream = r.u32(); m.tid = r.u32(); m.h = r.u32(); m.flags = r.u32(); m.last_ts = r.u64();
    m.frame0 = (uint32_t)frames_needed; m.pad = 0;
    if (m.stream >= ns || m.h > D || (m.flags & ~(uint32_t)(CS_HAS_TS | CS_OVERFLOW))) return THAPI_E_INVAL;
    if (!tkeys.insert({m.stream, m.tid}).second) return THAPI_E_INVAL;
    frames_needed += m.h;
  }
  if (frames_needed != nfr) return THAPI_E_INVAL;
  std::vector<Frame> frames(nfr);
  {
    uint64_t i = 0;
    for (uint64_t k = 0; k < nth; k++)
      for (uint32_t j = 0; j < th[k].h; j++, i++) {
        if (r.u32() != k) return THAPI_E_INVAL;
        Frame &f = frames[i];
        f.fn = r.u32(); f.ts = r.u64(); f.child = r.u64(); f.bytes = r.u64(); f.pad = 0;
        if (f.fn >= nf) return THAPI_E_INVAL;
      }
  }
  std::vector<MRow> rows(nrow);
  for (auto &m : rows) {
    m.thread = r.u32(); m.fn = r.u32();
    m.v.count = r.u64(); m.v.incl_sum = r.u64(); m.v.incl_min = r.u64(); m.v.incl_max = r.u64();
    m.v.self_sum = r.u64(); m.v.self_min = r.u64(); m.v.self_max = r.u64(); m.v.bytes_sum = r.u64();
    if (m.thread >= nth || m.fn >= nf) return THAPI_E_INVAL;
  }
  std::vector<MKRow> krows(nkr);
  for (auto &m : krows) {
    m.stream = r.u32(); m.kid = r.u32();
    m.v.count = r.u64(); m.v.sum = r.u64(); m.v.min = r.u64(); m.v.max = r.u64();
    if (m.stream >= ns || m.kid >= nk) return THAPI_E_INVAL;
  }
  std::lock_guard<std::mutex> run(t->run_mu);
  std::vector<uint32_t> sidx(ns);
  {
    std::lock_guard<std::mutex> g(t->mu);
    if (t->cfg.flags & THAPI_SERVICE) return THAPI_E_STATE;
    if (t->failed) return t->failed == THAPI_E_DEVICE ? THAPI_E_DEVICE : THAPI_E_STATE;
    if (t->finalized || !t->queue.empty()) return THAPI_E_STATE;
    size_t fresh = 0;
    for (auto &k : skeys) fresh += t->stream_idx.count(k) == 0;
    if (t->stream_keys.size() + fresh > t->cfg.max_streams) return THAPI_E_CAPACITY;
  }
  if (hipSetDevice(t->dev) != hipSuccess) return THAPI_E_DEVICE;
  HIPCHK(hipStreamSynchronize(t->st));
  // map the blob's streams to this handle's indices (registering new keys
  // only after the conflict check below has passed)
  std::vector<uint32_t> map_now(ns, EMPTY32);
  {
    std::lock_guard<std::mutex> g(t->mu);
    uint32_t next = (uint32_t)t->stream_keys.size();
    for (uint64_t i = 0; i < ns; i++) {
      auto it = t->stream_idx.find(skeys[i]);
      sidx[i] = it != t->stream_idx.end() ? it->second : next++;
    }
  }
  for (auto &m : th) m.stream = sidx[m.stream];
  for (auto &m : krows) m.stream = sidx[m.stream];
  // one device buffer: threads, frames, rows, krows, counters, stream map, thread map, conflict flag
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t o_th = 0, o_fr = o_th + al(sizeof(MThread) * nth), o_row = o_fr + al(sizeof(Frame) * nfr),
               o_kr = o_row + al(sizeof(MRow) * nrow), o_sc = o_kr + al(sizeof(MKRow) * nkr),
               o_si = o_sc + al(8 * ns * ST_N), o_gm = o_si + al(4 * ns), o_cf = o_gm + al(4 * nth),
               tot = o_cf + 256;
  HIPCHK(t->merge_buf.ensure(tot));
  uint8_t *d = t->merge_buf.as<uint8_t>();
  if (nth) HIPCHK(hipMemcpy(d + o_th, th.data(), sizeof(MThread) * nth, hipMemcpyHostToDevice));
  if (nfr) HIPCHK(hipMemcpy(d + o_fr, frames.data(), sizeof(Frame) * nfr, hipMemcpyHostToDevice));
  if (nrow) HIPCHK(hipMemcpy(d + o_row, rows.data(), sizeof(MRow) * nrow, hipMemcpyHostToDevice));
  if (nkr) HIPCHK(hipMemcpy(d + o_kr, krows.data(), sizeof(MKRow) * nkr, hipMemcpyHostToDevice));
  if (ns) HIPCHK(hipMemcpy(d + o_sc, scnt.data(), 8 * ns * ST_N, hipMemcpyHostToDevice));
  if (ns) HIPCHK(hipMemcpy(d + o_si, sidx.data(), 4 * ns, hipMemcpyHostToDevice));
  HIPCHK(launch_fill32((uint32_t *)(d + o_cf), 1, 0, t->st));
  const Tables &tb = t->tb;
  uint32_t *conflict = (uint32_t *)(d + o_cf);
  HIPCHK(launch_merge(tb, (const MThread *)(d + o_th), (uint32_t)nth, (const Frame *)(d + o_fr),
                      (uint32_t *)(d + o_gm), (const MRow *)(d + o_row), (uint32_t)nrow, (const MKRow *)(d + o_kr),
                      (uint32_t)nkr, (const uint64_t *)(d + o_sc), (const uint32_t *)(d + o_si), (uint32_t)ns,
                      conflict, true, t->st));
  HIPCHK(hipMemcpyAsync(t->h_pinned, conflict, 4, hipMemcpyDeviceToHost, t->st));
  HIPCHK(hipStreamSynchronize(t->st));
  if (*(const uint32_t *)t->h_pinned) return THAPI_E_STATE;   // open calls on both sides of one thread
  {
    std::lock_guard<std::mutex> g(t->mu);
    for (uint64_t i = 0; i < ns; i++) {
      if (sidx[i] == t->stream_keys.size()) {
        t->stream_idx[skeys[i]] = sidx[i];
        t->stream_keys.push_back(skeys[i]);
        t->dropped.push_back(0);
      }
      t->dropped[sidx[i]] += sdrop[i];
    }
    t->gen++;
    t->flushed_any = true;
    t->iv_valid = false;   // (a merge tallies no call of a flush)
  }
  HIPCHK(launch_fill32(t->tb.err, 1, 0, t->st));
  HIPCHK(launch_merge(tb, (const MThread *)(d + o_th), (uint32_t)nth, (const Frame *)(d + o_fr),
                      (uint32_t *)(d + o_gm), (const MRow *)(d + o_row), (uint32_t)nrow, (const MKRow *)(d + o_kr),
                      (uint32_t)nkr, (const uint64_t *)(d + o_sc), (const uint32_t *)(d + o_si), (uint32_t)ns,
                      conflict, false, t->st));
  HIPCHK(hipMemcpyAsync(t->h_pinned, t->tb.err, 4, hipMemcpyDeviceToHost, t->st));
  HIPCHK(hipStreamSynchronize(t->st));
  if (*(const uint32_t *)t->h_pinned & ERR_CAPACITY) {
    std::lock_guard<std::mutex> g(t->mu);
    t->failed = THAPI_E_CAPACITY;
    return THAPI_E_CAPACITY;
  }
  return THAPI_OK;
}

}  // extern "C"
