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
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "thapi_tally.h"
#include "tt_common.h"

namespace tt {
size_t range_lds_bytes(uint32_t T, uint32_t E, uint32_t KL, uint32_t D, int fmt);
hipError_t launch_range(int fmt, uint32_t T, const Seg *segs, const Range *ranges, uint32_t n_ranges,
                        const Tables &tb, const Shape &sh, RHdr *rhdr, UItem *ru, OItem *ro, uint32_t *rnslots,
                        hipStream_t st);
hipError_t launch_paylen(const Seg *segs, Range *ranges, uint32_t n_ranges, const uint32_t *seg_first_range,
                         uint32_t n_segs, uint64_t *paylen, hipStream_t st);
hipError_t launch_fill64(uint64_t *p, size_t n, uint64_t v, hipStream_t st);
hipError_t launch_fill32(uint32_t *p, size_t n, uint32_t v, hipStream_t st);
hipError_t launch_init_tables(const Tables &tb, size_t n_tally, size_t n_ktally, hipStream_t st);
hipError_t launch_combine(const uint32_t *spans, uint32_t n_spans, const RHdr *rhdr, const UItem *ru,
                          const OItem *ro, const uint32_t *rnslots, const Tables &tb, hipStream_t st);
hipError_t launch_final(const Tables &tb, uint32_t max_threads, hipStream_t st);
hipError_t launch_thread_stats(const Tables &tb, uint32_t max_threads, unsigned long long *out, hipStream_t st);
hipError_t launch_sort_threads(const Tables &tb, const uint32_t *stream_rank, uint64_t *keys, uint32_t *vals,
                               uint64_t *keys2, uint32_t *vals2, uint32_t n, int rank_bits, hipStream_t st);
hipError_t launch_group_bounds(const uint64_t *keys, uint32_t n, uint32_t *gbeg, uint32_t *gend, uint32_t n_ranks,
                               hipStream_t st);
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

namespace {

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
};

using SKey = std::array<uint32_t, 3>;

enum { TM_PREPASS = 0, TM_RANGE, TM_COMBINE, TM_FINAL, TM_READOUT, TM_N };

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
       *d_err = nullptr, *d_hs = nullptr;
  Shape shape{};

  DevBuf segs, ranges, rhdr, ru, ro, rnslots, spans, paylen, segfirst;
  DevBuf keys, vals, keys2, vals2, gbeg, gend, cnt, off, rank_stream, rank_key, trace_span, stream_rank, rows, tstats;
  void *h_pinned = nullptr;  // small pinned staging for results of device->host copies
  size_t h_pinned_cap = 0;

  double timings[TM_N] = {0};
  hipEvent_t ev[2 * TM_N] = {};
};

namespace {

int hip_fail(thapi_tally *t, hipError_t e) {
  if (e == hipSuccess) return THAPI_OK;
  if (t) t->failed = THAPI_E_DEVICE;
  return THAPI_E_DEVICE;
}
#define HIPCHK(x) do { hipError_t _e = (x); if (_e != hipSuccess) return hip_fail(t, _e); } while (0)

uint32_t record_size(const thapi_tally *t) { return t->cfg.format == THAPI_FMT_VAR16 ? 16u : 24u; }

hipError_t init_tables(thapi_tally *t) {
  const thapi_tally_config &c = t->cfg;
  hipError_t e;
  if ((e = launch_fill64((uint64_t *)t->d_gkeys, t->gcap, EMPTY64, t->st)) != hipSuccess) return e;
  if ((e = launch_fill32((uint32_t *)t->d_gvals, t->gcap, GV_PENDING, t->st)) != hipSuccess) return e;
  if ((e = launch_fill32((uint32_t *)t->d_ngs, 1, 0, t->st)) != hipSuccess) return e;
  if ((e = launch_fill32((uint32_t *)t->d_err, 1, 0, t->st)) != hipSuccess) return e;
  if ((e = launch_init_tables(t->tb, (size_t)c.max_threads * c.n_fns, (size_t)c.max_streams * c.n_kernel_ids,
                              t->st)) != hipSuccess)
    return e;
  if ((e = launch_fill32((uint32_t *)t->d_cstate, (size_t)c.max_threads * sizeof(CState) / 4, 0, t->st)) != hipSuccess)
    return e;
  if ((e = launch_fill64((uint64_t *)t->d_sstats, (size_t)c.max_streams * ST_N, 0, t->st)) != hipSuccess) return e;
  return hipStreamSynchronize(t->st);
}

void free_all(thapi_tally *t) {
  void *ps[] = {t->d_gkeys, t->d_gvals, t->d_ngs, t->d_ths, t->d_tht, t->d_tally, t->d_ktally,
                t->d_cstate, t->d_cstack, t->d_sstats, t->d_err, t->d_hs};
  for (void *p : ps) if (p) hipFree(p);
  DevBuf *bs[] = {&t->segs, &t->ranges, &t->rhdr, &t->ru, &t->ro, &t->rnslots, &t->spans, &t->paylen, &t->segfirst,
                  &t->keys, &t->vals, &t->keys2, &t->vals2, &t->gbeg, &t->gend, &t->cnt, &t->off,
                  &t->rank_stream, &t->rank_key, &t->trace_span, &t->stream_rank, &t->rows, &t->tstats};
  for (DevBuf *b : bs) b->release();
  for (auto &c : t->queue) if (c.owned) hipFree(c.owned);
  t->queue.clear();
  if (t->h_pinned) hipHostFree(t->h_pinned);
  for (auto &e : t->ev) if (e) hipEventDestroy(e);
  if (t->own_stream && t->st) hipStreamDestroy(t->st);
}

// Picks the range kernel's tile and LDS tally size for the format and depth:
// the largest tile and tally that fit the LDS, preferring a full tally (2048
// entries) over a larger tile.  THAPI_TALLY_SHAPE="T,E" overrides the choice
// (used to tune the launch shape).
Shape pick_shape(const thapi_tally *t) {
  Shape s{};
  const uint32_t D = t->cfg.max_depth;
  const int fmt = (int)t->cfg.format;
  s.KL = std::min<uint32_t>(t->cfg.n_kernel_ids, KL_MAX);
  auto fits = [&](uint32_t T, uint32_t E) {
    size_t b = range_lds_bytes(T, E, s.KL, D, fmt);
    if (b > t->lds_limit) return false;
    s.T = T; s.E = E; s.lds_bytes = (uint32_t)b;
    return true;
  };
  if (const char *env = getenv("THAPI_TALLY_SHAPE")) {
    unsigned T = 0, E = 0;
    if (sscanf(env, "%u,%u", &T, &E) == 2 && (T == 1024 || T == 2048) && E >= 64 &&
        (E & (E - 1)) == 0 && fits(T, E))
      return s;
  }
  const uint32_t cand[][2] = {{2048, 2048}, {1024, 2048}, {2048, 1024}, {1024, 1024},
                              {1024, 512}, {1024, 256}, {1024, 128}, {1024, 64}};
  for (auto &c : cand)
    if (fits(c[0], c[1])) return s;
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

// Sum of payload_len of a device VAR16 header buffer (used to validate a
// device-input submit before it is accepted).
__global__ void k_sum_plen(const uint8_t *rec, uint64_t n, unsigned long long *out) {
  uint64_t s = 0;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    s += rec[i * 16 + 15];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if ((threadIdx.x & 63) == 0 && s) atomicAdd(out, (unsigned long long)s);
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

int thapi_tally_open(const thapi_tally_config *cfg, thapi_tally **out) {
  if (!cfg || !out) return THAPI_E_INVAL;
  if (cfg->abi_version != THAPI_TALLY_ABI_VERSION) return THAPI_E_INVAL;
  if (cfg->format != THAPI_FMT_FIXED24 && cfg->format != THAPI_FMT_VAR16) return THAPI_E_INVAL;
  if (cfg->n_fns < 1 || cfg->n_fns > 65536 || cfg->n_kernel_ids > 65536) return THAPI_E_INVAL;
  if (cfg->max_depth > THAPI_MAX_DEPTH_LIMIT || cfg->reserved) return THAPI_E_INVAL;
  if (cfg->max_threads > (1u << 30) || cfg->max_streams > (1u << 24)) return THAPI_E_INVAL;
  thapi_tally *t = new (std::nothrow) thapi_tally();
  if (!t) return THAPI_E_NOMEM;
  t->cfg = *cfg;
  if (!t->cfg.max_depth) t->cfg.max_depth = 16;
  if (!t->cfg.max_threads) t->cfg.max_threads = 65536;
  if (!t->cfg.max_streams) t->cfg.max_streams = 4096;
  if (!t->cfg.device_budget_bytes) t->cfg.device_budget_bytes = 16ull << 30;
  t->cfg.fn_has_size = nullptr;
  t->cfg.autotune_cache = nullptr;
  if (cfg->format == THAPI_FMT_VAR16 && cfg->fn_has_size)
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
  };
  for (auto &a : allocs) {
    hipError_t e = hipMalloc(a.p, a.bytes);
    if (e != hipSuccess) { hipGetLastError(); return bail(THAPI_E_NOMEM); }
  }
  Tables &tb = t->tb;
  tb.gkeys = (uint64_t *)t->d_gkeys; tb.gvals = (uint32_t *)t->d_gvals; tb.gmask = t->gcap - 1;
  tb.n_gslots = (uint32_t *)t->d_ngs; tb.max_threads = c.max_threads;
  tb.th_stream = (uint32_t *)t->d_ths; tb.th_tid = (uint32_t *)t->d_tht;
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
  t->shape = pick_shape(t);
  if (!t->shape.T) return bail(THAPI_E_INVAL);
  if (init_tables(t) != hipSuccess) return bail(THAPI_E_DEVICE);
  *out = t;
  return THAPI_OK;
}

int thapi_tally_submit(thapi_tally *t, const thapi_stream_key *key, const void *records, size_t record_bytes,
                       const void *payload, size_t payload_bytes, uint64_t *ticket_out) {
  if (!t || !key || key->reserved) return THAPI_E_INVAL;
  const uint32_t rs = record_size(t);
  if (record_bytes % rs) return THAPI_E_INVAL;
  if (record_bytes && !records) return THAPI_E_INVAL;
  const bool var = t->cfg.format == THAPI_FMT_VAR16;
  if (!var && (payload || payload_bytes)) return THAPI_E_INVAL;
  if (payload_bytes && !payload) return THAPI_E_INVAL;
  const bool dev_in = (t->cfg.flags & THAPI_DEVICE_INPUT) != 0;
  if (dev_in && ((uintptr_t)records & 7)) return THAPI_E_INVAL;
  const uint64_t n_rec = record_bytes / rs;
  {
    std::lock_guard<std::mutex> g(t->mu);
    if (t->failed) return THAPI_E_STATE;
    if (t->finalized) return THAPI_E_STATE;
  }
  if (hipSetDevice(t->dev) != hipSuccess) return THAPI_E_DEVICE;
  // VAR16: the payload heap must hold exactly the declared payload lengths
  if (var && n_rec) {
    uint64_t sum = 0;
    if (!dev_in) {
      const uint8_t *r = (const uint8_t *)records;
      for (uint64_t i = 0; i < n_rec; i++) sum += r[i * 16 + 15];
    } else {
      unsigned long long *d = nullptr;
      if (hipMalloc(&d, 8) != hipSuccess) return THAPI_E_NOMEM;
      launch_fill64((uint64_t *)d, 1, 0, t->st);
      hipLaunchKernelGGL(k_sum_plen, dim3(std::min<uint64_t>((n_rec + 255) / 256, 4096)), dim3(256), 0, t->st,
                         (const uint8_t *)records, n_rec, d);
      unsigned long long hs = 0;
      hipError_t e = hipMemcpyAsync(&hs, d, 8, hipMemcpyDeviceToHost, t->st);
      if (e == hipSuccess) e = hipStreamSynchronize(t->st);
      hipFree(d);
      if (e != hipSuccess) { std::lock_guard<std::mutex> g(t->mu); return hip_fail(t, e); }
      sum = hs;
    }
    if (sum != payload_bytes) return THAPI_E_INVAL;
  } else if (var && payload_bytes) {
    return THAPI_E_INVAL;
  }
  std::unique_lock<std::mutex> lk(t->mu);
  SKey sk{key->trace_id, key->host_id, key->pid};
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
  c.stream = sidx;
  c.n_rec = n_rec;
  c.pay_bytes = payload_bytes;
  if (dev_in) {
    c.rec = (const uint8_t *)records;
    c.pay = (const uint8_t *)payload;
  } else if (n_rec) {
    const uint64_t bytes = record_bytes + payload_bytes + 64;
    if (bytes > t->cfg.device_budget_bytes) return THAPI_E_NOMEM;
    while (t->budget_used + bytes > t->cfg.device_budget_bytes) {
      if (t->cfg.flags & THAPI_DROP_ON_FULL) {
        t->dropped[sidx] += n_rec;
        if (ticket_out) *ticket_out = 0;
        return THAPI_OK;
      }
      if (t->cfg.flags & THAPI_NONBLOCKING) return THAPI_E_AGAIN;
      t->cv.wait(lk);
      if (t->failed) return THAPI_E_STATE;
    }
    t->budget_used += bytes;
    lk.unlock();
    void *d = nullptr;
    hipError_t e = hipMalloc(&d, bytes);
    if (e == hipSuccess) e = hipMemcpy(d, records, record_bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess && payload_bytes)
      e = hipMemcpy((uint8_t *)d + ((record_bytes + 15) / 16 * 16), payload, payload_bytes, hipMemcpyHostToDevice);
    lk.lock();
    if (e != hipSuccess) {
      if (d) hipFree(d);
      t->budget_used -= bytes;
      t->cv.notify_all();
      return e == hipErrorOutOfMemory ? THAPI_E_NOMEM : hip_fail(t, e);
    }
    c.owned = d;
    c.owned_bytes = bytes;
    c.rec = (const uint8_t *)d;
    c.pay = payload_bytes ? (const uint8_t *)d + ((record_bytes + 15) / 16 * 16) : nullptr;
  }
  c.ticket = t->next_ticket++;
  if (ticket_out) *ticket_out = c.ticket;
  t->queue.push_back(c);
  return THAPI_OK;
}

int thapi_tally_flush(thapi_tally *t, uint64_t ticket, uint32_t flags) {
  if (!t) return THAPI_E_INVAL;
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
  if (hipSetDevice(t->dev) != hipSuccess) return THAPI_E_DEVICE;
  for (int k = 0; k < TM_N; k++) t->timings[k] = 0;
  // chunks grouped by stream, each stream's chunks in ticket order
  std::stable_sort(work.begin(), work.end(), [](const Chunk &a, const Chunk &b) { return a.stream < b.stream; });
  std::vector<Seg> segs;
  std::vector<Range> ranges;
  std::vector<uint32_t> segfirst;
  std::vector<uint32_t> spans;
  uint64_t total = 0;
  for (auto &c : work) total += c.n_rec;
  const uint32_t T = t->shape.T;
  // At most one range per CU (the range kernel holds one workgroup per CU):
  // with n_seg chunks, ranges of ceil(total / (n_cu - n_seg)) records give at
  // most n_cu ranges in all (each chunk adds at most one partial range).
  // Ranges are never shorter than 16 tiles.
  uint64_t n_seg = 0;
  for (auto &c : work) n_seg += c.n_rec ? 1 : 0;
  const uint64_t ncu = std::max<uint64_t>(1, (uint64_t)t->n_cu);
  const uint64_t target = ncu > 2 * n_seg ? ncu - n_seg : std::max<uint64_t>(1, ncu / 2);
  uint64_t rlen = (total + target - 1) / target;
  rlen = std::max<uint64_t>(rlen, 16ull * T);
  rlen = std::min<uint64_t>(rlen, 1ull << 30);
  for (size_t i = 0; i < work.size(); i++) {
    const Chunk &c = work[i];
    if (!c.n_rec) continue;
    Seg s{};
    s.rec = c.rec; s.pay = c.pay; s.n_rec = c.n_rec; s.pay_bytes = c.pay_bytes; s.stream = c.stream;
    segfirst.push_back((uint32_t)ranges.size());
    const uint32_t si = (uint32_t)segs.size();
    segs.push_back(s);
    const uint64_t nr = (c.n_rec + rlen - 1) / rlen;
    const uint64_t step = (c.n_rec + nr - 1) / nr;
    for (uint64_t b = 0; b < c.n_rec; b += step) {
      Range r{};
      r.seg = si; r.stream = c.stream; r.begin = b; r.n = std::min<uint64_t>(step, c.n_rec - b); r.pay_begin = 0;
      if (spans.empty() || spans[spans.size() - 3] != c.stream) {
        spans.push_back(c.stream); spans.push_back((uint32_t)ranges.size()); spans.push_back((uint32_t)ranges.size());
      }
      ranges.push_back(r);
      spans[spans.size() - 1] = (uint32_t)ranges.size();
    }
  }
  segfirst.push_back((uint32_t)ranges.size());
  const uint32_t nR = (uint32_t)ranges.size(), nS = (uint32_t)segs.size(), nSp = (uint32_t)(spans.size() / 3);
  const uint32_t D = t->cfg.max_depth;
  int rc = THAPI_OK;
  if (nR) {
    HIPCHK(t->segs.ensure(sizeof(Seg) * nS));
    HIPCHK(t->ranges.ensure(sizeof(Range) * nR));
    HIPCHK(t->segfirst.ensure(4ull * (nS + 1)));
    HIPCHK(t->spans.ensure(4ull * spans.size()));
    HIPCHK(t->rhdr.ensure(sizeof(RHdr) * (size_t)nR * S_MAX));
    HIPCHK(t->ru.ensure(sizeof(UItem) * (size_t)nR * S_MAX * D));
    HIPCHK(t->ro.ensure(sizeof(OItem) * (size_t)nR * S_MAX * D));
    HIPCHK(t->rnslots.ensure(4ull * nR));
    HIPCHK(t->paylen.ensure(8ull * nR));
    HIPCHK(hipMemcpyAsync(t->segs.p, segs.data(), sizeof(Seg) * nS, hipMemcpyHostToDevice, t->st));
    HIPCHK(hipMemcpyAsync(t->ranges.p, ranges.data(), sizeof(Range) * nR, hipMemcpyHostToDevice, t->st));
    HIPCHK(hipMemcpyAsync(t->segfirst.p, segfirst.data(), 4ull * (nS + 1), hipMemcpyHostToDevice, t->st));
    HIPCHK(hipMemcpyAsync(t->spans.p, spans.data(), 4ull * spans.size(), hipMemcpyHostToDevice, t->st));
    HIPCHK(launch_fill32(t->tb.err, 1, 0, t->st));
    if (t->cfg.format == THAPI_FMT_VAR16) {
      HIPCHK(timed_begin(t, TM_PREPASS));
      HIPCHK(launch_paylen(t->segs.as<Seg>(), t->ranges.as<Range>(), nR, t->segfirst.as<uint32_t>(), nS,
                           t->paylen.as<uint64_t>(), t->st));
      HIPCHK(timed_end(t, TM_PREPASS));
    }
    HIPCHK(timed_begin(t, TM_RANGE));
    HIPCHK(launch_range((int)t->cfg.format, T, t->segs.as<Seg>(), t->ranges.as<Range>(), nR, t->tb, t->shape,
                        t->rhdr.as<RHdr>(), t->ru.as<UItem>(), t->ro.as<OItem>(), t->rnslots.as<uint32_t>(), t->st));
    HIPCHK(timed_end(t, TM_RANGE));
    HIPCHK(timed_begin(t, TM_COMBINE));
    HIPCHK(launch_combine(t->spans.as<uint32_t>(), nSp, t->rhdr.as<RHdr>(), t->ru.as<UItem>(), t->ro.as<OItem>(),
                          t->rnslots.as<uint32_t>(), t->tb, t->st));
    HIPCHK(timed_end(t, TM_COMBINE));
  }
  if (flags & THAPI_FLUSH_FINAL) {
    HIPCHK(timed_begin(t, TM_FINAL));
    HIPCHK(launch_final(t->tb, t->cfg.max_threads, t->st));
    HIPCHK(timed_end(t, TM_FINAL));
  }
  HIPCHK(ensure_pinned(t, 64));
  uint32_t *herr = (uint32_t *)t->h_pinned;
  HIPCHK(hipMemcpyAsync(herr, t->tb.err, 4, hipMemcpyDeviceToHost, t->st));
  HIPCHK(hipStreamSynchronize(t->st));
  const uint32_t err = *herr;
  if (nR) {
    if (t->cfg.format == THAPI_FMT_VAR16) collect_timing(t, TM_PREPASS);
    collect_timing(t, TM_RANGE);
    collect_timing(t, TM_COMBINE);
  }
  if (flags & THAPI_FLUSH_FINAL) collect_timing(t, TM_FINAL);
  {
    std::lock_guard<std::mutex> g(t->mu);
    for (auto &c : work) {
      if (c.owned) { hipFree(c.owned); t->budget_used -= c.owned_bytes; }
    }
    t->cv.notify_all();
    if (err & (ERR_CAPACITY | ERR_RANGE_THREADS)) { t->failed = THAPI_E_CAPACITY; rc = THAPI_E_CAPACITY; }
    else if (err & ERR_DEPTH) { t->failed = THAPI_E_DEPTH; rc = THAPI_E_DEPTH; }
    if (flags & THAPI_FLUSH_FINAL) t->finalized = true;
  }
  if (rc == THAPI_OK && (t->cfg.flags & THAPI_STRICT)) {
    // strict mode: any anomaly counted so far fails the flush
    std::vector<uint64_t> h((size_t)t->stream_keys.size() * ST_N);
    if (!h.empty()) {
      HIPCHK(hipMemcpy(h.data(), t->tb.sstats, 8 * h.size(), hipMemcpyDeviceToHost));
      for (size_t i = 0; i < t->stream_keys.size(); i++) {
        const uint64_t *c = &h[i * ST_N];
        if (c[ST_ORPHAN] || c[ST_MISMATCH] || c[ST_NEGDUR] || c[ST_UNDER] || c[ST_TSREG] || c[ST_UNCLOSED] ||
            c[ST_BAD])
          rc = THAPI_E_MALFORMED;
      }
    }
  }
  return rc;
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
  HIPCHK(ensure_pinned(t, 64));
  uint32_t *hng = (uint32_t *)t->h_pinned;
  HIPCHK(hipMemcpyAsync(hng, t->tb.n_gslots, 4, hipMemcpyDeviceToHost, t->st));
  HIPCHK(hipStreamSynchronize(t->st));
  const uint32_t ng = std::min<uint32_t>(*hng, t->cfg.max_threads);
  // per-stream thread statistics
  HIPCHK(t->tstats.ensure(24ull * std::max<uint32_t>(nstreams, 1)));
  HIPCHK(launch_fill64(t->tstats.as<uint64_t>(), 3ull * std::max<uint32_t>(nstreams, 1), 0, t->st));
  if (ng) HIPCHK(launch_thread_stats(t->tb, ng, t->tstats.as<unsigned long long>(), t->st));
  std::vector<uint64_t> ts3(3ull * std::max<uint32_t>(nstreams, 1), 0), sst((size_t)std::max<uint32_t>(nstreams, 1) * ST_N, 0);
  HIPCHK(hipMemcpyAsync(ts3.data(), t->tstats.p, 24ull * std::max<uint32_t>(nstreams, 1), hipMemcpyDeviceToHost, t->st));
  if (nstreams) HIPCHK(hipMemcpyAsync(sst.data(), t->tb.sstats, 8ull * nstreams * ST_N, hipMemcpyDeviceToHost, t->st));
  HIPCHK(hipStreamSynchronize(t->st));
  if (stats) {
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
    *stats = s;
  }
  // threads of the selected streams, sorted canonically
  uint32_t nsel_threads = 0;
  for (uint32_t i : sel) nsel_threads += (uint32_t)ts3[3 * i];
  int rank_bits = 1;
  while ((1u << rank_bits) <= nrank + 1 && rank_bits < 32) rank_bits++;
  HIPCHK(t->stream_rank.ensure(4ull * srank.size()));
  HIPCHK(t->rank_key.ensure(4ull * rank_key.size()));
  HIPCHK(t->trace_span.ensure(4ull * std::max<size_t>(tspan.size(), 2)));
  HIPCHK(t->keys.ensure(8ull * std::max<uint32_t>(ng, 1)));
  HIPCHK(t->vals.ensure(4ull * std::max<uint32_t>(ng, 1)));
  HIPCHK(t->keys2.ensure(8ull * std::max<uint32_t>(ng, 1)));
  HIPCHK(t->vals2.ensure(4ull * std::max<uint32_t>(ng, 1)));
  HIPCHK(t->gbeg.ensure(4ull * std::max<uint32_t>(nrank, 1)));
  HIPCHK(t->gend.ensure(4ull * std::max<uint32_t>(nrank, 1)));
  const uint32_t maxg = std::max<uint32_t>(std::max<uint32_t>(nsel_threads, nrank), 1);
  HIPCHK(t->cnt.ensure(4ull * maxg));
  HIPCHK(t->off.ensure(8ull * (maxg + 1)));
  HIPCHK(hipMemcpyAsync(t->stream_rank.p, srank.data(), 4ull * srank.size(), hipMemcpyHostToDevice, t->st));
  HIPCHK(hipMemcpyAsync(t->rank_key.p, rank_key.data(), 4ull * rank_key.size(), hipMemcpyHostToDevice, t->st));
  if (!tspan.empty())
    HIPCHK(hipMemcpyAsync(t->trace_span.p, tspan.data(), 4ull * tspan.size(), hipMemcpyHostToDevice, t->st));
  HIPCHK(launch_fill32(t->gbeg.as<uint32_t>(), std::max<uint32_t>(nrank, 1), 0, t->st));
  HIPCHK(launch_fill32(t->gend.as<uint32_t>(), std::max<uint32_t>(nrank, 1), 0, t->st));
  if (ng) {
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
  std::vector<uint32_t> rank_stream(std::max<uint32_t>(nrank, 1), 0);
  for (uint32_t r = 0; r < nrank; r++) rank_stream[r] = sel[r];
  DevBuf rstream;
  HIPCHK(rstream.ensure(4ull * rank_stream.size()));
  HIPCHK(hipMemcpyAsync(rstream.p, rank_stream.data(), 4ull * rank_stream.size(), hipMemcpyHostToDevice, t->st));
  rc.rank_stream = rstream.as<uint32_t>();
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
  if (total > capacity) {
    hipStreamSynchronize(t->st);
    rstream.release();
    HIPCHK(timed_end(t, TM_READOUT));
    return capacity == 0 && !rows ? THAPI_OK : THAPI_E_BUFSZ;
  }
  if (total) {
    HIPCHK(t->rows.ensure(88ull * total));
    HIPCHK(launch_group_rows(rc, t->tb, ngroups, t->cnt.as<uint32_t>(), t->off.as<uint64_t>(), t->rows.as<uint8_t>(),
                             t->st));
    HIPCHK(hipMemcpyAsync(rows, t->rows.p, 88ull * total, hipMemcpyDeviceToHost, t->st));
  }
  HIPCHK(timed_end(t, TM_READOUT));
  HIPCHK(hipStreamSynchronize(t->st));
  collect_timing(t, TM_READOUT);
  rstream.release();
  return THAPI_OK;
}

int thapi_tally_reset(thapi_tally *t) {
  if (!t) return THAPI_E_INVAL;
  std::lock_guard<std::mutex> run(t->run_mu);
  {
    std::lock_guard<std::mutex> g(t->mu);
    if (!t->queue.empty()) return THAPI_E_STATE;
    if (t->failed == THAPI_E_DEVICE) return THAPI_E_DEVICE;
  }
  if (hipSetDevice(t->dev) != hipSuccess) return THAPI_E_DEVICE;
  if (init_tables(t) != hipSuccess) return hip_fail(t, hipErrorUnknown);
  std::lock_guard<std::mutex> g(t->mu);
  t->stream_idx.clear();
  t->stream_keys.clear();
  t->dropped.clear();
  t->failed = 0;
  t->finalized = false;
  return THAPI_OK;
}

int thapi_tally_close(thapi_tally *t) {
  if (!t) return THAPI_E_INVAL;
  {
    std::lock_guard<std::mutex> run(t->run_mu);
    hipSetDevice(t->dev);
    if (t->st) hipStreamSynchronize(t->st);
    free_all(t);
  }
  delete t;
  return THAPI_OK;
}

int thapi_tally_timings(thapi_tally *t, double *ms, int n) {
  if (!t || (n && !ms)) return THAPI_E_INVAL;
  int k = std::min<int>(n, TM_N);
  for (int i = 0; i < k; i++) ms[i] = t->timings[i];
  return k;
}

}  // extern "C"
