// tt_range.hip -- the fused per-range kernel of the tally pipeline.
//
// One workgroup owns one contiguous range of one stream's records and walks
// it tile by tile.  Per tile of T records it
//   1. decodes the records with coalesced 8-byte loads (FIXED24: 3 words per
//      record; VAR16: 2 header words plus, for entries of sized functions and
//      kernel records, the u64 at payload offset 0, located by an exclusive
//      prefix scan of payload_len across the tile); the next tile's loads are
//      issued as soon as the current tile is decoded;
//   2. tallies device-kernel records (kind 2) straight into an LDS table;
//   3. maps each API record's thread id to a range-local slot through an LDS
//      hash (new threads are resolved to a global thread slot once per range);
//   4. sorts the tile's API records stably by slot with wavefront ballots
//      (the rank of a record among equal slots is a popcount of the ballot
//      match mask), so each thread's records become contiguous and stay in
//      record order;
//   5. cuts every thread's records into runs of at most R and lets each lane
//      walk one run with a run-local call stack (entry: push; exit: pop and
//      match), the stack operations that define a call's interval (paper
//      section 3.3) and its tally (section 3.4, the table of section 4.3);
//   6. folds the runs in parallel: a segmented scan gives every run its start
//      depth, so an exit that found its run's stack empty knows the level it
//      closes; the run that opened that level is the nearest earlier run of
//      the thread whose lowest level lies below it (a previous-smaller-value
//      search), or the thread's stack carried from earlier tiles; children
//      time is credited to parents with LDS atomics, then self time and the
//      tally are computed for every call in one parallel pass;
//   7. updates each thread's carried stack with the calls still open.
// An exit that closes a call opened before the range is written to the range
// summary (U item) with the children time that call collected inside the
// range; the calls still open at the range end are written as O items.  The
// combine kernel folds the summaries of consecutive ranges onto the thread
// stacks carried on the device between ranges and flushes.
#include "tt_common.h"

namespace tt {

constexpr uint32_t NIL16 = 0xFFFFu;
// tile_fk bits: [0,16) fn | 16 kind (0 entry, 1 exit) | flags | [24,32) rank of a U item in its run
constexpr uint32_t FK_EXIT = 1u << 16;
constexpr uint32_t FK_U = 1u << 17;      // exit that found its run's stack empty
constexpr uint32_t FK_LOCAL = 1u << 18;  // exit matched inside its run
constexpr uint32_t FK_MIS = 1u << 19;    // popped entry has another fn: not tallied
constexpr uint32_t FK_NEG = 1u << 20;    // exit earlier than its entry: not tallied
constexpr uint32_t FK_REAL = 1u << 21;   // U item matched to a real entry (tile or carried stack)
// partner references of U items (tile_lnk after the fold)
constexpr uint32_t REF_CARRIED = 0x8000u;  // | position in the carried stack
constexpr uint32_t REF_VIRTUAL = 0xC000u;  // | levels below the thread's floor (opened before the range)
constexpr uint32_t REF_LOST = 0xBFFFu;     // beyond the stack capacity (depth overflow)
constexpr int32_t BIG = 0x3FFFFFFF;

struct RangeLds {
  // tile, sorted by slot
  uint64_t *tile_ts;   // timestamp (a real U item's slot is reused for its inclusive time)
  uint64_t *tile_ch;   // entry: children time; local exit: inclusive time; U item: children time in run
  uint64_t *tile_by;   // VAR16 transfer size of entries
  uint32_t *tile_fk;
  uint16_t *tile_lnk;  // entry: entry below it on its run stack; local exit: its entry; U item: run, then partner
  uint8_t *tile_slot;
  // runs
  uint32_t *run_info;  // start (16) | length (8) | slot (8)
  uint32_t *run_uo;    // U items (16) | open entries at the end (16)
  uint32_t *run_hm;    // max local height (16) | max local level (16, signed)
  uint64_t *run_base;  // children time owed to the call below the run's entries at its end
  int32_t *run_ds, *run_m, *run_pm, *run_suf;  // start level, lowest level, prefix / suffix minimum
  uint16_t *oidx;      // [run][level - m - 1] -> open entry
  // thread slots
  uint32_t *s_gslot, *s_flags, *s_run0;
  int32_t *s_u, *s_o, *s_H, *s_M;
  uint64_t *s_facc, *s_first, *s_last, *s_lastnew;
  // carried stacks [slot][D] and children time of virtual levels [slot][D]
  uint64_t *c_ts, *c_ch, *c_by, *vacc;
  uint16_t *c_fn;
  // tally hash
  uint32_t *t_key, *t_cnt, *t_imin, *t_imax, *t_smin, *t_smax;
  uint64_t *t_isum, *t_ssum, *t_bsum;
  // kernel tally
  uint32_t *q_cnt, *q_min, *q_max;
  uint64_t *q_sum;
  // thread map and sort
  uint64_t *tidmap;
  uint32_t *wcnt, *wbase, *soff;
  uint32_t *newtid, *newbucket;
  uint32_t *misc;   // [0] nslots, [1] new ids, [2] runs in tile, [3] API records in tile
  uint32_t *cnt;    // [ST_N] range-local counters
  uint32_t *wsum;   // [NWAVES] per-wave payload sums
};

__host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
__host__ __device__ inline uint32_t nruns_max(uint32_t T, uint32_t R) { return T / R + S_MAX; }
// Distinct threads one range can hold: their carried stacks live in LDS.
__host__ __device__ inline uint32_t slot_cap(uint32_t D) { return D <= 16 ? (uint32_t)S_MAX : 1024u / D; }

// Byte layout of the dynamic LDS; the same function sizes it on the host.
template <bool CARVE>
__host__ __device__ inline size_t range_lds_layout(uint8_t *base, RangeLds *L, uint32_t T, uint32_t R, uint32_t E,
                                                   uint32_t KL, uint32_t D, int fmt) {
  size_t o = 0;
  auto take = [&](size_t bytes) -> uint8_t * {
    o = align_up(o, 16);
    uint8_t *p = CARVE ? base + o : nullptr;
    o += bytes;
    return p;
  };
  const uint32_t NR = nruns_max(T, R);
  uint8_t *p;
#define TAKE(field, type, count) p = take(sizeof(type) * (size_t)(count)); if (CARVE) L->field = (type *)p
  TAKE(tile_ts, uint64_t, T);
  TAKE(tile_ch, uint64_t, T);
  TAKE(tile_by, uint64_t, fmt == 2 ? T : 0);
  TAKE(tile_fk, uint32_t, T);
  TAKE(tile_lnk, uint16_t, T);
  TAKE(tile_slot, uint8_t, T);
  TAKE(run_info, uint32_t, NR);
  TAKE(run_uo, uint32_t, NR);
  TAKE(run_hm, uint32_t, NR);
  TAKE(run_base, uint64_t, NR);
  TAKE(run_ds, int32_t, NR);
  TAKE(run_m, int32_t, NR);
  TAKE(run_pm, int32_t, NR);
  TAKE(run_suf, int32_t, NR);
  TAKE(oidx, uint16_t, (size_t)NR * R);
  TAKE(s_gslot, uint32_t, S_MAX);
  TAKE(s_flags, uint32_t, S_MAX);
  TAKE(s_run0, uint32_t, S_MAX + 1);
  TAKE(s_u, int32_t, S_MAX);
  TAKE(s_o, int32_t, S_MAX);
  TAKE(s_H, int32_t, S_MAX);
  TAKE(s_M, int32_t, S_MAX);
  TAKE(s_facc, uint64_t, S_MAX);
  TAKE(s_first, uint64_t, S_MAX);
  TAKE(s_last, uint64_t, S_MAX);
  TAKE(s_lastnew, uint64_t, S_MAX);
  TAKE(c_ts, uint64_t, (size_t)slot_cap(D) * D);
  TAKE(c_ch, uint64_t, (size_t)slot_cap(D) * D);
  TAKE(c_by, uint64_t, fmt == 2 ? (size_t)slot_cap(D) * D : 0);
  TAKE(vacc, uint64_t, (size_t)slot_cap(D) * D);
  TAKE(c_fn, uint16_t, (size_t)slot_cap(D) * D);
  TAKE(t_key, uint32_t, E);
  TAKE(t_cnt, uint32_t, E);
  TAKE(t_imin, uint32_t, E);
  TAKE(t_imax, uint32_t, E);
  TAKE(t_smin, uint32_t, E);
  TAKE(t_smax, uint32_t, E);
  TAKE(t_isum, uint64_t, E);
  TAKE(t_ssum, uint64_t, E);
  TAKE(t_bsum, uint64_t, fmt == 2 ? E : 0);
  TAKE(q_cnt, uint32_t, KL);
  TAKE(q_min, uint32_t, KL);
  TAKE(q_max, uint32_t, KL);
  TAKE(q_sum, uint64_t, KL);
  TAKE(tidmap, uint64_t, TIDMAP);
  TAKE(wcnt, uint32_t, NWAVES * S_MAX);
  TAKE(wbase, uint32_t, NWAVES * S_MAX);
  TAKE(soff, uint32_t, S_MAX + 1);
  TAKE(newtid, uint32_t, TIDMAP);
  TAKE(newbucket, uint32_t, TIDMAP);
  TAKE(misc, uint32_t, 8);
  TAKE(cnt, uint32_t, ST_N);
  TAKE(wsum, uint32_t, NWAVES * 2);
#undef TAKE
  return align_up(o, 16);
}

size_t range_lds_bytes(uint32_t T, uint32_t R, uint32_t E, uint32_t KL, uint32_t D, int fmt) {
  return range_lds_layout<false>(nullptr, nullptr, T, R, E, KL, D, fmt);
}

// ---------------------------------------------------------------- helpers
__device__ inline uint64_t lanemask_lt() {
  const uint32_t lane = __lane_id();
  return lane ? (~0ull >> (64 - lane)) : 0ull;
}
__device__ inline uint32_t wave_incl_scan(uint32_t v) {
  const int lane = __lane_id();
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    uint32_t t = __shfl_up(v, o, WAVE);
    if (lane >= o) v += t;
  }
  return v;
}
__device__ inline void lds_add32(uint32_t *p, uint32_t v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ inline void lds_add64(uint64_t *p, uint64_t v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ inline void lds_min32(uint32_t *p, uint32_t v) {
  __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ inline void lds_max32(uint32_t *p, uint32_t v) {
  __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ inline void g_add64(uint64_t *p, uint64_t v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void g_min64(uint64_t *p, uint64_t v) {
  __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void g_max64(uint64_t *p, uint64_t v) {
  __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The u64 at byte offset `off` of a buffer of any alignment: two aligned
// 8-byte loads and a funnel shift (the aligned words lie in the allocation's
// granule, so they never cross it).
typedef const __attribute__((address_space(1))) uint64_t gu64;  // global-memory view (no flat accesses)

__device__ inline uint64_t load_u64_unaligned(const uint8_t *base, uint64_t off) {
  const uintptr_t a = (uintptr_t)(base + off);
  gu64 *p = (gu64 *)(a & ~(uintptr_t)7);
  const uint32_t sh = (uint32_t)(a & 7) * 8;
  const uint64_t lo = __builtin_nontemporal_load(p);
  if (sh == 0) return lo;
  const uint64_t hi = __builtin_nontemporal_load(p + 1);
  return (lo >> sh) | (hi << (64 - sh));
}

// Resolves (stream, tid) to its global thread slot, inserting it on first
// sight.  Lock-free open addressing in two phases: every lane first inserts
// or finds its key, and an inserting lane publishes the slot id before the
// probe loop ends; only after the whole wave has left that loop does a lane
// that found a key inserted elsewhere wait for its slot id.  (Waiting inside
// the probe loop could deadlock: a lane of one wave spinning on a key whose
// inserter is a masked-off lane of another spinning wave, and vice versa.)
__device__ uint32_t resolve_gslot(const Tables &tb, uint32_t stream, uint32_t tid) {
  const uint64_t key = ((uint64_t)stream << 32) | tid;
  uint32_t h = (uint32_t)hash64(key) & tb.gmask;
  uint32_t result = GV_INVALID;
  bool wait = false;
  for (uint32_t probe = 0; probe <= tb.gmask; probe++) {
    const uint64_t old = atomicCAS((unsigned long long *)&tb.gkeys[h], (unsigned long long)EMPTY64,
                                   (unsigned long long)key);
    if (old == EMPTY64) {
      uint32_t g = atomicAdd(tb.n_gslots, 1u);
      if (g >= tb.max_threads) {
        atomicOr(tb.err, ERR_CAPACITY);
        g = GV_INVALID;
      } else {
        tb.th_stream[g] = stream;
        tb.th_tid[g] = tid;
      }
      __hip_atomic_store(&tb.gvals[h], g, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      result = g;
      break;
    }
    if (old == key) { wait = true; break; }
    h = (h + 1) & tb.gmask;
  }
  if (wait) {
    uint32_t v;
    while ((v = __hip_atomic_load(&tb.gvals[h], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)) == GV_PENDING)
      __builtin_amdgcn_s_sleep(2);
    result = v;
  } else if (result == GV_INVALID) {
    atomicOr(tb.err, ERR_CAPACITY);
  }
  return result;
}

// LDS tally layout: the first `direct_slots(n_fns, E) * n_fns` entries are
// indexed directly by slot * n_fns + fn (no probing); the rest is an
// open-addressing hash keyed (slot << 16 | fn) for slots beyond that.
__host__ __device__ inline uint32_t direct_slots(uint32_t n_fns, uint32_t E) {
  const uint32_t d = n_fns <= E ? E / n_fns : 0;
  return d < (uint32_t)S_MAX ? d : (uint32_t)S_MAX;
}

// Adds one completed call to the (slot, fn) entry of the LDS tally.
// Durations that do not fit 32 bits update the global min/max directly; a
// key that finds no room goes to the global tally with atomics.
template <int FMT>
__device__ inline void tally_call(const RangeLds &L, uint32_t E, const Tables &tb, uint32_t slot, uint32_t gslot,
                                  uint32_t fn, uint64_t incl, uint64_t self, uint64_t bytes) {
  if (fn >= tb.n_fns || slot >= (uint32_t)S_MAX) return;
  const uint32_t nd = direct_slots(tb.n_fns, E);
  const uint32_t d0 = nd * tb.n_fns;
  uint32_t h = 0;
  bool found = false;
  if (slot < nd) {
    h = slot * tb.n_fns + fn;
    found = true;
  } else if (E > d0) {
    const uint32_t key = (slot << 16) | fn;
    const uint32_t span = E - d0;
    h = d0 + hash32(key) % span;
    for (uint32_t probe = 0; probe < span; probe++) {
      const uint32_t k = L.t_key[h];
      if (k == key) { found = true; break; }
      if (k == EMPTY32) {
        const uint32_t old = atomicCAS(&L.t_key[h], EMPTY32, key);
        if (old == EMPTY32 || old == key) { found = true; break; }
      }
      h = h + 1 < E ? h + 1 : d0;
    }
  }
  Tally *g = gslot < tb.max_threads ? &tb.tally[(size_t)gslot * tb.n_fns + fn] : nullptr;
  if (found) {
    lds_add32(&L.t_cnt[h], 1u);
    lds_add64(&L.t_isum[h], incl);
    lds_add64(&L.t_ssum[h], self);
    if (FMT == 2 && bytes) lds_add64(&L.t_bsum[h], bytes);
    if (incl < EMPTY32) { lds_min32(&L.t_imin[h], (uint32_t)incl); lds_max32(&L.t_imax[h], (uint32_t)incl); }
    else if (g) { g_min64(&g->incl_min, incl); g_max64(&g->incl_max, incl); }
    if (self < EMPTY32) { lds_min32(&L.t_smin[h], (uint32_t)self); lds_max32(&L.t_smax[h], (uint32_t)self); }
    else if (g) { g_min64(&g->self_min, self); g_max64(&g->self_max, self); }
  } else if (g) {
    g_add64(&g->count, 1);
    g_add64(&g->incl_sum, incl); g_min64(&g->incl_min, incl); g_max64(&g->incl_max, incl);
    g_add64(&g->self_sum, self); g_min64(&g->self_min, self); g_max64(&g->self_max, self);
    if (bytes) g_add64(&g->bytes_sum, bytes);
  }
}

// ------------------------------------------------------------------ scans
// Wave-level segmented inclusive scans over int32; `head` marks the first
// element of a segment (forward) or `tail` its last element (backward).
// `closed` returns whether the lane's segment boundary lies inside the wave.
__device__ inline int32_t seg_scan_add(int32_t v, bool head, bool &closed) {
  const int lane = __lane_id();
  int f = head;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const int32_t t = __shfl_up(v, o, WAVE);
    const int tf = __shfl_up(f, o, WAVE);
    if (lane >= o) { if (!f) v += t; f |= tf; }
  }
  closed = f;
  return v;
}
__device__ inline int32_t seg_scan_min(int32_t v, bool head, bool &closed) {
  const int lane = __lane_id();
  int f = head;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const int32_t t = __shfl_up(v, o, WAVE);
    const int tf = __shfl_up(f, o, WAVE);
    if (lane >= o) { if (!f) v = t < v ? t : v; f |= tf; }
  }
  closed = f;
  return v;
}
__device__ inline int32_t seg_rscan_min(int32_t v, bool tail, bool &closed) {
  const int lane = __lane_id();
  int f = tail;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const int32_t t = __shfl_down(v, o, WAVE);
    const int tf = __shfl_down(f, o, WAVE);
    if (lane + o < WAVE) { if (!f) v = t < v ? t : v; f |= tf; }
  }
  closed = f;
  return v;
}

// One tile of the range: decode `cur*`, prefetch the next tile into `nxt*`,
// then slot map, sort, walk, fold, tally and carry.  Force-inlined twice by
// the kernel so the two register buffers alternate without copies.
struct Counters { uint32_t c[ST_N]; };

template <int FMT, int ROWS, int R>
__device__ __forceinline__ void tile_pass(RangeLds &L, const Tables &tb, const uint32_t E, const uint32_t KL,
                                          const uint32_t D, const Range &rg, const Seg &sg, gu64 *grec,
                                          const uint64_t last_rec, const uint64_t t0, const uint64_t (&cur0)[ROWS],
                                          const uint64_t (&cur1)[ROWS], const uint64_t (&cur2)[ROWS],
                                          uint64_t (&nxt0)[ROWS], uint64_t (&nxt1)[ROWS], uint64_t (&nxt2)[ROWS],
                                          uint64_t &pay_run, const size_t sbase, UItem *__restrict__ ru,
                                          Counters &C) {
  constexpr uint32_t T = ROWS * WG;
  constexpr uint32_t RS = FMT == 2 ? 16 : 24;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid >> 6;
  const uint32_t n = (uint32_t)((rg.n - t0) < T ? (rg.n - t0) : T);
    uint64_t r_ts[ROWS], r_x[ROWS], r_by[ROWS];
    uint32_t r_tid[ROWS], r_fk[ROWS], r_slot[ROWS], r_rank[ROWS];
    // ---- P1. decode, then prefetch the next tile
#pragma unroll
    for (int r = 0; r < ROWS; r++) {
      r_ts[r] = cur0[r];
      r_tid[r] = (uint32_t)cur1[r];
      r_fk[r] = (uint32_t)(cur1[r] >> 32);  // fn | kind << 16 | payload_len << 24
      r_x[r] = cur2[r];
      r_by[r] = 0;
    }
#pragma unroll
    for (int r = 0; r < ROWS; r++) {
      const uint32_t li = (uint32_t)w * (T / NWAVES) + (uint32_t)r * WAVE + lane;
      uint64_t idx = rg.begin + t0 + T + li;
      idx = idx < last_rec ? idx : last_rec;
      gu64 *p = grec + idx * (RS / 8);
      nxt0[r] = __builtin_nontemporal_load(p);
      nxt1[r] = __builtin_nontemporal_load(p + 1);
      nxt2[r] = FMT == 1 ? __builtin_nontemporal_load(p + 2) : 0;
    }
    // VAR16: payload offsets by an exclusive scan of payload_len in record order
    if (FMT == 2) {
      uint32_t run = 0;
      uint32_t excl[ROWS];
#pragma unroll
      for (int r = 0; r < ROWS; r++) {
        const uint32_t li = (uint32_t)w * (T / NWAVES) + (uint32_t)r * WAVE + lane;
        const uint32_t v = li < n ? (r_fk[r] >> 24) : 0;
        const uint32_t inc = wave_incl_scan(v);
        excl[r] = run + inc - v;
        run += __shfl(inc, WAVE - 1, WAVE);
      }
      if (lane == 0) L.wsum[w] = run;
      __syncthreads();
      uint32_t wpre = 0, tot = 0;
      for (int k = 0; k < NWAVES; k++) { const uint32_t s = L.wsum[k]; if (k < w) wpre += s; tot += s; }
#pragma unroll
      for (int r = 0; r < ROWS; r++) {
        const uint32_t li = (uint32_t)w * (T / NWAVES) + (uint32_t)r * WAVE + lane;
        const uint32_t fn = r_fk[r] & 0xFFFFu, kind = (r_fk[r] >> 16) & 0xFFu, plen = r_fk[r] >> 24;
        const uint64_t off = pay_run + wpre + excl[r];
        const bool sized = li < n && kind == 0 && fn < tb.n_fns && plen >= 8 && tb.has_size && tb.has_size[fn];
        const bool kend = li < n && kind == 2 && plen >= 8;
        if (sized || kend) {
          const uint64_t v = load_u64_unaligned(sg.pay, off);
          if (sized) r_by[r] = v; else r_x[r] = v;
        }
      }
      pay_run += tot;
      __syncthreads();
    }
    // ---- P2. kernel records, validity, counters
    uint32_t n_ent = 0, n_exi = 0, n_kern = 0, n_bad = 0;
#pragma unroll
    for (int r = 0; r < ROWS; r++) {
      const uint32_t li = (uint32_t)w * (T / NWAVES) + (uint32_t)r * WAVE + lane;
      const uint32_t fn = r_fk[r] & 0xFFFFu, kind = (r_fk[r] >> 16) & 0xFFu, plen = r_fk[r] >> 24;
      r_slot[r] = EMPTY32;
      if (li >= n) continue;
      if (kind == 2) {
        const uint64_t end = r_x[r];
        const bool ok = fn < tb.n_kid && (FMT == 1 || plen >= 8) && end >= r_ts[r];
        if (ok) {
          const uint64_t d = end - r_ts[r];
          n_kern++;
          if (fn < KL) {
            lds_add32(&L.q_cnt[fn], 1u);
            lds_add64(&L.q_sum[fn], d);
            if (d < EMPTY32) { lds_min32(&L.q_min[fn], (uint32_t)d); lds_max32(&L.q_max[fn], (uint32_t)d); }
            else {
              KTally *kt = &tb.ktally[(size_t)sg.stream * tb.n_kid + fn];
              g_min64(&kt->min, d); g_max64(&kt->max, d);
            }
          } else {
            KTally *kt = &tb.ktally[(size_t)sg.stream * tb.n_kid + fn];
            g_add64(&kt->count, 1); g_add64(&kt->sum, d); g_min64(&kt->min, d); g_max64(&kt->max, d);
          }
        } else {
          n_bad++;
        }
      } else if (kind <= 1 && fn < tb.n_fns) {
        r_slot[r] = 0;
        if (kind == 0) n_ent++; else n_exi++;
      } else {
        n_bad++;
      }
    }
    C.c[ST_ENTRIES] += n_ent;
    C.c[ST_EXITS] += n_exi;
    C.c[ST_KERNEL] += n_kern;
    C.c[ST_BAD] += n_bad;
    if (tid == 0) C.c[ST_RECORDS] += n;
    // ---- P3. thread id -> local slot
    // bucket word: bit 63 occupied, bit 62 pending, [32,40) slot, [0,32) tid
    bool any_miss = false;
#pragma unroll
    for (int r = 0; r < ROWS; r++) {
      if (r_slot[r] == EMPTY32) continue;
      const uint32_t t = r_tid[r];
      uint32_t h = hash32(t) & (TIDMAP - 1);
      for (uint32_t probe = 0; probe < TIDMAP; probe++) {
        const uint64_t e = L.tidmap[h];
        if (e == 0) { any_miss = true; r_slot[r] = EMPTY32 - 1; break; }
        if ((uint32_t)e == t) {
          if (e & (1ull << 62)) { any_miss = true; r_slot[r] = EMPTY32 - 1; }
          else r_slot[r] = (uint32_t)(e >> 32) & 0xFFu;
          break;
        }
        h = (h + 1) & (TIDMAP - 1);
      }
    }
    if (__syncthreads_or(any_miss)) {
#pragma unroll
      for (int r = 0; r < ROWS; r++) {
        if (r_slot[r] != EMPTY32 - 1) continue;
        const uint32_t t = r_tid[r];
        uint32_t h = hash32(t) & (TIDMAP - 1);
        for (uint32_t probe = 0; probe < TIDMAP; probe++) {
          const uint64_t want = (1ull << 63) | (1ull << 62) | t;
          const uint64_t old = atomicCAS((unsigned long long *)&L.tidmap[h], 0ull, (unsigned long long)want);
          if (old == 0) {
            const uint32_t k = atomicAdd(&L.misc[1], 1u);
            L.newtid[k] = t;
            L.newbucket[k] = h;
            break;
          }
          if ((uint32_t)old == t) break;
          h = (h + 1) & (TIDMAP - 1);
        }
      }
      __syncthreads();
      const uint32_t n_new = L.misc[1], base = L.misc[0];
      const uint32_t scap = slot_cap(D);
      if ((uint32_t)tid < n_new) {
        const uint32_t s = base + tid;
        const uint32_t t = L.newtid[tid];
        if (s < scap) {
          L.s_gslot[s] = resolve_gslot(tb, sg.stream, t);
          L.tidmap[L.newbucket[tid]] = (1ull << 63) | ((uint64_t)s << 32) | t;
        } else {
          atomicOr(tb.err, ERR_RANGE_THREADS);
          L.tidmap[L.newbucket[tid]] = (1ull << 63) | (0xFFull << 32) | t;
        }
      }
      __syncthreads();
      if (tid == 0) { L.misc[0] = base + n_new < scap ? base + n_new : scap; L.misc[1] = 0; }
#pragma unroll
      for (int r = 0; r < ROWS; r++) {
        if (r_slot[r] != EMPTY32 - 1) continue;
        const uint32_t t = r_tid[r];
        uint32_t h = hash32(t) & (TIDMAP - 1);
        r_slot[r] = EMPTY32;
        for (uint32_t probe = 0; probe < TIDMAP; probe++) {
          const uint64_t e = L.tidmap[h];
          if (e == 0) break;
          if ((uint32_t)e == t) { r_slot[r] = (uint32_t)(e >> 32) & 0xFFu; break; }
          h = (h + 1) & (TIDMAP - 1);
        }
        if (r_slot[r] >= scap) r_slot[r] = EMPTY32;  // over the per-range thread limit: the flush fails
      }
      __syncthreads();
    }
    const uint32_t nslots = L.misc[0];
    // ---- P4. stable sort of the API records by slot
    uint32_t nbits = 0;
    while ((1u << nbits) < nslots) nbits++;
    if (lane < S_MAX) L.wcnt[w * S_MAX + lane] = 0;
#pragma unroll
    for (int r = 0; r < ROWS; r++) {
      const bool valid = r_slot[r] != EMPTY32;
      const uint32_t s = valid ? r_slot[r] : 0;
      uint64_t mask = __ballot(valid);
      for (uint32_t b = 0; b < nbits; b++) {
        const uint64_t bb = __ballot(valid && ((s >> b) & 1u));
        mask &= ((s >> b) & 1u) ? bb : ~bb;
      }
      const uint32_t rk = (uint32_t)__popcll(mask & lanemask_lt());
      const uint32_t c = (uint32_t)__popcll(mask);
      uint32_t base = 0;
      if (valid) base = L.wcnt[w * S_MAX + s];
      r_rank[r] = base + rk;
      if (valid && rk == 0) L.wcnt[w * S_MAX + s] = base + c;
    }
    __syncthreads();
    if (w == 0) {
      uint32_t tot = 0;
      if ((uint32_t)lane < nslots)
        for (int k = 0; k < NWAVES; k++) tot += L.wcnt[k * S_MAX + lane];
      const uint32_t inc = wave_incl_scan(tot);
      if ((uint32_t)lane < nslots) {
        uint32_t acc = inc - tot;
        L.soff[lane] = acc;
        for (int k = 0; k < NWAVES; k++) { L.wbase[k * S_MAX + lane] = acc; acc += L.wcnt[k * S_MAX + lane]; }
      }
      if (lane == WAVE - 1) L.soff[nslots] = inc;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ROWS; r++) {
      if (r_slot[r] == EMPTY32) continue;
      const uint32_t pos = L.wbase[w * S_MAX + r_slot[r]] + r_rank[r];
      L.tile_ts[pos] = r_ts[r];
      L.tile_fk[pos] = (r_fk[r] & 0xFFFFu) | (((r_fk[r] >> 16) & 1u) << 16);
      L.tile_slot[pos] = (uint8_t)r_slot[r];
      if (FMT == 2) L.tile_by[pos] = r_by[r];
    }
    __syncthreads();
    const uint32_t napi = L.soff[nslots];
    // ---- P5. timestamp order per thread; runs of at most R records per thread
    {
      uint32_t c_tsreg = 0;
      for (uint32_t p = tid; p < napi; p += WG) {
        const uint32_t s = L.tile_slot[p];
        const uint64_t ts = L.tile_ts[p];
        if (p > L.soff[s]) {
          if (ts < L.tile_ts[p - 1]) c_tsreg++;
        } else if (L.s_flags[s] & RF_HAS_TS) {
          if (ts < L.s_last[s]) c_tsreg++;
        } else {
          L.s_first[s] = ts;
        }
        if (p + 1 == L.soff[s + 1]) L.s_lastnew[s] = ts;
      }
      C.c[ST_TSREG] += c_tsreg;
    }
    if (w == 0) {
      const uint32_t c = (uint32_t)lane < nslots ? L.soff[lane + 1] - L.soff[lane] : 0;
      const uint32_t nr = (c + R - 1) / R;
      const uint32_t inc = wave_incl_scan(nr);
      if ((uint32_t)lane < nslots) L.s_run0[lane] = inc - nr;
      if (lane == WAVE - 1) { L.s_run0[nslots] = inc; L.misc[2] = inc; }
    }
    for (uint32_t i = tid; i < nslots * D; i += WG) L.vacc[i] = 0;
    __syncthreads();
    const uint32_t NR = L.misc[2];
    for (uint32_t t = tid; t < NR; t += WG) {
      uint32_t lo = 0, hi = nslots - 1;
      while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (L.s_run0[mid] <= t) lo = mid; else hi = mid - 1;
      }
      const uint32_t s = lo;
      const uint32_t a = L.soff[s] + (t - L.s_run0[s]) * R;
      const uint32_t len = (L.soff[s + 1] - a) < R ? (L.soff[s + 1] - a) : R;
      L.run_info[t] = a | (len << 16) | (s << 24);
    }
    __syncthreads();
    // ---- P6. walk: one lane per run, run-local stack linked through the tile
    for (uint32_t t = tid; t < NR; t += WG) {
      const uint32_t info = L.run_info[t];
      const uint32_t a = info & 0xFFFFu, len = (info >> 16) & 0xFFu;
      uint32_t top = NIL16;
      uint64_t topc = 0, pend = 0;
      int32_t h = 0, nu = 0, Hr = 0, Mr = 0;
#pragma unroll
      for (int i = 0; i < R; i++) {
        if ((uint32_t)i >= len) break;
        const uint32_t p = a + i;
        const uint64_t ts = L.tile_ts[p];
        const uint32_t fk = L.tile_fk[p];
        if (!(fk & FK_EXIT)) {
          if (top != NIL16) L.tile_ch[top] = topc;
          L.tile_lnk[p] = (uint16_t)top;
          top = p;
          topc = 0;
          h++;
          Hr = h > Hr ? h : Hr;
          Mr = h - nu > Mr ? h - nu : Mr;
        } else if (top != NIL16) {
          const uint32_t e = top;
          const uint64_t ets = L.tile_ts[e];
          const uint32_t efn = L.tile_fk[e] & 0xFFFFu;
          const uint32_t nt = L.tile_lnk[e];
          L.tile_ch[e] = topc;
          uint32_t fl = FK_LOCAL;
          uint64_t incl = 0;
          if (efn != (fk & 0xFFFFu)) fl |= FK_MIS;
          else if (ts < ets) fl |= FK_NEG;
          else incl = ts - ets;
          L.tile_fk[p] = fk | fl;
          L.tile_ch[p] = incl;
          L.tile_lnk[p] = (uint16_t)e;
          const uint64_t add = (fl & (FK_MIS | FK_NEG)) ? 0 : incl;
          h--;
          top = nt;
          if (nt != NIL16) topc = L.tile_ch[nt] + add;
          else { pend += add; topc = 0; }
        } else {
          L.tile_fk[p] = fk | FK_U | ((uint32_t)nu << 24);
          L.tile_ch[p] = pend;
          L.tile_lnk[p] = (uint16_t)t;
          pend = 0;
          nu++;
        }
      }
      if (top != NIL16) L.tile_ch[top] = topc;
      uint32_t q = top;
      for (int32_t k = h - 1; k >= 0; k--) { L.oidx[t * R + k] = (uint16_t)q; q = L.tile_lnk[q]; }
      L.run_uo[t] = (uint32_t)nu | ((uint32_t)h << 16);
      L.run_base[t] = pend;
      L.run_hm[t] = ((uint32_t)Hr & 0xFFFFu) | ((uint32_t)Mr << 16);
    }
    __syncthreads();
    // ---- P7. per-thread scans over runs: start level, lowest level, floor, suffix minimum
    if (w == 0) {
      int32_t csum = 0, cmin = BIG, cslot = -1;
      for (uint32_t c0 = 0; c0 < NR; c0 += WAVE) {
        const uint32_t r = c0 + lane;
        const bool valid = r < NR;
        const int32_t s = valid ? (int32_t)(L.run_info[r] >> 24) : -1;
        const bool head = !valid || r == L.s_run0[s];
        const uint32_t uo = valid ? L.run_uo[r] : 0;
        const int32_t nu = (int32_t)(uo & 0xFFFFu), no = (int32_t)(uo >> 16);
        const int32_t v = no - nu;
        bool cl;
        int32_t inc = seg_scan_add(v, head, cl);
        if (!cl && s == cslot) inc += csum;
        const int32_t su = valid ? L.s_u[s] : 0;
        const int32_t ds = valid ? (L.s_o[s] - su) + inc - v : 0;
        const int32_t m = ds - nu;
        bool cl2;
        int32_t imin = seg_scan_min(valid ? m : BIG, head, cl2);
        if (!cl2 && s == cslot) imin = imin < cmin ? imin : cmin;
        const int32_t prev = __shfl_up(imin, 1, WAVE);
        int32_t exmin = BIG;
        if (!head) exmin = lane == 0 ? cmin : prev;
        const int32_t F = exmin < -su ? exmin : -su;
        if (valid) {
          L.run_ds[r] = ds;
          L.run_m[r] = m;
          L.run_pm[r] = exmin;
          const uint32_t hm = L.run_hm[r];
          const int32_t Hr = (int32_t)(hm & 0xFFFFu), Mr = (int32_t)(hm >> 16);
          const int32_t hh = ds - F + Mr > Hr ? ds - F + Mr : Hr;
          atomicMax(&L.s_H[s], hh);
          atomicMax(&L.s_M[s], ds + Mr);
        }
        csum = __shfl(inc, WAVE - 1, WAVE);
        cmin = __shfl(imin, WAVE - 1, WAVE);
        cslot = __shfl(s, WAVE - 1, WAVE);
      }
      int32_t rmin = BIG, rslot = -1;
      const int32_t nch = (int32_t)((NR + WAVE - 1) / WAVE);
      for (int32_t c = nch - 1; c >= 0; c--) {
        const uint32_t r = (uint32_t)c * WAVE + lane;
        const bool valid = r < NR;
        const int32_t s = valid ? (int32_t)(L.run_info[r] >> 24) : -1;
        const bool tail = !valid || r + 1 == L.s_run0[s + 1];
        const int32_t m = valid ? L.run_m[r] : BIG;
        bool cl;
        int32_t inc = seg_rscan_min(m, tail, cl);
        if (!cl && s == rslot) inc = inc < rmin ? inc : rmin;
        const int32_t nxt = __shfl_down(inc, 1, WAVE);
        int32_t suf = BIG;
        if (!tail) suf = lane == WAVE - 1 ? rmin : nxt;
        if (valid) L.run_suf[r] = suf;
        rmin = __shfl(inc, 0, WAVE);
        rslot = __shfl(s, 0, WAVE);
      }
    }
    __syncthreads();
    // ---- P8. fold: match exits that left their run, credit children time to parents
    // psv(r, lev): the open entry at level `lev` as seen from run r
    auto psv = [&](uint32_t r, int32_t lev, uint32_t s) -> uint32_t {
      if (L.run_pm[r] < lev) {  // some earlier run of this tile went below lev: the nearest one opened it
        int32_t j = (int32_t)r - 1;
        while (L.run_m[j] >= lev) j--;
        return L.oidx[(uint32_t)j * R + (uint32_t)(lev - L.run_m[j] - 1)];
      }
      const int32_t fl = -L.s_u[s];
      if (lev > fl) {
        const uint32_t pos = (uint32_t)(lev - fl - 1);
        return pos < D ? (REF_CARRIED | pos) : REF_LOST;
      }
      const uint32_t vk = (uint32_t)(fl - lev);
      return REF_VIRTUAL | (vk < 0x3FFFu ? vk : 0x3FFFu);
    };
    auto add_child = [&](uint32_t ref, uint32_t s, uint64_t v) {
      if (!v) return;
      if (ref < REF_CARRIED) lds_add64(&L.tile_ch[ref], v);
      else if (ref == REF_LOST) return;
      else if (ref < REF_VIRTUAL) lds_add64(&L.c_ch[s * D + (ref & 0x3FFFu)], v);
      else {
        const uint32_t vk = ref & 0x3FFFu;
        if (vk == 0) lds_add64(&L.s_facc[s], v);
        else if (vk - 1 < D && (uint32_t)L.s_u[s] + vk < D) lds_add64(&L.vacc[s * D + vk - 1], v);
      }
    };
    for (uint32_t p = tid; p < napi; p += WG) {
      const uint32_t fk = L.tile_fk[p];
      if (!(fk & FK_U)) continue;
      const uint32_t s = L.tile_slot[p];
      const uint32_t r = L.tile_lnk[p];
      const int32_t lev = L.run_ds[r] - (int32_t)(fk >> 24);
      const uint32_t ref = psv(r, lev, s);
      L.tile_lnk[p] = (uint16_t)ref;
      if (ref >= REF_VIRTUAL || ref == REF_LOST) continue;
      uint64_t ets;
      uint32_t efn;
      if (ref < REF_CARRIED) { ets = L.tile_ts[ref]; efn = L.tile_fk[ref] & 0xFFFFu; }
      else { const uint32_t i = s * D + (ref & 0x3FFFu); ets = L.c_ts[i]; efn = L.c_fn[i]; }
      const uint64_t ts = L.tile_ts[p];
      if (efn != (fk & 0xFFFFu)) { L.tile_fk[p] = fk | FK_MIS; continue; }
      if (ts < ets) { L.tile_fk[p] = fk | FK_NEG; continue; }
      const uint64_t incl = ts - ets;
      L.tile_ts[p] = incl;
      L.tile_fk[p] = fk | FK_REAL;
      add_child(psv(r, lev - 1, s), s, incl);
    }
    for (uint32_t t = tid; t < NR; t += WG) {
      const uint64_t b = L.run_base[t];
      if (!b) continue;
      const uint32_t s = L.run_info[t] >> 24;
      add_child(psv(t, L.run_m[t], s), s, b);
    }
    __syncthreads();
    // ---- P9. self time and tally of every call closed in this tile
    {
      uint32_t c_mis = 0, c_neg = 0, c_under = 0, c_orph = 0;
      for (uint32_t p = tid; p < napi; p += WG) {
        const uint32_t fk = L.tile_fk[p];
        if (!(fk & FK_EXIT)) continue;
        if (fk & FK_MIS) { c_mis++; continue; }
        if (fk & FK_NEG) { c_neg++; continue; }
        const uint32_t s = L.tile_slot[p];
        const uint32_t fn = fk & 0xFFFFu;
        uint64_t incl, ch, by = 0;
        if (fk & FK_LOCAL) {
          incl = L.tile_ch[p];
          const uint32_t e = L.tile_lnk[p];
          ch = L.tile_ch[e];
          if (FMT == 2) by = L.tile_by[e];
        } else if (fk & FK_REAL) {
          incl = L.tile_ts[p];
          const uint32_t ref = L.tile_lnk[p];
          if (ref < REF_CARRIED) {
            ch = L.tile_ch[ref] + L.tile_ch[p];
            if (FMT == 2) by = L.tile_by[ref];
          } else {
            const uint32_t i = s * D + (ref & 0x3FFFu);
            ch = L.c_ch[i] + L.tile_ch[p];
            if (FMT == 2) by = L.c_by[i];
          }
        } else {
          const uint32_t ref = L.tile_lnk[p];
          if (ref < REF_VIRTUAL) continue;  // beyond the stack capacity: the flush fails anyway
          const uint32_t vk = ref & 0x3FFFu;
          const uint32_t gi = (uint32_t)L.s_u[s] + vk;
          if (gi < D) {
            const uint64_t acc = vk == 0 ? L.s_facc[s] : (vk - 1 < D ? L.vacc[s * D + vk - 1] : 0);
            UItem *u = &ru[(sbase + s) * D + gi];
            u->ts = L.tile_ts[p]; u->child = acc + L.tile_ch[p]; u->fn = fn; u->pad = 0; u->pad2 = 0;
          } else {
            c_orph++;  // deeper than any stack can be: certainly an orphan exit
          }
          continue;
        }
        uint64_t self;
        if (ch <= incl) self = incl - ch; else { self = 0; c_under++; }
        tally_call<FMT>(L, E, tb, s, L.s_gslot[s], fn, incl, self, by);
      }
      C.c[ST_MISMATCH] += c_mis;
      C.c[ST_NEGDUR] += c_neg;
      C.c[ST_UNDER] += c_under;
      C.c[ST_ORPHAN] += c_orph;
    }
    __syncthreads();
    // ---- P10. carried stacks and thread state for the next tile
    for (uint32_t t = tid; t < NR; t += WG) {
      const uint32_t no = L.run_uo[t] >> 16;
      if (!no) continue;
      const uint32_t s = L.run_info[t] >> 24;
      const int32_t m = L.run_m[t], suf = L.run_suf[t];
      const uint32_t last = L.s_run0[s + 1] - 1;
      int32_t fl = L.run_pm[last] < L.run_m[last] ? L.run_pm[last] : L.run_m[last];
      fl = fl < -L.s_u[s] ? fl : -L.s_u[s];
      for (uint32_t k = 0; k < no; k++) {
        const int32_t lev = m + 1 + (int32_t)k;
        if (lev > suf) break;  // closed by a later run of this tile
        const uint32_t e = L.oidx[t * R + k];
        const uint32_t pos = (uint32_t)(lev - fl - 1);
        if (pos < D) {
          const uint32_t i = s * D + pos;
          L.c_ts[i] = L.tile_ts[e];
          L.c_ch[i] = L.tile_ch[e];
          L.c_fn[i] = (uint16_t)(L.tile_fk[e] & 0xFFFFu);
          if (FMT == 2) L.c_by[i] = L.tile_by[e];
        } else {
          atomicOr(&L.s_flags[s], RF_OVERFLOW);
        }
      }
    }
    if ((uint32_t)tid < nslots) {
      const uint32_t s = tid, r0 = L.s_run0[s], r1 = L.s_run0[s + 1];
      if (r1 > r0) {
        const uint32_t last = r1 - 1;
        const int32_t fl_old = -L.s_u[s];
        int32_t fl = L.run_pm[last] < L.run_m[last] ? L.run_pm[last] : L.run_m[last];
        fl = fl < fl_old ? fl : fl_old;
        const uint32_t uo = L.run_uo[last];
        const int32_t depth = L.run_ds[last] - (int32_t)(uo & 0xFFFFu) + (int32_t)(uo >> 16);
        if (fl < fl_old) {
          const uint32_t vk = (uint32_t)(fl_old - fl);
          L.s_facc[s] = (vk - 1 < D && (uint32_t)L.s_u[s] + vk < D) ? L.vacc[s * D + vk - 1] : 0;
        }
        L.s_u[s] = -fl;
        L.s_o[s] = depth - fl;
        atomicOr(&L.s_flags[s], RF_HAS_TS);
        L.s_last[s] = L.s_lastnew[s];
      }
    }
    __syncthreads();
}

// ------------------------------------------------------------------ kernel
template <int FMT, int ROWS, int R>
__global__ __launch_bounds__(WG) void k_range(const Seg *__restrict__ segs, const Range *__restrict__ ranges,
                                              Tables tb, Shape sh, RHdr *__restrict__ rhdr,
                                              UItem *__restrict__ ru, OItem *__restrict__ ro,
                                              uint32_t *__restrict__ rnslots) {
  extern __shared__ __align__(16) uint8_t smem[];
  constexpr uint32_t T = ROWS * WG;
  constexpr uint32_t RS = FMT == 2 ? 16 : 24;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid >> 6;
  const uint32_t D = tb.D, E = sh.E, KL = sh.KL;
  const Range rg = ranges[blockIdx.x];
  const Seg sg = segs[rg.seg];
  RangeLds L;
  range_lds_layout<true>(smem, &L, T, R, E, KL, D, FMT);

  for (uint32_t i = tid; i < E; i += WG) {
    L.t_key[i] = EMPTY32; L.t_cnt[i] = 0; L.t_imin[i] = EMPTY32; L.t_imax[i] = 0;
    L.t_smin[i] = EMPTY32; L.t_smax[i] = 0; L.t_isum[i] = 0; L.t_ssum[i] = 0;
    if (FMT == 2) L.t_bsum[i] = 0;
  }
  for (uint32_t i = tid; i < KL; i += WG) { L.q_cnt[i] = 0; L.q_min[i] = EMPTY32; L.q_max[i] = 0; L.q_sum[i] = 0; }
  for (uint32_t i = tid; i < TIDMAP; i += WG) L.tidmap[i] = 0;
  for (uint32_t i = tid; i < S_MAX; i += WG) {
    L.s_gslot[i] = GV_INVALID; L.s_flags[i] = 0; L.s_u[i] = 0; L.s_o[i] = 0; L.s_H[i] = 0; L.s_M[i] = 0;
    L.s_facc[i] = 0; L.s_first[i] = 0; L.s_last[i] = 0; L.s_lastnew[i] = 0;
  }
  for (uint32_t i = tid; i < ST_N; i += WG) L.cnt[i] = 0;
  if (tid < 8) L.misc[tid] = 0;
  __syncthreads();

  const size_t sbase = (size_t)blockIdx.x * S_MAX;
  uint64_t pay_run = rg.pay_begin;  // payload offset of the current tile's first record

  // raw words of the tile being decoded; the next tile's loads are issued
  // right after the current one is decoded.  Loads are unconditional (index
  // clamped to the range) so that nothing waits for them before the next tile.
  gu64 *grec = (gu64 *)sg.rec;
  const uint64_t last_rec = rg.begin + rg.n - 1;
  uint64_t a0[ROWS], a1[ROWS], a2[ROWS], b0[ROWS], b1[ROWS], b2[ROWS];
#pragma unroll
  for (int r = 0; r < ROWS; r++) {
    const uint32_t li = (uint32_t)w * (T / NWAVES) + (uint32_t)r * WAVE + lane;
    uint64_t idx = rg.begin + li;
    idx = idx < last_rec ? idx : last_rec;
    gu64 *p = grec + idx * (RS / 8);
    a0[r] = __builtin_nontemporal_load(p);
    a1[r] = __builtin_nontemporal_load(p + 1);
    a2[r] = FMT == 1 ? __builtin_nontemporal_load(p + 2) : 0;
  }
  Counters C;
#pragma unroll
  for (int k = 0; k < ST_N; k++) C.c[k] = 0;
  for (uint64_t t0 = 0; t0 < rg.n; t0 += 2 * T) {
    tile_pass<FMT, ROWS, R>(L, tb, E, KL, D, rg, sg, grec, last_rec, t0, a0, a1, a2, b0, b1, b2, pay_run, sbase, ru, C);
    if (t0 + T < rg.n)
      tile_pass<FMT, ROWS, R>(L, tb, E, KL, D, rg, sg, grec, last_rec, t0 + T, b0, b1, b2, a0, a1, a2, pay_run, sbase,
                              ru, C);
  }
#pragma unroll
  for (int k = 0; k < ST_N; k++)
    if (C.c[k]) lds_add32(&L.cnt[k], C.c[k]);
  __syncthreads();


  // ---- range end: summaries, tally and counter flush
  const uint32_t nslots = L.misc[0];
  if (tid == 0) rnslots[blockIdx.x] = nslots;
  if ((uint32_t)tid < nslots) {
    const uint32_t s = tid;
    RHdr hd;
    hd.gslot = L.s_gslot[s];
    hd.nu_total = (uint32_t)L.s_u[s];
    hd.nu_listed = hd.nu_total < D ? hd.nu_total : D;
    hd.n_o = (uint32_t)L.s_o[s];
    hd.floor = L.s_facc[s];
    hd.H = L.s_H[s]; hd.M = L.s_M[s];
    hd.first_ts = L.s_first[s]; hd.last_ts = L.s_last[s];
    hd.flags = L.s_flags[s];
    hd.pad = 0; hd.pad2 = 0;
    rhdr[sbase + s] = hd;
    const uint32_t no = hd.n_o < D ? hd.n_o : D;
    for (uint32_t k = 0; k < no; k++) {
      OItem *o = &ro[(sbase + s) * D + k];
      o->ts = L.c_ts[(size_t)s * D + k];
      o->child = L.c_ch[(size_t)s * D + k];
      o->bytes = FMT == 2 ? L.c_by[(size_t)s * D + k] : 0;
      o->fn = L.c_fn[(size_t)s * D + k];
      o->pad = 0;
    }
  }
  const uint32_t nd = direct_slots(tb.n_fns, E), d0 = nd * tb.n_fns;
  for (uint32_t i = tid; i < E; i += WG) {
    uint32_t s, fn;
    if (i < d0) {
      if (!L.t_cnt[i]) continue;
      s = i / tb.n_fns;
      fn = i - s * tb.n_fns;
    } else {
      const uint32_t key = L.t_key[i];
      if (key == EMPTY32) continue;
      s = key >> 16;
      fn = key & 0xFFFFu;
    }
    const uint32_t gs = L.s_gslot[s];
    if (gs >= tb.max_threads) continue;
    Tally *g = &tb.tally[(size_t)gs * tb.n_fns + fn];
    g_add64(&g->count, L.t_cnt[i]);
    g_add64(&g->incl_sum, L.t_isum[i]);
    g_add64(&g->self_sum, L.t_ssum[i]);
    if (FMT == 2 && L.t_bsum[i]) g_add64(&g->bytes_sum, L.t_bsum[i]);
    if (L.t_imin[i] != EMPTY32) g_min64(&g->incl_min, L.t_imin[i]);
    if (L.t_imax[i]) g_max64(&g->incl_max, L.t_imax[i]);
    if (L.t_smin[i] != EMPTY32) g_min64(&g->self_min, L.t_smin[i]);
    if (L.t_smax[i]) g_max64(&g->self_max, L.t_smax[i]);
  }
  for (uint32_t i = tid; i < KL; i += WG) {
    if (!L.q_cnt[i]) continue;
    KTally *kt = &tb.ktally[(size_t)sg.stream * tb.n_kid + i];
    g_add64(&kt->count, L.q_cnt[i]);
    g_add64(&kt->sum, L.q_sum[i]);
    if (L.q_min[i] != EMPTY32) g_min64(&kt->min, L.q_min[i]);
    if (L.q_max[i]) g_max64(&kt->max, L.q_max[i]);
  }
  for (uint32_t i = tid; i < ST_N; i += WG)
    if (L.cnt[i]) atomicAdd(&tb.sstats[(size_t)sg.stream * ST_N + i], (unsigned long long)L.cnt[i]);
}

// VAR16 pre-pass: payload bytes of each range (sum of payload_len).
__global__ __launch_bounds__(WG) void k_range_paylen(const Seg *__restrict__ segs, Range *__restrict__ ranges,
                                                     uint64_t *__restrict__ out) {
  __shared__ unsigned long long acc;
  if (threadIdx.x == 0) acc = 0;
  __syncthreads();
  const Range rg = ranges[blockIdx.x];
  const Seg sg = segs[rg.seg];
  uint64_t s = 0;
  for (uint64_t i = threadIdx.x; i < rg.n; i += WG) {
    const uint64_t w1 = __builtin_nontemporal_load((gu64 *)(sg.rec + (rg.begin + i) * 16) + 1);
    s += w1 >> 56;
  }
  atomicAdd(&acc, (unsigned long long)s);
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = acc;
}

// VAR16: exclusive prefix of the range payload sizes within each segment.
__global__ void k_range_payoff(const Seg *__restrict__ segs, uint32_t n_segs, const uint32_t *__restrict__ seg_first_range,
                               Range *__restrict__ ranges, const uint64_t *__restrict__ paylen) {
  const uint32_t sgi = blockIdx.x * blockDim.x + threadIdx.x;
  if (sgi >= n_segs) return;
  uint64_t acc = 0;
  for (uint32_t r = seg_first_range[sgi]; r < seg_first_range[sgi + 1]; r++) {
    ranges[r].pay_begin = acc;
    acc += paylen[r];
  }
}

// --------------------------------------------------------------- launchers
hipError_t launch_range(int fmt, uint32_t T, uint32_t R, const Seg *segs, const Range *ranges, uint32_t n_ranges,
                        const Tables &tb, const Shape &sh, RHdr *rhdr, UItem *ru, OItem *ro,
                        uint32_t *rnslots, hipStream_t st) {
  if (!n_ranges) return hipSuccess;
  dim3 grid(n_ranges), block(WG);
#define TT_LAUNCH(F, ROWS_, R_)                                                                                 \
  do {                                                                                                          \
    hipError_t e = hipFuncSetAttribute((const void *)k_range<F, ROWS_, R_>,                                    \
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh.lds_bytes);          \
    if (e != hipSuccess) return e;                                                                              \
    hipLaunchKernelGGL((k_range<F, ROWS_, R_>), grid, block, sh.lds_bytes, st, segs, ranges, tb, sh, rhdr, ru,  \
                       ro, rnslots);                                                                            \
    return hipGetLastError();                                                                                   \
  } while (0)
#define TT_SHAPES(F)                                  \
  if (T == 1024 && R == 8) TT_LAUNCH(F, 4, 8);        \
  if (T == 1024 && R == 16) TT_LAUNCH(F, 4, 16);      \
  if (T == 2048 && R == 8) TT_LAUNCH(F, 8, 8);        \
  if (T == 2048 && R == 16) TT_LAUNCH(F, 8, 16);
  if (fmt == 1) { TT_SHAPES(1) } else { TT_SHAPES(2) }
#undef TT_SHAPES
#undef TT_LAUNCH
  return hipErrorInvalidValue;
}

hipError_t launch_paylen(const Seg *segs, Range *ranges, uint32_t n_ranges, const uint32_t *seg_first_range,
                         uint32_t n_segs, uint64_t *paylen, hipStream_t st) {
  if (!n_ranges) return hipSuccess;
  hipLaunchKernelGGL(k_range_paylen, dim3(n_ranges), dim3(WG), 0, st, segs, ranges, paylen);
  hipLaunchKernelGGL(k_range_payoff, dim3((n_segs + 255) / 256), dim3(256), 0, st, segs, n_segs, seg_first_range,
                     ranges, paylen);
  return hipGetLastError();
}

}  // namespace tt
