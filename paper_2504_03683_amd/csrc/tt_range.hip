// tt_range.hip -- the fused per-range kernel of the tally pipeline.
//
// One workgroup owns one contiguous range of one stream's records and walks
// it tile by tile.  Per tile of T records it
//   1. decodes the records with coalesced 8-byte loads (FIXED24: 3 words per
//      record; VAR16: 2 header words plus, for entries of sized functions and
//      kernel records, the u64 at payload offset 0, located by an exclusive
//      prefix scan of payload_len across the tile);
//   2. tallies device-kernel records (kind 2) straight into an LDS table;
//   3. maps each API record's thread id to a range-local slot through an LDS
//      hash (new threads are resolved to a global thread slot once per range);
//   4. sorts the tile's API records stably by slot with wavefront ballots
//      (the rank of a record among equal slots is a popcount of the ballot
//      match mask), so each thread's records become contiguous and stay in
//      record order;
//   5. walks each slot's records with that thread's call stack kept in LDS
//      (entry: push; exit: pop, match, inclusive and self time, tally), the
//      exact sequence of stack operations of the definition of a call's
//      interval (paper section 3.3) and of the tally (section 3.4 / 4.3).
// An exit that finds the range-local stack empty closes a call opened before
// the range: it is written to the range summary (U item) with the children
// time that call collected inside the range, and the calls still open at the
// range end are written as O items.  The combine kernel folds the summaries
// of consecutive ranges onto the thread stacks carried on the device.
#include "tt_common.h"

namespace tt {

struct RangeLds {
  uint64_t *tile_ts, *tile_bytes;
  uint16_t *tile_fn;
  uint8_t *tile_kind;
  uint32_t *s_gslot, *s_nu, *s_flags;
  int32_t *s_h, *s_H, *s_M;
  uint64_t *s_floor, *s_first, *s_last;
  uint64_t *k_ts, *k_child, *k_bytes;
  uint16_t *k_fn;
  uint32_t *t_key, *t_cnt, *t_imin, *t_imax, *t_smin, *t_smax;
  uint64_t *t_isum, *t_ssum, *t_bsum;
  uint32_t *q_cnt, *q_min, *q_max;
  uint64_t *q_sum;
  uint64_t *tidmap;
  uint32_t *wcnt, *wbase, *soff;
  uint32_t *newtid, *newbucket;
  uint32_t *misc;   // [0] nslots, [1] n_new, [2] tile payload total low, [3] high
  uint32_t *cnt;    // [ST_N] range-local counters
  uint32_t *wsum;   // [NWAVES] per-wave payload sums
};

__host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Byte layout of the dynamic LDS; the same function sizes it on the host.
template <bool CARVE>
__host__ __device__ inline size_t range_lds_layout(uint8_t *base, RangeLds *L, uint32_t T, uint32_t E,
                                                   uint32_t KL, uint32_t D, int fmt) {
  size_t o = 0;
  auto take = [&](size_t bytes, size_t al) -> uint8_t * {
    o = align_up(o, al);
    uint8_t *p = CARVE ? base + o : nullptr;
    o += bytes;
    return p;
  };
  uint8_t *p;
  p = take(8ull * T, 16);                  if (CARVE) L->tile_ts = (uint64_t *)p;
  p = take(fmt == 2 ? 8ull * T : 0, 16);   if (CARVE) L->tile_bytes = (uint64_t *)p;
  p = take(2ull * T, 16);                  if (CARVE) L->tile_fn = (uint16_t *)p;
  p = take(1ull * T, 16);                  if (CARVE) L->tile_kind = (uint8_t *)p;
  p = take(4ull * S_MAX, 16);              if (CARVE) L->s_gslot = (uint32_t *)p;
  p = take(4ull * S_MAX, 16);              if (CARVE) L->s_nu = (uint32_t *)p;
  p = take(4ull * S_MAX, 16);              if (CARVE) L->s_flags = (uint32_t *)p;
  p = take(4ull * S_MAX, 16);              if (CARVE) L->s_h = (int32_t *)p;
  p = take(4ull * S_MAX, 16);              if (CARVE) L->s_H = (int32_t *)p;
  p = take(4ull * S_MAX, 16);              if (CARVE) L->s_M = (int32_t *)p;
  p = take(8ull * S_MAX, 16);              if (CARVE) L->s_floor = (uint64_t *)p;
  p = take(8ull * S_MAX, 16);              if (CARVE) L->s_first = (uint64_t *)p;
  p = take(8ull * S_MAX, 16);              if (CARVE) L->s_last = (uint64_t *)p;
  p = take(8ull * S_MAX * D, 16);          if (CARVE) L->k_ts = (uint64_t *)p;
  p = take(8ull * S_MAX * D, 16);          if (CARVE) L->k_child = (uint64_t *)p;
  p = take(fmt == 2 ? 8ull * S_MAX * D : 0, 16); if (CARVE) L->k_bytes = (uint64_t *)p;
  p = take(2ull * S_MAX * D, 16);          if (CARVE) L->k_fn = (uint16_t *)p;
  p = take(4ull * E, 16);                  if (CARVE) L->t_key = (uint32_t *)p;
  p = take(4ull * E, 16);                  if (CARVE) L->t_cnt = (uint32_t *)p;
  p = take(4ull * E, 16);                  if (CARVE) L->t_imin = (uint32_t *)p;
  p = take(4ull * E, 16);                  if (CARVE) L->t_imax = (uint32_t *)p;
  p = take(4ull * E, 16);                  if (CARVE) L->t_smin = (uint32_t *)p;
  p = take(4ull * E, 16);                  if (CARVE) L->t_smax = (uint32_t *)p;
  p = take(8ull * E, 16);                  if (CARVE) L->t_isum = (uint64_t *)p;
  p = take(8ull * E, 16);                  if (CARVE) L->t_ssum = (uint64_t *)p;
  p = take(fmt == 2 ? 8ull * E : 0, 16);   if (CARVE) L->t_bsum = (uint64_t *)p;
  p = take(4ull * KL, 16);                 if (CARVE) L->q_cnt = (uint32_t *)p;
  p = take(4ull * KL, 16);                 if (CARVE) L->q_min = (uint32_t *)p;
  p = take(4ull * KL, 16);                 if (CARVE) L->q_max = (uint32_t *)p;
  p = take(8ull * KL, 16);                 if (CARVE) L->q_sum = (uint64_t *)p;
  p = take(8ull * TIDMAP, 16);             if (CARVE) L->tidmap = (uint64_t *)p;
  p = take(4ull * NWAVES * S_MAX, 16);     if (CARVE) L->wcnt = (uint32_t *)p;
  p = take(4ull * NWAVES * S_MAX, 16);     if (CARVE) L->wbase = (uint32_t *)p;
  p = take(4ull * (S_MAX + 1), 16);        if (CARVE) L->soff = (uint32_t *)p;
  p = take(4ull * TIDMAP, 16);             if (CARVE) L->newtid = (uint32_t *)p;
  p = take(4ull * TIDMAP, 16);             if (CARVE) L->newbucket = (uint32_t *)p;
  p = take(4ull * 8, 16);                  if (CARVE) L->misc = (uint32_t *)p;
  p = take(4ull * ST_N, 16);               if (CARVE) L->cnt = (uint32_t *)p;
  p = take(4ull * NWAVES * 2, 16);         if (CARVE) L->wsum = (uint32_t *)p;
  return align_up(o, 16);
}

size_t range_lds_bytes(uint32_t T, uint32_t E, uint32_t KL, uint32_t D, int fmt) {
  return range_lds_layout<false>(nullptr, nullptr, T, E, KL, D, fmt);
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
__device__ inline uint64_t load_u64_unaligned(const uint8_t *base, uint64_t off) {
  const uintptr_t a = (uintptr_t)(base + off);
  const uint64_t *p = (const uint64_t *)(a & ~(uintptr_t)7);
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

// Adds one completed call to the (slot, fn) entry of the LDS tally hash.
// Durations that do not fit 32 bits update the global min/max directly.
template <int FMT>
__device__ inline void tally_call(const RangeLds &L, uint32_t E, const Tables &tb, uint32_t slot, uint32_t gslot,
                                  uint32_t fn, uint64_t incl, uint64_t self, uint64_t bytes) {
  const uint32_t key = (slot << 16) | fn;
  uint32_t h = hash32(key) & (E - 1);
  bool found = false;
  for (uint32_t probe = 0; probe < E; probe++) {
    uint32_t k = L.t_key[h];
    if (k == key) { found = true; break; }
    if (k == EMPTY32) {
      uint32_t old = atomicCAS(&L.t_key[h], EMPTY32, key);
      if (old == EMPTY32 || old == key) { found = true; break; }
    }
    h = (h + 1) & (E - 1);
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

// ------------------------------------------------------------------ kernel
template <int FMT, int ROWS>
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
  range_lds_layout<true>(smem, &L, T, E, KL, D, FMT);

  for (uint32_t i = tid; i < E; i += WG) {
    L.t_key[i] = EMPTY32; L.t_cnt[i] = 0; L.t_imin[i] = EMPTY32; L.t_imax[i] = 0;
    L.t_smin[i] = EMPTY32; L.t_smax[i] = 0; L.t_isum[i] = 0; L.t_ssum[i] = 0;
    if (FMT == 2) L.t_bsum[i] = 0;
  }
  for (uint32_t i = tid; i < KL; i += WG) { L.q_cnt[i] = 0; L.q_min[i] = EMPTY32; L.q_max[i] = 0; L.q_sum[i] = 0; }
  for (uint32_t i = tid; i < TIDMAP; i += WG) L.tidmap[i] = 0;
  for (uint32_t i = tid; i < S_MAX; i += WG) {
    L.s_gslot[i] = GV_INVALID; L.s_nu[i] = 0; L.s_flags[i] = 0; L.s_h[i] = 0; L.s_H[i] = 0; L.s_M[i] = 0;
    L.s_floor[i] = 0; L.s_first[i] = 0; L.s_last[i] = 0;
  }
  for (uint32_t i = tid; i < ST_N; i += WG) L.cnt[i] = 0;
  if (tid < 8) L.misc[tid] = 0;
  __syncthreads();

  uint64_t pay_run = rg.pay_begin;  // payload offset of the current tile's first record
  const size_t sbase = (size_t)blockIdx.x * S_MAX;

  for (uint64_t t0 = 0; t0 < rg.n; t0 += T) {
    const uint32_t n = (uint32_t)((rg.n - t0) < T ? (rg.n - t0) : T);
    uint64_t r_ts[ROWS], r_x[ROWS];
    uint32_t r_tid[ROWS], r_fk[ROWS], r_slot[ROWS], r_rank[ROWS];
    uint64_t r_bytes[ROWS];
    // ---- 1. decode
#pragma unroll
    for (int r = 0; r < ROWS; r++) {
      const uint32_t li = (uint32_t)w * (T / NWAVES) + (uint32_t)r * WAVE + lane;
      r_ts[r] = 0; r_tid[r] = 0; r_fk[r] = 0xFFu << 16; r_x[r] = 0; r_bytes[r] = 0;
      if (li < n) {
        const uint64_t *p = (const uint64_t *)(sg.rec + (rg.begin + t0 + li) * RS);
        const uint64_t w0 = __builtin_nontemporal_load(p);
        const uint64_t w1 = __builtin_nontemporal_load(p + 1);
        r_ts[r] = w0;
        r_tid[r] = (uint32_t)w1;
        // fn (16 bits) | kind (8 bits) << 16 | payload_len (8 bits) << 24
        r_fk[r] = (uint32_t)(w1 >> 32);
        if (FMT == 1) r_x[r] = __builtin_nontemporal_load(p + 2);
      }
    }
    // ---- VAR16: payload offsets by an exclusive scan of payload_len in record order
    if (FMT == 2) {
      uint32_t run = 0;
      uint32_t excl[ROWS];
#pragma unroll
      for (int r = 0; r < ROWS; r++) {
        const uint32_t v = r_fk[r] >> 24;
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
        const uint32_t fn = r_fk[r] & 0xFFFFu, kind = (r_fk[r] >> 16) & 0xFFu, plen = r_fk[r] >> 24;
        const uint64_t off = pay_run + wpre + excl[r];
        const bool sized = kind == 0 && fn < tb.n_fns && plen >= 8 && tb.has_size && tb.has_size[fn];
        const bool kend = kind == 2 && plen >= 8;
        if (sized || kend) {
          const uint64_t v = load_u64_unaligned(sg.pay, off);
          if (sized) r_bytes[r] = v; else r_x[r] = v;
        }
      }
      pay_run += tot;
      __syncthreads();  // wsum is reused next tile
    }
    // ---- 2. kernel records, validity, counters
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
        r_slot[r] = 0;  // API record, slot resolved below
        if (kind == 0) n_ent++; else n_exi++;
      } else {
        n_bad++;
      }
    }
    if (n_ent) lds_add32(&L.cnt[ST_ENTRIES], n_ent);
    if (n_exi) lds_add32(&L.cnt[ST_EXITS], n_exi);
    if (n_kern) lds_add32(&L.cnt[ST_KERNEL], n_kern);
    if (n_bad) lds_add32(&L.cnt[ST_BAD], n_bad);
    if (tid == 0) lds_add32(&L.cnt[ST_RECORDS], n);
    // ---- 3. thread id -> local slot
    // bucket word: bit 63 occupied, bit 62 pending, [32,40) slot, [0,32) tid
    bool any_miss = false;
    uint32_t r_bucket[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; r++) {
      r_bucket[r] = EMPTY32;
      if (r_slot[r] == EMPTY32) continue;
      const uint32_t t = r_tid[r];
      uint32_t h = hash32(t) & (TIDMAP - 1);
      for (uint32_t probe = 0; probe < TIDMAP; probe++) {
        const uint64_t e = L.tidmap[h];
        if (e == 0) { any_miss = true; r_slot[r] = EMPTY32 - 1; break; }          // absent
        if ((uint32_t)e == t) {
          if (e & (1ull << 62)) { any_miss = true; r_slot[r] = EMPTY32 - 1; }     // not published yet
          else r_slot[r] = (uint32_t)(e >> 32) & 0xFFu;
          break;
        }
        h = (h + 1) & (TIDMAP - 1);
      }
    }
    if (__syncthreads_or(any_miss)) {
      // claim buckets for absent thread ids; one claimant per id lists it
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
      if ((uint32_t)tid < n_new) {
        const uint32_t s = base + tid;
        const uint32_t t = L.newtid[tid];
        if (s < S_MAX) {
          L.s_gslot[s] = resolve_gslot(tb, sg.stream, t);
          L.tidmap[L.newbucket[tid]] = (1ull << 63) | ((uint64_t)s << 32) | t;
        } else {
          atomicOr(tb.err, ERR_RANGE_THREADS);
          L.tidmap[L.newbucket[tid]] = (1ull << 63) | (0xFFull << 32) | t;
        }
      }
      __syncthreads();
      if (tid == 0) { L.misc[0] = base + n_new < S_MAX ? base + n_new : S_MAX; L.misc[1] = 0; }
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
        if (r_slot[r] >= S_MAX) r_slot[r] = EMPTY32;  // over the per-range thread limit: flush fails
      }
      __syncthreads();
    }
    const uint32_t nslots = L.misc[0];
    // ---- 4. stable sort of the API records by slot
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
      L.tile_fn[pos] = (uint16_t)(r_fk[r] & 0xFFFFu);
      L.tile_kind[pos] = (uint8_t)((r_fk[r] >> 16) & 1u);
      if (FMT == 2) L.tile_bytes[pos] = r_bytes[r];
    }
    __syncthreads();
    // ---- 5. per-thread stack walk (one lane per slot)
    if ((uint32_t)tid < nslots) {
      const uint32_t s = tid;
      const uint32_t gs = L.s_gslot[s];
      int32_t h = L.s_h[s], H = L.s_H[s], M = L.s_M[s];
      uint32_t nu = L.s_nu[s], flags = L.s_flags[s];
      uint64_t floor_ = L.s_floor[s], first = L.s_first[s], last = L.s_last[s];
      uint32_t c_tsreg = 0, c_orphan = 0, c_mis = 0, c_neg = 0, c_under = 0;
      uint64_t *kts = L.k_ts + (size_t)s * D, *kch = L.k_child + (size_t)s * D;
      uint16_t *kfn = L.k_fn + (size_t)s * D;
      uint64_t *kby = FMT == 2 ? L.k_bytes + (size_t)s * D : nullptr;
      const uint32_t pe = L.soff[s + 1];
      for (uint32_t p = L.soff[s]; p < pe; p++) {
        const uint64_t ts = L.tile_ts[p];
        const uint32_t fn = L.tile_fn[p];
        const uint32_t kind = L.tile_kind[p];
        if (flags & RF_HAS_TS) { if (ts < last) c_tsreg++; }
        else { first = ts; flags |= RF_HAS_TS; }
        last = ts;
        if (kind == 0) {
          if (h < (int32_t)D) {
            kts[h] = ts; kch[h] = 0; kfn[h] = (uint16_t)fn;
            if (FMT == 2) kby[h] = L.tile_bytes[p];
          } else {
            flags |= RF_OVERFLOW;
          }
          h++;
          if (h > H) H = h;
          if (h - (int32_t)nu > M) M = h - (int32_t)nu;
        } else if (h > 0) {
          h--;
          if (h < (int32_t)D) {
            const uint64_t ets = kts[h];
            uint64_t incl = 0;
            bool ok = true;
            if (kfn[h] != fn) { c_mis++; ok = false; }
            else if (ts < ets) { c_neg++; ok = false; }
            if (ok) {
              incl = ts - ets;
              const uint64_t ch = kch[h];
              uint64_t self;
              if (ch <= incl) self = incl - ch; else { self = 0; c_under++; }
              tally_call<FMT>(L, E, tb, s, gs, fn, incl, self, FMT == 2 ? kby[h] : 0);
              if (h > 0) { if (h - 1 < (int32_t)D) kch[h - 1] += incl; }
              else floor_ += incl;
            }
          }
        } else {
          // closes a call opened before this range
          if (nu < D) {
            UItem *u = &ru[(sbase + s) * D + nu];
            u->ts = ts; u->child = floor_; u->fn = fn; u->pad = 0; u->pad2 = 0;
          } else {
            c_orphan++;  // deeper than any stack can be: certainly an orphan exit
          }
          nu++;
          floor_ = 0;
        }
      }
      L.s_h[s] = h; L.s_H[s] = H; L.s_M[s] = M; L.s_nu[s] = nu; L.s_flags[s] = flags;
      L.s_floor[s] = floor_; L.s_first[s] = first; L.s_last[s] = last;
      if (c_tsreg) lds_add32(&L.cnt[ST_TSREG], c_tsreg);
      if (c_orphan) lds_add32(&L.cnt[ST_ORPHAN], c_orphan);
      if (c_mis) lds_add32(&L.cnt[ST_MISMATCH], c_mis);
      if (c_neg) lds_add32(&L.cnt[ST_NEGDUR], c_neg);
      if (c_under) lds_add32(&L.cnt[ST_UNDER], c_under);
    }
    __syncthreads();
  }

  // ---- range end: summaries, tally and counter flush
  const uint32_t nslots = L.misc[0];
  if (tid == 0) rnslots[blockIdx.x] = nslots;
  if ((uint32_t)tid < nslots) {
    const uint32_t s = tid;
    RHdr hd;
    hd.gslot = L.s_gslot[s];
    hd.nu_total = L.s_nu[s];
    hd.nu_listed = hd.nu_total < D ? hd.nu_total : D;
    hd.n_o = (uint32_t)L.s_h[s];
    hd.floor = L.s_floor[s];
    hd.H = L.s_H[s]; hd.M = L.s_M[s];
    hd.first_ts = L.s_first[s]; hd.last_ts = L.s_last[s];
    hd.flags = L.s_flags[s];
    hd.pad = 0; hd.pad2 = 0;
    rhdr[sbase + s] = hd;
    const uint32_t no = hd.n_o < D ? hd.n_o : D;
    for (uint32_t k = 0; k < no; k++) {
      OItem *o = &ro[(sbase + s) * D + k];
      o->ts = L.k_ts[(size_t)s * D + k];
      o->child = L.k_child[(size_t)s * D + k];
      o->bytes = FMT == 2 ? L.k_bytes[(size_t)s * D + k] : 0;
      o->fn = L.k_fn[(size_t)s * D + k];
      o->pad = 0;
    }
  }
  for (uint32_t i = tid; i < E; i += WG) {
    const uint32_t key = L.t_key[i];
    if (key == EMPTY32) continue;
    const uint32_t s = key >> 16, fn = key & 0xFFFFu;
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
    const uint64_t w1 = __builtin_nontemporal_load((const uint64_t *)(sg.rec + (rg.begin + i) * 16) + 1);
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
hipError_t launch_range(int fmt, uint32_t T, const Seg *segs, const Range *ranges, uint32_t n_ranges,
                        const Tables &tb, const Shape &sh, RHdr *rhdr, UItem *ru, OItem *ro,
                        uint32_t *rnslots, hipStream_t st) {
  if (!n_ranges) return hipSuccess;
  dim3 grid(n_ranges), block(WG);
#define TT_LAUNCH(F, R)                                                                                   \
  do {                                                                                                    \
    hipError_t e = hipFuncSetAttribute((const void *)k_range<F, R>,                                     \
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh.lds_bytes);    \
    if (e != hipSuccess) return e;                                                                        \
    hipLaunchKernelGGL((k_range<F, R>), grid, block, sh.lds_bytes, st, segs, ranges, tb, sh, rhdr, ru, ro, \
                       rnslots);                                                                          \
    return hipGetLastError();                                                                             \
  } while (0)
  if (fmt == 1) {
    if (T == 1024) TT_LAUNCH(1, 4);
    if (T == 2048) TT_LAUNCH(1, 8);
  } else {
    if (T == 1024) TT_LAUNCH(2, 4);
    if (T == 2048) TT_LAUNCH(2, 8);
  }
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
