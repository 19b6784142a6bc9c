// tt_range.hip -- the fused per-range kernel of the tally pipeline.
//
// One workgroup of 1024 lanes owns one contiguous range of one stream's
// records and walks it tile by tile.  Per tile of T records it
//   1. decodes the records with coalesced 8-byte loads (FIXED24: 3 words per
//      record; VAR16: 2 header words plus, for entries of sized functions and
//      kernel records, the u64 at payload offset 0, located by an exclusive
//      prefix scan of payload_len across the tile); the next tile's loads are
//      in flight while the current tile is processed;
//   2. tallies device-kernel records (kind 2) straight into an LDS table;
//   3. maps each API record's thread id to a range-local slot through an LDS
//      hash (new threads are resolved to a global thread slot once per range);
//   4. sorts the tile's API records stably by slot with wavefront ballots
//      (the rank of a record among equal slots is a popcount of the ballot
//      match mask), so each thread's records become contiguous and stay in
//      record order;
//   5. hands each thread's records to one wavefront, 64 records per step
//      (a window).  Within a window everything is lane-parallel: the depth
//      after each record is the carried depth plus a popcount of entries
//      minus exits before it; an exit's entry is the last earlier lane whose
//      entry opened the same level (highest set bit of that level's entry
//      ballot below the lane), and its parent the last earlier entry one
//      level down; entries opened before the window are on the thread's
//      stack carried in LDS, indexed by level.  These are the stack
//      operations that define a call's interval (paper section 3.3) and its
//      tally (section 3.4, the table of section 4.3), done for 64 records at
//      once.  Children time reaches parents through one LDS atomic per call,
//      then self time and the tally follow, and the calls still open at the
//      window end become the carried stack.
// In the default (pipelined) schedule half of the wavefronts build sorted
// tiles (steps 1-4) into one half of the tile region while the other half
// walk the previous tile (step 5); a thread's windows run across tile
// boundaries.
// An exit that closes a call opened before the range is written to the range
// summary (U item) with the children time that call collected inside the
// range; the calls still open at the range end are written as O items.  The
// combine kernel folds the summaries of consecutive ranges onto the thread
// stacks carried on the device between ranges and flushes.
#include "tt_common.h"

namespace tt {

constexpr int RWG = 1024;           // lanes of the range kernel's workgroup
constexpr int RNW = RWG / WAVE;     // its wavefronts
constexpr uint32_t FK_EXIT = 1u << 16;  // tile_fk: [0,16) fn | 16 kind (0 entry, 1 exit)
constexpr int32_t BIG = 0x3FFFFFFF;

// LDS records are arrays of structs, so that one base address serves every
// field (the field offset goes into the instruction).
// A thread slot: depth relative to the range start, virtual closes (calls
// opened before the range that it closed), excursion, flags, global slot,
// children time of the call at the floor, first and last timestamps.
struct SRec {
  int32_t d, u, H, M;
  uint32_t flags, gslot;
  uint64_t facc, first, last;
};
// A carried frame: an entry still open, by level above the floor.
struct CFrame1 { uint64_t ts, ch; uint32_t fn, pad; };
struct CFrame2 { uint64_t ts, ch, by; uint32_t fn, pad; };
template <int FMT> struct CFrameOf { typedef CFrame1 T; };
template <> struct CFrameOf<2> { typedef CFrame2 T; };
// An LDS tally entry: key (hashed region), count, 32-bit min/max, u64 sums.
struct TEnt1 { uint32_t key, cnt, imin, imax, smin, smax; uint64_t isum, ssum; };
struct TEnt2 { uint32_t key, cnt, imin, imax, smin, smax; uint64_t isum, ssum, bsum; };
template <int FMT> struct TEntOf { typedef TEnt1 T; };
template <> struct TEntOf<2> { typedef TEnt2 T; };

struct RangeLds {
  uint64_t *tile_ts;   // tile sorted by slot: timestamp
  uint64_t *tile_by;   // VAR16 transfer size of entries
  uint32_t *tile_fk;   // fn | kind << 16
  SRec *srec;          // [S_MAX] thread slots
  void *cfr;           // [slot][D] carried frames (CFrame1 / CFrame2)
  // per-wave scratch: children time of the window's lanes, of virtual levels
  uint64_t *w_ch, *w_vt;
  void *tal;           // [E] tally entries (TEnt1 / TEnt2)
  // kernel tally
  uint32_t *q_cnt, *q_min, *q_max;
  uint64_t *q_sum;
  // thread map and sort
  uint64_t *tidmap;
  uint32_t *wcnt, *soff;
  uint32_t *newtid, *newbucket;
  uint32_t *misc;   // [0] nslots, [1] new ids, [2] nd, [3] builder barrier, [5] tiles built x producer waves,
                    // [7..8] nslots per half, [9] threads left to extra passes, [10] LDS tally has
                    // filled up, [11] ordinals of the partial tally, [16..] tiles walked per walking wave
  uint32_t *cnt;    // [ST_N] range-local counters
  uint32_t nd;      // slots of the direct-mapped tally region, chosen per range at its first tile
  uint32_t *wsum;   // [RNW] per-wave payload sums
};

__host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Byte layout of the dynamic LDS; the same function sizes it on the host.
template <bool CARVE>
__host__ __device__ inline size_t range_lds_layout(uint8_t *base, RangeLds *L, uint32_t T, uint32_t E, uint32_t KL,
                                                   uint32_t D, int fmt) {
  size_t o = 0;
  auto take = [&](size_t bytes) -> uint8_t * {
    o = align_up(o, 16);
    uint8_t *p = CARVE ? base + o : nullptr;
    o += bytes;
    return p;
  };
  const size_t SC = slot_cap(D);
  uint8_t *p;
#define TAKE(field, type, count) p = take(sizeof(type) * (size_t)(count)); if (CARVE) L->field = (type *)p
  TAKE(tile_ts, uint64_t, T);
  TAKE(tile_by, uint64_t, fmt == 2 ? T : 0);
  TAKE(tile_fk, uint32_t, T);
  TAKE(srec, SRec, S_MAX);
  TAKE(cfr, uint8_t, SC * D * (fmt == 2 ? sizeof(CFrame2) : sizeof(CFrame1)));
  TAKE(w_ch, uint64_t, (size_t)RNW * WAVE);
  TAKE(w_vt, uint64_t, (size_t)RNW * (D + 1));
  TAKE(tal, uint8_t, E * (fmt == 2 ? sizeof(TEnt2) : sizeof(TEnt1)));
  TAKE(q_cnt, uint32_t, KL);
  TAKE(q_min, uint32_t, KL);
  TAKE(q_max, uint32_t, KL);
  TAKE(q_sum, uint64_t, KL);
  TAKE(tidmap, uint64_t, TIDMAP);
  TAKE(wcnt, uint32_t, RNW * S_MAX);
  TAKE(soff, uint32_t, 2 * (S_MAX + 1));
  TAKE(newtid, uint32_t, TIDMAP);
  TAKE(newbucket, uint32_t, TIDMAP);
  TAKE(misc, uint32_t, 32);
  TAKE(cnt, uint32_t, ST_N);
  TAKE(wsum, uint32_t, RNW);
#undef TAKE
  return align_up(o, 16);
}

size_t range_lds_bytes(uint32_t T, uint32_t E, uint32_t KL, uint32_t D, int fmt) {
  return range_lds_layout<false>(nullptr, nullptr, T, E, KL, D, fmt);
}

// ---------------------------------------------------------------- helpers
// First bucket of a thread id in the range's tid map: multiplicative
// (Fibonacci) hashing, the top bits of t * 2^32/phi; one multiply, and ids
// that differ by a constant stride spread over the table.
constexpr uint32_t TIDMAP_BITS = 8;
static_assert(TIDMAP == 1 << TIDMAP_BITS, "tid map size");
__device__ __forceinline__ uint32_t tid_bucket(uint32_t t) { return (t * 0x9E3779B1u) >> (32 - TIDMAP_BITS); }
// A set of at most S_MAX global thread slots in TIDMAP u32 words of LDS
// (open addressing, EMPTY32 = free): the threads an extra pass skips.
__device__ inline bool in_gset(const uint32_t *set, uint32_t g) {
  uint32_t h = tid_bucket(g);
  for (uint32_t probe = 0; probe < TIDMAP; probe++) {
    const uint32_t v = set[h];
    if (v == g) return true;
    if (v == EMPTY32) return false;
    h = (h + 1) & (TIDMAP - 1);
  }
  return false;
}
// Lanes of the wavefront for which p holds (p stays a lane mask; HIP's
// __ballot takes an int and round-trips the predicate through a register).
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ inline uint64_t lanemask_lt() {
  const uint32_t lane = __lane_id();
  return lane ? (~0ull >> (64 - lane)) : 0ull;
}
// Inclusive prefix sum over the 64 lanes with DPP row shifts and row
// broadcasts (gfx9 encodings: row_shr:k = 0x110 + k, row_bcast:15 = 0x142,
// row_bcast:31 = 0x143; lanes without a source add 0).
__device__ inline uint32_t wave_incl_scan(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)v, 0x111, 0xF, 0xF, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)v, 0x112, 0xF, 0xF, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)v, 0x114, 0xF, 0xF, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)v, 0x118, 0xF, 0xF, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)v, 0x142, 0xA, 0xF, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)v, 0x143, 0xC, 0xF, false);
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
typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) u64x2 gu64x2;

__device__ inline uint64_t load_u64_unaligned(const uint8_t *base, uint64_t off) {
  const uintptr_t a = (uintptr_t)(base + off);
  gu64 *p = (gu64 *)(a & ~(uintptr_t)7);
  const uint32_t sh = (uint32_t)(a & 7) * 8;
  const uint64_t lo = __builtin_nontemporal_load(p);
  if (sh == 0) return lo;
  const uint64_t hi = __builtin_nontemporal_load(p + 1);
  return (lo >> sh) | (hi << (64 - sh));
}

// LDS tally layout: the first nd * n_fns entries are indexed directly by
// slot * n_fns + fn (no probing); the rest is an open-addressing hash keyed
// (slot << 16 | fn) for slots beyond that.  nd is direct_slots(n_fns, E), or
// 0 for a range whose first tile already has more threads than that.
__host__ __device__ inline uint32_t direct_slots(uint32_t n_fns, uint32_t E) {
  const uint32_t d = n_fns <= E ? E / n_fns : 0;
  return d < (uint32_t)S_MAX ? d : (uint32_t)S_MAX;
}

// Positions of the LDS tally hash a key may take (linear probing) before its
// call falls back to the global tally; once some key of the range has found
// none, later calls probe only the first TALLY_PROBES_FULL of them (each
// probe is a dependent LDS round trip, and in a table that has filled up the
// keys that probe far are mostly not in it).
constexpr uint32_t TALLY_PROBES = 8;
constexpr uint32_t TALLY_PROBES_FULL = 2;

// Adds one completed call to the (slot, fn) entry of the LDS tally.
// Durations that do not
// fit 32 bits update the global min/max directly; a key that finds no room
// goes to the global tally with atomics.
template <int FMT>
__device__ inline void tally_call(const RangeLds &L, uint32_t E, const Tables &tb, uint32_t slot, uint32_t gslot,
                                  uint32_t fn, uint64_t incl, uint64_t self, uint64_t bytes) {
  if (fn >= tb.n_fns || slot >= (uint32_t)S_MAX) return;
  typedef typename TEntOf<FMT>::T TE;
  TE *const tal = (TE *)L.tal;
  const uint32_t nd = L.nd;
  uint32_t h = 0;
  bool found = false;
  if (slot < nd) {
    h = slot * tb.n_fns + fn;
    found = true;
  } else {
    const uint32_t d0 = nd * tb.n_fns;
    if (E > d0) {
      // a key's positions [p, p + reach) never wrap: the first comes from a
      // multiplicative hash mapped by a multiply-shift onto the span - reach
      // + 1 starts (so the span need not be a power of two); a key sits
      // before the first free position of its sequence, since entries are
      // never freed
      const uint32_t key = (slot << 16) | fn;
      const uint32_t span = E - d0;
      const uint32_t reach = span < TALLY_PROBES ? span : TALLY_PROBES;
      const uint32_t full = __hip_atomic_load(&L.misc[10], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      uint32_t p = d0 + (uint32_t)(((uint64_t)(key * 0x9E3779B1u) * (span - reach + 1)) >> 32);
      const uint32_t probes = full && reach > TALLY_PROBES_FULL ? TALLY_PROBES_FULL : reach;
      for (uint32_t i = 0; i < probes; i++, p++) {
        const uint32_t k = tal[p].key;
        if (k == key) { found = true; break; }
        if (k == EMPTY32) {
          const uint32_t old = atomicCAS(&tal[p].key, EMPTY32, key);
          if (old == EMPTY32 || old == key) { found = true; break; }
        }
      }
      if (found) h = p;
      else if (!full)   // no room among the key's positions: the table has filled up
        __hip_atomic_store(&L.misc[10], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
  }
  if (found) {
    lds_add32(&tal[h].cnt, 1u);
    lds_add64(&tal[h].isum, incl);
    lds_add64(&tal[h].ssum, self);
    if constexpr (FMT == 2) { if (bytes) lds_add64(&tal[h].bsum, bytes); }
    if (incl < EMPTY32) { lds_min32(&tal[h].imin, (uint32_t)incl); lds_max32(&tal[h].imax, (uint32_t)incl); }
    if (self < EMPTY32) { lds_min32(&tal[h].smin, (uint32_t)self); lds_max32(&tal[h].smax, (uint32_t)self); }
  }
  if ((!found || incl >= EMPTY32 || self >= EMPTY32) && gslot < tb.max_threads) {
    Tally *g = &tb.tally[(size_t)gslot * tb.n_fns + fn];
    if (!found) {
      g_add64(&g->count, 1);
      g_add64(&g->incl_sum, incl);
      g_add64(&g->self_sum, self);
      if (bytes) g_add64(&g->bytes_sum, bytes);
    }
    if (!found || incl >= EMPTY32) { g_min64(&g->incl_min, incl); g_max64(&g->incl_max, incl); }
    if (!found || self >= EMPTY32) { g_min64(&g->self_min, self); g_max64(&g->self_max, self); }
  }
}

// Orders this wavefront's LDS accesses around it (all lanes take part).
__device__ inline void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// ------------------------------------------------------------------ window

// DPP lane moves (gfx9 encodings): row_shr:k = 0x110 + k, wave_shr:1 = 0x138,
// row_bcast:15 = 0x142, row_bcast:31 = 0x143.  Lanes whose source is out of
// range, or whose row is masked off, keep `old`.
template <int CTRL, int ROWM = 0xF>
__device__ __forceinline__ int32_t dpp(int32_t old, int32_t v) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWM, 0xF, false);
}
__device__ __forceinline__ int32_t imin(int32_t a, int32_t b) { return a < b ? a : b; }
__device__ __forceinline__ int32_t imax(int32_t a, int32_t b) { return a > b ? a : b; }
// Inclusive prefix minimum / maximum over the 64 lanes (row scans, then the
// row ends broadcast to the rows above).  Lanes without a source see the
// operation's identity, so each step can be a single DPP min / max.
constexpr int32_t I32_MAX = 0x7FFFFFFF, I32_MIN = -0x7FFFFFFF - 1;
__device__ __forceinline__ int32_t wave_scan_min(int32_t v) {
  v = imin(v, dpp<0x111>(I32_MAX, v));
  v = imin(v, dpp<0x112>(I32_MAX, v));
  v = imin(v, dpp<0x114>(I32_MAX, v));
  v = imin(v, dpp<0x118>(I32_MAX, v));
  v = imin(v, dpp<0x142, 0xA>(I32_MAX, v));
  v = imin(v, dpp<0x143, 0xC>(I32_MAX, v));
  return v;
}
__device__ __forceinline__ int32_t wave_scan_max(int32_t v) {
  v = imax(v, dpp<0x111>(I32_MIN, v));
  v = imax(v, dpp<0x112>(I32_MIN, v));
  v = imax(v, dpp<0x114>(I32_MIN, v));
  v = imax(v, dpp<0x118>(I32_MIN, v));
  v = imax(v, dpp<0x142, 0xA>(I32_MIN, v));
  v = imax(v, dpp<0x143, 0xC>(I32_MIN, v));
  return v;
}
// Both scans at once, step by step (two independent chains).
__device__ __forceinline__ void wave_scan_minmax(int32_t &mn, int32_t &mx) {
  mn = imin(mn, dpp<0x111>(I32_MAX, mn)); mx = imax(mx, dpp<0x111>(I32_MIN, mx));
  mn = imin(mn, dpp<0x112>(I32_MAX, mn)); mx = imax(mx, dpp<0x112>(I32_MIN, mx));
  mn = imin(mn, dpp<0x114>(I32_MAX, mn)); mx = imax(mx, dpp<0x114>(I32_MIN, mx));
  mn = imin(mn, dpp<0x118>(I32_MAX, mn)); mx = imax(mx, dpp<0x118>(I32_MIN, mx));
  mn = imin(mn, dpp<0x142, 0xA>(I32_MAX, mn)); mx = imax(mx, dpp<0x142, 0xA>(I32_MIN, mx));
  mn = imin(mn, dpp<0x143, 0xC>(I32_MAX, mn)); mx = imax(mx, dpp<0x143, 0xC>(I32_MIN, mx));
}
// v_writelane: lane `lane` of the result is v (uniform), the others keep old.
__device__ int32_t amd_writelane(int32_t v, int32_t lane, int32_t old) __asm("llvm.amdgcn.writelane.i32");
__device__ __forceinline__ int32_t lane63(int32_t v) { return __builtin_amdgcn_readlane(v, 63); }
__device__ __forceinline__ uint64_t bperm64(uint32_t lo, uint32_t hi, int32_t src) {
  const uint32_t l = (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int32_t)lo);
  const uint32_t h = (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int32_t)hi);
  return ((uint64_t)h << 32) | l;
}
__device__ __forceinline__ int32_t msb64(uint64_t m) { return m ? 63 - (int32_t)__clzll(m) : -1; }
__device__ __forceinline__ uint64_t uread64(uint64_t v, uint32_t lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)v, (int32_t)lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)(v >> 32), (int32_t)lane);
  return ((uint64_t)hi << 32) | lo;
}

// State of one thread slot while a wavefront walks its records; lives in
// registers across the windows of one tile and in LDS between tiles.
struct SlotState {
  int32_t d;        // depth relative to the range start
  int32_t fl;       // floor: lowest depth reached (<= 0); -fl calls opened before the range were closed
  int32_t H, M;     // excursion: a value above max_depth iff the height above the floor ever was; max level
  uint32_t flags;   // RF_*
  uint64_t facc;    // children time of the call at the floor (opened before the range)
  uint64_t first, last;
};

// One window: records [a, a + nw) of slot s (nw <= 64), one per lane of the
// calling wavefront (all 64 lanes call).  Every exit finds its entry as the
// last earlier entry that opened the same level in the window, else on the
// carried stack (level above the floor), else it closes a call opened before
// the range (level at or below the floor); its parent is found the same way
// one level down.
// The lane's record (ts, fk, by) was loaded by the caller ahead of time; the
// records of one window may come from two consecutive tiles.
// wvt[0] holds the children time of the call at the floor across windows.
template <int FMT, bool IV>
__device__ __forceinline__ void slot_window(RangeLds &L, const Tables &tb, const uint32_t E, const uint32_t D,
                                            const uint32_t s, const uint32_t gslot,
                                            const uint32_t nw, const uint64_t ts, const uint32_t fk,
                                            const uint64_t by, SlotState &S, UItem *__restrict__ us,
                                            uint64_t *__restrict__ wch, uint64_t *__restrict__ wvt,
                                            IvRec *__restrict__ ivr) {
  const uint32_t lane = __lane_id();
  const bool valid = lane < nw;
  const uint32_t fn = fk & 0xFFFFu;
  const bool ex = valid && (fk & FK_EXIT);
  const bool en = valid && !(fk & FK_EXIT);
  const int32_t d0 = S.d, fl0 = S.fl, u0 = -fl0;
  // timestamp order within the thread (lane 0 compares with the previous window)
  {
    const uint32_t plo = (uint32_t)dpp<0x138>((int32_t)(uint32_t)S.last, (int32_t)(uint32_t)ts);
    const uint32_t phi = (uint32_t)dpp<0x138>((int32_t)(uint32_t)(S.last >> 32), (int32_t)(uint32_t)(ts >> 32));
    const uint64_t prev = ((uint64_t)phi << 32) | plo;
    const uint64_t bad = ballot(valid && (lane > 0 || (S.flags & RF_HAS_TS)) && ts < prev);
    if (bad && lane == 0) lds_add32(&L.cnt[ST_TSREG], (uint32_t)__popcll(bad));
    if (!(S.flags & RF_HAS_TS)) S.first = uread64(ts, 0);
    S.last = uread64(ts, nw - 1);
    S.flags |= RF_HAS_TS;
  }
  // depth after each record and the level each record opens (entry) or closes (exit)
  const uint64_t Em = ballot(en), Xm = ballot(ex);
  const uint64_t lt = lanemask_lt();
  const int32_t da = d0 + (int32_t)__popcll(Em & lt) - (int32_t)__popcll(Xm & lt) + (en ? 1 : 0) - (ex ? 1 : 0);
  const int32_t lev = en ? da : da + 1;
  const int32_t d_end = d0 + (int32_t)__popcll(Em) - (int32_t)__popcll(Xm);
  int32_t pmin = valid ? da : BIG, pmax = valid ? da : -BIG;
  wave_scan_minmax(pmin, pmax);
  const int32_t damin = imin(lane63(pmin), d0);     // lowest depth in the window
  const int32_t dmax = imax(lane63(pmax), d0);
  const int32_t fl1 = imin(damin, fl0);             // floor after the window
  {
    const int32_t hub = dmax - fl1;                 // bounds the height above the floor in the window
    if (hub <= (int32_t)D) {
      S.H = imax(S.H, hub);
    } else {
      const int32_t h = lane63(wave_scan_max(en ? lev - imin(fl0, pmin) : -BIG));
      S.H = imax(S.H, h);
    }
    S.M = imax(S.M, dmax);
  }
  // entries by level: lane k of (tlo, thi) holds the ballot of entries opening level damin + 1 + k
  int32_t tlo = 0, thi = 0;
  const int32_t vend = imin(dmax, damin + WAVE);    // (the levels of 64 records span at most 64)
  {
    const int32_t levE = en ? lev : -BIG;           // entries only
    for (int32_t v = damin + 1, j = 0; v <= vend; v++, j++) {
      const uint64_t Ev = ballot(levE == v);
      tlo = amd_writelane((int32_t)(uint32_t)Ev, j, tlo);
      thi = amd_writelane((int32_t)(uint32_t)(Ev >> 32), j, thi);
    }
  }
  const int32_t k = valid ? lev - damin - 1 : 0;
  const uint64_t Elev = bperm64(tlo, thi, k);
  const uint64_t Epar = bperm64(tlo, thi, k > 0 ? k - 1 : 0);
  const int32_t partner = ex ? msb64(Elev & lt) : -1;
  const int32_t parent = (ex && k > 0) ? msb64(Epar & lt) : -1;
  const bool open_at_end = en && lev <= d_end && msb64(Elev) == (int32_t)lane;
  wch[lane] = 0;
  if (lane >= 1 && lane <= D) wvt[lane] = 0;
  // the entry each exit closes: in the window (inw), on the carried stack
  // (car), or opened before the range (pre); an exit whose carried position
  // lies beyond the stack capacity closes nothing here (the range is already
  // flagged as overflowing).  Both candidate entries are read by every lane.
  const bool inw = ex && partner >= 0;
  const uint32_t cpos = (uint32_t)(lev - fl0 - 1);
  const bool car = ex && partner < 0 && lev > fl0 && cpos < D;
  const bool pre = ex && partner < 0 && lev <= fl0;
  // the partner lane holds the entry's record (every lane takes part in the
  // permutes: a permute reads 0 from a lane that does not)
  const int32_t psrc = partner >= 0 ? partner : 0;
  const uint32_t ci = s * D + (car ? cpos : 0u);
  typedef typename CFrameOf<FMT>::T CF;
  CF *const cfr = (CF *)L.cfr;
  const uint64_t wts = bperm64((uint32_t)ts, (uint32_t)(ts >> 32), psrc), cts = cfr[ci].ts;
  const uint32_t wfn = (uint32_t)__builtin_amdgcn_ds_bpermute(psrc << 2, (int32_t)fk) & 0xFFFFu, cfn = cfr[ci].fn;
  const uint64_t wby = FMT == 2 ? bperm64((uint32_t)by, (uint32_t)(by >> 32), psrc) : 0;
  const uint64_t pts = inw ? wts : cts;
  const uint32_t pfn = inw ? wfn : cfn;
  uint64_t pby = 0;
  if constexpr (FMT == 2) pby = inw ? wby : cfr[ci].by;
  const bool matched = inw || car;
  const bool mis = matched && pfn != fn;
  const bool neg = matched && pfn == fn && ts < pts;
  const bool ok = matched && pfn == fn && ts >= pts;
  const uint64_t incl = ok ? ts - pts : 0;
  if (ballot(mis || neg)) {
    const uint64_t mm = ballot(mis), nm = ballot(neg);
    if (lane == 0) {
      if (mm) lds_add32(&L.cnt[ST_MISMATCH], (uint32_t)__popcll(mm));
      if (nm) lds_add32(&L.cnt[ST_NEGDUR], (uint32_t)__popcll(nm));
    }
  }
  wave_lds_fence();
  // children time to the parent: in the window, on the carried stack, or the
  // accumulator of a level below the floor
  {
    const int32_t pl = lev - 1;
    const uint32_t pp = (uint32_t)(pl - fl0 - 1), vk = (uint32_t)(fl0 - pl);
    const bool to_w = parent >= 0;
    const bool to_c = !to_w && pl > fl0 && pp < D;
    const bool to_v = !to_w && pl <= fl0 && (vk == 0 || (vk <= D && (uint32_t)u0 + vk < D));
    // (byte offsets from the window-lane array, chosen by selects)
    const int32_t o_w = (parent >= 0 ? parent : 0) * 8;
    const int32_t o_c = (int32_t)((uint8_t *)&cfr[s * D + (to_c ? pp : 0u)].ch - (uint8_t *)wch);
    const int32_t o_v = (int32_t)((uint8_t *)&wvt[to_v ? vk : 0u] - (uint8_t *)wch);
    int32_t off = to_c ? o_c : o_v;
    off = to_w ? o_w : off;
    if (ok && (to_w || to_c || to_v)) lds_add64((uint64_t *)((uint8_t *)wch + off), incl);
  }
  wave_lds_fence();
  // self time and tally of every call closed here
  {
    const uint64_t wc = wch[partner >= 0 ? partner : 0], cc = cfr[ci].ch;
    const uint64_t ch = inw ? wc : cc;
    const bool under = ok && ch > incl;
    const uint64_t self = (ok && !under) ? incl - ch : 0;
    const uint64_t um = ballot(under);
    if (um && lane == 0) lds_add32(&L.cnt[ST_UNDER], (uint32_t)__popcll(um));
    const bool tally = ok && fn < tb.n_fns;
    if (s < L.nd) {
      // direct-mapped rows of this slot; 32-bit min/max take no-op operands
      // for durations of 2^32 ns or more, which go to the global row instead
      typedef typename TEntOf<FMT>::T TE;
      TE *const te = (TE *)L.tal + s * tb.n_fns + (tally ? fn : 0u);
      if (tally) {
        lds_add32(&te->cnt, 1u);
        lds_add64(&te->isum, incl);
        lds_add64(&te->ssum, self);
        if constexpr (FMT == 2) lds_add64(&te->bsum, pby);
        const bool ib = incl >= EMPTY32, sb = self >= EMPTY32;
        lds_min32(&te->imin, ib ? EMPTY32 : (uint32_t)incl);
        lds_max32(&te->imax, ib ? 0u : (uint32_t)incl);
        lds_min32(&te->smin, sb ? EMPTY32 : (uint32_t)self);
        lds_max32(&te->smax, sb ? 0u : (uint32_t)self);
      }
      const bool big = tally && (incl >= EMPTY32 || self >= EMPTY32) && gslot < tb.max_threads;
      if (ballot(big)) {
        if (big) {
          Tally *g = &tb.tally[(size_t)gslot * tb.n_fns + fn];
          if (incl >= EMPTY32) { g_min64(&g->incl_min, incl); g_max64(&g->incl_max, incl); }
          if (self >= EMPTY32) { g_min64(&g->self_min, self); g_max64(&g->self_max, self); }
        }
      }
    } else if (tally) {
      tally_call<FMT>(L, E, tb, s, gslot, fn, incl, self, pby);
    }
  }
  // intervals: every call tallied here, with its parent when that is in the
  // window or on the carried stack; depth and a parent opened before the
  // range are left relative to the floor at the call's entry (the lowest
  // depth before this exit: no depth below the call's level occurs while it
  // is open, so the floor is the same at its entry)
  if constexpr (IV) {
    const bool emit = ok && fn < tb.n_fns;
    const uint64_t em = ballot(emit);
    const int32_t psrc2 = parent >= 0 ? parent : 0;
    const uint64_t pts_w = bperm64((uint32_t)ts, (uint32_t)(ts >> 32), psrc2);
    const uint32_t pfn_w = (uint32_t)__builtin_amdgcn_ds_bpermute(psrc2 << 2, (int32_t)fk) & 0xFFFFu;
    const int32_t f = imin(fl0, dpp<0x138>(BIG, pmin));
    if (em) {
      const int32_t pl = lev - 1;
      const uint32_t pp = (uint32_t)(pl - fl0 - 1);
      const bool p_w = parent >= 0;
      const bool p_c = !p_w && pl > fl0 && pp < D;
      const uint32_t pci = s * D + (p_c ? pp : 0u);
      const uint64_t pcts = cfr[pci].ts;
      const uint32_t pcfn = cfr[pci].fn;
      uint32_t base = 0;
      if (lane == 0)
        base = __hip_atomic_fetch_add(&L.misc[6], (uint32_t)__popcll(em), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_WORKGROUP);
      base = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)base);
      if (emit) {
        const uint32_t dl = (uint32_t)imin(lev - f, 255), fneg = (uint32_t)imin(-f, 255);
        const uint64_t pst = p_w ? pts_w : (p_c ? pcts : 0ull);
        const uint32_t pfn = p_w ? pfn_w : (p_c ? pcfn : 0u);
        const uint64_t w3 = (uint64_t)fn | ((uint64_t)(pfn & 0xFFFFu) << 16) | ((uint64_t)s << 32) |
                            ((uint64_t)dl << 40) | ((uint64_t)fneg << 48) |
                            ((uint64_t)((p_w || p_c) ? IV_PARENT_SET : 0u) << 56);
        gu64x2 *d = (gu64x2 *)(ivr + base + (uint32_t)__popcll(em & lt));
        __builtin_nontemporal_store(u64x2{pts, ts}, d);
        __builtin_nontemporal_store(u64x2{pst, w3}, d + 1);
      }
    }
  }
  // exits that close calls opened before the range become U items
  if (ballot(pre)) {
    if (pre) {
      const uint32_t vk = (uint32_t)(fl0 - lev);
      const uint32_t gi = (uint32_t)u0 + vk;
      if (gi < D) {
        UItem *u = &us[gi];
        u->ts = ts; u->child = wvt[vk]; u->fn = fn; u->pad = 0; u->pad2 = 0;
      } else {
        lds_add32(&L.cnt[ST_ORPHAN], 1u);  // deeper than any stack can be: certainly an orphan exit
      }
    }
  }
  wave_lds_fence();
  // calls still open at the window end become the carried stack
  if (open_at_end) {
    const uint32_t pos = (uint32_t)(lev - fl1 - 1);
    if (pos < D) {
      const uint32_t i = s * D + pos;
      cfr[i].ts = ts; cfr[i].ch = wch[lane]; cfr[i].fn = fn;
      if constexpr (FMT == 2) cfr[i].by = by;
    }
  }
  if (ballot(open_at_end && (uint32_t)(lev - fl1 - 1) >= D)) S.flags |= RF_OVERFLOW;
  if (fl1 < fl0 && lane == 0) {
    // the floor moved down: its call's children time is that of the level reached
    const uint32_t dv = (uint32_t)(fl0 - fl1);
    wvt[0] = (dv <= D && (uint32_t)u0 + dv < D) ? wvt[dv] : 0;
  }
  S.d = d_end;
  S.fl = fl1;
  wave_lds_fence();
}

// ------------------------------------------------------------------ sync
// Bounded waits between the wave groups of one workgroup (all resident on one
// CU).  A wait that runs out raises ERR_PIPE and returns, so every wave always
// reaches the end of the kernel; the host then reports a device error.
constexpr uint32_t SPIN_LIMIT = 1u << 22;

__device__ inline void wait_at_least(uint32_t *ctr, uint32_t v, uint32_t *err) {
  if (__lane_id() == 0) {
    uint32_t i = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < v) {
      __builtin_amdgcn_s_sleep(2);
      if (++i == SPIN_LIMIT) { atomicOr(err, ERR_PIPE); break; }
    }
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Waits until ctr[k] >= v for every k < n (n <= 64): lane k polls ctr[k].
__device__ inline void wait_all_at_least(uint32_t *ctr, uint32_t n, uint32_t v, uint32_t *err) {
  const uint32_t lane = __lane_id();
  uint32_t i = 0;
  while (ballot(lane < n && __hip_atomic_load(&ctr[lane < n ? lane : 0], __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_WORKGROUP) < v)) {
    __builtin_amdgcn_s_sleep(1);
    if (++i == SPIN_LIMIT) { if (lane == 0) atomicOr(err, ERR_PIPE); break; }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Barrier of `nw` waves: the counter only grows, by nw per episode.
__device__ inline void group_barrier(uint32_t *ctr, uint32_t nw, uint32_t *err) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  if (__lane_id() == 0) {
    const uint32_t old = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
    const uint32_t target = (old / nw + 1) * nw;
    uint32_t i = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++i == SPIN_LIMIT) { atomicOr(err, ERR_PIPE); break; }
    }
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Makes this group's LDS writes visible, then (one lane) sets *ctr = v.
__device__ inline void publish(uint32_t *ctr, uint32_t v, bool me) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  if (me) __hip_atomic_store(ctr, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// A walking wave keeps the state of the slot it walks in registers (and its
// floor accumulator in wvt[0]) from one tile to the next while it walks that
// slot only; it goes back to LDS when the wave turns to another slot and at
// the range end.  With two alternating tile halves, the slot's last records of
// a tile that do not fill a window wait for the next tile in registers (one
// record per lane), so that windows run across tile boundaries instead of
// ending ragged.
struct WalkCache {
  uint32_t slot;      // EMPTY32: nothing cached
  uint32_t gslot;
  SlotState S;
  uint32_t pend;      // deferred records of the slot (< WAVE), lane i holds the i-th
  uint64_t dts, dby;
  uint32_t dfk;
};

__device__ __forceinline__ void slot_load(const RangeLds &L, const uint32_t s, WalkCache &c, uint64_t *wvt) {
  c.slot = s;
  c.pend = 0;
  const SRec &r = L.srec[s];
  c.S.d = __builtin_amdgcn_readfirstlane(r.d);
  c.S.fl = -__builtin_amdgcn_readfirstlane(r.u);
  c.S.H = __builtin_amdgcn_readfirstlane(r.H);
  c.S.M = __builtin_amdgcn_readfirstlane(r.M);
  c.S.flags = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)r.flags);
  c.S.facc = 0;  // (lives in wvt[0])
  c.S.first = uread64(r.first, 0);
  c.S.last = uread64(r.last, 0);
  c.gslot = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)r.gslot);
  if (__lane_id() == 0) wvt[0] = r.facc;
  wave_lds_fence();
}

// (the deferred records must have been walked)
__device__ __forceinline__ void slot_store(RangeLds &L, WalkCache &c, const uint64_t *wvt) {
  if (c.slot == EMPTY32) return;
  const uint32_t s = c.slot;
  if (__lane_id() == 0) {
    SRec &r = L.srec[s];
    r.d = c.S.d; r.u = -c.S.fl; r.H = c.S.H; r.M = c.S.M; r.flags = c.S.flags;
    r.facc = wvt[0]; r.first = c.S.first; r.last = c.S.last;
  }
  c.slot = EMPTY32;
  wave_lds_fence();
}

// Walks the cached slot's deferred records followed by records [b, e) of the
// tile region, in windows of WAVE records.  With `defer`, a last partial
// window that lies within [b, e) is kept for the next tile instead; with HOLD
// as well, fewer than a window of records all wait (the new ones join the
// waiting ones in registers).
template <int FMT, bool IV, bool HOLD = false>
__device__ __forceinline__ void slot_walk(RangeLds &L, const Tables &tb, const uint32_t E, const uint32_t D,
                                          WalkCache &c, const uint32_t b, const uint32_t e, const bool defer,
                                          const size_t sbase, UItem *__restrict__ ru, uint64_t *__restrict__ wch,
                                          uint64_t *__restrict__ wvt, IvRec *__restrict__ ivr) {
  const uint32_t s = c.slot;
  UItem *us = ru + (sbase + s) * D;
  const uint32_t lane = __lane_id();
  const uint32_t pend = c.pend;
  const uint32_t ntot = pend + (e - b);
  if (HOLD && defer && ntot < WAVE) {
    // fewer than a window: the new records join the waiting ones in registers
    if (lane >= pend && lane < ntot) {
      const uint32_t p = b + (lane - pend);
      c.dts = L.tile_ts[p];
      c.dfk = L.tile_fk[p];
      c.dby = FMT == 2 ? L.tile_by[p] : 0;
    }
    c.pend = ntot;
    return;
  }
  uint32_t nwalk = ntot;
  if (defer) {
    const uint32_t r = ntot & (WAVE - 1);
    if (r && ntot - r >= pend) nwalk = ntot - r;   // (the tail must lie within [b, e))
  }
  if (nwalk) {
    // the v-th record of the sequence (v >= pend) sits at b + v - pend; each
    // window's records are loaded one window ahead (the tile does not change
    // during the walk)
    const uint32_t last = e > b ? e - 1 : 0u;   // reads stay within [b, e) (index 0 when it is empty)
    const uint32_t v = lane < nwalk ? lane : 0u;
    uint32_t p = v < pend ? (b < last ? b : last) : b + (v - pend);
    uint64_t ts = L.tile_ts[p], by = FMT == 2 ? L.tile_by[p] : 0;
    uint32_t fk = L.tile_fk[p];
    if (lane < pend) { ts = c.dts; fk = c.dfk; by = c.dby; }
    for (uint32_t v0 = 0; v0 < nwalk; v0 += WAVE) {
      const uint32_t vn = v0 + WAVE;
      p = vn < nwalk ? b + (vn - pend) + (lane < nwalk - vn ? lane : 0u) : (b < last ? b : last);
      const uint64_t ts_n = L.tile_ts[p], by_n = FMT == 2 ? L.tile_by[p] : 0;
      const uint32_t fk_n = L.tile_fk[p];
      slot_window<FMT, IV>(L, tb, E, D, s, c.gslot, (nwalk - v0) < WAVE ? (nwalk - v0) : WAVE, ts, fk, by, c.S,
                           us, wch, wvt, ivr);
      ts = ts_n; fk = fk_n; by = by_n;
    }
  }
  // records [b + nwalk - pend, e) wait for the next tile
  c.pend = ntot - nwalk;
  if (c.pend) {
    const uint32_t p = b + (nwalk - pend) + (lane < c.pend ? lane : 0u);
    c.dts = L.tile_ts[p];
    c.dfk = L.tile_fk[p];
    c.dby = FMT == 2 ? L.tile_by[p] : 0;
  }
}

// Waiting records of the slots a non-pipelined walker wave owns (slots w +
// j * RNW, j < DEFER_SETS: every slot a range holds): the partial last window
// of each, one record per lane, kept in registers until the slot's next
// records arrive, so that windows run full across tiles for every slot.
constexpr uint32_t DEFER_SETS = S_MAX / RNW;
struct WalkDefer {
  uint32_t n[DEFER_SETS];
  uint64_t ts[DEFER_SETS], by[DEFER_SETS];
  uint32_t fk[DEFER_SETS];
};

// The walk of one sorted tile (the tile region's half hb): wavefront w walks
// the thread slots w, w + nww, ... (nww walking waves), each slot's records in
// order.  With `defer`, the last slot's partial last window may wait for the
// next tile (WalkCache); any other deferred records are walked here.  With
// `dw` (non-pipelined, nww = RNW), every slot's may wait, in dw.
template <int FMT, bool IV>
__device__ __forceinline__ void walk_tile(RangeLds &L, const Tables &tb, const uint32_t E, const uint32_t D,
                                          const uint32_t hb, const uint32_t half, const uint32_t nww,
                                          const bool defer, const size_t sbase, UItem *__restrict__ ru,
                                          WalkCache &c, IvRec *__restrict__ ivr, WalkDefer *dw = nullptr) {
  const uint32_t w = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));   // (wave-uniform)
  const uint32_t *soff = L.soff + hb * (S_MAX + 1);
  const uint32_t base = hb * half;
  L.nd = L.misc[2];
  const uint32_t nslots = L.misc[7 + hb];
  uint64_t *wch = L.w_ch + w * WAVE, *wvt = L.w_vt + w * (D + 1);
  if (dw) {
    // (the loop is unrolled over the sets, so that each set stays in registers)
#pragma unroll
    for (uint32_t j = 0; j < DEFER_SETS; j++) {
      const uint32_t s = w + j * RNW;
      if (s >= nslots) break;
      const uint32_t b = base + soff[s], e = base + soff[s + 1];
      if (b == e && !dw->n[j]) continue;
      if (c.slot != s) {
        slot_store(L, c, wvt);
        slot_load(L, s, c, wvt);
      }
      c.pend = dw->n[j];
      c.dts = dw->ts[j];
      c.dfk = dw->fk[j];
      c.dby = dw->by[j];
      slot_walk<FMT, IV, true>(L, tb, E, D, c, b, e, defer, sbase, ru, wch, wvt, ivr);
      dw->n[j] = c.pend;
      dw->ts[j] = c.dts;
      dw->fk[j] = c.dfk;
      dw->by[j] = c.dby;
      c.pend = 0;
    }
    return;
  }
  for (uint32_t s = w; s < nslots; s += nww) {
    const uint32_t b = base + soff[s], e = base + soff[s + 1];
    if (c.slot != s) {
      if (b == e) continue;
      if (c.pend) slot_walk<FMT, IV>(L, tb, E, D, c, b, b, false, sbase, ru, wch, wvt, ivr);
      slot_store(L, c, wvt);
      slot_load(L, s, c, wvt);
    }
    if (b == e && !c.pend) continue;
    slot_walk<FMT, IV>(L, tb, E, D, c, b, e, defer && s + nww >= nslots, sbase, ru, wch, wvt, ivr);
  }
}

// Walks what the cached slot still defers, then puts its state back to LDS.
template <int FMT, bool IV>
__device__ __forceinline__ void walk_finish(RangeLds &L, const Tables &tb, const uint32_t E, const uint32_t D,
                                            const size_t sbase, UItem *__restrict__ ru, WalkCache &c,
                                            IvRec *__restrict__ ivr) {
  const uint32_t w = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));
  uint64_t *wch = L.w_ch + w * WAVE, *wvt = L.w_vt + w * (D + 1);
  if (c.slot != EMPTY32 && c.pend) slot_walk<FMT, IV>(L, tb, E, D, c, 0, 0, false, sbase, ru, wch, wvt, ivr);
  slot_store(L, c, wvt);
}

// ------------------------------------------------------------------ tile
// Front half of one tile: decode `cur*`, prefetch the next tile into `nxt*`,
// kernel records (wave totals of entries, exits, kernel, bad and -- wave 0 --
// all records accumulate in wc), slot map and stable sort into half `hb` of
// the tile region
// (the whole region when PIPE is off).  With PIPE the producer group (the
// upper RNW / 2 waves) runs it alone and synchronises through group barriers;
// otherwise the whole workgroup runs it between workgroup barriers.
template <int FMT, int ROWS, bool PIPE, bool XP>
__device__ __forceinline__ void front_tile(RangeLds &L, const Tables &tb, const uint32_t E, const uint32_t KL,
                                           const uint32_t D, const Range &rg, const Seg &sg, gu64 *grec,
                                           const uint64_t last_rec, const uint64_t t0, const uint32_t hb,
                                           const uint64_t (&cur0)[ROWS], const uint64_t (&cur1)[ROWS],
                                           const uint64_t (&cur2)[ROWS], uint64_t (&nxt0)[ROWS],
                                           uint64_t (&nxt1)[ROWS], uint64_t (&nxt2)[ROWS], uint64_t &pay_run,
                                           uint32_t (&wc)[5]) {
  constexpr uint32_t GW = PIPE ? RNW / 2 : RNW;     // waves of the group
  constexpr uint32_t T = ROWS * GW * WAVE;          // records per tile
  constexpr uint32_t RS = FMT == 2 ? 16 : 24;
  const int lane = threadIdx.x & (WAVE - 1);
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) - (PIPE ? (int)(RNW / 2) : 0);   // wave within the group
  const int tid = w * WAVE + lane;                                       // lane within the group
  const uint32_t n = (uint32_t)((rg.n - t0) < T ? (rg.n - t0) : T);
  uint64_t *const tts = L.tile_ts + hb * T;
  uint32_t *const tfk = L.tile_fk + hb * T;
  uint64_t *const tby = L.tile_by + hb * T;
  uint32_t *const soff = L.soff + hb * (S_MAX + 1);
  auto gbar = [&]() {
    if (PIPE) group_barrier(&L.misc[3], GW, tb.err);
    else __syncthreads();
  };
    uint64_t r_ts[ROWS], r_x[ROWS], r_by[ROWS];
    uint32_t r_tid[ROWS], r_fk[ROWS], r_slot[ROWS], r_rank[ROWS] = {};
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
      const uint32_t li = (uint32_t)w * (T / GW) + (uint32_t)r * WAVE + lane;
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
        const uint32_t li = (uint32_t)w * (T / GW) + (uint32_t)r * WAVE + lane;
        const uint32_t v = li < n ? (r_fk[r] >> 24) : 0;
        const uint32_t inc = wave_incl_scan(v);
        excl[r] = run + inc - v;
        run += __shfl(inc, WAVE - 1, WAVE);
      }
      if (lane == 0) L.wsum[w] = run;
      gbar();
      uint32_t wpre = 0, tot = 0;
      for (int k = 0; k < (int)GW; k++) { const uint32_t s = L.wsum[k]; if (k < w) wpre += s; tot += s; }
#pragma unroll
      for (int r = 0; r < ROWS; r++) {
        const uint32_t li = (uint32_t)w * (T / GW) + (uint32_t)r * WAVE + lane;
        const uint32_t fn = r_fk[r] & 0xFFFFu, kind = (r_fk[r] >> 16) & 0xFFu, plen = r_fk[r] >> 24;
        const uint64_t off = pay_run + wpre + excl[r];
        // off + 8 <= pay_bytes holds for every well-formed chunk; a chunk whose
        // payload_len sum disagrees with its heap fails the flush (ERR_PAYLOAD)
        // and reads nothing outside the heap
        const bool in_heap = off + 8 <= sg.pay_bytes;
        const bool sized = li < n && kind == 0 && fn < tb.n_fns && plen >= 8 && in_heap && tb.has_size &&
                           tb.has_size[fn];
        const bool kend = li < n && kind == 2 && plen >= 8 && in_heap;
        if (sized || kend) {
          const uint64_t v = load_u64_unaligned(sg.pay, off);
          if (sized) r_by[r] = v; else r_x[r] = v;
        }
      }
      pay_run += tot;
      gbar();
    }
    // ---- P2. kernel records, validity, counters (wave totals by ballot); an
    // extra pass over the range only takes the API records of its threads
    constexpr bool first_pass = !XP;
#pragma unroll
    for (int r = 0; r < ROWS; r++) {
      const uint32_t li = (uint32_t)w * (T / GW) + (uint32_t)r * WAVE + lane;
      const uint32_t fn = r_fk[r] & 0xFFFFu, kind = (r_fk[r] >> 16) & 0xFFu, plen = r_fk[r] >> 24;
      const bool in = li < n;
      const bool api = in && kind <= 1 && fn < tb.n_fns;
      r_slot[r] = api ? 0u : EMPTY32;
      if constexpr (XP) continue;
      const uint64_t end = r_x[r], d = end - r_ts[r];
      const bool kern_ok = in && kind == 2 && fn < tb.n_kid && (FMT == 1 || plen >= 8) && end >= r_ts[r];
      const bool bad = in && !api && !kern_ok;
      // kernel durations: LDS rows for ids below KL and durations below 2^32
      // ns; the rest goes to the global rows
      const bool kl = kern_ok && fn < KL && d < EMPTY32;
      if (kl) {
        lds_add32(&L.q_cnt[fn], 1u);
        lds_add64(&L.q_sum[fn], d);
        lds_min32(&L.q_min[fn], (uint32_t)d);
        lds_max32(&L.q_max[fn], (uint32_t)d);
      }
      const bool kg = kern_ok && !kl;
      if (ballot(kg)) {
        if (kg) {
          KTally *kt = &tb.ktally[(size_t)sg.stream * tb.n_kid + fn];
          if (fn < KL) { lds_add32(&L.q_cnt[fn], 1u); lds_add64(&L.q_sum[fn], d); }
          else { g_add64(&kt->count, 1); g_add64(&kt->sum, d); }
          g_min64(&kt->min, d); g_max64(&kt->max, d);
        }
      }
      wc[0] += (uint32_t)__popcll(ballot(api && kind == 0));
      wc[1] += (uint32_t)__popcll(ballot(api && kind == 1));
      wc[2] += (uint32_t)__popcll(ballot(kern_ok));
      wc[3] += (uint32_t)__popcll(ballot(bad));
    }
    if (w == 0 && first_pass) wc[4] += n;
    // ---- P3. thread id -> local slot
    // bucket word: bit 63 occupied, bit 62 pending, [32,40) slot, [0,32) tid.
    // A lane that finds no bucket for its tid claims one as pending and lists
    // the tid; its record is ranked after the listed tids get slots.
    uint32_t r_late = 0;   // bit r: row r's thread has no slot yet
    // (the first bucket settles nearly every record; the probe loop runs for
    // the other lanes only)
    uint32_t r_open = 0;   // bit r: row r still probing
    const uint32_t scap = slot_cap(D);
    if constexpr (XP) {
      // extra pass: the thread of each record through the global thread map;
      // slot = ordinal - c0 for the threads of this pass's class that the
      // range's first pass did not take (the set in L.newtid)
      const uint32_t c0 = (rg.pass - 1) * scap;
#pragma unroll
      for (int r = 0; r < ROWS; r++) {
        if (r_slot[r] == EMPTY32) continue;
        const uint32_t g = lookup_gslot(tb, sg.stream, r_tid[r]);
        uint32_t sl = EMPTY32;
        if (g < tb.max_threads) {
          const uint32_t o = tb.th_ord[g];
          if (o - c0 < scap && !in_gset(L.newtid, g)) {
            sl = o - c0;
            L.srec[sl].gslot = g;   // (every such lane writes the same value)
          }
        }
        r_slot[r] = sl;
      }
    } else {
#pragma unroll
    for (int r = 0; r < ROWS; r++) {
      const uint32_t t = r_tid[r];
      const uint64_t e = L.tidmap[tid_bucket(t)];
      const bool done = (e >> 63) && !((e >> 62) & 1u) && (uint32_t)e == t;
      const uint32_t sl = (uint32_t)(e >> 32) & 0xFFu;
      const bool act = r_slot[r] != EMPTY32;
      if (act && done) r_slot[r] = sl < scap ? sl : EMPTY32;  // beyond the range's slots: an extra pass takes it
      if (act && !done) r_open |= 1u << r;
    }
    if (ballot(r_open != 0)) {
    // the next bucket settles a tid whose first bucket was taken by another
    // (in a stream with such a pair, nearly every wave holds records of the
    // displaced thread, so this keeps those waves out of the probe loop)
#pragma unroll
    for (int r = 0; r < ROWS; r++) {
      if (!(r_open & (1u << r))) continue;
      const uint32_t t = r_tid[r];
      const uint64_t e = L.tidmap[(tid_bucket(t) + 1u) & (TIDMAP - 1)];
      if ((e >> 63) && !((e >> 62) & 1u) && (uint32_t)e == t) {
        const uint32_t sl = (uint32_t)(e >> 32) & 0xFFu;
        r_slot[r] = sl < scap ? sl : EMPTY32;  // beyond the range's slots: an extra pass takes it
        r_open &= ~(1u << r);
      }
    }
    }
    if (ballot(r_open != 0)) {
#pragma unroll
    for (int r = 0; r < ROWS; r++) {
      if (!(r_open & (1u << r))) continue;
      const uint32_t t = r_tid[r];
      uint32_t h = tid_bucket(t);
      bool placed = false;
      for (uint32_t probe = 0; probe < TIDMAP; probe++) {
        uint64_t e = L.tidmap[h];
        if (e == 0) {
          const uint64_t want = (1ull << 63) | (1ull << 62) | t;
          e = atomicCAS((unsigned long long *)&L.tidmap[h], 0ull, (unsigned long long)want);
          if (e == 0) {
            const uint32_t k = atomicAdd(&L.misc[1], 1u);
            L.newtid[k] = t;
            L.newbucket[k] = h;
            r_slot[r] = EMPTY32 - 1;
            r_late |= 1u << r;
            placed = true;
            break;
          }
        }
        if ((uint32_t)e == t) {
          const uint32_t sl = (uint32_t)(e >> 32) & 0xFFu;
          if (e & (1ull << 62)) { r_slot[r] = EMPTY32 - 1; r_late |= 1u << r; }
          else r_slot[r] = sl < scap ? sl : EMPTY32;  // beyond the range's slots: an extra pass takes it
          placed = true;
          break;
        }
        h = (h + 1) & (TIDMAP - 1);
      }
      if (!placed) {
        // the map is full: the thread is registered (so it has an ordinal)
        // and left to an extra pass
        resolve_gslot(tb, sg.stream, t);
        r_slot[r] = EMPTY32;
        L.misc[9] = 1u;
      }
    }
    }
    }
    // ---- P4. stable sort of the API records by slot: rank each record among
    // the wave's records of its slot (ballot match masks over the slot bits;
    // per-wave counters carry the rank across rows).  Records of threads new
    // in this tile are ranked after their slots exist; no other record of
    // those slots is in the tile, so the order stays stable.
    const uint32_t nslots0 = L.misc[0];
    // per-wave counts of this half (PIPE: the two halves use separate rows,
    // so a wave may start the next tile while others still read these)
    uint32_t *const wcnt = L.wcnt + (PIPE ? hb * GW * S_MAX : 0u);
    if (lane < S_MAX) wcnt[w * S_MAX + lane] = 0;
    auto rank_rows = [&](const bool late, const uint32_t ns) {
      uint32_t nbits = 0;
      while ((1u << nbits) < ns) nbits++;
#pragma unroll
      for (int r = 0; r < ROWS; r++) {
        const bool valid = late ? (r_late & (1u << r)) && r_slot[r] != EMPTY32
                                : r_slot[r] != EMPTY32 && r_slot[r] != EMPTY32 - 1;
        const uint32_t s = valid ? r_slot[r] : 0;
        uint64_t mask = ballot(valid);
        for (uint32_t b = 0; b < nbits; b++) {
          const uint64_t bb = ballot(valid && ((s >> b) & 1u));
          mask &= ((s >> b) & 1u) ? bb : ~bb;
        }
        const uint32_t rk = (uint32_t)__popcll(mask & lanemask_lt());
        const uint32_t c = (uint32_t)__popcll(mask);
        const uint32_t base = wcnt[w * S_MAX + s];
        r_rank[r] = valid ? base + rk : r_rank[r];
        if (valid && rk == 0) wcnt[w * S_MAX + s] = base + c;
      }
    };
    rank_rows(false, nslots0);
    gbar();
    const uint32_t n_new = L.misc[1];
    uint32_t nslots = nslots0;
    if (n_new) {
      // threads seen for the first time in this range: global slot, local slot
      if ((uint32_t)tid < n_new) {
        // (a thread beyond the range's slots is registered too, so that it
        // has an ordinal, and left to an extra pass over the range)
        const uint32_t s = nslots0 + tid;
        const uint32_t t = L.newtid[tid];
        const uint32_t g = resolve_gslot(tb, sg.stream, t);
        if (s < scap) L.srec[s].gslot = g;
        else L.misc[9] = 1u;
        L.tidmap[L.newbucket[tid]] = (1ull << 63) | ((uint64_t)(s < scap ? s : 0xFFu) << 32) | t;
      }
      gbar();
      nslots = nslots0 + n_new < scap ? nslots0 + n_new : scap;
      if (tid == 0) { L.misc[0] = nslots; L.misc[1] = 0; }
#pragma unroll
      for (int r = 0; r < ROWS; r++) {
        if (!(r_late & (1u << r))) continue;
        const uint32_t t = r_tid[r];
        uint32_t h = tid_bucket(t);
        r_slot[r] = EMPTY32;
        for (uint32_t probe = 0; probe < TIDMAP; probe++) {
          const uint64_t e = L.tidmap[h];
          if (e == 0) break;
          if ((uint32_t)e == t) { r_slot[r] = (uint32_t)(e >> 32) & 0xFFu; break; }
          h = (h + 1) & (TIDMAP - 1);
        }
        if (r_slot[r] >= scap) r_slot[r] = EMPTY32;  // beyond the range's slots: an extra pass takes it
      }
      rank_rows(true, nslots);
      gbar();
    }
    // the tally layout of this range, fixed before its first call is tallied:
    // direct-mapped rows for every thread when the first tile's threads all
    // fit, otherwise one open-addressing table over all entries
    if (t0 == 0 && tid == 0) {
      const uint32_t dcap = direct_slots(tb.n_fns, E);
      L.misc[2] = nslots <= dcap ? dcap : 0;
    }
    // each wave: lane s counts slot s over all waves and over the waves before
    // this one, so every wave knows where its records of each slot go
    uint32_t wb;
    {
      uint32_t tot = 0, before = 0;
      if ((uint32_t)lane < nslots)
        for (int k = 0; k < (int)GW; k++) {
          const uint32_t c = wcnt[k * S_MAX + lane];
          tot += c;
          before += k < w ? c : 0;
        }
      const uint32_t inc = wave_incl_scan(tot);
      wb = inc - tot + before;
      if (w == 0) {
        if ((uint32_t)lane < nslots) soff[lane] = inc - tot;
        if (lane == WAVE - 1) soff[nslots] = inc;
        if (lane == 0) L.misc[7 + hb] = nslots;
      }
    }
#pragma unroll
    for (int r = 0; r < ROWS; r++) {
      const uint32_t sl = r_slot[r] == EMPTY32 ? 0u : r_slot[r];
      const uint32_t pos = (uint32_t)__builtin_amdgcn_ds_bpermute((int32_t)(sl << 2), (int32_t)wb) + r_rank[r];
      if (r_slot[r] == EMPTY32) continue;
      tts[pos] = r_ts[r];
      tfk[pos] = (r_fk[r] & 0xFFFFu) | (((r_fk[r] >> 16) & 1u) << 16);
      if (FMT == 2) tby[pos] = r_by[r];
    }
    // PIPE: each wave publishes its part of the tile itself (no barrier)
    if (!PIPE) __syncthreads();
}


// ------------------------------------------------------------------ kernel
// One whole range: LDS set-up, every tile, then the range summaries and the
// flush of the LDS tallies and counters to the global tables.
//
// PIPE off: all 16 waves run the front half of a tile, then the walk, in
// lockstep (workgroup barriers).  PIPE on: waves RNW/2 .. RNW-1 (producers)
// build sorted tiles into the two halves of the tile region alternately while
// waves 0 .. RNW/2-1 (walkers) walk the previous one; a tile is handed over
// through LDS counters: every producer wave counts each tile it finished,
// every walker publishes the tiles it has walked.
template <int FMT, int ROWS, bool PIPE, bool IV, bool XP>
__device__ __forceinline__ void range_body(RangeLds &L, const Seg *__restrict__ segs,
                                           const Range *__restrict__ ranges, const uint32_t rid,
                                           const uint32_t sid, const Range *__restrict__ pranges, const Tables &tb,
                                           const Shape &sh, RHdr *__restrict__ rhdr, UItem *__restrict__ ru,
                                           OItem *__restrict__ ro, uint32_t *__restrict__ rnslots,
                                           uint32_t *__restrict__ rmore) {
  constexpr uint32_t GW = PIPE ? RNW / 2 : RNW;     // waves that build tiles
  constexpr uint32_t T = ROWS * GW * WAVE;          // records per tile
  constexpr uint32_t RS = FMT == 2 ? 16 : 24;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t D = tb.D, E = sh.E, KL = sh.KL;
  Range rg = ranges[rid];
  if (XP) rg.pay_begin = pranges[rg.parent].pay_begin;   // (filled on the device for the first pass)
  const Seg sg = segs[rg.seg];
  typedef typename TEntOf<FMT>::T TE;
  typedef typename CFrameOf<FMT>::T CF;
  TE *const tal = (TE *)L.tal;
  const CF *const cfr = (const CF *)L.cfr;
  for (uint32_t i = tid; i < E; i += RWG) {
    TE &te = tal[i];
    te.key = EMPTY32; te.cnt = 0; te.imin = EMPTY32; te.imax = 0;
    te.smin = EMPTY32; te.smax = 0; te.isum = 0; te.ssum = 0;
    if constexpr (FMT == 2) te.bsum = 0;
  }
  for (uint32_t i = tid; i < KL; i += RWG) { L.q_cnt[i] = 0; L.q_min[i] = EMPTY32; L.q_max[i] = 0; L.q_sum[i] = 0; }
  for (uint32_t i = tid; i < TIDMAP; i += RWG) L.tidmap[i] = 0;
  for (uint32_t i = tid; i < S_MAX; i += RWG) {
    SRec &r = L.srec[i];
    r.gslot = GV_INVALID; r.flags = 0; r.d = 0; r.u = 0; r.H = 0; r.M = 0;
    r.facc = 0; r.first = 0; r.last = 0;
  }
  for (uint32_t i = tid; i < ST_N; i += RWG) L.cnt[i] = 0;
  if (tid < 32) L.misc[tid] = 0;
  if (XP) for (uint32_t i = tid; i < TIDMAP; i += RWG) L.newtid[i] = EMPTY32;
  __syncthreads();
  if (XP) {
    // an extra pass: all of its class's slots exist from the start, and the
    // threads the range's first pass took are skipped (a set in L.newtid)
    const uint32_t nf = rnslots[rg.parent];
    if ((uint32_t)tid < nf) {
      const uint32_t g = rhdr[(size_t)rg.parent * S_MAX + tid].gslot;
      uint32_t h = tid_bucket(g);
      for (uint32_t probe = 0; probe < TIDMAP; probe++) {
        const uint32_t old = atomicCAS(&L.newtid[h], EMPTY32, g);
        if (old == EMPTY32 || old == g) break;
        h = (h + 1) & (TIDMAP - 1);
      }
    }
    if (tid == 0) L.misc[0] = slot_cap(D);
    __syncthreads();
  }

  const size_t sbase = (size_t)sid * S_MAX;
  const uint64_t ntiles = (rg.n + T - 1) / T;
  IvRec *const ivr = IV ? tb.iv + rg.iv_base : nullptr;
  if (!PIPE || w >= (int)GW) {
    // tile builder: two register buffers of raw record words alternate
    // between tiles; the loads are unconditional (index clamped to the range)
    // so that nothing waits for them before the tile that uses them
    const int gw = PIPE ? w - (int)GW : w;
    uint64_t pay_run = rg.pay_begin;  // payload offset of the current tile's first record
    gu64 *grec = (gu64 *)sg.rec;
    const uint64_t last_rec = rg.begin + rg.n - 1;
    uint64_t a0[ROWS], a1[ROWS], a2[ROWS], b0[ROWS], b1[ROWS], b2[ROWS];
    uint32_t wc[5] = {0, 0, 0, 0, 0};   // this wave's record counts over the range
    WalkCache wcache;
    wcache.slot = EMPTY32;
    wcache.pend = 0;
    WalkDefer dw;
#pragma unroll
    for (uint32_t j = 0; j < DEFER_SETS; j++) { dw.n[j] = 0; dw.ts[j] = 0; dw.by[j] = 0; dw.fk[j] = 0; }
#pragma unroll
    for (int r = 0; r < ROWS; r++) {
      const uint32_t li = (uint32_t)gw * (T / GW) + (uint32_t)r * WAVE + lane;
      uint64_t idx = rg.begin + li;
      idx = idx < last_rec ? idx : last_rec;
      gu64 *p = grec + idx * (RS / 8);
      a0[r] = __builtin_nontemporal_load(p);
      a1[r] = __builtin_nontemporal_load(p + 1);
      a2[r] = FMT == 1 ? __builtin_nontemporal_load(p + 2) : 0;
    }
    for (uint64_t t = 0; t < ntiles; t++) {
      const uint32_t hb = PIPE ? (uint32_t)(t & 1) : 0u;
      // PIPE: the half of tile t - 2 must have been walked
      if (PIPE && t >= 2) wait_all_at_least(&L.misc[16], GW, (uint32_t)(t - 1), tb.err);
      front_tile<FMT, ROWS, PIPE, XP>(L, tb, E, KL, D, rg, sg, grec, last_rec, t * T, hb, a0, a1, a2, b0, b1, b2,
                                      pay_run, wc);
      if (PIPE) {
        // one count per builder wave and tile
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        if (lane == 0) __hip_atomic_fetch_add(&L.misc[5], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      // (FIXED24: every slot's partial window waits for its next records;
      // VAR16 keeps the registers for its payload words)
      else if (FMT == 1) walk_tile<FMT, IV>(L, tb, E, D, 0, T, RNW, t + 1 < ntiles, sbase, ru, wcache, ivr, &dw);
      else walk_tile<FMT, IV>(L, tb, E, D, 0, T, RNW, false, sbase, ru, wcache, ivr);
      if (!PIPE) __syncthreads();
#pragma unroll
      for (int r = 0; r < ROWS; r++) { a0[r] = b0[r]; a1[r] = b1[r]; a2[r] = b2[r]; }
    }
    if (!PIPE) slot_store(L, wcache, L.w_vt + w * (D + 1));   // (the last tile walks every waiting record)
    if (lane == 0) {
      const int idx[5] = {ST_ENTRIES, ST_EXITS, ST_KERNEL, ST_BAD, ST_RECORDS};
#pragma unroll
      for (int k = 0; k < 5; k++)
        if (wc[k]) lds_add32(&L.cnt[idx[k]], wc[k]);
    }
  } else {
    // walker: its own progress counter tells the builders which half is free
    WalkCache wcache;
    wcache.slot = EMPTY32;
    wcache.pend = 0;
    for (uint64_t t = 0; t < ntiles; t++) {
      wait_at_least(&L.misc[5], (uint32_t)(t + 1) * GW, tb.err);
      walk_tile<FMT, IV>(L, tb, E, D, (uint32_t)(t & 1), T, GW, true, sbase, ru, wcache, ivr);
      publish(&L.misc[16 + w], (uint32_t)(t + 1), lane == 0);
    }
    walk_finish<FMT, IV>(L, tb, E, D, sbase, ru, wcache, ivr);
  }
  __syncthreads();
  L.nd = L.misc[2];

  // ---- range end: summaries, tally and counter flush
  const uint32_t nslots = L.misc[0];
  if (tid == 0) {
    rnslots[sid] = nslots;
    rmore[sid] = L.misc[9];   // threads left to extra passes
    if (L.misc[9]) atomicOr(tb.err, ERR_WIDE);
  }
  if (IV && tid == 0) tb.iv_n[sid] = L.misc[6];
  if ((uint32_t)tid < nslots) {
    const uint32_t s = tid;
    const SRec &r = L.srec[s];
    RHdr hd;
    hd.gslot = r.gslot;
    hd.nu_total = (uint32_t)r.u;
    hd.nu_listed = hd.nu_total < D ? hd.nu_total : D;
    hd.n_o = (uint32_t)(r.d + r.u);
    hd.floor = r.facc;
    hd.H = r.H; hd.M = r.M;
    hd.first_ts = r.first; hd.last_ts = r.last;
    hd.flags = r.flags;
    hd.pad = 0; hd.pad2 = 0;
    rhdr[sbase + s] = hd;
    if (!XP) L.newtid[s] = r.gslot < tb.max_threads ? tb.th_ord[r.gslot] : EMPTY32;   // (for the partial tally)
    const uint32_t no = hd.n_o < D ? hd.n_o : D;
    for (uint32_t k = 0; k < no; k++) {
      OItem *o = &ro[(sbase + s) * D + k];
      const CF &cf = cfr[(size_t)s * D + k];
      o->ts = cf.ts;
      o->child = cf.ch;
      if constexpr (FMT == 2) o->bytes = cf.by; else o->bytes = 0;
      o->fn = (uint16_t)cf.fn;
      o->pad = 0;
    }
  }
  const uint32_t nd = L.nd, d0 = nd * tb.n_fns;
  // a range whose threads all have direct-mapped rows and stream ordinals
  // below PART_ORDS stores its rows as a partial tally (merged per row after
  // the combine); any other range adds its entries with global atomics
  uint32_t pmask = 0;
  if (!XP && rid < tb.part_ranges) {
    __syncthreads();
    if (tid == 0) {
      uint32_t m = 0;
      bool ok = nslots <= nd;
      for (uint32_t s = 0; ok && s < nslots; s++) {
        const uint32_t o = L.newtid[s];
        if (o < PART_ORDS) m |= 1u << o;
        else ok = false;
      }
      L.misc[11] = ok ? m : 0u;
      tb.part_mask[rid] = ok ? m : 0u;
    }
    __syncthreads();
    pmask = L.misc[11];
  }
  if (pmask) {
    TE *const dst = (TE *)tb.part + (size_t)rid * PART_ORDS * tb.n_fns;
    for (uint32_t i = tid; i < nslots * tb.n_fns; i += RWG) {
      const uint32_t s = i / tb.n_fns, fn = i - s * tb.n_fns;
      dst[(size_t)L.newtid[s] * tb.n_fns + fn] = tal[i];
    }
    if ((uint32_t)tid < nslots) tb.part_gslot[rid * PART_ORDS + L.newtid[tid]] = L.srec[tid].gslot;
  }
  for (uint32_t i = pmask ? E : (uint32_t)tid; i < E; i += RWG) {
    uint32_t s, fn;
    const TE &te = tal[i];
    if (i < d0) {
      if (!te.cnt) continue;
      s = i / tb.n_fns;
      fn = i - s * tb.n_fns;
    } else {
      const uint32_t key = te.key;
      if (key == EMPTY32) continue;
      s = key >> 16;
      fn = key & 0xFFFFu;
    }
    const uint32_t gs = L.srec[s].gslot;
    if (gs >= tb.max_threads) continue;
    Tally *g = &tb.tally[(size_t)gs * tb.n_fns + fn];
    g_add64(&g->count, te.cnt);
    g_add64(&g->incl_sum, te.isum);
    g_add64(&g->self_sum, te.ssum);
    if constexpr (FMT == 2) { if (te.bsum) g_add64(&g->bytes_sum, te.bsum); }
    if (te.imin != EMPTY32) g_min64(&g->incl_min, te.imin);
    if (te.imax) g_max64(&g->incl_max, te.imax);
    if (te.smin != EMPTY32) g_min64(&g->self_min, te.smin);
    if (te.smax) g_max64(&g->self_max, te.smax);
  }
  for (uint32_t i = tid; i < KL; i += RWG) {
    if (!L.q_cnt[i]) continue;
    KTally *kt = &tb.ktally[(size_t)sg.stream * tb.n_kid + i];
    g_add64(&kt->count, L.q_cnt[i]);
    g_add64(&kt->sum, L.q_sum[i]);
    if (L.q_min[i] != EMPTY32) g_min64(&kt->min, L.q_min[i]);
    if (L.q_max[i]) g_max64(&kt->max, L.q_max[i]);
  }
  for (uint32_t i = tid; i < ST_N; i += RWG)
    if (L.cnt[i]) atomicAdd(&tb.sstats[(size_t)sg.stream * ST_N + i], (unsigned long long)L.cnt[i]);
}

// Persistent work-list launch: each workgroup (one per CU) takes the next
// entry of `order` (range ids, longest first) until the list is exhausted.
// `qhead` must be 0 at launch.  Range i writes its summaries as summary row
// rid_base + i (rmore: whether threads were left to extra passes).  XP: a
// launch of extra passes, whose entries name their first pass's range in
// `pranges` (rid_base: the number of those ranges, > 0).
template <int FMT, int ROWS, bool PIPE, bool IV, bool XP>
__global__ __launch_bounds__(RWG) void k_range(const Seg *__restrict__ segs, const Range *__restrict__ ranges,
                                               const uint32_t *__restrict__ order, const uint32_t n_ranges,
                                               uint32_t *__restrict__ qhead, Tables tb, Shape sh,
                                               RHdr *__restrict__ rhdr, UItem *__restrict__ ru,
                                               OItem *__restrict__ ro, uint32_t *__restrict__ rnslots,
                                               uint32_t *__restrict__ rmore, const Range *__restrict__ pranges,
                                               const uint32_t rid_base) {
  extern __shared__ __align__(16) uint8_t smem[];
  __shared__ uint32_t next;
  RangeLds L;
  range_lds_layout<true>(smem, &L, ROWS * RWG, sh.E, sh.KL, tb.D, FMT);   // (PIPE: two halves of ROWS * RWG / 2)
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(qhead, 1u);
    __syncthreads();
    const uint32_t q = next;
    __syncthreads();
    if (q >= n_ranges) break;
    const uint32_t rid = order[q];
    range_body<FMT, ROWS, PIPE, IV, XP>(L, segs, ranges, rid, XP ? rid_base + rid : rid, pranges, tb, sh, rhdr, ru,
                                        ro, rnslots, rmore);
  }
}

// VAR16 pre-pass: payload bytes of each slice of PAY_SLICE records (sum of
// payload_len), one workgroup per slice.
__global__ __launch_bounds__(WG) void k_slice_paylen(const Seg *__restrict__ segs, const Range *__restrict__ ranges,
                                                     uint32_t n_ranges, const uint32_t *__restrict__ slice_first,
                                                     uint64_t *__restrict__ out) {
  __shared__ unsigned long long acc;
  if (threadIdx.x == 0) acc = 0;
  __syncthreads();
  const uint32_t r = range_of_slice(slice_first, n_ranges, blockIdx.x);
  const Range rg = ranges[r];
  const Seg sg = segs[rg.seg];
  const uint64_t lo = (uint64_t)(blockIdx.x - slice_first[r]) * PAY_SLICE;
  const uint64_t n = rg.n - lo < PAY_SLICE ? rg.n - lo : PAY_SLICE;
  uint64_t s = 0;
  gu64 *hdr = (gu64 *)(sg.rec + (rg.begin + lo) * 16) + 1;   // word 1 of each header: payload_len in its top byte
  uint64_t i = threadIdx.x;
  for (; i + 7 * WG < n; i += 8 * WG) {               // eight independent loads in flight per lane
    uint64_t w[8];
#pragma unroll
    for (int k = 0; k < 8; k++) w[k] = __builtin_nontemporal_load(hdr + 2 * (i + (uint64_t)k * WG));
#pragma unroll
    for (int k = 0; k < 8; k++) s += w[k] >> 56;
  }
  for (; i < n; i += WG) s += __builtin_nontemporal_load(hdr + 2 * i) >> 56;
  atomicAdd(&acc, (unsigned long long)s);
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = acc;
}

// VAR16: exclusive prefix of the slice payload sizes within each segment,
// in place (paylen[b] becomes the payload offset of slice b), and each
// range's pay_begin (that of its first slice); a segment whose payload_len
// sum is not its heap size raises ERR_PAYLOAD.  One workgroup per segment
// (its slices are consecutive), PO_WG slices at a time.
constexpr uint32_t PO_WG = 256;
__global__ __launch_bounds__(PO_WG) void k_range_payoff(const Seg *__restrict__ segs,
                                                        const uint32_t *__restrict__ seg_first_range,
                                                        Range *__restrict__ ranges,
                                                        const uint32_t *__restrict__ slice_first,
                                                        uint64_t *__restrict__ paylen, uint32_t *err) {
  __shared__ uint64_t ws[PO_WG / WAVE];
  const uint32_t sgi = blockIdx.x, lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  const uint32_t r0 = seg_first_range[sgi], r1 = seg_first_range[sgi + 1];
  const uint32_t b0 = slice_first[r0], b1 = slice_first[r1];
  uint64_t carry = 0;
  for (uint32_t c = b0; c < b1; c += PO_WG) {
    const uint32_t b = c + threadIdx.x;
    const uint64_t v = b < b1 ? paylen[b] : 0;
    uint64_t inc = v;
    for (uint32_t d = 1; d < WAVE; d <<= 1) {
      const uint64_t t = __shfl_up(inc, d, WAVE);
      if (lane >= d) inc += t;
    }
    if (lane == WAVE - 1) ws[w] = inc;
    __syncthreads();
    uint64_t before = 0, tot = 0;
    for (uint32_t k = 0; k < PO_WG / WAVE; k++) { before += k < w ? ws[k] : 0; tot += ws[k]; }
    if (b < b1) paylen[b] = carry + before + inc - v;
    carry += tot;
    __syncthreads();
  }
  for (uint32_t r = r0 + threadIdx.x; r < r1; r += PO_WG) ranges[r].pay_begin = paylen[slice_first[r]];
  if (threadIdx.x == 0 && carry != segs[sgi].pay_bytes) atomicOr(err, ERR_PAYLOAD);
}

// --------------------------------------------------------------- launchers
// Allows every range-kernel variant up to max_lds_bytes of dynamic LDS (set
// once, outside any stream capture).
// Merge of the partial tallies: one lane per (stream, ordinal, fn) row sums
// the row over the stream's ranges that stored it (count and sums, 32-bit
// min / max with the LDS tally's sentinels) and adds the result to the global
// row once.  spans[3 j .. 3 j + 2] = {stream, first range, end range}.
template <int FMT>
__global__ __launch_bounds__(256) void k_part_merge(const uint32_t *__restrict__ spans, uint32_t n_spans, Tables tb) {
  typedef typename TEntOf<FMT>::T TE;
  const uint32_t idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= PART_ORDS * tb.n_fns) return;
  const uint32_t ord = idx / tb.n_fns, fn = idx - ord * tb.n_fns;
  const TE *const part = (const TE *)tb.part;
  for (uint32_t sp = blockIdx.y; sp < n_spans; sp += gridDim.y) {
    const uint32_t r0 = spans[3 * sp + 1], r1e = spans[3 * sp + 2];
    const uint32_t r1 = r1e < tb.part_ranges ? r1e : tb.part_ranges;
    uint64_t cnt = 0, isum = 0, ssum = 0, bsum = 0;
    uint32_t imin = EMPTY32, imax = 0, smin = EMPTY32, smax = 0, g = EMPTY32;
    // (four ranges' entries in flight at once; an entry its range never
    // touched holds a zero count and sums and the min / max sentinels, so it
    // adds nothing)
    for (uint32_t r = r0; r < r1; r += 4) {
      TE e[4];
      uint32_t gk[4];
#pragma unroll
      for (uint32_t k = 0; k < 4; k++) {
        const bool in = r + k < r1 && ((tb.part_mask[r + k] >> ord) & 1u);
        gk[k] = EMPTY32;
        if (in) {
          e[k] = part[((size_t)(r + k) * PART_ORDS + ord) * tb.n_fns + fn];
          gk[k] = tb.part_gslot[(r + k) * PART_ORDS + ord];
        } else {
          e[k].cnt = 0; e[k].isum = 0; e[k].ssum = 0;
          e[k].imin = EMPTY32; e[k].imax = 0; e[k].smin = EMPTY32; e[k].smax = 0;
          if constexpr (FMT == 2) e[k].bsum = 0;
        }
      }
#pragma unroll
      for (uint32_t k = 0; k < 4; k++) {
        if (gk[k] != EMPTY32) g = gk[k];
        cnt += e[k].cnt;
        isum += e[k].isum;
        ssum += e[k].ssum;
        if constexpr (FMT == 2) bsum += e[k].bsum;
        imin = e[k].imin < imin ? e[k].imin : imin;
        imax = e[k].imax > imax ? e[k].imax : imax;
        smin = e[k].smin < smin ? e[k].smin : smin;
        smax = e[k].smax > smax ? e[k].smax : smax;
      }
    }
    if (!cnt || g >= tb.max_threads) continue;
    Tally *row = &tb.tally[(size_t)g * tb.n_fns + fn];
    g_add64(&row->count, cnt);
    g_add64(&row->incl_sum, isum);
    g_add64(&row->self_sum, ssum);
    if (bsum) g_add64(&row->bytes_sum, bsum);
    if (imin != EMPTY32) g_min64(&row->incl_min, imin);
    if (imax) g_max64(&row->incl_max, imax);
    if (smin != EMPTY32) g_min64(&row->self_min, smin);
    if (smax) g_max64(&row->self_max, smax);
  }
}

// Bytes of one range's partial tally.
size_t part_range_bytes(uint32_t n_fns, int fmt) {
  return (size_t)PART_ORDS * n_fns * (fmt == 2 ? sizeof(TEnt2) : sizeof(TEnt1));
}

hipError_t launch_part_merge(int fmt, const uint32_t *spans, uint32_t n_spans, const Tables &tb, hipStream_t st) {
  if (!tb.part_ranges || !n_spans) return hipSuccess;
  const dim3 grid((PART_ORDS * tb.n_fns + 255) / 256, n_spans < 65535u ? n_spans : 65535u);
  if (fmt == 2) hipLaunchKernelGGL(k_part_merge<2>, grid, dim3(256), 0, st, spans, n_spans, tb);
  else hipLaunchKernelGGL(k_part_merge<1>, grid, dim3(256), 0, st, spans, n_spans, tb);
  return hipGetLastError();
}

hipError_t prepare_range_kernels(uint32_t max_lds_bytes) {
  const void *ks[] = {
#define TT_K(F, R, P, I, X) (const void *)k_range<F, R, P, I, X>
      TT_K(1, 1, false, false, false), TT_K(1, 2, false, false, false), TT_K(2, 1, false, false, false),
      TT_K(2, 2, false, false, false), TT_K(1, 1, true, false, false),  TT_K(1, 2, true, false, false),
      TT_K(2, 1, true, false, false),  TT_K(2, 2, true, false, false),  TT_K(1, 1, false, true, false),
      TT_K(1, 2, false, true, false),  TT_K(2, 1, false, true, false),  TT_K(2, 2, false, true, false),
      TT_K(1, 1, true, true, false),   TT_K(1, 2, true, true, false),   TT_K(2, 1, true, true, false),
      TT_K(2, 2, true, true, false),   TT_K(1, 1, false, false, true),  TT_K(1, 2, false, false, true),
      TT_K(2, 1, false, false, true),  TT_K(2, 2, false, false, true),  TT_K(1, 1, false, true, true),
      TT_K(1, 2, false, true, true),   TT_K(2, 1, false, true, true),   TT_K(2, 2, false, true, true),
      // (4096-record tiles: FIXED24 only; a VAR16 tile of 4096 records does not fit in LDS)
      TT_K(1, 4, false, false, false), TT_K(1, 4, true, false, false),  TT_K(1, 4, false, true, false),
      TT_K(1, 4, true, true, false),   TT_K(1, 4, false, false, true),  TT_K(1, 4, false, true, true),
#undef TT_K
  };
  for (const void *k : ks) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds_bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// n_wg: workgroups of the persistent launch (at most one per CU is resident);
// *qhead must be 0 (the caller clears it with a kernel, so the launch can be
// captured in a graph).  T: records of the LDS tile region (1024, 2048, or
// 4096 for FIXED24);
// with sh.pipe the tiles are half of it.
hipError_t launch_range(int fmt, uint32_t T, const Seg *segs, const Range *ranges, const uint32_t *order,
                        uint32_t n_ranges, uint32_t *qhead, uint32_t n_wg, const Tables &tb, const Shape &sh,
                        RHdr *rhdr, UItem *ru, OItem *ro, uint32_t *rnslots, uint32_t *rmore,
                        const Range *pranges, uint32_t rid_base, hipStream_t st) {
  if (!n_ranges) return hipSuccess;
  dim3 grid(n_wg < n_ranges ? n_wg : n_ranges), block(RWG);
#define TT_LAUNCH(F, ROWS_, P_)                                                                                 \
  do {                                                                                                          \
    if (iv)                                                                                                     \
      hipLaunchKernelGGL((k_range<F, ROWS_, P_, true, false>), grid, block, sh.lds_bytes, st, segs, ranges,    \
                         order, n_ranges, qhead, tb, sh, rhdr, ru, ro, rnslots, rmore, pranges, rid_base);      \
    else                                                                                                        \
      hipLaunchKernelGGL((k_range<F, ROWS_, P_, false, false>), grid, block, sh.lds_bytes, st, segs, ranges,   \
                         order, n_ranges, qhead, tb, sh, rhdr, ru, ro, rnslots, rmore, pranges, rid_base);      \
    return hipGetLastError();                                                                                   \
  } while (0)
  // extra passes: one schedule (all waves build a tile, then walk it)
#define TT_LAUNCH_XP(F, ROWS_)                                                                                  \
  do {                                                                                                          \
    if (iv)                                                                                                     \
      hipLaunchKernelGGL((k_range<F, ROWS_, false, true, true>), grid, block, sh.lds_bytes, st, segs, ranges,  \
                         order, n_ranges, qhead, tb, sh, rhdr, ru, ro, rnslots, rmore, pranges, rid_base);      \
    else                                                                                                        \
      hipLaunchKernelGGL((k_range<F, ROWS_, false, false, true>), grid, block, sh.lds_bytes, st, segs, ranges, \
                         order, n_ranges, qhead, tb, sh, rhdr, ru, ro, rnslots, rmore, pranges, rid_base);      \
    return hipGetLastError();                                                                                   \
  } while (0)
  const bool p = sh.pipe != 0, iv = tb.iv != nullptr, xp = rid_base != 0;
  if (xp) {
    if (fmt == 1) {
      if (T == 1024) TT_LAUNCH_XP(1, 1);
      if (T == 2048) TT_LAUNCH_XP(1, 2);
      if (T == 4096) TT_LAUNCH_XP(1, 4);
    } else {
      if (T == 1024) TT_LAUNCH_XP(2, 1);
      if (T == 2048) TT_LAUNCH_XP(2, 2);
    }
    return hipErrorInvalidValue;
  }
  if (fmt == 1) {
    if (T == 1024) { if (p) TT_LAUNCH(1, 1, true); else TT_LAUNCH(1, 1, false); }
    if (T == 2048) { if (p) TT_LAUNCH(1, 2, true); else TT_LAUNCH(1, 2, false); }
    if (T == 4096) { if (p) TT_LAUNCH(1, 4, true); else TT_LAUNCH(1, 4, false); }
  } else {
    if (T == 1024) { if (p) TT_LAUNCH(2, 1, true); else TT_LAUNCH(2, 1, false); }
    if (T == 2048) { if (p) TT_LAUNCH(2, 2, true); else TT_LAUNCH(2, 2, false); }
  }
#undef TT_LAUNCH_XP
#undef TT_LAUNCH
  return hipErrorInvalidValue;
}

hipError_t launch_paylen(const Seg *segs, Range *ranges, uint32_t n_ranges, const uint32_t *seg_first_range,
                         uint32_t n_segs, const uint32_t *slice_first, uint32_t n_slices, uint64_t *paylen,
                         uint32_t *err, hipStream_t st) {
  if (!n_ranges) return hipSuccess;
  hipLaunchKernelGGL(k_slice_paylen, dim3(n_slices), dim3(WG), 0, st, segs, ranges, n_ranges, slice_first, paylen);
  hipLaunchKernelGGL(k_range_payoff, dim3(n_segs), dim3(PO_WG), 0, st, segs, seg_first_range, ranges, slice_first,
                     paylen, err);
  return hipGetLastError();
}

}  // namespace tt
