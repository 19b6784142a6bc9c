// tt_common.h -- device-side layouts shared by the library's kernels and host runtime.
//
// Everything is integer: timestamps are u64 ns, sums/min/max are u64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tt {

constexpr int WAVE = 64;
constexpr int WG = 256;              // workgroup of the helper kernels
constexpr int S_MAX = 64;            // distinct threads one range may interleave (== THAPI_MAX_RANGE_THREADS)
constexpr int TIDMAP = 256;          // LDS buckets of the tid -> local slot map (power of two)
constexpr uint32_t EMPTY32 = 0xFFFFFFFFu;
constexpr uint64_t EMPTY64 = ~0ull;
constexpr uint32_t GV_PENDING = 0xFFFFFFFFu;  // global thread map: slot id not published yet
constexpr uint32_t GV_INVALID = 0xFFFFFFFEu;  // global thread map: capacity exceeded
constexpr uint32_t KL_MAX = 256;     // kernel ids pre-aggregated in LDS; larger ids go to global atomics

// Distinct threads of one stream one range holds in one pass: their carried
// stacks live in LDS (S_MAX x 16 frames); more take extra passes.
__host__ __device__ inline uint32_t slot_cap(uint32_t D) { return D <= 16 ? (uint32_t)S_MAX : 1024u / D; }

// Per-stream counters kept on the device (indices into a [stream][ST_N] u64 array).
enum : int {
  ST_RECORDS = 0, ST_ENTRIES, ST_EXITS, ST_KERNEL, ST_ORPHAN, ST_MISMATCH, ST_NEGDUR, ST_UNDER,
  ST_TSREG, ST_UNCLOSED, ST_BAD, ST_N
};

// Error bits raised by kernels (sticky per flush).
// ERR_WIDE is not a failure: some range met more threads than it holds in
// LDS, and its other threads wait for extra passes (the combine and the final
// flush leave the flush to the host, which launches those passes).
enum : uint32_t { ERR_CAPACITY = 1u, ERR_WIDE = 2u, ERR_DEPTH = 4u, ERR_PIPE = 8u, ERR_PAYLOAD = 16u };

// One submitted chunk, as the kernels see it.
struct Seg {
  const uint8_t *rec;   // record bytes (8-byte aligned)
  const uint8_t *pay;   // VAR16 payload heap (any alignment) or null
  uint64_t n_rec;
  uint64_t pay_bytes;
  uint32_t stream;
  uint32_t pad;
};

// A contiguous run of one segment's records processed by one workgroup.
struct Range {
  uint32_t seg;
  uint32_t stream;
  uint64_t begin;       // first record (index into the segment)
  uint64_t n;           // records
  uint64_t pay_begin;   // VAR16: payload offset of `begin` within the segment (filled on device)
  uint64_t iv_base;     // intervals: first IvRec of the range (the flush's records before it)
  uint32_t pass;        // 0: the range's first pass; k > 0: an extra pass over the records of range
                        // `parent`, for the threads of the stream with ordinal in [(k-1) C, k C) that
                        // its first pass did not take (C: the threads one range holds in LDS)
  uint32_t parent;
};

// Intervals (the span from a call's entry to its exit, with its depth and
// the call that was the stack top when it was entered).
// A call matched inside a range, as the range kernel writes it: the depth
// and a parent opened before the range depend on the stack the thread
// carried into the range, which the combine finds later.  With the floor f
// (the lowest depth the range had reached, relative to its start, when the
// call was entered; -f = fneg) and the carried height h0, the call's depth
// is max(0, h0 - fneg) + dl, and without IV_PARENT_SET its parent is the
// carried frame fneg below the top, if max(0, h0 - fneg) > 0 (else none).
struct IvRec {
  uint64_t start, end, pstart;
  uint16_t fn, pfn;     // pfn / pstart: the parent, with IV_PARENT_SET
  uint8_t slot;         // range-local thread slot
  uint8_t dl;           // levels above the floor (>= 1; capped at 255)
  uint8_t fneg;         // -floor (capped at 255)
  uint8_t flags;
};
enum : uint8_t { IV_PARENT_SET = 1u };
// A call the combine closed (opened before its range): complete.
struct CIval { uint64_t start, end, pstart; uint32_t gslot, depth, fn, pfn; };
// One frame of the stack a thread carried into a range, top first.
struct IvFrame { uint64_t ts; uint32_t fn, pad; };

// Summary a range leaves for one of its threads (the boundary of the range):
// exits that closed calls opened before the range (U items, in order), the
// children time those calls accumulated inside the range, the calls still
// open at the range end (O items, bottom to top), and the depth excursion.
struct RHdr {
  uint32_t gslot;       // global thread slot
  uint32_t nu_listed;   // U items stored (<= max_depth)
  uint32_t nu_total;    // exits that found the range-local stack empty
  uint32_t n_o;         // calls open at the range end (stored: min(n_o, max_depth))
  uint64_t floor;       // children time owed to the call below the range's own entries
  int32_t H, M;         // depth excursion: max over the range of h and of (h - u)
  uint64_t first_ts, last_ts;  // first / last API timestamp of the thread in the range
  uint32_t flags;       // RF_*
  uint32_t pad;
  uint64_t pad2;
};
enum : uint32_t { RF_HAS_TS = 1u, RF_OVERFLOW = 2u };

struct UItem { uint64_t ts, child; uint32_t fn, pad; uint64_t pad2; };
struct OItem { uint64_t ts, child, bytes; uint32_t fn, pad; };

// Global tally of one (thread, fn): the fields of a result row.
struct Tally { uint64_t count, incl_sum, incl_min, incl_max, self_sum, self_min, self_max, bytes_sum; };
struct KTally { uint64_t count, sum, min, max; };

// The tables a handle resets, for the one-launch initialisation.
struct InitSet {
  uint32_t *s_nth; size_t n_s_nth;
  uint64_t *gkeys; size_t n_gkeys;
  uint32_t *gvals; size_t n_gvals;
  uint32_t *ngs, *err;
  Tally *tally; size_t n_tally;
  KTally *ktally; size_t n_ktally;
  uint32_t *cstate; size_t n_cstate;
  uint64_t *sstats; size_t n_sstats;
};

// Per-thread state carried on the device across ranges and flushes.
struct CState { uint32_t h; uint32_t flags; uint64_t last_ts; };
enum : uint32_t { CS_HAS_TS = 1u, CS_OVERFLOW = 2u };
struct Frame { uint64_t ts, child, bytes; uint32_t fn, pad; };

// Merge input (thapi_tally_merge): one thread of an exported aggregate with
// its stream mapped to this handle's index, its open calls (frames
// [frame0, frame0 + h) of the frame array), flags and last timestamp; one
// tally row of a blob thread; one kernel row of a mapped stream.
struct MThread { uint32_t stream, tid, h, flags; uint64_t last_ts; uint32_t frame0, pad; };
struct MRow { uint32_t thread, fn; Tally v; };
struct MKRow { uint32_t stream, kid; KTally v; };

// Device tables of one handle.
struct Tables {
  uint64_t *gkeys;      // thread map keys: (stream << 32) | tid, EMPTY64 = free
  uint32_t *gvals;      // thread map values: global slot
  uint32_t gmask;       // capacity - 1
  uint32_t *n_gslots;
  uint32_t max_threads;
  uint32_t *th_stream, *th_tid;
  uint32_t *th_ord;     // [max_threads] the thread's ordinal within its stream (order of registration)
  uint32_t *s_nth;      // [max_streams] threads registered per stream
  Tally *tally;         // [max_threads][n_fns]
  uint32_t n_fns;
  KTally *ktally;       // [max_streams][n_kid]
  uint32_t n_kid;
  CState *cstate;       // [max_threads]
  Frame *cstack;        // [max_threads][D]
  uint32_t D;           // max_depth
  unsigned long long *sstats;  // [max_streams][ST_N]
  uint32_t *err;
  const uint8_t *has_size;     // [n_fns] or null
  // intervals of the current flush (all null when they are not kept)
  IvRec *iv;                   // range r writes from its iv_base
  uint32_t *iv_n;              // [ranges] IvRecs written
  uint32_t *iv_h0;             // [ranges][S_MAX] carried height at the range start (combine)
  IvFrame *iv_snap;            // [ranges][S_MAX][D] that stack, top first (combine)
  CIval *civ;                  // calls closed by the combine
  uint32_t *civ_n;             // their count (zero at launch)
  uint32_t civ_cap;
  // partial tallies of the current flush: a range whose threads all have
  // direct-mapped LDS rows and stream ordinals below PART_ORDS writes its rows
  // here with plain stores ([range][ordinal][n_fns] LDS tally entries,
  // part_gslot[range][ordinal] their global slots, part_mask[range] the
  // ordinals present, 0 when the range used global atomics instead), and a
  // merge after the combine adds each row over the stream's ranges once.
  // Ranges from part_ranges on (all of them when it is 0) use the atomics.
  uint8_t *part;
  uint32_t *part_gslot;
  uint32_t *part_mask;
  uint32_t part_ranges;
};
constexpr uint32_t PART_ORDS = 16;

// Payload analytics tables (tt_payload.hip).  hs: 0 free, else stream + 1;
// hk: the slot's handle, EMPTY64 until written.
struct PayTables {
  const uint8_t *roles;        // [n_fns] 0, copy 1, create 2, release 3
  uint64_t *copies;            // [max_streams][n_fns][4] {count, bytes}
  uint64_t *hk;                // [cap] handle values
  uint32_t *hs;                // [cap] stream + 1
  uint32_t *hc, *hr;           // [cap] creates, releases
  uint32_t *hx;                // [max_streams][2] creates, releases of the handle EMPTY64
  uint64_t *hl_key;            // [hl_cap] handle records of the flush waiting to be joined
  uint32_t *hl_meta;           // [hl_cap] stream << 1 | (release)
  uint32_t *hl_n;              // their count (may exceed hl_cap: the rest were joined at once)
  uint32_t hl_cap;
  uint32_t hmask;              // cap - 1
  uint32_t n_fns;
  uint32_t n_streams;          // max_streams
  uint32_t *err;
};

// VAR16 payload offsets are found per slice of PAY_SLICE records of a range
// (slice_first[r] = the first slice of range r, a prefix over ranges).
constexpr uint32_t PAY_SLICE = 8192;
__device__ __forceinline__ uint32_t range_of_slice(const uint32_t *slice_first, uint32_t n_ranges, uint32_t b) {
  uint32_t lo = 0, hi = n_ranges - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) / 2;
    if (slice_first[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// One packed chunk of a flush (tt_payload.hip decodes them together).
struct PkChunk {
  const uint8_t *buf;        // packet bytes
  uint64_t nbytes;
  const uint64_t *index;     // packet offsets
  uint64_t pad;
};

// Launch shape of the range kernel (tile of T records, LDS tally of E entries).
struct Shape {
  uint32_t T;           // records per tile (a multiple of the range kernel's 1024 lanes)
  uint32_t E;           // LDS tally entries (power of two)
  uint32_t KL;          // kernel ids pre-aggregated in LDS (<= KL_MAX)
  uint32_t lds_bytes;
  uint32_t rpc;         // ranges per CU the records are cut into (work-list length / CUs)
  uint32_t pipe;        // 1: producer and walker waves overlap (tiles of T / 2 records)
};

__host__ __device__ inline uint32_t hash32(uint32_t x) {
  x ^= x >> 16; x *= 0x7feb352du; x ^= x >> 15; x *= 0x846ca68bu; x ^= x >> 16;
  return x;
}
__host__ __device__ inline uint64_t hash64(uint64_t x) {
  x ^= x >> 33; x *= 0xff51afd7ed558ccdull; x ^= x >> 33; x *= 0xc4ceb9fe1a85ec53ull; x ^= x >> 33;
  return x;
}

// Resolves (stream, tid) to its global thread slot, inserting it on first
// sight.  Lock-free open addressing in two phases: every lane first inserts
// or finds its key, and an inserting lane publishes the slot id before the
// probe loop ends; only after the whole wave has left that loop does a lane
// that found a key inserted elsewhere wait for its slot id.  (Waiting inside
// the probe loop could deadlock: a lane of one wave spinning on a key whose
// inserter is a masked-off lane of another spinning wave, and vice versa.)
__device__ inline uint32_t resolve_gslot(const Tables &tb, uint32_t stream, uint32_t tid) {
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
        tb.th_ord[g] = atomicAdd(&tb.s_nth[stream], 1u);
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

// The global thread slot of (stream, tid) if the thread map holds it (and
// its slot id is published), else GV_INVALID; inserts nothing.
__device__ inline uint32_t lookup_gslot(const Tables &tb, uint32_t stream, uint32_t tid) {
  const uint64_t key = ((uint64_t)stream << 32) | tid;
  uint32_t h = (uint32_t)hash64(key) & tb.gmask;
  for (uint32_t probe = 0; probe <= tb.gmask; probe++) {
    const uint64_t k = __hip_atomic_load(&tb.gkeys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (k == EMPTY64) return GV_INVALID;
    if (k == key) {
      const uint32_t v = __hip_atomic_load(&tb.gvals[h], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
      return v == GV_PENDING ? GV_INVALID : v;
    }
    h = (h + 1) & tb.gmask;
  }
  return GV_INVALID;
}

}  // namespace tt
