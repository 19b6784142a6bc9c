// tt_payload.hip -- payload work beside the tally: packed (CTF-like) chunks
// turned into the VAR16 layout, and the payload analytics of functions given
// a role (per-direction copy bytes, the create / release join by handle).
//
// Packed chunk: packets one after the other, each a 16-byte header {u32
// magic "THPK", u32 packet bytes, u32 events, u32 0} and its events, every
// event a VAR16 header with its payload inline, padded to 8 bytes.  A
// packet's events can only be found one after the other (each event's size
// is in its own header), so the packet index the caller gives (the offset of
// every packet) is what lets packets be decoded in parallel: one lane per
// packet walks its events, first to count them and the payload bytes kept,
// then (after a scan over packets) to write them out.
//
// The tally and the analytics read at most the first 24 bytes of a payload,
// and only test payload_len >= 8 and >= 24, so the VAR16 form written here
// keeps 0, 8 or 24 bytes of each payload (payload_len 0, 8 or 24 accordingly):
// every result is that of the full payloads, and the heap stays 8-byte aligned.
#include "tt_common.h"

namespace tt {

hipError_t launch_fill32(uint32_t *p, size_t n, uint32_t v, hipStream_t st);

constexpr uint32_t PACKET_MAGIC = 0x4B504854u;   // "THPK"

// Payload bytes kept for a payload of `len` bytes.
__device__ __forceinline__ uint32_t kept_len(uint32_t len) { return len >= 24 ? 24u : (len >= 8 ? 8u : 0u); }

typedef const __attribute__((address_space(1))) uint64_t gq64;

// Decode: one lane per packet, every packed chunk of a flush in one launch
// (packet k of the flush belongs to the chunk j with first[j] <= k <
// first[j + 1]).  A packet's events form a chain (each header gives the next
// one's offset), so a lane walks it; many packets in flight hide the latency
// of each step, and the bytes a lane reads next usually share the cache line
// of the bytes it has just read.
// Lane l's value of x, as a scalar.  (readlane returns a signed int: each
// half goes through uint32_t so that the low one is not sign-extended.)
__device__ __forceinline__ uint64_t uni_lane64(uint64_t x, uint32_t l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)x, (int32_t)l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)(x >> 32), (int32_t)l);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t chunk_of(const uint64_t *first, uint32_t nc, uint64_t k) {
  uint32_t lo = 0, hi = nc - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) / 2;
    if (first[mid] <= k) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Count pass: ev[k] = events of packet k, pay[k] = its kept payload bytes
// (both 0, and ERR_PAYLOAD raised, when it is malformed).
__global__ __launch_bounds__(256) void k_pk_count(const PkChunk *__restrict__ chunks, const uint64_t *__restrict__ first,
                                                  uint32_t nc, uint32_t *ev, uint64_t *pay, uint32_t *err) {
  const uint64_t n = first[nc];
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t j = chunk_of(first, nc, k);
    const PkChunk c = chunks[j];
    const uint64_t kk = k - first[j], npk = first[j + 1] - first[j];
    const uint64_t off = c.index[kk];
    bool ok = off % 8 == 0 && off + 16 <= c.nbytes && (kk != 0 || off == 0);
    uint32_t pbytes = 0, pev = 0;
    gq64 *p = (gq64 *)(c.buf + (ok ? off : 0));
    if (ok) {
      const uint64_t h0 = p[0], h1 = p[1];
      pbytes = (uint32_t)(h0 >> 32);
      pev = (uint32_t)h1;
      const uint64_t next = kk + 1 < npk ? c.index[kk + 1] : c.nbytes;
      ok = (uint32_t)h0 == PACKET_MAGIC && !(h1 >> 32) && pbytes >= 16 && pbytes % 8 == 0 &&
           off + pbytes <= c.nbytes && next == off + pbytes;
    }
    const uint32_t pw = pbytes / 8;
    uint32_t o = 2;          // next event, in words
    uint64_t kept = 0;
    for (uint32_t e = 0; ok && e < pev; e++) {
      if (o + 2 > pw) { ok = false; break; }
      const uint32_t len = (uint32_t)(p[o + 1] >> 56);
      const uint32_t words = 2 + (len + 7) / 8;
      if (o + words > pw) { ok = false; break; }
      kept += kept_len(len);
      o += words;
    }
    ok = ok && o == pw;
    ev[k] = ok ? pev : 0;
    pay[k] = ok ? kept : 0;
    if (!ok) atomicOr(err, ERR_PAYLOAD);
  }
}

// Write pass (after the count pass found every packet well formed and the
// scan turned the counts into offsets): each wave takes 64 consecutive
// packets, one per lane.  In turns, every lane walks up to PKE_BATCH more
// events of its packet and notes where they start (LDS, as 16-bit word
// offsets from the turn's first event: a turn spans at most 64 events of at
// most 34 words); then the wave copies the noted events packet by packet, one
// event per lane, so that the headers and kept payload words of a packet are
// written by consecutive lanes to consecutive addresses.
constexpr uint32_t PKE_WAVES = 4;
constexpr uint32_t PKE_BATCH = WAVE;
__global__ __launch_bounds__(PKE_WAVES * WAVE) void k_pk_emit(const PkChunk *__restrict__ chunks,
                                                              const uint64_t *__restrict__ first, uint32_t nc,
                                                              const uint64_t *__restrict__ ev_off,
                                                              const uint64_t *__restrict__ pay_off, uint64_t *hdr,
                                                              uint64_t *heap) {
  __shared__ uint16_t pos[PKE_WAVES][WAVE][PKE_BATCH];
  const uint32_t lane = threadIdx.x & (WAVE - 1);
  const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const uint64_t n = first[nc];
  const uint64_t k0 = ((uint64_t)blockIdx.x * PKE_WAVES + wv) * WAVE;
  if (k0 >= n) return;
  const uint64_t k = k0 + lane;
  const bool in = k < n;
  // this lane's packet
  gq64 *p = nullptr;
  uint32_t pev = 0;
  uint64_t eb = 0, hb = 0;   // next event's index, next kept payload byte
  if (in) {
    const uint32_t j = chunk_of(first, nc, k);
    const PkChunk c = chunks[j];
    p = (gq64 *)(c.buf + c.index[k - first[j]]);
    pev = (uint32_t)p[1];
    eb = ev_off[k];
    hb = pay_off[k];
  }
  uint32_t o = 2, e = 0;
  for (;;) {
    // walk: up to PKE_BATCH events of this lane's packet
    const uint32_t o0 = o;   // (this turn's first event)
    uint32_t m = 0;
    while (m < PKE_BATCH && e + m < pev) {
      pos[wv][lane][m] = (uint16_t)(o - o0);
      const uint32_t len = (uint32_t)(p[o + 1] >> 56);
      o += 2 + (len + 7) / 8;
      m++;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // copy: packet by packet, one event per lane
    uint64_t more = __ballot(m != 0);
    while (more) {
      const uint32_t l = (uint32_t)__builtin_ctzll(more);
      more &= more - 1;
      const uint32_t ml = __builtin_amdgcn_readlane(m, l);
      const uint64_t pl = uni_lane64((uint64_t)(uintptr_t)p, l), ebl = uni_lane64(eb, l), hbl = uni_lane64(hb, l);
      gq64 *pp = (gq64 *)(uintptr_t)pl + (uint32_t)__builtin_amdgcn_readlane((int32_t)o0, (int32_t)l);
      uint32_t kl = 0;
      uint64_t w0 = 0, w1 = 0, x0 = 0, x1 = 0, x2 = 0;
      if (lane < ml) {
        const uint32_t q = pos[wv][l][lane];
        w0 = pp[q];
        w1 = pp[q + 1];
        kl = kept_len((uint32_t)(w1 >> 56));
        // (the kept words lie inside the event: its payload has kl bytes or more)
        if (kl >= 8) x0 = pp[q + 2];
        if (kl == 24) { x1 = pp[q + 3]; x2 = pp[q + 4]; }
      }
      uint32_t inc = kl;
      for (uint32_t d = 1; d < WAVE; d <<= 1) {
        const uint32_t t = __shfl_up(inc, d, WAVE);
        if (lane >= d) inc += t;
      }
      const uint32_t tot = __shfl(inc, WAVE - 1, WAVE);
      if (lane < ml) {
        uint64_t *hd = hdr + 2 * (ebl + lane);
        hd[0] = w0;
        hd[1] = (w1 & 0x00FFFFFFFFFFFFFFull) | ((uint64_t)kl << 56);
        uint64_t *hp = heap + (hbl + inc - kl) / 8;
        if (kl >= 8) hp[0] = x0;
        if (kl == 24) { hp[1] = x1; hp[2] = x2; }
      }
      if (lane == l) { eb += ml; hb += tot; }
    }
    e += m;
    if (!__ballot(e < pev)) break;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// Exclusive prefix sums of (ev, pay) over n packets in three launches: tile
// totals, a scan of the tile totals (one workgroup), and each tile rescanned
// from its offset.  Tiles of SC_TILE packets, SC_ITEMS consecutive ones per
// lane.
constexpr uint32_t SC_WG = 256, SC_ITEMS = 8, SC_TILE = SC_WG * SC_ITEMS;

// Block-wide exclusive scan of one u64 per lane; returns the block total too.
__device__ inline uint64_t block_excl(uint64_t v, uint64_t *ws, uint64_t *total) {
  const uint32_t lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  uint64_t inc = v;
  for (uint32_t d = 1; d < WAVE; d <<= 1) {
    const uint64_t t = __shfl_up(inc, d, WAVE);
    if (lane >= d) inc += t;
  }
  if (lane == WAVE - 1) ws[w] = inc;
  __syncthreads();
  uint64_t before = 0, tot = 0;
  for (uint32_t k = 0; k < SC_WG / WAVE; k++) { before += k < w ? ws[k] : 0; tot += ws[k]; }
  __syncthreads();
  *total = tot;
  return before + inc - v;
}

__global__ __launch_bounds__(SC_WG) void k_pk_scan_tiles(const uint32_t *ev, const uint64_t *pay, uint64_t n,
                                                         uint64_t *tev, uint64_t *tpay) {
  __shared__ uint64_t ws[SC_WG / WAVE];
  const uint64_t b = (uint64_t)blockIdx.x * SC_TILE + (uint64_t)threadIdx.x * SC_ITEMS;
  uint64_t a = 0, c = 0;
  for (uint32_t i = 0; i < SC_ITEMS; i++)
    if (b + i < n) { a += ev[b + i]; c += pay[b + i]; }
  uint64_t ta, tc;
  block_excl(a, ws, &ta);
  block_excl(c, ws, &tc);
  if (threadIdx.x == 0) { tev[blockIdx.x] = ta; tpay[blockIdx.x] = tc; }
}

// In place over the nt tile totals; tot[0], tot[1] = the grand totals.
__global__ __launch_bounds__(SC_WG) void k_pk_scan_top(uint64_t *tev, uint64_t *tpay, uint64_t nt, uint64_t *tot) {
  __shared__ uint64_t ws[SC_WG / WAVE];
  uint64_t ra = 0, rc = 0;
  for (uint64_t b = 0; b < nt; b += SC_WG) {
    const uint64_t i = b + threadIdx.x;
    const uint64_t a = i < nt ? tev[i] : 0, c = i < nt ? tpay[i] : 0;
    uint64_t ta, tc;
    const uint64_t xa = block_excl(a, ws, &ta), xc = block_excl(c, ws, &tc);
    if (i < nt) { tev[i] = ra + xa; tpay[i] = rc + xc; }
    ra += ta;
    rc += tc;
  }
  if (threadIdx.x == 0) { tot[0] = ra; tot[1] = rc; }
}

// ev_off[k] = events before packet k; pay[k] (in place) = kept payload bytes before it.
__global__ __launch_bounds__(SC_WG) void k_pk_scan_down(const uint32_t *ev, uint64_t *pay, uint64_t n,
                                                        const uint64_t *tev, const uint64_t *tpay, uint64_t *ev_off) {
  __shared__ uint64_t ws[SC_WG / WAVE];
  const uint64_t b = (uint64_t)blockIdx.x * SC_TILE + (uint64_t)threadIdx.x * SC_ITEMS;
  uint32_t e[SC_ITEMS];
  uint64_t q[SC_ITEMS];
  uint64_t a = 0, c = 0;
  for (uint32_t i = 0; i < SC_ITEMS; i++) {
    e[i] = b + i < n ? ev[b + i] : 0;
    q[i] = b + i < n ? pay[b + i] : 0;
    a += e[i];
    c += q[i];
  }
  uint64_t ta, tc;
  uint64_t ra = tev[blockIdx.x] + block_excl(a, ws, &ta);
  uint64_t rc = tpay[blockIdx.x] + block_excl(c, ws, &tc);
  for (uint32_t i = 0; i < SC_ITEMS; i++)
    if (b + i < n) {
      ev_off[b + i] = ra;
      pay[b + i] = rc;
      ra += e[i];
      rc += q[i];
    }
}

// out[2 j], out[2 j + 1] = events and kept bytes before chunk j's first packet
// (j < nc); out[2 nc], out[2 nc + 1] = the totals.
__global__ void k_pk_gather(const uint64_t *first, uint32_t nc, const uint64_t *ev_off, const uint64_t *pay,
                            const uint64_t *tot, uint64_t *out) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < nc) { out[2 * j] = ev_off[first[j]]; out[2 * j + 1] = pay[first[j]]; }
  else if (j == nc) { out[2 * j] = tot[0]; out[2 * j + 1] = tot[1]; }
}

// ------------------------------------------------------- payload analytics
// Handle table: open addressing on (stream, handle).  hs[i]: 0 free, else
// stream + 1, set by the compare-and-swap that claims the slot; hk[i]: the
// handle, EMPTY64 until the claiming lane writes it (it does so right after
// its claim, in the same straight-line code).  Every word is read and
// written with device-scope atomics and no ordering is relied on between
// the two words: a lane that finds its stream in a slot whose key still
// reads EMPTY64 notes the slot and, once it has left its probe loop (so that
// the writer, which may be a lane of its own wave, has gone on), waits for
// the key, then looks again.  The one handle value equal to EMPTY64 is
// counted per stream beside the table (hx).
enum : uint8_t { ROLE_COPY = 1, ROLE_CREATE = 2, ROLE_RELEASE = 3 };

__device__ inline uint64_t pay_u64(const uint8_t *base, uint64_t off) {
  const uintptr_t a = (uintptr_t)(base + off);
  gq64 *p = (gq64 *)(a & ~(uintptr_t)7);
  const uint32_t sh = (uint32_t)(a & 7) * 8;
  const uint64_t lo = p[0];
  if (sh == 0) return lo;
  return (lo >> sh) | (p[1] << (64 - sh));
}

__device__ __forceinline__ uint64_t ld_key(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The slot of (s, h), h != EMPTY64, inserted on first sight; EMPTY32 when
// the table is full.
__device__ inline uint32_t handle_slot(const PayTables &pt, uint32_t s, uint64_t h) {
  uint32_t i = (uint32_t)hash64(h ^ ((uint64_t)s * 0x9E3779B97F4A7C15ull)) & pt.hmask;
  const uint32_t mine = s + 1;
  uint32_t probe = 0;
  for (;;) {
    uint32_t pending = EMPTY32;
    for (; probe <= pt.hmask; probe++, i = (i + 1) & pt.hmask) {
      uint32_t v = __hip_atomic_load(&pt.hs[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (v == 0) {
        v = atomicCAS(&pt.hs[i], 0u, mine);
        if (v == 0) {
          __hip_atomic_store(&pt.hk[i], h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          return i;
        }
      }
      if (v != mine) continue;
      const uint64_t k = ld_key(&pt.hk[i]);
      if (k == h) return i;
      if (k == EMPTY64) { pending = i; break; }   // claimed for this stream, key not visible yet
    }
    if (pending == EMPTY32) return EMPTY32;      // every slot holds another key
    while (ld_key(&pt.hk[pending]) == EMPTY64) __builtin_amdgcn_s_sleep(1);
  }
}

// Adds one create (release false) or release of handle h in stream s.
__device__ inline void handle_add(const PayTables &pt, uint32_t s, uint64_t h, bool release) {
  if (h == EMPTY64) {
    atomicAdd(&pt.hx[2 * s + (release ? 1 : 0)], 1u);
    return;
  }
  const uint32_t k = handle_slot(pt, s, h);
  if (k == EMPTY32) atomicOr(pt.err, ERR_CAPACITY);
  else atomicAdd(release ? &pt.hr[k] : &pt.hc[k], 1u);
}

// One workgroup per slice of PAY_SLICE records of a range (sliceoff[b]: the
// payload offset of slice b), PA_ITEMS consecutive records per lane and
// step: each record's payload offset is the running sum of payload_len, and
// every record of a function with a role adds to the copy table or the
// handle join.  Copies of functions below PA_LDS_FNS are summed in LDS over
// the slice (its records all belong to one stream) and added to the device
// table once per workgroup: a few functions carry most copies, and device-wide atomics on
// their few counters would serialise.  Handle records are listed in LDS and
// moved to the device list (one atomic per move); k_handle_list joins them
// one thread each, so that this streaming loop never waits on the table.
// Records that find the device list full are joined here.
constexpr uint32_t PA_WG = 256;
constexpr uint32_t PA_ITEMS = 4;
constexpr uint32_t PA_LDS_FNS = 512;
constexpr uint32_t PA_MOVE = 256;                       // move the LDS list once it holds more
constexpr uint32_t PA_LIST = PA_MOVE + PA_WG * PA_ITEMS;

__device__ inline void move_list(const PayTables &pt, uint32_t stream, const uint64_t *lk, const uint8_t *lr,
                                 uint32_t n, uint32_t *base) {
  if (threadIdx.x == 0) *base = atomicAdd(pt.hl_n, n);
  __syncthreads();
  const uint32_t b = *base;
  for (uint32_t i = threadIdx.x; i < n; i += PA_WG) {
    const uint64_t at = (uint64_t)b + i;
    if (at < pt.hl_cap) {
      pt.hl_key[at] = lk[i];
      pt.hl_meta[at] = stream << 1 | lr[i];
    } else {
      handle_add(pt, stream, lk[i], lr[i] != 0);
    }
  }
}

__global__ __launch_bounds__(PA_WG) void k_payload(const Seg *__restrict__ segs, const Range *__restrict__ ranges,
                                                   uint32_t n_ranges, const uint32_t *__restrict__ slice_first,
                                                   const uint64_t *__restrict__ sliceoff, PayTables pt) {
  extern __shared__ unsigned long long ctab[];     // [min(n_fns, PA_LDS_FNS)][4 directions] {count, bytes}
  __shared__ uint64_t wsum[PA_WG / WAVE];
  __shared__ uint64_t lk[PA_LIST];
  __shared__ uint8_t lr[PA_LIST];
  __shared__ uint32_t ln, lbase;
  __shared__ uint64_t run;
  const uint32_t r = range_of_slice(slice_first, n_ranges, blockIdx.x);
  const Range rg = ranges[r];
  const Seg sg = segs[rg.seg];
  const uint64_t lo = (uint64_t)(blockIdx.x - slice_first[r]) * PAY_SLICE;
  const uint64_t nrec = rg.n - lo < PAY_SLICE ? rg.n - lo : PAY_SLICE;
  const uint32_t lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  const uint32_t nl = (pt.n_fns < PA_LDS_FNS ? pt.n_fns : PA_LDS_FNS) * 8;
  for (uint32_t k = threadIdx.x; k < nl; k += PA_WG) ctab[k] = 0;
  if (threadIdx.x == 0) { run = sliceoff[blockIdx.x]; ln = 0; }
  __syncthreads();
  gq64 *hw = (gq64 *)(sg.rec + (rg.begin + lo) * 16);
  for (uint64_t c0 = 0; c0 < nrec; c0 += PA_WG * PA_ITEMS) {
    const uint64_t i0 = c0 + (uint64_t)threadIdx.x * PA_ITEMS;
    uint64_t w1[PA_ITEMS];
    uint32_t mine = 0;
#pragma unroll
    for (uint32_t q = 0; q < PA_ITEMS; q++) {
      w1[q] = i0 + q < nrec ? hw[2 * (i0 + q) + 1] : 0;
      mine += (uint32_t)(w1[q] >> 56);
    }
    // exclusive prefix of payload_len over the step's records
    uint32_t incl = mine;
    for (uint32_t d = 1; d < WAVE; d <<= 1) {
      const uint32_t t = __shfl_up(incl, d, WAVE);
      if (lane >= d) incl += t;
    }
    if (lane == WAVE - 1) wsum[w] = incl;
    __syncthreads();
    uint64_t before = 0, total = 0;
    for (uint32_t k = 0; k < PA_WG / WAVE; k++) { before += k < w ? wsum[k] : 0; total += wsum[k]; }
    uint64_t poff = run + before + incl - mine;
#pragma unroll
    for (uint32_t q = 0; q < PA_ITEMS; q++) {
      const uint32_t len = (uint32_t)(w1[q] >> 56);
      const uint32_t fn = (uint32_t)(w1[q] >> 32) & 0xFFFFu, kind = (uint32_t)(w1[q] >> 48) & 0xFFu;
      const uint8_t role = i0 + q < nrec && kind <= 1 && fn < pt.n_fns ? pt.roles[fn] : 0;
      // (a chunk whose payload_len sum disagrees with its heap fails the
      // flush; nothing is read outside the heap meanwhile)
      if (role == ROLE_COPY && kind == 0 && len >= 24 && poff + 24 <= sg.pay_bytes) {
        const uint64_t size = pay_u64(sg.pay, poff), dst = pay_u64(sg.pay, poff + 8);
        const uint64_t src = pay_u64(sg.pay, poff + 16);
        const uint32_t dir = ((src >> 56) == 0xFF ? 2u : 0u) + ((dst >> 56) == 0xFF ? 1u : 0u);
        if (fn < PA_LDS_FNS) {
          atomicAdd(&ctab[(fn * 4 + dir) * 2], 1ull);
          atomicAdd(&ctab[(fn * 4 + dir) * 2 + 1], (unsigned long long)size);
        } else {
          uint64_t *c = pt.copies + (((size_t)sg.stream * pt.n_fns + fn) * 4 + dir) * 2;
          atomicAdd((unsigned long long *)&c[0], 1ull);
          atomicAdd((unsigned long long *)&c[1], (unsigned long long)size);
        }
      } else if (((role == ROLE_CREATE && kind == 1) || (role == ROLE_RELEASE && kind == 0)) && len >= 8 &&
                 poff + 8 <= sg.pay_bytes) {
        const uint32_t at = atomicAdd(&ln, 1u);   // < PA_LIST: at most PA_MOVE entries carried in
        lk[at] = pay_u64(sg.pay, poff);
        lr[at] = role == ROLE_RELEASE ? 1 : 0;
      }
      poff += len;
    }
    __syncthreads();
    const uint32_t n_list = ln;
    if (n_list > PA_MOVE) {
      move_list(pt, sg.stream, lk, lr, n_list, &lbase);
      __syncthreads();
      if (threadIdx.x == 0) ln = 0;
    }
    if (threadIdx.x == 0) run += total;
    __syncthreads();
  }
  if (ln) move_list(pt, sg.stream, lk, lr, ln, &lbase);
  uint64_t *cs = pt.copies + (size_t)sg.stream * pt.n_fns * 8;
  for (uint32_t k = threadIdx.x; k < nl; k += PA_WG) {
    const unsigned long long v = ctab[k];
    if (v) atomicAdd((unsigned long long *)&cs[k], v);
  }
}

// The listed handle records, one thread each (grid-stride over the count).
__global__ __launch_bounds__(256) void k_handle_list(PayTables pt) {
  const uint32_t n = *pt.hl_n < pt.hl_cap ? *pt.hl_n : pt.hl_cap;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t m = pt.hl_meta[i];
    handle_add(pt, m >> 1, pt.hl_key[i], (m & 1) != 0);
  }
}

// Per-stream join results: out[s * 5 + {0..4}] += creates, releases,
// distinct handles, unreleased (creates - releases when positive), releases
// that match no create (releases - creates when positive), over the table
// and the EMPTY64 counters (indices past the table).  Streams below
// HS_LDS_STREAMS are summed in LDS per workgroup first.
constexpr uint32_t HS_LDS_STREAMS = 128;
__global__ __launch_bounds__(256) void k_handle_stats(PayTables pt, unsigned long long *out, uint32_t ns) {
  __shared__ unsigned long long acc[HS_LDS_STREAMS * 5];
  const uint32_t nls = ns < HS_LDS_STREAMS ? ns : HS_LDS_STREAMS;
  for (uint32_t k = threadIdx.x; k < nls * 5; k += blockDim.x) acc[k] = 0;
  __syncthreads();
  const uint64_t n = (uint64_t)pt.hmask + 1 + ns;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t s, c, r;
    if (i <= pt.hmask) {
      const uint32_t v = pt.hs[i];
      if (!v) continue;
      s = v - 1;
      c = pt.hc[i];
      r = pt.hr[i];
    } else {
      s = (uint32_t)(i - pt.hmask - 1);
      c = pt.hx[2 * s];
      r = pt.hx[2 * s + 1];
      if (!c && !r) continue;
    }
    unsigned long long *o = s < nls ? &acc[s * 5] : out + (size_t)s * 5;
    atomicAdd(&o[0], (unsigned long long)c);
    atomicAdd(&o[1], (unsigned long long)r);
    atomicAdd(&o[2], 1ull);
    if (c > r) atomicAdd(&o[3], (unsigned long long)(c - r));
    else if (r > c) atomicAdd(&o[4], (unsigned long long)(r - c));
  }
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < nls * 5; k += blockDim.x)
    if (acc[k]) atomicAdd(&out[k], acc[k]);
}

// --------------------------------------------------------------- launchers
// The packed decode of nc chunks (descriptors and packet prefix `first`,
// nc + 1 entries, on the device; np packets in all).  scr: scratch of
// pk_scratch_bytes(np) bytes.  Count pass, scan and gather; `tot_out` (2 nc +
// 2 u64 on the device) receives the per-chunk offsets and totals.
size_t pk_scratch_bytes(uint64_t np) {
  const uint64_t nt = (np + SC_TILE - 1) / SC_TILE;
  auto al = [](uint64_t x) { return (x + 255) & ~(uint64_t)255; };
  return al(4 * np) + al(8 * np) + al(8 * np) + 2 * al(8 * nt) + al(16);
}
struct PkScr {
  uint32_t *ev;
  uint64_t *pay, *evoff, *tev, *tpay, *tot;
};
static PkScr pk_views(uint8_t *scr, uint64_t np) {
  const uint64_t nt = (np + SC_TILE - 1) / SC_TILE;
  auto al = [](uint64_t x) { return (x + 255) & ~(uint64_t)255; };
  PkScr v;
  v.ev = (uint32_t *)scr;
  scr += al(4 * np);
  v.pay = (uint64_t *)scr;
  scr += al(8 * np);
  v.evoff = (uint64_t *)scr;
  scr += al(8 * np);
  v.tev = (uint64_t *)scr;
  scr += al(8 * nt);
  v.tpay = (uint64_t *)scr;
  scr += al(8 * nt);
  v.tot = (uint64_t *)scr;
  return v;
}
// The count pass's workgroups each reserve 48 KiB of LDS they do not use: at
// most three are resident per CU, so fewer lanes walk at once and each lane's
// current cache line stays in L2 until it reaches its next event (with 32
// waves per CU the lines are evicted and fetched again: 5.9 GB read for a
// 2.6 GB input; measured 0.82 ms with no reservation, 0.63 ms with 32 KiB,
// 0.57 ms with 48 KiB).  The emit pass's own 32 KiB of event positions
// already limit it.
constexpr uint32_t PKC_RESERVED_LDS = 48u << 10;
static uint32_t pk_blocks(uint64_t np) {
  const uint64_t want = (np + 255) / 256;
  return (uint32_t)(want < 256u * 64u ? want : 256u * 64u);
}
hipError_t launch_pk_count(const PkChunk *chunks, const uint64_t *first, uint32_t nc, uint64_t np, uint8_t *scr,
                           uint64_t *tot_out, uint32_t *err, hipStream_t st) {
  if (!np) return hipSuccess;
  const PkScr v = pk_views(scr, np);
  const uint64_t nt = (np + SC_TILE - 1) / SC_TILE;
  hipLaunchKernelGGL(k_pk_count, dim3(pk_blocks(np)), dim3(256), PKC_RESERVED_LDS, st, chunks, first, nc, v.ev, v.pay,
                     err);
  hipLaunchKernelGGL(k_pk_scan_tiles, dim3((uint32_t)nt), dim3(SC_WG), 0, st, v.ev, v.pay, np, v.tev, v.tpay);
  hipLaunchKernelGGL(k_pk_scan_top, dim3(1), dim3(SC_WG), 0, st, v.tev, v.tpay, nt, v.tot);
  hipLaunchKernelGGL(k_pk_scan_down, dim3((uint32_t)nt), dim3(SC_WG), 0, st, v.ev, v.pay, np, v.tev, v.tpay,
                     v.evoff);
  hipLaunchKernelGGL(k_pk_gather, dim3((nc + 256) / 256), dim3(256), 0, st, first, nc, v.evoff, v.pay, v.tot,
                     tot_out);
  return hipGetLastError();
}
hipError_t launch_pk_write(const PkChunk *chunks, const uint64_t *first, uint32_t nc, uint64_t np, uint8_t *scr,
                           uint64_t *hdr, uint64_t *heap, uint32_t *err, hipStream_t st) {
  if (!np) return hipSuccess;
  const PkScr v = pk_views(scr, np);
  const uint64_t waves = (np + WAVE - 1) / WAVE;
  hipLaunchKernelGGL(k_pk_emit, dim3((uint32_t)((waves + PKE_WAVES - 1) / PKE_WAVES)), dim3(PKE_WAVES * WAVE),
                     0, st,
                     chunks, first, nc, (const uint64_t *)v.evoff, (const uint64_t *)v.pay, hdr, heap);
  return hipGetLastError();
}
hipError_t launch_payload(const Seg *segs, const Range *ranges, uint32_t n_ranges, const uint32_t *slice_first,
                          uint32_t n_slices, const uint64_t *sliceoff, const PayTables &pt, hipStream_t st) {
  if (!n_ranges) return hipSuccess;
  const uint32_t nl = pt.n_fns < PA_LDS_FNS ? pt.n_fns : PA_LDS_FNS;
  hipError_t e = launch_fill32(pt.hl_n, 1, 0, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_payload, dim3(n_slices), dim3(PA_WG), 64 * nl, st, segs, ranges, n_ranges, slice_first,
                     sliceoff, pt);
  const uint32_t want = (pt.hl_cap + 255) / 256;
  hipLaunchKernelGGL(k_handle_list, dim3(want < 2048 ? want : 2048), dim3(256), 0, st, pt);
  return hipGetLastError();
}
hipError_t launch_handle_stats(const PayTables &pt, unsigned long long *out, uint32_t ns, hipStream_t st) {
  const uint64_t n = (uint64_t)pt.hmask + 1 + ns;
  const uint64_t want = (n + 255) / 256;
  hipLaunchKernelGGL(k_handle_stats, dim3((uint32_t)(want < 1024 ? want : 1024)), dim3(256), 0, st, pt, out, ns);
  return hipGetLastError();
}

}  // namespace tt
