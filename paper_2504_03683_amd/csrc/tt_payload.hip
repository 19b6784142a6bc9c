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

constexpr uint32_t PACKET_MAGIC = 0x4B504854u;   // "THPK"
constexpr uint32_t PK_WG = 256;

// Payload bytes kept for a payload of `len` bytes.
__device__ __forceinline__ uint32_t kept_len(uint32_t len) { return len >= 24 ? 24u : (len >= 8 ? 8u : 0u); }

typedef const __attribute__((address_space(1))) uint64_t gq64;

// Walks one packet; returns false when it is malformed.  With `hdr` set,
// writes its events' headers (payload_len replaced by the kept length) and
// kept payload words.
__device__ inline bool walk_packet(const uint8_t *buf, uint64_t nbytes, const uint64_t *index, uint32_t n_packets,
                                   uint32_t k, uint32_t *n_ev, uint64_t *n_pay, uint64_t *hdr, uint64_t *heap) {
  const uint64_t off = index[k];
  if (off % 8 || off + 16 > nbytes || (k == 0 && off != 0)) return false;
  gq64 *p = (gq64 *)(buf + off);
  const uint64_t h0 = p[0], h1 = p[1];
  const uint32_t magic = (uint32_t)h0, pbytes = (uint32_t)(h0 >> 32), pev = (uint32_t)h1;
  if (magic != PACKET_MAGIC || (h1 >> 32) || pbytes < 16 || pbytes % 8 || off + pbytes > nbytes) return false;
  const uint64_t next = k + 1 < n_packets ? index[k + 1] : nbytes;
  if (next != off + pbytes) return false;
  uint64_t o = 2;          // in words
  const uint64_t end = pbytes / 8;
  uint64_t pay = 0;
  for (uint32_t e = 0; e < pev; e++) {
    if (o + 2 > end) return false;
    const uint64_t w0 = p[o], w1 = p[o + 1];
    const uint32_t len = (uint32_t)(w1 >> 56);
    const uint64_t words = 2 + (len + 7) / 8;
    if (o + words > end) return false;
    const uint32_t kl = kept_len(len);
    if (hdr) {
      hdr[2 * e] = w0;
      hdr[2 * e + 1] = (w1 & 0x00FFFFFFFFFFFFFFull) | ((uint64_t)kl << 56);
      for (uint32_t j = 0; j < kl / 8; j++) heap[pay / 8 + j] = p[o + 2 + j];
    }
    pay += kl;
    o += words;
  }
  if (o != end) return false;
  *n_ev = pev;
  *n_pay = pay;
  return true;
}

// Pass 1: events and kept payload bytes of every packet.
__global__ __launch_bounds__(PK_WG) void k_pk_count(const uint8_t *buf, uint64_t nbytes, const uint64_t *index,
                                                    uint32_t n_packets, uint32_t *ev, uint64_t *pay, uint32_t *err) {
  const uint32_t k = blockIdx.x * PK_WG + threadIdx.x;
  if (k >= n_packets) return;
  uint32_t e = 0;
  uint64_t b = 0;
  if (!walk_packet(buf, nbytes, index, n_packets, k, &e, &b, nullptr, nullptr)) {
    atomicOr(err, ERR_PAYLOAD);
    e = 0;
    b = 0;
  }
  ev[k] = e;
  pay[k] = b;
}

// Exclusive prefix sums of the per-packet counts (one workgroup: each lane
// sums a contiguous share, the shares are scanned, then each lane writes its
// share's prefixes); the totals go to tot[0] (events) and tot[1] (bytes).
__global__ __launch_bounds__(1024) void k_pk_scan(uint32_t *ev, uint64_t *pay, uint32_t n, uint64_t *ev_off,
                                                  uint64_t *tot) {
  __shared__ uint64_t se[1024], sp[1024];
  const uint32_t t = threadIdx.x;
  const uint32_t share = (n + 1023) / 1024, lo = t * share, hi = lo + share < n ? lo + share : n;
  uint64_t a = 0, b = 0;
  for (uint32_t i = lo; i < hi; i++) { a += ev[i]; b += pay[i]; }
  se[t] = a;
  sp[t] = b;
  __syncthreads();
  for (uint32_t s = 1; s < 1024; s <<= 1) {
    const uint64_t x = t >= s ? se[t - s] : 0, y = t >= s ? sp[t - s] : 0;
    __syncthreads();
    se[t] += x;
    sp[t] += y;
    __syncthreads();
  }
  uint64_t ra = se[t] - a, rb = sp[t] - b;
  for (uint32_t i = lo; i < hi; i++) {
    const uint64_t x = ev[i], y = pay[i];
    ev_off[i] = ra;
    pay[i] = rb;   // (in place: the byte offset of the packet's kept payload)
    ra += x;
    rb += y;
  }
  if (t == 1023) { tot[0] = se[1023]; tot[1] = sp[1023]; }
}

// Pass 2: headers and kept payload words of every packet, at its offsets.
__global__ __launch_bounds__(PK_WG) void k_pk_write(const uint8_t *buf, uint64_t nbytes, const uint64_t *index,
                                                    uint32_t n_packets, const uint64_t *ev_off,
                                                    const uint64_t *pay_off, uint64_t *hdr, uint64_t *heap,
                                                    uint32_t *err) {
  const uint32_t k = blockIdx.x * PK_WG + threadIdx.x;
  if (k >= n_packets) return;
  uint32_t e = 0;
  uint64_t b = 0;
  if (!walk_packet(buf, nbytes, index, n_packets, k, &e, &b, hdr + 2 * ev_off[k], heap + pay_off[k] / 8))
    atomicOr(err, ERR_PAYLOAD);
}

// ------------------------------------------------------- payload analytics
// Handle table: open addressing on (stream, handle).  hs: 0 free, s + 1
// (stream s) once the slot's handle is written, CLAIM | (s + 1) while a lane
// writes it.  A lane never waits for another inside its probe loop (a lane
// of its own wave could be the writer, masked off meanwhile); it notes the
// slot and waits after the loop, when every lane of the wave has left it.
constexpr uint32_t HS_CLAIM = 0x80000000u;

enum : uint8_t { ROLE_COPY = 1, ROLE_CREATE = 2, ROLE_RELEASE = 3 };

__device__ inline uint64_t pay_u64(const uint8_t *base, uint64_t off) {
  const uintptr_t a = (uintptr_t)(base + off);
  gq64 *p = (gq64 *)(a & ~(uintptr_t)7);
  const uint32_t sh = (uint32_t)(a & 7) * 8;
  const uint64_t lo = p[0];
  if (sh == 0) return lo;
  return (lo >> sh) | (p[1] << (64 - sh));
}

// The slot of (s, h), inserted on first sight; EMPTY32 when the table is full.
__device__ inline uint32_t handle_slot(const PayTables &pt, uint32_t s, uint64_t h) {
  uint32_t i = (uint32_t)hash64(h ^ ((uint64_t)s * 0x9E3779B97F4A7C15ull)) & pt.hmask;
  const uint32_t mine = s + 1;
  uint32_t probe = 0;
  for (;;) {
    // phase 1: find or claim, never waiting for another lane
    uint32_t pending = EMPTY32;
    for (; probe <= pt.hmask; probe++, i = (i + 1) & pt.hmask) {
      uint32_t v = __hip_atomic_load(&pt.hs[i], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
      if (v == 0) {
        v = atomicCAS(&pt.hs[i], 0u, HS_CLAIM | mine);
        if (v == 0) {
          pt.hk[i] = h;
          __hip_atomic_store(&pt.hs[i], mine, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
          return i;
        }
      }
      if (v == mine) {
        if (pt.hk[i] == h) return i;
        continue;
      }
      if (v == (HS_CLAIM | mine)) { pending = i; break; }   // its handle is not written yet
    }
    if (pending == EMPTY32) return EMPTY32;   // every slot holds another key
    // phase 2: the slot's writer has left its loop; wait for it, then look again
    while (__hip_atomic_load(&pt.hs[pending], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) & HS_CLAIM)
      __builtin_amdgcn_s_sleep(1);
  }
}

// One workgroup per range of a VAR16 chunk (ranges[] with pay_begin filled):
// each record's payload offset is the running sum of payload_len, and every
// record of a function with a role adds to the copy table or the handle table.
constexpr uint32_t PA_WG = 256;
__global__ __launch_bounds__(PA_WG) void k_payload(const Seg *__restrict__ segs, const Range *__restrict__ ranges,
                                                   PayTables pt) {
  __shared__ uint32_t wsum[PA_WG / WAVE];
  __shared__ uint64_t run;
  const Range rg = ranges[blockIdx.x];
  const Seg sg = segs[rg.seg];
  const uint32_t lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  if (threadIdx.x == 0) run = rg.pay_begin;
  __syncthreads();
  gq64 *hw = (gq64 *)(sg.rec + rg.begin * 16);
  for (uint64_t c0 = 0; c0 < rg.n; c0 += PA_WG) {
    const uint64_t i = c0 + threadIdx.x;
    const bool in = i < rg.n;
    const uint64_t w1 = in ? hw[2 * i + 1] : 0;
    const uint32_t len = (uint32_t)(w1 >> 56);
    // exclusive prefix of payload_len over the workgroup's records
    uint32_t incl = len;
    for (uint32_t d = 1; d < WAVE; d <<= 1) {
      const uint32_t t = __shfl_up(incl, d, WAVE);
      if (lane >= d) incl += t;
    }
    if (lane == WAVE - 1) wsum[w] = incl;
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (uint32_t k = 0; k < PA_WG / WAVE; k++) { before += k < w ? wsum[k] : 0; total += wsum[k]; }
    const uint64_t poff = run + before + incl - len;
    const uint32_t fn = (uint32_t)(w1 >> 32) & 0xFFFFu, kind = (uint32_t)(w1 >> 48) & 0xFFu;
    const uint8_t role = in && kind <= 1 && fn < pt.n_fns ? pt.roles[fn] : 0;
    // (a chunk whose payload_len sum disagrees with its heap fails the flush;
    // nothing is read outside the heap meanwhile)
    if (role == ROLE_COPY && kind == 0 && len >= 24 && poff + 24 <= sg.pay_bytes) {
      const uint64_t size = pay_u64(sg.pay, poff), dst = pay_u64(sg.pay, poff + 8), src = pay_u64(sg.pay, poff + 16);
      const uint32_t dir = ((src >> 56) == 0xFF ? 2u : 0u) + ((dst >> 56) == 0xFF ? 1u : 0u);
      uint64_t *c = pt.copies + (((size_t)sg.stream * pt.n_fns + fn) * 4 + dir) * 2;
      atomicAdd((unsigned long long *)&c[0], 1ull);
      atomicAdd((unsigned long long *)&c[1], (unsigned long long)size);
    } else if (((role == ROLE_CREATE && kind == 1) || (role == ROLE_RELEASE && kind == 0)) && len >= 8 &&
               poff + 8 <= sg.pay_bytes) {
      const uint32_t k = handle_slot(pt, sg.stream, pay_u64(sg.pay, poff));
      if (k == EMPTY32) atomicOr(pt.err, ERR_CAPACITY);
      else atomicAdd(role == ROLE_CREATE ? &pt.hc[k] : &pt.hr[k], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) run += total;
    __syncthreads();
  }
}

// Per-stream join results: out[s * 5 + {0..4}] += creates, releases,
// distinct handles, unreleased (creates - releases when positive), releases
// that match no create (releases - creates when positive).
__global__ void k_handle_stats(PayTables pt, unsigned long long *out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > pt.hmask) return;
  const uint32_t v = pt.hs[i];
  if (!v || (v & HS_CLAIM)) return;
  unsigned long long *o = out + (size_t)(v - 1) * 5;
  const uint32_t c = pt.hc[i], r = pt.hr[i];
  atomicAdd(&o[0], (unsigned long long)c);
  atomicAdd(&o[1], (unsigned long long)r);
  atomicAdd(&o[2], 1ull);
  if (c > r) atomicAdd(&o[3], (unsigned long long)(c - r));
  else if (r > c) atomicAdd(&o[4], (unsigned long long)(r - c));
}

// --------------------------------------------------------------- launchers
hipError_t launch_pk_count(const uint8_t *buf, uint64_t nbytes, const uint64_t *index, uint32_t n_packets,
                           uint32_t *ev, uint64_t *pay, uint32_t *err, hipStream_t st) {
  if (!n_packets) return hipSuccess;
  hipLaunchKernelGGL(k_pk_count, dim3((n_packets + PK_WG - 1) / PK_WG), dim3(PK_WG), 0, st, buf, nbytes, index,
                     n_packets, ev, pay, err);
  return hipGetLastError();
}
hipError_t launch_pk_scan(uint32_t *ev, uint64_t *pay, uint32_t n, uint64_t *ev_off, uint64_t *tot, hipStream_t st) {
  hipLaunchKernelGGL(k_pk_scan, dim3(1), dim3(1024), 0, st, ev, pay, n, ev_off, tot);
  return hipGetLastError();
}
hipError_t launch_pk_write(const uint8_t *buf, uint64_t nbytes, const uint64_t *index, uint32_t n_packets,
                           const uint64_t *ev_off, const uint64_t *pay_off, uint64_t *hdr, uint64_t *heap,
                           uint32_t *err, hipStream_t st) {
  if (!n_packets) return hipSuccess;
  hipLaunchKernelGGL(k_pk_write, dim3((n_packets + PK_WG - 1) / PK_WG), dim3(PK_WG), 0, st, buf, nbytes, index,
                     n_packets, ev_off, pay_off, hdr, heap, err);
  return hipGetLastError();
}
hipError_t launch_payload(const Seg *segs, const Range *ranges, uint32_t n_ranges, const PayTables &pt,
                          hipStream_t st) {
  if (!n_ranges) return hipSuccess;
  hipLaunchKernelGGL(k_payload, dim3(n_ranges), dim3(PA_WG), 0, st, segs, ranges, pt);
  return hipGetLastError();
}
hipError_t launch_handle_stats(const PayTables &pt, unsigned long long *out, hipStream_t st) {
  hipLaunchKernelGGL(k_handle_stats, dim3((pt.hmask + 256) / 256), dim3(256), 0, st, pt, out);
  return hipGetLastError();
}

}  // namespace tt
