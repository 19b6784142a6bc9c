// tt_post.hip -- kernels after the range pass: the carry combine, the final
// flush, per-stream thread statistics and the readout (canonical ordering,
// compaction and rollups of the tally tables into result rows).
#include "tt_common.h"

namespace tt {

__device__ inline void ga64(uint64_t *p, uint64_t v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void gmin64(uint64_t *p, uint64_t v) {
  __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void gmax64(uint64_t *p, uint64_t v) {
  __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Intervals: a call the combine closes (its frame at stack position pos, its
// parent the frame below, if any).
__device__ inline void emit_civ(const Tables &tb, const uint32_t g, const uint32_t pos, const uint64_t start,
                                const uint64_t end, const uint32_t fn, const Frame *stk) {
  CIval c;
  c.start = start; c.end = end; c.gslot = g; c.depth = pos + 1; c.fn = fn;
  if (pos > 0) { c.pstart = stk[pos - 1].ts; c.pfn = stk[pos - 1].fn; }
  else { c.pstart = 0; c.pfn = EMPTY32; }
  const uint32_t i = atomicAdd(tb.civ_n, 1u);
  if (i < tb.civ_cap) tb.civ[i] = c;
}

// ---------------------------------------------------------------- combine
// One workgroup per stream that had ranges in this flush.  Each distinct
// thread of the stream is owned by one lane (a group of 8 lanes when the
// span's summaries and the stacks fit in LDS), which folds the thread's range
// summaries in range order onto the thread's carried stack: every U item pops
// the call it closes (orphan exit when the stack is empty), checks fn and
// time order, tallies inclusive and self time and credits the parent; the
// range's floor time goes to the call left on top; O items are pushed.
constexpr int CB_SET = 2048;
constexpr int CB_MAP = 16384;   // (range, thread) -> slot table, used when the span fits
constexpr int CB_STK = 512;     // frames of the carried stacks held in LDS during the fold, when they fit
constexpr int CB_DYN = 96 * 1024;  // dynamic LDS for the span's summaries, staged when they fit

template <bool LIST, bool IV>
__global__ __launch_bounds__(256) void k_combine(const uint32_t *__restrict__ spans, const RHdr *__restrict__ rhdr,
                                                 const UItem *__restrict__ ru, const OItem *__restrict__ ro,
                                                 const uint32_t *__restrict__ rnslots, Tables tb,
                                                 const uint32_t *__restrict__ clist) {
  __shared__ uint32_t set_key[CB_SET];
  __shared__ uint32_t set_val[CB_SET];
  __shared__ uint32_t list[CB_SET];
  __shared__ uint8_t smap[CB_MAP];
  __shared__ Frame lstk[CB_STK];
  extern __shared__ __align__(16) uint8_t cdyn[];   // CB_DYN bytes: the span's staged summaries
  __shared__ uint32_t nlist;
  __shared__ uint32_t lcnt[ST_N];
  // threads left to extra passes: the host folds after those passes (the
  // flag is checked before the first global write, once it has arrived)
  const uint32_t err0 = __hip_atomic_load(tb.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t stream = spans[3 * blockIdx.x], rb = spans[3 * blockIdx.x + 1], re = spans[3 * blockIdx.x + 2];
  // the span's positions [rb, re) name summary rows through clist (extra
  // passes of a range follow it), or are the rows themselves
  auto R = [&](const uint32_t p) -> size_t { return LIST ? clist[p] : p; };
  const int tid = threadIdx.x;
  const uint32_t D = tb.D;
  for (int i = tid; i < CB_SET; i += 256) set_key[i] = EMPTY32;
  if (tid < ST_N) lcnt[tid] = 0;
  if (tid == 0) nlist = 0;
  __syncthreads();
  // (range, slot) pairs are spread over all lanes, so the header loads of
  // different ranges are in flight together
  for (uint32_t x = tid; x < (re - rb) * (uint32_t)S_MAX; x += 256) {
    const uint32_t r = rb + x / S_MAX, s = x % S_MAX;
    if (s >= rnslots[R(r)]) continue;
    {
      const uint32_t g = rhdr[R(r) * S_MAX + s].gslot;
      if (g >= tb.max_threads) continue;
      uint32_t h = hash32(g) & (CB_SET - 1);
      for (int probe = 0; probe < CB_SET; probe++) {
        const uint32_t old = atomicCAS(&set_key[h], EMPTY32, g);
        if (old == EMPTY32) {
          const uint32_t k = atomicAdd(&nlist, 1u);
          if (k < CB_SET) list[k] = g;
          set_val[h] = k;
          break;
        }
        if (old == g) break;
        h = (h + 1) & (CB_SET - 1);
      }
    }
  }
  __syncthreads();
  if (err0 & ERR_WIDE) return;
  const uint32_t n = nlist < CB_SET ? nlist : CB_SET;
  if (tid == 0 && nlist >= (uint32_t)CB_SET) atomicOr(tb.err, ERR_CAPACITY);
  // where each thread sits in each range's summaries (0xFF: not in that range)
  const bool use_map = (uint64_t)(re - rb) * n <= (uint64_t)CB_MAP;
  if (use_map) {
    for (uint32_t i = tid; i < (re - rb) * n; i += 256) smap[i] = 0xFF;
    __syncthreads();
    for (uint32_t x = tid; x < (re - rb) * (uint32_t)S_MAX; x += 256) {
      const uint32_t r = rb + x / S_MAX, s = x % S_MAX;
      if (s >= rnslots[R(r)]) continue;
      {
        const uint32_t g = rhdr[R(r) * S_MAX + s].gslot;
        if (g >= tb.max_threads) continue;
        uint32_t h = hash32(g) & (CB_SET - 1);
        for (int probe = 0; probe < CB_SET; probe++) {
          const uint32_t k = set_key[h];
          if (k == g) {
            const uint32_t i = set_val[h];
            if (i < n) smap[(r - rb) * n + i] = (uint8_t)s;
            break;
          }
          if (k == EMPTY32) break;
          h = (h + 1) & (CB_SET - 1);
        }
      }
    }
    __syncthreads();
  }
  // the carried stacks move to LDS for the fold when they fit (set_val, no
  // longer needed, holds each listed thread's height)
  const bool lds_stack = (uint64_t)n * D <= (uint64_t)CB_STK;
  if (lds_stack) {
    for (uint32_t i = tid; i < n; i += 256) set_val[i] = tb.cstate[list[i]].h;
    __syncthreads();
    for (uint32_t x = tid; x < n * D; x += 256) {
      const uint32_t i = x / D, f = x - i * D;
      if (f < set_val[i]) lstk[x] = tb.cstack[(size_t)list[i] * D + f];
    }
    __syncthreads();
  }
  // The span's summaries staged in LDS when they fit: headers by (range,
  // thread) pair, then each pair's U items followed by its O items, packed by
  // an exclusive scan of the pairs' item counts (set_key, no longer needed,
  // holds the per-lane partial sums).  The fold then reads LDS only.
  bool staged = false;
  RHdr *const hdrL = (RHdr *)cdyn;
  uint32_t *offL = nullptr;
  uint8_t *itL = nullptr;
  if (use_map) {
    const uint32_t np = (re - rb) * n;
    const size_t hbytes = (size_t)np * sizeof(RHdr), obytes = ((size_t)np * 4 + 15) & ~(size_t)15;
    if (hbytes + obytes <= (size_t)CB_DYN) {
      offL = (uint32_t *)(cdyn + hbytes);
      itL = cdyn + hbytes + obytes;
      for (uint32_t x = tid; x < np; x += 256) {
        const uint32_t sl = smap[x];
        if (sl != 0xFF) hdrL[x] = rhdr[R(rb + x / n) * S_MAX + sl];
      }
      __syncthreads();
      auto cnt = [&](const uint32_t x) -> uint32_t {
        if (smap[x] == 0xFF) return 0;
        return hdrL[x].nu_listed + (hdrL[x].n_o < D ? hdrL[x].n_o : D);
      };
      const uint32_t chunk = (np + 255) / 256, lo = tid * chunk, hi = lo + chunk < np ? lo + chunk : np;
      uint32_t part = 0;
      for (uint32_t x = lo; x < hi; x++) part += cnt(x);
      set_key[tid] = part;
      __syncthreads();
      if (tid == 0) {
        uint32_t acc = 0;
        for (int k = 0; k < 256; k++) { const uint32_t v = set_key[k]; set_key[k] = acc; acc += v; }
        set_key[256] = acc;
      }
      __syncthreads();
      uint32_t run = set_key[tid];
      for (uint32_t x = lo; x < hi; x++) { offL[x] = run; run += cnt(x); }
      const uint32_t total = set_key[256];
      __syncthreads();
      if (hbytes + obytes + (size_t)total * 32 <= (size_t)CB_DYN) {
        staged = true;
        for (uint32_t x = tid; x < np; x += 256) {
          const uint32_t sl = smap[x];
          if (sl == 0xFF) continue;
          const size_t ib = (R(rb + x / n) * S_MAX + sl) * D;
          const RHdr &hd = hdrL[x];
          UItem *du = (UItem *)(itL + (size_t)offL[x] * 32);
          for (uint32_t k = 0; k < hd.nu_listed; k++) du[k] = ru[ib + k];
          OItem *dq = (OItem *)(du + hd.nu_listed);
          const uint32_t no = hd.n_o < D ? hd.n_o : D;
          for (uint32_t k = 0; k < no; k++) dq[k] = ro[ib + k];
        }
        __syncthreads();
      }
    }
  }
  uint32_t c_tsreg = 0, c_orphan = 0, c_mis = 0, c_neg = 0, c_under = 0;
  if (lds_stack && use_map) {
    // A group of CG lanes per listed thread takes a range summary's U items
    // CG at a time.  U item k pops the frame k below the top the range found
    // (k at or above that height: an orphan exit), so the items are
    // independent once each knows what the item before it credited to the
    // frame it pops: that item's inclusive time when it was tallied (a
    // shuffle within the group).  Then one lane credits the new top (the
    // last item's time and the floor) and the group pushes the O items.
    // hdr_of / u_of / o_of read the summaries from LDS when the span is
    // staged, else from global memory (one instantiation each).
    constexpr uint32_t CG = 8;
    const uint32_t j = (uint32_t)tid % CG;
    auto grouped = [&](auto &&hdr_of, auto &&u_of, auto &&o_of) {
      for (uint32_t i = (uint32_t)tid / CG; i < n; i += 256 / CG) {
        const uint32_t g = list[i];
        CState cs = tb.cstate[g];
        Frame *stk = lstk + (size_t)i * D;
        for (uint32_t r = rb; r < re; r++) {
          const uint32_t x = (r - rb) * n + i;
          const uint32_t sl = smap[x];
          if (sl == 0xFF) continue;
          const RHdr hd = hdr_of(r, x, sl);
          if (hd.flags & RF_HAS_TS) {
            if ((cs.flags & CS_HAS_TS) && hd.first_ts < cs.last_ts && j == 0) c_tsreg++;
            cs.last_ts = hd.last_ts;
            cs.flags |= CS_HAS_TS;
          }
          const int32_t ds = (int32_t)cs.h;
          if ((hd.flags & RF_OVERFLOW) || hd.H > (int32_t)D || ds + hd.M > (int32_t)D) cs.flags |= CS_OVERFLOW;
          const uint32_t h0 = cs.h, nu = hd.nu_listed;
          if (IV) {
            // intervals: the stack this thread carried into the range, top first
            const size_t rs = R(r) * S_MAX + sl;
            if (j == 0) tb.iv_h0[rs] = h0;
            for (uint32_t k = j; k < h0; k += CG) {
              const Frame &f = stk[h0 - 1 - k];
              tb.iv_snap[rs * D + k] = IvFrame{f.ts, f.fn, 0u};
            }
          }
          uint64_t carry = 0;      // the previous chunk's last item: its time when tallied
          uint64_t last = 0;       // the range's last U item: its time when tallied
          for (uint32_t k0 = 0; k0 < nu; k0 += CG) {
            const uint32_t k = k0 + j;
            bool ok = false;
            uint64_t incl = 0, uchild = 0, echild = 0, bytes = 0;
            uint32_t fn = 0;
            if (k < nu) {
              if (k >= h0) {
                c_orphan++;
              } else {
                const UItem u = u_of(r, x, sl, hd, k);
                const Frame e = stk[h0 - 1 - k];
                if (e.fn != u.fn || u.fn >= tb.n_fns) c_mis++;
                else if (u.ts < e.ts) c_neg++;
                else {
                  ok = true; incl = u.ts - e.ts; uchild = u.child; echild = e.child; bytes = e.bytes; fn = u.fn;
                  if (IV) emit_civ(tb, g, h0 - 1 - k, e.ts, u.ts, u.fn, stk);
                }
              }
            }
            const uint64_t mine = ok ? incl : 0;
            const uint64_t before = __shfl_up(mine, 1, CG);
            const uint64_t credit = j == 0 ? carry : before;
            carry = __shfl(mine, CG - 1, CG);
            if (k0 + CG >= nu) last = __shfl(mine, (nu - 1) % CG, CG);
            if (ok) {
              const uint64_t ch = echild + uchild + credit;
              uint64_t self;
              if (ch <= incl) self = incl - ch; else { self = 0; c_under++; }
              Tally *t = &tb.tally[(size_t)g * tb.n_fns + fn];
              ga64(&t->count, 1);
              ga64(&t->incl_sum, incl); gmin64(&t->incl_min, incl); gmax64(&t->incl_max, incl);
              ga64(&t->self_sum, self); gmin64(&t->self_min, self); gmax64(&t->self_max, self);
              if (bytes) ga64(&t->bytes_sum, bytes);
            }
          }
          uint32_t h = h0 > nu ? h0 - nu : 0;
          if (h > 0 && j == 0) stk[h - 1].child += last + hd.floor;
          const uint32_t no = hd.n_o < D ? hd.n_o : D;
          for (uint32_t k = j; k < no; k += CG) {
            if (h + k < D) {
              const OItem o = o_of(r, x, sl, hd, k);
              Frame f;
              f.ts = o.ts; f.child = o.child; f.bytes = o.bytes; f.fn = o.fn; f.pad = 0;
              stk[h + k] = f;
            }
          }
          if (h + no > D) cs.flags |= CS_OVERFLOW;
          cs.h = h + no < D ? h + no : D;
        }
        if (j == 0) {
          if (cs.flags & CS_OVERFLOW) atomicOr(tb.err, ERR_DEPTH);
          tb.cstate[g] = cs;
          set_val[i] = cs.h;
        }
      }
    };
    if (staged) {
      grouped([&](uint32_t, uint32_t x, uint32_t) { return hdrL[x]; },
              [&](uint32_t, uint32_t x, uint32_t, const RHdr &, uint32_t k) {
                return ((const UItem *)(itL + (size_t)offL[x] * 32))[k];
              },
              [&](uint32_t, uint32_t x, uint32_t, const RHdr &hd, uint32_t k) {
                return ((const OItem *)(itL + (size_t)(offL[x] + hd.nu_listed) * 32))[k];
              });
    } else {
      grouped([&](uint32_t r, uint32_t, uint32_t sl) { return rhdr[R(r) * S_MAX + sl]; },
              [&](uint32_t r, uint32_t, uint32_t sl, const RHdr &, uint32_t k) {
                return ru[(R(r) * S_MAX + sl) * D + k];
              },
              [&](uint32_t r, uint32_t, uint32_t sl, const RHdr &, uint32_t k) {
                return ro[(R(r) * S_MAX + sl) * D + k];
              });
    }
  } else {
    for (uint32_t i = tid; i < n; i += 256) {
      const uint32_t g = list[i];
      CState cs = tb.cstate[g];
      // The fold is instantiated once for the stack in LDS and once for the
      // stack in global memory, so that stack accesses are LDS or global
      // instructions: through a generic pointer each of them would wait for
      // the tally atomics issued before it.
      auto fold_thread = [&](Frame *stk) {
        // one range summary onto the carried stack; uat(k) / oat(k) give its
        // U / O items (read four at a time)
        auto fold_one = [&](const RHdr &hd, const size_t rs, auto &&uat, auto &&oat) {
          if (IV) {
            // intervals: the stack this thread carried into the range, top first
            tb.iv_h0[rs] = cs.h;
            for (uint32_t k = 0; k < cs.h; k++) tb.iv_snap[rs * D + k] = IvFrame{stk[cs.h - 1 - k].ts, stk[cs.h - 1 - k].fn, 0u};
          }
          if (hd.flags & RF_HAS_TS) {
            if ((cs.flags & CS_HAS_TS) && hd.first_ts < cs.last_ts) c_tsreg++;
            cs.last_ts = hd.last_ts;
            cs.flags |= CS_HAS_TS;
          }
          const int32_t ds = (int32_t)cs.h;
          if ((hd.flags & RF_OVERFLOW) || hd.H > (int32_t)D || ds + hd.M > (int32_t)D) cs.flags |= CS_OVERFLOW;
          for (uint32_t k0 = 0; k0 < hd.nu_listed; k0 += 4) {
            UItem uu[4];
#pragma unroll
            for (int j = 0; j < 4; j++)
              if (k0 + j < hd.nu_listed) uu[j] = uat(k0 + j);
#pragma unroll
            for (int j = 0; j < 4; j++) {
              if (k0 + j >= hd.nu_listed) break;
              const UItem &u = uu[j];
              if (cs.h == 0) { c_orphan++; continue; }
              cs.h--;
              const Frame e = stk[cs.h];
              if (e.fn != u.fn || u.fn >= tb.n_fns) { c_mis++; continue; }
              if (u.ts < e.ts) { c_neg++; continue; }
              const uint64_t incl = u.ts - e.ts;
              const uint64_t ch = e.child + u.child;
              uint64_t self;
              if (ch <= incl) self = incl - ch; else { self = 0; c_under++; }
              Tally *t = &tb.tally[(size_t)g * tb.n_fns + u.fn];
              ga64(&t->count, 1);
              ga64(&t->incl_sum, incl); gmin64(&t->incl_min, incl); gmax64(&t->incl_max, incl);
              ga64(&t->self_sum, self); gmin64(&t->self_min, self); gmax64(&t->self_max, self);
              if (e.bytes) ga64(&t->bytes_sum, e.bytes);
              if (IV) emit_civ(tb, g, cs.h, e.ts, u.ts, u.fn, stk);
              if (cs.h > 0) stk[cs.h - 1].child += incl;
            }
          }
          if (cs.h > 0) stk[cs.h - 1].child += hd.floor;
          const uint32_t no = hd.n_o < D ? hd.n_o : D;
          for (uint32_t k0 = 0; k0 < no; k0 += 4) {
            OItem oo[4];
#pragma unroll
            for (int j = 0; j < 4; j++)
              if (k0 + j < no) oo[j] = oat(k0 + j);
#pragma unroll
            for (int j = 0; j < 4; j++) {
              if (k0 + j >= no) break;
              if (cs.h < D) {
                Frame f;
                f.ts = oo[j].ts; f.child = oo[j].child; f.bytes = oo[j].bytes; f.fn = oo[j].fn; f.pad = 0;
                stk[cs.h] = f;
                cs.h++;
              } else {
                cs.flags |= CS_OVERFLOW;
              }
            }
          }
        };
        if (staged) {
          for (uint32_t r = rb; r < re; r++) {
            const uint32_t x = (r - rb) * n + i;
            if (smap[x] == 0xFF) continue;
            const RHdr hd = hdrL[x];
            const UItem *lu = (const UItem *)(itL + (size_t)offL[x] * 32);
            const OItem *lo = (const OItem *)(lu + hd.nu_listed);
            fold_one(hd, R(r) * S_MAX + smap[x], [&](uint32_t k) { return lu[k]; },
                     [&](uint32_t k) { return lo[k]; });
          }
        } else {
          // slot of this thread in range r's summaries, S_MAX when it has none
          auto slot_in = [&](const uint32_t r) -> uint32_t {
            if (use_map) {
              const uint32_t sl = smap[(r - rb) * n + i];
              return sl == 0xFF ? (uint32_t)S_MAX : sl;
            }
            const uint32_t ns = rnslots[R(r)];
            const RHdr *hp = rhdr + R(r) * S_MAX;
            uint32_t sl = 0;
            while (sl < ns && hp[sl].gslot != g) sl++;
            return sl < ns ? sl : (uint32_t)S_MAX;
          };
          auto next_range = [&](uint32_t r, uint32_t &sl) {
            for (; r < re; r++) {
              sl = slot_in(r);
              if (sl < (uint32_t)S_MAX) break;
            }
            return r;
          };
          // each range's header is loaded while the previous range is folded
          uint32_t sl = 0;
          uint32_t r = next_range(rb, sl);
          RHdr hd_next;
          if (r < re) hd_next = rhdr[R(r) * S_MAX + sl];
          while (r < re) {
            const RHdr hd = hd_next;
            const size_t ib = (R(r) * S_MAX + sl) * D;
            uint32_t sl2 = 0;
            const uint32_t r2 = next_range(r + 1, sl2);
            if (r2 < re) hd_next = rhdr[R(r2) * S_MAX + sl2];
            fold_one(hd, R(r) * S_MAX + sl, [&](uint32_t k) { return ru[ib + k]; },
                     [&](uint32_t k) { return ro[ib + k]; });
            r = r2;
            sl = sl2;
          }
        }
      };
      if (lds_stack) fold_thread(lstk + (size_t)i * D);
      else fold_thread(tb.cstack + (size_t)g * D);
      if (cs.flags & CS_OVERFLOW) atomicOr(tb.err, ERR_DEPTH);
      tb.cstate[g] = cs;
      if (lds_stack) set_val[i] = cs.h;
    }
  }
  if (lds_stack) {
    __syncthreads();
    for (uint32_t x = tid; x < n * D; x += 256) {
      const uint32_t i = x / D, f = x - i * D;
      if (f < set_val[i]) tb.cstack[(size_t)list[i] * D + f] = lstk[x];
    }
  }
  if (c_tsreg) atomicAdd(&lcnt[ST_TSREG], c_tsreg);
  if (c_orphan) atomicAdd(&lcnt[ST_ORPHAN], c_orphan);
  if (c_mis) atomicAdd(&lcnt[ST_MISMATCH], c_mis);
  if (c_neg) atomicAdd(&lcnt[ST_NEGDUR], c_neg);
  if (c_under) atomicAdd(&lcnt[ST_UNDER], c_under);
  __syncthreads();
  if (tid < ST_N && lcnt[tid]) atomicAdd(&tb.sstats[(size_t)stream * ST_N + tid], (unsigned long long)lcnt[tid]);
}

// ------------------------------------------------------------- intervals
// The public interval record (thapi_tally_interval).
struct IvOut { uint32_t trace, host, pid, tid, fn, depth; uint64_t start, end, pstart; uint32_t pfn, pad; };

// One flush's intervals in the public layout.  Grid (n_ranges + 1, IV_SPLIT):
// the blocks of column r < n_ranges convert summary row r's IvRecs (from
// ivbase[r]), to out + off[r], with
// their depth and a parent opened before the range resolved from the stack
// the combine recorded for the range's thread (each block first caches the
// range's slots -- stream key, tid, carried height -- in LDS); the last column
// copies the combine's own intervals to out + off[n_ranges].  skeys: (trace,
// host, pid) of each stream.
constexpr uint32_t IV_SPLIT = 32;
__global__ __launch_bounds__(256) void k_iv_out(Tables tb, const uint64_t *__restrict__ ivbase,
                                                const RHdr *__restrict__ rhdr, const uint32_t n_ranges,
                                                const uint32_t *__restrict__ rnslots,
                                                const uint64_t *__restrict__ off, const uint32_t *__restrict__ skeys,
                                                IvOut *__restrict__ out) {
  __shared__ uint32_t s_key[S_MAX][4];   // trace, host, pid, tid
  __shared__ uint32_t s_h0[S_MAX];
  __shared__ uint64_t s_stage[256 / WAVE][WAVE * 7];   // per wave: 64 records in the public layout
  const uint32_t D = tb.D, r = blockIdx.x;
  auto key_of = [&](const uint32_t g, uint32_t *k) {
    if (g < tb.max_threads) {
      const uint32_t st = tb.th_stream[g];
      k[0] = skeys[3 * st]; k[1] = skeys[3 * st + 1]; k[2] = skeys[3 * st + 2]; k[3] = tb.th_tid[g];
    } else {
      k[0] = k[1] = k[2] = k[3] = EMPTY32;
    }
  };
  const uint32_t step = gridDim.y * blockDim.x;
  if (r < n_ranges) {
    const uint32_t ns = rnslots[r] < (uint32_t)S_MAX ? rnslots[r] : (uint32_t)S_MAX;
    if (threadIdx.x < ns) {
      const size_t rs = (size_t)r * S_MAX + threadIdx.x;
      key_of(rhdr[rs].gslot, s_key[threadIdx.x]);
      s_h0[threadIdx.x] = tb.iv_h0[rs];
    }
    __syncthreads();
    const uint32_t n = tb.iv_n[r];
    const IvRec *src = tb.iv + ivbase[r];
    uint64_t *const dst = (uint64_t *)(out + off[r]);
    // each wave converts 64 consecutive records into its LDS block, then
    // writes the block's 8-byte words out in order (512 contiguous bytes per
    // store instruction instead of 64 records 56 bytes apart)
    const uint32_t lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    uint64_t *const blk = s_stage[w];
    for (uint32_t i0 = blockIdx.y * blockDim.x + w * WAVE; i0 < n; i0 += step) {
      const uint32_t i = i0 + lane;
      if (i < n) {
        const IvRec v = src[i];
        const uint32_t sl = v.slot, h0 = s_h0[sl];
        const uint32_t base = h0 > v.fneg ? h0 - v.fneg : 0u;   // height below the floor, if any
        uint64_t pst = 0;
        uint32_t pfn = EMPTY32;
        if (v.flags & IV_PARENT_SET) {
          pst = v.pstart; pfn = v.pfn;
        } else if (base > 0) {
          const IvFrame f = tb.iv_snap[((size_t)r * S_MAX + sl) * D + v.fneg];   // position base - 1
          pst = f.ts; pfn = f.fn;
        }
        uint64_t *o = blk + lane * 7;   // the IvOut layout, word by word
        o[0] = (uint64_t)s_key[sl][0] | ((uint64_t)s_key[sl][1] << 32);
        o[1] = (uint64_t)s_key[sl][2] | ((uint64_t)s_key[sl][3] << 32);
        o[2] = (uint64_t)v.fn | ((uint64_t)(base + v.dl) << 32);
        o[3] = v.start;
        o[4] = v.end;
        o[5] = pst;
        o[6] = pfn;
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      const uint32_t words = 7 * (n - i0 < WAVE ? n - i0 : WAVE);
      for (uint32_t k = lane; k < words; k += WAVE) dst[(size_t)i0 * 7 + k] = blk[k];
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
  } else {
    const uint32_t n = *tb.civ_n < tb.civ_cap ? *tb.civ_n : tb.civ_cap;
    IvOut *dst = out + off[n_ranges];
    for (uint32_t i = blockIdx.y * blockDim.x + threadIdx.x; i < n; i += step) {
      const CIval c = tb.civ[i];
      IvOut o;
      uint32_t k[4];
      key_of(c.gslot, k);
      o.trace = k[0]; o.host = k[1]; o.pid = k[2]; o.tid = k[3];
      o.fn = c.fn; o.depth = c.depth; o.start = c.start; o.end = c.end; o.pstart = c.pstart; o.pfn = c.pfn;
      o.pad = 0;
      dst[i] = o;
    }
  }
}

// Final flush: every call still open is counted as unclosed and forgotten.
__global__ void k_final(Tables tb) {
  if (*tb.err & ERR_WIDE) return;   // (the host closes the streams after the extra passes)
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= *tb.n_gslots || g >= tb.max_threads) return;
  const uint32_t h = tb.cstate[g].h;
  if (h) {
    atomicAdd(&tb.sstats[(size_t)tb.th_stream[g] * ST_N + ST_UNCLOSED], (unsigned long long)h);
    tb.cstate[g].h = 0;
  }
}

// The readout's statistics in one buffer, for one copy to the host:
// out[0] the thread count; from out[8], per stream, threads, open calls and
// overflowed threads (3 x u64, zero on entry); from out[8 + 3 * ns1] the
// per-stream counters of the ns streams (ST_N x u64 each).
__global__ void k_thread_stats(Tables tb, unsigned long long *__restrict__ out, uint32_t ns, uint32_t ns1) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) out[0] = *tb.n_gslots;
    for (uint32_t i = threadIdx.x; i < ns * ST_N; i += blockDim.x) out[8 + 3 * (size_t)ns1 + i] = tb.sstats[i];
  }
  if (g >= *tb.n_gslots || g >= tb.max_threads) return;
  unsigned long long *ts = out + 8 + 3 * (size_t)tb.th_stream[g];
  atomicAdd(&ts[0], 1ull);
  const CState cs = tb.cstate[g];
  if (cs.h) atomicAdd(&ts[1], (unsigned long long)cs.h);
  if (cs.flags & CS_OVERFLOW) atomicAdd(&ts[2], 1ull);
}

// --------------------------------------------------------------- readout
// Thread keys in canonical order: key = (canonical stream rank << 32) | tid;
// streams outside the trace filter get rank 0xFFFFFFFF and sort last.
__global__ void k_thread_keys(Tables tb, const uint32_t *__restrict__ stream_rank, uint64_t *__restrict__ keys,
                              uint32_t *__restrict__ vals, uint32_t n) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  keys[g] = ((uint64_t)stream_rank[tb.th_stream[g]] << 32) | tb.th_tid[g];
  vals[g] = g;
}

// Stable LSD radix sort of (key, val) pairs by one workgroup of 1024 lanes,
// 8-bit digits; bits [lo_bit, hi_bit) of the key are sorted.  Each pass:
// digit histogram, exclusive scan, then a stable scatter in chunks of 1024
// where a record's rank among equal digits in its wave comes from ballots.
constexpr int RS_WG = 1024;
__global__ __launch_bounds__(RS_WG) void k_radix_sort(uint64_t *keys, uint32_t *vals, uint64_t *keys2,
                                                      uint32_t *vals2, uint32_t n, int lo_bit, int hi_bit) {
  __shared__ uint32_t hist[256];
  __shared__ uint32_t base[256];
  __shared__ uint32_t wc[RS_WG / WAVE][256];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  uint64_t *ks = keys, *kd = keys2;
  uint32_t *vs = vals, *vd = vals2;
  for (int b = lo_bit; b < hi_bit; b += 8) {
    for (int i = tid; i < 256; i += RS_WG) hist[i] = 0;
    __syncthreads();
    for (uint32_t i = tid; i < n; i += RS_WG) atomicAdd(&hist[(ks[i] >> b) & 0xFF], 1u);
    __syncthreads();
    if (tid == 0) {
      uint32_t acc = 0;
      for (int d = 0; d < 256; d++) { base[d] = acc; acc += hist[d]; }
    }
    __syncthreads();
    for (uint32_t c0 = 0; c0 < n; c0 += RS_WG) {
      for (int i = lane; i < 256; i += WAVE) wc[w][i] = 0;
      const uint32_t i = c0 + tid;
      const bool valid = i < n;
      const uint64_t k = valid ? ks[i] : 0;
      const uint32_t v = valid ? vs[i] : 0;
      const uint32_t d = (uint32_t)(k >> b) & 0xFF;
      uint64_t mask = __builtin_amdgcn_ballot_w64(valid);
      for (int bit = 0; bit < 8; bit++) {
        const uint64_t bb = __builtin_amdgcn_ballot_w64(valid && ((d >> bit) & 1u));
        mask &= ((d >> bit) & 1u) ? bb : ~bb;
      }
      const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
      const uint32_t rk = (uint32_t)__popcll(mask & lt);
      if (valid && rk == 0) wc[w][d] = (uint32_t)__popcll(mask);
      __syncthreads();
      if (valid) {
        uint32_t pre = 0;
        for (int ww = 0; ww < w; ww++) pre += wc[ww][d];
        const uint32_t pos = base[d] + pre + rk;
        kd[pos] = k;
        vd[pos] = v;
      }
      __syncthreads();
      if (tid < 256) {
        uint32_t tot = 0;
        for (int ww = 0; ww < RS_WG / WAVE; ww++) tot += wc[ww][tid];
        base[tid] += tot;
      }
      __syncthreads();
    }
    uint64_t *tk = ks; ks = kd; kd = tk;
    uint32_t *tv = vs; vs = vd; vd = tv;
  }
  // the result must end in keys/vals: copy back after an odd number of passes
  if (ks != keys) {
    for (uint32_t i = tid; i < n; i += RS_WG) { keys[i] = ks[i]; vals[i] = vs[i]; }
  }
}

// Small thread sets (at most SORT_SMALL threads): the keys, a stable sort
// and the group bounds in one workgroup.  Each lane ranks its key by counting
// the keys that order before it, ties by position, over a copy in LDS (all
// lanes read the same key at a time); gbeg/gend are cleared first.
constexpr int SORT_SMALL = 256;
__global__ __launch_bounds__(SORT_SMALL) void k_sort_small(Tables tb, const uint32_t *__restrict__ stream_rank,
                                                           uint64_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                                           uint32_t n, uint32_t *__restrict__ gbeg,
                                                           uint32_t *__restrict__ gend, uint32_t n_ranks) {
  __shared__ uint64_t k_in[SORT_SMALL];
  __shared__ uint64_t k_out[SORT_SMALL];
  const uint32_t i = threadIdx.x;
  uint64_t k = 0;
  if (i < n) {
    k = ((uint64_t)stream_rank[tb.th_stream[i]] << 32) | tb.th_tid[i];
    k_in[i] = k;
  }
  for (uint32_t r = i; r < n_ranks; r += SORT_SMALL) { gbeg[r] = 0; gend[r] = 0; }
  __syncthreads();
  if (i < n) {
    uint32_t rank = 0;
    for (uint32_t j = 0; j < n; j++) {
      const uint64_t kj = k_in[j];
      rank += (kj < k || (kj == k && j < i)) ? 1u : 0u;
    }
    k_out[rank] = k;
    keys[rank] = k;
    vals[rank] = i;
  }
  __syncthreads();
  if (i < n) {
    const uint32_t sr = (uint32_t)(k_out[i] >> 32);
    if (sr < n_ranks) {
      if (i == 0 || (uint32_t)(k_out[i - 1] >> 32) != sr) gbeg[sr] = i;
      if (i == n - 1 || (uint32_t)(k_out[i + 1] >> 32) != sr) gend[sr] = i + 1;
    }
  }
}

// Group bounds: for every canonical stream rank, the positions of its threads
// in the sorted key array.
__global__ void k_group_bounds(const uint64_t *__restrict__ keys, uint32_t n, uint32_t *__restrict__ gbeg,
                               uint32_t *__restrict__ gend, uint32_t n_ranks) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t sr = (uint32_t)(keys[i] >> 32);
  if (sr >= n_ranks) return;
  if (i == 0 || (uint32_t)(keys[i - 1] >> 32) != sr) gbeg[sr] = i;
  if (i == n - 1 || (uint32_t)(keys[i + 1] >> 32) != sr) gend[sr] = i + 1;
}

// Row groups: a group emits one row per id (fn or kernel id) with a non-empty
// tally, ids ascending.  mode 1 THREAD: group = a thread (sorted position);
// mode 2 PROCESS: group = a canonical stream, members = its threads; mode 3 FN:
// group = a trace, members = the threads of its streams; mode 4 KERNEL: group
// = a canonical stream, source = its kernel tallies.
struct RowCtx {
  int mode;
  uint32_t n_ids;                 // n_fns or n_kid
  const uint64_t *keys;           // sorted thread keys
  const uint32_t *vals;           // sorted thread slots
  const uint32_t *gbeg, *gend;    // per canonical stream rank
  const uint32_t *rank_stream;    // canonical rank -> stream index
  const uint32_t *rank_key;       // canonical rank -> (trace, host, pid) as 3 u32
  const uint32_t *trace_span;     // FN mode: group -> [rank_begin, rank_end)
};

struct Acc { uint64_t v[8]; };

__device__ inline void acc_init(Acc &a) {
  a.v[0] = 0; a.v[1] = 0; a.v[2] = ~0ull; a.v[3] = 0; a.v[4] = 0; a.v[5] = ~0ull; a.v[6] = 0; a.v[7] = 0;
}
__device__ inline void acc_add(Acc &a, const Tally &t) {
  a.v[0] += t.count;
  a.v[1] += t.incl_sum; a.v[2] = t.incl_min < a.v[2] ? t.incl_min : a.v[2]; a.v[3] = t.incl_max > a.v[3] ? t.incl_max : a.v[3];
  a.v[4] += t.self_sum; a.v[5] = t.self_min < a.v[5] ? t.self_min : a.v[5]; a.v[6] = t.self_max > a.v[6] ? t.self_max : a.v[6];
  a.v[7] += t.bytes_sum;
}

__device__ inline void group_value(const RowCtx &c, const Tables &tb, uint32_t grp, uint32_t id, Acc &a) {
  acc_init(a);
  if (c.mode == 1) {
    acc_add(a, tb.tally[(size_t)c.vals[grp] * tb.n_fns + id]);
  } else if (c.mode == 2) {
    for (uint32_t i = c.gbeg[grp]; i < c.gend[grp]; i++) acc_add(a, tb.tally[(size_t)c.vals[i] * tb.n_fns + id]);
  } else if (c.mode == 3) {
    for (uint32_t r = c.trace_span[2 * grp]; r < c.trace_span[2 * grp + 1]; r++)
      for (uint32_t i = c.gbeg[r]; i < c.gend[r]; i++) acc_add(a, tb.tally[(size_t)c.vals[i] * tb.n_fns + id]);
  } else {
    const KTally k = tb.ktally[(size_t)c.rank_stream[grp] * tb.n_kid + id];
    a.v[0] = k.count; a.v[1] = k.sum; a.v[2] = k.min; a.v[3] = k.max;
    a.v[4] = 0; a.v[5] = 0; a.v[6] = 0; a.v[7] = 0;
  }
}

// Pass 1 (out == null): count the non-empty ids of each group into cnt[grp].
// Pass 2: write them at off[grp] + (rank among the group's non-empty ids).
__global__ __launch_bounds__(256) void k_group_rows(RowCtx c, Tables tb, uint32_t *__restrict__ cnt,
                                                    const uint64_t *__restrict__ off, uint8_t *__restrict__ out) {
  __shared__ uint32_t wsum[4];
  __shared__ uint32_t run;
  const uint32_t grp = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid == 0) run = 0;
  __syncthreads();
  for (uint32_t id0 = 0; id0 < c.n_ids; id0 += 256) {
    const uint32_t id = id0 + tid;
    Acc a;
    bool ne = false;
    if (id < c.n_ids) { group_value(c, tb, grp, id, a); ne = a.v[0] != 0; }
    const uint64_t m = __builtin_amdgcn_ballot_w64(ne);
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    if (lane == 0) wsum[w] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t pre = run;
    for (int k = 0; k < w; k++) pre += wsum[k];
    if (ne && out) {
      const uint64_t pos = off[grp] + pre + (uint32_t)__popcll(m & lt);
      uint32_t *row = (uint32_t *)(out + pos * 88);
      uint32_t tr, ho, pi, ti;
      if (c.mode == 1) {
        const uint32_t rank = (uint32_t)(c.keys[grp] >> 32);
        tr = c.rank_key[3 * rank]; ho = c.rank_key[3 * rank + 1]; pi = c.rank_key[3 * rank + 2];
        ti = (uint32_t)c.keys[grp];
      } else if (c.mode == 2 || c.mode == 4) {
        tr = c.rank_key[3 * grp]; ho = c.rank_key[3 * grp + 1]; pi = c.rank_key[3 * grp + 2];
        ti = EMPTY32;
      } else {
        tr = c.rank_key[3 * c.trace_span[2 * grp]]; ho = EMPTY32; pi = EMPTY32; ti = EMPTY32;
      }
      row[0] = tr; row[1] = ho; row[2] = pi; row[3] = ti;
      row[4] = (id & 0xFFFFu) | ((c.mode == 4 ? 2u : 1u) << 16);
      row[5] = 0;
      uint64_t *f = (uint64_t *)(out + pos * 88 + 24);
      for (int k = 0; k < 8; k++) f[k] = a.v[k];
    }
    __syncthreads();
    if (tid == 0) { uint32_t t = 0; for (int k = 0; k < 4; k++) t += wsum[k]; run += t; }
    __syncthreads();
  }
  if (!out && tid == 0) cnt[grp] = run;
}

// Exclusive scan of cnt[0..n) into off[0..n] by one workgroup (off[n] = total).
__global__ __launch_bounds__(1024) void k_scan_counts(const uint32_t *__restrict__ cnt, uint64_t *__restrict__ off,
                                                      uint32_t n) {
  __shared__ uint64_t part[1024];
  __shared__ uint64_t carry;
  const int tid = threadIdx.x;
  if (tid == 0) carry = 0;
  __syncthreads();
  for (uint32_t c0 = 0; c0 < n; c0 += 1024) {
    const uint32_t i = c0 + tid;
    const uint64_t v = i < n ? cnt[i] : 0;
    part[tid] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const uint64_t t = tid >= o ? part[tid - o] : 0;
      __syncthreads();
      part[tid] += t;
      __syncthreads();
    }
    if (i < n) off[i] = carry + part[tid] - v;
    __syncthreads();
    if (tid == 0) carry += part[1023];
    __syncthreads();
  }
  if (tid == 0) off[n] = carry;
}

// ---------------------------------------------------------- fills / init
__global__ void k_fill64(uint64_t *p, size_t n, uint64_t v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill32(uint32_t *p, size_t n, uint32_t v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

// Every table of a handle at its initial value, in one launch.
__global__ void k_init_all(InitSet is) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t i0 = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  for (size_t i = i0; i < is.n_gkeys; i += stride) is.gkeys[i] = EMPTY64;
  for (size_t i = i0; i < is.n_gvals; i += stride) is.gvals[i] = GV_PENDING;
  for (size_t i = i0; i < is.n_tally; i += stride) {
    Tally v;
    v.count = 0; v.incl_sum = 0; v.incl_min = ~0ull; v.incl_max = 0;
    v.self_sum = 0; v.self_min = ~0ull; v.self_max = 0; v.bytes_sum = 0;
    is.tally[i] = v;
  }
  for (size_t i = i0; i < is.n_ktally; i += stride) {
    KTally v;
    v.count = 0; v.sum = 0; v.min = ~0ull; v.max = 0;
    is.ktally[i] = v;
  }
  for (size_t i = i0; i < is.n_cstate; i += stride) is.cstate[i] = 0;
  for (size_t i = i0; i < is.n_sstats; i += stride) is.sstats[i] = 0;
  for (size_t i = i0; i < is.n_s_nth; i += stride) is.s_nth[i] = 0;
  if (i0 == 0) { *is.ngs = 0; *is.err = 0; }
}

// ----------------------------------------------------------------- merge
// Merge of an exported aggregate into the tables (the host has validated it
// and mapped its streams to this handle's stream indices).

// Pass 1 (run alone first): a blob thread with open calls must find no open
// call on the same (stream, tid) here; a conflict sets *conflict, and the
// host then runs no later pass.
__global__ void k_merge_check(Tables tb, const MThread *__restrict__ th, uint32_t n, uint32_t *conflict) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !th[i].h) return;
  const uint32_t g = lookup_gslot(tb, th[i].stream, th[i].tid);
  if (g < tb.max_threads && tb.cstate[g].h) atomicOr(conflict, 1u);
}

// Pass 2: every blob thread gets its slot here (inserted on first sight),
// its open calls and last timestamp are installed, its flags combined.
__global__ void k_merge_threads(Tables tb, const MThread *__restrict__ th, uint32_t n,
                                const Frame *__restrict__ frames, uint32_t *__restrict__ gmap) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const MThread m = th[i];
  const uint32_t g = resolve_gslot(tb, m.stream, m.tid);
  gmap[i] = g;
  if (g >= tb.max_threads) return;
  CState cs = tb.cstate[g];
  if (m.h) {
    for (uint32_t k = 0; k < m.h; k++) tb.cstack[(size_t)g * tb.D + k] = frames[m.frame0 + k];
    cs.h = m.h;
  }
  if (m.flags & CS_HAS_TS)
    cs.last_ts = (cs.flags & CS_HAS_TS) && cs.last_ts > m.last_ts ? cs.last_ts : m.last_ts;
  cs.flags |= m.flags;
  tb.cstate[g] = cs;
}

// Pass 3: tally rows, kernel rows and stream counters, combined with u64
// add / min / max (order-independent).
__global__ void k_merge_rows(Tables tb, const uint32_t *__restrict__ gmap, const MRow *__restrict__ rows,
                             uint32_t n_rows, const MKRow *__restrict__ krows, uint32_t n_krows,
                             const uint64_t *__restrict__ scnt, const uint32_t *__restrict__ sidx, uint32_t n_streams) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_rows) {
    const MRow r = rows[i];
    const uint32_t g = gmap[r.thread];
    if (g < tb.max_threads) {
      Tally *d = &tb.tally[(size_t)g * tb.n_fns + r.fn];
      ga64(&d->count, r.v.count);
      ga64(&d->incl_sum, r.v.incl_sum);
      ga64(&d->self_sum, r.v.self_sum);
      ga64(&d->bytes_sum, r.v.bytes_sum);
      gmin64(&d->incl_min, r.v.incl_min);
      gmax64(&d->incl_max, r.v.incl_max);
      gmin64(&d->self_min, r.v.self_min);
      gmax64(&d->self_max, r.v.self_max);
    }
  }
  if (i < n_krows) {
    const MKRow r = krows[i];
    KTally *d = &tb.ktally[(size_t)r.stream * tb.n_kid + r.kid];
    ga64(&d->count, r.v.count);
    ga64(&d->sum, r.v.sum);
    gmin64(&d->min, r.v.min);
    gmax64(&d->max, r.v.max);
  }
  if (i < n_streams * (uint32_t)ST_N) {
    const uint32_t s = i / ST_N, k = i - s * ST_N;
    if (scnt[i]) ga64((uint64_t *)&tb.sstats[(size_t)sidx[s] * ST_N + k], scnt[i]);
  }
}

// --------------------------------------------------------------- launchers
static dim3 fill_grid(size_t n) {
  size_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  if (b == 0) b = 1;
  return dim3((unsigned)b);
}
hipError_t launch_fill64(uint64_t *p, size_t n, uint64_t v, hipStream_t st) {
  if (n) hipLaunchKernelGGL(k_fill64, fill_grid(n), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill32(uint32_t *p, size_t n, uint32_t v, hipStream_t st) {
  if (n) hipLaunchKernelGGL(k_fill32, fill_grid(n), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}
hipError_t launch_init_all(const InitSet &is, hipStream_t st) {
  size_t n = is.n_gkeys > is.n_tally ? is.n_gkeys : is.n_tally;
  if (is.n_ktally > n) n = is.n_ktally;
  if (is.n_cstate > n) n = is.n_cstate;
  if (is.n_sstats > n) n = is.n_sstats;
  hipLaunchKernelGGL(k_init_all, fill_grid(n), dim3(256), 0, st, is);
  return hipGetLastError();
}
// Allows the combine its dynamic LDS (set once, outside any stream capture).
hipError_t prepare_combine_kernel() {
  const void *ks[] = {(const void *)k_combine<false, false>, (const void *)k_combine<false, true>,
                      (const void *)k_combine<true, false>, (const void *)k_combine<true, true>};
  for (const void *k : ks) {
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, CB_DYN);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
hipError_t launch_combine(const uint32_t *spans, uint32_t n_spans, const RHdr *rhdr, const UItem *ru,
                          const OItem *ro, const uint32_t *rnslots, const Tables &tb, const uint32_t *clist,
                          hipStream_t st) {
  if (!n_spans) return hipSuccess;
#define TT_COMBINE(L_, I_) \
  hipLaunchKernelGGL((k_combine<L_, I_>), dim3(n_spans), dim3(256), CB_DYN, st, spans, rhdr, ru, ro, rnslots, tb, clist)
  const bool iv = tb.iv != nullptr;
  if (clist) { if (iv) TT_COMBINE(true, true); else TT_COMBINE(true, false); }
  else { if (iv) TT_COMBINE(false, true); else TT_COMBINE(false, false); }
#undef TT_COMBINE
  return hipGetLastError();
}
hipError_t launch_iv_out(const Tables &tb, const uint64_t *ivbase, const RHdr *rhdr, uint32_t n_ranges,
                         const uint32_t *rnslots, const uint64_t *off, const uint32_t *skeys, void *out,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_iv_out, dim3(n_ranges + 1, IV_SPLIT), dim3(256), 0, st, tb, ivbase, rhdr, n_ranges, rnslots,
                     off, skeys, (IvOut *)out);
  return hipGetLastError();
}

hipError_t launch_final(const Tables &tb, uint32_t max_threads, hipStream_t st) {
  hipLaunchKernelGGL(k_final, dim3((max_threads + 255) / 256), dim3(256), 0, st, tb);
  return hipGetLastError();
}
hipError_t launch_thread_stats(const Tables &tb, uint32_t max_threads, unsigned long long *out, uint32_t ns,
                               uint32_t ns1, hipStream_t st) {
  hipLaunchKernelGGL(k_thread_stats, dim3((max_threads + 255) / 256), dim3(256), 0, st, tb, out, ns, ns1);
  return hipGetLastError();
}
hipError_t launch_sort_threads(const Tables &tb, const uint32_t *stream_rank, uint64_t *keys, uint32_t *vals,
                               uint64_t *keys2, uint32_t *vals2, uint32_t n, int rank_bits, hipStream_t st) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_thread_keys, dim3((n + 255) / 256), dim3(256), 0, st, tb, stream_rank, keys, vals, n);
  // tid: 32 bits; canonical stream rank (or the 0xFFFFFFFF filter mark): 32 bits
  hipLaunchKernelGGL(k_radix_sort, dim3(1), dim3(RS_WG), 0, st, keys, vals, keys2, vals2, n, 0, 32 + rank_bits);
  return hipGetLastError();
}
bool sort_small_fits(uint32_t n) { return n <= (uint32_t)SORT_SMALL; }
hipError_t launch_sort_small(const Tables &tb, const uint32_t *stream_rank, uint64_t *keys, uint32_t *vals, uint32_t n,
                             uint32_t *gbeg, uint32_t *gend, uint32_t n_ranks, hipStream_t st) {
  if (n > (uint32_t)SORT_SMALL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sort_small, dim3(1), dim3(SORT_SMALL), 0, st, tb, stream_rank, keys, vals, n, gbeg, gend,
                     n_ranks);
  return hipGetLastError();
}
hipError_t launch_group_bounds(const uint64_t *keys, uint32_t n, uint32_t *gbeg, uint32_t *gend, uint32_t n_ranks,
                               hipStream_t st) {
  if (n) hipLaunchKernelGGL(k_group_bounds, dim3((n + 255) / 256), dim3(256), 0, st, keys, n, gbeg, gend, n_ranks);
  return hipGetLastError();
}
hipError_t launch_group_rows(const RowCtx &c, const Tables &tb, uint32_t n_groups, uint32_t *cnt, uint64_t *off,
                             uint8_t *out, hipStream_t st) {
  if (!n_groups) return hipSuccess;
  if (!out) {
    hipLaunchKernelGGL(k_group_rows, dim3(n_groups), dim3(256), 0, st, c, tb, cnt, (const uint64_t *)nullptr,
                       (uint8_t *)nullptr);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, st, cnt, off, n_groups);
  } else {
    hipLaunchKernelGGL(k_group_rows, dim3(n_groups), dim3(256), 0, st, c, tb, cnt, (const uint64_t *)off, out);
  }
  return hipGetLastError();
}

hipError_t launch_merge(const Tables &tb, const MThread *th, uint32_t n_th, const Frame *frames, uint32_t *gmap,
                        const MRow *rows, uint32_t n_rows, const MKRow *krows, uint32_t n_krows, const uint64_t *scnt,
                        const uint32_t *sidx, uint32_t n_streams, uint32_t *conflict, bool check_only,
                        hipStream_t st) {
  if (check_only) {
    if (n_th) hipLaunchKernelGGL(k_merge_check, dim3((n_th + 255) / 256), dim3(256), 0, st, tb, th, n_th, conflict);
    return hipGetLastError();
  }
  if (n_th) hipLaunchKernelGGL(k_merge_threads, dim3((n_th + 255) / 256), dim3(256), 0, st, tb, th, n_th, frames, gmap);
  uint32_t n = n_rows > n_krows ? n_rows : n_krows;
  if (n < n_streams * (uint32_t)ST_N) n = n_streams * (uint32_t)ST_N;
  if (n) hipLaunchKernelGGL(k_merge_rows, dim3((n + 255) / 256), dim3(256), 0, st, tb, gmap, rows, n_rows, krows,
                            n_krows, scnt, sidx, n_streams);
  return hipGetLastError();
}

}  // namespace tt
