/*
 * oracle.c -- plain single-threaded CPU oracle of the trace tally.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no header, helper, table or constant with the GPU
 * path and parses the record bytes itself.
 *
 * What it computes (the tally of the paper's section 3.4 and the worked
 * table of section 4.3, with the interval definition of section 3.3):
 * every API call is an entry event followed later, on the same thread, by
 * an exit event (section 3.2: all API entry and exit points are traced);
 * its interval is [entry ts, exit ts] (section 3.3, interval plugins); the
 * tally keeps, per function, the number of calls and the summed, minimum and
 * maximum inclusive duration (the Time / Calls / Min / Max columns of the
 * section 4.3 table, where Time is inclusive: a HIP call and the Level-Zero
 * calls nested in it are both counted).  Threads are told apart by host,
 * process and thread id (the record of section 1.1); LTTng may drop events
 * (section 3.1), so unmatched events are counted, not assumed away.
 *
 * Per stream (chunks in submit order), per record in order:
 *   kernel record (kind 2): if kernel_id < n_kernel_ids and end >= start,
 *     K[stream, kernel_id] += {1, end-start}; otherwise a bad record.
 *   entry (kind 0, fn < n_fns): ts below the thread's previous API ts counts
 *     a ts regression; push {fn, ts, child = 0, bytes}; a stack deeper than
 *     max_depth marks the thread as overflowed.
 *   exit (kind 1, fn < n_fns): ts regression as above; empty stack -> orphan
 *     exit; else pop e: e.fn != fn -> fn mismatch (not tallied, nothing added
 *     to the parent); ts < e.ts -> negative duration (same); else
 *     incl = ts - e.ts, self = incl - e.child (or 0 and a self underflow when
 *     e.child > incl), T[stream, tid, fn] += {1, incl, self, e.bytes} and the
 *     new stack top (if any) gets child += incl.
 *   anything else: a bad record.
 * Final flush: every entry still open counts as unclosed and is not tallied.
 * All arithmetic is unsigned 64-bit integer (modulo 2^64).
 *
 * Payload analytics (VAR16 only), per record in order and independent of
 * call matching, for functions given a role (oracle_set_roles):
 *   copy (role 1): an entry with payload_len >= 24 carries size (u64 at 0),
 *     destination and source pointers (u64 at 8 and 16); a pointer whose top
 *     byte is 0xff is device memory, any other host memory (section 1.1
 *     reads a copy's direction from these prefixes); per (stream, fn,
 *     direction = 2 * source-on-device + destination-on-device) the entries
 *     are counted and their sizes summed.
 *   create (role 2): an exit with payload_len >= 8 returns a handle (u64 at 0).
 *   release (role 3): an entry with payload_len >= 8 takes a handle (u64 at 0).
 *   Per stream, creates and releases are joined by handle value (section 4.2:
 *   a validation pass reports unhandled releases): a value created C times
 *   and released R times leaves max(0, C - R) handles unreleased and
 *   max(0, R - C) releases that match no create; record order is not
 *   considered.
 * Packed chunks (oracle_submit_packed): CTF-like packets, each a 16-byte
 * header {u32 magic "THPK", u32 packet bytes, u32 events, u32 0} followed by
 * its events, each a VAR16 header and its payload inline, padded to a
 * multiple of 8 bytes; the events are taken in order into the VAR16 path.
 *
 * On request (oracle_keep_intervals) every tallied call is also kept as an
 * interval (section 3.3: an interval plugin turns the entry and exit events
 * of a call into one record spanning them; section 3.6 draws such records on
 * a timeline): {stream, tid, fn, depth, entry ts, exit ts, and the entry ts
 * and fn of the call that was the stack top when this one was entered (its
 * parent; none at the top level)}, depth 1 being the top level.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- maps */
/* Open addressing on a (u64, u64) key.  Obviously-correct, not fast. */
typedef struct { uint64_t a, b; int used; uint32_t val; } slot_t;
typedef struct { slot_t *s; size_t cap, n; } map_t;

static uint64_t mix(uint64_t x) {
  x ^= x >> 33; x *= 0xff51afd7ed558ccdull; x ^= x >> 33; x *= 0xc4ceb9fe1a85ec53ull; x ^= x >> 33;
  return x;
}
static void map_init(map_t *m) { m->cap = 1024; m->n = 0; m->s = (slot_t *)calloc(m->cap, sizeof(slot_t)); }
static void map_free(map_t *m) { free(m->s); m->s = NULL; m->cap = m->n = 0; }
static slot_t *map_find(map_t *m, uint64_t a, uint64_t b) {
  size_t i = (size_t)(mix(a * 31 + mix(b)) & (m->cap - 1));
  for (;;) {
    slot_t *s = &m->s[i];
    if (!s->used) return s;
    if (s->a == a && s->b == b) return s;
    i = (i + 1) & (m->cap - 1);
  }
}
static void map_grow(map_t *m) {
  map_t n; n.cap = m->cap * 2; n.n = 0; n.s = (slot_t *)calloc(n.cap, sizeof(slot_t));
  for (size_t i = 0; i < m->cap; i++)
    if (m->s[i].used) { slot_t *d = map_find(&n, m->s[i].a, m->s[i].b); *d = m->s[i]; n.n++; }
  free(m->s); *m = n;
}
/* returns the value index for the key, inserting `fresh` when absent */
static uint32_t map_get(map_t *m, uint64_t a, uint64_t b, uint32_t fresh, int *inserted) {
  if ((m->n + 1) * 2 > m->cap) map_grow(m);
  slot_t *s = map_find(m, a, b);
  if (s->used) { *inserted = 0; return s->val; }
  s->used = 1; s->a = a; s->b = b; s->val = fresh; m->n++;
  *inserted = 1;
  return fresh;
}

/* ------------------------------------------------------------- state */
typedef struct { uint16_t fn; uint64_t ts, child, bytes; } frame_t;
typedef struct {
  uint32_t stream, tid;
  frame_t *stk; size_t h, cap;
  uint64_t last_ts; int seen; int overflowed;
} thread_t;
typedef struct { uint32_t trace, host, pid; uint64_t st[17]; int has_record; } stream_t;
typedef struct { uint32_t stream, tid, fn; uint64_t v[8]; } tally_t;   /* count, incl sum/min/max, self sum/min/max, bytes */
typedef struct { uint32_t stream, kid; uint64_t v[4]; } ktally_t;       /* count, dur sum/min/max */
typedef struct { uint32_t stream, tid, fn, depth; uint64_t start, end, pstart; uint32_t pfn, pad; } ival_t;
typedef struct { uint32_t stream, fn, dir; uint64_t count, bytes; } copy_t;
typedef struct { uint32_t stream; uint64_t handle, creates, releases; } handle_t;

enum { S_RECORDS, S_ENTRIES, S_EXITS, S_KERNEL, S_ORPHAN, S_MISMATCH, S_NEGDUR, S_SELFUNDER,
       S_TSREG, S_UNCLOSED, S_OPEN, S_DEPTH, S_BAD, S_DROPPED, S_HOSTS, S_PROCS, S_THREADS, S_N };

typedef struct oracle {
  int format; uint32_t n_fns, n_kernel_ids, max_depth;
  uint8_t *has_size;
  map_t smap, tmap, tally_map, kmap;
  stream_t *streams; size_t ns, scap;
  thread_t *threads; size_t nt, tcap;
  tally_t *tallies; size_t ntal, talcap;
  ktally_t *kt; size_t nkt, ktcap;
  int keep_ivals;
  ival_t *iv; size_t niv, ivcap;
  uint8_t *roles;                          /* per fn: 0, 1 copy, 2 create, 3 release */
  map_t copy_map; copy_t *cp; size_t ncp, cpcap;
  map_t hmap; handle_t *hd; size_t nhd, hdcap;
} oracle;

#define GROW(arr, n, cap) do { if ((n) == (cap)) { (cap) = (cap) ? (cap) * 2 : 64; \
  (arr) = realloc((arr), (cap) * sizeof(*(arr))); } } while (0)

oracle *oracle_new(int format, uint32_t n_fns, uint32_t n_kernel_ids, uint32_t max_depth,
                   const uint8_t *has_size) {
  oracle *o = (oracle *)calloc(1, sizeof(oracle));
  o->format = format; o->n_fns = n_fns; o->n_kernel_ids = n_kernel_ids; o->max_depth = max_depth;
  o->has_size = (uint8_t *)calloc(n_fns ? n_fns : 1, 1);
  if (has_size) memcpy(o->has_size, has_size, n_fns);
  map_init(&o->smap); map_init(&o->tmap); map_init(&o->tally_map); map_init(&o->kmap);
  map_init(&o->copy_map); map_init(&o->hmap);
  o->roles = (uint8_t *)calloc(n_fns ? n_fns : 1, 1);
  return o;
}

void oracle_free(oracle *o) {
  if (!o) return;
  for (size_t i = 0; i < o->nt; i++) free(o->threads[i].stk);
  free(o->threads); free(o->streams); free(o->tallies); free(o->kt); free(o->has_size); free(o->iv);
  free(o->roles); free(o->cp); free(o->hd);
  map_free(&o->smap); map_free(&o->tmap); map_free(&o->tally_map); map_free(&o->kmap);
  map_free(&o->copy_map); map_free(&o->hmap);
  free(o);
}

static uint64_t rd64(const uint8_t *p) { uint64_t v; memcpy(&v, p, 8); return v; }
static uint32_t rd32(const uint8_t *p) { uint32_t v; memcpy(&v, p, 4); return v; }
static uint16_t rd16(const uint8_t *p) { uint16_t v; memcpy(&v, p, 2); return v; }

static uint32_t stream_of(oracle *o, uint32_t trace, uint32_t host, uint32_t pid) {
  int ins;
  uint64_t a = ((uint64_t)trace << 32) | host;
  uint32_t id = map_get(&o->smap, a, pid, (uint32_t)o->ns, &ins);
  if (ins) {
    GROW(o->streams, o->ns, o->scap);
    stream_t *s = &o->streams[o->ns++];
    memset(s, 0, sizeof *s);
    s->trace = trace; s->host = host; s->pid = pid;
  }
  return id;
}
static thread_t *thread_of(oracle *o, uint32_t stream, uint32_t tid) {
  int ins;
  uint32_t id = map_get(&o->tmap, stream, tid, (uint32_t)o->nt, &ins);
  if (ins) {
    GROW(o->threads, o->nt, o->tcap);
    thread_t *t = &o->threads[o->nt++];
    memset(t, 0, sizeof *t);
    t->stream = stream; t->tid = tid;
  }
  return &o->threads[id];
}
static void tally_add(oracle *o, uint32_t stream, uint32_t tid, uint16_t fn,
                      uint64_t incl, uint64_t self, uint64_t bytes) {
  int ins;
  uint32_t id = map_get(&o->tally_map, ((uint64_t)stream << 32) | tid, fn, (uint32_t)o->ntal, &ins);
  if (ins) {
    GROW(o->tallies, o->ntal, o->talcap);
    tally_t *t = &o->tallies[o->ntal++];
    t->stream = stream; t->tid = tid; t->fn = fn;
    t->v[0] = 0; t->v[1] = 0; t->v[2] = UINT64_MAX; t->v[3] = 0;
    t->v[4] = 0; t->v[5] = UINT64_MAX; t->v[6] = 0; t->v[7] = 0;
  }
  tally_t *t = &o->tallies[id];
  t->v[0] += 1;
  t->v[1] += incl; if (incl < t->v[2]) t->v[2] = incl; if (incl > t->v[3]) t->v[3] = incl;
  t->v[4] += self; if (self < t->v[5]) t->v[5] = self; if (self > t->v[6]) t->v[6] = self;
  t->v[7] += bytes;
}
static void ktally_add(oracle *o, uint32_t stream, uint16_t kid, uint64_t dur) {
  int ins;
  uint32_t id = map_get(&o->kmap, stream, kid, (uint32_t)o->nkt, &ins);
  if (ins) {
    GROW(o->kt, o->nkt, o->ktcap);
    ktally_t *k = &o->kt[o->nkt++];
    k->stream = stream; k->kid = kid;
    k->v[0] = 0; k->v[1] = 0; k->v[2] = UINT64_MAX; k->v[3] = 0;
  }
  ktally_t *k = &o->kt[id];
  k->v[0] += 1; k->v[1] += dur;
  if (dur < k->v[2]) k->v[2] = dur;
  if (dur > k->v[3]) k->v[3] = dur;
}

void oracle_set_roles(oracle *o, const uint8_t *roles) { memcpy(o->roles, roles, o->n_fns); }

/* The payload analytics of one VAR16 record (see the header). */
static void payload_roles(oracle *o, uint32_t sid, uint16_t fn, uint8_t kind, const uint8_t *p, uint32_t plen) {
  if (kind > 1 || fn >= o->n_fns) return;
  const uint8_t role = o->roles[fn];
  int ins;
  if (role == 1 && kind == 0 && plen >= 24) {
    const uint64_t size = rd64(p), dst = rd64(p + 8), src = rd64(p + 16);
    const uint32_t dir = ((src >> 56) == 0xFF ? 2u : 0u) + ((dst >> 56) == 0xFF ? 1u : 0u);
    uint32_t id = map_get(&o->copy_map, ((uint64_t)sid << 32) | fn, dir, (uint32_t)o->ncp, &ins);
    if (ins) {
      GROW(o->cp, o->ncp, o->cpcap);
      copy_t *c = &o->cp[o->ncp++];
      c->stream = sid; c->fn = fn; c->dir = dir; c->count = 0; c->bytes = 0;
    }
    o->cp[id].count += 1;
    o->cp[id].bytes += size;
  } else if ((role == 2 && kind == 1 && plen >= 8) || (role == 3 && kind == 0 && plen >= 8)) {
    const uint64_t h = rd64(p);
    uint32_t id = map_get(&o->hmap, sid, h, (uint32_t)o->nhd, &ins);
    if (ins) {
      GROW(o->hd, o->nhd, o->hdcap);
      handle_t *x = &o->hd[o->nhd++];
      x->stream = sid; x->handle = h; x->creates = 0; x->releases = 0;
    }
    if (role == 2) o->hd[id].creates += 1;
    else o->hd[id].releases += 1;
  }
}

/* Validates a chunk like the library does; returns 0 or -1 (nothing changed). */
static int check_chunk(const oracle *o, const uint8_t *rec, size_t rb, const uint8_t *pay, size_t pb) {
  size_t rs = o->format == 2 ? 16 : 24;
  if (rb % rs) return -1;
  if (rb && !rec) return -1;
  if (o->format == 2) {
    uint64_t sum = 0;
    for (size_t i = 0; i < rb / rs; i++) sum += rec[i * rs + 15];
    if (sum != pb) return -1;
    if (pb && !pay) return -1;
  } else if (pb) {
    return -1;
  }
  return 0;
}

int oracle_submit(oracle *o, uint32_t trace, uint32_t host, uint32_t pid,
                  const uint8_t *rec, size_t rec_bytes, const uint8_t *pay, size_t pay_bytes) {
  if (check_chunk(o, rec, rec_bytes, pay, pay_bytes)) return -1;
  uint32_t sid = stream_of(o, trace, host, pid);
  size_t rs = o->format == 2 ? 16 : 24;
  size_t n = rec_bytes / rs;
  uint64_t poff = 0;
  for (size_t i = 0; i < n; i++) {
    stream_t *st = &o->streams[sid];
    const uint8_t *r = rec + i * rs;
    uint64_t ts = rd64(r);
    uint32_t tid = rd32(r + 8);
    uint16_t fn = rd16(r + 12);
    uint8_t kind = r[14];
    uint32_t plen = o->format == 2 ? r[15] : 0;
    const uint8_t *p = o->format == 2 ? pay + poff : NULL;
    poff += plen;
    st->st[S_RECORDS]++;
    if (o->format == 2) payload_roles(o, sid, fn, kind, p, plen);
    if (kind == 2) {
      uint64_t end;
      int ok = fn < o->n_kernel_ids;
      if (o->format == 2) { ok = ok && plen >= 8; end = ok ? rd64(p) : 0; }
      else end = rd64(r + 16);
      if (ok && end >= ts) {
        ktally_add(o, sid, fn, end - ts);
        st->st[S_KERNEL]++;
        st->has_record = 1;
      } else {
        st->st[S_BAD]++;
      }
      continue;
    }
    if (kind > 1 || fn >= o->n_fns) { st->st[S_BAD]++; continue; }
    st->has_record = 1;
    thread_t *t = thread_of(o, sid, tid);
    st = &o->streams[sid];
    if (t->seen && ts < t->last_ts) st->st[S_TSREG]++;
    t->seen = 1; t->last_ts = ts;
    if (kind == 0) {
      st->st[S_ENTRIES]++;
      uint64_t bytes = 0;
      if (o->format == 2 && o->has_size[fn] && plen >= 8) bytes = rd64(p);
      if (t->h == t->cap) { t->cap = t->cap ? t->cap * 2 : 16; t->stk = realloc(t->stk, t->cap * sizeof(frame_t)); }
      frame_t *f = &t->stk[t->h++];
      f->fn = fn; f->ts = ts; f->child = 0; f->bytes = bytes;
      if (t->h > o->max_depth) t->overflowed = 1;
    } else {
      st->st[S_EXITS]++;
      if (t->h == 0) { st->st[S_ORPHAN]++; continue; }
      frame_t e = t->stk[--t->h];
      if (e.fn != fn) { st->st[S_MISMATCH]++; continue; }
      if (ts < e.ts) { st->st[S_NEGDUR]++; continue; }
      uint64_t incl = ts - e.ts, self;
      if (e.child <= incl) self = incl - e.child;
      else { self = 0; st->st[S_SELFUNDER]++; }
      tally_add(o, sid, tid, fn, incl, self, e.bytes);
      if (o->keep_ivals) {
        GROW(o->iv, o->niv, o->ivcap);
        ival_t *v = &o->iv[o->niv++];
        v->stream = sid; v->tid = tid; v->fn = fn; v->depth = (uint32_t)t->h + 1;
        v->start = e.ts; v->end = ts;
        v->pstart = t->h ? t->stk[t->h - 1].ts : 0;
        v->pfn = t->h ? t->stk[t->h - 1].fn : 0xFFFFFFFFu;
        v->pad = 0;
      }
      if (t->h) t->stk[t->h - 1].child += incl;
    }
  }
  return 0;
}

/* A packed chunk (see the header): its packets are taken in index order,
 * each checked (magic, size, event count, events exactly filling it, packets
 * contiguous and covering the chunk) and its events passed on as one VAR16
 * chunk.  Returns 0, or -1 when the chunk is malformed (nothing changed). */
int oracle_submit_packed(oracle *o, uint32_t trace, uint32_t host, uint32_t pid, const uint8_t *buf,
                         size_t nbytes, const uint64_t *index, size_t n_packets) {
  if (o->format != 2) return -1;
  if ((nbytes && !buf) || (n_packets && !index) || (nbytes && !n_packets)) return -1;
  size_t nev = 0, npay = 0;
  for (int pass = 0; pass < 2; pass++) {
    uint8_t *hdr = NULL, *pay = NULL;
    if (pass == 1) {
      hdr = (uint8_t *)malloc(nev ? nev * 16 : 1);
      pay = (uint8_t *)malloc(npay ? npay : 1);
    }
    size_t ei = 0, pi = 0, expect = 0;
    for (size_t k = 0; k < n_packets; k++) {
      const uint64_t off = index[k];
      if (off != expect || off % 8 || off + 16 > nbytes) { free(hdr); free(pay); return -1; }
      const uint8_t *pk = buf + off;
      const uint32_t magic = rd32(pk), pbytes = rd32(pk + 4), pev = rd32(pk + 8), z = rd32(pk + 12);
      if (magic != 0x4B504854u || z || pbytes < 16 || pbytes % 8 || off + pbytes > nbytes) {
        free(hdr); free(pay); return -1;
      }
      size_t o2 = 16;
      for (uint32_t e = 0; e < pev; e++) {
        if (o2 + 16 > pbytes) { free(hdr); free(pay); return -1; }
        const uint32_t len = pk[o2 + 15];
        const size_t esz = (16 + len + 7) / 8 * 8;
        if (o2 + esz > pbytes) { free(hdr); free(pay); return -1; }
        if (pass == 1) {
          memcpy(hdr + ei * 16, pk + o2, 16);
          memcpy(pay + pi, pk + o2 + 16, len);
        }
        ei++;
        pi += len;
        o2 += esz;
      }
      if (o2 != pbytes) { free(hdr); free(pay); return -1; }
      expect = off + pbytes;
    }
    if (expect != nbytes) { free(hdr); free(pay); return -1; }
    if (pass == 0) { nev = ei; npay = pi; continue; }
    const int rc = oracle_submit(o, trace, host, pid, hdr, nev * 16, pay, npay);
    free(hdr); free(pay);
    return rc;
  }
  return -1;
}

/* Final flush: open entries are counted as unclosed and dropped. */
void oracle_finish(oracle *o) {
  for (size_t i = 0; i < o->nt; i++) {
    thread_t *t = &o->threads[i];
    o->streams[t->stream].st[S_UNCLOSED] += t->h;
    t->h = 0;
  }
}

/* ---------------------------------------------------------------- read */
typedef struct {
  uint32_t trace, host, pid, tid;
  uint16_t id; uint8_t row_kind; uint8_t pad; uint32_t pad2;
  uint64_t count, incl_sum, incl_min, incl_max, self_sum, self_min, self_max, bytes_sum;
} orow_t;

enum { SCOPE_THREAD = 1, SCOPE_PROCESS = 2, SCOPE_FN = 3, SCOPE_KERNEL = 4 };
#define ALL32 0xFFFFFFFFu

static int row_cmp(const void *x, const void *y) {
  const orow_t *a = (const orow_t *)x, *b = (const orow_t *)y;
#define C(f) if (a->f != b->f) return a->f < b->f ? -1 : 1;
  C(trace) C(host) C(pid) C(tid) C(row_kind) C(id)
#undef C
  return 0;
}

static void merge_into(orow_t *d, const uint64_t *v) {
  d->count += v[0];
  d->incl_sum += v[1]; if (v[2] < d->incl_min) d->incl_min = v[2]; if (v[3] > d->incl_max) d->incl_max = v[3];
  d->self_sum += v[4]; if (v[5] < d->self_min) d->self_min = v[5]; if (v[6] > d->self_max) d->self_max = v[6];
  d->bytes_sum += v[7];
}

/* All rows of a scope for a trace filter (ALL32 = every trace), in canonical
 * order.  Returns the row count; writes at most `cap` rows. */
size_t oracle_rows(oracle *o, int scope, uint32_t trace_filter, orow_t *out, size_t cap) {
  orow_t *rows = NULL; size_t n = 0, rcap = 0;
  if (scope == SCOPE_KERNEL) {
    for (size_t i = 0; i < o->nkt; i++) {
      ktally_t *k = &o->kt[i];
      stream_t *s = &o->streams[k->stream];
      if (trace_filter != ALL32 && s->trace != trace_filter) continue;
      GROW(rows, n, rcap);
      orow_t *r = &rows[n++];
      memset(r, 0, sizeof *r);
      r->trace = s->trace; r->host = s->host; r->pid = s->pid; r->tid = ALL32;
      r->id = (uint16_t)k->kid; r->row_kind = 2;
      r->count = k->v[0]; r->incl_sum = k->v[1]; r->incl_min = k->v[2]; r->incl_max = k->v[3];
    }
  } else {
    /* one row per finest key, with the summed-away fields blanked ... */
    for (size_t i = 0; i < o->ntal; i++) {
      tally_t *t = &o->tallies[i];
      stream_t *s = &o->streams[t->stream];
      if (trace_filter != ALL32 && s->trace != trace_filter) continue;
      GROW(rows, n, rcap);
      orow_t *r = &rows[n++];
      memset(r, 0, sizeof *r);
      r->trace = s->trace; r->host = s->host; r->pid = s->pid; r->tid = t->tid;
      if (scope == SCOPE_PROCESS) r->tid = ALL32;
      if (scope == SCOPE_FN) { r->host = ALL32; r->pid = ALL32; r->tid = ALL32; }
      r->id = (uint16_t)t->fn; r->row_kind = 1;
      r->incl_min = UINT64_MAX; r->self_min = UINT64_MAX;
      merge_into(r, t->v);
    }
    /* ... then sorted, and equal neighbours merged (sum, min, max) */
    if (n) qsort(rows, n, sizeof(orow_t), row_cmp);
    size_t m = 0;
    for (size_t i = 0; i < n; i++) {
      if (m && row_cmp(&rows[m - 1], &rows[i]) == 0) {
        uint64_t v[8] = {rows[i].count, rows[i].incl_sum, rows[i].incl_min, rows[i].incl_max,
                         rows[i].self_sum, rows[i].self_min, rows[i].self_max, rows[i].bytes_sum};
        merge_into(&rows[m - 1], v);
      } else {
        rows[m++] = rows[i];
      }
    }
    n = m;
  }
  if (n) qsort(rows, n, sizeof(orow_t), row_cmp);
  size_t w = n < cap ? n : cap;
  if (out && w) memcpy(out, rows, w * sizeof(orow_t));
  free(rows);
  return n;
}

/* Stats summed over the streams of a trace (ALL32 = all traces). */
void oracle_stats(oracle *o, uint32_t trace_filter, uint64_t *out) {
  memset(out, 0, S_N * sizeof(uint64_t));
  for (size_t i = 0; i < o->ns; i++) {
    stream_t *s = &o->streams[i];
    if (trace_filter != ALL32 && s->trace != trace_filter) continue;
    for (int k = 0; k < S_N; k++) out[k] += s->st[k];
  }
  out[S_OPEN] = 0;
  out[S_DEPTH] = 0;
  for (size_t i = 0; i < o->nt; i++) {
    thread_t *t = &o->threads[i];
    stream_t *s = &o->streams[t->stream];
    if (trace_filter != ALL32 && s->trace != trace_filter) continue;
    out[S_OPEN] += t->h;
    out[S_DEPTH] += t->overflowed ? 1 : 0;
    out[S_THREADS] += 1;
  }
  /* processes: streams with a valid record; hosts: distinct (trace, host) among them */
  map_t hosts; map_init(&hosts);
  for (size_t i = 0; i < o->ns; i++) {
    stream_t *s = &o->streams[i];
    if (trace_filter != ALL32 && s->trace != trace_filter) continue;
    if (!s->has_record) continue;
    out[S_PROCS] += 1;
    int ins;
    map_get(&hosts, s->trace, s->host, 0, &ins);
    if (ins) out[S_HOSTS] += 1;
  }
  map_free(&hosts);
}

uint64_t oracle_row_size(void) { return sizeof(orow_t); }

/* ----------------------------------------------------------- intervals */
void oracle_keep_intervals(oracle *o, int on) { o->keep_ivals = on; }

typedef struct {
  uint32_t trace, host, pid, tid;
  uint32_t fn, depth;
  uint64_t start, end, parent_start;
  uint32_t parent_fn, pad;
} oival_t;

static int ival_cmp(const void *x, const void *y) {
  const oival_t *a = (const oival_t *)x, *b = (const oival_t *)y;
#define C(f) if (a->f != b->f) return a->f < b->f ? -1 : 1;
  C(trace) C(host) C(pid) C(tid) C(start) C(depth) C(end) C(fn) C(parent_start) C(parent_fn)
#undef C
  return 0;
}

/* Every kept interval, sorted by (trace, host, pid, tid, start, depth, end,
 * fn, parent).  Returns the count; writes at most `cap`. */
size_t oracle_intervals(oracle *o, oival_t *out, size_t cap) {
  oival_t *v = (oival_t *)calloc(o->niv ? o->niv : 1, sizeof(oival_t));
  for (size_t i = 0; i < o->niv; i++) {
    const ival_t *a = &o->iv[i];
    const stream_t *s = &o->streams[a->stream];
    v[i].trace = s->trace; v[i].host = s->host; v[i].pid = s->pid; v[i].tid = a->tid;
    v[i].fn = a->fn; v[i].depth = a->depth; v[i].start = a->start; v[i].end = a->end;
    v[i].parent_start = a->pstart; v[i].parent_fn = a->pfn;
  }
  if (o->niv) qsort(v, o->niv, sizeof(oival_t), ival_cmp);
  size_t w = o->niv < cap ? o->niv : cap;
  if (out && w) memcpy(out, v, w * sizeof(oival_t));
  free(v);
  return o->niv;
}

uint64_t oracle_interval_size(void) { return sizeof(oival_t); }

/* ------------------------------------------------------ payload analytics */
typedef struct {
  uint32_t trace, host, pid, fn, dir, pad;
  uint64_t count, bytes;
} ocopy_t;
typedef struct {
  uint32_t trace, host, pid, pad;
  uint64_t creates, releases, handles, unreleased, unmatched;
} ohandle_t;

static int copy_cmp(const void *x, const void *y) {
  const ocopy_t *a = (const ocopy_t *)x, *b = (const ocopy_t *)y;
#define C(f) if (a->f != b->f) return a->f < b->f ? -1 : 1;
  C(trace) C(host) C(pid) C(fn) C(dir)
#undef C
  return 0;
}
static int handle_cmp(const void *x, const void *y) {
  const ohandle_t *a = (const ohandle_t *)x, *b = (const ohandle_t *)y;
#define C(f) if (a->f != b->f) return a->f < b->f ? -1 : 1;
  C(trace) C(host) C(pid)
#undef C
  return 0;
}

/* Copy tallies, one row per (stream, fn, direction) with entries, in order
 * (trace, host, pid, fn, dir). */
size_t oracle_copies(oracle *o, ocopy_t *out, size_t cap) {
  ocopy_t *v = (ocopy_t *)calloc(o->ncp ? o->ncp : 1, sizeof(ocopy_t));
  for (size_t i = 0; i < o->ncp; i++) {
    const copy_t *c = &o->cp[i];
    const stream_t *s = &o->streams[c->stream];
    v[i].trace = s->trace; v[i].host = s->host; v[i].pid = s->pid; v[i].fn = c->fn; v[i].dir = c->dir;
    v[i].count = c->count; v[i].bytes = c->bytes;
  }
  if (o->ncp) qsort(v, o->ncp, sizeof(ocopy_t), copy_cmp);
  if (out) memcpy(out, v, (o->ncp < cap ? o->ncp : cap) * sizeof(ocopy_t));
  free(v);
  return o->ncp;
}

/* The create / release join, one row per stream that had either, in order
 * (trace, host, pid): creates, releases, distinct handle values, handles
 * left unreleased and releases matching no create (summed over values). */
size_t oracle_handles(oracle *o, ohandle_t *out, size_t cap) {
  ohandle_t *v = (ohandle_t *)calloc(o->ns ? o->ns : 1, sizeof(ohandle_t));
  uint8_t *used = (uint8_t *)calloc(o->ns ? o->ns : 1, 1);
  for (size_t i = 0; i < o->nhd; i++) {
    const handle_t *h = &o->hd[i];
    ohandle_t *r = &v[h->stream];
    used[h->stream] = 1;
    r->creates += h->creates;
    r->releases += h->releases;
    r->handles += 1;
    if (h->creates > h->releases) r->unreleased += h->creates - h->releases;
    else r->unmatched += h->releases - h->creates;
  }
  size_t n = 0;
  for (size_t i = 0; i < o->ns; i++) {
    if (!used[i]) continue;
    const stream_t *s = &o->streams[i];
    v[i].trace = s->trace; v[i].host = s->host; v[i].pid = s->pid; v[i].pad = 0;
    v[n++] = v[i];
  }
  if (n) qsort(v, n, sizeof(ohandle_t), handle_cmp);
  if (out) memcpy(out, v, (n < cap ? n : cap) * sizeof(ohandle_t));
  free(v); free(used);
  return n;
}

uint64_t oracle_copy_size(void) { return sizeof(ocopy_t); }
uint64_t oracle_handle_size(void) { return sizeof(ohandle_t); }
