/*
 * synth.c -- seeded synthetic API-trace generator.
 *
 * Produces the bytes of one trace stream (one (trace, host, pid) key): the
 * entry/exit records of every thread of that process, merged in timestamp
 * order, plus device-kernel records for layered workloads.  It models the
 * traces of the paper's evaluation (section 5): stacked programming-model
 * layers (section 1, section 4.3: a portable model on a runtime on a driver),
 * heavy call-count skew and durations from hundreds of ns to ms (the tally
 * of section 4.3), and typed argument payloads with pointers, sizes and names
 * (the event record printed in section 1.1).
 *
 * This module is an INPUT generator only.  It encodes records; it never
 * matches exits to entries, never computes a duration sum and never tallies.
 * For test pins it can also hand back the explicit list of calls it planned
 * (thread, fn, entry ts, exit ts, parent), which is the tree it generated,
 * not a result derived from the record stream.
 *
 * Random numbers: splitmix64 (seeding) and xoshiro256** (Blackman & Vigna,
 * "Scrambled linear pseudorandom number generators", 2021), written from
 * their published definitions.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ RNG */
static uint64_t sm64_next(uint64_t *s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
typedef struct { uint64_t s[4]; } rng_t;
static inline uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
static uint64_t rng_u64(rng_t *r) {
  uint64_t *s = r->s;
  uint64_t out = rotl64(s[1] * 5, 7) * 9;
  uint64_t t = s[1] << 17;
  s[2] ^= s[0];
  s[3] ^= s[1];
  s[1] ^= s[2];
  s[0] ^= s[3];
  s[2] ^= t;
  s[3] = rotl64(s[3], 45);
  return out;
}
static void rng_seed(rng_t *r, uint64_t a, uint64_t b, uint64_t c) {
  uint64_t sm = a ^ (b * 0xD1B54A32D192ED03ull) ^ (c * 0x8CB92BA72F3D8DD7ull);
  for (int i = 0; i < 4; i++) r->s[i] = sm64_next(&sm);
}
/* uniform in [0,1) with 53 random bits */
static double rng_unif(rng_t *r) { return (double)(rng_u64(r) >> 11) * (1.0 / 9007199254740992.0); }
/* uniform integer in [lo, hi] (multiply-high, no modulo) */
static uint64_t rng_range(rng_t *r, uint64_t lo, uint64_t hi) {
  uint64_t n = hi - lo + 1;
  __uint128_t m = (__uint128_t)rng_u64(r) * n;
  return lo + (uint64_t)(m >> 64);
}
static double rng_normal(rng_t *r) {
  /* Box-Muller, one output per call */
  double u1 = rng_unif(r), u2 = rng_unif(r);
  if (u1 < 1e-300) u1 = 1e-300;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}
/* exponential with the given mean, floored to integer ns (0 allowed) */
static uint64_t rng_exp_ns(rng_t *r, double mean) {
  double v = -mean * log(1.0 - rng_unif(r));
  return (uint64_t)floor(v);
}
/* lognormal(mu, sigma), rounded to nearest ns, at least 1 */
static uint64_t rng_lognormal_ns(rng_t *r, double mu, double sigma) {
  double v = exp(mu + sigma * rng_normal(r));
  if (v > 1e15) v = 1e15;
  uint64_t x = (uint64_t)llround(v);
  return x < 1 ? 1 : x;
}

/* Zipf(s=1) sampler over n ranks via its cumulative table */
typedef struct { int n; double *cdf; } zipf_t;
static void zipf_init(zipf_t *z, int n) {
  z->n = n;
  z->cdf = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  double acc = 0;
  for (int i = 0; i < n; i++) { acc += 1.0 / (double)(i + 1); z->cdf[i] = acc; }
  for (int i = 0; i < n; i++) z->cdf[i] /= acc;
}
static int zipf_draw(const zipf_t *z, rng_t *r) {
  double u = rng_unif(r);
  int lo = 0, hi = z->n - 1;
  while (lo < hi) { int mid = (lo + hi) >> 1; if (z->cdf[mid] > u) hi = mid; else lo = mid + 1; }
  return lo;
}

/* ------------------------------------------------------------ workload */
typedef struct {
  int32_t layered;      /* 0: one layer of n_fns; 1: portable -> runtime -> driver */
  int32_t n_fns;        /* single layer: fns [0, n_fns) */
  int32_t n_portable, n_runtime, n_driver; /* layered split (fn ids consecutive) */
  int32_t max_depth;    /* top level is depth 1 */
  double p_child;       /* probability of another child, while depth < max_depth */
  double dur_mu, dur_sigma; /* lognormal of a leaf, and of a parent's tail after its last child */
  double gap_mean;      /* exponential gap before each child and between top-level calls */
  int32_t rt_min, rt_max;   /* runtime calls per portable call */
  int32_t drv_min, drv_max; /* driver calls per runtime call */
  double p_launch;      /* expected device kernels launched per runtime call */
  int32_t n_kernel_ids, n_queues;
  double k_mu, k_sigma; /* lognormal kernel duration */
  int32_t format;       /* 1 = fixed 24-byte records, 2 = 16-byte header + payload heap */
  int32_t payload_max;  /* VAR16: payload_len ~ U{0..payload_max} */
  double p_has_size;    /* VAR16: share of fns whose payload starts with a u64 size */
  uint64_t t0;          /* epoch of the stream, ns */
  double start_jitter;  /* per-thread start offset U[0, start_jitter) ns */
} synth_cfg;

typedef struct {        /* one planned call, for test pins */
  uint32_t thread;      /* thread index within the stream */
  uint16_t fn;
  uint16_t depth;
  int64_t parent;       /* index into the call list, -1 for top level */
  uint64_t t_entry, t_exit;
} synth_call;

typedef struct { uint64_t ts; uint16_t fn; uint8_t kind; uint8_t pad; uint32_t call; } ev_t;
typedef struct { uint64_t launch; uint32_t thread; uint16_t kid; } launch_t;

typedef struct {
  const synth_cfg *cfg;
  rng_t rng;
  zipf_t zf, zp, zr, zd;
  ev_t *ev; size_t nev, cap;
  launch_t *ln; size_t nln, lncap;
  synth_call *calls; size_t ncalls, callcap; int want_calls;
  uint32_t thread;
  uint64_t t;
} gen_t;

static void push_ev(gen_t *g, uint16_t fn, uint8_t kind, uint32_t call) {
  if (g->nev == g->cap) { g->cap = g->cap ? g->cap * 2 : 4096; g->ev = (ev_t *)realloc(g->ev, g->cap * sizeof(ev_t)); }
  ev_t *e = &g->ev[g->nev++];
  e->ts = g->t; e->fn = fn; e->kind = kind; e->pad = 0; e->call = call;
}
static uint32_t new_call(gen_t *g, uint16_t fn, uint16_t depth, int64_t parent) {
  if (!g->want_calls) return 0;
  if (g->ncalls == g->callcap) { g->callcap = g->callcap ? g->callcap * 2 : 4096; g->calls = (synth_call *)realloc(g->calls, g->callcap * sizeof(synth_call)); }
  synth_call *c = &g->calls[g->ncalls];
  c->thread = g->thread; c->fn = fn; c->depth = depth; c->parent = parent; c->t_entry = g->t; c->t_exit = 0;
  return (uint32_t)g->ncalls++;
}
static void close_call(gen_t *g, uint32_t id) { if (g->want_calls) g->calls[id].t_exit = g->t; }

static void gen_simple(gen_t *g, int depth, int64_t parent) {
  const synth_cfg *c = g->cfg;
  uint16_t fn = (uint16_t)zipf_draw(&g->zf, &g->rng);
  uint32_t id = new_call(g, fn, (uint16_t)depth, parent);
  push_ev(g, fn, 0, id);
  while (depth < c->max_depth && rng_unif(&g->rng) < c->p_child) {
    g->t += rng_exp_ns(&g->rng, c->gap_mean);
    gen_simple(g, depth + 1, g->want_calls ? (int64_t)id : -1);
  }
  g->t += rng_lognormal_ns(&g->rng, c->dur_mu, c->dur_sigma);
  close_call(g, id);
  push_ev(g, fn, 1, id);
}

static void gen_driver(gen_t *g, int depth, int64_t parent) {
  const synth_cfg *c = g->cfg;
  uint16_t fn = (uint16_t)(c->n_portable + c->n_runtime + zipf_draw(&g->zd, &g->rng));
  uint32_t id = new_call(g, fn, (uint16_t)depth, parent);
  push_ev(g, fn, 0, id);
  while (depth < c->max_depth && rng_unif(&g->rng) < c->p_child) {
    g->t += rng_exp_ns(&g->rng, c->gap_mean);
    gen_driver(g, depth + 1, g->want_calls ? (int64_t)id : -1);
  }
  g->t += rng_lognormal_ns(&g->rng, c->dur_mu, c->dur_sigma);
  close_call(g, id);
  push_ev(g, fn, 1, id);
}

static void gen_runtime(gen_t *g, int depth, int64_t parent) {
  const synth_cfg *c = g->cfg;
  uint16_t fn = (uint16_t)(c->n_portable + zipf_draw(&g->zr, &g->rng));
  uint32_t id = new_call(g, fn, (uint16_t)depth, parent);
  push_ev(g, fn, 0, id);
  int nd = (int)rng_range(&g->rng, (uint64_t)c->drv_min, (uint64_t)c->drv_max);
  for (int i = 0; i < nd && depth < c->max_depth; i++) {
    g->t += rng_exp_ns(&g->rng, c->gap_mean);
    gen_driver(g, depth + 1, g->want_calls ? (int64_t)id : -1);
  }
  g->t += rng_lognormal_ns(&g->rng, c->dur_mu, c->dur_sigma);
  close_call(g, id);
  push_ev(g, fn, 1, id);
  /* p_launch is the expected number of kernels a runtime call launches:
   * floor(p_launch) kernels, plus one more with probability frac(p_launch) */
  if (c->n_kernel_ids > 0 && c->p_launch > 0) {
    int nk = (int)floor(c->p_launch);
    if (rng_unif(&g->rng) < c->p_launch - floor(c->p_launch)) nk++;
    for (int k = 0; k < nk; k++) {
      if (g->nln == g->lncap) { g->lncap = g->lncap ? g->lncap * 2 : 1024; g->ln = (launch_t *)realloc(g->ln, g->lncap * sizeof(launch_t)); }
      launch_t *l = &g->ln[g->nln++];
      l->launch = g->t; l->thread = g->thread;
      l->kid = (uint16_t)rng_range(&g->rng, 0, (uint64_t)c->n_kernel_ids - 1);
    }
  }
}

static void gen_portable(gen_t *g) {
  const synth_cfg *c = g->cfg;
  uint16_t fn = (uint16_t)zipf_draw(&g->zp, &g->rng);
  uint32_t id = new_call(g, fn, 1, -1);
  push_ev(g, fn, 0, id);
  int nr = (int)rng_range(&g->rng, (uint64_t)c->rt_min, (uint64_t)c->rt_max);
  for (int i = 0; i < nr; i++) {
    g->t += rng_exp_ns(&g->rng, c->gap_mean);
    gen_runtime(g, 2, g->want_calls ? (int64_t)id : -1);
  }
  g->t += rng_lognormal_ns(&g->rng, c->dur_mu, c->dur_sigma);
  close_call(g, id);
  push_ev(g, fn, 1, id);
}

/* ------------------------------------------------------------ streams */
typedef struct {
  uint8_t *rec; uint64_t rec_bytes;
  uint8_t *pay; uint64_t pay_bytes;
  synth_call *calls; uint64_t ncalls;
  uint64_t n_api, n_kernel;
} synth_stream;

typedef struct { uint64_t key; uint32_t src; uint32_t idx; } mrg_t;

static int cmp_launch(const void *a, const void *b) {
  const launch_t *x = (const launch_t *)a, *y = (const launch_t *)b;
  if (x->launch != y->launch) return x->launch < y->launch ? -1 : 1;
  return x->thread < y->thread ? -1 : (x->thread > y->thread);
}

static void put_u64(uint8_t *p, uint64_t v) { memcpy(p, &v, 8); }
static void put_u32(uint8_t *p, uint32_t v) { memcpy(p, &v, 4); }
static void put_u16(uint8_t *p, uint16_t v) { memcpy(p, &v, 2); }

static const char NAME_ALPHA[] = "ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789_";

/* payload for one VAR16 record: a leading u64 (size or kernel end) when
 * `lead` is set, then pointer-like u64 words, then a name */
static void fill_payload(rng_t *r, uint8_t *p, int len, int lead, uint64_t lead_val) {
  int o = 0;
  if (lead && len >= 8) { put_u64(p, lead_val); o = 8; }
  int nptr = 0;
  while (len - o >= 8 && nptr < 2) {
    uint64_t v = rng_u64(r);
    uint64_t ptr = (v & 1) ? (0xff00000000000000ull | (v >> 16 << 4))
                           : (0x00007f0000000000ull | ((v >> 24) << 4 & 0xffffffffffull));
    put_u64(p + o, ptr); o += 8; nptr++;
  }
  while (o < len) { p[o++] = (uint8_t)NAME_ALPHA[rng_range(r, 0, sizeof(NAME_ALPHA) - 2)]; }
}

/* fn_has_size flags for a workload: a seeded share p of the fns */
void synth_has_size(uint64_t seed, int n_fns, double p, uint8_t *out) {
  rng_t r; rng_seed(&r, seed, 0x51CEull, 7);
  for (int i = 0; i < n_fns; i++) out[i] = rng_unif(&r) < p ? 1 : 0;
}

synth_stream *synth_stream_new(const synth_cfg *cfg, uint64_t seed, uint32_t stream_no, uint32_t pid,
                               uint32_t n_threads, uint64_t api_quota, int want_calls,
                               const uint8_t *has_size) {
  synth_stream *out = (synth_stream *)calloc(1, sizeof(synth_stream));
  gen_t g; memset(&g, 0, sizeof g);
  g.cfg = cfg; g.want_calls = want_calls;
  if (cfg->layered) {
    zipf_init(&g.zp, cfg->n_portable); zipf_init(&g.zr, cfg->n_runtime); zipf_init(&g.zd, cfg->n_driver);
  } else {
    zipf_init(&g.zf, cfg->n_fns);
  }
  uint64_t per_thread = n_threads ? (api_quota + n_threads - 1) / n_threads : 0;
  size_t *th_start = (size_t *)calloc(n_threads + 1, sizeof(size_t));
  for (uint32_t th = 0; th < n_threads; th++) {
    rng_seed(&g.rng, seed, stream_no + 1, th + 1);
    g.thread = th;
    g.t = cfg->t0 + (uint64_t)floor(rng_unif(&g.rng) * cfg->start_jitter);
    th_start[th] = g.nev;
    while ((uint64_t)(g.nev - th_start[th]) < per_thread) {
      g.t += rng_exp_ns(&g.rng, cfg->gap_mean);
      if (cfg->layered) gen_portable(&g); else gen_simple(&g, 1, -1);
    }
  }
  th_start[n_threads] = g.nev;
  /* device kernels: launches of the process in launch order, queues serialised */
  rng_t kr; rng_seed(&kr, seed, stream_no + 1, 0xC0DEull);
  qsort(g.ln, g.nln, sizeof(launch_t), cmp_launch);
  uint64_t *kstart = (uint64_t *)malloc(sizeof(uint64_t) * (g.nln + 1));
  uint64_t *kend = (uint64_t *)malloc(sizeof(uint64_t) * (g.nln + 1));
  uint32_t *kq = (uint32_t *)malloc(sizeof(uint32_t) * (g.nln + 1));
  uint64_t qfree[64]; memset(qfree, 0, sizeof qfree);
  int nq = cfg->n_queues > 0 ? (cfg->n_queues < 64 ? cfg->n_queues : 64) : 1;
  for (size_t i = 0; i < g.nln; i++) {
    uint32_t q = (uint32_t)rng_range(&kr, 0, (uint64_t)nq - 1);
    uint64_t s = g.ln[i].launch > qfree[q] ? g.ln[i].launch : qfree[q];
    uint64_t e = s + rng_lognormal_ns(&kr, cfg->k_mu, cfg->k_sigma);
    qfree[q] = e; kstart[i] = s; kend[i] = e; kq[i] = q;
  }
  /* kernels are emitted in end-time order: stable bottom-up merge sort by end */
  mrg_t *kk = (mrg_t *)malloc(sizeof(mrg_t) * (g.nln + 1));
  for (size_t i = 0; i < g.nln; i++) { kk[i].key = kend[i]; kk[i].src = 0; kk[i].idx = (uint32_t)i; }
  {
    mrg_t *tmp = (mrg_t *)malloc(sizeof(mrg_t) * (g.nln + 1));
    for (size_t w = 1; w < g.nln; w *= 2) {
      for (size_t lo = 0; lo < g.nln; lo += 2 * w) {
        size_t mid = lo + w < g.nln ? lo + w : g.nln, hi = lo + 2 * w < g.nln ? lo + 2 * w : g.nln;
        size_t a = lo, b = mid, o = lo;
        while (a < mid && b < hi) tmp[o++] = (kk[b].key < kk[a].key) ? kk[b++] : kk[a++];
        while (a < mid) tmp[o++] = kk[a++];
        while (b < hi) tmp[o++] = kk[b++];
      }
      mrg_t *sw = kk; kk = tmp; tmp = sw;
    }
    free(tmp);
  }
  uint64_t total = g.nev + g.nln;
  size_t rs = cfg->format == 2 ? 16 : 24;
  out->rec = (uint8_t *)malloc(total * rs + 1);
  out->rec_bytes = total * rs;
  out->n_api = g.nev; out->n_kernel = g.nln;
  size_t *head = (size_t *)malloc(sizeof(size_t) * (n_threads + 1));
  for (uint32_t th = 0; th < n_threads; th++) head[th] = th_start[th];
  /* binary min-heap of thread heads keyed by (ts, thread) */
  uint32_t *hp = (uint32_t *)malloc(sizeof(uint32_t) * (n_threads + 1));
  uint32_t hn = 0;
#define HKEY_LT(a, b) (g.ev[head[a]].ts < g.ev[head[b]].ts || (g.ev[head[a]].ts == g.ev[head[b]].ts && (a) < (b)))
  for (uint32_t th = 0; th < n_threads; th++) {
    if (head[th] >= th_start[th + 1]) continue;
    uint32_t i = hn++; hp[i] = th;
    while (i > 0) { uint32_t p = (i - 1) / 2; if (HKEY_LT(hp[i], hp[p])) { uint32_t t = hp[i]; hp[i] = hp[p]; hp[p] = t; i = p; } else break; }
  }
  size_t kh = 0;
  uint32_t tid_base = pid + 1;
  uint64_t pay_cap = cfg->format == 2 ? total * (uint64_t)(cfg->payload_max > 0 ? cfg->payload_max : 1) + 1 : 1;
  if (cfg->format == 2) out->pay = (uint8_t *)malloc(pay_cap);
  uint64_t pay_off = 0;
  rng_t pr; rng_seed(&pr, seed, stream_no + 1, 0x9A71ull);
  for (uint64_t o = 0; o < total; o++) {
    /* smallest head: (ts, thread) for API records; kernels sort after threads on ties */
    int best = hn ? (int)hp[0] : -1;
    uint64_t bts = hn ? g.ev[head[hp[0]]].ts : UINT64_MAX;
    int take_kernel = 0;
    if (kh < g.nln) {
      uint64_t ke = kk[kh].key;
      if (best < 0 || ke < bts) take_kernel = 1;
    }
    uint8_t *r = out->rec + o * rs;
    memset(r, 0, rs);
    if (take_kernel) {
      size_t ki = kk[kh++].idx;
      put_u64(r, kstart[ki]); put_u32(r + 8, kq[ki]); put_u16(r + 12, g.ln[ki].kid); r[14] = 2;
      if (cfg->format == 1) {
        put_u64(r + 16, kend[ki]);
      } else {
        int len = (int)rng_range(&pr, 8, (uint64_t)(cfg->payload_max >= 8 ? cfg->payload_max : 8));
        r[15] = (uint8_t)len;
        fill_payload(&pr, out->pay + pay_off, len, 1, kend[ki]);
        pay_off += (uint64_t)len;
      }
    } else {
      ev_t *e = &g.ev[head[best]++];
      /* re-heapify the head thread */
      if (head[best] >= th_start[best + 1]) { hp[0] = hp[--hn]; }
      {
        uint32_t i = 0;
        for (;;) {
          uint32_t l = 2 * i + 1, rr = l + 1, m = i;
          if (l < hn && HKEY_LT(hp[l], hp[m])) m = l;
          if (rr < hn && HKEY_LT(hp[rr], hp[m])) m = rr;
          if (m == i) break;
          uint32_t t = hp[i]; hp[i] = hp[m]; hp[m] = t; i = m;
        }
      }
      put_u64(r, e->ts);
      put_u32(r + 8, tid_base + (uint32_t)best * 7919u);
      put_u16(r + 12, e->fn);
      r[14] = e->kind;
      if (cfg->format == 2) {
        int len = (int)rng_range(&pr, 0, (uint64_t)cfg->payload_max);
        r[15] = (uint8_t)len;
        int lead = e->kind == 0 && has_size && has_size[e->fn];
        uint64_t sz = 0;
        if (lead) {
          double lv = rng_unif(&pr) * log(1073741824.0);
          sz = (uint64_t)floor(exp(lv));
          if (sz < 1) sz = 1;
        }
        fill_payload(&pr, out->pay + pay_off, len, lead, sz);
        pay_off += (uint64_t)len;
      }
    }
  }
  out->pay_bytes = pay_off;
  if (want_calls) { out->calls = g.calls; out->ncalls = g.ncalls; g.calls = NULL; }
  free(hp); free(head); free(kk); free(kstart); free(kend); free(kq);
  free(th_start); free(g.ev); free(g.ln); free(g.calls);
  free(g.zf.cdf); free(g.zp.cdf); free(g.zr.cdf); free(g.zd.cdf);
  return out;
}

void synth_stream_sizes(const synth_stream *s, uint64_t *rec_bytes, uint64_t *pay_bytes, uint64_t *ncalls,
                        uint64_t *n_api, uint64_t *n_kernel) {
  *rec_bytes = s->rec_bytes; *pay_bytes = s->pay_bytes; *ncalls = s->ncalls;
  *n_api = s->n_api; *n_kernel = s->n_kernel;
}
void synth_stream_copy(const synth_stream *s, uint8_t *rec, uint8_t *pay, synth_call *calls) {
  if (rec && s->rec_bytes) memcpy(rec, s->rec, s->rec_bytes);
  if (pay && s->pay_bytes) memcpy(pay, s->pay, s->pay_bytes);
  if (calls && s->ncalls) memcpy(calls, s->calls, s->ncalls * sizeof(synth_call));
}
void synth_stream_free(synth_stream *s) {
  if (!s) return;
  free(s->rec); free(s->pay); free(s->calls); free(s);
}
uint64_t synth_call_size(void) { return sizeof(synth_call); }
uint64_t synth_cfg_size(void) { return sizeof(synth_cfg); }

/* ------------------------------------------------- payload roles, packing */
/* Handles in the payloads of a VAR16 stream (in place), for functions given
 * a role: the exit of a create function (role 2) with payload_len >= 8
 * returns a fresh handle (host-like values, 16 apart); the entry of a release
 * function (role 3) with payload_len >= 8 takes, with probability p_bogus, a
 * value never created, else one of the handles created so far in this stream
 * (uniformly, so some are released twice and some never). */
void synth_apply_handles(uint8_t *hdr, uint64_t n, uint8_t *pay, const uint8_t *roles, uint32_t n_fns,
                         uint64_t seed, double p_bogus) {
  rng_t r;
  rng_seed(&r, seed, 0x48414E44u, n);
  uint64_t *pool = NULL, np = 0, cap = 0, off = 0;
  for (uint64_t i = 0; i < n; i++) {
    uint8_t *h = hdr + i * 16;
    const uint32_t len = h[15];
    const uint16_t fn = (uint16_t)(h[12] | (h[13] << 8));
    const uint8_t kind = h[14];
    const uint8_t role = fn < n_fns ? roles[fn] : 0;
    if (len >= 8 && role == 2 && kind == 1) {
      const uint64_t v = 0x0000000005000000ull + 16 * np;
      put_u64(pay + off, v);
      if (np == cap) { cap = cap ? cap * 2 : 1024; pool = (uint64_t *)realloc(pool, cap * 8); }
      pool[np++] = v;
    } else if (len >= 8 && role == 3 && kind == 0) {
      uint64_t v;
      if (!np || rng_unif(&r) < p_bogus) v = 0x0000000007000000ull + 16 * rng_range(&r, 0, 1u << 20);
      else v = pool[rng_range(&r, 0, np - 1)];
      put_u64(pay + off, v);
    }
    off += len;
  }
  free(pool);
}

/* Packed form of a VAR16 stream: packets of up to `per_packet` events, each a
 * 16-byte header {magic "THPK", packet bytes, events, 0} and its events, every
 * event its 16-byte header and payload, padded with zeros to 8 bytes.  With
 * buf / index NULL only the sizes are returned (*nbytes, *npackets). */
void synth_pack(const uint8_t *hdr, uint64_t n, const uint8_t *pay, uint32_t per_packet, uint8_t *buf,
                uint64_t *index, uint64_t *nbytes, uint64_t *npackets) {
  uint64_t o = 0, pk = 0, poff = 0;
  for (uint64_t i = 0; i < n; i += per_packet) {
    const uint64_t e1 = i + per_packet < n ? i + per_packet : n;
    const uint64_t start = o;
    o += 16;
    for (uint64_t j = i; j < e1; j++) {
      const uint32_t len = hdr[j * 16 + 15];
      const uint64_t sz = (16 + len + 7) / 8 * 8;
      if (buf) {
        memcpy(buf + o, hdr + j * 16, 16);
        memcpy(buf + o + 16, pay + poff, len);
        memset(buf + o + 16 + len, 0, sz - 16 - len);
      }
      poff += len;
      o += sz;
    }
    if (buf) {
      const uint32_t h[4] = {0x4B504854u, (uint32_t)(o - start), (uint32_t)(e1 - i), 0};
      memcpy(buf + start, h, 16);
      index[pk] = start;
    }
    pk++;
  }
  *nbytes = o;
  *npackets = pk;
}
