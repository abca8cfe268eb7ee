/*
 * Seeded synthetic genomes and reads.
 *
 * This module holds no part of the seeding method: it only draws the inputs that both the
 * CPU oracle and the GPU library consume (a reference over {A,C,G,T} and sequencing reads
 * sampled from it).  Everything is a deterministic function of (recipe, size, seed):
 * each segment / read draws from its own counter-derived SplitMix64 stream, so the
 * generation is parallel (OpenMP) and the output does not depend on the thread count.
 *
 * Base codes: A=0 C=1 G=2 T=3.  Reads are emitted as ASCII.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

/* ---------------- RNG: SplitMix64 (Steele, Lea, Flood 2014) ---------------- */
static inline uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
typedef struct { uint64_t s; } rng_t;
static inline rng_t rng_stream(uint64_t seed, uint64_t tag, uint64_t idx) {
  rng_t r; r.s = mix64(mix64(seed ^ (tag * 0xD1B54A32D192ED03ull)) ^ (idx * 0x8CB92BA72F3D8DD7ull)); return r;
}
static inline uint64_t rng_next(rng_t *r) { uint64_t z = r->s; r->s += 0x9E3779B97F4A7C15ull; return mix64(z); }
static inline double rng_unif(rng_t *r) { return (rng_next(r) >> 11) * (1.0 / 9007199254740992.0); }
static inline uint32_t rng_below(rng_t *r, uint32_t n) { return (uint32_t)(((rng_next(r) >> 32) * (uint64_t)n) >> 32); }
static inline double rng_normal(rng_t *r) {
  double u1 = rng_unif(r), u2 = rng_unif(r);
  if (u1 < 1e-300) u1 = 1e-300;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

enum { TAG_FAMILY = 1, TAG_SEG = 2, TAG_PLAN = 3, TAG_READ = 4, TAG_LEN = 5, TAG_SATFAM = 6, TAG_BS = 7 };

/* ---------------- mutation of a template (substitutions + 1-3 bp indels) ---------------- */
/* Walk src[0..len); per base, with prob p_sub substitute to a different base, with prob p_indel
 * start an indel event of length U{1,2,3} (insertion or deletion, 50/50).  Emits into dst (may be
 * NULL to count only).  Stops after max_out bases if max_out > 0.  Returns #bases emitted. */
static uint64_t mutate(const uint8_t *src, uint64_t len, double p_sub, double p_indel, rng_t *r,
                       uint8_t *dst, uint64_t max_out, uint64_t *consumed) {
  uint64_t o = 0, p = 0;
  while (p < len && (max_out == 0 || o < max_out)) {
    double u = rng_unif(r);
    if (u < p_indel) {
      uint32_t L = 1 + rng_below(r, 3);
      if (rng_next(r) & 1) { /* insertion of L random bases before src[p] */
        for (uint32_t t = 0; t < L && (max_out == 0 || o < max_out); ++t) { uint8_t b = (uint8_t)(rng_next(r) & 3); if (dst) dst[o] = b; ++o; }
      } else { /* deletion of src[p..p+L) */
        p += L;
      }
      continue;
    }
    uint8_t b = src[p++];
    if (u < p_indel + p_sub) b = (uint8_t)((b + 1 + rng_below(r, 3)) & 3);
    if (dst) dst[o] = b;
    ++o;
  }
  if (consumed) *consumed = p;
  return o;
}

static void revcomp_inplace(uint8_t *s, uint64_t n) {
  for (uint64_t i = 0, j = n ? n - 1 : 0; i < j; ++i, --j) { uint8_t t = s[i]; s[i] = (uint8_t)(3 - s[j]); s[j] = (uint8_t)(3 - t); }
  if (n & 1) s[n / 2] = (uint8_t)(3 - s[n / 2]);
}

/* ---------------- reference recipes ---------------- */
enum { SEG_RANDOM = 0, SEG_COPY = 1, SEG_SAT = 2 };
typedef struct {
  uint8_t type;      /* SEG_* */
  uint8_t orient;    /* 1 = reverse complement */
  uint32_t fam;      /* family index (copy: into fam table; sat: monomer family) */
  uint32_t units;    /* satellite: number of units */
  double div;        /* divergence */
  uint64_t len;      /* random: length; others: computed */
  uint64_t off;      /* output offset */
} seg_t;

typedef struct {
  int recipe;
  uint64_t seed, target, total;
  uint32_t nfam; uint8_t **fam; uint32_t *famlen;       /* interspersed repeat consensi */
  uint32_t nsat; uint8_t **sat;                          /* satellite monomer consensi (171 bp) */
  uint64_t nseg; seg_t *seg;
} ref_plan;

static void gen_random(uint8_t *dst, uint64_t len, rng_t *r) {
  uint64_t i = 0;
  while (i < len) { uint64_t w = rng_next(r); for (int t = 0; t < 32 && i < len; ++t, w >>= 2) dst[i++] = (uint8_t)(w & 3); }
}

#define SAT_UNIT 171
/* Fill (or count, if dst == NULL) segment g; returns its length. */
static uint64_t seg_fill(const ref_plan *pl, uint64_t g, uint8_t *dst) {
  const seg_t *s = &pl->seg[g];
  rng_t r = rng_stream(pl->seed, TAG_SEG, g);
  if (s->type == SEG_RANDOM) { if (dst) gen_random(dst, s->len, &r); return s->len; }
  if (s->type == SEG_COPY) {
    double pind = s->div * 0.1, psub = s->div * 0.9;
    uint64_t n = mutate(pl->fam[s->fam], pl->famlen[s->fam], psub, pind, &r, dst, 0, NULL);
    if (dst && s->orient) revcomp_inplace(dst, n);
    return n;
  }
  /* satellite array: array consensus = monomer family at 5% substitutions; units at s->div */
  uint8_t cons[SAT_UNIT];
  for (int t = 0; t < SAT_UNIT; ++t) {
    uint8_t b = pl->sat[s->fam][t];
    if (rng_unif(&r) < 0.05) b = (uint8_t)((b + 1 + rng_below(&r, 3)) & 3);
    cons[t] = b;
  }
  uint64_t n = 0;
  for (uint32_t u = 0; u < s->units; ++u)
    n += mutate(cons, SAT_UNIT, s->div * 0.9, s->div * 0.1, &r, dst ? dst + n : NULL, 0, NULL);
  if (dst && s->orient) revcomp_inplace(dst, n);
  return n;
}

static void plan_push(ref_plan *pl, uint64_t *cap, seg_t s) {
  if (pl->nseg == *cap) { *cap = *cap ? *cap * 2 : 1024; pl->seg = (seg_t *)realloc(pl->seg, *cap * sizeof(seg_t)); }
  pl->seg[pl->nseg++] = s;
}

/* recipe 0: `target` uniform random bases with 20 copies of one 2 kbp consensus at 5% divergence
 *           inserted at uniform cut points.
 * recipe 1: 55% random segments (length ~ Exp(mean 3 kbp)), 35% interspersed repeat copies (half
 *           from 300 bp families, half from 6 kbp families; divergence U[2%,20%], random
 *           orientation), 10% tandem satellite arrays of 171 bp units (U[20,2000] units, per-array
 *           divergence U[1%,3%]); segments shuffled.  Families x10 in count at >= 1 Gbp. */
ref_plan *synth_ref_plan(int recipe, uint64_t target, uint64_t seed) {
  ref_plan *pl = (ref_plan *)calloc(1, sizeof(ref_plan));
  pl->recipe = recipe; pl->seed = seed; pl->target = target;
  rng_t pr = rng_stream(seed, TAG_PLAN, 0);
  uint64_t cap = 0;
  if (recipe == 0) {
    pl->nfam = 1; pl->fam = (uint8_t **)malloc(sizeof(uint8_t *)); pl->famlen = (uint32_t *)malloc(4);
    pl->famlen[0] = 2000; pl->fam[0] = (uint8_t *)malloc(2000);
    rng_t fr = rng_stream(seed, TAG_FAMILY, 0); gen_random(pl->fam[0], 2000, &fr);
    uint64_t cuts[21]; cuts[0] = 0;
    for (int c = 1; c <= 20; ++c) cuts[c] = rng_next(&pr) % (target + 1);
    for (int a = 1; a <= 20; ++a) for (int b = a + 1; b <= 20; ++b) if (cuts[b] < cuts[a]) { uint64_t t = cuts[a]; cuts[a] = cuts[b]; cuts[b] = t; }
    for (int c = 0; c <= 20; ++c) {
      uint64_t end = c == 20 ? target : cuts[c + 1];
      seg_t s = {SEG_RANDOM, 0, 0, 0, 0.0, end - cuts[c], 0};
      plan_push(pl, &cap, s);
      if (c < 20) { seg_t cp = {SEG_COPY, (uint8_t)(rng_next(&pr) & 1), 0, 0, 0.05, 0, 0}; plan_push(pl, &cap, cp); }
    }
  } else {
    uint32_t scale = target >= 1000000000ull ? 10 : 1;
    uint32_t n300 = 30 * scale, n6k = 10 * scale;
    pl->nfam = n300 + n6k;
    pl->fam = (uint8_t **)malloc(pl->nfam * sizeof(uint8_t *)); pl->famlen = (uint32_t *)malloc(pl->nfam * 4);
    for (uint32_t f = 0; f < pl->nfam; ++f) {
      pl->famlen[f] = f < n300 ? 300 : 6000;
      pl->fam[f] = (uint8_t *)malloc(pl->famlen[f]);
      rng_t fr = rng_stream(seed, TAG_FAMILY, f); gen_random(pl->fam[f], pl->famlen[f], &fr);
    }
    pl->nsat = 5; pl->sat = (uint8_t **)malloc(pl->nsat * sizeof(uint8_t *));
    for (uint32_t f = 0; f < pl->nsat; ++f) { pl->sat[f] = (uint8_t *)malloc(SAT_UNIT); rng_t fr = rng_stream(seed, TAG_SATFAM, f); gen_random(pl->sat[f], SAT_UNIT, &fr); }
    double brand = 0.55 * target, b300 = 0.175 * target, b6k = 0.175 * target, bsat = 0.10 * target;
    for (double acc = 0; acc < brand;) {
      uint64_t L = (uint64_t)(-3000.0 * log(1.0 - rng_unif(&pr))) + 1;
      seg_t s = {SEG_RANDOM, 0, 0, 0, 0.0, L, 0}; plan_push(pl, &cap, s); acc += (double)L;
    }
    for (double acc = 0; acc < b300; acc += 300) {
      seg_t s = {SEG_COPY, (uint8_t)(rng_next(&pr) & 1), rng_below(&pr, n300), 0, 0.02 + 0.18 * rng_unif(&pr), 0, 0}; plan_push(pl, &cap, s);
    }
    for (double acc = 0; acc < b6k; acc += 6000) {
      seg_t s = {SEG_COPY, (uint8_t)(rng_next(&pr) & 1), n300 + rng_below(&pr, n6k), 0, 0.02 + 0.18 * rng_unif(&pr), 0, 0}; plan_push(pl, &cap, s);
    }
    for (double acc = 0; acc < bsat;) {
      uint32_t units = 20 + rng_below(&pr, 1981);
      seg_t s = {SEG_SAT, (uint8_t)(rng_next(&pr) & 1), rng_below(&pr, pl->nsat), units, 0.01 + 0.02 * rng_unif(&pr), 0, 0};
      plan_push(pl, &cap, s); acc += (double)units * SAT_UNIT;
    }
    /* Fisher-Yates shuffle of the segment order */
    for (uint64_t i = pl->nseg - 1; i > 0; --i) {
      uint64_t j = rng_next(&pr) % (i + 1);
      seg_t t = pl->seg[i]; pl->seg[i] = pl->seg[j]; pl->seg[j] = t;
    }
  }
  /* lengths (parallel), offsets, then pad / truncate to exactly `target` */
  #pragma omp parallel for schedule(dynamic, 64)
  for (int64_t g = 0; g < (int64_t)pl->nseg; ++g)
    if (pl->seg[g].type != SEG_RANDOM) pl->seg[g].len = seg_fill(pl, (uint64_t)g, NULL);
  uint64_t off = 0;
  for (uint64_t g = 0; g < pl->nseg; ++g) { pl->seg[g].off = off; off += pl->seg[g].len; }
  if (recipe != 0 && off < target) {
    seg_t s = {SEG_RANDOM, 0, 0, 0, 0.0, target - off, off}; plan_push(pl, &cap, s); off = target;
  }
  pl->total = recipe == 0 ? off : target;
  return pl;
}

uint64_t synth_ref_len(const ref_plan *pl) { return pl->total; }

/* Fill out[0..total) with base codes. */
void synth_ref_fill(const ref_plan *pl, uint8_t *out) {
  #pragma omp parallel
  {
    uint8_t *tmp = NULL; uint64_t tcap = 0;
    #pragma omp for schedule(dynamic, 16)
    for (int64_t g = 0; g < (int64_t)pl->nseg; ++g) {
      const seg_t *s = &pl->seg[g];
      if (s->off >= pl->total) continue;
      uint64_t keep = s->len;
      if (s->off + keep > pl->total) keep = pl->total - s->off;
      if (keep == s->len) { seg_fill(pl, (uint64_t)g, out + s->off); continue; }
      if (tcap < s->len) { free(tmp); tcap = s->len; tmp = (uint8_t *)malloc(tcap); }
      seg_fill(pl, (uint64_t)g, tmp);
      memcpy(out + s->off, tmp, keep);
    }
    free(tmp);
  }
}

/* Satellite intervals [beg, end) in reference coordinates; returns count, fills out (2 per) if non-NULL. */
uint64_t synth_ref_sats(const ref_plan *pl, uint64_t *out) {
  uint64_t c = 0;
  for (uint64_t g = 0; g < pl->nseg; ++g) {
    const seg_t *s = &pl->seg[g];
    if (s->type != SEG_SAT || s->off >= pl->total) continue;
    uint64_t e = s->off + s->len; if (e > pl->total) e = pl->total;
    if (out) { out[2 * c] = s->off; out[2 * c + 1] = e; }
    ++c;
  }
  return c;
}

void synth_ref_free(ref_plan *pl) {
  if (!pl) return;
  for (uint32_t f = 0; f < pl->nfam; ++f) free(pl->fam[f]);
  for (uint32_t f = 0; f < pl->nsat; ++f) free(pl->sat[f]);
  free(pl->fam); free(pl->famlen); free(pl->sat); free(pl->seg); free(pl);
}

/* ---------------- reads ---------------- */
static const char ACGT[4] = {'A', 'C', 'G', 'T'};

typedef struct {
  const uint8_t *ref; uint64_t ref_len;
  const uint64_t *sats; uint64_t nsat; double sat_frac;
  double p_sub, p_indel;
  uint64_t seed;
} read_ctx;

/* pick a fragment start uniformly (or inside a satellite interval with prob sat_frac) */
static uint64_t pick_start(const read_ctx *c, uint64_t flen, rng_t *r) {
  if (c->nsat && rng_unif(r) < c->sat_frac) {
    for (int tries = 0; tries < 8; ++tries) {
      uint64_t k = rng_next(r) % c->nsat;
      uint64_t b = c->sats[2 * k], e = c->sats[2 * k + 1];
      if (e - b >= flen) return b + rng_next(r) % (e - b - flen + 1);
    }
  }
  return rng_next(r) % (c->ref_len - flen + 1);
}

/* extract template (forward or reverse complement) into buf */
static void take(const read_ctx *c, uint64_t st, uint64_t len, int rev, uint8_t *buf) {
  memcpy(buf, c->ref + st, len);
  if (rev) revcomp_inplace(buf, len);
}

/* Simulate reads of fixed length `rlen` (paired if `paired`: n_frag pairs -> 2*n_frag reads,
 * read 2 = reverse complement of the fragment end; insert ~ round(N(ins_mean, ins_sd)) >= rlen).
 * Output: fixed stride `rlen` ASCII in out, actual lengths in lens (indels at the template end may
 * shorten a read), truth positions/strands (of read 1 / fragment) in tpos/tstrand (may be NULL). */
void synth_reads_fixed(const uint8_t *ref, uint64_t ref_len, const uint64_t *sats, uint64_t nsat, double sat_frac,
                       uint64_t n_frag, uint32_t rlen, int paired, double ins_mean, double ins_sd,
                       double p_sub, double p_indel, uint64_t seed,
                       char *out, uint32_t *lens, uint64_t *tpos, uint8_t *tstrand) {
  read_ctx c = {ref, ref_len, sats, nsat, sat_frac, p_sub, p_indel, seed};
  #pragma omp parallel
  {
    uint64_t cap = 0; uint8_t *tmpl = NULL, *rd = NULL;
    #pragma omp for schedule(static, 1024)
    for (int64_t f = 0; f < (int64_t)n_frag; ++f) {
      rng_t r = rng_stream(seed, TAG_READ, (uint64_t)f);
      uint64_t il = rlen;
      if (paired) {
        int64_t x = (int64_t)llround(ins_mean + ins_sd * rng_normal(&r));
        if (x > (int64_t)rlen) il = (uint64_t)x;
      }
      uint64_t flen = il + 32;
      if (flen > ref_len) flen = ref_len;
      if (il > flen) il = flen;
      if (cap < flen) { free(tmpl); free(rd); cap = flen; tmpl = (uint8_t *)malloc(cap); rd = (uint8_t *)malloc(cap + 8); }
      uint64_t st = pick_start(&c, flen, &r);
      int rev = (int)(rng_next(&r) & 1);
      take(&c, st, flen, rev, tmpl);
      uint64_t nr = paired ? 2 : 1;
      for (uint64_t m = 0; m < nr; ++m) {
        uint64_t id = (uint64_t)f * nr + m;
        uint64_t n;
        if (m == 0) {
          n = mutate(tmpl, flen, p_sub, p_indel, &r, rd, rlen, NULL);
        } else { /* mate: reverse complement of the insert, read from its far end */
          revcomp_inplace(tmpl, il);
          n = mutate(tmpl, il, p_sub, p_indel, &r, rd, rlen, NULL);
        }
        char *o = out + id * (uint64_t)rlen;
        for (uint64_t t = 0; t < n; ++t) o[t] = ACGT[rd[t]];
        for (uint64_t t = n; t < rlen; ++t) o[t] = 'N';
        lens[id] = (uint32_t)n;
        if (tpos) tpos[id] = st;
        if (tstrand) tstrand[id] = (uint8_t)(rev ^ (int)m);
      }
    }
    free(tmpl); free(rd);
  }
}

/* Variable-length single-end reads: lengths exp(N(ln median, sigma^2)) resampled into [lo, hi]. */
void synth_read_lengths(uint64_t n, double median, double sigma, uint32_t lo, uint32_t hi, uint64_t seed, uint32_t *lens) {
  #pragma omp parallel for schedule(static, 4096)
  for (int64_t i = 0; i < (int64_t)n; ++i) {
    rng_t r = rng_stream(seed, TAG_LEN, (uint64_t)i);
    for (;;) {
      double L = exp(log(median) + sigma * rng_normal(&r));
      if (L >= lo && L <= hi + 0.999999) { lens[i] = (uint32_t)L; break; }
    }
  }
}

/* Fill CSR reads with the given lengths (offsets[i] = start of read i in out). */
void synth_reads_var(const uint8_t *ref, uint64_t ref_len, uint64_t n, const uint32_t *lens, const uint64_t *offsets,
                     double p_sub, double p_indel, uint64_t seed, char *out, uint64_t *tpos, uint8_t *tstrand) {
  read_ctx c = {ref, ref_len, NULL, 0, 0.0, p_sub, p_indel, seed};
  #pragma omp parallel
  {
    uint64_t cap = 0; uint8_t *tmpl = NULL, *rd = NULL;
    #pragma omp for schedule(dynamic, 256)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
      rng_t r = rng_stream(seed, TAG_READ, (uint64_t)i);
      uint64_t rl = lens[i];
      uint64_t flen = rl + rl / 16 + 32;
      if (flen > ref_len) flen = ref_len;
      if (cap < flen) { free(tmpl); free(rd); cap = flen; tmpl = (uint8_t *)malloc(cap); rd = (uint8_t *)malloc(cap + 8); }
      uint64_t st = pick_start(&c, flen, &r);
      int rev = (int)(rng_next(&r) & 1);
      take(&c, st, flen, rev, tmpl);
      uint64_t got = mutate(tmpl, flen, p_sub, p_indel, &r, rd, rl, NULL);
      char *o = out + offsets[i];
      for (uint64_t t = 0; t < got; ++t) o[t] = ACGT[rd[t]];
      for (uint64_t t = got; t < rl; ++t) o[t] = ACGT[rng_next(&r) & 3]; /* template exhausted: pad randomly */
      if (tpos) tpos[i] = st;
      if (tstrand) tstrand[i] = (uint8_t)rev;
    }
    free(tmpl); free(rd);
  }
}

/* Directional bisulfite reads (read-1 form), fixed length: strand OT/OB 50/50; on the source
 * strand each C is converted to T with probability p_cpg if followed by G, else p_noncpg; then
 * errors.  Output fixed stride like synth_reads_fixed. */
void synth_reads_bs(const uint8_t *ref, uint64_t ref_len, uint64_t n, uint32_t rlen, double p_cpg, double p_noncpg,
                    double p_sub, double p_indel, uint64_t seed, char *out, uint32_t *lens, uint64_t *tpos, uint8_t *tstrand) {
  read_ctx c = {ref, ref_len, NULL, 0, 0.0, p_sub, p_indel, seed};
  #pragma omp parallel
  {
    uint64_t flen = rlen + 33;
    uint8_t *tmpl = (uint8_t *)malloc(flen), *rd = (uint8_t *)malloc(flen + 8);
    #pragma omp for schedule(static, 1024)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
      rng_t r = rng_stream(seed, TAG_BS, (uint64_t)i);
      uint64_t st = pick_start(&c, flen, &r);
      int rev = (int)(rng_next(&r) & 1);
      take(&c, st, flen, rev, tmpl);
      for (uint64_t t = 0; t + 1 < flen; ++t)
        if (tmpl[t] == 1) { double p = tmpl[t + 1] == 2 ? p_cpg : p_noncpg; if (rng_unif(&r) < p) tmpl[t] = 3; }
      uint64_t got = mutate(tmpl, flen - 1, p_sub, p_indel, &r, rd, rlen, NULL);
      char *o = out + (uint64_t)i * rlen;
      for (uint64_t t = 0; t < got; ++t) o[t] = ACGT[rd[t]];
      for (uint64_t t = got; t < rlen; ++t) o[t] = 'N';
      lens[i] = (uint32_t)got;
      if (tpos) tpos[i] = st;
      if (tstrand) tstrand[i] = (uint8_t)rev;
    }
    free(tmpl); free(rd);
  }
}
