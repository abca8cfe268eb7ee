/*
 * ORACLE — test infrastructure only.
 *
 * A plain, slow CPU statement of what the seeding path computes, used to check the GPU library
 * element by element.  Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this code; the product library never does.  It shares no code, header, table or
 * helper with the GPU path.
 *
 * Paper: "Fast genomic read alignment with minibwa" (arXiv 2606.15357).
 *
 *   Definitions (Section 2.1):
 *     T = R . revcomp(R) . $,  n = |T|, $ smaller than A<C<G<T            -> build_text()
 *     S(i) = start of the i-th smallest suffix (suffix array)              -> sort_suffixes()
 *     B[i] = T[S(i) - 1], with T[-1] = $                                   -> orc_build()
 *     pi(a, k) = |{i : B[i] < a}| + |{i < k : B[i] = a}|                   -> fm_pi()
 *     ds-interval (lo(P), lo(revcomp P), occ(P)), lo(P) = |{i : T[i,n) < P}|,
 *       occ(P) = |{i : T[i, i+|P|) = P}|                                    -> def_interval()
 *     (l,c)-match / (l,c)-SMEM (containment-maximal matches)              -> def_smems()
 *   Algorithm 1 (BackwardExt / ForwardExt)                                 -> fm_backward(), fm_forward()
 *   Algorithm 2 (LocateSlow over an SA sampled at multiples of r)          -> fm_locate_slow()
 *   Algorithm 3 (BatchFindSMEM stages 1-3 with BackStep), one query at a time -> alg3_smems()
 *   Section 2.6 (two seeding rounds: re-seed long, rare SMEMs)             -> seed_query()
 *   Section 2.9 (bisulfite: 3-base index of C->T(R) . G->A(R), read conversion, strand filter)
 *   Section 2.7 (mate-rescue prefilter: q-mer matches per diagonal, M_t)  -> rescue_diag()
 *
 * Two oracles live here:
 *   O1 ("definition"): full suffix array by comparison sort; intervals by binary search over the
 *       full SA; SMEMs from the definition via e(i) = max{ j : occ(P[i,j)) >= c }; positions read
 *       straight from the full SA.
 *   O2 ("paper algorithm"): an FM-index (one byte per BWT symbol, counts every 64 symbols) with
 *       Algorithm 1, a serial Algorithm 3, and Algorithm 2's LocateSlow over a sampled SA.  It also
 *       counts the index lines a given line layout would touch (the algorithmic traffic).
 *
 * Symbol coding inside the oracle: $ = 0, A = 1, C = 2, G = 3, T = 4; a read byte outside ACGT
 * becomes 5, which equals no text symbol (so no match ever spans it).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#include <omp.h>

typedef struct {
  uint64_t n;        /* |T| */
  uint64_t len_r;    /* |R| of the original reference */
  int bisulfite;     /* 1: T built from C->T(R) . G->A(R) */
  uint8_t *T;        /* n symbols, T[n-1] = $ */
  uint64_t *SA;      /* full suffix array (O1) */
  uint8_t *B;        /* BWT */
  uint64_t C[6];     /* C[a] = |{i : B[i] < a}| */
  uint64_t primary;  /* the row whose BWT symbol is $ (S(primary) = 0) */
  uint64_t *occ64;   /* O2: occ64[5*(x/64) + a] = |{i < 64*(x/64) : B[i] = a}| */
  int r;             /* O2: SA sampling rate */
  uint64_t *ssa;     /* O2: ssa[x/r] = S(x) for x % r == 0 */
} orc_index;

/* ------------------------------------------------------------------------------------------ */
/* T = R . revcomp(R) . $   (Section 2.1).  In bisulfite mode R is first replaced by
 * C->T(R) . G->A(R)  (Section 2.9), so T holds the four converted copies.                    */
static uint8_t *build_text(const uint8_t *R, uint64_t len_r, int bisulfite, uint64_t *n_out) {
  uint64_t lr = bisulfite ? 2 * len_r : len_r;
  uint64_t n = 2 * lr + 1;
  uint8_t *T = (uint8_t *)malloc(n);
  for (uint64_t i = 0; i < len_r; ++i) {
    uint8_t a = (uint8_t)(R[i] + 1);                 /* 0..3 -> A..T = 1..4 */
    if (bisulfite) {
      T[i] = a == 2 ? 4 : a;                          /* C -> T */
      T[len_r + i] = a == 3 ? 1 : a;                  /* G -> A */
    } else {
      T[i] = a;
    }
  }
  for (uint64_t i = 0; i < lr; ++i) T[lr + i] = (uint8_t)(5 - T[lr - 1 - i]); /* complement: A<->T, C<->G */
  T[n - 1] = 0;
  *n_out = n;
  return T;
}

/* ------------------------------------------------------------------------------------------ */
/* Suffix array by sorting (definition of S in Section 2.1): positions ordered by the suffix
 * T[i,n).  Suffixes are first bucketed by their first 8 symbols (base-5 digits, $ = 0, padding
 * after $ = 0: distinct suffixes that reach $ inside the window get distinct keys because $
 * occurs once), buckets are visited in key order, and each bucket is sorted by direct suffix
 * comparison.  memcmp never returns 0 for i != j since $ is unique and smallest.               */
static const uint8_t *g_T;
static uint64_t g_n;
static int cmp_suffix(const void *pa, const void *pb) {
  uint64_t i = *(const uint64_t *)pa, j = *(const uint64_t *)pb;
  uint64_t li = g_n - i, lj = g_n - j;
  int c = memcmp(g_T + i, g_T + j, li < lj ? li : lj);
  return c < 0 ? -1 : c > 0 ? 1 : (li < lj ? -1 : 1);
}
#define BK 8
static uint32_t bucket_key(const uint8_t *T, uint64_t n, uint64_t i) {
  uint32_t k = 0;
  for (int t = 0; t < BK; ++t) k = k * 5 + (i + t < n ? T[i + t] : 0);
  return k;
}
static uint64_t *sort_suffixes(const uint8_t *T, uint64_t n) {
  uint64_t nb = 390625; /* 5^8 */
  uint64_t *cnt = (uint64_t *)calloc(nb + 1, sizeof(uint64_t));
  uint32_t *key = (uint32_t *)malloc(n * sizeof(uint32_t));
  #pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)n; ++i) key[i] = bucket_key(T, n, (uint64_t)i);
  for (uint64_t i = 0; i < n; ++i) cnt[key[i] + 1]++;
  for (uint64_t b = 0; b < nb; ++b) cnt[b + 1] += cnt[b];
  uint64_t *SA = (uint64_t *)malloc(n * sizeof(uint64_t));
  uint64_t *fill = (uint64_t *)malloc(nb * sizeof(uint64_t));
  memcpy(fill, cnt, nb * sizeof(uint64_t));
  for (uint64_t i = 0; i < n; ++i) SA[fill[key[i]]++] = i;
  free(fill); free(key);
  g_T = T; g_n = n;
  #pragma omp parallel for schedule(dynamic, 64)
  for (int64_t b = 0; b < (int64_t)nb; ++b) {
    uint64_t lo = cnt[b], hi = cnt[b + 1];
    if (hi - lo > 1) qsort(SA + lo, hi - lo, sizeof(uint64_t), cmp_suffix);
  }
  free(cnt);
  return SA;
}

/* ------------------------------------------------------------------------------------------ */
orc_index *orc_build(const uint8_t *R, uint64_t len_r, int bisulfite, int sa_rate) {
  orc_index *ix = (orc_index *)calloc(1, sizeof(orc_index));
  ix->len_r = len_r; ix->bisulfite = bisulfite; ix->r = sa_rate > 0 ? sa_rate : 1;
  ix->T = build_text(R, len_r, bisulfite, &ix->n);
  uint64_t n = ix->n;
  ix->SA = sort_suffixes(ix->T, n);
  ix->B = (uint8_t *)malloc(n);
  for (uint64_t x = 0; x < n; ++x) {                 /* B[x] = T[S(x) - 1], T[-1] = $ */
    uint64_t s = ix->SA[x];
    ix->B[x] = s ? ix->T[s - 1] : 0;
    if (!s) ix->primary = x;
  }
  uint64_t tot[6] = {0};
  for (uint64_t x = 0; x < n; ++x) tot[ix->B[x]]++;
  ix->C[0] = 0;
  for (int a = 1; a < 6; ++a) ix->C[a] = ix->C[a - 1] + tot[a - 1];
  /* O2 structures: counts every 64 rows and the SA sampled at multiples of r */
  uint64_t nblk = n / 64 + 2;
  ix->occ64 = (uint64_t *)calloc(nblk * 5, sizeof(uint64_t));
  uint64_t run[5] = {0};
  for (uint64_t x = 0; x <= n; ++x) {
    if (x % 64 == 0) memcpy(ix->occ64 + 5 * (x / 64), run, sizeof(run));
    if (x < n) run[ix->B[x]]++;
  }
  uint64_t ns = (n + ix->r - 1) / ix->r;
  ix->ssa = (uint64_t *)malloc(ns * sizeof(uint64_t));
  for (uint64_t x = 0; x < n; x += ix->r) ix->ssa[x / ix->r] = ix->SA[x];
  return ix;
}

void orc_free(orc_index *ix) {
  if (!ix) return;
  free(ix->T); free(ix->SA); free(ix->B); free(ix->occ64); free(ix->ssa); free(ix);
}

uint64_t orc_n(const orc_index *ix) { return ix->n; }
uint64_t orc_primary(const orc_index *ix) { return ix->primary; }
void orc_copy_text(const orc_index *ix, uint8_t *out) { memcpy(out, ix->T, ix->n); }
void orc_copy_sa(const orc_index *ix, uint64_t *out) { memcpy(out, ix->SA, ix->n * 8); }
void orc_copy_bwt(const orc_index *ix, uint8_t *out) { memcpy(out, ix->B, ix->n); }
void orc_copy_c(const orc_index *ix, uint64_t *out) { memcpy(out, ix->C, sizeof(ix->C)); }

/* ------------------------------------------------------------------------------------------ */
/* O1: ds-interval by its definition (Section 2.1) using binary search over the full SA.       */

/* compare suffix T[i,n) with pattern P[0,m) over the first m symbols:
 * <0 if T[i,n) < P with a difference in the first m symbols (or $ reached), 0 if P is a prefix
 * of T[i,n), >0 otherwise. */
static int cmp_prefix(const orc_index *ix, uint64_t i, const uint8_t *P, uint64_t m) {
  for (uint64_t t = 0; t < m; ++t) {
    uint8_t a = ix->T[i + t], b = P[t];   /* T[n-1] = $ = 0 < b, so i+t never passes n-1 */
    if (a != b) return a < b ? -1 : 1;
  }
  return 0;
}
/* first SA row whose suffix is >= P (strict=0) or > every suffix having prefix P (strict=1) */
static uint64_t sa_bound(const orc_index *ix, const uint8_t *P, uint64_t m, int strict) {
  uint64_t lo = 0, hi = ix->n;
  while (lo < hi) {
    uint64_t mid = lo + (hi - lo) / 2;
    int c = cmp_prefix(ix, ix->SA[mid], P, m);
    if (c < 0 || (strict && c == 0)) lo = mid + 1; else hi = mid;
  }
  return lo;
}
static void revcomp_sym(const uint8_t *P, uint64_t m, uint8_t *out) {
  for (uint64_t t = 0; t < m; ++t) { uint8_t a = P[m - 1 - t]; out[t] = a >= 1 && a <= 4 ? (uint8_t)(5 - a) : a; }
}
/* (lo(P), lo(revcomp P), occ(P)) */
static void def_interval(const orc_index *ix, const uint8_t *P, uint64_t m, uint64_t out[3]) {
  uint8_t *Q = (uint8_t *)malloc(m + 1);
  revcomp_sym(P, m, Q);
  uint64_t a = sa_bound(ix, P, m, 0), b = sa_bound(ix, P, m, 1);
  out[0] = a; out[1] = sa_bound(ix, Q, m, 0); out[2] = b - a;
  free(Q);
}

/* exported: interval of an ASCII pattern (for tests) */
static uint8_t enc_ascii(uint8_t ch) {
  switch (ch) { case 'A': case 'a': return 1; case 'C': case 'c': return 2; case 'G': case 'g': return 3;
                case 'T': case 't': return 4; default: return 5; }
}
void orc_interval_ascii(const orc_index *ix, const uint8_t *p, uint64_t m, uint64_t out[3]) {
  uint8_t *P = (uint8_t *)malloc(m + 1);
  for (uint64_t t = 0; t < m; ++t) P[t] = enc_ascii(p[t]);
  def_interval(ix, P, m, out);
  free(P);
}

/* Given the SA range [lo,hi) of P[0,len), narrow it to P[0,len+1) (all suffixes in the range
 * share the prefix, so only the symbol at offset len is compared). */
static void narrow(const orc_index *ix, uint64_t *lo, uint64_t *hi, uint64_t len, uint8_t b) {
  uint64_t a = *lo, z = *hi;
  while (a < z) { uint64_t mid = a + (z - a) / 2; if (ix->T[ix->SA[mid] + len] < b) a = mid + 1; else z = mid; }
  uint64_t L = a; z = *hi;
  while (a < z) { uint64_t mid = a + (z - a) / 2; if (ix->T[ix->SA[mid] + len] <= b) a = mid + 1; else z = mid; }
  *lo = L; *hi = a;
}

typedef struct { uint32_t qbeg, qend; uint64_t k, kr, s; } smem_t;
typedef struct { smem_t *v; uint64_t n, cap; } smem_vec;
static void push_smem(smem_vec *V, smem_t x) {
  if (V->n == V->cap) { V->cap = V->cap ? 2 * V->cap : 16; V->v = (smem_t *)realloc(V->v, V->cap * sizeof(smem_t)); }
  V->v[V->n++] = x;
}

/* (l,c)-SMEMs of P[0,m) from the definition (Section 2.1): with e(i) = max{ j >= i :
 * occ(P[i,j)) >= c } (occ of the empty string is n), the SMEMs are exactly the intervals
 * [i, e(i)) with e(i) - i >= l and (i == 0 or e(i-1) < e(i)).  Coordinates are shifted by `base`. */
static void def_smems(const orc_index *ix, const uint8_t *P, uint64_t m, int l, uint64_t c, uint32_t base, smem_vec *out) {
  uint64_t eprev = 0;
  for (uint64_t i = 0; i < m; ++i) {
    uint64_t j = i > 0 && eprev > i ? eprev : i;
    uint64_t lo, hi;
    if (j > i) { lo = sa_bound(ix, P + i, j - i, 0); hi = sa_bound(ix, P + i, j - i, 1); }
    else { lo = 0; hi = ix->n; }
    if (hi - lo < c) { eprev = j; continue; } /* only when c > n */
    while (j < m) {
      uint64_t a = lo, z = hi;
      narrow(ix, &a, &z, j - i, P[j]);
      if (z - a < c) break;
      lo = a; hi = z; ++j;
    }
    if ((i == 0 || eprev < j) && j - i >= (uint64_t)l) {
      uint64_t iv[3];
      def_interval(ix, P + i, j - i, iv);
      smem_t s = {(uint32_t)(base + i), (uint32_t)(base + j), iv[0], iv[1], iv[2]};
      push_smem(out, s);
    }
    eprev = j;
  }
}

/* ------------------------------------------------------------------------------------------ */
/* O2: FM-index primitives and Algorithm 1.                                                    */

typedef struct {             /* algorithmic line counting for a given index line layout */
  uint64_t bases_per_line;   /* rows of B covered by one index line (0 = do not count) */
  uint64_t lines;            /* extension + LF lines touched */
  uint64_t kmer_lookups;     /* one line each */
  uint64_t sa_reads;         /* one SA-sample read each */
  uint64_t steps;            /* extension steps (Algorithm 1 calls) */
  uint64_t lf_steps;         /* LF steps in locate */
} line_ctr;

/* Occ(a, k) = |{i < k : B[i] = a}| from the 64-row checkpoints and a scan of B. */
static inline uint64_t fm_occ(const orc_index *ix, uint8_t a, uint64_t k) {
  uint64_t v = ix->occ64[5 * (k / 64) + a];
  for (uint64_t x = k & ~63ull; x < k; ++x) v += ix->B[x] == a;
  return v;
}
/* pi(a, k) = |{i : B[i] < a}| + |{i < k : B[i] = a}|  (Section 2.1) */
static inline uint64_t fm_pi(const orc_index *ix, uint8_t a, uint64_t k) { return ix->C[a] + fm_occ(ix, a, k); }

static inline void count_step(line_ctr *lc, uint64_t x1, uint64_t x2) {
  if (!lc) return;
  lc->steps++;
  if (!lc->bases_per_line) return;
  lc->lines += (x1 / lc->bases_per_line == x2 / lc->bases_per_line) ? 1 : 2;
}

/* Algorithm 1, BackwardExt: ds-interval of aP from that of P.  Symbols b range over $ and the
 * bases smaller than the complement of a; comp($) = $. */
static void fm_backward(const orc_index *ix, uint64_t iv[3], uint8_t a, line_ctr *lc) {
  uint64_t k = iv[0], kr = iv[1], s = iv[2];
  if (a < 1 || a > 4) { iv[0] = 0; iv[1] = 0; iv[2] = 0; return; } /* a read symbol that matches nothing */
  count_step(lc, k, k + s);
  uint8_t abar = (uint8_t)(5 - a);
  for (uint8_t b = 0; b < abar; ++b) {               /* b = $, A, ... (b < comp(a)) */
    uint8_t bbar = b == 0 ? 0 : (uint8_t)(5 - b);
    kr += fm_pi(ix, bbar, k + s) - fm_pi(ix, bbar, k);
  }
  uint64_t lo = fm_pi(ix, a, k);
  s = fm_pi(ix, a, k + s) - lo;
  iv[0] = lo; iv[1] = kr; iv[2] = s;
}
/* Algorithm 1, ForwardExt: ds-interval of Pa = BackwardExt on the swapped interval with comp(a). */
static void fm_forward(const orc_index *ix, uint64_t iv[3], uint8_t a, line_ctr *lc) {
  uint64_t sw[3] = {iv[1], iv[0], iv[2]};
  uint8_t abar = a >= 1 && a <= 4 ? (uint8_t)(5 - a) : a;
  fm_backward(ix, sw, abar, lc);
  iv[0] = sw[1]; iv[1] = sw[0]; iv[2] = sw[2];
}

/* Optional k-mer shortcut (Section 2.5: the ds-intervals of all k-mers are precomputed so that
 * the first k single steps of a backward run are replaced by one lookup).  The oracle computes
 * the looked-up value with k BackwardExt calls but counts one line for it.  When the k-mer's
 * occurrence count is below c the run falls back to single steps from the start, so the result
 * never depends on the shortcut. */

/* ------------------------------------------------------------------------------------------ */
/* Algorithm 3 for one query string P[0,m).  The batched queue of the paper interleaves many
 * queries; records of one query are processed in order, so running the queue for one query at
 * a time yields the same SMEMs.  Records are (stage u, i, j, interval). */
static void alg3_smems(const orc_index *ix, const uint8_t *P, uint64_t m, int l, uint64_t c, int kmer_k,
                       uint32_t base, smem_vec *out, line_ctr *lc) {
  if (!((uint64_t)(l - 1) < m)) return;              /* Alg. 3 initialisation: needs l-1 < |P| */
  int u = 1;
  int64_t i = 0, j = l - 1;
  uint64_t iv[3] = {0, 0, ix->n};
  int fresh = 1;                                      /* interval is the initial (0,0,|B|) */
  for (;;) {
    if (u == 1 || u == 3) {
      if (u == 1 && j < i) { u = 2; j = i + l; fresh = 0; continue; }           /* stage 1 -> 2 */
      if (u == 3 && j <= i) { u = 1; i = j + 1; j = j + l; iv[0] = 0; iv[1] = 0; iv[2] = ix->n; fresh = 1; continue; }
      /* k-mer shortcut at the start of a backward run */
      if (fresh && kmer_k > 0 && j - kmer_k + 1 >= (u == 1 ? i : i + 1)) {
        uint64_t t[3] = {0, 0, ix->n};
        for (int q = 0; q < kmer_k; ++q) fm_backward(ix, t, P[j - q], NULL);
        if (lc) lc->kmer_lookups++;
        if (t[2] >= c) { iv[0] = t[0]; iv[1] = t[1]; iv[2] = t[2]; j -= kmer_k; fresh = 0; continue; }
      }
      fresh = 0;
      /* BackStep */
      uint64_t nv[3] = {iv[0], iv[1], iv[2]};
      fm_backward(ix, nv, P[j], lc);
      if (nv[2] >= c) { iv[0] = nv[0]; iv[1] = nv[1]; iv[2] = nv[2]; j -= 1; continue; }
      if ((uint64_t)(j + l) < m) { u = 1; i = j + 1; j = j + l; iv[0] = 0; iv[1] = 0; iv[2] = ix->n; fresh = 1; continue; }
      return;
    }
    /* stage 2: forward extension to the SMEM end */
    if ((uint64_t)j == m) {
      smem_t s = {(uint32_t)(base + i), (uint32_t)(base + j), iv[0], iv[1], iv[2]};
      push_smem(out, s);
      return;
    }
    uint64_t nv[3] = {iv[0], iv[1], iv[2]};
    fm_forward(ix, nv, P[j], lc);
    if (nv[2] >= c) { iv[0] = nv[0]; iv[1] = nv[1]; iv[2] = nv[2]; j += 1; continue; }
    smem_t s = {(uint32_t)(base + i), (uint32_t)(base + j), iv[0], iv[1], iv[2]};
    push_smem(out, s);
    u = 3; iv[0] = 0; iv[1] = 0; iv[2] = ix->n; fresh = 1;   /* j stays: the mismatching symbol */
  }
}

/* Algorithm 2, LocateSlow for one row k: LF-walk until the row is a multiple of r, then add the
 * number of steps to the sampled value.  LF of the $ row goes to row 0 (pi($, k) = 0), whose
 * suffix starts at n-1, so the sum is taken mod n. */
static uint64_t fm_locate_slow(const orc_index *ix, uint64_t k, line_ctr *lc) {
  uint64_t i = 0;
  while (k % ix->r != 0) {
    if (lc) { lc->lf_steps++; if (lc->bases_per_line) lc->lines++; }
    uint8_t b = ix->B[k];
    k = fm_pi(ix, b, k);
    ++i;
  }
  if (lc) lc->sa_reads++;
  return (i + ix->ssa[k / ix->r]) % ix->n;
}

/* ------------------------------------------------------------------------------------------ */
/* Seeding of one query (Section 2.6): round 1 = (l,c)-SMEMs; round 2: for every round-1 SMEM
 * [i,j) with j-i >= reseed_len and occurrence s <= reseed_occ, the (floor((j-i)/2), s+1)-SMEMs of
 * P[i,j).  Union with duplicates (same [qbeg,qend)) removed; sorted by (qbeg, qend). */
typedef struct {
  int min_len;         /* l */
  int min_occ;         /* c */
  int max_occ;         /* locate only seeds with s <= max_occ */
  int reseed;          /* run round 2 */
  int reseed_len;      /* 38 */
  int reseed_occ;      /* 10 */
  int bs_role;         /* 0 plain, 1 read-1 (C->T), 2 read-2 (G->A) */
  int method;          /* 0 = O1 definition, 1 = O2 Algorithm 3 */
  int kmer_k;          /* O2 only */
  int bases_per_line;  /* O2 line counting, 0 = off */
} orc_opts;

static int cmp_smem(const void *a, const void *b) {
  const smem_t *x = (const smem_t *)a, *y = (const smem_t *)b;
  if (x->qbeg != y->qbeg) return x->qbeg < y->qbeg ? -1 : 1;
  if (x->qend != y->qend) return x->qend < y->qend ? -1 : 1;
  return 0;
}
static void find_smems(const orc_index *ix, const uint8_t *P, uint64_t m, int l, uint64_t c, const orc_opts *o,
                       uint32_t base, smem_vec *out, line_ctr *lc) {
  if (o->method == 0) def_smems(ix, P, m, l, c, base, out);
  else alg3_smems(ix, P, m, l, c, o->kmer_k, base, out, lc);
}
static void seed_query(const orc_index *ix, const uint8_t *P, uint64_t m, const orc_opts *o, smem_vec *out, line_ctr *lc) {
  out->n = 0;
  find_smems(ix, P, m, o->min_len, (uint64_t)o->min_occ, o, 0, out, lc);
  if (o->reseed) {
    uint64_t n1 = out->n;
    for (uint64_t t = 0; t < n1; ++t) {
      smem_t s = out->v[t];
      if (s.qend - s.qbeg >= (uint32_t)o->reseed_len && s.s <= (uint64_t)o->reseed_occ)
        find_smems(ix, P + s.qbeg, s.qend - s.qbeg, (int)((s.qend - s.qbeg) / 2), s.s + 1, o, s.qbeg, out, lc);
    }
  }
  if (out->n > 1) qsort(out->v, out->n, sizeof(smem_t), cmp_smem);
  uint64_t w = 0;
  for (uint64_t t = 0; t < out->n; ++t)
    if (w == 0 || cmp_smem(&out->v[w - 1], &out->v[t]) != 0) out->v[w++] = out->v[t];
  out->n = w;
}

/* ------------------------------------------------------------------------------------------ */
/* Batch driver: reads are ASCII, CSR (offsets[n_reads+1]).  Results are returned in a handle:
 * seeds sorted by (read, qbeg, qend), each seed's positions ascending.                        */
typedef struct {
  uint64_t n_seeds, n_pos;
  uint32_t *read_id, *qbeg, *qend, *npos, *flags;
  uint64_t *k, *kr, *s, *pos_off, *pos;
  line_ctr lines;
} orc_result;

static int cmp_u64(const void *a, const void *b) {
  uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
  return x < y ? -1 : x > y;
}

/* segment of T (bisulfite index): 0 fwd C->T, 1 fwd G->A, 2 rev G->A, 3 rev C->T (Section 2.9) */
static inline int bs_keep(const orc_index *ix, int role, uint64_t pos) {
  uint64_t seg = pos / ix->len_r;
  if (role == 1) return seg == 0 || seg == 2;
  if (role == 2) return seg == 1 || seg == 3;
  return 1;
}

orc_result *orc_seed(const orc_index *ix, const uint8_t *reads, const uint64_t *offsets, uint64_t n_reads,
                     const orc_opts *o, int n_threads) {
  if (n_threads > 0) omp_set_num_threads(n_threads);
  int nt = omp_get_max_threads();
  smem_vec *per = (smem_vec *)calloc(n_reads, sizeof(smem_vec));
  uint64_t **ppos = (uint64_t **)calloc(n_reads, sizeof(uint64_t *));   /* kept positions, seed by seed */
  uint32_t **pcnt = (uint32_t **)calloc(n_reads, sizeof(uint32_t *));   /* kept count per seed */
  line_ctr *tl = (line_ctr *)calloc((size_t)nt, sizeof(line_ctr));
  #pragma omp parallel
  {
    int tid = omp_get_thread_num();
    line_ctr *lc = &tl[tid];
    lc->bases_per_line = (uint64_t)(o->bases_per_line > 0 ? o->bases_per_line : 0);
    uint8_t *P = NULL; uint64_t pcap = 0;
    #pragma omp for schedule(dynamic, 16)
    for (int64_t r = 0; r < (int64_t)n_reads; ++r) {
      uint64_t b = offsets[r], m = offsets[r + 1] - b;
      if (pcap < m + 1) { free(P); pcap = m + 1; P = (uint8_t *)malloc(pcap); }
      for (uint64_t t = 0; t < m; ++t) {
        uint8_t a = enc_ascii(reads[b + t]);
        if (o->bs_role == 1 && a == 2) a = 4;          /* read 1: C -> T */
        if (o->bs_role == 2 && a == 3) a = 1;          /* read 2: G -> A */
        P[t] = a;
      }
      seed_query(ix, P, m, o, &per[r], o->method == 1 ? lc : NULL);
      uint64_t tot = 0;
      for (uint64_t q = 0; q < per[r].n; ++q) if (per[r].v[q].s <= (uint64_t)o->max_occ) tot += per[r].v[q].s;
      uint64_t *pp = (uint64_t *)malloc((tot ? tot : 1) * sizeof(uint64_t));
      uint32_t *pc = (uint32_t *)calloc(per[r].n + 1, sizeof(uint32_t));
      uint64_t w = 0;
      for (uint64_t q = 0; q < per[r].n; ++q) {
        smem_t *s = &per[r].v[q];
        if (s->s > (uint64_t)o->max_occ) continue;
        uint64_t w0 = w;
        for (uint64_t x = s->k; x < s->k + s->s; ++x) {
          uint64_t p = o->method == 0 ? ix->SA[x] : fm_locate_slow(ix, x, lc);
          if (bs_keep(ix, o->bs_role, p)) pp[w++] = p;
        }
        qsort(pp + w0, w - w0, sizeof(uint64_t), cmp_u64);
        pc[q] = (uint32_t)(w - w0);
      }
      ppos[r] = pp; pcnt[r] = pc;
    }
    free(P);
  }
  orc_result *res = (orc_result *)calloc(1, sizeof(orc_result));
  uint64_t ns = 0, np = 0;
  for (uint64_t r = 0; r < n_reads; ++r) { ns += per[r].n; for (uint64_t q = 0; q < per[r].n; ++q) np += pcnt[r][q]; }
  res->n_seeds = ns; res->n_pos = np;
  res->read_id = (uint32_t *)malloc((ns + 1) * 4); res->qbeg = (uint32_t *)malloc((ns + 1) * 4);
  res->qend = (uint32_t *)malloc((ns + 1) * 4); res->npos = (uint32_t *)malloc((ns + 1) * 4);
  res->flags = (uint32_t *)malloc((ns + 1) * 4);
  res->k = (uint64_t *)malloc((ns + 1) * 8); res->kr = (uint64_t *)malloc((ns + 1) * 8);
  res->s = (uint64_t *)malloc((ns + 1) * 8); res->pos_off = (uint64_t *)malloc((ns + 1) * 8);
  res->pos = (uint64_t *)malloc((np + 1) * 8);
  uint64_t si = 0, pw = 0;
  for (uint64_t r = 0; r < n_reads; ++r) {
    uint64_t rp = 0;
    for (uint64_t q = 0; q < per[r].n; ++q) {
      smem_t *s = &per[r].v[q];
      res->read_id[si] = (uint32_t)r; res->qbeg[si] = s->qbeg; res->qend[si] = s->qend;
      res->k[si] = s->k; res->kr[si] = s->kr; res->s[si] = s->s;
      res->pos_off[si] = pw;
      res->flags[si] = s->s > (uint64_t)o->max_occ ? 1u : 0u;   /* 1: not located (occurrence above max_occ) */
      res->npos[si] = pcnt[r][q];
      memcpy(res->pos + pw, ppos[r] + rp, (uint64_t)pcnt[r][q] * 8);
      rp += pcnt[r][q]; pw += pcnt[r][q];
      ++si;
    }
    free(per[r].v); free(ppos[r]); free(pcnt[r]);
  }
  for (int t = 0; t < nt; ++t) {
    res->lines.lines += tl[t].lines; res->lines.kmer_lookups += tl[t].kmer_lookups;
    res->lines.sa_reads += tl[t].sa_reads; res->lines.steps += tl[t].steps; res->lines.lf_steps += tl[t].lf_steps;
  }
  res->lines.bases_per_line = (uint64_t)o->bases_per_line;
  free(per); free(ppos); free(pcnt); free(tl);
  return res;
}

uint64_t orc_result_nseeds(const orc_result *r) { return r->n_seeds; }
uint64_t orc_result_npos(const orc_result *r) { return r->n_pos; }
void orc_result_copy(const orc_result *r, uint32_t *read_id, uint32_t *qbeg, uint32_t *qend, uint64_t *k,
                     uint64_t *kr, uint64_t *s, uint32_t *npos, uint32_t *flags, uint64_t *pos_off, uint64_t *pos) {
  uint64_t n = r->n_seeds;
  memcpy(read_id, r->read_id, n * 4); memcpy(qbeg, r->qbeg, n * 4); memcpy(qend, r->qend, n * 4);
  memcpy(k, r->k, n * 8); memcpy(kr, r->kr, n * 8); memcpy(s, r->s, n * 8);
  memcpy(npos, r->npos, n * 4); memcpy(flags, r->flags, n * 4); memcpy(pos_off, r->pos_off, n * 8);
  memcpy(pos, r->pos, r->n_pos * 8);
}
void orc_result_lines(const orc_result *r, uint64_t out[5]) {
  out[0] = r->lines.lines; out[1] = r->lines.kmer_lookups; out[2] = r->lines.sa_reads;
  out[3] = r->lines.steps; out[4] = r->lines.lf_steps;
}
void orc_result_free(orc_result *r) {
  if (!r) return;
  free(r->read_id); free(r->qbeg); free(r->qend); free(r->npos); free(r->flags);
  free(r->k); free(r->kr); free(r->s); free(r->pos_off); free(r->pos); free(r);
}

/* Exported single-step primitives for tests (O2 Algorithm 1 on raw intervals). */
void orc_backward(const orc_index *ix, uint64_t iv[3], uint8_t a) { fm_backward(ix, iv, a, NULL); }
void orc_forward(const orc_index *ix, uint64_t iv[3], uint8_t a) { fm_forward(ix, iv, a, NULL); }
uint64_t orc_pi(const orc_index *ix, uint8_t a, uint64_t k) { return fm_pi(ix, a, k); }
uint64_t orc_locate_slow(const orc_index *ix, uint64_t k) { return fm_locate_slow(ix, k, NULL); }

/* ------------------------------------------------------------------------------------------ */
/* O3 ("scan"): (l,c)-SMEMs and their positions for a sample of reads over a text too large to
 * sort, straight from the definitions of Section 2.2, with no index at all.
 *
 * Every match P[i,j) of length >= q begins with an occurrence of the q-mer P[i,i+q).  One pass
 * over T therefore collects every occurrence p of every q-mer of the reads (q = the smallest
 * seed length any round may ask for, at most 32).  Extending each occurrence to the right by
 * direct comparison gives len(i,p) = the longest common prefix of P[i..] and T[p..], so
 *     occ(P[i,j)) = |{p : len(i,p) >= j - i}|      for every j >= i + q,
 * hence e(i) = max{ j : occ(P[i,j)) >= c } (the c-th largest len), the SMEM set
 * {[i, e(i)) : (i = first offset or e(i-1) < e(i)) and e(i) - i >= l}, each SMEM's s and its
 * exact position set {p : len(i,p) >= e(i) - i}.  Offsets whose q-mer occurs fewer than c times
 * have e(i) < i + q and can neither start an SMEM nor block the next offset.  The ds-interval
 * bounds lo(P), lo(revcomp P) need the sorted suffixes and are not produced (k = k' = ~0).
 * Round 2 (Section 2.6) reuses the same occurrence lists with lengths capped at the sub-query's
 * end.                                                                                       */
typedef struct { uint64_t key; uint32_t read, off; } qmer_t;
typedef struct { uint32_t kid; uint32_t pad; uint64_t p; } hit_t;

static int cmp_qmer(const void *a, const void *b) {
  const qmer_t *x = (const qmer_t *)a, *y = (const qmer_t *)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  if (x->read != y->read) return x->read < y->read ? -1 : 1;
  return x->off < y->off ? -1 : x->off > y->off;
}
static inline uint64_t qmix(uint64_t k) { return (k * 0x9E3779B97F4A7C15ull) >> 40; }   /* 24-bit bucket */

typedef struct { uint32_t len; uint64_t p; } occ_t;       /* one occurrence of the q-mer at an offset */

/* e(i) over the query [qb, qe) for minimum occurrence c: i + the c-th largest match length
 * (capped at the query end); -1 when fewer than c occurrences of the q-mer exist (then
 * e(i) < i + q).  `hist` has room for qe - i + 1 counters.                                    */
static int64_t scan_e(const occ_t *o, uint64_t no, uint64_t i, uint64_t qe, uint64_t c, uint64_t *hist) {
  if (no < c) return -1;
  const uint64_t cap = qe - i;
  memset(hist, 0, (cap + 1) * 8);
  for (uint64_t t = 0; t < no; ++t) hist[o[t].len < cap ? o[t].len : cap]++;
  uint64_t cnt = 0;
  for (uint64_t m = cap;; --m) {
    cnt += hist[m];
    if (cnt >= c) return (int64_t)(i + m);
    if (m == 0) return -1;
  }
}

static void scan_smems(const occ_t *const *occ, const uint64_t *nocc, uint64_t qb, uint64_t qe, int l, uint64_t c,
                       int q, uint64_t *hist, smem_vec *out) {
  int64_t prev = -1;
  for (uint64_t i = qb; i < qe; ++i) {
    int64_t e = (i + (uint64_t)q <= qe) ? scan_e(occ[i], nocc[i], i, qe, c, hist) : -1;
    if (e >= 0 && e - (int64_t)i < q) e = -1;                 /* shorter than a q-mer: not exact here */
    if (e >= 0 && e - (int64_t)i >= l && (i == qb || prev < e)) {
      smem_t s;
      s.qbeg = (uint32_t)i; s.qend = (uint32_t)e; s.k = ~0ull; s.kr = ~0ull; s.s = 0;
      for (uint64_t t = 0; t < nocc[i]; ++t) s.s += occ[i][t].len >= (uint64_t)(e - (int64_t)i);
      push_smem(out, s);
    }
    prev = e;
  }
}

orc_result *orc_scan_seed(const uint8_t *R, uint64_t len_r, int bisulfite, const uint8_t *reads, const uint64_t *offsets,
                          uint64_t n_reads, const orc_opts *o, int n_threads) {
  if (n_threads > 0) omp_set_num_threads(n_threads);
  int q = o->min_len;
  if (o->reseed && o->reseed_len / 2 < q) q = o->reseed_len / 2;
  if (q > 32) q = 32;
  if (q < 1) return NULL;
  uint64_t n = 0;
  uint8_t *T = build_text(R, len_r, bisulfite, &n);
  const uint64_t lr_seg = len_r;   /* bisulfite segment length */
  /* encode reads (Section 2.9 conversion by role), collect their q-mers */
  uint64_t tot = offsets[n_reads];
  uint8_t *P = (uint8_t *)malloc(tot + 1);
  for (uint64_t t = 0; t < tot; ++t) {
    uint8_t a = enc_ascii(reads[t]);
    if (o->bs_role == 1 && a == 2) a = 4;
    if (o->bs_role == 2 && a == 3) a = 1;
    P[t] = a;
  }
  uint64_t nq = 0;
  qmer_t *Q = (qmer_t *)malloc((tot + 1) * sizeof(qmer_t));
  const uint64_t kmask = q == 32 ? ~0ull : ((1ull << (2 * q)) - 1);
  for (uint64_t r = 0; r < n_reads; ++r) {
    uint64_t b = offsets[r], m = offsets[r + 1] - b, key = 0, run = 0;
    for (uint64_t t = 0; t < m; ++t) {
      uint8_t a = P[b + t];
      if (a < 1 || a > 4) { run = 0; key = 0; continue; }
      key = ((key << 2) | (uint64_t)(a - 1)) & kmask;
      if (++run >= (uint64_t)q) { Q[nq].key = key; Q[nq].read = (uint32_t)r; Q[nq].off = (uint32_t)(t + 1 - q); ++nq; }
    }
  }
  qsort(Q, nq, sizeof(qmer_t), cmp_qmer);
  uint64_t nu = 0;
  uint64_t *U = (uint64_t *)malloc((nq + 1) * 8);
  uint32_t *qkid = (uint32_t *)malloc((nq + 1) * 4);          /* key id of each read q-mer */
  for (uint64_t t = 0; t < nq; ++t) {
    if (nu == 0 || U[nu - 1] != Q[t].key) U[nu++] = Q[t].key;
    qkid[t] = (uint32_t)(nu - 1);
  }
  uint64_t *bitmap = (uint64_t *)calloc((1u << 24) / 64, 8);
  for (uint64_t t = 0; t < nu; ++t) { uint64_t h = qmix(U[t]); bitmap[h >> 6] |= 1ull << (h & 63); }
  /* one pass over T: every occurrence of every read q-mer */
  int nt = omp_get_max_threads();
  hit_t **th = (hit_t **)calloc((size_t)nt, sizeof(hit_t *));
  uint64_t *thn = (uint64_t *)calloc((size_t)nt, 8), *thc = (uint64_t *)calloc((size_t)nt, 8);
  #pragma omp parallel
  {
    int tid = omp_get_thread_num();
    uint64_t chunk = (n + (uint64_t)nt - 1) / (uint64_t)nt;
    uint64_t a0 = chunk * (uint64_t)tid, a1 = a0 + chunk < n ? a0 + chunk : n;   /* start positions [a0, a1) */
    uint64_t key = 0, run = 0;
    for (uint64_t p = a0; p < a1 + (uint64_t)q - 1 && p < n; ++p) {
      uint8_t a = T[p];
      if (a < 1 || a > 4) { run = 0; key = 0; continue; }
      key = ((key << 2) | (uint64_t)(a - 1)) & kmask;
      if (++run < (uint64_t)q) continue;
      uint64_t st = p + 1 - (uint64_t)q;
      if (st < a0) continue;
      uint64_t h = qmix(key);
      if (!((bitmap[h >> 6] >> (h & 63)) & 1)) continue;
      uint64_t lo = 0, hi = nu;
      while (lo < hi) { uint64_t mid = (lo + hi) / 2; if (U[mid] < key) lo = mid + 1; else hi = mid; }
      if (lo < nu && U[lo] == key) {
        if (thn[tid] == thc[tid]) { thc[tid] = thc[tid] ? 2 * thc[tid] : 4096; th[tid] = (hit_t *)realloc(th[tid], thc[tid] * sizeof(hit_t)); }
        th[tid][thn[tid]].kid = (uint32_t)lo; th[tid][thn[tid]].pad = 0; th[tid][thn[tid]].p = st; thn[tid]++;
      }
    }
  }
  /* group the hits by key id (counting sort): hits of key id u are H[hstart[u], hstart[u+1]) */
  uint64_t nh = 0;
  for (int t = 0; t < nt; ++t) nh += thn[t];
  uint64_t *hstart = (uint64_t *)calloc(nu + 2, 8);
  for (int t = 0; t < nt; ++t)
    for (uint64_t x = 0; x < thn[t]; ++x) hstart[th[t][x].kid + 1]++;
  for (uint64_t u = 0; u < nu; ++u) hstart[u + 1] += hstart[u];
  uint64_t *fill = (uint64_t *)malloc((nu + 1) * 8);
  memcpy(fill, hstart, (nu + 1) * 8);
  hit_t *H = (hit_t *)malloc((nh + 1) * sizeof(hit_t));
  for (int t = 0; t < nt; ++t) {
    for (uint64_t x = 0; x < thn[t]; ++x) H[fill[th[t][x].kid]++] = th[t][x];
    free(th[t]);
  }
  free(fill); free(th); free(thn); free(thc);
  /* per read: occurrence lists with their match lengths, then the SMEMs of both rounds */
  uint32_t *kid_at = (uint32_t *)malloc((tot + 1) * 4);
  for (uint64_t t = 0; t < tot; ++t) kid_at[t] = 0xFFFFFFFFu;
  for (uint64_t t = 0; t < nq; ++t) kid_at[offsets[Q[t].read] + Q[t].off] = qkid[t];
  smem_vec *per = (smem_vec *)calloc(n_reads, sizeof(smem_vec));
  uint64_t **ppos = (uint64_t **)calloc(n_reads, sizeof(uint64_t *));
  uint32_t **pcnt = (uint32_t **)calloc(n_reads, sizeof(uint32_t *));
  #pragma omp parallel for schedule(dynamic, 1)
  for (int64_t r = 0; r < (int64_t)n_reads; ++r) {
    uint64_t b = offsets[r], m = offsets[r + 1] - b;
    occ_t **occ = (occ_t **)calloc(m + 1, sizeof(occ_t *));
    uint64_t *nocc = (uint64_t *)calloc(m + 1, 8);
    for (uint64_t i = 0; i < m; ++i) {
      uint32_t u = kid_at[b + i];
      if (u == 0xFFFFFFFFu) continue;
      uint64_t h0 = hstart[u], h1 = hstart[u + 1];
      nocc[i] = h1 - h0;
      occ[i] = (occ_t *)malloc((nocc[i] + 1) * sizeof(occ_t));
      for (uint64_t t = h0; t < h1; ++t) {
        uint64_t p = H[t].p, len = (uint64_t)q;
        while (i + len < m && p + len < n && P[b + i + len] == T[p + len] && T[p + len] >= 1 && T[p + len] <= 4) ++len;
        occ[i][t - h0].len = (uint32_t)len; occ[i][t - h0].p = p;
      }
    }
    uint64_t *tmp = (uint64_t *)malloc((m + 2) * 8);
    smem_vec *V = &per[r];
    V->n = 0;
    scan_smems((const occ_t *const *)occ, nocc, 0, m, o->min_len, (uint64_t)o->min_occ, q, tmp, V);
    if (o->reseed) {
      uint64_t n1 = V->n;
      for (uint64_t t = 0; t < n1; ++t) {
        smem_t s = V->v[t];
        if (s.qend - s.qbeg >= (uint32_t)o->reseed_len && s.s <= (uint64_t)o->reseed_occ)
          scan_smems((const occ_t *const *)occ, nocc, s.qbeg, s.qend, (int)((s.qend - s.qbeg) / 2), s.s + 1, q, tmp, V);
      }
    }
    qsort(V->v, V->n, sizeof(smem_t), cmp_smem);
    uint64_t w = 0;
    for (uint64_t t = 0; t < V->n; ++t)
      if (w == 0 || cmp_smem(&V->v[w - 1], &V->v[t]) != 0) V->v[w++] = V->v[t];
    V->n = w;
    uint64_t np = 0;
    for (uint64_t t = 0; t < V->n; ++t) if (V->v[t].s <= (uint64_t)o->max_occ) np += V->v[t].s;
    uint64_t *pp = (uint64_t *)malloc((np + 1) * 8);
    uint32_t *pc = (uint32_t *)calloc(V->n + 1, 4);
    uint64_t pw = 0;
    for (uint64_t t = 0; t < V->n; ++t) {
      smem_t *s = &V->v[t];
      if (s->s > (uint64_t)o->max_occ) continue;
      uint64_t w0 = pw, need = s->qend - s->qbeg;
      for (uint64_t x = 0; x < nocc[s->qbeg]; ++x) {
        const occ_t *oc = &occ[s->qbeg][x];
        if (oc->len < need) continue;
        uint64_t seg = oc->p / lr_seg;
        int keep = o->bs_role == 1 ? (seg == 0 || seg == 2) : o->bs_role == 2 ? (seg == 1 || seg == 3) : 1;
        if (keep) pp[pw++] = oc->p;
      }
      qsort(pp + w0, pw - w0, 8, cmp_u64);
      pc[t] = (uint32_t)(pw - w0);
    }
    ppos[r] = pp; pcnt[r] = pc;
    for (uint64_t i = 0; i < m; ++i) free(occ[i]);
    free(occ); free(nocc); free(tmp);
  }
  orc_result *res = (orc_result *)calloc(1, sizeof(orc_result));
  uint64_t ns = 0, npos = 0;
  for (uint64_t r = 0; r < n_reads; ++r) { ns += per[r].n; for (uint64_t t = 0; t < per[r].n; ++t) npos += pcnt[r][t]; }
  res->n_seeds = ns; res->n_pos = npos;
  res->read_id = (uint32_t *)malloc((ns + 1) * 4); res->qbeg = (uint32_t *)malloc((ns + 1) * 4);
  res->qend = (uint32_t *)malloc((ns + 1) * 4); res->npos = (uint32_t *)malloc((ns + 1) * 4);
  res->flags = (uint32_t *)malloc((ns + 1) * 4);
  res->k = (uint64_t *)malloc((ns + 1) * 8); res->kr = (uint64_t *)malloc((ns + 1) * 8);
  res->s = (uint64_t *)malloc((ns + 1) * 8); res->pos_off = (uint64_t *)malloc((ns + 1) * 8);
  res->pos = (uint64_t *)malloc((npos + 1) * 8);
  uint64_t si = 0, pw = 0;
  for (uint64_t r = 0; r < n_reads; ++r) {
    uint64_t rp = 0;
    for (uint64_t t = 0; t < per[r].n; ++t) {
      smem_t *s = &per[r].v[t];
      res->read_id[si] = (uint32_t)r; res->qbeg[si] = s->qbeg; res->qend[si] = s->qend;
      res->k[si] = s->k; res->kr[si] = s->kr; res->s[si] = s->s; res->pos_off[si] = pw;
      res->flags[si] = s->s > (uint64_t)o->max_occ ? 1u : 0u;
      res->npos[si] = pcnt[r][t];
      memcpy(res->pos + pw, ppos[r] + rp, (uint64_t)pcnt[r][t] * 8);
      rp += pcnt[r][t]; pw += pcnt[r][t]; ++si;
    }
    free(per[r].v); free(ppos[r]); free(pcnt[r]);
  }
  free(per); free(ppos); free(pcnt);
  free(kid_at); free(hstart); free(H); free(bitmap); free(qkid); free(U); free(Q); free(P); free(T);
  return res;
}

/* ------------------------------------------------------------------------------------------ */
/* Bisulfite seed refinement (Section 2.9).  A retained seed match pairs the read bases
 * P[qbeg, qend) with the text T[pos, pos + qend - qbeg) of the four-copy index.  Every text base
 * has an original reference base: for t < 2|R| (the forward C->T and G->A copies) it is R[t mod |R|],
 * for 2|R| <= t < 4|R| (the reverse copies) the complement of R[(4|R| - 1 - t) mod |R|].  Comparing
 * the original read base with it, a read C over a reference T (read 1; read 2: a read G over a
 * reference A) cannot come from bisulfite conversion; the seed match is split at every such base and
 * the pieces of at least min_len bases are kept, each with its own text position.
 * Output: pieces sorted by (read, qbeg, qend, pos). */
typedef struct { uint32_t read_id, qbeg, qend, seed; uint64_t pos; } orc_piece;
static int cmp_piece(const void *a, const void *b) {
  const orc_piece *x = (const orc_piece *)a, *y = (const orc_piece *)b;
  if (x->read_id != y->read_id) return x->read_id < y->read_id ? -1 : 1;
  if (x->qbeg != y->qbeg) return x->qbeg < y->qbeg ? -1 : 1;
  if (x->qend != y->qend) return x->qend < y->qend ? -1 : 1;
  return x->pos < y->pos ? -1 : x->pos > y->pos;
}
static inline int orig_ref_base(const uint8_t *R, uint64_t L, uint64_t t) {   /* 0..3 */
  if (t < 2 * L) return R[t % L];
  return 3 - R[(4 * L - 1 - t) % L];
}
/* seeds: n_seeds records (read_id, qbeg, qend, pos_off, npos) of a bisulfite seeding result;
 * returns the number of pieces and a malloc'ed array in *out. */
uint64_t orc_bs_refine(const uint8_t *R, uint64_t L, const uint8_t *reads, const uint64_t *offsets,
                       const uint32_t *read_id, const uint32_t *qbeg, const uint32_t *qend, const uint64_t *pos_off,
                       const uint32_t *npos, uint64_t n_seeds, const uint64_t *pos, int role, int min_len,
                       orc_piece **out) {
  uint64_t cap = 1024, n = 0;
  orc_piece *v = (orc_piece *)malloc(cap * sizeof(orc_piece));
  for (uint64_t t = 0; t < n_seeds; ++t) {
    const uint8_t *P = reads + offsets[read_id[t]];
    for (uint32_t q = 0; q < npos[t]; ++q) {
      const uint64_t p = pos[pos_off[t] + q];
      uint32_t start = qbeg[t];
      for (uint32_t i = qbeg[t]; i <= qend[t]; ++i) {
        int cut = i == qend[t];
        if (!cut) {
          const uint8_t a = enc_ascii(P[i]);                 /* 1..4 = A..T, 5 = other */
          const int rb = orig_ref_base(R, L, p + (i - qbeg[t]));
          cut = (role == 1) ? (a == 2 && rb == 3) : (a == 3 && rb == 0);
        }
        if (cut) {
          if (i - start >= (uint32_t)min_len) {
            if (n == cap) { cap *= 2; v = (orc_piece *)realloc(v, cap * sizeof(orc_piece)); }
            v[n].read_id = read_id[t]; v[n].qbeg = start; v[n].qend = i; v[n].seed = (uint32_t)t;
            v[n].pos = p + (start - qbeg[t]);
            ++n;
          }
          start = i + 1;
        }
      }
    }
  }
  qsort(v, n, sizeof(orc_piece), cmp_piece);
  *out = v;
  return n;
}
/* ---------------------------------------------------------------------------------------------
 * Mate-rescue prefilter (Section 2.7), straight from its definition.  For a read P and a window W
 * of the text,
 *     M_t = |{(i, j) : P[i, i+q) = W[j, j+q) and j - i = t}|,   0 <= i <= |P|-q, 0 <= j <= |W|-q,
 * counted pair by pair.  A read base outside ACGT (code 5) equals no text symbol, so a q-mer that
 * holds one matches nothing.  M is stored at index t + |P| - q (|P| + |W| - 2q + 1 entries).
 * Reported per candidate: max_t M_t and the smallest t attaining it (0 when the maximum is 0,
 * which includes |P| < q and |W| < q).
 */
static void rescue_diag(const uint8_t *P, uint64_t np, const uint8_t *W, uint64_t nw, int q, uint32_t *M) {
  if (np < (uint64_t)q || nw < (uint64_t)q) return;
  for (uint64_t i = 0; i + q <= np; ++i)
    for (uint64_t j = 0; j + q <= nw; ++j) {
      int eq = 1;
      for (int d = 0; d < q && eq; ++d) eq = P[i + d] >= 1 && P[i + d] <= 4 && P[i + d] == W[j + d];
      if (eq) M[j - i + np - q] += 1;
    }
}

static void rescue_best(const uint32_t *M, uint64_t np, uint64_t nw, int q, uint32_t *max_hits, int32_t *best_t) {
  *max_hits = 0; *best_t = 0;
  if (np < (uint64_t)q || nw < (uint64_t)q) return;
  uint64_t nd = np + nw - 2 * (uint64_t)q + 1;
  for (uint64_t x = 0; x < nd; ++x)
    if (M[x] > *max_hits) { *max_hits = M[x]; *best_t = (int32_t)((int64_t)x - (int64_t)(np - q)); }
}

static uint8_t rescue_read_sym(uint8_t ch, int role) {
  uint8_t a = enc_ascii(ch);
  if (role == 1 && a == 2) a = 4;   /* read 1: C -> T (Section 2.9) */
  if (role == 2 && a == 3) a = 1;   /* read 2: G -> A */
  return a;
}

/* The whole vector M for one ASCII read and one ASCII window (pins and tests). */
void orc_rescue_diag_ascii(const uint8_t *p, uint64_t np, const uint8_t *w, uint64_t nw, int q, int role, uint32_t *M) {
  uint8_t *P = (uint8_t *)malloc(np + 1), *W = (uint8_t *)malloc(nw + 1);
  for (uint64_t t = 0; t < np; ++t) P[t] = rescue_read_sym(p[t], role);
  for (uint64_t t = 0; t < nw; ++t) { W[t] = enc_ascii(w[t]); if (W[t] > 4) W[t] = 6; }  /* window N: matches nothing */
  if (np >= (uint64_t)q && nw >= (uint64_t)q) memset(M, 0, (np + nw - 2 * (uint64_t)q + 1) * sizeof(uint32_t));
  rescue_diag(P, np, W, nw, q, M);
  free(P); free(W);
}

/* Candidates (read_id[c], window T[win_beg[c], win_beg[c] + win_len[c])) over the text of R
 * (plain, or the four-copy bisulfite text).  Returns 0, or -1 for a read id or window out of range. */
int orc_rescue(const uint8_t *R, uint64_t len_r, int bisulfite, const uint8_t *reads, const uint64_t *offsets,
               uint64_t n_reads, const uint32_t *read_id, const uint64_t *win_beg, const uint32_t *win_len,
               uint64_t n_cand, int q, int role, uint32_t *max_hits, int32_t *best_t, int n_threads) {
  if (q < 1) return -1;
  uint64_t n = 0;
  uint8_t *T = build_text(R, len_r, bisulfite, &n);
  for (uint64_t c = 0; c < n_cand; ++c)
    if (read_id[c] >= n_reads || win_beg[c] > n - 1 || win_len[c] > n - 1 - win_beg[c]) { free(T); return -1; }
  if (n_threads > 0) omp_set_num_threads(n_threads);
  #pragma omp parallel
  {
    uint8_t *P = NULL; uint32_t *M = NULL; uint64_t pcap = 0, mcap = 0;
    #pragma omp for schedule(dynamic, 16)
    for (int64_t c = 0; c < (int64_t)n_cand; ++c) {
      uint64_t b = offsets[read_id[c]], np = offsets[read_id[c] + 1] - b, nw = win_len[c];
      if (pcap < np + 1) { free(P); pcap = np + 1; P = (uint8_t *)malloc(pcap); }
      for (uint64_t t = 0; t < np; ++t) P[t] = rescue_read_sym(reads[b + t], role);
      uint64_t nd = np + nw + 1;
      if (mcap < nd) { free(M); mcap = nd; M = (uint32_t *)malloc(mcap * sizeof(uint32_t)); }
      memset(M, 0, nd * sizeof(uint32_t));
      rescue_diag(P, np, T + win_beg[c], nw, q, M);
      rescue_best(M, np, nw, q, &max_hits[c], &best_t[c]);
    }
    free(P); free(M);
  }
  free(T);
  return 0;
}

void orc_free_ptr(void *p) { free(p); }

/* ---------------------------------------------------------------------------------------------
 * Chaining (Section 2.6): minibwa chains its variable-length seeds with the chaining of minimap2
 * (Li 2018, Bioinformatics 34:3094, Section 2.1), adapted to seeds of different lengths, and keeps
 * up to 50 chains per read.  The paper states no formula of its own; this is the published
 * recurrence with the readings below (fixed so that every value is an integer and exact).
 *
 * Anchors.  Every located (seed, position) pair of a read is an anchor: the seed P[qbeg, qend)
 * matches T[p, p + w), w = qend - qbeg; its end is (x, y) = (p + w - 1, qend - 1) and its copy
 * g = floor(x / L) (L = |R|: 0 forward, 1 reverse strand; four copies for a bisulfite index).
 * A read's anchors are sorted by (x, y, w).
 * Recurrence.  f(i) = max( w_i, max_j f(j) + alpha(j, i) - beta(j, i) ) over the h anchors
 * before i in that order (j = i-h .. i-1) with g_j = g_i, x_j < x_i, y_j < y_i and
 * max(x_i - x_j, y_i - y_j) <= G, where alpha(j, i) = min(x_i - x_j, y_i - y_j, w_i) and
 * beta(j, i) = gamma(|(y_i - y_j) - (x_i - x_j)|), gamma(0) = 0,
 * gamma(l) = floor(l * wbar / 100) + floor(floor(log2 l) / 2), wbar = floor(mean span of the
 * read's anchors).  The predecessor p(i) is the largest such j attaining the maximum when that
 * maximum exceeds w_i, else -1.
 * Chains.  Anchors are taken in order of descending f (equal f: smaller index first); from each
 * anchor not used yet, p is followed, marking every anchor reached as used, until p = -1 or the
 * next anchor is already used.  The chain is the anchors visited; its score is f(end) minus f of
 * the used anchor it stopped at (f(end) when it stopped at p = -1).  Chains scoring at least
 * min_score are kept, ordered by score (descending; equal scores by end index ascending), and the
 * first max_chains returned, each with its anchors in ascending order.
 */
typedef struct { uint64_t x; uint32_t y, w, g; uint32_t qbeg, qend; uint64_t pos; } orc_anchor;
typedef struct { int max_gap, max_pred, max_chains, min_score; } orc_chain_opts;

static int cmp_anchor(const void *a, const void *b) {
  const orc_anchor *u = (const orc_anchor *)a, *v = (const orc_anchor *)b;
  if (u->x != v->x) return u->x < v->x ? -1 : 1;
  if (u->y != v->y) return u->y < v->y ? -1 : 1;
  return u->w < v->w ? -1 : u->w > v->w;
}

static int64_t chain_gamma(int64_t l, int64_t wbar) {
  if (l < 0) l = -l;
  if (l == 0) return 0;
  int lg = 0;
  while ((l >> (lg + 1)) != 0) ++lg;                    /* floor(log2 l) */
  return l * wbar / 100 + lg / 2;
}

/* f and p of anchors already in chaining order (x, y, w ascending) */
static void chain_dp(const uint64_t *x, const uint32_t *y, const uint32_t *w, const uint32_t *g, uint64_t N,
                     int max_gap, int max_pred, int32_t *f, int64_t *p) {
  if (N == 0) return;
  uint64_t sw = 0;
  for (uint64_t i = 0; i < N; ++i) sw += w[i];
  const int64_t wbar = (int64_t)(sw / N);
  for (uint64_t i = 0; i < N; ++i) {
    int64_t best = w[i], bj = -1;
    uint64_t j0 = i > (uint64_t)max_pred ? i - (uint64_t)max_pred : 0;
    for (uint64_t j = j0; j < i; ++j) {
      if (g[j] != g[i] || x[j] >= x[i] || y[j] >= y[i]) continue;
      int64_t dx = (int64_t)(x[i] - x[j]), dy = (int64_t)y[i] - (int64_t)y[j];
      if (dx > max_gap || dy > max_gap) continue;
      int64_t a = dx < dy ? dx : dy;
      if (a > (int64_t)w[i]) a = w[i];
      int64_t sc = f[j] + a - chain_gamma(dy - dx, wbar);
      if (sc > best || (sc == best && bj >= 0)) { best = sc; bj = (int64_t)j; }   /* later j wins a tie */
    }
    f[i] = (int32_t)best;
    p[i] = bj;
  }
}

/* exported for the pins: anchors given in chaining order */
void orc_chain_dp(const uint64_t *x, const uint32_t *y, const uint32_t *w, const uint32_t *g, uint64_t N, int max_gap,
                  int max_pred, int32_t *f, int64_t *p) {
  chain_dp(x, y, w, g, N, max_gap, max_pred, f, p);
}

typedef struct { int32_t score; uint64_t end, start, n; } orc_chain_rec;
static const int32_t *g_chain_f;
static int cmp_by_f(const void *a, const void *b) {
  uint64_t i = *(const uint64_t *)a, j = *(const uint64_t *)b;
  if (g_chain_f[i] != g_chain_f[j]) return g_chain_f[i] > g_chain_f[j] ? -1 : 1;
  return i < j ? -1 : 1;
}
static int cmp_chain_rec(const void *a, const void *b) {
  const orc_chain_rec *u = (const orc_chain_rec *)a, *v = (const orc_chain_rec *)b;
  if (u->score != v->score) return u->score > v->score ? -1 : 1;
  return u->end < v->end ? -1 : u->end > v->end;
}

/* Chains of every read of a seeding result (seeds sorted by read, each seed's npos positions at
 * pos[pos_off ..]).  Output: for each read its chains in rank order -> chain arrays (read, score,
 * number of anchors, copy, offset into the anchor arrays) and the anchors of every chain in
 * ascending order (qbeg, qend, pos).  Returns the chain count; arrays malloc'ed. */
uint64_t orc_chain(const uint32_t *read_id, const uint32_t *qbeg, const uint32_t *qend, const uint64_t *pos_off,
                   const uint32_t *npos, uint64_t n_seeds, const uint64_t *pos, uint64_t seg_len,
                   const orc_chain_opts *o, uint32_t **c_read, int32_t **c_score, uint32_t **c_n, uint32_t **c_g,
                   uint64_t **c_off, uint32_t **a_qbeg, uint32_t **a_qend, uint64_t **a_pos, uint64_t *n_anchors_out) {
  uint64_t ccap = 1024, nc = 0, acap = 1024, na = 0;
  uint32_t *cr = malloc(ccap * 4), *cn = malloc(ccap * 4), *cg = malloc(ccap * 4);
  int32_t *cs = malloc(ccap * 4);
  uint64_t *co = malloc(ccap * 8);
  uint32_t *aq = malloc(acap * 4), *ae = malloc(acap * 4);
  uint64_t *ap = malloc(acap * 8);
  uint64_t t0 = 0;
  while (t0 < n_seeds) {
    uint64_t t1 = t0;
    while (t1 < n_seeds && read_id[t1] == read_id[t0]) ++t1;
    uint64_t N = 0;
    for (uint64_t t = t0; t < t1; ++t) N += npos[t];
    if (N) {
      orc_anchor *A = malloc(N * sizeof(orc_anchor));
      uint64_t k = 0;
      for (uint64_t t = t0; t < t1; ++t)
        for (uint32_t q = 0; q < npos[t]; ++q, ++k) {
          uint32_t w = qend[t] - qbeg[t];
          A[k].pos = pos[pos_off[t] + q];
          A[k].x = A[k].pos + w - 1; A[k].y = qend[t] - 1; A[k].w = w;
          A[k].g = (uint32_t)(A[k].x / seg_len); A[k].qbeg = qbeg[t]; A[k].qend = qend[t];
        }
      qsort(A, N, sizeof(orc_anchor), cmp_anchor);
      uint64_t *x = malloc(N * 8);
      uint32_t *y = malloc(N * 4), *w = malloc(N * 4), *g = malloc(N * 4);
      for (uint64_t i = 0; i < N; ++i) { x[i] = A[i].x; y[i] = A[i].y; w[i] = A[i].w; g[i] = A[i].g; }
      int32_t *f = malloc(N * 4);
      int64_t *p = malloc(N * 8);
      chain_dp(x, y, w, g, N, o->max_gap, o->max_pred, f, p);
      /* backtracking in order of descending f */
      uint64_t *ord = malloc(N * 8);
      for (uint64_t i = 0; i < N; ++i) ord[i] = i;
      g_chain_f = f;
      qsort(ord, N, 8, cmp_by_f);
      uint8_t *used = calloc(N, 1);
      orc_chain_rec *R = malloc(N * sizeof(orc_chain_rec));
      uint64_t nr = 0;
      for (uint64_t q = 0; q < N; ++q) {
        uint64_t e = ord[q];
        if (used[e]) continue;
        uint64_t i = e, n = 0;
        int32_t sc = f[e];
        for (;;) {
          used[i] = 1; ++n;
          if (p[i] < 0) break;
          if (used[p[i]]) { sc = f[e] - f[p[i]]; break; }
          i = (uint64_t)p[i];
        }
        if (sc >= o->min_score) { R[nr].score = sc; R[nr].end = e; R[nr].start = i; R[nr].n = n; ++nr; }
      }
      qsort(R, nr, sizeof(orc_chain_rec), cmp_chain_rec);
      if (nr > (uint64_t)o->max_chains) nr = (uint64_t)o->max_chains;
      for (uint64_t c = 0; c < nr; ++c) {
        if (nc == ccap) {
          ccap *= 2;
          cr = realloc(cr, ccap * 4); cn = realloc(cn, ccap * 4); cg = realloc(cg, ccap * 4);
          cs = realloc(cs, ccap * 4); co = realloc(co, ccap * 8);
        }
        cr[nc] = read_id[t0]; cs[nc] = R[c].score; cn[nc] = (uint32_t)R[c].n; cg[nc] = A[R[c].end].g; co[nc] = na;
        while (na + R[c].n > acap) {
          acap *= 2;
          aq = realloc(aq, acap * 4); ae = realloc(ae, acap * 4); ap = realloc(ap, acap * 8);
        }
        uint64_t i = R[c].end;
        for (uint64_t m = R[c].n; m-- > 0;) {               /* backwards along p, written ascending */
          aq[na + m] = A[i].qbeg; ae[na + m] = A[i].qend; ap[na + m] = A[i].pos;
          if (m) i = (uint64_t)p[i];
        }
        na += R[c].n;
        ++nc;
      }
      free(A); free(x); free(y); free(w); free(g); free(f); free(p); free(ord); free(used); free(R);
    }
    t0 = t1;
  }
  *c_read = cr; *c_score = cs; *c_n = cn; *c_g = cg; *c_off = co;
  *a_qbeg = aq; *a_qend = ae; *a_pos = ap; *n_anchors_out = na;
  return nc;
}
