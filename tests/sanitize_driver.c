/* Runs the oracle under AddressSanitizer / UndefinedBehaviorSanitizer on small inputs: plain and
 * bisulfite indexes, both oracle methods with reseeding and the k-mer shortcut, and the rescue
 * prefilter.  Exit status 0 when every call returns; the sanitizers abort on a memory or UB error. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct orc_index orc_index;
typedef struct orc_result orc_result;
typedef struct {
  int min_len, min_occ, max_occ, reseed, reseed_len, reseed_occ, bs_role, method, kmer_k, bases_per_line;
} orc_opts;

orc_index *orc_build(const uint8_t *R, uint64_t len_r, int bisulfite, int sa_rate);
void orc_free(orc_index *ix);
orc_result *orc_seed(const orc_index *ix, const uint8_t *reads, const uint64_t *offsets, uint64_t n_reads,
                     const orc_opts *o, int n_threads);
uint64_t orc_result_nseeds(const orc_result *r);
void orc_result_free(orc_result *r);
int orc_rescue(const uint8_t *R, uint64_t len_r, int bisulfite, const uint8_t *reads, const uint64_t *offsets,
               uint64_t n_reads, const uint32_t *read_id, const uint64_t *win_beg, const uint32_t *win_len,
               uint64_t n_cand, int q, int role, uint32_t *max_hits, int32_t *best_t, int n_threads);

static uint64_t rng = 88172645463325252ull;
static uint64_t next(void) { rng ^= rng << 13; rng ^= rng >> 7; rng ^= rng << 17; return rng; }

int main(void) {
  const uint64_t L = 20000, NR = 300;
  uint8_t *R = malloc(L);
  for (uint64_t i = 0; i < L; ++i) R[i] = (uint8_t)(next() & 3);
  for (uint64_t i = 5000; i < 5600; ++i) R[i] = R[i - 300];          /* a repeat */
  uint64_t *off = malloc((NR + 1) * sizeof(uint64_t));
  uint8_t *reads = malloc(NR * 200);
  off[0] = 0;
  for (uint64_t r = 0; r < NR; ++r) {
    uint64_t len = next() % 200, st = next() % (L - 200);
    for (uint64_t t = 0; t < len; ++t) {
      uint8_t c = "ACGT"[R[st + t]];
      if (next() % 100 == 0) c = "ACGTN"[next() % 5];
      reads[off[r] + t] = c;
    }
    off[r + 1] = off[r] + len;
  }
  for (int bis = 0; bis < 2; ++bis) {
    orc_index *ix = orc_build(R, L, bis, 8);
    for (int method = 0; method < 2; ++method) {
      orc_opts o = {19, 1, 500, 1, 38, 10, bis, method, method ? 6 : 0, method ? 384 : 0};
      orc_result *res = orc_seed(ix, reads, off, NR, &o, 2);
      printf("bisulfite %d method %d: %llu seeds\n", bis, method, (unsigned long long)orc_result_nseeds(res));
      orc_result_free(res);
    }
    orc_free(ix);
    uint32_t rid[64], wl[64], mh[64];
    uint64_t wb[64];
    int32_t bt[64];
    const uint64_t m = (bis ? 4 : 2) * L;
    for (int c = 0; c < 64; ++c) { rid[c] = (uint32_t)(next() % NR); wl[c] = (uint32_t)(next() % 700); wb[c] = next() % (m - wl[c] + 1); }
    if (orc_rescue(R, L, bis, reads, off, NR, rid, wb, wl, 64, 7, bis, mh, bt, 2) != 0) return 1;
    printf("bisulfite %d rescue: first max %u\n", bis, mh[0]);
  }
  free(R); free(off); free(reads);
  return 0;
}
