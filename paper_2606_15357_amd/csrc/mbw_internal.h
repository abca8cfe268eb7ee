// Internal definitions shared by the mbw HIP sources: index layout and device rank helpers.
//
// Resident FM-index (paper Sections 2.1, 2.2 and 2.4; the line format is this library's own,
// sized for gfx950 where a random HBM access moves one 128-byte L2 line):
//   * occurrence lines, 128 bytes each (8 slices of 16 bytes), one per 384 rows of B:
//       slice 0     u32 counts of A, C, G, T in B from the start of the line's superblock (2^23
//                   lines) up to the line (the $ row is stored and counted as A; rank corrects it)
//       slice 1     three u32 sub-checkpoints: counts of A, C, G (10 bits each) in the line's
//                   first 96, 192 and 288 rows (T follows from the row count); one u32 unused
//       slices 2-7  the line's 384 rows of B at 2 bits (row t in u64 word t/32, bits 2(t%32))
//     so a rank query reads one line and counts at most 96 rows (three words) by popcount.
//   * superblock table: absolute counts of A, C, G, T before each superblock, plus their suffix
//     sums (for the k' update of backward extension).
//   * sampled SA: ssa[x / r] = S(x) for rows x that are multiples of r.
//   * k-mer table: 4^K packed ds-intervals (16 bytes); the code of P[0..K) is sum_q P[q] 4^q.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#define MBW_BPL 384            // rows of B per occurrence line
#define MBW_LINE_BYTES 128
#define MBW_LINE_U4 8          // 16-byte slices per line
#define MBW_SUB 96             // rows per sub-checkpoint block
#define MBW_SB_SHIFT 23        // lines per superblock = 2^23 (3.2 G rows < 2^32)
#define MBW_MAX_SB 8
#define MBW_MAX_READ 65535

struct mbw_index {
  int device;
  uint64_t n, len_r, primary, n_lines, n_ssa;
  uint64_t C[5];               // C[$], C[A], C[C], C[G], C[T]
  int sa_sample, kmer_k, bisulfite;
  int n_sb;
  uint64_t sb_host[MBW_MAX_SB * 8];
  uint4 *lines;                // n_lines * 8
  uint64_t *ssa;               // n_ssa
  uint4 *kmer;                 // 4^K (or nullptr)
  uint64_t *sbtab;             // n_sb * 8: counts of A,C,G,T before the superblock, then sums of d > c
  uint64_t bytes;
};

// Read-only view passed by value to kernels.
struct IndexView {
  const uint4 *__restrict__ lines;
  const uint64_t *__restrict__ ssa;
  const uint4 *__restrict__ kmer;
  const uint64_t *__restrict__ sbtab;
  uint64_t n, primary;
  uint64_t Cb[4];              // C of base a (A..T) = |{i : B[i] < a}| (includes the $ row)
  uint32_t r;
  int K;
  int n_sb;
};

static inline IndexView make_view(const mbw_index *ix) {
  IndexView v;
  v.lines = ix->lines; v.ssa = ix->ssa; v.kmer = ix->kmer; v.sbtab = ix->sbtab;
  v.n = ix->n; v.primary = ix->primary;
  for (int a = 0; a < 4; ++a) v.Cb[a] = ix->C[a + 1];
  v.r = (uint32_t)ix->sa_sample; v.K = ix->kmer_k; v.n_sb = ix->n_sb;
  return v;
}

// ---------------------------------------------------------------------------------------------
// error reporting (host)
void mbw_set_error(const std::string &msg);
#define MBW_HIP_TRY(call)                                                                      \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess) {                                                                    \
      mbw_set_error(std::string(#call) + ": " + hipGetErrorString(e_));                        \
      return e_ == hipErrorOutOfMemory ? -2 : -3;                                              \
    }                                                                                          \
  } while (0)

// ---------------------------------------------------------------------------------------------
// device helpers

// x / 384 = (x >> 7) / 3; (x >> 7) < 2^32 for every row of an index (n < 2^39)
__device__ __forceinline__ uint32_t line_of(uint64_t x) { return __umulhi((uint32_t)(x >> 7), 0xAAAAAAABu) >> 1; }
__device__ __forceinline__ int block_of(int o) { return (o * 683) >> 16; }   // o / 96 for 0 <= o < 384

#define M55 0x5555555555555555ull

__device__ __forceinline__ uint64_t sel4(uint64_t a0, uint64_t a1, uint64_t a2, uint64_t a3, int c) {
  return c == 0 ? a0 : (c == 1 ? a1 : (c == 2 ? a2 : a3));
}

// bits of the first m (0..32) rows of a word, restricted to the low bit of each 2-bit field
__device__ __forceinline__ uint64_t pmask(int m) {
  return m >= 32 ? M55 : (m <= 0 ? 0ull : (((1ull << (2 * m)) - 1) & M55));
}

// Per-symbol constants of the popcount rank: rows equal to c are the fields where w ^ patc is 00;
// rows greater than c are ((hi & (w | ga)) | (w & gb)) & ge (hi = high bit of each field moved to
// the low position; only low-position bits survive the row mask).
struct SymMasks { uint64_t patc, ga, gb, ge; };
__device__ __forceinline__ SymMasks sym_masks(int c) {
  SymMasks m;
  m.patc = (uint64_t)c * M55;
  m.ga = c <= 1 ? M55 : 0ull;
  m.gb = c == 0 ? M55 : 0ull;
  m.ge = c == 3 ? 0ull : M55;
  return m;
}

// rows equal to c (e) and greater than c (g) among the first r (0..96) rows of a 96-row block
__device__ __forceinline__ void block_eg(uint64_t w0, uint64_t w1, uint64_t w2, int r, const SymMasks &sm,
                                         uint32_t &e, uint32_t &g) {
  const uint64_t p0 = pmask(r), p1 = pmask(r - 32), p2 = pmask(r - 64);
  const uint64_t x0 = w0 ^ sm.patc, x1 = w1 ^ sm.patc, x2 = w2 ^ sm.patc;
  const uint64_t e0 = ~(x0 | (x0 >> 1)), e1 = ~(x1 | (x1 >> 1)), e2 = ~(x2 | (x2 >> 1));
  const uint64_t h0 = w0 >> 1, h1 = w1 >> 1, h2 = w2 >> 1;
  const uint64_t g0 = ((h0 & (w0 | sm.ga)) | (w0 & sm.gb)) & sm.ge;
  const uint64_t g1 = ((h1 & (w1 | sm.ga)) | (w1 & sm.gb)) & sm.ge;
  const uint64_t g2 = ((h2 & (w2 | sm.ga)) | (w2 & sm.gb)) & sm.ge;
  e = __popcll(e0 & p0) + __popcll(e1 & p1) + __popcll(e2 & p2);
  g = __popcll(g0 & p0) + __popcll(g1 & p1) + __popcll(g2 & p2);
}

// Words 3b..3b+2 (the rows of block b) from the two 16-byte slices 2 + (3b >> 1) and the next one.
__device__ __forceinline__ void block_words(uint4 sa, uint4 sbk, int b, uint64_t &w0, uint64_t &w1, uint64_t &w2) {
  const uint64_t a0 = ((uint64_t)sa.y << 32) | sa.x, a1 = ((uint64_t)sa.w << 32) | sa.z;
  const uint64_t b0 = ((uint64_t)sbk.y << 32) | sbk.x, b1 = ((uint64_t)sbk.w << 32) | sbk.z;
  if (b & 1) { w0 = a1; w1 = b0; w2 = b1; }   // 3b odd: the block starts in the second half
  else { w0 = a0; w1 = a1; w2 = b0; }
}

__device__ __forceinline__ int block_slice(int o) { return 2 + ((3 * block_of(o)) >> 1); }

// Occ(c, x) (E) and sum_{d > c} Occ(d, x) (G), x at offset o of a line, from the line's two header
// slices, the two slices of block o/96, and the superblock values sbe = count of c before the
// superblock, sbg = sum over d > c of the counts before it.  The $ row is not corrected here.
__device__ __forceinline__ void rank_eg(uint4 h0, uint4 h1, uint4 sa, uint4 sbk, int o, int c, const SymMasks &sm,
                                        uint64_t sbe, uint64_t sbg, uint64_t &E, uint64_t &G) {
  const int b = block_of(o), r = o - MBW_SUB * b;
  const uint32_t sw = b == 0 ? 0u : (b == 1 ? h1.x : (b == 2 ? h1.y : h1.z));
  const uint32_t sA = sw & 1023u, sC = (sw >> 10) & 1023u, sG = (sw >> 20) & 1023u;
  const uint32_t sT = (uint32_t)(MBW_SUB * b) - sA - sC - sG;
  const uint32_t tA = h0.x + sA, tC = h0.y + sC, tG = h0.z + sG, tT = h0.w + sT;
  uint64_t w0, w1, w2;
  block_words(sa, sbk, b, w0, w1, w2);
  uint32_t e, g;
  block_eg(w0, w1, w2, r, sm, e, g);
  const uint32_t te = c == 0 ? tA : (c == 1 ? tC : (c == 2 ? tG : tT));
  const uint32_t tg = (c < 1 ? tC : 0u) + (c < 2 ? tG : 0u) + (c < 3 ? tT : 0u);
  E = sbe + te + e;
  G = sbg + tg + g;
}

// B[x] (2-bit code; the $ row reads as A) from the block slices of row o
__device__ __forceinline__ int bwt_from_block(uint4 sa, uint4 sbk, int o) {
  const int b = block_of(o);
  uint64_t w0, w1, w2;
  block_words(sa, sbk, b, w0, w1, w2);
  const int q = (o >> 5) - 3 * b;
  const uint64_t w = q == 0 ? w0 : (q == 1 ? w1 : w2);
  return (int)((w >> (2 * (o & 31))) & 3);
}

// Superblock values for symbol c: count of c before superblock s, and the sum over d > c.
__device__ __forceinline__ void sb_values(const uint64_t *sbtab, uint32_t line, int c, uint64_t &sbe, uint64_t &sbg) {
  const uint64_t *t = sbtab + 8 * (line >> MBW_SB_SHIFT);
  sbe = t[c];
  sbg = t[4 + c];
}

// Algorithm 1 as one unified step.  (x, y, s) is the interval with x the side that is LF-mapped
// (backward: (k, k'), forward: (k', k)) and c the symbol mapped (backward: a, forward: comp(a)).
//   s'  = Occ(c, x+s) - Occ(c, x)
//   x'  = C(c) + Occ(c, x)
//   y'  = y + [x <= primary < x+s] + sum_{d > c} (Occ(d, x+s) - Occ(d, x))
// The last line is the k' update of BackwardExt: the symbols b < comp(c) (b = $ included) are
// exactly $ and the complements of the bases d > c.  E1/G1 and E2/G2 are (Occ(c,.), sum_{d>c}
// Occ(d,.)) at x and x+s before the $ correction.
__device__ __forceinline__ void ext_update(uint64_t E1, uint64_t G1, uint64_t E2, uint64_t G2, int c, uint64_t x,
                                           uint64_t s, uint64_t y, uint64_t primary, const uint64_t Cb[4],
                                           uint64_t &nx, uint64_t &ny, uint64_t &ns) {
  const uint64_t x2 = x + s;
  if (c == 0) { E1 -= x > primary ? 1 : 0; E2 -= x2 > primary ? 1 : 0; }
  const uint64_t dol = (x <= primary && primary < x2) ? 1 : 0;
  ns = E2 - E1;
  nx = sel4(Cb[0], Cb[1], Cb[2], Cb[3], c) + E1;
  ny = y + dol + (G2 - G1);
}

// Single-lane rank straight from global memory (plain kernels, index builder).
__device__ __forceinline__ void rank_global(const IndexView &ix, uint64_t x, int c, uint64_t &E, uint64_t &G) {
  const uint32_t L = line_of(x);
  const int o = (int)(x - (uint64_t)L * MBW_BPL);
  const uint4 *ln = ix.lines + (uint64_t)L * MBW_LINE_U4;
  const int sl = block_slice(o);
  const uint4 h0 = ln[0], h1 = ln[1], sa = ln[sl], sbk = ln[sl + 1];
  uint64_t sbe, sbg;
  sb_values(ix.sbtab, L, c, sbe, sbg);
  rank_eg(h0, h1, sa, sbk, o, c, sym_masks(c), sbe, sbg, E, G);
}

// B[x] from global memory
__device__ __forceinline__ int bwt_global(const IndexView &ix, uint64_t x) {
  const uint32_t L = line_of(x);
  const int o = (int)(x - (uint64_t)L * MBW_BPL);
  const uint64_t *w = (const uint64_t *)(ix.lines + (uint64_t)L * MBW_LINE_U4);
  return (int)((w[4 + (o >> 5)] >> (2 * (o & 31))) & 3);
}

// unpack a k-mer table entry (k:40 | k':40 | s:40)
__device__ __forceinline__ void kmer_unpack(uint4 e, uint64_t &k, uint64_t &kr, uint64_t &s) {
  uint64_t w0 = ((uint64_t)e.y << 32) | e.x, w1 = ((uint64_t)e.w << 32) | e.z;
  k = w0 & ((1ull << 40) - 1);
  kr = (w0 >> 40) | ((w1 & 0xffff) << 24);
  s = w1 >> 16;
}
__host__ __device__ __forceinline__ uint4 kmer_pack(uint64_t k, uint64_t kr, uint64_t s) {
  uint64_t w0 = (k & ((1ull << 40) - 1)) | (kr << 40);
  uint64_t w1 = ((kr >> 24) & 0xffff) | (s << 16);
  uint4 e;
  e.x = (uint32_t)w0; e.y = (uint32_t)(w0 >> 32); e.z = (uint32_t)w1; e.w = (uint32_t)(w1 >> 32);
  return e;
}
