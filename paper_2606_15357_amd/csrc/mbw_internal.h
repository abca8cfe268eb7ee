// Internal definitions shared by the mbw HIP sources: index layout and device rank helpers.
//
// Resident FM-index (paper Sections 2.1, 2.2 and 2.4; the line format is this library's own,
// sized for gfx950 where a random HBM access moves one 128-byte L2 line):
//   * occurrence lines, 128 bytes each (8 slices of 16 bytes), one per 384 rows of B:
//       slice 0     u32 counts of A, C, G in B from the start of the line's superblock (2^h
//                   lines, h = 23 by default and smaller on request) up to the line (the $ row is
//                   stored and counted as A; rank corrects it), then sub-checkpoint 1
//       slice 1     sub-checkpoints 2, 3, 4, 5
//                   (sub-checkpoint b: counts of A, C, G in the line's first 64 b rows, 9 bits
//                   each at bits 0, 9, 18 of a u32)
//       slices 2-7  the six 64-row blocks as bit planes: u64 of low code bits, then u64 of high
//                   code bits, row t of the block at bit t
//     T counts follow from row counts, so a rank query reads three slices of one line (the two
//     header slices and its block) and counts at most 63 rows by popcount.
//   * superblock table: absolute counts of A, C, G, T before each superblock, plus their suffix
//     sums (for the k' update of backward extension).
//   * sampled SA: ssa[x / r] = S(x) for rows x that are multiples of r.
//   * k-mer table: 4^K packed ds-intervals (16 bytes); the code of P[0..K) is sum_q P[q] 4^q.
//   * optional: the text T without its $ (2 bits per symbol, 32 per u64, first symbol in the low
//     bits) and the inverse suffix array at text positions that are multiples of q,
//     isa[t / q] = the row whose suffix starts at t.
//   * bisulfite indexes: the original (unconverted) reference R, packed like the text.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#define MBW_BPL 384            // rows of B per occurrence line
#define MBW_LINE_BYTES 128
#define MBW_LINE_U4 8          // 16-byte slices per line
#define MBW_BLK 64             // rows per block (one 16-byte slice)
#define MBW_SB_SHIFT 23        // default and largest log2 of the lines per superblock (3.2 G rows < 2^32)
#define MBW_MAX_SB 8           // superblocks an index may have (the table lives in LDS)
#define MBW_MAX_READ 65535

struct mbw_index {
  int device;
  uint64_t n, len_r, primary, n_lines, n_ssa;
  uint64_t C[5];               // C[$], C[A], C[C], C[G], C[T]
  int sa_sample, kmer_k, bisulfite;
  int n_sb;
  int sb_shift;                // log2 of the lines per superblock (1..MBW_SB_SHIFT)
  uint64_t sb_host[MBW_MAX_SB * 8];
  uint4 *lines;                // n_lines * 8
  uint64_t *ssa;               // n_ssa
  uint4 *kmer;                 // 4^K (or nullptr)
  uint64_t *sbtab;             // n_sb * 8: counts of A,C,G,T before the superblock, then sums of d > c
  int isa_sample;              // 0: no text / inverse-SA samples
  uint64_t n_text, n_isa;      // u64 words of the packed text, inverse-SA samples
  uint64_t *text;
  uint64_t *isa;
  uint64_t n_orig;             // bisulfite indexes: the original reference, packed like the text
  uint64_t *orig;
  uint64_t bytes;
  struct mbw_contigs *contigs; // host: the reference's records (names, start and length in R)
  int users;                   // contexts and servers using the index (mbw_index_retain)
  bool free_pending;           // mbw_index_free came while it was in use: freed by the last release
};

// An index stays allocated while contexts or servers use it: they retain it when created and
// release it when freed; mbw_index_free on an index in use defers the free to the last release.
void mbw_index_retain(const mbw_index *ix);
void mbw_index_release(const mbw_index *ix);

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
  uint32_t sb_shift;           // superblock of line L: L >> sb_shift
  const uint64_t *__restrict__ text;   // packed T without $ (nullptr when absent)
  const uint64_t *__restrict__ isa;    // isa[t / ri] = row of the suffix at t
  uint32_t ri;
  const uint64_t *__restrict__ orig;   // bisulfite: the original reference, packed (nullptr otherwise)
  uint64_t len_r;
};

static inline IndexView make_view(const mbw_index *ix) {
  IndexView v;
  v.lines = ix->lines; v.ssa = ix->ssa; v.kmer = ix->kmer; v.sbtab = ix->sbtab;
  v.n = ix->n; v.primary = ix->primary;
  for (int a = 0; a < 4; ++a) v.Cb[a] = ix->C[a + 1];
  v.r = (uint32_t)ix->sa_sample; v.K = ix->kmer_k; v.n_sb = ix->n_sb; v.sb_shift = (uint32_t)ix->sb_shift;
  v.text = ix->text; v.isa = ix->isa; v.ri = (uint32_t)ix->isa_sample;
  v.orig = ix->orig; v.len_r = ix->len_r;
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

__device__ __forceinline__ uint64_t sel4(uint64_t a0, uint64_t a1, uint64_t a2, uint64_t a3, int c) {
  return c == 0 ? a0 : (c == 1 ? a1 : (c == 2 ? a2 : a3));
}

// Per-symbol constants of the bit-plane rank.  Rows equal to c: low plane xor lc and high plane
// xor hc both zero.  Rows greater than c: (hi & (lo | ga)) | (lo & gb), kept only if c < 3.
struct SymMasks { uint32_t lc, hc, ga, gb; bool any_gt; };
__device__ __forceinline__ SymMasks sym_masks(int c) {
  SymMasks m;
  m.lc = (c & 1) ? ~0u : 0u;
  m.hc = (c & 2) ? ~0u : 0u;
  m.ga = c <= 1 ? ~0u : 0u;
  m.gb = c == 0 ? ~0u : 0u;
  m.any_gt = c < 3;
  return m;
}

// rows equal to c (e) and greater than c (g) among the first r (0..63) rows of a block
__device__ __forceinline__ void block_eg(uint4 blk, int r, const SymMasks &sm, uint32_t &e, uint32_t &g) {
  const uint64_t m = (1ull << r) - 1;
  const uint32_t m0 = (uint32_t)m, m1 = (uint32_t)(m >> 32);
  const uint32_t l0 = blk.x, l1 = blk.y, h0 = blk.z, h1 = blk.w;
  const uint32_t x0 = (l0 ^ sm.lc) | (h0 ^ sm.hc), x1 = (l1 ^ sm.lc) | (h1 ^ sm.hc);
  e = __popc(m0 & ~x0) + __popc(m1 & ~x1);
  const uint32_t g0 = (h0 & (l0 | sm.ga)) | (l0 & sm.gb), g1 = (h1 & (l1 | sm.ga)) | (l1 & sm.gb);
  g = sm.any_gt ? __popc(m0 & g0) + __popc(m1 & g1) : 0u;
}

// the sub-checkpoint word of block b (0 for block 0)
__device__ __forceinline__ uint32_t sub_word(uint4 h0, uint4 h1, int b) {
  return b == 0 ? 0u : (b == 1 ? h0.w : (b == 2 ? h1.x : (b == 3 ? h1.y : (b == 4 ? h1.z : h1.w))));
}

// Occ(c, x) (E) and sum_{d > c} Occ(d, x) (G), x at offset o of a line that is line Lrel of its
// superblock, from the line's two header slices and the slice of block o / 64, and the superblock
// values sbe = count of c before the superblock, sbg = sum over d > c of the counts before it.  The
// $ row is not corrected here.
__device__ __forceinline__ void rank_eg(uint4 h0, uint4 h1, uint4 blk, uint32_t Lrel, int o, int c, const SymMasks &sm,
                                        uint64_t sbe, uint64_t sbg, uint64_t &E, uint64_t &G) {
  const int b = o >> 6, r = o & 63;
  const uint32_t sw = sub_word(h0, h1, b);
  const uint32_t sA = sw & 511u, sC = (sw >> 9) & 511u, sG = (sw >> 18) & 511u;
  const uint32_t rows = MBW_BPL * Lrel + MBW_BLK * b;   // rows of the superblock before the block
  const uint32_t tA = h0.x + sA, tC = h0.y + sC, tG = h0.z + sG, tT = rows - tA - tC - tG;
  uint32_t e, g;
  block_eg(blk, r, sm, e, g);
  const uint32_t te = c == 0 ? tA : (c == 1 ? tC : (c == 2 ? tG : tT));
  const uint32_t tg = (c < 1 ? tC : 0u) + (c < 2 ? tG : 0u) + (c < 3 ? tT : 0u);
  E = sbe + (uint64_t)(te + e);
  G = sbg + (uint64_t)(tg + g);
}

// B[x] (2-bit code; the $ row reads as A) from the block slice of row o
__device__ __forceinline__ int bwt_from_block(uint4 blk, int o) {
  const int r = o & 63;
  const uint32_t lo = r < 32 ? blk.x : blk.y, hi = r < 32 ? blk.z : blk.w;
  return (int)(((lo >> (r & 31)) & 1u) | (((hi >> (r & 31)) & 1u) << 1));
}

// Superblock values for symbol c: count of c before the superblock of `line`, and the sum over d > c.
__device__ __forceinline__ void sb_values(const uint64_t *sbtab, uint32_t line, uint32_t sb_shift, int c, uint64_t &sbe,
                                          uint64_t &sbg) {
  const uint64_t *t = sbtab + 8 * (line >> sb_shift);
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
// Occ(d,.)) at x and x+s before the $ correction; Cc = C(c).
__device__ __forceinline__ void ext_update(uint64_t E1, uint64_t G1, uint64_t E2, uint64_t G2, int c, uint64_t x,
                                           uint64_t s, uint64_t y, uint64_t primary, uint64_t Cc,
                                           uint64_t &nx, uint64_t &ny, uint64_t &ns) {
  const uint64_t x2 = x + s;
  if (c == 0) { E1 -= x > primary ? 1 : 0; E2 -= x2 > primary ? 1 : 0; }
  const uint64_t dol = (x <= primary && primary < x2) ? 1 : 0;
  ns = E2 - E1;
  nx = Cc + E1;
  ny = y + dol + (G2 - G1);
}

// Single-lane rank straight from global memory (plain kernels, index builder).
__device__ __forceinline__ void rank_global(const IndexView &ix, uint64_t x, int c, uint64_t &E, uint64_t &G) {
  const uint32_t L = line_of(x);
  const int o = (int)(x - (uint64_t)L * MBW_BPL);
  const uint4 *ln = ix.lines + (uint64_t)L * MBW_LINE_U4;
  const uint4 h0 = ln[0], h1 = ln[1], blk = ln[2 + (o >> 6)];
  uint64_t sbe, sbg;
  sb_values(ix.sbtab, L, ix.sb_shift, c, sbe, sbg);
  rank_eg(h0, h1, blk, L & ((1u << ix.sb_shift) - 1), o, c, sym_masks(c), sbe, sbg, E, G);
}

// B[x] from global memory
__device__ __forceinline__ int bwt_global(const IndexView &ix, uint64_t x) {
  const uint32_t L = line_of(x);
  const int o = (int)(x - (uint64_t)L * MBW_BPL);
  return bwt_from_block(ix.lines[(uint64_t)L * MBW_LINE_U4 + 2 + (o >> 6)], o);
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
