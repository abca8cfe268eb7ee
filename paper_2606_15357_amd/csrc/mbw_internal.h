// Internal definitions shared by the mbw HIP sources (index layout, device rank helpers).
//
// Layout of the resident FM-index (Sections 2.1, 2.2 and 2.4 of the paper, redesigned for gfx950):
//   * occurrence lines: 128 bytes each, 128-byte aligned.  Words 0..3 hold the counts of A, C, G, T
//     in B[0, 384*line) (the $ row is stored and counted as A; rank corrects for it), words 4..15 hold
//     rows 384*line .. 384*line+383 of B at 2 bits (row t in word 4 + t/32, bits 2*(t%32)).
//     A random HBM access on MI355X moves one 128-byte L2 line, so one rank query costs exactly one
//     line transfer; eight lanes fetch the line together (16 bytes each, one load instruction).
//   * sampled SA: ssa[x / r] = S(x) for rows x that are multiples of r.
//   * k-mer table: 4^K packed ds-intervals (16 bytes), code = sum_q P[q] * 4^(K-1-q).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#define MBW_BPL 384            // rows of B per occurrence line
#define MBW_LINE_BYTES 128
#define MBW_LINE_U4 8          // uint4 per line
#define MBW_GROUP 8            // lanes that cooperate on one line
#define MBW_MAX_READ 65535

struct mbw_index {
  int device;
  uint64_t n, len_r, primary, n_lines, n_ssa;
  uint64_t C[5];               // C[$], C[A], C[C], C[G], C[T]
  int sa_sample, kmer_k, bisulfite;
  uint4 *lines;                // n_lines * 8
  uint64_t *ssa;               // n_ssa
  uint4 *kmer;                 // 4^K (or nullptr)
  uint64_t bytes;
};

// Read-only view passed by value to kernels.
struct IndexView {
  const uint4 *__restrict__ lines;
  const uint64_t *__restrict__ ssa;
  const uint4 *__restrict__ kmer;
  uint64_t n, primary;
  uint64_t Cb[4];              // C of base a (A..T) = |{i : B[i] < a}| (includes the $ row)
  uint32_t r;
  int K;
};

static inline IndexView make_view(const mbw_index *ix) {
  IndexView v;
  v.lines = ix->lines; v.ssa = ix->ssa; v.kmer = ix->kmer;
  v.n = ix->n; v.primary = ix->primary;
  for (int a = 0; a < 4; ++a) v.Cb[a] = ix->C[a + 1];
  v.r = (uint32_t)ix->sa_sample; v.K = ix->kmer_k;
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

// x / 384 = (x >> 7) / 3, the division by 3 as a multiply-high by ceil(2^65 / 3)
__device__ __forceinline__ uint64_t line_of(uint64_t x) { return __umul64hi(x >> 7, 0xAAAAAAAAAAAAAAABull) >> 1; }

#define M55 0x5555555555555555ull

// Counts of A, C, G (packed 3 x 16 bits; T is derived) among the first m (0..32) rows of a word.
__device__ __forceinline__ uint64_t word_counts(uint64_t w, int m) {
  uint64_t mask = m >= 32 ? M55 : (((1ull << (2 * m)) - 1) & M55);
  uint64_t hi = (w >> 1) & M55, lo = w & M55;
  uint32_t nA = __popcll(~(hi | lo) & mask);
  uint32_t nC = __popcll(~hi & lo & mask);
  uint32_t nG = __popcll(hi & ~lo & mask);
  uint32_t nT = (uint32_t)m - nA - nC - nG;
  return (uint64_t)nA | ((uint64_t)nC << 16) | ((uint64_t)nG << 32) | ((uint64_t)nT << 48);
}

// Cooperative part: this lane's 16-byte slice `d` of a line (slice q of 8).  Returns the packed
// 4 x 16-bit counts of A,C,G,T among rows [0, o) of the line that lie in this slice (0 for the
// two count slices).
__device__ __forceinline__ uint64_t slice_counts(uint4 d, int q, int o) {
  if (q < 2) return 0;
  int m = o - (q - 2) * 64;
  m = m < 0 ? 0 : (m > 64 ? 64 : m);
  uint64_t w0 = ((uint64_t)d.y << 32) | d.x, w1 = ((uint64_t)d.w << 32) | d.z;
  int m0 = m < 32 ? m : 32, m1 = m > 32 ? m - 32 : 0;
  return word_counts(w0, m0) + word_counts(w1, m1);
}

__device__ __forceinline__ uint64_t group_sum(uint64_t v) {
  v += __shfl_xor(v, 1, MBW_GROUP);
  v += __shfl_xor(v, 2, MBW_GROUP);
  v += __shfl_xor(v, 4, MBW_GROUP);
  return v;
}

__device__ __forceinline__ uint64_t f16(uint64_t packed, int a) { return (packed >> (16 * a)) & 0xffff; }

// Occ(a, x) for all four bases from a line held cooperatively: hdr = the line's four counts
// (every lane), inl = group-summed packed in-line counts for offset x % 384.  The $ row is stored
// as A, so Occ(A, x) loses one when x > primary.
struct Occ4 { uint64_t v[4]; };
__device__ __forceinline__ Occ4 occ_from(const uint64_t hdr[4], uint64_t inl, uint64_t x, uint64_t primary) {
  Occ4 o;
#pragma unroll
  for (int a = 0; a < 4; ++a) o.v[a] = hdr[a] + f16(inl, a);
  o.v[0] -= (x > primary) ? 1 : 0;
  return o;
}

// Broadcast the four header counts of a line held by the group (slices 0 and 1).
__device__ __forceinline__ void group_header(uint4 d, uint64_t hdr[4]) {
  uint64_t lo = ((uint64_t)d.y << 32) | d.x, hi = ((uint64_t)d.w << 32) | d.z;
  hdr[0] = __shfl(lo, 0, MBW_GROUP);
  hdr[1] = __shfl(hi, 0, MBW_GROUP);
  hdr[2] = __shfl(lo, 1, MBW_GROUP);
  hdr[3] = __shfl(hi, 1, MBW_GROUP);
}

__device__ __forceinline__ uint64_t sel4(uint64_t a0, uint64_t a1, uint64_t a2, uint64_t a3, int c) {
  return c == 0 ? a0 : (c == 1 ? a1 : (c == 2 ? a2 : a3));
}

// Algorithm 1 as one unified step.  (x, y, s) is the interval with x the side that is LF-mapped
// (backward: (k, k'), forward: (k', k)) and c the symbol mapped (backward: a, forward: comp(a)).
//   s'  = Occ(c, x+s) - Occ(c, x)
//   x'  = C(c) + Occ(c, x)
//   y'  = y + [x <= primary < x+s] + sum_{d > c} (Occ(d, x+s) - Occ(d, x))
// The last line is the k' update of BackwardExt: the symbols b < comp(c) (b = $ included) are
// exactly $ and the complements of the bases d > c.
__device__ __forceinline__ void ext_update(const Occ4 &o1, const Occ4 &o2, int c, uint64_t x, uint64_t s,
                                           uint64_t y, uint64_t primary, const uint64_t Cb[4],
                                           uint64_t &nx, uint64_t &ny, uint64_t &ns) {
  uint64_t a1 = sel4(o1.v[0], o1.v[1], o1.v[2], o1.v[3], c);
  uint64_t a2 = sel4(o2.v[0], o2.v[1], o2.v[2], o2.v[3], c);
  uint64_t gt = (c < 1 ? o2.v[1] - o1.v[1] : 0) + (c < 2 ? o2.v[2] - o1.v[2] : 0) + (c < 3 ? o2.v[3] - o1.v[3] : 0);
  uint64_t dol = (x <= primary && primary < x + s) ? 1 : 0;
  ns = a2 - a1;
  nx = sel4(Cb[0], Cb[1], Cb[2], Cb[3], c) + a1;
  ny = y + dol + gt;
}

// ---- cooperative rank: eight lanes, one 16-byte slice of a 128-byte line each ----------------

// DPP exchanges inside each group of eight lanes (quad_perm [1,0,3,2], [2,3,0,1], row_half_mirror)
__device__ __forceinline__ uint32_t dpp_x1(uint32_t v) { return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false); }
__device__ __forceinline__ uint32_t dpp_x2(uint32_t v) { return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false); }
__device__ __forceinline__ uint32_t dpp_hm(uint32_t v) { return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false); }
__device__ __forceinline__ uint64_t dpp64(uint64_t v, int which) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  if (which == 0) { lo = dpp_x1(lo); hi = dpp_x1(hi); }
  else if (which == 1) { lo = dpp_x2(lo); hi = dpp_x2(hi); }
  else { lo = dpp_hm(lo); hi = dpp_hm(hi); }
  return ((uint64_t)hi << 32) | lo;
}
// sum over the eight lanes of the group, result in every lane
__device__ __forceinline__ uint64_t grp_sum64(uint64_t v) {
  v += dpp64(v, 0);
  v += dpp64(v, 1);
  v += dpp64(v, 2);
  return v;
}
__device__ __forceinline__ uint32_t grp_sum32(uint32_t v) {
  v += dpp_x1(v);
  v += dpp_x2(v);
  v += dpp_hm(v);
  return v;
}

// rows of symbol c (eq) and of symbols greater than c (gt) among the first m (0..32) rows of a word
__device__ __forceinline__ void word_eq_gt(uint64_t w, int m, int c, uint32_t &eq, uint32_t &gt) {
  uint64_t mask = m >= 32 ? M55 : (((1ull << (2 * m)) - 1) & M55);
  uint64_t hi = (w >> 1) & M55, lo = w & M55;
  uint64_t e = c == 0 ? ~(hi | lo) : (c == 1 ? (~hi & lo) : (c == 2 ? (hi & ~lo) : (hi & lo)));
  uint64_t g = c == 0 ? (hi | lo) : (c == 1 ? hi : (c == 2 ? (hi & lo) : 0ull));
  eq = __popcll(e & mask);
  gt = __popcll(g & mask);
}

// This lane's share of Occ(c, x) (E) and of sum_{d>c} Occ(d, x) (G), x at offset o of the line
// whose slice q is d: slices 0/1 contribute the line's prefix counts, slices 2..7 their rows < o.
__device__ __forceinline__ void slice_eg(uint4 d, int q, int o, int c, uint64_t &E, uint64_t &G) {
  uint64_t w0 = ((uint64_t)d.y << 32) | d.x, w1 = ((uint64_t)d.w << 32) | d.z;
  if (q == 0) {            // counts of A, C
    E = c == 0 ? w0 : (c == 1 ? w1 : 0);
    G = c == 0 ? w1 : 0;
  } else if (q == 1) {     // counts of G, T
    E = c == 2 ? w0 : (c == 3 ? w1 : 0);
    G = (c <= 1 ? w0 : 0) + (c <= 2 ? w1 : 0);
  } else {
    int m = o - (q - 2) * 64;
    m = m < 0 ? 0 : (m > 64 ? 64 : m);
    uint32_t e0, g0, e1, g1;
    word_eq_gt(w0, m < 32 ? m : 32, c, e0, g0);
    word_eq_gt(w1, m > 32 ? m - 32 : 0, c, e1, g1);
    E = e0 + e1;
    G = g0 + g1;
  }
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

// Single-lane rank (no cooperation): Occ(a, x) for all a, reading the line's counts and only the
// 16-byte slices that hold rows before x.  Used by the plain kernels and the index builder.
__device__ __forceinline__ Occ4 occ_single(const uint4 *__restrict__ lines, uint64_t x, uint64_t primary) {
  uint64_t L = line_of(x);
  int o = (int)(x - L * MBW_BPL);
  const uint4 *ln = lines + L * MBW_LINE_U4;
  uint4 h0 = ln[0], h1 = ln[1];
  uint64_t inl = 0;
  for (int q = 2; q < 8 && (q - 2) * 64 < o; ++q) inl += slice_counts(ln[q], q, o);
  uint64_t hdr[4] = {((uint64_t)h0.y << 32) | h0.x, ((uint64_t)h0.w << 32) | h0.z,
                     ((uint64_t)h1.y << 32) | h1.x, ((uint64_t)h1.w << 32) | h1.z};
  return occ_from(hdr, inl, x, primary);
}

// B[x] (2-bit code; the $ row reads as A) from a single lane.
__device__ __forceinline__ int bwt_single(const uint4 *__restrict__ lines, uint64_t x) {
  uint64_t L = line_of(x);
  int o = (int)(x - L * MBW_BPL);
  const uint64_t *w = (const uint64_t *)(lines + L * MBW_LINE_U4);
  return (int)((w[4 + (o >> 5)] >> (2 * (o & 31))) & 3);
}
