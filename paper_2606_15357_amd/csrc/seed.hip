// Batched (l,c)-SMEM seeding and sampled-SA locate (paper Sections 2.1, 2.4, 2.5, 2.6, 2.9).
//
// Pipeline of one mbw_seed call (all on one stream):
//   encode      ASCII -> codes 0..3 (4 = matches nothing), bisulfite read conversion (Section 2.9),
//               then 2-bit packing (32 bases per word + one N bit per base)
//   smem        round 1: (l,c)-SMEMs of every read (Algorithm 3), appended to a seed list; SMEMs that
//               qualify for re-seeding are appended to a sub-query list
//   smem        round 2 (Section 2.6): (floor(len/2), s+1)-SMEMs of each sub-query
//   sort/dedup  seeds sorted by (read, qbeg, qend); duplicates from overlapping parents dropped
//   scan        per-seed position counts (s <= max_occ) -> offsets
//   locate      Algorithm 2: LF-walk every SA row of every located seed to a sampled row
//   filter      bisulfite strand filter on positions (Section 2.9)
//
// Two kernel families run the smem and locate steps:
//   * wave (default): persistent kernels in which every lane owns one query (or one locate walk)
//     and each iteration has exactly one memory phase: every lane issues the loads its step needs
//     (the three 16-byte slices of each occurrence line its rank reads, into registers), k-mer
//     table entries, records of new queries and the words of reads being staged (those three
//     straight into LDS), and the wave waits once; then each lane ranks from its own registers.
//     Reads of up to 160 bases are staged in LDS for the whole query.
//   * plain (the baseline): one thread runs the serial algorithm for one read (round 2 inline) and
//     one thread locates one seed; ranks read their line straight from global memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>
#include <type_traits>
#include <cstdio>
#include <cstdlib>

#include "ctx.h"
#include "mbw_internal.h"
#include "prim.h"
#include "../../include/mbw.h"

#define TRY(call) MBW_HIP_TRY(call)

namespace {

// a query string: read_id's bases [qbeg, qend) with its own (l, c); rlen / woff locate the packed read.
// A long query is split into segments: the segment [qbeg, send) of the query [q0, qend) reports the
// SMEMs of P[q0, qend) whose start lies in [qbeg, send).  Those are the SMEMs of P[qbeg, qend) with
// such a start, except that one starting at qbeg > q0 is an SMEM of the whole query only if it
// cannot be extended to the left (SEG_CHECK: one backward step decides).
#define SEG_CHECK 1u
struct Query { uint32_t read_id, qbeg, qend, l, c, rlen, woff_lo, woff_hi, send, flags, pad0, pad1; };   // 48 bytes
// A query resumed after a unique match that a continuation pass finished: the lane starts in stage 3
// at the match [pad0, pad1) instead of stage 1 at qbeg.
#define Q_RESUME 2u
// A unique match handed from the SMEM kernel to the continuation kernel: the query (its record's
// first eight words), the match P[i, j) with interval (k, kr) and s = 1.
struct UTask { uint32_t read_id, qbeg, qend, l, c, rlen, woff_lo, woff_hi, i, j, pad0, pad1; uint64_t k, kr; };   // 64 bytes
#define INVALID_READ 0xFFFFFFFFu   // unused slot of a per-wave output chunk
// pos: the text position of the SMEM when the unique-match path found it (s = 1), else NO_POS
#define NO_POS 0xFFFFFFFFFFFFFFFFull
struct SeedRec { uint32_t read_id, qbeg, qend, flags; uint64_t k, kr, s, pos; };

// control block (device): counters shared by the kernels of one call
enum { C_WORK = 0, C_NSEEDS = 1, C_NSUBQ = 2, C_LINES = 3, C_STEPS = 4, C_KMER = 5, C_LFSTEPS = 6, C_SAREADS = 7,
       C_LINES_LOC = 8, C_WORK2 = 9, C_MAXLEN = 10, C_ERR = 11, C_WITER = 12, C_LITER = 13, C_MAXCHAIN = 14,
       C_PASSQ = 15,   // slots of the task or resume list a continuation pass writes
       C_COUNT = 16 };

struct SeedParams {
  const uint8_t *__restrict__ codes;   // one code per base (plain kernel)
  const uint64_t *__restrict__ offs;   // read offsets (n_reads + 1)
  const Query *__restrict__ queries;   // round 2; nullptr in round 1
  uint64_t n_queries;
  uint32_t chunk;                      // queries per work-queue grab
  int l, c;                            // round 1 parameters
  int reseed, reseed_len, reseed_occ, round;
  int use_kmer;
  int uniq;                            // extend s = 1 matches against the text (index has text + ISA)
  uint32_t rmask;                      // r - 1 (the unique path needs r a power of two)
  int rshift;                          // log2 r
  int rishift;                         // log2 of the inverse-SA sampling step
  SeedRec *__restrict__ seeds;
  uint64_t seed_cap;
  Query *__restrict__ subq;
  uint64_t subq_cap;
  unsigned long long *__restrict__ ctl;
  // unique-match continuations (round 1, staged reads): the SMEM kernel writes tasks, the
  // continuation kernel reads them (n_queries of them) and writes the queries to resume
  UTask *__restrict__ tasks;
  uint64_t task_cap;
  Query *__restrict__ resume;
  uint64_t resume_cap;
  // captured graphs: the query count on the device (at most n_queries, which sized the grid)
  const unsigned long long *__restrict__ nq_dev;
};

struct ReadWords {
  const uint64_t *__restrict__ pw;     // packed bases, 2 bits each, 32 per word (read-aligned)
  const uint32_t *__restrict__ pn;     // one N bit per base, 32 per word
  const uint64_t *__restrict__ woff;   // first word of each read (n_reads + 1)
};

inline unsigned grid_for(uint64_t n, unsigned bs = 256, unsigned cap = 65536u * 8) {
  uint64_t g = (n + bs - 1) / bs;
  if (g < 1) g = 1;
  return (unsigned)std::min<uint64_t>(g, cap);
}

// ---------------------------------------------------------------------------------------------
// encode / pack
__global__ void k_encode(const uint8_t *__restrict__ in, uint64_t total, int role, uint8_t *__restrict__ out) {
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < total; t += (uint64_t)gridDim.x * blockDim.x) {
    uint8_t ch = in[t], c;
    switch (ch) {
      case 'A': case 'a': c = 0; break;
      case 'C': case 'c': c = 1; break;
      case 'G': case 'g': c = 2; break;
      case 'T': case 't': c = 3; break;
      default: c = 4;
    }
    if (role == 1 && c == 1) c = 3;   // read 1: C -> T
    if (role == 2 && c == 2) c = 0;   // read 2: G -> A
    out[t] = c;
  }
}

__global__ void k_widen(const uint32_t *__restrict__ len, uint64_t n, uint64_t *__restrict__ out,
                        unsigned long long *__restrict__ maxlen) {
  uint32_t mx = 0;
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t <= n; t += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t v = t < n ? len[t] : 0u;
    out[t] = v;
    mx = v > mx ? v : mx;
  }
  for (int d = 32; d >= 1; d >>= 1) {                   // wave maximum, one atomic per wave
    const uint32_t o = (uint32_t)__shfl_xor((int)mx, d);
    mx = o > mx ? o : mx;
  }
  if ((threadIdx.x & 63) == 0 && mx) atomicMax(maxlen, (unsigned long long)mx);
}

__global__ void k_read_words(const uint64_t *__restrict__ offs, uint64_t n, uint64_t *__restrict__ nwords) {
  for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r <= n; r += (uint64_t)gridDim.x * blockDim.x)
    nwords[r] = r < n ? (offs[r + 1] - offs[r] + 31) / 32 : 0;
}

// owner read of every packed word (word w of read r: wread[woff[r] + w] = r)
__global__ void k_word_owner(const uint64_t *__restrict__ woff, uint64_t n, uint32_t *__restrict__ wread) {
  for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r < n; r += (uint64_t)gridDim.x * blockDim.x)
    for (uint64_t w = woff[r]; w < woff[r + 1]; ++w) wread[w] = (uint32_t)r;
}

// one thread per packed word: 32 ASCII bases -> 2-bit codes + N bits (bisulfite conversion as in
// k_encode; the code of an ACGT byte is its bits 1-2 with the Gray-code swap of G and T).  The words of a block cover one contiguous byte range of the reads (reads are stored
// back to back and split into words in order), which the block first copies into LDS with
// coalesced 16-byte loads (byte loads at the ends of the buffer).
#define PACK_BLOCK 256
__global__ void __launch_bounds__(PACK_BLOCK) k_pack_words(const uint8_t *__restrict__ ascii, uint64_t total,
                                                           const uint64_t *__restrict__ offs, const uint64_t *__restrict__ woff,
                                                           const uint32_t *__restrict__ wread, uint64_t totw, int role,
                                                           uint64_t *__restrict__ pw, uint32_t *__restrict__ pn,
                                                           const uint64_t *__restrict__ total_p = nullptr,
                                                           const uint64_t *__restrict__ totw_p = nullptr) {
  // total_p / totw_p (captured graphs): the batch's bytes and words on the device, at most the
  // capacities total / totw that the grid was sized for
  if (total_p) total = min(total, *total_p);
  if (totw_p) totw = min(totw, *totw_p);
  // the range (<= 32 * PACK_BLOCK + 30 bytes from a 16-byte boundary) in 32-bit words, one pad word
  // after every 8 (word i at i + i / 8), so that the 32 words that a thread converts, 8 words after its
  // neighbour's, fall in distinct banks
  __shared__ uint32_t buf[(PACK_BLOCK * 8 + 16) * 9 / 8 + 4];
  __shared__ uint64_t range[2];
  const uint64_t w0 = (uint64_t)blockIdx.x * PACK_BLOCK;
  if (w0 >= totw) return;
  const uint64_t w1 = min(w0 + PACK_BLOCK, totw);
  if (threadIdx.x == 0) {
    const uint32_t r0 = wread[w0], r1 = wread[w1 - 1];
    range[0] = offs[r0] + 32 * (w0 - woff[r0]);
    range[1] = min(offs[r1] + 32 * (w1 - 1 - woff[r1]) + 32, offs[r1 + 1]);
  }
  __syncthreads();
  const uint64_t b0 = range[0], b1 = range[1];
  const uint64_t a0 = b0 & ~15ull;                      // first 16-byte boundary of the range
  const uint32_t nq = (uint32_t)((b1 - a0 + 15) >> 4);  // 16-byte pieces, <= 2 * PACK_BLOCK + 2
  const bool aligned = (((uintptr_t)ascii) & 15) == 0;
  auto pad = [](uint32_t i) { return i + (i >> 3); };
  for (uint32_t t = threadIdx.x; t < nq; t += PACK_BLOCK) {
    const uint64_t byte = a0 + 16ull * t;
    uint32_t v[4];
    if (aligned && byte + 16 <= total) {
      const uint4 x = *(const uint4 *)(ascii + byte);
      v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        v[u] = 0;
        for (int q = 0; q < 4; ++q)
          if (byte + 4 * u + q < total) v[u] |= (uint32_t)ascii[byte + 4 * u + q] << (8 * q);
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) buf[pad(4 * t + u)] = v[u];
  }
  __syncthreads();
  const uint64_t w = w0 + threadIdx.x;
  if (w >= w1) return;
  const uint32_t r = wread[w];
  const uint64_t first = offs[r] + 32 * (w - woff[r]), end = offs[r + 1];
  const int cnt = (int)min<uint64_t>(32, end - first);
  const uint32_t boff = (uint32_t)(first - a0);
  uint64_t v = 0;
  uint32_t nb = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {                        // four bases per step, no branches
    const uint32_t bo = boff + 4 * q, sh = (bo & 3) * 8;
    const uint32_t lo = buf[pad(bo >> 2)], hi = buf[pad((bo >> 2) + 1)];
    const uint32_t d = sh ? (lo >> sh) | (hi << (32 - sh)) : lo;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int idx = 4 * q + t;
      const uint32_t ch = (d >> (8 * t)) & 0xffu, lc = ch | 0x20u;
      const uint32_t x = (ch >> 1) & 3u;                 // A 0, C 1, G 3, T 2 (either case)
      uint32_t code = x ^ (x >> 1);                      // A 0, C 1, G 2, T 3
      const bool valid = lc == 'a' || lc == 'c' || lc == 'g' || lc == 't';
      code = (role == 1 && code == 1) ? 3u : code;       // read 1: C -> T
      code = (role == 2 && code == 2) ? 0u : code;       // read 2: G -> A
      const bool in = idx < cnt;
      v |= (uint64_t)((in && valid) ? code : 0u) << (2 * idx);
      nb |= ((in && !valid) ? 1u : 0u) << idx;
    }
  }
  pw[w] = v;
  pn[w] = nb;
}

// ---------------------------------------------------------------------------------------------
// wave-level work and output distribution.  Hot counters see one atomic per chunk (device-scope
// atomics on a single address serialise).  All 64 lanes of a wave call these together.
#define WORK_CHUNK 256   // largest work chunk; short queues use smaller ones (see chunk_for)
#define OUT_CHUNK 256

// Give each lane with `want` the next item of the wave's current chunk (grabbing new chunks as
// needed); returns the item or ~0 when the queue is exhausted.
__device__ __forceinline__ uint64_t wave_take(bool want, uint64_t &cb, uint64_t &ce, unsigned long long *counter,
                                              uint64_t total, int lane, uint32_t chunk = WORK_CHUNK) {
  uint64_t m = __ballot(want);
  uint64_t res = ~0ull;
  const uint64_t below = (1ull << lane) - 1;
  while (m) {
    if (cb >= ce) {
      unsigned long long b0 = 0;
      if (lane == 0) b0 = atomicAdd(counter, (unsigned long long)chunk);
      b0 = __shfl(b0, 0);
      if (b0 >= total) { cb = ce = total; break; }
      cb = b0;
      ce = b0 + chunk < total ? b0 + chunk : total;
    }
    const uint64_t avail = ce - cb;
    const uint32_t rank = __popcll(m & below);
    const bool mine = ((m >> lane) & 1) && rank < avail;
    if (mine) res = cb + rank;
    const uint64_t got = __ballot(mine);
    cb += __popcll(got);
    m &= ~got;
  }
  return res;
}

// Reserve one output slot for every lane with `em`, from the wave's current output chunk.
__device__ __forceinline__ uint64_t wave_slot(bool em, uint64_t &ob, uint64_t &oe, unsigned long long *counter, int lane) {
  uint64_t m = __ballot(em);
  uint64_t res = ~0ull;
  const uint64_t below = (1ull << lane) - 1;
  while (m) {
    if (ob >= oe) {
      unsigned long long b0 = 0;
      if (lane == 0) b0 = atomicAdd(counter, (unsigned long long)OUT_CHUNK);
      b0 = __shfl(b0, 0);
      ob = b0;
      oe = b0 + OUT_CHUNK;
    }
    const uint64_t avail = oe - ob;
    const uint32_t rank = __popcll(m & below);
    const bool mine = ((m >> lane) & 1) && rank < avail;
    if (mine) res = ob + rank;
    const uint64_t got = __ballot(mine);
    ob += __popcll(got);
    m &= ~got;
  }
  return res;
}

// s carries KNOWN_POS when the unique-match path found the match's text position (in the lane's
// text-position slot)
#define KNOWN_POS (1ull << 63)
struct Emit { uint32_t i, j; uint64_t k, kr, s; };
struct WaveOut { uint64_t sb, se, qb, qe; };

// this iteration's SMEMs (at most one per lane) and, in round 1, their re-seeding queries
__device__ __forceinline__ void wave_emit(const SeedParams &P, int lane, bool em, uint32_t read_id, const Emit &e, WaveOut &wo,
                                          uint32_t rlen, uint64_t woff, const uint64_t *pos) {
  if (!__ballot(em)) return;
  const uint64_t slot = wave_slot(em, wo.sb, wo.se, &P.ctl[C_NSEEDS], lane);
  if (em && slot < P.seed_cap) {
    SeedRec r;
    r.read_id = read_id; r.qbeg = e.i; r.qend = e.j; r.flags = P.round == 2 ? MBW_SEED_ROUND2 : 0u;
    r.k = e.k; r.kr = e.kr; r.s = e.s & ~KNOWN_POS; r.pos = (e.s & KNOWN_POS) ? *pos : NO_POS;
    P.seeds[slot] = r;
  }
  const uint64_t es = e.s & ~KNOWN_POS;
  const bool rq = em && P.round == 1 && P.reseed && (int)(e.j - e.i) >= P.reseed_len && es <= (uint64_t)P.reseed_occ;
  if (!__ballot(rq)) return;
  const uint64_t qs = wave_slot(rq, wo.qb, wo.qe, &P.ctl[C_NSUBQ], lane);
  if (rq && qs < P.subq_cap) {
    Query q;
    q.read_id = read_id; q.qbeg = e.i; q.qend = e.j; q.l = (e.j - e.i) / 2; q.c = (uint32_t)(es + 1);
    q.rlen = rlen; q.woff_lo = (uint32_t)woff; q.woff_hi = (uint32_t)(woff >> 32);
    q.send = e.j; q.flags = 0;
    P.subq[qs] = q;
  }
}

// mark the unused tail of the wave's output chunks invalid
__device__ __forceinline__ void wave_close(const SeedParams &P, int lane, const WaveOut &wo) {
  for (uint64_t t = wo.sb + lane; t < wo.se; t += 64)
    if (t < P.seed_cap) { SeedRec r; r.read_id = INVALID_READ; r.qbeg = r.qend = r.flags = 0; r.k = r.kr = r.s = 0; r.pos = NO_POS; P.seeds[t] = r; }
  for (uint64_t t = wo.qb + lane; t < wo.qe; t += 64)
    if (t < P.subq_cap) {
      Query q; q.read_id = INVALID_READ; q.qbeg = q.qend = q.l = q.rlen = q.woff_lo = q.woff_hi = q.send = q.flags = 0; q.c = 1;
      P.subq[t] = q;
    }
}

// Per-launch statistics: summed (or maximised) over the wave and added to the control block by
// lane 0, and only when not zero: same-address device-scope atomics serialise, and a persistent
// grid ends thousands of waves, most of them idle on a small batch, at about the same time.
__device__ __forceinline__ void wave_stat(unsigned long long *dst, uint64_t v, bool is_max = false) {
  unsigned long long x = v;
  for (int d = 32; d >= 1; d >>= 1) {
    const unsigned long long o = __shfl_xor(x, d);
    x = is_max ? (o > x ? o : x) : x + o;
  }
  if ((threadIdx.x & 63) == 0 && x) { if (is_max) atomicMax(dst, x); else atomicAdd(dst, x); }
}

// ---------------------------------------------------------------------------------------------
// SMEM kernel, wave schedule (Algorithm 3 per lane; persistent).
//
// Lane states: IDLE (takes a query), REC (the query's record is loaded in this iteration's memory
// phase), STAGE (the read's packed words are loaded; STAGED only), ACTIVE (one memory action per
// iteration: a k-mer table lookup or a backward/forward extension), DRAINED.  Stage changes that
// need no memory are taken before the memory phase.  In the memory phase every lane issues all of
// its loads (the three 16-byte slices of each index line a rank needs, a k-mer entry, a query
// record or the words of a read being staged) and the wave waits once.
//
// Unique matches.  When forward extension (stage 2) reaches an interval with s = 1, P[i, j) occurs
// at exactly one text position p, and P[i, j') occurs iff T[p, p + j' - i) = P[i, j'): the
// extension is finished by comparing read and text directly, which gives the same end j.  The
// interval of the result keeps k (the same single suffix) and s = 1; k' is the row of the suffix
// at the mirrored position m - p - (j - i) (T without $ is its own reverse complement), found from
// the nearest inverse-SA sample by LF steps.  Stages: 4 = LF walk from row k (in the staged
// kernel also from the reverse-complement row k', in step) until a sampled row is reached
// (Algorithm 2; the second walk gives the mirror of p), 5 = text comparison, 6 = inverse-SA sample
// read, 7 = LF walk to k'.  The seed carries p to locate, which does not walk it again.
//
// Deferred unique matches (DEFER; staged reads, round 1).  A wave runs the code of every state any
// of its lanes is in, so stages 4-7 in the same loop as the extensions make every iteration pay for
// them.  With DEFER the kernel runs the extension loop alone: a lane whose forward extension
// reaches s = 1 writes the match and its query to a task list and takes the next query; the
// continuation kernel (k_unique_wave) runs stages 4-7 for every task, reports the SMEM and lists
// the query for another pass of this kernel, which resumes it in stage 3 after the match.  Passes
// alternate until no query is left; the SMEMs are the same.
#define STAGE_WORDS 5   // staged reads of up to 160 bases
#define SOLO_STEPS 1024 // extension steps the tail loop takes in one iteration
#define SMEM_WAVES 4    // waves per block
enum { ACT_DONE = 0, ACT_KMER = 1, ACT_BWD = 2, ACT_FWD = 3, ACT_LF = 4, ACT_SSA = 5, ACT_TEXT = 6, ACT_ISA = 7, ACT_SKIP = 8 };
enum { ST_IDLE = 0, ST_REC = 1, ST_STAGE = 2, ST_ACTIVE = 3, ST_DRAINED = 4 };

// STAGED: reads staged in LDS (the short-read bin; never segmented).  UNIQ: the unique-match path
// is compiled in (round 1; in round 2 every interval has s >= c' >= 2).  Segment handling is
// compiled into the unstaged kernel only.
typedef __attribute__((address_space(3))) void lds_void;

// Records that arrive in the memory phase (query records, k-mer entries, staged read words) are
// loaded straight into LDS (global_load_lds: lane L's bytes land at base + size * L), so they
// occupy no registers while the wave waits.
template <bool STAGED, bool UNIQ, bool DEFER = false>
__global__ void __launch_bounds__(64 * SMEM_WAVES) __attribute__((amdgpu_waves_per_eu(4))) k_smem_wave(IndexView ix, SeedParams P, ReadWords R) {
  static_assert(!DEFER || (STAGED && !UNIQ), "deferred unique matches: staged kernel without the in-lane path");
  constexpr bool SEG = !STAGED;
  // the unique path's first walk follows both rows of the match in the staged kernel only: in the
  // unstaged one the second row's state made the compiler spill four times as many scalar
  // registers, which cost more than the shorter walk saves
  constexpr bool DUAL = STAGED;
  __shared__ uint32_t swl[SMEM_WAVES][STAGED ? STAGE_WORDS * 64 : 1];  // staged bases: low / high halves of
  __shared__ uint32_t swh[SMEM_WAVES][STAGED ? STAGE_WORDS * 64 : 1];  // word w of lane L at [64 w + L]
  __shared__ uint32_t sn[SMEM_WAVES][STAGED ? STAGE_WORDS * 64 : 1];   // staged N bits
  __shared__ uint4 sq[SMEM_WAVES][3][64];                              // query records (48 bytes)
  __shared__ uint4 sk[SMEM_WAVES][64];                                 // k-mer table entries
  __shared__ uint64_t sbt[MBW_MAX_SB * 8];
  __shared__ uint64_t scb[4];
  for (int t = threadIdx.x; t < 8 * ix.n_sb; t += blockDim.x) sbt[t] = ix.sbtab[t];
  if (threadIdx.x < 4) scb[threadIdx.x] = ix.Cb[threadIdx.x];
  __syncthreads();
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t sbm = (1u << ix.sb_shift) - 1;   // line index within its superblock
  uint32_t *mwl = swl[wv], *mwh = swh[wv];
  uint32_t *mn = sn[wv];
  const int K = (P.use_kmer && ix.kmer) ? ix.K : 0;
  int st = ST_IDLE;
  uint32_t qi = 0;                // queue index of the query being loaded (queues hold < 2^32 queries)
  uint64_t wo = 0;                // unstaged: first packed word of the read (the staged kernel reads it from LDS)
  uint32_t nw = 0;
  // cold fields of the current query, read from its record in LDS (written once per query)
  auto q_read_id = [&]() -> uint32_t { return sq[wv][0][lane].x; };
  auto q_rlen = [&]() -> uint32_t { return sq[wv][1][lane].y; };
  auto q_wo = [&]() -> uint64_t {
    if (!STAGED) return wo;
    const uint4 q1 = sq[wv][1][lane];
    return ((uint64_t)q1.w << 32) | q1.z;
  };
  auto word_at = [&](int w) -> uint64_t {
    return STAGED ? (((uint64_t)mwh[64 * w + lane] << 32) | mwl[64 * w + lane]) : R.pw[wo + w];
  };
  auto nbits_at = [&](int w) -> uint32_t { return STAGED ? mn[64 * w + lane] : R.pn[wo + w]; };
  auto base_at = [&](int p) -> int {
    const int w = p >> 5, b = p & 31;
    return ((nbits_at(w) >> b) & 1) ? 4 : (int)((word_at(w) >> (2 * b)) & 3);
  };
  const uint64_t tm = ix.n - 1;   // text length without $
  const uint64_t nq_total = P.nq_dev ? min(P.n_queries, (uint64_t)*P.nq_dev) : P.n_queries;
  uint32_t qbeg = 0, qend = 0, l = 0, c = 1, segend = 0;
  uint32_t segchk = 0;            // 1: the SMEM starting at qbeg still needs its left check (stage 8)
  int u = 0, i = 0, j = 0;
  uint64_t k = 0, kr = 0, s = 0;
  uint32_t budget = 0;            // iteration guard of the current query (a corrupt index cannot loop forever)
  uint64_t wrow = 0;              // unique path: walk row (or sample index)
  uint64_t wrow2 = 0;             // unique path, first walk: the row of the reverse-complement match
  // (wcnt's top bit: the occurrence was found by the reverse-complement walk)
  __shared__ uint64_t stp[SMEM_WAVES][64];   // unique path: text position of P[i] (rarely read: kept in LDS)
  uint64_t *tpl = &stp[wv][lane];
  uint32_t wcnt = 0;              // unique path: LF steps taken (stage 4) or still to take (stage 7)
  // this iteration's SMEM (at most one per lane) waits in LDS, in the parts of the lane's query
  // record that were copied to registers when it was loaded: k, k' in the third word, i, j and the
  // low half of s in the first (after the read id), the high half of s in the second
  bool em = false;
  auto put_emit = [&](int ei, int ej, uint64_t ek, uint64_t ekr, uint64_t es) {
    em = true;
    sq[wv][2][lane] = make_uint4((uint32_t)ek, (uint32_t)(ek >> 32), (uint32_t)ekr, (uint32_t)(ekr >> 32));
    sq[wv][0][lane].y = (uint32_t)ei;
    sq[wv][0][lane].z = (uint32_t)ej;
    sq[wv][0][lane].w = (uint32_t)es;
    sq[wv][1][lane].x = (uint32_t)(es >> 32);
  };
  constexpr uint32_t WMIR = 1u << 31;
  // 1: the interval is (0, 0, n) and the k-mer shortcut is still to try (an integer except in the
  // staged kernel with the unique-match path, where a lane mask measured faster)
  typename std::conditional<STAGED && UNIQ, bool, uint32_t>::type fresh = 0;
  uint32_t n_lines = 0, n_steps = 0, n_kmer = 0;   // per lane (well below 2^32 per launch)
  uint64_t n_iter = 0, n_busy = 0;                 // per wave
  uint32_t chain = 0, max_chain = 0;   // iterations of the current query; longest so far
  uint64_t cb = 0, ce = 0;
  WaveOut wout = {0, 0, 0, 0};
  uint64_t tkb = 0, tke = 0;      // DEFER: the wave's current chunk of the task list
  for (;;) {
    // ---- idle lanes take a query (its record is loaded in this iteration's memory phase)
    const bool want = st == ST_IDLE;
    if (__ballot(want)) {
      const uint64_t t = wave_take(want, cb, ce, &P.ctl[C_WORK], nq_total, lane, P.chunk);
      if (want) { if (t == ~0ull) st = ST_DRAINED; else { qi = (uint32_t)t; st = ST_REC; } }
    }
    if (__ballot(st != ST_DRAINED) == 0) break;
    ++n_iter;
    n_busy += __popcll(__ballot(st != ST_DRAINED && st != ST_IDLE));
    if (st == ST_REC) chain = 0;
    if (st != ST_DRAINED && st != ST_IDLE) { ++chain; max_chain = chain > max_chain ? chain : max_chain; }
    // ---- active lanes: stage transitions up to the next memory action
    int act = ACT_DONE, a = 0;
    uint32_t code = 0;
    em = false;
    bool dfr = false;             // DEFER: the match reached s = 1; it goes to the task list
    if (st == ST_ACTIVE && --budget == 0) { atomicOr(&P.ctl[C_ERR], 1ull); st = ST_IDLE; }
    if (st == ST_ACTIVE) {
      for (;;) {
        if ((UNIQ || SEG) && u >= 4) {                  // unique path (4-7), segment left check (8)
          if (UNIQ && u == 4) {   // walk both rows of the match until one reaches a sampled row
            const bool s1 = (wrow & P.rmask) == 0, s2 = DUAL && (wrow2 & P.rmask) == 0;
            if (s1 || s2) { if (!s1) { wrow = wrow2; wcnt |= WMIR; } act = ACT_SSA; break; }
            if (!DUAL && wrow == ix.primary) { wrow = 0; ++wcnt; continue; }   // LF of the $ row is row 0
            act = ACT_LF; break;
          }
          if (UNIQ && u == 5) { act = ACT_TEXT; break; }
          if (UNIQ && u == 6) { act = ACT_ISA; break; }
          if (UNIQ && u == 7) {
            if (wcnt > 0) { act = ACT_LF; break; }
            if (SEG && segchk != 0 && i == (int)qbeg) { segchk = 0; kr = wrow; s = 1; u = 8; continue; }
            put_emit(i, j, k, wrow, 1 | KNOWN_POS);
            if (j == (int)qend) { act = ACT_DONE; break; }
            u = 3; k = 0; kr = 0; s = ix.n; fresh = 1;
            continue;
          }
          // u == 8: left check of a segment's first SMEM [qbeg, j) with interval (k, kr, s)
          a = base_at(i - 1);
          if (a <= 3) { act = ACT_BWD; break; }
          put_emit(i, j, k, kr, s);   // P[i-1] matches nothing
          if (j == (int)qend) { act = ACT_DONE; break; }
          u = 3; k = 0; kr = 0; s = ix.n; fresh = 1;
          continue;
        }
        if (u == 2) {
          const bool qe = j == (int)qend;
          a = qe ? 4 : base_at(j);
          if (UNIQ && !qe && P.uniq && s == 1) { u = 4; wrow = k; wrow2 = kr; wcnt = 0; continue; }
          if (DEFER && !qe && s == 1) { dfr = true; act = ACT_DONE; break; }
          if (a > 3) {                                  // end of the query, or a non-ACGT base: SMEM [i, j)
            if (SEG && segchk != 0 && i == (int)qbeg) { segchk = 0; u = 8; continue; }
            put_emit(i, j, k, kr, s);
            if (qe) { act = ACT_DONE; break; }
            u = 3; k = 0; kr = 0; s = ix.n; fresh = 1;
            continue;
          }
          act = ACT_FWD; break;
        }
        if (u == 1 && j < i) { u = 2; j = i + (int)l; fresh = 0; continue; }
        if (u == 3 && j <= i) {
          if (SEG && j + 1 >= (int)segend) { act = ACT_DONE; break; }   // the next start belongs to the next segment
          u = 1; i = j + 1; j = j + (int)l; k = 0; kr = 0; s = ix.n; fresh = 1; continue;
        }
        if (fresh != 0 && K > 0 && j - K + 1 >= (u == 1 ? i : i + 1)) {
          // k-mer P[j-K+1 .. j] from the packed read: its code is the bit field 2(j-K+1) .. 2(j+1)
          const int a0 = j - K + 1, w = a0 >> 5, b0 = a0 & 31;
          uint64_t bits = word_at(w) >> (2 * b0);
          uint32_t nbits = nbits_at(w) >> b0;
          if (b0 + K > 32) { bits |= word_at(w + 1) << (64 - 2 * b0); nbits |= nbits_at(w + 1) << (32 - b0); }
          fresh = 0;
          if ((nbits & ((1u << K) - 1)) == 0) { code = (uint32_t)(bits & ((1ull << (2 * K)) - 1)); act = ACT_KMER; break; }
        }
        fresh = 0;
        a = base_at(j);
        if (a > 3) {                                    // BackStep fails on a non-ACGT base
          if (j + (int)l < (int)qend && (!SEG || j + 1 < (int)segend)) {
            u = 1; i = j + 1; j = j + (int)l; k = 0; kr = 0; s = ix.n; fresh = 1; continue;
          }
          act = ACT_DONE; break;
        }
        act = ACT_BWD; break;
      }
      if (act == ACT_DONE) st = ST_IDLE;
    }
    const bool selig = (act == ACT_BWD && (u == 1 || u == 3)) || (act == ACT_FWD && u == 2);
    const uint64_t sbusy = __ballot(st != ST_DRAINED);
    if (sbusy != 0 && __ballot(selig) == sbusy) {
      // Every lane of the wave that still has work is extending (backward in stages 1 and 3,
      // forward in stage 2), and none takes a query, stages a read or loads a record: their
      // extension steps run back to back here, without the rest of the iteration (the same steps
      // in the same order), until the first lane stops: a failing step, a non-ACGT base, the end of
      // the stage and a unique match (s = 1, for the unique-match path) are left to the next
      // iteration, as is a step beyond SOLO_STEPS or the lane's work budget.  This happens mid-launch
      // whenever all 64 lanes extend at once, and always at the end of a launch, where the queue is
      // exhausted and a few long queries are left.  Each step counts against the query's budget and
      // its chain length like an iteration.
      const bool sbwd = act == ACT_BWD;
      bool go = selig;
      for (int t = 0; t < SOLO_STEPS; ++t) {
        if (go && budget <= 1) go = false;             // the guard of the main loop decides
        if (go) {
          const int sc = sbwd ? a : 3 - a;
          const uint64_t sx1 = sbwd ? k : kr, sx2 = sx1 + s, sy = sbwd ? kr : k;
          const uint32_t sL1 = line_of(sx1), sL2 = line_of(sx2);
          const int so1 = (int)(sx1 - (uint64_t)sL1 * MBW_BPL), so2 = (int)(sx2 - (uint64_t)sL2 * MBW_BPL);
          const uint4 *p1 = ix.lines + (uint64_t)sL1 * MBW_LINE_U4, *p2 = ix.lines + (uint64_t)sL2 * MBW_LINE_U4;
          const bool stwo = sL1 != sL2, sblk2 = stwo || (so1 >> 6) != (so2 >> 6);
          const uint4 g0 = p1[0], g1 = p1[1], gb = p1[2 + (so1 >> 6)];
          const uint4 q0 = stwo ? p2[0] : g0, q1 = stwo ? p2[1] : g1, qb = sblk2 ? p2[2 + (so2 >> 6)] : gb;
          const SymMasks ssm = sym_masks(sc);
          const uint32_t sb1 = 8 * (sL1 >> ix.sb_shift), sb2 = 8 * (sL2 >> ix.sb_shift);
          uint64_t E1, G1, E2, G2, nx, ny, ns;
          rank_eg(g0, g1, gb, sL1 & sbm, so1, sc, ssm, sbt[sb1 + sc], sbt[sb1 + 4 + sc], E1, G1);
          rank_eg(q0, q1, qb, sL2 & sbm, so2, sc, ssm, sbt[sb2 + sc], sbt[sb2 + 4 + sc], E2, G2);
          ext_update(E1, G1, E2, G2, sc, sx1, s, sy, ix.primary, scb[sc], nx, ny, ns);
          if (ns < c) go = false;
          else {
            n_lines += stwo ? 2 : 1;
            ++n_steps;
            --budget;
            ++chain;
            if (sbwd) { k = nx; kr = ny; j -= 1; }
            else { kr = nx; k = ny; j += 1; }
            s = ns;
            act = ACT_SKIP;
            if (sbwd ? ((u == 1 && j < i) || (u == 3 && j <= i)) : (j == (int)qend || (((UNIQ && P.uniq) || DEFER) && s == 1))) go = false;
            else {
              a = base_at(j);
              if (a > 3) go = false;
            }
          }
        }
        if (__ballot(selig && !go)) break;
      }
      max_chain = chain > max_chain ? chain : max_chain;
    }
    const bool ext = act == ACT_BWD || act == ACT_FWD;
    const bool bwd = act == ACT_BWD;
    const bool lfa = UNIQ && act == ACT_LF;
    const bool lf1 = lfa && u == 4;                      // first walk
    const bool lf2 = DUAL && lf1;                        // ... LF of both rows of the match
    const uint64_t x1 = lfa ? wrow : (bwd ? k : kr), y = bwd ? kr : k;
    const int cc = bwd ? a : 3 - a;
    const uint64_t x2 = lf2 ? wrow2 : x1 + (lfa ? 0ull : s);   // a single LF step ranks one row
    const uint32_t L1 = line_of(x1), L2 = line_of(x2);
    const int o1 = (int)(x1 - (uint64_t)L1 * MBW_BPL), o2 = (int)(x2 - (uint64_t)L2 * MBW_BPL);
    const bool two = (ext || lf2) && L1 != L2;                          // a second index line
    const bool blk2 = (ext || lf2) && (two || (o1 >> 6) != (o2 >> 6));  // a second block slice
    // ---- the memory phase: everything the lane needs, issued together, waited for once
    const uint4 z4 = make_uint4(0, 0, 0, 0);
    const uint4 *l1p = ix.lines + (uint64_t)L1 * MBW_LINE_U4, *l2p = ix.lines + (uint64_t)L2 * MBW_LINE_U4;
    uint4 h0a = z4, h1a = z4, ba = z4, h0b = z4, h1b = z4, bb = z4;
    if (ext || lfa) { h0a = l1p[0]; h1a = l1p[1]; ba = l1p[2 + (o1 >> 6)]; }
    if (two) { h0b = l2p[0]; h1b = l2p[1]; }
    if (blk2) bb = l2p[2 + (o2 >> 6)];
    // unique path: a sampled SA / inverse-SA value, or 32 bytes of text around position tq
    const uint64_t tq = (UNIQ && act == ACT_TEXT ? *tpl : 0ull) + (uint64_t)(j - i);
    const bool txt = UNIQ && act == ACT_TEXT && tq < tm;
    if (txt) {
      const uint4 *tw = (const uint4 *)(ix.text + ((tq >> 5) & ~1ull));
      h0b = tw[0]; h1b = tw[1];
    }
    uint64_t mval = 0;
    if (UNIQ && act == ACT_SSA) mval = ix.ssa[wrow >> P.rshift];
    if (UNIQ && act == ACT_ISA) mval = ix.isa[wrow];
    if (act == ACT_KMER) __builtin_amdgcn_global_load_lds((const void *)(ix.kmer + code), (lds_void *)sk[wv], 16, 0, 0);
    const int st_mem = st;
    if (st_mem == ST_REC) {
      const uint4 *qp = (const uint4 *)(P.queries + qi);
      __builtin_amdgcn_global_load_lds((const void *)qp, (lds_void *)sq[wv][0], 16, 0, 0);
      __builtin_amdgcn_global_load_lds((const void *)(qp + 1), (lds_void *)sq[wv][1], 16, 0, 0);
      __builtin_amdgcn_global_load_lds((const void *)(qp + 2), (lds_void *)sq[wv][2], 16, 0, 0);
    }
    if (STAGED && st_mem == ST_STAGE) {
#pragma unroll
      for (int w = 0; w < STAGE_WORDS; ++w)
        if ((uint32_t)w < nw) {
          const uint32_t *wp = (const uint32_t *)(R.pw + q_wo() + w);
          __builtin_amdgcn_global_load_lds((const void *)wp, (lds_void *)(mwl + 64 * w), 4, 0, 0);
          __builtin_amdgcn_global_load_lds((const void *)(wp + 1), (lds_void *)(mwh + 64 * w), 4, 0, 0);
          __builtin_amdgcn_global_load_lds((const void *)(R.pn + q_wo() + w), (lds_void *)(mn + 64 * w), 4, 0, 0);
        }
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    // ---- compute
    if (act == ACT_KMER) {
      uint64_t ek, ekr, es;
      kmer_unpack(sk[wv][lane], ek, ekr, es);
      ++n_kmer;
      if (es >= c) { k = ek; kr = ekr; s = es; j -= K; }
    }
    if (ext || lfa) {
      // an LF step (unique path) is the first rank of an extension by its own row's symbol
      const int cx = lfa ? bwt_from_block(ba, o1) : cc;
      if (!two) { h0b = h0a; h1b = h1a; }
      if (!blk2) bb = ba;
      const int cx2 = lf2 ? bwt_from_block(bb, o2) : cx;   // the second walk ranks its own row's symbol
      const SymMasks sm = sym_masks(cx), sm2 = sym_masks(cx2);
      const uint32_t sb1 = 8 * (L1 >> ix.sb_shift), sb2 = 8 * (L2 >> ix.sb_shift);
      uint64_t E1, G1, E2, G2;
      rank_eg(h0a, h1a, ba, L1 & sbm, o1, cx, sm, sbt[sb1 + cx], sbt[sb1 + 4 + cx], E1, G1);
      rank_eg(h0b, h1b, bb, L2 & sbm, o2, cx2, sm2, sbt[sb2 + cx2], sbt[sb2 + 4 + cx2], E2, G2);
      uint64_t nx, ny, ns;
      ext_update(E1, G1, E2, G2, cx, x1, lfa ? 0ull : s, y, ix.primary, scb[cx], nx, ny, ns);
      if (lf2) {                                          // LF of both rows; the $ row maps to row 0
        wrow = x1 == ix.primary ? 0ull : nx;
        wrow2 = x2 == ix.primary ? 0ull : scb[cx2] + E2 - ((cx2 == 0 && x2 > ix.primary) ? 1ull : 0ull);
        ++wcnt;
        n_lines += two ? 2 : 1;
      } else if (lfa) {                                   // single-row walk (the second never meets the $ row)
        wrow = nx;
        if (lf1) ++wcnt; else --wcnt;
        ++n_lines;
      } else {
        n_lines += two ? 2 : 1;
        ++n_steps;
        if (SEG && u == 8) {                              // left check: report unless P[i-1, j) occurs c times
          if (ns < c) put_emit(i, j, k, kr, s);
          if (j == (int)qend) st = ST_IDLE;
          else { u = 3; k = 0; kr = 0; s = ix.n; fresh = 1; }
        } else if (ns >= c) {
          if (bwd) { k = nx; kr = ny; s = ns; j -= 1; }
          else { kr = nx; k = ny; s = ns; j += 1; }
        } else if (bwd) {                                 // BackStep failure: jump past j
          if (j + (int)l < (int)qend && (!SEG || j + 1 < (int)segend)) { u = 1; i = j + 1; j = j + (int)l; k = 0; kr = 0; s = ix.n; fresh = 1; }
          else st = ST_IDLE;
        } else if (SEG && segchk != 0 && i == (int)qbeg) {   // forward failure at a segment's first SMEM
          segchk = 0; u = 8;
        } else {                                          // forward failure: report, then stage 3 from j
          put_emit(i, j, k, kr, s);
          u = 3; k = 0; kr = 0; s = ix.n; fresh = 1;
        }
      }
    }
    if (UNIQ && act == ACT_SSA) {                       // the occurrence: p = S(row) + steps (mod n)
      uint64_t pp = mval + (wcnt & ~WMIR);
      if (pp >= ix.n) pp -= ix.n;
      if (DUAL && (wcnt & WMIR)) pp = tm - pp - (uint64_t)(j - i);   // the mirror of the reverse-complement match
      *tpl = pp;
      u = 5;
      ++n_lines;
    }
    if (UNIQ && act == ACT_TEXT) {                      // compare up to 64 bases of read and text
      const int lim0 = min(64, (int)qend - j);
      int first = 0;
      if (txt) {
        const uint64_t wv0 = ((uint64_t)h0b.y << 32) | h0b.x, wv1 = ((uint64_t)h0b.w << 32) | h0b.z;
        const uint64_t wv2 = ((uint64_t)h1b.y << 32) | h1b.x, wv3 = ((uint64_t)h1b.w << 32) | h1b.z;
        const int off = 2 * (int)(tq - 32 * ((tq >> 5) & ~1ull));   // bit offset of tq in the window, 0..126
        const int sh = off & 63;
        const uint64_t lo = off < 64 ? wv0 : wv1, mid = off < 64 ? wv1 : wv2, hi = off < 64 ? wv2 : wv3;
        const uint64_t t0 = sh ? (lo >> sh) | (mid << (64 - sh)) : lo;
        const uint64_t t1 = sh ? (mid >> sh) | (hi << (64 - sh)) : mid;
        // read bases j .. j+63: words past the read's end hold stale bases, which the limit
        // qend - j cuts off (staged: indexes clamped into the lane's LDS area; unstaged: the packed
        // batch ends with two spare words)
        const int w0 = j >> 5, rb = j & 31;
        const int w1 = STAGED ? min(w0 + 1, STAGE_WORDS - 1) : w0 + 1;
        const int w2 = STAGED ? min(w0 + 2, STAGE_WORDS - 1) : w0 + 2;
        const uint64_t a0 = word_at(w0), a1 = word_at(w1), a2 = word_at(w2);
        const uint32_t n0 = nbits_at(w0), n1 = nbits_at(w1), n2 = nbits_at(w2);
        const uint64_t r0 = rb ? (a0 >> (2 * rb)) | (a1 << (64 - 2 * rb)) : a0;
        const uint64_t r1 = rb ? (a1 >> (2 * rb)) | (a2 << (64 - 2 * rb)) : a1;
        const uint64_t nb = (((uint64_t)n2 << 32 | n1) << (32 - rb)) | ((uint64_t)n0 >> rb);
        const uint64_t d0 = r0 ^ t0, d1 = r1 ^ t1;
        const uint64_t f0 = (d0 | (d0 >> 1)) & 0x5555555555555555ull, f1 = (d1 | (d1 >> 1)) & 0x5555555555555555ull;
        const int mm = f0 ? (__ffsll((long long)f0) - 1) >> 1 : (f1 ? 32 + ((__ffsll((long long)f1) - 1) >> 1) : 64);
        const int nf = nb ? __ffsll((long long)nb) - 1 : 64;
        const uint64_t left = tm - tq;                  // text symbols before the $
        first = min(min(mm, nf), min(lim0, left < 64 ? (int)left : 64));
        n_lines += ((((tq >> 5) & ~1ull) & 15) == 14) ? 2 : 1;
      }
      j += first;
      if (first == 64 && j < (int)qend) {
        // the whole window matched: continue with the next one
      } else {                                          // end of the match: k' from the mirror position
        const uint64_t pm = tm - *tpl - (uint64_t)(j - i);
        const uint64_t q = ((pm >> P.rishift) + ((pm & ((1ull << P.rishift) - 1)) ? 1 : 0)) << P.rishift;
        if (q >= tm) { wrow = 0; wcnt = (uint32_t)(tm - pm); u = 7; }   // row 0 holds the suffix at tm ($)
        else { wrow = q >> P.rishift; wcnt = (uint32_t)(q - pm); u = 6; }
      }
    }
    if (UNIQ && act == ACT_ISA) { wrow = mval; u = 7; ++n_lines; }
    if (st_mem == ST_REC) {
      const uint4 q0 = sq[wv][0][lane], q1 = sq[wv][1][lane], q2 = sq[wv][2][lane];
      const uint32_t read_id = q0.x, rlen = q1.y;
      qbeg = q0.y; qend = q0.z; l = q0.w; c = q1.x;
      if (!STAGED) wo = ((uint64_t)q1.w << 32) | q1.z;
      segend = q2.x; segchk = (SEG && (q2.y & SEG_CHECK) != 0) ? 1u : 0u;
      nw = (rlen + 31) >> 5;
      // Algorithm 3 queues a string only if l - 1 < |P|
      const bool work = read_id != INVALID_READ && l >= 1 && l - 1 < qend - qbeg && (!STAGED || nw <= STAGE_WORDS);
      st = !work ? ST_IDLE : (STAGED ? ST_STAGE : ST_ACTIVE);
    }
    if ((STAGED && st_mem == ST_STAGE) || (!STAGED && st_mem == ST_REC && st == ST_ACTIVE)) {
      u = 1; i = (int)qbeg; j = (int)(qbeg + l - 1);
      k = 0; kr = 0; s = ix.n; fresh = 1;
      if (DEFER) {                                      // a query resumed after its unique match
        const uint4 q2 = sq[wv][2][lane];
        if (q2.y & Q_RESUME) { u = 3; i = (int)q2.z; j = (int)q2.w; }
      }
      {
        const uint64_t b = 8ull * (qend - qbeg) * (qend - qbeg) + 64;
        budget = b > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)b;
      }
      st = ST_ACTIVE;
    }
    {
      Emit e = {0, 0, 0, 0, 0};
      if (em) {
        const uint4 r0 = sq[wv][0][lane], r2 = sq[wv][2][lane];
        e.i = r0.y; e.j = r0.z; e.s = ((uint64_t)sq[wv][1][lane].x << 32) | r0.w;
        e.k = ((uint64_t)r2.y << 32) | r2.x; e.kr = ((uint64_t)r2.w << 32) | r2.z;
      }
      wave_emit(P, lane, em, q_read_id(), e, wout, q_rlen(), q_wo(), tpl);
    }
    if (DEFER && __ballot(dfr)) {                       // its read id, length and word offset are still in LDS
      const uint64_t ts = wave_slot(dfr, tkb, tke, &P.ctl[C_PASSQ], lane);
      if (dfr && ts < P.task_cap) {
        const uint4 q0 = sq[wv][0][lane], q1 = sq[wv][1][lane];
        UTask t;
        t.read_id = q0.x; t.qbeg = qbeg; t.qend = qend; t.l = l;
        t.c = c; t.rlen = q1.y; t.woff_lo = q1.z; t.woff_hi = q1.w;
        t.i = (uint32_t)i; t.j = (uint32_t)j; t.pad0 = 0; t.pad1 = 0; t.k = k; t.kr = kr;
        P.tasks[ts] = t;
      }
    }
  }
  wave_close(P, lane, wout);
  if (DEFER)                                            // the unused tail of the wave's task chunk
    for (uint64_t t = tkb + lane; t < tke; t += 64)
      if (t < P.task_cap) P.tasks[t].read_id = INVALID_READ;
  // n_iter and n_busy are per wave (the same in every lane); the rest are per lane
  if ((threadIdx.x & 63) == 0 && n_iter) { atomicAdd(&P.ctl[C_WITER], (unsigned long long)n_iter); atomicAdd(&P.ctl[C_LITER], (unsigned long long)n_busy); }
  wave_stat(&P.ctl[C_MAXCHAIN], max_chain, true);
  wave_stat(&P.ctl[C_LINES], (uint64_t)n_lines + n_kmer);
  wave_stat(&P.ctl[C_STEPS], n_steps);
  wave_stat(&P.ctl[C_KMER], n_kmer);
}

// ---------------------------------------------------------------------------------------------
// Continuation kernel of deferred unique matches (persistent; one task per lane at a time).
//
// A task is a match P[i, j) with s = 1 found by forward extension.  Its lane walks LF from both
// rows of the match (k and the reverse-complement row kr) until one reaches a sampled SA row
// (stage 4), reads that sample (5: the occurrence p, or its mirror from the second walk), compares
// the read with the packed text 64 bases at a time from P[j] on (6), reads the inverse-SA sample at
// or after the mirrored position of the extended match and walks LF to it (7: k'), then reports the
// SMEM [i, j') with (k, k', 1) and its position, and lists the query for the next pass of the SMEM
// kernel unless j' is the query's end.  The read's packed words come from global memory.
#define UNIQ_WAVES 4
#define AUTO_TASKS 4000   // automatic grid sizing: tasks per block and CU

__global__ void __launch_bounds__(64 * UNIQ_WAVES) k_unique_wave(IndexView ix, SeedParams P, ReadWords R) {
  __shared__ uint64_t sbt[MBW_MAX_SB * 8];
  __shared__ uint64_t scb[4];
  __shared__ uint64_t stp[UNIQ_WAVES][64];   // text position of P[i] (read when a seed is written)
  for (int t = threadIdx.x; t < 8 * ix.n_sb; t += blockDim.x) sbt[t] = ix.sbtab[t];
  if (threadIdx.x < 4) scb[threadIdx.x] = ix.Cb[threadIdx.x];
  __syncthreads();
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t sbm = (1u << ix.sb_shift) - 1;
  const uint64_t tm = ix.n - 1;   // text length without $
  uint64_t *tpl = &stp[wv][lane];
  int st = ST_IDLE;
  uint32_t ti = 0;                // task being loaded
  uint32_t read_id = 0, qbeg = 0, qend = 0, l = 0, c = 1, rlen = 0;
  uint64_t wo = 0;                // first packed word of the read
  int i = 0, j = 0, u = 0;
  uint64_t k = 0, wrow = 0, wrow2 = 0;
  bool wmir = false;
  uint32_t wcnt = 0, budget = 0;
  uint32_t n_lines = 0;
  uint64_t n_iter = 0, n_busy = 0;
  uint64_t cb = 0, ce = 0, rb = 0, re = 0;
  WaveOut wout = {0, 0, 0, 0};
  for (;;) {
    const bool want = st == ST_IDLE;
    if (__ballot(want)) {
      const uint64_t t = wave_take(want, cb, ce, &P.ctl[C_WORK], P.n_queries, lane, P.chunk);
      if (want) { if (t == ~0ull) st = ST_DRAINED; else { ti = (uint32_t)t; st = ST_REC; } }
    }
    if (__ballot(st != ST_DRAINED) == 0) break;
    ++n_iter;
    n_busy += __popcll(__ballot(st != ST_DRAINED && st != ST_IDLE));
    int act = ACT_DONE;
    bool em = false, rs = false;
    Emit e;
    e.i = 0; e.j = 0; e.k = 0; e.kr = 0; e.s = 0;
    if (st == ST_ACTIVE && --budget == 0) { atomicOr(&P.ctl[C_ERR], 1ull); st = ST_IDLE; }
    if (st == ST_ACTIVE) {
      if (u == 4) {
        const bool s1 = (wrow & P.rmask) == 0, s2 = (wrow2 & P.rmask) == 0;
        if (s1 || s2) { wmir = !s1; if (!s1) wrow = wrow2; act = ACT_SSA; }
        else act = ACT_LF;
      } else if (u == 5) act = ACT_TEXT;
      else if (u == 6) act = ACT_ISA;
      else if (wcnt > 0) act = ACT_LF;
      else {                                            // u == 7, at k': the SMEM [i, j) with (k, k', 1)
        em = true; e.i = (uint32_t)i; e.j = (uint32_t)j; e.k = k; e.kr = wrow; e.s = 1 | KNOWN_POS;
        rs = j != (int)qend;
        st = ST_IDLE;
      }
    }
    const bool lfa = act == ACT_LF;
    const bool lf2 = lfa && u == 4;                      // both rows of the match
    const uint64_t x1 = wrow, x2 = lf2 ? wrow2 : wrow;
    const uint32_t L1 = line_of(x1), L2 = line_of(x2);
    const int o1 = (int)(x1 - (uint64_t)L1 * MBW_BPL), o2 = (int)(x2 - (uint64_t)L2 * MBW_BPL);
    const bool two = lf2 && L1 != L2;
    const bool blk2 = lf2 && (two || (o1 >> 6) != (o2 >> 6));
    // ---- the memory phase
    const uint4 z4 = make_uint4(0, 0, 0, 0);
    const uint4 *l1p = ix.lines + (uint64_t)L1 * MBW_LINE_U4, *l2p = ix.lines + (uint64_t)L2 * MBW_LINE_U4;
    uint4 h0a = z4, h1a = z4, ba = z4, h0b = z4, h1b = z4, bb = z4;
    if (lfa) { h0a = l1p[0]; h1a = l1p[1]; ba = l1p[2 + (o1 >> 6)]; }
    if (two) { h0b = l2p[0]; h1b = l2p[1]; }
    if (blk2) bb = l2p[2 + (o2 >> 6)];
    const uint64_t tq = (act == ACT_TEXT ? *tpl : 0ull) + (uint64_t)(j - i);
    const bool txt = act == ACT_TEXT && tq < tm;
    uint64_t a0 = 0, a1 = 0, a2 = 0;
    uint32_t n0 = 0, n1 = 0, n2 = 0;
    if (txt) {
      const uint4 *tw = (const uint4 *)(ix.text + ((tq >> 5) & ~1ull));
      h0b = tw[0]; h1b = tw[1];
      // read bases j .. j+63 (the packed batch ends with two spare words)
      const uint64_t w0 = wo + (uint64_t)(j >> 5);
      a0 = R.pw[w0]; a1 = R.pw[w0 + 1]; a2 = R.pw[w0 + 2];
      n0 = R.pn[w0]; n1 = R.pn[w0 + 1]; n2 = R.pn[w0 + 2];
    }
    uint64_t mval = 0;
    if (act == ACT_SSA) mval = ix.ssa[wrow >> P.rshift];
    if (act == ACT_ISA) mval = ix.isa[wrow];
    const int st_mem = st;
    uint4 t0 = z4, t1 = z4, t2 = z4, t3 = z4;
    if (st_mem == ST_REC) {
      const uint4 *tp = (const uint4 *)(P.tasks + ti);
      t0 = tp[0]; t1 = tp[1]; t2 = tp[2]; t3 = tp[3];
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    // ---- compute
    if (lfa) {                                          // LF of the walked row(s); the $ row maps to row 0
      const int cx = bwt_from_block(ba, o1);
      if (!two) { h0b = h0a; h1b = h1a; }
      if (!blk2) bb = ba;
      const uint32_t sb1 = 8 * (L1 >> ix.sb_shift);
      uint64_t E1, G1;
      rank_eg(h0a, h1a, ba, L1 & sbm, o1, cx, sym_masks(cx), sbt[sb1 + cx], sbt[sb1 + 4 + cx], E1, G1);
      wrow = x1 == ix.primary ? 0ull : scb[cx] + E1 - ((cx == 0 && x1 > ix.primary) ? 1ull : 0ull);
      if (lf2) {
        const int cx2 = bwt_from_block(bb, o2);
        const uint32_t sb2 = 8 * (L2 >> ix.sb_shift);
        uint64_t E2, G2;
        rank_eg(h0b, h1b, bb, L2 & sbm, o2, cx2, sym_masks(cx2), sbt[sb2 + cx2], sbt[sb2 + 4 + cx2], E2, G2);
        wrow2 = x2 == ix.primary ? 0ull : scb[cx2] + E2 - ((cx2 == 0 && x2 > ix.primary) ? 1ull : 0ull);
        ++wcnt;
        n_lines += two ? 2 : 1;
      } else {
        --wcnt;
        ++n_lines;
      }
    }
    if (act == ACT_SSA) {                               // the occurrence: p = S(row) + steps (mod n)
      uint64_t pp = mval + wcnt;
      if (pp >= ix.n) pp -= ix.n;
      if (wmir) pp = tm - pp - (uint64_t)(j - i);       // the mirror of the reverse-complement match
      *tpl = pp;
      u = 5;
      ++n_lines;
    }
    if (act == ACT_TEXT) {                              // compare up to 64 bases of read and text
      const int lim0 = min(64, (int)qend - j);
      int first = 0;
      if (txt) {
        const uint64_t wv0 = ((uint64_t)h0b.y << 32) | h0b.x, wv1 = ((uint64_t)h0b.w << 32) | h0b.z;
        const uint64_t wv2 = ((uint64_t)h1b.y << 32) | h1b.x, wv3 = ((uint64_t)h1b.w << 32) | h1b.z;
        const int off = 2 * (int)(tq - 32 * ((tq >> 5) & ~1ull));   // bit offset of tq in the window, 0..126
        const int sh = off & 63;
        const uint64_t lo = off < 64 ? wv0 : wv1, mid = off < 64 ? wv1 : wv2, hi = off < 64 ? wv2 : wv3;
        const uint64_t tt0 = sh ? (lo >> sh) | (mid << (64 - sh)) : lo;
        const uint64_t tt1 = sh ? (mid >> sh) | (hi << (64 - sh)) : mid;
        const int rb2 = j & 31;
        const uint64_t r0 = rb2 ? (a0 >> (2 * rb2)) | (a1 << (64 - 2 * rb2)) : a0;
        const uint64_t r1 = rb2 ? (a1 >> (2 * rb2)) | (a2 << (64 - 2 * rb2)) : a1;
        const uint64_t nb = (((uint64_t)n2 << 32 | n1) << (32 - rb2)) | ((uint64_t)n0 >> rb2);
        const uint64_t d0 = r0 ^ tt0, d1 = r1 ^ tt1;
        const uint64_t f0 = (d0 | (d0 >> 1)) & 0x5555555555555555ull, f1 = (d1 | (d1 >> 1)) & 0x5555555555555555ull;
        const int mm = f0 ? (__ffsll((long long)f0) - 1) >> 1 : (f1 ? 32 + ((__ffsll((long long)f1) - 1) >> 1) : 64);
        const int nf = nb ? __ffsll((long long)nb) - 1 : 64;
        const uint64_t left = tm - tq;                  // text symbols before the $
        first = min(min(mm, nf), min(lim0, left < 64 ? (int)left : 64));
        n_lines += ((((tq >> 5) & ~1ull) & 15) == 14) ? 2 : 1;
      }
      j += first;
      if (!(first == 64 && j < (int)qend)) {            // end of the match: k' from the mirror position
        const uint64_t pm = tm - *tpl - (uint64_t)(j - i);
        const uint64_t q = ((pm >> P.rishift) + ((pm & ((1ull << P.rishift) - 1)) ? 1 : 0)) << P.rishift;
        if (q >= tm) { wrow = 0; wcnt = (uint32_t)(tm - pm); u = 7; }   // row 0 holds the suffix at tm ($)
        else { wrow = q >> P.rishift; wcnt = (uint32_t)(q - pm); u = 6; }
      }
    }
    if (act == ACT_ISA) { wrow = mval; u = 7; ++n_lines; }
    if (st_mem == ST_REC) {
      read_id = t0.x; qbeg = t0.y; qend = t0.z; l = t0.w;
      c = t1.x; rlen = t1.y; wo = ((uint64_t)t1.w << 32) | t1.z;
      i = (int)t2.x; j = (int)t2.y;
      k = ((uint64_t)t3.y << 32) | t3.x;
      wrow = k; wrow2 = ((uint64_t)t3.w << 32) | t3.z;
      wcnt = 0; u = 4;
      const uint64_t b = 8ull * (qend - qbeg) * (qend - qbeg) + 64;
      budget = b > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)b;
      st = read_id == INVALID_READ ? ST_IDLE : ST_ACTIVE;
    }
    wave_emit(P, lane, em, read_id, e, wout, rlen, wo, tpl);
    if (__ballot(rs)) {                                 // the rest of the query: another pass
      const uint64_t rsl = wave_slot(rs, rb, re, &P.ctl[C_PASSQ], lane);
      if (rs && rsl < P.resume_cap) {
        Query q;
        q.read_id = read_id; q.qbeg = qbeg; q.qend = qend; q.l = l; q.c = c; q.rlen = rlen;
        q.woff_lo = (uint32_t)wo; q.woff_hi = (uint32_t)(wo >> 32); q.send = qend; q.flags = Q_RESUME;
        q.pad0 = (uint32_t)i; q.pad1 = (uint32_t)j;
        P.resume[rsl] = q;
      }
    }
  }
  wave_close(P, lane, wout);
  for (uint64_t t = rb + lane; t < re; t += 64)
    if (t < P.resume_cap) P.resume[t].read_id = INVALID_READ;
  if ((threadIdx.x & 63) == 0 && n_iter) { atomicAdd(&P.ctl[C_WITER], (unsigned long long)n_iter); atomicAdd(&P.ctl[C_LITER], (unsigned long long)n_busy); }
  wave_stat(&P.ctl[C_LINES], (uint64_t)n_lines);
}

// ---------------------------------------------------------------------------------------------
// length bins: queries of reads that fit the LDS staging area run in the staged kernel, the rest
// (longest first) in the unstaged one

#define STAGE_MAX (32 * STAGE_WORDS)

__global__ void k_read_bins(const uint64_t *__restrict__ offs, uint64_t n, int stage, uint32_t *__restrict__ flag) {
  for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r < n; r += (uint64_t)gridDim.x * blockDim.x)
    flag[r] = (stage && offs[r + 1] - offs[r] <= STAGE_MAX) ? 1u : 0u;
}

// stable partition of read ids by flag (short reads first); sort keys of the long ones (longest first)
__global__ void k_read_partition(const uint64_t *__restrict__ offs, const uint32_t *__restrict__ flag,
                                 const uint32_t *__restrict__ pos, uint64_t n, uint64_t nshort, uint32_t *__restrict__ ids,
                                 uint32_t *__restrict__ lkey) {
  for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r < n; r += (uint64_t)gridDim.x * blockDim.x) {
    if (flag[r]) ids[pos[r]] = (uint32_t)r;
    else {
      const uint64_t t = r - pos[r];
      ids[nshort + t] = (uint32_t)r;
      lkey[t] = 65535u - (uint32_t)(offs[r + 1] - offs[r]);
    }
  }
}

// round-1 query records of reads ids[0..n)
__global__ void k_make_queries(const uint32_t *__restrict__ ids, uint64_t n, const uint64_t *__restrict__ offs,
                               const uint64_t *__restrict__ woff, uint32_t l, uint32_t c, Query *__restrict__ q,
                               const uint64_t *__restrict__ n_p = nullptr) {
  if (n_p) n = min(n, *n_p);   // captured graphs: the count on the device
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < n; t += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t r = ids ? ids[t] : (uint32_t)t;   // no ids: every read, in order
    const uint32_t len = (uint32_t)(offs[r + 1] - offs[r]);
    const uint64_t wo = woff[r];
    Query x;
    x.read_id = r; x.qbeg = 0; x.qend = len; x.l = l; x.c = c; x.rlen = len;
    x.woff_lo = (uint32_t)wo; x.woff_hi = (uint32_t)(wo >> 32);
    x.send = len; x.flags = 0;
    q[t] = x;
  }
}

// round-2 queries: short (staged) and long bins; unused slots of the per-wave output chunks dropped
__global__ void k_query_bins(const Query *__restrict__ q, uint64_t n, int stage, uint32_t *__restrict__ fs,
                             uint32_t *__restrict__ fl) {
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < n; t += (uint64_t)gridDim.x * blockDim.x) {
    const bool valid = q[t].read_id != INVALID_READ;
    const bool sh = stage && q[t].rlen <= STAGE_MAX;
    fs[t] = (valid && sh) ? 1u : 0u;
    fl[t] = (valid && !sh) ? 1u : 0u;
  }
}

// segments of long queries: [qbeg, qend) becomes ceil((qend - qbeg) / seg) queries, each reporting
// the SMEMs that start in its own seg bases (every segment after the first checks its first SMEM)
__global__ void k_seg_count(const Query *__restrict__ q, uint64_t n, uint32_t seg, uint32_t *__restrict__ cnt) {
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < n; t += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t len = q[t].qend > q[t].qbeg ? q[t].qend - q[t].qbeg : 0u;
    cnt[t] = len > seg ? (len + seg - 1) / seg : 1u;
  }
}

__global__ void k_seg_write(const Query *__restrict__ q, uint64_t n, uint32_t seg, const uint32_t *__restrict__ cnt,
                            const uint32_t *__restrict__ off, Query *__restrict__ out) {
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < n; t += (uint64_t)gridDim.x * blockDim.x) {
    const Query x = q[t];
    const uint32_t m = cnt[t];
    for (uint32_t g = 0; g < m; ++g) {
      Query y = x;
      y.qbeg = x.qbeg + g * seg;
      y.send = g + 1 < m ? y.qbeg + seg : x.send;
      y.flags = g > 0 ? (x.flags | SEG_CHECK) : x.flags;
      out[off[t] + g] = y;
    }
  }
}

__global__ void k_query_partition(const Query *__restrict__ in, const uint32_t *__restrict__ fs, const uint32_t *__restrict__ ps,
                                  const uint32_t *__restrict__ fl, const uint32_t *__restrict__ pl, uint64_t n,
                                  uint64_t nshort, Query *__restrict__ out) {
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < n; t += (uint64_t)gridDim.x * blockDim.x) {
    if (fs[t]) out[ps[t]] = in[t];
    else if (fl[t]) out[nshort + pl[t]] = in[t];
  }
}

// ---------------------------------------------------------------------------------------------
// plain SMEM kernel: one thread = one read, the serial algorithm, round 2 run inline

// One output slot for each lane active here: one atomic per group of simultaneously emitting lanes.
__device__ __forceinline__ uint64_t active_slot(unsigned long long *counter) {
  const uint64_t m = __ballot(1);
  const int lane = (int)(threadIdx.x & 63);
  const int leader = __ffsll((unsigned long long)m) - 1;
  unsigned long long b0 = 0;
  if (lane == leader) b0 = atomicAdd(counter, (unsigned long long)__popcll(m));
  b0 = __shfl(b0, leader);
  return b0 + __popcll(m & ((1ull << lane) - 1));
}

struct PlainCtx {
  IndexView ix;
  const SeedParams *P;
  const uint8_t *rb;
  uint32_t read_id;
  uint64_t lines, steps;
};

__device__ __forceinline__ uint64_t plain_step(PlainCtx &C, bool bwd, int a, uint64_t k, uint64_t kr, uint64_t s,
                                               uint64_t &nk, uint64_t &nkr) {
  const uint64_t x = bwd ? k : kr, y = bwd ? kr : k;
  const int cc = bwd ? a : 3 - a;
  uint64_t E1, G1, E2, G2;
  rank_global(C.ix, x, cc, E1, G1);
  rank_global(C.ix, x + s, cc, E2, G2);
  C.lines += line_of(x) == line_of(x + s) ? 1 : 2;
  C.steps++;
  uint64_t nx, ny, ns;
  ext_update(E1, G1, E2, G2, cc, x, s, y, C.ix.primary, sel4(C.ix.Cb[0], C.ix.Cb[1], C.ix.Cb[2], C.ix.Cb[3], cc), nx, ny, ns);
  if (bwd) { nk = nx; nkr = ny; } else { nkr = nx; nk = ny; }
  return ns;
}

template <int ROUND>
__device__ void emit_plain(PlainCtx &C, int i, int j, uint64_t k, uint64_t kr, uint64_t s);

template <int ROUND>
__device__ void plain_alg3(PlainCtx &C, int qbeg, int qend, int l, uint64_t c) {
  const SeedParams &P = *C.P;
  if (!(l >= 1 && l - 1 < qend - qbeg)) return;
  const uint64_t n = C.ix.n;
  int u = 1, i = qbeg, j = qbeg + l - 1;
  uint64_t k = 0, kr = 0, s = n;
  uint64_t budget = 8ull * (qend - qbeg) * (qend - qbeg) + 64;
  for (;;) {
    if (--budget == 0) { atomicOr(&P.ctl[C_ERR], 1ull); return; }
    if (u == 1 || u == 3) {
      if (u == 1 && j < i) { u = 2; j = i + l; continue; }
      if (u == 3 && j <= i) { u = 1; i = j + 1; j = j + l; k = 0; kr = 0; s = n; continue; }
      const int a = C.rb[j];
      uint64_t nk = 0, nkr = 0, ns = 0;
      if (a < 4) ns = plain_step(C, true, a, k, kr, s, nk, nkr);
      if (ns >= c) { k = nk; kr = nkr; s = ns; j -= 1; continue; }
      if (j + l < qend) { u = 1; i = j + 1; j = j + l; k = 0; kr = 0; s = n; continue; }
      return;
    }
    if (j == qend) { emit_plain<ROUND>(C, i, j, k, kr, s); return; }
    const int a = C.rb[j];
    uint64_t nk = 0, nkr = 0, ns = 0;
    if (a < 4) ns = plain_step(C, false, a, k, kr, s, nk, nkr);
    if (ns >= c) { k = nk; kr = nkr; s = ns; j += 1; continue; }
    emit_plain<ROUND>(C, i, j, k, kr, s);
    u = 3; k = 0; kr = 0; s = n;
  }
}

__device__ __forceinline__ void plain_record(PlainCtx &C, int round, int i, int j, uint64_t k, uint64_t kr, uint64_t s) {
  const SeedParams &P = *C.P;
  const uint64_t slot = active_slot(&P.ctl[C_NSEEDS]);
  if (slot < P.seed_cap) {
    SeedRec r;
    r.read_id = C.read_id; r.qbeg = (uint32_t)i; r.qend = (uint32_t)j; r.flags = round == 2 ? MBW_SEED_ROUND2 : 0u;
    r.k = k; r.kr = kr; r.s = s; r.pos = NO_POS;
    P.seeds[slot] = r;
  }
}

template <>
__device__ void emit_plain<2>(PlainCtx &C, int i, int j, uint64_t k, uint64_t kr, uint64_t s) {
  plain_record(C, 2, i, j, k, kr, s);
}

template <>
__device__ void emit_plain<1>(PlainCtx &C, int i, int j, uint64_t k, uint64_t kr, uint64_t s) {
  plain_record(C, 1, i, j, k, kr, s);
  if (C.P->reseed && j - i >= C.P->reseed_len && s <= (uint64_t)C.P->reseed_occ)
    plain_alg3<2>(C, i, j, (j - i) / 2, s + 1);
}

__global__ void __launch_bounds__(256) k_smem_plain(IndexView ix, SeedParams P) {
  uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (r >= P.n_queries) return;
  PlainCtx C;
  C.ix = ix; C.P = &P; C.read_id = (uint32_t)r; C.rb = P.codes + P.offs[r]; C.lines = 0; C.steps = 0;
  const int len = (int)(P.offs[r + 1] - P.offs[r]);
  plain_alg3<1>(C, 0, len, P.l, (uint64_t)P.c);
  atomicAdd(&P.ctl[C_LINES], (unsigned long long)C.lines);
  atomicAdd(&P.ctl[C_STEPS], (unsigned long long)C.steps);
}

// ---------------------------------------------------------------------------------------------
// seeds: sort keys, dedup, counts

// sort key (read, qbeg, qend); unused slots (read_id INVALID_READ) get key n_reads << 32, after all
// sort key (read, qbeg, qend) with qb bits for each offset (qb = bit length of the longest read);
// unused slots sort last as n_reads << 2 qb
// ns_p (captured graphs): the records written, on the device; slots from there to the capacity ns
// sort last like unused ones
__global__ void k_seed_keys(const SeedRec *__restrict__ raw, uint64_t ns, uint64_t n_reads, int qb, uint64_t *__restrict__ key,
                            uint32_t *__restrict__ val, const unsigned long long *__restrict__ ns_p = nullptr) {
  const uint64_t nv = ns_p ? min(ns, (uint64_t)*ns_p) : ns;
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < ns; t += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t rid = t < nv ? raw[t].read_id : INVALID_READ;
    key[t] = rid == INVALID_READ ? (n_reads << (2 * qb))
                                 : (((uint64_t)rid << (2 * qb)) | ((uint64_t)raw[t].qbeg << qb) | (uint64_t)raw[t].qend);
    val[t] = (uint32_t)t;
  }
}

__global__ void k_dedup_mark(const uint64_t *__restrict__ key, uint64_t ns, uint64_t n_reads, int qb, uint32_t *__restrict__ flag) {
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < ns; t += (uint64_t)gridDim.x * blockDim.x)
    flag[t] = (key[t] < (n_reads << (2 * qb)) && (t == 0 || key[t] != key[t - 1])) ? 1u : 0u;
}

__global__ void k_seed_emit(const SeedRec *__restrict__ raw, const uint32_t *__restrict__ val, const uint32_t *__restrict__ flag,
                            const uint32_t *__restrict__ idx, uint64_t ns, uint64_t max_occ, mbw_seed_t *__restrict__ out,
                            uint64_t *__restrict__ npos, uint64_t *__restrict__ kpos) {
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < ns; t += (uint64_t)gridDim.x * blockDim.x) {
    if (!flag[t]) continue;
    SeedRec r = raw[val[t]];
    mbw_seed_t o;
    o.read_id = r.read_id; o.qbeg = r.qbeg; o.qend = r.qend;
    o.k = r.k; o.kr = r.kr; o.s = r.s; o.pos_off = 0; o.reserved = 0;
    const bool loc = r.s <= max_occ;
    o.flags = r.flags | (loc ? 0u : MBW_SEED_UNLOCATED);
    o.npos = loc ? (uint32_t)r.s : 0u;
    const uint32_t d = idx[t];
    out[d] = o;
    npos[d] = o.npos;
    kpos[d] = r.pos;
  }
}

__global__ void k_seed_posoff(mbw_seed_t *__restrict__ out, const uint64_t *__restrict__ off, uint64_t ns) {
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < ns; t += (uint64_t)gridDim.x * blockDim.x)
    out[t].pos_off = off[t];
}

// start row of every (seed, occurrence) pair: X[pos_off + i] = k + i, with pos_off (the exclusive
// sum of the seeds' position counts) also stored in the seed.  A wave takes 64 seeds; a seed with
// few rows is written by its own lane (neighbouring lanes write neighbouring runs), a seed with many
// by all lanes of the wave (coalesced).  A seed whose position the unique-match path already found
// gets it written to the output and NO_POS in X (locate skips it).
#define EXPAND_LANE_MAX 8
// nu_p / xcap (captured graphs): the seed count on the device, at most ns; rows and positions are
// written only below xcap, and every row below it is written (NO_POS for a seed cut off by it), so
// that locate never reads a row that was not set
__global__ void __launch_bounds__(256) k_expand_rows(mbw_seed_t *__restrict__ seeds, const uint64_t *__restrict__ posoff,
                                                     const uint64_t *__restrict__ kpos, uint64_t ns, uint64_t *__restrict__ X,
                                                     uint64_t *__restrict__ pos, const uint32_t *__restrict__ nu_p = nullptr,
                                                     uint64_t xcap = ~0ull) {
  if (nu_p) ns = min(ns, (uint64_t)*nu_p);
  const int lane = threadIdx.x & 63;
  const uint64_t nwave = (uint64_t)gridDim.x * (blockDim.x >> 6);
  for (uint64_t base = ((uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 64; base < ns; base += nwave * 64) {
    uint64_t k = 0, off = 0, kp = NO_POS;
    uint32_t np = 0;
    if (base + lane < ns) {
      const uint64_t t = base + lane;
      k = seeds[t].k; np = seeds[t].npos; off = posoff[t]; kp = kpos[t];
      seeds[t].pos_off = off;
    }
    if (off + np > xcap) {          // past the capacity: rows below it that the seed would have
      for (uint64_t q = off; q < xcap; ++q) X[q] = NO_POS;   // started are marked for locate to skip
      np = 0;
    }
    const bool mine = np <= EXPAND_LANE_MAX;
    if (mine && np == 1 && kp != NO_POS) { X[off] = NO_POS; pos[off] = kp; }
    else if (mine)
      for (uint32_t q = 0; q < np; ++q) X[off + q] = k + q;
    uint64_t big = __ballot(!mine);
    while (big) {
      const int t = __ffsll((long long)big) - 1;
      big &= big - 1;
      const uint64_t kt = __shfl(k, t), ot = __shfl(off, t);
      const uint32_t nt = (uint32_t)__shfl((int)np, t);
      for (uint32_t q = (uint32_t)lane; q < nt; q += 64) X[ot + q] = kt + q;
    }
  }
}

// ---------------------------------------------------------------------------------------------
// locate (Algorithm 2)
__device__ __forceinline__ bool sampled(uint64_t x, uint32_t r, uint32_t rmask) {
  return rmask ? (x & rmask) == 0 : (x % r) == 0;
}
// x / r for a sampled row (r a power of two: shift)
__device__ __forceinline__ uint64_t sample_index(uint64_t x, uint32_t r, int rshift) {
  return rshift >= 0 ? (x >> rshift) : x / r;
}

// plain: one thread = one seed, LocateSlow for each of its rows
__global__ void __launch_bounds__(256) k_locate_plain(IndexView ix, const mbw_seed_t *__restrict__ seeds, uint64_t ns,
                                                      uint64_t *__restrict__ pos, uint32_t rmask, int rshift,
                                                      unsigned long long *__restrict__ ctl) {
  const uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (t >= ns) return;
  const mbw_seed_t sd = seeds[t];
  uint64_t lines = 0, lf = 0;
  for (uint32_t w = 0; w < sd.npos; ++w) {
    uint64_t x = sd.k + w, steps = 0;
    while (!sampled(x, ix.r, rmask)) {
      if (steps > ix.n) { atomicOr(&ctl[C_ERR], 2ull); x = 0; break; }
      if (x == ix.primary) { x = 0; ++steps; continue; }   // LF of the $ row is row 0
      const int b = bwt_global(ix, x);
      uint64_t E, G;
      rank_global(ix, x, b, E, G);
      if (b == 0 && x > ix.primary) E -= 1;
      x = sel4(ix.Cb[0], ix.Cb[1], ix.Cb[2], ix.Cb[3], b) + E;
      ++steps; ++lines; ++lf;
    }
    uint64_t p = steps + ix.ssa[sample_index(x, ix.r, rshift)];
    if (p >= ix.n) p -= ix.n;
    pos[sd.pos_off + w] = p;
    ++lines;
  }
  if (lines) {
    atomicAdd(&ctl[C_LINES_LOC], (unsigned long long)lines);
    atomicAdd(&ctl[C_LFSTEPS], (unsigned long long)lf);
  }
}

// wave: every lane walks one SA row; one memory phase per iteration holds the line fetches of the
// walking lanes, the SA-sample reads of lanes whose row is sampled and the start row of each
// lane's next walk (taken one walk ahead, so a finished lane continues at once).
__global__ void __launch_bounds__(256) k_locate_wave(IndexView ix, const uint64_t *__restrict__ X, uint64_t n_pos,
                                                     uint64_t *__restrict__ pos, uint32_t rmask, int rshift,
                                                     unsigned long long *__restrict__ ctl,
                                                     const uint64_t *__restrict__ np_p = nullptr) {
  if (np_p) n_pos = min(n_pos, *np_p);   // captured graphs: the row count on the device
  __shared__ uint64_t sbt[MBW_MAX_SB * 8];
  for (int t = threadIdx.x; t < 8 * ix.n_sb; t += blockDim.x) sbt[t] = ix.sbtab[t];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const uint32_t sbm = (1u << ix.sb_shift) - 1;
  enum { W_NONE = 0, W_WALK = 1 };
  enum { P_NONE = 0, P_PENDING = 1, P_READY = 2 };
  int cur = W_NONE, pre = P_NONE;
  bool drained = false;
  uint64_t w = 0, x = 0, steps = 0, pw = 0, px = 0;
  uint64_t lines = 0, lf = 0, cb = 0, ce = 0;
  for (;;) {
    if (cur == W_NONE && pre == P_READY) { cur = W_WALK; w = pw; x = px; steps = 0; pre = P_NONE; }
    const bool want = pre == P_NONE && !drained;
    if (__ballot(want)) {
      const uint64_t t = wave_take(want, cb, ce, &ctl[C_WORK2], n_pos, lane);
      if (want) { if (t == ~0ull) drained = true; else { pw = t; pre = P_PENDING; } }
    }
    if (__ballot(cur != W_NONE || pre != P_NONE) == 0) break;
    bool need = false, fin = false;
    if (cur == W_WALK) {
      if (sampled(x, ix.r, rmask)) fin = true;
      else if (x == ix.primary || steps > ix.n) {       // LF of the $ row is row 0 (the cap guards a corrupt index)
        if (steps > ix.n) atomicOr(&ctl[C_ERR], 2ull);
        x = 0; ++steps;
      } else need = true;
    }
    const uint32_t L = line_of(x);
    const int o = (int)(x - (uint64_t)L * MBW_BPL);
    // ---- memory phase
    const uint4 z4 = make_uint4(0, 0, 0, 0);
    uint4 h0 = z4, h1 = z4, blk = z4;
    if (need) {
      const uint4 *lp = ix.lines + (uint64_t)L * MBW_LINE_U4;
      h0 = lp[0]; h1 = lp[1]; blk = lp[2 + (o >> 6)];
    }
    uint64_t sv = 0;
    if (fin) sv = ix.ssa[sample_index(x, ix.r, rshift)];
    const bool ld = pre == P_PENDING;
    if (ld) px = X[pw];
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    // ---- compute
    if (ld) pre = px == NO_POS ? P_NONE : P_READY;   // NO_POS: located by the SMEM kernel already
    if (fin) {
      uint64_t p = steps + sv;
      if (p >= ix.n) p -= ix.n;
      pos[w] = p;
      ++lines;
      cur = W_NONE;
    }
    if (need) {
      const int b = bwt_from_block(blk, o);
      const uint32_t sbi = 8 * (L >> ix.sb_shift);
      uint64_t E, G;
      rank_eg(h0, h1, blk, L & sbm, o, b, sym_masks(b), sbt[sbi + b], sbt[sbi + 4 + b], E, G);
      if (b == 0 && x > ix.primary) E -= 1;
      x = sel4(ix.Cb[0], ix.Cb[1], ix.Cb[2], ix.Cb[3], b) + E;
      ++steps; ++lines; ++lf;
    }
  }
  wave_stat(&ctl[C_LINES_LOC], lines);
  wave_stat(&ctl[C_LFSTEPS], lf);
}

// ---------------------------------------------------------------------------------------------
// bisulfite strand filter (Section 2.9): segment = pos / |R| of T over the four copies
// np_p (captured graphs): the positions on the device, at most the capacity np; slots from there
// to np are not kept
__global__ void k_bs_mark(const uint64_t *__restrict__ pos, uint64_t np, uint64_t len_r, int role, uint32_t *__restrict__ keep,
                          const uint64_t *__restrict__ np_p = nullptr) {
  const uint64_t nv = np_p ? min(np, *np_p) : np;
  for (uint64_t w = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; w <= np; w += (uint64_t)gridDim.x * blockDim.x) {
    if (w >= nv) { keep[w] = 0; continue; }
    const uint64_t seg = pos[w] / len_r;
    keep[w] = (role == 1) ? (seg == 0 || seg == 2) : (seg == 1 || seg == 3);
  }
}

__global__ void k_bs_compact(const uint64_t *__restrict__ pos, const uint32_t *__restrict__ keep, const uint64_t *__restrict__ kidx,
                             uint64_t np, uint64_t *__restrict__ out) {
  for (uint64_t w = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; w < np; w += (uint64_t)gridDim.x * blockDim.x)
    if (keep[w]) out[kidx[w]] = pos[w];
}

// ns_p / cap (captured graphs): the seed count on the device; position offsets clamped to the
// position capacity (past it the result is refused anyway)
__global__ void k_bs_seeds(mbw_seed_t *__restrict__ seeds, uint64_t ns, const uint64_t *__restrict__ kidx,
                           const uint32_t *__restrict__ ns_p = nullptr, uint64_t cap = ~0ull) {
  if (ns_p) ns = min(ns, (uint64_t)*ns_p);
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < ns; t += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t a = min(seeds[t].pos_off, cap), b = min(seeds[t].pos_off + seeds[t].npos, cap);
    seeds[t].pos_off = kidx[a];
    seeds[t].npos = (uint32_t)(kidx[b] - kidx[a]);
  }
}

// ---------------------------------------------------------------------------------------------
// bisulfite seed refinement (Section 2.9): every kept (seed, position) pair is compared base by
// base with the original read and the original reference; it is split where read 1 has a C over a
// reference T (read 2: G over A), which bisulfite conversion cannot produce, and pieces of at
// least min_len bases are kept with their own text positions

// the seed of every kept position
__global__ void __launch_bounds__(256) k_pos_seed(const mbw_seed_t *__restrict__ seeds, uint64_t ns, uint32_t *__restrict__ ps,
                                                  const uint32_t *__restrict__ ns_p = nullptr, uint64_t cap = ~0ull) {
  if (ns_p) ns = min(ns, (uint64_t)*ns_p);   // captured graphs: the seed count on the device; ps holds cap
  const int lane = threadIdx.x & 63;
  const uint64_t nwave = (uint64_t)gridDim.x * (blockDim.x >> 6);
  for (uint64_t base = ((uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 64; base < ns; base += nwave * 64) {
    uint64_t off = 0;
    uint32_t np = 0;
    if (base + lane < ns) { off = seeds[base + lane].pos_off; np = seeds[base + lane].npos; }
    const int cnt = (int)min<uint64_t>(64, ns - base);
    for (int t = 0; t < cnt; ++t) {
      const uint64_t ot = __shfl(off, t);
      const uint32_t nt = (uint32_t)__shfl((int)np, t);
      for (uint32_t q = (uint32_t)lane; q < nt && ot + q < cap; q += 64) ps[ot + q] = (uint32_t)(base + t);
    }
  }
}

// original reference base (0..3) under text position t of the four-copy bisulfite text
__device__ __forceinline__ int orig_base(const uint64_t *__restrict__ orig, uint64_t L, uint64_t t) {
  uint64_t q;
  bool rc = t >= 2 * L;
  q = rc ? 4 * L - 1 - t : t;
  if (q >= L) q -= L;
  const int b = (int)((orig[q >> 5] >> (2 * (q & 31))) & 3);
  return rc ? 3 - b : b;
}

// pass 0 (out == nullptr): pieces per position into cnt; pass 1: write them at poff
__global__ void k_refine(const mbw_seed_t *__restrict__ seeds, const uint32_t *__restrict__ pseed,
                         const uint64_t *__restrict__ pos, uint64_t np, const uint8_t *__restrict__ ascii,
                         const uint64_t *__restrict__ offs, const uint64_t *__restrict__ orig, uint64_t L, int role,
                         int min_len, uint32_t *__restrict__ cnt, const uint64_t *__restrict__ poff,
                         mbw_piece_t *__restrict__ out, const uint64_t *__restrict__ np_p = nullptr,
                         uint64_t pcap = ~0ull) {
  if (np_p) np = min(np, *np_p);   // captured graphs: the positions on the device; pieces written below pcap
  const uint32_t bad = role == 1 ? 'C' : 'G';          // read base that cannot face ...
  const int over = role == 1 ? 3 : 0;                  // ... this original reference base
  for (uint64_t w = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; w < np; w += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t t = pseed[w];
    const mbw_seed_t sd = seeds[t];
    const uint64_t p = pos[w];
    const uint8_t *P = ascii + offs[sd.read_id];
    uint32_t start = sd.qbeg, c = 0;
    for (uint32_t i = sd.qbeg; i <= sd.qend; ++i) {
      bool cut = i == sd.qend;
      if (!cut) cut = ((uint32_t)P[i] & 0xDFu) == bad && orig_base(orig, L, p + (i - sd.qbeg)) == over;
      if (cut) {
        if (i - start >= (uint32_t)min_len) {
          if (out && poff[w] + c < pcap) {
            mbw_piece_t x;
            x.read_id = sd.read_id; x.qbeg = start; x.qend = i; x.seed = t; x.pos = p + (start - sd.qbeg);
            out[poff[w] + c] = x;
          }
          ++c;
        }
        start = i + 1;
      }
    }
    if (!out) cnt[w] = c;
  }
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// context (struct mbw_ctx and its buffer helpers: ctx.h)
static_assert(C_COUNT <= MBW_CTL_WORDS, "control block larger than the context's host copy");

static int scratch_init(int device);

extern "C" int mbw_ctx_create(const mbw_index *ix, mbw_ctx **out) {
  if (!ix || !out) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  *out = nullptr;
  TRY(hipSetDevice(ix->device));
  mbw_ctx *c = new mbw_ctx();
  c->ix = ix;
  mbw_index_retain(ix);   // released by mbw_ctx_free, also on the failure paths below
  c->device = ix->device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, ix->device) != hipSuccess) { mbw_ctx_free(c); mbw_set_error("hipGetDeviceProperties failed"); return MBW_E_HIP; }
  c->n_cu = prop.multiProcessorCount;
  if (hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking) != hipSuccess) {
    c->own = nullptr; mbw_ctx_free(c); mbw_set_error("hipStreamCreate failed"); return MBW_E_HIP;
  }
  for (int t = 0; t < 8; ++t)
    if (hipEventCreate(&c->ev[t]) != hipSuccess) { mbw_ctx_free(c); mbw_set_error("hipEventCreate failed"); return MBW_E_HIP; }
  for (int t = 0; t < 2 * mbw_ctx::kLaunchSlots; ++t)
    if (hipEventCreate(&c->lev[t]) != hipSuccess) { mbw_ctx_free(c); mbw_set_error("hipEventCreate failed"); return MBW_E_HIP; }
  {
    // keep memory freed by growing buffers in the device's pool instead of returning it at every sync
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, ix->device) == hipSuccess) {
      uint64_t thr = ~0ull;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
  }
  if (grow(c, c->ctl, C_COUNT * sizeof(unsigned long long))) { mbw_ctx_free(c); return MBW_E_NOMEM; }
  // the device address of the static scratch array, looked up once for this device (it is current)
  if (int rs = scratch_init(ix->device)) { mbw_ctx_free(c); return rs; }
  if (hipHostMalloc((void **)&c->hfetch, MBW_CTL_WORDS * sizeof(uint64_t), hipHostMallocCoherent) != hipSuccess ||
      hipHostGetDevicePointer((void **)&c->dfetch, c->hfetch, 0) != hipSuccess) {
    mbw_ctx_free(c);
    mbw_set_error("pinned host buffer allocation failed");
    return MBW_E_NOMEM;
  }
  (void)hipStreamSynchronize(nullptr);
  *out = c;
  return MBW_OK;
}

// Entry points wait for their stream before they return, except when they fail part way; the
// device-wide wait covers that case without touching the caller's last stream (which may be gone).
// The buffers are then freed on the context's own stream and the device's pool gives the freed
// memory back.
extern "C" void mbw_ctx_free(mbw_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  if (c->own) {
    for (auto *b : c->buffers()) if (b->p) (void)hipFreeAsync(b->p, c->own);
    (void)hipStreamSynchronize(c->own);
    (void)hipStreamDestroy(c->own);
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, c->device) == hipSuccess) (void)hipMemPoolTrimTo(pool, 0);
  }
  for (int t = 0; t < 8; ++t) if (c->ev[t]) (void)hipEventDestroy(c->ev[t]);
  for (int t = 0; t < 2 * mbw_ctx::kLaunchSlots; ++t) if (c->lev[t]) (void)hipEventDestroy(c->lev[t]);
  if (c->hfetch) (void)hipHostFree(c->hfetch);
  const mbw_index *ix = c->ix;
  delete c;
  if (ix) mbw_index_release(ix);
}

// Persistent grid: blocks per CU as requested (> 0), the occupancy limit (< 0), or (0) sized by
// the launch's work, `per_block` items per block and CU, up to the occupancy limit.  A small batch
// is bound by its longest chains of dependent loads: more waves per SIMD only slow each one
// (they share the SIMD) and add same-address atomics on the work counter, which serialise.
static int persistent_grid(const void *kern, int block, size_t lds, int n_cu, int per_cu_req, uint64_t work,
                           uint64_t per_block, int auto_max = 0) {
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, block, lds) != hipSuccess || per < 1) per = 4;
  int want = per_cu_req;
  if (want == 0) {
    const uint64_t unit = per_block * (uint64_t)n_cu;
    const int cap = auto_max > 0 ? std::min(per, auto_max) : per;
    want = (int)std::min<uint64_t>((uint64_t)cap, std::max<uint64_t>(1, (work + unit - 1) / unit));
  }
  if (want > 0 && want < per) per = want;
  return per * n_cu;
}

// automatic sizing (blocks_per_cu = 0): items per block and CU, measured at 3.1 Gbp on 150 bp
// reads (a round-2 query costs less than a round-1 one: most fail their first test)
#define AUTO_QUERIES_R1 1200
#define AUTO_QUERIES_R2 4000
#define AUTO_ROWS_LOCATE 24000
// ... and at most 4 locate blocks (4 waves per SIMD) per CU: on the 3.1 Gbp index the random line
// reads of the walks complete faster with 4 waves per SIMD than with the 8 the registers allow
// (36.7 ms against 43.5 ms for 442 M rows; 5, 6 and 8 waves: 39.4, 41.4, 43.2 ms)
#define AUTO_LOCATE_MAX_PER_CU 4

template <bool STAGED, bool UNIQ, bool DEFER = false>
static int wave_grid(mbw_ctx *c, const SeedParams &P, const mbw_seed_opts &o) {
  return persistent_grid((const void *)k_smem_wave<STAGED, UNIQ, DEFER>, 64 * SMEM_WAVES, 0, c->n_cu, o.blocks_per_cu,
                         P.n_queries, P.round == 1 ? AUTO_QUERIES_R1 : AUTO_QUERIES_R2);
}

// kinds of SMEM-stage launch: the SMEM kernel, with deferred unique matches, the continuation kernel
enum { L_SMEM = 0, L_DEFER = 1, L_UNIQUE = 2 };

static int smem_grid(mbw_ctx *c, const SeedParams &P, const mbw_seed_opts &o, bool staged, int kind = L_SMEM) {
  if (kind == L_UNIQUE)
    return persistent_grid((const void *)k_unique_wave, 64 * UNIQ_WAVES, 0, c->n_cu, o.blocks_per_cu, P.n_queries,
                           AUTO_TASKS);
  if (kind == L_DEFER) return wave_grid<true, false, true>(c, P, o);
  const bool uniq = P.uniq && P.round == 1;
  if (staged) return uniq ? wave_grid<true, true>(c, P, o) : wave_grid<true, false>(c, P, o);
  return uniq ? wave_grid<false, true>(c, P, o) : wave_grid<false, false>(c, P, o);
}

static int launch_smem(const IndexView &v, SeedParams &P, const ReadWords &R, const mbw_seed_opts &o, bool staged,
                       int grid, hipStream_t st, int kind) {
  const bool uniq = P.uniq && P.round == 1;
  const int bs = 64 * SMEM_WAVES;
  if (kind == L_UNIQUE) k_unique_wave<<<grid, 64 * UNIQ_WAVES, 0, st>>>(v, P, R);
  else if (kind == L_DEFER) k_smem_wave<true, false, true><<<grid, bs, 0, st>>>(v, P, R);
  else if (o.kernel == MBW_KERNEL_PLAIN) k_smem_plain<<<grid_for(P.n_queries, 256), 256, 0, st>>>(v, P);
  else if (staged) {
    if (uniq) k_smem_wave<true, true><<<grid, bs, 0, st>>>(v, P, R);
    else k_smem_wave<true, false><<<grid, bs, 0, st>>>(v, P, R);
  } else {
    if (uniq) k_smem_wave<false, true><<<grid, bs, 0, st>>>(v, P, R);
    else k_smem_wave<false, false><<<grid, bs, 0, st>>>(v, P, R);
  }
  TRY(hipGetLastError());
  return 0;
}

// MBW_TRACE=1: one JSON line on stderr per SMEM launch and per mbw_seed call
static bool trace_on() {
  static const bool on = getenv("MBW_TRACE") && getenv("MBW_TRACE")[0] == '1';
  return on;
}

// Device times of the SMEM launches recorded so far, read after the host has waited for the
// stream (every launch is followed by such a wait before its slot could be needed again).
static int flush_launch_times(mbw_ctx *c) {
  for (int t = 0; t < c->n_pending; ++t) {
    float ms = 0;
    TRY(hipEventElapsedTime(&ms, c->lev[2 * t], c->lev[2 * t + 1]));
    c->ms_smem += ms;
    const mbw_ctx::LaunchNote &n = c->pending[t];
    if (trace_on())
      fprintf(stderr, "{\"mbw\": \"smem_launch\", \"round\": %d, \"staged\": %d, \"kind\": \"%s\", \"queries\": %llu, "
              "\"blocks\": %d, \"chunk\": %u, \"ms\": %.3f}\n", n.round, n.staged,
              n.kind == L_UNIQUE ? "unique" : (n.kind == L_DEFER ? "defer" : "smem"), (unsigned long long)n.queries, n.grid,
              n.chunk, ms);
  }
  c->n_pending = 0;
  return 0;
}

static int run_smem(mbw_ctx *c, const IndexView &v, SeedParams &P, const ReadWords &R, const mbw_seed_opts &o, bool staged,
                    hipStream_t st, int kind = L_SMEM) {
  if (P.n_queries == 0) return 0;
  const int grid = (o.kernel == MBW_KERNEL_PLAIN && kind == L_SMEM) ? 0 : smem_grid(c, P, o, staged, kind);
  // at least ~8 grabs per wave of the persistent grid, so that long queries (queued longest
  // first) spread over the whole chip
  if (o.wave_chunk > 0) P.chunk = (uint32_t)std::min(WORK_CHUNK, o.wave_chunk);
  else {
    const uint64_t waves = (uint64_t)std::max(grid, 1) * (kind == L_UNIQUE ? UNIQ_WAVES : SMEM_WAVES);
    uint64_t ch = P.n_queries / (waves * 8);
    P.chunk = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(WORK_CHUNK, ch));
  }
  if (c->n_pending == mbw_ctx::kLaunchSlots) {   // not reached by mbw_seed's launch sequence
    TRY(hipStreamSynchronize(st));
    int r = flush_launch_times(c);
    if (r) return r;
  }
  const int slot = c->n_pending++;
  c->pending[slot] = {P.round, (int)staged, kind, grid, P.n_queries, P.chunk};
  TRY(hipEventRecord(c->lev[2 * slot], st));
  int r = launch_smem(v, P, R, o, staged, grid, st, kind);
  if (r) return r;
  TRY(hipEventRecord(c->lev[2 * slot + 1], st));
  c->n_smem_launches++;
  return 0;
}

// Sizes the host needs before it can launch the next steps (counts, scan totals): one kernel copies
// up to FETCH_MAX device words into the context's pinned host buffer and the host waits once.  A
// device-to-host copy per value costs a copy dispatch of its own, about 30 us each on a small batch.
#define FETCH_MAX MBW_CTL_WORDS
static_assert(C_COUNT <= FETCH_MAX, "the whole control block fits one fetch");
struct FetchList { const void *p[FETCH_MAX]; int wide[FETCH_MAX]; int n; };
struct FetchItem { const void *p; int wide; };   // wide: 8-byte word, else 4-byte
__global__ void k_fetch(FetchList f, uint64_t *dst) {
  const int t = threadIdx.x;
  if (t < f.n) dst[t] = f.wide[t] ? *(const uint64_t *)f.p[t] : (uint64_t)*(const uint32_t *)f.p[t];
  __threadfence_system();
}
static int fetch(mbw_ctx *c, hipStream_t st, std::initializer_list<FetchItem> items, uint64_t *out) {
  if (items.size() > FETCH_MAX) { mbw_set_error("internal: too many values in one fetch"); return MBW_E_INVAL; }
  FetchList f;
  f.n = 0;
  for (const FetchItem &it : items) { f.p[f.n] = it.p; f.wide[f.n] = it.wide; ++f.n; }
  k_fetch<<<1, 64, 0, st>>>(f, c->dfetch);
  TRY(hipGetLastError());
  TRY(hipStreamSynchronize(st));
  for (int t = 0; t < f.n; ++t) out[t] = ((volatile uint64_t *)c->hfetch)[t];
  return flush_launch_times(c);
}
#define FETCH(...) do { int r_ = fetch(c, st, __VA_ARGS__); if (r_) return r_; } while (0)

// zero two counters of the control block
__global__ void k_ctl_zero(unsigned long long *ctl, int a, int b) {
  if (threadIdx.x == 0) { ctl[a] = 0; ctl[b] = 0; }
}

// Slots a pass of the deferred unique-match path may need beyond its valid entries: one partly
// used output chunk per wave of the largest grid.
static uint64_t defer_slack(const mbw_ctx *c) {
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)k_smem_wave<true, false, true>, 64 * SMEM_WAVES, 0) !=
          hipSuccess || per < 1)
    per = 4;
  int per_u = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_u, (const void *)k_unique_wave, 64 * UNIQ_WAVES, 0) != hipSuccess ||
      per_u < 1)
    per_u = 8;
  const uint64_t waves = (uint64_t)c->n_cu * std::max(per * SMEM_WAVES, per_u * UNIQ_WAVES);
  return waves * OUT_CHUNK;
}

#define DEFER_SLACK_PASSES 4         // passes whose partly used output chunks the first sizing allows for

// Round 1 of the staged bin with deferred unique matches: the SMEM kernel over the queries writes
// the unique matches it reaches to the task list, the continuation kernel finishes them and lists
// the queries that go on; the two alternate until no query is left.  Every pass advances each of
// its queries past at least one SMEM end, so a read of at most STAGE_MAX bases needs at most
// STAGE_MAX + 1 passes.
static int run_deferred(mbw_ctx *c, const IndexView &v, SeedParams &P, const ReadWords &R, const mbw_seed_opts &o,
                        const Query *qs, uint64_t ns, hipStream_t st) {
  const uint64_t cap = ns + defer_slack(c);
  GROW(c->utask, cap * sizeof(UTask));
  GROW(c->ures, cap * sizeof(Query));
  const Query *q = qs;
  uint64_t nq = ns;
  for (int pass = 0;; ++pass) {
    if (pass > STAGE_MAX + 1) { mbw_set_error("internal: unique-match passes did not end"); return MBW_E_INVAL; }
    k_ctl_zero<<<1, 64, 0, st>>>(P.ctl, C_WORK, C_PASSQ);
    TRY(hipGetLastError());
    SeedParams Pd = P;
    Pd.queries = q; Pd.n_queries = nq; Pd.tasks = (UTask *)c->utask.p; Pd.task_cap = cap;
    int r = run_smem(c, v, Pd, R, o, true, st, L_DEFER);
    if (r) return r;
    uint64_t nt = 0;
    FETCH({{P.ctl + C_PASSQ, 1}}, &nt);
    if (nt > cap) { mbw_set_error("internal: task list overflow"); return MBW_E_INVAL; }
    if (!nt) break;
    k_ctl_zero<<<1, 64, 0, st>>>(P.ctl, C_WORK, C_PASSQ);
    TRY(hipGetLastError());
    SeedParams Pu = P;
    Pu.tasks = (UTask *)c->utask.p; Pu.n_queries = nt; Pu.resume = (Query *)c->ures.p; Pu.resume_cap = cap;
    r = run_smem(c, v, Pu, R, o, true, st, L_UNIQUE);
    if (r) return r;
    uint64_t nr = 0;
    FETCH({{P.ctl + C_PASSQ, 1}}, &nr);
    if (nr > cap) { mbw_set_error("internal: resume list overflow"); return MBW_E_INVAL; }
    if (!nr) break;
    q = (const Query *)c->ures.p;
    nq = nr;
  }
  return 0;
}

// one seeding round: the staged kernel over qs[0, ns), the unstaged one over ql[0, nl); each launch
// starts its own work counter
static int run_binned(mbw_ctx *c, const IndexView &v, SeedParams &P, const ReadWords &R, const mbw_seed_opts &o,
                      const Query *qs, uint64_t ns, const Query *ql, uint64_t nl, hipStream_t st, bool defer = false) {
  if (ns && defer) {
    int r = run_deferred(c, v, P, R, o, qs, ns, st);
    if (r) return r;
  } else if (ns) {
    TRY(hipMemsetAsync(P.ctl + C_WORK, 0, 8, st));
    P.queries = qs; P.n_queries = ns;
    int r = run_smem(c, v, P, R, o, true, st);
    if (r) return r;
  }
  if (nl) {
    TRY(hipMemsetAsync(P.ctl + C_WORK, 0, 8, st));
    P.queries = ql; P.n_queries = nl;
    int r = run_smem(c, v, P, R, o, false, st);
    if (r) return r;
  }
  return 0;
}


// round 2 starts from round 1's seed count and line statistics again on a retry
__global__ void k_ctl_restore(unsigned long long *ctl, unsigned long long n1, unsigned long long l0, unsigned long long l1,
                              unsigned long long l2) {
  if (threadIdx.x == 0) { ctl[C_NSEEDS] = n1; ctl[C_LINES] = l0; ctl[C_LINES + 1] = l1; ctl[C_LINES + 2] = l2; }
}

// split the n queries of q into segments (ctx buffer `out`); returns the segment count in *nseg
static int segment_queries(mbw_ctx *c, const Query *q, uint64_t n, uint32_t seg, mbw_ctx::Buf &out, uint64_t *nseg,
                           hipStream_t st) {
  *nseg = 0;
  if (!n) return 0;
  GROW(c->sc0, (n + 1) * 4); GROW(c->sc1, (n + 1) * 4);
  uint32_t *cnt = (uint32_t *)c->sc0.p, *off = (uint32_t *)c->sc1.p;
  k_seg_count<<<grid_for(n), 256, 0, st>>>(q, n, seg, cnt);
  TRY(hipGetLastError());
  int r = prim_call(c, [&](void *tp, size_t &tb) { return prim::exclusive_sum(tp, tb, cnt, off, n, st); });
  if (r) return r;
  uint64_t tail[2] = {0, 0};
  FETCH({{cnt + n - 1, 0}, {off + n - 1, 0}}, tail);
  *nseg = tail[0] + tail[1];
  GROW(out, (*nseg + 1) * sizeof(Query));
  k_seg_write<<<grid_for(n), 256, 0, st>>>(q, n, seg, cnt, off, (Query *)out.p);
  TRY(hipGetLastError());
  return 0;
}

// A generous estimate of the work space one call takes, from its read count and bases (the seeding
// result is assumed typical; grids as the automatic sizing picks them).  A work space call that
// runs short reports the larger of this and the exact need so far, so that a caller who enlarges
// to the report usually needs one retry.
static MbwSizeModel size_model(const mbw_ctx *c, uint64_t n, uint64_t bases, bool host_reads, const mbw_seed_opts &o) {
  const uint64_t words = bases / 32 + n + 2;
  uint64_t per_cu = 4;   // round-1 blocks per CU: as persistent_grid sizes them
  if (o.blocks_per_cu > 0) per_cu = std::min<uint64_t>(4, (uint64_t)o.blocks_per_cu);
  else if (o.blocks_per_cu == 0)
    per_cu = std::min<uint64_t>(4, std::max<uint64_t>(1, (n + AUTO_QUERIES_R1 * (uint64_t)c->n_cu - 1) /
                                                             (AUTO_QUERIES_R1 * (uint64_t)c->n_cu)));
  const uint64_t slack = 2 * per_cu * (uint64_t)c->n_cu * SMEM_WAVES * OUT_CHUNK;
  // typical result: 8 seeds and 64 positions per read, or one seed per 16 bases and one position
  // per 2 bases for long reads
  const uint64_t recs = std::max<uint64_t>(8 * n, bases / 16);
  const uint64_t rows = std::max<uint64_t>(64 * n, bases / 2);
  const uint64_t seeds = std::max<uint64_t>(1 << 16, recs) + slack;
  uint64_t b = 0;
  b += n * (4 + 8 + 8 + 8 + 8 + 48 + 6 * 4 + 8 + 96);   // lengths, offsets, word counts, queries, bins, segments
  b += host_reads ? bases + 16 : 0;
  b += words * (8 + 4 + 4);                              // packed words, N masks, word owners
  b += seeds * (sizeof(SeedRec) + sizeof(Query) + 16 + 8 + 8 + 24);   // seeds, sub-queries, sort, per-seed counts
  b += rows * (8 + 8 + 4 + 8 + 8 + 4 + 4 + 8);           // rows, positions, filter and refinement arrays
  b += 16ull << 20;                                      // temporary storage of sorts and scans
  if (o.unique_defer == 1)                               // task and resume lists, output chunks of the passes
    b += (n + defer_slack(c)) * (sizeof(UTask) + sizeof(Query)) +
         DEFER_SLACK_PASSES * defer_slack(c) * (sizeof(SeedRec) + sizeof(Query) + 16 + 8 + 8 + 24);
  MbwSizeModel m;
  m.ws = b;
  m.seeds = recs;
  m.pos = rows;
  m.pieces = o.bs_refine ? rows : 0;
  return m;
}

static uint64_t ws_estimate(const mbw_ctx *c, uint64_t n, uint64_t bases, bool host_reads, const mbw_seed_opts &o) {
  return size_model(c, n, bases, host_reads, o).ws;
}

MbwSizeModel mbw_size_model(const mbw_ctx *c, uint64_t n, uint64_t bases, bool host_reads, const mbw_seed_opts *o) {
  return size_model(c, n, bases, host_reads, *o);
}

// The whole path of one call.  ob == nullptr: buffers are the context's own (grown as needed);
// otherwise the context is in work space mode (ArenaScope) and the seeds, positions and pieces go to
// the caller's buffers, whose required sizes are written back as they become known.
static int seed_impl(mbw_ctx *c, const uint8_t *reads, const uint32_t *lengths, uint64_t n_reads, int min_seed_len,
                     int max_occ, const mbw_seed_opts *opts, void *stream, mbw_seed_buffers *ob, mbw_result *out) {
  if (!c || !out) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  memset(out, 0, sizeof(*out));
  if (min_seed_len < 1 || max_occ < 1) { mbw_set_error("min_seed_len and max_occ must be >= 1"); return MBW_E_INVAL; }
  if (n_reads > 0 && (!reads || !lengths)) { mbw_set_error("NULL reads or lengths"); return MBW_E_INVAL; }
  if (n_reads >= (1ull << 31)) { mbw_set_error("too many reads in one call"); return MBW_E_INVAL; }
  mbw_seed_opts o;
  if (opts) o = *opts;
  else {
    memset(&o, 0, sizeof(o));
    o.min_occ = 1; o.reseed = 1; o.reseed_len = 38; o.reseed_occ = 10; o.use_kmer = 1; o.unique_ext = 1;
  }
  if (o.min_occ < 1) { mbw_set_error("min_occ must be >= 1"); return MBW_E_INVAL; }
  if (o.wave_chunk < 0 || o.wave_chunk > WORK_CHUNK) { mbw_set_error("wave_chunk must be in [0,256]"); return MBW_E_INVAL; }
  if (o.unique_defer < 0 || o.unique_defer > 1) { mbw_set_error("unique_defer must be 0 or 1"); return MBW_E_INVAL; }
  if (o.bs_role && !c->ix->bisulfite) { mbw_set_error("bs_role needs a bisulfite index"); return MBW_E_INVAL; }
  if (o.bs_refine && (!o.bs_role || !c->ix->orig)) {
    mbw_set_error("bs_refine needs bs_role and a bisulfite index"); return MBW_E_INVAL;
  }
  if (o.bs_role < 0 || o.bs_role > 2) { mbw_set_error("bs_role must be 0, 1 or 2"); return MBW_E_INVAL; }
  if (o.kernel != MBW_KERNEL_COOP && o.kernel != MBW_KERNEL_PLAIN) { mbw_set_error("unknown kernel"); return MBW_E_INVAL; }
  TRY(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  c->cur = st;
  const mbw_index *ix = c->ix;
  const IndexView v = make_view(ix);
  unsigned long long *ctl = (unsigned long long *)c->ctl.p;
  if (c->arena) c->arena_hint = ws_estimate(c, n_reads, 300 * n_reads, true, o);
  TRY(hipMemsetAsync(ctl, 0, C_COUNT * sizeof(unsigned long long), st));
  c->ms_smem = 0;
  c->n_smem_launches = 0;
  c->n_pending = 0;
  TRY(hipEventRecord(c->ev[0], st));
  if (n_reads == 0) {
    TRY(hipStreamSynchronize(st));
    return MBW_OK;
  }
  // lengths -> offsets (u64), max length
  GROW(c->lens, (n_reads + 1) * sizeof(uint32_t));
  const uint32_t *dlen = lengths;
  if (!is_device_ptr(lengths)) {
    TRY(hipMemcpyAsync(c->lens.p, lengths, n_reads * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    dlen = (const uint32_t *)c->lens.p;
  }
  GROW(c->offs, (n_reads + 2) * sizeof(uint64_t));
  GROW(c->npos, (n_reads + 2) * sizeof(uint64_t));
  uint64_t *wide = (uint64_t *)c->npos.p;
  k_widen<<<grid_for(n_reads + 1, 256, 1024u), 256, 0, st>>>(dlen, n_reads, wide, ctl + C_MAXLEN);
  TRY(hipGetLastError());
  uint64_t *offs = (uint64_t *)c->offs.p;
  int r = prim_call(c, [&](void *tp, size_t &tb) { return prim::exclusive_sum(tp, tb, wide, offs, n_reads + 1, st); });
  if (r) return r;
  const bool coop = o.kernel != MBW_KERNEL_PLAIN;
  // wave kernels: packed-word offsets and the LDS-staging bins follow from the offsets alone, so
  // their scans run before the one wait that reads every size the next steps need
  uint64_t *nwd = nullptr, *woff = nullptr;
  uint32_t *flag1 = nullptr, *pos1 = nullptr;
  if (coop) {
    GROW(c->nwords, (n_reads + 1) * 8);
    GROW(c->woffs, (n_reads + 1) * 8);
    nwd = (uint64_t *)c->nwords.p; woff = (uint64_t *)c->woffs.p;
    k_read_words<<<grid_for(n_reads + 1), 256, 0, st>>>(offs, n_reads, nwd);
    TRY(hipGetLastError());
    r = prim_call(c, [&](void *tp, size_t &tb) { return prim::exclusive_sum(tp, tb, nwd, woff, n_reads + 1, st); });
    if (r) return r;
    GROW(c->q1, (n_reads + 1) * sizeof(Query));
    GROW(c->bf0, (n_reads + 1) * 4); GROW(c->bp0, (n_reads + 1) * 4);
    GROW(c->bid0, (n_reads + 1) * 4); GROW(c->bid1, (n_reads + 1) * 4);
    GROW(c->bk0, (n_reads + 1) * 4); GROW(c->bk1, (n_reads + 1) * 4);
    flag1 = (uint32_t *)c->bf0.p; pos1 = (uint32_t *)c->bp0.p;
    k_read_bins<<<grid_for(n_reads), 256, 0, st>>>(offs, n_reads, o.no_stage ? 0 : 1, flag1);
    TRY(hipGetLastError());
    r = prim_call(c, [&](void *tp, size_t &tb) { return prim::exclusive_sum(tp, tb, flag1, pos1, n_reads, st); });
    if (r) return r;
  }
  uint64_t total = 0, totw = 0, maxlen = 0, lastf = 0, lastp = 0;
  {
    uint64_t v[5] = {0, 0, 0, 0, 0};
    if (coop) FETCH({{offs + n_reads, 1}, {ctl + C_MAXLEN, 1}, {woff + n_reads, 1}, {flag1 + n_reads - 1, 0}, {pos1 + n_reads - 1, 0}}, v);
    else FETCH({{offs + n_reads, 1}, {ctl + C_MAXLEN, 1}}, v);
    total = v[0]; maxlen = v[1]; totw = v[2]; lastf = v[3]; lastp = v[4];
  }
  if (maxlen > MBW_MAX_READ) { mbw_set_error("read longer than 65535 bases"); return MBW_E_INVAL; }
  if (c->arena) c->arena_hint = ws_estimate(c, n_reads, total, !is_device_ptr(reads), o);
  // encode (plain kernel) or pack (wave kernels)
  const uint8_t *dreads = reads;
  if (!is_device_ptr(reads)) {
    GROW(c->ascii, total + 16);
    TRY(hipMemcpyAsync(c->ascii.p, reads, total, hipMemcpyHostToDevice, st));
    dreads = (const uint8_t *)c->ascii.p;
  }
  if (!coop) {   // the plain kernel reads one code per base
    GROW(c->codes, total + 16);
    k_encode<<<grid_for(total), 256, 0, st>>>(dreads, total, o.bs_role, (uint8_t *)c->codes.p);
    TRY(hipGetLastError());
  }
  ReadWords R;
  R.pw = nullptr; R.pn = nullptr; R.woff = nullptr;
  if (coop) {
    GROW(c->pwords, (totw + 2) * 8);
    GROW(c->pnmask, (totw + 2) * 4);
    GROW(c->wread, (totw + 2) * 4);
    k_word_owner<<<grid_for(n_reads), 256, 0, st>>>(woff, n_reads, (uint32_t *)c->wread.p);
    TRY(hipGetLastError());
    if (totw) {
      const uint64_t nblk = (totw + PACK_BLOCK - 1) / PACK_BLOCK;
      if (nblk > 0x7fffffffull) { mbw_set_error("batch too large"); return MBW_E_INVAL; }
      k_pack_words<<<(unsigned)nblk, PACK_BLOCK, 0, st>>>(dreads, total, offs, woff, (const uint32_t *)c->wread.p, totw,
                                                         o.bs_role, (uint64_t *)c->pwords.p, (uint32_t *)c->pnmask.p);
    }
    TRY(hipGetLastError());
    R.pw = (const uint64_t *)c->pwords.p;
    R.pn = (const uint32_t *)c->pnmask.p;
    R.woff = woff;
  }
  SeedParams P;
  memset(&P, 0, sizeof(P));
  P.codes = (const uint8_t *)c->codes.p; P.offs = offs; P.queries = nullptr; P.n_queries = n_reads;
  P.l = min_seed_len; P.c = o.min_occ; P.reseed = o.reseed; P.reseed_len = o.reseed_len; P.reseed_occ = o.reseed_occ;
  P.round = 1; P.use_kmer = o.use_kmer; P.ctl = ctl;
  {
    auto pow2 = [](int v) { return v > 0 && (v & (v - 1)) == 0; };
    auto lg = [](int v) { int t = 0; while ((1 << t) < v) ++t; return t; };
    P.uniq = (o.unique_ext && ix->text && ix->isa && pow2(ix->sa_sample) && pow2(ix->isa_sample)) ? 1 : 0;
    P.rmask = (uint32_t)(ix->sa_sample - 1);
    P.rshift = pow2(ix->sa_sample) ? lg(ix->sa_sample) : 0;
    P.rishift = pow2(ix->isa_sample) ? lg(ix->isa_sample) : 0;
  }
  // round-1 query records: reads that fit the LDS staging area first, then the others, longest first
  uint64_t nshort1 = 0, nlong1 = 0;
  const Query *q1 = nullptr;
  const uint32_t seg_len = o.seg_len > 0 ? (uint32_t)std::max(32, o.seg_len) : 256u;
  if (coop) {
    uint32_t *ids = (uint32_t *)c->bid0.p;
    nshort1 = lastp + lastf;
    const uint64_t nlong = n_reads - nshort1;
    k_read_partition<<<grid_for(n_reads), 256, 0, st>>>(offs, flag1, pos1, n_reads, nshort1, ids, (uint32_t *)c->bk0.p);
    TRY(hipGetLastError());
    const uint32_t *long_ids = ids + nshort1;
    if (nlong > 1) {
      prim::dbuf<uint32_t> bk((uint32_t *)c->bk0.p, (uint32_t *)c->bk1.p);
      prim::dbuf<uint32_t> bv(ids + nshort1, (uint32_t *)c->bid1.p);
      r = prim_call(c, [&](void *tp, size_t &tb) { return prim::sort_pairs(tp, tb, bk, bv, nlong, 0, 16, st); });
      if (r) return r;
      long_ids = bv.current();
    }
    Query *qq = (Query *)c->q1.p;
    if (nshort1)
      k_make_queries<<<grid_for(nshort1), 256, 0, st>>>(ids, nshort1, offs, R.woff, (uint32_t)min_seed_len, (uint32_t)o.min_occ, qq);
    if (nlong)
      k_make_queries<<<grid_for(nlong), 256, 0, st>>>(long_ids, nlong, offs, R.woff, (uint32_t)min_seed_len, (uint32_t)o.min_occ,
                                                      qq + nshort1);
    TRY(hipGetLastError());
    q1 = qq;
    r = segment_queries(c, qq + nshort1, nlong, seg_len, c->q1s, &nlong1, st);
    if (r) return r;
  }
  // Seed and sub-query buffers.  Every wave of a round-1 launch holds one output chunk of each at a
  // time, so up to one partly used chunk per wave and launch is left as slack.
  uint64_t chunk_slack = 0;
  if (coop)
    for (int b = 0; b < 2; ++b) {
      const uint64_t nqb = b == 0 ? nshort1 : nlong1;
      if (!nqb) continue;
      SeedParams Pg = P;
      Pg.n_queries = nqb;
      chunk_slack += (uint64_t)smem_grid(c, Pg, o, b == 0) * SMEM_WAVES * OUT_CHUNK;
    }
  // Deferred unique matches (staged reads, round 1), when asked for: every pass may leave partly
  // used output chunks (the first few passes carry nearly all the work)
  const bool defer = coop && P.uniq && nshort1 > 0 && o.unique_defer == 1;
  if (defer) chunk_slack += DEFER_SLACK_PASSES * defer_slack(c);
  uint64_t seed_cap = std::max<uint64_t>(1 << 16, n_reads * 6) + chunk_slack;
  if (c->raw.bytes / sizeof(SeedRec) > seed_cap) seed_cap = c->raw.bytes / sizeof(SeedRec);
  uint64_t subq_cap = std::max<uint64_t>(1 << 14, n_reads) + chunk_slack;
  if (c->subq.bytes / sizeof(Query) > subq_cap) subq_cap = c->subq.bytes / sizeof(Query);
  unsigned long long n1 = 0, nq = 0, stats1[3] = {0, 0, 0};
  for (int attempt = 0;; ++attempt) {
    GROW(c->raw, seed_cap * sizeof(SeedRec));
    GROW(c->subq, subq_cap * sizeof(Query));
    seed_cap = c->raw.bytes / sizeof(SeedRec);
    subq_cap = c->subq.bytes / sizeof(Query);
    P.seeds = (SeedRec *)c->raw.p; P.seed_cap = seed_cap; P.subq = (Query *)c->subq.p; P.subq_cap = subq_cap;
    TRY(hipMemsetAsync(ctl, 0, 8 * sizeof(unsigned long long), st));
    if (coop) r = run_binned(c, v, P, R, o, q1, nshort1, (const Query *)c->q1s.p, nlong1, st, defer);
    else r = run_smem(c, v, P, R, o, false, st);
    if (r) return r;
    {
      uint64_t v[5];
      FETCH({{ctl + C_NSEEDS, 1}, {ctl + C_NSUBQ, 1}, {ctl + C_LINES, 1}, {ctl + C_LINES + 1, 1}, {ctl + C_LINES + 2, 1}}, v);
      n1 = v[0]; nq = v[1]; stats1[0] = v[2]; stats1[1] = v[3]; stats1[2] = v[4];
    }
    if (n1 <= seed_cap && nq <= subq_cap) break;
    if (attempt > 3) { mbw_set_error("seed buffer did not converge"); return MBW_E_NOMEM; }
    seed_cap = std::max<uint64_t>(seed_cap, n1 + n1 / 2 + 1024);
    subq_cap = std::max<uint64_t>(subq_cap, nq + nq / 2 + 1024);
  }
  unsigned long long ntot = n1;
  // Slot counts include the unused tails of per-wave output chunks, which depend on scheduling; in
  // work space mode buffers sized by them take the (deterministic) slot capacity instead, so that a
  // call needs the same work space every time.
  const uint64_t nq_alloc = c->arena ? std::max<uint64_t>(nq, c->subq.bytes / sizeof(Query)) : nq;
  if (coop && o.reseed && nq > 0) {
    // round-2 queries by bin (unused chunk slots dropped)
    GROW(c->q2, (nq_alloc + 1) * sizeof(Query));
    GROW(c->bf0, (nq_alloc + 1) * 4); GROW(c->bf1, (nq_alloc + 1) * 4); GROW(c->bp0, (nq_alloc + 1) * 4);
    GROW(c->bp1, (nq_alloc + 1) * 4);
    uint32_t *fs = (uint32_t *)c->bf0.p, *fl = (uint32_t *)c->bf1.p, *ps = (uint32_t *)c->bp0.p, *pl = (uint32_t *)c->bp1.p;
    const Query *sq = (const Query *)c->subq.p;
    if (c->arena) {
      r = reserve_temp(c, [&](void *tp, size_t &tb) { return prim::exclusive_sum(tp, tb, fs, ps, nq_alloc, st); });
      if (r) return r;
    }
    k_query_bins<<<grid_for(nq), 256, 0, st>>>(sq, nq, o.no_stage ? 0 : 1, fs, fl);
    TRY(hipGetLastError());
    r = prim_call(c, [&](void *tp, size_t &tb) { return prim::exclusive_sum(tp, tb, fs, ps, nq, st); });
    if (r) return r;
    r = prim_call(c, [&](void *tp, size_t &tb) { return prim::exclusive_sum(tp, tb, fl, pl, nq, st); });
    if (r) return r;
    uint64_t tail[4] = {0, 0, 0, 0};
    FETCH({{fs + nq - 1, 0}, {ps + nq - 1, 0}, {fl + nq - 1, 0}, {pl + nq - 1, 0}}, tail);
    const uint64_t nshort2 = tail[0] + tail[1], nlong2 = tail[2] + tail[3];
    k_query_partition<<<grid_for(nq), 256, 0, st>>>(sq, fs, ps, fl, pl, nq, nshort2, (Query *)c->q2.p);
    TRY(hipGetLastError());
    uint64_t nlong2s = 0;
    r = segment_queries(c, (const Query *)c->q2.p + nshort2, nlong2, seg_len, c->q2s, &nlong2s, st);
    if (r) return r;
    SeedParams P2 = P;
    P2.round = 2;
    for (int attempt = 0;; ++attempt) {
      k_ctl_restore<<<1, 64, 0, st>>>(ctl, n1, stats1[0], stats1[1], stats1[2]);
      TRY(hipGetLastError());
      P2.seeds = (SeedRec *)c->raw.p; P2.seed_cap = c->raw.bytes / sizeof(SeedRec);
      r = run_binned(c, v, P2, R, o, (const Query *)c->q2.p, nshort2, (const Query *)c->q2s.p, nlong2s, st);
      if (r) return r;
      {
        uint64_t v[1];
        FETCH({{ctl + C_NSEEDS, 1}}, v);
        ntot = v[0];
      }
      if (ntot <= P2.seed_cap) break;
      if (attempt > 3) { mbw_set_error("seed buffer did not converge"); return MBW_E_NOMEM; }
      // keep the round-1 records: grow by copying
      mbw_ctx::Buf nb;
      int rr = grow(c, nb, (ntot + ntot / 2 + 1024) * sizeof(SeedRec));
      if (rr) return rr;
      TRY(hipMemcpyAsync(nb.p, c->raw.p, n1 * sizeof(SeedRec), hipMemcpyDeviceToDevice, st));
      release(c, c->raw, st);
      c->raw = nb;
    }
  }
  // sort by (read, qbeg, qend), dedup, counts
  const uint64_t ns = ntot;
  const uint64_t ns_alloc = c->arena ? std::max<uint64_t>(ns, c->raw.bytes / sizeof(SeedRec)) : ns;
  GROW(c->keys0, ns_alloc * 8); GROW(c->keys1, ns_alloc * 8); GROW(c->vals0, ns_alloc * 4); GROW(c->vals1, ns_alloc * 4);
  GROW(c->flag, ns_alloc * 4 + 8); GROW(c->idx, ns_alloc * 4 + 8);
  prim::dbuf<uint64_t> dk((uint64_t *)c->keys0.p, (uint64_t *)c->keys1.p);
  prim::dbuf<uint32_t> dv((uint32_t *)c->vals0.p, (uint32_t *)c->vals1.p);
  uint32_t *flag = (uint32_t *)c->flag.p, *idx = (uint32_t *)c->idx.p;
  uint64_t nu = 0;
  if (c->arena && ns) {   // temporary storage for the capacity, not the scheduling-dependent count
    r = reserve_temp(c, [&](void *tp, size_t &tb) {
      return prim::sort_pairs(tp, tb, dk, dv, ns_alloc, 0, 64, st);
    });
    if (r) return r;
    r = reserve_temp(c, [&](void *tp, size_t &tb) { return prim::exclusive_sum(tp, tb, flag, idx, ns_alloc, st); });
    if (r) return r;
  }
  if (ns) {
    int qb = 1;       // bits of an offset within a read (offsets run to the longest read's length)
    while ((1ull << qb) <= maxlen) ++qb;
    k_seed_keys<<<grid_for(ns), 256, 0, st>>>((const SeedRec *)c->raw.p, ns, n_reads, qb, (uint64_t *)c->keys0.p,
                                               (uint32_t *)c->vals0.p);
    TRY(hipGetLastError());
    int hibit = 2 * qb + 1;   // every key < (n_reads + 1) << 2 qb
    while (hibit < 64 && (1ull << (hibit - 2 * qb)) <= n_reads) ++hibit;
    if (ns > 1) {
      r = prim_call(c, [&](void *tp, size_t &tb) { return prim::sort_pairs(tp, tb, dk, dv, ns, 0, hibit, st); });
      if (r) return r;
    }
    k_dedup_mark<<<grid_for(ns), 256, 0, st>>>(dk.current(), ns, n_reads, qb, flag);
    TRY(hipGetLastError());
    r = prim_call(c, [&](void *tp, size_t &tb) { return prim::exclusive_sum(tp, tb, flag, idx, ns, st); });
    if (r) return r;
    uint64_t v[2];
    FETCH({{flag + ns - 1, 0}, {idx + ns - 1, 0}}, v);
    nu = v[1] + v[0];
  }
  mbw_seed_t *seeds;
  if (ob) {
    ob->seeds_needed = nu;
    if (nu > ob->seeds_cap) {
      mbw_set_error("seed buffer too small: " + std::to_string(nu) + " records needed, " + std::to_string(ob->seeds_cap) + " given");
      return MBW_E_CAPACITY;
    }
    seeds = ob->seeds;
  } else {
    GROW(c->seeds, (nu + 1) * sizeof(mbw_seed_t));
    seeds = (mbw_seed_t *)c->seeds.p;
  }
  GROW(c->npos, (nu + 2) * 8);
  GROW(c->posoff, (nu + 2) * 8);
  GROW(c->kpos, (nu + 1) * 8);
  uint64_t *npos = (uint64_t *)c->npos.p, *posoff = (uint64_t *)c->posoff.p;
  if (ns) {
    k_seed_emit<<<grid_for(ns), 256, 0, st>>>((const SeedRec *)c->raw.p, dv.current(), flag, idx, ns, (uint64_t)max_occ, seeds, npos,
                                              (uint64_t *)c->kpos.p);
    TRY(hipGetLastError());
  }
  uint64_t n_pos = 0;
  if (nu) {
    TRY(hipMemsetAsync(npos + nu, 0, 8, st));
    r = prim_call(c, [&](void *tp, size_t &tb) { return prim::exclusive_sum(tp, tb, npos, posoff, nu + 1, st); });
    if (r) return r;
    FETCH({{posoff + nu, 1}}, &n_pos);
    if (!coop || !n_pos) {   // the wave path stores the offsets while it expands the rows
      k_seed_posoff<<<grid_for(nu), 256, 0, st>>>(seeds, posoff, nu);
      TRY(hipGetLastError());
    }
  }
  // positions: straight into the caller's buffer unless a bisulfite filter follows
  uint64_t *posbuf;
  if (ob && !o.bs_role) {
    ob->pos_needed = n_pos;
    if (n_pos > ob->pos_cap) {
      mbw_set_error("position buffer too small: " + std::to_string(n_pos) + " needed, " + std::to_string(ob->pos_cap) + " given");
      return MBW_E_CAPACITY;
    }
    posbuf = ob->pos;
  } else {
    GROW(c->pos, (n_pos + 1) * 8);
    posbuf = (uint64_t *)c->pos.p;
  }
  // locate
  uint32_t rmask = (ix->sa_sample & (ix->sa_sample - 1)) == 0 ? (uint32_t)(ix->sa_sample - 1) : 0u;
  int rshift = -1;
  if ((ix->sa_sample & (ix->sa_sample - 1)) == 0) { rshift = 0; while ((1 << rshift) < ix->sa_sample) ++rshift; }
  TRY(hipEventRecord(c->ev[3], st));
  if (n_pos) {
    if (!coop) {
      TRY(hipEventRecord(c->ev[3], st));
      k_locate_plain<<<grid_for(nu), 256, 0, st>>>(v, seeds, nu, posbuf, rmask, rshift, ctl);
      TRY(hipGetLastError());
    } else {
      GROW(c->xrows, (n_pos + 1) * 8);
      k_expand_rows<<<grid_for((nu + 63) / 64 * 64 / 4, 256, 65536u), 256, 0, st>>>(seeds, posoff, (const uint64_t *)c->kpos.p,
                                                                                     nu, (uint64_t *)c->xrows.p, posbuf);
      TRY(hipGetLastError());
      const int grid = persistent_grid((const void *)k_locate_wave, 256, 0, c->n_cu, o.blocks_per_cu, n_pos, AUTO_ROWS_LOCATE,
                                     AUTO_LOCATE_MAX_PER_CU);
      TRY(hipEventRecord(c->ev[3], st));
      k_locate_wave<<<grid, 256, 0, st>>>(v, (const uint64_t *)c->xrows.p, n_pos, posbuf, rmask, rshift, ctl);
      TRY(hipGetLastError());
    }
  }
  TRY(hipEventRecord(c->ev[4], st));
  // bisulfite strand filter
  const uint64_t *final_pos = posbuf;
  if (o.bs_role && n_pos) {
    GROW(c->keep, (n_pos + 1) * 4);
    GROW(c->kidx, (n_pos + 1) * 8);
    uint32_t *keep = (uint32_t *)c->keep.p;
    uint64_t *kidx = (uint64_t *)c->kidx.p;
    k_bs_mark<<<grid_for(n_pos + 1), 256, 0, st>>>(posbuf, n_pos, ix->len_r, o.bs_role, keep);
    TRY(hipGetLastError());
    r = prim_call(c, [&](void *tp, size_t &tb) { return prim::exclusive_sum(tp, tb, keep, kidx, n_pos + 1, st); });
    if (r) return r;
    uint64_t kept = 0;
    FETCH({{kidx + n_pos, 1}}, &kept);
    uint64_t *dst;
    if (ob) {
      ob->pos_needed = kept;
      if (kept > ob->pos_cap) {
        mbw_set_error("position buffer too small: " + std::to_string(kept) + " needed, " + std::to_string(ob->pos_cap) + " given");
        return MBW_E_CAPACITY;
      }
      dst = ob->pos;
    } else {
      GROW(c->pos2, (kept + 1) * 8);
      dst = (uint64_t *)c->pos2.p;
    }
    k_bs_compact<<<grid_for(n_pos), 256, 0, st>>>(posbuf, keep, kidx, n_pos, dst);
    TRY(hipGetLastError());
    k_bs_seeds<<<grid_for(nu), 256, 0, st>>>(seeds, nu, kidx);
    TRY(hipGetLastError());
    n_pos = kept;
    final_pos = dst;
  } else if (ob && o.bs_role) {
    ob->pos_needed = 0;
  }
  // bisulfite refinement of every kept (seed, position) pair
  uint64_t n_pieces = 0;
  if (o.bs_refine && n_pos) {
    GROW(c->pseed, (n_pos + 1) * 4);
    GROW(c->pcnt, (n_pos + 1) * 4);
    GROW(c->ppoff, (n_pos + 1) * 8);
    uint32_t *ps = (uint32_t *)c->pseed.p, *pc = (uint32_t *)c->pcnt.p;
    uint64_t *po = (uint64_t *)c->ppoff.p;
    k_pos_seed<<<grid_for((nu + 63) / 64 * 64 / 4, 256, 65536u), 256, 0, st>>>(seeds, nu, ps);
    TRY(hipGetLastError());
    k_refine<<<grid_for(n_pos), 256, 0, st>>>(seeds, ps, final_pos, n_pos, dreads, offs, ix->orig, ix->len_r, o.bs_role,
                                              min_seed_len, pc, nullptr, nullptr);
    TRY(hipGetLastError());
    TRY(hipMemsetAsync(pc + n_pos, 0, 4, st));
    r = prim_call(c, [&](void *tp, size_t &tb) { return prim::exclusive_sum(tp, tb, pc, po, n_pos + 1, st); });
    if (r) return r;
    FETCH({{po + n_pos, 1}}, &n_pieces);
    mbw_piece_t *pdst;
    if (ob) {
      ob->pieces_needed = n_pieces;
      if (n_pieces > ob->pieces_cap) {
        mbw_set_error("piece buffer too small: " + std::to_string(n_pieces) + " needed, " + std::to_string(ob->pieces_cap) +
                      " given");
        return MBW_E_CAPACITY;
      }
      pdst = ob->pieces;
    } else {
      GROW(c->pieces, (n_pieces + 1) * sizeof(mbw_piece_t));
      pdst = (mbw_piece_t *)c->pieces.p;
    }
    if (n_pieces) {
      k_refine<<<grid_for(n_pos), 256, 0, st>>>(seeds, ps, final_pos, n_pos, dreads, offs, ix->orig, ix->len_r, o.bs_role,
                                                min_seed_len, pc, po, pdst);
      TRY(hipGetLastError());
    }
    out->pieces = pdst;
  }
  TRY(hipEventRecord(c->ev[5], st));
  {
    FetchList f;
    f.n = C_COUNT;
    for (int t = 0; t < C_COUNT; ++t) { f.p[t] = ctl + t; f.wide[t] = 1; }
    k_fetch<<<1, 64, 0, st>>>(f, c->dfetch);
    TRY(hipGetLastError());
    TRY(hipStreamSynchronize(st));
    for (int t = 0; t < C_COUNT; ++t) c->host_ctl[t] = ((volatile uint64_t *)c->hfetch)[t];
    r = flush_launch_times(c);
    if (r) return r;
  }
  if (c->host_ctl[C_ERR]) {
    mbw_set_error(std::string("kernel guard tripped (") + std::to_string(c->host_ctl[C_ERR]) + "): corrupt index or internal error");
    return MBW_E_HIP;
  }
  float t_loc = 0, t_tot = 0;
  (void)hipEventElapsedTime(&t_loc, c->ev[3], c->ev[4]);
  (void)hipEventElapsedTime(&t_tot, c->ev[0], c->ev[5]);
  out->n_seeds = nu;
  out->n_pos = n_pos;
  out->seeds = seeds;
  out->pos = final_pos;
  out->lines_smem = c->host_ctl[C_LINES];
  out->lines_locate = c->host_ctl[C_LINES_LOC];
  out->steps = c->host_ctl[C_STEPS];
  out->lf_steps = c->host_ctl[C_LFSTEPS];
  out->ms_smem = c->ms_smem;
  out->ms_locate = t_loc;
  out->ms_total = t_tot;
  out->n_smem_launches = c->n_smem_launches;
  out->wave_iters = c->host_ctl[C_WITER];
  out->lane_iters = c->host_ctl[C_LITER];
  out->max_chain = c->host_ctl[C_MAXCHAIN];
  out->n_pieces = n_pieces;
  if (!n_pieces) out->pieces = nullptr;
  if (ob) ob->workspace_needed = c->arena_need;
  if (trace_on())
    fprintf(stderr, "{\"mbw\": \"seed\", \"reads\": %llu, \"seeds\": %llu, \"positions\": %llu, \"pieces\": %llu, "
            "\"smem_launches\": %d, \"ms_smem\": %.3f, \"ms_locate\": %.3f, \"ms_total\": %.3f, \"lines_smem\": %llu, "
            "\"lines_locate\": %llu, \"wave_iters\": %llu, \"lane_iters\": %llu, \"max_chain\": %llu}\n",
            (unsigned long long)n_reads, (unsigned long long)nu, (unsigned long long)n_pos, (unsigned long long)n_pieces,
            out->n_smem_launches, out->ms_smem, out->ms_locate, out->ms_total, (unsigned long long)out->lines_smem,
            (unsigned long long)out->lines_locate, (unsigned long long)out->wave_iters, (unsigned long long)out->lane_iters,
            (unsigned long long)out->max_chain);
  return MBW_OK;
}

extern "C" int mbw_seed(mbw_ctx *c, const uint8_t *reads, const uint32_t *lengths, uint64_t n_reads, int min_seed_len,
                        int max_occ, const mbw_seed_opts *opts, void *stream, mbw_result *out) {
  return seed_impl(c, reads, lengths, n_reads, min_seed_len, max_occ, opts, stream, nullptr, out);
}

static void clear_needed(mbw_seed_buffers *b) {
  b->workspace_needed = b->seeds_needed = b->pos_needed = b->pieces_needed = 0;
}

extern "C" int mbw_seed_into(mbw_ctx *c, const uint8_t *reads, const uint32_t *lengths, uint64_t n_reads, int min_seed_len,
                             int max_occ, const mbw_seed_opts *opts, void *stream, mbw_seed_buffers *bufs, mbw_result *out) {
  if (!c || !bufs || !out) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  clear_needed(bufs);
  if (!bufs->workspace || ((uintptr_t)bufs->workspace & 255)) {
    mbw_set_error("the work space must be a device buffer aligned to 256 bytes"); return MBW_E_INVAL;
  }
  if ((bufs->seeds_cap && !bufs->seeds) || (bufs->pos_cap && !bufs->pos) || (bufs->pieces_cap && !bufs->pieces)) {
    mbw_set_error("a result buffer with a capacity but no pointer"); return MBW_E_INVAL;
  }
  TRY(hipSetDevice(c->device));
  ArenaScope scope(c, bufs->workspace, bufs->workspace_bytes);
  const int r = seed_impl(c, reads, lengths, n_reads, min_seed_len, max_occ, opts, stream, bufs, out);
  bufs->workspace_needed = c->arena_need;   // also when the call stopped part way
  return r;
}

// ---------------------------------------------------------------------------------------------
// Allocation-free seeding: the work space of mbw_seed_into becomes a file-scope device array of
// MBW_SCRATCH_BYTES.  Each GPU that the library runs on holds its own copy until the process ends;
// its device address is looked up once per device when a context is created on it (host code uses
// that address, never the array's name).  Calls that overlap on one GPU share the array and race.
#define MBW_SCRATCH_BYTES (128ull << 20)
static __device__ __align__(256) uint8_t scratch[MBW_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[64];

// with `device` current
static int scratch_init(int device) {
  if (device < 0 || device >= 64) { mbw_set_error("device ordinal out of range for the scratch table"); return MBW_E_INVAL; }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return MBW_OK;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    mbw_set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    return MBW_E_HIP;
  }
  g_scratch_ptr[device] = ptr;
  return MBW_OK;
}

extern "C" int mbw_seed_static(mbw_ctx *c, const uint8_t *reads, const uint32_t *lengths, uint64_t n_reads, int min_seed_len,
                               int max_occ, const mbw_seed_opts *opts, void *stream, mbw_seed_buffers *bufs, mbw_result *out) {
  if (!c || !bufs || !out) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  clear_needed(bufs);
  if (n_reads && (!reads || !lengths || !is_device_ptr(reads) || !is_device_ptr(lengths))) {
    mbw_set_error("mbw_seed_static takes reads and lengths in device memory"); return MBW_E_INVAL;
  }
  if ((bufs->seeds_cap && !bufs->seeds) || (bufs->pos_cap && !bufs->pos) || (bufs->pieces_cap && !bufs->pieces)) {
    mbw_set_error("a result buffer with a capacity but no pointer"); return MBW_E_INVAL;
  }
  TRY(hipSetDevice(c->device));
  void *ws = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    ws = (c->device >= 0 && c->device < 64) ? g_scratch_ptr[c->device] : nullptr;
  }
  if (!ws) { mbw_set_error("no scratch address for this device (context not created through mbw_ctx_create)"); return MBW_E_HIP; }
  int r;
  {
    ArenaScope scope(c, ws, MBW_SCRATCH_BYTES);
    r = seed_impl(c, reads, lengths, n_reads, min_seed_len, max_occ, opts, stream, bufs, out);
    bufs->workspace_needed = c->arena_need;
  }
  if (r == MBW_E_CAPACITY && bufs->workspace_needed > MBW_SCRATCH_BYTES)
    mbw_set_error("batch too large for the allocation-free entry point: it needs at least " +
                  std::to_string(bufs->workspace_needed) + " bytes of work space, the static array holds " +
                  std::to_string(MBW_SCRATCH_BYTES) + " (use mbw_seed_into with a larger work space)");
  return r;
}

extern "C" int mbw_result_download_pieces(mbw_ctx *c, const mbw_result *res, mbw_piece_t *pieces) {
  if (!c || !res) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  TRY(hipSetDevice(c->device));
  if (pieces && res->n_pieces)
    TRY(hipMemcpyAsync(pieces, res->pieces, res->n_pieces * sizeof(mbw_piece_t), hipMemcpyDeviceToHost, c->cur));
  TRY(hipStreamSynchronize(c->cur));
  return MBW_OK;
}

// ---------------------------------------------------------------------------------------------
// autotuner: every candidate schedule gives the same seeds; each is run once to size the buffers
// and once timed (device time of the whole call), and the fastest wins
extern "C" int mbw_tune(mbw_ctx *c, const uint8_t *reads, const uint32_t *lengths, uint64_t n_reads, int min_seed_len,
                        int max_occ, const mbw_seed_opts *base, void *stream, mbw_seed_opts *best, float *best_ms) {
  if (!c || !best || !best_ms) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  mbw_seed_opts b;
  if (base) b = *base;
  else {
    memset(&b, 0, sizeof(b));
    b.min_occ = 1; b.reseed = 1; b.reseed_len = 38; b.reseed_occ = 10; b.use_kmer = 1; b.unique_ext = 1;
  }
  b.kernel = MBW_KERNEL_COOP;
  const int stage_opts[2] = {0, 1};            // no_stage
  const int seg_opts[3] = {128, 256, 1024};
  const int bpc_opts[3] = {0, -1, 2};         // sized by the work, occupancy limit, 2
  const int uniq_opts[2] = {1, 0};
  float bt = 0;
  bool have = false;
  for (int u = 0; u < 2; ++u)
    for (int ns = 0; ns < 2; ++ns)
      for (int sg = 0; sg < 3; ++sg)
        for (int bp = 0; bp < 3; ++bp) {
          mbw_seed_opts o = b;
          o.unique_ext = uniq_opts[u]; o.no_stage = stage_opts[ns]; o.seg_len = seg_opts[sg]; o.blocks_per_cu = bpc_opts[bp];
          mbw_result res;
          int r = mbw_seed(c, reads, lengths, n_reads, min_seed_len, max_occ, &o, stream, &res);
          if (r) return r;
          r = mbw_seed(c, reads, lengths, n_reads, min_seed_len, max_occ, &o, stream, &res);
          if (r) return r;
          if (!have || res.ms_total < bt) { bt = res.ms_total; *best = o; have = true; }
        }
  // then the reads each wave takes from the work queue at a time, with the rest of the best schedule
  const int chunk_opts[3] = {16, 64, 256};
  const mbw_seed_opts grid_best = *best;
  for (int ch = 0; ch < 3; ++ch) {
    mbw_seed_opts o = grid_best;
    o.wave_chunk = chunk_opts[ch];
    mbw_result res;
    int r = mbw_seed(c, reads, lengths, n_reads, min_seed_len, max_occ, &o, stream, &res);
    if (r) return r;
    r = mbw_seed(c, reads, lengths, n_reads, min_seed_len, max_occ, &o, stream, &res);
    if (r) return r;
    if (res.ms_total < bt) { bt = res.ms_total; *best = o; }
  }
  *best_ms = bt;
  return MBW_OK;
}

extern "C" int mbw_result_download(mbw_ctx *c, const mbw_result *res, mbw_seed_t *seeds, uint64_t *pos) {
  if (!c || !res) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  TRY(hipSetDevice(c->device));
  // on the stream of the call that produced the result (a null-stream copy would wait for every stream)
  if (seeds && res->n_seeds)
    TRY(hipMemcpyAsync(seeds, res->seeds, res->n_seeds * sizeof(mbw_seed_t), hipMemcpyDeviceToHost, c->cur));
  if (pos && res->n_pos) TRY(hipMemcpyAsync(pos, res->pos, res->n_pos * sizeof(uint64_t), hipMemcpyDeviceToHost, c->cur));
  TRY(hipStreamSynchronize(c->cur));
  return MBW_OK;
}

// ---------------------------------------------------------------------------------------------
// Captured graphs (mbw_graph_*).  The seeding path of a batch of reads that fit the LDS staging area
// is recorded once as a HIP graph over buffers sized by a plan (reads, bases, seeds, sub-queries and
// positions at most) and replayed for every batch.  Nothing in it needs the host: every count the
// eager path waits for (bases, packed words, seeds, sub-queries, unique seeds, positions) stays on
// the device, the kernels that consume one read it there, and grids, sorts and scans span the
// plan's capacities (unused slots sort last and hold nothing).  The host copies the batch in,
// launches the graph and waits once, for the counts, which it checks against the plan.  The graph
// records no memset operation: clearing is done by kernels, and the sorts take rocPRIM's
// merge-based path, whose resets are kernels too.
namespace {

// zero the control block and the lengths of the plan's unused reads (the replayed batch may be
// smaller than the plan), and the flag past the last seed slot (the unique-seed scan reads it)
__global__ void k_graph_prep(uint32_t *__restrict__ lens, uint64_t N, const uint64_t *__restrict__ nreads,
                             unsigned long long *__restrict__ ctl, uint32_t *__restrict__ flag_end) {
  const uint64_t n = *nreads;
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < N; t += (uint64_t)gridDim.x * blockDim.x)
    if (t >= n) lens[t] = 0;
  if (blockIdx.x == 0) {
    if (threadIdx.x < C_COUNT) ctl[threadIdx.x] = 0;
    if (threadIdx.x == 0) *flag_end = 0;
  }
}

// Length bins with the counts on the device.  Reads: flag 1 for those staged in LDS (the plan's
// unused reads have length 0 and count as staged); fs[N] = 0 so that a scan over N + 1 ends in the
// count.
__global__ void k_graph_rflags(const uint64_t *__restrict__ offs, uint64_t N, uint64_t *__restrict__ fs) {
  for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r <= N; r += (uint64_t)gridDim.x * blockDim.x)
    fs[r] = (r < N && offs[r + 1] - offs[r] <= STAGE_MAX) ? 1u : 0u;
}
// staged read ids in order; the others with sort keys that put the longest first (slots past the
// last of them keep the filler key, which sorts after every length); nlong = N - staged
__global__ void k_graph_rsplit(const uint64_t *__restrict__ offs, uint64_t N, const uint64_t *__restrict__ fs,
                               const uint64_t *__restrict__ ps, uint32_t *__restrict__ ids_s, uint32_t *__restrict__ lkey,
                               uint32_t *__restrict__ lid, uint64_t *__restrict__ nlong) {
  for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r < N; r += (uint64_t)gridDim.x * blockDim.x) {
    if (fs[r]) ids_s[ps[r]] = (uint32_t)r;
    else {
      const uint64_t t = r - ps[r];
      lid[t] = (uint32_t)r;
      lkey[t] = 65535u - (uint32_t)(offs[r + 1] - offs[r]);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *nlong = N - ps[N];
}
// Re-seeding queries that round 1 wrote (its list has unused slots of per-wave chunks, and nothing
// past the count on the device), flagged by bin; [n] = 0
__global__ void k_graph_qflags(const Query *__restrict__ q, uint64_t n, const unsigned long long *__restrict__ count,
                               uint64_t *__restrict__ fs, uint64_t *__restrict__ fl) {
  const uint64_t m = min(n, (uint64_t)*count);
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t <= n; t += (uint64_t)gridDim.x * blockDim.x) {
    const bool valid = t < m && q[t].read_id != INVALID_READ;
    const bool sh = valid && q[t].rlen <= STAGE_MAX;
    fs[t] = (valid && sh) ? 1u : 0u;
    fl[t] = (valid && !sh) ? 1u : 0u;
  }
}
// ... moved to the front of their bin's list, in order
__global__ void k_graph_qsplit(const Query *__restrict__ q, const uint64_t *__restrict__ fs, const uint64_t *__restrict__ ps,
                               const uint64_t *__restrict__ fl, const uint64_t *__restrict__ pl, uint64_t n,
                               Query *__restrict__ qs, Query *__restrict__ ql) {
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < n; t += (uint64_t)gridDim.x * blockDim.x) {
    if (fs[t]) qs[ps[t]] = q[t];
    else if (fl[t]) ql[pl[t]] = q[t];
  }
}
// segments of the first *count queries (as k_seg_count / k_seg_write); [n] = 0; segments at or past
// cap are not written (the host reports the shortfall from the count)
__global__ void k_graph_segcount(const Query *__restrict__ q, uint64_t n, const uint64_t *__restrict__ count, uint32_t seg,
                                 uint64_t *__restrict__ cnt) {
  const uint64_t m = min(n, *count);
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t <= n; t += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t k = 0;
    if (t < m) {
      const uint32_t len = q[t].qend > q[t].qbeg ? q[t].qend - q[t].qbeg : 0u;
      k = len > seg ? (len + seg - 1) / seg : 1u;
    }
    cnt[t] = k;
  }
}
__global__ void k_graph_segwrite(const Query *__restrict__ q, uint64_t n, const uint64_t *__restrict__ count, uint32_t seg,
                                 const uint64_t *__restrict__ cnt, const uint64_t *__restrict__ off, uint64_t cap,
                                 Query *__restrict__ out) {
  const uint64_t m = min(n, *count);
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < m; t += (uint64_t)gridDim.x * blockDim.x) {
    const Query x = q[t];
    const uint64_t k = cnt[t];
    for (uint64_t g = 0; g < k && off[t] + g < cap; ++g) {
      Query y = x;
      y.qbeg = x.qbeg + (uint32_t)g * seg;
      y.send = g + 1 < k ? y.qbeg + seg : x.send;
      y.flags = g > 0 ? (x.flags | SEG_CHECK) : x.flags;
      out[off[t] + g] = y;
    }
  }
}
__global__ void k_fill_u32(uint32_t *__restrict__ p, uint64_t n, uint32_t v) {
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < n; t += (uint64_t)gridDim.x * blockDim.x) p[t] = v;
}

__global__ void k_fill_u64(uint64_t *__restrict__ p, uint64_t n, uint64_t v) {
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < n; t += (uint64_t)gridDim.x * blockDim.x) p[t] = v;
}

// the counts the host checks after a replay, into pinned host memory: the control block, the
// unique seeds and the positions
__global__ void k_graph_counts(const unsigned long long *__restrict__ ctl, const uint32_t *__restrict__ nu,
                               const uint64_t *__restrict__ npos, uint64_t *__restrict__ out,
                               const uint64_t *__restrict__ seg1, const uint64_t *__restrict__ seg2,
                               const uint64_t *__restrict__ kept, const uint64_t *__restrict__ pieces) {
  const int t = threadIdx.x;
  if (t < C_COUNT) out[t] = ctl[t];
  if (t == C_COUNT) out[t] = *nu;
  if (t == C_COUNT + 1) out[t] = *npos;
  if (t == C_COUNT + 2) out[t] = seg1 ? *seg1 : 0;   // segments of the long reads and of their sub-queries
  if (t == C_COUNT + 3) out[t] = seg2 ? *seg2 : 0;
  if (t == C_COUNT + 4) out[t] = kept ? *kept : 0;       // bisulfite: positions kept by the strand filter
  if (t == C_COUNT + 5) out[t] = pieces ? *pieces : 0;   // ... and refined pieces
  __threadfence_system();
}

}  // namespace

struct mbw_graph {
  mbw_ctx *ctx = nullptr;
  const mbw_index *ix = nullptr;    // kept alive while the graph exists (its kernels read it)
  int device = 0;
  uint64_t N = 0, B = 0, L = 0, W = 0, S = 0, Q = 0, X = 0, QS1 = 0, QS2 = 0, PC = 0;
  int reseed = 0, launches = 0, bs_role = 0, refine = 0;
  uint64_t *pos_kept = nullptr;     // bisulfite: the positions the strand filter keeps
  mbw_piece_t *pieces = nullptr;
  const uint64_t *seg_counts[2] = {nullptr, nullptr};
  std::vector<void *> dev;          // device allocations
  uint8_t *reads = nullptr;
  uint32_t *lens = nullptr;
  uint64_t *nreads = nullptr;
  mbw_seed_t *seeds = nullptr;
  uint64_t *pos = nullptr;
  uint64_t *hio = nullptr, *dio = nullptr;   // pinned host words: [0] read count in; counts out from [1]
  uint32_t *hlens = nullptr;        // pinned host copy of a batch's lengths given on the device
  hipStream_t cs = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

static void graph_destroy(mbw_graph *g) {
  if (!g) return;
  (void)hipSetDevice(g->device);
  if (g->cs) (void)hipStreamSynchronize(g->cs);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  for (void *p : g->dev) (void)hipFree(p);
  if (g->hio) (void)hipHostFree(g->hio);
  if (g->hlens) (void)hipHostFree(g->hlens);
  if (g->ev0) (void)hipEventDestroy(g->ev0);
  if (g->ev1) (void)hipEventDestroy(g->ev1);
  if (g->cs) (void)hipStreamDestroy(g->cs);
  if (g->ix) mbw_index_release(g->ix);
  delete g;
}

// one device allocation of the graph
template <class T>
static int graph_alloc(mbw_graph *g, T *&p, uint64_t count) {
  void *q = nullptr;
  if (hipMalloc(&q, std::max<uint64_t>(count, 1) * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    mbw_set_error("graph: device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed");
    return MBW_E_NOMEM;
  }
  g->dev.push_back(q);
  p = (T *)q;
  return 0;
}
#define GALLOC(p, n) do { int r_ = graph_alloc(g, p, n); if (r_) { graph_destroy(g); return r_; } } while (0)
#define GTRY(call) do { hipError_t e_ = (call); if (e_ != hipSuccess) {                              \
    mbw_set_error(std::string("graph: ") + #call + ": " + hipGetErrorString(e_));                   \
    hipGraph_t dummy_ = nullptr; if (capturing) (void)hipStreamEndCapture(g->cs, &dummy_);           \
    if (dummy_) (void)hipGraphDestroy(dummy_);                                                        \
    graph_destroy(g); return e_ == hipErrorOutOfMemory ? MBW_E_NOMEM : MBW_E_HIP; } } while (0)

extern "C" int mbw_graph_create(mbw_ctx *c, const mbw_graph_plan *plan, int min_seed_len, int max_occ,
                                const mbw_seed_opts *opts, mbw_graph **out) {
  if (!c || !plan || !out) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  *out = nullptr;
  if (min_seed_len < 1 || max_occ < 1) { mbw_set_error("min_seed_len and max_occ must be >= 1"); return MBW_E_INVAL; }
  mbw_seed_opts o;
  if (opts) o = *opts;
  else {
    memset(&o, 0, sizeof(o));
    o.min_occ = 1; o.reseed = 1; o.reseed_len = 38; o.reseed_occ = 10; o.use_kmer = 1; o.unique_ext = 1;
  }
  if (o.min_occ < 1) { mbw_set_error("min_occ must be >= 1"); return MBW_E_INVAL; }
  if (o.kernel != MBW_KERNEL_COOP || o.no_stage || o.unique_defer) {
    mbw_set_error("graph: the wave kernels with LDS staging only (no plain kernel, no_stage or unique_defer)");
    return MBW_E_INVAL;
  }
  if (o.bs_role < 0 || o.bs_role > 2) { mbw_set_error("bs_role must be 0, 1 or 2"); return MBW_E_INVAL; }
  if (o.bs_role && !c->ix->bisulfite) { mbw_set_error("bs_role needs a bisulfite index"); return MBW_E_INVAL; }
  if (o.bs_refine && (!o.bs_role || !c->ix->orig)) {
    mbw_set_error("bs_refine needs bs_role and a bisulfite index"); return MBW_E_INVAL;
  }
  if (o.wave_chunk < 0 || o.wave_chunk > WORK_CHUNK) { mbw_set_error("wave_chunk must be in [0,256]"); return MBW_E_INVAL; }
  const uint64_t N = plan->max_reads;
  if (N < 1 || N >= (1ull << 31)) { mbw_set_error("graph: max_reads must be in [1, 2^31)"); return MBW_E_INVAL; }
  const uint64_t L = plan->max_read_len ? plan->max_read_len : STAGE_MAX;
  if (L > MBW_MAX_READ) { mbw_set_error("graph: max_read_len above 65535"); return MBW_E_INVAL; }
  const uint64_t B = plan->max_bases ? plan->max_bases : N * L;
  if (B > N * L) { mbw_set_error("graph: max_bases above max_reads x max_read_len"); return MBW_E_INVAL; }
  const bool binned = L > STAGE_MAX;          // reads too long for LDS staging: the unstaged bin, in segments
  const uint32_t seg = o.seg_len > 0 ? (uint32_t)std::max(32, o.seg_len) : 256u;
  TRY(hipSetDevice(c->device));
  const mbw_index *ix = c->ix;
  const IndexView v = make_view(ix);
  mbw_graph *g = new mbw_graph;
  g->ctx = c;
  g->device = c->device;
  g->ix = ix;
  mbw_index_retain(ix);
  g->N = N; g->B = B; g->L = L;
  g->W = B / 32 + N + 2;                      // packed words: each read adds at most one partial word
  g->reseed = o.reseed;
  // seeding parameters, as the eager path sets them
  SeedParams P;
  memset(&P, 0, sizeof(P));
  P.l = min_seed_len; P.c = o.min_occ; P.reseed = o.reseed; P.reseed_len = o.reseed_len; P.reseed_occ = o.reseed_occ;
  P.round = 1; P.use_kmer = o.use_kmer;
  {
    auto pow2 = [](int x) { return x > 0 && (x & (x - 1)) == 0; };
    auto lg = [](int x) { int t = 0; while ((1 << t) < x) ++t; return t; };
    P.uniq = (o.unique_ext && ix->text && ix->isa && pow2(ix->sa_sample) && pow2(ix->isa_sample)) ? 1 : 0;
    P.rmask = (uint32_t)(ix->sa_sample - 1);
    P.rshift = pow2(ix->sa_sample) ? lg(ix->sa_sample) : 0;
    P.rishift = pow2(ix->isa_sample) ? lg(ix->isa_sample) : 0;
  }
  // capacities and grids.  Every launch that writes seeds or re-seeding queries leaves at most one
  // partly used output chunk per wave, which the seed and sub-query capacities add.
  const uint64_t QS1 = binned ? B / seg + N + 1 : 0;   // segments of the long reads
  SeedParams P1s = P, P1l = P;
  P1s.n_queries = N;
  P1l.n_queries = QS1;
  const int g1s = P.uniq ? wave_grid<true, true>(c, P1s, o) : wave_grid<true, false>(c, P1s, o);
  const int g1l = binned ? (P.uniq ? wave_grid<false, true>(c, P1l, o) : wave_grid<false, false>(c, P1l, o)) : 0;
  const uint64_t slack1 = (uint64_t)(g1s + g1l) * SMEM_WAVES * OUT_CHUNK;
  g->Q = (plan->max_subqueries ? plan->max_subqueries : 2 * N) + slack1;
  const uint64_t Q = g->Q;
  const uint64_t QS2 = binned ? Q + 4 * (B / seg) + 1 : 0;   // segments of the long reads' sub-queries
  SeedParams P2s = P, P2l = P;
  P2s.round = P2l.round = 2; P2s.uniq = P2l.uniq = 0;
  P2s.n_queries = Q;
  P2l.n_queries = QS2;
  const int g2s = wave_grid<true, false>(c, P2s, o);
  const int g2l = binned ? wave_grid<false, false>(c, P2l, o) : 0;
  g->S = (plan->max_seeds ? plan->max_seeds : 8 * N) + slack1 + (o.reseed ? (uint64_t)(g2s + g2l) * SMEM_WAVES * OUT_CHUNK : 0);
  g->X = plan->max_positions ? plan->max_positions : 64 * N;
  g->QS1 = QS1; g->QS2 = QS2;
  g->bs_role = o.bs_role; g->refine = o.bs_refine;
  g->PC = o.bs_refine ? (plan->max_pieces ? plan->max_pieces : g->X) : 0;
  if (g->S >= (1ull << 32) - 2) { mbw_set_error("graph: too many seeds for one plan"); graph_destroy(g); return MBW_E_INVAL; }
  const uint64_t S = g->S, X = g->X, W = g->W;
  // device buffers
  uint64_t *wide, *offs, *nwords, *woff, *pw, *keys0, *keys1, *npos, *posoff, *kpos, *xrows;
  uint64_t *f2s, *p2s, *f2l, *p2l;
  uint32_t *wread, *pn, *vals0, *vals1, *flag, *idx;
  Query *q1, *subq, *q2s;
  SeedRec *raw;
  unsigned long long *ctl;
  GALLOC(g->reads, B + 64);
  GALLOC(g->lens, N + 1);
  GALLOC(g->nreads, 1);
  GALLOC(wide, N + 1); GALLOC(offs, N + 1); GALLOC(nwords, N + 1); GALLOC(woff, N + 1);
  GALLOC(wread, W); GALLOC(pw, W + 2); GALLOC(pn, W + 2);
  GALLOC(q1, N); GALLOC(raw, S); GALLOC(subq, Q); GALLOC(q2s, Q);
  GALLOC(f2s, Q + 1); GALLOC(p2s, Q + 1); GALLOC(f2l, Q + 1); GALLOC(p2l, Q + 1);
  GALLOC(keys0, S); GALLOC(keys1, S); GALLOC(vals0, S); GALLOC(vals1, S); GALLOC(flag, S + 1); GALLOC(idx, S + 1);
  GALLOC(g->seeds, S); GALLOC(npos, S + 1); GALLOC(posoff, S + 1); GALLOC(kpos, S + 1);
  GALLOC(xrows, X + 1); GALLOC(g->pos, X + 1);
  GALLOC(ctl, C_COUNT);
  // the unstaged bin
  uint64_t *fs1 = nullptr, *ps1 = nullptr, *nlong = nullptr, *c1 = nullptr, *o1 = nullptr, *c2 = nullptr, *o2 = nullptr;
  uint32_t *ids_s = nullptr, *lk0 = nullptr, *lk1 = nullptr, *li0 = nullptr, *li1 = nullptr;
  Query *ql = nullptr, *q1seg = nullptr, *q2l = nullptr, *q2seg = nullptr;
  if (binned) {
    GALLOC(fs1, N + 1); GALLOC(ps1, N + 1); GALLOC(nlong, 1);
    GALLOC(ids_s, N); GALLOC(lk0, N); GALLOC(lk1, N); GALLOC(li0, N); GALLOC(li1, N);
    GALLOC(ql, N); GALLOC(c1, N + 1); GALLOC(o1, N + 1); GALLOC(q1seg, QS1);
    GALLOC(q2l, Q); GALLOC(c2, Q + 1); GALLOC(o2, Q + 1); GALLOC(q2seg, QS2);
  }
  // bisulfite strand filter and refinement
  uint32_t *keep = nullptr, *ps = nullptr, *pc = nullptr;
  uint64_t *kidx = nullptr, *po = nullptr;
  const uint64_t PC = g->PC;
  if (o.bs_role) { GALLOC(keep, X + 1); GALLOC(kidx, X + 1); GALLOC(g->pos_kept, X + 1); }
  if (o.bs_refine) { GALLOC(ps, X + 1); GALLOC(pc, X + 1); GALLOC(po, X + 1); GALLOC(g->pieces, PC); }
  g->seg_counts[0] = o1 ? o1 + N : nullptr;
  g->seg_counts[1] = o2 ? o2 + Q : nullptr;
  bool capturing = false;
  GTRY(hipMemset(xrows, 0xff, (X + 1) * sizeof(uint64_t)));   // every row starts as NO_POS
  if (hipHostMalloc((void **)&g->hio, 64 * sizeof(uint64_t), hipHostMallocCoherent) != hipSuccess ||
      hipHostGetDevicePointer((void **)&g->dio, g->hio, 0) != hipSuccess) {
    (void)hipGetLastError();
    mbw_set_error("graph: pinned host allocation failed");
    graph_destroy(g);
    return MBW_E_NOMEM;
  }
  int qb = 1;                                   // bits of an offset within a read of at most L bases
  while ((1ull << qb) <= L) ++qb;
  int hibit = 2 * qb + 1;
  while (hibit < 64 && (1ull << (hibit - 2 * qb)) <= N) ++hibit;
  // temporary storage: the largest any sort or scan of the graph asks for
  prim::dbuf<uint64_t> dk(keys0, keys1);
  prim::dbuf<uint32_t> dv(vals0, vals1);
  prim::dbuf<uint32_t> dlk(lk0, lk1), dli(li0, li1);
  size_t tb = 0, t1 = 0;
  GTRY(prim::exclusive_sum((void *)nullptr, t1, wide, offs, N + 1, (hipStream_t)0)); tb = std::max(tb, t1);
  GTRY(prim::sort_pairs_merge((void *)nullptr, t1, dk, dv, S, 0, hibit, (hipStream_t)0)); tb = std::max(tb, t1);
  GTRY(prim::exclusive_sum((void *)nullptr, t1, flag, idx, S + 1, (hipStream_t)0)); tb = std::max(tb, t1);
  GTRY(prim::exclusive_sum((void *)nullptr, t1, npos, posoff, S + 1, (hipStream_t)0)); tb = std::max(tb, t1);
  GTRY(prim::exclusive_sum((void *)nullptr, t1, f2s, p2s, Q + 1, (hipStream_t)0)); tb = std::max(tb, t1);
  if (binned) {
    GTRY(prim::sort_pairs_merge((void *)nullptr, t1, dlk, dli, N, 0, 17, (hipStream_t)0)); tb = std::max(tb, t1);
  }
  if (o.bs_role) { GTRY(prim::exclusive_sum((void *)nullptr, t1, keep, kidx, X + 1, (hipStream_t)0)); tb = std::max(tb, t1); }
  if (o.bs_refine) { GTRY(prim::exclusive_sum((void *)nullptr, t1, pc, po, X + 1, (hipStream_t)0)); tb = std::max(tb, t1); }
  uint8_t *temp;
  GALLOC(temp, tb + 256);
  GTRY(hipStreamCreateWithFlags(&g->cs, hipStreamNonBlocking));
  GTRY(hipEventCreate(&g->ev0));
  GTRY(hipEventCreate(&g->ev1));
  ReadWords R;
  R.pw = pw; R.pn = pn; R.woff = woff;
  for (SeedParams *pp : {&P1s, &P1l}) {
    pp->seeds = raw; pp->seed_cap = S; pp->subq = subq; pp->subq_cap = Q; pp->ctl = ctl;
  }
  for (SeedParams *pp : {&P2s, &P2l}) {
    pp->seeds = raw; pp->seed_cap = S; pp->subq = nullptr; pp->subq_cap = 0; pp->ctl = ctl;
  }
  P1s.queries = q1; P1s.nq_dev = binned ? (const unsigned long long *)(ps1 + N) : nullptr;
  P1l.queries = q1seg; P1l.nq_dev = binned ? (const unsigned long long *)(o1 + N) : nullptr;
  P2s.queries = q2s; P2s.nq_dev = (const unsigned long long *)(p2s + Q);
  P2l.queries = q2seg; P2l.nq_dev = binned ? (const unsigned long long *)(o2 + Q) : nullptr;
  auto chunk_for = [&](int grid, uint64_t n) {
    if (o.wave_chunk > 0) return (uint32_t)std::min(WORK_CHUNK, o.wave_chunk);
    const uint64_t waves = (uint64_t)std::max(grid, 1) * SMEM_WAVES;
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(WORK_CHUNK, n / (waves * 8)));
  };
  // expected counts (the plan's reads, about 1.5 sub-queries per read) set the automatic takes
  P1s.chunk = chunk_for(g1s, N);
  P1l.chunk = chunk_for(g1l, B / seg);
  P2s.chunk = chunk_for(g2s, 2 * N);
  P2l.chunk = chunk_for(g2l, B / seg);
  uint32_t rmask = (ix->sa_sample & (ix->sa_sample - 1)) == 0 ? (uint32_t)(ix->sa_sample - 1) : 0u;
  int rshift = -1;
  if ((ix->sa_sample & (ix->sa_sample - 1)) == 0) { rshift = 0; while ((1 << rshift) < ix->sa_sample) ++rshift; }
  const int gridL = persistent_grid((const void *)k_locate_wave, 256, 0, c->n_cu, o.blocks_per_cu, X, AUTO_ROWS_LOCATE,
                                     AUTO_LOCATE_MAX_PER_CU);
  const int bs = 64 * SMEM_WAVES;
  hipStream_t st = g->cs;
  GTRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  capturing = true;
  size_t have = tb + 256;
  // lengths -> offsets, packed words (as the eager path)
  k_graph_prep<<<grid_for(N), 256, 0, st>>>(g->lens, N, g->nreads, ctl, flag + S);
  k_widen<<<grid_for(N + 1, 256, 1024u), 256, 0, st>>>(g->lens, N, wide, ctl + C_MAXLEN);
  GTRY(prim::exclusive_sum((void *)temp, have, wide, offs, N + 1, st));
  k_read_words<<<grid_for(N + 1), 256, 0, st>>>(offs, N, nwords);
  have = tb + 256;
  GTRY(prim::exclusive_sum((void *)temp, have, nwords, woff, N + 1, st));
  k_word_owner<<<grid_for(N), 256, 0, st>>>(woff, N, wread);
  k_pack_words<<<(unsigned)((W + PACK_BLOCK - 1) / PACK_BLOCK), PACK_BLOCK, 0, st>>>(g->reads, B, offs, woff, wread, W,
                                                                                       o.bs_role, pw, pn, offs + N, woff + N);
  // round 1: the staged bin in read order, the other reads longest first and in segments
  if (!binned) {
    k_make_queries<<<grid_for(N), 256, 0, st>>>(nullptr, N, offs, woff, (uint32_t)min_seed_len, (uint32_t)o.min_occ, q1);
  } else {
    k_graph_rflags<<<grid_for(N + 1), 256, 0, st>>>(offs, N, fs1);
    have = tb + 256;
    GTRY(prim::exclusive_sum((void *)temp, have, fs1, ps1, N + 1, st));
    k_fill_u32<<<grid_for(N), 256, 0, st>>>(lk0, N, 0x10000u);
    k_graph_rsplit<<<grid_for(N), 256, 0, st>>>(offs, N, fs1, ps1, ids_s, lk0, li0, nlong);
    have = tb + 256;
    GTRY(prim::sort_pairs_merge((void *)temp, have, dlk, dli, N, 0, 17, st));
    k_make_queries<<<grid_for(N), 256, 0, st>>>(ids_s, N, offs, woff, (uint32_t)min_seed_len, (uint32_t)o.min_occ, q1,
                                                ps1 + N);
    k_make_queries<<<grid_for(N), 256, 0, st>>>(dli.current(), N, offs, woff, (uint32_t)min_seed_len, (uint32_t)o.min_occ,
                                                ql, nlong);
    k_graph_segcount<<<grid_for(N + 1), 256, 0, st>>>(ql, N, nlong, seg, c1);
    have = tb + 256;
    GTRY(prim::exclusive_sum((void *)temp, have, c1, o1, N + 1, st));
    k_graph_segwrite<<<grid_for(N), 256, 0, st>>>(ql, N, nlong, seg, c1, o1, QS1, q1seg);
  }
  k_ctl_zero<<<1, 64, 0, st>>>(ctl, C_WORK, C_WORK);
  if (P.uniq) k_smem_wave<true, true><<<g1s, bs, 0, st>>>(v, P1s, R);
  else k_smem_wave<true, false><<<g1s, bs, 0, st>>>(v, P1s, R);
  g->launches = 1;
  if (binned) {
    k_ctl_zero<<<1, 64, 0, st>>>(ctl, C_WORK, C_WORK);
    if (P.uniq) k_smem_wave<false, true><<<g1l, bs, 0, st>>>(v, P1l, R);
    else k_smem_wave<false, false><<<g1l, bs, 0, st>>>(v, P1l, R);
    ++g->launches;
  }
  // round 2: the re-seeding queries by bin, compacted, the long ones in segments
  if (o.reseed) {
    k_graph_qflags<<<grid_for(Q + 1), 256, 0, st>>>(subq, Q, ctl + C_NSUBQ, f2s, f2l);
    have = tb + 256;
    GTRY(prim::exclusive_sum((void *)temp, have, f2s, p2s, Q + 1, st));
    have = tb + 256;
    GTRY(prim::exclusive_sum((void *)temp, have, f2l, p2l, Q + 1, st));
    k_graph_qsplit<<<grid_for(Q), 256, 0, st>>>(subq, f2s, p2s, f2l, p2l, Q, q2s, binned ? q2l : q2s);
    k_ctl_zero<<<1, 64, 0, st>>>(ctl, C_WORK, C_WORK);
    k_smem_wave<true, false><<<g2s, bs, 0, st>>>(v, P2s, R);
    ++g->launches;
    if (binned) {
      k_graph_segcount<<<grid_for(Q + 1), 256, 0, st>>>(q2l, Q, p2l + Q, seg, c2);
      have = tb + 256;
      GTRY(prim::exclusive_sum((void *)temp, have, c2, o2, Q + 1, st));
      k_graph_segwrite<<<grid_for(Q), 256, 0, st>>>(q2l, Q, p2l + Q, seg, c2, o2, QS2, q2seg);
      k_ctl_zero<<<1, 64, 0, st>>>(ctl, C_WORK, C_WORK);
      k_smem_wave<false, false><<<g2l, bs, 0, st>>>(v, P2l, R);
      ++g->launches;
    }
  }
  // sort by (read, qbeg, qend), dedup, counts, rows, locate (as the eager path, over capacities)
  k_seed_keys<<<grid_for(S), 256, 0, st>>>(raw, S, N, qb, keys0, vals0, ctl + C_NSEEDS);
  have = tb + 256;
  GTRY(prim::sort_pairs_merge((void *)temp, have, dk, dv, S, 0, hibit, st));
  k_dedup_mark<<<grid_for(S), 256, 0, st>>>(dk.current(), S, N, qb, flag);
  have = tb + 256;
  GTRY(prim::exclusive_sum((void *)temp, have, flag, idx, S + 1, st));
  k_fill_u64<<<grid_for(S + 1), 256, 0, st>>>(npos, S + 1, 0);
  k_seed_emit<<<grid_for(S), 256, 0, st>>>(raw, dv.current(), flag, idx, S, (uint64_t)max_occ, g->seeds, npos, kpos);
  have = tb + 256;
  GTRY(prim::exclusive_sum((void *)temp, have, npos, posoff, S + 1, st));
  k_expand_rows<<<grid_for((S + 63) / 64 * 64 / 4, 256, 65536u), 256, 0, st>>>(g->seeds, posoff, kpos, S, xrows, g->pos,
                                                                                 idx + S, X);
  k_locate_wave<<<gridL, 256, 0, st>>>(v, xrows, X, g->pos, rmask, rshift, ctl, posoff + S);
  // bisulfite: the strand filter on the positions, then the refinement of every kept pair (as the
  // eager path, over the position capacity)
  if (o.bs_role) {
    k_bs_mark<<<grid_for(X + 1), 256, 0, st>>>(g->pos, X, ix->len_r, o.bs_role, keep, posoff + S);
    have = tb + 256;
    GTRY(prim::exclusive_sum((void *)temp, have, keep, kidx, X + 1, st));
    k_bs_compact<<<grid_for(X), 256, 0, st>>>(g->pos, keep, kidx, X, g->pos_kept);
    k_bs_seeds<<<grid_for(S), 256, 0, st>>>(g->seeds, S, kidx, idx + S, X);
  }
  if (o.bs_refine) {
    k_pos_seed<<<grid_for((S + 63) / 64 * 64 / 4, 256, 65536u), 256, 0, st>>>(g->seeds, S, ps, idx + S, X);
    k_fill_u32<<<grid_for(X + 1), 256, 0, st>>>(pc, X + 1, 0u);
    k_refine<<<grid_for(X), 256, 0, st>>>(g->seeds, ps, g->pos_kept, X, g->reads, offs, ix->orig, ix->len_r, o.bs_role,
                                          min_seed_len, pc, nullptr, nullptr, kidx + X);
    have = tb + 256;
    GTRY(prim::exclusive_sum((void *)temp, have, pc, po, X + 1, st));
    k_refine<<<grid_for(X), 256, 0, st>>>(g->seeds, ps, g->pos_kept, X, g->reads, offs, ix->orig, ix->len_r, o.bs_role,
                                          min_seed_len, pc, po, g->pieces, kidx + X, PC);
  }
  k_graph_counts<<<1, 64, 0, st>>>(ctl, idx + S, posoff + S, g->dio + 1, g->seg_counts[0], g->seg_counts[1],
                                   o.bs_role ? kidx + X : nullptr, o.bs_refine ? po + X : nullptr);
  GTRY(hipGetLastError());
  capturing = false;
  GTRY(hipStreamEndCapture(st, &g->graph));
  GTRY(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
  *out = g;
  return MBW_OK;
}
#undef GALLOC

extern "C" int mbw_graph_info(const mbw_graph *g, mbw_graph_plan *plan) {
  if (!g || !plan) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  memset(plan, 0, sizeof(*plan));
  plan->max_reads = g->N; plan->max_bases = g->B; plan->max_seeds = g->S; plan->max_subqueries = g->Q;
  plan->max_positions = g->X; plan->max_read_len = g->L; plan->max_pieces = g->PC;
  return MBW_OK;
}

extern "C" int mbw_graph_seed(mbw_graph *g, const uint8_t *reads, const uint32_t *lengths, uint64_t n_reads, void *stream,
                              mbw_result *out) {
  if (!g || !out) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  memset(out, 0, sizeof(*out));
  if (n_reads > g->N) { mbw_set_error("graph: " + std::to_string(n_reads) + " reads, the plan holds " + std::to_string(g->N)); return MBW_E_INVAL; }
  if (n_reads > 0 && (!reads || !lengths)) { mbw_set_error("NULL reads or lengths"); return MBW_E_INVAL; }
  TRY(hipSetDevice(g->device));
  hipStream_t st = (hipStream_t)stream;
  g->ctx->cur = st;
  // the lengths on the host, checked against the plan before anything reaches the graph
  const uint32_t *hl = lengths;
  if (n_reads && is_device_ptr(lengths)) {
    if (!g->hlens && hipHostMalloc((void **)&g->hlens, g->N * sizeof(uint32_t), 0) != hipSuccess) {
      (void)hipGetLastError();
      g->hlens = nullptr;
      mbw_set_error("graph: pinned host allocation failed");
      return MBW_E_NOMEM;
    }
    TRY(hipMemcpyAsync(g->hlens, lengths, n_reads * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    TRY(hipStreamSynchronize(st));
    hl = g->hlens;
  }
  uint64_t total = 0;
  for (uint64_t r = 0; r < n_reads; ++r) {
    if (hl[r] > g->L) {
      mbw_set_error("graph: read " + std::to_string(r) + " has " + std::to_string(hl[r]) + " bases, the plan's reads at most " +
                    std::to_string(g->L));
      return MBW_E_INVAL;
    }
    total += hl[r];
  }
  if (total > g->B) {
    mbw_set_error("graph: " + std::to_string(total) + " bases, the plan holds " + std::to_string(g->B));
    return MBW_E_INVAL;
  }
  // the batch into the graph's input buffers, its read count into the device word the graph reads
  if (n_reads) {
    TRY(hipMemcpyAsync(g->lens, lengths, n_reads * sizeof(uint32_t), hipMemcpyDefault, st));
    if (total) TRY(hipMemcpyAsync(g->reads, reads, total, hipMemcpyDefault, st));
  }
  g->hio[0] = n_reads;
  TRY(hipMemcpyAsync(g->nreads, g->hio, sizeof(uint64_t), hipMemcpyHostToDevice, st));
  TRY(hipEventRecord(g->ev0, st));
  TRY(hipGraphLaunch(g->exec, st));
  TRY(hipEventRecord(g->ev1, st));
  TRY(hipStreamSynchronize(st));
  uint64_t cnt[C_COUNT + 6];
  for (int t = 0; t < C_COUNT + 6; ++t) cnt[t] = ((volatile uint64_t *)g->hio)[1 + t];
  if (cnt[C_ERR]) {
    mbw_set_error("kernel guard tripped (" + std::to_string(cnt[C_ERR]) + "): corrupt index or internal error");
    return MBW_E_HIP;
  }
  const uint64_t nu = cnt[C_COUNT], n_pos = cnt[C_COUNT + 1];
  if (cnt[C_NSEEDS] > g->S || cnt[C_NSUBQ] > g->Q || n_pos > g->X || cnt[C_COUNT + 2] > g->QS1 || cnt[C_COUNT + 3] > g->QS2) {
    mbw_set_error("graph: the batch needs " + std::to_string(cnt[C_NSEEDS]) + " seed slots, " + std::to_string(cnt[C_NSUBQ]) +
                  " sub-query slots, " + std::to_string(n_pos) + " positions and " + std::to_string(cnt[C_COUNT + 2]) + " + " +
                  std::to_string(cnt[C_COUNT + 3]) + " segments; the plan holds " + std::to_string(g->S) + ", " +
                  std::to_string(g->Q) + ", " + std::to_string(g->X) + " and " + std::to_string(g->QS1) + " + " +
                  std::to_string(g->QS2) + " (seed it with mbw_seed, or use a larger plan)");
    return MBW_E_CAPACITY;
  }
  if (g->refine && cnt[C_COUNT + 5] > g->PC) {
    mbw_set_error("graph: the batch needs " + std::to_string(cnt[C_COUNT + 5]) + " refined pieces; the plan holds " +
                  std::to_string(g->PC) + " (seed it with mbw_seed, or use a larger plan)");
    return MBW_E_CAPACITY;
  }
  float ms = 0;
  (void)hipEventElapsedTime(&ms, g->ev0, g->ev1);
  out->n_seeds = nu;
  out->n_pos = g->bs_role ? cnt[C_COUNT + 4] : n_pos;
  out->seeds = g->seeds;
  out->pos = g->bs_role ? g->pos_kept : g->pos;
  out->n_pieces = g->refine ? cnt[C_COUNT + 5] : 0;
  out->pieces = g->refine ? g->pieces : nullptr;
  out->lines_smem = cnt[C_LINES];
  out->lines_locate = cnt[C_LINES_LOC];
  out->steps = cnt[C_STEPS];
  out->lf_steps = cnt[C_LFSTEPS];
  out->ms_total = ms;
  out->n_smem_launches = g->launches;
  out->wave_iters = cnt[C_WITER];
  out->lane_iters = cnt[C_LITER];
  out->max_chain = cnt[C_MAXCHAIN];
  return MBW_OK;
}

extern "C" void mbw_graph_free(mbw_graph *g) { graph_destroy(g); }
