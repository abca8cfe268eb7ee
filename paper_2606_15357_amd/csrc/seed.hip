// Batched (l,c)-SMEM seeding and sampled-SA locate (paper Sections 2.1, 2.4, 2.5, 2.6, 2.9).
//
// Pipeline of one mbw_seed call (all on one stream):
//   encode      ASCII -> codes 0..3 (4 = matches nothing), bisulfite read conversion (Section 2.9)
//   smem        round 1: (l,c)-SMEMs of every read (Algorithm 3), appended to a seed list; SMEMs that
//               qualify for re-seeding are appended to a sub-query list
//   smem        round 2 (Section 2.6): (floor(len/2), s+1)-SMEMs of each sub-query
//   sort/dedup  seeds sorted by (read, qbeg, qend); duplicates from overlapping parents dropped
//   scan        per-seed position counts (s <= max_occ) -> offsets
//   locate      Algorithm 2: LF-walk every SA row of every located seed to a sampled row
//   filter      bisulfite strand filter on positions (Section 2.9)
//
// Two kernel families do the smem and locate steps:
//   * cooperative (default): persistent work queues; eight lanes hold one query (or one locate walk)
//     and fetch each 128-byte occurrence line with a single 16-byte load per lane; the read is staged
//     in LDS; the first k backward steps of a run come from the k-mer table (Section 2.5).
//   * plain (baseline): one thread runs the serial algorithm for one read (round 2 inline), one
//     thread locates one seed; ranks read the line header and the needed 16-byte slices.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "mbw_internal.h"
#include "../../include/mbw.h"

#define TRY(call) MBW_HIP_TRY(call)

namespace {

struct Query { uint32_t read_id, qbeg, qend, l, c; };
#define INVALID_READ 0xFFFFFFFFu   // unused slot of a per-wave output chunk
struct SeedRec { uint32_t read_id, qbeg, qend, flags; uint64_t k, kr, s; };

// control block (device): counters shared by the kernels of one call
enum { C_WORK = 0, C_NSEEDS = 1, C_NSUBQ = 2, C_LINES = 3, C_STEPS = 4, C_KMER = 5, C_LFSTEPS = 6, C_SAREADS = 7,
       C_LINES_LOC = 8, C_WORK2 = 9, C_MAXLEN = 10, C_ERR = 11, C_COUNT = 16 };

struct SeedParams {
  const uint8_t *__restrict__ codes;
  const uint64_t *__restrict__ offs;
  const Query *__restrict__ queries;   // round 2; nullptr in round 1
  uint64_t n_queries;
  int l, c;                            // round 1 parameters
  int reseed, reseed_len, reseed_occ, round;
  int use_kmer, grab;
  SeedRec *__restrict__ seeds;
  uint64_t seed_cap;
  Query *__restrict__ subq;
  uint64_t subq_cap;
  unsigned long long *__restrict__ ctl;
};

// Append one seed (and, in round 1, its re-seeding query) from whatever lanes are active here:
// one atomic per group of simultaneously emitting lanes.
__device__ __forceinline__ uint64_t active_slot(unsigned long long *counter) {
  const uint64_t m = __ballot(1);
  const int lane = (int)(threadIdx.x & 63);
  const int leader = __ffsll((unsigned long long)m) - 1;
  unsigned long long b0 = 0;
  if (lane == leader) b0 = atomicAdd(counter, (unsigned long long)__popcll(m));
  b0 = __shfl(b0, leader);
  return b0 + __popcll(m & ((1ull << lane) - 1));
}

__device__ __forceinline__ void emit_seed(const SeedParams &P, uint32_t read_id, int i, int j, uint64_t k, uint64_t kr,
                                          uint64_t s) {
  const uint64_t slot = active_slot(&P.ctl[C_NSEEDS]);
  if (slot < P.seed_cap) {
    SeedRec r;
    r.read_id = read_id; r.qbeg = (uint32_t)i; r.qend = (uint32_t)j; r.flags = P.round == 2 ? MBW_SEED_ROUND2 : 0u;
    r.k = k; r.kr = kr; r.s = s;
    P.seeds[slot] = r;
  }
  if (P.round == 1 && P.reseed && j - i >= P.reseed_len && s <= (uint64_t)P.reseed_occ) {
    const uint64_t qs = active_slot(&P.ctl[C_NSUBQ]);
    if (qs < P.subq_cap) {
      Query q; q.read_id = read_id; q.qbeg = (uint32_t)i; q.qend = (uint32_t)j; q.l = (uint32_t)((j - i) / 2);
      q.c = (uint32_t)(s + 1);
      P.subq[qs] = q;
    }
  }
}

__device__ __forceinline__ void load_query(const SeedParams &P, uint64_t qi, uint32_t &read_id, uint32_t &qbeg,
                                           uint32_t &qend, uint32_t &l, uint32_t &c) {
  if (P.queries) {
    Query q = P.queries[qi];
    read_id = q.read_id; qbeg = q.qbeg; qend = q.qend; l = q.l; c = q.c;
  } else {
    read_id = (uint32_t)qi; qbeg = 0; qend = (uint32_t)(P.offs[qi + 1] - P.offs[qi]); l = (uint32_t)P.l; c = (uint32_t)P.c;
  }
}

// ---------------------------------------------------------------------------------------------
// encode
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
  atomicMax(maxlen, (unsigned long long)mx);
}

// ---------------------------------------------------------------------------------------------
// cooperative SMEM kernel (Algorithm 3 per 8-lane group; persistent work queue)
//
// Each group holds one query's record (u, i, j, (k, k', s)) in registers (all eight lanes hold the
// same values) and advances it by one memory action per iteration: a k-mer table lookup, a
// backward step or a forward step.  Stage changes that need no memory are taken in between.
enum { ACT_DONE = 0, ACT_KMER = 1, ACT_BWD = 2, ACT_FWD = 3 };

template <int SLOT>
__global__ void __launch_bounds__(256) k_smem_coop(IndexView ix, SeedParams P) {
  extern __shared__ uint8_t lds[];
  const int q = threadIdx.x & (MBW_GROUP - 1);
  uint8_t *slot = lds + (threadIdx.x / MBW_GROUP) * (SLOT > 0 ? SLOT : 1);
  const uint8_t *rb = nullptr;
  uint32_t read_id = 0, qbeg = 0, qend = 0, l = 0, c = 1;
  int u = 0, i = 0, j = 0;
  uint64_t k = 0, kr = 0, s = 0;
  bool fresh = false, active = false;
  uint64_t n_lines = 0, n_steps = 0, n_kmer = 0;
  uint64_t qnext = 0, qlast = 0;
  uint64_t budget = 0;   // iterations left for the current query (guards against a runaway state)
  const int K = (P.use_kmer && ix.kmer) ? ix.K : 0;

  auto base_at = [&](int p) -> int {
    if (SLOT > 0) return slot[p - (int)qbeg];
    return rb[p];
  };

  for (;;) {
    if (!active) {
      if (qnext >= qlast) {
        unsigned long long b0 = 0;
        if (q == 0) b0 = atomicAdd(&P.ctl[C_WORK], (unsigned long long)P.grab);
        b0 = __shfl(b0, 0, MBW_GROUP);
        if (b0 >= P.n_queries) break;
        qnext = b0;
        qlast = b0 + (uint64_t)P.grab < P.n_queries ? b0 + (uint64_t)P.grab : P.n_queries;
      }
      uint64_t qi = qnext++;
      load_query(P, qi, read_id, qbeg, qend, l, c);
      if (read_id == INVALID_READ || !(l >= 1 && l - 1 < qend - qbeg)) continue;   // Algorithm 3 queues a string only if l-1 < |P|
      rb = P.codes + P.offs[read_id];
      if (SLOT > 0) {
        int len = (int)(qend - qbeg);
        for (int t = q; t < len; t += MBW_GROUP) slot[t] = rb[qbeg + t];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      }
      u = 1; i = (int)qbeg; j = (int)(qbeg + l - 1);
      k = 0; kr = 0; s = ix.n; fresh = true; active = true;
      budget = 8ull * (qend - qbeg) * (qend - qbeg) + 64;
    }
    if (--budget == 0) {
      if (q == 0) atomicOr(&P.ctl[C_ERR], 1ull);
      active = false;
      continue;
    }
    // ---- stage transitions without memory traffic
    int act = ACT_DONE;
    int a = 0;
    uint32_t code = 0;
    for (;;) {
      if (u == 2) {
        if (j == (int)qend) {                         // reached the end of P: report the SMEM
          if (q == 0) emit_seed(P, read_id, i, j, k, kr, s);
          act = ACT_DONE; break;
        }
        a = base_at(j);
        if (a > 3) {                                  // forward extension fails on a non-ACGT base
          if (q == 0) emit_seed(P, read_id, i, j, k, kr, s);
          u = 3; k = 0; kr = 0; s = ix.n; fresh = true;
          continue;
        }
        act = ACT_FWD; break;
      }
      if (u == 1 && j < i) { u = 2; j = i + (int)l; fresh = false; continue; }
      if (u == 3 && j <= i) { u = 1; i = j + 1; j = j + (int)l; k = 0; kr = 0; s = ix.n; fresh = true; continue; }
      if (fresh && K > 0 && j - K + 1 >= (u == 1 ? i : i + 1)) {
        bool ok = true;
        code = 0;
        for (int t = j - K + 1; t <= j; ++t) { int b = base_at(t); ok = ok && b < 4; code = code * 4 + (uint32_t)(b & 3); }
        fresh = false;
        if (ok) { act = ACT_KMER; break; }
      }
      fresh = false;
      a = base_at(j);
      if (a > 3) {                                     // BackStep fails on a non-ACGT base
        if (j + (int)l < (int)qend) { u = 1; i = j + 1; j = j + (int)l; k = 0; kr = 0; s = ix.n; fresh = true; continue; }
        act = ACT_DONE; break;
      }
      act = ACT_BWD; break;
    }
    if (act == ACT_DONE) { active = false; continue; }
    if (act == ACT_KMER) {
      uint4 e = ix.kmer[code];
      uint64_t ek, ekr, es;
      kmer_unpack(e, ek, ekr, es);
      ++n_kmer;
      if (es >= c) { k = ek; kr = ekr; s = es; j -= K; }
      continue;
    }
    // ---- one extension step (Algorithm 1), one or two lines
    const bool bwd = act == ACT_BWD;
    const uint64_t x = bwd ? k : kr, y = bwd ? kr : k;
    const int cc = bwd ? a : 3 - a;
    const uint64_t x2 = x + s;
    const uint64_t L1 = line_of(x), L2 = line_of(x2);
    uint4 d1 = ix.lines[L1 * MBW_LINE_U4 + q];
    uint4 d2 = d1;
    if (L2 != L1) d2 = ix.lines[L2 * MBW_LINE_U4 + q];
    n_lines += (L2 != L1) ? 2 : 1;
    ++n_steps;
    uint64_t E1, G1, E2, G2;
    slice_eg(d1, q, (int)(x - L1 * MBW_BPL), cc, E1, G1);
    slice_eg(d2, q, (int)(x2 - L2 * MBW_BPL), cc, E2, G2);
    uint64_t sE1 = grp_sum64(E1);
    uint64_t dE = grp_sum64(E2 - E1);
    uint64_t dG = grp_sum64(G2 - G1);
    if (cc == 0) {                      // the $ row is stored as A
      uint64_t c1 = x > ix.primary ? 1 : 0, c2 = x2 > ix.primary ? 1 : 0;
      sE1 -= c1;
      dE -= c2 - c1;
    }
    const uint64_t dol = (x <= ix.primary && ix.primary < x2) ? 1 : 0;
    const uint64_t ns = dE;
    const uint64_t nx = sel4(ix.Cb[0], ix.Cb[1], ix.Cb[2], ix.Cb[3], cc) + sE1;
    const uint64_t ny = y + dol + dG;
    if (ns >= c) {
      if (bwd) { k = nx; kr = ny; s = ns; j -= 1; }
      else { kr = nx; k = ny; s = ns; j += 1; }
      continue;
    }
    if (bwd) {                                        // BackStep failure: jump past j
      if (j + (int)l < (int)qend) { u = 1; i = j + 1; j = j + (int)l; k = 0; kr = 0; s = ix.n; fresh = true; }
      else active = false;
    } else {                                          // forward failure: report, then stage 3 from j
      if (q == 0) emit_seed(P, read_id, i, j, k, kr, s);
      u = 3; k = 0; kr = 0; s = ix.n; fresh = true;
    }
  }
  if (q == 0) {
    atomicAdd(&P.ctl[C_LINES], (unsigned long long)(n_lines + n_kmer));
    atomicAdd(&P.ctl[C_STEPS], (unsigned long long)n_steps);
    atomicAdd(&P.ctl[C_KMER], (unsigned long long)n_kmer);
  }
}

// ---------------------------------------------------------------------------------------------
// Wave-cooperative fetch (default schedule): every lane owns one query (or one locate walk).  Each
// step the wave gathers the lines its lanes need with eight 16-byte loads per lane: in load t, the
// eight lanes 8g..8g+7 fetch the eight slices of the line wanted by lane 8t+g, so one instruction
// moves eight whole 128-byte lines.  The slices land in LDS (8 KB per wave, rotated by lane to
// spread banks) and each lane then ranks its own line without any cross-lane reduction.
#define WAVE_U4 (64 * MBW_LINE_U4)

__device__ __forceinline__ int slot_of(int r, int j) { return r * MBW_LINE_U4 + ((j + r) & 7); }

#define WF_LOAD(t)                                                                             \
  {                                                                                            \
    const int src = 8 * (t) + (lane >> 3);                                                     \
    const uint32_t Ls = (uint32_t)__shfl((int)myL, src);                                       \
    if (__shfl((int)myneed, src)) d##t = lines[(uint64_t)Ls * MBW_LINE_U4 + (lane & 7)];       \
  }
#define WF_STORE(t) buf[slot_of(8 * (t) + (lane >> 3), lane & 7)] = d##t;

// Slices of lanes that need nothing are stored too (stale data in slots nobody reads).
__device__ __forceinline__ void wave_fetch(const uint4 *__restrict__ lines, uint32_t myL, bool myneed, uint4 *buf, int lane) {
  uint4 d0 = make_uint4(0, 0, 0, 0), d1 = d0, d2 = d0, d3 = d0, d4 = d0, d5 = d0, d6 = d0, d7 = d0;
  WF_LOAD(0) WF_LOAD(1) WF_LOAD(2) WF_LOAD(3) WF_LOAD(4) WF_LOAD(5) WF_LOAD(6) WF_LOAD(7)
  WF_STORE(0) WF_STORE(1) WF_STORE(2) WF_STORE(3) WF_STORE(4) WF_STORE(5) WF_STORE(6) WF_STORE(7)
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint64_t pmask(int m) { return m >= 32 ? M55 : (((1ull << (2 * (m < 0 ? 0 : m))) - 1) & M55); }
__device__ __forceinline__ uint64_t eq_bits(uint64_t w, int c) {
  uint64_t hi = (w >> 1) & M55, lo = w & M55;
  return c == 0 ? (~(hi | lo) & M55) : (c == 1 ? (~hi & lo) : (c == 2 ? (hi & ~lo) : (hi & lo)));
}
__device__ __forceinline__ uint64_t gt_bits(uint64_t w, int c) {
  uint64_t hi = (w >> 1) & M55, lo = w & M55;
  return c == 0 ? (hi | lo) : (c == 1 ? hi : (c == 2 ? (hi & lo) : 0ull));
}

// Occ(c, .) (E) and sum_{d>c} Occ(d, .) (G) at offsets o1 and o2 (o2 < 0: not needed) of the line
// staged for this lane; $ not corrected.
__device__ __forceinline__ void lane_eg(const uint4 *buf, int lane, int c, int o1, int o2, uint64_t &E1, uint64_t &G1,
                                        uint64_t &E2, uint64_t &G2) {
  const uint4 h0 = buf[slot_of(lane, 0)], h1 = buf[slot_of(lane, 1)];
  const uint64_t cA = ((uint64_t)h0.y << 32) | h0.x, cC = ((uint64_t)h0.w << 32) | h0.z;
  const uint64_t cG = ((uint64_t)h1.y << 32) | h1.x, cT = ((uint64_t)h1.w << 32) | h1.z;
  const uint64_t he = sel4(cA, cC, cG, cT, c);
  const uint64_t hg = (c < 1 ? cC : 0) + (c < 2 ? cG : 0) + (c < 3 ? cT : 0);
  uint32_t e1 = 0, g1 = 0, e2 = 0, g2 = 0;
  const int omax = o1 > o2 ? o1 : o2;
#pragma unroll
  for (int sl = 2; sl < 8; ++sl) {
    const int base = (sl - 2) * 64;
    if (base < omax) {
      const uint4 d = buf[slot_of(lane, sl)];
      const uint64_t w0 = ((uint64_t)d.y << 32) | d.x, w1 = ((uint64_t)d.w << 32) | d.z;
      const uint64_t ea = eq_bits(w0, c), eb = eq_bits(w1, c), ga = gt_bits(w0, c), gb = gt_bits(w1, c);
      const int m1 = o1 - base, m2 = o2 - base;
      const uint64_t p1a = pmask(m1), p1b = pmask(m1 - 32), p2a = pmask(m2), p2b = pmask(m2 - 32);
      e1 += __popcll(ea & p1a) + __popcll(eb & p1b);
      g1 += __popcll(ga & p1a) + __popcll(gb & p1b);
      e2 += __popcll(ea & p2a) + __popcll(eb & p2b);
      g2 += __popcll(ga & p2a) + __popcll(gb & p2b);
    }
  }
  E1 = he + e1; G1 = hg + g1; E2 = he + e2; G2 = hg + g2;
}

struct Emit { uint32_t i, j; uint64_t k, kr, s; };

// Work and output are handed out in chunks per wave so that hot counters see one atomic per chunk
// (device-scope atomics on a single address serialise).  All 64 lanes must call these together.
#define WORK_CHUNK 256
#define OUT_CHUNK 256

// Give each lane with `want` the next item of the wave's current chunk (grabbing new chunks as
// needed); returns the item or ~0 when the queue is exhausted.
__device__ __forceinline__ uint64_t wave_take(bool want, uint64_t &cb, uint64_t &ce, unsigned long long *counter,
                                              uint64_t total, int lane) {
  uint64_t m = __ballot(want);
  uint64_t res = ~0ull;
  const uint64_t below = (1ull << lane) - 1;
  while (m) {
    if (cb >= ce) {
      unsigned long long b0 = 0;
      if (lane == 0) b0 = atomicAdd(counter, (unsigned long long)WORK_CHUNK);
      b0 = __shfl(b0, 0);
      if (b0 >= total) { cb = ce = total; break; }
      cb = b0;
      ce = b0 + WORK_CHUNK < total ? b0 + WORK_CHUNK : total;
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
// Slots past `cap` are reported as ~0 (the host grows the buffer and runs again).
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

struct WaveOut { uint64_t sb, se, qb, qe; };

__device__ __forceinline__ void wave_emit(const SeedParams &P, int lane, bool em, uint32_t read_id, const Emit &e, WaveOut &wo) {
  if (!__ballot(em)) return;
  const uint64_t slot = wave_slot(em, wo.sb, wo.se, &P.ctl[C_NSEEDS], lane);
  if (em && slot < P.seed_cap) {
    SeedRec r;
    r.read_id = read_id; r.qbeg = e.i; r.qend = e.j; r.flags = P.round == 2 ? MBW_SEED_ROUND2 : 0u;
    r.k = e.k; r.kr = e.kr; r.s = e.s;
    P.seeds[slot] = r;
  }
  const bool rq = em && P.round == 1 && P.reseed && (int)(e.j - e.i) >= P.reseed_len && e.s <= (uint64_t)P.reseed_occ;
  if (!__ballot(rq)) return;
  const uint64_t qs = wave_slot(rq, wo.qb, wo.qe, &P.ctl[C_NSUBQ], lane);
  if (rq && qs < P.subq_cap) {
    Query q; q.read_id = read_id; q.qbeg = e.i; q.qend = e.j; q.l = (e.j - e.i) / 2; q.c = (uint32_t)(e.s + 1);
    P.subq[qs] = q;
  }
}

// mark the unused tail of the wave's output chunks invalid
__device__ __forceinline__ void wave_close(const SeedParams &P, int lane, const WaveOut &wo) {
  for (uint64_t t = wo.sb + lane; t < wo.se; t += 64)
    if (t < P.seed_cap) { SeedRec r; r.read_id = INVALID_READ; r.qbeg = r.qend = r.flags = 0; r.k = r.kr = r.s = 0; P.seeds[t] = r; }
  for (uint64_t t = wo.qb + lane; t < wo.qe; t += 64)
    if (t < P.subq_cap) { Query q; q.read_id = INVALID_READ; q.qbeg = q.qend = q.l = 0; q.c = 1; P.subq[t] = q; }
}

__global__ void __launch_bounds__(256) k_smem_wave(IndexView ix, SeedParams P) {
  __shared__ uint4 lbuf[4 * WAVE_U4];
  const int lane = threadIdx.x & 63;
  uint4 *buf = lbuf + (threadIdx.x >> 6) * WAVE_U4;
  const int K = (P.use_kmer && ix.kmer) ? ix.K : 0;
  const uint8_t *rb = nullptr;
  uint32_t read_id = 0, qbeg = 0, qend = 0, l = 0, c = 1;
  int u = 0, i = 0, j = 0;
  uint64_t k = 0, kr = 0, s = 0, budget = 0;
  bool fresh = false, active = false, drained = false;
  uint64_t n_lines = 0, n_steps = 0, n_kmer = 0;
  uint64_t cb = 0, ce = 0;
  WaveOut wo = {0, 0, 0, 0};
  for (;;) {
    // ---- refill idle lanes from the wave's work chunk
    const bool want = !active && !drained;
    if (__ballot(want)) {
      const uint64_t qi = wave_take(want, cb, ce, &P.ctl[C_WORK], P.n_queries, lane);
      if (want) {
        if (qi == ~0ull) drained = true;
        else {
          load_query(P, qi, read_id, qbeg, qend, l, c);
          if (read_id != INVALID_READ && l >= 1 && l - 1 < qend - qbeg) {
            rb = P.codes + P.offs[read_id];
            u = 1; i = (int)qbeg; j = (int)(qbeg + l - 1);
            k = 0; kr = 0; s = ix.n; fresh = true; active = true;
            budget = 8ull * (qend - qbeg) * (qend - qbeg) + 64;
          }
        }
      }
    }
    if (__ballot(active) == 0) {
      if (__ballot(!drained) == 0) break;
      continue;
    }
    // ---- per-lane stage transitions up to the next memory action
    int act = ACT_DONE, a = 0;
    uint32_t code = 0;
    bool em = false;
    Emit e;
    e.i = 0; e.j = 0; e.k = 0; e.kr = 0; e.s = 0;
    if (active) {
      if (--budget == 0) { atomicOr(&P.ctl[C_ERR], 1ull); active = false; }
    }
    if (active) {
      for (;;) {
        if (u == 2) {
          if (j == (int)qend) { em = true; e.i = i; e.j = j; e.k = k; e.kr = kr; e.s = s; act = ACT_DONE; break; }
          a = rb[j];
          if (a > 3) {
            em = true; e.i = i; e.j = j; e.k = k; e.kr = kr; e.s = s;
            u = 3; k = 0; kr = 0; s = ix.n; fresh = true;
            continue;
          }
          act = ACT_FWD; break;
        }
        if (u == 1 && j < i) { u = 2; j = i + (int)l; fresh = false; continue; }
        if (u == 3 && j <= i) { u = 1; i = j + 1; j = j + (int)l; k = 0; kr = 0; s = ix.n; fresh = true; continue; }
        if (fresh && K > 0 && j - K + 1 >= (u == 1 ? i : i + 1)) {
          bool ok = true;
          code = 0;
          for (int t = j - K + 1; t <= j; ++t) { int b = rb[t]; ok = ok && b < 4; code = code * 4 + (uint32_t)(b & 3); }
          fresh = false;
          if (ok) { act = ACT_KMER; break; }
        }
        fresh = false;
        a = rb[j];
        if (a > 3) {
          if (j + (int)l < (int)qend) { u = 1; i = j + 1; j = j + (int)l; k = 0; kr = 0; s = ix.n; fresh = true; continue; }
          act = ACT_DONE; break;
        }
        act = ACT_BWD; break;
      }
      if (act == ACT_DONE) active = false;
    }
    // ---- k-mer lookups (one 16-byte load per lane)
    if (act == ACT_KMER) {
      uint64_t ek, ekr, es;
      kmer_unpack(ix.kmer[code], ek, ekr, es);
      ++n_kmer;
      if (es >= c) { k = ek; kr = ekr; s = es; j -= K; }
    }
    // ---- extension steps (Algorithm 1) with the wave-cooperative fetch
    const bool ext = act == ACT_BWD || act == ACT_FWD;
    const bool bwd = act == ACT_BWD;
    const uint64_t x1 = bwd ? k : kr, y = bwd ? kr : k;
    const int cc = bwd ? a : 3 - a;
    const uint64_t x2 = x1 + s;
    const uint32_t L1 = ext ? (uint32_t)line_of(x1) : 0u, L2 = ext ? (uint32_t)line_of(x2) : 0u;
    if (__ballot(ext)) {
      wave_fetch(ix.lines, L1, ext, buf, lane);
      const bool same = L1 == L2;
      uint64_t E1 = 0, G1 = 0, E2 = 0, G2 = 0;
      if (ext) lane_eg(buf, lane, cc, (int)(x1 - (uint64_t)L1 * MBW_BPL), same ? (int)(x2 - (uint64_t)L2 * MBW_BPL) : -1,
                       E1, G1, E2, G2);
      const bool two = ext && !same;
      if (__ballot(two)) {
        wave_fetch(ix.lines, L2, two, buf, lane);
        if (two) {
          uint64_t t1, t2;
          lane_eg(buf, lane, cc, (int)(x2 - (uint64_t)L2 * MBW_BPL), -1, E2, G2, t1, t2);
        }
      }
      if (ext) {
        n_lines += two ? 2 : 1;
        ++n_steps;
        if (cc == 0) { E1 -= x1 > ix.primary ? 1 : 0; E2 -= x2 > ix.primary ? 1 : 0; }
        const uint64_t dol = (x1 <= ix.primary && ix.primary < x2) ? 1 : 0;
        const uint64_t ns = E2 - E1;
        const uint64_t nx = sel4(ix.Cb[0], ix.Cb[1], ix.Cb[2], ix.Cb[3], cc) + E1;
        const uint64_t ny = y + dol + (G2 - G1);
        if (ns >= c) {
          if (bwd) { k = nx; kr = ny; s = ns; j -= 1; }
          else { kr = nx; k = ny; s = ns; j += 1; }
        } else if (bwd) {
          if (j + (int)l < (int)qend) { u = 1; i = j + 1; j = j + (int)l; k = 0; kr = 0; s = ix.n; fresh = true; }
          else active = false;
        } else {
          em = true; e.i = i; e.j = j; e.k = k; e.kr = kr; e.s = s;
          u = 3; k = 0; kr = 0; s = ix.n; fresh = true;
        }
      }
    }
    wave_emit(P, lane, em, read_id, e, wo);
  }
  wave_close(P, lane, wo);
  atomicAdd(&P.ctl[C_LINES], (unsigned long long)(n_lines + n_kmer));
  atomicAdd(&P.ctl[C_STEPS], (unsigned long long)n_steps);
  atomicAdd(&P.ctl[C_KMER], (unsigned long long)n_kmer);
}

// ---------------------------------------------------------------------------------------------
// plain SMEM kernel: one thread = one read, the serial algorithm with round 2 run inline
struct PlainCtx {
  IndexView ix;
  const SeedParams *P;
  const uint8_t *rb;
  uint32_t read_id;
  uint64_t lines, steps;
};

__device__ __forceinline__ uint64_t plain_step(PlainCtx &C, bool bwd, int a, uint64_t &k, uint64_t &kr, uint64_t s,
                                               uint64_t &nk, uint64_t &nkr) {
  const uint64_t x = bwd ? k : kr, y = bwd ? kr : k;
  const int cc = bwd ? a : 3 - a;
  const uint64_t x2 = x + s;
  Occ4 o1 = occ_single(C.ix.lines, x, C.ix.primary);
  Occ4 o2 = occ_single(C.ix.lines, x2, C.ix.primary);
  C.lines += line_of(x) == line_of(x2) ? 1 : 2;
  C.steps++;
  uint64_t nx, ny, ns;
  ext_update(o1, o2, cc, x, s, y, C.ix.primary, C.ix.Cb, nx, ny, ns);
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
      int a = C.rb[j];
      uint64_t nk = 0, nkr = 0, ns = 0;
      if (a < 4) ns = plain_step(C, true, a, k, kr, s, nk, nkr);
      if (ns >= c) { k = nk; kr = nkr; s = ns; j -= 1; continue; }
      if (j + l < qend) { u = 1; i = j + 1; j = j + l; k = 0; kr = 0; s = n; continue; }
      return;
    }
    if (j == qend) {
      emit_plain<ROUND>(C, i, j, k, kr, s);
      return;
    }
    int a = C.rb[j];
    uint64_t nk = 0, nkr = 0, ns = 0;
    if (a < 4) ns = plain_step(C, false, a, k, kr, s, nk, nkr);
    if (ns >= c) { k = nk; kr = nkr; s = ns; j += 1; continue; }
    emit_plain<ROUND>(C, i, j, k, kr, s);
    u = 3; k = 0; kr = 0; s = n;
  }
}

template <>
__device__ void emit_plain<2>(PlainCtx &C, int i, int j, uint64_t k, uint64_t kr, uint64_t s) {
  SeedParams P2 = *C.P;
  P2.round = 2;
  emit_seed(P2, C.read_id, i, j, k, kr, s);
}

template <>
__device__ void emit_plain<1>(PlainCtx &C, int i, int j, uint64_t k, uint64_t kr, uint64_t s) {
  SeedParams P1 = *C.P;
  P1.round = 1;
  P1.reseed = 0;   // the sub-query runs inline below instead of being queued
  emit_seed(P1, C.read_id, i, j, k, kr, s);
  if (C.P->reseed && j - i >= C.P->reseed_len && s <= (uint64_t)C.P->reseed_occ)
    plain_alg3<2>(C, i, j, (j - i) / 2, s + 1);
}

__global__ void __launch_bounds__(256) k_smem_plain(IndexView ix, SeedParams P) {
  uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (r >= P.n_queries) return;
  PlainCtx C;
  C.ix = ix; C.P = &P; C.read_id = (uint32_t)r; C.rb = P.codes + P.offs[r]; C.lines = 0; C.steps = 0;
  int len = (int)(P.offs[r + 1] - P.offs[r]);
  plain_alg3<1>(C, 0, len, P.l, (uint64_t)P.c);
  atomicAdd(&P.ctl[C_LINES], (unsigned long long)C.lines);
  atomicAdd(&P.ctl[C_STEPS], (unsigned long long)C.steps);
}

// ---------------------------------------------------------------------------------------------
// seeds: sort keys, dedup, counts
// sort key (read, qbeg, qend); unused slots (read_id INVALID_READ) get key n_reads << 32, after all
__global__ void k_seed_keys(const SeedRec *__restrict__ raw, uint64_t ns, uint64_t n_reads, uint64_t *__restrict__ key,
                            uint32_t *__restrict__ val) {
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < ns; t += (uint64_t)gridDim.x * blockDim.x) {
    SeedRec r = raw[t];
    key[t] = r.read_id == INVALID_READ ? (n_reads << 32)
                                       : (((uint64_t)r.read_id << 32) | ((uint64_t)r.qbeg << 16) | (uint64_t)r.qend);
    val[t] = (uint32_t)t;
  }
}

__global__ void k_dedup_mark(const uint64_t *__restrict__ key, uint64_t ns, uint64_t n_reads, uint32_t *__restrict__ flag) {
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < ns; t += (uint64_t)gridDim.x * blockDim.x)
    flag[t] = (key[t] < (n_reads << 32) && (t == 0 || key[t] != key[t - 1])) ? 1u : 0u;
}

__global__ void k_seed_emit(const SeedRec *__restrict__ raw, const uint32_t *__restrict__ val, const uint32_t *__restrict__ flag,
                            const uint32_t *__restrict__ idx, uint64_t ns, uint64_t max_occ, mbw_seed_t *__restrict__ out,
                            uint64_t *__restrict__ npos) {
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < ns; t += (uint64_t)gridDim.x * blockDim.x) {
    if (!flag[t]) continue;
    SeedRec r = raw[val[t]];
    mbw_seed_t o;
    o.read_id = r.read_id; o.qbeg = r.qbeg; o.qend = r.qend;
    o.k = r.k; o.kr = r.kr; o.s = r.s; o.pos_off = 0; o.reserved = 0;
    bool loc = r.s <= max_occ;
    o.flags = r.flags | (loc ? 0u : MBW_SEED_UNLOCATED);
    o.npos = loc ? (uint32_t)r.s : 0u;
    uint32_t d = idx[t];
    out[d] = o;
    npos[d] = o.npos;
  }
}

__global__ void k_seed_posoff(mbw_seed_t *__restrict__ out, const uint64_t *__restrict__ off, uint64_t ns,
                              uint32_t *__restrict__ sid_seed) {
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < ns; t += (uint64_t)gridDim.x * blockDim.x) {
    out[t].pos_off = off[t];
    if (sid_seed && out[t].npos) sid_seed[off[t]] = (uint32_t)t;
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
  uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (t >= ns) return;
  mbw_seed_t sd = seeds[t];
  uint64_t lines = 0, lf = 0;
  for (uint32_t w = 0; w < sd.npos; ++w) {
    uint64_t x = sd.k + w, steps = 0;
    while (!sampled(x, ix.r, rmask)) {
      if (steps > ix.n) { atomicOr(&ctl[C_ERR], 2ull); x = 0; break; }
      if (x == ix.primary) { x = 0; ++steps; continue; }   // LF of the $ row is row 0
      int b = bwt_single(ix.lines, x);
      Occ4 o = occ_single(ix.lines, x, ix.primary);
      x = ix.Cb[b] + o.v[b];
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

// cooperative: persistent; each 8-lane group walks one SA row at a time, refilling from a queue
// of all (seed, row) pairs (BatchLocate's refill of finished walks).
__global__ void __launch_bounds__(256) k_locate_coop(IndexView ix, const mbw_seed_t *__restrict__ seeds,
                                                     const uint32_t *__restrict__ sid, uint64_t n_pos,
                                                     uint64_t *__restrict__ pos, uint32_t rmask, int rshift, int grab,
                                                     unsigned long long *__restrict__ ctl) {
  const int q = threadIdx.x & (MBW_GROUP - 1);
  uint64_t wnext = 0, wlast = 0, w = 0, x = 0, steps = 0;
  bool active = false;
  uint64_t lines = 0, lf = 0;
  for (;;) {
    if (!active) {
      if (wnext >= wlast) {
        unsigned long long b0 = 0;
        if (q == 0) b0 = atomicAdd(&ctl[C_WORK2], (unsigned long long)grab);
        b0 = __shfl(b0, 0, MBW_GROUP);
        if (b0 >= n_pos) break;
        wnext = b0;
        wlast = b0 + (uint64_t)grab < n_pos ? b0 + (uint64_t)grab : n_pos;
      }
      w = wnext++;
      uint32_t t = sid[w];
      x = seeds[t].k + (w - seeds[t].pos_off);
      steps = 0;
      active = true;
    }
    if (sampled(x, ix.r, rmask)) {
      uint64_t p = steps + ix.ssa[sample_index(x, ix.r, rshift)];
      if (p >= ix.n) p -= ix.n;
      if (q == 0) pos[w] = p;
      ++lines;
      active = false;
      continue;
    }
    if (x == ix.primary || steps > ix.n) {   // LF of the $ row is row 0; the cap only guards a corrupt index
      if (steps > ix.n && q == 0) atomicOr(&ctl[C_ERR], 2ull);
      x = 0; ++steps; continue;
    }
    const uint64_t L = line_of(x);
    const int o = (int)(x - L * MBW_BPL);
    uint4 d = ix.lines[L * MBW_LINE_U4 + q];
    const uint64_t w0 = ((uint64_t)d.y << 32) | d.x, w1 = ((uint64_t)d.w << 32) | d.z;
    // one reduction carries the in-line counts of A, C, G (16 bits each) and B[x] + 1 (top 16 bits,
    // from the slice holding row o); a second one the line's prefix count of B[x]
    uint64_t pk = 0;
    if (q >= 2) {
      pk = slice_counts(d, q, o) & 0xFFFFFFFFFFFFull;
      if (q == 2 + (o >> 6)) {
        uint64_t wsel = (o & 63) < 32 ? w0 : w1;
        pk |= (((wsel >> (2 * (o & 31))) & 3) + 1) << 48;
      }
    }
    pk = grp_sum64(pk);
    const int b = (int)(pk >> 48) - 1;
    uint64_t hv = 0;
    if (q == 0) hv = b == 0 ? w0 : (b == 1 ? w1 : 0);
    else if (q == 1) hv = b == 2 ? w0 : (b == 3 ? w1 : 0);
    hv = grp_sum64(hv);
    const uint64_t nA = pk & 0xffff, nC = (pk >> 16) & 0xffff, nG = (pk >> 32) & 0xffff;
    const uint64_t inl = b == 0 ? nA : (b == 1 ? nC : (b == 2 ? nG : (uint64_t)o - nA - nC - nG));
    const uint64_t occ = hv + inl - ((b == 0 && x > ix.primary) ? 1 : 0);
    x = sel4(ix.Cb[0], ix.Cb[1], ix.Cb[2], ix.Cb[3], b) + occ;
    ++steps; ++lines; ++lf;
  }
  if (q == 0 && lines) {
    atomicAdd(&ctl[C_LINES_LOC], (unsigned long long)lines);
    atomicAdd(&ctl[C_LFSTEPS], (unsigned long long)lf);
  }
}

// wave-cooperative locate: every lane walks one SA row; idle lanes refill from the queue of all
// (seed, row) pairs (one atomic per wave); lines are fetched with the wave-cooperative loads.
__global__ void __launch_bounds__(256) k_locate_wave(IndexView ix, const mbw_seed_t *__restrict__ seeds,
                                                     const uint32_t *__restrict__ sid, uint64_t n_pos,
                                                     uint64_t *__restrict__ pos, uint32_t rmask, int rshift,
                                                     unsigned long long *__restrict__ ctl) {
  __shared__ uint4 lbuf[4 * WAVE_U4];
  const int lane = threadIdx.x & 63;
  uint4 *buf = lbuf + (threadIdx.x >> 6) * WAVE_U4;
  uint64_t w = 0, x = 0, steps = 0, lines = 0, lf = 0;
  uint64_t cb = 0, ce = 0;
  bool active = false, drained = false;
  for (;;) {
    const bool want = !active && !drained;
    if (__ballot(want)) {
      const uint64_t wi = wave_take(want, cb, ce, &ctl[C_WORK2], n_pos, lane);
      if (want) {
        w = wi;
        if (w == ~0ull) drained = true;
        else {
          const uint32_t t = sid[w];
          x = seeds[t].k + (w - seeds[t].pos_off);
          steps = 0;
          active = true;
        }
      }
    }
    if (__ballot(active) == 0) {
      if (__ballot(!drained) == 0) break;
      continue;
    }
    bool need = false;
    if (active) {
      if (sampled(x, ix.r, rmask)) {
        uint64_t p = steps + ix.ssa[sample_index(x, ix.r, rshift)];
        if (p >= ix.n) p -= ix.n;
        pos[w] = p;
        ++lines;
        active = false;
      } else if (x == ix.primary || steps > ix.n) {   // LF of the $ row is row 0 (the cap guards a corrupt index)
        if (steps > ix.n) atomicOr(&ctl[C_ERR], 2ull);
        x = 0;
        ++steps;
      } else {
        need = true;
      }
    }
    const uint32_t L = need ? (uint32_t)line_of(x) : 0u;
    if (__ballot(need)) {
      wave_fetch(ix.lines, L, need, buf, lane);
      if (need) {
        const int o = (int)(x - (uint64_t)L * MBW_BPL);
        const uint4 bd = buf[slot_of(lane, 2 + (o >> 6))];
        const uint64_t wsel = (o & 63) < 32 ? (((uint64_t)bd.y << 32) | bd.x) : (((uint64_t)bd.w << 32) | bd.z);
        const int b = (int)((wsel >> (2 * (o & 31))) & 3);
        uint64_t E, G, t1, t2;
        lane_eg(buf, lane, b, o, -1, E, G, t1, t2);
        if (b == 0 && x > ix.primary) E -= 1;
        x = sel4(ix.Cb[0], ix.Cb[1], ix.Cb[2], ix.Cb[3], b) + E;
        ++steps; ++lines; ++lf;
      }
    }
  }
  atomicAdd(&ctl[C_LINES_LOC], (unsigned long long)lines);
  atomicAdd(&ctl[C_LFSTEPS], (unsigned long long)lf);
}

// ---------------------------------------------------------------------------------------------
// bisulfite strand filter (Section 2.9): segment = pos / |R| of T over the four copies
__global__ void k_bs_mark(const uint64_t *__restrict__ pos, uint64_t np, uint64_t len_r, int role, uint32_t *__restrict__ keep) {
  for (uint64_t w = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; w <= np; w += (uint64_t)gridDim.x * blockDim.x) {
    if (w == np) { keep[w] = 0; continue; }
    uint64_t seg = pos[w] / len_r;
    keep[w] = (role == 1) ? (seg == 0 || seg == 2) : (seg == 1 || seg == 3);
  }
}

__global__ void k_bs_compact(const uint64_t *__restrict__ pos, const uint32_t *__restrict__ keep, const uint64_t *__restrict__ kidx,
                             uint64_t np, uint64_t *__restrict__ out) {
  for (uint64_t w = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; w < np; w += (uint64_t)gridDim.x * blockDim.x)
    if (keep[w]) out[kidx[w]] = pos[w];
}

__global__ void k_bs_seeds(mbw_seed_t *__restrict__ seeds, uint64_t ns, const uint64_t *__restrict__ kidx) {
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < ns; t += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t a = seeds[t].pos_off, b = a + seeds[t].npos;
    seeds[t].pos_off = kidx[a];
    seeds[t].npos = (uint32_t)(kidx[b] - kidx[a]);
  }
}

inline unsigned grid_for(uint64_t n, unsigned bs = 256, unsigned cap = 65536u * 8) {
  uint64_t g = (n + bs - 1) / bs;
  if (g < 1) g = 1;
  return (unsigned)std::min<uint64_t>(g, cap);
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// context
struct mbw_ctx {
  const mbw_index *ix;
  int device;
  int n_cu;
  // grow-only device buffers
  struct Buf { void *p = nullptr; size_t bytes = 0; };
  Buf codes, ascii, lens, offs, raw, subq, keys0, keys1, vals0, vals1, flag, idx, seeds, npos, posoff, sid, pos, pos2,
      keep, kidx, temp, ctl;
  hipEvent_t ev[8];
  unsigned long long host_ctl[C_COUNT];
  float ms_smem;
  int n_smem_launches;
};

static int grow(mbw_ctx::Buf &b, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (b.bytes >= bytes) return 0;
  if (b.p) { (void)hipFree(b.p); b.p = nullptr; b.bytes = 0; }
  size_t want = bytes + bytes / 4 + 256;
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) { b.p = nullptr; mbw_set_error(std::string("hipMalloc(") + std::to_string(want) + "): " + hipGetErrorString(e)); return MBW_E_NOMEM; }
  b.bytes = want;
  return 0;
}
#define GROW(buf, bytes) do { int r_ = grow(buf, bytes); if (r_) return r_; } while (0)

extern "C" int mbw_ctx_create(const mbw_index *ix, mbw_ctx **out) {
  if (!ix || !out) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  *out = nullptr;
  TRY(hipSetDevice(ix->device));
  mbw_ctx *c = new mbw_ctx();
  c->ix = ix;
  c->device = ix->device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, ix->device) != hipSuccess) { delete c; mbw_set_error("hipGetDeviceProperties failed"); return MBW_E_HIP; }
  c->n_cu = prop.multiProcessorCount;
  for (int t = 0; t < 8; ++t)
    if (hipEventCreate(&c->ev[t]) != hipSuccess) { delete c; mbw_set_error("hipEventCreate failed"); return MBW_E_HIP; }
  if (grow(c->ctl, C_COUNT * sizeof(unsigned long long))) { delete c; return MBW_E_NOMEM; }
  *out = c;
  return MBW_OK;
}

extern "C" void mbw_ctx_free(mbw_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  mbw_ctx::Buf *bs[] = {&c->codes, &c->ascii, &c->lens, &c->offs, &c->raw, &c->subq, &c->keys0, &c->keys1, &c->vals0,
                        &c->vals1, &c->flag, &c->idx, &c->seeds, &c->npos, &c->posoff, &c->sid, &c->pos, &c->pos2,
                        &c->keep, &c->kidx, &c->temp, &c->ctl};
  for (auto *b : bs) if (b->p) (void)hipFree(b->p);
  for (int t = 0; t < 8; ++t) (void)hipEventDestroy(c->ev[t]);
  delete c;
}

static bool is_device_ptr(const void *p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) { (void)hipGetLastError(); return false; }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

template <class F>
static int cub_call(mbw_ctx *c, F f) {
  size_t tb = 0;
  TRY(f((void *)nullptr, tb));
  GROW(c->temp, tb);
  size_t have = c->temp.bytes;
  TRY(f(c->temp.p, have));
  return 0;
}

static int persistent_grid(const void *kern, int block, size_t lds, int n_cu, int per_cu_req) {
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, block, lds) != hipSuccess || per < 1) per = 4;
  if (per_cu_req > 0 && per_cu_req < per) per = per_cu_req;
  return per * n_cu;
}

static int launch_smem(mbw_ctx *c, const IndexView &v, SeedParams &P, const mbw_seed_opts &o, int maxlen, hipStream_t st);
static int run_smem(mbw_ctx *c, const IndexView &v, SeedParams &P, const mbw_seed_opts &o, int maxlen, hipStream_t st) {
  if (P.n_queries == 0) return 0;
  TRY(hipEventRecord(c->ev[1], st));
  int r = launch_smem(c, v, P, o, maxlen, st);
  if (r) return r;
  TRY(hipEventRecord(c->ev[2], st));
  TRY(hipEventSynchronize(c->ev[2]));
  float ms = 0;
  TRY(hipEventElapsedTime(&ms, c->ev[1], c->ev[2]));
  c->ms_smem += ms;
  c->n_smem_launches++;
  return 0;
}

static int launch_smem(mbw_ctx *c, const IndexView &v, SeedParams &P, const mbw_seed_opts &o, int maxlen, hipStream_t st) {
  if (o.kernel == MBW_KERNEL_PLAIN) {
    k_smem_plain<<<grid_for(P.n_queries, 256), 256, 0, st>>>(v, P);
    TRY(hipGetLastError());
    return 0;
  }
  if (o.schedule == MBW_SCHED_WAVE) {
    int grid = persistent_grid((const void *)k_smem_wave, 256, 0, c->n_cu, o.blocks_per_cu);
    k_smem_wave<<<grid, 256, 0, st>>>(v, P);
    TRY(hipGetLastError());
    return 0;
  }
  int gpb = o.groups_per_block > 0 ? o.groups_per_block : 32;
  if (gpb > 32) gpb = 32;
  int block = gpb * MBW_GROUP;
  if (maxlen <= 256) {
    size_t lds = (size_t)gpb * 256;
    int grid = persistent_grid((const void *)k_smem_coop<256>, block, lds, c->n_cu, o.blocks_per_cu);
    k_smem_coop<256><<<grid, block, lds, st>>>(v, P);
  } else {
    int grid = persistent_grid((const void *)k_smem_coop<0>, block, 0, c->n_cu, o.blocks_per_cu);
    k_smem_coop<0><<<grid, block, 0, st>>>(v, P);
  }
  TRY(hipGetLastError());
  return 0;
}

extern "C" int mbw_seed(mbw_ctx *c, const uint8_t *reads, const uint32_t *lengths, uint64_t n_reads, int min_seed_len,
                        int max_occ, const mbw_seed_opts *opts, void *stream, mbw_result *out) {
  if (!c || !out) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  memset(out, 0, sizeof(*out));
  if (min_seed_len < 1 || max_occ < 1) { mbw_set_error("min_seed_len and max_occ must be >= 1"); return MBW_E_INVAL; }
  if (n_reads > 0 && (!reads || !lengths)) { mbw_set_error("NULL reads or lengths"); return MBW_E_INVAL; }
  if (n_reads >= (1ull << 32)) { mbw_set_error("too many reads in one call"); return MBW_E_INVAL; }
  mbw_seed_opts o;
  if (opts) o = *opts;
  else { memset(&o, 0, sizeof(o)); o.min_occ = 1; o.reseed = 1; o.reseed_len = 38; o.reseed_occ = 10; o.use_kmer = 1; }
  if (o.min_occ < 1) { mbw_set_error("min_occ must be >= 1"); return MBW_E_INVAL; }
  if (o.bs_role && !c->ix->bisulfite) { mbw_set_error("bs_role needs a bisulfite index"); return MBW_E_INVAL; }
  if (o.bs_role < 0 || o.bs_role > 2) { mbw_set_error("bs_role must be 0, 1 or 2"); return MBW_E_INVAL; }
  if (o.grab <= 0) o.grab = 8;
  if (o.grab_locate <= 0) o.grab_locate = 64;
  TRY(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  const mbw_index *ix = c->ix;
  IndexView v = make_view(ix);
  unsigned long long *ctl = (unsigned long long *)c->ctl.p;
  TRY(hipMemsetAsync(ctl, 0, C_COUNT * sizeof(unsigned long long), st));
  c->ms_smem = 0;
  c->n_smem_launches = 0;
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
  k_widen<<<grid_for(n_reads + 1), 256, 0, st>>>(dlen, n_reads, wide, ctl + C_MAXLEN);
  TRY(hipGetLastError());
  uint64_t *offs = (uint64_t *)c->offs.p;
  int r = cub_call(c, [&](void *tp, size_t &tb) { return hipcub::DeviceScan::ExclusiveSum(tp, tb, wide, offs, n_reads + 1, st); });
  if (r) return r;
  uint64_t total = 0;
  unsigned long long maxlen = 0;
  TRY(hipMemcpyAsync(&total, offs + n_reads, 8, hipMemcpyDeviceToHost, st));
  TRY(hipMemcpyAsync(&maxlen, ctl + C_MAXLEN, 8, hipMemcpyDeviceToHost, st));
  TRY(hipStreamSynchronize(st));
  if (maxlen > MBW_MAX_READ) { mbw_set_error("read longer than 65535 bases"); return MBW_E_INVAL; }
  // encode
  GROW(c->codes, total + 16);
  const uint8_t *dreads = reads;
  if (!is_device_ptr(reads)) {
    GROW(c->ascii, total + 16);
    TRY(hipMemcpyAsync(c->ascii.p, reads, total, hipMemcpyHostToDevice, st));
    dreads = (const uint8_t *)c->ascii.p;
  }
  k_encode<<<grid_for(total), 256, 0, st>>>(dreads, total, o.bs_role, (uint8_t *)c->codes.p);
  TRY(hipGetLastError());
  // SMEM rounds
  // per-wave output chunks leave up to one partly used chunk per wave of the persistent grid
  const uint64_t chunk_slack = (uint64_t)c->n_cu * 32 * OUT_CHUNK;
  uint64_t seed_cap = std::max<uint64_t>(1 << 16, n_reads * 4) + chunk_slack;
  if (c->raw.bytes / sizeof(SeedRec) > seed_cap) seed_cap = c->raw.bytes / sizeof(SeedRec);
  uint64_t subq_cap = std::max<uint64_t>(1 << 14, n_reads / 2) + chunk_slack;
  if (c->subq.bytes / sizeof(Query) > subq_cap) subq_cap = c->subq.bytes / sizeof(Query);
  SeedParams P;
  memset(&P, 0, sizeof(P));
  P.codes = (const uint8_t *)c->codes.p; P.offs = offs; P.queries = nullptr; P.n_queries = n_reads;
  P.l = min_seed_len; P.c = o.min_occ; P.reseed = o.reseed; P.reseed_len = o.reseed_len; P.reseed_occ = o.reseed_occ;
  P.round = 1; P.use_kmer = o.use_kmer; P.grab = o.grab; P.ctl = ctl;
  unsigned long long n1 = 0, nq = 0;
  for (int attempt = 0;; ++attempt) {
    GROW(c->raw, seed_cap * sizeof(SeedRec));
    GROW(c->subq, subq_cap * sizeof(Query));
    seed_cap = c->raw.bytes / sizeof(SeedRec);
    subq_cap = c->subq.bytes / sizeof(Query);
    P.seeds = (SeedRec *)c->raw.p; P.seed_cap = seed_cap; P.subq = (Query *)c->subq.p; P.subq_cap = subq_cap;
    TRY(hipMemsetAsync(ctl, 0, 8 * sizeof(unsigned long long), st));
    r = run_smem(c, v, P, o, (int)maxlen, st);
    if (r) return r;
    TRY(hipMemcpyAsync(&n1, ctl + C_NSEEDS, 8, hipMemcpyDeviceToHost, st));
    TRY(hipMemcpyAsync(&nq, ctl + C_NSUBQ, 8, hipMemcpyDeviceToHost, st));
    TRY(hipStreamSynchronize(st));
    if (n1 <= seed_cap && nq <= subq_cap) break;
    if (attempt > 3) { mbw_set_error("seed buffer did not converge"); return MBW_E_NOMEM; }
    seed_cap = std::max<uint64_t>(seed_cap, n1 + n1 / 2 + 1024);
    subq_cap = std::max<uint64_t>(subq_cap, nq + nq / 2 + 1024);
  }
  unsigned long long stats1[3];
  TRY(hipMemcpyAsync(stats1, ctl + C_LINES, 3 * 8, hipMemcpyDeviceToHost, st));
  unsigned long long ntot = n1;
  if (o.kernel != MBW_KERNEL_PLAIN && o.reseed && nq > 0) {
    SeedParams P2 = P;
    P2.queries = (const Query *)c->subq.p; P2.n_queries = nq; P2.round = 2;
    for (int attempt = 0;; ++attempt) {
      TRY(hipMemcpyAsync(ctl + C_NSEEDS, &n1, 8, hipMemcpyHostToDevice, st));
      unsigned long long zero = 0;
      TRY(hipMemcpyAsync(ctl + C_WORK, &zero, 8, hipMemcpyHostToDevice, st));
      TRY(hipMemcpyAsync(ctl + C_LINES, stats1, 3 * 8, hipMemcpyHostToDevice, st));
      P2.seeds = (SeedRec *)c->raw.p; P2.seed_cap = c->raw.bytes / sizeof(SeedRec);
      r = run_smem(c, v, P2, o, (int)maxlen, st);
      if (r) return r;
      TRY(hipMemcpyAsync(&ntot, ctl + C_NSEEDS, 8, hipMemcpyDeviceToHost, st));
      TRY(hipStreamSynchronize(st));
      if (ntot <= P2.seed_cap) break;
      if (attempt > 3) { mbw_set_error("seed buffer did not converge"); return MBW_E_NOMEM; }
      // keep round-1 records: grow by copying
      mbw_ctx::Buf nb;
      int rr = grow(nb, (ntot + ntot / 2 + 1024) * sizeof(SeedRec));
      if (rr) return rr;
      TRY(hipMemcpyAsync(nb.p, c->raw.p, n1 * sizeof(SeedRec), hipMemcpyDeviceToDevice, st));
      TRY(hipStreamSynchronize(st));
      (void)hipFree(c->raw.p);
      c->raw = nb;
    }
  }
  // sort by (read, qbeg, qend), dedup, counts
  uint64_t ns = ntot;
  GROW(c->keys0, ns * 8); GROW(c->keys1, ns * 8); GROW(c->vals0, ns * 4); GROW(c->vals1, ns * 4);
  GROW(c->flag, ns * 4 + 8); GROW(c->idx, ns * 4 + 8);
  if (ns) {
    k_seed_keys<<<grid_for(ns), 256, 0, st>>>((const SeedRec *)c->raw.p, ns, n_reads, (uint64_t *)c->keys0.p, (uint32_t *)c->vals0.p);
    TRY(hipGetLastError());
  }
  int hibit = 33;   // key < (n_reads + 1) << 32
  while (hibit < 64 && (1ull << (hibit - 32)) <= n_reads) ++hibit;
  hipcub::DoubleBuffer<uint64_t> dk((uint64_t *)c->keys0.p, (uint64_t *)c->keys1.p);
  // (ns may be 0: every step below is skipped then)
  hipcub::DoubleBuffer<uint32_t> dv((uint32_t *)c->vals0.p, (uint32_t *)c->vals1.p);
  if (ns > 1) {
    r = cub_call(c, [&](void *tp, size_t &tb) { return hipcub::DeviceRadixSort::SortPairs(tp, tb, dk, dv, ns, 0, hibit, st); });
    if (r) return r;
  }
  uint32_t *flag = (uint32_t *)c->flag.p, *idx = (uint32_t *)c->idx.p;
  uint64_t nu = 0;
  if (ns) {
    k_dedup_mark<<<grid_for(ns), 256, 0, st>>>(dk.Current(), ns, n_reads, flag);
    TRY(hipGetLastError());
    r = cub_call(c, [&](void *tp, size_t &tb) { return hipcub::DeviceScan::ExclusiveSum(tp, tb, flag, idx, ns, st); });
    if (r) return r;
    uint32_t lastf = 0, lasti = 0;
    TRY(hipMemcpyAsync(&lastf, flag + ns - 1, 4, hipMemcpyDeviceToHost, st));
    TRY(hipMemcpyAsync(&lasti, idx + ns - 1, 4, hipMemcpyDeviceToHost, st));
    TRY(hipStreamSynchronize(st));
    nu = (uint64_t)lasti + lastf;
  }
  GROW(c->seeds, (nu + 1) * sizeof(mbw_seed_t));
  GROW(c->npos, (nu + 2) * 8);
  GROW(c->posoff, (nu + 2) * 8);
  mbw_seed_t *seeds = (mbw_seed_t *)c->seeds.p;
  uint64_t *npos = (uint64_t *)c->npos.p, *posoff = (uint64_t *)c->posoff.p;
  if (ns) {
    k_seed_emit<<<grid_for(ns), 256, 0, st>>>((const SeedRec *)c->raw.p, dv.Current(), flag, idx, ns, (uint64_t)max_occ, seeds, npos);
    TRY(hipGetLastError());
  }
  uint64_t n_pos = 0;
  if (nu) {
    TRY(hipMemsetAsync(npos + nu, 0, 8, st));
    r = cub_call(c, [&](void *tp, size_t &tb) { return hipcub::DeviceScan::ExclusiveSum(tp, tb, npos, posoff, nu + 1, st); });
    if (r) return r;
    TRY(hipMemcpyAsync(&n_pos, posoff + nu, 8, hipMemcpyDeviceToHost, st));
    TRY(hipStreamSynchronize(st));
  }
  const bool coop = o.kernel != MBW_KERNEL_PLAIN;
  GROW(c->pos, (n_pos + 1) * 8);
  uint32_t *sid = nullptr;
  if (coop && n_pos) {
    GROW(c->sid, (n_pos + 1) * 4);
    GROW(c->keep, (n_pos + 1) * 4);
    sid = (uint32_t *)c->sid.p;
    TRY(hipMemsetAsync(c->keep.p, 0, (n_pos + 1) * 4, st));
  }
  if (nu) {
    k_seed_posoff<<<grid_for(nu), 256, 0, st>>>(seeds, posoff, nu, coop && n_pos ? (uint32_t *)c->keep.p : nullptr);
    TRY(hipGetLastError());
  }
  // locate
  uint32_t rmask = (ix->sa_sample & (ix->sa_sample - 1)) == 0 ? (uint32_t)(ix->sa_sample - 1) : 0u;
  if (ix->sa_sample == 1) rmask = 0;   // every row sampled: x % 1 == 0 path
  int rshift = -1;
  if ((ix->sa_sample & (ix->sa_sample - 1)) == 0) { rshift = 0; while ((1 << rshift) < ix->sa_sample) ++rshift; }
  TRY(hipEventRecord(c->ev[3], st));   // re-recorded right before the locate launch below
  if (n_pos) {
    if (!coop) {
      TRY(hipEventRecord(c->ev[3], st));
      k_locate_plain<<<grid_for(nu), 256, 0, st>>>(v, seeds, nu, (uint64_t *)c->pos.p, rmask, rshift, ctl);
      TRY(hipGetLastError());
    } else {
      uint32_t *seedmark = (uint32_t *)c->keep.p;
      r = cub_call(c, [&](void *tp, size_t &tb) { return hipcub::DeviceScan::InclusiveScan(tp, tb, seedmark, sid, hipcub::Max(), n_pos, st); });
      if (r) return r;
      if (o.schedule == MBW_SCHED_WAVE) {
        int grid = persistent_grid((const void *)k_locate_wave, 256, 0, c->n_cu, o.blocks_per_cu);
        TRY(hipEventRecord(c->ev[3], st));
        k_locate_wave<<<grid, 256, 0, st>>>(v, seeds, sid, n_pos, (uint64_t *)c->pos.p, rmask, rshift, ctl);
        TRY(hipGetLastError());
      } else {
      int gpb = o.groups_per_block > 0 ? std::min(o.groups_per_block, 32) : 32;
      int block = gpb * MBW_GROUP;
      int grid = persistent_grid((const void *)k_locate_coop, block, 0, c->n_cu, o.blocks_per_cu);
      TRY(hipEventRecord(c->ev[3], st));
      k_locate_coop<<<grid, block, 0, st>>>(v, seeds, sid, n_pos, (uint64_t *)c->pos.p, rmask, rshift,
                                             o.grab_locate, ctl);
      TRY(hipGetLastError());
      }
    }
  }
  TRY(hipEventRecord(c->ev[4], st));
  // bisulfite strand filter
  const uint64_t *final_pos = (const uint64_t *)c->pos.p;
  if (o.bs_role && n_pos) {
    GROW(c->keep, (n_pos + 1) * 4);
    GROW(c->kidx, (n_pos + 1) * 8);
    GROW(c->pos2, (n_pos + 1) * 8);
    uint32_t *keep = (uint32_t *)c->keep.p;
    uint64_t *kidx = (uint64_t *)c->kidx.p;
    k_bs_mark<<<grid_for(n_pos + 1), 256, 0, st>>>((const uint64_t *)c->pos.p, n_pos, ix->len_r, o.bs_role, keep);
    TRY(hipGetLastError());
    r = cub_call(c, [&](void *tp, size_t &tb) { return hipcub::DeviceScan::ExclusiveSum(tp, tb, keep, kidx, n_pos + 1, st); });
    if (r) return r;
    k_bs_compact<<<grid_for(n_pos), 256, 0, st>>>((const uint64_t *)c->pos.p, keep, kidx, n_pos, (uint64_t *)c->pos2.p);
    TRY(hipGetLastError());
    k_bs_seeds<<<grid_for(nu), 256, 0, st>>>(seeds, nu, kidx);
    TRY(hipGetLastError());
    uint64_t kept = 0;
    TRY(hipMemcpyAsync(&kept, kidx + n_pos, 8, hipMemcpyDeviceToHost, st));
    TRY(hipStreamSynchronize(st));
    n_pos = kept;
    final_pos = (const uint64_t *)c->pos2.p;
  }
  TRY(hipMemcpyAsync(c->host_ctl, ctl, C_COUNT * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
  TRY(hipStreamSynchronize(st));
  if (c->host_ctl[C_ERR]) {
    mbw_set_error(std::string("kernel guard tripped (") + std::to_string(c->host_ctl[C_ERR]) + "): corrupt index or internal error");
    return MBW_E_HIP;
  }
  TRY(hipEventRecord(c->ev[5], st));
  TRY(hipEventSynchronize(c->ev[5]));
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
  out->ms_smem = c->ms_smem; out->ms_locate = t_loc; out->ms_total = t_tot;
  out->n_smem_launches = c->n_smem_launches;
  return MBW_OK;
}

extern "C" int mbw_result_download(mbw_ctx *c, const mbw_result *res, mbw_seed_t *seeds, uint64_t *pos) {
  if (!c || !res) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  TRY(hipSetDevice(c->device));
  if (seeds && res->n_seeds) TRY(hipMemcpy(seeds, res->seeds, res->n_seeds * sizeof(mbw_seed_t), hipMemcpyDeviceToHost));
  if (pos && res->n_pos) TRY(hipMemcpy(pos, res->pos, res->n_pos * sizeof(uint64_t), hipMemcpyDeviceToHost));
  return MBW_OK;
}
