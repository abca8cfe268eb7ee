// Chaining of variable-length seeds (paper Section 2.6: minibwa chains its SMEMs with minimap2's
// chaining, Li 2018, adapted to seeds of different lengths, and keeps up to 50 chains per read).
//
// Anchors.  Every located (seed, position) pair of a seeding result is an anchor: seed
// P[qbeg, qend) at text position p, span w = qend - qbeg, end (x, y) = (p + w - 1, qend - 1), copy
// g = x / |R| (strand; four copies in a bisulfite index).  A read's anchors are sorted by
// (x, y, w) with two stable device-wide radix sorts: by (y, w), then by (read, x).
//
// Recurrence (exact integers).  f(i) = max(w_i, max_j f(j) + alpha(j,i) - beta(j,i)) over the h
// anchors j before i with g_j = g_i, x_j < x_i, y_j < y_i, x_i - x_j <= G, y_i - y_j <= G;
// alpha = min(x_i - x_j, y_i - y_j, w_i); beta = gamma(|(y_i - y_j) - (x_i - x_j)|) with
// gamma(l) = floor(l * wbar / 100) + floor(floor(log2 l) / 2), gamma(0) = 0, wbar the read's mean
// anchor span rounded down.  The predecessor is the nearest j reaching the maximum when it exceeds
// w_i.  Chains: from anchors in order of descending f (equal f: earlier first), follow the
// predecessors until none is left or the next is already used, marking what is visited; the chain
// scores f(end) minus f of the used anchor it stopped at; chains scoring >= min_score are ranked by
// score (equal scores: earlier end first) and the best max_chains kept.
//
// GPU form: one wave per read.  The recurrence runs over the read's anchors in order with the h
// candidate predecessors spread over the lanes (anchor j stays in lane j mod 64), one DPP wave
// maximum per anchor.  f, predecessors and used flags sit in the wave's LDS area (global memory for
// the rare read with more than 1,024 anchors).  Chains are extracted by repeated wave maxima over
// the unused anchors; the kept chains live one per lane, in rank order, and each lane finally
// writes its chain's anchors by walking the predecessors.  The search stops as soon as no unused
// anchor can reach min_score or displace the last kept chain (a chain never scores above f of its
// end), so a read with many anchors does not pay for chains it cannot keep.
#include <hip/hip_runtime.h>

#include <cstring>

#include <algorithm>
#include <string>

#include "ctx.h"
#include "mbw_internal.h"
#include "prim.h"
#include "../../include/mbw.h"

#define TRY(call) MBW_HIP_TRY(call)

namespace {

struct Anchor { uint64_t x; uint32_t yw; uint32_t g; };   // yw = y << 16 | w (y, w < 2^16)
struct ChainRec { int32_t score; uint32_t end, n, off; };   // end: index of the last anchor in the read

// control words: bad input seeds, the read work counter, guard trips of the chaining kernel, the
// largest anchor count of a read, reads chained from global memory (more than CH_CAP anchors)
enum { CH_BAD = 0, CH_NEXT = 1, CH_GUARD = 2, CH_MAXN = 3, CH_BIG = 4, CH_CTL = 8 };

inline unsigned grid_for(uint64_t n, unsigned bs = 256, unsigned cap = 65536u * 8) {
  uint64_t g = (n + bs - 1) / bs;
  if (g < 1) g = 1;
  return (unsigned)std::min<uint64_t>(g, cap);
}

// Anchors of every (seed, position) pair, their sort keys and the anchor count of every read.
// A wave takes 64 seeds; a seed with few positions is written by its own lane, one with many by
// the whole wave.
#define CH_LANE_MAX 8
__global__ void __launch_bounds__(256) k_ch_anchors(const mbw_seed_t *__restrict__ seeds, uint64_t ns,
                                                    const uint64_t *__restrict__ pos, uint64_t L, uint64_t n_reads,
                                                    int xb, Anchor *__restrict__ A, uint32_t *__restrict__ k2,
                                                    uint64_t *__restrict__ k1, uint32_t *__restrict__ val,
                                                    unsigned long long *__restrict__ rcnt,
                                                    unsigned long long *__restrict__ ctl) {
  const int lane = threadIdx.x & 63;
  const uint64_t nwave = (uint64_t)gridDim.x * (blockDim.x >> 6);
  for (uint64_t base = ((uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 64; base < ns; base += nwave * 64) {
    uint64_t off = 0;
    uint32_t np = 0, rd = 0, qb = 0, qe = 0;
    if (base + lane < ns) {
      const mbw_seed_t sd = seeds[base + lane];
      off = sd.pos_off; np = sd.npos; rd = sd.read_id; qb = sd.qbeg; qe = sd.qend;
      if (rd >= n_reads || qe <= qb || qe > 65535u) { atomicAdd(&ctl[CH_BAD], 1ull); np = 0; }
      if (np) atomicAdd(&rcnt[rd], (unsigned long long)np);
    }
    auto put = [&](uint64_t w, uint32_t read, uint32_t b, uint32_t e) {
      const uint32_t span = e - b;
      const uint64_t x = pos[w] + span - 1;
      const uint32_t yw = ((e - 1) << 16) | span;
      Anchor a;
      a.x = x; a.yw = yw; a.g = (uint32_t)(x / L);
      A[w] = a;
      k2[w] = yw;
      k1[w] = ((uint64_t)read << xb) | x;
      val[w] = (uint32_t)w;
    };
    const bool mine = np <= CH_LANE_MAX;
    if (mine)
      for (uint32_t q = 0; q < np; ++q) put(off + q, rd, qb, qe);
    uint64_t big = __ballot(!mine);
    while (big) {
      const int t = __ffsll((long long)big) - 1;
      big &= big - 1;
      const uint64_t ot = __shfl(off, t);
      const uint32_t nt = (uint32_t)__shfl((int)np, t), rt = (uint32_t)__shfl((int)rd, t);
      const uint32_t bt = (uint32_t)__shfl((int)qb, t), et = (uint32_t)__shfl((int)qe, t);
      for (uint32_t q = (uint32_t)lane; q < nt; q += 64) put(ot + q, rt, bt, et);
    }
  }
}

__global__ void k_ch_gather_k1(const uint64_t *__restrict__ k1, const uint32_t *__restrict__ v, uint64_t n,
                               uint64_t *__restrict__ out) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = k1[v[i]];
}

__global__ void k_ch_gather_anchors(const Anchor *__restrict__ A, const uint32_t *__restrict__ v, uint64_t n,
                                    Anchor *__restrict__ out) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = A[v[i]];
}

// per read: chain slots (at most max_chains, at most the anchor count)
__global__ void k_ch_slots(const unsigned long long *__restrict__ cnt, uint64_t n_reads, uint32_t maxc,
                           unsigned long long *__restrict__ slots) {
  for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r <= n_reads; r += (uint64_t)gridDim.x * blockDim.x)
    slots[r] = r < n_reads ? (cnt[r] < maxc ? cnt[r] : (unsigned long long)maxc) : 0ull;
}

// Values every lane of the wave agrees on are moved into scalar registers (readfirstlane), so that
// the loops and branches they control compile to scalar branches and the wave stays converged: a
// cross-lane read (ds_bpermute) inside a loop the compiler has to treat as divergent could read a
// lane that already left it.
__device__ __forceinline__ uint32_t uni(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni(uint64_t v) {
  return ((uint64_t)uni((uint32_t)(v >> 32)) << 32) | uni((uint32_t)v);
}

// Maximum / minimum of a 32-bit value over the wave with DPP row operations (swap within quads,
// mirror within half rows and rows, then the row broadcasts of 15 and 31), which leave the result
// in lane 63; returned in a scalar register.
template <bool MAX> __device__ __forceinline__ uint32_t dpp_pick(uint32_t a, uint32_t b) {
  return MAX ? (a > b ? a : b) : (a < b ? a : b);
}
template <bool MAX> __device__ __forceinline__ uint32_t wave_reduce_u32(uint32_t v) {
  v = dpp_pick<MAX>(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0xB1, 0xf, 0xf, false));    // quad_perm 1,0,3,2
  v = dpp_pick<MAX>(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x4E, 0xf, 0xf, false));    // quad_perm 2,3,0,1
  v = dpp_pick<MAX>(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x141, 0xf, 0xf, false));   // row_half_mirror
  v = dpp_pick<MAX>(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x140, 0xf, 0xf, false));   // row_mirror
  v = dpp_pick<MAX>(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x142, 0xa, 0xf, false));   // row_bcast:15
  v = dpp_pick<MAX>(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x143, 0xc, 0xf, false));   // row_bcast:31
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ __forceinline__ int64_t chain_gap(int64_t l, int64_t wbar) {
  if (l < 0) l = -l;
  if (l == 0) return 0;
  const int lg = 63 - __clzll((unsigned long long)l);
  return l * wbar / 100 + lg / 2;
}

struct ChainArgs {
  const Anchor *__restrict__ As;        // anchors sorted by (read, x, y, w)
  const unsigned long long *__restrict__ aoff;   // first anchor of every read (n_reads + 1)
  const unsigned long long *__restrict__ cslot;  // first chain slot of every read
  uint64_t n_reads;
  int64_t G;
  int h, maxc, minsc;
  int32_t *__restrict__ F;              // reads with more than CH_CAP anchors: f of every anchor,
  int32_t *__restrict__ P;              // its predecessor (index within the read) or -1,
  uint8_t *__restrict__ U;              // and whether a chain has used it
  ChainRec *__restrict__ CH;            // kept chains, per read from cslot[r]
  uint32_t *__restrict__ CA;            // anchors of the kept chains (index within the read), per read from aoff[r]
  unsigned long long *__restrict__ nch, *__restrict__ nanc;   // per read
  unsigned long long *__restrict__ ctl;    // CH_NEXT: work counter (reads); CH_GUARD: guard trips
  uint64_t na;                             // anchors in total
  uint32_t chunk;                          // reads per grab of the work counter
};

// A read's f, predecessors and used flags live in the wave's LDS area when it has at most CH_CAP
// anchors (nearly all reads), else in the global arrays; either way only the wave that chains the
// read touches them.
#define CH_CAP 1024
#define CH_WAVES 4

// One read: the recurrence, chain extraction and output.  Returns false when a guard bound was
// reached.  Every loop is bounded by the read's anchor count N.
__device__ __forceinline__ bool chain_read(const ChainArgs &a, uint64_t r, uint64_t a0, uint32_t N, int32_t *F, int32_t *P,
                                           uint8_t *U, int lane) {
  const Anchor *As = a.As + a0;
  uint64_t sw = 0;
  for (uint32_t i = lane; i < N; i += 64) sw += As[i].yw & 0xffffu;
  for (int d = 32; d >= 1; d >>= 1) sw += __shfl_xor(sw, d);
  const int64_t wbar = (int64_t)(uni(sw) / N);
  // ---- the recurrence.  Lane t keeps the last anchor j with j = t (mod 64): (x, y, copy, f, j);
  // the h <= 64 candidate predecessors of anchor i are then in distinct lanes and nothing moves
  // between lanes from one anchor to the next.  The anchors themselves stream through registers 64
  // at a time (lane t loads anchor c0 + t; the next chunk is in flight while this one is used) and
  // each step reads its anchor from its lane with readlane.
  uint64_t px = 0;
  uint32_t py = 0, pg = 0;
  int32_t pf = 0;
  int64_t pj = -1;
  Anchor cur = {0, 0, 0}, nxt = {0, 0, 0};
  if ((uint32_t)lane < N) cur = As[lane];
  if (64u + lane < N) nxt = As[64 + lane];
  for (uint32_t c0 = 0; c0 < N; c0 += 64) {
    const uint32_t cnt = N - c0 < 64u ? N - c0 : 64u;
    for (uint32_t t = 0; t < cnt; ++t) {
      const uint32_t i = c0 + t;
      const uint64_t xi = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(cur.x >> 32), (int)t) << 32) |
                          (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)cur.x, (int)t);
      const uint32_t yw = (uint32_t)__builtin_amdgcn_readlane((int)cur.yw, (int)t);
      const uint32_t gi = (uint32_t)__builtin_amdgcn_readlane((int)cur.g, (int)t);
      const uint32_t yi = yw >> 16, wi = yw & 0xffffu;
      uint32_t key = 0;
      if (pj >= 0 && pj >= (int64_t)i - a.h && pg == gi && px < xi && py < yi) {
        const int64_t dx = (int64_t)(xi - px), dy = (int64_t)(yi - py);
        if (dx <= a.G && dy <= a.G) {
          int64_t al = dx < dy ? dx : dy;
          if (al > (int64_t)wi) al = wi;
          const int64_t sc = (int64_t)pf + al - chain_gap(dy - dx, wbar);
          // sc <= f_j + w_i < 2^17: it fits with the predecessor's distance in 32 bits;
          // equal scores: the nearer predecessor (larger j) wins
          if (sc > (int64_t)wi) key = ((uint32_t)sc << 6) | (uint32_t)(pj + 64 - (int64_t)i);
        }
      }
      key = wave_reduce_u32<true>(key);
      int32_t fi = (int32_t)wi, pi = -1;
      if (key) { fi = (int32_t)(key >> 6); pi = (int32_t)i - 64 + (int32_t)(key & 63); }
      if ((uint32_t)lane == t) {
        F[i] = fi; P[i] = pi; U[i] = 0;
        px = xi; py = yi; pg = gi; pf = fi; pj = i;
      }
    }
    cur = nxt;
    if (c0 + 128 + lane < N) nxt = As[c0 + 128 + lane];
  }
  __threadfence_block();   // f, p and cleared flags written by one lane each are read by every lane below
  // ---- chains, in order of descending f; the kept ones one per lane in rank order
  int nc = 0;
  int32_t cs = 0;
  uint32_t ce = 0, cn = 0;
  for (uint32_t round = 0;; ++round) {
    if (round > N) return false;   // every round uses at least one anchor
    // the unused anchor of largest f (equal f: smallest index): f first, then the index
    uint32_t bf = 0, bi = 0xffffffffu;
    for (uint32_t i = lane; i < N; i += 64) {
      const uint32_t f = U[i] ? 0u : (uint32_t)F[i];   // f >= 1
      if (f > bf) { bf = f; bi = i; }                  // i grows: the first of equal f is kept
    }
    const uint32_t fmax = wave_reduce_u32<true>(bf);
    if (!fmax) break;
    const uint32_t im = wave_reduce_u32<false>(bf == fmax ? bi : 0xffffffffu);
    const int32_t fm = (int32_t)fmax;
    if (fm < a.minsc) break;                                       // no chain can reach min_score
    if (nc == a.maxc) {
      // a new chain scores <= fm and ranks before the last kept one only with a higher score, or
      // an equal one and an earlier end; later candidates have smaller f, or equal f and a later end
      const int32_t last = uni(__shfl(cs, a.maxc - 1));
      const uint32_t last_end = uni((uint32_t)__shfl((int)ce, a.maxc - 1));
      if (fm < last || (fm == last && im > last_end)) break;
    }
    int32_t sc = fm;
    uint32_t n = 0, bad = 0;
    if (lane == 0) {
      uint32_t k = im;
      for (;;) {
        U[k] = 1;
        ++n;
        const int32_t pk = P[k];
        if (pk < 0) break;
        if ((uint32_t)pk >= k || n >= N) { bad = 1; break; }   // predecessors lie strictly before
        if (U[pk]) { sc = fm - F[pk]; break; }
        k = (uint32_t)pk;
      }
    }
    __threadfence_block();
    if (uni((uint32_t)__shfl((int)bad, 0))) return false;
    sc = uni(__shfl(sc, 0));
    n = uni((uint32_t)__shfl((int)n, 0));
    if (sc >= a.minsc) {
      const bool before = lane < nc && (cs > sc || (cs == sc && ce < im));
      const int q = (int)uni((uint32_t)__popcll(__ballot(before)));
      const int32_t us = __shfl_up(cs, 1);
      const uint32_t ue = __shfl_up(ce, 1), un = __shfl_up(cn, 1);
      if (lane > q) { cs = us; ce = ue; cn = un; }
      if (lane == q) { cs = sc; ce = im; cn = n; }
      nc = nc < a.maxc ? nc + 1 : a.maxc;
    }
  }
  // ---- output: chain records and each chain's anchors (walked back from its end)
  uint32_t mine = lane < nc ? cn : 0u, off = mine;
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t o = (uint32_t)__shfl_up((int)off, d);
    if (lane >= d) off += o;
  }
  const uint32_t total = uni((uint32_t)__shfl((int)off, 63));
  off -= mine;
  bool ok = true;
  if (lane < nc) {
    ChainRec c;
    c.score = cs; c.end = ce; c.n = cn; c.off = off;
    a.CH[a.cslot[r] + lane] = c;
    uint32_t k = ce;
    for (uint32_t m = cn; m-- > 0;) {   // cn <= N, and every k stays below N (checked when walked above)
      a.CA[a0 + off + m] = k;
      if (m) k = (uint32_t)P[k];
      if (k >= N) { ok = false; break; }
    }
  }
  if (__ballot(!ok)) return false;
  if (lane == 0) { a.nch[r] = (unsigned long long)nc; a.nanc[r] = total; }
  return true;
}

__global__ void __launch_bounds__(64 * CH_WAVES) k_chain(ChainArgs a) {
  // Every loop has a hard bound taken from the validated anchor count N of the read; a bound that is
  // reached marks CH_GUARD and ends the work of the wave on that read, so a corrupt input can only
  // produce an error, never a runaway loop.  Waves take `chunk` reads per grab of the work counter
  // (device-scope atomics on one address serialise: one per read would cost more than the work).
  __shared__ int32_t sF[CH_WAVES][CH_CAP], sP[CH_WAVES][CH_CAP];
  __shared__ uint8_t sU[CH_WAVES][CH_CAP];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t maxn = 0, big = 0;
  for (uint64_t grab = 0; grab <= a.n_reads; ++grab) {
    unsigned long long t = 0;
    if (lane == 0) t = atomicAdd(&a.ctl[CH_NEXT], (unsigned long long)a.chunk);
    const uint64_t r0 = uni((uint64_t)__shfl(t, 0));
    if (r0 >= a.n_reads) break;
    const uint64_t r1 = r0 + a.chunk < a.n_reads ? r0 + a.chunk : a.n_reads;
    for (uint64_t r = r0; r < r1; ++r) {
      const uint64_t a0 = uni((uint64_t)a.aoff[r]);
      const uint64_t a1 = uni((uint64_t)a.aoff[r + 1]);
      if (a1 < a0 || a1 > a.na) {
        if (lane == 0) { atomicOr(&a.ctl[CH_GUARD], 1ull); a.nch[r] = 0; a.nanc[r] = 0; }
        continue;
      }
      const uint32_t N = (uint32_t)(a1 - a0);
      if (N == 0) {
        if (lane == 0) { a.nch[r] = 0; a.nanc[r] = 0; }
        continue;
      }
      maxn = N > maxn ? N : maxn;
      big += N > CH_CAP ? 1u : 0u;
      const bool ok = N <= CH_CAP ? chain_read(a, r, a0, N, sF[wv], sP[wv], sU[wv], lane)
                                  : chain_read(a, r, a0, N, a.F + a0, a.P + a0, a.U + a0, lane);
      if (!ok && lane == 0) { atomicOr(&a.ctl[CH_GUARD], 2ull); a.nch[r] = 0; a.nanc[r] = 0; }
    }
  }
  if (lane == 0 && maxn) {
    atomicMax(&a.ctl[CH_MAXN], (unsigned long long)maxn);
    if (big) atomicAdd(&a.ctl[CH_BIG], (unsigned long long)big);
  }
}

// final records: one wave per read
__global__ void __launch_bounds__(256) k_ch_emit(const Anchor *__restrict__ As, const unsigned long long *__restrict__ aoff,
                                                 const unsigned long long *__restrict__ cslot, const ChainRec *__restrict__ CH,
                                                 const uint32_t *__restrict__ CA, const unsigned long long *__restrict__ nch,
                                                 const unsigned long long *__restrict__ nanc,
                                                 const unsigned long long *__restrict__ choff,
                                                 const unsigned long long *__restrict__ anoff, uint64_t n_reads,
                                                 mbw_chain_t *__restrict__ chains, mbw_anchor_t *__restrict__ anchors) {
  const int lane = threadIdx.x & 63;
  const uint64_t nwave = (uint64_t)gridDim.x * (blockDim.x >> 6);
  for (uint64_t r = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); r < n_reads; r += nwave) {
    const uint64_t a0 = aoff[r], cb = choff[r], ab = anoff[r];
    const uint32_t nc = (uint32_t)nch[r], na = (uint32_t)nanc[r];
    for (uint32_t q = lane; q < nc; q += 64) {
      const ChainRec c = CH[cslot[r] + q];
      mbw_chain_t o;
      o.read_id = (uint32_t)r; o.n_anchors = c.n; o.score = c.score; o.copy = As[a0 + c.end].g;
      o.anchor_off = ab + c.off;
      chains[cb + q] = o;
    }
    for (uint32_t m = lane; m < na; m += 64) {
      const Anchor A = As[a0 + CA[a0 + m]];
      const uint32_t y = A.yw >> 16, w = A.yw & 0xffffu;
      mbw_anchor_t o;
      o.qbeg = y + 1 - w; o.qend = y + 1; o.pos = A.x + 1 - w;
      anchors[ab + m] = o;
    }
  }
}

}  // namespace

extern "C" int mbw_chain(mbw_ctx *c, const mbw_result *res, uint64_t n_reads, const mbw_chain_opts *opts, void *stream,
                         mbw_chain_result *out) {
  if (!c || !res || !out) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  memset(out, 0, sizeof(*out));
  mbw_chain_opts o;
  if (opts) o = *opts;
  else { o.max_gap = 5000; o.max_pred = 50; o.max_chains = 50; o.min_score = 19; }
  if (o.max_gap < 1 || o.max_pred < 1 || o.max_pred > 64 || o.max_chains < 1 || o.max_chains > 64) {
    mbw_set_error("chain options: max_gap >= 1, max_pred and max_chains in 1..64"); return MBW_E_INVAL;
  }
  if (n_reads >= (1ull << 31)) { mbw_set_error("too many reads"); return MBW_E_INVAL; }
  if ((res->n_seeds && !res->seeds) || (res->n_pos && !res->pos)) { mbw_set_error("result without arrays"); return MBW_E_INVAL; }
  const uint64_t na = res->n_pos, ns = res->n_seeds;
  if (na >= (1ull << 32)) { mbw_set_error("more than 2^32 anchors in one call"); return MBW_E_INVAL; }
  const mbw_index *ix = c->ix;
  int xb = 1, rb = 1;
  while (xb < 64 && (1ull << xb) < ix->n) ++xb;
  while (rb < 63 && (1ull << rb) <= n_reads) ++rb;
  if (xb + rb > 64) { mbw_set_error("too many reads for the anchor sort keys of this index"); return MBW_E_INVAL; }
  TRY(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  c->cur = st;
  TRY(hipEventRecord(c->ev[0], st));
  GROW(c->ch_ctl, CH_CTL * 8);
  unsigned long long *ctl = (unsigned long long *)c->ch_ctl.p;
  TRY(hipMemsetAsync(ctl, 0, CH_CTL * 8, st));
  GROW(c->ch_cnt, (n_reads + 1) * 8);
  GROW(c->ch_aoff, (n_reads + 1) * 8);
  GROW(c->ch_slot, (n_reads + 1) * 8);
  GROW(c->ch_cslot, (n_reads + 1) * 8);
  unsigned long long *cnt = (unsigned long long *)c->ch_cnt.p, *aoff = (unsigned long long *)c->ch_aoff.p;
  unsigned long long *slot = (unsigned long long *)c->ch_slot.p, *cslot = (unsigned long long *)c->ch_cslot.p;
  TRY(hipMemsetAsync(cnt, 0, (n_reads + 1) * 8, st));
  GROW(c->ch_A, (na + 1) * sizeof(Anchor));
  GROW(c->ch_As, (na + 1) * sizeof(Anchor));
  GROW(c->ch_k2a, (na + 1) * 4); GROW(c->ch_k2b, (na + 1) * 4);
  GROW(c->ch_k1a, (na + 1) * 8); GROW(c->ch_k1b, (na + 1) * 8);
  GROW(c->ch_va, (na + 1) * 4); GROW(c->ch_vb, (na + 1) * 4);
  Anchor *A = (Anchor *)c->ch_A.p, *As = (Anchor *)c->ch_As.p;
  uint32_t *k2a = (uint32_t *)c->ch_k2a.p, *k2b = (uint32_t *)c->ch_k2b.p;
  uint64_t *k1a = (uint64_t *)c->ch_k1a.p, *k1b = (uint64_t *)c->ch_k1b.p;
  uint32_t *va = (uint32_t *)c->ch_va.p, *vb = (uint32_t *)c->ch_vb.p;
  if (ns) {
    k_ch_anchors<<<grid_for((ns + 63) / 64 * 64 / 4, 256, 65536u), 256, 0, st>>>(res->seeds, ns, res->pos, ix->len_r, n_reads,
                                                                              xb, A, k2a, k1a, va, cnt, ctl);
    TRY(hipGetLastError());
  }
  int r = 0;
  const uint32_t *order = va;   // anchor indices in (read, x, y, w) order
  if (na > 1) {
    // (y, w), then (read, x): both stable, so the anchors end up in (read, x, y, w) order
    prim::dbuf<uint32_t> kb2(k2a, k2b), vb2(va, vb);
    r = prim_call(c, [&](void *tp, size_t &tb) { return prim::sort_pairs(tp, tb, kb2, vb2, na, 0, 32, st); });
    if (r) return r;
    k_ch_gather_k1<<<grid_for(na), 256, 0, st>>>(k1a, vb2.current(), na, k1b);
    TRY(hipGetLastError());
    prim::dbuf<uint64_t> kb1(k1b, k1a);
    prim::dbuf<uint32_t> vb1(vb2.current(), vb2.alternate());
    r = prim_call(c, [&](void *tp, size_t &tb) {
      return prim::sort_pairs(tp, tb, kb1, vb1, na, 0, xb + rb, st);
    });
    if (r) return r;
    order = vb1.current();
  }
  if (na) {
    k_ch_gather_anchors<<<grid_for(na), 256, 0, st>>>(A, order, na, As);   // one anchor: va[0] = 0 from the anchor kernel
    TRY(hipGetLastError());
  }
  r = prim_call(c, [&](void *tp, size_t &tb) { return prim::exclusive_sum(tp, tb, cnt, aoff, n_reads + 1, st); });
  if (r) return r;
  k_ch_slots<<<grid_for(n_reads + 1), 256, 0, st>>>(cnt, n_reads, (uint32_t)o.max_chains, slot);
  TRY(hipGetLastError());
  r = prim_call(c, [&](void *tp, size_t &tb) { return prim::exclusive_sum(tp, tb, slot, cslot, n_reads + 1, st); });
  if (r) return r;
  {
    // the per-read ranges must tile the anchors exactly before the chaining kernel relies on them
    uint64_t chk[3] = {0, 0, 0};
    TRY(hipMemcpyAsync(&chk[0], aoff + n_reads, 8, hipMemcpyDeviceToHost, st));
    TRY(hipMemcpyAsync(&chk[1], cslot + n_reads, 8, hipMemcpyDeviceToHost, st));
    TRY(hipMemcpyAsync(&chk[2], ctl + CH_BAD, 8, hipMemcpyDeviceToHost, st));
    TRY(hipStreamSynchronize(st));
    if (chk[2]) { mbw_set_error("seeds with a read id >= n_reads or an empty or over-long interval"); return MBW_E_INVAL; }
    if (chk[0] != na || chk[1] > std::min<uint64_t>(na, n_reads * (uint64_t)o.max_chains)) {
      mbw_set_error("internal: anchor ranges do not cover the anchors"); return MBW_E_HIP;
    }
  }
  // slots in total: at most max_chains per read
  const uint64_t slots_cap = std::min<uint64_t>(na, n_reads * (uint64_t)o.max_chains) + 1;
  GROW(c->ch_F, (na + 1) * 4); GROW(c->ch_P, (na + 1) * 4); GROW(c->ch_U, na + 1);
  GROW(c->ch_CH, slots_cap * sizeof(ChainRec)); GROW(c->ch_CA, (na + 1) * 4);
  GROW(c->ch_nch, (n_reads + 1) * 8); GROW(c->ch_nanc, (n_reads + 1) * 8);
  GROW(c->ch_choff, (n_reads + 1) * 8); GROW(c->ch_anoff, (n_reads + 1) * 8);
  unsigned long long *nch = (unsigned long long *)c->ch_nch.p, *nanc = (unsigned long long *)c->ch_nanc.p;
  unsigned long long *choff = (unsigned long long *)c->ch_choff.p, *anoff = (unsigned long long *)c->ch_anoff.p;
  TRY(hipMemsetAsync(nch + n_reads, 0, 8, st));
  TRY(hipMemsetAsync(nanc + n_reads, 0, 8, st));
  ChainArgs ca;
  ca.As = As; ca.aoff = aoff; ca.cslot = cslot; ca.n_reads = n_reads; ca.G = o.max_gap; ca.h = o.max_pred;
  ca.maxc = o.max_chains; ca.minsc = o.min_score;
  ca.F = (int32_t *)c->ch_F.p; ca.P = (int32_t *)c->ch_P.p; ca.U = (uint8_t *)c->ch_U.p;
  ca.CH = (ChainRec *)c->ch_CH.p; ca.CA = (uint32_t *)c->ch_CA.p; ca.nch = nch; ca.nanc = nanc; ca.ctl = ctl; ca.na = na;
  TRY(hipEventRecord(c->ev[1], st));
  if (n_reads) {
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)k_chain, 64 * CH_WAVES, 0) != hipSuccess || per < 1)
      per = 4;
    const uint64_t grid = std::min<uint64_t>((n_reads + CH_WAVES - 1) / CH_WAVES, (uint64_t)per * c->n_cu);
    // about 16 grabs per wave, at most 64 reads each, so that reads with many anchors still spread
    ca.chunk = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(64, n_reads / (grid * CH_WAVES * 16)));
    k_chain<<<(unsigned)grid, 64 * CH_WAVES, 0, st>>>(ca);
    TRY(hipGetLastError());
  }
  TRY(hipEventRecord(c->ev[2], st));
  r = prim_call(c, [&](void *tp, size_t &tb) { return prim::exclusive_sum(tp, tb, nch, choff, n_reads + 1, st); });
  if (r) return r;
  r = prim_call(c, [&](void *tp, size_t &tb) { return prim::exclusive_sum(tp, tb, nanc, anoff, n_reads + 1, st); });
  if (r) return r;
  uint64_t h[5] = {0, 0, 0, 0, 0};
  TRY(hipMemcpyAsync(&h[3], ctl + CH_MAXN, 16, hipMemcpyDeviceToHost, st));
  TRY(hipMemcpyAsync(&h[0], ctl + CH_GUARD, 8, hipMemcpyDeviceToHost, st));
  TRY(hipMemcpyAsync(&h[1], choff + n_reads, 8, hipMemcpyDeviceToHost, st));
  TRY(hipMemcpyAsync(&h[2], anoff + n_reads, 8, hipMemcpyDeviceToHost, st));
  TRY(hipStreamSynchronize(st));
  if (h[0]) { mbw_set_error("chaining kernel guard tripped (" + std::to_string(h[0]) + ")"); return MBW_E_HIP; }
  const uint64_t n_chains = h[1], n_anch = h[2];
  GROW(c->ch_out, (n_chains + 1) * sizeof(mbw_chain_t));
  GROW(c->ch_outa, (n_anch + 1) * sizeof(mbw_anchor_t));
  if (n_reads) {
    k_ch_emit<<<grid_for((n_reads + 3) / 4 * 256, 256, 65536u), 256, 0, st>>>(As, aoff, cslot, ca.CH, ca.CA, nch, nanc, choff,
                                                                            anoff, n_reads, (mbw_chain_t *)c->ch_out.p,
                                                                            (mbw_anchor_t *)c->ch_outa.p);
    TRY(hipGetLastError());
  }
  TRY(hipEventRecord(c->ev[3], st));
  TRY(hipEventSynchronize(c->ev[3]));
  float tk = 0, tt = 0;
  (void)hipEventElapsedTime(&tk, c->ev[1], c->ev[2]);
  (void)hipEventElapsedTime(&tt, c->ev[0], c->ev[3]);
  out->n_chains = n_chains;
  out->n_anchors = n_anch;
  out->n_input_anchors = na;
  out->chains = (const mbw_chain_t *)c->ch_out.p;
  out->anchors = (const mbw_anchor_t *)c->ch_outa.p;
  out->ms_kernel = tk;
  out->ms_total = tt;
  out->max_read_anchors = h[3];
  out->reads_over_lds = h[4];
  return MBW_OK;
}

extern "C" int mbw_chain_download(mbw_ctx *c, const mbw_chain_result *res, mbw_chain_t *chains, mbw_anchor_t *anchors) {
  if (!c || !res) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  TRY(hipSetDevice(c->device));
  if (chains && res->n_chains)
    TRY(hipMemcpyAsync(chains, res->chains, res->n_chains * sizeof(mbw_chain_t), hipMemcpyDeviceToHost, c->cur));
  if (anchors && res->n_anchors)
    TRY(hipMemcpyAsync(anchors, res->anchors, res->n_anchors * sizeof(mbw_anchor_t), hipMemcpyDeviceToHost, c->cur));
  TRY(hipStreamSynchronize(c->cur));
  return MBW_OK;
}
