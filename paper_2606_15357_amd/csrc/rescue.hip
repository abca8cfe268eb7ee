// Mate-rescue prefilter (paper Section 2.7).
//
// For a candidate (read P, window W of the index text), M_t is the number of pairs (i, j) with
// P[i, i+q) = W[j, j+q) and j - i = t; Smith-Waterman is worth starting only when max_t M_t is
// large enough.  One wave owns one candidate at a time and works in its own LDS area:
//   1. read planes   the read's 2-bit codes become a low-bit plane, a high-bit plane and an N
//                    plane, 64 bases per wave ballot;
//   2. window planes each lane splits one 32-base text word into its low and high bits;
//   3. table         every read q-mer without N (key = low bits | high bits << q) is inserted into
//                    an open-addressing hash table whose slots chain the read positions of the key,
//                    and marked in a 2^14-bit presence filter (indexed by the key itself for q <= 7,
//                    so exact there; by a hash of it above);
//   4. diagonals     every window q-mer whose filter bit is set looks its key up and adds one to
//                    the (16-bit) counter of diagonal j - i for each read position i in the chain;
//   5. reduce        (max counter, smallest diagonal holding it) over the wave.
// The work per candidate is O(|P| + |W| + matching pairs) rather than the O(|P| |W|) of testing
// every diagonal; the pass list is a device-wide selection of candidates with max >= min_hits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>

#include "ctx.h"
#include "mbw_internal.h"
#include "prim.h"
#include "../../include/mbw.h"

#define TRY(call) MBW_HIP_TRY(call)

namespace {

constexpr uint32_t RC_NONE = 0xFFFFFFFFu;   // end of a position chain / empty head
constexpr size_t RC_MAX_LDS = 64 * 1024;    // per wave (one wave per workgroup)
enum { RC_BAD = 0, RC_MAXLEN = 1, RC_MAXWIN = 2, RC_NSEL = 3, RC_ERR = 4, RC_CTL = 8 };

struct RescueArgs {
  const uint8_t *__restrict__ reads;
  const uint64_t *__restrict__ offs;
  uint64_t n_reads;
  const mbw_rescue_cand_t *__restrict__ cand;
  uint64_t n_cand;
  const uint64_t *__restrict__ text;   // 2 bits per base, 32 bases per word
  uint64_t m;                          // text symbols (n - 1)
  int q, role;
  uint32_t min_hits;
  uint32_t tbits;                      // log2 of the hash table slots
  uint32_t cap_p, cap_w;               // LDS capacity: read and window bases
  mbw_rescue_hit_t *__restrict__ hits;
  uint8_t *__restrict__ flags;
  unsigned long long *__restrict__ ctl;
};

// LDS areas of one wave, in 32-bit words; every area starts on a 16-byte boundary and spans a
// multiple of four words (cleared and scanned with 16-byte accesses)
constexpr uint32_t RC_FBITS = 14;                     // presence filter: 2^14 bits
constexpr uint32_t RC_FWORDS = (1u << RC_FBITS) / 32;

struct RcLayout {
  uint32_t ts, cw, rw, ww;
  uint32_t key, head, filt, next, cnt, rlo, rhi, rn, wlo, whi, total;
};

__host__ __device__ inline uint32_t rc_up4(uint32_t x) { return (x + 3) & ~3u; }

__host__ __device__ inline RcLayout rc_layout(uint32_t tbits, uint32_t cap_p, uint32_t cap_w) {
  RcLayout L;
  L.ts = 1u << tbits;
  L.cw = rc_up4((cap_p + cap_w + 1) / 2);       // two 16-bit diagonal counters per word
  L.rw = rc_up4(2 * ((cap_p + 63) / 64) + 2);   // read planes: two words per 64 bases + padding
  L.ww = rc_up4((cap_w + 63) / 32 + 2);         // window planes: the window may start at bit 31
  L.key = 0;
  L.head = L.key + L.ts;
  L.filt = L.head + L.ts;
  L.next = L.filt + RC_FWORDS;
  L.cnt = L.next + rc_up4(cap_p);
  L.rlo = L.cnt + L.cw;
  L.rhi = L.rlo + L.rw;
  L.rn = L.rhi + L.rw;
  L.wlo = L.rn + L.rw;
  L.whi = L.wlo + L.ww;
  L.total = L.whi + L.ww;
  return L;
}

// A0 C1 G2 T3 from ASCII without branches: bits 1-2 of the letter are 0, 1, 3, 2 for A, C, G, T
// (either case); anything else is 4
__device__ __forceinline__ uint32_t rc_code(uint32_t ch, int role) {
  const uint32_t u = ch | 0x20u;
  const bool ok = (u == 'a') | (u == 'c') | (u == 'g') | (u == 't');
  const uint32_t x = (ch >> 1) & 3u;
  uint32_t c = x ^ (x >> 1);
  c = (role == 1 && c == 1) ? 3u : c;   // read 1 of a bisulfite pair: C -> T
  c = (role == 2 && c == 2) ? 0u : c;   // read 2: G -> A
  return ok ? c : 4u;
}

// the even (low code) bits of a 32-base text word, packed into 32 bits
__device__ __forceinline__ uint32_t even_bits(uint64_t x) {
  x &= 0x5555555555555555ull;
  x = (x | (x >> 1)) & 0x3333333333333333ull;
  x = (x | (x >> 2)) & 0x0F0F0F0F0F0F0F0Full;
  x = (x | (x >> 4)) & 0x00FF00FF00FF00FFull;
  x = (x | (x >> 8)) & 0x0000FFFF0000FFFFull;
  x = (x | (x >> 16)) & 0x00000000FFFFFFFFull;
  return (uint32_t)x;
}

// bits [b, b + 32) of a plane of 32-bit words
__device__ __forceinline__ uint32_t plane_bits(const uint32_t *pl, uint32_t b) {
  return __builtin_amdgcn_alignbit(pl[(b >> 5) + 1], pl[b >> 5], b & 31);
}

// workgroup barrier that orders LDS only (global loads issued before it stay in flight)
__device__ __forceinline__ void rc_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ uint32_t rc_hash(uint32_t key, uint32_t tbits) {
  return (key * 0x9E3779B1u) >> (32 - tbits);
}

__global__ void __launch_bounds__(64) k_rescue(RescueArgs A) {
  extern __shared__ uint4 lds4[];
  uint32_t *lds = (uint32_t *)lds4;
  const RcLayout L = rc_layout(A.tbits, A.cap_p, A.cap_w);
  uint32_t *key = lds + L.key, *head = lds + L.head, *filt = lds + L.filt, *next = lds + L.next, *cnt = lds + L.cnt;
  uint32_t *rlo = lds + L.rlo, *rhi = lds + L.rhi, *rn = lds + L.rn, *wlo = lds + L.wlo, *whi = lds + L.whi;
  const uint32_t lane = threadIdx.x;
  const uint32_t q = (uint32_t)A.q, qm = (1u << q) - 1, tmask = L.ts - 1;
  const bool direct = 2 * q <= RC_FBITS;   // the filter is indexed by the key itself
  const uint4 zero4 = make_uint4(0, 0, 0, 0), none4 = make_uint4(RC_NONE, RC_NONE, RC_NONE, RC_NONE);

  for (uint64_t ci = blockIdx.x; ci < A.n_cand; ci += gridDim.x) {
    const mbw_rescue_cand_t cd = A.cand[ci];
    uint64_t o0 = 0, o1 = 0;
    if (cd.read_id < A.n_reads) { o0 = A.offs[cd.read_id]; o1 = A.offs[cd.read_id + 1]; }
    const uint64_t rb = o0, np = o1 - o0;
    const uint64_t nw = cd.win_len;
    const bool bad = cd.read_id >= A.n_reads || cd.win_beg > A.m || nw > A.m - cd.win_beg || np > A.cap_p ||
                     nw > A.cap_w;
    if (bad || np < q || nw < q) {   // (the host rejects bad candidates before the launch)
      if (lane == 0) {
        A.hits[ci].max_hits = 0;
        A.hits[ci].best_t = 0;
        A.flags[ci] = !bad && A.min_hits == 0;
        if (bad) atomicAdd(&A.ctl[RC_ERR], 1ull);
      }
      continue;
    }
    // 1. window text words (in flight while the read is encoded): words covering
    //    [win_beg, win_beg + nw), window base j at bit s0 + j of the planes
    const uint64_t wb = cd.win_beg >> 5;
    const uint32_t s0 = (uint32_t)(cd.win_beg & 31);
    const uint32_t nww = (uint32_t)((s0 + nw + 31) >> 5);
    const uint64_t tw0 = lane < nww ? A.text[wb + lane] : 0ull;
    // 2. read planes, 256 bases per round: four coalesced byte loads per lane (address clamped
    //    into the read, so all are issued before one wait), then one ballot per plane and 64
    //    bases (positions past the read count as N).  The first round is peeled off the loop so
    //    that its loads overlap the text load.
    const uint32_t nchunk = (uint32_t)((np + 63) / 64);
    auto read_round = [&](uint32_t k0) {
      uint32_t c[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint64_t p = (uint64_t)(k0 + u) * 64 + lane;
        c[u] = A.reads[rb + (p < np ? p : np - 1)];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool in = (uint64_t)(k0 + u) * 64 + lane < np;
        const uint32_t cu = in ? rc_code(c[u], A.role) : 4u;
        if (k0 + u < nchunk) {
          const uint64_t blo = __ballot(cu < 4 && (cu & 1)), bhi = __ballot(cu < 4 && (cu & 2));
          const uint64_t bn = __ballot(cu >= 4);
          if (lane < 2) {
            const uint32_t k = 2 * (k0 + u) + lane;
            rlo[k] = (uint32_t)(blo >> (32 * lane));
            rhi[k] = (uint32_t)(bhi >> (32 * lane));
            rn[k] = (uint32_t)(bn >> (32 * lane));
          }
        }
      }
    };
    read_round(0);
    for (uint32_t k0 = 4; k0 < nchunk; k0 += 4) read_round(k0);
    if (lane < 2) { rlo[2 * nchunk + lane] = 0; rhi[2 * nchunk + lane] = 0; rn[2 * nchunk + lane] = RC_NONE; }
    if (lane < nww) { wlo[lane] = even_bits(tw0); whi[lane] = even_bits(tw0 >> 1); }
    for (uint32_t k = lane + 64; k < nww; k += 64) {
      const uint64_t x = A.text[wb + k];
      wlo[k] = even_bits(x);
      whi[k] = even_bits(x >> 1);
    }
    if (lane == 0) { wlo[nww] = 0; whi[nww] = 0; }
    // 3. clear the table, the filter and the diagonal counters (diagonal t at t + |P| - q, two
    //    16-bit counters per word)
    const uint32_t base = (uint32_t)np - q;
    const uint32_t nd = (uint32_t)(np + nw) - 2 * q + 1;
    for (uint32_t k = lane; k < L.ts / 4; k += 64) { lds4[L.key / 4 + k] = zero4; lds4[L.head / 4 + k] = none4; }
    for (uint32_t k = lane; k < RC_FWORDS / 4; k += 64) lds4[L.filt / 4 + k] = zero4;
    const uint32_t ncw4 = ((nd + 1) / 2 + 3) / 4;
    for (uint32_t k = lane; k < ncw4; k += 64) lds4[L.cnt / 4 + k] = zero4;
    rc_sync();
    // 4. insert the read's q-mers
    for (uint32_t i = lane; i + q <= (uint32_t)np; i += 64) {
      if (plane_bits(rn, i) & qm) continue;
      const uint32_t code = (plane_bits(rlo, i) & qm) | ((plane_bits(rhi, i) & qm) << q);
      const uint32_t kk = code + 1;
      const uint32_t f = direct ? code : rc_hash(kk, RC_FBITS);
      atomicOr(&filt[f >> 5], 1u << (f & 31));
      uint32_t s = rc_hash(kk, A.tbits);
      for (uint32_t g = 0; g < L.ts; ++g) {   // more slots than read positions: an empty one exists
        const uint32_t old = atomicCAS(&key[s], 0u, kk);
        if (old == 0u || old == kk) break;
        s = (s + 1) & tmask;
      }
      next[i] = atomicExch(&head[s], i);
    }
    rc_sync();
    // 5. look up the window's q-mers whose filter bit is set, count per diagonal
    for (uint32_t j = lane; j + q <= (uint32_t)nw; j += 64) {
      const uint32_t b = s0 + j;
      const uint32_t code = (plane_bits(wlo, b) & qm) | ((plane_bits(whi, b) & qm) << q);
      const uint32_t kk = code + 1;
      const uint32_t f = direct ? code : rc_hash(kk, RC_FBITS);
      if (!((filt[f >> 5] >> (f & 31)) & 1u)) continue;
      uint32_t s = rc_hash(kk, A.tbits);
      for (uint32_t g = 0; g < L.ts; ++g) {
        const uint32_t k = key[s];
        if (k == 0u) break;
        if (k == kk) {   // a chain holds distinct read positions i <= |P| - q
          uint32_t i = head[s];
          for (uint32_t h = 0; i <= base && h <= base; ++h) {
            const uint32_t x = j - i + base;
            atomicAdd(&cnt[x >> 1], 1u << (16 * (x & 1)));
            i = next[i];
          }
          break;
        }
        s = (s + 1) & tmask;
      }
    }
    rc_sync();
    // 6. max over the diagonals, smallest t on ties (8 counters per lane and step, ascending)
    uint32_t bv = 0, bx = RC_NONE;
    for (uint32_t k = lane; k < ncw4; k += 64) {
      const uint4 v = lds4[L.cnt / 4 + k];
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t lo = w[u] & 0xFFFFu, hi = w[u] >> 16;
        if (lo > bv) { bv = lo; bx = 8 * k + 2 * u; }
        if (hi > bv) { bv = hi; bx = 8 * k + 2 * u + 1; }
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const uint32_t ov = __shfl_xor(bv, off), ox = __shfl_xor(bx, off);
      if (ov > bv || (ov == bv && ox < bx)) { bv = ov; bx = ox; }
    }
    if (lane == 0) {
      A.hits[ci].max_hits = bv;
      A.hits[ci].best_t = bv ? (int32_t)bx - (int32_t)base : 0;
      A.flags[ci] = bv >= A.min_hits;
    }
    rc_sync();   // the next candidate reuses the LDS area
  }
}

__global__ void k_rc_widen(const uint32_t *__restrict__ len, uint64_t n, uint64_t *__restrict__ wide,
                           unsigned long long *__restrict__ ctl) {
  uint32_t mx = 0;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i <= n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t v = i < n ? len[i] : 0u;
    wide[i] = v;
    mx = v > mx ? v : mx;
  }
  if (mx) atomicMax(&ctl[RC_MAXLEN], (unsigned long long)mx);
}

__global__ void k_rc_check(const mbw_rescue_cand_t *__restrict__ cand, uint64_t n, uint64_t n_reads, uint64_t m,
                           unsigned long long *__restrict__ ctl) {
  uint32_t mx = 0, bad = 0;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const mbw_rescue_cand_t c = cand[i];
    if (c.read_id >= n_reads || c.win_beg > m || c.win_len > m - c.win_beg) ++bad;
    mx = c.win_len > mx ? c.win_len : mx;
  }
  if (bad) atomicAdd(&ctl[RC_BAD], (unsigned long long)bad);
  if (mx) atomicMax(&ctl[RC_MAXWIN], (unsigned long long)mx);
}

inline unsigned rc_grid(uint64_t n, unsigned bs = 256, unsigned cap = 4096) {
  uint64_t g = (n + bs - 1) / bs;
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(g, cap));
}

}  // namespace

extern "C" int mbw_rescue_filter(mbw_ctx *c, const uint8_t *reads, const uint32_t *lengths, uint64_t n_reads,
                                 const mbw_rescue_cand_t *cands, uint64_t n_cands, const mbw_rescue_opts *opts,
                                 void *stream, mbw_rescue_result *out) {
  if (!c || !out) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  memset(out, 0, sizeof(*out));
  mbw_rescue_opts o;
  if (opts) o = *opts;
  else { o.q = 7; o.min_hits = 10; o.bs_role = 0; }
  if (o.q < 1 || o.q > 15) { mbw_set_error("q must be in 1..15"); return MBW_E_INVAL; }
  if (o.min_hits < 0) { mbw_set_error("min_hits must be >= 0"); return MBW_E_INVAL; }
  if (o.bs_role < 0 || o.bs_role > 2) { mbw_set_error("bs_role must be 0, 1 or 2"); return MBW_E_INVAL; }
  if (o.bs_role && !c->ix->bisulfite) { mbw_set_error("bs_role needs a bisulfite index"); return MBW_E_INVAL; }
  if (n_cands && !cands) { mbw_set_error("NULL candidates"); return MBW_E_INVAL; }
  if (n_reads && (!reads || !lengths)) { mbw_set_error("NULL reads or lengths"); return MBW_E_INVAL; }
  if (n_cands >= (1ull << 31) || n_reads >= (1ull << 31)) { mbw_set_error("batch too large"); return MBW_E_INVAL; }
  const mbw_index *ix = c->ix;
  if (!ix->text) { mbw_set_error("the index holds no text (built with isa_sample 0)"); return MBW_E_INVAL; }
  TRY(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  c->cur = st;
  out->n_cands = n_cands;
  TRY(hipEventRecord(c->ev[0], st));
  if (n_cands == 0) {
    TRY(hipEventRecord(c->ev[3], st));
    TRY(hipEventSynchronize(c->ev[3]));
    return MBW_OK;
  }
  GROW(c->rc_ctl, RC_CTL * sizeof(unsigned long long));
  unsigned long long *ctl = (unsigned long long *)c->rc_ctl.p;
  TRY(hipMemsetAsync(ctl, 0, RC_CTL * sizeof(unsigned long long), st));
  // read offsets
  GROW(c->rc_lens, (n_reads + 1) * sizeof(uint32_t));
  GROW(c->rc_wide, (n_reads + 1) * sizeof(uint64_t));
  GROW(c->rc_offs, (n_reads + 1) * sizeof(uint64_t));
  const uint32_t *dlen = lengths;
  if (n_reads && !is_device_ptr(lengths)) {
    TRY(hipMemcpyAsync(c->rc_lens.p, lengths, n_reads * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    dlen = (const uint32_t *)c->rc_lens.p;
  }
  uint64_t *wide = (uint64_t *)c->rc_wide.p, *offs = (uint64_t *)c->rc_offs.p;
  k_rc_widen<<<rc_grid(n_reads + 1), 256, 0, st>>>(dlen, n_reads, wide, ctl);
  TRY(hipGetLastError());
  int r = prim_call(c, [&](void *tp, size_t &tb) { return prim::exclusive_sum(tp, tb, wide, offs, n_reads + 1, st); });
  if (r) return r;
  // candidates
  const mbw_rescue_cand_t *dc = cands;
  if (!is_device_ptr(cands)) {
    GROW(c->rc_cand, n_cands * sizeof(mbw_rescue_cand_t));
    TRY(hipMemcpyAsync(c->rc_cand.p, cands, n_cands * sizeof(mbw_rescue_cand_t), hipMemcpyHostToDevice, st));
    dc = (const mbw_rescue_cand_t *)c->rc_cand.p;
  }
  const uint64_t m = ix->n - 1;
  k_rc_check<<<rc_grid(n_cands), 256, 0, st>>>(dc, n_cands, n_reads, m, ctl);
  TRY(hipGetLastError());
  unsigned long long h[RC_CTL];
  uint64_t total = 0;
  TRY(hipMemcpyAsync(h, ctl, sizeof(h), hipMemcpyDeviceToHost, st));
  TRY(hipMemcpyAsync(&total, offs + n_reads, 8, hipMemcpyDeviceToHost, st));
  TRY(hipStreamSynchronize(st));
  if (h[RC_BAD]) {
    mbw_set_error(std::to_string(h[RC_BAD]) + " candidate(s) with a read id >= n_reads or a window outside the text");
    return MBW_E_INVAL;
  }
  if (h[RC_MAXLEN] > MBW_MAX_READ) { mbw_set_error("read longer than 65535 bases"); return MBW_E_INVAL; }
  const uint32_t cap_p = (uint32_t)std::max<unsigned long long>(h[RC_MAXLEN], 1);
  const uint32_t cap_w = (uint32_t)std::max<unsigned long long>(h[RC_MAXWIN], 1);
  uint32_t tbits = 6;
  while ((1u << tbits) < cap_p + cap_p / 2 + 1) ++tbits;
  const RcLayout Lo = rc_layout(tbits, cap_p, cap_w);
  const size_t lds = (size_t)Lo.total * 4;
  if (tbits > 20 || lds > RC_MAX_LDS) {
    mbw_set_error("read and window too long for the prefilter (" + std::to_string(lds) + " bytes of LDS per wave)");
    return MBW_E_INVAL;
  }
  const uint8_t *dreads = reads;
  if (n_reads && !is_device_ptr(reads)) {
    GROW(c->rc_ascii, total + 16);
    TRY(hipMemcpyAsync(c->rc_ascii.p, reads, total, hipMemcpyHostToDevice, st));
    dreads = (const uint8_t *)c->rc_ascii.p;
  }
  GROW(c->rc_hits, n_cands * sizeof(mbw_rescue_hit_t));
  GROW(c->rc_flags, n_cands);
  GROW(c->rc_pass, n_cands * sizeof(uint32_t));
  RescueArgs A;
  A.reads = dreads; A.offs = offs; A.n_reads = n_reads;
  A.cand = dc; A.n_cand = n_cands;
  A.text = (const uint64_t *)ix->text; A.m = m;
  A.q = o.q; A.role = o.bs_role; A.min_hits = (uint32_t)o.min_hits;
  A.tbits = tbits; A.cap_p = cap_p; A.cap_w = cap_w;
  A.hits = (mbw_rescue_hit_t *)c->rc_hits.p; A.flags = (uint8_t *)c->rc_flags.p; A.ctl = ctl;
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)k_rescue, 64, lds) != hipSuccess || per < 1) per = 8;
  const uint64_t grid = std::min<uint64_t>(n_cands, (uint64_t)per * c->n_cu);
  TRY(hipEventRecord(c->ev[1], st));
  k_rescue<<<(unsigned)grid, 64, lds, st>>>(A);
  TRY(hipGetLastError());
  TRY(hipEventRecord(c->ev[2], st));
  uint32_t *nsel = (uint32_t *)(ctl + RC_NSEL);
  r = prim_call(c, [&](void *tp, size_t &tb) {
    return prim::flagged_indices(tp, tb, A.flags, (uint32_t *)c->rc_pass.p, nsel, n_cands, st);
  });
  if (r) return r;
  TRY(hipMemcpyAsync(h, ctl, sizeof(h), hipMemcpyDeviceToHost, st));
  TRY(hipEventRecord(c->ev[3], st));
  TRY(hipEventSynchronize(c->ev[3]));
  if (h[RC_ERR]) { mbw_set_error("prefilter kernel guard tripped"); return MBW_E_HIP; }
  float t_k = 0, t_tot = 0;
  (void)hipEventElapsedTime(&t_k, c->ev[1], c->ev[2]);
  (void)hipEventElapsedTime(&t_tot, c->ev[0], c->ev[3]);
  out->n_pass = (uint32_t)h[RC_NSEL];
  out->hits = A.hits;
  out->pass = (const uint32_t *)c->rc_pass.p;
  out->ms_kernel = t_k;
  out->ms_total = t_tot;
  return MBW_OK;
}

extern "C" int mbw_rescue_download(mbw_ctx *c, const mbw_rescue_result *res, mbw_rescue_hit_t *hits, uint32_t *pass) {
  if (!c || !res) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  TRY(hipSetDevice(c->device));
  if (hits && res->n_cands)
    TRY(hipMemcpyAsync(hits, res->hits, res->n_cands * sizeof(mbw_rescue_hit_t), hipMemcpyDeviceToHost, c->cur));
  if (pass && res->n_pass)
    TRY(hipMemcpyAsync(pass, res->pass, res->n_pass * sizeof(uint32_t), hipMemcpyDeviceToHost, c->cur));
  TRY(hipStreamSynchronize(c->cur));
  return MBW_OK;
}
