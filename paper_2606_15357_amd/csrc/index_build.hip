// Index construction on the GPU, index files, and index queries.
//
// Paper Section 2.1 defines T = R . revcomp(R) . $ (Section 2.9: in bisulfite mode R is replaced by
// C->T(R) . G->A(R)), the suffix array S, the BWT B[i] = T[S(i)-1] and the LF-mapping.  The
// suffix array is built here by MSD refinement on the GPU: suffixes are bucketed by their first six
// symbols, each bucket range (a "chunk" sized to the free HBM) is radix-sorted by a 63-bit key
// holding 21 symbols in 3-bit codes ($ = 0, A..T = 1..4), and groups of equal keys are re-sorted by
// the next 21 symbols until every group is a single suffix.  $ is unique, so a key that reaches
// the end of T is unique and needs no further refinement.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "mbw_internal.h"
#include "prim.h"
#include "../../include/mbw.h"

// The records of a reference: R is their sequences back to back, record i at [start[i], start[i] +
// len[i]).  An index built from memory has one record with an empty name.
struct mbw_contigs {
  std::vector<std::string> name;
  std::vector<uint64_t> start, len;

  // file form: u64 count, then per record u64 start, u64 length, u32 name bytes, the name
  std::vector<uint8_t> serialize() const {
    std::vector<uint8_t> b;
    auto put = [&](const void *p, size_t k) { const uint8_t *q = (const uint8_t *)p; b.insert(b.end(), q, q + k); };
    const uint64_t n = name.size();
    put(&n, 8);
    for (uint64_t i = 0; i < n; ++i) {
      const uint32_t nl = (uint32_t)name[i].size();
      put(&start[i], 8); put(&len[i], 8); put(&nl, 4); put(name[i].data(), nl);
    }
    while (b.size() % 8) b.push_back(0);
    return b;
  }
  // parse and check against |R|: records back to back from 0, non-empty, covering R exactly
  bool parse(const uint8_t *p, size_t bytes, uint64_t len_r) {
    size_t o = 0;
    auto get = [&](void *d, size_t k) { if (o + k > bytes) return false; memcpy(d, p + o, k); o += k; return true; };
    uint64_t n = 0;
    if (!get(&n, 8) || n == 0 || n > bytes / 20) return false;
    uint64_t at = 0;
    for (uint64_t i = 0; i < n; ++i) {
      uint64_t a, l; uint32_t nl;
      if (!get(&a, 8) || !get(&l, 8) || !get(&nl, 4) || o + nl > bytes) return false;
      if (a != at || l == 0) return false;
      name.emplace_back((const char *)p + o, nl);
      o += nl;
      start.push_back(a); len.push_back(l);
      at += l;
    }
    return at == len_r;
  }
};

namespace {

// ---------------------------------------------------------------------------------------------
// device buffers with RAII
template <class T>
struct DevBuf {
  T *p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  void release() { if (p) (void)hipFree(p); p = nullptr; n = 0; }
  hipError_t alloc(size_t count) {
    release();
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)&p, count * sizeof(T));
    if (e == hipSuccess) n = count; else p = nullptr;
    return e;
  }
  T *detach() { T *q = p; p = nullptr; n = 0; return q; }
};

struct Temp {
  DevBuf<uint8_t> b;
  hipError_t ensure(size_t bytes) { return bytes <= b.n ? hipSuccess : b.alloc(bytes + bytes / 8 + 256); }
};

#define TRY(call) MBW_HIP_TRY(call)

__host__ __device__ inline uint64_t splitmix(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

inline unsigned grid_for(uint64_t n, unsigned bs = 256, unsigned cap = 65536u * 8) {
  uint64_t g = (n + bs - 1) / bs;
  if (g < 1) g = 1;
  return (unsigned)std::min<uint64_t>(g, cap);
}

// ---------------------------------------------------------------------------------------------
// text

// T without its final $: Tm = R' . revcomp(R'), m = 2|R'| symbols, packed 32 per u64 (LSB first).
__global__ void k_pack_text(const uint8_t *__restrict__ Rp, uint64_t lrp, uint64_t *__restrict__ Tw, uint64_t nwords) {
  uint64_t m = 2 * lrp;
  for (uint64_t w = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; w < nwords; w += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t v = 0;
    for (int t = 0; t < 32; ++t) {
      uint64_t i = w * 32 + t;
      uint64_t a = 0;
      if (i < lrp) a = Rp[i];
      else if (i < m) a = 3 - Rp[m - 1 - i];
      v |= a << (2 * t);
    }
    Tw[w] = v;
  }
}

// the original reference of a bisulfite index from its two converted copies: a T in the C->T copy
// was a C or a T, which the G->A copy still tells apart; every other base is unchanged there
__global__ void k_pack_orig(const uint8_t *__restrict__ Rp, uint64_t len, uint64_t *__restrict__ ow, uint64_t nwords) {
  for (uint64_t w = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; w < nwords; w += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t v = 0;
    for (int t = 0; t < 32; ++t) {
      const uint64_t i = w * 32 + t;
      uint64_t a = 0;
      if (i < len) a = Rp[i] == 3 ? Rp[len + i] : Rp[i];
      v |= a << (2 * t);
    }
    ow[w] = v;
  }
}

__device__ __forceinline__ uint64_t text_sym(const uint64_t *__restrict__ Tw, uint64_t p) {
  return (Tw[p >> 5] >> (2 * (p & 31))) & 3;
}

// 21 symbols of T starting at p as a 63-bit key, MSB first, codes $/past-end = 0, A..T = 1..4.
__device__ __forceinline__ uint64_t key21(const uint64_t *__restrict__ Tw, uint64_t m, uint64_t p) {
  if (p >= m) return 0;
  uint64_t w = p >> 5;
  int sh = (int)(p & 31) * 2;
  uint64_t s = Tw[w] >> sh;
  if (sh) s |= Tw[w + 1] << (64 - sh);
  uint64_t left = m - p;  // symbols before $
  uint64_t key = 0;
#pragma unroll
  for (int t = 0; t < 21; ++t) {
    uint64_t c = ((uint64_t)t < left) ? ((s >> (2 * t)) & 3) + 1 : 0;
    key = (key << 3) | c;
  }
  return key;
}

// bucket = first 6 symbols as base-5 digits ($ / past-end = 0, A..T = 1..4): 5^6 buckets in
// lexicographic order of the 6-symbol prefix
#define NBUCKET 15625u
__device__ __forceinline__ uint32_t bucket_of(uint64_t key) {
  uint32_t b = 0;
#pragma unroll
  for (int t = 0; t < 6; ++t) b = b * 5 + (uint32_t)((key >> (60 - 3 * t)) & 7);
  return b;
}

__global__ void __launch_bounds__(256) k_bucket_hist(const uint64_t *__restrict__ Tw, uint64_t m, uint64_t n,
                                                     unsigned long long *__restrict__ hist) {
  __shared__ uint32_t h[NBUCKET];
  for (uint32_t t = threadIdx.x; t < NBUCKET; t += blockDim.x) h[t] = 0;
  __syncthreads();
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    atomicAdd(&h[bucket_of(key21(Tw, m, i))], 1u);
  __syncthreads();
  for (uint32_t t = threadIdx.x; t < NBUCKET; t += blockDim.x)
    if (h[t]) atomicAdd(&hist[t], (unsigned long long)h[t]);
}

// positions whose bucket lies in [blo, bhi) -> out (order is irrelevant: the sort fixes it).
// Each wave takes SEL_SUB x 64 consecutive positions, keeps its lane's selection bits in a register
// and reserves the output for all of them with one atomic: the reservation counter is a single
// address, and same-address device-scope atomics serialise (with one reservation per 64 positions
// the pass ran at about 5 G positions/s).
#define SEL_SUB 32
__global__ void k_select(const uint64_t *__restrict__ Tw, uint64_t m, uint64_t n, uint32_t blo, uint32_t bhi,
                         uint64_t *__restrict__ out, unsigned long long *__restrict__ count) {
  const int lane = threadIdx.x & 63;
  const uint64_t below = (1ull << lane) - 1;
  const uint64_t wave = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6;
  const uint64_t nwave = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  for (uint64_t base = wave * 64 * SEL_SUB; base < n; base += nwave * 64 * SEL_SUB) {
    uint32_t bits = 0;
    uint32_t cnt = 0;
#pragma unroll 4
    for (int t = 0; t < SEL_SUB; ++t) {
      const uint64_t i = base + (uint64_t)t * 64 + lane;
      bool f = false;
      if (i < n) {
        const uint32_t b = bucket_of(key21(Tw, m, i));
        f = b >= blo && b < bhi;
      }
      bits |= (f ? 1u : 0u) << t;
      cnt += __popcll(__ballot(f));
    }
    unsigned long long off = 0;
    if (lane == 0 && cnt) off = atomicAdd(count, (unsigned long long)cnt);
    off = __shfl(off, 0);
    for (int t = 0; t < SEL_SUB; ++t) {
      const bool f = (bits >> t) & 1u;
      const uint64_t mask = __ballot(f);
      if (f) out[off + __popcll(mask & below)] = base + (uint64_t)t * 64 + lane;
      off += __popcll(mask);
    }
  }
}

__global__ void k_keys(const uint64_t *__restrict__ Tw, uint64_t m, const uint64_t *__restrict__ pos, uint64_t M,
                       uint64_t d, uint64_t *__restrict__ key) {
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < M; x += (uint64_t)gridDim.x * blockDim.x)
    key[x] = key21(Tw, m, pos[x] + d);
}

// group boundaries after the first sort; grp seed for the max-scan
__global__ void k_init_bounds(const uint64_t *__restrict__ key, uint64_t M, uint8_t *__restrict__ bnd, uint32_t *__restrict__ gs) {
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x <= M; x += (uint64_t)gridDim.x * blockDim.x) {
    uint8_t b = (x == 0 || x == M) ? 1 : (key[x] != key[x - 1]);
    bnd[x] = b;
    if (x < M) gs[x] = b ? (uint32_t)x : 0u;
  }
}

// unresolved = member of a group of size >= 2
__global__ void k_mark_unres(const uint8_t *__restrict__ bnd, uint64_t M, uint32_t *__restrict__ flag) {
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < M; x += (uint64_t)gridDim.x * blockDim.x)
    flag[x] = (bnd[x] && bnd[x + 1]) ? 0u : 1u;
}

__global__ void k_scatter_unres(const uint32_t *__restrict__ flag, const uint32_t *__restrict__ idx, uint64_t M,
                                const uint32_t *__restrict__ grp, uint32_t *__restrict__ u_slot, uint32_t *__restrict__ u_gid) {
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < M; x += (uint64_t)gridDim.x * blockDim.x)
    if (flag[x]) { uint32_t u = idx[x]; u_slot[u] = (uint32_t)x; u_gid[u] = grp[x]; }
}

// later rounds look only at the previous round's unresolved rows (groups only split): the same
// test and compaction over that list, which keeps ascending row order
__global__ void k_mark_unres_list(const uint8_t *__restrict__ bnd, const uint32_t *__restrict__ list, uint64_t MU,
                                  uint32_t *__restrict__ flag) {
  for (uint64_t u = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; u < MU; u += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t x = list[u];
    flag[u] = (bnd[x] && bnd[x + 1]) ? 0u : 1u;
  }
}

__global__ void k_scatter_unres_list(const uint32_t *__restrict__ flag, const uint32_t *__restrict__ idx,
                                     const uint32_t *__restrict__ list, uint64_t MU, const uint32_t *__restrict__ grp,
                                     uint32_t *__restrict__ u_slot, uint32_t *__restrict__ u_gid) {
  for (uint64_t u = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; u < MU; u += (uint64_t)gridDim.x * blockDim.x)
    if (flag[u]) { const uint32_t x = list[u], v = idx[u]; u_slot[v] = x; u_gid[v] = grp[x]; }
}

__global__ void k_u_keys(const uint64_t *__restrict__ Tw, uint64_t m, const uint64_t *__restrict__ sa,
                         const uint32_t *__restrict__ u_slot, uint64_t MU, uint64_t d, uint64_t *__restrict__ nk,
                         uint32_t *__restrict__ iota) {
  for (uint64_t u = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; u < MU; u += (uint64_t)gridDim.x * blockDim.x) {
    nk[u] = key21(Tw, m, sa[u_slot[u]] + d);
    iota[u] = (uint32_t)u;
  }
}

__global__ void k_gather_u32(const uint32_t *__restrict__ src, const uint32_t *__restrict__ perm, uint64_t MU, uint32_t *__restrict__ dst) {
  for (uint64_t u = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; u < MU; u += (uint64_t)gridDim.x * blockDim.x)
    dst[u] = src[perm[u]];
}

// final order of this round: element perm[u] (index into the round's U) goes to slot u_slot[u]
__global__ void k_apply_gather(const uint64_t *__restrict__ sa, const uint32_t *__restrict__ u_slot,
                               const uint32_t *__restrict__ perm, const uint64_t *__restrict__ nk, uint64_t MU,
                               uint64_t *__restrict__ tmp_sa, uint64_t *__restrict__ tmp_nk) {
  for (uint64_t u = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; u < MU; u += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t v = perm[u];
    tmp_sa[u] = sa[u_slot[v]];
    tmp_nk[u] = nk[v];
  }
}

__global__ void k_apply_scatter(uint64_t *__restrict__ sa, uint8_t *__restrict__ bnd, const uint32_t *__restrict__ u_slot,
                                const uint64_t *__restrict__ tmp_sa, const uint64_t *__restrict__ tmp_nk, uint64_t MU,
                                uint32_t *__restrict__ gseed) {
  for (uint64_t u = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; u < MU; u += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t x = u_slot[u];
    sa[x] = tmp_sa[u];
    uint8_t b = bnd[x] | (uint8_t)(u > 0 && tmp_nk[u] != tmp_nk[u - 1]);
    bnd[x] = b;   // only this thread touches row x in this pass
    gseed[u] = b ? x : 0u;
  }
}

// new group start of every refined row (max-scan of the group-start seeds over U)
__global__ void k_apply_groups(uint32_t *__restrict__ grp, const uint32_t *__restrict__ u_slot,
                               const uint32_t *__restrict__ gscan, uint64_t MU) {
  for (uint64_t u = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; u < MU; u += (uint64_t)gridDim.x * blockDim.x)
    grp[u_slot[u]] = gscan[u];
}

// B rows and SA samples of a finished chunk
__global__ void k_emit_rows(const uint64_t *__restrict__ sa, uint64_t M, uint64_t base, const uint64_t *__restrict__ Tw,
                            uint32_t r, uint8_t *__restrict__ B, uint64_t *__restrict__ ssa, unsigned long long *__restrict__ primary,
                            uint32_t ri, uint64_t *__restrict__ isa) {
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < M; x += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t p = sa[x], row = base + x;
    uint8_t b = 0;
    if (p == 0) *primary = row;
    else b = (uint8_t)text_sym(Tw, p - 1);
    B[row] = b;
    if (row % r == 0) ssa[row / r] = p;
    if (isa && p % ri == 0) isa[p / ri] = row;   // inverse SA at sampled text positions
  }
}

// ---------------------------------------------------------------------------------------------
// occurrence lines

// the line's six 64-row blocks as bit planes, sub-checkpoints (A, C, G in the first 64 b rows),
// per-line totals
__global__ void k_line_counts(const uint8_t *__restrict__ B, uint64_t n, uint64_t n_lines, uint64_t *__restrict__ cnt /*4 x n_lines*/,
                              uint4 *__restrict__ lines) {
  for (uint64_t L = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; L < n_lines; L += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t c[4] = {0, 0, 0, 0};
    uint32_t *w32 = (uint32_t *)(lines + L * MBW_LINE_U4);
    uint64_t *w = (uint64_t *)(lines + L * MBW_LINE_U4);
    for (int b = 0; b < 6; ++b) {
      if (b > 0) w32[b == 1 ? 3 : 4 + (b - 2)] = c[0] | (c[1] << 9) | (c[2] << 18);
      uint64_t lo = 0, hi = 0;
      for (int t = 0; t < MBW_BLK; ++t) {
        const uint64_t row = L * MBW_BPL + (uint64_t)b * MBW_BLK + t;
        if (row < n) {
          const uint32_t v = B[row];
          lo |= (uint64_t)(v & 1u) << t;
          hi |= (uint64_t)(v >> 1) << t;
          c[v]++;
        }
      }
      w[4 + 2 * b] = lo;
      w[5 + 2 * b] = hi;
    }
    for (int a = 0; a < 4; ++a) cnt[a * n_lines + L] = c[a];
  }
}

// line header: counts of A, C, G before the line, relative to the start of its superblock
__global__ void k_line_headers(const uint64_t *__restrict__ pre /*4 x n_lines exclusive sums*/, uint64_t n_lines,
                               const uint64_t *__restrict__ sbtab, uint32_t sb_shift, uint4 *__restrict__ lines) {
  for (uint64_t L = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; L < n_lines; L += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t *w = (uint32_t *)(lines + L * MBW_LINE_U4);
    const uint64_t *t = sbtab + 8 * (L >> sb_shift);
    for (int a = 0; a < 3; ++a) w[a] = (uint32_t)(pre[a * n_lines + L] - t[a]);
  }
}

// ---------------------------------------------------------------------------------------------
// k-mer table: level t+1 from level t by one backward extension (Algorithm 1), every level in the
// table's packed form.  Level t+1 from level t: code(aP) = a + 4 code(P) (the first base is the
// least significant digit).
__global__ void k_kmer_level(IndexView ix, const uint4 *__restrict__ prev, uint64_t nprev, uint4 *__restrict__ next) {
  uint64_t total = nprev * 4;
  for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < total; e += (uint64_t)gridDim.x * blockDim.x) {
    const int a = (int)(e & 3);
    uint64_t pk, pkr, ps, ok = 0, okr = 0, os = 0;
    kmer_unpack(prev[e >> 2], pk, pkr, ps);
    if (ps != 0) {
      uint64_t E1, G1, E2, G2;
      rank_global(ix, pk, a, E1, G1);
      rank_global(ix, pk + ps, a, E2, G2);
      ext_update(E1, G1, E2, G2, a, pk, ps, pkr, ix.primary, sel4(ix.Cb[0], ix.Cb[1], ix.Cb[2], ix.Cb[3], a), ok, okr, os);
    }
    next[e] = kmer_pack(ok, okr, os);
  }
}

// ---------------------------------------------------------------------------------------------
// suffix sorting of one chunk; returns 0 or an MBW error code
int sort_chunk(const uint64_t *Tw, uint64_t m, uint64_t n, uint32_t blo, uint32_t bhi, uint64_t M,
               uint64_t *sa0, uint64_t *sa1, uint64_t *key0, uint64_t *key1, uint8_t *bnd, uint32_t *grp,
               uint32_t *flag, uint32_t *idx, uint32_t *u_slot, uint32_t *u_slot2, uint32_t *u_gid, uint32_t *iota0,
               uint32_t *iota1, uint64_t *nk1, uint32_t *gid1, uint32_t *gseed, uint32_t *gscan, uint64_t *tmp_sa,
               uint64_t *tmp_nk, unsigned long long *dcount, Temp &tmp, hipStream_t st, uint64_t **sa_out) {
  TRY(hipMemsetAsync(dcount, 0, sizeof(unsigned long long), st));
  k_select<<<grid_for(n), 256, 0, st>>>(Tw, m, n, blo, bhi, sa0, dcount);
  TRY(hipGetLastError());
  unsigned long long got = 0;
  TRY(hipMemcpyAsync(&got, dcount, sizeof(got), hipMemcpyDeviceToHost, st));
  TRY(hipStreamSynchronize(st));
  if (got != M) { mbw_set_error("suffix bucket selection count mismatch"); return MBW_E_HIP; }
  k_keys<<<grid_for(M), 256, 0, st>>>(Tw, m, sa0, M, 0, key0);
  TRY(hipGetLastError());
  prim::dbuf<uint64_t> dk(key0, key1), dv(sa0, sa1);
  size_t tb = 0;
  TRY(prim::sort_pairs(nullptr, tb, dk, dv, M, 0, 63, st));
  TRY(tmp.ensure(tb));
  TRY(prim::sort_pairs(tmp.b.p, tb, dk, dv, M, 0, 63, st));
  uint64_t *sa = dv.current();
  uint64_t *key = dk.current();
  k_init_bounds<<<grid_for(M + 1), 256, 0, st>>>(key, M, bnd, idx /*as seed*/);
  TRY(hipGetLastError());
  tb = 0;
  TRY(prim::inclusive_max(nullptr, tb, idx, grp, M, st));
  TRY(tmp.ensure(tb));
  TRY(prim::inclusive_max(tmp.b.p, tb, idx, grp, M, st));
  uint64_t MU = M;   // candidates of this round: all rows in the first, then the last round's unresolved list
  for (uint64_t round = 1;; ++round) {
    if (round > n / 21 + 4) { mbw_set_error("suffix refinement did not converge"); return MBW_E_HIP; }
    uint32_t *prev = u_slot;
    if (round == 1) k_mark_unres<<<grid_for(M), 256, 0, st>>>(bnd, M, flag);
    else k_mark_unres_list<<<grid_for(MU), 256, 0, st>>>(bnd, prev, MU, flag);
    TRY(hipGetLastError());
    tb = 0;
    TRY(prim::exclusive_sum(nullptr, tb, flag, idx, MU, st));
    TRY(tmp.ensure(tb));
    TRY(prim::exclusive_sum(tmp.b.p, tb, flag, idx, MU, st));
    uint32_t lastf = 0, lasti = 0;
    TRY(hipMemcpyAsync(&lastf, flag + MU - 1, 4, hipMemcpyDeviceToHost, st));
    TRY(hipMemcpyAsync(&lasti, idx + MU - 1, 4, hipMemcpyDeviceToHost, st));
    TRY(hipStreamSynchronize(st));
    const uint64_t MU0 = MU;
    MU = (uint64_t)lasti + lastf;
    if (MU == 0) break;
    if (round == 1) k_scatter_unres<<<grid_for(M), 256, 0, st>>>(flag, idx, M, grp, u_slot, u_gid);
    else {
      k_scatter_unres_list<<<grid_for(MU0), 256, 0, st>>>(flag, idx, prev, MU0, grp, u_slot2, u_gid);
      std::swap(u_slot, u_slot2);
    }
    TRY(hipGetLastError());
    uint64_t d = 21 * round;
    k_u_keys<<<grid_for(MU), 256, 0, st>>>(Tw, m, sa, u_slot, MU, d, tmp_nk /*nk*/, iota0);
    TRY(hipGetLastError());
    // stable LSD: by next key, then by group start
    prim::dbuf<uint64_t> k1(tmp_nk, nk1);
    prim::dbuf<uint32_t> v1(iota0, iota1);
    tb = 0;
    TRY(prim::sort_pairs(nullptr, tb, k1, v1, MU, 0, 63, st));
    TRY(tmp.ensure(tb));
    TRY(prim::sort_pairs(tmp.b.p, tb, k1, v1, MU, 0, 63, st));
    uint64_t *nk = (k1.current() == tmp_nk) ? tmp_nk : nk1;   // sorted keys (unused below)
    (void)nk;
    uint32_t *perm1 = v1.current();
    uint32_t *perm_alt = (perm1 == iota0) ? iota1 : iota0;
    k_gather_u32<<<grid_for(MU), 256, 0, st>>>(u_gid, perm1, MU, gid1);
    TRY(hipGetLastError());
    prim::dbuf<uint32_t> k2(gid1, gscan), v2(perm1, perm_alt);
    tb = 0;
    TRY(prim::sort_pairs(nullptr, tb, k2, v2, MU, 0, 32, st));
    TRY(tmp.ensure(tb));
    TRY(prim::sort_pairs(tmp.b.p, tb, k2, v2, MU, 0, 32, st));
    uint32_t *perm = v2.current();
    // the unsorted next keys of this round are needed by index: recompute into nk1
    k_u_keys<<<grid_for(MU), 256, 0, st>>>(Tw, m, sa, u_slot, MU, d, nk1, gscan /*scratch iota*/);
    TRY(hipGetLastError());
    k_apply_gather<<<grid_for(MU), 256, 0, st>>>(sa, u_slot, perm, nk1, MU, tmp_sa, tmp_nk);
    TRY(hipGetLastError());
    k_apply_scatter<<<grid_for(MU), 256, 0, st>>>(sa, bnd, u_slot, tmp_sa, tmp_nk, MU, gseed);
    TRY(hipGetLastError());
    tb = 0;
    TRY(prim::inclusive_max(nullptr, tb, gseed, gscan, MU, st));
    TRY(tmp.ensure(tb));
    TRY(prim::inclusive_max(tmp.b.p, tb, gseed, gscan, MU, st));
    k_apply_groups<<<grid_for(MU), 256, 0, st>>>(grp, u_slot, gscan, MU);
    TRY(hipGetLastError());
  }
  *sa_out = sa;
  return 0;
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// error state
static thread_local std::string g_err;
void mbw_set_error(const std::string &msg) { g_err = msg; }
extern "C" const char *mbw_last_error(void) { return g_err.c_str(); }

extern "C" const char *mbw_strerror(int code) {
  switch (code) {
    case MBW_OK: return "ok";
    case MBW_E_INVAL: return "invalid argument";
    case MBW_E_NOMEM: return "out of memory";
    case MBW_E_HIP: return "HIP runtime error";
    case MBW_E_IO: return "I/O error";
    case MBW_E_FORMAT: return "bad index file format";
    case MBW_E_CAPACITY: return "buffer too small";
    case MBW_E_BUSY: return "busy";
    default: return "unknown error";
  }
}

static std::mutex g_index_mu;   // guards users / free_pending of every index

static void index_destroy(mbw_index *ix) {
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(ix->device);
  if (ix->lines) (void)hipFree(ix->lines);
  if (ix->ssa) (void)hipFree(ix->ssa);
  if (ix->kmer) (void)hipFree(ix->kmer);
  if (ix->sbtab) (void)hipFree(ix->sbtab);
  if (ix->text) (void)hipFree(ix->text);
  if (ix->isa) (void)hipFree(ix->isa);
  if (ix->orig) (void)hipFree(ix->orig);
  delete ix->contigs;
  (void)hipSetDevice(cur);
  delete ix;
}

void mbw_index_retain(const mbw_index *ix) {
  std::lock_guard<std::mutex> lk(g_index_mu);
  ++const_cast<mbw_index *>(ix)->users;
}

void mbw_index_release(const mbw_index *ix) {
  mbw_index *m = const_cast<mbw_index *>(ix);
  bool last = false;
  {
    std::lock_guard<std::mutex> lk(g_index_mu);
    last = --m->users == 0 && m->free_pending;
  }
  if (last) index_destroy(m);
}

extern "C" void mbw_index_free(mbw_index *ix) {
  if (!ix) return;
  {
    std::lock_guard<std::mutex> lk(g_index_mu);
    if (ix->users > 0) { ix->free_pending = true; return; }
  }
  index_destroy(ix);
}

static int build_kmer_table(mbw_index *ix, hipStream_t st) {
  int K = ix->kmer_k;
  if (K <= 0) return 0;
  IndexView v = make_view(ix);
  const uint64_t ntop = 1ull << (2 * K);
  uint4 *tab = nullptr;
  TRY(hipMalloc((void **)&tab, ntop * sizeof(uint4)));
  ix->kmer = tab;
  ix->bytes += ntop * sizeof(uint4);
  // the levels alternate between the table and a scratch buffer of a quarter of its size, so that
  // level K lands in the table: level t lies in the table when K - t is even
  DevBuf<uint4> scratch;
  TRY(scratch.alloc(ntop / 4));
  uint4 *cur = (K % 2 == 0) ? tab : scratch.p;
  const uint4 root = kmer_pack(0, 0, ix->n);
  TRY(hipMemcpyAsync(cur, &root, sizeof(uint4), hipMemcpyHostToDevice, st));
  uint64_t cnt = 1;
  for (int t = 0; t < K; ++t) {
    uint4 *nxt = (cur == tab) ? scratch.p : tab;
    k_kmer_level<<<grid_for(cnt * 4), 256, 0, st>>>(v, cur, cnt, nxt);
    TRY(hipGetLastError());
    cur = nxt;
    cnt *= 4;
  }
  TRY(hipStreamSynchronize(st));
  return 0;
}

static int build_lines(mbw_index *ix, const uint8_t *B, hipStream_t st) {
  uint64_t n = ix->n, nl = n / MBW_BPL + 1;
  ix->n_lines = nl;
  ix->n_sb = (int)(((nl - 1) >> ix->sb_shift) + 1);
  if (ix->n_sb > MBW_MAX_SB) {
    mbw_set_error("reference too large for the superblock table (" + std::to_string(ix->n_sb) + " superblocks of 2^" +
                  std::to_string(ix->sb_shift) + " lines; at most " + std::to_string(MBW_MAX_SB) + ")");
    return MBW_E_INVAL;
  }
  TRY(hipMalloc((void **)&ix->lines, nl * MBW_LINE_BYTES));
  ix->bytes += nl * MBW_LINE_BYTES;
  DevBuf<uint64_t> cnt, pre;
  TRY(cnt.alloc(4 * nl + 1));
  TRY(pre.alloc(4 * nl + 1));
  k_line_counts<<<grid_for(nl), 256, 0, st>>>(B, n, nl, cnt.p, ix->lines);
  TRY(hipGetLastError());
  Temp tmp;
  for (int a = 0; a < 4; ++a) {
    size_t tb = 0;
    TRY(prim::exclusive_sum(nullptr, tb, cnt.p + a * nl, pre.p + a * nl, nl, st));
    TRY(tmp.ensure(tb));
    TRY(prim::exclusive_sum(tmp.b.p, tb, cnt.p + a * nl, pre.p + a * nl, nl, st));
  }
  uint64_t tot[4], last[4];
  for (int a = 0; a < 4; ++a) {
    TRY(hipMemcpyAsync(&tot[a], pre.p + a * nl + nl - 1, 8, hipMemcpyDeviceToHost, st));
    TRY(hipMemcpyAsync(&last[a], cnt.p + a * nl + nl - 1, 8, hipMemcpyDeviceToHost, st));
    for (int sb = 0; sb < ix->n_sb; ++sb)
      TRY(hipMemcpyAsync(&ix->sb_host[8 * sb + a], pre.p + a * nl + ((uint64_t)sb << ix->sb_shift), 8,
                         hipMemcpyDeviceToHost, st));
  }
  TRY(hipStreamSynchronize(st));
  for (int sb = 0; sb < ix->n_sb; ++sb)
    for (int c = 0; c < 4; ++c) {
      uint64_t g = 0;
      for (int d = c + 1; d < 4; ++d) g += ix->sb_host[8 * sb + d];
      ix->sb_host[8 * sb + 4 + c] = g;
    }
  TRY(hipMalloc((void **)&ix->sbtab, MBW_MAX_SB * 8 * sizeof(uint64_t)));
  ix->bytes += MBW_MAX_SB * 8 * sizeof(uint64_t);
  TRY(hipMemcpyAsync(ix->sbtab, ix->sb_host, MBW_MAX_SB * 8 * sizeof(uint64_t), hipMemcpyHostToDevice, st));
  k_line_headers<<<grid_for(nl), 256, 0, st>>>(pre.p, nl, ix->sbtab, (uint32_t)ix->sb_shift, ix->lines);
  TRY(hipGetLastError());
  TRY(hipStreamSynchronize(st));
  for (int a = 0; a < 4; ++a) tot[a] += last[a];
  // raw A total includes the $ row
  ix->C[0] = 0;
  ix->C[1] = 1;
  ix->C[2] = ix->C[1] + (tot[0] - 1);
  ix->C[3] = ix->C[2] + tot[1];
  ix->C[4] = ix->C[3] + tot[2];
  return 0;
}

extern "C" int mbw_index_build(const uint8_t *ref, uint64_t len, const mbw_build_opts *opts, mbw_index **out) {
  if (!out) { mbw_set_error("out is NULL"); return MBW_E_INVAL; }
  *out = nullptr;
  if (!ref || !opts || len == 0 || len >= (1ull << 38)) { mbw_set_error("bad reference or options"); return MBW_E_INVAL; }
  if (opts->sa_sample < 1 || opts->sa_sample > 1024) { mbw_set_error("sa_sample must be in [1,1024]"); return MBW_E_INVAL; }
  if (opts->kmer_k < -1 || opts->kmer_k > 15) { mbw_set_error("kmer_k must be -1 or in [0,15]"); return MBW_E_INVAL; }
  if (opts->isa_sample < 0 || opts->isa_sample > 64) { mbw_set_error("isa_sample must be in [0,64]"); return MBW_E_INVAL; }
  if (opts->sb_lines_log2 < 0 || opts->sb_lines_log2 > MBW_SB_SHIFT) {
    mbw_set_error("sb_lines_log2 must be in [0," + std::to_string(MBW_SB_SHIFT) + "]"); return MBW_E_INVAL;
  }
  TRY(hipSetDevice(opts->device));
  // host: codes, ambiguous bases -> random (counter-based SplitMix64), bisulfite conversion
  uint64_t lrp = opts->bisulfite ? 2 * len : len;
  std::vector<uint8_t> Rp;
  try { Rp.resize(lrp); } catch (...) { mbw_set_error("host allocation failed"); return MBW_E_NOMEM; }
  auto convert = [&](uint64_t lo, uint64_t hi) {
  for (uint64_t i = lo; i < hi; ++i) {
    uint8_t a = ref[i];
    int c;
    if (opts->ref_is_codes) c = a < 4 ? a : -1;
    else {
      switch (a) { case 'A': case 'a': c = 0; break; case 'C': case 'c': c = 1; break;
                   case 'G': case 'g': c = 2; break; case 'T': case 't': c = 3; break; default: c = -1; }
    }
    if (c < 0) c = (int)(splitmix(opts->rng_seed + (uint64_t)i * 0x9E3779B97F4A7C15ull) & 3);
    if (opts->bisulfite) {
      Rp[i] = (uint8_t)(c == 1 ? 3 : c);            // C -> T
      Rp[len + i] = (uint8_t)(c == 2 ? 0 : c);      // G -> A
    } else {
      Rp[i] = (uint8_t)c;
    }
  }
  };
  {
    unsigned nt = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
    if (len < (1u << 22)) nt = 1;
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t) th.emplace_back(convert, len * t / nt, len * (t + 1) / nt);
    for (auto &x : th) x.join();
  }
  mbw_index *ix = new mbw_index();
  memset(ix, 0, sizeof(*ix));
  ix->device = opts->device;
  ix->len_r = len;
  ix->bisulfite = opts->bisulfite ? 1 : 0;
  ix->sa_sample = opts->sa_sample;
  ix->isa_sample = opts->isa_sample;
  ix->sb_shift = opts->sb_lines_log2 ? opts->sb_lines_log2 : MBW_SB_SHIFT;
  uint64_t m = 2 * lrp, n = m + 1;
  ix->n = n;
  ix->kmer_k = opts->kmer_k;
  if (ix->kmer_k < 0) {   // automatic: the largest k whose k-mers occur about 4 times or more in T
    int lg = 0;
    while (lg < 31 && (1ull << (2 * (lg + 1))) <= n) ++lg;   // floor(log4 n)
    ix->kmer_k = std::max(1, std::min(15, lg - 1));
  }
  hipStream_t st;
  if (hipStreamCreate(&st) != hipSuccess) { delete ix; mbw_set_error("hipStreamCreate failed"); return MBW_E_HIP; }
  int rc = [&]() -> int {
    uint64_t nwords = (m + 31) / 32 + 4;   // slack: 32-byte text windows read past the last symbol
    DevBuf<uint64_t> Tw;
    TRY(Tw.alloc(nwords));
    {
      DevBuf<uint8_t> dR;
      TRY(dR.alloc(lrp));
      TRY(hipMemcpyAsync(dR.p, Rp.data(), lrp, hipMemcpyHostToDevice, st));
      k_pack_text<<<grid_for(nwords), 256, 0, st>>>(dR.p, lrp, Tw.p, nwords);
      TRY(hipGetLastError());
      if (ix->bisulfite) {
        ix->n_orig = (len + 31) / 32 + 2;
        TRY(hipMalloc((void **)&ix->orig, ix->n_orig * sizeof(uint64_t)));
        ix->bytes += ix->n_orig * sizeof(uint64_t);
        k_pack_orig<<<grid_for(ix->n_orig), 256, 0, st>>>(dR.p, len, ix->orig, ix->n_orig);
        TRY(hipGetLastError());
      }
      TRY(hipStreamSynchronize(st));
    }
    std::vector<uint8_t>().swap(Rp);
    // bucket histogram and chunk plan
    DevBuf<unsigned long long> hist;
    TRY(hist.alloc(NBUCKET + 1));
    TRY(hipMemsetAsync(hist.p, 0, (NBUCKET + 1) * sizeof(unsigned long long), st));
    k_bucket_hist<<<std::min<unsigned>(grid_for(n), 1024u), 256, 0, st>>>(Tw.p, m, n, hist.p);
    TRY(hipGetLastError());
    std::vector<unsigned long long> h(NBUCKET);
    TRY(hipMemcpyAsync(h.data(), hist.p, NBUCKET * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    TRY(hipStreamSynchronize(st));
    // outputs
    DevBuf<uint8_t> B;
    TRY(B.alloc(n));
    ix->n_ssa = (n + ix->sa_sample - 1) / ix->sa_sample;
    TRY(hipMalloc((void **)&ix->ssa, ix->n_ssa * sizeof(uint64_t)));
    ix->bytes += ix->n_ssa * sizeof(uint64_t);
    if (ix->isa_sample) {
      ix->n_isa = (n - 1) / ix->isa_sample + 1;   // text positions 0, q, 2q, ... <= n - 1
      TRY(hipMalloc((void **)&ix->isa, ix->n_isa * sizeof(uint64_t)));
      ix->bytes += ix->n_isa * sizeof(uint64_t);
    }
    // chunk capacity from free memory (about 100 bytes per suffix in flight)
    size_t fr = 0, tot = 0;
    TRY(hipMemGetInfo(&fr, &tot));
    uint64_t cap = (fr > (size_t)(2ull << 30)) ? (uint64_t)((fr - (2ull << 30)) / 108) : (uint64_t)(fr / 216);
    cap = std::min<uint64_t>(cap, (1ull << 31) - 1024);
    uint64_t maxb = *std::max_element(h.begin(), h.end());
    if (cap < maxb) cap = maxb;
    cap = std::min<uint64_t>(cap, n);
    DevBuf<uint64_t> sa0, sa1, key0, key1, nk1, tmp_sa, tmp_nk;
    DevBuf<uint8_t> bnd;
    DevBuf<uint32_t> grp, flag, idx, u_slot, u_slot2, u_gid, iota0, iota1, gid1, gseed, gscan;
    DevBuf<unsigned long long> dcount, dprim;
    TRY(sa0.alloc(cap)); TRY(sa1.alloc(cap)); TRY(key0.alloc(cap)); TRY(key1.alloc(cap));
    TRY(nk1.alloc(cap)); TRY(tmp_sa.alloc(cap)); TRY(tmp_nk.alloc(cap));
    TRY(bnd.alloc(cap + 1));
    TRY(grp.alloc(cap)); TRY(flag.alloc(cap)); TRY(idx.alloc(cap)); TRY(u_slot.alloc(cap)); TRY(u_slot2.alloc(cap));
    TRY(u_gid.alloc(cap));
    TRY(iota0.alloc(cap)); TRY(iota1.alloc(cap)); TRY(gid1.alloc(cap)); TRY(gseed.alloc(cap)); TRY(gscan.alloc(cap));
    TRY(dcount.alloc(1)); TRY(dprim.alloc(1));
    TRY(hipMemsetAsync(dprim.p, 0xff, 8, st));
    Temp tmp;
    uint64_t base = 0;
    uint32_t b = 0;
    while (b < NBUCKET) {
      uint32_t e = b;
      uint64_t M = 0;
      while (e < NBUCKET && M + h[e] <= cap) M += h[e++];
      if (M == 0) { b = e; continue; }
      uint64_t *sa = nullptr;
      int r = sort_chunk(Tw.p, m, n, b, e, M, sa0.p, sa1.p, key0.p, key1.p, bnd.p, grp.p, flag.p, idx.p, u_slot.p,
                         u_slot2.p, u_gid.p, iota0.p, iota1.p, nk1.p, gid1.p, gseed.p, gscan.p, tmp_sa.p, tmp_nk.p,
                         dcount.p, tmp, st, &sa);
      if (r) return r;
      k_emit_rows<<<grid_for(M), 256, 0, st>>>(sa, M, base, Tw.p, (uint32_t)ix->sa_sample, B.p, ix->ssa, dprim.p,
                                               (uint32_t)std::max(1, ix->isa_sample), ix->isa);
      TRY(hipGetLastError());
      base += M;
      b = e;
    }
    if (base != n) { mbw_set_error("suffix chunks do not cover the text"); return MBW_E_HIP; }
    unsigned long long prim = 0;
    TRY(hipMemcpyAsync(&prim, dprim.p, 8, hipMemcpyDeviceToHost, st));
    TRY(hipStreamSynchronize(st));
    ix->primary = prim;
    // free the sorting space before the lines are built
    sa0.release(); sa1.release(); key0.release(); key1.release(); nk1.release(); tmp_sa.release(); tmp_nk.release();
    bnd.release(); grp.release(); flag.release(); idx.release(); u_slot.release(); u_slot2.release(); u_gid.release();
    iota0.release();
    iota1.release(); gid1.release(); gseed.release(); gscan.release(); tmp.b.release();
    int r = build_lines(ix, B.p, st);
    if (r) return r;
    B.release();
    if (ix->isa_sample) {   // the packed text stays resident for direct extension of unique matches
      ix->n_text = Tw.n;
      ix->text = Tw.detach();
      ix->bytes += ix->n_text * sizeof(uint64_t);
    }
    r = build_kmer_table(ix, st);
    if (r) return r;
    TRY(hipStreamSynchronize(st));
    return 0;
  }();
  (void)hipStreamDestroy(st);
  if (!rc) {
    try {
      ix->contigs = new mbw_contigs();
      ix->contigs->name.push_back("");
      ix->contigs->start.push_back(0);
      ix->contigs->len.push_back(len);
    } catch (...) { mbw_set_error("host allocation failed"); rc = MBW_E_NOMEM; }
  }
  if (rc) { mbw_index_free(ix); return rc; }
  *out = ix;
  return MBW_OK;
}

extern "C" int mbw_index_info(const mbw_index *ix, mbw_index_info_t *o) {
  if (!ix || !o) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  o->n = ix->n; o->len_r = ix->len_r; o->primary = ix->primary; o->n_lines = ix->n_lines;
  o->bytes_resident = ix->bytes;
  for (int a = 0; a < 5; ++a) o->C[a] = ix->C[a];
  o->bases_per_line = MBW_BPL; o->line_bytes = MBW_LINE_BYTES; o->sa_sample = ix->sa_sample;
  o->kmer_k = ix->kmer_k; o->bisulfite = ix->bisulfite; o->device = ix->device;
  o->isa_sample = ix->isa_sample;
  o->sb_lines_log2 = ix->sb_shift;
  o->n_superblocks = ix->n_sb;
  return MBW_OK;
}

extern "C" int mbw_index_device_arrays(const mbw_index *ix, const void **lines, const void **ssa, const void **kmer) {
  if (!ix) { mbw_set_error("NULL index"); return MBW_E_INVAL; }
  if (lines) *lines = ix->lines;
  if (ssa) *ssa = ix->ssa;
  if (kmer) *kmer = ix->kmer;
  return MBW_OK;
}

extern "C" int mbw_index_superblock_table(const mbw_index *ix, const void **sbtab) {
  if (!ix || !sbtab) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  *sbtab = ix->sbtab;
  return MBW_OK;
}

extern "C" int mbw_index_contigs(const mbw_index *ix, uint64_t *n) {
  if (!ix || !n) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  *n = ix->contigs ? ix->contigs->name.size() : 0;
  return MBW_OK;
}

extern "C" int mbw_index_contig(const mbw_index *ix, uint64_t i, const char **name, uint64_t *start, uint64_t *len) {
  if (!ix || !ix->contigs) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  if (i >= ix->contigs->name.size()) { mbw_set_error("record index out of range"); return MBW_E_INVAL; }
  if (name) *name = ix->contigs->name[i].c_str();
  if (start) *start = ix->contigs->start[i];
  if (len) *len = ix->contigs->len[i];
  return MBW_OK;
}

extern "C" int mbw_ref_to_contig(const mbw_index *ix, uint64_t ref_pos, uint64_t *contig, uint64_t *offset) {
  if (!ix || !ix->contigs || !contig || !offset) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  if (ref_pos >= ix->len_r) { mbw_set_error("reference position out of range"); return MBW_E_INVAL; }
  const std::vector<uint64_t> &st = ix->contigs->start;
  const uint64_t i = (uint64_t)(std::upper_bound(st.begin(), st.end(), ref_pos) - st.begin()) - 1;
  *contig = i;
  *offset = ref_pos - st[i];
  return MBW_OK;
}

// Read a FASTA file: records start with '>' (the name is the header up to the first white space);
// sequence lines are concatenated with line breaks and blanks removed.
static int read_fasta(const char *path, std::vector<uint8_t> &seq, mbw_contigs &ct) {
  FILE *f = fopen(path, "rb");
  if (!f) { mbw_set_error(std::string("cannot open ") + path); return MBW_E_IO; }
  std::vector<char> buf(16u << 20);
  enum { LINE_START, IN_HEADER_NAME, IN_HEADER_REST, IN_SEQ } state = LINE_START;
  std::string name;
  bool any = false;
  int rc = MBW_OK;
  auto close_record = [&]() -> bool {
    if (!any) return true;
    const uint64_t l = seq.size() - ct.start.back();
    if (l == 0) { mbw_set_error("FASTA record '" + ct.name.back() + "' has no sequence"); return false; }
    ct.len.push_back(l);
    return true;
  };
  try {
    for (;;) {
      const size_t got = fread(buf.data(), 1, buf.size(), f);
      if (got == 0) break;
      for (size_t i = 0; i < got && !rc; ++i) {
        const char ch = buf[i];
        switch (state) {
          case LINE_START:
            if (ch == '>') {
              if (!close_record()) { rc = MBW_E_FORMAT; break; }
              any = true;
              name.clear();
              ct.start.push_back(seq.size());
              state = IN_HEADER_NAME;
              break;
            }
            state = IN_SEQ;
            [[fallthrough]];   // the first character of a sequence line
          case IN_SEQ:
            if (ch == '\n') { state = LINE_START; break; }
            if (ch == '\r' || ch == ' ' || ch == '\t') break;
            if (!any) { mbw_set_error("FASTA sequence before the first '>' header"); rc = MBW_E_FORMAT; break; }
            seq.push_back((uint8_t)ch);
            break;
          case IN_HEADER_NAME:
            if (ch == '\n') { ct.name.push_back(name); state = LINE_START; }
            else if (ch == ' ' || ch == '\t' || ch == '\r') { ct.name.push_back(name); state = IN_HEADER_REST; }
            else name.push_back(ch);
            break;
          case IN_HEADER_REST:
            if (ch == '\n') state = LINE_START;
            break;
        }
      }
      if (rc) break;
    }
    if (!rc && ferror(f)) { mbw_set_error(std::string("read failed: ") + path); rc = MBW_E_IO; }
    if (!rc && state == IN_HEADER_NAME) ct.name.push_back(name);
    if (!rc && !any) { mbw_set_error("no FASTA record in " + std::string(path)); rc = MBW_E_FORMAT; }
    if (!rc && !close_record()) rc = MBW_E_FORMAT;
  } catch (...) { mbw_set_error("host allocation failed"); rc = MBW_E_NOMEM; }
  fclose(f);
  return rc;
}

extern "C" int mbw_index_build_fasta(const char *fasta_path, const mbw_build_opts *opts, mbw_index **out) {
  if (!out) { mbw_set_error("out is NULL"); return MBW_E_INVAL; }
  *out = nullptr;
  if (!fasta_path || !opts) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  if (opts->ref_is_codes) { mbw_set_error("a FASTA reference is ASCII (ref_is_codes must be 0)"); return MBW_E_INVAL; }
  std::vector<uint8_t> seq;
  mbw_contigs *ct = new (std::nothrow) mbw_contigs();
  if (!ct) { mbw_set_error("host allocation failed"); return MBW_E_NOMEM; }
  int rc = read_fasta(fasta_path, seq, *ct);
  if (!rc) rc = mbw_index_build(seq.data(), seq.size(), opts, out);
  if (rc) { delete ct; return rc; }
  delete (*out)->contigs;
  (*out)->contigs = ct;
  return MBW_OK;
}

extern "C" int mbw_pos_to_ref(const mbw_index *ix, uint64_t pos, uint32_t len, int *strand, uint64_t *ref_pos) {
  if (!ix || !strand || !ref_pos) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  uint64_t half = (ix->n - 1) / 2;   // |R| (plain) or 2|R| (bisulfite)
  if (pos + len > ix->n - 1) { mbw_set_error("position out of range"); return MBW_E_INVAL; }
  uint64_t lr = ix->len_r;
  if (pos < half) { *strand = 0; *ref_pos = ix->bisulfite ? pos % lr : pos; }
  else {
    *strand = 1;
    uint64_t p = 2 * half - pos - len;  // position in the forward text of length `half`
    *ref_pos = ix->bisulfite ? p % lr : p;
  }
  return MBW_OK;
}

// ---------------------------------------------------------------------------------------------
// index files: header (magic, version, fields, FNV-1a of header and of each array) + arrays
static const uint64_t kMagic = 0x3158444e4957424dull;  // "MBWINDX1"
static const uint32_t kVersion = 7;

struct FileHeader {
  uint64_t magic;
  uint32_t version, bpl;
  uint64_t n, len_r, primary, n_lines, n_ssa;
  uint64_t C[5];
  int32_t sa_sample, kmer_k, bisulfite, n_sb;
  uint64_t sb[MBW_MAX_SB * 8];
  int32_t isa_sample, sb_shift;
  uint64_t n_text, n_isa, n_orig;
  uint64_t sum_lines, sum_ssa, sum_kmer, sum_text, sum_isa, sum_orig;
  uint64_t contig_bytes, sum_contigs;   // the record table (its file form), after the arrays
  uint64_t sum_header;
};

static uint64_t fnv(const void *p, size_t n, uint64_t h = 1469598103934665603ull) {
  const uint8_t *b = (const uint8_t *)p;
  for (size_t i = 0; i < n; ++i) { h ^= b[i]; h *= 1099511628211ull; }
  return h;
}

// checksum of a large array: FNV-1a over its 64-bit words, each added to its word index (order
// sensitive); computed chunk by chunk as the array streams through the host
struct SumWords {
  uint64_t h = 1469598103934665603ull, i = 0;
  void add(const void *p, size_t bytes) {
    const uint64_t *w = (const uint64_t *)p;
    for (size_t k = 0; k < bytes / 8; ++k, ++i) { h ^= w[k] + i; h *= 1099511628211ull; }
  }
};

// Arrays move between the device and an index file through two pinned host chunks on a stream of
// their own: host memory stays bounded whatever the index size (39 GB at 3.1 Gbp), the copy of
// one chunk overlaps the file I/O and checksum of the other, and every array is checksummed on
// the way.
static const size_t kChunk = 64ull << 20;

struct Staging {
  uint8_t *buf[2] = {nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipStream_t st = nullptr;
  int init() {
    TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    for (int b = 0; b < 2; ++b) {
      TRY(hipHostMalloc((void **)&buf[b], kChunk, hipHostMallocDefault));
      TRY(hipEventCreateWithFlags(&ev[b], hipEventDisableTiming));
      TRY(hipEventRecord(ev[b], st));
    }
    return 0;
  }
  ~Staging() {
    if (st) (void)hipStreamSynchronize(st);   // no copy may still use a chunk being freed
    for (int b = 0; b < 2; ++b) {
      if (ev[b]) (void)hipEventDestroy(ev[b]);
      if (buf[b]) (void)hipHostFree(buf[b]);
    }
    if (st) (void)hipStreamDestroy(st);
  }
};

// device -> file; the download of chunk c + 1 runs while chunk c is checksummed and written
static int save_array(Staging &S, FILE *f, const void *dev, size_t bytes, uint64_t *sum) {
  SumWords h;
  const uint8_t *d = (const uint8_t *)dev;
  const size_t nc = (bytes + kChunk - 1) / kChunk;
  auto fetch = [&](size_t c) -> int {
    const size_t off = c * kChunk;
    TRY(hipMemcpyAsync(S.buf[c & 1], d + off, std::min(kChunk, bytes - off), hipMemcpyDeviceToHost, S.st));
    TRY(hipEventRecord(S.ev[c & 1], S.st));
    return 0;
  };
  if (nc) { int r = fetch(0); if (r) return r; }
  for (size_t c = 0; c < nc; ++c) {
    const size_t len = std::min(kChunk, bytes - c * kChunk);
    TRY(hipEventSynchronize(S.ev[c & 1]));
    if (c + 1 < nc) { int r = fetch(c + 1); if (r) return r; }
    h.add(S.buf[c & 1], len);
    if (fwrite(S.buf[c & 1], 1, len, f) != len) { mbw_set_error("index file write failed"); return MBW_E_IO; }
  }
  *sum = h.h;
  return 0;
}

// file -> device; chunk c + 1 is read and checksummed while chunk c uploads
static int load_array(Staging &S, FILE *f, void *dev, size_t bytes, uint64_t *sum) {
  SumWords h;
  uint8_t *d = (uint8_t *)dev;
  for (size_t off = 0, c = 0; off < bytes; off += kChunk, ++c) {
    const size_t len = std::min(kChunk, bytes - off);
    TRY(hipEventSynchronize(S.ev[c & 1]));   // the chunk's previous upload has finished
    if (fread(S.buf[c & 1], 1, len, f) != len) { mbw_set_error("truncated index file"); return MBW_E_FORMAT; }
    h.add(S.buf[c & 1], len);
    TRY(hipMemcpyAsync(d + off, S.buf[c & 1], len, hipMemcpyHostToDevice, S.st));
    TRY(hipEventRecord(S.ev[c & 1], S.st));
  }
  TRY(hipStreamSynchronize(S.st));
  *sum = h.h;
  return 0;
}

static uint64_t kmer_bytes(int k) { return k ? (1ull << (2 * k)) * 16 : 0; }

extern "C" int mbw_index_save(const mbw_index *ix, const char *path) {
  if (!ix || !path) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  TRY(hipSetDevice(ix->device));
  FileHeader hd;
  memset(&hd, 0, sizeof(hd));
  hd.magic = kMagic; hd.version = kVersion; hd.bpl = MBW_BPL;
  hd.n = ix->n; hd.len_r = ix->len_r; hd.primary = ix->primary; hd.n_lines = ix->n_lines; hd.n_ssa = ix->n_ssa;
  for (int a = 0; a < 5; ++a) hd.C[a] = ix->C[a];
  hd.sa_sample = ix->sa_sample; hd.kmer_k = ix->kmer ? ix->kmer_k : 0; hd.bisulfite = ix->bisulfite;
  hd.n_sb = ix->n_sb;
  memcpy(hd.sb, ix->sb_host, sizeof(hd.sb));
  hd.isa_sample = ix->isa_sample; hd.sb_shift = ix->sb_shift; hd.n_text = ix->n_text; hd.n_isa = ix->n_isa; hd.n_orig = ix->n_orig;
  Staging S;
  int r = S.init();
  if (r) return r;
  FILE *f = fopen(path, "wb");
  if (!f) { mbw_set_error(std::string("cannot open ") + path); return MBW_E_IO; }
  // the header goes first with the checksums left zero, and is rewritten once they are known
  r = fwrite(&hd, sizeof(hd), 1, f) == 1 ? 0 : MBW_E_IO;
  if (r) mbw_set_error(std::string("write failed: ") + path);
  if (!r) r = save_array(S, f, ix->lines, hd.n_lines * MBW_LINE_BYTES, &hd.sum_lines);
  if (!r) r = save_array(S, f, ix->ssa, hd.n_ssa * 8, &hd.sum_ssa);
  if (!r) r = save_array(S, f, ix->kmer, kmer_bytes(hd.kmer_k), &hd.sum_kmer);
  if (!r) r = save_array(S, f, ix->text, hd.n_text * 8, &hd.sum_text);
  if (!r) r = save_array(S, f, ix->isa, hd.n_isa * 8, &hd.sum_isa);
  if (!r) r = save_array(S, f, ix->orig, hd.n_orig * 8, &hd.sum_orig);
  if (!r) {
    const std::vector<uint8_t> cb = ix->contigs->serialize();
    hd.contig_bytes = cb.size();
    hd.sum_contigs = fnv(cb.data(), cb.size());
    if (fwrite(cb.data(), 1, cb.size(), f) != cb.size()) { mbw_set_error(std::string("write failed: ") + path); r = MBW_E_IO; }
  }
  if (!r) {
    hd.sum_header = fnv(&hd, offsetof(FileHeader, sum_header));
    if (fseek(f, 0, SEEK_SET) != 0 || fwrite(&hd, sizeof(hd), 1, f) != 1) {
      mbw_set_error(std::string("write failed: ") + path); r = MBW_E_IO;
    }
  }
  if (fclose(f) != 0 && !r) { mbw_set_error(std::string("write failed: ") + path); r = MBW_E_IO; }
  return r;
}

extern "C" int mbw_index_load(const char *path, int device, mbw_index **out) {
  if (!path || !out) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  *out = nullptr;
  FILE *f = fopen(path, "rb");
  if (!f) { mbw_set_error(std::string("cannot open ") + path); return MBW_E_IO; }
  FileHeader hd;
  if (fread(&hd, sizeof(hd), 1, f) != 1) { fclose(f); mbw_set_error("short header"); return MBW_E_FORMAT; }
  // every field is checked against the limits the builder applies before anything is allocated: the
  // kernels index their LDS superblock table by line >> sb_shift, and row arithmetic assumes n < 2^39
  bool c_ok = hd.C[0] == 0 && hd.C[1] == 1;   // C[$] = 0 and exactly one $ row
  for (int a = 1; a < 4; ++a) c_ok = c_ok && hd.C[a] <= hd.C[a + 1];
  c_ok = c_ok && hd.C[4] <= hd.n;
  if (hd.magic != kMagic || hd.version != kVersion || hd.bpl != MBW_BPL ||
      hd.sum_header != fnv(&hd, offsetof(FileHeader, sum_header)) || hd.n < 3 || hd.n >= (1ull << 39) ||
      hd.len_r == 0 || hd.n != (hd.bisulfite ? 4 : 2) * hd.len_r + 1 || hd.primary >= hd.n || !c_ok ||
      hd.n_lines != hd.n / MBW_BPL + 1 || hd.sb_shift < 1 || hd.sb_shift > MBW_SB_SHIFT || hd.n_sb < 1 ||
      hd.n_sb > MBW_MAX_SB || (hd.bisulfite != 0 && hd.bisulfite != 1) ||
      hd.sa_sample < 1 || hd.sa_sample > 1024 || hd.n_ssa != (hd.n + hd.sa_sample - 1) / hd.sa_sample ||
      hd.kmer_k < 0 || hd.kmer_k > 15 || hd.n_sb != (int)(((hd.n_lines - 1) >> hd.sb_shift) + 1) ||
      hd.isa_sample < 0 || hd.isa_sample > 64 ||
      (hd.isa_sample ? (hd.n_isa != (hd.n - 1) / hd.isa_sample + 1 || hd.n_text != (hd.n - 1 + 31) / 32 + 4)
                     : (hd.n_isa != 0 || hd.n_text != 0)) ||
      hd.n_orig != (hd.bisulfite ? (hd.len_r + 31) / 32 + 2 : 0) || hd.contig_bytes < 8 ||
      hd.contig_bytes > (1ull << 32) || hd.contig_bytes % 8) {
    fclose(f); mbw_set_error("bad magic, version or header fields"); return MBW_E_FORMAT;
  }
  const uint64_t kb = kmer_bytes(hd.kmer_k);
  const uint64_t payload =
      hd.n_lines * MBW_LINE_BYTES + hd.n_ssa * 8 + kb + (hd.n_text + hd.n_isa + hd.n_orig) * 8 + hd.contig_bytes;
  // the file must hold exactly the arrays its header states (checked before any device allocation)
  if (fseeko(f, 0, SEEK_END) != 0) { fclose(f); mbw_set_error("cannot seek index file"); return MBW_E_IO; }
  const off_t fsize = ftello(f);
  if (fsize < 0 || (uint64_t)fsize != sizeof(hd) + payload || fseeko(f, (off_t)sizeof(hd), SEEK_SET) != 0) {
    fclose(f);
    mbw_set_error((fsize >= 0 && (uint64_t)fsize < sizeof(hd) + payload) ? "truncated index file"
                                                                          : "index file size differs from its header");
    return MBW_E_FORMAT;
  }
  int rc = [&]() -> int { TRY(hipSetDevice(device)); return 0; }();
  if (rc) { fclose(f); return rc; }
  mbw_index *ix = new mbw_index();
  memset(ix, 0, sizeof(*ix));
  ix->device = device; ix->n = hd.n; ix->len_r = hd.len_r; ix->primary = hd.primary; ix->n_lines = hd.n_lines;
  ix->n_ssa = hd.n_ssa; for (int a = 0; a < 5; ++a) ix->C[a] = hd.C[a];
  ix->sa_sample = hd.sa_sample; ix->kmer_k = hd.kmer_k; ix->bisulfite = hd.bisulfite;
  ix->n_sb = hd.n_sb;
  ix->sb_shift = hd.sb_shift;
  memcpy(ix->sb_host, hd.sb, sizeof(hd.sb));
  ix->isa_sample = hd.isa_sample; ix->n_text = hd.n_text; ix->n_isa = hd.n_isa; ix->n_orig = hd.n_orig;
  rc = [&]() -> int {
    Staging S;
    int r = S.init();
    if (r) return r;
    auto place = [&](auto **dst, uint64_t bytes, uint64_t want) -> int {
      uint64_t got = 0;
      if (bytes) TRY(hipMalloc((void **)dst, bytes));
      int e = load_array(S, f, *dst, bytes, &got);
      if (e) return e;
      if (got != want) { mbw_set_error("index checksum mismatch"); return MBW_E_FORMAT; }
      return 0;
    };
    TRY(hipMalloc((void **)&ix->sbtab, sizeof(hd.sb)));
    TRY(hipMemcpy(ix->sbtab, hd.sb, sizeof(hd.sb), hipMemcpyHostToDevice));
    if ((r = place(&ix->lines, hd.n_lines * MBW_LINE_BYTES, hd.sum_lines))) return r;
    if ((r = place(&ix->ssa, hd.n_ssa * 8, hd.sum_ssa))) return r;
    if ((r = place(&ix->kmer, kb, hd.sum_kmer))) return r;
    if ((r = place(&ix->text, hd.n_text * 8, hd.sum_text))) return r;
    if ((r = place(&ix->isa, hd.n_isa * 8, hd.sum_isa))) return r;
    if ((r = place(&ix->orig, hd.n_orig * 8, hd.sum_orig))) return r;
    std::vector<uint8_t> cb(hd.contig_bytes);
    if (fread(cb.data(), 1, cb.size(), f) != cb.size()) { mbw_set_error("truncated index file"); return MBW_E_FORMAT; }
    if (fnv(cb.data(), cb.size()) != hd.sum_contigs) { mbw_set_error("index checksum mismatch"); return MBW_E_FORMAT; }
    ix->contigs = new mbw_contigs();
    if (!ix->contigs->parse(cb.data(), cb.size(), hd.len_r)) { mbw_set_error("bad record table"); return MBW_E_FORMAT; }
    ix->bytes = hd.n_lines * MBW_LINE_BYTES + hd.n_ssa * 8 + kb + sizeof(hd.sb) + (hd.n_text + hd.n_isa + hd.n_orig) * 8;
    return 0;
  }();
  fclose(f);
  if (rc) { mbw_index_free(ix); return rc; }
  *out = ix;
  return MBW_OK;
}
