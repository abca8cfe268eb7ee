// Host-side state of one mbw_ctx (shared by the seeding and mate-rescue entry points) and the
// helpers that grow its device buffers.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <string>
#include <vector>

#include "mbw_internal.h"
#include "../../include/mbw.h"

#define MBW_CTL_WORDS 16   // u64 counters of the control block of one call

struct mbw_ctx {
  const mbw_index *ix;
  int device;
  int n_cu;
  // Device buffers: grow-only stream-ordered allocations, or (epoch != 0) carved for one call from a
  // work space that the caller provides
  struct Buf { void *p = nullptr; size_t bytes = 0; uint32_t epoch = 0; };
  // seeding
  Buf codes, ascii, lens, offs, raw, subq, keys0, keys1, vals0, vals1, flag, idx, seeds, npos, posoff, xrows, pos, pos2,
      keep, kidx, temp, ctl, pwords, pnmask, woffs, nwords, wread, q1, q2, bf0, bf1, bp0, bp1, bid0, bid1, bk0, bk1, q1s,
      q2s, sc0, sc1, pseed, pcnt, ppoff, pieces, kpos, utask, ures;
  // mate-rescue prefilter (its own buffers, so that it leaves the last seeding result intact)
  Buf rc_lens, rc_wide, rc_offs, rc_ascii, rc_cand, rc_ctl, rc_hits, rc_flags, rc_pass;
  // chaining (its own buffers likewise)
  Buf ch_ctl, ch_cnt, ch_aoff, ch_slot, ch_cslot, ch_A, ch_As, ch_k2a, ch_k2b, ch_k1a, ch_k1b, ch_va, ch_vb, ch_F, ch_P,
      ch_U, ch_CH, ch_CA, ch_nch, ch_nanc, ch_choff, ch_anoff, ch_out, ch_outa;
  // work space mode (mbw_seed_into and its variant on the static scratch array): every buffer of the
  // call is carved from [arena, arena + arena_size); arena_need is the high-water mark asked for
  uint8_t *arena = nullptr;
  size_t arena_size = 0, arena_used = 0, arena_need = 0;
  size_t arena_hint = 0;   // estimate of the whole call's need, reported when an allocation does not fit
  uint32_t epoch = 0;
  hipEvent_t ev[8] = {};
  // SMEM launches whose device time is still to be read: a start and an end event each, read once
  // the host has waited for the stream anyway (no wait of its own per launch)
  static const int kLaunchSlots = 8;
  hipEvent_t lev[2 * kLaunchSlots] = {};
  int n_pending = 0;
  struct LaunchNote { int round, staged, kind, grid; uint64_t queries; uint32_t chunk; };
  LaunchNote pending[kLaunchSlots];
  hipStream_t cur = nullptr;   // stream of the current / last call
  hipStream_t own = nullptr;   // the context's own stream: frees its buffers when it is destroyed
  unsigned long long host_ctl[MBW_CTL_WORDS];
  uint64_t *hfetch = nullptr;   // pinned host words that a kernel fills with the sizes the host waits for
  uint64_t *dfetch = nullptr;   // ... the same memory as the device addresses it
  float ms_smem;
  int n_smem_launches;

  std::vector<Buf *> buffers() {
    return {&codes, &ascii, &lens, &offs, &raw, &subq, &keys0, &keys1, &vals0, &vals1, &flag, &idx, &seeds, &npos,
            &posoff, &xrows, &pos, &pos2, &keep, &kidx, &temp, &ctl, &pwords, &pnmask, &woffs, &nwords, &wread, &q1,
            &q2, &bf0, &bf1, &bp0, &bp1, &bid0, &bid1, &bk0, &bk1, &q1s, &q2s, &sc0, &sc1, &pseed, &pcnt, &ppoff,
            &pieces, &kpos, &utask, &ures, &rc_lens, &rc_wide, &rc_offs, &rc_ascii, &rc_cand, &rc_ctl, &rc_hits, &rc_flags, &rc_pass,
            &ch_ctl, &ch_cnt, &ch_aoff, &ch_slot, &ch_cslot, &ch_A, &ch_As, &ch_k2a, &ch_k2b, &ch_k1a, &ch_k1b, &ch_va,
            &ch_vb, &ch_F, &ch_P, &ch_U, &ch_CH, &ch_CA, &ch_nch, &ch_nanc, &ch_choff, &ch_anoff, &ch_out, &ch_outa};
  }
};

// cap on the device work space of every context, 0 = none (mbw_debug_set_mem_limit)
extern std::atomic<unsigned long long> g_mbw_mem_limit;

// Buffers grow on the call's stream with the stream-ordered allocator, so that a context growing
// its work space does not wait for work of other contexts on other streams.  A growth the cap
// refuses leaves the buffer as it was.
static inline int grow(mbw_ctx *c, mbw_ctx::Buf &b, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (c->arena) {
    if (b.epoch == c->epoch && b.bytes >= bytes) return 0;
    const size_t want = (bytes + 255) & ~(size_t)255;
    if (c->arena_used + want > c->arena_size) {
      if (c->arena_used + want > c->arena_need) c->arena_need = c->arena_used + want;
      if (c->arena_hint > c->arena_need) c->arena_need = c->arena_hint;
      mbw_set_error("work space too small: this call needs at least " + std::to_string(c->arena_used + want) +
                    " bytes of the " + std::to_string(c->arena_size) + " given");
      return MBW_E_CAPACITY;
    }
    b.p = c->arena + c->arena_used;
    b.bytes = want;
    b.epoch = c->epoch;
    c->arena_used += want;
    if (c->arena_used > c->arena_need) c->arena_need = c->arena_used;
    return 0;
  }
  if (b.bytes >= bytes) return 0;
  size_t want = bytes + bytes / 2 + 256;
  if (const unsigned long long lim = g_mbw_mem_limit.load(std::memory_order_relaxed)) {
    unsigned long long used = 0;
    for (auto *x : c->buffers()) used += x->bytes;
    if (used - b.bytes + want > lim) {
      mbw_set_error("device work space over the debug cap (" + std::to_string(lim) + " bytes)");
      return MBW_E_NOMEM;
    }
  }
  if (b.p) { (void)hipFreeAsync(b.p, c->cur); b.p = nullptr; b.bytes = 0; }
  hipError_t e = hipMallocAsync(&b.p, want, c->cur);
  if (e != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();   // the failure is reported here: later launch checks must not see it
    mbw_set_error(std::string("hipMalloc(") + std::to_string(want) + "): " + hipGetErrorString(e));
    return MBW_E_NOMEM;
  }
  b.bytes = want;
  return 0;
}
#define GROW(buf, bytes) do { int r_ = grow(c, buf, bytes); if (r_) return r_; } while (0)

// A buffer that is no longer needed (work space mode: its space is simply not reused in this call).
static inline void release(mbw_ctx *c, mbw_ctx::Buf &b, hipStream_t st) {
  if (!c->arena && b.p) (void)hipFreeAsync(b.p, st);
  b = mbw_ctx::Buf();
}

// For the duration of one work-space call: the context's own buffers are set aside (they stay
// allocated for later calls) and every buffer of the call is carved from the caller's work space.
struct ArenaScope {
  mbw_ctx *c;
  std::vector<mbw_ctx::Buf> saved;
  ArenaScope(mbw_ctx *ctx, void *base, size_t bytes) : c(ctx) {
    for (auto *b : c->buffers()) {
      saved.push_back(*b);
      if (b != &c->ctl) *b = mbw_ctx::Buf();
    }
    c->arena = (uint8_t *)base;
    c->arena_size = bytes;
    c->arena_used = 0;
    c->arena_need = 0;
    c->arena_hint = 0;
    c->epoch = c->epoch + 1 ? c->epoch + 1 : 1;
  }
  ~ArenaScope() {
    auto bufs = c->buffers();
    for (size_t t = 0; t < bufs.size(); ++t) *bufs[t] = saved[t];
    c->arena = nullptr;
    c->arena_size = c->arena_used = 0;
  }
};

static inline bool is_device_ptr(const void *p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) { (void)hipGetLastError(); return false; }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// Make the temporary buffer large enough for f (a device-wide rocPRIM call of the size it captures) without
// running it: a later call on fewer items then needs no larger buffer.
template <class F>
static int reserve_temp(mbw_ctx *c, F f) {
  size_t tb = 0;
  MBW_HIP_TRY(f((void *)nullptr, tb));
  GROW(c->temp, tb);
  return 0;
}

// run a device-wide rocPRIM algorithm with the context's temporary buffer
template <class F>
static int prim_call(mbw_ctx *c, F f) {
  size_t tb = 0;
  MBW_HIP_TRY(f((void *)nullptr, tb));
  GROW(c->temp, tb);
  size_t have = c->temp.bytes;
  MBW_HIP_TRY(f(c->temp.p, have));
  return 0;
}

// The seeding path's sizing model for a call on n reads of `bases` bases in work space mode: the
// work space it is expected to need and the seeds, positions and refined pieces of a typical
// result (a real call may need less, or more for an atypical result).
struct MbwSizeModel { uint64_t ws, seeds, pos, pieces; };
MbwSizeModel mbw_size_model(const mbw_ctx *c, uint64_t n, uint64_t bases, bool host_reads, const mbw_seed_opts *o);
