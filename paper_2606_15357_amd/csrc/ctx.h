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
  struct Buf { void *p = nullptr; size_t bytes = 0; };   // grow-only device buffers (stream-ordered allocations)
  // seeding
  Buf codes, ascii, lens, offs, raw, subq, keys0, keys1, vals0, vals1, flag, idx, seeds, npos, posoff, xrows, pos, pos2,
      keep, kidx, temp, ctl, pwords, pnmask, woffs, nwords, wread, q1, q2, bf0, bf1, bp0, bp1, bid0, bid1, bk0, bk1, q1s,
      q2s, sc0, sc1, pseed, pcnt, ppoff, pieces, kpos;
  // mate-rescue prefilter (its own buffers, so that it leaves the last seeding result intact)
  Buf rc_lens, rc_wide, rc_offs, rc_ascii, rc_cand, rc_ctl, rc_hits, rc_flags, rc_pass;
  // chaining (its own buffers likewise)
  Buf ch_ctl, ch_cnt, ch_aoff, ch_slot, ch_cslot, ch_A, ch_As, ch_k2a, ch_k2b, ch_k1a, ch_k1b, ch_va, ch_vb, ch_F, ch_P,
      ch_U, ch_CH, ch_CA, ch_nch, ch_nanc, ch_choff, ch_anoff, ch_out, ch_outa;
  hipEvent_t ev[8] = {};
  // SMEM launches whose device time is still to be read: a start and an end event each, read once
  // the host has waited for the stream anyway (no wait of its own per launch)
  static const int kLaunchSlots = 8;
  hipEvent_t lev[2 * kLaunchSlots] = {};
  int n_pending = 0;
  struct LaunchNote { int round, staged, grid; uint64_t queries; uint32_t chunk; };
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
            &pieces, &kpos, &rc_lens, &rc_wide, &rc_offs, &rc_ascii, &rc_cand, &rc_ctl, &rc_hits, &rc_flags, &rc_pass,
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
    mbw_set_error(std::string("hipMalloc(") + std::to_string(want) + "): " + hipGetErrorString(e));
    return MBW_E_NOMEM;
  }
  b.bytes = want;
  return 0;
}
#define GROW(buf, bytes) do { int r_ = grow(c, buf, bytes); if (r_) return r_; } while (0)

static inline bool is_device_ptr(const void *p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) { (void)hipGetLastError(); return false; }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// run a hipcub device-wide algorithm with the context's temporary buffer
template <class F>
static int cub_call(mbw_ctx *c, F f) {
  size_t tb = 0;
  MBW_HIP_TRY(f((void *)nullptr, tb));
  GROW(c->temp, tb);
  size_t have = c->temp.bytes;
  MBW_HIP_TRY(f(c->temp.p, have));
  return 0;
}
