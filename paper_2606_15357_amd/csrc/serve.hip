// Serving runtime: a request loop around the seeding path with the index resident in HBM.
//
// Device memory is fixed when the server opens.  Every worker thread owns a seeding context, a HIP
// stream and one device arena: the work space of its calls plus result buffers for seeds,
// positions and refined pieces, sized from the batch budget (or from the device bytes the caller
// grants) with the seeding path's own sizing model.  Batches run through mbw_seed_into on that
// arena, so a running server allocates no device memory.
//
// Admission is by device memory.  A request whose estimated work space alone exceeds a worker's
// arena is refused at submission (MBW_E_CAPACITY).  A free worker takes queued requests in arrival
// order into one device batch while the batch's estimated work space fits its arena and the read /
// base budget holds, so requests that arrive while other batches run join the next batch at once
// (continuous batching), and the batches of different workers run on the device at the same time.
// A batch that still runs short (a result larger than the model assumes, or an allocation failure)
// is split in two and each half run again, down to single requests: a request never fails because
// of the requests it was batched with.
//
// Requests are queued with host copies of their reads, or by reference when the caller keeps the
// buffers until the request is finished.  A worker copies the next batch into pinned staging while
// the previous batch's results are still coming back over PCIe.  A batch's seeds come back sorted by
// read, so each request's seeds and positions are a contiguous slice; read ids and position offsets
// are made relative to each request on the device, and the batch is downloaded once into a pinned
// buffer its requests share.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ctx.h"
#include "mbw_internal.h"
#include "../../include/mbw.h"

namespace {

// grow-only pinned host buffer
struct Pinned {
  void *p = nullptr;
  size_t bytes = 0;
  // grow to at least `want` bytes (to twice that unless exact: a buffer sized once for its largest
  // use need not leave room)
  int ensure(size_t want, bool exact = false) {
    if (want <= bytes) return 0;
    if (p) { (void)hipHostFree(p); p = nullptr; bytes = 0; }
    const size_t b = exact ? want : 2 * want + 4096;
    if (hipHostMalloc(&p, b, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();   // reported by the return code: later launch checks must not see it
      p = nullptr;
      return MBW_E_NOMEM;
    }
    bytes = b;
    return 0;
  }
  ~Pinned() { if (p) (void)hipHostFree(p); }
};

// Per-request split of a batch's result, on the device.  Seeds come back sorted by read and
// positions and refined pieces follow their seeds, so request i (reads [rstart[i], rstart[i+1]))
// owns a contiguous run of each: SplitBound i holds the first seed, position and piece of that run
// (entry nreq closes the last one).  Read ids, position offsets and the pieces' seed indexes are
// then made relative to their request in place.
struct SplitBound { uint64_t t0, p0, c0; };

__device__ __forceinline__ uint64_t seeds_before_read(const mbw_seed_t *sd, uint64_t n, uint32_t r) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) / 2;
    if (sd[mid].read_id < r) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// the request holding read r: the last i with rstart[i] <= r (empty requests share their start
// with the next one)
__device__ __forceinline__ uint32_t request_of(const uint32_t *rstart, uint32_t nreq, uint32_t r) {
  uint32_t lo = 0, hi = nreq;   // rstart[0] = 0 <= r
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (rstart[mid] <= r) lo = mid; else hi = mid;
  }
  return lo;
}

__global__ void k_split_bounds(const mbw_seed_t *__restrict__ sd, uint64_t ns, uint64_t np, const mbw_piece_t *__restrict__ pc,
                               uint64_t nc, const uint32_t *__restrict__ rstart, uint32_t nreq, SplitBound *__restrict__ b) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= nreq; i += gridDim.x * blockDim.x) {
    const uint64_t t0 = i == nreq ? ns : seeds_before_read(sd, ns, rstart[i]);
    uint64_t lo = 0, hi = nc;
    while (lo < hi) {
      const uint64_t mid = (lo + hi) / 2;
      if (pc[mid].seed < t0) lo = mid + 1; else hi = mid;
    }
    b[i] = SplitBound{t0, t0 < ns ? sd[t0].pos_off : np, lo};
  }
}

__global__ void k_split_rebase(mbw_seed_t *__restrict__ sd, uint64_t ns, mbw_piece_t *__restrict__ pc, uint64_t nc,
                               const uint32_t *__restrict__ rstart, uint32_t nreq, const SplitBound *__restrict__ b) {
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < ns + nc; t += (uint64_t)gridDim.x * blockDim.x) {
    if (t < ns) {
      const uint32_t i = request_of(rstart, nreq, sd[t].read_id);
      sd[t].read_id -= rstart[i];
      sd[t].pos_off -= b[i].p0;
    } else {
      mbw_piece_t &q = pc[t - ns];
      const uint32_t i = request_of(rstart, nreq, q.read_id);
      q.read_id -= rstart[i];
      q.seed -= (uint32_t)b[i].t0;
    }
  }
}

// one batch's downloaded result, shared by its requests
struct BatchBuf {
  Pinned seeds, pos, pieces;
  int refs = 0;
  size_t bytes() const { return seeds.bytes + pos.bytes + pieces.bytes; }
};

static void pool_put(mbw_server *s, BatchBuf *b);

struct Request {
  uint64_t ticket = 0;
  std::vector<uint8_t> reads_copy;      // empty when submitted by reference
  std::vector<uint32_t> lengths_copy;
  const uint8_t *reads = nullptr;       // the copies or the caller's buffers
  const uint32_t *lengths = nullptr;
  uint64_t n_reads = 0, bases = 0;
  double t_submit = 0, t_start = 0, t_done = 0;
  uint64_t batch_id = 0, batch_reads = 0;
  uint32_t attempts = 0;                // device batches this request was part of
  int state = 0;   // 0 queued, 1 running, 2 done
  int rc = MBW_OK;
  std::string err;                      // the failure's message (errors are per thread)
  BatchBuf *buf = nullptr;          // the shared batch result
  uint64_t s0 = 0, ns = 0, p0 = 0, np = 0;   // this request's slice of it (seeds, positions,
  uint64_t c0 = 0, nc = 0;                    // refined pieces)
};

// requests in one device batch at most (sizes the per-batch split arrays)
constexpr uint32_t kMaxBatchRequests = 1u << 16;

// a worker's fixed device memory: one work space and two result slots (a batch's results are
// downloaded from one slot while the next batch seeds into the other)
struct ResultSlot {
  mbw_seed_t *seeds = nullptr;
  uint64_t *pos = nullptr;
  mbw_piece_t *pieces = nullptr;
  uint32_t *rstart = nullptr;     // per-batch split arrays (kMaxBatchRequests + 1 each)
  SplitBound *bounds = nullptr;
};

struct Arena {
  void *base = nullptr;
  uint64_t bytes = 0;
  void *ws = nullptr;
  uint64_t ws_bytes = 0;
  uint64_t seeds_cap = 0, pos_cap = 0, pieces_cap = 0;   // records per slot
  ResultSlot slot[2];
};

static uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

static uint64_t slot_bytes(const Arena &a) {
  return align256(a.seeds_cap * sizeof(mbw_seed_t)) + align256(a.pos_cap * sizeof(uint64_t)) +
         align256(a.pieces_cap * sizeof(mbw_piece_t)) + align256((kMaxBatchRequests + 1) * sizeof(uint32_t)) +
         align256((kMaxBatchRequests + 1) * sizeof(SplitBound));
}

// Carve an arena of `bytes` (0 = the size the model gives for a full batch of max_reads reads and
// max_bases bases) into work space and two result slots, in the proportions of that model.
static int plan_arena(const mbw_ctx *c, const mbw_serve_cfg &cfg, uint64_t bytes, Arena &a) {
  const uint64_t R = cfg.max_batch_reads, B = cfg.max_batch_bases;
  const uint64_t fixed = 2 * (align256((kMaxBatchRequests + 1) * sizeof(uint32_t)) +
                              align256((kMaxBatchRequests + 1) * sizeof(SplitBound))) + 8 * 256;
  const MbwSizeModel sm = mbw_size_model(c, R, B, true, &cfg.opts);
  const double m_ws = (double)sm.ws;
  const double m_seeds = (double)(sm.seeds + 4096) * sizeof(mbw_seed_t);
  const double m_pos = (double)(sm.pos + 4096) * sizeof(uint64_t);
  const double m_pieces = cfg.opts.bs_refine ? (double)(sm.pieces + 4096) * sizeof(mbw_piece_t) : 0.0;
  const double model = m_ws + 2 * (m_seeds + m_pos + m_pieces);
  if (bytes == 0) bytes = align256((uint64_t)model) + fixed;
  // the smallest arena admits one read of the longest length
  const MbwSizeModel one = mbw_size_model(c, 1, MBW_MAX_READ, true, &cfg.opts);
  double lf = ((double)one.ws + 256) / m_ws;
  lf = std::max(lf, (double)(one.seeds + 1) * sizeof(mbw_seed_t) / m_seeds);
  lf = std::max(lf, (double)(one.pos + 1) * sizeof(uint64_t) / m_pos);
  if (m_pieces > 0) lf = std::max(lf, (double)(one.pieces + 1) * sizeof(mbw_piece_t) / m_pieces);
  const uint64_t least = (uint64_t)(lf * model) + fixed + 4096;
  if (bytes < least) {
    mbw_set_error("serve device_bytes too small: each worker needs at least " + std::to_string(least) + " bytes");
    return MBW_E_INVAL;
  }
  const double f = (double)(bytes - fixed) / model;
  a.ws_bytes = align256((uint64_t)(m_ws * f)) - 256;
  a.seeds_cap = (uint64_t)(m_seeds * f) / sizeof(mbw_seed_t);
  a.pos_cap = (uint64_t)(m_pos * f) / sizeof(uint64_t);
  a.pieces_cap = (uint64_t)(m_pieces * f) / sizeof(mbw_piece_t);
  return MBW_OK;
}

static int alloc_arena(Arena &a) {
  const uint64_t want = align256(a.ws_bytes) + 2 * slot_bytes(a);
  if (const unsigned long long lim = g_mbw_mem_limit.load(std::memory_order_relaxed)) {
    if (want > lim) {
      mbw_set_error("serve arena of " + std::to_string(want) + " bytes over the debug cap (" + std::to_string(lim) +
                    " bytes)");
      return MBW_E_NOMEM;
    }
  }
  if (hipMalloc(&a.base, want) != hipSuccess) {
    (void)hipGetLastError();
    a.base = nullptr;
    mbw_set_error("hipMalloc of a serve arena (" + std::to_string(want) + " bytes) failed");
    return MBW_E_NOMEM;
  }
  uint8_t *p = (uint8_t *)a.base;
  a.ws = p; p += align256(a.ws_bytes);
  for (ResultSlot &r : a.slot) {
    r.seeds = (mbw_seed_t *)p; p += align256(a.seeds_cap * sizeof(mbw_seed_t));
    r.pos = (uint64_t *)p; p += align256(a.pos_cap * sizeof(uint64_t));
    r.pieces = a.pieces_cap ? (mbw_piece_t *)p : nullptr; p += align256(a.pieces_cap * sizeof(mbw_piece_t));
    r.rstart = (uint32_t *)p; p += align256((kMaxBatchRequests + 1) * sizeof(uint32_t));
    r.bounds = (SplitBound *)p; p += align256((kMaxBatchRequests + 1) * sizeof(SplitBound));
  }
  a.bytes = want;
  return MBW_OK;
}

}  // namespace

struct mbw_server {
  const mbw_index *ix = nullptr;
  mbw_serve_cfg cfg;
  std::mutex mu;
  std::condition_variable work_cv, done_cv;
  std::deque<Request *> queue;
  std::map<uint64_t, Request *> all;
  uint64_t next_ticket = 1, queued_bases = 0, next_batch = 1;
  bool stop = false;
  std::vector<std::thread> workers;
  std::chrono::steady_clock::time_point t0;
  mbw_serve_stats_t st{};
  bool trace = false;   // MBW_SERVE_TRACE=1: one line per batch on stderr
  std::vector<BatchBuf *> free_bufs;
  mbw_ctx *model_ctx = nullptr;   // worker 0's context, for the sizing model
  uint64_t ws_bytes = 0;          // every worker's work space and result buffers (records)
  uint64_t seeds_cap = 0, pos_cap = 0, pieces_cap = 0;

  void unref(BatchBuf *b) {   // with mu held: drop a request's reference to its batch result
    if (b && --b->refs == 0) pool_put(this, b);
  }

  double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }

  // whether a batch of n reads and `bases` bases fits a worker's arena by the sizing model (its
  // estimated work space in *need)
  bool fits(uint64_t n, uint64_t bases, uint64_t *need = nullptr) const {
    const MbwSizeModel m = mbw_size_model(model_ctx, n, bases, true, &cfg.opts);
    if (need) *need = m.ws;
    return m.ws <= ws_bytes && m.seeds <= seeds_cap && m.pos <= pos_cap && m.pieces <= pieces_cap;
  }
};

namespace {

// a batch whose results are on their way to the host
struct InFlight {
  std::vector<Request *> reqs;
  BatchBuf *bb = nullptr;
  int slot = 0;
  uint64_t bid = 0, nreads = 0;
  double tb0 = 0, tb1 = 0;
  float ms_device = 0;
};

// A worker: its context, compute stream, copy stream, arena and pinned staging.  Its finisher
// thread completes the batches whose downloads it queues, so the worker seeds the next batch into
// the other result slot meanwhile.
struct Worker {
  mbw_server *s = nullptr;
  mbw_ctx *ctx = nullptr;
  hipStream_t st = nullptr, cs = nullptr;
  hipEvent_t ev_split[2] = {nullptr, nullptr}, ev_done[2] = {nullptr, nullptr};
  Arena a;
  Pinned stage[2], lens[2], hreq, hbnd[2];
  std::mutex fmu;
  std::condition_variable fcv;
  std::deque<InFlight> fq;         // batches downloading, in order
  bool busy[2] = {false, false};   // result slot in use until its batch is completed
  bool fstop = false;
  std::thread finisher;
};

// Take queued requests for one batch (mu held): in arrival order while the batch's estimated work
// space fits the arena, within the read, base and request budgets.  The head request always fits
// (submission refused those that do not).
static std::vector<Request *> take_batch(mbw_server *s) {
  std::vector<Request *> batch;
  uint64_t nreads = 0, nbases = 0;
  while (!s->queue.empty() && batch.size() < kMaxBatchRequests) {
    Request *r = s->queue.front();
    if (!batch.empty() &&
        (nreads + r->n_reads > s->cfg.max_batch_reads || nbases + r->bases > s->cfg.max_batch_bases ||
         !s->fits(nreads + r->n_reads, nbases + r->bases)))
      break;
    s->queue.pop_front();
    s->queued_bases -= r->bases;
    batch.push_back(r);
    nreads += r->n_reads;
    nbases += r->bases;
  }
  if (!batch.empty()) {
    const double t = s->now();
    for (Request *r : batch) { r->state = 1; r->t_start = t; }
  }
  return batch;
}

// Concatenate a batch's reads and lengths into pinned staging slot k.  A large batch is copied by
// several threads (one thread's memcpy reaches about a third of the host's memory bandwidth).
static int stage_batch(Worker &w, int k, const std::vector<Request *> &batch) {
  uint64_t nreads = 0, nbases = 0;
  for (Request *r : batch) { nreads += r->n_reads; nbases += r->bases; }
  int rc = w.stage[k].ensure(nbases + 16);
  if (!rc) rc = w.lens[k].ensure((nreads + 1) * sizeof(uint32_t));
  if (rc) { mbw_set_error("pinned staging allocation failed"); return rc; }
  uint8_t *rb = (uint8_t *)w.stage[k].p;
  uint32_t *lb = (uint32_t *)w.lens[k].p;
  std::vector<uint64_t> ob(batch.size() + 1), orr(batch.size() + 1);
  for (size_t i = 0; i < batch.size(); ++i) {
    ob[i + 1] = ob[i] + batch[i]->bases;
    orr[i + 1] = orr[i] + batch[i]->n_reads;
  }
  auto copy = [&](size_t i0, size_t i1) {
    for (size_t i = i0; i < i1; ++i) {
      const Request *r = batch[i];
      if (r->bases) memcpy(rb + ob[i], r->reads, r->bases);
      if (r->n_reads) memcpy(lb + orr[i], r->lengths, r->n_reads * sizeof(uint32_t));
    }
  };
  const size_t nt = nbases >= (32ull << 20) ? std::min<size_t>(4, batch.size()) : 1;
  if (nt <= 1) { copy(0, batch.size()); return MBW_OK; }
  // split the requests into nt runs of about equal bytes
  std::vector<size_t> cut(nt + 1, batch.size());
  cut[0] = 0;
  for (size_t t = 1, i = 0; t < nt; ++t) {
    const uint64_t want = nbases * t / nt;
    while (i < batch.size() && ob[i] < want) ++i;
    cut[t] = std::max(i, cut[t - 1]);
  }
  std::vector<std::thread> th;
  try {
    for (size_t t = 1; t < nt; ++t) th.emplace_back(copy, cut[t], cut[t + 1]);
  } catch (...) {                 // no thread to be had: copy on this one
    for (auto &x : th) x.join();
    copy(0, batch.size());
    return MBW_OK;
  }
  copy(0, cut[1]);
  for (auto &x : th) x.join();
  return MBW_OK;
}

// A pinned buffer for a batch result of ns seeds, np positions and nc pieces: a pooled one that
// holds it if there is one (the smallest such), else the largest pooled one grown to it (rounded up
// to 64 MiB per array, so that few batches grow it again), else a new one.  Pinning host memory is
// slow, so buffers are kept for reuse; the pool holds at most 2 per worker.
static BatchBuf *get_buf(mbw_server *s, uint64_t ns, uint64_t np, uint64_t nc, int *rc) {
  const size_t want_s = (ns + 1) * sizeof(mbw_seed_t), want_p = (np + 1) * sizeof(uint64_t),
               want_c = nc ? (nc + 1) * sizeof(mbw_piece_t) : 0;
  auto fits = [&](const BatchBuf *b) {
    return b->seeds.bytes >= want_s && b->pos.bytes >= want_p && b->pieces.bytes >= want_c;
  };
  BatchBuf *b = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    size_t pick = s->free_bufs.size();
    for (size_t i = 0; i < s->free_bufs.size(); ++i) {
      const BatchBuf *x = s->free_bufs[i];
      if (fits(x) ? (pick == s->free_bufs.size() || !fits(s->free_bufs[pick]) || x->bytes() < s->free_bufs[pick]->bytes())
                  : (pick == s->free_bufs.size() || (!fits(s->free_bufs[pick]) && x->bytes() > s->free_bufs[pick]->bytes())))
        pick = i;
    }
    if (pick < s->free_bufs.size()) {
      b = s->free_bufs[pick];
      s->free_bufs.erase(s->free_bufs.begin() + pick);
    }
  }
  if (!b) b = new (std::nothrow) BatchBuf();
  if (!b) { mbw_set_error("host allocation failed"); *rc = MBW_E_NOMEM; return nullptr; }
  const size_t g = 64ull << 20;
  auto up = [&](size_t x) { return x ? (x + g - 1) / g * g : 0; };
  *rc = b->seeds.ensure(up(want_s), true);
  if (!*rc) *rc = b->pos.ensure(up(want_p), true);
  if (!*rc && want_c) *rc = b->pieces.ensure(up(want_c), true);
  if (*rc) {   // a buffer that could not grow is dropped, not pooled
    delete b;
    mbw_set_error("pinned result allocation failed");
    return nullptr;
  }
  return b;
}

// Return a buffer to the pool (mu held); beyond 2 per worker the smallest is freed.
static void pool_put(mbw_server *s, BatchBuf *b) {
  s->free_bufs.push_back(b);
  if (s->free_bufs.size() > 2 * (size_t)s->cfg.n_workers) {
    size_t m = 0;
    for (size_t i = 1; i < s->free_bufs.size(); ++i)
      if (s->free_bufs[i]->bytes() < s->free_bufs[m]->bytes()) m = i;
    delete s->free_bufs[m];
    s->free_bufs.erase(s->free_bufs.begin() + m);
  }
}

// Seed requests [i0, i1) of a staged batch (their reads start at staged byte rb0 and staged read
// rr0) into result slot `slot`, split the result per request on the device and start its download
// on the copy stream; on success `out` describes the batch in flight.
static int run_batch(Worker &w, int k, int slot, const std::vector<Request *> &batch, size_t i0, size_t i1,
                     uint64_t rb0, uint64_t rr0, InFlight &out) {
  mbw_server *s = w.s;
  const ResultSlot &rs_ = w.a.slot[slot];
  out.reqs.assign(batch.begin() + i0, batch.begin() + i1);
  out.slot = slot;
  const uint32_t nreq = (uint32_t)out.reqs.size();
  uint64_t nreads = 0;
  for (Request *r : out.reqs) nreads += r->n_reads;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    out.bid = s->next_batch++;
    s->st.batches++;
    s->st.batch_reads += nreads;
    for (Request *r : out.reqs) { r->batch_id = out.bid; r->batch_reads = nreads; r->attempts++; }
  }
  out.nreads = nreads;
  out.tb0 = s->now();
  mbw_seed_buffers ob;
  memset(&ob, 0, sizeof(ob));
  ob.workspace = w.a.ws; ob.workspace_bytes = w.a.ws_bytes;
  ob.seeds = rs_.seeds; ob.seeds_cap = w.a.seeds_cap;
  ob.pos = rs_.pos; ob.pos_cap = w.a.pos_cap;
  ob.pieces = rs_.pieces; ob.pieces_cap = w.a.pieces_cap;
  mbw_result res;
  memset(&res, 0, sizeof(res));
  int rc = mbw_seed_into(w.ctx, (const uint8_t *)w.stage[k].p + rb0, (const uint32_t *)w.lens[k].p + rr0, nreads,
                         s->cfg.min_seed_len, s->cfg.max_occ, &s->cfg.opts, (void *)w.st, &ob, &res);
  out.tb1 = s->now();
  out.ms_device = res.ms_total;
  if (rc) return rc;
  BatchBuf *bb = get_buf(s, res.n_seeds, res.n_pos, res.n_pieces, &rc);
  out.bb = bb;
  if (rc) return rc;
  // per-request split on the device, then the download of the batch and of the request bounds
  uint32_t *rs = (uint32_t *)w.hreq.p;
  uint64_t r0 = 0;
  for (uint32_t i = 0; i < nreq; ++i) { rs[i] = (uint32_t)r0; r0 += out.reqs[i]->n_reads; }
  rs[nreq] = (uint32_t)r0;
  const unsigned gb = (unsigned)std::min<uint64_t>((nreq + 256) / 256, 1024);
  const unsigned gr = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((res.n_seeds + res.n_pieces + 255) / 256, 4096));
#define SRV_TRY(x) do { if ((x) != hipSuccess) { mbw_set_error(std::string(#x) + ": " + hipGetErrorString(hipGetLastError())); return MBW_E_HIP; } } while (0)
  SRV_TRY(hipMemcpyAsync(rs_.rstart, rs, (nreq + 1) * sizeof(uint32_t), hipMemcpyHostToDevice, w.st));
  k_split_bounds<<<gb, 256, 0, w.st>>>(res.seeds, res.n_seeds, res.n_pos, res.pieces, res.n_pieces, rs_.rstart, nreq,
                                       rs_.bounds);
  if (res.n_seeds + res.n_pieces)
    k_split_rebase<<<gr, 256, 0, w.st>>>((mbw_seed_t *)res.seeds, res.n_seeds, (mbw_piece_t *)res.pieces, res.n_pieces,
                                         rs_.rstart, nreq, rs_.bounds);
  SRV_TRY(hipGetLastError());
  // hreq is rewritten by the next batch: the copy of it above must have been taken first
  SRV_TRY(hipEventRecord(w.ev_split[slot], w.st));
  SRV_TRY(hipStreamWaitEvent(w.cs, w.ev_split[slot], 0));
  SRV_TRY(hipMemcpyAsync(w.hbnd[slot].p, rs_.bounds, (nreq + 1) * sizeof(SplitBound), hipMemcpyDeviceToHost, w.cs));
  if (res.n_seeds)
    SRV_TRY(hipMemcpyAsync(bb->seeds.p, res.seeds, res.n_seeds * sizeof(mbw_seed_t), hipMemcpyDeviceToHost, w.cs));
  if (res.n_pos)
    SRV_TRY(hipMemcpyAsync(bb->pos.p, res.pos, res.n_pos * sizeof(uint64_t), hipMemcpyDeviceToHost, w.cs));
  if (res.n_pieces)
    SRV_TRY(hipMemcpyAsync(bb->pieces.p, res.pieces, res.n_pieces * sizeof(mbw_piece_t), hipMemcpyDeviceToHost, w.cs));
  SRV_TRY(hipEventRecord(w.ev_done[slot], w.cs));
  SRV_TRY(hipEventSynchronize(w.ev_split[slot]));
#undef SRV_TRY
  return MBW_OK;
}

// Complete requests with an error (rc != 0) or with their slices of a downloaded batch (after its
// download has finished).
static void complete(Worker &w, InFlight &f, int rc) {
  mbw_server *s = w.s;
  if (!rc && hipEventSynchronize(w.ev_done[f.slot]) != hipSuccess) {
    mbw_set_error(std::string("hipEventSynchronize: ") + hipGetErrorString(hipGetLastError()));
    rc = MBW_E_HIP;
  }
  const double tb2 = s->now();
  if (!rc) {
    const SplitBound *b = (const SplitBound *)w.hbnd[f.slot].p;
    for (size_t i = 0; i < f.reqs.size(); ++i) {
      Request *r = f.reqs[i];
      r->buf = f.bb; r->s0 = b[i].t0; r->ns = b[i + 1].t0 - b[i].t0; r->p0 = b[i].p0; r->np = b[i + 1].p0 - b[i].p0;
      r->c0 = b[i].c0; r->nc = b[i + 1].c0 - b[i].c0;
    }
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    const double t = s->now();
    if (f.bb) {
      f.bb->refs = rc ? 0 : (int)f.reqs.size();
      if (rc || f.reqs.empty()) pool_put(s, f.bb);
    }
    const std::string msg = rc ? std::string(mbw_last_error()) : std::string();
    for (Request *r : f.reqs) {
      r->rc = rc; r->state = 2; r->t_done = t;
      if (rc) { r->buf = nullptr; r->err = msg; s->st.failed_requests++; }
    }
    if (s->trace)
      fprintf(stderr, "[serve] batch %llu reads %llu requests %zu: seed %.2f ms (device %.2f), download %.2f ms%s\n",
              (unsigned long long)f.bid, (unsigned long long)f.nreads, f.reqs.size(), (f.tb1 - f.tb0) * 1e3,
              f.ms_device, (tb2 - f.tb1) * 1e3, rc ? " FAILED" : "");
  }
  s->done_cv.notify_all();
}

// the finisher: completes downloaded batches in order and frees their result slots
static void finisher_main(Worker *wp) {
  Worker &w = *wp;
  (void)hipSetDevice(w.s->cfg.device);
  for (;;) {
    InFlight f;
    {
      std::unique_lock<std::mutex> lk(w.fmu);
      w.fcv.wait(lk, [&] { return w.fstop || !w.fq.empty(); });
      if (w.fq.empty()) return;
      f = std::move(w.fq.front());
      w.fq.pop_front();
    }
    complete(w, f, MBW_OK);
    {
      std::lock_guard<std::mutex> lk(w.fmu);
      w.busy[f.slot] = false;
    }
    w.fcv.notify_all();
  }
}

// wait until result slot `slot` is free, and claim it
static void claim_slot(Worker &w, int slot) {
  std::unique_lock<std::mutex> lk(w.fmu);
  w.fcv.wait(lk, [&] { return !w.busy[slot]; });
  w.busy[slot] = true;
}

static void release_slot(Worker &w, int slot) {
  {
    std::lock_guard<std::mutex> lk(w.fmu);
    w.busy[slot] = false;
  }
  w.fcv.notify_all();
}

static void hand_to_finisher(Worker &w, InFlight &&f) {
  {
    std::lock_guard<std::mutex> lk(w.fmu);
    w.fq.push_back(std::move(f));
  }
  w.fcv.notify_all();
}

// Run requests [i0, i1) of a staged batch; a shortfall of the arena (MBW_E_CAPACITY) or an
// allocation failure splits them in two halves, each run again.  `slot` alternates between the two
// result slots over the runs of one worker.
static void run_split(Worker &w, int k, int &slot, const std::vector<Request *> &batch, size_t i0, size_t i1,
                      uint64_t rb0, uint64_t rr0) {
  InFlight f;
  claim_slot(w, slot);
  int rc = run_batch(w, k, slot, batch, i0, i1, rb0, rr0, f);
  if (!rc) {
    hand_to_finisher(w, std::move(f));
    slot ^= 1;
    return;
  }
  // a failure after the downloads were queued must not hand the buffer or the slot on while a
  // copy may still write them
  (void)hipStreamSynchronize(w.cs);
  (void)hipStreamSynchronize(w.st);
  release_slot(w, slot);
  if (f.bb) { std::lock_guard<std::mutex> lk(w.s->mu); pool_put(w.s, f.bb); f.bb = nullptr; }
  if ((rc == MBW_E_CAPACITY || rc == MBW_E_NOMEM) && i1 - i0 > 1) {
    {
      std::lock_guard<std::mutex> lk(w.s->mu);
      w.s->st.split_retries++;
    }
    const size_t mid = i0 + (i1 - i0) / 2;
    uint64_t rb = rb0, rr = rr0;
    for (size_t i = i0; i < mid; ++i) { rb += batch[i]->bases; rr += batch[i]->n_reads; }
    run_split(w, k, slot, batch, i0, mid, rb0, rr0);
    run_split(w, k, slot, batch, mid, i1, rb, rr);
    return;
  }
  complete(w, f, rc);
}

static void worker_main(Worker *wp) {
  Worker &w = *wp;
  mbw_server *s = w.s;
  (void)hipSetDevice(s->cfg.device);
  int k = 0, slot = 0;
  for (;;) {
    std::vector<Request *> batch;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->work_cv.wait(lk, [&] { return s->stop || !s->queue.empty(); });
      batch = take_batch(s);
    }
    if (batch.empty()) break;   // stopping with an empty queue
    const int rc = stage_batch(w, k, batch);
    if (rc) {
      InFlight f;
      f.reqs = batch;
      complete(w, f, rc);
      continue;
    }
    run_split(w, k, slot, batch, 0, batch.size(), 0, 0);
    k ^= 1;
  }
  {   // let the finisher drain and stop
    std::lock_guard<std::mutex> lk(w.fmu);
    w.fstop = true;
  }
  w.fcv.notify_all();
  w.finisher.join();
}

}  // namespace

extern "C" int mbw_serve_open(const mbw_index *ix, const mbw_serve_cfg *cfg, mbw_server **out) {
  if (!ix || !cfg || !out) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  *out = nullptr;
  if (cfg->n_workers < 1 || cfg->n_workers > 8 || cfg->max_batch_reads < 1 || cfg->max_batch_bases < 1 ||
      cfg->min_seed_len < 1 || cfg->max_occ < 1 || cfg->max_batch_reads >= (1ull << 31)) {
    mbw_set_error("bad serve configuration"); return MBW_E_INVAL;
  }
  if (cfg->device != ix->device) { mbw_set_error("serve device differs from the index device"); return MBW_E_INVAL; }
  if (cfg->opts.bs_role && !ix->bisulfite) { mbw_set_error("bs_role needs a bisulfite index"); return MBW_E_INVAL; }
  if (hipSetDevice(cfg->device) != hipSuccess) { mbw_set_error("hipSetDevice failed"); return MBW_E_HIP; }
  mbw_server *s = new mbw_server();
  s->ix = ix;
  mbw_index_retain(ix);   // released by mbw_serve_close (or below when the open fails)
  s->cfg = *cfg;
  s->t0 = std::chrono::steady_clock::now();
  s->trace = getenv("MBW_SERVE_TRACE") && getenv("MBW_SERVE_TRACE")[0] == '1';
  std::vector<Worker *> ws;
  auto destroy = [](Worker *w) {
    if (w->a.base) (void)hipFree(w->a.base);
    for (int k = 0; k < 2; ++k) {
      if (w->ev_split[k]) (void)hipEventDestroy(w->ev_split[k]);
      if (w->ev_done[k]) (void)hipEventDestroy(w->ev_done[k]);
    }
    if (w->st) (void)hipStreamDestroy(w->st);
    if (w->cs) (void)hipStreamDestroy(w->cs);
  };
  auto fail = [&](int r) {
    for (Worker *w : ws) {
      destroy(w);
      if (w->ctx) mbw_ctx_free(w->ctx);
      delete w;
    }
    mbw_index_release(ix);
    delete s;
    return r;
  };
  const uint64_t per_worker = cfg->device_bytes / (uint64_t)cfg->n_workers;
  if (cfg->device_bytes && per_worker == 0) { mbw_set_error("serve device_bytes too small"); return fail(MBW_E_INVAL); }
  for (int i = 0; i < cfg->n_workers; ++i) {
    Worker *w = new Worker();
    ws.push_back(w);
    w->s = s;
    int r = mbw_ctx_create(ix, &w->ctx);
    if (r) return fail(r);
    // non-blocking: the workers' streams never wait for work on the null stream
    bool ok = hipStreamCreateWithFlags(&w->st, hipStreamNonBlocking) == hipSuccess &&
              hipStreamCreateWithFlags(&w->cs, hipStreamNonBlocking) == hipSuccess;
    for (int k = 0; k < 2 && ok; ++k)
      ok = hipEventCreateWithFlags(&w->ev_split[k], hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&w->ev_done[k], hipEventDisableTiming) == hipSuccess;
    if (!ok) { mbw_set_error("hipStreamCreate / hipEventCreate failed"); return fail(MBW_E_HIP); }
    if (i == 0) s->model_ctx = w->ctx;
    r = plan_arena(w->ctx, *cfg, per_worker, w->a);
    if (!r) r = alloc_arena(w->a);
    if (r) return fail(r);
    s->ws_bytes = w->a.ws_bytes;
    s->seeds_cap = w->a.seeds_cap;
    s->pos_cap = w->a.pos_cap;
    s->pieces_cap = w->a.pieces_cap;
    // pinned staging and split arrays sized for a full batch up front (pinning while serving stalls)
    const uint64_t br = std::min<uint64_t>(cfg->max_batch_reads, 1ull << 22);
    const uint64_t bb = std::min<uint64_t>(cfg->max_batch_bases, br * 160);
    for (int k = 0; k < 2; ++k)
      if (w->stage[k].ensure(bb / 2 + 16) || w->lens[k].ensure(br * sizeof(uint32_t) / 2 + 16)) {
        mbw_set_error("pinned staging allocation failed"); return fail(MBW_E_NOMEM);
      }
    if (w->hreq.ensure((kMaxBatchRequests + 1) * sizeof(uint32_t), true) ||
        w->hbnd[0].ensure((kMaxBatchRequests + 1) * sizeof(SplitBound), true) ||
        w->hbnd[1].ensure((kMaxBatchRequests + 1) * sizeof(SplitBound), true)) {
      mbw_set_error("pinned staging allocation failed"); return fail(MBW_E_NOMEM);
    }
  }
  s->st.device_bytes = 0;
  for (Worker *w : ws) s->st.device_bytes += w->a.bytes;
  s->st.workspace_bytes = s->ws_bytes;
  s->st.seeds_cap = ws[0]->a.seeds_cap;
  s->st.pos_cap = ws[0]->a.pos_cap;
  s->st.pieces_cap = ws[0]->a.pieces_cap;
  size_t started = 0;
  try {
    for (; started < ws.size(); ++started) {
      Worker *w = ws[started];
      w->finisher = std::thread(finisher_main, w);
      try {
        s->workers.emplace_back([w, destroy] {
          worker_main(w);   // returns once its finisher has completed every batch
          (void)hipSetDevice(w->s->cfg.device);
          (void)hipStreamSynchronize(w->st);
          (void)hipStreamSynchronize(w->cs);
          destroy(w);
          if (w->ctx != w->s->model_ctx) mbw_ctx_free(w->ctx);
          else w->ctx = nullptr;   // freed by mbw_serve_close after every worker has ended
          delete w;
        });
      } catch (...) {   // no worker thread: stop this worker's finisher
        {
          std::lock_guard<std::mutex> lk(w->fmu);
          w->fstop = true;
        }
        w->fcv.notify_all();
        w->finisher.join();
        throw;
      }
    }
  } catch (...) {   // out of threads: stop what started (its workers free themselves), free the rest
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
    }
    s->work_cv.notify_all();
    for (auto &t : s->workers) t.join();
    for (size_t i = s->workers.size(); i < ws.size(); ++i) {
      destroy(ws[i]);
      if (ws[i]->ctx && ws[i]->ctx != s->model_ctx) mbw_ctx_free(ws[i]->ctx);
      delete ws[i];
    }
    if (s->model_ctx) mbw_ctx_free(s->model_ctx);
    mbw_index_release(ix);
    delete s;
    mbw_set_error("cannot start serve threads");
    return MBW_E_NOMEM;
  }
  *out = s;
  return MBW_OK;
}

static int submit_impl(mbw_server *s, const uint8_t *reads, const uint32_t *lengths, uint64_t n_reads, bool copy,
                       uint64_t *ticket) {
  if (!s || !ticket || (n_reads && (!reads || !lengths))) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  if (n_reads >= (1ull << 31)) { mbw_set_error("too many reads in one request"); return MBW_E_INVAL; }
  uint64_t bases = 0;
  for (uint64_t i = 0; i < n_reads; ++i) {
    if (lengths[i] > MBW_MAX_READ) { mbw_set_error("read longer than 65535 bases"); return MBW_E_INVAL; }
    bases += lengths[i];
  }
  // admission by device memory: the request alone must fit a worker's arena
  uint64_t need = 0;
  const bool fit = s->fits(n_reads, bases, &need);
  if (n_reads > s->cfg.max_batch_reads || bases > s->cfg.max_batch_bases || !fit) {
    mbw_set_error("request too large for the server: " + std::to_string(n_reads) + " reads, " + std::to_string(bases) +
                  " bases, an estimated " + std::to_string(need) + " bytes of device work space; a worker has " +
                  std::to_string(s->ws_bytes) + " bytes, " + std::to_string(s->cfg.max_batch_reads) + " reads and " +
                  std::to_string(s->cfg.max_batch_bases) + " bases per batch");
    return MBW_E_CAPACITY;
  }
  Request *r = new (std::nothrow) Request();
  if (!r) { mbw_set_error("host allocation failed"); return MBW_E_NOMEM; }
  if (copy) {
    try {
      r->reads_copy.assign(reads, reads + bases);
      r->lengths_copy.assign(lengths, lengths + n_reads);
    } catch (...) { delete r; mbw_set_error("host allocation failed"); return MBW_E_NOMEM; }
    r->reads = r->reads_copy.data();
    r->lengths = r->lengths_copy.data();
  } else {
    r->reads = reads;
    r->lengths = lengths;
  }
  r->n_reads = n_reads;
  r->bases = bases;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) { delete r; mbw_set_error("server is closing"); return MBW_E_INVAL; }
    if (!s->queue.empty() && s->queued_bases + bases > s->cfg.max_queued_bases) {
      delete r;
      mbw_set_error("queue full (bases waiting for a worker)");
      return MBW_E_BUSY;
    }
    r->ticket = s->next_ticket++;
    r->t_submit = s->now();
    s->queue.push_back(r);
    s->queued_bases += bases;
    s->all[r->ticket] = r;
    *ticket = r->ticket;
  }
  s->work_cv.notify_one();
  return MBW_OK;
}

extern "C" int mbw_serve_submit(mbw_server *s, const uint8_t *reads, const uint32_t *lengths, uint64_t n_reads,
                                uint64_t *ticket) {
  return submit_impl(s, reads, lengths, n_reads, true, ticket);
}

extern "C" int mbw_serve_submit_nocopy(mbw_server *s, const uint8_t *reads, const uint32_t *lengths, uint64_t n_reads,
                                       uint64_t *ticket) {
  return submit_impl(s, reads, lengths, n_reads, false, ticket);
}

extern "C" int mbw_serve_wait(mbw_server *s, uint64_t ticket, int timeout_ms, mbw_serve_result *out) {
  if (!s || !out) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) { mbw_set_error("unknown ticket"); return MBW_E_INVAL; }
  Request *r = it->second;
  auto ready = [&] { return r->state == 2; };
  if (timeout_ms < 0) s->done_cv.wait(lk, ready);
  else if (!s->done_cv.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) {
    mbw_set_error("request not finished"); return MBW_E_BUSY;
  }
  memset(out, 0, sizeof(*out));
  out->t_submit = r->t_submit;
  out->t_start = r->t_start;
  out->t_done = r->t_done;
  out->batch_id = r->batch_id;
  out->batch_reads = r->batch_reads;
  out->attempts = r->attempts;
  if (r->rc) { mbw_set_error(r->err); return r->rc; }
  out->n_seeds = r->ns;
  out->n_pos = r->np;
  out->seeds = r->buf ? (const mbw_seed_t *)r->buf->seeds.p + r->s0 : nullptr;
  out->pos = r->buf ? (const uint64_t *)r->buf->pos.p + r->p0 : nullptr;
  out->n_pieces = r->nc;
  out->pieces = r->buf && r->nc ? (const mbw_piece_t *)r->buf->pieces.p + r->c0 : nullptr;
  return MBW_OK;
}

extern "C" int mbw_serve_release(mbw_server *s, uint64_t ticket) {
  if (!s) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) { mbw_set_error("unknown ticket"); return MBW_E_INVAL; }
  if (it->second->state != 2) { mbw_set_error("request not finished"); return MBW_E_BUSY; }
  s->unref(it->second->buf);
  delete it->second;
  s->all.erase(it);
  return MBW_OK;
}

extern "C" int mbw_serve_stats(mbw_server *s, mbw_serve_stats_t *out) {
  if (!s || !out) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  out->queued = s->queue.size();
  return MBW_OK;
}

extern "C" void mbw_serve_close(mbw_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->work_cv.notify_all();
  for (auto &t : s->workers) t.join();   // queued requests are finished first
  if (s->model_ctx) mbw_ctx_free(s->model_ctx);
  for (auto &kv : s->all) { s->unref(kv.second->buf); delete kv.second; }
  for (BatchBuf *b : s->free_bufs) delete b;
  const mbw_index *ix = s->ix;
  delete s;
  mbw_index_release(ix);
}
