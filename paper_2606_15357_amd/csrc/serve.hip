// Serving runtime: a request loop around mbw_seed with the index resident in HBM.
//
// Requests (a few to tens of thousands of reads) are queued on submission; admission is bounded by
// the bases waiting in the queue.  Each worker thread owns a seeding context and its own HIP stream.
// A free worker forms a batch from the head of the queue (up to a read / base budget), so requests
// that arrive while other batches are on the device join the next batch at once (continuous
// batching), and batches of different workers run on the device at the same time.  A batch's
// seeds come back sorted by read, so each request's seeds and positions are a contiguous slice;
// read ids and position offsets are made relative to each request on the device, and the batch is
// downloaded once into a pinned buffer its requests share.
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

#include "mbw_internal.h"
#include "../../include/mbw.h"

namespace {

// grow-only pinned host buffer
struct Pinned {
  void *p = nullptr;
  size_t bytes = 0;
  int ensure(size_t want) {
    if (want <= bytes) return 0;
    if (p) { (void)hipHostFree(p); p = nullptr; bytes = 0; }
    const size_t b = 2 * want + 4096;
    if (hipHostMalloc(&p, b, hipHostMallocDefault) != hipSuccess) { p = nullptr; return MBW_E_NOMEM; }
    bytes = b;
    return 0;
  }
  ~Pinned() { if (p) (void)hipHostFree(p); }
};

// grow-only device buffer (per worker)
struct DevScratch {
  void *p = nullptr;
  size_t bytes = 0;
  int ensure(size_t want) {
    if (want <= bytes) return 0;
    if (p) { (void)hipFree(p); p = nullptr; bytes = 0; }
    const size_t b = 2 * want + 256;
    if (hipMalloc(&p, b) != hipSuccess) { p = nullptr; return MBW_E_NOMEM; }
    bytes = b;
    return 0;
  }
  ~DevScratch() { if (p) (void)hipFree(p); }
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
};

struct Request {
  uint64_t ticket = 0;
  std::vector<uint8_t> reads;
  std::vector<uint32_t> lengths;
  uint64_t bases = 0;
  double t_submit = 0, t_start = 0, t_done = 0;
  uint64_t batch_id = 0, batch_reads = 0;
  int state = 0;   // 0 queued, 1 running, 2 done
  int rc = MBW_OK;
  BatchBuf *buf = nullptr;          // the shared batch result
  uint64_t s0 = 0, ns = 0, p0 = 0, np = 0;   // this request's slice of it (seeds, positions,
  uint64_t c0 = 0, nc = 0;                    // refined pieces)
};

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
  uint64_t batches = 0, batch_reads_sum = 0;
  bool trace = false;   // MBW_SERVE_TRACE=1: one line per batch on stderr
  std::vector<BatchBuf *> free_bufs;

  void unref(BatchBuf *b) {   // with mu held
    if (b && --b->refs == 0) free_bufs.push_back(b);
  }

  double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

static void worker_main(mbw_server *s, mbw_ctx *ctx, hipStream_t st) {
  Pinned hreads, hlens, hreq, hbnd;
  DevScratch dreq, dbnd;
  (void)hipSetDevice(s->cfg.device);
  // pinned staging sized for a full batch up front (pinning memory while serving would stall)
  const uint64_t br = std::min<uint64_t>(s->cfg.max_batch_reads, 1ull << 22);
  (void)hreads.ensure(std::min<uint64_t>(s->cfg.max_batch_bases, br * 160) / 2 + 16);
  (void)hlens.ensure(br * sizeof(uint32_t) / 2 + 16);
  for (;;) {
    std::vector<Request *> batch;
    uint64_t nreads = 0, nbases = 0, bid = 0;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->work_cv.wait(lk, [&] { return s->stop || !s->queue.empty(); });
      if (s->queue.empty()) return;   // stopping
      while (!s->queue.empty()) {
        Request *r = s->queue.front();
        const uint64_t nr = r->lengths.size();
        if (!batch.empty() && (nreads + nr > s->cfg.max_batch_reads || nbases + r->bases > s->cfg.max_batch_bases)) break;
        s->queue.pop_front();
        s->queued_bases -= r->bases;
        batch.push_back(r);
        nreads += nr;
        nbases += r->bases;
      }
      bid = s->next_batch++;
      const double t = s->now();
      for (Request *r : batch) { r->state = 1; r->t_start = t; r->batch_id = bid; r->batch_reads = nreads; }
      s->batches++;
      s->batch_reads_sum += nreads;
    }
    // concatenate the batch in pinned memory and seed it
    const double tb0 = s->now();
    double tb1 = tb0, tb2 = tb0, tb3 = tb0;
    int rc = hreads.ensure(nbases + 16);
    if (!rc) rc = hlens.ensure((nreads + 1) * sizeof(uint32_t));
    mbw_result res;
    memset(&res, 0, sizeof(res));
    if (!rc) {
      uint8_t *rb = (uint8_t *)hreads.p;
      uint32_t *lb = (uint32_t *)hlens.p;
      uint64_t ob = 0, orr = 0;
      for (Request *r : batch) {
        if (!r->reads.empty()) memcpy(rb + ob, r->reads.data(), r->reads.size());
        if (!r->lengths.empty()) memcpy(lb + orr, r->lengths.data(), r->lengths.size() * sizeof(uint32_t));
        ob += r->reads.size();
        orr += r->lengths.size();
      }
      tb1 = s->now();
      rc = mbw_seed(ctx, rb, lb, nreads, s->cfg.min_seed_len, s->cfg.max_occ, &s->cfg.opts, (void *)st, &res);
      tb2 = s->now();
    }
    BatchBuf *bb = nullptr;
    if (!rc) {
      std::lock_guard<std::mutex> lk(s->mu);
      if (!s->free_bufs.empty()) { bb = s->free_bufs.back(); s->free_bufs.pop_back(); }
    }
    if (!rc && !bb) {
      bb = new BatchBuf();
      rc = bb->seeds.ensure(br * 4 * sizeof(mbw_seed_t));
      if (!rc) rc = bb->pos.ensure(br * 24 * sizeof(uint64_t));
    }
    // split into requests on the device (read ids, position offsets and piece seed indexes made
    // relative to each request), then one download of the batch and of the request bounds
    const uint32_t nreq = (uint32_t)batch.size();
    if (!rc) rc = hreq.ensure((nreq + 1) * sizeof(uint32_t));
    if (!rc) rc = hbnd.ensure((nreq + 1) * sizeof(SplitBound));
    if (!rc) rc = dreq.ensure((nreq + 1) * sizeof(uint32_t));
    if (!rc) rc = dbnd.ensure((nreq + 1) * sizeof(SplitBound));
    if (!rc) {
      uint32_t *rs = (uint32_t *)hreq.p;
      uint64_t r0 = 0;
      for (uint32_t i = 0; i < nreq; ++i) { rs[i] = (uint32_t)r0; r0 += batch[i]->lengths.size(); }
      rs[nreq] = (uint32_t)r0;
      const unsigned gb = (unsigned)std::min<uint64_t>((nreq + 256) / 256, 1024);
      const unsigned gr = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((res.n_seeds + res.n_pieces + 255) / 256, 4096));
      if (hipMemcpyAsync(dreq.p, rs, (nreq + 1) * sizeof(uint32_t), hipMemcpyHostToDevice, st) != hipSuccess) rc = MBW_E_HIP;
      if (!rc) {
        k_split_bounds<<<gb, 256, 0, st>>>(res.seeds, res.n_seeds, res.n_pos, res.pieces, res.n_pieces,
                                           (const uint32_t *)dreq.p, nreq, (SplitBound *)dbnd.p);
        if (res.n_seeds + res.n_pieces)
          k_split_rebase<<<gr, 256, 0, st>>>((mbw_seed_t *)res.seeds, res.n_seeds, (mbw_piece_t *)res.pieces, res.n_pieces,
                                             (const uint32_t *)dreq.p, nreq, (const SplitBound *)dbnd.p);
        if (hipGetLastError() != hipSuccess) rc = MBW_E_HIP;
      }
      if (!rc && hipMemcpyAsync(hbnd.p, dbnd.p, (nreq + 1) * sizeof(SplitBound), hipMemcpyDeviceToHost, st) != hipSuccess)
        rc = MBW_E_HIP;
    }
    if (!rc) rc = bb->seeds.ensure((res.n_seeds + 1) * sizeof(mbw_seed_t));
    if (!rc) rc = bb->pos.ensure((res.n_pos + 1) * sizeof(uint64_t));
    if (!rc) rc = mbw_result_download(ctx, &res, (mbw_seed_t *)bb->seeds.p, (uint64_t *)bb->pos.p);
    if (!rc && res.n_pieces) {
      rc = bb->pieces.ensure((res.n_pieces + 1) * sizeof(mbw_piece_t));
      if (!rc) rc = mbw_result_download_pieces(ctx, &res, (mbw_piece_t *)bb->pieces.p);
    }
    tb3 = s->now();
    if (!rc) {
      const SplitBound *b = (const SplitBound *)hbnd.p;
      for (uint32_t i = 0; i < nreq; ++i) {
        Request *r = batch[i];
        r->buf = bb; r->s0 = b[i].t0; r->ns = b[i + 1].t0 - b[i].t0; r->p0 = b[i].p0; r->np = b[i + 1].p0 - b[i].p0;
        r->c0 = b[i].c0; r->nc = b[i + 1].c0 - b[i].c0;
      }
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      const double t = s->now();
      if (bb) {
        bb->refs = rc ? 0 : (int)batch.size();
        if (rc) s->free_bufs.push_back(bb);
      }
      for (Request *r : batch) { r->rc = rc; r->state = 2; r->t_done = t; if (rc) r->buf = nullptr; }
      if (s->trace)
        fprintf(stderr, "[serve] batch %llu reads %llu: copy %.2f ms, seed %.2f ms (device %.2f), download %.2f ms, split %.2f ms\n",
                (unsigned long long)bid, (unsigned long long)nreads, (tb1 - tb0) * 1e3, (tb2 - tb1) * 1e3, res.ms_total,
                (tb3 - tb2) * 1e3, (t - tb3) * 1e3);
    }
    s->done_cv.notify_all();
  }
}

extern "C" int mbw_serve_open(const mbw_index *ix, const mbw_serve_cfg *cfg, mbw_server **out) {
  if (!ix || !cfg || !out) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  *out = nullptr;
  if (cfg->n_workers < 1 || cfg->n_workers > 8 || cfg->max_batch_reads < 1 || cfg->max_batch_bases < 1 ||
      cfg->min_seed_len < 1 || cfg->max_occ < 1) {
    mbw_set_error("bad serve configuration"); return MBW_E_INVAL;
  }
  if (cfg->device != ix->device) { mbw_set_error("serve device differs from the index device"); return MBW_E_INVAL; }
  mbw_server *s = new mbw_server();
  s->ix = ix;
  s->cfg = *cfg;
  s->t0 = std::chrono::steady_clock::now();
  s->trace = getenv("MBW_SERVE_TRACE") && getenv("MBW_SERVE_TRACE")[0] == '1';
  std::vector<std::pair<mbw_ctx *, hipStream_t>> res;
  for (int w = 0; w < cfg->n_workers; ++w) {
    mbw_ctx *c = nullptr;
    int r = mbw_ctx_create(ix, &c);
    hipStream_t st = nullptr;
    // non-blocking: the workers' streams never wait for work on the null stream
    if (!r && hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      mbw_ctx_free(c); mbw_set_error("hipStreamCreate failed"); r = MBW_E_HIP;
    }
    if (r) {
      for (auto &x : res) { mbw_ctx_free(x.first); (void)hipStreamDestroy(x.second); }
      delete s;
      return r;
    }
    res.emplace_back(c, st);
  }
  for (auto &x : res)
    s->workers.emplace_back([s, x] {
      worker_main(s, x.first, x.second);
      mbw_ctx_free(x.first);
      (void)hipStreamDestroy(x.second);
    });
  *out = s;
  return MBW_OK;
}

extern "C" int mbw_serve_submit(mbw_server *s, const uint8_t *reads, const uint32_t *lengths, uint64_t n_reads,
                                uint64_t *ticket) {
  if (!s || !ticket || (n_reads && (!reads || !lengths))) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  uint64_t bases = 0;
  for (uint64_t i = 0; i < n_reads; ++i) {
    if (lengths[i] > MBW_MAX_READ) { mbw_set_error("read longer than 65535 bases"); return MBW_E_INVAL; }
    bases += lengths[i];
  }
  Request *r = new Request();
  try {
    r->reads.assign(reads, reads + bases);
    r->lengths.assign(lengths, lengths + n_reads);
  } catch (...) { delete r; mbw_set_error("host allocation failed"); return MBW_E_NOMEM; }
  r->bases = bases;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) { delete r; mbw_set_error("server is closing"); return MBW_E_INVAL; }
    if (!s->queue.empty() && s->queued_bases + bases > s->cfg.max_queued_bases) {
      delete r;
      mbw_set_error("queue full (admission by queued bases)");
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
  if (r->rc) return r->rc;
  out->n_seeds = r->ns;
  out->n_pos = r->np;
  out->seeds = r->buf ? (const mbw_seed_t *)r->buf->seeds.p + r->s0 : nullptr;
  out->pos = r->buf ? (const uint64_t *)r->buf->pos.p + r->p0 : nullptr;
  out->t_submit = r->t_submit;
  out->t_start = r->t_start;
  out->t_done = r->t_done;
  out->batch_id = r->batch_id;
  out->batch_reads = r->batch_reads;
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

extern "C" int mbw_serve_stats(mbw_server *s, uint64_t *batches, uint64_t *batch_reads, uint64_t *queued) {
  if (!s) { mbw_set_error("NULL argument"); return MBW_E_INVAL; }
  std::lock_guard<std::mutex> lk(s->mu);
  if (batches) *batches = s->batches;
  if (batch_reads) *batch_reads = s->batch_reads_sum;
  if (queued) *queued = s->queue.size();
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
  for (auto &kv : s->all) { s->unref(kv.second->buf); delete kv.second; }
  for (BatchBuf *b : s->free_bufs) delete b;
  delete s;
}
