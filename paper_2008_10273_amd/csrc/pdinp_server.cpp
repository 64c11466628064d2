// Serving loop (pdi_server_*): frames from many client streams, of any
// resolution, are admitted as lanes and device memory free up, copied to the
// device, decoded on one of several HIP streams (their kernels overlap on the
// GPU) and completed asynchronously.  Continuous batching: a request that
// arrives while others run is admitted as soon as a lane and enough of the
// HBM budget are free, without waiting for the running ones to finish.
//
// Queued frames of one geometry and parameters are admitted together, up to
// PDI_MAX_BATCH at a time, and decoded by one decode_residual_batch launch
// (only frames already waiting join: a light load admits frames one by one,
// a deep queue drains in large launches);
// a frame's result does not depend on what it is batched with or on what
// else is in flight, so it is the same alone and in the mix.
#include "../../include/pdinp.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

namespace {

using Clock = std::chrono::steady_clock;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Buffer sizes are rounded up to 64 KiB so that frames of one resolution
// with different point counts reuse the same buffers.
size_t bucket(size_t x) { return (x + 65535) & ~(size_t)65535; }

struct Request {
  int64_t ticket = 0;
  pdi_frame frame{};
  int block_size = 16;
  pdi_params params{};
  int32_t chroma_shared = 0;
  int32_t n_mask_blocks = 0;
  int64_t out_elems = 0;
  size_t out_elem = 4;  // bytes per output pixel (4, or 1 with out_int8)
  // block_ptr at 0, pos at off_pos, values at off_val of the input buffer
  size_t off_pos = 0, off_val = 0, in_used = 0, in_bytes = 0, out_bytes = 0;
  void *h_in = nullptr;       // pinned staging of the input buffer
  void *h_out = nullptr;      // pinned staging of the result
  void *user_out = nullptr;   // host destination (may be null), written by pdi_wait
  void *user_dev = nullptr;   // caller-owned device destination (may be null)
  void *d_in = nullptr;
  void *d_out = nullptr;      // user_dev or a pooled buffer of out_bytes
  int lane = -1;
  Clock::time_point t_submit;
  double latency_us = 0.0;
  int status = PDI_OK;
  bool finished = false;
};

// Frames admitted together: one batched decode on one lane.
struct Group {
  std::vector<Request *> reqs;
  int lane = -1;
  hipEvent_t ev = nullptr;
};

}  // namespace

struct pdi_server {
  pdi_ctx *ctx = nullptr;
  int device = 0;
  size_t budget = 0;     // cap on the device bytes of running requests, 0 = none
  size_t in_use = 0;     // device bytes of running requests
  size_t allocated = 0;  // device bytes held (running requests + pool)
  int max_queue = 0;
  int max_batch = PDI_MAX_BATCH;  // frames joined per launch
  std::vector<hipStream_t> lanes;
  std::vector<int> lane_busy;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request *> queue;     // waiting for admission, arrival order
  std::vector<Group *> running;    // admitted, on the GPU
  std::vector<hipEvent_t> ev_pool; // completion events not in use
  std::map<int64_t, Request *> all;
  std::map<size_t, std::vector<void *>> pool;   // free device buffers by size
  std::map<size_t, std::vector<void *>> hpool;  // free pinned host buffers by size
  int64_t next_ticket = 1;
  bool hold = false;  // admission paused
  bool stop = false;
  std::thread worker;
};

namespace {

size_t dev_bytes(const Request *r) { return r->in_bytes + r->out_bytes; }

void pool_release_all(pdi_server *S) {
  for (auto &kv : S->pool)
    for (void *p : kv.second) {
      (void)hipFree(p);
      S->allocated -= kv.first;
    }
  S->pool.clear();
}

// Device buffer of a bucket size.  Admission keeps the bytes of running
// requests within the budget, so dropping the cached buffers always makes
// room for a new one.
void *pool_get(pdi_server *S, size_t bytes) {
  auto it = S->pool.find(bytes);
  if (it != S->pool.end() && !it->second.empty()) {
    void *p = it->second.back();
    it->second.pop_back();
    return p;
  }
  if (S->budget && S->allocated + bytes > S->budget) pool_release_all(S);
  void *p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  S->allocated += bytes;
  return p;
}

void *hpool_get(pdi_server *S, size_t bytes) {
  auto it = S->hpool.find(bytes);
  if (it != S->hpool.end() && !it->second.empty()) {
    void *p = it->second.back();
    it->second.pop_back();
    return p;
  }
  void *p = nullptr;
  if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
  return p;
}

size_t out_floats_bytes(const Request *r) { return bucket(r->out_elem * (size_t)r->out_elems); }

void release_host(pdi_server *S, Request *r) {
  if (r->h_in) S->hpool[r->in_bytes].push_back(r->h_in);
  if (r->h_out) S->hpool[out_floats_bytes(r)].push_back(r->h_out);
  r->h_in = nullptr;
  r->h_out = nullptr;
}

// Can b join a batched decode with a (same geometry, block size and params)?
bool same_kind(const Request *a, const Request *b) {
  const pdi_params &p = a->params, &q = b->params;
  return a->frame.width == b->frame.width && a->frame.height == b->frame.height &&
         a->frame.format == b->frame.format && a->block_size == b->block_size &&
         a->chroma_shared == b->chroma_shared && p.op == q.op && p.s == q.s && p.eval_dtype == q.eval_dtype &&
         p.refine == q.refine && p.validate == q.validate && p.path == q.path && p.refine_tau == q.refine_tau &&
         p.out_int8 == q.out_int8;
}

// Start an admitted group on its lane (lock held): H2D copies, one batched
// decode, D2H copies and a completion event, all asynchronous on the lane's
// stream.
int launch_group(pdi_server *S, Group *g) {
  const int n = (int)g->reqs.size();
  hipStream_t st = S->lanes[g->lane];
  pdi_mask mk[PDI_MAX_BATCH];
  const float *vals[PDI_MAX_BATCH];
  float *outs[PDI_MAX_BATCH];
  for (int k = 0; k < n; ++k) {
    Request *r = g->reqs[k];
    r->d_in = pool_get(S, r->in_bytes);
    r->d_out = r->user_dev ? r->user_dev : pool_get(S, r->out_bytes);
    if (!r->d_in || !r->d_out) return PDI_ENOMEM;
    if (hipMemcpyAsync(r->d_in, r->h_in, r->in_used, hipMemcpyHostToDevice, st) != hipSuccess) return PDI_EHIP;
    char *base = (char *)r->d_in;
    mk[k].block_ptr = (const int32_t *)base;
    mk[k].pos = (const uint16_t *)(base + r->off_pos);
    mk[k].n_mask_blocks = r->n_mask_blocks;
    mk[k].chroma_shared = r->chroma_shared;
    vals[k] = (const float *)(base + r->off_val);
    outs[k] = (float *)r->d_out;
  }
  const Request *r0 = g->reqs[0];
  const int rc = decode_residual_batch(S->ctx, n, &r0->frame, mk, vals, r0->block_size, &r0->params, outs, st);
  if (rc != PDI_OK) return rc;
  for (Request *r : g->reqs)
    if (r->user_out && hipMemcpyAsync(r->h_out, r->d_out, r->out_elem * (size_t)r->out_elems,
                                      hipMemcpyDeviceToHost, st) != hipSuccess)
      return PDI_EHIP;
  if (S->ev_pool.empty()) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return PDI_EHIP;
    S->ev_pool.push_back(e);
  }
  g->ev = S->ev_pool.back();
  S->ev_pool.pop_back();
  return hipEventRecord(g->ev, st) == hipSuccess ? PDI_OK : PDI_EHIP;
}

// Complete a request (lock held): return its device buffers and its share of
// the budget.  A host result stays in its pinned staging
// buffer until pdi_wait copies it out.
void finish_request(pdi_server *S, Request *r, int status) {
  r->status = status;
  if (r->d_in) S->pool[r->in_bytes].push_back(r->d_in);
  if (r->d_out && !r->user_dev) S->pool[r->out_bytes].push_back(r->d_out);
  r->d_in = nullptr;
  r->d_out = nullptr;
  S->in_use -= dev_bytes(r);
  if (r->h_in) S->hpool[r->in_bytes].push_back(r->h_in);
  r->h_in = nullptr;
  r->latency_us = std::chrono::duration<double, std::micro>(Clock::now() - r->t_submit).count();
  r->finished = true;
}

void worker_loop(pdi_server *S) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  while (true) {
    bool progressed = false;
    for (size_t i = 0; i < S->running.size();) {
      Group *g = S->running[i];
      const hipError_t q = hipEventQuery(g->ev);
      if (q == hipErrorNotReady) {
        ++i;
        continue;
      }
      // The lane holds no later work, so this returns at once; the status
      // word covers the whole batch.
      const int st = q == hipSuccess ? pdi_sync(S->ctx, S->lanes[g->lane]) : PDI_EHIP;
      for (Request *r : g->reqs) finish_request(S, r, st);
      S->lane_busy[g->lane] = 0;
      S->ev_pool.push_back(g->ev);
      delete g;
      S->running.erase(S->running.begin() + (long)i);
      progressed = true;
    }
    // Admission in arrival order while a lane and the budget allow: the
    // oldest frame, joined by queued frames of the same kind.
    while (!S->queue.empty() && !S->hold) {
      Request *r = S->queue.front();
      int lane = -1;
      for (size_t l = 0; l < S->lanes.size(); ++l)
        if (!S->lane_busy[l]) {
          lane = (int)l;
          break;
        }
      if (lane < 0) break;
      if (S->budget && S->in_use + dev_bytes(r) > S->budget) break;
      Group *g = new Group();
      g->lane = lane;
      g->reqs.push_back(r);
      S->queue.pop_front();
      S->in_use += dev_bytes(r);
      for (size_t k = 0; k < S->queue.size() && (int)g->reqs.size() < S->max_batch;) {
        Request *c = S->queue[k];
        if (same_kind(r, c) && (!S->budget || S->in_use + dev_bytes(c) <= S->budget)) {
          g->reqs.push_back(c);
          S->in_use += dev_bytes(c);
          S->queue.erase(S->queue.begin() + (long)k);
        } else {
          ++k;
        }
      }
      for (Request *c : g->reqs) c->lane = lane;
      S->lane_busy[lane] = 1;
      const int rc = launch_group(S, g);
      if (rc != PDI_OK) {
        (void)hipStreamSynchronize(S->lanes[lane]);  // buffers go back to the pool
        for (Request *c : g->reqs) finish_request(S, c, rc);
        S->lane_busy[lane] = 0;
        if (g->ev) S->ev_pool.push_back(g->ev);
        delete g;
      } else {
        S->running.push_back(g);
      }
      progressed = true;
    }
    if (progressed) S->cv.notify_all();
    if (S->stop && S->queue.empty() && S->running.empty()) break;
    if (S->running.empty()) {
      S->cv.wait(lk, [&] { return S->stop || (!S->queue.empty() && !S->hold); });
    } else {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(10));
      lk.lock();
    }
  }
}

}  // namespace

extern "C" {

int pdi_server_create(pdi_ctx *ctx, int nlanes, size_t hbm_budget_bytes, int max_queue,
                      pdi_server **out) {
  if (!ctx || !out || nlanes <= 0 || nlanes > 32 || max_queue <= 0) return PDI_EINVAL;
  *out = nullptr;
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return PDI_EHIP;
  pdi_server *S = new pdi_server();
  S->ctx = ctx;
  S->device = device;
  S->budget = hbm_budget_bytes;
  S->max_queue = max_queue;
  for (int i = 0; i < nlanes; ++i) {
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t t : S->lanes) (void)hipStreamDestroy(t);
      delete S;
      return PDI_EHIP;
    }
    S->lanes.push_back(s);
    S->lane_busy.push_back(0);
  }
  S->worker = std::thread(worker_loop, S);
  *out = S;
  return PDI_OK;
}

int pdi_submit(pdi_server *S, const pdi_frame *frame, const pdi_mask *mask, const float *values,
               int64_t n_values, int block_size, const pdi_params *params, void *out, void *out_dev,
               int64_t *ticket) {
  if (!S || !frame || !mask || !mask->block_ptr || !values || !ticket || n_values < 0) return PDI_EINVAL;
  int32_t nb = 0;
  int64_t nel = 0;
  if (pdi_frame_info(frame, block_size, mask->chroma_shared, &nb, &nel) != PDI_OK || nb != mask->n_mask_blocks)
    return PDI_EINVAL;
  const int64_t nnz = mask->block_ptr[nb];
  if (nnz < 0 || (nnz > 0 && !mask->pos)) return PDI_EINVAL;
  // Values: one per position, plus a second chroma run for a shared mask.
  const int32_t ny = ((frame->width + block_size - 1) / block_size) * ((frame->height + block_size - 1) / block_size);
  const int64_t need = (frame->format == PDI_YUV420 && mask->chroma_shared) ? 2 * nnz - mask->block_ptr[ny] : nnz;
  if (n_values < need) return PDI_EINVAL;
  pdi_params P;
  pdi_default_params(&P);
  if (params) P = *params;
  // With validation on, positions and values are checked here, on the host,
  // before anything reaches the device.
  if (P.validate) {
    const int rc = pdi_validate_host(frame, block_size, mask->block_ptr, mask->pos, nb, mask->chroma_shared, values);
    if (rc != PDI_OK) return rc;
    P.validate = 0;
  }
  Request *r = new Request();
  r->frame = *frame;
  r->block_size = block_size;
  r->params = P;
  r->chroma_shared = mask->chroma_shared;
  r->n_mask_blocks = nb;
  r->out_elems = nel;
  r->out_elem = P.out_int8 ? 1 : 4;
  r->user_out = out;
  r->user_dev = out_dev;
  r->off_pos = align256(sizeof(int32_t) * (size_t)(nb + 1));
  r->off_val = r->off_pos + align256(sizeof(uint16_t) * (size_t)std::max<int64_t>(nnz, 1));
  r->in_used = r->off_val + sizeof(float) * (size_t)need;
  r->in_bytes = bucket(r->in_used);
  r->out_bytes = out_dev ? 0 : out_floats_bytes(r);
  if (S->budget && dev_bytes(r) > S->budget) {
    delete r;
    return PDI_ENOMEM;
  }
  std::unique_lock<std::mutex> lk(S->mu);
  if ((int)S->queue.size() >= S->max_queue) {
    delete r;
    return PDI_EBUSY;
  }
  r->h_in = hpool_get(S, r->in_bytes);
  if (out) r->h_out = hpool_get(S, out_floats_bytes(r));
  if (!r->h_in || (out && !r->h_out)) {
    release_host(S, r);
    delete r;
    return PDI_ENOMEM;
  }
  char *h = (char *)r->h_in;
  std::memcpy(h, mask->block_ptr, sizeof(int32_t) * (size_t)(nb + 1));
  if (nnz > 0) std::memcpy(h + r->off_pos, mask->pos, sizeof(uint16_t) * (size_t)nnz);
  if (need > 0) std::memcpy(h + r->off_val, values, sizeof(float) * (size_t)need);
  r->ticket = S->next_ticket++;
  r->t_submit = Clock::now();
  S->queue.push_back(r);
  S->all[r->ticket] = r;
  *ticket = r->ticket;
  lk.unlock();
  S->cv.notify_all();
  return PDI_OK;
}

int pdi_poll(pdi_server *S, int64_t ticket, int *done, double *latency_us) {
  if (!S || !done) return PDI_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return PDI_EINVAL;
  const Request *r = it->second;
  *done = r->finished ? 1 : 0;
  if (latency_us) *latency_us = r->finished ? r->latency_us : 0.0;
  return r->finished ? r->status : PDI_OK;
}

int pdi_wait(pdi_server *S, int64_t ticket, double *latency_us) {
  if (!S) return PDI_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return PDI_EINVAL;
  Request *r = it->second;
  S->cv.wait(lk, [&] { return r->finished; });
  if (latency_us) *latency_us = r->latency_us;
  const int st = r->status;
  S->all.erase(it);
  void *h_out = r->h_out;
  r->h_out = nullptr;
  lk.unlock();
  if (st == PDI_OK && r->user_out && h_out)
    std::memcpy(r->user_out, h_out, r->out_elem * (size_t)r->out_elems);
  lk.lock();
  if (h_out) S->hpool[out_floats_bytes(r)].push_back(h_out);
  lk.unlock();
  delete r;
  return st;
}

int pdi_server_stats(pdi_server *S, int64_t *queued, int64_t *running, size_t *bytes_in_use,
                     size_t *bytes_allocated) {
  if (!S) return PDI_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  if (queued) *queued = (int64_t)S->queue.size();
  if (running) {
    int64_t n = 0;
    for (const Group *g : S->running) n += (int64_t)g->reqs.size();
    *running = n;
  }
  if (bytes_in_use) *bytes_in_use = S->in_use;
  if (bytes_allocated) *bytes_allocated = S->allocated;
  return PDI_OK;
}

int pdi_server_hold(pdi_server *S, int hold) {
  if (!S) return PDI_EINVAL;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->hold = hold != 0;
  }
  S->cv.notify_all();
  return PDI_OK;
}

void pdi_server_destroy(pdi_server *S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    S->hold = false;
  }
  S->cv.notify_all();
  if (S->worker.joinable()) S->worker.join();  // drains queued and running work
  (void)hipSetDevice(S->device);
  for (auto &kv : S->all) {
    release_host(S, kv.second);
    delete kv.second;
  }
  pool_release_all(S);
  for (hipEvent_t e : S->ev_pool) (void)hipEventDestroy(e);
  for (auto &kv : S->hpool)
    for (void *p : kv.second) (void)hipHostFree(p);
  for (hipStream_t s : S->lanes) (void)hipStreamDestroy(s);
  delete S;
}

}  // extern "C"
