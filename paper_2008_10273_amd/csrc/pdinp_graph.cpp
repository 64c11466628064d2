// Graph-captured decode of a frame sequence (pdi_seq_*): the decodes of n
// frames of one geometry are recorded once into a HIP graph, as batched
// decodes of up to PDI_MAX_BATCH frames spread over several streams joined
// by events (independent batches overlap on the GPU), and the graph is then
// replayed with one launch.
#include "../../include/pdinp.h"

#include <hip/hip_runtime.h>

#include <vector>

struct pdi_seq {
  pdi_ctx *ctx = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

void pdi_seq_destroy(pdi_seq *q) {
  if (!q) return;
  if (q->exec) (void)hipGraphExecDestroy(q->exec);
  if (q->graph) (void)hipGraphDestroy(q->graph);
  for (hipEvent_t e : q->events) (void)hipEventDestroy(e);
  for (hipStream_t s : q->streams) (void)hipStreamDestroy(s);
  delete q;
}

int pdi_seq_create(pdi_ctx *ctx, int n, const pdi_frame *frame, const pdi_mask *masks,
                   const float *const *values, int block_size, const pdi_params *params,
                   float *const *outs, int nstreams, pdi_seq **out) {
  if (!ctx || !frame || !masks || !values || !outs || !out || n <= 0 || nstreams <= 0 || nstreams > 16)
    return PDI_EINVAL;
  *out = nullptr;
  pdi_seq *q = new pdi_seq();
  q->ctx = ctx;
  int rc = PDI_OK;
  hipError_t e = hipSuccess;
  for (int i = 0; i < nstreams && e == hipSuccess; ++i) {
    hipStream_t s;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) q->streams.push_back(s);
  }
  for (int i = 0; i < 2 * nstreams && e == hipSuccess; ++i) {
    hipEvent_t ev;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) q->events.push_back(ev);
  }
  if (e != hipSuccess) {
    pdi_seq_destroy(q);
    return PDI_EHIP;
  }
  // Batches: consecutive frames, at most PDI_MAX_BATCH, spread evenly.
  const int per_stream = (n + nstreams - 1) / nstreams;
  const int bsize = per_stream < PDI_MAX_BATCH ? per_stream : PDI_MAX_BATCH;
  // Eager decodes of the largest batch on every stream first: tables and
  // per-stream workspaces are allocated outside the capture, and errors
  // surface here.
  for (int i = 0; i < nstreams && rc == PDI_OK; ++i) {
    const int cnt = bsize < n ? bsize : n;
    rc = decode_residual_batch(ctx, cnt, frame, masks, values, block_size, params, outs, q->streams[i]);
    if (rc == PDI_OK) rc = pdi_sync(ctx, q->streams[i]);
  }
  if (rc != PDI_OK) {
    pdi_seq_destroy(q);
    return rc;
  }
  hipStream_t origin = q->streams[0];
  e = hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    e = hipEventRecord(q->events[0], origin);
    for (int i = 1; i < nstreams && e == hipSuccess; ++i) e = hipStreamWaitEvent(q->streams[i], q->events[0], 0);
    for (int k0 = 0, b = 0; k0 < n && e == hipSuccess && rc == PDI_OK; k0 += bsize, ++b) {
      const int cnt = n - k0 < bsize ? n - k0 : bsize;
      rc = decode_residual_batch(ctx, cnt, frame, &masks[k0], &values[k0], block_size, params, &outs[k0],
                                 q->streams[b % nstreams]);
    }
    for (int i = 1; i < nstreams && e == hipSuccess; ++i) {
      e = hipEventRecord(q->events[nstreams + i], q->streams[i]);
      if (e == hipSuccess) e = hipStreamWaitEvent(origin, q->events[nstreams + i], 0);
    }
    hipError_t e2 = hipStreamEndCapture(origin, &q->graph);
    if (e == hipSuccess) e = e2;
  }
  if (e == hipSuccess && rc == PDI_OK) e = hipGraphInstantiate(&q->exec, q->graph, nullptr, nullptr, 0);
  if (e != hipSuccess || rc != PDI_OK) {
    pdi_seq_destroy(q);
    return rc != PDI_OK ? rc : PDI_EHIP;
  }
  *out = q;
  return PDI_OK;
}

int pdi_seq_launch(pdi_seq *q, void *stream) {
  if (!q || !q->exec) return PDI_EINVAL;
  return hipGraphLaunch(q->exec, (hipStream_t)stream) == hipSuccess ? PDI_OK : PDI_EHIP;
}

int pdi_seq_sync(pdi_seq *q, void *stream) {
  if (!q) return PDI_EINVAL;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return PDI_EHIP;
  int rc = PDI_OK;
  for (hipStream_t s : q->streams) {
    const int r = pdi_sync(q->ctx, s);
    if (rc == PDI_OK) rc = r;
  }
  return rc;
}

}  // extern "C"
