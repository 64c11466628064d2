// Internal descriptors shared by the host side (pdinp_host.cpp) and the
// gfx950 kernels (pdinp_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdi {

constexpr int kMaxShapes = 8;   // distinct (w, h) block shapes per frame
constexpr int kMaxGroups = 3;   // mask-plane groups: Y, (C) or (Cb, Cr)
constexpr int kFastKMax = 31;   // largest K of the wave-level path (R <= 32 rows)
constexpr int kLdsKMax = 96;    // largest K whose bordered system fits in LDS (general path)
constexpr int kDeferredGrid = 64;  // persistent workgroups of the general path
constexpr int kWaveItems = 4;      // blocks per wave in the wave-level path
constexpr int kFastItemsPerWG = 16;  // blocks per workgroup of the wave-level path (b <= 16)
constexpr int kWideItemsDefault = 2;  // blocks per workgroup of the wave-per-block path (1, 2 or 4)
constexpr int kWideKMax = 103;       // largest K of the wave-per-block path
// Point-count bins of the wave-per-block queues, handed out largest first,
// one per tile count of the bordered system (n = K + 1 rows, 16 per tile):
// bin 0 K >= 96 (7 tiles), bin 1 K >= 80 (6), bin 2 K >= 64 (5), bin 3 the
// rest (at most 4).
constexpr int kBinK0 = 96, kBinK1 = 80, kBinK2 = 64;
// Device counters: [0], [1] deferred-list lengths, [2] finished workgroups of
// the deferred pass, then per frame fi of the launch and wave-per-block queue
// q the lengths of its 4 bins at [kQueueCounters + 4 (fi kMaxShapes + q) + bin].
constexpr int kQueueCounters = 8;
constexpr int kMaxBatch = 32;  // frames of one geometry per launch (decode_residual_batch)
// Deferred-list entries hold (frame << kDeferFrameShift) | block.
constexpr int kDeferFrameShift = 24;
constexpr int kDeferItemMask = (1 << kDeferFrameShift) - 1;
// Zero-padded DCT-II matrices Dw, Dh and eigenvalues lam of a block shape,
// n x n (n = 16 for b <= 16, 32 for b = 32) with row stride n + 1, so that
// the evaluation's column gathers (16 lanes, 16 rows, one column) fall into
// 16 different LDS banks.
constexpr int kDct16Ld = 17, kDct16Floats = 16 * kDct16Ld;
// Row-pair table of a w x h shape (b <= 16): the block of row y holds h rows
// of w + 1 floats plus one pad float, so that lanes whose points differ in y
// read from different LDS banks (h (w + 1) = 272 alone is 16 mod 64).
__host__ __device__ constexpr int jrow(int w, int h) { return h * (w + 1) + 1; }
constexpr int kDct32Ld = 33, kDct32Floats = 32 * kDct32Ld;
static_assert(kDct16Floats % 4 == 0 && kDct32Floats % 4 == 0, "16-byte copies");
// The FP32 table buffer is padded by this many floats so that the wave-level
// path may read whole 16-byte vectors per thread past the last table.
constexpr int kTabPadFloats = 6 * 256 * 4;

// Device status bits (OR-ed by kernels, read by pdi_sync).
constexpr int kStatusMask = 1;
constexpr int kStatusValue = 2;
constexpr int kStatusSolve = 4;

// Per distinct block shape: offsets of its tables in the table buffers.
struct ShapeDev {
  int w, h;
  int hc32;       // FP32 compact Green table, (w+1)*(h+1), quarter-scaled (floats)
  int hc64;       // same in FP64 (doubles)
  int fast;       // block of the batched paths: for b <= 16 the row-pair table
                  // J[y*jrow(w,h) + y'*(w+1) + alpha] (jt_floats floats), then the
                  // zero-padded 16x16 DCT-II matrices Dw[p][x], Dh[q][y] and the
                  // eigenvalues lam[q][p] (kDct16Floats floats each, row
                  // stride kDct16Ld); for b = 32 the compact table
                  // (jt_floats floats) and the same three matrices padded to
                  // 32x32 (kDct32Floats floats each, row stride kDct32Ld)
  int jt_floats;  // size of the first table rounded up to a multiple of 4
};

// A run of blocks of one shape: block columns bx0 .. bx0+nx-1, rows by0 ..,
// `count` blocks in raster order, served by workgroups first_wg .. .
struct SegDev {
  int group, shape, bx0, nx, by0, count, first_wg;
};
constexpr int kMaxSegs = 4 * kMaxGroups;
constexpr int kNumCounters = kQueueCounters + 4 * kMaxShapes * kMaxBatch;

// Static device scratch of decode_residual_batch_noalloc (pdinp_noalloc.hip):
// the status word (4 ints) at byte 0, the counters at kNoAllocCountersOff
// (both start at zero), then the deferred list, the wave-per-block queues
// and the global-memory systems of one decode.
constexpr long long kNoAllocScratchBytes = 32ll << 20;
constexpr long long kNoAllocCountersOff = 256;
constexpr long long kNoAllocHeadBytes = kNoAllocCountersOff + ((4ll * kNumCounters + 255) / 256) * 256;
// Device address of the given device's copy of that scratch (taken once per
// device by hipGetSymbolAddress with the device current; its head is zeroed
// then).
hipError_t noalloc_setup(int device, void **ptr);

// The blocks of one shape for the wave-per-block path.  binlist[2 base ..
// 2 base + 2 count) holds them by point count: bin 0 from the front of the
// first half, bin 1 from its back, bins 2 and 3 likewise in the second half;
// workgroups first_wg .. take them in bin order.  In the binned wave-level
// path a queue is one segment (mask-plane group and edge kind) with the
// group's index in first_wg; its blocks are placed in f.fl.
struct QueueDev {
  int shape, count, base, first_wg;
};

// Per mask-plane group (Y; shared chroma; or Cb and Cr separately).
struct GroupDev {
  int first;            // first mask-block index of the group
  int W, H, nbx, nby;   // geometry of the plane the mask lives on
  int nv;               // value sets decoded with this mask (1, or 2 for shared chroma)
  int vplane[2];        // value planes (0 = Y, 1 = Cb, 2 = Cr)
  long long out_off[2]; // output offset of each value plane (floats)
  int shape[4];         // shape ids: full, right edge, bottom edge, corner
  int cbase[2];         // stored-coefficient decodes: index in consts[] of the
                        // first block of each value plane (block l of the
                        // group is at cbase[v] + l)
};

// Caller buffers of one frame of a launch.
struct FramePtrs {
  const int32_t *block_ptr;
  const uint16_t *pos;
  const float *values;
  float *out;  // FP32 planes, or int8 planes when out_i8
  const int8_t *coef;    // stored-coefficient decodes: codes, laid out like values
  const float *consts;   // and the constant of every block of every plane
  int8_t *qout;          // coefficient encodes: codes out, laid out like values
  float *aout;           // and the constant of every block of every plane
};

struct FrameDev {
  int b;
  int n_items;       // mask blocks
  int ngroups;
  int shared;        // shared chroma mask
  int chroma_first;  // first chroma mask block (shared Cr values are addressed from it)
  int nshapes;
  int validate;
  int refine;        // 0 off, 1 auto, 2 always
  float tau;         // auto-refine threshold on min/max pivot
  int eval;          // PDI_EVAL_*
  int out_i8;        // 1: out holds int8 pixels, clamp(rint(u), -128, 127)
  int coef;          // 1: stored coefficients (codes + constants), no solve
  int enc;           // 1: coefficient encode (solve, then quantise c and store a; no evaluation)
  // Mask selection (pdinp_select.hip): dense residual planes in, one 64-bit
  // mask word per block, then the packed mask and values out.
  const float *sel_planes;
  unsigned long long *sel_bits;
  int *sel_x;        // scratch: per-block prefix inside its tile of 256, then the tile totals
  int32_t *sel_bp;
  uint16_t *sel_pos;
  float *sel_vals;
  float sel_thr[2];  // luma, chroma thresholds on a rectangle's mean squared error
  int sel_rounds;
  float qstep[3];    // quantiser step per plane (coef, enc)
  float qrho;        // reconstruction offset (coef)
  GroupDev g[kMaxGroups];
  ShapeDev s[kMaxShapes];
  SegDev seg[kMaxSegs];
  int nsegs;
  int ipw;           // blocks per workgroup of the batched path
  int nq;            // queues of the binned paths (0: no queue counters to clear after
                     // the decode): the wave-per-block path (b = 32) has one per block
                     // shape, smallest first; the binned wave-level path (b <= 16) one
                     // per mask-plane group and edge kind (q[].shape is then the shape of
                     // that group's full, right-edge, bottom-edge or corner blocks)
  QueueDev q[kMaxSegs];
  int qof[kMaxShapes];  // queue of each shape (wave-per-block path)
  int qge[kMaxGroups][4];  // queue of each group and edge kind (binned wave-level path)
  int fast_wgs;      // workgroups per frame of the batched path (k_fast or k_wide)
  int fast_lds;      // its dynamic LDS (floats): largest table block
  int tab32_floats;  // size of the FP32 table buffer (floats)
  // buffers: frame fi of the launch (blockIdx.y in the batched kernels)
  int nframes;
  int tail_in_wg;  // k_fast decodes its leftover blocks itself (else: deferred list)
  FramePtrs fp[kMaxBatch];
  const float *tab32;
  const double *tab64;
  int *deferred;   // mask blocks left to the general path, as (fi << 24) | m
                   // (n_items * nframes entries)
  int *binlist;    // queues of the wave-per-block path (2 n_items entries per frame)
  // binned wave-level path: its blocks in hand-out order, 16 per k_fast2
  // workgroup (4 ints each: (fi << 24) | m, first point, K, first Cr value
  // or -1 for one value plane), a descriptor per workgroup (2 ints: bin |
  // valid entries << 8 | 16-byte table vectors << 16, or -1: none; the float
  // offset of the bin's shape tables) and the binning's per-workgroup bin
  // counts / offsets
  int *fl;
  int *wgdesc;
  int *hist;
  int *counters;   // kNumCounters device counters (layout above)
  int *status;     // device status word
  float *slots;    // global-memory systems for K > kLdsKMax, one slot per workgroup
  long long slot_floats;
  int slot_wgs;    // workgroups of the deferred pass that own a slot (<= kDeferredGrid)
};

// Launchers (pdinp_kernels.hip).  All asynchronous on `stream`.
hipError_t launch_fast(const FrameDev &f, hipStream_t stream);
// Binned residual decode for b <= 16 (k_fbin + k_fast2): f.q / f.qof / f.nq
// describe one queue per block shape, f.fast_wgs the k_fast2 grid.
hipError_t launch_fast2(const FrameDev &f, hipStream_t stream);
// The parts of a batched residual decode by k_wide on three streams: part 1
// on aux[0], parts 2 and then 3 on aux[1], forked from the caller's stream
// after the binning and joined back to it with the events, part 4 on the
// caller's stream.
constexpr int kWideAux = 2;
struct WideFork {
  hipStream_t aux[kWideAux];
  hipEvent_t fork;
  hipEvent_t join[kWideAux];
};
// binning kernel + k_wide (fork: null keeps every part on `stream`)
hipError_t launch_wide(const FrameDev &f, hipStream_t stream, const WideFork *fork = nullptr);
hipError_t launch_plain_all(const FrameDev &f, hipStream_t stream);
hipError_t launch_general_deferred(const FrameDev &f, hipStream_t stream);
hipError_t launch_coef_general(const FrameDev &f, hipStream_t stream);  // coef: the deferred blocks
hipError_t launch_select(const FrameDev &f, hipStream_t stream);        // mask selection, b = 8

// Global homogeneous diffusion inpainting (pdinp_diffusion.hip); all
// asynchronous on the stream.  Scalars (GAM = r.r and DEL = w.r per
// iteration, BB = |b|^2) are kHdSlots doubles each, summed by their readers.
constexpr int kHdSlots = 64;
hipError_t hd_restrict(const uint8_t *mf, const float *ff, int Wf, int Hf, uint8_t *mc, float *fc, int Wc, int Hc,
                       hipStream_t s);
hipError_t hd_init(const uint8_t *m, const float *f, int W, int H, const float *uc, int Wc, float *u, hipStream_t s);
hipError_t hd_residual(const uint8_t *m, const float *f, const float *u, int W, int H, float *r, double *rr,
                       double *bb, hipStream_t s);
// w = A r on the unknowns and DEL[0] += w . r (start of a level's CG).
hipError_t hd_start(const uint8_t *m, const float *r, int W, int H, float *w, double *del, hipStream_t s);
// One CG iteration (k_hd_cg): u, p in place; r, w, s read from ri, wi, si
// and written to ro, wo, so; GAM[it + 1], DEL[it + 1] accumulated and
// ALPHA[it] recorded.  GAM and DEL hold kHdSlots slots per iteration.
// Does nothing once GAM[it] <= tol2 * BB (converged).
hipError_t hd_iterate(const uint8_t *m, int W, int H, double *GAM, double *DEL, double *ALPHA, const double *BB,
                      double tol2, int it, float *u, float *p, const float *ri, const float *wi, const float *si,
                      float *ro, float *wo, float *so, hipStream_t s);
hipError_t hd_zero(double *a, int n, hipStream_t s);

}  // namespace pdi
