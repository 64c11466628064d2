#!/usr/bin/env python3
"""Residual-decode benchmark on one MI355X.

Workloads (synthetic, seeded; the recipe is in paper_2008_10273_amd/synth.py):
  --config 1 (default): 1920x1080 4:2:0 residual frames, 16x16 blocks,
      per-block mask density U[1%, 10%] (3-26 points per full block), values
      = smooth sum of 4 random sinusoids + N(0, 2) noise, clipped to
      [-64, 64].  One step = one decode_residual_batch call over --batch (32)
      different frames: every block assembled, solved and evaluated on the
      GPU, inputs resident in HBM.  Single-frame throughput and latency are
      reported beside it.
  --config 0 / 2: the 256x256 grey case / 1080p frames with 32x32 blocks and
      density U[2%, 10%].
  --config 3: 64 consecutive 1080p frames decoded as one HIP-graph replay
      (pdi_seq, frames spread over --nstreams streams); one step = one replay.
  --config 4: serving mix, 16 client streams (6x 854x480, 6x 1280x720,
      4x 1920x1080, 4:2:0, b16) with Poisson arrivals at 25 frames/s each,
      through the pdi_server request loop; latency counts from submission
      (host data) to completion on the device.
  --config 5: the paper's decoder split - 1080p 4:2:0 frames with 8x8 blocks
      (masks as config 1) decoded from stored int8 codes and block constants
      by decode_coefficients_batch over --batch frames (no solve).
  --config 7: the encoder side of that split - the same 1080p 4:2:0 frames
      (8x8 blocks, masks and residual values) solved per block and quantised
      to int8 codes + block constants by encode_coefficients_batch over
      --batch frames.
  --config 8: the encoder's mask selection - dense 1920x1080 4:2:0 residual
      planes, every 8x8 block's mask chosen by rectangular subdivision and
      the values at the points gathered (select_mask); one step = one frame.
  --config 6: intra prediction - global homogeneous diffusion inpainting of
      a 1920x1080 plane with a 4 % random mask (inpaint_homogeneous,
      cascadic CG to a relative residual of 1e-6); one step = one plane.

Prints one JSON line with the metric, latency percentiles, the error against
the FP64 oracle, a roofline record of the decode and the oracle timed on the
host cores.
"""
import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "1080p residual frames/s at ≤0.5 grey-level error; p99 frame latency"
HBM_PEAK_GBS = 8000.0
EVALS = {"fp32": 0, "fp16": 1, "bf16": 2, "bf16x2": 3}
# HBM bytes per batched step from rocprofv3 FETCH_SIZE + WRITE_SIZE counters
# of its kernels, scaled by the same counters read on a copy kernel of known
# size (profiles/*_counters.txt); only for the kernel build the counters were
# taken on (null after a kernel change).  (config, frames per step): bytes.
# Config 1: k_fbin_* + k_fast2 + deferred pass (k_fast2 ignores the launch
# choice).  Config 2: k_bin + the four k_wide parts + deferred pass, for the
# launch choice of 4 blocks per workgroup only (the (config, frames, blocks
# per workgroup) key); the 1- and 2-wave choices counted ~40 % more writes.
# Config 5: k_fast in coefficient mode + k_coef_general (no launch choice).
TRAFFIC = {(1, 32): 510359722, (2, 32, 4): 462664444, (5, 32): 463789739}


def algorithmic_bytes(fr) -> int:
    """Bytes the decode must move: packed mask + values in, FP32 planes out."""
    n_in = 4 * fr.block_ptr.size + 2 * fr.pos.size + 4 * fr.values.size
    return int(n_in + 4 * fr.out_size)


def _gen(job):
    from paper_2008_10273_amd import synth
    kind, a, b = job
    if kind == "cfg":
        return synth.config_frame(a, frame=b, keep_fields=False)
    if kind == "coef":
        return synth.coef_frame(b)
    return synth.serving_frame(a, b)


def generate(jobs, workers):
    """Frames generated in worker processes (before the GPU is touched)."""
    if workers <= 1 or len(jobs) <= 1:
        return [_gen(j) for j in jobs]
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_gen, jobs, chunksize=1))


def host_cores():
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(fr, min_seconds=5.0, min_frames=3, what="the benchmark frame"):
    """The FP64 oracle timed on the host cores (all threads, then one)."""
    import oracle
    cores = host_cores()
    oracle.decode(fr, nthreads=cores)  # load + warm

    def run(nt, secs, nmin):
        n, t0, r = 0, time.perf_counter(), None
        while n < nmin or time.perf_counter() - t0 < secs:
            r = oracle.decode_flat(fr, nthreads=nt)
            n += 1
        return r, n, time.perf_counter() - t0

    ref, n, dt = run(cores, min_seconds, min_frames)
    _, n1, dt1 = run(1, min_seconds / 2, 1)
    return ref, dict(value=n / dt, unit="frames/s", cores=cores, kind="oracle",
                     sample=f"{n} decodes of {what} (FP64 oracle, OpenMP over blocks), {dt:.1f} s",
                     one_thread=n1 / dt1, cpu_model=cpu_model(), nproc=os.cpu_count())


def copy_bandwidth(torch, mib=1024, reps=20, stream=None):
    """Device-to-device copy of `mib` MiB (torch's copy kernel): GB/s counted
    as bytes read + bytes written."""
    n = (mib << 20) // 4
    x = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    stream = stream or torch.cuda.current_stream()
    with torch.cuda.stream(stream):
        for _ in range(3):
            y.copy_(x)
        tm = StreamTimer(torch, stream)
        tm.start()
        for _ in range(reps):
            y.copy_(x)
        secs = tm.stop()
    return 2.0 * (mib << 20) * reps / secs / 1e9


def error_vs(got, ref):
    e = np.abs(got - ref)
    q = lambda x: np.clip(np.rint(x), -128, 127)
    return dict(max_abs=float(e.max()), round_agree=float(np.mean(q(got) == q(ref))))


def host_outputs(ds):
    return [dd["out"].cpu().numpy() for dd in ds]


def error_frames(outs, refs):
    """error_vs over the FP32 outputs of several frames (host arrays), one
    frame at a time (max of the maxima, pixel-weighted agreement)."""
    mx, agree, npx = 0.0, 0.0, 0
    for o, ref in zip(outs, refs):
        e = error_vs(o.astype(np.float64), ref)
        mx = max(mx, e["max_abs"])
        agree += e["round_agree"] * ref.size
        npx += ref.size
    return dict(max_abs=mx, round_agree=agree / npx, frames_checked=len(refs))


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


class StreamTimer:
    """HIP events recorded on the stream the decode kernels run on."""

    def __init__(self, torch, stream):
        self.torch, self.stream = torch, stream
        self.e0 = torch.cuda.Event(enable_timing=True)
        self.e1 = torch.cuda.Event(enable_timing=True)

    def start(self):
        self.e0.record(self.stream)

    def stop(self):
        self.e1.record(self.stream)
        self.e1.synchronize()
        return self.e0.elapsed_time(self.e1) / 1e3


def time_decodes(torch, dec, d, params, stream, steps, warmup):
    for _ in range(warmup):
        dec.decode(d, params, stream=stream)
    torch.cuda.synchronize()
    tm = StreamTimer(torch, stream)
    t0 = time.perf_counter()
    tm.start()
    for _ in range(steps):
        dec.decode(d, params, stream=stream)
    secs = tm.stop()
    torch.cuda.synchronize()
    return secs, time.perf_counter() - t0


def latencies(torch, dec, d, params, stream, iters):
    out = []
    tm = StreamTimer(torch, stream)
    for _ in range(iters):
        tm.start()
        dec.decode(d, params, stream=stream)
        out.append(1e3 * tm.stop())
    return np.array(out)


def overlapped(torch, dec, ds, params, nstreams, steps):
    """Frames in flight on several streams at once (each stream decodes its
    own frames back to back); whole-job frames/s."""
    streams = [torch.cuda.Stream() for _ in range(nstreams)]
    for k in range(2 * nstreams):
        dec.decode(ds[k % len(ds)], params, stream=streams[k % nstreams])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        dec.decode(ds[k % len(ds)], params, stream=streams[k % nstreams])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for s in streams:
        assert dec.sync(s) == 0
    return steps / dt


def oracle_flat(fr):
    import oracle
    return oracle.decode_flat(fr, nthreads=host_cores())


def meets_bar(err):
    """The acceptance bar: max-abs <= 0.5 grey levels and identical 8-bit
    rounding on >= 99.9 % of the pixels."""
    return bool(err["max_abs"] <= 0.5 and err["round_agree"] >= 0.999)


def dtype_sweep(args, torch, binding, dec, ds, refs, stream, tune_b):
    """The batched decode of the same frames with each evaluation dtype
    (FP32 solve; FP32, FP16, BF16 or split-BF16 operands in the evaluation,
    FP32 accumulation): frames/s over --dtype-steps steps and the error of
    every frame against the FP64 oracle."""
    out = {}
    B = len(ds)
    tm = StreamTimer(torch, stream)
    for name, ev in EVALS.items():
        p = binding.default_params(eval_dtype=ev)
        for _ in range(3):
            dec.decode_batch(ds, p, stream=stream)
        tm.start()
        for _ in range(args.dtype_steps):
            dec.decode_batch(ds, p, stream=stream)
        secs = tm.stop()
        assert dec.sync(stream) == 0, binding.pdi_last_error(dec.ctx)
        rec = dict(value=B * args.dtype_steps / secs, unit="frames/s", ms_per_step=1e3 * secs / args.dtype_steps)
        if refs is not None:
            e = error_frames(host_outputs(ds), refs)
            rec.update(max_abs=e["max_abs"], round_agree=e["round_agree"], meets_bar=meets_bar(e),
                       frames_checked=len(ds))
        out[name] = rec
        log(f"  eval {name}: {rec['value']:.1f} frames/s" +
            (f", max|err| {rec['max_abs']:.3e}, 8-bit agreement {rec['round_agree']:.6f}, "
             f"{'meets' if rec['meets_bar'] else 'FAILS'} the bar" if refs is not None else ""))
    return out


def bench_frame(args, torch, binding, synth):
    """One step = one decode_residual_batch call over `--batch` different
    frames of the workload (decode_residual for --batch 1)."""
    B = args.batch
    frames = generate([("cfg", args.config, k) for k in range(B)], args.workers if B > 1 else 1)
    fr = frames[0]
    cfg = synth.CONFIGS[args.config]
    dec = binding.Decoder(0)
    ds = [dec.upload(f) for f in frames]
    d = ds[0]
    stream = torch.cuda.Stream()
    params = binding.default_params(eval_dtype=EVALS[args.eval])
    # launch choices for this geometry (0: none to make), one for single-frame
    # decodes and one for launches of B frames
    tune = dec.autotune(d, params, stream=stream)
    tune_b = dec.autotune_batch(ds, params, stream=stream) if B > 1 else tune
    log(f"config {args.config} ({cfg['name']}), eval {args.eval}, {B} frames per step, {args.steps} steps, "
        f"autotune choice {tune_b} ({B} frames), {tune} (single frame)")

    def step():
        if B == 1:
            dec.decode(d, params, stream=stream)
        else:
            dec.decode_batch(ds, params, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    tm = StreamTimer(torch, stream)
    t0 = time.perf_counter()
    tm.start()
    for _ in range(args.steps):
        step()
    secs = tm.stop()
    wall = time.perf_counter() - t0
    assert dec.sync(stream) == 0, binding.pdi_last_error(dec.ctx)
    fps = B * args.steps / secs
    timed_outs = host_outputs(ds)  # every frame of the last timed step
    log(f"decode: {fps:.1f} frames/s, {1e3 * secs / args.steps:.4f} ms per step of {B} frames")

    # single frames: throughput and latency of one frame decoded alone
    s_secs, _ = time_decodes(torch, dec, d, params, stream, args.steps, max(5, args.warmup // 4))
    lat = latencies(torch, dec, d, params, stream, args.latency_iters)
    single = dict(value=args.steps / s_secs, unit="frames/s", ms_per_frame=1e3 * s_secs / args.steps)
    log(f"single frame: {single['value']:.1f} frames/s, p50 {np.percentile(lat, 50):.4f} ms, "
        f"p99 {np.percentile(lat, 99):.4f} ms")

    multi = None
    if len(ds) > 1:
        mfps = overlapped(torch, dec, ds, params, args.nstreams, args.steps)
        multi = dict(value=mfps, unit="frames/s", streams=args.nstreams, frames=len(ds),
                     note="single-frame decodes of these frames in flight on several streams")
        log(f"overlapped on {args.nstreams} streams: {mfps:.1f} frames/s")

    int8 = None
    if B > 1:
        # the same batched decode writing 8-bit planes clamp(rint(u)) (out_int8)
        p8 = binding.default_params(eval_dtype=EVALS[args.eval], out_int8=1)
        for _ in range(max(5, args.warmup // 4)):
            dec.decode_batch(ds, p8, stream=stream)
        s8 = max(10, args.steps // 2)
        tm.start()
        for _ in range(s8):
            dec.decode_batch(ds, p8, stream=stream)
        t8 = tm.stop()
        assert dec.sync(stream) == 0, binding.pdi_last_error(dec.ctx)
        int8 = dict(value=B * s8 / t8, unit="frames/s", ms_per_step=1e3 * t8 / s8,
                    note="out_int8: 8-bit planes instead of FP32 (a quarter of the output bytes), same decode")
        log(f"int8 output: {int8['value']:.1f} frames/s")

    plain = None
    if not args.no_plain:
        pp = binding.default_params(eval_dtype=EVALS[args.eval], path=binding.PDI_PATH_PLAIN)
        psteps = max(10, args.steps // 10)
        ps, _ = time_decodes(torch, dec, d, pp, stream, psteps, 5)
        plain = dict(value=psteps / ps, unit="frames/s", ms_per_step=1e3 * ps / psteps,
                     path="one workgroup per block, FP32 LDS Gauss-Jordan, direct VALU evaluation, single frames")
        log(f"plain path: {plain['value']:.1f} frames/s")

    err = cpu = refs = None
    if not args.no_cpu:
        ref, cpu = cpu_baseline(fr, min_seconds=args.cpu_seconds)
        # every frame of the timed batch against the oracle (the outputs of the last timed step)
        refs = [ref] + [oracle_flat(f) for f in frames[1:]]
        err = error_frames(timed_outs, refs)
        log(f"oracle: {cpu['value']:.2f} frames/s on {cpu['cores']} cores; max|err| over the {len(frames)} "
            f"timed frames {err['max_abs']:.3e}, 8-bit agreement {err['round_agree']:.6f}")
    per_dtype = dtype_sweep(args, torch, binding, dec, ds, refs, stream, tune_b) if args.dtypes else None

    ab = sum(algorithmic_bytes(f) for f in frames)
    t_step = secs / args.steps
    achieved = ab / t_step / 1e9
    copy_gbs = copy_bandwidth(torch, stream=stream)
    log(f"copy kernel: {copy_gbs:.0f} GB/s")
    binned = B > 1 and fr.n_mask_blocks * B >= 32768  # the library's threshold for the binned path
    kern = (("k_fbin_count + k_fbin_scan + k_fbin_place + k_fast2" if binned else "k_fast") if cfg["block_size"] <= 16
            else ("k_bin + k_wide (one launch per tile count: 7, 6, 5, <= 4)" if B > 1 else "k_bin + k_wide"))
    rec = dict(metric=METRIC, value=fps, unit="frames/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
               ms_per_step=1e3 * t_step, higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f32" if args.eval == "fp32" else f"f32 solve, {args.eval} eval", data="synthetic",
               config={"workload": cfg["name"], "width": cfg["width"], "height": cfg["height"],
                       "format": "4:2:0" if cfg["fmt"] == 1 else "gray", "block_size": cfg["block_size"],
                       "density": list(cfg["density"]), "frames_per_step": B,
                       "mask_blocks": fr.n_mask_blocks, "mask_points": int(fr.pos.size),
                       "blocks_per_workgroup": tune_b or None, "blocks_per_workgroup_single": tune or None},
               latency_ms={"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                           "mean": float(lat.mean()), "of": "one frame decoded alone"},
               single_frame=single, error_vs_oracle=err, per_dtype=per_dtype, plain_path=plain, overlapped=multi,
               int8_output=int8,
               roofline={"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS,
                         "traffic": (TRAFFIC.get((args.config, B, tune_b), TRAFFIC.get((args.config, B)))
                                     if args.eval == "fp32" else None),
                         "kernel": kern + (" (+ deferred pass)" if B > 1 or cfg["block_size"] > 16 else ""),
                         "algorithmic_bytes_per_launch": ab, "launch_ms": 1e3 * t_step,
                         "measured_copy_GBs": copy_gbs, "frac_of_measured_copy": achieved / copy_gbs},
               cpu_baseline=cpu, wall_s=wall)
    dec.close()
    return rec


def coef_bytes(fr, q, consts) -> int:
    """Bytes a stored-coefficient decode must move: packed mask, int8 codes
    and block constants in, FP32 planes out."""
    return int(4 * fr.block_ptr.size + 2 * fr.pos.size + q.size + 4 * consts.size + 4 * fr.out_size)


def bench_coef(args, torch, binding, synth):
    """Config 5: the paper's decoder split - 1080p 4:2:0 frames with 8x8
    blocks decoded from stored codes and constants (decode_coefficients).
    One step = one decode_coefficients_batch call over --batch frames."""
    B = args.batch
    c = synth.COEF_CONFIG
    items = generate([("coef", 5, k) for k in range(B)], args.workers if B > 1 else 1)
    dec = binding.Decoder(0)
    ds = [dec.upload_coef(fr, q, cs) for fr, q, cs in items]
    d = ds[0]
    fr, q0, c0 = items[0]
    stream = torch.cuda.Stream()
    params = binding.default_params(eval_dtype=EVALS[args.eval])
    qp = binding.coef_params(c["steps"], c["rho"])
    log(f"config 5 ({c['name']}), eval {args.eval}, {B} frames per step, {args.steps} steps")

    def step():
        if B == 1:
            dec.decode_coef(d, qp, params, stream=stream)
        else:
            dec.decode_coef_batch(ds, qp, params, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    tm = StreamTimer(torch, stream)
    t0 = time.perf_counter()
    tm.start()
    for _ in range(args.steps):
        step()
    secs = tm.stop()
    wall = time.perf_counter() - t0
    assert dec.sync(stream) == 0, binding.pdi_last_error(dec.ctx)
    fps = B * args.steps / secs
    got = d["out"].cpu().numpy().astype(np.float64)
    log(f"decode: {fps:.1f} frames/s, {1e3 * secs / args.steps:.4f} ms per step of {B} frames")
    lat = []
    for _ in range(args.latency_iters):
        tm.start()
        dec.decode_coef(d, qp, params, stream=stream)
        lat.append(1e3 * tm.stop())
    lat = np.array(lat)
    log(f"single frame: p50 {np.percentile(lat, 50):.4f} ms, p99 {np.percentile(lat, 99):.4f} ms")
    err = cpu = None
    if not args.no_cpu:
        import oracle
        cores = host_cores()
        oracle.decode_coef(fr, q0, c0, c["steps"], c["rho"], nthreads=cores)
        n, tc0 = 0, time.perf_counter()
        while n < 3 or time.perf_counter() - tc0 < 5.0:
            ref = oracle.decode_coef_flat(fr, q0, c0, c["steps"], c["rho"], nthreads=cores)
            n += 1
        dt = time.perf_counter() - tc0
        cpu = dict(value=n / dt, unit="frames/s", cores=cores, kind="oracle",
                   sample=f"{n} decodes of the benchmark frame (FP64 oracle, Eq. 2 summed directly, "
                          f"OpenMP over blocks), {dt:.1f} s", cpu_model=cpu_model(), nproc=os.cpu_count())
        err = error_vs(got, ref)
        log(f"oracle: {cpu['value']:.2f} frames/s on {cores} cores; max|err| {err['max_abs']:.3e}")
    ab = sum(coef_bytes(*it) for it in items)
    t_step = secs / args.steps
    achieved = ab / t_step / 1e9
    copy_gbs = copy_bandwidth(torch, stream=stream)
    rec = dict(metric="1080p residual frames/s decoded from stored coefficients (8x8 blocks)", value=fps,
               unit="frames/s", n_gpus=1, steps=args.steps, warmup=args.warmup, ms_per_step=1e3 * t_step,
               higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f32" if args.eval == "fp32" else f"{args.eval} eval", data="synthetic",
               config={"workload": c["name"], "width": c["width"], "height": c["height"], "format": "4:2:0",
                       "block_size": c["block_size"], "density": list(c["density"]), "frames_per_step": B,
                       "mask_blocks": fr.n_mask_blocks, "mask_points": int(fr.pos.size),
                       "quantiser_steps": list(c["steps"]), "rho": c["rho"]},
               latency_ms={"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                           "mean": float(lat.mean()), "of": "one frame decoded alone"},
               error_vs_oracle=err,
               roofline={"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS,
                         "traffic": TRAFFIC.get((5, B)) if args.eval == "fp32" else None,
                         "kernel": "k_fast (coefficient mode) + k_coef_general",
                         "algorithmic_bytes_per_launch": ab, "launch_ms": 1e3 * t_step,
                         "measured_copy_GBs": copy_gbs, "frac_of_measured_copy": achieved / copy_gbs},
               cpu_baseline=cpu, wall_s=wall)
    dec.close()
    return rec


def encode_bytes(fr) -> int:
    """Bytes a coefficient encode must move: packed mask and values in, int8
    codes and the FP32 constant of every block of every plane out."""
    b = fr.block_size
    dims = synth_plane_dims(fr)
    nblocks = sum(((W + b - 1) // b) * ((H + b - 1) // b) for W, H in dims)
    return int(4 * fr.block_ptr.size + 2 * fr.pos.size + 4 * fr.values.size + fr.values.size + 4 * nblocks)


def synth_plane_dims(fr):
    dims = [(fr.width, fr.height)]
    if fr.fmt != 0:
        dims += [((fr.width + 1) // 2, (fr.height + 1) // 2)] * 2
    return dims


def bench_encode(args, torch, binding, synth):
    """Config 7: coefficient encode of 1080p 4:2:0 frames in 8x8 blocks
    (encode_coefficients_batch: solve every block, quantise c, keep a).
    One step = one call over --batch frames."""
    B = args.batch
    c = synth.ENCODE_CONFIG
    items = generate([("coef", 5, k) for k in range(B)], args.workers if B > 1 else 1)
    frs = [it[0] for it in items]
    dec = binding.Decoder(0)
    ds = [dec.alloc_coef(dec.upload(fr)) for fr in frs]
    d = ds[0]
    fr = frs[0]
    stream = torch.cuda.Stream()
    params = binding.default_params()
    qp = binding.coef_params(c["steps"], 0.5)
    log(f"config 7 ({c['name']}), {B} frames per step, {args.steps} steps")

    def step():
        if B == 1:
            dec.encode_coef(d, qp, params, stream=stream)
        else:
            dec.encode_coef_batch(ds, qp, params, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    tm = StreamTimer(torch, stream)
    t0 = time.perf_counter()
    tm.start()
    for _ in range(args.steps):
        step()
    secs = tm.stop()
    wall = time.perf_counter() - t0
    assert dec.sync(stream) == 0, binding.pdi_last_error(dec.ctx)
    fps = B * args.steps / secs
    n = fr.values.size
    q = d["coef"].cpu().numpy()[:n].astype(np.int64)
    a = d["consts"].cpu().numpy().astype(np.float64)
    log(f"encode: {fps:.1f} frames/s, {1e3 * secs / args.steps:.4f} ms per step of {B} frames")
    lat = []
    for _ in range(args.latency_iters):
        tm.start()
        dec.encode_coef(d, qp, params, stream=stream)
        lat.append(1e3 * tm.stop())
    lat = np.array(lat)
    log(f"single frame: p50 {np.percentile(lat, 50):.4f} ms, p99 {np.percentile(lat, 99):.4f} ms")
    err = cpu = None
    if not args.no_cpu:
        import oracle
        cores = host_cores()
        n_run, tc0 = 0, time.perf_counter()
        while n_run < 3 or time.perf_counter() - tc0 < 5.0:
            qo, cex, ao = oracle.encode_coef(fr, c["steps"], nthreads=cores)
            n_run += 1
        dt = time.perf_counter() - tc0
        cpu = dict(value=n_run / dt, unit="frames/s", cores=cores, kind="oracle",
                   sample=f"{n_run} encodes of the benchmark frame (FP64 oracle: dense LU per block, "
                          f"OpenMP over blocks), {dt:.1f} s", cpu_model=cpu_model(), nproc=os.cpu_count())
        diff = q != qo.astype(np.int64)
        err = dict(codes_differing=int(diff.sum()), codes=int(n), max_code_diff=int(np.abs(q - qo).max()),
                   max_abs_const=float(np.abs(a - ao).max()))
        log(f"oracle: {cpu['value']:.2f} frames/s on {cores} cores; {err}")
    ab = sum(encode_bytes(f) for f in frs)
    t_step = secs / args.steps
    achieved = ab / t_step / 1e9
    rec = dict(metric="1080p 4:2:0 residual frames/s encoded to quantised coefficients (8x8 blocks)", value=fps,
               unit="frames/s", n_gpus=1, steps=args.steps, warmup=args.warmup, ms_per_step=1e3 * t_step,
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32 (int8 codes)",
               data="synthetic",
               config={"workload": c["name"], "width": c["width"], "height": c["height"], "format": "4:2:0",
                       "block_size": c["block_size"], "density": list(c["density"]), "frames_per_step": B,
                       "mask_blocks": fr.n_mask_blocks, "mask_points": int(fr.pos.size),
                       "quantiser_steps": list(c["steps"])},
               latency_ms={"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                           "mean": float(lat.mean()), "of": "one frame encoded alone"},
               error_vs_oracle=err,
               roofline={"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                         "kernel": "k_fast (encode mode) + k_general_deferred",
                         "algorithmic_bytes_per_launch": ab, "launch_ms": 1e3 * t_step},
               cpu_baseline=cpu, wall_s=wall)
    dec.close()
    return rec


def bench_select(args, torch, binding, synth):
    """Config 8: mask selection by rectangular subdivision on dense 1080p
    4:2:0 residual planes (select_mask); one step = one frame."""
    c = synth.SELECT_CONFIG
    W, H, fmt = c["width"], c["height"], c["fmt"]
    planes = synth.residual_planes(W, H, fmt, 0)
    dec = binding.Decoder(0)
    pl = torch.from_numpy(np.concatenate([p.ravel() for p in planes])).cuda()
    stream = torch.cuda.Stream()
    sp = binding.select_params(*c["threshold"])
    log(f"config 8 ({c['name']}), {args.steps} steps")
    _, d = dec.select(W, H, fmt, pl, True, sp, stream=stream)

    def step():
        lib = binding.lib()
        f = binding.pdi_frame(W, H, fmt)
        rc = lib.select_mask(dec.ctx, ctypes.byref(f), 1, pl.data_ptr(), 8, ctypes.byref(sp),
                             d["block_ptr"].data_ptr(), d["pos"].data_ptr(), d["values"].data_ptr(),
                             stream.cuda_stream)
        assert rc == 0

    import ctypes
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    tm = StreamTimer(torch, stream)
    t0 = time.perf_counter()
    tm.start()
    for _ in range(args.steps):
        step()
    secs = tm.stop()
    wall = time.perf_counter() - t0
    assert dec.sync(stream) == 0, binding.pdi_last_error(dec.ctx)
    fps = args.steps / secs
    bp = d["block_ptr"].cpu().numpy()
    nnz = int(bp[-1])
    ny = synth.plane_block_counts(W, H, fmt, 8)[0]
    nvals = 2 * nnz - int(bp[ny])
    npx = sum(w * h for w, h in synth.plane_dims(W, H, fmt))
    log(f"select: {fps:.1f} frames/s, {1e3 * secs / args.steps:.4f} ms per frame, {nnz} mask points")
    cpu = agree = None
    if not args.no_cpu:
        import oracle
        cores = host_cores()
        n_run, tc0 = 0, time.perf_counter()
        while n_run < 2 or time.perf_counter() - tc0 < 5.0:
            ref = oracle.select_mask(W, H, fmt, 8, planes, True, c["threshold"], nthreads=cores)
            n_run += 1
        dt = time.perf_counter() - tc0
        cpu = dict(value=n_run / dt, unit="frames/s", cores=cores, kind="oracle",
                   sample=f"{n_run} selections of the benchmark frame (FP64 oracle, OpenMP over blocks), {dt:.1f} s",
                   cpu_model=cpu_model(), nproc=os.cpu_count())
        refpts = int(sum(m.sum() for m in ref))
        agree = dict(mask_points=nnz, oracle_mask_points=refpts)
        log(f"oracle: {cpu['value']:.2f} frames/s on {cores} cores; {agree}")
    ab = 4 * npx + 4 * (bp.size) + 2 * nnz + 4 * nvals
    t_step = secs / args.steps
    achieved = ab / t_step / 1e9
    rec = dict(metric="1080p 4:2:0 residual frames/s through per-block mask selection (8x8, rectangular subdivision)",
               value=fps, unit="frames/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
               ms_per_step=1e3 * t_step, higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f32", data="synthetic",
               config={"workload": c["name"], "width": W, "height": H, "format": "4:2:0", "block_size": 8,
                       "threshold": list(c["threshold"]), "mask_points": nnz, "mask_density": nnz / float(
                           W * H + ((W + 1) // 2) * ((H + 1) // 2))},
               error_vs_oracle=agree,
               roofline={"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                         "kernel": "k_select8 + k_sel_count + k_sel_pack",
                         "algorithmic_bytes_per_launch": ab, "launch_ms": 1e3 * t_step},
               cpu_baseline=cpu, wall_s=wall)
    dec.close()
    return rec


def bench_intra(args, torch, binding, synth):
    """Config 6: global homogeneous diffusion inpainting of 1080p planes
    (inpaint_homogeneous, cascadic CG, tol 1e-6); one step = one plane.  The
    steps cycle through --intra-planes distinct seeded planes of the recipe
    (each solve starts from its own mask and values; the launch sizing that
    the previous call's iteration counts guide sees a different plane every
    time); the same plane solved over and over is reported beside it."""
    c = synth.INTRA_CONFIG
    W, H = c["width"], c["height"]
    P = max(1, args.intra_planes)
    planes = [synth.intra_frame(W, H, c["density"], k) for k in range(P)]
    dec = binding.Decoder(0)
    mts = [torch.from_numpy(m.astype(np.uint8)).cuda() for m, _ in planes]
    fts = [torch.from_numpy(f).cuda() for _, f in planes]
    u = torch.empty((H, W), dtype=torch.float32, device="cuda")
    stream = torch.cuda.Stream()
    cp = binding.cg_params()
    log(f"config 6 ({c['name']}), tol {cp.tol:g}, {args.steps} steps over {P} distinct planes")
    for k in range(args.warmup):
        dec.inpaint(mts[k % P], fts[k % P], cp, stream=stream, u=u)
    torch.cuda.synchronize()
    tm = StreamTimer(torch, stream)
    t0 = time.perf_counter()
    tm.start()
    its_all = []
    for k in range(args.steps):
        _, _, its = dec.inpaint(mts[k % P], fts[k % P], cp, stream=stream, u=u)
        its_all.append(its)
    secs = tm.stop()
    wall = time.perf_counter() - t0
    last = (args.steps - 1) % P
    pps = args.steps / secs
    log(f"inpaint: {pps:.1f} planes/s, {1e3 * secs / args.steps:.3f} ms per plane, CG iterations on "
        f"1920x1080 {min(its_all)}..{max(its_all)}")
    m, f = planes[last]
    g = u.cpu().numpy().astype(np.float64)
    # the same plane again and again (the launch sizing then knows each level's count exactly)
    tm.start()
    for _ in range(args.steps):
        dec.inpaint(mts[0], fts[0], cp, stream=stream, u=u)
    rsecs = tm.stop()
    replay = dict(value=args.steps / rsecs, unit="planes/s", ms_per_plane=1e3 * rsecs / args.steps,
                  note="one plane solved repeatedly")
    log(f"same plane repeated: {replay['value']:.1f} planes/s")
    # the solve's defining properties on the GPU result of the last timed
    # plane (the exact oracle solve of a 1080p plane is the CPU leg below;
    # parity is tested on smaller planes)
    exact_at_mask = bool(np.all(g[m] == f[m]))
    cpu = None
    if not args.no_cpu:
        import oracle
        tc0 = time.perf_counter()
        ref = oracle.homogeneous_inpaint(m, f.astype(np.float64))
        dt = time.perf_counter() - tc0
        cpu = dict(value=1.0 / dt, unit="planes/s", cores=1, kind="oracle",
                   sample=f"one exact sparse FP64 solve (SuperLU) of the last timed 1920x1080 plane, {dt:.1f} s",
                   cpu_model=cpu_model(), nproc=os.cpu_count(),
                   max_abs_vs_gpu=float(np.abs(ref - g).max()))
        log(f"oracle: {cpu['value']:.4f} planes/s; max|gpu - exact| {cpu['max_abs_vs_gpu']:.3e}")
    # bytes of the finest level's CG: per iteration k_hd_cg reads the mask
    # (1 B) and u, p, r, w, s (20 B) at every pixel (the vectors are read
    # without waiting for the mask byte; they are zero at known pixels),
    # writes p, r', w', s' (16 B) at every pixel and u (4 B) at the unknowns;
    # coarser levels and the convergence checks are in the time
    nfree = np.mean([int((~mm).sum()) for mm, _ in planes])
    ab = float(np.mean(its_all)) * (37 * W * H + 4 * nfree)
    achieved = ab / (secs / args.steps) / 1e9
    rec = dict(metric="1080p intra planes/s by global homogeneous diffusion inpainting (tol 1e-6)", value=pps,
               unit="planes/s", n_gpus=1, steps=args.steps, warmup=args.warmup, ms_per_step=1e3 * secs / args.steps,
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32 (FP64 dot products)",
               data="synthetic",
               config={"workload": c["name"], "width": W, "height": H, "density": c["density"], "tol": cp.tol,
                       "distinct_planes": P, "cg_iterations_finest": [min(its_all), max(its_all)]},
               same_plane_repeated=replay,
               properties={"exact_at_mask": exact_at_mask, "min": float(g.min()), "max": float(g.max())},
               roofline={"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS,
                         # 85.42 MB of HBM traffic per finest-level iteration (rocprofv3
                         # FETCH_SIZE / WRITE_SIZE, copy-calibrated; profiles/k_hd_cg_*)
                         "traffic": float(np.mean(its_all)) * 85415700,
                         "kernel": "k_hd_cg, finest level (whole solve timed)",
                         "algorithmic_bytes_per_launch": ab, "launch_ms": 1e3 * secs / args.steps},
               cpu_baseline=cpu, wall_s=wall)
    dec.close()
    return rec


def bench_sequence(args, torch, binding, synth):
    cfg = synth.CONFIGS[3]
    n = cfg["frames"]
    log(f"config 3: generating {n} frames")
    frames = generate([("cfg", 3, k) for k in range(n)], args.workers)
    dec = binding.Decoder(0)
    params = binding.default_params(eval_dtype=EVALS[args.eval])
    ds = [dec.upload(f) for f in frames]
    seq = binding.Sequence(dec, ds, params, nstreams=args.nstreams)
    stream = torch.cuda.Stream()
    for _ in range(args.warmup):
        seq.launch(stream)
    assert seq.sync(stream) == 0
    tm = StreamTimer(torch, stream)
    t0 = time.perf_counter()
    tm.start()
    for _ in range(args.steps):
        seq.launch(stream)
    secs = tm.stop()
    wall = time.perf_counter() - t0
    assert seq.sync(stream) == 0
    reps = []
    for _ in range(args.latency_iters // 10 + 5):
        tm.start()
        seq.launch(stream)
        reps.append(1e3 * tm.stop())
    reps = np.array(reps)
    fps = n * args.steps / secs
    log(f"graph replay: {fps:.1f} frames/s, {1e3 * secs / args.steps:.3f} ms per {n}-frame replay")

    # the same frames decoded eagerly, one stream, one after another
    for d in ds[:4]:
        dec.decode(d, params, stream=stream)
    torch.cuda.synchronize()
    tm.start()
    for d in ds:
        dec.decode(d, params, stream=stream)
    eager = n / tm.stop()
    log(f"eager single stream: {eager:.1f} frames/s")

    err = cpu = None
    got = ds[0]["out"].cpu().numpy().astype(np.float64)
    if not args.no_cpu:
        ref, cpu = cpu_baseline(frames[0], min_seconds=args.cpu_seconds, what="frame 0 of the sequence")
        err = error_vs(got, ref)
        log(f"oracle: {cpu['value']:.2f} frames/s; max|err| {err['max_abs']:.3e}")
    ab = sum(algorithmic_bytes(f) for f in frames)
    t_step = secs / args.steps
    achieved = ab / t_step / 1e9
    rec = dict(metric=METRIC, value=fps, unit="frames/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
               ms_per_step=1e3 * t_step, higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f32" if args.eval == "fp32" else f"f32 solve, {args.eval} eval", data="synthetic",
               config={"workload": cfg["name"], "width": cfg["width"], "height": cfg["height"], "format": "4:2:0",
                       "block_size": cfg["block_size"], "density": list(cfg["density"]), "frames_per_step": n,
                       "streams": args.nstreams, "capture": "one HIP graph per sequence"},
               latency_ms={"replay_p50": float(np.percentile(reps, 50)), "replay_p99": float(np.percentile(reps, 99)),
                           "per_frame_mean": float(np.mean(reps) / n)},
               eager_single_stream=dict(value=eager, unit="frames/s"),
               error_vs_oracle=err,
               roofline={"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_fast (graph replay)",
                         "algorithmic_bytes_per_launch": ab},
               cpu_baseline=cpu, wall_s=wall)
    seq.close()
    dec.close()
    return rec


def bench_serving(args, torch, binding, synth):
    nstreams = sum(c for _, _, c in synth.SERVING_MIX)
    per = args.serve_frames
    log(f"config 4: generating {per} frames for each of {nstreams} client streams")
    jobs = [("srv", s, j) for s in range(nstreams) for j in range(per)]
    flat = generate(jobs, args.workers)
    frames = [flat[s * per:(s + 1) * per] for s in range(nstreams)]
    dec = binding.Decoder(0)
    params = binding.default_params(eval_dtype=EVALS[args.eval])
    # device output ring per client stream (results stay in HBM)
    ring = 4
    outs = [[torch.empty(frames[s][0].out_size, dtype=torch.float32, device="cuda") for _ in range(ring)]
            for s in range(nstreams)]
    srv = binding.Server(dec, nlanes=args.lanes, hbm_budget_bytes=args.budget_mb << 20, max_queue=4096)
    # warm every geometry on every lane
    warm = [srv.submit(frames[s][0], params, want_output=False, out_dev=outs[s][0])
            for s in range(nstreams) for _ in range(args.lanes)]
    for rc, t, _ in warm:
        assert rc == 0 and srv.wait(t)[0] == 0

    rate = args.fps_per_stream
    T = args.warm_s + args.duration
    rng = np.random.default_rng(np.random.SeedSequence([20081027, 4, 999]))
    events = []
    for s in range(nstreams):
        t = rng.exponential(1.0 / rate)
        j = 0
        while t < T:
            events.append((t, s, j))
            t += rng.exponential(1.0 / rate)
            j += 1
    events.sort()
    log(f"serving: {len(events)} arrivals over {T:.1f} s, {args.lanes} lanes")
    tickets = []
    t0 = time.perf_counter()
    for (t, s, j) in events:
        now = time.perf_counter() - t0
        if t > now:
            time.sleep(t - now)
        rc, tk, _ = srv.submit(frames[s][j % per], params, want_output=False, out_dev=outs[s][j % ring])
        assert rc == 0, rc
        tickets.append((t, s, tk))
    lat, done_w = [], 0
    for (t, s, tk) in tickets:
        st, l_us = srv.wait(tk)
        assert st == 0, st
        if t >= args.warm_s:
            lat.append(l_us / 1e3)
            done_w += 1
    wall = time.perf_counter() - t0
    lat = np.array(lat)
    served_fps = done_w / args.duration
    log(f"serving: {served_fps:.1f} frames/s, p50 {np.percentile(lat, 50):.3f} ms, p99 {np.percentile(lat, 99):.3f} ms")

    # capacity: every frame submitted at once, drained as fast as the lanes go
    burst = [(s, j) for j in range(per) for s in range(nstreams)] * args.burst_rounds
    tb = time.perf_counter()
    tks = [srv.submit(frames[s][j], params, want_output=False, out_dev=outs[s][j % ring])[1] for s, j in burst]
    for tk in tks:
        assert srv.wait(tk)[0] == 0
    cap = len(burst) / (time.perf_counter() - tb)
    log(f"capacity (saturated): {cap:.1f} frames/s")
    srv.close()

    # one 1080p frame of the mix against the oracle
    err = cpu = None
    if not args.no_cpu:
        s1080 = nstreams - 1
        d = dec.upload(frames[s1080][0])
        dec.decode(d, params)
        assert dec.sync() == 0
        ref, cpu = cpu_baseline(frames[s1080][0], min_seconds=args.cpu_seconds,
                                what="one 1080p frame of the serving mix")
        err = error_vs(d["out"].cpu().numpy().astype(np.float64), ref)
    mix_px = sum(w * h * c for w, h, c in synth.SERVING_MIX) / nstreams
    rec = dict(metric=METRIC, value=served_fps, unit="frames/s", n_gpus=1, steps=done_w, warmup=len(tickets) - done_w,
               ms_per_step=1e3 * args.duration / max(done_w, 1), higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f32" if args.eval == "fp32" else f"f32 solve, {args.eval} eval",
               data="synthetic",
               config={"workload": "serving_mix16_420_b16_d1-10", "streams": nstreams,
                       "mix": [list(m) for m in synth.SERVING_MIX], "arrivals": f"Poisson, {rate} frames/s per stream",
                       "offered_fps": rate * nstreams, "lanes": args.lanes, "hbm_budget_mb": args.budget_mb,
                       "measured_s": args.duration, "mean_pixels_per_frame": mix_px},
               latency_ms={"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                           "mean": float(lat.mean()), "max": float(lat.max()),
                           "includes": "host submit, H2D copy, queueing, decode, completion"},
               capacity=dict(value=cap, unit="frames/s", note="all frames submitted at once"),
               error_vs_oracle=err, roofline=None, cpu_baseline=cpu, wall_s=wall)
    dec.close()
    return rec


def nested_legs(args, torch, binding, synth):
    """The other decode workloads of the metric, carried in the default
    config-1 line: config 2 (32x32 blocks; every evaluation dtype against the
    oracle), config 3 (64-frame sequence as HIP-graph replays) and config 4
    (serving mix: p50/p99 latency and capacity), each a full record of its
    own with shorter timing."""
    import copy
    out = {}
    a2 = copy.copy(args)
    a2.config, a2.steps, a2.warmup = 2, min(args.steps, 20), min(args.warmup, 5)
    a2.latency_iters, a2.no_plain, a2.cpu_seconds = 50, True, 3.0
    log("---- nested leg: config 2")
    out["config_2"] = bench_frame(a2, torch, binding, synth)
    a3 = copy.copy(args)
    a3.config, a3.steps, a3.warmup, a3.latency_iters, a3.dtypes = 3, 10, 2, 50, False
    a3.no_cpu = True  # its frames are config-1 frames: checked above
    log("---- nested leg: config 3")
    out["config_3"] = bench_sequence(a3, torch, binding, synth)
    a4 = copy.copy(args)
    a4.config, a4.duration, a4.warm_s, a4.burst_rounds, a4.dtypes = 4, 4.0, 0.5, 4, False
    a4.cpu_seconds = 3.0
    log("---- nested leg: config 4")
    out["config_4"] = bench_serving(a4, torch, binding, synth)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--config", type=int, default=1, choices=[0, 1, 2, 3, 4, 5, 6, 7, 8])
    ap.add_argument("--eval", default="fp32", choices=sorted(EVALS))
    ap.add_argument("--latency-iters", type=int, default=300)
    ap.add_argument("--nstreams", type=int, default=4, help="streams for overlapped / sequence decodes")
    ap.add_argument("--batch", type=int, default=32, help="frames per decode_residual_batch step (1 to 32)")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1), help="frame generator processes")
    ap.add_argument("--lanes", type=int, default=4, help="serving: GPU streams of the request loop")
    ap.add_argument("--budget-mb", type=int, default=2048, help="serving: HBM budget of admitted frames")
    ap.add_argument("--fps-per-stream", type=float, default=25.0)
    ap.add_argument("--duration", type=float, default=10.0, help="serving: measured seconds")
    ap.add_argument("--warm-s", type=float, default=1.0, help="serving: unmeasured seconds first")
    ap.add_argument("--serve-frames", type=int, default=4, help="serving: distinct frames per client stream")
    ap.add_argument("--burst-rounds", type=int, default=8)
    ap.add_argument("--intra-planes", type=int, default=8, help="config 6: distinct planes the steps cycle through")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run a device copy of this many MiB 10 times (HBM counter calibration)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-path comparison")
    ap.add_argument("--no-nested", action="store_true",
                    help="config 1: skip the nested config 2 / 3 / 4 legs (profiling runs)")
    ap.add_argument("--no-dtypes", dest="dtypes", action="store_false",
                    help="configs 0-2: skip the per-dtype sweep")
    ap.add_argument("--dtype-steps", type=int, default=20, help="steps per dtype in the sweep")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="oracle timing sample (seconds)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this decoder runs on one GPU; --gpus {args.gpus} is not supported "
              "(blocks and frames shard across GPUs with no exchange step)", file=sys.stderr)
        sys.exit(2)
    if args.steps is None:
        args.steps = {3: 30, 6: 50, 8: 100}.get(args.config, 500)
    if args.warmup is None:
        args.warmup = {3: 3, 6: 3, 8: 5}.get(args.config, 50)

    from paper_2008_10273_amd import synth
    # frames are generated before torch touches the GPU (worker processes)
    import torch
    from paper_2008_10273_amd import binding
    if args.copy_mib:
        gbs = copy_bandwidth(torch, args.copy_mib, reps=10)
        print(json.dumps({"copy_mib": args.copy_mib, "reps": 10, "GBs": gbs}), flush=True)
        return
    if args.config <= 2:
        rec = bench_frame(args, torch, binding, synth)
        if args.config == 1 and not args.no_nested:
            rec.update(nested_legs(args, torch, binding, synth))
    elif args.config == 3:
        rec = bench_sequence(args, torch, binding, synth)
    elif args.config == 5:
        rec = bench_coef(args, torch, binding, synth)
    elif args.config == 6:
        rec = bench_intra(args, torch, binding, synth)
    elif args.config == 7:
        rec = bench_encode(args, torch, binding, synth)
    elif args.config == 8:
        rec = bench_select(args, torch, binding, synth)
    else:
        rec = bench_serving(args, torch, binding, synth)
    assert torch.cuda.is_available()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
