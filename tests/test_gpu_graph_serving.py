"""Sequence graphs, concurrent streams and the serving loop on the GPU.

Results of the same decode are compared bitwise: the decode of a frame is
one fixed sequence of kernels whose arithmetic does not depend on the stream,
on what runs beside it or on graph capture, so replays and the serving mix
must reproduce the eager result exactly.  One frame of each kind is also
checked against the oracle.
"""
import numpy as np
import pytest

import oracle
from paper_2008_10273_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dec():
    from paper_2008_10273_amd import binding
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = binding.Decoder(0)
    yield d
    d.close()


def _eager(dec, fr, params=None):
    d = dec.upload(fr)
    dec.decode(d, params)
    assert dec.sync() == 0
    return d["out"].cpu().numpy()


def _oracle_ok(fr, got):
    ref = oracle.decode_flat(fr)
    err = np.abs(got.astype(np.float64) - ref)
    q = lambda x: np.clip(np.rint(x), -128, 127)
    agree = float(np.mean(q(got.astype(np.float64)) == q(ref)))
    print(f"  oracle: max|err|={err.max():.3e} agree={agree * 100:.4f}%", flush=True)
    assert err.max() <= 1e-2 and agree >= 0.999


def _seq_frames(n, W=320, H=184, b=16):
    return [synth.random_frame(W, H, synth.YUV420, b, (0.01, 0.1), seed=900 + k) for k in range(n)]


@pytest.mark.parametrize("b,nstreams", [(16, 3), (32, 2), (8, 1)])
def test_sequence_graph_replays_match_eager(dec, b, nstreams):
    from paper_2008_10273_amd import binding
    print(f"case seq b={b} nstreams={nstreams}", flush=True)
    frames = _seq_frames(6, b=b)
    ref = [_eager(dec, f) for f in frames]
    _oracle_ok(frames[0], ref[0])
    ds = [dec.upload(f) for f in frames]
    seq = binding.Sequence(dec, ds, nstreams=nstreams)
    other = dec.upload(synth.random_frame(200, 120, synth.YUV420, 16, (0.01, 0.2), seed=5))
    for rep in range(3):
        for d in ds:
            d["out"].zero_()
        assert seq.launch() == 0
        assert seq.sync() == 0
        for k, d in enumerate(ds):
            np.testing.assert_array_equal(d["out"].cpu().numpy(), ref[k], err_msg=f"replay {rep} frame {k}")
        # eager work between replays, on the same context and stream
        dec.decode(other)
        assert dec.sync() == 0
    # new contents at the same addresses are picked up by the next replay
    vals = np.ascontiguousarray(frames[0].values * -0.5, np.float32)
    ds[0]["values"].copy_(torch.from_numpy(vals))
    assert seq.launch() == 0 and seq.sync() == 0
    fr2 = synth.Frame(**{**frames[0].__dict__, "values": vals})
    np.testing.assert_array_equal(ds[0]["out"].cpu().numpy(), _eager(dec, fr2))
    seq.close()


def test_concurrent_streams_match_sequential(dec):
    """Decodes on several streams at once (per-stream workspaces) give the
    results of the same decodes one after another."""
    frames = [synth.random_frame(400 + 16 * k, 240 + 8 * k, synth.YUV420, 16, (0.01, 0.1), seed=40 + k)
              for k in range(4)] + [synth.random_frame(257, 130, synth.YUV420, 32, (0.02, 0.1), seed=49)]
    ref = [_eager(dec, f) for f in frames]
    ds = [dec.upload(f) for f in frames]
    streams = [torch.cuda.Stream() for _ in ds]
    torch.cuda.synchronize()
    for rep in range(3):
        for d, s in zip(ds, streams):
            d["out"].zero_()
        torch.cuda.synchronize()
        for d, s in zip(ds, streams):
            dec.decode(d, stream=s)
        for d, s, r in zip(ds, streams, ref):
            assert dec.sync(s) == 0
            np.testing.assert_array_equal(d["out"].cpu().numpy(), r)


def test_concurrent_batched_b32_streams(dec):
    """Batched 32x32-block decodes on three streams at once: each batch runs
    its four wave-per-block parts side by side on the context's streams
    (shared by the three callers); every frame equals its decode alone."""
    print("case concurrent b32 batches on 3 streams", flush=True)
    groups = [[synth.random_frame(290, 170, synth.YUV420, 32, (0.02, 0.1), seed=4100 + 10 * g + k)
               for k in range(5)] for g in range(3)]
    ref = [[_eager(dec, f) for f in grp] for grp in groups]
    dss = [[dec.upload(f) for f in grp] for grp in groups]
    streams = [torch.cuda.Stream() for _ in groups]
    for rep in range(2):
        for ds in dss:
            for d in ds:
                d["out"].zero_()
        torch.cuda.synchronize()
        for ds, st in zip(dss, streams):
            dec.decode_batch(ds, stream=st)
        for ds, st, rs in zip(dss, streams, ref):
            assert dec.sync(st) == 0
            for k, (d, r) in enumerate(zip(ds, rs)):
                np.testing.assert_array_equal(d["out"].cpu().numpy(), r, err_msg=f"rep {rep} frame {k}")


def test_serving_alone_equals_mix(dec):
    """Each frame of the 16-stream serving mix (6x 480p, 6x 720p, 4x 1080p,
    4:2:0, b16) decodes to the same result alone as inside the mix."""
    from paper_2008_10273_amd import binding
    frames = [synth.serving_frame(s, f) for f in range(2) for s in range(16)]
    alone = [_eager(dec, fr) for fr in frames]
    _oracle_ok(frames[0], alone[0])
    srv = binding.Server(dec, nlanes=4)
    # odd frames decode into caller-owned device buffers, even ones to host
    devs = [torch.empty(fr.out_size, dtype=torch.float32, device="cuda") if k % 2 else None
            for k, fr in enumerate(frames)]
    subs = [srv.submit(fr, want_output=dv is None, out_dev=dv) for fr, dv in zip(frames, devs)]
    for (rc, t, out), ref, fr, dv in zip(subs, alone, frames, devs):
        assert rc == 0
        st, lat = srv.wait(t)
        assert st == 0 and lat > 0
        got = out if dv is None else dv.cpu().numpy()
        np.testing.assert_array_equal(got, ref, err_msg=f"{fr.width}x{fr.height}")
    s = srv.stats()
    assert s["queued"] == 0 and s["running"] == 0 and s["bytes_in_use"] == 0
    srv.close()


def test_serving_b32_batches_equal_alone(dec):
    """32x32-block frames through the serving loop (lanes join queued frames
    of one geometry into batches, whose wave-per-block parts run on the
    context's extra streams): every frame equals its decode alone."""
    from paper_2008_10273_amd import binding
    print("case serving b32", flush=True)
    frames = [synth.random_frame(290, 170, synth.YUV420, 32, (0.02, 0.1), seed=4300 + k) for k in range(12)]
    alone = [_eager(dec, fr) for fr in frames]
    srv = binding.Server(dec, nlanes=2)
    assert srv.hold(True) == 0  # queue everything first, so that the lanes form batches
    subs = [srv.submit(fr) for fr in frames]
    assert srv.hold(False) == 0
    for (rc, t, out), ref in zip(subs, alone):
        assert rc == 0
        assert srv.wait(t)[0] == 0
        np.testing.assert_array_equal(out, ref)
    srv.close()


def test_serving_budget_admission_and_busy(dec):
    """A budget that fits about one 1080p frame still completes every
    request; a full queue answers PDI_EBUSY; bad masks are refused at
    submit with validation on."""
    from paper_2008_10273_amd import binding
    frames = [synth.serving_frame(s, 3) for s in (0, 6, 12, 13, 1, 7)]
    alone = [_eager(dec, fr) for fr in frames]
    budget = 48 << 20
    srv = binding.Server(dec, nlanes=3, hbm_budget_bytes=budget, max_queue=64)
    subs = [srv.submit(fr) for fr in frames]
    peak = 0
    for (rc, t, out), ref in zip(subs, alone):
        assert rc == 0
        while True:
            peak = max(peak, srv.stats()["bytes_in_use"])
            rcp, done, _ = srv.poll(t)
            if done:
                break
        assert srv.wait(t)[0] == 0
        np.testing.assert_array_equal(out, ref)
    assert 0 < peak <= budget
    srv.close()

    srv = binding.Server(dec, nlanes=1, max_queue=2)
    assert srv.hold(True) == 0
    big = synth.serving_frame(12, 0)
    rcs = [srv.submit(big) for _ in range(3)]
    assert [r[0] for r in rcs] == [0, 0, binding.PDI_EBUSY]
    assert srv.stats()["queued"] == 2 and srv.stats()["running"] == 0
    assert srv.hold(False) == 0
    ref = _eager(dec, big)
    for rc, t, out in rcs[:2]:
        assert srv.wait(t)[0] == 0
        np.testing.assert_array_equal(out, ref)
    bad = synth.serving_frame(0, 0)
    bad.pos = bad.pos.copy()
    bad.pos[1] = bad.pos[0]  # duplicate inside block 0 (K >= 3 there)
    rc, _, _ = srv.submit(bad, binding.default_params(validate=1))
    assert rc == binding.PDI_EMASK
    srv.close()


@pytest.mark.parametrize("b,path,i8", [(16, 0, 0), (32, 0, 0), (8, 0, 0), (16, 1, 0), (32, 1, 0), (16, 0, 1)])
def test_batch_equals_single(dec, b, path, i8):
    """decode_residual_batch over 1..32 frames equals decoding each frame alone,
    bitwise, including blocks left to the general path (K = 0, K = w*h,
    large K) in every frame of the batch."""
    from paper_2008_10273_amd import binding
    print(f"case batch b={b} path={path} int8={i8}", flush=True)
    params = binding.default_params(path=path, out_int8=i8)
    frames = [synth.random_frame(260, 150, synth.YUV420, b, (0.01, 0.12), seed=600 + k) for k in range(7)]
    # a frame with degenerate and large point counts
    W, H = 260, 150
    rng = np.random.default_rng(5)
    ms, fs = [], []
    for (pw, ph) in synth.plane_dims(W, H, synth.YUV420)[:2]:
        m = rng.uniform(size=(ph, pw)) < 0.08
        m[:b, :b] = False                      # K = 0
        m[:b, b:2 * b] = True                  # K = w*h
        m[b:2 * b, :b] = rng.uniform(size=(b, b)) < 0.6   # large K
        ms.append(m)
        fs.append(rng.uniform(-64, 64, (ph, pw)))
    fs.append(rng.uniform(-64, 64, fs[1].shape))
    frames.append(synth.pack_dense(W, H, synth.YUV420, b, ms, fs))
    key = "out_i8" if i8 else "out"
    alone = []
    for fr in frames:
        d = dec.upload(fr)
        dec.decode(d, params)
        assert dec.sync() == 0
        alone.append(d[key].cpu().numpy())
    for n in (1, 3, 8, 32):
        ds = [dec.upload(fr) for fr in (frames * 4)[-n:]]
        for d in ds:
            d[key].zero_()
        dec.decode_batch(ds, params)
        assert dec.sync() == 0
        for d, ref in zip(ds, (alone * 4)[-n:]):
            np.testing.assert_array_equal(d[key].cpu().numpy(), ref)
    ds = [dec.upload(frames[0]) for _ in range(33)]
    assert dec.decode_batch(ds, params, check=False) == binding.PDI_EINVAL
