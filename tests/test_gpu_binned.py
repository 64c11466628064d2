"""The binned wave-level path on the GPU: batched residual decodes with 8x8 or
16x16 blocks and at least 32768 mask blocks in the launch go through the
three binning passes and k_fast2 (blocks grouped by plane segment and exact
system size).  Its block arithmetic is that of the single-frame kernel, so
every frame of such a batch must equal the same frame decoded alone,
bitwise; a few frames are also checked against the FP64 oracle.  Frames
have ragged edges, densities from 1 % to 12 % (every size class, and blocks
past the wave-level path), and one frame with K = 0, K = w*h and large-K
blocks."""
import numpy as np
import pytest

import oracle
from paper_2008_10273_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP32_TOL = 1e-2
BINNED_MIN_BLOCKS = 32768  # batches with at least this many mask blocks are binned


@pytest.fixture(scope="module")
def dec():
    from paper_2008_10273_amd import binding
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = binding.Decoder(0)
    yield d
    d.close()


def _mask_blocks(W, H, b):
    y, cb, _ = synth.plane_block_counts(W, H, synth.YUV420, b)
    return y + cb  # one shared chroma mask


def _frames(W, H, b, n, seed):
    frames = [synth.random_frame(W, H, synth.YUV420, b, (0.01, 0.12), seed=seed + k) for k in range(n - 1)]
    rng = np.random.default_rng(seed)
    ms, fs = [], []
    for (pw, ph) in synth.plane_dims(W, H, synth.YUV420)[:2]:
        m = rng.uniform(size=(ph, pw)) < 0.06
        m[:b, :b] = False                                    # K = 0
        m[:b, b:2 * b] = True                                # K = w*h
        m[b:2 * b, :b] = rng.uniform(size=(b, b)) < 0.6     # K past the wave-level path
        m[b:2 * b, b:2 * b] = rng.uniform(size=(b, b)) < 0.11  # around the largest class
        ms.append(m)
        fs.append(rng.uniform(-64, 64, (ph, pw)))
    fs.append(rng.uniform(-64, 64, fs[1].shape))
    frames.insert(n // 2, synth.pack_dense(W, H, synth.YUV420, b, ms, fs))
    return frames


@pytest.mark.parametrize("b,W,H,n,ev,i8", [(16, 650, 490, 24, 0, 0), (16, 650, 490, 24, 1, 0),
                                          (16, 650, 490, 24, 0, 1), (8, 330, 250, 24, 0, 0)])
def test_binned_batch_equals_single(dec, b, W, H, n, ev, i8):
    from paper_2008_10273_amd import binding
    print(f"case binned b={b} {W}x{H} n={n} eval={ev} int8={i8}", flush=True)
    assert _mask_blocks(W, H, b) * n >= BINNED_MIN_BLOCKS
    params = binding.default_params(eval_dtype=ev, out_int8=i8)
    key = "out_i8" if i8 else "out"
    frames = _frames(W, H, b, n, seed=7000 + 10 * b + ev)
    alone = []
    for fr in frames:
        d = dec.upload(fr)
        dec.decode(d, params)
        assert dec.sync() == 0
        alone.append(d[key].cpu().numpy())
    ds = [dec.upload(fr) for fr in frames]
    for d in ds:
        d[key].zero_()
    dec.decode_batch(ds, params)
    assert dec.sync() == 0
    for k, (d, ref) in enumerate(zip(ds, alone)):
        np.testing.assert_array_equal(d[key].cpu().numpy(), ref, err_msg=f"frame {k}")
    if ev == 0 and not i8:
        for k in (0, n // 2, n - 1):
            err = np.abs(alone[k].astype(np.float64) - oracle.decode_flat(frames[k])).max()
            assert err <= FP32_TOL, (k, err)


def test_binned_batch_validation(dec):
    """A batch whose frame n/2 repeats a position inside a block: the binned
    decode with validation reports PDI_EMASK, and the next batch decodes."""
    from paper_2008_10273_amd import binding
    W, H, b, n = 650, 490, 16, 24
    frames = [synth.random_frame(W, H, synth.YUV420, b, (0.02, 0.1), seed=7500 + k) for k in range(n)]
    bad = frames[n // 2]
    bad.pos = bad.pos.copy()
    cnt = np.diff(bad.block_ptr)
    k = int(np.argmax((cnt >= 3) & (cnt <= 31)))  # a block of the wave-level path with 3 points or more
    bad.pos[bad.block_ptr[k] + 1] = bad.pos[bad.block_ptr[k]]
    print("case binned validation", flush=True)
    ds = [dec.upload(fr) for fr in frames]
    assert dec.decode_batch(ds, binding.default_params(validate=1), check=False) == binding.PDI_OK
    assert dec.sync() == binding.PDI_EMASK
    good = [dec.upload(synth.random_frame(W, H, synth.YUV420, b, (0.02, 0.1), seed=7600 + k)) for k in range(n)]
    dec.decode_batch(good, binding.default_params(validate=1))
    assert dec.sync() == 0


def test_binned_many_count_workgroups(dec):
    """32 gray 1032x1024 frames with 8x8 blocks: 65 counting workgroups per
    frame, 2080 in all, more than the per-bin scan takes in one round (8
    counts per thread), so the scan goes round by round.  Every frame must
    equal the same frame decoded alone, bitwise."""
    from paper_2008_10273_amd import binding
    W, H, b, n = 1032, 1024, 8, 32
    nblk = synth.plane_block_counts(W, H, synth.GRAY, b)[0]
    assert ((nblk + 255) // 256) * n > 8 * 256 and nblk * n >= BINNED_MIN_BLOCKS
    print(f"case binned b={b} {W}x{H} n={n} (scan rounds)", flush=True)
    frames = [synth.random_frame(W, H, synth.GRAY, b, (0.02, 0.3), seed=7800 + k) for k in range(4)]
    params = binding.default_params()
    alone = []
    for fr in frames:
        d = dec.upload(fr)
        dec.decode(d, params)
        assert dec.sync() == 0
        alone.append(d["out"].cpu().numpy())
    ds = [dec.upload(frames[k % 4]) for k in range(n)]
    for d in ds:
        d["out"].zero_()
    dec.decode_batch(ds, params)
    assert dec.sync() == 0
    for k, d in enumerate(ds):
        np.testing.assert_array_equal(d["out"].cpu().numpy(), alone[k % 4], err_msg=f"frame {k}")
