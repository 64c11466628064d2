"""decode_residual_batch_noalloc: the residual decode with its device scratch
in the library's static device array (nothing allocated), called through
the C ABI and compared with decode_residual_batch, the allocating entry
point, on the same frames: calls in a row, each with a smaller input (a
batch large enough for the binned path, then fewer frames, then another
block size).  The two entry points run the same
kernels with the same arithmetic, so results must be bitwise equal; the
first four frames of each call are also within FP32_TOL of the FP64 oracle
(the parity bar of the decoder).
Densities up to 45 % put blocks past the wave-level path (K > 31) and past
the LDS-sized systems (K > 96, global-memory systems in the scratch)."""
import numpy as np
import pytest

import oracle
from paper_2008_10273_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP32_TOL = 1e-2


@pytest.fixture(scope="module")
def dec():
    from paper_2008_10273_amd import binding
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = binding.Decoder(0)
    yield d
    d.close()


def _host(ds):
    return [d["out"].cpu().numpy().copy() for d in ds]


def test_noalloc_matches_batch_two_calls(dec):
    cases = [(650, 490, 16, 24, (0.01, 0.12), 400),  # 38568 mask blocks: the binned path, its entries in the scratch
             (300, 170, 16, 4, (0.01, 0.45), 500),   # K up to 115: all three paths of b = 16
             (100, 60, 32, 2, (0.02, 0.12), 600)]     # smaller: wave-per-block path, queues in the scratch
    for W, H, b, n, dens, seed in cases:
        print(f"case noalloc {W}x{H} 4:2:0 b{b} n={n} density {dens}", flush=True)
        frames = [synth.random_frame(W, H, synth.YUV420, b, dens, seed=seed + k) for k in range(n)]
        ds = [dec.upload(f) for f in frames]
        dec.decode_batch(ds)          # the allocating entry point (builds the tables)
        assert dec.sync() == 0
        ref = _host(ds)
        for d in ds:
            d["out"].fill_(float("nan"))
        dec.decode_batch_noalloc(ds)  # the static-scratch entry point
        assert dec.sync() == 0
        got = _host(ds)
        for k, fr in enumerate(frames):
            np.testing.assert_array_equal(got[k], ref[k])
            if k < 4:
                err = np.abs(got[k].astype(np.float64) - oracle.decode_flat(fr)).max()
                assert err <= FP32_TOL, (k, err)


def test_noalloc_limits(dec):
    """No tables yet for a geometry: PDI_EINVAL and nothing launched.  A
    decode whose scratch exceeds the static array (32 frames of a 4096x4096
    grey plane with 8x8 blocks: 33.6 MB of deferred-list entries alone):
    PDI_ENOMEM and nothing launched; one such frame fits and matches."""
    from paper_2008_10273_amd import binding
    fr = synth.random_frame(132, 68, synth.GRAY, 8, (0.02, 0.2), seed=7)
    d = dec.upload(fr)
    assert dec.decode_batch_noalloc([d], check=False) == binding.PDI_EINVAL
    big = synth.random_frame(4096, 4096, synth.GRAY, 8, (0.01, 0.05), seed=8)
    print("case noalloc 4096x4096 grey b8", flush=True)
    db = dec.upload(big)
    dec.decode_batch([db])
    assert dec.sync() == 0
    ref = db["out"].cpu().numpy().copy()
    assert dec.decode_batch_noalloc([db] * 32, check=False) == binding.PDI_ENOMEM
    db["out"].fill_(float("nan"))
    dec.decode_batch_noalloc([db])
    assert dec.sync() == 0
    np.testing.assert_array_equal(db["out"].cpu().numpy(), ref)
