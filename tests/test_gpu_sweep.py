"""Seeded sweep over small random geometries (sizes 1..90, grey and 4:2:0,
shared and separate chroma masks, 8x8 / 16x16 / 32x32 blocks, densities up
to 60 %, 30 % for 32x32 blocks): the residual decoder, the coefficient encoder and the mask
selection against the FP64 oracle, with the bars of the dedicated tests
(FP32_TOL for pixels and constants; codes equal away from interval edges;
masks equal away from threshold decisions).  Every input is valid."""
import numpy as np
import pytest

import oracle
import test_gpu_select
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


def _geometries(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        W, H = int(rng.integers(1, 91)), int(rng.integers(1, 91))
        fmt = int(rng.integers(0, 2))
        b = int(rng.choice([8, 16, 32]))
        lo = float(rng.uniform(0.0, 0.3))
        hi = min(0.6 if b < 32 else 0.3, lo + float(rng.uniform(0.01, 0.3)))  # b = 32: K <= ~300
        shared = bool(rng.integers(0, 2))
        out.append((W, H, fmt, b, (lo, hi), shared, 1000 + k))
    return out


@pytest.mark.parametrize("W,H,fmt,b,dens,shared,seed", _geometries(24, 7))
def test_sweep_decode_and_encode(dec, W, H, fmt, b, dens, shared, seed):
    from paper_2008_10273_amd import binding
    fr = synth.random_frame(W, H, fmt, b, dens, seed=seed, chroma_shared=shared)
    print(f"case sweep {W}x{H} fmt={fmt} b={b} dens={dens} shared={shared}", flush=True)
    d = dec.upload(fr)
    dec.decode(d)
    assert dec.sync() == 0
    got = d["out"].cpu().numpy().astype(np.float64)
    ref = oracle.decode_flat(fr)
    assert np.abs(got - ref).max() <= FP32_TOL
    steps = (0.5, 0.5, 0.5)
    d = dec.alloc_coef(d)
    dec.encode_coef(d, binding.coef_params(steps, 0.5))
    assert dec.sync() == 0
    a = d["consts"].cpu().numpy().astype(np.float64)
    q = d["coef"].cpu().numpy()[:fr.values.size].astype(np.int64)
    qo, cex, ao = oracle.encode_coef(fr, steps)
    assert np.abs(a - ao).max() <= FP32_TOL
    x = np.abs(cex) / 0.5
    near = np.abs(x - np.rint(x)) * 0.5 <= FP32_TOL
    assert np.all(np.abs(q - qo) <= 1) and not np.any((q != qo) & ~near)


@pytest.mark.parametrize("W,H,fmt,b,dens,shared,seed", _geometries(12, 8))
def test_sweep_select(dec, W, H, fmt, b, dens, shared, seed):
    from paper_2008_10273_amd import binding
    planes = synth.residual_planes(W, H, fmt, seed)
    T = (16.0, 32.0)
    print(f"case sweep select {W}x{H} fmt={fmt} shared={shared}", flush=True)
    rc, d = dec.select(W, H, fmt, planes, shared, binding.select_params(*T))
    assert dec.sync() == 0
    # every block whose mask differs from the oracle's must equal the
    # oracle's mask at a slightly shifted threshold (a decision within FP32
    # reach of the threshold), as in the dedicated selection tests
    masks, gathered = test_gpu_select._host_masks(d, W, H, fmt, shared)
    test_gpu_select._compare(planes, W, H, fmt, shared, T, masks, max_frac=0.02)
    groups = [[0]] if fmt == synth.GRAY else ([[0], [1, 2]] if shared else [[0], [1], [2]])
    for gi, gp in enumerate(groups):
        for pl in gp:
            assert np.array_equal(gathered[gi][pl][masks[gi]], planes[pl][masks[gi]])
