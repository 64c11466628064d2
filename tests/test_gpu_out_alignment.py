"""Output planes whose base address is not 16-byte aligned (FP32 shifted by
one element, int8 by one byte): the evaluations store four pixels at a time
only where the address allows it, so every path must write the same planes
as into an aligned buffer, bitwise.  Paths: single frames (b = 8, 16, 32),
a binned batch (b = 16, at least 32768 mask blocks) and a batch of 32 x 32
blocks (the k_wide parts); stored-coefficient decodes alike."""
import numpy as np
import pytest

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


def _shifted(t, shift):
    """A view of t's shape that starts `shift` elements into a larger buffer."""
    buf = torch.zeros(t.numel() + shift, dtype=t.dtype, device=t.device)
    return buf[shift:]


def _decode(dec, ds, params, key, shift):
    outs = []
    for d in ds:
        d[key] = _shifted(d[key], shift) if shift else torch.zeros_like(d[key])
        assert shift == 0 or d[key].data_ptr() % 16 != 0
    if len(ds) == 1:
        dec.decode(ds[0], params)
    else:
        dec.decode_batch(ds, params)
    assert dec.sync() == 0
    for d in ds:
        outs.append(d[key].cpu().numpy())
    return outs


CASES = {
    "single_b16": (650, 490, 16, 1, (0.01, 0.12)),
    "single_b8": (330, 250, 8, 1, (0.02, 0.3)),
    "single_b32": (150, 90, 32, 1, (0.02, 0.1)),
    "binned_b16": (650, 490, 16, 24, (0.01, 0.12)),
    "batch_b32": (290, 170, 32, 6, (0.02, 0.1)),
}


@pytest.mark.parametrize("i8", [0, 1])
@pytest.mark.parametrize("case", sorted(CASES))
def test_unaligned_output_planes(dec, case, i8):
    from paper_2008_10273_amd import binding
    W, H, b, n, dens = CASES[case]
    print(f"case {case} {W}x{H} b={b} n={n} int8={i8}", flush=True)
    frames = [synth.random_frame(W, H, synth.YUV420, b, dens, seed=8100 + 10 * b + k) for k in range(n)]
    params = binding.default_params(out_int8=i8)
    key = "out_i8" if i8 else "out"
    ref = _decode(dec, [dec.upload(fr) for fr in frames], params, key, 0)
    got = _decode(dec, [dec.upload(fr) for fr in frames], params, key, 1)
    for k, (g, r) in enumerate(zip(got, ref)):
        np.testing.assert_array_equal(g, r, err_msg=f"frame {k}")


@pytest.mark.parametrize("i8", [0, 1])
@pytest.mark.parametrize("b,W,H,n", [(8, 330, 250, 4), (32, 150, 90, 1)])
def test_unaligned_output_planes_coef(dec, b, W, H, n, i8):
    """The stored-coefficient decoder, single frame or batch, into shifted planes."""
    from paper_2008_10273_amd import binding
    print(f"case coef b={b} {W}x{H} n={n} int8={i8}", flush=True)
    frames = [synth.random_frame(W, H, synth.YUV420, b, (0.02, 0.2), seed=8200 + 10 * b + k) for k in range(n)]
    inputs = [synth.coef_inputs(fr, 20 + k) for k, fr in enumerate(frames)]
    qp = binding.coef_params((0.25, 0.5, 0.375), 0.5)
    params = binding.default_params(out_int8=i8)
    key = "out_i8" if i8 else "out"
    res = []
    for shift in (0, 1):
        ds = [dec.upload_coef(fr, q, c) for fr, (q, c) in zip(frames, inputs)]
        for d in ds:
            d[key] = _shifted(d[key], shift) if shift else torch.zeros_like(d[key])
        if n == 1:
            dec.decode_coef(ds[0], qp, params)
        else:
            dec.decode_coef_batch(ds, qp, params)
        assert dec.sync() == 0
        res.append([d[key].cpu().numpy() for d in ds])
    for k, (g, r) in enumerate(zip(res[1], res[0])):
        np.testing.assert_array_equal(g, r, err_msg=f"frame {k}")
