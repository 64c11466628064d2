"""Parity of per-block mask selection by rectangular subdivision
(select_mask, through the C ABI) with the FP64 oracle, and the selected
masks fed to the decoder and the coefficient encoder.

Bars.  The masks are integer results decided by floating point (a
rectangle's mean squared error against the threshold; FP32 on the GPU,
FP64 in the oracle).  Every block's mask must equal the oracle's, except
where a decision lies within FP32 reach of the threshold: such a block must
equal the oracle's mask with the threshold moved by a relative 1e-3 up or
down (the decision flipped), and those blocks must be few.  The gathered
values at the mask points are copies, so they are compared bit for bit.
"""
import numpy as np
import pytest

import oracle
from paper_2008_10273_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP32_TOL = 1e-2
DELTA = 1e-3


@pytest.fixture(scope="module")
def dec():
    from paper_2008_10273_amd import binding
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = binding.Decoder(0)
    yield d
    d.close()


def _host_masks(d, W, H, fmt, shared):
    """Dense masks and the values gathered per mask plane from the packed
    output, walking the documented layout."""
    bp = d["block_ptr"].cpu().numpy().astype(np.int64)
    pos = d["pos"].cpu().numpy().view(np.uint16).astype(np.int64)
    vals = d["values"].cpu().numpy()
    dims = synth.plane_dims(W, H, fmt)
    groups = [[0]] if fmt == synth.GRAY else ([[0], [1, 2]] if shared else [[0], [1], [2]])
    masks, gathered = [], []
    m = 0
    nnz = bp[-1]
    chroma_first = None
    for gp in groups:
        pw, ph = dims[gp[0]]
        if gp[0] == 1:
            chroma_first = m
        mk = np.zeros((ph, pw), bool)
        got = {pl: np.zeros((ph, pw), np.float32) for pl in gp}
        for (x0, y0, w, h) in synth.block_grid(pw, ph, 8):
            lo, hi = bp[m], bp[m + 1]
            p = pos[lo:hi]
            assert np.all(np.diff(p) > 0) and (p.size == 0 or p.max() < w * h)
            ys, xs = y0 + p // w, x0 + p % w
            mk[ys, xs] = True
            for k, pl in enumerate(gp):
                vb = nnz + (lo - bp[chroma_first]) if (k == 1) else lo
                got[pl][ys, xs] = vals[vb:vb + (hi - lo)]
            m += 1
        masks.append(mk)
        gathered.append(got)
    assert m == bp.size - 1
    return masks, gathered


def _block_planes(planes, fmt, gp, x0, y0, w, h):
    return [planes[pl][y0:y0 + h, x0:x0 + w] for pl in gp]


def _oracle_block(planes_b, w, h, T, two):
    """The oracle's selection on one block (two value planes: a 4:2:0 frame
    whose chroma planes are the block, its luma ignored)."""
    if not two:
        return oracle.select_mask(w, h, synth.GRAY, 8, planes_b, True, (T, T))[0]
    Y = np.zeros((2 * h, 2 * w))
    return oracle.select_mask(2 * w, 2 * h, synth.YUV420, 8, [Y] + planes_b, True, (1e300, T))[1]


def _compare(planes, W, H, fmt, shared, thr, got_masks, max_frac=0.01):
    ref = oracle.select_mask(W, H, fmt, 8, planes, shared, thr)
    dims = synth.plane_dims(W, H, fmt)
    groups = [[0]] if fmt == synth.GRAY else ([[0], [1, 2]] if shared else [[0], [1], [2]])
    nblocks = nflip = 0
    for gi, gp in enumerate(groups):
        pw, ph = dims[gp[0]]
        T = thr[0] if gi == 0 else thr[1]
        for (x0, y0, w, h) in synth.block_grid(pw, ph, 8):
            nblocks += 1
            g = got_masks[gi][y0:y0 + h, x0:x0 + w]
            r = ref[gi][y0:y0 + h, x0:x0 + w]
            if np.array_equal(g, r):
                continue
            nflip += 1
            pb = _block_planes(planes, fmt, gp, x0, y0, w, h)
            alts = [_oracle_block(pb, w, h, T * (1 + s * DELTA), len(gp) == 2) for s in (1, -1)]
            assert any(np.array_equal(g, a) for a in alts), (gi, x0, y0)
    print(f"  {nflip} of {nblocks} blocks decided differently within FP32 reach of the threshold", flush=True)
    assert nflip <= max(2, max_frac * nblocks)


@pytest.mark.parametrize("W,H,fmt,shared,thr", [
    (64, 48, synth.YUV420, True, (16.0, 32.0)),
    (61, 37, synth.YUV420, True, (8.0, 16.0)),      # ragged edge blocks
    (61, 37, synth.YUV420, False, (16.0, 32.0)),    # separate chroma masks
    (45, 27, synth.GRAY, True, (4.0, 4.0)),
    (160, 96, synth.YUV420, True, (30.0, 60.0)),
])
def test_select_parity(dec, W, H, fmt, shared, thr):
    from paper_2008_10273_amd import binding
    planes = synth.residual_planes(W, H, fmt, W * H)
    print(f"case select {W}x{H} fmt={fmt} shared={shared} thr={thr}", flush=True)
    rc, d = dec.select(W, H, fmt, planes, shared, binding.select_params(*thr))
    assert dec.sync() == 0
    masks, gathered = _host_masks(d, W, H, fmt, shared)
    _compare(planes, W, H, fmt, shared, thr, masks)
    # values at the mask points are the residual there, bit for bit
    groups = [[0]] if fmt == synth.GRAY else ([[0], [1, 2]] if shared else [[0], [1], [2]])
    for gi, gp in enumerate(groups):
        for pl in gp:
            mk = masks[gi]
            assert np.array_equal(gathered[gi][pl][mk], planes[pl][mk])


def test_select_limits(dec):
    """No split: exactly the corners of every block; always split: every
    pixel; zero rounds: the corners."""
    from paper_2008_10273_amd import binding
    W, H = 45, 27
    planes = synth.residual_planes(W, H, synth.YUV420, 5)
    dims = synth.plane_dims(W, H, synth.YUV420)
    print("case select limits", flush=True)
    for sp, kind in ((binding.select_params(1e30, 1e30), "corners"), (binding.select_params(-1.0, -1.0), "all"),
                     (binding.select_params(-1.0, -1.0, 0), "corners")):
        rc, d = dec.select(W, H, synth.YUV420, planes, True, sp)
        assert dec.sync() == 0
        masks, _ = _host_masks(d, W, H, synth.YUV420, True)
        for m, (pw, ph) in zip(masks, dims):
            if kind == "all":
                assert m.all()
            else:
                want = np.zeros((ph, pw), bool)
                for (x0, y0, w, h) in synth.block_grid(pw, ph, 8):
                    for x in (x0, x0 + w - 1):
                        for y in (y0, y0 + h - 1):
                            want[y, x] = True
                assert np.array_equal(m, want)


def _frame_from(d, W, H, fmt, shared):
    bp = d["block_ptr"].cpu().numpy().astype(np.int32)
    nnz = int(bp[-1])
    nvals = nnz if fmt == synth.GRAY else (2 * nnz - int(bp[sum(synth.plane_block_counts(W, H, fmt, 8)[:1])])
                                           if shared else nnz)
    pos = d["pos"].cpu().numpy().view(np.uint16)[:nnz]
    vals = d["values"].cpu().numpy()[:nvals]
    return synth.Frame(W, H, fmt, 8, bool(shared), bp, pos.copy(), vals.copy(), None)


def test_select_then_decode_and_encode(dec):
    """The selected mask and values are decoder and encoder inputs: the GPU
    decode of them matches the oracle's decode of the same packed frame, and
    GPU encode + GPU decode of the coefficients stays within the
    quantisation bound of it."""
    from paper_2008_10273_amd import binding
    W, H = 96, 64
    planes = synth.residual_planes(W, H, synth.YUV420, 11)
    print("case select -> decode / encode", flush=True)
    rc, d = dec.select(W, H, synth.YUV420, planes, True, binding.select_params(16.0, 32.0))
    assert dec.sync() == 0
    fr = _frame_from(d, W, H, synth.YUV420, True)
    ref = oracle.decode_flat(fr)
    up = dec.upload(fr)
    dec.decode(up)
    assert dec.sync() == 0
    got = up["out"].cpu().numpy().astype(np.float64)
    assert np.abs(got - ref).max() <= FP32_TOL
    # selected points reproduce the residual exactly at the mask
    cmax = np.abs(oracle.encode_coef(fr, (1.0, 1.0, 1.0))[1]).max()
    step = cmax / 127.0
    up = dec.alloc_coef(up)
    dec.encode_coef(up, binding.coef_params((step, step, step), 0.5))
    dec.decode_coef(up, binding.coef_params((step, step, step), 0.5))
    assert dec.sync() == 0
    got = up["out"].cpu().numpy().astype(np.float64)
    G = oracle.green_matrix(8, 8)
    bound = step * 64 * np.abs(G).max() + FP32_TOL
    assert np.abs(got - ref).max() <= bound


def test_select_full_frame(dec):
    """The selection workload at full size (1920x1080 4:2:0, 8x8 blocks)."""
    from paper_2008_10273_amd import binding
    c = synth.SELECT_CONFIG
    W, H = c["width"], c["height"]
    planes = synth.residual_planes(W, H, c["fmt"], 0)
    print("case select full frame", flush=True)
    rc, d = dec.select(W, H, c["fmt"], planes, True, binding.select_params(*c["threshold"]))
    assert dec.sync() == 0
    masks, _ = _host_masks(d, W, H, c["fmt"], True)
    _compare(planes, W, H, c["fmt"], True, c["threshold"], masks, max_frac=0.001)


def test_select_errors(dec):
    from paper_2008_10273_amd import binding
    import ctypes
    W, H = 32, 16
    planes = synth.residual_planes(W, H, synth.GRAY, 1)
    for sp in (binding.select_params(float("nan"), 1.0), binding.select_params(1.0, 1.0, 65),
               binding.select_params(1.0, 1.0, -1)):
        rc, _ = dec.select(W, H, synth.GRAY, planes, True, sp, check=False)
        assert rc == binding.PDI_EINVAL
    f = binding.pdi_frame(W, H, synth.GRAY)
    rc = binding.lib().select_mask(dec.ctx, ctypes.byref(f), 1, None, 8, None, None, None, None, None)
    assert rc == binding.PDI_EINVAL
    t = torch.zeros(W * H, device="cuda")
    rc = binding.lib().select_mask(dec.ctx, ctypes.byref(f), 1, t.data_ptr(), 16, None, t.data_ptr(),
                                   t.data_ptr(), t.data_ptr(), None)
    assert rc == binding.PDI_EINVAL


@pytest.mark.parametrize("W,H", [(1, 1), (1, 9), (9, 1), (3, 2), (17, 1)])
def test_select_tiny_planes(dec, W, H):
    """Degenerate blocks (one pixel, one row, one column): the corners already
    cover 1-pixel-wide blocks and rows split down to every pixel, so the
    masks are fixed without floating-point decisions near the threshold at
    thresholds -1 and 1e30."""
    from paper_2008_10273_amd import binding
    planes = synth.residual_planes(W, H, synth.GRAY, 100 + W * H)
    print(f"case select tiny {W}x{H}", flush=True)
    for T in (-1.0, 1e30):
        rc, d = dec.select(W, H, synth.GRAY, planes, True, binding.select_params(T, T))
        assert dec.sync() == 0
        masks, gathered = _host_masks(d, W, H, synth.GRAY, True)
        ref = oracle.select_mask(W, H, synth.GRAY, 8, planes, True, (T, T))
        assert np.array_equal(masks[0], ref[0])
        assert np.array_equal(gathered[0][0][masks[0]], planes[0][masks[0]])
