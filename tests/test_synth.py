"""The seeded generator: determinism, layout contract and workload shapes."""
import numpy as np
import pytest

from paper_2008_10273_amd import synth


def _check_layout(fr):
    nb = fr.n_mask_blocks
    assert fr.block_ptr.dtype == np.int32 and fr.pos.dtype == np.uint16
    assert fr.values.dtype == np.float32
    assert fr.block_ptr[0] == 0 and np.all(np.diff(fr.block_ptr) >= 0)
    blocks = list(fr.iter_blocks())
    assert len(blocks) == nb
    for blk in blocks:
        p = blk["pos"].astype(int)
        assert np.all(np.diff(p) > 0)
        assert p.size == 0 or p.max() < blk["w"] * blk["h"]
        for vp, vals in zip(blk["planes"], blk["values"]):
            assert vals.size == p.size
            if fr.fields is not None:
                px = blk["x0"] + p % blk["w"]
                py = blk["y0"] + p // blk["w"]
                np.testing.assert_array_equal(vals, fr.fields[vp][py, px].astype(np.float32))
    nnz = int(fr.block_ptr[-1])
    if fr.chroma_shared:
        nY = len(synth.block_grid(fr.width, fr.height, fr.block_size))
        nnz_c = nnz - int(fr.block_ptr[nY])
        assert fr.values.size == nnz + nnz_c
    else:
        assert fr.values.size == nnz
    return blocks


def test_determinism():
    a = synth.config_frame(0)
    b = synth.config_frame(0)
    np.testing.assert_array_equal(a.pos, b.pos)
    np.testing.assert_array_equal(a.values, b.values)
    c = synth.config_frame(0, frame=1)
    assert not np.array_equal(a.values, c.values)


def test_config0_shape():
    fr = synth.config_frame(0)
    blocks = _check_layout(fr)
    assert len(blocks) == 256
    assert set(np.diff(fr.block_ptr)) == {13}
    assert np.abs(fr.values).max() <= 64.0


@pytest.mark.parametrize("cfg,nblocks,kmin,kmax", [(1, 10200, 1, 26), (2, 2550, 15, 102)])
def test_fhd_configs(cfg, nblocks, kmin, kmax):
    fr = synth.config_frame(cfg, keep_fields=False)
    assert fr.n_mask_blocks == nblocks
    K = np.diff(fr.block_ptr)
    assert K.min() >= kmin and K.max() <= kmax
    b = fr.block_size
    nY = len(synth.block_grid(1920, 1080, b))
    full = [i for i, (x0, y0, w, h) in enumerate(synth.block_grid(1920, 1080, b)) if w * h == b * b]
    lo = 3 if b == 16 else 20
    assert K[full].min() >= lo
    assert fr.out_size == 1920 * 1080 + 2 * 960 * 540
    _check_layout(synth.random_frame(1920 // 8, 1080 // 8, synth.YUV420, b, (0.01, 0.1), 3))


def test_separate_chroma_layout():
    fr = synth.random_frame(50, 34, synth.YUV420, 16, (0.05, 0.3), seed=4, chroma_shared=False)
    assert not fr.chroma_shared
    _check_layout(fr)


def test_pack_dense_roundtrip():
    fr = synth.random_frame(40, 24, synth.GRAY, 8, (0.1, 0.3), seed=2)
    m = np.zeros((24, 40), bool)
    for blk in fr.iter_blocks():
        p = blk["pos"].astype(int)
        m[blk["y0"] + p // blk["w"], blk["x0"] + p % blk["w"]] = True
    fr2 = synth.pack_dense(40, 24, synth.GRAY, 8, [m], fr.fields)
    np.testing.assert_array_equal(fr.block_ptr, fr2.block_ptr)
    np.testing.assert_array_equal(fr.pos, fr2.pos)
    np.testing.assert_array_equal(fr.values, fr2.values)


def test_sequence_amplitudes_vary():
    amps = []
    for f in range(3):
        fr = synth.config_frame(3, frame=f)
        amps.append(np.abs(fr.fields[0]).max())
    assert len(set(np.round(amps, 3))) == 3
