"""C-ABI: the library loads, exports every symbol of include/pdinp.h, and the
host-only entry points behave (no GPU needed)."""
import os
import re

import numpy as np
import pytest

from paper_2008_10273_amd import binding, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pdinp.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "defined")))


def test_header_declares_the_binding_exports():
    assert set(_declared()) == set(binding.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = binding.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_default_params():
    p = binding.default_params()
    assert p.op == 0 and p.s == 1.0 and p.eval_dtype == 0 and p.refine == 1
    assert p.path == 0 and abs(p.refine_tau - 1 / 64) < 1e-15
    assert p.out_int8 == 0


@pytest.mark.parametrize("w,h,fmt,b,shared,nb,nel", [
    (1920, 1080, 1, 16, 1, 8160 + 2040, 1920 * 1080 + 2 * 960 * 540),
    (1920, 1080, 1, 32, 1, 2040 + 510, 1920 * 1080 + 2 * 960 * 540),
    (1920, 1080, 1, 16, 0, 8160 + 2 * 2040, 1920 * 1080 + 2 * 960 * 540),
    (256, 256, 0, 16, 0, 256, 65536),
    (70, 37, 1, 8, 1, 9 * 5 + 5 * 3, 70 * 37 + 2 * 35 * 19),
])
def test_frame_info(w, h, fmt, b, shared, nb, nel):
    rc, n, e = binding.pdi_frame_info(w, h, fmt, b, shared)
    assert rc == 0 and n == nb and e == nel


def test_frame_info_rejects_bad_geometry():
    assert binding.pdi_frame_info(0, 10, 0, 16, 0)[0] == binding.PDI_EINVAL
    assert binding.pdi_frame_info(10, 10, 0, 12, 0)[0] == binding.PDI_EINVAL
    assert binding.pdi_frame_info(10, 10, 7, 16, 0)[0] == binding.PDI_EINVAL


def test_decode_with_null_context_is_einval():
    rc = binding.decode_residual(0, 16, 16, 0, 0, 0, 1, False, 0, 16, None, 0, 0)
    assert rc == binding.PDI_EINVAL
    assert binding.pdi_sync(0, 0) == binding.PDI_EINVAL
    assert binding.pdi_last_error(0) == "null context"


def test_validate_host_accepts_generated_frames():
    for fr in (synth.config_frame(0),
               synth.random_frame(70, 37, synth.YUV420, 16, (0.02, 0.3), seed=3),
               synth.random_frame(70, 37, synth.YUV420, 8, (0.02, 0.3), seed=4, chroma_shared=False)):
        assert binding.pdi_validate_host(fr.width, fr.height, fr.fmt, fr.block_size, fr.block_ptr,
                                         fr.pos, fr.chroma_shared, fr.values) == binding.PDI_OK


def test_validate_host_rejects_bad_masks():
    fr = synth.config_frame(0)
    args = (fr.width, fr.height, fr.fmt, fr.block_size)
    pos = fr.pos.copy()
    pos[5] = pos[4]  # duplicate
    assert binding.pdi_validate_host(*args, fr.block_ptr, pos, False, fr.values) == binding.PDI_EMASK
    pos = fr.pos.copy()
    pos[0] = 256  # outside the block
    assert binding.pdi_validate_host(*args, fr.block_ptr, pos, False, fr.values) == binding.PDI_EMASK
    vals = fr.values.copy()
    vals[7] = np.nan
    assert binding.pdi_validate_host(*args, fr.block_ptr, fr.pos, False, vals) == binding.PDI_EVALUE
    assert binding.pdi_validate_host(*args, fr.block_ptr[:-1], fr.pos, False, fr.values) == binding.PDI_EINVAL


@pytest.mark.parametrize("shared", [True, False])
def test_pack_dense_matches_generator_layout(shared):
    fr = synth.random_frame(45, 29, synth.YUV420, 8, (0.05, 0.4), seed=6, chroma_shared=shared)
    dims = fr.planes
    masks = []
    groups = fr.mask_plane_groups()
    for mplane, _ in groups:
        W, H = dims[mplane]
        masks.append(np.zeros((H, W), np.uint8))
    for blk in fr.iter_blocks():
        gi = 0 if blk["planes"][0] == 0 else (1 if shared else blk["planes"][0])
        p = blk["pos"].astype(int)
        masks[gi][blk["y0"] + p // blk["w"], blk["x0"] + p % blk["w"]] = 1
    m = np.concatenate([x.ravel() for x in masks])
    f = np.concatenate([x.astype(np.float32).ravel() for x in fr.fields])
    bp, pos, vals = binding.pdi_pack_dense(fr.width, fr.height, fr.fmt, fr.block_size, shared, m, f)
    np.testing.assert_array_equal(bp, fr.block_ptr)
    np.testing.assert_array_equal(pos, fr.pos)
    np.testing.assert_array_equal(vals, fr.values)
