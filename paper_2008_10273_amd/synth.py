"""Seeded synthetic residual frames in the packed mask layout of the C-ABI.

This module only *draws inputs*: smooth random residual fields, per-block
random masks, and the values of the fields at the mask points, packed the
way ``decode_residual`` and the oracle both read them.  It holds none of
the inpainting arithmetic, so the GPU path and the oracle can share it.

Recipe (stand-in for the paper's Sintel residuals, which are only shown as
images in Sec. 2.3 and Fig. 3 of the paper):

* residual field per plane
  ``r = clip(sum_{k<4} A_k sin(2 pi (fx_k x + fy_k y) + phi_k) + n, -64, 64)``
  with ``fx, fy ~ U[-1/32, 1/32]`` cycles/pixel, ``phi ~ U[0, 2 pi)``,
  ``n ~ N(0, 2^2)`` i.i.d. per pixel and ``A_k = 20`` (or ``A_f / 4`` with a
  per-frame peak ``A_f`` for sequences);
* mask per block: density ``d ~ U[lo, hi]`` (or fixed), ``K = max(1,
  floor(d w h + 1/2))`` points drawn as a uniform K-subset of the w*h pixels;
* in 4:2:0 frames both chroma planes share one mask (Sec. 2.3 of the paper:
  one mask for both chroma channels), each with its own values.

Packed layout (identical to the C-ABI contract):

* planes: GRAY -> [Y]; YUV420 -> [Y (W x H), Cb, Cr (ceil(W/2) x ceil(H/2))];
* blocks of each plane in raster order, edge blocks truncated to
  ``w = min(b, W - x0)``, ``h = min(b, H - y0)``;
* mask blocks: Y blocks, then the chroma blocks once (shared mask) or Cb
  then Cr (separate masks);
* ``block_ptr[int32, n_mask_blocks + 1]`` CSR offsets into ``pos``;
* ``pos[uint16]``: in-block pixel index ``y * w + x``, strictly ascending;
* ``values[float32]``: Y values aligned with the Y part of ``pos``, then Cb
  values aligned with the chroma part, then Cr values (aligned with the
  chroma part again when the mask is shared).
"""
from __future__ import annotations

import dataclasses
from typing import Dict, Iterator, List, Optional, Sequence, Tuple

import numpy as np

GRAY = 0
YUV420 = 1

SEED_ROOT = 20081027


def plane_dims(width: int, height: int, fmt: int) -> List[Tuple[int, int]]:
    """(W, H) of every plane of a frame."""
    if fmt == GRAY:
        return [(width, height)]
    if fmt == YUV420:
        cw, ch = (width + 1) // 2, (height + 1) // 2
        return [(width, height), (cw, ch), (cw, ch)]
    raise ValueError(f"unknown format {fmt}")


def block_grid(W: int, H: int, b: int) -> np.ndarray:
    """Rows (x0, y0, w, h) of the blocks of a W x H plane, raster order."""
    nbx, nby = -(-W // b), -(-H // b)
    by, bx = np.meshgrid(np.arange(nby), np.arange(nbx), indexing="ij")
    x0 = (bx * b).ravel()
    y0 = (by * b).ravel()
    w = np.minimum(b, W - x0)
    h = np.minimum(b, H - y0)
    return np.stack([x0, y0, w, h], axis=1).astype(np.int64)


@dataclasses.dataclass
class Frame:
    width: int
    height: int
    fmt: int
    block_size: int
    chroma_shared: bool
    block_ptr: np.ndarray  # int32 [n_mask_blocks + 1]
    pos: np.ndarray  # uint16 [nnz]
    values: np.ndarray  # float32
    fields: Optional[List[np.ndarray]] = None  # float64 residual per plane

    @property
    def planes(self) -> List[Tuple[int, int]]:
        return plane_dims(self.width, self.height, self.fmt)

    @property
    def n_mask_blocks(self) -> int:
        return int(self.block_ptr.shape[0] - 1)

    @property
    def out_size(self) -> int:
        return sum(W * H for W, H in self.planes)

    def plane_offsets(self) -> List[int]:
        offs, o = [], 0
        for W, H in self.planes:
            offs.append(o)
            o += W * H
        return offs

    def mask_plane_groups(self) -> List[Tuple[int, List[int]]]:
        """(mask-plane index, [value planes]) in mask-block order."""
        if self.fmt == GRAY:
            return [(0, [0])]
        if self.chroma_shared:
            return [(0, [0]), (1, [1, 2])]
        return [(0, [0]), (1, [1]), (2, [2])]

    def iter_blocks(self) -> Iterator[dict]:
        """Every mask block with its geometry, positions and value runs."""
        nnz = int(self.block_ptr[-1])
        m = 0
        chroma_start = None
        for mplane, vplanes in self.mask_plane_groups():
            W, H = self.planes[mplane]
            grid = block_grid(W, H, self.block_size)
            if mplane == 1:
                chroma_start = int(self.block_ptr[m])
            for x0, y0, w, h in grid:
                lo, hi = int(self.block_ptr[m]), int(self.block_ptr[m + 1])
                runs = []
                for vp in vplanes:
                    if vp == 2 and self.chroma_shared:
                        base = nnz + (lo - chroma_start)
                        runs.append(self.values[base:base + (hi - lo)])
                    else:
                        runs.append(self.values[lo:hi])
                yield dict(index=m, planes=vplanes, x0=int(x0), y0=int(y0),
                           w=int(w), h=int(h), pos=self.pos[lo:hi],
                           values=runs)
                m += 1


def _field(rng: np.random.Generator, W: int, H: int, amp_each: float,
           noise_sigma: float = 2.0, clip: float = 64.0) -> np.ndarray:
    f = rng.uniform(-1.0 / 32.0, 1.0 / 32.0, size=(4, 2))
    phi = rng.uniform(0.0, 2.0 * np.pi, size=4)
    noise = rng.normal(0.0, noise_sigma, size=(H, W))
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    r = np.zeros((H, W))
    for k in range(4):
        r += amp_each * np.sin(2.0 * np.pi * (f[k, 0] * x + f[k, 1] * y) + phi[k])
    return np.clip(r + noise, -clip, clip)


def _mask_blocks(rng: np.random.Generator, grid: np.ndarray, b: int,
                 density: Tuple[float, float]) -> Tuple[np.ndarray, np.ndarray]:
    """Per-block counts and in-block positions (uniform K-subsets)."""
    nb = grid.shape[0]
    wh = grid[:, 2] * grid[:, 3]
    lo, hi = density
    d = np.full(nb, lo) if lo == hi else rng.uniform(lo, hi, size=nb)
    K = np.maximum(1, np.floor(d * wh + 0.5)).astype(np.int64)
    K = np.minimum(K, wh)
    keys = rng.random((nb, b * b))
    keys[np.arange(b * b)[None, :] >= wh[:, None]] = 2.0
    order = np.argsort(keys, axis=1, kind="stable")
    rank = np.empty_like(order)
    np.put_along_axis(rank, order, np.arange(b * b)[None, :].repeat(nb, 0), axis=1)
    sel = rank < K[:, None]
    rows, cols = np.nonzero(sel)  # row-major: ascending position per block
    return K, cols.astype(np.uint16)


def _gather(field: np.ndarray, grid: np.ndarray, K: np.ndarray,
            pos: np.ndarray) -> np.ndarray:
    blk = np.repeat(np.arange(grid.shape[0]), K)
    w = grid[blk, 2]
    px = grid[blk, 0] + pos.astype(np.int64) % w
    py = grid[blk, 1] + pos.astype(np.int64) // w
    return field[py, px].astype(np.float32)


def make_frame(width: int, height: int, fmt: int, block_size: int,
               density: Tuple[float, float], seed: Sequence[int],
               amp_each: float = 20.0, chroma_shared: bool = True,
               keep_fields: bool = True) -> Frame:
    """Draw one frame. ``seed`` feeds ``numpy.random.SeedSequence``.

    Draw order (fixed so frames are reproducible): the residual field of
    every plane (Y, Cb, Cr), then for each mask plane its densities and
    position keys.
    """
    rng = np.random.default_rng(np.random.SeedSequence(list(seed)))
    dims = plane_dims(width, height, fmt)
    fields = [_field(rng, W, H, amp_each) for (W, H) in dims]
    groups = ([(0, [0])] if fmt == GRAY else
              ([(0, [0]), (1, [1, 2])] if chroma_shared else
               [(0, [0]), (1, [1]), (2, [2])]))
    counts, poss, vals = [], [], []
    extra_cr = None
    for mplane, vplanes in groups:
        W, H = dims[mplane]
        grid = block_grid(W, H, block_size)
        K, pos = _mask_blocks(rng, grid, block_size, density)
        counts.append(K)
        poss.append(pos)
        vals.append(_gather(fields[vplanes[0]], grid, K, pos))
        if len(vplanes) == 2:
            extra_cr = _gather(fields[vplanes[1]], grid, K, pos)
    K_all = np.concatenate(counts)
    block_ptr = np.zeros(K_all.shape[0] + 1, dtype=np.int64)
    np.cumsum(K_all, out=block_ptr[1:])
    if block_ptr[-1] > np.iinfo(np.int32).max:
        raise ValueError("frame too large for int32 offsets")
    values = np.concatenate(vals + ([extra_cr] if extra_cr is not None else []))
    return Frame(width, height, fmt, block_size, bool(chroma_shared and fmt == YUV420),
                 block_ptr.astype(np.int32), np.concatenate(poss).astype(np.uint16),
                 values.astype(np.float32), fields if keep_fields else None)


def pack_dense(width: int, height: int, fmt: int, block_size: int,
               masks: List[np.ndarray], fields: List[np.ndarray],
               chroma_shared: bool = True) -> Frame:
    """Pack dense per-plane masks (bool, H x W) and fields into the CSR layout.

    With a shared chroma mask, ``masks`` holds [Y, C]; otherwise one mask per
    plane.  This is the host-side counterpart of the library's
    ``pdi_pack_dense``; it is used to build hand-made test frames.
    """
    dims = plane_dims(width, height, fmt)
    shared = bool(chroma_shared and fmt == YUV420)
    groups = ([(0, [0])] if fmt == GRAY else
              ([(0, [0]), (1, [1, 2])] if shared else [(0, [0]), (1, [1]), (2, [2])]))
    counts, poss, vals, extra = [], [], [], []
    for gi, (mplane, vplanes) in enumerate(groups):
        W, H = dims[mplane]
        m = np.asarray(masks[gi], dtype=bool)
        assert m.shape == (H, W)
        for x0, y0, w, h in block_grid(W, H, block_size):
            sub = m[y0:y0 + h, x0:x0 + w]
            t = np.flatnonzero(sub.ravel())
            counts.append(t.size)
            poss.append(t.astype(np.uint16))
            yy, xx = y0 + t // w, x0 + t % w
            vals.append(np.asarray(fields[vplanes[0]])[yy, xx].astype(np.float32))
            if len(vplanes) == 2:
                extra.append(np.asarray(fields[vplanes[1]])[yy, xx].astype(np.float32))
    block_ptr = np.zeros(len(counts) + 1, dtype=np.int64)
    np.cumsum(counts, out=block_ptr[1:])
    values = np.concatenate(vals + extra) if (vals or extra) else np.zeros(0, np.float32)
    return Frame(width, height, fmt, block_size, shared, block_ptr.astype(np.int32),
                 np.concatenate(poss).astype(np.uint16) if poss else np.zeros(0, np.uint16),
                 values.astype(np.float32),
                 [np.asarray(f, dtype=np.float64) for f in fields])


# Workload presets: the five measurement configurations and their sizes.
CONFIGS: Dict[int, dict] = {
    0: dict(name="gray256_b16_d5", width=256, height=256, fmt=GRAY,
            block_size=16, density=(0.05, 0.05)),
    1: dict(name="fhd420_b16_d1-10", width=1920, height=1080, fmt=YUV420,
            block_size=16, density=(0.01, 0.10)),
    2: dict(name="fhd420_b32_d2-10", width=1920, height=1080, fmt=YUV420,
            block_size=32, density=(0.02, 0.10)),
    3: dict(name="fhd420_b16_seq64", width=1920, height=1080, fmt=YUV420,
            block_size=16, density=(0.01, 0.10), frames=64, amp_range=(5.0, 64.0)),
}

# Coefficient-input workload: the paper's 8x8 residual blocks (Sec. 2.3) on a
# 1080p 4:2:0 frame, masks drawn as for config 1; see coef_inputs.
COEF_CONFIG = dict(name="fhd420_b8_coef_d1-10", width=1920, height=1080, fmt=YUV420,
                   block_size=8, density=(0.01, 0.10), steps=(0.25, 0.25, 0.25), rho=0.5)

# Coefficient encode: the masks and residual values of the stored-coefficient
# workload's frames, solved per 8x8 block and quantised with a step that
# maps the coefficients (|c| <= ~55 on these frames) into [-127, 127].
ENCODE_CONFIG = dict(name="fhd420_b8_encode_d1-10", width=1920, height=1080, fmt=YUV420,
                     block_size=8, density=(0.01, 0.10), steps=(0.5, 0.5, 0.5))

# Serving mix: (width, height, count) per resolution class, 4:2:0, b16.
SERVING_MIX = [(854, 480, 6), (1280, 720, 6), (1920, 1080, 4)]


def config_frame(cfg: int, frame: int = 0, stream: int = 0,
                 keep_fields: bool = True) -> Frame:
    """Frame ``frame`` of configuration ``cfg`` (0-3), seeded per frame."""
    c = CONFIGS[cfg]
    seed = (SEED_ROOT, cfg, stream, frame)
    amp = 20.0
    if "amp_range" in c:
        a_rng = np.random.default_rng(np.random.SeedSequence([SEED_ROOT, cfg, stream, frame, 1]))
        amp = float(a_rng.uniform(*c["amp_range"])) / 4.0
    return make_frame(c["width"], c["height"], c["fmt"], c["block_size"],
                      c["density"], seed, amp_each=amp, keep_fields=keep_fields)


def serving_frame(stream: int, frame: int, keep_fields: bool = False) -> Frame:
    """Frame ``frame`` of serving stream ``stream`` (0-15) of the mix."""
    s, cls = stream, 0
    for (w, h, n) in SERVING_MIX:
        if s < n:
            break
        s -= n
        cls += 1
    w, h, _ = SERVING_MIX[cls]
    return make_frame(w, h, YUV420, 16, (0.01, 0.10), (SEED_ROOT, 4, stream, frame),
                      keep_fields=keep_fields)


def serving_stream_dims(stream: int) -> Tuple[int, int]:
    s = stream
    for (w, h, n) in SERVING_MIX:
        if s < n:
            return w, h
        s -= n
    raise ValueError(stream)


def random_frame(width: int, height: int, fmt: int, block_size: int,
                 density: Tuple[float, float], seed: int, chroma_shared: bool = True) -> Frame:
    """A small seeded frame for parity tests (any geometry)."""
    return make_frame(width, height, fmt, block_size, density, (SEED_ROOT, 99, seed, 0),
                      chroma_shared=chroma_shared)


def plane_block_counts(width: int, height: int, fmt: int, block_size: int) -> List[int]:
    """Number of blocks of every plane (edge blocks included)."""
    return [((W + block_size - 1) // block_size) * ((H + block_size - 1) // block_size)
            for W, H in plane_dims(width, height, fmt)]


def coef_inputs(frame: Frame, seed) -> Tuple[np.ndarray, np.ndarray]:
    """Stored-coefficient inputs for ``frame``'s mask: int8 codes laid out like
    ``frame.values`` and one FP32 constant per block of every plane (Y, then
    Cb, then Cr, raster order).  Codes are rounded draws clipped to
    [-127, 127] with Laplace(0, 3) (mostly small, about 15 % zero: the shape a
    dead-zone quantiser leaves); constants are U[-64, 64].  Random numbers
    only."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_ROOT, 5] + list(np.atleast_1d(seed))))
    q = np.clip(np.rint(rng.laplace(0.0, 3.0, frame.values.size)), -127, 127).astype(np.int8)
    nb = sum(plane_block_counts(frame.width, frame.height, frame.fmt, frame.block_size))
    consts = rng.uniform(-64.0, 64.0, nb).astype(np.float32)
    return q, consts


def coef_frame(frame: int = 0) -> Tuple[Frame, np.ndarray, np.ndarray]:
    """Frame ``frame`` of the coefficient-input workload: (mask frame, codes,
    constants)."""
    c = COEF_CONFIG
    fr = make_frame(c["width"], c["height"], c["fmt"], c["block_size"], c["density"],
                    (SEED_ROOT, 5, 0, frame), keep_fields=False)
    q, consts = coef_inputs(fr, (0, frame))
    return fr, q, consts


def residual_planes(width: int, height: int, fmt: int, seed) -> List[np.ndarray]:
    """Dense residual planes (Y, then Cb and Cr for 4:2:0) from the residual
    field recipe, float32 (H, W) arrays: the encoder's input.  Random numbers
    only."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_ROOT, 8] + list(np.atleast_1d(seed))))
    return [_field(rng, W, H, 20.0).astype(np.float32) for W, H in plane_dims(width, height, fmt)]


# Mask selection workload: dense 1920x1080 4:2:0 residual planes, 8x8 blocks,
# rectangles split above a mean squared error of 16 (luma) / 32 (chroma):
# about 14 % / 9 % of the pixels become mask points on these planes.
SELECT_CONFIG = dict(name="fhd420_b8_select_t16-32", width=1920, height=1080, fmt=YUV420, block_size=8,
                     threshold=(16.0, 32.0))


# Intra-frame workload for global homogeneous diffusion inpainting (Sec. 2.1):
# one 1920x1080 plane, a uniform random mask of 4 % of the pixels, values
# from the residual field recipe.
INTRA_CONFIG = dict(name="fhd_gray_intra_d4", width=1920, height=1080, density=0.04)


def intra_frame(width: int, height: int, density: float, seed) -> Tuple[np.ndarray, np.ndarray]:
    """(mask, f): a (height, width) bool mask with each pixel known with
    probability ``density`` (at least one pixel), and a float32 plane drawn
    like a residual field (f is only read at the mask).  Random numbers only."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_ROOT, 6] + list(np.atleast_1d(seed))))
    m = rng.uniform(size=(height, width)) < density
    if not m.any():
        m[rng.integers(height), rng.integers(width)] = True
    f = _field(rng, width, height, 20.0)
    return m, f.astype(np.float32)
