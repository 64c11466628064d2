"""FP64 CPU oracle for block-based pseudodifferential residual inpainting.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the ``cpu_baseline`` leg of ``bench.py``, never by the product
package.  It shares no code with the GPU library and reads frames through the
documented packed layout only (any object with ``width, height, fmt,
block_size, chroma_shared, block_ptr, pos, values``).

The C source ``pdinp_oracle.c`` holds two independent routes from the paper
(Sec. 2.1-2.2): the plain definition, Eq. (1) solved per block, and the
Green's-function route, Eqs. (2)-(4); and the decoder of stored, dead-zone
quantised coefficients (Sec. 2.2 last paragraph, Sec. 2.3), Eq. (2) summed
directly.  Both are pinned by ``tests/`` against
facts the paper and the mathematics fix (closed forms, brute-force solves,
textbook routines).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from typing import List, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pdinp_oracle.c")
LIB_PATH = os.path.join(_HERE, "_pdinp_oracle.so")
_lock = threading.Lock()
_lib_handle = None

DIRECT = 0
GREEN = 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, -O2, no fast-math)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _lib():
    global _lib_handle
    with _lock:
        if _lib_handle is None:
            if not os.path.exists(LIB_PATH):
                build(force=False)
            L = ctypes.CDLL(LIB_PATH)
            P = ctypes.c_void_p
            i, d = ctypes.c_int, ctypes.c_double
            L.orc_block_direct.argtypes = [i, i, i, i, P, P, P]
            L.orc_block_direct.restype = i
            L.orc_eigenvalues.argtypes = [i, i, i, d, P]
            L.orc_eigenvalues.restype = None
            L.orc_green_table.argtypes = [i, i, P, P]
            L.orc_green_table.restype = None
            L.orc_green.argtypes = [i, i, P, i, i, i, i]
            L.orc_green.restype = d
            L.orc_block_green.argtypes = [i, i, i, d, i, P, i, P, P, P, P]
            L.orc_block_green.restype = i
            L.orc_decode.argtypes = [i, i, i, i, P, P, P, i, i, i, d, P, i]
            L.orc_decode.restype = i
            L.orc_dequant.argtypes = [i, d, d]
            L.orc_dequant.restype = d
            L.orc_decode_coef.argtypes = [i, i, i, i, P, P, P, i, P, P, d, i, d, P, i]
            L.orc_decode_coef.restype = i
            L.orc_quant.argtypes = [d, d]
            L.orc_quant.restype = i
            L.orc_encode_coef.argtypes = [i, i, i, i, P, P, P, i, P, i, d, P, P, P, i]
            L.orc_encode_coef.restype = i
            L.orc_select_mask.argtypes = [i, i, i, i, P, i, P, i, P, i]
            L.orc_select_mask.restype = i
            _lib_handle = L
    return _lib_handle


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def plane_dims(width: int, height: int, fmt: int) -> List[Tuple[int, int]]:
    if fmt == 0:
        return [(width, height)]
    cw, ch = (width + 1) // 2, (height + 1) // 2
    return [(width, height), (cw, ch), (cw, ch)]


def block_direct(w: int, h: int, pos, r, s: int = 1) -> np.ndarray:
    """Eq. (1) on one w x h block (plain definition); returns u as (h, w)."""
    pos = np.ascontiguousarray(pos, dtype=np.uint16)
    r = np.ascontiguousarray(r, dtype=np.float64)
    u = np.zeros(w * h)
    rc = _lib().orc_block_direct(w, h, int(s), int(pos.size), _ptr(pos), _ptr(r), _ptr(u))
    if rc != 0:
        raise ValueError("orc_block_direct failed")
    return u.reshape(h, w)


def eigenvalues(w: int, h: int, op: int = 0, s: float = 1.0) -> np.ndarray:
    lam = np.zeros(w * h)
    _lib().orc_eigenvalues(w, h, op, float(s), _ptr(lam))
    return lam.reshape(h, w)


def green_table(w: int, h: int, op: int = 0, s: float = 1.0) -> np.ndarray:
    lam = np.ascontiguousarray(eigenvalues(w, h, op, s).ravel())
    H = np.zeros((h + 1) * (w + 1))
    _lib().orc_green_table(w, h, _ptr(lam), _ptr(H))
    return H.reshape(h + 1, w + 1)


def green_matrix(w: int, h: int, op: int = 0, s: float = 1.0) -> np.ndarray:
    """The full N x N matrix G of one block shape, read from the table."""
    H = np.ascontiguousarray(green_table(w, h, op, s).ravel())
    L = _lib()
    N = w * h
    G = np.empty((N, N))
    for a in range(N):
        for b in range(N):
            G[a, b] = L.orc_green(w, h, _ptr(H), a % w, a // w, b % w, b // w)
    return G


def block_green(w: int, h: int, pos, r, op: int = 0, s: float = 1.0):
    """Green's route on one block.  r is (K,) or (nrhs, K).

    Returns (c, a, u) with c (nrhs, K), a (nrhs,), u (nrhs, h, w)."""
    pos = np.ascontiguousarray(pos, dtype=np.uint16)
    r2 = np.atleast_2d(np.asarray(r, dtype=np.float64))
    r2 = np.ascontiguousarray(r2)
    nrhs, K = r2.shape[0], pos.size
    c = np.zeros((nrhs, max(K, 1)))
    a = np.zeros(nrhs)
    u = np.zeros((nrhs, w * h))
    rc = _lib().orc_block_green(w, h, op, float(s), K, _ptr(pos), nrhs, _ptr(r2),
                                _ptr(c), _ptr(a), _ptr(u))
    if rc != 0:
        raise ValueError("orc_block_green failed")
    return c[:, :K], a, u.reshape(nrhs, h, w)


def decode(frame, method: int = DIRECT, op: int = 0, s: float = 1.0,
           nthreads: int = 0) -> List[np.ndarray]:
    """Decode a whole packed frame; returns one float64 (H, W) array per plane."""
    dims = plane_dims(frame.width, frame.height, frame.fmt)
    out = np.zeros(sum(W * H for W, H in dims))
    bp = np.ascontiguousarray(frame.block_ptr, dtype=np.int32)
    pos = np.ascontiguousarray(frame.pos, dtype=np.uint16)
    vals = np.ascontiguousarray(frame.values, dtype=np.float32)
    if pos.size == 0:
        pos = np.zeros(1, np.uint16)
    if vals.size == 0:
        vals = np.zeros(1, np.float32)
    rc = _lib().orc_decode(frame.width, frame.height, frame.fmt, frame.block_size,
                           _ptr(bp), _ptr(pos), _ptr(vals), int(bool(frame.chroma_shared)),
                           int(method), int(op), float(s), _ptr(out), int(nthreads))
    if rc != 0:
        raise ValueError("orc_decode failed")
    planes, o = [], 0
    for W, H in dims:
        planes.append(out[o:o + W * H].reshape(H, W))
        o += W * H
    return planes


def decode_flat(frame, **kw) -> np.ndarray:
    """Like :func:`decode` but returns the concatenated planes (C-ABI layout)."""
    return np.concatenate([p.ravel() for p in decode(frame, **kw)])


def dequant(q, step: float, rho: float) -> np.ndarray:
    """Dead-zone reconstruction of stored codes (Sec. 2.3): 0 stays 0, else
    sign(q) (|q| + rho) step."""
    q = np.asarray(q)
    L = _lib()
    return np.array([L.orc_dequant(int(v), float(step), float(rho)) for v in q.ravel()]).reshape(q.shape)


def decode_coef(frame, coef, consts, steps, rho: float, op: int = 0, s: float = 1.0,
                nthreads: int = 0) -> List[np.ndarray]:
    """Decode a frame from stored coefficients (Sec. 2.2, last paragraph):
    per block u = sum_i c_i G(., x_i) + a with c_i the dequantised codes
    (laid out like ``frame.values``) and a from ``consts`` (one per block of
    each plane: Y, then Cb, then Cr, raster order).  ``steps``: quantiser step
    per plane.  Returns one float64 (H, W) array per plane."""
    dims = plane_dims(frame.width, frame.height, frame.fmt)
    out = np.zeros(sum(W * H for W, H in dims))
    bp = np.ascontiguousarray(frame.block_ptr, dtype=np.int32)
    pos = np.ascontiguousarray(frame.pos, dtype=np.uint16)
    q = np.ascontiguousarray(coef, dtype=np.int8)
    cs = np.ascontiguousarray(consts, dtype=np.float32)
    st = np.zeros(3)
    st[:len(steps)] = steps
    if pos.size == 0:
        pos = np.zeros(1, np.uint16)
    if q.size == 0:
        q = np.zeros(1, np.int8)
    rc = _lib().orc_decode_coef(frame.width, frame.height, frame.fmt, frame.block_size,
                                _ptr(bp), _ptr(pos), _ptr(q), int(bool(frame.chroma_shared)),
                                _ptr(cs), _ptr(st), float(rho), int(op), float(s), _ptr(out), int(nthreads))
    if rc != 0:
        raise ValueError("orc_decode_coef failed")
    planes, o = [], 0
    for W, H in dims:
        planes.append(out[o:o + W * H].reshape(H, W))
        o += W * H
    return planes


def decode_coef_flat(frame, coef, consts, steps, rho: float, **kw) -> np.ndarray:
    """Like :func:`decode_coef` but returns the concatenated planes."""
    return np.concatenate([p.ravel() for p in decode_coef(frame, coef, consts, steps, rho, **kw)])


def quant(c, step: float) -> np.ndarray:
    """Dead-zone quantisation of coefficients (Sec. 2.3): sign(c) min(127,
    floor(|c| / step)); |c| < step gives 0."""
    c = np.asarray(c, dtype=np.float64)
    L = _lib()
    return np.array([L.orc_quant(float(v), float(step)) for v in c.ravel()], dtype=np.int64).reshape(c.shape)


def encode_coef(frame, steps, op: int = 0, s: float = 1.0, nthreads: int = 0):
    """Encode a frame's blocks (the encoder side of Sec. 2.2's split): per
    block and value plane, c and a of the bordered system with the values at
    the mask points, c quantised per plane by :func:`quant`.  Returns
    (codes int8 laid out like ``frame.values``, c unquantised in the same
    layout, consts float64: a of every block of every plane)."""
    dims = plane_dims(frame.width, frame.height, frame.fmt)
    b = frame.block_size
    nblocks = sum(((W + b - 1) // b) * ((H + b - 1) // b) for W, H in dims)
    bp = np.ascontiguousarray(frame.block_ptr, dtype=np.int32)
    pos = np.ascontiguousarray(frame.pos, dtype=np.uint16)
    vals = np.ascontiguousarray(frame.values, dtype=np.float32)
    nv = max(vals.size, 1)
    code = np.zeros(nv, np.int8)
    cex = np.zeros(nv)
    consts = np.zeros(nblocks)
    st = np.zeros(3)
    st[:len(steps)] = steps
    if pos.size == 0:
        pos = np.zeros(1, np.uint16)
    if vals.size == 0:
        vals = np.zeros(1, np.float32)
    rc = _lib().orc_encode_coef(frame.width, frame.height, frame.fmt, b, _ptr(bp), _ptr(pos), _ptr(vals),
                                int(bool(frame.chroma_shared)), _ptr(st), int(op), float(s),
                                _ptr(code), _ptr(cex), _ptr(consts), int(nthreads))
    if rc != 0:
        raise ValueError("orc_encode_coef failed")
    n = frame.values.size
    return code[:n], cex[:n], consts


def select_mask(width: int, height: int, fmt: int, b: int, planes, chroma_shared: bool, thr,
                max_rounds: int = 64, nthreads: int = 0) -> List[np.ndarray]:
    """Per-block mask selection by rectangular subdivision (the encoder's
    choice of each block's points, Sec. 2.3): see orc_select_block.
    ``planes``: dense residual planes (Y, Cb, Cr for 4:2:0) as (H, W)
    arrays; ``thr``: (luma, chroma) thresholds on a rectangle's mean squared
    error.  Returns the masks of the mask planes (Y, then one shared chroma
    mask or Cb and Cr) as (H, W) bool arrays."""
    dims = plane_dims(width, height, fmt)
    flat = np.ascontiguousarray(np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in planes]))
    if fmt == 0:
        mdims = dims[:1]
    elif chroma_shared:
        mdims = dims[:2]
    else:
        mdims = dims
    out = np.zeros(sum(W * H for W, H in mdims), np.uint8)
    t = np.ascontiguousarray(np.asarray(thr, dtype=np.float64).reshape(-1)[:2])
    if t.size == 1:
        t = np.array([t[0], t[0]])
    rc = _lib().orc_select_mask(width, height, fmt, b, _ptr(flat), int(bool(chroma_shared)), _ptr(t),
                                int(max_rounds), _ptr(out), int(nthreads))
    if rc != 0:
        raise ValueError("orc_select_mask failed")
    res, o = [], 0
    for W, H in mdims:
        res.append(out[o:o + W * H].reshape(H, W).astype(bool))
        o += W * H
    return res


def homogeneous_inpaint(mask, f) -> np.ndarray:
    """Global homogeneous diffusion inpainting (Sec. 2.1, Eq. (1) with
    A = -L on the whole image, reflecting boundaries): u = f at the mask
    pixels and (A u)_i = 0 at every other pixel.  Solved exactly in FP64:
    the unknowns satisfy A_UU u_U = -A_UK f_K, a sparse SPD system when the
    mask is not empty, factorised by a sparse LU (scipy's SuperLU).  An empty
    mask leaves the system singular (constants); u = 0 is returned then.
    mask: (H, W) bool; f: (H, W) values (read at the mask pixels only)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    m = np.asarray(mask, dtype=bool)
    H, W = m.shape
    fv = np.asarray(f, dtype=np.float64).ravel()
    N = W * H
    if not m.any():
        return np.zeros((H, W))
    # -L of the W x H grid: degree minus adjacency over the 4-neighbourhood
    # inside the image (a mirrored neighbour equals the pixel itself and adds
    # nothing).
    idx = np.arange(N).reshape(H, W)
    rows, cols = [], []
    rows.append(idx[:, :-1].ravel()); cols.append(idx[:, 1:].ravel())
    rows.append(idx[:-1, :].ravel()); cols.append(idx[1:, :].ravel())
    r = np.concatenate(rows); c = np.concatenate(cols)
    adj = sp.coo_matrix((np.ones(r.size), (r, c)), shape=(N, N))
    adj = (adj + adj.T).tocsr()
    deg = np.asarray(adj.sum(axis=1)).ravel()
    A = (sp.diags(deg) - adj).tocsr()
    K = m.ravel()
    U = ~K
    u = np.zeros(N)
    u[K] = fv[K]
    if U.any():
        A_UU = A[U][:, U].tocsc()
        rhs = -(A[U][:, K] @ fv[K])
        u[U] = spla.spsolve(A_UU, rhs)
    return u.reshape(H, W)
