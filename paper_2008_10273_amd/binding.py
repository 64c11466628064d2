"""Thin ctypes binding of ``libpdinp.so`` (include/pdinp.h), same names.

Argument marshalling only: every step of the decode runs in the library's
HIP kernels.  Device buffers are passed as raw pointers (``tensor.data_ptr()``)
and streams as ``hipStream_t`` handles (``torch.cuda.Stream.cuda_stream``).
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpdinp.so")

PDI_OK, PDI_EINVAL, PDI_EMASK, PDI_ENOMEM, PDI_EHIP, PDI_EBUSY, PDI_EVALUE, PDI_ESOLVE = 0, -1, -2, -3, -4, -5, -6, -7
PDI_GRAY, PDI_YUV420 = 0, 1
PDI_EVAL_FP32, PDI_EVAL_FP16, PDI_EVAL_BF16, PDI_EVAL_BF16X2 = 0, 1, 2, 3
PDI_PATH_AUTO, PDI_PATH_PLAIN = 0, 1
PDI_OP_DISCRETE, PDI_OP_CONTINUOUS = 0, 1

ERROR_NAMES = {0: "PDI_OK", -1: "PDI_EINVAL", -2: "PDI_EMASK", -3: "PDI_ENOMEM", -4: "PDI_EHIP",
               -5: "PDI_EBUSY", -6: "PDI_EVALUE", -7: "PDI_ESOLVE"}

EXPORTS = ["pdi_default_params", "pdi_create", "pdi_destroy", "decode_residual", "decode_residual_batch",
           "decode_residual_batch_noalloc",
           "decode_coefficients", "decode_coefficients_batch", "encode_coefficients",
           "encode_coefficients_batch", "pdi_default_select_params", "select_mask", "pdi_sync",
           "pdi_default_cg_params", "inpaint_homogeneous",
           "pdi_last_error", "pdi_frame_info", "pdi_pack_dense", "pdi_validate_host", "pdi_autotune", "pdi_autotune_batch",
           "pdi_seq_create", "pdi_seq_launch", "pdi_seq_sync", "pdi_seq_destroy",
           "pdi_server_create", "pdi_submit", "pdi_poll", "pdi_wait", "pdi_server_stats",
           "pdi_server_hold", "pdi_server_destroy"]


class pdi_frame(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("format", ctypes.c_int32)]


class pdi_mask(ctypes.Structure):
    _fields_ = [("block_ptr", ctypes.c_void_p), ("pos", ctypes.c_void_p),
                ("n_mask_blocks", ctypes.c_int32), ("chroma_shared", ctypes.c_int32)]


class pdi_params(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("s", ctypes.c_double), ("eval_dtype", ctypes.c_int32),
                ("refine", ctypes.c_int32), ("validate", ctypes.c_int32), ("path", ctypes.c_int32),
                ("refine_tau", ctypes.c_double), ("out_int8", ctypes.c_int32)]


class pdi_coef_params(ctypes.Structure):
    _fields_ = [("step", ctypes.c_float * 3), ("rho", ctypes.c_float)]


def coef_params(steps, rho: float) -> pdi_coef_params:
    q = pdi_coef_params()
    st = list(steps) + [0.0] * (3 - len(steps))
    for k in range(3):
        q.step[k] = float(st[k])
    q.rho = float(rho)
    return q


class pdi_select_params(ctypes.Structure):
    _fields_ = [("threshold", ctypes.c_float * 2), ("max_rounds", ctypes.c_int32)]


def select_params(thr_luma: float = None, thr_chroma: float = None, max_rounds: int = None) -> pdi_select_params:
    p = pdi_select_params()
    lib().pdi_default_select_params(ctypes.byref(p))
    if thr_luma is not None:
        p.threshold[0] = thr_luma
    if thr_chroma is not None:
        p.threshold[1] = thr_chroma
    if max_rounds is not None:
        p.max_rounds = max_rounds
    return p


class pdi_cg_params(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("check", ctypes.c_int32),
                ("coarse_tol", ctypes.c_double)]


def cg_params(**kw) -> pdi_cg_params:
    p = pdi_cg_params()
    lib().pdi_default_cg_params(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


class PdiError(RuntimeError):
    def __init__(self, code: int, msg: str = ""):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """Load the built library (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_2008_10273_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64p = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int64)
        L.pdi_default_params.argtypes = [ctypes.POINTER(pdi_params)]
        L.pdi_default_params.restype = None
        L.pdi_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), i32, ctypes.c_size_t]
        L.pdi_create.restype = i32
        L.pdi_destroy.argtypes = [P]
        L.pdi_destroy.restype = None
        L.decode_residual.argtypes = [P, ctypes.POINTER(pdi_frame), ctypes.POINTER(pdi_mask), P, i32,
                                      ctypes.POINTER(pdi_params), P, P]
        L.decode_residual.restype = i32
        L.decode_residual_batch.argtypes = [P, i32, ctypes.POINTER(pdi_frame), ctypes.POINTER(pdi_mask),
                                            ctypes.POINTER(ctypes.c_void_p), i32, ctypes.POINTER(pdi_params),
                                            ctypes.POINTER(ctypes.c_void_p), P]
        L.decode_residual_batch.restype = i32
        L.decode_residual_batch_noalloc.argtypes = L.decode_residual_batch.argtypes
        L.decode_residual_batch_noalloc.restype = i32
        VP = ctypes.POINTER(ctypes.c_void_p)
        L.decode_coefficients.argtypes = [P, ctypes.POINTER(pdi_frame), ctypes.POINTER(pdi_mask), P, P,
                                          ctypes.POINTER(pdi_coef_params), i32, ctypes.POINTER(pdi_params), P, P]
        L.decode_coefficients.restype = i32
        L.decode_coefficients_batch.argtypes = [P, i32, ctypes.POINTER(pdi_frame), ctypes.POINTER(pdi_mask), VP,
                                                VP, ctypes.POINTER(pdi_coef_params), i32,
                                                ctypes.POINTER(pdi_params), VP, P]
        L.decode_coefficients_batch.restype = i32
        L.encode_coefficients.argtypes = [P, ctypes.POINTER(pdi_frame), ctypes.POINTER(pdi_mask), P,
                                          ctypes.POINTER(pdi_coef_params), i32, ctypes.POINTER(pdi_params), P, P, P]
        L.encode_coefficients.restype = i32
        L.encode_coefficients_batch.argtypes = [P, i32, ctypes.POINTER(pdi_frame), ctypes.POINTER(pdi_mask), VP,
                                                ctypes.POINTER(pdi_coef_params), i32, ctypes.POINTER(pdi_params),
                                                VP, VP, P]
        L.encode_coefficients_batch.restype = i32
        L.pdi_default_select_params.argtypes = [ctypes.POINTER(pdi_select_params)]
        L.pdi_default_select_params.restype = None
        L.select_mask.argtypes = [P, ctypes.POINTER(pdi_frame), i32, P, i32, ctypes.POINTER(pdi_select_params),
                                  P, P, P, P]
        L.select_mask.restype = i32
        L.pdi_default_cg_params.argtypes = [ctypes.POINTER(pdi_cg_params)]
        L.pdi_default_cg_params.restype = None
        L.inpaint_homogeneous.argtypes = [P, i32, i32, P, P, ctypes.POINTER(pdi_cg_params), P, P,
                                          ctypes.POINTER(ctypes.c_int32)]
        L.inpaint_homogeneous.restype = i32
        L.pdi_sync.argtypes = [P, P]
        L.pdi_sync.restype = i32
        L.pdi_last_error.argtypes = [P]
        L.pdi_last_error.restype = ctypes.c_char_p
        L.pdi_frame_info.argtypes = [ctypes.POINTER(pdi_frame), i32, i32, ctypes.POINTER(ctypes.c_int32), i64p]
        L.pdi_frame_info.restype = i32
        L.pdi_pack_dense.argtypes = [ctypes.POINTER(pdi_frame), P, P, i32, i32, P, P, i64p, P, i64p]
        L.pdi_pack_dense.restype = i32
        L.pdi_validate_host.argtypes = [ctypes.POINTER(pdi_frame), i32, P, P, ctypes.c_int32,
                                        ctypes.c_int32, P]
        L.pdi_validate_host.restype = i32
        L.pdi_autotune.argtypes = [P, ctypes.POINTER(pdi_frame), ctypes.POINTER(pdi_mask), P, i32,
                                   ctypes.POINTER(pdi_params), P, P, ctypes.POINTER(ctypes.c_int)]
        L.pdi_autotune.restype = i32
        L.pdi_autotune_batch.argtypes = [P, i32, ctypes.POINTER(pdi_frame), ctypes.POINTER(pdi_mask),
                                         ctypes.POINTER(ctypes.c_void_p), i32, ctypes.POINTER(pdi_params),
                                         ctypes.POINTER(ctypes.c_void_p), P, ctypes.POINTER(ctypes.c_int)]
        L.pdi_autotune_batch.restype = i32
        PP = ctypes.POINTER(ctypes.c_void_p)
        L.pdi_seq_create.argtypes = [P, i32, ctypes.POINTER(pdi_frame), ctypes.POINTER(pdi_mask), PP, i32,
                                     ctypes.POINTER(pdi_params), PP, i32, PP]
        L.pdi_seq_create.restype = i32
        L.pdi_seq_launch.argtypes = [P, P]
        L.pdi_seq_launch.restype = i32
        L.pdi_seq_sync.argtypes = [P, P]
        L.pdi_seq_sync.restype = i32
        L.pdi_seq_destroy.argtypes = [P]
        L.pdi_seq_destroy.restype = None
        L.pdi_server_create.argtypes = [P, i32, ctypes.c_size_t, i32, PP]
        L.pdi_server_create.restype = i32
        L.pdi_submit.argtypes = [P, ctypes.POINTER(pdi_frame), ctypes.POINTER(pdi_mask), P, ctypes.c_int64,
                                 i32, ctypes.POINTER(pdi_params), P, P, i64p]
        L.pdi_submit.restype = i32
        L.pdi_poll.argtypes = [P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
        L.pdi_poll.restype = i32
        L.pdi_wait.argtypes = [P, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]
        L.pdi_wait.restype = i32
        L.pdi_server_stats.argtypes = [P, i64p, i64p, ctypes.POINTER(ctypes.c_size_t),
                                       ctypes.POINTER(ctypes.c_size_t)]
        L.pdi_server_stats.restype = i32
        L.pdi_server_hold.argtypes = [P, i32]
        L.pdi_server_hold.restype = i32
        L.pdi_server_destroy.argtypes = [P]
        L.pdi_server_destroy.restype = None
        _lib = L
    return _lib


def default_params(**kw) -> pdi_params:
    p = pdi_params()
    lib().pdi_default_params(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def pdi_create(device: int = 0, hbm_budget_bytes: int = 0) -> int:
    h = ctypes.c_void_p()
    rc = lib().pdi_create(ctypes.byref(h), device, hbm_budget_bytes)
    if rc != PDI_OK:
        raise PdiError(rc, "pdi_create")
    return h.value


def pdi_destroy(ctx: int) -> None:
    lib().pdi_destroy(ctx)


def pdi_last_error(ctx: int) -> str:
    return lib().pdi_last_error(ctx).decode()


def decode_residual(ctx: int, width: int, height: int, fmt: int, block_ptr: int, pos: int,
                    n_mask_blocks: int, chroma_shared: bool, values: int, block_size: int,
                    params: Optional[pdi_params], out: int, stream: int = 0) -> int:
    """Raw call: all buffer arguments are device addresses (ints)."""
    fr = pdi_frame(width, height, fmt)
    mk = pdi_mask(block_ptr, pos, n_mask_blocks, int(bool(chroma_shared)))
    return lib().decode_residual(ctx, ctypes.byref(fr), ctypes.byref(mk), values, block_size,
                                 ctypes.byref(params) if params is not None else None, out, stream)


def pdi_sync(ctx: int, stream: int = 0) -> int:
    return lib().pdi_sync(ctx, stream)


def pdi_frame_info(width: int, height: int, fmt: int, block_size: int, chroma_shared: bool):
    fr = pdi_frame(width, height, fmt)
    n = ctypes.c_int32()
    e = ctypes.c_int64()
    rc = lib().pdi_frame_info(ctypes.byref(fr), block_size, int(bool(chroma_shared)),
                              ctypes.byref(n), ctypes.byref(e))
    return rc, n.value, e.value


def pdi_validate_host(width, height, fmt, block_size, block_ptr, pos, chroma_shared, values) -> int:
    """block_ptr / pos / values are numpy arrays (host)."""
    import numpy as np
    bp = np.ascontiguousarray(block_ptr, dtype=np.int32)
    ps = np.ascontiguousarray(pos, dtype=np.uint16)
    vs = np.ascontiguousarray(values, dtype=np.float32)
    fr = pdi_frame(width, height, fmt)
    return lib().pdi_validate_host(ctypes.byref(fr), block_size, bp.ctypes.data, ps.ctypes.data,
                                   int(bp.size - 1), int(bool(chroma_shared)), vs.ctypes.data)


def pdi_pack_dense(width, height, fmt, block_size, chroma_shared, m, f):
    """Host packing of dense masks/planes (numpy) into (block_ptr, pos, values)."""
    import numpy as np
    rc, nb, nel = pdi_frame_info(width, height, fmt, block_size, chroma_shared)
    if rc != PDI_OK:
        raise PdiError(rc, "pdi_frame_info")
    m = np.ascontiguousarray(m, dtype=np.uint8)
    f = np.ascontiguousarray(f, dtype=np.float32)
    bp = np.zeros(nb + 1, np.int32)
    cap = int(m.size)
    pos = np.zeros(max(cap, 1), np.uint16)
    vals = np.zeros(max(2 * cap, 1), np.float32)
    pc, vc = ctypes.c_int64(pos.size), ctypes.c_int64(vals.size)
    fr = pdi_frame(width, height, fmt)
    rc = lib().pdi_pack_dense(ctypes.byref(fr), m.ctypes.data, f.ctypes.data, block_size,
                              int(bool(chroma_shared)), bp.ctypes.data, pos.ctypes.data,
                              ctypes.byref(pc), vals.ctypes.data, ctypes.byref(vc))
    if rc != PDI_OK:
        raise PdiError(rc, "pdi_pack_dense")
    return bp, pos[:pc.value].copy(), vals[:vc.value].copy()


class Decoder:
    """Convenience wrapper: a context plus torch device buffers for frames."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        import torch  # device memory and streams only
        self.torch = torch
        self.device = device
        self.ctx = pdi_create(device, hbm_budget_bytes)

    def close(self):
        if self.ctx:
            pdi_destroy(self.ctx)
            self.ctx = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def upload(self, frame):
        """Copy a packed frame (synth.Frame-like) to the device; returns a dict."""
        import numpy as np
        torch = self.torch
        dev = torch.device("cuda", self.device)
        bp = torch.from_numpy(np.ascontiguousarray(frame.block_ptr, np.int32)).to(dev)
        pos = np.ascontiguousarray(frame.pos, np.uint16).view(np.int16)
        pos_t = torch.from_numpy(pos if pos.size else np.zeros(1, np.int16)).to(dev)
        vals = np.ascontiguousarray(frame.values, np.float32)
        vals_t = torch.from_numpy(vals if vals.size else np.zeros(1, np.float32)).to(dev)
        rc, nb, nel = pdi_frame_info(frame.width, frame.height, frame.fmt, frame.block_size,
                                     frame.chroma_shared)
        out = torch.empty(nel, dtype=torch.float32, device=dev)
        out_i8 = torch.empty(nel, dtype=torch.int8, device=dev)
        return dict(frame=frame, block_ptr=bp, pos=pos_t, values=vals_t, out=out, out_i8=out_i8,
                    n_mask_blocks=int(frame.block_ptr.shape[0] - 1))

    def upload_coef(self, frame, coef, consts):
        """upload() plus stored-coefficient inputs: int8 codes (laid out like
        the values) and one FP32 constant per block of every plane."""
        import numpy as np
        torch = self.torch
        dev = torch.device("cuda", self.device)
        d = self.upload(frame)
        q = np.ascontiguousarray(coef, np.int8)
        d["coef"] = torch.from_numpy(q if q.size else np.zeros(1, np.int8)).to(dev)
        cs = np.ascontiguousarray(consts, np.float32)
        d["consts"] = torch.from_numpy(cs if cs.size else np.zeros(1, np.float32)).to(dev)
        return d

    def select(self, width: int, height: int, fmt: int, planes, chroma_shared: bool = True,
               sp: Optional[pdi_select_params] = None, stream=None, check=True):
        """select_mask on dense residual planes (a device FP32 tensor in the
        decode output layout, or host arrays to upload).  Returns (rc, d):
        d holds the geometry, the planes and the packed outputs on the
        device (block_ptr, pos, values, sized for every pixel), ready once
        the stream has run the call."""
        import numpy as np
        torch = self.torch
        dev = torch.device("cuda", self.device)
        rc, nb, nel = pdi_frame_info(width, height, fmt, 8, chroma_shared)
        if isinstance(planes, torch.Tensor):
            pl = planes
        else:
            pl = torch.from_numpy(np.ascontiguousarray(
                np.concatenate([np.asarray(p, np.float32).ravel() for p in planes]))).to(dev)
        nmask = width * height if fmt == 0 else (
            width * height + ((width + 1) // 2) * ((height + 1) // 2) * (1 if chroma_shared else 2))
        bp = torch.zeros(nb + 1, dtype=torch.int32, device=dev)
        pos = torch.zeros(max(nmask, 1), dtype=torch.int16, device=dev)
        vals = torch.zeros(max(nel, 1), dtype=torch.float32, device=dev)
        s = stream.cuda_stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        f = pdi_frame(width, height, fmt)
        rc = lib().select_mask(self.ctx, ctypes.byref(f), int(bool(chroma_shared)), pl.data_ptr(), 8,
                               ctypes.byref(sp) if sp is not None else None, bp.data_ptr(), pos.data_ptr(),
                               vals.data_ptr(), s)
        if check and rc != PDI_OK:
            raise PdiError(rc, pdi_last_error(self.ctx))
        return rc, dict(width=width, height=height, fmt=fmt, chroma_shared=bool(chroma_shared), planes=pl,
                        block_ptr=bp, pos=pos, values=vals, n_mask_blocks=nb)

    def alloc_coef(self, d):
        """Add device buffers for an encode's outputs to a frame from upload():
        int8 codes laid out like the values ("coef") and one FP32 constant
        per block of every plane ("consts"), as upload_coef holds them."""
        torch = self.torch
        dev = torch.device("cuda", self.device)
        fr = d["frame"]
        d["coef"] = torch.zeros(max(int(d["values"].numel()), 1), dtype=torch.int8, device=dev)
        d["consts"] = torch.zeros(max(int(self.plane_blocks(fr)), 1), dtype=torch.float32, device=dev)
        return d

    @staticmethod
    def plane_blocks(fr) -> int:
        """Blocks of every plane (the length of the constants array)."""
        b = fr.block_size
        dims = [(fr.width, fr.height)]
        if fr.fmt != 0:
            dims += [((fr.width + 1) // 2, (fr.height + 1) // 2)] * 2
        return sum(((W + b - 1) // b) * ((H + b - 1) // b) for W, H in dims)

    def encode_coef(self, d, qp: pdi_coef_params, params: Optional[pdi_params] = None, stream=None,
                    check=True) -> int:
        """encode_coefficients on a frame from upload() + alloc_coef(): codes
        into d["coef"], constants into d["consts"]."""
        fr = d["frame"]
        s = stream.cuda_stream if stream is not None else self.torch.cuda.current_stream(self.device).cuda_stream
        f = pdi_frame(fr.width, fr.height, fr.fmt)
        mk = pdi_mask(d["block_ptr"].data_ptr(), d["pos"].data_ptr(), d["n_mask_blocks"], int(bool(fr.chroma_shared)))
        rc = lib().encode_coefficients(self.ctx, ctypes.byref(f), ctypes.byref(mk), d["values"].data_ptr(),
                                       ctypes.byref(qp) if qp is not None else None, fr.block_size,
                                       ctypes.byref(params) if params is not None else None,
                                       d["coef"].data_ptr(), d["consts"].data_ptr(), s)
        if check and rc != PDI_OK:
            raise PdiError(rc, pdi_last_error(self.ctx))
        return rc

    def encode_coef_batch(self, ds, qp: pdi_coef_params, params: Optional[pdi_params] = None, stream=None,
                          check=True) -> int:
        """encode_coefficients_batch over frames from upload() + alloc_coef() (one geometry)."""
        n = len(ds)
        f0 = ds[0]["frame"]
        fr = pdi_frame(f0.width, f0.height, f0.fmt)
        masks = (pdi_mask * n)()
        vs = (ctypes.c_void_p * n)()
        qs = (ctypes.c_void_p * n)()
        cs = (ctypes.c_void_p * n)()
        for k, d in enumerate(ds):
            f = d["frame"]
            masks[k] = pdi_mask(d["block_ptr"].data_ptr(), d["pos"].data_ptr(), d["n_mask_blocks"],
                                int(bool(f.chroma_shared)))
            vs[k] = d["values"].data_ptr()
            qs[k] = d["coef"].data_ptr()
            cs[k] = d["consts"].data_ptr()
        s = stream.cuda_stream if stream is not None else self.torch.cuda.current_stream(self.device).cuda_stream
        rc = lib().encode_coefficients_batch(self.ctx, n, ctypes.byref(fr), masks, vs,
                                             ctypes.byref(qp) if qp is not None else None, f0.block_size,
                                             ctypes.byref(params) if params is not None else None, qs, cs, s)
        if check and rc != PDI_OK:
            raise PdiError(rc, pdi_last_error(self.ctx))
        return rc

    def decode_coef(self, d, qp: pdi_coef_params, params: Optional[pdi_params] = None, stream=None,
                    check=True) -> int:
        """decode_coefficients on a frame from upload_coef."""
        fr = d["frame"]
        out = d["out_i8"] if (params is not None and params.out_int8) else d["out"]
        s = stream.cuda_stream if stream is not None else self.torch.cuda.current_stream(self.device).cuda_stream
        f = pdi_frame(fr.width, fr.height, fr.fmt)
        mk = pdi_mask(d["block_ptr"].data_ptr(), d["pos"].data_ptr(), d["n_mask_blocks"], int(bool(fr.chroma_shared)))
        rc = lib().decode_coefficients(self.ctx, ctypes.byref(f), ctypes.byref(mk), d["coef"].data_ptr(),
                                       d["consts"].data_ptr(), ctypes.byref(qp) if qp is not None else None,
                                       fr.block_size, ctypes.byref(params) if params is not None else None,
                                       out.data_ptr(), s)
        if check and rc != PDI_OK:
            raise PdiError(rc, pdi_last_error(self.ctx))
        return rc

    def decode_coef_batch(self, ds, qp: pdi_coef_params, params: Optional[pdi_params] = None, stream=None,
                          check=True) -> int:
        """decode_coefficients_batch over frames from upload_coef (one geometry)."""
        n = len(ds)
        f0 = ds[0]["frame"]
        fr = pdi_frame(f0.width, f0.height, f0.fmt)
        masks = (pdi_mask * n)()
        qs = (ctypes.c_void_p * n)()
        cs = (ctypes.c_void_p * n)()
        outs = (ctypes.c_void_p * n)()
        i8 = params is not None and params.out_int8
        for k, d in enumerate(ds):
            f = d["frame"]
            masks[k] = pdi_mask(d["block_ptr"].data_ptr(), d["pos"].data_ptr(), d["n_mask_blocks"],
                                int(bool(f.chroma_shared)))
            qs[k] = d["coef"].data_ptr()
            cs[k] = d["consts"].data_ptr()
            outs[k] = (d["out_i8"] if i8 else d["out"]).data_ptr()
        s = stream.cuda_stream if stream is not None else self.torch.cuda.current_stream(self.device).cuda_stream
        rc = lib().decode_coefficients_batch(self.ctx, n, ctypes.byref(fr), masks, qs, cs,
                                             ctypes.byref(qp) if qp is not None else None, f0.block_size,
                                             ctypes.byref(params) if params is not None else None, outs, s)
        if check and rc != PDI_OK:
            raise PdiError(rc, pdi_last_error(self.ctx))
        return rc

    def inpaint(self, mask, f, cp: Optional[pdi_cg_params] = None, stream=None, check=True, u=None):
        """inpaint_homogeneous on a (H, W) mask (bool) and values; returns
        (rc, u device tensor, finest-level iterations).  mask / f may be numpy
        arrays (copied to the device) or device tensors (uint8 / float32)."""
        import numpy as np
        torch = self.torch
        dev = torch.device("cuda", self.device)
        if not torch.is_tensor(mask):
            mask = torch.from_numpy(np.ascontiguousarray(mask, dtype=np.uint8)).to(dev)
        if not torch.is_tensor(f):
            f = torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32)).to(dev)
        H, W = mask.shape
        if u is None:
            u = torch.empty((H, W), dtype=torch.float32, device=dev)
        s = stream.cuda_stream if stream is not None else self.torch.cuda.current_stream(self.device).cuda_stream
        its = ctypes.c_int32()
        rc = lib().inpaint_homogeneous(self.ctx, W, H, mask.data_ptr(), f.data_ptr(),
                                       ctypes.byref(cp) if cp is not None else None, u.data_ptr(), s,
                                       ctypes.byref(its))
        if check and rc != PDI_OK:
            raise PdiError(rc, pdi_last_error(self.ctx))
        return rc, u, its.value

    def decode(self, d, params: Optional[pdi_params] = None, stream=None, out=None, check=True) -> int:
        fr = d["frame"]
        if out is None:
            out = d["out_i8"] if (params is not None and params.out_int8) else d["out"]
        s = stream.cuda_stream if stream is not None else self.torch.cuda.current_stream(self.device).cuda_stream
        rc = decode_residual(self.ctx, fr.width, fr.height, fr.fmt, d["block_ptr"].data_ptr(),
                             d["pos"].data_ptr(), d["n_mask_blocks"], fr.chroma_shared,
                             d["values"].data_ptr(), fr.block_size, params, out.data_ptr(), s)
        if check and rc != PDI_OK:
            raise PdiError(rc, pdi_last_error(self.ctx))
        return rc

    def sync(self, stream=None) -> int:
        s = stream.cuda_stream if stream is not None else self.torch.cuda.current_stream(self.device).cuda_stream
        return pdi_sync(self.ctx, s)

    def decode_batch(self, ds, params: Optional[pdi_params] = None, stream=None, check=True) -> int:
        """decode_residual_batch over uploaded frames of one geometry."""
        n = len(ds)
        f0 = ds[0]["frame"]
        fr = pdi_frame(f0.width, f0.height, f0.fmt)
        masks = (pdi_mask * n)()
        vals = (ctypes.c_void_p * n)()
        outs = (ctypes.c_void_p * n)()
        i8 = params is not None and params.out_int8
        for k, d in enumerate(ds):
            f = d["frame"]
            masks[k] = pdi_mask(d["block_ptr"].data_ptr(), d["pos"].data_ptr(), d["n_mask_blocks"],
                                int(bool(f.chroma_shared)))
            vals[k] = d["values"].data_ptr()
            outs[k] = (d["out_i8"] if i8 else d["out"]).data_ptr()
        s = stream.cuda_stream if stream is not None else self.torch.cuda.current_stream(self.device).cuda_stream
        rc = lib().decode_residual_batch(self.ctx, n, ctypes.byref(fr), masks, vals, f0.block_size,
                                         ctypes.byref(params) if params is not None else None, outs, s)
        if check and rc != PDI_OK:
            raise PdiError(rc, pdi_last_error(self.ctx))
        return rc

    def decode_batch_noalloc(self, ds, params: Optional[pdi_params] = None, stream=None, check=True) -> int:
        """decode_residual_batch_noalloc over uploaded frames of one geometry
        (the library's static device scratch; nothing is allocated)."""
        n = len(ds)
        f0 = ds[0]["frame"]
        fr = pdi_frame(f0.width, f0.height, f0.fmt)
        masks = (pdi_mask * n)()
        vals = (ctypes.c_void_p * n)()
        outs = (ctypes.c_void_p * n)()
        i8 = params is not None and params.out_int8
        for k, d in enumerate(ds):
            f = d["frame"]
            masks[k] = pdi_mask(d["block_ptr"].data_ptr(), d["pos"].data_ptr(), d["n_mask_blocks"],
                                int(bool(f.chroma_shared)))
            vals[k] = d["values"].data_ptr()
            outs[k] = (d["out_i8"] if i8 else d["out"]).data_ptr()
        s = stream.cuda_stream if stream is not None else self.torch.cuda.current_stream(self.device).cuda_stream
        rc = lib().decode_residual_batch_noalloc(self.ctx, n, ctypes.byref(fr), masks, vals, f0.block_size,
                                                 ctypes.byref(params) if params is not None else None, outs, s)
        if check and rc != PDI_OK:
            raise PdiError(rc, pdi_last_error(self.ctx))
        return rc

    def autotune_batch(self, ds, params: Optional[pdi_params] = None, stream=None) -> int:
        """pdi_autotune_batch over uploaded frames of one geometry (the
        launch decode_batch makes); returns the launch choice."""
        n = len(ds)
        f0 = ds[0]["frame"]
        fr = pdi_frame(f0.width, f0.height, f0.fmt)
        masks = (pdi_mask * n)()
        vals = (ctypes.c_void_p * n)()
        outs = (ctypes.c_void_p * n)()
        i8 = params is not None and params.out_int8
        for k, d in enumerate(ds):
            f = d["frame"]
            masks[k] = pdi_mask(d["block_ptr"].data_ptr(), d["pos"].data_ptr(), d["n_mask_blocks"],
                                int(bool(f.chroma_shared)))
            vals[k] = d["values"].data_ptr()
            outs[k] = (d["out_i8"] if i8 else d["out"]).data_ptr()
        s = stream.cuda_stream if stream is not None else self.torch.cuda.current_stream(self.device).cuda_stream
        ch = ctypes.c_int()
        rc = lib().pdi_autotune_batch(self.ctx, n, ctypes.byref(fr), masks, vals, f0.block_size,
                                      ctypes.byref(params) if params is not None else None, outs, s,
                                      ctypes.byref(ch))
        if rc != PDI_OK:
            raise PdiError(rc, pdi_last_error(self.ctx))
        return ch.value

    def autotune(self, d, params: Optional[pdi_params] = None, stream=None) -> int:
        """pdi_autotune on an uploaded frame; returns the launch choice."""
        fr = d["frame"]
        s = stream.cuda_stream if stream is not None else self.torch.cuda.current_stream(self.device).cuda_stream
        f = pdi_frame(fr.width, fr.height, fr.fmt)
        mk = pdi_mask(d["block_ptr"].data_ptr(), d["pos"].data_ptr(), d["n_mask_blocks"], int(bool(fr.chroma_shared)))
        ch = ctypes.c_int()
        rc = lib().pdi_autotune(self.ctx, ctypes.byref(f), ctypes.byref(mk), d["values"].data_ptr(), fr.block_size,
                                ctypes.byref(params) if params is not None else None, d["out"].data_ptr(), s,
                                ctypes.byref(ch))
        if rc != PDI_OK:
            raise PdiError(rc, pdi_last_error(self.ctx))
        return ch.value


class Sequence:
    """pdi_seq: the decodes of n same-geometry frames captured into one HIP
    graph over ``nstreams`` internal streams.  ``frames`` are device dicts
    from ``Decoder.upload``; replays read their current buffer contents."""

    def __init__(self, dec: "Decoder", frames, params: Optional[pdi_params] = None, nstreams: int = 4):
        self.dec = dec
        self.frames = list(frames)
        n = len(self.frames)
        f0 = self.frames[0]["frame"]
        fr = pdi_frame(f0.width, f0.height, f0.fmt)
        masks = (pdi_mask * n)()
        vals = (ctypes.c_void_p * n)()
        outs = (ctypes.c_void_p * n)()
        for k, d in enumerate(self.frames):
            f = d["frame"]
            if (f.width, f.height, f.fmt, f.block_size, f.chroma_shared) != \
                    (f0.width, f0.height, f0.fmt, f0.block_size, f0.chroma_shared):
                raise ValueError("a sequence holds frames of one geometry")
            masks[k] = pdi_mask(d["block_ptr"].data_ptr(), d["pos"].data_ptr(), d["n_mask_blocks"],
                                int(bool(f.chroma_shared)))
            vals[k] = d["values"].data_ptr()
            outs[k] = d["out"].data_ptr()
        h = ctypes.c_void_p()
        rc = lib().pdi_seq_create(dec.ctx, n, ctypes.byref(fr), masks, vals, f0.block_size,
                                  ctypes.byref(params) if params is not None else None, outs, nstreams,
                                  ctypes.byref(h))
        if rc != PDI_OK:
            raise PdiError(rc, pdi_last_error(dec.ctx))
        self.handle = h.value

    def launch(self, stream=None) -> int:
        s = stream.cuda_stream if stream is not None else self.dec.torch.cuda.current_stream(self.dec.device).cuda_stream
        return lib().pdi_seq_launch(self.handle, s)

    def sync(self, stream=None) -> int:
        s = stream.cuda_stream if stream is not None else self.dec.torch.cuda.current_stream(self.dec.device).cuda_stream
        return lib().pdi_seq_sync(self.handle, s)

    def close(self):
        if getattr(self, "handle", None):
            lib().pdi_seq_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """pdi_server: continuous-batching request loop over ``nlanes`` streams.
    ``submit`` takes a host frame (synth.Frame-like, numpy arrays)."""

    def __init__(self, dec: "Decoder", nlanes: int = 4, hbm_budget_bytes: int = 0, max_queue: int = 1024):
        self.dec = dec
        h = ctypes.c_void_p()
        rc = lib().pdi_server_create(dec.ctx, nlanes, hbm_budget_bytes, max_queue, ctypes.byref(h))
        if rc != PDI_OK:
            raise PdiError(rc, "pdi_server_create")
        self.handle = h.value
        self._keep = {}

    def submit(self, frame, params: Optional[pdi_params] = None, want_output: bool = True, out_dev=None):
        """Returns (rc, ticket, out): ``out`` is the host array that ``wait``
        fills (None unless want_output); ``out_dev`` is an optional device
        tensor the decode writes into."""
        import numpy as np
        bp = np.ascontiguousarray(frame.block_ptr, np.int32)
        pos = np.ascontiguousarray(frame.pos, np.uint16)
        vals = np.ascontiguousarray(frame.values, np.float32)
        rc, nb, nel = pdi_frame_info(frame.width, frame.height, frame.fmt, frame.block_size, frame.chroma_shared)
        i8 = params is not None and params.out_int8
        out = np.empty(nel, np.int8 if i8 else np.float32) if want_output else None
        fr = pdi_frame(frame.width, frame.height, frame.fmt)
        mk = pdi_mask(bp.ctypes.data, pos.ctypes.data if pos.size else None, int(bp.size - 1),
                      int(bool(frame.chroma_shared)))
        t = ctypes.c_int64()
        rc = lib().pdi_submit(self.handle, ctypes.byref(fr), ctypes.byref(mk), vals.ctypes.data, int(vals.size),
                              frame.block_size, ctypes.byref(params) if params is not None else None,
                              out.ctypes.data if out is not None else None,
                              out_dev.data_ptr() if out_dev is not None else None, ctypes.byref(t))
        if rc == PDI_OK:
            self._keep[t.value] = (out, out_dev)
        return rc, t.value, out

    def poll(self, ticket: int):
        done = ctypes.c_int()
        lat = ctypes.c_double()
        rc = lib().pdi_poll(self.handle, ticket, ctypes.byref(done), ctypes.byref(lat))
        return rc, bool(done.value), lat.value

    def wait(self, ticket: int):
        lat = ctypes.c_double()
        rc = lib().pdi_wait(self.handle, ticket, ctypes.byref(lat))
        self._keep.pop(ticket, None)
        return rc, lat.value

    def stats(self):
        q, r = ctypes.c_int64(), ctypes.c_int64()
        u, a = ctypes.c_size_t(), ctypes.c_size_t()
        lib().pdi_server_stats(self.handle, ctypes.byref(q), ctypes.byref(r), ctypes.byref(u), ctypes.byref(a))
        return dict(queued=q.value, running=r.value, bytes_in_use=u.value, bytes_allocated=a.value)

    def hold(self, on: bool = True) -> int:
        return lib().pdi_server_hold(self.handle, int(bool(on)))

    def close(self):
        if getattr(self, "handle", None):
            lib().pdi_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
