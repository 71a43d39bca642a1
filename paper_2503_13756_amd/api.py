"""Python binding of libswalign with torch tensors as device memory.

Every function marshals pointers and sizes into one C entry point of
include/swalign.h and launches on the current torch stream; no step of the
computation runs in Python.  Inputs must be contiguous CUDA (HIP) tensors of
the stated dtypes."""
from __future__ import annotations

import ctypes

import torch

from . import _abi
from ._abi import check, sw_batch, sw_geom


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _need(t, dtype, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Context:
    """Owns a library context (device binding and scratch)."""

    def __init__(self, device: int = 0, tune_json: str | None = None):
        self._lib = _abi.load()
        h = ctypes.c_void_p()
        check(self._lib.sw_ctx_create(ctypes.byref(h), device,
                                      None if tune_json is None else tune_json.encode()))
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            check(self._lib.sw_ctx_destroy(self.handle))
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def geom(L, n, Q, levels=_abi.LEVELS_MIDPOINT):
    return sw_geom(int(L), int(n), int(Q), int(levels))


def project(ctx: Context, imgs: torch.Tensor, n: int, stream=None, out=None):
    """sw_project: [N, L, L] float32 -> [N, n, L] float32 projections."""
    _need(imgs, torch.float32, "imgs")
    N, L = imgs.shape[0], imgs.shape[-1]
    g = geom(L, n, 8)
    pmf = out if out is not None else torch.empty((N, n, L), dtype=torch.float32, device=imgs.device)
    check(ctx._lib.sw_project(ctx.handle, _ptr(imgs), N, ctypes.byref(g), _ptr(pmf), _stream(stream)))
    return pmf


def quantiles(ctx: Context, pmf: torch.Tensor, Q: int, levels=_abi.LEVELS_MIDPOINT, stream=None,
              out=None, aux=None):
    """sw_quantiles: [N, n, L] -> ([N, Q, n] float32, [N, 4] float64)."""
    _need(pmf, torch.float32, "pmf")
    N, n, L = pmf.shape
    g = geom(L, n, Q, levels)
    qt = out if out is not None else torch.empty((N, Q, n), dtype=torch.float32, device=pmf.device)
    ax = aux if aux is not None else torch.empty((N, 4), dtype=torch.float64, device=pmf.device)
    check(ctx._lib.sw_quantiles(ctx.handle, _ptr(pmf), N, ctypes.byref(g), _ptr(qt), _ptr(ax),
                                _stream(stream)))
    return qt, ax


def tables(ctx: Context, imgs: torch.Tensor, n: int, Q: int, levels=_abi.LEVELS_MIDPOINT,
           stream=None, out=None, aux=None):
    """sw_tables: images straight to quantile tables (fused projection)."""
    _need(imgs, torch.float32, "imgs")
    N, L = imgs.shape[0], imgs.shape[-1]
    g = geom(L, n, Q, levels)
    qt = out if out is not None else torch.empty((N, Q, n), dtype=torch.float32, device=imgs.device)
    ax = aux if aux is not None else torch.empty((N, 4), dtype=torch.float64, device=imgs.device)
    check(ctx._lib.sw_tables(ctx.handle, _ptr(imgs), N, ctypes.byref(g), _ptr(qt), _ptr(ax),
                             _stream(stream)))
    return qt, ax


def make_batch(ref_qt, ref_aux, img_qt, img_aux, L, pairs=None, mode=_abi.MODE_ROT_TRANS,
               prec=_abi.PREC_FP32, top_k=0, levels=_abi.LEVELS_MIDPOINT):
    _need(ref_qt, torch.float32, "ref_qt")
    _need(img_qt, torch.float32, "img_qt")
    _need(ref_aux, torch.float64, "ref_aux")
    _need(img_aux, torch.float64, "img_aux")
    nr, Q, n = ref_qt.shape
    ni = img_qt.shape[0]
    b = sw_batch()
    b.ref_qt, b.ref_aux, b.n_ref = ref_qt.data_ptr(), ref_aux.data_ptr(), nr
    b.img_qt, b.img_aux, b.n_img = img_qt.data_ptr(), img_aux.data_ptr(), ni
    if pairs is not None:
        _need(pairs, torch.int64, "pairs")
        b.pairs, b.n_pairs = pairs.data_ptr(), pairs.shape[0]
        P = pairs.shape[0]
    else:
        b.pairs, b.n_pairs = None, 0
        P = nr * ni
    b.geom = geom(L, n, Q, levels)
    b.mode, b.prec, b.top_k = int(mode), int(prec), int(top_k)
    return b, P


def align_batch(ctx: Context, ref_qt, ref_aux, img_qt, img_aux, L, pairs=None,
                mode=_abi.MODE_ROT_TRANS, prec=_abi.PREC_FP32, top_k=0, want_curve=False,
                levels=_abi.LEVELS_MIDPOINT, stream=None, out=None):
    """sw_align_batch.  Returns the raw [P, 6] int32 result records (see
    `unpack_results`) and the [P, n] curve when requested."""
    b, P = make_batch(ref_qt, ref_aux, img_qt, img_aux, L, pairs, mode, prec, top_k, levels)
    dev = img_qt.device
    res = out if out is not None else torch.empty((P, 6), dtype=torch.int32, device=dev)
    curve = torch.empty((P, b.geom.n_angles), dtype=torch.float32, device=dev) if want_curve else None
    check(ctx._lib.sw_align_batch(ctx.handle, ctypes.byref(b), _ptr(res), _ptr(curve),
                                  _stream(stream)))
    return res, curve


def unpack_results(res: torch.Tensor):
    """[P, 6] int32 records -> dict of numpy arrays (host copy)."""
    r = res.detach().cpu()
    f = r.view(torch.float32)
    return {
        "rot_index": r[:, 0].numpy().copy(),
        "theta_rad": f[:, 1].numpy().copy(),
        "shift_px": f[:, 2:4].numpy().copy(),
        "sw2sq": f[:, 4].numpy().copy(),
        "status": r[:, 5].numpy().copy(),
    }
