"""Python binding of libswalign with torch tensors as device memory.

Every function marshals pointers and sizes into one C entry point of
include/swalign.h and launches on the current torch stream; no step of the
computation runs in Python.  Inputs must be contiguous CUDA (HIP) tensors of
the stated dtypes."""
from __future__ import annotations

import ctypes

import torch

from . import _abi
from ._abi import check, sw_batch, sw_geom, sw_stack, sw_serve_cfg, sw_request, sw_serve_stats


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


def projection_plan(L: int, n: int):
    """sw_projection_plan (host only, no context): the projection work plan
    of (L, n) as numpy arrays: perm [ntasks, 64] (item = slot * L + bin, or
    -1) and rows [ntasks, 2] (first and last image row each task reads)."""
    import numpy as np

    lib = _abi.load()
    nt = ctypes.c_int32(0)
    check(lib.sw_projection_plan(int(L), int(n), 0, None, None, None, ctypes.byref(nt)))
    perm = np.empty((nt.value, 64), np.int32)
    lo = np.empty(nt.value, np.int32)
    hi = np.empty(nt.value, np.int32)
    check(lib.sw_projection_plan(int(L), int(n), nt.value, perm.ctypes.data, lo.ctypes.data,
                                 hi.ctypes.data, ctypes.byref(nt)))
    return perm, np.stack([lo, hi], axis=1)


def project(ctx: Context, imgs: torch.Tensor, n: int, stream=None, out=None):
    """sw_project: [N, L, L] float32 -> [N, n, L] float32 projections."""
    _need(imgs, torch.float32, "imgs")
    N, L = imgs.shape[0], imgs.shape[-1]
    g = geom(L, n, 8)
    pmf = out if out is not None else torch.empty((N, n, L), dtype=torch.float32, device=imgs.device)
    check(ctx._lib.sw_project(ctx.handle, _ptr(imgs), N, ctypes.byref(g), _ptr(pmf), _stream(stream)))
    return pmf


def _angles(theta, n):
    import numpy as np

    th = np.ascontiguousarray(theta, dtype=np.float64)
    if th.shape != (n,):
        raise ValueError(f"theta must hold n = {n} angles, got shape {th.shape}")
    return th, th.ctypes.data_as(ctypes.c_void_p)


def project_fourier(ctx: Context, imgs: torch.Tensor, n: int, stream=None, out=None, theta=None):
    """sw_project_fourier: [N, L, L] float32 -> [N, n, L] float32 projections
    by the Fourier slice theorem (L even, prime factors 2 and 3); with theta (n radians,
    host) sw_project_fourier_at at those directions."""
    _need(imgs, torch.float32, "imgs")
    N, L = imgs.shape[0], imgs.shape[-1]
    g = geom(L, n, 8)
    pmf = out if out is not None else torch.empty((N, n, L), dtype=torch.float32, device=imgs.device)
    if theta is None:
        check(ctx._lib.sw_project_fourier(ctx.handle, _ptr(imgs), N, ctypes.byref(g), _ptr(pmf),
                                          _stream(stream)))
    else:
        th, tp = _angles(theta, n)
        check(ctx._lib.sw_project_fourier_at(ctx.handle, _ptr(imgs), N, ctypes.byref(g), tp,
                                             _ptr(pmf), _stream(stream)))
    return pmf


def tables_fourier(ctx: Context, imgs: torch.Tensor, n: int, Q: int, levels=_abi.LEVELS_MIDPOINT,
                   stream=None, out=None, aux=None, theta=None):
    """sw_tables_fourier: images to quantile tables [N, Q, n] through the
    Fourier-slice projector; with theta, sw_tables_fourier_at."""
    _need(imgs, torch.float32, "imgs")
    N, L = imgs.shape[0], imgs.shape[-1]
    g = geom(L, n, Q, levels)
    qt = out if out is not None else torch.empty((N, Q, n), dtype=torch.float32, device=imgs.device)
    ax = aux if aux is not None else torch.empty((N, 4), dtype=torch.float64, device=imgs.device)
    if theta is None:
        check(ctx._lib.sw_tables_fourier(ctx.handle, _ptr(imgs), N, ctypes.byref(g), _ptr(qt),
                                         _ptr(ax), _stream(stream)))
    else:
        th, tp = _angles(theta, n)
        check(ctx._lib.sw_tables_fourier_at(ctx.handle, _ptr(imgs), N, ctypes.byref(g), tp,
                                            _ptr(qt), _ptr(ax), _stream(stream)))
    return qt, ax


def ramp(ctx: Context, pmf: torch.Tensor, stream=None, out=None):
    """sw_ramp: [N, n, L] projections -> ramp-filtered (signed) [N, n, L]."""
    _need(pmf, torch.float32, "pmf")
    N, n, L = pmf.shape
    g = geom(L, n, 8)
    o = out if out is not None else torch.empty_like(pmf)
    check(ctx._lib.sw_ramp(ctx.handle, _ptr(pmf), N, ctypes.byref(g), _ptr(o), _stream(stream)))
    return o


def quantiles(ctx: Context, pmf: torch.Tensor, Q: int, levels=_abi.LEVELS_MIDPOINT, stream=None,
              out=None, aux=None, ramp=False):
    """sw_quantiles: [N, n, L] -> ([N, Q, n] float32, [N, 4] float64).
    ramp=True: sw_quantiles_rf on ramp-filtered projections -> [N, 2Q, n]."""
    _need(pmf, torch.float32, "pmf")
    N, n, L = pmf.shape
    g = geom(L, n, Q, levels)
    rows = 2 * Q if ramp else Q
    qt = out if out is not None else torch.empty((N, rows, n), dtype=torch.float32,
                                                 device=pmf.device)
    ax = aux if aux is not None else torch.empty((N, 4), dtype=torch.float64, device=pmf.device)
    fn = ctx._lib.sw_quantiles_rf if ramp else ctx._lib.sw_quantiles
    check(fn(ctx.handle, _ptr(pmf), N, ctypes.byref(g), _ptr(qt), _ptr(ax), _stream(stream)))
    return qt, ax


def tables(ctx: Context, imgs: torch.Tensor, n: int, Q: int, levels=_abi.LEVELS_MIDPOINT,
           stream=None, out=None, aux=None, ramp=False):
    """sw_tables: images straight to quantile tables (fused projection).
    ramp=True: sw_tables_rf, stacked ramp-filtered tables [N, 2Q, n]."""
    _need(imgs, torch.float32, "imgs")
    N, L = imgs.shape[0], imgs.shape[-1]
    g = geom(L, n, Q, levels)
    rows = 2 * Q if ramp else Q
    qt = out if out is not None else torch.empty((N, rows, n), dtype=torch.float32,
                                                 device=imgs.device)
    ax = aux if aux is not None else torch.empty((N, 4), dtype=torch.float64, device=imgs.device)
    fn = ctx._lib.sw_tables_rf if ramp else ctx._lib.sw_tables
    check(fn(ctx.handle, _ptr(imgs), N, ctypes.byref(g), _ptr(qt), _ptr(ax), _stream(stream)))
    return qt, ax


def make_batch(ref_qt, ref_aux, img_qt, img_aux, L, pairs=None, mode=_abi.MODE_ROT_TRANS,
               prec=_abi.PREC_FP32, top_k=0, levels=_abi.LEVELS_MIDPOINT, ramp=False):
    _need(ref_qt, torch.float32, "ref_qt")
    _need(img_qt, torch.float32, "img_qt")
    _need(ref_aux, torch.float64, "ref_aux")
    _need(img_aux, torch.float64, "img_aux")
    nr, rows, n = ref_qt.shape
    Q = rows // 2 if ramp else rows
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
    b.filter = _abi.FILTER_RAMP if ramp else _abi.FILTER_NONE
    return b, P


def align_batch(ctx: Context, ref_qt, ref_aux, img_qt, img_aux, L, pairs=None,
                mode=_abi.MODE_ROT_TRANS, prec=_abi.PREC_FP32, top_k=0, want_curve=False,
                levels=_abi.LEVELS_MIDPOINT, stream=None, out=None, ramp=False, noalloc=False,
                curve_out=None):
    """sw_align_batch (noalloc=True: sw_align_batch_noalloc).  Returns the raw
    [P, 6] int32 result records (see `unpack_results`) and the [P, n] curve
    when requested (into curve_out when given).  ramp=True: the tables are
    stacked ramp-filtered tables and sw2sq is the ramp-filtered distance."""
    b, P = make_batch(ref_qt, ref_aux, img_qt, img_aux, L, pairs, mode, prec, top_k, levels,
                      ramp)
    dev = img_qt.device
    res = out if out is not None else torch.empty((P, 6), dtype=torch.int32, device=dev)
    curve = curve_out
    if want_curve and curve is None:
        curve = torch.empty((P, b.geom.n_angles), dtype=torch.float32, device=dev)
    fn = ctx._lib.sw_align_batch_noalloc if noalloc else ctx._lib.sw_align_batch
    check(fn(ctx.handle, ctypes.byref(b), _ptr(res), _ptr(curve), _stream(stream)))
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


def align_stacks(ctx: Context, stacks, n=None, Q=None, mode=_abi.MODE_ROT_TRANS,
                 prec=_abi.PREC_FP32, top_k=0, levels=_abi.LEVELS_MIDPOINT, stream=None):
    """sw_align_stacks over a list of (ref_img [L, L], imgs [N, L, L]) device
    tensors; n and Q default to L per stack.  Returns per stack a dict with
    the raw [N, 6] result records and the tables."""
    descs = (sw_stack * len(stacks))()
    keep = []
    for i, (ref, imgs) in enumerate(stacks):
        _need(ref, torch.float32, "ref_img")
        _need(imgs, torch.float32, "imgs")
        N, L = imgs.shape[0], imgs.shape[-1]
        nn = n if n is not None else L
        qq = Q if Q is not None else L
        dev = imgs.device
        o = {"ref_qt": torch.empty((qq, nn), dtype=torch.float32, device=dev),
             "ref_aux": torch.empty((4,), dtype=torch.float64, device=dev),
             "qt": torch.empty((N, qq, nn), dtype=torch.float32, device=dev),
             "aux": torch.empty((N, 4), dtype=torch.float64, device=dev),
             "res": torch.empty((N, 6), dtype=torch.int32, device=dev), "L": L}
        d = descs[i]
        d.ref_img, d.imgs, d.N = ref.data_ptr(), imgs.data_ptr(), N
        d.geom = geom(L, nn, qq, levels)
        d.ref_qt, d.ref_aux = o["ref_qt"].data_ptr(), o["ref_aux"].data_ptr()
        d.qt, d.aux, d.out = o["qt"].data_ptr(), o["aux"].data_ptr(), o["res"].data_ptr()
        keep.append(o)
    check(ctx._lib.sw_align_stacks(ctx.handle, descs, len(stacks), int(mode), int(prec),
                                   int(top_k), _stream(stream)))
    return keep


def autotune(ctx: Context, Ls, n_images=2048, out_json=None):
    arr = (ctypes.c_int32 * len(Ls))(*[int(x) for x in Ls])
    check(ctx._lib.sw_autotune(ctx.handle, arr, len(Ls), int(n_images),
                               None if out_json is None else out_json.encode()))


class Server:
    """Continuous-batching server on a context (sw_serve_*).  Requests hold
    host numpy arrays that must stay alive until polled or cancelled; this
    wrapper keeps a reference to them."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, max_slots=64, prec=_abi.PREC_BF16_SPLIT,
                 top_k=0, mode=_abi.MODE_ROT_TRANS, max_queue=4096, use_graphs=True,
                 max_per_step=0):
        self.ctx = ctx
        cfg = sw_serve_cfg(int(hbm_budget_bytes), int(max_slots), int(prec), int(top_k), int(mode),
                           int(max_queue), 1 if use_graphs else 0, int(max_per_step))
        check(ctx._lib.sw_serve_start(ctx.handle, ctypes.byref(cfg)))
        self._live = {}

    def submit(self, ref_img, imgs, n=None, Q=None, ref_key=0, levels=_abi.LEVELS_MIDPOINT):
        import numpy as np

        ref_img = np.ascontiguousarray(ref_img, dtype=np.float32)
        imgs = np.ascontiguousarray(imgs, dtype=np.float32)
        if imgs.ndim != 3 or imgs.shape[1] != imgs.shape[2]:
            raise ValueError(f"imgs must be [N, L, L], got shape {imgs.shape}")
        N, L = imgs.shape[0], imgs.shape[-1]
        if ref_img.shape != (L, L):
            raise ValueError(f"ref_img must be [{L}, {L}], got shape {ref_img.shape}")
        req = sw_request(ref_img.ctypes.data, imgs.ctypes.data, N,
                         geom(L, n or L, Q or L, levels), int(ref_key))
        t = ctypes.c_uint64()
        check(self.ctx._lib.sw_serve_submit(self.ctx.handle, ctypes.byref(req), ctypes.byref(t)))
        self._live[t.value] = (ref_img, imgs, N)
        return t.value

    def poll(self, ticket):
        """None while not ready, else the [N, 6] int32 result records (numpy)."""
        import numpy as np

        N = self._live[ticket][2] if ticket in self._live else 0
        out = np.zeros((N, 6), dtype=np.int32)
        st = self.ctx._lib.sw_serve_poll(self.ctx.handle, ctypes.c_uint64(ticket),
                                         out.ctypes.data_as(ctypes.c_void_p) if N else None)
        if st == _abi.SW_NOT_READY:
            return None
        self._live.pop(ticket, None)
        check(st)
        return out

    def cancel(self, ticket):
        check(self.ctx._lib.sw_serve_cancel(self.ctx.handle, ctypes.c_uint64(ticket)))
        self._live.pop(ticket, None)

    def stats(self):
        s = sw_serve_stats()
        check(self.ctx._lib.sw_serve_stats_get(self.ctx.handle, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in s._fields_}

    def stop(self):
        check(self.ctx._lib.sw_serve_stop(self.ctx.handle))
        self._live.clear()


def records_to_dict(rec):
    """[P, 6] int32 numpy records -> dict of arrays."""
    import numpy as np

    rec = np.asarray(rec, dtype=np.int32)
    f = rec.view(np.float32)
    return {"rot_index": rec[:, 0].copy(), "theta_rad": f[:, 1].copy(),
            "shift_px": f[:, 2:4].copy(), "sw2sq": f[:, 4].copy(), "status": rec[:, 5].copy()}
