"""Python entry to the FP64 CPU oracle (``sw_oracle.c``).

Test infrastructure only: the test suite, the smoke check and the CPU-baseline
leg of the benchmark use it; the product library never does.  It shares no
code with the GPU path.  Arrays are numpy; the C library is built with gcc on
first use if it is not there yet.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sw_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

LEVELS_MIDPOINT = 0
LEVELS_LEFT = 1
MODE_ROT_TRANS = 0
MODE_ROT_ONLY = 1
MODE_MAX_SLICED = 2
STATUS_OK = 0
STATUS_ZERO_MASS = 1
STATUS_NONFINITE = 2


def build(force: bool = False) -> str:
    """Compile the oracle with gcc -O2 -fopenmp (no SIMD intrinsics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
        lib.oracle_project.argtypes = [P, i64, i32, i32, P, P]
        lib.oracle_project.restype = None
        lib.oracle_quantiles.argtypes = [P, i64, i32, i32, i32, i32, P, P, P]
        lib.oracle_quantiles.restype = None
        lib.oracle_align.argtypes = [P, P, i64, P, P, i64, P, i64, i32, i32, i32, i32,
                                     P, P, P, P, P]
        lib.oracle_align.restype = None
        lib.oracle_align_rows.argtypes = [P, P, i64, P, P, i64, P, i64, i32, i32, i32, i32, i32,
                                          P, P, P, P, P, P]
        lib.oracle_align_rows.restype = None
        lib.oracle_ramp.argtypes = [P, i64, i32, i32, P]
        lib.oracle_ramp.restype = None
        lib.oracle_ramp_kernel.argtypes = [i32, P]
        lib.oracle_ramp_kernel.restype = None
        lib.oracle_quantiles_rf.argtypes = [P, i64, i32, i32, i32, i32, P, P, P]
        lib.oracle_quantiles_rf.restype = None
        lib.oracle_objective_at.argtypes = [P, P, i32, i32, i32, i32, dbl, dbl]
        lib.oracle_objective_at.restype = dbl
        lib.oracle_angle_table.argtypes = [i32, P, P]
        lib.oracle_angle_table.restype = None
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = i32
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return _load().oracle_num_threads()


def angle_table(n: int):
    cs = np.zeros(n, np.float64)
    sn = np.zeros(n, np.float64)
    _load().oracle_angle_table(n, _ptr(cs), _ptr(sn))
    return cs, sn


def project(img: np.ndarray, n: int):
    """Hat-weighted line projections.  img [N, L, L] float32 -> pmf [N, n, L]
    float64 and a per-image non-finite flag [N] int32."""
    img = np.ascontiguousarray(img, dtype=np.float32)
    if img.ndim == 2:
        img = img[None]
    N, L, L2 = img.shape
    assert L == L2
    pmf = np.zeros((N, n, L), np.float64)
    bad = np.zeros(N, np.int32)
    _load().oracle_project(_ptr(img), N, L, n, _ptr(pmf), _ptr(bad))
    return pmf, bad


def quantiles(pmf: np.ndarray, Q: int, levels: int = LEVELS_MIDPOINT, nonfinite=None):
    """pmf [N, n, L] -> quantile tables [N, Q, n] and aux [N, 4]
    (mass, E, Re a, Im a)."""
    pmf = np.ascontiguousarray(pmf, dtype=np.float64)
    if pmf.ndim == 2:
        pmf = pmf[None]
    N, n, L = pmf.shape
    qt = np.zeros((N, Q, n), np.float64)
    aux = np.zeros((N, 4), np.float64)
    nf = None if nonfinite is None else np.ascontiguousarray(nonfinite, dtype=np.int32)
    _load().oracle_quantiles(_ptr(pmf), N, L, n, Q, levels, _ptr(nf), _ptr(qt), _ptr(aux))
    return qt, aux


def ramp_kernel(L: int):
    """The ramp filter's cyclic kernel h[m], m < 2L (explicit cosine sum)."""
    hk = np.zeros(2 * L, np.float64)
    _load().oracle_ramp_kernel(L, _ptr(hk))
    return hk


def ramp(pmf: np.ndarray):
    """Ramp-filtered projections: pmf [N, n, L] -> signed [N, n, L]."""
    pmf = np.ascontiguousarray(pmf, dtype=np.float64)
    if pmf.ndim == 2:
        pmf = pmf[None]
    N, n, L = pmf.shape
    out = np.zeros_like(pmf)
    _load().oracle_ramp(_ptr(pmf), N, L, n, _ptr(out))
    return out


def quantiles_rf(pf: np.ndarray, Q: int, levels: int = LEVELS_MIDPOINT, nonfinite=None):
    """Signed filtered projections [N, n, L] -> stacked tables [N, 2Q, n]
    (positive part, then negative part) and aux [N, 4] (smallest part mass,
    E, Re a, Im a of the stacked table)."""
    pf = np.ascontiguousarray(pf, dtype=np.float64)
    if pf.ndim == 2:
        pf = pf[None]
    N, n, L = pf.shape
    qt = np.zeros((N, 2 * Q, n), np.float64)
    aux = np.zeros((N, 4), np.float64)
    nf = None if nonfinite is None else np.ascontiguousarray(nonfinite, dtype=np.int32)
    _load().oracle_quantiles_rf(_ptr(pf), N, L, n, Q, levels, _ptr(nf), _ptr(qt), _ptr(aux))
    return qt, aux


def _disk_mask(L: int):
    i, j = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    return (2 * j - L + 1) ** 2 + (2 * i - L + 1) ** 2 <= (L - 2) ** 2


def fourier_project(img: np.ndarray, n: int, cell: bool = True, angles=None):
    """Fourier-slice projections (Sec. 2.2, Fourier slice theorem; the
    discretisation of the fixed-angle error theorem with NUFFT precision in
    the appendix), written out as the exact non-uniform DFT that a NUFFT
    approximates.

    The image is the same pixel mass as for the line sum (positive part,
    inside the disk), pixel (i, j) at x_j = (j - c0) h, y_i = (i - c0) h,
    h = 2/L, c0 = (L-1)/2, L = 2M even.  For angle theta_a with direction
    d = (cos theta_a, -sin theta_a):
      yhat_k = sum_ij m_ij exp(-i k pi (d . x_ij)) * S_k,  k = -M .. M-1,
    with S_k = sinc(k pi d_x h/2) sinc(k pi d_y h/2) the transform of one
    pixel cell (cell=True: the image read as piecewise constant) or 1
    (cell=False: point masses); the projection is the trigonometric
    polynomial g(s) = (1/2) sum_k yhat_k exp(i k pi s) sampled at the bin
    centres s_b = -1 + (b + 1/2) h, P[a][b] = h * Re g(s_b).  Negative lobes
    are kept (the caller clips).  With `angles` (n radians) the slices are
    taken at those angles instead of theta_a = 2 pi a / n.  Returns (P [N,
    n, L] float64, non-finite flag [N] int32); an image with a non-finite
    value gives NaN.  Plain double sum per angle: O(n L^3) per image."""
    img = np.asarray(img, dtype=np.float64)
    if img.ndim == 2:
        img = img[None]
    N, L, L2 = img.shape
    assert L == L2 and L % 2 == 0
    M, h, c0 = L // 2, 2.0 / L, 0.5 * (L - 1)
    if angles is None:
        cs, sn = angle_table(n)
    else:
        angles = np.asarray(angles, dtype=np.float64)
        assert angles.shape == (n,)
        cs, sn = np.cos(angles), np.sin(angles)
    pos = (np.arange(L) - c0) * h            # x_j for columns, y_i for rows
    k = np.arange(-M, M, dtype=np.float64)
    sb = -1.0 + (np.arange(L) + 0.5) * h
    back = np.exp(1j * np.pi * np.outer(sb, k))  # [b, k]
    disk = _disk_mask(L)
    out = np.zeros((N, n, L), np.float64)
    bad = np.zeros(N, np.int32)
    for g in range(N):
        F = img[g]
        if not np.all(np.isfinite(F)):
            bad[g] = 1
            out[g] = np.nan
            continue
        m = np.where(disk & (F > 0), F, 0.0)
        for a in range(n):
            dx, dy = cs[a], -sn[a]
            ex = np.exp(-1j * np.pi * np.outer(k, pos) * dx)  # [k, j]
            ey = np.exp(-1j * np.pi * np.outer(k, pos) * dy)  # [k, i]
            yk = np.sum(ey * (m @ ex.T).T, axis=1)            # sum_i ey[k,i] sum_j m[i,j] ex[k,j]
            if cell:
                yk = yk * np.sinc(k * dx * h / 2) * np.sinc(k * dy * h / 2)
            out[g, a] = h * (0.5 * back @ yk).real
    return out, bad


def fourier_tables(img: np.ndarray, n: int, Q: int, levels: int = LEVELS_MIDPOINT, angles=None):
    """Quantile tables of the Fourier-slice projections with negative lobes
    clipped to zero before normalisation (Sec. 2.3: the outputs are
    normalised into probability measures); optionally at given angles."""
    P, bad = fourier_project(img, n, angles=angles)
    return quantiles(np.maximum(P, 0.0), Q, levels, bad)


def mc_align_images(ref_img, imgs, n: int, Q: int, angles, levels: int = LEVELS_MIDPOINT,
                    want_curve: bool = False):
    """Monte-Carlo SW2 over rotations (extended alignment results): the
    projections are taken at n given directions (sorted), and the discrete
    rotational SW2 scan is applied unchanged, lag l read as the rotation
    2 pi l / n; rotation only."""
    L = imgs.shape[-1]
    rq, ra = fourier_tables(ref_img, n, Q, levels, angles)
    iq, ia = fourier_tables(imgs, n, Q, levels, angles)
    return align(rq, ra, iq, ia, L, mode=MODE_ROT_ONLY, want_curve=want_curve)


def tables(img: np.ndarray, n: int, Q: int, levels: int = LEVELS_MIDPOINT, ramp: bool = False):
    """Image stack -> (qt, aux): projection followed by quantiles; with
    ramp=True the projections are ramp-filtered and the stacked signed-part
    tables [N, 2Q, n] are returned."""
    pmf, bad = project(img, n)
    if ramp:
        return quantiles_rf(globals()["ramp"](pmf), Q, levels, bad)
    return quantiles(pmf, Q, levels, bad)


def align(ref_qt, ref_aux, img_qt, img_aux, L: int, pairs=None, mode: int = MODE_ROT_TRANS,
          want_curve: bool = False, ramp: bool = False):
    """Exhaustive rotation scan with the closed-form translation.

    Returns a dict with rot_index [P], shift_px [P, 2], sw2sq [P], status [P],
    and, when requested, curve [P, n] = D*(l) and shift_curve [P, n, 2] =
    the closed-form shift s*(l) in pixels at every lag.  Pairs default to all ref x img in
    row-major order.  ramp=True: the tables are the stacked [2Q, n] tables of
    the ramp-filtered distance, whose objective sums the two parts."""
    ref_qt = np.ascontiguousarray(ref_qt, dtype=np.float64)
    img_qt = np.ascontiguousarray(img_qt, dtype=np.float64)
    ref_aux = np.ascontiguousarray(ref_aux, dtype=np.float64)
    img_aux = np.ascontiguousarray(img_aux, dtype=np.float64)
    if ref_qt.ndim == 2:
        ref_qt, ref_aux = ref_qt[None], ref_aux[None]
    if img_qt.ndim == 2:
        img_qt, img_aux = img_qt[None], img_aux[None]
    nr, rows, n = ref_qt.shape
    Q = rows // 2 if ramp else rows
    ni = img_qt.shape[0]
    if pairs is not None:
        pairs = np.ascontiguousarray(pairs, dtype=np.int64).reshape(-1, 2)
        P = pairs.shape[0]
    else:
        P = nr * ni
    out_l = np.zeros(P, np.int32)
    out_s = np.zeros((P, 2), np.float64)
    out_d = np.zeros(P, np.float64)
    st = np.zeros(P, np.int32)
    curve = np.zeros((P, n), np.float64) if want_curve else None
    scurve = np.zeros((P, n, 2), np.float64) if want_curve else None
    _load().oracle_align_rows(_ptr(ref_qt), _ptr(ref_aux), nr, _ptr(img_qt), _ptr(img_aux), ni,
                              _ptr(pairs), P, L, n, Q, rows, mode, _ptr(out_l), _ptr(out_s),
                              _ptr(out_d), _ptr(st), _ptr(curve), _ptr(scurve))
    res = {"rot_index": out_l, "shift_px": out_s, "sw2sq": out_d, "status": st,
           "theta_rad": 2.0 * np.pi * out_l / n}
    if want_curve:
        res["curve"] = curve
        res["shift_curve"] = scurve
    return res


def objective_at(U, V, l: int, sx: float, sy: float, ramp: bool = False) -> float:
    """D(l, s) for one pair of tables (s in unit-disk coordinates); ramp=True
    for stacked [2Q, n] tables (normalised by nQ)."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    V = np.ascontiguousarray(V, dtype=np.float64)
    rows, n = U.shape
    Q = rows // 2 if ramp else rows
    return _load().oracle_objective_at(_ptr(U), _ptr(V), n, Q, rows, l, sx, sy)


def align_images(ref_img, imgs, n: int, Q: int, levels: int = LEVELS_MIDPOINT,
                 mode: int = MODE_ROT_TRANS, want_curve: bool = False, ramp: bool = False):
    """Whole path from images: one reference image against a stack."""
    L = imgs.shape[-1]
    rq, ra = tables(ref_img, n, Q, levels, ramp=ramp)
    iq, ia = tables(imgs, n, Q, levels, ramp=ramp)
    return align(rq, ra, iq, ia, L, mode=mode, want_curve=want_curve, ramp=ramp)
