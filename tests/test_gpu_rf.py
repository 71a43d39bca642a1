"""GPU parity of the ramp-filtered path (ramp filter on the matrix cores,
signed-part quantile tables, alignment of the stacked tables) against the
FP64 oracle, through the C ABI."""
import numpy as np
import pytest

import synth
from tests import parity

pytestmark = pytest.mark.gpu

RF_GEOMS = [(16, 16, 16), (39, 48, 24), (40, 24, 20), (64, 64, 64), (65, 48, 48), (96, 96, 96),
            (128, 128, 128), (256, 64, 32)]


@pytest.fixture(scope="module")
def api():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_13756_amd import api as A

    return A


@pytest.fixture(scope="module")
def ctx(api):
    c = api.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctx_fused(api, tmp_path_factory):
    """Contexts that take the fused tables kernels at any batch size: two
    images per block where the geometry allows it, and one."""
    out = {}
    for name, txt in (("two", '{"small_batch": 0}'),
                      ("one", '{"small_batch": 0, "tables_images_per_block": 1}')):
        path = tmp_path_factory.mktemp("tune") / f"{name}.json"
        path.write_text(txt)
        out[name] = api.Context(0, tune_json=str(path))
    yield out
    for c in out.values():
        c.close()


def dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def blob_stack(L, N, seed):
    ref, imgs, _, _ = synth.make_stack(seed, L, N, K=6, shift_px=max(1.0, L / 16), jitter_px=1.0,
                                       snr=1.0)
    return ref, imgs


@pytest.mark.parametrize("L,n,Q", RF_GEOMS)
def test_ramp_filter_parity(api, ctx, oracle, L, n, Q):
    """The filter alone on the oracle's projections (rounded to FP32): FP32
    matrix-core sums against the FP64 cyclic convolution, relative to the
    largest filtered value; columns padded to 16 bins when L is not a
    multiple of 16; in place equals out of place."""
    _, imgs = blob_stack(L, 5, 700 + L)
    P0, _ = oracle.project(imgs, n)
    p32 = P0.astype(np.float32)
    x = dev(p32)
    pf = api.ramp(ctx, x).cpu().numpy()
    ref = oracle.ramp(p32.astype(np.float64))
    err = np.abs(pf - ref).max(axis=(1, 2)) / np.abs(ref).max(axis=(1, 2))
    assert err.max() < 1e-5, err
    api.ramp(ctx, x, out=x)
    assert np.array_equal(x.cpu().numpy(), pf)


@pytest.mark.parametrize("L,n,Q", RF_GEOMS)
@pytest.mark.parametrize("levels", [0, 1])
def test_quantiles_rf_parity(api, ctx, oracle, L, n, Q, levels):
    """Signed-part tables from the same FP32 filtered projections on both
    sides: positive part in rows 0..Q-1, negative part in rows Q..2Q-1, each
    normalised on its own; aux = smallest part mass, E, a of the stacked
    table."""
    _, imgs = blob_stack(L, 4, 800 + L)
    P0, _ = oracle.project(imgs, n)
    pf32 = oracle.ramp(P0).astype(np.float32)
    qt, aux = api.quantiles(ctx, dev(pf32), Q, levels, ramp=True)
    q0, a0 = oracle.quantiles_rf(pf32.astype(np.float64), Q, levels)
    qt, aux = qt.cpu().numpy(), aux.cpu().numpy()
    assert qt.shape == (4, 2 * Q, n)
    assert np.abs(qt - q0).max() < 2e-6
    assert np.allclose(aux[:, 0], a0[:, 0], rtol=1e-9)
    assert np.allclose(aux[:, 1], a0[:, 1], rtol=1e-6)
    assert np.abs(aux[:, 2:] - a0[:, 2:]).max() < 1e-6


@pytest.mark.parametrize("L,n,Q,kind", [(64, 64, 64, "clean"), (128, 128, 128, "clean"),
                                        (96, 96, 48, "clean"), (128, 128, 128, "raw"),
                                        (60, 48, 36, "raw")])
@pytest.mark.parametrize("mode,prec,top_k", [(0, 0, 1), (1, 0, 1), (0, 1, 4)])
def test_rf_end_to_end_parity(api, ctx, oracle, L, n, Q, kind, mode, prec, top_k):
    """Images -> stacked ramp-filtered tables -> alignment on the GPU against
    the oracle from the same images: rotation (tie-aware), shift and the
    ramp-filtered distance (sum of both parts, each normalised by nQ).  Raw
    inputs: the positive part and the disk mask come from the kernels."""
    if kind == "raw":
        ref, imgs = synth.make_raw_stack(900 + L, L, 24)
    else:
        ref, imgs = blob_stack(L, 24, 900 + L)
    rq, ra = api.tables(ctx, dev(ref[None]), n, Q, ramp=True)
    iq, ia = api.tables(ctx, dev(imgs), n, Q, ramp=True)
    res, curve = api.align_batch(ctx, rq, ra, iq, ia, L, mode=mode, prec=prec, top_k=top_k,
                                 want_curve=True, ramp=True)
    g = api.unpack_results(res)
    oq, oa = oracle.tables(ref[None], n, Q, ramp=True)
    iq0, ia0 = oracle.tables(imgs, n, Q, ramp=True)
    o = oracle.align(oq, oa, iq0, ia0, L, mode=mode, want_curve=True, ramp=True)
    parity.check(g, o, L, parity.TAU_RF, o["curve"])
    # the curve is the ramp-filtered objective too: FP32 to a small fraction
    # of its scale; with the BF16 correlation to bfloat16 rounding of the
    # energy term (E_U + E_V) / (nQ) it is computed from
    c = curve.cpu().numpy()
    if prec == 0:
        scale = np.abs(o["curve"]).max()
        assert np.abs(c - o["curve"]).max() < 1e-4 * scale
    else:
        energy = (oa[0, 1] + ia0[:, 1]) / (n * Q)
        assert np.all(np.abs(c - o["curve"]).max(axis=1) < 2.0 ** -7 * energy)


def test_rf_self_and_quarter_turn(api, ctx):
    """An image against itself and against its 90-degree rotations: lags 0
    and n/4 multiples, distance 0 to FP32 rounding of identical tables."""
    L = n = Q = 64
    _, imgs = blob_stack(L, 1, 990)
    f = imgs[0]
    stack = np.stack([f] + [np.ascontiguousarray(np.rot90(f, m)) for m in (1, 2, 3)])
    rq, ra = api.tables(ctx, dev(f[None]), n, Q, ramp=True)
    iq, ia = api.tables(ctx, dev(stack), n, Q, ramp=True)
    g = api.unpack_results(api.align_batch(ctx, rq, ra, iq, ia, L, ramp=True)[0])
    assert list(g["status"]) == [0, 0, 0, 0]
    assert g["rot_index"][0] == 0 and g["sw2sq"][0] == 0.0
    assert sorted(g["rot_index"][1:] % (n // 4)) == [0, 0, 0]
    assert np.all(np.abs(g["sw2sq"][1:]) < 1e-9)


def test_rf_status_and_validation(api, ctx):
    """Zero and non-finite images keep their status through the filter; a
    stacked table beyond 512 rows is refused before any device work."""
    from paper_2503_13756_amd._abi import SwError

    L = n = Q = 32
    _, imgs = blob_stack(L, 3, 991)
    imgs[1] = 0.0
    imgs[2, 5, 5] = np.nan
    q, a = api.tables(ctx, dev(imgs), n, Q, ramp=True)
    r = api.unpack_results(api.align_batch(ctx, q[:1].contiguous(), a[:1].contiguous(), q, a, L,
                                           ramp=True)[0])
    assert list(r["status"]) == [0, 1, 2]
    with pytest.raises(SwError):
        api.tables(ctx, dev(imgs), 32, 384, ramp=True)


@pytest.mark.parametrize("kind", ["clean", "raw"])
@pytest.mark.parametrize("L,n,Q", [(64, 64, 64), (128, 128, 128), (60, 48, 36), (120, 96, 64)])
def test_tables_rf_fused_equals_staged(api, ctx, ctx_fused, oracle, L, n, Q, kind):
    """The fused ramp-filtered tables kernels (projection, filter and both
    inversions in LDS; two images per block, the odd count leaving the last
    block one, and one image per block) give bitwise the tables and aux of
    sw_project, sw_ramp and sw_quantiles_rf in sequence; on raw inputs the
    tables also match the oracle's, which clips and masks the images itself."""
    if kind == "raw":
        _, imgs = synth.make_raw_stack(1300 + L, L, 7)
    else:
        _, imgs = blob_stack(L, 7, 1300 + L)
    x = dev(imgs)
    q1, a1 = api.tables(ctx_fused["two"], x, n, Q, ramp=True)
    q2, a2 = api.quantiles(ctx, api.ramp(ctx, api.project(ctx, x, n)), Q, ramp=True)
    q3, a3 = api.tables(ctx_fused["one"], x, n, Q, ramp=True)
    q4, a4 = api.tables(ctx, x, n, Q, ramp=True)  # a small batch: the split launches
    for q, a in ((q2, a2), (q3, a3), (q4, a4)):
        assert np.array_equal(q1.cpu().numpy(), q.cpu().numpy())
        assert np.array_equal(a1.cpu().numpy(), a.cpu().numpy())
    if kind == "raw":
        # the projections' FP32 rounding moves the signed parts' quantiles
        # where a part's CDF is nearly flat, so the table check is on the
        # part masses (aux[0]) and on most entries
        oq, oa = oracle.tables(imgs, n, Q, ramp=True)
        assert np.allclose(a1.cpu().numpy()[:, 0], oa[:, 0], rtol=1e-5)
        d = np.abs(q1.cpu().numpy() - oq)
        assert np.median(d) < 1e-6 and np.mean(d < 1e-4) > 0.999
