"""GPU parity of the max-sliced alignment mode (largest per-angle W2^2,
rotation only): matrix-core estimate of every lag, direct FP32 rescore of the
top_k lags, against the FP64 oracle through the C ABI."""
import numpy as np
import pytest

import synth
from tests import parity

pytestmark = pytest.mark.gpu

MSW = 2


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


def dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def blob_stack(L, N, seed):
    ref, imgs, _, _ = synth.make_stack(seed, L, N, K=6, shift_px=max(1.0, L / 16), jitter_px=1.0,
                                       snr=1.0)
    return ref, imgs


def curve_tol(rq, iq):
    """FP32 estimate |u_k|^2 + |v_k'|^2 - 2 C[k][k'] per column, over Q."""
    Q = rq.shape[-2]
    e = (rq ** 2).sum(axis=-2).max() + (iq ** 2).sum(axis=-2).max()
    return 1e-5 * e / Q


@pytest.mark.parametrize("L,n,Q", [(32, 16, 16), (40, 32, 24), (48, 48, 48), (64, 64, 64),
                                   (96, 96, 96), (128, 128, 128), (96, 128, 96), (48, 64, 40)])
@pytest.mark.parametrize("top_k", [1, 4])
def test_msw_parity_on_oracle_tables(api, ctx, oracle, L, n, Q, top_k):
    """Alignment stage alone on the oracle's tables rounded to FP32: the lag
    (tie-aware against the oracle's curve), shift 0, the rescored distance to
    the FP32 tolerance, and the per-lag estimate."""
    ref, imgs = blob_stack(L, 20, 1500 + L + Q)
    rq, ra = oracle.tables(ref, n, Q)
    iq, ia = oracle.tables(imgs, n, Q)
    rq32, iq32 = rq.astype(np.float32), iq.astype(np.float32)
    res, curve = api.align_batch(ctx, dev(rq32), dev(ra), dev(iq32), dev(ia), L, mode=MSW,
                                 top_k=top_k, want_curve=True)
    g = api.unpack_results(res)
    o = oracle.align(rq32.astype(np.float64), ra, iq32.astype(np.float64), ia, L, mode=MSW,
                     want_curve=True)
    parity.check(g, o, L, parity.TAU_FP32, o["curve"])
    assert np.all(g["shift_px"] == 0.0)
    c = curve.cpu().numpy()
    assert np.abs(c - o["curve"]).max() < curve_tol(rq32, iq32)


@pytest.mark.parametrize("L,n,Q", [(64, 64, 64), (128, 128, 128), (96, 96, 96), (39, 48, 48)])
def test_msw_end_to_end_and_pair_list(api, ctx, oracle, L, n, Q):
    """Images -> GPU tables -> max-sliced alignment against the oracle from the
    same images, on a pair list with a self pair and an out-of-range index."""
    ref, imgs = blob_stack(L, 10, 1600 + L)
    allimg = np.concatenate([ref[None], imgs])
    q, a = api.tables(ctx, dev(allimg), n, Q)
    pairs = np.array([[0, i] for i in range(11)] + [[3, 3], [0, 99]], np.int64)
    res, _ = api.align_batch(ctx, q, a, q, a, L, pairs=dev(pairs), mode=MSW)
    g = api.unpack_results(res)
    oq, oa = oracle.tables(allimg, n, Q)
    o = oracle.align(oq, oa, oq, oa, L, pairs=pairs[:-1], mode=MSW, want_curve=True)
    sub = {k: v[:-1] for k, v in g.items()}
    parity.check(sub, o, L, parity.TAU_FP32, o["curve"])
    assert g["status"][-1] == 3
    assert g["rot_index"][0] == 0 and g["sw2sq"][0] == 0.0
    assert g["rot_index"][11] == 0 and g["sw2sq"][11] == 0.0


def test_msw_quarter_turns_and_status(api, ctx):
    """90-degree rotations give l = m n/4 and distance 0; zero and non-finite
    images keep their status; n that are not multiples of 16 up to 128 are
    refused."""
    from paper_2503_13756_amd._abi import SwError

    L = n = Q = 64
    _, imgs = blob_stack(L, 1, 1700)
    f = imgs[0]
    bad0 = np.zeros_like(f)
    bad1 = f.copy()
    bad1[7, 7] = np.nan
    stack = np.stack([np.ascontiguousarray(np.rot90(f, m)) for m in (1, 2, 3)] + [bad0, bad1])
    rq, ra = api.tables(ctx, dev(f[None]), n, Q)
    iq, ia = api.tables(ctx, dev(stack), n, Q)
    g = api.unpack_results(api.align_batch(ctx, rq, ra, iq, ia, L, mode=MSW)[0])
    assert list(g["status"]) == [0, 0, 0, 1, 2]
    assert sorted(int(x) % (n // 4) for x in g["rot_index"][:3]) == [0, 0, 0]
    assert np.all(np.abs(g["sw2sq"][:3]) < 1e-9)
    for nn in (24, 192):
        qx, ax = api.tables(ctx, dev(stack[:1]), nn, 32)
        with pytest.raises(SwError):
            api.align_batch(ctx, qx, ax, qx, ax, L, mode=MSW)
