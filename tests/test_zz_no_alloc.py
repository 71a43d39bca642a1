"""sw_align_batch_noalloc, the allocation-free variant of sw_align_batch,
through the C ABI: two calls in a row (the second on a smaller input) must
give bitwise the records and curves of sw_align_batch and pass the oracle
parity rule; a call needing more scratch than the fixed array holds fails
before any launch; a fresh context allocates no device memory in it."""
import numpy as np
import pytest

import synth
from tests import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_13756_amd import api as A

    return A


def dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def stack(L, N, seed):
    ref, imgs, _, _ = synth.make_stack(seed, L, N, K=6, shift_px=max(1.0, L / 16), jitter_px=1.0,
                                       snr=1.0)
    return ref, imgs


def both(api, ctx, *args, **kw):
    a, ca = api.align_batch(ctx, *args, **kw)
    b, cb = api.align_batch(ctx, *args, noalloc=True, **kw)
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    if ca is not None:
        assert np.array_equal(ca.cpu().numpy(), cb.cpu().numpy())
    return b, cb


@pytest.mark.parametrize("L,n,prec", [(128, 128, 0), (128, 128, 1), (64, 64, 0), (96, 96, 1)])
def test_one_vs_many_twice(api, oracle, L, n, prec):
    """1 reference x many images (n = 128: register-FFT kernel; others: the
    LDS-FFT kernel), then a smaller batch against a second reference."""
    print(f"noalloc 1-vs-many L={L} n={n} prec={prec}", flush=True)
    ctx = api.Context(0)
    tau = parity.TAU_FP32 if prec == 0 else parity.TAU_BF16
    for ref_seed, N in ((3100, 40), (3101, 9)):
        ref, imgs = stack(L, N, ref_seed + L)
        rq, ra = api.tables(ctx, dev(ref[None]), n, n)
        iq, ia = api.tables(ctx, dev(imgs), n, n)
        res, curve = both(api, ctx, rq, ra, iq, ia, L, prec=prec, want_curve=True)
        orc = oracle.align_images(ref, imgs, n, n, want_curve=True)
        parity.check(api.unpack_results(res), orc, L, tau, orc["curve"])
    ctx.close()


def test_pair_list_twice(api, oracle):
    print("noalloc pair list L=64", flush=True)
    ctx = api.Context(0)
    L = n = 64
    _, imgs = stack(L, 12, 3200)
    q, a = api.tables(ctx, dev(imgs), n, n)
    rng = np.random.default_rng(7)
    oq, oa = oracle.tables(imgs, n, n)
    for P in (41, 13):
        pairs = rng.integers(0, 12, size=(P, 2)).astype(np.int64)
        res, _ = both(api, ctx, q, a, q, a, L, pairs=dev(pairs), top_k=3)
        orc = oracle.align(oq, oa, oq, oa, L, pairs=pairs, want_curve=True)
        parity.check(api.unpack_results(res), orc, L, parity.TAU_FP32, orc["curve"])
    ctx.close()


def test_all_pairs_mfma_twice(api, oracle):
    """Many-vs-many on the matrix cores (bf16 spectra and candidate lags in
    the fixed array), 40 x 40 and then 17 x 23."""
    print("noalloc all pairs L=64", flush=True)
    ctx = api.Context(0)
    L = n = 64
    _, imgs = stack(L, 40, 3300)
    oq, oa = oracle.tables(imgs, n, n)
    for nr, ni in ((40, 40), (17, 23)):
        rq, ra = api.tables(ctx, dev(imgs[:nr]), n, n)
        iq, ia = api.tables(ctx, dev(imgs[:ni]), n, n)
        res, _ = both(api, ctx, rq, ra, iq, ia, L, prec=1, top_k=4)
        orc = oracle.align(oq[:nr], oa[:nr], oq[:ni], oa[:ni], L, want_curve=True)
        parity.check(api.unpack_results(res), orc, L, parity.TAU_BF16, orc["curve"])
    ctx.close()


def test_too_large_fails_before_launch(api):
    """3,000 x 3,000 pairs at n = 64 need 72 MB of candidate lags: refused
    with SW_E_NOMEM, the output untouched; sw_align_batch runs it."""
    import torch
    from paper_2503_13756_amd._abi import SwError

    print("noalloc too large", flush=True)
    ctx = api.Context(0)
    N, L = 3000, 64
    q = torch.zeros((N, L, L), dtype=torch.float32, device="cuda")
    a = torch.zeros((N, 4), dtype=torch.float64, device="cuda")
    out = torch.full((N * N, 6), 7, dtype=torch.int32, device="cuda")
    with pytest.raises(SwError, match="NOMEM"):
        api.align_batch(ctx, q, a, q, a, L, prec=1, out=out, noalloc=True)
    torch.cuda.synchronize()
    assert int(out.min()) == 7 and int(out.max()) == 7
    ctx.close()


def test_fresh_context_allocates_nothing(api):
    """After the library is loaded on the device, a fresh context's first
    no-alloc call leaves the device's free memory unchanged, where the
    allocating entry point grows the context scratch."""
    import torch

    print("noalloc memory", flush=True)
    L = n = 64
    _, imgs = stack(L, 300, 3400)
    warm = api.Context(0)
    q, a = api.tables(warm, dev(imgs), n, n)
    out = torch.empty((300 * 300, 6), dtype=torch.int32, device="cuda")
    api.align_batch(warm, q, a, q, a, L, prec=1, out=out, noalloc=True)
    torch.cuda.synchronize()
    deltas = {}
    for noalloc in (True, False):
        c = api.Context(0)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        api.align_batch(c, q, a, q, a, L, prec=1, out=out, noalloc=noalloc)
        torch.cuda.synchronize()
        deltas[noalloc] = free0 - torch.cuda.mem_get_info()[0]
        c.close()
    print("free-memory drop:", deltas, flush=True)
    assert deltas[True] == 0 and deltas[False] > 0
    warm.close()
