"""GPU parity at the full sizes of the timed workloads, in the launch
configuration the benchmark uses (a default context: two images per block for
the tables, one pair per wave for the n = 128 alignment, the MFMA path for all
pairs), on outputs sampled for the oracle plus properties checked on every
output.

* 1 reference vs 10,000 images at L = n = Q = 128 (FP32 and the BF16 form):
  projections, tables and alignment of 48 sampled images against the oracle
  (the first, last and middle images among them); on all 10,000: status 0,
  finite non-negative distances, lags in range, a second run bitwise equal;
  an odd count (9,999) leaves the last block one image, whose tables must equal
  the even run's bitwise.
* all ordered pairs of 2,000 images at L = n = Q = 64 (BF16 correlation,
  top-4 FP32 rescore): 300 sampled pairs (the four corners among them) against
  the oracle; every self pair exactly 0 at lag 0.
* 50,000 images in uneven stacks (L from 64 to 256, tiles autotuned first):
  8 images per stack against the oracle, tiled copies bitwise equal."""
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


@pytest.fixture(scope="module")
def ctx(api):
    c = api.Context(0)
    yield c
    c.close()


def dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def check_all(g, n):
    assert np.all(g["status"] == 0)
    assert np.all(np.isfinite(g["sw2sq"])) and np.all(g["sw2sq"] >= 0.0)
    assert np.all((g["rot_index"] >= 0) & (g["rot_index"] < n))


@pytest.fixture(scope="module")
def headline(api, ctx):
    w = synth.workload(1)
    L, n, Q, N = w["L"], w["n"], w["Q"], len(w["imgs"])
    assert (L, n, Q, N) == (128, 128, 128, 10000)
    x = dev(w["imgs"])
    rq, ra = api.tables(ctx, dev(w["ref"][None]), n, Q)
    iq, ia = api.tables(ctx, x, n, Q)
    return w, x, rq, ra, iq, ia


def test_headline_tables_full_size(api, ctx, oracle, headline):
    w, x, rq, ra, iq, ia = headline
    L, n, Q, N = w["L"], w["n"], w["Q"], len(w["imgs"])
    rng = np.random.default_rng(11)
    S = np.unique(np.concatenate([[0, 1, 2, N // 2 - 1, N // 2, N - 2, N - 1],
                                  rng.choice(N, 41, replace=False)]))
    imgs = w["imgs"][S]
    # projections of the sample (the fused kernel's are bitwise these)
    pmf = api.project(ctx, dev(imgs), n).cpu().numpy()
    P0, _ = oracle.project(imgs, n)
    err = np.abs(pmf - P0).max(axis=(1, 2)) / P0.max(axis=(1, 2))
    assert err.max() < 1e-5, err
    # the full-size run's tables of the sample against the oracle's quantiles
    # of those FP32 projections, and bitwise against the staged launches on
    # the sample alone
    q_all, a_all = iq.cpu().numpy(), ia.cpu().numpy()
    q0, a0 = oracle.quantiles(pmf.astype(np.float64), Q, 0)
    qs, as_ = q_all[S], a_all[S]
    assert np.abs(qs - q0).max() < 2e-6
    assert np.allclose(as_[:, 0], a0[:, 0], rtol=1e-12)
    assert np.allclose(as_[:, 1], a0[:, 1], rtol=1e-6)
    q5, a5 = api.quantiles(ctx, api.project(ctx, dev(imgs), n), Q)
    assert np.array_equal(q5.cpu().numpy(), qs) and np.array_equal(a5.cpu().numpy(), as_)
    # every image: finite tables inside [-1, 1], positive finite mass
    assert np.all(np.isfinite(q_all)) and np.abs(q_all).max() <= 1.0
    assert np.all(np.isfinite(a_all[:, 0])) and np.all(a_all[:, 0] > 0.0)
    # a second run is bitwise the same
    iq2, ia2 = api.tables(ctx, x, n, Q)
    assert np.array_equal(iq2.cpu().numpy(), q_all) and np.array_equal(ia2.cpu().numpy(), a_all)
    # an odd count leaves the last block one image: its tables are the same
    iq3, ia3 = api.tables(ctx, x[: N - 1], n, Q)
    assert np.array_equal(iq3[N - 2].cpu().numpy(), q_all[N - 2])
    assert np.array_equal(ia3[N - 2].cpu().numpy(), a_all[N - 2])


@pytest.mark.parametrize("prec,tau", [(0, parity.TAU_FP32), (1, parity.TAU_BF16)])
def test_headline_alignment_full_size(api, ctx, oracle, headline, prec, tau):
    w, x, rq, ra, iq, ia = headline
    L, n, Q, N = w["L"], w["n"], w["Q"], len(w["imgs"])
    res, _ = api.align_batch(ctx, rq, ra, iq, ia, L, prec=prec)
    g = api.unpack_results(res)
    check_all(g, n)
    res2, _ = api.align_batch(ctx, rq, ra, iq, ia, L, prec=prec)
    assert np.array_equal(res2.cpu().numpy(), res.cpu().numpy())
    rng = np.random.default_rng(12 + prec)
    S = np.unique(np.concatenate([[0, N // 2, N - 1], rng.choice(N, 45, replace=False)]))
    orq, ora = oracle.tables(w["ref"][None], n, Q)
    oiq, oia = oracle.tables(w["imgs"][S], n, Q)
    o = oracle.align(orq, ora, oiq, oia, L, want_curve=True)
    rep = parity.check({k: v[S] for k, v in g.items()}, o, L, tau, o["curve"])
    print(rep)


def test_all_pairs_full_size(api, ctx, oracle):
    w = synth.workload(2)
    L, n, Q, N = w["L"], w["n"], w["Q"], len(w["imgs"])
    assert (L, n, Q, N) == (64, 64, 64, 2000)
    q, a = api.tables(ctx, dev(w["imgs"]), n, Q)
    res, _ = api.align_batch(ctx, q, a, q, a, L, prec=1, top_k=4)
    g = api.unpack_results(res)
    check_all(g, n)
    diag = np.arange(N) * N + np.arange(N)
    assert np.all(g["sw2sq"][diag] == 0.0) and np.all(g["rot_index"][diag] == 0)
    rng = np.random.default_rng(13)
    pairs = np.concatenate([[[0, 0], [0, N - 1], [N - 1, 0], [N - 1, N - 1]],
                            rng.integers(0, N, (296, 2))]).astype(np.int64)
    used = np.unique(pairs)
    oq, oa = oracle.tables(w["imgs"][used], n, Q)
    loc = np.searchsorted(used, pairs)
    o = oracle.align(oq, oa, oq, oa, L, pairs=loc, want_curve=True)
    sub = {k: v[pairs[:, 0] * N + pairs[:, 1]] for k, v in g.items()}
    rep = parity.check(sub, o, L, parity.TAU_BF16, o["curve"])
    print(rep)


def test_uneven_stacks_full_size(api, ctx, oracle, tmp_path):
    """50,000 images in 21 stacks of L in {64, ..., 256} with their own
    references, the tiles autotuned first as in the benchmark; each stack holds
    200 rendered images tiled to its drawn size, so copy k of an image must
    give bitwise its first copy's record; 8 images of every stack against the
    oracle."""
    import torch

    stacks = synth.uneven_stacks(total=50000, cap_per_stack=200)
    devs = []
    for L, ref, imgs, size in stacks:
        x = dev(imgs)
        reps = (size + len(imgs) - 1) // len(imgs)
        devs.append((dev(ref), x.repeat(reps, 1, 1)[:size].contiguous()))
    assert sum(int(d[1].shape[0]) for d in devs) == 50000
    api.autotune(ctx, sorted({s[0] for s in stacks}), out_json=str(tmp_path / "tiles.json"))
    outs = api.align_stacks(ctx, devs, prec=1)
    torch.cuda.synchronize()
    rng = np.random.default_rng(14)
    for (L, ref, imgs, size), o in zip(stacks, outs):
        rec = o["res"].cpu().numpy()
        g = api.unpack_results(o["res"])
        check_all(g, L)
        m = len(imgs)
        copies = rec.reshape(-1, 6)[: (size // m) * m].reshape(-1, m, 6)
        assert np.all(copies == copies[:1]), L
        tail = rec[(size // m) * m:]
        assert np.array_equal(tail, rec[: len(tail)]), L
        S = np.unique(np.concatenate([[0, min(m, size) - 1],
                                      rng.choice(min(m, size), 6, replace=False)]))
        orc = oracle.align_images(ref, imgs[S], L, L, want_curve=True)
        parity.check({k: v[S] for k, v in g.items()}, orc, L, parity.TAU_BF16, orc["curve"])


def test_ramp_filtered_full_size(api, ctx, oracle, headline):
    """The ramp-filtered form of the headline workload (10,000 images, two
    images per block in the fused ramp-filtered tables kernel): 24 sampled
    images against the oracle (FP32 and the BF16 form), the sample's fused
    tables bitwise those of the staged launches, every record valid."""
    w, x, _, _, _, _ = headline
    L, n, Q, N = w["L"], w["n"], w["Q"], len(w["imgs"])
    rq, ra = api.tables(ctx, dev(w["ref"][None]), n, Q, ramp=True)
    iq, ia = api.tables(ctx, x, n, Q, ramp=True)
    rng = np.random.default_rng(15)
    S = np.unique(np.concatenate([[0, 1, N - 2, N - 1], rng.choice(N, 20, replace=False)]))
    imgs = w["imgs"][S]
    q5, a5 = api.quantiles(ctx, api.ramp(ctx, api.project(ctx, dev(imgs), n)), Q, ramp=True)
    assert np.array_equal(q5.cpu().numpy(), iq.cpu().numpy()[S])
    assert np.array_equal(a5.cpu().numpy(), ia.cpu().numpy()[S])
    o = oracle.align_images(w["ref"], imgs, n, Q, want_curve=True, ramp=True)
    for prec in (0, 1):
        res, _ = api.align_batch(ctx, rq, ra, iq, ia, L, prec=prec, ramp=True)
        g = api.unpack_results(res)
        check_all(g, n)
        rep = parity.check({k: v[S] for k, v in g.items()}, o, L, parity.TAU_RF, o["curve"])
        print(prec, rep)
