"""GPU parity: every stage of the HIP path against the FP64 oracle on the
same seeded inputs, element by element, through the C ABI.

Sizes span several tiles and ragged tails: L in {16, 40, 64, 96, 128, 192,
256}, n with radix 3 (24, 96, 192), Q != n, both level rules, both modes,
explicit pair lists and top-k rescoring."""
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
def ctxs(api, tmp_path_factory):
    """Contexts for the launch policies of the image stages: the fused tables
    kernel (two images per block where the geometry allows it, or one), and
    several blocks per image (split projection, then the 16-wave quantile
    kernel)."""
    out = {}
    for name, txt in (("perimage", '{"small_batch": 0}'), ("split", '{"small_batch": 1073741824}'),
                      ("one", '{"small_batch": 0, "tables_images_per_block": 1}')):
        path = tmp_path_factory.mktemp("tune") / f"{name}.json"
        path.write_text(txt)
        out[name] = api.Context(0, tune_json=str(path))
    yield out
    for c in out.values():
        c.close()


@pytest.fixture(scope="module")
def ctx(ctxs):
    return ctxs["perimage"]


def dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def blob_stack(L, N, seed, snr=1.0):
    ref, imgs, _, _ = synth.make_stack(seed, L, N, K=6, shift_px=max(1.0, L / 16), jitter_px=1.0,
                                       snr=snr)
    return ref, imgs


def raw_stack(L, N, seed):
    """Unprocessed inputs (negative pixels, mass outside the disk, arbitrary
    scale): the clip and the disk mask are the kernels' to apply."""
    ref, imgs = synth.make_raw_stack(seed, L, N)
    keep = synth.disk_keep(L)
    # every image has negative pixels inside the disk and positive ones
    # outside it (at L >= 64 about a third of the disk is negative; the few
    # disk pixels of the smallest sides may all be positive, then the
    # smallest one is made negative)
    inside = imgs[:, keep]
    for g in np.nonzero(~(inside < 0).any(axis=1))[0]:
        k = int(np.argmin(inside[g]))
        inside[g, k] = -abs(inside[g, k]) - 1.0
    imgs[:, keep] = inside
    assert np.all((imgs[:, keep] < 0).any(axis=1))
    assert np.all((imgs[:, ~keep] > 0).all(axis=1))
    return ref, imgs


def inputs(kind, L, N, seed):
    return raw_stack(L, N, seed) if kind == "raw" else blob_stack(L, N, seed)


# odd sides too: L = 39 is the digits' size in the paper's timings (Table 4)
# with a radix-3 angle count, L = 127 takes the n = 128 register-FFT path
# (176, 144, 144) and (120, 256, 64): seven and eight tasks per wave of a
# 512-thread block (the one-image kernels beyond the two-image one); at
# L = 65 and 82 the one-image strips' height is set by the staging of the
# column runs, not by the LDS
GEOMS = [(8, 8, 8), (16, 16, 16), (39, 48, 48), (40, 24, 20), (64, 64, 64), (65, 48, 48),
         (82, 72, 72), (96, 96, 96), (127, 128, 128), (128, 128, 128), (64, 128, 48),
         (176, 144, 144), (120, 256, 64), (192, 192, 192), (256, 256, 256)]


@pytest.mark.parametrize("kind", ["clean", "raw"])
@pytest.mark.parametrize("policy", ["perimage", "split"])
@pytest.mark.parametrize("L,n,Q", GEOMS)
def test_project_parity(api, ctxs, oracle, L, n, Q, policy, kind):
    """Projections against the oracle's; raw inputs check the positive part
    (Sec. 4.4) and the disk support (Sec. 1.1) inside the kernels."""
    ref, imgs = inputs(kind, L, 5, 100 + L)
    if kind == "clean":
        imgs = np.concatenate([imgs, synth.uniform_images(7, L, 2)])
    pmf = api.project(ctxs[policy], dev(imgs), n).cpu().numpy()
    P0, _ = oracle.project(imgs, n)
    err = np.abs(pmf - P0).max(axis=(1, 2)) / P0.max(axis=(1, 2))
    assert err.max() < 1e-5, err


def test_every_side_projects_and_tables(api, ctxs, oracle):
    """Every side L = 8 .. 256 (odd and even: the strip heights, staging
    passes and column pairs of the four-kind strips change with L), raw
    inputs, n = Q = 8: the one-image projection and the two-image tables (an
    odd count leaves a block with one image) against the oracle."""
    worst_p = worst_q = 0.0
    for L in range(8, 257):
        _, imgs = raw_stack(L, 3, 4000 + L)
        x = dev(imgs)
        P0, _ = oracle.project(imgs, 8)
        pmf = api.project(ctxs["perimage"], x, 8).cpu().numpy()
        ep = (np.abs(pmf - P0).max(axis=(1, 2)) / P0.max(axis=(1, 2))).max()
        assert ep < 1e-5, (L, ep)
        # the fused tables against the oracle's quantiles of the GPU's own FP32
        # projections (the fused and staged projections are bitwise equal)
        q0, _ = oracle.quantiles(pmf.astype(np.float64), 8, 0)
        q1, _ = api.tables(ctxs["perimage"], x, 8, 8)
        eq = np.abs(q1.cpu().numpy() - q0).max()
        assert eq < 2e-6, (L, eq)
        # the one-image fused kernel gives bitwise the same tables
        q2, _ = api.tables(ctxs["one"], x, 8, 8)
        assert np.array_equal(q2.cpu().numpy(), q1.cpu().numpy()), L
        worst_p, worst_q = max(worst_p, ep), max(worst_q, eq)
    print(f"worst relative projection error {worst_p:.2e}, quantile error {worst_q:.2e}")
    # the persistent mixed kernel (stacks of every third side, 20 per launch)
    Ls = list(range(8, 257, 3))
    for c0 in range(0, len(Ls), 20):
        stacks, want = [], []
        for L in Ls[c0:c0 + 20]:
            ref, imgs = raw_stack(L, 3, 5000 + L)
            stacks.append((dev(ref), dev(imgs)))
            want.append(api.tables(ctxs["one"], dev(imgs), 8, 8)[0].cpu().numpy())
        got = api.align_stacks(ctxs["perimage"], stacks, n=8, Q=8)
        for L, g, w in zip(Ls[c0:c0 + 20], got, want):
            assert np.array_equal(g["qt"].cpu().numpy(), w), L


@pytest.mark.parametrize("policy", ["perimage", "split"])
@pytest.mark.parametrize("L,n,Q", GEOMS)
@pytest.mark.parametrize("levels", [0, 1])
def test_quantile_parity(api, ctxs, oracle, L, n, Q, levels, policy):
    _, imgs = blob_stack(L, 4, 200 + L)
    P0, _ = oracle.project(imgs, n)
    pmf32 = P0.astype(np.float32)
    qt, aux = api.quantiles(ctxs[policy], dev(pmf32), Q, levels)
    q0, a0 = oracle.quantiles(pmf32.astype(np.float64), Q, levels)
    qt, aux = qt.cpu().numpy(), aux.cpu().numpy()
    assert np.abs(qt - q0).max() < 2e-6
    assert np.allclose(aux[:, 0], a0[:, 0], rtol=1e-12)
    assert np.allclose(aux[:, 1], a0[:, 1], rtol=1e-6)
    assert np.abs(aux[:, 2:] - a0[:, 2:]).max() < 1e-6


@pytest.mark.parametrize("kind", ["clean", "raw"])
@pytest.mark.parametrize("L,n,Q", GEOMS)
def test_tables_fused_equals_staged(api, ctxs, L, n, Q, kind):
    """Fused (two images or one per block), staged and split launches give
    bitwise-equal tables; an odd count leaves the last two-image block with
    one image."""
    _, imgs = inputs(kind, L, 7, 300 + L)
    imgs[3, 2, 5] = np.nan  # a non-finite image beside a finite one in its block
    x = dev(imgs)
    ctx, cs = ctxs["perimage"], ctxs["split"]
    q1, a1 = api.tables(ctx, x, n, Q)
    q2, a2 = api.quantiles(ctx, api.project(ctx, x, n), Q)
    q3, a3 = api.tables(cs, x, n, Q)
    q4, a4 = api.quantiles(cs, api.project(ctx, x, n), Q)
    q5, a5 = api.tables(ctxs["one"], x, n, Q)
    assert np.isnan(a1.cpu().numpy()[3, 0]) and not np.isnan(a1.cpu().numpy()[2, 0])
    for q, a in ((q2, a2), (q3, a3), (q4, a4), (q5, a5)):
        assert np.array_equal(q1.cpu().numpy(), q.cpu().numpy(), equal_nan=True)
        assert np.array_equal(a1.cpu().numpy(), a.cpu().numpy(), equal_nan=True)


def oracle_results(oracle, rq, ra, iq, ia, L, pairs=None, mode=0):
    return oracle.align(rq, ra, iq, ia, L, pairs=pairs, mode=mode, want_curve=True)


@pytest.mark.parametrize("L,n,Q", GEOMS)
@pytest.mark.parametrize("mode", [0, 1])
def test_align_parity_on_oracle_tables(api, ctx, oracle, L, n, Q, mode):
    """Alignment stage alone: the oracle's tables, rounded to FP32, fed to
    both sides."""
    ref, imgs = blob_stack(L, 12, 400 + L)
    rq, ra = oracle.tables(ref, n, Q)
    iq, ia = oracle.tables(imgs, n, Q)
    rq32, iq32 = rq.astype(np.float32), iq.astype(np.float32)
    res, _ = api.align_batch(ctx, dev(rq32), dev(ra), dev(iq32), dev(ia), L, mode=mode)
    g = api.unpack_results(res)
    o = oracle_results(oracle, rq32.astype(np.float64), ra, iq32.astype(np.float64), ia, L, mode=mode)
    parity.check(g, o, L, parity.TAU_FP32, o["curve"])


@pytest.mark.parametrize("kind", ["clean", "raw"])
@pytest.mark.parametrize("L,n,Q", GEOMS)
def test_end_to_end_parity(api, ctx, oracle, L, n, Q, kind):
    """Images -> tables -> alignment on the GPU against the oracle from the
    same float32 images (raw ones: clipped and masked by the kernels)."""
    ref, imgs = inputs(kind, L, 16, 500 + L)
    rq, ra = api.tables(ctx, dev(ref[None]), n, Q)
    iq, ia = api.tables(ctx, dev(imgs), n, Q)
    res, curve = api.align_batch(ctx, rq, ra, iq, ia, L, want_curve=True)
    g = api.unpack_results(res)
    orq, ora = oracle.tables(ref, n, Q)
    oiq, oia = oracle.tables(imgs, n, Q)
    o = oracle_results(oracle, orq, ora, oiq, oia, L)
    rep = parity.check(g, o, L, parity.TAU_FP32, o["curve"])
    # the D*(l) curve at every lag.  It comes from the spectral cross term,
    # E_U + E_V - 2 C(l) over nQ, whose FP32 cancellation leaves errors of
    # about 1e-7 of the energies; at lags far from the minimum that is well
    # inside 1e-4 relative, near the minimum the curve is small and the
    # energy-relative floor decides, so both are stated
    c = curve.cpu().numpy()
    energy = (ora[0, 1] + oia[:, 1]) / (n * Q)
    tol = parity.dist_tol(o["curve"], L, parity.TAU_FP32) + 1e-6 * energy[:, None]
    assert np.all(np.abs(c - o["curve"]) <= tol)
    print(rep)


@pytest.mark.parametrize("L,n,Q,kind", [(256, 512, 512, "clean"), (256, 512, 512, "raw"),
                                         (96, 384, 8, "raw"), (8, 8, 8, "clean"),
                                         (9, 24, 12, "clean")])
def test_extreme_geometries_end_to_end(api, ctx, oracle, L, n, Q, kind):
    """The largest admissible geometry (L = 256, n = Q = 512: the angle FFT
    at its largest power of two, the fused tables beyond LDS), the largest
    radix-3 angle count with the fewest quantiles, and the smallest sides
    (L = 8, odd L = 9): images to results against the oracle."""
    ref, imgs = inputs(kind, L, 3, 950 + L + n)
    rq, ra = api.tables(ctx, dev(ref[None]), n, Q)
    iq, ia = api.tables(ctx, dev(imgs), n, Q)
    res, _ = api.align_batch(ctx, rq, ra, iq, ia, L)
    g = api.unpack_results(res)
    orq, ora = oracle.tables(ref, n, Q)
    oiq, oia = oracle.tables(imgs, n, Q)
    o = oracle_results(oracle, orq, ora, oiq, oia, L)
    assert np.abs(iq.cpu().numpy() - oiq).max() < 2e-6 * max(1.0, np.abs(oiq).max())
    parity.check(g, o, L, parity.TAU_FP32, o["curve"])


def test_single_pair_workload(api, ctx, oracle):
    """The single-pair workload (L = 64, 5 blobs, +-4 px) end to end."""
    w = synth.workload(0)
    L, n, Q = w["L"], w["n"], w["Q"]
    rq, ra = api.tables(ctx, dev(w["ref"][None]), n, Q)
    iq, ia = api.tables(ctx, dev(w["imgs"]), n, Q)
    res, _ = api.align_batch(ctx, rq, ra, iq, ia, L)
    g = api.unpack_results(res)
    o = oracle.align_images(w["ref"], w["imgs"], n, Q, want_curve=True)
    parity.check(g, o, L, parity.TAU_FP32, o["curve"])


def test_pairs_list_and_topk(api, ctx, oracle):
    import torch

    L, n, Q = 64, 64, 64
    _, imgs = blob_stack(L, 10, 600)
    q, a = api.tables(ctx, dev(imgs), n, Q)
    rng = np.random.default_rng(3)
    pairs = rng.integers(0, 10, size=(37, 2)).astype(np.int64)
    res, _ = api.align_batch(ctx, q, a, q, a, L, pairs=dev(pairs), top_k=4)
    g = api.unpack_results(res)
    oq, oa = oracle.tables(imgs, n, Q)
    o = oracle_results(oracle, oq, oa, oq, oa, L, pairs=pairs)
    parity.check(g, o, L, parity.TAU_FP32, o["curve"])
    # diagonal pairs are exactly zero
    diag = pairs[:, 0] == pairs[:, 1]
    assert np.all(g["sw2sq"][diag] == 0.0) and np.all(g["rot_index"][diag] == 0)
    del torch


def test_bf16_split_within_tolerance(api, ctx, oracle):
    L, n, Q = 128, 128, 128
    ref, imgs = blob_stack(L, 24, 700)
    rq, ra = api.tables(ctx, dev(ref[None]), n, Q)
    iq, ia = api.tables(ctx, dev(imgs), n, Q)
    res, _ = api.align_batch(ctx, rq, ra, iq, ia, L, prec=1)
    g = api.unpack_results(res)
    o = oracle.align_images(ref, imgs, n, Q, want_curve=True)
    parity.check(g, o, L, parity.TAU_BF16, o["curve"])


@pytest.mark.parametrize("m", [1, 2, 3])
def test_quarter_turns_and_self(api, ctx, m):
    L, n = 96, 96
    _, imgs = blob_stack(L, 1, 800, snr=None)
    f = imgs[0]
    g = np.ascontiguousarray(np.rot90(f, m))
    q, a = api.tables(ctx, dev(np.stack([f, g])), n, n)
    res, _ = api.align_batch(ctx, q[:1].contiguous(), a[:1].contiguous(), q, a, L)
    r = api.unpack_results(res)
    assert r["rot_index"][0] == 0 and r["sw2sq"][0] == 0.0
    assert r["rot_index"][1] == (m * n // 4) % n
    assert r["sw2sq"][1] < 1e-9 and np.all(np.abs(r["shift_px"][1]) < 1e-3)


def test_deterministic_and_independent_of_batch(api, ctx):
    """Same input twice gives bitwise-equal results, and a pair's result does
    not depend on what else is in the batch."""
    L, n = 64, 64
    ref, imgs = blob_stack(L, 30, 900)
    x = dev(imgs)
    q1, a1 = api.tables(ctx, x, n, n)
    q2, a2 = api.tables(ctx, x, n, n)
    assert np.array_equal(q1.cpu().numpy(), q2.cpu().numpy())
    rq, ra = api.tables(ctx, dev(ref[None]), n, n)
    r_all, _ = api.align_batch(ctx, rq, ra, q1, a1, L)
    r_one, _ = api.align_batch(ctx, rq, ra, q1[7:8].contiguous(), a1[7:8].contiguous(), L)
    assert np.array_equal(r_all.cpu().numpy()[7], r_one.cpu().numpy()[0])
    q3, a3 = api.tables(ctx, x[7:8].contiguous(), n, n)
    assert np.array_equal(q3.cpu().numpy()[0], q1.cpu().numpy()[7])
    # the default policy (one image: split launches) agrees bitwise
    c = api.Context(0)
    q4, a4 = api.tables(c, x[7:8].contiguous(), n, n)
    c.close()
    assert np.array_equal(q4.cpu().numpy()[0], q1.cpu().numpy()[7])
    assert np.array_equal(a4.cpu().numpy()[0], a1.cpu().numpy()[7])


@pytest.mark.parametrize("L", [32, 64, 128])
def test_mass_only_outside_disk_is_zero_mass(api, ctx, oracle, L):
    """Positive values only outside radius 1 - h (negative inside): after the
    clip and the disk mask nothing is left, so the image has zero mass on
    both sides; one positive pixel just inside the disk restores it."""
    keep = synth.disk_keep(L)
    rng = np.random.default_rng(L)
    imgs = np.zeros((3, L, L), np.float32)
    imgs[:] = np.where(keep, -rng.uniform(0.1, 1.0, (L, L)), rng.uniform(1.0, 5.0, (L, L)))
    ii, jj = np.nonzero(keep)
    edge = np.argmax(np.hypot(ii - (L - 1) / 2, jj - (L - 1) / 2))
    imgs[1, ii[edge], jj[edge]] = 2.0  # the outermost pixel kept by the mask
    imgs[2, L // 2, L // 3] = 1.0
    q, a = api.tables(ctx, dev(imgs), L, L)
    aa = a.cpu().numpy()
    _, oa = oracle.tables(imgs, L, L)
    assert aa[0, 0] == 0.0 and oa[0, 0] == 0.0
    assert np.allclose(aa[1:, 0], oa[1:, 0], rtol=1e-12) and np.all(oa[1:, 0] > 0)
    res, _ = api.align_batch(ctx, q[2:].contiguous(), a[2:].contiguous(), q, a, L)
    r = api.unpack_results(res)
    assert list(r["status"]) == [1, 0, 0]


def test_status_codes_and_empty(api, ctx):
    import torch

    L, n = 32, 32
    _, imgs = blob_stack(L, 3, 1000)
    imgs[1] = 0.0
    imgs[2, 5, 5] = np.nan
    q, a = api.tables(ctx, dev(imgs), n, n)
    res, _ = api.align_batch(ctx, q[:1].contiguous(), a[:1].contiguous(), q, a, L)
    r = api.unpack_results(res)
    assert list(r["status"]) == [0, 1, 2]
    # N = 0 is a no-op
    e = torch.empty((0, L, L), dtype=torch.float32, device="cuda")
    q0, a0 = api.tables(ctx, e, n, n)
    assert q0.shape[0] == 0


# ---------------------------------------------------------------- many-vs-many (MFMA)
@pytest.mark.parametrize("L,n,nr,ni", [(64, 64, 40, 40), (32, 32, 37, 53), (64, 64, 16, 17)])
def test_all_pairs_mfma_parity(api, ctx, oracle, L, n, nr, ni):
    """All reference x image pairs on the matrix cores (bf16 spectra, FP32
    accumulate, top-4 FP32 rescore), ragged tiles, BF16 tolerance."""
    _, imgs = blob_stack(L, max(nr, ni), 1100 + nr)
    rq, ra = api.tables(ctx, dev(imgs[:nr]), n, n)
    iq, ia = api.tables(ctx, dev(imgs[:ni]), n, n)
    res, _ = api.align_batch(ctx, rq, ra, iq, ia, L, prec=1, top_k=4)
    g = api.unpack_results(res)
    oq, oa = oracle.tables(imgs, n, n)
    o = oracle_results(oracle, oq[:nr], oa[:nr], oq[:ni], oa[:ni], L)
    parity.check(g, o, L, parity.TAU_BF16, o["curve"])
    # the same image against itself: lag 0, distance exactly 0
    m = min(nr, ni)
    diag = np.arange(m) * ni + np.arange(m)
    assert np.all(g["rot_index"][diag] == 0) and np.all(g["sw2sq"][diag] == 0.0)


@pytest.mark.parametrize("L,n,mode,top_k", [(64, 64, 1, 4), (32, 32, 1, 2), (64, 64, 0, 1),
                                            (32, 32, 0, 3)])
def test_all_pairs_mfma_modes_and_topk(api, ctx, oracle, L, n, mode, top_k):
    """All pairs on the matrix cores in rotation-only mode (no correction
    folded into the spectra) and with fewer than four candidates, against
    the oracle with the same mode, BF16 tolerance."""
    nr, ni = 19, 33
    _, imgs = blob_stack(L, ni, 1300 + 10 * mode + top_k)
    rq, ra = api.tables(ctx, dev(imgs[:nr]), n, n)
    iq, ia = api.tables(ctx, dev(imgs), n, n)
    res, _ = api.align_batch(ctx, rq, ra, iq, ia, L, mode=mode, prec=1, top_k=top_k)
    g = api.unpack_results(res)
    oq, oa = oracle.tables(imgs, n, n)
    o = oracle_results(oracle, oq[:nr], oa[:nr], oq, oa, L, mode=mode)
    parity.check(g, o, L, parity.TAU_BF16, o["curve"])


def test_all_pairs_mfma_same_set_sampled(api, ctx, oracle):
    """One set against itself (spectra computed once), 300 x 300 at L = 64,
    checked on a seeded sample of 400 pairs."""
    L, n, N = 64, 64, 300
    _, imgs = blob_stack(L, N, 1200)
    q, a = api.tables(ctx, dev(imgs), n, n)
    res, _ = api.align_batch(ctx, q, a, q, a, L, prec=1)
    g = api.unpack_results(res)
    rng = np.random.default_rng(5)
    pairs = np.stack([rng.integers(0, N, 400), rng.integers(0, N, 400)], axis=1).astype(np.int64)
    pidx = pairs[:, 0] * N + pairs[:, 1]
    oq, oa = oracle.tables(imgs, n, n)
    o = oracle_results(oracle, oq, oa, oq, oa, L, pairs=pairs)
    sub = {k: v[pidx] for k, v in g.items()}
    parity.check(sub, o, L, parity.TAU_BF16, o["curve"])


@pytest.fixture(scope="module")
def ctx_generic(api, tmp_path_factory):
    """Context that keeps n = 128 alignments on the LDS-FFT pair kernel."""
    path = tmp_path_factory.mktemp("tune") / "generic.json"
    path.write_text('{"align_kernel": "generic"}')
    c = api.Context(0, tune_json=str(path))
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctx_block(api, tmp_path_factory):
    """Context that runs the n = 128 register-FFT alignment one pair per
    block instead of one pair per wave."""
    path = tmp_path_factory.mktemp("tune") / "block128.json"
    path.write_text('{"align_kernel": "block128"}')
    c = api.Context(0, tune_json=str(path))
    yield c
    c.close()


@pytest.mark.parametrize("Q", [48, 128, 256])
@pytest.mark.parametrize("mode,prec,top_k", [(0, 0, 1), (1, 0, 3), (0, 1, 4), (0, 0, 8)])
def test_align128_wave_and_block_agree(api, ctx, ctx_block, oracle, Q, mode, prec, top_k):
    """One pair per wave and one pair per block: the same arithmetic summed in
    another order, so the same lags and distances to FP32 rounding, and both
    within the oracle's tolerance; pair lists with an out-of-range index and a
    self pair."""
    L, n = 127, 128
    ref, imgs = blob_stack(L, 21, 1300 + Q)
    x = dev(np.concatenate([ref[None], imgs]))
    q, a = api.tables(ctx, x, n, Q)
    pairs = np.array([[0, i] for i in range(1, 22)] + [[4, 4], [7, 2], [0, 99]], np.int64)
    r1, c1 = api.align_batch(ctx, q, a, q, a, L, pairs=dev(pairs), mode=mode, prec=prec,
                             top_k=top_k, want_curve=True)
    r2, c2 = api.align_batch(ctx_block, q, a, q, a, L, pairs=dev(pairs), mode=mode, prec=prec,
                             top_k=top_k, want_curve=True)
    g1, g2 = api.unpack_results(r1), api.unpack_results(r2)
    assert g1["status"][-1] == 3 and g2["status"][-1] == 3
    assert np.isnan(c1.cpu().numpy()[-1]).all() and np.isnan(c2.cpu().numpy()[-1]).all()
    oq, oa = oracle.tables(np.concatenate([ref[None], imgs]), n, Q)
    o = oracle.align(oq, oa, oq, oa, L, pairs=pairs[:-1], mode=mode, want_curve=True)
    tau = parity.TAU_FP32 if prec == 0 else parity.TAU_BF16
    for g in (g1, g2):
        parity.check({k: v[:-1] for k, v in g.items()}, o, L, tau, o["curve"])
        assert g["sw2sq"][21] == 0.0 and g["rot_index"][21] == 0  # the self pair
    ok = g1["status"] == 0
    same = ok & (g1["rot_index"] == g2["rot_index"])
    assert same.sum() >= ok.sum() - 1
    assert np.allclose(g1["sw2sq"][same], g2["sw2sq"][same], rtol=1e-5, atol=1e-9)
    c1, c2 = c1.cpu().numpy()[:-1], c2.cpu().numpy()[:-1]
    floor = 1e-5 * np.abs(c2).max(axis=1, keepdims=True)
    assert np.all(np.abs(c1 - c2) <= 1e-4 * np.abs(c2) + floor)


@pytest.mark.parametrize("Q", [48, 128, 256])
@pytest.mark.parametrize("mode,prec,top_k", [(0, 0, 1), (1, 0, 3), (0, 1, 4), (0, 0, 8)])
def test_align128_matches_oracle_and_generic(api, ctx, ctx_generic, oracle, Q, mode, prec, top_k):
    """The n = 128 register-FFT kernel against the oracle (tie-aware parity)
    and against the LDS-FFT kernel: same lags, distances and curves to FP32
    rounding; pair lists with an out-of-range index and a self pair."""
    L, n = 96, 128
    ref, imgs = blob_stack(L, 13, 1100 + Q)
    x = dev(np.concatenate([ref[None], imgs]))
    q, a = api.tables(ctx, x, n, Q)
    pairs = np.array([[0, i] for i in range(1, 14)] + [[3, 3], [5, 2], [0, 99]], np.int64)
    r1, c1 = api.align_batch(ctx, q, a, q, a, L, pairs=dev(pairs), mode=mode, prec=prec,
                             top_k=top_k, want_curve=True)
    r2, c2 = api.align_batch(ctx_generic, q, a, q, a, L, pairs=dev(pairs), mode=mode, prec=prec,
                             top_k=top_k, want_curve=True)
    g1, g2 = api.unpack_results(r1), api.unpack_results(r2)
    assert g1["status"][-1] == 3 and g2["status"][-1] == 3
    ok = g1["status"] == 0
    oq, oa = oracle.tables(np.concatenate([ref[None], imgs]), n, Q)
    o = oracle.align(oq, oa, oq, oa, L, pairs=pairs[:-1], mode=mode, want_curve=True)
    sub = {k: v[:-1] for k, v in g1.items()}
    parity.check(sub, o, L, parity.TAU_FP32 if prec == 0 else parity.TAU_BF16, o["curve"])
    if prec == 0:
        assert np.array_equal(g1["rot_index"][ok], g2["rot_index"][ok])
    same = ok & (g1["rot_index"] == g2["rot_index"])
    assert same.sum() >= ok.sum() - 1
    assert np.allclose(g1["sw2sq"][same], g2["sw2sq"][same], rtol=1e-5, atol=1e-9)
    # the curves come from the spectral path (FP32 cross term cancelling the
    # energies), so the floor scales with the largest value of each curve
    c1, c2 = c1.cpu().numpy()[:-1], c2.cpu().numpy()[:-1]
    if prec == 0:
        floor = 1e-5 * np.abs(c2).max(axis=1, keepdims=True)
        assert np.all(np.abs(c1 - c2) <= 1e-4 * np.abs(c2) + floor)
    else:
        # bf16 operands: the cross term is good to the bf16 epsilon of the
        # energies, rounded differently by the two kernels
        aa = a.cpu().numpy()
        energy = (aa[pairs[:-1, 0], 1] + aa[pairs[:-1, 1], 1]) / (n * Q)
        assert np.all(np.abs(c1 - c2) <= 2.0 ** -7 * energy[:, None])
    assert g1["sw2sq"][13] == 0.0 and g1["rot_index"][13] == 0  # the self pair


def test_align128_one_vs_many_batch_independent(api, ctx):
    """Reference x image grid at n = 128: a pair's record does not depend on
    the batch it is computed in."""
    L, n = 128, 128
    ref, imgs = blob_stack(L, 40, 1200)
    rq, ra = api.tables(ctx, dev(ref[None]), n, n)
    iq, ia = api.tables(ctx, dev(imgs), n, n)
    r_all, _ = api.align_batch(ctx, rq, ra, iq, ia, L)
    r_one, _ = api.align_batch(ctx, rq, ra, iq[17:18].contiguous(), ia[17:18].contiguous(), L)
    assert np.array_equal(r_all.cpu().numpy()[17], r_one.cpu().numpy()[0])


@pytest.mark.parametrize("prec", [0, 1])
def test_align128_repeat_bitwise(api, ctx, prec):
    """The n = 128 alignment copies table rows into LDS areas that its own
    reads of earlier rows share: repeated runs must give bitwise the same
    records and D*(l) curves (a copy landing before those reads returned
    once changed one pair's curve in a dozen runs)."""
    L, n = 128, 128
    ref, imgs = blob_stack(L, 400, 1700 + prec)
    rq, ra = api.tables(ctx, dev(ref[None]), n, n)
    iq, ia = api.tables(ctx, dev(imgs), n, n)
    r0, c0 = api.align_batch(ctx, rq, ra, iq, ia, L, prec=prec, want_curve=True)
    r0, c0 = r0.cpu().numpy(), c0.cpu().numpy()
    for _ in range(8):
        r, c = api.align_batch(ctx, rq, ra, iq, ia, L, prec=prec, want_curve=True)
        assert np.array_equal(r.cpu().numpy(), r0)
        assert np.array_equal(c.cpu().numpy(), c0)
