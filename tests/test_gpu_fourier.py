"""GPU parity of the Fourier-slice projector (type-2 NUFFT on an oversampled
grid, slices back to the detector by FP32 inverse FFTs) against the FP64
oracle's exact non-uniform DFT, through the C ABI."""
import numpy as np
import pytest

import synth
from tests import parity

pytestmark = pytest.mark.gpu

# NUFFT kernel error (about 5e-7 of the largest value with the width-7
# kernel, measured in FP64) plus FP32 rounding through two 2L-point and one
# L-point FFT (observed below 1e-6): 5e-6 of the image's largest projection value
TOL_PROJ = 5e-6

# powers of two (shift-indexed transforms) and other even L with factors 2
# and 3 (mixed-radix transforms of lengths L and 2L)
FGEOMS = [(8, 8, 8), (16, 16, 16), (32, 24, 16), (64, 64, 64), (128, 128, 128), (256, 64, 32),
          (12, 16, 8), (18, 16, 16), (24, 24, 24), (48, 48, 48), (96, 96, 96), (192, 48, 24)]


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


def raw_stack(L, N, seed):
    """Unprocessed inputs: negative pixels, mass outside the disk, any scale."""
    return synth.make_raw_stack(seed, L, N)


def proj_err(pmf, P0):
    """Largest deviation per image relative to its largest oracle value."""
    P0 = np.maximum(P0, 0.0)
    return np.abs(pmf - P0).max(axis=(1, 2)) / P0.max(axis=(1, 2))


@pytest.mark.parametrize("kind", ["clean", "raw"])
@pytest.mark.parametrize("L,n,Q", FGEOMS)
def test_fourier_projection_parity(api, ctx, oracle, L, n, Q, kind):
    """Blob images and uniform noise: every clipped projection value against
    the oracle's (clipped) exact DFT route.  Raw inputs (negative pixels,
    mass outside the disk) check the kernel's own positive part and mask."""
    N = 2 if L >= 128 else 4
    if kind == "raw":
        _, imgs = raw_stack(L, N + 1, 310 + L)
    else:
        _, imgs = blob_stack(L, N, 300 + L)
        imgs = np.concatenate([imgs, synth.uniform_images(11, L, 1)])
    pmf = api.project_fourier(ctx, dev(imgs), n).cpu().numpy()
    P0, _ = oracle.fourier_project(imgs, n)
    err = proj_err(pmf, P0)
    assert err.max() < TOL_PROJ, err


def test_fourier_more_images_than_slots(api, ctx, oracle):
    """A batch larger than the persistent grid (up to four blocks per CU): sampled
    images across the slot wrap-around, and a ragged end."""
    import torch

    L, n = 16, 16
    N = 4 * torch.cuda.get_device_properties(0).multi_processor_count + 37
    imgs = synth.uniform_images(12, L, N)
    pmf = api.project_fourier(ctx, dev(imgs), n).cpu().numpy()
    idx = [0, 1, N // 2, N - 38, N - 37, N - 1]
    P0, _ = oracle.fourier_project(imgs[idx], n)
    assert proj_err(pmf[idx], P0).max() < TOL_PROJ


def test_fourier_mass_half_turn_and_edge_cases(api, ctx):
    """Column sums carry the image mass up to the clipped negative lobes; the
    theta + pi mirror is exact; an empty image projects to zeros, an image
    with a NaN to NaN, N = 0 is a no-op."""
    import torch

    L, n = 64, 32
    _, imgs = blob_stack(L, 3, 77)
    zero = np.zeros((1, L, L), np.float32)
    nan = imgs[:1].copy()
    nan[0, 5, 9] = np.nan
    batch = np.concatenate([imgs, zero, nan])
    pmf = api.project_fourier(ctx, dev(batch), n).cpu().numpy()
    i, j = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    disk = (2 * j - L + 1) ** 2 + (2 * i - L + 1) ** 2 <= (L - 2) ** 2
    m = np.where(disk, np.maximum(imgs.astype(np.float64), 0), 0).sum(axis=(1, 2))
    cols = pmf[:3].sum(axis=2)
    assert np.all(cols >= m[:, None] * (1 - 1e-4))
    assert np.all(np.abs(cols - cols[:, :1]) < 2e-2 * cols[:, :1])
    assert np.array_equal(pmf[:3, n // 2:], pmf[:3, :n // 2, ::-1])
    assert np.all(pmf[3] == 0)
    assert np.all(np.isnan(pmf[4]))
    out = torch.full((1, n, L), 7.0, device="cuda")
    api.project_fourier(ctx, dev(imgs[:0]), n, out=out[:0])
    assert float(out.min()) == 7.0


def test_fourier_rejects_other_sizes(api, ctx):
    """L must be even with prime factors 2 and 3: other sizes (odd, or with a
    factor 5) are refused with an error, no launch."""
    for L in (27, 40):
        imgs = synth.uniform_images(3, L, 2)
        with pytest.raises(RuntimeError, match="factors 2 and 3"):
            api.project_fourier(ctx, dev(imgs), 24)


@pytest.mark.parametrize("L,n,Q,kind", [(32, 32, 32, "clean"), (64, 64, 64, "clean"),
                                        (128, 128, 128, "clean"), (64, 64, 64, "raw"),
                                        (128, 128, 128, "raw"), (96, 96, 96, "clean"),
                                        (48, 48, 48, "raw")])
def test_fourier_tables_and_alignment(api, ctx, oracle, L, n, Q, kind):
    """Images -> Fourier-slice tables -> alignment on the GPU against the
    oracle from the same images: tables, rotation (tie-aware), shift and
    distance."""
    N = 8 if L == 128 else 16
    ref, imgs = (raw_stack if kind == "raw" else blob_stack)(L, N, 500 + L)
    rq, ra = api.tables_fourier(ctx, dev(ref[None]), n, Q)
    iq, ia = api.tables_fourier(ctx, dev(imgs), n, Q)
    oq, oa = oracle.fourier_tables(ref[None], n, Q)
    iq0, ia0 = oracle.fourier_tables(imgs, n, Q)
    assert np.abs(iq.cpu().numpy() - iq0).max() < 2e-3
    res, _ = api.align_batch(ctx, rq, ra, iq, ia, L, want_curve=True)
    g = api.unpack_results(res)
    o = oracle.align(oq, oa, iq0, ia0, L, want_curve=True)
    parity.check(g, o, L, parity.TAU_FP32, o["curve"])


# ---------------------------------------------------------------- explicit angles, Monte-Carlo SW2
@pytest.mark.parametrize("L,n", [(16, 16), (64, 48), (128, 128), (96, 64)])
def test_fourier_at_random_angles_parity(api, ctx, oracle, L, n):
    """Slices at sorted random directions (each computed on its own, no
    half-turn mirror) against the oracle's exact DFT at the same angles."""
    theta = synth.mc_angles(n, 40 + L)
    _, imgs = blob_stack(L, 2, 700 + L)
    pmf = api.project_fourier(ctx, dev(imgs), n, theta=theta).cpu().numpy()
    P0, _ = oracle.fourier_project(imgs, n, angles=theta)
    assert proj_err(pmf, P0).max() < TOL_PROJ


def test_fourier_at_grid_angles_equals_default(api, ctx):
    """Explicit angles equal to the grid give the default projections: both
    approximate the same exact values to TOL_PROJ (the slices at theta + pi
    are computed directly here and mirrored by default)."""
    L, n = 64, 32
    _, imgs = blob_stack(L, 3, 91)
    a = api.project_fourier(ctx, dev(imgs), n).cpu().numpy()
    b = api.project_fourier(ctx, dev(imgs), n, theta=2 * np.pi * np.arange(n) / n).cpu().numpy()
    assert np.abs(a - b).max() <= 2 * TOL_PROJ * a.max(axis=(1, 2)).min()


def test_fourier_at_rejects_bad_angles(api, ctx):
    imgs = synth.uniform_images(5, 32, 1)
    th = np.zeros(16)
    th[3] = np.nan
    with pytest.raises(RuntimeError, match="not finite"):
        api.project_fourier(ctx, dev(imgs), 16, theta=th)


@pytest.mark.parametrize("L,n,Q", [(32, 64, 32), (128, 128, 128)])
def test_monte_carlo_sw_alignment_parity(api, ctx, oracle, L, n, Q):
    """Monte-Carlo SW2 over rotations: tables at sorted random directions,
    rotation-only scan on the GPU, against the oracle (rotation tie-aware,
    distance)."""
    theta = synth.mc_angles(n, 77)
    N = 6 if L == 128 else 12
    ref, imgs = blob_stack(L, N, 800 + L)
    rq, ra = api.tables_fourier(ctx, dev(ref[None]), n, Q, theta=theta)
    iq, ia = api.tables_fourier(ctx, dev(imgs), n, Q, theta=theta)
    res, _ = api.align_batch(ctx, rq, ra, iq, ia, L, mode=1, want_curve=True)
    g = api.unpack_results(res)
    o = oracle.mc_align_images(ref[None], imgs, n, Q, theta, want_curve=True)
    parity.check(g, o, L, parity.TAU_FP32, o["curve"])
