"""Seeded synthetic inputs for the alignment workloads.

This module only draws and renders input images: it holds none of the
alignment arithmetic and is shared, as plain numpy arrays, by the oracle tests
and by the GPU path.  Images are sums of isotropic Gaussian blobs standing in
for the paper's MNIST and cryo-EM data (neither is available here); target
copies are rotated, shifted, jittered and optionally noisy, following the
paper's experimental recipe (Sec. 4.4: uniform random rotation in [0, 2 pi),
pixel shifts, additive white Gaussian noise at a given SNR with the positive
part kept and renormalised).

Coordinates: pixel (i, j) of an L x L image sits at x = (j - (L-1)/2) h,
y = (i - (L-1)/2) h with h = 2 / L, i.e. x runs along +column and y along
+row.  A blob is a * exp(-|p - c|^2 / (2 sigma^2)), point-sampled at pixel
centres.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 1000


def _grid(L):
    h = 2.0 / L
    ax = (np.arange(L, dtype=np.float64) - 0.5 * (L - 1)) * h
    return ax, h


def disk_keep(L):
    """Pixels whose centre lies within radius 1 - h of the origin."""
    ax, h = _grid(L)
    rr = np.hypot(ax[None, :], ax[:, None])
    return rr <= (1.0 - h) * (1.0 + 1e-12)


def render(centres, sigmas, amps, L):
    """Sum of Gaussian blobs, float64 [L, L]; separable evaluation."""
    ax, _ = _grid(L)
    img = np.zeros((L, L), np.float64)
    for (cx, cy), s, a in zip(centres, sigmas, amps):
        gx = np.exp(-((ax - cx) ** 2) / (2.0 * s * s))
        gy = np.exp(-((ax - cy) ** 2) / (2.0 * s * s))
        img += a * np.outer(gy, gx)
    return img


def blob_params(rng, K, L, spread=0.6, sig_px=(2.0, 6.0), amp=(0.5, 1.5)):
    h = 2.0 / L
    centres = rng.uniform(-spread, spread, size=(K, 2))
    sigmas = rng.uniform(sig_px[0], sig_px[1], size=K) * h
    amps = rng.uniform(amp[0], amp[1], size=K)
    return centres, sigmas, amps


def finish(img, L, noise=None):
    """Optional additive noise, clip at 0, disk mask, unit mass; -> float32."""
    x = img if noise is None else img + noise
    x = np.where(x > 0.0, x, 0.0)
    x = np.where(disk_keep(L), x, 0.0)
    s = x.sum()
    if s > 0:
        x = x / s
    return x.astype(np.float32)


def rot(phi):
    c, s = math.cos(phi), math.sin(phi)
    return np.array([[c, -s], [s, c]])


def copies(rng, params, L, N, shift_px, jitter_px, snr):
    """N rotated/shifted/jittered (noisy) copies of a blob image.

    Draw order per copy: phi, t (2), jitter (K x 2), noise field (L*L).
    Returns images [N, L, L] float32 and the ground truth (theta, s_px) that
    aligns each copy back onto the reference: B ~ T_t R_phi A implies
    A ~ T_{-R_{-phi} t} R_{-phi} B."""
    centres, sigmas, amps = params
    K = len(amps)
    h = 2.0 / L
    clean0 = render(centres, sigmas, amps, L)
    out = np.zeros((N, L, L), np.float32)
    truth_theta = np.zeros(N)
    truth_shift = np.zeros((N, 2))
    for g in range(N):
        phi = rng.uniform(0.0, 2.0 * math.pi)
        t = rng.uniform(-shift_px, shift_px, size=2) * h
        eps = rng.normal(0.0, jitter_px, size=(K, 2)) * h if jitter_px > 0 else np.zeros((K, 2))
        c2 = centres @ rot(phi).T + t[None, :] + eps
        clean = render(c2, sigmas, amps, L)
        noise = None
        if snr is not None:
            sd = math.sqrt(clean.var() / snr)
            noise = rng.normal(0.0, sd, size=(L, L))
        out[g] = finish(clean, L, noise)
        truth_theta[g] = (-phi) % (2.0 * math.pi)
        truth_shift[g] = -(rot(-phi) @ t) / h
    del clean0
    return out, truth_theta, truth_shift


def raw_image(rng, clean, L, snr, corner=True, scale_range=(0.01, 100.0)):
    """An unprocessed image: `clean` plus white noise at `snr` (when given),
    NOT clipped, masked or normalised, times a log-uniform overall scale, with
    (when `corner`) positive values uniform in [0, 2 max(clean)] on every
    pixel outside radius 1 - h.  Draw order: noise field (L*L), scale, corner
    field (L*L).  The positive-part rule and the disk support are left to the
    code under test."""
    x = clean.copy()
    if snr is not None:
        sd = math.sqrt(clean.var() / snr)
        x = x + rng.normal(0.0, sd, size=(L, L))
    scale = math.exp(rng.uniform(math.log(scale_range[0]), math.log(scale_range[1])))
    if corner:
        c = rng.uniform(0.0, 2.0 * clean.max(), size=(L, L))
        x = np.where(disk_keep(L), x, c)
    return (x * scale).astype(np.float32)


def make_raw_stack(seed, L, N, K=6, shift_px=None, jitter_px=1.0, snr=1.0):
    """Like make_stack, but reference and copies are raw (see raw_image): the
    reference noisy as well, every image with about half its pixels negative,
    mass outside the disk and its own scale.  Per copy: phi, t, jitter, then
    raw_image's draws."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = 2.0 / L
    shift_px = max(1.0, L / 16) if shift_px is None else shift_px
    centres, sigmas, amps = blob_params(rng, K, L)
    ref = raw_image(rng, render(centres, sigmas, amps, L), L, snr)
    out = np.zeros((N, L, L), np.float32)
    for g in range(N):
        phi = rng.uniform(0.0, 2.0 * math.pi)
        t = rng.uniform(-shift_px, shift_px, size=2) * h
        eps = rng.normal(0.0, jitter_px, size=(K, 2)) * h
        c2 = centres @ rot(phi).T + t[None, :] + eps
        out[g] = raw_image(rng, render(c2, sigmas, amps, L), L, snr)
    return ref, out


def make_pair(seed=SEED_BASE, L=64, K=5, shift_px=4.0, jitter_px=1.0):
    """Single pair: reference A (K blobs) and one rotated/shifted copy B."""
    rng = np.random.Generator(np.random.PCG64(seed))
    params = blob_params(rng, K, L)
    ref = finish(render(*params, L), L)
    imgs, th, sh = copies(rng, params, L, 1, shift_px, jitter_px, None)
    return ref, imgs, th, sh


def make_stack(seed, L, N, K=8, shift_px=8.0, jitter_px=2.0, snr=1.0):
    """One clean reference and N noisy copies (the 1-vs-many workload)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    params = blob_params(rng, K, L)
    ref = finish(render(*params, L), L)
    imgs, th, sh = copies(rng, params, L, N, shift_px, jitter_px, snr)
    return ref, imgs, th, sh


def uniform_images(seed, L, N):
    """Dense U[0,1) images (the paper's timing inputs, Sec. 4.1), masked and
    normalised."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.zeros((N, L, L), np.float32)
    for g in range(N):
        out[g] = finish(rng.uniform(0.0, 1.0, size=(L, L)), L)
    return out


def mc_angles(n, seed):
    """n directions drawn uniformly on the circle (PCG64, `seed`), sorted: the
    random draw of Monte-Carlo sliced Wasserstein (an input to the method)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.uniform(0.0, 2.0 * math.pi, n))


def gaussian_image(L, centre, sigma):
    """A single isotropic Gaussian (unit coordinates), masked, unit mass."""
    return finish(render([centre], [sigma], [1.0], L), L)


WORKLOADS = {
    0: dict(desc="single pair, L=64, 5 blobs, +-4 px, jitter 1 px, no noise", L=64, n=64, Q=64),
    1: dict(desc="1 reference vs 10,000 images, L=128, 8 blobs, +-8 px, jitter 2 px, SNR 1",
            L=128, n=128, Q=128, N=10000),
    2: dict(desc="all pairs 2,000 x 2,000, L=64, images as in the 1-vs-many workload",
            L=64, n=64, Q=64, N=2000),
}


def workload(idx, N=None):
    """Inputs of a named workload: dict(ref, imgs, truth_theta, truth_shift, L, n, Q)."""
    w = dict(WORKLOADS[idx])
    seed = SEED_BASE + idx
    if idx == 0:
        ref, imgs, th, sh = make_pair(seed, L=64, K=5, shift_px=4.0, jitter_px=1.0)
    else:
        NN = w["N"] if N is None else N
        ref, imgs, th, sh = make_stack(seed, w["L"], NN, K=8, shift_px=8.0, jitter_px=2.0, snr=1.0)
    w.update(ref=ref, imgs=imgs, truth_theta=th, truth_shift=sh)
    return w


def uneven_stacks(seed=SEED_BASE + 3, total=50000, Ls=(64, 96, 128, 192, 256),
                  size_range=(100, 5000), cap_per_stack=None):
    """Stacks of mixed side length: list of (L, ref, imgs).  Sizes are drawn
    until `total` images are reached (the last stack truncated); each stack has
    its own 8-blob reference.  `cap_per_stack` renders only that many images
    per stack (for tests) while keeping the drawn sizes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    left = total
    while left > 0:
        L = int(rng.choice(Ls))
        size = int(rng.integers(size_range[0], size_range[1] + 1))
        size = min(size, left)
        left -= size
        sub = int(rng.integers(0, 2**31 - 1))
        nrender = size if cap_per_stack is None else min(size, cap_per_stack)
        ref, imgs, _, _ = make_stack(sub, L, nrender)
        out.append((L, ref, imgs, size))
    return out


def serving_trace(seed=SEED_BASE + 4, n_req=2000, Ls=(64, 128, 256), nmax=5000):
    """Request sizes and side lengths of the serving trace: list of
    (L, N, sub_seed); the arrival clock is applied by the caller."""
    rng = np.random.Generator(np.random.PCG64(seed))
    reqs = []
    for _ in range(n_req):
        L = int(rng.choice(Ls))
        N = int(round(math.exp(rng.uniform(0.0, math.log(nmax)))))
        N = max(1, min(nmax, N))
        reqs.append((L, N, int(rng.integers(0, 2**31 - 1))))
    return reqs
