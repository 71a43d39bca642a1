"""Parity rule between GPU results and the FP64 oracle.

Rotation: accept the GPU lag when it equals the oracle's, or when the
oracle's own objective at the GPU lag is within the distance tolerance of its
minimum (near-ties: the true angle falls between grid points, and FP32 may
legitimately pick the neighbour).
Translation: the rounded pixel shift must agree, unless the oracle's shift
is within 1e-3 of a rounding boundary.
Distance: |d_gpu - d_or| <= tau d_or + tau h^2 / 2 with tau = 1e-4 (FP32) or
1e-3 (BF16 correlation), the floor being tau times SW2^2 of a one-pixel
shift (Thm 3.2: |s|^2 / 2)."""
import numpy as np

TAU_FP32 = 1e-4
TAU_BF16 = 1e-3
# Ramp-filtered distance, both precision forms: a signed part's CDF has
# near-flat stretches between its lobes, where its inverse jumps, so the
# distance reacts about 1e3 times more than SW2 to the same FP32-level change
# of the projections (tests/test_oracle_pins.py,
# test_ramp_distance_sensitivity); FP32 projections then give ~1e-4 relative
# differences, and the tolerance is that of the BF16 form.
TAU_RF = 3e-4


def dist_tol(d_or, L, tau):
    h = 2.0 / L
    return tau * np.abs(d_or) + tau * h * h / 2


def _shift_ok(sg, so):
    """Rounded pixel shifts agree, except on an axis where the oracle's shift
    is within 1e-3 of a rounding boundary."""
    for a in range(2):
        fr = so[a] - np.floor(so[a])
        if abs(fr - 0.5) < 1e-3:
            continue
        if np.round(sg[a]) != np.round(so[a]):
            return False
    return True


def check(gpu, orc, L, tau=TAU_FP32, curve_or=None):
    """Compare result dicts (numpy) element by element.  Returns a report dict
    (pairs, exact rotations, near-tie rotations, pairs admitted only by the
    distance floor, the largest distance error in units of the tolerance);
    raises AssertionError with the first failures listed.  On a near tie the
    GPU's shift is compared with the oracle's closed-form shift at the GPU's
    lag (orc["shift_curve"], when the oracle returned it)."""
    lg, lo = gpu["rot_index"], orc["rot_index"]
    sg, so = gpu["shift_px"], orc["shift_px"]
    dg, do = gpu["sw2sq"], orc["sw2sq"]
    scurve = orc.get("shift_curve")
    P = len(lo)
    bad = []
    exact = ties = floor_only = 0
    worst = 0.0
    for p in range(P):
        if gpu["status"][p] != orc["status"][p]:
            bad.append((p, "status", gpu["status"][p], orc["status"][p]))
            continue
        if orc["status"][p] != 0:
            continue
        if lg[p] == lo[p]:
            exact += 1
            d_ref = do[p]
            if not _shift_ok(sg[p], so[p]):
                bad.append((p, "shift", tuple(sg[p]), tuple(so[p])))
        else:
            if curve_or is None:
                bad.append((p, "rot (no curve to check a tie)", int(lg[p]), int(lo[p])))
                continue
            ties += 1
            c = curve_or[p]
            if c[lg[p]] > c[lo[p]] + dist_tol(c[lo[p]], L, tau):
                bad.append((p, "rot", int(lg[p]), int(lo[p]), float(c[lg[p]]), float(c[lo[p]])))
                continue
            d_ref = c[lg[p]]
            if scurve is not None and not _shift_ok(sg[p], scurve[p, lg[p]]):
                bad.append((p, "shift@tie", tuple(sg[p]), tuple(scurve[p, lg[p]])))
        err = abs(dg[p] - d_ref)
        tol = dist_tol(d_ref, L, tau)
        worst = max(worst, err / tol)
        if err > tol:
            bad.append((p, "sw2sq" if lg[p] == lo[p] else "sw2sq@tie", float(dg[p]), float(d_ref)))
        elif err > tau * abs(d_ref):
            floor_only += 1
    rep = {"pairs": P, "exact_rot": exact, "near_ties": ties, "floor_admitted": floor_only,
           "worst_err_over_tol": worst, "failures": len(bad)}
    assert not bad, f"{len(bad)} parity failures of {P}: {bad[:8]}"
    return rep
