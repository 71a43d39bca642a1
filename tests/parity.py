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
TAU_RF = 1e-3


def dist_tol(d_or, L, tau):
    h = 2.0 / L
    return tau * np.abs(d_or) + tau * h * h / 2


def check(gpu, orc, L, tau=TAU_FP32, curve_or=None):
    """Compare result dicts (numpy) element by element.  Returns a report dict;
    raises AssertionError with the first failures listed."""
    lg, lo = gpu["rot_index"], orc["rot_index"]
    sg, so = gpu["shift_px"], orc["shift_px"]
    dg, do = gpu["sw2sq"], orc["sw2sq"]
    P = len(lo)
    bad = []
    exact = 0
    for p in range(P):
        if gpu["status"][p] != orc["status"][p]:
            bad.append((p, "status", gpu["status"][p], orc["status"][p]))
            continue
        if orc["status"][p] != 0:
            continue
        if lg[p] == lo[p]:
            exact += 1
            if abs(dg[p] - do[p]) > dist_tol(do[p], L, tau):
                bad.append((p, "sw2sq", float(dg[p]), float(do[p])))
            for a in range(2):
                fr = so[p, a] - np.floor(so[p, a])
                if abs(fr - 0.5) < 1e-3:
                    continue
                if np.round(sg[p, a]) != np.round(so[p, a]):
                    bad.append((p, "shift", tuple(sg[p]), tuple(so[p])))
                    break
        else:
            if curve_or is None:
                bad.append((p, "rot (no curve to check a tie)", int(lg[p]), int(lo[p])))
                continue
            c = curve_or[p]
            if c[lg[p]] > c[lo[p]] + dist_tol(c[lo[p]], L, tau):
                bad.append((p, "rot", int(lg[p]), int(lo[p]), float(c[lg[p]]), float(c[lo[p]])))
            elif abs(dg[p] - c[lg[p]]) > dist_tol(c[lg[p]], L, tau):
                bad.append((p, "sw2sq@tie", float(dg[p]), float(c[lg[p]])))
    rep = {"pairs": P, "exact_rot": exact, "failures": len(bad)}
    assert not bad, f"{len(bad)} parity failures of {P}: {bad[:8]}"
    return rep
