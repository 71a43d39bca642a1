"""The projection work plan (host logic, no GPU): every (slot, bin) item of
the line projection (Sec. 2.2/2.3) once, in units of 8 consecutive bins of
one slot, and every task's row range covering the rows where its items'
lines have a pixel of non-zero hat weight inside the disk.  The ranges are
recomputed here in FP64 from the geometry (bin centres, the hat of
half-width h / cos theta, the disk of radius 1 - h), independently of the
planner.  Rows outside a task's range are skipped by the kernels, so a range
that missed such a row would drop a non-zero contribution."""
import math

import numpy as np
import pytest

from paper_2503_13756_amd import api


def slot_angles(n):
    # slots m = 0 .. n/8: theta_m = 2 pi m / n, the angles of [0, pi/4]
    return [2.0 * math.pi * m / n for m in range(n // 8 + 1)]


def item_rows(L, n, m, b):
    """Rows i where the line of bin b at slot angle theta_m crosses a pixel
    (i, j) inside the disk with non-zero hat weight: column position of the
    line u(i) = (b - c + sin(theta) (i - c)) / cos(theta) + c (c = (L-1)/2),
    weight 1 - cos(theta) |j - u(i)| > 0."""
    th = slot_angles(n)[m]
    cth, sth = math.cos(th), math.sin(th)
    c = 0.5 * (L - 1)
    r2 = (L - 2) ** 2
    rows = []
    for i in range(L):
        u = (b - c + sth * (i - c)) / cth + c
        lo, hi = math.floor(u - 1.0 / cth), math.ceil(u + 1.0 / cth)
        for j in range(max(0, lo), min(L - 1, hi) + 1):
            if (2 * j - L + 1) ** 2 + (2 * i - L + 1) ** 2 <= r2 and cth * abs(j - u) < 1.0 - 1e-9:
                rows.append(i)
                break
    return rows


@pytest.mark.parametrize("L,n", [(16, 16), (39, 48), (40, 24), (64, 64), (64, 128)])
def test_plan_covers_every_item_and_row(L, n):
    perm, rows = api.projection_plan(L, n)
    slots = n // 8 + 1
    items = perm[perm >= 0]
    # every item exactly once
    assert np.array_equal(np.sort(items), np.arange(slots * L))
    # units: 8 lanes of consecutive bins of one slot (the last unit of a slot padded)
    for t in range(perm.shape[0]):
        for u in range(8):
            lanes = perm[t, 8 * u:8 * u + 8]
            live = lanes[lanes >= 0]
            if len(live) == 0:
                continue
            assert len(set(live // L)) == 1, (t, u, lanes)
            assert np.array_equal(live, np.arange(live[0], live[0] + len(live))), (t, u, lanes)
            assert live[0] % L % 8 == 0 and np.all(lanes[:len(live)] >= 0), (t, u, lanes)
    # every row with a non-zero weight inside the disk lies in its task's range
    for t in range(perm.shape[0]):
        lo, hi = rows[t]
        for it in perm[t][perm[t] >= 0]:
            r = item_rows(L, n, it // L, it % L)
            if r:
                assert lo <= min(r) and max(r) <= hi, (t, it, lo, hi, min(r), max(r))


def test_plan_is_deterministic_and_no_longer_than_the_centre_order():
    """Same plan on every call; the local search over unit swaps never ends
    with more task rows than the plain order by range centre."""
    L = n = 64
    p1, r1 = api.projection_plan(L, n)
    p2, r2 = api.projection_plan(L, n)
    assert np.array_equal(p1, p2) and np.array_equal(r1, r2)
    # the centre order, rebuilt from the independent row ranges
    units = []
    for m in range(n // 8 + 1):
        for b0 in range(0, L, 8):
            r = [x for b in range(b0, min(L, b0 + 8)) for x in item_rows(L, n, m, b)]
            units.append((min(r), max(r)) if r else None)
    key = [(u[0] + u[1]) if u else -1 for u in units]
    order = sorted(range(len(units)), key=lambda k: key[k])
    base = 0
    for t in range(0, len(order), 8):
        us = [units[k] for k in order[t:t + 8] if units[k]]
        if us:
            base += max(u[1] for u in us) - min(u[0] for u in us) + 1
    plan = int(sum(hi - lo + 1 for lo, hi in r2 if hi >= lo))
    assert plan <= base, (plan, base)


def test_plan_rejects_bad_geometry():
    with pytest.raises(Exception):
        api.projection_plan(4, 64)
    with pytest.raises(Exception):
        api.projection_plan(64, 60)
