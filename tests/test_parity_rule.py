"""The parity rule itself (tests/parity.py) on planted mistakes, CPU only:
a rule that let these through would hide real GPU errors."""
import numpy as np
import pytest

from tests import parity


def _orc():
    # two pairs on n = 8 lags; the second has a near tie between lags 2 and 3
    curve = np.array([[0.5, 0.4, 0.3, 0.2, 0.1, 0.2, 0.3, 0.4],
                      [0.5, 0.4, 0.100000001, 0.1, 0.2, 0.3, 0.4, 0.45]])
    sc = np.zeros((2, 8, 2))
    sc[0, 4] = (1.2, -2.7)
    sc[1, 3] = (0.2, 3.4)
    sc[1, 2] = (1.1, -0.6)
    return {"rot_index": np.array([4, 3]), "shift_px": np.array([[1.2, -2.7], [0.2, 3.4]]),
            "sw2sq": np.array([0.1, 0.1]), "status": np.array([0, 0]), "curve": curve,
            "shift_curve": sc}


def _gpu(**kw):
    g = {"rot_index": np.array([4, 3]), "shift_px": np.array([[1.2, -2.7], [0.2, 3.4]]),
         "sw2sq": np.array([0.1, 0.1]), "status": np.array([0, 0])}
    g.update(kw)
    return g


def test_accepts_exact_and_near_tie():
    o = _orc()
    rep = parity.check(_gpu(), o, 64, 1e-4, o["curve"])
    assert rep["exact_rot"] == 2 and rep["near_ties"] == 0
    g = _gpu(rot_index=np.array([4, 2]), shift_px=np.array([[1.2, -2.7], [1.1, -0.6]]),
             sw2sq=np.array([0.1, 0.100000001]))
    rep = parity.check(g, o, 64, 1e-4, o["curve"])
    assert rep["near_ties"] == 1


@pytest.mark.parametrize("what", ["rot", "shift", "shift_at_tie", "dist", "status"])
def test_rejects_planted_mistakes(what):
    o = _orc()
    g = _gpu()
    if what == "rot":
        g["rot_index"] = np.array([5, 3])
    elif what == "shift":
        g["shift_px"] = np.array([[0.2, -2.7], [0.2, 3.4]])
    elif what == "shift_at_tie":  # lag 2 accepted, but with lag 3's shift
        g["rot_index"] = np.array([4, 2])
        g["sw2sq"] = np.array([0.1, 0.100000001])
    elif what == "dist":
        g["sw2sq"] = np.array([0.1, 0.10002])
    else:
        g["status"] = np.array([0, 1])
    with pytest.raises(AssertionError):
        parity.check(g, o, 64, 1e-4, o["curve"])


def test_floor_admitted_is_counted():
    o = _orc()
    o["sw2sq"] = np.array([0.0, 0.1])
    o["curve"] = o["curve"].copy()
    o["curve"][0, 4] = 0.0
    g = _gpu(sw2sq=np.array([1e-10, 0.1]))  # below tau h^2 / 2 = 4.9e-8
    rep = parity.check(g, o, 64, 1e-4, o["curve"])
    assert rep["floor_admitted"] == 1
