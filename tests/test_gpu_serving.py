"""GPU tests of the uneven-stack path (mixed-geometry persistent launches),
the autotuner, and the continuous-batching server, through the C ABI."""
import json
import os
import time

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


def stack(L, N, seed):
    ref, imgs, _, _ = synth.make_stack(seed, L, N, K=6, shift_px=max(1.0, L / 16), jitter_px=1.0,
                                       snr=1.0)
    return ref, imgs


def oracle_for(oracle, ref, imgs, L):
    return oracle.align_images(ref, imgs, L, L, want_curve=True)


SIDES = [(64, 7), (96, 5), (128, 9), (192, 3), (256, 4), (64, 2)]


def raw(L, N, seed):
    """Unprocessed inputs: negative pixels, mass outside the disk, any scale."""
    return synth.make_raw_stack(seed, L, N)


@pytest.mark.parametrize("kind", ["clean", "raw"])
def test_align_stacks_parity(api, ctx, oracle, kind):
    make = raw if kind == "raw" else stack
    data = [make(L, N, 2000 + i) for i, (L, N) in enumerate(SIDES)]
    outs = api.align_stacks(ctx, [(dev(r), dev(x)) for r, x in data])
    for (L, N), (r, x), o in zip(SIDES, data, outs):
        g = api.unpack_results(o["res"])
        parity.check(g, oracle_for(oracle, r, x, L), L, parity.TAU_FP32,
                     oracle_for(oracle, r, x, L)["curve"])


def test_align_stacks_matches_single_geometry_path(api, ctx):
    data = [stack(L, N, 2100 + i) for i, (L, N) in enumerate(SIDES)]
    outs = api.align_stacks(ctx, [(dev(r), dev(x)) for r, x in data])
    for (L, N), (r, x), o in zip(SIDES, data, outs):
        rq, ra = api.tables(ctx, dev(r[None]), L, L)
        iq, ia = api.tables(ctx, dev(x), L, L)
        res, _ = api.align_batch(ctx, rq, ra, iq, ia, L)
        a, b = api.unpack_results(o["res"]), api.unpack_results(res)
        assert np.array_equal(a["rot_index"], b["rot_index"])
        assert np.allclose(a["sw2sq"], b["sw2sq"], rtol=1e-5, atol=1e-9)
        assert np.abs(o["qt"].cpu().numpy() - iq.cpu().numpy()).max() < 1e-6


def test_align_stacks_bf16(api, ctx, oracle):
    data = [stack(L, N, 2200 + i) for i, (L, N) in enumerate(SIDES[:3])]
    outs = api.align_stacks(ctx, [(dev(r), dev(x)) for r, x in data], prec=1)
    for (L, N), (r, x), o in zip(SIDES, data, outs):
        orc = oracle_for(oracle, r, x, L)
        parity.check(api.unpack_results(o["res"]), orc, L, parity.TAU_BF16, orc["curve"])


def test_autotune_table_roundtrip(api, ctx, tmp_path):
    path = str(tmp_path / "tiles.json")
    api.autotune(ctx, [64, 128], n_images=256, out_json=path)
    tiles = json.load(open(path))["tiles"]
    assert set(tiles) == {"64", "128"}
    for L, v in tiles.items():
        assert 1 <= v["R"] <= int(L) and v["ms"] > 0
        assert v.get("tpw", 5) in (5, 6, 9) and v.get("align_bpc", 8) in (2, 4, 6, 8)
    c2 = api.Context(0, tune_json=path)
    data = [stack(L, N, 2300 + i) for i, (L, N) in enumerate(SIDES[:3])]
    a = api.align_stacks(c2, [(dev(r), dev(x)) for r, x in data])
    b = api.align_stacks(ctx, [(dev(r), dev(x)) for r, x in data])
    for oa, ob in zip(a, b):
        # the strip height changes neither the summation order nor the result
        assert np.array_equal(oa["res"].cpu().numpy(), ob["res"].cpu().numpy())
    c2.close()


def strip_rows_max(L):
    """Largest strip height of the mixed launches' projection at side L: rows
    of (L + 5) | 1 sixteen-byte positions in 64 KiB, at most four staging
    passes of 512 threads over the ceil(L / 2) column pairs."""
    H = (L + 1) // 2
    return min(L, 65536 // (16 * ((L + 5) | 1)), 4 * (512 // H), 512 // -(-H // 4))


def test_tiles_never_change_results(api, ctx, tmp_path):
    """Every admissible strip height of the mixed launches gives bitwise the
    results and tables of the default (a row's line position depends on its
    image row only, never on where a strip starts), and so do both tasks-per-
    wave instances of the tables kernel (more or fewer task groups) and every
    alignment grid."""
    data = [stack(L, N, 2350 + i) for i, (L, N) in enumerate([(64, 5), (128, 6), (256, 3),
                                                             (96, 4)])]
    base = api.align_stacks(ctx, [(dev(r), dev(x)) for r, x in data])
    cases = [(L, R, 0, 0) for L in (64, 96, 128, 256) for R in range(1, strip_rows_max(L) + 1)]
    # the other knobs: tables tasks per wave and alignment blocks per CU
    # (the launch takes them from its L with the most projection work: 256)
    cases += [(256, 0, tpw, bpc) for tpw in (5, 6, 9) for bpc in (1, 2, 4, 6, 8)]
    for L, R, tpw, bpc in cases:
        path = tmp_path / f"t{L}_{R}_{tpw}_{bpc}.json"
        extra = (f', "tpw": {tpw}' if tpw else "") + (f', "align_bpc": {bpc}' if bpc else "")
        path.write_text('{"tiles": {"%d": {"R": %d%s}}}' % (L, R or strip_rows_max(L), extra))
        c = api.Context(0, tune_json=str(path))
        got = api.align_stacks(c, [(dev(r), dev(x)) for r, x in data])
        c.close()
        for a, b in zip(got, base):
            assert np.array_equal(a["qt"].cpu().numpy(), b["qt"].cpu().numpy()), (L, R, tpw, bpc)
            assert np.array_equal(a["res"].cpu().numpy(), b["res"].cpu().numpy()), (L, R, tpw, bpc)


# ---------------------------------------------------------------- serving
def wait_all(srv, tickets, timeout=60.0):
    out, t0 = {}, time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        assert time.time() - t0 < timeout, "serving timed out"
        time.sleep(0.001)
    return out


@pytest.mark.parametrize("prec,kind", [(0, "clean"), (1, "clean"), (0, "raw")])
def test_serving_alone_equals_mix(api, oracle, prec, kind):
    c = api.Context(0)
    srv = api.Server(c, hbm_budget_bytes=1 << 30, prec=prec)
    make = raw if kind == "raw" else stack
    A = make(128, 12, 2400)
    alone = wait_all(srv, [srv.submit(*A)])
    ra = list(alone.values())[0]
    mix = [make(64, 30, 2401), A, make(256, 5, 2402), make(128, 20, 2403), A]
    ts = [srv.submit(r, x) for r, x in mix]
    got = wait_all(srv, ts)
    for k in (1, 4):  # A in the mix, twice
        assert np.array_equal(got[ts[k]], ra)
    tau = parity.TAU_FP32 if prec == 0 else parity.TAU_BF16
    for t, (r, x) in zip(ts, mix):
        L = x.shape[-1]
        orc = oracle_for(oracle, r, x, L)
        parity.check(api.records_to_dict(got[t]), orc, L, tau, orc["curve"])
    st = srv.stats()
    assert st["completed"] == 6 and st["failed"] == 0
    srv.stop()
    c.close()


def test_serving_admission_by_budget_and_backpressure(api):
    c = api.Context(0)
    L, N = 128, 40
    per_req = N * L * L * 4 * 2 + 4 * L * L * 3  # images + tables + small parts, roughly
    budget = int(per_req * 2.5)
    srv = api.Server(c, hbm_budget_bytes=budget, prec=0, max_queue=3)
    reqs = [stack(L, N, 2500 + i) for i in range(6)]
    ts, busy = [], 0
    for i in range(12):
        try:
            ts.append(srv.submit(*reqs[i % 6]))
        except Exception as e:  # back-pressure: queue full
            assert "BUSY" in str(e)
            busy += 1
    assert busy >= 1 and len(ts) >= 3
    big = np.zeros((4000, L, L), np.float32)
    with pytest.raises(Exception) as ei:  # alone larger than the budget
        srv.submit(reqs[0][0], big)
    assert "NOMEM" in str(ei.value)
    got = wait_all(srv, ts)
    st = srv.stats()
    assert st["arena_peak"] <= budget
    assert st["completed"] == len(ts)
    # the same requests alone give the same results
    for t, (r, x) in zip(ts, reqs[:2]):
        one = wait_all(srv, [srv.submit(r, x)])
        assert np.array_equal(list(one.values())[0], got[t])
    srv.stop()
    c.close()


def test_serving_steps_in_flight_match_one_step(api):
    """max_per_step below max_slots: several steps in flight at once (the
    next step's copies beside the current step's kernels), each request's
    results the same as with every request in one step."""
    reqs = [stack(128, 5 + 3 * i, 2700 + i) for i in range(7)] + [stack(64, 11, 2710)]
    res = {}
    for per_step in (0, 2):
        c = api.Context(0)
        srv = api.Server(c, hbm_budget_bytes=1 << 29, prec=1, max_slots=8, max_per_step=per_step)
        ts = [srv.submit(r, x) for r, x in reqs]
        got = wait_all(srv, ts)
        res[per_step] = [got[t] for t in ts]
        st = srv.stats()
        assert st["completed"] == len(reqs)
        if per_step:
            assert st["steps"] >= 4  # at most two requests of one L per step
        srv.stop()
        c.close()
    for a, b in zip(res[0], res[2]):
        assert np.array_equal(a, b)


def test_serving_graph_replays_match_plain_launches(api):
    reqs = [stack(64, 9, 2600 + i) for i in range(4)] + [stack(96, 6, 2610)]
    res = {}
    for use_graphs in (0, 1):
        c = api.Context(0)
        srv = api.Server(c, hbm_budget_bytes=1 << 29, prec=1, use_graphs=use_graphs)
        outs = []
        for rep in range(3):  # several replays with host work in between
            ts = [srv.submit(r, x) for r, x in reqs]
            got = wait_all(srv, ts)
            outs.append([got[t] for t in ts])
            time.sleep(0.01)
        st = srv.stats()
        if use_graphs:
            assert st["graph_launches"] >= 3
        srv.stop()
        c.close()
        for o in outs[1:]:
            for a, b in zip(o, outs[0]):
                assert np.array_equal(a, b)
        res[use_graphs] = outs[0]
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)


def test_serving_reference_cache_and_cancel(api):
    c = api.Context(0)
    srv = api.Server(c, hbm_budget_bytes=1 << 29, prec=0)
    r, x = stack(64, 16, 2700)
    plain = wait_all(srv, [srv.submit(r, x)])
    t1 = srv.submit(r, x, ref_key=77)
    got1 = wait_all(srv, [t1])
    t2 = srv.submit(r, x[:5], ref_key=77)
    got2 = wait_all(srv, [t2])
    assert srv.stats()["cache_hits"] >= 1
    p = list(plain.values())[0]
    assert np.array_equal(got1[t1], p) and np.array_equal(got2[t2], p[:5])
    # a new key twice in a row (normally one step): the first request computes
    # the reference tables and its spectrum, the second reads the same tables
    t3 = srv.submit(r, x, ref_key=78)
    t4 = srv.submit(r, x[:7], ref_key=78)
    got34 = wait_all(srv, [t3, t4])
    assert np.array_equal(got34[t3], p) and np.array_equal(got34[t4], p[:7])
    # cancel: pending or in flight, the ticket is gone afterwards
    ts = [srv.submit(*stack(128, 50, 2710 + i)) for i in range(4)]
    srv.cancel(ts[3])
    with pytest.raises(Exception):
        srv.poll(ts[3])
    wait_all(srv, ts[:3])
    srv.stop()
    c.close()


def test_serving_cache_producer_failure_recomputes(api, oracle, tmp_path):
    """The request that would compute a cached reference table fails on the
    host (an injected copy failure, no device fault): a request with the same
    key queued behind it computes the tables itself, and later requests of
    that key hit the cache; all results match the oracle and the uncached
    path."""
    from paper_2503_13756_amd._abi import SwError

    path = tmp_path / "fail.json"
    path.write_text('{"serve_fail_ticket": 2}')
    c = api.Context(0, tune_json=str(path))
    srv = api.Server(c, hbm_budget_bytes=1 << 29, prec=0)
    r, x = stack(64, 16, 2800)
    plain = list(wait_all(srv, [srv.submit(r, x)]).values())[0]  # ticket 1
    t2 = srv.submit(r, x, ref_key=91)      # ticket 2: its copy "fails"
    t3 = srv.submit(r, x[:6], ref_key=91)  # queued behind it, same key
    got3 = wait_all(srv, [t3])
    with pytest.raises(SwError, match="injected"):
        for _ in range(20000):
            if srv.poll(t2) is not None:
                break
            time.sleep(0.001)
    assert np.array_equal(got3[t3], plain[:6])
    t4 = srv.submit(r, x, ref_key=91)
    got4 = wait_all(srv, [t4])
    assert np.array_equal(got4[t4], plain)
    st = srv.stats()
    assert st["failed"] == 1 and st["cache_hits"] >= 2
    orc = oracle_for(oracle, r, x, 64)
    parity.check(api.records_to_dict(got4[t4]), orc, 64, parity.TAU_FP32, orc["curve"])
    srv.stop()
    c.close()


def test_serving_rejects_mismatched_shapes(api):
    c = api.Context(0)
    srv = api.Server(c, hbm_budget_bytes=1 << 26, prec=0)
    r, x = stack(64, 3, 2900)
    with pytest.raises(ValueError):
        srv.submit(r[:32, :32], x)
    with pytest.raises(ValueError):
        srv.submit(r, x[:, :, :32])
    srv.stop()
    c.close()
