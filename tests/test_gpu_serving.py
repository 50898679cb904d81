"""Serving (continuous admission of many controllers): every request's result is the same
when its controller runs alone and when it runs in a concurrent mix whose HBM budget
forces evictions and re-admissions."""
import dataclasses

import numpy as np
import pytest

from paper_2410_09663_amd import oic
from paper_2410_09663_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _mix():
    base = wl.PRESETS["C1"]
    specs = [
        dataclasses.replace(base, name="a"),
        dataclasses.replace(base, name="b", seed_W=11, seed_X0=12),                  # same shape, other weights
        dataclasses.replace(wl.PRESETS["C2"], name="c", n=32, m=32, l=8, N=64, H=5, grf_length=4.0,
                            ref_center=(16.0, 8.0)),
        wl.small_preset(n=20, m=24, l=5, channels=(2, 16, 16, 1), N=24, H=4, name="d"),
        dataclasses.replace(wl.PRESETS["C3"], name="e", n=32, m=32, l=8, N=32, H=3, grf_length=4.0,
                            ref_center=(16.0, 8.0), precision=wl.PREC_BF16),
    ]
    return [wl.make_problem(p) for p in specs]


def _requests(problems, steps=3):
    reqs = []
    for k in range(steps):
        for cid, pr in enumerate(problems):
            p = pr.preset
            X0 = (pr.X0 * (1.0 + 0.1 * k)).astype(np.float32)
            reqs.append((cid, X0, wl.reference_window(p, k), 100 * cid + k))
    return reqs


def test_results_identical_alone_and_in_the_mix():
    problems = _mix()
    reqs = _requests(problems)
    alone = {}
    for cid, pr in enumerate(problems):
        with oic.Server(hbm_budget_bytes=8 << 30, max_inflight=1) as srv:
            sid = srv.add(pr, pr.preset.N, pr.preset.H)
            for (c, X0, ref, seed) in reqs:
                if c == cid:
                    alone[(c, seed)] = srv.wait(sid, srv.submit(sid, X0, ref, seed))[:2]
    # small budget: the largest controller only fits alone, so it and the others evict each
    # other back and forth -> evictions and re-admissions
    fps = [oic.Server.footprint(pr, pr.preset.N, pr.preset.H) for pr in problems]
    budget = int(1.05 * max(fps))
    with oic.Server(hbm_budget_bytes=budget, max_inflight=4) as srv:
        ids = [srv.add(pr, pr.preset.N, pr.preset.H) for pr in problems]
        lat = []
        # rounds of one request per controller: within a round the requests run concurrently
        # and the largest controller evicts the others; the next round re-admits them
        nprob = len(problems)
        for r0 in range(0, len(reqs), nprob):
            rnd = reqs[r0:r0 + nprob]
            tickets = [(c, seed, srv.submit(ids[c], X0, ref, seed)) for (c, X0, ref, seed) in rnd]
            for c, seed, t in tickets:
                U, X, ms, q = srv.wait(ids[c], t)
                lat.append(ms)
                Ua, Xa = alone[(c, seed)]
                assert np.array_equal(U, Ua), (c, seed)
                assert np.array_equal(X, Xa), (c, seed)
        st = srv.stats()
    print("serving stats", st, "p50 ms", np.percentile(lat, 50), flush=True)
    assert st["completed"] == len(reqs)
    assert st["evictions"] > 0 and st["admissions"] > len(problems)
    assert st["peak_bytes"] <= budget


def test_controller_larger_than_budget_is_rejected():
    pr = wl.make_problem(wl.PRESETS["C2"])
    with oic.Server(hbm_budget_bytes=1 << 20, max_inflight=1) as srv:
        with pytest.raises(oic.OicError) as e:
            srv.add(pr, pr.preset.N, pr.preset.H)
        assert e.value.code == oic.OIC_ENOMEM


def test_large_controller_is_not_starved_by_small_ones():
    """A controller that needs every other controller evicted is admitted after a bounded
    number of later requests have passed it (then nothing more starts ahead of it), even
    while two small controllers keep the budget busy with a continuous stream."""
    small = [wl.make_problem(dataclasses.replace(wl.PRESETS["C1"], name=f"s{k}", seed_W=20 + k)) for k in range(2)]
    big = wl.make_problem(dataclasses.replace(wl.PRESETS["C2"], name="big", n=48, m=48, l=8, N=96, H=6,
                                              grf_length=4.0, ref_center=(24.0, 12.0)))
    fs = oic.Server.footprint(small[0], small[0].preset.N, small[0].preset.H)
    fb = oic.Server.footprint(big, big.preset.N, big.preset.H)
    budget = fb + fs // 2  # the big controller fits only with both small ones evicted
    assert 2 * fs <= budget
    with oic.Server(hbm_budget_bytes=budget, max_inflight=2) as srv:
        sid = [srv.add(pr, pr.preset.N, pr.preset.H) for pr in small]
        bid = srv.add(big, big.preset.N, big.preset.H)
        sub = []
        for k in range(2):
            p = small[k].preset
            sub.append((sid[k], srv.submit(sid[k], small[k].X0, wl.reference_window(p, 0), k)))
        tb = srv.submit(bid, big.X0, wl.reference_window(big.preset, 0), 99)
        for r in range(40):
            k = r % 2
            p = small[k].preset
            sub.append((sid[k], srv.submit(sid[k], small[k].X0, wl.reference_window(p, r + 1), 100 + r)))
        lat_small = [srv.wait(c, t)[2] for c, t in sub]
        lat_big = srv.wait(bid, tb)[2]
    print(f"big controller latency {lat_big:.1f} ms; small requests: last {lat_small[-1]:.1f} ms", flush=True)
    assert lat_big < lat_small[-1]


@pytest.mark.parametrize("shape", ["c1_fp32", "bf16_32ch"])
def test_same_shape_admission_takes_over_the_handle(shape):
    """Two controllers of one shape with different weights, a budget for one handle and
    alternating requests: every admission after the first takes over the other
    controller's handle (weights and U_prev swapped in place, the captured solve kept).
    Each result is bitwise the controller's solve alone, so the taken-over solve reads the
    new weights, the evicted controller's U_prev comes back on its return, and a first
    admission starts from U_prev = 0."""
    if shape == "c1_fp32":
        base = wl.PRESETS["C1"]
    else:
        base = dataclasses.replace(wl.PRESETS["C3"], n=32, m=32, l=8, N=32, H=3, grf_length=4.0,
                                   ref_center=(16.0, 8.0), precision=wl.PREC_BF16)
    problems = [wl.make_problem(dataclasses.replace(base, name=f"{shape}{k}", seed_W=31 + k, seed_B=41 + k,
                                                    seed_X0=51 + k)) for k in range(2)]
    steps = 3
    reqs = []
    for k in range(steps):
        for cid, pr in enumerate(problems):
            p = pr.preset
            reqs.append((cid, (pr.X0 * (1.0 + 0.1 * k)).astype(np.float32), wl.reference_window(p, k),
                         200 * cid + k))
    alone = {}
    for cid, pr in enumerate(problems):
        with oic.Server(hbm_budget_bytes=8 << 30, max_inflight=1) as srv:
            sid = srv.add(pr, pr.preset.N, pr.preset.H)
            for (c, X0, ref, seed) in reqs:
                if c == cid:
                    alone[(c, seed)] = srv.wait(sid, srv.submit(sid, X0, ref, seed))[:2]
    fp = oic.Server.footprint(problems[0], base.N, base.H)
    with oic.Server(hbm_budget_bytes=int(1.5 * fp), max_inflight=1) as srv:
        ids = [srv.add(pr, pr.preset.N, pr.preset.H) for pr in problems]
        for (c, X0, ref, seed) in reqs:
            U, X, _, _ = srv.wait(ids[c], srv.submit(ids[c], X0, ref, seed))
            Ua, Xa = alone[(c, seed)]
            assert np.array_equal(U, Ua), (c, seed)
            assert np.array_equal(X, Xa), (c, seed)
        st = srv.stats()
    print(f"{shape}: {st}", flush=True)
    assert st["completed"] == len(reqs)
    assert st["admissions"] == len(reqs) and st["recycled"] == len(reqs) - 1
    assert st["peak_bytes"] == fp


def _alone(problems, reqs):
    """Each controller's results from a server that holds only it (one slot, its own
    solves), in the order its requests appear in reqs."""
    alone = {}
    for cid, pr in enumerate(problems):
        with oic.Server(hbm_budget_bytes=64 << 30, max_inflight=1) as srv:
            sid = srv.add(pr, pr.preset.N, pr.preset.H)
            for (c, X0, ref, seed) in reqs:
                if c == cid:
                    alone[(c, seed)] = srv.wait(sid, srv.submit(sid, X0, ref, seed))[:2]
    return alone


def test_same_shape_requests_run_as_grouped_batches():
    """Four BF16 controllers of one small shape, all requests submitted at once: the server
    puts them in one pack of four slots and solves queued requests of its controllers
    together (one launch per kernel for the batch).  Each result is bitwise the
    controller's solve alone."""
    base = wl.small_preset(n=32, m=32, l=8, channels=(2, 16, 16, 1), N=32, H=3)
    base = dataclasses.replace(base, precision=wl.PREC_BF16)
    problems = [wl.make_problem(dataclasses.replace(base, name=f"g{k}", seed_W=61 + k, seed_B=71 + k,
                                                    seed_X0=81 + k)) for k in range(4)]
    reqs = _requests(problems, steps=3)
    alone = _alone(problems, reqs)
    with oic.Server(hbm_budget_bytes=8 << 30, max_inflight=2, group_slots=4) as srv:
        ids = [srv.add(pr, pr.preset.N, pr.preset.H) for pr in problems]
        tickets = [(c, seed, srv.submit(ids[c], X0, ref, seed)) for (c, X0, ref, seed) in reqs]
        for c, seed, t in tickets:
            U, X, _, _ = srv.wait(ids[c], t)
            assert np.array_equal(U, alone[(c, seed)][0]), (c, seed)
            assert np.array_equal(X, alone[(c, seed)][1]), (c, seed)
        st = srv.stats()
    print("grouped serving stats", st, flush=True)
    assert st["completed"] == len(reqs)
    assert st["packs"] == 1 and st["grouped"] >= len(problems)
    assert st["batches"] < len(reqs)


def test_serving_mix_results_identical_alone_and_in_the_mix():
    """Sixteen controllers drawn from the serving mix at full size (grids 32..256, N 64..256,
    H 5..20, BF16; shapes that repeat share packs), two requests each, all submitted at
    once with four workers: each result is bitwise the controller's solve alone."""
    problems = [wl.make_problem(p) for p in wl.serving_mix(16, seed=10)]
    reqs = _requests(problems, steps=2)
    alone = _alone(problems, reqs)
    with oic.Server(hbm_budget_bytes=96 << 30, max_inflight=4) as srv:
        ids = [srv.add(pr, pr.preset.N, pr.preset.H) for pr in problems]
        tickets = [(c, seed, srv.submit(ids[c], X0, ref, seed)) for (c, X0, ref, seed) in reqs]
        for c, seed, t in tickets:
            U, X, _, _ = srv.wait(ids[c], t)
            assert np.array_equal(U, alone[(c, seed)][0]), (c, seed)
            assert np.array_equal(X, alone[(c, seed)][1]), (c, seed)
        st = srv.stats()
    print("serving mix stats", st, flush=True)
    assert st["completed"] == len(reqs) and st["grouped"] > 0
