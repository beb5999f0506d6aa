"""Serving: continuous batching of mixed zero- and finite-temperature
requests.  Each result equals the same request solved alone (bitwise: every
solve is deterministic and independent of what else runs); the budget is
enforced at submission and at admission."""
import threading
import time

import numpy as np
import pytest

import workloads
from gpu_util import dev, host, reference, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fdm():
    import paper_2301_04642_amd as m
    return m


def requests(count=10):
    reqs = workloads.serving_requests(count, n_lo=100, n_hi=700, rate=50.0)
    return [(r, workloads.serving_workload(r)) for r in reqs]


@pytest.mark.parametrize("grouped", [True, False])
def test_alone_equals_mix(fdm, grouped):
    reqs = requests(10)
    prec = "fp32"
    alone = {}
    for r, wl in reqs:
        say("alone", r["id"], wl.n)
        D, e, st = fdm.solve(dev(wl.hp), wl.n_occ, wl.kT, 1e-8, prec)
        alone[r["id"]] = (host(D), e)
    srv = fdm.Server(budget_bytes=8 << 30, max_active=4, precision=prec, grouped=grouped)
    shared = 0
    try:
        tickets = {}
        t0 = time.time()
        for r, wl in reqs:
            while time.time() - t0 < r["arrival"]:
                time.sleep(0.001)
            tickets[r["id"]] = srv.submit(wl.hp, wl.n_occ, wl.kT, 1e-8)
        starts, finishes = [], []
        for r, wl in reqs:
            say("mix result", r["id"])
            rc, d, e, st, times = srv.result(tickets[r["id"]], wl.n)
            assert rc == 0
            assert np.array_equal(d, alone[r["id"]][0]), r["id"]
            assert e == alone[r["id"]][1]
            d_ref, e_ref, _, _ = reference(wl)
            print(f"[report] request {r['id']} n={wl.n} kT={wl.kT} |dE|={abs(e - e_ref):.2e} "
                  f"queue={times[1] - times[0]:.3f}s run={times[2] - times[1]:.3f}s", flush=True)
            assert abs(e - e_ref) <= 1e-6
            starts.append(times[1])
            finishes.append(times[2])
            shared += st.tick_shared
            if grouped:
                assert st.tick_steps > 0
            else:
                assert st.tick_steps == 0
        # work overlapped: some request started before another had finished
        order = np.argsort(starts)
        overlapped = any(starts[order[i + 1]] < finishes[order[i]] for i in range(len(order) - 1))
        assert overlapped
        if grouped:
            # on the device: steps of different requests ran in the same
            # grouped product and decision launches
            print(f"[report] grouped ticks: {shared} shared steps", flush=True)
            assert shared > 0
    finally:
        srv.close()


def test_alone_equals_mix_wide(fdm):
    """A mix up to N ~ 4000 (log-uniform 500 ... 4000), half finite
    temperature, precisions FP32 / FP16x3 / BF16x3 per request: each served
    result is bitwise the solve alone."""
    reqs = [(r, workloads.serving_workload(r))
            for r in workloads.serving_requests(8, n_lo=500, n_hi=4000, rate=100.0, seed=77)]
    precs = ["fp32", "fp16x3", "bf16x3"]
    alone = {}
    for k, (r, wl) in enumerate(reqs):
        say("alone wide", r["id"], wl.n, wl.kT, precs[k % 3])
        D, e, st = fdm.solve(dev(wl.hp), wl.n_occ, wl.kT, 1e-8, precs[k % 3])
        alone[r["id"]] = (host(D), e)
    srv = fdm.Server(budget_bytes=40 << 30, max_active=4, precision="fp32")
    try:
        tickets = {r["id"]: srv.submit(wl.hp, wl.n_occ, wl.kT, 1e-8, precision=precs[k % 3])
                   for k, (r, wl) in enumerate(reqs)}
        shared = 0
        for r, wl in reqs:
            say("mix wide result", r["id"])
            rc, d, e, st, times = srv.result(tickets[r["id"]], wl.n)
            assert rc == 0
            assert np.array_equal(d, alone[r["id"]][0]), r["id"]
            assert e == alone[r["id"]][1]
            shared += st.tick_shared
        print(f"[report] wide mix: {shared} shared steps", flush=True)
        assert shared > 0
    finally:
        srv.close()


def test_edge_blocks_in_grouped_ticks(fdm):
    """FP16x3 requests whose 128-wide products run with edge blocks (N = 4000
    and 3500) and without (N = 3400) share grouped product launches (finite
    temperature, 500 K): each served result is bitwise the solve alone."""
    # finite temperature: long enough (several mu evaluations) to overlap
    wls = [workloads.standard_workload("uniform", n=n, seed_base=300 + n) for n in (4000, 3400, 3500)]
    alone = []
    for wl in wls:
        say("edge alone", wl.n)
        D, e, st = fdm.solve(dev(wl.hp), wl.n_occ, wl.kT, 1e-8, "fp16x3")
        assert st.status == 0
        d_ref, e_ref, _, _ = reference(wl)
        print(f"[report] edge alone n={wl.n}: |dE|={abs(e - e_ref):.2e} evals={st.mu_evals}",
              flush=True)
        assert abs(e - e_ref) <= 1e-6
        alone.append((host(D), e))
    srv = fdm.Server(budget_bytes=40 << 30, max_active=3, precision="fp16x3")
    try:
        ts = [srv.submit(wl.hp, wl.n_occ, wl.kT, 1e-8) for wl in wls]
        shared = 0
        for t, wl, (d0, e0) in zip(ts, wls, alone):
            say("edge mix result", wl.n)
            rc, d, e, st, times = srv.result(t, wl.n)
            assert rc == 0
            assert np.array_equal(d, d0) and e == e0, wl.n
            shared += st.tick_shared
        print(f"[report] edge-block mix: {shared} shared steps", flush=True)
        assert shared > 0
    finally:
        srv.close()


def test_held_memory_within_budget(fdm):
    """Device blocks held by the server (in use or pooled) never exceed the
    budget over a log-uniform mix of sizes."""
    reqs = [(r, workloads.serving_workload(r))
            for r in workloads.serving_requests(12, n_lo=200, n_hi=2500, rate=100.0, seed=78)]
    budget = 1 << 30
    srv = fdm.Server(budget_bytes=budget, max_active=4, precision="fp32")
    try:
        tickets = [(srv.submit(wl.hp, wl.n_occ, wl.kT, 1e-8), wl) for r, wl in reqs]
        peak = 0
        for t, wl in tickets:
            say("budget mix", wl.n)
            rc, d, e, st, times = srv.result(t, wl.n)
            assert rc == 0
            held, reserved, pooled = srv.memory()
            peak = max(peak, held)
            assert held <= budget and reserved <= budget
        print(f"[report] budget {budget >> 20} MiB: peak held {peak >> 20} MiB", flush=True)
    finally:
        srv.close()


def test_destroy_with_uncollected_results(fdm):
    """Closing a server whose budget fits one request at a time, with results
    nobody collected and requests that never started, returns."""
    n = 300
    foot = fdm.fdm_workspace_bytes(n, 0.0, fdm.FDM_FP32) + 2 * n * n * 8
    srv = fdm.Server(budget_bytes=foot + foot // 2, max_active=2, precision="fp32")
    wls = [workloads.standard_workload("gapped", n=n, seed_base=90 + i) for i in range(4)]
    ts = [srv.submit(w.hp, w.n_occ, 0.0, 1e-8) for w in wls]
    say("destroy: wait for the first result")
    while srv.poll(ts[0]) == 1:
        time.sleep(0.001)
    t0 = time.time()
    srv.close()
    assert time.time() - t0 < 30.0


def test_budget_enforced(fdm):
    n = 300
    foot = fdm.fdm_workspace_bytes(n, 0.0, fdm.FDM_FP32) + 2 * n * n * 8
    srv = fdm.Server(budget_bytes=foot + foot // 2, max_active=4, precision="fp32")
    try:
        big = workloads.standard_workload("gapped", n=600)
        with pytest.raises(fdm.FdmError) as ei:
            srv.submit(big.hp, big.n_occ, 0.0, 1e-8)
        assert ei.value.code == fdm.FDM_ENOMEM
        wls = [workloads.standard_workload("gapped", n=n, seed_base=77 + i) for i in range(4)]
        say("budget: serial admission")
        ts = [srv.submit(w.hp, w.n_occ, 0.0, 1e-8) for w in wls]
        spans = []
        for t, w in zip(ts, wls):
            rc, d, e, st, times = srv.result(t, n)
            assert rc == 0
            spans.append((times[1], times[2]))
        # only one footprint fits: executions never overlap
        spans.sort()
        for (s0, f0), (s1, f1) in zip(spans, spans[1:]):
            assert s1 >= f0
    finally:
        srv.close()


def test_result_collected_once(fdm):
    """Two threads collect the same ticket at once: one gets the result, the
    other FDM_EINVAL, and so does a later call."""
    wl = workloads.standard_workload("gapped", n=400)
    srv = fdm.Server(budget_bytes=1 << 30, max_active=2, precision="fp32")
    try:
        say("collect once")
        t = srv.submit(wl.hp, wl.n_occ, 0.0, 1e-8)
        out = []
        ths = [threading.Thread(target=lambda: out.append(srv.result(t, wl.n)[0]))
               for _ in range(2)]
        for th in ths:
            th.start()
        for th in ths:
            th.join(timeout=120)
        assert sorted(out) == [fdm.FDM_EINVAL, 0]
        assert srv.result(t, wl.n)[0] == fdm.FDM_EINVAL
    finally:
        srv.close()


def test_device_input_and_poll(fdm):
    wl = workloads.standard_workload("gapped", n=200)
    srv = fdm.Server(budget_bytes=1 << 30, max_active=2, precision="fp64")
    try:
        say("device input")
        t = srv.submit(dev(wl.hp), wl.n_occ, 0.0, 1e-10, precision="fp64")
        while srv.poll(t) == 1:
            time.sleep(0.001)
        rc, d, e, st, times = srv.result(t, wl.n)
        d_ref, e_ref, _, _ = reference(wl)
        assert rc == 0 and np.linalg.norm(d - d_ref) < 1e-10
        assert srv.poll(t) < 0
    finally:
        srv.close()
