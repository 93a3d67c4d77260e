"""GPU tests of the serving loop (continuous batching with HBM admission).

A request's result must be the same alone and in the mix: every partial sum
of a request is produced by one tile with the same kernel and node chunking
as a single sc_evaluate, so the comparison is bitwise.
"""
import math
import os
import subprocess
import sys
import threading
import time

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1609_08146_amd import Context
    c = Context(0)
    yield c
    c.close()


def small_requests(n, seed=3):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        w = workloads.sweep_instance(rng, i)
        nn = int(rng.integers(40, 120))
        w = w.with_nodes(nn, int(rng.integers(24, 80)))
        w = w.subset(obs_idx=np.arange(0, w.n_obs, int(rng.integers(3, 40))), k_idx=np.arange(min(w.n_k, 3)))
        out.append(w)
    return out


def alone(ctx, w, prec, t=None, dk=1.0):
    from paper_1609_08146_amd import problem_from_workload
    p = problem_from_workload(ctx, w)
    E, B = p.evaluate(prec)
    Et = Bt = None
    if t is not None:
        Et, Bt = p.to_time_at(dk, t)
    p.close()
    return E, B, Et, Bt


def test_same_result_alone_and_in_the_mix(ctx):
    from dataclasses import replace
    from paper_1609_08146_amd import Server
    ws = small_requests(8)
    # two curl-consistent beams: their tables do not factor, so quanta mix factored and general jobs
    ws[2] = replace(ws[2], consistent=1)
    ws[5] = replace(ws[5], consistent=1)
    precs = ["fp32_split"] * 6 + ["fp64", "fp32_split"]
    ref = [alone(ctx, w, pr, w.t[::32], w.dk) for w, pr in zip(ws, precs)]
    # at most three running at once, so later arrivals queue and join running work
    srv = Server(ctx, hbm_budget=int(3e9), max_running=3, quantum_ms=1.0)
    tickets = []
    for i, (w, pr) in enumerate(zip(ws, precs)):
        tickets.append(srv.submit(w, pr, t=w.t[::32], dk=w.dk))
        if i == 3:
            time.sleep(0.01)   # later arrivals join running work
    for tk, (E0, B0, Et0, Bt0) in zip(tickets, ref):
        E, B, Et, Bt, st = srv.wait(tk)
        assert np.array_equal(E, E0) and np.array_equal(B, B0)
        assert np.array_equal(Et, Et0) and np.array_equal(Bt, Bt0)
        assert st["total_ms"] >= st["run_ms"] >= 0 and st["evals"] > 0
    s = srv.stats()
    assert s["completed"] == len(ws) and s["rejected"] == 0
    assert s["hbm_in_use"] == 0
    assert s["launches"] >= 1
    srv.close()


def test_admission_respects_hbm_budget(ctx):
    from paper_1609_08146_amd import Server
    ws = small_requests(6, seed=11)
    # budget fits only one of these requests at a time
    from paper_1609_08146_amd import problem_from_workload
    p = problem_from_workload(ctx, ws[0])
    p.evaluate("fp32_split")
    one = p.device_bytes()
    p.close()
    biggest = max(w.n_k * (w.n_r + 1) * w.n_phi for w in ws)
    budget = int(max(one, 120 * biggest + 64 * max(w.n_obs for w in ws) * 200) * 1.6)
    srv = Server(ctx, hbm_budget=budget, max_running=8, quantum_ms=0.5)
    seen = []
    stop = threading.Event()

    def sample():
        while not stop.is_set():
            st = srv.stats()
            seen.append((st["hbm_in_use"], st["queued"], st["running"]))
            time.sleep(0.0005)

    th = threading.Thread(target=sample)
    th.start()
    tickets = []
    for w in ws:
        try:
            tickets.append(srv.submit(w, "fp32_split"))
        except Exception as e:   # a request larger than the whole budget is rejected up front
            assert "REJECTED" in str(e)
    for tk in tickets:
        srv.wait(tk)
    stop.set()
    th.join()
    assert all(h <= budget for h, _, _ in seen)
    assert srv.stats()["completed"] == len(tickets)
    srv.close()


@pytest.mark.timeout(180)
def test_close_while_requests_are_being_prepared(ctx):
    """Closing the server right after a burst of submissions: the requests admitted and still in
    preparation (tables enqueued, factoring flag not yet read) are completed and run before the
    scheduler stops, the queued ones are cancelled, and close returns."""
    from paper_1609_08146_amd import Server
    ws = small_requests(24, seed=19)
    srv = Server(ctx, hbm_budget=int(64e9), max_running=16, quantum_ms=2.0)
    tickets = [srv.submit(w, "fp32_split") for w in ws]
    assert len(tickets) == 24
    t0 = time.perf_counter()
    srv.close()
    assert time.perf_counter() - t0 < 120.0


def test_two_servers_on_one_device(ctx):
    """Two servers at once (each on a context of its own), closed in the order they were created:
    both serve their requests with the alone results, and the device's memory-pool settings that the
    servers share are restored by the last one."""
    from paper_1609_08146_amd import Context, Server
    ws = small_requests(4, seed=23)
    ref = [alone(ctx, w, "fp32_split") for w in ws]
    ctx2 = Context(0)
    s1 = Server(ctx, hbm_budget=int(8e9), max_running=4, quantum_ms=2.0)
    s2 = Server(ctx2, hbm_budget=int(8e9), max_running=4, quantum_ms=2.0)
    t1 = [s1.submit(w, "fp32_split") for w in ws[:2]]
    t2 = [s2.submit(w, "fp32_split") for w in ws[2:]]
    got = [s1.wait(t)[:2] for t in t1] + [s2.wait(t)[:2] for t in t2]
    s1.close()
    s2.close()
    ctx2.close()
    for (E, B), (Er, Br, _, _) in zip(got, ref):
        assert np.array_equal(E, Er) and np.array_equal(B, Br)


def test_rejection_cancel_timeout_and_bad_request(ctx):
    from paper_1609_08146_amd import ScError, Server
    from paper_1609_08146_amd._abi import SC_E_CANCELLED, SC_E_INVAL, SC_E_REJECTED, SC_E_TIMEOUT
    big = workloads.broadband(n_k=8, n_nodes=300)
    srv = Server(ctx, hbm_budget=int(64e6), max_running=1, quantum_ms=5.0)
    with pytest.raises(ScError) as e:
        srv.submit(big, "fp32_split")
    assert e.value.status == SC_E_REJECTED
    bad = workloads.mono().subset(obs_idx=[0, 1])
    bad.f = -1.0
    with pytest.raises(ScError) as e:
        srv.submit(bad, "fp32_split")
    assert e.value.status == SC_E_INVAL
    srv.close()
    # one long request occupies the only running slot; the next one queues and can be cancelled
    srv = Server(ctx, hbm_budget=int(8e9), max_running=1, quantum_ms=5.0)
    long_req = workloads.broadband(n_k=8, n_nodes=400)
    t1 = srv.submit(long_req, "fp32_split")
    t2 = srv.submit(workloads.mono().with_nodes(40, 32), "fp32_split")
    srv.cancel(t2)
    assert srv.wait_status(t2) == SC_E_CANCELLED
    st = srv.wait_status(t1, timeout_ms=0.0)
    assert st in (SC_E_TIMEOUT, 0)
    if st == SC_E_TIMEOUT:
        E, B, _, _, stats = srv.wait(t1)
        assert np.isfinite(E).all()
    s = srv.stats()
    assert s["cancelled"] == 1
    srv.close()


def test_injected_allocation_failure_is_isolated():
    """With the n-th device allocation forced to fail, that request fails cleanly and the others complete."""
    code = r'''
import os, sys
sys.path.insert(0, %r)
import numpy as np, workloads
from paper_1609_08146_amd import Context, Server, ScError
ctx = Context(0)
srv = Server(ctx, hbm_budget=int(8e9), max_running=1, quantum_ms=2.0)
ws = [workloads.mono().with_nodes(40, 32).subset(obs_idx=np.arange(0, 1024, 7)) for _ in range(3)]
tk = [srv.submit(w, "fp32_split") for w in ws]
res = []
for t in tk:
    try:
        srv.wait(t); res.append("ok")
    except ScError as e:
        res.append("fail:%%d" %% e.status)
print("RESULTS", res, srv.stats()["hbm_in_use"])
srv.close(); ctx.close()
''' % ROOT
    env = dict(os.environ, SC_DEBUG_FAIL_ALLOC="30")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    print(out.stdout[-2000:], out.stderr[-2000:])
    assert out.returncode == 0
    line = [l for l in out.stdout.splitlines() if l.startswith("RESULTS")][0]
    assert "fail:-2" in line            # SC_E_NOMEM for the request that hit the failure
    assert line.count("'ok'") == 2
    assert line.rstrip().endswith(" 0")  # nothing left charged


def test_failed_quantum_waits_for_queued_work_and_later_requests_match():
    """A quantum whose job-buffer reservation fails fails its running requests with SC_E_NOMEM only after
    the work already queued for them has drained; requests submitted afterwards give their alone results
    bitwise (their tables must not reuse memory that earlier kernels were still writing)."""
    code = r'''
import sys
sys.path.insert(0, %r)
import numpy as np, workloads
from paper_1609_08146_amd import Context, Server, ScError, problem_from_workload
ctx = Context(0)
big = workloads.broadband(n_k=6, n_nodes=200)
later = [workloads.mono().with_nodes(60 + 10 * i, 40).subset(obs_idx=np.arange(0, 1024, 5 + i)) for i in range(3)]
ref = []
for w in later:
    p = problem_from_workload(ctx, w); ref.append(p.evaluate("fp32_split")); p.close()
srv = Server(ctx, hbm_budget=int(8e9), max_running=2, quantum_ms=0.5)
t_big = srv.submit(big, "fp32_split")
try:
    srv.wait(t_big); print("BIG ok")
except ScError as e:
    print("BIG fail:%%d" %% e.status)
tk = [srv.submit(w, "fp32_split") for w in later]
same = []
for t, (E0, B0) in zip(tk, ref):
    E, B, _, _, _ = srv.wait(t)
    same.append(bool(np.array_equal(E, E0) and np.array_equal(B, B0)))
s = srv.stats()
print("LATER", same, s["completed"], s["hbm_in_use"])
srv.close(); ctx.close()
''' % ROOT
    env = dict(os.environ, SC_DEBUG_FAIL_QUANTUM="2")
    out = subprocess.run([sys.executable, "-u", "-c", code], env=env, capture_output=True, text=True, timeout=180)
    print(out.stdout[-2000:], out.stderr[-2000:])
    assert out.returncode == 0
    assert "BIG fail:-2" in out.stdout          # SC_E_NOMEM for the request whose tiles were in that quantum
    line = [l for l in out.stdout.splitlines() if l.startswith("LATER")][0]
    assert line == "LATER [True, True, True] 3 0"
