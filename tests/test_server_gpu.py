"""Serving (continuous batching) and host-forced stop conditions, on the GPU.

Each job's answer in the serving mix must equal its answer alone (plain
fastlec_es_check) and the oracle's, bit for bit; the admission rule must keep
the summed charge of jobs in flight within the budget.
"""
import ctypes
import threading
import time

import pytest

import miters
import oracle
import paper_2512_06627_amd as es

pytestmark = pytest.mark.gpu


def _jobs(seed, count, n_lo, n_hi, size_lo, size_hi, faulty_every=4):
    rng = miters.SplitMix64(seed)
    out = []
    for i in range(count):
        n = rng.between(n_lo, n_hi)
        fault = rng.between(1, 1000) if i % faulty_every == 0 else None
        g = miters.layered_cone_miter(seed * 1000 + i, n, rng.between(size_lo, size_hi), fault_seed=fault)
        out.append(g)
    return out


def _answer(r):
    assert r["verdict"] in (es.FASTLEC_EQUIVALENT, es.FASTLEC_NONEQUIVALENT), r
    return r["cex"] if r["verdict"] == es.FASTLEC_NONEQUIVALENT else None


def test_server_mix_equals_alone_and_oracle():
    gs = _jobs(11, 40, 10, 20, 200, 2500)
    circs = [es.fastlec_es_load_aig(g.to_aig()) for g in gs]
    alone = [_answer(es.fastlec_es_check(c, kernel="interp")) for c in circs]
    want = [oracle.check(g.to_aag(), threads=8) for g in gs]
    assert alone == want
    srv = es.Server(1 << 34)
    tickets = [srv.submit(c) for c in circs]
    res = [srv.poll(t, wait=True) for t in tickets]
    assert [_answer(r) for r in res] == want
    st = srv.stats()
    assert st["completed"] == len(gs) and st["peak_charge_bytes"] <= st["budget_bytes"]
    assert st["max_active"] >= 2  # jobs overlapped on the device
    assert all(r["latency_ms"] >= r["queued_ms"] >= 0 for r in res)
    srv.close()


def test_server_budget_bounds_jobs_in_flight():
    gs = _jobs(12, 16, 14, 18, 500, 1500)
    circs = [es.fastlec_es_load_aig(g.to_aig()) for g in gs]
    charges = []
    for c in circs:
        i = c.info()
        charges.append(i["peak_live_slots"] * min(1 << (i["num_pis"] - 6), 1 << 22) * 8)
    budget = 2 * max(charges)
    srv = es.Server(budget)
    tickets = [srv.submit(c) for c in circs]
    res = [srv.poll(t, wait=True) for t in tickets]
    st = srv.stats()
    assert st["peak_charge_bytes"] <= budget
    assert st["completed"] == len(gs)
    alone = [_answer(es.fastlec_es_check(c, kernel="interp")) for c in circs]
    assert [_answer(r) for r in res] == alone
    srv.close()


def test_server_rejects_job_that_can_never_fit():
    g = miters.layered_cone_miter(5, 20, 800)
    c = es.fastlec_es_load_aig(g.to_aig())
    i = c.info()
    budget = 3 << 20  # above the server's job table (about 2.3 MB), below this job's charge
    assert i["peak_live_slots"] * (1 << (i["num_pis"] - 6)) * 8 > budget
    srv = es.Server(budget)
    with pytest.raises(es.EsError) as ei:
        srv.submit(c)
    assert ei.value.code == es.FASTLEC_REJECTED
    assert srv.stats()["rejected"] == 1
    srv.close()


def test_server_arrivals_while_running():
    """Jobs submitted from another thread while earlier ones are on the device."""
    gs = _jobs(13, 24, 16, 22, 300, 3000)
    circs = [es.fastlec_es_load_aig(g.to_aig()) for g in gs]
    srv = es.Server(1 << 36)
    tickets = [None] * len(circs)

    def feeder():
        for i, c in enumerate(circs):
            tickets[i] = srv.submit(c)
            time.sleep(0.002)

    th = threading.Thread(target=feeder)
    th.start()
    th.join()
    res = [srv.poll(t, wait=True) for t in tickets]
    alone = [_answer(es.fastlec_es_check(c, kernel="interp")) for c in circs]
    assert [_answer(r) for r in res] == alone
    srv.close()


def test_poll_unknown_ticket_and_nonblocking():
    srv = es.Server(1 << 30)
    with pytest.raises(es.EsError) as ei:
        srv.poll(12345)
    assert ei.value.code == es.FASTLEC_ERR_INVALID
    c = es.fastlec_es_load_aig(miters.minterm_miter(12, [100]).to_aag())
    t = srv.submit(c)
    r = srv.poll(t, wait=True)
    assert r["cex"] == 100
    srv.close()


def test_deadline_and_cancel_forced_from_host():
    c = es.fastlec_es_load_aig(miters.workload("mult12_array_booth").to_aig())
    with pytest.raises(es.EsError) as ei:
        es.fastlec_es_check(c, kernel="interp", deadline_s=1e-9)
    assert ei.value.code == es.FASTLEC_TIMEOUT
    assert ei.value.result["next_word"] <= 1 << 18
    flag = ctypes.c_int(1)
    with pytest.raises(es.EsError) as ei:
        es.fastlec_es_check(c, kernel="interp", cancel_flag=flag)
    assert ei.value.code == es.FASTLEC_CANCELLED
    assert ei.value.result["patterns_evaluated"] == 0
    # an unraised flag and a generous deadline change nothing
    flag.value = 0
    r = es.fastlec_es_check(c, kernel="interp", cancel_flag=flag, deadline_s=600.0)
    assert r["verdict"] == es.FASTLEC_EQUIVALENT and r["patterns_evaluated"] == 1 << 24


def test_server_specialized_tier_switch_mid_job(monkeypatch):
    """Every job is handed to the compile thread (test hook) and steps are 1 ms, so jobs
    start on the interpreter and finish on their specialized kernel; each answer must equal
    the same circuit checked alone on the interpreter, and again when submitted a second
    time (compiled kernel reused from the first step)."""
    monkeypatch.setenv("FASTLEC_ES_SERVER_JIT", "2")
    monkeypatch.setenv("FASTLEC_ES_SERVER_STEP_MS", "1")
    gs = _jobs(31, 6, 20, 24, 800, 2000, faulty_every=2)
    circs = [es.fastlec_es_load_aig(g.to_aig()) for g in gs]
    alone = [_answer(es.fastlec_es_check(c, kernel="interp")) for c in circs]
    srv = es.Server(8 << 30)
    try:
        for rep in range(2):
            print("submission round", rep, flush=True)
            tickets = [srv.submit(c) for c in circs]
            got = [_answer(srv.poll(t, wait=True)) for t in tickets]
            assert got == alone, rep
        st = srv.stats()
        assert st["specialized_slices"] > 0, st
    finally:
        srv.close()


def test_server_compiles_queued_jobs_in_groups(monkeypatch):
    """More jobs than compile threads (one per compile helper process, each compiling one job's
    kernel at a time) or than one in-process compile group (eight), one circuit submitted twice
    in the same round (its kernel compiles once); in a second round the compiled kernels run from
    the first step.  Every answer equals the circuit checked alone (and the oracle's where it is
    cheap)."""
    monkeypatch.setenv("FASTLEC_ES_SERVER_JIT", "2")
    monkeypatch.setenv("FASTLEC_ES_SERVER_STEP_MS", "1")
    gs = _jobs(47, 11, 20, 24, 800, 2000, faulty_every=3)
    circs = [es.fastlec_es_load_aig(g.to_aig()) for g in gs]
    alone = [_answer(es.fastlec_es_check(c, kernel="interp")) for c in circs]
    for g, a in zip(gs, alone):
        if g.num_inputs <= 20:
            assert a == oracle.check(g.to_aag(), threads=16)
    srv = es.Server(8 << 30)
    try:
        subs = circs + [circs[0]]
        for rep in range(2):
            print("submission round", rep, flush=True)
            tickets = [srv.submit(c) for c in subs]
            got = [_answer(srv.poll(t, wait=True)) for t in tickets]
            assert got == alone + [alone[0]], rep
        assert srv.stats()["specialized_slices"] > 0
    finally:
        srv.close()
