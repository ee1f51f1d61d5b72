"""Device memory the library uses: caller-owned scratch for plain checks, pinned staging that
does not grow with device-memory value files, and a server whose real device memory stays
within its budget when jobs need value files in device memory."""
import pytest

import miters
import oracle
import paper_2512_06627_amd as es

pytestmark = pytest.mark.gpu


def _answer(r):
    assert r["verdict"] in (es.FASTLEC_EQUIVALENT, es.FASTLEC_NONEQUIVALENT), r
    return r["cex"] if r["verdict"] == es.FASTLEC_NONEQUIVALENT else None


def test_dev_scratch_replaces_library_buffers():
    import torch
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    gs = [miters.workload("mult12_array_booth_f3"), miters.workload("mult6_array_wallace"),
          miters.layered_cone_miter(4242, 20, 2500, fault_seed=7)]
    cs = [es.fastlec_es_load_aig(g.to_aig()) for g in gs]
    want = [oracle.Circuit(g.to_aag()).lowest_failure(threads=8)[0] for g in gs]
    kernels = ("interp", "interp_hbm", "specialized")
    for c in cs:  # warm: pool buffers, kernels, streams
        for k in kernels:
            es.fastlec_es_check(c, kernel=k, stream=stream)
    before = es.fastlec_es_memory_get()
    scratch = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    for c, w in zip(cs, want):
        for k in kernels:
            r = es.fastlec_es_check(c, kernel=k, stream=stream, scratch=scratch)
            assert _answer(r) == w, (k, r)
    after = es.fastlec_es_memory_get()
    assert after["device_bytes"] == before["device_bytes"], (before, after)
    tiny = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(es.EsError) as ei:
        es.fastlec_es_check(cs[0], kernel="interp", stream=stream, scratch=tiny)
    assert ei.value.code == es.FASTLEC_ERR_INVALID and "needs" in str(ei.value)


def test_pinned_staging_does_not_grow_with_value_files():
    # A wide cone on the device-memory tier: value files of hundreds of MB, staging of a few KB.
    g = miters.layered_cone_miter(4343, 14, 30000)
    c = es.fastlec_es_load_aig(g.to_aig())
    before = es.fastlec_es_memory_get()
    r = es.fastlec_es_check(c, kernel="interp_hbm")
    after = es.fastlec_es_memory_get()
    assert _answer(r) is None
    grew_dev = after["device_bytes"] - before["device_bytes"]
    grew_pinned = after["pinned_bytes"] - before["pinned_bytes"]
    assert grew_dev >= 64 << 20, (before, after)
    assert grew_pinned <= 1 << 20, (before, after)


def test_server_device_memory_within_budget_with_device_memory_tier():
    # Cones whose value files exceed LDS (peak live slots above 600) run on the device-memory
    # tier; the budget (8 MiB over the ~2.3 MB job table) caps their launch grid.
    big = [miters.layered_cone_miter(4400 + i, 12, 90000, fault_seed=(3 if i == 1 else None)) for i in range(2)]
    small = [miters.layered_cone_miter(4500 + i, 16, 1500, fault_seed=(i + 1 if i % 2 else None)) for i in range(4)]
    gs = big + small
    assert all(es.fastlec_es_load_aig(g.to_aig()).info()["peak_live_slots"] > 640 for g in big)
    cs = [es.fastlec_es_load_aig(g.to_aig()) for g in gs]
    want = [oracle.Circuit(g.to_aag()).lowest_failure(threads=8)[0] for g in gs]
    budget = 8 << 20
    srv = es.Server(budget + (3 << 20))
    try:
        res = [srv.poll(t, wait=True) for t in [srv.submit(c) for c in cs]]
        st = srv.stats()
    finally:
        srv.close()
    assert [_answer(r) for r in res] == want
    assert st["device_bytes"] <= st["budget_bytes"], st
    with pytest.raises(es.EsError):
        es.Server(1 << 20)  # smaller than the job table
