"""GPU parity of the interpreter's fused XOR instructions.

Parity miters built from the three common three-AND XOR forms: each side computes the parity of
the inputs in another form and order, the miter XORs the two sides.  The equivalent miter
exercises every fused instruction on every pattern; the faulty ones (an extra AND term, or a
dropped input) have a known lowest counterexample, which the oracle confirms.  Checked with the
interpreter at one, two and four words per lane and with value files in LDS and device memory.
"""
import pytest

import oracle
import paper_2512_06627_amd as es
from miters.aig import Aig

pytestmark = pytest.mark.gpu

N = 20


def parity_miter(fault=None):
    g = Aig(N)
    xs = [g.input(i) for i in range(N)]
    a = xs[0]
    for x in xs[1:]:
        a = g.XOR(a, x)
    order = xs[::-1]
    if fault == "drop13":
        order = [x for x in order if x != g.input(13)]
    b = order[0]
    for i, x in enumerate(order[1:]):
        b = (g.XOR_alt if i % 2 else g.XOR_andor)(b, x)
    if fault == "and3_17":
        b = g.XOR(b, g.AND(g.input(3), g.input(17)))
    g.add_output(g.XOR(a, b))
    return g


CASES = [(None, None), ("drop13", 1 << 13), ("and3_17", (1 << 3) | (1 << 17))]


@pytest.mark.parametrize("fault,want", CASES, ids=["equivalent", "drop13", "and3_17"])
@pytest.mark.parametrize("kernel", ["interp", "interp_hbm"])
@pytest.mark.parametrize("K", [1, 2, 4])
def test_parity_miters(fault, want, kernel, K):
    g = parity_miter(fault)
    assert oracle.check(g.to_aag(), threads=16) == want
    c = es.fastlec_es_load_aig(g.to_aig())
    assert c.info()["num_xors"] >= 2 * (N - 2)
    r = es.fastlec_es_check(c, kernel=kernel, words_per_thread=K)
    got = None if r["verdict"] == es.FASTLEC_EQUIVALENT else r["cex"]
    assert got == want
