"""Seeded input generators: determinism, cell library by closed form, workload shapes."""
import numpy as np
import pytest

import miters
import oracle
from miters.aig import Aig
from miters.miter import _cell_fa, _cell_ha, layered_cone_pair


def test_splitmix64_published_sequence():
    """First outputs of SplitMix64 from state 0, as published with the generator."""
    r = miters.SplitMix64(0)
    assert [r.next_u64() for _ in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_rng_below_is_uniform_enough_and_in_range():
    r = miters.SplitMix64(3)
    xs = [r.below(7) for _ in range(7000)]
    assert min(xs) == 0 and max(xs) == 6
    counts = np.bincount(xs)
    assert counts.min() > 850


@pytest.mark.parametrize("enc", [0, 1, 2])
def test_full_adder_cells_closed_form(enc):
    g = Aig(3)
    s, c = _cell_fa(g, enc, g.input(0), g.input(1), g.input(2))
    g.add_output(s)
    g.add_output(c)
    ps = np.arange(8, dtype=np.uint64)
    want = (ps & 1) + ((ps >> 1) & 1) + ((ps >> 2) & 1)
    assert np.array_equal(oracle.Circuit(g.to_aag()).outputs(ps), want)


@pytest.mark.parametrize("enc", [0, 1, 2])
def test_half_adder_cells_closed_form(enc):
    g = Aig(2)
    s, c = _cell_ha(g, enc, g.input(0), g.input(1))
    g.add_output(s)
    g.add_output(c)
    ps = np.arange(4, dtype=np.uint64)
    assert np.array_equal(oracle.Circuit(g.to_aag()).outputs(ps), (ps & 1) + (ps >> 1))


def test_cell_encodings_differ_structurally():
    sizes = set()
    for enc in range(3):
        g = Aig(3)
        _cell_fa(g, enc, g.input(0), g.input(1), g.input(2))
        sizes.add(tuple(g.ands))
    assert len(sizes) == 3


@pytest.mark.parametrize("seed,n,target", [(1, 10, 300), (2, 12, 600), (3, 14, 900), (4, 9, 200)])
def test_layered_cone_equivalent_by_oracle(seed, n, target):
    m = miters.layered_cone_miter(seed, n, target)
    assert m.num_inputs == n
    assert oracle.check(m.to_aag(), threads=4) is None


def test_layered_cone_shape():
    for seed in range(5):
        A, B = layered_cone_pair(seed, 20, 2000)
        assert 1 <= len(A.outputs) <= 16 and len(A.outputs) == len(B.outputs)
        # every input is in the output cone
        used = set()
        first = A.num_inputs + 1
        for k in A.tfi_ands():
            for r in A.ands[k]:
                if 1 <= r >> 1 < first:
                    used.add(r >> 1)
        assert used == set(range(1, 21))
        m = miters.miter_of(A, B)
        assert 1000 <= len(m.tfi_ands()) <= 4000


def test_layered_cone_deterministic():
    a = miters.layered_cone_miter(11, 22, 1500, fault_seed=3).to_aag()
    b = miters.layered_cone_miter(11, 22, 1500, fault_seed=3).to_aag()
    assert a == b


def test_fault_flips_exactly_one_fanin():
    c = miters.miter.mult_circuit("booth", 6)
    f = miters.inject_fault(c, 9)
    diff = [k for k, (x, y) in enumerate(zip(c.ands, f.ands)) if x != y]
    assert len(diff) == 1
    (a0, a1), (b0, b1) = c.ands[diff[0]], f.ands[diff[0]]
    assert (a0 ^ b0) + (a1 ^ b1) == 1


def test_faulty_layered_cone_has_failures_near_expected_rate():
    """Most single-fanin faults in these cones are observable (seeded; checked by the oracle)."""
    found = 0
    for s in range(1, 11):
        m = miters.layered_cone_miter(100 + s, 10, 300, fault_seed=s)
        found += oracle.check(m.to_aag(), threads=4) is not None
    assert found >= 7


def test_named_workload_sizes():
    """AND counts of the named workloads (input count, ANDs in the output cone)."""
    want = {
        "mult6_array_wallace": (12, 643),
        "mult12_array_booth": (24, 3078),
        "mult16_array_booth": (32, 5494),
        "mac8_fused_separate": (32, 2776),
    }
    for name, (n, ands) in want.items():
        g = miters.workload(name)
        assert (g.num_inputs, len(g.tfi_ands())) == (n, ands), name


def test_aig_binary_header_and_size():
    g = miters.mult_miter(4, "booth")
    b = g.to_aig(symbols=False)
    head = b.split(b"\n", 1)[0].decode().split()
    assert head == ["aig", str(g.max_var), "8", "0", "1", str(g.num_ands())]
