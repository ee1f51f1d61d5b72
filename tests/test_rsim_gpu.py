"""GPU parity of random-pattern simulation, signature hashing and candidate classes.

The HIP path (the interpreter kernel in simulation mode, the hash kernel, the
library's class grouping) is compared element by element with the plain CPU
oracle (oracle/rsim.py) on the same seeded input words: bit-exact for the
signature rows, the hashes, the ones counts and the class map.
"""
import numpy as np
import pytest

import miters
from miters.aig import Aig, import_into
from miters.miter import mult_circuit, mac_circuit
from oracle import rsim

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def es():
    import paper_2512_06627_amd as m
    return m


def words_of(n, W, seed):
    r = miters.SplitMix64(seed)
    return np.array([[r.next_u64() & 0xFFFFFFFF for _ in range(W)] for _ in range(n)],
                    dtype=np.uint32).reshape(n, W)


def gpu_sim(aag: bytes, words: np.ndarray, **opts):
    E = es()
    c = E.fastlec_es_load_aig(aag)
    info = c.info()
    n, W = words.shape
    V = info["num_pis"] + info["num_ands"]
    pi = torch.from_numpy(words.view(np.int32).copy()).cuda() if n else None
    sig = torch.full((V + 1, W), -1, dtype=torch.int32, device="cuda")
    # torch filled the buffers on its current stream: run on that stream, so the library's
    # kernels are ordered after the fills (another stream could overtake them)
    ms = E.fastlec_es_simulate(c, pi, W, sig, stream=torch.cuda.current_stream(), **opts)
    assert ms >= 0
    return sig, c


def gpu_hash(sig):
    E = es()
    rows, W = sig.shape
    h = torch.zeros(rows, dtype=torch.int64, device="cuda")
    ones = torch.zeros(rows, dtype=torch.int64, device="cuda")
    E.fastlec_es_signature_hash(sig, rows, W, h, ones, stream=torch.cuda.current_stream())
    return h.cpu().numpy().view(np.uint64), ones.cpu().numpy().view(np.uint64)


def paired_miter(w):
    a, b = mult_circuit("array", w), mult_circuit("booth", w)
    g = Aig(a.num_inputs)
    oa, ob = import_into(g, a), import_into(g, b)
    for x, y in zip(oa, ob):
        g.add_output(g.XOR(x, y))
    return g


def with_dead_gates():
    """Outputs use only part of the logic: the other gates are outside the outputs' cone."""
    g = mult_circuit("array", 5)
    live = list(g.outputs)
    g.outputs = live[:3]
    x = g.AND(g.input(0) ^ 1, g.input(7))
    g.AND(x, g.input(9) ^ 1)  # feeds nothing
    return g


CIRCUITS = {
    "mult8_array": lambda: mult_circuit("array", 8),
    "mult8_booth": lambda: mult_circuit("booth", 8),
    "mac4_fused": lambda: mac_circuit("fused", 4),
    "miter6_array_wallace": lambda: miters.workload("mult6_array_wallace"),
    "paired_miter8": lambda: paired_miter(8),
    "layered_n20": lambda: miters.layered_cone_miter(31, 20, 2000),
    "dead_gates": with_dead_gates,
}


@pytest.mark.parametrize("name", sorted(CIRCUITS))
@pytest.mark.parametrize("W", [1, 31, 64, 65, 200, 4096 + 7])
def test_signatures_hashes_classes_match_oracle(name, W):
    g = CIRCUITS[name]()
    aag = g.to_aag()
    words = words_of(g.num_inputs, W, seed=1000 + W)
    sig, _ = gpu_sim(g.to_aig(), words)
    got = sig.cpu().numpy().view(np.uint32)
    want = rsim.simulate(aag, words)
    assert got.shape == want.shape
    bad = np.argwhere(got != want)
    assert bad.size == 0, f"{name} W={W}: first mismatch at (row, word) {bad[0].tolist()}"
    h, ones = gpu_hash(sig)
    wh, wones = rsim.signature_hash(want)
    assert np.array_equal(h, wh)
    assert np.array_equal(ones, wones)
    assert np.array_equal(es().fastlec_es_classes(h), rsim.classes(wh))


@pytest.mark.parametrize("K", [1, 2, 4])
@pytest.mark.parametrize("kernel", ["interp", "interp_hbm"])
def test_lane_widths_and_value_file_tiers(K, kernel):
    g = paired_miter(8)
    W = 3000 + K
    words = words_of(16, W, seed=7 + K)
    sig, _ = gpu_sim(g.to_aig(), words, words_per_thread=K, kernel=kernel)
    assert np.array_equal(sig.cpu().numpy().view(np.uint32), rsim.simulate(g.to_aag(), words))


def test_small_workgroups_and_tiles():
    g = miters.layered_cone_miter(5, 18, 1500)
    W = 1000
    words = words_of(18, W, seed=3)
    sig, _ = gpu_sim(g.to_aig(), words, wg_size=64, tile_words=64)
    assert np.array_equal(sig.cpu().numpy().view(np.uint32), rsim.simulate(g.to_aag(), words))


def test_paired_outputs_share_classes_on_gpu():
    a, b = mult_circuit("array", 8), mult_circuit("booth", 8)
    g = Aig(16)
    oa, ob = import_into(g, a), import_into(g, b)
    for x, y in zip(oa, ob):
        g.add_output(g.XOR(x, y))
    sig, _ = gpu_sim(g.to_aig(), words_of(16, 256, seed=77))
    h, _ = gpu_hash(sig)
    cls = es().fastlec_es_classes(h)
    for x, y in zip(oa, ob):
        if x >> 1 and y >> 1:
            assert cls[x >> 1] == cls[y >> 1]


def test_repeated_calls_reuse_cached_program():
    g = paired_miter(6)
    words = words_of(12, 500, seed=5)
    first, c = gpu_sim(g.to_aig(), words)
    info = c.info()
    V = info["num_pis"] + info["num_ands"]
    for W in (500, 77):
        w = words[:, :W].copy()
        sig = torch.zeros((V + 1, W), dtype=torch.int32, device="cuda")
        es().fastlec_es_simulate(c, torch.from_numpy(w.view(np.int32)).cuda(), W, sig,
                                 stream=torch.cuda.current_stream())
        assert np.array_equal(sig.cpu().numpy().view(np.uint32), rsim.simulate(g.to_aag(), w))


def test_full_size_sampled_columns():
    """16x16 multiplier miter on 2^18 words (2^23 patterns), the benchmark's shape: sampled
    columns against the oracle (simulation is column-wise), every row's hash against the
    oracle's hash of the same rows."""
    g = miters.workload("mult16_array_booth")
    W = 1 << 18
    r = np.random.default_rng(12)
    words = r.integers(0, 1 << 32, size=(32, W), dtype=np.uint64).astype(np.uint32)
    sig, _ = gpu_sim(g.to_aig(), words)
    cols = np.concatenate([[0, 1, 63, 64, W - 1], r.choice(W, 59, replace=False)])
    got = sig[:, torch.from_numpy(cols).cuda()].cpu().numpy().view(np.uint32)
    want = rsim.simulate(g.to_aag(), words[:, cols])
    assert np.array_equal(got, want)
    h, ones = gpu_hash(sig)
    rows = np.concatenate([[0, 1, 32, 33, sig.shape[0] - 1], r.choice(sig.shape[0], 27, replace=False)])
    host_rows = sig[torch.from_numpy(rows).cuda()].cpu().numpy().view(np.uint32)
    wh, wones = rsim.signature_hash(host_rows)
    assert np.array_equal(h[rows], wh)
    assert np.array_equal(ones[rows], wones)


def test_invalid_arguments():
    E = es()
    c = E.fastlec_es_load_aig(mult_circuit("array", 4).to_aig())
    sig = torch.zeros((40, 8), dtype=torch.int32, device="cuda")
    with pytest.raises(E.EsError):
        E.fastlec_es_simulate(c, None, 8, sig)     # inputs needed
    with pytest.raises(E.EsError):
        E.fastlec_es_simulate(c, sig, 0, sig)      # no words
    with pytest.raises(E.EsError):
        E.fastlec_es_signature_hash(sig, 0, 8, sig, sig)


def _hand_files():
    import os
    d = os.path.join(os.path.dirname(__file__), "golden", "hand")
    out = []
    for f in sorted(os.listdir(d)):
        b = open(os.path.join(d, f), "rb").read()
        try:
            rsim.read_aag(b)
        except ValueError:
            continue  # not a canonical latch-free file (out-of-order lines, latches, cycles, ...)
        out.append((f, b))
    return out


@pytest.mark.parametrize("name,text", _hand_files(), ids=[f for f, _ in _hand_files()])
@pytest.mark.parametrize("W", [1, 70])
def test_hand_worked_files(name, text, W):
    """Constant outputs, zero inputs, multi-output and inverted outputs (hand-worked files)."""
    n = rsim.read_aag(text)[0]
    words = words_of(n, W, seed=len(name) + W)
    sig, _ = gpu_sim(text, words)
    want = rsim.simulate(text, words)
    assert np.array_equal(sig.cpu().numpy().view(np.uint32), want)
    h, ones = gpu_hash(sig)
    wh, wones = rsim.signature_hash(want)
    assert np.array_equal(h, wh) and np.array_equal(ones, wones)
