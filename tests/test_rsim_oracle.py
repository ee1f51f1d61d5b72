"""Pins of the random-simulation oracle (oracle/rsim.py) against facts outside it.

Sources of truth:
  * closed-form arithmetic: the output rows of multipliers and a MAC, simulated
    on seeded random input words, must equal a*b and a*b + c*d bit by bit;
  * exhaustive simulation of a miter (input words = all patterns) reduces to
    exact simulation: an equivalent miter's output row is zero everywhere and a
    faulty miter's lowest set bit is the lowest counterexample of the ES oracle;
  * the MurmurHash3 32-bit finaliser's published values (the x86_32 hash of the
    empty input is fmix32(seed)); a hash worked by hand from them;
  * functional facts about classes: the paired outputs of two multipliers are
    the same function, so they share a class; members of one class have equal
    normalised rows; a row and its complement hash alike.
Planted mistakes at the end check that each pin can fail.
"""
import numpy as np
import pytest

import miters
import oracle
from miters.aig import Aig, import_into
from miters.miter import mult_circuit, mac_circuit
from oracle import rsim


def random_words(n, W, seed):
    r = miters.SplitMix64(seed)
    return np.array([[r.next_u64() & 0xFFFFFFFF for _ in range(W)] for _ in range(n)], dtype=np.uint32)


def pattern_values(words, lo, count):
    """Integer formed by input rows lo..lo+count-1 at every pattern (bit j of word k = pattern 32k+j)."""
    W = words.shape[1]
    bits = np.unpackbits(words[lo:lo + count].view(np.uint8).reshape(count, W, 4)[:, :, ::-1], axis=2)
    bits = bits[:, :, ::-1].reshape(count, 32 * W).astype(np.uint64)
    return sum(bits[i] << np.uint64(i) for i in range(count))


def output_values(sig, outputs):
    W = sig.shape[1]
    acc = np.zeros(32 * W, dtype=np.uint64)
    for i, lit in enumerate(outputs):
        row = rsim.literal_row(sig, lit)
        bits = np.unpackbits(row.view(np.uint8).reshape(W, 4)[:, ::-1], axis=1)[:, ::-1].reshape(32 * W)
        acc |= bits.astype(np.uint64) << np.uint64(i)
    return acc


@pytest.mark.parametrize("kind,w", [("array", 8), ("wallace", 8), ("booth", 8), ("booth", 5)])
def test_multiplier_rows_match_products(kind, w):
    g = mult_circuit(kind, w)
    words = random_words(2 * w, 64, seed=11 + w)
    sig = rsim.simulate(g.to_aag(), words)
    a = pattern_values(words, 0, w)
    b = pattern_values(words, w, w)
    assert np.array_equal(output_values(sig, g.outputs), a * b)


def test_mac_rows_match_closed_form():
    w = 4
    g = mac_circuit("fused", w)
    words = random_words(4 * w, 48, seed=3)
    sig = rsim.simulate(g.to_aag(), words)
    a, b, c, d = (pattern_values(words, k * w, w) for k in range(4))
    assert np.array_equal(output_values(sig, g.outputs), a * b + c * d)


def exhaustive_words(n):
    """Input words that enumerate all 2^n patterns (pattern p sets input i to bit i of p)."""
    P = 1 << n
    p = np.arange(max(P, 32), dtype=np.uint64) % np.uint64(P)
    rows = []
    for i in range(n):
        bits = ((p >> np.uint64(i)) & np.uint64(1)).astype(np.uint32).reshape(-1, 32)
        rows.append((bits << np.arange(32, dtype=np.uint32)).sum(axis=1, dtype=np.uint32))
    return np.array(rows, dtype=np.uint32)


@pytest.mark.parametrize("name", ["mult6_array_wallace", "mult6_array_wallace_f1"])
def test_exhaustive_simulation_is_exact_simulation(name):
    g = miters.workload(name)
    aag = g.to_aag()
    sig = rsim.simulate(aag, exhaustive_words(g.num_inputs))
    miter = np.zeros(sig.shape[1], dtype=np.uint32)
    for lit in g.outputs:
        miter |= rsim.literal_row(sig, lit)
    nz = np.flatnonzero(miter)
    lowest = None if nz.size == 0 else int(32 * nz[0] + (int(miter[nz[0]]) & -int(miter[nz[0]])).bit_length() - 1)
    assert lowest == oracle.check(aag)


def test_fmix32_published_values():
    # MurmurHash3_x86_32 of the empty input with seed s is fmix32(s).
    assert int(rsim.fmix32(1)) == 0x514E28B7
    assert int(rsim.fmix32(0xFFFFFFFF)) == 0x81F16F39
    assert int(rsim.fmix32(0)) == 0


def test_hash_worked_by_hand():
    # key_0 = fmix32(0) | 1 = 1, key_1 = fmix32(1) | 1 = 0x514E28B7
    sig = np.array([[2, 3], [7, 3], [0, 0], [0xFFFFFFFF, 0xFFFFFFFF], [6, 0]], dtype=np.uint32)
    h, ones = rsim.signature_hash(sig)
    assert int(h[0]) == (2 + 3 * 0x514E28B7) % (1 << 64) == 0xF3EA7A27
    # row 1 starts with a 1: hashed as its complement [~7, ~3]
    assert int(h[1]) == (0xFFFFFFF8 + 0xFFFFFFFC * 0x514E28B7) % (1 << 64)
    assert int(h[2]) == 0 and int(h[3]) == 0       # constant 0 and constant 1 alike
    assert int(h[4]) == 6
    assert ones.tolist() == [3, 5, 0, 64, 2]


def test_hash_complement_and_equal_rows():
    rows = random_words(40, 33, seed=9)
    sig = np.concatenate([rows, ~rows, rows[:5]])
    h, ones = rsim.signature_hash(sig)
    assert np.array_equal(h[:40], h[40:80])
    assert np.array_equal(ones[:40] + ones[40:80], np.full(40, 32 * 33, dtype=np.uint64))
    assert np.array_equal(h[80:], h[:5])
    assert len(set(h[:40].tolist())) == 40           # distinct random rows, distinct hashes


def paired_miter(w):
    a, b = mult_circuit("array", w), mult_circuit("booth", w)
    g = Aig(a.num_inputs)
    oa, ob = import_into(g, a), import_into(g, b)
    for x, y in zip(oa, ob):
        g.add_output(g.XOR(x, y))
    return g, oa, ob


def test_paired_outputs_share_a_class():
    g, oa, ob = paired_miter(6)
    sig = rsim.simulate(g.to_aag(), random_words(12, 16, seed=21))
    h, _ = rsim.signature_hash(sig)
    cls = rsim.classes(h)
    for x, y in zip(oa, ob):
        if x >> 1 and y >> 1:
            assert cls[x >> 1] == cls[y >> 1]
    # brute force: members of a class have equal normalised rows
    norm = np.where((sig[:, :1] & 1).astype(bool), ~sig, sig)
    for r in range(sig.shape[0]):
        assert np.array_equal(norm[r], norm[cls[r]])
        assert cls[r] <= r


def test_classes_first_member():
    assert rsim.classes(np.array([5, 7, 5, 9, 7], dtype=np.uint64)).tolist() == [0, 1, 0, 3, 1]


# ---- planted mistakes: each must break a pin above ------------------------------------

def test_planted_mistakes_are_caught(monkeypatch):
    good_sim = rsim.simulate

    def drop_second_complement(aag, pi):
        n, ands, _ = rsim.read_aag(aag)
        sig = np.zeros((n + 1 + len(ands), pi.shape[1]), dtype=np.uint32)
        sig[1:n + 1] = pi
        for v, r0, r1 in ands:
            a = sig[r0 >> 1] ^ (np.uint32(0xFFFFFFFF) if r0 & 1 else np.uint32(0))
            sig[v] = a & sig[r1 >> 1]
        return sig

    monkeypatch.setattr(rsim, "simulate", drop_second_complement)
    with pytest.raises(AssertionError):
        test_multiplier_rows_match_products("array", 8)
    monkeypatch.setattr(rsim, "simulate", good_sim)

    good_keys = rsim.hash_keys
    monkeypatch.setattr(rsim, "hash_keys", lambda W: np.ones(W, dtype=np.uint64))
    with pytest.raises(AssertionError):
        test_hash_worked_by_hand()
    monkeypatch.setattr(rsim, "hash_keys", good_keys)

    good_hash = rsim.signature_hash

    def no_normalisation(sig):
        keys = rsim.hash_keys(sig.shape[1])
        with np.errstate(over="ignore"):
            h = (sig.astype(np.uint64) * keys[None, :]).sum(axis=1, dtype=np.uint64)
        return h, np.bitwise_count(sig).sum(axis=1, dtype=np.uint64)

    monkeypatch.setattr(rsim, "signature_hash", no_normalisation)
    with pytest.raises(AssertionError):
        test_hash_complement_and_equal_rows()
    monkeypatch.setattr(rsim, "signature_hash", good_hash)
