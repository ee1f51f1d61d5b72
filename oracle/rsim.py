"""Plain CPU oracle for random-pattern simulation and candidate-equivalence classes.

TEST INFRASTRUCTURE ONLY: the test suite and the benchmark's CPU-baseline leg
are its only users; the GPU path never calls it.

A sweeping flow starts with logic simulation that proposes potentially
equivalent (PE) node pairs, which the exact engines then check (paper,
Section 2.3, step 1 of the standard sweeping flow; Section 3.2 uses random
simulation again for its stability and entropy features).  This module
computes, one AND gate at a time over whole numpy rows:

* ``simulate``: the value of every variable of a latch-free ASCII AIGER file
  on caller-given input words.  Row v is variable v; row 0 is constant false,
  rows 1..n are the input words, every AND row is the AND of its two fan-in
  rows with the literal's complement applied (Section 2.1: AND gates and
  inverted edges).  Bit j of word k of a row is the value at pattern 32k + j.
* ``signature_hash``: per row, the number of ones, and a hash of the row
  normalised so that a node and its complement hash alike: the row is
  complemented when its first pattern is 1, then
  hash = sum over words k of word'_k * (fmix32(k) | 1)  (mod 2^64),
  with fmix32 the MurmurHash3 32-bit finaliser (Appleby), and the product of
  two 32-bit values taken exactly.
* ``classes``: rows with equal hashes form one class; every row is mapped to
  the lowest row of its class.

The reader here is this module's own; it accepts files whose inputs are
variables 1..n and whose AND gates define variables n+1..M in order (what
every generator in this repository writes, and what binary AIGER requires).
"""
import numpy as np


def read_aag(aag: bytes):
    """(n, ands [(lhs_var, rhs0, rhs1)], outputs) of a canonical latch-free ASCII AIGER file."""
    lines = aag.decode().split("\n")
    head = lines[0].split()
    if head[0] != "aag":
        raise ValueError("not ASCII AIGER")
    M, I, L, O, A = map(int, head[1:6])
    if L:
        raise ValueError("latches are not supported")
    for i in range(I):
        if int(lines[1 + i]) != 2 * (i + 1):
            raise ValueError("inputs must be variables 1..n in order")
    outputs = [int(lines[1 + I + j]) for j in range(O)]
    ands = []
    for k in range(A):
        lhs, r0, r1 = map(int, lines[1 + I + O + k].split())
        if lhs != 2 * (I + 1 + k):
            raise ValueError("AND gates must define variables n+1..M in order")
        if max(r0, r1) >= lhs:
            raise ValueError("an AND gate reads a variable not defined before it")
        ands.append((lhs >> 1, r0, r1))
    if M != I + A:
        raise ValueError("header M must equal I + A")
    return I, ands, outputs


def simulate(aag: bytes, pi_words: np.ndarray) -> np.ndarray:
    """uint32 array [M+1, W]: row v = value of variable v on the given input words."""
    n, ands, _ = read_aag(aag)
    pi = np.asarray(pi_words, dtype=np.uint32)
    if pi.ndim != 2 or pi.shape[0] != n:
        raise ValueError("pi_words must have one row per input")
    W = pi.shape[1]
    sig = np.zeros((n + 1 + len(ands), W), dtype=np.uint32)
    sig[1:n + 1] = pi
    full = np.uint32(0xFFFFFFFF)
    for v, r0, r1 in ands:
        a = sig[r0 >> 1] ^ (full if r0 & 1 else np.uint32(0))
        b = sig[r1 >> 1] ^ (full if r1 & 1 else np.uint32(0))
        sig[v] = a & b
    return sig


def literal_row(sig: np.ndarray, lit: int) -> np.ndarray:
    """Row of a literal: the variable's row, complemented for an odd literal."""
    row = sig[lit >> 1]
    return ~row if lit & 1 else row


def fmix32(x):
    """MurmurHash3's 32-bit finaliser on a uint32 scalar or array (wrapping arithmetic)."""
    h = np.asarray(x, dtype=np.uint32).copy()
    with np.errstate(over="ignore"):
        h ^= h >> np.uint32(16)
        h *= np.uint32(0x85EBCA6B)
        h ^= h >> np.uint32(13)
        h *= np.uint32(0xC2B2AE35)
        h ^= h >> np.uint32(16)
    return h


def hash_keys(W: int) -> np.ndarray:
    """Odd 32-bit key of each word position k (as uint64)."""
    return (fmix32(np.arange(W, dtype=np.uint32)) | np.uint32(1)).astype(np.uint64)


def signature_hash(sig: np.ndarray):
    """(hash uint64[rows], ones uint64[rows]) of every row of a signature matrix."""
    sig = np.asarray(sig, dtype=np.uint32)
    rows, W = sig.shape
    keys = hash_keys(W)
    pol = (sig[:, 0] & np.uint32(1)).astype(bool)
    norm = np.where(pol[:, None], ~sig, sig).astype(np.uint64)
    with np.errstate(over="ignore"):
        h = (norm * keys[None, :]).sum(axis=1, dtype=np.uint64)
    ones = np.bitwise_count(sig).sum(axis=1, dtype=np.uint64)
    return h, ones


def classes(hashes) -> np.ndarray:
    """uint32[rows]: the lowest row whose hash equals this row's hash."""
    first = {}
    out = np.empty(len(hashes), dtype=np.uint32)
    for r, h in enumerate(np.asarray(hashes, dtype=np.uint64).tolist()):
        out[r] = first.setdefault(h, r)
    return out
