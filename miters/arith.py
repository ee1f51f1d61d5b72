"""Unsigned arithmetic circuits as AIGs (XOR = three ANDs).

Every builder takes an ``Aig`` and lists of input literals (LSB first) and
returns output literals (LSB first).  The paper does not say which multiplier
architectures its Table 1 miters compare; these are the textbook ones named
by the workloads: a row ripple-carry array multiplier, a Wallace-tree
multiplier (3:2 and 2:2 compressors per column, ripple-carry final adder) and
an unsigned radix-4 Booth multiplier whose partial products are reduced by a
Wallace tree.
"""
from .aig import Aig


def half_adder(g: Aig, a: int, b: int):
    """(a ^ b, a & b); the XOR is (a & ~b) | (~a & b), three ANDs."""
    return g.XOR_alt(a, b), g.AND(a, b)


def majority(g: Aig, a: int, b: int, c: int) -> int:
    """(a & b) | (a & c) | (b & c), five ANDs."""
    return g.OR(g.OR(g.AND(a, b), g.AND(a, c)), g.AND(b, c))


def full_adder(g: Aig, a: int, b: int, c: int):
    """(a ^ b ^ c, majority(a, b, c)): eleven ANDs when no input is constant."""
    return g.XOR_alt(g.XOR_alt(a, b), c), majority(g, a, b, c)


def ripple_add(g: Aig, xs: list, ys: list, width: int) -> list:
    """x + y truncated to ``width`` bits (missing bits are constant 0)."""
    out, carry = [], 0
    for k in range(width):
        x = xs[k] if k < len(xs) else 0
        y = ys[k] if k < len(ys) else 0
        s, carry = full_adder(g, x, y, carry)
        out.append(s)
    return out


def array_mult(g: Aig, a: list, b: list) -> list:
    """Row ripple-carry array multiplier: 2w-bit product of two w-bit operands."""
    w = len(a)
    assert len(b) == w and w >= 1
    acc = [0] * (2 * w)
    for j in range(w):
        acc[j] = g.AND(a[j], b[0])
    for i in range(1, w):
        carry = 0
        for j in range(w):
            col = i + j
            acc[col], carry = full_adder(g, acc[col], g.AND(a[j], b[i]), carry)
        acc[i + w] = carry
    return acc


def wallace_reduce(g: Aig, cols: list, width: int) -> list:
    """Wallace reduction of bit columns to two rows, then a ripple-carry adder.

    ``cols[k]`` is the list of literals of weight 2^k.  Each stage compresses
    every column in groups of three (full adder) and a leftover pair (half
    adder); sums stay in the column, carries move one column up.  Bits of
    weight 2^width and above are dropped (the result is taken mod 2^width).
    """
    cols = [list(c) for c in cols[:width]] + [[] for _ in range(max(0, width - len(cols)))]
    cols = [[x for x in c if x != 0] for c in cols]
    while max((len(c) for c in cols), default=0) > 2:
        nxt = [[] for _ in range(width)]
        for k, c in enumerate(cols):
            i = 0
            while len(c) - i >= 3:
                s, cy = full_adder(g, c[i], c[i + 1], c[i + 2])
                nxt[k].append(s)
                if k + 1 < width:
                    nxt[k + 1].append(cy)
                i += 3
            if len(c) - i == 2:
                s, cy = half_adder(g, c[i], c[i + 1])
                nxt[k].append(s)
                if k + 1 < width:
                    nxt[k + 1].append(cy)
            elif len(c) - i == 1:
                nxt[k].append(c[i])
        cols = [[x for x in c if x != 0] for c in nxt]
    row0 = [c[0] if len(c) > 0 else 0 for c in cols]
    row1 = [c[1] if len(c) > 1 else 0 for c in cols]
    return ripple_add(g, row0, row1, width)


def wallace_mult(g: Aig, a: list, b: list) -> list:
    """Wallace-tree multiplier over the w*w AND partial products."""
    w = len(a)
    assert len(b) == w and w >= 1
    cols = [[] for _ in range(2 * w)]
    for i in range(w):
        for j in range(w):
            cols[i + j].append(g.AND(a[j], b[i]))
    return wallace_reduce(g, cols, 2 * w)


def booth_columns(g: Aig, a: list, b: list, width: int) -> list:
    """Partial-product bit columns of an unsigned radix-4 Booth multiplication, mod 2^width.

    b is zero-extended; digit k (k = 0..floor(w/2)) is
    d_k = -2*b[2k+1] + b[2k] + b[2k-1] in {-2..2}, with b[-1] = b[>=w] = 0, and
    a*b = sum_k d_k * a * 4^k.  Digit k is encoded as neg = b[2k+1],
    one = b[2k] ^ b[2k-1], two = (b[2k+1] & ~b[2k] & ~b[2k-1]) | (~b[2k+1] & b[2k] & b[2k-1]).
    The magnitude m = |d_k| * a has w+1 bits m_j = one&a_j | two&a_{j-1}.
    The two's-complement partial product is U_k + neg_k - neg_k*2^(w+1), where
    U_k is the unsigned (w+1)-bit value of m ^ neg.  Using
    -neg*2^q = (~neg)*2^q - 2^q, the sign terms become the bits ~neg_k at
    weight 2^(w+1+2k) plus one constant, -sum_k 2^(w+1+2k) mod 2^width, whose
    set bits are added as constant-1 bits.
    """
    w = len(a)
    cols = [[] for _ in range(width)]

    def bit(vec, i):
        return vec[i] if 0 <= i < len(vec) else 0

    def put(k, lit):
        if 0 <= k < width and lit != 0:
            cols[k].append(lit)

    const = 0
    for k in range(w // 2 + 1):
        hi, mid, lo = bit(b, 2 * k + 1), bit(b, 2 * k), bit(b, 2 * k - 1)
        neg = hi
        one = g.XOR(mid, lo)
        two = g.OR(g.AND(hi, g.AND(mid ^ 1, lo ^ 1)), g.AND(hi ^ 1, g.AND(mid, lo)))
        for j in range(w + 1):
            m = g.OR(g.AND(one, bit(a, j)), g.AND(two, bit(a, j - 1)))
            put(2 * k + j, g.XOR(m, neg))
        put(2 * k, neg)
        put(w + 1 + 2 * k, neg ^ 1)
        const -= 1 << (w + 1 + 2 * k)
    const %= 1 << width
    for k in range(width):
        if (const >> k) & 1:
            put(k, 1)
    return cols


def booth_wallace_mult(g: Aig, a: list, b: list) -> list:
    """Unsigned radix-4 Booth multiplier, partial products reduced by a Wallace tree."""
    w = len(a)
    assert len(b) == w and w >= 1
    return wallace_reduce(g, booth_columns(g, a, b, 2 * w), 2 * w)


def mac_fused(g: Aig, a: list, b: list, c: list, d: list) -> list:
    """a*b + c*d with all 2*w*w partial products in one Wallace tree (2w+1 bits)."""
    w = len(a)
    width = 2 * w + 1
    cols = [[] for _ in range(width)]
    for x, y in ((a, b), (c, d)):
        for i in range(w):
            for j in range(w):
                cols[i + j].append(g.AND(x[j], y[i]))
    return wallace_reduce(g, cols, width)


def mac_separate(g: Aig, a: list, b: list, c: list, d: list) -> list:
    """a*b + c*d as two array multipliers and a (2w+1)-bit ripple-carry adder."""
    w = len(a)
    return ripple_add(g, array_mult(g, a, b), array_mult(g, c, d), 2 * w + 1)
