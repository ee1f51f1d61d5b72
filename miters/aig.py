"""AIG construction with structural hashing, and AIGER serialisation.

Literal convention (AIGER): ``lit = 2*var + c``; var 0 is constant false, so
literal 0 is false and literal 1 is true; primary input i is var ``i + 1``;
AND gates follow the inputs in creation order, which is a topological order.
"""


class Aig:
    """A latch-free AIG built gate by gate.

    ``AND`` folds constants and trivial cases (x&x, x&~x) and merges
    structurally identical gates, the usual construction-time rules; it never
    evaluates the circuit.
    """

    def __init__(self, num_inputs: int):
        self.num_inputs = num_inputs
        self.ands = []        # (rhs0, rhs1) for var num_inputs + 1 + index, rhs0 >= rhs1
        self.outputs = []     # output literals
        self._strash = {}

    # ---- construction -------------------------------------------------
    def input(self, i: int) -> int:
        if not 0 <= i < self.num_inputs:
            raise IndexError(i)
        return 2 * (i + 1)

    def inputs(self, lo: int, count: int) -> list:
        return [self.input(lo + k) for k in range(count)]

    @property
    def max_var(self) -> int:
        return self.num_inputs + len(self.ands)

    def AND(self, a: int, b: int) -> int:
        if a > b:
            a, b = b, a
        if a == 0:
            return 0
        if a == 1:
            return b
        if a == b:
            return a
        if a ^ 1 == b:
            return 0
        key = (a, b)
        lit = self._strash.get(key)
        if lit is None:
            lit = 2 * (self.num_inputs + 1 + len(self.ands))
            self.ands.append((b, a))
            self._strash[key] = lit
        return lit

    def OR(self, a: int, b: int) -> int:
        return self.AND(a ^ 1, b ^ 1) ^ 1

    def XOR(self, a: int, b: int) -> int:
        """XOR as three ANDs: ~(a&b) & ~(~a&~b); a&b is shared with a half adder's carry."""
        return self.AND(self.AND(a, b) ^ 1, self.AND(a ^ 1, b ^ 1) ^ 1)

    def XOR_alt(self, a: int, b: int) -> int:
        """XOR as three ANDs in the other common form: (a&~b) | (~a&b)."""
        return self.OR(self.AND(a, b ^ 1), self.AND(a ^ 1, b))

    def XOR_andor(self, a: int, b: int) -> int:
        """XOR as (a|b) & ~(a&b)."""
        return self.AND(self.OR(a, b), self.AND(a, b) ^ 1)

    def MUX(self, s: int, t: int, e: int) -> int:
        """s ? t : e."""
        return self.OR(self.AND(s, t), self.AND(s ^ 1, e))

    def add_output(self, lit: int) -> None:
        self.outputs.append(lit)

    # ---- queries ------------------------------------------------------
    def num_ands(self) -> int:
        return len(self.ands)

    def tfi_ands(self, roots=None) -> list:
        """Indices of AND gates in the transitive fan-in of ``roots`` (default: all outputs)."""
        roots = self.outputs if roots is None else roots
        first = self.num_inputs + 1
        seen = set()
        stack = [r >> 1 for r in roots]
        while stack:
            v = stack.pop()
            if v < first or v in seen:
                continue
            seen.add(v)
            r0, r1 = self.ands[v - first]
            stack.append(r0 >> 1)
            stack.append(r1 >> 1)
        return sorted(v - first for v in seen)

    # ---- AIGER --------------------------------------------------------
    def to_aag(self, symbols: bool = True, comment: str = "") -> bytes:
        """AIGER ASCII format: header ``aag M I L O A``, then inputs, outputs, AND lines."""
        lines = [f"aag {self.max_var} {self.num_inputs} 0 {len(self.outputs)} {len(self.ands)}"]
        lines += [str(self.input(i)) for i in range(self.num_inputs)]
        lines += [str(o) for o in self.outputs]
        first = self.num_inputs + 1
        for k, (r0, r1) in enumerate(self.ands):
            lines.append(f"{2 * (first + k)} {r0} {r1}")
        if symbols:
            lines += [f"i{i} x{i}" for i in range(self.num_inputs)]
            lines += [f"o{j} y{j}" for j in range(len(self.outputs))]
        if comment:
            lines.append("c")
            lines.append(comment)
        return ("\n".join(lines) + "\n").encode()

    def to_aig(self, symbols: bool = True, comment: str = "") -> bytes:
        """AIGER binary format: text header and outputs, then delta-encoded AND gates."""
        head = [f"aig {self.max_var} {self.num_inputs} 0 {len(self.outputs)} {len(self.ands)}"]
        head += [str(o) for o in self.outputs]
        out = bytearray(("\n".join(head) + "\n").encode())
        first = self.num_inputs + 1
        for k, (r0, r1) in enumerate(self.ands):
            lhs = 2 * (first + k)
            _put_varint(out, lhs - r0)
            _put_varint(out, r0 - r1)
        tail = []
        if symbols:
            tail += [f"i{i} x{i}" for i in range(self.num_inputs)]
            tail += [f"o{j} y{j}" for j in range(len(self.outputs))]
        if comment:
            tail.append("c")
            tail.append(comment)
        if tail:
            out += ("\n".join(tail) + "\n").encode()
        return bytes(out)


def _put_varint(buf: bytearray, x: int) -> None:
    if x <= 0:
        raise ValueError("AIGER binary deltas must be positive")
    while x & ~0x7F:
        buf.append((x & 0x7F) | 0x80)
        x >>= 7
    buf.append(x)


def import_into(dst: Aig, src: Aig, input_lits=None) -> list:
    """Copy ``src``'s gates into ``dst`` (re-hashed) and return ``src``'s outputs as ``dst`` literals.

    ``input_lits[i]`` is the ``dst`` literal that drives ``src`` input i
    (default: the same-numbered input of ``dst``).
    """
    if input_lits is None:
        input_lits = [dst.input(i) for i in range(src.num_inputs)]
    lit_of = [0] * (src.max_var + 1)
    for i in range(src.num_inputs):
        lit_of[i + 1] = input_lits[i]

    def m(lit):
        return lit_of[lit >> 1] ^ (lit & 1)

    first = src.num_inputs + 1
    for k, (r0, r1) in enumerate(src.ands):
        lit_of[first + k] = dst.AND(m(r0), m(r1))
    return [m(o) for o in src.outputs]
