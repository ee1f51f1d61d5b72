"""Plain CPU oracle for sub-miter extraction by virtual sweeping.

TEST INFRASTRUCTURE ONLY: the test suite is its only user; the library never
calls it.

The paper builds its training and scheduling units by simulating a sweeping
pass without proving anything: each target signal pair is cut out with only
its fan-in cones, and the nodes before it in topological order are merged as
if every earlier candidate pair had already been proven (Section 3.2, data
features preparation; the sweeping flow it imitates is Section 2.3).  This
module writes that definition out for a latch-free AIG with candidate classes
from simulation (oracle/rsim.py):

* class_of[u] is the representative of u (the lowest member of its class,
  class_of[u] <= u); polarity[u] is u's value at the first simulated pattern,
  so u and its representative are candidates for equality when their
  polarities agree and for complement when they differ;
* a target is an AND variable v that is not its class's representative; its
  pair is (v, r = class_of[v]) with phase ph = polarity[v] ^ polarity[r];
* merging: inside the sub-miter every literal 2u + c with u a
  non-representative AND is replaced by 2 class_of[u] + (c ^ polarity[u] ^
  polarity[class_of[u]]); the target's own gate is kept (with merged fan-ins);
* the sub-miter holds the AND gates reachable from v's merged fan-ins and from
  r, and asks whether v differs from r ^ ph: its one output is
  XOR(v, r ^ ph), written as three AND gates t1 = a & b, t2 = ~a & ~b,
  out = ~t1 & ~t2.

Text layout (deterministic): inputs are the original inputs in the support,
in ascending order, as variables 1..k; then the kept AND gates in ascending
original variable order; then t1, t2, out.  Header ``aag M k 0 1 A``, the
input lines, the output line ``2*out``, the AND lines ``lhs rhs0 rhs1`` with
the operands in the original gate's order.  No symbols, no comments.  A
constant representative (class 0) is the literal 0 or 1.
"""
from .rsim import read_aag


def targets(class_of, n: int):
    """AND variables that are not their class's representative, ascending."""
    return [v for v in range(n + 1, len(class_of)) if class_of[v] != v]


def submiter_aag(aag: bytes, class_of, polarity, target: int):
    """(sub-miter as ASCII AIGER bytes, list of original input indices of its inputs)."""
    n, ands, _ = read_aag(aag)
    fanins = {v: (r0, r1) for v, r0, r1 in ands}
    if target not in fanins or class_of[target] == target:
        raise ValueError("target must be an AND variable that is not its class representative")

    def merged(lit):
        u = lit >> 1
        if u in fanins and class_of[u] != u:
            r = class_of[u]
            return 2 * r + ((lit & 1) ^ polarity[u] ^ polarity[r])
        return lit

    rep = class_of[target]
    ph = polarity[target] ^ polarity[rep]
    top = [(target, merged(fanins[target][0]), merged(fanins[target][1]))]
    kept = {target: (top[0][1], top[0][2])}
    stack = [top[0][1] >> 1, top[0][2] >> 1, rep]
    support = set()
    while stack:
        u = stack.pop()
        if u == 0:
            continue
        if u not in fanins:
            support.add(u)
            continue
        if u in kept:
            continue
        a, b = merged(fanins[u][0]), merged(fanins[u][1])
        kept[u] = (a, b)
        stack += [a >> 1, b >> 1]
    inputs = sorted(support)
    new_var = {0: 0}
    for k, u in enumerate(inputs):
        new_var[u] = k + 1
    for u in sorted(kept):
        new_var[u] = len(new_var)

    def lit_of(lit):
        return 2 * new_var[lit >> 1] + (lit & 1)

    a = lit_of(2 * target)
    b = lit_of(2 * rep) ^ ph
    k = len(inputs)
    t1 = len(new_var)
    t2, out = t1 + 1, t1 + 2
    lines = [f"aag {out} {k} 0 1 {len(kept) + 3}"]
    lines += [str(2 * (i + 1)) for i in range(k)]
    lines.append(str(2 * out))
    for u in sorted(kept):
        x, y = kept[u]
        lines.append(f"{2 * new_var[u]} {lit_of(x)} {lit_of(y)}")
    lines.append(f"{2 * t1} {a} {b}")
    lines.append(f"{2 * t2} {a ^ 1} {b ^ 1}")
    lines.append(f"{2 * out} {2 * t1 + 1} {2 * t2 + 1}")
    # original input index of each sub-miter input (variable u is input u - 1)
    return ("\n".join(lines) + "\n").encode(), [u - 1 for u in inputs]
