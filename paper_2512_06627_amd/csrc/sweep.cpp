// Sub-miter extraction by virtual sweeping (host side of the library).
//
// The paper cuts its scheduling units out of a miter by imitating one sweeping
// pass without proving anything: each candidate pair keeps only the fan-in
// cones of its two nodes, and every node before it is merged into its class
// representative as if all earlier pairs were already proven (Section 3.2,
// data features preparation; the sweeping flow is Section 2.3).  The classes
// come from random-pattern simulation (class_of = lowest member of a class,
// polarity = the value at the first simulated pattern).
//
// Rules, for target v (an AND variable with class_of[v] < v) and its
// representative r = class_of[v]:
//  * a literal 2u + c with u a non-representative AND variable is read as
//    2 class_of[u] + (c ^ polarity[u] ^ polarity[class_of[u]]); v's own gate
//    is kept with its fan-ins read that way;
//  * the kept gates are those reachable from v's read fan-ins and from r;
//  * the output is XOR(v, r ^ (polarity[v] ^ polarity[r])) as three AND gates
//    t1 = a & b, t2 = ~a & ~b, out = ~t1 & ~t2.
// Layout: the support inputs in ascending order are variables 1..k, then the
// kept gates in ascending original order, then t1, t2, out; operands keep the
// original gate's order.  The text is ASCII AIGER with no symbols.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "runtime.hpp"

namespace fes {

std::string submiter_aag(const Aig& g, const uint32_t* class_of, const uint8_t* polarity, uint64_t rows,
                         uint32_t target, std::vector<uint32_t>* inputs) {
    const uint32_t n = g.num_inputs, V = g.max_var();
    if (rows != (uint64_t)V + 1) throw Error{kErrInvalid, "class map must have max_var + 1 entries"};
    if (target <= n || target > V) throw Error{kErrInvalid, "target must be an AND variable"};
    if (class_of[target] >= target) throw Error{kErrInvalid, "target is its class's representative"};
    auto is_and = [&](uint32_t u) { return u > n && u <= V; };
    auto pol = [&](uint32_t u) -> uint32_t {
        if (polarity[u] > 1) throw Error{kErrInvalid, "polarity entries must be 0 or 1"};
        return polarity[u];
    };
    auto read = [&](uint32_t lit) -> uint32_t {
        const uint32_t u = lit >> 1;
        if (!is_and(u) || class_of[u] == u) return lit;
        const uint32_t r = class_of[u];
        if (r > u) throw Error{kErrInvalid, "class representative above its member"};
        return 2 * r + ((lit & 1) ^ pol(u) ^ pol(r));
    };
    const uint32_t rep = class_of[target];
    const uint32_t ph = pol(target) ^ pol(rep);
    // kept gates and their read fan-ins, by original variable
    std::vector<uint8_t> kept(V + 1, 0), in_support(n + 1, 0);
    std::vector<uint32_t> fa(V + 1, 0), fb(V + 1, 0);
    std::vector<uint32_t> stack;
    auto keep = [&](uint32_t u) {
        const uint32_t k = u - n - 1;
        kept[u] = 1;
        fa[u] = read(g.and_r0[k]);
        fb[u] = read(g.and_r1[k]);
        stack.push_back(fa[u] >> 1);
        stack.push_back(fb[u] >> 1);
    };
    keep(target);
    stack.push_back(rep);
    while (!stack.empty()) {
        const uint32_t u = stack.back();
        stack.pop_back();
        if (u == 0) continue;
        if (!is_and(u)) {
            in_support[u] = 1;
            continue;
        }
        if (!kept[u]) keep(u);
    }
    std::vector<uint32_t> new_var(V + 1, 0);
    uint32_t next = 1;
    if (inputs) inputs->clear();
    for (uint32_t u = 1; u <= n; ++u)
        if (in_support[u]) {
            new_var[u] = next++;
            if (inputs) inputs->push_back(u - 1);
        }
    const uint32_t k = next - 1;
    uint32_t num_kept = 0;
    for (uint32_t u = n + 1; u <= V; ++u)
        if (kept[u]) {
            new_var[u] = next++;
            ++num_kept;
        }
    auto lit_of = [&](uint32_t lit) { return 2 * new_var[lit >> 1] + (lit & 1); };
    const uint32_t a = lit_of(2 * target), b = lit_of(2 * rep) ^ ph;
    const uint32_t t1 = next, t2 = next + 1, out = next + 2;
    std::string s;
    s.reserve(16 * (num_kept + k + 8));
    s += "aag " + std::to_string(out) + " " + std::to_string(k) + " 0 1 " + std::to_string(num_kept + 3) + "\n";
    for (uint32_t i = 1; i <= k; ++i) s += std::to_string(2 * i) + "\n";
    s += std::to_string(2 * out) + "\n";
    auto line = [&](uint32_t lhs, uint32_t x, uint32_t y) {
        s += std::to_string(lhs) + " " + std::to_string(x) + " " + std::to_string(y) + "\n";
    };
    for (uint32_t u = n + 1; u <= V; ++u)
        if (kept[u]) line(2 * new_var[u], lit_of(fa[u]), lit_of(fb[u]));
    line(2 * t1, a, b);
    line(2 * t2, a ^ 1, b ^ 1);
    line(2 * out, 2 * t1 + 1, 2 * t2 + 1);
    return s;
}

}  // namespace fes
