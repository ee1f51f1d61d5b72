#include "plan.hpp"

#include <algorithm>
#include <functional>
#include <queue>
#include <string>

namespace fes {
namespace {

struct Cone {
    std::vector<uint8_t> in;      // per AND index
    std::vector<uint32_t> level;  // per var
    std::vector<uint32_t> label;  // per var: slots needed to evaluate a var's cone as a tree
};

inline bool is_and(const Aig& g, uint32_t var) { return var > g.num_inputs; }
inline uint32_t and_index(const Aig& g, uint32_t var) { return var - g.num_inputs - 1; }

Cone cone_of(const Aig& g) {
    Cone c;
    const uint32_t A = g.num_ands();
    c.in.assign(A, 0);
    std::vector<uint32_t> stack;
    for (uint32_t o : g.outputs)
        if (is_and(g, o >> 1)) stack.push_back(o >> 1);
    while (!stack.empty()) {
        uint32_t v = stack.back();
        stack.pop_back();
        uint32_t k = and_index(g, v);
        if (c.in[k]) continue;
        c.in[k] = 1;
        for (uint32_t f : {g.and_r0[k] >> 1, g.and_r1[k] >> 1})
            if (is_and(g, f)) stack.push_back(f);
    }
    c.level.assign(g.max_var() + 1, 0);
    c.label.assign(g.max_var() + 1, 0);
    for (uint32_t k = 0; k < A; ++k) {  // topological index order
        uint32_t v = g.num_inputs + 1 + k, a = g.and_r0[k] >> 1, b = g.and_r1[k] >> 1;
        c.level[v] = 1 + std::max(c.level[a], c.level[b]);
        uint32_t la = c.label[a], lb = c.label[b];
        c.label[v] = la == lb ? la + 1 : std::max(la, lb);
    }
    return c;
}

// Post-order DFS from the outputs; `first_child` picks which fanin to descend into first.
std::vector<uint32_t> dfs_order(const Aig& g, const Cone& c, bool by_label) {
    std::vector<uint32_t> order;
    std::vector<uint8_t> done(g.num_ands(), 0);
    std::vector<std::pair<uint32_t, uint8_t>> stack;  // (var, children pushed)
    for (uint32_t o : g.outputs) {
        uint32_t root = o >> 1;
        if (!is_and(g, root) || done[and_index(g, root)]) continue;
        stack.push_back({root, 0});
        while (!stack.empty()) {
            auto& top = stack.back();
            uint32_t v = top.first, k = and_index(g, v);
            if (done[k]) {
                stack.pop_back();
                continue;
            }
            if (top.second == 0) {
                top.second = 1;
                uint32_t a = g.and_r0[k] >> 1, b = g.and_r1[k] >> 1;
                uint32_t first = a, second = b;
                if (by_label && c.label[b] > c.label[a]) std::swap(first, second);
                // Push the second child below the first so the first is evaluated first.
                if (is_and(g, second) && !done[and_index(g, second)]) stack.push_back({second, 0});
                if (is_and(g, first) && !done[and_index(g, first)]) stack.push_back({first, 0});
                continue;
            }
            done[k] = 1;
            order.push_back(k);
            stack.pop_back();
        }
    }
    return order;
}

struct Alloc {
    std::vector<Instr> prog;
    uint32_t slots = 0;
    uint32_t gates = 0;
};

// Group an order into bundles of independent gates by list scheduling: a gate is ready when
// its AND fanins were computed in an earlier bundle; each bundle takes up to `B` ready gates
// in order of their position in `order`.
std::vector<std::vector<uint32_t>> bundle_order(const Aig& g, const std::vector<uint32_t>& order, uint32_t B) {
    std::vector<std::vector<uint32_t>> bundles;
    if (B <= 1) {
        for (uint32_t k : order) bundles.push_back({k});
        return bundles;
    }
    const uint32_t A = g.num_ands();
    std::vector<uint32_t> pos(A, UINT32_MAX), missing(A, 0);
    for (uint32_t i = 0; i < order.size(); ++i) pos[order[i]] = i;
    std::vector<std::vector<uint32_t>> users(A);
    for (uint32_t k : order)
        for (uint32_t f : {g.and_r0[k] >> 1, g.and_r1[k] >> 1})
            if (is_and(g, f)) {
                ++missing[k];
                users[and_index(g, f)].push_back(k);
            }
    std::priority_queue<uint32_t, std::vector<uint32_t>, std::greater<uint32_t>> ready;  // by position
    for (uint32_t k : order)
        if (missing[k] == 0) ready.push(pos[k]);
    size_t emitted = 0;
    while (emitted < order.size()) {
        std::vector<uint32_t> b;
        while (b.size() < B && !ready.empty()) {
            b.push_back(order[ready.top()]);
            ready.pop();
        }
        for (uint32_t k : b)
            for (uint32_t u : users[k])
                if (--missing[u] == 0) ready.push(pos[u]);
        emitted += b.size();
        bundles.push_back(std::move(b));
    }
    return bundles;
}

Alloc allocate(const Aig& g, const std::vector<std::vector<uint32_t>>& bundles, uint32_t B) {
    const uint32_t n = g.num_inputs, V = g.max_var();
    std::vector<uint32_t> rc(V + 1, 0), pos_refs(V + 1, 0), neg_refs(V + 1, 0), slot(V + 1, UINT32_MAX);
    for (auto& b : bundles)
        for (uint32_t k : b) {
            ++rc[g.and_r0[k] >> 1];
            ++rc[g.and_r1[k] >> 1];
        }
    for (uint32_t o : g.outputs) {
        ++rc[o >> 1];
        (o & 1 ? neg_refs : pos_refs)[o >> 1]++;
    }
    std::priority_queue<uint32_t, std::vector<uint32_t>, std::greater<uint32_t>> free_slots;
    Alloc al;
    auto row_of = [&](uint32_t var) { return is_and(g, var) ? n + 1 + slot[var] : var; };
    auto release = [&](uint32_t var) {
        if (is_and(g, var) && --rc[var] == 0) free_slots.push(slot[var]);
    };
    const Instr nop = {0u, 0u, UINT32_MAX, 0u};
    for (auto& b : bundles) {
        size_t first = al.prog.size();
        // Operands are read before any result of the bundle is written, so the slots whose
        // last reader is in this bundle are free for the bundle's own results.
        for (uint32_t k : b) {
            uint32_t a = g.and_r0[k], c = g.and_r1[k];
            Instr ins;
            ins.a = row_of(a >> 1) | ((a & 1) ? kCompl : 0u);
            ins.b = row_of(c >> 1) | ((c & 1) ? kCompl : 0u);
            ins.d = 0;
            ins.flags = 0;
            al.prog.push_back(ins);
        }
        for (uint32_t k : b) {
            release(g.and_r0[k] >> 1);
            release(g.and_r1[k] >> 1);
        }
        for (size_t t = 0; t < b.size(); ++t) {
            uint32_t v = n + 1 + b[t];
            if (free_slots.empty()) {
                slot[v] = al.slots++;
            } else {
                slot[v] = free_slots.top();
                free_slots.pop();
            }
            Instr& ins = al.prog[first + t];
            ins.d = n + 1 + slot[v];
            ins.flags = (pos_refs[v] ? kOutPos : 0u) | (neg_refs[v] ? kOutNeg : 0u) | (g.is_xor(b[t]) ? kXor : 0u);
        }
        for (uint32_t k : b) {
            uint32_t v = n + 1 + k;
            rc[v] -= pos_refs[v] + neg_refs[v];
            if (rc[v] == 0) free_slots.push(slot[v]);
        }
        al.gates += (uint32_t)b.size();
        while ((al.prog.size() - first) % B) al.prog.push_back(nop);
    }
    // Outputs driven by a constant or a primary input: value AND true, into the sink row.
    size_t first = al.prog.size();
    for (uint32_t o : g.outputs) {
        if (is_and(g, o >> 1)) continue;
        Instr ins;
        ins.a = (o >> 1) | ((o & 1) ? kCompl : 0u);
        ins.b = 0u | kCompl;
        ins.d = UINT32_MAX;
        ins.flags = kOutPos;
        al.prog.push_back(ins);
        ++al.gates;
    }
    while ((al.prog.size() - first) % B) al.prog.push_back(nop);
    for (Instr& ins : al.prog)
        if (ins.d == UINT32_MAX) ins.d = n + 1 + al.slots;  // sink row
    return al;
}

}  // namespace

Aig fuse_xors(const Aig& g) {
    const uint32_t A = g.num_ands();
    std::vector<uint32_t> readers(g.max_var() + 1, 0);
    for (uint32_t k = 0; k < A; ++k) {
        ++readers[g.and_r0[k] >> 1];
        ++readers[g.and_r1[k] >> 1];
    }
    for (uint32_t o : g.outputs) ++readers[o >> 1];
    Aig f = g;
    f.xor_gate.assign(A, 0);
    std::vector<uint8_t> absorbed(A, 0);
    for (uint32_t k = 0; k < A; ++k) {
        const uint32_t l1 = g.and_r0[k], l2 = g.and_r1[k];
        if (!(l1 & 1) || !(l2 & 1)) continue;  // both fanins complemented
        const uint32_t t1 = l1 >> 1, t2 = l2 >> 1;
        if (t1 == t2 || !is_and(g, t1) || !is_and(g, t2) || readers[t1] != 1 || readers[t2] != 1) continue;
        const uint32_t k1 = and_index(g, t1), k2 = and_index(g, t2);
        if (f.xor_gate[k1] || f.xor_gate[k2] || absorbed[k1] || absorbed[k2]) continue;
        const uint32_t x = g.and_r0[k1], y = g.and_r1[k1];
        const uint32_t p = g.and_r0[k2], q = g.and_r1[k2];
        if (!((p == (x ^ 1u) && q == (y ^ 1u)) || (p == (y ^ 1u) && q == (x ^ 1u)))) continue;
        if ((x >> 1) == (y >> 1)) continue;  // x & ~x: leave constant gates to the AND path
        f.and_r0[k] = x;
        f.and_r1[k] = y;
        f.xor_gate[k] = 1;
        absorbed[k1] = absorbed[k2] = 1;
    }
    return f;
}

Plan make_plan(const Aig& g, Order order, uint32_t bundle) {
    if (bundle == 0) bundle = 1;
    Cone c = cone_of(g);
    Plan p;
    p.num_inputs = g.num_inputs;
    p.num_ands_file = g.num_ands();
    p.num_outputs = (uint32_t)g.outputs.size();
    for (uint32_t k = 0; k < g.num_ands(); ++k) p.num_ands_tfi += c.in[k];
    for (uint32_t o : g.outputs) p.levels = std::max(p.levels, c.level[o >> 1]);

    std::vector<std::pair<Order, std::vector<uint32_t>>> cands;
    if (order == Order::Auto || order == Order::DfsLabel) cands.push_back({Order::DfsLabel, dfs_order(g, c, true)});
    if (order == Order::Auto || order == Order::DfsFanin0) cands.push_back({Order::DfsFanin0, dfs_order(g, c, false)});
    if (order == Order::Auto || order == Order::File) {
        std::vector<uint32_t> file;
        for (uint32_t k = 0; k < g.num_ands(); ++k)
            if (c.in[k]) file.push_back(k);
        cands.push_back({Order::File, std::move(file)});
    }
    bool have = false;
    for (auto& cand : cands) {
        Alloc al = allocate(g, bundle_order(g, cand.second, bundle), bundle);
        if (!have || al.slots < p.peak_slots) {
            have = true;
            p.peak_slots = al.slots;
            p.prog = std::move(al.prog);
            p.num_gate_instrs = al.gates;
            p.order_used = cand.first;
            p.order.clear();
            for (auto& b : bundle_order(g, cand.second, bundle))
                for (uint32_t k : b) p.order.push_back(k);
        }
    }
    p.bundle = bundle;
    p.rows = g.num_inputs + p.peak_slots + 2;
    // Gate instructions write a slot row and appear in the stream in evaluation order;
    // padding and output-only steps write the sink row.
    const uint32_t sink = g.num_inputs + 1 + p.peak_slots;
    p.instr_gate.assign(p.prog.size(), UINT32_MAX);
    size_t next = 0;
    for (size_t t = 0; t < p.prog.size(); ++t)
        if (p.prog[t].d != sink) p.instr_gate[t] = p.order[next++];
    if (next != p.order.size()) throw Error{kErrInvalid, "planner: gate instructions do not match the order"};
    return p;
}

std::string validate_plan(const Aig& g, const Plan& p) {
    // Symbolic replay of the stream.  holds[row] is the variable a row holds.  Within a
    // bundle all operands are resolved first, then all results are written; a result may
    // only overwrite a row whose value has no reads left once the bundle's reads are done.
    const uint32_t n = g.num_inputs, V = g.max_var(), sink = n + 1 + p.peak_slots;
    if (p.bundle == 0 || p.prog.size() % p.bundle) return "stream is not a whole number of bundles";
    std::vector<int64_t> holds(p.rows, -1);
    holds[0] = 0;
    for (uint32_t i = 1; i <= n; ++i) holds[i] = i;
    std::vector<std::vector<uint32_t>> by_fanin0(V + 1);
    for (uint32_t k = 0; k < g.num_ands(); ++k) by_fanin0[g.and_r0[k] >> 1].push_back(k);
    std::vector<uint32_t> reads(V + 1, 0);
    std::vector<uint8_t> in_cone(g.num_ands(), 0);
    {  // cone of the outputs and its read counts
        std::vector<uint32_t> st;
        for (uint32_t o : g.outputs) {
            ++reads[o >> 1];
            if (is_and(g, o >> 1)) st.push_back(o >> 1);
        }
        while (!st.empty()) {
            uint32_t k = and_index(g, st.back());
            st.pop_back();
            if (in_cone[k]) continue;
            in_cone[k] = 1;
            for (uint32_t f : {g.and_r0[k] >> 1, g.and_r1[k] >> 1}) {
                ++reads[f];
                if (is_and(g, f)) st.push_back(f);
            }
        }
    }
    std::vector<uint8_t> done(g.num_ands(), 0);
    std::vector<uint8_t> out_only_done(g.outputs.size(), 0);
    for (size_t b0 = 0; b0 < p.prog.size(); b0 += p.bundle) {
        struct Step { uint32_t la, lb, d, flags; int64_t gate; };
        std::vector<Step> steps;
        for (size_t t = b0; t < b0 + p.bundle; ++t) {
            const Instr& ins = p.prog[t];
            uint32_t ra = ins.a & kRowMask, rb = ins.b & kRowMask;
            if (ra >= p.rows || rb >= p.rows || ins.d >= p.rows) return "row out of range at " + std::to_string(t);
            if (holds[ra] < 0 || holds[rb] < 0) return "read of an empty row at " + std::to_string(t);
            Step s{2 * (uint32_t)holds[ra] + ((ins.a & kCompl) ? 1u : 0u),
                   2 * (uint32_t)holds[rb] + ((ins.b & kCompl) ? 1u : 0u), ins.d, ins.flags, -1};
            if (ins.d == sink) {
                if (ins.flags == 0) continue;  // padding
                bool found = false;
                for (size_t j = 0; j < g.outputs.size(); ++j)
                    if (g.outputs[j] == s.la && !is_and(g, s.la >> 1) && !out_only_done[j]) {
                        out_only_done[j] = 1;
                        found = true;
                        break;
                    }
                if (!found || s.lb != 1 || ins.flags != kOutPos) return "bad output-only step at " + std::to_string(t);
                --reads[s.la >> 1];
                continue;
            }
            for (uint32_t k : by_fanin0[s.la >> 1])
                if (!done[k] && in_cone[k] && g.and_r0[k] == s.la && g.and_r1[k] == s.lb &&
                    ((ins.flags & kXor) != 0) == g.is_xor(k)) {
                    bool taken = false;
                    for (auto& o : steps) taken |= o.gate == (int64_t)k;
                    if (!taken) { s.gate = k; break; }
                }
            if (s.gate < 0) return "instruction " + std::to_string(t) + " computes no pending cone gate";
            steps.push_back(s);
        }
        for (auto& s : steps) {
            --reads[s.la >> 1];
            --reads[s.lb >> 1];
        }
        for (size_t i = 0; i < steps.size(); ++i) {
            auto& s = steps[i];
            if (s.d <= n) return "write into a constant or input row";
            for (size_t j = 0; j < i; ++j)
                if (steps[j].d == s.d) return "two results of one bundle share a row";
            int64_t prev = holds[s.d];
            if (prev > (int64_t)n && reads[prev] != 0) return "live value overwritten";
        }
        for (auto& s : steps) {
            uint32_t v = n + 1 + (uint32_t)s.gate;
            holds[s.d] = v;
            done[s.gate] = 1;
            uint32_t want = 0;
            for (uint32_t o : g.outputs)
                if ((o >> 1) == v) {
                    want |= (o & 1) ? kOutNeg : kOutPos;
                    --reads[v];
                }
            if ((s.flags & ~kXor) != want) return "output flags wrong";
        }
    }
    for (uint32_t k = 0; k < g.num_ands(); ++k)
        if (in_cone[k] && !done[k]) return "cone gate never computed";
    for (size_t j = 0; j < g.outputs.size(); ++j)
        if (!is_and(g, g.outputs[j] >> 1) && !out_only_done[j]) return "output-only step missing";
    for (uint32_t v = 0; v <= V; ++v)
        if (reads[v] != 0) return "unbalanced reads of variable " + std::to_string(v);
    return "";
}

}  // namespace fes
