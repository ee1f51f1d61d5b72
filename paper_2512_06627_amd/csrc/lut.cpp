// Mapping of the output cone onto gfx950's three-input LUT instruction, for the
// specialized kernel.  See LutProgram in plan.hpp.
#include <algorithm>
#include <functional>
#include <map>
#include <stdexcept>

#include "plan.hpp"

namespace fes {
namespace {

constexpr uint32_t kInputWord[5] = {0xAAAAAAAAu, 0xCCCCCCCCu, 0xF0F0F0F0u, 0xFF00FF00u, 0xFFFF0000u};

struct Val {  // value of an AIG variable: ref, complemented when neg
    LutRef ref;
    bool neg;
};

bool same(const LutRef& a, const LutRef& b) { return a.kind == b.kind && a.index == b.index; }

struct Cover {  // a LUT in construction: function `tt` of `leaves` (bit idx = sum leaf_j << (2 - j))
    std::vector<LutRef> leaves;
    uint8_t tt = 0;
    uint32_t gates = 0;
};

// Truth table (over the first k positions, position j = bit 2-j of the index) of leaf j.
uint8_t proj(uint32_t j) { return j == 0 ? 0xF0 : j == 1 ? 0xCC : 0xAA; }

// Re-express `sub` (over its own leaves) over the leaf list `L`.
uint8_t remap(const Cover& sub, const std::vector<LutRef>& L) {
    uint8_t out = 0;
    for (uint32_t idx = 0; idx < 8; ++idx) {
        uint32_t local = 0;
        for (uint32_t j = 0; j < sub.leaves.size(); ++j) {
            uint32_t pos = 0;
            while (!same(L[pos], sub.leaves[j])) ++pos;
            const uint32_t bit = (idx >> (2 - pos)) & 1u;
            local |= bit << (2 - j);
        }
        if ((sub.tt >> local) & 1u) out |= (uint8_t)(1u << idx);
    }
    return out;
}

}  // namespace

LutProgram make_lut_program(const Aig& g, const Plan& plan, int scalar_policy) {
    LutProgram lp;
    const uint32_t n = g.num_inputs, V = g.max_var();
    lp.num_inputs = n;
    auto word = [&](uint32_t w) {
        for (uint32_t i = 0; i < lp.words.size(); ++i)
            if (lp.words[i] == w) return LutRef{LutRef::Word, i};
        lp.words.push_back(w);
        return LutRef{LutRef::Word, (uint32_t)lp.words.size() - 1};
    };
    auto is_scalar_ref = [&](const LutRef& r) {
        return r.kind == LutRef::Word || r.kind == LutRef::Uniform || (r.kind == LutRef::Input && r.index >= 11);
    };
    // ---- 1. classify: plan-time words, wave-uniform values, varying gates ----------------
    // val[v] holds the value of every non-varying variable; varying gates keep their fanins.
    std::vector<Val> val(V + 1);
    std::vector<uint8_t> varying(V + 1, 0);
    val[0] = {word(0u), false};
    for (uint32_t i = 0; i < n; ++i)
        val[i + 1] = i < 5 ? Val{word(kInputWord[i]), false} : Val{LutRef{LutRef::Input, i}, false};
    for (uint32_t i = 5; i < n && i < 11; ++i) varying[i + 1] = 2;  // lane input: a varying leaf
    struct Pending {
        uint32_t var;
        LutRef a, b;
        bool na, nb;
    };
    std::vector<LutStep> scalar_at(V + 1);  // scalar step of a uniform gate, emitted in order later
    std::vector<uint8_t> has_scalar(V + 1, 0);
    for (uint32_t k : plan.order) {
        const uint32_t v = n + 1 + k, la = g.and_r0[k], lb = g.and_r1[k];
        const uint32_t va = la >> 1, vb = lb >> 1;
        if (varying[va] == 1 || varying[vb] == 1 || varying[va] == 2 || varying[vb] == 2) {
            // at least one varying fanin; constants still fold
            auto cw = [&](uint32_t var, uint32_t lit, uint32_t& w) {
                if (varying[var] || val[var].ref.kind != LutRef::Word) return false;
                w = lp.words[val[var].ref.index] ^ ((val[var].neg ^ (lit & 1)) ? ~0u : 0u);
                return true;
            };
            uint32_t w;
            if ((cw(va, la, w) && w == 0) || (cw(vb, lb, w) && w == 0)) {
                val[v] = {word(0u), false};
                lp.folded_gates++;
                continue;
            }
            varying[v] = 1;
            continue;
        }
        Val a = val[va], b = val[vb];
        a.neg ^= (la & 1) != 0;
        b.neg ^= (lb & 1) != 0;
        auto eff_word = [&](const Val& x, uint32_t& w) {
            if (x.ref.kind != LutRef::Word) return false;
            w = lp.words[x.ref.index] ^ (x.neg ? ~0u : 0u);
            return true;
        };
        uint32_t wa, wb;
        const bool ka = eff_word(a, wa), kb = eff_word(b, wb);
        if (ka && kb) { val[v] = {word(wa & wb), false}; lp.folded_gates++; continue; }
        if ((ka && wa == 0) || (kb && wb == 0)) { val[v] = {word(0u), false}; lp.folded_gates++; continue; }
        if (ka && wa == ~0u) { val[v] = b; lp.folded_gates++; continue; }
        if (kb && wb == ~0u) { val[v] = a; lp.folded_gates++; continue; }
        // Scalar-unit policy: a uniform gate may instead join the VALU LUT network, where it
        // can be absorbed into LUTs (balances the scalar and vector issue load).
        if (scalar_policy == 2 || (scalar_policy == 1 && (ka || kb))) {
            varying[v] = 1;
            continue;
        }
        LutStep st{};
        st.op = LutStep::ScalarAnd;
        st.leaf[0] = a.ref;
        st.leaf[1] = b.ref;
        st.table = (uint8_t)((a.neg ? 1 : 0) | (b.neg ? 2 : 0));
        st.dst = lp.num_values++;
        scalar_at[v] = st;
        has_scalar[v] = 1;
        val[v] = {LutRef{LutRef::Uniform, st.dst}, false};
    }
    // Leaf of a varying gate's fanin literal: a varying gate (cut-able), or a fixed ref.
    struct Leaf {
        bool node;      // true: varying gate `var`; false: fixed ref
        uint32_t var;
        LutRef ref;
        bool neg;
    };
    auto leaf_of = [&](uint32_t lit) {
        const uint32_t var = lit >> 1;
        Leaf l{};
        if (varying[var] == 1) {
            l.node = true;
            l.var = var;
            l.neg = (lit & 1) != 0;
        } else {
            l.node = false;
            l.ref = val[var].ref;
            l.neg = val[var].neg ^ ((lit & 1) != 0);
        }
        return l;
    };
    // ---- 2. three-input cuts of varying gates, chosen by area flow --------------------
    // A cut leaf is a varying gate or a fixed ref (input, word or uniform value); key
    // encodes both so leaf sets can be compared.
    auto key_node = [](uint32_t var) { return (uint64_t)var; };
    auto key_ref = [](const LutRef& r) { return (1ull << 40) | ((uint64_t)r.kind << 32) | r.index; };
    struct Cut {
        std::vector<uint64_t> keys;  // sorted leaf keys
        uint8_t tt;                  // over keys in order (position j = bit 2-j)
        double af;
    };
    std::vector<uint32_t> fanout(V + 1, 0);
    for (uint32_t k : plan.order) {
        ++fanout[g.and_r0[k] >> 1];
        ++fanout[g.and_r1[k] >> 1];
    }
    for (uint32_t o : g.outputs) ++fanout[o >> 1];
    std::vector<std::vector<Cut>> cuts(V + 1);
    std::vector<double> best_af(V + 1, 0.0);
    auto tt_remap = [](const Cut& c, const std::vector<uint64_t>& L) {
        uint8_t out = 0;
        for (uint32_t idx = 0; idx < 8; ++idx) {
            uint32_t local = 0;
            for (uint32_t j = 0; j < c.keys.size(); ++j) {
                const uint32_t pos = (uint32_t)(std::find(L.begin(), L.end(), c.keys[j]) - L.begin());
                local |= ((idx >> (2 - pos)) & 1u) << (2 - j);
            }
            if ((c.tt >> local) & 1u) out |= (uint8_t)(1u << idx);
        }
        return out;
    };
    auto trivial = [&](uint64_t key) { return Cut{{key}, 0xF0, 0.0}; };
    std::map<uint64_t, LutRef> ref_of_key;
    auto cuts_of = [&](const Leaf& l) -> std::vector<Cut> {
        if (l.node) {
            std::vector<Cut> cs = cuts[l.var];
            Cut t = trivial(key_node(l.var));
            t.af = best_af[l.var] / std::max<uint32_t>(1, fanout[l.var]);
            cs.push_back(t);
            return cs;
        }
        ref_of_key[key_ref(l.ref)] = l.ref;
        Cut t = trivial(key_ref(l.ref));
        t.af = is_scalar_ref(l.ref) ? 0.25 : 0.0;  // a second scalar leaf costs a copy
        return {t};
    };
    constexpr size_t kMaxCuts = 10;
    for (uint32_t k : plan.order) {
        const uint32_t v = n + 1 + k;
        if (varying[v] != 1) continue;
        const Leaf A = leaf_of(g.and_r0[k]), B = leaf_of(g.and_r1[k]);
        const std::vector<Cut> ca = cuts_of(A), cb = cuts_of(B);
        std::vector<Cut> out;
        for (const Cut& x : ca)
            for (const Cut& y : cb) {
                std::vector<uint64_t> L = x.keys;
                for (uint64_t q : y.keys)
                    if (std::find(L.begin(), L.end(), q) == L.end()) L.push_back(q);
                if (L.size() > 3) continue;
                std::sort(L.begin(), L.end());
                Cut c;
                c.keys = L;
                const uint8_t tx = (uint8_t)(tt_remap(x, L) ^ (A.neg ? 0xFF : 0x00));
                const uint8_t ty = (uint8_t)(tt_remap(y, L) ^ (B.neg ? 0xFF : 0x00));
                c.tt = (uint8_t)(tx & ty);
                // area flow: this LUT plus the shared cost of its gate leaves
                c.af = 1.0;
                int scalars = 0;
                for (uint64_t q : L) {
                    if (q < (1ull << 40)) c.af += best_af[(uint32_t)q] / std::max<uint32_t>(1, fanout[(uint32_t)q]);
                    else if (is_scalar_ref(ref_of_key[q])) ++scalars;
                }
                if (scalars > 1) c.af += 0.25 * (scalars - 1);
                bool dup = false;
                for (Cut& e : out)
                    if (e.keys == c.keys) {
                        dup = true;
                        if (c.af < e.af) e = c;
                    }
                if (!dup) out.push_back(c);
            }
        std::sort(out.begin(), out.end(), [](const Cut& a, const Cut& b) {
            return a.af != b.af ? a.af < b.af : a.keys.size() < b.keys.size();
        });
        if (out.size() > kMaxCuts) out.resize(kMaxCuts);
        cuts[v] = out;
        best_af[v] = out.empty() ? 1.0 : out[0].af;
    }
    // ---- 3. cover: gates needed by the outputs through their chosen cuts --------------
    // Area flow picks cuts[v][0]; exact-area recovery then revisits every gate of the cover
    // in topological order and keeps the cut that adds the fewest LUTs given the rest of
    // the cover (reference counts over the chosen cuts), two rounds.
    std::vector<uint32_t> sel(V + 1, 0), ref(V + 1, 0);
    std::function<uint32_t(uint32_t, const Cut&)> ref_cut, deref_cut;
    ref_cut = [&](uint32_t, const Cut& c) {
        uint32_t a = 1;
        for (uint64_t q : c.keys)
            if (q < (1ull << 40) && ref[(uint32_t)q]++ == 0) a += ref_cut((uint32_t)q, cuts[(uint32_t)q][sel[(uint32_t)q]]);
        return a;
    };
    deref_cut = [&](uint32_t, const Cut& c) {
        uint32_t a = 1;
        for (uint64_t q : c.keys)
            if (q < (1ull << 40) && --ref[(uint32_t)q] == 0) a += deref_cut((uint32_t)q, cuts[(uint32_t)q][sel[(uint32_t)q]]);
        return a;
    };
    for (uint32_t o : g.outputs) {
        const uint32_t v = o >> 1;
        if (varying[v] == 1 && ref[v]++ == 0) ref_cut(v, cuts[v][sel[v]]);
    }
    for (int round = 0; round < 2; ++round) {
        for (uint32_t k : plan.order) {
            const uint32_t v = n + 1 + k;
            if (varying[v] != 1 || ref[v] == 0) continue;
            deref_cut(v, cuts[v][sel[v]]);
            uint32_t best = sel[v], best_area = UINT32_MAX;
            for (uint32_t i = 0; i < cuts[v].size(); ++i) {
                const uint32_t a = ref_cut(v, cuts[v][i]);
                deref_cut(v, cuts[v][i]);
                if (a < best_area) {
                    best_area = a;
                    best = i;
                }
            }
            sel[v] = best;
            ref_cut(v, cuts[v][best]);
        }
    }
    std::vector<uint8_t> required(V + 1, 0);
    for (uint32_t v = 0; v <= V; ++v) required[v] = ref[v] > 0 && varying[v] == 1;
    // uniform values actually read (by required LUTs, by outputs or by other scalar steps)
    std::vector<uint8_t> scalar_needed(V + 1, 0);
    std::map<uint32_t, uint32_t> var_of_uniform;  // uniform value id -> AIG var
    for (uint32_t v = 0; v <= V; ++v)
        if (has_scalar[v]) var_of_uniform[scalar_at[v].dst] = v;
    std::vector<uint32_t> stack;
    auto need_ref = [&](const LutRef& r) {
        if (r.kind != LutRef::Uniform) return;
        const uint32_t v = var_of_uniform[r.index];
        if (!scalar_needed[v]) {
            scalar_needed[v] = 1;
            stack.push_back(v);
        }
    };
    for (uint32_t v = 0; v <= V; ++v)
        if (required[v])
            for (uint64_t q : cuts[v][sel[v]].keys)
                if (q >= (1ull << 40)) need_ref(ref_of_key[q]);
    for (uint32_t o : g.outputs)
        if (varying[o >> 1] != 1) need_ref(val[o >> 1].ref);
    while (!stack.empty()) {
        const uint32_t v = stack.back();
        stack.pop_back();
        need_ref(scalar_at[v].leaf[0]);
        need_ref(scalar_at[v].leaf[1]);
    }
    // ---- 4. emit in the plan's order ------------------------------------------------------
    // LUT steps follow the plan's order.  A scalar step is emitted just before its first
    // reader (after its own operands), so wave-uniform values stay live only as long as needed.
    std::vector<uint32_t> value_of_var(V + 1, UINT32_MAX);
    std::vector<uint8_t> scalar_done(V + 1, 0);
    std::function<void(const LutRef&)> ensure = [&](const LutRef& r) {
        if (r.kind != LutRef::Uniform) return;
        const uint32_t v = var_of_uniform[r.index];
        if (scalar_done[v]) return;
        scalar_done[v] = 1;
        ensure(scalar_at[v].leaf[0]);
        ensure(scalar_at[v].leaf[1]);
        lp.steps.push_back(scalar_at[v]);
        lp.scalar_steps++;
    };
    uint32_t total_varying = 0;
    for (uint32_t k : plan.order) {
        const uint32_t v = n + 1 + k;
        if (varying[v] == 1) ++total_varying;
        if (varying[v] != 1 || !required[v]) continue;
        const Cut& c = cuts[v][sel[v]];
        LutStep st{};
        st.op = LutStep::Lut;
        st.nleaves = (uint8_t)c.keys.size();
        for (uint32_t j = 0; j < 3; ++j) {
            const uint64_t q = c.keys[std::min<size_t>(j, c.keys.size() - 1)];
            st.leaf[j] = q < (1ull << 40) ? LutRef{LutRef::Varying, value_of_var[(uint32_t)q]} : ref_of_key[q];
        }
        for (uint32_t j = 0; j < st.nleaves; ++j) ensure(st.leaf[j]);
        st.table = c.tt;
        st.dst = lp.num_values++;
        value_of_var[v] = st.dst;
        lp.steps.push_back(st);
        lp.lut_steps++;
    }
    lp.absorbed_gates = total_varying - lp.lut_steps;
    for (uint32_t o : g.outputs) {
        const uint32_t var = o >> 1;
        LutStep st{};
        st.op = LutStep::Output;
        if (varying[var] != 1) ensure(val[var].ref);
        if (varying[var] == 1) {
            st.leaf[0] = LutRef{LutRef::Varying, value_of_var[var]};
            st.out_neg = (o & 1) != 0;
        } else {
            st.leaf[0] = val[var].ref;
            st.out_neg = val[var].neg ^ ((o & 1) != 0);
        }
        lp.steps.push_back(st);
    }
    return lp;
}

uint32_t eval_lut_program(const LutProgram& lp, uint64_t hw) {
    std::vector<uint32_t> vals(lp.num_values, 0);
    auto get = [&](const LutRef& r) -> uint32_t {
        switch (r.kind) {
            case LutRef::Word: return lp.words[r.index];
            case LutRef::Input: return 0u - (uint32_t)((hw >> (r.index - 5)) & 1u);
            default: return vals[r.index];
        }
    };
    uint32_t m = 0;
    for (const LutStep& st : lp.steps) {
        if (st.op == LutStep::Lut) {
            const uint32_t s0 = get(st.leaf[0]), s1 = get(st.leaf[1]), s2 = get(st.leaf[2]);
            uint32_t r = 0;
            for (uint32_t idx = 0; idx < 8; ++idx) {
                if (!((st.table >> idx) & 1u)) continue;
                r |= ((idx & 4) ? s0 : ~s0) & ((idx & 2) ? s1 : ~s1) & ((idx & 1) ? s2 : ~s2);
            }
            vals[st.dst] = r;
        } else if (st.op == LutStep::ScalarAnd) {
            const uint32_t a = get(st.leaf[0]) ^ ((st.table & 1) ? ~0u : 0u);
            const uint32_t b = get(st.leaf[1]) ^ ((st.table & 2) ? ~0u : 0u);
            vals[st.dst] = a & b;
        } else {
            m |= get(st.leaf[0]) ^ (st.out_neg ? ~0u : 0u);
        }
    }
    return m;
}

}  // namespace fes
