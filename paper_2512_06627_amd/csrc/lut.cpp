// Mapping of the output cone onto gfx950's three-input LUT instruction, for the
// specialized kernel.  See LutProgram in plan.hpp.
#include <algorithm>
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

LutProgram make_lut_program(const Aig& g, const Plan& plan) {
    LutProgram lp;
    const uint32_t n = g.num_inputs, V = g.max_var();
    lp.num_inputs = n;
    std::vector<Val> val(V + 1);
    auto word = [&](uint32_t w) {
        for (uint32_t i = 0; i < lp.words.size(); ++i)
            if (lp.words[i] == w) return LutRef{LutRef::Word, i};
        lp.words.push_back(w);
        return LutRef{LutRef::Word, (uint32_t)lp.words.size() - 1};
    };
    val[0] = {word(0u), false};
    for (uint32_t i = 0; i < n; ++i) {
        const uint32_t v = i + 1;
        if (i < 5) val[v] = {word(kInputWord[i]), false};
        else if (i < 11) val[v] = {LutRef{LutRef::Input, i}, false};
        else val[v] = {LutRef{LutRef::Input, i}, false};
    }
    auto is_uniform_ref = [&](const LutRef& r) {
        return r.kind == LutRef::Word || r.kind == LutRef::Uniform || (r.kind == LutRef::Input && r.index >= 11);
    };
    // fan-out inside the cone, outputs included
    std::vector<uint32_t> fanout(V + 1, 0);
    for (uint32_t k : plan.order) {
        ++fanout[g.and_r0[k] >> 1];
        ++fanout[g.and_r1[k] >> 1];
    }
    std::vector<uint8_t> is_output(V + 1, 0);
    for (uint32_t o : g.outputs) {
        ++fanout[o >> 1];
        is_output[o >> 1] = 1;
    }
    // Varying AND gates not yet emitted, with their cover.
    std::vector<Cover> cover(V + 1);
    std::vector<uint8_t> pending(V + 1, 0);
    std::vector<uint32_t> node_of_value;  // varying value id -> AIG var (for diagnostics)
    auto emit = [&](uint32_t var) {  // emit a pending varying gate as its own LUT step
        const Cover& c = cover[var];
        LutStep st{};
        st.op = LutStep::Lut;
        st.nleaves = (uint8_t)c.leaves.size();
        for (uint32_t j = 0; j < 3; ++j) st.leaf[j] = c.leaves[std::min<size_t>(j, c.leaves.size() - 1)];
        st.table = c.tt;
        st.dst = lp.num_values++;
        lp.steps.push_back(st);
        lp.lut_steps++;
        pending[var] = 0;
        val[var] = {LutRef{LutRef::Varying, st.dst}, false};
    };
    auto value_of = [&](uint32_t lit) {  // literal as a leaf value; emits a pending gate first
        const uint32_t var = lit >> 1;
        if (pending[var]) emit(var);
        Val x = val[var];
        x.neg ^= (lit & 1) != 0;
        return x;
    };
    for (uint32_t k : plan.order) {
        const uint32_t v = n + 1 + k;
        const uint32_t la = g.and_r0[k], lb = g.and_r1[k];
        const uint32_t va = la >> 1, vb = lb >> 1;
        const bool absorb_a = pending[va] && fanout[va] == 1 && !is_output[va];
        const bool absorb_b = pending[vb] && fanout[vb] == 1 && !is_output[vb] && vb != va;
        if (!absorb_a && !absorb_b) {
            Val a = value_of(la), b = value_of(lb);
            if (a.ref.kind == LutRef::Word && b.ref.kind == LutRef::Word) {
                const uint32_t w = (lp.words[a.ref.index] ^ (a.neg ? ~0u : 0u)) & (lp.words[b.ref.index] ^ (b.neg ? ~0u : 0u));
                val[v] = {word(w), false};
                lp.folded_gates++;
                continue;
            }
            auto eff_word = [&](const Val& x, uint32_t& w) {
                if (x.ref.kind != LutRef::Word) return false;
                w = lp.words[x.ref.index] ^ (x.neg ? ~0u : 0u);
                return true;
            };
            uint32_t w;
            if ((eff_word(a, w) && w == 0) || (eff_word(b, w) && w == 0)) {
                val[v] = {word(0u), false};
                lp.folded_gates++;
                continue;
            }
            if (eff_word(a, w) && w == ~0u) { val[v] = b; lp.folded_gates++; continue; }
            if (eff_word(b, w) && w == ~0u) { val[v] = a; lp.folded_gates++; continue; }
            if (is_uniform_ref(a.ref) && is_uniform_ref(b.ref)) {
                LutStep st{};
                st.op = LutStep::ScalarAnd;
                st.leaf[0] = a.ref;
                st.leaf[1] = b.ref;
                st.table = (uint8_t)((a.neg ? 1 : 0) | (b.neg ? 2 : 0));
                st.dst = lp.num_values++;
                lp.steps.push_back(st);
                lp.scalar_steps++;
                val[v] = {LutRef{LutRef::Uniform, st.dst}, false};
                continue;
            }
        }
        // Varying gate: build its cover, absorbing single-reader pending fan-ins when the
        // union of leaves stays within three.
        struct Side {
            bool absorbed;
            Cover c;      // when absorbed
            Val leaf;     // when not
        };
        auto side_leaf = [&](uint32_t lit) {
            Side s{};
            s.absorbed = false;
            s.leaf = value_of(lit);
            return s;
        };
        auto side_abs = [&](uint32_t lit) {
            Side s{};
            s.absorbed = true;
            s.c = cover[lit >> 1];
            if (lit & 1) s.c.tt = (uint8_t)~s.c.tt;
            return s;
        };
        auto leaves_of = [&](const Side& s) {
            return s.absorbed ? s.c.leaves : std::vector<LutRef>{s.leaf.ref};
        };
        auto union_size = [&](const Side& x, const Side& y) {
            std::vector<LutRef> L = leaves_of(x);
            for (auto& r : leaves_of(y))
                if (std::none_of(L.begin(), L.end(), [&](const LutRef& q) { return same(q, r); })) L.push_back(r);
            return L;
        };
        // Candidate absorptions, best (most gates absorbed) first.
        std::vector<std::pair<bool, bool>> tries;
        if (absorb_a && absorb_b) tries.push_back({true, true});
        if (absorb_a && absorb_b && cover[vb].gates > cover[va].gates) {
            tries.push_back({false, true});
            tries.push_back({true, false});
        } else {
            if (absorb_a) tries.push_back({true, false});
            if (absorb_b) tries.push_back({false, true});
        }
        tries.push_back({false, false});
        Side A{}, B{};
        std::vector<LutRef> L;
        for (auto t : tries) {
            // Sides that are not absorbed become leaves (emitting them if pending) only once
            // the choice is final, so check leaf counts with their would-be refs first.
            auto peek = [&](uint32_t lit, bool abs) {
                if (abs) return side_abs(lit);
                Side s{};
                s.absorbed = false;
                const uint32_t var = lit >> 1;
                if (pending[var]) s.leaf = {LutRef{LutRef::Varying, 0xFFFFFFFFu - var}, (lit & 1) != 0};
                else {
                    s.leaf = val[var];
                    s.leaf.neg ^= (lit & 1) != 0;
                }
                return s;
            };
            Side a = peek(la, t.first), b = peek(lb, t.second);
            std::vector<LutRef> U = union_size(a, b);
            if (U.size() <= 3) {
                A = t.first ? a : side_leaf(la);
                B = t.second ? b : side_leaf(lb);
                L = union_size(A, B);
                break;
            }
        }
        // Constant-word leaves that are all zeros or all ones never reach here (folded above
        // when both sides are leaves); absorbed covers contain no such leaves either.
        Cover c;
        c.leaves = L;
        c.gates = 1 + (A.absorbed ? A.c.gates : 0) + (B.absorbed ? B.c.gates : 0);
        auto side_tt = [&](const Side& s) -> uint8_t {
            if (s.absorbed) return remap(s.c, L);
            uint32_t pos = 0;
            while (!same(L[pos], s.leaf.ref)) ++pos;
            return (uint8_t)(s.leaf.neg ? ~proj(pos) : proj(pos));
        };
        c.tt = (uint8_t)(side_tt(A) & side_tt(B));
        if (A.absorbed) lp.absorbed_gates += 1, pending[va] = 0;
        if (B.absorbed) lp.absorbed_gates += 1, pending[vb] = 0;
        cover[v] = c;
        pending[v] = 1;
    }
    for (uint32_t o : g.outputs) {
        Val x = value_of(o);
        LutStep st{};
        st.op = LutStep::Output;
        st.leaf[0] = x.ref;
        st.out_neg = x.neg;
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
