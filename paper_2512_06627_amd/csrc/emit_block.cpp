// Body of the specialized kernel as one inline-asm block with planner-assigned registers.
//
// The per-pass program is straight-line code, so the lifetime of every value is an
// interval and a linear scan over the steps assigns physical registers with the fewest
// registers that the order allows.  Emitting the whole pass as a single asm statement
// keeps the compiler out of the body: no wait states padded around many small asm
// statements, no register spills, no copies for the one-scalar-operand rule that the
// planner can avoid itself.  The compiler still owns everything around the body (claims,
// the early-exit test, the ballot) and keeps its values in the registers the block does
// not name.
//
// Register use inside the block:
//  * VGPRs: varying values (LUT results), temporaries that carry a second wave-uniform
//    operand of a LUT (a VALU instruction reads at most one SGPR), and plan-time words
//    that do not fit in the operand list;
//  * SGPRs: wave-uniform inputs 11.. (one s_bfe_i32 of the base index each, made just
//    before first use) and wave-uniform gate values.
// Nothing in the block touches memory, VCC or EXEC; SCC is clobbered by the scalar ops.
#include <algorithm>
#include <cstdio>
#include <map>
#include <set>
#include <climits>
#include <sstream>

#include "runtime.hpp"

namespace fes {
namespace {

enum class Kind : uint8_t { Vgpr, Sgpr, Operand, Inline, Lds };

struct Loc {
    Kind kind = Kind::Operand;
    int reg = -1;      // register number (Vgpr, Sgpr) or asm operand number (Operand)
    int64_t imm = 0;   // Inline: constant
};

std::string loc_text(const Loc& l) {
    switch (l.kind) {
        case Kind::Vgpr: return "v" + std::to_string(l.reg);
        case Kind::Sgpr: return "s" + std::to_string(l.reg);
        case Kind::Operand: return "%" + std::to_string(l.reg);
        default: {
            if (l.imm >= -16 && l.imm <= 64) return std::to_string(l.imm);
            char buf[16];
            std::snprintf(buf, sizeof buf, "0x%08x", (uint32_t)l.imm);
            return buf;
        }
    }
}

bool is_sgpr(const Loc& l) { return l.kind == Kind::Sgpr; }

// Pool of registers numbered from zero; hands out the lowest free register.
struct Pool {
    std::vector<int> free;  // kept sorted descending, so back() is the lowest
    int next = 0;
    int high = 0;
    int take() {
        int r;
        if (!free.empty()) {
            r = free.back();
            free.pop_back();
        } else {
            r = next++;
        }
        high = std::max(high, r + 1);
        return r;
    }
    void give(int r) {
        free.push_back(r);
        std::sort(free.begin(), free.end(), std::greater<int>());
    }
    // Lowest free register whose bank (number mod 4) is not in `avoid` (bit per bank); a new
    // register otherwise, skipping at most three numbers (they stay free for later) but never
    // past `cap`.
    int take_bank(unsigned avoid, int cap = 1 << 30) {
        if (avoid == 0 || avoid == 15) return take();
        for (size_t i = free.size(); i-- > 0;) {
            const int r = free[i];
            if (!((avoid >> (r & 3)) & 1u)) {
                free.erase(free.begin() + (long)i);
                high = std::max(high, r + 1);
                return r;
            }
        }
        if (!free.empty()) return take();
        while (((avoid >> (next & 3)) & 1u) && next + 1 < cap) give(next++);
        return take();
    }
};

uint64_t key_of(const LutRef& r) { return ((uint64_t)r.kind << 32) | r.index; }

// Order of the body: the program's own order, except that a step whose operands are not yet
// `dist` instructions old gives way to the next step that is ready.  The program's order
// (depth first, chosen for few live values) puts a gate right after its fan-ins; a wave
// then waits out the VALU latency on every step, which two or four waves per SIMD cannot
// hide.  Outputs are folded into the miter word two at a time.
std::vector<LutStep> schedule(const LutProgram& lp, int dist) {
    std::vector<LutStep> in;
    const LutStep* pending = nullptr;
    for (const LutStep& st : lp.steps) {
        if (st.op != LutStep::Output) {
            in.push_back(st);
            continue;
        }
        if (!pending) {
            pending = &st;
            continue;
        }
        LutStep pr{};
        pr.op = LutStep::Output;
        pr.nleaves = 2;
        pr.leaf[0] = pending->leaf[0];
        pr.leaf[1] = st.leaf[0];
        pr.table = (uint8_t)((pending->out_neg ? 1 : 0) | (st.out_neg ? 2 : 0));
        in.push_back(pr);
        pending = nullptr;
    }
    if (pending) {
        LutStep one{};
        one.op = LutStep::Output;
        one.nleaves = 1;
        one.leaf[0] = pending->leaf[0];
        one.table = pending->out_neg ? 1 : 0;
        in.push_back(one);
    }
    const size_t N = in.size();
    if (dist <= 1) return in;
    std::map<uint64_t, size_t> producer;
    for (size_t i = 0; i < N; ++i) {
        if (in[i].op == LutStep::Lut) producer[((uint64_t)LutRef::Varying << 32) | in[i].dst] = i;
        if (in[i].op == LutStep::ScalarAnd) producer[((uint64_t)LutRef::Uniform << 32) | in[i].dst] = i;
    }
    std::vector<std::vector<size_t>> preds(N), succs(N);
    for (size_t i = 0; i < N; ++i) {
        const LutStep& st = in[i];
        const uint32_t k = st.op == LutStep::ScalarAnd ? 2 : st.nleaves;
        for (uint32_t j = 0; j < k; ++j) {
            auto it = producer.find(((uint64_t)st.leaf[j].kind << 32) | st.leaf[j].index);
            if (it == producer.end()) continue;
            if (std::find(preds[i].begin(), preds[i].end(), it->second) == preds[i].end()) {
                preds[i].push_back(it->second);
                succs[it->second].push_back(i);
            }
        }
    }
    std::vector<size_t> waiting(N);
    std::set<size_t> ready;
    for (size_t i = 0; i < N; ++i) {
        waiting[i] = preds[i].size();
        if (!waiting[i]) ready.insert(i);
    }
    std::vector<int64_t> slot(N, -1);
    int64_t last_out = -(int64_t)dist, cur = 0;
    auto lat = [&](size_t p, size_t i) -> int64_t {
        // scalar results feed the next instruction; vector results need `dist` slots
        return in[p].op == LutStep::ScalarAnd ? 1 : (in[i].op == LutStep::ScalarAnd ? 1 : dist);
    };
    std::vector<LutStep> out;
    out.reserve(N);
    while (!ready.empty()) {
        size_t pick = N, best = N;
        int64_t best_t = INT64_MAX;
        for (size_t i : ready) {
            int64_t t = in[i].op == LutStep::Output ? last_out + dist : 0;
            for (size_t p : preds[i]) t = std::max(t, slot[p] + lat(p, i));
            if (t <= cur) {
                pick = i;
                break;
            }
            if (t < best_t) {
                best_t = t;
                best = i;
            }
        }
        if (pick == N) pick = best;
        ready.erase(pick);
        slot[pick] = cur++;
        if (in[pick].op == LutStep::Output) last_out = slot[pick];
        out.push_back(in[pick]);
        for (size_t q : succs[pick])
            if (--waiting[q] == 0) ready.insert(q);
    }
    return out;
}

// Order for few live vector values, used when the program's order needs more VGPRs than the
// occupancy target allows: list scheduling that takes the ready step which ends the most
// live values and starts the fewest (outputs fold their operands away), ties by the
// program's order.
std::vector<LutStep> schedule_min_live(const LutProgram& lp) {
    std::vector<LutStep> in = schedule(lp, 1);
    const size_t N = in.size();
    auto nleaves = [](const LutStep& st) -> uint32_t { return st.op == LutStep::ScalarAnd ? 2 : st.nleaves; };
    auto is_vec = [](const LutRef& r) { return r.kind == LutRef::Varying; };
    std::map<uint64_t, size_t> producer;
    std::map<uint64_t, uint32_t> remaining;  // unscheduled readers of a vector value
    for (size_t i = 0; i < N; ++i) {
        if (in[i].op == LutStep::Lut) producer[((uint64_t)LutRef::Varying << 32) | in[i].dst] = i;
        if (in[i].op == LutStep::ScalarAnd) producer[((uint64_t)LutRef::Uniform << 32) | in[i].dst] = i;
    }
    std::vector<std::vector<size_t>> succs(N);
    std::vector<size_t> waiting(N, 0);
    for (size_t i = 0; i < N; ++i) {
        std::vector<size_t> ps;
        for (uint32_t j = 0; j < nleaves(in[i]); ++j) {
            const uint64_t key = ((uint64_t)in[i].leaf[j].kind << 32) | in[i].leaf[j].index;
            if (is_vec(in[i].leaf[j])) ++remaining[key];
            auto it = producer.find(key);
            if (it != producer.end() && std::find(ps.begin(), ps.end(), it->second) == ps.end()) ps.push_back(it->second);
        }
        waiting[i] = ps.size();
        for (size_t p : ps) succs[p].push_back(i);
    }
    std::set<size_t> ready;
    for (size_t i = 0; i < N; ++i)
        if (!waiting[i]) ready.insert(i);
    std::vector<LutStep> out;
    out.reserve(N);
    while (!ready.empty()) {
        size_t pick = N;
        int best = 1 << 30;
        for (size_t i : ready) {
            const LutStep& st = in[i];
            int delta = 0;
            if (st.op == LutStep::Lut && remaining.count(((uint64_t)LutRef::Varying << 32) | st.dst)) delta += 1;
            std::vector<uint64_t> seen;
            for (uint32_t j = 0; j < nleaves(st); ++j) {
                if (!is_vec(st.leaf[j])) continue;
                const uint64_t key = ((uint64_t)st.leaf[j].kind << 32) | st.leaf[j].index;
                if (std::find(seen.begin(), seen.end(), key) != seen.end()) continue;
                seen.push_back(key);
                if (remaining[key] == 1) delta -= 1;
            }
            if (delta < best) {
                best = delta;
                pick = i;
                if (delta < 0) break;  // frees a value: take the earliest such step
            }
        }
        ready.erase(pick);
        const LutStep& st = in[pick];
        for (uint32_t j = 0; j < nleaves(st); ++j)
            if (is_vec(st.leaf[j])) --remaining[((uint64_t)st.leaf[j].kind << 32) | st.leaf[j].index];
        out.push_back(st);
        for (size_t q : succs[pick])
            if (--waiting[q] == 0) ready.insert(q);
    }
    return out;
}

bool emit_with_order(const LutProgram& lp, const std::vector<LutStep>& steps, int vgpr_limit, int sgpr_limit,
                     int sgpr_base, int word_operand_limit, bool bank_aware, int lds_slots, std::string* code,
                     BlockStats* stats) {
    const uint32_t n = lp.num_inputs;
    // ---- asm operand numbering ------------------------------------------------------------
    // %0 m (output), %1 low and %2 high word of the base half-word index, then the lane
    // inputs 5..min(n,11)-1, then plan-time words (VGPR operands) up to the limit.
    std::vector<std::string> in_cons;
    in_cons.push_back("\"s\"(base_lo)");
    in_cons.push_back("\"s\"(base_hi)");
    std::map<uint32_t, int> lane_operand;
    for (uint32_t i = 5; i < n && i < 11; ++i) {
        lane_operand[i] = 1 + (int)in_cons.size();
        in_cons.push_back("\"v\"(x" + std::to_string(i) + ")");
    }
    std::map<uint32_t, int> word_operand;
    auto inline_word = [](uint32_t w, int64_t* imm) {
        const int32_t s = (int32_t)w;
        if (s >= -16 && s <= 64) {
            *imm = s;
            return true;
        }
        return false;
    };
    // words read by LUTs or outputs, most-used first, become operands
    std::map<uint32_t, uint32_t> word_uses;
    for (const LutStep& st : steps) {
        if (st.op == LutStep::ScalarAnd) continue;
        const uint32_t k = st.nleaves;
        for (uint32_t j = 0; j < k; ++j)
            if (st.leaf[j].kind == LutRef::Word) ++word_uses[st.leaf[j].index];
    }
    std::vector<std::pair<uint32_t, uint32_t>> by_use;
    for (auto& kv : word_uses) {
        int64_t imm;
        if (!inline_word(lp.words[kv.first], &imm)) by_use.push_back({kv.second, kv.first});
    }
    std::sort(by_use.begin(), by_use.end(), std::greater<>());
    for (auto& u : by_use) {
        if ((int)word_operand.size() >= word_operand_limit) break;
        word_operand[u.second] = 1 + (int)in_cons.size();
        in_cons.push_back("\"v\"(w" + std::to_string(u.second) + ")");
    }
    // LDS spill slots: the lane's byte address in the wave's spill area; slot s is at offset
    // 256*s (64 lanes x 4 bytes).
    int spill_operand = -1;
    if (lds_slots > 0) {
        spill_operand = 1 + (int)in_cons.size();
        in_cons.push_back("\"v\"(spill_addr)");
    }

    // ---- uses of every value ------------------------------------------------------------
    std::map<uint64_t, size_t> last;
    std::map<uint64_t, size_t> last_scalar;  // last step that reads the value on the scalar unit
    for (size_t t = 0; t < steps.size(); ++t) {
        const LutStep& st = steps[t];
        const uint32_t k = st.op == LutStep::ScalarAnd ? 2 : st.nleaves;
        for (uint32_t j = 0; j < k; ++j) {
            last[key_of(st.leaf[j])] = t;
            if (st.op == LutStep::ScalarAnd) last_scalar[key_of(st.leaf[j])] = t;
        }
    }
    std::map<uint64_t, std::vector<size_t>> uses;
    for (size_t t = 0; t < steps.size(); ++t) {
        const LutStep& st = steps[t];
        const uint32_t k = st.op == LutStep::ScalarAnd ? 2 : st.nleaves;
        for (uint32_t j = 0; j < k; ++j) uses[key_of(st.leaf[j])].push_back(t);
    }

    // ---- linear scan ---------------------------------------------------------------------
    Pool vp, sp;
    std::map<uint64_t, Loc> where;
    std::map<uint64_t, int> vcopy;  // VGPR copy of a wave-uniform value held in an SGPR
    std::ostringstream a;  // asm text, one instruction per line
    uint32_t n_valu = 0, n_salu = 0, n_copies = 0;
    // One string literal per instruction (adjacent literals concatenate): clang analyses a
    // single literal with operand references in time quadratic in its length.
    auto line = [&](const std::string& s) { a << "        \"" << s << "\\n\\t\"\n"; };
    line("v_mov_b32 %0, 0");
    ++n_valu;
    // A new VGPR at step t.  When all vgpr_limit registers are taken and LDS slots are
    // available, the vector value whose next reader is farthest away goes to an LDS slot
    // (ds_write_b32) and is read back (ds_read_b32, then a wait) right before that reader.
    // Values read at step t stay in registers.  LDS operations of a wave execute in order, so
    // a read-back always sees its own write.
    Pool lp_slots;
    bool vgpr_failed = false;
    uint32_t n_lds = 0;
    auto take_v = [&](size_t t, unsigned avoid) -> int {
        if (!vp.free.empty() || vp.next < vgpr_limit || lds_slots <= 0) return vp.take_bank(avoid, vgpr_limit);
        uint64_t victim = 0;
        size_t far = 0;
        bool found = false;
        for (auto& kv : where) {
            if (kv.second.kind != Kind::Vgpr) continue;
            const std::vector<size_t>& u = uses[kv.first];
            auto nx = std::lower_bound(u.begin(), u.end(), t);
            if (nx != u.end() && *nx == t) continue;  // read at this step
            const size_t next = nx == u.end() ? SIZE_MAX : *nx;
            if (!found || next > far) {
                found = true;
                far = next;
                victim = kv.first;
            }
        }
        if (!found || (lp_slots.free.empty() && lp_slots.next >= lds_slots)) {
            vgpr_failed = true;
            return vp.take_bank(avoid);
        }
        Loc& l = where[victim];
        const int reg = l.reg;
        const int slot = lp_slots.take();
        char b[80];
        std::snprintf(b, sizeof b, "ds_write_b32 %%%d, v%d offset:%d", spill_operand, reg, 256 * slot);
        line(b);
        ++n_lds;
        l = Loc{Kind::Lds, slot, 0};
        return reg;
    };
    // A new SGPR at step t.  When the pool is full, the wave-uniform value with only VALU
    // readers left whose next reader is farthest moves to a VGPR (v_mov_b32 v, s); values
    // read at step t stay.  Values never move back: no VALU instruction writes an SGPR.
    bool spill_failed = false;
    uint32_t n_spills = 0;
    auto take_sgpr = [&](size_t t) -> int {
        if (!sp.free.empty() || sp.next < sgpr_limit) return sgpr_base + sp.take();
        uint64_t victim = 0;
        size_t far = 0;
        bool found = false;
        for (auto& kv : where) {
            if (kv.second.kind != Kind::Sgpr) continue;
            auto ls = last_scalar.find(kv.first);
            if (ls != last_scalar.end() && ls->second >= t) continue;
            const std::vector<size_t>& u = uses[kv.first];
            auto nx = std::lower_bound(u.begin(), u.end(), t);
            if (nx == u.end() || *nx == t) continue;
            if (!found || *nx > far) {
                found = true;
                far = *nx;
                victim = kv.first;
            }
        }
        if (!found) {
            spill_failed = true;
            return sgpr_base + sp.take();
        }
        Loc& l = where[victim];
        const int sreg = l.reg;
        const int vreg = take_v(t, 0);
        char b[64];
        std::snprintf(b, sizeof b, "v_mov_b32 v%d, s%d", vreg, sreg);
        line(b);
        ++n_valu;
        ++n_spills;
        l = Loc{Kind::Vgpr, vreg, 0};
        sp.give(sreg - sgpr_base);
        return sgpr_base + sp.take();
    };
    // Location of a leaf for a VALU (vector) or SALU (scalar) reader, materializing
    // uniform inputs and non-operand words on first use.
    auto locate = [&](const LutRef& r, bool scalar_reader, size_t t) -> Loc {
        Loc l;
        switch (r.kind) {
            case LutRef::Word: {
                int64_t imm;
                if (inline_word(lp.words[r.index], &imm)) {
                    l.kind = Kind::Inline;
                    l.imm = imm;
                    return l;
                }
                if (scalar_reader) {  // scalar ops take a 32-bit literal
                    l.kind = Kind::Inline;
                    l.imm = lp.words[r.index];
                    return l;
                }
                auto it = word_operand.find(r.index);
                if (it != word_operand.end()) return Loc{Kind::Operand, it->second, 0};
                auto w = where.find(key_of(r));
                if (w != where.end()) return w->second;
                l.kind = Kind::Vgpr;
                l.reg = take_v(t, 0);
                char buf[64];
                std::snprintf(buf, sizeof buf, "v_mov_b32 v%d, 0x%08x", l.reg, lp.words[r.index]);
                line(buf);
                ++n_valu;
                where[key_of(r)] = l;
                return l;
            }
            case LutRef::Input: {
                if (r.index < 11) return Loc{Kind::Operand, lane_operand.at(r.index), 0};
                auto w = where.find(key_of(r));
                if (w != where.end()) return w->second;
                l.kind = Kind::Sgpr;
                l.reg = take_sgpr(t);
                const uint32_t bit = r.index - 5;  // bit of the half-word index
                char buf[64];
                std::snprintf(buf, sizeof buf, "s_bfe_i32 s%d, %s, 0x%x", l.reg, bit < 32 ? "%1" : "%2",
                              (1u << 16) | (bit & 31u));
                line(buf);
                ++n_salu;
                where[key_of(r)] = l;
                return l;
            }
            default: {
                Loc& w = where.at(key_of(r));
                if (w.kind != Kind::Lds) return w;
                const int slot = w.reg;
                const int reg = take_v(t, 0);
                char buf[96];
                std::snprintf(buf, sizeof buf, "ds_read_b32 v%d, %%%d offset:%d", reg, spill_operand, 256 * slot);
                line(buf);
                line("s_waitcnt lgkmcnt(0)");
                ++n_lds;
                lp_slots.give(slot);
                Loc& w2 = where.at(key_of(r));  // take_v may have rehashed nothing, but re-find
                w2 = Loc{Kind::Vgpr, reg, 0};
                return w2;
            }
        }
    };
    auto release = [&](const LutRef& r, size_t t) {
        auto it = where.find(key_of(r));
        if (it == where.end()) return;
        auto lu = last.find(key_of(r));
        if (lu != last.end() && lu->second > t) return;
        if (it->second.kind == Kind::Vgpr) vp.give(it->second.reg);
        if (it->second.kind == Kind::Sgpr) sp.give(it->second.reg - sgpr_base);
        if (it->second.kind == Kind::Lds) lp_slots.give(it->second.reg);
        where.erase(it);
        auto vc = vcopy.find(key_of(r));
        if (vc != vcopy.end()) {
            vp.give(vc->second);
            vcopy.erase(vc);
        }
    };
    char buf[160];
    for (size_t t = 0; t < steps.size(); ++t) {
        const LutStep& st = steps[t];
        if (st.op == LutStep::ScalarAnd) {
            Loc x = locate(st.leaf[0], true, t);
            Loc y = locate(st.leaf[1], true, t);
            const bool na = st.table & 1, nb = (st.table >> 1) & 1;
            release(st.leaf[0], t);
            release(st.leaf[1], t);
            Loc d{Kind::Sgpr, take_sgpr(t), 0};
            const char* op = "s_and_b32";
            if (na && nb) op = "s_nor_b32";
            else if (nb) op = "s_andn2_b32";
            else if (na) { op = "s_andn2_b32"; std::swap(x, y); }
            std::snprintf(buf, sizeof buf, "%s s%d, %s, %s", op, d.reg, loc_text(x).c_str(), loc_text(y).c_str());
            line(buf);
            ++n_salu;
            LutRef self{LutRef::Uniform, st.dst};
            where[key_of(self)] = d;
            if (!last.count(key_of(self))) release(self, t);
            continue;
        }
        const uint32_t k = st.nleaves;
        Loc src[3];
        for (uint32_t j = 0; j < k; ++j) src[j] = locate(st.leaf[j], false, t);
        // At most one distinct SGPR per VALU instruction.  A wave-uniform value that already
        // has a VGPR copy is read from it; the others are copied (v_mov_b32), and a copy is
        // kept for later VALU readers while the value lives.
        std::vector<int> temps;
        for (uint32_t j = 0; j < k; ++j) {
            if (!is_sgpr(src[j])) continue;
            auto vc = vcopy.find(key_of(st.leaf[j]));
            if (vc != vcopy.end()) src[j] = Loc{Kind::Vgpr, vc->second, 0};
        }
        int sg = -1;
        for (uint32_t j = 0; j < k; ++j) {
            if (!is_sgpr(src[j])) continue;
            if (sg < 0 || sg == src[j].reg) {
                sg = src[j].reg;
                continue;
            }
            const int tv = take_v(t, 0);
            std::snprintf(buf, sizeof buf, "v_mov_b32 v%d, s%d", tv, src[j].reg);
            line(buf);
            ++n_valu;
            ++n_copies;
            if (last.at(key_of(st.leaf[j])) > t) vcopy[key_of(st.leaf[j])] = tv;
            else temps.push_back(tv);
            const int old = src[j].reg;
            for (uint32_t q = j; q < k; ++q)
                if (is_sgpr(src[q]) && src[q].reg == old) src[q] = Loc{Kind::Vgpr, tv, 0};
        }
        for (uint32_t j = 0; j < k; ++j) release(st.leaf[j], t);
        for (int tv : temps) vp.give(tv);
        if (st.op == LutStep::Lut) {
            // Bank choice: avoid the banks of the operands that this value's first reader
            // already has in VGPRs (three operands in one bank read serially).
            unsigned avoid = 0;
            if (bank_aware) {
                LutRef self{LutRef::Varying, st.dst};
                auto u = uses.find(key_of(self));
                if (u != uses.end() && !u->second.empty()) {
                    const LutStep& rd = steps[u->second.front()];
                    const uint32_t rk = rd.op == LutStep::ScalarAnd ? 2 : rd.nleaves;
                    for (uint32_t j = 0; j < rk; ++j) {
                        if (rd.leaf[j].kind == self.kind && rd.leaf[j].index == self.index) continue;
                        auto w = where.find(key_of(rd.leaf[j]));
                        if (w != where.end() && w->second.kind == Kind::Vgpr) avoid |= 1u << (w->second.reg & 3);
                    }
                }
            }
            Loc d{Kind::Vgpr, take_v(t, avoid), 0};
            const std::string s0 = loc_text(src[0]);
            const std::string s1 = loc_text(src[k >= 2 ? 1 : 0]);
            const std::string s2 = loc_text(src[k >= 3 ? 2 : (k >= 2 ? 1 : 0)]);
            std::snprintf(buf, sizeof buf, "v_bitop3_b32 v%d, %s, %s, %s bitop3:0x%02x", d.reg, s0.c_str(), s1.c_str(),
                          s2.c_str(), st.table);
            line(buf);
            ++n_valu;
            LutRef self{LutRef::Varying, st.dst};
            where[key_of(self)] = d;
            if (!last.count(key_of(self))) release(self, t);
        } else {
            // m = m | (x ^ neg_x) | (y ^ neg_y): table over (m, x, y); a single output repeats x
            const bool two = k == 2;
            uint8_t table = 0;
            for (uint32_t idx = 0; idx < 8; ++idx) {
                const uint32_t mm = (idx >> 2) & 1u, x = (idx >> 1) & 1u, y = idx & 1u;
                const uint32_t tx = x ^ (st.table & 1u), ty = two ? (y ^ ((st.table >> 1) & 1u)) : tx;
                if (mm | tx | ty) table |= (uint8_t)(1u << idx);
            }
            const std::string x = loc_text(src[0]), y = loc_text(src[two ? 1 : 0]);
            std::snprintf(buf, sizeof buf, "v_bitop3_b32 %%0, %%0, %s, %s bitop3:0x%02x", x.c_str(), y.c_str(), table);
            line(buf);
            ++n_valu;
        }
    }
    if (n_lds) line("s_waitcnt lgkmcnt(0)");  // no spill write outlives the block
    const int nv = vp.high, ns = sp.high;
    if (stats) {
        stats->vgprs = nv;
        stats->sgprs = ns;
        stats->valu = n_valu;
        stats->salu = n_salu;
        stats->copies = n_copies;
        stats->word_operands = (int)word_operand.size();
        stats->spills = n_spills;
        stats->lds_ops = n_lds;
        stats->lds_slots = lp_slots.high;
    }
    if (spill_failed || vgpr_failed || nv > vgpr_limit || ns > sgpr_limit) return false;
    // ---- the asm statement -------------------------------------------------------------
    std::ostringstream o;
    o << "      u32 m0;\n"
         "      asm volatile(\n" << a.str() << "        : \"=&v\"(m0)\n        : ";
    for (size_t i = 0; i < in_cons.size(); ++i) o << (i ? ", " : "") << in_cons[i];
    o << "\n        : \"scc\"";
    for (int r = 0; r < nv; ++r) o << ", \"v" << r << "\"";
    for (int r = 0; r < ns; ++r) o << ", \"s" << (sgpr_base + r) << "\"";
    o << ");\n";
    *code = o.str();
    return true;
}

}  // namespace

bool emit_block_body(const LutProgram& lp, int vgpr_limit, int sgpr_limit, int sgpr_base, int word_operand_limit,
                     int dist, bool bank_aware, int lds_slots, std::string* code, BlockStats* stats) {
    if (emit_with_order(lp, schedule(lp, dist), vgpr_limit, sgpr_limit, sgpr_base, word_operand_limit, bank_aware,
                        lds_slots, code, stats))
        return true;
    BlockStats first = stats ? *stats : BlockStats{};
    if (emit_with_order(lp, schedule_min_live(lp), vgpr_limit, sgpr_limit, sgpr_base, word_operand_limit,
                        bank_aware, lds_slots, code, stats)) {
        if (stats) stats->min_live_order = true;
        return true;
    }
    const int min_live_vgprs = stats ? stats->vgprs : 0;
    if (stats && first.vgprs < stats->vgprs) *stats = first;
    if (stats) stats->vgprs_min_live = min_live_vgprs;
    return false;
}

}  // namespace fes
