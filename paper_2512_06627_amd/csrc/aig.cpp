// AIGER reader (ASCII and binary) following the public AIGER 1.9 format
// description: header "aag|aig M I L O A [B C J F]", input lines (ASCII only),
// latch lines, output lines, AND gates (ASCII lines or binary deltas), then an
// optional symbol table and comment section, which are ignored.
#include "aig.hpp"

#include <algorithm>
#include <cstring>

namespace fes {
namespace {

[[noreturn]] void fail(int code, const std::string& m) { throw Error{code, m}; }

struct Reader {
    const uint8_t* p;
    size_t n, i = 0;
    Reader(const uint8_t* b, size_t l) : p(b), n(l) {}

    void spaces() {
        while (i < n && p[i] == ' ') ++i;
    }
    bool uint(uint64_t& v) {
        spaces();
        if (i >= n || p[i] < '0' || p[i] > '9') return false;
        uint64_t x = 0;
        while (i < n && p[i] >= '0' && p[i] <= '9') {
            x = x * 10 + (p[i] - '0');
            if (x > 0xFFFFFFFFull) return false;
            ++i;
        }
        v = x;
        return true;
    }
    uint64_t need_uint(const char* what) {
        uint64_t v;
        if (!uint(v)) fail(kErrParse, std::string("expected a number in ") + what);
        return v;
    }
    void eol(const char* what) {
        spaces();
        if (i < n && p[i] == '\r') ++i;
        if (i >= n) return;
        if (p[i] != '\n') fail(kErrParse, std::string("trailing characters in ") + what);
        ++i;
    }
    // Binary AIGER delta: 7 bits per byte, least significant group first, MSB = continue.
    uint64_t varint() {
        uint64_t x = 0;
        int shift = 0;
        for (;;) {
            if (i >= n) fail(kErrParse, "truncated binary AND section");
            uint8_t c = p[i++];
            x |= (uint64_t)(c & 0x7F) << shift;
            if (!(c & 0x80)) break;
            shift += 7;
            if (shift > 35) fail(kErrParse, "binary delta too large");
        }
        return x;
    }
};

}  // namespace

Aig parse_aiger(const uint8_t* bytes, size_t len) {
    if (!bytes) fail(kErrInvalid, "null AIGER buffer");
    if (len < 4 || (std::memcmp(bytes, "aag ", 4) != 0 && std::memcmp(bytes, "aig ", 4) != 0))
        fail(kErrParse, "not an AIGER file: header must start with 'aag' or 'aig'");
    const bool binary = bytes[1] == 'i';
    Reader r(bytes, len);
    r.i = 3;
    const uint64_t M = r.need_uint("header"), I = r.need_uint("header"), L = r.need_uint("header"),
                   O = r.need_uint("header"), A = r.need_uint("header");
    for (int k = 0; k < 4; ++k) {  // optional B C J F
        size_t save = r.i;
        uint64_t extra;
        if (!r.uint(extra)) {
            r.i = save;
            break;
        }
        if (extra) fail(kErrUnsupported, "bad-state, constraint, justice or fairness sections are sequential");
    }
    r.eol("header");
    if (L) fail(kErrUnsupported, "latches: only combinational (latch-free) AIGs are supported");
    if (I > 63) fail(kErrUnsupported, "more than 63 primary inputs");
    if (M < I + A) fail(kErrParse, "header: M < I + A");
    if (binary && M != I + A) fail(kErrParse, "binary header: M must equal I + L + A");

    // kind: 0 undefined, 1 constant, 2 input, 3 AND; idx = input index or AND line
    std::vector<uint8_t> kind(M + 1, 0);
    std::vector<uint32_t> idx(M + 1, 0);
    kind[0] = 1;
    std::vector<uint32_t> in_var(I);
    if (binary) {
        for (uint64_t k = 0; k < I; ++k) {
            in_var[k] = (uint32_t)(k + 1);
            kind[k + 1] = 2;
            idx[k + 1] = (uint32_t)k;
        }
    } else {
        for (uint64_t k = 0; k < I; ++k) {
            uint64_t lit = r.need_uint("input line");
            r.eol("input line");
            if ((lit & 1) || lit < 2 || (lit >> 1) > M) fail(kErrParse, "bad input literal");
            if (kind[lit >> 1]) fail(kErrParse, "variable defined twice");
            kind[lit >> 1] = 2;
            idx[lit >> 1] = (uint32_t)k;
            in_var[k] = (uint32_t)(lit >> 1);
        }
    }
    std::vector<uint32_t> out_lit(O);
    for (uint64_t k = 0; k < O; ++k) {
        uint64_t lit = r.need_uint("output line");
        r.eol("output line");
        if ((lit >> 1) > M) fail(kErrParse, "output literal out of range");
        out_lit[k] = (uint32_t)lit;
    }
    std::vector<uint32_t> lhs(A), f0(A), f1(A);
    for (uint64_t k = 0; k < A; ++k) {
        uint64_t l, a, b;
        if (binary) {
            l = 2 * (I + k + 1);
            uint64_t d0 = r.varint(), d1 = r.varint();
            if (d0 == 0 || d0 > l) fail(kErrParse, "binary AND: bad first delta");
            a = l - d0;
            if (d1 > a) fail(kErrParse, "binary AND: bad second delta");
            b = a - d1;
        } else {
            l = r.need_uint("AND line");
            a = r.need_uint("AND line");
            b = r.need_uint("AND line");
            r.eol("AND line");
        }
        if ((l & 1) || l < 2 || (l >> 1) > M || (a >> 1) > M || (b >> 1) > M) fail(kErrParse, "bad AND literal");
        if (kind[l >> 1]) fail(kErrParse, "variable defined twice");
        kind[l >> 1] = 3;
        idx[l >> 1] = (uint32_t)k;
        lhs[k] = (uint32_t)l;
        f0[k] = (uint32_t)a;
        f1[k] = (uint32_t)b;
    }
    for (uint32_t o : out_lit)
        if (!kind[o >> 1]) fail(kErrParse, "output uses an undefined variable");
    for (uint64_t k = 0; k < A; ++k)
        if (!kind[f0[k] >> 1] || !kind[f1[k] >> 1]) fail(kErrParse, "AND uses an undefined variable");

    // Topological order of AND lines: iterative post-order DFS; a gate met while on the
    // stack is a cycle.
    std::vector<uint32_t> order;
    order.reserve(A);
    std::vector<uint8_t> st(A, 0);  // 0 new, 1 open, 2 closed
    std::vector<uint32_t> stack;
    for (uint64_t root = 0; root < A; ++root) {
        if (st[root]) continue;
        stack.push_back((uint32_t)root);
        st[root] = 1;
        while (!stack.empty()) {
            uint32_t k = stack.back();
            uint32_t next = UINT32_MAX;
            for (uint32_t f : {f0[k] >> 1, f1[k] >> 1}) {
                if (kind[f] != 3) continue;
                uint32_t j = idx[f];
                if (st[j] == 1) fail(kErrParse, "combinational cycle");
                if (st[j] == 0) {
                    next = j;
                    break;
                }
            }
            if (next != UINT32_MAX) {
                st[next] = 1;
                stack.push_back(next);
            } else {
                st[k] = 2;
                stack.pop_back();
                order.push_back(k);
            }
        }
    }

    // Dense renumbering.
    Aig g;
    g.num_inputs = (uint32_t)I;
    std::vector<uint32_t> newvar(M + 1, 0);
    for (uint64_t k = 0; k < I; ++k) newvar[in_var[k]] = (uint32_t)(k + 1);
    for (uint64_t t = 0; t < A; ++t) newvar[lhs[order[t]] >> 1] = (uint32_t)(I + 1 + t);
    auto map = [&](uint32_t lit) { return 2 * newvar[lit >> 1] + (lit & 1); };
    g.and_r0.resize(A);
    g.and_r1.resize(A);
    for (uint64_t t = 0; t < A; ++t) {
        g.and_r0[t] = map(f0[order[t]]);
        g.and_r1[t] = map(f1[order[t]]);
    }
    g.outputs.resize(O);
    for (uint64_t k = 0; k < O; ++k) g.outputs[k] = map(out_lit[k]);
    return g;
}

}  // namespace fes
