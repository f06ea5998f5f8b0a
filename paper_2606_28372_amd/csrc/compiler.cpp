// Constraint compiler: Python integer expressions -> stack bytecode (host only).
//
// Section IV-A defines each constraint as a predicate over a subset of the
// tunable parameters; users write them as Python expressions over the
// parameter names.  This file parses that language (integer literals,
// True/False, names, + - * // %, unary - + not, abs/min/max calls, chained
// comparisons, and/or, parentheses) with Python's precedence, proves with
// interval arithmetic that no intermediate can leave int64, and emits one
// stack program per constraint (opcodes in ct_bytecode.h).
//
// Python semantics kept by the emitted code:
//   - `a and b` / `a or b` return an operand; evaluation of the second operand
//     cannot make the result raise when Python would have short-circuited
//     (each stack slot carries a "would raise" bit, see the interpreter);
//   - `a < b < c` is `(a < b) and (b < c)` (b emitted twice; it is pure);
//   - a division or modulo by zero makes the constraint false.
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ct.h"
#include "ct_bytecode.h"
#include "ct_host.h"

namespace {

typedef __int128 i128;

struct Node {
    enum Kind { NUM, PARAM, NEG, NOT, ABS, BIN, CMP, BOOL, MINMAX } kind;
    int64_t value = 0;          // NUM
    int param = -1;             // PARAM
    int op = 0;                 // BIN: opcode; BOOL: OP_AND/OP_OR; MINMAX: OP_MIN/OP_MAX
    std::vector<int> cmp_ops;   // CMP: opcodes between consecutive operands
    std::vector<Node> kids;
};

struct Parser {
    const char* src;
    size_t pos = 0;
    const std::vector<std::string>& names;
    std::string error;

    Parser(const char* s, const std::vector<std::string>& n) : src(s), names(n) {}

    void skip_ws() {
        while (src[pos] == ' ' || src[pos] == '\t' || src[pos] == '\n' || src[pos] == '\r') pos++;
    }
    bool fail(const std::string& msg) {
        if (error.empty()) error = msg + " at offset " + std::to_string(pos);
        return false;
    }
    static bool is_ident_start(char c) { return (c >= 'a' && c <= 'z') || (c >= 'A' && c <= 'Z') || c == '_'; }
    static bool is_ident(char c) { return is_ident_start(c) || (c >= '0' && c <= '9'); }

    // peek an identifier-like keyword without consuming
    bool peek_word(const char* w) {
        skip_ws();
        size_t n = strlen(w);
        return strncmp(src + pos, w, n) == 0 && !is_ident(src[pos + n]);
    }
    bool eat_word(const char* w) {
        if (!peek_word(w)) return false;
        pos += strlen(w);
        return true;
    }
    bool eat(const char* tok) {
        skip_ws();
        size_t n = strlen(tok);
        if (strncmp(src + pos, tok, n) != 0) return false;
        pos += n;
        return true;
    }

    bool parse_or(Node& out) { return parse_bool(out, OP_OR); }

    // or_test / and_test
    bool parse_bool(Node& out, int which) {
        Node first;
        if (!(which == OP_OR ? parse_bool(first, OP_AND) : parse_not(first))) return false;
        const char* kw = which == OP_OR ? "or" : "and";
        if (!peek_word(kw)) { out = std::move(first); return true; }
        out = Node{Node::BOOL};
        out.op = which;
        out.kids.push_back(std::move(first));
        while (eat_word(kw)) {
            Node nx;
            if (!(which == OP_OR ? parse_bool(nx, OP_AND) : parse_not(nx))) return false;
            out.kids.push_back(std::move(nx));
        }
        return true;
    }

    bool parse_not(Node& out) {
        if (eat_word("not")) {
            Node k;
            if (!parse_not(k)) return false;
            out = Node{Node::NOT};
            out.kids.push_back(std::move(k));
            return true;
        }
        return parse_cmp(out);
    }

    int cmp_op() {
        skip_ws();
        static const struct { const char* t; int op; } ops[] = {
            {"<=", OP_LE}, {">=", OP_GE}, {"==", OP_EQ}, {"!=", OP_NE}, {"<", OP_LT}, {">", OP_GT}};
        for (auto& o : ops) {
            size_t n = strlen(o.t);
            if (strncmp(src + pos, o.t, n) == 0) {
                if (n == 1 && (src[pos + 1] == '<' || src[pos + 1] == '>')) return 0;  // shifts
                pos += n;
                return o.op;
            }
        }
        if (peek_word("in") || peek_word("is")) { fail("'in'/'is' are not supported"); return -1; }
        return 0;
    }

    bool parse_cmp(Node& out) {
        Node first;
        if (!parse_arith(first)) return false;
        int op = cmp_op();
        if (op < 0) return false;
        if (op == 0) { out = std::move(first); return true; }
        out = Node{Node::CMP};
        out.kids.push_back(std::move(first));
        while (op > 0) {
            Node nx;
            if (!parse_arith(nx)) return false;
            out.cmp_ops.push_back(op);
            out.kids.push_back(std::move(nx));
            op = cmp_op();
            if (op < 0) return false;
        }
        return true;
    }

    bool parse_arith(Node& out) {
        if (!parse_term(out)) return false;
        for (;;) {
            skip_ws();
            int op = 0;
            if (src[pos] == '+') op = OP_ADD;
            else if (src[pos] == '-') op = OP_SUB;
            else return true;
            pos++;
            Node rhs;
            if (!parse_term(rhs)) return false;
            Node b{Node::BIN};
            b.op = op;
            b.kids.push_back(std::move(out));
            b.kids.push_back(std::move(rhs));
            out = std::move(b);
        }
    }

    bool parse_term(Node& out) {
        if (!parse_factor(out)) return false;
        for (;;) {
            skip_ws();
            int op = 0;
            if (src[pos] == '*' && src[pos + 1] == '*') return fail("'**' is not supported");
            if (src[pos] == '/' && src[pos + 1] == '/') { op = OP_FDIV; pos += 2; }
            else if (src[pos] == '/') return fail("true division '/' is not supported (use //)");
            else if (src[pos] == '*') { op = OP_MUL; pos++; }
            else if (src[pos] == '%') { op = OP_MOD; pos++; }
            else return true;
            Node rhs;
            if (!parse_factor(rhs)) return false;
            Node b{Node::BIN};
            b.op = op;
            b.kids.push_back(std::move(out));
            b.kids.push_back(std::move(rhs));
            out = std::move(b);
        }
    }

    bool parse_factor(Node& out) {
        skip_ws();
        if (src[pos] == '-') {
            pos++;
            Node k;
            if (!parse_factor(k)) return false;
            out = Node{Node::NEG};
            out.kids.push_back(std::move(k));
            return true;
        }
        if (src[pos] == '+') {
            pos++;
            return parse_factor(out);
        }
        if (src[pos] == '~') return fail("'~' is not supported");
        return parse_atom(out);
    }

    bool parse_atom(Node& out) {
        skip_ws();
        char c = src[pos];
        if (c == '(') {
            pos++;
            if (!parse_or(out)) return false;
            if (!eat(")")) return fail("expected ')'");
            return true;
        }
        if (c >= '0' && c <= '9') {
            i128 v = 0;
            int base = 10;
            if (c == '0' && (src[pos + 1] == 'x' || src[pos + 1] == 'X')) { base = 16; pos += 2; }
            bool any = false;
            for (;;) {
                char d = src[pos];
                int dv;
                if (d == '_') { pos++; continue; }
                if (d >= '0' && d <= '9') dv = d - '0';
                else if (base == 16 && d >= 'a' && d <= 'f') dv = d - 'a' + 10;
                else if (base == 16 && d >= 'A' && d <= 'F') dv = d - 'A' + 10;
                else break;
                v = v * base + dv;
                if (v > (i128)INT64_MAX) return fail("integer literal does not fit in int64");
                any = true;
                pos++;
            }
            if (!any) return fail("bad integer literal");
            if (src[pos] == '.' || src[pos] == 'e' || src[pos] == 'E' || src[pos] == 'j')
                return fail("only integer literals are supported");
            out = Node{Node::NUM};
            out.value = (int64_t)v;
            return true;
        }
        if (is_ident_start(c)) {
            size_t b = pos;
            while (is_ident(src[pos])) pos++;
            std::string id(src + b, pos - b);
            if (id == "True" || id == "False") {
                out = Node{Node::NUM};
                out.value = id == "True";
                return true;
            }
            if (id == "and" || id == "or" || id == "not" || id == "in" || id == "is" || id == "if" ||
                id == "else" || id == "lambda")
                return fail("unexpected keyword '" + id + "'");
            skip_ws();
            if (src[pos] == '(') {
                pos++;
                std::vector<Node> args;
                skip_ws();
                if (src[pos] != ')') {
                    for (;;) {
                        Node a;
                        if (!parse_or(a)) return false;
                        args.push_back(std::move(a));
                        if (eat(",")) continue;
                        break;
                    }
                }
                if (!eat(")")) return fail("expected ')' after call arguments");
                if (id == "abs") {
                    if (args.size() != 1) return fail("abs() takes one argument");
                    out = Node{Node::ABS};
                    out.kids = std::move(args);
                    return true;
                }
                if (id == "min" || id == "max") {
                    if (args.size() < 2) return fail(id + "() needs at least two arguments");
                    out = Node{Node::MINMAX};
                    out.op = id == "min" ? OP_MIN : OP_MAX;
                    out.kids = std::move(args);
                    return true;
                }
                return fail("call to unsupported function '" + id + "'");
            }
            for (size_t j = 0; j < names.size(); j++)
                if (names[j] == id) {
                    out = Node{Node::PARAM};
                    out.param = (int)j;
                    return true;
                }
            return fail("unknown name '" + id + "'");
        }
        if (c == '\'' || c == '"') return fail("strings are not supported");
        if (c == 0) return fail("unexpected end of expression");
        return fail(std::string("unexpected character '") + c + "'");
    }
};

struct Range { i128 lo, hi; };

const i128 I64MIN = (i128)INT64_MIN, I64MAX = (i128)INT64_MAX;

struct Emitter {
    const std::vector<int64_t>& pmin;
    const std::vector<int64_t>& pmax;
    std::vector<uint32_t> code;
    int depth = 0, max_depth = 0;
    bool overflow = false;

    Emitter(const std::vector<int64_t>& a, const std::vector<int64_t>& b) : pmin(a), pmax(b) {}

    void push_word(uint32_t op, int32_t imm) { code.push_back((op & 0xFFu) | ((uint32_t)imm << 8)); }
    void grow(int d) {
        depth += d;
        if (depth > max_depth) max_depth = depth;
    }
    Range check(Range r) {
        if (r.lo < I64MIN || r.hi > I64MAX) overflow = true;
        return r;
    }

    Range emit(const Node& n) {
        switch (n.kind) {
        case Node::NUM:
            if (n.value >= -(1 << 23) && n.value < (1 << 23)) {
                push_word(OP_CONST, (int32_t)n.value);
            } else {
                push_word(OP_CONST64, 0);
                code.push_back((uint32_t)(uint64_t)n.value);
                code.push_back((uint32_t)((uint64_t)n.value >> 32));
            }
            grow(1);
            return {n.value, n.value};
        case Node::PARAM:
            push_word(OP_PARAM, n.param);
            grow(1);
            return {pmin[n.param], pmax[n.param]};
        case Node::NEG: {
            Range a = emit(n.kids[0]);
            push_word(OP_NEG, 0);
            return check({-a.hi, -a.lo});
        }
        case Node::ABS: {
            Range a = emit(n.kids[0]);
            push_word(OP_ABS, 0);
            i128 hi = a.hi > -a.lo ? a.hi : -a.lo;
            i128 lo = (a.lo <= 0 && a.hi >= 0) ? 0 : (a.lo > 0 ? a.lo : -a.hi);
            return check({lo, hi});
        }
        case Node::NOT:
            emit(n.kids[0]);
            push_word(OP_NOT, 0);
            return {0, 1};
        case Node::BIN: {
            Range a = emit(n.kids[0]);
            Range b = emit(n.kids[1]);
            push_word(n.op, 0);
            grow(-1);
            switch (n.op) {
            case OP_ADD: return check({a.lo + b.lo, a.hi + b.hi});
            case OP_SUB: return check({a.lo - b.hi, a.hi - b.lo});
            case OP_MUL: {
                i128 p[4] = {a.lo * b.lo, a.lo * b.hi, a.hi * b.lo, a.hi * b.hi};
                i128 lo = p[0], hi = p[0];
                for (int k = 1; k < 4; k++) { if (p[k] < lo) lo = p[k]; if (p[k] > hi) hi = p[k]; }
                // operands are within int64, so |product| < 2^126: no i128 wrap
                return check({lo, hi});
            }
            case OP_FDIV: {
                // |a // b| <= |a| for integer b != 0
                i128 m = a.hi > -a.lo ? a.hi : -a.lo;
                return check({-m, m});
            }
            case OP_MOD: {
                i128 m = b.hi > -b.lo ? b.hi : -b.lo;
                return check({m > 0 ? -(m - 1) : 0, m > 0 ? m - 1 : 0});
            }
            }
            return {0, 0};
        }
        case Node::CMP: {
            // (k0 op0 k1) and (k1 op1 k2) and ...
            for (size_t i = 0; i + 1 < n.kids.size(); i++) {
                emit(n.kids[i]);
                emit(n.kids[i + 1]);
                push_word(n.cmp_ops[i], 0);
                grow(-1);
                if (i > 0) {
                    push_word(OP_AND, 0);
                    grow(-1);
                }
            }
            return {0, 1};
        }
        case Node::BOOL: {
            Range r = emit(n.kids[0]);
            for (size_t i = 1; i < n.kids.size(); i++) {
                Range b = emit(n.kids[i]);
                push_word(n.op, 0);
                grow(-1);
                r = {r.lo < b.lo ? r.lo : b.lo, r.hi > b.hi ? r.hi : b.hi};
            }
            return r;
        }
        case Node::MINMAX: {
            Range r = emit(n.kids[0]);
            for (size_t i = 1; i < n.kids.size(); i++) {
                Range b = emit(n.kids[i]);
                push_word(n.op, 0);
                grow(-1);
                if (n.op == OP_MIN) r = {r.lo < b.lo ? r.lo : b.lo, r.hi < b.hi ? r.hi : b.hi};
                else r = {r.lo > b.lo ? r.lo : b.lo, r.hi > b.hi ? r.hi : b.hi};
            }
            return r;
        }
        }
        return {0, 0};
    }
};

}  // namespace

extern "C" int ct_compile(const char* const* names, uint32_t n_params, const int64_t* values,
                          const uint32_t* radices, const char* const* constraints, uint32_t n_cons,
                          uint32_t* code, uint32_t code_cap, uint32_t* cons_offsets, uint32_t* code_len) {
    if (!names || !values || !radices || (n_cons && !constraints) || !cons_offsets || !code_len)
        return ct_fail(CT_EINVAL, "ct_compile: null argument");
    if (n_params < 1 || n_params > CT_MAX_PARAMS) return ct_fail(CT_EINVAL, "ct_compile: 1..32 parameters supported");
    if (n_cons > CT_MAX_PROGRAMS) return ct_fail(CT_EINVAL, "ct_compile: at most 64 constraints");
    std::vector<std::string> nm(n_params);
    std::vector<int64_t> pmin(n_params), pmax(n_params);
    size_t off = 0;
    for (uint32_t j = 0; j < n_params; j++) {
        if (!names[j]) return ct_fail(CT_EINVAL, "ct_compile: null parameter name");
        nm[j] = names[j];
        if (radices[j] < 1 || radices[j] > CT_MAX_RADIX) return ct_fail(CT_EINVAL, "ct_compile: radix must be 1..255");
        pmin[j] = pmax[j] = values[off];
        for (uint32_t k = 0; k < radices[j]; k++) {
            int64_t v = values[off + k];
            if (v < pmin[j]) pmin[j] = v;
            if (v > pmax[j]) pmax[j] = v;
        }
        off += radices[j];
    }
    std::vector<uint32_t> all;
    std::vector<uint32_t> offs;
    for (uint32_t c = 0; c < n_cons; c++) {
        if (!constraints[c]) return ct_fail(CT_EINVAL, "ct_compile: null constraint");
        Parser p(constraints[c], nm);
        Node root;
        bool ok = p.parse_or(root);
        if (ok) {
            p.skip_ws();
            if (p.src[p.pos] != 0) ok = p.fail("unexpected trailing text");
        }
        if (!ok)
            return ct_fail(CT_ESYNTAX, "constraint " + std::to_string(c) + " \"" + constraints[c] + "\": " + p.error);
        Emitter e(pmin, pmax);
        e.emit(root);
        if (e.overflow)
            return ct_fail(CT_EOVERFLOW, "constraint " + std::to_string(c) + " \"" + constraints[c] +
                                             "\": an intermediate value may not fit in int64");
        if (e.max_depth > 16)
            return ct_fail(CT_EINVAL, "constraint " + std::to_string(c) + ": expression nests too deeply (stack > 16)");
        offs.push_back((uint32_t)all.size());
        all.insert(all.end(), e.code.begin(), e.code.end());
    }
    offs.push_back((uint32_t)all.size());
    if (all.size() > code_cap || (all.size() && !code))
        return ct_fail(CT_EINVAL, "ct_compile: code capacity too small (need " + std::to_string(all.size()) + " words)");
    if (!all.empty()) memcpy(code, all.data(), all.size() * sizeof(uint32_t));
    memcpy(cons_offsets, offs.data(), offs.size() * sizeof(uint32_t));
    *code_len = (uint32_t)all.size();
    return CT_OK;
}
