// OpenQASM 2.0 frontend: program text -> gate records.
//
// The paper ingests its circuits as QASM text rather than as circuit objects,
// because building objects for 10^8 gates dominated its run time (Section
// 4.1); its gate set is the one of its Table 3.  This parser streams over the
// text (no token array), so a 10^6-gate program costs one pass and the output
// records.
//
// Accepted: the OPENQASM header; include lines (the standard gates are built
// in); qreg / creg declarations (qubits and classical bits are numbered across
// registers in declaration order); gate definitions with parameters, expanded
// with parameter substitution at each call; gate calls on single qubits or
// whole registers (broadcast over equal-size registers); measure (the
// classical bit index becomes the measurement slot), reset, barrier;
// parameter expressions with pi, + - * / ^, unary minus, parentheses and
// sin cos tan exp ln sqrt.  Rejected with QSIM_E_UNSUPPORTED: if, opaque, and
// gates the library does not lower (their name is given in the message).
#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <unordered_map>
#include <string>
#include <vector>

#include "host.h"

namespace qs {

namespace {

struct Tok {
    enum Kind { END, ID, NUM, STR, SYM } k = END;
    std::string s;   // identifier, string body or symbol
    double v = 0;    // number
    int line = 0;
};

// Streaming lexer over the program text, or over a stored token list (the
// body of a gate definition).
class Lexer {
  public:
    Lexer(const char *p, size_t n) : p_(p), end_(p + n) {}
    explicit Lexer(const std::vector<Tok> *toks) : toks_(toks) {}

    const Tok &peek() {
        if (!have_) {
            cur_ = toks_ ? (ti_ < toks_->size() ? (*toks_)[ti_++] : Tok{}) : scan();
            have_ = true;
        }
        return cur_;
    }
    Tok next() {
        peek();
        have_ = false;
        return cur_;
    }
    int line() { return peek().line; }

  private:
    Tok scan() {
        Tok t;
        for (;;) {
            while (p_ < end_ && std::isspace(static_cast<unsigned char>(*p_))) {
                if (*p_ == '\n') line_++;
                p_++;
            }
            if (p_ + 1 < end_ && p_[0] == '/' && p_[1] == '/') {
                while (p_ < end_ && *p_ != '\n') p_++;
                continue;
            }
            break;
        }
        t.line = line_;
        if (p_ >= end_) return t;
        const char c = *p_;
        if (std::isalpha(static_cast<unsigned char>(c)) || c == '_') {
            const char *b = p_;
            while (p_ < end_ && (std::isalnum(static_cast<unsigned char>(*p_)) || *p_ == '_')) p_++;
            t.k = Tok::ID;
            t.s.assign(b, p_);
            return t;
        }
        if (std::isdigit(static_cast<unsigned char>(c)) || (c == '.' && p_ + 1 < end_ && std::isdigit(static_cast<unsigned char>(p_[1])))) {
            t.k = Tok::NUM;
            // plain integers (qubit indices, mostly) without strtod
            const char *q = p_;
            uint64_t iv = 0;
            while (q < end_ && std::isdigit(static_cast<unsigned char>(*q)) && q - p_ < 18) iv = iv * 10 + uint64_t(*q++ - '0');
            if (q == end_ || (*q != '.' && *q != 'e' && *q != 'E' && !std::isdigit(static_cast<unsigned char>(*q)))) {
                t.v = double(iv);
                p_ = q;
                return t;
            }
            // the number's own characters, then strtod on a terminated copy
            q = p_;
            while (q < end_ && q - p_ < 64 &&
                   (std::isdigit(static_cast<unsigned char>(*q)) || *q == '.' || *q == 'e' || *q == 'E' ||
                    ((*q == '+' || *q == '-') && q > p_ && (q[-1] == 'e' || q[-1] == 'E'))))
                q++;
            char buf[72];
            const size_t m = size_t(q - p_);
            std::memcpy(buf, p_, m);
            buf[m] = 0;
            char *e = nullptr;
            t.v = std::strtod(buf, &e);
            p_ += (e - buf);
            return t;
        }
        if (c == '"') {
            const char *b = ++p_;
            while (p_ < end_ && *p_ != '"') p_++;
            t.k = Tok::STR;
            t.s.assign(b, p_);
            if (p_ < end_) p_++;
            return t;
        }
        t.k = Tok::SYM;
        if (p_ + 1 < end_ && ((c == '-' && p_[1] == '>') || (c == '=' && p_[1] == '='))) {
            t.s.assign(p_, 2);
            p_ += 2;
        } else {
            t.s.assign(1, c);
            p_++;
        }
        return t;
    }

    const char *p_ = nullptr, *end_ = nullptr;
    int line_ = 1;
    const std::vector<Tok> *toks_ = nullptr;
    size_t ti_ = 0;
    Tok cur_;
    bool have_ = false;
};

struct Builtin {
    int kind, np, nq;
};

const std::unordered_map<std::string, Builtin> &builtins() {
    static const std::unordered_map<std::string, Builtin> b = {
        {"id", {QSIM_G_ID, 0, 1}},      {"h", {QSIM_G_H, 0, 1}},       {"x", {QSIM_G_X, 0, 1}},
        {"y", {QSIM_G_Y, 0, 1}},        {"z", {QSIM_G_Z, 0, 1}},       {"s", {QSIM_G_S, 0, 1}},
        {"sdg", {QSIM_G_SDG, 0, 1}},    {"t", {QSIM_G_T, 0, 1}},       {"tdg", {QSIM_G_TDG, 0, 1}},
        {"sx", {QSIM_G_SX, 0, 1}},      {"rx", {QSIM_G_RX, 1, 1}},     {"ry", {QSIM_G_RY, 1, 1}},
        {"rz", {QSIM_G_RZ, 1, 1}},      {"u1", {QSIM_G_U1, 1, 1}},     {"p", {QSIM_G_U1, 1, 1}},
        {"u2", {QSIM_G_U2, 2, 1}},      {"u3", {QSIM_G_U3, 3, 1}},     {"u", {QSIM_G_U3, 3, 1}},
        {"U", {QSIM_G_U3, 3, 1}},       {"cx", {QSIM_G_CX, 0, 2}},     {"CX", {QSIM_G_CX, 0, 2}},
        {"cy", {QSIM_G_CY, 0, 2}},      {"cz", {QSIM_G_CZ, 0, 2}},     {"ch", {QSIM_G_CH, 0, 2}},
        {"swap", {QSIM_G_SWAP, 0, 2}},  {"crx", {QSIM_G_CRX, 1, 2}},   {"cry", {QSIM_G_CRY, 1, 2}},
        {"crz", {QSIM_G_CRZ, 1, 2}},    {"cu1", {QSIM_G_CU1, 1, 2}},   {"cp", {QSIM_G_CU1, 1, 2}},
        {"cu3", {QSIM_G_CU3, 3, 2}},    {"rxx", {QSIM_G_RXX, 1, 2}},   {"rzz", {QSIM_G_RZZ, 1, 2}},
        {"ccx", {QSIM_G_CCX, 0, 3}},    {"cswap", {QSIM_G_CSWAP, 0, 3}}, {"c3x", {QSIM_G_C3X, 0, 4}},
        {"c3sqrtx", {QSIM_G_C3XSQRTX, 0, 4}}, {"c4x", {QSIM_G_C4X, 0, 5}},
        {"rccx", {QSIM_G_RCCX, 0, 3}},  {"rc3x", {QSIM_G_RC3X, 0, 4}},
    };
    return b;
}

struct GateDef {
    std::vector<std::string> params, args;
    std::vector<Tok> body;
};

struct Reg {
    int offset, size;
};

struct ParseError {
    int code;
    int line;
    std::string msg;
};

class Parser {
  public:
    Parser(const char *text, size_t len, std::vector<qsim_gate> *out) : top_(text, len), out_(out) {}

    void program() {
        Lexer &L = top_;
        for (;;) {
            const Tok &t = L.peek();
            if (t.k == Tok::END) break;
            if (t.k != Tok::ID) fail(QSIM_E_ARG, L.line(), "statement expected");
            statement(L, nullptr, nullptr);
        }
    }
    int nq() const { return nq_; }
    int nc() const { return nc_; }

  private:
    [[noreturn]] void fail(int code, int line, const std::string &msg) { throw ParseError{code, line, msg}; }

    void expect(Lexer &L, const char *sym) {
        Tok t = L.next();
        if (t.k != Tok::SYM || t.s != sym) fail(QSIM_E_ARG, t.line, std::string("'") + sym + "' expected");
    }
    std::string ident(Lexer &L) {
        Tok t = L.next();
        if (t.k != Tok::ID) fail(QSIM_E_ARG, t.line, "identifier expected");
        return t.s;
    }
    bool accept(Lexer &L, const char *sym) {
        const Tok &t = L.peek();
        if (t.k == Tok::SYM && t.s == sym) {
            L.next();
            return true;
        }
        return false;
    }
    int integer(Lexer &L) {
        Tok t = L.next();
        if (t.k != Tok::NUM || t.v != std::floor(t.v) || t.v < 0 || t.v > 1e9)
            fail(QSIM_E_ARG, t.line, "non-negative integer expected");
        return int(t.v);
    }

    // ---- expressions (env: parameters of the gate being expanded)
    double expr(Lexer &L, const std::map<std::string, double> *env) {
        double v = term(L, env);
        for (;;) {
            if (accept(L, "+")) v += term(L, env);
            else if (accept(L, "-")) v -= term(L, env);
            else return v;
        }
    }
    double term(Lexer &L, const std::map<std::string, double> *env) {
        double v = power(L, env);
        for (;;) {
            if (accept(L, "*")) v *= power(L, env);
            else if (accept(L, "/")) v /= power(L, env);
            else return v;
        }
    }
    double power(Lexer &L, const std::map<std::string, double> *env) {
        const double b = unary(L, env);
        if (accept(L, "^")) return std::pow(b, power(L, env));   // right-associative
        return b;
    }
    double unary(Lexer &L, const std::map<std::string, double> *env) {
        if (accept(L, "-")) return -unary(L, env);
        if (accept(L, "+")) return unary(L, env);
        return primary(L, env);
    }
    double primary(Lexer &L, const std::map<std::string, double> *env) {
        Tok t = L.next();
        if (t.k == Tok::NUM) return t.v;
        if (t.k == Tok::SYM && t.s == "(") {
            const double v = expr(L, env);
            expect(L, ")");
            return v;
        }
        if (t.k == Tok::ID) {
            if (t.s == "pi") return M_PI;
            if (env) {
                auto it = env->find(t.s);
                if (it != env->end()) return it->second;
            }
            static const std::map<std::string, double (*)(double)> fn = {
                {"sin", [](double x) { return std::sin(x); }},  {"cos", [](double x) { return std::cos(x); }},
                {"tan", [](double x) { return std::tan(x); }},  {"exp", [](double x) { return std::exp(x); }},
                {"ln", [](double x) { return std::log(x); }},   {"sqrt", [](double x) { return std::sqrt(x); }},
            };
            auto f = fn.find(t.s);
            if (f != fn.end()) {
                expect(L, "(");
                const double v = expr(L, env);
                expect(L, ")");
                return f->second(v);
            }
            fail(QSIM_E_ARG, t.line, "unknown name '" + t.s + "' in expression");
        }
        fail(QSIM_E_ARG, t.line, "expression expected");
    }

    // ---- operands: a qubit, or a whole register (broadcast)
    struct Operand {
        int first, size;   // size 1 for an indexed qubit
    };
    Operand operand(Lexer &L, const std::map<std::string, Reg> &regs, const char *what) {
        const int line = L.line();
        const std::string name = ident(L);
        // the last register looked up (usually the same one, operand after operand)
        const Reg *r;
        if (&regs == last_map_ && name == last_name_) {
            r = &last_reg_;
        } else {
            auto it = regs.find(name);
            if (it == regs.end()) fail(QSIM_E_ARG, line, std::string("unknown ") + what + " '" + name + "'");
            last_map_ = &regs;
            last_name_ = name;
            last_reg_ = it->second;
            r = &last_reg_;
        }
        if (accept(L, "[")) {
            const int i = integer(L);
            expect(L, "]");
            if (i >= r->size) fail(QSIM_E_QUBIT, line, "index out of range of '" + name + "'");
            return {r->offset + i, 1};
        }
        return {r->offset, r->size};
    }
    const std::map<std::string, Reg> *last_map_ = nullptr;
    std::string last_name_;
    Reg last_reg_{0, 0};

    // small fixed-capacity lists of a call's parameters and qubits
    static constexpr int kMaxList = 16;
    struct Params {
        double v[kMaxList];
        int n = 0;
    };
    struct Qubits {
        int v[kMaxList];
        int n = 0;
    };

    void emit(int kind, const int *qs, int nq, const double *th, int np, int slot, int line) {
        qsim_gate g;
        std::memset(&g, 0, sizeof(g));
        g.kind = uint16_t(kind);
        g.nq = uint16_t(nq);
        for (int j = 0; j < nq && j < 5; j++) g.q[j] = qs[j];
        for (int j = 0; j < np && j < 3; j++) g.theta[j] = th[j];
        g.slot = slot;
        for (int a = 0; a < nq; a++)
            for (int b = 0; b < a; b++)
                if (qs[a] == qs[b]) fail(QSIM_E_QUBIT, line, "a gate names one qubit twice");
        out_->push_back(g);
    }
    void emit1(int kind, int q, int slot, int line) { emit(kind, &q, 1, nullptr, 0, slot, line); }

    // A gate call with evaluated parameters on resolved qubits.
    void call(const std::string &name, const Params &params, const Qubits &qs, int line, int depth) {
        auto b = builtins().find(name);
        if (b != builtins().end()) {
            if (params.n != b->second.np || qs.n != b->second.nq)
                fail(QSIM_E_ARG, line, "wrong number of parameters or qubits for '" + name + "'");
            emit(b->second.kind, qs.v, qs.n, params.v, params.n, -1, line);
            return;
        }
        auto d = defs_.find(name);
        if (d == defs_.end()) fail(QSIM_E_UNSUPPORTED, line, "unknown gate '" + name + "'");
        const GateDef &def = d->second;
        if (size_t(params.n) != def.params.size() || size_t(qs.n) != def.args.size())
            fail(QSIM_E_ARG, line, "wrong number of parameters or qubits for '" + name + "'");
        if (depth > 64) fail(QSIM_E_ARG, line, "gate definitions nested too deeply");
        std::map<std::string, double> env;
        for (int i = 0; i < params.n; i++) env[def.params[size_t(i)]] = params.v[i];
        std::map<std::string, int> amap;
        for (int i = 0; i < qs.n; i++) amap[def.args[size_t(i)]] = qs.v[i];
        Lexer B(&def.body);
        while (B.peek().k != Tok::END) statement(B, &env, &amap, depth + 1);
    }

    // One statement.  Inside a gate body env and amap are set: operands are
    // the definition's argument names and only gate calls and barriers occur.
    void statement(Lexer &L, const std::map<std::string, double> *env, const std::map<std::string, int> *amap,
                   int depth = 0) {
        const int line = L.line();
        const std::string kw = ident(L);
        if (!amap) {
            if (kw == "OPENQASM") {
                Tok v = L.next();
                if (v.k != Tok::NUM || v.v < 2.0 || v.v >= 3.0) fail(QSIM_E_UNSUPPORTED, line, "OPENQASM 2.x expected");
                expect(L, ";");
                return;
            }
            if (kw == "include") {
                Tok s = L.next();
                if (s.k != Tok::STR) fail(QSIM_E_ARG, line, "file name expected");
                expect(L, ";");
                return;
            }
            if (kw == "qreg" || kw == "creg") {
                const std::string name = ident(L);
                expect(L, "[");
                const int size = integer(L);
                expect(L, "]");
                expect(L, ";");
                auto &regs = kw == "qreg" ? qregs_ : cregs_;
                int &count = kw == "qreg" ? nq_ : nc_;
                if (regs.count(name) || size < 1) fail(QSIM_E_ARG, line, "bad or repeated register '" + name + "'");
                regs[name] = {count, size};
                count += size;
                last_map_ = nullptr;
                if (nq_ > kMaxQubits) fail(QSIM_E_CAPACITY, line, "too many qubits");
                return;
            }
            if (kw == "gate") {
                const std::string name = ident(L);
                if (builtins().count(name) || defs_.count(name))
                    fail(QSIM_E_ARG, line, "gate '" + name + "' defined twice");
                GateDef def;
                if (accept(L, "(")) {
                    if (!accept(L, ")")) {
                        do def.params.push_back(ident(L));
                        while (accept(L, ","));
                        expect(L, ")");
                    }
                }
                do def.args.push_back(ident(L));
                while (accept(L, ","));
                expect(L, "{");
                int level = 1;
                for (;;) {
                    Tok t = L.next();
                    if (t.k == Tok::END) fail(QSIM_E_ARG, line, "unterminated gate definition");
                    if (t.k == Tok::SYM && t.s == "{") level++;
                    if (t.k == Tok::SYM && t.s == "}" && --level == 0) break;
                    def.body.push_back(t);
                }
                defs_[name] = std::move(def);
                return;
            }
            if (kw == "opaque" || kw == "if") fail(QSIM_E_UNSUPPORTED, line, "'" + kw + "' is not supported");
            if (kw == "measure") {
                const Operand q = operand(L, qregs_, "qubit register");
                expect(L, "->");
                const Operand c = operand(L, cregs_, "classical register");
                expect(L, ";");
                if (q.size != c.size) fail(QSIM_E_ARG, line, "measure of registers of different sizes");
                for (int i = 0; i < q.size; i++) emit1(QSIM_G_MEASURE, q.first + i, c.first + i, line);
                return;
            }
            if (kw == "reset") {
                const Operand q = operand(L, qregs_, "qubit register");
                expect(L, ";");
                for (int i = 0; i < q.size; i++) emit1(QSIM_G_RESET, q.first + i, -1, line);
                return;
            }
        }
        if (kw == "barrier") {
            // a fusion fence; the operand list only needs to be well formed
            do {
                if (amap) ident(L);
                else operand(L, qregs_, "qubit register");
            } while (accept(L, ","));
            expect(L, ";");
            if (!amap) emit(QSIM_G_BARRIER, nullptr, 0, nullptr, 0, -1, line);
            return;
        }
        // a gate call
        Params params;
        if (accept(L, "(")) {
            if (!accept(L, ")")) {
                do {
                    if (params.n == kMaxList) fail(QSIM_E_ARG, line, "too many parameters");
                    params.v[params.n++] = expr(L, env);
                } while (accept(L, ","));
                expect(L, ")");
            }
        }
        if (amap) {
            Qubits qs;
            do {
                const int l2 = L.line();
                const std::string a = ident(L);
                auto it = amap->find(a);
                if (it == amap->end()) fail(QSIM_E_ARG, l2, "unknown argument '" + a + "'");
                if (qs.n == kMaxList) fail(QSIM_E_ARG, l2, "too many qubits");
                qs.v[qs.n++] = it->second;
            } while (accept(L, ","));
            expect(L, ";");
            call(kw, params, qs, line, depth);
            return;
        }
        Operand ops[kMaxList];
        int nops = 0;
        do {
            if (nops == kMaxList) fail(QSIM_E_ARG, line, "too many qubits");
            ops[nops++] = operand(L, qregs_, "qubit register");
        } while (accept(L, ","));
        expect(L, ";");
        int width = 1;
        for (int j = 0; j < nops; j++) {
            if (ops[j].size > 1) {
                if (width > 1 && ops[j].size != width) fail(QSIM_E_ARG, line, "broadcast over registers of different sizes");
                width = ops[j].size;
            }
        }
        Qubits qs;
        qs.n = nops;
        for (int i = 0; i < width; i++) {
            for (int j = 0; j < nops; j++) qs.v[j] = ops[j].first + (ops[j].size > 1 ? i : 0);
            call(kw, params, qs, line, 0);
        }
    }

    Lexer top_;
    std::vector<qsim_gate> *out_;
    std::map<std::string, Reg> qregs_, cregs_;
    std::map<std::string, GateDef> defs_;
    int nq_ = 0, nc_ = 0;
};

}  // namespace

int parse_qasm(const char *text, size_t len, std::vector<qsim_gate> *out, int *n_qubits, int *n_clbits,
               std::string *err) {
    out->clear();
    Parser P(text, len, out);
    try {
        P.program();
    } catch (const ParseError &e) {
        char buf[200];
        std::snprintf(buf, sizeof(buf), "qasm line %d: %s", e.line, e.msg.c_str());
        *err = buf;
        return e.code;
    }
    *n_qubits = P.nq();
    *n_clbits = P.nc();
    return QSIM_OK;
}

}  // namespace qs
