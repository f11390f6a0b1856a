// parse.cpp -- reader of DIMACS CNF and of the hybrid symmetric-constraint
// format of App. A, with the automatic simplifications listed there.
//
// Lines: comments ('c' or '*' first), the problem line "p cnf <vars> <cons>",
// and constraints: an optional 'h' marker, an optional type identifier and
// literals, terminated by 0; text after the terminating 0 on the same line is a
// comment, and a constraint may continue over several lines.  A line holding
// only '%' ends the input (some DIMACS collections end that way).
//   (none)        OR                 x / xor   XOR, odd parity
//   n / nae       NAE                a / amo   AMO
//   e / eo        EO                 k / ek K  exactly K
//   d / card T    cardinality, T one of: K (K > 0: >= K; K < 0: < |K|),
//                 >= K, > K (>= K+1), < K, <= K (< K+1)
// Simplification (App. A, "Automatic Simplification"):
//   - a one-literal OR or EO fixes that literal True (a unit);
//   - a one-literal AMO is dropped (always satisfied);
//   - CARD >= 1 becomes OR, EK 1 becomes EO;
//   - CARD >= k and EK k over k literals fix every literal True;
//   - CARD >= 0 is dropped; EK 0 fixes every literal False;
//   - two units fixing one variable to both values raise AFS_EUNSAT.
// Beyond those: a threshold no assignment meets (CARD >= K or EK K with K above
// the length, CARD < K with K <= 0, EK K with K < 0) raises AFS_EUNSAT, and
// CARD < K with K above the length (always met) is dropped.  A plain threshold
// of 0 reads as ">= 0".
// Units are reported, not propagated further: constraints are kept as read, and
// the solver holds the fixed variables at their values (Sec. 3.4).

#include "afsat.h"

#include <algorithm>
#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "instance.hpp"

struct afs_parsed {
    int32_t n = 0;                 // variables (from the problem line, else the largest index)
    int32_t declared_cons = -1;    // constraint count of the problem line (-1: none)
    std::vector<int64_t> con_off{0};
    std::vector<int32_t> lits, types, params;
    std::vector<int8_t> unit;      // per variable: 0 free, +1 fixed True, -1 fixed False
    int32_t n_units = 0;
    int32_t dropped = 0;           // constraints removed by simplification
};

namespace {

using afs::set_last_error;

bool parse_int(const std::string &t, long long &v)
{
    if (t.empty()) return false;
    char *end = nullptr;
    errno = 0;
    v = std::strtoll(t.c_str(), &end, 10);
    return errno == 0 && end && *end == '\0';
}

struct Pending {
    bool open = false;
    int type = AFS_OR;
    bool has_param = false;
    long long param = 0;           // normalised: CARD >= K (type CARD_GE) or < K (CARD_LT), EK K
    std::vector<int32_t> lits;
    int line = 0;
};

struct Reader {
    afs_parsed &P;
    std::string err;
    bool unsat = false;            // the error proves the instance unsatisfiable
    explicit Reader(afs_parsed &p) : P(p) {}

    bool fail(int line, const std::string &msg)
    {
        err = "line " + std::to_string(line) + ": " + msg;
        return false;
    }

    // fix literal l True (l > 0: variable True, l < 0: variable False)
    bool fix(int32_t l, int line)
    {
        const int32_t v = (l > 0 ? l : -l) - 1;
        if ((int32_t)P.unit.size() <= v) P.unit.resize(v + 1, 0);
        const int8_t want = l > 0 ? 1 : -1;
        if (P.unit[v] == -want) {
            unsat = true;
            return fail(line, "conflicting unit literals on variable " + std::to_string(v + 1));
        }
        if (P.unit[v] == 0) {
            P.unit[v] = want;
            ++P.n_units;
        }
        return true;
    }

    void emit(int type, long long param, const std::vector<int32_t> &lits)
    {
        P.lits.insert(P.lits.end(), lits.begin(), lits.end());
        P.con_off.push_back((int64_t)P.lits.size());
        P.types.push_back(type);
        P.params.push_back((int32_t)param);
    }

    // apply the simplifications, then keep or drop the constraint
    bool finish(const Pending &c)
    {
        const int k = (int)c.lits.size();
        if (k == 0) return fail(c.line, "constraint without literals");
        int type = c.type;
        long long K = c.param;
        if (type == AFS_CARD_GE && K == 1) type = AFS_OR;                 // CARD-1 -> CNF
        if (type == AFS_EK && K == 1) type = AFS_EO;                      // EK-1 -> EO
        if (type == AFS_CARD_GE && K <= 0) { ++P.dropped; return true; }  // CARD-0: always true
        if (type == AFS_AMO && k == 1) { ++P.dropped; return true; }      // unit AMO
        // thresholds no assignment can meet
        if ((type == AFS_CARD_GE && K > k) || (type == AFS_CARD_LT && K <= 0) ||
            (type == AFS_EK && (K < 0 || K > k))) {
            unsat = true;
            return fail(c.line, "constraint can never be satisfied");
        }
        if (type == AFS_CARD_LT && K > k) { ++P.dropped; return true; }   // always true
        if ((type == AFS_OR || type == AFS_EO) && k == 1) {               // unit CNF / EO
            ++P.dropped;
            return fix(c.lits[0], c.line);
        }
        if ((type == AFS_CARD_GE || type == AFS_EK) && K == k) {          // CARD-n, EK-n
            ++P.dropped;
            for (int32_t l : c.lits)
                if (!fix(l, c.line)) return false;
            return true;
        }
        if (type == AFS_EK && K == 0) {                                   // EK-0: all False
            ++P.dropped;
            for (int32_t l : c.lits)
                if (!fix(-l, c.line)) return false;
            return true;
        }
        if (type == AFS_XOR) K = 1;                                       // odd parity
        if (type != AFS_XOR && type != AFS_CARD_GE && type != AFS_CARD_LT && type != AFS_EK) K = 0;
        if (K < INT32_MIN || K > INT32_MAX) return fail(c.line, "threshold out of range");
        emit(type, K, c.lits);
        return true;
    }

    // threshold of a cardinality constraint -> (type, K).  The operator may be
    // written apart from its number ("d >= 2") or joined to it ("d >=2").
    bool card_threshold(const std::string &t, std::istringstream &ss, int line, int &type, long long &K)
    {
        std::string op, num = t;
        for (const char *o : {">=", "<=", ">", "<"}) {
            const size_t n = std::strlen(o);
            if (t.compare(0, n, o) == 0) {
                op = o;
                num = t.substr(n);
                break;
            }
        }
        if (!op.empty() && num.empty() && !(ss >> num)) return fail(line, "missing cardinality threshold");
        long long v = 0;
        if (!parse_int(num, v)) return fail(line, "bad cardinality threshold '" + t + "'");
        if (!op.empty() && v < 0) return fail(line, "negative threshold after an operator");
        if (op.empty()) {                                                 // plain: K > 0 >= K, K < 0 < |K|
            type = v >= 0 ? AFS_CARD_GE : AFS_CARD_LT;
            K = v >= 0 ? v : -v;
        } else if (op == ">=") { type = AFS_CARD_GE; K = v; }
        else if (op == ">") { type = AFS_CARD_GE; K = v + 1; }
        else if (op == "<") { type = AFS_CARD_LT; K = v; }
        else { type = AFS_CARD_LT; K = v + 1; }                          // <=
        return true;
    }

    bool run(std::istream &in)
    {
        std::string line;
        int lineno = 0;
        Pending c;
        bool seen_problem = false;
        while (std::getline(in, line)) {
            ++lineno;
            std::istringstream ss(line);
            std::string tok;
            if (!(ss >> tok)) continue;                                   // blank line
            if (!c.open) {
                if (tok == "c" || tok[0] == '*' || (tok[0] == 'c' && tok != "card")) continue;   // comment
                if (tok == "%") break;
                if (tok == "p") {
                    std::string fmt, a, b;
                    long long nv = 0, nc = 0;
                    if (!(ss >> fmt >> a >> b) || fmt != "cnf" || !parse_int(a, nv) || !parse_int(b, nc) || nv < 0 ||
                        nc < 0 || nv > INT32_MAX || nc > INT32_MAX)
                        return fail(lineno, "bad problem line");
                    if (seen_problem) return fail(lineno, "second problem line");
                    seen_problem = true;
                    P.n = (int32_t)nv;
                    P.declared_cons = (int32_t)nc;
                    continue;
                }
            }
            // constraint tokens (possibly continuing a constraint from earlier lines)
            bool more = true;
            while (more) {
                if (!c.open) {
                    c = Pending();
                    c.open = true;
                    c.line = lineno;
                    if (tok == "h") {
                        if (!(ss >> tok)) { more = false; break; }
                    }
                    if (tok == "x" || tok == "xor") c.type = AFS_XOR;
                    else if (tok == "n" || tok == "nae") c.type = AFS_NAE;
                    else if (tok == "a" || tok == "amo") c.type = AFS_AMO;
                    else if (tok == "e" || tok == "eo") c.type = AFS_EO;
                    else if (tok == "k" || tok == "ek" || tok == "d" || tok == "card") {
                        const bool ek = tok == "k" || tok == "ek";
                        std::string th;
                        if (!(ss >> th)) return fail(lineno, "missing threshold");
                        if (ek) {
                            long long v = 0;
                            if (!parse_int(th, v)) return fail(lineno, "bad EK count '" + th + "'");
                            c.type = AFS_EK;
                            c.param = v;
                        } else if (!card_threshold(th, ss, lineno, c.type, c.param)) {
                            return false;
                        }
                    } else {
                        long long v = 0;
                        if (!parse_int(tok, v)) return fail(lineno, "unexpected token '" + tok + "'");
                        if (v == 0) return fail(lineno, "empty constraint");
                        c.type = AFS_OR;
                        if (v < -INT32_MAX || v > INT32_MAX) return fail(lineno, "literal out of range");
                        if (seen_problem && (v > P.n || -v > P.n))
                            return fail(lineno, "variable " + std::to_string(v > 0 ? v : -v) +
                                                    " exceeds the problem line's " + std::to_string(P.n));
                        c.lits.push_back((int32_t)v);
                    }
                    if (!(ss >> tok)) { more = false; break; }
                }
                long long v = 0;
                if (!parse_int(tok, v)) return fail(lineno, "unexpected token '" + tok + "'");
                if (v == 0) {
                    c.open = false;
                    if (!finish(c)) return false;
                    more = false;                                         // rest of the line: comment
                    break;
                }
                if (v < -INT32_MAX || v > INT32_MAX) return fail(lineno, "literal out of range");
                if (seen_problem && (v > P.n || -v > P.n))
                    return fail(lineno, "variable " + std::to_string(v > 0 ? v : -v) + " exceeds the problem line's " +
                                            std::to_string(P.n));
                c.lits.push_back((int32_t)v);
                if (!(ss >> tok)) more = false;
            }
        }
        if (c.open) return fail(c.line, "constraint not terminated by 0");
        int32_t maxv = 0;
        for (int32_t l : P.lits) maxv = std::max(maxv, l > 0 ? l : -l);
        maxv = std::max(maxv, (int32_t)P.unit.size());
        if (seen_problem && maxv > P.n) return fail(lineno, "variable " + std::to_string(maxv) + " exceeds the problem line's " + std::to_string(P.n));
        if (!seen_problem) P.n = maxv;
        P.unit.resize(P.n, 0);
        return true;
    }
};

afs_status parse_stream(std::istream &in, afs_parsed **out)
{
    afs_parsed *P = new (std::nothrow) afs_parsed();
    if (!P) return set_last_error(AFS_ENOMEM, "host allocation failed");
    Reader r(*P);
    bool ok = false;
    try {
        ok = r.run(in);
    } catch (const std::bad_alloc &) {
        delete P;
        return set_last_error(AFS_ENOMEM, "host allocation failed");
    }
    if (!ok) {
        delete P;
        return set_last_error(r.unsat ? AFS_EUNSAT : AFS_EINVAL, r.err);
    }
    *out = P;
    return AFS_OK;
}

}  // namespace

extern "C" {

afs_status afs_parse_text(const char *text, size_t len, afs_parsed **out)
{
    if (!out || (!text && len)) return set_last_error(AFS_EINVAL, "text or out is NULL");
    *out = nullptr;
    std::istringstream in(std::string(text ? text : "", len));
    return parse_stream(in, out);
}

afs_status afs_parse_file(const char *path, afs_parsed **out)
{
    if (!out || !path) return set_last_error(AFS_EINVAL, "path or out is NULL");
    *out = nullptr;
    std::ifstream in(path);
    if (!in) return set_last_error(AFS_EINVAL, std::string("cannot open ") + path);
    return parse_stream(in, out);
}

afs_status afs_parsed_get_info(const afs_parsed *p, afs_parsed_info *out)
{
    if (!p || !out) return set_last_error(AFS_EINVAL, "NULL argument");
    out->n_vars = p->n;
    out->n_cons = (int32_t)p->types.size();
    out->n_lits = (int64_t)p->lits.size();
    out->n_units = p->n_units;
    out->n_dropped = p->dropped;
    out->declared_cons = p->declared_cons;
    return AFS_OK;
}

afs_status afs_parsed_arrays(const afs_parsed *p, int64_t *con_off, int32_t *lits, int32_t *types,
                             int32_t *params, int8_t *units)
{
    if (!p) return set_last_error(AFS_EINVAL, "NULL argument");
    if (con_off) std::memcpy(con_off, p->con_off.data(), p->con_off.size() * sizeof(int64_t));
    if (lits && !p->lits.empty()) std::memcpy(lits, p->lits.data(), p->lits.size() * sizeof(int32_t));
    if (types && !p->types.empty()) std::memcpy(types, p->types.data(), p->types.size() * sizeof(int32_t));
    if (params && !p->params.empty()) std::memcpy(params, p->params.data(), p->params.size() * sizeof(int32_t));
    if (units && !p->unit.empty()) std::memcpy(units, p->unit.data(), p->unit.size() * sizeof(int8_t));
    return AFS_OK;
}

void afs_parsed_destroy(afs_parsed *p)
{
    delete p;
}

afs_status afs_parsed_fold_units(const afs_parsed *p, int32_t n_partial, int8_t *values)
{
    if (!p || (!values && n_partial > 0)) return set_last_error(AFS_EINVAL, "NULL argument");
    if (n_partial < 0) return set_last_error(AFS_EINVAL, "n_partial must be >= 0");
    const int64_t n = p->n;
    for (int32_t r = 0; r < n_partial; ++r) {
        int8_t *row = values + (int64_t)r * n;
        for (int64_t v = 0; v < n; ++v) {
            const int8_t u = p->unit[(size_t)v];
            if (!u) continue;
            if (row[v] && (row[v] > 0) != (u > 0))
                return set_last_error(AFS_EUNSAT, "partial assignment " + std::to_string(r) +
                                                      " contradicts the unit on variable " + std::to_string(v + 1));
            row[v] = u;
        }
    }
    return AFS_OK;
}

}  // extern "C"
