// Reader under AddressSanitizer / UndefinedBehaviorSanitizer (host code only):
// random token streams and mutated structured inputs through every reader
// entry point, with the invariants afs_parsed_arrays promises checked on every
// accepted input.  Exit status 0 and "ok <accepted> <rejected>" on success.
#include "afsat.h"

#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

namespace afs {
afs_status set_last_error(afs_status s, const std::string &) { return s; }
}

static std::string random_tokens(std::mt19937_64 &rng)
{
    static const char *vocab[] = {
        "p", "cnf", "h", "x", "xor", "n", "nae", "a", "amo", "e", "eo", "k", "ek", "d", "card", ">=", ">",
        "<", "<=", "0", "1", "2", "3", "-1", "-2", "-3", "5", "-7", "10", "%", "c", "*", "\n", "\n", " ", "\t",
        "\r\n", "99999999999", "-2147483648", "2147483648", "4294967297", "1e3", "+3", "--2", ">=2", "<3",
        "abc", "p cnf 5 3\n", "p cnf 0 0\n", "p cnf -1 2\n", "p cnf 3000000 1\n", "0\n", "h x 1 2 3 0\n",
        "h d 2 1 2 3 0\n", "h k 0 1 2 0\n", "h d -2 1 2 0\n", "1 -1 0\n", "1 0\n-1 0\n"};
    const int nv = (int)(sizeof(vocab) / sizeof(vocab[0]));
    std::string s;
    const int ntok = 1 + (int)(rng() % 60);
    for (int t = 0; t < ntok; ++t) {
        const int r = (int)(rng() % 100);
        if (r < 85) {
            s += vocab[rng() % nv];
            if (rng() % 3) s += ' ';
        } else if (r < 95) {
            s += std::to_string((long long)(rng() % 41) - 20) + " ";
        } else {
            s += (char)(rng() % 256);
        }
    }
    return s;
}

static std::string structured(std::mt19937_64 &rng)
{
    static const char *types[] = {"", "x ", "xor ", "n ", "a ", "e ", "k ", "ek ", "d ", "card "};
    static const char *ops[] = {"", ">= ", "> ", "< ", "<= ", ">=", "<"};
    const int n = 1 + (int)(rng() % 12), m = (int)(rng() % 15);
    std::string s;
    if (rng() % 4) s += "p cnf " + std::to_string(n) + " " + std::to_string(m) + "\n";
    for (int c = 0; c < m; ++c) {
        const int t = (int)(rng() % 10);
        if (t || rng() % 2) s += "h ";
        s += types[t];
        if (t == 6 || t == 7) s += std::to_string((int)(rng() % 7) - 1) + " ";
        if (t == 8 || t == 9) s += std::string(ops[rng() % 7]) + std::to_string((int)(rng() % 9) - 3) + " ";
        const int k = (int)(rng() % 7);
        for (int i = 0; i < k; ++i) {
            const int v = 1 + (int)(rng() % (n + (rng() % 8 == 0)));
            s += std::to_string(rng() % 2 ? v : -v);
            s += (rng() % 10 == 0) ? "\n" : " ";
        }
        s += "0";
        if (rng() % 8 == 0) s += " trailing";
        s += "\n";
        if (rng() % 20 == 0) s += "c comment\n";
    }
    if (rng() % 10 == 0) s += "%\n0\n";
    const int mut = (int)(rng() % 3);
    for (int i = 0; i < mut && !s.empty(); ++i) s[rng() % s.size()] = "0123456789- \nhx%"[rng() % 16];
    return s;
}

#define CHECK(cond, what)                                             \
    do {                                                              \
        if (!(cond)) {                                                \
            fprintf(stderr, "case %d: %s\n", it, what);               \
            return 1;                                                 \
        }                                                             \
    } while (0)

int main(int argc, char **argv)
{
    const int iters = argc > 1 ? atoi(argv[1]) : 100000;
    std::mt19937_64 rng(argc > 2 ? strtoull(argv[2], nullptr, 10) : 12345);
    long accepted = 0, rejected = 0;
    for (int it = 0; it < iters; ++it) {
        const std::string s = it % 2 ? structured(rng) : random_tokens(rng);
        afs_parsed *p = nullptr;
        if (afs_parse_text(s.data(), s.size(), &p) != AFS_OK) {
            CHECK(p == nullptr, "output handle set on error");
            ++rejected;
            continue;
        }
        ++accepted;
        afs_parsed_info inf;
        CHECK(afs_parsed_get_info(p, &inf) == AFS_OK, "afs_parsed_get_info");
        if (inf.n_vars > 1000000) {    // a large declared count: nothing of that size to check here
            afs_parsed_destroy(p);
            continue;
        }
        std::vector<int64_t> off(inf.n_cons + 1);
        std::vector<int32_t> lits(inf.n_lits + 1), types(inf.n_cons + 1), params(inf.n_cons + 1);
        std::vector<int8_t> units(inf.n_vars + 1);
        CHECK(afs_parsed_arrays(p, off.data(), lits.data(), types.data(), params.data(), units.data()) == AFS_OK,
              "afs_parsed_arrays");
        CHECK(off[0] == 0 && off[inf.n_cons] == inf.n_lits, "offsets");
        for (int32_t c = 0; c < inf.n_cons; ++c) CHECK(off[c + 1] > off[c], "empty constraint kept");
        for (int64_t i = 0; i < inf.n_lits; ++i)
            CHECK(lits[i] != 0 && std::llabs((long long)lits[i]) <= inf.n_vars, "literal out of range");
        int32_t nu = 0;
        for (int32_t v = 0; v < inf.n_vars; ++v) {
            CHECK(units[v] >= -1 && units[v] <= 1, "unit value");
            nu += units[v] != 0;
        }
        CHECK(nu == inf.n_units, "unit count");
        // fold into two rows, the first free, the second random: the free row
        // must come back equal to the units
        std::vector<int8_t> vals(2 * (size_t)inf.n_vars + 1, 0);
        for (int32_t v = 0; v < inf.n_vars; ++v) vals[inf.n_vars + v] = (int8_t)((int)(rng() % 3) - 1);
        if (afs_parsed_fold_units(p, 2, vals.data()) == AFS_OK)
            for (int32_t v = 0; v < inf.n_vars; ++v) CHECK(vals[v] == units[v], "folded units");
        afs_parsed_destroy(p);
    }
    printf("ok %ld %ld\n", accepted, rejected);
    return 0;
}
