// Long-constraint decomposition under AddressSanitizer / UndefinedBehaviorSanitizer:
// random instances (chain types up to 3,000 literals, every other type within the
// kernels' limit, repeated variables, weights or none) through afs_decompose_size
// and afs_decompose at random piece lengths; the result must have the announced
// sizes, pieces within the length, the input's literals in order, and pack.
// Exit status 0 and "ok <decomposed> <rejected>".
#include "afsat.h"
#include "host.hpp"

#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

namespace afs {
afs_status set_last_error(afs_status s, const std::string &) { return s; }
}

int main(int argc, char **argv)
{
    const int iters = argc > 1 ? atoi(argv[1]) : 300;
    std::mt19937_64 rng(argc > 2 ? strtoull(argv[2], nullptr, 10) : 99);
    long done = 0, rejected = 0;
    for (int it = 0; it < iters; ++it) {
        const int n = 1 + (int)(rng() % 3000);
        const int C = (int)(rng() % 120);
        std::vector<int64_t> off{0};
        std::vector<int32_t> lits, types, params;
        std::vector<float> w;
        for (int c = 0; c < C; ++c) {
            const int t = (int)(rng() % 8);
            const bool chain = t == AFS_OR || t == AFS_XOR || t == AFS_NAE || t == AFS_AMO || t == AFS_EO;
            const int k = 1 + (int)(rng() % (chain && rng() % 3 == 0 ? 3000 : 200));
            for (int i = 0; i < k; ++i) {
                const int v = 1 + (int)(rng() % n);
                lits.push_back(rng() % 2 ? v : -v);
            }
            off.push_back((int64_t)lits.size());
            types.push_back(t);
            params.push_back(t == AFS_XOR ? (int)(rng() % 2) : (int)(rng() % (k + 3)) - 1);
            w.push_back(0.5f + (float)(rng() % 4));
        }
        if (rng() % 20 == 0 && !lits.empty()) lits[rng() % lits.size()] = (rng() % 2) ? 0 : n + 1;   // invalid
        const int32_t L = rng() % 10 == 0 ? (int32_t)(rng() % 1100) : 3 + (int32_t)(rng() % 60);
        const float *wp = rng() % 2 ? w.data() : nullptr;
        int32_t n_out = -1, c_out = -1;
        int64_t l_out = -1;
        if (afs_decompose_size(n, C, off.data(), types.data(), L, &n_out, &c_out, &l_out) != AFS_OK) {
            ++rejected;
            continue;
        }
        std::vector<int64_t> co(c_out + 1, -7);
        std::vector<int32_t> lo(l_out), to(c_out), po(c_out), og(c_out);
        std::vector<float> wo(c_out);
        if (afs_decompose(n, C, off.data(), lits.data(), types.data(), params.data(), wp, L, co.data(), lo.data(),
                          to.data(), po.data(), wp ? wo.data() : nullptr, og.data()) != AFS_OK) {
            ++rejected;
            continue;
        }
        ++done;
        auto fail = [&](const char *what) {
            fprintf(stderr, "case %d: %s\n", it, what);
            return 1;
        };
        if (co[0] != 0 || co[c_out] != l_out) return fail("offsets");
        int64_t maxk_in = 0;
        for (int c = 0; c < C; ++c) maxk_in = std::max(maxk_in, off[c + 1] - off[c]);
        // the input's literals, in order, are the non-link literals of its pieces
        int32_t c_in = -1;
        int64_t pos = 0;
        for (int32_t c = 0; c < c_out; ++c) {
            const int64_t k = co[c + 1] - co[c];
            if (k < 1) return fail("empty piece");
            if (og[c] < c_in || og[c] >= C) return fail("origin order");
            if (og[c] != c_in) {
                if (c_in >= 0 && pos != off[c_in + 1]) return fail("literals lost");
                c_in = og[c];
                pos = off[c_in];
            }
            if (to[c] != types[c_in]) return fail("type");
            if (wp && wo[c] != w[c_in]) return fail("weight");
            const bool split = off[c_in + 1] - off[c_in] != k || (c + 1 < c_out && og[c + 1] == c_in) ||
                               (c > 0 && og[c - 1] == c_in);
            if (split && k > L) return fail("piece longer than max_len");
            for (int64_t i = co[c]; i < co[c + 1]; ++i) {
                const int32_t l = lo[i];
                if (l == 0 || std::abs(l) > n_out) return fail("literal range");
                if (std::abs(l) > n) continue;           // a link
                if (pos >= off[c_in + 1] || lits[pos] != l) return fail("literal order");
                ++pos;
            }
        }
        if (C > 0 && (c_in != C - 1 || pos != off[C])) return fail("constraints lost");
        // the result packs when every piece is within the kernels' limit
        bool fits = true;
        for (int32_t c = 0; c < c_out; ++c) fits = fits && co[c + 1] - co[c] <= AFS_MAX_LEN;
        if (fits && c_out > 0) {
            afs::HostInstance H;
            const std::string msg = afs::build_instance(n_out, c_out, co.data(), lo.data(), to.data(), po.data(),
                                                        wp ? wo.data() : nullptr, afs::PackOptions(), H);
            if (!msg.empty()) return fail(msg.c_str());
        }
    }
    printf("ok %ld %ld\n", done, rejected);
    return 0;
}
