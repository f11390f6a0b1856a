// Host packing under AddressSanitizer / UndefinedBehaviorSanitizer: random
// instances of every constraint type (lengths up to the 1,024 maximum, repeated
// variables, weights or none), random shape and tile options, plain and
// block-diagonal batches.  Every packed instance is checked for the structure
// the kernels rely on: buckets partition the constraints, every slot holds the
// literal it came from, the variable-to-slot transpose is a permutation with
// ascending slots per variable, and every table row a constraint reads is
// inside the table and finite.  Exit status 0 and "ok <packed> <rejected>".
#include "host.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#define CHECK(cond, what)                                  \
    do {                                                   \
        if (!(cond)) {                                     \
            fprintf(stderr, "case %d: %s\n", it, what);    \
            return false;                                  \
        }                                                  \
    } while (0)

static bool check_packed(int it, const afs::HostInstance &H)
{
    int32_t c_next = 0;
    int64_t s_next = 0;
    for (const afs::Bucket &b : H.buckets) {
        CHECK(b.c0 == c_next && b.slot0 == s_next, "buckets are not contiguous");
        CHECK(b.J == 1 ? (b.S == b.k_lo && b.k_lo == b.k_hi) : (int64_t)b.J * b.S >= b.k_hi, "bucket shape");
        CHECK(b.tile >= 1 && (int64_t)b.ntiles * b.tile >= b.nc, "bucket tiles");
        CHECK(b.rpl == 0 || b.rpl == 1 || b.rpl == 2 || (b.rpl == 4 && b.J == 1 && b.S <= 8), "bucket restarts per lane");
        CHECK(b.J == 1 || b.rpl == 0, "restarts per lane on a segment bucket");
        for (int32_t c = b.c0; c < b.c0 + b.nc; ++c) {
            const int32_t o = H.bc_orig[c];
            CHECK(o >= 0 && o < H.C, "constraint index");
            const int k = (int)(H.con_off[o + 1] - H.con_off[o]);
            CHECK(H.bc_k[c] == k && k >= b.k_lo && k <= b.k_hi, "constraint length outside its bucket");
            CHECK(H.bc_slot0[c] >= b.slot0 && H.bc_slot0[c] + k <= b.slot0 + b.nslots, "slots outside the bucket");
            const int nroots = k / 2;
            CHECK(H.bc_tab[c] >= 0 && (size_t)H.bc_tab[c] + 1 + 2 * (size_t)nroots <= H.tab.size(), "table rows");
            for (int r = 0; r <= 2 * nroots; ++r) {
                const afs::TabRow &t = H.tab[H.bc_tab[c] + r];
                CHECK(std::isfinite(t.x) && std::isfinite(t.y) && std::isfinite(t.z) && std::isfinite(t.w),
                      "table value not finite");
            }
        }
        c_next += b.nc;
        s_next += b.nslots;
    }
    CHECK(c_next == H.C && s_next >= H.L, "buckets do not cover the constraints");
    std::vector<char> seen(H.C, 0);
    for (int32_t c = 0; c < H.C; ++c) {
        CHECK(!seen[H.bc_orig[c]], "constraint packed twice");
        seen[H.bc_orig[c]] = 1;
    }
    std::vector<char> lit_seen(H.L, 0);
    int64_t used = 0;
    for (size_t s = 0; s < H.slot_lit.size(); ++s) {
        const int32_t li = H.slot_to_lit[s];
        if (li < 0) continue;                      // padding slot
        CHECK(li < H.L && !lit_seen[li], "slot_to_lit is not a permutation");
        lit_seen[li] = 1;
        CHECK(H.slot_lit[s] == H.lits[li], "slot holds another literal");
        ++used;
    }
    CHECK(used == H.L, "literals missing from the slots");
    CHECK((int64_t)H.voff.size() == H.n + 1 && H.voff[0] == 0 && H.voff[H.n] == (int32_t)H.vslot.size(),
          "transpose offsets");
    CHECK((int64_t)H.vslot.size() == H.L, "transpose size");
    for (int32_t v = 0; v < H.n; ++v)
        for (int32_t i = H.voff[v]; i < H.voff[v + 1]; ++i) {
            const int32_t s = H.vslot[i];
            CHECK(s >= 0 && (size_t)s < H.slot_lit.size(), "transpose slot range");
            CHECK(std::abs(H.slot_lit[s]) - 1 == v, "transpose slot of another variable");
            CHECK(i == H.voff[v] || H.vslot[i - 1] < s, "transpose slots not ascending");
        }
    return true;
}

int main(int argc, char **argv)
{
    const int iters = argc > 1 ? atoi(argv[1]) : 300;
    std::mt19937_64 rng(argc > 2 ? strtoull(argv[2], nullptr, 10) : 777);
    long packed = 0, rejected = 0;
    for (int it = 0; it < iters; ++it) {
        const int n = 1 + (int)(rng() % 2000);
        const int C = (int)(rng() % 300);
        std::vector<int64_t> off{0};
        std::vector<int32_t> lits, types, params;
        std::vector<float> w;
        for (int c = 0; c < C; ++c) {
            const int r = (int)(rng() % 100);
            const int k = r < 60 ? 1 + (int)(rng() % 10)
                        : r < 95 ? 11 + (int)(rng() % 250)
                                 : 261 + (int)(rng() % (rng() % 50 ? 764 : 800));   // now and then too long
            for (int i = 0; i < k; ++i) {
                const int v = 1 + (int)(rng() % n);
                lits.push_back(rng() % 2 ? v : -v);
            }
            off.push_back((int64_t)lits.size());
            const int t = (int)(rng() % 8);
            types.push_back(t);
            params.push_back(t == 1 ? (int)(rng() % 2) : (t == 3 || t == 4 || t == 7) ? (int)(rng() % (k + 3)) - 1 : 0);
            w.push_back(0.25f + (float)(rng() % 8));
        }
        afs::PackOptions o;
        if (rng() % 3 == 0) {
            int kh = afs::kShortMax;
            const int nb = 1 + (int)(rng() % 4);
            const bool tiles = rng() % 2;
            for (int b = 0; b < nb; ++b) {
                const int J = 1 << (1 + (int)(rng() % 6));
                const int S = afs::kMinSeg + 2 * (int)(rng() % ((afs::kMaxSeg - afs::kMinSeg) / 2 + 1));
                const int next = std::min(J * S, kh + 1 + (int)(rng() % 300));
                if (next <= kh) break;
                kh = next;
                o.k_hi.push_back(kh);
                o.lanes.push_back(J);
                o.seg.push_back(S);
                if (tiles) o.tile.push_back((int)(rng() % 17));
            }
        }
        if (rng() % 4 == 0) o.tile_short = 1 + (int)(rng() % 64);
        if (rng() % 4 == 0) o.tile_long = 1 + (int)(rng() % 64);
        if (rng() % 3 == 0)
            for (int k = 1; k <= afs::kShortMax; ++k) {
                o.short_tile[k] = (int)(rng() % 20);
                const int r = (int)(rng() % 4);
                o.short_rpl[k] = r == 3 ? (k <= 8 ? 4 : 2) : r;      // 0, 1, 2, or 4 where allowed
            }
        if (!afs::check_options(o).empty()) {
            ++rejected;
            continue;
        }
        afs::HostInstance H;
        const std::string msg = afs::build_instance(n, C, off.data(), lits.data(), types.data(), params.data(),
                                                    rng() % 2 ? w.data() : nullptr, o, H);
        if (!msg.empty()) {
            ++rejected;
            continue;
        }
        ++packed;
        if (!check_packed(it, H)) return 1;
        if (it % 5 == 0) {
            std::vector<afs::PartRef> parts(1 + (int)(rng() % 3));
            for (afs::PartRef &p : parts) {
                p.n = n;
                p.C = C;
                p.con_off = off.data();
                p.lits = lits.data();
                p.types = types.data();
                p.params = params.data();
                p.weights = w.data();
            }
            afs::HostInstance Hb;
            if (afs::build_batch(parts, o, Hb).empty() && !check_packed(it, Hb)) return 1;
        }
    }
    printf("ok %ld %ld\n", packed, rejected);
    return 0;
}
