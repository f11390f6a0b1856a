// host.cpp -- host-side instance packing (see host.hpp).
#include "host.hpp"

#include "afsat.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <numeric>
#include <tuple>

namespace afs {

int satisfied(int type, int k, int param, int t)
{
    switch (type) {
    case 0: return t >= 1;                       // OR
    case 1: return (t & 1) == (param & 1);       // XOR, param = parity
    case 2: return t > 0 && t < k;               // NAE
    case 3: return t >= param;                   // CARD >= K
    case 4: return t < param;                    // CARD < K
    case 5: return t <= 1;                       // AMO
    case 6: return t == 1;                       // EO
    case 7: return t == param;                   // EK
    default: return -1;
    }
}

static bool uses_param(int type) { return type == 1 || type == 3 || type == 4 || type == 7; }

// Parameter reduced to a canonical value with the same truth table, so equal
// tables are shared.
static int canonical_param(int type, int k, int param)
{
    switch (type) {
    case 1: return param & 1;
    case 3:
    case 4: return std::min(std::max(param, 0), k + 1);
    case 7: return (param < 0 || param > k) ? k + 1 : param;
    default: return 0;
    }
}

// Roots of unity of order N for j = 0..N-1, computed for j <= N/2 and mirrored
// (conj) above, with exact values at the axis crossings.
void roots(int N, std::vector<long double> &c, std::vector<long double> &s)
{
    c.assign(N, 0.0L);
    s.assign(N, 0.0L);
    const long double two_pi = 6.283185307179586476925286766559005768L;
    for (int j = 0; 2 * j <= N; ++j) {
        long double cj, sj;
        if (j == 0) { cj = 1.0L; sj = 0.0L; }
        else if (2 * j == N) { cj = -1.0L; sj = 0.0L; }
        else if (4 * j == N) { cj = 0.0L; sj = 1.0L; }
        else {
            const long double th = two_pi * (long double)j / (long double)N;
            cj = cosl(th);
            sj = sinl(th);
        }
        c[j] = cj;
        s[j] = sj;
        if (j > 0 && 2 * j != N) { c[N - j] = cj; s[N - j] = -sj; }
    }
}

// d_m = (1/N) sum_t g(t) omega^(-m t).  A truth table is piecewise constant in t
// (two or three runs for every type but XOR), and over a run [a, b) of value v
// the sum is geometric: v (omega^(-m a) - omega^(-m b)) / (1 - omega^(-m)) for
// m != 0, so each coefficient costs O(runs) rather than O(N).  XOR alternates
// in t, which is geometric in -omega^(-m) over the whole range.  Powers of omega
// come from the mirrored root table with the exponent reduced mod N, so
// d_{N-m} = conj(d_m) exactly; everything is in long double and rounded once.
void coefficients(int type, int k, int param, double *re, double *im)
{
    const int N = k + 1;
    std::vector<long double> c, s;
    roots(N, c, s);
    std::vector<int> g(N);
    for (int t = 0; t <= k; ++t) g[t] = satisfied(type, k, param, t) == 1 ? -1 : 1;
    std::vector<int> start;                          // first t of each run of equal g
    for (int t = 0; t <= k; ++t)
        if (t == 0 || g[t] != g[t - 1]) start.push_back(t);
    const int runs = (int)start.size();
    // omega^(-j) for any integer j >= 0
    auto wneg = [&](int64_t j, long double &wr, long double &wi) {
        const int r = (int)(j % N);
        wr = c[r];
        wi = -s[r];
    };
    for (int m = 0; m <= k; ++m) {
        long double ar = 0.0L, ai = 0.0L;
        if (m == 0) {
            for (int t = 0; t <= k; ++t) ar += g[t];
        } else if (runs <= 8) {
            // sum over runs of v (w^a - w^b), then / (1 - w), w = omega^(-m)
            long double nr = 0.0L, ni = 0.0L;
            for (int q = 0; q < runs; ++q) {
                const int a = start[q], b = q + 1 < runs ? start[q + 1] : N;
                long double xr, xi, yr, yi;
                wneg((int64_t)m * a, xr, xi);
                wneg((int64_t)m * b, yr, yi);
                nr += g[a] * (xr - yr);
                ni += g[a] * (xi - yi);
            }
            long double dr, di;
            wneg(m, dr, di);
            dr = 1.0L - dr;                          // 1 - omega^(-m)
            di = -di;
            const long double den = dr * dr + di * di;
            ar = (nr * dr + ni * di) / den;
            ai = (ni * dr - nr * di) / den;
        } else if (type == AFS_XOR) {
            // g(t) = g(0) (-1)^t: g(0) sum_t (-w)^t = g(0) (1 - (-w)^N) / (1 + w), w = omega^(-m)
            long double wr, wi;
            wneg(m, wr, wi);
            if (2 * m == N) {
                ar = (long double)g[0] * N;          // -w = 1
            } else {
                const long double pn = (N % 2) ? -1.0L : 1.0L;       // (-1)^N, and w^N = 1
                const long double nr = 1.0L - pn, dr = 1.0L + wr, di = wi;
                const long double den = dr * dr + di * di;
                ar = g[0] * (nr * dr) / den;
                ai = g[0] * (-nr * di) / den;
            }
        } else {
            for (int t = 0; t <= k; ++t) {           // any other table: the sum itself
                long double xr, xi;
                wneg((int64_t)m * t, xr, xi);
                ar += g[t] * xr;
                ai += g[t] * xi;
            }
        }
        re[m] = (double)(ar / N);
        im[m] = (double)(ai / N);
    }
}

void bucket_shape(int k, int &J, int &S)
{
    if (k <= kShortMax) { J = 1; S = k; return; }
    // Cheapest (J, S) with J*S >= k by a simple instruction model: per lane and root,
    // about 9 VALU instructions per literal slot plus the butterfly's log2(J) levels
    // and a fixed part; per useful literal that is J * (9 S + 13 log2 J + 16) / k.
    double best = 1e30;
    J = 64; S = 16;
    for (int j = 2; j <= 64; j *= 2) {
        int lg = 0;
        while ((1 << lg) < j) ++lg;
        const double lanes = 13.0 * lg + 16.0 + (j > 16 ? 20.0 : 0.0);
        for (int s = 8; s <= kMaxSeg; s += 2) {
            if (j * s < k) continue;
            const double cost = j * (9.0 * s + lanes) / k;
            if (cost < best - 1e-9) { best = cost; J = j; S = s; }
        }
    }
}

// Rows m = 1..floor(k/2) of a coefficient table.
// With alpha_m = (1 + omega^m)/2 = c e^{i h} (h = pi m / N, c = cos h) every factor is
// a = alpha_m (1 + i z), z = -tan(h) y.  Kernels multiply the unit-real-part
// factors (1 + i z) and keep the magnitudes in range with real scale factors;
// the phases e^{i n h} of the alpha powers are constants folded into the rows.
//   Short kernel (k <= 16, one lane per restart, no scaling): the FE uses
//     2 d alpha^k, and the adjoint constant is Kc = 2 d beta alpha^(k-1),
//     beta = (1 - omega^m)/2.
//   Segment kernel (J lanes of S literals): a lane multiplies its running prefix
//     and suffix products by c^RP at the positions RP, 2 RP, ... < S (RP = 16
//     when every length in its bucket is <= 256, else 8) and its segment product
//     by c^F, F = S - RP floor((S-1)/RP); each lane product then carries c^S and
//     no phase.  So the FE uses 2 d' with d' = d e^{i J S h}, and the adjoint
//     constant, which restores what prefix * suffix * (other lanes) lacks, is
//     Kc = 2 d beta c^(F-1) e^{i (J S - 1) h}.
// Rows per root:
//   short:   {Re(2 d alpha^k), Im(2 d alpha^k), Re Kc, Im Kc}, {0, 0, -tan h, 0}
//   segment: {Re 2d', Im 2d', Re Kc, Im Kc}, {-tan h, c^RP, c^F, 0}
// (The magnitudes stay in FP32 range: |1 + i z| <= 1/c <= 1/sin(pi/(2N)), so 16
// unscaled factors stay below 2^128 up to k = 256 and 8 up to k = 1024, and c^RP
// stays above the smallest normal, 2^-126, at those lengths.)
int rescale_period(int J, int S) { return J * S <= 256 ? 16 : 8; }


// The per-root factors of the rows that do not depend on the coefficients: the
// same for every table of one length and kernel shape, so computed once per
// (k, J, S) and kept (the trigonometry in long double is most of a table's cost).
struct RootConsts {
    long double br, bi;      // beta = (1 - omega^m)/2
    long double er, ei;      // FE phase
    long double ck;          // FE magnitude: c^k (short kernel) or 1
    long double fr, fi;      // adjoint phase
    long double kmag;        // adjoint magnitude
    float mt, crp, cf;       // -tan h, c^RP, c^F
};

static const std::vector<RootConsts> &root_consts(int k, int J, int S)
{
    static std::mutex mu;
    static std::map<std::tuple<int, int, int>, std::vector<RootConsts>> memo;
    const bool shrt = k <= kShortMax;
    const auto key = shrt ? std::make_tuple(k, 1, k) : std::make_tuple(k, J, S);
    std::lock_guard<std::mutex> lock(mu);
    auto it = memo.find(key);
    if (it != memo.end()) return it->second;
    const int N = k + 1;
    const int M = k / 2;
    const long double pi = 3.141592653589793238462643383279502884L;
    // e^{i n h} with the angle n*h = pi (m n mod 2N) / N reduced exactly
    auto phase = [&](int m, int64_t n, long double &pr, long double &pim) {
        const long double ang = pi * (long double)(((int64_t)m * n) % (2 * N)) / (long double)N;
        pr = cosl(ang);
        pim = sinl(ang);
    };
    std::vector<RootConsts> v(M + 1);
    for (int m = 1; m <= M; ++m) {
        RootConsts &r = v[m];
        const long double h = pi * (long double)m / (long double)N;
        const long double sh = sinl(h), ch = cosl(h);
        // beta = (1 - omega)/2 = -i sin(h) e^{i h} = (sin^2 h, -sin h cos h)
        r.br = sh * sh;
        r.bi = -sh * ch;
        r.mt = (float)(-sh / ch);
        if (shrt) {
            phase(m, k, r.er, r.ei);                      // alpha^k = c^k e^{i k h}
            r.ck = powl(ch, (long double)k);
            phase(m, k - 1, r.fr, r.fi);                  // alpha^(k-1)
            r.kmag = powl(ch, (long double)(k - 1));
            r.crp = r.cf = 0.0f;
        } else {
            const int RP = rescale_period(J, S);
            const int F = S - RP * ((S - 1) / RP);
            phase(m, (int64_t)J * S, r.er, r.ei);         // d' = d e^{i J S h}
            r.ck = 1.0L;
            phase(m, (int64_t)J * S - 1, r.fr, r.fi);     // Kc = 2 d beta c^(F-1) e^{i (J S - 1) h}
            r.kmag = powl(ch, (long double)(F - 1));
            r.crp = (float)powl(ch, (long double)RP);
            r.cf = (float)powl(ch, (long double)F);
        }
    }
    return memo.emplace(key, std::move(v)).first->second;
}

void append_root_rows(int k, int J, int S, const double *re, const double *im, std::vector<TabRow> &tab)
{
    const int M = k / 2;
    const bool shrt = k <= kShortMax;
    const std::vector<RootConsts> &rc = root_consts(k, J, S);
    for (int m = 1; m <= M; ++m) {
        const RootConsts &r = rc[m];
        const long double dr = re[m], di = im[m];
        const long double tr = 2.0L * (dr * r.br - di * r.bi), ti = 2.0L * (dr * r.bi + di * r.br);   // 2 d beta
        const long double kr = r.kmag * (tr * r.fr - ti * r.fi), ki = r.kmag * (tr * r.fi + ti * r.fr);
        // short: 2 d alpha^k; segment: 2 d' = 2 d e^{i J S h}
        const long double fer = 2.0L * r.ck * (dr * r.er - di * r.ei), fei = 2.0L * r.ck * (dr * r.ei + di * r.er);
        tab.push_back({(float)fer, (float)fei, (float)kr, (float)ki});
        if (shrt)
            tab.push_back({0.0f, 0.0f, r.mt, 0.0f});
        else
            tab.push_back({r.mt, r.crp, r.cf, 0.0f});
    }
}

void bucket_shape(int k, const PackOptions &o, int &J, int &S)
{
    if (k > kShortMax) {
        for (size_t e = 0; e < o.k_hi.size(); ++e)
            if (k <= o.k_hi[e]) { J = o.lanes[e]; S = o.seg[e]; return; }
    }
    bucket_shape(k, J, S);
}

std::string check_options(const PackOptions &o)
{
    if (o.k_hi.size() != o.lanes.size() || o.k_hi.size() != o.seg.size()) return "shape arrays differ in length";
    int prev = kShortMax;
    for (size_t e = 0; e < o.k_hi.size(); ++e) {
        const int J = o.lanes[e], S = o.seg[e], kh = o.k_hi[e];
        if (kh <= prev) return "shape_k_hi must be ascending and > 16";
        if (kh > kMaxLen) return "shape_k_hi exceeds the maximum length";
        if (J < 2 || J > 64 || (J & (J - 1))) return "shape_lanes must be 2, 4, 8, 16, 32 or 64";
        if (S < kMinSeg || S > kMaxSeg || S % 2) return "shape_seg must be even, 4 to 32";
        if (J * S < kh) return "shape_lanes * shape_seg is smaller than shape_k_hi";
        prev = kh;
    }
    if (!o.tile.empty() && o.tile.size() != o.k_hi.size()) return "shape_tile differs in length from the shapes";
    for (int t : o.tile)
        if (t < 0 || t > kMaxTile) return "shape_tile out of range";
    if (o.tile_short < 0 || o.tile_long < 0 || o.tile_short > kMaxTile || o.tile_long > kMaxTile)
        return "tile out of range";
    for (int k = 1; k <= kShortMax; ++k) {
        if (o.short_tile[k] < 0 || o.short_tile[k] > kMaxTile) return "short_tile out of range";
        const int r = o.short_rpl[k];
        if (r != 0 && r != 1 && r != 2 && r != 4) return "short_rpl must be 0, 1, 2 or 4";
        if (r == 4 && k > 8) return "short_rpl 4 needs k <= 8";
    }
    return std::string();
}

void bucket_tiling(int k, const PackOptions &o, int &tile, int &rpl)
{
    rpl = 0;
    if (k <= kShortMax) {
        tile = o.short_tile[k] > 0 ? o.short_tile[k] : (o.tile_short > 0 ? o.tile_short : 4);
        rpl = o.short_rpl[k];
        return;
    }
    int J, S;
    bucket_shape(k, o, J, S);
    for (size_t e = 0; e < o.k_hi.size(); ++e)
        if (k <= o.k_hi[e]) {
            if (!o.tile.empty() && o.tile[e] > 0) { tile = o.tile[e]; return; }
            break;
        }
    tile = o.tile_long > 0 ? o.tile_long : (J >= 8 ? 1 : 8 / J);
}

std::string build_instance(int32_t n, int32_t C, const int64_t *con_off, const int32_t *lits,
                           const int32_t *types, const int32_t *params, const float *weights,
                           const PackOptions &opts, HostInstance &H)
{
    {
        const std::string e = check_options(opts);
        if (!e.empty()) return e;
    }
    if (n < 1) return "n_vars must be >= 1";
    if (C < 0) return "n_cons must be >= 0";
    if (!con_off) return "con_off is NULL";
    if (con_off[0] != 0) return "con_off[0] must be 0";
    if (C > 0 && !types) return "types is NULL";
    int max_k = 0;
    for (int32_t c = 0; c < C; ++c) {
        const int64_t k = con_off[c + 1] - con_off[c];
        if (k < 1) return "constraint " + std::to_string(c) + " has length < 1";
        if (k > kMaxLen)
            return "constraint " + std::to_string(c) + " is longer than " + std::to_string(kMaxLen);
        max_k = std::max(max_k, (int)k);
        if (types[c] < 0 || types[c] > 7) return "constraint " + std::to_string(c) + " has an unknown type";
        if (uses_param(types[c]) && !params) return "params is NULL but a constraint needs a parameter";
        if (weights && !std::isfinite(weights[c])) return "weight of constraint " + std::to_string(c) + " is not finite";
    }
    const int64_t L = C > 0 ? con_off[C] : 0;
    if (L >= ((int64_t)1 << 31)) return "more than 2^31-1 literals";
    if (L > 0 && !lits) return "lits is NULL";
    for (int64_t i = 0; i < L; ++i) {
        const int32_t l = lits[i];
        if (l == 0 || l > n || l < -n) return "literal " + std::to_string(i) + " is out of range";
    }

    H = HostInstance();
    H.n = n; H.C = C; H.L = L; H.max_k = max_k;
    H.con_off.assign(con_off, con_off + C + 1);
    H.lits.assign(lits, lits + L);
    H.types.assign(types, types + C);
    H.params.assign(C, 0);
    H.weights.assign(C, 1.0f);
    for (int32_t c = 0; c < C; ++c) {
        if (params) H.params[c] = params[c];
        if (weights) H.weights[c] = weights[c];
    }

    // ---- coefficient tables, one per distinct (type, k, canonical param) ----
    std::map<std::tuple<int, int, int>, std::pair<int32_t, int32_t>> table_of;   // -> (row, index)
    std::vector<int32_t> con_tab(C), con_tidx(C);
    std::vector<double> re, im;
    for (int32_t c = 0; c < C; ++c) {
        const int k = (int)(con_off[c + 1] - con_off[c]);
        const int p = canonical_param(types[c], k, H.params[c]);
        auto key = std::make_tuple(types[c], k, p);
        auto it = table_of.find(key);
        if (it != table_of.end()) {
            con_tab[c] = it->second.first;
            con_tidx[c] = it->second.second;
            continue;
        }
        const int32_t off = (int32_t)H.tab.size();
        table_of.emplace(key, std::make_pair(off, H.n_tables));
        con_tab[c] = off;
        con_tidx[c] = H.n_tables;
        re.assign(k + 1, 0.0);
        im.assign(k + 1, 0.0);
        coefficients(types[c], k, p, re.data(), im.data());
        const int N = k + 1;
        const double dhalf = (N % 2 == 0) ? re[N / 2] : 0.0;
        int J, S;
        bucket_shape(k, opts, J, S);
        H.tab.push_back({(float)re[0], (float)dhalf, 0.0f, 0.0f});
        append_root_rows(k, J, S, re.data(), im.data(), H.tab);
        ++H.n_tables;
    }
    // the kernels address table rows with 32-bit byte offsets
    if (H.tab.size() >= ((size_t)1 << 27)) return "coefficient tables exceed 2 GiB (too many distinct constraints)";

    // ---- buckets ----
    // Order: short buckets by length, then long ones by capacity J*S (then J),
    // within a bucket by length and table.  The kernel shape of each length is
    // worked out once, and each constraint gets one integer sort key.
    // Lengths of one class with different tilings stay apart: the sort below keeps
    // a class ordered by length, so each tiling's lengths are contiguous in it.
    auto klen = [&](int32_t c) { return (int)(con_off[c + 1] - con_off[c]); };
    std::vector<std::tuple<int, int, int, int>> shape_of_len(max_k + 1);   // (J, S, tile, rpl)
    for (int k = 1; k <= max_k; ++k) {
        int J, S, tile, rpl;
        bucket_shape(k, opts, J, S);
        bucket_tiling(k, opts, tile, rpl);
        shape_of_len[k] = std::make_tuple(J, J == 1 ? k : S, tile, rpl);
    }
    auto shape_key = [&](int32_t c) { return shape_of_len[klen(c)]; };
    std::vector<std::pair<uint64_t, int32_t>> keyed(C);
    for (int32_t c = 0; c < C; ++c) {
        const int J = std::get<0>(shape_key(c)), S = std::get<1>(shape_key(c));
        const uint64_t cls = J == 1 ? (uint64_t)S : (uint64_t)(J * S + 1000);
        // class (< 2^17) | J (< 2^7) | length (< 2^11) | table index (< 2^29: there are
        // at most 8 types x 1024 lengths x 1026 thresholds)
        const uint64_t key = (cls << 47) | ((uint64_t)J << 40) | ((uint64_t)klen(c) << 29) |
                             (uint64_t)con_tidx[c];
        keyed[c] = std::make_pair(key, c);
    }
    std::sort(keyed.begin(), keyed.end());             // ties broken by constraint index: stable
    std::vector<int32_t> order(C);
    for (int32_t i = 0; i < C; ++i) order[i] = keyed[i].second;

    H.bc_slot0.resize(C); H.bc_k.resize(C); H.bc_tab.resize(C); H.bc_orig.resize(C); H.bc_w.resize(C);
    H.slot_lit.resize(L); H.slot_to_lit.resize(L);
    int64_t slot = 0;
    int32_t tiles = 0;
    for (int32_t i = 0; i < C;) {
        const auto key = shape_key(order[i]);
        Bucket bk;
        bucket_shape(klen(order[i]), opts, bk.J, bk.S);
        bk.c0 = i;
        bk.slot0 = slot;
        bk.k_lo = klen(order[i]);
        int32_t j = i;
        while (j < C && shape_key(order[j]) == key) {
            const int32_t c = order[j];
            const int k = klen(c);
            H.bc_slot0[j] = (int32_t)slot;
            H.bc_k[j] = k;
            H.bc_tab[j] = con_tab[c];
            H.bc_orig[j] = c;
            H.bc_w[j] = H.weights[c];
            for (int q = 0; q < k; ++q) {
                H.slot_lit[slot + q] = lits[con_off[c] + q];
                H.slot_to_lit[slot + q] = (int32_t)(con_off[c] + q);
            }
            slot += k;
            bk.k_hi = k;
            ++j;
        }
        bk.nc = j - i;
        bk.nslots = slot - bk.slot0;
        bk.tile = std::get<2>(key);
        bk.rpl = std::get<3>(key);
        bk.ntiles = (bk.nc + bk.tile - 1) / bk.tile;
        bk.tile0 = tiles;
        tiles += bk.ntiles;
        H.buckets.push_back(bk);
        i = j;
    }
    H.total_tiles = tiles;

    // ---- variable -> slot transpose, ascending slots ----
    H.voff.assign(n + 1, 0);
    for (int64_t s = 0; s < L; ++s) H.voff[std::abs(H.slot_lit[s])]++;   // count into v+1
    for (int32_t v = 0; v < n; ++v) H.voff[v + 1] += H.voff[v];
    H.vslot.assign(L, 0);
    std::vector<int32_t> fill(H.voff.begin(), H.voff.end() - 1);
    for (int64_t s = 0; s < L; ++s) {
        const int v = std::abs(H.slot_lit[s]) - 1;
        H.vslot[fill[v]++] = (int32_t)s;
    }
    H.n_inst = 1;
    H.inst_var0 = {0, n};
    H.con_inst.assign(C, 0);
    H.var_inst.assign(n, 0);
    return std::string();
}

std::string build_batch(const std::vector<PartRef> &parts, const PackOptions &opts, HostInstance &H)
{
    if (parts.empty()) return "a batch needs at least one instance";
    int64_t n = 0, C = 0, L = 0;
    for (const PartRef &p : parts) {
        if (p.n < 1 || p.C < 0 || !p.con_off) return "invalid part";
        n += p.n;
        C += p.C;
        L += p.C > 0 ? p.con_off[p.C] : 0;
    }
    if (n >= ((int64_t)1 << 31) || C >= ((int64_t)1 << 31) || L >= ((int64_t)1 << 31))
        return "batch too large";
    std::vector<int64_t> con_off(C + 1, 0);
    std::vector<int32_t> lits(L), types(C), params(C);
    std::vector<float> weights(C);
    std::vector<int32_t> inst_var0(parts.size() + 1, 0), con_inst(C), var_inst(n);
    int64_t c0 = 0, l0 = 0;
    int32_t v0 = 0;
    for (size_t pi = 0; pi < parts.size(); ++pi) {
        const PartRef &p = parts[pi];
        const int64_t pl = p.C > 0 ? p.con_off[p.C] : 0;
        if (p.C > 0 && (!p.types || (pl > 0 && !p.lits))) return "invalid part arrays";
        for (int32_t c = 0; c < p.C; ++c) {
            con_off[c0 + c + 1] = l0 + p.con_off[c + 1];
            types[c0 + c] = p.types[c];
            params[c0 + c] = p.params ? p.params[c] : 0;
            weights[c0 + c] = p.weights ? p.weights[c] : 1.0f;
            con_inst[c0 + c] = (int32_t)pi;
        }
        for (int64_t i = 0; i < pl; ++i) {
            const int32_t l = p.lits[i];
            if (l == 0 || l > p.n || l < -p.n) return "literal out of range in part " + std::to_string(pi);
            lits[l0 + i] = l > 0 ? l + v0 : l - v0;
        }
        for (int32_t v = 0; v < p.n; ++v) var_inst[v0 + v] = (int32_t)pi;
        c0 += p.C;
        l0 += pl;
        v0 += p.n;
        inst_var0[pi + 1] = v0;
    }
    std::string e = build_instance((int32_t)n, (int32_t)C, con_off.data(), lits.data(), types.data(),
                                   params.data(), weights.data(), opts, H);
    if (!e.empty()) return e;
    H.n_inst = (int32_t)parts.size();
    H.inst_var0 = std::move(inst_var0);
    H.con_inst = std::move(con_inst);
    H.var_inst = std::move(var_inst);
    return std::string();
}

}  // namespace afs
