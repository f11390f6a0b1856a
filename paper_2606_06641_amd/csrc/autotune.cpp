// autotune.cpp -- on-device choice of the FE kernel configuration for each
// length range of an instance: the segment-kernel shape (J lanes per restart x S
// literals per lane) for lengths above 16 and, on request, the work-tile size of
// every range and the restarts per lane of the one-lane kernel for each length
// up to 16.
//
// For each range (every length <= 16 alone; above, the ranges between
// consecutive candidate capacities J*S) the constraints of the instance in that
// range (an evenly spaced sample of at most max_cons) are packed alone once per
// candidate, and the FE+gradient pass of that bucket is timed on the device
// (median of `reps` launches, HIP events on a private stream).  The shape stage
// takes the fastest shape at the default tile.  The optional second stage times
// the one-lane kernel's restarts per lane and then the tile sizes of the chosen
// configuration; a tile other than the default must win by 2% (the medians of
// neighbouring tiles are often within noise).  That stage is off by default:
// it ranks configurations by their time alone, and in an iteration the one-lane
// and the short segment buckets run beside the long ones, where its choices
// (more waves for the same work) made whole iterations slower.  Results are
// cached in a text file keyed by (GPU architecture, FE kernel source revision,
// restarts, range, size class of the range's constraint count), one line per
// entry:
//     <arch> <revision> <B> <k_lo> <k_hi> <class> <J> <S> <tile> <rpl> <median ms> <constraints timed>
// (tile and rpl 0: the defaults, from a shape-only tuning), so that other
// instances with about as many constraints in the same ranges reuse them and a
// change to the kernels invalidates them.

#include "afsat.h"

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <random>
#include <set>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "host.hpp"
#include "instance.hpp"

#ifndef AFS_FE_REV
#define AFS_FE_REV "unknown"
#endif

namespace {

constexpr int kLanes[] = {2, 4, 8, 16, 32, 64};

std::vector<int> capacities()
{
    std::set<int> caps;
    for (int J : kLanes)
        for (int S = afs::kMinSeg; S <= afs::kMaxSeg; S += 2)
            if (J * S > afs::kShortMax && J * S <= afs::kMaxLen) caps.insert(J * S);
    return std::vector<int>(caps.begin(), caps.end());
}

// [(k_lo, k_hi)]: 1..16 one length each, then 17..1024 split at every candidate
// capacity
std::vector<std::pair<int, int>> length_ranges()
{
    std::vector<std::pair<int, int>> out;
    for (int k = 1; k <= afs::kShortMax; ++k) out.emplace_back(k, k);
    int lo = afs::kShortMax + 1;
    for (int cap : capacities()) {
        if (cap >= lo) {
            out.emplace_back(lo, cap);
            lo = cap + 1;
        }
    }
    return out;
}

// The size class of a range: floor(log2(constraints of the instance in it)).  The
// best configuration depends on how many waves a launch has (a range of a few
// constraints runs in the latency regime, one of thousands fills the device), so
// instances whose ranges differ in size class are tuned apart.
int size_class(size_t count)
{
    int c = 0;
    while (count >= 2) {
        count >>= 1;
        ++c;
    }
    return c;
}

struct Key {
    std::string arch, rev;
    int B, lo, hi, cls;
    bool operator<(const Key &o) const
    {
        return std::tie(arch, rev, B, lo, hi, cls) < std::tie(o.arch, o.rev, o.B, o.lo, o.hi, o.cls);
    }
};

struct Choice {
    int J = 0, S = 0, tile = 0, rpl = 0;
    double ms = 0.0;
    int timed = 0;
};

void read_cache(const char *path, std::map<Key, Choice> &cache)
{
    if (!path) return;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        if (line.empty() || line[0] == '#') continue;
        std::istringstream in(line);
        Key k;
        Choice c;
        if (in >> k.arch >> k.rev >> k.B >> k.lo >> k.hi >> k.cls >> c.J >> c.S >> c.tile >> c.rpl >> c.ms >> c.timed)
            cache[k] = c;
    }
}

// Default work tile of a shape (as the packing chooses it when none is given).
int default_tile(int J) { return J == 1 ? 4 : (J >= 8 ? 1 : 8 / J); }

bool write_cache(const char *path, const std::map<Key, Choice> &cache, const std::string &rev)
{
    if (!path) return true;
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) return false;
        f << "# arch revision B k_lo k_hi size_class lanes seg tile rpl median_ms constraints_timed\n";
        for (const auto &kv : cache) {
            if (kv.first.rev != rev) continue;                  // stale kernel revisions are dropped
            char buf[256];
            std::snprintf(buf, sizeof buf, "%s %s %d %d %d %d %d %d %d %d %.6f %d\n", kv.first.arch.c_str(),
                          kv.first.rev.c_str(), kv.first.B, kv.first.lo, kv.first.hi, kv.first.cls, kv.second.J,
                          kv.second.S, kv.second.tile, kv.second.rpl, kv.second.ms, kv.second.timed);
            f << buf;
        }
        if (!f) return false;
    }
    return std::rename(tmp.c_str(), path) == 0;
}

// Time the FE+gradient pass of `cons` packed alone with the configuration c for
// the range ending at hi (J == 1: a one-lane length, S == hi).
afs_status time_shape(const afs::HostInstance &H, const std::vector<int32_t> &cons, int hi, const Choice &c,
                      int device, int B, const float *x, int reps, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                      double &ms)
{
    const int J = c.J, S = c.S;
    std::vector<int64_t> off(1, 0);
    std::vector<int32_t> lits, types, params;
    std::vector<float> w;
    for (int32_t c : cons) {
        for (int64_t o = H.con_off[c]; o < H.con_off[c + 1]; ++o) lits.push_back(H.lits[o]);
        off.push_back((int64_t)lits.size());
        types.push_back(H.types[c]);
        params.push_back(H.params[c]);
        w.push_back(H.weights.empty() ? 1.0f : H.weights[c]);
    }
    int32_t kh = hi, lanes = J, seg = S, tile = c.tile;
    int32_t short_tile[afs::kShortMax] = {}, short_rpl[afs::kShortMax] = {};
    afs_options o{};
    if (J > 1) {
        o.n_shapes = 1;
        o.shape_k_hi = &kh;
        o.shape_lanes = &lanes;
        o.shape_seg = &seg;
        o.shape_tile = &tile;
    } else {
        short_tile[hi - 1] = c.tile;
        short_rpl[hi - 1] = c.rpl;
        o.short_tile = short_tile;
        o.short_rpl = short_rpl;
    }
    afs_instance *sub = nullptr;
    afs_status st = afs_instance_create_ex(H.n, (int32_t)cons.size(), off.data(), lits.data(), types.data(),
                                           params.data(), w.data(), &o, device, &sub);
    if (st != AFS_OK) return st;
    size_t bytes = 0;
    void *ws = nullptr;
    afs_info info{};
    st = afs_workspace_bytes(sub, B, &bytes);
    if (st == AFS_OK) st = afs_instance_info(sub, &info);
    if (st == AFS_OK && hipMalloc(&ws, bytes) != hipSuccess) st = afs::set_last_error(AFS_ENOMEM, "hipMalloc");
    std::vector<float> t;
    for (int r = 0; st == AFS_OK && r <= reps; ++r) {
        if (hipEventRecord(e0, s) != hipSuccess) st = afs::set_last_error(AFS_EDEVICE, "hipEventRecord");
        if (st == AFS_OK) st = afs_fe_grad(sub, B, x, ws, bytes, 0, info.n_buckets, 0, nullptr, s);
        if (st == AFS_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
            st = afs::set_last_error(AFS_EDEVICE, "timing events");
        float e = 0.f;
        if (st == AFS_OK && hipEventElapsedTime(&e, e0, e1) != hipSuccess)
            st = afs::set_last_error(AFS_EDEVICE, "hipEventElapsedTime");
        if (st == AFS_OK && r > 0) t.push_back(e);              // launch 0 warms up
    }
    if (ws) (void)hipFree(ws);
    afs_instance_destroy(sub);
    if (st != AFS_OK) return st;
    std::sort(t.begin(), t.end());
    ms = t[t.size() / 2];
    return AFS_OK;
}

}  // namespace

extern "C" {

afs_status afs_autotune(const afs_instance *inst, int32_t device, int32_t B, int32_t reps, int32_t max_cons,
                        int32_t tiles, const char *cache_in, const char *cache_out, int32_t max_ranges, int32_t *k_lo,
                        int32_t *k_hi, int32_t *lanes, int32_t *seg, int32_t *tile, int32_t *rpl, float *ms,
                        int32_t *n_ranges)
{
    using afs::set_last_error;
    if (!inst || !n_ranges) return set_last_error(AFS_EINVAL, "inst or n_ranges is NULL");
    if (B <= 0 || reps < 1 || max_ranges < 0) return set_last_error(AFS_EINVAL, "need B >= 1, reps >= 1, max_ranges >= 0");
    if (max_ranges > 0 && (!k_lo || !k_hi || !lanes || !seg)) return set_last_error(AFS_EINVAL, "output arrays are NULL");
    *n_ranges = 0;
    const afs::HostInstance &H = inst->H;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return set_last_error(AFS_EINVAL, "no HIP device " + std::to_string(device));
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess)
        return set_last_error(AFS_EDEVICE, "hipSetDevice");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return set_last_error(AFS_EDEVICE, "hipGetDeviceProperties");
    std::string arch(prop.gcnArchName);
    arch = arch.substr(0, arch.find(':'));
    const std::string rev = AFS_FE_REV;

    // cache_out first: where both files hold a result for one key, cache_in's,
    // the one the caller names for reading, is the one used
    std::map<Key, Choice> cache;
    read_cache(cache_out, cache);
    read_cache(cache_in, cache);

    // constraints per range
    std::vector<std::pair<int, int>> ranges = length_ranges();
    std::vector<std::vector<int32_t>> members(ranges.size());
    for (int32_t c = 0; c < H.C; ++c) {
        const int k = (int)(H.con_off[c + 1] - H.con_off[c]);
        for (size_t r = 0; r < ranges.size(); ++r)
            if (k >= ranges[r].first && k <= ranges[r].second) {
                members[r].push_back(c);
                break;
            }
    }

    afs_status st = AFS_OK;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float *x = nullptr;
    bool device_ready = false;
    auto prepare = [&]() -> afs_status {
        if (device_ready) return AFS_OK;
        device_ready = true;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
            return set_last_error(AFS_EDEVICE, "hipStreamCreate");
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
            return set_last_error(AFS_EDEVICE, "hipEventCreate");
        // uniform points in [-1, 1], one column per restart
        std::vector<float> hx((size_t)std::max(H.n, 1) * B);
        std::mt19937 rng(12345u);
        std::uniform_real_distribution<float> u(-1.0f, 1.0f);
        for (float &v : hx) v = u(rng);
        if (hipMalloc(&x, hx.size() * sizeof(float)) != hipSuccess) return set_last_error(AFS_ENOMEM, "hipMalloc");
        if (hipMemcpy(x, hx.data(), hx.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
            return set_last_error(AFS_EDEVICE, "hipMemcpy");
        return AFS_OK;
    };

    int32_t out = 0;
    for (size_t r = 0; r < ranges.size() && st == AFS_OK; ++r) {
        if (members[r].empty()) continue;
        const int lo = ranges[r].first, hi = ranges[r].second;
        const Key key{arch, rev, B, lo, hi, size_class(members[r].size())};
        Choice best;
        float reported = -1.0f;                                 // cached: not timed now
        auto it = cache.find(key);
        // a shape-only entry (tile 0) does not answer a request for tiles
        const bool hit = it != cache.end() && (!tiles || it->second.tile > 0);
        if (!tiles && hi <= afs::kShortMax) {                   // one lane, defaults: nothing to time
            best.J = 1;
            best.S = hi;
            reported = 0.0f;
        } else if (hit) {
            best = it->second;
            if (!tiles) best.tile = best.rpl = 0;
        } else {
            if ((st = prepare()) != AFS_OK) break;
            std::vector<int32_t> cons = members[r];
            // one-lane lengths: a sample of at least 65,536 (a few hundred waves would
            // time launch latency, not the kernel)
            const int cap = (max_cons > 0 && hi <= afs::kShortMax) ? std::max(max_cons, 1 << 16) : max_cons;
            if (cap > 0 && (int)cons.size() > cap) {            // evenly spaced sample
                std::vector<int32_t> sample;
                for (int i = 0; i < cap; ++i) sample.push_back(cons[(size_t)i * cons.size() / cap]);
                cons.swap(sample);
            }
            auto timed = [&](Choice c, double &t) {
                return time_shape(H, cons, hi, c, device, B, x, reps, s, e0, e1, t);
            };
            best.ms = 1e30;
            if (hi <= afs::kShortMax) {                         // one lane: restarts per lane
                for (int rpl : {4, 2, 1}) {
                    if (rpl == 4 && hi > 8) continue;
                    if (st != AFS_OK || B % rpl) continue;
                    Choice c;
                    c.J = 1; c.S = hi; c.tile = default_tile(1); c.rpl = rpl;
                    double t = 0.0;
                    st = timed(c, t);
                    if (st == AFS_OK && t < best.ms) { best = c; best.ms = t; }
                }
            } else {                                            // segments: lanes x literals
                for (int J : kLanes) {
                    for (int S = afs::kMinSeg; S <= afs::kMaxSeg && st == AFS_OK; S += 2) {
                        if (J * S < hi || J * S >= 2 * hi + 64) continue;   // too small, or mostly padding
                        Choice c;
                        c.J = J; c.S = S; c.tile = default_tile(J);
                        double t = 0.0;
                        st = timed(c, t);
                        if (st == AFS_OK && t < best.ms) { best = c; best.ms = t; }
                    }
                }
            }
            // then the tile for that configuration
            const Choice base = best;
            for (int tile : {1, 2, 4, 8, 16}) {
                if (!tiles || st != AFS_OK || tile == base.tile) continue;
                Choice c = base;
                c.tile = tile;
                double t = 0.0;
                st = timed(c, t);
                if (st == AFS_OK && t < 0.98 * best.ms) { best = c; best.ms = t; }
            }
            if (st != AFS_OK) break;
            if (!tiles) best.tile = 0;                          // the default, whatever it is
            best.timed = (int)cons.size();
            cache[key] = best;
            reported = (float)best.ms;
        }
        if (out < max_ranges) {
            k_lo[out] = lo;
            k_hi[out] = hi;
            lanes[out] = best.J;
            seg[out] = best.S;
            if (tile) tile[out] = best.tile;
            if (rpl) rpl[out] = best.rpl;
            if (ms) ms[out] = reported;
        }
        ++out;
    }
    if (x) (void)hipFree(x);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    (void)hipSetDevice(prev);
    if (st != AFS_OK) return st;
    if (!write_cache(cache_out, cache, rev))
        return set_last_error(AFS_EINVAL, std::string("cannot write ") + cache_out);
    *n_ranges = out;
    return AFS_OK;
}

}  // extern "C"
