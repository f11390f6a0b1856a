// api.cpp -- the C ABI declared in include/afsat.h.
#include "afsat.h"

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "host.hpp"
#include "instance.hpp"
#include "kernels.hpp"


namespace {

thread_local std::string g_err;

afs_status fail(afs_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

afs_status dev_fail(hipError_t e, const char *what)
{
    return fail(AFS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

class DeviceGuard {
public:
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev_) != hipSuccess) { err_ = hipErrorNoDevice; return; }
        if (prev_ != dev) err_ = hipSetDevice(dev);
        dev_ = dev;
    }
    ~DeviceGuard()
    {
        if (err_ == hipSuccess && prev_ >= 0 && prev_ != dev_) (void)hipSetDevice(prev_);
    }
    hipError_t error() const { return err_; }

private:
    int prev_ = -1, dev_ = -1;
    hipError_t err_ = hipSuccess;
};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct WsLayout {
    int Bp = 0, W = 0;
    size_t adj = 0, part = 0, part2 = 0, bits = 0, viol = 0, moved = 0, total = 0;
};

WsLayout ws_layout(const afs::HostInstance &H, int B)
{
    WsLayout l;
    l.Bp = (B + 63) / 64 * 64;
    l.W = (B + 31) / 32;
    size_t off = 0;
    l.adj = off;
    off = align256(off + (size_t)H.L * l.Bp * sizeof(float));
    l.part = off;
    off = align256(off + (size_t)H.total_tiles * l.Bp * sizeof(float));
    l.part2 = off;
    off = align256(off + (size_t)((H.total_tiles + 31) / 32) * l.Bp * sizeof(float));
    l.bits = off;
    off = align256(off + (size_t)H.n * l.W * sizeof(uint32_t));
    l.viol = off;
    off = align256(off + (size_t)(H.C + 3) / 4 * 4 * l.W * sizeof(uint32_t));
    l.moved = off;                      // u8 [n_inst][B]: the epsilon test's "moved" flags
    off = align256(off + (size_t)H.n_inst * B);
    l.total = off;
    return l;
}

// Line-search workspace: gradient and trial point [n][B], per-tile partial sums
// of <g, xt - x> [vtiles][Bp] and their second-pass partials, per-restart f0,
// F(xt), <g, xt - x>, step length and decision flags.
struct SearchLayout {
    int vtiles = 0;
    size_t g = 0, xt = 0, dpart = 0, dpart2 = 0, f0 = 0, ft = 0, dot = 0, eta = 0, acc = 0, total = 0;
};

SearchLayout search_layout(const afs::HostInstance &H, int B)
{
    SearchLayout q;
    const size_t Bp = (size_t)(B + 63) / 64 * 64;
    q.vtiles = (H.n + afs::kTrialVars - 1) / afs::kTrialVars;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    q.g = take((size_t)H.n * B * sizeof(float));
    q.xt = take((size_t)H.n * B * sizeof(float));
    q.dpart = take((size_t)q.vtiles * Bp * sizeof(float));
    q.dpart2 = take((size_t)((q.vtiles + 31) / 32) * Bp * sizeof(float));
    q.f0 = take(Bp * sizeof(float));
    q.ft = take(Bp * sizeof(float));
    q.dot = take(Bp * sizeof(float));
    q.eta = take(Bp * sizeof(float));
    q.acc = take(Bp);
    q.total = off;
    return q;
}

// fixed / values hold n_partial rows (0 reads as 1), at most one per restart
template <class T>
afs_status check_partial(int32_t B, const T *fixed, int32_t n_partial)
{
    if (n_partial < 0) return fail(AFS_EINVAL, "n_partial must be >= 0");
    if (fixed && B > 0 && n_partial > B) return fail(AFS_EINVAL, "more partial assignments than restarts");
    return AFS_OK;
}

int partial_rows(int32_t n_partial) { return n_partial > 1 ? n_partial : 1; }

template <class T>
afs_status upload(afs_instance *I, const std::vector<T> &v, const T **out)
{
    void *p = nullptr;
    const size_t bytes = std::max<size_t>(v.size() * sizeof(T), 16);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return fail(AFS_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    I->allocs.push_back(p);
    if (!v.empty()) {
        e = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess) return dev_fail(e, "hipMemcpy");
    }
    *out = static_cast<const T *>(p);
    return AFS_OK;
}

void release(afs_instance *I)
{
    if (!I) return;
    if (I->device >= 0) {
        DeviceGuard g(I->device);
        // work still queued on any stream may read the tables: let the device finish first
        (void)hipDeviceSynchronize();
        for (void *p : I->allocs) (void)hipFree(p);
        if (I->fork) (void)hipEventDestroy(I->fork);
        if (I->join) (void)hipEventDestroy(I->join);
        if (I->side) (void)hipStreamDestroy(I->side);
        for (int t = 0; t < afs_instance::kLongSides; ++t) {
            if (I->join_long[t]) (void)hipEventDestroy(I->join_long[t]);
            if (I->side_long[t]) (void)hipStreamDestroy(I->side_long[t]);
        }
        if (I->drive_in) (void)hipEventDestroy(I->drive_in);
        if (I->drive_out) (void)hipEventDestroy(I->drive_out);
        if (I->drive) (void)hipStreamDestroy(I->drive);
        if (I->stepped) (void)hipEventDestroy(I->stepped);
        if (I->verified) (void)hipEventDestroy(I->verified);
        if (I->verify) (void)hipStreamDestroy(I->verify);
        if (I->counter_host) (void)hipHostFree(I->counter_host);
    }
    delete I;
}

afs_status check_call(const afs_instance *I, int32_t B)
{
    if (!I) return fail(AFS_EINVAL, "instance is NULL");
    if (I->device < 0) return fail(AFS_ESTATE, "instance was created host-only (device -1)");
    if (B < 0) return fail(AFS_EINVAL, "B must be >= 0");
    if ((int64_t)B * I->H.n >= ((int64_t)1 << 40)) return fail(AFS_EINVAL, "n*B too large");
    return AFS_OK;
}

afs_status check_ws(const afs_instance *I, int32_t B, const void *ws, size_t ws_bytes, WsLayout &l)
{
    l = ws_layout(I->H, B);
    if (!ws) return fail(AFS_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(AFS_EINVAL, "workspace is not 256-byte aligned");
    if (ws_bytes < l.total)
        return fail(AFS_EINVAL, "workspace too small: need " + std::to_string(l.total) + " bytes");
    return AFS_OK;
}

template <class T>
T *at(void *ws, size_t off) { return reinterpret_cast<T *>(static_cast<char *>(ws) + off); }

afs_status fe_grad_set(afs_instance *I, int B, const float *x, void *ws, const WsLayout &l,
                       const std::vector<int> &set, bool want_part, float *fe, hipStream_t s,
                       const float *dobj = nullptr, bool grad = true, const uint8_t *skip = nullptr);

afs_status fe_grad_range(afs_instance *I, int B, const float *x, void *ws, const WsLayout &l,
                         int lo, int hi, bool want_part, float *fe, hipStream_t s,
                         const float *dobj = nullptr, bool grad = true, const uint8_t *skip = nullptr)
{
    std::vector<int> set;
    for (int bi = lo; bi < hi; ++bi) set.push_back(bi);
    return fe_grad_set(I, B, x, ws, l, set, want_part, fe, s, dobj, grad, skip);
}

afs_status fe_grad_set(afs_instance *I, int B, const float *x, void *ws, const WsLayout &l,
                       const std::vector<int> &set, bool want_part, float *fe, hipStream_t s,
                       const float *dobj, bool grad, const uint8_t *skip)
{
    // Short buckets (one lane per restart, bound by memory traffic) go to the side
    // stream when long buckets (bound by arithmetic) share the range, so the two
    // kinds overlap.  Long buckets hold few constraints each and rarely fill the
    // device alone, so they are dealt to up to 1 + kLongSides streams (the
    // caller's and side_long[]), largest first to whichever has the least
    // estimated work (flops ~ literals x length).  Every bucket writes its own
    // adjoint rows and objective tiles.
    constexpr int NS = 1 + afs_instance::kLongSides;
    std::vector<int> shorts, longs;
    for (int bi : set) (I->H.buckets[bi].J == 1 ? shorts : longs).push_back(bi);
    const bool split_short = !shorts.empty() && !longs.empty() && I->side;
    const int nlong = std::min<int>(NS, (int)longs.size());   // streams the long buckets use
    std::vector<hipStream_t> stream_of(I->H.buckets.size(), s);
    if (split_short)
        for (int bi : shorts) stream_of[bi] = I->side;
    auto cost = [&](int bi) {
        const afs::Bucket &b = I->H.buckets[bi];
        return (double)b.nslots * (double)(b.k_lo + b.k_hi);
    };
    std::sort(longs.begin(), longs.end(), [&](int a, int b) { return cost(a) > cost(b); });
    if (nlong > 1) {
        double load[NS] = {};
        for (int bi : longs) {
            int t = 0;
            for (int u = 1; u < nlong; ++u)
                if (load[u] < load[t]) t = u;
            load[t] += cost(bi);
            stream_of[bi] = t ? I->side_long[t - 1] : s;
        }
    }
    std::unique_lock<std::mutex> lock(I->side_mu, std::defer_lock);
    if (split_short || nlong > 1) {
        lock.lock();
        hipError_t e = hipEventRecord(I->fork, s);
        if (e == hipSuccess && split_short) e = hipStreamWaitEvent(I->side, I->fork, 0);
        for (int t = 1; t < nlong && e == hipSuccess; ++t) e = hipStreamWaitEvent(I->side_long[t - 1], I->fork, 0);
        if (e != hipSuccess) return dev_fail(e, "fork to the side streams");
    }
    // long buckets largest first, then the short ones (on their own stream)
    std::vector<int> order(longs);
    order.insert(order.end(), shorts.begin(), shorts.end());
    for (int bi : order) {
        const afs::Bucket &b = I->H.buckets[bi];
        afs::BucketLaunch bl{b.J, b.S, b.c0, b.nc, b.tile, b.ntiles, b.tile0, b.rpl};
        hipError_t e = afs::launch_fe_grad(I->D, bl, B, l.Bp, x, at<float>(ws, l.adj),
                                           want_part ? at<float>(ws, l.part) : nullptr, fe, dobj,
                                           grad, stream_of[bi], skip);
        if (e != hipSuccess) return dev_fail(e, "fe_grad launch");
    }
    if (split_short) {
        hipError_t e = hipEventRecord(I->join, I->side);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, I->join, 0);
        if (e != hipSuccess) return dev_fail(e, "join from the side stream");
    }
    for (int t = 1; t < nlong; ++t) {
        hipError_t e = hipEventRecord(I->join_long[t - 1], I->side_long[t - 1]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, I->join_long[t - 1], 0);
        if (e != hipSuccess) return dev_fail(e, "join from a long-bucket stream");
    }
    return AFS_OK;
}


afs_status read_options(const afs_options *opts, afs::PackOptions &po)
{
    if (!opts) return AFS_OK;
    if (opts->n_shapes < 0 || (opts->n_shapes > 0 && (!opts->shape_k_hi || !opts->shape_lanes || !opts->shape_seg)))
        return fail(AFS_EINVAL, "invalid shape arrays");
    for (int32_t e = 0; e < opts->n_shapes; ++e) {
        po.k_hi.push_back(opts->shape_k_hi[e]);
        po.lanes.push_back(opts->shape_lanes[e]);
        po.seg.push_back(opts->shape_seg[e]);
    }
    po.tile_short = opts->tile_short;
    po.tile_long = opts->tile_long;
    if (opts->shape_tile) po.tile.assign(opts->shape_tile, opts->shape_tile + std::max(opts->n_shapes, 0));
    for (int k = 1; k <= afs::kShortMax; ++k) {
        if (opts->short_tile) po.short_tile[k] = opts->short_tile[k - 1];
        if (opts->short_rpl) po.short_rpl[k] = opts->short_rpl[k - 1];
    }
    return AFS_OK;
}

// Upload the packed host instance to `device` (or keep it host-only for device < 0).
afs_status finish_create(afs_instance *I, int32_t device, afs_instance **out)
{
    if (device < 0) {
        I->device = -1;
        *out = I;
        return AFS_OK;
    }
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device >= count) {
        delete I;
        return fail(AFS_EINVAL, "no HIP device " + std::to_string(device));
    }
    I->device = device;
    DeviceGuard g(device);
    if (g.error() != hipSuccess) {
        I->device = -1;
        delete I;
        return dev_fail(g.error(), "hipSetDevice");
    }
    const afs::HostInstance &H = I->H;
    afs::DevInstance &D = I->D;
    D.n = H.n; D.C = H.C; D.L = H.L; D.n_inst = H.n_inst;
    std::vector<int32_t> con_off32(H.C + 1);
    for (int32_t c = 0; c <= H.C; ++c) con_off32[c] = (int32_t)H.con_off[c];
    std::vector<float4> tab(H.tab.size());
    for (size_t i = 0; i < H.tab.size(); ++i) tab[i] = make_float4(H.tab[i].x, H.tab[i].y, H.tab[i].z, H.tab[i].w);
    afs_status st = AFS_OK;
    if (st == AFS_OK) st = upload(I, H.bc_slot0, &D.bc_slot0);
    if (st == AFS_OK) st = upload(I, H.bc_k, &D.bc_k);
    if (st == AFS_OK) st = upload(I, H.bc_tab, &D.bc_tab);
    if (st == AFS_OK) st = upload(I, H.bc_orig, &D.bc_orig);
    if (st == AFS_OK) st = upload(I, H.bc_w, &D.bc_w);
    if (st == AFS_OK) st = upload(I, H.slot_lit, &D.slot_lit);
    if (st == AFS_OK) st = upload(I, H.slot_to_lit, &D.slot_to_lit);
    if (st == AFS_OK) st = upload(I, tab, &D.tab);
    D.tab_rows = (int64_t)tab.size();
    if (st == AFS_OK) st = upload(I, H.voff, &D.voff);
    if (st == AFS_OK) st = upload(I, H.vslot, &D.vslot);
    if (st == AFS_OK) st = upload(I, con_off32, &D.con_off);
    std::vector<int32_t> lits_pad(H.lits);
    lits_pad.resize(H.lits.size() + afs::kLitPad, 0);
    if (st == AFS_OK) st = upload(I, lits_pad, &D.lits);
    if (st == AFS_OK) st = upload(I, H.types, &D.types);
    if (st == AFS_OK) st = upload(I, H.params, &D.params);
    if (st == AFS_OK) st = upload(I, H.con_inst, &D.con_inst);
    if (st == AFS_OK) st = upload(I, H.var_inst, &D.var_inst);
    std::vector<int32_t> counted;
    for (int32_t c = 0; c < (int32_t)H.types.size(); ++c)
        if (H.types[c] == AFS_CARD_GE || H.types[c] == AFS_CARD_LT || H.types[c] == AFS_EK) counted.push_back(c);
    D.n_counted = (int32_t)counted.size();
    if (st == AFS_OK) st = upload(I, counted, &D.counted);
    if (st == AFS_OK) {
        hipError_t e = hipStreamCreateWithFlags(&I->side, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&I->fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&I->join, hipEventDisableTiming);
        for (int t = 0; t < afs_instance::kLongSides && e == hipSuccess; ++t) {
            e = hipStreamCreateWithFlags(&I->side_long[t], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&I->join_long[t], hipEventDisableTiming);
        }
        if (e != hipSuccess) st = dev_fail(e, "side streams");
    }
    if (st != AFS_OK) {
        const std::string msg = g_err;
        release(I);
        g_err = msg;
        return st;
    }
    *out = I;
    return AFS_OK;
}

}  // namespace

namespace afs {
afs_status set_last_error(afs_status s, const std::string &msg)
{
    return fail(s, msg);
}
}  // namespace afs

extern "C" {

const char *afs_last_error(void) { return g_err.c_str(); }

afs_status afs_coefficients(int32_t type, int32_t k, int32_t param, double *re, double *im)
{
    if (!re || !im) return fail(AFS_EINVAL, "output is NULL");
    if (k < 1 || k > afs::kMaxLen) return fail(AFS_EINVAL, "k out of range");
    if (type < 0 || type > 7) return fail(AFS_EINVAL, "unknown type");
    afs::coefficients(type, k, param, re, im);
    return AFS_OK;
}

afs_status afs_instance_create(int32_t n_vars, int32_t n_cons, const int64_t *con_off,
                               const int32_t *lits, const int32_t *types, const int32_t *params,
                               const float *weights, int32_t device, afs_instance **out)
{
    return afs_instance_create_ex(n_vars, n_cons, con_off, lits, types, params, weights, nullptr,
                                  device, out);
}

afs_status afs_instance_create_ex(int32_t n_vars, int32_t n_cons, const int64_t *con_off,
                                  const int32_t *lits, const int32_t *types, const int32_t *params,
                                  const float *weights, const afs_options *opts, int32_t device,
                                  afs_instance **out)
{
    if (!out) return fail(AFS_EINVAL, "out is NULL");
    *out = nullptr;
    afs::PackOptions po;
    afs_status st = read_options(opts, po);
    if (st != AFS_OK) return st;
    afs_instance *I = new (std::nothrow) afs_instance();
    if (!I) return fail(AFS_ENOMEM, "host allocation failed");
    std::string err;
    try {
        err = afs::build_instance(n_vars, n_cons, con_off, lits, types, params, weights, po, I->H);
    } catch (const std::bad_alloc &) {
        delete I;
        return fail(AFS_ENOMEM, "host allocation failed");
    }
    if (!err.empty()) {
        delete I;
        return fail(AFS_EINVAL, err);
    }
    return finish_create(I, device, out);
}

afs_status afs_batch_create(const afs_instance *const *parts, int32_t n_parts, const afs_options *opts,
                            int32_t device, afs_instance **out)
{
    if (!out) return fail(AFS_EINVAL, "out is NULL");
    *out = nullptr;
    if (!parts || n_parts < 1) return fail(AFS_EINVAL, "a batch needs at least one instance");
    afs::PackOptions po;
    afs_status st = read_options(opts, po);
    if (st != AFS_OK) return st;
    std::vector<afs::PartRef> refs(n_parts);
    for (int32_t i = 0; i < n_parts; ++i) {
        if (!parts[i]) return fail(AFS_EINVAL, "part " + std::to_string(i) + " is NULL");
        const afs::HostInstance &P = parts[i]->H;
        if (P.n_inst != 1) return fail(AFS_EINVAL, "parts must be plain instances, not batches");
        refs[i] = afs::PartRef{P.n, P.C, P.con_off.data(), P.lits.data(), P.types.data(), P.params.data(),
                               P.weights.data()};
    }
    afs_instance *I = new (std::nothrow) afs_instance();
    if (!I) return fail(AFS_ENOMEM, "host allocation failed");
    std::string err;
    try {
        err = afs::build_batch(refs, po, I->H);
    } catch (const std::bad_alloc &) {
        delete I;
        return fail(AFS_ENOMEM, "host allocation failed");
    }
    if (!err.empty()) {
        delete I;
        return fail(AFS_EINVAL, err);
    }
    return finish_create(I, device, out);
}

afs_status afs_batch_var_offsets(const afs_instance *I, int32_t *var0)
{
    if (!I || !var0) return fail(AFS_EINVAL, "NULL argument");
    for (int32_t i = 0; i <= I->H.n_inst; ++i) var0[i] = I->H.inst_var0[i];
    return AFS_OK;
}

void afs_instance_destroy(afs_instance *inst) { release(inst); }

afs_status afs_instance_info(const afs_instance *I, afs_info *out)
{
    if (!I || !out) return fail(AFS_EINVAL, "NULL argument");
    out->n_vars = I->H.n;
    out->n_cons = I->H.C;
    out->n_lits = I->H.L;
    out->n_buckets = (int32_t)I->H.buckets.size();
    out->n_tables = I->H.n_tables;
    out->max_k = I->H.max_k;
    out->device = I->device;
    out->n_inst = I->H.n_inst;
    return AFS_OK;
}

afs_status afs_bucket_info_get(const afs_instance *I, int32_t b, afs_bucket_info *out)
{
    if (!I || !out) return fail(AFS_EINVAL, "NULL argument");
    if (b < 0 || b >= (int32_t)I->H.buckets.size()) return fail(AFS_EINVAL, "bucket index out of range");
    const afs::Bucket &k = I->H.buckets[b];
    out->k_lo = k.k_lo;
    out->k_hi = k.k_hi;
    out->n_cons = k.nc;
    out->n_lits = k.nslots;
    out->lanes_per_restart = k.J;
    out->lits_per_lane = k.S;
    out->slot0 = k.slot0;
    out->tile = k.tile;
    out->rpl = k.rpl;
    return AFS_OK;
}

afs_status afs_instance_slot_map(const afs_instance *I, int64_t *slot_to_lit)
{
    if (!I || (!slot_to_lit && I->H.L > 0)) return fail(AFS_EINVAL, "NULL argument");
    for (int64_t s = 0; s < I->H.L; ++s) slot_to_lit[s] = I->H.slot_to_lit[s];
    return AFS_OK;
}

afs_status afs_instance_transpose(const afs_instance *I, int64_t *voff, int64_t *vslot)
{
    if (!I || !voff || (!vslot && I->H.L > 0)) return fail(AFS_EINVAL, "NULL argument");
    for (int32_t v = 0; v <= I->H.n; ++v) voff[v] = I->H.voff[v];
    for (int64_t s = 0; s < I->H.L; ++s) vslot[s] = I->H.vslot[s];
    return AFS_OK;
}

afs_status afs_workspace_bytes(const afs_instance *I, int32_t B, size_t *bytes)
{
    if (!I || !bytes) return fail(AFS_EINVAL, "NULL argument");
    if (B < 0) return fail(AFS_EINVAL, "B must be >= 0");
    *bytes = ws_layout(I->H, B).total;
    return AFS_OK;
}

afs_status afs_fe_grad(afs_instance *I, int32_t B, const float *x, void *ws, size_t ws_bytes,
                       int32_t bucket_lo, int32_t bucket_hi, int32_t want_obj, float *fe,
                       void *stream)
{
    afs_status st = check_call(I, B);
    if (st != AFS_OK) return st;
    WsLayout l;
    if ((st = check_ws(I, B, ws, ws_bytes, l)) != AFS_OK) return st;
    const int nb = (int)I->H.buckets.size();
    if (bucket_lo < 0 || bucket_hi > nb || bucket_lo > bucket_hi) return fail(AFS_EINVAL, "bucket range out of range");
    if (!x && B > 0) return fail(AFS_EINVAL, "x is NULL");
    DeviceGuard g(I->device);
    if (g.error() != hipSuccess) return dev_fail(g.error(), "hipSetDevice");
    return fe_grad_range(I, B, x, ws, l, bucket_lo, bucket_hi, want_obj != 0, fe, (hipStream_t)stream);
}

afs_status afs_fe_grad_buckets(afs_instance *I, int32_t B, const float *x, void *ws, size_t ws_bytes,
                               const int32_t *buckets, int32_t n_buckets, int32_t want_obj, float *fe,
                               void *stream)
{
    afs_status st = check_call(I, B);
    if (st != AFS_OK) return st;
    WsLayout l;
    if ((st = check_ws(I, B, ws, ws_bytes, l)) != AFS_OK) return st;
    if (n_buckets < 0 || (n_buckets > 0 && !buckets)) return fail(AFS_EINVAL, "bucket list is NULL");
    const int nb = (int)I->H.buckets.size();
    std::vector<int> set;
    std::vector<char> seen(nb, 0);
    for (int32_t i = 0; i < n_buckets; ++i) {
        if (buckets[i] < 0 || buckets[i] >= nb) return fail(AFS_EINVAL, "bucket index out of range");
        if (seen[buckets[i]]) return fail(AFS_EINVAL, "bucket listed twice");
        seen[buckets[i]] = 1;
        set.push_back(buckets[i]);
    }
    if (!x && B > 0) return fail(AFS_EINVAL, "x is NULL");
    DeviceGuard g(I->device);
    if (g.error() != hipSuccess) return dev_fail(g.error(), "hipSetDevice");
    return fe_grad_set(I, B, x, ws, l, set, want_obj != 0, fe, (hipStream_t)stream);
}

afs_status afs_scatter(afs_instance *I, int32_t B, void *ws, size_t ws_bytes, float *obj,
                       float *grad, void *stream)
{
    afs_status st = check_call(I, B);
    if (st != AFS_OK) return st;
    WsLayout l;
    if ((st = check_ws(I, B, ws, ws_bytes, l)) != AFS_OK) return st;
    DeviceGuard g(I->device);
    if (g.error() != hipSuccess) return dev_fail(g.error(), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (grad && (e = afs::launch_scatter(I->D, B, l.Bp, at<float>(ws, l.adj), grad, s)) != hipSuccess)
        return dev_fail(e, "scatter launch");
    if (obj && (e = afs::launch_obj_reduce(I->H.total_tiles, B, l.Bp, at<float>(ws, l.part),
                                           at<float>(ws, l.part2), obj, s)) != hipSuccess)
        return dev_fail(e, "objective reduction launch");
    return AFS_OK;
}

}  // extern "C"

namespace {

// afs_eval after the workspace check: FE + adjoints into ws, then the gradient
// sum, the objective reduction and the literal-order adjoints as requested.
// Only the adjoint rows and the objective partials of ws are used (everything
// below l.bits).
afs_status eval_body(afs_instance *I, int32_t B, const float *x, void *ws, const WsLayout &l, float *obj,
                     float *grad, float *fe, float *adj, void *stream)
{
    if (!x && B > 0) return fail(AFS_EINVAL, "x is NULL");
    DeviceGuard g(I->device);
    if (g.error() != hipSuccess) return dev_fail(g.error(), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    const afs_status st = fe_grad_range(I, B, x, ws, l, 0, (int)I->H.buckets.size(), obj != nullptr, fe, s);
    if (st != AFS_OK) return st;
    hipError_t e;
    if (grad && (e = afs::launch_scatter(I->D, B, l.Bp, at<float>(ws, l.adj), grad, s)) != hipSuccess)
        return dev_fail(e, "scatter launch");
    if (obj && (e = afs::launch_obj_reduce(I->H.total_tiles, B, l.Bp, at<float>(ws, l.part),
                                           at<float>(ws, l.part2), obj, s)) != hipSuccess)
        return dev_fail(e, "objective reduction launch");
    if (adj && (e = afs::launch_permute_adj(I->D, B, l.Bp, at<float>(ws, l.adj), adj, s)) != hipSuccess)
        return dev_fail(e, "adjoint permute launch");
    return AFS_OK;
}

}  // namespace

namespace afs {

size_t eval_scratch_bytes(const afs_instance *I, int32_t B)
{
    return ws_layout(I->H, B).bits;
}

afs_status eval_in_scratch(afs_instance *I, int32_t B, const float *x, void *scratch, size_t scratch_bytes,
                           float *obj, float *grad, float *fe, float *adj, void *stream)
{
    afs_status st = check_call(I, B);
    if (st != AFS_OK) return st;
    const WsLayout l = ws_layout(I->H, B);
    if (reinterpret_cast<uintptr_t>(scratch) % 256) return fail(AFS_EINVAL, "scratch is not 256-byte aligned");
    if (l.bits > scratch_bytes)
        return fail(AFS_EINVAL, "evaluation needs " + std::to_string(l.bits) + " bytes of scratch, more than " +
                                    std::to_string(scratch_bytes));
    return eval_body(I, B, x, scratch, l, obj, grad, fe, adj, stream);
}

}  // namespace afs

extern "C" {

afs_status afs_eval(afs_instance *I, int32_t B, const float *x, void *ws, size_t ws_bytes,
                    float *obj, float *grad, float *fe, float *adj, void *stream)
{
    afs_status st = check_call(I, B);
    if (st != AFS_OK) return st;
    WsLayout l;
    if ((st = check_ws(I, B, ws, ws_bytes, l)) != AFS_OK) return st;
    return eval_body(I, B, x, ws, l, obj, grad, fe, adj, stream);
}

afs_status afs_eval_fwd(afs_instance *I, int32_t B, const float *x, void *ws, size_t ws_bytes,
                        float *obj, float *fe, void *stream)
{
    afs_status st = check_call(I, B);
    if (st != AFS_OK) return st;
    WsLayout l;
    if ((st = check_ws(I, B, ws, ws_bytes, l)) != AFS_OK) return st;
    if (B > 0 && (!x || !obj)) return fail(AFS_EINVAL, "x or obj is NULL");
    DeviceGuard g(I->device);
    if (g.error() != hipSuccess) return dev_fail(g.error(), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    st = fe_grad_range(I, B, x, ws, l, 0, (int)I->H.buckets.size(), true, fe, s, nullptr, false);
    if (st != AFS_OK) return st;
    hipError_t e = afs::launch_obj_reduce(I->H.total_tiles, B, l.Bp, at<float>(ws, l.part),
                                          at<float>(ws, l.part2), obj, s);
    return e == hipSuccess ? AFS_OK : dev_fail(e, "objective reduction launch");
}

afs_status afs_eval_adjoint(afs_instance *I, int32_t B, const float *x, const float *dobj, void *ws,
                            size_t ws_bytes, float *grad, float *adj, void *stream)
{
    afs_status st = check_call(I, B);
    if (st != AFS_OK) return st;
    WsLayout l;
    if ((st = check_ws(I, B, ws, ws_bytes, l)) != AFS_OK) return st;
    if (B > 0 && (!x || !grad)) return fail(AFS_EINVAL, "x or grad is NULL");
    DeviceGuard g(I->device);
    if (g.error() != hipSuccess) return dev_fail(g.error(), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    st = fe_grad_range(I, B, x, ws, l, 0, (int)I->H.buckets.size(), false, nullptr, s, dobj, true);
    if (st != AFS_OK) return st;
    hipError_t e = afs::launch_scatter(I->D, B, l.Bp, at<float>(ws, l.adj), grad, s);
    if (e != hipSuccess) return dev_fail(e, "scatter launch");
    if (adj && (e = afs::launch_permute_adj(I->D, B, l.Bp, at<float>(ws, l.adj), adj, s)) != hipSuccess)
        return dev_fail(e, "adjoint permute launch");
    return AFS_OK;
}

afs_status afs_step(afs_instance *I, int32_t B, float *x, const float *grad, float lr,
                    const uint8_t *fixed, int32_t n_partial, const uint8_t *done, void *stream)
{
    afs_status st = check_call(I, B);
    if (st != AFS_OK) return st;
    if (B > 0 && (!x || !grad)) return fail(AFS_EINVAL, "x or grad is NULL");
    if ((st = check_partial(B, fixed, n_partial)) != AFS_OK) return st;
    DeviceGuard g(I->device);
    if (g.error() != hipSuccess) return dev_fail(g.error(), "hipSetDevice");
    hipError_t e = afs::launch_step(I->D, B, x, grad, lr, fixed, partial_rows(n_partial), done, (hipStream_t)stream);
    return e == hipSuccess ? AFS_OK : dev_fail(e, "step launch");
}

afs_status afs_round_verify(afs_instance *I, int32_t B, const float *x, uint32_t *bits, void *ws,
                            size_t ws_bytes, int32_t *unsat, uint8_t *done, void *stream)
{
    afs_status st = check_call(I, B);
    if (st != AFS_OK) return st;
    if (B > 0 && (!x || !unsat)) return fail(AFS_EINVAL, "x or unsat is NULL");
    WsLayout l;
    if ((st = check_ws(I, B, ws, ws_bytes, l)) != AFS_OK) return st;
    if (!bits) bits = at<uint32_t>(ws, l.bits);
    DeviceGuard g(I->device);
    if (g.error() != hipSuccess) return dev_fail(g.error(), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    const int pairs = I->H.n_inst * B;
    hipError_t e = afs::launch_round(I->D, B, x, bits, unsat, s);
    if (e == hipSuccess) e = afs::launch_verify(I->D, B, bits, at<uint32_t>(ws, l.viol), unsat, s);
    if (e == hipSuccess && done)
        e = afs::launch_finalize(pairs, B, unsat, done, nullptr, nullptr, afs::FIN_VERIFY, s);
    return e == hipSuccess ? AFS_OK : dev_fail(e, "round/verify launch");
}

afs_status afs_pgd_init(afs_instance *I, int32_t B, const float *x, void *ws, size_t ws_bytes,
                        const afs_pgd_state *P, void *stream)
{
    afs_status st = check_call(I, B);
    if (st != AFS_OK) return st;
    WsLayout l;
    if ((st = check_ws(I, B, ws, ws_bytes, l)) != AFS_OK) return st;
    if (!P || !P->unsat || !P->done || !P->first_sat || !P->counter) return fail(AFS_EINVAL, "incomplete PGD state");
    if (B > 0 && !x) return fail(AFS_EINVAL, "x is NULL");
    DeviceGuard g(I->device);
    if (g.error() != hipSuccess) return dev_fail(g.error(), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    uint32_t *bits = at<uint32_t>(ws, l.bits);
    hipError_t e = afs::launch_round(I->D, B, x, bits, P->unsat, s);
    if (e == hipSuccess) e = afs::launch_verify(I->D, B, bits, at<uint32_t>(ws, l.viol), P->unsat, s);
    if (e == hipSuccess)
        e = afs::launch_finalize(I->H.n_inst * B, B, P->unsat, P->done, P->first_sat, P->counter, afs::FIN_INIT, s,
                                 nullptr, 0.0f, 0.0f, at<uint8_t>(ws, l.moved));
    return e == hipSuccess ? AFS_OK : dev_fail(e, "PGD init launch");
}

static afs_status pgd_call(afs_instance *I, int32_t B, float *x, float lr, const uint8_t *fixed, int32_t n_partial,
                           float delta, void *ws, size_t ws_bytes, const afs_pgd_state *P, void *stream, bool with_fe,
                           float *vel = nullptr, float mu = 0.0f)
{
    afs_status st = check_call(I, B);
    if (st != AFS_OK) return st;
    WsLayout l;
    if ((st = check_ws(I, B, ws, ws_bytes, l)) != AFS_OK) return st;
    if (!P || !P->unsat || !P->done || !P->first_sat || !P->counter) return fail(AFS_EINVAL, "incomplete PGD state");
    if (B > 0 && !x) return fail(AFS_EINVAL, "x is NULL");
    if ((st = check_partial(B, fixed, n_partial)) != AFS_OK) return st;
    DeviceGuard g(I->device);
    if (g.error() != hipSuccess) return dev_fail(g.error(), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    if (with_fe) {
        st = fe_grad_range(I, B, x, ws, l, 0, (int)I->H.buckets.size(), false, nullptr, s);
        if (st != AFS_OK) return st;
    }
    uint32_t *bits = at<uint32_t>(ws, l.bits);
    hipError_t e = afs::launch_scatter_step(I->D, B, l.Bp, at<float>(ws, l.adj), x, lr, fixed,
                                            partial_rows(n_partial), P->done, bits, P->unsat, s, nullptr, 0.0f,
                                            vel, mu);
    if (e == hipSuccess) e = afs::launch_verify(I->D, B, bits, at<uint32_t>(ws, l.viol), P->unsat, s);
    if (e == hipSuccess)
        e = afs::launch_finalize(I->H.n_inst * B, B, P->unsat, P->done, P->first_sat, P->counter, afs::FIN_STEP, s,
                                 nullptr, lr, delta);
    return e == hipSuccess ? AFS_OK : dev_fail(e, "PGD step launch");
}

afs_status afs_pgd_step(afs_instance *I, int32_t B, float *x, float lr, const uint8_t *fixed, int32_t n_partial,
                        void *ws, size_t ws_bytes, const afs_pgd_state *P, void *stream)
{
    return pgd_call(I, B, x, lr, fixed, n_partial, 0.0f, ws, ws_bytes, P, stream, true);
}

afs_status afs_pgd_update(afs_instance *I, int32_t B, float *x, float lr, const uint8_t *fixed, int32_t n_partial,
                          void *ws, size_t ws_bytes, const afs_pgd_state *P, void *stream)
{
    return pgd_call(I, B, x, lr, fixed, n_partial, 0.0f, ws, ws_bytes, P, stream, false);
}

afs_status afs_pgd_step_momentum(afs_instance *I, int32_t B, float *x, float *vel, float lr, float mu,
                                 const uint8_t *fixed, int32_t n_partial, void *ws, size_t ws_bytes,
                                 const afs_pgd_state *P, void *stream)
{
    if (B > 0 && !vel) return fail(AFS_EINVAL, "vel is NULL");
    if (!(mu >= 0.0f && mu < 1.0f)) return fail(AFS_EINVAL, "mu must lie in [0, 1)");
    return pgd_call(I, B, x, lr, fixed, n_partial, 0.0f, ws, ws_bytes, P, stream, true, vel, mu);
}

static afs_status check_search(const afs_line_search *ls)
{
    if (!ls) return fail(AFS_EINVAL, "line search parameters are NULL");
    if (!(ls->max_step > 0.0f) || !std::isfinite(ls->max_step)) return fail(AFS_EINVAL, "max_step must be > 0 and finite");
    if (!(ls->shrink > 0.0f && ls->shrink < 1.0f)) return fail(AFS_EINVAL, "shrink must lie in (0, 1)");
    if (!(ls->armijo >= 0.0f && ls->armijo < 1.0f)) return fail(AFS_EINVAL, "armijo must lie in [0, 1)");
    if (ls->trials < 1 || ls->trials > 64) return fail(AFS_EINVAL, "trials must lie in 1..64");
    return AFS_OK;
}

afs_status afs_search_workspace_bytes(const afs_instance *I, int32_t B, size_t *bytes)
{
    if (!I || !bytes) return fail(AFS_EINVAL, "NULL argument");
    if (B < 0) return fail(AFS_EINVAL, "B must be >= 0");
    *bytes = search_layout(I->H, B).total;
    return AFS_OK;
}

static afs_status search_call(afs_instance *I, int32_t B, float *x, const afs_line_search *ls, const uint8_t *fixed,
                              int32_t n_partial, float delta, float eps, void *ws, size_t ws_bytes, void *sws,
                              size_t sws_bytes, const afs_pgd_state *P, float *eta_out, hipStream_t s)
{
    afs_status st = check_call(I, B);
    if (st != AFS_OK) return st;
    if (I->H.n_inst != 1) return fail(AFS_EINVAL, "the line search takes a plain instance, not a batch");
    if ((st = check_search(ls)) != AFS_OK) return st;
    WsLayout l;
    if ((st = check_ws(I, B, ws, ws_bytes, l)) != AFS_OK) return st;
    const SearchLayout q = search_layout(I->H, B);
    if (!sws) return fail(AFS_EINVAL, "search workspace is NULL");
    if (reinterpret_cast<uintptr_t>(sws) % 256) return fail(AFS_EINVAL, "search workspace is not 256-byte aligned");
    if (sws_bytes < q.total)
        return fail(AFS_EINVAL, "search workspace too small: need " + std::to_string(q.total) + " bytes");
    if (!P || !P->unsat || !P->done || !P->first_sat || !P->counter) return fail(AFS_EINVAL, "incomplete PGD state");
    if (B > 0 && !x) return fail(AFS_EINVAL, "x is NULL");
    if ((st = check_partial(B, fixed, n_partial)) != AFS_OK) return st;
    const int rows = partial_rows(n_partial);
    const int nb = (int)I->H.buckets.size(), tiles = I->H.total_tiles;
    float *g = at<float>(sws, q.g), *xt = at<float>(sws, q.xt);
    float *f0 = at<float>(sws, q.f0), *ft = at<float>(sws, q.ft), *dot = at<float>(sws, q.dot);
    float *eta = eta_out ? eta_out : at<float>(sws, q.eta);
    uint8_t *acc = at<uint8_t>(sws, q.acc);
    float *part = at<float>(ws, l.part), *part2 = at<float>(ws, l.part2);
    // objective and gradient at x
    if ((st = fe_grad_range(I, B, x, ws, l, 0, nb, true, nullptr, s)) != AFS_OK) return st;
    hipError_t e = afs::launch_obj_reduce(tiles, B, l.Bp, part, part2, f0, s);
    if (e == hipSuccess) e = afs::launch_scatter(I->D, B, l.Bp, at<float>(ws, l.adj), g, s);
    if (e == hipSuccess) e = afs::launch_search_init(B, ls->max_step, P->done, eta, acc, s);
    if (e != hipSuccess) return dev_fail(e, "line search launch");
    for (int j = 0; j < ls->trials; ++j) {
        e = afs::launch_trial(I->D, B, l.Bp, x, g, eta, acc, fixed, rows, xt, at<float>(sws, q.dpart), s);
        if (e == hipSuccess)
            e = afs::launch_obj_reduce(q.vtiles, B, l.Bp, at<float>(sws, q.dpart), at<float>(sws, q.dpart2), dot, s);
        if (e != hipSuccess) return dev_fail(e, "line search trial launch");
        // restarts that have decided (acc != 0) are not needed: whole waves of them skip
        if ((st = fe_grad_range(I, B, xt, ws, l, 0, nb, true, nullptr, s, nullptr, false, acc)) != AFS_OK)
            return st;
        e = afs::launch_obj_reduce(tiles, B, l.Bp, part, part2, ft, s);
        if (e == hipSuccess)
            e = afs::launch_accept(B, f0, ft, dot, ls->armijo, ls->shrink, j == ls->trials - 1, eta, acc, s);
        if (e != hipSuccess) return dev_fail(e, "line search test launch");
    }
    uint32_t *bits = at<uint32_t>(ws, l.bits);
    uint8_t *moved = eps > 0.0f ? at<uint8_t>(ws, l.moved) : nullptr;
    e = afs::launch_search_step(I->D, B, x, g, eta, fixed, rows, P->done, bits, P->unsat, s, moved, eps);
    if (e == hipSuccess) e = afs::launch_verify(I->D, B, bits, at<uint32_t>(ws, l.viol), P->unsat, s);
    if (e == hipSuccess)
        e = afs::launch_finalize(B, B, P->unsat, P->done, P->first_sat, P->counter, afs::FIN_STEP, s, eta, 0.0f,
                                 delta, moved, eps);
    return e == hipSuccess ? AFS_OK : dev_fail(e, "line search step launch");
}

afs_status afs_pgd_search_step(afs_instance *I, int32_t B, float *x, const afs_line_search *ls,
                               const uint8_t *fixed, int32_t n_partial, float delta, void *ws, size_t ws_bytes,
                               void *sws, size_t sws_bytes, const afs_pgd_state *P, float *eta, void *stream)
{
    afs_status st = check_call(I, B);
    if (st != AFS_OK) return st;
    DeviceGuard g(I->device);
    if (g.error() != hipSuccess) return dev_fail(g.error(), "hipSetDevice");
    return search_call(I, B, x, ls, fixed, n_partial, delta, 0.0f, ws, ws_bytes, sws, sws_bytes, P, eta,
                       (hipStream_t)stream);
}

afs_status afs_init_points(afs_instance *I, int32_t B, uint64_t seed, const int8_t *values, int32_t n_partial,
                           float *x, void *stream)
{
    afs_status st = check_call(I, B);
    if (st != AFS_OK) return st;
    if (B > 0 && !x) return fail(AFS_EINVAL, "x is NULL");
    if ((st = check_partial(B, values, n_partial)) != AFS_OK) return st;
    DeviceGuard g(I->device);
    if (g.error() != hipSuccess) return dev_fail(g.error(), "hipSetDevice");
    hipError_t e = afs::launch_init_points(I->H.n, B, seed, values, partial_rows(n_partial), x, (hipStream_t)stream);
    return e == hipSuccess ? AFS_OK : dev_fail(e, "start point launch");
}

// Most iterations the driver captures into one graph.
constexpr int32_t kGraphIters = 64;

// One constant-step iteration of the driver with the verification on the
// instance's verify stream: FE of X_(t-1) on s; the step waits for the previous
// iteration's verification (it rewrites the bits and counts that one reads, and
// reads its done flags) unless this is the first iteration of a block; the
// verification of X_(t) then runs beside the next iteration's FE kernels.  The
// caller joins `verified` into s at the end of the block.  Arguments are
// validated by afs_pgd.
static afs_status overlapped_step(afs_instance *I, int32_t B, float *x, const afs_pgd_params *prm, void *ws,
                                  const WsLayout &l, const afs_pgd_state *P, hipStream_t s, bool wait_prev)
{
    afs_status st = fe_grad_range(I, B, x, ws, l, 0, (int)I->H.buckets.size(), false, nullptr, s);
    if (st != AFS_OK) return st;
    hipError_t e = wait_prev ? hipStreamWaitEvent(s, I->verified, 0) : hipSuccess;
    uint32_t *bits = at<uint32_t>(ws, l.bits);
    uint8_t *moved = prm->epsilon > 0.0f ? at<uint8_t>(ws, l.moved) : nullptr;
    float *vel = prm->momentum > 0.0f ? prm->velocity : nullptr;
    if (e == hipSuccess)
        e = afs::launch_scatter_step(I->D, B, l.Bp, at<float>(ws, l.adj), x, prm->lr, prm->fixed,
                                     partial_rows(prm->n_partial), P->done, bits, P->unsat, s, moved, prm->epsilon,
                                     vel, prm->momentum);
    if (e == hipSuccess) e = hipEventRecord(I->stepped, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(I->verify, I->stepped, 0);
    if (e == hipSuccess) e = afs::launch_verify(I->D, B, bits, at<uint32_t>(ws, l.viol), P->unsat, I->verify);
    if (e == hipSuccess)
        e = afs::launch_finalize(I->H.n_inst * B, B, P->unsat, P->done, P->first_sat, P->counter, afs::FIN_STEP,
                                 I->verify, nullptr, prm->lr, prm->delta, moved, prm->epsilon);
    if (e == hipSuccess) e = hipEventRecord(I->verified, I->verify);
    return e == hipSuccess ? AFS_OK : dev_fail(e, "PGD step launch");
}

afs_status afs_pgd(afs_instance *I, int32_t B, float *x, const afs_pgd_params *prm, void *ws, size_t ws_bytes,
                   const afs_pgd_state *P, float *obj, int32_t *iters, void *stream)
{
    afs_status st = check_call(I, B);
    if (st != AFS_OK) return st;
    if (!prm) return fail(AFS_EINVAL, "params is NULL");
    if (prm->max_iters < 0 || prm->poll < 1) return fail(AFS_EINVAL, "max_iters must be >= 0 and poll >= 1");
    if (!(prm->delta >= 0.0f) || !(prm->epsilon >= 0.0f) || !std::isfinite(prm->epsilon))
        return fail(AFS_EINVAL, "delta and epsilon must be >= 0 (epsilon finite)");
    if (prm->search && (st = check_search(prm->search)) != AFS_OK) return st;
    if (prm->search && I->H.n_inst != 1) return fail(AFS_EINVAL, "the line search takes a plain instance, not a batch");
    if (!(prm->momentum >= 0.0f && prm->momentum < 1.0f)) return fail(AFS_EINVAL, "momentum must lie in [0, 1)");
    if (prm->momentum > 0.0f && prm->search) return fail(AFS_EINVAL, "momentum does not combine with the line search");
    if (prm->momentum > 0.0f && B > 0 && !prm->velocity) return fail(AFS_EINVAL, "momentum needs a velocity array");
    if ((st = check_partial(B, prm->fixed, prm->n_partial)) != AFS_OK) return st;
    WsLayout l;
    if ((st = check_ws(I, B, ws, ws_bytes, l)) != AFS_OK) return st;
    if (!P || !P->unsat || !P->done || !P->first_sat || !P->counter) return fail(AFS_EINVAL, "incomplete PGD state");
    if (B > 0 && !x) return fail(AFS_EINVAL, "x is NULL");
    DeviceGuard g(I->device);
    if (g.error() != hipSuccess) return dev_fail(g.error(), "hipSetDevice");
    std::lock_guard<std::mutex> lock(I->drive_mu);
    // the driver's streams are made on its first use, so that instances that never
    // run it hold fewer streams than the device has hardware queues
    hipError_t e = hipSuccess;
    if (!I->drive) {
        hipStream_t dr = nullptr, vf = nullptr;
        hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
        void *pinned = nullptr;
        e = hipStreamCreateWithFlags(&dr, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&vf, hipStreamNonBlocking);
        for (int i = 0; i < 4 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
        if (e == hipSuccess) e = hipHostMalloc(&pinned, 4 * sizeof(int32_t), hipHostMallocDefault);
        if (e != hipSuccess) {
            if (pinned) (void)hipHostFree(pinned);
            for (hipEvent_t x : ev)
                if (x) (void)hipEventDestroy(x);
            if (vf) (void)hipStreamDestroy(vf);
            if (dr) (void)hipStreamDestroy(dr);
            return dev_fail(e, "driver streams");
        }
        I->counter_host = static_cast<int32_t *>(pinned);
        I->drive_in = ev[0];
        I->drive_out = ev[1];
        I->stepped = ev[2];
        I->verified = ev[3];
        I->verify = vf;
        I->drive = dr;
    }
    hipStream_t caller = (hipStream_t)stream, s = I->drive;
    e = hipEventRecord(I->drive_in, caller);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, I->drive_in, 0);
    if (e != hipSuccess) return dev_fail(e, "ordering the driver stream");

    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    auto finish = [&](afs_status result) {
        // the executable graph is destroyed only once its last replay has finished
        if (exec) {
            const hipError_t es = hipStreamSynchronize(s);
            if (result == AFS_OK && es != hipSuccess) result = dev_fail(es, "hipStreamSynchronize");
            (void)hipGraphExecDestroy(exec);
        }
        if (graph) (void)hipGraphDestroy(graph);
        // the caller's stream continues after everything enqueued here
        hipError_t e2 = hipEventRecord(I->drive_out, s);
        if (e2 == hipSuccess) e2 = hipStreamWaitEvent(caller, I->drive_out, 0);
        if (result == AFS_OK && e2 != hipSuccess) return dev_fail(e2, "ordering the caller's stream");
        return result;
    };
    // the counter comes back through the instance's pinned buffer, so the copy
    // never writes into pageable memory (here: this call's stack)
    auto read_counter = [&](int32_t *host) {
        hipError_t e2 = hipMemcpyAsync(I->counter_host, P->counter, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);
        if (e2 == hipSuccess)
            for (int i = 0; i < 4; ++i) host[i] = I->counter_host[i];
        return e2;
    };
    // one iteration: constant step (its verification overlapping the next
    // iteration's FE), or the backtracking line search
    auto iterate = [&](int32_t i) {
        if (prm->search)
            return search_call(I, B, x, prm->search, prm->fixed, prm->n_partial, prm->delta, prm->epsilon, ws, ws_bytes,
                               prm->search_ws, prm->search_ws_bytes, P, nullptr, s);
        return overlapped_step(I, B, x, prm, ws, l, P, s, i > 0);
    };
    // end of a block of iterations: s continues after the last verification
    auto join = [&]() { return prm->search ? hipSuccess : hipStreamWaitEvent(s, I->verified, 0); };

    if ((st = afs_pgd_init(I, B, x, ws, ws_bytes, P, s)) != AFS_OK) return finish(st);
    int32_t counter[4] = {0, 0, 0, 0};
    const int32_t pairs = I->H.n_inst * B;
    for (int32_t t = 0; t < prm->max_iters;) {
        if (prm->stop_on_sat || prm->delta > 0.0f || prm->epsilon > 0.0f) {
            if ((e = read_counter(counter)) != hipSuccess) return finish(dev_fail(e, "reading the counter"));
            if (prm->stop_on_sat && counter[1] > 0) break;
            if (counter[2] >= pairs) break;   // every restart verified or converged
        }
        const int32_t n = std::min(prm->poll, prm->max_iters - t);
        // with use_graph, whole blocks of `block` iterations replay one captured
        // graph (at most kGraphIters iterations, so a long poll period does not
        // make a huge graph); what is left of the poll period runs eagerly
        const int32_t block = std::min(prm->poll, kGraphIters);
        const int32_t replays = prm->use_graph ? n / block : 0;
        if (replays > 0 && !exec) {
            // capture `block` iterations once; every launch in them is allocation- and sync-free
            if ((e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal)) != hipSuccess)
                return finish(dev_fail(e, "hipStreamBeginCapture"));
            afs_status cs = AFS_OK;
            for (int32_t i = 0; i < block && cs == AFS_OK; ++i) cs = iterate(i);
            if (cs == AFS_OK && (e = join()) != hipSuccess) cs = dev_fail(e, "joining the verify stream");
            const hipError_t ec = hipStreamEndCapture(s, &graph);
            if (cs != AFS_OK) return finish(cs);
            if (ec != hipSuccess) return finish(dev_fail(ec, "hipStreamEndCapture"));
            if ((e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0)) != hipSuccess)
                return finish(dev_fail(e, "hipGraphInstantiate"));
        }
        for (int32_t r = 0; r < replays; ++r)
            if ((e = hipGraphLaunch(exec, s)) != hipSuccess) return finish(dev_fail(e, "hipGraphLaunch"));
        const int32_t rest = n - replays * block;
        if (rest > 0) {
            for (int32_t i = 0; i < rest; ++i)
                if ((st = iterate(i)) != AFS_OK) return finish(st);
            if ((e = join()) != hipSuccess) return finish(dev_fail(e, "joining the verify stream"));
        }
        t += n;
    }
    if (obj && (st = afs_eval_fwd(I, B, x, ws, ws_bytes, obj, nullptr, s)) != AFS_OK) return finish(st);
    if (iters) {
        if ((e = read_counter(counter)) != hipSuccess) return finish(dev_fail(e, "reading the counter"));
        *iters = counter[0];
    }
    return finish(AFS_OK);
}

}  // extern "C"
