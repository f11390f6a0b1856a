// decompose.cpp -- long-constraint decomposition (Sec. 5, constraint length
// ceiling): a long OR, XOR, NAE, AMO or EO constraint becomes a chain of shorter
// constraints of the same type joined by auxiliary variables, so that for every
// assignment of the original variables the constraint holds exactly when some
// values of the auxiliary variables satisfy every piece.
//
// Chain of p pieces over the literal groups G_1 .. G_p (the constraint's
// literals in order) and auxiliary variables a_1 .. a_(p-1):
//   OR, NAE, AMO, EO : piece i holds -a_(i-1) (i > 1), G_i, a_i (i < p).
//     OR/AMO/EO: a_i = "no literal of G_1 .. G_i is true" satisfies every piece
//     whenever the constraint holds, and a violated constraint leaves some piece
//     violated for every choice; NAE: two pieces meeting at a_i see it with
//     opposite values, so a monochrome input propagates through the chain.
//   XOR : piece i holds a_(i-1) (i > 1), G_i, a_i (i < p) with even parity, the
//     last piece the constraint's parity: a_i is the parity of G_1 .. G_i.
// p = ceil((k - 2) / (max_len - 2)) is the fewest pieces of at most max_len
// literals (the chain adds 2(p-1) auxiliary literals); the k + 2(p-1) literals
// are spread so that piece lengths differ by at most one.

#include "afsat.h"

#include <climits>
#include <cstdint>
#include <string>

#include "instance.hpp"

namespace {

bool decomposable(int32_t type)
{
    return type == AFS_OR || type == AFS_XOR || type == AFS_NAE || type == AFS_AMO || type == AFS_EO;
}

// Pieces for a constraint of length k (1 when it stays whole).
int64_t pieces(int32_t type, int64_t k, int32_t max_len)
{
    if (!decomposable(type) || k <= max_len) return 1;
    return (k - 2 + max_len - 3) / (max_len - 2);
}

// Length of piece i of p for a constraint of length k.
int64_t piece_len(int64_t k, int64_t p, int64_t i)
{
    const int64_t total = k + 2 * (p - 1);
    return total / p + (i < total % p ? 1 : 0);
}

afs_status check_input(int32_t n, int32_t C, const int64_t *con_off, const int32_t *types, int32_t max_len,
                       int64_t &n_out, int64_t &C_out, int64_t &L_out)
{
    if (n < 0 || C < 0) return afs::set_last_error(AFS_EINVAL, "n and C must be >= 0");
    if (C > 0 && (!con_off || !types)) return afs::set_last_error(AFS_EINVAL, "con_off or types is NULL");
    if (max_len < 3 || max_len > AFS_MAX_LEN)
        return afs::set_last_error(AFS_EINVAL, "max_len must be in [3, " + std::to_string(AFS_MAX_LEN) + "]");
    if (C > 0 && con_off[0] != 0) return afs::set_last_error(AFS_EINVAL, "con_off[0] must be 0");
    n_out = n;
    C_out = 0;
    L_out = 0;
    for (int32_t c = 0; c < C; ++c) {
        const int64_t k = con_off[c + 1] - con_off[c];
        if (k < 1) return afs::set_last_error(AFS_EINVAL, "constraint " + std::to_string(c) + " is empty");
        if (types[c] < AFS_OR || types[c] > AFS_EK)
            return afs::set_last_error(AFS_EINVAL, "constraint " + std::to_string(c) + " has an unknown type");
        const int64_t p = pieces(types[c], k, max_len);
        n_out += p - 1;
        C_out += p;
        L_out += k + 2 * (p - 1);
    }
    if (n_out > INT32_MAX || C_out > INT32_MAX)
        return afs::set_last_error(AFS_EINVAL, "the decomposed instance has more than 2^31 - 1 variables or constraints");
    return AFS_OK;
}

}  // namespace

extern "C" {

afs_status afs_decompose_size(int32_t n, int32_t C, const int64_t *con_off, const int32_t *types, int32_t max_len,
                              int32_t *n_out, int32_t *C_out, int64_t *L_out)
{
    int64_t no, co, lo;
    const afs_status st = check_input(n, C, con_off, types, max_len, no, co, lo);
    if (st != AFS_OK) return st;
    if (n_out) *n_out = (int32_t)no;
    if (C_out) *C_out = (int32_t)co;
    if (L_out) *L_out = lo;
    return AFS_OK;
}

afs_status afs_decompose(int32_t n, int32_t C, const int64_t *con_off, const int32_t *lits, const int32_t *types,
                         const int32_t *params, const float *weights, int32_t max_len, int64_t *con_off_out,
                         int32_t *lits_out, int32_t *types_out, int32_t *params_out, float *weights_out,
                         int32_t *origin_out)
{
    int64_t no, co, lo;
    afs_status st = check_input(n, C, con_off, types, max_len, no, co, lo);
    if (st != AFS_OK) return st;
    if (C > 0 && (!lits || !params)) return afs::set_last_error(AFS_EINVAL, "lits or params is NULL");
    if (!con_off_out || (lo > 0 && !lits_out) || (co > 0 && (!types_out || !params_out || !origin_out)))
        return afs::set_last_error(AFS_EINVAL, "an output array is NULL");
    if (weights && co > 0 && !weights_out) return afs::set_last_error(AFS_EINVAL, "weights_out is NULL");
    const int64_t L = C > 0 ? con_off[C] : 0;
    for (int64_t i = 0; i < L; ++i)
        if (lits[i] == 0 || lits[i] == INT32_MIN || (lits[i] < 0 ? -lits[i] : lits[i]) > n)
            return afs::set_last_error(AFS_EINVAL, "literal " + std::to_string(lits[i]) + " out of range");

    int64_t out_c = 0, out_l = 0;
    int32_t next_aux = n;             // last variable number in use
    con_off_out[0] = 0;
    auto emit_piece = [&](int32_t c, int32_t type, int32_t param) {
        types_out[out_c] = type;
        params_out[out_c] = param;
        origin_out[out_c] = c;
        if (weights) weights_out[out_c] = weights[c];
        con_off_out[++out_c] = out_l;
    };
    for (int32_t c = 0; c < C; ++c) {
        const int64_t k = con_off[c + 1] - con_off[c];
        const int32_t *src = lits + con_off[c];
        const int64_t p = pieces(types[c], k, max_len);
        if (p == 1) {
            for (int64_t i = 0; i < k; ++i) lits_out[out_l++] = src[i];
            emit_piece(c, types[c], params[c]);
            continue;
        }
        const bool xr = types[c] == AFS_XOR;
        int64_t used = 0;             // literals of the constraint placed so far
        for (int64_t i = 0; i < p; ++i) {
            const int64_t len = piece_len(k, p, i);
            const int64_t own = len - (i > 0) - (i + 1 < p);
            if (i > 0) lits_out[out_l++] = xr ? next_aux : -next_aux;   // a_(i-1), made by the previous piece
            for (int64_t j = 0; j < own; ++j) lits_out[out_l++] = src[used + j];
            used += own;
            if (i + 1 < p) lits_out[out_l++] = ++next_aux;               // a_i
            const int32_t param = xr ? (i + 1 < p ? 0 : (params[c] & 1)) : params[c];
            emit_piece(c, types[c], param);
        }
    }
    return AFS_OK;
}

}  // extern "C"
