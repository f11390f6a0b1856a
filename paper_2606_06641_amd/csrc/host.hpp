// host.hpp -- host-side instance packing for the Accelerated Fourier SAT hot path.
//
// Pure C++17 (no HIP): validation, per-constraint truth tables, FP64 coefficient
// tables, length buckets and the variable -> literal-slot transpose.  The device
// layer uploads what is built here.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "afsat.h"

namespace afs {

// Largest constraint length the kernels handle.
constexpr int kMaxLen = AFS_MAX_LEN;
// Lengths up to this use one lane per restart with the whole constraint in registers.
constexpr int kShortMax = 16;
// Fewest and most literals one lane holds in the segment kernels (even counts).
constexpr int kMinSeg = 4;
constexpr int kMaxSeg = 32;
// Largest number of constraints per work tile.
constexpr int kMaxTile = 4096;

// One row of a coefficient table, consumed by the kernels as a float4.
//   row 0             : {d_0, d_half, 0, 0}  (d_half = d_{N/2} when N = k+1 is even, else 0)
//   rows of root m>=1 : 2 rows, see append_root_rows
struct TabRow {
    float x, y, z, w;
};

// Rescale period of a segment kernel with J lanes of S literals.
int rescale_period(int J, int S);

// Append the rows of each complex root m = 1..floor(k/2) of a table whose
// coefficient vector is (re, im) (length k+1), for the kernel shape (J, S) of k.
void append_root_rows(int k, int J, int S, const double *re, const double *im, std::vector<TabRow> &tab);

struct Bucket {
    int k_lo = 0, k_hi = 0;
    int J = 1;            // lanes per restart
    int S = 1;            // literals per lane (J == 1: S == k exactly)
    int32_t c0 = 0;       // first bucket-ordered constraint
    int32_t nc = 0;       // number of constraints
    int64_t slot0 = 0;    // first literal slot
    int64_t nslots = 0;
    int32_t tile = 1;     // constraints per work tile
    int32_t ntiles = 0;
    int32_t tile0 = 0;    // first global tile index (objective partial rows)
    int32_t rpl = 0;      // J == 1: restarts per lane asked for (0: the launch's default)
};

struct HostInstance {
    int32_t n = 0, C = 0;
    int64_t L = 0;
    int32_t max_k = 0;
    // input (original order)
    std::vector<int64_t> con_off;
    std::vector<int32_t> lits, types, params;
    std::vector<float> weights;
    // coefficient tables
    std::vector<TabRow> tab;
    int32_t n_tables = 0;
    // buckets and bucket-ordered constraints
    std::vector<Bucket> buckets;
    int32_t total_tiles = 0;
    std::vector<int32_t> bc_slot0, bc_k, bc_tab, bc_orig;
    std::vector<float> bc_w;
    // literal slots (bucket order)
    std::vector<int32_t> slot_lit;      // DIMACS literal stored in the slot
    std::vector<int32_t> slot_to_lit;   // input literal index of the slot
    // variable -> slot transpose (ascending slots per variable)
    std::vector<int32_t> voff;          // [n+1]
    std::vector<int32_t> vslot;         // [L]
    // sub-instances of a block-diagonal batch (one for a plain instance)
    int32_t n_inst = 1;
    std::vector<int32_t> inst_var0;     // [n_inst+1] first variable of each sub-instance
    std::vector<int32_t> con_inst;      // [C] sub-instance of each constraint (input order)
    std::vector<int32_t> var_inst;      // [n] sub-instance of each variable
};



// Truth predicate of a constraint with t true literals out of k (Table 1 and
// Table 2; CARD normalised to ">= K" or "< K" as in Appendix A).
// Returns 1 satisfied, 0 violated, -1 unknown type.
int satisfied(int type, int k, int param, int t);

// FP64 coefficient vector d_m, m = 0..k, of a constraint of length k (N = k+1):
// d_m = (1/N) sum_t g(t) omega^(-m t), g = -1 satisfied / +1 violated,
// omega = exp(2 pi i / N); angles use the index m*t mod N and roots j > N/2 are
// mirrored conjugates of N - j, so conjugate symmetry is exact.
void coefficients(int type, int k, int param, double *re, double *im);

// omega^j = c[j] + i s[j], omega = exp(2 pi i / N), j = 0..N-1; computed for
// j <= N/2 and mirrored as conjugates above, exact at the axis crossings.
void roots(int N, std::vector<long double> &c, std::vector<long double> &s);

// Packing choices (see afs_options in afsat.h).
struct PackOptions {
    std::vector<int> k_hi, lanes, seg;   // shape overrides for k > kShortMax, ascending k_hi
    std::vector<int> tile;               // per override entry (empty, or 0: tile_long / default)
    int tile_short = 0, tile_long = 0;   // 0: defaults
    int short_tile[kShortMax + 1] = {};  // per length k <= kShortMax (0: tile_short / default)
    int short_rpl[kShortMax + 1] = {};   // per length k <= kShortMax (0: the launch's default)
};

// Work-tile size and restarts per lane of the bucket that evaluates length k.
void bucket_tiling(int k, const PackOptions &o, int &tile, int &rpl);

// Validate options; returns an empty string or a message.
std::string check_options(const PackOptions &o);

// Build the packed instance.  Returns an empty string on success, else a message.
std::string build_instance(int32_t n, int32_t C, const int64_t *con_off, const int32_t *lits,
                           const int32_t *types, const int32_t *params, const float *weights,
                           const PackOptions &opts, HostInstance &out);

// Default bucket shape (J lanes per restart, S literals per lane) for a length k.
void bucket_shape(int k, int &J, int &S);

// Shape for a length k under the options (overrides, else the default).
void bucket_shape(int k, const PackOptions &o, int &J, int &S);

// One sub-instance of a batch, given by its own CSR arrays (variables 1..n).
struct PartRef {
    int32_t n = 0, C = 0;
    const int64_t *con_off = nullptr;
    const int32_t *lits = nullptr, *types = nullptr, *params = nullptr;
    const float *weights = nullptr;
};

// Block-diagonal batch: variables and constraints of the parts concatenated (the
// variables of part p are shifted by the variables of parts 0..p-1), packed as one
// instance, with the part of every constraint and variable recorded.
std::string build_batch(const std::vector<PartRef> &parts, const PackOptions &opts, HostInstance &out);

}  // namespace afs
