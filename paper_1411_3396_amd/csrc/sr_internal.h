// Internal declarations shared by the device kernels (sr_kernels.hip) and the
// host library (sr_api.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "sr.h"

namespace sr {

constexpr int kWave = 64;
constexpr int kTargetsPerItem = 64;  // one target per lane in a dense cell
constexpr int kSparseGroup = 16;     // default: most targets per item of a cell with fewer than 64
constexpr int kMinSparseGroup = 8;   // the smallest group size (sizes the item list)
constexpr int kXcds = 8;             // XCDs of an MI355X; workgroups are dealt to them in turn
constexpr int kQueues = kXcds;       // one work queue per XCD
constexpr int kQueueBlock = 32;      // consecutive items a queue takes from the list
constexpr int kClasses = 32;         // cost classes (floor log2 of the per-lane pair count)
constexpr int kRadixTile = 2048;     // elements per radix-sort tile
constexpr int kScanBlock = 2048;     // elements per scan block (256 threads x 8)
constexpr int kMomTile = 65536;      // rows per momentum partial
constexpr int kMaxLeafDepth = 4;     // deepest in-cell octree order

// Constants of the pair kernel, evaluated in t = s + eps^2:
//   f_SR = t^-3/2 - Q(t),  Q(t) = sum_k q[k] t^k = sum_k poly[k] (t - eps^2)^k,
//   2 f_SR' = -3 t^-5/2 - D(t),  D(t) = 2 Q'(t).
// The adjoint evaluates both at the scale -1/3, which saves it one product
// per pair (the factor -3 is applied once per output row):
//   f_SR / -3 = A(t) - t^-3/2 / 3,   A(t) = sum_k qa[k] t^k = Q(t) / 3,
//   2 f_SR' / -3 = t^-5/2 + B(t),    B(t) = sum_k dqa[k] t^k = D(t) / 3.
struct PairConsts {
    float eps2;   // eps * eps
    float tc2;    // r_s^2 + eps^2: pairs with t < tc2 interact
    float cull2;  // r_s^2 (1 + 1e-5): sources farther than this from the targets' box are skipped
    float q[6];
    float qa[6];
    float dqa[5];
    int32_t softened;  // eps > 0
};

// One problem of a batch (a single problem is a batch of one).
struct SegParams {
    float lo[3];
    float len[3];
    float h[3];       // len / nc
    float inv_h[3];   // nc / len
    float inv_len[3]; // 1 / len
    int32_t nc[3];
    int32_t periodic;
    int32_t cell_off;  // first global cell
    int32_t part_off;  // first particle (input row)
    int32_t n;
    int32_t n_active;
    int32_t out_off;   // first output row of its accelerations
    int32_t tile_off;  // first momentum partial
    PairConsts pc;
    int32_t leaf_depth;  // octree depth of the in-cell order (1 = octants)
    int32_t pad[1];
};
static_assert(sizeof(SegParams) % 16 == 0, "SegParams must stay 16-byte sized");

// Workspace header words (uint32 offsets into the header block).
enum HdrWord : int {
    kHdrFlags = 0,
    kHdrNItems = 1,
    kHdrMagic = 2,          // written by the last binning kernel: bins are ready
    kHdrMassInfo = 3,       // 0 if every mass equals the first one
    kHdrBucketCount = 64,   // [32]
    kHdrBucketBase = 128,   // [33]
    kHdrBucketCursor = 192, // [32]
    kHdrQueue = 256,        // queue q at kHdrQueue + 32*q (separate 128-byte lines)
    kHdrPairs = 512,        // int64 pair counter (2 words)
    kHdrSymTotal = 516,     // int64 partial slots the symmetric tiles need (2 words)
    kHdrSymOk = 518,        // 1: symmetric tiles run (their partial slots fit the pool)
    kHdrSymNItems = 519,    // symmetric work items
    kHdrSymWork = 520,      // int64 tile steps of all symmetric items (2 words)
    kHdrSymMaxItem = 522,   // tile steps of the longest symmetric item
    kHdrSymBucketCount = 544,   // [32]
    kHdrSymBucketBase = 576,    // [33]
    kHdrSymBucketCursor = 640,  // [32]
    kHdrSymQueue = 768,     // symmetric queue q at kHdrSymQueue + 32*q
    kHdrWords = 1024
};

// Symmetric (Newton's third law) tiles of the dense cells: every unordered
// pair of two dense particles is evaluated once, its two opposite terms kept
// as partial sums in fixed slots and added up in a fixed order afterwards.
constexpr int kSymDirs = 14;        // the cell itself and the 13 directions of the upper half stencil
constexpr int kSymNdDirs = 27;      // all 27 directions: non-dense sources of a dense block
constexpr int kSymSegs = kSymDirs + kSymNdDirs;  // source segments of a symmetric item
// per cell: target slots, then source slots of its dense particles for the 14
// directions, then source slots of its non-dense particles for the 27
constexpr int kSymStride = 1 + kSymDirs + kSymNdDirs;
constexpr int kSymSlotsPerParticle = 16;  // partial-slot pool: this many 12-byte slots per particle

// Byte offsets of every buffer inside a workspace.
struct Layout {
    int64_t N = 0;     // particles (all segments)
    int64_t NC = 0;    // cells (all segments)
    int32_t B = 1;     // segments
    int32_t passes = 0, digit_bits = 0;
    int32_t code_bits = 3;  // leaf-code bits of the sort key: 3 per octree level
    int32_t key_bits = 3;   // low bits of the sort key below the cell: (passive flag +) leaf code
    int64_t ntiles = 0;     // radix tiles
    int64_t table = 0;      // radix table entries (R * ntiles)
    int64_t item_cap = 0;   // upper bound on work items
    int64_t mom_tiles = 0;  // momentum partials
    size_t hdr = 0, seg = 0, cell_of = 0, skey = 0, packed = 0, keys[2] = {0, 0}, vals[2] = {0, 0};
    size_t tab = 0, tabx = 0, nact = 0, start = 0, scan_tmp = 0;
    size_t bx = 0, by = 0, bz = 0, bm = 0, out_row = 0, gx = 0, gy = 0, gz = 0;
    size_t items = 0, info = 0, mom = 0;
    int64_t sym_cap = 0;    // partial slots of the pool
    int64_t sym_item_cap = 0;
    size_t sym_pref = 0, sym_tot = 0, sym_base = 0, sym_info = 0, sym_items = 0, sym_pool = 0;
    size_t total = 0;
    size_t perm() const { return vals[(passes - 1) & 1]; }
    size_t sorted_keys() const { return keys[(passes - 1) & 1]; }
    // Tag of a binned workspace for these sizes (never zero).
    uint32_t magic() const
    {
        uint32_t m = 0x9E3779B9u * (uint32_t)N ^ 0x85EBCA6Bu * (uint32_t)NC ^ 0xC2B2AE35u * (uint32_t)B ^
                     0x27D4EB2Fu * (uint32_t)key_bits ^ 0x165667B1u * (uint32_t)code_bits;
        return m ? m : 1u;
    }
};

// Sizes of the scan scratch for an array of m elements.
int64_t scan_scratch_elems(int64_t m);

// Device-path entry points implemented in sr_kernels.hip.  All enqueue on
// `st` and return hipSuccess or the first launch error.
struct DevArgs {
    char *ws;
    const Layout *L;
    const SegParams *seg_host;  // single segment: by value in kernel args
    const SegParams *seg_dev;   // batch: device table (nullptr for single)
    hipStream_t st;
    int waves_per_cu;
    int num_cu;
    int n_rows;  // rows of the force output (sum of n_active)
    int targets_per_lane;  // 1 or 2 for cells with more than 64 targets
    int occupancy;         // register-allocation hint of the pair kernels: 0, 6 or 8 waves/SIMD
    int sym_blocks;        // symmetric tiles: blocks of 64 targets per item (0: symmetric tiles off)
    int sym_window;        // symmetric tiles: sources per item window (256 or 512)
    int sym_rounds;        // symmetric tiles: consecutive windows per item (1 or 2)
    int sym_occupancy;     // symmetric tiles: register-allocation hint, 0 or 5 waves/SIMD
    double sym_balance;    // symmetric tiles run only if their steps per wave reach this many longest items
    int sparse_group;      // most targets per item of a cell (or remainder) with fewer than 64: 8, 16, 32 or 64
    int64_t pull_limit;    // most items one wave of a persistent kernel may pull (test hook)
};

hipError_t dev_bin(const DevArgs &a, const float *pos, const float *mass);
hipError_t dev_force(const DevArgs &a, float *acc);
hipError_t dev_vjp(const DevArgs &a, const float *g, float *grad);
hipError_t dev_count_pairs(const DevArgs &a, bool adjoint, int64_t *pairs);
hipError_t dev_zero(void *p, int64_t words, hipStream_t st);

// Shared building blocks (sr_kernels.hip) for other device passes.
struct RadixBufs {
    int *keys[2];
    int *vals[2];
    int *tab;       // digit table, (1 << digit_bits) * ntiles entries
    int *tabx;      // its exclusive scan, one more entry
    int *scan_tmp;  // scan_scratch_elems(table) entries
};
hipError_t radix_sort_pairs(const int *keys_in, const int *vals_in, int64_t n, int passes,
                            int digit_bits, int64_t ntiles, const RadixBufs &b, hipStream_t st);
hipError_t dev_scan(const int *in, int *out, int64_t m, int *tmp, hipStream_t st);
hipError_t dev_bounds(const int *sorted_keys, int64_t n, int64_t nk, int key_bits, int *start,
                      hipStream_t st);
hipError_t dev_momentum(const DevArgs &a, const float *acc, const float *mass, double *out);
// Device address and size of the fixed workspace of sr_force_static on the
// current device (looked up on the first call per device).
hipError_t static_workspace(void **ptr, size_t *bytes);

// Event timing hooks (sr_api.cpp).
void timing_begin(const char *name, hipStream_t st, void **token);
void timing_end(void *token, hipStream_t st);

}  // namespace sr
