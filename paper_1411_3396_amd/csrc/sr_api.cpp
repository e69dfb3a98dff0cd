// Host side of the short-range force library: argument validation, workspace
// layout, pair-kernel constants, batch plans (graph capture and replay),
// launch-parameter tuning and event timing.  The ABI is declared in sr.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "sr_internal.h"

using namespace sr;

namespace {

constexpr int64_t kMaxParticles = (int64_t(1) << 31) - 1;
constexpr int64_t kSymMaxSlots = (int64_t(1) << 31) - 1;  // partial slots are indexed in int32
constexpr int64_t kMaxCells = int64_t(1) << 26;  // cell << 4 fits the 31-bit sort key at depth 1

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool finitef(float x) { return std::isfinite(x); }

// Cells per dimension: floor(len / r_s) in float32 (>= 1; periodic >= 3).
sr_status grid_of(const sr_problem *p, int32_t nc[3])
{
    if (!p) return SR_E_ARG;
    if (!(p->r_s > 0.0f) || !finitef(p->r_s)) return SR_E_ARG;
    if (!(p->eps >= 0.0f) || !finitef(p->eps)) return SR_E_ARG;
    if (p->periodic != 0 && p->periodic != 1) return SR_E_ARG;
    if (p->leaf_depth < 0 || p->leaf_depth > kMaxLeafDepth) return SR_E_ARG;
    for (int k = 0; k < 6; ++k)
        if (!finitef(p->poly[k])) return SR_E_ARG;
    int64_t ncell = 1;
    for (int d = 0; d < 3; ++d) {
        if (!(p->len[d] > 0.0f) || !finitef(p->len[d]) || !finitef(p->lo[d])) return SR_E_ARG;
        if (p->periodic && p->lo[d] != 0.0f) return SR_E_ARG;
        const float q = std::floor(p->len[d] / p->r_s);
        if (!(q < 1.0e9f)) return SR_E_ARG;
        int v = (int)q;
        if (p->periodic) {
            if (v < 3) return SR_E_ARG;  // minimum image needs len >= 3 r_s here
        } else if (v < 1) {
            v = 1;
        }
        nc[d] = v;
        ncell *= v;
        if (ncell > kMaxCells) return SR_E_UNSUPPORTED;
    }
    const float tc2 = p->r_s * p->r_s + p->eps * p->eps;
    if (!finitef(tc2)) return SR_E_ARG;
    return SR_OK;
}

PairConsts pair_consts(const sr_problem *p)
{
    PairConsts pc{};
    pc.eps2 = p->eps * p->eps;
    const float rs2 = p->r_s * p->r_s;
    pc.tc2 = rs2 + pc.eps2;
    pc.cull2 = (float)((double)rs2 * (1.0 + 1e-5));
    pc.softened = p->eps > 0.0f ? 1 : 0;
    // Q(t) = P(t - e2): expand each c_k (t - e2)^k by the binomial theorem in double.
    const double e2 = (double)pc.eps2;
    double Q[6] = {0, 0, 0, 0, 0, 0};
    for (int k = 0; k < 6; ++k) {
        double binom = 1.0;  // C(k, m)
        for (int m = 0; m <= k; ++m) {
            if (m > 0) binom = binom * (k - m + 1) / m;
            Q[m] += (double)p->poly[k] * binom * std::pow(-e2, k - m);
        }
    }
    for (int m = 0; m < 6; ++m) pc.q[m] = (float)Q[m];
    for (int m = 0; m < 6; ++m) pc.qa[m] = (float)(Q[m] / 3.0);
    for (int m = 0; m < 5; ++m) pc.dqa[m] = (float)(2.0 * (m + 1) * Q[m + 1] / 3.0);
    return pc;
}

int leaf_depth_of(const sr_problem *p) { return p->leaf_depth > 0 ? p->leaf_depth : 1; }

// The sort key (cell << key_bits | passive << code_bits | code) must stay a
// non-negative int32.
bool key_fits(int64_t NC, int code_bits, bool any_passive)
{
    const int key_bits = code_bits + (any_passive ? 1 : 0);
    return NC <= ((int64_t(1) << 31) - 1) >> key_bits;
}

SegParams seg_of(const sr_problem *p, const int32_t nc[3])
{
    SegParams s{};
    for (int d = 0; d < 3; ++d) {
        s.lo[d] = p->lo[d];
        s.len[d] = p->len[d];
        s.h[d] = p->len[d] / (float)nc[d];
        s.inv_h[d] = (float)nc[d] / p->len[d];
        s.inv_len[d] = 1.0f / p->len[d];
        s.nc[d] = nc[d];
    }
    s.periodic = p->periodic;
    s.pc = pair_consts(p);
    s.leaf_depth = leaf_depth_of(p);
    return s;
}

// Bytes of a tail holding `cap` partial slots and the items they allow (an
// item writes at least 64 target slots).
size_t sym_tail_bytes(int64_t cap)
{
    return align256((size_t)(cap / kWave + 1) * 16) + align256((size_t)cap * 12);
}

// Lays the symmetric items and the pool over the workspace tail from
// L.sym_items to ws_bytes: the most slots that fit (at most 2^31 - 1).
void sym_tail(Layout &L, size_t ws_bytes)
{
    const size_t tail = ws_bytes > L.sym_items ? ws_bytes - L.sym_items : 0;
    int64_t cap = (int64_t)std::min<size_t>(tail > 512 ? (tail - 512) / 784 * 64 : 0, (size_t)kSymMaxSlots);
    while (cap > 0 && sym_tail_bytes(cap) > tail) cap -= 1 + cap / 256;
    if (cap < 0) cap = 0;
    L.sym_cap = cap;
    L.sym_item_cap = cap / kWave + 1;
    L.sym_pool = L.sym_items + align256((size_t)L.sym_item_cap * 16);
}

Layout make_layout(int64_t N, int64_t NC, int B, int64_t mom_tiles, bool any_passive, int code_bits)
{
    Layout L;
    L.N = N;
    L.NC = NC;
    L.B = B;
    L.code_bits = code_bits;
    L.key_bits = code_bits + (any_passive ? 1 : 0);
    int bits = 1;
    while ((int64_t(1) << bits) < (NC << L.key_bits)) ++bits;
    L.passes = (bits + 7) / 8;
    L.digit_bits = (bits + L.passes - 1) / L.passes;
    L.ntiles = std::max<int64_t>(1, (N + kRadixTile - 1) / kRadixTile);
    L.table = (int64_t(1) << L.digit_bits) * L.ntiles;
    // a run of n targets makes at most ceil(n / kSparseGroup) items, and a
    // cell has up to two runs (active targets; passive ones in the adjoint)
    L.item_cap = 2 * NC + (N + kMinSparseGroup - 1) / kMinSparseGroup + 1;
    L.mom_tiles = mom_tiles;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align256(o + std::max<size_t>(bytes, 1));
        return at;
    };
    const size_t n4 = (size_t)N * 4;
    L.hdr = take(kHdrWords * 4);
    L.seg = take((size_t)B * sizeof(SegParams));
    L.cell_of = take(n4);
    L.skey = take(n4);
    L.packed = take((size_t)N * 16);  // offsets from the cell centre + mass, input order
    L.keys[0] = take(n4);
    L.keys[1] = take(n4);
    L.vals[0] = take(n4);
    L.vals[1] = take(n4);
    L.tab = take((size_t)L.table * 4);
    L.tabx = take((size_t)(L.table + 1) * 4);
    L.nact = take((size_t)NC * 4);
    L.start = take((size_t)(NC + 1) * 4);
    L.scan_tmp = take((size_t)std::max(scan_scratch_elems(L.table), scan_scratch_elems(NC)) * 4);
    L.bx = take(n4);
    L.by = take(n4);
    L.bz = take(n4);
    L.bm = take(n4);
    L.out_row = take(n4);
    L.gx = take(n4);
    L.gy = take(n4);
    L.gz = take(n4);
    L.items = take((size_t)L.item_cap * 16);
    L.info = take((size_t)NC * 4);
    L.mom = take((size_t)(3 * mom_tiles + 3) * 8);
    // symmetric tiles: per cell and slot group the prefix of the partial-slot
    // counts, per cell their total and its exclusive scan, per cell the item
    // count and cost class, the items, and the pool of 12-byte partial slots
    // (at most 2^31 - 1 of them)
    L.sym_pref = take((size_t)kSymStride * NC * 4);
    L.sym_tot = take((size_t)NC * 4);
    L.sym_base = take(((size_t)NC + 1) * 4);
    L.sym_info = take((size_t)NC * 4);
    // the tail: symmetric items and the pool, sized for the default number of
    // slots per particle; a larger workspace lends the tail more (sym_tail)
    const int64_t cap = std::min<int64_t>((int64_t)kSymSlotsPerParticle * N, kSymMaxSlots);
    L.sym_items = o;
    L.total = o + sym_tail_bytes(cap);
    sym_tail(L, L.total);
    return L;
}


int64_t mom_tiles_of(int64_t rows) { return (rows + kMomTile - 1) / kMomTile; }

struct Single {
    int32_t nc[3];
    int64_t NC;
    SegParams seg;
    Layout L;
};

sr_status prepare_single(int64_t n, int64_t n_active, const sr_problem *p, Single &s)
{
    if (!p || n < 0 || n > kMaxParticles || n_active < 0 || n_active > n) return SR_E_ARG;
    sr_status st = grid_of(p, s.nc);
    if (st != SR_OK) return st;
    s.NC = (int64_t)s.nc[0] * s.nc[1] * s.nc[2];
    s.seg = seg_of(p, s.nc);
    s.seg.n = (int32_t)n;
    s.seg.n_active = (int32_t)n_active;
    const int code_bits = 3 * s.seg.leaf_depth;
    if (!key_fits(s.NC, code_bits, n_active < n)) return SR_E_UNSUPPORTED;
    s.L = make_layout(n, s.NC, 1, mom_tiles_of(n), n_active < n, code_bits);
    return SR_OK;
}

sr_status check_ws(const void *ws, size_t ws_bytes, const Layout &L)
{
    if (!ws) return SR_E_WORKSPACE;
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return SR_E_WORKSPACE;
    if (ws_bytes < L.total) return SR_E_WORKSPACE;
    return SR_OK;
}

// Launch parameters of the single-problem pair kernels, per kernel: [0] the
// forward kernel (and the pair count), [1] the adjoint.  Defaults are the
// fastest settings measured on the node-share workload.
constexpr int kCfgForce = 0, kCfgVjp = 1;
std::atomic<int> g_waves_default[2] = {{32}, {24}};
std::atomic<int> g_tpl_default[2] = {{1}, {2}};
std::atomic<int> g_occ_default[2] = {{6}, {0}};
// Symmetric tiles of the dense cells, per kernel: blocks of 64 targets per
// item (0: off) and sources per window (256 or 512).
std::atomic<int> g_sym_blocks[2] = {{16}, {16}};
std::atomic<int> g_sym_window[2] = {{256}, {256}};
std::atomic<int> g_sym_occ[2] = {{5}, {5}};
// Consecutive windows per symmetric item: an item sums its blocks' targets
// over both windows into one partial slot, halving the target slots the
// gather reads and the per-block set-up (boxes, target loads) per window.
std::atomic<int> g_sym_rounds[2] = {{2}, {2}};
std::atomic<double> g_sym_balance{1.0};
std::atomic<int> g_sparse_group{kSparseGroup};

// Launch defaults may be overridden for experiments (both kernels):
// SR_WAVES_PER_CU, SR_TARGETS_PER_LANE, SR_OCCUPANCY.
struct EnvDefaults {
    EnvDefaults()
    {
        for (int k = 0; k < 2; ++k) {
            if (const char *v = std::getenv("SR_WAVES_PER_CU")) {
                const int w = std::atoi(v);
                if (w >= 1 && w <= 64) g_waves_default[k] = w;
            }
            if (const char *v = std::getenv("SR_TARGETS_PER_LANE")) {
                const int t = std::atoi(v);
                if (t == 1 || t == 2) g_tpl_default[k] = t;
            }
            if (const char *v = std::getenv("SR_OCCUPANCY")) {
                const int o = std::atoi(v);
                if (o == 0 || o == 6 || o == 8) g_occ_default[k] = o;
            }
            if (const char *v = std::getenv("SR_SYM_BLOCKS")) {
                const int b = std::atoi(v);
                if (b >= 0 && b <= 256) g_sym_blocks[k] = b;
            }
            if (const char *v = std::getenv("SR_SYM_WINDOW")) {
                const int w = std::atoi(v);
                if (w == 256 || w == 512) g_sym_window[k] = w;
            }
            if (const char *v = std::getenv("SR_SYM_ROUNDS")) {
                const int r = std::atoi(v);
                if (r == 1 || r == 2) g_sym_rounds[k] = r;
            }
            if (const char *v = std::getenv("SR_SYM_OCC")) {
                const int o = std::atoi(v);
                if (o == 0 || o == 5 || o == 6) g_sym_occ[k] = o;
            }
        }
        if (const char *v = std::getenv("SR_SPARSE_GROUP")) {
            const int gsz = std::atoi(v);
            if (gsz == 8 || gsz == 16 || gsz == 32 || gsz == 64) g_sparse_group = gsz;
        }
        if (const char *v = std::getenv("SR_SYM_BALANCE")) {
            const double b = std::atof(v);
            if (b >= 0.0 && std::isfinite(b)) g_sym_balance = b;
        }
    }
} g_env_defaults;

// Most items one wave of a persistent kernel may pull.  The kernels bound
// their loops by the item count themselves; SR_PULL_LIMIT (read on every
// call) lowers the bound so that a test can make every wave stop early and
// check that the workspace is flagged and the kernel still exits.
int64_t pull_limit()
{
    if (const char *v = std::getenv("SR_PULL_LIMIT")) {
        const long long q = std::atoll(v);
        if (q >= 0) return (int64_t)q;
    }
    return INT64_MAX;
}

sr_status device_args(DevArgs &a, void *ws, const Layout *L, const SegParams *seg_host,
                      const SegParams *seg_dev, void *stream, int waves_per_cu, int64_t n_rows,
                      int cfg = kCfgForce)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SR_E_DEVICE;
    static std::mutex mu;
    static std::vector<int> cu_cache;
    int cus = 0;
    {
        std::lock_guard<std::mutex> lk(mu);
        if ((int)cu_cache.size() <= dev) cu_cache.resize(dev + 1, 0);
        if (cu_cache[dev] == 0) {
            if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
                return SR_E_DEVICE;
            cu_cache[dev] = cus;
        }
        cus = cu_cache[dev];
    }
    a.ws = static_cast<char *>(ws);
    a.L = L;
    a.seg_host = seg_host;
    a.seg_dev = seg_dev;
    a.st = static_cast<hipStream_t>(stream);
    a.waves_per_cu = waves_per_cu > 0 ? waves_per_cu : g_waves_default[cfg].load();
    a.num_cu = cus;
    a.n_rows = (int)n_rows;
    a.targets_per_lane = g_tpl_default[cfg].load();
    a.occupancy = g_occ_default[cfg].load();
    a.sym_blocks = g_sym_blocks[cfg].load();
    a.sym_window = g_sym_window[cfg].load();
    a.sym_rounds = g_sym_rounds[cfg].load();
    a.sym_occupancy = g_sym_occ[cfg].load();
    a.sym_balance = g_sym_balance.load();
    a.sparse_group = g_sparse_group.load();
    a.pull_limit = pull_limit();
    return SR_OK;
}

sr_status hip_status(hipError_t e) { return e == hipSuccess ? SR_OK : SR_E_DEVICE; }

// ------------------------------------------------------------ event timing

struct TimingRec {
    std::string name;
    hipEvent_t a = nullptr, b = nullptr;
};
std::mutex g_tmu;
bool g_timing = false;
std::vector<TimingRec> g_recs;

}  // namespace

namespace sr {

void timing_begin(const char *name, hipStream_t st, void **token)
{
    *token = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_tmu);
        if (!g_timing) return;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    auto *r = new TimingRec;
    r->name = name;
    if (hipEventCreate(&r->a) != hipSuccess || hipEventCreate(&r->b) != hipSuccess ||
        hipEventRecord(r->a, st) != hipSuccess) {
        delete r;
        return;
    }
    *token = r;
}

void timing_end(void *token, hipStream_t st)
{
    if (!token) return;
    auto *r = static_cast<TimingRec *>(token);
    (void)hipEventRecord(r->b, st);
    std::lock_guard<std::mutex> lk(g_tmu);
    g_recs.push_back(*r);
    delete r;
}

}  // namespace sr

// ------------------------------------------------------------------ batch plan

struct sr_batch_plan {
    int32_t B = 0;
    std::vector<int64_t> offsets, n_active;
    std::vector<sr_problem> probs;
    std::vector<SegParams> segs;        // batched layout
    std::vector<Single> singles;        // per-subvolume reference mode
    SegParams summary{};                // softened = all subvolumes softened
    Layout L;
    size_t ws_bytes = 0;
    int64_t total_active = 0;
    SegParams *pinned = nullptr;        // upload source of the segment table
    hipStream_t cap = nullptr;          // capture stream
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void *b_pos = nullptr, *b_mass = nullptr, *b_ws = nullptr, *b_acc = nullptr,
               *b_mom = nullptr;
    int waves_per_cu = 0;               // 0: not tuned yet
    int targets_per_lane = 1;
    int occupancy = 0;
    int sym_blocks = -1;                // symmetric tiles (-1: the forward kernel's current setting)
    int sym_window = -1;
    int sparse_group = -1;              // targets per item of sparse cells (-1: the process-wide value)
    std::string tune_cache;
    std::string tune_key;
    double tuned_ms = -1.0;
};

namespace {

sr_status run_batched(sr_batch_plan *P, const float *pos, const float *mass, void *ws, float *acc,
                      double *mom, hipStream_t st)
{
    DevArgs a;
    sr_status s = device_args(a, ws, &P->L, &P->summary, reinterpret_cast<SegParams *>(
                                  static_cast<char *>(ws) + P->L.seg), st, P->waves_per_cu,
                                  P->total_active);
    if (s != SR_OK) return s;
    a.targets_per_lane = P->targets_per_lane;
    a.occupancy = P->occupancy;
    if (P->sym_blocks >= 0) a.sym_blocks = P->sym_blocks;
    if (P->sym_window > 0) a.sym_window = P->sym_window;
    if (P->sparse_group > 0) a.sparse_group = P->sparse_group;
    // the plan's tuner already timed the tiles against none, and the same
    // decision must hold in every mode (bitwise agreement): no balance rule
    a.sym_balance = 0.0;
    // one window per item: the tuner's tile choices were timed that way, and
    // a plan's many small problems gain little from fewer target slots
    a.sym_rounds = 1;
    hipError_t e = hipMemcpyAsync(static_cast<char *>(ws) + P->L.seg, P->pinned,
                                  sizeof(SegParams) * P->B, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return SR_E_DEVICE;
    if ((e = dev_bin(a, pos, mass)) != hipSuccess) return SR_E_DEVICE;
    if (P->total_active > 0 && (e = dev_force(a, acc)) != hipSuccess) return SR_E_DEVICE;
    if (mom && (e = dev_momentum(a, acc, mass, mom)) != hipSuccess) return SR_E_DEVICE;
    return SR_OK;
}

sr_status run_per_subvolume(sr_batch_plan *P, const float *pos, const float *mass, void *ws,
                            float *acc, double *mom, hipStream_t st)
{
    int64_t out_off = 0;
    for (int b = 0; b < P->B; ++b) {
        Single &S = P->singles[b];
        const int64_t off = P->offsets[b];
        const int64_t n = P->offsets[b + 1] - off;
        DevArgs a;
        sr_status s = device_args(a, ws, &S.L, &S.seg, nullptr, st, P->waves_per_cu, P->n_active[b]);
        if (s != SR_OK) return s;
        a.targets_per_lane = P->targets_per_lane;
        a.occupancy = P->occupancy;
        if (P->sym_blocks >= 0) a.sym_blocks = P->sym_blocks;
        if (P->sym_window > 0) a.sym_window = P->sym_window;
        if (P->sparse_group > 0) a.sparse_group = P->sparse_group;
        a.sym_balance = 0.0;
        a.sym_rounds = 1;
        if (n > 0) {
            if (dev_bin(a, pos + 3 * off, mass + off) != hipSuccess) return SR_E_DEVICE;
            if (P->n_active[b] > 0 && dev_force(a, acc + 3 * out_off) != hipSuccess) return SR_E_DEVICE;
        }
        if (mom) {
            // momentum of this subvolume, scratch at the end of the workspace
            Single M;
            M.seg = S.seg;
            M.seg.n_active = (int32_t)P->n_active[b];
            M.L = Layout{};
            M.L.B = 1;
            M.L.mom_tiles = mom_tiles_of(P->n_active[b]);
            const size_t need = align256((size_t)(3 * M.L.mom_tiles + 3) * 8);
            M.L.mom = (P->ws_bytes - need) & ~size_t(255);
            DevArgs am;
            if ((s = device_args(am, ws, &M.L, &M.seg, nullptr, st, P->waves_per_cu, P->n_active[b])) !=
                SR_OK)
                return s;
            if (dev_momentum(am, acc + 3 * out_off, mass + off, mom + 3 * b) != hipSuccess)
                return SR_E_DEVICE;
        }
        out_off += P->n_active[b];
    }
    return SR_OK;
}

std::string arch_name()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return "unknown";
    return std::string(prop.gcnArchName);
}

// Minimal reader of the tune cache: one line per key, "key waves".
bool cache_lookup(const std::string &path, const std::string &key, int &waves, int &tpl, int &occ,
                  int &sym_blocks, int &sym_window, int &group)
{
    if (path.empty()) return false;
    std::ifstream in(path);
    if (!in) return false;
    std::string line;
    while (std::getline(in, line)) {
        // entries look like:  "key": {"waves_per_cu": 16, "ms": 1.25},
        const size_t q0 = line.find('"');
        if (q0 == std::string::npos) continue;
        const size_t q1 = line.find('"', q0 + 1);
        if (q1 == std::string::npos || line.substr(q0 + 1, q1 - q0 - 1) != key) continue;
        const size_t w = line.find("\"waves_per_cu\":", q1);
        if (w == std::string::npos) continue;
        const int v = std::atoi(line.c_str() + w + 15);
        const size_t t = line.find("\"targets_per_lane\":", q1);
        const int tv = t == std::string::npos ? 1 : std::atoi(line.c_str() + t + 19);
        const size_t o = line.find("\"occupancy\":", q1);
        const int ov = o == std::string::npos ? 0 : std::atoi(line.c_str() + o + 12);
        const size_t sb = line.find("\"sym_blocks\":", q1);
        const int sbv = sb == std::string::npos ? -1 : std::atoi(line.c_str() + sb + 13);
        const size_t sw = line.find("\"sym_window\":", q1);
        const int swv = sw == std::string::npos ? -1 : std::atoi(line.c_str() + sw + 13);
        const size_t sg = line.find("\"sparse_group\":", q1);
        const int sgv = sg == std::string::npos ? -1 : std::atoi(line.c_str() + sg + 15);
        if (v >= 1 && v <= 64 && (tv == 1 || tv == 2) && (ov == 0 || ov == 6 || ov == 8) && sbv >= -1 &&
            sbv <= 256 && (swv == -1 || swv == 256 || swv == 512) &&
            (sgv == -1 || sgv == 8 || sgv == 16 || sgv == 32 || sgv == 64)) {
            waves = v;
            tpl = tv;
            occ = ov;
            sym_blocks = sbv;
            sym_window = swv;
            group = sgv;
            return true;
        }
    }
    return false;
}

void cache_store(const std::string &path, const std::string &key, int waves, int tpl, int occ,
                 int sym_blocks, int sym_window, int group, double ms)
{
    if (path.empty()) return;
    std::vector<std::string> keep;
    {
        std::ifstream in(path);
        std::string line;
        while (in && std::getline(in, line)) {
            const size_t q0 = line.find('"');
            if (q0 == std::string::npos) continue;
            const size_t q1 = line.find('"', q0 + 1);
            if (q1 == std::string::npos) continue;
            if (line.find("\"waves_per_cu\":") == std::string::npos) continue;
            if (line.substr(q0 + 1, q1 - q0 - 1) == key) continue;
            std::string l = line;
            while (!l.empty() && (l.back() == ',' || l.back() == ' ')) l.pop_back();
            keep.push_back(l);
        }
    }
    std::ostringstream e;
    e << "  \"" << key << "\": {\"waves_per_cu\": " << waves << ", \"targets_per_lane\": " << tpl
      << ", \"occupancy\": " << occ << ", \"sym_blocks\": " << sym_blocks << ", \"sym_window\": "
      << sym_window << ", \"sparse_group\": " << group << ", \"ms\": " << ms << "}";
    keep.push_back(e.str());
    const std::string tmp = path + ".tmp";
    {
        std::ofstream out(tmp);
        if (!out) return;
        out << "{\n";
        for (size_t i = 0; i < keep.size(); ++i) out << keep[i] << (i + 1 < keep.size() ? ",\n" : "\n");
        out << "}\n";
    }
    std::rename(tmp.c_str(), path.c_str());
}

// Pick the launch parameters (persistent grid in waves per CU, targets per
// lane of dense items, register-allocation variant) by timing the batched
// sequence, then the tiles of the symmetric kernel (blocks per item, window,
// or off), then the targets per item of sparse cells, each stage with the
// choices before it.  Launch parameters do not change results; the tiles and
// the sparse groups change only the order of the float32 sums (and so the
// last bits), and are fixed once the plan is tuned.
sr_status tune(sr_batch_plan *P, const float *pos, const float *mass, void *ws, float *acc,
               hipStream_t st)
{
    int waves = 0, tpl = 1, occ = 0, sb = -1, sw = -1, sg = -1;
    if (cache_lookup(P->tune_cache, P->tune_key, waves, tpl, occ, sb, sw, sg)) {
        P->waves_per_cu = waves;
        P->targets_per_lane = tpl;
        P->occupancy = occ;
        P->sym_blocks = sb;
        P->sym_window = sw;
        P->sparse_group = sg;
        return SR_OK;
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return SR_E_DEVICE;
    // two timed runs after a warm one
    auto time_runs = [&](double &ms_out) -> sr_status {
        sr_status s = run_batched(P, pos, mass, ws, acc, nullptr, st);
        if (s != SR_OK) return s;
        float ms = 0.f;
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < 2; ++r) {
            s = run_batched(P, pos, mass, ws, acc, nullptr, st);
            if (s != SR_OK) return s;
        }
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess) return SR_E_DEVICE;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ms_out = ms;
        return SR_OK;
    };
    struct Cand {
        int w, t, o;
    };
    const Cand cand[] = {{16, 1, 0}, {32, 1, 0}, {16, 2, 0}, {32, 2, 0}, {24, 1, 6},
                         {32, 1, 6}, {24, 2, 6}, {32, 2, 6}, {32, 1, 8}, {32, 2, 8}};
    double best = 1e300;
    Cand pick{g_waves_default[kCfgForce].load(), 1, 0};
    P->sym_blocks = -1;
    P->sym_window = -1;
    P->sparse_group = -1;
    for (const Cand &c : cand) {
        P->waves_per_cu = c.w;
        P->targets_per_lane = c.t;
        P->occupancy = c.o;
        double ms = 0;
        const sr_status s = time_runs(ms);
        if (s != SR_OK) return s;
        if (ms < best) {
            best = ms;
            pick = c;
        }
    }
    P->waves_per_cu = pick.w;
    P->targets_per_lane = pick.t;
    P->occupancy = pick.o;
    struct Tile {
        int k, w;
    };
    const Tile tiles[] = {{16, 512}, {16, 256}, {64, 512}, {4, 512}, {0, 512}};
    Tile tpick{-1, -1};
    double best_t = 1e300;
    for (const Tile &t : tiles) {
        P->sym_blocks = t.k;
        P->sym_window = t.w;
        double ms = 0;
        const sr_status s = time_runs(ms);
        if (s != SR_OK) return s;
        if (ms < best_t) {
            best_t = ms;
            tpick = t;
        }
    }
    P->sym_blocks = tpick.k;
    P->sym_window = tpick.w;
    const int groups[] = {16, 32, 8};
    int gpick = kSparseGroup;
    double best_g = 1e300;
    for (const int gsz : groups) {
        P->sparse_group = gsz;
        double ms = 0;
        const sr_status s = time_runs(ms);
        if (s != SR_OK) return s;
        if (ms < best_g) {
            best_g = ms;
            gpick = gsz;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    P->sparse_group = gpick;
    P->tuned_ms = std::min(best, std::min(best_t, best_g)) / 2.0;
    cache_store(P->tune_cache, P->tune_key, pick.w, pick.t, pick.o, tpick.k, tpick.w, gpick, P->tuned_ms);
    return SR_OK;
}

void drop_graph(sr_batch_plan *P)
{
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    P->exec = nullptr;
    P->graph = nullptr;
}

}  // namespace

// ------------------------------------------------------------------ the ABI

extern "C" {

int sr_abi_version(void) { return SR_ABI_VERSION; }

const char *sr_status_str(int s)
{
    switch (s) {
    case SR_OK: return "ok";
    case SR_E_ARG: return "invalid argument";
    case SR_E_WORKSPACE: return "workspace missing, misaligned or too small";
    case SR_E_DEVICE: return "HIP runtime error";
    case SR_E_PLAN: return "invalid batch plan";
    case SR_E_UNSUPPORTED: return "unsupported size";
    default: return "unknown status";
    }
}

sr_status sr_grid(const sr_problem *prob, int32_t nc[3])
{
    if (!nc) return SR_E_ARG;
    return grid_of(prob, nc);
}

sr_status sr_workspace_bytes(int64_t n, const sr_problem *prob, size_t *bytes)
{
    if (!bytes) return SR_E_ARG;
    // large enough with and without passive particles (the sort key differs)
    Single all, some;
    sr_status st = prepare_single(n, n, prob, all);
    if (st != SR_OK) return st;
    st = prepare_single(n, n > 0 ? n - 1 : 0, prob, some);
    if (st != SR_OK) return st;
    *bytes = std::max(all.L.total, some.L.total);
    return SR_OK;
}

sr_status sr_bin(const float *pos, const float *mass, int64_t n, int64_t n_active,
                 const sr_problem *prob, void *ws, size_t ws_bytes, void *stream)
{
    Single s;
    sr_status st = prepare_single(n, n_active, prob, s);
    if (st != SR_OK) return st;
    if (n > 0 && (!pos || !mass)) return SR_E_ARG;
    if ((st = check_ws(ws, ws_bytes, s.L)) != SR_OK) return st;
    if (n == 0) return SR_OK;
    DevArgs a;
    if ((st = device_args(a, ws, &s.L, &s.seg, nullptr, stream, 0, n_active)) != SR_OK) return st;
    return hip_status(dev_bin(a, pos, mass));
}

sr_status sr_bin_view(const void *ws, int64_t n, int64_t n_active, const sr_problem *prob,
                      sr_bin_layout *out)
{
    if (!ws || !out) return SR_E_ARG;
    Single s;
    const sr_status st = prepare_single(n, n_active, prob, s);
    if (st != SR_OK) return st;
    const char *w = static_cast<const char *>(ws);
    for (int d = 0; d < 3; ++d) out->nc[d] = s.nc[d];
    out->ncell = s.NC;
    out->cell_of = reinterpret_cast<const int32_t *>(w + s.L.cell_of);
    out->cell_start = reinterpret_cast<const int32_t *>(w + s.L.start);
    out->cell_nact = reinterpret_cast<const int32_t *>(w + s.L.nact);
    out->perm = reinterpret_cast<const int32_t *>(w + s.L.perm());
    out->off_x = reinterpret_cast<const float *>(w + s.L.bx);
    out->off_y = reinterpret_cast<const float *>(w + s.L.by);
    out->off_z = reinterpret_cast<const float *>(w + s.L.bz);
    out->mass = reinterpret_cast<const float *>(w + s.L.bm);
    return SR_OK;
}

sr_status sr_force(const float *pos, const float *mass, int64_t n, int64_t n_active,
                   const sr_problem *prob, void *ws, size_t ws_bytes, unsigned flags, float *acc,
                   void *stream)
{
    Single s;
    sr_status st = prepare_single(n, n_active, prob, s);
    if (st != SR_OK) return st;
    if (flags & ~SR_REUSE_BINS) return SR_E_ARG;
    if (n > 0 && (!pos || !mass)) return SR_E_ARG;
    if (n_active > 0 && !acc) return SR_E_ARG;
    if ((st = check_ws(ws, ws_bytes, s.L)) != SR_OK) return st;
    if (n == 0) return SR_OK;
    sym_tail(s.L, ws_bytes);  // the whole tail of the caller's workspace holds partial slots
    DevArgs a;
    if ((st = device_args(a, ws, &s.L, &s.seg, nullptr, stream, 0, n_active)) != SR_OK) return st;
    if (!(flags & SR_REUSE_BINS) && dev_bin(a, pos, mass) != hipSuccess) return SR_E_DEVICE;
    if (n_active == 0) return SR_OK;
    return hip_status(dev_force(a, acc));
}

sr_status sr_force_static(const float *pos, const float *mass, int64_t n, int64_t n_active,
                          const sr_problem *prob, float *acc, void *stream)
{
    Single s;
    sr_status st = prepare_single(n, n_active, prob, s);
    if (st != SR_OK) return st;
    if (s.L.total > (size_t)SR_STATIC_WORKSPACE_BYTES) return SR_E_UNSUPPORTED;
    if (n > 0 && (!pos || !mass)) return SR_E_ARG;
    if (n_active > 0 && !acc) return SR_E_ARG;
    if (n == 0) return SR_OK;
    void *ws = nullptr;
    size_t bytes = 0;
    if (sr::static_workspace(&ws, &bytes) != hipSuccess) return SR_E_DEVICE;
    return sr_force(pos, mass, n, n_active, prob, ws, bytes, 0, acc, stream);
}

sr_status sr_force_vjp(const float *pos, const float *mass, int64_t n, int64_t n_active,
                       const sr_problem *prob, void *ws, size_t ws_bytes, unsigned flags,
                       const float *g, float *grad_pos, void *stream)
{
    Single s;
    sr_status st = prepare_single(n, n_active, prob, s);
    if (st != SR_OK) return st;
    if (flags & ~SR_REUSE_BINS) return SR_E_ARG;
    if (n > 0 && (!pos || !mass || !grad_pos)) return SR_E_ARG;
    if (n_active > 0 && !g) return SR_E_ARG;
    if ((st = check_ws(ws, ws_bytes, s.L)) != SR_OK) return st;
    if (n == 0) return SR_OK;
    sym_tail(s.L, ws_bytes);
    DevArgs a;
    if ((st = device_args(a, ws, &s.L, &s.seg, nullptr, stream, 0, n_active, kCfgVjp)) != SR_OK) return st;
    if (!(flags & SR_REUSE_BINS) && dev_bin(a, pos, mass) != hipSuccess) return SR_E_DEVICE;
    return hip_status(dev_vjp(a, g, grad_pos));
}

sr_status sr_count_pairs(int64_t n, int64_t n_active, const sr_problem *prob, void *ws,
                         size_t ws_bytes, unsigned flags, int64_t *pairs, void *stream)
{
    Single s;
    sr_status st = prepare_single(n, n_active, prob, s);
    if (st != SR_OK) return st;
    if (!pairs || (flags & ~SR_COUNT_ADJOINT)) return SR_E_ARG;
    if ((st = check_ws(ws, ws_bytes, s.L)) != SR_OK) return st;
    DevArgs a;
    if ((st = device_args(a, ws, &s.L, &s.seg, nullptr, stream, 0, n_active)) != SR_OK) return st;
    if (n == 0 || n_active == 0) return hip_status(dev_zero(pairs, 2, a.st));
    return hip_status(dev_count_pairs(a, (flags & SR_COUNT_ADJOINT) != 0, pairs));
}

sr_status sr_momentum(const float *acc, const float *mass, int64_t n_rows, void *ws,
                      size_t ws_bytes, double *out, void *stream)
{
    if (n_rows < 0 || n_rows > kMaxParticles || !out) return SR_E_ARG;
    if (n_rows > 0 && (!acc || !mass)) return SR_E_ARG;
    if (!ws || reinterpret_cast<uintptr_t>(ws) % 256 != 0) return SR_E_WORKSPACE;
    Single M;
    M.seg = SegParams{};
    M.seg.n = (int32_t)n_rows;
    M.seg.n_active = (int32_t)n_rows;
    M.L = Layout{};
    M.L.B = 1;
    M.L.mom_tiles = mom_tiles_of(n_rows);
    const size_t need = align256((size_t)(3 * M.L.mom_tiles + 3) * 8);
    if (ws_bytes < need + 256) return SR_E_WORKSPACE;
    M.L.mom = (ws_bytes - need) & ~size_t(255);
    DevArgs a;
    sr_status st = device_args(a, ws, &M.L, &M.seg, nullptr, stream, 0, n_rows);
    if (st != SR_OK) return st;
    return hip_status(dev_momentum(a, acc, mass, out));
}

sr_status sr_ws_flags(const void *ws, void *stream, uint32_t *flags)
{
    if (!ws || !flags) return SR_E_ARG;
    uint32_t v = 0;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(&v, ws, sizeof(v), hipMemcpyDeviceToHost, st) != hipSuccess) return SR_E_DEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return SR_E_DEVICE;
    *flags = v;
    return SR_OK;
}

sr_status sr_batch_plan_create(int32_t B, const int64_t *offsets, const int64_t *n_active,
                               const sr_problem *probs, const char *tune_cache,
                               sr_batch_plan **plan, size_t *ws_bytes)
{
    if (!plan || !ws_bytes || B < 1 || !offsets || !n_active || !probs) return SR_E_ARG;
    *plan = nullptr;
    if (offsets[0] != 0) return SR_E_ARG;
    for (int b = 0; b < B; ++b) {
        const int64_t n = offsets[b + 1] - offsets[b];
        if (n < 0 || n_active[b] < 0 || n_active[b] > n) return SR_E_ARG;
    }
    if (offsets[B] > kMaxParticles) return SR_E_UNSUPPORTED;
    auto *P = new sr_batch_plan;
    P->B = B;
    P->offsets.assign(offsets, offsets + B + 1);
    P->n_active.assign(n_active, n_active + B);
    P->probs.assign(probs, probs + B);
    P->segs.resize(B);
    P->singles.resize(B);
    int64_t cell_off = 0, out_off = 0, tile_off = 0;
    size_t single_max = 0;
    bool soft = true;
    for (int b = 0; b < B; ++b) {
        const int64_t n = offsets[b + 1] - offsets[b];
        sr_status st = prepare_single(n, n_active[b], &probs[b], P->singles[b]);
        if (st != SR_OK) {
            delete P;
            return st;
        }
        single_max = std::max(single_max, P->singles[b].L.total);
        SegParams s = P->singles[b].seg;
        s.cell_off = (int32_t)cell_off;
        s.part_off = (int32_t)offsets[b];
        s.out_off = (int32_t)out_off;
        s.tile_off = (int32_t)tile_off;
        P->segs[b] = s;
        soft = soft && s.pc.softened;
        cell_off += P->singles[b].NC;
        out_off += n_active[b];
        tile_off += mom_tiles_of(n_active[b]);
        if (cell_off > kMaxCells) {
            delete P;
            return SR_E_UNSUPPORTED;
        }
    }
    P->total_active = out_off;
    P->summary = P->segs[0];
    P->summary.pc.softened = soft ? 1 : 0;
    bool any_passive = false;
    int depth = 1;
    for (int b = 0; b < B; ++b) {
        any_passive = any_passive || (n_active[b] < offsets[b + 1] - offsets[b]);
        depth = std::max(depth, (int)P->segs[b].leaf_depth);
    }
    if (!key_fits(cell_off, 3 * depth, any_passive)) {
        delete P;
        return SR_E_UNSUPPORTED;
    }
    P->L = make_layout(offsets[B], cell_off, B, tile_off, any_passive, 3 * depth);
    // per-subvolume momentum scratch sits at the end of the workspace
    const size_t mom_tail = align256((size_t)(3 * mom_tiles_of(offsets[B]) + 3) * 8) + 512;
    P->ws_bytes = std::max(P->L.total, single_max + mom_tail);
    if (hipHostMalloc((void **)&P->pinned, sizeof(SegParams) * B, hipHostMallocDefault) != hipSuccess) {
        delete P;
        return SR_E_DEVICE;
    }
    std::memcpy(P->pinned, P->segs.data(), sizeof(SegParams) * B);
    if (hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking) != hipSuccess) {
        (void)hipHostFree(P->pinned);
        delete P;
        return SR_E_DEVICE;
    }
    if (tune_cache) P->tune_cache = tune_cache;
    {
        std::ostringstream k;
        int nb = 0;
        while ((int64_t(1) << (nb + 1)) <= std::max<int64_t>(1, offsets[B])) ++nb;
        k << arch_name() << "/force-v3/B" << B << "/log2N" << nb << "/soft" << (soft ? 1 : 0)
          << "/leaf" << P->L.code_bits / 3;
        P->tune_key = k.str();
    }
    *plan = P;
    *ws_bytes = P->ws_bytes;
    return SR_OK;
}

sr_status sr_batch_force(sr_batch_plan *P, const float *pos, const float *mass, void *ws,
                         size_t ws_bytes, float *acc, double *momentum, unsigned flags,
                         void *stream)
{
    if (!P || P->B < 1) return SR_E_PLAN;
    if (flags & ~(SR_BATCH_PER_SUBVOLUME | SR_BATCH_EAGER | SR_BATCH_RECAPTURE)) return SR_E_ARG;
    const int64_t N = P->offsets[P->B];
    if (N > 0 && (!pos || !mass)) return SR_E_ARG;
    if (P->total_active > 0 && !acc) return SR_E_ARG;
    if (!ws || reinterpret_cast<uintptr_t>(ws) % 256 != 0 || ws_bytes < P->ws_bytes)
        return SR_E_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // tuned before the first run of any mode, so that every mode uses the same tiles
    if (P->waves_per_cu == 0) {
        sr_status s = tune(P, pos, mass, ws, acc, st);
        if (s != SR_OK) return s;
    }
    if (flags & SR_BATCH_PER_SUBVOLUME) return run_per_subvolume(P, pos, mass, ws, acc, momentum, st);
    if (flags & SR_BATCH_EAGER) return run_batched(P, pos, mass, ws, acc, momentum, st);
    const bool bound = P->exec && P->b_pos == pos && P->b_mass == mass && P->b_ws == ws &&
                       P->b_acc == acc && P->b_mom == momentum;
    if (P->exec && !bound && !(flags & SR_BATCH_RECAPTURE)) return SR_E_PLAN;
    if (!bound) {
        // Capture waits for nothing on the caller's stream: order it first.
        // The old graph may still run there (an earlier replay), so it is
        // destroyed only once the stream has drained.
        hipEvent_t ev;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return SR_E_DEVICE;
        (void)hipEventRecord(ev, st);
        (void)hipStreamWaitEvent(P->cap, ev, 0);
        const hipError_t se = hipStreamSynchronize(P->cap);
        (void)hipEventDestroy(ev);
        if (se != hipSuccess) return SR_E_DEVICE;
        drop_graph(P);
        if (hipStreamBeginCapture(P->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return SR_E_DEVICE;
        sr_status s = run_batched(P, pos, mass, ws, acc, momentum, P->cap);
        hipGraph_t g = nullptr;
        const hipError_t ee = hipStreamEndCapture(P->cap, &g);
        if (s != SR_OK || ee != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            return s != SR_OK ? s : SR_E_DEVICE;
        }
        P->graph = g;
        if (hipGraphInstantiate(&P->exec, g, nullptr, nullptr, 0) != hipSuccess) {
            drop_graph(P);
            return SR_E_DEVICE;
        }
        P->b_pos = pos;
        P->b_mass = mass;
        P->b_ws = ws;
        P->b_acc = acc;
        P->b_mom = momentum;
    }
    return hip_status(hipGraphLaunch(P->exec, st));
}

sr_status sr_batch_plan_destroy(sr_batch_plan *P)
{
    if (!P) return SR_E_PLAN;
    drop_graph(P);
    if (P->cap) (void)hipStreamDestroy(P->cap);
    if (P->pinned) (void)hipHostFree(P->pinned);
    delete P;
    return SR_OK;
}

sr_status sr_batch_plan_info(const sr_batch_plan *P, char *buf, size_t buf_bytes)
{
    if (!P || !buf || buf_bytes == 0) return SR_E_ARG;
    std::ostringstream o;
    o << "{\"B\": " << P->B << ", \"n\": " << P->offsets[P->B] << ", \"n_active\": "
      << P->total_active << ", \"cells\": " << P->L.NC << ", \"ws_bytes\": " << P->ws_bytes
      << ", \"waves_per_cu\": " << P->waves_per_cu << ", \"targets_per_lane\": "
      << P->targets_per_lane << ", \"occupancy\": " << P->occupancy << ", \"sym_blocks\": "
      << P->sym_blocks << ", \"sym_window\": " << P->sym_window << ", \"sparse_group\": "
      << P->sparse_group << ", \"tuned_ms\": "
      << P->tuned_ms
      << ", \"tune_key\": \"" << P->tune_key << "\", \"graph\": " << (P->exec ? "true" : "false")
      << "}";
    const std::string s = o.str();
    if (s.size() + 1 > buf_bytes) return SR_E_ARG;
    std::memcpy(buf, s.c_str(), s.size() + 1);
    return SR_OK;
}

namespace {

sr_status set_config(int k, int waves_per_cu, int targets_per_lane, int occupancy)
{
    if (waves_per_cu < 0 || waves_per_cu > 64 || targets_per_lane < 0 || targets_per_lane > 2)
        return SR_E_ARG;
    if (occupancy != -1 && occupancy != 0 && occupancy != 6 && occupancy != 8) return SR_E_ARG;
    if (waves_per_cu > 0) g_waves_default[k] = waves_per_cu;
    if (targets_per_lane > 0) g_tpl_default[k] = targets_per_lane;
    if (occupancy >= 0) g_occ_default[k] = occupancy;
    return SR_OK;
}

void get_config(int k, int *cur)
{
    if (!cur) return;
    cur[0] = g_waves_default[k].load();
    cur[1] = g_tpl_default[k].load();
    cur[2] = g_occ_default[k].load();
}

}  // namespace

sr_status sr_launch_config(int waves_per_cu, int targets_per_lane, int occupancy, int *cur)
{
    // validate once, then apply to both kernels
    sr_status st = set_config(kCfgForce, waves_per_cu, targets_per_lane, occupancy);
    if (st != SR_OK) return st;
    (void)set_config(kCfgVjp, waves_per_cu, targets_per_lane, occupancy);
    get_config(kCfgForce, cur);
    return SR_OK;
}

sr_status sr_tile_config(const char *kernel, int blocks_per_item, int window, int *cur)
{
    if (!kernel) return SR_E_ARG;
    int k = -1;
    if (std::strcmp(kernel, "force") == 0) k = kCfgForce;
    if (std::strcmp(kernel, "vjp") == 0) k = kCfgVjp;
    if (k < 0) return SR_E_ARG;
    if (blocks_per_item < -1 || blocks_per_item > 256) return SR_E_ARG;
    if (window != -1 && window != 256 && window != 512) return SR_E_ARG;
    if (blocks_per_item >= 0) g_sym_blocks[k] = blocks_per_item;
    if (window > 0) g_sym_window[k] = window;
    if (cur) {
        cur[0] = g_sym_blocks[k].load();
        cur[1] = g_sym_window[k].load();
    }
    return SR_OK;
}

sr_status sr_sparse_group(int group, int *cur)
{
    if (group != -1 && group != 8 && group != 16 && group != 32 && group != 64) return SR_E_ARG;
    if (group > 0) g_sparse_group = group;
    if (cur) *cur = g_sparse_group.load();
    return SR_OK;
}

sr_status sr_tile_balance(double min_ratio, double *cur)
{
    if (!(min_ratio >= 0.0 || min_ratio == -1.0) || !std::isfinite(min_ratio)) return SR_E_ARG;
    if (min_ratio >= 0.0) g_sym_balance = min_ratio;
    if (cur) *cur = g_sym_balance.load();
    return SR_OK;
}

sr_status sr_launch_config_kernel(const char *kernel, int waves_per_cu, int targets_per_lane,
                                  int occupancy, int *cur)
{
    if (!kernel) return SR_E_ARG;
    int k = -1;
    if (std::strcmp(kernel, "force") == 0) k = kCfgForce;
    if (std::strcmp(kernel, "vjp") == 0) k = kCfgVjp;
    if (k < 0) return SR_E_ARG;
    const sr_status st = set_config(k, waves_per_cu, targets_per_lane, occupancy);
    if (st != SR_OK) return st;
    get_config(k, cur);
    return SR_OK;
}

sr_status sr_timing_enable(int on)
{
    std::vector<TimingRec> old;
    {
        std::lock_guard<std::mutex> lk(g_tmu);
        g_timing = on != 0;
        old.swap(g_recs);
    }
    for (auto &r : old) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    return SR_OK;
}

sr_status sr_timing_read(const char *kernel, double *total_ms, int64_t *launches)
{
    if (!kernel || !total_ms || !launches) return SR_E_ARG;
    std::lock_guard<std::mutex> lk(g_tmu);
    double sum = 0.0;
    int64_t cnt = 0;
    for (auto &r : g_recs) {
        if (r.name != kernel) continue;
        if (hipEventSynchronize(r.b) != hipSuccess) return SR_E_DEVICE;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return SR_E_DEVICE;
        sum += ms;
        ++cnt;
    }
    *total_ms = sum;
    *launches = cnt;
    return SR_OK;
}

}  // extern "C"
