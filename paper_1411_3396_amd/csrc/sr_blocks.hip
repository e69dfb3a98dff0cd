// Overlapping data blocks of one domain (paper Sec. 2.1).
//
// The domain's x-y extent is tiled by rectangles given in whole grid units;
// block b owns the active particles inside its rectangle (outer rectangles
// reach to infinity, so every particle has exactly one home) and receives, as
// passive copies, every particle within r_s of the rectangle in x and y.  Each
// block is then an independent open-domain problem; reconciling keeps each
// active particle's acceleration from its home block and drops the passive
// duplicates, and for gradients sums the contributions of every copy.
//
// Device passes: membership count, expansion to (block, passive) keys, the
// stable radix sort shared with the binning, block starts, then plain gathers
// and scatters.  A block lists its active members first, each group in domain
// index order, so block inputs and every reconciled result are deterministic.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <vector>

#include "sr_internal.h"

namespace sr {
namespace {

constexpr int kMaxBlocks = 1024;
constexpr int kRectChunk = 256;          // rectangles staged in LDS per round
constexpr double kShellMargin = 1e-5;    // relative widening of the r_s shell
constexpr int64_t kMaxEntries = (int64_t(1) << 31) - 1;

// Per block, 8 floats: home rectangle [x0, x1) x [y0, y1) (infinite at the
// tiling's outer edges) and its widening by the shell.
struct Rect {
    float x0, x1, y0, y1, wx0, wx1, wy0, wy1;
};

// Home block and memberships of one particle; calls emit(b, passive) in
// increasing b.  Every thread of the workgroup takes part in the LDS staging,
// so callers keep out-of-range threads in the loop with live = false.
template <class Emit>
__device__ __forceinline__ void for_each_member(const Rect *__restrict__ rects, int nb, float x,
                                                float y, bool live, bool active, Rect *lds,
                                                Emit emit)
{
    // pass 1: home, the rectangle that holds the point (none for NaN: block 0)
    int home = -1;
    for (int c0 = 0; c0 < nb; c0 += kRectChunk) {
        const int cn = min(kRectChunk, nb - c0);
        __syncthreads();
        if ((int)threadIdx.x < cn) lds[threadIdx.x] = rects[c0 + threadIdx.x];
        __syncthreads();
        if (live && home < 0) {
            for (int k = 0; k < cn; ++k) {
                const Rect r = lds[k];
                if (x >= r.x0 && x < r.x1 && y >= r.y0 && y < r.y1) {
                    home = c0 + k;
                    break;
                }
            }
        }
    }
    if (home < 0) home = 0;
    // pass 2: memberships in block order
    for (int c0 = 0; c0 < nb; c0 += kRectChunk) {
        const int cn = min(kRectChunk, nb - c0);
        __syncthreads();
        if ((int)threadIdx.x < cn) lds[threadIdx.x] = rects[c0 + threadIdx.x];
        __syncthreads();
        if (live) {
            for (int k = 0; k < cn; ++k) {
                const Rect r = lds[k];
                const int b = c0 + k;
                const bool in = x >= r.wx0 && x < r.wx1 && y >= r.wy0 && y < r.wy1;
                if (in || b == home) emit(b, !(active && b == home));
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_blk_count(const float *__restrict__ pos, int n, int nb,
                                                   const Rect *__restrict__ rects,
                                                   int *__restrict__ cnt)
{
    __shared__ Rect lds[kRectChunk];
    const int i = blockIdx.x * 256 + threadIdx.x;
    const bool live = i < n;
    const float x = live ? pos[3 * (int64_t)i] : 0.f;
    const float y = live ? pos[3 * (int64_t)i + 1] : 0.f;
    int c = 0;
    for_each_member(rects, nb, x, y, live, false, lds, [&](int, bool) { ++c; });
    if (live) cnt[i] = c;
}

// Entries of particle i at [first[i], first[i+1]): key 2b + passive, and the
// particle it copies.  The sort's values default to the entry index.
__global__ __launch_bounds__(256) void k_blk_expand(const float *__restrict__ pos, int n,
                                                    int n_active, int nb,
                                                    const Rect *__restrict__ rects,
                                                    const int *__restrict__ first,
                                                    int *__restrict__ key, int *__restrict__ owner)
{
    __shared__ Rect lds[kRectChunk];
    const int i = blockIdx.x * 256 + threadIdx.x;
    const bool live = i < n;
    const float x = live ? pos[3 * (int64_t)i] : 0.f;
    const float y = live ? pos[3 * (int64_t)i + 1] : 0.f;
    int e = live ? first[i] : 0;
    for_each_member(rects, nb, x, y, live, i < n_active, lds, [&](int b, bool passive) {
        key[e] = 2 * b + (passive ? 1 : 0);
        owner[e] = i;
        ++e;
    });
}

// Sorted slot s holds entry sv[s]: its particle, and the way back.
__global__ __launch_bounds__(256) void k_blk_slots(const int *__restrict__ sv, int m,
                                                   const int *__restrict__ owner,
                                                   int *__restrict__ src, int *__restrict__ inv)
{
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= m) return;
    const int e = sv[s];
    src[s] = owner[e];
    inv[e] = s;
}

// Active row r of the block outputs (blocks back to back, block c's rows
// [A[c], A[c+1])) -> domain index.
__global__ __launch_bounds__(256) void k_blk_rows(const int *__restrict__ src,
                                                  const int *__restrict__ S,
                                                  const int *__restrict__ A, int nb, int rows,
                                                  int *__restrict__ rowsrc)
{
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= rows) return;
    int lo = 0, hi = nb - 1;  // last c with A[c] <= r
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (A[mid] <= r)
            lo = mid;
        else
            hi = mid - 1;
    }
    rowsrc[r] = src[S[2 * lo] + (r - A[lo])];
}

__global__ __launch_bounds__(256) void k_blk_gather(const int *__restrict__ src, int m,
                                                    const float *__restrict__ pos,
                                                    const float *__restrict__ mass,
                                                    float *__restrict__ bpos,
                                                    float *__restrict__ bmass,
                                                    int *__restrict__ src_out)
{
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= m) return;
    const int i = src[s];
    const int64_t p = 3 * (int64_t)i, q = 3 * (int64_t)s;
    bpos[q] = pos[p];
    bpos[q + 1] = pos[p + 1];
    bpos[q + 2] = pos[p + 2];
    bmass[s] = mass[i];
    if (src_out) src_out[s] = i;
}

// 3-vectors: out[r] = in[map[r]] (to_rows) or out[map[r]] = in[r].
__global__ __launch_bounds__(256) void k_blk_rows_copy(const int *__restrict__ map, int rows,
                                                       const float *__restrict__ in,
                                                       float *__restrict__ out, int to_rows)
{
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= rows) return;
    const int64_t a = 3 * (int64_t)map[r], q = 3 * (int64_t)r;
    const int64_t from = to_rows ? a : q, to = to_rows ? q : a;
    out[to] = in[from];
    out[to + 1] = in[from + 1];
    out[to + 2] = in[from + 2];
}

// grad[i] = sum over the copies of particle i, in block order.
__global__ __launch_bounds__(256) void k_blk_sum_copies(const int *__restrict__ first,
                                                        const int *__restrict__ inv, int n,
                                                        const float *__restrict__ bgrad,
                                                        float *__restrict__ grad)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float gx = 0.f, gy = 0.f, gz = 0.f;
    for (int e = first[i]; e < first[i + 1]; ++e) {
        const int64_t q = 3 * (int64_t)inv[e];
        gx += bgrad[q];
        gy += bgrad[q + 1];
        gz += bgrad[q + 2];
    }
    const int64_t o = 3 * (int64_t)i;
    grad[o] = gx;
    grad[o + 1] = gy;
    grad[o + 2] = gz;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

struct BlockLayout {
    int passes = 1, digit_bits = 1;
    int64_t tiles = 1, table = 0;
    size_t cnt = 0, first = 0, scan_tmp = 0, keys[2] = {0, 0}, vals[2] = {0, 0}, owner = 0, inv = 0,
           src = 0, rowsrc = 0, S = 0, A = 0, rects = 0, tab = 0, tabx = 0, total = 0;
};

BlockLayout block_layout(int64_t n, int64_t n_active, int nb, int64_t cap)
{
    BlockLayout L;
    int bits = 1;
    while ((int64_t(1) << bits) < 2 * (int64_t)nb) ++bits;
    L.passes = (bits + 7) / 8;
    L.digit_bits = (bits + L.passes - 1) / L.passes;
    L.tiles = std::max<int64_t>(1, (cap + kRadixTile - 1) / kRadixTile);
    L.table = (int64_t(1) << L.digit_bits) * L.tiles;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align256(o + std::max<size_t>(bytes, 1));
        return at;
    };
    L.cnt = take((size_t)n * 4);
    L.first = take((size_t)(n + 1) * 4);
    L.scan_tmp = take((size_t)std::max(scan_scratch_elems(n), scan_scratch_elems(L.table)) * 4);
    for (int k = 0; k < 2; ++k) {
        L.keys[k] = take((size_t)cap * 4);
        L.vals[k] = take((size_t)cap * 4);
    }
    L.owner = take((size_t)cap * 4);
    L.inv = take((size_t)cap * 4);
    L.src = take((size_t)cap * 4);
    L.rowsrc = take((size_t)n_active * 4);
    L.S = take((size_t)(2 * nb + 1) * 4);
    L.A = take((size_t)(nb + 1) * 4);
    L.rects = take(sizeof(Rect) * nb);
    L.tab = take((size_t)L.table * 4);
    L.tabx = take((size_t)(L.table + 1) * 4);
    L.total = o;
    return L;
}

}  // namespace
}  // namespace sr

using namespace sr;

struct sr_blocks_plan {
    sr_problem domain{};
    int32_t ng[2] = {1, 1};
    std::vector<sr_block> blocks;
    std::vector<Rect> rects;
    std::vector<sr_problem> probs;
    int64_t n = 0, n_active = 0, cap = 0;
    BlockLayout L;
    int64_t members = -1;         // set by a partition
    std::vector<int64_t> counts;  // [nb][2], set by a partition
};

namespace {

// Grid-unit edge g of an axis: lo + g * len / ng, rounded once to float32.
// Adjacent blocks use the same value for a shared edge, so the half-open
// home rectangles tile the plane exactly.
float edge(const sr_problem &d, const int32_t ng[2], int axis, int g)
{
    return (float)((double)d.lo[axis] + (double)g * (double)d.len[axis] / (double)ng[axis]);
}

sr_status validate(const sr_problem *domain, const int32_t *ng, int32_t nb, const sr_block *blocks)
{
    if (!domain || !ng || !blocks || nb < 1 || nb > kMaxBlocks) return SR_E_ARG;
    int32_t nc[3];
    const sr_status st = sr_grid(domain, nc);
    if (st != SR_OK) return st;
    if (domain->periodic) return SR_E_UNSUPPORTED;  // rectangles of a periodic box would wrap
    if (ng[0] < 1 || ng[1] < 1 || ng[0] > (1 << 20) || ng[1] > (1 << 20)) return SR_E_ARG;
    int64_t area = 0;
    for (int b = 0; b < nb; ++b) {
        const sr_block &r = blocks[b];
        if (r.gx0 < 0 || r.gx0 >= r.gx1 || r.gx1 > ng[0] || r.gy0 < 0 || r.gy0 >= r.gy1 ||
            r.gy1 > ng[1])
            return SR_E_ARG;
        area += (int64_t)(r.gx1 - r.gx0) * (r.gy1 - r.gy0);
    }
    if (area != (int64_t)ng[0] * ng[1]) return SR_E_ARG;  // gaps or overlaps
    for (int a = 0; a < nb; ++a)
        for (int b = a + 1; b < nb; ++b) {
            const sr_block &p = blocks[a], &q = blocks[b];
            if (p.gx0 < q.gx1 && q.gx0 < p.gx1 && p.gy0 < q.gy1 && q.gy0 < p.gy1) return SR_E_ARG;
        }
    return SR_OK;
}

void make_rects(sr_blocks_plan &P)
{
    const int nb = (int)P.blocks.size();
    const float inf = std::numeric_limits<float>::infinity();
    const sr_problem &d = P.domain;
    const float rs = (float)((double)d.r_s * (1.0 + kShellMargin));
    const float pad = (float)((double)d.r_s * kShellMargin);
    const float dlo[2] = {d.lo[0], d.lo[1]};
    const float dhi[2] = {d.lo[0] + d.len[0], d.lo[1] + d.len[1]};
    P.rects.resize(nb);
    P.probs.resize(nb);
    for (int b = 0; b < nb; ++b) {
        const sr_block &k = P.blocks[b];
        const int g0[2] = {k.gx0, k.gy0}, g1[2] = {k.gx1, k.gy1};
        float h0[2], h1[2], w0[2], w1[2];
        sr_problem p = d;
        for (int a = 0; a < 2; ++a) {
            h0[a] = g0[a] == 0 ? -inf : edge(d, P.ng, a, g0[a]);
            h1[a] = g1[a] == P.ng[a] ? inf : edge(d, P.ng, a, g1[a]);
            w0[a] = h0[a] - rs;
            w1[a] = h1[a] + rs;
            // the block's domain: its widened rectangle clipped to the domain,
            // with a little room so no member sits on a float-rounded edge
            const float lo = g0[a] == 0 ? dlo[a] : std::max(dlo[a], w0[a] - pad);
            const float hi = g1[a] == P.ng[a] ? dhi[a] : std::min(dhi[a], w1[a] + pad);
            p.lo[a] = lo;
            p.len[a] = (g0[a] == 0 && g1[a] == P.ng[a]) ? d.len[a] : hi - lo;
        }
        P.rects[b] = Rect{h0[0], h1[0], h0[1], h1[1], w0[0], w1[0], w0[1], w1[1]};
        P.probs[b] = p;
    }
}

// Most widened rectangles a point can lie in: a point in k of them lies in
// one that meets the other k - 1.
int64_t overlap_bound(const std::vector<Rect> &R)
{
    int64_t best = 1;
    for (size_t a = 0; a < R.size(); ++a) {
        int64_t k = 0;
        for (size_t b = 0; b < R.size(); ++b)
            if (R[a].wx0 < R[b].wx1 && R[b].wx0 < R[a].wx1 && R[a].wy0 < R[b].wy1 && R[b].wy0 < R[a].wy1)
                ++k;
        best = std::max(best, k);
    }
    return best;
}

sr_status check_ws(const sr_blocks_plan *P, const void *ws, size_t ws_bytes)
{
    if (!ws || reinterpret_cast<uintptr_t>(ws) % 256 != 0 || ws_bytes < P->L.total) return SR_E_WORKSPACE;
    return SR_OK;
}

}  // namespace

extern "C" {

sr_status sr_blocks_plan_create(const sr_problem *domain, const int32_t *ng, int32_t nb,
                                const sr_block *blocks, int64_t n, int64_t n_active,
                                int64_t capacity, sr_blocks_plan **plan, size_t *ws_bytes)
{
    if (!plan || !ws_bytes) return SR_E_ARG;
    *plan = nullptr;
    sr_status st = validate(domain, ng, nb, blocks);
    if (st != SR_OK) return st;
    if (n < 0 || n > kMaxEntries || n_active < 0 || n_active > n || capacity < 0) return SR_E_ARG;
    auto *P = new sr_blocks_plan;
    P->domain = *domain;
    P->ng[0] = ng[0];
    P->ng[1] = ng[1];
    P->blocks.assign(blocks, blocks + nb);
    P->n = n;
    P->n_active = n_active;
    make_rects(*P);
    for (int b = 0; b < nb; ++b) {
        int32_t nc[3];
        if ((st = sr_grid(&P->probs[b], nc)) != SR_OK) {
            delete P;
            return st;
        }
    }
    // the membership scan counts in int32: the worst case must fit
    const int64_t bound = std::max<int64_t>(1, n) * overlap_bound(P->rects);
    int64_t cap = capacity > 0 ? std::min(capacity, bound) : bound;
    cap = std::max<int64_t>(cap, std::max<int64_t>(1, n));
    if (bound > kMaxEntries) {
        delete P;
        return SR_E_UNSUPPORTED;
    }
    P->cap = cap;
    P->L = block_layout(n, n_active, nb, cap);
    *plan = P;
    *ws_bytes = P->L.total;
    return SR_OK;
}

sr_status sr_blocks_plan_destroy(sr_blocks_plan *P)
{
    if (!P) return SR_E_PLAN;
    delete P;
    return SR_OK;
}

sr_status sr_blocks_problems(const sr_blocks_plan *P, sr_problem *out)
{
    if (!P) return SR_E_PLAN;
    if (!out) return SR_E_ARG;
    std::copy(P->probs.begin(), P->probs.end(), out);
    return SR_OK;
}

sr_status sr_blocks_partition(sr_blocks_plan *P, const float *pos, void *ws, size_t ws_bytes,
                              int64_t *members, int64_t *counts, void *stream)
{
    if (!P) return SR_E_PLAN;
    if (!members || !counts || (P->n > 0 && !pos)) return SR_E_ARG;
    sr_status st = check_ws(P, ws, ws_bytes);
    if (st != SR_OK) return st;
    const int nb = (int)P->blocks.size();
    const int64_t n = P->n;
    const BlockLayout &L = P->L;
    P->members = -1;
    *members = 0;
    if (n == 0) {
        std::fill(counts, counts + 2 * nb, int64_t(0));
        P->counts.assign(2 * nb, 0);
        P->members = 0;
        return SR_OK;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    auto I = [&](size_t off) { return reinterpret_cast<int *>(w + off); };
    Rect *rects = reinterpret_cast<Rect *>(w + L.rects);
    if (hipMemcpyAsync(rects, P->rects.data(), sizeof(Rect) * nb, hipMemcpyHostToDevice, s) != hipSuccess)
        return SR_E_DEVICE;
    k_blk_count<<<nblk(n), 256, 0, s>>>(pos, (int)n, nb, rects, I(L.cnt));
    if (hipGetLastError() != hipSuccess) return SR_E_DEVICE;
    if (dev_scan(I(L.cnt), I(L.first), n, I(L.scan_tmp), s) != hipSuccess) return SR_E_DEVICE;
    int m32 = 0;
    if (hipMemcpyAsync(&m32, I(L.first) + n, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return SR_E_DEVICE;
    const int64_t m = (uint32_t)m32;
    *members = m;
    if (m > P->cap) return SR_E_WORKSPACE;  // *members is the capacity needed
    // Entries start in key buffer 1; sort pass p writes buffer p & 1 and reads
    // the other, so the sorted keys and entry indices land in (passes-1) & 1.
    k_blk_expand<<<nblk(n), 256, 0, s>>>(pos, (int)n, (int)P->n_active, nb, rects, I(L.first),
                                        I(L.keys[1]), I(L.owner));
    if (hipGetLastError() != hipSuccess) return SR_E_DEVICE;
    const int64_t tiles = std::max<int64_t>(1, (m + kRadixTile - 1) / kRadixTile);
    const RadixBufs rb{{I(L.keys[0]), I(L.keys[1])}, {I(L.vals[0]), I(L.vals[1])}, I(L.tab),
                       I(L.tabx), I(L.scan_tmp)};
    if (radix_sort_pairs(I(L.keys[1]), nullptr, m, L.passes, L.digit_bits, tiles, rb, s) != hipSuccess)
        return SR_E_DEVICE;
    const int out = (L.passes - 1) & 1;
    if (dev_bounds(I(L.keys[out]), m, 2 * nb, 0, I(L.S), s) != hipSuccess) return SR_E_DEVICE;
    k_blk_slots<<<nblk(m), 256, 0, s>>>(I(L.vals[out]), (int)m, I(L.owner), I(L.src), I(L.inv));
    if (hipGetLastError() != hipSuccess) return SR_E_DEVICE;
    std::vector<int> S(2 * nb + 1);
    if (hipMemcpyAsync(S.data(), I(L.S), sizeof(int) * (2 * nb + 1), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return SR_E_DEVICE;
    std::vector<int> A(nb + 1, 0);
    std::vector<int64_t> cnt(2 * nb, 0);
    for (int c = 0; c < nb; ++c) {
        cnt[2 * c] = S[2 * c + 1] - S[2 * c];
        cnt[2 * c + 1] = S[2 * c + 2] - S[2 * c + 1];
        A[c + 1] = A[c] + (int)cnt[2 * c];
    }
    if (A[nb] != P->n_active || S[2 * nb] != m) return SR_E_DEVICE;  // one home per active particle
    if (hipMemcpyAsync(I(L.A), A.data(), sizeof(int) * (nb + 1), hipMemcpyHostToDevice, s) != hipSuccess)
        return SR_E_DEVICE;
    if (P->n_active > 0) {
        k_blk_rows<<<nblk(P->n_active), 256, 0, s>>>(I(L.src), I(L.S), I(L.A), nb, (int)P->n_active,
                                                      I(L.rowsrc));
        if (hipGetLastError() != hipSuccess) return SR_E_DEVICE;
    }
    if (hipStreamSynchronize(s) != hipSuccess) return SR_E_DEVICE;  // A is a host temporary
    P->counts = cnt;
    std::copy(cnt.begin(), cnt.end(), counts);
    P->members = m;
    return SR_OK;
}

sr_status sr_blocks_gather(const sr_blocks_plan *P, const float *pos, const float *mass,
                           const float *g, const void *ws, size_t ws_bytes, float *bpos,
                           float *bmass, float *bg, int32_t *src, void *stream)
{
    if (!P || P->members < 0) return SR_E_PLAN;  // no partition yet
    sr_status st = check_ws(P, ws, ws_bytes);
    if (st != SR_OK) return st;
    const int64_t m = P->members;
    if (m > 0 && (!pos || !mass || !bpos || !bmass)) return SR_E_ARG;
    if ((g == nullptr) != (bg == nullptr)) return SR_E_ARG;
    const BlockLayout &L = P->L;
    const char *w = static_cast<const char *>(ws);
    auto I = [&](size_t off) { return reinterpret_cast<const int *>(w + off); };
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (m > 0) {
        k_blk_gather<<<nblk(m), 256, 0, s>>>(I(L.src), (int)m, pos, mass, bpos, bmass, src);
        if (hipGetLastError() != hipSuccess) return SR_E_DEVICE;
    }
    if (g && P->n_active > 0) {
        k_blk_rows_copy<<<nblk(P->n_active), 256, 0, s>>>(I(L.rowsrc), (int)P->n_active, g, bg, 1);
        if (hipGetLastError() != hipSuccess) return SR_E_DEVICE;
    }
    return SR_OK;
}

sr_status sr_blocks_reconcile(const sr_blocks_plan *P, const void *ws, size_t ws_bytes,
                              const float *bacc, float *acc, void *stream)
{
    if (!P || P->members < 0) return SR_E_PLAN;
    sr_status st = check_ws(P, ws, ws_bytes);
    if (st != SR_OK) return st;
    if (P->n_active == 0) return SR_OK;
    if (!bacc || !acc) return SR_E_ARG;
    const char *w = static_cast<const char *>(ws);
    k_blk_rows_copy<<<nblk(P->n_active), 256, 0, static_cast<hipStream_t>(stream)>>>(
        reinterpret_cast<const int *>(w + P->L.rowsrc), (int)P->n_active, bacc, acc, 0);
    return hipGetLastError() == hipSuccess ? SR_OK : SR_E_DEVICE;
}

sr_status sr_blocks_reconcile_grad(const sr_blocks_plan *P, const void *ws, size_t ws_bytes,
                                   const float *bgrad, float *grad, void *stream)
{
    if (!P || P->members < 0) return SR_E_PLAN;
    sr_status st = check_ws(P, ws, ws_bytes);
    if (st != SR_OK) return st;
    if (P->n == 0) return SR_OK;
    if (!bgrad || !grad) return SR_E_ARG;
    const char *w = static_cast<const char *>(ws);
    k_blk_sum_copies<<<nblk(P->n), 256, 0, static_cast<hipStream_t>(stream)>>>(
        reinterpret_cast<const int *>(w + P->L.first), reinterpret_cast<const int *>(w + P->L.inv),
        (int)P->n, bgrad, grad);
    return hipGetLastError() == hipSuccess ? SR_OK : SR_E_DEVICE;
}

}  // extern "C"
