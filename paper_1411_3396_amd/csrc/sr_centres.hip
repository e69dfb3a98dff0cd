// Most-bound-particle halo centres (paper Sec. 2.2).
//
// For every particle of a halo, phi_i = -sum_{j in halo, j != i} m_j /
// sqrt(|x_j - x_i|^2 + eps^2), and per halo the particle with the smallest
// phi.  All pairs inside a halo, no cutoff: every evaluated pair is useful.
//
// Work items are (halo, up to 128 targets), heaviest first, pulled by
// persistent one-wave workgroups.  A wave stages 64 sources of its halo at a
// time in LDS (the next 64 are loaded into registers meanwhile) and every
// lane sums the staged sources for its targets: one target per lane, two
// per lane for items of more than 64 targets, or 2^lk lanes per target for
// halos of fewer than 64 particles.  Pair terms are float32; every 8 terms
// are added to a float64 accumulator, so the rounding does not grow with the
// halo size.  Each item also reduces its targets to a (phi, index) minimum,
// and a second pass takes the minimum over a halo's items.  The order of
// every sum is fixed by the item table, so results are bitwise reproducible.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "sr_internal.h"

namespace sr {
namespace {

constexpr float kFarAway = 1.0e18f;  // padding source: contributes m q = 0 * q
constexpr int kTargetsPerWave = 64;

// Workspace header: the condition word first (read by sr_ws_flags, like a
// force workspace's), the queue counter on its own 128-byte line.
struct CentreHeader {
    uint32_t flags;
    uint32_t pad0[31];
    uint32_t next;  // queue counter
    uint32_t pad1[31];
};

// Item: x = halo, y = first target, z = targets, w = lk | two << 4 | slot << 5.
__device__ __forceinline__ int4 uniform_item(const int4 *__restrict__ items, uint32_t g)
{
    const int4 it = items[g];
    return make_int4(__builtin_amdgcn_readfirstlane(it.x), __builtin_amdgcn_readfirstlane(it.y),
                     __builtin_amdgcn_readfirstlane(it.z), __builtin_amdgcn_readfirstlane(it.w));
}

// Source j of a halo as (x, y, z, m); past the end: far away and massless.
__device__ __forceinline__ float4 load_source(const float *__restrict__ pos,
                                              const float *__restrict__ mass, int j, int end)
{
    if (j < end) {
        const int64_t p = 3 * (int64_t)j;
        return make_float4(pos[p], pos[p + 1], pos[p + 2], mass[j]);
    }
    return make_float4(kFarAway, kFarAway, kFarAway, 0.f);
}

// m_j / sqrt(|d|^2 + eps^2), added to g.  Without softening a pair at zero
// distance (the target itself, or a coincident particle) adds nothing.
template <bool kSoft>
__device__ __forceinline__ float pot_term(const float4 s, float px, float py, float pz, float eps2,
                                          float g)
{
    const float dx = s.x - px, dy = s.y - py, dz = s.z - pz;
    const float t = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
    float q = __builtin_amdgcn_rsqf(t);
    if (!kSoft) q = t > 0.f ? q : 0.f;
    return fmaf(s.w, q, g);
}

struct MinIdx {
    float v;
    int i;
};

__device__ __forceinline__ bool better(float v, int i, float w, int j)
{
    // smaller phi first, then the smaller index; a NaN never wins against a number
    if (v < w) return true;
    if (v == w) return i < j;
    return !(v == v) ? false : !(w == w);
}

__device__ __forceinline__ MinIdx wave_argmin(float v, int i)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const float w = __shfl_xor(v, o);
        const int j = __shfl_xor(i, o);
        if (better(w, j, v, i)) {
            v = w;
            i = j;
        }
    }
    return MinIdx{v, i};
}

// Sums over the 64 staged sources.  `self*` is the stage index of the
// target itself in this chunk, or -1.  Groups of 8 float32 terms go into the
// float64 accumulators.

// One target per lane.
template <bool kSoft, bool kSelf>
__device__ __forceinline__ void sum_dense(const float4 *stage, float px, float py, float pz,
                                          float eps2, int self, double &acc)
{
    for (int k = 0; k < kTargetsPerWave; k += 8) {
        // even and odd sources in two float32 partial sums: two independent
        // FMA chains instead of one
        float g0 = 0.f, g1 = 0.f;
#pragma unroll
        for (int u = 0; u < 8; u += 2) {
            const float t0 = pot_term<kSoft>(stage[k + u], px, py, pz, eps2, g0);
            const float t1 = pot_term<kSoft>(stage[k + u + 1], px, py, pz, eps2, g1);
            g0 = (kSelf && k + u == self) ? g0 : t0;
            g1 = (kSelf && k + u + 1 == self) ? g1 : t1;
        }
        acc += (double)(g0 + g1);
    }
}

// Two targets per lane: each staged source is read once for both.
template <bool kSoft, bool kSelf>
__device__ __forceinline__ void sum_two(const float4 *stage, float ax, float ay, float az, float bx,
                                        float by, float bz, float eps2, int self_a, int self_b,
                                        double &acc_a, double &acc_b)
{
    for (int k = 0; k < kTargetsPerWave; k += 8) {
        // per target, even and odd sources in two float32 partial sums
        float ga0 = 0.f, ga1 = 0.f, gb0 = 0.f, gb1 = 0.f;
#pragma unroll
        for (int u = 0; u < 8; u += 2) {
            const float4 s0 = stage[k + u], s1 = stage[k + u + 1];
            const float ta0 = pot_term<kSoft>(s0, ax, ay, az, eps2, ga0);
            const float tb0 = pot_term<kSoft>(s0, bx, by, bz, eps2, gb0);
            const float ta1 = pot_term<kSoft>(s1, ax, ay, az, eps2, ga1);
            const float tb1 = pot_term<kSoft>(s1, bx, by, bz, eps2, gb1);
            ga0 = (kSelf && k + u == self_a) ? ga0 : ta0;
            gb0 = (kSelf && k + u == self_b) ? gb0 : tb0;
            ga1 = (kSelf && k + u + 1 == self_a) ? ga1 : ta1;
            gb1 = (kSelf && k + u + 1 == self_b) ? gb1 : tb1;
        }
        acc_a += (double)(ga0 + ga1);
        acc_b += (double)(gb0 + gb1);
    }
}

// 2^lk lanes per target (lk >= 1): lane sub takes stage entries sub, sub + 2^lk, ...
template <bool kSoft, bool kSelf>
__device__ __forceinline__ void sum_sparse(const float4 *stage, int lk, int sub, float px,
                                           float py, float pz, float eps2, int self, double &acc)
{
    const int kl = 1 << lk;
    const int per = kTargetsPerWave >> lk;  // 1 .. 32
    for (int k = 0; k < per; k += 8) {
        float g = 0.f;
        for (int u = 0; u < 8 && k + u < per; ++u) {
            const int at = (k + u) * kl + sub;
            const float t = pot_term<kSoft>(stage[at], px, py, pz, eps2, g);
            g = (kSelf && at == self) ? g : t;
        }
        acc += (double)g;
    }
}

template <bool kSoft>
__global__ __launch_bounds__(64, 4) void k_centre_potential(
    const int4 *__restrict__ items, uint32_t n_items, const int *__restrict__ hoff,
    const float *__restrict__ pos, const float *__restrict__ mass, float eps2,
    float *__restrict__ phi, int2 *__restrict__ partial, CentreHeader *hdr, int64_t pull_limit)
{
    __shared__ float4 stage[kTargetsPerWave];
    const int lane = threadIdx.x;
    // Loop bound: the counter hands out increasing values, so one wave's
    // items increase strictly and it cannot pull more than exist.  A pull
    // that breaks either rule ends the loop and flags the workspace instead
    // of spinning; pull_limit below the item count (a test hook) ends every
    // wave early on purpose.
    const int64_t limit = min((int64_t)n_items, pull_limit);
    int64_t pulls = 0, last = -1;
    bool bad = false;
    for (;;) {
        // Lane 0 takes the next item; the loop body below ends with no other
        // lane-0-only branch, so the compiler cannot merge the two into one
        // region across the loop's back edge (which would let the other
        // lanes start the next iteration without lane 0's new item).
        uint32_t g = 0;
        if (lane == 0) g = atomicAdd(&hdr->next, 1u);
        g = __builtin_amdgcn_readfirstlane(g);
        if (g >= n_items) break;
        if ((int64_t)g <= last || ++pulls > limit) {
            bad = true;
            break;
        }
        last = g;
        const int4 it = uniform_item(items, g);
        const int h = it.x, t0 = it.y, nt = it.z, lk = it.w & 15;
        const bool two = (it.w >> 4) & 1;
        const int slot = it.w >> 5;
        const int s0 = __builtin_amdgcn_readfirstlane(hoff[h]);
        const int s1 = __builtin_amdgcn_readfirstlane(hoff[h + 1]);
        const int kl = 1 << lk;
        const int tsub = lane >> lk, sub = lane & (kl - 1);
        // targets of this lane: a = t0 + tsub (dense: tsub = lane), b = a + 64
        const bool va = tsub < min(nt, kTargetsPerWave);
        const bool vb = two && lane + kTargetsPerWave < nt;
        const int ia = t0 + tsub, ib = t0 + kTargetsPerWave + lane;
        float ax = 0.f, ay = 0.f, az = 0.f, bx = 0.f, by = 0.f, bz = 0.f;
        if (va) {
            ax = pos[3 * (int64_t)ia];
            ay = pos[3 * (int64_t)ia + 1];
            az = pos[3 * (int64_t)ia + 2];
        }
        if (vb) {
            bx = pos[3 * (int64_t)ib];
            by = pos[3 * (int64_t)ib + 1];
            bz = pos[3 * (int64_t)ib + 2];
        }
        double acc_a = 0.0, acc_b = 0.0;
        float4 next = load_source(pos, mass, s0 + lane, s1);
        // Chunks start at s0 + 64 m and items at s0 + 128 k, so the targets'
        // own entries are in the chunks starting at t0 (a) and t0 + 64 (b).
        for (int base = s0; base < s1; base += kTargetsPerWave) {
            __syncthreads();
            stage[lane] = next;
            __syncthreads();
            if (base + kTargetsPerWave < s1) next = load_source(pos, mass, base + kTargetsPerWave + lane, s1);
            const bool own_a = base == t0, own_b = base == t0 + kTargetsPerWave;
            if (two) {
                if (own_a || own_b)
                    sum_two<kSoft, true>(stage, ax, ay, az, bx, by, bz, eps2, own_a ? lane : -1,
                                         own_b ? lane : -1, acc_a, acc_b);
                else
                    sum_two<kSoft, false>(stage, ax, ay, az, bx, by, bz, eps2, -1, -1, acc_a, acc_b);
            } else if (lk == 0) {
                if (own_a)
                    sum_dense<kSoft, true>(stage, ax, ay, az, eps2, lane, acc_a);
                else
                    sum_dense<kSoft, false>(stage, ax, ay, az, eps2, -1, acc_a);
            } else {
                if (own_a)
                    sum_sparse<kSoft, true>(stage, lk, sub, ax, ay, az, eps2, tsub, acc_a);
                else
                    sum_sparse<kSoft, false>(stage, lk, sub, ax, ay, az, eps2, -1, acc_a);
            }
        }
        // combine the lanes of a target (sparse items), in a fixed order
        for (int o = 1; o < kl; o <<= 1) acc_a += __shfl_xor(acc_a, o);
        const float pa = (float)(-acc_a), pb = (float)(-acc_b);
        if (va && sub == 0) phi[ia] = pa;
        if (vb) phi[ib] = pb;
        // minimum of the item's targets
        float v = __builtin_inff();
        int idx = 0x7fffffff;
        if (va && sub == 0) {
            v = pa;
            idx = ia;
        }
        if (vb && better(pb, ib, v, idx)) {
            v = pb;
            idx = ib;
        }
        // every lane holds the same minimum: all store it (one address)
        const MinIdx m = wave_argmin(v, idx);
        partial[slot] = make_int2(__float_as_int(m.v), m.i);
    }
    if (bad && lane == 0) atomicOr(&hdr->flags, (uint32_t)SR_FLAG_QUEUE);
}

// Per halo: the best of its items' minima (one wave per halo).
__global__ __launch_bounds__(256) void k_centre_argmin(const int2 *__restrict__ partial,
                                                       const int *__restrict__ hbase, int n_halos,
                                                       int64_t *__restrict__ mbp,
                                                       float *__restrict__ phi_min)
{
    const int lane = threadIdx.x & 63;
    const int h = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (h >= n_halos) return;  // whole waves leave together
    const int a = hbase[h], b = hbase[h + 1];
    float v = __builtin_inff();
    int idx = 0x7fffffff;
    for (int s = a + lane; s < b; s += 64) {
        const int2 p = partial[s];
        const float w = __int_as_float(p.x);
        if (better(w, p.y, v, idx)) {
            v = w;
            idx = p.y;
        }
    }
    const MinIdx m = wave_argmin(v, idx);
    if (lane == 0) {
        const bool found = a < b && m.i != 0x7fffffff;  // none when every phi is NaN
        mbp[h] = found ? (int64_t)m.i : -1;
        if (phi_min) phi_min[h] = found ? m.v : 0.f;
    }
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace
}  // namespace sr

using namespace sr;

struct sr_centres_plan {
    int32_t H = 0;
    int64_t n = 0;
    int64_t n_items = 0;
    size_t off_hoff = 0, off_hbase = 0, off_items = 0, off_partial = 0, upload_bytes = 0, ws_bytes = 0;
    std::vector<char> image;  // header + hoff + hbase + items, uploaded by every run
    char *pinned = nullptr;   // its pinned copy, made by the first run
    int num_cu = 0;
};

namespace {

int device_cus()
{
    int dev = 0, cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cu;
}

}  // namespace

extern "C" {

sr_status sr_centres_plan_create(int32_t n_halos, const int64_t *offsets, sr_centres_plan **plan,
                                 size_t *ws_bytes)
{
    if (!plan || !ws_bytes || !offsets || n_halos < 1 || n_halos > (1 << 26)) return SR_E_ARG;
    *plan = nullptr;
    if (offsets[0] != 0) return SR_E_ARG;
    for (int h = 0; h < n_halos; ++h)
        if (offsets[h + 1] < offsets[h]) return SR_E_ARG;
    const int64_t n = offsets[n_halos];
    if (n > (int64_t(1) << 31) - 1) return SR_E_UNSUPPORTED;
    // items of each halo: up to 128 targets (two per lane), a last group of at
    // most 64 one per lane, halos under 64 with 2^lk lanes per target
    struct Item {
        int h, t0, nt, w;
        double cost;
    };
    std::vector<Item> items;
    std::vector<int> hbase(n_halos + 1, 0);
    for (int h = 0; h < n_halos; ++h) {
        const int64_t nh = offsets[h + 1] - offsets[h];
        int chunk = 0;
        for (int64_t t = 0; t < nh;) {
            const int64_t left = nh - t;
            const int nt = (int)std::min<int64_t>(left, left > kTargetsPerWave ? 2 * kTargetsPerWave
                                                                              : kTargetsPerWave);
            int lk = 0;
            while ((nt << (lk + 1)) <= kTargetsPerWave) ++lk;
            const int two = nt > kTargetsPerWave ? 1 : 0;
            items.push_back(Item{h, (int)(offsets[h] + t), nt, lk | (two << 4), 0.0});
            items.back().cost = (double)nh * (two ? 2.0 : 1.0) / (double)(1 << lk);
            t += nt;
            ++chunk;
        }
        hbase[h + 1] = hbase[h] + chunk;
    }
    if (items.size() > (size_t(1) << 26)) return SR_E_UNSUPPORTED;
    // slot = position of the item inside its halo's range, fixed before sorting
    for (size_t k = 0, h = 0, c = 0; k < items.size(); ++k) {
        if ((int)h != items[k].h) {
            h = items[k].h;
            c = 0;
        }
        items[k].w |= (int)(hbase[h] + c) << 5;
        ++c;
    }
    std::stable_sort(items.begin(), items.end(), [](const Item &a, const Item &b) { return a.cost > b.cost; });
    auto *P = new sr_centres_plan;
    P->H = n_halos;
    P->n = n;
    P->n_items = (int64_t)items.size();
    size_t o = align256(sizeof(CentreHeader));
    P->off_hoff = o;
    o = align256(o + sizeof(int) * (n_halos + 1));
    P->off_hbase = o;
    o = align256(o + sizeof(int) * (n_halos + 1));
    P->off_items = o;
    o = align256(o + sizeof(int4) * std::max<size_t>(1, items.size()));
    P->upload_bytes = o;
    P->off_partial = o;
    o = align256(o + sizeof(int2) * std::max<size_t>(1, items.size()));
    P->ws_bytes = o;
    P->image.assign(P->upload_bytes, 0);
    int *hoff = reinterpret_cast<int *>(P->image.data() + P->off_hoff);
    for (int h = 0; h <= n_halos; ++h) hoff[h] = (int)offsets[h];
    std::memcpy(P->image.data() + P->off_hbase, hbase.data(), sizeof(int) * (n_halos + 1));
    int4 *it = reinterpret_cast<int4 *>(P->image.data() + P->off_items);
    for (size_t k = 0; k < items.size(); ++k) it[k] = make_int4(items[k].h, items[k].t0, items[k].nt, items[k].w);
    *plan = P;
    *ws_bytes = P->ws_bytes;
    return SR_OK;
}

sr_status sr_centres_plan_destroy(sr_centres_plan *P)
{
    if (!P) return SR_E_PLAN;
    if (P->pinned) (void)hipHostFree(P->pinned);
    delete P;
    return SR_OK;
}

sr_status sr_centres(sr_centres_plan *P, const float *pos, const float *mass, float eps, void *ws,
                     size_t ws_bytes, float *phi, int64_t *mbp, float *phi_min, void *stream)
{
    if (!P) return SR_E_PLAN;
    if (!(eps >= 0.f) || !std::isfinite(eps) || !mbp) return SR_E_ARG;
    if (P->n > 0 && (!pos || !mass || !phi)) return SR_E_ARG;
    if (!ws || reinterpret_cast<uintptr_t>(ws) % 256 != 0 || ws_bytes < P->ws_bytes) return SR_E_WORKSPACE;
    if (P->num_cu <= 0 && (P->num_cu = device_cus()) <= 0) return SR_E_DEVICE;
    if (!P->pinned) {
        if (hipHostMalloc((void **)&P->pinned, P->upload_bytes, hipHostMallocDefault) != hipSuccess) {
            P->pinned = nullptr;
            return SR_E_DEVICE;
        }
        std::memcpy(P->pinned, P->image.data(), P->upload_bytes);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    // tables and a zeroed queue counter, from pinned memory
    if (hipMemcpyAsync(w, P->pinned, P->upload_bytes, hipMemcpyHostToDevice, s) != hipSuccess)
        return SR_E_DEVICE;
    const int *hoff = reinterpret_cast<const int *>(w + P->off_hoff);
    const int *hbase = reinterpret_cast<const int *>(w + P->off_hbase);
    const int4 *items = reinterpret_cast<const int4 *>(w + P->off_items);
    int2 *partial = reinterpret_cast<int2 *>(w + P->off_partial);
    CentreHeader *hdr = reinterpret_cast<CentreHeader *>(w);
    if (P->n_items > 0) {
        const int64_t grid = std::min<int64_t>(P->n_items, (int64_t)P->num_cu * 32);
        const float eps2 = eps * eps;
        int64_t limit = INT64_MAX;
        if (const char *v = std::getenv("SR_PULL_LIMIT"))
            if (std::atoll(v) >= 0) limit = std::atoll(v);
        if (eps2 > 0.f)
            k_centre_potential<true><<<(unsigned)grid, 64, 0, s>>>(items, (uint32_t)P->n_items, hoff, pos,
                                                                 mass, eps2, phi, partial, hdr, limit);
        else
            k_centre_potential<false><<<(unsigned)grid, 64, 0, s>>>(items, (uint32_t)P->n_items, hoff, pos,
                                                                  mass, 0.f, phi, partial, hdr, limit);
        if (hipGetLastError() != hipSuccess) return SR_E_DEVICE;
    }
    k_centre_argmin<<<(unsigned)((P->H + 3) / 4), 256, 0, s>>>(partial, hbase, P->H, mbp, phi_min);
    return hipGetLastError() == hipSuccess ? SR_OK : SR_E_DEVICE;
}

}  // extern "C"
