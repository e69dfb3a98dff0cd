// Device kernels of the short-range force library, written for gfx950
// (CDNA4: 64-wide waves, 160 KB LDS per CU, 8 XCDs with private L2).
//
// Path (paper Sec. 2: accelerators sum the short-range part of the split
// force directly over particle pairs; Sec. 2.1: every block of particles is
// solved independently, active particles receiving forces and passive ones
// acting only as sources):
//
//   bin      cell index per particle (float32 rule of sr.h), stable LSD radix
//            sort of (cell, input index), cell starts, and a gather of offsets
//            from the cell centre and masses into structure-of-arrays order;
//   items    one work item per home cell and chunk of up to 64 targets,
//            grouped by cost class, heaviest first;
//   pairs    a persistent kernel: each 64-lane wave pulls items from one of
//            eight queues (one per XCD, stealing from the others when its own
//            runs dry), stages the 27 neighbour cells' particles in LDS
//            relative to the home-cell centre and sums the pair terms in
//            float32 registers; sparse cells give each target several lanes
//            and reduce them with cross-lane shuffles.
//
// Everything is integer-deterministic or summed in a fixed order: no float
// atomics, so results are bitwise reproducible run to run.
#include "sr_internal.h"

namespace sr {
namespace {

constexpr float kFar = 1.0e6f;  // position of padding sources (masked out)

// --------------------------------------------------------------- segments

struct OneSeg {
    SegParams p;
    __device__ __forceinline__ int seg_of_particle(int) const { return 0; }
    __device__ __forceinline__ int seg_of_cell(int) const { return 0; }
    __device__ __forceinline__ int seg_of_tile(int) const { return 0; }
    __device__ __forceinline__ const SegParams &get(int) const { return p; }
};

struct ManySeg {
    const SegParams *__restrict__ tab;
    int B;
    // largest s with key(s) <= x; keys are non-decreasing
    template <int kField>
    __device__ __forceinline__ int search(int x) const
    {
        int lo = 0, hi = B - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            const SegParams &s = tab[mid];
            const int key = kField == 0 ? s.part_off : (kField == 1 ? s.cell_off : s.tile_off);
            if (key <= x)
                lo = mid;
            else
                hi = mid - 1;
        }
        return lo;
    }
    __device__ __forceinline__ int seg_of_particle(int i) const { return search<0>(i); }
    __device__ __forceinline__ int seg_of_cell(int c) const { return search<1>(c); }
    __device__ __forceinline__ int seg_of_tile(int t) const { return search<2>(t); }
    __device__ __forceinline__ const SegParams &get(int s) const { return tab[s]; }
};

// --------------------------------------------------------------- binning rule

__device__ __forceinline__ float cell_centre(int i, float lo, float h)
{
#pragma clang fp contract(off)
    const float t = (float)i + 0.5f;
    const float c = t * h;
    return lo + c;
}

// One coordinate of the binning rule of sr.h (float32, no fused operations).
__device__ __forceinline__ int bin_coord(float x, float lo, float len, float inv_len, float h,
                                         float inv_h, int nc, int periodic, float &off,
                                         uint32_t &fl)
{
#pragma clang fp contract(off)
    const bool fin = __builtin_isfinite(x);
    if (!fin) fl |= SR_FLAG_NONFINITE;
    float w, u;
    if (periodic) {
        const float k = floorf(x * inv_len);
        const float p = k * len;
        w = x - p;
        u = w;
    } else {
        w = x;
        u = x - lo;
    }
    const float fi = floorf(u * inv_h);
    int i;
    if (!(fi >= 0.0f)) {
        i = 0;
        if (!periodic && fin) fl |= SR_FLAG_OUT_OF_DOMAIN;
    } else if (fi > (float)(nc - 1)) {
        i = nc - 1;
        if (!periodic && fin) fl |= SR_FLAG_OUT_OF_DOMAIN;
    } else {
        i = (int)fi;
    }
    off = w - cell_centre(i, lo, h);
    return i;
}

// Neighbour j = i + d in one dimension: false if outside an open domain.
// shift = centre of the neighbour's image minus centre(i).  Across a periodic
// face the box length is taken off whichever centre lies in the upper half of
// the box, a subtraction that is exact (Sterbenz), so no coordinate of
// magnitude len is ever rounded.
__device__ __forceinline__ bool neighbour(int i, int d, int nc, float lo, float h, float len,
                                          int periodic, int &j, float &shift)
{
#pragma clang fp contract(off)
    j = i + d;
    float cj, ci;
    if (j < 0) {
        if (!periodic) return false;
        j += nc;
        cj = cell_centre(j, lo, h) - len;
        ci = cell_centre(i, lo, h);
    } else if (j >= nc) {
        if (!periodic) return false;
        j -= nc;
        cj = cell_centre(j, lo, h);
        ci = cell_centre(i, lo, h) - len;
    } else {
        cj = cell_centre(j, lo, h);
        ci = cell_centre(i, lo, h);
    }
    shift = cj - ci;
    return true;
}

__device__ __forceinline__ void decode_cell(const SegParams &S, int cell, int &ix, int &iy, int &iz)
{
    const int local = cell - S.cell_off;
    iz = local % S.nc[2];
    const int r = local / S.nc[2];
    iy = r % S.nc[1];
    ix = r / S.nc[1];
}

// --------------------------------------------------------------- utilities

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t fill_u32(void *p, int64_t n, uint32_t v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    k_fill_u32<<<(unsigned)((n + 255) / 256), 256, 0, st>>>((uint32_t *)p, n, v);
    return hipGetLastError();
}

// Exclusive scan over a 256-thread block; returns this thread's prefix and
// the block total.  lds: 4 ints.
__device__ __forceinline__ int block_excl_scan(int v, int &total, int *lds)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63) lds[w] = x;
    __syncthreads();
    int woff = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int s = lds[k];
        if (k < w) woff += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return woff + x - v;
}

constexpr int kScanItems = kScanBlock / 256;

__global__ __launch_bounds__(256) void k_scan_reduce(const int *__restrict__ in, int64_t m,
                                                     int *__restrict__ sums)
{
    __shared__ int lds[4];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * kScanItems;
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < m) s += in[base + k];
    int total;
    block_excl_scan(s, total, lds);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// out[i] = offs[block] + sum_{k<i in block} in[k]; the last block also writes out[m].
__global__ __launch_bounds__(256) void k_scan_apply(const int *__restrict__ in, int64_t m,
                                                    const int *__restrict__ offs,
                                                    int *__restrict__ out)
{
    __shared__ int lds[4];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < m) ? in[base + k] : 0;
        s += v[k];
    }
    int total;
    int run = block_excl_scan(s, total, lds) + (offs ? offs[blockIdx.x] : 0);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < m) out[base + k] = run;
        run += v[k];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0)
        out[m] = (offs ? offs[blockIdx.x] : 0) + total;
}

// Exclusive scan of in[0..m) into out[0..m] (out[m] = total).  tmp holds
// scan_scratch_elems(m) ints.
hipError_t scan_i32(const int *in, int *out, int64_t m, int *tmp, hipStream_t st)
{
    const int64_t nb = (m + kScanBlock - 1) / kScanBlock;
    if (nb <= 1) {
        k_scan_apply<<<1, 256, 0, st>>>(in, m, nullptr, out);
        return hipGetLastError();
    }
    int *sums = tmp;
    int *sums_x = tmp + nb;
    int *next = sums_x + nb + 1;
    k_scan_reduce<<<(unsigned)nb, 256, 0, st>>>(in, m, sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = scan_i32(sums, sums_x, nb, next, st);
    if (e != hipSuccess) return e;
    k_scan_apply<<<(unsigned)nb, 256, 0, st>>>(in, m, sums_x, out);
    return hipGetLastError();
}

// --------------------------------------------------------------- A1: cell index

// Leaf code of one particle: the path from the cell to its sub-cell of an
// octree of the given depth, three bits (x, y, z) per level, the first level
// on top.  Each level takes the signs of the offsets from the current
// sub-cell's centre, then moves that centre a quarter of the current side
// towards the particle.  Only float32 subtractions, halvings and sign tests.
__device__ __forceinline__ int leaf_code(float ox, float oy, float oz, const SegParams &S)
{
    float qx = S.h[0] * 0.25f, qy = S.h[1] * 0.25f, qz = S.h[2] * 0.25f;
    int bx = ox >= 0.f, by = oy >= 0.f, bz = oz >= 0.f;
    int code = (bx << 2) | (by << 1) | bz;
    for (int l = 1; l < S.leaf_depth; ++l) {
        ox = bx ? ox - qx : ox + qx;
        oy = by ? oy - qy : oy + qy;
        oz = bz ? oz - qz : oz + qz;
        qx *= 0.5f;
        qy *= 0.5f;
        qz *= 0.5f;
        bx = ox >= 0.f;
        by = oy >= 0.f;
        bz = oz >= 0.f;
        code = (code << 3) | (bx << 2) | (by << 1) | bz;
    }
    return code;
}

// Cell of each particle and its sort key: (cell, passive, leaf code).  With
// key_bits == code_bits there is no passive bit (every particle is active).
// The offsets from the cell centre and the mass are kept in input order, one
// float4 per particle, for the gather into binned order.
template <class Acc>
__global__ __launch_bounds__(256) void k_bin_cells(Acc acc, const float *__restrict__ pos,
                                                   const float *__restrict__ mass, int N,
                                                   int key_bits, int code_bits, int *__restrict__ cell_of,
                                                   int *__restrict__ skey, float4 *__restrict__ packed,
                                                   uint32_t *hdr)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const SegParams &S = acc.get(acc.seg_of_particle(i));
    uint32_t fl = 0;
    float ox, oy, oz;
    const int64_t p = 3 * (int64_t)i;
    const int ix = bin_coord(pos[p], S.lo[0], S.len[0], S.inv_len[0], S.h[0], S.inv_h[0], S.nc[0],
                             S.periodic, ox, fl);
    const int iy = bin_coord(pos[p + 1], S.lo[1], S.len[1], S.inv_len[1], S.h[1], S.inv_h[1],
                             S.nc[1], S.periodic, oy, fl);
    const int iz = bin_coord(pos[p + 2], S.lo[2], S.len[2], S.inv_len[2], S.h[2], S.inv_h[2],
                             S.nc[2], S.periodic, oz, fl);
    const int cell = S.cell_off + (ix * S.nc[1] + iy) * S.nc[2] + iz;
    const int code = leaf_code(ox, oy, oz, S);
    const int passive = (i - S.part_off < S.n_active) ? 0 : 1;
    cell_of[i] = cell;
    skey[i] = (cell << key_bits) | (key_bits > code_bits ? passive << code_bits : 0) | code;
    packed[i] = make_float4(ox, oy, oz, mass[i]);
    if (fl) atomicOr(&hdr[kHdrFlags], fl);
}

// Cell starts from the sorted cell keys: slot b starts every cell in
// (key[b-1], key[b]]; slot N closes the list.  Each entry is written once.
__global__ __launch_bounds__(256) void k_cell_bounds(const int *__restrict__ key, int N, int NC,
                                                     int key_bits, int *__restrict__ start)
{
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b > N) return;
    const int lo = (b == 0) ? -1 : (key[b - 1] >> key_bits);
    const int hi = (b == N) ? NC : (key[b] >> key_bits);
    for (int c = lo + 1; c <= hi; ++c) start[c] = b;
}

// --------------------------------------------------------------- A2: stable radix sort

// Digit histogram of one tile: table[d * ntiles + tile].
__global__ __launch_bounds__(256) void k_radix_hist(const int *__restrict__ keys, int N, int shift,
                                                    int bits, int *__restrict__ table, int ntiles)
{
    __shared__ int h[256];
    const int R = 1 << bits;
    for (int d = threadIdx.x; d < R; d += 256) h[d] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
    for (int e = threadIdx.x; e < kRadixTile; e += 256) {
        const int64_t k = base + e;
        if (k < N) atomicAdd(&h[(keys[k] >> shift) & (R - 1)], 1);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < R; d += 256) table[(int64_t)d * ntiles + blockIdx.x] = h[d];
}

// Stable scatter of one tile of kRadixTile elements by four waves.  Each
// wave ranks its quarter of the tile (consecutive elements, 64 at a time)
// with one ballot per digit bit and per-wave digit counters.  The tile is then
// reordered by digit in LDS, keeping input order inside a digit (wave, then
// step, then lane), and written out in that order: each digit's run of the
// tile lands on consecutive global addresses.
constexpr int kScatterWaves = 4;
constexpr int kScatterSteps = kRadixTile / (kScatterWaves * kWave);

__global__ __launch_bounds__(kScatterWaves * kWave) void k_radix_scatter(
    const int *__restrict__ keys_in, const int *__restrict__ vals_in, int N, int shift, int bits,
    const int *__restrict__ table_x, int ntiles, int *__restrict__ keys_out, int *__restrict__ vals_out)
{
    constexpr int kThreads = kScatterWaves * kWave;
    __shared__ int cnt[kScatterWaves][256];  // per-wave digit counts, then per-wave offsets
    __shared__ int lstart[256];              // first slot of each digit in the reordered tile
    __shared__ int gstart[256];              // first global slot of each digit of this tile
    __shared__ int wsum[kScatterWaves];
    __shared__ int lkey[kRadixTile];
    __shared__ int lval[kRadixTile];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int R = 1 << bits;
    const int tile = blockIdx.x;
    gstart[tid] = tid < R ? table_x[(int64_t)tid * ntiles + tile] : 0;
#pragma unroll
    for (int w = 0; w < kScatterWaves; ++w) cnt[w][tid] = 0;
    __syncthreads();
    const int64_t tile0 = (int64_t)tile * kRadixTile;
    const int64_t base = tile0 + (int64_t)wv * (kScatterSteps * kWave);
    const uint64_t below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    int key[kScatterSteps], val[kScatterSteps], rk[kScatterSteps];
#pragma unroll
    for (int r = 0; r < kScatterSteps; ++r) {
        const int64_t e = base + r * kWave + lane;
        const bool valid = e < N;
        key[r] = valid ? keys_in[e] : 0;
        val[r] = valid ? (vals_in ? vals_in[e] : (int)e) : 0;
        const int d = (key[r] >> shift) & (R - 1);
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < bits; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const int rank = __popcll(peers & below);
        const int before = cnt[wv][d];
        rk[r] = valid ? before + rank : -1;
        __syncthreads();
        if (valid && rank == 0) cnt[wv][d] = before + __popcll(peers);
        __syncthreads();
    }
    // per-wave offsets inside each digit, and the digit totals
    int tot = 0;
#pragma unroll
    for (int w = 0; w < kScatterWaves; ++w) {
        const int c = cnt[w][tid];
        cnt[w][tid] = tot;
        tot += c;
    }
    // exclusive scan of the totals over the 256 digits (one per thread)
    int incl = tot;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    if (lane == kWave - 1) wsum[wv] = incl;
    __syncthreads();
    int prior = 0;
#pragma unroll
    for (int w = 0; w < kScatterWaves; ++w) prior += w < wv ? wsum[w] : 0;
    lstart[tid] = prior + incl - tot;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kScatterSteps; ++r) {
        if (rk[r] >= 0) {
            const int d = (key[r] >> shift) & (R - 1);
            const int at = lstart[d] + cnt[wv][d] + rk[r];
            lkey[at] = key[r];
            lval[at] = val[r];
        }
    }
    __syncthreads();
    const int n_tile = (int)min((int64_t)kRadixTile, (int64_t)N - tile0);
    for (int i = tid; i < n_tile; i += kThreads) {
        const int k = lkey[i];
        const int d = (k >> shift) & (R - 1);
        const int dest = gstart[d] + (i - lstart[d]);
        if (keys_out) keys_out[dest] = k;
        vals_out[dest] = lval[i];
    }
}

// --------------------------------------------------------------- A3: gather

// Binned order: slot b takes particle perm[b]'s offsets and mass (the float4
// the cell pass kept, one cache line per particle), its output row (-1 for a
// passive particle), and the last active slot of each cell records the cell's
// active count.  Slot 0 tags the workspace as binned for these sizes.
template <class Acc>
__global__ __launch_bounds__(256) void k_gather(Acc acc, int N, const int *__restrict__ perm,
                                                const int *__restrict__ key,
                                                const int *__restrict__ start,
                                                const float4 *__restrict__ packed,
                                                float *__restrict__ bx, float *__restrict__ by,
                                                float *__restrict__ bz, float *__restrict__ bm,
                                                int *__restrict__ out_row, int *__restrict__ nact,
                                                int key_bits, uint32_t *hdr, uint32_t magic)
{
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b == 0) hdr[kHdrMagic] = magic;
    if (b >= N) return;
    const int i = perm[b];
    const SegParams &S = acc.get(acc.seg_of_particle(i));
    const float4 v = packed[i];  // offsets from the cell centre and mass, from k_bin_cells
    bx[b] = v.x;
    by[b] = v.y;
    bz[b] = v.z;
    const float mi = v.w;
    bm[b] = mi;
    if (!(mi == packed[0].w)) atomicOr(&hdr[kHdrMassInfo], 1u);  // not every mass equal
    const int li = i - S.part_off;
    const bool act = li < S.n_active;
    out_row[b] = act ? S.out_off + li : -1;
    // active particles lead their cell (input order): the last one records the count
    if (act) {
        const int c = key[b] >> key_bits;
        bool last = (b + 1 == N) || (key[b + 1] >> key_bits) != c;
        if (!last) last = !(perm[b + 1] - S.part_off < S.n_active);
        if (last) nact[c] = b + 1 - start[c];
    }
}

// Cotangent rows in binned order (zero on passive particles).
__global__ __launch_bounds__(256) void k_gather_g(int N, int n_rows,
                                                  const int *__restrict__ out_row,
                                                  const float *__restrict__ g,
                                                  float *__restrict__ gx, float *__restrict__ gy,
                                                  float *__restrict__ gz)
{
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= N) return;
    const int r = out_row[b];
    float x = 0.f, y = 0.f, z = 0.f;
    if (r >= 0 && r < n_rows) {
        const int64_t q = 3 * (int64_t)r;
        x = g[q];
        y = g[q + 1];
        z = g[q + 2];
    }
    gx[b] = x;
    gy[b] = y;
    gz[b] = z;
}

// --------------------------------------------------------------- work items

// Items of a home cell with nt targets.  A cell of fewer than 64 targets is cut
// into items of at most `group` consecutive targets (leaf order), each with
// 2^lk lanes per target: a smaller group has a tighter box, so fewer of the
// sources it stages lie out of reach of its targets.  A larger cell is cut into
// items of 64 targets (128, two per lane, with `two`; then a last 64 when an
// odd number of 64s remain), and its last nt mod 64 targets are cut the same
// way as a small cell, so no item runs with mostly idle lanes.  Every target
// is summed in the same order whether or not `two` is set.

__device__ __forceinline__ int lanes_log2(int n)
{
    return n >= kTargetsPerItem ? 0 : (31 - __clz(kTargetsPerItem / n));
}

__device__ __forceinline__ int cell_items(int nt, bool two, int group)
{
    if (nt < kTargetsPerItem) return (nt + group - 1) / group;
    const int r = nt % kTargetsPerItem, groups = nt / kTargetsPerItem;
    const int dense = two ? (groups + 1) / 2 : groups;
    return dense + (r + group - 1) / group;
}

// Work item: x = home cell, y = first target slot, z = targets,
// w = lk | two << 3 | psrc << 4 | nd << 5 | seg << 6 (lk: log2 lanes per
// target; two: two targets per lane; psrc: the targets are passive and their
// sources are the active particles of the 27 cells only; nd: symmetric tiles
// run, the targets are non-dense and their sources here are only the
// non-dense particles of the 27 cells, the pairs with a dense particle being
// summed by the symmetric tiles; seg: the problem of a batch).
__device__ __forceinline__ int item_word(int lk, int two, int psrc, int seg, int nd = 0)
{
    return lk | (two << 3) | (psrc << 4) | (nd << 5) | (seg << 6);
}
__device__ __forceinline__ int item_lk(int w) { return w & 7; }
__device__ __forceinline__ bool item_two(int w) { return (w >> 3) & 1; }
__device__ __forceinline__ bool item_psrc(int w) { return (w >> 4) & 1; }
__device__ __forceinline__ bool item_nd(int w) { return (w >> 5) & 1; }
__device__ __forceinline__ int item_seg(int w) { return w >> 6; }

// Dense part of a cell with na active particles: its full blocks of 64 (the
// leading active particles), none when it has fewer than 64.  Dense blocks
// are the targets of the symmetric tiles.
__device__ __forceinline__ int dense_count(int na) { return na >= kWave ? (na & ~(kWave - 1)) : 0; }

// Items of a run of nt consecutive targets from slot s0 (the cut described
// above, groups of at most `group` targets); returns the number written,
// cell_items(nt, two, group).
__device__ __forceinline__ int write_run(int4 *__restrict__ items, uint32_t at, int c, int s0, int nt,
                                         bool two, int seg, int psrc, int nd, int group)
{
    if (nt <= 0) return 0;
    int k = 0;
    if (nt < kTargetsPerItem) {
        for (int t = 0; t < nt; t += group, ++k) {
            const int cn = min(group, nt - t);
            items[at + k] = make_int4(c, s0 + t, cn, item_word(lanes_log2(cn), 0, psrc, seg, nd));
        }
        return k;
    }
    const int r = nt % kTargetsPerItem, dense_end = nt - r;
    for (int t0 = 0; t0 < dense_end; ++k) {
        const int cn = (two && dense_end - t0 >= 2 * kTargetsPerItem) ? 2 * kTargetsPerItem : kTargetsPerItem;
        items[at + k] = make_int4(c, s0 + t0, cn, item_word(0, cn > kTargetsPerItem ? 1 : 0, psrc, seg, nd));
        t0 += cn;
    }
    for (int t = dense_end; t < nt; t += group, ++k) {
        const int cn = min(group, nt - t);
        items[at + k] = make_int4(c, s0 + t, cn, item_word(lanes_log2(cn), 0, psrc, seg, nd));
    }
    return k;
}

// Cost of the widest item of a run of nt targets that sees src sources:
// pairs one lane evaluates.
__device__ __forceinline__ int64_t run_cost(int nt, int64_t src, bool two, int group)
{
    if (nt <= 0) return 0;
    const int lk = nt >= kTargetsPerItem ? 0 : lanes_log2(min(nt, group));
    const int chunk = (two && nt > kTargetsPerItem) ? 2 * kTargetsPerItem : kTargetsPerItem;
    return ((src + (1 << lk) - 1) >> lk) * (chunk / kTargetsPerItem);
}

// Per home cell: number of items and cost class (floor log2 of the pairs one
// lane evaluates); counts items per class.  The forward takes the cell's
// active targets against every source of the 27 cells.  The adjoint also
// takes its passive targets, as items of their own whose sources are only
// the active particles of the 27 cells: a pair of two passive particles has
// u = m_k g_j - m_j g_k = 0, so it adds exactly nothing.
template <class Acc, bool kActiveOnly>
__device__ __forceinline__ void items_count_cell(const Acc &acc, int c, int NC,
                                                 const int *__restrict__ start,
                                                 const int *__restrict__ nact,
                                                 uint32_t *__restrict__ info, uint32_t *blk,
                                                 bool ok, int N, bool two, bool sym, int group)
{
    if (c >= NC) return;
    if (!ok) {
        info[c] = 0;
        return;
    }
    const int na = nact[c];
    const int np = kActiveOnly ? 0 : (start[c + 1] - start[c]) - na;
    if (na < 0 || np < 0 || na + np <= 0 || na + np > N) {
        info[c] = 0;
        return;
    }
    const SegParams &S = acc.get(acc.seg_of_cell(c));
    int ix, iy, iz;
    decode_cell(S, c, ix, iy, iz);
    int64_t src = 0, src_act = 0, src_nd = 0, src_act_nd = 0;
    for (int dx = -1; dx <= 1; ++dx) {
        int jx = ix + dx;
        if (jx < 0 || jx >= S.nc[0]) {
            if (!S.periodic) continue;
            jx = (jx + S.nc[0]) % S.nc[0];
        }
        for (int dy = -1; dy <= 1; ++dy) {
            int jy = iy + dy;
            if (jy < 0 || jy >= S.nc[1]) {
                if (!S.periodic) continue;
                jy = (jy + S.nc[1]) % S.nc[1];
            }
            for (int dz = -1; dz <= 1; ++dz) {
                int jz = iz + dz;
                if (jz < 0 || jz >= S.nc[2]) {
                    if (!S.periodic) continue;
                    jz = (jz + S.nc[2]) % S.nc[2];
                }
                const int cc = S.cell_off + (jx * S.nc[1] + jy) * S.nc[2] + jz;
                src += start[cc + 1] - start[cc];
                if (np > 0) src_act += nact[cc];
                if (sym) {
                    src_nd += start[cc + 1] - start[cc] - dense_count(nact[cc]);
                    src_act_nd += nact[cc] - dense_count(nact[cc]);
                }
            }
        }
    }
    // cost class from the cell's widest item: a group of min(nt, group) targets when sparse.
    // With symmetric tiles the dense blocks have no item here, and the other
    // targets take only the non-dense sources (the symmetric tiles give them
    // the terms of the dense ones)
    const int dn = sym ? dense_count(na) : 0;
    const int n_items = cell_items(na - dn, two, group) + cell_items(np, two, group);
    int64_t cost = sym ? max(run_cost(na - dn, src_nd, two, group), run_cost(np, src_act_nd, two, group))
                       : max(run_cost(na, src, two, group), run_cost(np, src_act, two, group));
    if (cost < 1) cost = 1;
    int cls = 63 - __clzll((unsigned long long)cost);
    cls = cls > 31 ? 31 : cls;
    info[c] = ((uint32_t)n_items << 5) | (uint32_t)cls;
    // per-block class totals, one global atomic per class and block
    atomicAdd(&blk[cls], (uint32_t)n_items);
}

template <class Acc, bool kActiveOnly>
__global__ __launch_bounds__(256) void k_items_count(Acc acc, int NC, const int *__restrict__ start,
                                                     const int *__restrict__ nact,
                                                     uint32_t *__restrict__ info, uint32_t *hdr,
                                                     uint32_t magic, int N, int two, int group)
{
    __shared__ uint32_t blk[kClasses];
    if (threadIdx.x < kClasses) blk[threadIdx.x] = 0;
    __syncthreads();
    const bool ok = hdr[kHdrMagic] == magic;
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (!ok && c == 0) atomicOr(&hdr[kHdrFlags], (uint32_t)SR_FLAG_NOT_BINNED);
    items_count_cell<Acc, kActiveOnly>(acc, c, NC, start, nact, info, blk, ok, N, two != 0,
                                       hdr[kHdrSymOk] != 0, group);
    __syncthreads();
    if (threadIdx.x < kClasses && blk[threadIdx.x])
        atomicAdd(&hdr[kHdrBucketCount + threadIdx.x], blk[threadIdx.x]);
}

// Class bases, heaviest class first; resets cursors and queue counters.
__global__ void k_items_base(uint32_t *hdr, uint32_t magic)
{
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int cls = kClasses - 1; cls >= 0; --cls) {
            hdr[kHdrBucketBase + cls] = run;
            run += hdr[kHdrBucketCount + cls];
        }
        hdr[kHdrNItems] = hdr[kHdrMagic] == magic ? run : 0u;
    }
    if (threadIdx.x < kClasses) hdr[kHdrBucketCursor + threadIdx.x] = 0;
    if (threadIdx.x < kQueues) hdr[kHdrQueue + 32 * threadIdx.x] = 0;
}

template <class Acc, bool kActiveOnly>
__global__ __launch_bounds__(256) void k_items_write(Acc acc, int NC, const int *__restrict__ start,
                                                     const int *__restrict__ nact,
                                                     const uint32_t *__restrict__ info,
                                                     uint32_t *hdr, int4 *__restrict__ items,
                                                     int two, int group)
{
    __shared__ uint32_t cnt[kClasses];
    __shared__ uint32_t base[kClasses];
    if (threadIdx.x < kClasses) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int c = blockIdx.x * 256 + threadIdx.x;
    const uint32_t inf = c < NC ? info[c] : 0u;
    const int n_items = (int)(inf >> 5);
    const int cls = (int)(inf & 31);
    uint32_t local = 0;
    if (inf) local = atomicAdd(&cnt[cls], (uint32_t)n_items);
    __syncthreads();
    if (threadIdx.x < kClasses && cnt[threadIdx.x])
        base[threadIdx.x] = hdr[kHdrBucketBase + threadIdx.x] +
                            atomicAdd(&hdr[kHdrBucketCursor + threadIdx.x], cnt[threadIdx.x]);
    __syncthreads();
    if (!inf) return;
    const int na = nact[c];
    const int nt = start[c + 1] - start[c];
    const int seg = acc.seg_of_cell(c);
    const uint32_t at = base[cls] + local;
    const int s0 = start[c];
    // active targets (all sources), then for the adjoint the passive ones (active sources);
    // with symmetric tiles only the non-dense targets, against the non-dense sources
    const int sym = hdr[kHdrSymOk] != 0 ? 1 : 0;
    const int dn = sym ? dense_count(na) : 0;
    const int k = write_run(items, at, c, s0 + dn, na - dn, two, seg, 0, sym, group);
    if (!kActiveOnly) write_run(items, at + k, c, s0 + na, nt - na, two, seg, 1, sym, group);
}

// --------------------------------------------------------------- pair kernels

// The 27 neighbour cells of a home cell, one per lane (lanes 0..26): first
// binned slot, count, exclusive prefix of counts, centre shift.
struct Stencil {
    int nstart, excl;
    float sx, sy, sz;
    int total;
};

// With act_only each cell contributes only its active particles (they lead
// the cell): the sources of an item of passive targets.
// With nd each cell contributes only its non-dense particles (those after its
// dense blocks; with act_only its active ones): when symmetric tiles run, the
// pairs with a dense source are theirs.
__device__ __forceinline__ void stencil_setup(const SegParams &S, int cell,
                                              const int *__restrict__ start,
                                              const int *__restrict__ nact, bool act_only, int lane,
                                              Stencil &st, bool nd = false)
{
    int ix, iy, iz;
    decode_cell(S, cell, ix, iy, iz);
    int cnt = 0;
    st.nstart = 0;
    st.sx = st.sy = st.sz = 0.f;
    if (lane < 27) {
        const int dx = lane / 9 - 1, dy = (lane / 3) % 3 - 1, dz = lane % 3 - 1;
        int jx, jy, jz;
        const bool ok = neighbour(ix, dx, S.nc[0], S.lo[0], S.h[0], S.len[0], S.periodic, jx, st.sx) &&
                        neighbour(iy, dy, S.nc[1], S.lo[1], S.h[1], S.len[1], S.periodic, jy, st.sy) &&
                        neighbour(iz, dz, S.nc[2], S.lo[2], S.h[2], S.len[2], S.periodic, jz, st.sz);
        if (ok) {
            const int c = S.cell_off + (jx * S.nc[1] + jy) * S.nc[2] + jz;
            st.nstart = start[c];
            if (nd) {
                const int d = dense_count(nact[c]);
                st.nstart += d;
                cnt = act_only ? nact[c] - d : start[c + 1] - st.nstart;
            } else {
                cnt = act_only ? nact[c] : start[c + 1] - st.nstart;
            }
        }
    }
    int incl = cnt;
#pragma unroll
    for (int d = 1; d < 32; d <<= 1) {
        const int y = __shfl_up(incl, d);
        if (lane >= d) incl += y;
    }
    st.excl = incl - cnt;
    st.total = __builtin_amdgcn_readfirstlane(__shfl(incl, 26));
}

// Source v of the stencil's virtual concatenation: binned slot and shift.
// Every lane must call it (cross-lane reads); v is clamped to the last source.
__device__ __forceinline__ int stencil_locate(const Stencil &st, int v, float &sx, float &sy,
                                              float &sz)
{
    const int vv = min(v, st.total - 1);
    int q = 0;
#pragma unroll
    for (int step = 16; step >= 1; step >>= 1) {
        const int cand = q + step;
        const int e = __shfl(st.excl, min(cand, 26));
        if (cand <= 26 && e <= vv) q = cand;
    }
    sx = __shfl(st.sx, q);
    sy = __shfl(st.sy, q);
    sz = __shfl(st.sz, q);
    return __shfl(st.nstart, q) + (vv - __shfl(st.excl, q));
}

struct Src {
    const float *__restrict__ x;
    const float *__restrict__ y;
    const float *__restrict__ z;
    const float *__restrict__ m;
};

__device__ __forceinline__ float4 fetch_pos(const Stencil &st, int v, const Src &s)
{
    float sx, sy, sz;
    const int j = stencil_locate(st, v, sx, sy, sz);
    float4 r;
    r.x = s.x[j] + sx;
    r.y = s.y[j] + sy;
    r.z = s.z[j] + sz;
    r.w = s.m[j];
    if (v >= st.total) r = make_float4(kFar, kFar, kFar, 0.f);
    return r;
}

// Pull the next work item: queues are interleaved blocks of kQueueBlock
// items of the cost-ordered list; a wave drains the queue of its XCD first.
// The persistent loops that call this end their bodies without a lane-0-only
// branch: otherwise the compiler may merge that branch with this one across
// the back edge and let the other lanes start the next item without lane 0.
__device__ __forceinline__ int64_t next_item(uint32_t *hdr, int q, int lane, int qbase = kHdrQueue)
{
    uint32_t c = 0;
    if (lane == 0) c = atomicAdd(&hdr[qbase + 32 * q], 1u);
    c = __builtin_amdgcn_readfirstlane(c);
    return ((int64_t)(c / kQueueBlock) * kQueues + q) * kQueueBlock + (c % kQueueBlock);
}

// Bound of a persistent loop.  A queue hands out increasing counter values,
// so the items one wave pulls from one queue increase strictly, and no wave
// can pull more items than exist.  A pull that breaks either rule (a loop
// whose lanes lost the item lane 0 was given, or a corrupted counter) ends
// the wave's loop and flags the workspace, so the kernel exits instead of
// spinning.  limit is at most the item count; a smaller one (the host's test
// hook) ends every wave early on purpose.  All values are wave-uniform.
struct PullGuard {
    int64_t limit, pulls = 0, last = -1;
    bool bad = false;
    __device__ __forceinline__ explicit PullGuard(int64_t lim) : limit(lim) {}
    __device__ __forceinline__ void next_queue() { last = -1; }
    // false: leave the loop (bad is set)
    __device__ __forceinline__ bool accept(int64_t g)
    {
        if (g <= last || ++pulls > limit) {
            bad = true;
            return false;
        }
        last = g;
        return true;
    }
    __device__ __forceinline__ void report(uint32_t *hdr, int lane) const
    {
        if (bad && lane == 0) atomicOr(&hdr[kHdrFlags], (uint32_t)SR_FLAG_QUEUE);
    }
};

// Work item with every field wave-uniform (scalar registers).
__device__ __forceinline__ int4 load_item(const int4 *__restrict__ items, int64_t g)
{
    const int4 it = items[g];
    return make_int4(__builtin_amdgcn_readfirstlane(it.x), __builtin_amdgcn_readfirstlane(it.y),
                     __builtin_amdgcn_readfirstlane(it.z), __builtin_amdgcn_readfirstlane(it.w));
}

// The adjoint's pair terms are evaluated at this scale.
constexpr float kMinusThird = -1.0f / 3.0f;

// Returns v held in a vector register that the compiler cannot re-derive from
// its scalar source.  The first Horner step reads the two top coefficients,
// and a three-operand instruction may read only one scalar register, so with
// both coefficients in scalar registers the compiler re-copies one of them in
// every pair step; one copy per work item takes that move out of the loops.
__device__ __forceinline__ float keep_in_vgpr(float v)
{
    asm volatile("" : "+v"(v));
    return v;
}

__device__ __forceinline__ float horner5(const float *q, float t)
{
    float p = fmaf(q[5], t, q[4]);
    p = fmaf(p, t, q[3]);
    p = fmaf(p, t, q[2]);
    p = fmaf(p, t, q[1]);
    return fmaf(p, t, q[0]);
}

__device__ __forceinline__ float horner4(const float *q, float t)
{
    float p = fmaf(q[4], t, q[3]);
    p = fmaf(p, t, q[2]);
    p = fmaf(p, t, q[1]);
    return fmaf(p, t, q[0]);
}

// One forward pair term: acc += m_j d f_SR(s) for t = s + eps^2 < tc2.  With
// kUM (every mass equal) the mass is applied once to the sum instead.
template <bool kSoft, bool kUM>
__device__ __forceinline__ void force_pair(const float4 s, float px, float py, float pz, float eps2,
                                           float tc2, const float *cq, float &ax, float &ay,
                                           float &az)
{
    const float dx = s.x - px, dy = s.y - py, dz = s.z - pz;
    const float tt = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
    const float qi = __builtin_amdgcn_rsqf(tt);
    const float q2 = qi * qi;
    const float f = fmaf(q2, qi, -horner5(cq, tt));
    const bool in = kSoft ? (tt < tc2) : (tt < tc2 && tt > 0.f);
    if (in) {  // an exec mask rather than a select (f may be infinite for padding)
        const float w = kUM ? f : s.w * f;
        ax = fmaf(w, dx, ax);
        ay = fmaf(w, dy, ay);
        az = fmaf(w, dz, az);
    }
}

// One adjoint pair term: r += f u + 2 f' (u.d) d, u = m_k g_j - m_j g_k,
// at the scale -1/3 (cq, cd: the adjoint's coefficients qa, dqa): the sums
// are multiplied by -3 once per output row.  With kUM, u / m = g_j - g_k is
// summed and the mass applied at the same time.
// Both products of u are rounded before the difference (no fused form), so u
// is exactly antisymmetric and the target's own entry (j = k, d = 0) adds
// exactly zero.  A distinct particle at the same position (d = 0) adds
// f(0) u: with softening the pair force m d f(|d|^2) is smooth through
// d = 0 and this is its derivative.
template <bool kSoft, bool kUM>
__device__ __forceinline__ void vjp_pair(const float4 s, const float4 gj, float px, float py,
                                         float pz, float mk, float gkx, float gky, float gkz,
                                         float eps2, float tc2, const float *cq, const float *cd,
                                         float &rx, float &ry, float &rz)
{
#pragma clang fp contract(off)
    const float dx = s.x - px, dy = s.y - py, dz = s.z - pz;
    const float tt = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
    const float qi = __builtin_amdgcn_rsqf(tt);
    const float q2 = qi * qi;
    const float q3 = q2 * qi;
    const bool in = kSoft ? (tt < tc2) : (tt < tc2 && tt > 0.f);
    const float f = fmaf(q3, kMinusThird, horner5(cq, tt));
    const float fp2 = fmaf(q3, q2, horner4(cd, tt));
    const float ux = kUM ? gj.x - gkx : mk * gj.x - s.w * gkx;
    const float uy = kUM ? gj.y - gky : mk * gj.y - s.w * gky;
    const float uz = kUM ? gj.z - gkz : mk * gj.z - s.w * gkz;
    const float c = fp2 * fmaf(ux, dx, fmaf(uy, dy, uz * dz));
    if (in) {  // an exec mask rather than selects (f, c may be infinite for padding)
        rx = fmaf(c, dx, fmaf(f, ux, rx));
        ry = fmaf(c, dy, fmaf(f, uy, ry));
        rz = fmaf(c, dz, fmaf(f, uz, rz));
    }
}

// ------------------------------------------------------------- source culling

// Survivors staged per pass of the pair loop (plus 64 padding entries): 4 KB
// of LDS per forward wave, 6 KB per adjoint wave (two float4 per source), so
// 32 forward or 24 adjoint waves fit in a CU's 160 KB.
constexpr int kStageForce = 192;
constexpr int kStageVjp = 128;

// Bounding box of the targets an item holds (in the home-cell frame).
struct Box {
    float lx, ly, lz, hx, hy, hz;
};

__device__ __forceinline__ float wave_min(float v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fminf(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

// Box of the valid targets of this wave: lane values (xa, ya, za) when va,
// (xb, yb, zb) when vb.
__device__ __forceinline__ Box target_box(bool va, float xa, float ya, float za, bool vb, float xb,
                                          float yb, float zb)
{
    const float inf = __builtin_huge_valf();
    Box b;
    b.lx = wave_min(fminf(va ? xa : inf, vb ? xb : inf));
    b.ly = wave_min(fminf(va ? ya : inf, vb ? yb : inf));
    b.lz = wave_min(fminf(va ? za : inf, vb ? zb : inf));
    b.hx = wave_max(fmaxf(va ? xa : -inf, vb ? xb : -inf));
    b.hy = wave_max(fmaxf(va ? ya : -inf, vb ? yb : -inf));
    b.hz = wave_max(fmaxf(va ? za : -inf, vb ? zb : -inf));
    return b;
}

// A source at (x, y, z) may interact with some target of the box: its squared
// gap to the box is at most cull2 = r_s^2 (1 + 1e-5).  The margin covers the
// float32 rounding of both this test and the pair kernel's own cutoff test, so
// no pair the pair kernel would count is ever dropped.
__device__ __forceinline__ bool may_reach(const Box &b, float x, float y, float z, float cull2)
{
    const float gx = fmaxf(fmaxf(b.lx - x, x - b.hx), 0.f);
    const float gy = fmaxf(fmaxf(b.ly - y, y - b.hy), 0.f);
    const float gz = fmaxf(fmaxf(b.lz - z, z - b.hz), 0.f);
    return fmaf(gx, gx, fmaf(gy, gy, gz * gz)) <= cull2;
}

// Stream the stencil's sources through LDS.  Candidates are fetched 64 at a
// time (the next batch is prefetched into registers), sources that cannot
// reach the target box are dropped, and survivors are packed into stage0
// (and stage1 for a second float4 per source) with a ballot.  The stage holds
// kCap survivors plus 64 entries of padding; compute(n) consumes entries
// [0, n) and may read up to 63 padding entries past n, which the pair terms
// mask out (far away, zero mass).  A larger kCap means fewer, fuller passes
// of the pair loop.  Every lane must call this (wave-uniform control flow).
template <int kParts, int kCap, class Fetch, class Compute>
__device__ __forceinline__ void stream_sources(const Stencil &st, const Box &box, float cull2,
                                               int lane, float4 *stage0, float4 *stage1,
                                               Fetch &&fetch, Compute &&compute)
{
    static_assert(kCap >= kWave && kCap % kWave == 0, "stage capacity in whole waves");
    const uint64_t below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    auto flush = [&](int n) {
        stage0[n + lane] = make_float4(kFar, kFar, kFar, 0.f);
        if (kParts == 2) stage1[n + lane] = make_float4(0.f, 0.f, 0.f, 0.f);
        __syncthreads();
        compute(n);
        __syncthreads();
    };
    int fill = 0;
    float4 c0, c1;
    fetch(lane, c0, c1);
    for (int base = 0; base < st.total; base += kWave) {
        const bool keep = (base + lane < st.total) && may_reach(box, c0.x, c0.y, c0.z, cull2);
        const uint64_t m = __ballot(keep);
        const int cnt = __popcll(m);
        if (fill + cnt > kCap) {
            flush(fill);
            fill = 0;
        }
        if (keep) {
            const int at = fill + __popcll(m & below);
            stage0[at] = c0;
            if (kParts == 2) stage1[at] = c1;
        }
        fill += cnt;
        if (base + kWave < st.total) fetch(base + kWave + lane, c0, c1);
    }
    if (fill > 0) flush(fill);
}

// Source v of the stencil for the adjoint: position (shifted) and mass, and
// the binned cotangent; padding past the end is far away with zero mass.
__device__ __forceinline__ void fetch_vjp(const Stencil &st, int v, const Src &src,
                                          const float *__restrict__ gx,
                                          const float *__restrict__ gy,
                                          const float *__restrict__ gz, float4 &p, float4 &gv)
{
    float sx, sy, sz;
    const int j = stencil_locate(st, v, sx, sy, sz);
    p = make_float4(src.x[j] + sx, src.y[j] + sy, src.z[j] + sz, src.m[j]);
    gv = make_float4(gx[j], gy[j], gz[j], 0.f);
    if (v >= st.total) {
        p = make_float4(kFar, kFar, kFar, 0.f);
        gv = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

__device__ __forceinline__ void store3(float *__restrict__ out, int n_out, int r, float x, float y,
                                       float z)
{
    if (r >= 0 && r < n_out) {
        const int64_t o3 = 3 * (int64_t)r;
        out[o3] = x;
        out[o3 + 1] = y;
        out[o3 + 2] = z;
    }
}

// ------------------------------------------------------------- forward kernel

// Forward: acc[out_row] = sum over the stencil of m_j d f_SR.
//  - dense items (one target per lane): every lane reads the same staged
//    source (LDS broadcast), in groups of 8;
//  - two-target items: lanes hold t0 + lane and t0 + 64 + lane and use each
//    staged source twice;
//  - sparse items: 2^lk lanes per target stride over the sources and reduce
//    with cross-lane butterflies.
template <class Acc, bool kSoft, bool kUM>
__device__ __forceinline__ void force_items(const Acc &acc, const int4 *__restrict__ items,
                                            uint32_t *hdr, const int *__restrict__ start,
                                            const int *__restrict__ nact,
                                            const Src &src, const int *__restrict__ out_row,
                                            float *__restrict__ out, int n_out, float4 *stage,
                                            int64_t pull_limit)
{
    const int lane = threadIdx.x;
    const float m0 = kUM ? src.m[0] : 1.0f;
    const int64_t n_items = hdr[kHdrNItems];
    const int q0 = blockIdx.x & (kQueues - 1);
    PullGuard guard(min(n_items, pull_limit));
    for (int qq = 0; qq < kQueues && !guard.bad; ++qq) {
        const int q = (q0 + qq) & (kQueues - 1);
        guard.next_queue();
        for (;;) {
            const int64_t g = next_item(hdr, q, lane);
            if (g >= n_items || !guard.accept(g)) break;
            const int4 it = load_item(items, g);
            const int t0 = it.y, nt = it.z, lk = item_lk(it.w);
            const SegParams &S = acc.get(item_seg(it.w));
            const float eps2 = S.pc.eps2, tc2 = S.pc.tc2, cull2 = S.pc.cull2;
            float cq[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) cq[k] = S.pc.q[k];
            cq[5] = keep_in_vgpr(cq[5]);
            Stencil st;
            stencil_setup(S, it.x, start, nact, false, lane, st, item_nd(it.w));
            auto fetch_p = [&](int v, float4 &c0, float4 &) { c0 = fetch_pos(st, v, src); };
            if (item_two(it.w)) {
                const bool va = lane < nt, vb = kWave + lane < nt;
                float pax = 0.f, pay = 0.f, paz = 0.f, pbx = 0.f, pby = 0.f, pbz = 0.f;
                if (va) {
                    pax = src.x[t0 + lane];
                    pay = src.y[t0 + lane];
                    paz = src.z[t0 + lane];
                }
                if (vb) {
                    pbx = src.x[t0 + kWave + lane];
                    pby = src.y[t0 + kWave + lane];
                    pbz = src.z[t0 + kWave + lane];
                }
                const Box box = target_box(va, pax, pay, paz, vb, pbx, pby, pbz);
                float aax = 0.f, aay = 0.f, aaz = 0.f, abx = 0.f, aby = 0.f, abz = 0.f;
                stream_sources<1, kStageForce>(st, box, cull2, lane, stage, stage, fetch_p, [&](int n) {
                    const int n4 = (n + 3) >> 2;
                    for (int u = 0; u < n4; ++u) {
#pragma unroll
                        for (int q4 = 0; q4 < 4; ++q4) {
                            const float4 sj = stage[4 * u + q4];
                            force_pair<kSoft, kUM>(sj, pax, pay, paz, eps2, tc2, cq, aax, aay, aaz);
                            force_pair<kSoft, kUM>(sj, pbx, pby, pbz, eps2, tc2, cq, abx, aby, abz);
                        }
                    }
                });
                if (va) store3(out, n_out, out_row[t0 + lane], m0 * aax, m0 * aay, m0 * aaz);
                if (vb) store3(out, n_out, out_row[t0 + kWave + lane], m0 * abx, m0 * aby, m0 * abz);
                continue;
            }
            const int kl = 1 << lk;
            const int t = lane >> lk, sub = lane & (kl - 1);
            const bool tv = t < nt;
            float px = 0.f, py = 0.f, pz = 0.f;
            if (tv) {
                px = src.x[t0 + t];
                py = src.y[t0 + t];
                pz = src.z[t0 + t];
            }
            const Box box = target_box(tv, px, py, pz, false, 0.f, 0.f, 0.f);
            float ax = 0.f, ay = 0.f, az = 0.f;
            stream_sources<1, kStageForce>(st, box, cull2, lane, stage, stage, fetch_p, [&](int n) {
                if (lk == 0) {
                    const int n8 = (n + 7) >> 3;
                    for (int u = 0; u < n8; ++u) {
#pragma unroll
                        for (int q8 = 0; q8 < 8; ++q8)
                            force_pair<kSoft, kUM>(stage[8 * u + q8], px, py, pz, eps2, tc2, cq, ax, ay, az);
                    }
                } else {
                    const int niter = (n + kl - 1) >> lk;
#pragma unroll 2
                    for (int i = 0; i < niter; ++i)
                        force_pair<kSoft, kUM>(stage[sub + (i << lk)], px, py, pz, eps2, tc2, cq, ax, ay, az);
                }
            });
            for (int o = 1; o < kl; o <<= 1) {
                ax += __shfl_xor(ax, o);
                ay += __shfl_xor(ay, o);
                az += __shfl_xor(az, o);
            }
            // every lane of a target's group holds the same sum: all store it, so the
            // loop body ends without a single-lane branch (see next_item)
            if (tv) store3(out, n_out, out_row[t0 + t], m0 * ax, m0 * ay, m0 * az);
        }
    }
    guard.report(hdr, lane);
}

template <class Acc, bool kSoft, int kOcc>
__global__ __launch_bounds__(64, kOcc > 0 ? kOcc : 1) void k_force(
    Acc acc, const int4 *__restrict__ items, uint32_t *hdr, const int *__restrict__ start,
    const int *__restrict__ nact, Src src, const int *__restrict__ out_row, float *__restrict__ out,
    int n_out, int64_t pull_limit)
{
    __shared__ float4 stage[kStageForce + kWave];
    if (hdr[kHdrMassInfo] == 0)
        force_items<Acc, kSoft, true>(acc, items, hdr, start, nact, src, out_row, out, n_out, stage, pull_limit);
    else
        force_items<Acc, kSoft, false>(acc, items, hdr, start, nact, src, out_row, out, n_out, stage, pull_limit);
}

// ------------------------------------------------------------- adjoint kernel

// Adjoint: grad[perm] = sum over the stencil of f u + 2 f' (u.d) d,
// u = m_k g_j - m_j g_k.  Same item shapes as the forward kernel; every
// source stages (x, y, z, m) and (g, 0).
template <class Acc, bool kSoft, bool kUM>
__device__ __forceinline__ void vjp_items(const Acc &acc, const int4 *__restrict__ items,
                                          uint32_t *hdr, const int *__restrict__ start,
                                          const int *__restrict__ nact, const Src &src,
                                          const float *__restrict__ gx,
                                          const float *__restrict__ gy,
                                          const float *__restrict__ gz,
                                          const int *__restrict__ perm, float *__restrict__ out,
                                          int n_out, float4 *stage_p, float4 *stage_g,
                                          int64_t pull_limit)
{
    const int lane = threadIdx.x;
    // the common mass (or 1), times -3: the pair sums are at the scale -1/3
    const float m0 = -3.0f * (kUM ? src.m[0] : 1.0f);
    const int64_t n_items = hdr[kHdrNItems];
    const int q0 = blockIdx.x & (kQueues - 1);
    PullGuard guard(min(n_items, pull_limit));
    for (int qq = 0; qq < kQueues && !guard.bad; ++qq) {
        const int q = (q0 + qq) & (kQueues - 1);
        guard.next_queue();
        for (;;) {
            const int64_t g = next_item(hdr, q, lane);
            if (g >= n_items || !guard.accept(g)) break;
            const int4 it = load_item(items, g);
            const int t0 = it.y, nt = it.z, lk = item_lk(it.w);
            const SegParams &S = acc.get(item_seg(it.w));
            const float eps2 = S.pc.eps2, tc2 = S.pc.tc2, cull2 = S.pc.cull2;
            float cq[6], cd[5];
#pragma unroll
            for (int k = 0; k < 6; ++k) cq[k] = S.pc.qa[k];
            cq[5] = keep_in_vgpr(cq[5]);
#pragma unroll
            for (int k = 0; k < 5; ++k) cd[k] = S.pc.dqa[k];
            Stencil st;
            stencil_setup(S, it.x, start, nact, item_psrc(it.w), lane, st, item_nd(it.w));
            auto fetch_pg = [&](int v, float4 &c0, float4 &c1) {
                fetch_vjp(st, v, src, gx, gy, gz, c0, c1);
            };
            if (item_two(it.w)) {
                const int ba = t0 + lane, bb = t0 + kWave + lane;
                const bool va = lane < nt, vb = kWave + lane < nt;
                float pax = 0.f, pay = 0.f, paz = 0.f, ma = 0.f, gax = 0.f, gay = 0.f, gaz = 0.f;
                float pbx = 0.f, pby = 0.f, pbz = 0.f, mb = 0.f, gbx = 0.f, gby = 0.f, gbz = 0.f;
                if (va) {
                    pax = src.x[ba]; pay = src.y[ba]; paz = src.z[ba]; ma = src.m[ba];
                    gax = gx[ba]; gay = gy[ba]; gaz = gz[ba];
                }
                if (vb) {
                    pbx = src.x[bb]; pby = src.y[bb]; pbz = src.z[bb]; mb = src.m[bb];
                    gbx = gx[bb]; gby = gy[bb]; gbz = gz[bb];
                }
                const Box box = target_box(va, pax, pay, paz, vb, pbx, pby, pbz);
                float rax = 0.f, ray = 0.f, raz = 0.f, rbx = 0.f, rby = 0.f, rbz = 0.f;
                stream_sources<2, kStageVjp>(st, box, cull2, lane, stage_p, stage_g, fetch_pg, [&](int n) {
                    const int n2 = (n + 1) >> 1;
                    for (int u = 0; u < n2; ++u) {
#pragma unroll
                        for (int q2 = 0; q2 < 2; ++q2) {
                            const float4 sp = stage_p[2 * u + q2];
                            const float4 sg = stage_g[2 * u + q2];
                            vjp_pair<kSoft, kUM>(sp, sg, pax, pay, paz, ma, gax, gay, gaz, eps2, tc2, cq,
                                            cd, rax, ray, raz);
                            vjp_pair<kSoft, kUM>(sp, sg, pbx, pby, pbz, mb, gbx, gby, gbz, eps2, tc2, cq,
                                            cd, rbx, rby, rbz);
                        }
                    }
                });
                if (va) store3(out, n_out, perm[ba], m0 * rax, m0 * ray, m0 * raz);
                if (vb) store3(out, n_out, perm[bb], m0 * rbx, m0 * rby, m0 * rbz);
                continue;
            }
            const int kl = 1 << lk;
            const int t = lane >> lk, sub = lane & (kl - 1);
            const bool tv = t < nt;
            float px = 0.f, py = 0.f, pz = 0.f, mk = 0.f, gkx = 0.f, gky = 0.f, gkz = 0.f;
            if (tv) {
                const int b = t0 + t;
                px = src.x[b];
                py = src.y[b];
                pz = src.z[b];
                mk = src.m[b];
                gkx = gx[b];
                gky = gy[b];
                gkz = gz[b];
            }
            const Box box = target_box(tv, px, py, pz, false, 0.f, 0.f, 0.f);
            float rx = 0.f, ry = 0.f, rz = 0.f;
            stream_sources<2, kStageVjp>(st, box, cull2, lane, stage_p, stage_g, fetch_pg, [&](int n) {
                if (lk == 0) {
                    const int n4 = (n + 3) >> 2;
                    for (int u = 0; u < n4; ++u) {
#pragma unroll
                        for (int q4 = 0; q4 < 4; ++q4)
                            vjp_pair<kSoft, kUM>(stage_p[4 * u + q4], stage_g[4 * u + q4], px, py, pz, mk,
                                            gkx, gky, gkz, eps2, tc2, cq, cd, rx, ry, rz);
                    }
                } else {
                    const int niter = (n + kl - 1) >> lk;
                    for (int i = 0; i < niter; ++i) {
                        const int e = sub + (i << lk);
                        vjp_pair<kSoft, kUM>(stage_p[e], stage_g[e], px, py, pz, mk, gkx, gky, gkz, eps2,
                                        tc2, cq, cd, rx, ry, rz);
                    }
                }
            });
            for (int o = 1; o < kl; o <<= 1) {
                rx += __shfl_xor(rx, o);
                ry += __shfl_xor(ry, o);
                rz += __shfl_xor(rz, o);
            }
            if (tv) store3(out, n_out, perm[t0 + t], m0 * rx, m0 * ry, m0 * rz);
        }
    }
    guard.report(hdr, lane);
}

template <class Acc, bool kSoft, int kOcc>
__global__ __launch_bounds__(64, kOcc > 0 ? kOcc : 1) void k_vjp(
    Acc acc, const int4 *__restrict__ items, uint32_t *hdr, const int *__restrict__ start,
    const int *__restrict__ nact, Src src, const float *__restrict__ gx,
    const float *__restrict__ gy, const float *__restrict__ gz, const int *__restrict__ perm,
    float *__restrict__ out, int n_out, int64_t pull_limit)
{
    __shared__ float4 stage_p[kStageVjp + kWave];
    __shared__ float4 stage_g[kStageVjp + kWave];
    if (hdr[kHdrMassInfo] == 0)
        vjp_items<Acc, kSoft, true>(acc, items, hdr, start, nact, src, gx, gy, gz, perm, out, n_out,
                                    stage_p, stage_g, pull_limit);
    else
        vjp_items<Acc, kSoft, false>(acc, items, hdr, start, nact, src, gx, gy, gz, perm, out, n_out,
                                     stage_p, stage_g, pull_limit);
}

// Ordered pairs (target, source) with 0 < s < r_s^2 over the items of one
// pass, decided exactly as in the pair kernels: with the forward items the
// pairs of an active target, with the adjoint items the pairs with at least
// one active end.
template <class Acc>
__global__ __launch_bounds__(64) void k_count(Acc acc, const int4 *__restrict__ items,
                                              uint32_t *hdr, const int *__restrict__ start,
                                              const int *__restrict__ nact, Src src,
                                              int64_t pull_limit)
{
    __shared__ float4 stage[kWave];
    const int lane = threadIdx.x;
    const int64_t n_items = hdr[kHdrNItems];
    const int q0 = blockIdx.x & (kQueues - 1);
    unsigned long long pairs = 0;
    PullGuard guard(min(n_items, pull_limit));
    for (int qq = 0; qq < kQueues && !guard.bad; ++qq) {
        const int q = (q0 + qq) & (kQueues - 1);
        guard.next_queue();
        for (;;) {
            const int64_t g = next_item(hdr, q, lane);
            if (g >= n_items || !guard.accept(g)) break;
            const int4 it = load_item(items, g);
            const int t0 = it.y, nt = it.z, lk = item_lk(it.w);
            const SegParams &S = acc.get(item_seg(it.w));
            const float eps2 = S.pc.eps2, tc2 = S.pc.tc2;
            Stencil st;
            stencil_setup(S, it.x, start, nact, item_psrc(it.w), lane, st);
            const int kl = 1 << lk;
            const int t = lane >> lk, sub = lane & (kl - 1);
            const bool tv = t < nt;
            float px = 0.f, py = 0.f, pz = 0.f;
            if (tv) {
                px = src.x[t0 + t];
                py = src.y[t0 + t];
                pz = src.z[t0 + t];
            }
            unsigned cnt_lane = 0;
            float4 nxt = fetch_pos(st, lane, src);
            for (int base = 0; base < st.total; base += kWave) {
                __syncthreads();
                stage[lane] = nxt;
                __syncthreads();
                if (base + kWave < st.total) nxt = fetch_pos(st, base + kWave + lane, src);
                const int cnt = min(kWave, st.total - base);
                const int niter = (cnt + kl - 1) >> lk;
                for (int i = 0; i < niter; ++i) {
                    const float4 s = stage[sub + (i << lk)];
                    const float dx = s.x - px, dy = s.y - py, dz = s.z - pz;
                    const float tt = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
                    const float s2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                    cnt_lane += (tt < tc2 && s2 > 0.f) ? 1u : 0u;
                }
            }
            if (tv) pairs += cnt_lane;
        }
    }
    guard.report(hdr, lane);
    for (int o = 32; o >= 1; o >>= 1) pairs += __shfl_xor(pairs, o);
    if (lane == 0 && pairs)
        atomicAdd((unsigned long long *)&hdr[kHdrPairs], pairs);
}

// --------------------------------------------------------------- symmetric tiles
//
// Newton's third law halves the pair work between dense particles (the full
// blocks of 64 active particles of a cell, dense_count).  The dense particles
// of a home cell A meet those of A itself and of the 13 cells of the upper
// half of its stencil (first nonzero offset positive): every unordered pair of
// dense particles within reach lies in exactly one such meeting, since a cell
// pair {A, B} is in the upper half of A or of B, never both (at least three
// cells per dimension).  The dense particles of these 14 cells, concatenated
// in a fixed order, are A's virtual source list, cut into windows of W
// sources; A's dense blocks are taken K at a time (a run).  A work item
// (A, run g, window k) sums, for every block of the run, the block's targets
// against the window's sources (culled by the block's box) and the opposite
// terms onto those sources.  Inside the cell only pairs with the source after
// the target count (the block itself as a triangle).  Both sums go to fixed
// partial slots of a pool:
//   target slots  for cell A, window k and dense particle i of A;
//   source slots  for cell B, direction e, run g of the cell A = B - dir_e and
//                 dense particle j of B.
// Every slot has exactly one writer.  k_sym_gather then adds the slots of each
// dense particle in a fixed order to what its one-sided item (non-dense
// sources only) wrote.  A forward pair term equals, bit for bit, the one the
// one-sided kernel evaluates from either end, and only the order of the sums
// differs.  An adjoint term T is formed once and added to one end and
// subtracted from the other (subtraction and the products of u are
// antisymmetric in float32); the one-sided kernel instead fuses its two
// products into the target's sum, so the two differ by rounding as well.
//
// A tile pairs 64 targets (one per lane) with 64 staged sources: at step s
// lane l takes source (l + s) mod 64, and the lane's running sum for that
// source moves one lane down after the step (a rotation of the wave), so
// after all 64 steps lane l holds the opposite sum of source l.  No cross-lane
// reduction is needed per source.

// Direction e of the symmetric stencil: 0 is the cell itself, 1..13 the upper
// half (dx = 1: 9 directions; dx = 0, dy = 1: 3; dx = dy = 0, dz = 1: 1).
__device__ __forceinline__ void half_dir(int e, int &dx, int &dy, int &dz)
{
    const int q = e - 1;
    dx = e == 0 ? 0 : (q < 9 ? 1 : 0);
    dy = e == 0 ? 0 : (q < 9 ? q / 3 - 1 : (q < 12 ? 1 : 0));
    dz = e == 0 ? 0 : (q < 9 ? q % 3 - 1 : (q < 12 ? q - 10 : 1));
}

// Cell at offset (dx, dy, dz) from cell (ix, iy, iz) of a problem and the
// shift of its centre (image) from the home centre; false outside an open domain.
__device__ __forceinline__ bool cell_at(const SegParams &S, int ix, int iy, int iz, int dx, int dy,
                                        int dz, int &cell, float &sx, float &sy, float &sz)
{
    int jx, jy, jz;
    if (!neighbour(ix, dx, S.nc[0], S.lo[0], S.h[0], S.len[0], S.periodic, jx, sx)) return false;
    if (!neighbour(iy, dy, S.nc[1], S.lo[1], S.h[1], S.len[1], S.periodic, jy, sy)) return false;
    if (!neighbour(iz, dz, S.nc[2], S.lo[2], S.h[2], S.len[2], S.periodic, jz, sz)) return false;
    cell = S.cell_off + (jx * S.nc[1] + jy) * S.nc[2] + jz;
    return true;
}

// Direction f of the full stencil (0..26): offsets (f / 9 - 1, (f / 3) % 3 - 1, f % 3 - 1).
__device__ __forceinline__ void full_dir(int f, int &dx, int &dy, int &dz)
{
    dx = f / 9 - 1;
    dy = (f / 3) % 3 - 1;
    dz = f % 3 - 1;
}

// Per cell c, the partial-slot counts of its row of kSymStride groups: [0]
// target slots (items per run, each R consecutive windows, times its dense
// particles); [1 + e] source slots
// of its dense particles for direction e of the half stencil (runs of the
// cell c - dir_e times the dense particles); [15 + f] source slots of its
// non-dense particles for direction f of the full stencil (runs of the cell
// c - dir_f times the non-dense particles).  Stored as the row's exclusive
// prefix sums in pref and the row total in tot[c]; a scan of tot gives each
// cell's first slot, so group e of cell c starts at base[c] + pref[c][e].
// Also the item count and cost class of c as a home cell (runs times window
// groups) in info[c], and the slot total of all cells (int64, header).  The
// workgroup's rows are assembled in LDS and stored as one contiguous run.
template <class Acc>
__global__ __launch_bounds__(256) void k_sym_count(Acc acc, int NC, const int *__restrict__ start,
                                                   const int *__restrict__ nact, int K, int W, int R,
                                                   int *__restrict__ pref, int *__restrict__ tot_out,
                                                   uint32_t *__restrict__ info, uint32_t *hdr,
                                                   uint32_t magic)
{
    __shared__ uint32_t blk[kClasses];
    __shared__ unsigned long long tot, work;
    __shared__ uint32_t longest;
    __shared__ int rows[256 * kSymStride];
    if (threadIdx.x < kClasses) blk[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        tot = 0;
        work = 0;
        longest = 0;
    }
    __syncthreads();
    const bool ok = hdr[kHdrMagic] == magic;
    const int c0 = blockIdx.x * 256;
    const int c = c0 + threadIdx.x;
    if (c < NC) {
        int *row = rows + kSymStride * threadIdx.x;
        uint32_t inf = 0;
        unsigned long long slots = 0;
        if (ok) {
            const int D = dense_count(nact[c]);
            const int ND = start[c + 1] - start[c] - D;
            const SegParams &S = acc.get(acc.seg_of_cell(c));
            int ix, iy, iz;
            decode_cell(S, c, ix, iy, iz);
            // dense and non-dense counts of the 27 cells of the stencil (0
            // outside an open domain), all loads in flight together; every
            // group below reads them from here
            int nd[kSymNdDirs], nn[kSymNdDirs];
#pragma unroll
            for (int f = 0; f < kSymNdDirs; ++f) {
                int dx, dy, dz, b;
                float sx, sy, sz;
                full_dir(f, dx, dy, dz);
                nd[f] = 0;
                nn[f] = 0;
                if ((D > 0 || ND > 0) && cell_at(S, ix, iy, iz, dx, dy, dz, b, sx, sy, sz)) {
                    nd[f] = dense_count(nact[b]);
                    nn[f] = start[b + 1] - start[b] - nd[f];
                }
            }
            // direction (dx, dy, dz) is full-stencil index f = 9 (dx + 1) + 3 (dy + 1) + dz + 1,
            // and its opposite 26 - f
            auto runs_of = [&](int f) { return (nd[f] / kWave + K - 1) / K; };
            int64_t sv = 0;
#pragma unroll
            for (int e = 0; e < kSymDirs; ++e) {
                int dx, dy, dz;
                half_dir(e, dx, dy, dz);
                const int f = 9 * (dx + 1) + 3 * (dy + 1) + dz + 1;
                int64_t sc = 0;
                if (D > 0) {
                    sv += nd[f];
                    sc = (int64_t)runs_of(kSymNdDirs - 1 - f) * D;
                }
                row[1 + e] = (int)min(sc, (int64_t)INT32_MAX);
                slots += (unsigned long long)sc;
            }
#pragma unroll
            for (int f = 0; f < kSymNdDirs; ++f) {
                if (D > 0) sv += nn[f];
                int64_t sc = 0;
                if (ND > 0) sc = (int64_t)runs_of(kSymNdDirs - 1 - f) * ND;
                row[1 + kSymDirs + f] = (int)min(sc, (int64_t)INT32_MAX);
                slots += (unsigned long long)sc;
            }
            row[0] = 0;
            if (D > 0) {
                const int nb = D / kWave;
                const int64_t C = (sv + W - 1) / W;         // windows
                const int64_t CR = (C + R - 1) / R;         // items per run: R windows each
                const int64_t G = (nb + K - 1) / K;
                row[0] = (int)min(CR * D, (int64_t)INT32_MAX);
                slots += (unsigned long long)(CR * D);
                const int64_t n_items = G * CR;
                // tile steps of the widest item: its blocks times its windows
                int64_t cost = (int64_t)min(nb, K) * min((int64_t)R * W, sv);
                if (cost < 1) cost = 1;
                int cls = 63 - __clzll((unsigned long long)cost);
                cls = cls > 31 ? 31 : cls;
                if (n_items < (int64_t(1) << 27)) {
                    inf = ((uint32_t)n_items << 5) | (uint32_t)cls;
                    atomicAdd(&blk[cls], (uint32_t)n_items);
                    // every block of the cell meets every source of its list once
                    atomicAdd(&work, (unsigned long long)nb * (unsigned long long)sv);
                    atomicMax(&longest, (uint32_t)min(cost, (int64_t)UINT32_MAX));
                } else {
                    slots = ~0ull >> 2;  // beyond any pool: the symmetric tiles stay off
                }
            }
        } else {
            for (int e = 0; e < kSymStride; ++e) row[e] = 0;
        }
        // counts to exclusive prefixes; a total past 2^31 - 1 exceeds every pool
        // (the header's int64 total turns the tiles off), so clamping is harmless
        int64_t run = 0;
        for (int e = 0; e < kSymStride; ++e) {
            const int v = row[e];
            row[e] = (int)min(run, (int64_t)INT32_MAX);
            run += v;
        }
        tot_out[c] = (int)min(run, (int64_t)INT32_MAX);
        info[c] = inf;
        if (slots) atomicAdd(&tot, slots);
    }
    __syncthreads();
    const int nrow = min(256, NC - c0);
    int *out = pref + (int64_t)kSymStride * c0;
    for (int i = threadIdx.x; i < nrow * kSymStride; i += 256) out[i] = rows[i];
    if (threadIdx.x < kClasses && blk[threadIdx.x])
        atomicAdd(&hdr[kHdrSymBucketCount + threadIdx.x], blk[threadIdx.x]);
    if (threadIdx.x == 0) {
        if (tot) atomicAdd((unsigned long long *)&hdr[kHdrSymTotal], tot);
        if (work) atomicAdd((unsigned long long *)&hdr[kHdrSymWork], work);
        if (longest) atomicMax(&hdr[kHdrSymMaxItem], longest);
    }
}

// Class bases of the symmetric items, heaviest first; the tiles run only when
// enabled, on bins of these sizes, when every partial slot fits the pool, and
// when their work spread over the persistent grid (waves) is at least
// balance times the longest item: otherwise a few long items would leave most
// waves idle, and the one-sided kernels, with items of at most 64 targets,
// finish sooner.
__global__ void k_sym_base(uint32_t *hdr, uint32_t magic, long long cap, int enabled, int waves,
                           double balance)
{
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int cls = kClasses - 1; cls >= 0; --cls) {
            hdr[kHdrSymBucketBase + cls] = run;
            run += hdr[kHdrSymBucketCount + cls];
        }
        const unsigned long long tot = *(const unsigned long long *)&hdr[kHdrSymTotal];
        const double work = (double)*(const unsigned long long *)&hdr[kHdrSymWork];
        const bool spread = work >= balance * (double)waves * (double)hdr[kHdrSymMaxItem];
        const bool ok = enabled && hdr[kHdrMagic] == magic && run > 0 && tot <= (unsigned long long)cap &&
                        spread;
        hdr[kHdrSymOk] = ok ? 1u : 0u;
        hdr[kHdrSymNItems] = ok ? run : 0u;
    }
    if (threadIdx.x < kClasses) hdr[kHdrSymBucketCursor + threadIdx.x] = 0;
    if (threadIdx.x < kQueues) hdr[kHdrSymQueue + 32 * threadIdx.x] = 0;
}

// Symmetric items (A, run, window, problem), in cost-class order.
template <class Acc>
__global__ __launch_bounds__(256) void k_sym_write(Acc acc, int NC, const int *__restrict__ nact,
                                                   int K, const uint32_t *__restrict__ info,
                                                   uint32_t *hdr, int4 *__restrict__ items)
{
    __shared__ uint32_t cnt[kClasses];
    __shared__ uint32_t base[kClasses];
    if (hdr[kHdrSymOk] == 0) return;  // uniform over the block
    if (threadIdx.x < kClasses) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int c = blockIdx.x * 256 + threadIdx.x;
    const uint32_t inf = c < NC ? info[c] : 0u;
    const int n_items = (int)(inf >> 5);
    const int cls = (int)(inf & 31);
    uint32_t local = 0;
    if (inf) local = atomicAdd(&cnt[cls], (uint32_t)n_items);
    __syncthreads();
    if (threadIdx.x < kClasses && cnt[threadIdx.x])
        base[threadIdx.x] = hdr[kHdrSymBucketBase + threadIdx.x] +
                            atomicAdd(&hdr[kHdrSymBucketCursor + threadIdx.x], cnt[threadIdx.x]);
    __syncthreads();
    if (!inf) return;
    const int nb = dense_count(nact[c]) / kWave;
    const int G = (nb + K - 1) / K;
    const int C = n_items / G;
    const int seg = acc.seg_of_cell(c);
    const uint32_t at = base[cls] + local;
    for (int g = 0; g < G; ++g)
        for (int k = 0; k < C; ++k) items[at + (uint32_t)(g * C + k)] = make_int4(c, g, k, seg);
}

// The source segments of a symmetric item, one per lane: lanes 0..13 the
// dense particles of the cell itself and of its 13 upper-half neighbours
// (each such pair once), lanes 14..40 the non-dense particles of all 27
// cells of its stencil (none of them is ever a symmetric target, so each of
// those pairs is met once too).  Per segment: first binned slot, count,
// prefix of the counts, centre shift, and the base of the source slots its
// particles receive from this cell.
struct SymStencil {
    int nstart, cnt, excl, sbase;
    float sx, sy, sz;
    int total;
};

__device__ __forceinline__ void sym_stencil_setup(const SegParams &S, int cell,
                                                  const int *__restrict__ start,
                                                  const int *__restrict__ nact,
                                                  const int *__restrict__ sym_base,
                                                  const int *__restrict__ sym_pref, int lane,
                                                  SymStencil &st)
{
    int ix, iy, iz;
    decode_cell(S, cell, ix, iy, iz);
    st.nstart = 0;
    st.cnt = 0;
    st.sbase = 0;
    st.sx = st.sy = st.sz = 0.f;
    if (lane < kSymSegs) {
        int dx, dy, dz, b;
        if (lane < kSymDirs)
            half_dir(lane, dx, dy, dz);
        else
            full_dir(lane - kSymDirs, dx, dy, dz);
        if (cell_at(S, ix, iy, iz, dx, dy, dz, b, st.sx, st.sy, st.sz)) {
            const int d = dense_count(nact[b]);
            st.nstart = start[b] + (lane < kSymDirs ? 0 : d);
            st.cnt = lane < kSymDirs ? d : start[b + 1] - start[b] - d;
            st.sbase = sym_base[b] + sym_pref[(int64_t)kSymStride * b + 1 + lane];
        }
    }
    int incl = st.cnt;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int y = __shfl_up(incl, d);
        if (lane >= d) incl += y;
    }
    st.excl = incl - st.cnt;
    st.total = __builtin_amdgcn_readfirstlane(__shfl(incl, kSymSegs - 1));
}

// Segment of virtual source v (clamped to the list); every lane must call it.
__device__ __forceinline__ int sym_locate(const SymStencil &st, int v)
{
    const int vv = min(v, st.total - 1);
    int q = 0;
#pragma unroll
    for (int step = 32; step >= 1; step >>= 1) {
        const int cand = q + step;
        const int e = __shfl(st.excl, min(cand, kSymSegs - 1));
        if (cand < kSymSegs && e <= vv) q = cand;
    }
    return q;
}

// Position (shifted into the home frame) and mass of virtual source v;
// padding (v >= end) is far away with zero mass.
__device__ __forceinline__ float4 sym_fetch_pos(const SymStencil &st, int v, int end, const Src &s,
                                                int &slot)
{
    const int q = sym_locate(st, v);
    const int j = __shfl(st.nstart, q) + (min(v, st.total - 1) - __shfl(st.excl, q));
    float4 r = make_float4(s.x[j] + __shfl(st.sx, q), s.y[j] + __shfl(st.sy, q),
                           s.z[j] + __shfl(st.sz, q), s.m[j]);
    slot = j;
    if (v >= end) r = make_float4(kFar, kFar, kFar, 0.f);
    return r;
}

// Lane l takes lane l + 1's value (mod 64): the rotation of a tile step.
__device__ __forceinline__ float rotate_down(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x134, 0xf, 0xf,
                                                              false));
}

// Lane l takes lane l + 1's value within its row of 16 lanes (mod 16): the
// rotation of a step of the row tiles that finish a stream.
__device__ __forceinline__ float rotate_row(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x12f, 0xf, 0xf,
                                                              false));
}

// Sum of v over the four rows of 16 lanes, the same on each row, in a fixed
// order: (row 0 + row 1) + (row 2 + row 3).
__device__ __forceinline__ float sum_rows(float v)
{
    v += __shfl_xor(v, 16);
    return v + __shfl_xor(v, 32);
}

// One forward step: target (px, py, pz, mi) gets m_j d f, the source's running
// sum gets -m_i d f (t = s + eps^2 < tc2).  With kUM both masses are applied
// once, by the gather.
template <bool kSoft, bool kUM>
__device__ __forceinline__ void sym_force_step(const float4 s, float px, float py, float pz, float mi,
                                               float eps2, float tc2, const float *cq, float &ax,
                                               float &ay, float &az, float &bx, float &by, float &bz)
{
    const float dx = s.x - px, dy = s.y - py, dz = s.z - pz;
    const float tt = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
    const float qi = __builtin_amdgcn_rsqf(tt);
    const float q2 = qi * qi;
    const float f = fmaf(q2, qi, -horner5(cq, tt));
    const bool in = kSoft ? (tt < tc2) : (tt < tc2 && tt > 0.f);
    // lanes out of reach skip the sums (an exec mask, not a select: one
    // instruction fewer per step; their f may be infinite for padding)
    if (in) {
        const float wt = kUM ? f : s.w * f;
        const float ws = kUM ? f : mi * f;
        ax = fmaf(wt, dx, ax);
        ay = fmaf(wt, dy, ay);
        az = fmaf(wt, dz, az);
        bx = fmaf(-ws, dx, bx);
        by = fmaf(-ws, dy, by);
        bz = fmaf(-ws, dz, bz);
    }
}

// One adjoint step: the target gets T = f u + 2 f' (u.d) d, the source -T
// (u = m_k g_j - m_j g_k, d = x_j - x_k; with kUM, u / m), at the scale -1/3
// of the one-sided adjoint.
template <bool kSoft, bool kUM>
__device__ __forceinline__ void sym_vjp_step(const float4 s, const float4 gj, float px, float py,
                                             float pz, float mk, float gkx, float gky, float gkz,
                                             float eps2, float tc2, const float *cq, const float *cd,
                                             float &rx, float &ry, float &rz, float &bx, float &by,
                                             float &bz)
{
#pragma clang fp contract(off)
    const float dx = s.x - px, dy = s.y - py, dz = s.z - pz;
    const float tt = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
    const float qi = __builtin_amdgcn_rsqf(tt);
    const float q2 = qi * qi;
    const float q3 = q2 * qi;
    const bool in = kSoft ? (tt < tc2) : (tt < tc2 && tt > 0.f);
    const float f = fmaf(q3, kMinusThird, horner5(cq, tt));
    const float fp2 = fmaf(q3, q2, horner4(cd, tt));
    const float ux = kUM ? gj.x - gkx : mk * gj.x - s.w * gkx;
    const float uy = kUM ? gj.y - gky : mk * gj.y - s.w * gky;
    const float uz = kUM ? gj.z - gkz : mk * gj.z - s.w * gkz;
    const float c = fp2 * fmaf(ux, dx, fmaf(uy, dy, uz * dz));
    const float tx = fmaf(c, dx, f * ux);
    const float ty = fmaf(c, dy, f * uy);
    const float tz = fmaf(c, dz, f * uz);
    if (in) {  // an exec mask: out-of-reach lanes (T possibly infinite for padding) add nothing
        rx += tx;
        ry += ty;
        rz += tz;
        bx -= tx;
        by -= ty;
        bz -= tz;
    }
}

// Window partial sums of the sources (opposite terms), one float per source
// and axis, in LDS.
template <int kW>
struct SymRed {
    float x[kW], y[kW], z[kW];
};

// Stream the window's sources [vs, w1) through the culling test against the
// block's box and gather the survivors straight into the tile (tile0, and
// tile1 for a second float4 per source; each entry stored twice, at e and
// e + 64, so that step s of lane l reads entry l + s without a wrap) with
// their window index in tix.  Whenever 64 are in, `tile(my)` runs (my: the
// window index of this lane's entry, -1 for padding); survivors of the same
// batch beyond the 64th start the next tile.  The last n <= 48 survivors of
// the stream run as `rows(c)`, c = ceil(n / 16) chunks of 16 entries (padded)
// that each meet all 64 targets in 16 steps, instead of a 64-step tile that
// is mostly padding.  Every lane must call this.
template <int kParts, class Fetch, class Tile, class Rows>
__device__ __forceinline__ void sym_stream(int vs, int w1, int w0, const Box &box, float cull2, int lane,
                                           float4 *tile0, float4 *tile1, int *tix, Fetch &&fetch,
                                           Tile &&tile, Rows &&rows)
{
    if (vs >= w1) return;
    const uint64_t below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    int fill = 0;
    auto put = [&](int at, const float4 &c0, const float4 &c1, int ix) {
        tile0[at] = c0;
        tile0[at + kWave] = c0;
        if (kParts == 2) {
            tile1[at] = c1;
            tile1[at + kWave] = c1;
        }
        tix[at] = ix;
    };
    auto run = [&]() {
        __syncthreads();
        const int my = tix[lane];
        tile(my);
        __syncthreads();
    };
    float4 c0, c1;
    fetch(vs + lane, c0, c1);
    for (int base = vs; base < w1; base += kWave) {
        const bool keep = (base + lane < w1) && may_reach(box, c0.x, c0.y, c0.z, cull2);
        const uint64_t m = __ballot(keep);
        const int cnt = __popcll(m);
        const int at = fill + __popcll(m & below);
        const int ix = base + lane - w0;
        if (keep && at < kWave) put(at, c0, c1, ix);
        if (fill + cnt >= kWave) {
            run();
            if (keep && at >= kWave) put(at - kWave, c0, c1, ix);
            fill += cnt - kWave;
        } else {
            fill += cnt;
        }
        if (base + kWave < w1) fetch(base + kWave + lane, c0, c1);
    }
    if (fill > 0) {
        if (lane >= fill)
            put(lane, make_float4(kFar, kFar, kFar, 0.f), make_float4(0.f, 0.f, 0.f, 0.f), -1);
        const int chunks = (fill + 15) >> 4;
        if (chunks < 4) {
            __syncthreads();
            rows(chunks);
            __syncthreads();
        } else {
            run();
        }
    }
}

// sym_stream for a window whose kB batches of 64 candidates an item fetched
// once into registers (held[i]: sources w0 + 64 i + lane), for the forward's
// one float4 per source: every block of the item culls the same held
// candidates instead of fetching the window again.  Batches before vs are
// skipped, entries of a batch before vs are masked.  Every lane must call it.
template <int kB, class Tile, class Rows>
__device__ __forceinline__ void sym_stream_held(const float4 (&held)[kB], int vs, int w1, int w0,
                                                const Box &box, float cull2, int lane, float4 *tile0,
                                                int *tix, Tile &&tile, Rows &&rows)
{
    if (vs >= w1) return;
    const uint64_t below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    int fill = 0;
    auto put = [&](int at, const float4 &c0, int ix) {
        tile0[at] = c0;
        tile0[at + kWave] = c0;
        tix[at] = ix;
    };
#pragma unroll
    for (int i = 0; i < kB; ++i) {
        const int base = w0 + i * kWave;
        if (base < w1 && base + kWave > vs) {
            const float4 c0 = held[i];
            const int v = base + lane;
            const bool keep = v >= vs && v < w1 && may_reach(box, c0.x, c0.y, c0.z, cull2);
            const uint64_t m = __ballot(keep);
            const int cnt = __popcll(m);
            const int at = fill + __popcll(m & below);
            const int ix = v - w0;
            if (keep && at < kWave) put(at, c0, ix);
            if (fill + cnt >= kWave) {
                __syncthreads();
                const int my = tix[lane];
                tile(my);
                __syncthreads();
                if (keep && at >= kWave) put(at - kWave, c0, ix);
                fill += cnt - kWave;
            } else {
                fill += cnt;
            }
        }
    }
    if (fill > 0) {
        if (lane >= fill) put(lane, make_float4(kFar, kFar, kFar, 0.f), -1);
        const int chunks = (fill + 15) >> 4;
        __syncthreads();
        if (chunks < 4) {
            rows(chunks);
        } else {
            const int my = tix[lane];
            tile(my);
        }
        __syncthreads();
    }
}

// Entry chunk k (16 entries) of a tile in the row layout: entry j at rt[j]
// and rt[j + 16], so that step s of lane l reads rt[(l mod 16) + s].  The
// second half of the tile (its wrap copy, unused by row tiles) holds it.
__device__ __forceinline__ void row_chunk(float4 *tile, int k, int lane)
{
    __syncthreads();
    if (lane < 16) {
        const float4 e = tile[16 * k + lane];
        tile[kWave + lane] = e;
        tile[kWave + 16 + lane] = e;
    }
    __syncthreads();
}

// Forward symmetric items.
template <class Acc, bool kSoft, bool kUM, int kW>
__device__ __forceinline__ void force_sym_items(const Acc &acc, const int4 *__restrict__ items,
                                                uint32_t *hdr, const int *__restrict__ start,
                                                const int *__restrict__ nact,
                                                const int *__restrict__ sym_base,
                                                const int *__restrict__ sym_pref, const Src &src,
                                                float *__restrict__ pool, int K, int R, float4 *tile,
                                                int *tix, SymRed<kW> &red, int64_t pull_limit)
{
    const int lane = threadIdx.x;
    const int64_t n_items = hdr[kHdrSymNItems];
    // tiles off (or nothing to do): leave before touching the queues, which
    // thousands of idle waves would otherwise all hit once per queue
    if (n_items == 0) return;
    const int q0 = blockIdx.x & (kQueues - 1);
    PullGuard guard(min(n_items, pull_limit));
    for (int qq = 0; qq < kQueues && !guard.bad; ++qq) {
        const int q = (q0 + qq) & (kQueues - 1);
        guard.next_queue();
        for (;;) {
            const int64_t gi = next_item(hdr, q, lane, kHdrSymQueue);
            if (gi >= n_items || !guard.accept(gi)) break;
            const int4 it = load_item(items, gi);
            const int c = it.x, g = it.y, kk = it.z;  // kk: the item's group of R windows
            const SegParams &S = acc.get(it.w);
            const float eps2 = S.pc.eps2, tc2 = S.pc.tc2, cull2 = S.pc.cull2;
            float cq[6];
#pragma unroll
            for (int i = 0; i < 6; ++i) cq[i] = S.pc.q[i];
            cq[5] = keep_in_vgpr(cq[5]);
            SymStencil st;
            sym_stencil_setup(S, c, start, nact, sym_base, sym_pref, lane, st);
            const int D = __shfl(st.cnt, 0);  // segment 0 is the cell itself
            const int c0s = start[c];
            const int tbase = sym_base[c] + kk * D;  // group 0: the target slots
            const int p0 = g * K, p1 = min(p0 + K, D / kWave);
            const int k_end = min((kk + 1) * R, (st.total + kW - 1) / kW);
            // the group's windows in turn: the first stores each block's target sums
            // to its slot, the next ones add to it (this wave alone writes the slot)
            for (int k = kk * R; k < k_end; ++k) {
                const bool first = k == kk * R;
                const int w0 = k * kW, w1 = min(w0 + kW, st.total);
                for (int i = lane; i < kW; i += kWave) red.x[i] = red.y[i] = red.z[i] = 0.f;
                auto fetch_p = [&](int v, float4 &a, float4 &) {
                    int slot;
                    a = sym_fetch_pos(st, v, w1, src, slot);
                };
                // windows of 256: the window's sources once, held in registers for all blocks
                constexpr int kHeld = kW == 256 ? kW / kWave : 1;
                float4 held[kHeld];
#pragma unroll
                for (int i = 0; i < kHeld; ++i) {
                    held[i] = make_float4(kFar, kFar, kFar, 0.f);
                    if (kW == 256 && w0 + i * kWave < w1) {
                        int slot;
                        held[i] = sym_fetch_pos(st, w0 + i * kWave + lane, w1, src, slot);
                    }
                }
                for (int p = p0; p < p1; ++p) {
                    const int b = c0s + p * kWave + lane;
                    const float px = src.x[b], py = src.y[b], pz = src.z[b];
                    const float mi = kUM ? 1.f : src.m[b];
                    const Box box = target_box(true, px, py, pz, false, 0.f, 0.f, 0.f);
                    float ax = 0.f, ay = 0.f, az = 0.f;
                    if (p * kWave >= w0 && p * kWave < w1) {
                        // the block against itself: steps 1..32, the last one on half the lanes
                        __syncthreads();
                        tile[lane] = make_float4(px, py, pz, src.m[b]);
                        tile[lane + kWave] = tile[lane];
                        __syncthreads();
                        float bx = 0.f, by = 0.f, bz = 0.f;
                        for (int s = 1; s <= kWave / 2; ++s) {
                            float4 sj = tile[lane + s];
                            if (s == kWave / 2 && lane >= kWave / 2) sj = make_float4(kFar, kFar, kFar, 0.f);
                            sym_force_step<kSoft, kUM>(sj, px, py, pz, mi, eps2, tc2, cq, ax, ay, az, bx, by, bz);
                            bx = rotate_down(bx);
                            by = rotate_down(by);
                            bz = rotate_down(bz);
                        }
                        const int r = p * kWave - w0 + ((lane + kWave / 2 + 1) & (kWave - 1));
                        red.x[r] += bx;
                        red.y[r] += by;
                        red.z[r] += bz;
                    }
                    const int vs = max(w0, (p + 1) * kWave);
                    auto tile_fn = [&](int my) {
                        float bx = 0.f, by = 0.f, bz = 0.f;
                        const float4 *t = tile + lane;
                        for (int s = 0; s < kWave; s += 8) {
#pragma unroll
                            for (int u = 0; u < 8; ++u) {
                                sym_force_step<kSoft, kUM>(t[s + u], px, py, pz, mi, eps2, tc2, cq, ax, ay, az,
                                                           bx, by, bz);
                                bx = rotate_down(bx);
                                by = rotate_down(by);
                                bz = rotate_down(bz);
                            }
                        }
                        if (my >= 0) {
                            red.x[my] += bx;
                            red.y[my] += by;
                            red.z[my] += bz;
                        }
                    };
                    auto rows_fn = [&](int chunks) {
                        const float4 *t = tile + kWave + (lane & 15);
                        for (int k = 0; k < chunks; ++k) {
                            row_chunk(tile, k, lane);
                            float bx = 0.f, by = 0.f, bz = 0.f;
                            for (int s = 0; s < 16; s += 8) {
#pragma unroll
                                for (int u = 0; u < 8; ++u) {
                                    sym_force_step<kSoft, kUM>(t[s + u], px, py, pz, mi, eps2, tc2, cq, ax, ay,
                                                               az, bx, by, bz);
                                    bx = rotate_row(bx);
                                    by = rotate_row(by);
                                    bz = rotate_row(bz);
                                }
                            }
                            bx = sum_rows(bx);
                            by = sum_rows(by);
                            bz = sum_rows(bz);
                            const int my = tix[16 * k + (lane & 15)];
                            if (lane < 16 && my >= 0) {
                                red.x[my] += bx;
                                red.y[my] += by;
                                red.z[my] += bz;
                            }
                        }
                    };
                    if constexpr (kW == 256)
                        sym_stream_held(held, vs, w1, w0, box, cull2, lane, tile, tix, tile_fn, rows_fn);
                    else
                        sym_stream<1>(vs, w1, w0, box, cull2, lane, tile, tile, tix, fetch_p, tile_fn, rows_fn);
                    const int64_t o = 3 * ((int64_t)tbase + p * kWave + lane);
                    if (first) {
                        pool[o] = ax;
                        pool[o + 1] = ay;
                        pool[o + 2] = az;
                    } else {
                        pool[o] += ax;
                        pool[o + 1] += ay;
                        pool[o + 2] += az;
                    }
                }
                __syncthreads();
                // the window's opposite sums to their source slots
                for (int i = 0; i < w1 - w0; i += kWave) {
                    const int v = w0 + i + lane;
                    const int q = sym_locate(st, v);
                    const int64_t slot = (int64_t)__shfl(st.sbase, q) + (int64_t)g * __shfl(st.cnt, q) +
                                         (min(v, st.total - 1) - __shfl(st.excl, q));
                    if (v < w1) {
                        pool[3 * slot] = red.x[i + lane];
                        pool[3 * slot + 1] = red.y[i + lane];
                        pool[3 * slot + 2] = red.z[i + lane];
                    }
                }
                __syncthreads();
            }
        }
    }
    guard.report(hdr, lane);
}

template <class Acc, bool kSoft, int kW, int kOcc>
__global__ __launch_bounds__(64, kOcc > 0 ? kOcc : 1) void k_force_sym(Acc acc, const int4 *__restrict__ items, uint32_t *hdr,
                                                  const int *__restrict__ start,
                                                  const int *__restrict__ nact,
                                                  const int *__restrict__ sym_base,
                                                  const int *__restrict__ sym_pref, Src src,
                                                  float *__restrict__ pool, int K, int R, int64_t pull_limit)
{
    __shared__ float4 tile[2 * kWave];
    __shared__ int tix[kWave];
    __shared__ SymRed<kW> red;
    if (hdr[kHdrMassInfo] == 0)
        force_sym_items<Acc, kSoft, true, kW>(acc, items, hdr, start, nact, sym_base, sym_pref, src, pool, K, R,
                                              tile, tix, red, pull_limit);
    else
        force_sym_items<Acc, kSoft, false, kW>(acc, items, hdr, start, nact, sym_base, sym_pref, src, pool, K, R,
                                               tile, tix, red, pull_limit);
}

// Adjoint symmetric items: as the forward, with the cotangent staged beside
// each source.
template <class Acc, bool kSoft, bool kUM, int kW>
__device__ __forceinline__ void vjp_sym_items(const Acc &acc, const int4 *__restrict__ items,
                                              uint32_t *hdr, const int *__restrict__ start,
                                              const int *__restrict__ nact,
                                              const int *__restrict__ sym_base,
                                              const int *__restrict__ sym_pref, const Src &src,
                                              const float *__restrict__ gx, const float *__restrict__ gy,
                                              const float *__restrict__ gz, float *__restrict__ pool,
                                              int K, int R, float4 *tile_p, float4 *tile_g, int *tix,
                                              SymRed<kW> &red, int64_t pull_limit)
{
    const int lane = threadIdx.x;
    const int64_t n_items = hdr[kHdrSymNItems];
    // tiles off (or nothing to do): leave before touching the queues, which
    // thousands of idle waves would otherwise all hit once per queue
    if (n_items == 0) return;
    const int q0 = blockIdx.x & (kQueues - 1);
    PullGuard guard(min(n_items, pull_limit));
    for (int qq = 0; qq < kQueues && !guard.bad; ++qq) {
        const int q = (q0 + qq) & (kQueues - 1);
        guard.next_queue();
        for (;;) {
            const int64_t gi = next_item(hdr, q, lane, kHdrSymQueue);
            if (gi >= n_items || !guard.accept(gi)) break;
            const int4 it = load_item(items, gi);
            const int c = it.x, g = it.y, kk = it.z;  // kk: the item's group of R windows
            const SegParams &S = acc.get(it.w);
            const float eps2 = S.pc.eps2, tc2 = S.pc.tc2, cull2 = S.pc.cull2;
            float cq[6], cd[5];
#pragma unroll
            for (int i = 0; i < 6; ++i) cq[i] = S.pc.qa[i];
            cq[5] = keep_in_vgpr(cq[5]);
#pragma unroll
            for (int i = 0; i < 5; ++i) cd[i] = S.pc.dqa[i];
            cd[4] = keep_in_vgpr(cd[4]);
            SymStencil st;
            sym_stencil_setup(S, c, start, nact, sym_base, sym_pref, lane, st);
            const int D = __shfl(st.cnt, 0);
            const int c0s = start[c];
            const int tbase = sym_base[c] + kk * D;  // group 0: the target slots
            const int p0 = g * K, p1 = min(p0 + K, D / kWave);
            const int k_end = min((kk + 1) * R, (st.total + kW - 1) / kW);
            // the group's windows in turn: the first stores each block's target sums
            // to its slot, the next ones add to it (this wave alone writes the slot)
            for (int k = kk * R; k < k_end; ++k) {
                const bool first = k == kk * R;
                const int w0 = k * kW, w1 = min(w0 + kW, st.total);
                for (int i = lane; i < kW; i += kWave) red.x[i] = red.y[i] = red.z[i] = 0.f;
                auto fetch_pg = [&](int v, float4 &a, float4 &gv) {
                    int slot;
                    a = sym_fetch_pos(st, v, w1, src, slot);
                    gv = make_float4(gx[slot], gy[slot], gz[slot], 0.f);
                    if (v >= w1) gv = make_float4(0.f, 0.f, 0.f, 0.f);
                };
                for (int p = p0; p < p1; ++p) {
                    const int b = c0s + p * kWave + lane;
                    const float px = src.x[b], py = src.y[b], pz = src.z[b], mk = src.m[b];
                    const float gkx = gx[b], gky = gy[b], gkz = gz[b];
                    const Box box = target_box(true, px, py, pz, false, 0.f, 0.f, 0.f);
                    float rx = 0.f, ry = 0.f, rz = 0.f;
                    if (p * kWave >= w0 && p * kWave < w1) {
                        __syncthreads();
                        tile_p[lane] = make_float4(px, py, pz, mk);
                        tile_p[lane + kWave] = tile_p[lane];
                        tile_g[lane] = make_float4(gkx, gky, gkz, 0.f);
                        tile_g[lane + kWave] = tile_g[lane];
                        __syncthreads();
                        float bx = 0.f, by = 0.f, bz = 0.f;
                        for (int s = 1; s <= kWave / 2; ++s) {
                            float4 sj = tile_p[lane + s];
                            float4 sg = tile_g[lane + s];
                            if (s == kWave / 2 && lane >= kWave / 2) {
                                sj = make_float4(kFar, kFar, kFar, 0.f);
                                sg = make_float4(0.f, 0.f, 0.f, 0.f);
                            }
                            sym_vjp_step<kSoft, kUM>(sj, sg, px, py, pz, mk, gkx, gky, gkz, eps2, tc2, cq, cd, rx,
                                                     ry, rz, bx, by, bz);
                            bx = rotate_down(bx);
                            by = rotate_down(by);
                            bz = rotate_down(bz);
                        }
                        const int r = p * kWave - w0 + ((lane + kWave / 2 + 1) & (kWave - 1));
                        red.x[r] += bx;
                        red.y[r] += by;
                        red.z[r] += bz;
                    }
                    const int vs = max(w0, (p + 1) * kWave);
                    sym_stream<2>(vs, w1, w0, box, cull2, lane, tile_p, tile_g, tix, fetch_pg,
                                  [&](int my) {
                                      float bx = 0.f, by = 0.f, bz = 0.f;
                                      const float4 *tp = tile_p + lane;
                                      const float4 *tg = tile_g + lane;
                                      for (int s = 0; s < kWave; s += 4) {
#pragma unroll
                                          for (int u = 0; u < 4; ++u) {
                                              sym_vjp_step<kSoft, kUM>(tp[s + u], tg[s + u], px, py, pz, mk, gkx,
                                                                       gky, gkz, eps2, tc2, cq, cd, rx, ry, rz,
                                                                       bx, by, bz);
                                              bx = rotate_down(bx);
                                              by = rotate_down(by);
                                              bz = rotate_down(bz);
                                          }
                                      }
                                      if (my >= 0) {
                                          red.x[my] += bx;
                                          red.y[my] += by;
                                          red.z[my] += bz;
                                      }
                                  },
                                  [&](int chunks) {
                                      const float4 *tp = tile_p + kWave + (lane & 15);
                                      const float4 *tg = tile_g + kWave + (lane & 15);
                                      for (int k = 0; k < chunks; ++k) {
                                          row_chunk(tile_p, k, lane);
                                          row_chunk(tile_g, k, lane);
                                          float bx = 0.f, by = 0.f, bz = 0.f;
                                          for (int s = 0; s < 16; s += 4) {
#pragma unroll
                                              for (int u = 0; u < 4; ++u) {
                                                  sym_vjp_step<kSoft, kUM>(tp[s + u], tg[s + u], px, py, pz, mk,
                                                                           gkx, gky, gkz, eps2, tc2, cq, cd, rx,
                                                                           ry, rz, bx, by, bz);
                                                  bx = rotate_row(bx);
                                                  by = rotate_row(by);
                                                  bz = rotate_row(bz);
                                              }
                                          }
                                          bx = sum_rows(bx);
                                          by = sum_rows(by);
                                          bz = sum_rows(bz);
                                          const int my = tix[16 * k + (lane & 15)];
                                          if (lane < 16 && my >= 0) {
                                              red.x[my] += bx;
                                              red.y[my] += by;
                                              red.z[my] += bz;
                                          }
                                      }
                                  });
                    const int64_t o = 3 * ((int64_t)tbase + p * kWave + lane);
                    if (first) {
                        pool[o] = rx;
                        pool[o + 1] = ry;
                        pool[o + 2] = rz;
                    } else {
                        pool[o] += rx;
                        pool[o + 1] += ry;
                        pool[o + 2] += rz;
                    }
                }
                __syncthreads();
                for (int i = 0; i < w1 - w0; i += kWave) {
                    const int v = w0 + i + lane;
                    const int q = sym_locate(st, v);
                    const int64_t slot = (int64_t)__shfl(st.sbase, q) + (int64_t)g * __shfl(st.cnt, q) +
                                         (min(v, st.total - 1) - __shfl(st.excl, q));
                    if (v < w1) {
                        pool[3 * slot] = red.x[i + lane];
                        pool[3 * slot + 1] = red.y[i + lane];
                        pool[3 * slot + 2] = red.z[i + lane];
                    }
                }
                __syncthreads();
            }
        }
    }
    guard.report(hdr, lane);
}

template <class Acc, bool kSoft, int kW, int kOcc>
__global__ __launch_bounds__(64, kOcc > 0 ? kOcc : 1) void k_vjp_sym(Acc acc, const int4 *__restrict__ items, uint32_t *hdr,
                                                const int *__restrict__ start,
                                                const int *__restrict__ nact,
                                                const int *__restrict__ sym_base,
                                                const int *__restrict__ sym_pref, Src src,
                                                const float *__restrict__ gx, const float *__restrict__ gy,
                                                const float *__restrict__ gz, float *__restrict__ pool, int K,
                                                int R, int64_t pull_limit)
{
    __shared__ float4 tile_p[2 * kWave];
    __shared__ float4 tile_g[2 * kWave];
    __shared__ int tix[kWave];
    __shared__ SymRed<kW> red;
    if (hdr[kHdrMassInfo] == 0)
        vjp_sym_items<Acc, kSoft, true, kW>(acc, items, hdr, start, nact, sym_base, sym_pref, src, gx, gy, gz, pool, K,
                                            R, tile_p, tile_g, tix, red, pull_limit);
    else
        vjp_sym_items<Acc, kSoft, false, kW>(acc, items, hdr, start, nact, sym_base, sym_pref, src, gx, gy, gz, pool, K,
                                             R, tile_p, tile_g, tix, red, pull_limit);
}

// Adds up the partial slots of every particle, in a fixed order.  A dense
// particle: its target slots over the windows, then its source slots over
// the 14 directions and runs; it has no one-sided item, so the sum is its
// row (out[row] = m0 * sum).  A non-dense particle: its source slots over the
// 27 directions and runs, added to the row its one-sided item wrote
// (out[row] += m0 * sum).  m0 is scale (1 forward, -3 adjoint) times the
// common mass when every mass is equal, else times 1.  rows: out_row
// (forward, n_out = rows of acc; passive particles have none) or perm
// (adjoint, n_out = N).
__global__ __launch_bounds__(256) void k_sym_gather(int N, int key_bits, const int *__restrict__ key,
                                                    const int *__restrict__ start,
                                                    const int *__restrict__ nact,
                                                    const int *__restrict__ sym_pref,
                                                    const int *__restrict__ sym_base,
                                                    const float *__restrict__ pool,
                                                    const int *__restrict__ rows,
                                                    const float *__restrict__ mass /*binned*/,
                                                    const uint32_t *hdr,
                                                    float *__restrict__ out, int n_out, float scale)
{
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= N || hdr[kHdrSymOk] == 0) return;
    const int r = rows[b];
    if (r < 0 || r >= n_out) return;
    const int c = key[b] >> key_bits;
    const int jl = b - start[c];
    const int D = dense_count(nact[c]);
    const bool dense = jl < D;
    const int per = dense ? D : start[c + 1] - start[c] - D;  // particles of a slot row
    const int j = dense ? jl : jl - D;
    const int e0 = dense ? 0 : 1 + kSymDirs, e1 = dense ? 1 + kSymDirs : kSymStride;
    const int *pf = sym_pref + (int64_t)kSymStride * c;
    const int cb = sym_base[c], ctot = sym_base[c + 1] - cb;
    struct F3 {
        float x, y, z;
    };
    const F3 *P = reinterpret_cast<const F3 *>(pool);
    // four running sums over the slots of a row group (loads in flight
    // together), combined in a fixed order at the end
    float x[4] = {0.f, 0.f, 0.f, 0.f}, y[4] = {0.f, 0.f, 0.f, 0.f}, z[4] = {0.f, 0.f, 0.f, 0.f};
    for (int e = e0; e < e1; ++e) {
        const int n = ((e + 1 < kSymStride ? pf[e + 1] : ctot) - pf[e]) / per;
        int64_t o = (int64_t)cb + pf[e] + j;
        int t = 0;
        for (; t + 4 <= n; t += 4, o += 4 * (int64_t)per) {
            F3 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = P[o + u * (int64_t)per];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                x[u] += v[u].x;
                y[u] += v[u].y;
                z[u] += v[u].z;
            }
        }
        for (; t < n; ++t, o += per) {
            const F3 v = P[o];
            x[0] += v.x;
            y[0] += v.y;
            z[0] += v.z;
        }
    }
    const float sx = (x[0] + x[1]) + (x[2] + x[3]);
    const float sy = (y[0] + y[1]) + (y[2] + y[3]);
    const float sz = (z[0] + z[1]) + (z[2] + z[3]);
    const float m0 = scale * (hdr[kHdrMassInfo] == 0 ? mass[0] : 1.0f);
    const int64_t q = 3 * (int64_t)r;
    if (dense) {
        out[q] = m0 * sx;
        out[q + 1] = m0 * sy;
        out[q + 2] = m0 * sz;
    } else {
        out[q] += m0 * sx;
        out[q + 1] += m0 * sy;
        out[q + 2] += m0 * sz;
    }
}

// --------------------------------------------------------------- A8: momentum

__device__ __forceinline__ double block_sum_d(double v, double *lds)
{
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
        __syncthreads();
    }
    const double r = lds[0];
    __syncthreads();
    return r;
}

template <class Acc>
__global__ __launch_bounds__(256) void k_mom_partial(Acc acc, const float *__restrict__ a,
                                                     const float *__restrict__ mass,
                                                     double *__restrict__ part)
{
    __shared__ double lds[256];
    const int tile = blockIdx.x;
    const SegParams &S = acc.get(acc.seg_of_tile(tile));
    const int64_t r0 = (int64_t)(tile - S.tile_off) * kMomTile;
    const int64_t r1 = min(r0 + kMomTile, (int64_t)S.n_active);
    double sx = 0, sy = 0, sz = 0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
        const double m = mass[S.part_off + r];
        const int64_t o3 = 3 * (S.out_off + r);
        sx += m * (double)a[o3];
        sy += m * (double)a[o3 + 1];
        sz += m * (double)a[o3 + 2];
    }
    sx = block_sum_d(sx, lds);
    sy = block_sum_d(sy, lds);
    sz = block_sum_d(sz, lds);
    if (threadIdx.x == 0) {
        part[3 * tile] = sx;
        part[3 * tile + 1] = sy;
        part[3 * tile + 2] = sz;
    }
}

template <class Acc>
__global__ void k_mom_final(Acc acc, int B, int ntiles, const double *__restrict__ part,
                            double *__restrict__ out)
{
    const int b = blockIdx.x;
    if (threadIdx.x != 0 || b >= B) return;
    const SegParams &S = acc.get(b);
    const int t1 = (b + 1 < B) ? acc.get(b + 1).tile_off : ntiles;
    double x = 0, y = 0, z = 0;
    for (int t = S.tile_off; t < t1; ++t) {
        x += part[3 * t];
        y += part[3 * t + 1];
        z += part[3 * t + 2];
    }
    out[3 * b] = x;
    out[3 * b + 1] = y;
    out[3 * b + 2] = z;
}

// --------------------------------------------------------------- dispatch

template <class F>
hipError_t with_acc(const DevArgs &a, F &&f)
{
    if (a.seg_dev) return f(ManySeg{a.seg_dev, a.L->B});
    return f(OneSeg{*a.seg_host});
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

template <class T>
T *at(const DevArgs &a, size_t off)
{
    return reinterpret_cast<T *>(a.ws + off);
}

bool all_softened(const DevArgs &a)
{
    if (a.seg_dev) return a.seg_host != nullptr && a.seg_host->pc.softened;  // host summary
    return a.seg_host->pc.softened != 0;
}

template <bool kActiveOnly>
hipError_t build_items(const DevArgs &a, int two)
{
    const Layout &L = *a.L;
    uint32_t *hdr = at<uint32_t>(a, L.hdr);
    hipError_t e = fill_u32(hdr + kHdrBucketCount, kClasses, 0, a.st);
    if (e != hipSuccess) return e;
    return with_acc(a, [&](auto acc) -> hipError_t {
        const unsigned nb = blocks_for(L.NC, 256);
        k_items_count<decltype(acc), kActiveOnly><<<nb, 256, 0, a.st>>>(
            acc, (int)L.NC, at<int>(a, L.start), at<int>(a, L.nact), at<uint32_t>(a, L.info), hdr,
            L.magic(), (int)L.N, two, a.sparse_group);
        k_items_base<<<1, 64, 0, a.st>>>(hdr, L.magic());
        k_items_write<decltype(acc), kActiveOnly><<<nb, 256, 0, a.st>>>(
            acc, (int)L.NC, at<int>(a, L.start), at<int>(a, L.nact), at<uint32_t>(a, L.info), hdr,
            at<int4>(a, L.items), two, a.sparse_group);
        return hipGetLastError();
    });
}

// Symmetric tiles: partial-slot counts and the scan of their cell totals, the go/no-go decision
// (hdr[kHdrSymOk]) and the items.  Must precede build_items, whose dense
// items then take only the non-dense sources.  With the tiles switched off
// the decision is no.
unsigned persistent_grid(const DevArgs &a);

hipError_t build_sym(const DevArgs &a)
{
    const Layout &L = *a.L;
    uint32_t *hdr = at<uint32_t>(a, L.hdr);
    hipError_t e = fill_u32(hdr + kHdrSymTotal, 7, 0, a.st);  // total, ok, n_items, work, longest
    if (e != hipSuccess || a.sym_blocks <= 0) return e;
    if ((e = fill_u32(hdr + kHdrSymBucketCount, kClasses, 0, a.st)) != hipSuccess) return e;
    const int W = a.sym_window;
    return with_acc(a, [&](auto acc) -> hipError_t {
        const unsigned nb = blocks_for(L.NC, 256);
        k_sym_count<<<nb, 256, 0, a.st>>>(acc, (int)L.NC, at<int>(a, L.start), at<int>(a, L.nact),
                                          a.sym_blocks, W, a.sym_rounds,
                                          at<int>(a, L.sym_pref), at<int>(a, L.sym_tot),
                                          at<uint32_t>(a, L.sym_info), hdr, L.magic());
        hipError_t e2 = hipGetLastError();
        if (e2 != hipSuccess) return e2;
        if ((e2 = scan_i32(at<int>(a, L.sym_tot), at<int>(a, L.sym_base), L.NC, at<int>(a, L.scan_tmp),
                           a.st)) != hipSuccess)
            return e2;
        int64_t waves = persistent_grid(a);
        if (waves > L.sym_item_cap) waves = L.sym_item_cap;
        k_sym_base<<<1, 64, 0, a.st>>>(hdr, L.magic(), (long long)L.sym_cap, 1, (int)waves, a.sym_balance);
        k_sym_write<<<nb, 256, 0, a.st>>>(acc, (int)L.NC, at<int>(a, L.nact), a.sym_blocks,
                                          at<uint32_t>(a, L.sym_info), hdr, at<int4>(a, L.sym_items));
        return hipGetLastError();
    });
}

unsigned persistent_grid(const DevArgs &a)
{
    int64_t g = (int64_t)a.num_cu * a.waves_per_cu;
    if (g > a.L->item_cap) g = a.L->item_cap;
    if (g < 1) g = 1;
    return (unsigned)g;
}

Src src_of(const DevArgs &a)
{
    const Layout &L = *a.L;
    return Src{at<float>(a, L.bx), at<float>(a, L.by), at<float>(a, L.bz), at<float>(a, L.bm)};
}

}  // namespace

int64_t scan_scratch_elems(int64_t m)
{
    int64_t total = 0;
    int64_t nb = (m + kScanBlock - 1) / kScanBlock;
    while (nb > 1) {
        total += 2 * nb + 1 + 64;
        nb = (nb + kScanBlock - 1) / kScanBlock;
    }
    return total + 64;
}

hipError_t dev_zero(void *p, int64_t words, hipStream_t st) { return fill_u32(p, words, 0, st); }

hipError_t dev_scan(const int *in, int *out, int64_t m, int *tmp, hipStream_t st)
{
    return scan_i32(in, out, m, tmp, st);
}

hipError_t dev_bounds(const int *sorted_keys, int64_t n, int64_t nk, int key_bits, int *start,
                      hipStream_t st)
{
    k_cell_bounds<<<blocks_for(n + 1, 256), 256, 0, st>>>(sorted_keys, (int)n, (int)nk, key_bits, start);
    return hipGetLastError();
}

// Stable LSD radix sort of (key, value) pairs: keys in [0, 2^(passes*digit_bits)),
// values default to the element index.  The result is in keys[(passes-1)&1],
// vals[(passes-1)&1].
hipError_t radix_sort_pairs(const int *keys_in, const int *vals_in, int64_t n, int passes,
                            int digit_bits, int64_t ntiles, const RadixBufs &b, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    if (digit_bits < 1 || digit_bits > 8 || passes < 1) return hipErrorInvalidValue;
    const int *kin = keys_in;
    const int *vin = vals_in;
    const int R = 1 << digit_bits;
    hipError_t e;
    for (int p = 0; p < passes; ++p) {
        const int shift = p * digit_bits;
        int *kout = b.keys[p & 1];
        int *vout = b.vals[p & 1];
        k_radix_hist<<<(unsigned)ntiles, 256, 0, st>>>(kin, (int)n, shift, digit_bits, b.tab,
                                                     (int)ntiles);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = scan_i32(b.tab, b.tabx, (int64_t)R * ntiles, b.scan_tmp, st)) != hipSuccess) return e;
        k_radix_scatter<<<(unsigned)ntiles, kScatterWaves * kWave, 0, st>>>(kin, vin, (int)n, shift,
                                                                           digit_bits, b.tabx,
                                                        (int)ntiles, kout, vout);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        kin = kout;
        vin = vout;
    }
    return hipSuccess;
}

hipError_t dev_bin(const DevArgs &a, const float *pos, const float *mass)
{
    const Layout &L = *a.L;
    hipError_t e;
    if ((e = fill_u32(at<uint32_t>(a, L.hdr), kHdrWords, 0, a.st)) != hipSuccess) return e;
    if ((e = fill_u32(at<uint32_t>(a, L.nact), L.NC, 0, a.st)) != hipSuccess) return e;
    if (L.N == 0) return hipSuccess;
    e = with_acc(a, [&](auto acc) -> hipError_t {
        k_bin_cells<<<blocks_for(L.N, 256), 256, 0, a.st>>>(acc, pos, mass, (int)L.N, L.key_bits, L.code_bits,
                                                             at<int>(a, L.cell_of), at<int>(a, L.skey),
                                                             at<float4>(a, L.packed),
                                                             at<uint32_t>(a, L.hdr));
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    RadixBufs rb{{at<int>(a, L.keys[0]), at<int>(a, L.keys[1])},
                 {at<int>(a, L.vals[0]), at<int>(a, L.vals[1])},
                 at<int>(a, L.tab), at<int>(a, L.tabx), at<int>(a, L.scan_tmp)};
    if ((e = radix_sort_pairs(at<int>(a, L.skey), nullptr, L.N, L.passes, L.digit_bits, L.ntiles, rb,
                              a.st)) != hipSuccess)
        return e;
    if ((e = dev_bounds(at<int>(a, L.sorted_keys()), L.N, L.NC, L.key_bits, at<int>(a, L.start),
                        a.st)) != hipSuccess)
        return e;
    return with_acc(a, [&](auto acc) -> hipError_t {
        k_gather<<<blocks_for(L.N, 256), 256, 0, a.st>>>(
            acc, (int)L.N, at<int>(a, L.perm()), at<int>(a, L.sorted_keys()), at<int>(a, L.start),
            at<float4>(a, L.packed), at<float>(a, L.bx), at<float>(a, L.by), at<float>(a, L.bz), at<float>(a, L.bm),
            at<int>(a, L.out_row), at<int>(a, L.nact), L.key_bits, at<uint32_t>(a, L.hdr), L.magic());
        return hipGetLastError();
    });
}

template <class Acc, bool kSoft, int kOcc>
void launch_force(const DevArgs &a, Acc acc, float *acc_out)
{
    const Layout &L = *a.L;
    k_force<Acc, kSoft, kOcc><<<persistent_grid(a), kWave, 0, a.st>>>(
        acc, at<int4>(a, L.items), at<uint32_t>(a, L.hdr), at<int>(a, L.start), at<int>(a, L.nact),
        src_of(a), at<int>(a, L.out_row), acc_out, a.n_rows, a.pull_limit);
}

template <class Acc, bool kSoft, int kOcc>
void launch_vjp(const DevArgs &a, Acc acc, float *grad)
{
    const Layout &L = *a.L;
    k_vjp<Acc, kSoft, kOcc><<<persistent_grid(a), kWave, 0, a.st>>>(
        acc, at<int4>(a, L.items), at<uint32_t>(a, L.hdr), at<int>(a, L.start), at<int>(a, L.nact),
        src_of(a), at<float>(a, L.gx), at<float>(a, L.gy), at<float>(a, L.gz), at<int>(a, L.perm()),
        grad, (int)L.N, a.pull_limit);
}

template <class Acc, bool kSoft, int kW, int kOcc>
void launch_force_sym_v(const DevArgs &a, Acc acc, unsigned grid)
{
    const Layout &L = *a.L;
    k_force_sym<Acc, kSoft, kW, kOcc><<<grid, kWave, 0, a.st>>>(
        acc, at<int4>(a, L.sym_items), at<uint32_t>(a, L.hdr), at<int>(a, L.start), at<int>(a, L.nact),
        at<int>(a, L.sym_base), at<int>(a, L.sym_pref), src_of(a), at<float>(a, L.sym_pool), a.sym_blocks,
        a.sym_rounds, a.pull_limit);
}

template <class Acc, bool kSoft>
void launch_force_sym(const DevArgs &a, Acc acc)
{
    unsigned grid = persistent_grid(a);
    if ((int64_t)grid > a.L->sym_item_cap) grid = (unsigned)a.L->sym_item_cap;
    if (a.sym_window >= 512) {
        if (a.sym_occupancy >= 6) launch_force_sym_v<Acc, kSoft, 512, 6>(a, acc, grid);
        else if (a.sym_occupancy >= 5) launch_force_sym_v<Acc, kSoft, 512, 5>(a, acc, grid);
        else launch_force_sym_v<Acc, kSoft, 512, 0>(a, acc, grid);
    } else {
        if (a.sym_occupancy >= 6) launch_force_sym_v<Acc, kSoft, 256, 6>(a, acc, grid);
        else if (a.sym_occupancy >= 5) launch_force_sym_v<Acc, kSoft, 256, 5>(a, acc, grid);
        else launch_force_sym_v<Acc, kSoft, 256, 0>(a, acc, grid);
    }
}

template <class Acc, bool kSoft, int kW, int kOcc>
void launch_vjp_sym_v(const DevArgs &a, Acc acc, unsigned grid)
{
    const Layout &L = *a.L;
    k_vjp_sym<Acc, kSoft, kW, kOcc><<<grid, kWave, 0, a.st>>>(
        acc, at<int4>(a, L.sym_items), at<uint32_t>(a, L.hdr), at<int>(a, L.start), at<int>(a, L.nact),
        at<int>(a, L.sym_base), at<int>(a, L.sym_pref), src_of(a), at<float>(a, L.gx), at<float>(a, L.gy),
        at<float>(a, L.gz), at<float>(a, L.sym_pool), a.sym_blocks, a.sym_rounds, a.pull_limit);
}

template <class Acc, bool kSoft>
void launch_vjp_sym(const DevArgs &a, Acc acc)
{
    unsigned grid = persistent_grid(a);
    if ((int64_t)grid > a.L->sym_item_cap) grid = (unsigned)a.L->sym_item_cap;
    if (a.sym_window >= 512) {
        if (a.sym_occupancy >= 5) launch_vjp_sym_v<Acc, kSoft, 512, 5>(a, acc, grid);
        else launch_vjp_sym_v<Acc, kSoft, 512, 0>(a, acc, grid);
    } else {
        if (a.sym_occupancy >= 5) launch_vjp_sym_v<Acc, kSoft, 256, 5>(a, acc, grid);
        else launch_vjp_sym_v<Acc, kSoft, 256, 0>(a, acc, grid);
    }
}

// Adds the symmetric partial sums to the rows the one-sided kernel wrote.
hipError_t sym_gather(const DevArgs &a, const int *rows, float *out, int n_out, float scale)
{
    const Layout &L = *a.L;
    k_sym_gather<<<blocks_for(L.N, 256), 256, 0, a.st>>>(
        (int)L.N, L.key_bits, at<int>(a, L.sorted_keys()), at<int>(a, L.start), at<int>(a, L.nact),
        at<int>(a, L.sym_pref), at<int>(a, L.sym_base), at<float>(a, L.sym_pool), rows, at<float>(a, L.bm),
        at<uint32_t>(a, L.hdr), out, n_out, scale);
    return hipGetLastError();
}

hipError_t dev_force(const DevArgs &a, float *acc_out)
{
    hipError_t e = build_sym(a);
    if (e != hipSuccess) return e;
    e = build_items<true>(a, a.targets_per_lane >= 2 ? 1 : 0);
    if (e != hipSuccess) return e;
    const bool soft = all_softened(a);
    return with_acc(a, [&](auto acc) -> hipError_t {
        using A = decltype(acc);
        void *tok = nullptr;
        timing_begin("force", a.st, &tok);
        if (soft) {
            if (a.occupancy >= 8) launch_force<A, true, 8>(a, acc, acc_out);
            else if (a.occupancy >= 6) launch_force<A, true, 6>(a, acc, acc_out);
            else launch_force<A, true, 0>(a, acc, acc_out);
        } else {
            if (a.occupancy >= 8) launch_force<A, false, 8>(a, acc, acc_out);
            else if (a.occupancy >= 6) launch_force<A, false, 6>(a, acc, acc_out);
            else launch_force<A, false, 0>(a, acc, acc_out);
        }
        hipError_t le = hipGetLastError();
        if (le == hipSuccess && a.sym_blocks > 0) {
            // dense pairs once each; the device skips both when the tiles are off
            if (soft) launch_force_sym<A, true>(a, acc);
            else launch_force_sym<A, false>(a, acc);
            if ((le = hipGetLastError()) == hipSuccess)
                le = sym_gather(a, at<int>(a, a.L->out_row), acc_out, a.n_rows, 1.0f);
        }
        timing_end(tok, a.st);
        return le;
    });
}

hipError_t dev_vjp(const DevArgs &a, const float *g, float *grad)
{
    const Layout &L = *a.L;
    k_gather_g<<<blocks_for(L.N, 256), 256, 0, a.st>>>((int)L.N, a.n_rows, at<int>(a, L.out_row), g,
                                                      at<float>(a, L.gx), at<float>(a, L.gy),
                                                      at<float>(a, L.gz));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = build_sym(a)) != hipSuccess) return e;
    if ((e = build_items<false>(a, a.targets_per_lane >= 2 ? 1 : 0)) != hipSuccess) return e;
    const bool soft = all_softened(a);
    return with_acc(a, [&](auto acc) -> hipError_t {
        using A = decltype(acc);
        void *tok = nullptr;
        timing_begin("vjp", a.st, &tok);
        // the adjoint kernel spills at 8 waves per SIMD: 6 is its tightest hint
        if (soft) {
            if (a.occupancy >= 6) launch_vjp<A, true, 6>(a, acc, grad);
            else launch_vjp<A, true, 0>(a, acc, grad);
        } else {
            if (a.occupancy >= 6) launch_vjp<A, false, 6>(a, acc, grad);
            else launch_vjp<A, false, 0>(a, acc, grad);
        }
        hipError_t le = hipGetLastError();
        if (le == hipSuccess && a.sym_blocks > 0) {
            if (soft) launch_vjp_sym<A, true>(a, acc);
            else launch_vjp_sym<A, false>(a, acc);
            if ((le = hipGetLastError()) == hipSuccess)
                le = sym_gather(a, at<int>(a, a.L->perm()), grad, (int)a.L->N, -3.0f);
        }
        timing_end(tok, a.st);
        return le;
    });
}

__global__ void k_copy_pairs(const uint32_t *hdr, int64_t *out)
{
    if (threadIdx.x == 0) *out = *(const int64_t *)&hdr[kHdrPairs];
}

hipError_t dev_count_pairs(const DevArgs &a, bool adjoint, int64_t *pairs)
{
    const Layout &L = *a.L;
    // every ordered pair from its target's end: no symmetric tiles here
    DevArgs one = a;
    one.sym_blocks = 0;
    hipError_t e = build_sym(one);
    if (e != hipSuccess) return e;
    e = adjoint ? build_items<false>(a, 0) : build_items<true>(a, 0);
    if (e != hipSuccess) return e;
    if ((e = fill_u32(at<uint32_t>(a, L.hdr) + kHdrPairs, 2, 0, a.st)) != hipSuccess) return e;
    e = with_acc(a, [&](auto acc) -> hipError_t {
        k_count<<<persistent_grid(a), kWave, 0, a.st>>>(acc, at<int4>(a, L.items),
                                                       at<uint32_t>(a, L.hdr), at<int>(a, L.start),
                                                       at<int>(a, L.nact), src_of(a), a.pull_limit);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    k_copy_pairs<<<1, 64, 0, a.st>>>(at<uint32_t>(a, L.hdr), pairs);
    return hipGetLastError();
}

hipError_t dev_momentum(const DevArgs &a, const float *acc_rows, const float *mass, double *out)
{
    const Layout &L = *a.L;
    if (L.mom_tiles <= 0) {
        return with_acc(a, [&](auto acc) -> hipError_t {
            k_mom_final<<<(unsigned)L.B, 64, 0, a.st>>>(acc, L.B, 0, at<double>(a, L.mom), out);
            return hipGetLastError();
        });
    }
    return with_acc(a, [&](auto acc) -> hipError_t {
        k_mom_partial<<<(unsigned)L.mom_tiles, 256, 0, a.st>>>(acc, acc_rows, mass, at<double>(a, L.mom));
        k_mom_final<<<(unsigned)L.B, 64, 0, a.st>>>(acc, L.B, (int)L.mom_tiles, at<double>(a, L.mom), out);
        return hipGetLastError();
    });
}

}  // namespace sr
