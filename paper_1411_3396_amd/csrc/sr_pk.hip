// Power spectrum of the particles on the fly (paper Sec. 4.1): cloud-in-cell
// deposit onto an ng^3 periodic grid, a real-to-complex FFT, |delta(k)|^2
// divided by the CIC window and averaged in bins of |k|.
//
// Device passes: the deposit into the FFT's padded in-place layout, a
// float64 mass sum in a fixed order, the FFT (rocFFT, in place), and the
// binning.  Two deposits, both reproducible bit for bit.  For ng a multiple of
// 8, particles are sorted by brick of 8^3 cells and each run of a brick's
// particles sums its weights exactly, in fixed point, into a tile of grid
// points in LDS (below).  Otherwise particles are sorted by the cell of their
// lower corner point (the binning's radix sort), a segmented scan sums each
// cell's corner contributions per wave, and every grid point adds the
// partials of its 8 cells in float64, in a fixed order.  Binning: every mode of
// the half spectrum adds w |rho_k|^2 / W(k)^2 (w = 2 for modes whose mirror
// is not stored) into per-wave float64 bins in LDS by segmented sums along
// rows; a workgroup adds its waves' bins in wave order, and a last pass adds
// the workgroups' partials with a fixed tree.  The spectrum is reproducible
// bit for bit too.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include <rocfft/rocfft.h>

#include "sr_internal.h"

namespace sr {
namespace {

constexpr int kBinBlocks = 1024;  // workgroups of the binning pass
constexpr int kSumBlocks = 256;  // workgroups of the mass sum
constexpr int kMaxBins = 2048;
constexpr int kMaxGrid = 1024;  // ng^3 cell keys fit 30 bits

// Sorted deposit, step 1: per particle the grid cell of its lower corner
// point (the sort key) and (f_x, f_y, f_z, m), by the same wrap rule.
__global__ __launch_bounds__(256) void k_cic_key(const float *__restrict__ pos,
                                                 const float *__restrict__ mass, int n, int ng,
                                                 float inv_h, int *__restrict__ key,
                                                 float4 *__restrict__ pf)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float fng = (float)ng;
    int i0[3];
    float f[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        float u = pos[3 * (int64_t)i + d] * inv_h;
        // for 0 <= u < ng, u / ng rounds below 1, so the wrap is the identity
        if (!(u >= 0.f && u < fng)) u = u - floorf(u / fng) * fng;
        float fk = floorf(u);
        float fr = u - fk;
        // u rounded up to ng wraps to 0; a NaN (from a non-finite position)
        // takes cell 0 and keeps its NaN weights
        if (fk >= fng || fk < 0.f) {
            fk = 0.f;
            fr = 0.f;
        } else if (fk != fk) {
            fk = 0.f;
        }
        i0[d] = (int)fk;
        f[d] = fr;
    }
    key[i] = (i0[0] * ng + i0[1]) * ng + i0[2];
    pf[i] = make_float4(f[0], f[1], f[2], mass[i]);
}

__global__ __launch_bounds__(256) void k_cic_pack(const int *__restrict__ perm, int n,
                                                  const float4 *__restrict__ pf,
                                                  float4 *__restrict__ spf)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) spf[i] = pf[perm[i]];
}

// Sorted deposit, step 2: each particle's 8 corner contributions
// m w_x w_y w_z (float products, widened to float64), summed over the runs of
// equal cells inside each 64-slot wave of the sorted order by a segmented
// scan.  The last slot of each run stores the run's 8 sums at seg[8 slot + k],
// k = 4 c_x + 2 c_y + c_z for the corner point (lower corner + (c_x, c_y, c_z)).
// A cell's particles thus end up as one partial per wave they touch, stored
// at the wave's last slot inside the cell and at the cell's last slot.
__global__ __launch_bounds__(256) void k_cic_runs(const int *__restrict__ skey,
                                                  const float4 *__restrict__ spf, int n,
                                                  double *__restrict__ seg)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool valid = i < n;
    const int key = valid ? skey[i] : -1;
    const float4 v = valid ? spf[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    double c[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float wx = (k & 4) ? v.x : 1.f - v.x;
        const float wy = (k & 2) ? v.y : 1.f - v.y;
        const float wz = (k & 1) ? v.z : 1.f - v.z;
        c[k] = (double)(v.w * wx * wy * wz);
    }
    const int prev = __shfl_up(key, 1);
    const uint64_t heads = __ballot(lane == 0 || prev != key);
    const uint64_t upto = (lane == 63) ? heads : (heads & ((2ull << lane) - 1));
    const int first = 63 - __clzll(upto);  // first lane of this run
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const double y = __shfl_up(c[k], o);
            if (lane - o >= first) c[k] += y;
        }
    }
    const int next = __shfl_down(key, 1);
    if (valid && (lane == 63 || next != key)) {
        double *out = seg + 8 * (int64_t)i;
#pragma unroll
        for (int k = 0; k < 8; ++k) out[k] = c[k];
    }
}

// Sorted deposit, step 3: every grid point adds, in float64 and a fixed order,
// the partials of the 8 cells whose lower corner is the point or its lower
// neighbours (cells (p - c) for c in {0,1}^3, periodic): for a cell of slots
// [a, b), the partials at the last slot of each 64-slot wave below b - 1, then
// at b - 1.
__global__ __launch_bounds__(256) void k_cic_points(const int *__restrict__ cstart,
                                                    const double *__restrict__ seg, int ng, int pad,
                                                    float *__restrict__ grid)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t total = (int64_t)ng * ng * ng;
    if (g >= total) return;
    const int iz = (int)(g % ng);
    const int64_t r = g / ng;
    const int iy = (int)(r % ng), ix = (int)(r / ng);
    const int zm = iz == 0 ? ng - 1 : iz - 1;
    double sum = 0.0;
#pragma unroll
    for (int cx = 0; cx < 2; ++cx) {
        const int x = cx ? (ix == 0 ? ng - 1 : ix - 1) : ix;
#pragma unroll
        for (int cy = 0; cy < 2; ++cy) {
            const int y = cy ? (iy == 0 ? ng - 1 : iy - 1) : iy;
            // cells (x, y, iz) and (x, y, zm): their slot ranges share the bound at
            // (x, y, iz) unless zm wrapped to the end of the row
            const int row = (x * ng + y) * ng;
            const int s0 = cstart[row + iz], e0 = cstart[row + iz + 1];
            const int sm = cstart[row + zm], em = iz == 0 ? cstart[row + ng] : s0;
#pragma unroll
            for (int cz = 0; cz < 2; ++cz) {
                const int a = cz ? sm : s0, b = cz ? em : e0;
                if (a < b) {
                    const int k = 4 * cx + 2 * cy + cz;
                    for (int p = a | 63; p < b - 1; p += 64) sum += seg[8 * (int64_t)p + k];
                    sum += seg[8 * (int64_t)(b - 1) + k];
                }
            }
        }
    }
    grid[((int64_t)ix * ng + iy) * pad + iz] = (float)sum;
}

// ------------------------------------------------------------ brick deposit
//
// For grids whose side is a multiple of 8 the deposit works per brick of 8^3
// cells.  Particles are sorted by brick only (a key of 3 log2(ng / 8) bits, so
// fewer radix passes than a sort by cell), and the passes move each particle's
// 16-byte payload along with its key, so no gather follows the sort.  Each
// workgroup then adds the 8 corner weights of up to kChunk consecutive
// particles of one brick into a 9^3 tile of grid points in LDS, and a last pass
// adds, for every grid point, the tiles that cover it.
//
// Tile sums are exact integers: a weight c = m w_x w_y w_z (float32 products,
// as in the cell deposit) is scaled by S = 2^(62 - e), where e bounds
// kChunk max|m| < 2^e, and split into x = c S = hi + lo 2^-32 with hi =
// floor(x) and lo = round((x - hi) 2^32).  |x| < 2^51, so hi sums over a
// chunk stay below 2^62 in magnitude and lo sums below 2^43, and integer sums do not depend on their order,
// so every tile is the same whatever order the LDS atomics land in.  x is exact
// in float64 (c has 24 significant bits, S is a power of two), so only weights
// below 2^(e - 71) lose bits, by at most 2^(e - 95).  A tile point holds
// hi / S + lo / (2^32 S), computed in float64 and rounded to float32; chunk boundaries are fixed by
// the stable sort, and the last pass adds the tiles in a fixed order in float64.
// A non-finite weight makes its whole tile NaN, so it still reaches the
// spectrum.

constexpr int kBrick = 8;                                   // cells per brick side
constexpr int kTile = kBrick + 1;                           // grid points per tile side
constexpr int kTilePts = kTile * kTile * kTile;             // 729
constexpr int kChunk = 2048;                                // most particles per workgroup
constexpr int kSortThreads = 256;                           // four waves per sort tile
constexpr int kSortSteps = kRadixTile / kSortThreads;
constexpr double kMagic52 = 6755399441055744.0;             // 1.5 * 2^52

// Brick of particle i (the sort key) and its payload (lu_x, lu_y, lu_z, m), lu
// the coordinate in grid units from the brick's lower corner.  u wraps by the
// cell deposit's rule; lu = u - 8 b is exact (Sterbenz), so floor(lu) and
// lu - floor(lu) are the cell deposit's cell offset and fraction bit for bit.
__device__ __forceinline__ void brick_of(const float (&x)[3], float m, int ng, float inv_h, int &key, float4 &v)
{
    const float fng = (float)ng;
    const int nb = ng / kBrick;
    int b[3];
    float lu[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        float u = x[d] * inv_h;
        // for 0 <= u < ng, u / ng rounds below 1, so the wrap is the identity
        if (!(u >= 0.f && u < fng)) u = u - floorf(u / fng) * fng;
        float fk = floorf(u);
        // u rounded up to ng wraps to 0; a NaN (from a non-finite position)
        // takes brick 0 and keeps its NaN payload
        if (fk >= fng || fk < 0.f) {
            fk = 0.f;
            u = 0.f;
        } else if (fk != fk) {
            fk = 0.f;
        }
        const int k = (int)fk;
        b[d] = k / kBrick;
        lu[d] = u - (float)(b[d] * kBrick);
    }
    key = (b[0] * nb + b[1]) * nb + b[2];
    v = make_float4(lu[0], lu[1], lu[2], m);
}

// Keys and payloads of one tile of kRadixTile particles, the first sort
// pass's digit counts of the tile (table[d * ntiles + tile]), and the tile's
// float64 mass sum (a fixed order per thread, then a fixed tree) and largest
// |m|.
__global__ __launch_bounds__(kSortThreads) void k_brick_hist0(const float *__restrict__ pos,
                                                              const float *__restrict__ mass, int n,
                                                              int ng, float inv_h, int bits,
                                                              int *__restrict__ table, int ntiles,
                                                              int *__restrict__ keys,
                                                              float4 *__restrict__ vals,
                                                              double *__restrict__ msum,
                                                              float *__restrict__ mmax)
{
    __shared__ int h[256];
    __shared__ double ls[kSortThreads];
    __shared__ float lm[kSortThreads];
    __shared__ float4 lp4[3 * kRadixTile / 4];  // the tile's positions, staged with 16-byte loads
    const float *lp = reinterpret_cast<const float *>(lp4);
    const int tid = threadIdx.x;
    const int R = 1 << bits;
    if (tid < R) h[tid] = 0;
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
    const int nt = (int)min((int64_t)kRadixTile, (int64_t)n - base);
    {
        // 3 nt floats from pos + 3 base, as float4 when pos is 16-byte aligned
        // (then so is pos + 3 base: base is a multiple of 2048)
        const int nf = 3 * nt;
        const int n4 = (reinterpret_cast<uintptr_t>(pos) & 15) == 0 ? nf / 4 : 0;
        const float4 *g4 = reinterpret_cast<const float4 *>(pos + 3 * base);
        for (int j = tid; j < n4; j += kSortThreads) lp4[j] = g4[j];
        float *lpw = reinterpret_cast<float *>(lp4);
        for (int j = 4 * n4 + tid; j < nf; j += kSortThreads) lpw[j] = pos[3 * base + j];
    }
    __syncthreads();
    double s = 0.0;
    float mx = 0.f;
    for (int r = 0; r < kSortSteps; ++r) {
        const int e = r * kSortThreads + tid;
        const int64_t i = base + e;
        if (e < nt) {
            int key;
            float4 v;
            const float x[3] = {lp[3 * e], lp[3 * e + 1], lp[3 * e + 2]};
            brick_of(x, mass[i], ng, inv_h, key, v);
            keys[i] = key;
            vals[i] = v;
            atomicAdd(&h[key & (R - 1)], 1);
            s += (double)v.w;
            mx = fmaxf(mx, fabsf(v.w));
        }
    }
    ls[tid] = s;
    lm[tid] = mx;
    __syncthreads();
    for (int o = kSortThreads / 2; o > 0; o >>= 1) {
        if (tid < o) {
            ls[tid] += ls[tid + o];
            lm[tid] = fmaxf(lm[tid], lm[tid + o]);
        }
        __syncthreads();
    }
    if (tid < R) table[(int64_t)tid * ntiles + blockIdx.x] = h[tid];
    if (tid == 0) {
        msum[blockIdx.x] = ls[0];
        mmax[blockIdx.x] = lm[0];
    }
}

// Later sort passes, histogram side: digit counts of one tile of keys.  Each
// thread takes kSortSteps consecutive keys and adds each run of equal digits
// with one LDS atomic (sorted, clustered keys come in long runs).
__global__ __launch_bounds__(kSortThreads) void k_brick_hist(const int *__restrict__ keys, int n, int shift,
                                                             int bits, int *__restrict__ table, int ntiles)
{
    __shared__ int h[256];
    const int tid = threadIdx.x;
    const int R = 1 << bits;
    if (tid < R) h[tid] = 0;
    __syncthreads();
    const int64_t e0 = (int64_t)blockIdx.x * kRadixTile + (int64_t)tid * kSortSteps;
    static_assert(kSortSteps == 8, "two int4 loads per thread");
    int d[kSortSteps];
    if (e0 + kSortSteps <= n) {
        // keys is 16-byte aligned and e0 a multiple of 8
        const int4 *k4 = reinterpret_cast<const int4 *>(keys + e0);
        const int4 a = k4[0], b = k4[1];
        const int k[kSortSteps] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
        for (int j = 0; j < kSortSteps; ++j) d[j] = (k[j] >> shift) & (R - 1);
    } else {
        // the tail: digits past n are -1 and come last
#pragma unroll
        for (int j = 0; j < kSortSteps; ++j) d[j] = e0 + j < n ? (keys[e0 + j] >> shift) & (R - 1) : -1;
    }
    int cur = d[0], run = 1;
#pragma unroll
    for (int j = 1; j < kSortSteps; ++j) {
        if (d[j] == cur) {
            ++run;
        } else {
            if (cur >= 0) atomicAdd(&h[cur], run);
            cur = d[j];
            run = 1;
        }
    }
    if (cur >= 0) atomicAdd(&h[cur], run);
    __syncthreads();
    if (tid < R) table[(int64_t)tid * ntiles + blockIdx.x] = h[tid];
}

// Stable scatter of one tile: each wave ranks 64 particles at a time within
// their digit (one ballot per digit bit, per-wave digit counters), the tile is
// reordered by digit in LDS keeping input order inside a digit, and each
// digit's run is written to consecutive addresses from the scanned table.
__global__ __launch_bounds__(kSortThreads) void k_brick_scatter(
    const int *__restrict__ keys_in, const float4 *__restrict__ v_in, int n, int shift, int bits,
    const int *__restrict__ table_x, int ntiles, int *__restrict__ keys_out, float4 *__restrict__ v_out)
{
    constexpr int kWaves = kSortThreads / kWave;
    constexpr int kPerWave = kRadixTile / kWaves;
    __shared__ int cnt[kWaves][256];
    __shared__ int lstart[256];
    __shared__ int gstart[256];
    __shared__ int wsum[kWaves];
    __shared__ int lkey[kRadixTile];
    __shared__ float4 lv[kRadixTile];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int R = 1 << bits;
    // tiles renumbered so that each XCD takes a contiguous run of them: a
    // digit's runs from neighbouring tiles are neighbours in the output, and
    // their partial cache lines then merge in one L2
    const int tile = ntiles % kXcds == 0 ? (int)((blockIdx.x % kXcds) * (ntiles / kXcds) + blockIdx.x / kXcds)
                                         : (int)blockIdx.x;
    gstart[tid] = tid < R ? table_x[(int64_t)tid * ntiles + tile] : 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) cnt[w][tid] = 0;
    __syncthreads();
    const int64_t tile0 = (int64_t)tile * kRadixTile;
    const int64_t base = tile0 + (int64_t)wv * kPerWave;
    const uint64_t below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    int key[kSortSteps], rk[kSortSteps];
    float4 v[kSortSteps];
#pragma unroll
    for (int r = 0; r < kSortSteps; ++r) {
        const int64_t e = base + r * kWave + lane;
        const bool valid = e < n;
        key[r] = 0;
        v[r] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (valid) {
            key[r] = keys_in[e];
            v[r] = v_in[e];
        }
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
    int tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        const int c = cnt[w][tid];
        cnt[w][tid] = tot;
        tot += c;
    }
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
    for (int w = 0; w < kWaves; ++w) prior += w < wv ? wsum[w] : 0;
    lstart[tid] = prior + incl - tot;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortSteps; ++r) {
        if (rk[r] >= 0) {
            const int d = (key[r] >> shift) & (R - 1);
            const int at = lstart[d] + cnt[wv][d] + rk[r];
            lkey[at] = key[r];
            lv[at] = v[r];
        }
    }
    __syncthreads();
    const int n_tile = (int)min((int64_t)kRadixTile, (int64_t)n - tile0);
    for (int i = tid; i < n_tile; i += kSortThreads) {
        const int k = lkey[i];
        const int d = (k >> shift) & (R - 1);
        const int dest = gstart[d] + (i - lstart[d]);
        keys_out[dest] = k;
        v_out[dest] = lv[i];
    }
}

// Brick starts from the sorted brick keys: slot b starts every brick in
// (key[b-1], key[b]], and slot n every brick after the last key, so each
// entry of start[0 .. nbricks] is written once.  Four keys per thread.
__global__ __launch_bounds__(256) void k_brick_bounds(const int *__restrict__ key, int n, int nbricks,
                                                      int *__restrict__ start)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t b0 = 4 * q;  // slots b0 .. b0 + 3
    if (b0 > n) return;
    int k[5];  // k[0] = key[b0 - 1] (-1 before the first), k[1 + j] = key[b0 + j] (nbricks from n on)
    k[0] = b0 == 0 ? -1 : key[b0 - 1];
    if (b0 + 4 <= n) {
        // key is 16-byte aligned
        const int4 v = reinterpret_cast<const int4 *>(key)[q];
        k[1] = v.x;
        k[2] = v.y;
        k[3] = v.z;
        k[4] = v.w;
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) k[1 + j] = b0 + j < n ? key[b0 + j] : nbricks;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (b0 + j > n) break;
        for (int c = k[j] + 1; c <= k[j + 1]; ++c) start[c] = (int)(b0 + j);
    }
}

// Total mass (the tiles' sums in tile order, then a fixed tree) into out[0]
// and the largest |m| into out[1], by one workgroup of 256 threads.
__device__ __forceinline__ void mass_totals(const double *__restrict__ msum, const float *__restrict__ mmax,
                                            int tiles, double *__restrict__ out)
{
    __shared__ double ls[256];
    __shared__ float lm[256];
    const int tid = threadIdx.x;
    double s = 0.0;
    float mx = 0.f;
    // eight loads in flight per thread, then added in the same order as a
    // plain strided loop (a missing partial adds 0, which leaves s as it is)
    constexpr int kU = 8;
    for (int t0 = tid; t0 < tiles; t0 += kU * 256) {
        double v[kU];
        float m[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int t = t0 + u * 256;
            v[u] = t < tiles ? msum[t] : 0.0;
            m[u] = t < tiles ? mmax[t] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            s += v[u];
            mx = fmaxf(mx, m[u]);
        }
    }
    ls[tid] = s;
    lm[tid] = mx;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) {
            ls[tid] += ls[tid + o];
            lm[tid] = fmaxf(lm[tid], lm[tid + o]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        out[0] = ls[0];
        out[1] = (double)lm[0];
    }
}

__global__ __launch_bounds__(256) void k_brick_mass(const double *__restrict__ msum,
                                                    const float *__restrict__ mmax, int tiles,
                                                    double *__restrict__ out)
{
    mass_totals(msum, mmax, tiles, out);
}

// Workgroups of each brick: ceil(particles / kChunk), none for an empty brick.
// Workgroup 0 also takes the mass totals (k_brick_mass's sums).
__global__ __launch_bounds__(256) void k_brick_chunks(const int *__restrict__ bstart, int nbricks,
                                                      int *__restrict__ chunks,
                                                      const double *__restrict__ msum,
                                                      const float *__restrict__ mmax, int tiles,
                                                      double *__restrict__ mstat)
{
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b < nbricks) {
        const int np = bstart[b + 1] - bstart[b];
        chunks[b] = (np + kChunk - 1) / kChunk;
    }
    if (blockIdx.x == 0) mass_totals(msum, mmax, tiles, mstat);
}

// Every chunk's record: its brick and its range of sorted particles.
__global__ __launch_bounds__(256) void k_brick_owner(const int *__restrict__ bstart,
                                                     const int *__restrict__ cbase, int nbricks,
                                                     int4 *__restrict__ rec)
{
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= nbricks) return;
    const int s0 = bstart[b], s1 = bstart[b + 1];
    for (int w = cbase[b], p = s0; w < cbase[b + 1]; ++w, p += kChunk)
        rec[w] = make_int4(b, p, min(p + kChunk, s1), 0);
}

// One chunk of one brick: exact integer corner sums in a 9^3 LDS tile, then
// the tile as float32 into chunk slot w of ctile.  Launched with at least as
// many workgroups as chunks; the others leave at once.
__global__ __launch_bounds__(256) void k_brick_tile(const int *__restrict__ cbase, int nbricks,
                                                    const int4 *__restrict__ rec,
                                                    const float4 *__restrict__ v_sorted,
                                                    const double *__restrict__ mstat,
                                                    float *__restrict__ ctile)
{
    __shared__ unsigned long long thi[kTilePts];
    __shared__ unsigned long long tlo[kTilePts];
    __shared__ int bad;  // a non-finite weight: the whole tile becomes NaN
    const int w = blockIdx.x;
    // independent loads: the chunk count, this chunk's record, the mass bound
    const int nchunks = cbase[nbricks];
    const int4 r = rec[min(w, nchunks > 0 ? nchunks - 1 : 0)];
    const double mmax = mstat[1];
    if (w >= nchunks) return;  // uniform over the workgroup
    for (int t = threadIdx.x; t < kTilePts; t += 256) {
        thi[t] = 0ull;
        tlo[t] = 0ull;
    }
    if (threadIdx.x == 0) bad = 0;
    int e = 0;
    const double bound = (double)kChunk * mmax;
    if (bound > 0.0) (void)frexp(bound, &e);  // bound < 2^e
    const double S = ldexp(1.0, 62 - e);
    __syncthreads();
    for (int p = r.y + (int)threadIdx.x; p < r.z; p += 256) {
        const float4 v = v_sorted[p];
        // offsets in [0, 7] for any payload (fmaxf drops a NaN; its weights stay NaN)
        const float lx = fminf(fmaxf(floorf(v.x), 0.f), 7.f);
        const float ly = fminf(fmaxf(floorf(v.y), 0.f), 7.f);
        const float lz = fminf(fmaxf(floorf(v.z), 0.f), 7.f);
        const float fx = v.x - lx, fy = v.y - ly, fz = v.z - lz;
        const int base = ((int)lx * kTile + (int)ly) * kTile + (int)lz;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const float wx = (k & 4) ? fx : 1.f - fx;
            const float wy = (k & 2) ? fy : 1.f - fy;
            const float wz = (k & 1) ? fz : 1.f - fz;
            const double x = (double)(v.w * wx * wy * wz) * S;
            if (!(fabs(x) < 2251799813685248.0)) {  // NaN, or not below 2^51
                bad = 1;
                continue;
            }
            // integer-valued doubles of magnitude below 2^51 to int64: added to
            // 1.5 * 2^52 they land in [2^52, 2^53), where the low bits of the
            // representation are the integer (exact); for r 2^32 the same add
            // rounds to the nearest integer, as rint would
            const double xh = floor(x);
            const double r = x - xh;
            const int at = base + (k >> 2) * kTile * kTile + ((k >> 1) & 1) * kTile + (k & 1);
            const long long hi = __double_as_longlong(xh + kMagic52) - __double_as_longlong(kMagic52);
            const long long lo = __double_as_longlong(fma(r, 4294967296.0, kMagic52)) -
                                 __double_as_longlong(kMagic52);
            if (hi != 0) atomicAdd(&thi[at], (unsigned long long)hi);
            if (lo != 0) atomicAdd(&tlo[at], (unsigned long long)lo);
        }
    }
    __syncthreads();
    float *out = ctile + (int64_t)w * kTilePts;
    const double inv_s = 1.0 / S, inv_s32 = inv_s / 4294967296.0;
    const float nan = __int_as_float(0x7fc00000);
    for (int t = threadIdx.x; t < kTilePts; t += 256)
        out[t] = bad ? nan : (float)((double)(long long)thi[t] * inv_s + (double)tlo[t] * inv_s32);
}

// Grid point (ix, iy, iz): per axis, its own brick at offset i mod 8 and, for
// i mod 8 == 0, also the brick below at tile index 8; the chunk tiles of those
// (up to 8) bricks are added in a fixed order in float64.  One thread takes
// the 8 points of a brick row along z (a workgroup covers the z bricks of one
// grid row): one lookup of a brick's chunks serves 8 independent loads, and a
// wave stores 64 x 32 contiguous bytes.
__global__ __launch_bounds__(256) void k_brick_combine(const int *__restrict__ cbase, int ng, int gx,
                                                       const float *__restrict__ ctile, int pad,
                                                       float *__restrict__ grid)
{
    const int nb = ng / kBrick;
    // workgroups go to the 8 XCDs in turn: renumbered so that each XCD takes a
    // contiguous run of rows, whose points share tiles (and so its L2)
    const unsigned nwg = gridDim.x;
    const unsigned L = nwg % kXcds == 0 ? (blockIdx.x % kXcds) * (nwg / kXcds) + blockIdx.x / kXcds
                                        : blockIdx.x;
    const int row = (int)(L / (unsigned)gx);
    const int bz = (int)(L - (unsigned)row * gx) * blockDim.x + threadIdx.x;
    if (bz >= nb) return;
    const int iy = row % ng, ix = row / ng;
    const int bx = ix >> 3, by = iy >> 3;
    const int tx = ix & 7, ty = iy & 7;
    const int bzm = bz == 0 ? nb - 1 : bz - 1;
    double sum[kBrick];
#pragma unroll
    for (int k = 0; k < kBrick; ++k) sum[k] = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        if (a == 1 && tx != 0) break;
        const int px = a ? (bx == 0 ? nb - 1 : bx - 1) : bx, sx = a ? kBrick : tx;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            if (c == 1 && ty != 0) break;
            const int py = c ? (by == 0 ? nb - 1 : by - 1) : by, sy = c ? kBrick : ty;
            const int row = (sx * kTile + sy) * kTile;  // tile index of z offset 0
            const int own = (px * nb + py) * nb + bz, below = (px * nb + py) * nb + bzm;
            const int w0 = cbase[own], w1 = cbase[own + 1];
            const int v0 = cbase[below], v1 = cbase[below + 1];
            for (int w = w0; w < w1; ++w) {
                const float *t = ctile + (int64_t)w * kTilePts + row;
                float v[kBrick];
#pragma unroll
                for (int k = 0; k < kBrick; ++k) v[k] = t[k];
#pragma unroll
                for (int k = 0; k < kBrick; ++k) sum[k] += v[k];
            }
            // the brick below in z reaches only offset 0, from its tile index 8
            for (int w = v0; w < v1; ++w) sum[0] += ctile[(int64_t)w * kTilePts + row + kBrick];
        }
    }
    float *g = grid + ((int64_t)ix * ng + iy) * pad + bz * kBrick;
#pragma unroll
    for (int k = 0; k < kBrick; ++k) g[k] = (float)sum[k];
}

// Float64 sum of the masses: strided partial sums per thread, a fixed tree
// per workgroup, then one workgroup over the partials.
__device__ __forceinline__ double block_sum(double v, double *lds)
{
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
        __syncthreads();
    }
    return lds[0];
}

__global__ __launch_bounds__(256) void k_mass_partial(const float *__restrict__ mass, int n,
                                                      double *__restrict__ part)
{
    __shared__ double lds[256];
    double v = 0.0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) v += (double)mass[i];
    const double s = block_sum(v, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_mass_final(const double *__restrict__ part, int parts,
                                                    double *__restrict__ total)
{
    __shared__ double lds[256];
    double v = 0.0;
    for (int i = threadIdx.x; i < parts; i += 256) v += part[i];
    const double s = block_sum(v, lds);
    if (threadIdx.x == 0) total[0] = s;
}

// Modes of the half spectrum (iz in [0, ng/2]).  Each wave of a workgroup
// takes whole rows (ix, iy) in a fixed order and keeps its own bins in LDS.
// Along a row |n| grows with iz, so each bin is one run of consecutive modes.
// Lane l takes the S = ceil((ng/2 + 1) / 64) modes from l S on and sums its
// runs in order; a run that starts and ends inside the lane goes to the bins
// at once.  The runs at the lane edges are joined across lanes: F(l), the sum
// of lane l's last run from where it starts (possibly in earlier lanes whose
// single run it continues), is a segmented scan over the lanes, in a fixed
// tree; a lane's first run adds F(l - 1) when it continues it; and each run is
// added to the bins by the lane where it ends.  Within a row every bin is added
// once and no two lanes touch one bin in the same instruction.  The waves'
// bins are then added in wave order and written transposed,
// part[(3 b + j) blocks + workgroup], for the last pass.  The sums therefore do
// not depend on scheduling: the spectrum is bitwise reproducible.
// iw[i] = 1 / sinc^4(pi n_i / ng) for the mode index n_i of array index i.
__global__ __launch_bounds__(256) void k_pk_bins(const float2 *__restrict__ c, int ng, int n_bins,
                                                 double inv_dn, const double *__restrict__ iw,
                                                 double *__restrict__ part)
{
    extern __shared__ double bins[];  // per wave [3][n_bins]: sum of w P', sum of w |n|, sum of w
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    const int nb3 = 3 * n_bins;
    double *wb = bins + (int64_t)wv * nb3;
    for (int b = threadIdx.x; b < nw * nb3; b += blockDim.x) bins[b] = 0.0;
    __syncthreads();
    const int nzh = ng / 2 + 1;
    const int S = (nzh + kWave - 1) / kWave;  // modes per lane
    const int64_t rows = (int64_t)ng * ng;
    const int64_t stride = (int64_t)gridDim.x * nw;
    const uint64_t upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1);
    auto add = [&](int key, double p, double km, double wt) {
        if (key >= 0 && key < n_bins) {
            wb[key] += p;
            wb[n_bins + key] += km;
            wb[2 * n_bins + key] += wt;
        }
    };
    for (int64_t r = (int64_t)blockIdx.x * nw + wv; r < rows; r += stride) {
        const int iy = (int)(r % ng), ix = (int)(r / ng);
        const int nx = ix <= ng / 2 ? ix : ix - ng;
        const int ny = iy <= ng / 2 ? iy : iy - ng;
        const double wxy = iw[ix] * iw[iy];
        const double r2 = (double)nx * nx + (double)ny * ny;
        // this lane's runs: the first (hk; hp, hm, hw), the current one (tk; tp, tm, tw);
        // keys: a bin, -1 for k = 0, n_bins beyond the last bin (both never added)
        int hk = -2, tk = -2, have = 0, single = 1;
        double hp = 0.0, hm = 0.0, hw = 0.0, tp = 0.0, tm = 0.0, tw = 0.0;
        for (int j = 0; j < S; ++j) {
            const int iz = lane * S + j;
            if (iz >= nzh) break;
            double p = 0.0, km = 0.0, wt = 0.0;
            const double mag = sqrt(r2 + (double)iz * iz);
            const int b = (int)floor(mag * inv_dn);
            int key = n_bins;
            if (mag == 0.0) {
                key = -1;
            } else if (b < n_bins) {
                const float2 v = c[r * nzh + iz];
                const double w = (iz == 0 || 2 * iz == ng) ? 1.0 : 2.0;
                p = w * (((double)v.x * v.x + (double)v.y * v.y) * (wxy * iw[iz]));
                km = w * mag;
                wt = w;
                key = b;
            }
            if (!have) {
                have = 1;
                hk = tk = key;
                tp = p;
                tm = km;
                tw = wt;
            } else if (key == tk) {
                tp += p;
                tm += km;
                tw += wt;
            } else {
                if (single) {  // the first run ends here: it may continue an earlier lane's
                    hp = tp;
                    hm = tm;
                    hw = tw;
                    single = 0;
                } else {  // a run inside this lane
                    add(tk, tp, tm, tw);
                }
                tk = key;
                tp = p;
                tm = km;
                tw = wt;
            }
        }
        // F: sum of this lane's last run from its start, over the lanes whose single run it continues
        const int ptk = __shfl_up(tk, 1), phave = __shfl_up(have, 1);
        const bool joins = lane > 0 && have && phave && ptk == hk;  // first run continues lane l - 1's last
        const bool cont = joins && single;
        const uint64_t heads = __ballot(!cont);
        const int first = 63 - __clzll(heads & upto);
        double fp = tp, fm = tm, fw = tw;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const double yp = __shfl_up(fp, o), ym = __shfl_up(fm, o), yw = __shfl_up(fw, o);
            if (lane - o >= first) {
                fp += yp;
                fm += ym;
                fw += yw;
            }
        }
        const double cp = __shfl_up(fp, 1), cm = __shfl_up(fm, 1), cw = __shfl_up(fw, 1);
        // a first run that ends inside this lane, with what it continues
        if (have && !single) {
            if (joins) add(hk, hp + cp, hm + cm, hw + cw);
            else add(hk, hp, hm, hw);
        }
        // the last run, by the lane where it ends
        const int nhk = __shfl_down(hk, 1), nhave = __shfl_down(have, 1);
        const bool goes_on = lane < kWave - 1 && nhave && nhk == tk;
        if (have && !goes_on) add(tk, fp, fm, fw);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nb3; b += blockDim.x) {
        double t = bins[b];
        for (int w = 1; w < nw; ++w) t += bins[(int64_t)w * nb3 + b];
        part[(int64_t)b * gridDim.x + blockIdx.x] = t;
    }
}

// One workgroup per bin: the workgroups' partials of each sum added with a
// fixed stride per thread and a fixed tree.
// P(bin) = box^3 / M^2 * sum(w P') / sum(w), k = 2 pi / box * sum(w |n|) / sum(w).
__global__ __launch_bounds__(256) void k_pk_final(const double *__restrict__ part, int blocks,
                                                  int n_bins, const double *__restrict__ mtot,
                                                  double box, double *__restrict__ pk,
                                                  double *__restrict__ kmean,
                                                  int64_t *__restrict__ modes)
{
    __shared__ double red[3][256];
    const int b = blockIdx.x, t = threadIdx.x;
    double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const double *q = part + (int64_t)(j * n_bins + b) * blocks;
        for (int g = t; g < blocks; g += 256) acc[j] += q[g];
        red[j][t] = acc[j];
    }
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) {
#pragma unroll
            for (int j = 0; j < 3; ++j) red[j][t] += red[j][t + o];
        }
        __syncthreads();
    }
    if (t != 0) return;
    const double sp = red[0][0], sk = red[1][0], sw = red[2][0];
    const double M = mtot[0];
    const double two_pi = 6.283185307179586476925;
    pk[b] = sw > 0.0 ? sp / sw * box * box * box / (M * M) : 0.0;
    if (kmean) kmean[b] = sw > 0.0 ? sk / sw * two_pi / box : 0.0;
    if (modes) modes[b] = (int64_t)(sw + 0.5);
}

// iw[i] = 1 / sinc^4(pi n / ng) for the mode index n of array index i.
__global__ __launch_bounds__(256) void k_pk_sinc(int ng, double *__restrict__ iw)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= ng) return;
    const int nm = i <= ng / 2 ? i : i - ng;
    const double x = 3.14159265358979323846 * nm / ng;
    const double s = nm == 0 ? 1.0 : sin(x) / x;
    const double s2 = s * s;
    iw[i] = 1.0 / (s2 * s2);
}

// Waves per workgroup of the binning: up to 4, as many as their bins fit 64 KiB of LDS.
int bin_waves(int n_bins) { return std::max(1, std::min(4, 65536 / (24 * n_bins))); }

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

std::once_flag g_fft_setup;

}  // namespace
}  // namespace sr

using namespace sr;

struct sr_pk_plan {
    int ng = 0, n_bins = 0;
    double box = 0.0, dn = 1.0;
    int64_t n_max = 0;
    int passes = 1, digit_bits = 1, key_bits = 1;
    int64_t tiles = 1;
    bool brick = false;      // brick deposit (ng a multiple of 8), else the cell deposit
    int64_t nbricks = 0, max_chunks = 0;
    size_t grid_off = 0, grid_bytes = 0, sinc_off = 0, mass_off = 0, part_off = 0, work_off = 0,
           key_off[2] = {0, 0}, val_off[2] = {0, 0}, pf_off = 0, spf_off = 0, seg_off = 0, cstart_off = 0,
           tab_off = 0, tabx_off = 0, scan_off = 0, chunks_off = 0, cbase_off = 0, owner_off = 0,
           ctile_off = 0, msum_off = 0, mmax_off = 0, ws_bytes = 0;
    rocfft_plan fft = nullptr;
    size_t work_bytes = 0;
    bool fft_failed = false;
};

namespace {

// rocFFT plan, made at the first run (it compiles or loads kernels and keeps
// its twiddle tables in device memory).
sr_status ensure_fft(sr_pk_plan *P)
{
    if (P->fft) return SR_OK;
    if (P->fft_failed) return SR_E_DEVICE;
    std::call_once(g_fft_setup, [] { (void)rocfft_setup(); });
    const size_t len[3] = {(size_t)P->ng, (size_t)P->ng, (size_t)P->ng};  // fastest first
    if (rocfft_plan_create(&P->fft, rocfft_placement_inplace, rocfft_transform_type_real_forward,
                           rocfft_precision_single, 3, len, 1, nullptr) != rocfft_status_success) {
        P->fft = nullptr;
        P->fft_failed = true;
        return SR_E_DEVICE;
    }
    size_t wb = 0;
    if (rocfft_plan_get_work_buffer_size(P->fft, &wb) != rocfft_status_success) return SR_E_DEVICE;
    if (wb > P->work_bytes) {
        // the workspace was sized with the query made at plan creation
        (void)rocfft_plan_destroy(P->fft);
        P->fft = nullptr;
        P->fft_failed = true;
        return SR_E_UNSUPPORTED;
    }
    return SR_OK;
}

sr_status check_pk_ws(const sr_pk_plan *P, const void *ws, size_t ws_bytes)
{
    if (!ws || reinterpret_cast<uintptr_t>(ws) % 256 != 0 || ws_bytes < P->ws_bytes) return SR_E_WORKSPACE;
    return SR_OK;
}

sr_status deposit_bricks(sr_pk_plan *P, const float *pos, const float *mass, int64_t n, char *w,
                         hipStream_t s)
{
    float *grid = reinterpret_cast<float *>(w + P->grid_off);
    const int pad = 2 * (P->ng / 2 + 1);
    const float inv_h = (float)(P->ng / P->box);
    auto I = [&](size_t off) { return reinterpret_cast<int *>(w + off); };
    auto V = [&](size_t off) { return reinterpret_cast<float4 *>(w + off); };
    double *mstat = reinterpret_cast<double *>(w + P->mass_off) + kSumBlocks;  // total, max |m|
    const int nbricks = (int)P->nbricks;
    int *bstart = I(P->cstart_off), *cbase = I(P->cbase_off);
    float *ctile = reinterpret_cast<float *>(w + P->ctile_off);
    if (n > 0) {
        const int tiles = (int)((n + kRadixTile - 1) / kRadixTile);
        double *msum = reinterpret_cast<double *>(w + P->msum_off);
        float *mmax = reinterpret_cast<float *>(w + P->mmax_off);
        // keys and payloads (with the first pass's digit counts) into buffer
        // passes & 1, then a stable radix sort by brick moving the payloads
        // with the keys; pass p reads buffer (passes + p) & 1 and writes the
        // other, so the last lands in buffer 0
        auto K = [&](int q) { return I(P->key_off[q]); };
        auto Vb = [&](int q) { return V(q ? P->spf_off : P->pf_off); };
        const int first = P->passes & 1;
        for (int p = 0; p < P->passes; ++p) {
            // the last pass takes only the key bits left
            const int shift = p * P->digit_bits;
            const int bits = std::min(P->digit_bits, P->key_bits - shift);
            const int R = 1 << bits;
            const int in = (first + p) & 1, out = in ^ 1;
            if (p == 0)
                k_brick_hist0<<<tiles, kSortThreads, 0, s>>>(pos, mass, (int)n, P->ng, inv_h, bits,
                                                             I(P->tab_off), tiles, K(in), Vb(in), msum, mmax);
            else
                k_brick_hist<<<tiles, kSortThreads, 0, s>>>(K(in), (int)n, shift, bits, I(P->tab_off),
                                                            tiles);
            if (hipGetLastError() != hipSuccess) return SR_E_DEVICE;
            if (dev_scan(I(P->tab_off), I(P->tabx_off), (int64_t)R * tiles, I(P->scan_off), s) != hipSuccess)
                return SR_E_DEVICE;
            k_brick_scatter<<<tiles, kSortThreads, 0, s>>>(K(in), Vb(in), (int)n, shift, bits,
                                                           I(P->tabx_off), tiles, K(out), Vb(out));
            if (hipGetLastError() != hipSuccess) return SR_E_DEVICE;
        }
        k_brick_bounds<<<(unsigned)((n / 4 + 1 + 255) / 256), 256, 0, s>>>(K(0), (int)n, nbricks, bstart);
        if (hipGetLastError() != hipSuccess) return SR_E_DEVICE;
        int4 *rec = reinterpret_cast<int4 *>(w + P->owner_off);
        const unsigned bb = (unsigned)((nbricks + 255) / 256);
        k_brick_chunks<<<bb, 256, 0, s>>>(bstart, nbricks, I(P->chunks_off), msum, mmax, tiles, mstat);
        if (hipGetLastError() != hipSuccess) return SR_E_DEVICE;
        if (dev_scan(I(P->chunks_off), cbase, nbricks, I(P->scan_off), s) != hipSuccess) return SR_E_DEVICE;
        k_brick_owner<<<bb, 256, 0, s>>>(bstart, cbase, nbricks, rec);
        if (hipGetLastError() != hipSuccess) return SR_E_DEVICE;
        // workgroups: an upper bound on the chunks, sum over bricks of ceil(np / kChunk)
        const int64_t bound = n / kChunk + std::min<int64_t>(nbricks, n);
        k_brick_tile<<<(unsigned)bound, 256, 0, s>>>(cbase, nbricks, rec, Vb(0), mstat, ctile);
        if (hipGetLastError() != hipSuccess) return SR_E_DEVICE;
    } else {
        // no chunks, and a zero mass
        if (dev_zero(cbase, nbricks + 1, s) != hipSuccess) return SR_E_DEVICE;
        k_brick_mass<<<1, 256, 0, s>>>(nullptr, nullptr, 0, mstat);
        if (hipGetLastError() != hipSuccess) return SR_E_DEVICE;
    }
    const int nbz = P->ng / kBrick;
    const int tz = std::min(256, (nbz + 63) / 64 * 64);
    const int gx = (nbz + tz - 1) / tz;
    k_brick_combine<<<(unsigned)((int64_t)gx * P->ng * P->ng), tz, 0, s>>>(cbase, P->ng, gx, ctile, pad, grid);
    return hipGetLastError() == hipSuccess ? SR_OK : SR_E_DEVICE;
}

sr_status deposit(sr_pk_plan *P, const float *pos, const float *mass, int64_t n, char *w, hipStream_t s)
{
    if (P->brick) return deposit_bricks(P, pos, mass, n, w, s);
    float *grid = reinterpret_cast<float *>(w + P->grid_off);
    const int pad = 2 * (P->ng / 2 + 1);
    const float inv_h = (float)(P->ng / P->box);
    auto I = [&](size_t off) { return reinterpret_cast<int *>(w + off); };
    {
        const int64_t cells = (int64_t)P->ng * P->ng * P->ng;
        float4 *pf = reinterpret_cast<float4 *>(w + P->pf_off);
        float4 *spf = reinterpret_cast<float4 *>(w + P->spf_off);
        double *seg = reinterpret_cast<double *>(w + P->seg_off);
        if (n > 0) {
            k_cic_key<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(pos, mass, (int)n, P->ng, inv_h,
                                                                 I(P->key_off[1]), pf);
            if (hipGetLastError() != hipSuccess) return SR_E_DEVICE;
            // stable radix sort of the cell keys; pass p writes buffer p & 1
            const int64_t tiles = std::max<int64_t>(1, (n + kRadixTile - 1) / kRadixTile);
            const RadixBufs rb{{I(P->key_off[0]), I(P->key_off[1])}, {I(P->val_off[0]), I(P->val_off[1])},
                               I(P->tab_off), I(P->tabx_off), I(P->scan_off)};
            if (radix_sort_pairs(I(P->key_off[1]), nullptr, n, P->passes, P->digit_bits, tiles, rb, s) !=
                hipSuccess)
                return SR_E_DEVICE;
            const int out = (P->passes - 1) & 1;
            k_cic_pack<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(I(P->val_off[out]), (int)n, pf, spf);
            if (hipGetLastError() != hipSuccess) return SR_E_DEVICE;
            if (dev_bounds(I(P->key_off[out]), n, cells, 0, I(P->cstart_off), s) != hipSuccess)
                return SR_E_DEVICE;
            k_cic_runs<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(I(P->key_off[out]), spf, (int)n, seg);
            if (hipGetLastError() != hipSuccess) return SR_E_DEVICE;
        } else if (dev_zero(I(P->cstart_off), cells + 1, s) != hipSuccess) {
            return SR_E_DEVICE;
        }
        k_cic_points<<<(unsigned)((cells + 255) / 256), 256, 0, s>>>(I(P->cstart_off), seg, P->ng, pad, grid);
        if (hipGetLastError() != hipSuccess) return SR_E_DEVICE;
    }
    double *part = reinterpret_cast<double *>(w + P->mass_off);
    k_mass_partial<<<kSumBlocks, 256, 0, s>>>(mass, (int)n, part);
    k_mass_final<<<1, 256, 0, s>>>(part, kSumBlocks, part + kSumBlocks);
    return hipGetLastError() == hipSuccess ? SR_OK : SR_E_DEVICE;
}

}  // namespace

extern "C" {

sr_status sr_pk_plan_create(int32_t ng, double box, int32_t n_bins, double dn, int64_t n_max,
                            sr_pk_plan **plan, size_t *ws_bytes)
{
    if (!plan || !ws_bytes) return SR_E_ARG;
    *plan = nullptr;
    if (ng < 2 || ng > kMaxGrid || (ng & 1) || !(box > 0.0) || !std::isfinite(box) || n_bins < 1 ||
        n_bins > kMaxBins || !(dn > 0.0) || !std::isfinite(dn) || n_max < 0 ||
        n_max > (int64_t(1) << 31) - 1)
        return SR_E_ARG;
    auto *P = new sr_pk_plan;
    P->ng = ng;
    P->box = box;
    P->n_bins = n_bins;
    P->dn = dn;
    P->n_max = n_max;
    const int nzh = ng / 2 + 1;
    P->grid_bytes = (size_t)ng * ng * 2 * nzh * sizeof(float);
    size_t o = 0;
    P->grid_off = o;
    o = align256(o + P->grid_bytes);
    P->sinc_off = o;
    o = align256(o + sizeof(double) * ng);
    P->mass_off = o;
    o = align256(o + sizeof(double) * (kSumBlocks + 2));
    P->part_off = o;
    o = align256(o + sizeof(double) * 3 * n_bins * kBinBlocks);
    P->work_off = o;
    // rocFFT's work buffer for this size; queried without a device by a
    // conservative bound (one complex grid), checked again at the first run
    P->work_bytes = (size_t)ng * ng * nzh * 2 * sizeof(float);
    o = align256(o + P->work_bytes);
    P->brick = ng % kBrick == 0;
    if (P->brick) {
        const int64_t nb = ng / kBrick;
        P->nbricks = nb * nb * nb;  // brick keys fit 21 bits
        int bits = 1;
        while ((int64_t(1) << bits) < P->nbricks) ++bits;
        P->key_bits = bits;
        P->passes = (bits + 7) / 8;
        P->digit_bits = (bits + P->passes - 1) / P->passes;
        const int64_t m = std::max<int64_t>(1, n_max);
        P->tiles = std::max<int64_t>(1, (m + kRadixTile - 1) / kRadixTile);
        const int64_t table = (int64_t(1) << P->digit_bits) * P->tiles;
        P->max_chunks = m / kChunk + std::min<int64_t>(P->nbricks, m);
        for (int k = 0; k < 2; ++k) {
            P->key_off[k] = o;
            o = align256(o + sizeof(int) * m);
        }
        P->pf_off = o;  // payloads of sort buffer 0; buffer 1 at spf_off
        o = align256(o + sizeof(float4) * m);
        P->spf_off = o;
        o = align256(o + sizeof(float4) * m);
        P->cstart_off = o;  // first sorted slot of each brick
        o = align256(o + sizeof(int) * (P->nbricks + 1));
        P->chunks_off = o;
        o = align256(o + sizeof(int) * P->nbricks);
        P->cbase_off = o;
        o = align256(o + sizeof(int) * (P->nbricks + 1));
        P->owner_off = o;  // chunk records (brick, first, end)
        o = align256(o + sizeof(int4) * P->max_chunks);
        P->ctile_off = o;
        o = align256(o + sizeof(float) * kTilePts * P->max_chunks);
        P->msum_off = o;
        o = align256(o + sizeof(double) * P->tiles);
        P->mmax_off = o;
        o = align256(o + sizeof(float) * P->tiles);
        P->tab_off = o;
        o = align256(o + sizeof(int) * table);
        P->tabx_off = o;
        o = align256(o + sizeof(int) * (table + 1));
        P->scan_off = o;
        o = align256(o + sizeof(int) * scan_scratch_elems(std::max<int64_t>(table, P->nbricks)));
    } else {
        const int64_t cells = (int64_t)ng * ng * ng;  // cell keys fit 30 bits
        int bits = 1;
        while ((int64_t(1) << bits) < cells) ++bits;
        P->key_bits = bits;
        P->passes = (bits + 7) / 8;
        P->digit_bits = (bits + P->passes - 1) / P->passes;
        const int64_t m = std::max<int64_t>(1, n_max);
        P->tiles = std::max<int64_t>(1, (m + kRadixTile - 1) / kRadixTile);
        const int64_t table = (int64_t(1) << P->digit_bits) * P->tiles;
        for (int k = 0; k < 2; ++k) {
            P->key_off[k] = o;
            o = align256(o + sizeof(int) * m);
            P->val_off[k] = o;
            o = align256(o + sizeof(int) * m);
        }
        P->pf_off = o;
        o = align256(o + sizeof(float4) * m);
        P->spf_off = o;
        o = align256(o + sizeof(float4) * m);
        P->seg_off = o;
        o = align256(o + sizeof(double) * 8 * m);
        P->cstart_off = o;
        o = align256(o + sizeof(int) * (cells + 1));
        P->tab_off = o;
        o = align256(o + sizeof(int) * table);
        P->tabx_off = o;
        o = align256(o + sizeof(int) * (table + 1));
        P->scan_off = o;
        o = align256(o + sizeof(int) * scan_scratch_elems(table));
    }
    P->ws_bytes = o;
    *plan = P;
    *ws_bytes = P->ws_bytes;
    return SR_OK;
}

sr_status sr_pk_plan_destroy(sr_pk_plan *P)
{
    if (!P) return SR_E_PLAN;
    if (P->fft) (void)rocfft_plan_destroy(P->fft);
    delete P;
    return SR_OK;
}

sr_status sr_pk_deposit(sr_pk_plan *P, const float *pos, const float *mass, int64_t n, void *ws,
                        size_t ws_bytes, void *stream)
{
    if (!P) return SR_E_PLAN;
    if (n < 0 || n > P->n_max || (n > 0 && (!pos || !mass))) return SR_E_ARG;
    const sr_status st = check_pk_ws(P, ws, ws_bytes);
    if (st != SR_OK) return st;
    return deposit(P, pos, mass, n, static_cast<char *>(ws), static_cast<hipStream_t>(stream));
}

sr_status sr_pk_grid(const sr_pk_plan *P, const void *ws, const float **grid, int32_t *row_pitch,
                     const double **mass_total)
{
    if (!P) return SR_E_PLAN;
    if (!ws || !grid || !row_pitch) return SR_E_ARG;
    const char *w = static_cast<const char *>(ws);
    *grid = reinterpret_cast<const float *>(w + P->grid_off);
    *row_pitch = 2 * (P->ng / 2 + 1);
    if (mass_total) *mass_total = reinterpret_cast<const double *>(w + P->mass_off) + kSumBlocks;
    return SR_OK;
}

sr_status sr_power_spectrum(sr_pk_plan *P, const float *pos, const float *mass, int64_t n, void *ws,
                            size_t ws_bytes, double *pk, double *k, int64_t *modes, void *stream)
{
    if (!P) return SR_E_PLAN;
    if (n < 1 || n > P->n_max || !pos || !mass || !pk) return SR_E_ARG;
    sr_status st = check_pk_ws(P, ws, ws_bytes);
    if (st != SR_OK) return st;
    if ((st = ensure_fft(P)) != SR_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    if ((st = deposit(P, pos, mass, n, w, s)) != SR_OK) return st;
    k_pk_sinc<<<(unsigned)((P->ng + 255) / 256), 256, 0, s>>>(P->ng, reinterpret_cast<double *>(w + P->sinc_off));
    if (hipGetLastError() != hipSuccess) return SR_E_DEVICE;
    rocfft_execution_info info = nullptr;
    if (rocfft_execution_info_create(&info) != rocfft_status_success) return SR_E_DEVICE;
    bool ok = rocfft_execution_info_set_stream(info, s) == rocfft_status_success &&
              rocfft_execution_info_set_work_buffer(info, w + P->work_off, P->work_bytes) ==
                  rocfft_status_success;
    void *buf[1] = {w + P->grid_off};
    ok = ok && rocfft_execute(P->fft, buf, nullptr, info) == rocfft_status_success;
    (void)rocfft_execution_info_destroy(info);
    if (!ok) return SR_E_DEVICE;
    double *part = reinterpret_cast<double *>(w + P->part_off);
    const int nw = bin_waves(P->n_bins);
    k_pk_bins<<<kBinBlocks, nw * kWave, sizeof(double) * 3 * nw * P->n_bins, s>>>(
        reinterpret_cast<const float2 *>(w + P->grid_off), P->ng, P->n_bins, 1.0 / P->dn,
        reinterpret_cast<const double *>(w + P->sinc_off), part);
    k_pk_final<<<(unsigned)P->n_bins, 256, 0, s>>>(
        part, kBinBlocks, P->n_bins, reinterpret_cast<const double *>(w + P->mass_off) + kSumBlocks, P->box,
        pk, k, modes);
    return hipGetLastError() == hipSuccess ? SR_OK : SR_E_DEVICE;
}

}  // extern "C"
