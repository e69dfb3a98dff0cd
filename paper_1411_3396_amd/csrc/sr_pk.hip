// Power spectrum of the particles on the fly (paper Sec. 4.1): cloud-in-cell
// deposit onto an ng^3 periodic grid, a real-to-complex FFT, |delta(k)|^2
// divided by the CIC window and averaged in bins of |k|.
//
// Device passes: the deposit into the FFT's padded in-place layout, a
// float64 mass sum in a fixed order, the FFT (rocFFT, in place), and the
// binning.  The deposit is atomic-free: particles are sorted by the cell of
// their lower corner point (the binning's radix sort), a segmented scan sums
// each cell's corner contributions per wave, and every grid point adds the
// partials of its 8 cells in float64, in a fixed order.  Binning: every mode of
// the half spectrum adds w |rho_k|^2 / W(k)^2 (w = 2 for modes whose mirror
// is not stored) into per-workgroup float64 bins in LDS; a last pass adds
// the workgroups' bins in workgroup order.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include <rocfft/rocfft.h>

#include "sr_internal.h"

namespace sr {
namespace {

constexpr int kBinBlocks = 1024;  // one-wave workgroups of the binning pass
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
        u = u - floorf(u / fng) * fng;
        int k = (int)floorf(u);
        float fr = u - (float)k;
        if (k >= ng) {
            k = 0;
            fr = 0.f;
        }
        if (k < 0) k = 0;
        i0[d] = k;
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

// Modes of the half spectrum (iz in [0, ng/2]), one wave per workgroup, each
// taking whole rows (ix, iy) in a fixed order.  Along a row |n| grows with iz,
// so the bins of 64 consecutive modes form runs: a segmented scan sums each
// run in a fixed tree order and the run's last lane adds it to the
// workgroup's bins in LDS (within a chunk every run has its own bin, so no two
// lanes touch one bin at once, and chunks go in order).  The sums therefore
// do not depend on scheduling: the spectrum is bitwise reproducible.
// sinc2[i] = sinc^2(pi n_i / ng) for the mode index n_i of array index i.
__global__ __launch_bounds__(64) void k_pk_bins(const float2 *__restrict__ c, int ng, int n_bins,
                                                double inv_dn, const double *__restrict__ sinc2,
                                                double *__restrict__ part)
{
    extern __shared__ double bins[];  // [3][n_bins]: sum of w P', sum of w |n|, sum of w
    const int lane = threadIdx.x;
    for (int b = lane; b < 3 * n_bins; b += kWave) bins[b] = 0.0;
    __syncthreads();
    const int nzh = ng / 2 + 1;
    const int64_t rows = (int64_t)ng * ng;
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const int iy = (int)(r % ng), ix = (int)(r / ng);
        const int nx = ix <= ng / 2 ? ix : ix - ng;
        const int ny = iy <= ng / 2 ? iy : iy - ng;
        const double sxy = sinc2[ix] * sinc2[iy];
        for (int z0 = 0; z0 < nzh; z0 += kWave) {
            const int iz = z0 + lane;
            double p = 0.0, km = 0.0, wt = 0.0;
            int key = -1;  // outside every bin: k = 0, beyond the last bin, past the row
            if (iz < nzh) {
                const double mag = sqrt((double)nx * nx + (double)ny * ny + (double)iz * iz);
                const int b = (int)floor(mag * inv_dn);
                if (mag != 0.0 && b < n_bins) {
                    const float2 v = c[r * nzh + iz];
                    const double w = (iz == 0 || 2 * iz == ng) ? 1.0 : 2.0;
                    const double win = sxy * sinc2[iz];
                    p = w * (((double)v.x * v.x + (double)v.y * v.y) / (win * win));
                    km = w * mag;
                    wt = w;
                    key = b;
                } else if (mag != 0.0) {
                    key = n_bins;
                }
            }
            const int prev = __shfl_up(key, 1);
            const uint64_t heads = __ballot(lane == 0 || prev != key);
            const uint64_t upto = (lane == 63) ? heads : (heads & ((2ull << lane) - 1));
            const int first = 63 - __clzll(upto);  // first lane of this lane's run
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
                const double yp = __shfl_up(p, o), yk = __shfl_up(km, o), yw = __shfl_up(wt, o);
                if (lane - o >= first) {
                    p += yp;
                    km += yk;
                    wt += yw;
                }
            }
            const int next = __shfl_down(key, 1);
            if ((lane == 63 || next != key) && key >= 0 && key < n_bins) {
                bins[key] += p;
                bins[n_bins + key] += km;
                bins[2 * n_bins + key] += wt;
            }
        }
    }
    __syncthreads();
    for (int b = lane; b < 3 * n_bins; b += kWave) part[(int64_t)blockIdx.x * 3 * n_bins + b] = bins[b];
}

// P(bin) = box^3 / M^2 * sum(w P') / sum(w), k = 2 pi / box * sum(w |n|) / sum(w).
__global__ __launch_bounds__(256) void k_pk_final(const double *__restrict__ part, int blocks,
                                                  int n_bins, const double *__restrict__ mtot,
                                                  double box, double *__restrict__ pk,
                                                  double *__restrict__ kmean,
                                                  int64_t *__restrict__ modes)
{
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= n_bins) return;
    double sp = 0.0, sk = 0.0, sw = 0.0;
    for (int g = 0; g < blocks; ++g) {
        const double *q = part + (int64_t)g * 3 * n_bins;
        sp += q[b];
        sk += q[n_bins + b];
        sw += q[2 * n_bins + b];
    }
    const double M = mtot[0];
    const double two_pi = 6.283185307179586476925;
    pk[b] = sw > 0.0 ? sp / sw * box * box * box / (M * M) : 0.0;
    if (kmean) kmean[b] = sw > 0.0 ? sk / sw * two_pi / box : 0.0;
    if (modes) modes[b] = (int64_t)(sw + 0.5);
}

// sinc2[i] = sinc^2(pi n / ng) for the mode index n of array index i.
__global__ __launch_bounds__(256) void k_pk_sinc(int ng, double *__restrict__ sinc2)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= ng) return;
    const int nm = i <= ng / 2 ? i : i - ng;
    const double x = 3.14159265358979323846 * nm / ng;
    const double s = nm == 0 ? 1.0 : sin(x) / x;
    sinc2[i] = s * s;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

std::once_flag g_fft_setup;

}  // namespace
}  // namespace sr

using namespace sr;

struct sr_pk_plan {
    int ng = 0, n_bins = 0;
    double box = 0.0, dn = 1.0;
    int64_t n_max = 0;
    int passes = 1, digit_bits = 1;
    int64_t tiles = 1;
    size_t grid_off = 0, grid_bytes = 0, sinc_off = 0, mass_off = 0, part_off = 0, work_off = 0,
           key_off[2] = {0, 0}, val_off[2] = {0, 0}, pf_off = 0, spf_off = 0, seg_off = 0, cstart_off = 0,
           tab_off = 0, tabx_off = 0, scan_off = 0, ws_bytes = 0;
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

sr_status deposit(sr_pk_plan *P, const float *pos, const float *mass, int64_t n, char *w, hipStream_t s)
{
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
    o = align256(o + sizeof(double) * (kSumBlocks + 1));
    P->part_off = o;
    o = align256(o + sizeof(double) * 3 * n_bins * kBinBlocks);
    P->work_off = o;
    // rocFFT's work buffer for this size; queried without a device by a
    // conservative bound (one complex grid), checked again at the first run
    P->work_bytes = (size_t)ng * ng * nzh * 2 * sizeof(float);
    o = align256(o + P->work_bytes);
    {
        const int64_t cells = (int64_t)ng * ng * ng;  // cell keys fit 30 bits
        int bits = 1;
        while ((int64_t(1) << bits) < cells) ++bits;
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
    k_pk_bins<<<kBinBlocks, kWave, sizeof(double) * 3 * P->n_bins, s>>>(
        reinterpret_cast<const float2 *>(w + P->grid_off), P->ng, P->n_bins, 1.0 / P->dn,
        reinterpret_cast<const double *>(w + P->sinc_off), part);
    k_pk_final<<<(unsigned)((P->n_bins + 255) / 256), 256, 0, s>>>(
        part, kBinBlocks, P->n_bins, reinterpret_cast<const double *>(w + P->mass_off) + kSumBlocks, P->box,
        pk, k, modes);
    return hipGetLastError() == hipSuccess ? SR_OK : SR_E_DEVICE;
}

}  // extern "C"
