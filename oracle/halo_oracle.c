/*
 * halo_oracle.c -- plain CPU reference for the most-bound-particle halo
 * centre finder.  TEST INFRASTRUCTURE ONLY: the test suite, the package's
 * smoke check and the benchmark's CPU-baseline leg call it; the library never
 * does.  It shares no code, header or constant with the device path.
 *
 * What it computes (paper Sec. 2.2: the centre of a halo is the particle at
 * its potential minimum, the "most bound" particle, found after the
 * friends-of-friends halo finder has assigned particles to halos):
 *
 *   phi_i = - sum_{j in halo(i), j != i}  m_j / sqrt(|x_j - x_i|^2 + eps^2)
 *
 * over the particles of the same halo only (G = 1), and per halo the index of
 * the particle with the smallest phi (ties: the smallest index).  With
 * eps = 0, coincident pairs (|d| = 0) contribute nothing.  Halo h holds the
 * particles [offsets[h], offsets[h+1]); coordinates are taken as given (the
 * halo finder's unwrapped positions).  Everything is float64, one direct sum
 * per target, OpenMP over targets.
 *
 * Return values: 0 on success, negative on invalid arguments.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

static int check_offsets(const int64_t *offsets, int64_t n_halos, int64_t n)
{
    if (!offsets || n_halos < 0 || offsets[0] != 0 || offsets[n_halos] != n) return -1;
    for (int64_t h = 0; h < n_halos; ++h)
        if (offsets[h + 1] < offsets[h]) return -1;
    return 0;
}

/* Halo of particle i: the h with offsets[h] <= i < offsets[h+1]. */
static int64_t halo_of(const int64_t *offsets, int64_t n_halos, int64_t i)
{
    int64_t lo = 0, hi = n_halos - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (offsets[mid] <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

/* phi of the listed targets (all particles when targets is NULL, then
 * n_targets must equal n). */
int oracle_halo_potential(const double *pos, const double *mass, int64_t n, const int64_t *offsets,
                          int64_t n_halos, double eps, const int64_t *targets, int64_t n_targets,
                          double *phi)
{
    if (!pos || !mass || !phi || n < 0 || !(eps >= 0.0)) return -1;
    if (check_offsets(offsets, n_halos, n) != 0) return -1;
    if (!targets && n_targets != n) return -1;
    const double e2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < n_targets; ++t) {
        const int64_t i = targets ? targets[t] : t;
        if (i < 0 || i >= n) {
            phi[t] = NAN;
            continue;
        }
        const int64_t h = halo_of(offsets, n_halos, i);
        double sum = 0.0;
        for (int64_t j = offsets[h]; j < offsets[h + 1]; ++j) {
            if (j == i) continue;
            const double dx = pos[3 * j] - pos[3 * i];
            const double dy = pos[3 * j + 1] - pos[3 * i + 1];
            const double dz = pos[3 * j + 2] - pos[3 * i + 2];
            const double r2 = dx * dx + dy * dy + dz * dz + e2;
            if (r2 > 0.0) sum += mass[j] / sqrt(r2);
        }
        phi[t] = -sum;
    }
    return 0;
}
