/*
 * sr_oracle.c -- plain CPU reference for the short-range particle-particle
 * force.  TEST INFRASTRUCTURE ONLY: the test suite, the package's smoke check
 * and the benchmark's CPU-baseline leg call it; the library never does.  It
 * shares no code, header or constant with the device path.
 *
 * What it computes (paper Sec. 2: the force is split into a long-range
 * particle-mesh part and a short-range part that accelerators sum directly
 * over particle pairs; Sec. 2 and 2.1: each domain holds its own "active"
 * particles plus overloaded "passive" copies that act only as sources):
 *
 *   a_i = sum_{j != i, 0 < s_ij < r_s^2}  m_j d_ij f_SR(s_ij),  i active,
 *   d_ij = x_j - x_i  (minimum image in a periodic box),  s = |d|^2,
 *   f_SR(s) = (s + eps^2)^(-3/2) - sum_{k=0..5} c_k s^k .
 *
 * The kernel form (softened Newton minus a degree-5 polynomial filter in s)
 * is not written out in the paper, which defers it to the HACC method papers;
 * the coefficients are therefore an argument.  Everything here is float64,
 * evaluated on the caller's values (the tests pass the exact float32 inputs
 * widened to double).  Active particles are indices [0, n_active).
 *
 * Functions:
 *   oracle_bin_reference  the float32 cell-binning rule the library's binning
 *                         must reproduce bit for bit (the rule is a reading:
 *                         the paper names chaining-mesh binning only through
 *                         the HACC papers), with the particles of each cell
 *                         ordered by the leaves of an octree of a given depth
 *                         inside the cell (tree codes are the paper's
 *                         short-range solver on CPU systems, Sec. 2);
 *   oracle_force          the sum above through a float64 cell list;
 *   oracle_force_brute    the same sum over all pairs and all 27 periodic
 *                         images, no cells;
 *   oracle_vjp            the adjoint of a with respect to the positions;
 *   oracle_vjp_brute      the adjoint over all pairs and images.
 *
 * Return values: 0 on success, negative on invalid arguments.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_NONFINITE 1u
#define OR_OUT_OF_DOMAIN 2u

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads the calling thread's later calls use (the caller runs many small
 * oracle calls from its own pool of threads). */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------ */
/* float32 binning rule                                                 */
/* ------------------------------------------------------------------ */

/* Cells per dimension: floor(len / r_s) in float32; at least 1 for an open
 * domain.  A periodic box needs at least 3 cells per dimension so that the
 * 27 neighbour cells are distinct (and len > 2 r_s, the minimum-image
 * condition). */
int oracle_grid(const float len[3], float r_s, int periodic, int32_t nc[3])
{
    if (!(r_s > 0.0f)) return -1;
    for (int d = 0; d < 3; ++d) {
        if (!(len[d] > 0.0f)) return -1;
        float q = floorf(len[d] / r_s);
        if (!(q < 1.0e9f)) return -1;
        int v = (int)q;
        if (periodic) {
            if (v < 3) return -2;
        } else if (v < 1) {
            v = 1;
        }
        nc[d] = v;
    }
    return 0;
}

/* One coordinate, all float32, round-to-nearest, no fused operations (the
 * file is compiled with -ffp-contract=off):
 *   periodic: k = floor(x * (1/len)), w = x - k*len, u = w   (lo must be 0)
 *   open:     w = x, u = x - lo
 *   i = clamp(floor(u * (nc/len)), 0, nc-1)  (NaN -> 0)
 *   centre = lo + (i + 0.5) * (len/nc),  offset = w - centre            */
static int bin_coord(float x, float lo, float len, int nc, int periodic, float *off,
                     uint32_t *flags)
{
    const float inv_len = 1.0f / len;
    const float h = len / (float)nc;
    const float inv_h = (float)nc / len;
    float w, u;
    if (!isfinite(x)) *flags |= OR_NONFINITE;
    if (periodic) {
        float k = floorf(x * inv_len);
        float p = k * len;
        w = x - p;
        u = w;
    } else {
        w = x;
        u = x - lo;
    }
    float fi = floorf(u * inv_h);
    int i;
    if (!(fi >= 0.0f)) {
        i = 0;
        if (!periodic && isfinite(x)) *flags |= OR_OUT_OF_DOMAIN;
    } else if (fi > (float)(nc - 1)) {
        i = nc - 1;
        if (!periodic && isfinite(x)) *flags |= OR_OUT_OF_DOMAIN;
    } else {
        i = (int)fi;
    }
    float t = (float)i + 0.5f;
    float c = t * h;
    c = lo + c;
    *off = w - c;
    return i;
}

/* Leaf of an octree of `depth` levels inside the cell that holds a particle
 * at offset o from the cell centre (cell sides h).  Per axis, level 1 takes
 * the sign of the offset; each deeper level first re-centres the offset on
 * the half it fell in (subtract or add a quarter of the current side, in
 * float32) and takes the sign again.  The code lists the levels from the
 * top, one octal digit 4 b_x + 2 b_y + b_z each (Z order). */
static int64_t leaf_code(const float o[3], const float h[3], int depth)
{
    int b[3][8];
    for (int d = 0; d < 3; ++d) {
        float off = o[d];
        float quarter = h[d] * 0.25f;
        for (int l = 0; l < depth; ++l) {
            b[d][l] = off >= 0.0f;
            off = b[d][l] ? off - quarter : off + quarter;
            quarter = quarter * 0.5f;
        }
    }
    int64_t code = 0;
    for (int l = 0; l < depth; ++l) code = 8 * code + 4 * b[0][l] + 2 * b[1][l] + b[2][l];
    return code;
}

typedef struct {
    int64_t key; /* (cell, passive, leaf code) */
    int64_t p;   /* input index */
} bin_entry;

static int cmp_entry(const void *a, const void *b)
{
    const bin_entry *x = (const bin_entry *)a, *y = (const bin_entry *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->p > y->p) - (x->p < y->p);
}

/* cell_of[n] (input order), cell_start[ncell+1], perm[n] (binned slot ->
 * input index) and off[3n] (binned order).  Cells are numbered
 * (ix*ncy + iy)*ncz + iz.  Slots are ordered by (cell, passive, leaf code,
 * input index): passive = index >= n_active; the leaf code is that of an
 * octree of leaf_depth levels (1..4); at depth 1 it is the octant
 * 4 [off_x >= 0] + 2 [off_y >= 0] + [off_z >= 0]. */
int oracle_bin_reference(const float *pos, int64_t n, int64_t n_active, const float lo[3],
                         const float len[3], int periodic, float r_s, int leaf_depth,
                         int32_t *cell_of, int32_t *cell_start, int32_t *perm, float *off,
                         uint32_t *flags_out)
{
    int32_t nc[3];
    int rc = oracle_grid(len, r_s, periodic, nc);
    if (rc) return rc;
    if (periodic && (lo[0] != 0.0f || lo[1] != 0.0f || lo[2] != 0.0f)) return -3;
    if (n_active < 0 || n_active > n) return -1;
    if (leaf_depth < 1 || leaf_depth > 4) return -1;
    const int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    float h[3];
    for (int d = 0; d < 3; ++d) h[d] = len[d] / (float)nc[d];
    uint32_t flags = 0;
    float *o = (float *)malloc(sizeof(float) * 3 * (size_t)(n > 0 ? n : 1));
    bin_entry *e = (bin_entry *)malloc(sizeof(bin_entry) * (size_t)(n > 0 ? n : 1));
    const int64_t leaves = (int64_t)1 << (3 * leaf_depth);
    for (int64_t p = 0; p < n; ++p) {
        int ic[3];
        for (int d = 0; d < 3; ++d)
            ic[d] = bin_coord(pos[3 * p + d], lo[d], len[d], nc[d], periodic, &o[3 * p + d], &flags);
        cell_of[p] = (int32_t)(((int64_t)ic[0] * nc[1] + ic[1]) * nc[2] + ic[2]);
        e[p].key = (2 * (int64_t)cell_of[p] + (p >= n_active ? 1 : 0)) * leaves + leaf_code(&o[3 * p], h, leaf_depth);
        e[p].p = p;
    }
    qsort(e, (size_t)n, sizeof(bin_entry), cmp_entry);
    /* the first slot of each cell: count per cell, then an exclusive prefix sum */
    for (int64_t c = 0; c <= ncell; ++c) cell_start[c] = 0;
    for (int64_t p = 0; p < n; ++p) cell_start[cell_of[p] + 1]++;
    for (int64_t c = 0; c < ncell; ++c) cell_start[c + 1] += cell_start[c];
    for (int64_t s = 0; s < n; ++s) {
        const int64_t p = e[s].p;
        perm[s] = (int32_t)p;
        off[3 * s + 0] = o[3 * p + 0];
        off[3 * s + 1] = o[3 * p + 1];
        off[3 * s + 2] = o[3 * p + 2];
    }
    free(e);
    free(o);
    if (flags_out) *flags_out = flags;
    return 0;
}

/* ------------------------------------------------------------------ */
/* float64 kernel                                                       */
/* ------------------------------------------------------------------ */

typedef struct {
    double lo[3], len[3];
    int periodic;
    double rs2, eps2;
    double c[6];
} prob_t;

/* f_SR(s) */
static double f_sr(const prob_t *P, double s)
{
    double t = s + P->eps2;
    double newton = 1.0 / (t * sqrt(t));
    double poly = P->c[5];
    for (int k = 4; k >= 0; --k) poly = poly * s + P->c[k];
    return newton - poly;
}

/* d f_SR / ds */
static double df_sr(const prob_t *P, double s)
{
    double t = s + P->eps2;
    double newton = -1.5 / (t * t * sqrt(t));
    double dpoly = 5.0 * P->c[5];
    for (int k = 4; k >= 1; --k) dpoly = dpoly * s + k * P->c[k];
    return newton - dpoly;
}

static void min_image(const prob_t *P, double d[3])
{
    if (!P->periodic) return;
    for (int a = 0; a < 3; ++a) d[a] -= P->len[a] * nearbyint(d[a] / P->len[a]);
}

static int make_prob(prob_t *P, const double lo[3], const double len[3], int periodic,
                     double r_s, double eps, const double poly[6])
{
    if (!(r_s > 0.0) || !(eps >= 0.0)) return -1;
    for (int d = 0; d < 3; ++d) {
        if (!(len[d] > 0.0)) return -1;
        P->lo[d] = lo[d];
        P->len[d] = len[d];
        if (periodic && !(len[d] >= 3.0 * r_s)) return -2;
    }
    P->periodic = periodic;
    P->rs2 = r_s * r_s;
    P->eps2 = eps * eps;
    for (int k = 0; k < 6; ++k) P->c[k] = poly[k];
    return 0;
}

/* float64 cell list with cells of side >= r_s */
typedef struct {
    int nc[3];
    double h[3];
    int64_t ncell;
    int64_t *start; /* [ncell+1] */
    int64_t *idx;   /* particles by cell */
    int32_t *cell;  /* cell of each particle */
} clist_t;

static int cell_coord(const prob_t *P, const clist_t *C, int a, double x)
{
    double u;
    if (P->periodic) {
        u = x - P->len[a] * floor(x / P->len[a]);
    } else {
        u = x - P->lo[a];
    }
    double q = floor(u / C->h[a]);
    if (!(q >= 0.0)) return 0;
    if (q > C->nc[a] - 1) return C->nc[a] - 1;
    return (int)q;
}

static void clist_build(clist_t *C, const prob_t *P, const double *pos, int64_t n)
{
    double r_s = sqrt(P->rs2);
    for (int a = 0; a < 3; ++a) {
        int v = (int)floor(P->len[a] / r_s);
        if (v < 1) v = 1;
        while (v > 1 && P->len[a] / v < r_s) --v;
        C->nc[a] = v;
        C->h[a] = P->len[a] / v;
    }
    C->ncell = (int64_t)C->nc[0] * C->nc[1] * C->nc[2];
    C->start = (int64_t *)calloc((size_t)C->ncell + 1, sizeof(int64_t));
    C->idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    C->cell = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t p = 0; p < n; ++p) {
        int ix = cell_coord(P, C, 0, pos[3 * p]);
        int iy = cell_coord(P, C, 1, pos[3 * p + 1]);
        int iz = cell_coord(P, C, 2, pos[3 * p + 2]);
        C->cell[p] = (int32_t)(((int64_t)ix * C->nc[1] + iy) * C->nc[2] + iz);
        C->start[C->cell[p] + 1]++;
    }
    for (int64_t c = 0; c < C->ncell; ++c) C->start[c + 1] += C->start[c];
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)C->ncell);
    memcpy(cur, C->start, sizeof(int64_t) * (size_t)C->ncell);
    for (int64_t p = 0; p < n; ++p) C->idx[cur[C->cell[p]]++] = p;
    free(cur);
}

static void clist_free(clist_t *C)
{
    free(C->start);
    free(C->idx);
    free(C->cell);
}

/* Collect the distinct neighbour cells (27 in a periodic box with nc >= 3,
 * fewer at the faces of an open domain or when nc < 3 there). */
static int neighbour_cells(const prob_t *P, const clist_t *C, int32_t cell, int64_t out[27])
{
    int iz = cell % C->nc[2];
    int iy = (cell / C->nc[2]) % C->nc[1];
    int ix = cell / (C->nc[2] * C->nc[1]);
    int m = 0;
    for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
                int j[3] = {ix + dx, iy + dy, iz + dz};
                int ok = 1;
                for (int a = 0; a < 3; ++a) {
                    if (j[a] < 0 || j[a] >= C->nc[a]) {
                        if (P->periodic)
                            j[a] = (j[a] + C->nc[a]) % C->nc[a];
                        else
                            ok = 0;
                    }
                }
                if (!ok) continue;
                int64_t c = ((int64_t)j[0] * C->nc[1] + j[1]) * C->nc[2] + j[2];
                int dup = 0;
                for (int q = 0; q < m; ++q) dup |= (out[q] == c);
                if (!dup) out[m++] = c;
            }
    return m;
}

static int64_t *default_targets(int64_t count)
{
    int64_t *t = (int64_t *)malloc(sizeof(int64_t) * (size_t)(count > 0 ? count : 1));
    for (int64_t i = 0; i < count; ++i) t[i] = i;
    return t;
}

/* acc[3*q] for each target q (targets NULL: all active, in order).
 * pairs_out (nullable): number of ordered pairs (target, source) with
 * 0 < s < r_s^2. */
int oracle_force(const double *pos, const double *mass, int64_t n, int64_t n_active,
                 const double lo[3], const double len[3], int periodic, double r_s, double eps,
                 const double poly[6], const int64_t *targets, int64_t n_targets, double *acc,
                 int64_t *pairs_out)
{
    prob_t P;
    int rc = make_prob(&P, lo, len, periodic, r_s, eps, poly);
    if (rc) return rc;
    if (n_active < 0 || n_active > n) return -1;
    int64_t *own = NULL;
    if (!targets) {
        own = default_targets(n_active);
        targets = own;
        n_targets = n_active;
    }
    for (int64_t q = 0; q < n_targets; ++q)
        if (targets[q] < 0 || targets[q] >= n_active) {
            free(own);
            return -4;
        }
    clist_t C;
    clist_build(&C, &P, pos, n);
    int64_t pairs = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : pairs)
    for (int64_t q = 0; q < n_targets; ++q) {
        const int64_t i = targets[q];
        int64_t nb[27];
        int m = neighbour_cells(&P, &C, C.cell[i], nb);
        double ax = 0, ay = 0, az = 0;
        for (int c = 0; c < m; ++c) {
            for (int64_t k = C.start[nb[c]]; k < C.start[nb[c] + 1]; ++k) {
                int64_t j = C.idx[k];
                if (j == i) continue;
                double d[3] = {pos[3 * j] - pos[3 * i], pos[3 * j + 1] - pos[3 * i + 1],
                               pos[3 * j + 2] - pos[3 * i + 2]};
                min_image(&P, d);
                double s = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                if (!(s > 0.0 && s < P.rs2)) continue;
                double w = mass[j] * f_sr(&P, s);
                ax += w * d[0];
                ay += w * d[1];
                az += w * d[2];
                pairs++;
            }
        }
        acc[3 * q] = ax;
        acc[3 * q + 1] = ay;
        acc[3 * q + 2] = az;
    }
    clist_free(&C);
    free(own);
    if (pairs_out) *pairs_out = pairs;
    return 0;
}

/* Same sum, no cells: every source and every one of the 27 periodic images
 * (positions first wrapped into the box), or the plain difference in an
 * open domain.  O(n_active * n). */
int oracle_force_brute(const double *pos, const double *mass, int64_t n, int64_t n_active,
                       const double lo[3], const double len[3], int periodic, double r_s,
                       double eps, const double poly[6], double *acc)
{
    prob_t P;
    int rc = make_prob(&P, lo, len, periodic, r_s, eps, poly);
    if (rc) return rc;
    if (periodic)
        for (int a = 0; a < 3; ++a)
            if (!(len[a] > 2.0 * r_s)) return -2;
    double *x = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    for (int64_t p = 0; p < 3 * n; ++p) {
        int a = (int)(p % 3);
        x[p] = periodic ? pos[p] - len[a] * floor(pos[p] / len[a]) : pos[p];
    }
    const int R = periodic ? 1 : 0;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n_active; ++i) {
        double ax = 0, ay = 0, az = 0;
        for (int64_t j = 0; j < n; ++j)
            for (int sx = -R; sx <= R; ++sx)
                for (int sy = -R; sy <= R; ++sy)
                    for (int sz = -R; sz <= R; ++sz) {
                        if (j == i && sx == 0 && sy == 0 && sz == 0) continue;
                        double d0 = x[3 * j] + sx * len[0] - x[3 * i];
                        double d1 = x[3 * j + 1] + sy * len[1] - x[3 * i + 1];
                        double d2 = x[3 * j + 2] + sz * len[2] - x[3 * i + 2];
                        double s = d0 * d0 + d1 * d1 + d2 * d2;
                        if (!(s > 0.0 && s < P.rs2)) continue;
                        double w = mass[j] * f_sr(&P, s);
                        ax += w * d0;
                        ay += w * d1;
                        az += w * d2;
                    }
        acc[3 * i] = ax;
        acc[3 * i + 1] = ay;
        acc[3 * i + 2] = az;
    }
    free(x);
    return 0;
}

/* Adjoint.  For L = sum_{i active} g_i . a_i (g_j = 0 for passive j), the
 * gradient with respect to x_k, any k, is
 *   sum_{j != k, s < r_s^2} [ f u + 2 f' (u . d) d ],
 *   d = x_j - x_k,  u = m_k g_j - m_j g_k,  f = f_SR(s), f' = df_SR/ds.
 * (Differentiating a_k gives -m_j [f g_k + 2 f' (g_k.d) d]; differentiating
 * each a_j in which x_k is a source gives m_k [f g_j + 2 f' (g_j.d) d].)
 * The jump of the cutoff is not differentiated.  A pair at s = 0 (a distinct
 * particle at the same position) contributes nothing to the forces, but with
 * softening its force term m d f(|d|^2) is smooth through d = 0 with
 * Jacobian m f(0) I, so it adds f(0) u here; without softening f is
 * singular there and the pair is left out, as in the forward sum.
 * grad[3*q] for target q (targets NULL: all n particles). */

/* Does the adjoint take a pair at squared distance s?  (j != k is checked
 * by the caller.) */
static int vjp_takes(const prob_t *P, double s)
{
    if (!(s < P->rs2)) return 0;
    return s > 0.0 || P->eps2 > 0.0;
}
int oracle_vjp(const double *pos, const double *mass, int64_t n, int64_t n_active,
               const double lo[3], const double len[3], int periodic, double r_s, double eps,
               const double poly[6], const double *g, const int64_t *targets, int64_t n_targets,
               double *grad)
{
    prob_t P;
    int rc = make_prob(&P, lo, len, periodic, r_s, eps, poly);
    if (rc) return rc;
    if (n_active < 0 || n_active > n) return -1;
    int64_t *own = NULL;
    if (!targets) {
        own = default_targets(n);
        targets = own;
        n_targets = n;
    }
    for (int64_t q = 0; q < n_targets; ++q)
        if (targets[q] < 0 || targets[q] >= n) {
            free(own);
            return -4;
        }
    clist_t C;
    clist_build(&C, &P, pos, n);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < n_targets; ++q) {
        const int64_t k = targets[q];
        const double gk[3] = {k < n_active ? g[3 * k] : 0.0, k < n_active ? g[3 * k + 1] : 0.0,
                              k < n_active ? g[3 * k + 2] : 0.0};
        int64_t nb[27];
        int m = neighbour_cells(&P, &C, C.cell[k], nb);
        double r0 = 0, r1 = 0, r2 = 0;
        for (int c = 0; c < m; ++c) {
            for (int64_t e = C.start[nb[c]]; e < C.start[nb[c] + 1]; ++e) {
                int64_t j = C.idx[e];
                if (j == k) continue;
                double d[3] = {pos[3 * j] - pos[3 * k], pos[3 * j + 1] - pos[3 * k + 1],
                               pos[3 * j + 2] - pos[3 * k + 2]};
                min_image(&P, d);
                double s = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                if (!vjp_takes(&P, s)) continue;
                double gj[3] = {0, 0, 0};
                if (j < n_active) {
                    gj[0] = g[3 * j];
                    gj[1] = g[3 * j + 1];
                    gj[2] = g[3 * j + 2];
                }
                double u[3];
                for (int a = 0; a < 3; ++a) u[a] = mass[k] * gj[a] - mass[j] * gk[a];
                double f = f_sr(&P, s), fp = df_sr(&P, s);
                double ud = u[0] * d[0] + u[1] * d[1] + u[2] * d[2];
                r0 += f * u[0] + 2.0 * fp * ud * d[0];
                r1 += f * u[1] + 2.0 * fp * ud * d[1];
                r2 += f * u[2] + 2.0 * fp * ud * d[2];
            }
        }
        grad[3 * q] = r0;
        grad[3 * q + 1] = r1;
        grad[3 * q + 2] = r2;
    }
    clist_free(&C);
    free(own);
    return 0;
}

/* Adjoint over all pairs and periodic images, no cells: grad[3n]. */
int oracle_vjp_brute(const double *pos, const double *mass, int64_t n, int64_t n_active,
                     const double lo[3], const double len[3], int periodic, double r_s,
                     double eps, const double poly[6], const double *g, double *grad)
{
    prob_t P;
    int rc = make_prob(&P, lo, len, periodic, r_s, eps, poly);
    if (rc) return rc;
    double *x = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    for (int64_t p = 0; p < 3 * n; ++p) {
        int a = (int)(p % 3);
        x[p] = periodic ? pos[p] - len[a] * floor(pos[p] / len[a]) : pos[p];
    }
    const int R = periodic ? 1 : 0;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n; ++k) {
        double gk[3] = {0, 0, 0};
        if (k < n_active)
            for (int a = 0; a < 3; ++a) gk[a] = g[3 * k + a];
        double r[3] = {0, 0, 0};
        for (int64_t j = 0; j < n; ++j) {
            double gj[3] = {0, 0, 0};
            if (j < n_active)
                for (int a = 0; a < 3; ++a) gj[a] = g[3 * j + a];
            for (int sx = -R; sx <= R; ++sx)
                for (int sy = -R; sy <= R; ++sy)
                    for (int sz = -R; sz <= R; ++sz) {
                        if (j == k && sx == 0 && sy == 0 && sz == 0) continue;
                        double d[3] = {x[3 * j] + sx * len[0] - x[3 * k],
                                       x[3 * j + 1] + sy * len[1] - x[3 * k + 1],
                                       x[3 * j + 2] + sz * len[2] - x[3 * k + 2]};
                        double s = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                        if (!vjp_takes(&P, s)) continue;
                        double f = f_sr(&P, s), fp = df_sr(&P, s);
                        double u[3], ud = 0;
                        for (int a = 0; a < 3; ++a) {
                            u[a] = mass[k] * gj[a] - mass[j] * gk[a];
                            ud += u[a] * d[a];
                        }
                        for (int a = 0; a < 3; ++a) r[a] += f * u[a] + 2.0 * fp * ud * d[a];
                    }
        }
        for (int a = 0; a < 3; ++a) grad[3 * k + a] = r[a];
    }
    free(x);
    return 0;
}
