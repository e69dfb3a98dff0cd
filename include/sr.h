/*
 * sr.h -- C ABI of the short-range particle-particle force library (libsr).
 *
 * The library computes the short-range half of a split gravitational force
 * (paper Sec. 2: the long-range part is solved on a spectrally filtered
 * particle-mesh grid, the short-range part by direct particle-particle sums on
 * the accelerator).  For every active particle i
 *
 *     a_i = sum_{j != i, 0 < s_ij < r_s^2}  m_j d_ij f_SR(s_ij)
 *     d_ij = x_j - x_i (minimum image when periodic),  s = |d|^2
 *     f_SR(s) = (s + eps^2)^(-3/2) - sum_{k=0..5} poly[k] s^k
 *
 * in units with G = 1 and lengths in grid cells.  Active particles are the
 * first n_active rows; the remaining rows are passive copies (the overload
 * or ghost zone of Sec. 2 and the passive block particles of Sec. 2.1) that
 * act only as sources.  The filter polynomial and its coefficients are not
 * printed in the paper (it defers them to the HACC method papers), so they
 * are an argument.
 *
 * Conventions for every entry point:
 *  - Pointers are DEVICE pointers unless marked (host).  Arrays are row-major
 *    float32: positions [n][3], masses [n], accelerations [n_active][3].
 *  - The caller owns all device memory.  The library never allocates device
 *    memory (except the FFT tables of a power-spectrum plan, see
 *    sr_power_spectrum) and never synchronises, except where stated
 *    (sr_ws_flags, plan creation, the first run of a batch plan, and
 *    sr_blocks_partition).  Work is enqueued on
 *    `stream` (a hipStream_t passed as an opaque pointer; NULL is the null
 *    stream) and the call returns at once.
 *  - The workspace is caller-allocated scratch of at least the size
 *    reported by sr_workspace_bytes / sr_batch_plan_create, aligned to 256 B.
 *    Two calls that run concurrently must use different workspaces.
 *  - Argument errors are detected on the host and returned before anything
 *    is enqueued (no partial work).  n == 0 is a valid no-op.
 *  - Conditions found on the device (non-finite positions, positions outside
 *    an open domain) set bits in the workspace, read by sr_ws_flags.
 *  - All functions are thread-safe except that one plan (batch, blocks,
 *    centres or power spectrum) must not be used from two threads at once.
 */
#ifndef SR_H
#define SR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SR_ABI_VERSION 6

typedef enum sr_status {
    SR_OK = 0,
    SR_E_ARG = 1,         /* invalid argument (null pointer, bad size, bad problem) */
    SR_E_WORKSPACE = 2,   /* workspace missing, misaligned or too small */
    SR_E_DEVICE = 3,      /* a HIP runtime call failed */
    SR_E_PLAN = 4,        /* batch plan invalid or used with other sizes */
    SR_E_UNSUPPORTED = 5  /* valid request outside what this build supports */
} sr_status;

/* sr_force / sr_force_vjp flags */
#define SR_REUSE_BINS 1u /* the workspace already holds the bins of exactly these
                            pos/mass/n/n_active/problem (from sr_bin or an earlier
                            call); skips binning.  The caller guarantees it. */

/* sr_batch_force flags */
#define SR_BATCH_PER_SUBVOLUME 1u /* reference mode: one sr_force per subvolume */
#define SR_BATCH_EAGER 2u         /* batched kernels launched directly, no graph */
#define SR_BATCH_RECAPTURE 4u     /* graph mode with pointers other than those the plan's
                                     graph is bound to: capture it again (waits for the
                                     stream) instead of returning SR_E_PLAN */

/* sr_count_pairs flags */
#define SR_COUNT_ADJOINT 1u /* count the pairs the adjoint evaluates (at least one
                               active end) instead of those of the forward */

/* sr_ws_flags bits */
#define SR_FLAG_NONFINITE 1u     /* some position was NaN or infinite */
#define SR_FLAG_OUT_OF_DOMAIN 2u /* open domain: some position outside [lo, lo+len) */
#define SR_FLAG_NOT_BINNED 4u    /* SR_REUSE_BINS on a workspace without bins for these
                                    sizes: nothing was computed */
#define SR_FLAG_QUEUE 8u         /* a persistent kernel's work loop was cut short: one of
                                    its waves pulled an item out of order or more items
                                    than exist (a defect of the build or a corrupted
                                    workspace, never of the input); results incomplete */

/* One short-range problem (paper Sec. 2; softening length from Sec. 3.1).
 *  lo, len   domain origin and extent per dimension.  Periodic boxes need
 *            lo = 0 and len >= 3 r_s (at least three cells of side >= r_s
 *            per dimension, so the minimum image is the only image inside
 *            the cutoff).  Open domains accept particles anywhere; those
 *            outside [lo, lo+len) still interact correctly but set
 *            SR_FLAG_OUT_OF_DOMAIN.
 *  periodic  1: minimum-image periodic box; 0: open domain.
 *  r_s       cutoff radius (> 0).
 *  eps       Plummer softening length (>= 0); eps^2 is added to s.
 *  poly      filter polynomial coefficients poly[k] of s^k.
 *  leaf_depth  depth D of the octree inside each chaining cell whose leaves
 *            order the cell's particles (the tree-leaf variant of the binning
 *            for strongly clustered matter; tree codes are the paper's
 *            short-range solver on CPU systems, Sec. 2).  1..4; 0 means 1.
 *            D = 1 orders a cell by octant; larger D by the Z-order (Morton)
 *            code of 2^D x 2^D x 2^D sub-cells, so that each run of 64
 *            targets the pair kernels take as one item is a compact leaf.
 *            Every D gives the same interactions; only the grouping of
 *            targets, and so the work per item, changes.  Needs
 *            ncell * 2^(3 D + 1) < 2^31, else SR_E_UNSUPPORTED. */
typedef struct sr_problem {
    float lo[3];
    float len[3];
    int32_t periodic;
    float r_s;
    float eps;
    float poly[6];
    int32_t leaf_depth;
} sr_problem;

/* Device arrays of a binned workspace (all in binned order unless noted).
 * Binning rule (float32, round to nearest, no fused operations):
 *   nc_d = floor(len_d / r_s) (>= 1; >= 3 required when periodic)
 *   periodic: w = x - floor(x * (1/len)) * len;  open: w = x, u = x - lo
 *   i_d = clamp(floor(u * (nc/len)), 0, nc-1)   (u = w when periodic; NaN -> 0)
 *   cell = (i_x * nc_y + i_y) * nc_z + i_z
 *   offset = w - (lo + (i + 0.5) * (len/nc))    (distance from the cell centre)
 *   leaf code, per axis: o = offset, q = (len/nc) * 0.25;  level 1 bit
 *     b = [o >= 0];  each further level: o = b ? o - q : o + q (float32),
 *     q = q * 0.5, b = [o >= 0].  Level l contributes 4 b_x + 2 b_y + b_z
 *     as the l-th octal digit from the top: code = sum_l 8^(D-l) digit_l.
 *     With D = 1 the code is the octant 4 [off_x >= 0] + 2 [off_y >= 0] +
 *     [off_z >= 0].
 * Particles are ordered by (cell, passive, leaf code, input index): within a
 * cell the active particles come first, each group sorted by leaf code. */
typedef struct sr_bin_layout {
    int32_t nc[3];
    int64_t ncell;
    const int32_t *cell_of;    /* [n] cell of each particle, input order */
    const int32_t *cell_start; /* [ncell+1] first binned slot of each cell */
    const int32_t *cell_nact;  /* [ncell] active particles per cell (they come first) */
    const int32_t *perm;       /* [n] binned slot -> input index */
    const float *off_x;        /* [n] offsets from the cell centre */
    const float *off_y;
    const float *off_z;
    const float *mass;         /* [n] masses */
} sr_bin_layout;

typedef struct sr_batch_plan sr_batch_plan;

int sr_abi_version(void);
const char *sr_status_str(int status);

/* Host only.  Cells per dimension for a problem (the rule above). */
sr_status sr_grid(const sr_problem *prob /*host*/, int32_t nc[3] /*host out*/);

/* Host only.  Workspace bytes for sr_bin/sr_force/sr_force_vjp/sr_count_pairs/
 * sr_momentum with n particles of this problem. */
sr_status sr_workspace_bytes(int64_t n, const sr_problem *prob /*host*/, size_t *bytes /*host out*/);

/* Bin the particles into the chaining mesh: cell of each particle, stable
 * counting sort by cell, binned offsets and masses (the layout above).
 * The paper names the short-range solver's neighbour structures (chaining
 * mesh, tree) only through the HACC method papers (Sec. 2); the binning rule
 * above is this library's reading: cells of side >= r_s, so that every pair
 * inside the cutoff lies in the 27 cells around a particle's own.
 * pos [n][3], mass [n] (device, read only); 0 <= n_active <= n < 2^31.  The
 * workspace receives the bins (read by sr_force / sr_force_vjp with
 * SR_REUSE_BINS and by sr_bin_view).  Returns SR_E_ARG for a bad problem or
 * a null pointer with n > 0, SR_E_WORKSPACE for a workspace that is null,
 * misaligned or smaller than sr_workspace_bytes, SR_E_UNSUPPORTED when the
 * cells and leaf depth do not fit the 31-bit sort key. */
sr_status sr_bin(const float *pos, const float *mass, int64_t n, int64_t n_active,
                 const sr_problem *prob /*host*/, void *ws, size_t ws_bytes, void *stream);

/* Host only, no device access.  Device pointers into a workspace binned for
 * (n, n_active, prob). */
sr_status sr_bin_view(const void *ws, int64_t n, int64_t n_active, const sr_problem *prob /*host*/,
                      sr_bin_layout *out /*host out*/);

/* Short-range accelerations of the active particles: acc [n_active][3], in
 * input order, overwritten.  Bins first unless flags has SR_REUSE_BINS (then
 * n and n_active must be those of the binning: a workspace binned for other
 * sizes computes nothing and sets SR_FLAG_NOT_BINNED). */
sr_status sr_force(const float *pos, const float *mass, int64_t n, int64_t n_active,
                   const sr_problem *prob /*host*/, void *ws, size_t ws_bytes, unsigned flags,
                   float *acc, void *stream);

/* Vector-Jacobian product of the accelerations with respect to the
 * positions.  The paper has no adjoint: this is the derivative of the
 * short-range sum above (Sec. 2), added so that the force step can sit
 * inside a differentiable program.  For L = sum_{i < n_active} g_i . a_i,
 *   grad_pos[k] = dL/dx_k = sum_{j != k, s < r_s^2} [ f u + 2 f' (u.d) d ],
 *   d = x_j - x_k, u = m_k g_j - m_j g_k (g = 0 on passive rows),
 * f = f_SR(s), f' = df_SR/ds.  Pairs of two passive particles add nothing
 * (u = 0) and are not evaluated.  A pair at s = 0 (a distinct particle at the
 * same position) adds f(0) u when eps > 0, the derivative of its force term
 * m d f(|d|^2), which is smooth through d = 0; with eps = 0 it is left out.
 * Masses are constants; the jump of the cutoff is not differentiated.
 * g [n_active][3] (device, read only); grad_pos [n][3] (device, overwritten;
 * passive particles receive gradient as sources).  Pair terms are
 * recomputed, not stored.  Bins first unless flags has SR_REUSE_BINS.
 * Errors as for sr_force (SR_E_ARG also for g null with n_active > 0). */
sr_status sr_force_vjp(const float *pos, const float *mass, int64_t n, int64_t n_active,
                       const sr_problem *prob /*host*/, void *ws, size_t ws_bytes, unsigned flags,
                       const float *g, float *grad_pos, void *stream);

/* Size of the fixed device workspace of sr_force_static (64 MiB). */
#define SR_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)

/* Forward without any device allocation, for callers that cannot allocate:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Computes what sr_force computes without SR_REUSE_BINS (bin,
 * then the forward pair kernels; the same kernels, so bitwise the same
 * accelerations), but its workspace is a fixed device array of
 * SR_STATIC_WORKSPACE_BYTES inside the library, one per GPU, held until the
 * process ends.  The caller passes only inputs and outputs: pos [n][3], mass
 * [n] (device, read only), acc [n_active][3] (device, overwritten).
 * Returns SR_E_UNSUPPORTED, before touching the device, when the problem
 * needs a larger workspace than that (sr_workspace_bytes gives the need:
 * about 80 B per particle plus 12 B per cell); SR_E_DEVICE if the array's
 * address cannot be looked up; other errors as sr_force.  Never calls
 * hipMalloc or hipFree.  Every call on one GPU shares that GPU's array and
 * leaves its contents there (each call re-initialises what it reads), so
 * calls that overlap on one GPU (two streams or threads at once) race and
 * give wrong results: serialise them.  Device conditions are flagged inside
 * the array, which sr_ws_flags cannot reach.  The first call on a device
 * looks the array's address up (no allocation); make it outside stream
 * capture. */
sr_status sr_force_static(const float *pos, const float *mass, int64_t n, int64_t n_active,
                          const sr_problem *prob /*host*/, float *acc, void *stream);

/* Number of ordered pairs (i active, j) with 0 < s_ij < r_s^2, decided with
 * the same float32 arithmetic as sr_force, written to *pairs (device int64).
 * With SR_COUNT_ADJOINT: the ordered pairs (k, j) with 0 < s < r_s^2 of
 * which at least one end is active, the pairs sr_force_vjp evaluates.
 * Needs a workspace binned for these inputs. */
sr_status sr_count_pairs(int64_t n, int64_t n_active, const sr_problem *prob /*host*/, void *ws,
                         size_t ws_bytes, unsigned flags, int64_t *pairs, void *stream);

/* Momentum check: out[0..2] = sum_{i < n_rows} mass[i] * acc[i] in float64
 * (device double[3]), summed in a fixed order.  Uses the workspace as
 * scratch (size from sr_workspace_bytes for at least n_rows particles). */
sr_status sr_momentum(const float *acc, const float *mass, int64_t n_rows, void *ws,
                      size_t ws_bytes, double *out, void *stream);

/* Copy the device condition bits of a workspace to *flags (host).  Waits for
 * `stream`. */
sr_status sr_ws_flags(const void *ws, void *stream, uint32_t *flags /*host out*/);

/* Batches: B independent problems stored back to back (the independent
 * overlapping blocks of Sec. 2.1, each with its own active and passive
 * particles).  Subvolume b owns input rows [offsets[b], offsets[b+1]); its
 * first n_active[b] rows are active.  Its accelerations are written to rows
 * [A_b, A_b + n_active[b]) of acc, A_b = sum_{c<b} n_active[c].
 *
 * sr_batch_plan_create (host) validates the batch, lays out the workspace
 * and reports its size in *ws_bytes.  tune_cache (host, nullable) names a
 * JSON file in which the launch parameters, symmetric tiles and sparse-cell
 * item size measured on the first run are kept (the last two change only the
 * order of float32 sums).
 * The plan owns only host memory, one HIP stream and, after the first run
 * in graph mode, a captured HIP graph of the whole bin-then-force sequence
 * bound to the pointers (pos, mass, ws, acc, momentum) of that run.  A later
 * graph-mode run with other pointers returns SR_E_PLAN before enqueuing
 * anything, unless flags has SR_BATCH_RECAPTURE: then it waits for the stream
 * and captures again. */
sr_status sr_batch_plan_create(int32_t B, const int64_t *offsets /*host [B+1]*/,
                               const int64_t *n_active /*host [B]*/,
                               const sr_problem *probs /*host [B]*/, const char *tune_cache,
                               sr_batch_plan **plan /*host out*/, size_t *ws_bytes /*host out*/);

/* Run a batch: acc [sum n_active][3]; momentum (nullable) [B][3] float64 =
 * sum over active rows of mass * acc per subvolume.  flags:
 * SR_BATCH_PER_SUBVOLUME (one sr_force per subvolume, the reference mode),
 * SR_BATCH_EAGER (batched kernels without a graph), 0 (graph replay; with
 * SR_BATCH_RECAPTURE, capture again for new pointers).  The first run, in
 * any mode, tunes the launch parameters, the symmetric tiles and the targets
 * per item of cells with fewer than 64 targets (16, 32 or 8) by timing
 * batched runs (it synchronises), so that every mode then uses the same. */
sr_status sr_batch_force(sr_batch_plan *plan, const float *pos, const float *mass, void *ws,
                         size_t ws_bytes, float *acc, double *momentum, unsigned flags,
                         void *stream);

sr_status sr_batch_plan_destroy(sr_batch_plan *plan);

/* Host-side description of a plan: B, total particles, launch parameters
 * chosen by the tuner (writes a NUL-terminated JSON string). */
sr_status sr_batch_plan_info(const sr_batch_plan *plan, char *buf /*host*/, size_t buf_bytes);

/* Overlapping data blocks (Sec. 2.1): a domain's x-y extent is tiled by
 * rectangles in whole grid units, and each block is solved as an independent
 * open-domain problem holding its own active particles plus, as passive
 * copies, every particle within r_s of its rectangle in x and y (z is not
 * cut).  Afterwards each active particle's result is taken from its home
 * block and the duplicated passive copies are dropped.
 *
 * A rectangle [gx0, gx1) x [gy0, gy1) counts grid units of the domain: the
 * edge of unit g along an axis is lo + g * len / ng (rounded once to
 * float32).  The rectangles must tile [0, ng_x) x [0, ng_y) without gaps or
 * overlaps; the outer ones reach to infinity, so every particle, even one
 * outside the domain, has exactly one home.  Membership: a particle belongs
 * to block b if it lies within r_s (1 + 1e-5) of b's rectangle in x and in y;
 * it is active in b when it is active in the domain and b is its home.
 * Within a block the active members come first, each group in domain index
 * order.  Block b's problem is the domain with x and y cut to its widened
 * rectangle (sr_blocks_problems).  Open domains only (SR_E_UNSUPPORTED for
 * periodic ones); at most 1024 blocks. */
typedef struct sr_block {
    int32_t gx0, gx1, gy0, gy1;
} sr_block;

typedef struct sr_blocks_plan sr_blocks_plan;

/* Host only.  Validate the tiling for n particles (the first n_active
 * active) and lay out the workspace.  capacity bounds the total number of
 * memberships (0: the worst case, n times the most widened rectangles any
 * point can lie in). */
sr_status sr_blocks_plan_create(const sr_problem *domain /*host*/, const int32_t *ng /*host [2]*/,
                                int32_t nb, const sr_block *blocks /*host [nb]*/, int64_t n,
                                int64_t n_active, int64_t capacity,
                                sr_blocks_plan **plan /*host out*/, size_t *ws_bytes /*host out*/);
sr_status sr_blocks_plan_destroy(sr_blocks_plan *plan);

/* Host only.  The nb block problems (open domains). */
sr_status sr_blocks_problems(const sr_blocks_plan *plan, sr_problem *out /*host [nb]*/);

/* Assign particles to blocks.  Writes the total number of memberships to
 * *members and, per block, its active and passive member counts to
 * counts[2b], counts[2b+1] (host).  Waits for `stream` (the counts size the
 * block arrays).  If the memberships exceed the plan's capacity it returns
 * SR_E_WORKSPACE with *members set to the capacity needed.  The workspace
 * then holds the partition for the calls below until it is used otherwise. */
sr_status sr_blocks_partition(sr_blocks_plan *plan, const float *pos, void *ws, size_t ws_bytes,
                              int64_t *members /*host out*/, int64_t *counts /*host out [2 nb]*/,
                              void *stream);

/* Block inputs, blocks back to back in block order: bpos [members][3],
 * bmass [members], src [members] (nullable) = domain index of each member.
 * With g [n_active][3] (nullable, together with bg) also the cotangent rows
 * of the block outputs: bg [n_active][3], block b's active rows first after
 * those of blocks < b. */
sr_status sr_blocks_gather(const sr_blocks_plan *plan, const float *pos, const float *mass,
                           const float *g, const void *ws, size_t ws_bytes, float *bpos,
                           float *bmass, float *bg, int32_t *src, void *stream);

/* Reconcile block accelerations bacc [n_active][3] (the block outputs back
 * to back, as sr_batch_force writes them) into acc [n_active][3], domain
 * order: each active particle receives the row of its home block, once. */
sr_status sr_blocks_reconcile(const sr_blocks_plan *plan, const void *ws, size_t ws_bytes,
                              const float *bacc, float *acc, void *stream);

/* Reconcile block position gradients bgrad [members][3] (every member's row,
 * blocks back to back) into grad [n][3]: each particle receives the sum over
 * its copies, in block order. */
sr_status sr_blocks_reconcile_grad(const sr_blocks_plan *plan, const void *ws, size_t ws_bytes,
                                   const float *bgrad, float *grad, void *stream);

/* Most-bound-particle halo centres (Sec. 2.2: a halo's centre is the
 * particle at its potential minimum, found after friends-of-friends halo
 * finding).  For every particle i of halo h
 *
 *     phi_i = - sum_{j in h, j != i} m_j / sqrt(|x_j - x_i|^2 + eps^2)
 *
 * (G = 1; with eps = 0 a pair at zero distance adds nothing), and per halo
 * the particle with the smallest phi, ties to the smaller index.  Halo h
 * holds particles [offsets[h], offsets[h+1]) of pos [n][3] / mass [n];
 * coordinates are used as given (a halo finder's unwrapped positions).
 * Pair terms are float32; they are accumulated in float64 in groups of 8, so
 * the rounding does not grow with the halo size.  The most-bound choice is
 * made on the float32 phi that is returned.  Results do not depend on the
 * launch (every sum has a fixed order). */
typedef struct sr_centres_plan sr_centres_plan;

/* Host only.  Work items for n_halos halos (1 <= n_halos <= 2^26, offsets
 * non-decreasing from 0, n = offsets[n_halos] < 2^31); reports the workspace
 * size.  The plan owns only host memory (a pinned copy of its tables from
 * the first run on, where the device is first touched). */
sr_status sr_centres_plan_create(int32_t n_halos, const int64_t *offsets /*host [n_halos+1]*/,
                                 sr_centres_plan **plan /*host out*/, size_t *ws_bytes /*host out*/);
sr_status sr_centres_plan_destroy(sr_centres_plan *plan);

/* phi [n] (required), mbp [n_halos] int64 = index of the most bound particle
 * (-1 for an empty halo or one whose every phi is NaN), phi_min [n_halos]
 * (nullable) = its phi (0 when none).  eps >= 0. */
sr_status sr_centres(sr_centres_plan *plan, const float *pos, const float *mass, float eps, void *ws,
                     size_t ws_bytes, float *phi, int64_t *mbp, float *phi_min, void *stream);

/* Power spectrum on the fly (Sec. 4.1): cloud-in-cell deposit of the
 * particles onto an ng^3 periodic grid of cell h = box / ng, a DFT, and
 * P(k) = |delta(k)|^2 box^3 / ng^6 divided by the CIC window
 * W(k)^2 = prod_d sinc^4(pi n_d / ng), averaged over the modes of each bin
 * b = floor(|n| / dn) (n the integer mode vector, k = 2 pi n / box; k = 0 is
 * left out), with delta = rho / mean(rho) - 1.  Deposit: a particle at
 * u = x / h, wrapped into [0, ng), gives m (1 - f) to grid point floor(u) and
 * m f to floor(u) + 1 per axis (f = u - floor(u)), the product over axes to
 * each of 8 points; grid points sit at multiples of h.  For ng a multiple
 * of 8 the particles are sorted (stably) by brick of 8^3 cells, each run of up
 * to 2048 particles of a brick sums its weights exactly as 2^-(94 - e) fixed
 * point (2^e > 2048 max|m|; weights below 2^(e - 71) are rounded by at most
 * 2^(e - 95)) into a 9^3 tile stored as float32, and every grid point adds
 * the tiles covering it in float64 in a fixed order.  For other ng they are
 * sorted by cell, each cell's contributions are summed in float64 per
 * 64-particle run, and every grid point adds its 8 cells' partials in a fixed
 * order.  Either way the grid is reproducible bit for bit.  The FFT is rocFFT's
 * single-precision real-to-complex transform, in place in the workspace;
 * mode sums are float64.  Non-finite positions make the spectrum
 * non-finite. */
typedef struct sr_pk_plan sr_pk_plan;

/* Host only.  2 <= ng <= 1024, ng even; box > 0; 1 <= n_bins <= 2048; dn > 0
 * (bin width in units of the fundamental 2 pi / box); n_max: the most
 * particles a call will pass (sizes the workspace), 0 <= n_max < 2^31. */
sr_status sr_pk_plan_create(int32_t ng, double box, int32_t n_bins, double dn, int64_t n_max,
                            sr_pk_plan **plan /*host out*/, size_t *ws_bytes /*host out*/);
/* Releases the plan and the FFT plan's device tables. */
sr_status sr_pk_plan_destroy(sr_pk_plan *plan);

/* Deposit only: the mass grid and the total mass, in the workspace (see
 * sr_pk_grid). pos [n][3], mass [n], 0 <= n <= n_max. */
sr_status sr_pk_deposit(sr_pk_plan *plan, const float *pos, const float *mass, int64_t n, void *ws,
                        size_t ws_bytes, void *stream);

/* Host only, no device access.  Device pointers into the workspace: the grid
 * (mass at point (ix, iy, iz) at grid[(ix * ng + iy) * row_pitch + iz], valid
 * after sr_pk_deposit and overwritten by the FFT of sr_power_spectrum) and the
 * float64 total mass (nullable). */
sr_status sr_pk_grid(const sr_pk_plan *plan, const void *ws, const float **grid /*host out*/,
                     int32_t *row_pitch /*host out*/, const double **mass_total /*host out*/);

/* Deposit, FFT and bins: pk [n_bins] float64, k [n_bins] float64 (nullable:
 * the bin's mean |k|), modes [n_bins] int64 (nullable: modes in the bin, the
 * full grid counted).  Empty bins give 0.  The first call creates the rocFFT
 * plan on the current device: it compiles or loads the transform's kernels
 * and keeps its twiddle tables in device memory it allocates itself (the one
 * device allocation the library makes), released by sr_pk_plan_destroy. */
sr_status sr_power_spectrum(sr_pk_plan *plan, const float *pos, const float *mass, int64_t n, void *ws,
                            size_t ws_bytes, double *pk, double *k, int64_t *modes, void *stream);

/* Host only.  Process-wide launch parameters of the single-problem entry
 * points (batch plans tune their own):
 *   waves_per_cu      persistent grid of the pair kernels, in waves per compute
 *                     unit (1..64; 0 keeps the current value);
 *   targets_per_lane  1 or 2: with 2, a wave holds two targets per lane in cells
 *                     with more than 64 targets (0 keeps the current value);
 *   occupancy         register-allocation variant of the pair kernels: 0 (none),
 *                     6 or 8 waves per SIMD (-1 keeps the current value).
 * None of them changes results: every target sums its sources in the same
 * order.  sr_launch_config sets the forward and adjoint kernels alike and
 * writes the forward kernel's values in effect to cur (host, nullable,
 * int[3]).  The initial values differ per kernel (forward: 32, 1, 6; adjoint:
 * 24, 2, 0, the fastest measured); SR_WAVES_PER_CU / SR_TARGETS_PER_LANE /
 * SR_OCCUPANCY override them for both (see also sr_sparse_group). */
sr_status sr_launch_config(int waves_per_cu, int targets_per_lane, int occupancy,
                           int *cur /*host out*/);

/* Host only.  The same for one kernel: "force" (also sr_count_pairs) or
 * "vjp"; cur receives that kernel's values. */
sr_status sr_launch_config_kernel(const char *kernel /*host*/, int waves_per_cu,
                                  int targets_per_lane, int occupancy, int *cur /*host out*/);

/* Host only.  Tiles of the symmetric pair kernels of one kernel ("force" or
 * "vjp").  Inside cells with at least 64 active particles (their full
 * blocks of 64 are the dense particles) each unordered pair of dense
 * particles is evaluated once and its opposite term kept as well (Newton's
 * third law on the short-range sum of Sec. 2); the rest is summed from both
 * ends as before.  blocks_per_item: blocks of 64 targets one work item takes
 * (1..256; 0 switches the symmetric tiles off; -1 keeps the value); window:
 * sources per work item, 256 or 512 (-1 keeps).  Larger tiles need fewer
 * partial slots but make longer items.  The partial slots (12 bytes each)
 * fill the tail of the workspace: sr_workspace_bytes reserves about 15 per
 * particle, and a larger workspace passed to sr_force / sr_force_vjp lends
 * its whole tail to them.  A problem that needs more (very large cells) runs
 * without symmetric tiles.  Results differ from the one-sided sums only in rounding
 * order; for fixed tiles they are bitwise reproducible.  cur (nullable)
 * receives {blocks_per_item, window}. */
sr_status sr_tile_config(const char *kernel /*host*/, int blocks_per_item, int window,
                         int *cur /*host out*/);

/* Host only.  Most targets per item of a cell, or the remainder of a cell,
 * with fewer than 64 targets: 8, 16, 32 or 64 (-1 keeps the value; initial
 * 16, or SR_SPARSE_GROUP).  Smaller groups have tighter boxes and stage their
 * sources more often; the choice changes only the order of float32 sums.
 * Batch plans tune their own.  cur (nullable) receives the value in effect. */
sr_status sr_sparse_group(int group, int *cur /*host out*/);

/* Host only.  When the symmetric tiles pay: they run only if their work (tile
 * steps of all items) spread over the persistent grid's waves is at least
 * min_ratio times the longest item, so that a few long items cannot leave
 * most waves idle; the decision is taken on the device after binning, like
 * the pool check.  min_ratio >= 0 (0: whenever the partial slots fit; -1
 * keeps the value); initial value 1, or SR_SYM_BALANCE.  Batch plans do not
 * apply it: their tuner times the tiles against none, and every mode of a
 * plan takes the same decision.  Results of either path agree to rounding
 * order; cur (nullable) receives the value in effect. */
sr_status sr_tile_balance(double min_ratio, double *cur /*host out*/);

/* Kernel timing with HIP events recorded on the launch stream around every
 * launch of the pair kernels ("force", "vjp").  sr_timing_enable(1) clears
 * and starts recording; sr_timing_read waits for the recorded events and
 * returns the summed milliseconds and the launch count of one kernel. */
sr_status sr_timing_enable(int on);
sr_status sr_timing_read(const char *kernel, double *total_ms /*host out*/,
                         int64_t *launches /*host out*/);

#ifdef __cplusplus
}
#endif
#endif /* SR_H */
