/*
 * md.h -- C ABI of libmdgpu: the per-step hot path of short-range
 * Lennard-Jones molecular dynamics on one MI355X (gfx950).
 *
 * Method: H. Watanabe, M. Suzuki, N. Ito, "Huge-scale Molecular Dynamics
 * Simulation of Multibubble Nuclei" (arXiv:1210.3450):
 *   - pair potential: Eq. (1), Sec. II.A, truncated at rc with c2, c0 chosen so
 *     that V(rc) = V'(rc) = 0;
 *   - pair search: grid (cell / linked-list) algorithm, Sec. II.A;
 *   - pair list: bookkeeping (Verlet) list registering pairs within
 *     r_list = rc + skin, reused for several steps, Sec. II.A; key/partner
 *     sorted form of Fig. 1 (KeyPointer / SortedList);
 *   - list validity: dynamic upper time cutoff (DUTC) checked every step,
 *     Sec. II.A;
 *   - force: the scalar f(r) = (24 r^6 - 48) / r^14 + 8 c2 of Algorithm 1
 *     (Sec. III.C), F_i += f (q_j - q_i), full list, no scattered stores;
 *   - integrator: second-order symplectic (velocity Verlet), Sec. III.B.
 * Reduced LJ units: sigma = epsilon = k_B = 1 (Sec. II.A).
 *
 * Conventions for every entry point:
 *   - Every function returns md_status.  The library never throws, aborts or
 *     exits.  On failure md_last_error(ctx) holds a message.
 *   - Array arguments named "device" are HIP device pointers; "host" are host
 *     pointers.  Particle arrays are [n][3] float64, row-major, in CALLER order
 *     (the order given to md_set_state; for an ensemble, boxes concatenated in
 *     box order).
 *   - The caller owns every pointer it passes.  The library copies what it needs
 *     on the context's stream and keeps no caller pointer after returning.
 *   - The context owns all internal device memory; it is allocated in
 *     md_create / md_batch_create.  Afterwards only a list build whose capacity
 *     overflowed grows the list, md_rescale_box re-allocates the cell arrays
 *     when the number of cells changes, and md_autotune re-allocates the cell
 *     and list arrays for the layout it picks (plus a caller-order copy of the
 *     state on its first call).  No allocation happens per step otherwise.
 *   - Calls are asynchronous on the context stream unless marked
 *     "synchronizing".  A context is not thread-safe; distinct contexts are
 *     independent.
 *   - A device failure (HIP error) is sticky: every later call returns
 *     MD_EHIP until md_destroy.
 */
#ifndef MDGPU_MD_H
#define MDGPU_MD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct md_ctx md_ctx; /* opaque: one box, or an ensemble of boxes */

typedef enum {
    MD_OK = 0,
    MD_EINVAL = -1,    /* bad argument, geometry or parameter */
    MD_ENOMEM = -2,    /* device allocation failed */
    MD_EHIP = -3,      /* HIP runtime or kernel failure (sticky) */
    MD_ENUMERIC = -4,  /* non-finite position, or outside [-L, 2L) at binning */
    MD_ESTATE = -5,    /* call out of order (e.g. step before set_state) */
    MD_ELIST = -6      /* list verifier found a pair within rc missing from the list */
} md_status;

/* precision of the pair force */
#define MD_PREC_FP64 0        /* all arithmetic in FP64 */
#define MD_PREC_FP32_MIXED 1  /* pair forces in FP32 on cell-relative coordinates,
                                 compensated FP32 sums per particle; positions,
                                 velocities, integration and energy totals FP64 */
/* cutoff scheme */
#define MD_CUT_EQ1 0   /* Eq. (1): c2, c0 from V(rc) = V'(rc) = 0 (default) */
#define MD_CUT_SHIFT 1 /* c2 = 0, c0 from V(rc) = 0 (tests) */
#define MD_CUT_RAW 2   /* c2 = c0 = 0 inside rc (tests) */
/* list rebuild policy */
#define MD_REBUILD_DUTC 0          /* D += dt * max|v| after each drift; rebuild when 2D > skin */
#define MD_REBUILD_DISPLACEMENT 1  /* rebuild when 2 * max_i |q_i - q_i(build)| > skin */
#define MD_REBUILD_EVERY_STEP 2
#define MD_REBUILD_NEVER 3         /* tests only: the list goes stale */
/* flags */
#define MD_F_VERIFY_LIST 1u        /* debug: after every force evaluation count pairs within
                                      rc missing from the list (O(n^2) per box) */
#define MD_F_GRAPH 2u              /* replay md_step chunks as captured HIP graphs */
#define MD_F_TILE_ON 4u            /* row tiles (threads_per_key 0 or 1; the FP32-mixed default for a
                                      largest box of 2^23 particles or more): each row of cells is
                                      cut into runs of cells whose partners (the 9 neighbouring rows,
                                      one cell wider each side) a block stages in LDS once (fixed-point
                                      records for FP32-mixed, FP64 positions for FP64); list entries
                                      name staged records and the force pass reads every partner from
                                      LDS.  A context whose cells are too crowded for the staging
                                      capacity (about 2400 particles around one cell) switches to the
                                      gather format by itself. */
#define MD_F_TILE_OFF 8u           /* the gather format instead of row tiles (every partner read from
                                      global memory by cell and rank; the default for FP64 and for
                                      smaller FP32-mixed boxes) */
#define MD_F_FAST_RCP 16u          /* FP64 path: 1/r^2 from the hardware reciprocal, with the
                                      correction of Sec. III.C applied to r^-6, r^-8, r^-12 and
                                      r^-14 (r^-2n ~ xt^n ((n + 1) - n xt r^2)) instead of a division */
#define MD_F_HALF_LIST 32u         /* half list with Newton's third law (Sec. II.A, Fig. 1 holds each
                                      pair once): a key lists its partners in the home cell after
                                      itself and in the 13 forward stencil cells; the force pass sends
                                      each pair's reaction to the partner (accumulated per wavefront in
                                      LDS and flushed with atomic adds where the wavefront's partners
                                      form contiguous row segments, else added atomically at once), then
                                      a separate pass integrates.  One lane per key (threads_per_key 0 or 1); not
                                      with MD_F_VERIFY_LIST or MD_F_TILE_ON.  Forces agree with the
                                      full list within the precision's tolerance but are not bitwise
                                      reproducible (the order of the atomic additions varies). */

typedef struct {
    int64_t n;            /* particles in the box, >= 2 */
    double box[3];        /* orthorhombic periodic lengths; each >= 3 * (rc + skin) */
    double rc;            /* cutoff, > 0 (2.5 benchmarks, 3.0 cavitation) */
    double skin;          /* list margin, >= 0; r_list = rc + skin */
    double dt;            /* time step, > 0 */
    double mass;          /* particle mass, > 0 */
    int32_t precision;    /* MD_PREC_* */
    int32_t cutoff;       /* MD_CUT_* */
    int32_t rebuild;      /* MD_REBUILD_* */
    uint32_t flags;       /* MD_F_* */
    int32_t threads_per_key; /* lanes cooperating on one particle's list: 0 = default,
                                else 1, 2, 4 or 8 */
    int32_t list_cap;     /* list entries per particle: 0 = estimate from density */
    double cell_scale;    /* grid cells of side >= cell_scale * r_list (Sec. II.A grid
                             algorithm: any side >= r_list keeps the 27-cell search exact):
                             0 = 1, the smallest such cells; else in [1, 2] */
    uint64_t reserved[5]; /* must be zero */
} md_params;

typedef struct {
    int64_t steps;        /* steps taken by md_step since creation */
    int64_t rebuilds;     /* list builds (all boxes summed) */
    int64_t list_regrows; /* capacity overflows recovered by growing the list */
    int64_t missed_pairs; /* with MD_F_VERIFY_LIST: pairs within rc absent from the list */
    int64_t list_entries; /* entries in the current lists (all boxes) */
    int32_t max_list_len; /* longest list of any particle */
    int32_t list_cap;     /* current capacity per particle */
    int32_t threads_per_key;
    int32_t nbox;
    double D;             /* DUTC bound accumulated since the last build (box 0) */
    double force_ms;      /* with timing on: summed force-kernel time (HIP events) */
    int64_t force_launches;
    double rebuild_ms;    /* with timing on: summed time of list-build chains */
    int64_t rebuild_launches;
    int32_t row_tiles;    /* 1: the force pass reads partners from row tiles staged in LDS;
                             0: from global memory (gather format) */
    int32_t ncell[3];     /* box 0's cells per axis */
    double cell_scale;    /* cell side lower bound in use, as a multiple of r_list */
} md_stats;

/* ---- lifetime ---------------------------------------------------------- */

/* Creates a context for one periodic box (all of Sec. II.A's hot path).
 * params: host pointer, validated synchronously: MD_EINVAL for n < 2,
 * rc <= 0, skin < 0, dt <= 0, mass <= 0, non-finite values, a box side below
 * 3 * (rc + skin) (the 27-cell search needs >= 3 cells per axis), unknown
 * enum values, nonzero reserved words, or more than 2^27 particle slots.
 * stream: a hipStream_t, or NULL for a stream owned by the context.
 * On MD_OK *out holds the context; on failure *out is NULL. */
md_status md_create(const md_params *params, void *stream, md_ctx **out);

/* Ensemble of nbox independent periodic boxes advanced together (every kernel
 * covers all boxes in one launch).  boxes: host array [nbox]; rc, skin, dt,
 * mass, precision, cutoff, rebuild, flags and threads_per_key must agree
 * across boxes (MD_EINVAL otherwise); n and box may differ.  Particle arrays
 * of the other calls are concatenated in box order. */
md_status md_batch_create(const md_params *boxes, int32_t nbox, void *stream, md_ctx **out);

/* Frees everything the context owns.  NULL-safe. */
md_status md_destroy(md_ctx *ctx);

/* ---- state ------------------------------------------------------------- */

/* Loads positions and velocities: device [n][3] each (n = total particles).
 * Positions must lie in [-L, 2L) per axis (checked at the next binning).
 * Invalidates the list and the stored forces. */
md_status md_set_state(md_ctx *ctx, const double *pos, const double *vel);

/* Copies the current state out: device [n][3] each (either may be NULL).
 * Positions are as integrated: wrapped into [0, L) at the last list build and
 * drifted since.  Velocities are at the same (synchronized) time. */
md_status md_get_state(md_ctx *ctx, double *pos, double *vel);

/* Scales every box length and position by alpha (> 0), keeping velocities:
 * the uniform adiabatic expansion of Sec. IV.A.  MD_EINVAL if a box would
 * drop below 3 * (rc + skin) per axis.  Invalidates list and forces. */
md_status md_rescale_box(md_ctx *ctx, double alpha);

/* Multiplies every velocity of box b by scale[b] (host array [nbox]).
 * Temperature control by rescaling during equilibration. */
md_status md_scale_velocities(md_ctx *ctx, const double *scale);

/* ---- hot path ---------------------------------------------------------- */

/* Grid binning at the current positions (Sec. II.A grid algorithm):
 * wraps positions into [0, L), assigns each particle the cell
 * min((int)(x * n/L), n - 1) per axis with n = floor(L / r_list), and
 * counting-sorts particles by cell (ties by caller id) into the context's
 * coalesced arrays.  MD_ENUMERIC if a position is not finite or outside
 * [-L, 2L) (reported at the next synchronizing call). */
md_status md_build_cells(md_ctx *ctx);

/* Builds the bookkeeping pair list (Sec. II.A, Fig. 1) from fresh cells: every
 * ordered pair (i, j), i != j, with minimum-image distance < rc + skin.
 * Resets the DUTC bound D to 0.  Grows the list if a particle has more
 * partners than the capacity. */
md_status md_build_neighbors(md_ctx *ctx);

/* Forces at the current positions (Algorithm 1's scalar, full list), without
 * moving anything.  Rebuilds the list first if it is not valid.
 * force: device [n][3] in caller order, or NULL (forces kept internally). */
md_status md_compute_forces(md_ctx *ctx, double *force);

/* Advances nsteps velocity-Verlet steps (Sec. III.B).  Per step: half kick,
 * drift, DUTC check (Sec. II.A), list rebuild when needed, forces, half kick.
 * energy_every > 0 records KE and PE every energy_every steps (read back with
 * md_energy_series).  With MD_F_VERIFY_LIST returns MD_ELIST if the verifier
 * found a missed pair.  Synchronizes every 200 steps and at the end of the call
 * to check list overflow and numeric errors.  A list build that overflows (the
 * list's capacity, or a row tile's staging capacity) stops the kernels of its
 * step; the library then grows the list (or switches to the gather format) and
 * goes on from that build, so the run equals one that had room from the start.
 * If growing the list fails (MD_ENOMEM) the state is left drifted within that
 * step and the next call rebuilds the list. */
md_status md_step(md_ctx *ctx, int32_t nsteps, int32_t energy_every);

/* Kinetic and potential energy at the current (synchronized) state, summed
 * over all boxes: ke = 1/2 m sum v^2, pe = sum over pairs i<j, r < rc of V(r)
 * (Eq. 1).  host pointers (either may be NULL).  Synchronizing. */
md_status md_energy(md_ctx *ctx, double *ke, double *pe);

/* Per-box energies at the current state: host arrays [nbox].  Synchronizing. */
md_status md_batch_energy(md_ctx *ctx, double *ke, double *pe);

/* Energies recorded by md_step(energy_every > 0) since the last md_set_state:
 * host arrays [max][nbox] (sample-major); *count receives the number of
 * samples available (at most the internal capacity of 4096).  Synchronizing. */
md_status md_energy_series(md_ctx *ctx, double *ke, double *pe, int32_t max, int32_t *count);

/* Pair virial and thermostat share at the same samples as md_energy_series:
 * host arrays [max][nbox]: vir = sum over pairs i < j within rc of f(r) r^2
 * (f = V'(r)/r, the Algorithm 1 scalar), so that the pressure of box b at a
 * sample is P = (2 KE - vir) / (3 V); thermostat = Q xi^2 / 2 + g T eta (zero
 * without a thermostat), so that KE + PE + thermostat is conserved.
 * Synchronizing; either pointer may be NULL. */
md_status md_observable_series(md_ctx *ctx, double *vir, double *thermostat, int32_t max, int32_t *count);

/* Virial pressure of every box at the current state, P = (2 KE - vir) / (3 V)
 * (host double [nbox]).  Evaluates forces and energies (like md_energy);
 * synchronizing. */
md_status md_pressure(md_ctx *ctx, double *pressure);

/* Nose-Hoover thermostat for the equilibration of the cavitation runs (Sec. IV.A):
 * dv/dt = F/m - xi v, dxi/dt = (2 KE - g T) / Q, deta/dt = xi, with g = 3N - 3 and
 * Q = g T tau^2, integrated as thermostat(dt/2), velocity Verlet, thermostat(dt/2)
 * per step (KE + PE + Q xi^2 / 2 + g T eta is conserved).  T: host double [nbox]
 * (> 0), tau: relaxation time; tau <= 0 switches the thermostat off (NVE, T may
 * be NULL).  Resets xi = eta = 0; the setting survives md_set_state.  While a
 * thermostat is on, md_step runs every step unfused (no graph replay). */
md_status md_set_thermostat(md_ctx *ctx, const double *T, double tau);
md_status md_get_thermostat(md_ctx *ctx, double *xi, double *eta);  /* host [nbox], nullable */

/* ---- bubble identification (Sec. IV.B) ---------------------------------- */

typedef struct {
    int32_t nsub[3];   /* subcells per axis, floor(L / side) */
    int32_t pad;
    double side[3];    /* subcell edges L / nsub */
    double threshold;  /* a subcell is gas iff its count < rho_gas * volume of a subcell */
    int64_t ngas;      /* gas subcells */
    int64_t nbubbles;  /* bubbles: clusters of face-adjacent gas subcells, periodic */
    int64_t largest;   /* subcells in the largest bubble, 0 without bubbles */
} md_bubble_info;

/* Bubbles of box `box` at the current positions, as in the analysis of Sec. IV.B.
 * The box is cut into nsub = floor(L / side) subcells per axis (edge L / nsub,
 * so at least `side`); every particle is wrapped into [0, L) and binned with
 * min((int)(x * nsub / L), nsub - 1).  A subcell's particle count is held in
 * one unsigned byte (saturating at 255); the subcell is gas when that count is
 * below rho_gas * (L0/n0) * (L1/n1) * (L2/n2) (FP64, evaluated left to right).
 * Gas subcells sharing a face, across periodic faces too, form one bubble
 * (site percolation on the simple cubic lattice); each bubble is labelled by
 * its smallest linear subcell index (cz * ny + cy) * nx + cx.
 *   counts  device uint8 [nsub total] or NULL: the byte counts;
 *   labels  device int32 [nsub total] or NULL: bubble label, -1 for liquid;
 *   roots, sizes  host int64 [cap] or NULL (cap = 0): the first min(cap,
 *           nbubbles) bubbles in ascending label order and their sizes in
 *           subcells;
 *   info    host, required.
 * MD_EINVAL: bad box index, side not finite or <= 0, rho_gas not finite or
 * < 0, fewer than 1 or more than 1024 subcells on an axis, info NULL.
 * MD_ESTATE without a state; MD_ENUMERIC for a position outside [-L, 2L).
 * Work buffers (about 17 bytes per subcell) are allocated on the first call and
 * grown when needed.  Synchronizing. */
md_status md_bubbles(md_ctx *ctx, int32_t box, double side, double rho_gas, uint8_t *counts,
                     int32_t *labels, int64_t *roots, int64_t *sizes, int64_t cap,
                     md_bubble_info *info);

/* The same analysis for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * arguments, results, errors and ordering exactly as md_bubbles, but every work
 * buffer lives in a fixed device array of the library (about 32 MiB per GPU,
 * taken when the library's code is loaded on that GPU and held until the
 * process ends), so the call performs no device allocation or free.  Limit:
 * at most 2^20 subcells per call (MD_EINVAL beyond).  All calls on one GPU
 * share that array and each call clears what it needs first; calls that
 * overlap in time on one GPU (several threads, or several streams) race and
 * must be serialised by the caller.  Synchronizing. */
md_status md_bubbles_noalloc(md_ctx *ctx, int32_t box, double side, double rho_gas, uint8_t *counts,
                             int32_t *labels, int64_t *roots, int64_t *sizes, int64_t cap,
                             md_bubble_info *info);

/* ---- diagnostics and parity (synchronizing) ----------------------------- */

/* Cell of every particle at the last binning, box-local linear id
 * (cz * ny + cy) * nx + cx: device int32 [n] in caller order.
 * ncell: host int32 [3] (box 0's grid).  MD_ESTATE before any binning. */
md_status md_get_cells(md_ctx *ctx, int32_t *cell_of_particle, int32_t *ncell);

/* The current pair list as the full sorted list of Fig. 1 in caller ids:
 * key_ptr device int64 [n + 1], partners device int32 [cap], partners of
 * each key ascending (box-local caller ids for ensembles are global ids).
 * With MD_F_HALF_LIST each pair appears once, under the key whose forward
 * stencil (or later rank in the same cell) holds the partner.
 * *total (host) receives the entry count; if it exceeds cap nothing is
 * written to partners and MD_EINVAL is returned.  MD_ESTATE without a list. */
md_status md_get_neighbors(md_ctx *ctx, int64_t *key_ptr, int32_t *partners, int64_t cap,
                           int64_t *total);

/* Counters and timings.  host pointer. */
md_status md_get_stats(md_ctx *ctx, md_stats *out);

/* Turns per-launch HIP-event timing of the force kernel and of list-build
 * chains on (1) or off (0); timings accumulate in md_stats. */
md_status md_set_timing(md_ctx *ctx, int32_t on);

/* Picks the layout of the force pass and the grid by timing them on the current
 * state: the cell side (cell_scale 1, 1.15 or 1.3 times r_list), the list format
 * (row tiles or gather format, FP32-mixed only) and threads_per_key (1, 2, 4 or 8,
 * gather format), for a cost of force-pass time + list-build time / R, where R is
 * the context's mean rebuild interval so far (10 steps before any step).  Leaves
 * the state as it was and rebuilds the list in the chosen layout; md_get_stats
 * reports the choice.  cache_path (nullable): a text file of lines
 * "precision density_bucket n_bucket ensemble threads_per_key row_tiles
 * cell_scale_percent", consulted first (a matching line skips the timing) and
 * appended to.  MD_F_TILE_OFF and MD_F_TILE_ON restrict the format; a
 * threads_per_key fixed at creation restricts that; a cell_scale given at
 * creation restricts the cell side.  With MD_F_HALF_LIST nothing is timed.
 * Synchronizing. */
md_status md_autotune(md_ctx *ctx, const char *cache_path);

/* ---- errors ------------------------------------------------------------ */

const char *md_status_str(md_status s);
/* Message of the last failure on ctx; with ctx == NULL, of the calling
 * thread's last failed md_create / md_batch_create.  "" when none; never NULL. */
const char *md_last_error(const md_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* MDGPU_MD_H */
