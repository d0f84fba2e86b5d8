/*
 * md_oracle.c -- plain, slow FP64 CPU oracle for the truncated Lennard-Jones
 * hot path.  TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the
 * benchmark's CPU-baseline leg call it; the HIP library never links, loads or
 * calls it, and it shares no code with the HIP library.
 *
 * What it computes (Watanabe, Suzuki & Ito, "Huge-scale Molecular Dynamics
 * Simulation of Multibubble Nuclei"):
 *   - the truncated pair potential of Eq. (1), Sec. II.A, with c2 and c0 fixed
 *     by V(rc) = V'(rc) = 0;
 *   - the pair force scalar of Algorithm 1 (Sec. III.C), f(r) = V'(r)/r, applied
 *     as F_i += f * (q_j - q_i);
 *   - the grid (linked-list) search for pairs, Sec. II.A;
 *   - the bookkeeping (Verlet) pair list with a margin beyond rc, Sec. II.A, held
 *     as the sorted list of Fig. 1: KeyPointer[N+1] + SortedList[], key = the
 *     smaller index; the full (both-direction) form is also produced;
 *   - a second-order symplectic step (velocity Verlet, kick-drift-kick), the
 *     benchmark integrator of Sec. III.B;
 *   - the list-validity check of Sec. II.A (dynamic upper time cutoff): the
 *     accumulated bound D += dt * max|v| after each drift, rebuild when
 *     2D > skin;
 *   - the pair virial and a Nose-Hoover thermostat (the equilibration of the
 *     cavitation runs, Sec. IV.A), with the conserved extended energy;
 *   - the approximate reciprocal of Sec. III.C and its correction of r^-8 and
 *     r^-14 (a model instruction with relative error below 1/256), as an
 *     alternative force evaluation for the energy-conservation comparison.
 *   - the bubble identification of Sec. IV.B: per-subcell particle counts in
 *     one byte, a gas threshold on the local density and site percolation of
 *     gas subcells on the periodic simple cubic lattice.
 *
 * Readings where the paper is silent are listed in the repository's design
 * notes; the ones that shape arithmetic here are: strict "<" at rc and at the
 * list radius; minimum image d = t - L*rint(t/L) with ties to even; mass 1 unless
 * given; wrap "if (x < 0) x += L; if (x >= L) x -= L" before binning; cell count
 * floor(L / r_list) per axis with the cell index min((int)(x * (n/L)), n-1).
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC.
 * No FMA contraction anywhere, so list decisions are reproducible bit for bit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_CUT_EQ1 0   /* Eq. (1): c2, c0 from V(rc) = V'(rc) = 0 */
#define ORC_CUT_SHIFT 1 /* plain shift: c2 = 0, V(rc) = 0 only (tests) */
#define ORC_CUT_RAW 2   /* untruncated 12-6 shape inside rc: c2 = c0 = 0 (tests) */

#define ORC_REBUILD_DUTC 0
#define ORC_REBUILD_DISPLACEMENT 1
#define ORC_REBUILD_EVERY_STEP 2
#define ORC_REBUILD_NEVER 3

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------- potential */

/* c2 and c0 of Eq. (1).  V/4 = r^-12 - r^-6 + c2 r^2 + c0.
 * V'(rc) = 0: -12 rc^-13 + 6 rc^-7 + 2 c2 rc = 0  ->  c2 = 6 rc^-14 - 3 rc^-8.
 * V(rc)  = 0: c0 = -rc^-12 + rc^-6 - c2 rc^2      ->  c0 = -7 rc^-12 + 4 rc^-6. */
void orc_coeffs(double rc, int mode, double *c2, double *c0) {
    double s = 1.0 / (rc * rc);
    double s3 = s * s * s;
    if (mode == ORC_CUT_EQ1) {
        *c2 = 6.0 * s3 * s3 * s - 3.0 * s3 * s;
        *c0 = -7.0 * s3 * s3 + 4.0 * s3;
    } else if (mode == ORC_CUT_SHIFT) {
        *c2 = 0.0;
        *c0 = -(s3 * s3 - s3);
    } else {
        *c2 = 0.0;
        *c0 = 0.0;
    }
}

/* V(r) of Eq. (1) inside the cutoff (the caller applies r^2 < rc^2). */
double orc_pair_v(double r2, double c2, double c0) {
    double s = 1.0 / r2;
    double s3 = s * s * s;
    return 4.0 * (s3 * s3 - s3 + c2 * r2 + c0);
}

/* f(r) = (24 r^6 - 48) / r^14 + 8 c2 of Algorithm 1, i.e. V'(r)/r.
 * With s = r^-2: 24 s^4 - 48 s^7 + 8 c2. */
double orc_pair_f(double r2, double c2) {
    double s = 1.0 / r2;
    double s3 = s * s * s;
    return (24.0 * s3 - 48.0 * s3 * s3) * s + 8.0 * c2;
}

/* ------------------------------------------------- approximate reciprocal (Sec. III.C)
 * The paper's SIMD kernel replaces the divide by a reciprocal approximation with
 * relative error below 1/256 and corrects the powers of it that the force needs:
 * with xt the approximation of 1/r^2 and xt r^2 = 1 + e,
 *   r^-2n = xt^n (1 + e)^-n = xt^n (1 - n e + O(e^2)) = xt^n ((n + 1) - n xt r^2) + O(e^2).
 * orc_rcp_approx models such an instruction: 1/x with its mantissa cut to 8 bits
 * after the leading one (relative error below 2^-8). */
double orc_rcp_approx(double x) {
    int e;
    double m = frexp(1.0 / x, &e); /* 1/x = m 2^e, m in [0.5, 1) */
    return ldexp(floor(m * 512.0) / 512.0, e);
}

/* xt^n, times the correction factor (n + 1) - n xt r^2 when corr != 0. */
double orc_rpow_approx(double r2, double xt, int n, int corr) {
    double p = 1.0;
    for (int k = 0; k < n; ++k) p *= xt;
    return corr ? p * ((double)(n + 1) - (double)n * xt * r2) : p;
}

/* f(r) and V(r) of Eq. (1) from an approximate reciprocal xt of r^2:
 * f = 24 r^-8 - 48 r^-14 + 8 c2, V = 4 (r^-12 - r^-6 + c2 r^2 + c0). */
double orc_pair_f_rcp(double r2, double c2, double xt, int corr) {
    return 24.0 * orc_rpow_approx(r2, xt, 4, corr) - 48.0 * orc_rpow_approx(r2, xt, 7, corr) + 8.0 * c2;
}
double orc_pair_v_rcp(double r2, double c2, double c0, double xt, int corr) {
    return 4.0 * (orc_rpow_approx(r2, xt, 6, corr) - orc_rpow_approx(r2, xt, 3, corr) + c2 * r2 + c0);
}

/* Reciprocal modes of the force evaluation:
 *   0 IEEE division (the plain definition),
 *   1 approximate reciprocal (orc_rcp_approx) without correction,
 *   2 approximate reciprocal with the correction,
 *   3 exact reciprocal through the corrected formulas (the correction then vanishes). */
static void pair_fv(double r2, double c2, double c0, int rcp, double *f, double *v) {
    if (rcp == 0) {
        *f = orc_pair_f(r2, c2);
        *v = orc_pair_v(r2, c2, c0);
        return;
    }
    double xt = rcp == 3 ? 1.0 / r2 : orc_rcp_approx(r2);
    int corr = rcp != 1;
    *f = orc_pair_f_rcp(r2, c2, xt, corr);
    *v = orc_pair_v_rcp(r2, c2, c0, xt, corr);
}

/* ---------------------------------------------------------------- geometry */

/* Minimum image of t = q_j - q_i along one axis of length L (ties to even). */
static double min_image(double t, double L) { return t - L * rint(t / L); }

static double dist2(const double *q, int64_t i, int64_t j, const double *L, double *d) {
    double dx = min_image(q[3 * j + 0] - q[3 * i + 0], L[0]);
    double dy = min_image(q[3 * j + 1] - q[3 * i + 1], L[1]);
    double dz = min_image(q[3 * j + 2] - q[3 * i + 2], L[2]);
    if (d) { d[0] = dx; d[1] = dy; d[2] = dz; }
    return dx * dx + dy * dy + dz * dz;
}

/* Cells per axis, n = floor(L / r_list), and the factor n / L. */
void orc_cell_grid(const double *L, double r_list, int32_t *n, double *inv) {
    for (int a = 0; a < 3; ++a) {
        n[a] = (int32_t)floor(L[a] / r_list);
        inv[a] = (double)n[a] / L[a];
    }
}

/* Wrap positions into [0, L) in place and compute each particle's linear cell
 * id (cz*ny + cy)*nx + cx.  Returns 0, or -1 when a coordinate is not finite or
 * lies outside [-L, 2L), or -2 when some axis has fewer than 3 cells. */
int orc_cells(int64_t n, double *q, const double *L, double r_list, int32_t *cell, int32_t *ncell) {
    double inv[3];
    orc_cell_grid(L, r_list, ncell, inv);
    for (int a = 0; a < 3; ++a)
        if (ncell[a] < 3) return -2;
    int bad = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t c[3];
        for (int a = 0; a < 3; ++a) {
            double x = q[3 * i + a];
            if (!(x >= -L[a] && x < 2.0 * L[a])) { bad = 1; c[a] = 0; continue; }
            if (x < 0.0) x += L[a];
            if (x >= L[a]) x -= L[a];
            q[3 * i + a] = x;
            int32_t k = (int32_t)(x * inv[a]);
            if (k > ncell[a] - 1) k = ncell[a] - 1;
            c[a] = k;
        }
        cell[i] = (c[2] * ncell[1] + c[1]) * ncell[0] + c[0];
    }
    return bad ? -1 : 0;
}

/* Linked-list cell structure: head[cell] -> first particle, next[i] -> next
 * particle of the same cell, -1 terminates.  Particles are pushed in
 * descending index order so each chain lists its members ascending. */
typedef struct {
    int32_t n[3];
    int64_t ncell;
    int64_t *head;
    int64_t *next;
    int32_t *cell;
} cell_list;

static void cells_free(cell_list *cl) {
    free(cl->head); free(cl->next); free(cl->cell);
    memset(cl, 0, sizeof(*cl));
}

static int cells_build(int64_t n, double *q, const double *L, double r_list, cell_list *cl) {
    memset(cl, 0, sizeof(*cl));
    cl->cell = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int rc = orc_cells(n, q, L, r_list, cl->cell, cl->n);
    if (rc != 0) { cells_free(cl); return rc; }
    cl->ncell = (int64_t)cl->n[0] * cl->n[1] * cl->n[2];
    cl->head = (int64_t *)malloc(sizeof(int64_t) * (size_t)cl->ncell);
    cl->next = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t c = 0; c < cl->ncell; ++c) cl->head[c] = -1;
    for (int64_t i = n - 1; i >= 0; --i) {
        cl->next[i] = cl->head[cl->cell[i]];
        cl->head[cl->cell[i]] = i;
    }
    return 0;
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Partners of particle i within r_list (all j != i, or only j > i when half),
 * ascending, found by scanning the 27 cells around i's cell.  n >= 3 cells per
 * axis makes the 27 cells distinct.  Returns the count; writes at most cap. */
static int64_t scan_partners(const cell_list *cl, const double *q, const double *L, double rl2,
                             int64_t i, int half, int32_t *out, int64_t cap) {
    int32_t c = cl->cell[i];
    int32_t cx = c % cl->n[0], cy = (c / cl->n[0]) % cl->n[1], cz = c / (cl->n[0] * cl->n[1]);
    int64_t cnt = 0;
    for (int oz = -1; oz <= 1; ++oz)
        for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox) {
                int32_t x = (cx + ox + cl->n[0]) % cl->n[0];
                int32_t y = (cy + oy + cl->n[1]) % cl->n[1];
                int32_t z = (cz + oz + cl->n[2]) % cl->n[2];
                int64_t nb = ((int64_t)z * cl->n[1] + y) * cl->n[0] + x;
                for (int64_t j = cl->head[nb]; j >= 0; j = cl->next[j]) {
                    if (j == i || (half && j < i)) continue;
                    if (dist2(q, i, j, L, NULL) < rl2) {
                        if (cnt < cap) out[cnt] = (int32_t)j;
                        ++cnt;
                    }
                }
            }
    if (cnt > 1 && cnt <= cap) qsort(out, (size_t)cnt, sizeof(int32_t), cmp_i32);  /* out may be NULL when cap = 0 */
    return cnt;
}

/* ---------------------------------------------------------------- pair lists */

/* Pair list within r_list = rc + skin, found with the cell grid.  half = 0 gives
 * the full list (every ordered pair), half = 1 the sorted list of Fig. 1 (key =
 * smaller index).  key_ptr[n+1] is written; partners are written when
 * partners != NULL and cap suffices.  Positions are wrapped in place.
 * Returns the total entry count, or a negative orc_cells code. */
int64_t orc_neighbors(int64_t n, double *q, const double *L, double r_list, int half,
                      int64_t *key_ptr, int32_t *partners, int64_t cap) {
    cell_list cl;
    int rc = cells_build(n, q, L, r_list, &cl);
    if (rc != 0) return rc;
    double rl2 = r_list * r_list;
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) cnt[i] = scan_partners(&cl, q, L, rl2, i, half, NULL, 0);
    key_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) key_ptr[i + 1] = key_ptr[i] + cnt[i];
    int64_t total = key_ptr[n];
    if (partners && total <= cap) {
#pragma omp parallel for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i)
            scan_partners(&cl, q, L, rl2, i, half, partners + key_ptr[i], cnt[i]);
    }
    free(cnt);
    cells_free(&cl);
    return total;
}

/* The same set by brute force over all pairs, O(n^2).  No cell grid, no wrap:
 * only the minimum-image distance.  Full list when half = 0. */
int64_t orc_neighbors_brute(int64_t n, const double *q, const double *L, double r_list, int half,
                            int64_t *key_ptr, int32_t *partners, int64_t cap) {
    double rl2 = r_list * r_list;
    int64_t total = 0;
    key_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = half ? i + 1 : 0; j < n; ++j) {
            if (j == i) continue;
            if (dist2(q, i, j, L, NULL) < rl2) {
                if (partners && total < cap) partners[total] = (int32_t)j;
                ++total;
            }
        }
        key_ptr[i + 1] = total;
    }
    return total;
}

/* ---------------------------------------------------------------- forces */

/* Forces, potential energy and per-particle absolute pair-force sums from a
 * full pair list (key_ptr/partners, any superset of the pairs within rc):
 *   F_i = sum_{j in list(i), r_ij < rc} f(r_ij) d_ij,  d_ij = minimum image of q_j - q_i
 *   PE  = sum over pairs i < j with r_ij < rc of V(r_ij)
 *   A_i = sum_{j} |f(r_ij) d_ij|   (normalisation for force-error metrics)
 * pe_i (nullable) receives 1/2 sum_j V(r_ij) per particle.  Returns PE. */
double orc_forces_list_rcp(int64_t n, const double *q, const double *L, double rc, double c2, double c0,
                           const int64_t *key_ptr, const int32_t *partners,
                           double *F, double *A, double *pe_i, int rcp) {
    double rc2 = rc * rc, pe = 0.0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : pe)
    for (int64_t i = 0; i < n; ++i) {
        double fx = 0.0, fy = 0.0, fz = 0.0, a = 0.0, e = 0.0;
        for (int64_t k = key_ptr[i]; k < key_ptr[i + 1]; ++k) {
            int64_t j = partners[k];
            double d[3];
            double r2 = dist2(q, i, j, L, d);
            if (r2 < rc2) {
                double f, v;
                pair_fv(r2, c2, c0, rcp, &f, &v);
                fx += f * d[0]; fy += f * d[1]; fz += f * d[2];
                a += sqrt((f * d[0]) * (f * d[0]) + (f * d[1]) * (f * d[1]) + (f * d[2]) * (f * d[2]));
                e += 0.5 * v;
                if (j > i) pe += v;
            }
        }
        F[3 * i + 0] = fx; F[3 * i + 1] = fy; F[3 * i + 2] = fz;
        if (A) A[i] = a;
        if (pe_i) pe_i[i] = e;
    }
    return pe;
}

double orc_forces_list(int64_t n, const double *q, const double *L, double rc, double c2, double c0,
                       const int64_t *key_ptr, const int32_t *partners,
                       double *F, double *A, double *pe_i) {
    return orc_forces_list_rcp(n, q, L, rc, c2, c0, key_ptr, partners, F, A, pe_i, 0);
}

/* Pair virial sum over a full list: sum_{i<j, r<rc} f(r) r^2, where f = V'(r)/r.
 * The pair contribution to the pressure is W = -sum_{i<j} f r^2 (the force on i
 * from j is f (q_j - q_i), against q_i - q_j), so P = (2 KE + W) / (3 V). */
double orc_virial_list(int64_t n, const double *q, const double *L, double rc, double c2,
                       const int64_t *key_ptr, const int32_t *partners) {
    double rc2 = rc * rc, w = 0.0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : w)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t k = key_ptr[i]; k < key_ptr[i + 1]; ++k) {
            int64_t j = partners[k];
            if (j <= i) continue;
            double d[3];
            double r2 = dist2(q, i, j, L, d);
            if (r2 < rc2) w += orc_pair_f(r2, c2) * r2;
        }
    }
    return w;
}

/* Forces and PE by brute force over all pairs (no list, no cells). */
double orc_forces_brute(int64_t n, const double *q, const double *L, double rc, double c2, double c0,
                        double *F, double *A) {
    double rc2 = rc * rc, pe = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double fx = 0.0, fy = 0.0, fz = 0.0, a = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            double r2 = dist2(q, i, j, L, d);
            if (r2 < rc2) {
                double f = orc_pair_f(r2, c2);
                fx += f * d[0]; fy += f * d[1]; fz += f * d[2];
                a += sqrt((f * d[0]) * (f * d[0]) + (f * d[1]) * (f * d[1]) + (f * d[2]) * (f * d[2]));
                if (j > i) pe += orc_pair_v(r2, c2, c0);
            }
        }
        F[3 * i + 0] = fx; F[3 * i + 1] = fy; F[3 * i + 2] = fz;
        if (A) A[i] = a;
    }
    return pe;
}

/* Forces on a sample of particles only (ids[m]), from a fresh cell grid over
 * all n positions: F, A and 1/2 sum_j V per sampled particle.  For checks at
 * sizes where the full oracle would be slow.  q is wrapped in place. */
int orc_forces_sample(int64_t n, double *q, const double *L, double rc, double c2, double c0,
                      int64_t m, const int64_t *ids, double *F, double *A, double *pe_i) {
    cell_list cl;
    int rcode = cells_build(n, q, L, rc, &cl);
    if (rcode != 0) return rcode;
    double rc2 = rc * rc;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t s = 0; s < m; ++s) {
        int64_t i = ids[s];
        int32_t c = cl.cell[i];
        int32_t cx = c % cl.n[0], cy = (c / cl.n[0]) % cl.n[1], cz = c / (cl.n[0] * cl.n[1]);
        double fx = 0.0, fy = 0.0, fz = 0.0, a = 0.0, e = 0.0;
        for (int oz = -1; oz <= 1; ++oz)
            for (int oy = -1; oy <= 1; ++oy)
                for (int ox = -1; ox <= 1; ++ox) {
                    int32_t x = (cx + ox + cl.n[0]) % cl.n[0];
                    int32_t y = (cy + oy + cl.n[1]) % cl.n[1];
                    int32_t z = (cz + oz + cl.n[2]) % cl.n[2];
                    int64_t nb = ((int64_t)z * cl.n[1] + y) * cl.n[0] + x;
                    for (int64_t j = cl.head[nb]; j >= 0; j = cl.next[j]) {
                        if (j == i) continue;
                        double d[3];
                        double r2 = dist2(q, i, j, L, d);
                        if (r2 < rc2) {
                            double f = orc_pair_f(r2, c2);
                            fx += f * d[0]; fy += f * d[1]; fz += f * d[2];
                            a += sqrt((f * d[0]) * (f * d[0]) + (f * d[1]) * (f * d[1]) +
                                      (f * d[2]) * (f * d[2]));
                            e += 0.5 * orc_pair_v(r2, c2, c0);
                        }
                    }
                }
        F[3 * s + 0] = fx; F[3 * s + 1] = fy; F[3 * s + 2] = fz;
        A[s] = a;
        pe_i[s] = e;
    }
    cells_free(&cl);
    return 0;
}

/* Full-list partners of a sample of particles: for sampled id ids[s], the
 * partners within r_list go to out[s*cap ...] ascending, counts to cnt[s]. */
int orc_neighbors_sample(int64_t n, double *q, const double *L, double r_list, int64_t m,
                         const int64_t *ids, int32_t *out, int64_t cap, int64_t *cnt) {
    cell_list cl;
    int rcode = cells_build(n, q, L, r_list, &cl);
    if (rcode != 0) return rcode;
    double rl2 = r_list * r_list;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t s = 0; s < m; ++s)
        cnt[s] = scan_partners(&cl, q, L, rl2, ids[s], 0, out + s * cap, cap);
    cells_free(&cl);
    return 0;
}

double orc_kinetic(int64_t n, const double *v, double mass) {
    double s = 0.0;
    for (int64_t i = 0; i < 3 * n; ++i) s += v[i] * v[i];
    return 0.5 * mass * s;
}

/* ---------------------------------------------------------------- dynamics */

typedef struct {
    double rc, skin, dt, mass;
    int32_t cutoff;   /* ORC_CUT_* */
    int32_t rebuild;  /* ORC_REBUILD_* */
    int32_t verify;   /* nonzero: count pairs within rc missing from the list, every step */
    int32_t rcp;      /* reciprocal mode of the force evaluation (see pair_fv) */
} orc_params;

typedef struct {
    int64_t steps;
    int64_t rebuilds;
    int64_t missed_pairs;  /* with verify: pairs within rc absent from the list */
    double D;              /* accumulated DUTC bound since the last build */
} orc_stats;

typedef struct {
    int64_t n;
    double L[3];
    double *q, *v, *F;       /* caller arrays, [n][3] */
    double *qb;              /* positions at the last build (unwrapped tracking) */
    int64_t *kp;
    int32_t *pl;
    int64_t cap;
    double c2, c0;
} orc_sys;

static int sys_build(orc_sys *s, const orc_params *p) {
    double rl = p->rc + p->skin;
    for (;;) {
        int64_t tot = orc_neighbors(s->n, s->q, s->L, rl, 0, s->kp, s->pl, s->cap);
        if (tot < 0) return (int)tot;
        if (tot <= s->cap) break;
        free(s->pl);
        s->cap = tot + tot / 4 + 64;
        s->pl = (int32_t *)malloc(sizeof(int32_t) * (size_t)s->cap);
    }
    memcpy(s->qb, s->q, sizeof(double) * 3 * (size_t)s->n);
    return 0;
}

/* Pairs within rc (minimum image) that the current list lacks, by brute force
 * against a fresh cell-grid list at rc on a copy of q. */
static int64_t sys_missed(const orc_sys *s, const orc_params *p) {
    double *qc = (double *)malloc(sizeof(double) * 3 * (size_t)s->n);
    memcpy(qc, s->q, sizeof(double) * 3 * (size_t)s->n);
    int64_t *kp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(s->n + 1));
    int64_t tot = orc_neighbors(s->n, qc, s->L, p->rc, 0, kp, NULL, 0);
    int32_t *pl = (int32_t *)malloc(sizeof(int32_t) * (size_t)(tot > 0 ? tot : 1));
    memcpy(qc, s->q, sizeof(double) * 3 * (size_t)s->n);
    orc_neighbors(s->n, qc, s->L, p->rc, 0, kp, pl, tot);
    int64_t missed = 0;
    for (int64_t i = 0; i < s->n; ++i) {
        /* both lists are ascending: merge-walk */
        int64_t a = s->kp[i], ae = s->kp[i + 1];
        for (int64_t k = kp[i]; k < kp[i + 1]; ++k) {
            while (a < ae && s->pl[a] < pl[k]) ++a;
            if (a >= ae || s->pl[a] != pl[k]) ++missed;
        }
    }
    free(qc); free(kp); free(pl);
    return missed;
}

/* Nose-Hoover thermostat state of a run (used when tau > 0).  The equations
 * dv/dt = F/m - xi v, dxi/dt = (2 KE - g T) / Q, deta/dt = xi, with g = 3N - 3
 * degrees of freedom and Q = g T tau^2, conserve H = KE + PE + Q xi^2 / 2 + g T eta.
 * A step is the symmetric splitting
 *   thermostat(dt/2); velocity Verlet (kick, drift, forces, kick); thermostat(dt/2),
 * where thermostat(h) is: xi += (h/2) G; v *= exp(-xi h); eta += xi h; xi += (h/2) G
 * with G = (2 KE - g T) / Q evaluated from the current velocities. */
typedef struct {
    double T, tau;   /* target temperature and relaxation time; tau <= 0: NVE */
    double xi, eta;  /* thermostat variable and its time integral (in and out) */
} orc_thermo;

static double kin(int64_t n, const double *v, double mass) { return orc_kinetic(n, v, mass); }

static void thermo_half(int64_t n, double *v, double mass, orc_thermo *th, double h) {
    double g = 3.0 * (double)n - 3.0;
    double Q = g * th->T * th->tau * th->tau;
    double G = (2.0 * kin(n, v, mass) - g * th->T) / Q;
    th->xi = th->xi + 0.5 * h * G;
    double sc = exp(-th->xi * h);
    for (int64_t i = 0; i < 3 * n; ++i) v[i] = v[i] * sc;
    th->eta = th->eta + th->xi * h;
    G = (2.0 * kin(n, v, mass) - g * th->T) / Q;
    th->xi = th->xi + 0.5 * h * G;
}

/* Thermostat's share of the conserved quantity: Q xi^2 / 2 + g T eta. */
static double thermo_energy(int64_t n, const orc_thermo *th) {
    double g = 3.0 * (double)n - 3.0;
    double Q = g * th->T * th->tau * th->tau;
    return 0.5 * Q * th->xi * th->xi + g * th->T * th->eta;
}

/* Advance (q, v) by nsteps velocity-Verlet steps.
 *   On entry: q, v at time t (caller order).  If F_valid == 0 the initial list
 *   and forces are built first; otherwise F holds F(q) and D is taken from stats.
 *   Per step: v += (dt/2m) F; q += dt v; DUTC update; rebuild if required;
 *   F = F(q); v += (dt/2m) F  (wrapped in thermostat half steps when th->tau > 0).
 *   energy_every > 0: after every energy_every-th step, KE and PE go to
 *   ke_out[k], pe_out[k] (k counts samples); vir_out[k] (nullable) receives the
 *   pair virial sum_{i<j} f r^2 and th_out[k] (nullable) the thermostat's share
 *   of the conserved quantity.
 * Returns 0 or a negative code.  stats accumulate. */
int orc_run_obs(int64_t n, double *q, double *v, double *F, const double *L, const orc_params *p,
                orc_thermo *th, int64_t nsteps, int64_t energy_every, double *ke_out, double *pe_out,
                double *vir_out, double *th_out, orc_stats *stats, int32_t F_valid) {
    orc_sys s;
    memset(&s, 0, sizeof(s));
    s.n = n; s.q = q; s.v = v; s.F = F;
    memcpy(s.L, L, sizeof(double) * 3);
    orc_coeffs(p->rc, p->cutoff, &s.c2, &s.c0);
    s.qb = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    s.kp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    s.cap = 64 * n + 64;
    s.pl = (int32_t *)malloc(sizeof(int32_t) * (size_t)s.cap);
    int thermo = th && th->tau > 0.0;
    int rcode = sys_build(&s, p);
    if (rcode != 0) goto done;
    if (!F_valid) {
        orc_forces_list_rcp(n, q, s.L, p->rc, s.c2, s.c0, s.kp, s.pl, F, NULL, NULL, p->rcp);
        stats->D = 0.0;
        stats->rebuilds += 1;
    }
    /* a list built from q at entry is only as valid as the caller's D says;
     * rebuilding at entry and resetting D is always safe, and exact forces do
     * not depend on when the list was built. */
    stats->D = 0.0;
    double h = p->dt / (2.0 * p->mass);
    int64_t k = 0;
    for (int64_t step = 1; step <= nsteps; ++step) {
        double vmax2 = 0.0;
        if (thermo) thermo_half(n, v, p->mass, th, 0.5 * p->dt);
        for (int64_t i = 0; i < 3 * n; ++i) v[i] = v[i] + h * F[i];
        for (int64_t i = 0; i < 3 * n; ++i) q[i] = q[i] + p->dt * v[i];
        for (int64_t i = 0; i < n; ++i) {
            double w = v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] + v[3 * i + 2] * v[3 * i + 2];
            if (w > vmax2) vmax2 = w;
        }
        stats->D = stats->D + p->dt * sqrt(vmax2);
        int rebuild = 0;
        if (p->rebuild == ORC_REBUILD_DUTC) {
            rebuild = 2.0 * stats->D > p->skin;
        } else if (p->rebuild == ORC_REBUILD_DISPLACEMENT) {
            double m2 = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                double dx = q[3 * i] - s.qb[3 * i], dy = q[3 * i + 1] - s.qb[3 * i + 1],
                       dz = q[3 * i + 2] - s.qb[3 * i + 2];
                double w = dx * dx + dy * dy + dz * dz;
                if (w > m2) m2 = w;
            }
            rebuild = 2.0 * sqrt(m2) > p->skin;
        } else if (p->rebuild == ORC_REBUILD_EVERY_STEP) {
            rebuild = 1;
        }
        if (rebuild) {
            rcode = sys_build(&s, p);
            if (rcode != 0) goto done;
            stats->D = 0.0;
            stats->rebuilds += 1;
        }
        if (p->verify) stats->missed_pairs += sys_missed(&s, p);
        double pe = orc_forces_list_rcp(n, q, s.L, p->rc, s.c2, s.c0, s.kp, s.pl, F, NULL, NULL, p->rcp);
        for (int64_t i = 0; i < 3 * n; ++i) v[i] = v[i] + h * F[i];
        if (thermo) thermo_half(n, v, p->mass, th, 0.5 * p->dt);
        stats->steps += 1;
        if (energy_every > 0 && step % energy_every == 0) {
            ke_out[k] = orc_kinetic(n, v, p->mass);
            pe_out[k] = pe;
            if (vir_out) vir_out[k] = orc_virial_list(n, q, s.L, p->rc, s.c2, s.kp, s.pl);
            if (th_out) th_out[k] = thermo ? thermo_energy(n, th) : 0.0;
            ++k;
        }
    }
done:
    free(s.qb); free(s.kp); free(s.pl);
    return rcode;
}

int orc_run(int64_t n, double *q, double *v, double *F, const double *L, const orc_params *p,
            int64_t nsteps, int64_t energy_every, double *ke_out, double *pe_out,
            orc_stats *stats, int32_t F_valid) {
    return orc_run_obs(n, q, v, F, L, p, NULL, nsteps, energy_every, ke_out, pe_out, NULL, NULL, stats, F_valid);
}

/* ------------------------------------------------------------------ bubbles
 *
 * Bubble identification of Sec. IV.B.  The box is cut into subcells of edge
 * at least `side` (n_a = floor(L_a / side) per axis, edge L_a / n_a).  Each
 * particle is wrapped into [0, L) and binned with min((int)(x * (n/L)), n-1),
 * the same rule as the cell grid.  A subcell's particle count is kept as one
 * unsigned byte (saturating at 255).  A subcell is gas when that count is below
 * rho_gas times the subcell volume, the volume being (L0/n0)*(L1/n1)*(L2/n2)
 * evaluated left to right.  Gas subcells that share a face, across the
 * periodic boundaries too, belong to one bubble (site percolation on the
 * simple cubic lattice).  Each gas subcell is labelled with the smallest linear
 * index (cz*ny + cy)*nx + cx in its bubble; liquid subcells get -1.
 *
 * Labelling is a flood fill: subcells are visited in increasing index, and an
 * unlabelled gas subcell starts a breadth-first search over its six periodic
 * neighbours, so the seed is the smallest index of the bubble.
 *
 * Returns the number of bubbles, -1 for a bad argument or a position outside
 * [-L, 2L), -3 when out of memory. */
void orc_subcell_grid(const double *L, double side, int32_t *n, double *inv, double *thr, double rho_gas) {
    for (int a = 0; a < 3; ++a) {
        n[a] = (int32_t)floor(L[a] / side);
        inv[a] = (double)n[a] / L[a];
    }
    const double vol = (L[0] / n[0]) * (L[1] / n[1]) * (L[2] / n[2]);
    *thr = rho_gas * vol;
}

int64_t orc_bubbles(int64_t n, const double *q, const double *L, double side, double rho_gas,
                    uint8_t *counts, int32_t *labels) {
    int32_t ns[3];
    double inv[3], thr;
    if (!(side > 0.0) || !(rho_gas >= 0.0)) return -1;
    orc_subcell_grid(L, side, ns, inv, &thr, rho_gas);
    if (ns[0] < 1 || ns[1] < 1 || ns[2] < 1) return -1;
    const int64_t nsub = (int64_t)ns[0] * ns[1] * ns[2];
    int64_t *cnt = (int64_t *)calloc((size_t)nsub, sizeof(int64_t));
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)nsub);
    if (!cnt || !queue) { free(cnt); free(queue); return -3; }
    for (int64_t i = 0; i < n; ++i) {
        int32_t c[3];
        for (int a = 0; a < 3; ++a) {
            double x = q[3 * i + a];
            if (!(x >= -L[a] && x < 2.0 * L[a])) { free(cnt); free(queue); return -1; }
            if (x < 0.0) x += L[a];
            if (x >= L[a]) x -= L[a];
            int32_t k = (int32_t)(x * inv[a]);
            if (k > ns[a] - 1) k = ns[a] - 1;
            c[a] = k;
        }
        cnt[((int64_t)c[2] * ns[1] + c[1]) * ns[0] + c[0]] += 1;
    }
    for (int64_t s = 0; s < nsub; ++s) {
        counts[s] = (uint8_t)(cnt[s] > 255 ? 255 : cnt[s]);
        labels[s] = (double)counts[s] < thr ? -2 : -1; /* -2: gas, not yet labelled */
    }
    int64_t nb = 0;
    for (int64_t seed = 0; seed < nsub; ++seed) {
        if (labels[seed] != -2) continue;
        nb += 1;
        int64_t head = 0, tail = 0;
        labels[seed] = (int32_t)seed;
        queue[tail++] = seed;
        while (head < tail) {
            const int64_t s = queue[head++];
            const int32_t x = (int32_t)(s % ns[0]);
            const int32_t y = (int32_t)((s / ns[0]) % ns[1]);
            const int32_t z = (int32_t)(s / ((int64_t)ns[0] * ns[1]));
            for (int k = 0; k < 6; ++k) {
                int32_t c[3] = {x, y, z};
                const int a = k >> 1;
                c[a] += (k & 1) ? 1 : -1;
                if (c[a] < 0) c[a] += ns[a];
                if (c[a] >= ns[a]) c[a] -= ns[a];
                const int64_t t = ((int64_t)c[2] * ns[1] + c[1]) * ns[0] + c[0];
                if (labels[t] == -2) {
                    labels[t] = (int32_t)seed;
                    queue[tail++] = t;
                }
            }
        }
    }
    free(cnt); free(queue);
    return nb;
}
