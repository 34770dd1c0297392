/*
 * oracle.c -- plain FP64 CPU reference for the slice-streaming Lennard-Jones path.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  It shares no code
 * with the HIP library.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fopenmp -fPIC -shared (no fast-math),
 * so every product and sum below is one IEEE operation, in the order written.
 *
 * Paper: "Cyclic Data Streaming on GPUs for Short Range Stencils Applied to
 * Molecular Dynamics" (arXiv 2507.11289).
 */
#include "oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_EUNSTABLE (-6)

void oracle_set_threads(int nthreads) { if (nthreads > 0) omp_set_num_threads(nthreads); }
int oracle_get_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------
 * Geometry (Sec. 4, paragraph on the cell grid and the slicing).
 * The paper cuts a cubic box into N_xyz = floor(b/rc) cells per edge, cell edge
 * l = b/N_xyz, and uses one cell layer per slice.  Here the number of x-slices is
 * given; each slice holds ncx = floor((Lx/S)/rc) cell layers, so slice and cell
 * boundaries coincide.  The paper asks for l > rc while floor() only gives
 * l >= rc: when an edge is within a relative 2^-40 of rc, the count drops by one.
 * ------------------------------------------------------------------------ */
int oracle_geometry(const double box[3], int slices, double rc, orc_geom *g)
{
    const double margin = 1.0 + ldexp(1.0, -40);
    if (!g || !box) return ORC_EINVAL;
    memset(g, 0, sizeof(*g));
    if (!(rc > 0.0) || !isfinite(rc) || slices < 3) return ORC_EINVAL;
    for (int d = 0; d < 3; d++)
        if (!(box[d] > 0.0) || !isfinite(box[d])) return ORC_EINVAL;
    if (box[0] / slices < rc) return ORC_EINVAL;

    int ncx = (int)floor((box[0] / slices) / rc);
    if (box[0] / (double)(slices * ncx) < rc * margin) ncx -= 1;
    int gy = (int)floor(box[1] / rc);
    if (box[1] / (double)gy < rc * margin) gy -= 1;
    int gz = (int)floor(box[2] / rc);
    if (box[2] / (double)gz < rc * margin) gz -= 1;
    if (ncx < 1 || gy < 3 || gz < 3) return ORC_EINVAL;

    g->S = slices;
    g->ncx = ncx;
    g->G[0] = slices * ncx;
    g->G[1] = gy;
    g->G[2] = gz;
    for (int d = 0; d < 3; d++) {
        g->L[d] = box[d];
        g->halfL[d] = 0.5 * box[d];
        g->l[d] = box[d] / (double)g->G[d];
        g->inv_l[d] = 1.0 / g->l[d];
    }
    g->rc = rc;
    g->rc2 = rc * rc;
    /* energy shift: the pair energy 4(r^-12 - r^-6) evaluated at rc */
    double ir2c = 1.0 / g->rc2;
    double ir6c = ir2c * ir2c * ir2c;
    g->uc = 4.0 * ir6c * (ir6c - 1.0);
    g->cells_per_slice = (int64_t)ncx * gy * gz;
    g->ncell = g->cells_per_slice * slices;
    return 0;
}

/* Cell coordinate along one axis: floor(x * (1/l)), one IEEE multiply, clamped to
 * [0, G-1] (a coordinate equal to L after wrapping lands in the last cell). */
static int cell_coord(double x, double inv_l, int G)
{
    double f = floor(x * inv_l);
    if (!(f >= 0.0)) return 0;
    if (f > (double)(G - 1)) return G - 1;
    return (int)f;
}

static int64_t cell_id(const orc_geom *g, int cx, int cy, int cz)
{
    int s = cx / g->ncx;
    int64_t local = ((int64_t)(cx % g->ncx) * g->G[1] + cy) * g->G[2] + cz;
    return (int64_t)s * g->cells_per_slice + local;
}

void oracle_bin(const orc_geom *g, int64_t n, const double *pos, int32_t *gxyz,
                int32_t *slice, int64_t *cell)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        int c[3];
        for (int d = 0; d < 3; d++) c[d] = cell_coord(pos[3 * i + d], g->inv_l[d], g->G[d]);
        if (gxyz) { gxyz[3 * i] = c[0]; gxyz[3 * i + 1] = c[1]; gxyz[3 * i + 2] = c[2]; }
        if (slice) slice[i] = c[0] / g->ncx;
        if (cell) cell[i] = cell_id(g, c[0], c[1], c[2]);
    }
}

/* ------------------------------------------------------------------------
 * One pair (Algorithm 1, body of the neighbour loop).
 *   r_ij = r_i - r_j under the minimum-image convention (periodic box, L >= 3 rc,
 *   so the image within rc is unique);
 *   in range iff r_ij . r_ij <= rc^2;
 *   F_abs = 24 (2 r^-12 - r^-6) / r^2, force on i = F_abs * r_ij;
 *   pair energy 4 (r^-12 - r^-6) minus its value at rc;
 *   pair virial r_ij . f_ij = 24 (2 r^-12 - r^-6).
 * scale = 24 (2 r^-13 + r^-7): the sum of the magnitudes of the two terms of the
 * pair force, used to normalise force errors.
 * ------------------------------------------------------------------------ */
static double min_image(double d, double L, double halfL)
{
    if (d > halfL) return d - L;
    if (d < -halfL) return d + L;
    return d;
}

int oracle_pair(const orc_geom *g, const double ri[3], const double rj[3], double f[3],
                double *u, double *w, double *scale, double *r2_out)
{
    double dx = min_image(ri[0] - rj[0], g->L[0], g->halfL[0]);
    double dy = min_image(ri[1] - rj[1], g->L[1], g->halfL[1]);
    double dz = min_image(ri[2] - rj[2], g->L[2], g->halfL[2]);
    double r2 = (dx * dx + dy * dy) + dz * dz;
    if (r2_out) *r2_out = r2;
    if (!(r2 <= g->rc2)) {
        f[0] = f[1] = f[2] = 0.0;
        if (u) *u = 0.0;
        if (w) *w = 0.0;
        if (scale) *scale = 0.0;
        return 0;
    }
    double ir2 = 1.0 / r2;
    double ir6 = ir2 * ir2 * ir2;
    double t = 2.0 * ir6 - 1.0;
    double fr = 24.0 * ir2 * ir6 * t;
    f[0] = fr * dx;
    f[1] = fr * dy;
    f[2] = fr * dz;
    if (u) *u = 4.0 * ir6 * (ir6 - 1.0) - g->uc;
    if (w) *w = 24.0 * ir6 * t;
    if (scale) *scale = 24.0 * ir6 * (2.0 * ir6 + 1.0) / sqrt(r2);
    return 1;
}

/* ------------------------------------------------------------------------
 * Brute force: the plain definition -- every pair i<j, minimum image.
 * ------------------------------------------------------------------------ */
int oracle_forces_brute(const orc_geom *g, int64_t n, const double *pos, double *F,
                        double *U, double *W, int64_t *pairs)
{
    if (!g || n < 0 || (n > 0 && (!pos || !F))) return ORC_EINVAL;
    memset(F, 0, sizeof(double) * 3 * (size_t)n);
    double usum = 0.0, wsum = 0.0;
    int64_t np = 0;
    for (int64_t i = 0; i < n; i++) {
        for (int64_t j = i + 1; j < n; j++) {
            double f[3], u, w;
            if (oracle_pair(g, pos + 3 * i, pos + 3 * j, f, &u, &w, NULL, NULL)) {
                for (int d = 0; d < 3; d++) {
                    F[3 * i + d] += f[d];
                    F[3 * j + d] -= f[d];
                }
                usum += u;
                wsum += w;
                np++;
            }
        }
    }
    if (U) *U = usum;
    if (W) *W = wsum;
    if (pairs) *pairs = np;
    return 0;
}

/* ------------------------------------------------------------------------
 * Cell list (Sec. 4: neighbours of a molecule lie in its own cell and the
 * adjacent ones because the cell edge exceeds rc).  Cells are filled by a
 * stable counting sort, so each cell lists its atoms in id order.
 * ------------------------------------------------------------------------ */
typedef struct {
    int64_t *start; /* ncell + 1 */
    int64_t *order; /* n atom ids, cell by cell */
    int32_t *gxyz;  /* n x 3 */
} cell_list;

static void cells_free(cell_list *cl)
{
    free(cl->start);
    free(cl->order);
    free(cl->gxyz);
    memset(cl, 0, sizeof(*cl));
}

static int cells_build(const orc_geom *g, int64_t n, const double *pos, cell_list *cl)
{
    memset(cl, 0, sizeof(*cl));
    int64_t *cell = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    cl->start = calloc((size_t)g->ncell + 1, sizeof(int64_t));
    cl->order = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    cl->gxyz = malloc(sizeof(int32_t) * 3 * (size_t)(n > 0 ? n : 1));
    if (!cell || !cl->start || !cl->order || !cl->gxyz) {
        free(cell);
        cells_free(cl);
        return ORC_ENOMEM;
    }
    oracle_bin(g, n, pos, cl->gxyz, NULL, cell);
    for (int64_t i = 0; i < n; i++) cl->start[cell[i] + 1]++;
    for (int64_t c = 0; c < g->ncell; c++) cl->start[c + 1] += cl->start[c];
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)g->ncell);
    if (!fill) {
        free(cell);
        cells_free(cl);
        return ORC_ENOMEM;
    }
    memcpy(fill, cl->start, sizeof(int64_t) * (size_t)g->ncell);
    for (int64_t i = 0; i < n; i++) cl->order[fill[cell[i]]++] = i;
    free(fill);
    free(cell);
    return 0;
}

/* Sum over the 27 cells around atom i (periodic in all three axes). */
static void atom_forces(const orc_geom *g, const cell_list *cl, const double *pos, int64_t i,
                        double Fi[3], double *uh, double *wh, double *sc, int64_t *cand,
                        int64_t *inr)
{
    const int *G = g->G;
    int cx = cl->gxyz[3 * i], cy = cl->gxyz[3 * i + 1], cz = cl->gxyz[3 * i + 2];
    double f0 = 0.0, f1 = 0.0, f2 = 0.0, us = 0.0, ws = 0.0, ss = 0.0;
    int64_t nc = 0, np = 0;
    for (int ox = -1; ox <= 1; ox++) {
        int nx = (cx + ox + G[0]) % G[0];
        for (int oy = -1; oy <= 1; oy++) {
            int ny = (cy + oy + G[1]) % G[1];
            for (int oz = -1; oz <= 1; oz++) {
                int nz = (cz + oz + G[2]) % G[2];
                int64_t c = cell_id(g, nx, ny, nz);
                for (int64_t k = cl->start[c]; k < cl->start[c + 1]; k++) {
                    int64_t j = cl->order[k];
                    if (j == i) continue;
                    nc++;
                    double f[3], u, w, s;
                    if (oracle_pair(g, pos + 3 * i, pos + 3 * j, f, &u, &w, &s, NULL)) {
                        f0 += f[0];
                        f1 += f[1];
                        f2 += f[2];
                        us += u;
                        ws += w;
                        ss += s;
                        np++;
                    }
                }
            }
        }
    }
    Fi[0] = f0;
    Fi[1] = f1;
    Fi[2] = f2;
    if (uh) *uh = 0.5 * us;
    if (wh) *wh = 0.5 * ws;
    if (sc) *sc = ss;
    if (cand) *cand = nc;
    if (inr) *inr = np;
}

int oracle_forces_cells(const orc_geom *g, int64_t n, const double *pos, double *F,
                        double *u_half, double *w_half, double *scale, int64_t *cand,
                        int64_t *inr)
{
    if (!g || n < 0 || (n > 0 && (!pos || !F))) return ORC_EINVAL;
    cell_list cl;
    int rc = cells_build(g, n, pos, &cl);
    if (rc) return rc;
#pragma omp parallel for schedule(dynamic, 512)
    for (int64_t i = 0; i < n; i++) {
        double uh, wh, sc;
        int64_t nc, np;
        atom_forces(g, &cl, pos, i, F + 3 * i, &uh, &wh, &sc, &nc, &np);
        if (u_half) u_half[i] = uh;
        if (w_half) w_half[i] = wh;
        if (scale) scale[i] = sc;
        if (cand) cand[i] = nc;
        if (inr) inr[i] = np;
    }
    cells_free(&cl);
    return 0;
}

int oracle_forces_subset(const orc_geom *g, int64_t n, const double *pos, int64_t m,
                         const int64_t *ids, double *F, double *scale, int64_t *cand,
                         int64_t *inr)
{
    if (!g || n < 0 || m < 0 || (m > 0 && (!ids || !F || !pos))) return ORC_EINVAL;
    for (int64_t k = 0; k < m; k++)
        if (ids[k] < 0 || ids[k] >= n) return ORC_EINVAL;
    cell_list cl;
    int rc = cells_build(g, n, pos, &cl);
    if (rc) return rc;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t k = 0; k < m; k++) {
        double sc;
        int64_t nc, np;
        atom_forces(g, &cl, pos, ids[k], F + 3 * k, NULL, NULL, &sc, &nc, &np);
        if (scale) scale[k] = sc;
        if (cand) cand[k] = nc;
        if (inr) inr[k] = np;
    }
    cells_free(&cl);
    return 0;
}

static double kinetic(int64_t n, const double *vel)
{
    double k = 0.0;
    for (int64_t i = 0; i < n; i++) {
        const double *v = vel + 3 * i;
        k += 0.5 * ((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
    }
    return k;
}

static void sum_halves(int64_t n, const double *uh, const double *wh, double *U, double *W)
{
    double us = 0.0, ws = 0.0;
    for (int64_t i = 0; i < n; i++) {
        us += uh[i];
        ws += wh[i];
    }
    *U = us;
    *W = ws;
}

int oracle_energy(const orc_geom *g, int64_t n, const double *pos, const double *vel,
                  double *U, double *K, double *W)
{
    if (!g || n < 0) return ORC_EINVAL;
    size_t nn = (size_t)(n > 0 ? n : 1);
    double *F = malloc(sizeof(double) * 3 * nn), *uh = malloc(sizeof(double) * nn),
           *wh = malloc(sizeof(double) * nn);
    if (!F || !uh || !wh) {
        free(F); free(uh); free(wh);
        return ORC_ENOMEM;
    }
    int rc = oracle_forces_cells(g, n, pos, F, uh, wh, NULL, NULL, NULL);
    if (!rc) {
        double u, w;
        sum_halves(n, uh, wh, &u, &w);
        if (U) *U = u;
        if (W) *W = w;
        if (K) *K = kinetic(n, vel);
    }
    free(F); free(uh); free(wh);
    return rc;
}

/* ------------------------------------------------------------------------
 * Velocity-Verlet (Algorithm 1).  Algorithm 1 keeps {r(t), v(t - dt), F(t - dt)}
 * and does: compute F(t); v(t) = v(t-dt) + (F(t) + F(t-dt)) dt/2;
 * r(t+dt) = r(t) + v(t) dt + F(t) dt^2/2.  The same trajectory written on the
 * synchronous state {r(t), v(t), F(t)}, with F(0) computed from the initial
 * positions, is one step:
 *     v_half = v + (dt/2) F          (half kick)
 *     r      = r + dt v_half         (drift), wrapped into the box
 *     F      = F(r)                  (forces at the new positions)
 *     v      = v_half + (dt/2) F     (half kick)
 * The step in which the new x-coordinate falls into another slice is a migration
 * to the left or right neighbour (Sec. 4: a propagating molecule lands in the same,
 * the left or the right slice); any larger slice change is an error.
 * ------------------------------------------------------------------------ */
static double wrap1(double x, double L)
{
    if (x >= L) return x - L;
    if (x < 0.0) return x + L;
    return x;
}

/* ------------------------------------------------------------------------
 * Velocity-scaling thermostat (Sec. 4: a scale factor for the velocities is computed
 * from the new velocities and applied before the positions are advanced; Sec. 4.2 runs
 * the canonical ensemble with it).  The factor belongs to one slice -- the unit of
 * work the kernels of Sec. 4 process -- and brings that slice's kinetic temperature to
 * the target:  T_s = 2 K_s / (3 n_s),  lambda_s = sqrt(T0 / T_s)
 *                                              = sqrt(3 n_s T0 / (2 K_s)),
 * with K_s = sum over the slice's atoms of |v(t)|^2 / 2 (unit mass, k_B = 1).  A slice
 * without atoms or without motion keeps its velocities (lambda = 1).  On the
 * synchronous state the scaling is the first operation of a step, applied to v(t)
 * of the atoms by the slice that holds them at time t.
 * ------------------------------------------------------------------------ */
static void thermostat_slices(const orc_geom *g, int64_t n, double *vel, const int32_t *slice, double T0,
                              double *Ks, int64_t *ns, double *lam)
{
    for (int s = 0; s < g->S; s++) { Ks[s] = 0.0; ns[s] = 0; }
    for (int64_t i = 0; i < n; i++) {
        const double *v = vel + 3 * i;
        Ks[slice[i]] += 0.5 * ((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
        ns[slice[i]]++;
    }
    for (int s = 0; s < g->S; s++)
        lam[s] = (ns[s] > 0 && Ks[s] > 0.0) ? sqrt((3.0 * (double)ns[s] * T0) / (2.0 * Ks[s])) : 1.0;
    for (int64_t i = 0; i < n; i++)
        for (int d = 0; d < 3; d++) vel[3 * i + d] *= lam[slice[i]];
}

static int run_impl(const orc_geom *g, int64_t n, double *pos, double *vel, double *F, double dt,
                    int64_t nsteps, double T0, int64_t every, double *elog, int64_t *nsamples,
                    int32_t *miglog, int64_t *steps_done)
{
    if (!g || n < 0 || nsteps < 0 || !(dt > 0.0) || (n > 0 && (!pos || !vel || !F)) || !(T0 >= 0.0) ||
        !isfinite(T0))
        return ORC_EINVAL;
    size_t nn = (size_t)(n > 0 ? n : 1);
    double *uh = malloc(sizeof(double) * nn), *wh = malloc(sizeof(double) * nn);
    int32_t *s_old = malloc(sizeof(int32_t) * nn), *s_new = malloc(sizeof(int32_t) * nn);
    double *Ks = malloc(sizeof(double) * (size_t)g->S), *lam = malloc(sizeof(double) * (size_t)g->S);
    int64_t *ns_ = malloc(sizeof(int64_t) * (size_t)g->S);
    if (!uh || !wh || !s_old || !s_new || !Ks || !lam || !ns_) {
        free(uh); free(wh); free(s_old); free(s_new); free(Ks); free(lam); free(ns_);
        return ORC_ENOMEM;
    }
    const double hdt = 0.5 * dt;
    int64_t ns = 0, done = 0;
    int status = oracle_forces_cells(g, n, pos, F, uh, wh, NULL, NULL, NULL);
    if (!status && every > 0 && elog) {
        double U, W;
        sum_halves(n, uh, wh, &U, &W);
        elog[0] = 0.0; elog[1] = U; elog[2] = kinetic(n, vel); elog[3] = W;
        ns = 1;
    }
    for (int64_t step = 0; step < nsteps && !status; step++) {
        oracle_bin(g, n, pos, NULL, s_old, NULL);
        if (T0 > 0.0) thermostat_slices(g, n, vel, s_old, T0, Ks, ns_, lam);
        int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
        for (int64_t i = 0; i < n; i++) {
            for (int d = 0; d < 3; d++) {
                double vh = vel[3 * i + d] + hdt * F[3 * i + d];
                double x = pos[3 * i + d] + dt * vh;
                x = wrap1(x, g->L[d]);
                vel[3 * i + d] = vh;
                pos[3 * i + d] = x;
                if (!isfinite(x) || !isfinite(vh) || x < 0.0 || x > g->L[d]) bad = 1;
            }
        }
        if (bad) { status = ORC_EUNSTABLE; break; }
        oracle_bin(g, n, pos, NULL, s_new, NULL);
        if (miglog) memset(miglog + (size_t)step * g->S * 2, 0, sizeof(int32_t) * 2 * g->S);
        for (int64_t i = 0; i < n; i++) {
            int delta = ((s_new[i] - s_old[i]) % g->S + g->S) % g->S;
            if (delta == 0) continue;
            if (delta == 1) {
                if (miglog) miglog[((size_t)step * g->S + s_old[i]) * 2 + 1]++;
            } else if (delta == g->S - 1) {
                if (miglog) miglog[((size_t)step * g->S + s_old[i]) * 2 + 0]++;
            } else {
                bad = 1;
            }
        }
        if (bad) { status = ORC_EUNSTABLE; break; }
        status = oracle_forces_cells(g, n, pos, F, uh, wh, NULL, NULL, NULL);
        if (status) break;
#pragma omp parallel for schedule(static) reduction(| : bad)
        for (int64_t i = 0; i < n; i++) {
            for (int d = 0; d < 3; d++) {
                double v = vel[3 * i + d] + hdt * F[3 * i + d];
                vel[3 * i + d] = v;
                if (!isfinite(v) || !isfinite(F[3 * i + d])) bad = 1;
            }
        }
        if (bad) { status = ORC_EUNSTABLE; break; }
        done = step + 1;
        if (every > 0 && elog && done % every == 0) {
            double U, W;
            sum_halves(n, uh, wh, &U, &W);
            double *row = elog + 4 * ns;
            row[0] = (double)done; row[1] = U; row[2] = kinetic(n, vel); row[3] = W;
            ns++;
        }
    }
    if (nsamples) *nsamples = ns;
    if (steps_done) *steps_done = done;
    free(uh); free(wh); free(s_old); free(s_new); free(Ks); free(lam); free(ns_);
    return status;
}

int oracle_run(const orc_geom *g, int64_t n, double *pos, double *vel, double *F, double dt,
               int64_t nsteps, int64_t every, double *elog, int64_t *nsamples,
               int32_t *miglog, int64_t *steps_done)
{
    return run_impl(g, n, pos, vel, F, dt, nsteps, 0.0, every, elog, nsamples, miglog, steps_done);
}

int oracle_run_nvt(const orc_geom *g, int64_t n, double *pos, double *vel, double *F, double dt,
                   int64_t nsteps, double T0, int64_t every, double *elog, int64_t *nsamples,
                   int32_t *miglog, int64_t *steps_done)
{
    if (!(T0 > 0.0)) return ORC_EINVAL;
    return run_impl(g, n, pos, vel, F, dt, nsteps, T0, every, elog, nsamples, miglog, steps_done);
}

int oracle_slice_scale(const orc_geom *g, int64_t n, const double *pos, double *vel, double T0,
                       double *lam)
{
    if (!g || n < 0 || (n > 0 && (!pos || !vel)) || !(T0 > 0.0) || !isfinite(T0)) return ORC_EINVAL;
    size_t nn = (size_t)(n > 0 ? n : 1);
    int32_t *sl = malloc(sizeof(int32_t) * nn);
    double *Ks = malloc(sizeof(double) * (size_t)g->S), *lm = malloc(sizeof(double) * (size_t)g->S);
    int64_t *ns_ = malloc(sizeof(int64_t) * (size_t)g->S);
    if (!sl || !Ks || !lm || !ns_) {
        free(sl); free(Ks); free(lm); free(ns_);
        return ORC_ENOMEM;
    }
    oracle_bin(g, n, pos, NULL, sl, NULL);
    thermostat_slices(g, n, vel, sl, T0, Ks, ns_, lm);
    if (lam) memcpy(lam, lm, sizeof(double) * (size_t)g->S);
    free(sl); free(Ks); free(lm); free(ns_);
    return 0;
}
