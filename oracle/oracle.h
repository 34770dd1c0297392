/*
 * oracle.h -- plain FP64 CPU reference for the slice-streaming LJ path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or constant with the HIP library: every formula here is written
 * out again from the paper.
 *
 * What it computes (paper, Sec. 4 and Algorithm 1):
 *   - a truncated-and-shifted Lennard-Jones 12-6 fluid, sigma = epsilon = m = 1,
 *     pairs taken when r^2 <= rc^2 (the Algorithm 1 cutoff test is inclusive);
 *   - the velocity-Verlet trajectory of Algorithm 1, written in its synchronous
 *     form {r(t), v(t), F(t)} (see oracle_run);
 *   - the potential energy U and virial W of Algorithm 1, with the energy shift
 *     chosen so that the pair energy vanishes at rc;
 *   - the slice/cell geometry of Sec. 4 (cells of edge >= rc, slices cut
 *     perpendicular to x, neighbours within one cell), generalised to a given
 *     number of x-slices holding an integer number of cell layers.
 *
 * All functions return 0 on success, -1 for invalid arguments, -6 when the
 * trajectory becomes unstable (non-finite values, or an atom crossing more
 * than one slice in one step).
 */
#ifndef LJ_ORACLE_H
#define LJ_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double L[3];      /* box edges */
    double halfL[3];  /* L/2 (minimum-image threshold) */
    double l[3];      /* cell edges */
    double inv_l[3];  /* 1 / cell edges */
    double rc, rc2;   /* cutoff and its square */
    double uc;        /* pair energy at rc, subtracted from every pair */
    int S;            /* x-slices */
    int ncx;          /* cell layers per slice */
    int G[3];         /* cells per axis, G[0] = S * ncx */
    int64_t cells_per_slice;
    int64_t ncell;
} orc_geom;

int oracle_geometry(const double box[3], int slices, double rc, orc_geom *g);

/* Binning of every atom: per-axis cell, slice and global cell id
 * (slice * cells_per_slice + local).  Any output pointer may be NULL. */
void oracle_bin(const orc_geom *g, int64_t n, const double *pos, int32_t *gxyz /* n x 3 */,
                int32_t *slice, int64_t *cell);

/* Single pair (two atoms) -- returns 1 when in range. */
int oracle_pair(const orc_geom *g, const double ri[3], const double rj[3], double f[3],
                double *u, double *w, double *scale, double *r2_out);

/* O(N^2) minimum-image brute force over all i<j pairs. */
int oracle_forces_brute(const orc_geom *g, int64_t n, const double *pos, double *F,
                        double *U, double *W, int64_t *pairs);

/* Cell-list forces.  F, u_half, w_half, scale, cand, inr are per atom (any may be NULL
 * except F).  u_half/w_half are half the sums over the atom's in-range partners. */
int oracle_forces_cells(const orc_geom *g, int64_t n, const double *pos, double *F,
                        double *u_half, double *w_half, double *scale, int64_t *cand,
                        int64_t *inr);

/* Cell-list forces for the atoms in ids[0..m) only (same outputs, indexed by k). */
int oracle_forces_subset(const orc_geom *g, int64_t n, const double *pos, int64_t m,
                         const int64_t *ids, double *F, double *scale, int64_t *cand,
                         int64_t *inr);

/* U, K, W of a state (cell-list forces). */
int oracle_energy(const orc_geom *g, int64_t n, const double *pos, const double *vel,
                  double *U, double *K, double *W);

/* Velocity-Verlet NVE trajectory from {pos, vel} (F(0) computed here).
 *   elog:   [nsamples][4] = t, U, K, W for every t in [0, nsteps] with t % every == 0
 *           (every <= 0: no samples); capacity nsteps/every + 1 rows
 *   miglog: [nsteps][S][2] atoms leaving slice s to the left / right in step t -> t+1
 *           (may be NULL)
 * On return pos, vel, F hold the state at t = nsteps (or at the failing step). */
int oracle_run(const orc_geom *g, int64_t n, double *pos, double *vel, double *F, double dt,
               int64_t nsteps, int64_t every, double *elog, int64_t *nsamples,
               int32_t *miglog, int64_t *steps_done);

/* The same trajectory under the velocity-scaling thermostat of Sec. 4.1 / Sec. 4.2 at
 * temperature T0 > 0: at the start of every step, the velocities v(t) of the atoms of
 * each slice are scaled by lambda_s = sqrt(3 n_s T0 / (2 K_s)) (lambda_s = 1 for a
 * slice without atoms or kinetic energy), slices taken from the positions at t.
 * Energy samples report K of the unscaled v(t). */
int oracle_run_nvt(const orc_geom *g, int64_t n, double *pos, double *vel, double *F, double dt,
                   int64_t nsteps, double T0, int64_t every, double *elog, int64_t *nsamples,
                   int32_t *miglog, int64_t *steps_done);

/* One thermostat scaling of vel in place (slices from pos); lam[S] receives the factors
 * (may be NULL). */
int oracle_slice_scale(const orc_geom *g, int64_t n, const double *pos, double *vel, double T0,
                       double *lam);

void oracle_set_threads(int nthreads);
int oracle_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
