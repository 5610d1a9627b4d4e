/*
 * Plain FP64 CPU oracle for the short-range pair-force step of molecular
 * dynamics (Rovigatti, Sulc, Reguly, Romano, "A comparison between
 * parallelization approaches in molecular dynamics simulations on GPUs").
 *
 * TEST INFRASTRUCTURE ONLY.  This library is what the GPU engine is checked
 * against; it is loaded by the test-suite, by the smoke check and by the CPU
 * baseline leg of the benchmark, and by nothing else.  It shares no source,
 * header, table or helper with the GPU engine.
 *
 * Everything is FP64, unblocked, and written as the plain definition:
 *   - neighbour set:   all unordered pairs {i,j} with minimum-image distance
 *                      r_ij < r_v = r_c + r_s   (Methods section, Verlet lists)
 *   - LJ force/energy: truncated-and-shifted Lennard-Jones, Eq. (1) and the
 *                      text below it (cut and shifted at r_c)
 *   - patchy:          WCA core plus Gaussian patch-patch attraction with a
 *                      cos^2 angular modulation (four tetrahedral patches);
 *                      the paper's own form is Eqs. (2)-(4), the exact reading
 *                      used here is stated at or_patchy_pair() below
 *   - integrator:      velocity Verlet (rotational velocity Verlet for patchy)
 *                      in FP64, as the Methods section prescribes FP64
 *                      integration of positions and momenta.
 *
 * Arrays are row-major AoS in original particle order: x[3*i+c], q[4*i+k]
 * (Hamilton quaternion w,x,y,z), etc.  No function allocates memory that it
 * returns; all outputs go to caller-owned buffers.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared oracle.c -o liboracle.so -lm
 */
#ifndef MD_ORACLE_H
#define MD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Minimum-image displacement of one component: d - L*rint(d/L). */
double or_min_image(double d, double L);

/* Threads of the OpenMP per-particle loops of the force routines (results do
 * not depend on it), and the current maximum. */
void or_set_threads(int threads);
int or_max_threads(void);

/* Neighbour set (Verlet list contents, Methods section).  Writes the unordered
 * pairs (i<j) with r_ij < rv into pairs[2*k], pairs[2*k+1] for k < cap and
 * returns the total count (which may exceed cap; then only cap are written).
 * or_pairs_brute is the O(N^2) definition; or_pairs_cells enumerates candidates
 * with a cell list of side >= rv and falls back to brute force when fewer than
 * three cells fit per dimension. */
int64_t or_pairs_brute(int n, const double* x, double L, double rv,
                       int32_t* pairs, int64_t cap);
int64_t or_pairs_cells(int n, const double* x, double L, double rv,
                       int32_t* pairs, int64_t cap);

/* Full neighbour list of one particle i by brute force (j ascending).
 * Returns the count; writes at most cap ids. */
int or_neighbors_of(int i, int n, const double* x, double L, double rv,
                    int32_t* out, int cap);

/* Smallest |r_ij - R_k| over all pairs with r_ij < max(R)+1 and over the
 * radii R_0..R_{nr-1}.  Used to reject generated states whose neighbour set
 * would hinge on the last bits of a distance. */
double or_pair_margin(int n, const double* x, double L, const double* radii, int nr);

/* ---- Lennard-Jones, truncated and shifted (Eq. 1) ------------------------ */
/* Pair quantities at squared distance r2 (r2 < rc^2 assumed by the caller):
 * returns V_ts(r) and writes fscal such that the force on j is fscal * r_ij
 * (r_ij = x_j - x_i). */
double or_lj_pair(double r2, double eps, double sigma, double rc, double* fscal);

/* Forces F (3N), per-particle energies e_i = 1/2 sum_j V_ts(r_ij) and
 * per-particle virials w_i = 1/2 sum_j r_ij . F_j(ij), summing over every
 * j != i with r_ij < rc (each pair visited from both ends).  use_cells != 0
 * enumerates candidates with the oracle's own cell list.  Fabs (3N) gets
 * sum_j |F_ij,c|, the scale against which a differently ordered sum is judged;
 * Eabs (N) gets 1/2 sum_j (|4 eps (sigma/r)^12| + |4 eps (sigma/r)^6| + |V(rc)|),
 * the same kind of scale for e_i.  e, w, Fabs and Eabs may be NULL. */
void or_lj_forces(int n, const double* x, double L, double eps, double sigma,
                  double rc, int use_cells, double* F, double* e, double* w,
                  double* Fabs, double* Eabs);

/* Force and energy of one particle by brute force over all j. */
void or_lj_force_one(int i, int n, const double* x, double L, double eps,
                     double sigma, double rc, double* f3, double* e);

/* ---- Patchy particles ------------------------------------------------------ */
typedef struct {
    double eps;        /* WCA core strength                     */
    double sigma;      /* core diameter                         */
    double rcut;       /* centre-centre cut-off                 */
    double eps_p;      /* patch strength                        */
    double w;          /* Gaussian patch width                  */
    double delta;      /* patch distance from the centre        */
    double rpc;        /* patch-patch cut-off (<=0: none)       */
    int model;         /* 0: four patches, WCA core, cosine     */
                       /*    factors; 1: two polar patches,     */
                       /*    (sigma/r)^200 core (see oracle.c)  */
} or_patchy_params;

/* Rotation matrix of a unit Hamilton quaternion q=(w,x,y,z), row-major. */
void or_quat_to_matrix(const double* q, double* R9);

/* One pair: x_i, x_j are positions, qi/qj quaternions.  Returns V_ij and
 * writes the force on j (Fj, the force on i is -Fj), the torque on i (ti) and
 * the torque on j (tj).  Zero beyond rcut. */
double or_patchy_pair(const double* xi, const double* xj, const double* qi,
                      const double* qj, double L, const or_patchy_params* p,
                      double* Fj, double* ti, double* tj);

/* Forces, torques, per-particle energies and virials over all pairs; Fabs and
 * Tabs (optional) get, per component, the sums of the magnitudes of all the
 * terms (WCA, and the Gaussian and two cosine parts of every patch pair) that
 * make up the force and the torque. */
void or_patchy_forces(int n, const double* x, const double* q, double L,
                      const or_patchy_params* p, int use_cells, double* F,
                      double* T, double* e, double* w, double* Fabs, double* Tabs);

/* Per-pair scales of the force tolerance: Fpair (3N) gets
 * sum_j |F_i(ij),c| and Tpair (3N) sum_j |tau_i(ij),c|, the magnitudes of the
 * net pair force and of the pair's torque on i, summed over the pairs of i.
 * A pair whose terms cancel contributes less here than to Fabs / Tabs of
 * or_patchy_forces, which sum the magnitudes of the individual terms. */
void or_patchy_pair_scales(int n, const double* x, const double* q, double L,
                           const or_patchy_params* p, int use_cells, double* Fpair,
                           double* Tpair);

/* ---- Integration ------------------------------------------------------------ */
typedef struct {
    int pot;           /* 0 = LJ, 1 = patchy                     */
    double mass, inertia, dt, skin;
    double eps, sigma, rcut;       /* LJ, and WCA core for patchy */
    or_patchy_params patchy;
} or_run_params;

/* Velocity Verlet (rotational for patchy) over nsteps.  x, v (and q, angmom
 * for patchy) are updated in place.  energies (optional, 3*(nsteps+1)) gets
 * (E_kin, E_pot, virial) at t=0 and after every full step.  rebuild_steps
 * (optional, cap rb_cap) gets every step at which the Verlet list would be
 * rebuilt (step 0 is the initial build); the count is returned.  disp_margin
 * (optional) gets the smallest |max displacement - skin/2| seen. */
int or_run(int n, double* x, double* v, double* q, double* angmom, double L,
           const or_run_params* p, int nsteps, double* energies,
           int32_t* rebuild_steps, int rb_cap, double* disp_margin);

/* ------------------------------------------------------------------------- */
/* Stochastic thermostat                                                       */
/* ------------------------------------------------------------------------- */

/* Philox4x64-10, the counter-based generator of Salmon, Moraes, Dror and Shaw
 * ("Parallel random numbers: as easy as 1, 2, 3", SC 2011): out = the ten
 * keyed rounds applied to the 256-bit counter ctr under the 128-bit key. */
void or_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* One application of the NVT thermostat in the reading of the Methods section
 * (the Brownian scheme it cites: every so many steps, each particle's momenta
 * are redrawn from the Maxwell-Boltzmann distribution at temperature T with
 * probability prob).  Particle i (its index in x, v) draws two Philox blocks,
 * A = philox({i, counter, 0, 0}, {seed, 0}) and B = philox({i, counter, 1, 0},
 * {seed, 0}); u(r) = ((r >> 11) + 1/2) 2^-53.  It is refreshed when
 * u(A0) < prob, with Box-Muller normals g(a, b) = sqrt(-2 ln u(a))
 * (cos 2 pi u(b), sin 2 pi u(b)) taken in the order g(A1, A2), g(A3, B0),
 * g(B1, B2): the first three are v_i sqrt(m / T), the next three (patchy)
 * L_i / sqrt(I T).  angmom may be NULL (LJ).  Returns the number refreshed. */
int or_thermostat(int n, double* v, double* angmom, double T, double mass, double inertia,
                  double prob, uint64_t seed, uint64_t counter);

#ifdef __cplusplus
}
#endif
#endif
