/*
 * Plain FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Written from the paper's statement of the method (Methods section: Verlet
 * lists of radius r_v = r_c + r_s rebuilt with a cell algorithm; FP64
 * integration of positions and momenta) and its models (Eq. 1 Lennard-Jones,
 * cut and shifted at r_c; patchy particles, Eqs. 2-4, in the reading given at
 * or_patchy_pair).  Every sum is a straight loop; nothing is blocked, fused or
 * reordered beyond what the definitions state.
 *
 * Build with -O2 -ffp-contract=off so that no multiply-add is fused.  The
 * per-particle loops of the force routines run under OpenMP: every particle's
 * sums are formed by one thread in the same fixed order of j whatever the
 * thread count, so the results are bitwise independent of it.
 */
#include "oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Geometry                                                                    */
/* ------------------------------------------------------------------------- */

double or_min_image(double d, double L) { return d - L * rint(d / L); }

void or_set_threads(int t) { omp_set_num_threads(t > 0 ? t : 1); }

int or_max_threads(void) { return omp_get_max_threads(); }

/* Minimum-image vector from particle i to particle j and its squared length. */
static double sep(const double* x, int i, int j, double L, double d[3]) {
    for (int c = 0; c < 3; c++) d[c] = or_min_image(x[3 * j + c] - x[3 * i + c], L);
    return d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
}

int64_t or_pairs_brute(int n, const double* x, double L, double rv, int32_t* pairs,
                       int64_t cap) {
    double rv2 = rv * rv, d[3];
    int64_t k = 0;
    for (int i = 0; i < n; i++)
        for (int j = i + 1; j < n; j++)
            if (sep(x, i, j, L, d) < rv2) {
                if (k < cap) {
                    pairs[2 * k] = i;
                    pairs[2 * k + 1] = j;
                }
                k++;
            }
    return k;
}

int or_neighbors_of(int i, int n, const double* x, double L, double rv, int32_t* out,
                    int cap) {
    double rv2 = rv * rv, d[3];
    int k = 0;
    for (int j = 0; j < n; j++) {
        if (j == i) continue;
        if (sep(x, i, j, L, d) < rv2) {
            if (k < cap) out[k] = j;
            k++;
        }
    }
    return k;
}

/* A plain cell list: nc cells per side, each of side L/nc >= r.  head/next
 * linked lists, built from scratch on every call. */
typedef struct {
    int nc;
    int* head;
    int* next;
} cells_t;

static int cell_coord(double xc, double L, int nc) {
    double w = xc - L * floor(xc / L); /* into [0, L) */
    int c = (int)floor(w / L * nc);
    if (c >= nc) c = nc - 1;
    if (c < 0) c = 0;
    return c;
}

static int cells_build(cells_t* cl, int n, const double* x, double L, double r) {
    int nc = (int)floor(L / r);
    cl->nc = nc;
    cl->head = NULL;
    cl->next = NULL;
    if (nc < 3) return 0; /* stencil would visit a cell twice: caller uses brute force */
    cl->head = (int*)malloc(sizeof(int) * (size_t)nc * nc * nc);
    cl->next = (int*)malloc(sizeof(int) * (size_t)n);
    for (int c = 0; c < nc * nc * nc; c++) cl->head[c] = -1;
    /* insert in descending order so each cell's chain is ascending in id */
    for (int i = n - 1; i >= 0; i--) {
        int cx = cell_coord(x[3 * i], L, nc), cy = cell_coord(x[3 * i + 1], L, nc),
            cz = cell_coord(x[3 * i + 2], L, nc);
        int c = (cz * nc + cy) * nc + cx;
        cl->next[i] = cl->head[c];
        cl->head[c] = i;
    }
    return 1;
}

static void cells_free(cells_t* cl) {
    free(cl->head);
    free(cl->next);
}

/* Calls visit(j) for every j in the 27 cells around particle i (j may equal i). */
#define FOR_CANDIDATES(cl, x, L, i, j, BODY)                                           \
    do {                                                                               \
        int nc_ = (cl).nc;                                                             \
        int cx_ = cell_coord((x)[3 * (i)], (L), nc_);                                  \
        int cy_ = cell_coord((x)[3 * (i) + 1], (L), nc_);                              \
        int cz_ = cell_coord((x)[3 * (i) + 2], (L), nc_);                              \
        for (int dz_ = -1; dz_ <= 1; dz_++)                                            \
            for (int dy_ = -1; dy_ <= 1; dy_++)                                        \
                for (int dx_ = -1; dx_ <= 1; dx_++) {                                  \
                    int ax_ = (cx_ + dx_ + nc_) % nc_, ay_ = (cy_ + dy_ + nc_) % nc_,  \
                        az_ = (cz_ + dz_ + nc_) % nc_;                                 \
                    for (int j = (cl).head[(az_ * nc_ + ay_) * nc_ + ax_]; j >= 0;     \
                         j = (cl).next[j]) {                                           \
                        BODY                                                           \
                    }                                                                  \
                }                                                                      \
    } while (0)

int64_t or_pairs_cells(int n, const double* x, double L, double rv, int32_t* pairs,
                       int64_t cap) {
    cells_t cl;
    if (!cells_build(&cl, n, x, L, rv)) return or_pairs_brute(n, x, L, rv, pairs, cap);
    double rv2 = rv * rv, d[3];
    int64_t k = 0;
    for (int i = 0; i < n; i++) {
        FOR_CANDIDATES(cl, x, L, i, j, {
            if (j > i && sep(x, i, j, L, d) < rv2) {
                if (k < cap) {
                    pairs[2 * k] = i;
                    pairs[2 * k + 1] = j;
                }
                k++;
            }
        });
    }
    cells_free(&cl);
    return k;
}

double or_pair_margin(int n, const double* x, double L, const double* radii, int nr) {
    double rmax = 0;
    for (int k = 0; k < nr; k++)
        if (radii[k] > rmax) rmax = radii[k];
    double reach = rmax + 1.0, d[3], best = INFINITY;
    cells_t cl;
    int have = cells_build(&cl, n, x, L, reach);
    for (int i = 0; i < n; i++) {
        if (have) {
            FOR_CANDIDATES(cl, x, L, i, j, {
                if (j > i) {
                    double r = sqrt(sep(x, i, j, L, d));
                    if (r < reach)
                        for (int k = 0; k < nr; k++)
                            if (fabs(r - radii[k]) < best) best = fabs(r - radii[k]);
                }
            });
        } else {
            for (int j = i + 1; j < n; j++) {
                double r = sqrt(sep(x, i, j, L, d));
                if (r < reach)
                    for (int k = 0; k < nr; k++)
                        if (fabs(r - radii[k]) < best) best = fabs(r - radii[k]);
            }
        }
    }
    if (have) cells_free(&cl);
    return best;
}

/* ------------------------------------------------------------------------- */
/* Lennard-Jones, cut and shifted at rc (Eq. 1)                                */
/* ------------------------------------------------------------------------- */

/* V(r) = 4 eps [ (sigma/r)^12 - (sigma/r)^6 ] */
static double lj_v(double r2, double eps, double sigma) {
    double s2 = sigma * sigma / r2;
    double s6 = s2 * s2 * s2;
    return 4.0 * eps * (s6 * s6 - s6);
}

double or_lj_pair(double r2, double eps, double sigma, double rc, double* fscal) {
    double s2 = sigma * sigma / r2;
    double s6 = s2 * s2 * s2;
    /* -dV/dr * (1/r) = 24 eps [2 (sigma/r)^12 - (sigma/r)^6] / r^2; the force on
     * j along r_ij = x_j - x_i is this times r_ij. */
    *fscal = 24.0 * eps * (2.0 * s6 * s6 - s6) / r2;
    return lj_v(r2, eps, sigma) - lj_v(rc * rc, eps, sigma);
}

/* Magnitude scale of one pair energy: the sum of the absolute values of its
 * three additive terms, 4 eps (sigma/r)^12, 4 eps (sigma/r)^6 and the shift
 * V(rc).  Rounding errors of any evaluation of V are measured against it. */
static double lj_v_scale(double r2, double eps, double sigma, double rc) {
    double s2 = sigma * sigma / r2;
    double s6 = s2 * s2 * s2;
    return fabs(4.0 * eps * s6 * s6) + fabs(4.0 * eps * s6) + fabs(lj_v(rc * rc, eps, sigma));
}

static void lj_accumulate(const double* x, int i, int j, double L, double eps,
                          double sigma, double rc2, double rc, double* f3, double* e,
                          double* w, double* a3, double* ea) {
    double d[3];
    double r2 = sep(x, i, j, L, d);
    if (r2 < rc2) {
        double fs;
        double v = or_lj_pair(r2, eps, sigma, rc, &fs);
        /* force on i is -fs * r_ij */
        for (int c = 0; c < 3; c++) {
            f3[c] -= fs * d[c];
            a3[c] += fabs(fs * d[c]);
        }
        *e += 0.5 * v;
        *ea += 0.5 * lj_v_scale(r2, eps, sigma, rc);
        *w += 0.5 * fs * r2; /* r_ij . F_j */
    }
}

void or_lj_force_one(int i, int n, const double* x, double L, double eps, double sigma,
                     double rc, double* f3, double* e) {
    double rc2 = rc * rc, w = 0, a3[3] = {0, 0, 0}, ea = 0;
    f3[0] = f3[1] = f3[2] = 0;
    *e = 0;
    for (int j = 0; j < n; j++)
        if (j != i) lj_accumulate(x, i, j, L, eps, sigma, rc2, rc, f3, e, &w, a3, &ea);
}

void or_lj_forces(int n, const double* x, double L, double eps, double sigma, double rc,
                  int use_cells, double* F, double* e, double* w, double* Fabs, double* Eabs) {
    double rc2 = rc * rc;
    cells_t cl;
    int have = use_cells ? cells_build(&cl, n, x, L, rc) : 0;
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < n; i++) {
        double f3[3] = {0, 0, 0}, a3[3] = {0, 0, 0}, ei = 0, wi = 0, ea = 0;
        if (have) {
            FOR_CANDIDATES(cl, x, L, i, j, {
                if (j != i)
                    lj_accumulate(x, i, j, L, eps, sigma, rc2, rc, f3, &ei, &wi, a3, &ea);
            });
        } else {
            for (int j = 0; j < n; j++)
                if (j != i) lj_accumulate(x, i, j, L, eps, sigma, rc2, rc, f3, &ei, &wi, a3, &ea);
        }
        for (int c = 0; c < 3; c++) {
            F[3 * i + c] = f3[c];
            if (Fabs) Fabs[3 * i + c] = a3[c];
        }
        if (e) e[i] = ei;
        if (w) w[i] = wi;
        if (Eabs) Eabs[i] = ea;
    }
    if (have) cells_free(&cl);
}

/* ------------------------------------------------------------------------- */
/* Patchy particles                                                            */
/* ------------------------------------------------------------------------- */
/*
 * Reading used (the paper's Eqs. 2-4 print a core (sigma/r)^200 and a patch
 * term exp[1/2 (r_pp/0.12 sigma)^n] whose sign and exponent did not survive;
 * the workload studied here is the four-patch variant):
 *
 *   V_ij = V_WCA(r) + sum_a sum_b g(s_ab) A(c_i^a) A(c_j^b)        for r < rcut
 *   V_WCA(r) = 4 eps [(sigma/r)^12 - (sigma/r)^6] + eps            for r^2 < 2^(1/3) sigma^2
 *   d_ab = r_ij + delta (u_j^b - u_i^a),  s_ab = |d_ab|,  r_ij = x_j - x_i
 *   g(s)  = -eps_p exp(-s^2 / w^2)                                 for s < rpc
 *   c_i^a =  u_i^a . r_hat,   c_j^b = -u_j^b . r_hat
 *   A(c)  = c^2 for c > 0, else 0
 *   u_i^a = R(q_i) e_a,  e_a in {(1,1,1),(1,-1,-1),(-1,1,-1),(-1,-1,1)}/sqrt(3)
 *
 * Force on j: -dV/dr_ij.  Torque on i: sum_a u_i^a x (-dV/du_i^a), same for j.
 */

static const double PATCH_BODY[4][3] = {
    {1, 1, 1}, {1, -1, -1}, {-1, 1, -1}, {-1, -1, 1}};

void or_quat_to_matrix(const double* q, double* R) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z);
    R[1] = 2 * (x * y - w * z);
    R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);
    R[4] = 1 - 2 * (x * x + z * z);
    R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);
    R[7] = 2 * (y * z + w * x);
    R[8] = 1 - 2 * (x * x + y * y);
}

static void patch_vectors(const double* q, double u[4][3]) {
    double R[9];
    or_quat_to_matrix(q, R);
    double inv = 1.0 / sqrt(3.0);
    for (int a = 0; a < 4; a++)
        for (int r = 0; r < 3; r++)
            u[a][r] = (R[3 * r] * PATCH_BODY[a][0] + R[3 * r + 1] * PATCH_BODY[a][1] +
                       R[3 * r + 2] * PATCH_BODY[a][2]) *
                      inv;
}

static void cross(const double* a, const double* b, double* c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot(const double* a, const double* b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* fmag and timag (optional) accumulate, per component, the magnitudes of the
 * individual terms that make up the force on j and the torque on i (the WCA
 * term, and for every patch pair the Gaussian and the two cosine parts): the
 * scale against which a differently rounded evaluation is judged. */
static double patchy_pair_impl(const double* xi, const double* xj, const double* qi,
                               const double* qj, double L, const or_patchy_params* p, double* Fj,
                               double* ti, double* tj, double* fmag, double* timag) {
    double d[3];
    for (int c = 0; c < 3; c++) {
        d[c] = or_min_image(xj[c] - xi[c], L);
        Fj[c] = ti[c] = tj[c] = 0;
    }
    double r2 = dot(d, d);
    if (!(r2 < p->rcut * p->rcut)) return 0.0;
    double r = sqrt(r2);
    double rhat[3] = {d[0] / r, d[1] / r, d[2] / r};
    double V = 0, dVdr[3] = {0, 0, 0};

    /* WCA core */
    double rwca2 = cbrt(2.0) * p->sigma * p->sigma;
    if (r2 < rwca2) {
        double s2 = p->sigma * p->sigma / r2, s6 = s2 * s2 * s2;
        V += 4.0 * p->eps * (s6 * s6 - s6) + p->eps;
        /* dV/dr_vec = -24 eps [2 s^12 - s^6] / r^2 * r_vec */
        double f = 24.0 * p->eps * (2.0 * s6 * s6 - s6) / r2;
        for (int c = 0; c < 3; c++) {
            dVdr[c] -= f * d[c];
            if (fmag) fmag[c] += fabs(f * d[c]);
        }
    }

    double ui[4][3], uj[4][3];
    patch_vectors(qi, ui);
    patch_vectors(qj, uj);
    double dVdui[4][3], dVduj[4][3];
    memset(dVdui, 0, sizeof dVdui);
    memset(dVduj, 0, sizeof dVduj);
    double w2 = p->w * p->w;

    for (int a = 0; a < 4; a++) {
        double ci = dot(ui[a], rhat);
        if (!(ci > 0)) continue; /* A(c_i) = 0 and A'(c_i) = 0 */
        double Ai = ci * ci;
        for (int b = 0; b < 4; b++) {
            double cj = -dot(uj[b], rhat);
            if (!(cj > 0)) continue;
            double Aj = cj * cj;
            double dab[3];
            for (int c = 0; c < 3; c++) dab[c] = d[c] + p->delta * (uj[b][c] - ui[a][c]);
            double s2 = dot(dab, dab);
            if (p->rpc > 0 && !(s2 < p->rpc * p->rpc)) continue;
            double g = -p->eps_p * exp(-s2 / w2);
            double G = g * Ai * Aj;
            V += G;
            if (fmag && timag) {
                double v1[3], v2[3], t1[3], t2[3];
                for (int c = 0; c < 3; c++) {
                    fmag[c] += fabs(2.0 * G * dab[c] / w2) +
                               fabs(g * Aj * 2.0 * ci * (ui[a][c] - ci * rhat[c]) / r) +
                               fabs(g * Ai * 2.0 * cj * (-uj[b][c] - cj * rhat[c]) / r);
                    v1[c] = 2.0 * p->delta * G * dab[c] / w2;
                    v2[c] = g * Aj * 2.0 * ci * rhat[c];
                }
                cross(ui[a], v1, t1);
                cross(ui[a], v2, t2);
                for (int c = 0; c < 3; c++) timag[c] += fabs(t1[c]) + fabs(t2[c]);
            }
            for (int c = 0; c < 3; c++) {
                /* d/dr of g: g * (-2/w^2) d_ab; of c_i: (u_i - c_i rhat)/r;
                 * of c_j: (-u_j - c_j rhat)/r */
                dVdr[c] += -2.0 * G * dab[c] / w2 +
                           g * Aj * 2.0 * ci * (ui[a][c] - ci * rhat[c]) / r +
                           g * Ai * 2.0 * cj * (-uj[b][c] - cj * rhat[c]) / r;
                /* d/du_i: d_ab depends on -delta u_i, c_i on rhat */
                dVdui[a][c] += 2.0 * p->delta * G * dab[c] / w2 + g * Aj * 2.0 * ci * rhat[c];
                dVduj[b][c] += -2.0 * p->delta * G * dab[c] / w2 - g * Ai * 2.0 * cj * rhat[c];
            }
        }
    }
    for (int c = 0; c < 3; c++) Fj[c] = -dVdr[c];
    for (int a = 0; a < 4; a++) {
        double m[3], t[3];
        for (int c = 0; c < 3; c++) m[c] = -dVdui[a][c];
        cross(ui[a], m, t);
        for (int c = 0; c < 3; c++) ti[c] += t[c];
        for (int c = 0; c < 3; c++) m[c] = -dVduj[a][c];
        cross(uj[a], m, t);
        for (int c = 0; c < 3; c++) tj[c] += t[c];
    }
    return V;
}

/*
 * Two-patch model of the paper's Eqs. 2-4 (M = 2), in the reading used here:
 * the sign of the patch term's exponent is restored so that the attraction
 * decays, its power n is 10, and the two patches sit at the poles of the body
 * z axis, a distance delta from the centre:
 *
 *   V_ij = (sigma / r)^200 - eps_p sum_a sum_b exp(-1/2 (s_ab / w)^10) [s_ab < rpc]
 *   for r < rcut, with d_ab = r_ij + delta (u_j^b - u_i^a), s_ab = |d_ab|,
 *   u^0 = R(q) z_hat, u^1 = -R(q) z_hat.
 *
 * With w = 0.12 sigma and rpc = 0.18 sigma the truncated patch term is
 * eps_p exp(-1/2 1.5^10) = 3.0e-13 eps_p; rcut = 2 delta + rpc covers every
 * patch pair.  dV/dd_ab of a patch pair is 5 eps_p E (s/w)^8 / w^2 d_ab with
 * E = exp(-1/2 (s/w)^10); the core gives dV/dr = -200 (sigma/r)^200 r_ij / r^2.
 */
static double patchy2_pair_impl(const double* xi, const double* xj, const double* qi,
                                const double* qj, double L, const or_patchy_params* p,
                                double* Fj, double* ti, double* tj, double* fmag, double* timag) {
    double d[3];
    for (int c = 0; c < 3; c++) {
        d[c] = or_min_image(xj[c] - xi[c], L);
        Fj[c] = ti[c] = tj[c] = 0;
    }
    double r2 = dot(d, d);
    if (!(r2 < p->rcut * p->rcut)) return 0.0;
    double V = 0, dVdr[3] = {0, 0, 0};

    /* core */
    double vc = pow(p->sigma * p->sigma / r2, 100.0);
    V += vc;
    for (int c = 0; c < 3; c++) {
        double t = -200.0 * vc / r2 * d[c];
        dVdr[c] += t;
        if (fmag) fmag[c] += fabs(t);
    }

    double Ri[9], Rj[9], ui[2][3], uj[2][3];
    or_quat_to_matrix(qi, Ri);
    or_quat_to_matrix(qj, Rj);
    for (int c = 0; c < 3; c++) {
        ui[0][c] = Ri[3 * c + 2];
        ui[1][c] = -Ri[3 * c + 2];
        uj[0][c] = Rj[3 * c + 2];
        uj[1][c] = -Rj[3 * c + 2];
    }
    double dVdui[2][3], dVduj[2][3];
    memset(dVdui, 0, sizeof dVdui);
    memset(dVduj, 0, sizeof dVduj);
    double w2 = p->w * p->w;
    for (int a = 0; a < 2; a++) {
        for (int b = 0; b < 2; b++) {
            double dab[3];
            for (int c = 0; c < 3; c++) dab[c] = d[c] + p->delta * (uj[b][c] - ui[a][c]);
            double s2 = dot(dab, dab);
            if (p->rpc > 0 && !(s2 < p->rpc * p->rpc)) continue;
            double x = s2 / w2;               /* (s/w)^2 */
            double x4 = x * x * x * x;        /* (s/w)^8 */
            double E = exp(-0.5 * x4 * x);    /* exp(-1/2 (s/w)^10) */
            V += -p->eps_p * E;
            double k = 5.0 * p->eps_p * E * x4 / w2;  /* dV/dd_ab = k d_ab */
            for (int c = 0; c < 3; c++) {
                dVdr[c] += k * dab[c];
                dVdui[a][c] += -p->delta * k * dab[c];
                dVduj[b][c] += p->delta * k * dab[c];
            }
            if (fmag && timag) {
                double m[3], t[3];
                for (int c = 0; c < 3; c++) {
                    fmag[c] += fabs(k * dab[c]);
                    m[c] = p->delta * k * dab[c];
                }
                cross(ui[a], m, t);
                for (int c = 0; c < 3; c++) timag[c] += fabs(t[c]);
            }
        }
    }
    for (int c = 0; c < 3; c++) Fj[c] = -dVdr[c];
    for (int a = 0; a < 2; a++) {
        double m[3], t[3];
        for (int c = 0; c < 3; c++) m[c] = -dVdui[a][c];
        cross(ui[a], m, t);
        for (int c = 0; c < 3; c++) ti[c] += t[c];
        for (int c = 0; c < 3; c++) m[c] = -dVduj[a][c];
        cross(uj[a], m, t);
        for (int c = 0; c < 3; c++) tj[c] += t[c];
    }
    return V;
}

double or_patchy_pair(const double* xi, const double* xj, const double* qi,
                      const double* qj, double L, const or_patchy_params* p, double* Fj,
                      double* ti, double* tj) {
    if (p->model == 1) return patchy2_pair_impl(xi, xj, qi, qj, L, p, Fj, ti, tj, NULL, NULL);
    return patchy_pair_impl(xi, xj, qi, qj, L, p, Fj, ti, tj, NULL, NULL);
}

static void patchy_accumulate(const double* x, const double* q, int i, int j, double L,
                              const or_patchy_params* p, double* f3, double* t3,
                              double* e, double* w, double* fa, double* ta) {
    double Fj[3], ti[3], tj[3], d[3];
    double v = p->model == 1
                   ? patchy2_pair_impl(&x[3 * i], &x[3 * j], &q[4 * i], &q[4 * j], L, p, Fj, ti, tj,
                                       fa, ta)
                   : patchy_pair_impl(&x[3 * i], &x[3 * j], &q[4 * i], &q[4 * j], L, p, Fj, ti, tj,
                                      fa, ta);
    for (int c = 0; c < 3; c++) {
        f3[c] -= Fj[c];
        t3[c] += ti[c];
    }
    *e += 0.5 * v;
    sep(x, i, j, L, d);
    *w += 0.5 * dot(d, Fj);
}

void or_patchy_forces(int n, const double* x, const double* q, double L,
                      const or_patchy_params* p, int use_cells, double* F, double* T,
                      double* e, double* w, double* Fabs, double* Tabs) {
    cells_t cl;
    int have = use_cells ? cells_build(&cl, n, x, L, p->rcut) : 0;
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < n; i++) {
        double f3[3] = {0, 0, 0}, t3[3] = {0, 0, 0}, ei = 0, wi = 0;
        double fa[3] = {0, 0, 0}, ta[3] = {0, 0, 0};
        if (have) {
            FOR_CANDIDATES(cl, x, L, i, j, {
                if (j != i) patchy_accumulate(x, q, i, j, L, p, f3, t3, &ei, &wi, fa, ta);
            });
        } else {
            for (int j = 0; j < n; j++)
                if (j != i) patchy_accumulate(x, q, i, j, L, p, f3, t3, &ei, &wi, fa, ta);
        }
        for (int c = 0; c < 3; c++) {
            F[3 * i + c] = f3[c];
            T[3 * i + c] = t3[c];
            if (Fabs) Fabs[3 * i + c] = fa[c];
            if (Tabs) Tabs[3 * i + c] = ta[c];
        }
        if (e) e[i] = ei;
        if (w) w[i] = wi;
    }
    if (have) cells_free(&cl);
}

void or_patchy_pair_scales(int n, const double* x, const double* q, double L,
                           const or_patchy_params* p, int use_cells, double* Fpair,
                           double* Tpair) {
    cells_t cl;
    int have = use_cells ? cells_build(&cl, n, x, L, p->rcut) : 0;
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < n; i++) {
        double fa[3] = {0, 0, 0}, ta[3] = {0, 0, 0};
        double Fj[3], ti[3], tj[3];
        if (have) {
            FOR_CANDIDATES(cl, x, L, i, j, {
                if (j != i) {
                    or_patchy_pair(&x[3 * i], &x[3 * j], &q[4 * i], &q[4 * j], L, p, Fj, ti, tj);
                    for (int c = 0; c < 3; c++) {
                        fa[c] += fabs(Fj[c]); /* |F_i(ij)| = |F_j(ij)| */
                        ta[c] += fabs(ti[c]);
                    }
                }
            });
        } else {
            for (int j = 0; j < n; j++) {
                if (j == i) continue;
                or_patchy_pair(&x[3 * i], &x[3 * j], &q[4 * i], &q[4 * j], L, p, Fj, ti, tj);
                for (int c = 0; c < 3; c++) {
                    fa[c] += fabs(Fj[c]);
                    ta[c] += fabs(ti[c]);
                }
            }
        }
        for (int c = 0; c < 3; c++) {
            Fpair[3 * i + c] = fa[c];
            Tpair[3 * i + c] = ta[c];
        }
    }
    if (have) cells_free(&cl);
}

/* ------------------------------------------------------------------------- */
/* Velocity Verlet                                                             */
/* ------------------------------------------------------------------------- */

static void compute_forces(int n, const double* x, const double* q, double L,
                           const or_run_params* p, double* F, double* T, double* e,
                           double* w) {
    if (p->pot == 0)
        or_lj_forces(n, x, L, p->eps, p->sigma, p->rcut, 1, F, e, w, NULL, NULL);
    else
        or_patchy_forces(n, x, q, L, &p->patchy, 1, F, T, e, w, NULL, NULL);
}

/* Hamilton product a (x) b. */
static void quat_mul(const double* a, const double* b, double* c) {
    c[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    c[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    c[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    c[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

static void energies(int n, const double* v, const double* angmom, const or_run_params* p,
                     const double* e, const double* w, double* out3) {
    double ke = 0, pe = 0, vir = 0;
    for (int i = 0; i < n; i++) {
        ke += 0.5 * p->mass * (v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] +
                               v[3 * i + 2] * v[3 * i + 2]);
        if (p->pot == 1)
            ke += 0.5 *
                  (angmom[3 * i] * angmom[3 * i] + angmom[3 * i + 1] * angmom[3 * i + 1] +
                   angmom[3 * i + 2] * angmom[3 * i + 2]) /
                  p->inertia;
        pe += e[i];
        vir += w[i];
    }
    out3[0] = ke;
    out3[1] = pe;
    out3[2] = vir;
}

int or_run(int n, double* x, double* v, double* q, double* angmom, double L,
           const or_run_params* p, int nsteps, double* en, int32_t* rebuild_steps,
           int rb_cap, double* disp_margin) {
    double* F = (double*)calloc((size_t)3 * n, sizeof(double));
    double* T = (double*)calloc((size_t)3 * n, sizeof(double));
    double* e = (double*)calloc((size_t)n, sizeof(double));
    double* w = (double*)calloc((size_t)n, sizeof(double));
    double* xb = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    double hdt = 0.5 * p->dt;
    int nrb = 0;
    double margin = INFINITY;

    memcpy(xb, x, sizeof(double) * 3 * (size_t)n); /* list built at t = 0 */
    if (rebuild_steps && nrb < rb_cap) rebuild_steps[nrb] = 0;
    nrb++;
    compute_forces(n, x, q, L, p, F, T, e, w);
    if (en) energies(n, v, angmom, p, e, w, en);

    for (int s = 1; s <= nsteps; s++) {
        for (int i = 0; i < n; i++)
            for (int c = 0; c < 3; c++) {
                v[3 * i + c] += hdt * F[3 * i + c] / p->mass;
                if (p->pot == 1) angmom[3 * i + c] += hdt * T[3 * i + c];
            }
        for (int i = 0; i < n; i++) {
            for (int c = 0; c < 3; c++) {
                double y = x[3 * i + c] + p->dt * v[3 * i + c];
                if (y >= L) y -= L;
                if (y < 0) y += L;
                x[3 * i + c] = y;
            }
            if (p->pot == 1) {
                /* free rotation of an isotropic rotor: angle |L|/I dt about L */
                double* Lv = &angmom[3 * i];
                double Ln = sqrt(Lv[0] * Lv[0] + Lv[1] * Lv[1] + Lv[2] * Lv[2]);
                if (Ln > 0) {
                    double th = Ln / p->inertia * p->dt;
                    double sh = sin(0.5 * th), ch = cos(0.5 * th);
                    double rq[4] = {ch, sh * Lv[0] / Ln, sh * Lv[1] / Ln, sh * Lv[2] / Ln};
                    double nq[4];
                    quat_mul(rq, &q[4 * i], nq);
                    double nn = sqrt(nq[0] * nq[0] + nq[1] * nq[1] + nq[2] * nq[2] + nq[3] * nq[3]);
                    for (int k = 0; k < 4; k++) q[4 * i + k] = nq[k] / nn;
                }
            }
        }
        /* Verlet-list rebuild rule: largest displacement since the last build
         * strictly above half the skin */
        double dmax2 = 0;
        for (int i = 0; i < n; i++) {
            double dd = 0;
            for (int c = 0; c < 3; c++) {
                double t = or_min_image(x[3 * i + c] - xb[3 * i + c], L);
                dd += t * t;
            }
            if (dd > dmax2) dmax2 = dd;
        }
        double dmax = sqrt(dmax2);
        if (fabs(dmax - 0.5 * p->skin) < margin) margin = fabs(dmax - 0.5 * p->skin);
        if (dmax > 0.5 * p->skin) {
            memcpy(xb, x, sizeof(double) * 3 * (size_t)n);
            if (rebuild_steps && nrb < rb_cap) rebuild_steps[nrb] = s;
            nrb++;
        }
        compute_forces(n, x, q, L, p, F, T, e, w);
        for (int i = 0; i < n; i++)
            for (int c = 0; c < 3; c++) {
                v[3 * i + c] += hdt * F[3 * i + c] / p->mass;
                if (p->pot == 1) angmom[3 * i + c] += hdt * T[3 * i + c];
            }
        if (en) energies(n, v, angmom, p, e, w, en + 3 * s);
    }
    if (disp_margin) *disp_margin = margin;
    free(F);
    free(T);
    free(e);
    free(w);
    free(xb);
    return nrb;
}

/* ------------------------------------------------------------------------- */
/* Stochastic thermostat                                                       */
/* ------------------------------------------------------------------------- */

/* 64 x 64 -> 128-bit product, high and low words. */
static void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
    unsigned __int128 p = (unsigned __int128)a * b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void or_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    /* multipliers of the S-box and the Weyl increments of the key schedule */
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; r++) {
        if (r > 0) { /* the key advances between rounds */
            k0 += W0;
            k1 += W1;
        }
        uint64_t h0, l0, h1, l1;
        mulhilo64(M0, x0, &h0, &l0);
        mulhilo64(M1, x2, &h1, &l1);
        uint64_t y0 = h1 ^ x1 ^ k0, y1 = l1, y2 = h0 ^ x3 ^ k1, y3 = l0;
        x0 = y0;
        x1 = y1;
        x2 = y2;
        x3 = y3;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

/* uniform on (0, 1) from the top 53 bits */
static double unit53(uint64_t r) { return ((double)(r >> 11) + 0.5) * 0x1.0p-53; }

/* Box-Muller: two standard normals from two words */
static void box_muller(uint64_t a, uint64_t b, double* g0, double* g1) {
    const double two_pi = 6.283185307179586476925286766559;
    double rad = sqrt(-2.0 * log(unit53(a)));
    double ang = two_pi * unit53(b);
    *g0 = rad * cos(ang);
    *g1 = rad * sin(ang);
}

int or_thermostat(int n, double* v, double* angmom, double T, double mass, double inertia,
                  double prob, uint64_t seed, uint64_t counter) {
    int hits = 0;
    const uint64_t key[2] = {seed, 0};
    for (int i = 0; i < n; i++) {
        uint64_t ca[4] = {(uint64_t)i, counter, 0, 0}, cb[4] = {(uint64_t)i, counter, 1, 0};
        uint64_t A[4], B[4];
        or_philox4x64(ca, key, A);
        if (!(unit53(A[0]) < prob)) continue;
        or_philox4x64(cb, key, B);
        double g[6];
        box_muller(A[1], A[2], &g[0], &g[1]);
        box_muller(A[3], B[0], &g[2], &g[3]);
        box_muller(B[1], B[2], &g[4], &g[5]);
        double sv = sqrt(T / mass), sl = sqrt(inertia * T);
        for (int c = 0; c < 3; c++) v[3 * i + c] = sv * g[c];
        if (angmom)
            for (int c = 0; c < 3; c++) angmom[3 * i + c] = sl * g[3 + c];
        hits++;
    }
    return hits;
}
