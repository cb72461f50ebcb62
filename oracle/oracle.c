/*
 * FP64 brute-force CPU oracle of the clumped-sphere DEM timestep.
 * TEST INFRASTRUCTURE ONLY -- see oracle.h.  Built with -ffp-contract=off and
 * without -ffast-math so that every +, -, *, / and sqrt is a single IEEE-754
 * double operation evaluated in the order written.
 *
 * One step, state S_n -> S_{n+1} (paper Sec. 2.1, with the readings listed
 * where the paper leaves a choice open):
 *   1. per clump, the rotation matrix A(q) and the world angular velocity
 *      A w_body;
 *   2. sphere centres x_s = x_c + A o_s (multi-sphere clump, Sec. 2.1);
 *   3. the contact set by brute force: every pair a < b of spheres of
 *      different clumps in the same scene with d^2 < (Ra+Rb)^2 (strict), and
 *      every sphere / boundary pair with signed distance phi < R; a triangle
 *      of a mesh is a boundary whose distance is that to its closest point;
 *   4. per contact: normal n from a to b, penetration delta, contact point at
 *      the middle of the overlap, lever arms from each clump's CoM, relative
 *      velocity split into normal and tangential parts (Eq. kinematicsContactInfo);
 *   5. the Hertz-Mindlin law (Eq. normal_tangential_force_model1/2) with
 *      stiffness and damping derived from E, nu and CoR: E* and G* from the two
 *      materials, damping ratio beta(CoR), f = sqrt(Rbar delta);
 *      tangential history update and projection (Eq. updateUt), Coulomb cap on
 *      the trial tangential force with the history clamped so the spring part
 *      equals the cap (Eq. cappingOfut, with k_t taken as the contact's
 *      tangential stiffness f*k_t);
 *   6. per sphere: the sum of its contact forces and torques r x F (r from the
 *      clump CoM to the contact point, normal and tangential parts both), in
 *      ascending partner id (spheres, then boundaries); per clump: the sum over
 *      its spheres in ascending id, then + M g (Eq. newton_law_1/2);
 *   7. symplectic Euler: v += h F/M, x += h v; body-frame Euler equations with
 *      the gyroscopic term; q += (h/2) q (x) (0, w_body), renormalised;
 *   8. meshes follow their prescribed velocities: x += h v,
 *      q += (h/2) (0, w) (x) q (world-frame w), renormalised.
 *
 * Fixed-point positions (pos_exp = E > 0; a state representation beyond
 * IEEE double, Sec. 3 and the data types Sec. 1 builds on): a clump's CoM is
 * an integer k per axis, x = k 2^-E.  The vector between two spheres of
 * different clumps is (k_b - k_a) 2^-E, exact, plus the difference of their
 * rotated offsets A o; a lever arm from a CoM is the sphere's rotated offset
 * plus its part of the contact normal, never a difference of world
 * coordinates; and step 7 adds the position increment rounded to the grid,
 * k += rint(h v 2^E).  Distances to boundaries and meshes stay in FP64 world
 * coordinates (x = k 2^-E converted to double).
 */
#include "oracle.h"

#include <math.h>
#include <omp.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define NPARAM_BND 12
#define NPARAM_PRESC 12

static char g_err[256];
static void set_err(const char *m) { snprintf(g_err, sizeof g_err, "%s", m); }
const char *dem_oracle_last_error(void) { return g_err; }
void dem_oracle_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }

struct dem_oracle {
    double h;
    int64_t step;
    int64_t nc, ns;
    int32_t nsc, nb;
    /* clump state and static data (x: the CoM in FP64; with fixed-point
     * positions its decoded value, the state being xq) */
    double *x, *q, *v, *w;
    int32_t pos_exp;        /* 0, or E of the fixed-point positions x = xq 2^-E */
    double eps;             /* 2^-E */
    int64_t *xq;            /* [nc][3] fixed-point CoM */
    double *xr;             /* [ns][3] rotated sphere offsets A o_s (this step) */
    int bad_pos;            /* a fixed-point position left its range */
    double *mass, *inertia; /* per clump */
    uint32_t *scene;        /* per clump */
    int64_t *sbeg;          /* [nc+1] sphere range per clump */
    int32_t *presc;         /* per clump: -1 or index into presc_param */
    double *presc_param;
    /* sphere static data */
    uint32_t *owner;
    double *ofs;            /* [ns][3] body offsets */
    double *rad;
    double *me, *mg, *mmu, *mbeta; /* (1-nu^2)/E, 2(2-nu)(1+nu)/E, mu, beta(CoR) */
    /* boundaries: nb analytic primitives, then ntri mesh triangles (nw in all) */
    int32_t nw;
    int32_t *btype, *bscene;
    double *bparam, *bvel, *bomega;
    double *be, *bg, *bmu, *bbeta;   /* [nw] */
    /* meshes */
    int32_t nm;
    int64_t ntri;
    double *mx, *mq, *mv, *mw;       /* per mesh: reference point, orientation, velocity, world angular velocity */
    int32_t *tmesh;                  /* [ntri] */
    double *tvb, *tv;                /* [ntri][9] vertices in the mesh frame; in the world (this step) */
    double *grav;
    /* history: contacts of the previous step, ascending key, with their u */
    int64_t nh;
    uint64_t *hkey;
    double *hu;
    /* per-step work */
    double *A;              /* [nc][9] */
    double *ww;             /* [nc][3] world angular velocity */
    double *xs;             /* [ns][3] */
    int64_t ncont, capcont;
    uint64_t *ckey;
    double *cdelta, *cF, *cu, *cra, *crb; /* per contact: delta, F on b, new u, lever arms */
    double *sF, *sT;        /* per sphere */
    double *cFc, *cTc;      /* per clump */
    /* transposed contact index: for sphere s, contacts in which s is the
     * higher id (partner < s), ascending partner */
    int64_t *lo_beg, *lo_idx;
};

static void *xmalloc(size_t n) {
    void *p = malloc(n ? n : 1);
    if (!p) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
    return p;
}
static double *dup_d(const double *src, size_t n) {
    double *p = (double *)xmalloc(n * sizeof(double));
    if (n) memcpy(p, src, n * sizeof(double));
    return p;
}

/* Damping ratio of a coefficient of restitution e in (0, 1]: ln e / sqrt(ln^2 e + pi^2).
 * It is <= 0, zero for e = 1, and increasing in e, so the pair value min(beta_a, beta_b)
 * is the damping of min(e_a, e_b). */
static double beta_of_cor(double e) {
    double l = log(e);
    return l / sqrt(l * l + M_PI * M_PI);
}

dem_oracle *dem_oracle_create(const dem_oracle_desc *d) {
    if (!d || d->n_clumps < 0 || d->n_templates < 1 || !(d->h > 0)) { set_err("invalid descriptor"); return NULL; }
    dem_oracle *o = (dem_oracle *)calloc(1, sizeof *o);
    o->h = d->h;
    o->nc = d->n_clumps;
    o->nsc = d->n_scenes;
    o->nb = d->n_bnd;
    int64_t nc = o->nc;
    o->sbeg = (int64_t *)xmalloc((nc + 1) * sizeof(int64_t));
    o->sbeg[0] = 0;
    for (int64_t c = 0; c < nc; c++) {
        uint32_t t = d->clump_template[c];
        if ((int32_t)t >= d->n_templates || d->clump_scene[c] >= (uint32_t)d->n_scenes) {
            set_err("clump template or scene out of range");
            dem_oracle_destroy(o);
            return NULL;
        }
        o->sbeg[c + 1] = o->sbeg[c] + (d->tmpl_sphere_begin[t + 1] - d->tmpl_sphere_begin[t]);
    }
    int64_t ns = o->ns = o->sbeg[nc];
    o->x = dup_d(d->x, 3 * nc);
    o->pos_exp = d->pos_exp;
    if (o->pos_exp != 0 && (o->pos_exp < 8 || o->pos_exp > 60)) {
        set_err("position exponent must be 0 or in [8, 60]");
        dem_oracle_destroy(o);
        return NULL;
    }
    o->eps = ldexp(1.0, -o->pos_exp);
    o->xq = (int64_t *)xmalloc(3 * (nc ? nc : 1) * sizeof(int64_t));
    o->xr = (double *)xmalloc(3 * (ns ? ns : 1) * sizeof(double));
    if (o->pos_exp) {
        for (int64_t k = 0; k < 3 * nc; k++) {
            double u = ldexp(d->x[k], o->pos_exp);  /* exact: a power-of-two scaling */
            if (!(fabs(u) < ldexp(1.0, 60))) {
                set_err("position outside the fixed-point range");
                dem_oracle_destroy(o);
                return NULL;
            }
            o->xq[k] = (int64_t)rint(u);
            o->x[k] = ldexp((double)o->xq[k], -o->pos_exp);
        }
    }
    o->q = dup_d(d->q, 4 * nc);
    o->v = dup_d(d->v, 3 * nc);
    o->w = dup_d(d->w, 3 * nc);
    o->mass = (double *)xmalloc(nc * sizeof(double));
    o->inertia = (double *)xmalloc(3 * nc * sizeof(double));
    o->scene = (uint32_t *)xmalloc(nc * sizeof(uint32_t));
    o->presc = (int32_t *)xmalloc(nc * sizeof(int32_t));
    o->owner = (uint32_t *)xmalloc(ns * sizeof(uint32_t));
    o->ofs = (double *)xmalloc(3 * ns * sizeof(double));
    o->rad = (double *)xmalloc(ns * sizeof(double));
    o->me = (double *)xmalloc(ns * sizeof(double));
    o->mg = (double *)xmalloc(ns * sizeof(double));
    o->mmu = (double *)xmalloc(ns * sizeof(double));
    o->mbeta = (double *)xmalloc(ns * sizeof(double));
    for (int64_t c = 0; c < nc; c++) {
        uint32_t t = d->clump_template[c];
        o->mass[c] = d->tmpl_mass[t];
        for (int k = 0; k < 3; k++) o->inertia[3 * c + k] = d->tmpl_inertia[3 * t + k];
        o->scene[c] = d->clump_scene[c];
        o->presc[c] = -1;
        uint32_t tb = d->tmpl_sphere_begin[t];
        for (int64_t s = o->sbeg[c]; s < o->sbeg[c + 1]; s++) {
            uint32_t ts = tb + (uint32_t)(s - o->sbeg[c]);
            o->owner[s] = (uint32_t)c;
            for (int k = 0; k < 3; k++) o->ofs[3 * s + k] = d->tmpl_offset[3 * ts + k];
            o->rad[s] = d->tmpl_radius[ts];
        }
    }
    for (int64_t s = 0; s < ns; s++) {
        const double *m = d->sphere_mat + 4 * s;
        double E = m[0], nu = m[1];
        o->me[s] = (1.0 - nu * nu) / E;
        o->mg[s] = 2.0 * (2.0 - nu) * (1.0 + nu) / E;
        o->mmu[s] = m[2];
        o->mbeta[s] = beta_of_cor(m[3]);
    }
    o->presc_param = dup_d(d->presc_param, (size_t)NPARAM_PRESC * d->n_presc);
    for (int32_t i = 0; i < d->n_presc; i++) {
        int32_t c = d->presc_clump[i];
        if (c < 0 || c >= nc) { set_err("prescribed clump out of range"); dem_oracle_destroy(o); return NULL; }
        o->presc[c] = i;
    }
    int32_t nb = o->nb;
    o->nm = d->n_mesh;
    o->ntri = d->n_tri;
    if (o->nm < 0 || o->ntri < 0 || (o->ntri && o->nm < 1) || (int64_t)nb + o->ntri > 0x7fffffff) {
        set_err("bad mesh sizes");
        dem_oracle_destroy(o);
        return NULL;
    }
    int32_t nw = o->nw = nb + (int32_t)o->ntri;
    o->btype = (int32_t *)xmalloc(nw * sizeof(int32_t));
    o->bscene = (int32_t *)xmalloc(nw * sizeof(int32_t));
    if (nb) {
        memcpy(o->btype, d->bnd_type, nb * sizeof(int32_t));
        memcpy(o->bscene, d->bnd_scene, nb * sizeof(int32_t));
    }
    o->bparam = dup_d(d->bnd_param, (size_t)NPARAM_BND * nb);
    o->bvel = dup_d(d->bnd_vel, 3 * (size_t)nb);
    o->bomega = dup_d(d->bnd_omega, 3 * (size_t)nb);
    o->be = (double *)xmalloc(nw * sizeof(double));
    o->bg = (double *)xmalloc(nw * sizeof(double));
    o->bmu = (double *)xmalloc(nw * sizeof(double));
    o->bbeta = (double *)xmalloc(nw * sizeof(double));
    for (int32_t i = 0; i < nb; i++) {
        const double *m = d->bnd_mat + 4 * i;
        double E = m[0], nu = m[1];
        o->be[i] = (1.0 - nu * nu) / E;
        o->bg[i] = 2.0 * (2.0 - nu) * (1.0 + nu) / E;
        o->bmu[i] = m[2];
        o->bbeta[i] = beta_of_cor(m[3]);
        if (o->btype[i] < 0 || o->btype[i] > 3) { set_err("unknown boundary type"); dem_oracle_destroy(o); return NULL; }
    }
    int32_t nm = o->nm;
    o->mx = (double *)xmalloc(3 * (size_t)nm * sizeof(double));
    o->mq = (double *)xmalloc(4 * (size_t)nm * sizeof(double));
    o->mv = (double *)xmalloc(3 * (size_t)nm * sizeof(double));
    o->mw = (double *)xmalloc(3 * (size_t)nm * sizeof(double));
    for (int32_t m = 0; m < nm; m++) dem_oracle_set_mesh_state(o, m, d->mesh_state + 13 * m);
    o->tmesh = (int32_t *)xmalloc(o->ntri * sizeof(int32_t));
    o->tvb = dup_d(d->tri_vertex, 9 * (size_t)o->ntri);
    o->tv = (double *)xmalloc(9 * (size_t)o->ntri * sizeof(double));
    for (int64_t k = 0; k < o->ntri; k++) {
        int32_t m = d->tri_mesh[k];
        if (m < 0 || m >= nm || d->mesh_scene[m] < 0 || d->mesh_scene[m] >= o->nsc) {
            set_err("triangle mesh or mesh scene out of range");
            dem_oracle_destroy(o);
            return NULL;
        }
        o->tmesh[k] = m;
        int32_t w = nb + (int32_t)k;  /* the triangle as a boundary: its mesh's material and scene */
        const double *mm = d->mesh_mat + 4 * m;
        double E = mm[0], nu = mm[1];
        o->be[w] = (1.0 - nu * nu) / E;
        o->bg[w] = 2.0 * (2.0 - nu) * (1.0 + nu) / E;
        o->bmu[w] = mm[2];
        o->bbeta[w] = beta_of_cor(mm[3]);
        o->bscene[w] = d->mesh_scene[m];
        o->btype[w] = -1;
    }
    o->grav = dup_d(d->gravity, 3 * (size_t)o->nsc);
    o->A = (double *)xmalloc(9 * nc * sizeof(double));
    o->ww = (double *)xmalloc(3 * nc * sizeof(double));
    o->xs = (double *)xmalloc(3 * ns * sizeof(double));
    o->sF = (double *)xmalloc(3 * ns * sizeof(double));
    o->sT = (double *)xmalloc(3 * ns * sizeof(double));
    o->cFc = (double *)xmalloc(3 * nc * sizeof(double));
    o->cTc = (double *)xmalloc(3 * nc * sizeof(double));
    o->lo_beg = (int64_t *)xmalloc((ns + 1) * sizeof(int64_t));
    return o;
}

void dem_oracle_destroy(dem_oracle *o) {
    if (!o) return;
    void *ptrs[] = {o->x, o->q, o->v, o->w, o->mass, o->inertia, o->scene, o->sbeg, o->presc,
                    o->presc_param, o->owner, o->ofs, o->rad, o->me, o->mg, o->mmu, o->mbeta,
                    o->btype, o->bscene, o->bparam, o->bvel, o->bomega, o->be, o->bg, o->bmu,
                    o->bbeta, o->grav, o->hkey, o->hu, o->A, o->ww, o->xs, o->ckey, o->cdelta,
                    o->cF, o->cu, o->cra, o->crb, o->sF, o->sT, o->cFc, o->cTc, o->lo_beg, o->lo_idx,
                    o->mx, o->mq, o->mv, o->mw, o->tmesh, o->tvb, o->tv, o->xq, o->xr};
    for (size_t i = 0; i < sizeof ptrs / sizeof ptrs[0]; i++) free(ptrs[i]);
    free(o);
}

int64_t dem_oracle_step_count(const dem_oracle *o) { return o->step; }
int dem_oracle_positions_ok(const dem_oracle *o) { return !o->bad_pos; }
void dem_oracle_read_fixed_positions(const dem_oracle *o, int64_t *k) {
    for (int64_t i = 0; i < 3 * o->nc; i++) k[i] = o->pos_exp ? o->xq[i] : 0;
}
int64_t dem_oracle_n_spheres(const dem_oracle *o) { return o->ns; }

/* ---------------- kinematics of the current state ---------------- */

/* Rotation matrix of a unit quaternion (w, x, y, z), row-major. */
static void quat_to_matrix(const double *q, double *A) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    A[0] = 1.0 - 2.0 * (y * y + z * z);
    A[1] = 2.0 * (x * y - w * z);
    A[2] = 2.0 * (x * z + w * y);
    A[3] = 2.0 * (x * y + w * z);
    A[4] = 1.0 - 2.0 * (x * x + z * z);
    A[5] = 2.0 * (y * z - w * x);
    A[6] = 2.0 * (x * z - w * y);
    A[7] = 2.0 * (y * z + w * x);
    A[8] = 1.0 - 2.0 * (x * x + y * y);
}

static void compute_poses(dem_oracle *o) {
    int64_t nc = o->nc;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; c++) {
        double *A = o->A + 9 * c;
        quat_to_matrix(o->q + 4 * c, A);
        const double *wb = o->w + 3 * c;
        for (int i = 0; i < 3; i++) o->ww[3 * c + i] = A[3 * i] * wb[0] + A[3 * i + 1] * wb[1] + A[3 * i + 2] * wb[2];
        for (int64_t s = o->sbeg[c]; s < o->sbeg[c + 1]; s++) {
            const double *of = o->ofs + 3 * s;
            for (int i = 0; i < 3; i++) {
                o->xr[3 * s + i] = A[3 * i] * of[0] + A[3 * i + 1] * of[1] + A[3 * i + 2] * of[2];
                o->xs[3 * s + i] = o->x[3 * c + i] + o->xr[3 * s + i];
            }
        }
    }
    /* triangle vertices in the world: x_mesh + A(q_mesh) v */
    for (int64_t k = 0; k < o->ntri; k++) {
        int32_t m = o->tmesh[k];
        double A[9];
        quat_to_matrix(o->mq + 4 * m, A);
        for (int j = 0; j < 3; j++) {
            const double *vb = o->tvb + 9 * k + 3 * j;
            for (int i = 0; i < 3; i++)
                o->tv[9 * k + 3 * j + i] = o->mx[3 * m + i] + (A[3 * i] * vb[0] + A[3 * i + 1] * vb[1] + A[3 * i + 2] * vb[2]);
        }
    }
}

/* ---------------- mesh triangles ---------------- */

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Closest point c of triangle (A, B, C) to point p, by the Voronoi regions
 * of its vertices, edges and face (the region tests of Ericson, Real-Time
 * Collision Detection, Sec. 5.1.5): barycentric coordinates from dot
 * products, the first region that holds p decides. */
static void closest_on_triangle(const double *A, const double *B, const double *C, const double *p, double *c) {
    double ab[3], ac[3], ap[3], bp[3], cp[3];
    for (int i = 0; i < 3; i++) { ab[i] = B[i] - A[i]; ac[i] = C[i] - A[i]; ap[i] = p[i] - A[i]; }
    double d1 = dot3(ab, ap), d2 = dot3(ac, ap);
    if (d1 <= 0.0 && d2 <= 0.0) { for (int i = 0; i < 3; i++) c[i] = A[i]; return; }
    for (int i = 0; i < 3; i++) bp[i] = p[i] - B[i];
    double d3 = dot3(ab, bp), d4 = dot3(ac, bp);
    if (d3 >= 0.0 && d4 <= d3) { for (int i = 0; i < 3; i++) c[i] = B[i]; return; }
    double vc = d1 * d4 - d3 * d2;
    if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
        double v = d1 / (d1 - d3);
        for (int i = 0; i < 3; i++) c[i] = A[i] + v * ab[i];
        return;
    }
    for (int i = 0; i < 3; i++) cp[i] = p[i] - C[i];
    double d5 = dot3(ab, cp), d6 = dot3(ac, cp);
    if (d6 >= 0.0 && d5 <= d6) { for (int i = 0; i < 3; i++) c[i] = C[i]; return; }
    double vb = d5 * d2 - d1 * d6;
    if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
        double w = d2 / (d2 - d6);
        for (int i = 0; i < 3; i++) c[i] = A[i] + w * ac[i];
        return;
    }
    double va = d3 * d6 - d5 * d4;
    double e43 = d4 - d3, e56 = d5 - d6;
    if (va <= 0.0 && e43 >= 0.0 && e56 >= 0.0) {
        double w = e43 / (e43 + e56);
        for (int i = 0; i < 3; i++) c[i] = B[i] + w * (C[i] - B[i]);
        return;
    }
    double den = (va + vb) + vc;
    double v = vb / den, w = vc / den;
    for (int i = 0; i < 3; i++) c[i] = (A[i] + ab[i] * v) + ac[i] * w;
}

/* Distance of p from triangle k and the unit normal from its closest point
 * towards p; 0 when p lies on the triangle (no normal). */
static int triangle_distance(const dem_oracle *o, int64_t k, const double *p, double *phi, double *n) {
    const double *V = o->tv + 9 * k;
    double c[3], d[3];
    closest_on_triangle(V, V + 3, V + 6, p, c);
    for (int i = 0; i < 3; i++) d[i] = p[i] - c[i];
    double dd = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (!(dd > 0.0)) return 0;
    *phi = dd;
    for (int i = 0; i < 3; i++) n[i] = d[i] / dd;
    return 1;
}

/* ---------------- analytic boundaries ---------------- */

/* Signed distance phi of point p from boundary b at time t (positive on the
 * domain side) and the unit normal n pointing from the wall into the domain.
 * Returns 0 when the boundary cannot touch p (outside its active range or on
 * a degenerate axis point). */
static int boundary_distance(const dem_oracle *o, int32_t b, double t, const double *p, double *phi, double *n) {
    if (b >= o->nb) return triangle_distance(o, b - o->nb, p, phi, n);
    const double *P = o->bparam + NPARAM_BND * b;
    const double *vel = o->bvel + 3 * b;
    double r0[3], d[3];
    for (int i = 0; i < 3; i++) r0[i] = P[i] + t * vel[i];
    for (int i = 0; i < 3; i++) d[i] = p[i] - r0[i];
    int type = o->btype[b];
    if (type == 0) { /* plane through r0 with unit normal P[3..5] into the domain */
        *phi = d[0] * P[3] + d[1] * P[4] + d[2] * P[5];
        n[0] = P[3]; n[1] = P[4]; n[2] = P[5];
        return 1;
    }
    /* axisymmetric primitives: axial coordinate ta and radial vector rho */
    const double *a = P + 3;
    double ta = d[0] * a[0] + d[1] * a[1] + d[2] * a[2];
    double rho[3];
    for (int i = 0; i < 3; i++) rho[i] = d[i] - ta * a[i];
    double r = sqrt(rho[0] * rho[0] + rho[1] * rho[1] + rho[2] * rho[2]);
    if (type == 1) { /* inside a cylinder of radius P[6] */
        if (!(r > 0.0)) return 0;
        *phi = P[6] - r;
        for (int i = 0; i < 3; i++) n[i] = -(rho[i] / r);
        return 1;
    }
    double sn = P[6], cs = P[7];
    if (type == 2) { /* outside a solid cone (apex r0, axis a into the solid) topped by a shaft */
        double H = P[8];
        double rb = H * (sn / cs);
        double lam = ta * cs + r * sn;
        if (ta >= H) { /* beside the shaft */
            if (!(r > 0.0)) return 0;
            *phi = r - rb;
            for (int i = 0; i < 3; i++) n[i] = rho[i] / r;
            return 1;
        }
        if (lam <= 0.0) { /* nearest point is the apex */
            double dd = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            if (!(dd > 0.0)) return 0;
            *phi = dd;
            for (int i = 0; i < 3; i++) n[i] = d[i] / dd;
            return 1;
        }
        if (!(r > 0.0)) return 0;
        if (lam <= H / cs) { /* lateral surface */
            *phi = r * cs - ta * sn;
            for (int i = 0; i < 3; i++) n[i] = (rho[i] / r) * cs - a[i] * sn;
            return 1;
        }
        /* nearest point is the base rim */
        double dt = ta - H, dr = r - rb;
        double dd = sqrt(dt * dt + dr * dr);
        if (!(dd > 0.0)) return 0;
        *phi = dd;
        for (int i = 0; i < 3; i++) n[i] = (dt * a[i] + dr * (rho[i] / r)) / dd;
        return 1;
    }
    /* type 3: inside an upward-opening cone (funnel wall) for t0 <= ta <= t1 */
    if (ta < P[8] || ta > P[9] || !(r > 0.0)) return 0;
    *phi = ta * sn - r * cs;
    for (int i = 0; i < 3; i++) n[i] = a[i] * sn - (rho[i] / r) * cs;
    return 1;
}

/* ---------------- contact law ---------------- */

/* Hertz-Mindlin force on body b of a contact with normal n (a -> b),
 * penetration delta > 0, relative velocity vrel = v_b - v_a at the contact
 * point, effective radius and mass, combined material, and the tangential
 * history u_old.  Writes the force F and the updated history u_new. */
static void contact_law(const double *n, double delta, const double *vrel, double Rbar, double mbar,
                        double estar, double gstar, double mu, double beta, double h,
                        const double *u_old, double *F, double *u_new) {
    const double kdamp = -2.0 * sqrt(5.0 / 6.0);
    double vn_s = vrel[0] * n[0] + vrel[1] * n[1] + vrel[2] * n[2];
    double vn[3], vt[3];
    for (int i = 0; i < 3; i++) vn[i] = vn_s * n[i];
    for (int i = 0; i < 3; i++) vt[i] = vrel[i] - vn[i];
    double sq = sqrt(Rbar * delta);
    /* normal: Hertz spring (4/3) E* sqrt(Rbar delta) delta and CoR-calibrated dashpot */
    double Sn = 2.0 * estar * sq;
    double gn = kdamp * beta * sqrt(Sn * mbar);
    double kn = (4.0 / 3.0) * estar * sq * delta;
    double Fn[3];
    for (int i = 0; i < 3; i++) Fn[i] = kn * n[i] - gn * vn[i];
    /* tangential: history update and projection onto the tangent plane */
    double up[3];
    for (int i = 0; i < 3; i++) up[i] = u_old[i] + h * vt[i];
    double upn = up[0] * n[0] + up[1] * n[1] + up[2] * n[2];
    double ut[3];
    for (int i = 0; i < 3; i++) ut[i] = up[i] - upn * n[i];
    double St = 8.0 * gstar * sq;
    double gt = kdamp * beta * sqrt(St * mbar);
    double Ft[3];
    for (int i = 0; i < 3; i++) Ft[i] = -(St * ut[i]) - gt * vt[i];
    double fn_norm = sqrt(Fn[0] * Fn[0] + Fn[1] * Fn[1] + Fn[2] * Fn[2]);
    double ft_norm = sqrt(Ft[0] * Ft[0] + Ft[1] * Ft[1] + Ft[2] * Ft[2]);
    double cap = mu * fn_norm;
    if (ft_norm > cap) {
        double scale = cap / ft_norm;
        for (int i = 0; i < 3; i++) Ft[i] = Ft[i] * scale;
        double ut_norm = sqrt(ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2]);
        if (ut_norm > 0.0) {
            double fac = (cap / St) / ut_norm;
            for (int i = 0; i < 3; i++) u_new[i] = fac * ut[i];
        } else {
            for (int i = 0; i < 3; i++) u_new[i] = 0.0;
        }
    } else {
        for (int i = 0; i < 3; i++) u_new[i] = ut[i];
    }
    for (int i = 0; i < 3; i++) F[i] = Fn[i] + Ft[i];
}

static void cross(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static int64_t find_history(const dem_oracle *o, uint64_t key) {
    int64_t lo = 0, hi = o->nh;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (o->hkey[mid] < key) lo = mid + 1; else hi = mid;
    }
    return (lo < o->nh && o->hkey[lo] == key) ? lo : -1;
}

/* Vector from sphere a to sphere b, and (fixed-point positions) the CoM
 * difference dc = x_cb - x_ca it contains: the world difference of the two
 * centres, or the exact integer difference of the CoMs plus the difference
 * of the rotated offsets. */
static void sphere_vec(const dem_oracle *o, int64_t a, int64_t b, double *dx, double *dc) {
    if (!o->pos_exp) {
        for (int i = 0; i < 3; i++) dx[i] = o->xs[3 * b + i] - o->xs[3 * a + i];
        return;
    }
    uint32_t ca = o->owner[a], cb = o->owner[b];
    for (int i = 0; i < 3; i++) {
        dc[i] = (double)(o->xq[3 * cb + i] - o->xq[3 * ca + i]) * o->eps;
        dx[i] = dc[i] + (o->xr[3 * b + i] - o->xr[3 * a + i]);
    }
}

/* ---------------- contact set (brute force) ---------------- */

/* Count (pass 0) or write (pass 1) the enlarged-geometry pairs of row a. */
static int64_t row_pairs(const dem_oracle *o, int64_t a, double t, const double *margin, uint64_t *out) {
    int64_t cnt = 0;
    const double *xa = o->xs + 3 * a;
    double Ra = o->rad[a];
    double ma = margin ? margin[a] : 0.0;
    uint32_t ca = o->owner[a];
    uint32_t sa = o->scene[ca];
    for (int64_t b = a + 1; b < o->ns; b++) {
        uint32_t cb = o->owner[b];
        if (cb == ca || o->scene[cb] != sa) continue;
        double v[3], dc[3];
        if (!o->pos_exp) {  /* (sphere_vec's first case, written out in this O(N^2) loop) */
            const double *xb = o->xs + 3 * b;
            v[0] = xb[0] - xa[0]; v[1] = xb[1] - xa[1]; v[2] = xb[2] - xa[2];
        } else {
            sphere_vec(o, a, b, v, dc);
        }
        double d2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        double S = o->rad[a] + o->rad[b];
        if (margin) S = S + (ma + margin[b]);
        if (d2 < S * S) {
            if (out) out[cnt] = ((uint64_t)a << 32) | (uint64_t)b;
            cnt++;
        }
    }
    for (int32_t w = 0; w < o->nw; w++) {
        if ((uint32_t)o->bscene[w] != sa) continue;
        double phi, n[3];
        if (!boundary_distance(o, w, t, xa, &phi, n)) continue;
        double lim = margin ? Ra + ma : Ra;
        if (phi < lim) {
            if (out) out[cnt] = ((uint64_t)a << 32) | (uint64_t)(o->ns + w);
            cnt++;
        }
    }
    return cnt;
}

static int64_t collect_pairs(const dem_oracle *o, const double *margin, uint64_t **keys_out) {
    int64_t ns = o->ns;
    double t = (double)o->step * o->h;
    int64_t *cnt = (int64_t *)xmalloc((ns + 1) * sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t a = 0; a < ns; a++) cnt[a] = row_pairs(o, a, t, margin, NULL);
    int64_t total = 0;
    for (int64_t a = 0; a < ns; a++) { int64_t c = cnt[a]; cnt[a] = total; total += c; }
    uint64_t *keys = (uint64_t *)xmalloc(total * sizeof(uint64_t));
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t a = 0; a < ns; a++) row_pairs(o, a, t, margin, keys + cnt[a]);
    free(cnt);
    *keys_out = keys;
    return total;
}

/* One candidate pair (a < b; b >= ns is boundary b - ns): penetration, and
 * when it is positive the force on body b and the updated history (Sec. 2.1).
 * ra, rb: lever arms from the bodies' reference points to the contact point. */
static double pair_eval(const dem_oracle *o, int64_t a, int64_t b, double t, const double *u_old, double *F,
                        double *un, double *ra, double *rb) {
    int64_t ns = o->ns;
    double h = o->h;
    double n[3], delta, p[3], vrel[3];
    double Rbar, mbar, estar, gstar, mu, beta;
    if (b < ns) {
        const double *xa = o->xs + 3 * a;
        double Ra = o->rad[a], Rb = o->rad[b];
        uint32_t ca = o->owner[a], cb = o->owner[b];
        double dx[3], dc[3];
        sphere_vec(o, a, b, dx, dc);
        double d = sqrt(dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2]);
        delta = (Ra + Rb) - d;
        for (int i = 0; i < 3; i++) n[i] = dx[i] / d;
        double lever = Ra - 0.5 * delta;
        if (!o->pos_exp) {
            for (int i = 0; i < 3; i++) p[i] = xa[i] + lever * n[i];
            for (int i = 0; i < 3; i++) { ra[i] = p[i] - o->x[3 * ca + i]; rb[i] = p[i] - o->x[3 * cb + i]; }
        } else {  /* from the CoM of a: its offset, then along n; from b's: less dc */
            for (int i = 0; i < 3; i++) { ra[i] = o->xr[3 * a + i] + lever * n[i]; rb[i] = ra[i] - dc[i]; }
        }
        double wa[3], wb[3];
        cross(o->ww + 3 * ca, ra, wa);
        cross(o->ww + 3 * cb, rb, wb);
        for (int i = 0; i < 3; i++) vrel[i] = (o->v[3 * cb + i] + wb[i]) - (o->v[3 * ca + i] + wa[i]);
        Rbar = (Ra * Rb) / (Ra + Rb);
        double Ma = o->mass[ca], Mb = o->mass[cb];
        mbar = (Ma * Mb) / (Ma + Mb);
        estar = 1.0 / (o->me[a] + o->me[b]);
        gstar = 1.0 / (o->mg[a] + o->mg[b]);
        mu = fmin(o->mmu[a], o->mmu[b]);
        beta = fmin(o->mbeta[a], o->mbeta[b]);
    } else {
        /* boundary contact: the boundary is body a, the sphere is body b */
        int32_t wi = (int32_t)(b - ns);
        int64_t s = a;
        const double *xsph = o->xs + 3 * s;
        double R = o->rad[s], phi;
        uint32_t cs = o->owner[s];
        boundary_distance(o, wi, t, xsph, &phi, n);
        delta = R - phi;
        double lever = R - 0.5 * delta;
        for (int i = 0; i < 3; i++) p[i] = xsph[i] - lever * n[i];
        /* the wall's reference point and velocity: an analytic boundary's
         * first parameters moved with its translation, or a mesh's reference
         * point; velocity v + w x (p - reference) */
        const double *vel, *om;
        double cwall[3], wv[3], pw[3];
        if (wi < o->nb) {
            const double *P = o->bparam + NPARAM_BND * wi;
            vel = o->bvel + 3 * wi;
            om = o->bomega + 3 * wi;
            for (int i = 0; i < 3; i++) cwall[i] = P[i] + t * vel[i];
        } else {
            int32_t m = o->tmesh[wi - o->nb];
            vel = o->mv + 3 * m;
            om = o->mw + 3 * m;
            for (int i = 0; i < 3; i++) cwall[i] = o->mx[3 * m + i];
        }
        for (int i = 0; i < 3; i++) {
            ra[i] = p[i] - cwall[i];
            rb[i] = o->pos_exp ? o->xr[3 * s + i] - lever * n[i] : p[i] - o->x[3 * cs + i];
        }
        cross(om, ra, pw);
        double wb[3];
        cross(o->ww + 3 * cs, rb, wb);
        for (int i = 0; i < 3; i++) wv[i] = vel[i] + pw[i];
        for (int i = 0; i < 3; i++) vrel[i] = (o->v[3 * cs + i] + wb[i]) - wv[i];
        Rbar = R;
        mbar = o->mass[cs];
        estar = 1.0 / (o->be[wi] + o->me[s]);
        gstar = 1.0 / (o->bg[wi] + o->mg[s]);
        mu = fmin(o->bmu[wi], o->mmu[s]);
        beta = fmin(o->bbeta[wi], o->mbeta[s]);
    }
    if (delta > 0.0) {
        contact_law(n, delta, vrel, Rbar, mbar, estar, gstar, mu, beta, h, u_old, F, un);
    } else {
        for (int i = 0; i < 3; i++) { F[i] = 0.0; un[i] = 0.0; }
    }
    return delta;
}

/* ---------------- one evaluation ---------------- */

int64_t dem_oracle_eval(dem_oracle *o) {
    int64_t ns = o->ns, nc = o->nc;
    double h = o->h;
    double t = (double)o->step * h;
    compute_poses(o);
    free(o->ckey);
    o->ckey = NULL;
    int64_t nk = collect_pairs(o, NULL, &o->ckey);
    o->ncont = nk;
    free(o->cdelta); free(o->cF); free(o->cu); free(o->cra); free(o->crb);
    o->cdelta = (double *)xmalloc(nk * sizeof(double));
    o->cF = (double *)xmalloc(3 * nk * sizeof(double));
    o->cu = (double *)xmalloc(3 * nk * sizeof(double));
    o->cra = (double *)xmalloc(3 * nk * sizeof(double));
    o->crb = (double *)xmalloc(3 * nk * sizeof(double));

#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nk; k++) {
        uint64_t key = o->ckey[k];
        int64_t a = (int64_t)(key >> 32), b = (int64_t)(key & 0xffffffffu);
        int64_t hi = find_history(o, key);
        double u_old[3] = {0.0, 0.0, 0.0};
        if (hi >= 0) for (int i = 0; i < 3; i++) u_old[i] = o->hu[3 * hi + i];
        double *F = o->cF + 3 * k, *un = o->cu + 3 * k;
        double delta = pair_eval(o, a, b, t, u_old, F, un, o->cra + 3 * k, o->crb + 3 * k);
        o->cdelta[k] = delta;
    }

    /* transposed index: contacts in which sphere s is the higher sphere id */
    for (int64_t s = 0; s <= ns; s++) o->lo_beg[s] = 0;
    for (int64_t k = 0; k < nk; k++) {
        int64_t b = (int64_t)(o->ckey[k] & 0xffffffffu);
        if (b < ns) o->lo_beg[b + 1]++;
    }
    for (int64_t s = 0; s < ns; s++) o->lo_beg[s + 1] += o->lo_beg[s];
    free(o->lo_idx);
    o->lo_idx = (int64_t *)xmalloc((o->lo_beg[ns] + 1) * sizeof(int64_t));
    {
        int64_t *fill = (int64_t *)xmalloc((ns + 1) * sizeof(int64_t));
        memcpy(fill, o->lo_beg, (ns + 1) * sizeof(int64_t));
        for (int64_t k = 0; k < nk; k++) {
            int64_t b = (int64_t)(o->ckey[k] & 0xffffffffu);
            if (b < ns) o->lo_idx[fill[b]++] = k;
        }
        free(fill);
    }
    /* row start of each sphere's own (higher-partner) contacts */
    int64_t *hi_beg = (int64_t *)xmalloc((ns + 1) * sizeof(int64_t));
    {
        int64_t k = 0;
        for (int64_t s = 0; s < ns; s++) {
            hi_beg[s] = k;
            while (k < nk && (int64_t)(o->ckey[k] >> 32) == s) k++;
        }
        hi_beg[ns] = nk;
    }

    /* per-sphere sums in ascending partner id */
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < ns; s++) {
        double Fs[3] = {0.0, 0.0, 0.0}, Ts[3] = {0.0, 0.0, 0.0};
        for (int64_t j = o->lo_beg[s]; j < o->lo_beg[s + 1]; j++) { /* s is body b */
            int64_t k = o->lo_idx[j];
            if (!(o->cdelta[k] > 0.0)) continue;
            const double *F = o->cF + 3 * k;
            double tq[3];
            cross(o->crb + 3 * k, F, tq);
            for (int i = 0; i < 3; i++) { Fs[i] = Fs[i] + F[i]; Ts[i] = Ts[i] + tq[i]; }
        }
        for (int64_t k = hi_beg[s]; k < hi_beg[s + 1]; k++) {
            if (!(o->cdelta[k] > 0.0)) continue;
            int64_t b = (int64_t)(o->ckey[k] & 0xffffffffu);
            const double *F = o->cF + 3 * k;
            double tq[3], f[3];
            if (b < ns) { /* s is body a: receives -F */
                for (int i = 0; i < 3; i++) f[i] = -F[i];
                cross(o->cra + 3 * k, f, tq);
            } else {      /* boundary contact: s is body b */
                for (int i = 0; i < 3; i++) f[i] = F[i];
                cross(o->crb + 3 * k, f, tq);
            }
            for (int i = 0; i < 3; i++) { Fs[i] = Fs[i] + f[i]; Ts[i] = Ts[i] + tq[i]; }
        }
        for (int i = 0; i < 3; i++) { o->sF[3 * s + i] = Fs[i]; o->sT[3 * s + i] = Ts[i]; }
    }
    free(hi_beg);

    /* per-clump sums in ascending sphere id, then gravity */
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; c++) {
        double Fc[3] = {0.0, 0.0, 0.0}, Tc[3] = {0.0, 0.0, 0.0};
        for (int64_t s = o->sbeg[c]; s < o->sbeg[c + 1]; s++)
            for (int i = 0; i < 3; i++) { Fc[i] = Fc[i] + o->sF[3 * s + i]; Tc[i] = Tc[i] + o->sT[3 * s + i]; }
        const double *g = o->grav + 3 * o->scene[c];
        for (int i = 0; i < 3; i++) Fc[i] = Fc[i] + o->mass[c] * g[i];
        for (int i = 0; i < 3; i++) { o->cFc[3 * c + i] = Fc[i]; o->cTc[3 * c + i] = Tc[i]; }
    }
    return nk;
}

/* ---------------- integration ---------------- */

/* x += h v; with fixed-point positions the increment h v is rounded to the
 * grid (ties to even) and added to the integer, then decoded. */
static void advance_position(dem_oracle *o, int64_t c, double *x, const double *v) {
    double h = o->h;
    if (!o->pos_exp) {
        for (int i = 0; i < 3; i++) x[i] = x[i] + h * v[i];
        return;
    }
    int64_t *k = o->xq + 3 * c;
    for (int i = 0; i < 3; i++) {
        double u = rint(ldexp(h * v[i], o->pos_exp));
        if (!(fabs(u) < ldexp(1.0, 61)) || llabs(k[i]) >= ((int64_t)1 << 61)) {
            o->bad_pos = 1;
            continue;
        }
        k[i] = k[i] + (int64_t)u;
        x[i] = ldexp((double)k[i], -o->pos_exp);
    }
}

static void integrate(dem_oracle *o) {
    int64_t nc = o->nc;
    double h = o->h;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; c++) {
        const double *F = o->cFc + 3 * c, *T = o->cTc + 3 * c, *A = o->A + 9 * c;
        double *x = o->x + 3 * c, *v = o->v + 3 * c, *w = o->w + 3 * c, *q = o->q + 4 * c;
        double M = o->mass[c];
        const double *I = o->inertia + 3 * c;
        int32_t pi = o->presc[c];
        if (pi < 0) {
            for (int i = 0; i < 3; i++) v[i] = v[i] + h * (F[i] / M);
            advance_position(o, c, x, v);
            /* body-frame torque and Euler's equations with the gyroscopic term */
            double tb[3];
            for (int i = 0; i < 3; i++) tb[i] = A[i] * T[0] + A[3 + i] * T[1] + A[6 + i] * T[2];
            double L[3] = {I[0] * w[0], I[1] * w[1], I[2] * w[2]};
            double gy[3];
            cross(w, L, gy);
            for (int i = 0; i < 3; i++) w[i] = w[i] + h * ((tb[i] - gy[i]) / I[i]);
        } else {
            const double *P = o->presc_param + NPARAM_PRESC * pi;
            for (int i = 0; i < 3; i++) {
                if (P[3 + i] != 0.0) v[i] = v[i] + h * ((F[i] + P[9 + i]) / M);
                else v[i] = P[i];
            }
            advance_position(o, c, x, v);
            for (int i = 0; i < 3; i++) w[i] = P[6 + i];
        }
        /* q <- q + (h/2) q (x) (0, w), then renormalise */
        double dq[4];
        dq[0] = -(q[1] * w[0] + q[2] * w[1] + q[3] * w[2]);
        dq[1] = q[0] * w[0] + q[2] * w[2] - q[3] * w[1];
        dq[2] = q[0] * w[1] + q[3] * w[0] - q[1] * w[2];
        dq[3] = q[0] * w[2] + q[1] * w[1] - q[2] * w[0];
        double hh = 0.5 * h;
        for (int i = 0; i < 4; i++) q[i] = q[i] + hh * dq[i];
        double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        for (int i = 0; i < 4; i++) q[i] = q[i] / qn;
    }
}

/* Meshes follow their prescribed motion: x += h v; the orientation turns at
 * the world-frame angular velocity w, q += (h/2) (0, w) (x) q, renormalised. */
static void advance_meshes(dem_oracle *o) {
    double h = o->h, hh = 0.5 * h;
    for (int32_t m = 0; m < o->nm; m++) {
        double *x = o->mx + 3 * m, *q = o->mq + 4 * m;
        const double *v = o->mv + 3 * m, *w = o->mw + 3 * m;
        for (int i = 0; i < 3; i++) x[i] = x[i] + h * v[i];
        double dq[4];
        dq[0] = -(w[0] * q[1] + w[1] * q[2] + w[2] * q[3]);
        dq[1] = q[0] * w[0] + (w[1] * q[3] - w[2] * q[2]);
        dq[2] = q[0] * w[1] + (w[2] * q[1] - w[0] * q[3]);
        dq[3] = q[0] * w[2] + (w[0] * q[2] - w[1] * q[1]);
        for (int i = 0; i < 4; i++) q[i] = q[i] + hh * dq[i];
        double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        for (int i = 0; i < 4; i++) q[i] = q[i] / qn;
    }
}

void dem_oracle_step(dem_oracle *o, int64_t n) {
    for (int64_t it = 0; it < n; it++) {
        dem_oracle_eval(o);
        /* commit history: every contact of this step with its updated u */
        free(o->hkey);
        free(o->hu);
        o->nh = o->ncont;
        o->hkey = (uint64_t *)xmalloc(o->nh * sizeof(uint64_t));
        o->hu = (double *)xmalloc(3 * o->nh * sizeof(double));
        if (o->nh) {
            memcpy(o->hkey, o->ckey, o->nh * sizeof(uint64_t));
            memcpy(o->hu, o->cu, 3 * o->nh * sizeof(double));
        }
        integrate(o);
        advance_meshes(o);
        o->step++;
    }
}

/* ---------------- readers ---------------- */

void dem_oracle_read_contacts(const dem_oracle *o, uint32_t *a, uint32_t *b, double *delta, double *F, double *u) {
    for (int64_t k = 0; k < o->ncont; k++) {
        if (a) a[k] = (uint32_t)(o->ckey[k] >> 32);
        if (b) b[k] = (uint32_t)(o->ckey[k] & 0xffffffffu);
        if (delta) delta[k] = o->cdelta[k];
    }
    if (F && o->ncont) memcpy(F, o->cF, 3 * o->ncont * sizeof(double));
    if (u && o->ncont) memcpy(u, o->cu, 3 * o->ncont * sizeof(double));
}

void dem_oracle_read_contact_torques(const dem_oracle *o, double *Ta, double *Tb) {
    /* per contact of the last evaluation: the torque r x F the contact exerts
     * on each body about its reference point (Eq. newton_law_2 with the
     * lever arms of Eq. kinematicsContactInfo); body a receives -F, body b F */
    for (int64_t k = 0; k < o->ncont; k++) {
        const double *F = o->cF + 3 * k;
        double f[3] = {-F[0], -F[1], -F[2]};
        if (Ta) cross(o->cra + 3 * k, f, Ta + 3 * k);
        if (Tb) cross(o->crb + 3 * k, F, Tb + 3 * k);
    }
}

void dem_oracle_read_clump_forces(const dem_oracle *o, double *F, double *T) {
    if (F) memcpy(F, o->cFc, 3 * o->nc * sizeof(double));
    if (T) memcpy(T, o->cTc, 3 * o->nc * sizeof(double));
}

void dem_oracle_read_sphere_forces(const dem_oracle *o, double *F, double *T) {
    if (F) memcpy(F, o->sF, 3 * o->ns * sizeof(double));
    if (T) memcpy(T, o->sT, 3 * o->ns * sizeof(double));
}

void dem_oracle_read_boundary_forces(const dem_oracle *o, double *F, double *T) {
    /* Newton's third law on each boundary contact of the last evaluation, in
     * ascending contact order: the boundary receives -F (F acts on the sphere)
     * at the contact point, lever arm cra = p - (boundary reference point) */
    for (int64_t i = 0; i < 3 * (int64_t)o->nb; i++) { F[i] = 0.0; T[i] = 0.0; }
    for (int64_t k = 0; k < o->ncont; k++) {
        int64_t b = (int64_t)(o->ckey[k] & 0xffffffffu);
        if (b < o->ns || !(o->cdelta[k] > 0.0)) continue;
        int64_t w = b - o->ns;
        if (w >= o->nb) continue;  /* a mesh triangle: see dem_oracle_read_mesh_forces */
        double f[3] = {-o->cF[3 * k], -o->cF[3 * k + 1], -o->cF[3 * k + 2]}, tq[3];
        cross(o->cra + 3 * k, f, tq);
        for (int i = 0; i < 3; i++) { F[3 * w + i] = F[3 * w + i] + f[i]; T[3 * w + i] = T[3 * w + i] + tq[i]; }
    }
}

void dem_oracle_read_mesh_forces(const dem_oracle *o, double *F, double *T) {
    for (int32_t m = 0; m < 3 * o->nm; m++) { F[m] = 0.0; T[m] = 0.0; }
    for (int64_t k = 0; k < o->ncont; k++) {
        int64_t b = (int64_t)(o->ckey[k] & 0xffffffffu) - o->ns - o->nb;
        if (b < 0 || !(o->cdelta[k] > 0.0)) continue;
        int32_t m = o->tmesh[b];
        double f[3], tq[3];
        for (int i = 0; i < 3; i++) f[i] = -o->cF[3 * k + i];  /* the mesh receives -F at the contact point */
        cross(o->cra + 3 * k, f, tq);
        for (int i = 0; i < 3; i++) { F[3 * m + i] = F[3 * m + i] + f[i]; T[3 * m + i] = T[3 * m + i] + tq[i]; }
    }
}

void dem_oracle_read_mesh_state(const dem_oracle *o, double *st) {
    for (int32_t m = 0; m < o->nm; m++) {
        double *r = st + 13 * m;
        for (int i = 0; i < 3; i++) { r[i] = o->mx[3 * m + i]; r[7 + i] = o->mv[3 * m + i]; r[10 + i] = o->mw[3 * m + i]; }
        for (int i = 0; i < 4; i++) r[3 + i] = o->mq[4 * m + i];
    }
}

int dem_oracle_set_mesh_state(dem_oracle *o, int32_t m, const double *st) {
    if (m < 0 || m >= o->nm) return -1;
    for (int i = 0; i < 3; i++) { o->mx[3 * m + i] = st[i]; o->mv[3 * m + i] = st[7 + i]; o->mw[3 * m + i] = st[10 + i]; }
    for (int i = 0; i < 4; i++) o->mq[4 * m + i] = st[3 + i];
    return 0;
}

void dem_oracle_read_state(const dem_oracle *o, double *x, double *q, double *v, double *w) {
    if (x) memcpy(x, o->x, 3 * o->nc * sizeof(double));
    if (q) memcpy(q, o->q, 4 * o->nc * sizeof(double));
    if (v) memcpy(v, o->v, 3 * o->nc * sizeof(double));
    if (w) memcpy(w, o->w, 3 * o->nc * sizeof(double));
}

void dem_oracle_read_sphere_pos(const dem_oracle *o, double *xs) {
    /* positions of the current state */
    compute_poses((dem_oracle *)o);
    memcpy(xs, o->xs, 3 * o->ns * sizeof(double));
}

int64_t dem_oracle_candidates(dem_oracle *o, const double *margin, uint32_t *a, uint32_t *b, int64_t cap) {
    compute_poses(o);
    uint64_t *keys = NULL;
    int64_t n = collect_pairs(o, margin, &keys);
    for (int64_t k = 0; k < n && k < cap; k++) {
        if (a) a[k] = (uint32_t)(keys[k] >> 32);
        if (b) b[k] = (uint32_t)(keys[k] & 0xffffffffu);
    }
    free(keys);
    return n;
}

/* ---------------- sampled evaluation (large scenes) ---------------- */

typedef struct sample_row {
    int64_t n, cap;
    uint64_t *key;
    double *delta, *F;
} sample_row;

static void row_push(sample_row *r, uint64_t key, double delta, const double *F) {
    if (r->n == r->cap) {
        r->cap = r->cap ? 2 * r->cap : 16;
        r->key = (uint64_t *)realloc(r->key, r->cap * sizeof(uint64_t));
        r->delta = (double *)realloc(r->delta, r->cap * sizeof(double));
        r->F = (double *)realloc(r->F, 3 * r->cap * sizeof(double));
        if (!r->key || !r->delta || !r->F) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
    }
    r->key[r->n] = key;
    r->delta[r->n] = delta;
    for (int i = 0; i < 3; i++) r->F[3 * r->n + i] = F[i];
    r->n++;
}

/* Force and torque on sphere s from every contact it has at the current state,
 * summed in ascending partner id exactly as the full evaluation sums them;
 * the contacts themselves go to row r. */
static void sphere_sample(const dem_oracle *o, int64_t s, double t, double *Fs, double *Ts, sample_row *r) {
    int64_t ns = o->ns;
    uint32_t cs = o->owner[s], sc = o->scene[cs];
    const double *xs = o->xs + 3 * s;
    for (int i = 0; i < 3; i++) { Fs[i] = 0.0; Ts[i] = 0.0; }
    for (int64_t p = 0; p <= ns + o->nw - 1; p++) {
        if (p == s) continue;
        int64_t a, b;
        if (p < ns) {
            a = s < p ? s : p;
            b = s < p ? p : s;
            /* the exact predicate of the contact set, evaluated from the lower sphere */
            double v[3], dc[3];
            sphere_vec(o, a, b, v, dc);
            double d2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
            double S = o->rad[a] + o->rad[b];
            if (!(d2 < S * S)) continue;
            uint32_t cp = o->owner[p];
            if (cp == cs || o->scene[cp] != sc) continue;
        } else {
            int32_t w = (int32_t)(p - ns);
            if ((uint32_t)o->bscene[w] != sc) continue;
            double phi, n[3];
            if (!boundary_distance(o, w, t, xs, &phi, n) || !(phi < o->rad[s])) continue;
            a = s;
            b = p;
        }
        uint64_t key = ((uint64_t)a << 32) | (uint64_t)b;
        int64_t hi = find_history(o, key);
        double u_old[3] = {0.0, 0.0, 0.0}, F[3], un[3], ra[3], rb[3];
        if (hi >= 0) for (int i = 0; i < 3; i++) u_old[i] = o->hu[3 * hi + i];
        double delta = pair_eval(o, a, b, t, u_old, F, un, ra, rb);
        row_push(r, key, delta, F);
        if (!(delta > 0.0)) continue;
        double f[3], tq[3];
        if (b == s || b >= ns) { /* s is body b */
            for (int i = 0; i < 3; i++) f[i] = F[i];
            cross(rb, f, tq);
        } else {                 /* s is body a */
            for (int i = 0; i < 3; i++) f[i] = -F[i];
            cross(ra, f, tq);
        }
        for (int i = 0; i < 3; i++) { Fs[i] = Fs[i] + f[i]; Ts[i] = Ts[i] + tq[i]; }
    }
}

int64_t dem_oracle_sample_spheres(dem_oracle *o, const int64_t *ids, int64_t n, double *F, double *T, int64_t cap,
                                  int64_t *beg, uint32_t *ca, uint32_t *cb, double *cdelta, double *cF) {
    if (n < 0) { set_err("sample: negative count"); return -1; }
    for (int64_t k = 0; k < n; k++)
        if (ids[k] < 0 || ids[k] >= o->ns) { set_err("sample: sphere id out of range"); return -1; }
    compute_poses(o);
    double t = (double)o->step * o->h;
    sample_row *rows = (sample_row *)calloc((size_t)(n ? n : 1), sizeof(sample_row));
    if (!rows) { set_err("sample: out of memory"); return -1; }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < n; k++) {
        double Fs[3], Ts[3];
        sphere_sample(o, ids[k], t, Fs, Ts, &rows[k]);
        for (int i = 0; i < 3; i++) {
            if (F) F[3 * k + i] = Fs[i];
            if (T) T[3 * k + i] = Ts[i];
        }
    }
    int64_t m = 0;
    for (int64_t k = 0; k < n; k++) {
        if (beg) beg[k] = m;
        for (int64_t j = 0; j < rows[k].n; j++, m++) {
            if (m >= cap) continue;
            if (ca) ca[m] = (uint32_t)(rows[k].key[j] >> 32);
            if (cb) cb[m] = (uint32_t)(rows[k].key[j] & 0xffffffffu);
            if (cdelta) cdelta[m] = rows[k].delta[j];
            if (cF) for (int i = 0; i < 3; i++) cF[3 * m + i] = rows[k].F[3 * j + i];
        }
        free(rows[k].key); free(rows[k].delta); free(rows[k].F);
    }
    if (beg) beg[n] = m;
    free(rows);
    return m;
}

int dem_oracle_sample_clumps(dem_oracle *o, const int64_t *clumps, int64_t n, double *F, double *T) {
    int64_t tot = 0;
    for (int64_t k = 0; k < n; k++) {
        if (clumps[k] < 0 || clumps[k] >= o->nc) { set_err("sample: clump id out of range"); return -1; }
        tot += o->sbeg[clumps[k] + 1] - o->sbeg[clumps[k]];
    }
    int64_t *ids = (int64_t *)xmalloc((tot ? tot : 1) * sizeof(int64_t));
    double *sF = (double *)xmalloc(3 * (tot ? tot : 1) * sizeof(double));
    double *sT = (double *)xmalloc(3 * (tot ? tot : 1) * sizeof(double));
    int64_t m = 0;
    for (int64_t k = 0; k < n; k++)
        for (int64_t s = o->sbeg[clumps[k]]; s < o->sbeg[clumps[k] + 1]; s++) ids[m++] = s;
    if (dem_oracle_sample_spheres(o, ids, tot, sF, sT, 0, NULL, NULL, NULL, NULL, NULL) < 0) {
        free(ids); free(sF); free(sT);
        return -1;
    }
    /* per-clump sums in ascending sphere id, then gravity, as in the full evaluation */
    m = 0;
    for (int64_t k = 0; k < n; k++) {
        int64_t c = clumps[k];
        double Fc[3] = {0.0, 0.0, 0.0}, Tc[3] = {0.0, 0.0, 0.0};
        for (int64_t s = o->sbeg[c]; s < o->sbeg[c + 1]; s++, m++)
            for (int i = 0; i < 3; i++) { Fc[i] = Fc[i] + sF[3 * m + i]; Tc[i] = Tc[i] + sT[3 * m + i]; }
        const double *g = o->grav + 3 * o->scene[c];
        for (int i = 0; i < 3; i++) Fc[i] = Fc[i] + o->mass[c] * g[i];
        for (int i = 0; i < 3; i++) { F[3 * k + i] = Fc[i]; T[3 * k + i] = Tc[i]; }
    }
    free(ids); free(sF); free(sT);
    return 0;
}
