/*
 * FP64 brute-force CPU oracle of the clumped-sphere DEM timestep.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP implementation.
 *
 * What it computes (paper: Sec. 2.1 and Sec. 2.2):
 *   sphere world positions from clump poses (multi-sphere clumps, Sec. 2.1);
 *   the contact set by O(N^2) brute force (every candidate pair tested,
 *   no binning, no margin);
 *   sphere-boundary contacts against analytic primitives and against the
 *   triangles of rigid meshes whose motion is prescribed;
 *   the Hertz-Mindlin law of Eq. "normal_tangential_force_model1/2" with the
 *   kinematics of Eq. "kinematicsContactInfo", the tangential history update
 *   of Eq. "updateUt" and its Coulomb clamp of Eq. "cappingOfut";
 *   accumulation onto clumps and the Newton-Euler equations of
 *   Eq. "newton_law_1/2", advanced by symplectic Euler.
 *
 * Everything is IEEE FP64, evaluated in a fixed order (see oracle.c).
 * All arrays are SI, structure-of-arrays, 0-based; the descriptor is borrowed
 * for the duration of dem_oracle_create only.
 */
#ifndef DEM_ORACLE_H
#define DEM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dem_oracle dem_oracle;

typedef struct dem_oracle_desc {
    double h;                          /* time step [s] */
    int32_t n_templates;
    const uint32_t *tmpl_sphere_begin; /* [n_templates+1] CSR into template spheres */
    const double *tmpl_offset;         /* [n_tmpl_spheres][3] body frame, about the CoM */
    const double *tmpl_radius;         /* [n_tmpl_spheres] */
    const double *tmpl_mass;           /* [n_templates] */
    const double *tmpl_inertia;        /* [n_templates][3] principal moments */
    int64_t n_clumps;
    const uint32_t *clump_template;    /* [n_clumps] */
    const uint32_t *clump_scene;       /* [n_clumps] */
    const double *x;                   /* [n_clumps][3] CoM position (world) */
    const double *q;                   /* [n_clumps][4] unit quaternion w,x,y,z (body->world) */
    const double *v;                   /* [n_clumps][3] CoM velocity (world) */
    const double *w;                   /* [n_clumps][3] angular velocity (body frame) */
    const double *sphere_mat;          /* [n_spheres][4] E, nu, mu, CoR per sphere instance */
    int32_t n_scenes;
    const double *gravity;             /* [n_scenes][3] */
    int32_t n_bnd;
    const int32_t *bnd_type;           /* [n_bnd] 0 plane, 1 cyl_in, 2 cone_out, 3 frustum_in */
    const double *bnd_param;           /* [n_bnd][12] geometry at t = 0 */
    const double *bnd_mat;             /* [n_bnd][4] E, nu, mu, CoR */
    const double *bnd_vel;             /* [n_bnd][3] prescribed translation velocity */
    const double *bnd_omega;           /* [n_bnd][3] prescribed spin about the reference point */
    const int32_t *bnd_scene;          /* [n_bnd] */
    int32_t n_presc;
    const int32_t *presc_clump;        /* [n_presc] */
    const double *presc_param;         /* [n_presc][12] v_fixed, free mask, w_body, f_extra */
    /* triangle meshes: rigid boundaries whose motion is prescribed */
    int32_t n_mesh;
    const double *mesh_state;          /* [n_mesh][13] x[3] reference point, q[4] (mesh->world),
                                          v[3], w[3] angular velocity (world frame) */
    const double *mesh_mat;            /* [n_mesh][4] E, nu, mu, CoR */
    const int32_t *mesh_scene;         /* [n_mesh] */
    int64_t n_tri;
    const int32_t *tri_mesh;           /* [n_tri] */
    const double *tri_vertex;          /* [n_tri][3][3] vertices in the mesh frame */
    /* clump positions: 0 = FP64; E in [8, 60] = fixed point, x = k 2^-E with
     * an integer k per axis (the voxel id k >> 32 and the sub-voxel offset
     * k mod 2^32 of a voxel of side 2^(32-E)), so that the vector between
     * two spheres is an exact integer difference plus their rotated offsets */
    int32_t pos_exp;
} dem_oracle_desc;

/* Returns NULL on invalid input (message via dem_oracle_last_error). */
dem_oracle *dem_oracle_create(const dem_oracle_desc *d);
void dem_oracle_destroy(dem_oracle *o);
const char *dem_oracle_last_error(void);
void dem_oracle_set_threads(int n);

/* Advance n steps; each step evaluates contacts and forces, commits the
 * tangential history and integrates. */
void dem_oracle_step(dem_oracle *o, int64_t n);
int64_t dem_oracle_step_count(const dem_oracle *o);
/* 0 once a fixed-point position has left its range (|k| >= 2^61). */
int dem_oracle_positions_ok(const dem_oracle *o);
/* The fixed-point CoM integers [n_clumps][3] (zeros with FP64 positions). */
void dem_oracle_read_fixed_positions(const dem_oracle *o, int64_t *k);

/* Evaluate contacts and forces at the current state without advancing and
 * without committing history.  Returns the number of contacts (sphere-sphere
 * and sphere-boundary).  The results stay readable until the next call. */
int64_t dem_oracle_eval(dem_oracle *o);

/* Contacts of the last evaluation, ascending by (a, b).  Sphere-sphere pairs
 * have a < b < n_spheres; a boundary contact has a = sphere and
 * b = n_spheres + boundary index.  F is the force on b (the negative acts on
 * a), u the tangential history after this step's update and clamp.
 * Any output pointer may be NULL. */
void dem_oracle_read_contacts(const dem_oracle *o, uint32_t *a, uint32_t *b, double *delta,
                              double *F, double *u);
/* Per contact of the last evaluation (same order as read_contacts): the
 * torque the contact exerts on body a (r_a x -F) and on body b (r_b x F),
 * each about the body's reference point (a sphere's clump centre of mass, a
 * boundary's reference point); [n][3] each, either may be NULL. */
void dem_oracle_read_contact_torques(const dem_oracle *o, double *Ta, double *Tb);
void dem_oracle_read_clump_forces(const dem_oracle *o, double *F, double *T);
void dem_oracle_read_sphere_forces(const dem_oracle *o, double *F, double *T);
/* Force exerted on each boundary by the spheres (minus the contact forces on
 * them) and its torque about the boundary's reference point, from the last
 * evaluation; [n_bnd][3] each, in the description's boundary order. */
void dem_oracle_read_boundary_forces(const dem_oracle *o, double *F, double *T);
void dem_oracle_read_state(const dem_oracle *o, double *x, double *q, double *v, double *w);
/* Triangle meshes.  A contact of sphere s with triangle k has
 * b = n_spheres + n_bnd + k.  Force the spheres exert on each mesh and its
 * torque about the mesh's reference point, from the last evaluation,
 * [n_mesh][3] each. */
void dem_oracle_read_mesh_forces(const dem_oracle *o, double *F, double *T);
/* Mesh states [n_mesh][13] (x, q, v, w as in the descriptor). */
void dem_oracle_read_mesh_state(const dem_oracle *o, double *state);
/* Prescribe a mesh's state (13 doubles); returns -1 for a bad index. */
int dem_oracle_set_mesh_state(dem_oracle *o, int32_t mesh, const double *state);
void dem_oracle_read_sphere_pos(const dem_oracle *o, double *xs);
int64_t dem_oracle_n_spheres(const dem_oracle *o);

/* Brute-force enlarged-geometry candidates at the current state:
 * sphere pairs with d^2 < ((Ra+Rb)+(ma+mb))^2 and boundary pairs with
 * phi < R + m.  margin may be NULL (all zero).  Writes at most cap pairs,
 * returns the total count. */
int64_t dem_oracle_candidates(dem_oracle *o, const double *margin, uint32_t *a, uint32_t *b,
                              int64_t cap);

/* Sampled evaluation for scenes too large for the O(N^2) sweep: for each
 * sphere ids[k], its force and torque at the current state (F, T [n][3],
 * identical to what dem_oracle_eval would give that sphere) and its contacts,
 * listed sample by sample in ascending partner id as canonical (a, b) with
 * the penetration and the force on b; beg [n+1] receives where each sample's
 * list starts.  A pair of two sampled spheres appears once per sample.  Each candidate partner is tested by brute force: cost
 * O(n * n_spheres).  Writes at most cap contacts; returns the total, or -1 on
 * an invalid id.  Does not advance or commit history.  Output pointers may be
 * NULL. */
int64_t dem_oracle_sample_spheres(dem_oracle *o, const int64_t *ids, int64_t n, double *F, double *T,
                                  int64_t cap, int64_t *beg, uint32_t *ca, uint32_t *cb, double *cdelta,
                                  double *cF);
/* Force (contacts + gravity) and torque of each clump clumps[k], [n][3], as
 * dem_oracle_eval would give them.  Returns 0, or -1 on an invalid id. */
int dem_oracle_sample_clumps(dem_oracle *o, const int64_t *clumps, int64_t n, double *F, double *T);

#ifdef __cplusplus
}
#endif
#endif
