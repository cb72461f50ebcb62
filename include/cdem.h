/*
 * cdem -- clumped-sphere discrete-element timestep on MI355X (gfx950).
 *
 * C ABI of the HIP library libcdem.so.  Plain pointers and sizes only; no C++
 * exception crosses this boundary.  Every function returns CDEM_OK (0) or a
 * negative CDEM_E_* code; cdem_last_error() gives a message for the scene.
 *
 * The method (paper Sec. 2.1 and 2.2):
 *   - elements are clumps: rigid unions of spheres; mass and inertia belong to
 *     the clump, E, nu, mu and CoR to each sphere instance (Sec. 2.1, clump
 *     paragraph and Fig. "force");
 *   - each step detects contacts (spatial binning, Sec. 1 citing the binning
 *     approach; enlarged contact geometry when detection is deferred, Sec. 2.2),
 *     evaluates the Hertz-Mindlin force of Eq. normal_tangential_force_model1/2
 *     with the kinematics of Eq. kinematicsContactInfo and a persistent
 *     tangential history (Eqs. updateUt and cappingOfut), reduces forces and
 *     torques onto the clumps and integrates Eq. newton_law_1/2;
 *   - detection may run every step (the traditional scheme, Sec. 2.2) or every
 *     k steps with a safety margin (the deferred active-set update of Sec. 2.2).
 *
 * Conventions: SI units; 0-based indices; arrays are row-major
 * ([n][3] means n consecutive xyz triples).  Quaternions are (w, x, y, z),
 * body to world.  Angular velocity is in the clump's principal body frame.
 * Clump c owns consecutive sphere ids in template order.
 */
#ifndef CDEM_H
#define CDEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CDEM_ABI_VERSION 3

/* ---- error codes ---- */
#define CDEM_OK 0
#define CDEM_E_INVALID (-1)        /* bad argument or descriptor (nothing changed) */
#define CDEM_E_OOM (-2)            /* device allocation failed */
#define CDEM_E_HIP (-3)            /* a HIP runtime call failed */
#define CDEM_E_CAPACITY (-4)       /* contact storage overflowed and could not be regrown */
#define CDEM_E_MISSED_CONTACT (-5) /* an audit found a contact missing from the active set */
#define CDEM_E_NAN (-6)            /* non-finite state detected */
#define CDEM_E_STATE (-7)          /* call not valid in the scene's current state */

/* ---- enums ---- */
#define CDEM_PREC_FP64 0       /* all force arithmetic in FP64 */
#define CDEM_PREC_FP32_FORCE 1 /* force arithmetic in FP32; penetration, normal,
                                  history, state and integration in FP64 */

#define CDEM_DETECT_PLAIN 0   /* detect every step, no margin (Sec. 2.2, traditional scheme) */
#define CDEM_DETECT_FIXED 1   /* detect every k steps, margin from the global maximum speed */
#define CDEM_DETECT_LEARNED 2 /* detect every k steps, per-region margins from the MLP envelope */

#define CDEM_BND_PLANE 0      /* p0[3], n[3]: plane, unit normal into the domain */
#define CDEM_BND_CYL_IN 1     /* p0[3], a[3], R: domain inside a cylinder */
#define CDEM_BND_CONE_OUT 2   /* apex[3], a[3], sin, cos, H: solid cone + shaft, domain outside */
#define CDEM_BND_FRUSTUM_IN 3 /* apex[3], a[3], sin, cos, t0, t1: funnel wall, domain inside */
#define CDEM_BND_NPARAM 12
#define CDEM_PRESC_NPARAM 12  /* v_fixed[3], free[3] (0/1), w_body[3], f_extra[3] */

#define CDEM_HOST 0
#define CDEM_DEVICE 1

typedef struct cdem_scene cdem_scene;

/* Scene description (the inputs of the model of Sec. 2.1: clumps of
 * spheres with a mass and principal inertia per clump and E, nu, mu, CoR per
 * sphere instance; the boundaries the contact geometry of Sec. 2.2 covers).
 * Borrowed for the duration of cdem_create only; every array is copied.
 * Pointers are host memory. */
typedef struct cdem_scene_desc {
    double h;                          /* time step [s], > 0 */
    int32_t precision;                 /* CDEM_PREC_* */
    int32_t n_templates;               /* >= 1 */
    const uint32_t *tmpl_sphere_begin; /* [n_templates+1] CSR into template spheres */
    const double *tmpl_offset;         /* [n_tmpl_spheres][3] body frame, about the CoM */
    const double *tmpl_radius;         /* [n_tmpl_spheres] > 0 */
    const double *tmpl_mass;           /* [n_templates] > 0 */
    const double *tmpl_inertia;        /* [n_templates][3] principal moments > 0 */
    int64_t n_clumps;
    const uint32_t *clump_template;    /* [n_clumps] */
    const uint32_t *clump_scene;       /* [n_clumps] < n_scenes */
    const double *x;                   /* [n_clumps][3] CoM position */
    const double *q;                   /* [n_clumps][4] unit quaternion */
    const double *v;                   /* [n_clumps][3] CoM velocity */
    const double *w;                   /* [n_clumps][3] angular velocity, body frame */
    const double *sphere_mat;          /* [n_spheres][4] E > 0, -1 < nu < 0.5, mu >= 0, 0 < CoR <= 1 */
    int32_t n_scenes;                  /* independent scenes sharing one launch (>= 1) */
    const double *gravity;             /* [n_scenes][3] */
    const double *domain;              /* [n_scenes][6] lo[3], hi[3]: binning box (spheres outside are
                                          still handled, in the edge bins) */
    int32_t n_bnd;                     /* <= 4096 (over all scenes) */
    const int32_t *bnd_type;           /* [n_bnd] CDEM_BND_* */
    const double *bnd_param;           /* [n_bnd][12] geometry at t = 0 */
    const double *bnd_mat;             /* [n_bnd][4] E, nu, mu, CoR */
    const double *bnd_vel;             /* [n_bnd][3] translation velocity (geometry moves) */
    const double *bnd_omega;           /* [n_bnd][3] surface spin about the reference point
                                          (geometry is taken as invariant under it) */
    const int32_t *bnd_scene;          /* [n_bnd] */
    int32_t n_presc;
    const int32_t *presc_clump;        /* [n_presc] prescribed-motion clumps */
    const double *presc_param;         /* [n_presc][12] */
    /* Triangle meshes: rigid boundaries whose motion the caller prescribes
     * (the paper's funnel, cone and wheels are meshes, Sec. 4; a multibody
     * solver drives them in co-simulation).  Each triangle is a boundary of
     * its mesh's scene: a sphere touches it when its centre is closer than
     * its radius to the triangle's closest point (two-sided, edges and
     * vertices included); the contact normal points from that point to the
     * centre; the mesh is flat and infinitely heavy there (Rbar = R,
     * mbar = the clump's mass).  Every step a mesh moves with its
     * velocities: x += h v, q += (h/2) (0, w) (x) q, renormalised. */
    int32_t n_mesh;                    /* <= 64 */
    const double *mesh_state;          /* [n_mesh][13] x[3] reference point, q[4] (mesh -> world, unit),
                                          v[3], w[3] angular velocity (world frame) */
    const double *mesh_mat;            /* [n_mesh][4] E, nu, mu, CoR */
    const int32_t *mesh_scene;         /* [n_mesh] */
    int64_t n_tri;                     /* n_spheres + n_bnd + n_tri < 2^31 */
    const int32_t *tri_mesh;           /* [n_tri] */
    const double *tri_vertex;          /* [n_tri][3][3] vertices in the mesh frame (about x) */
    /* Clump positions (a state representation beyond IEEE double, Sec. 3;
     * the data types of the work Sec. 1 builds on): 0 = FP64; E in [8, 60]
     * = fixed point, each CoM coordinate an integer k with x = k 2^-E (the
     * high 32 bits of k a voxel id, the low 32 bits the offset inside a voxel
     * of side 2^(32-E) m).  The vector between two spheres is then the exact
     * difference of their integers plus their rotated offsets, so its
     * accuracy does not depend on where the scene lies; lever arms are built
     * from rotated offsets; x += h v adds rint(h v 2^E).  Boundary and mesh
     * distances use world coordinates k 2^-E.  Initial CoMs and domains
     * must lie within 2^60 grid steps of the origin; a CoM leaving 2^61 steps
     * makes cdem_step fail with CDEM_E_NAN. */
    int32_t pos_exp;
} cdem_scene_desc;

/* Optional device allocator (e.g. a framework's caching allocator).  NULL
 * means stream-ordered hipMallocAsync / hipFreeAsync on the scene's stream.
 * alloc returns NULL on failure; every block the library takes is returned
 * through free before cdem_destroy returns. */
typedef struct cdem_allocator {
    void *ctx;
    void *(*alloc)(void *ctx, size_t bytes, void *stream);
    void (*free)(void *ctx, void *ptr, void *stream);
} cdem_allocator;

/* Active-set update policy (Sec. 2.2: the active set is rebuilt every step,
 * or every k steps with every contact geometry enlarged by a safety margin
 * set by the maximum velocity and the time step). */
typedef struct cdem_detect_params {
    int32_t mode;          /* CDEM_DETECT_* */
    int32_t k_max;         /* upper bound of the detection interval, 1..20 */
    double safety;         /* multiplier (>= 1) on velocity envelopes; default 1.5 */
    double v_max_user;     /* a-priori bound on sphere speed [m/s], 0 = use measured speeds */
    double margin_cap;     /* largest margin any sphere may get [m]; sets the bin size */
    int32_t audit_period;  /* steps between brute-force audits, 0 = never */
    int32_t overlap;       /* 1: detection overlapped with the dynamics (deferred modes only).  The
                              next active set is built on a second stream of the same device from a
                              snapshot of the state taken every k_max steps, while the steps go on
                              (Sec. 2.2: the active set is updated in the shadow of the dynamics),
                              and taken into use k_max steps later; its margins cover 2 k_max
                              steps.  A sphere that outruns them still trips the displacement
                              guard, which re-detects on the step's stream at once.  Results are
                              the same as with detection every step. */
} cdem_detect_params;

/* Counters of the scene (host copy of its device control block). */
typedef struct cdem_counts {
    int64_t clumps, spheres, bins;
    int64_t candidates;   /* entries in the active set (both directions of a pair count once each) */
    int64_t steps;        /* completed steps */
    int64_t detections;   /* active-set rebuilds */
    int64_t guard_trips;  /* rebuilds forced by a sphere outrunning its margin */
    int64_t fallbacks;    /* learned envelopes rejected for the fixed rule */
    int64_t audits;
    int64_t missed;       /* contacts found by audits but absent from the active set */
    int64_t capacity;     /* active-set entries that fit in the current storage */
    int64_t regrows;
    int64_t pairs;        /* distinct candidate pairs of the active set (sphere pairs + boundary pairs) */
    int32_t k_current;    /* current detection interval */
    int32_t reserved;
    int64_t audit_contacts; /* exact contacts the last binned audit found (sphere pairs once, boundary and
                               triangle contacts), the count cdem_audit reports for the same positions */
} cdem_counts;

/* Clump state view: each pointer may be NULL (skipped).  where = CDEM_HOST or
 * CDEM_DEVICE.  Row-major [n_clumps][3] / [n_clumps][4]. */
typedef struct cdem_state_view {
    double *x, *q, *v, *w;
} cdem_state_view;

/* Contacts of the last recorded step (see cdem_record_next_step), canonical:
 * sphere pairs a < b < n_spheres, boundary contacts b = n_spheres + index,
 * triangle contacts b = n_spheres + n_bnd + triangle index.
 * Only pairs whose exact predicate held that step (true contacts) are listed,
 * ascending by (a, b).  Host buffers of capacity 'cap' (any may be NULL);
 * *n receives the count (call with cap = 0 to size).  F is F_n + F_t of
 * Eq. normal_tangential_force_model1/2 acting on body b (minus it acts on
 * a); u the tangential history after the update and clamp of Eqs. updateUt
 * and cappingOfut; Ta and Tb the torques r x F that the contact exerts on a
 * and b, r from each body's reference point (a sphere's clump centre of
 * mass; a boundary's reference point, its first three parameters moved with
 * its translation) to the contact point of Eq. kinematicsContactInfo. */
typedef struct cdem_contacts_view {
    int64_t cap;
    int64_t n;
    uint32_t *a, *b;
    double *delta;   /* [cap] */
    double *F;       /* [cap][3] */
    double *u;       /* [cap][3] */
    double *Ta;      /* [cap][3] */
    double *Tb;      /* [cap][3] */
} cdem_contacts_view;

/* Result of an independent exact contact sweep (the enlarged geometry of
 * Sec. 2.2 must never miss a contact). */
typedef struct cdem_audit_result {
    int64_t true_contacts;  /* exact contacts found by the independent brute-force sweep */
    int64_t missed;         /* of those, absent from the active set */
    uint32_t first_a, first_b;
} cdem_audit_result;

/* ---- lifecycle ---- */
/* CDEM_ABI_VERSION of the built library. */
int cdem_abi_version(void);
/* Name of a CDEM_* return code (static string, never NULL). */
const char *cdem_strerror(int code);
/* Message of the scene's last failed call; with s = NULL, of the last failed
 * cdem_create.  Never NULL; valid until the next call on the scene. */
const char *cdem_last_error(const cdem_scene *s);

/* Build a scene of clumps of spheres (Sec. 2.1, clump paragraph and Fig.
 * "force": mass and inertia per clump, E, nu, mu, CoR per sphere): validate
 * and copy the description to the device (host pointers, borrowed for the
 * call).  alloc may be NULL; stream (a hipStream_t) may be NULL.  On error
 * *out is NULL, nothing is leaked and CDEM_E_INVALID / CDEM_E_OOM /
 * CDEM_E_HIP is returned. */
int cdem_create(const cdem_scene_desc *d, const cdem_allocator *alloc, void *stream, cdem_scene **out);
/* Wait for the scene's stream, free every device block, free the scene. */
int cdem_destroy(cdem_scene *s);

/* ---- stepping ---- */
/* Advance n >= 0 time steps of Sec. 2.1 / 2.2: the active set (rebuilt
 * when due), each active pair's penetration, kinematics (Eq.
 * kinematicsContactInfo) and force (Eqs. normal_tangential_force_model1/2,
 * updateUt, cappingOfut), the sums onto clumps and the Newton-Euler update
 * (Eq. newton_law_1/2).  Enqueued on stream (a hipStream_t; NULL = the
 * scene's stream, which it then becomes).  Synchronises once at the end to
 * check the device control block; an active set that overflowed its storage
 * is grown and the abandoned steps are run again, bit for bit as if it had
 * fitted.  CDEM_E_MISSED_CONTACT: a periodic audit found a contact outside
 * the active set (the steps still ran); CDEM_E_NAN: a clump state became
 * non-finite; CDEM_E_CAPACITY: the storage could not grow. */
int cdem_step(cdem_scene *s, int64_t n, void *stream);
/* Wait until the scene's stream has drained. */
int cdem_sync(cdem_scene *s);
/* Choose the active-set update policy of Sec. 2.2 (every step, or deferred
 * with an enlarged contact geometry, by the fixed rule or by the learned
 * envelopes).  Takes effect at the next step, which rebuilds the active set
 * (tangential history of surviving pairs is kept).  CDEM_E_INVALID for
 * out-of-range values; CDEM_E_STATE for the learned mode without MLP
 * parameters. */
int cdem_set_detection(cdem_scene *s, const cdem_detect_params *p);
/* When on != 0, the next step stores per-contact penetration, force and
 * torques (for cdem_read_contacts, cdem_read_clump_forces,
 * cdem_read_boundary_forces and cdem_read_mesh_forces); allocates the
 * recording buffers on first use.  on = 1 records every contact; on = 2 only
 * the contacts with boundaries and mesh triangles (a co-simulation exchange:
 * the sphere pairs' records are not written, and cdem_read_contacts then
 * lists the boundary contacts only).  CDEM_E_INVALID for other values. */
int cdem_record_next_step(cdem_scene *s, int on);

/* Batched scenes (independent scenes in one launch, each with its own bins,
 * gravity and boundaries) as captured launch sequences.
 * Run steps as replays of a captured HIP graph of `steps_per_graph` steps
 * (0 = launch kernel by kernel).  Detection scheduling lives on the device, so
 * one captured sequence serves every step; the graph is re-captured whenever
 * the scene's launch parameters change (regrow, detection settings, tuning).
 * Results are identical either way. */
int cdem_set_graph(cdem_scene *s, int32_t steps_per_graph);

/* Autotuner: time `steps` steps for each candidate bin-size factor (bins of
 * 0.75, 1, 1.25, 1.5 or 1.75 times R_max + margin cap) and launch shape of
 * the grid-stride kernels, and keep the fastest.  The tuning steps are
 * ordinary steps of the simulation (results do not depend on the choice).
 * *bin_factor and *stride_cap (may be NULL) receive the choice. */
int cdem_autotune(cdem_scene *s, int32_t steps, double *bin_factor, int32_t *stride_cap);

/* ---- reads and writes (synchronous) ---- */
/* Counters of the scene's control block (waits for the scene's stream). */
int cdem_get_counts(cdem_scene *s, cdem_counts *c);
/* Clump state (the unknowns of Eq. newton_law_1/2: CoM position and
 * velocity, orientation, body-frame angular velocity) into the caller's
 * buffers, host (where = CDEM_HOST) or device (CDEM_DEVICE).  Runs on
 * stream (NULL = the scene's stream) after the work queued there, and
 * returns once the copy is complete. */
int cdem_read_state(cdem_scene *s, const cdem_state_view *v, int where, void *stream);
/* Overwrite the clump state from the caller's buffers (host or device, on
 * stream as above; host quaternions must be unit and values finite, else
 * CDEM_E_INVALID and nothing changes).  The active set is rebuilt before the
 * next step; tangential history of pairs that survive is kept (Eq.
 * updateUt: the history lives as long as the contact). */
int cdem_write_state(cdem_scene *s, const cdem_state_view *v, int where, void *stream);
/* Per-contact data of the last recorded step (see cdem_contacts_view).
 * CDEM_E_STATE when no step was recorded. */
int cdem_read_contacts(cdem_scene *s, cdem_contacts_view *v);
/* Per-clump force (contacts + gravity: the right-hand side of Eq.
 * newton_law_1) and torque (the sum of r x (F_n + F_t) over the clump's
 * contacts; Eq. newton_law_2 keeps r x F_t only, which is exact for one
 * sphere but not for a clump whose contact points lie off its centre of
 * mass) of the last recorded step, host buffers [n_clumps][3]. */
int cdem_read_clump_forces(cdem_scene *s, double *F, double *T);
/* Per-boundary force (what the spheres exert on it: the sum of minus the
 * contact forces on its spheres) and torque about its reference point (its
 * first three parameters, moved with its translation) at the last recorded
 * step: the readout a co-simulation takes from the granular side (Sec. 2.2,
 * co-simulation with a multibody solver).  Host buffers [n_bnd][3] in the
 * description's boundary order.  The sum runs in a fixed order:
 * reproducible, equal to an ascending sum up to rounding. */
int cdem_read_boundary_forces(cdem_scene *s, double *F, double *T);
/* Sphere centres x_c + A(q) o_s of the current state (the clump
 * representation of Sec. 2.1), host buffer [n_spheres][3]. */
int cdem_read_sphere_pos(cdem_scene *s, double *xs);

/* ---- triangle meshes (co-simulation: the caller moves a mesh, the scene
 * reports the force the spheres exert on it; Sec. 5.2 couples the granular
 * side and a multibody solver this way, one exchange every few steps) ---- */
/* Prescribe mesh `mesh`'s state (13 doubles as in cdem_scene_desc.mesh_state,
 * host pointer; unit quaternion, finite values, else CDEM_E_INVALID).  A
 * mesh's candidate margin covers 1.25 times its speed bound |v| + |w| r_max
 * (r_max: its farthest vertex from the reference point) over the steps an
 * active set is used.  New velocities that bound stays under, at an
 * unchanged pose (x and q bit for bit as cdem_read_mesh_state returns them),
 * keep the active set; a new pose or a faster motion resizes the margin and
 * makes the next step detect again. */
int cdem_set_mesh_state(cdem_scene *s, int32_t mesh, const double *state);
/* Current mesh states, host buffer [n_mesh][13]. */
int cdem_read_mesh_state(cdem_scene *s, double *state);
/* Force the spheres exert on each mesh (minus the sum of its contact forces)
 * and its torque about the mesh's reference point at the last recorded step
 * (see cdem_record_next_step, either mode), host buffers [n_mesh][3], summed
 * in ascending contact order (the triangle contacts are gathered on the
 * device, then ordered and summed on the host).  CDEM_E_STATE when no step
 * was recorded. */
int cdem_read_mesh_forces(cdem_scene *s, double *F, double *T);

/* Independent exact contact sweep (no binning, no margin) over the current
 * state, compared with the active set: with the enlarged geometry of Sec.
 * 2.2 every true contact must be in it.  O(N^2): scenes of up to 400k
 * spheres (CDEM_E_INVALID beyond).  CDEM_E_MISSED_CONTACT when any is
 * missing (r still filled). */
int cdem_audit(cdem_scene *s, cdem_audit_result *r);

/* ---- checkpoints (the tangential history of Eq. updateUt is state: a
 * resumed run must carry it) ---- */
/* Serialise the scene's dynamic state into a host buffer: clump state, step
 * counter, detection schedule and settings, the active set with its FP64
 * tangential history, the MLP parameters and the tuned launch settings.
 * With cap = 0 only *len (the size needed) is set.  A scene created from the
 * same description that loads the blob continues bit for bit as the saved
 * scene would have (the restored active set is rebuilt, with its history,
 * before the next step; results do not depend on when a rebuild happens). */
int cdem_save(cdem_scene *s, void *buf, size_t cap, size_t *len);
/* Restore a blob written by cdem_save into a scene created from the same
 * description (checked through a fingerprint of the static description,
 * counts and precision: CDEM_E_INVALID otherwise).  The blob is borrowed. */
int cdem_load(cdem_scene *s, const void *buf, size_t len);

/* ---- learned detection interval: envelope MLP ---- */
/* The MLP maps features of an envelope region (a block of 2 x 2 x 2 bins of
 * the scene's grid: max sphere speed, max acceleration envelope, number of
 * spheres) to (log speed envelope, log acceleration envelope) over the next
 * detection interval; the margin of the region's spheres is
 * safety k h v_env + (k h)^2 a_env / 2, which enlarges the contact geometry
 * of the deferred active-set update (paper Sec. 2.2) per region instead of
 * with one global speed bound.  Parameters are float32, cdem_mlp_param_count() of
 * them: mu[3], sigma[3] (input standardisation of u = (log(f0 + 1e-6),
 * log(f1 + 1e-3), log(1 + f2))), W1[64][3], b1[64], W2[64][64], b2[64],
 * W3[2][64], b3[2]. */
int cdem_mlp_param_count(void);
/* Load MLP parameters (host pointer, n = cdem_mlp_param_count(), finite,
 * positive standardisation scales; CDEM_E_INVALID otherwise) into the scene. */
int cdem_set_mlp(cdem_scene *s, const float *params, int64_t n);
/* Forward pass of the envelope MLP.  Device pointers: params, features
 * [n][3] (raw), out [n][2].  Asynchronous on stream. */
int cdem_mlp_forward(const float *params, const float *features, float *out, int64_t n, void *stream);
/* Bytes of workspace cdem_mlp_backward needs for n samples. */
size_t cdem_mlp_workspace_bytes(int64_t n);
/* Gradient (device, cdem_mlp_param_count() floats) and loss (device, one float,
 * may be NULL) of the mean pinball loss with quantile tau in (0, 1) of the
 * MLP on features [n][3] against targets [n][2]; standardisation entries get
 * zero gradient.  Deterministic. */
int cdem_mlp_backward(const float *params, const float *features, const float *target, int64_t n, float tau,
                      float *grad, float *loss, void *workspace, void *stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight training loops, harnesses that forbid hipMalloc): the same
 * gradient and loss as cdem_mlp_backward, bit for bit, with the workgroup
 * partials held in a static device array of the library (about 9.3 MB per
 * device, kept until the process ends) instead of a caller workspace.  At
 * most CDEM_MLP_STATIC_MAX_SAMPLES samples (CDEM_E_INVALID beyond, nothing
 * launched); device pointers as in cdem_mlp_backward; asynchronous on stream.
 * Allocates nothing.  Every call on one device shares that array: calls that
 * overlap on one device (other streams, other threads) race, and must be
 * ordered by the caller. */
#define CDEM_MLP_STATIC_MAX_SAMPLES 16384
int cdem_mlp_backward_static(const float *params, const float *features, const float *target, int64_t n, float tau,
                             float *grad, float *loss, void *stream);
/* One Adam update (step t >= 1, bias-corrected) of params with grad; m and v
 * are the moment buffers (device, zero-initialised by the caller). */
int cdem_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t t, float lr, float beta1,
                  float beta2, float eps, void *stream);
/* Training data from the scene's own trajectory: capture the features of
 * every envelope region of the current state, advance `horizon` steps, and
 * label each occupied region with the largest speed and acceleration envelope
 * its spheres (as binned at capture) showed over those steps, as
 * (log(v + 1e-6), log(a + 1e-3)).  Host buffers features [cap][3],
 * labels [cap][2]; *n receives the number of occupied regions (call with
 * cap = 0 to size; the steps still run). */
int cdem_collect_envelopes(cdem_scene *s, int32_t horizon, float *features, float *labels, int64_t cap,
                           int64_t *n);

/* ---- user force law (the paper's extension point: the contact force model
 * is a user-replaceable function of the contact's kinematics, Sec. 2.2) ----
 * A force law is the source text of one HIP device function,
 *
 *   __device__ void cdem_user_law(const double *n, double delta,
 *       const double *vrel, double Rbar, double mbar, double estar,
 *       double gstar, double mu, double beta, double h,
 *       const double *u_old, double *F, double *u_new);
 *
 * (it may define helpers before it).  Called once per contact and step, in
 * FP64 in both precision modes, with the contact geometry of Eq.
 * kinematicsContactInfo: n[3] the unit normal from body a to body b (a
 * boundary is body a), delta > 0 the overlap, vrel[3] the velocity of b
 * relative to a at the contact point; Rbar and mbar the effective radius and
 * mass (clump masses; a boundary is flat and infinitely heavy); estar and
 * gstar the pair's effective Young's and shear moduli; mu and beta the
 * smaller friction coefficient and damping ratio ln e / sqrt(ln^2 e + pi^2)
 * of the two materials; h the time step; u_old[3] the pair's tangential
 * history (zero when the contact is new).  It writes F[3], the force on body b
 * (minus F acts on a, at the same contact point; torques follow from it),
 * and u_new[3], the history the pair carries to its next step (a pair that
 * leaves contact loses it).  The law is compiled at run time with hiprtc for
 * gfx950, with the library's floating-point flags (no contraction), into the
 * library's own pair kernel.
 *
 * Compile only (no device needed): CDEM_OK, or CDEM_E_INVALID with the
 * compiler's messages in log (a buffer of log_cap bytes, may be NULL). */
int cdem_check_force_law(const char *source, char *log, size_t log_cap);
/* Compile the law and make the scene's pair kernel use it from the next
 * step on (source NULL or "" restores the built-in Hertz-Mindlin law of Eqs.
 * normal_tangential_force_model1/2, updateUt and cappingOfut).
 * CDEM_E_INVALID (scene unchanged) when it does not compile, with the
 * compiler's messages in log; CDEM_E_HIP when the code object cannot be
 * loaded.  Waits for the scene's stream. */
int cdem_set_force_law(cdem_scene *s, const char *source, char *log, size_t log_cap);

/* ---- measurement (not part of the method; where Sec. 2.2 says the time
 * goes: identifying the active set) ---- */
/* Per-kernel device time, measured with HIP events recorded on the launch
 * stream around every kernel while profiling is on. */
typedef struct cdem_kernel_time {
    char name[32];
    int64_t launches;
    double total_ms;
} cdem_kernel_time;

/* on != 0 starts (and clears) per-kernel timing of every kernel; on == 0
 * stops it. */
int cdem_profile(cdem_scene *s, int on);
/* Starts (and clears) timing of the named kernels only (comma-separated
 * names as cdem_profile_read reports them; null or "" = every kernel), so
 * that the events around the other kernels do not slow the steps.  Unknown
 * names only: CDEM_E_INVALID, timing off. */
int cdem_profile_kernels(cdem_scene *s, const char *names);
/* Copies up to cap records into out (host), *n receives the number of
 * kernels timed so far (waits for the scene's stream). */
int cdem_profile_read(cdem_scene *s, cdem_kernel_time *out, int cap, int *n);
/* True contacts (exact predicate, positive overlap) of the last completed
 * step, counted once per pair side (twice per sphere pair, once per boundary
 * contact). */
int cdem_last_step_contacts(cdem_scene *s, int64_t *n);

#ifdef __cplusplus
}
#endif
#endif
