// Internal declarations of libcdem (HIP, gfx950).  Shared by the kernel
// translation unit and the host runtime; not part of the public ABI.
#pragma once

#ifndef __HIPCC_RTC__  // (the run-time compiler provides the HIP device environment itself)
#include <hip/hip_runtime.h>
#endif
#include <stdint.h>

namespace cdem {

constexpr int kMaxBnd = 4096;
constexpr int kMaxMesh = 64;
constexpr int kNarrowBlock = 512;  // narrow-phase workgroup: eight wavefronts share one segment allocation
constexpr int kMaxRow = 16;        // candidates the narrow phase sorts in LDS per sphere (more: k_narrow_over)
// Workgroup cap of the binning, bin-scan, segment-writing and audit kernels,
// which loop over logical blocks: most steps launch them with nothing to do, and a
// capped grid returns in a few microseconds where one workgroup per block
// took ~30-50.  (The narrow phase's first pass keeps one workgroup per block:
// looped, it needs more registers, and its detections took half as long
// again.)
constexpr int kStepGrid = 8192;
// Workgroups (of one wavefront) of the narrow phase's exact pass over the
// spheres its first pass leaves: few spheres, so a small grid whose launch
// on a step without detection costs next to nothing.
constexpr int kFbGrid = 512;
constexpr int kBigClump = 64;      // clumps with more spheres reduce through a workgroup
constexpr int kRegionBins = 2;     // edge of an envelope region of the learned margins, in bins

// Analytic boundary as the kernels see it (geometry at t = 0 plus motion).
struct Bnd {
    int32_t type, scene;
    double p[12];
    double vel[3], omg[3];
    double e, g, mu, beta;   // (1-nu^2)/E, 2(2-nu)(1+nu)/E, mu, damping ratio of CoR
    float ef, gf, muf, betaf;
    double margin;           // extra candidate margin covering the boundary's own motion
};

// A triangle mesh as the kernels see it: a rigid boundary with prescribed
// motion (its state advances every step) and a material.  Its triangles are
// boundary partners ns + n_bnd + k of the spheres.
struct Mesh {
    double x[3], q[4], v[3], w[3];   // reference point, orientation (mesh -> world), velocity, world angular velocity
    double e, g, mu, beta;           // (1-nu^2)/E, 2(2-nu)(1+nu)/E, mu, damping ratio of CoR
    float ef, gf, muf, betaf;
    double margin;                   // extra candidate margin covering the mesh's own motion
    double rmax;                     // largest distance of a vertex from the reference point
    int32_t scene, pad;
};

// Per-scene uniform grid (scenes never share a bin, so no pair crosses scenes).
struct Grid {
    double ox, oy, oz;       // lower corner
    double inv;              // 1 / bin size
    int32_t nx, ny, nz, sid;  // bins per axis; the scene's index
    int64_t cell0;           // first global bin id of the scene
    int32_t bnd_beg, bnd_end;   // the scene's analytic boundaries
    int32_t tri_beg, tri_end;   // the scene's mesh triangles
    int32_t chunk_beg, chunk_end;  // ... in chunks of at most 64 (chunks never span two scenes)
    double gx, gy, gz;       // gravity
    float pre_eps;           // slack of the FP32 prefilter: bounds its rounding of positions relative to (ox, oy, oz)
    float pre_lim;           // beyond this distance from the origin a sphere skips the prefilter
    double b;                // bin size
    double rm_max;           // largest radius + the margin cap (bounds the partner side of any reach)
    double r_max;            // largest radius (the partner side of the audit's reach)
    int32_t rnx, rny, rnz, rpad;  // envelope regions: blocks of kRegionBins^3 bins
    int64_t reg0;            // first global region id of the scene
};

// Device-resident control block: decides on the device whether a detection
// runs this step, so that a captured sequence of launches stays static.
struct Ctl {
    int64_t step;            // completed steps
    int64_t n_up;            // upper-segment entries written by the detection in progress
    int64_t n_up_cur;        // upper-segment entries of the active set in use
    int64_t detections, guard_trips, fallbacks, audits, missed;
    int32_t buf;             // which of the three active-set structure slots is in use
    int32_t det_due;         // a detection runs at the start of this step
    int32_t since_det;       // steps completed since the last detection
    int32_t k_cur;           // current detection interval
    int32_t overflow;        // active-set storage overflowed: later kernels of the step skip
    int32_t row_overflow;    // more spheres exceeded kMaxRow candidates than the overflow list holds
    int32_t guard;           // a clump may have moved past its margin: re-detect
    int32_t record;          // store per-contact data this step (1 every contact, 2 boundary contacts)
    int32_t nonfinite;       // a clump state became NaN/Inf
    int32_t n_over;          // spheres of this detection with more than kMaxRow candidates
    uint32_t m_max_bits;     // largest margin any sphere takes at the detection in progress (float bits, >= 0)
    int32_t n_fb;            // spheres of this detection whose candidates k_narrow_fb finds
    int64_t n_afb;           // spheres of the audit in progress whose sphere partners k_audit_fb checks
    int64_t n_pairs;         // pairs of the detection in progress
    int64_t n_pairs_cur;     // pairs of the active set in use
    int32_t asym;            // an entry had no mirror (never expected): the step is abandoned
    int32_t collecting;      // training-data capture in progress: accumulate horizon labels
    uint32_t vmax_bits;      // max sphere speed of the current state (float bits, >= 0), set by k_pose
    uint32_t amax_bits;      // max sphere acceleration estimate of the step in progress
    uint32_t amax_last;      // ... of the last completed step
    float margin_cur;        // margin of every sphere at the last detection (fixed rule)
    int64_t audit_true;      // exact contacts seen by the last binned audit (sphere pairs once)
    int64_t audit_last_missed;
    int64_t n_bp;            // boundary pairs written by the detection in progress
    int32_t guard_next;      // guard trips of the clumps integrated outside the wave reduction
    int32_t hb;              // which of the two history buffers holds the history of the set in use
    // interval rule of the learned envelopes: the modelled bytes per step
    int64_t contact_sides_last;  // contact sides of the last completed step (2 per sphere pair, 1 per boundary)
    double c_cal;                // measured / modelled false-positive pairs at the last detection (0: none yet)
    double dpred_last;           // modelled false-positive pairs per sphere of the set in use (0: none)
    int32_t ahead_dropped;       // a set built ahead overflowed its storage and was not adopted
    int32_t stale;               // (second stream) its set was outrun before its adoption: not adopted
    int32_t bslot;               // the structure slot reserved for the second stream's set (never buf);
                                 // in the second stream's block: the slot its detection writes
    int32_t rec_last;            // record mode of the last recorded step (1 all contacts, 2 walls only)
};

// Detection plan parameters (fixed rule), set by cdem_set_detection.
struct Plan {
    int32_t k_max;
    int32_t audit_period;
    float safety;
    float margin_cap;
    float margin_floor;
    float v_user;            // a-priori speed bound (0 = measured)
    int32_t test_zero_margin; // testing aid: margins forced to zero
    float r_mean;            // mean sphere radius (the false-positive model of the interval rule)
};

// Everything a step kernel needs, by value (kernel argument).
struct DevScene {
    int64_t nc, ns;
    int32_t n_scenes, n_bnd, precision, detect_mode;
    double h;
    int64_t n_cells;
    int64_t cap;                     // pairs (and upper-segment entries) per active-set buffer
    // Clump state: one 128-byte record per clump, four double4:
    // (x, M), (v, r_acc), (q), (w_body, r_ctr); M the mass, r_acc the largest
    // |o_s| + R_s and r_ctr the largest |o_s| of its spheres (static words
    // kept with the state so that one aligned record serves every reader).
    double4 *cst;                    // [nc][4]
    // clump static
    const double4 *tmpl_mi;          // [n_templates]: mass, principal moments of inertia
    const int64_t *sbeg;             // [nc+1]
    const int32_t *presc;            // [nc] -1 or index
    const double *presc_param;       // [n_presc][12]
    const uint32_t *clump_tmpl, *clump_scene;
    const uint32_t *tmpl_sbeg;
    const double *tmpl_ofs;          // [n_ts][3]
    const double *tmpl_rad;
    // sphere static
    const uint32_t *owner, *sscene;
    const double4 *mat64;            // (1-nu^2)/E, 2(2-nu)(1+nu)/E, mu, beta
    const float4 *mat32;
    // sphere dynamic
    double4 *spos;                   // (x, y, z, R), written by k_pose when a step needs positions
    float *smargin[3];               // margin each sphere took at the detection of the set in that slot
    double4 *cdet;                   // [nc][2] clump pose at the last detection: (x, 0), q
    double *sF, *sT;                 // [ns][3] per-sphere sums (big clumps only)
    // binning
    const Grid *grids;
    uint32_t *cell_of, *cell_count;
    uint32_t *cell_start;            // [n_cells + 1] exclusive scan of the counts, then the total
    uint32_t *scan_bsum;             // block sums of the bin-count scan
    uint32_t *cell_rank;             // [ns] each sphere's rank within its bin, taken when counting
    uint4 *sorted_meta;              // per slot of the bins: sphere id, clump, margin (float bits; 0 in the
                                     // audit's binning), 0
    double4 *sorted_pos;
    float4 *sorted_f4;               // FP32 prefilter record: position - grid origin, radius + margin
    uint32_t *stage;                 // [kMaxRow][ns] each sphere's candidates from the narrow phase's first pass
    uint2 *stage_n;                  // [ns] their count; how many lie below the sphere (low 16 bits) and are
                                     // boundaries (high 16); beyond kMaxRow candidates: count, how many below,
                                     // and the boundaries in the sphere's first entry
    unsigned long long *narrow_part; // [ceil(ns / kNarrowBlock)][3] per narrow-phase workgroup: its upper entries,
                                     // pairs and boundary pairs, then (scanned) their bases
    uint32_t *narrow_woff;           // [ceil(ns / kNarrowBlock)][kNarrowBlock / 64][2] each wavefront's upper
                                     // entries and pairs below it in its workgroup
    // Active set, pair-major.  Each candidate pair is stored once, in the
    // "lower segment" of its lower-id sphere (partners above that id,
    // ascending, boundaries last), with its tangential history; the higher
    // sphere lists the pair in its "upper segment" (partners below its id,
    // ascending) through a link to the pair.  The structure comes in three
    // slots: the set in use (ctl->buf), the one a detection on the step's
    // stream builds (the third slot besides the one in use and ctl->bslot),
    // and ctl->bslot, which a detection running ahead on a second stream
    // builds while the steps go on (overlap mode; unused otherwise).  The
    // tangential history comes in two buffers (ctl->hb holds the set in
    // use's): a detection carries it from the set in use into the other
    // buffer, laid out for the new set.
    uint32_t *lo_beg[3], *lo_cnt[3];  // [ns] each sphere's lower segment in the pair arrays
    uint32_t *pt[3];                  // [cap] partner of the pair: sphere id, or ns + boundary
    double *hist[2];                  // [cap][3]
    uint32_t *ps[3];                  // [cap] the pair's lower sphere
    void *cS, *cTs, *cTt;             // [cap] per pair this step: force on the lower sphere (float4 / double4,
                                      // w: 1 if in contact), torque on the lower sphere and on the partner sphere
                                      // (three floats / doubles, packed)
    uint32_t *up_beg[3], *up_cnt[3];  // [ns] each sphere's upper segment
    uint32_t *ut[3], *us[3], *um[3];  // [cap] upper entries: partner (lower id), own sphere, linked pair
    // per-workgroup partial results, reduced by the next single-workgroup kernel
    // (device-wide same-address atomics serialise; these do not)
    uint32_t *part_r;                 // [n_rblocks + 256][3] reduction: max acceleration, max speed, guard trip
    int64_t n_rblocks;
    unsigned long long *part_a;       // [n_ablocks][2] audit: true contacts, missed
    uint32_t *part_c;                 // [pair_blocks] contact sides counted by each workgroup of k_pairs
    double *part_k;                   // [2][region-kernel workgroups] sums of the interval rule's margin model
    int64_t n_ablocks;
    uint32_t *over_list;             // [over_cap] spheres whose rows k_narrow_over fills
    uint32_t *fb_list;               // [ns] spheres whose candidates k_narrow_fb finds (FP64 scan)
    int64_t over_cap;
    // recording
    uint8_t *rec_state;              // per pair of the recorded step
    double *rec_delta, *rec_F;       // [cap], [cap][3] (F: on the partner body b)
    double *rec_R;                   // [cap][3] boundary pairs: contact point relative to the boundary's reference point
    double *rec_Ta, *rec_Tb;         // [cap][3] torque on body a / body b about its reference point
    double *rec_cF, *rec_cT;         // [nc][3]
    const Bnd *bnd;
    // fixed-point clump positions: 0, or E with x = k 2^-E (pos_eps = 2^-E)
    int32_t pos_exp, pad_p;
    double pos_eps, pos_inv;          // 2^-E, 2^E
    // triangle meshes
    int32_t n_mesh, pad_m;
    int64_t n_tri;
    Mesh *mesh;                       // [n_mesh], state advanced by k_step_end
    const double *tri_vb;             // [n_tri][9] vertices in the mesh frame
    const int32_t *tri_mesh;          // [n_tri]
    int64_t n_chunk;
    const int32_t *chunk_tri;         // [n_chunk + 1] first triangle of each chunk
    // world boxes (lo[3], hi[3]) at the last detection: [n_tri] triangles,
    // then [n_chunk] chunks and [n_scenes] scenes, those two grown by the
    // margins of their meshes
    double *tri_box;
    Ctl *ctl;
    // big clumps
    const int32_t *big_list;         // clump ids
    const int64_t *big_sbeg;         // [n_big+1] first sphere of each big clump in bdet
    double4 *bdet;                   // sphere poses of the big clumps at the last detection
    int32_t n_big;
    int32_t guard_on;                // the displacement guard is checked (deferred detection)
    int32_t guard_exact;             // testing aid: every clump takes the per-sphere guard test
    Plan plan;
    // learned envelopes and training-data collection
    int32_t store_speed;             // k_pose writes each sphere's speed to sspeed
    int32_t store_acc;               // integration writes each clump's acceleration envelope to cacc
    float *sspeed;                   // [ns]
    float *cacc;                     // [nc]
    int64_t n_regions;               // envelope regions (learned margins), over all scenes
    uint32_t *bin_v, *bin_a;         // [n_regions] max speed / acceleration in the region (float bits)
    uint32_t *reg_occ;               // [n_regions] spheres in the region
    float *bin_margin;               // [n_regions] margin of the region's spheres this detection
    const float *mlp;                // envelope MLP parameters (device), null if none loaded
    uint32_t *cell_t, *occ_t;        // collection: regions of the spheres and region occupancy at capture
    uint32_t *lab_v, *lab_a;         // collection: max speed / acceleration over the horizon (float bits)
    // wave schedule of the reduction: wave w covers spheres wave_s[2w] ..
    // wave_s[2w+1]-1 (whole clumps, at most 64 spheres; big clumps excluded)
    const int32_t *wave_s;
    const uint32_t *wave_c;          // [n_waves] first clump of each wave
    const uint32_t *sinfo;           // [ns] index of the sphere in its clump | clump size << 8 (clumps of <= 64)
    const uint32_t *sts;             // [ns] template sphere of each sphere
    int64_t n_waves;
    // launch shape of the grid-stride kernels (tunable; results do not depend on it)
    int32_t stride_cap;              // maximum workgroups of k_pairs / k_link / k_bin_margin
    // detection overlapped with the dynamics (a second stream builds the next
    // active set from a snapshot of the state while the steps go on)
    int32_t overlap;                 // on: detections are scheduled by the host (the device re-detects on a guard trip)
    int32_t bchain;                  // this launch belongs to the second stream's detection
    int32_t horizon;                 // steps the margins of a second-stream detection cover
    int32_t pad3;
};

// Workgroups of the grid-stride kernels over the active set (k_pairs, k_link):
// enough for every slot of the storage, at most the tuned stride cap.
constexpr int kPairBlocksMax = 16384;
__host__ __device__ inline unsigned pair_blocks(int64_t cap, int32_t stride_cap) {
    const int64_t c = stride_cap > 0 && stride_cap < kPairBlocksMax ? stride_cap : kPairBlocksMax;
    int64_t n = (cap + 255) / 256;
    n = n < c ? n : c;
    return (unsigned)(n > 1 ? n : 1);
}
// Workgroups of the kernels over the envelope regions.
constexpr int kRegionBlocksMax = 16384;
__host__ __device__ inline unsigned region_blocks(int64_t n_regions) {
    int64_t n = (n_regions + 255) / 256;
    n = n < kRegionBlocksMax ? n : kRegionBlocksMax;
    return (unsigned)(n > 1 ? n : 1);
}

#ifndef __HIPCC_RTC__  // host side of the library only
// Optional per-kernel timing: when non-null, launchers bracket every kernel
// with events taken from the pool and note which kernel each pair belongs to.
struct KernelTimer {
    virtual void before(int kernel_id, hipStream_t st) = 0;
    virtual void after(int kernel_id, hipStream_t st) = 0;
    virtual ~KernelTimer() {}
};
enum KernelId { K_POSE, K_DETECT_BEGIN, K_CELL_COUNT, K_SCAN_REDUCE, K_SCAN_BSUM, K_SCAN_FINAL, K_CELL_SCATTER,
                K_NARROW, K_DETECT_END, K_FORCE, K_FORCE_BIG, K_INTEGRATE_BIG, K_STEP_END, K_PLAN, K_AUDIT,
                K_LINK, K_REDUCE, K_BIN_FEATURES, K_BIN_MARGIN, K_NARROW_OVER, K_REGION_MARGIN, K_GUARD_BIG, K_BINS_BEGIN,
                K_AUDIT_ALL, K_PICK_INTERVAL, K_NARROW_ROWS, K_NARROW_BASE, K_CARRY, K_NARROW_FB, K_COUNT };
extern const char *const kKernelNames[K_COUNT];
extern KernelTimer *g_timer;

// Launchers (kernels.hip).  Every launcher enqueues on `st` and returns the
// hipError_t of the launch.
// Sphere poses (spos) and, where the settings ask, speeds.  In a step
// (force = false) the kernel works only when the step needs positions (a
// detection, an audit, training-data capture); readouts pass force = true.
hipError_t launch_pose(const DevScene &S, hipStream_t st, bool force);
hipError_t launch_detect(const DevScene &S, hipStream_t st);
// Detection ahead (overlap mode): snapshot on the step's stream (S), the
// detection chain on the second stream (B: the second stream's view), and
// the adoption of its set on the step's stream.
hipError_t launch_snapshot(const DevScene &S, const DevScene &B, hipStream_t st);
hipError_t launch_detect_ahead(const DevScene &B, hipStream_t st);
hipError_t launch_adopt(const DevScene &S, const DevScene &B, hipStream_t st);
// user_pairs: the pair kernel of a user force law compiled at run time (its
// DevScene argument by value, 256 lanes per workgroup), or null for the
// built-in law.
hipError_t launch_force_integrate(const DevScene &S, hipStream_t st, hipFunction_t user_pairs);
hipError_t launch_step_end(const DevScene &S, hipStream_t st);
hipError_t launch_audit_brute(const DevScene &S, unsigned long long *counts, uint32_t *first, hipStream_t st);
// Periodic binned exact audit (every plan.audit_period steps, decided on the device).
hipError_t launch_audit_binned(const DevScene &S, hipStream_t st);
// Training-data capture: bin features of the current state, then per-step labels.
hipError_t launch_collect_begin(const DevScene &S, hipStream_t st);
hipError_t launch_collect_speed(const DevScene &S, hipStream_t st);
hipError_t launch_collect_acc(const DevScene &S, hipStream_t st);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t st);
// Contact sides of the last evaluated step: one partial per workgroup into part[nblk].
hipError_t launch_count_contacts(const DevScene &S, unsigned long long *part, int nblk, hipStream_t st);
// Force and torque on every boundary from the recorded step: partial [n_bnd][kBndParts][6], out [n_bnd][6].
constexpr int kBndParts = 64;
hipError_t launch_bnd_forces(const DevScene &S, double *partial, double *out, hipStream_t st);
#endif  // __HIPCC_RTC__

}  // namespace cdem
