// HIP kernels of the clumped-sphere DEM step (gfx950, wave64).
//
// One step (paper Sec. 2.1 / 2.2), launched as a static sequence whose work
// the device-resident control block switches on and off:
//   k_bins_begin, k_pose  sphere centres x_s = x_c + A(q) o_s from each
//                    clump's state record (multi-sphere clumps, Sec. 2.1),
//                    only on steps that detect or audit; the same pass
//                    counts spheres into per-scene uniform bins and gathers
//                    the learned envelopes' region features;
//   detection        (when due: every step, or every k steps with the
//                    enlarged contact geometry of Sec. 2.2) scan of the bin
//                    counts, scatter into bin order, k_narrow (one thread
//                    per sphere): FP32 prefilter over the bins in reach,
//                    exact FP64 predicate (boundary partners: analytic
//                    boundaries, and mesh triangles through the boxes of
//                    k_tri_boxes / k_tri_scene_boxes), candidates sorted by
//                    partner id in LDS and staged per sphere (k_narrow_fb
//                    takes the rare sphere with more than 16 prefilter
//                    hits through one exact FP64 pass);
//                    k_narrow_base scans the workgroups' counts into
//                    segment bases (no atomics), k_narrow_rows writes the
//                    segments, k_link points each higher sphere's entry at
//                    its pair, k_carry carries the tangential history over
//                    from the current active set;
//   k_pairs          every candidate pair once, one lane per pair: exact
//                    predicate, kinematics of Eq. kinematicsContactInfo and
//                    the Hertz-Mindlin law of Eqs. normal_tangential_force_model1/2,
//                    updateUt and cappingOfut; the force and both torques go
//                    to per-pair contribution slots;
//   k_reduce_waves   one lane per sphere: its contributions in ascending
//                    partner id, then per clump its spheres in ascending id,
//                    + M g, symplectic Euler of Eq. newton_law_1/2 with the
//                    gyroscopic term, and the displacement guard of
//                    deferred detection (clumps of more than 64 spheres
//                    through k_reduce_big_spheres / k_integrate_big /
//                    k_guard_big);
//   k_step_end       folds the per-workgroup partials, moves the meshes and
//                    schedules the next detection and audit (k_audit_cells:
//                    exact binned check that every contact is in the active
//                    set).
// With a second stream (k_snap, k_adopt_*) the next active set is built from
// a snapshot while the steps go on.  The pair, narrow-phase and audit kernels
// are instantiated per force precision, kind of positions (FP64 or fixed
// point) and presence of triangles.
//
// No atomic touches a floating-point result and every sum runs in a fixed
// order, so the step is deterministic.  Compiled with -ffp-contract=off: the
// FP64 path performs exactly the IEEE operations written, in the order
// written.
#include "cdem_internal.h"
#include "mlp_dev.h"
#include "pair_dev.h"
#include "step_dev.h"

#include <math.h>

namespace cdem {

// Raise a device-wide float maximum kept as bits in the control block.  The
// current value is read at device scope first (a plain load may see a stale
// per-XCD L2 copy), so the atomic is issued only by the few values that
// still raise it.
__device__ __forceinline__ void raise_max(uint32_t *slot, float v) {
    if (!(v > 0.0f)) return;
    const uint32_t cur = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (v > __uint_as_float(cur)) atomicMax(slot, __float_as_uint(v));
}

// Positions need refreshing at the start of a step that detects, audits or
// captures training data; the other steps never read them.
__device__ __forceinline__ bool due(const Ctl *c) { return (c->det_due | c->guard) != 0; }
__device__ __forceinline__ bool audit_due(const DevScene &S) {
    return S.plan.audit_period > 0 && (S.ctl->step % S.plan.audit_period) == 0;
}

// ---------------------------------------------------------------- binning
__device__ __forceinline__ void cell_coords(const Grid &g, double x, double y, double z, int &ix, int &iy, int &iz) {
    double fx = floor((x - g.ox) * g.inv), fy = floor((y - g.oy) * g.inv), fz = floor((z - g.oz) * g.inv);
    fx = fmin(fmax(fx, 0.0), (double)(g.nx - 1));
    fy = fmin(fmax(fy, 0.0), (double)(g.ny - 1));
    fz = fmin(fmax(fz, 0.0), (double)(g.nz - 1));
    ix = (int)fx; iy = (int)fy; iz = (int)fz;
}

// Visit the sorted-slot ranges of every bin row that a ball of radius `reach`
// around (px, py, pz) touches: rows (iz, iy) within reach, and in each row the
// contiguous x-range of bins the ball's section covers.  Edge bins extend to
// infinity (positions outside the domain are clamped into them), so spheres
// outside the domain are still found.  f(jb, je) receives each slot range.
__device__ __forceinline__ double slab_gap(double p, double o, double b, int i, int n) {
    double lo = (i == 0) ? -1e300 : o + (double)i * b;
    double hi = (i == n - 1) ? 1e300 : o + (double)(i + 1) * b;
    return p < lo ? lo - p : (p > hi ? p - hi : 0.0);
}

__device__ __forceinline__ int clamp_cell(double v, int n) {
    v = floor(v);
    v = fmin(fmax(v, 0.0), (double)(n - 1));
    return (int)v;
}

template <typename F>
__device__ __forceinline__ void scan_reach(const DevScene &S, const Grid &g, double px, double py, double pz,
                                           double reach, F &&f) {
    int z0 = clamp_cell((pz - reach - g.oz) * g.inv, g.nz), z1 = clamp_cell((pz + reach - g.oz) * g.inv, g.nz);
    int y0 = clamp_cell((py - reach - g.oy) * g.inv, g.ny), y1 = clamp_cell((py + reach - g.oy) * g.inv, g.ny);
    double r2 = reach * reach;
    for (int zz = z0; zz <= z1; zz++) {
        double gz = slab_gap(pz, g.oz, g.b, zz, g.nz);
        double rz = r2 - gz * gz;
        if (rz < 0.0) continue;
        for (int yy = y0; yy <= y1; yy++) {
            double gy = slab_gap(py, g.oy, g.b, yy, g.ny);
            double ry = rz - gy * gy;
            if (ry < 0.0) continue;
            double rx = sqrt(ry);
            int x0 = clamp_cell((px - rx - g.ox) * g.inv, g.nx), x1 = clamp_cell((px + rx - g.ox) * g.inv, g.nx);
            int64_t rowc = g.cell0 + ((int64_t)zz * g.ny + yy) * g.nx;
            uint32_t jb = S.cell_start[rowc + x0];
            uint32_t je = S.cell_start[rowc + x1 + 1];
            f(jb, je);
        }
    }
}

// The same visit in FP32, on positions relative to the grid origin, for the
// FP32 prefilter passes: the caller widens the reach by twice the prefilter
// slack, which bounds the rounding of every quantity here, so the rows and
// x-ranges visited include all those of the FP64 visit (a few more at most).
__device__ __forceinline__ float slab_gap32(float p, float b, int i, int n) {
    const float lo = (i == 0) ? -3.0e38f : (float)i * b;
    const float hi = (i == n - 1) ? 3.0e38f : (float)(i + 1) * b;
    return p < lo ? lo - p : (p > hi ? p - hi : 0.0f);
}
__device__ __forceinline__ int clamp_cell32(float v, int n) {
    v = floorf(v);
    v = fminf(fmaxf(v, 0.0f), (float)(n - 1));
    return (int)v;
}

// The rows are visited one behind the loads: the bin range of the next row
// in reach is requested before the current row's records are visited, so
// that each row waits for one load (its records) instead of two (its bin
// range, then its records).
template <typename F>
__device__ __forceinline__ void scan_reach32(const DevScene &S, const Grid &g, float px, float py, float pz,
                                             float reach, F &&f) {
    const float inv = (float)g.inv, b = (float)g.b;
    const int z0 = clamp_cell32((pz - reach) * inv, g.nz), z1 = clamp_cell32((pz + reach) * inv, g.nz);
    const int y0 = clamp_cell32((py - reach) * inv, g.ny), y1 = clamp_cell32((py + reach) * inv, g.ny);
    const float r2 = reach * reach;
    int zz = z0, yy = y0 - 1;
    // the next row in reach after (zz, yy), with its bin range; false when none is left
    auto advance = [&](uint32_t &jb, uint32_t &je) {
        for (;;) {
            if (++yy > y1) { yy = y0; if (++zz > z1) return false; }
            const float gz = slab_gap32(pz, b, zz, g.nz);
            const float rz = r2 - gz * gz;
            if (rz < 0.0f) { yy = y1; continue; }  // the whole slab is out of reach
            const float gy = slab_gap32(py, b, yy, g.ny);
            const float ry = rz - gy * gy;
            if (ry < 0.0f) continue;
            const float rx = sqrtf(ry);
            const int x0 = clamp_cell32((px - rx) * inv, g.nx), x1 = clamp_cell32((px + rx) * inv, g.nx);
            const int64_t rowc = g.cell0 + ((int64_t)zz * g.ny + yy) * g.nx;
            jb = S.cell_start[rowc + x0];
            je = S.cell_start[rowc + x1 + 1];  // the next bin's start
            return true;
        }
    };
    uint32_t jb, je, nb = 0, ne = 0;
    bool more = advance(jb, je);
    while (more) {
        more = advance(nb, ne);
        f(jb, je);
        jb = nb; je = ne;
    }
}

// Envelope region (block of kRegionBins^3 bins of the scene's grid) of a bin.
__device__ __forceinline__ int64_t region_of(const Grid &g, uint32_t cell) {
    // a scene holds at most 2^27 bins: 32-bit division suffices
    uint32_t r = (uint32_t)((int64_t)cell - g.cell0);
    uint32_t ix = r % (uint32_t)g.nx, t = r / (uint32_t)g.nx;
    uint32_t iy = t % (uint32_t)g.ny, iz = t / (uint32_t)g.ny;
    return g.reg0 + ix / kRegionBins + (int64_t)g.rnx * (iy / kRegionBins + (int64_t)g.rny * (iz / kRegionBins));
}


// which = 0: the detection chain; which = 1: the periodic audit's own binning
// which = 2: training-data capture (always runs when launched)
// (on a step that also detects, the audit uses the detection's bins: the
// sorted records then carry the margins, which only widens its prefilter)
__device__ __forceinline__ bool chain_active(const DevScene &S, int which) {
    if (which == 2) return true;
    if (aborted(S.ctl)) return false;  // the step is abandoned until the active set has grown
    return which ? audit_due(S) && S.ctl->since_det != 0 : due(S.ctl);
}

// Start of a step that bins the spheres (a detection or an audit): clear the
// bin counters, the region features of the learned margins and the step's
// detection or audit counters.  k_pose then counts the spheres into the bins.
__global__ void __launch_bounds__(256) k_bins_begin(DevScene S) {
    if (aborted(S.ctl)) return;
    const bool det = due(S.ctl), aud = audit_due(S);
    if (!(det || aud)) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = i; k < S.n_cells; k += stride) {
        S.cell_count[k] = 0;
    }
    if (det && S.detect_mode == 2)
        for (int64_t k = i; k < S.n_regions; k += stride) { S.bin_v[k] = 0; S.bin_a[k] = 0; S.reg_occ[k] = 0; }
    if (i == 0 && det) {
        S.ctl->n_up = 0; S.ctl->n_pairs = 0; S.ctl->n_bp = 0; S.ctl->row_overflow = 0; S.ctl->asym = 0;
        S.ctl->n_over = 0; S.ctl->n_fb = 0;
    }
    if (i == 0 && aud) { S.ctl->audit_true = 0; S.ctl->audit_last_missed = 0; S.ctl->n_afb = 0; }
}

// Poses of the current state, one lane per sphere, and the speed of each
// sphere's centre |v_c + w x (x_s - x_c)| where the settings use it (learned
// envelopes and training data per sphere, the fixed rule's maximum).  On a
// step that bins the spheres the same pass finds each sphere's bin and counts
// it, and on a learned detection also collects the region features (maximum
// speed, maximum acceleration envelope of the spheres' clumps at the last
// step, sphere count): neighbouring spheres mostly share a region, so the
// lanes of a wavefront first combine runs of equal region and only each run's
// first lane updates it.
__global__ void __launch_bounds__(256) k_pose(DevScene S, int force) {
    const Ctl *ctl = S.ctl;
    const bool det = due(ctl), aud = audit_due(S);
    if (!force && (aborted(ctl) || !(det || aud || ctl->collecting))) return;
    const bool bin = !force && (det || aud);
    const bool feat = bin && det && S.detect_mode == 2;
    const int lane = threadIdx.x & 63;
    const bool speeds = S.store_speed || ctl->collecting || S.detect_mode != 0;
    float smax = 0.0f;  // this lane's largest sphere speed
    // logical blocks of 256 spheres, at most kStepGrid workgroups (a launch on
    // a step that neither detects nor audits returns at once)
    const int64_t nvb = (S.ns + 255) / 256;
    for (int64_t vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
        const int64_t s = vb * 256 + threadIdx.x;
        float speed = 0.0f, acc = 0.0f;
        int64_t r = -1;
        if (s < S.ns) {
            const uint32_t c = S.owner[s], ts = S.sts[s];
            const SphereKin k = sphere_kin_of(S, c, ts);
            S.spos[s] = make_double4(k.p[0], k.p[1], k.p[2], k.R);
            if (speeds) {
                const double r0 = k.p[0] - k.xc[0], r1 = k.p[1] - k.xc[1], r2 = k.p[2] - k.xc[2];
                const double u0 = k.v[0] + (k.W[1] * r2 - k.W[2] * r1), u1 = k.v[1] + (k.W[2] * r0 - k.W[0] * r2),
                             u2 = k.v[2] + (k.W[0] * r1 - k.W[1] * r0);
                speed = (float)sqrt(u0 * u0 + u1 * u1 + u2 * u2) * 1.000001f;
                if (S.store_speed || ctl->collecting) S.sspeed[s] = speed;
            }
            if (bin) {
                const Grid &g = S.grids[S.sscene[s]];
                int ix, iy, iz;
                cell_coords(g, k.p[0], k.p[1], k.p[2], ix, iy, iz);
                const uint32_t cell = (uint32_t)(g.cell0 + ((int64_t)iz * g.ny + iy) * g.nx + ix);
                S.cell_of[s] = cell;
                S.cell_rank[s] = atomicAdd(&S.cell_count[cell], 1u);
                if (feat) { r = region_of(g, cell); acc = S.cacc[c]; }
            }
        }
        if (feat) {
            float v = speed, a = acc;
            const int rl = (int)r, rh = (int)(r >> 32);
            const int pl = __shfl_up(rl, 1, 64), ph = __shfl_up(rh, 1, 64);
            const bool head = lane == 0 || pl != rl || ph != rh;
            const unsigned long long heads = __ballot(head);
            for (int off = 1; off < 64; off <<= 1) {  // run maxima, from the lanes further down the run
                const int ol = __shfl_down(rl, off, 64), oh = __shfl_down(rh, off, 64);
                const float ov = __shfl_down(v, off, 64), oa = __shfl_down(a, off, 64);
                if (lane + off < 64 && ol == rl && oh == rh) { v = fmaxf(v, ov); a = fmaxf(a, oa); }
            }
            if (head && r >= 0) {
                const unsigned long long later = lane < 63 ? heads >> (lane + 1) : 0ull;
                const int next = later ? lane + 1 + __builtin_ctzll(later) : 64;
                if (v > 0.f) atomicMax(&S.bin_v[r], __float_as_uint(v));
                if (a > 0.f) atomicMax(&S.bin_a[r], __float_as_uint(a));
                atomicAdd(&S.reg_occ[r], (uint32_t)(next - lane));
            }
        }
        smax = fmaxf(smax, speed);
    }
    if (S.detect_mode == 0) return;
    // the global speed maximum (the fixed rule, and the learned rule's
    // fallback): one filtered atomic per workgroup
    __shared__ float wmax[4];
    float speed = smax;
    for (int off = 32; off > 0; off >>= 1) speed = fmaxf(speed, __shfl_xor(speed, off, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = speed;
    __syncthreads();
    if (threadIdx.x == 0) raise_max(&S.ctl->vmax_bits, fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3])));
}

__global__ void __launch_bounds__(256) k_detect_begin(DevScene S, int which) {
    if (!chain_active(S, which)) return;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const bool bins = which == 2 || (which == 0 && S.detect_mode == 2);
    for (int64_t k = i; k < S.n_cells; k += stride) {
        S.cell_count[k] = 0;
    }
    if (bins)
        for (int64_t k = i; k < S.n_regions; k += stride) { S.bin_v[k] = 0; S.bin_a[k] = 0; S.reg_occ[k] = 0; }
    if (i == 0 && !which) {
        S.ctl->n_up = 0; S.ctl->n_pairs = 0; S.ctl->n_bp = 0; S.ctl->row_overflow = 0; S.ctl->asym = 0;
        S.ctl->n_over = 0; S.ctl->n_fb = 0;
    }
    if (i == 0 && which == 1) { S.ctl->audit_true = 0; S.ctl->audit_last_missed = 0; }
}

__global__ void __launch_bounds__(256) k_cell_count(DevScene S, int which) {
    if (!chain_active(S, which)) return;
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S.ns) return;
    double4 p = S.spos[s];
    const Grid &g = S.grids[S.sscene[s]];
    int ix, iy, iz;
    cell_coords(g, p.x, p.y, p.z, ix, iy, iz);
    uint32_t cell = (uint32_t)(g.cell0 + ((int64_t)iz * g.ny + iy) * g.nx + ix);
    S.cell_of[s] = cell;
    S.cell_rank[s] = atomicAdd(&S.cell_count[cell], 1u);
}

// Exclusive scan of cell_count -> cell_start in three passes (1024 bins per block).
constexpr int kScanBlock = 256, kScanItems = 4, kScanTile = kScanBlock * kScanItems;

__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *sh, uint32_t &total) {
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
        uint32_t add = t >= off ? sh[t - off] : 0u;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    total = sh[kScanBlock - 1];
    uint32_t incl = sh[t];
    __syncthreads();
    return incl - v;
}

// Both passes take the tiles of kScanTile bins on at most kStepGrid
// workgroups (a step that bins nothing returns at once).
__global__ void __launch_bounds__(kScanBlock) k_scan_reduce(DevScene S, uint32_t *bsum, int which) {
    if (!chain_active(S, which)) return;
    __shared__ uint32_t sh[kScanBlock];
    const int64_t ntile = (S.n_cells + kScanTile - 1) / kScanTile;
    for (int64_t b = blockIdx.x; b < ntile; b += gridDim.x) {  // block_excl_scan ends on a barrier
        const int64_t base = b * kScanTile + threadIdx.x * kScanItems;
        uint32_t v = 0;
        for (int k = 0; k < kScanItems; k++) if (base + k < S.n_cells) v += S.cell_count[base + k];
        uint32_t tot;
        block_excl_scan(v, sh, tot);
        if (threadIdx.x == 0) bsum[b] = tot;
    }
}

// Exclusive scan of the block sums in place: one workgroup of 1024 lanes,
// eight consecutive sums per lane per pass.
constexpr int kBsumBlock = 1024, kBsumItems = 8;
__global__ void __launch_bounds__(kBsumBlock) k_scan_bsum(DevScene S, uint32_t *bsum, int64_t nblk, int which) {
    if (!chain_active(S, which)) return;
    __shared__ uint32_t wt[kBsumBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t carry = 0;
    for (int64_t b0 = 0; b0 < nblk; b0 += (int64_t)kBsumBlock * kBsumItems) {
        const int64_t i0 = b0 + (int64_t)threadIdx.x * kBsumItems;
        uint32_t loc[kBsumItems], v = 0;
        for (int k = 0; k < kBsumItems; k++) {
            loc[k] = i0 + k < nblk ? bsum[i0 + k] : 0u;
            v += loc[k];
        }
        uint32_t x = v;  // inclusive wave scan
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane == 63) wt[wid] = x;
        __syncthreads();
        uint32_t below = 0, tot = 0;
        for (int k = 0; k < kBsumBlock / 64; k++) {
            const uint32_t t = wt[k];
            if (k < wid) below += t;
            tot += t;
        }
        uint32_t ex = carry + below + (x - v);
        for (int k = 0; k < kBsumItems; k++) {
            if (i0 + k < nblk) bsum[i0 + k] = ex;
            ex += loc[k];
        }
        carry += tot;
        __syncthreads();  // wt is rewritten by the next pass
    }
}

__global__ void __launch_bounds__(kScanBlock) k_scan_final(DevScene S, const uint32_t *bsum, int which) {
    if (!chain_active(S, which)) return;
    __shared__ uint32_t sh[kScanBlock];
    const int64_t ntile = (S.n_cells + kScanTile - 1) / kScanTile;
    for (int64_t b = blockIdx.x; b < ntile; b += gridDim.x) {  // block_excl_scan ends on a barrier
        const int64_t base = b * kScanTile + threadIdx.x * kScanItems;
        uint32_t loc[kScanItems];
        uint32_t v = 0;
        for (int k = 0; k < kScanItems; k++) {
            loc[k] = base + k < S.n_cells ? S.cell_count[base + k] : 0u;
            v += loc[k];
        }
        uint32_t tot;
        uint32_t ex = block_excl_scan(v, sh, tot) + bsum[b];
        for (int k = 0; k < kScanItems; k++) {
            if (base + k < S.n_cells) S.cell_start[base + k] = ex;
            ex += loc[k];
            if (base + k == S.n_cells - 1) S.cell_start[S.n_cells] = ex;  // the end of the last bin
        }
    }
}

// Scatter spheres into their bins.  For a detection, every sphere also takes
// this detection's margin (fixed rule: one value; learned: per sphere), from
// which the integration sets its clump's displacement guard.
__device__ __forceinline__ void scatter_sphere(const DevScene &S, const float *margin_src, int which, int64_t s) {
    uint32_t cell = S.cell_of[s];
    uint32_t slot = S.cell_start[cell] + S.cell_rank[s];  // its rank within the bin, from the count
    double4 p = S.spos[s];
    const uint32_t own = S.owner[s];
    S.sorted_pos[slot] = p;
    const Grid &g = S.grids[S.sscene[s]];
    if (which) {  // the audit's binning: prefilter records without margin
        S.sorted_meta[slot] = make_uint4((uint32_t)s, own, 0u, 0u);
        S.sorted_f4[slot] = make_float4((float)(p.x - g.ox), (float)(p.y - g.oy), (float)(p.z - g.oz), (float)p.w);
        return;
    }
    float m = S.detect_mode == 2 ? S.bin_margin[region_of(g, cell)] : (margin_src ? margin_src[s] : S.ctl->margin_cur);
    S.sorted_meta[slot] = make_uint4((uint32_t)s, own, __float_as_uint(m), 0u);
    S.sorted_f4[slot] = make_float4((float)(p.x - g.ox), (float)(p.y - g.oy), (float)(p.z - g.oz), (float)p.w + m);
    slot3(S.smargin, out_slot(S))[s] = m;
}

__global__ void __launch_bounds__(256) k_cell_scatter(DevScene S, const float *margin_src, int which) {
    if (!chain_active(S, which)) return;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < S.ns; s += (int64_t)gridDim.x * blockDim.x)
        scatter_sphere(S, margin_src, which, s);
}

// Fixed rule of the enlarged contact geometry: the margin covers k steps of
// motion at the measured speed and acceleration envelopes,
// m = safety k h v + (k h)^2 a / 2, with the longest k <= k_max whose margin
// stays below the cap.  A sphere that still outruns it trips the guard.
__global__ void k_plan(DevScene S) {
    Ctl *c = S.ctl;
    if (!due(c) || aborted(c)) return;
    c->m_max_bits = 0u;  // raised below (fixed rule) or by k_region_margin (learned)
    if (S.detect_mode == 0) { c->margin_cur = 0.0f; c->k_cur = 1; return; }
    if (S.detect_mode == 2) {  // per-region margins; k_bin_margin may shorten the interval
        c->k_cur = S.plan.k_max;
        c->margin_cur = 0.0f;
        return;
    }
    float v = fmaxf(__uint_as_float(c->vmax_bits), S.plan.v_user);
    float a = __uint_as_float(c->amax_last);
    if (S.bchain) {
        // a set built ahead, from a snapshot, must cover the steps until its
        // adoption and its interval of use: the fixed horizon, capped (a
        // sphere that outruns the cap trips the guard)
        const double T = (double)S.horizon * S.h;
        double m = (double)S.plan.safety * (T * (double)v) + 0.5 * (double)a * T * T;
        m = fmax(fmin(m, (double)S.plan.margin_cap), (double)S.plan.margin_floor);
        c->margin_cur = (float)m;
        c->m_max_bits = __float_as_uint(c->margin_cur);
        c->k_cur = S.plan.k_max;
        return;
    }
    int k = S.plan.k_max;
    double m = 0.0;
    for (; k >= 1; k--) {
        double T = (double)k * S.h;
        m = (double)S.plan.safety * (T * (double)v) + 0.5 * (double)a * T * T;
        if (m <= (double)S.plan.margin_cap) break;
    }
    if (k < 1) { k = 1; m = S.plan.margin_cap; }
    m = fmax(m, (double)S.plan.margin_floor);
    if (S.plan.test_zero_margin) { m = 0.0; k = S.plan.k_max; }
    c->margin_cur = (float)m;
    c->m_max_bits = __float_as_uint(c->margin_cur);
    c->k_cur = k;
}

// ---------------------------------------------------------------- learned envelopes
// Features of the envelope regions (blocks of kRegionBins^3 bins): max sphere
// speed, max acceleration envelope of the spheres' clumps (last step),
// occupancy (spheres in the region).
// Neighbouring spheres mostly share a region: the lanes of a wavefront first
// combine runs of equal region (maxima by shuffles, counts from the run
// heads), and only each run's first lane updates the region.
__global__ void __launch_bounds__(256) k_bin_features(DevScene S, int which) {
    if (!(which == 2 || (due(S.ctl) && S.detect_mode == 2))) return;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int64_t r = -1;
    float v = 0.f, a = 0.f;
    if (s < S.ns) {
        r = region_of(S.grids[S.sscene[s]], S.cell_of[s]);
        v = S.sspeed[s];
        a = S.cacc[S.owner[s]];
    }
    const int rl = (int)r, rh = (int)(r >> 32);
    const int pl = __shfl_up(rl, 1, 64), ph = __shfl_up(rh, 1, 64);
    const bool head = lane == 0 || pl != rl || ph != rh;
    const unsigned long long heads = __ballot(head);
    // run maxima: combine with lanes further down the same run
    for (int off = 1; off < 64; off <<= 1) {
        const int ol = __shfl_down(rl, off, 64), oh = __shfl_down(rh, off, 64);
        const float ov = __shfl_down(v, off, 64), oa = __shfl_down(a, off, 64);
        if (lane + off < 64 && ol == rl && oh == rh) { v = fmaxf(v, ov); a = fmaxf(a, oa); }
    }
    if (!head || r < 0) return;
    const unsigned long long later = lane < 63 ? heads >> (lane + 1) : 0ull;
    const int next = later ? lane + 1 + __builtin_ctzll(later) : 64;
    const uint32_t n = (uint32_t)(next - lane);  // the run (an invalid lane has r < 0: a run of its own)
    if (v > 0.f) atomicMax(&S.bin_v[r], __float_as_uint(v));
    if (a > 0.f) atomicMax(&S.bin_a[r], __float_as_uint(a));
    atomicAdd(&S.reg_occ[r], n);
}

// Envelopes of each occupied region for this detection: the MLP predicts the
// region's speed and acceleration envelopes over the interval (never below
// what the region shows now); a non-finite or implausible prediction falls
// back to the fixed rule's global envelopes.  The envelopes replace the
// features in bin_v / bin_a.  The interval becomes the longest k <= k_max
// whose margin m = safety k h v + (k h)^2 a / 2 stays within the cap in every
// region (reduced on the device; k_plan starts it at k_max).
__global__ void __launch_bounds__(256) k_bin_margin(DevScene S) {
    Ctl *c = S.ctl;
    if (!due(c) || aborted(c) || S.detect_mode != 2) return;
    __shared__ float P[kMlpParams];
    __shared__ __align__(16) float Wt[kMlpH * kMlpH];  // second-layer weights, transposed
    for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) P[i] = S.mlp[i];
    for (int k = threadIdx.x; k < kMlpH * kMlpH; k += blockDim.x)
        Wt[(k % kMlpH) * kMlpH + k / kMlpH] = S.mlp[kMlpOffW2 + k];
    __syncthreads();
    const float vg = fmaxf(__uint_as_float(c->vmax_bits), S.plan.v_user);
    const float ag = __uint_as_float(c->amax_last);
    const int kmax = S.plan.k_max;
    uint32_t nfb = 0;
    int kmin = kmax;
    // the interval rule's false-positive model: sums over the regions of
    // n_r rho_r v_env and n_r rho_r a_env (n_r spheres in the region, rho_r
    // their number density)
    double wv = 0.0, wa = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < S.n_regions;
         r += (int64_t)gridDim.x * blockDim.x) {
        uint32_t occ = S.reg_occ[r];
        if (!occ) continue;
        // keeps the LDS weights from being hoisted out of the region loop
        // into registers (they would spill)
        __asm__ volatile("" ::: "memory");
        float vn = __uint_as_float(S.bin_v[r]), an = __uint_as_float(S.bin_a[r]);
        float y0, y1;
        mlp_forward_t(P, Wt, vn, an, (float)occ, y0, y1);
        float ve = expf(y0), ae = expf(y1);
        if (!(ve < 1e3f) || !(ae < 1e9f) || !(ve >= 0.f) || !(ae >= 0.f)) {  // NaN fails every test
            ve = vg;
            ae = ag;
            nfb++;
        }
        ve = fmaxf(ve, vn);
        ae = fmaxf(ae, an);
        S.bin_v[r] = __float_as_uint(ve);
        S.bin_a[r] = __float_as_uint(ae);
        {
            int lo = 0, hi = S.n_scenes - 1;  // the region's scene: grids are in region order
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (S.grids[mid].reg0 <= r) lo = mid; else hi = mid - 1;
            }
            const double edge = (double)kRegionBins * S.grids[lo].b;
            const double w = (double)occ * ((double)occ / (edge * edge * edge));
            wv += w * (double)ve;
            wa += w * (double)ae;
        }
        int k = kmax;
        for (; k > 1; k--) {
            const double T = (double)k * S.h;
            if ((double)S.plan.safety * (T * (double)ve) + 0.5 * (double)ae * T * T <= (double)S.plan.margin_cap) break;
        }
        kmin = min(kmin, k);
    }
    for (int off = 32; off > 0; off >>= 1) {
        nfb += __shfl_xor(nfb, off, 64);
        kmin = min(kmin, __shfl_xor(kmin, off, 64));
        wv += __shfl_xor(wv, off, 64);
        wa += __shfl_xor(wa, off, 64);
    }
    __shared__ double ws[2][4];
    if ((threadIdx.x & 63) == 0) {
        if (nfb) atomicAdd((unsigned long long *)&c->fallbacks, (unsigned long long)nfb);
        if (kmin < kmax) atomicMin(&c->k_cur, kmin);
        ws[0][threadIdx.x >> 6] = wv;
        ws[1][threadIdx.x >> 6] = wa;
    }
    __syncthreads();
    if (threadIdx.x == 0) {  // this workgroup's sums, in a fixed order
        S.part_k[blockIdx.x] = ((ws[0][0] + ws[0][1]) + ws[0][2]) + ws[0][3];
        S.part_k[kRegionBlocksMax + blockIdx.x] = ((ws[1][0] + ws[1][1]) + ws[1][2]) + ws[1][3];
    }
}

// Detection interval of the learned envelopes: the k <= k_fit (the longest
// interval whose margins fit the cap in every region, found above) that
// minimises the modelled bytes per sphere-step of the deferred path,
//   B(k) = 8 (p_m - p) + (244 + 72 p_m) / k  (+ terms that do not depend on k),
// p the contact pairs per sphere of the last step and p_m = p + D(k) the
// candidate pairs per sphere, with D(k) the false positives the margins
// m_r(k) = safety k h v_r + (k h)^2 a_r / 2 add: each sphere of region r
// finds rho_r 4 pi (2 R)^2 (2 m_r) extra partners in the shell the margins
// add (R the mean radius), so D(k) = c 16 pi R^2 sum_r n_r rho_r m_r(k) / N,
// with c the ratio of the measured to the modelled false positives of the
// set in use (the density next to a contact is not the mean density).  The
// 8 B per false positive and the 244 + 72 p_m B per detection are the
// per-unit terms of the deferred path's byte model.  One workgroup; the
// workgroup sums of the margin model are added in a fixed order.
__global__ void __launch_bounds__(256) k_pick_interval(DevScene S, unsigned nblk) {
    Ctl *c = S.ctl;
    if (!due(c) || aborted(c) || S.detect_mode != 2 || S.overlap) return;  // overlapped: the host's interval
    __shared__ double sv[256], sa[256];
    double v = 0.0, a = 0.0;
    for (unsigned b = threadIdx.x; b < nblk; b += blockDim.x) {
        v += S.part_k[b];
        a += S.part_k[kRegionBlocksMax + b];
    }
    sv[threadIdx.x] = v;
    sa[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sv[threadIdx.x] += sv[threadIdx.x + w];
            sa[threadIdx.x] += sa[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double ns = (double)(S.ns > 0 ? S.ns : 1);
    const double p = (double)c->contact_sides_last / 2.0 / ns;
    if (c->dpred_last > 0.0 && c->n_pairs_cur > 0) {  // calibrate on the set in use
        const double meas = (double)c->n_pairs_cur / ns - p;
        c->c_cal = fmin(fmax(meas / c->dpred_last, 0.05), 20.0);
    }
    const double cal = c->c_cal > 0.0 ? c->c_cal : 1.0;
    const double G = 16.0 * 3.14159265358979323846 * (double)S.plan.r_mean * (double)S.plan.r_mean / ns;
    const int kfit = c->k_cur;
    int best = kfit;
    double bestB = 1e300, bestD = 0.0;
    for (int k = 1; k <= kfit; k++) {
        const double T = (double)k * S.h;
        const double D = G * ((double)S.plan.safety * T * sv[0] + 0.5 * T * T * sa[0]);
        const double B = 8.0 * cal * D + (244.0 + 72.0 * (p + cal * D)) / (double)k;
        if (B < bestB) { bestB = B; best = k; bestD = D; }
    }
    c->k_cur = best;
    c->dpred_last = bestD;
}

// Margin of every occupied region for the interval chosen above (clamped to
// [floor, cap]: a region that still needs more relies on the guard).
// The largest of them bounds the partner side of the narrow phase's reach.
__global__ void __launch_bounds__(256) k_region_margin(DevScene S) {
    Ctl *c = S.ctl;
    if (!due(c) || aborted(c) || S.detect_mode != 2) return;
    const double T = (double)(S.bchain ? S.horizon : c->k_cur) * S.h;
    float mmax = 0.0f;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < S.n_regions;
         r += (int64_t)gridDim.x * blockDim.x) {
        if (!S.reg_occ[r]) continue;
        const double ve = (double)__uint_as_float(S.bin_v[r]), ae = (double)__uint_as_float(S.bin_a[r]);
        double m = (double)S.plan.safety * (T * ve) + 0.5 * ae * T * T;
        m = fmin(fmax(m, (double)S.plan.margin_floor), (double)S.plan.margin_cap);
        const float mf = S.plan.test_zero_margin ? 0.0f : (float)m;
        S.bin_margin[r] = mf;
        mmax = fmaxf(mmax, mf);
    }
    for (int off = 32; off > 0; off >>= 1) mmax = fmaxf(mmax, __shfl_xor(mmax, off, 64));
    if ((threadIdx.x & 63) == 0 && mmax > 0.0f) raise_max(&c->m_max_bits, mmax);  // filtered: few atomics land
}

// Training-data capture: remember each sphere's region and each region's
// occupancy at capture time, and clear the horizon labels.
__global__ void __launch_bounds__(256) k_collect_init(DevScene S) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = i; k < S.ns; k += stride) S.cell_t[k] = (uint32_t)region_of(S.grids[S.sscene[k]], S.cell_of[k]);
    for (int64_t k = i; k < S.n_regions; k += stride) { S.occ_t[k] = S.reg_occ[k]; S.lab_v[k] = 0; S.lab_a[k] = 0; }
}

// Horizon labels: the largest speed / acceleration envelope any sphere of the
// region (as binned at capture) shows during the following steps.
__global__ void __launch_bounds__(256) k_collect_speed(DevScene S) {
    if (!S.ctl->collecting) return;
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S.ns) return;
    float v = S.sspeed[s];
    if (v > 0.f) atomicMax(&S.lab_v[S.cell_t[s]], __float_as_uint(v));
}

__global__ void __launch_bounds__(256) k_collect_acc(DevScene S) {
    if (!S.ctl->collecting) return;
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S.ns) return;
    float a = S.cacc[S.owner[s]];
    if (a > 0.f) atomicMax(&S.lab_a[S.cell_t[s]], __float_as_uint(a));
}

// ---------------------------------------------------------------- narrow phase
// Wave64 exclusive scan of per-lane counts; returns the lane's offset and the total.
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t &total) {
    int lane = threadIdx.x & 63;
    uint32_t x = v;
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    total = __shfl(x, 63, 64);
    return x - v;
}

// Candidate partners of sphere s for the detection in progress, in no
// particular order: spheres of other clumps inside the enlarged contact
// geometry, d^2 < ((R_s + R_t) + (m_s + m_t))^2, then boundaries with
// phi < R_s + (m_s + boundary margin).  emit(t) is called once per candidate.
// What the narrow phase knows of the sphere it works for.
struct NarrowSelf {
    double4 P;        // centre, radius
    float4 Pf;        // FP32 prefilter record: centre - grid origin, radius + margin
    uint32_t own;     // clump
    float ms;         // margin
    bool exact_only;  // far outside the domain the FP32 slack no longer bounds the rounding
    double reach;     // its own (R + m) plus the largest partner (R + m), plus a small slack
    double slack;     // fixed-point positions: twice the rounding of a distance of world centres
};
__device__ __forceinline__ NarrowSelf narrow_self(const DevScene &S, const Grid &g, uint32_t s) {
    NarrowSelf n;
    n.P = S.spos[s];
    n.own = S.owner[s];
    n.ms = slot3(S.smargin, out_slot(S))[s];  // this detection's margin
    n.Pf = make_float4((float)(n.P.x - g.ox), (float)(n.P.y - g.oy), (float)(n.P.z - g.oz), (float)n.P.w + n.ms);
    n.exact_only = !(fabsf(n.Pf.x) < g.pre_lim && fabsf(n.Pf.y) < g.pre_lim && fabsf(n.Pf.z) < g.pre_lim);
    // With fixed-point positions the force kernel decides contact from exact
    // CoM differences, the detection from world centres (a few ulps of their
    // coordinates off): the slack covers twice that rounding, so that every
    // contact the force kernel or an audit can see is a candidate.
    n.slack = 0.0;
    if (S.pos_exp)
        n.slack = ldexp(fmax(fmax(fabs(n.P.x), fabs(n.P.y)), fabs(n.P.z)) + (n.P.w + (double)n.ms) + g.rm_max +
                            4.0 * g.r_max, -46);
    // the partner side: the largest radius and the largest margin any sphere
    // takes at this detection
    n.reach = (n.P.w + (double)n.ms) + (g.r_max + (double)__uint_as_float(S.ctl->m_max_bits)) + 1e-9 + n.slack;
    return n;
}

// The conservative FP32 test of sorted slot j: it can only admit extra
// candidates, which the exact FP64 predicate then rejects.
__device__ __forceinline__ bool narrow_prefilter_rec(const Grid &g, const NarrowSelf &n, float4 Qf) {
    const float fx = Qf.x - n.Pf.x, fy = Qf.y - n.Pf.y, fz = Qf.z - n.Pf.z;
    const float fr = (n.Pf.w + Qf.w) + g.pre_eps;
    return n.exact_only || fx * fx + fy * fy + fz * fz < fr * fr;
}
__device__ __forceinline__ bool narrow_prefilter(const DevScene &S, const Grid &g, const NarrowSelf &n, uint32_t j) {
    return narrow_prefilter_rec(g, n, S.sorted_f4[j]);
}

// Visit the slots [jb, je) four at a time, the four records loaded before
// any is tested (more loads in flight per lane); f(j, passed) in slot order.
constexpr uint32_t kSlotBatch = 4;
template <typename T, typename F>
__device__ __forceinline__ void slot_batches(const float4 *rec, uint32_t jb, uint32_t je, T &&test, F &&f) {
    for (uint32_t j = jb; j < je; j += kSlotBatch) {
        float4 q[kSlotBatch];
#pragma unroll
        for (uint32_t u = 0; u < kSlotBatch; u++)
            if (j + u < je) q[u] = rec[j + u];
#pragma unroll
        for (uint32_t u = 0; u < kSlotBatch; u++)
            if (j + u < je && test(q[u])) f(j + u);
    }
}

// The exact predicate of the enlarged geometry for slot j (another clump,
// d^2 < ((R_s + R_t) + (m_s + m_t))^2); returns the partner's id or ~0u.
__device__ __forceinline__ uint32_t narrow_exact(const DevScene &S, const NarrowSelf &n, uint32_t j) {
    const uint4 md = S.sorted_meta[j];
    if (md.y == n.own) return ~0u;
    const double4 Q = S.sorted_pos[j];
    const double dx = Q.x - n.P.x, dy = Q.y - n.P.y, dz = Q.z - n.P.z;
    const double d2 = dx * dx + dy * dy + dz * dz;
    double Sr = n.P.w + Q.w;
    Sr = Sr + (((double)n.ms + (double)__uint_as_float(md.z)) + n.slack);
    return d2 < Sr * Sr ? md.x : ~0u;
}
// The same test with the slot's record loaded beforehand (so that the loads
// of several slots are in flight together).
struct SlotRec { double4 Q; uint32_t own, id; float m; };
__device__ __forceinline__ SlotRec load_slot(const DevScene &S, uint32_t j) {
    const uint4 md = S.sorted_meta[j];
    return SlotRec{S.sorted_pos[j], md.y, md.x, __uint_as_float(md.z)};
}
__device__ __forceinline__ uint32_t narrow_exact_rec(const NarrowSelf &n, const SlotRec &r) {
    if (r.own == n.own) return ~0u;
    const double dx = r.Q.x - n.P.x, dy = r.Q.y - n.P.y, dz = r.Q.z - n.P.z;
    const double d2 = dx * dx + dy * dy + dz * dz;
    double Sr = n.P.w + r.Q.w;
    Sr = Sr + (((double)n.ms + (double)r.m) + n.slack);
    return d2 < Sr * Sr ? r.id : ~0u;
}

// The triangles of the sphere's scene that may lie within r of point p
// (within r plus their mesh's margin of their box at the last detection),
// after the scene's and each chunk's box: f(k, r + margin) for each, in
// ascending k.
template <class F>
__device__ __forceinline__ void tri_near(const DevScene &S, const Grid &g, const double *p, double r, F f) {
    if (g.chunk_beg >= g.chunk_end) return;
    auto outside = [&](const double *b, double d) {
        return p[0] < b[0] - d || p[1] < b[1] - d || p[2] < b[2] - d || p[0] > b[3] + d || p[1] > b[4] + d ||
               p[2] > b[5] + d;
    };
    if (outside(S.tri_box + 6 * (S.n_tri + S.n_chunk + g.sid), r)) return;
    for (int64_t c = g.chunk_beg; c < g.chunk_end; c++) {
        if (outside(S.tri_box + 6 * (S.n_tri + c), r)) continue;
        for (int64_t k = S.chunk_tri[c]; k < S.chunk_tri[c + 1]; k++) {
            const double lim = r + S.mesh[S.tri_mesh[k]].margin;
            if (outside(S.tri_box + 6 * k, lim)) continue;
            f(k, lim);
        }
    }
}

// Boundary candidates of sphere s: phi < R_s + (m_s + boundary margin), for
// the analytic boundaries of its scene, then the triangles of its scene's
// meshes (a triangle whose bounding box at this detection is farther than
// that is skipped without the distance).
template <bool TRI, class Emit>
__device__ __forceinline__ void narrow_boundaries(const DevScene &S, const Grid &g, const NarrowSelf &n, Emit emit) {
    const double tnow = (double)S.ctl->step * S.h;
    for (int b = g.bnd_beg; b < g.bnd_end; b++) {
        double phi, nv[3];
        if (!bnd_distance(S.bnd[b], tnow, n.P.x, n.P.y, n.P.z, phi, nv)) continue;
        if (phi < n.P.w + ((double)n.ms + S.bnd[b].margin)) emit((uint32_t)(S.ns + b));
    }
    if constexpr (TRI) {
        const double p[3] = {n.P.x, n.P.y, n.P.z};
        tri_near(S, g, p, n.P.w + (double)n.ms, [&](int64_t k, double lim) {
            double phi, nv[3];
            if (tri_distance(S, k, p, phi, nv) && phi < lim) emit((uint32_t)(S.ns + S.n_bnd + k));
        });
    }
}

// World boxes of the triangles, of their chunks and of each scene's
// triangles at the detection in progress (the meshes' current poses); the
// chunk and scene boxes are grown by the margins of their meshes, so they
// hold every position a triangle takes while the active set is in use.  One
// wavefront per chunk.
__global__ void __launch_bounds__(256) k_tri_boxes(DevScene S) {
    if (!due(S.ctl) || aborted(S.ctl)) return;
    const int lane = threadIdx.x & 63;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; c < S.n_chunk; c += nw) {
        const int64_t k = (int64_t)S.chunk_tri[c] + lane;
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        if (k < S.chunk_tri[c + 1]) {
            double V[9];
            tri_world(S, k, V);
            double *bx = S.tri_box + 6 * k;
            const double m = S.mesh[S.tri_mesh[k]].margin;
            for (int i = 0; i < 3; i++) {
                bx[i] = fmin(fmin(V[i], V[3 + i]), V[6 + i]);
                bx[3 + i] = fmax(fmax(V[i], V[3 + i]), V[6 + i]);
                lo[i] = bx[i] - m;
                hi[i] = bx[3 + i] + m;
            }
        }
        for (int off = 32; off > 0; off >>= 1)
            for (int i = 0; i < 3; i++) {
                lo[i] = fmin(lo[i], __shfl_xor(lo[i], off, 64));
                hi[i] = fmax(hi[i], __shfl_xor(hi[i], off, 64));
            }
        if (lane == 0) {
            double *cb = S.tri_box + 6 * (S.n_tri + c);
            for (int i = 0; i < 3; i++) { cb[i] = lo[i]; cb[3 + i] = hi[i]; }
        }
    }
}
// ... and the scene boxes, one workgroup per scene over its chunk boxes.
__global__ void __launch_bounds__(256) k_tri_scene_boxes(DevScene S) {
    if (!due(S.ctl) || aborted(S.ctl)) return;
    const Grid &g = S.grids[blockIdx.x];
    double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int64_t c = g.chunk_beg + threadIdx.x; c < g.chunk_end; c += blockDim.x) {
        const double *cb = S.tri_box + 6 * (S.n_tri + c);
        for (int i = 0; i < 3; i++) { v[i] = fmin(v[i], cb[i]); v[3 + i] = fmax(v[3 + i], cb[3 + i]); }
    }
    __shared__ double sh[6][256];
    for (int i = 0; i < 6; i++) sh[i][threadIdx.x] = v[i];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int i = 0; i < 6; i++)
                sh[i][threadIdx.x] = i < 3 ? fmin(sh[i][threadIdx.x], sh[i][threadIdx.x + w])
                                           : fmax(sh[i][threadIdx.x], sh[i][threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x < 6) S.tri_box[6 * (S.n_tri + S.n_chunk + blockIdx.x) + threadIdx.x] = sh[threadIdx.x][0];
}

template <bool TRI, class Emit>
__device__ __forceinline__ void narrow_candidates(const DevScene &S, uint32_t s, Emit emit) {
    const Grid &g = S.grids[S.sscene[s]];
    const NarrowSelf n = narrow_self(S, g, s);
    scan_reach(S, g, n.P.x, n.P.y, n.P.z, n.reach, [&](uint32_t jb, uint32_t je) {
        for (uint32_t j = jb; j < je; j++) {
            if (!narrow_prefilter(S, g, n, j)) continue;
            const uint32_t t = narrow_exact(S, n, j);
            if (t != ~0u) emit(t);
        }
    });
    narrow_boundaries<TRI>(S, g, n, emit);
}

// Carry the tangential history of sphere s's new lower segment (partners
// t_k, ascending, at lb in the pair arrays) from its lower segment in the set
// in use: a pair present there keeps its history, a new pair starts at zero.
// Reads history buffer hb (laid out for the set in use), writes buffer hb ^ 1
// (laid out for the new set).
template <class Get>
__device__ __forceinline__ void carry_history(const DevScene &S, uint32_t s, uint32_t lb, int n_lo, Get get) {
    const int cur = S.ctl->buf, hb = S.ctl->hb;
    const uint32_t ob = slot3(S.lo_beg, cur)[s], oc = slot3(S.lo_cnt, cur)[s];
    const uint32_t *opt = slot3(S.pt, cur) + ob;
    const double *oh = pick(S.hist, hb) + 3 * (int64_t)ob;
    double *nh = pick(S.hist, hb ^ 1);
    uint32_t j = 0;
    for (int k = 0; k < n_lo; k++) {
        const uint32_t t = get(k);
        const int64_t p = (int64_t)lb + k;
        while (j < oc && opt[j] < t) j++;
        double h0 = 0.0, h1 = 0.0, h2 = 0.0;
        if (j < oc && opt[j] == t) { h0 = oh[3 * j]; h1 = oh[3 * j + 1]; h2 = oh[3 * j + 2]; }
        nh[3 * p] = h0; nh[3 * p + 1] = h1; nh[3 * p + 2] = h2;
    }
}

// Write the new segments of sphere s from its ascending candidates get(k):
// the first n_up (partners below s) to its upper segment at ub, the other
// n_lo (partners above s, boundaries last) to its lower segment at lb as
// pairs of the new set, in the detection's output slot.  (k_carry then
// carries the tangential history over.)
template <class Get>
__device__ __forceinline__ void write_rows(const DevScene &S, uint32_t s, uint32_t ub, int n_up, uint32_t lb, int n_lo,
                                           Get get) {
    const int out = out_slot(S);
    uint32_t *ut = slot3(S.ut, out), *us = slot3(S.us, out);
    for (int k = 0; k < n_up; k++) {
        ut[ub + k] = get(k);
        us[ub + k] = s;
    }
    uint32_t *npt = slot3(S.pt, out), *nps = slot3(S.ps, out);
    for (int k = 0; k < n_lo; k++) {
        const int64_t p = (int64_t)lb + k;
        npt[p] = get(n_up + k);
        nps[p] = s;
    }
}

// Narrow phase, first pass: one thread per sphere id (ids are spatially
// coherent: clumps are laid out in Morton order, so a wavefront's neighbour
// scans share cache lines).  Each sphere's candidates, up to kMaxRow kept
// sorted in LDS while they are found, are staged with its counts, entry k of
// every sphere together (a wavefront writes, and the second pass reads, each
// entry as one contiguous run); a sphere with more candidates stages only its
// counts (its segments are filled by k_narrow_over).  Each workgroup also
// sums its spheres' upper entries, pairs and boundary pairs, which
// k_narrow_base turns into the bases of their segments.
// TRI: the scene has triangles (the kernel without them keeps fewer registers).
// Candidate t of sphere s: inserted in order into the lane's LDS column
// (entry k at col[k stride], at most kMaxRow kept); all candidates, those
// below s and the boundary ones are counted.
__device__ __forceinline__ void emit_sorted(uint32_t *col, int stride, uint32_t t, uint32_t s, int64_t ns, int &cnt,
                                            int &nup, int &nbp) {
    if (cnt < kMaxRow) {
        int k = cnt;
        while (k > 0 && col[(k - 1) * stride] > t) {
            col[k * stride] = col[(k - 1) * stride];
            k--;
        }
        col[k * stride] = t;
    }
    cnt++;
    nup += t < s;
    nbp += t >= (uint32_t)ns;
}

// Staging of sphere s: its counts (below it and boundaries packed for a
// listed sphere), then entry k at stage[k ns + s]; a sphere with more than
// kMaxRow candidates stages its counts only.
template <class Get>
__device__ __forceinline__ void stage_sphere(const DevScene &S, uint32_t s, int cnt, int nup, int nbp, Get get) {
    if (cnt > kMaxRow) {
        S.stage_n[s] = make_uint2((uint32_t)cnt, (uint32_t)nup);
        S.stage[s] = (uint32_t)nbp;
        return;
    }
    S.stage_n[s] = make_uint2((uint32_t)cnt, (uint32_t)nup | ((uint32_t)nbp << 16));
    for (int k = 0; k < cnt; k++) S.stage[(int64_t)k * S.ns + s] = get(k);
}

template <bool TRI>
__device__ __forceinline__ void narrow_sphere(const DevScene &S, uint32_t s, uint32_t *lst, int &cnt, int &nup,
                                              int &nbp) {
    const int tid = threadIdx.x;
    auto emit = [&](uint32_t t) { emit_sorted(lst + tid, kNarrowBlock, t, s, S.ns, cnt, nup, nbp); };
    const Grid &g = S.grids[S.sscene[s]];
    // First the cheap FP32 test over every slot in reach, keeping the slots
    // that pass in the LDS list; then the exact test over that short list.
    // Split this way, a wavefront runs the exact test and the sorted insert
    // as often as its busiest lane has prefilter hits, not as often as it
    // has slots in reach. The scan holds only the FP32 view of the sphere;
    // its FP64 record is read again for the exact tests.
    float4 Pf;
    float reach32;
    bool exact_only;
    {
        const NarrowSelf n0 = narrow_self(S, g, s);
        Pf = n0.Pf;
        reach32 = (float)n0.reach + 2.0f * g.pre_eps;
        exact_only = n0.exact_only;
    }
    int npre = 0;
    if (!exact_only)
        scan_reach32(S, g, Pf.x, Pf.y, Pf.z, reach32, [&](uint32_t jb, uint32_t je) {
            slot_batches(S.sorted_f4, jb, je, [&](float4 q) {
                             const float fx = q.x - Pf.x, fy = q.y - Pf.y, fz = q.z - Pf.z;
                             const float fr = (Pf.w + q.w) + g.pre_eps;
                             return fx * fx + fy * fy + fz * fz < fr * fr;
                         },
                         [&](uint32_t q) {
                             if (npre < kMaxRow) lst[npre * kNarrowBlock + tid] = q;
                             npre++;
                         });
        });
    uint32_t s2 = s;
    asm volatile("" : "+v"(s2));  // a fresh read, not the values loaded before the scan
    const NarrowSelf n = narrow_self(S, g, s2);
    if (n.exact_only || npre > kMaxRow) {
        // many slots pass the prefilter (or the sphere is far outside its
        // grid): k_narrow_fb finds its candidates with one exact pass and
        // adds its counts to the workgroup's sums; kept out of this kernel,
        // that pass's registers do not limit the wavefronts in flight here
        const uint32_t k = atomicAdd((uint32_t *)&S.ctl->n_fb, 1u);
        S.fb_list[k] = s;
        return;
    }
    {
        // two listed slots at a time, both read before either is inserted:
        // an insert writes at most at the position of the later slot read
        for (int k = 0; k < npre; k += 2) {
            const bool two = k + 1 < npre;
            const uint32_t j0 = lst[k * kNarrowBlock + tid];
            const uint32_t j1 = two ? lst[(k + 1) * kNarrowBlock + tid] : j0;
            const SlotRec r0 = load_slot(S, j0), r1 = load_slot(S, j1);
            const uint32_t t0 = narrow_exact_rec(n, r0);
            if (t0 != ~0u) emit(t0);
            if (two) {
                const uint32_t t1 = narrow_exact_rec(n, r1);
                if (t1 != ~0u) emit(t1);
            }
        }
        narrow_boundaries<TRI>(S, g, n, emit);
    }
    stage_sphere(S, s, cnt, nup, nbp, [&](int k) { return lst[k * kNarrowBlock + tid]; });
}

template <bool TRI>
__global__ void __launch_bounds__(kNarrowBlock) k_narrow(DevScene S) {
    // nothing in this launch raises the abort flags: the test is uniform
    if (!due(S.ctl) || aborted(S.ctl)) return;
    __shared__ uint32_t lst[kMaxRow * kNarrowBlock];
    const int64_t blk = xcd_block(), i = blk * kNarrowBlock + threadIdx.x;
    int cnt = 0, nup = 0, nbp = 0;
    if (i < S.ns) narrow_sphere<TRI>(S, (uint32_t)i, lst, cnt, nup, nbp);
    unsigned long long v[3] = {(unsigned long long)nup, (unsigned long long)(cnt - nup), (unsigned long long)nbp};
    __shared__ unsigned long long sh[3][kNarrowBlock / 64];
    for (int q = 0; q < 3; q++) {
        for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_xor(v[q], off, 64);
        if ((threadIdx.x & 63) == 0) sh[q][threadIdx.x >> 6] = v[q];
    }
    __syncthreads();
    constexpr int kWaves = kNarrowBlock / 64;
    if (threadIdx.x < 3) {
        unsigned long long t = 0;
        for (int k = 0; k < kWaves; k++) t += sh[threadIdx.x][k];
        S.narrow_part[3 * blk + threadIdx.x] = t;
    } else if (threadIdx.x >= 64 && threadIdx.x < 64 + 2 * kWaves) {
        // each wavefront's upper entries and pairs below it in the workgroup
        const int w = (threadIdx.x - 64) >> 1, q = (threadIdx.x - 64) & 1;
        unsigned long long t = 0;
        for (int k = 0; k < w; k++) t += sh[q][k];
        S.narrow_woff[(blk * kWaves + w) * 2 + q] = (uint32_t)t;
    }
}

// Candidates of the spheres the first pass left (more than kMaxRow slots
// through its prefilter, or far outside their grid): one exact FP64 pass over
// the slots in reach, staged as the first pass stages, the counts added to
// the sums of the sphere's workgroup and to the offsets of the wavefronts
// after its own there (integer adds, so their order does not matter).
template <bool TRI>
__global__ void __launch_bounds__(64) k_narrow_fb(DevScene S) {
    if (!due(S.ctl) || aborted(S.ctl)) return;
    __shared__ uint32_t lst[kMaxRow * 64];
    constexpr int kWaves = kNarrowBlock / 64;
    const int tid = threadIdx.x;
    const int64_t n = S.ctl->n_fb;
    for (int64_t k = (int64_t)blockIdx.x * 64 + tid; k < n; k += (int64_t)gridDim.x * 64) {
        const uint32_t s = S.fb_list[k];
        int cnt = 0, nup = 0, nbp = 0;
        narrow_candidates<TRI>(S, s, [&](uint32_t t) { emit_sorted(lst + tid, 64, t, s, S.ns, cnt, nup, nbp); });
        stage_sphere(S, s, cnt, nup, nbp, [&](int q) { return lst[q * 64 + tid]; });
        const int64_t blk = s / kNarrowBlock;
        const int w = (int)(s % kNarrowBlock) / 64;
        atomicAdd(&S.narrow_part[3 * blk], (unsigned long long)nup);
        atomicAdd(&S.narrow_part[3 * blk + 1], (unsigned long long)(cnt - nup));
        atomicAdd(&S.narrow_part[3 * blk + 2], (unsigned long long)nbp);
        for (int v = w + 1; v < kWaves; v++) {
            atomicAdd(&S.narrow_woff[(blk * kWaves + v) * 2], (uint32_t)nup);
            atomicAdd(&S.narrow_woff[(blk * kWaves + v) * 2 + 1], (uint32_t)(cnt - nup));
        }
    }
}

// Narrow phase, second pass: the segments of the new set, in sphere id
// order (pairs follow their lower sphere's id, so that the pair kernel and
// the reduction stream them), placed by a scan of the workgroup sums of the
// first pass rather than by atomics (tens of thousands of workgroups adding
// to one counter serialise): k_narrow_base turns the sums into bases (and the
// totals, which also size a regrow), k_narrow_rows writes the segments (with
// each wavefront's offset in its workgroup, also from the first pass),
// k_carry the history.
__device__ __forceinline__ void staged_counts(const DevScene &S, int64_t i, int &cnt, int &nup, int &nbp) {
    cnt = 0; nup = 0; nbp = 0;
    if (i >= S.ns) return;
    const uint2 c = S.stage_n[i];
    cnt = (int)c.x;
    if (cnt <= kMaxRow) { nup = (int)(c.y & 0xffffu); nbp = (int)(c.y >> 16); }
    else { nup = (int)c.y; nbp = (int)S.stage[i]; }
}

// Exclusive scan of the workgroup sums in place: one workgroup, each lane
// taking kBaseItems consecutive workgroups per pass (their loads issued
// together); the totals go to the control block, and a set beyond the
// storage's capacity aborts the step (it is regrown).
constexpr int kBaseBlock = 1024, kBaseItems = 4;
__global__ void __launch_bounds__(kBaseBlock) k_narrow_base(DevScene S, int64_t nblk) {
    Ctl *c = S.ctl;
    if (!due(c) || aborted(c)) return;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    unsigned long long *P = S.narrow_part;
    __shared__ unsigned long long wt[3][kBaseBlock / 64];
    unsigned long long carry[3] = {0, 0, 0};
    for (int64_t b0 = 0; b0 < nblk; b0 += (int64_t)kBaseBlock * kBaseItems) {
        const int64_t i0 = b0 + (int64_t)threadIdx.x * kBaseItems;
        unsigned long long loc[kBaseItems][3], v[3] = {0, 0, 0};
#pragma unroll
        for (int k = 0; k < kBaseItems; k++)
#pragma unroll
            for (int q = 0; q < 3; q++) {
                loc[k][q] = i0 + k < nblk ? P[3 * (i0 + k) + q] : 0ull;
                v[q] += loc[k][q];
            }
        unsigned long long x[3];
#pragma unroll
        for (int q = 0; q < 3; q++) {  // inclusive wave scans
            x[q] = v[q];
            for (int off = 1; off < 64; off <<= 1) {
                const unsigned long long y = __shfl_up(x[q], off, 64);
                if (lane >= off) x[q] += y;
            }
            if (lane == 63) wt[q][wid] = x[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 3; q++) {
            unsigned long long below = 0, tot = 0;
            for (int k = 0; k < kBaseBlock / 64; k++) {
                const unsigned long long t = wt[q][k];
                if (k < wid) below += t;
                tot += t;
            }
            unsigned long long ex = carry[q] + below + (x[q] - v[q]);
#pragma unroll
            for (int k = 0; k < kBaseItems; k++) {
                if (i0 + k < nblk) P[3 * (i0 + k) + q] = ex;
                ex += loc[k][q];
            }
            carry[q] += tot;
        }
        __syncthreads();  // wt is rewritten by the next pass
    }
    if (threadIdx.x == 0) {
        c->n_up = (int64_t)carry[0];
        c->n_pairs = (int64_t)carry[1];
        c->n_bp = (int64_t)carry[2];
        if (carry[0] > (unsigned long long)S.cap || carry[1] > (unsigned long long)S.cap) c->overflow = 1;
    }
}

// The segments, one wavefront per 64 spheres of a first-pass workgroup (its
// base: the workgroup's scanned sums plus the wavefront's offset within the
// workgroup, both from the first pass), over at most kStepGrid workgroups: a
// step without a detection returns at once.  No barriers: each wavefront
// works alone.
__global__ void __launch_bounds__(kNarrowBlock) k_narrow_rows(DevScene S) {
    if (!due(S.ctl) || aborted(S.ctl)) return;  // uniform: set before this launch or not at all
    constexpr int kWaves = kNarrowBlock / 64;
    const int lane = threadIdx.x & 63, out = out_slot(S);
    const int64_t nw = (S.ns + 63) / 64;  // wavefronts of spheres
    for (int64_t gw = (int64_t)xcd_block() * kWaves + (threadIdx.x >> 6); gw < nw; gw += (int64_t)gridDim.x * kWaves) {
        const int64_t blk = gw / kWaves, i = gw * 64 + lane;
        int cnt, nup, nbp;
        staged_counts(S, i, cnt, nup, nbp);
        const int nlo = cnt - nup;
        uint32_t totu, totl;
        const uint32_t offu = wave_excl_scan((uint32_t)nup, totu);
        const uint32_t offl = wave_excl_scan((uint32_t)nlo, totl);
        const uint32_t *wo = S.narrow_woff + gw * 2;
        const unsigned long long bu = S.narrow_part[3 * blk] + wo[0], bl = S.narrow_part[3 * blk + 1] + wo[1];
        if (i >= S.ns) continue;
        const uint32_t s = (uint32_t)i;
        const uint32_t ub = (uint32_t)(bu + offu), lb = (uint32_t)(bl + offl);
        slot3(S.up_beg, out)[s] = ub;
        slot3(S.up_cnt, out)[s] = (uint32_t)nup;
        slot3(S.lo_beg, out)[s] = lb;
        slot3(S.lo_cnt, out)[s] = (uint32_t)nlo;
        if (cnt > kMaxRow) {
            const uint32_t k = atomicAdd((uint32_t *)&S.ctl->n_over, 1u);
            if (k < (uint32_t)S.over_cap) S.over_list[k] = s;
            else S.ctl->row_overflow = 1;
            continue;
        }
        write_rows(S, s, ub, nup, lb, nlo, [&](int k) { return S.stage[(int64_t)k * S.ns + i]; });
    }
}

// Segments of the spheres with more than kMaxRow candidates: the same scan,
// each segment kept sorted in place in the active set.
template <bool TRI>
__global__ void __launch_bounds__(64) k_narrow_over(DevScene S) {
    const Ctl *c = S.ctl;
    if (!due(c) || c->overflow || c->row_overflow) return;
    const int out = out_slot(S);
    const int64_t n = min((int64_t)c->n_over, (int64_t)S.over_cap);
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t s = S.over_list[k];
        const uint32_t ub = slot3(S.up_beg, out)[s], nu = slot3(S.up_cnt, out)[s];
        const uint32_t lb = slot3(S.lo_beg, out)[s], nl = slot3(S.lo_cnt, out)[s];
        uint32_t *urow = slot3(S.ut, out) + ub;
        uint32_t *lrow = slot3(S.pt, out) + lb;
        uint32_t mu = 0, ml = 0;
        // the predicate is the one that sized the segments: the counts cannot be exceeded
        narrow_candidates<TRI>(S, s, [&](uint32_t t) {
            uint32_t *row = t < s ? urow : lrow;
            uint32_t &m = t < s ? mu : ml;
            if (m >= (t < s ? nu : nl)) return;
            uint32_t q = m;
            while (q > 0 && row[q - 1] > t) { row[q] = row[q - 1]; q--; }
            row[q] = t;
            m++;
        });
        write_rows(S, s, ub, (int)mu, lb, (int)ml, [&](int q) { return q < (int)mu ? urow[q] : lrow[q - (int)mu]; });
    }
}

// Links of the new active set: upper entry (s, t), t < s, points to the
// pair (t, s) in t's lower segment (binary search), so that both spheres sum
// the one evaluation of the pair.
__global__ void __launch_bounds__(256) k_link(DevScene S) {
    Ctl *ctl = S.ctl;
    if (!due(ctl) || ctl->overflow || ctl->row_overflow) return;
    const int out = out_slot(S);
    const uint32_t *pt = slot3(S.pt, out), *lb = slot3(S.lo_beg, out), *lc = slot3(S.lo_cnt, out);
    const uint32_t *us = slot3(S.us, out), *ut = slot3(S.ut, out);
    uint32_t *um = slot3(S.um, out);
    const int64_t n = ctl->n_up;
    for (int64_t u = (int64_t)xcd_block() * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t s = us[u], t = ut[u];
        const uint32_t b0 = lb[t], cnt = lc[t];
        uint32_t lo = 0, hi = cnt;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (pt[b0 + mid] < s) lo = mid + 1; else hi = mid;
        }
        if (lo < cnt && pt[b0 + lo] == s) um[u] = b0 + lo;
        else ctl->asym = 1;  // segments not symmetric: the step is abandoned
    }
}

// Tangential history of the new set, one lane per new pair (s, t): a pair
// present in s's lower segment of the set in use keeps its history (binary
// search), a new pair starts at zero.  Reads history buffer hb (laid out for
// the set in use), writes buffer hb ^ 1 (laid out for the new set).  Only a
// detection on the step's stream carries: the second stream's set takes the
// history when it is adopted (the steps go on changing it meanwhile).
__global__ void __launch_bounds__(256) k_carry(DevScene S) {
    Ctl *ctl = S.ctl;
    if (!due(ctl) || ctl->overflow || ctl->row_overflow) return;
    const int out = out_slot(S), cur = ctl->buf, hb = ctl->hb;
    const uint32_t *nps = slot3(S.ps, out), *npt = slot3(S.pt, out);
    const uint32_t *olb = slot3(S.lo_beg, cur), *olc = slot3(S.lo_cnt, cur), *opt = slot3(S.pt, cur);
    const double *oh = pick(S.hist, hb);
    double *nh = pick(S.hist, hb ^ 1);
    const int64_t n = min(ctl->n_pairs, S.cap);
    for (int64_t p = (int64_t)xcd_block() * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t s = nps[p], t = npt[p];
        double h0 = 0.0, h1 = 0.0, h2 = 0.0;
        if (s < (uint32_t)S.ns) {
            const uint32_t b0 = olb[s], cnt = olc[s];
            uint32_t lo = 0, hi = cnt;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (opt[b0 + mid] < t) lo = mid + 1; else hi = mid;
            }
            if (lo < cnt && opt[b0 + lo] == t) {
                const double *h = oh + 3 * ((int64_t)b0 + lo);
                h0 = h[0]; h1 = h[1]; h2 = h[2];
            }
        }
        nh[3 * p] = h0; nh[3 * p + 1] = h1; nh[3 * p + 2] = h2;
    }
}

__global__ void k_detect_end(DevScene S) {
    Ctl *c = S.ctl;
    if (!due(c) || c->overflow) return;
    if (c->n_pairs - c->n_bp != c->n_up) c->asym = 1;  // every sphere pair has exactly one upper entry
    if (c->row_overflow || c->asym) { c->overflow = 1; return; }
    if (S.bchain) {  // the second stream's set waits for its adoption
        c->det_due = 0;
        return;
    }
    if (c->guard && !c->det_due) c->guard_trips++;
    c->buf = out_slot(S);
    c->hb ^= 1;
    c->n_up_cur = c->n_up;
    c->n_pairs_cur = c->n_pairs;
    c->detections++;
    c->since_det = 0;
    c->det_due = 0;
    c->guard = 0;
}

// Instantiated per force precision, kind of positions and presence of
// triangles, so that each scene runs a pair kernel without the others' code.
template <bool FP32, int FX, bool TRI>
__global__ void __launch_bounds__(256) k_pairs(DevScene S) {
    pairs_body<FP32, HertzMindlin, FX, TRI>(S);
}

// Contact sides of the last evaluated step (each sphere pair in contact counts
// twice, a boundary contact once), from the pairs' contact flags; one partial
// per workgroup.
template <bool FP32>
__global__ void __launch_bounds__(256) k_count_contacts(DevScene S, unsigned long long *part) {
    using V = typename Contrib<FP32>::V;
    const V *cS = (const V *)S.cS;
    const uint32_t *pt = slot3(S.pt, S.ctl->buf);
    const int64_t n = S.ctl->n_pairs_cur;
    unsigned long long v = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        if (cS[e].w != 0) v += pt[e] < (uint32_t)S.ns ? 2 : 1;
    __shared__ unsigned long long sh[4];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// Force and torque on sphere s from its contacts, summed in ascending
// partner id: the upper segment (partners below s; the pair's force on s is
// minus the stored force on the partner), then the lower segment (partners
// above s, boundaries last).
template <bool FP32>
__device__ __forceinline__ void sphere_sum(const DevScene &S, uint32_t ub, uint32_t nu, uint32_t lb, uint32_t nl,
                                           double *Fs, double *Ts) {
    using V = typename Contrib<FP32>::V;
    using T = typename Contrib<FP32>::T;
    const V *cS = (const V *)S.cS;
    const T *cTs = (const T *)S.cTs, *cTt = (const T *)S.cTt;
    const uint32_t *um = slot3(S.um, S.ctl->buf);
    // Entries are taken in batches whose loads are all issued before the first
    // is used (the sums stay in ascending partner order).  Six per batch keep
    // the reduction at five waves per SIMD with no spilled register (eight
    // spill; holding the first lower batch through the upper one spills too).
    constexpr uint32_t kB = 6;
    V la[kB];
    T lt[kB];
    for (uint32_t k0 = 0; k0 < nu; k0 += kB) {
        int64_t e[kB];
#pragma unroll
        for (uint32_t j = 0; j < kB; j++) e[j] = k0 + j < nu ? (int64_t)um[ub + k0 + j] : -1;
        V a[kB];
        T b[kB];
#pragma unroll
        for (uint32_t j = 0; j < kB; j++)
            if (e[j] >= 0) { a[j] = cS[e[j]]; b[j] = cTt[e[j]]; }
#pragma unroll
        for (uint32_t j = 0; j < kB; j++) {
            if (e[j] < 0 || a[j].w == 0) continue;
            Fs[0] = Fs[0] + (double)(-a[j].x); Fs[1] = Fs[1] + (double)(-a[j].y); Fs[2] = Fs[2] + (double)(-a[j].z);
            Ts[0] = Ts[0] + (double)b[j].x; Ts[1] = Ts[1] + (double)b[j].y; Ts[2] = Ts[2] + (double)b[j].z;
        }
    }
    for (uint32_t k0 = 0; k0 < nl; k0 += kB) {
#pragma unroll
        for (uint32_t j = 0; j < kB; j++)
            if (k0 + j < nl) { la[j] = cS[(int64_t)lb + k0 + j]; lt[j] = cTs[(int64_t)lb + k0 + j]; }
#pragma unroll
        for (uint32_t j = 0; j < kB; j++) {
            if (k0 + j >= nl || la[j].w == 0) continue;
            Fs[0] = Fs[0] + (double)la[j].x; Fs[1] = Fs[1] + (double)la[j].y; Fs[2] = Fs[2] + (double)la[j].z;
            Ts[0] = Ts[0] + (double)lt[j].x; Ts[1] = Ts[1] + (double)lt[j].y; Ts[2] = Ts[2] + (double)lt[j].z;
        }
    }
}

// Symplectic Euler of clump c from the sum F, T of its contact forces and
// torques (world frame), plus gravity; the record is read and rewritten in
// place.  Returns an acceleration envelope of its spheres, |a_c| + |dw/dt|
// r_acc + |w|^2 r_acc.  `pose` takes the new CoM and orientation (x', q')
// and the old ones (x, q), `rctr` the bound r_ctr on the distance of a sphere
// centre from the CoM (both are private arrays of the caller, never null: a
// null test on them would keep them out of registers).
__device__ __forceinline__ float integrate_clump(const DevScene &S, int64_t c, double *F, const double *T,
                                                 double *pose, double *rctr) {
    const double h = S.h;
    double4 *rec = S.cst + 4 * c;
    const double4 k0 = rec[0], k1 = rec[1], k2 = rec[2], k3 = rec[3];
    const int32_t pi = S.presc[c];
    const Grid &g = S.grids[S.clump_scene[c]];
    const double M = k0.w;
    F[0] = F[0] + M * g.gx; F[1] = F[1] + M * g.gy; F[2] = F[2] + M * g.gz;
    if (S.ctl->record)
        for (int i = 0; i < 3; i++) { S.rec_cF[3 * c + i] = F[i]; S.rec_cT[3 * c + i] = T[i]; }
    double A[9];
    quat_mat(k2.x, k2.y, k2.z, k2.w, A);
    double v[3] = {k1.x, k1.y, k1.z}, x[3] = {k0.x, k0.y, k0.z};
    double w[3] = {k3.x, k3.y, k3.z};
    bool pos_ok;
    if (pi < 0) {
        const double4 mi = S.tmpl_mi[S.clump_tmpl[c]];
        for (int i = 0; i < 3; i++) v[i] = v[i] + h * (F[i] / M);
        pos_ok = advance_position(S, x, v);
        double I[3] = {mi.y, mi.z, mi.w};
        double tb[3];
        for (int i = 0; i < 3; i++) tb[i] = A[i] * T[0] + A[3 + i] * T[1] + A[6 + i] * T[2];
        double L[3] = {I[0] * w[0], I[1] * w[1], I[2] * w[2]};
        double gy[3];
        cross3(w, L, gy);
        for (int i = 0; i < 3; i++) w[i] = w[i] + h * ((tb[i] - gy[i]) / I[i]);
    } else {
        const double *P = S.presc_param + 12 * pi;
        for (int i = 0; i < 3; i++) {
            if (P[3 + i] != 0.0) v[i] = v[i] + h * ((F[i] + P[9 + i]) / M);
            else v[i] = P[i];
        }
        pos_ok = advance_position(S, x, v);
        for (int i = 0; i < 3; i++) w[i] = P[6 + i];
    }
    double acc_env = 0.0;
    {
        double dv0 = v[0] - k1.x, dv1 = v[1] - k1.y, dv2 = v[2] - k1.z;
        double dw0 = w[0] - k3.x, dw1 = w[1] - k3.y, dw2 = w[2] - k3.z;
        double rb = k1.w;
        acc_env = (sqrt(dv0 * dv0 + dv1 * dv1 + dv2 * dv2) + rb * sqrt(dw0 * dw0 + dw1 * dw1 + dw2 * dw2)) / h +
                  rb * (w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    }
    double q[4] = {k2.x, k2.y, k2.z, k2.w};
    double dq[4];
    dq[0] = -(q[1] * w[0] + q[2] * w[1] + q[3] * w[2]);
    dq[1] = q[0] * w[0] + q[2] * w[2] - q[3] * w[1];
    dq[2] = q[0] * w[1] + q[3] * w[0] - q[1] * w[2];
    dq[3] = q[0] * w[2] + q[1] * w[1] - q[2] * w[0];
    double hh = 0.5 * h;
    for (int i = 0; i < 4; i++) q[i] = q[i] + hh * dq[i];
    double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int i = 0; i < 4; i++) q[i] = q[i] / qn;
    rec[0] = make_double4(x[0], x[1], x[2], M);
    rec[1] = make_double4(v[0], v[1], v[2], k1.w);
    rec[2] = make_double4(q[0], q[1], q[2], q[3]);
    rec[3] = make_double4(w[0], w[1], w[2], k3.w);
    {
        for (int i = 0; i < 3; i++) pose[i] = x[i];
        for (int i = 0; i < 4; i++) pose[3 + i] = q[i];
        pose[7] = k0.x; pose[8] = k0.y; pose[9] = k0.z;
        pose[10] = k2.x; pose[11] = k2.y; pose[12] = k2.z; pose[13] = k2.w;
    }
    *rctr = k3.w;
    const bool x_ok = S.pos_exp ? pos_ok : (isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]));
    if (!(x_ok && isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]) && isfinite(w[0]) && isfinite(w[1]) &&
          isfinite(w[2])))
        S.ctl->nonfinite = 1;
    float aenv = (float)acc_env * 1.000001f;
    if (S.store_acc) S.cacc[c] = aenv;
    return aenv;
}

// One lane per sphere.  Waves are scheduled on clump boundaries (wave w
// covers the spheres wave_s[2w] .. wave_s[2w+1]-1, whole clumps, at most 64
// spheres, starting with clump wave_c[w]), so the spheres of a clump sit in
// adjacent lanes: each lane sums its sphere's row, then the clump's first
// lane sums its spheres in ascending id by shuffles and integrates the clump.
template <bool FP32>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8))) k_reduce_waves(DevScene S) {
    if (aborted(S.ctl)) return;
    const int lane = threadIdx.x & 63;
    const int64_t w = (int64_t)xcd_block() * 4 + (threadIdx.x >> 6);
    // a wave past the schedule has no sphere, but still joins the workgroup's flag reduction
    const bool live = w < S.n_waves;
    const int64_t S0 = live ? S.wave_s[2 * w] : 0, S1 = live ? S.wave_s[2 * w + 1] : 0;
    const int64_t s = S0 + lane;
    const bool active = s < S1;
    const int cur = S.ctl->buf;
    // on the step of a detection the guard takes the detection's poses
    const bool fresh = S.guard_on && S.ctl->since_det == 0;
    uint32_t info = 0, ub = 0, nu = 0, lb = 0, nl = 0;
    uint32_t c0 = 0;
    float m = 3.0e38f;
    if (active) {
        info = S.sinfo[s];
        ub = slot3(S.up_beg, cur)[s]; nu = slot3(S.up_cnt, cur)[s];
        lb = slot3(S.lo_beg, cur)[s]; nl = slot3(S.lo_cnt, cur)[s];
        if (fresh) m = slot3(S.smargin, cur)[s];
    }
    if (live) c0 = S.wave_c[w];
    const int cnt = (int)(info >> 8);  // the clump's sphere count
    double Fs[3] = {0.0, 0.0, 0.0}, Ts[3] = {0.0, 0.0, 0.0};
    if (active) sphere_sum<FP32>(S, ub, nu, lb, nl, Fs, Ts);
    const bool leader = active && (info & 0xffu) == 0;
    // the leader's clump: the wave's first clump plus the leaders in lanes below
    const unsigned long long leaders = __ballot(leader);
    const int64_t c = (int64_t)c0 + __popcll(leaders & ((1ull << lane) - 1ull));
    // the clump sums, through LDS: each lane stores its sphere's sums, the
    // leader adds its clump's lanes in ascending order (the wave only reads
    // what its own lanes wrote, so no barrier is needed, only program order)
    // one LDS buffer: rows 0-2 carry the sums, later rows 0-6 the poses
    __shared__ double2 xs[7][256];
    xs[0][threadIdx.x] = make_double2(Fs[0], Fs[1]);
    xs[1][threadIdx.x] = make_double2(Fs[2], Ts[0]);
    xs[2][threadIdx.x] = make_double2(Ts[1], Ts[2]);
    if (fresh) xs[3][threadIdx.x] = make_double2((double)m, 0.0);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double Fc[3], Tc[3];
    for (int i = 0; i < 3; i++) { Fc[i] = 0.0 + Fs[i]; Tc[i] = 0.0 + Ts[i]; }
    double mmin = (double)m;  // the clump's smallest margin (steps of a detection)
    if (leader) {
        for (int j = 1; j < cnt; j++) {
            const double2 a = xs[0][threadIdx.x + j], b = xs[1][threadIdx.x + j], d = xs[2][threadIdx.x + j];
            Fc[0] = Fc[0] + a.x; Fc[1] = Fc[1] + a.y; Fc[2] = Fc[2] + b.x;
            Tc[0] = Tc[0] + b.y; Tc[1] = Tc[1] + d.x; Tc[2] = Tc[2] + d.y;
        }
        if (fresh)
            for (int j = 1; j < cnt; j++) mmin = fmin(mmin, xs[3][threadIdx.x + j].x);
    }
    float acc = 0.0f;
    // leader: the new CoM and orientation, then those at the last detection
    double g[14];
#pragma unroll
    for (int i = 0; i < 14; i++) g[i] = 0.0;
    double rc = 0.0;
    uint32_t tb = 0;
    bool exact = false;  // the leader's clump needs the per-sphere test
    if (leader) {
        acc = integrate_clump(S, c, Fc, Tc, g, &rc);
        if (S.guard_on) {
            double4 *cd = S.cdet + 2 * c;
            if (fresh) {  // the detection saw the state before this step's update
                cd[0] = make_double4(g[7], g[8], g[9], mmin);
                cd[1] = make_double4(g[10], g[11], g[12], g[13]);
                exact = true;
            } else {
                const double4 d0 = cd[0], d1 = cd[1];
                g[7] = d0.x; g[8] = d0.y; g[9] = d0.z;
                g[10] = d1.x; g[11] = d1.y; g[12] = d1.z; g[13] = d1.w;
                // A bound on every sphere's displacement: the CoM's, plus
                // 2 sin(theta/2) r_ctr for the rotation theta between the two
                // orientations (|sin(theta/2)| is the norm of the vector part
                // of conj(q_det) q).  Below 0.999 times the clump's smallest
                // margin, with room for the rounding of either side, no
                // sphere can trip and the per-sphere test is skipped.
                const double ex = S.pos_exp ? fx_diff(S, g[0], d0.x) : g[0] - d0.x;
                const double ey = S.pos_exp ? fx_diff(S, g[1], d0.y) : g[1] - d0.y;
                const double ez = S.pos_exp ? fx_diff(S, g[2], d0.z) : g[2] - d0.z;
                const double vx = d1.x * g[4] - g[3] * d1.y - (d1.z * g[6] - d1.w * g[5]);
                const double vy = d1.x * g[5] - g[3] * d1.z - (d1.w * g[4] - d1.y * g[6]);
                const double vz = d1.x * g[6] - g[3] * d1.w - (d1.y * g[5] - d1.z * g[4]);
                const double bound = sqrt(ex * ex + ey * ey + ez * ez) +
                                     2.0 * sqrt(vx * vx + vy * vy + vz * vz) * rc;
                exact = S.guard_exact || !(bound * (1.0 + 1e-9) + 1e-12 < 0.999 * d0.w);
            }
            if (exact) tb = S.tmpl_sbeg[S.clump_tmpl[c]];
        }
    }
    // Displacement guard: every sphere's centre now against where it stood at
    // the last detection (both from its clump's pose, the same arithmetic as
    // every other pose), tripping at 0.999 times its margin; a wavefront
    // whose clumps all pass the bound above skips it.
    bool trip = false;
    if (S.guard_on && __ballot(exact) != 0) {
        // the leader's poses to its lanes, through LDS (after every leader of
        // the wave has read the sums)
        double2(*gs)[256] = xs;
        __shared__ uint32_t tbs[256];
        if (leader) {
#pragma unroll
            for (int i = 0; i < 7; i++) gs[i][threadIdx.x] = make_double2(g[2 * i], g[2 * i + 1]);
            tbs[threadIdx.x] = exact ? tb : 0xffffffffu;  // all ones: the clump passed the bound
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int ldr = (int)threadIdx.x - (int)(info & 0xffu);
        const uint32_t tbl = active ? tbs[ldr] : 0xffffffffu;
        if (tbl != 0xffffffffu) {
            if (!fresh) m = slot3(S.smargin, cur)[s];
#pragma unroll
            for (int i = 0; i < 7; i++) { const double2 v = gs[i][ldr]; g[2 * i] = v.x; g[2 * i + 1] = v.y; }
            const uint32_t ts = tbl + (info & 0xffu);
            const double o0 = S.tmpl_ofs[3 * ts], o1 = S.tmpl_ofs[3 * ts + 1], o2 = S.tmpl_ofs[3 * ts + 2];
            double A[9], D[9];
            quat_mat(g[3], g[4], g[5], g[6], A);
            quat_mat(g[10], g[11], g[12], g[13], D);
            const double ax = A[0] * o0 + A[1] * o1 + A[2] * o2, ay = A[3] * o0 + A[4] * o1 + A[5] * o2,
                         az = A[6] * o0 + A[7] * o1 + A[8] * o2;
            const double bx = D[0] * o0 + D[1] * o1 + D[2] * o2, by = D[3] * o0 + D[4] * o1 + D[5] * o2,
                         bz = D[6] * o0 + D[7] * o1 + D[8] * o2;
            double dx, dy, dz;
            if (S.pos_exp) {  // the exact CoM displacement plus that of the rotated offset
                dx = fx_diff(S, g[0], g[7]) + (ax - bx);
                dy = fx_diff(S, g[1], g[8]) + (ay - by);
                dz = fx_diff(S, g[2], g[9]) + (az - bz);
            } else {
                dx = (g[0] + ax) - (g[7] + bx);
                dy = (g[1] + ay) - (g[8] + by);
                dz = (g[2] + az) - (g[9] + bz);
            }
            const double lim = 0.999 * (double)m;
            trip = !(dx * dx + dy * dy + dz * dz < lim * lim);
        }
    }
    // workgroup partials of the acceleration maximum and the guard, reduced by k_step_end
    __shared__ float pa[4];
    __shared__ uint32_t pt_[4];
    float am = acc;
    for (int off = 32; off > 0; off >>= 1) am = fmaxf(am, __shfl_xor(am, off, 64));
    const unsigned long long trips = __ballot(trip);
    if (lane == 0) { pa[threadIdx.x >> 6] = am; pt_[threadIdx.x >> 6] = trips != 0; }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t *o = S.part_r + 3 * (int64_t)blockIdx.x;
        o[0] = __float_as_uint(fmaxf(fmaxf(pa[0], pa[1]), fmaxf(pa[2], pa[3])));
        o[1] = 0u;
        o[2] = pt_[0] | pt_[1] | pt_[2] | pt_[3];
    }
}

// Clumps with many spheres (a wheel): per-sphere sums first, then one workgroup
// per clump sums them (in ascending sphere id in the all-FP64 mode, in a
// fixed tree order otherwise) and integrates.
template <bool FP32>
__global__ void __launch_bounds__(256) k_reduce_big_spheres(DevScene S) {
    if (aborted(S.ctl)) return;
    int32_t c = S.big_list[blockIdx.y];
    int64_t s0 = S.sbeg[c], s1 = S.sbeg[c + 1];
    const int cur = S.ctl->buf;
    for (int64_t s = s0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < s1; s += (int64_t)gridDim.x * blockDim.x) {
        double Fs[3] = {0.0, 0.0, 0.0}, Ts[3] = {0.0, 0.0, 0.0};
        sphere_sum<FP32>(S, slot3(S.up_beg, cur)[s], slot3(S.up_cnt, cur)[s], slot3(S.lo_beg, cur)[s],
                         slot3(S.lo_cnt, cur)[s], Fs, Ts);
        for (int i = 0; i < 3; i++) { S.sF[3 * s + i] = Fs[i]; S.sT[3 * s + i] = Ts[i]; }
    }
}

__global__ void __launch_bounds__(256) k_integrate_big(DevScene S) {
    if (aborted(S.ctl)) return;
    __shared__ double sh[6][256];
    int32_t c = S.big_list[blockIdx.x];
    int64_t s0 = S.sbeg[c], s1 = S.sbeg[c + 1];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    if (S.precision != 1) {
        // all-FP64 mode (precision 1 is FP32 force): the spheres in ascending id, as for every other clump
        // (256 sphere sums at a time staged in LDS, added in order by one lane)
        for (int64_t b = s0; b < s1; b += blockDim.x) {
            const int64_t s = b + threadIdx.x;
            if (s < s1)
                for (int i = 0; i < 3; i++) { sh[i][threadIdx.x] = S.sF[3 * s + i]; sh[3 + i][threadIdx.x] = S.sT[3 * s + i]; }
            __syncthreads();
            if (threadIdx.x == 0) {
                const int n = (int)(s1 - b < (int64_t)blockDim.x ? s1 - b : (int64_t)blockDim.x);
                for (int j = 0; j < n; j++)
                    for (int i = 0; i < 6; i++) acc[i] = acc[i] + sh[i][j];
            }
            __syncthreads();
        }
    } else {
        // FP32-force mode: a fixed tree order (the same every run)
        for (int64_t s = s0 + threadIdx.x; s < s1; s += blockDim.x)
            for (int i = 0; i < 3; i++) { acc[i] = acc[i] + S.sF[3 * s + i]; acc[3 + i] = acc[3 + i] + S.sT[3 * s + i]; }
        for (int i = 0; i < 6; i++) sh[i][threadIdx.x] = acc[i];
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w)
                for (int i = 0; i < 6; i++) sh[i][threadIdx.x] = sh[i][threadIdx.x] + sh[i][threadIdx.x + w];
            __syncthreads();
        }
        for (int i = 0; i < 6; i++) acc[i] = sh[i][0];
    }
    if (threadIdx.x == 0) {
        double Fc[3] = {acc[0], acc[1], acc[2]}, Tc[3] = {acc[3], acc[4], acc[5]};
        double pose[14], rc;  // unused
        float a = integrate_clump(S, c, Fc, Tc, pose, &rc);
        if (S.detect_mode != 0 && a > __uint_as_float(S.ctl->amax_bits)) atomicMax(&S.ctl->amax_bits, __float_as_uint(a));
    }
}

// Guard of the clumps too big for one wavefront, after their integration,
// one slice of spheres per workgroup.  Such a clump turns its far spheres
// through regions of very different margins (a wheel), so, as for every
// other clump, each sphere's displacement since the detection (its pose then
// is saved on the step of the detection) is held against 0.999 times its own
// margin.
__global__ void __launch_bounds__(256) k_guard_big(DevScene S) {
    if (aborted(S.ctl) || !S.guard_on) return;
    const int32_t c = S.big_list[blockIdx.y];
    const int64_t s0 = S.sbeg[c], s1 = S.sbeg[c + 1];
    const bool fresh = S.ctl->since_det == 0;
    const double4 k0 = S.cst[4 * (int64_t)c], k2 = S.cst[4 * (int64_t)c + 2];
    double A[9];
    quat_mat(k2.x, k2.y, k2.z, k2.w, A);
    double nx[3] = {k0.x, k0.y, k0.z};
    if (S.pos_exp)
        for (int i = 0; i < 3; i++) nx[i] = fx_decode(S, fx_bits(nx[i]));
    const uint32_t tb = S.tmpl_sbeg[S.clump_tmpl[c]];
    double4 *det = S.bdet + S.big_sbeg[blockIdx.y];
    int trip = 0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < s1 - s0; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = s0 + k;
        const uint32_t ts = tb + (uint32_t)k;
        const double o0 = S.tmpl_ofs[3 * ts], o1 = S.tmpl_ofs[3 * ts + 1], o2 = S.tmpl_ofs[3 * ts + 2];
        const double xs = nx[0] + (A[0] * o0 + A[1] * o1 + A[2] * o2);
        const double ys = nx[1] + (A[3] * o0 + A[4] * o1 + A[5] * o2);
        const double zs = nx[2] + (A[6] * o0 + A[7] * o1 + A[8] * o2);
        double4 d;
        if (fresh) { d = S.spos[s]; det[k] = d; }
        else d = det[k];
        const double dx = xs - d.x, dy = ys - d.y, dz = zs - d.z;
        double lim = 0.999 * (double)slot3(S.smargin, S.ctl->buf)[s];
        // fixed-point positions: world centres, so less the rounding of their coordinates
        if (S.pos_exp) lim = lim - ldexp(fmax(fmax(fabs(xs), fabs(ys)), fabs(zs)) + 1.0, -48);
        if (!(dx * dx + dy * dy + dz * dz < lim * lim) || !(lim > 0.0)) trip = 1;
    }
    if (__syncthreads_or(trip) && threadIdx.x == 0) S.ctl->guard_next = 1;
}

// The reduction's workgroup partials folded into kFold partials (maxima are
// of non-negative floats, so their bit patterns order like the values).
constexpr int kFold = 256;
__global__ void __launch_bounds__(256) k_fold_partials(DevScene S) {
    if (S.ctl->overflow) return;
    uint32_t am = 0, vm = 0, tr = 0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < S.n_rblocks; k += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t *o = S.part_r + 3 * k;
        am = max(am, o[0]);
        vm = max(vm, o[1]);
        tr |= o[2];
    }
    __shared__ uint32_t sh[3][4];
    for (int off = 32; off > 0; off >>= 1) {
        am = max(am, (uint32_t)__shfl_xor((int)am, off, 64));
        vm = max(vm, (uint32_t)__shfl_xor((int)vm, off, 64));
        tr |= (uint32_t)__shfl_xor((int)tr, off, 64);
    }
    if ((threadIdx.x & 63) == 0) { sh[0][threadIdx.x >> 6] = am; sh[1][threadIdx.x >> 6] = vm; sh[2][threadIdx.x >> 6] = tr; }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t *o = S.part_r + 3 * (S.n_rblocks + blockIdx.x);
        o[0] = max(max(sh[0][0], sh[0][1]), max(sh[0][2], sh[0][3]));
        o[1] = max(max(sh[1][0], sh[1][1]), max(sh[1][2], sh[1][3]));
        o[2] = sh[2][0] | sh[2][1] | sh[2][2] | sh[2][3];
    }
}

// End of step: fold the partials of the reduction, then the schedule.  One
// workgroup.
__global__ void __launch_bounds__(1024) k_step_end(DevScene S) {
    Ctl *c = S.ctl;
    const bool ok = !c->overflow;
    uint32_t am = 0, vm = 0, tr = 0;
    if (ok && S.n_rblocks > 0)
        for (int64_t k = threadIdx.x; k < kFold; k += blockDim.x) {
            const uint32_t *o = S.part_r + 3 * (S.n_rblocks + k);
            am = max(am, o[0]);
            vm = max(vm, o[1]);
            tr |= o[2];
        }
    __shared__ uint32_t sh[3][16];
    for (int off = 32; off > 0; off >>= 1) {
        am = max(am, (uint32_t)__shfl_xor((int)am, off, 64));
        vm = max(vm, (uint32_t)__shfl_xor((int)vm, off, 64));
        tr |= (uint32_t)__shfl_xor((int)tr, off, 64);
    }
    if ((threadIdx.x & 63) == 0) { sh[0][threadIdx.x >> 6] = am; sh[1][threadIdx.x >> 6] = vm; sh[2][threadIdx.x >> 6] = tr; }
    __syncthreads();
    // contact sides of the step, from the pair kernel's workgroups
    unsigned long long ncs = 0;
    if (ok) {
        const unsigned pb = pair_blocks(S.cap, S.stride_cap);
        for (unsigned k = threadIdx.x; k < pb; k += blockDim.x) ncs += S.part_c[k];
    }
    for (int off = 32; off > 0; off >>= 1) ncs += __shfl_xor(ncs, off, 64);
    __shared__ unsigned long long shc[16];
    if ((threadIdx.x & 63) == 0) shc[threadIdx.x >> 6] = ncs;
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int k = 1; k < (int)(blockDim.x >> 6); k++) {
        am = max(am, sh[0][k]); vm = max(vm, sh[1][k]); tr |= sh[2][k]; ncs += shc[k];
    }
    am = max(am, sh[0][0]); vm = max(vm, sh[1][0]); tr |= sh[2][0];
    const int32_t rec_mode = c->record;
    c->record = 0;
    if (!ok) return;
    if (rec_mode) c->rec_last = rec_mode;
    c->contact_sides_last = (int64_t)ncs;
    // the clumps too big for one wavefront report through the atomic slots
    c->amax_last = S.detect_mode != 0 ? max(c->amax_bits, am) : 0u;
    c->amax_bits = 0;
    (void)vm;
    c->vmax_bits = 0;  // measured again by k_pose when the next detection needs it
    c->guard = (c->guard_next | (int32_t)tr) != 0;
    c->guard_next = 0;
    c->step++;
    c->since_det++;
    c->det_due = (S.detect_mode == 0 || (!S.overlap && c->since_det >= c->k_cur)) ? 1 : 0;
    // meshes follow their prescribed motion: x += h v, and the orientation
    // turns at the world angular velocity, q += (h/2) (0, w) (x) q, renormalised
    const double h = S.h, hh = 0.5 * S.h;
    for (int32_t k = 0; k < S.n_mesh; k++) {
        Mesh &m = S.mesh[k];
        for (int i = 0; i < 3; i++) m.x[i] = m.x[i] + h * m.v[i];
        const double *w = m.w, *q = m.q;
        double dq[4];
        dq[0] = -(w[0] * q[1] + w[1] * q[2] + w[2] * q[3]);
        dq[1] = q[0] * w[0] + (w[1] * q[3] - w[2] * q[2]);
        dq[2] = q[0] * w[1] + (w[2] * q[1] - w[0] * q[3]);
        dq[3] = q[0] * w[2] + (w[0] * q[2] - w[1] * q[1]);
        double nq[4];
        for (int i = 0; i < 4; i++) nq[i] = q[i] + hh * dq[i];
        const double qn = sqrt(nq[0] * nq[0] + nq[1] * nq[1] + nq[2] * nq[2] + nq[3] * nq[3]);
        for (int i = 0; i < 4; i++) m.q[i] = nq[i] / qn;
    }
}

// ---------------------------------------------------------------- audit
// Exhaustive exact sweep: every true contact must be in the current active set.
__global__ void __launch_bounds__(256) k_audit_brute(DevScene S, unsigned long long *counts, uint32_t *first) {
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= S.ns) return;
    const int cur = S.ctl->buf;
    // every exact contact (a, b) with b above a is a pair of a's lower segment
    uint32_t beg = slot3(S.lo_beg, cur)[a], cnt = slot3(S.lo_cnt, cur)[a];
    const uint32_t *nb = slot3(S.pt, cur) + beg;
    double4 P = S.spos[a];
    uint32_t own = S.owner[a], sc = S.sscene[a];
    unsigned long long found = 0, missed = 0;
    auto check = [&](uint32_t t) {
        found++;
        uint32_t lo = 0, hi = cnt;
        while (lo < hi) { uint32_t m = (lo + hi) >> 1; if (nb[m] < t) lo = m + 1; else hi = m; }
        if (!(lo < cnt && nb[lo] == t)) {
            missed++;
            unsigned long long key = ((unsigned long long)a << 32) | t;
            atomicMin((unsigned long long *)first, key);
        }
    };
    for (int64_t b = a + 1; b < S.ns; b++) {
        if (S.owner[b] == own || S.sscene[b] != sc) continue;
        double4 Q = S.spos[b];
        double dx = Q.x - P.x, dy = Q.y - P.y, dz = Q.z - P.z;
        double d2 = dx * dx + dy * dy + dz * dz;
        double Sr = P.w + Q.w;
        if (d2 < Sr * Sr) check((uint32_t)b);
    }
    double tnow = (double)S.ctl->step * S.h;
    const Grid &g = S.grids[sc];
    for (int b = g.bnd_beg; b < g.bnd_end; b++) {
        double phi, n[3];
        if (bnd_distance(S.bnd[b], tnow, P.x, P.y, P.z, phi, n) && phi < P.w) check((uint32_t)(S.ns + b));
    }
    const double p[3] = {P.x, P.y, P.z};
    for (int64_t k = g.tri_beg; k < g.tri_end; k++) {
        double phi, n[3];
        if (tri_distance(S, k, p, phi, n) && phi < P.w) check((uint32_t)(S.ns + S.n_bnd + k));
    }
    if (found) atomicAdd(&counts[0], found);
    if (missed) atomicAdd(&counts[1], missed);
}

__global__ void k_zero(uint8_t *p, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0;
}

// ---------------------------------------------------------------- binned audit
// Exact contacts of the current positions, found in freshly built bins with no
// margin, must each be in both partners' rows of the active set.

// Sphere s's rows of the active set in use: has(t) tells whether partner t
// is in its upper (t < s) or lower segment (binary search).
struct AuditRows {
    const uint32_t *lrow, *urow;
    uint32_t lc, uc, s;
    __device__ __forceinline__ AuditRows(const DevScene &S, uint32_t s_) : s(s_) {
        const int cur = S.ctl->buf;
        lrow = slot3(S.pt, cur) + slot3(S.lo_beg, cur)[s];
        lc = slot3(S.lo_cnt, cur)[s];
        urow = slot3(S.ut, cur) + slot3(S.up_beg, cur)[s];
        uc = slot3(S.up_cnt, cur)[s];
    }
    __device__ __forceinline__ bool has(uint32_t t) const {
        const uint32_t *nb = t < s ? urow : lrow;
        const uint32_t cnt = t < s ? uc : lc;
        uint32_t lo = 0, hi = cnt;
        while (lo < hi) { uint32_t m = (lo + hi) >> 1; if (nb[m] < t) lo = m + 1; else hi = m; }
        return lo < cnt && nb[lo] == t;
    }
};

// The partner side of the audit's reach: the largest radius (no margins).
__device__ __forceinline__ double audit_reach(const Grid &g, const double4 &P) { return P.w + g.r_max + 1e-9; }

// One lane per sphere: the FP32 prefilter over the bins in reach into an LDS
// list, then the exact test over it, then the boundaries and triangles (each
// contact counted once: a sphere pair by its lower sphere; a miss by either
// side whose row lacks it).  A
// sphere with more than kMaxRow prefilter hits (or far outside its grid)
// leaves its sphere partners to k_audit_fb, so that the rare long exact pass
// does not set this kernel's registers; the scan holds only the sphere's
// FP32 view, its FP64 record and rows are read afterwards.
template <bool TRI>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) k_audit_cells(DevScene S) {
    // an abandoned step (active-set overflow) is audited when it is run again
    if (!audit_due(S) || aborted(S.ctl)) return;
    __shared__ uint32_t alst[kMaxRow * 256];  // each lane reads back only its own column
    unsigned long long found = 0, missed = 0;
    // logical blocks of 256 spheres over at most kStepGrid workgroups; one
    // partial per workgroup
    const int64_t nvb = (S.ns + 255) / 256;
    for (int64_t vb = xcd_block(); vb < nvb; vb += gridDim.x) {
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));  // nothing derived from the lane is held across iterations
        const int64_t i = vb * 256 + tid;
        if (i < S.ns) {
            const uint32_t s = (uint32_t)i;
            const Grid &g = S.grids[S.sscene[s]];
            // the FP32 prefilter of the narrow phase, without margins
            float4 Pf;
            float reach32;
            bool exact_only;
            {
                const double4 P0 = S.spos[s];
                Pf = make_float4((float)(P0.x - g.ox), (float)(P0.y - g.oy), (float)(P0.z - g.oz), (float)P0.w);
                exact_only = !(fabsf(Pf.x) < g.pre_lim && fabsf(Pf.y) < g.pre_lim && fabsf(Pf.z) < g.pre_lim);
                reach32 = (float)audit_reach(g, P0) + 2.0f * g.pre_eps;
            }
            int npre = 0;
            if (!exact_only)
                scan_reach32(S, g, Pf.x, Pf.y, Pf.z, reach32, [&](uint32_t jb, uint32_t je) {
                    slot_batches(S.sorted_f4, jb, je, [&](float4 Qf) {
                        const float fx = Qf.x - Pf.x, fy = Qf.y - Pf.y, fz = Qf.z - Pf.z, fr = (Pf.w + Qf.w) + g.pre_eps;
                        return fx * fx + fy * fy + fz * fz < fr * fr;
                    }, [&](uint32_t j) {
                        if (npre < kMaxRow) alst[npre * 256 + tid] = j;
                        npre++;
                    });
                });
            uint32_t s2 = s;
            asm volatile("" : "+v"(s2));  // fresh reads, not the values loaded before the scan
            const double4 P = S.spos[s2];
            const uint32_t own = S.owner[s2];
            const AuditRows rows(S, s2);
            if (exact_only || npre > kMaxRow) {
                const unsigned long long k = atomicAdd((unsigned long long *)&S.ctl->n_afb, 1ull);
                S.fb_list[k] = s;
            } else {
                // two listed slots at a time, their records loaded together
                for (int k = 0; k < npre; k += 2) {
                    const bool two = k + 1 < npre;
                    const uint32_t j0 = alst[k * 256 + tid], j1 = two ? alst[(k + 1) * 256 + tid] : j0;
                    const uint4 m0 = S.sorted_meta[j0], m1 = S.sorted_meta[j1];
                    const double4 Q0 = S.sorted_pos[j0], Q1 = S.sorted_pos[j1];
                    const uint32_t o0 = m0.y, o1 = m1.y, i0 = m0.x, i1 = m1.x;
                    for (int u = 0; u < (two ? 2 : 1); u++) {
                        const uint32_t o = u ? o1 : o0, id = u ? i1 : i0;
                        const double4 Q = u ? Q1 : Q0;
                        if (o == own) continue;
                        const double dx = Q.x - P.x, dy = Q.y - P.y, dz = Q.z - P.z;
                        const double d2 = dx * dx + dy * dy + dz * dz;
                        const double Sr = P.w + Q.w;
                        if (d2 < Sr * Sr) { found += id > s; if (!rows.has(id)) missed++; }
                    }
                }
            }
            double tnow = (double)S.ctl->step * S.h;
            for (int b = g.bnd_beg; b < g.bnd_end; b++) {
                double phi, n[3];
                if (bnd_distance(S.bnd[b], tnow, P.x, P.y, P.z, phi, n) && phi < P.w) {
                    found++;
                    if (!rows.has((uint32_t)(S.ns + b))) missed++;
                }
            }
            // the triangles through the boxes of the last detection: grown by
            // their meshes' margins, they hold the triangles' current positions
            if constexpr (TRI) {
                const double p[3] = {P.x, P.y, P.z};
                tri_near(S, g, p, P.w, [&](int64_t k, double) {
                    double phi, n[3];
                    if (tri_distance(S, k, p, phi, n) && phi < P.w) {
                        found++;
                        if (!rows.has((uint32_t)(S.ns + S.n_bnd + k))) missed++;
                    }
                });
            }
        }
    }
    __shared__ unsigned long long sh[2][4];
    for (int off = 32; off > 0; off >>= 1) {
        found += __shfl_xor(found, off, 64);
        missed += __shfl_xor(missed, off, 64);
    }
    if ((threadIdx.x & 63) == 0) { sh[0][threadIdx.x >> 6] = found; sh[1][threadIdx.x >> 6] = missed; }
    __syncthreads();
    if (threadIdx.x == 0) {
        S.part_a[2 * blockIdx.x] = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
        S.part_a[2 * blockIdx.x + 1] = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
    }
}

// The sphere partners of the spheres k_audit_cells left: every slot in reach
// through the prefilter (all of them far outside the grid), then the exact
// test; the counts are added to the first workgroup's partial.
template <bool TRI>
__global__ void __launch_bounds__(64) k_audit_fb(DevScene S) {
    if (!audit_due(S) || aborted(S.ctl)) return;
    unsigned long long found = 0, missed = 0;
    const int64_t n = S.ctl->n_afb;
    for (int64_t k = (int64_t)blockIdx.x * 64 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 64) {
        const uint32_t s = S.fb_list[k];
        const double4 P = S.spos[s];
        const uint32_t own = S.owner[s];
        const AuditRows rows(S, s);
        const Grid &g = S.grids[S.sscene[s]];
        const float4 Pf = make_float4((float)(P.x - g.ox), (float)(P.y - g.oy), (float)(P.z - g.oz), (float)P.w);
        const bool exact_only = !(fabsf(Pf.x) < g.pre_lim && fabsf(Pf.y) < g.pre_lim && fabsf(Pf.z) < g.pre_lim);
        scan_reach(S, g, P.x, P.y, P.z, audit_reach(g, P), [&](uint32_t jb, uint32_t je) {
            for (uint32_t j = jb; j < je; j++) {
                const float4 Qf = S.sorted_f4[j];
                const float fx = Qf.x - Pf.x, fy = Qf.y - Pf.y, fz = Qf.z - Pf.z, fr = (Pf.w + Qf.w) + g.pre_eps;
                if (!(exact_only || fx * fx + fy * fy + fz * fz < fr * fr)) continue;
                const uint4 md = S.sorted_meta[j];
                if (md.y == own) continue;
                const double4 Q = S.sorted_pos[j];
                const double dx = Q.x - P.x, dy = Q.y - P.y, dz = Q.z - P.z;
                const double d2 = dx * dx + dy * dy + dz * dz;
                const double Sr = P.w + Q.w;
                if (d2 < Sr * Sr) { found += md.x > s; if (!rows.has(md.x)) missed++; }
            }
        });
    }
    for (int off = 32; off > 0; off >>= 1) {
        found += __shfl_xor(found, off, 64);
        missed += __shfl_xor(missed, off, 64);
    }
    if (threadIdx.x == 0 && (found | missed)) {
        atomicAdd(&S.part_a[0], found);
        atomicAdd(&S.part_a[1], missed);
    }
}

__global__ void __launch_bounds__(1024) k_audit_end(DevScene S) {
    if (!audit_due(S) || aborted(S.ctl)) return;
    unsigned long long f = 0, m = 0;
    for (int64_t k = threadIdx.x; k < S.n_ablocks; k += blockDim.x) { f += S.part_a[2 * k]; m += S.part_a[2 * k + 1]; }
    __shared__ unsigned long long sh[2][16];
    for (int off = 32; off > 0; off >>= 1) { f += __shfl_xor(f, off, 64); m += __shfl_xor(m, off, 64); }
    if ((threadIdx.x & 63) == 0) { sh[0][threadIdx.x >> 6] = f; sh[1][threadIdx.x >> 6] = m; }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tf = 0, tm = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); k++) { tf += sh[0][k]; tm += sh[1][k]; }
        S.ctl->audit_true = (int64_t)tf;
        S.ctl->audit_last_missed = (int64_t)tm;
        S.ctl->audits++;
        S.ctl->missed += (int64_t)tm;
    }
}

// ---------------------------------------------------------------- detection ahead (overlap)
// The next active set is built on a second stream from a snapshot of the
// state while the steps go on (the detection of Sec. 2.2 runs in the shadow
// of the dynamics), then adopted at the start of a later step.

// Snapshot for a detection ahead: the clump records and acceleration
// envelopes of the state at the start of this step, and the second stream's
// control block reset for one detection at this step's time.  B is the
// second stream's view (its records, envelopes and control block).
__global__ void __launch_bounds__(256) k_snap(DevScene S, DevScene B) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = i; k < 4 * S.nc; k += stride) B.cst[k] = S.cst[k];
    for (int64_t k = i; k < S.nc; k += stride) B.cacc[k] = S.cacc[k];
    for (int64_t k = i; k < S.n_mesh; k += stride) B.mesh[k] = S.mesh[k];
    if (i == 0) {
        Ctl *b = B.ctl;
        const Ctl *a = S.ctl;
        b->step = a->step;
        b->amax_last = a->amax_last;
        b->vmax_bits = 0;
        b->det_due = 1; b->guard = 0;
        b->overflow = 0; b->row_overflow = 0; b->asym = 0; b->n_over = 0; b->n_fb = 0;
        b->n_up = 0; b->n_pairs = 0; b->n_bp = 0;
        b->k_cur = S.plan.k_max;
        b->fallbacks = 0;
        b->collecting = 0; b->record = 0;
        b->stale = 0;
        // the second stream's slot: any but the one in use (the step's
        // stream avoids it from now on)
        b->bslot = (a->buf + 1) % 3;
        S.ctl->bslot = b->bslot;
    }
}

// A set built ahead is usable unless its storage overflowed or a sphere
// outran its margin before the adoption.
__device__ __forceinline__ bool ahead_built(const Ctl *b) {
    return b->det_due == 0 && !b->overflow && !b->row_overflow && !b->asym;
}
__device__ __forceinline__ bool ahead_ok(const Ctl *b) { return ahead_built(b) && !b->stale; }

// Adoption, per sphere: the set built ahead (slot bctl->bslot) takes the
// tangential history of the pairs it shares with the set in use.
__global__ void __launch_bounds__(256) k_adopt_rows(DevScene S, const Ctl *bctl) {
    if (!ahead_ok(bctl) || aborted(S.ctl)) return;
    const int64_t i = (int64_t)xcd_block() * blockDim.x + threadIdx.x;
    if (i >= S.ns) return;
    const uint32_t s = (uint32_t)i;
    const int bs = bctl->bslot;
    const uint32_t lb = slot3(S.lo_beg, bs)[s];
    const int nl = (int)slot3(S.lo_cnt, bs)[s];
    const uint32_t *npt = slot3(S.pt, bs) + lb;
    carry_history(S, s, lb, nl, [&](int k) { return npt[k]; });
}

// Adoption, per clump: the displacement guard's reference becomes the
// snapshot's pose and the smallest margin the clump's spheres took (big
// clumps: the snapshot's sphere centres).  B is the second stream's view.
__global__ void __launch_bounds__(256) k_adopt_clumps(DevScene S, DevScene B) {
    if (!ahead_ok(B.ctl) || aborted(S.ctl)) return;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= S.nc) return;
    const float *m = slot3(S.smargin, B.ctl->bslot);
    float mm = 3.0e38f;
    for (int64_t s = S.sbeg[c]; s < S.sbeg[c + 1]; s++) mm = fminf(mm, m[s]);
    const double4 *r = B.cst + 4 * c;
    const double4 x = r[0], q = r[2];
    S.cdet[2 * c] = make_double4(x.x, x.y, x.z, (double)mm);
    S.cdet[2 * c + 1] = q;
}
// ... and the triangle boxes of the snapshot's detection (the binned audit
// finds the triangles through them).
__global__ void __launch_bounds__(256) k_adopt_boxes(DevScene S, DevScene B) {
    if (!ahead_ok(B.ctl) || aborted(S.ctl)) return;
    const int64_t n = 6 * (S.n_tri + S.n_chunk + S.n_scenes);
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        S.tri_box[k] = B.tri_box[k];
}
__global__ void __launch_bounds__(256) k_adopt_big(DevScene S, DevScene B) {
    if (!ahead_ok(B.ctl) || aborted(S.ctl)) return;
    const int32_t c = S.big_list[blockIdx.y];
    const int64_t s0 = S.sbeg[c], s1 = S.sbeg[c + 1];
    double4 *det = S.bdet + S.big_sbeg[blockIdx.y];
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < s1 - s0; k += (int64_t)gridDim.x * blockDim.x)
        det[k] = B.spos[s0 + k];
}

// Adoption, first the guard: the set built ahead is valid from this step on
// only if no sphere has moved 0.999 of its margin since the snapshot (the
// guard of the steps since then watched the set in use).  Otherwise it is
// not adopted (its history would miss the contacts it lost) and the set in
// use stays, with its own guard.  B is the second stream's view (its
// records are the snapshot's).
__global__ void __launch_bounds__(256) k_adopt_guard(DevScene S, DevScene B) {
    if (!ahead_built(B.ctl) || aborted(S.ctl)) return;
    const int64_t s = (int64_t)xcd_block() * blockDim.x + threadIdx.x;
    bool trip = false;
    if (s < S.ns) {
        const uint32_t c = S.owner[s], ts = S.sts[s];
        const SphereKin now = sphere_kin_of(S, c, ts), then = sphere_kin_of(B, c, ts);
        double d[3], dc[3];
        sphere_vec(S, then, now, d, dc);
        const double dx = d[0], dy = d[1], dz = d[2];
        const double lim = 0.999 * (double)slot3(S.smargin, B.ctl->bslot)[s];
        trip = !(dx * dx + dy * dy + dz * dz < lim * lim);
    }
    if (__syncthreads_or(trip) && threadIdx.x == 0) atomicOr(&B.ctl->stale, 1);
}

// Adoption, last: the set built ahead becomes the set in use (a set whose
// storage overflowed is dropped; the host grows the storage).
__global__ void k_adopt_end(DevScene S, const Ctl *bctl) {
    Ctl *c = S.ctl;
    if (aborted(c)) return;
    if (!ahead_ok(bctl)) {
        if (!ahead_built(bctl)) c->ahead_dropped = 1;  // storage too small: the host grows it
        return;
    }
    c->buf = bctl->bslot;
    c->hb ^= 1;
    c->n_up_cur = bctl->n_up;
    c->n_pairs_cur = bctl->n_pairs;
    c->detections++;
    c->fallbacks += bctl->fallbacks;
    c->since_det = 1;  // the guard's reference was set from the snapshot
}

// ---------------------------------------------------------------- launchers
static inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }
static inline unsigned capped_blocks(int64_t n, int b, int cap) {
    return (unsigned)std::min<int64_t>((n + b - 1) / b, cap);
}
// grid of a grid-stride kernel over at most n items (the count lives on the device)
static inline unsigned stride_blocks(int64_t n, int32_t cap = 16384) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, cap > 0 ? cap : 16384));
}

// ---------------------------------------------------------------- boundary forces
// Force the spheres exert on boundary blockIdx.x at the recorded step (minus
// the force on each sphere) and its torque about the boundary's reference
// point.  Workgroup (b, part) sums a contiguous range of spheres, each lane a
// contiguous sub-range in ascending id; lanes then combine in a fixed tree:
// the result is reproducible run to run.  Boundary pairs sit at the end of
// every lower segment (their partner ids exceed every sphere id).
__global__ void __launch_bounds__(256) k_bnd_partial(DevScene S, double *partial) {
    __shared__ double red[6][256];
    const uint32_t tgt = (uint32_t)S.ns + blockIdx.x;
    const int cur = S.ctl->buf;
    const uint32_t *rb = slot3(S.lo_beg, cur), *rc = slot3(S.lo_cnt, cur), *nb = slot3(S.pt, cur);
    const int64_t per_part = (S.ns + kBndParts - 1) / kBndParts;
    const int64_t p0 = (int64_t)blockIdx.y * per_part, p1 = min(S.ns, p0 + per_part);
    const int64_t per_lane = (per_part + 255) / 256;
    const int64_t s0 = p0 + (int64_t)threadIdx.x * per_lane, s1 = min(p1, s0 + per_lane);
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t s = s0; s < s1; s++) {
        const uint32_t beg = rb[s], cnt = rc[s];
        for (uint32_t k = cnt; k-- > 0;) {
            const int64_t e = (int64_t)beg + k;
            const uint32_t t = nb[e];
            if (t < (uint32_t)S.ns) break;
            if (t != tgt || S.rec_state[e] != 1 || !(S.rec_delta[e] > 0.0)) continue;
            const double f[3] = {-S.rec_F[3 * e], -S.rec_F[3 * e + 1], -S.rec_F[3 * e + 2]};
            const double r[3] = {S.rec_R[3 * e], S.rec_R[3 * e + 1], S.rec_R[3 * e + 2]};
            double tq[3];
            cross3(r, f, tq);
            for (int i = 0; i < 3; i++) { acc[i] = acc[i] + f[i]; acc[3 + i] = acc[3 + i] + tq[i]; }
        }
    }
    for (int i = 0; i < 6; i++) red[i][threadIdx.x] = acc[i];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int i = 0; i < 6; i++) red[i][threadIdx.x] = red[i][threadIdx.x] + red[i][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 6) partial[((int64_t)blockIdx.x * kBndParts + blockIdx.y) * 6 + threadIdx.x] = red[threadIdx.x][0];
}

// The triangle contacts of the recorded step, compacted: per sphere, the
// triangle partners at the end of its row (partners ascend, triangles last)
// whose contact held, appended as (sphere << 32 | partner, F, lever arm of
// the mesh) in no particular order; *count receives their number (entries
// past cap are counted, not written).
__global__ void __launch_bounds__(256) k_mesh_contacts(DevScene S, unsigned long long *keys, double *FR,
                                                       unsigned long long *count, int64_t cap) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S.ns) return;
    const int cur = S.ctl->buf;
    const uint32_t beg = slot3(S.lo_beg, cur)[s], cnt = slot3(S.lo_cnt, cur)[s];
    const uint32_t *nb = slot3(S.pt, cur);
    const uint32_t t0 = (uint32_t)(S.ns + S.n_bnd);
    for (uint32_t k = cnt; k-- > 0;) {
        const int64_t e = (int64_t)beg + k;
        const uint32_t t = nb[e];
        if (t < t0) break;
        if (S.rec_state[e] != 1 || !(S.rec_delta[e] > 0.0)) continue;
        const unsigned long long i = atomicAdd(count, 1ull);
        if ((int64_t)i >= cap) continue;
        keys[i] = ((unsigned long long)s << 32) | t;
        for (int j = 0; j < 3; j++) { FR[6 * i + j] = S.rec_F[3 * e + j]; FR[6 * i + 3 + j] = S.rec_R[3 * e + j]; }
    }
}

hipError_t launch_mesh_contacts(const DevScene &S, unsigned long long *keys, double *FR, unsigned long long *count,
                                int64_t cap, hipStream_t st) {
    if (S.ns == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mesh_contacts, dim3(blocks_for(S.ns, 256)), dim3(256), 0, st, S, keys, FR, count, cap);
    return hipGetLastError();
}

__global__ void k_bnd_final(int n_bnd, const double *partial, double *out) {
    const int b = blockIdx.x, i = threadIdx.x;
    if (b >= n_bnd || i >= 6) return;
    double a = 0.0;
    for (int p = 0; p < kBndParts; p++) a = a + partial[((int64_t)b * kBndParts + p) * 6 + i];
    out[6 * b + i] = a;
}

const char *const kKernelNames[K_COUNT] = {"k_pose", "k_detect_begin", "k_cell_count", "k_scan_reduce",
                                           "k_scan_bsum", "k_scan_final", "k_cell_scatter", "k_narrow",
                                           "k_detect_end", "k_pairs", "k_reduce_big_spheres",
                                           "k_integrate_big", "k_step_end", "k_plan", "k_audit_cells",
                                           "k_link", "k_reduce_waves", "k_bin_features", "k_bin_margin",
                                           "k_narrow_over", "k_region_margin", "k_guard_big", "k_bins_begin",
                                           "audit_total", "k_pick_interval", "k_narrow_rows", "k_narrow_base",
                                           "k_carry", "k_narrow_fb"};
KernelTimer *g_timer = nullptr;

#define TIMED(id, launch)                           \
    do {                                            \
        if (g_timer) g_timer->before((id), st);     \
        launch;                                     \
        if (g_timer) g_timer->after((id), st);      \
    } while (0)

hipError_t launch_zero(void *p, size_t bytes, hipStream_t st) {
    if (!bytes) return hipSuccess;
    unsigned nb = (unsigned)std::min<size_t>((bytes + 255) / 256, 65536);
    hipLaunchKernelGGL(k_zero, dim3(nb), dim3(256), 0, st, (uint8_t *)p, bytes);
    return hipGetLastError();
}

hipError_t launch_pose(const DevScene &S, hipStream_t st, bool force) {
    if (S.ns == 0) return hipSuccess;
    if (!force) {
        unsigned zb = (unsigned)std::min<int64_t>(blocks_for(S.n_cells, 256), 16384);
        TIMED(K_BINS_BEGIN, hipLaunchKernelGGL(k_bins_begin, dim3(zb), dim3(256), 0, st, S));
    }
    TIMED(K_POSE, hipLaunchKernelGGL(k_pose, dim3(capped_blocks(S.ns, 256, kStepGrid)), dim3(256), 0, st, S, force ? 1 : 0));
    return hipGetLastError();
}

// The second pass of the narrow phase: counts, bases, segments.
static void narrow_rows(const DevScene &S, hipStream_t st) {
    const unsigned nb = blocks_for(S.ns, kNarrowBlock);
    TIMED(K_NARROW_BASE, hipLaunchKernelGGL(k_narrow_base, dim3(1), dim3(kBaseBlock), 0, st, S, (int64_t)nb));
    TIMED(K_NARROW_ROWS, hipLaunchKernelGGL(k_narrow_rows, dim3(std::min<unsigned>(nb, kStepGrid)), dim3(kNarrowBlock), 0,
                                            st, S));
}

// Bin every sphere of the current positions.  In a step (which = 0: the
// detection, 1: the audit) the bins were cleared and counted by k_bins_begin
// and k_pose: scan and scatter (a detection first turns the learned region
// features into margins).  Training-data capture (which = 2) needs the bin
// counts and the features only: clear, count, features.
static void binning(const DevScene &S, int which, hipStream_t st) {
    if (which == 2) {
        unsigned zb = (unsigned)std::min<int64_t>(blocks_for(S.n_cells, 256), 16384);
        TIMED(K_DETECT_BEGIN, hipLaunchKernelGGL(k_detect_begin, dim3(zb), dim3(256), 0, st, S, which));
        TIMED(K_CELL_COUNT, hipLaunchKernelGGL(k_cell_count, dim3(blocks_for(S.ns, 256)), dim3(256), 0, st, S, which));
        TIMED(K_BIN_FEATURES, hipLaunchKernelGGL(k_bin_features, dim3(blocks_for(S.ns, 256)), dim3(256), 0, st, S, which));
        return;
    }
    if (which == 0 && S.detect_mode == 2) {
        const unsigned rb = region_blocks(S.n_regions);
        TIMED(K_BIN_MARGIN, hipLaunchKernelGGL(k_bin_margin, dim3(rb), dim3(256), 0, st, S));
        TIMED(K_PICK_INTERVAL, hipLaunchKernelGGL(k_pick_interval, dim3(1), dim3(256), 0, st, S, rb));
        TIMED(K_REGION_MARGIN, hipLaunchKernelGGL(k_region_margin, dim3(rb), dim3(256), 0, st, S));
    }
    int64_t nblk = (S.n_cells + kScanTile - 1) / kScanTile;
    uint32_t *bsum = S.scan_bsum;
    const unsigned sb = (unsigned)std::min<int64_t>(nblk, kStepGrid);
    TIMED(K_SCAN_REDUCE, hipLaunchKernelGGL(k_scan_reduce, dim3(sb), dim3(kScanBlock), 0, st, S, bsum, which));
    TIMED(K_SCAN_BSUM, hipLaunchKernelGGL(k_scan_bsum, dim3(1), dim3(kBsumBlock), 0, st, S, bsum, nblk, which));
    TIMED(K_SCAN_FINAL, hipLaunchKernelGGL(k_scan_final, dim3(sb), dim3(kScanBlock), 0, st, S,
                                           (const uint32_t *)bsum, which));
    TIMED(K_CELL_SCATTER, hipLaunchKernelGGL(k_cell_scatter, dim3(capped_blocks(S.ns, 256, kStepGrid)), dim3(256), 0, st, S,
                                             (const float *)nullptr, which));
}

hipError_t launch_detect(const DevScene &S, hipStream_t st) {
    if (S.ns == 0) return hipSuccess;
    TIMED(K_PLAN, hipLaunchKernelGGL(k_plan, dim3(1), dim3(1), 0, st, S));
    binning(S, 0, st);
    if (S.n_tri) {
        hipLaunchKernelGGL(k_tri_boxes, dim3(stride_blocks(S.n_chunk * 64, 1024)), dim3(256), 0, st, S);
        hipLaunchKernelGGL(k_tri_scene_boxes, dim3(S.n_scenes), dim3(256), 0, st, S);
    }
    if (S.n_tri) {
        TIMED(K_NARROW, hipLaunchKernelGGL(k_narrow<true>, dim3(blocks_for(S.ns, kNarrowBlock)), dim3(kNarrowBlock), 0, st, S));
        TIMED(K_NARROW_FB, hipLaunchKernelGGL(k_narrow_fb<true>, dim3(kFbGrid), dim3(64), 0, st, S));
        narrow_rows(S, st);
        TIMED(K_NARROW_OVER, hipLaunchKernelGGL(k_narrow_over<true>, dim3(256), dim3(64), 0, st, S));
    } else {
        TIMED(K_NARROW, hipLaunchKernelGGL(k_narrow<false>, dim3(blocks_for(S.ns, kNarrowBlock)), dim3(kNarrowBlock), 0, st, S));
        TIMED(K_NARROW_FB, hipLaunchKernelGGL(k_narrow_fb<false>, dim3(kFbGrid), dim3(64), 0, st, S));
        narrow_rows(S, st);
        TIMED(K_NARROW_OVER, hipLaunchKernelGGL(k_narrow_over<false>, dim3(256), dim3(64), 0, st, S));
    }
    TIMED(K_LINK, hipLaunchKernelGGL(k_link, dim3(stride_blocks(S.cap, S.stride_cap)), dim3(256), 0, st, S));
    if (!S.bchain)
        TIMED(K_CARRY, hipLaunchKernelGGL(k_carry, dim3(stride_blocks(S.cap, S.stride_cap)), dim3(256), 0, st, S));
    TIMED(K_DETECT_END, hipLaunchKernelGGL(k_detect_end, dim3(1), dim3(1), 0, st, S));
    return hipGetLastError();
}

hipError_t launch_snapshot(const DevScene &S, const DevScene &B, hipStream_t st) {
    if (S.nc == 0) return hipSuccess;
    hipLaunchKernelGGL(k_snap, dim3(stride_blocks(4 * S.nc)), dim3(256), 0, st, S, B);
    return hipGetLastError();
}

hipError_t launch_detect_ahead(const DevScene &B, hipStream_t st) {
    if (B.ns == 0) return hipSuccess;
    hipError_t e = launch_pose(B, st, false);  // bins and region features of the snapshot
    return e == hipSuccess ? launch_detect(B, st) : e;
}

hipError_t launch_adopt(const DevScene &S, const DevScene &B, hipStream_t st) {
    if (S.ns == 0) return hipSuccess;
    hipLaunchKernelGGL(k_adopt_guard, dim3(blocks_for(S.ns, 256)), dim3(256), 0, st, S, B);
    hipLaunchKernelGGL(k_adopt_rows, dim3(blocks_for(S.ns, 256)), dim3(256), 0, st, S, (const Ctl *)B.ctl);
    hipLaunchKernelGGL(k_adopt_clumps, dim3(blocks_for(S.nc, 256)), dim3(256), 0, st, S, B);
    if (S.n_big) hipLaunchKernelGGL(k_adopt_big, dim3(16, S.n_big), dim3(256), 0, st, S, B);
    if (S.n_tri)
        hipLaunchKernelGGL(k_adopt_boxes, dim3(stride_blocks(6 * (S.n_tri + S.n_chunk + S.n_scenes), 256)), dim3(256),
                           0, st, S, B);
    hipLaunchKernelGGL(k_adopt_end, dim3(1), dim3(1), 0, st, S, (const Ctl *)B.ctl);
    return hipGetLastError();
}

hipError_t launch_bnd_forces(const DevScene &S, double *partial, double *out, hipStream_t st) {
    if (S.n_bnd == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bnd_partial, dim3(S.n_bnd, kBndParts), dim3(256), 0, st, S, partial);
    hipLaunchKernelGGL(k_bnd_final, dim3(S.n_bnd), dim3(64), 0, st, S.n_bnd, (const double *)partial, out);
    return hipGetLastError();
}

hipError_t launch_count_contacts(const DevScene &S, unsigned long long *part, int nblk, hipStream_t st) {
    if (S.precision == 1) hipLaunchKernelGGL(k_count_contacts<true>, dim3(nblk), dim3(256), 0, st, S, part);
    else hipLaunchKernelGGL(k_count_contacts<false>, dim3(nblk), dim3(256), 0, st, S, part);
    return hipGetLastError();
}

hipError_t launch_collect_begin(const DevScene &S, hipStream_t st) {
    binning(S, 2, st);
    hipLaunchKernelGGL(k_collect_init, dim3(stride_blocks(std::max<int64_t>(S.ns, S.n_regions))), dim3(256), 0, st, S);
    return hipGetLastError();
}

hipError_t launch_collect_speed(const DevScene &S, hipStream_t st) {
    if (S.ns) hipLaunchKernelGGL(k_collect_speed, dim3(blocks_for(S.ns, 256)), dim3(256), 0, st, S);
    return hipGetLastError();
}

hipError_t launch_collect_acc(const DevScene &S, hipStream_t st) {
    if (S.ns) hipLaunchKernelGGL(k_collect_acc, dim3(blocks_for(S.ns, 256)), dim3(256), 0, st, S);
    return hipGetLastError();
}

// (the whole chain is also timed as one bracket, "audit_total": its binning,
// the exact check and the fold; the kernels do work on audit steps only)
hipError_t launch_audit_binned(const DevScene &S, hipStream_t st) {
    if (S.ns == 0 || S.plan.audit_period <= 0) return hipSuccess;
    if (g_timer) g_timer->before(K_AUDIT_ALL, st);
    binning(S, 1, st);
    if (S.n_tri) TIMED(K_AUDIT, hipLaunchKernelGGL(k_audit_cells<true>, dim3(S.n_ablocks), dim3(256), 0, st, S));
    else TIMED(K_AUDIT, hipLaunchKernelGGL(k_audit_cells<false>, dim3(S.n_ablocks), dim3(256), 0, st, S));
    if (S.n_tri) hipLaunchKernelGGL(k_audit_fb<true>, dim3(kFbGrid), dim3(64), 0, st, S);
    else hipLaunchKernelGGL(k_audit_fb<false>, dim3(kFbGrid), dim3(64), 0, st, S);
    hipLaunchKernelGGL(k_audit_end, dim3(1), dim3(1024), 0, st, S);
    if (g_timer) g_timer->after(K_AUDIT_ALL, st);
    return hipGetLastError();
}

hipError_t launch_force_integrate(const DevScene &S, hipStream_t st, hipFunction_t user_pairs) {
    if (S.nc == 0) return hipSuccess;
    const bool f32 = S.precision == 1;
    const unsigned pb = pair_blocks(S.cap, S.stride_cap);
    if (user_pairs) {
        DevScene arg = S;
        void *args[] = {&arg};
        hipError_t e = hipSuccess;
        TIMED(K_FORCE, e = hipModuleLaunchKernel(user_pairs, pb, 1, 1, 256, 1, 1, 0, st, args, nullptr));
        if (e != hipSuccess) return e;
    } else {
        const int sel = (f32 ? 4 : 0) + (S.pos_exp ? 2 : 0) + (S.n_tri ? 1 : 0);
#define CDEM_PAIRS(A, B, C) TIMED(K_FORCE, hipLaunchKernelGGL((k_pairs<A, B, C>), dim3(pb), dim3(256), 0, st, S))
        switch (sel) {
            case 0: CDEM_PAIRS(false, 0, false); break;
            case 1: CDEM_PAIRS(false, 0, true); break;
            case 2: CDEM_PAIRS(false, 1, false); break;
            case 3: CDEM_PAIRS(false, 1, true); break;
            case 4: CDEM_PAIRS(true, 0, false); break;
            case 5: CDEM_PAIRS(true, 0, true); break;
            case 6: CDEM_PAIRS(true, 1, false); break;
            default: CDEM_PAIRS(true, 1, true); break;
        }
#undef CDEM_PAIRS
    }
    unsigned wb = (unsigned)((S.n_waves + 3) / 4);
    if (wb) {
        if (f32) TIMED(K_REDUCE, hipLaunchKernelGGL(k_reduce_waves<true>, dim3(wb), dim3(256), 0, st, S));
        else TIMED(K_REDUCE, hipLaunchKernelGGL(k_reduce_waves<false>, dim3(wb), dim3(256), 0, st, S));
    }
    if (S.n_big) {
        if (f32)
            TIMED(K_FORCE_BIG, hipLaunchKernelGGL(k_reduce_big_spheres<true>, dim3(64, S.n_big), dim3(256), 0, st, S));
        else
            TIMED(K_FORCE_BIG, hipLaunchKernelGGL(k_reduce_big_spheres<false>, dim3(64, S.n_big), dim3(256), 0, st, S));
        TIMED(K_INTEGRATE_BIG, hipLaunchKernelGGL(k_integrate_big, dim3(S.n_big), dim3(256), 0, st, S));
        if (S.guard_on) TIMED(K_GUARD_BIG, hipLaunchKernelGGL(k_guard_big, dim3(16, S.n_big), dim3(256), 0, st, S));
    }
    return hipGetLastError();
}

hipError_t launch_step_end(const DevScene &S, hipStream_t st) {
    if (S.n_rblocks > 0) TIMED(K_STEP_END, hipLaunchKernelGGL(k_fold_partials, dim3(kFold), dim3(256), 0, st, S));
    TIMED(K_STEP_END, hipLaunchKernelGGL(k_step_end, dim3(1), dim3(1024), 0, st, S));
    return hipGetLastError();
}

hipError_t launch_audit_brute(const DevScene &S, unsigned long long *counts, uint32_t *first, hipStream_t st) {
    if (S.ns == 0) return hipSuccess;
    hipLaunchKernelGGL(k_audit_brute, dim3(blocks_for(S.ns, 256)), dim3(256), 0, st, S, counts, first);
    return hipGetLastError();
}

// ---------------------------------------------------------------- state transfer
// Row-major [n][3]/[n][4] device buffers <-> the clump records (null buffers
// are skipped; the static words of a record are kept).
// With fixed-point positions x is decoded on the way out and rounded to the
// grid on the way in (an x out of range leaves the position and flags the
// state as non-finite), unless `raw` copies the integers (checkpoints).
__global__ void __launch_bounds__(256) k_pack_state(DevScene S, double *x, double *q, double *v, double *w, int unpack,
                                                    int raw) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= S.nc) return;
    double4 *r = S.cst + 4 * c;
    double4 k0 = r[0], k1 = r[1], k2 = r[2], k3 = r[3];
    const bool dec = S.pos_exp && !raw;
    if (!unpack) {
        if (x && dec) {
            for (int i = 0; i < 3; i++) x[3 * c + i] = fx_decode(S, fx_bits(i == 0 ? k0.x : (i == 1 ? k0.y : k0.z)));
        } else if (x) {
            x[3 * c] = k0.x; x[3 * c + 1] = k0.y; x[3 * c + 2] = k0.z;
        }
        if (v) { v[3 * c] = k1.x; v[3 * c + 1] = k1.y; v[3 * c + 2] = k1.z; }
        if (q) { q[4 * c] = k2.x; q[4 * c + 1] = k2.y; q[4 * c + 2] = k2.z; q[4 * c + 3] = k2.w; }
        if (w) { w[3 * c] = k3.x; w[3 * c + 1] = k3.y; w[3 * c + 2] = k3.z; }
        return;
    }
    if (x && dec) {
        double e[3];
        for (int i = 0; i < 3; i++) {
            const double u = x[3 * c + i] * S.pos_inv;
            if (!(fabs(u) < (double)kFxLimit)) { S.ctl->nonfinite = 1; return; }
            e[i] = fx_slot((long long)rint(u));
        }
        k0.x = e[0]; k0.y = e[1]; k0.z = e[2];
    } else if (x) {
        k0.x = x[3 * c]; k0.y = x[3 * c + 1]; k0.z = x[3 * c + 2];
    }
    if (v) { k1.x = v[3 * c]; k1.y = v[3 * c + 1]; k1.z = v[3 * c + 2]; }
    if (q) { k2.x = q[4 * c]; k2.y = q[4 * c + 1]; k2.z = q[4 * c + 2]; k2.w = q[4 * c + 3]; }
    if (w) { k3.x = w[3 * c]; k3.y = w[3 * c + 1]; k3.z = w[3 * c + 2]; }
    r[0] = k0; r[1] = k1; r[2] = k2; r[3] = k3;
}

hipError_t launch_pack_state(const DevScene &S, double *x, double *q, double *v, double *w, int unpack, hipStream_t st,
                             int raw) {
    if (S.nc == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_state, dim3(blocks_for(S.nc, 256)), dim3(256), 0, st, S, x, q, v, w, unpack, raw);
    return hipGetLastError();
}

}  // namespace cdem
