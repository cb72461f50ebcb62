// Device helpers shared by the step kernels and the run-time compiled pair
// kernel of a user force law: control-block and buffer selection, clump
// rotation and sphere poses, analytic boundary distances, XCD-aware
// workgroup numbering.
#pragma once

#include "cdem_internal.h"

namespace cdem {

__device__ __forceinline__ bool aborted(const Ctl *c) { return c->overflow != 0; }

// Active-set buffer k of a double-buffered array.  A select keeps the pointer
// in registers; indexing the by-value kernel argument with a runtime k would
// copy the pointer pair to scratch memory.
template <typename T>
__device__ __forceinline__ T *pick(T *const (&a)[2], int k) { return k ? a[1] : a[0]; }
// Slot k of an active-set structure array (three slots).
template <typename T>
__device__ __forceinline__ T *slot3(T *const (&a)[3], int k) { return k == 0 ? a[0] : (k == 1 ? a[1] : a[2]); }
// The slot a detection writes: the second stream's own (its control block's
// bslot), or for a detection on the step's stream the slot that is neither
// in use nor reserved for the second stream.
__device__ __forceinline__ int out_slot(const DevScene &S) {
    return S.bchain ? S.ctl->bslot : 3 - S.ctl->buf - S.ctl->bslot;
}

// ---------------------------------------------------------------- rotation
__device__ __forceinline__ void quat_mat(double w, double x, double y, double z, double *A) {
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

// ---------------------------------------------------------------- fixed-point positions
// With fixed-point positions (S.pos_exp = E > 0) a clump record's CoM slots
// hold 64-bit integers k, x = k 2^-E (the high 32 bits a voxel id, the low
// 32 bits the offset in a voxel of side 2^(32-E)), stored bit for bit in the
// double slots.
__device__ __forceinline__ long long fx_bits(double d) { return __double_as_longlong(d); }
__device__ __forceinline__ double fx_slot(long long k) { return __longlong_as_double(k); }
// The world coordinate of an integer position (rounded when |k| > 2^53).
__device__ __forceinline__ double fx_decode(const DevScene &S, long long k) { return (double)k * S.pos_eps; }
// The exact difference of two integer positions (|ka - kb| < 2^53).
__device__ __forceinline__ double fx_diff(const DevScene &S, double a, double b) {
    return (double)(fx_bits(a) - fx_bits(b)) * S.pos_eps;
}
// Fixed-point positions on a code path: F = 0 never, 1 always (kernels
// instantiated for one kind of scene, with the other path compiled out),
// 2 as the scene says.
template <int FX>
__device__ __forceinline__ bool fixed_pos(const DevScene &S) { return FX == 2 ? S.pos_exp != 0 : FX == 1; }

// Integer positions stay below 2^61 in magnitude (a quarter of the range).
constexpr long long kFxLimit = 1LL << 61;
// x += h v: in FP64, or with the increment rounded to the grid (ties to
// even) and added to the integer.  Returns false when a position would leave
// its range (the position is then kept).
__device__ __forceinline__ bool advance_position(const DevScene &S, double *x, const double *v) {
    if (!S.pos_exp) {
        for (int i = 0; i < 3; i++) x[i] = x[i] + S.h * v[i];
        return true;
    }
    bool ok = true;
    for (int i = 0; i < 3; i++) {
        const double u = rint((S.h * v[i]) * S.pos_inv);
        const long long k = fx_bits(x[i]);
        if (!(fabs(u) < (double)kFxLimit) || k >= kFxLimit || k <= -kFxLimit) { ok = false; continue; }
        x[i] = fx_slot(k + (long long)u);
    }
    return ok;
}

// ---------------------------------------------------------------- pose (per sphere)
// Kinematics of sphere s from its clump's state record: centre x_s = x_c +
// A(q) o_s and radius, the rotated offset r = A(q) o_s, and the clump's CoM,
// mass, velocity and world angular velocity A(q) w_body (with fixed-point
// positions: the CoM decoded to world coordinates, and its integers in cq).
// Every kernel that needs a sphere's pose computes it this one way, so the
// positions of a detection, of the force kernel and of a readout are the same
// numbers.
struct SphereKin { double p[3], R, xc[3], M, v[3], W[3], r[3], cq[3]; };
// ... of the sphere that is template sphere ts of clump c
template <int FX = 2>
__device__ __forceinline__ SphereKin sphere_kin_of(const DevScene &S, uint32_t c, uint32_t ts) {
    const double4 *r = S.cst + 4 * (int64_t)c;
    const double4 k0 = r[0], k1 = r[1], k2 = r[2], k3 = r[3];
    const double o0 = S.tmpl_ofs[3 * ts], o1 = S.tmpl_ofs[3 * ts + 1], o2 = S.tmpl_ofs[3 * ts + 2];
    SphereKin k;
    k.R = S.tmpl_rad[ts];
    double A[9];
    quat_mat(k2.x, k2.y, k2.z, k2.w, A);
    k.r[0] = A[0] * o0 + A[1] * o1 + A[2] * o2;
    k.r[1] = A[3] * o0 + A[4] * o1 + A[5] * o2;
    k.r[2] = A[6] * o0 + A[7] * o1 + A[8] * o2;
    k.cq[0] = k0.x; k.cq[1] = k0.y; k.cq[2] = k0.z;
    if (fixed_pos<FX>(S)) {
        k.xc[0] = fx_decode(S, fx_bits(k0.x)); k.xc[1] = fx_decode(S, fx_bits(k0.y)); k.xc[2] = fx_decode(S, fx_bits(k0.z));
    } else {
        k.xc[0] = k0.x; k.xc[1] = k0.y; k.xc[2] = k0.z;
    }
    k.p[0] = k.xc[0] + k.r[0];
    k.p[1] = k.xc[1] + k.r[1];
    k.p[2] = k.xc[2] + k.r[2];
    k.M = k0.w;
    k.v[0] = k1.x; k.v[1] = k1.y; k.v[2] = k1.z;
    k.W[0] = A[0] * k3.x + A[1] * k3.y + A[2] * k3.z;
    k.W[1] = A[3] * k3.x + A[4] * k3.y + A[5] * k3.z;
    k.W[2] = A[6] * k3.x + A[7] * k3.y + A[8] * k3.z;
    return k;
}
__device__ __forceinline__ SphereKin sphere_kin(const DevScene &S, uint32_t s) {
    return sphere_kin_of(S, S.owner[s], S.sts[s]);
}
// Vector d from sphere a to sphere b: the difference of their centres, or
// with fixed-point positions the exact CoM difference dc plus the difference
// of the rotated offsets.
template <int FX = 2>
__device__ __forceinline__ void sphere_vec(const DevScene &S, const SphereKin &a, const SphereKin &b, double *d,
                                           double *dc) {
    if (fixed_pos<FX>(S)) {
        for (int i = 0; i < 3; i++) {
            dc[i] = fx_diff(S, b.cq[i], a.cq[i]);
            d[i] = dc[i] + (b.r[i] - a.r[i]);
        }
    } else {
        for (int i = 0; i < 3; i++) { d[i] = b.p[i] - a.p[i]; dc[i] = 0.0; }
    }
}


// ---------------------------------------------------------------- boundaries
// Signed distance of p from boundary b at time t (positive on the domain side)
// and the unit normal from the wall into the domain.  Returns false where the
// boundary cannot touch p.
__device__ __forceinline__ bool bnd_distance(const Bnd &B, double t, double px, double py, double pz, double &phi, double *n) {
    const double *P = B.p;
    double r0x = P[0] + t * B.vel[0], r0y = P[1] + t * B.vel[1], r0z = P[2] + t * B.vel[2];
    double d0 = px - r0x, d1 = py - r0y, d2 = pz - r0z;
    if (B.type == 0) {
        phi = d0 * P[3] + d1 * P[4] + d2 * P[5];
        n[0] = P[3]; n[1] = P[4]; n[2] = P[5];
        return true;
    }
    double a0 = P[3], a1 = P[4], a2 = P[5];
    double ta = d0 * a0 + d1 * a1 + d2 * a2;
    double rho0 = d0 - ta * a0, rho1 = d1 - ta * a1, rho2 = d2 - ta * a2;
    double r = sqrt(rho0 * rho0 + rho1 * rho1 + rho2 * rho2);
    if (B.type == 1) {
        if (!(r > 0.0)) return false;
        phi = P[6] - r;
        n[0] = -(rho0 / r); n[1] = -(rho1 / r); n[2] = -(rho2 / r);
        return true;
    }
    double sn = P[6], cs = P[7];
    if (B.type == 2) {
        double H = P[8];
        double rb = H * (sn / cs);
        double lam = ta * cs + r * sn;
        if (ta >= H) {
            if (!(r > 0.0)) return false;
            phi = r - rb;
            n[0] = rho0 / r; n[1] = rho1 / r; n[2] = rho2 / r;
            return true;
        }
        if (lam <= 0.0) {
            double dd = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
            if (!(dd > 0.0)) return false;
            phi = dd;
            n[0] = d0 / dd; n[1] = d1 / dd; n[2] = d2 / dd;
            return true;
        }
        if (!(r > 0.0)) return false;
        if (lam <= H / cs) {
            phi = r * cs - ta * sn;
            n[0] = (rho0 / r) * cs - a0 * sn;
            n[1] = (rho1 / r) * cs - a1 * sn;
            n[2] = (rho2 / r) * cs - a2 * sn;
            return true;
        }
        double dt = ta - H, dr = r - rb;
        double dd = sqrt(dt * dt + dr * dr);
        if (!(dd > 0.0)) return false;
        phi = dd;
        n[0] = (dt * a0 + dr * (rho0 / r)) / dd;
        n[1] = (dt * a1 + dr * (rho1 / r)) / dd;
        n[2] = (dt * a2 + dr * (rho2 / r)) / dd;
        return true;
    }
    if (ta < P[8] || ta > P[9] || !(r > 0.0)) return false;
    phi = ta * sn - r * cs;
    n[0] = a0 * sn - (rho0 / r) * cs;
    n[1] = a1 * sn - (rho1 / r) * cs;
    n[2] = a2 * sn - (rho2 / r) * cs;
    return true;
}

// The hardware hands workgroup i of a launch to XCD i mod 8, and each XCD has
// its own L2.  xcd_block() renumbers the workgroups so that every XCD works on
// one contiguous range of logical blocks: neighbouring items (spheres of one
// bin, pairs of nearby spheres, the spheres of a clump) then share one L2
// instead of being fetched by several.  A bijection of [0, gridDim.x).
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_block() {
    const uint32_t b = blockIdx.x, n = gridDim.x;
    const uint32_t x = b % kXcds, k = b / kXcds, per = n / kXcds, rem = n % kXcds;
    return x * per + min(x, rem) + k;
}

// ---------------------------------------------------------------- triangle meshes
// World vertices of triangle k: x_mesh + A(q_mesh) v for each vertex.
__device__ __forceinline__ void tri_world(const DevScene &S, int64_t k, double *V) {
    const Mesh &M = S.mesh[S.tri_mesh[k]];
    double A[9];
    quat_mat(M.q[0], M.q[1], M.q[2], M.q[3], A);
    const double *vb = S.tri_vb + 9 * k;
    for (int j = 0; j < 3; j++) {
        const double b0 = vb[3 * j], b1 = vb[3 * j + 1], b2 = vb[3 * j + 2];
        V[3 * j] = M.x[0] + (A[0] * b0 + A[1] * b1 + A[2] * b2);
        V[3 * j + 1] = M.x[1] + (A[3] * b0 + A[4] * b1 + A[5] * b2);
        V[3 * j + 2] = M.x[2] + (A[6] * b0 + A[7] * b1 + A[8] * b2);
    }
}

__device__ __forceinline__ double dot3d(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Closest point c of triangle (A, B, C) to p: the Voronoi region of a
// vertex, an edge or the face that holds p, found from dot products of the
// edge vectors (the region tests of Ericson, Real-Time Collision Detection,
// Sec. 5.1.5), in a fixed order.
__device__ __forceinline__ void closest_on_triangle(const double *A, const double *B, const double *C, const double *p,
                                                    double *c) {
    double ab[3], ac[3], ap[3], bp[3], cp[3];
    for (int i = 0; i < 3; i++) { ab[i] = B[i] - A[i]; ac[i] = C[i] - A[i]; ap[i] = p[i] - A[i]; }
    const double d1 = dot3d(ab, ap), d2 = dot3d(ac, ap);
    if (d1 <= 0.0 && d2 <= 0.0) { for (int i = 0; i < 3; i++) c[i] = A[i]; return; }
    for (int i = 0; i < 3; i++) bp[i] = p[i] - B[i];
    const double d3 = dot3d(ab, bp), d4 = dot3d(ac, bp);
    if (d3 >= 0.0 && d4 <= d3) { for (int i = 0; i < 3; i++) c[i] = B[i]; return; }
    const double vc = d1 * d4 - d3 * d2;
    if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
        const double v = d1 / (d1 - d3);
        for (int i = 0; i < 3; i++) c[i] = A[i] + v * ab[i];
        return;
    }
    for (int i = 0; i < 3; i++) cp[i] = p[i] - C[i];
    const double d5 = dot3d(ab, cp), d6 = dot3d(ac, cp);
    if (d6 >= 0.0 && d5 <= d6) { for (int i = 0; i < 3; i++) c[i] = C[i]; return; }
    const double vb = d5 * d2 - d1 * d6;
    if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
        const double w = d2 / (d2 - d6);
        for (int i = 0; i < 3; i++) c[i] = A[i] + w * ac[i];
        return;
    }
    const double va = d3 * d6 - d5 * d4;
    const double e43 = d4 - d3, e56 = d5 - d6;
    if (va <= 0.0 && e43 >= 0.0 && e56 >= 0.0) {
        const double w = e43 / (e43 + e56);
        for (int i = 0; i < 3; i++) c[i] = B[i] + w * (C[i] - B[i]);
        return;
    }
    const double den = (va + vb) + vc;
    const double v = vb / den, w = vc / den;
    for (int i = 0; i < 3; i++) c[i] = (A[i] + ab[i] * v) + ac[i] * w;
}

// Distance of p from triangle k (at the mesh's current pose) and the unit
// normal from its closest point towards p; false when p lies on it.
__device__ __forceinline__ bool tri_distance(const DevScene &S, int64_t k, const double *p, double &phi, double *n) {
    double V[9], c[3], d[3];
    tri_world(S, k, V);
    closest_on_triangle(V, V + 3, V + 6, p, c);
    for (int i = 0; i < 3; i++) d[i] = p[i] - c[i];
    const double dd = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (!(dd > 0.0)) return false;
    phi = dd;
    for (int i = 0; i < 3; i++) n[i] = d[i] / dd;
    return true;
}

}  // namespace cdem
