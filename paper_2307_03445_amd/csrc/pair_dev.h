// Pair evaluation of the step (Sec. 2.1): contact kinematics of Eq.
// kinematicsContactInfo, the Hertz-Mindlin law of Eqs.
// normal_tangential_force_model1/2 with the history update and cap of Eqs.
// updateUt and cappingOfut, and the per-pair contributions the reduction
// sums.  Shared by the step kernels and the run-time compiled pair kernel of
// a user force law (the force law is a template parameter).
#pragma once

#include "step_dev.h"

namespace cdem {

// ---------------------------------------------------------------- contact law
struct Acc { double F[3], T[3]; };

__device__ __forceinline__ void cross3(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ __forceinline__ void cross3f(const float *a, const float *b, float *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// FP64 Hertz-Mindlin law: force on body b and updated history.
__device__ __forceinline__ void law64(const double *n, double delta, const double *vrel, double Rbar, double mbar,
                      double estar, double gstar, double mu, double beta, double h, const double *u_old,
                      double *F, double *u_new) {
    const double kdamp = -2.0 * sqrt(5.0 / 6.0);
    double vn_s = vrel[0] * n[0] + vrel[1] * n[1] + vrel[2] * n[2];
    double vn[3], vt[3];
    for (int i = 0; i < 3; i++) vn[i] = vn_s * n[i];
    for (int i = 0; i < 3; i++) vt[i] = vrel[i] - vn[i];
    double sq = sqrt(Rbar * delta);
    double Sn = 2.0 * estar * sq;
    double gn = kdamp * beta * sqrt(Sn * mbar);
    double kn = (4.0 / 3.0) * estar * sq * delta;
    double Fn[3];
    for (int i = 0; i < 3; i++) Fn[i] = kn * n[i] - gn * vn[i];
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

// FP32 law: force arithmetic in FP32; the history update, its projection and
// the clamp of the history stay in FP64.
__device__ __forceinline__ void law32(const double *nd, double delta_d, const float *vrel, float Rbar, float mbar, float estar,
                      float gstar, float mu, float beta, double h, const double *u_old, float *F, double *u_new) {
    const float kdamp = -2.0f * sqrtf(5.0f / 6.0f);
    float n[3] = {(float)nd[0], (float)nd[1], (float)nd[2]};
    float delta = (float)delta_d;
    float vn_s = vrel[0] * n[0] + vrel[1] * n[1] + vrel[2] * n[2];
    float vn[3], vt[3];
    for (int i = 0; i < 3; i++) vn[i] = vn_s * n[i];
    for (int i = 0; i < 3; i++) vt[i] = vrel[i] - vn[i];
    float sq = sqrtf(Rbar * delta);
    float Sn = 2.0f * estar * sq;
    float gn = kdamp * beta * sqrtf(Sn * mbar);
    float kn = (4.0f / 3.0f) * estar * sq * delta;
    float Fn[3];
    for (int i = 0; i < 3; i++) Fn[i] = kn * n[i] - gn * vn[i];
    double up[3];
    for (int i = 0; i < 3; i++) up[i] = u_old[i] + h * (double)vt[i];
    double upn = up[0] * nd[0] + up[1] * nd[1] + up[2] * nd[2];
    double ut[3];
    for (int i = 0; i < 3; i++) ut[i] = up[i] - upn * nd[i];
    float St = 8.0f * gstar * sq;
    float gt = kdamp * beta * sqrtf(St * mbar);
    float Ft[3];
    for (int i = 0; i < 3; i++) Ft[i] = -(St * (float)ut[i]) - gt * vt[i];
    float fn_norm = sqrtf(Fn[0] * Fn[0] + Fn[1] * Fn[1] + Fn[2] * Fn[2]);
    float ft_norm = sqrtf(Ft[0] * Ft[0] + Ft[1] * Ft[1] + Ft[2] * Ft[2]);
    float cap = mu * fn_norm;
    if (ft_norm > cap) {
        float scale = cap / ft_norm;
        for (int i = 0; i < 3; i++) Ft[i] = Ft[i] * scale;
        double ut_norm = sqrt(ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2]);
        if (ut_norm > 0.0) {
            double fac = (double)(cap / St) / ut_norm;
            for (int i = 0; i < 3; i++) u_new[i] = fac * ut[i];
        } else {
            for (int i = 0; i < 3; i++) u_new[i] = 0.0;
        }
    } else {
        for (int i = 0; i < 3; i++) u_new[i] = ut[i];
    }
    for (int i = 0; i < 3; i++) F[i] = Fn[i] + Ft[i];
}

// Per-pair contribution storage: force on the pair's lower sphere with the
// contact flag in w, that sphere's torque about its clump CoM, and the
// partner sphere's torque (its force is minus the first); FP32 mode stores
// floats.
// Stores that mark their lines non-temporal: the pair contributions are
// read once, by the next kernel, long after the L2 has turned over.
__device__ __forceinline__ void store_nt(float4 *p, float4 v) {
    __builtin_nontemporal_store(v.x, &p->x); __builtin_nontemporal_store(v.y, &p->y);
    __builtin_nontemporal_store(v.z, &p->z); __builtin_nontemporal_store(v.w, &p->w);
}
__device__ __forceinline__ void store_nt(double4 *p, double4 v) {
    __builtin_nontemporal_store(v.x, &p->x); __builtin_nontemporal_store(v.y, &p->y);
    __builtin_nontemporal_store(v.z, &p->z); __builtin_nontemporal_store(v.w, &p->w);
}

// A torque contribution: three components, packed (12 or 24 bytes a pair).
template <class T> struct Vec3 { T x, y, z; };
template <class T> __device__ __forceinline__ void store_nt(Vec3<T> *p, Vec3<T> v) {
    __builtin_nontemporal_store(v.x, &p->x); __builtin_nontemporal_store(v.y, &p->y);
    __builtin_nontemporal_store(v.z, &p->z);
}

template <bool FP32> struct Contrib;
// Force contributions carry a fourth word (1 when the pair is in contact);
// torque contributions are three words.
template <> struct Contrib<true> {
    using V = float4;
    using T = Vec3<float>;
    static __device__ __forceinline__ V make(const double *a, double w) {
        return make_float4((float)a[0], (float)a[1], (float)a[2], (float)w);
    }
    static __device__ __forceinline__ T make3(const double *a) { return T{(float)a[0], (float)a[1], (float)a[2]}; }
};
template <> struct Contrib<false> {
    using V = double4;
    using T = Vec3<double>;
    static __device__ __forceinline__ V make(const double *a, double w) { return make_double4(a[0], a[1], a[2], w); }
    static __device__ __forceinline__ T make3(const double *a) { return T{a[0], a[1], a[2]}; }
};

// Torque r x f, in FP32 when the force law ran in FP32.
template <bool FP32>
__device__ __forceinline__ void torque(const double *r, const double *f, double *t) {
    if (!FP32) {
        cross3(r, f, t);
    } else {
        float rf[3] = {(float)r[0], (float)r[1], (float)r[2]}, ff[3] = {(float)f[0], (float)f[1], (float)f[2]}, tf[3];
        cross3f(rf, ff, tf);
        t[0] = tf[0]; t[1] = tf[1]; t[2] = tf[2];
    }
}

// Evaluate pair e of the active set once, for both bodies: sphere pairs
// have the lower sphere as body a; a boundary pair has the sphere as body b.
// Writes the pair's history and contributions, and returns the contact
// sides it created.
// Ids of a pair and the clumps and template spheres of its spheres (b unused
// for a boundary pair).
struct PairIds { uint32_t s, t, ca, ta, cb, tb; };
__device__ __forceinline__ PairIds pair_ids(const DevScene &S, uint32_t s, uint32_t t) {
    PairIds q{s, t, S.owner[s], S.sts[s], 0u, 0u};
    if (t < (uint32_t)S.ns) { q.cb = S.owner[t]; q.tb = S.sts[t]; }
    return q;
}

// The built-in force law (Eqs. normal_tangential_force_model1/2, updateUt
// and cappingOfut with the readings above): law64 in the all-FP64 mode,
// law32 in the FP32-force mode.  A user force law compiled at run time has
// the same interface as law64 and runs in FP64 in both modes (kFP32 false;
// the FP32-force mode then only stores its contributions in FP32).
struct HertzMindlin {
    static constexpr bool kFP32 = true;
    __device__ static __forceinline__ void f64(const double *n, double delta, const double *vrel, double Rbar,
                                               double mbar, double estar, double gstar, double mu, double beta,
                                               double h, const double *u_old, double *F, double *u_new) {
        law64(n, delta, vrel, Rbar, mbar, estar, gstar, mu, beta, h, u_old, F, u_new);
    }
};

// What a boundary contact needs of its boundary: combined-material terms,
// the reference point (torques, and the lever arm of its surface velocity),
// velocity and angular velocity.
struct WallView {
    double e, g, mu, beta;
    float ef, gf, muf, betaf;
    double ref[3], vel[3], omg[3];
};

// rec_mode: 0 nothing recorded, 1 every pair, 2 boundary pairs only.  F:
// fixed-point positions (see fixed_pos); TRI: the scene may have triangles.
template <bool FP32, class Law, int FX, bool TRI>
__device__ __forceinline__ uint32_t eval_pair(const DevScene &S, int64_t e, const PairIds &id, double *hist,
                                              double tnow, int rec_mode) {
    using V = typename Contrib<FP32>::V;
    using T = typename Contrib<FP32>::T;
    V *cS = (V *)S.cS;
    T *cTs = (T *)S.cTs, *cTt = (T *)S.cTt;
    const double zero3[3] = {0.0, 0.0, 0.0};
    const uint32_t s = id.s, t = id.t;
    double *h = hist + 3 * e;
    if (t < (uint32_t)S.ns) {
        const bool rec = rec_mode == 1;
        const uint32_t a = s, b = t;  // a < b: pairs live in the lower sphere's segment
        const SphereKin ka = sphere_kin_of<FX>(S, id.ca, id.ta), kb = sphere_kin_of<FX>(S, id.cb, id.tb);
        double dv[3], dc[3];
        sphere_vec<FX>(S, ka, kb, dv, dc);
        double dx = dv[0], dy = dv[1], dz = dv[2];
        double d2 = dx * dx + dy * dy + dz * dz;
        double Sr = ka.R + kb.R;
        if (!(d2 < Sr * Sr)) {  // a false positive of the enlarged geometry: no force, no history
            cS[e] = Contrib<FP32>::make(zero3, 0.0);
            if (h[0] != 0.0 || h[1] != 0.0 || h[2] != 0.0) { h[0] = 0.0; h[1] = 0.0; h[2] = 0.0; }
            if (rec) S.rec_state[e] = 0;
            return 0;
        }
        double d = sqrt(d2);
        double delta = Sr - d;
        if (!(delta > 0.0)) {
            cS[e] = Contrib<FP32>::make(zero3, 0.0);
            h[0] = 0.0; h[1] = 0.0; h[2] = 0.0;
            if (rec) { S.rec_state[e] = 1; S.rec_delta[e] = delta; S.rec_F[3 * e] = 0; S.rec_F[3 * e + 1] = 0; S.rec_F[3 * e + 2] = 0; }
            return 0;
        }
        double n[3] = {dx / d, dy / d, dz / d};
        double lever = ka.R - 0.5 * delta;
        double ra[3], rb[3];  // lever arms from the two CoMs to the contact point
        if (!fixed_pos<FX>(S)) {
            double p[3] = {ka.p[0] + lever * n[0], ka.p[1] + lever * n[1], ka.p[2] + lever * n[2]};
            for (int i = 0; i < 3; i++) { ra[i] = p[i] - ka.xc[i]; rb[i] = p[i] - kb.xc[i]; }
        } else {  // a's rotated offset, then along n; from b's CoM, less the CoM difference
            for (int i = 0; i < 3; i++) { ra[i] = ka.r[i] + lever * n[i]; rb[i] = ra[i] - dc[i]; }
        }
        // contact kinematics in FP64 (relative velocities of similar speeds cancel)
        double ca3[3], cb3[3];
        cross3(ka.W, ra, ca3);
        cross3(kb.W, rb, cb3);
        double vrel[3] = {(kb.v[0] + cb3[0]) - (ka.v[0] + ca3[0]), (kb.v[1] + cb3[1]) - (ka.v[1] + ca3[1]),
                          (kb.v[2] + cb3[2]) - (ka.v[2] + ca3[2])};
        double u_old[3] = {h[0], h[1], h[2]}, u_new[3], F[3];
        if constexpr (!(FP32 && Law::kFP32)) {
            double Rbar = (ka.R * kb.R) / (ka.R + kb.R);
            double mbar = (ka.M * kb.M) / (ka.M + kb.M);
            double4 ma = S.mat64[a], mb = S.mat64[b];
            Law::f64(n, delta, vrel, Rbar, mbar, 1.0 / (ma.x + mb.x), 1.0 / (ma.y + mb.y), fmin(ma.z, mb.z),
                     fmin(ma.w, mb.w), S.h, u_old, F, u_new);
        } else {
            float vrf[3] = {(float)vrel[0], (float)vrel[1], (float)vrel[2]};
            float Ra = (float)ka.R, Rb = (float)kb.R, Ma = (float)ka.M, Mb = (float)kb.M;
            float4 ma = S.mat32[a], mb = S.mat32[b];
            float Ff[3];
            law32(n, delta, vrf, (Ra * Rb) / (Ra + Rb), (Ma * Mb) / (Ma + Mb), 1.0f / (ma.x + mb.x),
                  1.0f / (ma.y + mb.y), fminf(ma.z, mb.z), fminf(ma.w, mb.w), S.h, u_old, Ff, u_new);
            F[0] = Ff[0]; F[1] = Ff[1]; F[2] = Ff[2];
        }
        h[0] = u_new[0]; h[1] = u_new[1]; h[2] = u_new[2];
        double fa[3] = {-F[0], -F[1], -F[2]}, ta[3], tb[3];
        torque<FP32>(ra, fa, ta);
        torque<FP32>(rb, F, tb);
        store_nt(cS + e, Contrib<FP32>::make(fa, 1.0));
        store_nt(cTs + e, Contrib<FP32>::make3(ta));
        store_nt(cTt + e, Contrib<FP32>::make3(tb));
        if (rec) {
            S.rec_state[e] = 1; S.rec_delta[e] = delta;
            for (int i = 0; i < 3; i++) {
                S.rec_F[3 * e + i] = F[i]; S.rec_Ta[3 * e + i] = ta[i]; S.rec_Tb[3 * e + i] = tb[i];
            }
        }
        return 2;
    }
    const bool rec = rec_mode != 0;
    // boundary pair: the boundary is body a, sphere s is body b; an analytic
    // boundary, or a triangle of a mesh (its mesh's reference point, motion
    // and material)
    const uint32_t wi = t - (uint32_t)S.ns;
    const bool tri = TRI && wi >= (uint32_t)S.n_bnd;
    const SphereKin ks = sphere_kin_of<FX>(S, id.ca, id.ta);
    double phi, n[3];
    WallView B;
    bool contact;
    if (!tri) {
        const Bnd &b = S.bnd[wi];
        contact = bnd_distance(b, tnow, ks.p[0], ks.p[1], ks.p[2], phi, n) && phi < ks.R;
        B = WallView{b.e, b.g, b.mu, b.beta, b.ef, b.gf, b.muf, b.betaf,
                     {b.p[0] + tnow * b.vel[0], b.p[1] + tnow * b.vel[1], b.p[2] + tnow * b.vel[2]},
                     {b.vel[0], b.vel[1], b.vel[2]}, {b.omg[0], b.omg[1], b.omg[2]}};
    } else {
        const int64_t k = (int64_t)(wi - (uint32_t)S.n_bnd);
        contact = tri_distance(S, k, ks.p, phi, n) && phi < ks.R;
        const Mesh &m = S.mesh[S.tri_mesh[k]];
        B = WallView{m.e, m.g, m.mu, m.beta, m.ef, m.gf, m.muf, m.betaf, {m.x[0], m.x[1], m.x[2]},
                     {m.v[0], m.v[1], m.v[2]}, {m.w[0], m.w[1], m.w[2]}};
    }
    if (!contact) {
        cS[e] = Contrib<FP32>::make(zero3, 0.0);
        if (h[0] != 0.0 || h[1] != 0.0 || h[2] != 0.0) { h[0] = 0.0; h[1] = 0.0; h[2] = 0.0; }
        if (rec) S.rec_state[e] = 0;
        return 0;
    }
    double R = ks.R;
    double delta = R - phi;
    double lever = R - 0.5 * delta;
    double p[3] = {ks.p[0] - lever * n[0], ks.p[1] - lever * n[1], ks.p[2] - lever * n[2]};
    const double *cw = B.ref;
    double ra[3] = {p[0] - cw[0], p[1] - cw[1], p[2] - cw[2]};
    double rb[3];
    for (int i = 0; i < 3; i++) rb[i] = fixed_pos<FX>(S) ? ks.r[i] - lever * n[i] : p[i] - ks.xc[i];
    double pw[3], cb3[3];
    cross3(B.omg, ra, pw);
    cross3(ks.W, rb, cb3);
    double wv[3] = {B.vel[0] + pw[0], B.vel[1] + pw[1], B.vel[2] + pw[2]};
    double vrel[3] = {(ks.v[0] + cb3[0]) - wv[0], (ks.v[1] + cb3[1]) - wv[1], (ks.v[2] + cb3[2]) - wv[2]};
    double u_old[3] = {h[0], h[1], h[2]}, u_new[3], F[3];
    if constexpr (!(FP32 && Law::kFP32)) {
        double4 ms = S.mat64[s];
        Law::f64(n, delta, vrel, R, ks.M, 1.0 / (B.e + ms.x), 1.0 / (B.g + ms.y), fmin(B.mu, ms.z),
                 fmin(B.beta, ms.w), S.h, u_old, F, u_new);
    } else {
        float vrf[3] = {(float)vrel[0], (float)vrel[1], (float)vrel[2]};
        float4 ms = S.mat32[s];
        float Ff[3];
        law32(n, delta, vrf, (float)R, (float)ks.M, 1.0f / (B.ef + ms.x), 1.0f / (B.gf + ms.y), fminf(B.muf, ms.z),
              fminf(B.betaf, ms.w), S.h, u_old, Ff, u_new);
        F[0] = Ff[0]; F[1] = Ff[1]; F[2] = Ff[2];
    }
    h[0] = u_new[0]; h[1] = u_new[1]; h[2] = u_new[2];
    double tb[3];
    torque<FP32>(rb, F, tb);
    cS[e] = Contrib<FP32>::make(F, 1.0);
    cTs[e] = Contrib<FP32>::make3(tb);
    if (rec) {
        S.rec_state[e] = 1; S.rec_delta[e] = delta;
        double fw[3] = {-F[0], -F[1], -F[2]}, tw[3];  // the boundary receives -F at the contact point
        cross3(ra, fw, tw);
        for (int i = 0; i < 3; i++) {
            S.rec_F[3 * e + i] = F[i]; S.rec_R[3 * e + i] = ra[i];
            S.rec_Ta[3 * e + i] = tw[i]; S.rec_Tb[3 * e + i] = tb[i];
        }
    }
    return 1;
}

// Every candidate pair of the active set, evaluated once, one lane per pair
// (grid-stride in memory order, which follows the sphere ids and so is
// spatially coherent): the body of the pair kernel, for the built-in law
// (k_pairs) and for a user law compiled at run time.  256 lanes per
// workgroup.
template <bool FP32, class Law, int FX = 2, bool TRI = true>
__device__ __forceinline__ void pairs_body(const DevScene &S) {
    if (aborted(S.ctl)) return;
    const int cur = S.ctl->buf;
    const uint32_t *pt = slot3(S.pt, cur), *ps = slot3(S.ps, cur);
    double *hist = pick(S.hist, S.ctl->hb);
    const int64_t n = S.ctl->n_pairs_cur;
    const int rec = S.ctl->record;
    const double tnow = (double)S.ctl->step * S.h;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t e = (int64_t)xcd_block() * blockDim.x + threadIdx.x;
    // Software pipeline over the grid-stride loop: while pair e is evaluated,
    // the clumps of the next pair and the ids of the one after are in flight.
    PairIds now{};
    uint32_t s2 = 0, t2 = 0;
    if (e < n) now = pair_ids(S, ps[e], pt[e]);
    if (e + stride < n) { s2 = ps[e + stride]; t2 = pt[e + stride]; }
    uint32_t sides = 0;  // contact sides this lane created
    for (; e < n; e += stride) {
        PairIds nxt{};
        if (e + stride < n) nxt = pair_ids(S, s2, t2);
        if (e + 2 * stride < n) { s2 = ps[e + 2 * stride]; t2 = pt[e + 2 * stride]; }
        sides += eval_pair<FP32, Law, FX, TRI>(S, e, now, hist, tnow, rec);
        now = nxt;
    }
    // the workgroup's count, for the interval rule (folded by k_step_end)
    for (int off = 32; off > 0; off >>= 1) sides += __shfl_xor(sides, off, 64);
    __shared__ uint32_t wsides[4];
    if ((threadIdx.x & 63) == 0) wsides[threadIdx.x >> 6] = sides;
    __syncthreads();
    if (threadIdx.x == 0) S.part_c[blockIdx.x] = wsides[0] + wsides[1] + wsides[2] + wsides[3];
}

}  // namespace cdem
