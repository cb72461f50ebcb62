// Host runtime and C ABI of libcdem (see include/cdem.h).
//
// A scene owns device copies of the clump templates, clump state, per-sphere
// materials and analytic boundaries, plus the working buffers of the step:
// per-scene uniform bins, the double-buffered active set with its tangential
// history, and a device-resident control block that schedules detections.
// cdem_step enqueues pose -> (detection when due) -> force/reduce/integrate ->
// step bookkeeping per step and synchronises once at the end to check for
// active-set overflow, which it repairs by growing the storage and resuming
// from the first step that did not complete.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/cdem.h"
#include "cdem_internal.h"
#include "rtc_embed.inc"

using namespace cdem;

namespace cdem {
hipError_t launch_mesh_contacts(const DevScene &S, unsigned long long *keys, double *FR, unsigned long long *count,
                                int64_t cap, hipStream_t st);
hipError_t launch_pack_state(const DevScene &S, double *x, double *q, double *v, double *w, int unpack,
                             hipStream_t st, int raw = 0);
}

// Event pool for per-kernel timing (read after the stream is synchronised).
// Brackets may nest (a bracket around a sequence of timed kernels): each
// before() opens one, the matching after() closes the innermost.
struct EventTimer : KernelTimer {
    std::vector<hipEvent_t> pool;
    struct Span { int id; size_t e0, e1; };
    std::vector<Span> spans;    // closed brackets, in launch order
    std::vector<Span> open;     // brackets awaiting their after()
    size_t used = 0;            // events in use
    double total_ms[K_COUNT] = {};
    int64_t launches[K_COUNT] = {};
    bool sel[K_COUNT];          // kernels that are timed
    EventTimer() { for (int i = 0; i < K_COUNT; i++) sel[i] = true; }
    hipEvent_t next() {
        if (used == pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
    void before(int id, hipStream_t st) override {
        if (!sel[id]) return;
        hipEvent_t e = next();
        if (e) (void)hipEventRecord(e, st);
        open.push_back(Span{e ? id : -1, used - 1, 0});
    }
    void after(int id, hipStream_t st) override {
        if (!sel[id] || open.empty()) return;
        Span sp = open.back();
        open.pop_back();
        hipEvent_t e = next();
        if (e) (void)hipEventRecord(e, st);
        sp.e1 = used - 1;
        if (!e) sp.id = -1;
        spans.push_back(sp);
    }
    // accumulate every closed bracket (the stream must be idle)
    void harvest() {
        for (const Span &sp : spans) {
            float ms = 0.f;
            if (sp.id >= 0 && hipEventElapsedTime(&ms, pool[sp.e0], pool[sp.e1]) == hipSuccess) {
                total_ms[sp.id] += ms;
                launches[sp.id]++;
            }
        }
        spans.clear();
        if (open.empty()) used = 0;
    }
    ~EventTimer() override { for (auto e : pool) (void)hipEventDestroy(e); }
};

struct cdem_scene {
    EventTimer *timer = nullptr;
    // graph replay
    int32_t graph_steps = 0;
    hipStream_t gstream = nullptr;
    hipGraphExec_t gexec = nullptr;
    DevScene gkey{};               // launch parameters the graph was captured with
    double bin_factor = 1.0;       // bins are bin_factor x the minimum size
    bool test_no_guard = false;   // testing aid: deferred detection without the displacement guard
    bool collecting = false;      // cdem_collect_envelopes in progress
    std::string err;
    cdem_allocator alloc{};
    bool custom_alloc = false;
    hipStream_t stream = nullptr;
    DevScene S{};
    cdem_detect_params det{};
    // host copies needed for regridding and reads
    std::vector<Grid> grids;
    std::vector<double> dom;           // [n_scenes][6]
    std::vector<int32_t> bnd_user;     // device boundary order -> user index
    std::vector<Bnd> bnd;
    // triangle meshes: velocities, materials and margins are the host's; the
    // device advances positions and orientations every step
    std::vector<Mesh> mesh;
    std::vector<double> mesh_speed;    // speed bound |v| + |w| rmax each mesh's margin was sized for
    std::vector<int32_t> tri_user;     // device triangle order -> user index
    std::vector<int32_t> tri_mesh;     // device triangle order -> mesh
    int64_t tri_box_len = 0;           // doubles of the triangle, chunk and scene boxes
    int64_t mesh_cap = 0;              // triangle contacts the last mesh-force readout held
    double rmax = 0.0;
    int64_t n_cells_alloc = 0;
    int64_t n_regions_alloc = 0;
    int64_t rec_cap = 0;
    std::vector<void *> owned;         // every device allocation, freed on destroy
    int64_t regrows = 0;
    uint64_t fingerprint = 0;          // of the description's static parts (checkpoints must match)
    // user force law compiled at run time (null: the built-in law)
    hipModule_t law_module = nullptr;
    hipFunction_t law_pairs = nullptr;
    int nslots = 2;                    // active-set slots with pair storage (3 in overlap mode)
    // detection ahead on a second stream (overlap mode)
    struct Ahead {
        bool on = false;
        int32_t K = 0;                 // interval: a snapshot every K steps, adopted K steps later
        int64_t origin = 0;            // step the intervals are counted from
        bool inflight = false;         // a set is being built (or built and not yet adopted)
        hipStream_t stream = nullptr;
        hipEvent_t ev_snap = nullptr, ev_det = nullptr;
        Ctl *ctl = nullptr;
        double4 *cst = nullptr, *spos = nullptr, *sorted_pos = nullptr;
        float *cacc = nullptr, *bin_margin = nullptr;
        uint4 *sorted_meta = nullptr;
        float4 *sorted_f4 = nullptr;
        uint32_t *stage = nullptr;
        uint2 *stage_n = nullptr;
        unsigned long long *narrow_part = nullptr;
        uint32_t *narrow_woff = nullptr;
        uint32_t *cell_of = nullptr, *cell_rank = nullptr;
        uint32_t *over_list = nullptr, *fb_list = nullptr, *cell_count = nullptr, *cell_start = nullptr, *scan_bsum = nullptr;
        uint32_t *bin_v = nullptr, *bin_a = nullptr, *reg_occ = nullptr;
        double *part_k = nullptr;
        Mesh *mesh = nullptr;          // the meshes at the snapshot
        double *tri_box = nullptr;
        int64_t n_cells_alloc = 0, n_regions_alloc = 0;
    } ahead;
};

// FNV-1a over raw bytes: identifies the static description a checkpoint belongs to.
static uint64_t fnv1a(uint64_t h, const void *p, size_t n) {
    const unsigned char *b = (const unsigned char *)p;
    for (size_t i = 0; i < n; i++) { h ^= b[i]; h *= 1099511628211ull; }
    return h;
}

static uint64_t desc_fingerprint(const cdem_scene_desc *d, int64_t ns) {
    uint64_t h = 14695981039346656037ull;
    uint32_t nts = d->tmpl_sphere_begin[d->n_templates];
    h = fnv1a(h, &d->h, 8);
    h = fnv1a(h, &d->n_templates, 4);
    h = fnv1a(h, d->tmpl_sphere_begin, 4 * ((size_t)d->n_templates + 1));
    h = fnv1a(h, d->tmpl_offset, 24 * (size_t)nts);
    h = fnv1a(h, d->tmpl_radius, 8 * (size_t)nts);
    h = fnv1a(h, d->tmpl_mass, 8 * (size_t)d->n_templates);
    h = fnv1a(h, d->tmpl_inertia, 24 * (size_t)d->n_templates);
    h = fnv1a(h, &d->n_clumps, 8);
    if (d->n_clumps) {
        h = fnv1a(h, d->clump_template, 4 * (size_t)d->n_clumps);
        h = fnv1a(h, d->clump_scene, 4 * (size_t)d->n_clumps);
    }
    if (ns) h = fnv1a(h, d->sphere_mat, 32 * (size_t)ns);
    h = fnv1a(h, &d->n_scenes, 4);
    h = fnv1a(h, d->gravity, 24 * (size_t)d->n_scenes);
    h = fnv1a(h, d->domain, 48 * (size_t)d->n_scenes);
    h = fnv1a(h, &d->n_bnd, 4);
    if (d->n_bnd) {
        h = fnv1a(h, d->bnd_type, 4 * (size_t)d->n_bnd);
        h = fnv1a(h, d->bnd_param, 96 * (size_t)d->n_bnd);
        h = fnv1a(h, d->bnd_mat, 32 * (size_t)d->n_bnd);
        h = fnv1a(h, d->bnd_vel, 24 * (size_t)d->n_bnd);
        h = fnv1a(h, d->bnd_omega, 24 * (size_t)d->n_bnd);
        h = fnv1a(h, d->bnd_scene, 4 * (size_t)d->n_bnd);
    }
    h = fnv1a(h, &d->n_presc, 4);
    if (d->n_presc) {
        h = fnv1a(h, d->presc_clump, 4 * (size_t)d->n_presc);
        h = fnv1a(h, d->presc_param, 96 * (size_t)d->n_presc);
    }
    h = fnv1a(h, &d->n_mesh, 4);
    if (d->n_mesh) {
        h = fnv1a(h, d->mesh_mat, 32 * (size_t)d->n_mesh);
        h = fnv1a(h, d->mesh_scene, 4 * (size_t)d->n_mesh);
    }
    h = fnv1a(h, &d->pos_exp, 4);
    h = fnv1a(h, &d->n_tri, 8);
    if (d->n_tri) {
        h = fnv1a(h, d->tri_mesh, 4 * (size_t)d->n_tri);
        h = fnv1a(h, d->tri_vertex, 72 * (size_t)d->n_tri);
    }
    return h;
}

static const char *kErrNames[] = {"ok", "invalid argument", "out of device memory", "HIP runtime error",
                                  "active-set capacity exceeded", "missed contact", "non-finite state",
                                  "invalid state"};

extern "C" int cdem_abi_version(void) { return CDEM_ABI_VERSION; }

extern "C" const char *cdem_strerror(int code) {
    int i = -code;
    if (i < 0 || i > 7) return "unknown error";
    return kErrNames[i];
}

// Message of the last failed cdem_create (which returns no scene to ask).
static std::string g_create_err = "no error";

extern "C" const char *cdem_last_error(const cdem_scene *s) { return s ? s->err.c_str() : g_create_err.c_str(); }

static void drop_graph(cdem_scene *sc);

static int fail(cdem_scene *s, int code, const std::string &msg) {
    if (s) s->err = msg;
    return code;
}

#define HIPCHK(expr)                                                                       \
    do {                                                                                   \
        hipError_t _e = (expr);                                                            \
        if (_e != hipSuccess)                                                              \
            return fail(sc, CDEM_E_HIP, std::string(#expr ": ") + hipGetErrorString(_e)); \
    } while (0)

// Device blocks come from the caller's allocator, else from the stream-ordered
// allocator on the scene's stream.  A block is used on that stream and, by
// host copies, after the stream has been synchronised; the allocation itself
// is synchronised once so that a block is valid on every stream and for
// synchronous copies from the moment it is returned.
static void *dev_alloc(cdem_scene *sc, size_t bytes) {
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (sc->custom_alloc) {
        p = sc->alloc.alloc(sc->alloc.ctx, bytes, (void *)sc->stream);
    } else if (hipMallocAsync(&p, bytes, sc->stream) != hipSuccess || hipStreamSynchronize(sc->stream) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
    }
    if (p) sc->owned.push_back(p);
    return p;
}

static void dev_free(cdem_scene *sc, void *p) {
    if (!p) return;
    auto it = std::find(sc->owned.begin(), sc->owned.end(), p);
    if (it != sc->owned.end()) sc->owned.erase(it);
    if (sc->custom_alloc) sc->alloc.free(sc->alloc.ctx, p, (void *)sc->stream);
    else (void)hipFreeAsync(p, sc->stream);
}

template <typename T>
static T *upload(cdem_scene *sc, const T *src, size_t n, int &rc) {
    T *d = (T *)dev_alloc(sc, n * sizeof(T));
    if (!d) { rc = fail(sc, CDEM_E_OOM, "device allocation failed"); return nullptr; }
    if (n && src) {
        hipError_t e = hipMemcpyAsync(d, src, n * sizeof(T), hipMemcpyHostToDevice, sc->stream);
        if (e != hipSuccess) { rc = fail(sc, CDEM_E_HIP, hipGetErrorString(e)); return nullptr; }
    }
    return d;
}

static double beta_of_cor(double e) {
    double l = std::log(e);
    return l / std::sqrt(l * l + M_PI * M_PI);
}

static bool finite_all(const double *p, size_t n) {
    for (size_t i = 0; i < n; i++) if (!std::isfinite(p[i])) return false;
    return true;
}

// (Re)build the per-scene grids for bin size b = 2 (R_max + margin cap) and
// allocate the bin arrays when they grow.
static int build_grids(cdem_scene *sc) {
    DevScene &S = sc->S;
    // bins of about R_max + margin cap: a sphere's candidates lie within its
    // reach (R + m) + (R_max + m), and the scan visits only the bins that
    // reach touches (smaller bins fit it more tightly, at more rows)
    double b = (sc->rmax + std::max(0.0, sc->det.margin_cap)) * sc->bin_factor;
    if (!(b > 0.0)) b = 1.0;  // no spheres: any positive bin size will do
    int64_t cell0 = 0, reg0 = 0;
    for (int k = 0; k < S.n_scenes; k++) {
        Grid &g = sc->grids[k];
        const double *d = &sc->dom[6 * k];
        double bb = b;
        int64_t nx, ny, nz;
        for (;;) {
            nx = std::max<int64_t>(1, (int64_t)std::ceil((d[3] - d[0]) / bb));
            ny = std::max<int64_t>(1, (int64_t)std::ceil((d[4] - d[1]) / bb));
            nz = std::max<int64_t>(1, (int64_t)std::ceil((d[5] - d[2]) / bb));
            if (nx * ny * nz <= (int64_t)1 << 27) break;
            bb *= 1.25;  // keep the bin count bounded for huge, sparse domains
        }
        g.ox = d[0]; g.oy = d[1]; g.oz = d[2];
        g.inv = 1.0 / bb;
        g.b = bb;
        g.rm_max = sc->rmax + std::max(0.0, sc->det.margin_cap);
        g.r_max = sc->rmax;
        // FP32 prefilter slack: positions relative to the origin are rounded to
        // float (half an ulp of the largest coordinate each), differences of
        // two of them and the float distance add a few more ulps; 32 ulps of
        // the domain's extent (plus one bin of sphere outside it) bounds all
        {
            double ext = std::max({d[3] - d[0], d[4] - d[1], d[5] - d[2]}) + 2.0 * bb;
            g.pre_eps = (float)(32.0 * ext * std::ldexp(1.0, -24));
            g.pre_lim = (float)(2.0 * ext);
        }
        g.nx = (int32_t)nx; g.ny = (int32_t)ny; g.nz = (int32_t)nz;
        g.cell0 = cell0;
        cell0 += nx * ny * nz;
        g.rnx = (int32_t)((nx + kRegionBins - 1) / kRegionBins);
        g.rny = (int32_t)((ny + kRegionBins - 1) / kRegionBins);
        g.rnz = (int32_t)((nz + kRegionBins - 1) / kRegionBins);
        g.rpad = 0;
        g.reg0 = reg0;
        reg0 += (int64_t)g.rnx * g.rny * g.rnz;
    }
    S.n_regions = reg0;
    if (cell0 >= ((int64_t)1 << 32)) return fail(sc, CDEM_E_INVALID, "too many bins");
    S.n_cells = cell0;
    int rc = CDEM_OK;
    Grid *dg = (Grid *)S.grids;
    if (!dg) {
        dg = upload(sc, sc->grids.data(), sc->grids.size(), rc);
        if (!dg) return rc;
        S.grids = dg;
    } else {
        hipError_t e = hipMemcpyAsync(dg, sc->grids.data(), sc->grids.size() * sizeof(Grid), hipMemcpyHostToDevice, sc->stream);
        if (e != hipSuccess) return fail(sc, CDEM_E_HIP, hipGetErrorString(e));
    }
    if (cell0 > sc->n_cells_alloc) {
        dev_free(sc, S.cell_count);
        dev_free(sc, S.cell_start);
        dev_free(sc, S.scan_bsum);
        int64_t nblk = (cell0 + 1023) / 1024 + 1;
        S.cell_count = (uint32_t *)dev_alloc(sc, cell0 * 4);
        S.cell_start = (uint32_t *)dev_alloc(sc, (cell0 + 1) * 4);  // + the end of the last bin
        S.scan_bsum = (uint32_t *)dev_alloc(sc, nblk * 4);
        if (!S.cell_count || !S.cell_start || !S.scan_bsum) return fail(sc, CDEM_E_OOM, "bin arrays");
        sc->n_cells_alloc = cell0;
    }
    if (reg0 > sc->n_regions_alloc) {
        dev_free(sc, S.bin_v); dev_free(sc, S.bin_a); dev_free(sc, S.reg_occ); dev_free(sc, S.bin_margin);
        dev_free(sc, S.occ_t); dev_free(sc, S.lab_v); dev_free(sc, S.lab_a);
        S.bin_v = (uint32_t *)dev_alloc(sc, reg0 * 4);
        S.bin_a = (uint32_t *)dev_alloc(sc, reg0 * 4);
        S.reg_occ = (uint32_t *)dev_alloc(sc, reg0 * 4);
        S.bin_margin = (float *)dev_alloc(sc, reg0 * 4);
        S.occ_t = (uint32_t *)dev_alloc(sc, reg0 * 4);
        S.lab_v = (uint32_t *)dev_alloc(sc, reg0 * 4);
        S.lab_a = (uint32_t *)dev_alloc(sc, reg0 * 4);
        if (!S.bin_v || !S.bin_a || !S.reg_occ || !S.bin_margin || !S.occ_t || !S.lab_v || !S.lab_a)
            return fail(sc, CDEM_E_OOM, "region arrays");
        sc->n_regions_alloc = reg0;
    }
    return CDEM_OK;
}

// Pair and upper-entry offsets are 32-bit (segment starts, links): the
// active set holds at most kMaxCap entries per buffer.
constexpr int64_t kMaxCap = (int64_t)0xffffffffu;

static int alloc_active_set(cdem_scene *sc, int64_t cap, bool keep) {
    DevScene &S = sc->S;
    if (cap > kMaxCap)
        return fail(sc, CDEM_E_CAPACITY, "the active set would exceed 2^32 - 1 entries (32-bit pair offsets)");
    const int nslots = sc->nslots;
    uint32_t *pt[3] = {nullptr, nullptr, nullptr};
    double *hs[2];
    for (int k = 0; k < nslots; k++) {
        pt[k] = (uint32_t *)dev_alloc(sc, cap * 4);
        if (!pt[k]) return fail(sc, CDEM_E_OOM, "active-set storage");
    }
    for (int k = 0; k < 2; k++) {
        hs[k] = (double *)dev_alloc(sc, cap * 24);
        if (!hs[k]) return fail(sc, CDEM_E_OOM, "active-set storage");
    }
    // per-pair and upper-segment arrays rebuilt at each detection (no content to keep)
    dev_free(sc, S.cS); dev_free(sc, S.cTs); dev_free(sc, S.cTt);
    for (int k = 0; k < 3; k++) {
        dev_free(sc, S.ps[k]); dev_free(sc, S.ut[k]); dev_free(sc, S.us[k]); dev_free(sc, S.um[k]);
        S.ps[k] = S.ut[k] = S.us[k] = S.um[k] = nullptr;
    }
    const size_t cw = S.precision == CDEM_PREC_FP32_FORCE ? 16 : 32;  // force: float4 / double4
    const size_t tw = S.precision == CDEM_PREC_FP32_FORCE ? 12 : 24;  // torques: three floats / doubles
    S.cS = dev_alloc(sc, cap * cw);
    S.cTs = dev_alloc(sc, cap * tw);
    S.cTt = dev_alloc(sc, cap * tw);
    if (!S.cS || !S.cTs || !S.cTt) return fail(sc, CDEM_E_OOM, "active-set storage");
    for (int k = 0; k < nslots; k++) {
        S.ps[k] = (uint32_t *)dev_alloc(sc, cap * 4);
        S.ut[k] = (uint32_t *)dev_alloc(sc, cap * 4);
        S.us[k] = (uint32_t *)dev_alloc(sc, cap * 4);
        S.um[k] = (uint32_t *)dev_alloc(sc, cap * 4);
        if (!S.ps[k] || !S.ut[k] || !S.us[k] || !S.um[k]) return fail(sc, CDEM_E_OOM, "active-set storage");
    }
    if (keep) {
        // preserve the current pairs and their history (lower segments point into them)
        Ctl c;
        if (hipMemcpy(&c, S.ctl, sizeof c, hipMemcpyDeviceToHost) != hipSuccess) return fail(sc, CDEM_E_HIP, "ctl read");
        const int cur = c.buf, hb = c.hb;
        size_t n = (size_t)std::min<int64_t>(c.n_pairs_cur, S.cap);
        if (n && S.pt[cur]) {
            if (hipMemcpyAsync(pt[cur], S.pt[cur], n * 4, hipMemcpyDeviceToDevice, sc->stream) != hipSuccess ||
                hipMemcpyAsync(hs[hb], S.hist[hb], n * 24, hipMemcpyDeviceToDevice, sc->stream) != hipSuccess)
                return fail(sc, CDEM_E_HIP, "active-set copy");
        }
        if (hipStreamSynchronize(sc->stream) != hipSuccess) return fail(sc, CDEM_E_HIP, "sync");
    }
    if (sc->rec_cap) {
        // the recording arrays follow the capacity (a step armed to record
        // writes them, also when it is run again after this regrow), with the
        // recorded step's entries kept at their indices like the pairs
        uint8_t *rs = (uint8_t *)dev_alloc(sc, cap);
        double *rd = (double *)dev_alloc(sc, 8 * cap), *rf[4];
        for (int k = 0; k < 4; k++) rf[k] = (double *)dev_alloc(sc, 24 * cap);
        if (!rs || !rd || !rf[0] || !rf[1] || !rf[2] || !rf[3]) return fail(sc, CDEM_E_OOM, "recording buffers");
        double **old[4] = {&S.rec_F, &S.rec_R, &S.rec_Ta, &S.rec_Tb};
        if (keep) {
            Ctl c;
            if (hipMemcpy(&c, S.ctl, sizeof c, hipMemcpyDeviceToHost) != hipSuccess) return fail(sc, CDEM_E_HIP, "ctl read");
            const size_t n = (size_t)std::min<int64_t>(c.n_pairs_cur, std::min(sc->rec_cap, cap));
            hipError_t e = hipSuccess;
            if (n) {
                e = hipMemcpyAsync(rs, S.rec_state, n, hipMemcpyDeviceToDevice, sc->stream);
                if (e == hipSuccess) e = hipMemcpyAsync(rd, S.rec_delta, 8 * n, hipMemcpyDeviceToDevice, sc->stream);
                for (int k = 0; k < 4 && e == hipSuccess; k++)
                    e = hipMemcpyAsync(rf[k], *old[k], 24 * n, hipMemcpyDeviceToDevice, sc->stream);
            }
            if (e == hipSuccess) e = hipStreamSynchronize(sc->stream);
            if (e != hipSuccess) return fail(sc, CDEM_E_HIP, "recording copy");
        }
        dev_free(sc, S.rec_state); dev_free(sc, S.rec_delta);
        S.rec_state = rs; S.rec_delta = rd;
        for (int k = 0; k < 4; k++) { dev_free(sc, *old[k]); *old[k] = rf[k]; }
        sc->rec_cap = cap;
    }
    for (int k = 0; k < 3; k++) { dev_free(sc, S.pt[k]); S.pt[k] = pt[k]; }
    for (int k = 0; k < 2; k++) { dev_free(sc, S.hist[k]); S.hist[k] = hs[k]; }
    S.cap = cap;
    return CDEM_OK;
}

// ---------------------------------------------------------------- detection ahead
// Wait for the second stream; with discard, a set in flight is dropped (it
// is rebuilt at the next interval; results do not depend on when a detection
// runs).  Called before anything that reallocates, regrids or rewrites the
// state the second stream reads.
static int ahead_drain(cdem_scene *sc, bool discard) {
    auto &a = sc->ahead;
    if (a.stream) HIPCHK(hipStreamSynchronize(a.stream));
    if (discard) a.inflight = false;
    return CDEM_OK;
}

// The second stream's buffers: a snapshot of the clump records and
// acceleration envelopes, its own sphere positions, bins, sorted records,
// envelope regions, overflow list and control block.
static int ahead_alloc(cdem_scene *sc) {
    auto &a = sc->ahead;
    DevScene &S = sc->S;
    const int64_t ns = std::max<int64_t>(S.ns, 1), nc = std::max<int64_t>(S.nc, 1);
    if (!a.stream) {
        HIPCHK(hipStreamCreateWithFlags(&a.stream, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&a.ev_snap, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&a.ev_det, hipEventDisableTiming));
        a.ctl = (Ctl *)dev_alloc(sc, sizeof(Ctl));
        a.cst = (double4 *)dev_alloc(sc, 4 * sizeof(double4) * nc);
        a.cacc = (float *)dev_alloc(sc, 4 * nc);
        a.spos = (double4 *)dev_alloc(sc, sizeof(double4) * ns);
        a.cell_of = (uint32_t *)dev_alloc(sc, 4 * ns);
        a.cell_rank = (uint32_t *)dev_alloc(sc, 4 * ns);
        a.sorted_meta = (uint4 *)dev_alloc(sc, sizeof(uint4) * ns);
        a.sorted_pos = (double4 *)dev_alloc(sc, sizeof(double4) * ns);
        a.sorted_f4 = (float4 *)dev_alloc(sc, sizeof(float4) * ns);
        a.stage = (uint32_t *)dev_alloc(sc, 4 * (size_t)kMaxRow * ns);
        a.stage_n = (uint2 *)dev_alloc(sc, sizeof(uint2) * ns);
        a.narrow_part = (unsigned long long *)dev_alloc(sc, 24 * (size_t)((ns + kNarrowBlock - 1) / kNarrowBlock));
        a.narrow_woff =
            (uint32_t *)dev_alloc(sc, 8 * (kNarrowBlock / 64) * (size_t)((ns + kNarrowBlock - 1) / kNarrowBlock));
        a.over_list = (uint32_t *)dev_alloc(sc, 4 * S.over_cap);
        a.fb_list = (uint32_t *)dev_alloc(sc, 4 * std::max<int64_t>(S.ns, 1));
        a.part_k = (double *)dev_alloc(sc, 2 * 8 * (size_t)kRegionBlocksMax);
        a.mesh = (Mesh *)dev_alloc(sc, sizeof(Mesh) * std::max<int64_t>(S.n_mesh, 1));
        a.tri_box = (double *)dev_alloc(sc, 8 * (size_t)std::max<int64_t>(sc->tri_box_len, 1));
        if (!a.ctl || !a.cst || !a.cacc || !a.spos || !a.cell_of || !a.cell_rank || !a.sorted_meta ||
            !a.sorted_pos || !a.sorted_f4 || !a.stage || !a.stage_n || !a.narrow_part ||
            !a.narrow_woff || !a.over_list || !a.fb_list || !a.part_k || !a.mesh || !a.tri_box)
            return fail(sc, CDEM_E_OOM, "buffers of the detection ahead");
        Ctl z;
        memset(&z, 0, sizeof z);
        HIPCHK(hipMemcpyAsync(a.ctl, &z, sizeof z, hipMemcpyHostToDevice, sc->stream));
        HIPCHK(hipStreamSynchronize(sc->stream));
    }
    if (S.n_cells > a.n_cells_alloc) {
        dev_free(sc, a.cell_count); dev_free(sc, a.cell_start); dev_free(sc, a.scan_bsum);
        const int64_t nblk = (S.n_cells + 1023) / 1024 + 1;
        a.cell_count = (uint32_t *)dev_alloc(sc, S.n_cells * 4);
        a.cell_start = (uint32_t *)dev_alloc(sc, (S.n_cells + 1) * 4);
        a.scan_bsum = (uint32_t *)dev_alloc(sc, nblk * 4);
        if (!a.cell_count || !a.cell_start || !a.scan_bsum) return fail(sc, CDEM_E_OOM, "bins of the detection ahead");
        a.n_cells_alloc = S.n_cells;
    }
    if (S.n_regions > a.n_regions_alloc) {
        dev_free(sc, a.bin_v); dev_free(sc, a.bin_a); dev_free(sc, a.reg_occ); dev_free(sc, a.bin_margin);
        const int64_t nr = std::max<int64_t>(S.n_regions, 1);
        a.bin_v = (uint32_t *)dev_alloc(sc, nr * 4);
        a.bin_a = (uint32_t *)dev_alloc(sc, nr * 4);
        a.reg_occ = (uint32_t *)dev_alloc(sc, nr * 4);
        a.bin_margin = (float *)dev_alloc(sc, nr * 4);
        if (!a.bin_v || !a.bin_a || !a.reg_occ || !a.bin_margin)
            return fail(sc, CDEM_E_OOM, "regions of the detection ahead");
        a.n_regions_alloc = S.n_regions;
    }
    return CDEM_OK;
}

// The second stream's view of the scene: its own snapshot, positions, bins,
// regions and control block (whose bslot names the structure slot it writes).
static DevScene ahead_view(const cdem_scene *sc) {
    const auto &a = sc->ahead;
    DevScene B = sc->S;
    B.bchain = 1;
    B.horizon = 2 * a.K;
    B.ctl = a.ctl;
    B.cst = a.cst; B.cacc = a.cacc; B.spos = a.spos;
    B.cell_of = a.cell_of; B.cell_rank = a.cell_rank; B.cell_count = a.cell_count; B.cell_start = a.cell_start;
    B.scan_bsum = a.scan_bsum;
    B.sorted_meta = a.sorted_meta; B.sorted_pos = a.sorted_pos; B.sorted_f4 = a.sorted_f4;
    B.stage = a.stage; B.stage_n = a.stage_n; B.narrow_part = a.narrow_part; B.narrow_woff = a.narrow_woff;
    B.bin_v = a.bin_v; B.bin_a = a.bin_a; B.reg_occ = a.reg_occ; B.bin_margin = a.bin_margin;
    B.part_k = a.part_k; B.over_list = a.over_list; B.fb_list = a.fb_list;
    B.mesh = a.mesh; B.tri_box = a.tri_box;
    B.store_speed = 0; B.store_acc = 0;
    B.plan.audit_period = 0;
    return B;
}

static double norm3(const double *a) { return std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]); }

// Speed bound of every point of a mesh: |v| + |w| rmax.
static double mesh_speed_of(const Mesh &m) { return norm3(m.v) + norm3(m.w) * m.rmax; }
// A mesh's margin covers 1.25 times its speed bound, so that a
// co-simulation's small changes of speed keep the active set.
constexpr double kMeshSpeedHeadroom = 1.25;

// Candidate margins covering a boundary's own motion over the steps a set is
// used: speed x steps x h, plus 1 %.
static int margin_steps(const cdem_scene *sc) {
    int kmax = sc->det.mode == CDEM_DETECT_PLAIN ? 0 : std::max(1, sc->det.k_max);
    if (sc->ahead.on) kmax *= 2;  // a set built ahead is used up to 2 k_max steps after its snapshot
    return kmax;
}

static void set_bnd_margins(cdem_scene *sc) {
    const double kh = (double)margin_steps(sc) * sc->S.h * 1.01;
    for (auto &b : sc->bnd) b.margin = norm3(b.vel) * kh;
    for (size_t i = 0; i < sc->mesh.size(); i++) {
        sc->mesh_speed[i] = kMeshSpeedHeadroom * mesh_speed_of(sc->mesh[i]);
        sc->mesh[i].margin = sc->mesh_speed[i] * kh;
    }
}

// Device mesh records from the host's, keeping the positions and
// orientations the device has advanced (the stream is drained first).
static int push_meshes(cdem_scene *sc) {
    const size_t n = sc->mesh.size();
    if (!n) return CDEM_OK;
    std::vector<Mesh> dev(n);
    HIPCHK(hipStreamSynchronize(sc->stream));
    HIPCHK(hipMemcpy(dev.data(), sc->S.mesh, n * sizeof(Mesh), hipMemcpyDeviceToHost));
    for (size_t i = 0; i < n; i++) {
        memcpy(sc->mesh[i].x, dev[i].x, sizeof dev[i].x);
        memcpy(sc->mesh[i].q, dev[i].q, sizeof dev[i].q);
    }
    HIPCHK(hipMemcpy(sc->S.mesh, sc->mesh.data(), n * sizeof(Mesh), hipMemcpyHostToDevice));
    return CDEM_OK;
}

// Validates a mesh state (13 doubles: x, unit q, v, w).
static bool mesh_state_ok(const double *st) {
    if (!finite_all(st, 13)) return false;
    const double qn = st[3] * st[3] + st[4] * st[4] + st[5] * st[5] + st[6] * st[6];
    return std::fabs(qn - 1.0) < 1e-10;
}

static void mesh_set_state(Mesh &m, const double *st) {
    for (int i = 0; i < 3; i++) { m.x[i] = st[i]; m.v[i] = st[7 + i]; m.w[i] = st[10 + i]; }
    for (int i = 0; i < 4; i++) m.q[i] = st[3 + i];
}

// A contact partner as the caller numbers it: spheres as they are, analytic
// boundaries and triangles in the description's order.
static uint32_t user_partner(const cdem_scene *sc, uint32_t t) {
    const uint32_t ns = (uint32_t)sc->S.ns, nb = (uint32_t)sc->S.n_bnd;
    if (t < ns) return t;
    const uint32_t w = t - ns;
    if (w < nb) return ns + (uint32_t)sc->bnd_user[w];
    return ns + nb + (uint32_t)sc->tri_user[w - nb];
}

extern "C" int cdem_create(const cdem_scene_desc *d, const cdem_allocator *alloc, void *stream, cdem_scene **out) {
    if (!out) return CDEM_E_INVALID;
    *out = nullptr;
    if (!d) return CDEM_E_INVALID;
    cdem_scene *sc = new (std::nothrow) cdem_scene();
    if (!sc) return CDEM_E_OOM;
    auto bail = [&](int rc) { g_create_err = sc->err; cdem_destroy(sc); return rc; };
    auto invalid = [&](const char *m) { g_create_err = m; cdem_destroy(sc); return CDEM_E_INVALID; };
    // ---- validation
    if (!(d->h > 0) || !std::isfinite(d->h)) return invalid("time step must be positive");
    if (d->precision != CDEM_PREC_FP64 && d->precision != CDEM_PREC_FP32_FORCE) return invalid("unknown precision");
    if (d->n_templates < 1 || !d->tmpl_sphere_begin || d->tmpl_sphere_begin[0] != 0) return invalid("templates");
    if (d->n_clumps < 0 || d->n_clumps >= ((int64_t)1 << 31)) return invalid("clump count");
    if (d->n_scenes < 1 || !d->gravity || !d->domain) return invalid("scenes");
    if (d->n_bnd < 0 || d->n_bnd > kMaxBnd) return invalid("at most 4096 boundaries");
    int nt = d->n_templates;
    for (int t = 0; t < nt; t++)
        if (d->tmpl_sphere_begin[t + 1] <= d->tmpl_sphere_begin[t]) return invalid("empty template");
    uint32_t nts = d->tmpl_sphere_begin[nt];
    for (uint32_t i = 0; i < nts; i++)
        if (!(d->tmpl_radius[i] > 0) || !std::isfinite(d->tmpl_radius[i])) return invalid("template radius");
    if (!finite_all(d->tmpl_offset, 3 * (size_t)nts)) return invalid("template offsets");
    for (int t = 0; t < nt; t++) {
        if (!(d->tmpl_mass[t] > 0)) return invalid("template mass");
        for (int k = 0; k < 3; k++) if (!(d->tmpl_inertia[3 * t + k] > 0)) return invalid("template inertia");
    }
    int64_t nc = d->n_clumps;
    std::vector<int64_t> sbeg(nc + 1, 0);
    for (int64_t c = 0; c < nc; c++) {
        uint32_t t = d->clump_template[c];
        if ((int)t >= nt || d->clump_scene[c] >= (uint32_t)d->n_scenes) return invalid("clump template/scene");
        sbeg[c + 1] = sbeg[c] + (d->tmpl_sphere_begin[t + 1] - d->tmpl_sphere_begin[t]);
        double qn = 0;
        for (int k = 0; k < 4; k++) qn += d->q[4 * c + k] * d->q[4 * c + k];
        if (!(std::fabs(qn - 1.0) < 1e-10)) return invalid("quaternions must be unit");
    }
    int64_t ns = sbeg[nc];
    if (ns >= ((int64_t)1 << 31) - kMaxBnd) return invalid("too many spheres");
    if (!finite_all(d->x, 3 * nc) || !finite_all(d->v, 3 * nc) || !finite_all(d->w, 3 * nc)) return invalid("state");
    if (d->pos_exp != 0 && (d->pos_exp < 8 || d->pos_exp > 60)) return invalid("position exponent must be 0 or in [8, 60]");
    if (d->pos_exp) {  // fixed-point positions: CoMs and domains within 2^60 grid steps of the origin
        for (int64_t k = 0; k < 3 * nc; k++)
            if (!(std::fabs(std::ldexp(d->x[k], d->pos_exp)) < std::ldexp(1.0, 60)))
                return invalid("position outside the fixed-point range");
        for (int64_t k = 0; k < 6 * (int64_t)d->n_scenes; k++)
            if (!(std::fabs(std::ldexp(d->domain[k], d->pos_exp)) < std::ldexp(1.0, 60)))
                return invalid("domain outside the fixed-point range");
    }
    for (int64_t s = 0; s < ns; s++) {
        const double *m = d->sphere_mat + 4 * s;
        if (!(m[0] > 0) || !(m[1] > -1 && m[1] < 0.5) || !(m[2] >= 0) || !(m[3] > 0 && m[3] <= 1))
            return invalid("sphere material out of range");
    }
    for (int k = 0; k < d->n_bnd; k++) {
        const double *m = d->bnd_mat + 4 * k;
        if (d->bnd_type[k] < 0 || d->bnd_type[k] > 3) return invalid("boundary type");
        if (d->bnd_scene[k] < 0 || d->bnd_scene[k] >= d->n_scenes) return invalid("boundary scene");
        if (!(m[0] > 0) || !(m[1] > -1 && m[1] < 0.5) || !(m[2] >= 0) || !(m[3] > 0 && m[3] <= 1))
            return invalid("boundary material out of range");
    }
    for (int k = 0; k < d->n_scenes; k++) {
        const double *dm = d->domain + 6 * k;
        for (int j = 0; j < 3; j++) if (!(dm[j + 3] > dm[j])) return invalid("empty domain");
    }
    std::vector<int32_t> presc(nc, -1);
    for (int k = 0; k < d->n_presc; k++) {
        int32_t c = d->presc_clump[k];
        if (c < 0 || c >= nc) return invalid("prescribed clump out of range");
        presc[c] = k;
    }
    if (d->n_mesh < 0 || d->n_mesh > kMaxMesh || d->n_tri < 0 || (d->n_tri > 0 && d->n_mesh < 1))
        return invalid("mesh counts (at most 64 meshes)");
    if (ns + (int64_t)d->n_bnd + d->n_tri >= ((int64_t)1 << 31) - 1) return invalid("too many spheres and triangles");
    if (d->n_mesh && (!d->mesh_state || !d->mesh_mat || !d->mesh_scene)) return invalid("mesh arrays");
    if (d->n_tri && (!d->tri_mesh || !d->tri_vertex)) return invalid("triangle arrays");
    for (int k = 0; k < d->n_mesh; k++) {
        const double *m = d->mesh_mat + 4 * k;
        if (d->mesh_scene[k] < 0 || d->mesh_scene[k] >= d->n_scenes) return invalid("mesh scene");
        if (!(m[0] > 0) || !(m[1] > -1 && m[1] < 0.5) || !(m[2] >= 0) || !(m[3] > 0 && m[3] <= 1))
            return invalid("mesh material out of range");
        if (!mesh_state_ok(d->mesh_state + 13 * k)) return invalid("mesh state (finite, unit quaternion)");
    }
    for (int64_t k = 0; k < d->n_tri; k++)
        if (d->tri_mesh[k] < 0 || d->tri_mesh[k] >= d->n_mesh) return invalid("triangle mesh out of range");
    if (!finite_all(d->tri_vertex, 9 * (size_t)d->n_tri)) return invalid("triangle vertices");
    // ---- host-side derived arrays
    sc->custom_alloc = alloc && alloc->alloc && alloc->free;
    if (sc->custom_alloc) sc->alloc = *alloc;
    sc->stream = (hipStream_t)stream;
    DevScene &S = sc->S;
    S.nc = nc; S.ns = ns; S.n_scenes = d->n_scenes; S.n_bnd = d->n_bnd;
    S.precision = d->precision; S.detect_mode = CDEM_DETECT_PLAIN; S.h = d->h;
    S.pos_exp = d->pos_exp;
    S.pos_eps = std::ldexp(1.0, -d->pos_exp);
    S.pos_inv = std::ldexp(1.0, d->pos_exp);
    sc->det.mode = CDEM_DETECT_PLAIN; sc->det.k_max = 1; sc->det.safety = 1.5; sc->det.margin_cap = 0.0;
    sc->det.audit_period = 0;
    std::vector<uint32_t> owner(ns), sscene(ns);
    std::vector<double4> mat64(ns);
    std::vector<float4> mat32(ns);
    double rmax = 0;
    for (int64_t c = 0; c < nc; c++) {
        uint32_t t = d->clump_template[c];
        for (int64_t s = sbeg[c]; s < sbeg[c + 1]; s++) {
            owner[s] = (uint32_t)c;
            sscene[s] = d->clump_scene[c];
            rmax = std::max(rmax, d->tmpl_radius[d->tmpl_sphere_begin[t] + (s - sbeg[c])]);
        }
    }
    for (int64_t s = 0; s < ns; s++) {
        const double *m = d->sphere_mat + 4 * s;
        double E = m[0], nu = m[1];
        double e = (1.0 - nu * nu) / E, g = 2.0 * (2.0 - nu) * (1.0 + nu) / E, b = beta_of_cor(m[3]);
        mat64[s] = make_double4(e, g, m[2], b);
        mat32[s] = make_float4((float)e, (float)g, (float)m[2], (float)b);
    }
    sc->rmax = rmax;
    sc->fingerprint = desc_fingerprint(d, ns);
    // boundaries sorted by scene
    std::vector<int32_t> order(d->n_bnd);
    for (int k = 0; k < d->n_bnd; k++) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return d->bnd_scene[a] < d->bnd_scene[b]; });
    sc->bnd_user = order;
    sc->bnd.resize(d->n_bnd);
    for (int i = 0; i < d->n_bnd; i++) {
        int k = order[i];
        Bnd &B = sc->bnd[i];
        memset(&B, 0, sizeof B);
        B.type = d->bnd_type[k]; B.scene = d->bnd_scene[k];
        for (int j = 0; j < 12; j++) B.p[j] = d->bnd_param[12 * k + j];
        for (int j = 0; j < 3; j++) { B.vel[j] = d->bnd_vel[3 * k + j]; B.omg[j] = d->bnd_omega[3 * k + j]; }
        const double *m = d->bnd_mat + 4 * k;
        B.e = (1.0 - m[1] * m[1]) / m[0];
        B.g = 2.0 * (2.0 - m[1]) * (1.0 + m[1]) / m[0];
        B.mu = m[2]; B.beta = beta_of_cor(m[3]);
        B.ef = (float)B.e; B.gf = (float)B.g; B.muf = (float)B.mu; B.betaf = (float)B.beta;
    }
    // meshes, and their triangles sorted by scene (stable)
    sc->mesh.resize(d->n_mesh);
    sc->mesh_speed.assign(d->n_mesh, 0.0);
    for (int k = 0; k < d->n_mesh; k++) {
        Mesh &M = sc->mesh[k];
        memset(&M, 0, sizeof M);
        mesh_set_state(M, d->mesh_state + 13 * k);
        const double *m = d->mesh_mat + 4 * k;
        M.e = (1.0 - m[1] * m[1]) / m[0];
        M.g = 2.0 * (2.0 - m[1]) * (1.0 + m[1]) / m[0];
        M.mu = m[2]; M.beta = beta_of_cor(m[3]);
        M.ef = (float)M.e; M.gf = (float)M.g; M.muf = (float)M.mu; M.betaf = (float)M.beta;
        M.scene = d->mesh_scene[k];
    }
    for (int64_t k = 0; k < d->n_tri; k++) {  // rmax: the farthest vertex from its mesh's reference point
        Mesh &M = sc->mesh[d->tri_mesh[k]];
        for (int j = 0; j < 3; j++) M.rmax = std::max(M.rmax, norm3(d->tri_vertex + 9 * k + 3 * j));
    }
    std::vector<double> tri_vb(9 * (size_t)d->n_tri);
    {
        std::vector<int32_t> tord(d->n_tri);
        for (int64_t k = 0; k < d->n_tri; k++) tord[k] = (int32_t)k;
        std::stable_sort(tord.begin(), tord.end(), [&](int32_t a, int32_t b) {
            return d->mesh_scene[d->tri_mesh[a]] < d->mesh_scene[d->tri_mesh[b]];
        });
        sc->tri_user = tord;
        sc->tri_mesh.resize(d->n_tri);
        for (int64_t i = 0; i < d->n_tri; i++) {
            sc->tri_mesh[i] = d->tri_mesh[tord[i]];
            memcpy(&tri_vb[9 * i], d->tri_vertex + 9 * (size_t)tord[i], 72);
        }
    }
    S.n_mesh = d->n_mesh;
    S.n_tri = d->n_tri;
    set_bnd_margins(sc);
    sc->grids.resize(d->n_scenes);
    sc->dom.assign(d->domain, d->domain + 6 * d->n_scenes);
    for (int k = 0; k < d->n_scenes; k++) {
        Grid &g = sc->grids[k];
        memset(&g, 0, sizeof g);
        g.gx = d->gravity[3 * k]; g.gy = d->gravity[3 * k + 1]; g.gz = d->gravity[3 * k + 2];
        g.bnd_beg = g.bnd_end = 0;
    }
    std::vector<int32_t> chunk_tri;
    {
        int i = 0;
        for (int k = 0; k < d->n_scenes; k++) {
            sc->grids[k].bnd_beg = i;
            while (i < d->n_bnd && sc->bnd[i].scene == k) i++;
            sc->grids[k].bnd_end = i;
        }
        int64_t j = 0;
        for (int k = 0; k < d->n_scenes; k++) {
            Grid &g = sc->grids[k];
            g.sid = k;
            g.tri_beg = (int32_t)j;
            while (j < d->n_tri && sc->mesh[sc->tri_mesh[j]].scene == k) j++;
            g.tri_end = (int32_t)j;
            // chunks of at most 64 consecutive triangles of this scene
            g.chunk_beg = (int32_t)chunk_tri.size();
            for (int64_t t = g.tri_beg; t < g.tri_end; t += 64) chunk_tri.push_back((int32_t)t);
            g.chunk_end = (int32_t)chunk_tri.size();
        }
        S.n_chunk = (int64_t)chunk_tri.size();
        chunk_tri.push_back((int32_t)d->n_tri);
    }
    std::vector<int32_t> big;
    for (int64_t c = 0; c < nc; c++) if (sbeg[c + 1] - sbeg[c] > kBigClump) big.push_back((int32_t)c);
    sc->tri_box_len = 6 * (S.n_tri + S.n_chunk + S.n_scenes);
    // per template: the largest |o_s| + R_s (acceleration envelope) and the
    // largest |o_s| (displacement guard) of its spheres, stored as floats
    std::vector<double> r_acc(nt), r_ctr(nt);
    for (int32_t t = 0; t < nt; t++) {
        double ra = 0, rc = 0;
        for (uint32_t i = d->tmpl_sphere_begin[t]; i < d->tmpl_sphere_begin[t + 1]; i++) {
            const double *o = d->tmpl_offset + 3 * i;
            const double r = std::sqrt(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]);
            ra = std::max(ra, r + d->tmpl_radius[i]);
            rc = std::max(rc, r);
        }
        r_acc[t] = (double)(float)ra;
        r_ctr[t] = (double)std::nextafter((float)rc, 3.0e38f);  // rounded up
    }
    // wave schedule of the force kernel: pack whole clumps into groups of at
    // most 64 spheres, as (first, end) clump pairs; big clumps are skipped
    std::vector<int32_t> wsched;
    std::vector<uint32_t> wclump;
    for (int64_t c = 0; c < nc;) {
        if (sbeg[c + 1] - sbeg[c] > kBigClump) { c++; continue; }
        int64_t start = c, n = 0;
        while (c < nc) {
            int64_t k = sbeg[c + 1] - sbeg[c];
            if (k > kBigClump || n + k > 64) break;
            n += k;
            c++;
        }
        wsched.push_back((int32_t)sbeg[start]);
        wsched.push_back((int32_t)sbeg[c]);
        wclump.push_back((uint32_t)start);
    }
    std::vector<uint32_t> sinfo(ns), sts(ns);
    for (int64_t c = 0; c < nc; c++) {
        const int64_t k = sbeg[c + 1] - sbeg[c];
        const uint32_t t = d->clump_template[c];
        for (int64_t s = sbeg[c]; s < sbeg[c + 1]; s++) {
            sinfo[s] = k <= kBigClump ? (uint32_t)(s - sbeg[c]) | ((uint32_t)k << 8) : 0u;
            sts[s] = d->tmpl_sphere_begin[t] + (uint32_t)(s - sbeg[c]);
        }
    }
    S.n_waves = (int64_t)wsched.size() / 2;
    S.n_rblocks = (S.n_waves + 3) / 4;            // workgroups of the reduction (four waves each)
    S.n_ablocks = std::min<int64_t>((ns + 255) / 256, kStepGrid);  // workgroups of the audit
    S.part_r = (uint32_t *)dev_alloc(sc, 12 * (S.n_rblocks + 256));  // + the folded partials
    S.part_a = (unsigned long long *)dev_alloc(sc, 16 * std::max<int64_t>(S.n_ablocks, 1));
    S.part_c = (uint32_t *)dev_alloc(sc, 4 * (size_t)kPairBlocksMax);
    S.part_k = (double *)dev_alloc(sc, 2 * 8 * (size_t)kRegionBlocksMax);
    if (!S.part_r || !S.part_a || !S.part_c || !S.part_k) return bail(fail(sc, CDEM_E_OOM, "partials"));
    S.stride_cap = 16384;
    S.plan.k_max = 1; S.plan.audit_period = 0; S.plan.safety = 1.5f;
    S.plan.margin_cap = 0.0f; S.plan.margin_floor = 0.0f; S.plan.v_user = 0.0f; S.plan.test_zero_margin = 0;
    {
        double rs = 0.0;  // mean radius of the sphere instances (the interval rule's false-positive model)
        for (int64_t c = 0; c < nc; c++) {
            const uint32_t t = d->clump_template[c];
            for (uint32_t i = d->tmpl_sphere_begin[t]; i < d->tmpl_sphere_begin[t + 1]; i++) rs += d->tmpl_radius[i];
        }
        S.plan.r_mean = ns ? (float)(rs / (double)ns) : 0.0f;
    }
    // ---- device arrays
    int rc = CDEM_OK;
    {
        // clump records, (x, M), (v, r_acc), q, (w_body, r_ctr), uploaded in slices
        const int64_t slice = 1 << 20;
        std::vector<double4> rec(4 * std::min<int64_t>(std::max<int64_t>(nc, 1), slice));
        S.cst = (double4 *)dev_alloc(sc, 4 * sizeof(double4) * std::max<int64_t>(nc, 1));
        if (!S.cst) return bail(fail(sc, CDEM_E_OOM, "device allocation failed"));
        for (int64_t c0 = 0; c0 < nc; c0 += slice) {
            const int64_t n = std::min(slice, nc - c0);
            for (int64_t k = 0; k < n; k++) {
                const int64_t c = c0 + k;
                const uint32_t t = d->clump_template[c];
                const double *x = d->x + 3 * c, *q = d->q + 4 * c, *v = d->v + 3 * c, *w = d->w + 3 * c;
                double xe[3] = {x[0], x[1], x[2]};
                if (d->pos_exp)  // the integer k = rint(x 2^E), stored bit for bit
                    for (int i = 0; i < 3; i++) {
                        const long long kq = (long long)std::rint(std::ldexp(x[i], d->pos_exp));
                        memcpy(&xe[i], &kq, 8);
                    }
                rec[4 * k + 0] = make_double4(xe[0], xe[1], xe[2], d->tmpl_mass[t]);
                rec[4 * k + 1] = make_double4(v[0], v[1], v[2], r_acc[t]);
                rec[4 * k + 2] = make_double4(q[0], q[1], q[2], q[3]);
                rec[4 * k + 3] = make_double4(w[0], w[1], w[2], r_ctr[t]);
            }
            if (hipMemcpy(S.cst + 4 * c0, rec.data(), 4 * sizeof(double4) * n, hipMemcpyHostToDevice) != hipSuccess)
                return bail(fail(sc, CDEM_E_HIP, "upload"));
        }
    }
    std::vector<double4> tmi(nt);
    for (int32_t t = 0; t < nt; t++)
        tmi[t] = make_double4(d->tmpl_mass[t], d->tmpl_inertia[3 * t], d->tmpl_inertia[3 * t + 1],
                              d->tmpl_inertia[3 * t + 2]);
#define UP(field, src, n)                                   \
    do {                                                    \
        auto *p_ = upload(sc, (src), (n), rc);              \
        if (!p_) return bail(rc);                           \
        S.field = p_;                                       \
    } while (0)
    UP(tmpl_mi, tmi.data(), nt);
    UP(sbeg, sbeg.data(), nc + 1);
    UP(presc, presc.data(), nc);
    UP(presc_param, d->presc_param, 12 * (size_t)d->n_presc);
    UP(clump_tmpl, d->clump_template, nc);
    UP(clump_scene, d->clump_scene, nc);
    UP(tmpl_sbeg, d->tmpl_sphere_begin, nt + 1);
    UP(tmpl_ofs, d->tmpl_offset, 3 * (size_t)nts);
    UP(tmpl_rad, d->tmpl_radius, nts);
    UP(owner, owner.data(), ns);
    UP(sscene, sscene.data(), ns);
    UP(mat64, mat64.data(), ns);
    UP(mat32, mat32.data(), ns);
    UP(bnd, sc->bnd.data(), sc->bnd.size());
    UP(mesh, sc->mesh.data(), sc->mesh.size());
    UP(tri_vb, tri_vb.data(), tri_vb.size());
    UP(tri_mesh, sc->tri_mesh.data(), sc->tri_mesh.size());
    UP(chunk_tri, chunk_tri.data(), chunk_tri.size());
    UP(big_list, big.data(), big.size());
    {
        std::vector<int64_t> bsb(big.size() + 1, 0);
        for (size_t k = 0; k < big.size(); k++) bsb[k + 1] = bsb[k] + (sbeg[big[k] + 1] - sbeg[big[k]]);
        UP(big_sbeg, bsb.data(), bsb.size());
        S.bdet = (double4 *)dev_alloc(sc, sizeof(double4) * std::max<int64_t>(bsb.back(), 1));
        if (!S.bdet) return bail(fail(sc, CDEM_E_OOM, "device allocation failed"));
    }
    UP(wave_s, wsched.data(), wsched.size());
    UP(wave_c, wclump.data(), wclump.size());
    UP(sinfo, sinfo.data(), sinfo.size());
    UP(sts, sts.data(), sts.size());
#undef UP
    S.n_big = (int32_t)big.size();
    S.spos = (double4 *)dev_alloc(sc, sizeof(double4) * std::max<int64_t>(ns, 1));
    S.cdet = (double4 *)dev_alloc(sc, 2 * sizeof(double4) * std::max<int64_t>(nc, 1));
    S.cell_of = (uint32_t *)dev_alloc(sc, 4 * std::max<int64_t>(ns, 1));
    S.cell_rank = (uint32_t *)dev_alloc(sc, 4 * std::max<int64_t>(ns, 1));
    S.sorted_meta = (uint4 *)dev_alloc(sc, sizeof(uint4) * std::max<int64_t>(ns, 1));
    S.sorted_pos = (double4 *)dev_alloc(sc, sizeof(double4) * std::max<int64_t>(ns, 1));
    S.sorted_f4 = (float4 *)dev_alloc(sc, sizeof(float4) * std::max<int64_t>(ns, 1));
    S.stage = (uint32_t *)dev_alloc(sc, 4 * (size_t)kMaxRow * std::max<int64_t>(ns, 1));
    S.stage_n = (uint2 *)dev_alloc(sc, sizeof(uint2) * std::max<int64_t>(ns, 1));
    const size_t nnb = (size_t)((std::max<int64_t>(ns, 1) + kNarrowBlock - 1) / kNarrowBlock);
    S.narrow_part = (unsigned long long *)dev_alloc(sc, 24 * nnb);
    S.narrow_woff = (uint32_t *)dev_alloc(sc, 8 * (kNarrowBlock / 64) * nnb);
    if (!S.sorted_f4 || !S.stage || !S.stage_n || !S.narrow_part || !S.narrow_woff)
        return bail(fail(sc, CDEM_E_OOM, "device allocation failed"));
    S.rec_cF = (double *)dev_alloc(sc, 24 * std::max<int64_t>(nc, 1));
    S.rec_cT = (double *)dev_alloc(sc, 24 * std::max<int64_t>(nc, 1));
    S.ctl = (Ctl *)dev_alloc(sc, sizeof(Ctl));
    S.sspeed = (float *)dev_alloc(sc, 4 * std::max<int64_t>(ns, 1));
    S.cacc = (float *)dev_alloc(sc, 4 * std::max<int64_t>(nc, 1));
    S.cell_t = (uint32_t *)dev_alloc(sc, 4 * std::max<int64_t>(ns, 1));
    // spheres with more than kMaxRow candidates are rare (a large sphere among
    // many small ones); a list of ns/8 (at least 4096) of them per detection
    S.over_cap = std::max<int64_t>(4096, ns / 8);
    S.over_list = (uint32_t *)dev_alloc(sc, 4 * S.over_cap);
    S.fb_list = (uint32_t *)dev_alloc(sc, 4 * std::max<int64_t>(S.ns, 1));
    if (!S.sspeed || !S.cacc || !S.cell_t || !S.over_list || !S.fb_list) return bail(fail(sc, CDEM_E_OOM, "device allocation failed"));
    if (d->n_tri) {
        S.tri_box = (double *)dev_alloc(sc, 8 * (size_t)sc->tri_box_len);
        if (!S.tri_box) return bail(fail(sc, CDEM_E_OOM, "device allocation failed"));
    }
    for (int k = 0; k < 3; k++) {  // per-sphere structure of the three active-set slots
        S.lo_beg[k] = (uint32_t *)dev_alloc(sc, 4 * std::max<int64_t>(ns, 1));
        S.lo_cnt[k] = (uint32_t *)dev_alloc(sc, 4 * std::max<int64_t>(ns, 1));
        S.up_beg[k] = (uint32_t *)dev_alloc(sc, 4 * std::max<int64_t>(ns, 1));
        S.up_cnt[k] = (uint32_t *)dev_alloc(sc, 4 * std::max<int64_t>(ns, 1));
        S.smargin[k] = (float *)dev_alloc(sc, 4 * std::max<int64_t>(ns, 1));
        if (!S.lo_beg[k] || !S.lo_cnt[k] || !S.up_beg[k] || !S.up_cnt[k] || !S.smargin[k])
            return bail(fail(sc, CDEM_E_OOM, "device allocation failed"));
    }
    if (!S.cdet || !S.spos || !S.cell_of || !S.cell_rank || !S.sorted_meta || !S.sorted_pos || !S.rec_cF ||
        !S.rec_cT || !S.ctl)
        return bail(fail(sc, CDEM_E_OOM, "device allocation failed"));
    if (!big.empty()) {
        S.sF = (double *)dev_alloc(sc, 24 * ns);
        S.sT = (double *)dev_alloc(sc, 24 * ns);
        if (!S.sF || !S.sT) return bail(fail(sc, CDEM_E_OOM, "device allocation failed"));
    }
    if ((rc = build_grids(sc)) != CDEM_OK) return bail(rc);
    // testing aid: deferred detection with zero margin and no guard, which
    // misses contacts on purpose so the audit's failure path can be tested
    sc->test_no_guard = getenv("CDEM_TEST_NO_GUARD") != nullptr;
    // testing aid: the displacement guard without its per-clump bound
    sc->S.guard_exact = getenv("CDEM_TEST_EXACT_GUARD") != nullptr ? 1 : 0;
    int64_t cap0 = std::max<int64_t>(4 * ns, 1024);  // pairs; grown on demand
    if (const char *ev = getenv("CDEM_INITIAL_CAPACITY")) cap0 = std::max<int64_t>(atoll(ev), 64);  // testing aid
    if ((rc = alloc_active_set(sc, cap0, false)) != CDEM_OK) return bail(rc);
    Ctl c;
    memset(&c, 0, sizeof c);
    c.det_due = 1;
    c.k_cur = 1;
    c.bslot = 2;  // no detection ahead yet: slots 0 and 1 alternate
    if (hipMemcpyAsync(S.ctl, &c, sizeof c, hipMemcpyHostToDevice, sc->stream) != hipSuccess) return bail(fail(sc, CDEM_E_HIP, "ctl"));
    for (int k = 0; k < 3; k++) {
        if (launch_zero(S.lo_beg[k], 4 * (size_t)ns, sc->stream) != hipSuccess ||
            launch_zero(S.lo_cnt[k], 4 * (size_t)ns, sc->stream) != hipSuccess ||
            launch_zero(S.up_beg[k], 4 * (size_t)ns, sc->stream) != hipSuccess ||
            launch_zero(S.up_cnt[k], 4 * (size_t)ns, sc->stream) != hipSuccess ||
            launch_zero(S.smargin[k], 4 * (size_t)ns, sc->stream) != hipSuccess)
            return bail(fail(sc, CDEM_E_HIP, "zero"));
    }
    if (launch_zero(S.part_c, 4 * (size_t)kPairBlocksMax, sc->stream) != hipSuccess ||
        launch_zero(S.part_k, 2 * 8 * (size_t)kRegionBlocksMax, sc->stream) != hipSuccess)
        return bail(fail(sc, CDEM_E_HIP, "zero"));
    if (launch_zero(S.cacc, 4 * (size_t)nc, sc->stream) != hipSuccess ||
        launch_zero(S.sspeed, 4 * (size_t)ns, sc->stream) != hipSuccess ||
        launch_zero(S.cdet, 2 * sizeof(double4) * nc, sc->stream) != hipSuccess)
        return bail(fail(sc, CDEM_E_HIP, "zero"));
    if (hipStreamSynchronize(sc->stream) != hipSuccess) return bail(fail(sc, CDEM_E_HIP, "sync"));
    *out = sc;
    return CDEM_OK;
}

extern "C" int cdem_destroy(cdem_scene *sc) {
    if (!sc) return CDEM_E_INVALID;
    (void)hipStreamSynchronize(sc->stream);
    drop_graph(sc);
    if (sc->gstream) { (void)hipStreamSynchronize(sc->gstream); (void)hipStreamDestroy(sc->gstream); }
    delete sc->timer;
    sc->timer = nullptr;
    if (sc->law_module) (void)hipModuleUnload(sc->law_module);
    if (sc->ahead.stream) {
        (void)hipStreamSynchronize(sc->ahead.stream);
        (void)hipStreamDestroy(sc->ahead.stream);
        (void)hipEventDestroy(sc->ahead.ev_snap);
        (void)hipEventDestroy(sc->ahead.ev_det);
        sc->ahead.stream = nullptr;
    }
    auto owned = sc->owned;
    for (void *p : owned) dev_free(sc, p);
    (void)hipStreamSynchronize(sc->stream);  // stream-ordered frees complete before the scene is gone
    delete sc;
    return CDEM_OK;
}

static int read_ctl(cdem_scene *sc, Ctl &c) {
    HIPCHK(hipStreamSynchronize(sc->stream));
    HIPCHK(hipMemcpy(&c, sc->S.ctl, sizeof c, hipMemcpyDeviceToHost));
    return CDEM_OK;
}

static int write_ctl(cdem_scene *sc, const Ctl &c) {
    HIPCHK(hipMemcpyAsync(sc->S.ctl, &c, sizeof c, hipMemcpyHostToDevice, sc->stream));
    HIPCHK(hipStreamSynchronize(sc->stream));
    return CDEM_OK;
}

// Enqueue the kernels of n steps on st (timed when a timer is set and we are
// not capturing a graph).
static int enqueue_on(cdem_scene *sc, int64_t n, hipStream_t st, bool capturing, int64_t step0 = 0) {
    const DevScene &S = sc->S;
    auto &a = sc->ahead;

    g_timer = capturing ? nullptr : sc->timer;
    for (int64_t i = 0; i < n; i++) {
        hipError_t e = hipSuccess;
        if (a.on && (step0 + i - a.origin) % a.K == 0) {
            // adopt the set built ahead during the last interval, then take
            // the snapshot the next one is built from
            if (a.inflight) {
                if (hipStreamWaitEvent(st, a.ev_det, 0) != hipSuccess) { g_timer = nullptr; return fail(sc, CDEM_E_HIP, "wait"); }
                e = launch_adopt(S, ahead_view(sc), st);
                a.inflight = false;
            }
            const DevScene B = ahead_view(sc);
            if (e == hipSuccess) e = launch_snapshot(S, B, st);
            if (e == hipSuccess) e = hipEventRecord(a.ev_snap, st);
            if (e == hipSuccess) e = hipStreamWaitEvent(a.stream, a.ev_snap, 0);
            if (e == hipSuccess) e = launch_detect_ahead(B, a.stream);
            if (e == hipSuccess) e = hipEventRecord(a.ev_det, a.stream);
            if (e != hipSuccess) { g_timer = nullptr; return fail(sc, CDEM_E_HIP, hipGetErrorString(e)); }
            a.inflight = true;
        }
        e = launch_pose(S, st, false);
        if (e == hipSuccess && sc->collecting) e = launch_collect_speed(S, st);
        if (e == hipSuccess) e = launch_detect(S, st);
        if (e == hipSuccess) e = launch_audit_binned(S, st);
        if (e == hipSuccess) e = launch_force_integrate(S, st, sc->law_pairs);
        if (e == hipSuccess && sc->collecting) e = launch_collect_acc(S, st);
        if (e == hipSuccess) e = launch_step_end(S, st);
        if (e != hipSuccess) { g_timer = nullptr; return fail(sc, CDEM_E_HIP, hipGetErrorString(e)); }
        if (!capturing && sc->timer && sc->timer->used > 4096) {  // bound the event pool
            HIPCHK(hipStreamSynchronize(st));
            if (a.stream) HIPCHK(hipStreamSynchronize(a.stream));
            sc->timer->harvest();
        }
    }
    g_timer = nullptr;
    return CDEM_OK;
}

static void drop_graph(cdem_scene *sc) {
    if (sc->gexec) (void)hipGraphExecDestroy(sc->gexec);
    sc->gexec = nullptr;
}

// Capture graph_steps steps once per set of launch parameters.
static int ensure_graph(cdem_scene *sc) {
    if (sc->gexec && memcmp(&sc->gkey, &sc->S, sizeof(DevScene)) == 0) return CDEM_OK;
    drop_graph(sc);
    if (!sc->gstream) HIPCHK(hipStreamCreateWithFlags(&sc->gstream, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(sc->gstream, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_on(sc, sc->graph_steps, sc->gstream, true);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(sc->gstream, &g);
    if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
    if (e != hipSuccess) return fail(sc, CDEM_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&sc->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) { sc->gexec = nullptr; return fail(sc, CDEM_E_HIP, hipGetErrorString(e)); }
    sc->gkey = sc->S;
    return CDEM_OK;
}

static int enqueue_steps(cdem_scene *sc, int64_t n, int64_t step0) {
    // graphs carry no per-kernel events: a timed or collecting run goes eager;
    // so does the overlap mode (the host schedules its second stream)
    if (sc->ahead.on || sc->graph_steps <= 0 || sc->timer || sc->collecting || n < sc->graph_steps)
        return enqueue_on(sc, n, sc->stream, false, step0);
    int rc = ensure_graph(sc);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(sc->stream));
    int64_t reps = n / sc->graph_steps;
    for (int64_t r = 0; r < reps; r++) HIPCHK(hipGraphLaunch(sc->gexec, sc->gstream));
    HIPCHK(hipStreamSynchronize(sc->gstream));
    return enqueue_on(sc, n - reps * sc->graph_steps, sc->stream, false);
}

extern "C" int cdem_step(cdem_scene *sc, int64_t n, void *stream) {
    if (!sc || n < 0) return fail(sc, CDEM_E_INVALID, "bad arguments");
    if (stream) sc->stream = (hipStream_t)stream;
    Ctl c;
    int rc = read_ctl(sc, c);
    if (rc) return rc;
    int64_t target = c.step + n;
    int64_t missed0 = c.missed;
    const int64_t step0 = c.step;
    const int32_t rec0 = c.record;  // the recording asked for the first step
    for (int attempt = 0; attempt < 8; attempt++) {
        int64_t left = target - c.step;
        if (left <= 0) break;
        if ((rc = enqueue_steps(sc, left, c.step)) != CDEM_OK) return rc;
        if ((rc = read_ctl(sc, c)) != CDEM_OK) return rc;
        if (sc->timer) {
            if ((rc = ahead_drain(sc, false)) != CDEM_OK) return rc;
            sc->timer->harvest();
        }
        if (c.nonfinite) return fail(sc, CDEM_E_NAN, "non-finite clump state");
        if (c.ahead_dropped) {
            // a set built ahead outgrew the storage: grow it (the steps ran on
            // the set in use, which the guard kept valid)
            if ((rc = ahead_drain(sc, true)) != CDEM_OK) return rc;
            Ctl b;
            HIPCHK(hipMemcpy(&b, sc->ahead.ctl, sizeof b, hipMemcpyDeviceToHost));
            if (b.row_overflow)
                return fail(sc, CDEM_E_CAPACITY, "too many spheres with more than 16 candidate partners (margin too large)");
            int64_t need = (int64_t)(1.3 * (double)std::max(b.n_up, b.n_pairs)) + 1024;
            int64_t cap = std::max<int64_t>(2 * sc->S.cap, need);
            if (cap > kMaxCap && std::max(b.n_up, b.n_pairs) < kMaxCap) cap = kMaxCap;
            if ((rc = alloc_active_set(sc, cap, true)) != CDEM_OK) return rc;
            sc->regrows++;
            c.ahead_dropped = 0;
            if ((rc = write_ctl(sc, c)) != CDEM_OK) return rc;
        }
        if (!c.overflow) break;
        if (c.row_overflow)
            return fail(sc, CDEM_E_CAPACITY, "too many spheres with more than 16 candidate partners (margin too large)");
        if (c.asym) return fail(sc, CDEM_E_STATE, "active-set rows are not symmetric");
        // grow the active set and resume from the step that did not complete
        if ((rc = ahead_drain(sc, true)) != CDEM_OK) return rc;
        int64_t need = (int64_t)(1.3 * (double)std::max(c.n_up, c.n_pairs)) + 1024;
        int64_t cap = std::max<int64_t>(2 * sc->S.cap, need);
        if (cap > kMaxCap && std::max(c.n_up, c.n_pairs) < kMaxCap) cap = kMaxCap;
        if ((rc = alloc_active_set(sc, cap, true)) != CDEM_OK) return rc;
        sc->regrows++;
        c.overflow = 0;
        c.row_overflow = 0;
        c.asym = 0;
        c.det_due = 1;
        c.record = c.step == step0 ? rec0 : 0;  // a recorded step that did not complete records when run again
        if ((rc = write_ctl(sc, c)) != CDEM_OK) return rc;
    }
    if (c.step != target) return fail(sc, CDEM_E_CAPACITY, "active set could not be grown");
    if (c.missed > missed0)
        return fail(sc, CDEM_E_MISSED_CONTACT, "an audit found contacts missing from the active set");
    return CDEM_OK;
}

extern "C" int cdem_sync(cdem_scene *sc) {
    if (!sc) return CDEM_E_INVALID;
    HIPCHK(hipStreamSynchronize(sc->stream));
    return CDEM_OK;
}

extern "C" int cdem_set_detection(cdem_scene *sc, const cdem_detect_params *p) {
    if (!sc || !p) return fail(sc, CDEM_E_INVALID, "null argument");
    if (p->mode < 0 || p->mode > 2 || p->k_max < 1 || p->k_max > 20 || !(p->safety >= 1.0) ||
        !(p->margin_cap >= 0.0) || p->audit_period < 0 || !(p->v_max_user >= 0.0))
        return fail(sc, CDEM_E_INVALID, "detection parameters out of range");
    if (p->mode != CDEM_DETECT_PLAIN && !(p->margin_cap > 0.0))
        return fail(sc, CDEM_E_INVALID, "deferred detection needs a positive margin cap");
    if (p->mode == CDEM_DETECT_LEARNED && !sc->S.mlp)
        return fail(sc, CDEM_E_STATE, "learned detection needs MLP parameters (cdem_set_mlp)");
    if (p->overlap != 0 && p->overlap != 1) return fail(sc, CDEM_E_INVALID, "overlap is 0 or 1");
    if (p->overlap && p->mode == CDEM_DETECT_PLAIN)
        return fail(sc, CDEM_E_INVALID, "overlap needs deferred detection (a margin covers the steps ahead)");
    int rc = ahead_drain(sc, true);
    if (rc) return rc;
    Ctl c;
    if ((rc = read_ctl(sc, c)) != CDEM_OK) return rc;
    if (p->overlap && sc->nslots < 3) {  // the third slot's pair storage
        sc->nslots = 3;
        if ((rc = alloc_active_set(sc, sc->S.cap, true)) != CDEM_OK) return rc;
    }
    auto &a = sc->ahead;
    a.on = p->overlap != 0;
    a.K = std::max(1, p->k_max);
    a.origin = c.step;
    // the slot reserved for the second stream: never the set in use (a
    // detection on the step's stream takes the third; with two slots of pair
    // storage, slots 0 and 1 alternate)
    c.bslot = sc->nslots == 3 ? (c.buf + 2) % 3 : 2;
    sc->S.overlap = a.on ? 1 : 0;
    sc->det = *p;
    sc->S.detect_mode = p->mode;
    sc->S.plan.k_max = p->mode == CDEM_DETECT_PLAIN ? 1 : p->k_max;
    sc->S.plan.audit_period = p->audit_period;
    sc->S.plan.safety = (float)p->safety;
    sc->S.plan.margin_cap = (float)p->margin_cap;
    sc->S.plan.margin_floor = (float)std::min(1e-7, 0.5 * p->margin_cap);
    sc->S.plan.v_user = (float)p->v_max_user;
    sc->S.plan.test_zero_margin = sc->test_no_guard ? 1 : 0;
    sc->S.store_speed = p->mode == CDEM_DETECT_LEARNED ? 1 : 0;
    sc->S.store_acc = p->mode == CDEM_DETECT_LEARNED ? 1 : 0;
    sc->S.guard_on = p->mode != CDEM_DETECT_PLAIN && !sc->test_no_guard ? 1 : 0;
    set_bnd_margins(sc);
    HIPCHK(hipMemcpyAsync((void *)sc->S.bnd, sc->bnd.data(), sc->bnd.size() * sizeof(Bnd), hipMemcpyHostToDevice, sc->stream));
    if ((rc = push_meshes(sc)) != CDEM_OK) return rc;
    if ((rc = build_grids(sc)) != CDEM_OK) return rc;
    if (a.on && (rc = ahead_alloc(sc)) != CDEM_OK) return rc;
    c.det_due = 1;
    c.k_cur = p->mode == CDEM_DETECT_PLAIN ? 1 : p->k_max;
    return write_ctl(sc, c);
}

extern "C" int cdem_record_next_step(cdem_scene *sc, int on) {
    if (!sc) return CDEM_E_INVALID;
    if (on < 0 || on > 2) return fail(sc, CDEM_E_INVALID, "record mode is 0, 1 or 2");
    DevScene &S = sc->S;
    const bool fresh = on && sc->rec_cap < S.cap;  // new arrays: the last recorded step is gone
    if (fresh) {
        dev_free(sc, S.rec_state); dev_free(sc, S.rec_delta); dev_free(sc, S.rec_F); dev_free(sc, S.rec_R);
        dev_free(sc, S.rec_Ta); dev_free(sc, S.rec_Tb);
        S.rec_state = (uint8_t *)dev_alloc(sc, S.cap);
        S.rec_delta = (double *)dev_alloc(sc, 8 * S.cap);
        S.rec_F = (double *)dev_alloc(sc, 24 * S.cap);
        S.rec_R = (double *)dev_alloc(sc, 24 * S.cap);
        S.rec_Ta = (double *)dev_alloc(sc, 24 * S.cap);
        S.rec_Tb = (double *)dev_alloc(sc, 24 * S.cap);
        if (!S.rec_state || !S.rec_delta || !S.rec_F || !S.rec_R || !S.rec_Ta || !S.rec_Tb) {
            sc->rec_cap = 0;  // nothing may record into them
            return fail(sc, CDEM_E_OOM, "recording buffers");
        }
        sc->rec_cap = S.cap;
    }
    Ctl c;
    int rc = read_ctl(sc, c);
    if (rc) return rc;
    c.record = on;
    if (fresh) c.rec_last = 0;
    return write_ctl(sc, c);
}

extern "C" int cdem_get_counts(cdem_scene *sc, cdem_counts *out) {
    if (!sc || !out) return fail(sc, CDEM_E_INVALID, "null argument");
    Ctl c;
    int rc = read_ctl(sc, c);
    if (rc) return rc;
    memset(out, 0, sizeof *out);
    out->clumps = sc->S.nc; out->spheres = sc->S.ns; out->bins = sc->S.n_cells;
    out->candidates = c.n_pairs_cur + c.n_up_cur; out->steps = c.step; out->detections = c.detections;
    out->guard_trips = c.guard_trips; out->fallbacks = c.fallbacks; out->audits = c.audits;
    out->missed = c.missed; out->capacity = sc->S.cap; out->regrows = sc->regrows; out->k_current = c.k_cur;
    out->pairs = c.n_pairs_cur;
    out->audit_contacts = c.audit_true;
    return CDEM_OK;
}

// The clump state as row-major host arrays x [nc][3], q [nc][4], v [nc][3],
// w [nc][3] (any may be null), through a device staging buffer.
// raw: with fixed-point positions, the integers bit for bit (checkpoints)
static int state_to_host(cdem_scene *sc, double *x, double *q, double *v, double *w, bool raw = false) {
    const DevScene &S = sc->S;
    const int64_t nc = S.nc;
    if (nc == 0) return CDEM_OK;
    double *stage = (double *)dev_alloc(sc, 13 * 8 * (size_t)nc);
    if (!stage) return fail(sc, CDEM_E_OOM, "state staging buffer");
    double *dx = stage, *dq = stage + 3 * nc, *dv = stage + 7 * nc, *dw = stage + 10 * nc;
    hipError_t e = launch_pack_state(S, dx, dq, dv, dw, 0, sc->stream, raw ? 1 : 0);
    if (e == hipSuccess) e = hipStreamSynchronize(sc->stream);
    double *dst[4] = {x, q, v, w}, *src[4] = {dx, dq, dv, dw};
    const int width[4] = {3, 4, 3, 3};
    for (int a = 0; a < 4 && e == hipSuccess; a++)
        if (dst[a]) e = hipMemcpy(dst[a], src[a], 8 * width[a] * (size_t)nc, hipMemcpyDeviceToHost);
    dev_free(sc, stage);
    if (e != hipSuccess) return fail(sc, CDEM_E_HIP, hipGetErrorString(e));
    return CDEM_OK;
}

static int state_from_host(cdem_scene *sc, const double *x, const double *q, const double *v, const double *w,
                           bool raw = false) {
    const DevScene &S = sc->S;
    const int64_t nc = S.nc;
    if (nc == 0) return CDEM_OK;
    double *stage = (double *)dev_alloc(sc, 13 * 8 * (size_t)nc);
    if (!stage) return fail(sc, CDEM_E_OOM, "state staging buffer");
    double *dx = stage, *dq = stage + 3 * nc, *dv = stage + 7 * nc, *dw = stage + 10 * nc;
    const double *src[4] = {x, q, v, w};
    double *dst[4] = {dx, dq, dv, dw};
    const int width[4] = {3, 4, 3, 3};
    hipError_t e = hipSuccess;
    for (int a = 0; a < 4 && e == hipSuccess; a++)
        if (src[a]) e = hipMemcpy(dst[a], src[a], 8 * width[a] * (size_t)nc, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = launch_pack_state(S, x ? dx : nullptr, q ? dq : nullptr, v ? dv : nullptr, w ? dw : nullptr, 1, sc->stream,
                              raw ? 1 : 0);
    if (e == hipSuccess) e = hipStreamSynchronize(sc->stream);
    dev_free(sc, stage);
    if (e != hipSuccess) return fail(sc, CDEM_E_HIP, hipGetErrorString(e));
    return CDEM_OK;
}

extern "C" int cdem_read_state(cdem_scene *sc, const cdem_state_view *v, int where, void *stream) {
    if (!sc || !v || (where != CDEM_HOST && where != CDEM_DEVICE)) return fail(sc, CDEM_E_INVALID, "bad arguments");
    const DevScene &S = sc->S;
    if (stream) sc->stream = (hipStream_t)stream;
    HIPCHK(hipStreamSynchronize(sc->stream));
    if (where == CDEM_DEVICE) {
        HIPCHK(launch_pack_state(S, v->x, v->q, v->v, v->w, 0, sc->stream));
        HIPCHK(hipStreamSynchronize(sc->stream));
        return CDEM_OK;
    }
    return state_to_host(sc, v->x, v->q, v->v, v->w);
}

extern "C" int cdem_write_state(cdem_scene *sc, const cdem_state_view *v, int where, void *stream) {
    if (!sc || !v || (where != CDEM_HOST && where != CDEM_DEVICE)) return fail(sc, CDEM_E_INVALID, "bad arguments");
    const DevScene &S = sc->S;
    int64_t nc = S.nc;
    if (stream) sc->stream = (hipStream_t)stream;
    HIPCHK(hipStreamSynchronize(sc->stream));
    if (int rc0 = ahead_drain(sc, true)) return rc0;  // a set built from the old state is dropped
    if (where == CDEM_DEVICE) {
        HIPCHK(launch_pack_state(S, v->x, v->q, v->v, v->w, 1, sc->stream));
    } else {
        if (v->q)
            for (int64_t c = 0; c < nc; c++) {
                double qn = 0;
                for (int k = 0; k < 4; k++) qn += v->q[4 * c + k] * v->q[4 * c + k];
                if (!(std::fabs(qn - 1.0) < 1e-10)) return fail(sc, CDEM_E_INVALID, "quaternions must be unit");
            }
        const double *src[4] = {v->x, v->q, v->v, v->w};
        const int width[4] = {3, 4, 3, 3};
        for (int a = 0; a < 4; a++)
            if (src[a] && !finite_all(src[a], width[a] * (size_t)nc)) return fail(sc, CDEM_E_INVALID, "non-finite state");
        int rc = state_from_host(sc, v->x, v->q, v->v, v->w);
        if (rc) return rc;
    }
    Ctl c;
    int rc = read_ctl(sc, c);
    if (rc) return rc;
    c.det_due = 1;
    return write_ctl(sc, c);
}

extern "C" int cdem_read_sphere_pos(cdem_scene *sc, double *xs) {
    if (!sc || !xs) return fail(sc, CDEM_E_INVALID, "null argument");
    const DevScene &S = sc->S;
    HIPCHK(launch_pose(S, sc->stream, true));
    std::vector<double4> p(S.ns);
    HIPCHK(hipStreamSynchronize(sc->stream));
    HIPCHK(hipMemcpy(p.data(), S.spos, S.ns * sizeof(double4), hipMemcpyDeviceToHost));
    for (int64_t s = 0; s < S.ns; s++) { xs[3 * s] = p[s].x; xs[3 * s + 1] = p[s].y; xs[3 * s + 2] = p[s].z; }
    return CDEM_OK;
}

extern "C" int cdem_read_contacts(cdem_scene *sc, cdem_contacts_view *v) {
    if (!sc || !v) return fail(sc, CDEM_E_INVALID, "null argument");
    const DevScene &S = sc->S;
    if (!sc->rec_cap) return fail(sc, CDEM_E_STATE, "no recorded step (call cdem_record_next_step first)");
    Ctl c;
    int rc = read_ctl(sc, c);
    if (rc) return rc;
    if (!c.rec_last) return fail(sc, CDEM_E_STATE, "no recorded step (call cdem_record_next_step first)");
    int cur = c.buf;
    int64_t ne = c.n_pairs_cur, ns = S.ns;
    std::vector<uint32_t> beg(ns), cnt(ns), nb(ne);
    std::vector<uint8_t> st(ne);
    std::vector<double> dl(ne), F(3 * ne), H(3 * ne), Ta(v->Ta ? 3 * ne : 0), Tb(v->Tb ? 3 * ne : 0);
    if (ns) {
        HIPCHK(hipMemcpy(beg.data(), S.lo_beg[cur], 4 * ns, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(cnt.data(), S.lo_cnt[cur], 4 * ns, hipMemcpyDeviceToHost));
    }
    if (ne) {
        HIPCHK(hipMemcpy(nb.data(), S.pt[cur], 4 * ne, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(st.data(), S.rec_state, ne, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(dl.data(), S.rec_delta, 8 * ne, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(F.data(), S.rec_F, 24 * ne, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(H.data(), S.hist[c.hb], 24 * ne, hipMemcpyDeviceToHost));
        if (v->Ta) HIPCHK(hipMemcpy(Ta.data(), S.rec_Ta, 24 * ne, hipMemcpyDeviceToHost));
        if (v->Tb) HIPCHK(hipMemcpy(Tb.data(), S.rec_Tb, 24 * ne, hipMemcpyDeviceToHost));
    }
    struct Row { uint64_t key; int64_t e; };
    std::vector<Row> rows;
    for (int64_t s = 0; s < ns; s++)
        for (uint32_t k = 0; k < cnt[s]; k++) {
            int64_t e = (int64_t)beg[s] + k;
            uint32_t t = nb[e];
            if (!st[e] || (c.rec_last == 2 && t < (uint32_t)ns)) continue;
            // pairs are listed once, in the lower sphere's segment
            rows.push_back({((uint64_t)s << 32) | user_partner(sc, t), e});
        }
    std::sort(rows.begin(), rows.end(), [](const Row &x, const Row &y) { return x.key < y.key; });
    v->n = (int64_t)rows.size();
    for (int64_t i = 0; i < std::min<int64_t>(v->n, v->cap); i++) {
        int64_t e = rows[i].e;
        if (v->a) v->a[i] = (uint32_t)(rows[i].key >> 32);
        if (v->b) v->b[i] = (uint32_t)(rows[i].key & 0xffffffffu);
        if (v->delta) v->delta[i] = dl[e];
        for (int k = 0; k < 3; k++) {
            if (v->F) v->F[3 * i + k] = F[3 * e + k];
            if (v->u) v->u[3 * i + k] = H[3 * e + k];
            if (v->Ta) v->Ta[3 * i + k] = Ta[3 * e + k];
            if (v->Tb) v->Tb[3 * i + k] = Tb[3 * e + k];
        }
    }
    return CDEM_OK;
}

extern "C" int cdem_read_boundary_forces(cdem_scene *sc, double *F, double *T) {
    if (!sc) return CDEM_E_INVALID;
    const DevScene &S = sc->S;
    if (!sc->rec_cap) return fail(sc, CDEM_E_STATE, "no recorded step (call cdem_record_next_step first)");
    const int nb = S.n_bnd;
    if (nb == 0) return CDEM_OK;
    {
        Ctl c;
        if (int rc = read_ctl(sc, c)) return rc;
        if (!c.rec_last) return fail(sc, CDEM_E_STATE, "no recorded step (call cdem_record_next_step first)");
    }
    double *part = (double *)dev_alloc(sc, sizeof(double) * 6 * kBndParts * (size_t)nb);
    double *out = (double *)dev_alloc(sc, sizeof(double) * 6 * (size_t)nb);
    std::vector<double> h(6 * (size_t)nb);
    int rc = CDEM_OK;
    if (!part || !out) {
        rc = fail(sc, CDEM_E_OOM, "boundary force buffers");
    } else if (launch_bnd_forces(S, part, out, sc->stream) != hipSuccess ||
               hipStreamSynchronize(sc->stream) != hipSuccess ||
               hipMemcpy(h.data(), out, h.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
        rc = fail(sc, CDEM_E_HIP, "boundary force reduction");
    }
    dev_free(sc, part);
    dev_free(sc, out);
    if (rc) return rc;
    for (int b = 0; b < nb; b++) {
        const int u = sc->bnd_user[b];
        for (int k = 0; k < 3; k++) {
            if (F) F[3 * u + k] = h[6 * b + k];
            if (T) T[3 * u + k] = h[6 * b + 3 + k];
        }
    }
    return CDEM_OK;
}

extern "C" int cdem_read_clump_forces(cdem_scene *sc, double *F, double *T) {
    if (!sc) return CDEM_E_INVALID;
    HIPCHK(hipStreamSynchronize(sc->stream));
    if (F) HIPCHK(hipMemcpy(F, sc->S.rec_cF, 24 * sc->S.nc, hipMemcpyDeviceToHost));
    if (T) HIPCHK(hipMemcpy(T, sc->S.rec_cT, 24 * sc->S.nc, hipMemcpyDeviceToHost));
    return CDEM_OK;
}

extern "C" int cdem_audit(cdem_scene *sc, cdem_audit_result *r) {
    if (!sc || !r) return fail(sc, CDEM_E_INVALID, "null argument");
    const DevScene &S = sc->S;
    if (S.ns > 400000) return fail(sc, CDEM_E_INVALID, "exhaustive audit is limited to 400k spheres");
    unsigned long long *cnt = (unsigned long long *)dev_alloc(sc, 3 * 8);
    if (!cnt) return fail(sc, CDEM_E_OOM, "audit counters");
    unsigned long long init[3] = {0, 0, ~0ull};
    HIPCHK(hipMemcpyAsync(cnt, init, sizeof init, hipMemcpyHostToDevice, sc->stream));
    HIPCHK(launch_pose(S, sc->stream, true));
    HIPCHK(launch_audit_brute(S, cnt, (uint32_t *)(cnt + 2), sc->stream));
    HIPCHK(hipStreamSynchronize(sc->stream));
    unsigned long long out[3];
    HIPCHK(hipMemcpy(out, cnt, sizeof out, hipMemcpyDeviceToHost));
    dev_free(sc, cnt);
    r->true_contacts = (int64_t)out[0];
    r->missed = (int64_t)out[1];
    r->first_a = out[1] ? (uint32_t)(out[2] >> 32) : 0;
    uint32_t fb = (uint32_t)(out[2] & 0xffffffffu);
    if (out[1]) fb = user_partner(sc, fb);
    r->first_b = out[1] ? fb : 0;
    return out[1] ? CDEM_E_MISSED_CONTACT : CDEM_OK;
}

extern "C" int cdem_profile(cdem_scene *sc, int on) {
    if (!sc) return CDEM_E_INVALID;
    HIPCHK(hipStreamSynchronize(sc->stream));
    delete sc->timer;
    sc->timer = on ? new (std::nothrow) EventTimer() : nullptr;
    if (on && !sc->timer) return fail(sc, CDEM_E_OOM, "timer");
    return CDEM_OK;
}

extern "C" int cdem_profile_kernels(cdem_scene *sc, const char *names) {
    if (!sc) return CDEM_E_INVALID;
    int rc = cdem_profile(sc, 1);
    if (rc || !names || !*names) return rc;
    bool any = false;
    for (int i = 0; i < K_COUNT; i++) {
        sc->timer->sel[i] = false;
        const size_t len = strlen(kKernelNames[i]);
        for (const char *p = names; *p;) {
            const char *q = strchr(p, ',');
            const size_t l = q ? (size_t)(q - p) : strlen(p);
            if (l == len && strncmp(p, kKernelNames[i], l) == 0) sc->timer->sel[i] = true;
            if (!q) break;
            p = q + 1;
        }
        any = any || sc->timer->sel[i];
    }
    if (!any) {
        delete sc->timer;
        sc->timer = nullptr;
        return fail(sc, CDEM_E_INVALID, "no kernel of that name");
    }
    return CDEM_OK;
}

extern "C" int cdem_profile_read(cdem_scene *sc, cdem_kernel_time *out, int cap, int *n) {
    if (!sc || !n || (cap > 0 && !out)) return fail(sc, CDEM_E_INVALID, "bad arguments");
    int k = 0;
    if (sc->timer) {
        HIPCHK(hipStreamSynchronize(sc->stream));
        sc->timer->harvest();
        for (int i = 0; i < K_COUNT; i++) {
            if (!sc->timer->launches[i]) continue;
            if (k < cap) {
                memset(&out[k], 0, sizeof out[k]);
                snprintf(out[k].name, sizeof out[k].name, "%s", kKernelNames[i]);
                out[k].launches = sc->timer->launches[i];
                out[k].total_ms = sc->timer->total_ms[i];
            }
            k++;
        }
    }
    *n = k;
    return CDEM_OK;
}

extern "C" int cdem_last_step_contacts(cdem_scene *sc, int64_t *n) {
    if (!sc || !n) return CDEM_E_INVALID;
    *n = 0;
    Ctl c;
    int rc = read_ctl(sc, c);
    if (rc) return rc;
    if (c.step == 0 || c.n_pairs_cur == 0) return CDEM_OK;  // nothing evaluated yet
    constexpr int kBlk = 1024;
    unsigned long long *part = (unsigned long long *)dev_alloc(sc, kBlk * sizeof(unsigned long long));
    if (!part) return fail(sc, CDEM_E_OOM, "contact count partials");
    std::vector<unsigned long long> h(kBlk);
    if (launch_count_contacts(sc->S, part, kBlk, sc->stream) != hipSuccess ||
        hipStreamSynchronize(sc->stream) != hipSuccess ||
        hipMemcpy(h.data(), part, kBlk * sizeof(unsigned long long), hipMemcpyDeviceToHost) != hipSuccess)
        rc = fail(sc, CDEM_E_HIP, "contact count");
    dev_free(sc, part);
    for (unsigned long long v : h) *n += (int64_t)v;
    return rc;
}

namespace cdem {
hipError_t launch_collect_begin(const DevScene &S, hipStream_t st);
}

extern "C" int cdem_set_mlp(cdem_scene *sc, const float *params, int64_t n) {
    if (!sc || !params || n != cdem_mlp_param_count()) return fail(sc, CDEM_E_INVALID, "MLP parameter count");
    for (int64_t i = 0; i < n; i++)
        if (!std::isfinite(params[i])) return fail(sc, CDEM_E_INVALID, "non-finite MLP parameter");
    for (int k = 0; k < 3; k++)
        if (!(params[3 + k] > 0.f)) return fail(sc, CDEM_E_INVALID, "MLP standardisation scale must be positive");
    if (!sc->S.mlp) {
        sc->S.mlp = (const float *)dev_alloc(sc, n * sizeof(float));
        if (!sc->S.mlp) return fail(sc, CDEM_E_OOM, "MLP parameters");
    }
    HIPCHK(hipMemcpyAsync((void *)sc->S.mlp, params, n * sizeof(float), hipMemcpyHostToDevice, sc->stream));
    HIPCHK(hipStreamSynchronize(sc->stream));
    return CDEM_OK;
}

extern "C" int cdem_collect_envelopes(cdem_scene *sc, int32_t horizon, float *features, float *labels, int64_t cap,
                                      int64_t *n) {
    if (!sc || !n || horizon < 1 || cap < 0 || (cap > 0 && (!features || !labels)))
        return fail(sc, CDEM_E_INVALID, "bad arguments");
    if (int rc0 = ahead_drain(sc, false)) return rc0;
    DevScene &S = sc->S;
    int32_t ss = S.store_speed, sa = S.store_acc;
    S.store_speed = 1;
    S.store_acc = 1;
    auto restore = [&](int rc) { S.store_speed = ss; S.store_acc = sa; sc->collecting = false; return rc; };
    int rc = cdem_step(sc, 1, nullptr);  // one step so that every clump has an acceleration envelope
    if (rc) return restore(rc);
    hipError_t e = launch_pose(S, sc->stream, true);
    if (e == hipSuccess) e = launch_collect_begin(S, sc->stream);
    if (e != hipSuccess) return restore(fail(sc, CDEM_E_HIP, hipGetErrorString(e)));
    int64_t nb = S.n_regions;
    std::vector<uint32_t> fv(nb), fa(nb), occ(nb), lv(nb), la(nb);
    if (hipStreamSynchronize(sc->stream) != hipSuccess ||
        hipMemcpy(fv.data(), S.bin_v, 4 * nb, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(fa.data(), S.bin_a, 4 * nb, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(occ.data(), S.occ_t, 4 * nb, hipMemcpyDeviceToHost) != hipSuccess)
        return restore(fail(sc, CDEM_E_HIP, "feature copy"));
    Ctl c;
    if ((rc = read_ctl(sc, c)) != CDEM_OK) return restore(rc);
    c.collecting = 1;
    if ((rc = write_ctl(sc, c)) != CDEM_OK) return restore(rc);
    sc->collecting = true;
    rc = cdem_step(sc, horizon, nullptr);
    sc->collecting = false;
    int rc2 = read_ctl(sc, c);
    c.collecting = 0;
    if (!rc2) rc2 = write_ctl(sc, c);
    if (rc) return restore(rc);
    if (rc2) return restore(rc2);
    if (hipMemcpy(lv.data(), S.lab_v, 4 * nb, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(la.data(), S.lab_a, 4 * nb, hipMemcpyDeviceToHost) != hipSuccess)
        return restore(fail(sc, CDEM_E_HIP, "label copy"));
    auto f32 = [](uint32_t b) { float x; memcpy(&x, &b, 4); return x; };
    int64_t k = 0;
    for (int64_t i = 0; i < nb; i++) {
        if (!occ[i]) continue;
        if (k < cap) {
            features[3 * k] = f32(fv[i]);
            features[3 * k + 1] = f32(fa[i]);
            features[3 * k + 2] = (float)occ[i];
            labels[2 * k] = std::log(f32(lv[i]) + 1e-6f);
            labels[2 * k + 1] = std::log(f32(la[i]) + 1e-3f);
        }
        k++;
    }
    *n = k;
    return restore(CDEM_OK);
}

extern "C" int cdem_set_graph(cdem_scene *sc, int32_t steps_per_graph) {
    if (!sc || steps_per_graph < 0 || steps_per_graph > 1000) return fail(sc, CDEM_E_INVALID, "steps per graph 0..1000");
    HIPCHK(hipStreamSynchronize(sc->stream));
    drop_graph(sc);
    sc->graph_steps = steps_per_graph;
    return CDEM_OK;
}

extern "C" int cdem_autotune(cdem_scene *sc, int32_t steps, double *bin_factor, int32_t *stride_cap) {
    if (!sc || steps < 1) return fail(sc, CDEM_E_INVALID, "bad arguments");
    const double factors[] = {0.75, 1.0, 1.25, 1.5, 1.75};
    const int32_t caps[] = {2048, 4096, 8192, 16384};
    double best = 1e300, bf = sc->bin_factor;
    int32_t bc = sc->S.stride_cap;
    int rc = cdem_step(sc, 1, nullptr);  // settle allocations before timing
    if (rc) return rc;
    if (!sc->gstream) HIPCHK(hipStreamCreateWithFlags(&sc->gstream, hipStreamNonBlocking));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    for (double f : factors) {
        sc->bin_factor = f;
        if ((rc = ahead_drain(sc, true)) != CDEM_OK) break;  // the second stream reads the grids
        if ((rc = build_grids(sc)) != CDEM_OK) break;
        if (sc->ahead.on && (rc = ahead_alloc(sc)) != CDEM_OK) break;
        for (int32_t cap : caps) {
            sc->S.stride_cap = cap;
            Ctl c;
            if ((rc = read_ctl(sc, c)) != CDEM_OK) break;
            c.det_due = 1;  // the new bins need a detection
            if ((rc = write_ctl(sc, c)) != CDEM_OK) break;
            (void)hipEventRecord(e0, sc->stream);
            if ((rc = cdem_step(sc, steps, nullptr)) != CDEM_OK) break;
            (void)hipEventRecord(e1, sc->stream);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < best) { best = ms; bf = f; bc = cap; }
        }
        if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    sc->bin_factor = bf;
    sc->S.stride_cap = bc;
    if ((rc = ahead_drain(sc, true)) != CDEM_OK) return rc;
    if ((rc = build_grids(sc)) != CDEM_OK) return rc;
    if (sc->ahead.on && (rc = ahead_alloc(sc)) != CDEM_OK) return rc;
    Ctl c;
    if ((rc = read_ctl(sc, c)) != CDEM_OK) return rc;
    c.det_due = 1;
    if ((rc = write_ctl(sc, c)) != CDEM_OK) return rc;
    if (bin_factor) *bin_factor = bf;
    if (stride_cap) *stride_cap = bc;
    return CDEM_OK;
}

// ---------------------------------------------------------------- triangle meshes
extern "C" int cdem_read_mesh_state(cdem_scene *sc, double *state) {
    if (!sc || (!state && sc->S.n_mesh)) return fail(sc, CDEM_E_INVALID, "null argument");
    const int32_t n = sc->S.n_mesh;
    if (!n) return CDEM_OK;
    std::vector<Mesh> dev(n);
    HIPCHK(hipStreamSynchronize(sc->stream));
    HIPCHK(hipMemcpy(dev.data(), sc->S.mesh, n * sizeof(Mesh), hipMemcpyDeviceToHost));
    for (int32_t m = 0; m < n; m++) {
        double *r = state + 13 * m;
        for (int i = 0; i < 3; i++) { r[i] = dev[m].x[i]; r[7 + i] = dev[m].v[i]; r[10 + i] = dev[m].w[i]; }
        for (int i = 0; i < 4; i++) r[3 + i] = dev[m].q[i];
    }
    return CDEM_OK;
}

// A new velocity whose speed bound the mesh's margin still covers, at an
// unchanged pose, keeps the active set (every point of the mesh moves no
// farther per step than the margin assumed); anything else, a new pose or a
// faster motion, resizes the margin and detects again before the next step.
extern "C" int cdem_set_mesh_state(cdem_scene *sc, int32_t mesh, const double *state) {
    if (!sc || !state) return fail(sc, CDEM_E_INVALID, "null argument");
    if (mesh < 0 || mesh >= sc->S.n_mesh) return fail(sc, CDEM_E_INVALID, "mesh index out of range");
    if (!mesh_state_ok(state)) return fail(sc, CDEM_E_INVALID, "mesh state (finite, unit quaternion)");
    int rc;
    HIPCHK(hipStreamSynchronize(sc->stream));
    Mesh cur;
    HIPCHK(hipMemcpy(&cur, sc->S.mesh + mesh, sizeof(Mesh), hipMemcpyDeviceToHost));
    Mesh &M = sc->mesh[mesh];
    mesh_set_state(M, state);
    const bool same_pose = memcmp(cur.x, M.x, sizeof M.x) == 0 && memcmp(cur.q, M.q, sizeof M.q) == 0;
    const bool covered = mesh_speed_of(M) <= sc->mesh_speed[mesh];
    if (same_pose && covered) {  // only the velocities change; the margin is kept
        M.margin = cur.margin;
        HIPCHK(hipMemcpy(sc->S.mesh + mesh, &M, sizeof(Mesh), hipMemcpyHostToDevice));
        return CDEM_OK;
    }
    if ((rc = ahead_drain(sc, true)) != CDEM_OK) return rc;  // a set built for the old motion is dropped
    const double kh = (double)margin_steps(sc) * sc->S.h * 1.01;
    sc->mesh_speed[mesh] = kMeshSpeedHeadroom * mesh_speed_of(M);
    M.margin = sc->mesh_speed[mesh] * kh;
    HIPCHK(hipMemcpy(sc->S.mesh + mesh, &M, sizeof(Mesh), hipMemcpyHostToDevice));
    Ctl c;
    if ((rc = read_ctl(sc, c)) != CDEM_OK) return rc;
    c.det_due = 1;
    return write_ctl(sc, c);
}

extern "C" int cdem_read_mesh_forces(cdem_scene *sc, double *F, double *T) {
    if (!sc) return CDEM_E_INVALID;
    const DevScene &S = sc->S;
    if (!sc->rec_cap) return fail(sc, CDEM_E_STATE, "no recorded step (call cdem_record_next_step first)");
    const int32_t nm = S.n_mesh;
    if (!nm) return CDEM_OK;
    {
        Ctl c;
        if (int rc = read_ctl(sc, c)) return rc;
        if (!c.rec_last) return fail(sc, CDEM_E_STATE, "no recorded step (call cdem_record_next_step first)");
    }
    // the triangle contacts of the recorded step, compacted on the device
    // (a few per mesh-touching sphere), then ordered by (a, b) as the caller
    // numbers them: Newton's third law at each contact point, the mesh
    // receiving -F with the lever arm from its reference point
    int64_t cap = std::max<int64_t>(sc->mesh_cap, 1024);
    std::vector<unsigned long long> keys;
    std::vector<double> FR;
    unsigned long long n = 0;
    for (int pass = 0; pass < 2; pass++) {
        char *buf = (char *)dev_alloc(sc, 8 + 56 * (size_t)cap);
        if (!buf) return fail(sc, CDEM_E_OOM, "mesh contact buffer");
        unsigned long long *cnt = (unsigned long long *)buf, *k = cnt + 1;
        double *fr = (double *)(k + cap);
        hipError_t e = launch_zero(cnt, 8, sc->stream);
        if (e == hipSuccess) e = launch_mesh_contacts(S, k, fr, cnt, cap, sc->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(sc->stream);
        if (e == hipSuccess) e = hipMemcpy(&n, cnt, 8, hipMemcpyDeviceToHost);
        if (e == hipSuccess && (int64_t)n <= cap) {
            keys.resize(n);
            FR.resize(6 * n);
            if (n) e = hipMemcpy(keys.data(), k, 8 * n, hipMemcpyDeviceToHost);
            if (e == hipSuccess && n) e = hipMemcpy(FR.data(), fr, 48 * n, hipMemcpyDeviceToHost);
        }
        dev_free(sc, buf);
        if (e != hipSuccess) return fail(sc, CDEM_E_HIP, hipGetErrorString(e));
        if ((int64_t)n <= cap) break;
        cap = (int64_t)n + (int64_t)n / 4 + 1024;  // grown once, to what the recorded step holds
    }
    sc->mesh_cap = cap;
    const uint32_t t0 = (uint32_t)(S.ns + S.n_bnd);
    struct Row { uint64_t key; int64_t i; int32_t mesh; };
    std::vector<Row> rows(n);
    for (unsigned long long i = 0; i < n; i++) {
        const uint32_t s = (uint32_t)(keys[i] >> 32), t = (uint32_t)(keys[i] & 0xffffffffu);
        rows[i] = {((uint64_t)s << 32) | user_partner(sc, t), (int64_t)i, sc->tri_mesh[t - t0]};
    }
    std::sort(rows.begin(), rows.end(), [](const Row &x, const Row &y) { return x.key < y.key; });
    std::vector<double> f(3 * nm, 0.0), tq(3 * nm, 0.0);
    for (const Row &r : rows) {
        const double *Fr = &FR[6 * r.i], *a = &FR[6 * r.i + 3];
        const double g[3] = {-Fr[0], -Fr[1], -Fr[2]};
        const double x[3] = {a[1] * g[2] - a[2] * g[1], a[2] * g[0] - a[0] * g[2], a[0] * g[1] - a[1] * g[0]};
        for (int i = 0; i < 3; i++) {
            f[3 * r.mesh + i] = f[3 * r.mesh + i] + g[i];
            tq[3 * r.mesh + i] = tq[3 * r.mesh + i] + x[i];
        }
    }
    if (F) memcpy(F, f.data(), 24 * (size_t)nm);
    if (T) memcpy(T, tq.data(), 24 * (size_t)nm);
    return CDEM_OK;
}

// ---------------------------------------------------------------- checkpoints
namespace {
struct SaveHeader {
    char magic[8];
    int32_t abi, precision;
    int64_t nc, ns, n_bnd, n_scenes;
    uint64_t fingerprint;
    int64_t entries;
    cdem_detect_params det;
    int32_t has_mlp, stride_cap;
    double bin_factor;
    Ctl ctl;
};
constexpr char kSaveMagic[8] = {'C', 'D', 'E', 'M', 'S', 'A', 'V', '2'};

size_t save_size(const DevScene &S, int64_t entries, bool mlp) {
    return sizeof(SaveHeader) + 13 * 8 * (size_t)S.nc + 13 * 8 * (size_t)S.n_mesh + 8 * (size_t)S.ns +
           4 * (size_t)entries + 24 * (size_t)entries + (mlp ? 4 * (size_t)cdem_mlp_param_count() : 0);
}
}  // namespace

extern "C" int cdem_save(cdem_scene *sc, void *buf, size_t cap, size_t *len) {
    if (!sc || !len || (cap > 0 && !buf)) return fail(sc, CDEM_E_INVALID, "bad arguments");
    const DevScene &S = sc->S;
    Ctl c;
    int rc = read_ctl(sc, c);
    if (rc) return rc;
    const int64_t E = c.n_pairs_cur;
    const bool mlp = S.mlp != nullptr;
    const size_t need = save_size(S, E, mlp);
    *len = need;
    if (cap == 0) return CDEM_OK;
    if (cap < need) return fail(sc, CDEM_E_INVALID, "checkpoint buffer too small");
    SaveHeader hd{};
    memcpy(hd.magic, kSaveMagic, 8);
    hd.abi = CDEM_ABI_VERSION;
    hd.precision = S.precision;
    hd.nc = S.nc; hd.ns = S.ns; hd.n_bnd = S.n_bnd; hd.n_scenes = S.n_scenes;
    hd.fingerprint = sc->fingerprint;
    hd.entries = E;
    hd.det = sc->det;
    hd.has_mlp = mlp ? 1 : 0;
    hd.stride_cap = S.stride_cap;
    hd.bin_factor = sc->bin_factor;
    hd.ctl = c;
    char *o = (char *)buf;
    memcpy(o, &hd, sizeof hd);
    o += sizeof hd;
    {  // the clump state: x [nc][3], q [nc][4], v [nc][3], w [nc][3]
        double *st = (double *)o;
        const int64_t nc = S.nc;
        if ((rc = state_to_host(sc, st, st + 3 * nc, st + 7 * nc, st + 10 * nc, true)) != CDEM_OK) return rc;
        o += 13 * 8 * (size_t)nc;
    }
    if (S.n_mesh) {  // the mesh states [n_mesh][13]
        if ((rc = cdem_read_mesh_state(sc, (double *)o)) != CDEM_OK) return rc;
        o += 13 * 8 * (size_t)S.n_mesh;
    }
    const int cur = c.buf;
    if (S.ns) {
        HIPCHK(hipMemcpy(o, S.lo_beg[cur], 4 * S.ns, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(o + 4 * S.ns, S.lo_cnt[cur], 4 * S.ns, hipMemcpyDeviceToHost));
    }
    o += 8 * S.ns;
    if (E) {
        HIPCHK(hipMemcpy(o, S.pt[cur], 4 * E, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(o + 4 * E, S.hist[c.hb], 24 * E, hipMemcpyDeviceToHost));
    }
    o += 28 * E;
    if (mlp) HIPCHK(hipMemcpy(o, S.mlp, 4 * (size_t)cdem_mlp_param_count(), hipMemcpyDeviceToHost));
    return CDEM_OK;
}

extern "C" int cdem_load(cdem_scene *sc, const void *buf, size_t len) {
    if (!sc || !buf || len < sizeof(SaveHeader)) return fail(sc, CDEM_E_INVALID, "bad arguments");
    if (int rc0 = ahead_drain(sc, true)) return rc0;
    SaveHeader hd;
    memcpy(&hd, buf, sizeof hd);
    DevScene &S = sc->S;
    if (memcmp(hd.magic, kSaveMagic, 8) != 0 || hd.abi != CDEM_ABI_VERSION)
        return fail(sc, CDEM_E_INVALID, "not a checkpoint of this library version");
    if (hd.precision != S.precision || hd.nc != S.nc || hd.ns != S.ns || hd.n_bnd != S.n_bnd ||
        hd.n_scenes != S.n_scenes || hd.fingerprint != sc->fingerprint)
        return fail(sc, CDEM_E_INVALID, "checkpoint belongs to another scene description");
    const int64_t E = hd.entries;
    if (E < 0 || E >= ((int64_t)1 << 32) || len != save_size(S, E, hd.has_mlp != 0))
        return fail(sc, CDEM_E_INVALID, "checkpoint size does not match its header");
    const char *p = (const char *)buf + sizeof hd;
    const double *mst = (const double *)(p + 13 * 8 * (size_t)S.nc);
    for (int32_t m = 0; m < S.n_mesh; m++)
        if (!mesh_state_ok(mst + 13 * m)) return fail(sc, CDEM_E_INVALID, "checkpoint mesh state");
    const char *rows = p + 13 * 8 * (size_t)(S.nc + S.n_mesh);
    const uint32_t *rb = (const uint32_t *)rows, *rn = (const uint32_t *)(rows + 4 * S.ns);
    for (int64_t s = 0; s < S.ns; s++)
        if ((uint64_t)rb[s] + rn[s] > (uint64_t)E) return fail(sc, CDEM_E_INVALID, "checkpoint rows out of range");
    int rc;
    if (hd.has_mlp) {
        const float *w = (const float *)(rows + 8 * S.ns + 28 * (size_t)E);
        if ((rc = cdem_set_mlp(sc, w, (size_t)cdem_mlp_param_count())) != CDEM_OK) return rc;
    }
    sc->bin_factor = hd.bin_factor > 0.0 ? hd.bin_factor : 1.0;
    S.stride_cap = hd.stride_cap > 0 && hd.stride_cap <= 16384 ? hd.stride_cap : 16384;
    for (int32_t m = 0; m < S.n_mesh; m++) mesh_set_state(sc->mesh[m], mst + 13 * m);
    if (S.n_mesh) {  // the saved poses and velocities (cdem_set_detection sizes the margins for them)
        HIPCHK(hipStreamSynchronize(sc->stream));
        HIPCHK(hipMemcpy(S.mesh, sc->mesh.data(), S.n_mesh * sizeof(Mesh), hipMemcpyHostToDevice));
    }
    if ((rc = cdem_set_detection(sc, &hd.det)) != CDEM_OK) return rc;
    if (E > S.cap && (rc = alloc_active_set(sc, E + E / 4 + 1024, false)) != CDEM_OK) return rc;
    Ctl c;
    if ((rc = read_ctl(sc, c)) != CDEM_OK) return rc;
    const int cur = c.buf;
    {
        const double *st = (const double *)p;
        const int64_t nc = S.nc;
        if ((rc = state_from_host(sc, st, st + 3 * nc, st + 7 * nc, st + 10 * nc, true)) != CDEM_OK) return rc;
    }
    if (S.ns) {
        HIPCHK(hipMemcpy(S.lo_beg[cur], rb, 4 * S.ns, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(S.lo_cnt[cur], rn, 4 * S.ns, hipMemcpyHostToDevice));
    }
    if (E) {
        HIPCHK(hipMemcpy(S.pt[cur], rows + 8 * S.ns, 4 * E, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(S.hist[c.hb], rows + 8 * S.ns + 4 * E, 24 * E, hipMemcpyHostToDevice));
    }
    // resume the saved schedule on this scene's buffers; the active set is
    // rebuilt (with the saved history carried over) before the next step
    Ctl n = hd.ctl;
    n.buf = cur;
    n.hb = c.hb;
    n.bslot = c.bslot;
    n.ahead_dropped = 0;
    n.n_pairs_cur = E;
    n.det_due = 1;
    n.overflow = 0; n.row_overflow = 0; n.asym = 0; n.record = 0; n.collecting = 0; n.nonfinite = 0;
    n.rec_last = 0;  // no step of this scene has been recorded since
    n.guard = 0;
    n.guard_next = 0;
    return write_ctl(sc, n);
}

// ---------------------------------------------------------------- user force law
// The pair kernel of the step with the force law replaced by a device
// function the caller supplies, compiled at run time with hiprtc for gfx950
// with the library's own floating-point flags.  The kernel source is the
// library's pair evaluation (headers embedded at build time) instantiated with
// the user's law.
static const char kRtcMain[] = R"CDEM_RTC_MAIN(
#include "pair_dev.h"
namespace cdem {
struct UserLaw {
    static constexpr bool kFP32 = false;
    __device__ static __forceinline__ void f64(const double *n, double delta, const double *vrel, double Rbar,
                                               double mbar, double estar, double gstar, double mu, double beta,
                                               double h, const double *u_old, double *F, double *u_new) {
        ::cdem_user_law(n, delta, vrel, Rbar, mbar, estar, gstar, mu, beta, h, u_old, F, u_new);
    }
};
}  // namespace cdem
extern "C" __global__ void __launch_bounds__(256) cdem_user_pairs64(cdem::DevScene S) {
    cdem::pairs_body<false, cdem::UserLaw>(S);
}
extern "C" __global__ void __launch_bounds__(256) cdem_user_pairs32(cdem::DevScene S) {
    cdem::pairs_body<true, cdem::UserLaw>(S);
}
)CDEM_RTC_MAIN";

static const char kRtcLawDecl[] =
    "__device__ void cdem_user_law(const double *n, double delta, const double *vrel, double Rbar, double mbar,\n"
    "                              double estar, double gstar, double mu, double beta, double h,\n"
    "                              const double *u_old, double *F, double *u_new);\n";

static void copy_log(const std::string &log, char *out, size_t cap) {
    if (!out || cap == 0) return;
    size_t n = std::min(cap - 1, log.size());
    memcpy(out, log.data(), n);
    out[n] = 0;
}

// Compile the user law into a code object; false with the compiler's log on error.
static bool compile_law(const char *source, std::vector<char> &code, std::string &log) {
    std::string src = std::string(kRtcLawDecl) + "#line 1 \"user_law\"\n" + source + "\n#line 1 \"cdem_pairs\"\n" +
                      kRtcMain;
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "cdem_user_pairs.hip", kRtcHeaderCount, kRtcHeaderTexts,
                            kRtcHeaderNames) != HIPRTC_SUCCESS) {
        log = "hiprtcCreateProgram failed";
        return false;
    }
    const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
                          "-fhip-fp32-correctly-rounded-divide-sqrt", "-Xclang", "-target-feature", "-Xclang",
                          "-packed-fp32-ops"};
    hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
    size_t ls = 0;
    hiprtcGetProgramLogSize(prog, &ls);
    log.assign(ls, '\0');
    if (ls) hiprtcGetProgramLog(prog, &log[0]);
    while (!log.empty() && log.back() == '\0') log.pop_back();
    bool ok = r == HIPRTC_SUCCESS;
    if (ok) {
        size_t cs = 0;
        ok = hiprtcGetCodeSize(prog, &cs) == HIPRTC_SUCCESS && cs > 0;
        if (ok) {
            code.resize(cs);
            ok = hiprtcGetCode(prog, code.data()) == HIPRTC_SUCCESS;
        }
        if (!ok && log.empty()) log = "no code object produced";
    }
    hiprtcDestroyProgram(&prog);
    return ok;
}

extern "C" int cdem_check_force_law(const char *source, char *log, size_t log_cap) {
    copy_log("", log, log_cap);
    if (!source || !*source) return CDEM_E_INVALID;
    std::vector<char> code;
    std::string lg;
    bool ok = compile_law(source, code, lg);
    copy_log(lg, log, log_cap);
    return ok ? CDEM_OK : CDEM_E_INVALID;
}

extern "C" int cdem_set_force_law(cdem_scene *sc, const char *source, char *log, size_t log_cap) {
    if (!sc) return CDEM_E_INVALID;
    copy_log("", log, log_cap);
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
    if (source && *source) {
        std::vector<char> code;
        std::string lg;
        if (!compile_law(source, code, lg)) {
            copy_log(lg, log, log_cap);
            return fail(sc, CDEM_E_INVALID, "the force law did not compile: " + lg.substr(0, 2000));
        }
        copy_log(lg, log, log_cap);
        HIPCHK(hipStreamSynchronize(sc->stream));
        if (hipModuleLoadData(&mod, code.data()) != hipSuccess)
            return fail(sc, CDEM_E_HIP, "hipModuleLoadData of the compiled force law failed");
        const char *name = sc->S.precision == 1 ? "cdem_user_pairs32" : "cdem_user_pairs64";
        if (hipModuleGetFunction(&fn, mod, name) != hipSuccess) {
            (void)hipModuleUnload(mod);
            return fail(sc, CDEM_E_HIP, "compiled force law has no pair kernel");
        }
    }
    HIPCHK(hipStreamSynchronize(sc->stream));
    drop_graph(sc);  // captured launches name the previous pair kernel
    if (sc->law_module) (void)hipModuleUnload(sc->law_module);
    sc->law_module = mod;
    sc->law_pairs = fn;
    return CDEM_OK;
}
