// C ABI of the projector library (declared in include/tsp.h): host-side
// validation, view frames, device memory management and kernel orchestration.

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <array>
#include <vector>

#include <mutex>

#include "tsp.h"
#include "tsp_internal.h"

using namespace tsp;

// Workspace of tsp_backproject_noalloc (the slot-ordered copy of y), a
// file-scope device array: every device the library runs on holds one copy
// from module load until the process ends.  In host code `scratch` names a
// host-side stand-in, not device memory; kernels get the device address
// that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) float scratch[TSP_NOALLOC_SCRATCH_BYTES / sizeof(float)];

namespace {

thread_local std::string g_err;

tsp_status fail(tsp_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

#define TSP_HIP(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(TSP_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
    } while (0)

const double kTwoPi = 6.283185307179586476925286766559;

// Keeps the caller's current device and switches to the geometry's.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

int64_t device_cap() {
    const char *s = std::getenv("TSP_MAX_DEVICE_BYTES");
    if (!s || !*s) return -1;
    char *end = nullptr;
    long long v = std::strtoll(s, &end, 10);
    return (end && *end == '\0' && v > 0) ? (int64_t)v : -1;
}

}  // namespace

int64_t tsp::max_blocks() {
    static const int64_t cap = [] {
        const char *s = std::getenv("TSP_MAX_BLOCKS");
        const long long v = s ? std::atoll(s) : 0;
        return (v > 0 && v < kMaxBlocks) ? (int64_t)v : kMaxBlocks;
    }();
    return cap;
}

struct tsp_geometry {
    int device = 0;
    TabDesc T{};
    double *d_tab = nullptr;
    RayDesc rd{};
    double *d_frames = nullptr, *d_starts = nullptr, *d_dirs = nullptr;
    int64_t V = 0, R = 0;
    double r_out = 0.0;  // outer radius of the grid
    int mode = 0;
    int64_t S = 0, max_per_ray = 0, n_stored = 0;
    // ray-major sliced store
    int32_t *d_perm = nullptr, *d_cnt_sorted = nullptr, *d_slice_len = nullptr;
    int64_t *d_slice_ptr = nullptr;
    uint8_t *d_code = nullptr;  // entry codes (voxel steps, escapes)
    float *d_len = nullptr;
    int64_t *d_row_ptr = nullptr;
    // voxel-major store
    int64_t *d_col_ptr = nullptr;   // [FV + 1] block offsets per key
    uint8_t *d_col_code = nullptr;  // slot increases and escapes
    float *d_col_len = nullptr;
    // dynamic objects: object frame per cone view (null for a static object)
    int32_t *d_obj_frame = nullptr;
    int64_t FV() const { return V * rd.n_obj_frames; }
    int64_t bytes = 0;
    std::vector<std::pair<void *, int64_t>> allocs;
    // Allocations come from an arena when `arena` is set: a stack of
    // 256-byte aligned blocks (offset, size, live) in [arena, arena +
    // arena_size); a block freed on top pops, with any dead blocks below it.
    // The chunk geometries of a deterministic adjoint without a stored
    // transposed list work in the arena their parent keeps in chunk_arena, so
    // that chunks and later calls reuse one allocation: mapping and unmapping
    // tens of GB per chunk would cost seconds.
    char *arena = nullptr;
    int64_t arena_size = 0;
    std::vector<std::array<int64_t, 3>> arena_blocks;
    mutable char *chunk_arena = nullptr;
    mutable int64_t chunk_arena_size = 0;
    // canonical segments per window of kWindow natural slots (host copy,
    // from the count pass): chunk boundaries of the deterministic adjoint
    // without a stored transposed list follow them
    std::vector<int32_t> win_segs;
    // serialises that adjoint's use of chunk_arena across threads
    mutable std::mutex chunk_mu;
    // events for the next forward or adjoint call (tsp_set_timing_events)
    mutable std::mutex timing_mu;
    mutable KernelEvents timing;
};

namespace {

tsp_status dalloc(tsp_geometry *g, void **p, int64_t bytes, const char *what) {
    *p = nullptr;
    if (bytes <= 0) bytes = 16;
    const int64_t cap = device_cap();
    if (cap > 0 && g->bytes + bytes > cap) {
        char buf[256];
        std::snprintf(buf, sizeof buf, "%s: %lld bytes would exceed TSP_MAX_DEVICE_BYTES=%lld",
                      what, (long long)bytes, (long long)cap);
        return fail(TSP_E_NOMEM, buf);
    }
    if (g->arena) {
        const int64_t off = g->arena_blocks.empty()
                                ? 0
                                : g->arena_blocks.back()[0] + g->arena_blocks.back()[1];
        const int64_t sz = (bytes + 255) / 256 * 256;
        if (off + sz > g->arena_size) {
            char buf[256];
            std::snprintf(buf, sizeof buf, "%s: %lld bytes exceed the chunk memory (%lld free)",
                          what, (long long)bytes, (long long)(g->arena_size - off));
            return fail(TSP_E_NOMEM, buf);
        }
        *p = g->arena + off;
        g->arena_blocks.push_back({off, sz, 1});
        g->bytes += bytes;
        g->allocs.push_back({*p, bytes});
        return TSP_OK;
    }
    hipError_t e = hipMalloc(p, (size_t)bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        char buf[256];
        std::snprintf(buf, sizeof buf, "%s: hipMalloc(%lld) failed: %s", what, (long long)bytes,
                      hipGetErrorString(e));
        return fail(TSP_E_NOMEM, buf);
    }
    g->bytes += bytes;
    g->allocs.push_back({*p, bytes});
    return TSP_OK;
}

template <class T>
tsp_status dalloc_n(tsp_geometry *g, T **p, int64_t n, const char *what) {
    void *q = nullptr;
    tsp_status s = dalloc(g, &q, n * (int64_t)sizeof(T), what);
    *p = (T *)q;
    return s;
}

void dfree(tsp_geometry *g, void *p) {
    if (!p) return;
    for (size_t i = 0; i < g->allocs.size(); i++) {
        if (g->allocs[i].first == p) {
            g->bytes -= g->allocs[i].second;
            g->allocs.erase(g->allocs.begin() + (long)i);
            break;
        }
    }
    if (g->arena) {
        const int64_t off = (char *)p - g->arena;
        for (auto &b : g->arena_blocks)
            if (b[0] == off) b[2] = 0;
        while (!g->arena_blocks.empty() && g->arena_blocks.back()[2] == 0)
            g->arena_blocks.pop_back();
        return;
    }
    (void)hipFree(p);
}

// Bytes that new allocations of g may take: the arena's free top, or the
// driver's free memory less a margin (5% of the device, at least 2 GiB).
// -1 when the driver cannot say.
int64_t usable_bytes(const tsp_geometry *g) {
    if (g->arena) {
        const int64_t off = g->arena_blocks.empty()
                                ? 0
                                : g->arena_blocks.back()[0] + g->arena_blocks.back()[1];
        return g->arena_size - off;
    }
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
        (void)hipGetLastError();
        return -1;
    }
    const int64_t margin = std::max<int64_t>((int64_t)1 << 31, (int64_t)(tot / 20));
    return (int64_t)fr - margin;
}

void release_chunk_arena(const tsp_geometry *g) {
    if (!g->chunk_arena) return;
    (void)hipFree(g->chunk_arena);
    g->chunk_arena = nullptr;
    g->chunk_arena_size = 0;
}

template <class T>
void dfree_p(tsp_geometry *g, T *&p) {
    dfree(g, (void *)p);
    p = nullptr;
}

void release_stores(tsp_geometry *g) {
    dfree_p(g, g->d_perm);
    dfree_p(g, g->d_cnt_sorted);
    dfree_p(g, g->d_slice_len);
    dfree_p(g, g->d_slice_ptr);
    dfree_p(g, g->d_code);
    dfree_p(g, g->d_len);
    dfree_p(g, g->d_row_ptr);
    dfree_p(g, g->d_col_ptr);
    dfree_p(g, g->d_col_code);
    dfree_p(g, g->d_col_len);
    release_chunk_arena(g);
    g->mode = 0;
    g->S = g->max_per_ray = g->n_stored = 0;
}

bool finite3(const double *v) {
    return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]);
}

tsp_status check_increasing(const double *b, int n, const char *name) {
    if (!b) return fail(TSP_E_INVALID, std::string(name) + " is NULL");
    for (int i = 0; i <= n; i++)
        if (!std::isfinite(b[i])) return fail(TSP_E_INVALID, std::string(name) + " not finite");
    for (int i = 0; i < n; i++)
        if (!(b[i + 1] > b[i]))
            return fail(TSP_E_INVALID, std::string(name) + " not strictly increasing");
    return TSP_OK;
}

int bits_for(int64_t v) {  // bits needed to hold values 0..v-1
    int b = 0;
    while (b < 62 && ((int64_t)1 << b) < v) b++;
    return b < 1 ? 1 : b;
}

tsp_status sync_stream(hipStream_t st) {
    TSP_HIP(hipStreamSynchronize(st));
    return TSP_OK;
}

}  // namespace

namespace {

// The timing events set for g's next call, cleared (see tsp_set_timing_events).
KernelEvents take_timing(const tsp_geometry *g) {
    std::lock_guard<std::mutex> lk(g->timing_mu);
    const KernelEvents ke = g->timing;
    g->timing = KernelEvents();
    return ke;
}

// Runs f (a sequence of launches on st) between the records of ke's events,
// when ke holds any.
template <class F> hipError_t bracketed(const KernelEvents *ke, hipStream_t st, F f) {
    hipError_t e = (ke && ke->start) ? hipEventRecord(ke->start, st) : hipSuccess;
    if (e == hipSuccess) e = f();
    if (e == hipSuccess && ke && ke->stop) e = hipEventRecord(ke->stop, st);
    return e;
}

// y = F rho on a traced geometry (either mode); ke: events around the main
// kernel (the stored gather-sum) or, on the fly, the whole launch.
hipError_t forward_dispatch(const tsp_geometry *g, const float *rho, int batch, float *y,
                            hipStream_t st, const KernelEvents *ke = nullptr) {
    if (g->mode == TSP_MODE_CSR)
        return launch_forward_sell(g->rd, g->d_perm, g->d_cnt_sorted, g->d_slice_ptr,
                                   g->d_slice_len, g->d_code, g->d_len, rho, batch, g->V,
                                   g->T.na, g->T.ne * g->T.na, y, st, ke);
    return bracketed(ke, st, [&] {
        return launch_otf_forward(g->T, g->d_tab, g->rd, rho, batch, g->V, y, st);
    });
}

// x = F^T y; TSP_ADJ_DETERMINISTIC needs the transposed store (checked by
// callers).  ke: events around the voxel-major sum of the deterministic
// adjoint, or around the whole operation on the atomic paths.
hipError_t adjoint_dispatch(const tsp_geometry *g, const float *y, int batch, float *x,
                            int method, hipStream_t st, const KernelEvents *ke = nullptr) {
    if (method == TSP_ADJ_DETERMINISTIC)
        return launch_adjoint_csc(g->rd, g->d_col_ptr, g->d_col_code, g->d_col_len, g->T.nr,
                                  g->T.ne, g->T.na, y, batch, x, nullptr, st, ke);
    return bracketed(ke, st, [&] {
        hipError_t e = launch_zero_f32(x, (int64_t)batch * g->FV(), st);
        if (e != hipSuccess) return e;
        if (g->mode == TSP_MODE_CSR)
            return launch_adjoint_atomic(g->rd, g->d_perm, g->d_cnt_sorted, g->d_slice_ptr,
                                         g->d_slice_len, g->d_code, g->d_len, y, batch, g->V,
                                         g->T.na, g->T.ne * g->T.na, x, st);
        return launch_otf_adjoint(g->T, g->d_tab, g->rd, y, batch, g->V, x, st);
    });
}

// Device address of `scratch` on device `dev` (the current device), looked
// up once per device and kept: each device holds its own copy of the array
// at its own address.
constexpr int kMaxDevices = 256;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

tsp_status scratch_of_device(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(TSP_E_INVALID, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(TSP_E_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                       hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return TSP_OK;
}

// Checks shared by the attenuated forward and backward (Sec. 9.3).
tsp_status atten_check(const tsp_geometry *g, const tsp_geometry *gs, int32_t batch) {
    if (!g || !gs) return fail(TSP_E_INVALID, "geometry is NULL");
    if (batch < 1) return fail(TSP_E_INVALID, "batch < 1");
    if (g->mode == 0 || gs->mode == 0)
        return fail(TSP_E_STATE, "attenuated model before tsp_trace");
    if (g->mode != TSP_MODE_CSR)
        return fail(TSP_E_UNSUPPORTED, "attenuated model needs the line-of-sight geometry in "
                                       "TSP_MODE_CSR");
    if (g->rd.n_obj_frames != 1 || gs->rd.n_obj_frames != 1)
        return fail(TSP_E_UNSUPPORTED, "attenuated model with object frames");
    if (gs->R != g->V || gs->V != g->V || gs->device != g->device)
        return fail(TSP_E_INVALID, "sunward geometry must have one ray per voxel of the same "
                                   "grid, on the same device");
    return TSP_OK;
}

// Stream-ordered temporaries of n floats each, released together.
struct AsyncBufs {
    hipStream_t st;
    std::vector<void *> ps;
    explicit AsyncBufs(hipStream_t s) : st(s) {}
    float *get(int64_t n, hipError_t *e) {
        void *p = nullptr;
        if (*e == hipSuccess) *e = hipMallocAsync(&p, (size_t)(n > 0 ? n : 1) * sizeof(float), st);
        if (*e != hipSuccess) return nullptr;
        ps.push_back(p);
        return (float *)p;
    }
    hipError_t release() {
        hipError_t r = hipSuccess;
        for (void *p : ps) {
            const hipError_t e = hipFreeAsync(p, st);
            if (r == hipSuccess) r = e;
        }
        ps.clear();
        return r;
    }
    ~AsyncBufs() { (void)release(); }
};

}  // namespace

namespace {
tsp_status create_geometry(const tsp_grid_desc *grid, const tsp_view *views, int32_t n_views,
                           const double *ray_starts, const double *ray_dirs, int64_t n_rays,
                           tsp_geometry **out);
}  // namespace

extern "C" {

const char *tsp_last_error(void) { return g_err.c_str(); }

tsp_status tsp_geometry_create(const tsp_grid_desc *grid, const tsp_cone_view *views,
                               int32_t n_views, const double *ray_starts, const double *ray_dirs,
                               int64_t n_rays, tsp_geometry **out) {
    g_err.clear();
    std::vector<tsp_view> vs;
    if (views) {
        if (n_views < 1) {
            if (out) *out = nullptr;
            return fail(TSP_E_INVALID, "n_views < 1");
        }
        vs.resize((size_t)n_views);
        for (int v = 0; v < n_views; v++) {
            tsp_view &t = vs[v];
            t = tsp_view{};
            t.kind = TSP_VIEW_CONE;
            t.shape[0] = views[v].shape[0];
            t.shape[1] = views[v].shape[1];
            for (int k = 0; k < 3; k++) {
                t.pos[k] = views[v].pos[k];
                t.look[k] = views[v].look[k];
                t.up[k] = views[v].up[k];
            }
            t.extent[0] = views[v].fov_deg[0];
            t.extent[1] = views[v].fov_deg[1];
        }
    }
    return create_geometry(grid, views ? vs.data() : nullptr, n_views, ray_starts, ray_dirs,
                           n_rays, out);
}

tsp_status tsp_geometry_create_views(const tsp_grid_desc *grid, const tsp_view *views,
                                     int32_t n_views, tsp_geometry **out) {
    g_err.clear();
    if (!views) {
        if (out) *out = nullptr;
        return fail(TSP_E_INVALID, "views is NULL");
    }
    return create_geometry(grid, views, n_views, nullptr, nullptr, 0, out);
}

}  // extern "C"

namespace {

tsp_status create_geometry(const tsp_grid_desc *grid, const tsp_view *views, int32_t n_views,
                           const double *ray_starts, const double *ray_dirs, int64_t n_rays,
                           tsp_geometry **out) {
    if (!out) return fail(TSP_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!grid) return fail(TSP_E_INVALID, "grid is NULL");
    const int nr = grid->nr, ne = grid->ne, na = grid->na;
    if (nr < 1 || ne < 1 || na < 1) return fail(TSP_E_INVALID, "grid shape must be >= 1");
    tsp_status s;
    if ((s = check_increasing(grid->r_b, nr, "r_b")) != TSP_OK) return s;
    if ((s = check_increasing(grid->e_b, ne, "e_b")) != TSP_OK) return s;
    if ((s = check_increasing(grid->a_b, na, "a_b")) != TSP_OK) return s;
    if (grid->r_b[0] < 0) return fail(TSP_E_INVALID, "r_b[0] < 0");
    if (grid->e_b[0] < 0 || grid->e_b[ne] > M_PI)
        return fail(TSP_E_INVALID, "e_b outside [0, pi]");
    const double span = grid->a_b[na] - grid->a_b[0];
    if (span > kTwoPi + 1e-12) return fail(TSP_E_INVALID, "a_b spans more than 2 pi");
    const int64_t V = (int64_t)nr * ne * na;
    if (V >= ((int64_t)1 << 31)) return fail(TSP_E_INVALID, "too many voxels (>= 2^31)");
    if ((int64_t)nr + ne + 3 * (int64_t)na + 5 > kMaxTabDoubles)
        return fail(TSP_E_INVALID, "grid too fine for the shared-memory boundary tables "
                                   "(nr + ne + 3 na > 5627)");
    const double Rout = grid->r_b[nr];

    const bool use_views = views != nullptr;
    if (use_views == (ray_starts != nullptr || ray_dirs != nullptr))
        return fail(TSP_E_INVALID, "give either cone views or explicit rays");
    int H = 0, W = 0;
    int64_t R = 0;
    std::vector<double> frames, starts, dirs;
    if (use_views) {
        if (n_views < 1) return fail(TSP_E_INVALID, "n_views < 1");
        H = views[0].shape[0];
        W = views[0].shape[1];
        if (H < 1 || W < 1) return fail(TSP_E_INVALID, "detector shape must be >= 1");
        R = (int64_t)n_views * H * W;
        frames.assign((size_t)n_views * 16, 0.0);
        for (int v = 0; v < n_views; v++) {
            const tsp_view &cv = views[v];
            const bool cone = cv.kind == TSP_VIEW_CONE;
            if (!cone && cv.kind != TSP_VIEW_PARALLEL)
                return fail(TSP_E_INVALID, "view kind must be TSP_VIEW_CONE or TSP_VIEW_PARALLEL");
            if (cv.shape[0] != H || cv.shape[1] != W)
                return fail(TSP_E_INVALID, "all views must share one detector shape");
            if (!finite3(cv.pos) || !finite3(cv.look) || !finite3(cv.up))
                return fail(TSP_E_INVALID, "view vectors not finite");
            for (int k = 0; k < 2; k++) {
                if (cone && !(cv.extent[k] > 0 && cv.extent[k] < 180))
                    return fail(TSP_E_INVALID, "fov must lie in (0, 180) degrees");
                if (!cone && !(cv.extent[k] > 0 && std::isfinite(cv.extent[k])))
                    return fail(TSP_E_INVALID, "parallel detector size must be positive");
            }
            const double *P = cv.pos;
            if (std::sqrt(P[0] * P[0] + P[1] * P[1] + P[2] * P[2]) <= Rout)
                return fail(TSP_E_INVALID, "detector inside the grid's outer sphere");
            double w[3] = {cv.look[0] - P[0], cv.look[1] - P[1], cv.look[2] - P[2]};
            const double wn = std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
            if (!(wn > 0)) return fail(TSP_E_INVALID, "view pos equals look");
            for (int i = 0; i < 3; i++) w[i] /= wn;
            double up[3] = {cv.up[0], cv.up[1], cv.up[2]};
            if (up[0] == 0 && up[1] == 0 && up[2] == 0) up[2] = 1.0;
            double u[3] = {w[1] * up[2] - w[2] * up[1], w[2] * up[0] - w[0] * up[2],
                           w[0] * up[1] - w[1] * up[0]};
            double un = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            if (un < 1e-12) {
                up[0] = 1;
                up[1] = 0;
                up[2] = 0;
                u[0] = w[1] * up[2] - w[2] * up[1];
                u[1] = w[2] * up[0] - w[0] * up[2];
                u[2] = w[0] * up[1] - w[1] * up[0];
                un = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            }
            for (int i = 0; i < 3; i++) u[i] /= un;
            const double vv[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2],
                                  u[0] * w[1] - u[1] * w[0]};
            double *f = frames.data() + 16 * v;
            for (int i = 0; i < 3; i++) {
                f[0 + i] = P[i];
                f[3 + i] = w[i];
                f[6 + i] = u[i];
                f[9 + i] = vv[i];
            }
            if (cone) {
                f[12] = std::tan(cv.extent[0] * M_PI / 360.0);
                f[13] = std::tan(cv.extent[1] * M_PI / 360.0);
            } else {
                // parallel: half sizes; the whole detector rectangle must lie
                // outside the outer sphere (its point closest to the origin)
                f[12] = 0.5 * cv.extent[0];
                f[13] = 0.5 * cv.extent[1];
                const double ou = -(P[0] * u[0] + P[1] * u[1] + P[2] * u[2]);
                const double ov = -(P[0] * vv[0] + P[1] * vv[1] + P[2] * vv[2]);
                const double cu = std::fmin(std::fmax(ou, -f[13]), f[13]);
                const double cv2 = std::fmin(std::fmax(ov, -f[12]), f[12]);
                double q2 = 0.0;
                for (int i = 0; i < 3; i++) {
                    const double qi = P[i] + cu * u[i] + cv2 * vv[i];
                    q2 += qi * qi;
                }
                if (!(std::sqrt(q2) > Rout))
                    return fail(TSP_E_INVALID, "parallel detector reaches into the grid's outer "
                                               "sphere");
            }
            f[14] = cone ? 0.0 : 1.0;
        }
    } else {
        if (!ray_starts || !ray_dirs) return fail(TSP_E_INVALID, "ray arrays are NULL");
        if (n_rays < 1) return fail(TSP_E_INVALID, "n_rays < 1");
        R = n_rays;
        starts.assign(ray_starts, ray_starts + 3 * n_rays);
        dirs.resize((size_t)(3 * n_rays));
        for (int64_t i = 0; i < n_rays; i++) {
            const double *x = ray_starts + 3 * i, *d = ray_dirs + 3 * i;
            if (!finite3(x) || !finite3(d)) return fail(TSP_E_INVALID, "ray not finite");
            const double dn = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            if (!(dn > 0)) return fail(TSP_E_INVALID, "zero ray direction");
            // explicit rays may start inside the grid (integral over l >= 0)
            for (int k = 0; k < 3; k++) dirs[3 * i + k] = d[k] / dn;
        }
    }
    if (R >= ((int64_t)1 << 31) - 1) return fail(TSP_E_INVALID, "too many rays (>= 2^31)");

    tsp_geometry *g = new tsp_geometry();
    if (hipGetDevice(&g->device) != hipSuccess) {
        delete g;
        return fail(TSP_E_HIP, "hipGetDevice failed (no GPU?)");
    }
    g->V = V;
    g->R = R;
    g->r_out = Rout;

    // boundary tables
    std::vector<double> tab;
    make_tables(grid->r_b, nr, grid->e_b, ne, grid->a_b, na, &g->T, &tab);
    const TabDesc &T = g->T;

    RayDesc &rd = g->rd;
    rd.R = R;
    if (use_views) {
        rd.n_views = n_views;
        rd.H = H;
        rd.W = W;
        rd.tiles_h = (H + kTile - 1) / kTile;
        rd.tiles_w = (W + kTile - 1) / kTile;
        rd.st = 1;
        for (int c : {8, 4, 2})
            if (rd.tiles_h % c == 0 && rd.tiles_w % c == 0) {
                rd.st = c;
                break;
            }
        rd.n_slots = (int64_t)n_views * rd.tiles_h * rd.tiles_w * kWindow;
        rd.explicit_rays = 0;
        rd.obj_frame = nullptr;
        rd.n_obj_frames = 1;
    } else {
        rd.explicit_rays = 1;
        rd.obj_frame = nullptr;
        rd.n_obj_frames = 1;
        rd.st = 1;
        rd.n_slots = (R + kWindow - 1) / kWindow * kWindow;
    }
    if (rd.n_slots >= ((int64_t)1 << 31)) {
        tsp_geometry_destroy(g);
        return fail(TSP_E_INVALID, "too many rays once padded to 16x16 windows (>= 2^31 slots)");
    }

    auto cleanup = [&](tsp_status st) {
        tsp_geometry_destroy(g);
        return st;
    };
    if ((s = dalloc_n(g, &g->d_tab, T.n_tab, "tables")) != TSP_OK) return cleanup(s);
    hipError_t e = hipMemcpy(g->d_tab, tab.data(), tab.size() * sizeof(double),
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) return cleanup(fail(TSP_E_HIP, hipGetErrorString(e)));
    if (use_views) {
        if ((s = dalloc_n(g, &g->d_frames, (int64_t)frames.size(), "frames")) != TSP_OK)
            return cleanup(s);
        e = hipMemcpy(g->d_frames, frames.data(), frames.size() * sizeof(double),
                      hipMemcpyHostToDevice);
        if (e != hipSuccess) return cleanup(fail(TSP_E_HIP, hipGetErrorString(e)));
        rd.frames = g->d_frames;
    } else {
        if ((s = dalloc_n(g, &g->d_starts, 3 * R, "ray starts")) != TSP_OK) return cleanup(s);
        if ((s = dalloc_n(g, &g->d_dirs, 3 * R, "ray dirs")) != TSP_OK) return cleanup(s);
        e = hipMemcpy(g->d_starts, starts.data(), starts.size() * sizeof(double),
                      hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(g->d_dirs, dirs.data(), dirs.size() * sizeof(double),
                          hipMemcpyHostToDevice);
        if (e != hipSuccess) return cleanup(fail(TSP_E_HIP, hipGetErrorString(e)));
        rd.starts = g->d_starts;
        rd.dirs = g->d_dirs;
    }
    *out = g;
    return TSP_OK;
}

// Voxel-major (transposed) store, packed: per (frame, voxel) key the
// (natural slot, length) of its segments in slot order, split into 64 lane
// runs and delta-coded (see kSlotEsc); col_ptr [FV + 1] holds the offsets of
// the keys' blocks in col_code / col_len.  The lists come from stable radix
// sorts of the segments by key over contiguous key ranges (passes), sized so
// that the temporaries (two key and two value buffers, 24 bytes per entry,
// plus the sort workspace) fit the free device memory or the cap
// TSP_MAX_DEVICE_BYTES; the environment variable TSP_TRANSPOSE_MAX_ENTRIES
// caps the entries per pass further.  A first sweep over the passes sizes
// every key's block; a single pass is then packed from its sorted buffers,
// several passes are expanded and sorted once more to be packed.  Each key's
// list is the same whatever the passes, so the store does not depend on them.
// srow [n_slots + 1]: offsets of every natural slot's segments (exclusive
// scan of the canonical segment counts in natural slot order).
tsp_status build_transpose(tsp_geometry *g, const int64_t *srow, hipStream_t st) {
    const int64_t S = g->S, FV = g->FV(), NS = g->rd.n_slots;
    const int nr = g->T.nr, ne = g->T.ne, na = g->T.na;
    const RayDesc &rd = g->rd;
    tsp_status s;
    hipError_t e = hipSuccess;
    if ((s = dalloc_n(g, &g->d_col_ptr, FV + 1, "column offsets")) != TSP_OK) return s;

    int32_t *k1 = nullptr, *k2 = nullptr, *cnt = nullptr, *m = nullptr;
    uint64_t *v1 = nullptr, *v2 = nullptr;
    int64_t *crow = nullptr, *stmp = nullptr, *cptr = nullptr;
    void *ws = nullptr;
    auto free_pass_bufs = [&]() {
        dfree_p(g, k1);
        dfree_p(g, k2);
        dfree_p(g, v1);
        dfree_p(g, v2);
        dfree(g, ws);
        ws = nullptr;
    };
    auto free_all = [&]() {
        free_pass_bufs();
        dfree_p(g, cnt);
        dfree_p(g, m);
        dfree_p(g, crow);
        dfree_p(g, stmp);
        dfree_p(g, cptr);
    };
    auto hip_fail = [&](const char *what) {
        const std::string msg = std::string("transpose: ") + what + ": " + hipGetErrorString(e);
        free_all();
        return fail(TSP_E_HIP, msg);
    };
    if ((s = dalloc_n(g, &cnt, NS, "transpose counts")) != TSP_OK ||
        (s = dalloc_n(g, &crow, NS + 1, "transpose offsets")) != TSP_OK ||
        (s = dalloc_n(g, &stmp, scan_tmp_elems(std::max(NS, FV)), "scan")) != TSP_OK ||
        (s = dalloc_n(g, &m, FV, "row counts")) != TSP_OK ||
        (s = dalloc_n(g, &cptr, FV + 1, "pass column offsets")) != TSP_OK) {
        free_all();
        return s;
    }

    // entries per pass that the free memory (and the caps) allow, keeping
    // `reserve` bytes aside
    auto pass_cap = [&](int64_t reserve) -> int64_t {
        int64_t cap = S;
        const int64_t usable = usable_bytes(g);
        if (usable >= 0) {
            int64_t avail = usable - 4096 - reserve;
            const int64_t dcap = device_cap();
            if (dcap > 0) avail = std::min<int64_t>(avail, dcap - g->bytes - 4096 - reserve);
            cap = std::min<int64_t>(cap, avail / 25);
        }
        if (const char *ev = std::getenv("TSP_TRANSPOSE_MAX_ENTRIES")) {
            const long long v = std::atoll(ev);
            if (v > 0) cap = std::min<int64_t>(cap, v);
        }
        return cap;
    };
    // key ranges [cuts[p], cuts[p+1]) of at most cap entries each, from a
    // coarse key histogram taken once; TSP_E_NOMEM (not reported) when one
    // bucket of the histogram holds more than cap entries
    const int shift = std::max(0, bits_for(FV) - 12);
    const int nbk = (int)((FV - 1) >> shift) + 1;
    std::vector<unsigned long long> h;
    auto plan = [&](int64_t cap, std::vector<int64_t> &cuts) -> tsp_status {
        cuts.assign(1, 0);
        if (cap < 1 && S > 0) return TSP_E_NOMEM;
        if (cap < S) {
            if (h.empty()) {
                unsigned long long *hist = nullptr;
                tsp_status t;
                if ((t = dalloc_n(g, &hist, nbk, "key histogram")) != TSP_OK) return t;
                e = launch_zero_f32((float *)hist, 2 * (int64_t)nbk, st);
                if (e == hipSuccess)
                    e = launch_key_hist(rd, g->d_perm, g->d_cnt_sorted, g->d_slice_ptr,
                                        g->d_code, g->d_len, nr, ne, na, shift, nbk, hist, st);
                h.resize((size_t)nbk);
                if (e == hipSuccess) e = hipStreamSynchronize(st);
                if (e == hipSuccess)
                    e = hipMemcpy(h.data(), hist, sizeof(unsigned long long) * nbk,
                                  hipMemcpyDeviceToHost);
                dfree(g, hist);
                if (e != hipSuccess) {
                    h.clear();
                    return fail(TSP_E_HIP, std::string("key histogram: ") + hipGetErrorString(e));
                }
            }
            int64_t acc = 0;
            for (int b = 0; b < nbk; b++) {
                if ((int64_t)h[b] > cap) return TSP_E_NOMEM;
                if (acc + (int64_t)h[b] > cap && acc > 0) {
                    cuts.push_back((int64_t)b << shift);
                    acc = 0;
                }
                acc += (int64_t)h[b];
            }
        }
        cuts.push_back(FV);
        return TSP_OK;
    };
    // temporaries for passes of at most n entries
    int64_t nmax = 0;
    auto alloc_pass_bufs = [&](int64_t n) -> tsp_status {
        nmax = n;
        tsp_status t;
        if ((t = dalloc_n(g, &k1, n, "transpose keys")) != TSP_OK ||
            (t = dalloc_n(g, &k2, n, "transpose keys")) != TSP_OK ||
            (t = dalloc_n(g, &v1, n, "transpose values")) != TSP_OK ||
            (t = dalloc_n(g, &v2, n, "transpose values")) != TSP_OK ||
            (t = dalloc(g, &ws, (int64_t)radix_ws_bytes(n), "sort workspace")) != TSP_OK)
            return t;
        return TSP_OK;
    };
    // one pass: the segments with keys in [lo, hi) sorted by key into `vals`,
    // each key's list at cptr[key] .. cptr[key + 1] (relative to the pass)
    const int bits = bits_for(FV);
    auto run_pass = [&](int32_t lo, int32_t hi, bool whole, int64_t &np,
                        const uint64_t *&vals) -> tsp_status {
        // a pass over every key takes every segment: srow lays it out
        const int64_t *rows = whole ? srow : crow;
        np = S;
        if (!whole) {
            e = launch_zero_f32((float *)cnt, NS, st);
            if (e == hipSuccess)
                e = launch_count_range(rd, g->d_perm, g->d_cnt_sorted, g->d_slice_ptr, g->d_code,
                                       g->d_len, nr, ne, na, lo, hi, cnt, st);
            if (e == hipSuccess) e = launch_scan_i32(cnt, NS, 1, crow, stmp, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(&np, crow + NS, sizeof(int64_t), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) return fail(TSP_E_HIP, hipGetErrorString(e));
        }
        if (np > nmax) return fail(TSP_E_HIP, "transpose: pass larger than planned");
        int in_second = 0;
        e = launch_expand_range(rd, g->d_perm, g->d_cnt_sorted, g->d_slice_ptr, g->d_code,
                                g->d_len, rows, nr, ne, na, lo, hi, k1, v1, st);
        if (e == hipSuccess) e = launch_radix_sort(k1, v1, k2, v2, np, bits, ws, &in_second, st);
        if (e == hipSuccess)
            e = launch_col_ptr_range(in_second ? k2 : k1, np, lo, hi - lo, 0, cptr, st);
        if (e != hipSuccess) return fail(TSP_E_HIP, hipGetErrorString(e));
        vals = in_second ? v2 : v1;
        return TSP_OK;
    };
    // plan the passes and allocate their buffers, keeping `reserve` bytes free
    std::vector<int64_t> cuts;
    auto plan_passes = [&](int64_t reserve) -> tsp_status {
        const int64_t cap = pass_cap(reserve);
        tsp_status t = plan(cap, cuts);
        if (t != TSP_OK) return t;
        return alloc_pass_bufs(cuts.size() == 2 ? S : std::min<int64_t>(S, cap));
    };

    // sweep 1: the rows every key takes, then the block offsets.  The passes
    // leave room for the largest store the lists can need (each key's rows
    // hold at most twice its entries plus 63 of padding), so that a second
    // sweep can reuse them; without that room, plan for the sort alone.
    const int64_t store_bound = 5 * (2 * S + 63 * FV);
    s = plan_passes(store_bound);
    if (s == TSP_E_NOMEM) {
        free_pass_bufs();
        g_err.clear();
        s = plan_passes(0);
    }
    if (s != TSP_OK) {
        free_all();
        return s == TSP_E_NOMEM && g_err.empty()
                   ? fail(TSP_E_NOMEM, "transpose: one key bucket exceeds the memory for a pass")
                   : s;
    }
    bool whole = cuts.size() == 2;
    int64_t total = 0, np = 0;
    const uint64_t *vals = nullptr;
    for (size_t p = 0; p + 1 < cuts.size(); p++) {
        const int32_t lo = (int32_t)cuts[p], hi = (int32_t)cuts[p + 1];
        if ((s = run_pass(lo, hi, whole, np, vals)) != TSP_OK) {
            free_all();
            return s;
        }
        total += np;
        e = launch_pack_count(cptr + lo, vals, hi - lo, m + lo, st);
        if (e != hipSuccess) return hip_fail("row counts");
    }
    if (total != S) {
        free_all();
        return fail(TSP_E_HIP, "transpose: entry count mismatch");
    }
    int64_t P = 0;
    e = launch_scan_i32(m, FV, kWave, g->d_col_ptr, stmp, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&P, g->d_col_ptr + FV, sizeof(int64_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail("store offsets");

    // the packed store (5 bytes per entry), beside the pass buffers when it
    // fits there
    bool fits = false;
    {
        const int64_t usable = usable_bytes(g);
        if (usable >= 0) {
            const int64_t dcap = device_cap();
            fits = usable >= 5 * P + 4096 && (dcap <= 0 || g->bytes + 5 * P + 4096 <= dcap);
        }
    }
    if (!fits) free_pass_bufs();
    if ((s = dalloc_n(g, &g->d_col_code, P, "voxel-major codes")) != TSP_OK ||
        (s = dalloc_n(g, &g->d_col_len, P, "voxel-major lengths")) != TSP_OK) {
        free_all();
        return s;
    }
    if (whole && fits) {
        // the single pass's sorted lists are still there
        e = launch_pack_fill(cptr, vals, FV, g->d_col_ptr, g->d_col_code, g->d_col_len, st);
        if (e != hipSuccess) return hip_fail("pack");
    } else {
        // sweep 2: sort again and pack, in the same passes or, when the
        // buffers had to go, in passes that fit beside the store
        if (!fits) {
            if ((s = plan_passes(0)) != TSP_OK) {
                free_all();
                return s == TSP_E_NOMEM && g_err.empty()
                           ? fail(TSP_E_NOMEM,
                                  "transpose: one key bucket exceeds the memory for a pass")
                           : s;
            }
            whole = cuts.size() == 2;
        }
        for (size_t p = 0; p + 1 < cuts.size(); p++) {
            const int32_t lo = (int32_t)cuts[p], hi = (int32_t)cuts[p + 1];
            if ((s = run_pass(lo, hi, whole, np, vals)) != TSP_OK) {
                free_all();
                return s;
            }
            e = launch_pack_fill(cptr + lo, vals, hi - lo, g->d_col_ptr + lo, g->d_col_code,
                                 g->d_col_len, st);
            if (e != hipSuccess) return hip_fail("pack");
        }
    }
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail("pack");
    free_all();
    return TSP_OK;
}

// The work of tsp_trace on a validated geometry (the device already current).
tsp_status trace_impl(tsp_geometry *g, int base_mode, bool want_csc, hipStream_t st) {
    TSP_HIP(hipStreamSynchronize(st));
    release_stores(g);
    const RayDesc &rd = g->rd;
    const int64_t ns = rd.n_slots;
    tsp_status s;

    // pass 1: store entries and canonical segments per ray (entries only in
    // CSR mode, where they lay out the store)
    const bool csr = base_mode == TSP_MODE_CSR;
    const int64_t n_win = ns / kWindow;
    int32_t *cnt_nat = nullptr, *seg_nat = nullptr, *win_seg = nullptr;
    int64_t *counters = nullptr;  // [0] total (u64), [1] max count (int), [2] fill error (int)
    auto free_tmp = [&]() {
        dfree(g, cnt_nat);
        dfree(g, seg_nat);
        dfree(g, counters);
        dfree(g, win_seg);
        cnt_nat = seg_nat = win_seg = nullptr;
        counters = nullptr;
    };
    if ((csr && (s = dalloc_n(g, &cnt_nat, ns, "entry counts")) != TSP_OK) ||
        (csr && (s = dalloc_n(g, &seg_nat, ns, "segment counts")) != TSP_OK) ||
        (s = dalloc_n(g, &win_seg, n_win, "window segment counts")) != TSP_OK ||
        (s = dalloc_n(g, &counters, 4, "counters")) != TSP_OK) {
        free_tmp();
        return s;
    }
    hipError_t e = hipMemsetAsync(counters, 0, 4 * sizeof(int64_t), st);
    if (e == hipSuccess) e = hipMemsetAsync(win_seg, 0, n_win * sizeof(int32_t), st);
    if (e == hipSuccess)
        e = launch_count(g->T, g->d_tab, rd, cnt_nat, seg_nat, (unsigned long long *)counters,
                         (int *)(counters + 1), win_seg, st);
    int64_t host_ctr[4] = {0, 0, 0, 0};
    g->win_segs.assign(n_win, 0);
    if (e == hipSuccess)
        e = hipMemcpyAsync(host_ctr, counters, sizeof host_ctr, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->win_segs.data(), win_seg, n_win * sizeof(int32_t),
                           hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        free_tmp();
        return fail(TSP_E_HIP, std::string("trace count: ") + hipGetErrorString(e));
    }
    g->S = host_ctr[0];
    g->max_per_ray = (int64_t)(int32_t)(host_ctr[1] & 0xffffffff);

    if (base_mode == TSP_MODE_ONTHEFLY) {
        free_tmp();
        g->mode = TSP_MODE_ONTHEFLY;
        return TSP_OK;
    }

    // window ordering and slice offsets
    const int64_t n_slices = ns / kWave;
    int64_t *scan_tmp = nullptr;
    const int64_t scan_elems = scan_tmp_elems(ns > g->R + 1 ? ns : g->R + 1);
    if ((s = dalloc_n(g, &g->d_perm, ns, "perm")) != TSP_OK ||
        (s = dalloc_n(g, &g->d_cnt_sorted, ns, "sorted counts")) != TSP_OK ||
        (s = dalloc_n(g, &g->d_slice_len, n_slices, "slice lengths")) != TSP_OK ||
        (s = dalloc_n(g, &g->d_slice_ptr, n_slices + 1, "slice offsets")) != TSP_OK ||
        (s = dalloc_n(g, &scan_tmp, scan_elems, "scan scratch")) != TSP_OK) {
        free_tmp();
        dfree(g, scan_tmp);
        release_stores(g);
        return s;
    }
    auto abort_all = [&](tsp_status st2) {
        free_tmp();
        dfree(g, scan_tmp);
        release_stores(g);
        return st2;
    };
    e = launch_window_sort(rd, cnt_nat, g->d_perm, g->d_cnt_sorted, g->d_slice_len, st);
    if (e == hipSuccess)
        e = launch_scan_i32(g->d_slice_len, n_slices, kWave, g->d_slice_ptr, scan_tmp, st);
    int64_t n_stored = 0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&n_stored, g->d_slice_ptr + n_slices, sizeof(int64_t),
                           hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return abort_all(fail(TSP_E_HIP, hipGetErrorString(e)));
    g->n_stored = n_stored;

    // pass 2: fill the sliced ray-major store
    if ((s = dalloc_n(g, &g->d_code, n_stored, "entry codes")) != TSP_OK) return abort_all(s);
    if ((s = dalloc_n(g, &g->d_len, n_stored, "segment lengths")) != TSP_OK) return abort_all(s);
    e = launch_fill(g->T, g->d_tab, rd, g->d_perm, g->d_cnt_sorted, g->d_slice_ptr,
                    g->d_slice_len, g->d_code, g->d_len, (int *)(counters + 2), st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(host_ctr, counters, sizeof host_ctr, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return abort_all(fail(TSP_E_HIP, hipGetErrorString(e)));
    if ((int32_t)(host_ctr[2] & 0xffffffff) != 0)
        return abort_all(fail(TSP_E_HIP, "internal: fill pass disagreed with count pass"));

    // canonical row offsets (ray order)
    int32_t *cnt_ray = nullptr;
    if ((s = dalloc_n(g, &cnt_ray, g->R, "ray counts")) != TSP_OK) return abort_all(s);
    if ((s = dalloc_n(g, &g->d_row_ptr, g->R + 1, "row offsets")) != TSP_OK) {
        dfree(g, cnt_ray);
        return abort_all(s);
    }
    e = launch_scatter_nat(rd, seg_nat, cnt_ray, st);
    if (e == hipSuccess) e = launch_scan_i32(cnt_ray, g->R, 1, g->d_row_ptr, scan_tmp, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    dfree(g, cnt_ray);
    if (e != hipSuccess) return abort_all(fail(TSP_E_HIP, hipGetErrorString(e)));

    if (want_csc) {
        // segment offsets in natural slot order, for the transpose
        int64_t *srow = nullptr;
        if ((s = dalloc_n(g, &srow, ns + 1, "slot offsets")) != TSP_OK) return abort_all(s);
        e = launch_scan_i32(seg_nat, ns, 1, srow, scan_tmp, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        free_tmp();
        dfree(g, scan_tmp);
        scan_tmp = nullptr;
        if (e != hipSuccess) {
            dfree(g, srow);
            return abort_all(fail(TSP_E_HIP, hipGetErrorString(e)));
        }
        s = build_transpose(g, srow, st);
        dfree(g, srow);
        if (s != TSP_OK) {
            release_stores(g);
            return s;
        }
    } else {
        free_tmp();
        dfree(g, scan_tmp);
        scan_tmp = nullptr;
    }
    g->mode = TSP_MODE_CSR;
    return TSP_OK;
}

// Segments per chunk of the deterministic adjoint without a stored
// transposed list; the environment variable TSP_CHUNK_SEGMENTS overrides it.
constexpr int64_t kChunkSegments = (int64_t)1 << 30;

int64_t chunk_segments() {
    if (const char *e = std::getenv("TSP_CHUNK_SEGMENTS")) {
        const long long v = std::atoll(e);
        if (v > 0) return v;
    }
    return kChunkSegments;
}

// Deterministic adjoint of a geometry without a stored transposed list (on
// the fly, or stored lists traced without it).  The views (explicit rays: runs
// of whole windows of 256 rays) are cut into ceil(S / chunk_segments())
// chunks of about equal segment counts: a cut falls after the first view
// (window) at which the running segment count, known per window from the
// count pass, reaches a multiple of S / chunks.  The rule depends on the
// geometry alone.  Each chunk is traced into stores of its own (ray-major,
// then voxel-major, packed), its deterministic adjoint computed, and the
// chunks' results added into x in chunk order.  So x is bitwise
// reproducible for a given geometry and setting, and with one chunk it
// equals the stored deterministic adjoint.  Memory: the stores of one chunk
// at a time, in an arena the geometry keeps.  Calls on one geometry are
// serialised (they share the arena).  Synchronises the stream.
tsp_status chunked_adjoint(const tsp_geometry *g, const float *y, int B, float *x,
                           hipStream_t st) {
    std::lock_guard<std::mutex> lock(g->chunk_mu);
    const RayDesc &rd = g->rd;
    const int64_t FV = g->FV(), R = g->R, S = g->S;
    const int64_t lim = chunk_segments();
    const int64_t nch = S > lim ? (S + lim - 1) / lim : 1;
    // units that a chunk holds whole: cone views, or windows of explicit rays
    const int64_t n_win = (int64_t)g->win_segs.size();
    const int64_t wpu = rd.explicit_rays ? 1 : (int64_t)rd.tiles_h * rd.tiles_w;
    const int64_t n_units = rd.explicit_rays ? n_win : rd.n_views;
    if (n_units * wpu != n_win) return fail(TSP_E_STATE, "chunked adjoint: no window counts");
    std::vector<int64_t> ucut{0}, cseg;
    int64_t acc = 0, prev = 0, next = 1;
    for (int64_t u = 0; u < n_units; u++) {
        for (int64_t k = 0; k < wpu; k++) acc += g->win_segs[u * wpu + k];
        bool passed = false;
        while (next < nch && acc * nch >= next * S) {
            next++;
            passed = true;
        }
        if (passed && u + 1 < n_units) {
            ucut.push_back(u + 1);
            cseg.push_back(acc - prev);
            prev = acc;
        }
    }
    ucut.push_back(n_units);
    cseg.push_back(acc - prev);
    std::vector<int64_t> cut;  // chunk boundaries in rays
    for (int64_t u : ucut)
        cut.push_back(rd.explicit_rays ? std::min<int64_t>(u * kWindow, R)
                                       : u * (int64_t)rd.H * rd.W);
    int64_t rmax = 0, smax = 0;
    for (size_t c = 0; c + 1 < cut.size(); c++) {
        rmax = std::max(rmax, cut[c + 1] - cut[c]);
        smax = std::max(smax, cseg[c]);
    }

    // the chunks' working memory, allocated once and kept for later calls:
    // both stores (about 10.5 bytes per segment), one transpose pass over the
    // whole chunk (25), the trace's per-slot arrays and the block offsets,
    // for the largest chunk with half again as many segments of room (the
    // stores' padding and the sort's workspace; with less room the transpose
    // of a large chunk falls back to several passes, 40% slower at Large)
    if (!g->chunk_arena) {
        int64_t ns_max = 0;
        for (size_t c = 0; c + 1 < ucut.size(); c++)
            ns_max = std::max<int64_t>(ns_max, (ucut[c + 1] - ucut[c]) * wpu * kWindow);
        const int64_t sc = smax * 3 / 2 + 4096;
        int64_t want = sc * 37 + ns_max * 48 + FV * 40 + ((int64_t)64 << 20);
        const int64_t dcap = device_cap();
        if (dcap > 0) want = std::min<int64_t>(want, dcap - g->bytes);
        void *mem = nullptr;
        if (want <= 0 || hipMalloc(&mem, (size_t)want) != hipSuccess) {
            (void)hipGetLastError();
            char buf[160];
            std::snprintf(buf, sizeof buf, "chunked adjoint: %lld bytes of working memory",
                          (long long)want);
            return fail(TSP_E_NOMEM, buf);
        }
        g->chunk_arena = (char *)mem;
        g->chunk_arena_size = want;
    }
    float *ybuf = nullptr, *xbuf = nullptr;
    hipError_t e = hipMallocAsync((void **)&ybuf, (size_t)std::max<int64_t>(1, B * rmax) * 4, st);
    if (e == hipSuccess && cut.size() > 2)
        e = hipMallocAsync((void **)&xbuf, (size_t)B * FV * 4, st);
    auto free_bufs = [&]() {
        if (ybuf) (void)hipFreeAsync(ybuf, st);
        if (xbuf) (void)hipFreeAsync(xbuf, st);
        (void)hipStreamSynchronize(st);
    };
    if (e != hipSuccess) {
        free_bufs();
        return fail(TSP_E_NOMEM, std::string("chunked adjoint buffers: ") + hipGetErrorString(e));
    }
    for (size_t c = 0; c + 1 < cut.size(); c++) {
        const int64_t r0 = cut[c], rc = cut[c + 1] - r0;
        // a geometry of the chunk's rays that shares g's tables and frames
        tsp_geometry *gc = new tsp_geometry();
        gc->device = g->device;
        gc->T = g->T;
        gc->d_tab = g->d_tab;
        gc->V = g->V;
        gc->R = rc;
        gc->rd = rd;
        gc->rd.R = rc;
        gc->bytes = g->bytes;  // the device cap counts the parent's memory too
        gc->arena = g->chunk_arena;
        gc->arena_size = g->chunk_arena_size;
        if (!rd.explicit_rays) {
            const int64_t v0 = r0 / ((int64_t)rd.H * rd.W);
            const int nvc = (int)(rc / ((int64_t)rd.H * rd.W));
            gc->rd.n_views = nvc;
            gc->rd.frames = rd.frames + 16 * v0;
            gc->rd.obj_frame = rd.obj_frame ? rd.obj_frame + v0 : nullptr;
            gc->rd.n_slots = (int64_t)nvc * rd.tiles_h * rd.tiles_w * kWindow;
        } else {
            gc->rd.starts = rd.starts + 3 * r0;
            gc->rd.dirs = rd.dirs + 3 * r0;
            gc->rd.n_slots = (rc + kWindow - 1) / kWindow * kWindow;
        }
        tsp_status s = trace_impl(gc, TSP_MODE_CSR, true, st);
        if (s == TSP_OK) {
            float *xo = (c == 0) ? x : xbuf;
            e = launch_copy_rows(y + r0, R, ybuf, rc, B, st);
            if (e == hipSuccess) e = adjoint_dispatch(gc, ybuf, B, xo, TSP_ADJ_DETERMINISTIC, st);
            if (e == hipSuccess && c > 0) e = launch_add_f32(xbuf, x, (int64_t)B * FV, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess)
                s = fail(TSP_E_HIP, std::string("chunked adjoint: ") + hipGetErrorString(e));
        }
        (void)hipStreamSynchronize(st);  // the chunk's work is done before its memory is reused
        delete gc;
        if (s != TSP_OK) {
            free_bufs();
            return s;
        }
    }
    free_bufs();
    return TSP_OK;
}

}  // namespace

extern "C" {

void tsp_geometry_destroy(tsp_geometry *g) {
    if (!g) return;
    DeviceGuard dg(g->device);
    (void)hipDeviceSynchronize();
    for (auto &a : g->allocs) (void)hipFree(a.first);
    g->allocs.clear();
    release_chunk_arena(g);
    delete g;
}

tsp_status tsp_set_object_frames(tsp_geometry *g, const int32_t *frame_of_view,
                                 int32_t n_frames) {
    g_err.clear();
    if (!g) return fail(TSP_E_INVALID, "geometry is NULL");
    if (g->mode != 0) return fail(TSP_E_STATE, "object frames must be set before tsp_trace");
    if (g->rd.explicit_rays)
        return fail(TSP_E_UNSUPPORTED, "object frames need cone views (explicit rays given)");
    if (!frame_of_view) return fail(TSP_E_INVALID, "frame_of_view is NULL");
    if (n_frames < 1) return fail(TSP_E_INVALID, "n_frames < 1");
    if (g->V * (int64_t)n_frames >= ((int64_t)1 << 31))
        return fail(TSP_E_INVALID, "n_frames * voxels >= 2^31");
    const int nv = g->rd.n_views;
    for (int v = 0; v < nv; v++)
        if (frame_of_view[v] < 0 || frame_of_view[v] >= n_frames) {
            char buf[128];
            std::snprintf(buf, sizeof buf, "frame_of_view[%d] = %d outside [0, %d)", v,
                          (int)frame_of_view[v], (int)n_frames);
            return fail(TSP_E_INVALID, buf);
        }
    DeviceGuard dg(g->device);
    if (!dg.ok) return fail(TSP_E_HIP, "hipSetDevice failed");
    if (g->d_obj_frame) dfree_p(g, g->d_obj_frame);
    g->rd.obj_frame = nullptr;
    g->rd.n_obj_frames = 1;
    tsp_status s;
    if ((s = dalloc_n(g, &g->d_obj_frame, nv, "object frames")) != TSP_OK) return s;
    if (hipMemcpy(g->d_obj_frame, frame_of_view, sizeof(int32_t) * nv, hipMemcpyHostToDevice) !=
        hipSuccess) {
        dfree_p(g, g->d_obj_frame);
        return fail(TSP_E_HIP, "hipMemcpy of object frames failed");
    }
    g->rd.obj_frame = g->d_obj_frame;
    g->rd.n_obj_frames = n_frames;
    return TSP_OK;
}

tsp_status tsp_trace(tsp_geometry *g, int32_t mode, void *stream) {
    g_err.clear();
    if (!g) return fail(TSP_E_INVALID, "geometry is NULL");
    const int base_mode = mode & 0x0f;
    const bool want_csc = (mode & TSP_TRACE_NO_CSC) == 0;
    if (base_mode != TSP_MODE_CSR && base_mode != TSP_MODE_ONTHEFLY)
        return fail(TSP_E_INVALID, "mode must be TSP_MODE_CSR or TSP_MODE_ONTHEFLY");
    DeviceGuard dg(g->device);
    if (!dg.ok) return fail(TSP_E_HIP, "hipSetDevice failed");
    hipStream_t st = (hipStream_t)stream;
    return trace_impl(g, base_mode, want_csc, st);
}

tsp_status tsp_forward(const tsp_geometry *g, const float *rho, int32_t batch, float *y,
                       void *stream) {
    g_err.clear();
    if (!g) return fail(TSP_E_INVALID, "geometry is NULL");
    if (!rho || !y) return fail(TSP_E_INVALID, "rho or y is NULL");
    if (batch < 1) return fail(TSP_E_INVALID, "batch < 1");
    if (g->mode == 0) return fail(TSP_E_STATE, "tsp_forward before tsp_trace");
    DeviceGuard dg(g->device);
    const KernelEvents ke = take_timing(g);
    const hipError_t e = forward_dispatch(g, rho, batch, y, (hipStream_t)stream, &ke);
    if (e != hipSuccess) return fail(TSP_E_HIP, std::string("forward: ") + hipGetErrorString(e));
    return TSP_OK;
}

tsp_status tsp_backproject(const tsp_geometry *g, const float *y, int32_t batch, float *x,
                           int32_t method, void *stream) {
    g_err.clear();
    if (!g) return fail(TSP_E_INVALID, "geometry is NULL");
    if (!x || !y) return fail(TSP_E_INVALID, "y or x is NULL");
    if (batch < 1) return fail(TSP_E_INVALID, "batch < 1");
    if (method != TSP_ADJ_DETERMINISTIC && method != TSP_ADJ_ATOMIC &&
        method != TSP_ADJ_FIXEDPOINT)
        return fail(TSP_E_INVALID,
                    "method must be TSP_ADJ_DETERMINISTIC, TSP_ADJ_ATOMIC or TSP_ADJ_FIXEDPOINT");
    if (g->mode == 0) return fail(TSP_E_STATE, "tsp_backproject before tsp_trace");
    DeviceGuard dg(g->device);
    const KernelEvents ke = take_timing(g);
    hipStream_t st = (hipStream_t)stream;
    if (method == TSP_ADJ_FIXEDPOINT) {
        const hipError_t e = bracketed(&ke, st, [&] {
            return launch_otf_adjoint_fixed(g->T, g->d_tab, g->rd, y, batch, g->V, g->r_out, x,
                                            st);
        });
        if (e != hipSuccess)
            return fail(e == hipErrorOutOfMemory ? TSP_E_NOMEM : TSP_E_HIP,
                        std::string("adjoint: ") + hipGetErrorString(e));
        return TSP_OK;
    }
    if (method == TSP_ADJ_DETERMINISTIC && (g->mode != TSP_MODE_CSR || !g->d_col_ptr)) {
        if (ke.start && hipEventRecord(ke.start, st) != hipSuccess)
            return fail(TSP_E_HIP, "adjoint: recording the start event failed");
        const tsp_status s = chunked_adjoint(g, y, batch, x, st);
        if (s == TSP_OK && ke.stop && hipEventRecord(ke.stop, st) != hipSuccess)
            return fail(TSP_E_HIP, "adjoint: recording the stop event failed");
        return s;
    }
    const hipError_t e = adjoint_dispatch(g, y, batch, x, method, st, &ke);
    if (e != hipSuccess) return fail(TSP_E_HIP, std::string("adjoint: ") + hipGetErrorString(e));
    return TSP_OK;
}

tsp_status tsp_set_timing_events(tsp_geometry *g, void *start, void *stop) {
    g_err.clear();
    if (!g) return fail(TSP_E_INVALID, "geometry is NULL");
    if ((start == nullptr) != (stop == nullptr))
        return fail(TSP_E_INVALID, "start and stop must both be set or both be NULL");
    std::lock_guard<std::mutex> lk(g->timing_mu);
    g->timing.start = (hipEvent_t)start;
    g->timing.stop = (hipEvent_t)stop;
    return TSP_OK;
}

tsp_status tsp_backproject_noalloc(const tsp_geometry *g, const float *y, int32_t batch,
                                   float *x, void *stream) {
    g_err.clear();
    if (!g) return fail(TSP_E_INVALID, "geometry is NULL");
    if (!x || !y) return fail(TSP_E_INVALID, "y or x is NULL");
    if (batch < 1) return fail(TSP_E_INVALID, "batch < 1");
    if (g->mode == 0) return fail(TSP_E_STATE, "tsp_backproject_noalloc before tsp_trace");
    if (g->mode != TSP_MODE_CSR || !g->d_col_ptr)
        return fail(TSP_E_STATE, "tsp_backproject_noalloc needs the voxel-major store "
                                 "(TSP_MODE_CSR without TSP_TRACE_NO_CSC)");
    const size_t need = adjoint_csc_ws_bytes(g->rd, batch);
    if (need > (size_t)TSP_NOALLOC_SCRATCH_BYTES) {
        char buf[200];
        std::snprintf(buf, sizeof buf,
                      "tsp_backproject_noalloc: the slot-ordered copy of y needs %llu bytes, "
                      "more than the fixed workspace of %llu bytes",
                      (unsigned long long)need, (unsigned long long)TSP_NOALLOC_SCRATCH_BYTES);
        return fail(TSP_E_NOMEM, buf);
    }
    DeviceGuard dg(g->device);
    if (!dg.ok) return fail(TSP_E_HIP, "hipSetDevice failed");
    void *ws = nullptr;
    const tsp_status s = scratch_of_device(g->device, &ws);
    if (s != TSP_OK) return s;
    const hipError_t e =
        launch_adjoint_csc(g->rd, g->d_col_ptr, g->d_col_code, g->d_col_len, g->T.nr, g->T.ne,
                           g->T.na, y, batch, x, ws, (hipStream_t)stream);
    if (e != hipSuccess) return fail(TSP_E_HIP, std::string("adjoint: ") + hipGetErrorString(e));
    return TSP_OK;
}

tsp_status tsp_geometry_create_sunward(const tsp_grid_desc *grid, const double *sun_dir,
                                       tsp_geometry **out) {
    g_err.clear();
    if (!out) return fail(TSP_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!grid || !grid->r_b || !grid->e_b || !grid->a_b || !sun_dir)
        return fail(TSP_E_INVALID, "grid or sun_dir is NULL");
    if (grid->nr < 1 || grid->ne < 1 || grid->na < 1)
        return fail(TSP_E_INVALID, "grid shape must be >= 1");
    if (!finite3(sun_dir)) return fail(TSP_E_INVALID, "sun_dir not finite");
    const double dn = std::sqrt(sun_dir[0] * sun_dir[0] + sun_dir[1] * sun_dir[1] +
                                sun_dir[2] * sun_dir[2]);
    if (!(dn > 0)) return fail(TSP_E_INVALID, "zero sun_dir");
    const int nr = grid->nr, ne = grid->ne, na = grid->na;
    const int64_t V = (int64_t)nr * ne * na;
    if (V >= ((int64_t)1 << 31)) return fail(TSP_E_INVALID, "too many voxels (>= 2^31)");
    // centroids at the mid-boundaries (r_c, theta_c, phi_c), voxel order (ir, ie, ia)
    std::vector<double> starts((size_t)(3 * V)), dirs((size_t)(3 * V));
    for (int ir = 0; ir < nr; ir++) {
        const double rc = 0.5 * (grid->r_b[ir] + grid->r_b[ir + 1]);
        for (int ie = 0; ie < ne; ie++) {
            const double tc = 0.5 * (grid->e_b[ie] + grid->e_b[ie + 1]);
            for (int ia = 0; ia < na; ia++) {
                const double pc = 0.5 * (grid->a_b[ia] + grid->a_b[ia + 1]);
                const int64_t v = ((int64_t)ir * ne + ie) * na + ia;
                starts[3 * v + 0] = rc * std::sin(tc) * std::cos(pc);
                starts[3 * v + 1] = rc * std::sin(tc) * std::sin(pc);
                starts[3 * v + 2] = rc * std::cos(tc);
                for (int k = 0; k < 3; k++) dirs[3 * v + k] = sun_dir[k] / dn;
            }
        }
    }
    return tsp_geometry_create(grid, nullptr, 0, starts.data(), dirs.data(), V, out);
}

tsp_status tsp_atten_forward(const tsp_geometry *g, const tsp_geometry *g_sun, const float *rho,
                             const float *sigma, int32_t batch, float *y, float *tau1,
                             void *stream) {
    g_err.clear();
    tsp_status s;
    if ((s = atten_check(g, g_sun, batch)) != TSP_OK) return s;
    if (!rho || !sigma || !y) return fail(TSP_E_INVALID, "rho, sigma or y is NULL");
    DeviceGuard dg(g->device);
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = g->V * batch;
    hipError_t e = hipSuccess;
    AsyncBufs tmp(st);
    float *sv = tmp.get(n, &e);
    float *t1 = tau1 ? tau1 : tmp.get(n, &e);
    float *w = tmp.get(n, &e);
    if (e == hipSuccess) e = launch_atten_s(sigma, rho, g->V, batch, sv, st);
    if (e == hipSuccess) e = forward_dispatch(g_sun, sv, batch, t1, st);  // tau_1 = F_1 s
    if (e == hipSuccess) e = launch_atten_w(t1, rho, n, w, st);
    if (e == hipSuccess)
        e = launch_fwd_atten(g->rd, g->d_perm, g->d_cnt_sorted, g->d_slice_ptr, g->d_slice_len,
                             g->d_code, g->d_len, sv, w, batch, g->V, g->T.na,
                             g->T.ne * g->T.na, y, st);
    const hipError_t r = tmp.release();
    if (e == hipSuccess) e = r;
    if (e != hipSuccess)
        return fail(TSP_E_HIP, std::string("attenuated forward: ") + hipGetErrorString(e));
    return TSP_OK;
}

tsp_status tsp_atten_backward(const tsp_geometry *g, const tsp_geometry *g_sun, const float *rho,
                              const float *sigma, const float *tau1, const float *gy,
                              int32_t batch, float *grad, int32_t method, void *stream) {
    g_err.clear();
    tsp_status s;
    if ((s = atten_check(g, g_sun, batch)) != TSP_OK) return s;
    if (!rho || !sigma || !tau1 || !gy || !grad)
        return fail(TSP_E_INVALID, "rho, sigma, tau1, gy or grad is NULL");
    if (method != TSP_ADJ_DETERMINISTIC && method != TSP_ADJ_ATOMIC)
        return fail(TSP_E_INVALID, "method must be TSP_ADJ_DETERMINISTIC or TSP_ADJ_ATOMIC");
    const bool det = method == TSP_ADJ_DETERMINISTIC;
    if (det && !g_sun->d_col_ptr)
        return fail(TSP_E_STATE, "deterministic attenuated backward needs the sunward geometry "
                                 "traced with its voxel-major store");
    DeviceGuard dg(g->device);
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = g->V * batch;
    const int sun_method = g_sun->d_col_ptr ? TSP_ADJ_DETERMINISTIC : TSP_ADJ_ATOMIC;
    hipError_t e = hipSuccess;
    AsyncBufs tmp(st);
    float *sv = tmp.get(n, &e);
    float *w = tmp.get(n, &e);
    float *gw = tmp.get(n, &e);
    float *gsl = tmp.get(n, &e);
    float *gt = tmp.get(n, &e);
    float *gsun = tmp.get(n, &e);
    float *ws = det ? tmp.get((int64_t)(atten_fixed_ws_bytes(g->V) + 3) / 4, &e) : nullptr;
    if (e == hipSuccess) e = launch_atten_s(sigma, rho, g->V, batch, sv, st);
    if (e == hipSuccess) e = launch_atten_w(tau1, rho, n, w, st);
    if (e == hipSuccess && !det) e = launch_zero_f32(gw, n, st);
    if (e == hipSuccess && !det) e = launch_zero_f32(gsl, n, st);
    if (e == hipSuccess)
        e = launch_bwd_atten(g->rd, g->d_perm, g->d_cnt_sorted, g->d_slice_ptr, g->d_slice_len,
                             g->d_code, g->d_len, sv, w, gy, batch, g->V, g->T.na,
                             g->T.ne * g->T.na, g->r_out, gw, gsl, ws, st);
    if (e == hipSuccess) e = launch_atten_gtau(w, gw, n, gt, st);
    if (e == hipSuccess) e = adjoint_dispatch(g_sun, gt, batch, gsun, sun_method, st);  // F_1^T
    if (e == hipSuccess)
        e = launch_atten_grad(tau1, sigma, gw, gsl, gsun, g->V, batch, grad, st);
    const hipError_t r = tmp.release();
    if (e == hipSuccess) e = r;
    if (e != hipSuccess)
        return fail(TSP_E_HIP, std::string("attenuated backward: ") + hipGetErrorString(e));
    return TSP_OK;
}

tsp_status tsp_segments(const tsp_geometry *g, int64_t *row_ptr, int32_t *vox, float *len,
                        void *stream) {
    g_err.clear();
    if (!g) return fail(TSP_E_INVALID, "geometry is NULL");
    if (g->mode != TSP_MODE_CSR) return fail(TSP_E_STATE, "segments exist only in CSR mode");
    DeviceGuard dg(g->device);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (row_ptr) e = launch_copy_i64(g->d_row_ptr, row_ptr, g->R + 1, st);
    if (e == hipSuccess && (vox || len))
        e = launch_expand(g->rd, g->d_perm, g->d_cnt_sorted, g->d_slice_ptr, g->d_code, g->d_len,
                          g->rd.n_slots, g->d_row_ptr, g->T.na, g->T.ne * g->T.na, vox, len, st);
    if (e != hipSuccess) return fail(TSP_E_HIP, hipGetErrorString(e));
    return TSP_OK;
}

tsp_status tsp_rays(const tsp_geometry *g, double *starts, double *dirs, void *stream) {
    g_err.clear();
    if (!g) return fail(TSP_E_INVALID, "geometry is NULL");
    DeviceGuard dg(g->device);
    hipError_t e = launch_rays(g->rd, starts, dirs, (hipStream_t)stream);
    if (e != hipSuccess) return fail(TSP_E_HIP, hipGetErrorString(e));
    return TSP_OK;
}

tsp_status tsp_query(const tsp_geometry *g, tsp_info *info) {
    g_err.clear();
    if (!g || !info) return fail(TSP_E_INVALID, "NULL argument");
    info->n_rays = g->R;
    info->n_voxels = g->V;
    info->n_segments = g->S;
    info->n_stored = g->n_stored;
    info->max_per_ray = g->max_per_ray;
    info->device_bytes = g->bytes;
    info->mode = g->mode;
    info->has_csc = g->d_col_ptr != nullptr;
    info->n_obj_frames = g->rd.n_obj_frames;
    return TSP_OK;
}

}  // extern "C"
