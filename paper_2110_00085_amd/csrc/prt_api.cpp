// Host side of the C ABI declared in include/prt.h: argument validation,
// contexts, path-store lifecycle, kernel launches and telemetry.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <mutex>
#include <vector>

#include "../../include/prt.h"
#include "../../include/prt_surface.h"
#include "launch.hpp"
#include "surface.hpp"

using namespace prt;

namespace {

thread_local std::string g_err = "no error";

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                                  \
    do {                                                                                              \
        hipError_t e_ = (expr);                                                                       \
        if (e_ != hipSuccess) return fail(PRT_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));       \
    } while (0)

enum KernelId {
    K_SAMPLE = 0, K_SORT, K_PACK, K_PREP, K_RENDER, K_FINALIZE, K_GRAD, K_REWEIGHT, K_LOSS, K_ADAM,
    K_RENDER_REDUCE, K_GRAD_REDUCE, K_GRAD_WEIGHTS, K_RENDER_PREFIX, K_GRAD_BIN, K_GRAD_RECOMPUTE, K_TPP_LAYOUT,
    K_TPP_RENDER, K_TPP_GRAD, K_SURF_SAMPLE, K_SURF_TAPE, K_SURF_RENDER, K_SURF_GRAD, K_SURF_REWEIGHT,
    K_SURF_ADAM, K_COUNT
};
const char* kKernelNames[K_COUNT] = {"sample", "sort",          "pack",        "prep",         "render",
                                     "render_finalize", "grad",  "reweight",    "loss",         "adam",
                                     "render_reduce",   "grad_reduce", "grad_weights", "render_prefix",
                                     "grad_bin",        "grad_recompute", "tpp_layout",   "tpp_render",
                                     "tpp_grad",        "surf_sample", "surf_tape",    "surf_render",
                                     "surf_grad",       "surf_reweight", "surf_adam"};

struct Timed {
    int id;
    hipEvent_t a, b;
};

constexpr int kMismatchWord = 6;
constexpr int kOvfFullWord = 7;

}  // namespace

struct prt_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    int fp64 = 0;
    int n_cu = 1;               // compute units on the device (persistent launches)
    void* gpart = nullptr;      // per-workgroup gradient partials
    size_t gpart_bytes = 0;
    void* rpart = nullptr;      // per-workgroup image partials
    size_t gw_bytes = 0, gaux_bytes = 0, pb_bytes = 0;
    void* pb = nullptr;         // render prefix weights per vertex record (double)
    void* gw = nullptr;         // gradient weights per (vertex, camera), tape layout
    void* gaux = nullptr;       // per-vertex gradient sums (float4)
    // binned gradient: task slab ranges, per-slab counts (+ scan scratch), task lists
    void* bin_trange = nullptr;
    size_t bin_trange_bytes = 0;
    void* bin_cnt = nullptr;
    size_t bin_cnt_bytes = 0;
    void* bin_list = nullptr;
    size_t bin_list_bytes = 0;
    void* bin_part = nullptr;   // per-chunk slab partials
    size_t bin_part_bytes = 0;
    void* bin_rtape = nullptr;  // per-connection slab ranges (tape layout)
    size_t bin_rtape_bytes = 0;
    void* bin_brange = nullptr; // per (row of 64 records, camera group) slab ranges
    size_t bin_brange_bytes = 0;
    size_t rpart_bytes = 0;
    // sampling / sorting temporaries (grow-only)
    void* s_tmp = nullptr;
    size_t s_tmp_bytes = 0;
    void* s_ovf = nullptr;      // overflow segment counter (16 bytes), then a first segment per path id
    size_t s_ovf_bytes = 0;
    void* s_keys = nullptr;     // tB and tnv
    size_t s_keys_bytes = 0;
    void* s_hist = nullptr;
    size_t s_hist_bytes = 0;
    void* s_off = nullptr;      // import offsets
    void* s_perm = nullptr;     // permutation after the sort's first pass, then id -> slot
    size_t s_perm_bytes = 0;
    // largest one-pass sampling temporary; larger resamples take two passes
    uint64_t sample_tmp_limit = (uint64_t)40 << 30;
    size_t s_off_bytes = 0;
    // pinned host words the kernels write directly (read after a stream sync):
    // the store's meta words after packing (words 0-2 and kMetaFirstGe on),
    // the reweight's 2 sums (bytes 32-47, words 4-5 of the meta layout) and
    // the two-pass sampler's mismatch flag (word kMismatchWord)
    void* hpin = nullptr;
    int64_t* hmeta = nullptr;
    double* hsum = nullptr;
    int64_t* dmeta = nullptr;   // the same words as device pointers
    double* dsum = nullptr;
    void* grid_tot = nullptr;
    void* grid_dlt = nullptr;
    size_t grid_bytes = 0;
    void* grid_tile = nullptr;  // grid_tot in the z-tiled layout (render walks over a grid in global memory)
    size_t tile_bytes = 0;
    double* pix = nullptr;      // rho scratch
    size_t pix_n = 0;
    double* part = nullptr;     // reduction partials
    size_t part_n = 0;
    unsigned long long* counters = nullptr;  // 4
    int* flag = nullptr;        // device flag: the tape matches beta_t
    unsigned int* work = nullptr;  // task counters of the persistent kernels [kWorkWords]
    uint64_t paths_done = 0;
    uint32_t timing = 0;  // bit k set: kernel id k is timed
    std::vector<Timed> pending;
    std::vector<hipEvent_t> pool;
    double total_ms[K_COUNT] = {};
    int64_t launches[K_COUNT] = {};
};

struct prt_paths_s {
    int device = 0;
    // allocated element counts of each buffer (a refill reuses a buffer when
    // it is large enough)
    int64_t cap_perm = 0, cap_slots = 0, cap_nv = 0, cap_boff = 0, cap_records = 0, cap_nu = 0;
    uint64_t n = 0;
    int64_t nb = 0, n_slots = 0, first_slot = 0;
    // largest B, and for b = 1..bmax the batch of the first sorted slot with B >= b
    int bmax = 0;
    int32_t first_batch_ge[kMaxOrder + 1] = {};
    int32_t max_order = 0, nx = 0, ny = 0, nz = 0;
    uint64_t seed = 0;
    float4* vtx = nullptr;
    int64_t n_records = 0;
    int64_t* batch_off = nullptr;
    uint8_t* B = nullptr;
    uint8_t* nv = nullptr;
    int32_t* perm = nullptr;
    float* beta_ref = nullptr;
    uint64_t bytes = 0;
    int64_t tape_base = 0;      // batch_off of the first batch with scattering paths
    // Transmittance tape written by prt_render (FP32 traversal mode), reused by
    // prt_grad when beta_t, the cameras and the scene constants are unchanged.
    float2* tape = nullptr;
    size_t tape_cap = 0;        // entries (c, pixel)
    float* tape_beta = nullptr; // beta_t of the render that wrote the tape
    bool tape_valid = false;
    DevCams tape_cams{};
    DevScene tape_scene{};
    // per-path copies for the path-sorting ablation, one per order (built on
    // first use after each (re)fill)
    struct TppCopy {
        float4* rec = nullptr;
        int64_t* off = nullptr;
        uint8_t* B = nullptr;
        int32_t* inv = nullptr;
        int64_t cap_rec = 0, cap_n = 0;
        bool valid = false;
    } tpp[2];
};

// Reflectometry store: paths as rows per vertex order, their tape, the
// scene (spheres on the device), the cameras and theta_ref.
struct prt_surface_paths_s {
    int device = 0;
    int64_t n = 0, cap = 0;          // paths, paths the buffers hold
    int M = 0, n_cams = 0, cap_cams = 0;
    int32_t* B = nullptr;
    double4* pos = nullptr;
    int32_t* sid = nullptr;
    double2* tv = nullptr;
    double2* tc = nullptr;
    int32_t* pix = nullptr;
    double* theta_ref = nullptr;     // device [2]
    double* sph = nullptr;           // device [kMaxSpheres][kSphStride]
    double sph_host[kSphStride * kMaxSpheres] = {};  // what sph holds (n_sph of them)
    int n_sph = -1;
    double* omega = nullptr;         // reciprocal pixel solid angles [n_cams][W*H]
    int64_t cap_omega = 0;
    bool omega_valid = false;        // omega belongs to `cams`
    unsigned long long* work = nullptr;  // [2] sphere tests and vertices of the last draw
    double* part = nullptr;          // render partial images / gradient and reweight pairs
    size_t part_n = 0;
    SurfScene scene{};
    DevCams cams{};
};

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

hipEvent_t take_event(prt_ctx c)
{
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Records an event pair around the launches made while it is alive.
struct TimedScope {
    prt_ctx c;
    Timed t{};
    bool on;
    TimedScope(prt_ctx ctx, int id) : c(ctx), on(((ctx->timing >> id) & 1u) != 0)
    {
        if (!on) return;
        t.id = id;
        t.a = take_event(c);
        t.b = take_event(c);
        if (!t.a || !t.b) {
            on = false;
            return;
        }
        (void)hipEventRecord(t.a, c->stream);
    }
    ~TimedScope()
    {
        if (!on) return;
        (void)hipEventRecord(t.b, c->stream);
        c->pending.push_back(t);
    }
};

bool finite_all(std::initializer_list<double> v)
{
    for (double x : v)
        if (!std::isfinite(x)) return false;
    return true;
}

int check_scene(const prt_scene* s)
{
    if (!s) return fail(PRT_E_INVALID, "scene is NULL");
    if (s->nx < 1 || s->ny < 1 || s->nz < 1) return fail(PRT_E_INVALID, "grid dims must be >= 1");
    if ((int64_t)s->nx * s->ny * s->nz >= (int64_t)1 << 31)
        return fail(PRT_E_CAPACITY, "grid has more than 2^31 - 1 voxels");
    if (s->nx > PRT_MAX_DIM || s->ny > PRT_MAX_DIM || s->nz > PRT_MAX_DIM)
        return fail(PRT_E_CAPACITY, "grid dims must be <= %d", PRT_MAX_DIM);
    if (s->max_order < 1 || s->max_order > PRT_MAX_ORDER)
        return fail(PRT_E_CAPACITY, "max_order %d outside [1, %d]", s->max_order, PRT_MAX_ORDER);
    if (!finite_all({s->voxel_km, s->beta_air, s->albedo_cloud, s->albedo_air, s->g, s->sun_zenith_deg,
                     s->sun_azimuth_deg, s->sun_flux}))
        return fail(PRT_E_INVALID, "non-finite scene parameter");
    if (!(s->voxel_km > 0)) return fail(PRT_E_INVALID, "voxel_km must be > 0");
    if (!(s->beta_air >= 0)) return fail(PRT_E_INVALID, "beta_air must be >= 0");
    if (!(s->albedo_cloud > 0 && s->albedo_cloud <= 1) || !(s->albedo_air > 0 && s->albedo_air <= 1))
        return fail(PRT_E_INVALID, "albedos must lie in (0, 1]");
    if (!(std::fabs(s->g) < 1)) return fail(PRT_E_INVALID, "|g| must be < 1");
    if (!(s->sun_zenith_deg >= 0 && s->sun_zenith_deg < 90)) return fail(PRT_E_INVALID, "sun zenith must be in [0, 90)");
    if (!(s->sun_flux > 0)) return fail(PRT_E_INVALID, "sun_flux must be > 0");
    if (!s->beta_cloud) return fail(PRT_E_INVALID, "beta_cloud is NULL");
    return PRT_OK;
}

DevScene make_dev_scene(const prt_scene* s)
{
    DevScene d{};
    d.nx = s->nx;
    d.ny = s->ny;
    d.nz = s->nz;
    d.max_order = s->max_order;
    d.vk = s->voxel_km;
    d.beta_air = s->beta_air;
    d.w_c = s->albedo_cloud;
    d.w_a = s->albedo_air;
    d.g = s->g;
    d.hg_num = (1.0 - s->g * s->g) / (4.0 * kPi);
    const double th = s->sun_zenith_deg * kPi / 180.0, ph = s->sun_azimuth_deg * kPi / 180.0;
    d.sun[0] = std::sin(th) * std::cos(ph);
    d.sun[1] = std::sin(th) * std::sin(ph);
    d.sun[2] = -std::cos(th);
    const double Lx = s->nx * s->voxel_km, Ly = s->ny * s->voxel_km, Lz = s->nz * s->voxel_km;
    d.a_top = Lx * Ly * std::fabs(d.sun[2]);
    d.a_x = Ly * Lz * std::fabs(d.sun[0]);
    d.a_y = Lx * Lz * std::fabs(d.sun[1]);
    d.w0 = s->sun_flux * (d.a_top + d.a_x + d.a_y);
    d.x_face = d.sun[0] > 0 ? 0.0 : (double)s->nx;
    d.y_face = d.sun[1] > 0 ? 0.0 : (double)s->ny;
    d.inv_nx = 1.0 / (double)s->nx;
    d.inv_ny = 1.0 / (double)s->ny;
    d.inv_nxy = 1.0 / ((double)s->nx * (double)s->ny);
    return d;
}

int make_dev_cams(const prt_cameras* c, const prt_scene* s, DevCams* out)
{
    if (!c) return fail(PRT_E_INVALID, "cameras is NULL");
    if (c->n < 1 || c->n > PRT_MAX_CAMERAS) return fail(PRT_E_CAPACITY, "camera count %d outside [1, %d]", c->n, PRT_MAX_CAMERAS);
    if (c->width < 1 || c->height < 1 || c->width > 16384 || c->height > 16384)
        return fail(PRT_E_INVALID, "image size must be in [1, 16384]");
    if (!c->pos || !c->rot || !c->f_px) return fail(PRT_E_INVALID, "camera arrays must be non-NULL");
    std::memset(out, 0, sizeof *out);
    out->n = c->n;
    out->W = c->width;
    out->H = c->height;
    const double vk = s->voxel_km;
    out->outside = 1;
    for (int d = 0; d < c->n; ++d) {
        for (int k = 0; k < 3; ++k) {
            if (!std::isfinite(c->pos[3 * d + k])) return fail(PRT_E_INVALID, "non-finite camera position");
            out->pos[d][k] = c->pos[3 * d + k] / vk;
        }
        for (int k = 0; k < 9; ++k) {
            if (!std::isfinite(c->rot[9 * d + k])) return fail(PRT_E_INVALID, "non-finite camera rotation");
            out->rot[d][k] = c->rot[9 * d + k];
        }
        if (!(c->f_px[d] > 0) || !std::isfinite(c->f_px[d])) return fail(PRT_E_INVALID, "focal length must be > 0");
        out->f[d] = c->f_px[d];
        const double* q = out->pos[d];
        const bool out_d = q[0] < 0.0 || q[0] > s->nx || q[1] < 0.0 || q[1] > s->ny || q[2] < 0.0 || q[2] > s->nz;
        if (!out_d) out->outside = 0;
    }
    return PRT_OK;
}

// Camera groups per path task: three groups balance the persistent waves
// (a task is at most a third of a path's local estimates) at the cost of
// walking each free-flight segment once per group.
int camera_groups(int n_cams) { return n_cams < 3 ? n_cams : 3; }

int check_match(const prt_scene* s, prt_paths p)
{
    if (!p) return fail(PRT_E_INVALID, "paths is NULL");
    if (s->nx != p->nx || s->ny != p->ny || s->nz != p->nz || s->max_order != p->max_order)
        return fail(PRT_E_MISMATCH, "scene grid %dx%dx%d/order %d differs from the store's %dx%dx%d/order %d", s->nx,
                    s->ny, s->nz, s->max_order, p->nx, p->ny, p->nz, p->max_order);
    return PRT_OK;
}

template <typename T>
int dalloc(T** p, size_t count, uint64_t* bytes = nullptr)
{
    *p = nullptr;
    if (count == 0) count = 1;
    if (hipMalloc((void**)p, count * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(PRT_E_NOMEM, "hipMalloc of %zu bytes failed", count * sizeof(T));
    }
    if (bytes) *bytes += count * sizeof(T);
    return PRT_OK;
}

// Capacity for a buffer that must hold count elements, with 1/8 headroom:
// store sizes vary from one resample to the next, and regrowing a buffer
// (hipFree synchronises the device) on every new maximum would stall the
// iteration loop.
int64_t with_headroom(int64_t count) { return count + count / 8; }

int ensure_grids(prt_ctx c, int64_t nu)
{
    const size_t need = (size_t)nu * (c->fp64 ? 8 : 4);
    if (c->grid_bytes >= need) return PRT_OK;
    (void)hipFree(c->grid_tot);
    (void)hipFree(c->grid_dlt);
    c->grid_tot = c->grid_dlt = nullptr;
    c->grid_bytes = 0;
    if (hipMalloc(&c->grid_tot, need) != hipSuccess || hipMalloc(&c->grid_dlt, need) != hipSuccess)
        return fail(PRT_E_NOMEM, "grid scratch allocation failed");
    c->grid_bytes = need;
    return PRT_OK;
}

// The render's z-tiled copy of grid_tot (whole tiles of kTileZ layers).
int ensure_tile(prt_ctx c, int nx, int ny, int nz)
{
    const size_t need = (size_t)((nz + kTileZ - 1) / kTileZ) * kTileZ * nx * ny * (c->fp64 ? 8 : 4);
    if (c->tile_bytes >= need) return PRT_OK;
    (void)hipFree(c->grid_tile);
    c->grid_tile = nullptr;
    c->tile_bytes = 0;
    if (hipMalloc(&c->grid_tile, need) != hipSuccess) return fail(PRT_E_NOMEM, "grid scratch allocation failed");
    c->tile_bytes = need;
    return PRT_OK;
}

// Grows a context scratch buffer to at least `bytes`.
int ensure_scratch(void** buf, size_t* have, size_t bytes)
{
    if (bytes <= *have) return PRT_OK;
    (void)hipFree(*buf);
    *buf = nullptr;
    *have = 0;
    bytes = (size_t)with_headroom((int64_t)bytes);
    if (hipMalloc(buf, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *buf = nullptr;
        return fail(PRT_E_NOMEM, "scratch allocation of %zu bytes failed", bytes);
    }
    *have = bytes;
    return PRT_OK;
}

int ensure_pix(prt_ctx c, size_t n)
{
    if (c->pix_n >= n) return PRT_OK;
    (void)hipFree(c->pix);
    c->pix = nullptr;
    c->pix_n = 0;
    int rc = dalloc(&c->pix, n);
    if (rc) return rc;
    c->pix_n = n;
    return PRT_OK;
}

int ensure_part(prt_ctx c, size_t n)
{
    if (c->part_n >= n) return PRT_OK;
    (void)hipFree(c->part);
    c->part = nullptr;
    c->part_n = 0;
    int rc = dalloc(&c->part, n);
    if (rc) return rc;
    c->part_n = n;
    return PRT_OK;
}

// Frees a store.  It does not touch the context it was built with (the
// context may already be gone); it waits for all work on the store's device.
void free_store(prt_paths p)
{
    if (!p) return;
    DeviceGuard g(p->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(p->vtx);
    (void)hipFree(p->batch_off);
    (void)hipFree(p->B);
    (void)hipFree(p->nv);
    (void)hipFree(p->perm);
    (void)hipFree(p->beta_ref);
    (void)hipFree(p->tape);
    (void)hipFree(p->tape_beta);
    for (auto& t : p->tpp) {
        (void)hipFree(t.rec);
        (void)hipFree(t.off);
        (void)hipFree(t.B);
        (void)hipFree(t.inv);
    }
    delete p;
}

// Grows one buffer to hold `count` elements (contents not kept); *cap is
// the element count currently allocated for exactly this buffer.
template <typename T>
int grow(T** buf, int64_t* cap, int64_t count)
{
    count = std::max<int64_t>(count, 1);
    if (*buf && count <= *cap) return PRT_OK;
    (void)hipFree(*buf);
    *buf = nullptr;
    *cap = 0;
    const int64_t want = with_headroom(count);
    int rc = dalloc(buf, (size_t)want);
    if (rc == PRT_OK) *cap = want;
    return rc;
}

// Per-path arrays of a store for n paths (perm, sizes, batch offsets).
int reserve_paths(prt_paths p, int64_t n)
{
    const int64_t nb = (n + kWave - 1) / kWave;
    int rc;
    if ((rc = grow(&p->perm, &p->cap_perm, n))) return rc;
    if ((rc = grow(&p->B, &p->cap_slots, nb * kWave))) return rc;
    if ((rc = grow(&p->nv, &p->cap_nv, nb * kWave))) return rc;
    return grow(&p->batch_off, &p->cap_boff, nb + 1);
}

uint64_t store_bytes(const prt_paths_s* p)
{
    return (uint64_t)p->cap_perm * 4 + (uint64_t)p->cap_slots + (uint64_t)p->cap_nv + (uint64_t)p->cap_boff * 8 +
           (uint64_t)p->cap_records * 16 + (uint64_t)p->cap_nu * 4 + (uint64_t)p->tape_cap * 8 +
           (p->tape_beta ? (uint64_t)p->cap_nu * 4 : 0);
}

// Shared part of sample, resample and import: sort the paths by size (and
// spatial key), lay out the wavefront batches and read back the store size
// (one synchronisation), then grow the store's record buffer.  With inv,
// also writes inv[path id] = sorted slot.
int layout_store(prt_ctx c, prt_paths p, const uint8_t* tB, const uint8_t* tnv, const uint16_t* tC, int32_t** inv)
{
    const int64_t n = (int64_t)p->n;
    p->nb = (n + kWave - 1) / kWave;
    p->n_slots = p->nb * kWave;
    const int nbins = p->max_order + 1;
    int rc;
    if ((rc = reserve_paths(p, n))) return rc;
    if ((rc = ensure_scratch(&c->s_hist, &c->s_hist_bytes, sort_scratch_words(n, nbins) * sizeof(uint32_t)))) return rc;
    const int64_t n_i32 = n * (inv ? 2 : 1);
    if ((rc = ensure_scratch(&c->s_perm, &c->s_perm_bytes, (size_t)n_i32 * sizeof(int32_t) + (size_t)n * 2))) return rc;
    if (inv) *inv = (int32_t*)c->s_perm + n;
    uint16_t* carry = (uint16_t*)((int32_t*)c->s_perm + n_i32);
    {
        TimedScope ts(c, K_SORT);
        HIPCHK(launch_sort_paths(c->stream, tB, tnv, tC, n, p->n_slots, nbins, (uint32_t*)c->s_hist,
                                 (int32_t*)c->s_perm, carry, p->perm, p->B, p->nv, inv ? *inv : nullptr));
        HIPCHK(launch_batch_offsets(c->stream, p->nv, p->nb, p->batch_off, c->s_hist));
        HIPCHK(launch_store_meta(c->stream, p->B, n, p->batch_off, p->nb, c->dmeta));
    }
    // store_meta_kernel wrote the sizes into pinned host memory
    HIPCHK(hipStreamSynchronize(c->stream));
    p->n_records = c->hmeta[0];
    p->first_slot = c->hmeta[1];
    p->tape_base = c->hmeta[2];
    p->bmax = 0;
    for (int k = 1; k <= p->max_order && k <= kMaxOrder; ++k) {
        const int64_t f = c->hmeta[kMetaFirstGe + k];
        if (f >= n) break;
        p->bmax = k;
        p->first_batch_ge[k] = (int32_t)(f / kWave);
    }
    return grow(&p->vtx, &p->cap_records, p->n_records);
}

// Sort temporary paths (rows of tmp addressed by tmp_off, CSR, or by
// id * tmp_stride) into the store.
int build_store(prt_ctx c, prt_paths p, const float4* tmp, const int64_t* tmp_off, int64_t tmp_stride,
                const uint8_t* tB, const uint8_t* tnv, const uint16_t* tC, const float4* ovf = nullptr,
                const int32_t* ovf_slot = nullptr)
{
    int rc;
    if ((rc = layout_store(c, p, tB, tnv, tC, nullptr))) return rc;
    const int64_t n = (int64_t)p->n;
    {
        TimedScope ts(c, K_PACK);
        HIPCHK(launch_pack(c->stream, p->perm, tmp, tmp_off, tmp_stride, p->nv, p->batch_off, n, p->n_slots, p->vtx,
                           ovf, ovf_slot));
    }
    return PRT_OK;
}

// Records per path in the short rows of a one-pass draw that does not fit
// whole rows: an entry and an exit, all a path without a scatter needs.
constexpr int kShortRows = 2;
// Overflow segments a wavefront claims at a time: about a sixteenth of its
// share of the estimate, within these bounds (a wavefront leaves fewer than a
// chunk unused; small chunks make the shared counter's atomics contend).
constexpr int64_t kOvfChunkMin = 16, kOvfChunkMax = 256;

// Samples n paths into p (allocated or reused) under scene->beta_cloud.  When
// the one-pass temporary (max_order+2 records per path) would exceed the
// context's limit, the paths are drawn once into short rows and a pool of
// overflow segments; when that does not fit either, or the pool runs out,
// every path is drawn twice: first only its size and sort key, then, once
// the sort has fixed its slot, its vertices straight into the store.
int fill_sampled(prt_ctx c, const prt_scene* s, uint64_t seed, int64_t n, prt_paths p)
{
    const int64_t nu = (int64_t)s->nx * s->ny * s->nz;
    const int64_t stride = s->max_order + 2;
    const bool one_pass = (uint64_t)n * (uint64_t)stride * sizeof(float4) <= c->sample_tmp_limit;
    // otherwise short rows and an overflow pool of segments of kSegRecords - 1
    // records (and a link).  A refill estimates the segments from the
    // store's previous draw (a path of B scatters stores at most B records
    // past its short row, so it takes one segment for each of B >= 1, 8,
    // 15, ...; counted per batch from the sorted store's first batch with
    // B >= k and scaled to n) and takes a quarter more plus the
    // chunks the sampler's wavefronts (1024 threads per workgroup, at most two
    // workgroups per CU) may leave unused; a new store assumes a quarter of
    // its paths need a segment and takes twice that.  Either is cut to what
    // the limit leaves and used when it still holds the estimate.
    const int64_t seg_rec = kSegRecords - 1;
    const int64_t rows_recs = ((int64_t)n * kShortRows + kSegRecords - 1) / kSegRecords * kSegRecords;
    int64_t ovf_segs = 0;
    int ovf_chunk = (int)kOvfChunkMin;
    bool compact = false;
    const uint64_t rows_bytes = (uint64_t)rows_recs * sizeof(float4) + (uint64_t)n * sizeof(int32_t);
    if (!one_pass && stride > kShortRows && rows_bytes < c->sample_tmp_limit) {
        const bool refill = p->n_records > 0 && p->n > 0 && p->first_slot <= (int64_t)p->n;
        int64_t est = n / 4;
        if (refill) {
            double segs = 0;
            for (int k = 1; k <= p->bmax; k += (int)seg_rec)
                segs += (double)std::max<int64_t>((int64_t)p->n - (int64_t)p->first_batch_ge[k] * kWave, 0);
            est = (int64_t)(segs / (double)p->n * (double)n);
        }
        const int64_t waves = std::min<int64_t>((n + 1023) / 1024, (int64_t)c->n_cu * 2) * (1024 / kWave);
        ovf_chunk = (int)std::min<int64_t>(std::max<int64_t>(est / (16 * waves), kOvfChunkMin), kOvfChunkMax);
        const int64_t fit = (int64_t)((c->sample_tmp_limit - rows_bytes) / (kSegRecords * sizeof(float4)));
        ovf_segs = std::min<int64_t>(refill ? est + est / 4 + ovf_chunk * waves : 2 * est + ovf_chunk * waves, fit);
        compact = ovf_segs >= est && ovf_segs > 0 && ovf_segs < ((int64_t)1 << 31);
    }
    int rc;
    // earlier work may still read the store's or the context's buffers
    HIPCHK(hipDeviceSynchronize());
    if ((rc = ensure_grids(c, nu)) || (rc = ensure_tile(c, s->nx, s->ny, s->nz))) return rc;
    if ((rc = grow(&p->beta_ref, &p->cap_nu, nu))) return rc;
    if (one_pass && (rc = ensure_scratch(&c->s_tmp, &c->s_tmp_bytes, (size_t)n * stride * sizeof(float4)))) return rc;
    if (compact &&
        ((rc = ensure_scratch(&c->s_tmp, &c->s_tmp_bytes,
                              ((size_t)rows_recs + (size_t)ovf_segs * kSegRecords) * sizeof(float4))) ||
         (rc = ensure_scratch(&c->s_ovf, &c->s_ovf_bytes, (size_t)n * sizeof(int32_t) + 16))))
        return rc;
    if ((rc = ensure_scratch(&c->s_keys, &c->s_keys_bytes, 4 * (size_t)n))) return rc;
    p->n = (uint64_t)n;
    p->seed = seed;
    p->max_order = s->max_order;
    p->nx = s->nx;
    p->ny = s->ny;
    p->nz = s->nz;
    p->tape_valid = false;
    p->tpp[0].valid = p->tpp[1].valid = false;
    uint8_t* tB = (uint8_t*)c->s_keys;
    uint8_t* tnv = tB + n;
    uint16_t* tC = (uint16_t*)(tB + 2 * n);
    {
        // the reference snapshot beta_ref = beta_t, the sampler's grid and its id counter
        TimedScope ts(c, K_PREP);
        // (and its z-tiled copy, walked when the grid does not fit the LDS)
        HIPCHK(launch_prep_grids(c->stream, c->fp64, s->beta_cloud, nullptr, s->beta_air, nu, c->grid_tot, nullptr,
                                 p->beta_ref, c->work + 2, c->grid_tile, s->nx, s->ny));
    }
    SampleArgs a;
    a.s = make_dev_scene(s);
    a.beta_c = p->beta_ref;
    a.grid_tot = c->grid_tot;
    a.grid_tile = c->grid_tile;
    a.seed = seed;
    a.n = n;
    a.tmp = (one_pass || compact) ? (float4*)c->s_tmp : nullptr;
    a.tmp_rows = compact ? kShortRows : (int)stride;
    a.ovf = compact ? (float4*)c->s_tmp + rows_recs : nullptr;
    a.ovf_cap = compact ? ovf_segs : 0;
    a.ovf_chunk = ovf_chunk;
    a.ovf_next = compact ? (unsigned long long*)c->s_ovf : nullptr;
    a.ovf_slot = compact ? (int32_t*)((unsigned char*)c->s_ovf + 16) : nullptr;
    a.ovf_full = compact ? (int*)(c->dmeta + kOvfFullWord) : nullptr;
    volatile int* ovf_full = (volatile int*)(c->hmeta + kOvfFullWord);
    if (compact) {
        *ovf_full = 0;
        HIPCHK(hipMemsetAsync(c->s_ovf, 0, 16, c->stream));
    }
    a.vtx = nullptr;
    a.batch_off = nullptr;
    a.inv = nullptr;
    a.mismatch = nullptr;
    a.tB = tB;
    a.tnv = tnv;
    a.tC = tC;
    a.next = c->work + 2;
    {
        TimedScope ts(c, K_SAMPLE);
        HIPCHK(launch_sample(c->stream, c->fp64, a, c->n_cu));
    }
    if (one_pass) return build_store(c, p, (const float4*)c->s_tmp, nullptr, stride, tB, tnv, tC);
    if (compact) {
        HIPCHK(hipStreamSynchronize(c->stream));
        if (*ovf_full == 0)
            return build_store(c, p, (const float4*)c->s_tmp, nullptr, kShortRows, tB, tnv, tC, a.ovf, a.ovf_slot);
        // the pool ran out: the sizes and keys are complete, so the second
        // pass of the two-pass draw finishes the store
    }
    int32_t* inv = nullptr;
    if ((rc = layout_store(c, p, tB, tnv, tC, &inv))) return rc;
    // second pass: padding rows are zero, the sampler writes every path's records
    volatile int* mismatch = (volatile int*)(c->hmeta + kMismatchWord);
    *mismatch = 0;
    HIPCHK(hipMemsetAsync(p->vtx, 0, (size_t)p->n_records * sizeof(float4), c->stream));
    HIPCHK(hipMemsetAsync(c->work + 2, 0, sizeof(unsigned int), c->stream));
    a.tmp = nullptr;
    a.tmp_rows = (int)stride;
    a.ovf = nullptr;
    a.ovf_cap = 0;
    a.ovf_chunk = 0;
    a.ovf_next = nullptr;
    a.ovf_slot = nullptr;
    a.ovf_full = nullptr;
    a.vtx = p->vtx;
    a.batch_off = p->batch_off;
    a.inv = inv;
    a.mismatch = (int*)(c->dmeta + kMismatchWord);
    {
        TimedScope ts(c, K_SAMPLE);
        HIPCHK(launch_sample(c->stream, c->fp64, a, c->n_cu));
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    if (*mismatch != 0)
        return fail(PRT_E_HIP, "two-pass resample: a path redrawn in the second pass differs from the first");
    return PRT_OK;
}

// Tape capacity: one (FP32 c, pixel) entry per (vertex record, camera) from the first
// scattering batch on; capped so that large workloads recompute instead.
constexpr size_t kMaxTapeBytes = (size_t)64 << 30;
// Tape-driven gradients whose grid needs at most this many LDS slabs walk
// every task once per slab; larger grids bin the walks by slab.
constexpr int kSlabWalkMax = 4;
// Largest task-list allocation of the binned gradient (every task in every slab).
constexpr size_t kMaxBinListBytes = (size_t)8 << 30;

int ensure_tape(prt_paths p, size_t n_cams, int64_t nu)
{
    const size_t need = (size_t)(p->n_records - p->tape_base) * n_cams;
    if (need * sizeof(float2) > kMaxTapeBytes) return PRT_E_CAPACITY;
    if (!p->tape_beta && hipMalloc((void**)&p->tape_beta, (size_t)nu * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        p->tape_beta = nullptr;
        return PRT_E_NOMEM;
    }
    if (need <= p->tape_cap && p->tape) return PRT_OK;
    (void)hipFree(p->tape);
    p->tape = nullptr;
    p->tape_cap = 0;
    const size_t want = std::max<size_t>((size_t)with_headroom((int64_t)need), 1);
    if (hipMalloc((void**)&p->tape, want * sizeof(float2)) != hipSuccess) {
        (void)hipGetLastError();
        p->tape = nullptr;
        return PRT_E_NOMEM;
    }
    p->tape_cap = want;
    return PRT_OK;
}

prt_paths new_store(prt_ctx c, const prt_scene* s, uint64_t n, uint64_t seed)
{
    prt_paths p = new prt_paths_s();
    p->device = c->device;
    p->n = n;
    p->seed = seed;
    p->max_order = s->max_order;
    p->nx = s->nx;
    p->ny = s->ny;
    p->nz = s->nz;
    return p;
}

// Per-vertex task levels of the store up to scatter index bmax.
VertexLevels task_levels(const prt_paths_s* p, int bmax)
{
    VertexLevels lv{};
    lv.bmax = std::min(bmax, p->bmax);
    for (int b = lv.bmax; b >= 1; --b) {
        lv.first_batch[b] = p->first_batch_ge[b];
        lv.start[b] = lv.total;
        lv.total += (uint32_t)(p->nb - p->first_batch_ge[b]);
    }
    return lv;
}

StoreView view_of(prt_paths p)
{
    StoreView v;
    v.vtx = p->vtx;
    v.batch_off = p->batch_off;
    v.B = p->B;
    v.nv = p->nv;
    v.n_slots = p->n_slots;
    v.first_slot = p->first_slot;
    v.beta_ref = p->beta_ref;
    return v;
}

}  // namespace

// ------------------------------------------------ no-allocation scratch

// Device scratch of prt_reweight_noalloc: one fixed array per GPU, held until
// the process ends.  Host code never passes its name to a kernel (on the host
// it is only a stand-in for the symbol); it uses the device address that
// hipGetSymbolAddress returns, looked up once per device by prt_create with
// that device current.
static __device__ __align__(256) unsigned char scratch[PRT_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (the device is current).
int lookup_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return fail(PRT_E_CAPACITY, "device %d beyond %d", device, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return PRT_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return fail(PRT_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    }
    g_scratch_ptr[device] = p;
    return PRT_OK;
}

void* scratch_of(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

// ================================================================== C ABI

extern "C" {

const char* prt_last_error(void) { return g_err.c_str(); }

int prt_create(int device, void* hip_stream, int precision, prt_ctx* out)
{
    if (!out) return fail(PRT_E_INVALID, "out is NULL");
    *out = nullptr;
    if (precision != PRT_TRAVERSAL_FP32 && precision != PRT_ALL_FP64) return fail(PRT_E_INVALID, "unknown precision %d", precision);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(PRT_E_HIP, "no HIP device available");
    if (device < 0 || device >= ndev) return fail(PRT_E_INVALID, "device %d out of range (have %d)", device, ndev);
    DeviceGuard g(device);
    // the no-allocation entry point's scratch address on this device
    if (int rc = lookup_scratch(device)) return rc;
    prt_ctx c = new prt_ctx_s();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->fp64 = precision == PRT_ALL_FP64;
    if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || c->n_cu < 1)
        c->n_cu = 1;
    void* dpin = nullptr;
    if (hipMalloc((void**)&c->counters, 4 * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc((void**)&c->flag, sizeof(int)) != hipSuccess ||
        hipMalloc((void**)&c->work, kWorkWords * sizeof(unsigned int)) != hipSuccess ||
        hipHostMalloc(&c->hpin, kMetaWords * sizeof(int64_t), hipHostMallocCoherent) != hipSuccess ||
        hipHostGetDevicePointer(&dpin, c->hpin, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(c->work);
        (void)hipFree(c->flag);
        (void)hipFree(c->counters);
        if (c->hpin) (void)hipHostFree(c->hpin);
        delete c;
        return fail(PRT_E_NOMEM, "context allocation failed");
    }
    c->hmeta = (int64_t*)c->hpin;
    c->hsum = (double*)((char*)c->hpin + 32);
    c->dmeta = (int64_t*)dpin;
    c->dsum = (double*)((char*)dpin + 32);
    // task counters start at zero
    if (hipMemset(c->counters, 0, 4 * sizeof(unsigned long long)) != hipSuccess ||
        hipMemset(c->work, 0, kWorkWords * sizeof(unsigned int)) != hipSuccess) {
        (void)hipFree(c->work);
        (void)hipFree(c->flag);
        (void)hipFree(c->counters);
        (void)hipHostFree(c->hpin);
        delete c;
        return fail(PRT_E_HIP, "context init failed");
    }
    *out = c;
    return PRT_OK;
}

void prt_destroy(prt_ctx c)
{
    if (!c) return;
    DeviceGuard g(c->device);
    (void)hipDeviceSynchronize();
    for (auto& t : c->pending) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (auto e : c->pool) (void)hipEventDestroy(e);
    (void)hipFree(c->grid_tot);
    (void)hipFree(c->grid_dlt);
    (void)hipFree(c->grid_tile);
    (void)hipFree(c->pix);
    (void)hipFree(c->gpart);
    (void)hipFree(c->rpart);
    (void)hipFree(c->gw);
    (void)hipFree(c->gaux);
    (void)hipFree(c->bin_trange);
    (void)hipFree(c->bin_cnt);
    (void)hipFree(c->bin_list);
    (void)hipFree(c->bin_part);
    (void)hipFree(c->bin_rtape);
    (void)hipFree(c->bin_brange);
    (void)hipFree(c->pb);
    (void)hipFree(c->s_tmp);
    (void)hipFree(c->s_ovf);
    (void)hipFree(c->s_keys);
    (void)hipFree(c->s_hist);
    (void)hipFree(c->s_off);
    (void)hipFree(c->s_perm);
    (void)hipHostFree(c->hpin);
    (void)hipFree(c->part);
    (void)hipFree(c->flag);
    (void)hipFree(c->work);
    (void)hipFree(c->counters);
    delete c;
}

int prt_set_sample_scratch_limit(prt_ctx c, uint64_t bytes)
{
    if (!c) return fail(PRT_E_INVALID, "ctx is NULL");
    c->sample_tmp_limit = bytes;
    return PRT_OK;
}

int prt_set_stream(prt_ctx c, void* hip_stream)
{
    if (!c) return fail(PRT_E_INVALID, "ctx is NULL");
    c->stream = (hipStream_t)hip_stream;
    return PRT_OK;
}

int prt_sample(prt_ctx c, const prt_scene* s, uint64_t seed, uint64_t n_paths, prt_paths* out)
{
    if (!c || !out) return fail(PRT_E_INVALID, "ctx/out is NULL");
    *out = nullptr;
    int rc = check_scene(s);
    if (rc) return rc;
    if (n_paths < 1 || n_paths > ((uint64_t)1 << 31) - 64) return fail(PRT_E_CAPACITY, "n_paths must be in [1, 2^31-64]");
    DeviceGuard g(c->device);
    prt_paths p = new_store(c, s, n_paths, seed);
    if ((rc = fill_sampled(c, s, seed, (int64_t)n_paths, p))) {
        (void)hipStreamSynchronize(c->stream);
        free_store(p);
        return rc;
    }
    *out = p;
    return PRT_OK;
}

int prt_resample(prt_ctx c, const prt_scene* s, uint64_t seed, uint64_t n_paths, prt_paths p)
{
    if (!c || !p) return fail(PRT_E_INVALID, "ctx/paths is NULL");
    int rc = check_scene(s);
    if (rc) return rc;
    if (n_paths < 1 || n_paths > ((uint64_t)1 << 31) - 64) return fail(PRT_E_CAPACITY, "n_paths must be in [1, 2^31-64]");
    if (p->device != c->device) return fail(PRT_E_INVALID, "store lives on device %d, context on %d", p->device, c->device);
    DeviceGuard g(c->device);
    if ((rc = fill_sampled(c, s, seed, (int64_t)n_paths, p))) {
        // the store is left empty but valid
        p->n = 0;
        p->nb = p->n_slots = p->first_slot = p->n_records = 0;
        p->bmax = 0;
        p->tape_valid = false;
        p->tpp[0].valid = p->tpp[1].valid = false;
        return rc;
    }
    return PRT_OK;
}

int prt_paths_import(prt_ctx c, const prt_scene* s, uint64_t n_paths, const int64_t* off, const float* xyz,
                     const int32_t* vox, const int32_t* B, const float* beta_ref, uint64_t seed, prt_paths* out)
{
    if (!c || !out) return fail(PRT_E_INVALID, "ctx/out is NULL");
    *out = nullptr;
    int rc = check_scene(s);
    if (rc) return rc;
    if (!off || !xyz || !vox || !B || !beta_ref) return fail(PRT_E_INVALID, "import arrays must be non-NULL");
    if (n_paths < 1 || n_paths > ((uint64_t)1 << 31) - 64) return fail(PRT_E_CAPACITY, "n_paths must be in [1, 2^31-64]");
    const int64_t nu = (int64_t)s->nx * s->ny * s->nz;
    const int64_t n = (int64_t)n_paths;
    if (off[0] != 0) return fail(PRT_E_INVALID, "off[0] must be 0");
    for (int64_t i = 0; i < n; ++i) {
        const int64_t cnt = off[i + 1] - off[i];
        const int b = B[i];
        if (b < 0 || b > s->max_order) return fail(PRT_E_INVALID, "path %lld: B=%d outside [0, max_order]", (long long)i, b);
        const int64_t want = b == s->max_order ? b + 1 : b + 2;
        if (cnt != want)
            return fail(PRT_E_INVALID, "path %lld: %lld vertices for B=%d", (long long)i, (long long)cnt, b);
        for (int64_t k = 0; k < cnt; ++k) {
            const int32_t v = vox[off[i] + k];
            const bool exit_vertex = (k == cnt - 1) && (cnt == b + 2);
            if (exit_vertex ? v != -1 : (v < 0 || v >= nu))
                return fail(PRT_E_INVALID, "path %lld vertex %lld: voxel %d invalid", (long long)i, (long long)k, v);
            for (int a = 0; a < 3; ++a)
                if (!std::isfinite(xyz[3 * (off[i] + k) + a])) return fail(PRT_E_INVALID, "non-finite vertex");
        }
    }
    DeviceGuard g(c->device);
    const int64_t nrec = off[n];
    std::vector<float4> h(nrec);
    for (int64_t r = 0; r < nrec; ++r) {
        float4 q;
        q.x = xyz[3 * r];
        q.y = xyz[3 * r + 1];
        q.z = xyz[3 * r + 2];
        std::memcpy(&q.w, &vox[r], 4);
        h[r] = q;
    }
    std::vector<uint8_t> hB(n), hnv(n);
    std::vector<uint16_t> hC(n);
    for (int64_t i = 0; i < n; ++i) {
        hB[i] = (uint8_t)B[i];
        hnv[i] = (uint8_t)(off[i + 1] - off[i]);
        hC[i] = (uint16_t)cell_key(vox[off[i] + (B[i] > 0 ? 1 : 0)], s->nx, s->ny, s->nz);
    }
    prt_paths p = new_store(c, s, n_paths, seed);
    auto bail = [&](int code) {
        (void)hipStreamSynchronize(c->stream);
        free_store(p);
        return code;
    };
    if ((rc = grow(&p->beta_ref, &p->cap_nu, nu))) return bail(rc);
    if ((rc = ensure_scratch(&c->s_tmp, &c->s_tmp_bytes, (size_t)nrec * sizeof(float4)))) return bail(rc);
    if ((rc = ensure_scratch(&c->s_off, &c->s_off_bytes, (size_t)(n + 1) * sizeof(int64_t)))) return bail(rc);
    if ((rc = ensure_scratch(&c->s_keys, &c->s_keys_bytes, 4 * (size_t)n))) return bail(rc);
    float4* tmp = (float4*)c->s_tmp;
    int64_t* toff = (int64_t*)c->s_off;
    uint8_t* tB = (uint8_t*)c->s_keys;
    uint8_t* tnv = tB + n;
    uint16_t* tC = (uint16_t*)(tB + 2 * n);
    hipError_t e = hipMemcpy(tmp, h.data(), nrec * sizeof(float4), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(toff, off, (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(tB, hB.data(), n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(tnv, hnv.data(), n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(tC, hC.data(), n * sizeof(uint16_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->beta_ref, beta_ref, nu * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bail(fail(PRT_E_HIP, "import upload: %s", hipGetErrorString(e)));
    if ((rc = build_store(c, p, tmp, toff, 0, tB, tnv, tC))) return bail(rc);
    *out = p;
    return PRT_OK;
}

int prt_paths_export(prt_ctx c, prt_paths p, int64_t* off, float* xyz, int32_t* vox, int32_t* B, float* beta_ref)
{
    if (!c || !p || !off || !B) return fail(PRT_E_INVALID, "ctx/paths/off/B must be non-NULL");
    DeviceGuard g(p->device);
    HIPCHK(hipStreamSynchronize(c->stream));
    const int64_t n = (int64_t)p->n;
    std::vector<int32_t> perm(n);
    std::vector<uint8_t> hB(p->n_slots), hnv(p->n_slots);
    std::vector<int64_t> boff(p->nb + 1);
    HIPCHK(hipMemcpy(perm.data(), p->perm, n * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(hB.data(), p->B, p->n_slots, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(hnv.data(), p->nv, p->n_slots, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(boff.data(), p->batch_off, (p->nb + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
    std::vector<int64_t> slot_of(n);
    for (int64_t i = 0; i < n; ++i) slot_of[perm[i]] = i;
    off[0] = 0;
    for (int64_t id = 0; id < n; ++id) {
        off[id + 1] = off[id] + hnv[slot_of[id]];
        B[id] = hB[slot_of[id]];
    }
    if (xyz || vox) {
        std::vector<float4> hv(p->n_records);
        HIPCHK(hipMemcpy(hv.data(), p->vtx, p->n_records * sizeof(float4), hipMemcpyDeviceToHost));
        for (int64_t id = 0; id < n; ++id) {
            const int64_t i = slot_of[id];
            const int64_t base = boff[i / kWave] + i % kWave;
            for (int k = 0; k < hnv[i]; ++k) {
                const float4 q = hv[base + (int64_t)k * kWave];
                const int64_t r = off[id] + k;
                if (xyz) {
                    xyz[3 * r] = q.x;
                    xyz[3 * r + 1] = q.y;
                    xyz[3 * r + 2] = q.z;
                }
                if (vox) std::memcpy(&vox[r], &q.w, 4);
            }
        }
    }
    if (beta_ref)
        HIPCHK(hipMemcpy(beta_ref, p->beta_ref, (size_t)p->nx * p->ny * p->nz * sizeof(float), hipMemcpyDeviceToHost));
    return PRT_OK;
}

int prt_paths_permutation(prt_ctx c, prt_paths p, int32_t* perm)
{
    if (!c || !p || !perm) return fail(PRT_E_INVALID, "ctx/paths/perm must be non-NULL");
    DeviceGuard g(p->device);
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(perm, p->perm, p->n * sizeof(int32_t), hipMemcpyDeviceToHost));
    return PRT_OK;
}

int prt_paths_info(prt_paths p, prt_paths_info_t* info)
{
    if (!p || !info) return fail(PRT_E_INVALID, "paths/info is NULL");
    info->n_paths = p->n;
    info->n_vertices = (uint64_t)p->n_records;
    info->n_batches = (uint64_t)p->nb;
    info->seed = p->seed;
    info->bytes = store_bytes(p);
    info->max_order = p->max_order;
    info->nx = p->nx;
    info->ny = p->ny;
    info->nz = p->nz;
    return PRT_OK;
}

void prt_paths_destroy(prt_paths p) { free_store(p); }

int prt_render(prt_ctx c, const prt_scene* s, const prt_cameras* cams, prt_paths p, int32_t max_order_render,
               double* images)
{
    if (!c) return fail(PRT_E_INVALID, "ctx is NULL");
    int rc = check_scene(s);
    if (rc) return rc;
    if ((rc = check_match(s, p))) return rc;
    if (!images) return fail(PRT_E_INVALID, "images is NULL");
    if (max_order_render < 0) return fail(PRT_E_INVALID, "max_order_render must be >= 0");
    TraceArgs a{};
    DevCams dc;
    if ((rc = make_dev_cams(cams, s, &dc))) return rc;
    DeviceGuard g(c->device);
    const int64_t nu = (int64_t)s->nx * s->ny * s->nz;
    if ((rc = ensure_grids(c, nu))) return rc;
    const int64_t npx = (int64_t)dc.n * dc.W * dc.H;
    // batches with scattering paths (the kernels have nothing to do without them)
    const bool work = p->n_slots > p->first_slot;
    a.s = make_dev_scene(s);
    a.st = view_of(p);
    a.bc_t = s->beta_cloud;
    a.grid_tot = c->grid_tot;
    a.grid_dlt = c->grid_dlt;
    a.img = images;
    a.brender = std::min(max_order_render, s->max_order);
    a.counters = c->counters;
    a.work = c->work;
    a.groups = camera_groups(dc.n);
    a.tape_base = p->tape_base;
    if ((rc = ensure_scratch(&c->pb, &c->pb_bytes, (size_t)(p->n_records - p->tape_base) * sizeof(double))))
        return rc;
    a.pbase = (double*)c->pb;
    // record the transmittance tape when the render covers every order (FP32 mode)
    p->tape_valid = false;
    if (!c->fp64 && a.brender >= s->max_order && (rc = ensure_tape(p, (size_t)dc.n, nu)) == PRT_OK) {
        a.tape = p->tape;
        a.copy_beta = p->tape_beta;  // by the render prefix kernel
        p->tape_valid = true;
        p->tape_cams = dc;
        p->tape_scene = a.s;
    }
    const RenderPlan plan = plan_render(c->fp64, nu, dc, a.tape != nullptr, p->n_slots, p->first_slot, c->n_cu);
    if (work && !plan.grid_lds && (rc = ensure_tile(c, s->nx, s->ny, s->nz))) return rc;
    a.grid_tile = plan.grid_lds ? nullptr : c->grid_tile;
    {
        TimedScope ts(c, K_PREP);
        // the reductions write every pixel; otherwise tallies add up on zeros
        if (!work || !plan.img_tape) HIPCHK(launch_fill(c->stream, images, npx, 0.0));
        // kernels that hold a grid in LDS form it there from the fields
        if (work && (!plan.grid_lds || !delta_grid_lds(c->fp64, nu)))
            HIPCHK(launch_prep_grids(c->stream, c->fp64, s->beta_cloud, p->beta_ref, s->beta_air, nu, c->grid_tot,
                                     c->grid_dlt, nullptr, nullptr, plan.grid_lds ? nullptr : c->grid_tile, s->nx,
                                     s->ny));
    }
    if ((rc = ensure_scratch(&c->rpart, &c->rpart_bytes, plan.partial_bytes))) return rc;
    if (work) {
        {
            TimedScope ts(c, K_RENDER_PREFIX);
            // also zeroes the render's task counters and copies the tape's beta_t
            HIPCHK(launch_render_prefix(c->stream, c->fp64, a, task_levels(p, a.brender), c->n_cu));
        }
        {
            TimedScope ts(c, K_RENDER);
            HIPCHK(launch_render(c->stream, c->fp64, a, dc, plan));
        }
        TimedScope ts(c, K_RENDER_REDUCE);
        HIPCHK(launch_render_reduce(c->stream, a, dc, plan, c->rpart, 1.0 / (double)p->n, images));
    }
    // the reductions above also divide by N Omega_p; atomic tallies get it here
    if (work && !plan.img_tape) {
        TimedScope ts(c, K_FINALIZE);
        HIPCHK(launch_render_finalize(c->stream, images, dc, 1.0 / (double)p->n));
    }
    c->paths_done += p->n;
    return PRT_OK;
}

int prt_grad(prt_ctx c, const prt_scene* s, const prt_cameras* cams, prt_paths p, const double* residual, double* grad)
{
    if (!c) return fail(PRT_E_INVALID, "ctx is NULL");
    int rc = check_scene(s);
    if (rc) return rc;
    if ((rc = check_match(s, p))) return rc;
    if (!residual || !grad) return fail(PRT_E_INVALID, "residual/grad is NULL");
    DevCams dc;
    if ((rc = make_dev_cams(cams, s, &dc))) return rc;
    DeviceGuard g(c->device);
    const int64_t nu = (int64_t)s->nx * s->ny * s->nz;
    if ((rc = ensure_grids(c, nu))) return rc;
    const int64_t npx = (int64_t)dc.n * dc.W * dc.H;
    if ((rc = ensure_pix(c, npx))) return rc;
    // batches with scattering paths (the kernels have nothing to do without them)
    const bool work = p->n_slots > p->first_slot;
    const DevScene ds = make_dev_scene(s);
    const size_t recs = (size_t)(p->n_records - p->tape_base);  // records from the first scattering batch on
    // the tape of the last render serves when it was recorded for these
    // cameras and this scene (and, checked on the device, this beta_t)
    bool tape = work && recs > 0 && p->tape_valid && !c->fp64 && std::memcmp(&p->tape_cams, &dc, sizeof dc) == 0 &&
                std::memcmp(&p->tape_scene, &ds, sizeof ds) == 0;
    if (tape) {
        // weights and per-vertex sums for the walks on the tape; without room
        // for them the gradient recomputes
        if (ensure_scratch(&c->gw, &c->gw_bytes, recs * dc.n * sizeof(float)) != PRT_OK ||
            ensure_scratch(&c->gaux, &c->gaux_bytes, recs * sizeof(float4)) != PRT_OK)
            tape = false;
    }
    // with the tape, a grid needing more than a few LDS slabs has its walks
    // binned by slab (one persistent launch) when the lists fit; the slab
    // loop below then only holds the recomputing kernel, which works when the
    // tape turns out not to match beta_t.  Up to kSlabWalkMax slabs, one walk
    // launch per slab costs less than the binning.
    GradBins bins{};
    bool binned = false;
    const GradPlan per_slab = plan_grad(s->nx, s->ny, s->nz, p->n_slots, p->first_slot, c->n_cu, true);
    if (tape && !(per_slab.lds && per_slab.n_slabs <= kSlabWalkMax)) {
        const int64_t kinds = camera_groups(dc.n) + 1;
        // tasks as the walk kernels number them: every batch from the one
        // holding the first scattering path, times the walk kinds
        bins = choose_grad_bins(ds, dc, (p->nb - p->first_slot / kWave) * kinds);
        const size_t list_words = (size_t)bins.n_tasks * (size_t)bins.n_slabs;
        const int64_t cnt_words = (int64_t)bins.n_slabs * bins.n_blocks + 1;
        binned = grad_bins_fit(ds, bins) && list_words * sizeof(uint32_t) <= kMaxBinListBytes &&
                 ensure_scratch(&c->bin_trange, &c->bin_trange_bytes, (size_t)bins.n_tasks * 2 * sizeof(int)) ==
                     PRT_OK &&
                 ensure_scratch(&c->bin_cnt, &c->bin_cnt_bytes,
                                (size_t)(cnt_words + scan_u32_scratch_words(cnt_words)) * sizeof(uint32_t)) == PRT_OK &&
                 ensure_scratch(&c->bin_list, &c->bin_list_bytes,
                                (std::max<size_t>(list_words, 1) + bins.n_slabs + 2) * sizeof(uint32_t)) == PRT_OK &&
                 ensure_scratch(&c->bin_part, &c->bin_part_bytes, grad_bin_partial_bytes(ds, bins, c->n_cu)) == PRT_OK &&
                 ensure_scratch(&c->bin_rtape, &c->bin_rtape_bytes, recs * dc.n * sizeof(uint16_t)) == PRT_OK &&
                 ensure_scratch(&c->bin_brange, &c->bin_brange_bytes,
                                (recs / kWave + 1) * (size_t)(kinds - 1) * sizeof(uint32_t)) == PRT_OK;
        if (binned) {
            bins.cnt = (uint32_t*)c->bin_cnt;
            bins.list = (uint32_t*)c->bin_list;
            bins.list_cap = (int64_t)list_words;
            bins.chunks = bins.list + std::max<size_t>(list_words, 1);
            bins.partial = (double*)c->bin_part;
        }
    }
    const GradPlan plan = plan_grad(s->nx, s->ny, s->nz, p->n_slots, p->first_slot, c->n_cu, tape && !binned);
    TraceArgs a{};
    a.s = ds;
    a.st = view_of(p);
    a.grad = grad;
    if (binned) {
        a.trange = (int*)c->bin_trange;
        a.rtape = (uint16_t*)c->bin_rtape;
        a.brange = (uint32_t*)c->bin_brange;
        a.bin_axis = bins.axis;
        a.bin_layers = bins.layers;
    }
    {
        TimedScope ts(c, K_PREP);
        // the slabs' reductions write every voxel; otherwise atomics add up on zeros
        if (!work || (!plan.lds && !binned)) HIPCHK(launch_fill(c->stream, grad, nu, 0.0));
        if (!work) return PRT_OK;
        // empty task ranges and a zeroed gradient for the binned walk
        if (binned) HIPCHK(launch_grad_bin_init(c->stream, a, bins));
        HIPCHK(launch_prep_grids(c->stream, c->fp64, s->beta_cloud, p->beta_ref, s->beta_air, nu, c->grid_tot,
                                 c->grid_dlt));
        // also sets the tape flag (cleared by launch_equal_flag on a mismatch) and
        // zeroes the first slab's task counters
        HIPCHK(launch_grad_prep(c->stream, residual, c->pix, dc, 1.0 / (double)p->n, tape ? c->flag : nullptr,
                                c->work));
    }
    a.bc_t = s->beta_cloud;
    a.grid_tot = c->grid_tot;
    a.grid_dlt = c->grid_dlt;
    a.rho = c->pix;
    a.brender = s->max_order;
    a.counters = c->counters;
    a.work = c->work;
    a.groups = camera_groups(dc.n);
    if (tape) {
        // the tape is used only if beta_t equals the field it was recorded with
        HIPCHK(launch_equal_flag(c->stream, s->beta_cloud, p->tape_beta, nu, c->flag));
        a.tape = p->tape;
        a.tape_base = p->tape_base;
        a.tape_flag = c->flag;
        a.wtape = (float*)c->gw;
        a.vaux = (float4*)c->gaux;
        TimedScope ts(c, K_GRAD_WEIGHTS);
        HIPCHK(launch_grad_weights(c->stream, a, dc, task_levels(p, p->bmax), c->n_cu));
    }
    if (binned) {
        {
            TimedScope ts(c, K_GRAD_BIN);
            HIPCHK(launch_grad_bin_lists(c->stream, a, bins,
                                         (uint32_t*)c->bin_cnt + (int64_t)bins.n_slabs * bins.n_blocks + 1));
        }
        {
            TimedScope ts(c, K_GRAD);
            HIPCHK(launch_grad_bin_walk(c->stream, a, dc, bins, c->n_cu));
        }
        TimedScope ts(c, K_GRAD_REDUCE);
        HIPCHK(launch_grad_bin_reduce(c->stream, a, bins));
    }
    if ((rc = ensure_scratch(&c->gpart, &c->gpart_bytes, plan.partial_bytes))) return rc;
    // task counters: zeroed by launch_grad_prep for the first slab, by each
    // slab's reduction for the next (one slab only when there is no reduction)
    for (int i = 0; i < plan.n_slabs; ++i) {
        {
            TimedScope ts(c, binned ? K_GRAD_RECOMPUTE : K_GRAD);
            HIPCHK(launch_grad(c->stream, c->fp64, a, dc, plan, i, c->gpart, !binned));
        }
        TimedScope ts(c, K_GRAD_REDUCE);
        HIPCHK(launch_grad_reduce(c->stream, plan, s->nx, s->ny, s->nz, i, c->gpart, grad, c->work,
                                  binned ? c->flag : nullptr));
    }
    return PRT_OK;
}

// The per-path copy of store p in `order` for the ablation kernels (built
// on first use): sizes, offsets and records.
int tpp_copy(prt_ctx c, prt_paths p, int order, TppView* v)
{
    auto& t = p->tpp[order];
    const int64_t n = (int64_t)p->n;
    v->n = n;
    if (!t.valid) {
        int rc;
        if (t.cap_n < n + 1) {
            (void)hipFree(t.off);
            (void)hipFree(t.B);
            (void)hipFree(t.inv);
            t.off = nullptr;
            t.B = nullptr;
            t.inv = nullptr;
            t.cap_n = 0;
            if ((rc = dalloc(&t.off, (size_t)n + 1)) || (rc = dalloc(&t.B, (size_t)n + 1)) ||
                (rc = dalloc(&t.inv, (size_t)n + 1)))
                return rc;
            t.cap_n = n + 1;
        }
        if (t.cap_rec < p->n_records) {
            (void)hipFree(t.rec);
            t.rec = nullptr;
            t.cap_rec = 0;
            if ((rc = dalloc(&t.rec, (size_t)std::max<int64_t>(p->n_records, 1)))) return rc;
            t.cap_rec = p->n_records;
        }
        if ((rc = ensure_scratch(&c->s_hist, &c->s_hist_bytes,
                                 (size_t)scan_u32_scratch_words(n + 1) * sizeof(int64_t))))
            return rc;
        TimedScope ts(c, K_TPP_LAYOUT);
        const StoreView sv = view_of(p);
        HIPCHK(launch_tpp_layout(c->stream, sv, n, p->perm, order, t.inv, t.off, t.B, c->s_hist));
        HIPCHK(launch_tpp_copy(c->stream, sv, n, t.inv, order, t.off, t.rec));
        t.valid = true;
    }
    v->rec = t.rec;
    v->off = t.off;
    v->B = t.B;
    return PRT_OK;
}

int prt_tpp_render(prt_ctx c, const prt_scene* s, const prt_cameras* cams, prt_paths p, int32_t order,
                   double* images)
{
    if (!c) return fail(PRT_E_INVALID, "ctx is NULL");
    int rc = check_scene(s);
    if (rc) return rc;
    if ((rc = check_match(s, p))) return rc;
    if (!images) return fail(PRT_E_INVALID, "images is NULL");
    if (order != PRT_ORDER_BY_SIZE && order != PRT_ORDER_BY_ID) return fail(PRT_E_INVALID, "unknown order %d", order);
    DevCams dc;
    if ((rc = make_dev_cams(cams, s, &dc))) return rc;
    DeviceGuard g(c->device);
    const int64_t nu = (int64_t)s->nx * s->ny * s->nz;
    if ((rc = ensure_grids(c, nu))) return rc;
    TppView v{};
    if ((rc = tpp_copy(c, p, order, &v))) return rc;
    TraceArgs a{};
    a.s = make_dev_scene(s);
    a.st = view_of(p);
    a.bc_t = s->beta_cloud;
    a.grid_tot = c->grid_tot;
    a.grid_dlt = c->grid_dlt;
    a.img = images;
    a.brender = s->max_order;
    a.counters = c->counters;
    {
        TimedScope ts(c, K_PREP);
        HIPCHK(launch_fill(c->stream, images, (int64_t)dc.n * dc.W * dc.H, 0.0));
        HIPCHK(launch_prep_grids(c->stream, c->fp64, s->beta_cloud, p->beta_ref, s->beta_air, nu, c->grid_tot,
                                 c->grid_dlt));
    }
    {
        TimedScope ts(c, K_TPP_RENDER);
        HIPCHK(launch_tpp_render(c->stream, c->fp64, a, dc, v, c->n_cu));
    }
    TimedScope ts(c, K_FINALIZE);
    HIPCHK(launch_render_finalize(c->stream, images, dc, 1.0 / (double)p->n));
    return PRT_OK;
}

int prt_tpp_grad(prt_ctx c, const prt_scene* s, const prt_cameras* cams, prt_paths p, int32_t order,
                 const double* residual, double* grad)
{
    if (!c) return fail(PRT_E_INVALID, "ctx is NULL");
    int rc = check_scene(s);
    if (rc) return rc;
    if ((rc = check_match(s, p))) return rc;
    if (!residual || !grad) return fail(PRT_E_INVALID, "residual/grad is NULL");
    if (order != PRT_ORDER_BY_SIZE && order != PRT_ORDER_BY_ID) return fail(PRT_E_INVALID, "unknown order %d", order);
    DevCams dc;
    if ((rc = make_dev_cams(cams, s, &dc))) return rc;
    DeviceGuard g(c->device);
    const int64_t nu = (int64_t)s->nx * s->ny * s->nz;
    if ((rc = ensure_grids(c, nu))) return rc;
    const int64_t npx = (int64_t)dc.n * dc.W * dc.H;
    if ((rc = ensure_pix(c, npx))) return rc;
    TppView v{};
    if ((rc = tpp_copy(c, p, order, &v))) return rc;
    const GradPlan plan = plan_grad(s->nx, s->ny, s->nz, p->n_slots, 0, c->n_cu, false);
    if ((rc = ensure_scratch(&c->gpart, &c->gpart_bytes, plan.partial_bytes))) return rc;
    TraceArgs a{};
    a.s = make_dev_scene(s);
    a.st = view_of(p);
    a.bc_t = s->beta_cloud;
    a.grid_tot = c->grid_tot;
    a.grid_dlt = c->grid_dlt;
    a.rho = c->pix;
    a.grad = grad;
    a.counters = c->counters;
    {
        TimedScope ts(c, K_PREP);
        if (!plan.lds) HIPCHK(launch_fill(c->stream, grad, nu, 0.0));
        HIPCHK(launch_prep_grids(c->stream, c->fp64, s->beta_cloud, p->beta_ref, s->beta_air, nu, c->grid_tot,
                                 c->grid_dlt));
        HIPCHK(launch_grad_prep(c->stream, residual, c->pix, dc, 1.0 / (double)p->n, nullptr, c->work));
    }
    for (int i = 0; i < plan.n_slabs; ++i) {
        {
            TimedScope ts(c, K_TPP_GRAD);
            HIPCHK(launch_tpp_grad(c->stream, c->fp64, a, dc, v, plan, i, (double*)c->gpart));
        }
        TimedScope ts(c, K_GRAD_REDUCE);
        HIPCHK(launch_grad_reduce(c->stream, plan, s->nx, s->ny, s->nz, i, c->gpart, grad, c->work));
    }
    return PRT_OK;
}

int prt_reweight(prt_ctx c, const prt_scene* s, prt_paths p, double* mean_r, double* ess)
{
    if (!c) return fail(PRT_E_INVALID, "ctx is NULL");
    int rc = check_scene(s);
    if (rc) return rc;
    if ((rc = check_match(s, p))) return rc;
    if (!mean_r || !ess) return fail(PRT_E_INVALID, "mean_r/ess is NULL");
    DeviceGuard g(c->device);
    const int64_t nu = (int64_t)s->nx * s->ny * s->nz;
    if ((rc = ensure_grids(c, nu))) return rc;
    const int64_t nblk = (p->n_slots + 255) / 256;
    if ((rc = ensure_part(c, 2 * nblk))) return rc;
    if (!delta_grid_lds(c->fp64, nu)) {
        TimedScope ts(c, K_PREP);
        HIPCHK(launch_prep_grids(c->stream, c->fp64, s->beta_cloud, p->beta_ref, s->beta_air, nu, c->grid_tot,
                                 c->grid_dlt));
    }
    TraceArgs a{};
    a.s = make_dev_scene(s);
    a.st = view_of(p);
    a.bc_t = s->beta_cloud;
    a.grid_tot = c->grid_tot;
    a.grid_dlt = c->grid_dlt;
    a.partial = c->part;
    a.counters = c->counters;
    int64_t nb = 0;
    {
        TimedScope ts(c, K_REWEIGHT);
        HIPCHK(launch_reweight(c->stream, c->fp64, a, c->n_cu, &nb));
        HIPCHK(launch_sum_pairs(c->stream, c->part, nb, c->dsum));
    }
    // the sums went to pinned host memory
    HIPCHK(hipStreamSynchronize(c->stream));
    const double h[2] = {c->hsum[0], c->hsum[1]};
    *mean_r = h[0] / (double)p->n;
    *ess = h[1] > 0 ? h[0] * h[0] / h[1] : 0.0;
    return PRT_OK;
}

int prt_reweight_noalloc(prt_ctx c, const prt_scene* s, prt_paths p, double* stats)
{
    if (!c) return fail(PRT_E_INVALID, "ctx is NULL");
    int rc = check_scene(s);
    if (rc) return rc;
    if ((rc = check_match(s, p))) return rc;
    if (!stats) return fail(PRT_E_INVALID, "stats is NULL");
    const int64_t nu = (int64_t)s->nx * s->ny * s->nz;
    // scratch layout: the per-workgroup (sum r, sum r^2) pairs, then (for
    // grids larger than the LDS) the field beta_t - beta_ref
    const int64_t nb = reweight_blocks(p->n_slots, c->n_cu);
    const size_t pair_bytes = ((size_t)nb * 2 * sizeof(double) + 255) / 256 * 256;
    const bool grid_lds = delta_grid_lds(c->fp64, nu);
    const size_t need = pair_bytes + (grid_lds ? 0 : (size_t)nu * (c->fp64 ? 8 : 4));
    if (need > PRT_NOALLOC_SCRATCH_BYTES)
        return fail(PRT_E_CAPACITY, "reweight needs %zu bytes of scratch, more than the %u available", need,
                    (unsigned)PRT_NOALLOC_SCRATCH_BYTES);
    unsigned char* base = (unsigned char*)scratch_of(c->device);
    if (!base) return fail(PRT_E_HIP, "no scratch address for device %d", c->device);
    DeviceGuard g(c->device);
    TraceArgs a{};
    a.s = make_dev_scene(s);
    a.st = view_of(p);
    a.bc_t = s->beta_cloud;
    a.grid_dlt = grid_lds ? nullptr : base + pair_bytes;
    a.partial = (double*)base;
    a.counters = c->counters;
    if (!grid_lds)
        HIPCHK(launch_prep_grids(c->stream, c->fp64, s->beta_cloud, p->beta_ref, s->beta_air, nu, nullptr,
                                 base + pair_bytes));
    int64_t used = 0;
    HIPCHK(launch_reweight(c->stream, c->fp64, a, c->n_cu, &used));
    HIPCHK(launch_reweight_stats(c->stream, a.partial, used, (double)p->n, stats));
    return PRT_OK;
}

int prt_loss(prt_ctx c, int64_t n, const double* images, const double* target, double* residual, double* loss)
{
    if (!c) return fail(PRT_E_INVALID, "ctx is NULL");
    if (n < 1 || !images || !target || !residual || !loss) return fail(PRT_E_INVALID, "bad loss arguments");
    DeviceGuard g(c->device);
    int rc = ensure_part(c, 2 * loss_blocks(n));
    if (rc) return rc;
    TimedScope ts(c, K_LOSS);
    HIPCHK(launch_loss(c->stream, n, images, target, residual, c->part, loss));
    return PRT_OK;
}

int prt_adam(prt_ctx c, int64_t n, double* beta, float* beta_f32, const double* grad, double* m, double* v, int32_t t,
             double lr, double b1, double b2, double eps)
{
    if (!c) return fail(PRT_E_INVALID, "ctx is NULL");
    if (n < 1 || !beta || !beta_f32 || !grad || !m || !v) return fail(PRT_E_INVALID, "bad adam arguments");
    if (t < 1 || !finite_all({lr, b1, b2, eps}) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps > 0))
        return fail(PRT_E_INVALID, "bad adam hyper-parameters");
    DeviceGuard g(c->device);
    TimedScope ts(c, K_ADAM);
    HIPCHK(launch_adam(c->stream, n, beta, beta_f32, grad, m, v, lr, b1, b2, eps, 1.0 - std::pow(b1, t),
                       1.0 - std::pow(b2, t)));
    return PRT_OK;
}

int prt_downsample_images(prt_ctx c, const prt_cameras* cams, const double* images, int32_t factor, double* coarse)
{
    if (!c) return fail(PRT_E_INVALID, "ctx is NULL");
    if (!images || !coarse) return fail(PRT_E_INVALID, "images/coarse is NULL");
    if (factor < 1) return fail(PRT_E_INVALID, "factor must be >= 1");
    if (!cams || cams->n < 1 || cams->n > kMaxCams || cams->width < 1 || cams->height < 1 || !cams->f_px)
        return fail(PRT_E_INVALID, "bad cameras");
    if (cams->width % factor || cams->height % factor)
        return fail(PRT_E_INVALID, "image sides %dx%d are not multiples of %d", cams->width, cams->height, factor);
    DevCams dc{};
    dc.n = cams->n;
    dc.W = cams->width;
    dc.H = cams->height;
    for (int d = 0; d < dc.n; ++d) {
        if (!std::isfinite(cams->f_px[d]) || !(cams->f_px[d] > 0)) return fail(PRT_E_INVALID, "bad focal length");
        dc.f[d] = cams->f_px[d];
    }
    DeviceGuard g(c->device);
    HIPCHK(launch_downsample(c->stream, dc, factor, images, coarse));
    return PRT_OK;
}

int prt_volume_errors(prt_ctx c, int64_t n, const double* beta_est, const float* beta_true, double* errors)
{
    if (!c) return fail(PRT_E_INVALID, "ctx is NULL");
    if (n < 1 || !beta_est || !beta_true || !errors) return fail(PRT_E_INVALID, "bad volume-error arguments");
    DeviceGuard g(c->device);
    int rc = ensure_part(c, 3 * volume_error_blocks(n));
    if (rc) return rc;
    HIPCHK(launch_volume_errors(c->stream, n, beta_est, beta_true, c->part, errors));
    return PRT_OK;
}

int prt_space_carve(prt_ctx c, const prt_scene* s, const prt_cameras* cams, const double* images,
                    const double* threshold, double fill_value, uint8_t* mask, float* beta_out)
{
    if (!c) return fail(PRT_E_INVALID, "ctx is NULL");
    int rc = check_scene(s);
    if (rc) return rc;
    if (!images || !threshold || !mask) return fail(PRT_E_INVALID, "images/threshold/mask is NULL");
    if (!std::isfinite(fill_value) || fill_value < 0) return fail(PRT_E_INVALID, "fill_value must be finite and >= 0");
    DevCams dc;
    if ((rc = make_dev_cams(cams, s, &dc))) return rc;
    CarveThresholds t{};
    for (int d = 0; d < dc.n; ++d) {
        if (std::isnan(threshold[d])) return fail(PRT_E_INVALID, "threshold %d is NaN", d);
        t.t[d] = threshold[d];
    }
    DeviceGuard g(c->device);
    HIPCHK(launch_space_carve(c->stream, s->nx, s->ny, s->nz, s->voxel_km, dc, t, images, (float)fill_value, mask,
                              beta_out));
    return PRT_OK;
}

int prt_counters(prt_ctx c, prt_counters_t* out, int reset)
{
    if (!c || !out) return fail(PRT_E_INVALID, "ctx/out is NULL");
    DeviceGuard g(c->device);
    unsigned long long h[4];
    HIPCHK(hipMemcpyAsync(h, c->counters, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    out->voxel_segments = h[0];
    out->local_estimates = h[1];
    out->paths = c->paths_done;
    out->overhead_segments = h[3];
    if (reset) {
        c->paths_done = 0;
        HIPCHK(hipMemsetAsync(c->counters, 0, sizeof h, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
    }
    return PRT_OK;
}

int prt_enable_timing(prt_ctx c, int enable)
{
    if (!c) return fail(PRT_E_INVALID, "ctx is NULL");
    c->timing = enable != 0 ? ~0u : 0u;
    return PRT_OK;
}

int prt_enable_timing_mask(prt_ctx c, uint32_t kernel_mask)
{
    if (!c) return fail(PRT_E_INVALID, "ctx is NULL");
    c->timing = kernel_mask;
    return PRT_OK;
}

int prt_kernel_times(prt_ctx c, double* total_ms, int64_t* launches, int n, int reset)
{
    if (!c) return fail(PRT_E_INVALID, "ctx is NULL");
    DeviceGuard g(c->device);
    HIPCHK(hipStreamSynchronize(c->stream));
    for (auto& t : c->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
            c->total_ms[t.id] += ms;
            c->launches[t.id] += 1;
        }
        c->pool.push_back(t.a);
        c->pool.push_back(t.b);
    }
    c->pending.clear();
    for (int i = 0; i < n && i < K_COUNT; ++i) {
        if (total_ms) total_ms[i] = c->total_ms[i];
        if (launches) launches[i] = c->launches[i];
    }
    if (reset)
        for (int i = 0; i < K_COUNT; ++i) {
            c->total_ms[i] = 0;
            c->launches[i] = 0;
        }
    return K_COUNT;
}

const char* prt_kernel_name(int id) { return (id >= 0 && id < K_COUNT) ? kKernelNames[id] : "unknown"; }

}  // extern "C"

// ------------------------------------------------------ reflectometry

namespace {

bool inside_box(const double* x, double L) { return x[0] > 0 && x[0] < L && x[1] > 0 && x[1] < L && x[2] > 0 && x[2] < L; }

bool outside_spheres(const prt_surface_scene* s, const double* x)
{
    for (int k = 0; k < s->n_spheres; ++k) {
        const double* c = s->center + 3 * k;
        const double d2 = (x[0] - c[0]) * (x[0] - c[0]) + (x[1] - c[1]) * (x[1] - c[1]) + (x[2] - c[2]) * (x[2] - c[2]);
        if (!(d2 > s->radius[k] * s->radius[k])) return false;
    }
    return true;
}

int check_surface_scene(const prt_surface_scene* s)
{
    if (!s) return fail(PRT_E_INVALID, "surface scene is NULL");
    if (!(s->box > 0) || !std::isfinite(s->box)) return fail(PRT_E_INVALID, "box must be finite and > 0");
    if (s->n_spheres < 0 || s->n_spheres > PRT_SURFACE_MAX_SPHERES)
        return fail(PRT_E_CAPACITY, "sphere count %d outside [0, %d]", s->n_spheres, PRT_SURFACE_MAX_SPHERES);
    if (s->phong < -1 || s->phong >= s->n_spheres) return fail(PRT_E_INVALID, "phong index %d out of range", s->phong);
    if (s->max_order < 1 || s->max_order > PRT_MAX_ORDER)
        return fail(PRT_E_CAPACITY, "max_order %d outside [1, %d]", s->max_order, PRT_MAX_ORDER);
    for (int k = 0; k < 6; ++k)
        if (!(s->wall_albedo[k] >= 0 && s->wall_albedo[k] <= 1)) return fail(PRT_E_INVALID, "wall albedo outside [0, 1]");
    if (!(s->intensity > 0) || !std::isfinite(s->intensity)) return fail(PRT_E_INVALID, "intensity must be finite and > 0");
    if (s->n_spheres > 0 && (!s->center || !s->radius || !s->albedo))
        return fail(PRT_E_INVALID, "sphere arrays must be non-NULL");
    for (int k = 0; k < s->n_spheres; ++k) {
        const double* c = s->center + 3 * k;
        const double r = s->radius[k];
        if (!finite_all({c[0], c[1], c[2], r}) || !(r > 0)) return fail(PRT_E_INVALID, "sphere %d: bad centre/radius", k);
        for (int a = 0; a < 3; ++a)
            if (!(c[a] - r >= 0 && c[a] + r <= s->box)) return fail(PRT_E_INVALID, "sphere %d leaves the box", k);
        if (!(s->albedo[k] >= 0 && s->albedo[k] <= 1)) return fail(PRT_E_INVALID, "sphere %d: albedo outside [0, 1]", k);
    }
    if (!finite_all({s->light[0], s->light[1], s->light[2]}) || !inside_box(s->light, s->box) ||
        !outside_spheres(s, s->light))
        return fail(PRT_E_INVALID, "the light must lie strictly inside the box and outside every sphere");
    return PRT_OK;
}

int check_theta_ref(const double* t)
{
    if (!t) return fail(PRT_E_INVALID, "theta_ref is NULL");
    if (!(t[0] >= 0 && t[0] < 1)) return fail(PRT_E_INVALID, "theta_ref kappa_s must lie in [0, 1)");
    if (!(t[1] >= 0 && t[1] <= 1e4)) return fail(PRT_E_INVALID, "theta_ref gamma must lie in [0, 1e4]");
    return PRT_OK;
}

int make_surface_cams(const prt_cameras* c, const prt_surface_scene* s, DevCams* out)
{
    if (!c) return fail(PRT_E_INVALID, "cameras is NULL");
    if (c->n < 1 || c->n > PRT_MAX_CAMERAS) return fail(PRT_E_CAPACITY, "camera count %d outside [1, %d]", c->n, PRT_MAX_CAMERAS);
    if (c->width < 1 || c->height < 1 || c->width > 16384 || c->height > 16384)
        return fail(PRT_E_INVALID, "image size must be in [1, 16384]");
    if (!c->pos || !c->rot || !c->f_px) return fail(PRT_E_INVALID, "camera arrays must be non-NULL");
    std::memset(out, 0, sizeof *out);
    out->n = c->n;
    out->W = c->width;
    out->H = c->height;
    for (int d = 0; d < c->n; ++d) {
        const double* q = c->pos + 3 * d;
        if (!finite_all({q[0], q[1], q[2]}) || !inside_box(q, s->box) || !outside_spheres(s, q))
            return fail(PRT_E_INVALID, "camera %d must lie strictly inside the box and outside every sphere", d);
        for (int k = 0; k < 3; ++k) out->pos[d][k] = q[k];
        for (int k = 0; k < 9; ++k) {
            if (!std::isfinite(c->rot[9 * d + k])) return fail(PRT_E_INVALID, "non-finite camera rotation");
            out->rot[d][k] = c->rot[9 * d + k];
        }
        if (!(c->f_px[d] > 0) || !std::isfinite(c->f_px[d])) return fail(PRT_E_INVALID, "focal length must be > 0");
        out->f[d] = c->f_px[d];
    }
    return PRT_OK;
}

void free_surface(prt_surface_paths p)
{
    if (!p) return;
    DeviceGuard g(p->device);
    (void)hipDeviceSynchronize();
    for (void* q : {(void*)p->B, (void*)p->pos, (void*)p->sid, (void*)p->tv, (void*)p->tc, (void*)p->pix,
                    (void*)p->theta_ref, (void*)p->sph, (void*)p->part, (void*)p->omega, (void*)p->work})
        (void)hipFree(q);
    delete p;
}

SurfStore view_of(prt_surface_paths p)
{
    SurfStore v{};
    v.n = p->n;
    v.B = p->B;
    v.pos = p->pos;
    v.sid = p->sid;
    v.tv = p->tv;
    v.tc = p->tc;
    v.pix = p->pix;
    v.theta_ref = p->theta_ref;
    v.omega = p->omega;
    v.work = p->work;
    return v;
}

bool same_cams(const DevCams& a, const DevCams& b)
{
    if (a.n != b.n || a.W != b.W || a.H != b.H || a.outside != b.outside) return false;
    for (int d = 0; d < a.n; ++d) {
        if (a.f[d] != b.f[d]) return false;
        for (int k = 0; k < 3; ++k)
            if (a.pos[d][k] != b.pos[d][k]) return false;
        for (int k = 0; k < 9; ++k)
            if (a.rot[d][k] != b.rot[d][k]) return false;
    }
    return true;
}

// Buffers for n paths of the scene's order and the cameras (reused when
// large enough), and the scene's spheres and the cameras' pixel solid angles
// on the device (uploaded or recomputed only when they change, so that a
// redraw of the same scene costs no host round trip).
int surface_prepare(prt_ctx c, prt_surface_paths p, const prt_surface_scene* s, const DevCams& dc, int64_t n)
{
    const int M = s->max_order;
    double h[kSphStride * kMaxSpheres];
    for (int k = 0; k < s->n_spheres; ++k) {
        for (int a = 0; a < 3; ++a) h[kSphStride * k + a] = s->center[3 * k + a];
        h[kSphStride * k + 3] = s->radius[k];
        h[kSphStride * k + 4] = s->albedo[k];
        h[kSphStride * k + 5] = 1.0 / s->radius[k];
    }
    const size_t sph_bytes = (size_t)kSphStride * s->n_spheres * sizeof(double);
    const bool grow_rows = n > p->cap || M > p->M || dc.n > p->cap_cams || !p->B;
    const bool new_sph = !p->sph || p->n_sph != s->n_spheres || std::memcmp(p->sph_host, h, sph_bytes) != 0;
    const int64_t npx = (int64_t)dc.n * dc.W * dc.H;
    const bool new_cams = !p->omega_valid || npx > p->cap_omega || !same_cams(p->cams, dc);
    // earlier calls on the stream may still read the buffers being replaced
    if (grow_rows || new_sph || new_cams) HIPCHK(hipStreamSynchronize(c->stream));
    if (grow_rows) {
        for (void** q : {(void**)&p->B, (void**)&p->pos, (void**)&p->sid, (void**)&p->tv, (void**)&p->tc,
                         (void**)&p->pix}) {
            (void)hipFree(*q);
            *q = nullptr;
        }
        const int64_t cap = std::max<int64_t>(n, p->cap);
        const int Mc = std::max(M, p->M), nc = std::max(dc.n, p->cap_cams);
        const size_t rows = (size_t)Mc * (size_t)cap, crows = rows * (size_t)nc;
        int rc;
        if ((rc = dalloc(&p->B, (size_t)cap)) || (rc = dalloc(&p->pos, rows)) || (rc = dalloc(&p->sid, rows)) ||
            (rc = dalloc(&p->tv, rows)) || (rc = dalloc(&p->tc, crows)) || (rc = dalloc(&p->pix, crows))) {
            p->cap = 0;
            return rc;
        }
        p->cap = cap;
        p->M = Mc;
        p->cap_cams = nc;
    }
    int rc;
    if (!p->theta_ref && (rc = dalloc(&p->theta_ref, 2))) return rc;
    if (!p->sph && (rc = dalloc(&p->sph, (size_t)kSphStride * kMaxSpheres))) return rc;
    if (new_sph) {
        // (a synchronous copy of a host array that the caller may free on return)
        p->n_sph = -1;
        if (s->n_spheres > 0) HIPCHK(hipMemcpy(p->sph, h, sph_bytes, hipMemcpyHostToDevice));
        std::memcpy(p->sph_host, h, sph_bytes);
        p->n_sph = s->n_spheres;
    }
    if (new_cams) {
        p->omega_valid = false;
        if ((rc = grow(&p->omega, &p->cap_omega, npx))) return rc;
        HIPCHK(launch_surf_omega(c->stream, dc, p->omega));
        p->omega_valid = true;
    }
    if (!p->work && (rc = dalloc(&p->work, 2))) return rc;
    HIPCHK(hipMemsetAsync(p->work, 0, 2 * sizeof(unsigned long long), c->stream));
    p->n = n;
    p->M = M;
    p->n_cams = dc.n;
    p->cams = dc;
    SurfScene& d = p->scene;
    d.box = s->box;
    for (int k = 0; k < 6; ++k) d.wall_albedo[k] = s->wall_albedo[k];
    for (int k = 0; k < 3; ++k) d.light[k] = s->light[k];
    d.intensity = s->intensity;
    d.n_spheres = s->n_spheres;
    d.phong = s->phong;
    d.max_order = M;
    d.sph = p->sph;
    return PRT_OK;
}

// The rows of the store use M = the scene's max_order as stride: a store
// whose buffers were sized for a larger order keeps M rows per order anyway.
int surface_draw(prt_ctx c, prt_surface_paths p, uint64_t seed, const DrawTheta& th)
{
    TimedScope ts(c, K_SURF_SAMPLE);
    HIPCHK(launch_surf_draw(c->stream, p->scene, p->cams, view_of(p), seed, 0, th, c->n_cu));
    return PRT_OK;
}

int ensure_surface_part(prt_surface_paths p, size_t n)
{
    if (p->part_n >= n) return PRT_OK;
    (void)hipFree(p->part);
    p->part = nullptr;
    p->part_n = 0;
    int rc = dalloc(&p->part, n);
    if (rc == PRT_OK) p->part_n = n;
    return rc;
}

int check_surface_call(prt_ctx c, prt_surface_paths p)
{
    if (!c) return fail(PRT_E_INVALID, "ctx is NULL");
    if (!p) return fail(PRT_E_INVALID, "paths is NULL");
    if (p->device != c->device) return fail(PRT_E_MISMATCH, "store and context are on different devices");
    return PRT_OK;
}

}  // namespace

extern "C" {

int prt_surface_sample(prt_ctx c, const prt_surface_scene* s, const prt_cameras* cams, const double* theta_ref,
                       uint64_t seed, int64_t n_paths, prt_surface_paths* out)
{
    if (!c) return fail(PRT_E_INVALID, "ctx is NULL");
    if (!out) return fail(PRT_E_INVALID, "out is NULL");
    *out = nullptr;
    prt_surface_paths p = new prt_surface_paths_s();
    p->device = c->device;
    int rc = prt_surface_resample(c, p, s, cams, theta_ref, seed, n_paths);
    if (rc) {
        free_surface(p);
        return rc;
    }
    *out = p;
    return PRT_OK;
}

int prt_surface_resample(prt_ctx c, prt_surface_paths p, const prt_surface_scene* s, const prt_cameras* cams,
                         const double* theta_ref, uint64_t seed, int64_t n_paths)
{
    int rc = check_surface_call(c, p);
    if (rc || (rc = check_surface_scene(s)) || (rc = check_theta_ref(theta_ref))) return rc;
    if (n_paths < 1 || n_paths > ((int64_t)1 << 40)) return fail(PRT_E_INVALID, "n_paths must be in [1, 2^40]");
    DevCams dc;
    if ((rc = make_surface_cams(cams, s, &dc))) return rc;
    DeviceGuard g(c->device);
    if ((rc = surface_prepare(c, p, s, dc, n_paths))) return rc;
    return surface_draw(c, p, seed, DrawTheta{theta_ref[0], theta_ref[1], nullptr});
}

int prt_surface_resample_device(prt_ctx c, prt_surface_paths p, const prt_surface_scene* s,
                                const prt_cameras* cams, const double* theta_ref, uint64_t seed, int64_t n_paths)
{
    int rc = check_surface_call(c, p);
    if (rc || (rc = check_surface_scene(s))) return rc;
    if (!theta_ref) return fail(PRT_E_INVALID, "theta_ref is NULL");
    if (n_paths < 1 || n_paths > ((int64_t)1 << 40)) return fail(PRT_E_INVALID, "n_paths must be in [1, 2^40]");
    DevCams dc;
    if ((rc = make_surface_cams(cams, s, &dc))) return rc;
    DeviceGuard g(c->device);
    if ((rc = surface_prepare(c, p, s, dc, n_paths))) return rc;
    return surface_draw(c, p, seed, DrawTheta{0.0, 0.0, theta_ref});
}

int prt_surface_import(prt_ctx c, const prt_surface_scene* s, const prt_cameras* cams, const double* theta_ref,
                       int64_t n_paths, const int32_t* B, const double* pos, const int32_t* sid,
                       prt_surface_paths* out)
{
    if (!c) return fail(PRT_E_INVALID, "ctx is NULL");
    if (!out) return fail(PRT_E_INVALID, "out is NULL");
    *out = nullptr;
    int rc;
    if ((rc = check_surface_scene(s)) || (rc = check_theta_ref(theta_ref))) return rc;
    if (n_paths < 1 || n_paths > ((int64_t)1 << 34)) return fail(PRT_E_INVALID, "n_paths must be in [1, 2^34]");
    if (!B || !pos || !sid) return fail(PRT_E_INVALID, "path arrays must be non-NULL");
    const int M = s->max_order;
    const int n_ids = 6 + s->n_spheres;
    for (int64_t i = 0; i < n_paths; ++i) {
        if (B[i] < 0 || B[i] > M) return fail(PRT_E_INVALID, "path %lld: B outside [0, max_order]", (long long)i);
        for (int b = 0; b < B[i]; ++b) {
            const int32_t id = sid[i * M + b];
            const double* x = pos + (i * M + b) * 3;
            if (id < 0 || id >= n_ids || !finite_all({x[0], x[1], x[2]}))
                return fail(PRT_E_INVALID, "path %lld vertex %d: bad surface id or position", (long long)i, b);
        }
    }
    DevCams dc;
    if ((rc = make_surface_cams(cams, s, &dc))) return rc;
    DeviceGuard g(c->device);
    prt_surface_paths p = new prt_surface_paths_s();
    p->device = c->device;
    if ((rc = surface_prepare(c, p, s, dc, n_paths)) ||
        (hipMemcpy(p->theta_ref, theta_ref, 2 * sizeof(double), hipMemcpyHostToDevice) != hipSuccess &&
         (rc = fail(PRT_E_HIP, "copy of theta_ref failed")))) {
        free_surface(p);
        return rc;
    }
    // rows per vertex order on the host, then one copy each
    std::vector<int32_t> hsid((size_t)M * n_paths, -1);
    std::vector<double4> hpos((size_t)M * n_paths);
    for (int64_t i = 0; i < n_paths; ++i)
        for (int b = 0; b < M; ++b) {
            const size_t r = (size_t)b * n_paths + i;
            if (b < B[i]) {
                const double* x = pos + (i * M + b) * 3;
                hpos[r] = make_double4(x[0], x[1], x[2], 0.0);
                hsid[r] = sid[i * M + b];
            } else {
                hpos[r] = make_double4(0.0, 0.0, 0.0, 0.0);
            }
        }
    if (hipMemcpy(p->B, B, (size_t)n_paths * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->pos, hpos.data(), hpos.size() * sizeof(double4), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->sid, hsid.data(), hsid.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) {
        free_surface(p);
        return fail(PRT_E_HIP, "copy of the imported paths failed");
    }
    {
        TimedScope ts(c, K_SURF_TAPE);
        hipError_t e = launch_surf_tape(c->stream, p->scene, p->cams, view_of(p), c->n_cu);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) {
            free_surface(p);
            return fail(PRT_E_HIP, "surface tape: %s", hipGetErrorString(e));
        }
    }
    *out = p;
    return PRT_OK;
}

int prt_surface_export(prt_ctx c, prt_surface_paths p, int32_t* B, double* pos, int32_t* sid)
{
    int rc = check_surface_call(c, p);
    if (rc) return rc;
    if (!B || !pos || !sid) return fail(PRT_E_INVALID, "output arrays must be non-NULL");
    DeviceGuard g(c->device);
    HIPCHK(hipStreamSynchronize(c->stream));
    const int64_t n = p->n;
    const int M = p->M;
    std::vector<double4> hpos((size_t)M * n);
    std::vector<int32_t> hsid((size_t)M * n);
    HIPCHK(hipMemcpy(B, p->B, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(hpos.data(), p->pos, hpos.size() * sizeof(double4), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(hsid.data(), p->sid, hsid.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < n; ++i)
        for (int b = 0; b < M; ++b) {
            const size_t r = (size_t)b * n + i;
            double* x = pos + (i * M + b) * 3;
            const bool in = b < B[i];
            x[0] = in ? hpos[r].x : 0.0;
            x[1] = in ? hpos[r].y : 0.0;
            x[2] = in ? hpos[r].z : 0.0;
            sid[i * M + b] = in ? hsid[r] : -1;
        }
    return PRT_OK;
}

int prt_surface_info(prt_surface_paths p, int64_t* n_paths, int32_t* max_order)
{
    if (!p) return fail(PRT_E_INVALID, "paths is NULL");
    if (n_paths) *n_paths = p->n;
    if (max_order) *max_order = p->M;
    return PRT_OK;
}

int prt_surface_work(prt_ctx c, prt_surface_paths p, uint64_t* sphere_tests, uint64_t* vertices)
{
    int rc = check_surface_call(c, p);
    if (rc) return rc;
    DeviceGuard g(c->device);
    HIPCHK(hipStreamSynchronize(c->stream));
    unsigned long long h[2] = {0, 0};
    HIPCHK(hipMemcpy(h, p->work, sizeof h, hipMemcpyDeviceToHost));
    if (sphere_tests) *sphere_tests = h[0];
    if (vertices) *vertices = h[1];
    return PRT_OK;
}

int prt_surface_render(prt_ctx c, prt_surface_paths p, const double* theta, double* images)
{
    int rc = check_surface_call(c, p);
    if (rc) return rc;
    if (!theta || !images) return fail(PRT_E_INVALID, "theta/images is NULL");
    DeviceGuard g(c->device);
    const int npx = p->cams.W * p->cams.H;
    const int np = surf_render_parts(p->n, p->n_cams, npx, c->n_cu);
    if ((rc = ensure_surface_part(p, std::max<size_t>((size_t)np * p->n_cams * npx, 2 * (size_t)surf_pair_blocks(p->n, c->n_cu)))))
        return rc;
    const double w0 = 4.0 * kPi * p->scene.intensity / (double)p->n;
    TimedScope ts(c, K_SURF_RENDER);
    HIPCHK(launch_surf_render(c->stream, view_of(p), p->n_cams, npx, w0, theta, images, p->part, c->n_cu));
    return PRT_OK;
}

int prt_surface_grad(prt_ctx c, prt_surface_paths p, const double* theta, const double* residual, double* grad)
{
    int rc = check_surface_call(c, p);
    if (rc) return rc;
    if (!theta || !residual || !grad) return fail(PRT_E_INVALID, "theta/residual/grad is NULL");
    DeviceGuard g(c->device);
    const int npx = p->cams.W * p->cams.H;
    if ((rc = ensure_surface_part(p, 2 * (size_t)surf_pair_blocks(p->n, c->n_cu)))) return rc;
    const double w0 = 4.0 * kPi * p->scene.intensity / (double)p->n;
    TimedScope ts(c, K_SURF_GRAD);
    HIPCHK(launch_surf_grad(c->stream, view_of(p), p->n_cams, npx, w0, theta, residual, p->part, grad, c->n_cu));
    return PRT_OK;
}

int prt_surface_reweight(prt_ctx c, prt_surface_paths p, const double* theta, double* stats)
{
    int rc = check_surface_call(c, p);
    if (rc) return rc;
    if (!theta || !stats) return fail(PRT_E_INVALID, "theta/stats is NULL");
    DeviceGuard g(c->device);
    if ((rc = ensure_surface_part(p, 2 * (size_t)surf_pair_blocks(p->n, c->n_cu)))) return rc;
    TimedScope ts(c, K_SURF_REWEIGHT);
    HIPCHK(launch_surf_reweight(c->stream, view_of(p), theta, p->part, stats, c->n_cu));
    return PRT_OK;
}

int prt_surface_adam(prt_ctx c, double* theta, const double* grad, double* m, double* v, int32_t t, double lr_kappa,
                     double lr_gamma, double b1, double b2, double eps)
{
    if (!c) return fail(PRT_E_INVALID, "ctx is NULL");
    if (!theta || !grad || !m || !v) return fail(PRT_E_INVALID, "bad adam arguments");
    if (t < 1 || !finite_all({lr_kappa, lr_gamma, b1, b2, eps}) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) ||
        !(eps > 0) || lr_kappa < 0 || lr_gamma < 0)
        return fail(PRT_E_INVALID, "bad adam hyper-parameters");
    DeviceGuard g(c->device);
    TimedScope ts(c, K_SURF_ADAM);
    HIPCHK(launch_surf_adam(c->stream, theta, grad, m, v, lr_kappa, lr_gamma, b1, b2, eps, 1.0 - std::pow(b1, t),
                            1.0 - std::pow(b2, t)));
    return PRT_OK;
}

void prt_surface_destroy(prt_surface_paths p) { free_surface(p); }

}  // extern "C"
