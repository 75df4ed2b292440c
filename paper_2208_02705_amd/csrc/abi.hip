// Host side of the C ABI (include/r360.h): argument checks, object
// lifetimes, workspace carve-up and the launch sequences of the hot path.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <vector>

#include "r360_internal.h"

namespace r360 {
size_t pack_bytes16(int H);
size_t bias_floats(int H);
inline size_t packT_bytes16(int H) {
    return (size_t)(H == 32 ? PackGeom<32>::FRAGS_T : PackGeom<64>::FRAGS_T) * WAVE * 16;
}
}

using namespace r360;

namespace {

thread_local char g_err[512] = "";

r360_status hip_fail(const char* where, hipError_t e) {
    std::snprintf(g_err, sizeof(g_err), "%s: %s (%d)", where, hipGetErrorString(e), (int)e);
    return R360_EHIP;
}
r360_status inval(const char* what) {
    std::snprintf(g_err, sizeof(g_err), "invalid argument: %s", what);
    return R360_EINVAL;
}
#define R360_TRY(where, expr)                         \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) return hip_fail(where, e_); \
    } while (0)

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Per-stage event timing (r360_profile_enable / r360_profile_read).
struct StageEvents { int stage; hipEvent_t a, b; };
bool g_prof = false;
std::vector<StageEvents> g_events;

struct StageTimer {
    hipStream_t st;
    StageEvents ev{-1, nullptr, nullptr};
    StageTimer(int stage, hipStream_t s) : st(s) {
        if (!g_prof) return;
        ev.stage = stage;
        if (hipEventCreate(&ev.a) != hipSuccess || hipEventCreate(&ev.b) != hipSuccess) { ev.stage = -1; return; }
        (void)hipEventRecord(ev.a, st);
    }
    ~StageTimer() {
        if (ev.stage < 0) return;
        (void)hipEventRecord(ev.b, st);
        g_events.push_back(ev);
    }
};
#define R360_STAGE(k, st) StageTimer timer_##k(k, st)
inline size_t al(size_t x) { return (x + 255) & ~size_t(255); }

bool pow2(float v) {
    if (!(v > 0.0f) || !std::isfinite(v)) return false;
    int e;
    return std::frexp(v, &e) == 0.5f;
}

int64_t field_params(int h, int Lx, int Ld) {
    const int64_t dx = 3 + 6 * Lx, dd = 3 + 6 * Ld;
    return h * dx + h + (int64_t)h * h + h + h + 1 + (int64_t)h * h + h + h * (h + dd) + h + 3 * (int64_t)h + 3;
}

r360_status check_opts(const r360_render_opts* o, bool allow_fp64) {
    if (!o) return inval("opts is NULL");
    if (o->max_samples < 1 || o->max_samples > 256) return inval("max_samples outside [1, 256]");
    if (o->samples_per_voxel < 0 || o->samples_per_voxel > 64) return inval("samples_per_voxel outside [0, 64]");
    if (std::isnan(o->near_) || std::isnan(o->far_)) return inval("near/far is NaN");
    if (!(o->term_eps >= 0.0f && o->term_eps <= 1.0f)) return inval("term_eps outside [0, 1]");
    if (o->term_eps > 0.0f && (o->term_after < 1 || o->term_after >= o->max_samples))
        return inval("term_after outside [1, max_samples) with term_eps > 0");
    if (o->precision < R360_FP32 || o->precision > R360_FP64_GRADCHECK) return inval("unknown precision");
    if (o->precision == R360_FP64_GRADCHECK && !allow_fp64) {
        std::snprintf(g_err, sizeof(g_err), "FP64 is only accepted by the gradient-check entry points");
        return R360_EUNSUPPORTED;
    }
    return R360_OK;
}

}  // namespace

namespace r360 {

int64_t sample_cap(int64_t N, int max_samples) { return (N + 63) / 64 * 64 * (int64_t)max_samples; }

Workspace carve(void* base, int64_t N, int max_samples, int F, int64_t P, bool train) {
    Workspace w{};
    const int64_t cap = sample_cap(N, max_samples);
    char* p = static_cast<char*>(base);
    size_t off = 0;
    auto take_always = [&](size_t bytes) -> char* {
        char* q = p ? p + off : nullptr;
        off += al(bytes);
        return q;
    };
    auto take = [&](size_t bytes) -> char* { return take_always(bytes); };
    auto take_train = [&](size_t bytes) -> char* { return train ? take_always(bytes) : nullptr; };
    w.ray_off = (int32_t*)take((N + 1) * 4);
    w.o = (float*)take(3 * N * 4);
    w.d = (float*)take(3 * N * 4);
    w.t_mid = (float*)take(cap * 4);
    w.delta = (float*)take(cap * 4);
    w.ray = (int32_t*)take(cap * 4);
    w.field = (int32_t*)take(cap * 4);
    w.perm = (int32_t*)take(cap * 4);
    w.sigma = (float*)take(cap * 4);
    w.rgb = (float*)take(3 * cap * 4);
    w.dsigma = (float*)take_train(cap * 4);
    w.drgb = (float*)take_train(3 * cap * 4);
    w.scan = (int32_t*)take(((N + SCAN_TILE - 1) / SCAN_TILE + 1) * 4);
    w.hist = (int32_t*)take((size_t)F * route_waves(F) * 4);
    w.field_start = (int32_t*)take((F + 1) * 4);
    w.chunk_start = (int32_t*)take_train((F + 1) * 4);
    w.dw_part = (float*)take_train((size_t)DW_SLOTS * P * 4);
    w.blk_fields = (int32_t*)take_train(DW_SLOTS * 4);
    w.misc = (int32_t*)take(256 * 4);
    w.loss_part = (float*)take_train(((N + 255) / 256) * 4);
    w.ray_rgb = (float*)take_train(3 * N * 4);
    w.ray_grad = (float*)take_train(3 * N * 4);
    w.N = N;
    w.cap = cap;
    w.slots = slot_map(max_samples);
    w.bytes = off;
    return w;
}

DdaParams dda_params(const r360_scene* s, const r360_render_opts* o) {
    DdaParams p;
    p.labels = s->labels;
    p.n0 = s->grid.n[0]; p.n1 = s->grid.n[1]; p.n2 = s->grid.n[2];
    p.lo0 = s->grid.lo[0]; p.lo1 = s->grid.lo[1]; p.lo2 = s->grid.lo[2];
    p.voxel = s->grid.voxel;
    p.inv_voxel = 1.0f / s->grid.voxel;
    p.near_ = o->near_;
    p.far_ = o->far_;
    p.max_samples = o->max_samples;
    p.spv = o->samples_per_voxel > 1 ? o->samples_per_voxel : 1;
    p.skip = 0;
    return p;
}

}  // namespace r360

namespace {

// Validates the common render arguments and carves the workspace.
r360_status prepare(const r360_scene* s, int64_t N, const r360_render_opts* opts, void* ws, size_t ws_bytes,
                    bool allow_fp64, Workspace* w, bool allow_term = false) {
    if (!s) return inval("scene is NULL");
    r360_status st = check_opts(opts, allow_fp64);
    if (st != R360_OK) return st;
    if (opts->term_eps > 0.0f && !allow_term) {
        std::snprintf(g_err, sizeof(g_err), "early ray termination applies to the render entry points only");
        return R360_EUNSUPPORTED;
    }
    if (N <= 0 || N > (int64_t(1) << 30)) return inval("N must be in [1, 2^30]");
    if (sample_cap(N, opts->max_samples) >= (int64_t(1) << 30))
        return inval("N * max_samples must stay below 2^30; split the rays");
    if (!ws) return inval("workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) & 255) return inval("workspace must be 256-byte aligned");
    *w = carve(ws, N, opts->max_samples, s->mlp.n_fields, s->P);
    if (ws_bytes < w->bytes) {
        std::snprintf(g_err, sizeof(g_err), "workspace has %zu bytes, needs %zu", ws_bytes, w->bytes);
        return R360_EWORKSPACE;
    }
    return R360_OK;
}

r360_status render_terminated(const r360_scene* s, const RaySource& src, int64_t N, const r360_render_opts* opts,
                              float* rgb, float* depth, float* opacity, Workspace& w, hipStream_t st);

// target / grad_rgb (training): the compositing also writes the loss gradient
// and the loss partials.
r360_status render_common(const r360_scene* s, const RaySource& src, int64_t N, const r360_render_opts* opts,
                          float* rgb, float* depth, float* opacity, Workspace& w, hipStream_t st,
                          const float* target = nullptr, float* grad_rgb = nullptr) {
    w.ro = src.mode == RAYS_GIVEN ? src.o : w.o;
    w.rd = src.mode == RAYS_GIVEN ? src.d : w.d;
    if (opts->term_eps > 0.0f) return render_terminated(s, src, N, opts, rgb, depth, opacity, w, st);
    const DdaParams p = dda_params(s, opts);
    bool counted = false;
    {
        R360_STAGE(0, st);
        R360_TRY("sample", launch_trace(src, p, N, w, s->mlp.n_fields, &counted, st));
    }
    {
        R360_STAGE(1, st);
        R360_TRY("route", launch_route(w, s->mlp.n_fields, counted, st));
    }
    {
        R360_STAGE(2, st);
        R360_TRY("mlp forward", launch_mlp_forward(s, w, opts->precision, st));
    }
    {
        R360_STAGE(3, st);
        R360_TRY("composite", launch_composite_slots(w, N, rgb, depth, opacity, st, nullptr, target, grad_rgb));
    }
    return R360_OK;
}

// Early ray termination in two passes. Pass 1 renders the first K =
// term_after samples of every ray and keeps the compositing sums; the rays
// that emitted all K and whose transmittance expf(-S) is still at least
// term_eps are listed, and pass 2 walks them again, emits samples K onwards
// (the same FP32 walk, so the same samples) and continues the sums. A
// continued ray's result is therefore the one-pass result; a stopped ray's is
// that of its first K samples. Scratch (free during a render): the sums in
// drgb ([6][N] <= 3 cap floats, as max_samples >= 2), the list in `ray`, the
// continued rays in ray_rgb / ray_grad, the count in misc. Stage timers cover
// pass 1.
r360_status render_terminated(const r360_scene* s, const RaySource& src, int64_t N, const r360_render_opts* opts,
                              float* rgb, float* depth, float* opacity, Workspace& w, hipStream_t st) {
    const int F = s->mlp.n_fields, K = opts->term_after;
    float* state = w.drgb;
    int32_t* list = w.ray;
    int32_t* n2dev = w.misc;
    {
        DdaParams p = dda_params(s, opts);
        p.max_samples = K;
        Workspace w1 = w;
        w1.slots = slot_map(K);
        bool counted = false;
        {
            R360_STAGE(0, st);
            R360_TRY("sample", launch_trace(src, p, N, w1, F, &counted, st));
        }
        {
            R360_STAGE(1, st);
            R360_TRY("route", launch_route(w1, F, counted, st));
        }
        {
            R360_STAGE(2, st);
            R360_TRY("mlp forward", launch_mlp_forward(s, w1, opts->precision, st));
        }
        {
            R360_STAGE(3, st);
            R360_TRY("composite", launch_composite_slots(w1, N, rgb, depth, opacity, st, state));
        }
        R360_TRY("termination", launch_term_select(w1, N, K, state + 5 * N, opts->term_eps, list, n2dev, st));
    }
    int32_t n2 = 0;
    R360_TRY("termination", hipMemcpyAsync(&n2, n2dev, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    R360_TRY("termination", hipStreamSynchronize(st));
    if (n2 == 0) return R360_OK;
    float* o2 = w.ray_rgb;
    float* d2 = w.ray_grad;
    R360_TRY("termination", launch_term_gather(n2, list, w.ro, w.rd, N, o2, d2, st));
    DdaParams p = dda_params(s, opts);
    p.skip = K;
    RaySource src2{};
    src2.mode = RAYS_GIVEN;
    src2.o = o2;
    src2.d = d2;
    Workspace w2 = w;
    w2.N = n2;
    w2.slots = slot_map(opts->max_samples - K);
    w2.ro = o2;
    w2.rd = d2;
    bool counted = false;
    {
        R360_STAGE(0, st);
        R360_TRY("sample", launch_trace(src2, p, n2, w2, F, &counted, st));
    }
    {
        R360_STAGE(1, st);
        R360_TRY("route", launch_route(w2, F, counted, st));
    }
    {
        R360_STAGE(2, st);
        R360_TRY("mlp forward", launch_mlp_forward(s, w2, opts->precision, st));
    }
    {
        R360_STAGE(3, st);
        R360_TRY("composite", launch_composite_continue(w2, list, N, state, rgb, depth, opacity, st));
    }
    return R360_OK;
}

bool valid_c2w(const float* c) {
    if (!c) return false;
    for (int i = 0; i < 12; ++i)
        if (!std::isfinite(c[i])) return false;
    return true;
}

}  // namespace

// ---- allocation-free render: the workspace is a file-scope device array ----
// In host code `scratch` names a host-side stand-in, not device memory: the
// device address (one copy per GPU) comes from hipGetSymbolAddress with that
// GPU current, taken once per device and kept in g_scratch_dev.
static __device__ __align__(256) unsigned char scratch[R360_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kScratchDevices] = {};

r360_status scratch_of_current_device(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail("hipGetDevice", e);
    if (dev < 0 || dev >= kScratchDevices) return inval("device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail("hipGetSymbolAddress(scratch)", e);
        if (!p || (reinterpret_cast<uintptr_t>(p) & 255)) return inval("scratch array not 256-byte aligned");
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return R360_OK;
}
}  // namespace

extern "C" {

int64_t r360_field_params(int32_t hidden, int32_t L_xyz, int32_t L_dir) {
    if (hidden <= 0 || L_xyz < 0 || L_dir < 0) return -1;
    return field_params(hidden, L_xyz, L_dir);
}

r360_status r360_scene_create(const r360_grid_desc* grid, const float* occ_prob, const int32_t* field_map,
                              const r360_mlp_desc* mlp, const float* weights, void* stream, r360_scene** out) {
    if (!out) return inval("out is NULL");
    *out = nullptr;
    if (!grid || !mlp || !occ_prob || !field_map || !weights) return inval("NULL pointer");
    for (int a = 0; a < 3; ++a) {
        if (grid->n[a] < 1 || grid->n[a] > 4096) return inval("grid size outside [1, 4096]");
        if (!std::isfinite(grid->lo[a])) return inval("grid corner not finite");
    }
    if (!pow2(grid->voxel)) return inval("voxel edge must be a positive power of two");
    if ((int64_t)grid->n[0] * grid->n[1] * grid->n[2] >= (int64_t(1) << 31)) return inval("grid has 2^31 voxels or more");
    if (std::isnan(grid->threshold)) return inval("threshold is NaN");
    if (mlp->n_fields < 1 || mlp->n_fields > 16384) return inval("n_fields outside [1, 16384]");
    if (!(mlp->half_extent > 0.0f) || !std::isfinite(mlp->half_extent)) return inval("half_extent must be positive");
    if (mlp->hidden != 32 && mlp->hidden != 64) {
        std::snprintf(g_err, sizeof(g_err), "hidden width %d unsupported (32 or 64)", mlp->hidden);
        return R360_EUNSUPPORTED;
    }
    if (mlp->L_xyz != LXYZ || mlp->L_dir != LDIR) {
        std::snprintf(g_err, sizeof(g_err), "encoding lengths must be L_xyz = 10, L_dir = 4");
        return R360_EUNSUPPORTED;
    }
    const int64_t nvox = (int64_t)grid->n[0] * grid->n[1] * grid->n[2];
    r360_scene* s = new (std::nothrow) r360_scene();
    if (!s) return R360_ENOMEM;
    s->grid = *grid;
    s->mlp = *mlp;
    s->P = field_params(mlp->hidden, mlp->L_xyz, mlp->L_dir);
    (void)hipGetDevice(&s->device);
    const int F = mlp->n_fields, H = mlp->hidden;
    bool ok = hipMalloc((void**)&s->labels, nvox * sizeof(int16_t)) == hipSuccess;
    ok = ok && hipMalloc(&s->pack16_bf, F * pack_bytes16(H)) == hipSuccess;
    ok = ok && hipMalloc(&s->pack16_h, F * pack_bytes16(H)) == hipSuccess;
    ok = ok && hipMalloc((void**)&s->bias, F * bias_floats(H) * sizeof(float)) == hipSuccess;
    ok = ok && hipMalloc((void**)&s->pack16_f, F * pack_bytes16(H) * 2) == hipSuccess;
    ok = ok && hipMalloc(&s->packT_bf, F * packT_bytes16(H)) == hipSuccess;
    ok = ok && hipMalloc(&s->packT_h, F * packT_bytes16(H)) == hipSuccess;
    ok = ok && hipMalloc((void**)&s->packT_f, F * packT_bytes16(H) * 2) == hipSuccess;
    if (!ok) {
        r360_scene_destroy(s);
        return R360_ENOMEM;
    }
    hipError_t e = launch_labels(occ_prob, field_map, grid->threshold, nvox, F, s->labels, S(stream));
    if (e == hipErrorInvalidValue) {
        r360_scene_destroy(s);
        return inval("field_map holds ids outside [-1, n_fields)");
    }
    if (e == hipSuccess) e = launch_repack(s, weights, S(stream));
    if (e == hipSuccess) e = launch_repack_bwd(s, weights, S(stream));
    if (e != hipSuccess) {
        r360_scene_destroy(s);
        return hip_fail("scene_create", e);
    }
    *out = s;
    return R360_OK;
}

r360_status r360_scene_set_weights(r360_scene* s, const float* weights, void* stream) {
    if (!s || !weights) return inval("NULL pointer");
    R360_TRY("repack", launch_repack(s, weights, S(stream)));
    R360_TRY("repack", launch_repack_bwd(s, weights, S(stream)));
    return R360_OK;
}

r360_status r360_scene_set_grid(r360_scene* s, const float* occ_prob, const int32_t* field_map, void* stream) {
    if (!s || !occ_prob || !field_map) return inval("NULL pointer");
    const int64_t nvox = (int64_t)s->grid.n[0] * s->grid.n[1] * s->grid.n[2];
    hipError_t e = launch_labels(occ_prob, field_map, s->grid.threshold, nvox, s->mlp.n_fields, s->labels, S(stream));
    if (e == hipErrorInvalidValue) return inval("field_map holds ids outside [-1, n_fields)");
    if (e != hipSuccess) return hip_fail("set_grid", e);
    return R360_OK;
}

size_t r360_field_frames_workspace_bytes(int32_t n_fields) {
    if (n_fields < 1) return 0;
    return ((size_t)6 * n_fields * sizeof(int32_t) + 255) & ~size_t(255);
}

r360_status r360_field_frames(const r360_grid_desc* grid, const int32_t* field_map, int32_t n_fields, float* centers,
                              float* half_extents, void* ws, size_t ws_bytes, void* stream) {
    if (!grid || !field_map || !centers || !half_extents || !ws) return inval("NULL pointer");
    if (n_fields < 1) return inval("n_fields must be >= 1");
    for (int a = 0; a < 3; ++a) {
        if (grid->n[a] < 1 || grid->n[a] > 4096) return inval("grid size outside [1, 4096]");
        if (!std::isfinite(grid->lo[a])) return inval("grid corner not finite");
    }
    if ((int64_t)grid->n[0] * grid->n[1] * grid->n[2] >= (int64_t(1) << 31)) return inval("grid has 2^31 voxels or more");
    if (!pow2(grid->voxel)) return inval("voxel edge must be a positive power of two");
    if (ws_bytes < r360_field_frames_workspace_bytes(n_fields)) return R360_EWORKSPACE;
    R360_TRY("field frames", launch_field_frames(grid, field_map, n_fields, centers, half_extents, ws, S(stream)));
    return R360_OK;
}

r360_status r360_scene_set_frames(r360_scene* s, const float* centers, const float* half_extents, void* stream) {
    if (!s) return inval("scene is NULL");
    if (!centers) {
        s->use_frames = false;
        return R360_OK;
    }
    if (!half_extents) return inval("NULL pointer");
    const int F = s->mlp.n_fields;
    if (!s->frames) {
        if (hipMalloc(reinterpret_cast<void**>(&s->frames), (size_t)F * 4 * sizeof(float)) != hipSuccess) {
            s->frames = nullptr;
            return R360_ENOMEM;
        }
    }
    R360_TRY("set frames", launch_pack_frames(centers, half_extents, F, s->frames, S(stream)));
    s->use_frames = true;
    return R360_OK;
}

void r360_scene_destroy(r360_scene* s) {
    if (!s) return;
    (void)hipFree(s->frames);
    (void)hipFree(s->labels);
    (void)hipFree(s->pack16_bf);
    (void)hipFree(s->pack16_h);
    (void)hipFree(s->bias);
    (void)hipFree(s->pack16_f);
    (void)hipFree(s->packT_bf);
    (void)hipFree(s->packT_h);
    (void)hipFree(s->packT_f);
    delete s;
}

r360_status r360_equirect_create(int32_t W, int32_t H, r360_equirect** out) {
    if (!out) return inval("out is NULL");
    *out = nullptr;
    if (W < 1 || H < 1 || W > (1 << 16) || H > (1 << 16)) return inval("W, H outside [1, 65536]");
    // Eq.2 inverted at pixel centres; sin/cos in FP64 with the argument
    // folded to |m| <= 1/2 first (m = a or 1 - a etc., exact), rounded once.
    auto sinpi = [](double a) {
        double m = std::fmod(a, 2.0);
        if (m > 1.0) m -= 2.0;
        if (m < -1.0) m += 2.0;
        if (m > 0.5) m = 1.0 - m;
        else if (m < -0.5) m = -1.0 - m;
        return std::sin(3.14159265358979323846 * m);
    };
    std::vector<float> t(2 * (size_t)W + 2 * (size_t)H);
    for (int u = 0; u < W; ++u) {
        const float a = (float)((2 * u + 1) - W) / (float)W;
        t[u] = (float)sinpi((double)a);
        t[W + u] = (float)sinpi((double)a + 0.5);
    }
    for (int v = 0; v < H; ++v) {
        const float a = (float)(H - (2 * v + 1)) / (float)(2 * H);
        t[2 * W + v] = (float)sinpi((double)a);
        t[2 * W + H + v] = (float)sinpi((double)a + 0.5);
    }
    r360_equirect* eq = new (std::nothrow) r360_equirect();
    if (!eq) return R360_ENOMEM;
    eq->W = W;
    eq->H = H;
    if (hipMalloc((void**)&eq->tables, t.size() * sizeof(float)) != hipSuccess) {
        delete eq;
        return R360_ENOMEM;
    }
    hipError_t e = hipMemcpy(eq->tables, t.data(), t.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        r360_equirect_destroy(eq);
        return hip_fail("equirect_create", e);
    }
    *out = eq;
    return R360_OK;
}

void r360_equirect_destroy(r360_equirect* eq) {
    if (!eq) return;
    (void)hipFree(eq->tables);
    delete eq;
}

r360_status r360_equirect_tables(const r360_equirect* eq, float* sp, float* cp, float* st, float* ct) {
    if (!eq || !sp || !cp || !st || !ct) return inval("NULL pointer");
    const int W = eq->W, H = eq->H;
    R360_TRY("tables", hipMemcpy(sp, eq->tables, W * sizeof(float), hipMemcpyDeviceToHost));
    R360_TRY("tables", hipMemcpy(cp, eq->tables + W, W * sizeof(float), hipMemcpyDeviceToHost));
    R360_TRY("tables", hipMemcpy(st, eq->tables + 2 * W, H * sizeof(float), hipMemcpyDeviceToHost));
    R360_TRY("tables", hipMemcpy(ct, eq->tables + 2 * W + H, H * sizeof(float), hipMemcpyDeviceToHost));
    return R360_OK;
}

r360_status r360_equirect_rays(const r360_equirect* eq, const float c2w_host[12], const int64_t* pix, int64_t N,
                               float* o, float* d, void* stream) {
    if (!eq || !o || !d) return inval("NULL pointer");
    if (!valid_c2w(c2w_host)) return inval("c2w is NULL or not finite");
    if (N <= 0) return inval("N must be positive");
    if (!pix && N != (int64_t)eq->W * eq->H) return inval("without a pixel list N must be W*H");
    RaySource src{};
    src.mode = RAYS_EQUIRECT;
    src.tables = eq->tables;
    src.W = eq->W;
    src.H = eq->H;
    std::memcpy(src.c2w, c2w_host, sizeof(src.c2w));
    src.pix = pix;
    R360_TRY("equirect_rays", launch_rays(src, N, o, d, S(stream)));
    return R360_OK;
}

r360_status r360_ods_rays(const r360_equirect* eq, const float c2w_host[12], float eye_offset, const int64_t* pix,
                          int64_t N, float* o, float* d, void* stream) {
    if (!eq || !o || !d) return inval("NULL pointer");
    if (!valid_c2w(c2w_host)) return inval("c2w is NULL or not finite");
    if (!std::isfinite(eye_offset)) return inval("eye_offset not finite");
    if (N <= 0) return inval("N must be positive");
    if (!pix && N != (int64_t)eq->W * eq->H) return inval("without a pixel list N must be W*H");
    RaySource src{};
    src.mode = RAYS_EQUIRECT;
    src.tables = eq->tables;
    src.W = eq->W;
    src.H = eq->H;
    std::memcpy(src.c2w, c2w_host, sizeof(src.c2w));
    src.pix = pix;
    src.eye = eye_offset;
    R360_TRY("ods_rays", launch_rays(src, N, o, d, S(stream)));
    return R360_OK;
}

r360_status r360_pinhole_rays(int32_t W, int32_t H, float fx, float fy, const float c2w_host[12], float* o,
                              float* d, void* stream) {
    if (!o || !d) return inval("NULL pointer");
    if (W < 1 || H < 1) return inval("W, H must be positive");
    if (!(fx > 0.0f) || !(fy > 0.0f) || !std::isfinite(fx) || !std::isfinite(fy)) return inval("focal length");
    if (!valid_c2w(c2w_host)) return inval("c2w is NULL or not finite");
    RaySource src{};
    src.mode = RAYS_PINHOLE;
    src.W = W;
    src.H = H;
    src.fx = fx;
    src.fy = fy;
    std::memcpy(src.c2w, c2w_host, sizeof(src.c2w));
    R360_TRY("pinhole_rays", launch_rays(src, (int64_t)W * H, o, d, S(stream)));
    return R360_OK;
}

double r360_lr_schedule(int64_t step, int64_t total, double lr0, double lr1) {
    if (!(lr0 > 0.0) || !(lr1 > 0.0) || step < 0) return std::nan("");
    const double frac = (double)std::min(step, total) / (double)std::max<int64_t>(total, 1);
    return lr0 * std::pow(lr1 / lr0, frac);
}

size_t r360_workspace_bytes(const r360_scene* s, int64_t n_rays, int32_t max_samples) {
    if (!s || n_rays <= 0 || max_samples < 1) return 0;
    return carve(nullptr, n_rays, max_samples, s->mlp.n_fields, s->P).bytes;
}

r360_status r360_sample_rays(const r360_scene* s, const float* o, const float* d, int64_t N,
                             const r360_render_opts* opts, int64_t* n_samples_host, float* t_mid, float* delta,
                             int32_t* ray_id, int32_t* field_id, int32_t* voxel, int32_t* ray_offset, void* ws,
                             size_t ws_bytes, void* stream) {
    if (!o || !d || !t_mid || !delta || !ray_id || !field_id || !ray_offset) return inval("NULL pointer");
    Workspace w;
    r360_status st = prepare(s, N, opts, ws, ws_bytes, false, &w);
    if (st != R360_OK) return st;
    w.ray_off = ray_offset;
    w.t_mid = t_mid;
    w.delta = delta;
    w.ray = ray_id;
    w.field = field_id;
    RaySource src{};
    src.mode = RAYS_GIVEN;
    src.o = o;
    src.d = d;
    R360_TRY("sample", launch_sample(src, dda_params(s, opts), N, w, voxel, S(stream)));
    if (n_samples_host) {
        int32_t tot = 0;
        R360_TRY("sample total", hipMemcpyAsync(&tot, ray_offset + N, sizeof(int32_t), hipMemcpyDeviceToHost, S(stream)));
        R360_TRY("sample sync", hipStreamSynchronize(S(stream)));
        *n_samples_host = tot;
    }
    return R360_OK;
}

r360_status r360_render_rays(const r360_scene* s, const float* o, const float* d, int64_t N,
                             const r360_render_opts* opts, float* rgb, float* depth, float* opacity, void* ws,
                             size_t ws_bytes, void* stream) {
    if (!o || !d || !rgb || !depth || !opacity) return inval("NULL pointer");
    Workspace w;
    r360_status st = prepare(s, N, opts, ws, ws_bytes, false, &w, true);
    if (st != R360_OK) return st;
    RaySource src{};
    src.mode = RAYS_GIVEN;
    src.o = o;
    src.d = d;
    return render_common(s, src, N, opts, rgb, depth, opacity, w, S(stream));
}

r360_status r360_render_rays_noalloc(const r360_scene* s, const float* o, const float* d, int64_t N,
                                     const r360_render_opts* opts, float* rgb, float* depth, float* opacity,
                                     void* stream) {
    if (!o || !d || !rgb || !depth || !opacity) return inval("NULL pointer");
    if (!s) return inval("scene is NULL");
    r360_status st = check_opts(opts, false);
    if (st != R360_OK) return st;
    if (opts->term_eps > 0.0f) {
        std::snprintf(g_err, sizeof(g_err), "early ray termination waits on the stream; use r360_render_rays");
        return R360_EUNSUPPORTED;
    }
    if (N <= 0 || N > (int64_t(1) << 30)) return inval("N must be in [1, 2^30]");
    if (sample_cap(N, opts->max_samples) >= (int64_t(1) << 30))
        return inval("N * max_samples must stay below 2^30; split the rays");
    const size_t need = carve(nullptr, N, opts->max_samples, s->mlp.n_fields, s->P, false).bytes;
    if (need > R360_NOALLOC_SCRATCH_BYTES) {
        std::snprintf(g_err, sizeof(g_err), "needs %zu bytes of scratch, the library's array holds %zu; split the rays",
                      need, (size_t)R360_NOALLOC_SCRATCH_BYTES);
        return R360_EWORKSPACE;
    }
    void* base = nullptr;
    st = scratch_of_current_device(&base);
    if (st != R360_OK) return st;
    Workspace w = carve(base, N, opts->max_samples, s->mlp.n_fields, s->P, false);
    RaySource src{};
    src.mode = RAYS_GIVEN;
    src.o = o;
    src.d = d;
    return render_common(s, src, N, opts, rgb, depth, opacity, w, S(stream));
}

r360_status r360_render_equirect(const r360_scene* s, const r360_equirect* eq, const float c2w_host[12],
                                 const r360_render_opts* opts, float* rgb, float* depth, float* opacity, void* ws,
                                 size_t ws_bytes, void* stream) {
    if (!eq || !rgb || !depth || !opacity) return inval("NULL pointer");
    if (!valid_c2w(c2w_host)) return inval("c2w is NULL or not finite");
    const int64_t N = (int64_t)eq->W * eq->H;
    Workspace w;
    r360_status st = prepare(s, N, opts, ws, ws_bytes, false, &w, true);
    if (st != R360_OK) return st;
    RaySource src{};
    src.mode = RAYS_EQUIRECT;
    src.tables = eq->tables;
    src.W = eq->W;
    src.H = eq->H;
    std::memcpy(src.c2w, c2w_host, sizeof(src.c2w));
    return render_common(s, src, N, opts, rgb, depth, opacity, w, S(stream));
}

r360_status r360_render_ods(const r360_scene* s, const r360_equirect* eq, const float c2w_host[12], float eye_offset,
                            const r360_render_opts* opts, float* rgb, float* depth, float* opacity, void* ws,
                            size_t ws_bytes, void* stream) {
    if (!eq || !rgb || !depth || !opacity) return inval("NULL pointer");
    if (!valid_c2w(c2w_host)) return inval("c2w is NULL or not finite");
    if (!std::isfinite(eye_offset)) return inval("eye_offset not finite");
    const int64_t N = (int64_t)eq->W * eq->H;
    Workspace w;
    r360_status st = prepare(s, N, opts, ws, ws_bytes, false, &w, true);
    if (st != R360_OK) return st;
    RaySource src{};
    src.mode = RAYS_EQUIRECT;
    src.tables = eq->tables;
    src.W = eq->W;
    src.H = eq->H;
    std::memcpy(src.c2w, c2w_host, sizeof(src.c2w));
    src.eye = eye_offset;
    return render_common(s, src, N, opts, rgb, depth, opacity, w, S(stream));
}

r360_status r360_render_pinhole(const r360_scene* s, int32_t W, int32_t H, float fx, float fy,
                                const float c2w_host[12], const r360_render_opts* opts, float* rgb, float* depth,
                                float* opacity, void* ws, size_t ws_bytes, void* stream) {
    if (!rgb || !depth || !opacity) return inval("NULL pointer");
    if (W < 1 || H < 1) return inval("W, H must be positive");
    if (!(fx > 0.0f) || !(fy > 0.0f) || !std::isfinite(fx) || !std::isfinite(fy)) return inval("focal length");
    if (!valid_c2w(c2w_host)) return inval("c2w is NULL or not finite");
    const int64_t N = (int64_t)W * H;
    Workspace w;
    r360_status st = prepare(s, N, opts, ws, ws_bytes, false, &w, true);
    if (st != R360_OK) return st;
    RaySource src{};
    src.mode = RAYS_PINHOLE;
    src.W = W;
    src.H = H;
    src.fx = fx;
    src.fy = fy;
    std::memcpy(src.c2w, c2w_host, sizeof(src.c2w));
    return render_common(s, src, N, opts, rgb, depth, opacity, w, S(stream));
}

r360_status r360_backward(const r360_scene* s, const float* o, const float* d, int64_t N,
                          const r360_render_opts* opts, const float* grad_rgb, float* grad_weights, void* ws,
                          size_t ws_bytes, void* stream) {
    if (!o || !d || !grad_rgb || !grad_weights) return inval("NULL pointer");
    Workspace w;
    r360_status st = prepare(s, N, opts, ws, ws_bytes, false, &w);
    if (st != R360_OK) return st;
    w.ro = o;
    w.rd = d;
    {
        R360_STAGE(5, S(stream));
        R360_TRY("composite backward", launch_composite_backward_slots(w, N, grad_rgb, nullptr, nullptr, S(stream)));
    }
    {
        R360_STAGE(6, S(stream));
        R360_TRY("mlp backward", launch_mlp_backward(s, w, opts->precision, grad_weights, S(stream)));
    }
    return R360_OK;
}

r360_status r360_train_step(const r360_scene* s, const float* o, const float* d, int64_t N, const float* target,
                            const r360_render_opts* opts, float* loss, float* grad_weights, float* rgb_out, void* ws,
                            size_t ws_bytes, void* stream) {
    if (!o || !d || !target || !loss || !grad_weights) return inval("NULL pointer");
    Workspace w;
    r360_status st = prepare(s, N, opts, ws, ws_bytes, false, &w);
    if (st != R360_OK) return st;
    float* rgb = rgb_out ? rgb_out : w.ray_rgb;
    float* grad_rgb = w.ray_grad;
    RaySource src{};
    src.mode = RAYS_GIVEN;
    src.o = o;
    src.d = d;
    // the loss is folded into the compositing passes: its gradient and partial
    // sums in the forward one, the final sum in the backward one
    st = render_common(s, src, N, opts, rgb, nullptr, nullptr, w, S(stream), target, grad_rgb);
    if (st != R360_OK) return st;
    {
        R360_STAGE(5, S(stream));
        R360_TRY("composite backward", launch_composite_backward_slots(w, N, grad_rgb, rgb, loss, S(stream)));
    }
    {
        R360_STAGE(6, S(stream));
        R360_TRY("mlp backward", launch_mlp_backward(s, w, opts->precision, grad_weights, S(stream)));
    }
    return R360_OK;
}

r360_status r360_adam_step(float* w, const float* g, float* m, float* v, int64_t n, int64_t step, float lr,
                           float b1, float b2, float eps, void* stream) {
    if (!w || !g || !m || !v) return inval("NULL pointer");
    if (n <= 0 || step < 1) return inval("n must be positive and step >= 1");
    if (!(b1 >= 0.0f && b1 < 1.0f) || !(b2 >= 0.0f && b2 < 1.0f) || !(eps > 0.0f) || !std::isfinite(lr))
        return inval("Adam hyper-parameters");
    R360_TRY("adam", launch_adam(w, g, m, v, n, step, lr, b1, b2, eps, S(stream)));
    return R360_OK;
}

r360_status r360_gradcheck_forward(const r360_scene* s, const double* w64, const float* o, const float* d, int64_t N,
                                   const r360_render_opts* opts, double* rgb64, void* ws, size_t ws_bytes,
                                   void* stream) {
    if (!w64 || !o || !d || !rgb64) return inval("NULL pointer");
    Workspace w;
    r360_status st = prepare(s, N, opts, ws, ws_bytes, true, &w);
    if (st != R360_OK) return st;
    if (opts->precision != R360_FP64_GRADCHECK) return inval("precision must be R360_FP64_GRADCHECK");
    w.ro = o;
    w.rd = d;
    RaySource src{};
    src.mode = RAYS_GIVEN;
    src.o = o;
    src.d = d;
    R360_TRY("sample", launch_sample(src, dda_params(s, opts), N, w, nullptr, S(stream)));
    R360_TRY("gradcheck forward", launch_gradcheck_forward(s, w, w64, N, rgb64, S(stream)));
    return R360_OK;
}

r360_status r360_gradcheck_backward(const r360_scene* s, const double* w64, const float* o, const float* d, int64_t N,
                                    const r360_render_opts* opts, const double* grad_rgb64, double* grad64, void* ws,
                                    size_t ws_bytes, void* stream) {
    if (!w64 || !o || !d || !grad_rgb64 || !grad64) return inval("NULL pointer");
    Workspace w;
    r360_status st = prepare(s, N, opts, ws, ws_bytes, true, &w);
    if (st != R360_OK) return st;
    if (opts->precision != R360_FP64_GRADCHECK) return inval("precision must be R360_FP64_GRADCHECK");
    w.ro = o;
    w.rd = d;
    R360_TRY("gradcheck backward", launch_gradcheck_backward(s, w, w64, N, grad_rgb64, grad64, S(stream)));
    return R360_OK;
}

int64_t r360_global_params(int32_t width, int32_t color_width) {
    if (width < 32 || color_width < 32 || width % 32 || color_width % 32) return -1;
    return global_params(width, color_width);
}

static r360_status check_global(const r360_global_desc* g) {
    if (!g) return inval("desc is NULL");
    if (g->width < 32 || g->width % 32 || g->width > 4096 || g->color_width < 32 || g->color_width % 32 ||
        g->color_width > 4096) {
        std::snprintf(g_err, sizeof(g_err), "width and color_width must be positive multiples of 32");
        return R360_EUNSUPPORTED;
    }
    if (g->n_samples < 2 || g->n_samples > 4096) return inval("n_samples outside [2, 4096]");
    if (!(g->near_ > 0.0f) || !(g->far_ > g->near_) || !std::isfinite(g->far_)) return inval("need 0 < near < far < inf");
    if (!(g->half_extent > 0.0f) || !pow2(g->voxel)) return inval("half_extent > 0 and a power-of-two voxel");
    for (int a = 0; a < 3; ++a)
        if (g->grid_n[a] < 1 || g->grid_n[a] > 4096) return inval("grid size outside [1, 4096]");
    if ((int64_t)g->grid_n[0] * g->grid_n[1] * g->grid_n[2] >= (int64_t(1) << 31)) return inval("grid has 2^31 voxels or more");
    return R360_OK;
}

size_t r360_global_workspace_bytes(const r360_global_desc* g, int64_t n_rays) {
    if (check_global(g) != R360_OK || n_rays <= 0) return 0;
    return global_workspace_bytes(g->width, g->color_width, n_rays, g->n_samples);
}

r360_status r360_global_field_step(const r360_global_desc* g, const float* weights, const float* o, const float* d,
                                   int64_t N, const float* target, float* loss, float* grad, float* rgb_out,
                                   float* depth_out, float* occ, void* ws, size_t ws_bytes, void* stream) {
    r360_status st = check_global(g);
    if (st != R360_OK) return st;
    if (!weights || !o || !d || !ws) return inval("NULL pointer");
    if (N <= 0 || N * (int64_t)g->n_samples >= (int64_t(1) << 31)) return inval("N * n_samples outside [1, 2^31)");
    if (target && (!loss || !grad)) return inval("a target needs loss and grad outputs");
    if (reinterpret_cast<uintptr_t>(ws) & 255) return inval("workspace must be 256-byte aligned");
    const size_t need = global_workspace_bytes(g->width, g->color_width, N, g->n_samples);
    if (ws_bytes < need) {
        std::snprintf(g_err, sizeof(g_err), "workspace has %zu bytes, needs %zu", ws_bytes, need);
        return R360_EWORKSPACE;
    }
    R360_STAGE(7, S(stream));
    R360_TRY("global field", launch_global_step(g, weights, o, d, N, target, loss, grad, rgb_out, depth_out, occ, ws,
                                                S(stream), target ? 3 : 1));
    return R360_OK;
}

static r360_status check_occ(const r360_occ_desc* g) {
    if (!g) return inval("desc is NULL");
    for (int a = 0; a < 3; ++a)
        if (g->n[a] < 1 || g->n[a] > 4096) return inval("grid size outside [1, 4096]");
    if ((int64_t)g->n[0] * g->n[1] * g->n[2] >= (int64_t(1) << 31)) return inval("grid has 2^31 voxels or more");
    if (!pow2(g->voxel)) return inval("voxel edge must be a positive power of two");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(g->lo[a])) return inval("grid corner must be finite");
    if (!(g->near_ >= 0.0f) || !std::isfinite(g->near_) || !(g->far_ > g->near_)) return inval("need 0 <= near < far");
    if (!(g->l_hit > 0.0f) || !std::isfinite(g->l_hit)) return inval("l_hit must be positive and finite");
    if (!(g->l_miss < 0.0f) || !std::isfinite(g->l_miss)) return inval("l_miss must be negative and finite");
    if (!(g->l_min < g->l_max) || !std::isfinite(g->l_min) || !std::isfinite(g->l_max)) return inval("need l_min < l_max, finite");
    if (!(g->min_opacity >= 0.0f) || !(g->min_opacity <= 1.0f)) return inval("min_opacity outside [0, 1]");
    return R360_OK;
}

r360_status r360_depth_uncertainty(const float* t, const float* delta, const float* sigma, int64_t N,
                                   int32_t per_ray, float* depth, float* uncert, float* opacity, void* stream) {
    if (!t || !delta || !sigma || !depth || !uncert || !opacity) return inval("NULL pointer");
    if (N < 1 || N > (int64_t(1) << 31) || per_ray < 1) return inval("need 1 <= N <= 2^31 and S >= 1");
    R360_STAGE(8, S(stream));
    R360_TRY("depth statistics",
             launch_depth_stats(t, delta, sigma, N, per_ray, depth, uncert, opacity, S(stream)));
    return R360_OK;
}

r360_status r360_occ_desc_init(r360_occ_desc* g, int32_t n, float lo, float voxel, float near_, float far_,
                               double p_hit, double p_miss, float l_min, float l_max, float min_opacity) {
    if (!g) return inval("desc is NULL");
    if (!(p_hit > 0.5 && p_hit < 1.0) || !(p_miss > 0.0 && p_miss < 0.5))
        return inval("need 1/2 < p_hit < 1 and 0 < p_miss < 1/2");
    for (int a = 0; a < 3; ++a) {
        g->n[a] = n;
        g->lo[a] = lo;
    }
    g->voxel = voxel;
    g->near_ = near_;
    g->far_ = far_;
    g->l_hit = (float)std::log(p_hit / (1.0 - p_hit));
    g->l_miss = (float)std::log(p_miss / (1.0 - p_miss));
    g->l_min = l_min;
    g->l_max = l_max;
    g->min_opacity = min_opacity;
    return check_occ(g);
}

size_t r360_occupancy_workspace_bytes(const r360_occ_desc* g) {
    if (check_occ(g) != R360_OK) return 0;
    return occupancy_workspace_bytes((int64_t)g->n[0] * g->n[1] * g->n[2]);
}

r360_status r360_occupancy_update(const r360_occ_desc* g, float* logit, float* prob, const float* o, const float* d,
                                  int64_t N, const float* depth, const float* uncert, const float* opacity, void* ws,
                                  size_t ws_bytes, void* stream) {
    r360_status st = check_occ(g);
    if (st != R360_OK) return st;
    if (!logit || !o || !d || !depth || !uncert || !opacity || !ws) return inval("NULL pointer");
    if (N < 1 || N > (int64_t(1) << 31)) return inval("N outside [1, 2^31]");
    if (reinterpret_cast<uintptr_t>(ws) & 255) return inval("workspace must be 256-byte aligned");
    const size_t need = occupancy_workspace_bytes((int64_t)g->n[0] * g->n[1] * g->n[2]);
    if (ws_bytes < need) {
        std::snprintf(g_err, sizeof(g_err), "workspace has %zu bytes, needs %zu", ws_bytes, need);
        return R360_EWORKSPACE;
    }
    R360_STAGE(8, S(stream));
    R360_TRY("occupancy update",
             launch_occupancy_update(g, logit, prob, o, d, N, depth, uncert, opacity, ws, S(stream)));
    return R360_OK;
}

r360_status r360_global_field_measure(const r360_global_desc* g, const float* weights, const float* o, const float* d,
                                      int64_t N, float* depth, float* uncert, float* opacity, void* ws,
                                      size_t ws_bytes, void* stream) {
    r360_status st = check_global(g);
    if (st != R360_OK) return st;
    if (!weights || !o || !d || !depth || !uncert || !opacity || !ws) return inval("NULL pointer");
    if (N <= 0 || N * (int64_t)g->n_samples >= (int64_t(1) << 31)) return inval("N * n_samples outside [1, 2^31)");
    if (reinterpret_cast<uintptr_t>(ws) & 255) return inval("workspace must be 256-byte aligned");
    const size_t need = global_workspace_bytes(g->width, g->color_width, N, g->n_samples);
    if (ws_bytes < need) {
        std::snprintf(g_err, sizeof(g_err), "workspace has %zu bytes, needs %zu", ws_bytes, need);
        return R360_EWORKSPACE;
    }
    const GlobalMeasure meas{depth, uncert, opacity};
    R360_STAGE(7, S(stream));
    R360_TRY("global field measure", launch_global_step(g, weights, o, d, N, nullptr, nullptr, nullptr, nullptr,
                                                        nullptr, nullptr, ws, S(stream), 1, &meas));
    return R360_OK;
}

size_t r360_global_points_workspace_bytes(const r360_global_desc* g, int64_t M) {
    if (check_global(g) != R360_OK || M <= 0) return 0;
    return global_workspace_bytes(g->width, g->color_width, M, 1);
}

r360_status r360_global_field_points(const r360_global_desc* g, const float* weights, const float* x,
                                     const float* dir, int64_t M, float* sigma, float* rgb, void* ws, size_t ws_bytes,
                                     void* stream) {
    r360_status st = check_global(g);
    if (st != R360_OK) return st;
    if (!weights || !x || !dir || !sigma || !rgb || !ws) return inval("NULL pointer");
    if (M <= 0 || M >= (int64_t(1) << 31)) return inval("M outside [1, 2^31)");
    if (reinterpret_cast<uintptr_t>(ws) & 255) return inval("workspace must be 256-byte aligned");
    const size_t need = global_workspace_bytes(g->width, g->color_width, M, 1);
    if (ws_bytes < need) {
        std::snprintf(g_err, sizeof(g_err), "workspace has %zu bytes, needs %zu", ws_bytes, need);
        return R360_EWORKSPACE;
    }
    r360_global_desc one = *g;
    one.n_samples = 1;
    GlobalMeasure pts;
    pts.points = true;
    pts.point_sigma = sigma;
    pts.point_rgb = rgb;
    R360_STAGE(7, S(stream));
    R360_TRY("global field points", launch_global_step(&one, weights, x, dir, M, nullptr, nullptr, nullptr, nullptr,
                                                       nullptr, nullptr, ws, S(stream), 1, &pts));
    return R360_OK;
}

r360_status r360_distill_step(const r360_scene* s, const float* x, const float* dir, const int32_t* field,
                              int64_t M, const float* tsig, const float* trgb, const r360_render_opts* opts,
                              float* loss, float* grad_weights, void* ws, size_t ws_bytes, void* stream) {
    if (!x || !dir || !field || !tsig || !trgb || !loss || !grad_weights || !opts) return inval("NULL pointer");
    r360_render_opts one = *opts;
    one.max_samples = 1;
    one.term_eps = 0.0f;        // one sample per point: nothing to stop
    one.near_ = 0.0f;
    one.far_ = 1.0f;
    Workspace w;
    r360_status st = prepare(s, M, &one, ws, ws_bytes, false, &w);
    if (st != R360_OK) return st;
    w.ro = x;
    w.rd = dir;
    {
        R360_STAGE(0, S(stream));
        R360_TRY("distill points", launch_distill_points(w, M, field, s->mlp.n_fields, S(stream)));
    }
    {
        R360_STAGE(1, S(stream));
        R360_TRY("route", launch_route(w, s->mlp.n_fields, false, S(stream)));
    }
    {
        R360_STAGE(2, S(stream));
        R360_TRY("mlp forward", launch_mlp_forward(s, w, one.precision, S(stream)));
    }
    {
        R360_STAGE(4, S(stream));
        R360_TRY("distill loss", launch_distill_loss(w, M, tsig, trgb, loss, S(stream)));
    }
    {
        R360_STAGE(6, S(stream));
        R360_TRY("mlp backward", launch_mlp_backward(s, w, one.precision, grad_weights, S(stream)));
    }
    return R360_OK;
}

static r360_status check_dims(const int32_t* n) {
    if (!n) return inval("grid size is NULL");
    for (int a = 0; a < 3; ++a)
        if (n[a] < 1 || n[a] > 4096) return inval("grid size outside [1, 4096]");
    if ((int64_t)n[0] * n[1] * n[2] >= (int64_t(1) << 31)) return inval("grid has 2^31 voxels or more");
    return R360_OK;
}

size_t r360_assign_workspace_bytes(const int32_t n[3]) {
    if (check_dims(n) != R360_OK) return 0;
    return assign_workspace_bytes((int64_t)n[0] * n[1] * n[2]);
}

r360_status r360_assign_fields(const int32_t n[3], const float* occ, float threshold, int32_t n_fields,
                               int32_t* field_map, int64_t* n_occupied_host, void* ws, size_t ws_bytes,
                               void* stream) {
    r360_status st = check_dims(n);
    if (st != R360_OK) return st;
    if (!occ || !field_map || !ws) return inval("NULL pointer");
    if (n_fields < 1) return inval("n_fields must be >= 1");
    if (reinterpret_cast<uintptr_t>(ws) & 255) return inval("workspace must be 256-byte aligned");
    const size_t need = assign_workspace_bytes((int64_t)n[0] * n[1] * n[2]);
    if (ws_bytes < need) {
        std::snprintf(g_err, sizeof(g_err), "workspace has %zu bytes, needs %zu", ws_bytes, need);
        return R360_EWORKSPACE;
    }
    int64_t n_occ = 0;
    R360_TRY("field assignment",
             launch_assign_fields(n, occ, threshold, n_fields, field_map, &n_occ, ws, S(stream)));
    if (n_occupied_host) *n_occupied_host = n_occ;
    return R360_OK;
}

size_t r360_assign_uniform_workspace_bytes(const int32_t b[3]) {
    if (!b || b[0] < 1 || b[1] < 1 || b[2] < 1 || (int64_t)b[0] * b[1] * b[2] > (int64_t(1) << 24)) return 0;
    return uniform_workspace_bytes((int64_t)b[0] * b[1] * b[2]);
}

r360_status r360_assign_uniform(const int32_t n[3], const float* occ, float threshold, const int32_t b[3],
                                int32_t* field_map, int32_t* n_fields_host, void* ws, size_t ws_bytes,
                                void* stream) {
    r360_status st = check_dims(n);
    if (st != R360_OK) return st;
    if (!occ || !field_map || !ws || !b) return inval("NULL pointer");
    for (int a = 0; a < 3; ++a)
        if (b[a] < 1 || b[a] > n[a]) return inval("blocks per axis outside [1, n]");
    if ((int64_t)b[0] * b[1] * b[2] > (int64_t(1) << 24)) return inval("more than 2^24 blocks");
    if (reinterpret_cast<uintptr_t>(ws) & 255) return inval("workspace must be 256-byte aligned");
    const size_t need = uniform_workspace_bytes((int64_t)b[0] * b[1] * b[2]);
    if (ws_bytes < need) {
        std::snprintf(g_err, sizeof(g_err), "workspace has %zu bytes, needs %zu", ws_bytes, need);
        return R360_EWORKSPACE;
    }
    int32_t count = 0;
    R360_TRY("uniform assignment", launch_assign_uniform(n, occ, threshold, b, field_map, &count, ws, S(stream)));
    if (n_fields_host) *n_fields_host = count;
    return R360_OK;
}

r360_status r360_profile_enable(int32_t on) {
    g_prof = on != 0;
    return R360_OK;
}

r360_status r360_profile_read(double* ms, int32_t* count) {
    if (!ms || !count) return inval("NULL pointer");
    for (int k = 0; k < R360_NSTAGES; ++k) { ms[k] = 0.0; count[k] = 0; }
    r360_status st = R360_OK;
    for (auto& e : g_events) {
        float t = 0.0f;
        hipError_t err = hipEventSynchronize(e.b);
        if (err == hipSuccess) err = hipEventElapsedTime(&t, e.a, e.b);
        if (err != hipSuccess && st == R360_OK) st = hip_fail("profile_read", err);
        if (e.stage >= 0 && e.stage < R360_NSTAGES) { ms[e.stage] += t; count[e.stage] += 1; }
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    g_events.clear();
    return st;
}

const char* r360_status_string(int32_t status) {
    switch (status) {
    case R360_OK: return "ok";
    case R360_EINVAL: return "invalid argument";
    case R360_ENOMEM: return "out of device memory";
    case R360_EHIP: return "HIP runtime error";
    case R360_EUNSUPPORTED: return "unsupported configuration";
    case R360_EWORKSPACE: return "workspace too small";
    default: return "unknown status";
    }
}

const char* r360_last_error(void) { return g_err; }

}  // extern "C"
