// Ray generation and occupied-voxel sampling.
//
// Rays: equirect (Sec. 3.2, Eq.2 inverted at pixel centres, Eq.3) from
// per-resolution sine/cosine tables, pinhole viewports, or caller rays.
// Sampling: FP32 voxel traversal over a label grid; one midpoint sample per
// occupied voxel segment of positive length (Sec. 4.2 dense sampling of the
// occupied voxels; Sec. 5 ray casting over the labelled occupancy map).
//
// Two passes over the rays (count, then fill at scanned offsets) keep each
// ray's samples contiguous and in t order, so compositing reads one
// contiguous run per ray and the whole result is deterministic.
//
// Bit-exact contract: this file is compiled without floating-point
// contraction; every operation below is a correctly rounded FP32 add, mul,
// div or explicit fma, in the order of the traversal specification, so a
// CPU implementation of the same specification yields identical samples.
#include "r360_internal.h"

namespace r360 {

namespace {

__device__ __forceinline__ float mn(float a, float b) { return (b < a) ? b : a; }
__device__ __forceinline__ float mx(float a, float b) { return (a < b) ? b : a; }

// Direction of ray r from its source; o, d out.
template <int MODE>
__device__ __forceinline__ void make_ray(const RaySource& s, int64_t N, int64_t r, float o[3], float d[3]) {
    if constexpr (MODE == RAYS_GIVEN) {
        o[0] = s.o[r]; o[1] = s.o[N + r]; o[2] = s.o[2 * N + r];
        d[0] = s.d[r]; d[1] = s.d[N + r]; d[2] = s.d[2 * N + r];
        return;
    } else {
        float dc[3];
        if constexpr (MODE == RAYS_EQUIRECT) {
            const int64_t p = s.pix ? s.pix[r] : r;
            if (p < 0 || p >= (int64_t)s.W * s.H) {   // out-of-range pixel: a NaN ray that samples nothing
                o[0] = o[1] = o[2] = d[0] = d[1] = d[2] = __builtin_nanf("");
                return;
            }
            const int u = (int)(p % s.W), v = (int)(p / s.W);
            const float sphi = s.tables[u], cphi = s.tables[s.W + u];
            const float sth = s.tables[2 * s.W + v], cth = s.tables[2 * s.W + s.H + v];
            dc[0] = cth * sphi; dc[1] = -sth; dc[2] = cth * cphi;
        } else {
            const int u = (int)(r % s.W), v = (int)(r / s.W);
            const float x = ((float)u + 0.5f - 0.5f * (float)s.W) / s.fx;
            const float y = ((float)v + 0.5f - 0.5f * (float)s.H) / s.fy;
            const float nrm = __builtin_sqrtf(__builtin_fmaf(x, x, __builtin_fmaf(y, y, 1.0f)));
            dc[0] = x / nrm; dc[1] = y / nrm; dc[2] = 1.0f / nrm;
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const float* R = s.c2w + 4 * i;
            d[i] = __builtin_fmaf(R[2], dc[2], __builtin_fmaf(R[1], dc[1], R[0] * dc[0]));
            o[i] = R[3];
        }
    }
}

// Voxel traversal. Emits (t_mid, delta, voxel, field) for the first
// max_samples occupied segments; returns the count. With FILL false only
// counts. Per step only the crossed axis's next-plane distance changes; the
// others are reused (their plane index did not change, so the recomputation
// would give the same bits).
// Where emitted samples go: nowhere (count pass), straight to the global
// arrays, or to the wave's LDS window (packed lane << 16 | field).
struct CountSink {
    __device__ void emit(int, float, float, int, int64_t) {}
};
struct GlobalSink {
    int64_t base; int32_t ray_id;
    float *t_mid, *delta; int32_t *ray, *field, *voxel;
    __device__ void emit(int k, float tm, float dl, int lab, int64_t lin) {
        const int64_t j = base + k;
        t_mid[j] = tm; delta[j] = dl; ray[j] = ray_id; field[j] = lab;
        if (voxel) voxel[j] = (int32_t)lin;
    }
};
// Samples whose wave-local position falls inside the window go to LDS, the
// rest straight to memory.
struct WindowSink {
    int pos; int lane; int win;
    float *l_t, *l_d; int32_t* l_tag;
    GlobalSink far_;
    __device__ void emit(int k, float tm, float dl, int lab, int64_t lin) {
        if (pos + k < win) {
            l_t[pos + k] = tm; l_d[pos + k] = dl; l_tag[pos + k] = (lane << 16) | lab;
        } else {
            far_.emit(k, tm, dl, lab, lin);
        }
    }
};

template <class Sink>
__device__ int traverse(const DdaParams& P, const float o[3], const float d[3], Sink& sink) {
    const float INF = __builtin_inff();
    const int n[3] = {P.n0, P.n1, P.n2};
    const float lo[3] = {P.lo0, P.lo1, P.lo2};
    float inv[3];
    bool act[3];
    float t0 = P.near_, t1 = P.far_;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (!(o[a] == o[a]) || !(d[a] == d[a])) return 0;   // NaN ray: no samples
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float hi = lo[a] + (float)n[a] * P.voxel;
        act[a] = d[a] != 0.0f;
        if (act[a]) {
            inv[a] = 1.0f / d[a];
            const float ta = (lo[a] - o[a]) * inv[a];
            const float tb = (hi - o[a]) * inv[a];
            t0 = mx(t0, mn(ta, tb));
            t1 = mn(t1, mx(ta, tb));
        } else {
            inv[a] = 0.0f;
            if (!(o[a] >= lo[a] && o[a] < hi)) return 0;
        }
    }
    if (!(t0 < t1)) return 0;
    int idx[3], step[3];
    float tn[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float p = __builtin_fmaf(t0, d[a], o[a]);
        const float q = (p - lo[a]) * P.inv_voxel;
        const float fq = __builtin_floorf(q);
        int i = (int)fq;
        if (q == fq && d[a] < 0.0f) i -= 1;
        idx[a] = i < 0 ? 0 : (i > n[a] - 1 ? n[a] - 1 : i);
        step[a] = d[a] > 0.0f ? 1 : -1;
        tn[a] = act[a] ? (__builtin_fmaf((float)(idx[a] + (d[a] > 0.0f ? 1 : 0)), P.voxel, lo[a]) - o[a]) * inv[a]
                       : INF;
    }
    const int64_t sx = 1, sy = P.n0, sz = (int64_t)P.n0 * P.n1;
    int64_t lin = idx[0] + sy * idx[1] + sz * idx[2];
    int count = 0;
    float t_in = t0;
    for (;;) {
        int am = 0;
        if (tn[1] < tn[am]) am = 1;
        if (tn[2] < tn[am]) am = 2;
        const float tna = tn[am];
        const float t_out = mn(tna, t1);
        const int lab = P.labels[lin];
        if (t_out > t_in && lab >= 0) {
            sink.emit(count, (t_in + t_out) * 0.5f, t_out - t_in, lab, lin);
            if (++count == P.max_samples) break;
        }
        if (!(tna < t1)) break;
        t_in = mx(t_in, tna);
        const int ni = idx[am] + step[am];
        if (ni < 0 || ni >= n[am]) break;
        idx[am] = ni;
        const int64_t stride = am == 0 ? sx : (am == 1 ? sy : sz);
        lin += step[am] > 0 ? stride : -stride;
        tn[am] = (__builtin_fmaf((float)(ni + (d[am] > 0.0f ? 1 : 0)), P.voxel, lo[am]) - o[am]) * inv[am];
    }
    return count;
}

template <int MODE>
__global__ __launch_bounds__(256) void k_rays(RaySource src, int64_t N, float* __restrict__ o, float* __restrict__ d) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    float oo[3], dd[3];
    make_ray<MODE>(src, N, r, oo, dd);
#pragma unroll
    for (int a = 0; a < 3; ++a) { o[a * N + r] = oo[a]; d[a * N + r] = dd[a]; }
}

// Pass 1: per-ray sample counts into ray_off[r]; generated rays are stored
// for the later passes.
template <int MODE>
__global__ __launch_bounds__(256) void k_count(RaySource src, DdaParams P, int64_t N, int32_t* __restrict__ cnt,
                                               float* __restrict__ o_ws, float* __restrict__ d_ws) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    float o[3], d[3];
    make_ray<MODE>(src, N, r, o, d);
    if constexpr (MODE != RAYS_GIVEN) {
#pragma unroll
        for (int a = 0; a < 3; ++a) { o_ws[a * N + r] = o[a]; d_ws[a * N + r] = d[a]; }
    }
    CountSink sink;
    cnt[r] = traverse(P, o, d, sink);
}

// Pass 2: the same traversal writes the samples at the ray's offset. The 64
// rays of a wave own one contiguous output range; its first FILL_WIN samples
// are emitted into the wave's LDS window and copied out with coalesced
// stores, the rest (and everything when voxel ids are requested) go straight
// to memory. The window is kept small so that the traversal,
// which waits on one label load per step, keeps enough waves resident (9 KB per wave).
constexpr int FILL_WIN = 768;

__global__ __launch_bounds__(256) void k_fill(DdaParams P, int64_t N, const float* __restrict__ o_in,
                                              const float* __restrict__ d_in, const int32_t* __restrict__ off,
                                              float* __restrict__ t_mid, float* __restrict__ delta,
                                              int32_t* __restrict__ ray, int32_t* __restrict__ field,
                                              int32_t* __restrict__ voxel) {
    __shared__ float l_t[4][FILL_WIN], l_d[4][FILL_WIN];
    __shared__ int32_t l_tag[4][FILL_WIN];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t r0 = ((int64_t)blockIdx.x * 4 + wv) * 64;
    if (r0 >= N) return;
    const int64_t r = r0 + lane;
    const bool live = r < N;
    const int wa = off[r0], wb = off[min(r0 + 64, N)];
    float o[3] = {0.f, 0.f, 0.f}, d[3] = {0.f, 0.f, 0.f};
    if (live) {
#pragma unroll
        for (int a = 0; a < 3; ++a) { o[a] = o_in[a * N + r]; d[a] = d_in[a * N + r]; }
    }
    if (voxel == nullptr) {
        if (live) {
            WindowSink sink{off[r] - wa, lane, FILL_WIN, l_t[wv], l_d[wv], l_tag[wv],
                            GlobalSink{off[r], (int32_t)r, t_mid, delta, ray, field, nullptr}};
            traverse(P, o, d, sink);
        }
        __builtin_amdgcn_wave_barrier();
        const int nwin = min(wb - wa, FILL_WIN);
        for (int k = lane; k < nwin; k += 64) {
            const int tag = l_tag[wv][k];
            t_mid[wa + k] = l_t[wv][k];
            delta[wa + k] = l_d[wv][k];
            ray[wa + k] = (int32_t)(r0 + (tag >> 16));
            field[wa + k] = tag & 0xFFFF;
        }
    } else if (live) {
        GlobalSink sink{off[r], (int32_t)r, t_mid, delta, ray, field, voxel};
        traverse(P, o, d, sink);
    }
}

// ---------------------------------------------------------------------------
// Exclusive scan of per-ray counts (in place), total at [N].
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        const int t = __shfl_up(v, s, 64);
        if (lane >= s) v += t;
    }
    return v;
}

// Block-wide exclusive scan of one value per thread (1024 threads); returns
// the exclusive prefix, *total gets the block sum.
__device__ __forceinline__ int block_excl_scan(int v, int* total) {
    __shared__ int wsum[16];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int inc = wave_incl_scan(v);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    if (w == 0) {
        int x = lane < 16 ? wsum[lane] : 0;
        x = wave_incl_scan(x);
        if (lane < 16) wsum[lane] = x;
    }
    __syncthreads();
    const int before = w > 0 ? wsum[w - 1] : 0;
    *total = wsum[15];
    __syncthreads();
    return before + inc - v;
}

__global__ __launch_bounds__(1024) void k_scan_reduce(const int32_t* __restrict__ x, int64_t N, int32_t* __restrict__ sums) {
    const int64_t b0 = (int64_t)blockIdx.x * SCAN_TILE;
    int s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t i = b0 + threadIdx.x * 4 + k;
        if (i < N) s += x[i];
    }
    int tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_top(int32_t* __restrict__ sums, int nb, int32_t* __restrict__ total_out) {
    int carry = 0;
    for (int base = 0; base < nb; base += 1024) {
        const int i = base + threadIdx.x;
        const int v = i < nb ? sums[i] : 0;
        int tot;
        const int ex = block_excl_scan(v, &tot);
        if (i < nb) sums[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *total_out = carry;
}

__global__ __launch_bounds__(1024) void k_scan_down(int32_t* __restrict__ x, int64_t N, const int32_t* __restrict__ sums) {
    const int64_t b0 = (int64_t)blockIdx.x * SCAN_TILE;
    int v[4];
    int s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t i = b0 + threadIdx.x * 4 + k;
        v[k] = i < N ? x[i] : 0;
        s += v[k];
    }
    int tot;
    int ex = block_excl_scan(s, &tot) + sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t i = b0 + threadIdx.x * 4 + k;
        if (i < N) x[i] = ex;
        ex += v[k];
    }
}

__global__ __launch_bounds__(256) void k_labels(const float* __restrict__ occ, const int32_t* __restrict__ fmap,
                                                float thr, int64_t n, int n_fields, int16_t* __restrict__ lab,
                                                int32_t* __restrict__ bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int f = fmap[i];
    const bool occd = occ[i] > thr;
    if (f >= n_fields || f < -1) atomicAdd(bad, 1);
    lab[i] = (int16_t)((occd && f >= 0 && f < n_fields) ? f : -1);
}

__global__ void k_zero_i32(int32_t* p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_rays(const RaySource& src, int64_t N, float* o, float* d, hipStream_t st) {
    const unsigned nb = blocks_for(N, 256);
    if (src.mode == RAYS_EQUIRECT) hipLaunchKernelGGL(k_rays<RAYS_EQUIRECT>, dim3(nb), dim3(256), 0, st, src, N, o, d);
    else if (src.mode == RAYS_PINHOLE) hipLaunchKernelGGL(k_rays<RAYS_PINHOLE>, dim3(nb), dim3(256), 0, st, src, N, o, d);
    else hipLaunchKernelGGL(k_rays<RAYS_GIVEN>, dim3(nb), dim3(256), 0, st, src, N, o, d);
    return hipGetLastError();
}

hipError_t launch_sample(const RaySource& src, const DdaParams& p, int64_t N, const Workspace& w,
                         int32_t* voxel_out, hipStream_t st) {
    const unsigned nb = blocks_for(N, 256);
    if (src.mode == RAYS_EQUIRECT)
        hipLaunchKernelGGL(k_count<RAYS_EQUIRECT>, dim3(nb), dim3(256), 0, st, src, p, N, w.ray_off, w.o, w.d);
    else if (src.mode == RAYS_PINHOLE)
        hipLaunchKernelGGL(k_count<RAYS_PINHOLE>, dim3(nb), dim3(256), 0, st, src, p, N, w.ray_off, w.o, w.d);
    else
        hipLaunchKernelGGL(k_count<RAYS_GIVEN>, dim3(nb), dim3(256), 0, st, src, p, N, w.ray_off, w.o, w.d);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned ns = blocks_for(N, SCAN_TILE);
    hipLaunchKernelGGL(k_scan_reduce, dim3(ns), dim3(1024), 0, st, w.ray_off, N, w.scan);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, w.scan, (int)ns, w.ray_off + N);
    hipLaunchKernelGGL(k_scan_down, dim3(ns), dim3(1024), 0, st, w.ray_off, N, w.scan);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const float* o = src.mode == RAYS_GIVEN ? src.o : w.o;
    const float* d = src.mode == RAYS_GIVEN ? src.d : w.d;
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(N, 256)), dim3(256), 0, st, p, N, o, d, w.ray_off, w.t_mid, w.delta,
                       w.ray, w.field, voxel_out);
    return hipGetLastError();
}

hipError_t launch_labels(const float* occ, const int32_t* fmap, float thr, int64_t nvox, int n_fields,
                         int16_t* labels, hipStream_t st) {
    int32_t* bad = nullptr;
    hipError_t e = hipMallocAsync((void**)&bad, sizeof(int32_t), st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, bad, 1);
    hipLaunchKernelGGL(k_labels, dim3(blocks_for(nvox, 256)), dim3(256), 0, st, occ, fmap, thr, nvox, n_fields,
                       labels, bad);
    e = hipGetLastError();
    int32_t hb = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hb, bad, sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFreeAsync(bad, st);
    if (e != hipSuccess) return e;
    return hb ? hipErrorInvalidValue : hipSuccess;
}

}  // namespace r360
