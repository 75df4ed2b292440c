// Ray generation and occupied-voxel sampling.
//
// Rays: equirect (Sec. 3.2, Eq.2 inverted at pixel centres, Eq.3) from
// per-resolution sine/cosine tables, pinhole viewports, or caller rays.
// Sampling: FP32 voxel traversal over a label grid; one midpoint sample per
// occupied voxel segment of positive length (Sec. 4.2 dense sampling of the
// occupied voxels; Sec. 5 ray casting over the labelled occupancy map).
//
// One traversal per ray writes sample k of ray r to slot
// (r - r % 64) * max_samples + 64 k + r % 64 of the staging arrays (lanes at
// the same k write neighbouring addresses) and its count. The render path
// consumes that slot layout directly; the compact form (launch_sample) adds
// an exclusive scan of the counts and a pass that moves each ray's samples to
// one contiguous run in t order at its offset. The render path also gathers
// the routing pass's per-field counts during the walk (RouteCounts).
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
        float oc0 = 0.0f, oc2 = 0.0f;   // stereo eye offset in the camera frame (equirect only)
        bool eye = false;
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
            if (s.eye != 0.0f) {      // omni-directional stereo: origin on the viewing circle, across the heading
                eye = true;
                oc0 = s.eye * cphi;
                oc2 = -(s.eye * sphi);
            }
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
            o[i] = eye ? R[3] + __builtin_fmaf(R[2], oc2, __builtin_fmaf(R[1], 0.0f, R[0] * oc0)) : R[3];
        }
    }
}

// Voxel traversal. Emits (t_mid, delta, voxel, field) for the first
// max_samples occupied segments, except the first P.skip of them (which are
// walked but not emitted; the rest are numbered from 0); returns the number
// emitted. Per step only the
// crossed axis's next-plane distance changes; the others are reused (their
// plane index did not change, so the recomputation would give the same bits).
//
// Sample k of ray r goes to slot base + 64 k, base = (r - r % 64) * S +
// r % 64 with S = max_samples - skip slots per ray: each wave of 64 rays
// stages into one contiguous block of 64 S slots, and lanes at the same k
// write neighbouring addresses (k < S, so slots stay below the workspace's
// sample capacity < 2^31).
//
// With `count` set, every emitted sample also adds one to its field's entry
// of the wave's LDS histogram h.
// With the routing's level ranges (RouteMap lr > 1) the counts go to the
// histogram of the range holding k: h advances by F at every ls-th sample.
struct SlotSink {
    int base;
    float *t, *dl;
    int32_t *fld, *vox;
    int32_t* h;
    bool count;
    int F, ls, bound;
    __device__ void emit(int k, float tm, float d, int lab, int lin) {
        const unsigned j = (unsigned)(base + 64 * k);
        st32(t, j, tm); st32(dl, j, d); st32(fld, j, (int32_t)lab);
        if (vox) st32(vox, j, (int32_t)lin);
        if (count) {
            if (k == bound) { h += F; bound += ls; }
            atomicAdd(h + lab, 1);
        }
    }
};

// MULTI: several samples per occupied segment (P.spv > 1); the single-sample
// form is a separate instantiation with the plain midpoint emission.
template <class Sink, bool MULTI>
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
    // Per axis: pk = index of the next plane to cross (as an exact float),
    // sf = +-1, tn = its distance, ds = signed step of the linear index.
    // Kept in scalars (not arrays): the per-step selection among the axes
    // must stay register selects.
    float pk0, pk1, pk2, sf0, sf1, sf2, tn0, tn1, tn2;
    int ds0, ds1, ds2;
    int lin = 0;
    {
        float pk[3], sf[3], tn[3];
        int ds[3];
        const int stride[3] = {1, P.n0, P.n0 * P.n1};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float p = __builtin_fmaf(t0, d[a], o[a]);
            const float q = (p - lo[a]) * P.inv_voxel;
            const float fq = __builtin_floorf(q);
            int i = (int)fq;
            if (q == fq && d[a] < 0.0f) i -= 1;
            i = i < 0 ? 0 : (i > n[a] - 1 ? n[a] - 1 : i);
            lin += i * stride[a];
            const bool up = d[a] > 0.0f;
            pk[a] = (float)(i + (up ? 1 : 0));
            sf[a] = up ? 1.0f : -1.0f;
            ds[a] = up ? stride[a] : -stride[a];
            tn[a] = act[a] ? (__builtin_fmaf(pk[a], P.voxel, lo[a]) - o[a]) * inv[a] : INF;
        }
        pk0 = pk[0]; pk1 = pk[1]; pk2 = pk[2];
        sf0 = sf[0]; sf1 = sf[1]; sf2 = sf[2];
        tn0 = tn[0]; tn1 = tn[1]; tn2 = tn[2];
        ds0 = ds[0]; ds1 = ds[1]; ds2 = ds[2];
    }
    const float o0 = o[0], o1 = o[1], o2 = o[2];
    // the grid corner in vector registers: the per-step fma(plane, voxel,
    // corner) then reads one scalar operand (the voxel edge), the most a
    // vector instruction may, instead of copying the corner in every step
    float lo0 = lo[0], lo1 = lo[1], lo2 = lo[2];
    asm volatile("" : "+v"(lo0), "+v"(lo1), "+v"(lo2));
    const float iv0 = inv[0], iv1 = inv[1], iv2 = inv[2];
    const unsigned nvox = (unsigned)P.n0 * (unsigned)P.n1 * (unsigned)P.n2;
    // labels read as unsigned 16-bit words: free labels (-1) become 0xFFFF,
    // field ids stay as they are
    const uint16_t* labels = reinterpret_cast<const uint16_t*>(P.labels);
    int count = 0;
    float t_in = t0;
    // The walk in two halves per step. The crossing out of a voxel (nearest
    // plane, ties to the lowest axis; its distance, the next voxel, whether
    // the walk goes on) depends only on the ray, so it is computed one voxel
    // ahead of the voxel being handled, and each label is requested two
    // voxels ahead: a load has two steps of arithmetic to arrive in. The
    // voxel being handled uses exactly the values the one-voxel-at-a-time
    // walk computes, in the same order.
    // R360_DDA_CROSS(S): the crossing out of the walk-ahead voxel `lin` into
    // set S (tna, tout, next, more), then the walk-ahead state moves on (the
    // crossed axis's next plane; unused once the walk has ended).
#define R360_DDA_CROSS(S)                                                            \
    {                                                                                \
        const bool c1 = tn1 < tn0;                                                   \
        const float m01 = c1 ? tn1 : tn0;                                            \
        const bool c2 = tn2 < m01;                                                   \
        S##tna = c2 ? tn2 : m01;                                                     \
        S##tout = mn(S##tna, t1);                                                    \
        S##next = lin + (c2 ? ds2 : (c1 ? ds1 : ds0));                               \
        S##more = S##tna < t1 && (unsigned)S##next < nvox;                           \
        const float pn0 = pk0 + sf0, pn1 = pk1 + sf1, pn2 = pk2 + sf2;               \
        const float tm0 = (__builtin_fmaf(pn0, P.voxel, lo0) - o0) * iv0;            \
        const float tm1 = (__builtin_fmaf(pn1, P.voxel, lo1) - o1) * iv1;            \
        const float tm2 = (__builtin_fmaf(pn2, P.voxel, lo2) - o2) * iv2;            \
        const bool x0 = !c1 && !c2, x1 = c1 && !c2;                                  \
        pk0 = x0 ? pn0 : pk0; tn0 = x0 ? tm0 : tn0;                                  \
        pk1 = x1 ? pn1 : pk1; tn1 = x1 ? tm1 : tn1;                                  \
        pk2 = c2 ? pn2 : pk2; tn2 = c2 ? tm2 : tn2;                                  \
        lin = S##next;                                                               \
    }
    // One step: voxel `cl` (label `cur`, crossing set C) is handled while the
    // crossing of the next voxel goes into set N and the label of the voxel
    // after it is requested into `nx2` (that voxel exists when both
    // crossings go on; otherwise a voxel known to exist is read instead).
    // Leaves the loop when the walk ends or the cap is reached. Unrolled six
    // times so that three label registers and two crossing sets rotate
    // without copies. (A macro, not a lambda: captured references would turn
    // the per-axis selects into loads through selected pointers.)
#define R360_DDA_STEP(cur, nx2, C, N)                                                \
    {                                                                                \
        R360_DDA_CROSS(N)                                                            \
        nx2 = ld32(labels, (unsigned)(C##more && N##more ? N##next : cl));           \
        __builtin_amdgcn_sched_barrier(0);                                           \
        const float t_out = C##tout;                                                 \
        const bool hit = t_out > t_in && cur < 0x8000;                               \
        if constexpr (!MULTI) {                                                      \
            if (hit && count >= P.skip)                                              \
                sink.emit(count - P.skip, (t_in + t_out) * 0.5f, t_out - t_in, (int)cur, cl); \
            count += hit ? 1 : 0;                                                    \
        } else if (hit) {                                                            \
            /* P.spv pieces cut at fma(j, length / k, t_in) */                       \
            const float piece = (t_out - t_in) / (float)P.spv;                       \
            float b0 = t_in;                                                         \
            for (int q = 0; q < P.spv; ++q) {                                        \
                const float b1 = q + 1 == P.spv ? t_out                              \
                                                : __builtin_fmaf((float)(q + 1), piece, t_in); \
                if (count >= P.skip)                                                 \
                    sink.emit(count - P.skip, (b0 + b1) * 0.5f, b1 - b0, (int)cur, cl); \
                b0 = b1;                                                             \
                if (++count == P.max_samples) break;                                 \
            }                                                                        \
        }                                                                            \
        if (!C##more || count == P.max_samples) break;                               \
        t_in = mx(t_in, C##tna);                                                     \
        cl = C##next;                                                                \
    }
    // Leaving the grid means crossing one of its boundary planes, whose
    // distance is that axis's box exit (the plane position is computed with
    // one rounding either way), which is >= t1: the walk ends on tna >= t1
    // first. The index test in `more` only guards the loads.
    int cl = lin;                                        // the voxel being handled
    float Atna, Atout, Btna, Btout;
    int Anext, Bnext;
    bool Amore, Bmore;
    uint16_t la = ld32(labels, (unsigned)lin), lb, lc = 0;
    R360_DDA_CROSS(A)                                    // the first voxel's crossing
    lb = ld32(labels, (unsigned)(Amore ? Anext : cl));
    for (;;) {
        R360_DDA_STEP(la, lc, A, B)
        R360_DDA_STEP(lb, la, B, A)
        R360_DDA_STEP(lc, lb, A, B)
        R360_DDA_STEP(la, lc, B, A)
        R360_DDA_STEP(lb, la, A, B)
        R360_DDA_STEP(lc, lb, B, A)
    }
#undef R360_DDA_STEP
#undef R360_DDA_CROSS
    return count > P.skip ? count - P.skip : 0;
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

// Pass 1: traversal. Per-ray sample counts go to ray_off[r], the samples to
// the staging slots; generated rays are stored for the later passes.
struct Staging {
    float* t; float* dl; int32_t* fld; int32_t* vox;
};

// Routing counts gathered during the walk: the number of samples of each
// field in every routing wave's unit (RouteMap in r360_internal.h), added
// into hist[f][w] (zeroed beforehand). hist == nullptr: not gathered here.
struct RouteCounts {
    int32_t* hist;
    int F, rw;
    RouteMap m;
};

template <int MODE, bool MULTI>
__global__ __launch_bounds__(256) void k_trace(RaySource src, DdaParams P, int64_t N, int32_t* __restrict__ cnt,
                                               float* __restrict__ o_ws, float* __restrict__ d_ws, Staging sg,
                                               RouteCounts rc) {
    extern __shared__ int32_t l_hist[];   // [4][lr][F] while counting
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool counting = rc.hist != nullptr;
    const int nh = rc.m.lr * rc.F;
    int32_t* h = l_hist + (threadIdx.x >> 6) * nh;
    if (counting) {
        for (int f = lane; f < nh; f += 64) h[f] = 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (r < N) {
        float o[3], d[3];
        make_ray<MODE>(src, N, r, o, d);
        if constexpr (MODE != RAYS_GIVEN) {
#pragma unroll
            for (int a = 0; a < 3; ++a) { o_ws[a * N + r] = o[a]; d_ws[a * N + r] = d[a]; }
        }
        SlotSink sink{(int)(r & ~int64_t(63)) * (P.max_samples - P.skip) + (int)(r & 63), sg.t, sg.dl, sg.fld, sg.vox,
                      h, counting, rc.F, rc.m.ls, rc.m.ls};
        cnt[r] = traverse<SlotSink, MULTI>(P, o, d, sink);
    }
    if (counting) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int64_t r0 = r - lane;             // the wave's first ray
        if (r0 < N) {
            const int64_t blk = r0 >> 6;
            for (int q = 0; q < rc.m.lr; ++q) {
                const int w = rc.m.lr == 1 ? (int)(blk / rc.m.per) : (int)(blk * rc.m.lr + q);
                for (int f = lane; f < rc.F; f += 64) {
                    const int v = h[q * rc.F + f];
                    if (v) atomicAdd(rc.hist + (int64_t)f * rc.rw + w, v);
                }
            }
        }
    }
}

// Pass 2 (after the scan): compaction. The 64 rays of a wave own one
// contiguous output range, assembled window by window in LDS: each lane
// copies its own ray's staging slots (lanes at the same k read neighbouring
// addresses of the wave's staging block) into the window, eight samples per batch so that
// the wave waits for memory once per batch; the window is then written out
// with coalesced stores.
constexpr int CWIN = 512;
constexpr int CBATCH = 8;

__global__ __launch_bounds__(256) void k_compact(int64_t N, int max_samples, const int32_t* __restrict__ off, Staging sg,
                                                 float* __restrict__ t_mid, float* __restrict__ delta,
                                                 int32_t* __restrict__ ray, int32_t* __restrict__ field,
                                                 int32_t* __restrict__ voxel) {
    __shared__ float l_t[4][CWIN], l_d[4][CWIN];
    __shared__ int32_t l_g[4][CWIN], l_v[4][CWIN];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t r0 = ((int64_t)blockIdx.x * 4 + wv) * 64;
    if (r0 >= N) return;
    const int64_t r = r0 + lane;
    const bool live = r < N;
    const int wa = off[r0], wb = off[min(r0 + 64, N)];
    const int mine = live ? off[r] - wa : 0;
    const int cnt = live ? off[r + 1] - off[r] : 0;
    const bool with_vox = voxel != nullptr;
    const int sbase = (int)r0 * max_samples + lane;
    for (int base = 0; base < wb - wa; base += CWIN) {
        const int k0 = max(0, base - mine), k1 = min(cnt, base + CWIN - mine);
        for (int k = k0; k < k1; k += CBATCH) {
            float tv[CBATCH], dv[CBATCH];
            int32_t fv[CBATCH], vv[CBATCH];
#pragma unroll
            for (int u = 0; u < CBATCH; ++u) {
                const int j = sbase + 64 * min(k + u, k1 - 1);   // past k1: repeat the last slot
                tv[u] = sg.t[j];
                dv[u] = sg.dl[j];
                fv[u] = sg.fld[j];
                vv[u] = with_vox ? sg.vox[j] : 0;
            }
#pragma unroll
            for (int u = 0; u < CBATCH; ++u) {
                if (k + u < k1) {
                    const int q = mine + k + u - base;
                    l_t[wv][q] = tv[u];
                    l_d[wv][q] = dv[u];
                    l_g[wv][q] = (lane << 16) | fv[u];
                    l_v[wv][q] = vv[u];
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int nwin = min(wb - wa - base, CWIN);
        const int at = wa + base;
        for (int q = lane; q < nwin; q += 64) {
            const int tag = l_g[wv][q];
            t_mid[at + q] = l_t[wv][q];
            delta[at + q] = l_d[wv][q];
            ray[at + q] = (int32_t)(r0 + (tag >> 16));
            field[at + q] = tag & 0xFFFF;
            if (with_vox) voxel[at + q] = l_v[wv][q];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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

// The traversal kernel for the ray source and the samples-per-voxel form.
__global__ __launch_bounds__(256) void k_fill_zero(int32_t* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

static hipError_t trace_any(const RaySource& src, const DdaParams& p, int64_t N, const Workspace& w, const Staging& sg,
                     unsigned nb, hipStream_t st, const RouteCounts& rc = RouteCounts{nullptr, 0, 1, RouteMap{1, 1, 1}}) {
    const size_t lds = rc.hist ? (size_t)4 * rc.m.lr * rc.F * sizeof(int32_t) : 0;
    if (p.spv > 1) {
        if (src.mode == RAYS_EQUIRECT)
            hipLaunchKernelGGL((k_trace<RAYS_EQUIRECT, true>), dim3(nb), dim3(256), lds, st, src, p, N, w.ray_off, w.o, w.d, sg, rc);
        else if (src.mode == RAYS_PINHOLE)
            hipLaunchKernelGGL((k_trace<RAYS_PINHOLE, true>), dim3(nb), dim3(256), lds, st, src, p, N, w.ray_off, w.o, w.d, sg, rc);
        else
            hipLaunchKernelGGL((k_trace<RAYS_GIVEN, true>), dim3(nb), dim3(256), lds, st, src, p, N, w.ray_off, w.o, w.d, sg, rc);
    } else {
        if (src.mode == RAYS_EQUIRECT)
            hipLaunchKernelGGL((k_trace<RAYS_EQUIRECT, false>), dim3(nb), dim3(256), lds, st, src, p, N, w.ray_off, w.o, w.d, sg, rc);
        else if (src.mode == RAYS_PINHOLE)
            hipLaunchKernelGGL((k_trace<RAYS_PINHOLE, false>), dim3(nb), dim3(256), lds, st, src, p, N, w.ray_off, w.o, w.d, sg, rc);
        else
            hipLaunchKernelGGL((k_trace<RAYS_GIVEN, false>), dim3(nb), dim3(256), lds, st, src, p, N, w.ray_off, w.o, w.d, sg, rc);
    }
    return hipGetLastError();
}

hipError_t launch_sample(const RaySource& src, const DdaParams& p, int64_t N, const Workspace& w,
                         int32_t* voxel_out, hipStream_t st) {
    const unsigned nb = blocks_for(N, 256);
    // staging slots live in the sigma/rgb arrays, which are not needed until the field MLPs run
    const Staging sg{w.sigma, w.rgb, reinterpret_cast<int32_t*>(w.rgb + w.cap),
                     voxel_out ? reinterpret_cast<int32_t*>(w.rgb + 2 * w.cap) : nullptr};
    hipError_t e = trace_any(src, p, N, w, sg, nb, st);
    if (e != hipSuccess) return e;
    const unsigned ns = blocks_for(N, SCAN_TILE);
    hipLaunchKernelGGL(k_scan_reduce, dim3(ns), dim3(1024), 0, st, w.ray_off, N, w.scan);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, w.scan, (int)ns, w.ray_off + N);
    hipLaunchKernelGGL(k_scan_down, dim3(ns), dim3(1024), 0, st, w.ray_off, N, w.scan);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_compact, dim3(nb), dim3(256), 0, st, N, p.max_samples, w.ray_off, sg, w.t_mid, w.delta, w.ray,
                       w.field, voxel_out);
    return hipGetLastError();
}

hipError_t launch_trace(const RaySource& src, const DdaParams& p, int64_t N, const Workspace& w, int F,
                        bool* counted, hipStream_t st) {
    const unsigned nb = blocks_for(N, 256);
    const Staging sg{w.t_mid, w.delta, w.field, nullptr};
    *counted = false;
    if (F < 1 || F > TRACE_COUNT_MAX_FIELDS) return trace_any(src, p, N, w, sg, nb, st);
    const int rw = route_waves(F);
    const RouteCounts rc{w.hist, F, rw, route_map(N, w.slots.smax, F)};
    const int64_t n = (int64_t)F * rw;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)std::min<int64_t>(1024, (n + 255) / 256)), dim3(256), 0, st, w.hist, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = trace_any(src, p, N, w, sg, nb, st, rc);
    *counted = e == hipSuccess;
    return e;
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
