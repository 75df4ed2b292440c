// Stage I of Alg.1 (Sec. 4.1): progressive probabilistic occupancy from the
// global field's depth and uncertainty.
//
// Measurement per ray (k_depth_stats): with the Eq.5 weights w_i of its
// samples, opacity A = sum w_i, depth D = sum w_i t_i / A (the Eq.4 depth
// over normalised weights) and uncertainty U = sqrt(sum w_i (t_i - D)^2 / A);
// A = 0 gives D = U = 0. One wave per ray, samples in chunks of 64 lanes; the
// transmittance prefix is a wave scan carried across chunks.
//
// Update per sampling position (one pose), the logit form of Eq.6 with an
// inverse sensor model in the manner of the OctoMap framework the paper
// adopts; each voxel takes at most one measurement per pose:
//   k_occ_clear  zeroes the per-voxel hit and free marks (workspace);
//   k_occ_rays   walks each measuring ray's voxels (the sampler's FP32
//                traversal, every voxel, no occupancy test): a segment ending
//                at or before D - U marks its voxel free; the voxel whose
//                segment [t_in, t_out) holds D takes the hit logit
//                l_hit / (1 + U / voxel) by an atomic max of its (positive)
//                float bits, and the walk stops; voxels in the band between
//                D - U and the hit get nothing;
//   k_occ_apply  per voxel: l += hit if any ray ended there, else l_miss if
//                a ray passed freely; clamped to [l_min, l_max] (-2 and 3.5,
//                probability 0.12 to 0.97); probability 1 / (1 + e^-l).
// The marks are order-independent (max of positive bits, idempotent stores),
// so the update is deterministic.
//
// This file is compiled without floating-point contraction: the band edge
// D - U, the hit logit and the traversal are correctly rounded FP32
// operations in the order written, so a CPU implementation of the same
// specification marks the same voxels with the same values.
#include "r360_internal.h"

namespace r360 {

namespace {

__device__ __forceinline__ float mn(float a, float b) { return (b < a) ? b : a; }
__device__ __forceinline__ float mx(float a, float b) { return (a < b) ? b : a; }

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, WAVE);
    return v;
}

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ float wave_scan(float v, int lane) {
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) {
        const float u = __shfl_up(v, off, WAVE);
        if (lane >= off) v += u;
    }
    return v;
}

constexpr int DS_RAYS = 4;   // rays (waves) per block

__global__ __launch_bounds__(256) void k_depth_stats(const float* __restrict__ t, const float* __restrict__ delta,
                                                     const float* __restrict__ sigma, int64_t N, int S,
                                                     float* __restrict__ depth, float* __restrict__ uncert,
                                                     float* __restrict__ opacity) {
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * DS_RAYS + (threadIdx.x >> 6);
    if (r >= N) return;                                   // uniform per wave
    const int64_t base = r * S;
    // weight of sample k (lane's chunk position), carrying sum_{j<k} tau_j
    auto weight = [&](int k, float& carry, float& tk) -> float {
        const bool v = k < S;
        const float tau = v ? sigma[base + k] * delta[base + k] : 0.0f;
        tk = v ? t[base + k] : 0.0f;
        const float inc = wave_scan(tau, lane);
        float exc = __shfl_up(inc, 1, WAVE);
        if (lane == 0) exc = 0.0f;
        const float w = v ? expf(-(carry + exc)) * -expm1f(-tau) : 0.0f;
        carry += __shfl(inc, WAVE - 1, WAVE);
        return w;
    };
    float carry = 0.0f, a = 0.0f, dw = 0.0f;
    for (int k0 = 0; k0 < S; k0 += WAVE) {
        float tk;
        const float w = weight(k0 + lane, carry, tk);
        a += w;
        dw += w * tk;
    }
    const float A = wave_sum(a);
    const float D = A > 0.0f ? wave_sum(dw) / A : 0.0f;
    float var = 0.0f;
    if (A > 0.0f) {
        carry = 0.0f;
        for (int k0 = 0; k0 < S; k0 += WAVE) {
            float tk;
            const float w = weight(k0 + lane, carry, tk);
            const float e = tk - D;
            var += w * e * e;
        }
        var = wave_sum(var);
    }
    if (lane == 0) {
        depth[r] = D;
        uncert[r] = A > 0.0f ? sqrtf(var / A) : 0.0f;
        opacity[r] = A;
    }
}

struct OccArgs {
    int n0, n1, n2;
    float lo0, lo1, lo2;
    float voxel, inv_voxel;
    float near_, far_;
    float l_hit, l_miss, l_min, l_max, min_opacity;
    const float *o, *d, *depth, *uncert, *opacity;
    int64_t N;
    uint32_t* hit;      // per voxel: max hit logit as float bits (0 = none)
    uint8_t* freed;     // per voxel: 1 if a ray passed freely
    float* logit;       // [n2][n1][n0], in/out
    float* prob;        // optional
    int64_t nvox;
};

__global__ __launch_bounds__(256) void k_occ_clear(uint4* __restrict__ p, int64_t n16) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = uint4{0u, 0u, 0u, 0u};
}

__global__ __launch_bounds__(256) void k_occ_rays(OccArgs A) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= A.N) return;
    const float Dr = A.depth[r], Ur = A.uncert[r], Ar = A.opacity[r];
    if (!(Ar >= A.min_opacity) || !__builtin_isfinite(Dr) || !__builtin_isfinite(Ur) || !(Ur >= 0.0f)) return;
    const float o[3] = {A.o[r], A.o[A.N + r], A.o[2 * A.N + r]};
    const float d[3] = {A.d[r], A.d[A.N + r], A.d[2 * A.N + r]};
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (!(o[a] == o[a]) || !(d[a] == d[a])) return;   // NaN ray: no measurement
    const float edge = Dr - Ur;                            // free space ends here
    const float h = A.l_hit / (1.0f + Ur * A.inv_voxel);   // hit logit, weakened by the spread
    const uint32_t hb = __float_as_uint(h);

    // Set-up of the traversal specification (box clip, direction-aware entry
    // voxel, next-plane distances recomputed from the plane index).
    const float INF = __builtin_inff();
    const int n[3] = {A.n0, A.n1, A.n2};
    const float lo[3] = {A.lo0, A.lo1, A.lo2};
    float inv[3];
    bool act[3];
    float t0 = A.near_, t1 = A.far_;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float hi = lo[a] + (float)n[a] * A.voxel;
        act[a] = d[a] != 0.0f;
        if (act[a]) {
            inv[a] = 1.0f / d[a];
            const float ta = (lo[a] - o[a]) * inv[a];
            const float tb = (hi - o[a]) * inv[a];
            t0 = mx(t0, mn(ta, tb));
            t1 = mn(t1, mx(ta, tb));
        } else {
            inv[a] = 0.0f;
            if (!(o[a] >= lo[a] && o[a] < hi)) return;
        }
    }
    if (!(t0 < t1)) return;
    float pk0, pk1, pk2, sf0, sf1, sf2, tn0, tn1, tn2;
    int ds0, ds1, ds2;
    int lin = 0;
    {
        float pk[3], sf[3], tn[3];
        int ds[3];
        const int stride[3] = {1, A.n0, A.n0 * A.n1};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float p = __builtin_fmaf(t0, d[a], o[a]);
            const float q = (p - lo[a]) * A.inv_voxel;
            const float fq = __builtin_floorf(q);
            int i = (int)fq;
            if (q == fq && d[a] < 0.0f) i -= 1;
            i = i < 0 ? 0 : (i > n[a] - 1 ? n[a] - 1 : i);
            lin += i * stride[a];
            const bool up = d[a] > 0.0f;
            pk[a] = (float)(i + (up ? 1 : 0));
            sf[a] = up ? 1.0f : -1.0f;
            ds[a] = up ? stride[a] : -stride[a];
            tn[a] = act[a] ? (__builtin_fmaf(pk[a], A.voxel, lo[a]) - o[a]) * inv[a] : INF;
        }
        pk0 = pk[0]; pk1 = pk[1]; pk2 = pk[2];
        sf0 = sf[0]; sf1 = sf[1]; sf2 = sf[2];
        tn0 = tn[0]; tn1 = tn[1]; tn2 = tn[2];
        ds0 = ds[0]; ds1 = ds[1]; ds2 = ds[2];
    }
    const float o0 = o[0], o1 = o[1], o2 = o[2];
    const float iv0 = inv[0], iv1 = inv[1], iv2 = inv[2];
    const unsigned nvox = (unsigned)A.nvox;
    float t_in = t0;
    for (;;) {
        const bool c1 = tn1 < tn0;                         // nearest plane, ties to the lowest axis
        const float m01 = c1 ? tn1 : tn0;
        const bool c2 = tn2 < m01;
        const float tna = c2 ? tn2 : m01;
        const float t_out = mn(tna, t1);
        if (t_out > t_in) {                                // zero-length touches are skipped
            if (t_out <= edge) {
                A.freed[lin] = 1;
            } else if (Dr < t_out) {
                if (t_in <= Dr && hb != 0u) atomicMax(A.hit + lin, hb);
                break;
            }
        }
        const int lin_next = lin + (c2 ? ds2 : (c1 ? ds1 : ds0));
        // leaving the grid crosses a boundary plane, whose distance is that
        // axis's box exit >= t1, so the walk ends on the first test; the
        // index test keeps every store inside the grid regardless
        if (!(tna < t1) || (unsigned)lin_next >= nvox) break;
        t_in = mx(t_in, tna);
        const float pka = c2 ? pk2 : (c1 ? pk1 : pk0);
        const float sfa = c2 ? sf2 : (c1 ? sf1 : sf0);
        const float loa = c2 ? A.lo2 : (c1 ? A.lo1 : A.lo0);
        const float oa = c2 ? o2 : (c1 ? o1 : o0);
        const float ia = c2 ? iv2 : (c1 ? iv1 : iv0);
        const float pkn = pka + sfa;
        const float tnn = (__builtin_fmaf(pkn, A.voxel, loa) - oa) * ia;
        const bool x0 = !c1 && !c2, x1 = c1 && !c2;
        pk0 = x0 ? pkn : pk0; tn0 = x0 ? tnn : tn0;
        pk1 = x1 ? pkn : pk1; tn1 = x1 ? tnn : tn1;
        pk2 = c2 ? pkn : pk2; tn2 = c2 ? tnn : tn2;
        lin = lin_next;
    }
}

__global__ __launch_bounds__(256) void k_occ_apply(OccArgs A) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < A.nvox;
         v += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t hv = A.hit[v];
        const uint8_t fv = A.freed[v];
        float l = A.logit[v];
        if (hv != 0u || fv != 0) {
            l = hv != 0u ? l + __uint_as_float(hv) : l + A.l_miss;
            l = mn(mx(l, A.l_min), A.l_max);
            A.logit[v] = l;
        }
        if (A.prob) A.prob[v] = 1.0f / (1.0f + expf(-l));
    }
}

size_t up256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

size_t occupancy_workspace_bytes(int64_t nvox) { return up256((size_t)nvox * 4) + up256((size_t)nvox); }

hipError_t launch_depth_stats(const float* t, const float* delta, const float* sigma, int64_t N, int S,
                              float* depth, float* uncert, float* opacity, hipStream_t st) {
    const unsigned blocks = (unsigned)((N + DS_RAYS - 1) / DS_RAYS);
    hipLaunchKernelGGL(k_depth_stats, dim3(blocks), dim3(64 * DS_RAYS), 0, st, t, delta, sigma, N, S, depth, uncert,
                       opacity);
    return hipGetLastError();
}

hipError_t launch_occupancy_update(const r360_occ_desc* g, float* logit, float* prob, const float* o, const float* d,
                                   int64_t N, const float* depth, const float* uncert, const float* opacity,
                                   void* ws, hipStream_t st) {
    OccArgs A;
    A.n0 = g->n[0]; A.n1 = g->n[1]; A.n2 = g->n[2];
    A.lo0 = g->lo[0]; A.lo1 = g->lo[1]; A.lo2 = g->lo[2];
    A.voxel = g->voxel; A.inv_voxel = 1.0f / g->voxel;     // exact: power-of-two voxel
    A.near_ = g->near_; A.far_ = g->far_;
    A.l_hit = g->l_hit; A.l_miss = g->l_miss; A.l_min = g->l_min; A.l_max = g->l_max;
    A.min_opacity = g->min_opacity;
    A.o = o; A.d = d; A.depth = depth; A.uncert = uncert; A.opacity = opacity; A.N = N;
    A.nvox = (int64_t)g->n[0] * g->n[1] * g->n[2];
    char* base = static_cast<char*>(ws);
    A.hit = reinterpret_cast<uint32_t*>(base);
    A.freed = reinterpret_cast<uint8_t*>(base + up256((size_t)A.nvox * 4));
    A.logit = logit; A.prob = prob;
    const int64_t n16 = (int64_t)(occupancy_workspace_bytes(A.nvox) / 16);
    hipLaunchKernelGGL(k_occ_clear, dim3(1024), dim3(256), 0, st, reinterpret_cast<uint4*>(ws), n16);
    hipLaunchKernelGGL(k_occ_rays, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, A);
    const int64_t ab = std::min<int64_t>((A.nvox + 255) / 256, 4096);
    hipLaunchKernelGGL(k_occ_apply, dim3((unsigned)ab), dim3(256), 0, st, A);
    return hipGetLastError();
}

}  // namespace r360
