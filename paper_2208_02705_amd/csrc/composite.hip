// Volume-rendering compositing (Sec. 3.2, Eq.4 and Eq.5), its backward, the
// L2 photometric loss of fine-tuning (Sec. 4.2) and Adam (Sec. 6.3).
//
// Per ray, samples are contiguous and in t order (sample.hip). With
// tau_i = sigma_i delta_i the transmittance is kept as the FP32 prefix sum
// logT_i = -sum_{k<i} tau_k, alpha_i = -expm1(-tau_i), w_i = exp(logT_i) alpha_i,
// C = sum w_i c_i, D = sum w_i t_i, A = sum w_i. No background colour.
#include <climits>

#include "r360_internal.h"

namespace r360 {

namespace {

// exp(-x) from the hardware exponential (relative error about x 2^-24 from
// the scaling by log2 e plus an ulp, far inside the FP32 render tolerance).
__device__ __forceinline__ float exp_neg(float x) { return __expf(-x); }

// alpha = 1 - exp(-x) for x >= 0: below 1/4 its Taylor series to x^7 in
// nested form (the first omitted term, x^8 / 8!, is below 4e-10, about 2e-9
// of the result), above from the hardware exponential (no cancellation:
// the result is at least 0.22).
constexpr double fct(int k) { return k <= 1 ? 1.0 : k * fct(k - 1); }
constexpr float kA2 = (float)(-1.0 / fct(2)), kA3 = (float)(1.0 / fct(3)), kA4 = (float)(-1.0 / fct(4)),
                kA5 = (float)(1.0 / fct(5)), kA6 = (float)(-1.0 / fct(6)), kA7 = (float)(1.0 / fct(7));
__device__ __forceinline__ float one_minus_exp_neg(float x) {
    float p = __builtin_fmaf(x, kA7, kA6);
    p = __builtin_fmaf(x, p, kA5);
    p = __builtin_fmaf(x, p, kA4);
    p = __builtin_fmaf(x, p, kA3);
    p = __builtin_fmaf(x, p, kA2);
    p = __builtin_fmaf(x, p, 1.0f) * x;
    return x < 0.25f ? p : 1.0f - __expf(-x);
}

// Sample-parallel compositing. Each wave owns `rpw` consecutive rays, whose
// samples form one contiguous range, and walks that range 64 samples at a
// time with one sample per lane (coalesced loads of every per-sample array,
// all lanes busy whatever the rays' lengths). Within a chunk the per-ray
// prefix of tau and the per-ray sums are segmented wave scans; a ray that
// continues into the next chunk carries its partial sums. The summation
// order is fixed, so results are deterministic.

// Wave-level data movement with DPP (no LDS traffic): row_shr:d within rows
// of 16 lanes, row_bcast:15 / row_bcast:31 across rows, wave_shr:1 and
// wave_shl:1 by one lane. Lanes without a source (or outside row_mask) get
// `old`.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dppf(float old, float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old), __builtin_bit_cast(int, v),
                                                                 CTRL, ROW_MASK, 0xf, false));
}
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ int dppi(int old, int v) {
    return __builtin_amdgcn_update_dpp(old, v, CTRL, ROW_MASK, 0xf, false);
}
constexpr int DPP_ROW_SHR = 0x110, DPP_WAVE_SHL1 = 0x130, DPP_WAVE_SHR1 = 0x138, DPP_BCAST15 = 0x142,
              DPP_BCAST31 = 0x143;

// Inclusive sum over the lanes of this lane's segment up to this lane
// (`seg` = first lane of the segment): in-row Kogge-Stone steps, then the
// row totals of rows 0 and 2 into rows 1 and 3, then that of rows 0-1 into
// rows 2-3, each added only where it lies in the lane's segment.
__device__ __forceinline__ float seg_scan(float v, int lane, int seg) {
    float t;
    t = dppf<DPP_ROW_SHR + 1>(0.0f, v); if (lane - 1 >= seg) v += t;
    t = dppf<DPP_ROW_SHR + 2>(0.0f, v); if (lane - 2 >= seg) v += t;
    t = dppf<DPP_ROW_SHR + 4>(0.0f, v); if (lane - 4 >= seg) v += t;
    t = dppf<DPP_ROW_SHR + 8>(0.0f, v); if (lane - 8 >= seg) v += t;
    t = dppf<DPP_BCAST15, 0xa>(0.0f, v); if (seg < (lane & ~15)) v += t;
    t = dppf<DPP_BCAST31, 0xc>(0.0f, v); if (seg < 32) v += t;
    return v;
}

// Inclusive max over lanes 0..lane (values >= 0).
__device__ __forceinline__ int max_scan(int v) {
    v = max(v, dppi<DPP_ROW_SHR + 1>(0, v));
    v = max(v, dppi<DPP_ROW_SHR + 2>(0, v));
    v = max(v, dppi<DPP_ROW_SHR + 4>(0, v));
    v = max(v, dppi<DPP_ROW_SHR + 8>(0, v));
    v = max(v, dppi<DPP_BCAST15, 0xa>(0, v));
    v = max(v, dppi<DPP_BCAST31, 0xc>(0, v));
    return v;
}

__device__ __forceinline__ float lane63(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

// Segment bookkeeping of one chunk: ray id per lane (INT_MAX past the
// range), segment start, whether the lane's segment continues the carried
// ray, whether the lane holds its ray's last sample. `next_first` is the ray
// of the sample after the chunk (INT_MAX if none).
struct ChunkSeg {
    int ray, seg;
    bool valid, cont, ends;
};

__device__ __forceinline__ ChunkSeg chunk_seg(int ray, bool valid, int next_first, int lane, int c_ray) {
    ChunkSeg c;
    c.valid = valid;
    c.ray = ray;
    // lane 0 compares with the carried ray, lane 63 with the next chunk's first
    const int prev = dppi<DPP_WAVE_SHR1>(c_ray, c.ray);
    const bool head = c.ray != prev;
    c.seg = max_scan(head ? lane : 0);
    c.cont = c.seg == 0 && __builtin_amdgcn_readlane(c.ray, 0) == c_ray;
    const int nxt = dppi<DPP_WAVE_SHL1>(next_first, c.ray);
    c.ends = c.valid && nxt != c.ray;
    return c;
}

// Per-lane inputs of one 64-sample chunk; a wave loads CPB chunks at once so
// that several chunks' loads are in flight together.
constexpr int CPB = 4;
struct ChunkIn {
    int ray;
    bool valid;
    float sg, dl, q0, q1, q2, tm;
};

__device__ __forceinline__ ChunkIn load_chunk(const int32_t* __restrict__ ray, const float* __restrict__ sigma,
                                              const float* __restrict__ rgb, const float* __restrict__ t_mid,
                                              const float* __restrict__ delta, int64_t cap, int s, int sb) {
    ChunkIn c;
    c.valid = s < sb;
    const int i = c.valid ? s : sb - 1;     // in-range stand-in
    c.ray = c.valid ? ray[i] : INT_MAX;
    c.sg = sigma[i];
    c.dl = delta[i];
    c.q0 = rgb[i]; c.q1 = rgb[cap + i]; c.q2 = rgb[2 * cap + i];
    c.tm = t_mid ? t_mid[i] : 0.0f;
    return c;
}

__device__ __forceinline__ void zero_empty_rays(const int32_t* __restrict__ off, int64_t N, int64_t r0, int64_t r1,
                                                int lane, float* out_rgb, float* depth, float* opacity) {
    for (int64_t r = r0 + lane; r < r1; r += 64) {
        if (off[r] != off[r + 1]) continue;
        if (out_rgb) { out_rgb[r] = 0.0f; out_rgb[N + r] = 0.0f; out_rgb[2 * N + r] = 0.0f; }
        if (depth) depth[r] = 0.0f;
        if (opacity) opacity[r] = 0.0f;
    }
}

__global__ __launch_bounds__(256) void k_composite(const int32_t* __restrict__ off, const int32_t* __restrict__ ray,
                                                   int64_t N, int64_t cap, int rpw, const float* __restrict__ sigma,
                                                   const float* __restrict__ rgb, const float* __restrict__ t_mid,
                                                   const float* __restrict__ delta, float* __restrict__ out_rgb,
                                                   float* __restrict__ depth, float* __restrict__ opacity) {
    const int lane = threadIdx.x & 63;
    const int64_t r0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * rpw;
    if (r0 >= N) return;
    const int64_t r1 = min(r0 + rpw, N);
    zero_empty_rays(off, N, r0, r1, lane, out_rgb, depth, opacity);
    const int sa = off[r0], sb = off[r1];
    // carried partial sums of a ray that continues from the previous chunk
    int c_ray = -1;
    float cS = 0.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, cD = 0.0f, cA = 0.0f;
    for (int blk = sa; blk < sb; blk += 64 * CPB) {
        ChunkIn in[CPB];
#pragma unroll
        for (int u = 0; u < CPB; ++u) in[u] = load_chunk(ray, sigma, rgb, t_mid, delta, cap, blk + 64 * u + lane, sb);
        const int after = blk + 64 * CPB < sb ? ray[blk + 64 * CPB] : INT_MAX;
#pragma unroll
        for (int u = 0; u < CPB; ++u) {
            if (blk + 64 * u >= sb) break;
            const int next_first = u + 1 < CPB ? __builtin_amdgcn_readlane(in[u + 1 < CPB ? u + 1 : u].ray, 0) : after;
            const ChunkSeg cs = chunk_seg(in[u].ray, in[u].valid, next_first, lane, c_ray);
            const float tau = cs.valid ? in[u].sg * in[u].dl : 0.0f;
            // S = sum of tau over the ray's earlier samples (log-space transmittance)
            const float incl = seg_scan(tau, lane, cs.seg);
            float S = dppf<DPP_WAVE_SHR1>(0.0f, incl);
            if (lane == cs.seg) S = 0.0f;
            if (cs.cont) S += cS;
            const float w = cs.valid ? exp_neg(S) * one_minus_exp_neg(tau) : 0.0f;
            float a0 = seg_scan(w * in[u].q0, lane, cs.seg), a1 = seg_scan(w * in[u].q1, lane, cs.seg);
            float a2 = seg_scan(w * in[u].q2, lane, cs.seg), aD = seg_scan(w * in[u].tm, lane, cs.seg);
            float aA = seg_scan(w, lane, cs.seg);
            if (cs.cont) { a0 += c0; a1 += c1; a2 += c2; aD += cD; aA += cA; }
            if (cs.ends) {
                if (out_rgb) { out_rgb[cs.ray] = a0; out_rgb[N + cs.ray] = a1; out_rgb[2 * N + cs.ray] = a2; }
                if (depth) depth[cs.ray] = aD;
                if (opacity) opacity[cs.ray] = aA;
            }
            // lane 63's ray continues into the next chunk unless it ended here
            const bool open = __builtin_amdgcn_readlane(cs.valid && !cs.ends ? 1 : 0, 63) != 0;
            c_ray = open ? __builtin_amdgcn_readlane(cs.ray, 63) : -1;
            cS = lane63(S + tau);
            c0 = lane63(a0); c1 = lane63(a1); c2 = lane63(a2); cD = lane63(aD); cA = lane63(aA);
        }
    }
}

// Compositing over the slot layout: one lane per ray (64 rays per wave),
// walking its samples in t order; the lanes of a wave read sample k of their
// rays from one contiguous 256-byte run, so every load is coalesced. Loads
// are issued four samples at a time, only for the lanes whose ray still has
// those samples. The sums run in sample order, as in the
// definition.
constexpr int CB = 4;
constexpr int CBB = 8;   // backward: training batches leave about one wave per SIMD, so more loads per batch

// The training loss L = 1/(3N) sum (C - C*)^2, split over the kernels that
// already touch the rays: the forward compositing writes dL/dC = 2 (C - C*)
// / (3N) per ray and channel and one partial sum per block of 256 rays (a
// fixed tree order), and block 0 of the compositing backward adds the
// partials (a fixed order again).
struct LossOut {
    const float* target;   // [3][N]
    float* grad;           // [3][N]
    float* part;           // [blocks of the forward compositing]
};
__device__ __forceinline__ float block_sum256(float v) {
    __shared__ float red[256];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    const float r = red[0];
    __syncthreads();
    return r;
}

// One lane per ray over the slot layout. CONT: the second pass of early
// termination: lane i composites the slots of continued ray i and adds them
// to the saved sums of the original ray list[i] (the same operations in the
// same order as one pass over all its samples). Otherwise lane i is ray i,
// starting from zero; with `state` set the final sums are also saved
// ([6][N]: C0, C1, C2, depth, opacity, S). Outputs go to the original ray.
// The compositing of one ray (lane i); returns its squared colour error
// when lo is set (and writes the loss gradient), else 0.
template <bool CONT>
__device__ __forceinline__ float composite_one(int64_t i, const int32_t* __restrict__ cnt, int64_t cap, int smax,
                                               const float* __restrict__ sigma, const float* __restrict__ rgb,
                                               const float* __restrict__ t_mid, const float* __restrict__ delta,
                                               const int32_t* __restrict__ list, int64_t N, float* __restrict__ state,
                                               float* __restrict__ out_rgb, float* __restrict__ depth,
                                               float* __restrict__ opacity, const LossOut* lo) {
    const int64_t r = CONT ? (int64_t)list[i] : i;
    const int c = cnt[i];
    // slot indices stay below 2^30: 32-bit offsets from each array's base
    const unsigned base = (unsigned)((i & ~int64_t(63)) * smax + (i & 63));
    const float* rgb1 = rgb + cap;
    const float* rgb2 = rgb + 2 * cap;
    float S = 0.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, D = 0.0f, A = 0.0f;
    if constexpr (CONT) {
        c0 = state[r]; c1 = state[N + r]; c2 = state[2 * N + r];
        D = state[3 * N + r]; A = state[4 * N + r]; S = state[5 * N + r];
    }
    for (int k = 0; k < c; k += CB) {
        float sg[CB], dl[CB], tm[CB], q0[CB], q1[CB], q2[CB];
#pragma unroll
        for (int u = 0; u < CB; ++u) {
            if (k + u < c) {
                const unsigned j = base + 64u * (unsigned)(k + u);
                sg[u] = ld32(sigma, j); dl[u] = ld32(delta, j); tm[u] = ld32(t_mid, j);
                q0[u] = ld32(rgb, j); q1[u] = ld32(rgb1, j); q2[u] = ld32(rgb2, j);
            } else {
                sg[u] = 0.f; dl[u] = 0.f; tm[u] = 0.f; q0[u] = 0.f; q1[u] = 0.f; q2[u] = 0.f;
            }
        }
#pragma unroll
        for (int u = 0; u < CB; ++u) {
            if (k + u < c) {
                const float tau = sg[u] * dl[u];
                const float w = exp_neg(S) * one_minus_exp_neg(tau);
                c0 += w * q0[u]; c1 += w * q1[u]; c2 += w * q2[u];
                D += w * tm[u];
                A += w;
                S += tau;
            }
        }
    }
    if (out_rgb) { out_rgb[r] = c0; out_rgb[N + r] = c1; out_rgb[2 * N + r] = c2; }
    if (depth) depth[r] = D;
    if (opacity) opacity[r] = A;
    if (!CONT && state) {
        state[r] = c0; state[N + r] = c1; state[2 * N + r] = c2;
        state[3 * N + r] = D; state[4 * N + r] = A; state[5 * N + r] = S;
    }
    float l = 0.0f;
    if (lo) {
        const float inv = 1.0f / (3.0f * (float)N);
        const float cc[3] = {c0, c1, c2};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float diff = cc[k] - lo->target[k * N + r];
            l += diff * diff;
            lo->grad[k * N + r] = 2.0f * diff * inv;
        }
    }
    return l;
}

// LOSS (training, not with CONT): also the loss gradient and the block's
// loss partial (LossOut); every thread of the block then reaches the sum.
template <bool CONT, bool LOSS = false>
__global__ __launch_bounds__(256) void k_composite_slots(const int32_t* __restrict__ cnt, int64_t n, int64_t cap,
                                                         int smax, const float* __restrict__ sigma,
                                                         const float* __restrict__ rgb, const float* __restrict__ t_mid,
                                                         const float* __restrict__ delta,
                                                         const int32_t* __restrict__ list, int64_t N,
                                                         float* __restrict__ state, float* __restrict__ out_rgb,
                                                         float* __restrict__ depth, float* __restrict__ opacity,
                                                         LossOut lo = LossOut{}) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if constexpr (LOSS) {
        float l = 0.0f;
        if (i < n) l = composite_one<CONT>(i, cnt, cap, smax, sigma, rgb, t_mid, delta, list, N, state, out_rgb, depth,
                                           opacity, &lo);
        const float sum = block_sum256(l);
        if (threadIdx.x == 0) lo.part[blockIdx.x] = sum;
        return;
    }
    if (i >= n) return;
    composite_one<CONT>(i, cnt, cap, smax, sigma, rgb, t_mid, delta, list, N, state, out_rgb, depth, opacity, nullptr);
}

// Early termination: the rays that continue after their first K samples are
// those that emitted all K and whose transmittance exp(-S) is still at least
// eps. The list order (atomic) affects no result: every ray is composited on
// its own and every sample's field MLP output is independent of its batch.
__global__ __launch_bounds__(256) void k_term_select(int64_t N, const int32_t* __restrict__ cnt, int K,
                                                     const float* __restrict__ S, float eps,
                                                     int32_t* __restrict__ list, int32_t* __restrict__ n2) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    if (cnt[r] == K && exp_neg(S[r]) >= eps) list[atomicAdd(n2, 1)] = (int32_t)r;
}

__global__ void k_term_zero(int32_t* __restrict__ n2) { *n2 = 0; }

// The continued rays' origins and directions, [3][n2] each.
__global__ __launch_bounds__(256) void k_term_gather(int64_t n2, const int32_t* __restrict__ list,
                                                     const float* __restrict__ ro, const float* __restrict__ rd,
                                                     int64_t N, float* __restrict__ o2, float* __restrict__ d2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n2) return;
    const int64_t r = list[i];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        o2[a * n2 + i] = ro[a * N + r];
        d2[a * n2 + i] = rd[a * N + r];
    }
}

// Backward over the slot layout, one lane per ray:
//   dL/dc_i = w_i g,  dL/dsigma_i = delta_i [T_{i+1} (c_i . g) - ((C - C_{<=i}) . g)],
// with C - C_{<=i} a difference of identically computed partial sums
// (exactly 0 after the last sample). HAVE_C: C is the forward pass's colour
// (crgb [3][N]), whose accumulation is the same operations in the same
// order; otherwise a first pass recomputes it.
// With loss set, block 0 first adds the forward compositing's nb loss
// partials (the loss's last step).
template <bool HAVE_C>
__global__ __launch_bounds__(256) void k_composite_bwd_slots(const int32_t* __restrict__ cnt, int64_t N, int64_t cap,
                                                             int smax, const float* __restrict__ sigma,
                                                             const float* __restrict__ rgb,
                                                             const float* __restrict__ delta,
                                                             const float* __restrict__ grad,
                                                             const float* __restrict__ crgb, float* __restrict__ dsigma,
                                                             float* __restrict__ drgb, const float* __restrict__ lpart,
                                                             int nb, float* __restrict__ loss) {
    if (loss && blockIdx.x == 0) {
        float sp = 0.0f;
        for (int k = threadIdx.x; k < nb; k += 256) sp += lpart[k];
        const float tot = block_sum256(sp);
        if (threadIdx.x == 0) *loss = tot / (3.0f * (float)N);
    }
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    const int c = cnt[r];
    const unsigned base = (unsigned)((r & ~int64_t(63)) * smax + (r & 63));
    const float* rgb1 = rgb + cap;
    const float* rgb2 = rgb + 2 * cap;
    float* drgb1 = drgb + cap;
    float* drgb2 = drgb + 2 * cap;
    const float g0 = grad[r], g1 = grad[N + r], g2 = grad[2 * N + r];
    float C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    if constexpr (HAVE_C) { C0 = crgb[r]; C1 = crgb[N + r]; C2 = crgb[2 * N + r]; }
    for (int pass = HAVE_C ? 1 : 0; pass < 2; ++pass) {
        float S = 0.0f, P0 = 0.0f, P1 = 0.0f, P2 = 0.0f;
        for (int k = 0; k < c; k += CBB) {
            float sg[CBB], dl[CBB], q0[CBB], q1[CBB], q2[CBB];
#pragma unroll
            for (int u = 0; u < CBB; ++u) {
                const unsigned i = base + 64u * (unsigned)min(k + u, c - 1);
                sg[u] = ld32(sigma, i); dl[u] = ld32(delta, i);
                q0[u] = ld32(rgb, i); q1[u] = ld32(rgb1, i); q2[u] = ld32(rgb2, i);
            }
#pragma unroll
            for (int u = 0; u < CBB; ++u) {
                if (k + u < c) {
                    const float tau = sg[u] * dl[u];
                    const float w = exp_neg(S) * one_minus_exp_neg(tau);
                    P0 += w * q0[u]; P1 += w * q1[u]; P2 += w * q2[u];
                    S += tau;
                    if (pass == 1) {
                        const unsigned i = base + 64u * (unsigned)(k + u);
                        const float cg = q0[u] * g0 + q1[u] * g1 + q2[u] * g2;
                        const float rg = (C0 - P0) * g0 + (C1 - P1) * g1 + (C2 - P2) * g2;
                        st32(dsigma, i, dl[u] * (exp_neg(S) * cg - rg));
                        st32(drgb, i, w * g0); st32(drgb1, i, w * g1); st32(drgb2, i, w * g2);
                    }
                }
            }
        }
        C0 = P0; C1 = P1; C2 = P2;
    }
}

// Loss L = 1/(3N) sum (C - C*)^2: per-block partial sums (fixed order), and
// dL/dC = 2 (C - C*) / (3N) per ray and channel.
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ rgb, const float* __restrict__ target, int64_t N,
                                              float* __restrict__ grad, float* __restrict__ part) {
    __shared__ float red[256];
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.0f;
    if (r < N) {
        const float inv = 1.0f / (3.0f * (float)N);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float diff = rgb[c * N + r] - target[c * N + r];
            l += diff * diff;
            grad[c * N + r] = 2.0f * diff * inv;
        }
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_loss_final(const float* __restrict__ part, int nb, int64_t N, float* __restrict__ loss) {
    __shared__ float red[256];
    float s = 0.0f;
    for (int i = threadIdx.x; i < nb; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0] / (3.0f * (float)N);
}

// Backward of compositing, sample-parallel like the forward. With
// u_i = w_i (c_i . g) and g = dL/dC of the sample's ray:
//   dL/dc_i = w_i g,  dL/dsigma_i = delta_i [T_{i+1} (c_i . g) - sum_{j>i} u_j].
// Pass 1 sums u per ray (kept in LDS); pass 2 repeats the same scans, so the
// tail sum is the ray total minus an identically computed inclusive prefix
// (exactly 0 at the ray's last sample).
__global__ __launch_bounds__(256) void k_composite_bwd(const int32_t* __restrict__ off, const int32_t* __restrict__ ray,
                                                       int64_t N, int64_t cap, int rpw, const float* __restrict__ sigma,
                                                       const float* __restrict__ rgb, const float* __restrict__ delta,
                                                       const float* __restrict__ grad, float* __restrict__ dsigma,
                                                       float* __restrict__ drgb) {
    __shared__ float u_tot[4][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t r0 = ((int64_t)blockIdx.x * 4 + wv) * rpw;
    if (r0 >= N) return;
    const int64_t r1 = min(r0 + rpw, N);
    const int sa = off[r0], sb = off[r1];
    const int rb = (int)r0;
    for (int pass = 0; pass < 2; ++pass) {
        int c_ray = -1;
        float cS = 0.0f, cU = 0.0f;
        for (int blk = sa; blk < sb; blk += 64 * CPB) {
            ChunkIn in[CPB];
#pragma unroll
            for (int u = 0; u < CPB; ++u) in[u] = load_chunk(ray, sigma, rgb, nullptr, delta, cap, blk + 64 * u + lane, sb);
            const int after = blk + 64 * CPB < sb ? ray[blk + 64 * CPB] : INT_MAX;
#pragma unroll
            for (int u = 0; u < CPB; ++u) {
                if (blk + 64 * u >= sb) break;
                const int next_first = u + 1 < CPB ? __builtin_amdgcn_readlane(in[u + 1 < CPB ? u + 1 : u].ray, 0) : after;
                const ChunkSeg cs = chunk_seg(in[u].ray, in[u].valid, next_first, lane, c_ray);
                const int ry = cs.valid ? cs.ray : rb;
                const float dl = in[u].dl;
                const float tau = cs.valid ? in[u].sg * dl : 0.0f;
                const float q0 = in[u].q0, q1 = in[u].q1, q2 = in[u].q2;
                const float g0 = grad[ry], g1 = grad[N + ry], g2 = grad[2 * N + ry];
                const float incl = seg_scan(tau, lane, cs.seg);
                float S = dppf<DPP_WAVE_SHR1>(0.0f, incl);
                if (lane == cs.seg) S = 0.0f;
                if (cs.cont) S += cS;
                const float w = cs.valid ? exp_neg(S) * one_minus_exp_neg(tau) : 0.0f;
                const float cg = q0 * g0 + q1 * g1 + q2 * g2;
                float U = seg_scan(w * cg, lane, cs.seg);
                if (cs.cont) U += cU;
                const int s = blk + 64 * u + lane;
                if (pass == 0) {
                    if (cs.ends) u_tot[wv][cs.ray - rb] = U;
                } else if (cs.valid) {
                    const float tail = u_tot[wv][cs.ray - rb] - U;
                    const float Tn = exp_neg(S + tau);
                    dsigma[s] = dl * (Tn * cg - tail);
                    drgb[s] = w * g0;
                    drgb[cap + s] = w * g1;
                    drgb[2 * cap + s] = w * g2;
                }
                const bool open = __builtin_amdgcn_readlane(cs.valid && !cs.ends ? 1 : 0, 63) != 0;
                c_ray = open ? __builtin_amdgcn_readlane(cs.ray, 63) : -1;
                cS = lane63(S + tau);
                cU = lane63(U);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

// Rays per wave: 64 when there are enough rays, fewer (down to 1) so that
// small batches of long rays still spread over at least 8192 waves.
inline int rays_per_wave(int64_t N) {
    int rpw = 64;
    while (rpw > 1 && (N + rpw - 1) / rpw < 8192) rpw >>= 1;
    return rpw;
}
inline unsigned wave_blocks(int64_t N, int rpw) { return (unsigned)(((N + rpw - 1) / rpw + 3) / 4); }

hipError_t launch_composite(const Workspace& w, int64_t N, float* rgb, float* depth, float* opacity, hipStream_t st) {
    const int rpw = rays_per_wave(N);
    hipLaunchKernelGGL(k_composite, dim3(wave_blocks(N, rpw)), dim3(256), 0, st, w.ray_off, w.ray, N, w.cap, rpw,
                       w.sigma, w.rgb, w.t_mid, w.delta, rgb, depth, opacity);
    return hipGetLastError();
}

hipError_t launch_composite_slots(const Workspace& w, int64_t N, float* rgb, float* depth, float* opacity,
                                  hipStream_t st, float* state, const float* target, float* grad_rgb) {
    if (target)
        hipLaunchKernelGGL((k_composite_slots<false, true>), dim3(nblk(N)), dim3(256), 0, st, w.ray_off, N, w.cap,
                           w.slots.smax, w.sigma, w.rgb, w.t_mid, w.delta, nullptr, N, state, rgb, depth, opacity,
                           LossOut{target, grad_rgb, w.loss_part});
    else
        hipLaunchKernelGGL((k_composite_slots<false, false>), dim3(nblk(N)), dim3(256), 0, st, w.ray_off, N, w.cap,
                           w.slots.smax, w.sigma, w.rgb, w.t_mid, w.delta, nullptr, N, state, rgb, depth, opacity,
                           LossOut{});
    return hipGetLastError();
}

hipError_t launch_composite_continue(const Workspace& w2, const int32_t* list, int64_t N, const float* state,
                                     float* rgb, float* depth, float* opacity, hipStream_t st) {
    hipLaunchKernelGGL((k_composite_slots<true, false>), dim3(nblk(w2.N)), dim3(256), 0, st, w2.ray_off, w2.N,
                       w2.cap, w2.slots.smax, w2.sigma, w2.rgb, w2.t_mid, w2.delta, list, N, const_cast<float*>(state),
                       rgb, depth, opacity, LossOut{});
    return hipGetLastError();
}

hipError_t launch_term_select(const Workspace& w, int64_t N, int K, const float* S, float eps, int32_t* list,
                              int32_t* n2, hipStream_t st) {
    hipLaunchKernelGGL(k_term_zero, dim3(1), dim3(1), 0, st, n2);
    hipLaunchKernelGGL(k_term_select, dim3(nblk(N)), dim3(256), 0, st, N, w.ray_off, K, S, eps, list, n2);
    return hipGetLastError();
}

hipError_t launch_term_gather(int64_t n2, const int32_t* list, const float* ro, const float* rd, int64_t N, float* o2,
                              float* d2, hipStream_t st) {
    hipLaunchKernelGGL(k_term_gather, dim3(nblk(n2)), dim3(256), 0, st, n2, list, ro, rd, N, o2, d2);
    return hipGetLastError();
}

hipError_t launch_composite_backward_slots(const Workspace& w, int64_t N, const float* grad_rgb, const float* crgb,
                                           float* loss, hipStream_t st) {
    const int nb = (int)nblk(N);
    if (crgb)
        hipLaunchKernelGGL(k_composite_bwd_slots<true>, dim3(nb), dim3(256), 0, st, w.ray_off, N, w.cap,
                           w.slots.smax, w.sigma, w.rgb, w.delta, grad_rgb, crgb, w.dsigma, w.drgb, w.loss_part, nb,
                           loss);
    else
        hipLaunchKernelGGL(k_composite_bwd_slots<false>, dim3(nb), dim3(256), 0, st, w.ray_off, N, w.cap,
                           w.slots.smax, w.sigma, w.rgb, w.delta, grad_rgb, crgb, w.dsigma, w.drgb, w.loss_part, nb,
                           loss);
    return hipGetLastError();
}

hipError_t launch_loss_grad(const Workspace& w, int64_t N, const float* rgb, const float* target, float* loss,
                            float* grad_rgb, hipStream_t st) {
    const unsigned nb = nblk(N);
    hipLaunchKernelGGL(k_loss, dim3(nb), dim3(256), 0, st, rgb, target, N, grad_rgb, w.loss_part);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, st, w.loss_part, (int)nb, N, loss);
    return hipGetLastError();
}

hipError_t launch_composite_backward(const Workspace& w, int64_t N, const float* grad_rgb, hipStream_t st) {
    const int rpw = rays_per_wave(N);
    hipLaunchKernelGGL(k_composite_bwd, dim3(wave_blocks(N, rpw)), dim3(256), 0, st, w.ray_off, w.ray, N, w.cap, rpw,
                       w.sigma, w.rgb, w.delta, grad_rgb, w.dsigma, w.drgb);
    return hipGetLastError();
}

hipError_t launch_adam(float* w, const float* g, float* m, float* v, int64_t n, int64_t step, float lr, float b1,
                       float b2, float eps, hipStream_t st) {
    const float c1 = (float)(1.0 - std::pow((double)b1, (double)step));
    const float c2 = (float)(1.0 - std::pow((double)b2, (double)step));
    hipLaunchKernelGGL(k_adam, dim3(nblk(n)), dim3(256), 0, st, w, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace r360
