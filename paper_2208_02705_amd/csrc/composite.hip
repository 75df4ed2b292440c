// Volume-rendering compositing (Sec. 3.2, Eq.4 and Eq.5), its backward, the
// L2 photometric loss of fine-tuning (Sec. 4.2) and Adam (Sec. 6.3).
//
// Per ray, samples are contiguous and in t order (sample.hip). With
// tau_i = sigma_i delta_i the transmittance is kept as the FP32 prefix sum
// logT_i = -sum_{k<i} tau_k, alpha_i = -expm1(-tau_i), w_i = exp(logT_i) alpha_i,
// C = sum w_i c_i, D = sum w_i t_i, A = sum w_i. No background colour.
#include "r360_internal.h"

namespace r360 {

namespace {

// Each wave owns 64 consecutive rays, whose samples are one contiguous
// range. The range is staged through LDS in chunks with coalesced loads;
// each lane then walks its own ray's samples from LDS. (Walking them straight
// from global memory would make every load instruction touch ~20 cache lines
// and thrash L1.)
constexpr int CCH = 512;                      // samples per staged chunk and wave

struct Stage6 { float s[CCH], dl[CCH], t[CCH], r[CCH], g[CCH], b[CCH]; };

// All loads of a chunk are issued before any LDS store, so the wave waits
// for memory once per chunk rather than once per 64 samples.
__device__ __forceinline__ void stage_chunk(Stage6& L, int base, int end, int lane, int64_t cap,
                                            const float* __restrict__ sigma, const float* __restrict__ rgb,
                                            const float* __restrict__ t_mid, const float* __restrict__ delta) {
    constexpr int IT = CCH / 64;
    float v[IT][6];
#pragma unroll
    for (int u = 0; u < IT; ++u) {
        const int i0 = base + lane + 64 * u;
        const int i = i0 < end ? i0 : base;           // base < end: an in-range stand-in
        v[u][0] = sigma[i];
        v[u][1] = delta[i];
        v[u][2] = t_mid ? t_mid[i] : 0.0f;
        v[u][3] = rgb[i];
        v[u][4] = rgb[cap + i];
        v[u][5] = rgb[2 * cap + i];
    }
#pragma unroll
    for (int u = 0; u < IT; ++u) {
        const int k = lane + 64 * u;
        if (base + k < end) {
            L.s[k] = v[u][0]; L.dl[k] = v[u][1]; L.t[k] = v[u][2];
            L.r[k] = v[u][3]; L.g[k] = v[u][4]; L.b[k] = v[u][5];
        }
    }
}

__global__ __launch_bounds__(256) void k_composite(const int32_t* __restrict__ off, int64_t N, int64_t cap,
                                                   const float* __restrict__ sigma, const float* __restrict__ rgb,
                                                   const float* __restrict__ t_mid, const float* __restrict__ delta,
                                                   float* __restrict__ out_rgb, float* __restrict__ depth,
                                                   float* __restrict__ opacity) {
    __shared__ Stage6 lds[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    Stage6& L = lds[wv];
    const int64_t r0 = ((int64_t)blockIdx.x * 4 + wv) * 64;
    if (r0 >= N) return;
    const int64_t r = r0 + lane;
    const bool live = r < N;
    const int wa = off[r0], wb = off[min(r0 + 64, N)];
    const int a = live ? off[r] : 0, b = live ? off[r + 1] : 0;
    float logT = 0.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, D = 0.0f, A = 0.0f;
    for (int base = wa; base < wb; base += CCH) {
        stage_chunk(L, base, wb, lane, cap, sigma, rgb, t_mid, delta);
        __builtin_amdgcn_wave_barrier();
        const int lo = max(a, base) - base, hi = min(b, base + CCH) - base;
        for (int k = lo; k < hi; ++k) {
            const float tau = L.s[k] * L.dl[k];
            const float w = expf(logT) * -expm1f(-tau);
            c0 += w * L.r[k];
            c1 += w * L.g[k];
            c2 += w * L.b[k];
            D += w * L.t[k];
            A += w;
            logT -= tau;
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (!live) return;
    if (out_rgb) { out_rgb[r] = c0; out_rgb[N + r] = c1; out_rgb[2 * N + r] = c2; }
    if (depth) depth[r] = D;
    if (opacity) opacity[r] = A;
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

// Backward of compositing. Pass 1 recomputes C; pass 2 repeats the same
// accumulation so that C - C_{<=i} is a difference of identical partial sums:
//   dL/dc_i = w_i g,  dL/dsigma_i = delta_i [T_{i+1} (c_i . g) - ((C - C_{<=i}) . g)].
// Both passes stage the wave's sample range through LDS as the forward does;
// pass 2 writes the per-sample gradients back through LDS, coalesced.
__global__ __launch_bounds__(256) void k_composite_bwd(const int32_t* __restrict__ off, int64_t N, int64_t cap,
                                                       const float* __restrict__ sigma, const float* __restrict__ rgb,
                                                       const float* __restrict__ delta, const float* __restrict__ grad,
                                                       float* __restrict__ dsigma, float* __restrict__ drgb) {
    __shared__ Stage6 lds[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    Stage6& L = lds[wv];
    const int64_t r0 = ((int64_t)blockIdx.x * 4 + wv) * 64;
    if (r0 >= N) return;
    const int64_t r = r0 + lane;
    const bool live = r < N;
    const int wa = off[r0], wb = off[min(r0 + 64, N)];
    const int a = live ? off[r] : 0, b = live ? off[r + 1] : 0;
    const float g0 = live ? grad[r] : 0.0f, g1 = live ? grad[N + r] : 0.0f, g2 = live ? grad[2 * N + r] : 0.0f;
    float logT = 0.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    for (int base = wa; base < wb; base += CCH) {
        stage_chunk(L, base, wb, lane, cap, sigma, rgb, nullptr, delta);
        __builtin_amdgcn_wave_barrier();
        const int lo = max(a, base) - base, hi = min(b, base + CCH) - base;
        for (int k = lo; k < hi; ++k) {
            const float tau = L.s[k] * L.dl[k];
            const float w = expf(logT) * -expm1f(-tau);
            C0 += w * L.r[k]; C1 += w * L.g[k]; C2 += w * L.b[k];
            logT -= tau;
        }
        __builtin_amdgcn_wave_barrier();
    }
    float P0 = 0.0f, P1 = 0.0f, P2 = 0.0f;
    logT = 0.0f;
    for (int base = wa; base < wb; base += CCH) {
        stage_chunk(L, base, wb, lane, cap, sigma, rgb, nullptr, delta);
        __builtin_amdgcn_wave_barrier();
        const int lo = max(a, base) - base, hi = min(b, base + CCH) - base;
        for (int k = lo; k < hi; ++k) {
            const float tau = L.s[k] * L.dl[k];
            const float w = expf(logT) * -expm1f(-tau);
            const float q0 = L.r[k], q1 = L.g[k], q2 = L.b[k];
            P0 += w * q0; P1 += w * q1; P2 += w * q2;
            logT -= tau;
            const float Tn = expf(logT);
            const float cg = q0 * g0 + q1 * g1 + q2 * g2;
            const float rg = (C0 - P0) * g0 + (C1 - P1) * g1 + (C2 - P2) * g2;
            // results overwrite the staged inputs of this sample (read above)
            L.s[k] = L.dl[k] * (Tn * cg - rg);
            L.r[k] = w * g0; L.g[k] = w * g1; L.b[k] = w * g2;
        }
        __builtin_amdgcn_wave_barrier();
        for (int k = lane; k < CCH && base + k < wb; k += 64) {
            const int i = base + k;
            dsigma[i] = L.s[k];
            drgb[i] = L.r[k]; drgb[cap + i] = L.g[k]; drgb[2 * cap + i] = L.b[k];
        }
        __builtin_amdgcn_wave_barrier();
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

inline unsigned nwblk(int64_t n) { return (unsigned)((n + 255) / 256); }   // 4 waves x 64 rays per block

hipError_t launch_composite(const Workspace& w, int64_t N, float* rgb, float* depth, float* opacity, hipStream_t st) {
    hipLaunchKernelGGL(k_composite, dim3(nwblk(N)), dim3(256), 0, st, w.ray_off, N, w.cap, w.sigma, w.rgb, w.t_mid,
                       w.delta, rgb, depth, opacity);
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
    hipLaunchKernelGGL(k_composite_bwd, dim3(nwblk(N)), dim3(256), 0, st, w.ray_off, N, w.cap, w.sigma, w.rgb,
                       w.delta, grad_rgb, w.dsigma, w.drgb);
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
