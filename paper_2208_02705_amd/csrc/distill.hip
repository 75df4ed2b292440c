// Distillation of the global field into the local fields (Sec. 4.2, Eq.7).
//
// Each local field k is fitted to the global field's density and colour at
// I_k points inside its own region:
//   L = sum_k (1/I_k) sum_{i of field k} [(sigma^k_i - sigma_i)^2 + |c^k_i - c_i|^2].
// The points ride the renderer's machinery as rays with one sample at t = 0
// (the sample position fma(0, d, x) is the point x itself, and the view
// direction d feeds the colour branch), in the slot layout with one slot per
// ray: routing by field, the grouped MLP forward, this file's loss, and the
// MLP backward with its deterministic per-field reduction. A point whose
// field id lies outside [0, n_fields) takes no part. The loss partials are
// summed per block in a fixed order, so loss and gradient are reproducible.
#include "r360_internal.h"

namespace r360 {

namespace {

// One sample per point at slot j = j (one-slot layout): t = 0, delta = 0,
// count 1 where the field id is valid.
__global__ __launch_bounds__(256) void k_dist_points(int64_t M, const int32_t* __restrict__ field, int F,
                                                     float* __restrict__ t, float* __restrict__ delta,
                                                     int32_t* __restrict__ fld, int32_t* __restrict__ count) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const int k = field[j];
    const bool ok = k >= 0 && k < F;
    t[j] = 0.0f;
    delta[j] = 0.0f;
    fld[j] = ok ? k : 0;
    count[j] = ok ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_dist_loss(int64_t M, int64_t cap, const int32_t* __restrict__ count,
                                                   const int32_t* __restrict__ fld,
                                                   const int32_t* __restrict__ field_start,
                                                   const float* __restrict__ sigma, const float* __restrict__ rgb,
                                                   const float* __restrict__ tsig, const float* __restrict__ trgb,
                                                   float* __restrict__ dsigma, float* __restrict__ drgb,
                                                   float* __restrict__ part) {
    __shared__ float red[256];
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.0f;
    if (j < M && count[j]) {
        const int k = fld[j];
        const float inv = 1.0f / (float)(field_start[k + 1] - field_start[k]);
        const float ds = sigma[j] - tsig[j];
        dsigma[j] = 2.0f * ds * inv;
        float s = ds * ds;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float dc = rgb[c * cap + j] - trgb[c * M + j];
            s += dc * dc;
            drgb[c * cap + j] = 2.0f * dc * inv;
        }
        l = s * inv;
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_dist_final(const float* __restrict__ part, int nb, float* __restrict__ loss) {
    __shared__ float red[256];
    float s = 0.0f;
    for (int i = threadIdx.x; i < nb; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = red[0];
}

}  // namespace

hipError_t launch_distill_points(const Workspace& w, int64_t M, const int32_t* field, int F, hipStream_t st) {
    const unsigned nb = (unsigned)((M + 255) / 256);
    hipLaunchKernelGGL(k_dist_points, dim3(nb), dim3(256), 0, st, M, field, F, w.t_mid, w.delta, w.field, w.ray_off);
    return hipGetLastError();
}

hipError_t launch_distill_loss(const Workspace& w, int64_t M, const float* tsig, const float* trgb, float* loss,
                               hipStream_t st) {
    const unsigned nb = (unsigned)((M + 255) / 256);
    hipLaunchKernelGGL(k_dist_loss, dim3(nb), dim3(256), 0, st, M, w.cap, w.ray_off, w.field, w.field_start, w.sigma,
                       w.rgb, tsig, trgb, w.dsigma, w.drgb, w.loss_part);
    hipLaunchKernelGGL(k_dist_final, dim3(1), dim3(256), 0, st, w.loss_part, (int)nb, loss);
    return hipGetLastError();
}

}  // namespace r360
