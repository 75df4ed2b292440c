// Positional encoding + per-field tiny MLP as grouped MFMA GEMMs.
//
// Network (Sec. 3.1 Eq.1 in its tiny form, App. C; hidden width H):
//   h1 = relu(W1 g(x) + b1); h2 = relu(W2 h1 + b2);
//   sigma = softplus(ws h2 + bs); f = Wf h2 + bf;
//   h3 = relu(W3 [f ; g(d)] + b3); rgb = sigmoid(W4 h3 + b4).
//
// Mapping onto MFMA. Each layer is computed transposed, out^T = W x^T: the
// weights are the A operand (16 output rows per tile), 16 samples are the
// 16 columns. The 16x16 accumulator leaves lane l holding rows
// 4(l/16)+r, r = 0..3, of column l%16; the next layer's B operand wants
// lane l to hold a run of k values of column l%16. Instead of moving data,
// the next layer's weight columns are stored permuted so that the k slots a
// lane supplies are exactly the rows it already holds (see hidden_col()).
// The encoding is produced directly in B-operand order: lane l evaluates
// the encoding values of sample l%16 that its lane group l/16 owns
// (pe_slot_feature(), dir_slot_feature()).
// Layer biases ride along as an encoding slot holding 1 (L1, L3) or as the
// accumulator's initial value (L2, HEAD, L4).
//
// Work split: samples arrive sorted by field (route.hip). A block of four
// waves takes a contiguous slice of the sorted samples; for every field in
// its slice it stages that field's A fragments in LDS once, and each wave
// then processes chunks of 64 samples as four independent 16-column tiles,
// so every fragment read from LDS feeds four MFMAs and the four dependency
// chains keep the matrix unit busy while the encoding runs on the VALU.
// Block indices are remapped so that the blocks resident on one XCD (blocks
// are dealt round-robin over the 8 XCDs) take neighbouring slices, which
// mostly share fields and so their weights in that XCD's L2.
//
// Precision: BF16 or FP16 operands with FP32 accumulation, or FP32 (each
// K = 32 step as eight 16x16x4 FP32 MFMAs over the same fragment layout).
//
// Each layer's MFMA loop runs at raised wave priority (s_setprio 1) and the
// conversions at normal priority, so that a wave entering its MFMA phase
// issues ahead of waves doing vector work and the two units overlap more.
//
// Scheduling barriers separate the layers: without them the compiler hoists
// the LDS reads of every weight fragment of the network to the top of the
// chunk, which needs more than 256 registers and spills to scratch (the
// spill traffic then saturates HBM); with them each layer holds only its
// own fragments and the kernel runs three waves per SIMD without spills.
#include "r360_internal.h"

namespace r360 {

namespace {

template <int H>
__global__ __launch_bounds__(256) void k_repack(const float* __restrict__ weights, int F, __bf16* __restrict__ pbf,
                                                _Float16* __restrict__ ph, float* __restrict__ pf,
                                                float* __restrict__ bias) {
    using G = PackGeom<H>;
    constexpr FieldLayout L{H};
    const int64_t n16 = (int64_t)F * G::FRAGS16 * WAVE * 8;
    const int64_t nb = (int64_t)F * G::BIAS_FLOATS;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n16) {
        const int e = (int)(i & 7), lane = (int)((i >> 3) & 63);
        const int64_t fr_all = i >> 9;
        const int f = (int)(fr_all / G::FRAGS16), fr = (int)(fr_all % G::FRAGS16);
        const float v = packed_source16<H>(weights + (int64_t)f * L.P(), fr, lane, e);
        pbf[i] = (__bf16)v;
        ph[i] = (_Float16)v;
        pf[i] = v;
    }
    if (i < nb) {
        const int f = (int)(i / G::BIAS_FLOATS), k = (int)(i % G::BIAS_FLOATS);
        const int tile = k >> 4, v = k & 15;
        const float* w = weights + (int64_t)f * L.P();
        float b;
        if (tile < G::NT) b = w[L.b2() + 16 * tile + v];
        else if (tile < 2 * G::NT + 1) {
            const int row = 16 * (tile - G::NT) + v;
            b = row < H ? w[L.bf() + row] : (((row - H) & 3) == 0 ? w[L.bs()] : 0.0f);
        } else b = (v & 3) < 3 ? w[L.b4() + (v & 3)] : 0.0f;
        bias[i] = b;
    }
}

// ---------------------------------------------------------------------------
// Forward
// ---------------------------------------------------------------------------
// Output activations with the hardware exp/log/reciprocal (relative error
// ~1e-7, far inside every tolerance of the path).
__device__ __forceinline__ float softplusf(float z) { return fmaxf(z, 0.0f) + __logf(1.0f + __expf(-fabsf(z))); }
__device__ __forceinline__ float sigmoidf(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

struct FwdArgs {
    const int32_t* field_start;  // [F+1], field_start[F] = number of samples
    const int32_t* perm;         // sorted position -> slot
    const float* t_mid;          // [cap] slot layout
    SlotMap slots;
    const float* o[3];           // per component, [N] each
    const float* d[3];
    int64_t N, cap;
    int F;
    float c0, c1, c2, inv_h;
    const float* frames;         // [F][4] per-field (centre, 1 / half extent), or null: the scene's frame
    const void* pack;            // [F][FRAGS16][64] fragments of the chosen element type
    const float* bias;
    float* sigma;
    float* rgb0;                 // the three colour planes of rgb [3][cap]
    float* rgb1;
    float* rgb2;
};

__device__ __forceinline__ int find_field(const int32_t* start, int F, int pos) {
    int lo = 0, hi = F;            // largest f with start[f] <= pos
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= pos) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int xcd_block(int b, int nb) { return (b & 7) * (nb >> 3) + (b >> 3); }

// 16-sample column tiles per wave chunk and blocks per CU: 16-bit fragments
// take three tiles (146 VGPRs at hidden 64) so that three blocks, three waves
// per SIMD, are resident; FP32 fragments fill LDS with two blocks and keep
// four tiles.
template <typename T> constexpr int fwd_tiles() { return sizeof(T) == 2 ? 3 : 4; }
template <typename T> constexpr int fwd_blocks() { return sizeof(T) == 2 ? 3 : 2; }
constexpr int FWD_WAVES = 4;

template <int H, typename T>
__global__ __launch_bounds__(64 * FWD_WAVES, fwd_blocks<T>()) void k_fwd(FwdArgs a) {
    using G = PackGeom<H>;
    constexpr int NTILE = fwd_tiles<T>();
    constexpr int FCH = 16 * NTILE;        // samples per wave chunk
    using F8 = typename FragT<T>::type;
    constexpr int NT = G::NT, KH = G::KH16, FR = G::FRAGS16;
    extern __shared__ __attribute__((aligned(32))) char smem[];
    F8* lw = reinterpret_cast<F8*>(smem);                                          // [FR][64]
    float* lb = reinterpret_cast<float*>(smem + (size_t)FR * WAVE * sizeof(F8));   // [BIAS_FLOATS]
    const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15, wv = threadIdx.x >> 6;
    const int nb = gridDim.x;
    const int b = xcd_block(blockIdx.x, nb);
    const int S = a.field_start[a.F];
    constexpr int BCHK = FWD_WAVES * FCH;
    const int per = (((S + nb - 1) / nb) + BCHK - 1) / BCHK * BCHK;
    const int beg = min(S, b * per), end = min(S, beg + per);
    const F8* pk = reinterpret_cast<const F8*>(a.pack);
    for (int pos = beg; pos < end;) {
        const int f = find_field(a.field_start, a.F, pos);
        const int fend = min(end, a.field_start[f + 1]);
        // the encoding frame of this field
        const float cc[3] = {a.frames ? a.frames[4 * f] : a.c0, a.frames ? a.frames[4 * f + 1] : a.c1,
                             a.frames ? a.frames[4 * f + 2] : a.c2};
        const float inv_h = a.frames ? a.frames[4 * f + 3] : a.inv_h;
        __syncthreads();                               // the previous field's fragments are no longer read
        const F8* src = pk + (int64_t)f * FR * WAVE;
        for (int i = threadIdx.x; i < FR * WAVE; i += 64 * FWD_WAVES) lw[i] = src[i];
        for (int i = threadIdx.x; i < G::BIAS_FLOATS; i += 64 * FWD_WAVES) lb[i] = a.bias[(int64_t)f * G::BIAS_FLOATS + i];
        __syncthreads();
        const F8* W = lw + lane;
        const f32x4* bias = reinterpret_cast<const f32x4*>(lb) + g;
        // Gathered inputs of a chunk: the sample behind each column (orig),
        // its position input xh and direction dv. The next chunk's are
        // loaded while this chunk's layers run: permutation entries before
        // L1, t and ray before L2, the ray's o and d before L3 (each level
        // needs the previous one), so the loads have a layer of MFMA work to
        // arrive in.
        int c = pos + FCH * wv;
        // (no early exit here: every wave must reach the advance of pos and the
        // barriers of the next field segment)
        int orig[NTILE];
        float xh[NTILE][3], dv[NTILE][3];
        const int c0 = c < fend ? c : pos;             // an in-range stand-in when the wave has no chunk
#pragma unroll
        for (int n = 0; n < NTILE; ++n) {
            const int sp = c0 + 16 * n + j;
            orig[n] = ld32(a.perm, (unsigned)(sp < fend ? sp : c0));
        }
#pragma unroll
        for (int n = 0; n < NTILE; ++n) {
            const unsigned u = (unsigned)orig[n];
            const float t = ld32(a.t_mid, u);
            const unsigned r = ray_of_slot(u, a.slots);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                dv[n][k] = ld32(a.d[k], r);
                xh[n][k] = (__builtin_fmaf(t, dv[n][k], ld32(a.o[k], r)) - cc[k]) * inv_h;
            }
        }
        for (; c < fend; c += BCHK) {   // no iterations when this wave has no chunk here
            const int cn = c + BCHK;
            const bool has_next = cn < fend;
            int orig_n[NTILE];
            float t_n[NTILE];
            unsigned r_n[NTILE];
#pragma unroll
            for (int n = 0; n < NTILE; ++n) {
                const int sp = cn + 16 * n + j;
                orig_n[n] = ld32(a.perm, (unsigned)(has_next ? (sp < fend ? sp : cn) : c));
            }
            F8 x0[NTILE], x1[NTILE];
#pragma unroll
            for (int n = 0; n < NTILE; ++n) {
                float pe[16];
                pe_position<__is_same(T, float)>(g, xh[n], pe);
                x0[n] = pack8<T>(pe);
                x1[n] = pack8<T>(pe + 8);
            }
            f32x4 acc[NTILE][NT + 1];
            F8 hb[NTILE][KH];
            __builtin_amdgcn_sched_barrier(0);
            // L1: encoding -> h (bias in the encoding's constant slot)
            __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int ot = 0; ot < NT; ++ot) {
                const F8 A0 = W[(2 * ot) * WAVE], A1 = W[(2 * ot + 1) * WAVE];
#pragma unroll
                for (int n = 0; n < NTILE; ++n) {
                    acc[n][ot] = mma<T>(A0, x0[n], f32x4{0.f, 0.f, 0.f, 0.f});
                    acc[n][ot] = mma<T>(A1, x1[n], acc[n][ot]);
                }
            }
            __builtin_amdgcn_s_setprio(0);
#pragma unroll
            for (int n = 0; n < NTILE; ++n)
#pragma unroll
                for (int ks = 0; ks < KH; ++ks) hb[n][ks] = hand<T, true>(acc[n][2 * ks], acc[n][2 * ks + 1]);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int n = 0; n < NTILE; ++n) {
                const unsigned u = (unsigned)orig_n[n];
                t_n[n] = ld32(a.t_mid, u);
                r_n[n] = ray_of_slot(u, a.slots);
            }
            // L2: h -> h
            __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int ot = 0; ot < NT; ++ot) {
                const f32x4 bb = bias[ot * 4];
#pragma unroll
                for (int ks = 0; ks < KH; ++ks) {
                    const F8 A = W[(G::F_L1 + ot * KH + ks) * WAVE];
#pragma unroll
                    for (int n = 0; n < NTILE; ++n) acc[n][ot] = mma<T>(A, hb[n][ks], ks == 0 ? bb : acc[n][ot]);
                }
            }
            __builtin_amdgcn_s_setprio(0);
#pragma unroll
            for (int n = 0; n < NTILE; ++n)
#pragma unroll
                for (int ks = 0; ks < KH; ++ks) hb[n][ks] = hand<T, true>(acc[n][2 * ks], acc[n][2 * ks + 1]);
            __builtin_amdgcn_sched_barrier(0);
            // HEAD: h -> [f ; sigma] (sigma replicated in rows H, H+4, H+8, H+12)
            __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int ot = 0; ot < NT + 1; ++ot) {
                const f32x4 bb = bias[(NT + ot) * 4];
#pragma unroll
                for (int ks = 0; ks < KH; ++ks) {
                    const F8 A = W[(G::F_L1 + G::F_L2 + ot * KH + ks) * WAVE];
#pragma unroll
                    for (int n = 0; n < NTILE; ++n) acc[n][ot] = mma<T>(A, hb[n][ks], ks == 0 ? bb : acc[n][ot]);
                }
            }
            __builtin_amdgcn_s_setprio(0);
            float zs[NTILE];
#pragma unroll
            for (int n = 0; n < NTILE; ++n) {
                zs[n] = acc[n][NT][0];
#pragma unroll
                for (int ks = 0; ks < KH; ++ks) hb[n][ks] = hand<T, false>(acc[n][2 * ks], acc[n][2 * ks + 1]);
            }
            __builtin_amdgcn_sched_barrier(0);
            float o_n[NTILE][3], d_n[NTILE][3];
#pragma unroll
            for (int n = 0; n < NTILE; ++n)
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    o_n[n][k] = ld32(a.o[k], r_n[n]);
                    d_n[n][k] = ld32(a.d[k], r_n[n]);
                }
            // L3: [f ; g(d)] -> h (bias in the direction encoding's constant slot)
#pragma unroll
            for (int n = 0; n < NTILE; ++n) {
                float dpe[8];
                pe_direction<__is_same(T, float)>(g, dv[n], dpe);
                x0[n] = pack8<T>(dpe);
            }
            constexpr int O3 = G::F_L1 + G::F_L2 + G::F_HD;
            __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int ot = 0; ot < NT; ++ot) {
#pragma unroll
                for (int n = 0; n < NTILE; ++n) acc[n][ot] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < KH + 1; ++ks) {
                    const F8 A = W[(O3 + ot * (KH + 1) + ks) * WAVE];
#pragma unroll
                    for (int n = 0; n < NTILE; ++n) acc[n][ot] = mma<T>(A, ks < KH ? hb[n][ks < KH ? ks : 0] : x0[n], acc[n][ot]);
                }
            }
            __builtin_amdgcn_s_setprio(0);
#pragma unroll
            for (int n = 0; n < NTILE; ++n)
#pragma unroll
                for (int ks = 0; ks < KH; ++ks) hb[n][ks] = hand<T, true>(acc[n][2 * ks], acc[n][2 * ks + 1]);
            __builtin_amdgcn_sched_barrier(0);
            // L4: h -> rgb (rows 4g .. 4g+2 of every lane group g)
            __builtin_amdgcn_s_setprio(1);
            constexpr int O4 = O3 + G::F_L3;
            {
                const f32x4 bb = bias[(2 * NT + 1) * 4];
#pragma unroll
                for (int ks = 0; ks < KH; ++ks) {
                    const F8 A = W[(O4 + ks) * WAVE];
#pragma unroll
                    for (int n = 0; n < NTILE; ++n) acc[n][0] = mma<T>(A, hb[n][ks], ks == 0 ? bb : acc[n][0]);
                }
            }
            __builtin_amdgcn_s_setprio(0);
            // Outputs: the sigma and rgb rows are replicated in every lane
            // group, so lane group g finishes tile g (groups past NTILE idle).
            {
                static_assert(NTILE <= 4, "one output tile per lane group");
                float z = zs[0], q0 = acc[0][0][0], q1 = acc[0][0][1], q2 = acc[0][0][2];
                int og = orig[0];
#pragma unroll
                for (int n = 1; n < NTILE; ++n) {
                    if (g == n) {
                        z = zs[n]; q0 = acc[n][0][0]; q1 = acc[n][0][1]; q2 = acc[n][0][2]; og = orig[n];
                    }
                }
                if (g < NTILE && c + 16 * g + j < fend) {
                    const unsigned u = (unsigned)og;
                    st32(a.sigma, u, softplusf(z));
                    st32(a.rgb0, u, sigmoidf(q0));
                    st32(a.rgb1, u, sigmoidf(q1));
                    st32(a.rgb2, u, sigmoidf(q2));
                }
            }
            // the next chunk's position inputs
#pragma unroll
            for (int n = 0; n < NTILE; ++n) {
                orig[n] = orig_n[n];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    dv[n][k] = d_n[n][k];
                    xh[n][k] = (__builtin_fmaf(t_n[n], d_n[n][k], o_n[n][k]) - cc[k]) * inv_h;
                }
            }
        }
        pos = fend;
    }
}

template <typename K>
int resident_blocks(K kernel, size_t lds) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64 * FWD_WAVES, lds) != hipSuccess || per_cu < 1) per_cu = 1;
    hipDeviceProp_t prop;
    int cus = 256;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
    int nb = per_cu * cus;
    return (nb + 7) & ~7;
}

template <int H, typename T>
hipError_t fwd_launch(const FwdArgs& a, hipStream_t st) {
    using G = PackGeom<H>;
    const size_t lds = (size_t)G::FRAGS16 * WAVE * sizeof(typename FragT<T>::type) + G::BIAS_FLOATS * sizeof(float);
    static int nb = 0;
    if (!nb) nb = resident_blocks(k_fwd<H, T>, lds);
    hipLaunchKernelGGL((k_fwd<H, T>), dim3(nb), dim3(64 * FWD_WAVES), lds, st, a);
    return hipGetLastError();
}

template <int H>
hipError_t fwd_h(const r360_scene* s, const Workspace& w, int precision, hipStream_t st) {
    FwdArgs a;
    a.field_start = w.field_start;
    a.perm = w.perm;
    a.t_mid = w.t_mid;
    a.slots = w.slots;
    for (int k = 0; k < 3; ++k) { a.o[k] = w.ro + k * w.N; a.d[k] = w.rd + k * w.N; }
    a.N = w.N; a.cap = w.cap;
    a.F = s->mlp.n_fields;
    a.c0 = s->mlp.center[0]; a.c1 = s->mlp.center[1]; a.c2 = s->mlp.center[2];
    a.inv_h = 1.0f / s->mlp.half_extent;
    a.frames = s->use_frames ? s->frames : nullptr;
    a.bias = s->bias;
    a.sigma = w.sigma; a.rgb0 = w.rgb; a.rgb1 = w.rgb + w.cap; a.rgb2 = w.rgb + 2 * w.cap;
    if (precision == R360_BF16) { a.pack = s->pack16_bf; return fwd_launch<H, __bf16>(a, st); }
    if (precision == R360_FP16) { a.pack = s->pack16_h; return fwd_launch<H, _Float16>(a, st); }
    a.pack = s->pack16_f;
    return fwd_launch<H, float>(a, st);
}

template <int H>
hipError_t repack_h(r360_scene* s, const float* weights, hipStream_t st) {
    using G = PackGeom<H>;
    const int F = s->mlp.n_fields;
    const int64_t n = std::max<int64_t>((int64_t)F * G::FRAGS16 * WAVE * 8, (int64_t)F * G::BIAS_FLOATS);
    hipLaunchKernelGGL(k_repack<H>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, weights, F,
                       (__bf16*)s->pack16_bf, (_Float16*)s->pack16_h, s->pack16_f, s->bias);
    return hipGetLastError();
}

}  // namespace

size_t pack_bytes16(int H) { return H == 32 ? PackGeom<32>::BYTES16 : PackGeom<64>::BYTES16; }
size_t bias_floats(int H) { return H == 32 ? PackGeom<32>::BIAS_FLOATS : PackGeom<64>::BIAS_FLOATS; }

hipError_t launch_repack(r360_scene* s, const float* weights, hipStream_t st) {
    return s->mlp.hidden == 32 ? repack_h<32>(s, weights, st) : repack_h<64>(s, weights, st);
}

hipError_t launch_mlp_forward(const r360_scene* s, const Workspace& w, int precision, hipStream_t st) {
    return s->mlp.hidden == 32 ? fwd_h<32>(s, w, precision, st) : fwd_h<64>(s, w, precision, st);
}

}  // namespace r360
