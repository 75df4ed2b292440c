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
// Work split: samples arrive sorted by field (route.hip). 16-bit forms: each
// wave takes a contiguous slice of the sorted samples and keeps the current
// field's A fragments in registers, reloading them only when the slice
// crosses into the next field. FP32 form: a block takes a contiguous slice;
// its four waves share the field's FP32 fragments staged in LDS.
// Block indices are remapped so that the blocks resident on one XCD (blocks
// are dealt round-robin over the 8 XCDs) take neighbouring slices, which
// mostly share a field and so its weights in that XCD's L2.
#include "r360_internal.h"

namespace r360 {

namespace {

// FP32 forward: k-step ks is register ks%4 of tile ks/4.
__host__ __device__ constexpr int hidden_col32(int ks, int g) { return 16 * (ks >> 2) + 4 * g + (ks & 3); }

template <int H>
__device__ void step32(int st, int& ly, int& ot, int& ks) {
    using G = PackGeom<H>;
    int nks;
    if (st < G::S_L1) { ly = LY_L1; nks = 16; }
    else if ((st -= G::S_L1) < G::S_L2) { ly = LY_L2; nks = G::KH32; }
    else if ((st -= G::S_L2) < G::S_HD) { ly = LY_HD; nks = G::KH32; }
    else if ((st -= G::S_HD) < G::S_L3) { ly = LY_L3; nks = G::KH32 + 8; }
    else { st -= G::S_L3; ly = LY_L4; nks = G::KH32; }
    ot = st / nks;
    ks = st % nks;
}

template <int H>
__device__ float packed_source32(const float* w, int st, int lane) {
    int ly, ot, ks;
    step32<H>(st, ly, ot, ks);
    const int g = lane >> 4, row = 16 * ot + (lane & 15);
    if (ly == LY_L1) return canon_weight<H>(w, ly, row, true, pe_slot_feature(g, ks));
    if (ly == LY_L3 && ks >= PackGeom<H>::KH32) return canon_weight<H>(w, ly, row, true, dir_slot_feature(g, ks - PackGeom<H>::KH32));
    return canon_weight<H>(w, ly, row, false, hidden_col32(ks, g));
}

template <int H>
__global__ __launch_bounds__(256) void k_repack(const float* __restrict__ weights, int F, __bf16* __restrict__ pbf,
                                                _Float16* __restrict__ ph, float* __restrict__ p32,
                                                float* __restrict__ bias) {
    using G = PackGeom<H>;
    constexpr FieldLayout L{H};
    const int64_t n16 = (int64_t)F * G::FRAGS16 * WAVE * 8;
    const int64_t n32 = (int64_t)F * G::STEPS32 * WAVE;
    const int64_t nb = (int64_t)F * G::BIAS_FLOATS;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n16) {
        const int e = (int)(i & 7), lane = (int)((i >> 3) & 63);
        const int64_t fr_all = i >> 9;
        const int f = (int)(fr_all / G::FRAGS16), fr = (int)(fr_all % G::FRAGS16);
        const float v = packed_source16<H>(weights + (int64_t)f * L.P(), fr, lane, e);
        pbf[i] = (__bf16)v;
        ph[i] = (_Float16)v;
    }
    if (i < n32) {
        // stored as float4 groups of 4 consecutive k-steps: [F][STEPS32/4][64][4]
        const int e = (int)(i & 3), lane = (int)((i >> 2) & 63);
        const int64_t grp_all = i >> 8;
        const int f = (int)(grp_all / (G::STEPS32 / 4)), grp = (int)(grp_all % (G::STEPS32 / 4));
        p32[i] = packed_source32<H>(weights + (int64_t)f * L.P(), grp * 4 + e, lane);
    }
    if (i < nb) {
        const int f = (int)(i / G::BIAS_FLOATS), k = (int)(i % G::BIAS_FLOATS);
        const int tile = k >> 4, v = k & 15;
        const float* w = weights + (int64_t)f * L.P();
        float b;
        if (tile < G::NT) b = w[L.b2() + 16 * tile + v];
        else if (tile < 2 * G::NT + 1) {
            const int row = 16 * (tile - G::NT) + v;
            b = row < H ? w[L.bf() + row] : (row == H ? w[L.bs()] : 0.0f);
        } else b = v < 3 ? w[L.b4() + v] : 0.0f;
        bias[i] = b;
    }
}

// ---------------------------------------------------------------------------
// Forward
// ---------------------------------------------------------------------------
template <typename T> struct V8of;
template <> struct V8of<__bf16> { typedef bf16x8 type; };
template <> struct V8of<_Float16> { typedef f16x8 type; };

template <typename T>
__device__ __forceinline__ f32x4 mfma16(typename V8of<T>::type a, typename V8of<T>::type b, f32x4 c) {
    if constexpr (sizeof(T) == 2 && __is_same(T, __bf16)) return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    else return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

template <typename T>
__device__ __forceinline__ typename V8of<T>::type to8(const float* v) {
    typename V8of<T>::type r;
#pragma unroll
    for (int e = 0; e < 8; ++e) r[e] = (T)v[e];
    return r;
}

// ReLU (optional) of two accumulator tiles into one 16-bit B operand.
template <typename T, bool RELU>
__device__ __forceinline__ typename V8of<T>::type handoff(f32x4 a, f32x4 b) {
    float v[8] = {a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
    if (RELU) {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = v[e] > 0.0f ? v[e] : 0.0f;
    }
    return to8<T>(v);
}

__device__ __forceinline__ float softplusf(float z) { return fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z))); }
__device__ __forceinline__ float sigmoidf(float z) { return 1.0f / (1.0f + expf(-z)); }

struct FwdArgs {
    const int32_t* total;        // ray_off + N
    const int32_t* field_start;  // [F+1]
    const int32_t* perm;
    const float* t_mid;
    const int32_t* ray;
    const float* o;              // [3][N]
    const float* d;
    int64_t N, cap;
    int F;
    float c0, c1, c2, inv_h;
    const void* pack;            // 16-bit fragments or FP32 groups
    const float* bias;
    float* sigma;
    float* rgb;                  // [3][cap]
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

// Per-sample inputs, gathered in three dependent steps (sorted position ->
// sample index -> ray); the chunk loops issue the steps for the next chunk
// while the current one computes.
struct SampleIn {
    int orig;
    float t;
    int64_t ray;
    float o[3], d[3];
};

__device__ __forceinline__ void fetch_index(const FwdArgs& a, int pos, int fend, int j, SampleIn& s) {
    const int jp = pos + j;
    s.orig = a.perm[jp < fend ? jp : pos];
}
__device__ __forceinline__ void fetch_sample(const FwdArgs& a, SampleIn& s) {
    s.t = a.t_mid[s.orig];
    s.ray = a.ray[s.orig];
}
__device__ __forceinline__ void fetch_ray(const FwdArgs& a, SampleIn& s) {
    const int64_t r = s.ray;
    s.o[0] = a.o[r]; s.o[1] = a.o[a.N + r]; s.o[2] = a.o[2 * a.N + r];
    s.d[0] = a.d[r]; s.d[1] = a.d[a.N + r]; s.d[2] = a.d[2 * a.N + r];
}

// Encoding input xhat = (fma(t, d, o) - center) / half_extent (FP32 spec).
__device__ __forceinline__ void sample_xhat(const FwdArgs& a, const SampleIn& s, float xh[3]) {
    const float cc[3] = {a.c0, a.c1, a.c2};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float p = __builtin_fmaf(s.t, s.d[k], s.o[k]);
        xh[k] = (p - cc[k]) * a.inv_h;
    }
}

template <int H, typename T>
__global__ __launch_bounds__(256) void k_fwd16(FwdArgs a) {
    using G = PackGeom<H>;
    using V8 = typename V8of<T>::type;
    constexpr int NT = G::NT, KH = G::KH16;
    const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15;
    const int nw = gridDim.x * 4;
    const int w = xcd_block(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    const int S = *a.total;
    const int per = (((S + nw - 1) / nw) + 15) & ~15;
    const int beg = min(S, w * per), end = min(S, beg + per);

    V8 w1[NT][2], w2[NT][KH], wh[NT + 1][KH], w3[NT][KH + 1], w4[KH];
    const V8* pk = reinterpret_cast<const V8*>(a.pack);
    int cur = -1;
    for (int pos = beg; pos < end;) {
        const int f = find_field(a.field_start, a.F, pos);
        const int fend = min(end, a.field_start[f + 1]);
        if (f != cur) {
            cur = f;
            const V8* p = pk + (int64_t)f * G::FRAGS16 * WAVE + lane;
            int k = 0;
#pragma unroll
            for (int ot = 0; ot < NT; ++ot)
#pragma unroll
                for (int ks = 0; ks < 2; ++ks) w1[ot][ks] = p[(k++) * WAVE];
#pragma unroll
            for (int ot = 0; ot < NT; ++ot)
#pragma unroll
                for (int ks = 0; ks < KH; ++ks) w2[ot][ks] = p[(k++) * WAVE];
#pragma unroll
            for (int ot = 0; ot < NT + 1; ++ot)
#pragma unroll
                for (int ks = 0; ks < KH; ++ks) wh[ot][ks] = p[(k++) * WAVE];
#pragma unroll
            for (int ot = 0; ot < NT; ++ot)
#pragma unroll
                for (int ks = 0; ks < KH + 1; ++ks) w3[ot][ks] = p[(k++) * WAVE];
#pragma unroll
            for (int ks = 0; ks < KH; ++ks) w4[ks] = p[(k++) * WAVE];
        }
        const f32x4* bias = reinterpret_cast<const f32x4*>(a.bias + (int64_t)f * G::BIAS_FLOATS) + g;
        SampleIn nx;
        fetch_index(a, pos, fend, j, nx);
        fetch_sample(a, nx);
        fetch_ray(a, nx);
        for (; pos < fend; pos += 16) {
            const SampleIn cur = nx;
            const bool valid = pos + j < fend;
            const int orig = cur.orig;
            const bool more = pos + 16 < fend;
            if (more) fetch_index(a, pos + 16, fend, j, nx);
            float xh[3];
            sample_xhat(a, cur, xh);
            const float dv[3] = {cur.d[0], cur.d[1], cur.d[2]};
            float pe[16];
            pe_position(g, xh, pe);
            const V8 x0 = to8<T>(pe), x1 = to8<T>(pe + 8);
            // L1
            f32x4 acc[NT + 1];
#pragma unroll
            for (int ot = 0; ot < NT; ++ot) {
                acc[ot] = f32x4{0.f, 0.f, 0.f, 0.f};
                acc[ot] = mfma16<T>(w1[ot][0], x0, acc[ot]);
                acc[ot] = mfma16<T>(w1[ot][1], x1, acc[ot]);
            }
            V8 hb[KH];
#pragma unroll
            for (int ks = 0; ks < KH; ++ks) hb[ks] = handoff<T, true>(acc[2 * ks], acc[2 * ks + 1]);
            if (more) fetch_sample(a, nx);
            // L2
#pragma unroll
            for (int ot = 0; ot < NT; ++ot) {
                acc[ot] = bias[ot * 4];
#pragma unroll
                for (int ks = 0; ks < KH; ++ks) acc[ot] = mfma16<T>(w2[ot][ks], hb[ks], acc[ot]);
            }
#pragma unroll
            for (int ks = 0; ks < KH; ++ks) hb[ks] = handoff<T, true>(acc[2 * ks], acc[2 * ks + 1]);
            // HEAD: [f ; sigma]
#pragma unroll
            for (int ot = 0; ot < NT + 1; ++ot) {
                acc[ot] = bias[(NT + ot) * 4];
#pragma unroll
                for (int ks = 0; ks < KH; ++ks) acc[ot] = mfma16<T>(wh[ot][ks], hb[ks], acc[ot]);
            }
            const float zs = acc[NT][0];
#pragma unroll
            for (int ks = 0; ks < KH; ++ks) hb[ks] = handoff<T, false>(acc[2 * ks], acc[2 * ks + 1]);
            if (more) fetch_ray(a, nx);
            float dpe[8];
            pe_direction(g, dv, dpe);
            const V8 xd = to8<T>(dpe);
            // L3 on [f ; g(d)]
#pragma unroll
            for (int ot = 0; ot < NT; ++ot) {
                acc[ot] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < KH; ++ks) acc[ot] = mfma16<T>(w3[ot][ks], hb[ks], acc[ot]);
                acc[ot] = mfma16<T>(w3[ot][KH], xd, acc[ot]);
            }
#pragma unroll
            for (int ks = 0; ks < KH; ++ks) hb[ks] = handoff<T, true>(acc[2 * ks], acc[2 * ks + 1]);
            // L4
            f32x4 o4 = bias[(2 * NT + 1) * 4];
#pragma unroll
            for (int ks = 0; ks < KH; ++ks) o4 = mfma16<T>(w4[ks], hb[ks], o4);
            if (g == 0 && valid) {
                a.sigma[orig] = softplusf(zs);
                a.rgb[orig] = sigmoidf(o4[0]);
                a.rgb[a.cap + orig] = sigmoidf(o4[1]);
                a.rgb[2 * a.cap + orig] = sigmoidf(o4[2]);
            }
        }
    }
}

// FP32 form: block-wide slices; the field's fragments are staged in LDS.
template <int H>
__global__ __launch_bounds__(256) void k_fwd32(FwdArgs a) {
    using G = PackGeom<H>;
    constexpr int NT = G::NT, KH = G::KH32;
    extern __shared__ float4 lw[];                         // [STEPS32/4][64] float4, then bias
    float* lbias = reinterpret_cast<float*>(lw + (G::STEPS32 / 4) * WAVE);
    const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15, wv = threadIdx.x >> 6;
    const int nb = gridDim.x;
    const int b = xcd_block(blockIdx.x, nb);
    const int S = *a.total;
    const int per = (((S + nb - 1) / nb) + 63) & ~63;
    const int beg = min(S, b * per), end = min(S, beg + per);
    const float4* pk = reinterpret_cast<const float4*>(a.pack);
    for (int pos = beg; pos < end;) {
        const int f = find_field(a.field_start, a.F, pos);
        const int fend = min(end, a.field_start[f + 1]);
        __syncthreads();
        const float4* src = pk + (int64_t)f * (G::STEPS32 / 4) * WAVE;
        for (int i = threadIdx.x; i < (G::STEPS32 / 4) * WAVE; i += 256) lw[i] = src[i];
        for (int i = threadIdx.x; i < G::BIAS_FLOATS; i += 256) lbias[i] = a.bias[(int64_t)f * G::BIAS_FLOATS + i];
        __syncthreads();
        SampleIn nx;
        if (pos + 16 * wv < fend) {
            fetch_index(a, pos + 16 * wv, fend, j, nx);
            fetch_sample(a, nx);
            fetch_ray(a, nx);
        }
        for (int c = pos + 16 * wv; c < fend; c += 64) {
            const SampleIn cur = nx;
            const bool valid = c + j < fend;
            const int orig = cur.orig;
            const bool more = c + 64 < fend;
            if (more) {
                fetch_index(a, c + 64, fend, j, nx);
                fetch_sample(a, nx);
                fetch_ray(a, nx);
            }
            float xh[3];
            sample_xhat(a, cur, xh);
            const float dv[3] = {cur.d[0], cur.d[1], cur.d[2]};
            float pe[16];
            pe_position(g, xh, pe);
            const float4* p = lw + lane;
            f32x4 acc[NT + 1];
            // L1: 16 k-steps
#pragma unroll
            for (int ot = 0; ot < NT; ++ot) {
                acc[ot] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kg = 0; kg < 4; ++kg) {
                    const float4 w4v = p[(ot * 4 + kg) * WAVE];
                    acc[ot] = __builtin_amdgcn_mfma_f32_16x16x4f32(w4v.x, pe[4 * kg + 0], acc[ot], 0, 0, 0);
                    acc[ot] = __builtin_amdgcn_mfma_f32_16x16x4f32(w4v.y, pe[4 * kg + 1], acc[ot], 0, 0, 0);
                    acc[ot] = __builtin_amdgcn_mfma_f32_16x16x4f32(w4v.z, pe[4 * kg + 2], acc[ot], 0, 0, 0);
                    acc[ot] = __builtin_amdgcn_mfma_f32_16x16x4f32(w4v.w, pe[4 * kg + 3], acc[ot], 0, 0, 0);
                }
            }
            p += G::S_L1 / 4 * WAVE;
            f32x4 h[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) h[t][r] = acc[t][r] > 0.0f ? acc[t][r] : 0.0f;
            const float4* lb = reinterpret_cast<const float4*>(lbias) + g;
            // L2
#pragma unroll
            for (int ot = 0; ot < NT; ++ot) {
                const float4 bb = lb[ot * 4];
                acc[ot] = f32x4{bb.x, bb.y, bb.z, bb.w};
#pragma unroll
                for (int kg = 0; kg < KH / 4; ++kg) {
                    const float4 w4v = p[(ot * (KH / 4) + kg) * WAVE];
                    acc[ot] = __builtin_amdgcn_mfma_f32_16x16x4f32(w4v.x, h[kg][0], acc[ot], 0, 0, 0);
                    acc[ot] = __builtin_amdgcn_mfma_f32_16x16x4f32(w4v.y, h[kg][1], acc[ot], 0, 0, 0);
                    acc[ot] = __builtin_amdgcn_mfma_f32_16x16x4f32(w4v.z, h[kg][2], acc[ot], 0, 0, 0);
                    acc[ot] = __builtin_amdgcn_mfma_f32_16x16x4f32(w4v.w, h[kg][3], acc[ot], 0, 0, 0);
                }
            }
            p += G::S_L2 / 4 * WAVE;
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) h[t][r] = acc[t][r] > 0.0f ? acc[t][r] : 0.0f;
            // HEAD
#pragma unroll
            for (int ot = 0; ot < NT + 1; ++ot) {
                const float4 bb = lb[(NT + ot) * 4];
                acc[ot] = f32x4{bb.x, bb.y, bb.z, bb.w};
#pragma unroll
                for (int kg = 0; kg < KH / 4; ++kg) {
                    const float4 w4v = p[(ot * (KH / 4) + kg) * WAVE];
                    acc[ot] = __builtin_amdgcn_mfma_f32_16x16x4f32(w4v.x, h[kg][0], acc[ot], 0, 0, 0);
                    acc[ot] = __builtin_amdgcn_mfma_f32_16x16x4f32(w4v.y, h[kg][1], acc[ot], 0, 0, 0);
                    acc[ot] = __builtin_amdgcn_mfma_f32_16x16x4f32(w4v.z, h[kg][2], acc[ot], 0, 0, 0);
                    acc[ot] = __builtin_amdgcn_mfma_f32_16x16x4f32(w4v.w, h[kg][3], acc[ot], 0, 0, 0);
                }
            }
            p += G::S_HD / 4 * WAVE;
            const float zs = acc[NT][0];
#pragma unroll
            for (int t = 0; t < NT; ++t) h[t] = acc[t];
            float dpe[8];
            pe_direction(g, dv, dpe);
            // L3 on [f ; g(d)]
#pragma unroll
            for (int ot = 0; ot < NT; ++ot) {
                acc[ot] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kg = 0; kg < KH / 4 + 2; ++kg) {
                    const float4 w4v = p[(ot * (KH / 4 + 2) + kg) * WAVE];
                    const float b0 = kg < KH / 4 ? h[kg < KH / 4 ? kg : 0][0] : dpe[4 * (kg - KH / 4) + 0];
                    const float b1 = kg < KH / 4 ? h[kg < KH / 4 ? kg : 0][1] : dpe[4 * (kg - KH / 4) + 1];
                    const float b2 = kg < KH / 4 ? h[kg < KH / 4 ? kg : 0][2] : dpe[4 * (kg - KH / 4) + 2];
                    const float b3 = kg < KH / 4 ? h[kg < KH / 4 ? kg : 0][3] : dpe[4 * (kg - KH / 4) + 3];
                    acc[ot] = __builtin_amdgcn_mfma_f32_16x16x4f32(w4v.x, b0, acc[ot], 0, 0, 0);
                    acc[ot] = __builtin_amdgcn_mfma_f32_16x16x4f32(w4v.y, b1, acc[ot], 0, 0, 0);
                    acc[ot] = __builtin_amdgcn_mfma_f32_16x16x4f32(w4v.z, b2, acc[ot], 0, 0, 0);
                    acc[ot] = __builtin_amdgcn_mfma_f32_16x16x4f32(w4v.w, b3, acc[ot], 0, 0, 0);
                }
            }
            p += G::S_L3 / 4 * WAVE;
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) h[t][r] = acc[t][r] > 0.0f ? acc[t][r] : 0.0f;
            // L4
            const float4 bb = lb[(2 * NT + 1) * 4];
            f32x4 o4 = f32x4{bb.x, bb.y, bb.z, bb.w};
#pragma unroll
            for (int kg = 0; kg < KH / 4; ++kg) {
                const float4 w4v = p[kg * WAVE];
                o4 = __builtin_amdgcn_mfma_f32_16x16x4f32(w4v.x, h[kg][0], o4, 0, 0, 0);
                o4 = __builtin_amdgcn_mfma_f32_16x16x4f32(w4v.y, h[kg][1], o4, 0, 0, 0);
                o4 = __builtin_amdgcn_mfma_f32_16x16x4f32(w4v.z, h[kg][2], o4, 0, 0, 0);
                o4 = __builtin_amdgcn_mfma_f32_16x16x4f32(w4v.w, h[kg][3], o4, 0, 0, 0);
            }
            if (g == 0 && valid) {
                a.sigma[orig] = softplusf(zs);
                a.rgb[orig] = sigmoidf(o4[0]);
                a.rgb[a.cap + orig] = sigmoidf(o4[1]);
                a.rgb[2 * a.cap + orig] = sigmoidf(o4[2]);
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
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, lds) != hipSuccess || per_cu < 1) per_cu = 1;
    hipDeviceProp_t prop;
    int cus = 256;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
    int nb = per_cu * cus;
    return (nb + 7) & ~7;
}

template <int H>
hipError_t fwd_h(const r360_scene* s, const Workspace& w, int precision, hipStream_t st) {
    FwdArgs a;
    a.total = w.ray_off + w.N;
    a.field_start = w.field_start;
    a.perm = w.perm;
    a.t_mid = w.t_mid;
    a.ray = w.ray;
    a.o = w.ro; a.d = w.rd;
    a.N = w.N; a.cap = w.cap;
    a.F = s->mlp.n_fields;
    a.c0 = s->mlp.center[0]; a.c1 = s->mlp.center[1]; a.c2 = s->mlp.center[2];
    a.inv_h = 1.0f / s->mlp.half_extent;
    a.bias = s->bias;
    a.sigma = w.sigma; a.rgb = w.rgb;
    if (precision == R360_FP32) {
        a.pack = s->pack32;
        const size_t lds = (size_t)PackGeom<H>::BYTES32 + PackGeom<H>::BIAS_FLOATS * 4;
        static int nb = 0;
        if (!nb) nb = resident_blocks(k_fwd32<H>, lds);
        hipLaunchKernelGGL(k_fwd32<H>, dim3(nb), dim3(256), lds, st, a);
    } else if (precision == R360_BF16) {
        a.pack = s->pack16_bf;
        static int nb = 0;
        if (!nb) nb = resident_blocks(k_fwd16<H, __bf16>, 0);
        hipLaunchKernelGGL((k_fwd16<H, __bf16>), dim3(nb), dim3(256), 0, st, a);
    } else {
        a.pack = s->pack16_h;
        static int nb = 0;
        if (!nb) nb = resident_blocks(k_fwd16<H, _Float16>, 0);
        hipLaunchKernelGGL((k_fwd16<H, _Float16>), dim3(nb), dim3(256), 0, st, a);
    }
    return hipGetLastError();
}

template <int H>
hipError_t repack_h(r360_scene* s, const float* weights, hipStream_t st) {
    using G = PackGeom<H>;
    const int F = s->mlp.n_fields;
    const int64_t n = std::max<int64_t>((int64_t)F * G::FRAGS16 * WAVE * 8,
                                        std::max<int64_t>((int64_t)F * G::STEPS32 * WAVE, (int64_t)F * G::BIAS_FLOATS));
    hipLaunchKernelGGL(k_repack<H>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, weights, F,
                       (__bf16*)s->pack16_bf, (_Float16*)s->pack16_h, s->pack32, s->bias);
    return hipGetLastError();
}

}  // namespace

size_t pack_bytes16(int H) { return H == 32 ? PackGeom<32>::BYTES16 : PackGeom<64>::BYTES16; }
size_t pack_bytes32(int H) { return H == 32 ? PackGeom<32>::BYTES32 : PackGeom<64>::BYTES32; }
size_t bias_floats(int H) { return H == 32 ? PackGeom<32>::BIAS_FLOATS : PackGeom<64>::BIAS_FLOATS; }

hipError_t launch_repack(r360_scene* s, const float* weights, hipStream_t st) {
    return s->mlp.hidden == 32 ? repack_h<32>(s, weights, st) : repack_h<64>(s, weights, st);
}

hipError_t launch_mlp_forward(const r360_scene* s, const Workspace& w, int precision, hipStream_t st) {
    return s->mlp.hidden == 32 ? fwd_h<32>(s, w, precision, st) : fwd_h<64>(s, w, precision, st);
}

}  // namespace r360
