// Global omnidirectional field stage (360NeRF, Sec. 3.2 and the 360NeRF
// architecture table of App. C): rays sampled uniformly in inverse depth,
// positional encoding, an 8 x 256 MLP with the encoding concatenated again
// at the fifth layer input, a density head and a feature layer, the colour
// branch on [feature ; encoded direction], compositing (Eq.4/Eq.5), L2 loss
// and the full backward pass; the per-sample densities are max-reduced into
// an occupancy grid (the density source of Sec. 4.1's occupancy estimation).
//
// Every layer is one BF16 MFMA GEMM over all M = rays x samples rows with
// FP32 accumulation, activations kept in HBM as BF16 for the backward pass
// (≈2.7 GB at 4,096 rays x 128 samples). The GEMM stages 128 x 128 x 32
// tiles of both operands through LDS; an operand whose contraction index is
// not contiguous in memory (the weight gradients, which contract over the
// samples) is transposed while it is staged. Epilogues apply bias and
// activation, write straight into the next layer's (concatenated) input,
// mask the input gradients with the ReLU pattern of the forward activations,
// or emit per-slice FP32 weight-gradient partials (and the bias gradients as
// column sums of the staged output-gradient tile). The partials are reduced
// in slice order, so the gradient is deterministic.
#include <algorithm>
#include <utility>

#include "r360_internal.h"

namespace r360 {

namespace {

typedef __bf16 bf16;
typedef unsigned u32;

// ---------------------------------------------------------------------------
// Layer matrices. All layers are stored as BF16 [N][K] (row = output, K
// contiguous) and as their transposes [K][NC] (NC = N padded to a multiple
// of 32), with biases either folded into a constant-1 input column (L1, L5,
// L10) or kept as FP32 vectors added in the epilogue.
// ---------------------------------------------------------------------------
enum GLayer { G1 = 0, G2, G3, G4, G5, G6, G7, G8, GH, G10, G11, NGL };

struct GLayerGeom {
    int N, K, NC;         // rows, padded contraction width, padded rows for the transpose
    int bias_col;         // input column holding the constant 1 (folded bias), or -1
    int64_t w_off, t_off; // offsets (elements) of W and W^T in the bf16 arena
    int64_t b_off;        // offset (floats) of the epilogue bias, or -1
    int64_t g_off;        // offset (floats) of this layer's gradient partial [N][K]
    int64_t gb_off;       // offset (floats) of its bias-gradient partial [N], or -1
};

struct GNet {
    int w, c;             // width 256, colour width 128
    GLayerGeom L[NGL];
    int64_t w_elems, b_elems, g_elems;   // arena sizes
    int64_t P;            // canonical parameter count
};

constexpr int GDX = DXYZ;   // 63
constexpr int GDD = DDIR;   // 27

inline int up32(int x) { return (x + 31) & ~31; }

GNet make_net(int w, int c) {
    GNet n{};
    n.w = w; n.c = c;
    auto set = [&](int i, int N, int K, int bias_col, bool epi_bias) {
        GLayerGeom& g = n.L[i];
        g.N = N; g.K = K; g.NC = up32(N); g.bias_col = bias_col;
        g.w_off = n.w_elems; n.w_elems += (int64_t)N * K;
        g.t_off = n.w_elems; n.w_elems += (int64_t)K * g.NC;
        g.b_off = epi_bias ? n.b_elems : -1; if (epi_bias) n.b_elems += N;
        g.g_off = n.g_elems; n.g_elems += (int64_t)N * K;
        g.gb_off = epi_bias ? n.g_elems : -1; if (epi_bias) n.g_elems += N;
    };
    set(G1, w, 64, GDX, false);                        // [gx (63) | 1]
    set(G2, w, w, -1, true); set(G3, w, w, -1, true); set(G4, w, w, -1, true);
    set(G5, w, w + 64, w + GDX, false);                // [h4 | gx | 1]
    set(G6, w, w, -1, true); set(G7, w, w, -1, true); set(G8, w, w, -1, true);
    set(GH, w + 1, w, -1, true);                       // rows [f (w) ; sigma]
    set(G10, c, up32(w + GDD + 1), w + GDD, false);    // [f | gd (27) | 1 | 0..]
    set(G11, 3, c, -1, true);
    n.P = (int64_t)w * GDX + w + 3 * ((int64_t)w * w + w) + (int64_t)w * (w + GDX) + w + 3 * ((int64_t)w * w + w)
          + w + 1 + (int64_t)w * w + w + (int64_t)c * (w + GDD) + c + 3 * (int64_t)c + 3;
    return n;
}

// Canonical parameter p -> (layer, row, column or -1 for an epilogue bias).
// Canonical order: W1 b1 W2 b2 ... W8 b8 ws bs Wf bf W10 b10 W11 b11.
__host__ __device__ inline void canon_to_layer(int w, int c, int64_t p, int& ly, int& row, int& col) {
    const int64_t in0 = GDX, in4 = w + GDX;
    for (int k = 0; k < 8; ++k) {
        const int64_t in = (k == 0) ? in0 : (k == 4 ? in4 : w);
        if (p < (int64_t)w * in) {
            ly = k; row = (int)(p / in); col = (int)(p % in);
            return;
        }
        p -= (int64_t)w * in;
        if (p < w) {                          // bias
            ly = k; row = (int)p;
            col = (k == 0) ? GDX : (k == 4 ? w + GDX : -1);
            return;
        }
        p -= w;
    }
    if (p < w) { ly = GH; row = w; col = (int)p; return; }          // ws
    p -= w;
    if (p < 1) { ly = GH; row = w; col = -1; return; }              // bs
    p -= 1;
    if (p < (int64_t)w * w) { ly = GH; row = (int)(p / w); col = (int)(p % w); return; }   // Wf
    p -= (int64_t)w * w;
    if (p < w) { ly = GH; row = (int)p; col = -1; return; }         // bf
    p -= w;
    if (p < (int64_t)c * (w + GDD)) { ly = G10; row = (int)(p / (w + GDD)); col = (int)(p % (w + GDD)); return; }
    p -= (int64_t)c * (w + GDD);
    if (p < c) { ly = G10; row = (int)p; col = w + GDD; return; }   // b10 (folded)
    p -= c;
    if (p < 3 * (int64_t)c) { ly = G11; row = (int)(p / c); col = (int)(p % c); return; }
    p -= 3 * (int64_t)c;
    ly = G11; row = (int)p; col = -1;                                 // b11
}

struct GNetDev {
    int w, c;
    int64_t P;
    GLayerGeom L[NGL];
};

// Zero fill of the BF16 arena: the padding of every layer matrix (columns
// past K's real inputs, rows past N in the transposes) must hold 0, since
// the GEMMs contract over it against zero activations and 0 * NaN is NaN.
__global__ void k_gzero(u32* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0u;
}

// FP32 canonical weights -> BF16 layer matrices, their transposes and the
// FP32 epilogue biases (one thread per canonical parameter).
__global__ void k_gnet_pack(GNetDev n, const float* __restrict__ wc, bf16* __restrict__ arena, float* __restrict__ bias) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n.P) return;
    int ly, row, col;
    canon_to_layer(n.w, n.c, p, ly, row, col);
    const GLayerGeom& g = n.L[ly];
    const float v = wc[p];
    if (col < 0) {
        bias[g.b_off + row] = v;
    } else {
        arena[g.w_off + (int64_t)row * g.K + col] = (bf16)v;
        arena[g.t_off + (int64_t)col * g.NC + row] = (bf16)v;
    }
}

// Weight gradient: canonical parameter <- sum over slices of its partial.
// A block of four waves takes 64 consecutive parameters, one per lane; wave
// j adds the slices k = j mod 4 in order, so each load of a wave reads 64
// consecutive partials of one slice (whole cache lines), and the four sums
// are then added as (s0 + s1) + (s2 + s3) (a fixed order).
__global__ __launch_bounds__(256) void k_gnet_grad(GNetDev n, const float* __restrict__ part, int64_t part_stride,
                                                   int slices, float* __restrict__ grad) {
    __shared__ float red[4][64];
    const int lane = threadIdx.x & 63, j = threadIdx.x >> 6;
    const int64_t p = (int64_t)blockIdx.x * 64 + lane;
    float s = 0.0f;
    if (p < n.P) {
        int ly, row, col;
        canon_to_layer(n.w, n.c, p, ly, row, col);
        const GLayerGeom& g = n.L[ly];
        const int64_t off = col < 0 ? g.gb_off + row : g.g_off + (int64_t)row * g.K + col;
        const float* src = part + off;
        int k = j;
        for (; k + 28 < slices; k += 32) {            // eight loads in flight
            float v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = src[(int64_t)(k + 4 * q) * part_stride];
#pragma unroll
            for (int q = 0; q < 8; ++q) s += v[q];
        }
        for (; k < slices; k += 4) s += src[(int64_t)k * part_stride];
    }
    red[j][lane] = s;
    __syncthreads();
    if (j == 0 && p < n.P) grad[p] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

// ---------------------------------------------------------------------------
// Samples and encodings: sample k of ray r is row m = 128 r + k (ray-major).
// t_k = 1 / fma(s_k, 1/far, (1 - s_k) / near) with s_k = k / (S - 1) (uniform
// in inverse depth, exact at both ends), delta_k = t_{k+1} - t_k, delta_last
// = 0; p = fma(t, d, o); xhat = (p - center) / half_extent.
// ---------------------------------------------------------------------------
struct GSampleArgs {
    const float* o; const float* d;
    int64_t N; int S;
    float a_near, b_far;       // 1/near, 1/far
    float c0, c1, c2, inv_h;
    float lo0, lo1, lo2, inv_vox;
    int g0, g1, g2;            // occupancy grid size
    bf16* x5;                  // [M][w + 64]: cols w.. = gx | 1
    bf16* x10;                 // [M][K10]:   cols w.. = gd | 1 | 0
    int w, k10;
    float* t; float* delta;    // [M]
    int32_t* voxel;            // [M] linear cell or -1
    int32_t* ray;              // [M] ray of each sample
    int32_t* ray_off;          // [N+1]
    int points;                // one sample per ray at t = 0 (the origin itself)
};

__device__ inline float inv_depth_t(const GSampleArgs& a, int k) {
    const float s = (float)k / (float)(a.S - 1);
    return 1.0f / __builtin_fmaf(s, a.b_far, (1.0f - s) * a.a_near);
}

__global__ __launch_bounds__(256) void k_gsamples(GSampleArgs a) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t M = a.N * a.S;
    if (m <= a.N) a.ray_off[m] = (int32_t)(m * a.S);
    if (m >= M) return;
    const int64_t r = m / a.S;
    const int k = (int)(m % a.S);
    const float t = a.points ? 0.0f : inv_depth_t(a, k);
    a.t[m] = t;
    a.ray[m] = (int32_t)r;
    a.delta[m] = (!a.points && k + 1 < a.S) ? inv_depth_t(a, k + 1) - t : 0.0f;
    const float o[3] = {a.o[r], a.o[a.N + r], a.o[2 * a.N + r]};
    const float d[3] = {a.d[r], a.d[a.N + r], a.d[2 * a.N + r]};
    const float cc[3] = {a.c0, a.c1, a.c2};
    const float lo[3] = {a.lo0, a.lo1, a.lo2};
    const int gn[3] = {a.g0, a.g1, a.g2};
    float xh[3];
    int cell[3];
    bool inside = true;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const float p = __builtin_fmaf(t, d[q], o[q]);
        xh[q] = (p - cc[q]) * a.inv_h;
        const float u = (p - lo[q]) * a.inv_vox;
        inside = inside && (u >= 0.0f) && (u < (float)gn[q]);
        cell[q] = inside ? (int)__builtin_floorf(u) : 0;
    }
    a.voxel[m] = inside ? cell[0] + gn[0] * (cell[1] + gn[1] * cell[2]) : -1;
    // the encodings are assembled in registers and stored 16 bytes at a time
    // (row strides and the first encoding column are multiples of 32 elements)
    static_assert(GDX + 1 == 64 && GDD + 1 <= 32, "encoding widths");
    bf16x8 xv[8];
#pragma unroll
    for (int q = 0; q < 3; ++q) xv[0][q] = (bf16)xh[q];
#pragma unroll
    for (int l = 0; l < LXYZ; ++l) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            float s, cth;
            sincospi(__builtin_ldexpf(xh[q], l), s, cth);
            const int is = 3 + 6 * l + q, ic = 6 + 6 * l + q;
            xv[is >> 3][is & 7] = (bf16)s;
            xv[ic >> 3][ic & 7] = (bf16)cth;
        }
    }
    xv[GDX >> 3][GDX & 7] = (bf16)1.0f;
    bf16x8* x = reinterpret_cast<bf16x8*>(a.x5 + m * (a.w + 64) + a.w);
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = xv[j];
    bf16x8 yv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int e = 0; e < 8; ++e) yv[j][e] = (bf16)0.0f;
#pragma unroll
    for (int q = 0; q < 3; ++q) yv[0][q] = (bf16)d[q];
#pragma unroll
    for (int l = 0; l < LDIR; ++l) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            float s, cth;
            sincospi(__builtin_ldexpf(d[q], l), s, cth);
            const int is = 3 + 6 * l + q, ic = 6 + 6 * l + q;
            yv[is >> 3][is & 7] = (bf16)s;
            yv[ic >> 3][ic & 7] = (bf16)cth;
        }
    }
    yv[GDD >> 3][GDD & 7] = (bf16)1.0f;
    bf16x8* y = reinterpret_cast<bf16x8*>(a.x10 + m * a.k10 + a.w);    // k10 - w = 32 columns
#pragma unroll
    for (int j = 0; j < 4; ++j) y[j] = yv[j];
}

// ---------------------------------------------------------------------------
// GEMMs. Row GEMM (forward layers and input gradients):
//   out[r][c] = epi(sum_k A[r][k] B[c][k]), r < R, c < C, k < Kc (multiple of 32),
// both operands K-contiguous (element (row, k) at p[row * sr + k]).
// Weight-gradient GEMM: part[slice][n][k'] = sum_m A[m][n] B[m][k'] over the
// slice's samples m, both operands sample-major (element (m, col) at
// p[m * sr + col]).
// ---------------------------------------------------------------------------
enum Epi { EPI_FWD = 0, EPI_RGB, EPI_DX, EPI_DW };

struct GemmArgs {
    const bf16* A; int64_t a_sr;
    const bf16* B; int64_t b_sr;
    int R, C, Kc;              // rows, columns, contraction length (per slice for EPI_DW)
    // EPI_FWD: out[r * ldo + c] = act(acc + bias[c]) for c < n_out; column c == sig_col
    // goes to sig[r] (ReLU) instead
    const float* bias;
    bool relu;
    bf16* out; int64_t ldo;
    int n_out;
    int sig_col; float* sig;
    // EPI_RGB: rgb[c * R + r] = sigmoid(acc + bias[c]) for c < 3
    float* rgb;
    // EPI_DX: out[r * ldo + c] = acc * [mask[r * ldm + c] > 0] (mask may be null)
    const bf16* mask; int64_t ldm;
    // The ReLU pattern as sign bits, bit c % 8 of byte mbits[r * ldb + c / 8]
    // set where the stored output is > 0: written by EPI_FWD when mbits is set
    // (weight-resident kernel only), read by EPI_DX from mbits_in in place of
    // mask (a sixteenth of the bytes).
    uint8_t* mbits; const uint8_t* mbits_in; int64_t ldb;
    // EPI_DW: total samples M; readable columns of A and B (multiples of 8);
    // part[slice * pstride + r * ldp + c] = acc; row sums at part[slice * pstride + boff + r]
    int64_t Mtot; int a_lim, b_lim;
    float* part; int64_t pstride, ldp, boff;   // boff < 0: no bias gradient
};

constexpr int GT = 128;         // tile rows
constexpr int GK = 32;          // contraction step of the row GEMM
constexpr int GPAD = 40;        // LDS row stride (elements) of 32-wide k slabs: 80 bytes

typedef __attribute__((ext_vector_type(4))) unsigned u4;

// Row GEMM, tile GT x BN, four waves of 64 x BN/2. Operand slabs are double
// buffered in LDS: the global loads of step k+1 are issued before the MFMAs
// of step k and stored to the other buffer after them, one barrier per step.
template <int EPI, int BN>
__global__ __launch_bounds__(256, 2) void k_gemm(GemmArgs g) {
    constexpr int WN = BN / 2, TJ = WN / 16, BQ = BN / 64;
    constexpr int SP = 64 + 8;                                   // epilogue staging row stride (elements)
    constexpr int OPER = 2 * GT * GPAD + 2 * BN * GPAD, STAGE = 4 * 64 * SP;
    // one LDS buffer: double-buffered operand slabs during the K loop, then
    // the epilogue's staging area
    __shared__ __attribute__((aligned(16))) bf16 smem[OPER > STAGE ? OPER : STAGE];
    bf16 (*la)[GT * GPAD] = reinterpret_cast<bf16 (*)[GT * GPAD]>(smem);
    bf16 (*lb)[BN * GPAD] = reinterpret_cast<bf16 (*)[BN * GPAD]>(smem + 2 * GT * GPAD);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wm = wv >> 1, wn = wv & 1;
    const int r0 = blockIdx.x * GT, c0 = blockIdx.y * BN;
    f32x4 acc[4][TJ];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    u4 va[2], vb[BQ];
    // piece p of a slab: row p / 4, k offset 8 (p % 4)
#define R360_GLOAD(k0)                                                                                   \
    {                                                                                                    \
        _Pragma("unroll") for (int q = 0; q < 2; ++q) {                                                  \
            const int p = tid + 256 * q, row = r0 + (p >> 2);                                            \
            va[q] = row < g.R ? *reinterpret_cast<const u4*>(g.A + row * g.a_sr + (k0) + 8 * (p & 3))    \
                              : u4{0u, 0u, 0u, 0u};                                                      \
        }                                                                                                \
        _Pragma("unroll") for (int q = 0; q < BQ; ++q) {                                                 \
            const int p = tid + 256 * q, row = c0 + (p >> 2);                                            \
            vb[q] = row < g.C ? *reinterpret_cast<const u4*>(g.B + row * g.b_sr + (k0) + 8 * (p & 3))    \
                              : u4{0u, 0u, 0u, 0u};                                                      \
        }                                                                                                \
    }
#define R360_LSTORE(buf)                                                                                 \
    {                                                                                                    \
        _Pragma("unroll") for (int q = 0; q < 2; ++q) {                                                  \
            const int p = tid + 256 * q;                                                                 \
            *reinterpret_cast<u4*>(&la[buf][(p >> 2) * GPAD + 8 * (p & 3)]) = va[q];                     \
        }                                                                                                \
        _Pragma("unroll") for (int q = 0; q < BQ; ++q) {                                                 \
            const int p = tid + 256 * q;                                                                 \
            *reinterpret_cast<u4*>(&lb[buf][(p >> 2) * GPAD + 8 * (p & 3)]) = vb[q];                     \
        }                                                                                                \
    }
    R360_GLOAD(0)
    R360_LSTORE(0)
    __syncthreads();
    const int nk = g.Kc / GK;
    for (int it = 0; it < nk; ++it) {
        const int cur = it & 1;
        const bool more = it + 1 < nk;
        if (more) R360_GLOAD((it + 1) * GK)
        bf16x8 fa[4], fb[TJ];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            fa[i] = *reinterpret_cast<const bf16x8*>(&la[cur][(64 * wm + 16 * i + (lane & 15)) * GPAD + 8 * (lane >> 4)]);
#pragma unroll
        for (int j = 0; j < TJ; ++j)
            fb[j] = *reinterpret_cast<const bf16x8*>(&lb[cur][(WN * wn + 16 * j + (lane & 15)) * GPAD + 8 * (lane >> 4)]);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < TJ; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
        if (more) R360_LSTORE(cur ^ 1)
        __syncthreads();
    }
#undef R360_GLOAD
#undef R360_LSTORE
    // Epilogue. Lane holds rows 16 i + 4 (lane / 16) + q, column 16 j + lane % 16
    // of its wave's 64 x WN part. BF16 outputs go through LDS (the operand
    // buffers are free now), 64 columns at a time per wave, and leave as
    // 16-byte row pieces; the input-gradient mask is read the same way.
    const int g4 = lane >> 4, l16 = lane & 15;
    if constexpr (EPI == EPI_RGB) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = r0 + 64 * wm + 16 * i + 4 * g4 + q;
                const int c = c0 + WN * wn + l16;
                if (r < g.R && c < 3) g.rgb[(int64_t)c * g.R + r] = 1.0f / (1.0f + expf(-(acc[i][0][q] + g.bias[c])));
            }
        return;
    } else {
        bf16* stg = smem + wv * 64 * SP;
        const int rw = r0 + 64 * wm;                                 // first row of this wave
#pragma unroll
        for (int h = 0; h < WN / 64; ++h) {
            const int cw = c0 + WN * wn + 64 * h;                    // first column of this half
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int j = 4 * h + jj;
                    const int c = cw + 16 * jj + l16;
                    float bsum = 0.0f;
                    if constexpr (EPI == EPI_FWD) bsum = (g.bias && c < g.C) ? g.bias[c] : 0.0f;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        float v = acc[i][j][q] + bsum;
                        if constexpr (EPI == EPI_FWD) {
                            if (g.relu) v = v > 0.0f ? v : 0.0f;
                            const int r = rw + 16 * i + 4 * g4 + q;
                            if (c == g.sig_col && r < g.R) g.sig[r] = v;
                        }
                        stg[(16 * i + 4 * g4 + q) * SP + 16 * jj + l16] = (bf16)v;
                    }
                }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int ncols = EPI == EPI_FWD ? min(g.C, g.n_out) : g.C;   // columns that go to `out`
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int ch = lane + 64 * t;                        // 512 pieces of 8 columns
                const int rr = ch >> 3, cc = 8 * (ch & 7);
                const int r = rw + rr, c = cw + cc;
                if (r >= g.R || c >= ncols) continue;
                u4 val = *reinterpret_cast<const u4*>(&stg[rr * SP + cc]);
                if constexpr (EPI == EPI_DX) {
                    if (g.mask) {
                        // keep the gradient where the forward activation is > 0 (ReLU)
                        const u4 m = *reinterpret_cast<const u4*>(g.mask + (int64_t)r * g.ldm + c);
#pragma unroll
                        for (int d = 0; d < 4; ++d) {
                            const unsigned lo = m[d] & 0xFFFFu, hi = m[d] >> 16;
                            const unsigned keep = ((lo != 0u && !(lo & 0x8000u)) ? 0xFFFFu : 0u) |
                                                  ((hi != 0u && !(hi & 0x8000u)) ? 0xFFFF0000u : 0u);
                            val[d] &= keep;
                        }
                    }
                }
                bf16* dst = g.out + (int64_t)r * g.ldo + c;
                if (c + 8 <= ncols) {
                    *reinterpret_cast<u4*>(dst) = val;
                } else {
                    const bf16x8 e8 = __builtin_bit_cast(bf16x8, val);
#pragma unroll
                    for (int e = 0; e < 8; ++e)
                        if (c + e < ncols) dst[e] = e8[e];
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
}

// Weight-resident row GEMM for the forward and input-gradient layers whose
// B (C <= 272 rows of Kc) fits in LDS: out[r][c] = sum_k A[r][k] B[c][k].
// One block per CU stages B in LDS once (rows padded to whole 16-row tiles
// with zeros, row stride Kc + 16 elements: a 16-byte LDS read is served 32
// lanes at a time over 32 slots of 16 bytes, and the lanes (row l, piece q)
// of a fragment read then fall in distinct slots, which a row stride of
// Kc + 8 (an odd number of slots) does not give); each wave then walks 16-row tiles of A on
// its own, with no block barrier: the tile's operand fragments come straight
// from memory (lane group q reads the 16-byte piece 8q of each 32-wide k
// step of its row) and the next tile's are loaded while the current one is
// computed. The product is formed transposed, out^T = B A^T, so a lane ends
// with four consecutive output columns of one row; pairs of lane groups
// swap halves so that each stores eight (16 bytes). Four output tiles are
// accumulated at a time, so consecutive MFMAs are independent.
// A 320-wide contraction (the skip layer: 256 features, 63 encoded inputs
// and the ones column that carries its bias) fills the LDS exactly with
// unpadded rows of 40 pieces (8 slots apart, mod 32): there the pieces of
// rows l .. l + 12 step 4 would share slots, so row l stores piece p at
// p ^ (2 ((l >> 2) & 3)), which gives the 32 lanes of a read distinct slots
// again and keeps every piece inside its row; it has no epilogue bias.
constexpr int RW_KS_SWZ = 10;
// waves per block: 16, or 8 for the 320-wide case, whose two 10-piece
// fragment buffers do not fit 128 registers (16 waves spill 10 and run no
// faster)
template <int KS>
constexpr int rw_waves() { return KS == RW_KS_SWZ ? 8 : 16; }

template <int KS>
constexpr int rw_kp() { return KS == RW_KS_SWZ ? 32 * KS : 32 * KS + 16; }   // LDS row stride (elements)

// Epilogue of two output tiles (a, b: the accumulators of tiles ta and ta+1
// for row r). A lane of an even group keeps its four columns of tile ta and
// takes the next four from its partner group (lane + 16); a lane of an odd
// group does the same for tile ta+1. Each lane then owns eight consecutive
// columns (16 bytes) and a row receives 64 contiguous bytes per store.
// The exchange is one v_permlane16_swap per element: it swaps the odd 16-lane
// rows of its first operand with the even rows of its second, which leaves
// the first operand holding (a of an even row, b of the even row below an
// odd row) and the second (a of the odd row above an even row, b of an odd
// row), exactly the lane's first and last four columns.
// First of the lane's eight columns in the epilogue of tiles ta, ta+1.
__device__ __forceinline__ int rw_col0(int ta, int g4) { return 16 * (ta + (g4 & 1)) + 4 * (g4 & 2); }

// The ReLU pattern of an input-gradient epilogue at those eight columns of
// row r (zero past ncols or past the last row): the forward activations, or
// their sign bits (one byte; c0 is a multiple of 8), loaded before the
// tiles' products so that the latency overlaps them.
struct MaskIn {
    bf16x8 m;
    uint32_t bits;
};
__device__ __forceinline__ MaskIn rw_mask(const GemmArgs& g, int r, int ta, int g4, int ncols) {
    MaskIn mi{};
    const int c0 = rw_col0(ta, g4);
    if (g.mbits_in) {
        mi.bits = (r < g.R && c0 < ncols) ? (uint32_t)g.mbits_in[(int64_t)r * g.ldb + (c0 >> 3)] : 0u;
        return mi;
    }
    const bf16* mp = g.mask + (int64_t)r * g.ldm + c0;
    if (r < g.R && c0 + 8 <= ncols) {
        mi.m = *reinterpret_cast<const bf16x8*>(mp);
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) mi.m[q] = (r < g.R && c0 + q < ncols) ? mp[q] : (bf16)0.0f;
    }
    return mi;
}

// Returns, for the forward epilogue with sign bits wanted, the lane's eight
// sign bits (0 past the last row or column); the caller packs them.
template <int EPI>
__device__ __forceinline__ uint32_t rw_epilogue2(const GemmArgs& g, int r, int ta, int g4, f32x4 a, f32x4 b,
                                                 int ncols, const MaskIn& m) {
    float x[8];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const auto sw = __builtin_amdgcn_permlane16_swap(__float_as_uint(a[q]), __float_as_uint(b[q]), false, false);
        x[q] = __uint_as_float(sw[0]);
        x[4 + q] = __uint_as_float(sw[1]);
    }
    const int c0 = rw_col0(ta, g4);
    if (r >= g.R) return 0u;
    if constexpr (EPI == EPI_FWD) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int c = c0 + q;
            float y = x[q];                                         // the bias is in the accumulator
            if (g.relu) y = y > 0.0f ? y : 0.0f;
            if (c == g.sig_col) g.sig[r] = y;
            x[q] = y;
        }
    }
    if (c0 >= ncols) return 0u;
    bf16x8 o;
#pragma unroll
    for (int q = 0; q < 8; ++q) o[q] = (bf16)x[q];
    const bool whole = c0 + 8 <= ncols;
    if constexpr (EPI == EPI_DX) {
        // keep the gradient where the forward activation is > 0 (ReLU)
        if (g.mbits_in) {
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (!((m.bits >> q) & 1u)) o[q] = (bf16)0.0f;
        } else if (g.mask) {
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (!((float)m.m[q] > 0.0f)) o[q] = (bf16)0.0f;
        }
    }
    uint32_t bits = 0;
    if constexpr (EPI == EPI_FWD) {
        if (g.mbits) {
#pragma unroll
            for (int q = 0; q < 8; ++q) bits |= (c0 + q < ncols && (float)o[q] > 0.0f) ? (1u << q) : 0u;
        }
    }
    bf16* dst = g.out + (int64_t)r * g.ldo + c0;
    if (whole) {
        *reinterpret_cast<bf16x8*>(dst) = o;
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (c0 + q < ncols) dst[q] = o[q];
    }
    return bits;
}

// The sign bits of output tiles ta, ta+1 of row r as one word, in lane group
// 0: lane groups 0, 2, 1, 3 hold columns 16 ta + 0, 8, 16, 24 of the row.
// The values of lanes + 16, + 32 and + 48 come from the half-swaps (the
// second result of a swap holds, in the lower row or half, the upper one of
// the first operand), with no LDS traffic; other lane groups get other
// values, which they do not use.
__device__ __forceinline__ uint32_t rw_bits_word(uint32_t b, int lane) {
    (void)lane;
    const uint32_t b2 = __builtin_amdgcn_permlane32_swap(b, b, false, false)[1];    // lanes 0..31: b[lane + 32]
    const uint32_t b1 = __builtin_amdgcn_permlane16_swap(b, b, false, false)[1];    // even rows: b[lane + 16]
    const uint32_t b3 = __builtin_amdgcn_permlane16_swap(b2, b2, false, false)[1];  // row 0: b[lane + 48]
    return b | (b2 << 8) | (b1 << 16) | (b3 << 24);
}

template <int EPI, int KS>
__global__ __launch_bounds__(64 * rw_waves<KS>(), 1) void k_rowmm(GemmArgs g, int CT) {
    constexpr int RW_WAVES = rw_waves<KS>();
    extern __shared__ __attribute__((aligned(16))) char rw_raw[];
    bf16* const wsm = reinterpret_cast<bf16*>(rw_raw);
    constexpr bool SWZ = KS == RW_KS_SWZ;
    constexpr int KP = rw_kp<KS>();
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    {
        constexpr int PQ = 4 * KS;                         // 16-byte pieces per row
        for (int i = tid; i < 16 * CT * PQ; i += 64 * RW_WAVES) {
            const int c = i / PQ, pq = i % PQ;
            const int sq = SWZ ? pq ^ (2 * ((c >> 2) & 3)) : pq;
            const u4 v = c < g.C ? *reinterpret_cast<const u4*>(g.B + (int64_t)c * g.b_sr + 8 * pq) : u4{0u, 0u, 0u, 0u};
            *reinterpret_cast<u4*>(wsm + c * KP + 8 * sq) = v;
        }
    }
    // the forward bias (zero past C) after the weights: each accumulator
    // starts from its four rows' biases
    float* const bsm = reinterpret_cast<float*>(wsm + 16 * CT * KP);
    if constexpr (EPI == EPI_FWD && !SWZ)
        for (int c = tid; c < 16 * CT; c += 64 * RW_WAVES) bsm[c] = (g.bias && c < g.C) ? g.bias[c] : 0.0f;
    __syncthreads();
    const int l16 = lane & 15, g4 = lane >> 4;
    const int ntile = (g.R + 15) / 16;
    const int stride = gridDim.x * RW_WAVES;
    const int ncols = EPI == EPI_FWD ? min(g.C, g.n_out) : g.C;
    // this lane's fragment origin; with the swizzle, piece 4 ks + g4 of row
    // l16 sits at 4 (ks ^ jh) + (g4 ^ 2 jl) for j = (l16 >> 2) & 3, so even
    // and odd k-steps take origins one k-step ahead and behind
    const int jsw = SWZ ? (l16 >> 2) & 3 : 0;
    const bf16* wl = wsm + l16 * KP + 8 * (g4 ^ (2 * (jsw & 1)));
    const bf16* wl_even = wl + ((jsw >> 1) ? 32 : 0);
    const bf16* wl_odd = wl - ((jsw >> 1) ? 32 : 0);
    bf16x8 xa[KS], xb[KS];
    auto load = [&](bf16x8* x, int tile) {
        const int row = tile * 16 + l16;
        const bf16* src = g.A + (int64_t)row * g.a_sr + 8 * g4;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
            x[ks] = row < g.R ? *reinterpret_cast<const bf16x8*>(src + 32 * ks) : bf16x8{};
    };
    auto tile_mm = [&](const bf16x8* x, int tile) {
        const int r = tile * 16 + l16;
        for (int ot0 = 0; ot0 < CT; ot0 += 4) {
            MaskIn m0{}, m1{};
            if constexpr (EPI == EPI_DX) {
                if (g.mask || g.mbits_in) {
                    m0 = rw_mask(g, r, ot0, g4, ncols);
                    if (ot0 + 2 < CT) m1 = rw_mask(g, r, ot0 + 2, g4, ncols);
                }
            }
            f32x4 acc[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int ot = ot0 + j < CT ? ot0 + j : CT - 1;
                if constexpr (EPI == EPI_FWD && !SWZ) acc[j] = *reinterpret_cast<const f32x4*>(bsm + 16 * ot + 4 * g4);
                else acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int ot = ot0 + j < CT ? ot0 + j : CT - 1;   // past the last tile: recompute it, unused
                    const bf16* wk = SWZ ? ((ks & 1) ? wl_odd : wl_even) : wl;
                    const bf16x8 w = *reinterpret_cast<const bf16x8*>(wk + 16 * ot * KP + 32 * ks);
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, x[ks], acc[j], 0, 0, 0);
                }
            // tiles past CT were computed from a repeated fragment: their
            // columns lie beyond C and are neither stored nor read
            const uint32_t s0 = rw_epilogue2<EPI>(g, r, ot0, g4, acc[0], acc[1], ncols, m0);
            const uint32_t s1 = ot0 + 2 < CT ? rw_epilogue2<EPI>(g, r, ot0 + 2, g4, acc[2], acc[3], ncols, m1) : 0u;
            if constexpr (EPI == EPI_FWD) {
                if (g.mbits) {
                    // 64 columns of sign bits per row: one 8-byte store (4 if
                    // only the first 32 columns exist) by lane group 0
                    const uint32_t w0 = rw_bits_word(s0, lane), w1 = rw_bits_word(s1, lane);
                    if (g4 == 0 && r < g.R && 16 * ot0 < ncols) {
                        uint8_t* bp = g.mbits + (int64_t)r * g.ldb + 2 * ot0;
                        if (16 * ot0 + 32 < ncols) *reinterpret_cast<uint2*>(bp) = uint2{w0, w1};
                        else *reinterpret_cast<uint32_t*>(bp) = w0;
                    }
                }
            }
        }
    };
    int t = blockIdx.x * RW_WAVES + wv;
    if (t < ntile) load(xa, t);
    // two tiles per round with the fragment buffers alternating, so the
    // loads in flight are never copied
    for (; t < ntile; t += 2 * stride) {
        const int t1 = t + stride;
        if (t1 < ntile) load(xb, t1);
        tile_mm(xa, t);
        if (t1 >= ntile) break;
        const int t2 = t1 + stride;
        if (t2 < ntile) load(xa, t2);
        tile_mm(xb, t1);
    }
}

template <int EPI, int KS>
static hipError_t rowmm_launch(const GemmArgs& a, int CT, size_t lds, hipStream_t st) {
    static bool attr = false;      // more than 64 KB of dynamic LDS must be allowed explicitly
    if (!attr) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rowmm<EPI, KS>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const int ntile = (a.R + 15) / 16;
    constexpr int RW_WAVES = rw_waves<KS>();
    const int blocks = std::max(1, std::min(256, (ntile + RW_WAVES - 1) / RW_WAVES));
    hipLaunchKernelGGL((k_rowmm<EPI, KS>), dim3(blocks), dim3(64 * RW_WAVES), lds, st, a, CT);
    return hipGetLastError();
}

// LDS bytes of the weight-resident kernel: the weights, then (except for
// the swizzled 320-wide case, which has no epilogue bias) the bias.
static size_t rowmm_lds(const GemmArgs& a) {
    const int KS = a.Kc / 32, CT = (a.C + 15) / 16;
    if (KS == RW_KS_SWZ) return (size_t)16 * CT * a.Kc * sizeof(bf16);
    return (size_t)16 * CT * (a.Kc + 16) * sizeof(bf16) + (size_t)16 * CT * sizeof(float);
}

// The weight-resident kernel when B fits: returns false if it does not apply
// (the 320-wide case only for a forward layer without an epilogue bias).
static bool rowmm_applies(const GemmArgs& a, int epi) {
    if (a.Kc % 32 || a.C > 272 || a.R < 1) return false;
    const int KS = a.Kc / 32;
    if (KS == RW_KS_SWZ && (epi != EPI_FWD || a.bias)) return false;
    return rowmm_lds(a) <= (size_t)160 * 1024 &&
           (KS == 1 || KS == 2 || KS == 4 || KS == 8 || KS == 9 || KS == RW_KS_SWZ);
}

template <int EPI>
static bool rowmm(const GemmArgs& a, hipStream_t st, hipError_t* err) {
    if (!rowmm_applies(a, EPI)) return false;
    const int KS = a.Kc / 32, CT = (a.C + 15) / 16;
    const size_t lds = rowmm_lds(a);
    switch (KS) {
    case 1: *err = rowmm_launch<EPI, 1>(a, CT, lds, st); return true;
    case 2: *err = rowmm_launch<EPI, 2>(a, CT, lds, st); return true;
    case 4: *err = rowmm_launch<EPI, 4>(a, CT, lds, st); return true;
    case 8: *err = rowmm_launch<EPI, 8>(a, CT, lds, st); return true;
    case 9: *err = rowmm_launch<EPI, 9>(a, CT, lds, st); return true;
    case RW_KS_SWZ:
        if constexpr (EPI == EPI_FWD) { *err = rowmm_launch<EPI, RW_KS_SWZ>(a, CT, lds, st); return true; }
        return false;
    default: return false;
    }
}

// Weight-gradient GEMM, tile GT x GT over one slice of the samples, DK
// samples per step. Threads 0..127 load an 8 (samples) x 8 (columns) block
// of A, threads 128..255 one of B, and transpose it in registers so that each
// LDS row (one output row n, or one input column k') holds DK consecutive
// samples: the MFMA fragments are then plain 16-byte LDS reads. The next
// step's blocks are loaded while this step's MFMAs run. Bias gradients (row
// sums of A over the samples) come from extra MFMAs against a ones fragment.
// LDS rows are 160 bytes (ten 16-byte slots, an even number not divisible
// by four): a 16-byte read is served 32 lanes at a time over 32 slots, and
// the fragment reads (16 rows, two pieces per 32 lanes) then fall in
// distinct slots. Within a row the eight 8-sample chunks are permuted by an
// XOR with 2 ((row >> 4) & 3), which spreads the transposed 16-byte stores
// of a wave (16 or 32 column blocks, rows 8 apart) while the 16 rows a
// fragment read covers share one permutation.
constexpr int DK = 64;
constexpr int DPAD = DK + 16;   // 160-byte LDS rows

__device__ __forceinline__ void transpose8(const u4 in[8], u4 out[8]) {
    // in[q] = 8 columns of sample row q (two 16-bit columns per dword);
    // out[e] = 8 samples of column e (two consecutive samples per dword)
#pragma unroll
    for (int d = 0; d < 4; ++d)
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const unsigned lo = in[2 * p][d], hi = in[2 * p + 1][d];
            out[2 * d][p] = (lo & 0xFFFFu) | (hi << 16);
            out[2 * d + 1][p] = (lo >> 16) | (hi & 0xFFFF0000u);
        }
}

// TILE x TILE output tile: TILE = 128 with four waves of 64 x 64, or
// TILE = 256 with eight waves of 64 x 128 (then each sample row of the
// operands is read once per slice for a 256 x 256 layer).
template <int TILE>
__global__ __launch_bounds__(2 * TILE) void k_gemm_dw(GemmArgs g) {
    constexpr int WM = TILE / 64, NW = 2 * TILE / 64, WNC = NW / WM, WCW = TILE / WNC, TJ = WCW / 16;
    static_assert(WCW % 64 == 0, "a wave's first operand row is a multiple of 64 (chunk permutation i & 3, j & 3)");
    extern __shared__ __attribute__((aligned(16))) char dw_smem[];
    bf16* la = reinterpret_cast<bf16*>(dw_smem);
    bf16* lb = la + TILE * DPAD;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wm = wv % WM, wn = wv / WM;
    const int r0 = blockIdx.x * TILE, c0 = blockIdx.y * TILE;
    const int slice = blockIdx.z;
    const int64_t mbeg = (int64_t)slice * g.Kc;
    const int64_t mend = min(mbeg + g.Kc, g.Mtot);
    // this thread's 8 x 8 block: samples 8 mb .. 8 mb + 7 of the step, columns 8 cb .. 8 cb + 7
    const bool isA = tid < TILE;
    const int blk = tid % TILE, mb = blk / (TILE / 8), cb = blk % (TILE / 8);
    const bf16* src = isA ? g.A : g.B;
    const int64_t sr = isA ? g.a_sr : g.b_sr;
    const int col = (isA ? r0 : c0) + 8 * cb;
    const bool col_ok = col < (isA ? g.a_lim : g.b_lim);
    bf16* dst = (isA ? la : lb) + 8 * cb * DPAD + 8 * (mb ^ (2 * ((cb >> 1) & 3)));
    const bool do_bias = g.boff >= 0 && blockIdx.y == 0 && wn == 0;
    f32x4 acc[4][TJ], accb[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        accb[i] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int j = 0; j < TJ; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    bf16x8 ones;
#pragma unroll
    for (int e = 0; e < 8; ++e) ones[e] = (bf16)1.0f;
    u4 v[8];
#define R360_DWLOAD(m0)                                                                                  \
    _Pragma("unroll") for (int q = 0; q < 8; ++q) {                                                      \
        const int64_t m = (m0) + 8 * mb + q;                                                             \
        v[q] = (col_ok && m < mend) ? *reinterpret_cast<const u4*>(src + m * sr + col) : u4{0u, 0u, 0u, 0u}; \
    }
    R360_DWLOAD(mbeg)
    for (int64_t m0 = mbeg; m0 < mend; m0 += DK) {
        u4 t[8];
        transpose8(v, t);
        __syncthreads();                       // the previous step's fragments have been read
#pragma unroll
        for (int e = 0; e < 8; ++e) *reinterpret_cast<u4*>(dst + e * DPAD) = t[e];
        __syncthreads();
        if (m0 + DK < mend) R360_DWLOAD(m0 + DK)
#pragma unroll
        for (int ks = 0; ks < DK / 32; ++ks) {
            bf16x8 fa[4], fb[TJ];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                fa[i] = *reinterpret_cast<const bf16x8*>(&la[(64 * wm + 16 * i + (lane & 15)) * DPAD + 8 * ((4 * ks + (lane >> 4)) ^ (2 * (i & 3)))]);
#pragma unroll
            for (int j = 0; j < TJ; ++j)
                fb[j] = *reinterpret_cast<const bf16x8*>(&lb[(WCW * wn + 16 * j + (lane & 15)) * DPAD + 8 * ((4 * ks + (lane >> 4)) ^ (2 * (j & 3)))]);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < TJ; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
            if (do_bias) {
#pragma unroll
                for (int i = 0; i < 4; ++i) accb[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], ones, accb[i], 0, 0, 0);
            }
        }
    }
#undef R360_DWLOAD
    const int g4 = lane >> 4, l16 = lane & 15;
    float* part = g.part + (int64_t)slice * g.pstride;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = r0 + 64 * wm + 16 * i + 4 * g4 + q;
            if (r >= g.R) continue;
#pragma unroll
            for (int j = 0; j < TJ; ++j) {
                const int c = c0 + WCW * wn + 16 * j + l16;
                if (c < g.C) part[(int64_t)r * g.ldp + c] = acc[i][j][q];
            }
            if (do_bias && l16 == 0) part[g.boff + r] = accb[i][q];
        }
    }
}

// dZ11 = drgb * s (1 - s) in the first 3 of 32 columns; dZhead column w = dsigma * [sigma > 0].
__global__ void k_gout_grads(int64_t M, const float* __restrict__ rgb, const float* __restrict__ drgb,
                             bf16* __restrict__ dz11, const float* __restrict__ sig, const float* __restrict__ dsig,
                             bf16* __restrict__ dzh, int ldh, int w) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    // both rows are written as whole 16-byte pieces: dz11 is 32 columns wide,
    // and dzh's columns w .. ldh - 1 are the 32 after the w feature rows
    // (w and ldh = w + 32 are multiples of 32)
    bf16x8 z[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int e = 0; e < 8; ++e) z[j][e] = (bf16)0.0f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float s = rgb[c * M + m];
        z[0][c] = (bf16)(drgb[c * M + m] * s * (1.0f - s));
    }
    bf16x8* d11 = reinterpret_cast<bf16x8*>(dz11 + m * 32);
#pragma unroll
    for (int j = 0; j < 4; ++j) d11[j] = z[j];
    z[0][0] = (bf16)(sig[m] > 0.0f ? dsig[m] : 0.0f);
    z[0][1] = (bf16)0.0f; z[0][2] = (bf16)0.0f;
    bf16x8* dh = reinterpret_cast<bf16x8*>(dzh + m * ldh + w);
#pragma unroll
    for (int j = 0; j < 4; ++j) dh[j] = z[j];
}

// Per-sample density max into the occupancy grid. The density is >= 0 (its
// bits as a signed integer are >= 0 and ordered like the floats), and every
// negative float (-0 included) has a negative signed pattern, so a signed
// integer max gives max(cell, sigma) whatever non-NaN value the cell held.
// Consecutive samples of a ray that lie in one cell are neighbouring lanes:
// each run's first lane takes the maximum over the run (a doubling over the
// following lanes with the same cell; lanes of the same cell further on may
// join it, which changes nothing) and alone issues the atomic.
__global__ __launch_bounds__(256) void k_gocc(int64_t M, const float* __restrict__ sig,
                                              const int32_t* __restrict__ voxel, int* __restrict__ grid) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int v = -1, best = 0;
    if (m < M) {
        v = voxel[m];
        best = __float_as_int(sig[m] > 0.0f ? sig[m] : 0.0f);
    }
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int vo = __shfl_down(v, d, 64);
        const int bo = __shfl_down(best, d, 64);
        if (lane + d < 64 && vo == v) best = max(best, bo);
    }
    const int prev = __shfl_up(v, 1, 64);
    if (v >= 0 && (lane == 0 || prev != v)) atomicMax(grid + v, best);
}

GNetDev dev_net(const GNet& n) {
    GNetDev d;
    d.w = n.w; d.c = n.c; d.P = n.P;
    for (int i = 0; i < NGL; ++i) d.L[i] = n.L[i];
    return d;
}

}  // namespace

// Workspace of the global stage.
// Sign bits of the ReLU outputs that later mask an input gradient: h1..h7,
// the feature f (x10's first columns) and h10.
enum { MB_F = 8, MB_H10 = 9, MB_N = 10 };
struct GlobalWs {
    bf16 *arena, *x5, *h[9], *x10, *h10, *dza, *dzb, *dz11;   // h[1..3], h[5..8]
    uint8_t* mb[MB_N];                                        // mb[1..7], mb[MB_F], mb[MB_H10]
    float *bias, *sig, *rgb, *t, *delta, *dsig, *drgb, *part, *ray_rgb, *ray_grad, *loss_part;
    int32_t *voxel, *ray, *ray_off;
    size_t bytes;
};

constexpr int G_SLICES = 256;     // sample slices of the weight-gradient GEMMs

static GlobalWs gcarve(void* base, const GNet& n, int64_t Nr, int S) {
    GlobalWs g{};
    const int64_t M = Nr * S;
    char* p = static_cast<char*>(base);
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        char* q = p ? p + off : nullptr;
        off += (bytes + 255) & ~size_t(255);
        return q;
    };
    const int w = n.w;
    g.arena = (bf16*)take(n.w_elems * 2);
    g.bias = (float*)take(n.b_elems * 4);
    g.x5 = (bf16*)take(M * (w + 64) * 2);
    for (int k : {1, 2, 3, 5, 6, 7, 8}) g.h[k] = (bf16*)take(M * w * 2);
    g.x10 = (bf16*)take(M * n.L[G10].K * 2);
    g.h10 = (bf16*)take(M * n.c * 2);
    g.dza = (bf16*)take(M * (w + 64) * 2);
    g.dzb = (bf16*)take(M * (w + 64) * 2);
    g.dz11 = (bf16*)take(M * 32 * 2);
    g.sig = (float*)take(M * 4);
    g.rgb = (float*)take(3 * M * 4);
    g.t = (float*)take(M * 4);
    g.delta = (float*)take(M * 4);
    g.dsig = (float*)take(M * 4);
    g.drgb = (float*)take(3 * M * 4);
    g.voxel = (int32_t*)take(M * 4);
    g.ray = (int32_t*)take(M * 4);
    g.ray_off = (int32_t*)take((Nr + 1) * 4);
    g.part = (float*)take((size_t)G_SLICES * n.g_elems * 4);
    g.ray_rgb = (float*)take(3 * Nr * 4);
    g.ray_grad = (float*)take(3 * Nr * 4);
    g.loss_part = (float*)take(((Nr + 255) / 256) * 4);
    for (int k = 1; k <= 7; ++k) g.mb[k] = (uint8_t*)take(M * (w / 8));
    g.mb[MB_F] = (uint8_t*)take(M * (w / 8));
    g.mb[MB_H10] = (uint8_t*)take(M * (n.c / 8));
    g.bytes = off;
    return g;
}

size_t global_workspace_bytes(int w, int c, int64_t Nr, int S) { return gcarve(nullptr, make_net(w, c), Nr, S).bytes; }
int64_t global_params(int w, int c) { return make_net(w, c).P; }

static hipError_t gemm(int epi, GemmArgs a, int slices, hipStream_t st) {
    if (epi == EPI_DW) {
        // 256 x 256 tiles when both sides reach 256 (each operand row read once per slice for a 256 x 256
        // layer; a 257 x 256 or 256 x 320 layer reads one operand twice, where 128 x 128 tiles read
        // both two or three times); 128 x 128 otherwise
        const size_t lds256 = (size_t)2 * 256 * DPAD * sizeof(bf16), lds128 = (size_t)2 * 128 * DPAD * sizeof(bf16);
        if (a.R >= 256 && a.C >= 256) {
            static bool attr = false;       // more than 64 KB of dynamic LDS must be allowed explicitly
            if (!attr) {
                const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gemm_dw<256>),
                                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds256);
                if (e != hipSuccess) return e;
                attr = true;
            }
            hipLaunchKernelGGL(k_gemm_dw<256>, dim3((a.R + 255) / 256, (a.C + 255) / 256, slices), dim3(512), lds256, st,
                               a);
        }
        else
            hipLaunchKernelGGL(k_gemm_dw<128>, dim3((a.R + GT - 1) / GT, (a.C + GT - 1) / GT, slices), dim3(256), lds128,
                               st, a);
        return hipGetLastError();
    }
    {
        hipError_t e = hipSuccess;
        if (epi == EPI_FWD && rowmm<EPI_FWD>(a, st, &e)) return e;
        if (epi == EPI_DX && rowmm<EPI_DX>(a, st, &e)) return e;
    }
    // full-width tiles for 256 output columns (each input row is read once); 128 otherwise
    const bool wide = a.C > 128 && a.C <= 256;
    const dim3 grid((a.R + GT - 1) / GT, wide ? 1 : (a.C + 127) / 128);
    switch (epi) {
    case EPI_FWD:
        if (wide) hipLaunchKernelGGL((k_gemm<EPI_FWD, 256>), grid, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_gemm<EPI_FWD, 128>), grid, dim3(256), 0, st, a);
        break;
    case EPI_RGB: hipLaunchKernelGGL((k_gemm<EPI_RGB, 128>), grid, dim3(256), 0, st, a); break;
    default:
        if (wide) hipLaunchKernelGGL((k_gemm<EPI_DX, 256>), grid, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_gemm<EPI_DX, 128>), grid, dim3(256), 0, st, a);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_global_step(const r360_global_desc* desc, const float* weights, const float* o, const float* d,
                              int64_t Nr, const float* target, float* loss, float* grad, float* rgb_out,
                              float* depth_out, float* occ, void* ws, hipStream_t st, int stage_mask,
                              const GlobalMeasure* meas) {
    const GNet n = make_net(desc->width, desc->color_width);
    const GNetDev nd = dev_net(n);
    const int S = desc->n_samples, w = n.w, c = n.c;
    const int64_t M = Nr * S;
    GlobalWs g = gcarve(ws, n, Nr, S);
    const unsigned nbP = (unsigned)((n.P + 255) / 256);
    hipLaunchKernelGGL(k_gzero, dim3(256), dim3(256), 0, st, reinterpret_cast<u32*>(g.arena), (n.w_elems + 1) / 2);
    hipLaunchKernelGGL(k_gnet_pack, dim3(nbP), dim3(256), 0, st, nd, weights, g.arena, g.bias);
    // samples and encodings
    GSampleArgs sa;
    sa.o = o; sa.d = d; sa.N = Nr; sa.S = S;
    sa.a_near = 1.0f / desc->near_; sa.b_far = 1.0f / desc->far_;
    sa.c0 = desc->center[0]; sa.c1 = desc->center[1]; sa.c2 = desc->center[2];
    sa.inv_h = 1.0f / desc->half_extent;
    sa.lo0 = desc->grid_lo[0]; sa.lo1 = desc->grid_lo[1]; sa.lo2 = desc->grid_lo[2];
    sa.inv_vox = 1.0f / desc->voxel;
    sa.g0 = desc->grid_n[0]; sa.g1 = desc->grid_n[1]; sa.g2 = desc->grid_n[2];
    sa.x5 = g.x5; sa.x10 = g.x10; sa.w = w; sa.k10 = n.L[G10].K;
    sa.t = g.t; sa.delta = g.delta; sa.voxel = g.voxel; sa.ray = g.ray; sa.ray_off = g.ray_off;
    sa.points = (meas && meas->points) ? 1 : 0;
    hipLaunchKernelGGL(k_gsamples, dim3((unsigned)((std::max<int64_t>(M, Nr + 1) + 255) / 256)), dim3(256), 0, st, sa);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;

    const bf16* W = g.arena;
    auto Wm = [&](int ly) { return W + n.L[ly].w_off; };
    auto Wt = [&](int ly) { return W + n.L[ly].t_off; };
    auto Bv = [&](int ly) { return n.L[ly].b_off >= 0 ? g.bias + n.L[ly].b_off : nullptr; };
    const int64_t ld5 = w + 64, ld10 = n.L[G10].K;
    // ReLU sign bits written by the forward layers that run in the
    // weight-resident kernel (null where another kernel ran), with their row
    // strides in bytes
    const uint8_t* bits[MB_N] = {};
    int64_t bits_ld[MB_N] = {};
    auto want_bits = [&](GemmArgs& a, int k) {
        if (k < 0 || !(stage_mask & 2) || !rowmm_applies(a, EPI_FWD)) return;     // only when a backward follows
        a.mbits = g.mb[k]; a.ldb = a.n_out / 8;
        bits[k] = a.mbits; bits_ld[k] = a.ldb;
    };
    // forward: layer(A input [M x K] with row stride lda) -> out
    auto fwd = [&](int ly, const bf16* A, int64_t lda, bf16* out, int64_t ldo, bool relu, int mbk) {
        GemmArgs a{};
        a.A = A; a.a_sr = lda; 
        a.B = Wm(ly); a.b_sr = n.L[ly].K;
        a.R = (int)M; a.C = n.L[ly].N; a.Kc = n.L[ly].K;
        a.bias = Bv(ly); a.relu = relu; a.out = out; a.ldo = ldo; a.n_out = n.L[ly].N; a.sig_col = -1;
        want_bits(a, mbk);
        return gemm(EPI_FWD, a, 1, st);
    };
    if ((e = fwd(G1, g.x5 + w, ld5, g.h[1], w, true, 1)) != hipSuccess) return e;
    if ((e = fwd(G2, g.h[1], w, g.h[2], w, true, 2)) != hipSuccess) return e;
    if ((e = fwd(G3, g.h[2], w, g.h[3], w, true, 3)) != hipSuccess) return e;
    if ((e = fwd(G4, g.h[3], w, g.x5, ld5, true, 4)) != hipSuccess) return e;
    if ((e = fwd(G5, g.x5, ld5, g.h[5], w, true, 5)) != hipSuccess) return e;
    if ((e = fwd(G6, g.h[5], w, g.h[6], w, true, 6)) != hipSuccess) return e;
    if ((e = fwd(G7, g.h[6], w, g.h[7], w, true, 7)) != hipSuccess) return e;
    if ((e = fwd(G8, g.h[7], w, g.h[8], w, false, -1)) != hipSuccess) return e;
    {   // head: relu(Wf h8 + bf) -> x10[:, :w]; relu(ws h8 + bs) -> sigma
        GemmArgs a{};
        a.A = g.h[8]; a.a_sr = w; 
        a.B = Wm(GH); a.b_sr = w;
        a.R = (int)M; a.C = w + 1; a.Kc = w;
        a.bias = Bv(GH); a.relu = true; a.out = g.x10; a.ldo = ld10; a.n_out = w; a.sig_col = w; a.sig = g.sig;
        want_bits(a, MB_F);
        if ((e = gemm(EPI_FWD, a, 1, st)) != hipSuccess) return e;
    }
    if ((e = fwd(G10, g.x10, ld10, g.h10, c, true, MB_H10)) != hipSuccess) return e;
    {
        GemmArgs a{};
        a.A = g.h10; a.a_sr = c; 
        a.B = Wm(G11); a.b_sr = c;
        a.R = (int)M; a.C = 3; a.Kc = c;
        a.bias = Bv(G11); a.rgb = g.rgb;
        if ((e = gemm(EPI_RGB, a, 1, st)) != hipSuccess) return e;
    }
    if (meas && meas->points) {
        if ((e = hipMemcpyAsync(meas->point_sigma, g.sig, M * sizeof(float), hipMemcpyDeviceToDevice, st)) != hipSuccess)
            return e;
        return hipMemcpyAsync(meas->point_rgb, g.rgb, 3 * M * sizeof(float), hipMemcpyDeviceToDevice, st);
    }
    if (occ) hipLaunchKernelGGL(k_gocc, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st, M, g.sig, g.voxel,
                                reinterpret_cast<int*>(occ));
    // compositing, loss and its backward reuse the local path's kernels
    Workspace lw{};
    lw.ray_off = g.ray_off; lw.ray = g.ray; lw.sigma = g.sig; lw.rgb = g.rgb; lw.t_mid = g.t; lw.delta = g.delta;
    lw.dsigma = g.dsig; lw.drgb = g.drgb; lw.loss_part = g.loss_part; lw.N = Nr; lw.cap = M;
    float* ray_rgb = rgb_out ? rgb_out : g.ray_rgb;
    if ((e = launch_composite(lw, Nr, ray_rgb, depth_out, nullptr, st)) != hipSuccess) return e;
    if (meas && meas->depth &&
        (e = launch_depth_stats(g.t, g.delta, g.sig, Nr, S, meas->depth, meas->uncert, meas->opacity, st)) != hipSuccess)
        return e;
    if (!(stage_mask & 2)) return hipSuccess;      // forward only
    if ((e = launch_loss_grad(lw, Nr, ray_rgb, target, loss, g.ray_grad, st)) != hipSuccess) return e;
    if ((e = launch_composite_backward(lw, Nr, g.ray_grad, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_gout_grads, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st, M, g.rgb, g.drgb, g.dz11,
                       g.sig, g.dsig, g.dzb, (int)up32(w + 1), w);

    // samples per slice: a multiple of the GEMM's step; the last slice is clipped to M
    const int64_t kslice = ((M + G_SLICES - 1) / G_SLICES + DK - 1) / DK * DK;
    // input gradient: dX[M x K'] = dZ [M x NC] . W^T -> masked by act (if any)
    // (mbk: the sign bits of act, used in its place when the forward wrote
    // them and this product runs in the weight-resident kernel)
    auto dx = [&](int ly, const bf16* dz, int64_t ldz, bf16* out, int64_t ldo, int ncols, const bf16* act,
                  int64_t ldact, int mbk) {
        GemmArgs a{};
        a.A = dz; a.a_sr = ldz; 
        a.B = Wt(ly); a.b_sr = n.L[ly].NC;
        a.R = (int)M; a.C = ncols; a.Kc = n.L[ly].NC;
        a.out = out; a.ldo = ldo; a.mask = act; a.ldm = ldact;
        if (mbk >= 0 && bits[mbk] && rowmm_applies(a, EPI_DX)) { a.mbits_in = bits[mbk]; a.ldb = bits_ld[mbk]; }
        return gemm(EPI_DX, a, 1, st);
    };
    // weight gradient partials: dW[N x K] = dZ^T [N x M] . X [M x K], sliced over M
    auto dw = [&](int ly, const bf16* dz, int64_t ldz, const bf16* x, int64_t ldx) {
        GemmArgs a{};
        a.A = dz; a.a_sr = ldz; a.a_lim = (int)std::min<int64_t>(ldz, up32(n.L[ly].N));
        a.B = x; a.b_sr = ldx; a.b_lim = n.L[ly].K;
        a.R = n.L[ly].N; a.C = n.L[ly].K; a.Kc = (int)kslice; a.Mtot = M;
        a.part = g.part + n.L[ly].g_off; a.pstride = n.g_elems; a.ldp = n.L[ly].K;
        a.boff = n.L[ly].gb_off >= 0 ? n.L[ly].gb_off - n.L[ly].g_off : -1;
        return gemm(EPI_DW, a, G_SLICES, st);
    };
    const int ldh = up32(w + 1);
    // L11
    if ((e = dw(G11, g.dz11, 32, g.h10, c)) != hipSuccess) return e;
    if ((e = dx(G11, g.dz11, 32, g.dza, c, c, g.h10, c, MB_H10)) != hipSuccess) return e;      // dz10
    // L10 (feature part of the input only) -> dZf into dzb[:, :w]
    if ((e = dw(G10, g.dza, c, g.x10, ld10)) != hipSuccess) return e;
    if ((e = dx(G10, g.dza, c, g.dzb, ldh, w, g.x10, ld10, MB_F)) != hipSuccess) return e;
    // head -> dz8 (layer 8 is linear)
    if ((e = dw(GH, g.dzb, ldh, g.h[8], w)) != hipSuccess) return e;
    if ((e = dx(GH, g.dzb, ldh, g.dza, w, w, nullptr, 0, -1)) != hipSuccess) return e;
    // layers 8..6
    bf16* cur = g.dza; bf16* nxt = g.dzb;
    const int back[3] = {G8, G7, G6};
    const bf16* inputs[3] = {g.h[7], g.h[6], g.h[5]};
    for (int q = 0; q < 3; ++q) {
        if ((e = dw(back[q], cur, w, inputs[q], w)) != hipSuccess) return e;
        if ((e = dx(back[q], cur, w, nxt, w, w, inputs[q], w, 7 - q)) != hipSuccess) return e;
        std::swap(cur, nxt);
    }
    // layer 5: input [h4 | gx | 1]; only the h4 part propagates
    if ((e = dw(G5, cur, w, g.x5, ld5)) != hipSuccess) return e;
    if ((e = dx(G5, cur, w, nxt, w, w, g.x5, ld5, 4)) != hipSuccess) return e;
    std::swap(cur, nxt);
    const int back2[3] = {G4, G3, G2};
    const bf16* inputs2[3] = {g.h[3], g.h[2], g.h[1]};
    for (int q = 0; q < 3; ++q) {
        if ((e = dw(back2[q], cur, w, inputs2[q], w)) != hipSuccess) return e;
        if ((e = dx(back2[q], cur, w, nxt, w, w, inputs2[q], w, 3 - q)) != hipSuccess) return e;
        std::swap(cur, nxt);
    }
    if ((e = dw(G1, cur, w, g.x5 + w, ld5)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_gnet_grad, dim3((unsigned)((4 * n.P + 255) / 256)), dim3(256), 0, st, nd, g.part, n.g_elems,
                       G_SLICES, grad);
    return hipGetLastError();
}

}  // namespace r360
