// Internal declarations shared by the HIP translation units of libr360.
// Device helpers (MFMA fragment types, the exact-argument sin/cos of pi x,
// encoding slot tables) and the host-side launcher prototypes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "r360.h"

namespace r360 {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(8))) _Float16 f16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

constexpr int WAVE = 64;
constexpr int LXYZ = 10;                 // position encoding frequencies
constexpr int LDIR = 4;                  // direction encoding frequencies
constexpr int DXYZ = 3 + 6 * LXYZ;       // 63
constexpr int DDIR = 3 + 6 * LDIR;       // 27

// ---------------------------------------------------------------------------
// Canonical parameter offsets of one local field (hidden width h):
// W1[h x 63] b1 W2[h x h] b2 ws[1 x h] bs Wf[h x h] bf W3[h x (h+27)] b3 W4[3 x h] b4
// ---------------------------------------------------------------------------
struct FieldLayout {
    int h;
    __host__ __device__ constexpr int W1() const { return 0; }
    __host__ __device__ constexpr int b1() const { return h * DXYZ; }
    __host__ __device__ constexpr int W2() const { return b1() + h; }
    __host__ __device__ constexpr int b2() const { return W2() + h * h; }
    __host__ __device__ constexpr int ws() const { return b2() + h; }
    __host__ __device__ constexpr int bs() const { return ws() + h; }
    __host__ __device__ constexpr int Wf() const { return bs() + 1; }
    __host__ __device__ constexpr int bf() const { return Wf() + h * h; }
    __host__ __device__ constexpr int W3() const { return bf() + h; }
    __host__ __device__ constexpr int b3() const { return W3() + h * (h + DDIR); }
    __host__ __device__ constexpr int W4() const { return b3() + h; }
    __host__ __device__ constexpr int b4() const { return W4() + 3 * h; }
    __host__ __device__ constexpr int P() const { return b4() + 3; }
};

// ---------------------------------------------------------------------------
// Encoding slots. Each lane group g (lanes 16g..16g+15 of a wave) evaluates
// 16 position-encoding values and 8 direction-encoding values of its sample
// with one uniform instruction stream; these tables say which canonical
// encoding feature each (g, slot) holds. Canonical feature index:
// 0..2 raw components, 3 + 6l + c = sin(2^l pi x_c), 6 + 6l + c = cos(...).
// SLOT_BIAS carries a constant 1 (the layer bias); SLOT_ZERO is padding.
// ---------------------------------------------------------------------------
constexpr int SLOT_BIAS = -1;
constexpr int SLOT_ZERO = -2;

__host__ __device__ constexpr int pe_slot_feature(int g, int s) {
    // g < 3: component g, frequency m = s/2 (sin even, cos odd), m = 0..7.
    // g = 3: frequencies 8 and 9 of x, y, z plus the raw components and the bias.
    return g < 3 ? ((s & 1) ? 6 + 6 * (s >> 1) + g : 3 + 6 * (s >> 1) + g)
                 : (s == 0 ? 51 : s == 1 ? 54 : s == 2 ? 57 : s == 3 ? 60 : s == 4 ? 0 : s == 5 ? 1 :
                    s == 6 ? 52 : s == 7 ? 55 : s == 8 ? 58 : s == 9 ? 61 : s == 10 ? 2 : s == 11 ? SLOT_BIAS :
                    s == 12 ? 53 : s == 13 ? 56 : s == 14 ? 59 : 62);
}
__host__ __device__ constexpr int dir_slot_feature(int g, int s) {
    return g < 3 ? ((s & 1) ? 6 + 6 * (s >> 1) + g : 3 + 6 * (s >> 1) + g)
                 : (s < 3 ? s : s == 3 ? SLOT_BIAS : SLOT_ZERO);
}

// ---------------------------------------------------------------------------
// sin(pi x) and cos(pi x) for an exactly known FP32 argument x.
// x = n/2 + f with n = rint(2x) and |f| <= 1/4 (the subtraction is exact);
// then truncated Taylor series of sin(pi f)/f and cos(pi f), whose first
// omitted terms are below 2e-9 on |f| <= 1/4, and the quadrant n mod 4.
// ---------------------------------------------------------------------------
constexpr double PI_D = 3.14159265358979323846;
constexpr double pw(double x, int k) { return k == 0 ? 1.0 : x * pw(x, k - 1); }
constexpr double fact(int k) { return k <= 1 ? 1.0 : k * fact(k - 1); }
constexpr float TS(int k) { return (float)(((k / 2) % 2 ? -1.0 : 1.0) * pw(PI_D, k) / fact(k)); }
// evaluated at compile time (constexpr variables), never at run time
constexpr float kS1 = TS(1), kS3 = TS(3), kS5 = TS(5), kS7 = TS(7), kS9 = TS(9);
constexpr float kC2 = TS(2), kC4 = TS(4), kC6 = TS(6), kC8 = TS(8), kC10 = TS(10);

__device__ __forceinline__ void sincospi(float x, float& s, float& c) {
    const float n = __builtin_rintf(x + x);
    const float f = __builtin_fmaf(n, -0.5f, x);
    const float f2 = f * f;
    float ps = __builtin_fmaf(f2, kS9, kS7);
    ps = __builtin_fmaf(f2, ps, kS5);
    ps = __builtin_fmaf(f2, ps, kS3);
    ps = __builtin_fmaf(f2, ps, kS1);
    ps = ps * f;
    float pc = __builtin_fmaf(f2, kC10, kC8);
    pc = __builtin_fmaf(f2, pc, kC6);
    pc = __builtin_fmaf(f2, pc, kC4);
    pc = __builtin_fmaf(f2, pc, kC2);
    pc = __builtin_fmaf(f2, pc, 1.0f);
    const int q = (int)n & 3;
    float sv = (q & 1) ? pc : ps;
    float cv = (q & 1) ? ps : pc;
    s = (q & 2) ? -sv : sv;
    c = ((q + 1) & 2) ? -cv : cv;
}

// Angle doubling: (sin 2a, cos 2a) from (sin a, cos a). EXACT: 2 s c and
// (c - s)(c + s); otherwise (inputs to 8- or 11-bit rounding) t = 2 s,
// t c and 1 - t s, three instructions.
template <bool EXACT = true>
__device__ __forceinline__ void dbl(float s, float c, float& s2, float& c2) {
    if constexpr (EXACT) {
        s2 = 2.0f * s * c;
        c2 = (c - s) * (c + s);
    } else {
        const float t = s + s;
        s2 = t * c;
        c2 = __builtin_fmaf(-t, s, 1.0f);
    }
}

// (sin pi a, cos pi a) for a = 2^l x. EXACT: the reduced polynomial above.
// Otherwise the hardware sine/cosine of the exactly reduced argument in
// revolutions (a/2 minus the nearest integer), accurate to about 2^-20
// absolute: used only where the result is rounded to 8 or 11 bits next.
template <bool EXACT>
__device__ __forceinline__ void sincos_oct(float x, int l, float& s, float& c) {
    if constexpr (EXACT) {
        sincospi(__builtin_ldexpf(x, l), s, c);
    } else {
        float r = __builtin_ldexpf(x, l - 1);
        r = r - __builtin_rintf(r);
        s = __builtin_amdgcn_sinf(r);
        c = __builtin_amdgcn_cosf(r);
    }
}

// x[c] for a lane-dependent c in {0, 1, 2}, branch-free and exact (the
// weights are 0 or 1).
__device__ __forceinline__ float sel3(int c, const float x[3]) {
    const float w1 = (float)(c == 1), w2 = (float)(c == 2), w0 = 1.0f - w1 - w2;
    return __builtin_fmaf(w2, x[2], __builtin_fmaf(w1, x[1], w0 * x[0]));
}

// Position encoding values of lane group g in slot order (16 values): three
// chains of octaves (exact evaluation, then angle doubling) per lane; lane
// group 3 replaces its two spare pairs by the raw components and the bias 1.
template <bool EXACT = true>
__device__ __forceinline__ void pe_position(int g, const float xh[3], float v[16]) {
    const bool g3 = (g == 3);
    float s, c;
    sincos_oct<EXACT>(sel3(g3 ? 0 : g, xh), g3 ? 8 : 0, s, c);
    v[0] = s; v[1] = c;
    dbl<EXACT>(s, c, v[2], v[3]);
    dbl<EXACT>(v[2], v[3], v[4], v[5]);
    sincos_oct<EXACT>(sel3(g3 ? 1 : g, xh), g3 ? 8 : 3, s, c);
    v[6] = s; v[7] = c;
    dbl<EXACT>(s, c, v[8], v[9]);
    dbl<EXACT>(v[8], v[9], v[10], v[11]);
    sincos_oct<EXACT>(sel3(g3 ? 2 : g, xh), g3 ? 8 : 6, s, c);
    v[12] = s; v[13] = c;
    dbl<EXACT>(s, c, v[14], v[15]);
    v[4] = g3 ? xh[0] : v[4];
    v[5] = g3 ? xh[1] : v[5];
    v[10] = g3 ? xh[2] : v[10];
    v[11] = g3 ? 1.0f : v[11];
}

// Direction encoding values of lane group g in slot order (8 values; lane
// group 3: the raw components, the bias 1 and four padding slots).
template <bool EXACT = true>
__device__ __forceinline__ void pe_direction(int g, const float d[3], float v[8]) {
    const bool g3 = (g == 3);
    float s, c;
    sincos_oct<EXACT>(sel3(g3 ? 0 : g, d), 0, s, c);
    v[0] = s; v[1] = c;
    dbl<EXACT>(v[0], v[1], v[2], v[3]);
    dbl<EXACT>(v[2], v[3], v[4], v[5]);
    dbl<EXACT>(v[4], v[5], v[6], v[7]);
    v[0] = g3 ? d[0] : v[0];
    v[1] = g3 ? d[1] : v[1];
    v[2] = g3 ? d[2] : v[2];
    v[3] = g3 ? 1.0f : v[3];
    // lane group 3's slots 4..7 are padding: their weight columns are zero
    // and their values (sines and cosines, finite) contribute exactly 0
}

// ---------------------------------------------------------------------------
// MFMA fragments. A K = 32 step is one 16x16x32 BF16/FP16 MFMA, or eight
// 16x16x4 FP32 MFMAs that use element e of every lane in the e-th
// instruction; both pair lane (16g + i, element e) of A with lane
// (16g + j, element e) of B, so one fragment layout serves all three types.
// ---------------------------------------------------------------------------
typedef __attribute__((ext_vector_type(8))) float f32x8;
template <typename T> struct FragT;
template <> struct FragT<__bf16> { typedef bf16x8 type; };
template <> struct FragT<_Float16> { typedef f16x8 type; };
template <> struct FragT<float> { typedef f32x8 type; };

template <typename T>
__device__ __forceinline__ f32x4 mma(typename FragT<T>::type a, typename FragT<T>::type b, f32x4 c) {
    if constexpr (__is_same(T, __bf16)) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    } else if constexpr (__is_same(T, _Float16)) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[e], b[e], c, 0, 0, 0);
        return c;
    }
}

typedef __attribute__((ext_vector_type(4))) unsigned u32x4;
typedef __attribute__((ext_vector_type(2))) float f32x2;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
template <typename T>
__device__ __forceinline__ typename FragT<T>::type pack8(const float* v) {
    const f32x8 x = {v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]};
    if constexpr (__is_same(T, float)) {
        return x;
    } else if constexpr (__is_same(T, __bf16)) {
        // one round-to-nearest-even pair conversion per two values
        u32x4 r;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const f32x2 pr = {v[2 * k], v[2 * k + 1]};
            r[k] = __builtin_bit_cast(unsigned, __builtin_convertvector(pr, bf16x2));
        }
        return __builtin_bit_cast(bf16x8, r);
    } else {
        return __builtin_convertvector(x, typename FragT<T>::type);
    }
}

// Two accumulator tiles as one B operand (elements 0..3 from a, 4..7 from b).
// For 16-bit types the ReLU is applied after rounding, on the bit patterns:
// a BF16/FP16 value with the sign bit set is a negative int16, so a packed
// integer max with 0 zeroes exactly the negative values (and -0).
typedef __attribute__((ext_vector_type(8))) short i16x8;
template <typename T, bool RELU>
__device__ __forceinline__ typename FragT<T>::type hand(f32x4 a, f32x4 b) {
    float v[8] = {a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
    if constexpr (__is_same(T, float)) {
        if (RELU) {
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = __builtin_fmaxf(v[e], 0.0f);
        }
        return pack8<T>(v);
    } else {
        typename FragT<T>::type r = pack8<T>(v);
        if (RELU) {
            i16x8 q = __builtin_bit_cast(i16x8, r);
            q = __builtin_elementwise_max(q, (i16x8)0);
            r = __builtin_bit_cast(typename FragT<T>::type, q);
        }
        return r;
    }
}

// ---------------------------------------------------------------------------
// Packed weights. For each layer the A operand of every MFMA is stored in
// the exact per-lane order the instruction consumes (see mlp.hip for the
// index maps). Layers in order: L1 (encoding -> h), L2 (h -> h), HEAD
// (h -> [f ; sigma], h + 16 rows), L3 ([f ; dir] -> h), L4 (h -> rgb, 16 rows).
// ---------------------------------------------------------------------------
template <int H>
struct PackGeom {
    static constexpr int NT = H / 16;                 // 16-row output tiles of a hidden layer
    // 16-bit (K = 32 per MFMA)
    static constexpr int KH16 = H / 32;               // k-steps over a hidden input
    static constexpr int F_L1 = NT * 2;
    static constexpr int F_L2 = NT * KH16;
    static constexpr int F_HD = (NT + 1) * KH16;
    static constexpr int F_L3 = NT * (KH16 + 1);
    static constexpr int F_L4 = KH16;
    static constexpr int FRAGS16 = F_L1 + F_L2 + F_HD + F_L3 + F_L4;
    static constexpr int BYTES16 = FRAGS16 * WAVE * 16;
    // biases added through the accumulator (L2, HEAD, L4): 16 floats per tile
    static constexpr int BIAS_TILES = NT + (NT + 1) + 1;
    static constexpr int BIAS_FLOATS = BIAS_TILES * 16;
    // backward: transposed A fragments (K = 32 per k-step) for the input
    // gradients: W4^T (k over the 16 padded rgb rows + 16 zero rows), W3^T
    // restricted to the feature inputs, [Wf ; ws]^T (k over the H + 16 head
    // rows, padded to whole k-steps) and W2^T
    static constexpr int KHD = (NT + 2) / 2;          // k-steps over the head's NT+1 tiles
    static constexpr int T_L4 = NT;
    static constexpr int T_L3 = NT * KH16;
    static constexpr int T_HD = NT * KHD;
    static constexpr int T_L2 = NT * KH16;
    static constexpr int FRAGS_T = T_L4 + T_L3 + T_HD + T_L2;
};

// Column of the previous layer's output that k slot (ks, e) of lane group g
// carries, for a hidden-width input. 16-bit: k-step ks covers the two 16-row
// tiles 2ks and 2ks+1; element e < 4 comes from tile 2ks, row 4g + e.
__host__ __device__ constexpr int hidden_col16(int ks, int g, int e) { return 16 * (2 * ks + (e >> 2)) + 4 * g + (e & 3); }

enum Layer { LY_L1 = 0, LY_L2, LY_HD, LY_L3, LY_L4 };

// Canonical weight (or 0) for output row `row` of layer `ly` and the input
// described either as a hidden column (col >= 0) or an encoding feature.
template <int H>
__device__ float canon_weight(const float* w, int ly, int row, bool is_enc, int feat_or_col) {
    constexpr FieldLayout L{H};
    switch (ly) {
    case LY_L1:
        if (feat_or_col == SLOT_ZERO) return 0.0f;
        return feat_or_col == SLOT_BIAS ? w[L.b1() + row] : w[L.W1() + row * DXYZ + feat_or_col];
    case LY_L2:
        return w[L.W2() + row * H + feat_or_col];
    case LY_HD:
        // the density row is repeated at H, H+4, H+8, H+12 so that every lane
        // group of the accumulator holds it (the forward pass reads it there)
        if (row < H) return w[L.Wf() + row * H + feat_or_col];
        if (((row - H) & 3) == 0) return w[L.ws() + feat_or_col];
        return 0.0f;
    case LY_L3:
        if (!is_enc) return w[L.W3() + row * (H + DDIR) + feat_or_col];
        if (feat_or_col == SLOT_ZERO) return 0.0f;
        return feat_or_col == SLOT_BIAS ? w[L.b3() + row] : w[L.W3() + row * (H + DDIR) + H + feat_or_col];
    default:   // rgb rows repeated at 4g .. 4g+2 for every lane group g
        return (row & 3) < 3 ? w[L.W4() + (row & 3) * H + feat_or_col] : 0.0f;
    }
}

// Layer, output tile and k-step of 16-bit fragment `fr`.
template <int H>
__device__ void frag16(int fr, int& ly, int& ot, int& ks, int& nks) {
    using G = PackGeom<H>;
    if (fr < G::F_L1) { ly = LY_L1; nks = 2; }
    else if ((fr -= G::F_L1) < G::F_L2) { ly = LY_L2; nks = G::KH16; }
    else if ((fr -= G::F_L2) < G::F_HD) { ly = LY_HD; nks = G::KH16; }
    else if ((fr -= G::F_HD) < G::F_L3) { ly = LY_L3; nks = G::KH16 + 1; }
    else { fr -= G::F_L3; ly = LY_L4; nks = G::KH16; }
    ot = fr / nks;
    ks = fr % nks;
}

template <int H>
__device__ float packed_source16(const float* w, int fr, int lane, int e) {
    int ly, ot, ks, nks;
    frag16<H>(fr, ly, ot, ks, nks);
    const int g = lane >> 4, row = 16 * ot + (lane & 15);
    if (ly == LY_L1) return canon_weight<H>(w, ly, row, true, pe_slot_feature(g, 8 * ks + e));
    if (ly == LY_L3 && ks == PackGeom<H>::KH16) return canon_weight<H>(w, ly, row, true, dir_slot_feature(g, e));
    return canon_weight<H>(w, ly, row, false, hidden_col16(ks, g, e));
}

}  // namespace r360

// ---------------------------------------------------------------------------
// Opaque objects
// ---------------------------------------------------------------------------
struct r360_scene {
    r360_grid_desc grid;
    r360_mlp_desc mlp;
    int64_t P;
    int16_t* labels;         // [n2][n1][n0]: field id of occupied voxels, -1 elsewhere
    void* pack16_bf;         // [F][FRAGS16][64][8] bf16
    void* pack16_h;          // [F][FRAGS16][64][8] f16
    float* bias;             // [F][BIAS_FLOATS]
    float* pack16_f;         // [F][FRAGS16][64][8] f32: the same fragment layout in FP32
    void* packT_bf;          // [F][FRAGS_T][64][8] bf16 transposed fragments (backward)
    void* packT_h;           // [F][FRAGS_T][64][8] f16
    float* packT_f;          // [F][FRAGS_T][64][8] f32
    float* frames;           // [F][4] per-field encoding frame (centre, 1 / half extent), or null
    bool use_frames;         // encode each field in its own frame
    int device;
};

struct r360_equirect {
    int32_t W, H;
    float* tables;           // device [sin_phi W | cos_phi W | sin_theta H | cos_theta H]
};

namespace r360 {

// Workspace carve-up (all offsets 256-byte aligned).
// Sample layouts. Renders and training keep the traversal's slot layout:
// sample k of ray r at slot (r - r % 64) * S + 64 k + r % 64 (S =
// max_samples), per-ray counts in ray_off[0..N) and no prefix sum; the ray
// of a slot follows from its index (ray_of_slot). The sampling entry point
// and the FP64 gradient check use the compact layout: ray r's samples at
// ray_off[r] .. ray_off[r+1] (exclusive prefix, ray_off[N] = total).
struct SlotMap {
    int smax;            // S
    uint64_t magic;      // ceil(2^40 / S): (slot / 64) / S by a multiply (exact for slot < 2^31, S <= 256)
};
inline SlotMap slot_map(int smax) { return SlotMap{smax, ((uint64_t(1) << 40) + smax - 1) / smax}; }
__device__ __forceinline__ unsigned ray_of_slot(unsigned slot, const SlotMap& m) {
    const unsigned q = slot >> 6;                                   // block * S + k
    const unsigned blk = (unsigned)(((uint64_t)q * m.magic) >> 40);
    return (blk << 6) | (slot & 63u);
}

// Element idx of an array through a 32-bit byte offset, so the load or store
// addresses as (scalar base + vector offset) instead of 64-bit vector
// arithmetic. Valid for arrays below 4 GiB: sample arrays hold fewer than
// 2^30 entries and ray arrays are passed per component.
template <typename T>
__device__ __forceinline__ T ld32(const T* base, unsigned idx) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + idx * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void st32(T* base, unsigned idx, T v) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + idx * (unsigned)sizeof(T)) = v;
}

struct Workspace {
    int32_t* ray_off;   // [N+1]   per-ray counts (slot layout) or their exclusive prefix (compact layout)
    float* o;           // [3][N]  generated rays (equirect / pinhole)
    float* d;           // [3][N]
    float* t_mid;       // [cap]
    float* delta;       // [cap]
    int32_t* ray;       // [cap]
    int32_t* field;     // [cap]
    int32_t* perm;      // [cap]   field-sorted position -> ray-major sample index
    float* sigma;       // [cap]
    float* rgb;         // [3][cap]
    float* dsigma;      // [cap]   backward
    float* drgb;        // [3][cap]
    int32_t* scan;      // scan block sums
    int32_t* hist;      // [F][ROUTE_WAVES]
    int32_t* field_start;  // [F+1]
    int32_t* chunk_start;  // [F+1]   backward: prefix of the fields' work units (128-sample chunks and field switches)
    float* dw_part;     // [DW_SLOTS][P] per-slot gradient partials
    int32_t* blk_fields;  // [DW_SLOTS] first and last field of each backward block's slice
    int32_t* misc;      // small counters
    float* loss_part;   // per-block loss partial sums
    float* ray_rgb;     // [3][N] per-ray colour (train step)
    float* ray_grad;    // [3][N] dL/dC (train step)
    const float* ro;    // rays the downstream passes read: caller's or o/d above
    const float* rd;
    int64_t N, cap;
    SlotMap slots;      // slot layout geometry (max_samples)
    size_t bytes;
};

constexpr int ROUTE_BLOCKS = 2048;        // 4 waves each
constexpr int ROUTE_WAVES = ROUTE_BLOCKS * 4;
constexpr int SCAN_TILE = 4096;           // elements per scan block (1024 threads x 4)
constexpr int DW_SLOTS = 1024;            // two gradient partial slots per backward block

// Per-sample array length: N rounded up to whole waves of 64 rays, times
// max_samples (the traversal stages sample k of ray r at slot
// (r - r % 64) * max_samples + 64 k + r % 64).
int64_t sample_cap(int64_t N, int max_samples);
// train = false leaves out what only training and early termination use
// (the gradient, partial and per-ray training arrays; those pointers are null).
Workspace carve(void* base, int64_t N, int max_samples, int F, int64_t P, bool train = true);

// launchers (return hipError_t of the launch)
enum RayMode { RAYS_GIVEN = 0, RAYS_EQUIRECT = 1, RAYS_PINHOLE = 2 };
struct RaySource {
    int mode;
    const float* o;       // RAYS_GIVEN
    const float* d;
    const float* tables;  // RAYS_EQUIRECT
    int W, H;
    float fx, fy;         // RAYS_PINHOLE
    float c2w[12];
    const int64_t* pix;   // optional pixel list (equirect)
    float eye;            // equirect: signed half eye distance (stereo), 0 for one centre
};
struct DdaParams {
    const int16_t* labels;
    int n0, n1, n2;
    float lo0, lo1, lo2;
    float voxel, inv_voxel;
    float near_, far_;
    int max_samples;
    int spv;              // samples per occupied segment (>= 1)
    int skip;             // samples 0 .. skip-1 are walked but not emitted (early termination's second pass)
};
DdaParams dda_params(const r360_scene* s, const r360_render_opts* opts);

hipError_t launch_rays(const RaySource& src, int64_t N, float* o, float* d, hipStream_t st);
// Compact layout into w.t_mid/delta/ray/field (+ voxel ids), offsets in w.ray_off.
hipError_t launch_sample(const RaySource& src, const DdaParams& p, int64_t N, const Workspace& w,
                         int32_t* voxel_out, hipStream_t st);
// Slot layout into w.t_mid/delta/field, per-ray counts in w.ray_off. For
// 1 <= F <= TRACE_COUNT_MAX_FIELDS the walk also fills the routing counts
// w.hist (*counted = true), so launch_route skips its counting pass.
constexpr int TRACE_COUNT_MAX_FIELDS = 1024;
hipError_t launch_trace(const RaySource& src, const DdaParams& p, int64_t N, const Workspace& w, int F,
                        bool* counted, hipStream_t st);
hipError_t launch_labels(const float* occ, const int32_t* fmap, float thr, int64_t nvox, int n_fields,
                         int16_t* labels, hipStream_t st);
// Routing counts per routing wave (route_waves(F) of them) in w.hist:
// computed here unless `counted` (gathered by launch_trace).
int route_waves(int F);
// The routing walk's units, one per routing wave. With at least as many
// 64-ray blocks as waves, unit w is the run of blocks [w per, (w + 1) per)
// over all their sample levels (lr = 1). With fewer blocks, every block's
// sample levels are cut into lr ranges of ls levels and unit w is range
// w % lr of block w / lr, so that small batches still spread over many
// waves. Either way the units in order visit (block, level, lane) in the
// same order, so the routing result does not depend on the cut.
struct RouteMap {
    int per, lr, ls;
};
RouteMap route_map(int64_t N, int smax, int F);
hipError_t launch_route(const Workspace& w, int F, bool counted, hipStream_t st);
hipError_t launch_repack(r360_scene* s, const float* weights, hipStream_t st);
hipError_t launch_repack_bwd(r360_scene* s, const float* weights, hipStream_t st);
hipError_t launch_mlp_forward(const r360_scene* s, const Workspace& w, int precision, hipStream_t st);
// Compositing over the compact layout with ray ids (w.ray_off offsets, w.ray) ...
hipError_t launch_composite(const Workspace& w, int64_t N, float* rgb, float* depth, float* opacity,
                            hipStream_t st);
// ... and over the slot layout (w.ray_off counts); with target [3][N] also
// the training loss's gradient grad_rgb [3][N] and its per-block partials
// (w.loss_part), summed by launch_composite_backward_slots.
hipError_t launch_composite_slots(const Workspace& w, int64_t N, float* rgb, float* depth, float* opacity,
                                  hipStream_t st, float* state = nullptr, const float* target = nullptr,
                                  float* grad_rgb = nullptr);
// Early termination: the second pass's compositing from the saved sums
// (state [6][N]), the selection of the rays that continue (list, count n2 on
// the device) and the gather of their rays ([3][n2] each).
hipError_t launch_composite_continue(const Workspace& w2, const int32_t* list, int64_t N, const float* state,
                                     float* rgb, float* depth, float* opacity, hipStream_t st);
hipError_t launch_term_select(const Workspace& w, int64_t N, int K, const float* S, float eps, int32_t* list,
                              int32_t* n2, hipStream_t st);
hipError_t launch_term_gather(int64_t n2, const int32_t* list, const float* ro, const float* rd, int64_t N, float* o2,
                              float* d2, hipStream_t st);
// crgb: the forward pass's per-ray colour [3][N], or null to recompute it;
// loss: where to finish the loss from the forward compositing's partials,
// or null.
hipError_t launch_composite_backward_slots(const Workspace& w, int64_t N, const float* grad_rgb, const float* crgb,
                                           float* loss, hipStream_t st);
hipError_t launch_loss_grad(const Workspace& w, int64_t N, const float* rgb, const float* target, float* loss,
                            float* grad_rgb, hipStream_t st);
hipError_t launch_composite_backward(const Workspace& w, int64_t N, const float* grad_rgb, hipStream_t st);
hipError_t launch_mlp_backward(const r360_scene* s, const Workspace& w, int precision, float* grad_weights,
                               hipStream_t st);
hipError_t launch_adam(float* w, const float* g, float* m, float* v, int64_t n, int64_t step, float lr,
                       float b1, float b2, float eps, hipStream_t st);
// Optional extras of the global forward: the per-ray Stage I measurement
// (depth over normalised weights, uncertainty, opacity), or the points mode
// (one sample per "ray" at t = 0, i.e. at the ray origin, whose density and
// colour are copied out and nothing is composited).
struct GlobalMeasure {
    float* depth = nullptr;
    float* uncert = nullptr;
    float* opacity = nullptr;
    bool points = false;
    float* point_sigma = nullptr;   // [M]
    float* point_rgb = nullptr;     // [3][M]
};
hipError_t launch_global_step(const r360_global_desc* desc, const float* weights, const float* o, const float* d,
                              int64_t Nr, const float* target, float* loss, float* grad, float* rgb_out,
                              float* depth_out, float* occ, void* ws, hipStream_t st, int stage_mask,
                              const GlobalMeasure* meas = nullptr);
size_t global_workspace_bytes(int w, int c, int64_t Nr, int S);
int64_t global_params(int w, int c);
// Stage I occupancy: per-ray depth statistics over dense [N][S] samples, and
// one pose's logit-grid update (workspace: occupancy_workspace_bytes).
hipError_t launch_depth_stats(const float* t, const float* delta, const float* sigma, int64_t N, int S,
                              float* depth, float* uncert, float* opacity, hipStream_t st);
size_t occupancy_workspace_bytes(int64_t nvox);
// Distillation (Eq.7): points as one-sample rays in the one-slot layout, and
// the per-field averaged squared error with its per-sample gradients.
hipError_t launch_distill_points(const Workspace& w, int64_t M, const int32_t* field, int F, hipStream_t st);
hipError_t launch_distill_loss(const Workspace& w, int64_t M, const float* tsig, const float* trgb, float* loss,
                               hipStream_t st);
// Stage II field assignment (synchronises the stream once to read the
// number of occupied voxels) and the uniform block decomposition.
size_t assign_workspace_bytes(int64_t nvox);
// Per-field encoding frames: the box of each field's voxels, and the packed
// (centre, 1 / half extent) table the field kernels read.
hipError_t launch_field_frames(const r360_grid_desc* g, const int32_t* fmap, int F, float* centers, float* halves,
                               void* ws, hipStream_t st);
hipError_t launch_pack_frames(const float* centers, const float* halves, int F, float* frames, hipStream_t st);
size_t uniform_workspace_bytes(int64_t nblocks);
hipError_t launch_assign_fields(const int32_t n[3], const float* occ, float thr, int32_t n_fields, int32_t* fmap,
                                int64_t* S_out, void* ws, hipStream_t st);
hipError_t launch_assign_uniform(const int32_t n[3], const float* occ, float thr, const int32_t b[3], int32_t* fmap,
                                 int32_t* count_out, void* ws, hipStream_t st);
hipError_t launch_occupancy_update(const r360_occ_desc* g, float* logit, float* prob, const float* o, const float* d,
                                   int64_t N, const float* depth, const float* uncert, const float* opacity,
                                   void* ws, hipStream_t st);
hipError_t launch_gradcheck_forward(const r360_scene* s, const Workspace& w, const double* w64, int64_t N,
                                    double* rgb64, hipStream_t st);
hipError_t launch_gradcheck_backward(const r360_scene* s, const Workspace& w, const double* w64, int64_t N,
                                     const double* grad_rgb64, double* grad64, hipStream_t st);

}  // namespace r360
