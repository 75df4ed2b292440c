// Backward of the per-field MLPs for fine-tuning (Sec. 4.2: all tiny
// networks are fine-tuned with an L2 photometric loss), and the FP64
// gradient-check forms.
//
// Inputs: the field-sorted samples of the preceding render (route.hip) and,
// per sample, dL/dsigma and dL/drgb from the compositing backward.
//
// Per block of 8 waves and per chunk of 128 samples of one field:
//  1. each wave recomputes the forward pass of its 16 samples on MFMA
//     (activations are recomputed, never stored in memory);
//  2. it runs the input-gradient chain dz4 -> dh3 -> dz3 -> df, dzs -> dh2 ->
//     dz2 -> dh1 -> dz1 on MFMA with transposed weight fragments, where every
//     accumulator layout feeds the next product directly (the same k-slot
//     permutation as the forward pass);
//  3. for each layer, the eight waves write their layer inputs x and output
//     gradients dz for the 128 samples into an LDS panel, transposed so that
//     samples run along k, and every wave accumulates its share of the
//     16x16 tiles of dW = dz x^T (the bias gradient rides along as a row of
//     ones in x).
// The work is cut into chunks that never straddle a field (a field of n
// samples has ceil(n / 128) of them) and shared out by cost: a chunk counts
// two units and each field a block enters one more (loading its weight
// fragments and writing its gradient cost about half a chunk), and block b
// of nb takes the chunks whose first unit lies in [b U / nb, (b + 1) U / nb)
// of the U in field order. Blocks then differ by about one chunk whatever
// the field sizes (an equal share of samples would give a block one extra,
// mostly empty chunk and a field switch per field it touches).
// The weight-gradient tiles stay in registers while the block stays on one
// field. A field that lies entirely inside one block's range is written to
// the gradient directly; the pieces of fields shared by neighbouring blocks
// go to two per-block partial slots and a reduction kernel adds them in block
// order, so the result does not depend on scheduling.
//
// Precision: BF16 or FP16 MFMA operands with FP32 accumulation, or FP32
// throughout (each K = 32 step then issues eight 16x16x4 FP32 MFMAs with the
// same k-slot layout).
#include "r360_internal.h"

namespace r360 {

namespace {

__device__ __forceinline__ float sigmoidf_(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

__device__ __forceinline__ int find_field(const int32_t* start, int F, int pos) {
    int lo = 0, hi = F;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= pos) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int xcd_block(int b, int nb) { return (b & 7) * (nb >> 3) + (b >> 3); }
constexpr int BW = 8;                           // waves per backward block
constexpr int BCH = 16 * BW;                    // samples per backward chunk
// Work units: field f (n_f samples, c_f = ceil(n_f / BCH) chunks) spans
// units [u_f, u_f + 2 c_f + 1) (none if n_f = 0); its chunk j starts at
// unit u_f + 2 j. Block b of nb owns units [b U / nb, (b + 1) U / nb), and
// with them the chunks that start there; unit u belongs to block
// ceil((u + 1) nb / U) - 1.
constexpr int UNITS_PER_CHUNK = 2;
__device__ __forceinline__ int unit_lo(int b, int U, int nb) { return (int)((int64_t)b * U / nb); }
__device__ __forceinline__ int block_of_unit(int u, int U, int nb) {
    return (int)(((int64_t)(u + 1) * nb + U - 1) / U) - 1;
}
// The chunks [*j0, *j1) of the field whose units start at uf (c chunks) that
// start inside [lo, hi).
__device__ __forceinline__ void chunks_in(int uf, int c, int lo, int hi, int* j0, int* j1) {
    const int a = max(lo, uf) - uf, e = min(hi, uf + UNITS_PER_CHUNK * c) - uf;
    *j0 = (a + UNITS_PER_CHUNK - 1) / UNITS_PER_CHUNK;
    *j1 = e > 0 ? (e + UNITS_PER_CHUNK - 1) / UNITS_PER_CHUNK : 0;
}

// unit_start[f] = sum over g < f of (n_g > 0 ? 2 ceil(n_g / BCH) + 1 : 0),
// unit_start[F] = U (n_g = start[g + 1] - start[g]); one block of 1024 threads.
__global__ __launch_bounds__(1024) void k_chunk_starts(const int32_t* __restrict__ start, int F,
                                                       int32_t* __restrict__ chunk_start) {
    __shared__ int32_t sc[1024];
    int carry = 0;
    for (int base = 0; base < F; base += 1024) {
        const int i = base + (int)threadIdx.x;
        const int n = i < F ? start[i + 1] - start[i] : 0;
        const int v = n > 0 ? UNITS_PER_CHUNK * ((n + BCH - 1) / BCH) + 1 : 0;
        sc[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {          // inclusive scan in LDS
            const int t = threadIdx.x >= (unsigned)off ? sc[threadIdx.x - off] : 0;
            __syncthreads();
            sc[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < F) chunk_start[i] = carry + sc[threadIdx.x] - v;
        carry += sc[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) chunk_start[F] = carry;
}

// ---------------------------------------------------------------------------
// Transposed fragments for the input-gradient chain. Fragment (ot, ks) of a
// transposed layer: lane l, element e holds W[k][i] with i = 16 ot + l%16
// (an input feature of the forward layer) and k = hidden_col16(ks, l/16, e)
// (an output row of the forward layer, in the accumulator hand-off order).
// ---------------------------------------------------------------------------
template <int H>
__device__ float packedT_source(const float* w, int fr, int lane, int e) {
    using G = PackGeom<H>;
    constexpr FieldLayout L{H};
    const int g = lane >> 4;
    int ly, ot, ks;
    if (fr < G::T_L4) { ly = 4; ot = fr; ks = 0; }
    else if ((fr -= G::T_L4) < G::T_L3) { ly = 3; ot = fr / G::KH16; ks = fr % G::KH16; }
    else if ((fr -= G::T_L3) < G::T_HD) { ly = 2; ot = fr / G::KHD; ks = fr % G::KHD; }
    else { fr -= G::T_HD; ly = 1; ot = fr / G::KH16; ks = fr % G::KH16; }
    const int i = 16 * ot + (lane & 15);
    const int k = hidden_col16(ks, g, e);
    switch (ly) {
    case 4: return k < 3 ? w[L.W4() + k * H + i] : 0.0f;
    case 3: return w[L.W3() + k * (H + DDIR) + i];
    case 2: return k < H ? w[L.Wf() + k * H + i] : (k == H ? w[L.ws() + i] : 0.0f);
    default: return w[L.W2() + k * H + i];
    }
}

template <int H>
__global__ __launch_bounds__(256) void k_repack_bwd(const float* __restrict__ weights, int F,
                                                    __bf16* __restrict__ tbf, _Float16* __restrict__ th,
                                                    float* __restrict__ tf) {
    using G = PackGeom<H>;
    constexpr FieldLayout L{H};
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nt = (int64_t)F * G::FRAGS_T * WAVE * 8;
    const int e = (int)(i & 7), lane = (int)((i >> 3) & 63);
    const int64_t fr_all = i >> 9;
    if (i < nt) {
        const int f = (int)(fr_all / G::FRAGS_T), fr = (int)(fr_all % G::FRAGS_T);
        const float v = packedT_source<H>(weights + (int64_t)f * L.P(), fr, lane, e);
        tbf[i] = (__bf16)v;
        th[i] = (_Float16)v;
        tf[i] = v;
    }
}

// ---------------------------------------------------------------------------
// Weight-gradient tiles: canonical parameter index of tile element
// (out row, in column) of each layer, or -1 for padding.
// ---------------------------------------------------------------------------
template <int H>
__device__ __forceinline__ int dw_index(int ly, int out, int in) {
    constexpr FieldLayout L{H};
    switch (ly) {
    case LY_L1: {
        // panel row hidden_col16(s >> 3, g, s & 7) holds slot s of lane group g
        const int feat = pe_slot_feature((in >> 2) & 3, 4 * (in >> 4) + (in & 3));
        return feat == SLOT_BIAS ? L.b1() + out : L.W1() + out * DXYZ + feat;
    }
    case LY_L2:
        return in < H ? L.W2() + out * H + in : (in == H ? L.b2() + out : -1);
    case LY_HD:
        if (out < H) return in < H ? L.Wf() + out * H + in : (in == H ? L.bf() + out : -1);
        if (out == H) return in < H ? L.ws() + in : (in == H ? L.bs() : -1);
        return -1;
    case LY_L3: {
        if (in < H) return L.W3() + out * (H + DDIR) + in;
        const int q = in - H;
        const int feat = dir_slot_feature((q >> 2) & 3, 4 * (q >> 4) + (q & 3));
        if (feat == SLOT_ZERO) return -1;
        return feat == SLOT_BIAS ? L.b3() + out : L.W3() + out * (H + DDIR) + H + feat;
    }
    default:
        if (out >= 3) return -1;
        return in < H ? L.W4() + out * H + in : (in == H ? L.b4() + out : -1);
    }
}

struct BwdArgs {
    const int32_t* field_start;
    const int32_t* chunk_start; // [F+1] prefix of the fields' work units
    const int32_t* perm;        // sorted position -> slot
    const float* t_mid;         // slot layout
    SlotMap slots;
    const float* o[3];          // per component, [N] each
    const float* d[3];
    const float* dsigma;
    const float* drgb[3];       // colour planes of [3][cap]
    int64_t N, cap;
    int F;
    int P;
    float c0, c1, c2, inv_h;
    const float* frames;         // [F][4] per-field (centre, 1 / half extent), or null: the scene's frame
    const void* pack;           // forward fragments in the K = 32 layout, element type T
    const void* packT;          // transposed fragments
    const float* bias;
    float* grad;                // [F][P]
    float* part;                // [2 * gridDim][P]
    int32_t* blk_fields;        // [2 * gridDim] first and last field of each block's slice
};

template <int H>
struct BwdGeom {
    using G = PackGeom<H>;
    static constexpr int NT = G::NT, KH = G::KH16, KHD = G::KHD;
    // weight-gradient tiles per layer (out tiles x in tiles)
    static constexpr int OT[5] = {NT, NT, NT + 1, NT, 1};
    static constexpr int IT[5] = {4, NT + 1, NT + 1, NT + 2, NT + 1};
    static constexpr int TILES(int ly) { return OT[ly] * IT[ly]; }
    static constexpr int PER_WAVE(int ly) { return (TILES(ly) + BW - 1) / BW; }
    static constexpr int ROWS = 2 * H + 32;        // largest x + dz panel (L3 / HEAD)
    static constexpr int PSTRIDE = BCH + 8;        // samples per panel row, padded
    static_assert(ROWS % 32 == 0, "panel rows in whole 32-row blocks (prow)");
};

// Panel row of logical row base16 + low (base16 a multiple of 16, low < 16):
// the two 16-row tiles of each 32-row block are interleaved (physical row
// 2 low + tile parity). A 16-byte LDS read is served 32 lanes at a time over
// 32 slots of 16 bytes; with 272-byte rows (17 slots) a fragment read's 16
// consecutive rows would put two lanes in one slot, while every other row
// (an even slot step) puts the 16 rows and two pieces in distinct slots.
__device__ __forceinline__ int prow(int base16, int low) { return (base16 & ~31) | (low << 1) | ((base16 >> 4) & 1); }

// Tiles of one layer's OT x IT weight-gradient grid (row-major) held by wave
// wv: the contiguous range [wv T / BW, (wv + 1) T / BW) (wv is wave-uniform).
__device__ __forceinline__ int tile_lo(int wv, int T) { return wv * T / BW; }

// One layer's weight-gradient stage: the panel holds x rows [0, XR) and dz
// rows [XR, XR + 16 OT) for the chunk's samples; wave wv accumulates its
// tiles one after the other. (Keeping a tile's dz fragments for the next
// tile that shares them, or running the k-steps outermost, cuts the LDS
// reads by about a third but was measured no faster: the stage waits on
// latency, not on LDS bandwidth.)
template <typename T, int NACC>
__device__ __forceinline__ void dw_stage(const T* panel, int pstride, int XR, int OT, int IT, int wv, int lane,
                                         f32x4* acc) {
    using F8 = typename FragT<T>::type;
    const int g = lane >> 4, l16 = lane & 15;
    const int t0 = tile_lo(wv, OT * IT), t1 = tile_lo(wv + 1, OT * IT);
#pragma unroll
    for (int q = 0; q < NACC; ++q) {
        const int k = t0 + q;
        __builtin_amdgcn_sched_barrier(0);
        if (k < t1) {
            const int ot = k / IT, it = k % IT;
#pragma unroll
            for (int ks = 0; ks < BCH / 32; ++ks) {
                const F8 A = *reinterpret_cast<const F8*>(panel + prow(XR + 16 * ot, l16) * pstride + 32 * ks + 8 * g);
                const F8 B = *reinterpret_cast<const F8*>(panel + prow(16 * it, l16) * pstride + 32 * ks + 8 * g);
                acc[q] = mma<T>(A, B, acc[q]);
            }
        }
    }
}

// dz *= [h > 0] on hand-off fragments, h a ReLU output as stored (zero or
// positive; in 16 bits, h > 0 exactly when its bits are not zero).
template <typename T>
__device__ __forceinline__ typename FragT<T>::type relu_mask(typename FragT<T>::type dz,
                                                            typename FragT<T>::type h) {
    if constexpr (__is_same(T, float)) {
#pragma unroll
        for (int e = 0; e < 8; ++e) dz[e] = h[e] > 0.0f ? dz[e] : 0.0f;
        return dz;
    } else {
        typedef __attribute__((ext_vector_type(8))) unsigned short u16x8;
        const u16x8 one = __builtin_elementwise_min(__builtin_bit_cast(u16x8, h), (u16x8)1);
        const u16x8 m = (u16x8)0 - one;                      // 0xffff where h > 0
        return __builtin_bit_cast(typename FragT<T>::type, __builtin_bit_cast(u16x8, dz) & m);
    }
}

template <int H, int NACC>
__device__ __forceinline__ void dw_flush(int ly, int OT, int IT, int wv, int lane, f32x4* acc, float* dst) {
    // opaque copies: the flush indices are recomputed here, once per field,
    // instead of being hoisted out of the field loop into live registers
    asm volatile("" : "+v"(lane));
    asm volatile("" : "+s"(wv));
    const int g = lane >> 4, l16 = lane & 15;
    const int t0 = tile_lo(wv, OT * IT), t1 = tile_lo(wv + 1, OT * IT);
#pragma unroll
    for (int q = 0; q < NACC; ++q) {
        const int k = t0 + q;
        if (k < t1) {
            const int ot = k / IT, it = k % IT;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int idx = dw_index<H>(ly, 16 * ot + 4 * g + r, 16 * it + l16);
                if (idx >= 0) dst[idx] = acc[q][r];
            }
        }
        acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
}

template <int H, typename T>
__global__ __launch_bounds__(64 * BW, 1) void k_bwd(BwdArgs a) {
    using BG = BwdGeom<H>;
    using G = PackGeom<H>;
    using F8 = typename FragT<T>::type;
    constexpr int NT = BG::NT, KH = BG::KH, KHD = BG::KHD, PS = BG::PSTRIDE;
    constexpr int N1 = BG::PER_WAVE(0), N2 = BG::PER_WAVE(1), NH = BG::PER_WAVE(2), N3 = BG::PER_WAVE(3),
                  N4 = BG::PER_WAVE(4);
    extern __shared__ __attribute__((aligned(32))) char smem_raw[];
    // Two panels, used by alternate stages: a stage's panel is written while
    // slower waves may still read the other one, so each stage needs a
    // single barrier (after its panel is written; every wave has finished
    // the stage before the previous one by then, which used this buffer).
    // (FP32 panels are twice as large and do not fit twice in LDS: there the
    // single panel is kept and the stage ends with a second barrier.)
    constexpr bool DB = sizeof(T) == 2;
    T* const panels = reinterpret_cast<T*>(smem_raw);
    // 16-bit types also keep the current field's forward and transposed
    // weight fragments in LDS (72 KB at H = 64, beside the two panels): every
    // layer of every chunk then reads them at LDS latency instead of going
    // back to L2. FP32 fragments are twice as large and are read from memory.
    constexpr bool WL = sizeof(T) == 2;
    F8* const wlds = reinterpret_cast<F8*>(smem_raw + (DB ? 2 : 1) * BG::ROWS * BG::PSTRIDE * sizeof(T));
    T* panel = panels;
    auto flip = [&]() {
        if constexpr (DB) panel = (panel == panels) ? panels + BG::ROWS * BG::PSTRIDE : panels;
        else __syncthreads();
    };
    const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int col = 16 * wv + j;                     // this lane's sample column in the panel
    const int nb = gridDim.x;
    const int b = xcd_block(blockIdx.x, nb);
    const int U = a.chunk_start[a.F];
    const int u_lo = unit_lo(b, U, nb), u_hi = unit_lo(b + 1, U, nb);
    // the first and last fields with a chunk that starts in this block's units
    // (a unit maps to its field like a sample index: the last field whose
    // first unit is not after it, which has units)
    auto chunks_of = [&](int f, int* j0, int* j1) {
        chunks_in(a.chunk_start[f], (a.field_start[f + 1] - a.field_start[f] + BCH - 1) / BCH, u_lo, u_hi, j0, j1);
    };
    int first = -1, last = -1;
    for (int u = u_lo; u < u_hi;) {
        const int f = find_field(a.chunk_start, a.F, u);
        int j0, j1;
        chunks_of(f, &j0, &j1);
        if (j1 > j0) { if (first < 0) first = f; last = f; }
        u = a.chunk_start[f + 1];
    }
    if (first < 0) return;
    if (threadIdx.x == 0) { a.blk_fields[2 * b] = first; a.blk_fields[2 * b + 1] = last; }
    const F8* pk = reinterpret_cast<const F8*>(a.pack);
    const F8* pt = reinterpret_cast<const F8*>(a.packT);
    f32x4 w1[N1], w2[N2], wh[NH], w3[N3], w4[N4];
    auto zero = [](f32x4* v, int n) { for (int q = 0; q < n; ++q) v[q] = f32x4{0.f, 0.f, 0.f, 0.f}; };
    zero(w1, N1); zero(w2, N2); zero(wh, NH); zero(w3, N3); zero(w4, N4);

    for (int f = first; f <= last; ++f) {
        int j0, j1;
        chunks_of(f, &j0, &j1);
        if (j1 <= j0) continue;                                   // an empty field between first and last
        const int fs0 = a.field_start[f];
        const int pos = fs0 + j0 * BCH;                             // this block's samples of field f
        const int fend = min(a.field_start[f + 1], fs0 + j1 * BCH);
        // the encoding frame of this field
        const float cc[3] = {a.frames ? a.frames[4 * f] : a.c0, a.frames ? a.frames[4 * f + 1] : a.c1,
                             a.frames ? a.frames[4 * f + 2] : a.c2};
        const float inv_h = a.frames ? a.frames[4 * f + 3] : a.inv_h;
        const F8* P = pk + (int64_t)f * G::FRAGS16 * WAVE + lane;
        const F8* PT = pt + (int64_t)f * G::FRAGS_T * WAVE + lane;
        if constexpr (WL) {
            // all of a thread's fragment loads are issued before its first LDS
            // store, so the copy waits for memory once rather than per fragment
            constexpr int NFP = G::FRAGS16 * WAVE, NFR = (G::FRAGS16 + G::FRAGS_T) * WAVE;
            constexpr int NIT = (NFR + 64 * BW - 1) / (64 * BW);
            const F8* srcP = pk + (int64_t)f * G::FRAGS16 * WAVE;
            const F8* srcT = pt + (int64_t)f * G::FRAGS_T * WAVE;
            F8 stage[NIT];
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                const int i = (int)threadIdx.x + 64 * BW * it;
                if (i < NFR) stage[it] = i < NFP ? srcP[i] : srcT[i - NFP];
            }
            __syncthreads();                      // every wave is done with the previous field's fragments
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                const int i = (int)threadIdx.x + 64 * BW * it;
                if (i < NFR) wlds[i] = stage[it];
            }
            __syncthreads();
        }
        const f32x4* bias = reinterpret_cast<const f32x4*>(a.bias + (int64_t)f * G::BIAS_FLOATS) + g;
        // Gathered inputs of this lane's sample in the current chunk; the next
        // chunk's are loaded while this chunk is processed (permutation entry
        // first, then t, then o, d and the output gradients).
        int orig;
        float xh[3], dv[3], gsig, grgb[3];
        {
            const int sp = pos + col;
            orig = ld32(a.perm, (unsigned)(sp < fend ? sp : pos));
            const unsigned u = (unsigned)orig;
            const float t = ld32(a.t_mid, u);
            const unsigned r = ray_of_slot(u, a.slots);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                dv[k] = ld32(a.d[k], r);
                xh[k] = (__builtin_fmaf(t, dv[k], ld32(a.o[k], r)) - cc[k]) * inv_h;
                grgb[k] = ld32(a.drgb[k], u);
            }
            gsig = ld32(a.dsigma, u);
        }
        for (int c = pos; c < fend; c += BCH) {
            // Keep the weight fragments out of registers across chunks: the
            // compiler would otherwise hoist all ~70 per-field fragment loads
            // out of this loop and spill. They are re-read from L1/L2 instead.
            // The scheduling barriers below likewise keep each phase's loads
            // within that phase.
            const F8* Pc;
            const F8* PTc;
            if constexpr (WL) {
                // an opaque lane offset (not an opaque pointer), so the reads
                // stay LDS reads
                int lo = lane;
                asm volatile("" : "+v"(lo));
                Pc = wlds + lo;
                PTc = wlds + G::FRAGS16 * WAVE + lo;
            } else {
                Pc = P;
                PTc = PT;
                asm volatile("" : "+v"(Pc));
                asm volatile("" : "+v"(PTc));
            }
            const bool valid = c + col < fend;
            const int cn = c + BCH;
            const int spn = cn + col;
            const int orig_n = ld32(a.perm, (unsigned)(cn < fend ? (spn < fend ? spn : cn) : c));

            __builtin_amdgcn_sched_barrier(0);
            // ---- forward recompute ----
            F8 x0, x1;
            {
                float pe[16];
                pe_position<__is_same(T, float)>(g, xh, pe);      // as the forward pass evaluates it
                x0 = pack8<T>(pe);
                x1 = pack8<T>(pe + 8);
            }
            f32x4 acc[NT + 1];
            const F8* q = Pc;
#pragma unroll
            for (int ot = 0; ot < NT; ++ot) {
                acc[ot] = f32x4{0.f, 0.f, 0.f, 0.f};
                acc[ot] = mma<T>(q[(2 * ot) * WAVE], x0, acc[ot]);
                acc[ot] = mma<T>(q[(2 * ot + 1) * WAVE], x1, acc[ot]);
            }
            __builtin_amdgcn_sched_barrier(0);
            q += G::F_L1 * WAVE;
            const unsigned un = (unsigned)orig_n;
            const float t_n = ld32(a.t_mid, un);
            const unsigned r_n = ray_of_slot(un, a.slots);
            F8 h1[KH], h2[KH], fb[KH], h3[KH];
#pragma unroll
            for (int ks = 0; ks < KH; ++ks) h1[ks] = hand<T, true>(acc[2 * ks], acc[2 * ks + 1]);
#pragma unroll
            for (int ot = 0; ot < NT; ++ot) {
                acc[ot] = bias[ot * 4];
#pragma unroll
                for (int ks = 0; ks < KH; ++ks) acc[ot] = mma<T>(q[(ot * KH + ks) * WAVE], h1[ks], acc[ot]);
            }
            __builtin_amdgcn_sched_barrier(0);
            q += G::F_L2 * WAVE;
#pragma unroll
            for (int ks = 0; ks < KH; ++ks) h2[ks] = hand<T, true>(acc[2 * ks], acc[2 * ks + 1]);
#pragma unroll
            for (int ot = 0; ot < NT + 1; ++ot) {
                acc[ot] = bias[(NT + ot) * 4];
#pragma unroll
                for (int ks = 0; ks < KH; ++ks) acc[ot] = mma<T>(q[(ot * KH + ks) * WAVE], h2[ks], acc[ot]);
            }
            __builtin_amdgcn_sched_barrier(0);
            q += G::F_HD * WAVE;
            float o_n[3], d_n[3], grgb_n[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                o_n[k] = ld32(a.o[k], r_n);
                d_n[k] = ld32(a.d[k], r_n);
                grgb_n[k] = ld32(a.drgb[k], un);
            }
            const float gsig_n = ld32(a.dsigma, un);
            const float zs = acc[NT][0];
#pragma unroll
            for (int ks = 0; ks < KH; ++ks) fb[ks] = hand<T, false>(acc[2 * ks], acc[2 * ks + 1]);
            F8 xd;
            {
                float dpe[8];
                pe_direction<__is_same(T, float)>(g, dv, dpe);
                xd = pack8<T>(dpe);
            }
#pragma unroll
            for (int ot = 0; ot < NT; ++ot) {
                acc[ot] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < KH; ++ks) acc[ot] = mma<T>(q[(ot * (KH + 1) + ks) * WAVE], fb[ks], acc[ot]);
                acc[ot] = mma<T>(q[(ot * (KH + 1) + KH) * WAVE], xd, acc[ot]);
            }
            __builtin_amdgcn_sched_barrier(0);
            q += G::F_L3 * WAVE;
#pragma unroll
            for (int ks = 0; ks < KH; ++ks) h3[ks] = hand<T, true>(acc[2 * ks], acc[2 * ks + 1]);
            f32x4 o4 = bias[(2 * NT + 1) * 4];
#pragma unroll
            for (int ks = 0; ks < KH; ++ks) o4 = mma<T>(q[ks * WAVE], h3[ks], o4);

            __builtin_amdgcn_sched_barrier(0);
            // ---- output gradients (lane group 0 holds rows 0..3 of each tile) ----
            float dzs = 0.0f;
            f32x4 dz4 = f32x4{0.f, 0.f, 0.f, 0.f};
            if (g == 0 && valid) {
                dzs = gsig * sigmoidf_(zs);                           // softplus' = sigmoid
#pragma unroll
                for (int cch = 0; cch < 3; ++cch) {
                    const float s = sigmoidf_(o4[cch]);
                    dz4[cch] = grgb[cch] * s * (1.0f - s);
                }
            }

            // Panel writers: hidden features from hand-off fragments, C-layout tiles.
            // 16-bit paths: neighbouring lanes (samples 2m, 2m + 1) swap halves of
            // each packed pair of rows (one DPP move and one byte permute), so
            // that each lane stores two samples of one row with a 4-byte store:
            // the even lane the pair's first row, the odd lane its second.
            constexpr bool SM = sizeof(T) == 2;
            const int odd = j & 1;
            const unsigned psel = odd ? 0x03020706u : 0x05040100u;
            // dword w holds rows (low, low + 1) of tile base16 for this lane's sample
            auto st2 = [&](int base16, int low, unsigned w) {
                const unsigned theirs = (unsigned)__builtin_amdgcn_mov_dpp((int)w, 0xB1, 0xF, 0xF, false);
                const unsigned out = __builtin_amdgcn_perm(theirs, w, psel);
                *reinterpret_cast<unsigned*>(panel + prow(base16, low + odd) * PS + col - odd) = out;
            };
            auto st_frag = [&](int base16_lo, int base16_hi, F8 v) {
                if constexpr (SM) {
                    const u32x4 w = __builtin_bit_cast(u32x4, v);
                    st2(base16_lo, 4 * g, w[0]);
                    st2(base16_lo, 4 * g + 2, w[1]);
                    st2(base16_hi, 4 * g, w[2]);
                    st2(base16_hi, 4 * g + 2, w[3]);
                }
            };
            auto put_hidden = [&](int row0, const F8* hb) {
#pragma unroll
                for (int ks = 0; ks < KH; ++ks) {
                    if constexpr (SM) {
                        st_frag(row0 + 32 * ks, row0 + 32 * ks + 16, hb[ks]);
                    } else {
#pragma unroll
                        for (int e = 0; e < 8; ++e) panel[prow(row0 + 16 * (2 * ks + (e >> 2)), 4 * g + (e & 3)) * PS + col] = hb[ks][e];
                    }
                }
            };
            auto put_ones = [&](int row0) {
                if constexpr (SM) {
                    // row 0 of the tile is 1 for every sample, rows 1..15 are 0
                    const unsigned one = __builtin_bit_cast(unsigned short, (T)1.0f);
#pragma unroll
                    for (int rr = 0; rr < 4; rr += 2) {
                        const unsigned v = (4 * g + rr + odd == 0) ? (one | (one << 16)) : 0u;
                        *reinterpret_cast<unsigned*>(panel + prow(row0, 4 * g + rr + odd) * PS + col - odd) = v;
                    }
                } else {
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) panel[prow(row0, 4 * g + rr) * PS + col] = (T)((4 * g + rr) == 0 ? 1.0f : 0.0f);
                }
            };
            auto put_tiles = [&](int row0, const f32x4* tl, int ntl) {
                for (int tt = 0; tt < ntl; ++tt) {
                    if constexpr (SM) {
                        const F8 v = hand<T, false>(tl[tt], f32x4{0.f, 0.f, 0.f, 0.f});
                        const u32x4 w = __builtin_bit_cast(u32x4, v);
                        st2(row0 + 16 * tt, 4 * g, w[0]);
                        st2(row0 + 16 * tt, 4 * g + 2, w[1]);
                    } else {
#pragma unroll
                        for (int rr = 0; rr < 4; ++rr) panel[prow(row0 + 16 * tt, 4 * g + rr) * PS + col] = (T)tl[tt][rr];
                    }
                }
            };
            // tiles [0, ntl) of hand-off fragments (tile 2ks + e/4, row 4g + e%4)
            auto put_frags = [&](int row0, const F8* fb_, int ntl) {
#pragma unroll
                for (int ks = 0; ks < (ntl + 1) / 2; ++ks) {
                    if constexpr (SM) {
                        const u32x4 w = __builtin_bit_cast(u32x4, fb_[ks]);
                        if (2 * ks < ntl) { st2(row0 + 32 * ks, 4 * g, w[0]); st2(row0 + 32 * ks, 4 * g + 2, w[1]); }
                        if (2 * ks + 1 < ntl) { st2(row0 + 32 * ks + 16, 4 * g, w[2]); st2(row0 + 32 * ks + 16, 4 * g + 2, w[3]); }
                    } else {
#pragma unroll
                        for (int e = 0; e < 8; ++e)
                            if (2 * ks + (e >> 2) < ntl) panel[prow(row0 + 16 * (2 * ks + (e >> 2)), 4 * g + (e & 3)) * PS + col] = fb_[ks][e];
                    }
                }
            };
            // dz in fragment form, masked by the layer input's ReLU
            auto masked = [&](F8* bz, const f32x4* dz, const F8* hb) {
#pragma unroll
                for (int ks = 0; ks < KH; ++ks) bz[ks] = relu_mask<T>(hand<T, false>(dz[2 * ks], dz[2 * ks + 1]), hb[ks]);
            };

            __builtin_amdgcn_sched_barrier(0);
            // ---- L4: dW4 and dh3 = W4^T dz4 ----
            put_hidden(0, h3);
            put_ones(H);
            put_tiles(H + 16, &dz4, 1);
            __syncthreads();
            dw_stage<T, N4>(panel, PS, H + 16, 1, NT + 1, wv, lane, w4);
            flip();
            f32x4 dz[NT + 1];
            {
                const F8 bz = hand<T, false>(dz4, f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
                for (int ot = 0; ot < NT; ++ot) dz[ot] = mma<T>(PTc[ot * WAVE], bz, f32x4{0.f, 0.f, 0.f, 0.f});
            }
            F8 bz3[KH];
            masked(bz3, dz, h3);
            __builtin_amdgcn_sched_barrier(0);
            // ---- L3: dW3 over [f ; g(d)] and df = W3_f^T dz3 ----
            put_hidden(0, fb);
            if constexpr (SM) {
                st_frag(H, H + 16, xd);
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) panel[prow(H + 16 * (e >> 2), 4 * g + (e & 3)) * PS + col] = xd[e];
            }
            put_frags(H + 32, bz3, NT);
            __syncthreads();
            dw_stage<T, N3>(panel, PS, H + 32, NT, NT + 2, wv, lane, w3);
            flip();
            f32x4 df[NT + 1];
            {
                const F8* bz = bz3;
                const F8* q3 = PTc + G::T_L4 * WAVE;
#pragma unroll
                for (int ot = 0; ot < NT; ++ot) {
                    df[ot] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int ks = 0; ks < KH; ++ks) df[ot] = mma<T>(q3[(ot * KH + ks) * WAVE], bz[ks], df[ot]);
                }
            }
            df[NT] = f32x4{dzs, 0.f, 0.f, 0.f};           // the sigma row H sits in tile NT, row 0
            __builtin_amdgcn_sched_barrier(0);
            // ---- HEAD: d[Wf ; ws] and dh2 = [Wf ; ws]^T [df ; dzs] ----
            F8 bzh[KHD];
#pragma unroll
            for (int ks = 0; ks < KHD; ++ks) {
                const f32x4 t0 = df[2 * ks];
                const f32x4 t1 = (2 * ks + 1 <= NT) ? df[(2 * ks + 1 <= NT) ? 2 * ks + 1 : 0] : f32x4{0.f, 0.f, 0.f, 0.f};
                bzh[ks] = hand<T, false>(t0, t1);
            }
            put_hidden(0, h2);
            put_ones(H);
            put_frags(H + 16, bzh, NT + 1);
            __syncthreads();
            dw_stage<T, NH>(panel, PS, H + 16, NT + 1, NT + 1, wv, lane, wh);
            flip();
            {
                const F8* qh = PTc + (G::T_L4 + G::T_L3) * WAVE;
#pragma unroll
                for (int ot = 0; ot < NT; ++ot) {
                    dz[ot] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int ks = 0; ks < KHD; ++ks) dz[ot] = mma<T>(qh[(ot * KHD + ks) * WAVE], bzh[ks], dz[ot]);
                }
            }
            F8 bz2[KH];
            masked(bz2, dz, h2);
            __builtin_amdgcn_sched_barrier(0);
            // ---- L2: dW2 and dh1 = W2^T dz2 ----
            put_hidden(0, h1);
            put_ones(H);
            put_frags(H + 16, bz2, NT);
            __syncthreads();
            dw_stage<T, N2>(panel, PS, H + 16, NT, NT + 1, wv, lane, w2);
            flip();
            {
                const F8* bz = bz2;
                const F8* q2 = PTc + (G::T_L4 + G::T_L3 + G::T_HD) * WAVE;
                f32x4 t1[NT];
#pragma unroll
                for (int ot = 0; ot < NT; ++ot) {
                    t1[ot] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int ks = 0; ks < KH; ++ks) t1[ot] = mma<T>(q2[(ot * KH + ks) * WAVE], bz[ks], t1[ot]);
                }
#pragma unroll
                for (int ot = 0; ot < NT; ++ot) dz[ot] = t1[ot];
            }
            F8 bz1[KH];
            masked(bz1, dz, h1);
            __builtin_amdgcn_sched_barrier(0);
            // ---- L1: dW1 over the encoding slots ----
            if constexpr (SM) {
                st_frag(0, 16, x0);
                st_frag(32, 48, x1);
            } else {
#pragma unroll
                for (int s2 = 0; s2 < 8; ++s2) {
                    panel[prow(16 * (s2 >> 2), 4 * g + (s2 & 3)) * PS + col] = x0[s2];
                    panel[prow(16 * (2 + (s2 >> 2)), 4 * g + (s2 & 3)) * PS + col] = x1[s2];
                }
            }
            put_frags(64, bz1, NT);
            __syncthreads();
            dw_stage<T, N1>(panel, PS, 64, NT, 4, wv, lane, w1);
            flip();
            // the next chunk's inputs
            orig = orig_n;
            gsig = gsig_n;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                dv[k] = d_n[k];
                grgb[k] = grgb_n[k];
                xh[k] = (__builtin_fmaf(t_n, d_n[k], o_n[k]) - cc[k]) * inv_h;
            }
        }
        // flush this field's tiles: every wave scatters its tiles into the
        // panel area (free now) in canonical parameter order, then the block
        // writes the field's P floats out in whole pieces
        float* dst;
        if (f == first) dst = a.part + (int64_t)(2 * b) * a.P;
        else if (f == last) dst = a.part + (int64_t)(2 * b + 1) * a.P;
        else dst = a.grad + (int64_t)f * a.P;
        constexpr int PF = FieldLayout{H}.P();
        static_assert(PF % 4 == 0, "field parameters in whole 16-byte pieces");
        static_assert(PF * sizeof(float) <= (DB ? 2 : 1) * BG::ROWS * BG::PSTRIDE * sizeof(T), "gradient fits the panels");
        float* gst = reinterpret_cast<float*>(smem_raw);
        __syncthreads();                                  // the last stage is done with the panels
        for (int i = threadIdx.x; i < PF / 4; i += 64 * BW) reinterpret_cast<f32x4*>(gst)[i] = f32x4{0.f, 0.f, 0.f, 0.f};
        __syncthreads();
        dw_flush<H, N1>(LY_L1, NT, 4, wv, lane, w1, gst);
        dw_flush<H, N2>(LY_L2, NT, NT + 1, wv, lane, w2, gst);
        dw_flush<H, NH>(LY_HD, NT + 1, NT + 1, wv, lane, wh, gst);
        dw_flush<H, N3>(LY_L3, NT, NT + 2, wv, lane, w3, gst);
        dw_flush<H, N4>(LY_L4, 1, NT + 1, wv, lane, w4, gst);
        __syncthreads();
        if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
            for (int i = threadIdx.x; i < PF / 4; i += 64 * BW)
                reinterpret_cast<f32x4*>(dst)[i] = reinterpret_cast<const f32x4*>(gst)[i];
        } else {
            for (int i = threadIdx.x; i < PF; i += 64 * BW) dst[i] = gst[i];
        }
        __syncthreads();                                  // before the panels are written again
    }
}

// Adds the partial slots of fields shared by several blocks, in block order.
// bf: the first and last field of every block's slice (written by k_bwd).
// Blocks (x, f): field f, the x-th of gridDim.x interleaved parts of its P
// parameters; the field's contributing slots are listed once per block.
// P is a multiple of 4 and every row starts on 16 bytes (16-byte loads).
constexpr int DWR_PARTS = 16;
__global__ __launch_bounds__(256) void k_dw_reduce(const float* __restrict__ part, float* __restrict__ grad,
                                                   const int32_t* __restrict__ start,
                                                   const int32_t* __restrict__ chunk_start,
                                                   const int32_t* __restrict__ bf, int F, int P, int nb) {
    __shared__ int slots[DW_SLOTS / 2];      // at most one per backward block (nb <= DW_SLOTS / 2)
    __shared__ int nslot;
    const int f = blockIdx.y;
    const int U = chunk_start[F];
    const int uf = chunk_start[f];
    const int c = (start[f + 1] - start[f] + BCH - 1) / BCH;
    const int P4 = P / 4;
    f32x4* g4 = reinterpret_cast<f32x4*>(grad + (int64_t)f * P);
    if (c == 0) {
        for (int i = blockIdx.x * 256 + threadIdx.x; i < P4; i += gridDim.x * 256) g4[i] = f32x4{0.f, 0.f, 0.f, 0.f};
        return;
    }
    const int b0 = block_of_unit(uf, U, nb), b1 = block_of_unit(uf + UNITS_PER_CHUNK * (c - 1), U, nb);
    if (b0 == b1 && f != bf[2 * b0] && f != bf[2 * b0 + 1]) return;   // written directly
    if (threadIdx.x == 0) {
        // blocks where no chunk of this field starts (with fewer units than
        // blocks, empty ones lie in between) wrote nothing for it
        int n = 0;
        for (int b = b0; b <= b1; ++b) {
            int j0, j1;
            chunks_in(uf, c, unit_lo(b, U, nb), unit_lo(b + 1, U, nb), &j0, &j1);
            if (j1 > j0) slots[n++] = (f == bf[2 * b]) ? 2 * b : 2 * b + 1;
        }
        nslot = n;
    }
    __syncthreads();
    const int n = nslot;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < P4; i += gridDim.x * 256) {
        f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int k = 0; k < n; ++k) {
            const f32x4 v = reinterpret_cast<const f32x4*>(part + (int64_t)slots[k] * P)[i];
            acc[0] += v[0]; acc[1] += v[1]; acc[2] += v[2]; acc[3] += v[3];
        }
        g4[i] = acc;
    }
}

template <typename K>
int resident(K kernel, size_t lds) {
    int dev = 0, per_cu = 0;
    (void)hipGetDevice(&dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64 * BW, lds) != hipSuccess || per_cu < 1) per_cu = 1;
    hipDeviceProp_t prop;
    int cus = 256;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
    int nb = per_cu * cus;
    nb = nb > DW_SLOTS / 2 ? DW_SLOTS / 2 : nb;
    nb &= ~7;
    return nb < 8 ? 8 : nb;
}

template <int H, typename T>
hipError_t bwd_launch(const r360_scene* s, const Workspace& w, const void* pack, const void* packT, float* grad,
                      hipStream_t st) {
    using BG = BwdGeom<H>;
    BwdArgs a;
    a.field_start = w.field_start;
    a.chunk_start = w.chunk_start;
    a.perm = w.perm;
    a.t_mid = w.t_mid;
    a.slots = w.slots;
    for (int k = 0; k < 3; ++k) {
        a.o[k] = w.ro + k * w.N; a.d[k] = w.rd + k * w.N; a.drgb[k] = w.drgb + k * w.cap;
    }
    a.dsigma = w.dsigma;
    a.N = w.N; a.cap = w.cap;
    a.F = s->mlp.n_fields;
    a.P = (int)s->P;
    a.c0 = s->mlp.center[0]; a.c1 = s->mlp.center[1]; a.c2 = s->mlp.center[2];
    a.inv_h = 1.0f / s->mlp.half_extent;
    a.frames = s->use_frames ? s->frames : nullptr;
    a.pack = pack; a.packT = packT;
    a.bias = s->bias;
    a.grad = grad;
    a.part = w.dw_part;
    a.blk_fields = w.blk_fields;
    using G = PackGeom<H>;
    const size_t lds = (size_t)(sizeof(T) == 2 ? 2 : 1) * BG::ROWS * BG::PSTRIDE * sizeof(T) +
                       (sizeof(T) == 2 ? (size_t)(G::FRAGS16 + G::FRAGS_T) * WAVE * 16 : 0);
    static int nb = 0;
    if (!nb) {
        // more than 64 KB of dynamic LDS must be allowed explicitly
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bwd<H, T>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        nb = resident(k_bwd<H, T>, lds);
    }
    hipLaunchKernelGGL(k_chunk_starts, dim3(1), dim3(1024), 0, st, w.field_start, a.F, w.chunk_start);
    hipLaunchKernelGGL((k_bwd<H, T>), dim3(nb), dim3(64 * BW), lds, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dw_reduce, dim3(DWR_PARTS, a.F), dim3(256), 0, st, w.dw_part, grad, w.field_start,
                       w.chunk_start, w.blk_fields, a.F, a.P, nb);
    return hipGetLastError();
}

template <int H>
hipError_t bwd_h(const r360_scene* s, const Workspace& w, int precision, float* grad, hipStream_t st) {
    if (precision == R360_BF16) return bwd_launch<H, __bf16>(s, w, s->pack16_bf, s->packT_bf, grad, st);
    if (precision == R360_FP16) return bwd_launch<H, _Float16>(s, w, s->pack16_h, s->packT_h, grad, st);
    return bwd_launch<H, float>(s, w, s->pack16_f, s->packT_f, grad, st);
}

template <int H>
hipError_t repack_bwd_h(r360_scene* s, const float* weights, hipStream_t st) {
    using G = PackGeom<H>;
    const int F = s->mlp.n_fields;
    const int64_t n = (int64_t)F * G::FRAGS_T * WAVE * 8;
    hipLaunchKernelGGL(k_repack_bwd<H>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, weights, F,
                       (__bf16*)s->packT_bf, (_Float16*)s->packT_h, s->packT_f);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 gradient-check forms: one block per ray, one thread per neuron,
// activations in LDS, plain FP64 arithmetic; weight gradients with FP64
// atomics. Small inputs only.
// ---------------------------------------------------------------------------
struct GcArgs {
    const int32_t* off;
    const float* t_mid;
    const float* delta;
    const int32_t* field;
    const float* o;
    const float* d;
    int64_t N;
    float c0, c1, c2, inv_h;
    const float* frames;         // [F][4] per-field (centre, 1 / half extent), or null: the scene's frame
    const double* w;
    int P;
    const double* grad_rgb;    // [3][N] (backward)
    double* out;               // forward: rgb [3][N]; backward: grad [F][P]
};

constexpr int GC_MAXS = 256;

template <int H>
struct GcNet {
    double gx[DXYZ], gd[DDIR], z1[H], h1[H], z2[H], h2[H], in3[H + DDIR], z3[H], h3[H], z4[3], zs;
    double dz4[3], dh3[H], dz3[H], din3[H + DDIR], dh2[H], dz2[H], dh1[H], dz1[H], dzs;
};

__device__ double enc_value(const double* x, int k) {
    if (k < 3) return x[k];
    const int l = (k - 3) / 6, m = (k - 3) % 6;
    const double r = ldexp(x[m % 3], l);
    return m < 3 ? sinpi(r) : cospi(r);
}

// Forward of one sample by the block's threads (tid < H active for layers).
template <int H>
__device__ void gc_forward(GcNet<H>& n, const double* w, const double xh[3], const double dd[3], int tid) {
    constexpr FieldLayout L{H};
    for (int k = tid; k < DXYZ; k += 64) n.gx[k] = enc_value(xh, k);
    for (int k = tid; k < DDIR; k += 64) n.gd[k] = enc_value(dd, k);
    __syncthreads();
    if (tid < H) {
        double acc = w[L.b1() + tid];
        for (int i = 0; i < DXYZ; ++i) acc += w[L.W1() + tid * DXYZ + i] * n.gx[i];
        n.z1[tid] = acc; n.h1[tid] = acc > 0.0 ? acc : 0.0;
    }
    __syncthreads();
    if (tid < H) {
        double acc = w[L.b2() + tid];
        for (int i = 0; i < H; ++i) acc += w[L.W2() + tid * H + i] * n.h1[i];
        n.z2[tid] = acc; n.h2[tid] = acc > 0.0 ? acc : 0.0;
    }
    __syncthreads();
    if (tid < H) {
        double acc = w[L.bf() + tid];
        for (int i = 0; i < H; ++i) acc += w[L.Wf() + tid * H + i] * n.h2[i];
        n.in3[tid] = acc;
    }
    if (tid == 0) {
        double acc = w[L.bs()];
        for (int i = 0; i < H; ++i) acc += w[L.ws() + i] * n.h2[i];
        n.zs = acc;
    }
    for (int k = tid; k < DDIR; k += 64) n.in3[H + k] = n.gd[k];
    __syncthreads();
    if (tid < H) {
        double acc = w[L.b3() + tid];
        for (int i = 0; i < H + DDIR; ++i) acc += w[L.W3() + tid * (H + DDIR) + i] * n.in3[i];
        n.z3[tid] = acc; n.h3[tid] = acc > 0.0 ? acc : 0.0;
    }
    __syncthreads();
    if (tid < 3) {
        double acc = w[L.b4() + tid];
        for (int i = 0; i < H; ++i) acc += w[L.W4() + tid * H + i] * n.h3[i];
        n.z4[tid] = acc;
    }
    __syncthreads();
}

__device__ double softplus_d(double z) { return fmax(z, 0.0) + log1p(exp(-fabs(z))); }
__device__ double sigmoid_d(double z) { return 1.0 / (1.0 + exp(-z)); }

template <int H>
__device__ void gc_inputs(const GcArgs& a, int64_t r, int j, double xh[3], double dd[3]) {
    const float t = a.t_mid[j];
    const int f = a.field[j];
    const float cc[3] = {a.frames ? a.frames[4 * f] : a.c0, a.frames ? a.frames[4 * f + 1] : a.c1,
                         a.frames ? a.frames[4 * f + 2] : a.c2};
    const float inv_h = a.frames ? a.frames[4 * f + 3] : a.inv_h;
    for (int k = 0; k < 3; ++k) {
        const float dk = a.d[k * a.N + r];
        const float p = __builtin_fmaf(t, dk, a.o[k * a.N + r]);
        xh[k] = (double)((p - cc[k]) * inv_h);
        dd[k] = (double)dk;
    }
}

template <int H>
__global__ __launch_bounds__(64) void k_gc_forward(GcArgs a) {
    __shared__ GcNet<H> n;
    __shared__ double sig[GC_MAXS], col[GC_MAXS][3];
    const int64_t r = blockIdx.x;
    const int tid = threadIdx.x;
    const int s0 = a.off[r], s1 = a.off[r + 1];
    for (int j = s0; j < s1; ++j) {
        double xh[3], dd[3];
        gc_inputs<H>(a, r, j, xh, dd);
        gc_forward<H>(n, a.w + (int64_t)a.field[j] * a.P, xh, dd, tid);
        if (tid == 0) {
            sig[j - s0] = softplus_d(n.zs);
            for (int c = 0; c < 3; ++c) col[j - s0][c] = sigmoid_d(n.z4[c]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        double C[3] = {0, 0, 0}, S = 0.0;
        for (int k = 0; k < s1 - s0; ++k) {
            const double tau = sig[k] * (double)a.delta[s0 + k];
            const double wgt = exp(-S) * (-expm1(-tau));
            for (int c = 0; c < 3; ++c) C[c] += wgt * col[k][c];
            S += tau;
        }
        for (int c = 0; c < 3; ++c) a.out[c * a.N + r] = C[c];
    }
}

template <int H>
__global__ __launch_bounds__(64) void k_gc_backward(GcArgs a) {
    constexpr FieldLayout L{H};
    __shared__ GcNet<H> n;
    __shared__ double sig[GC_MAXS], col[GC_MAXS][3], dsig[GC_MAXS], dcol[GC_MAXS][3];
    const int64_t r = blockIdx.x;
    const int tid = threadIdx.x;
    const int s0 = a.off[r], s1 = a.off[r + 1];
    for (int j = s0; j < s1; ++j) {
        double xh[3], dd[3];
        gc_inputs<H>(a, r, j, xh, dd);
        gc_forward<H>(n, a.w + (int64_t)a.field[j] * a.P, xh, dd, tid);
        if (tid == 0) {
            sig[j - s0] = softplus_d(n.zs);
            for (int c = 0; c < 3; ++c) col[j - s0][c] = sigmoid_d(n.z4[c]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        // dL/dc_i = w_i g; dL/dsigma_i = delta_i [T_{i+1} (c_i . g) - ((C - C_{<=i}) . g)]
        const double g[3] = {a.grad_rgb[r], a.grad_rgb[a.N + r], a.grad_rgb[2 * a.N + r]};
        const int n_s = s1 - s0;
        double C[3] = {0, 0, 0}, S = 0.0;
        for (int k = 0; k < n_s; ++k) {
            const double tau = sig[k] * (double)a.delta[s0 + k];
            const double wgt = exp(-S) * (-expm1(-tau));
            for (int c = 0; c < 3; ++c) C[c] += wgt * col[k][c];
            S += tau;
        }
        double Cle[3] = {0, 0, 0};
        S = 0.0;
        for (int k = 0; k < n_s; ++k) {
            const double tau = sig[k] * (double)a.delta[s0 + k];
            const double wgt = exp(-S) * (-expm1(-tau));
            S += tau;
            double cg = 0.0, rg = 0.0;
            for (int c = 0; c < 3; ++c) {
                Cle[c] += wgt * col[k][c];
                cg += col[k][c] * g[c];
                rg += (C[c] - Cle[c]) * g[c];
                dcol[k][c] = wgt * g[c];
            }
            dsig[k] = (double)a.delta[s0 + k] * (exp(-S) * cg - rg);
        }
    }
    __syncthreads();
    for (int j = s0; j < s1; ++j) {
        const int k = j - s0;
        double xh[3], dd[3];
        gc_inputs<H>(a, r, j, xh, dd);
        const double* w = a.w + (int64_t)a.field[j] * a.P;
        double* gw = a.out + (int64_t)a.field[j] * a.P;
        gc_forward<H>(n, w, xh, dd, tid);
        if (tid < 3) {
            const double s = sigmoid_d(n.z4[tid]);
            n.dz4[tid] = dcol[k][tid] * s * (1.0 - s);
        }
        if (tid == 0) n.dzs = dsig[k] * sigmoid_d(n.zs);
        __syncthreads();
        if (tid < H) {
            double acc = 0.0;
            for (int o = 0; o < 3; ++o) {
                acc += w[L.W4() + o * H + tid] * n.dz4[o];
                atomicAdd(&gw[L.W4() + o * H + tid], n.dz4[o] * n.h3[tid]);
            }
            n.dh3[tid] = acc;
            n.dz3[tid] = n.z3[tid] > 0.0 ? acc : 0.0;
        }
        if (tid < 3) atomicAdd(&gw[L.b4() + tid], n.dz4[tid]);
        __syncthreads();
        for (int i = tid; i < H + DDIR; i += 64) {
            double acc = 0.0;
            for (int o = 0; o < H; ++o) {
                acc += w[L.W3() + o * (H + DDIR) + i] * n.dz3[o];
                atomicAdd(&gw[L.W3() + o * (H + DDIR) + i], n.dz3[o] * n.in3[i]);
            }
            n.din3[i] = acc;
        }
        if (tid < H) atomicAdd(&gw[L.b3() + tid], n.dz3[tid]);
        __syncthreads();
        if (tid < H) {
            double acc = w[L.ws() + tid] * n.dzs;
            atomicAdd(&gw[L.ws() + tid], n.dzs * n.h2[tid]);
            for (int o = 0; o < H; ++o) {
                acc += w[L.Wf() + o * H + tid] * n.din3[o];
                atomicAdd(&gw[L.Wf() + o * H + tid], n.din3[o] * n.h2[tid]);
            }
            n.dh2[tid] = acc;
            n.dz2[tid] = n.z2[tid] > 0.0 ? acc : 0.0;
            atomicAdd(&gw[L.bf() + tid], n.din3[tid]);
        }
        if (tid == 0) atomicAdd(&gw[L.bs()], n.dzs);
        __syncthreads();
        if (tid < H) {
            double acc = 0.0;
            for (int o = 0; o < H; ++o) {
                acc += w[L.W2() + o * H + tid] * n.dz2[o];
                atomicAdd(&gw[L.W2() + o * H + tid], n.dz2[o] * n.h1[tid]);
            }
            n.dh1[tid] = acc;
            n.dz1[tid] = n.z1[tid] > 0.0 ? acc : 0.0;
            atomicAdd(&gw[L.b2() + tid], n.dz2[tid]);
        }
        __syncthreads();
        for (int i = tid; i < DXYZ; i += 64)
            for (int o = 0; o < H; ++o) atomicAdd(&gw[L.W1() + o * DXYZ + i], n.dz1[o] * n.gx[i]);
        if (tid < H) atomicAdd(&gw[L.b1() + tid], n.dz1[tid]);
        __syncthreads();
    }
}

__global__ void k_zero_f64(double* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

GcArgs gc_args(const r360_scene* s, const Workspace& w, const double* w64) {
    GcArgs a;
    a.off = w.ray_off;
    a.t_mid = w.t_mid;
    a.delta = w.delta;
    a.field = w.field;
    a.o = w.ro; a.d = w.rd;
    a.N = w.N;
    a.c0 = s->mlp.center[0]; a.c1 = s->mlp.center[1]; a.c2 = s->mlp.center[2];
    a.inv_h = 1.0f / s->mlp.half_extent;
    a.frames = s->use_frames ? s->frames : nullptr;
    a.w = w64;
    a.P = (int)s->P;
    a.grad_rgb = nullptr;
    a.out = nullptr;
    return a;
}

}  // namespace

hipError_t launch_repack_bwd(r360_scene* s, const float* weights, hipStream_t st) {
    return s->mlp.hidden == 32 ? repack_bwd_h<32>(s, weights, st) : repack_bwd_h<64>(s, weights, st);
}

hipError_t launch_mlp_backward(const r360_scene* s, const Workspace& w, int precision, float* grad, hipStream_t st) {
    return s->mlp.hidden == 32 ? bwd_h<32>(s, w, precision, grad, st) : bwd_h<64>(s, w, precision, grad, st);
}

hipError_t launch_gradcheck_forward(const r360_scene* s, const Workspace& w, const double* w64, int64_t N,
                                    double* rgb64, hipStream_t st) {
    GcArgs a = gc_args(s, w, w64);
    a.out = rgb64;
    if (s->mlp.hidden == 32) hipLaunchKernelGGL(k_gc_forward<32>, dim3((unsigned)N), dim3(64), 0, st, a);
    else hipLaunchKernelGGL(k_gc_forward<64>, dim3((unsigned)N), dim3(64), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_gradcheck_backward(const r360_scene* s, const Workspace& w, const double* w64, int64_t N,
                                     const double* grad_rgb64, double* grad64, hipStream_t st) {
    GcArgs a = gc_args(s, w, w64);
    a.grad_rgb = grad_rgb64;
    a.out = grad64;
    const int64_t n = (int64_t)s->mlp.n_fields * s->P;
    hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, grad64, n);
    if (s->mlp.hidden == 32) hipLaunchKernelGGL(k_gc_backward<32>, dim3((unsigned)N), dim3(64), 0, st, a);
    else hipLaunchKernelGGL(k_gc_backward<64>, dim3((unsigned)N), dim3(64), 0, st, a);
    return hipGetLastError();
}

}  // namespace r360
