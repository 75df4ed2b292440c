// Stage II of Alg.1 (Sec. 4.2): adaptive assignment of the occupied voxels
// to n local fields, and the uniform block decomposition (the 360Roam-u
// variant of Sec. 6).
//
// Adaptive assignment. S voxels are occupied (occ > threshold); field k
// receives s_k = floor(S/n) + (k < S mod n) of them. For k = 0, 1, ...: the
// anchor is the unassigned occupied voxel of smallest linear index (the
// minimum coordinate, z then y then x) and the field takes the s_k
// unassigned voxels nearest to it (squared distance d^2 between voxel
// indices, ties to the smaller linear index).
//
// Selection. The occupied voxels are listed in increasing linear index, so
// among voxels at one distance the list order is the tie order. Field k is
// therefore every unassigned entry with d^2 < D, plus the first r entries
// in list order with d^2 = D, where D is the d^2 of its s_k-th nearest
// voxel. D is found by a radix select over the digits of d^2 alone (d^2 <
// 2^26 for grids up to 4096^3): one or two histogram levels of up to 12
// bits from the top (one for grids up to 256^3), then a final digit of up
// to 6 bits whose counts are kept per block, each block counting one
// contiguous chunk of the list. With those counts the block holding the
// r-th tie and the rank inside its chunk follow from a prefix over the
// blocks; each block also keeps the list position of its first tie per
// value, so only a tie that is not the first of its chunk needs a scan of
// that chunk for the position of the last entry taken. A level whose picked
// bin is taken whole ends the search.
//
// Launches per field: one step kernel that settles the previous field's
// threshold (final pick and tie position), assigns it, finds this field's
// anchor, writes this field's d^2 and counts its top digit; then one kernel
// per further digit (the last one keeps per-block counts). A level's digit
// is picked from the previous level's histogram by every block of the
// kernel that needs it (the same deterministic scan in each; block 0 stores
// the result for the kernels after it). Fields alternate between two sets
// of histograms and d^2 arrays: the step kernel settles field k from one
// while it writes field k + 1's into the other, and the first digit kernel
// of field k + 1 clears field k's histograms.
//
// Layout: the list of occupied voxels and two d^2 arrays per entry (SENT
// marks an entry assigned before the field), padded to whole groups of 16
// entries; the passes take units of 4 consecutive entries per thread
// (16-byte loads and stores), the chunk scan whole groups. The walk over
// the list starts at the first unassigned entry, which only moves forward.
// Every step is a deterministic function of the occupancy (the histogram
// atomics only count), so the field map is reproducible bit for bit.
#include "r360_internal.h"

namespace r360 {

namespace {

constexpr int CB = 4096;            // voxels per compaction block (256 threads x 16)
constexpr int DIG = 12;             // widest histogram digit
constexpr int NBIN = 1 << DIG;      // histogram bins per level
constexpr int HLMAX = 2;            // histogram levels (d^2 < 2^26: at most 20 bits above the final digit)
constexpr int FW = 6;               // widest final digit
constexpr int NFIN = 1 << FW;       // its values
constexpr int ST = 1024;            // threads per block of the selection kernels
constexpr int GMAX = 64;            // their blocks, at most
constexpr int TP = 1;               // first ties per block and value whose list positions are kept
constexpr uint32_t SENT = 0xFFFFFFFFu;   // d^2 of an entry outside the field's candidates
// One histogram set: level 0 in NCOPY copies (block b adds into copy b mod
// NCOPY, so that the blocks' flushes meet at fewer addresses; the pick adds
// the copies), the further levels, then the final digit's totals. Two
// copies halve the contention of the flush atomics for one more 16 KB read
// per pick; three, four or eight cost more than they save.
constexpr int NCOPY = 2;
constexpr int HSET = (NCOPY + HLMAX - 1) * NBIN + NFIN;
constexpr int HTOT = (NCOPY + HLMAX - 1) * NBIN;
__host__ __device__ constexpr int lv_off(int l) { return l == 0 ? 0 : (NCOPY + l - 1) * NBIN; }
__host__ __device__ constexpr int lv_copies(int l) { return l == 0 ? NCOPY : 1; }
// Blocks of the selection kernels: one per 2 K occupied voxels, at most
// 64. Few, wide blocks: each block adds its histogram into the global one
// with one atomic per non-empty bin, so the block count sets how many
// atomics meet at each bin.
inline unsigned sel_grid(int64_t S) {
    return (unsigned)std::min<int64_t>(GMAX, std::max<int64_t>(1, (S + 2047) / 2048));
}

// Digits of d^2 from the top: nh histogram levels (level l: w[l] bits at
// shift sh[l]), then the final digit of wf bits at shift 0.
struct Geom {
    int nh, wf;
    int w[HLMAX], sh[HLMAX];
};

// Radix-select state after some levels: if found, the field is the entries
// with d^2 <= dlim; otherwise its s_k-th entry has d^2 >> (shift after the
// level) = prefix, at rank `need` among those.
struct Pick {
    uint32_t prefix;
    uint32_t dlim;
    int64_t need;
    int32_t found;
    int32_t pad;
};
struct FieldSel {
    int32_t first;        // first list entry not assigned before this field
    int32_t anchor;       // its linear index
    int32_t pad[2];
    Pick lv[HLMAX + 1];   // lv[0]: before any level; lv[l + 1]: after picking level l
};

struct AssignWs {
    int32_t* list;        // [nvox16] occupied voxels, increasing linear index (packed coordinates where they fit)
    uint32_t* d2[2];      // [nvox16] d^2 to the anchor of the fields using each set, SENT for entries assigned before
    int32_t* bcount;      // [blocks] occupied voxels per compaction block, then their offsets
    uint32_t* hist;       // [2][HSET] two histogram sets
    uint32_t* cnt;        // [NFIN][GMAX] final-digit counts per block
    int32_t* tpos;        // [NFIN][GMAX] list position of each block's first tie per value (-1 none)
    int32_t* agt;         // [GMAX] each block's first entry whose d^2 lies above the picked prefix (INT_MAX none)
    FieldSel* sel;        // [2]
    int32_t* total;       // S
};

size_t up256(size_t b) { return (b + 255) & ~size_t(255); }

AssignWs carve_assign(void* base, int64_t nvox) {
    AssignWs w;
    char* p = static_cast<char*>(base);
    size_t off = 0;
    auto take = [&](size_t bytes) { char* q = p + off; off += up256(bytes); return q; };
    const int64_t nb = (nvox + CB - 1) / CB, n16 = (nvox + 15) & ~int64_t(15);
    w.list = reinterpret_cast<int32_t*>(take(n16 * 4));
    w.d2[0] = reinterpret_cast<uint32_t*>(take(n16 * 4));
    w.d2[1] = reinterpret_cast<uint32_t*>(take(n16 * 4));
    w.bcount = reinterpret_cast<int32_t*>(take(nb * 4));
    w.hist = reinterpret_cast<uint32_t*>(take((size_t)2 * HSET * 4));
    w.cnt = reinterpret_cast<uint32_t*>(take((size_t)NFIN * GMAX * 4));
    w.tpos = reinterpret_cast<int32_t*>(take((size_t)NFIN * GMAX * TP * 4));
    w.agt = reinterpret_cast<int32_t*>(take((size_t)GMAX * 4));
    w.sel = reinterpret_cast<FieldSel*>(take(2 * sizeof(FieldSel)));
    w.total = reinterpret_cast<int32_t*>(take(4));
    return w;
}

size_t assign_bytes(int64_t nvox) {
    const int64_t nb = (nvox + CB - 1) / CB, n16 = (nvox + 15) & ~int64_t(15);
    return up256(n16 * 4) + 2 * up256(n16 * 4) + up256(nb * 4) + up256((size_t)2 * HSET * 4) +
           up256((size_t)NFIN * GMAX * 4) + up256((size_t)NFIN * GMAX * TP * 4) + up256((size_t)GMAX * 4) +
           up256(2 * sizeof(FieldSel)) + up256(4);
}

// Exclusive prefix over a block of NT threads; returns the block total.
template <int NT>
__device__ int block_scan(int v, int& excl) {
    __shared__ int wsum[NT / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int inc = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int u = __shfl_up(inc, off, 64);
        if (lane >= off) inc += u;
    }
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();
    int before = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < NT / 64; ++q) {
        before += q < wv ? wsum[q] : 0;
        tot += wsum[q];
    }
    excl = before + inc - v;
    __syncthreads();
    return tot;
}
__device__ __forceinline__ int block_scan256(int v, int& excl) { return block_scan<256>(v, excl); }

__global__ __launch_bounds__(256) void k_fill(int32_t* __restrict__ p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Occupied voxels per compaction block (16 consecutive voxels per thread).
__global__ __launch_bounds__(256) void k_occ_count(const float* __restrict__ occ, float thr, int64_t nvox,
                                                   int32_t* __restrict__ bcount) {
    const int64_t v0 = (int64_t)blockIdx.x * CB + threadIdx.x * 16;
    int c = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) c += (v0 + j < nvox && occ[v0 + j] > thr) ? 1 : 0;
    int excl;
    const int tot = block_scan256(c, excl);
    if (threadIdx.x == 0) bcount[blockIdx.x] = tot;
}

// Exclusive offsets of the blocks (one block walks them in chunks of 256);
// total = S.
__global__ __launch_bounds__(256) void k_block_offsets(int32_t* __restrict__ bcount, int64_t nb,
                                                       int32_t* __restrict__ total) {
    int carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += 256) {
        const int64_t b = b0 + threadIdx.x;
        const int v = b < nb ? bcount[b] : 0;
        int excl;
        const int tot = block_scan256(v, excl);
        if (b < nb) bcount[b] = carry + excl;
        carry += tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

// List entries: the voxel's coordinates packed as x | y << 11 | z << 22
// when the grid is at most 2048 x 2048 x 1024 (the same order as the
// linear index, and unpacked with three bit-field extracts), else its
// linear index.
template <bool PACKED>
__global__ __launch_bounds__(256) void k_occ_scatter(const float* __restrict__ occ, float thr, int64_t nvox,
                                                     int n0, int n1, const int32_t* __restrict__ boff,
                                                     int32_t* __restrict__ list) {
    const int64_t v0 = (int64_t)blockIdx.x * CB + threadIdx.x * 16;
    uint32_t bits = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) bits |= (v0 + j < nvox && occ[v0 + j] > thr) ? (1u << j) : 0u;
    int excl;
    block_scan256(__builtin_popcount(bits), excl);
    int pos = boff[blockIdx.x] + excl;
#pragma unroll
    for (int j = 0; j < 16; ++j)
        if (bits & (1u << j)) {
            const int64_t v = v0 + j;
            if constexpr (PACKED) {
                const int64_t q = v / n0;
                list[pos++] = (int32_t)((uint32_t)(v - q * n0) | (uint32_t)(q % n1) << 11 | (uint32_t)(q / n1) << 22);
            } else {
                list[pos++] = (int32_t)v;
            }
        }
}

typedef __attribute__((ext_vector_type(4))) unsigned u32x4h;
typedef __attribute__((ext_vector_type(4))) int i32x4h;

typedef __attribute__((ext_vector_type(4))) int i32x4h;
__device__ __forceinline__ void load_d2(const uint32_t* __restrict__ d2, int64_t g, uint32_t (&d)[16]) {
    const u32x4h* p = reinterpret_cast<const u32x4h*>(d2 + 16 * g);
    u32x4h v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = p[q];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) d[4 * q + e] = v[q][e];
}

// Exact unsigned division of n < 2^31 by 2 <= d <= 4096 as one high
// multiply: with l = ceil(log2 d) and m = ceil(2^(31+l) / d) < 2^32,
// floor(n / d) = floor(n m / 2^(31+l)) (the excess m d - 2^(31+l) is below
// d <= 2^l, so n times it stays below 2^(31+l)). For d = 1 the multiplier
// is 0 and the numerator passes through a mask, so there is no branch.
struct Divisor {
    uint32_t m, d, one;   // one: all ones for d = 1, else 0
    int sh;               // l - 1 (0 for d = 1)
};
inline Divisor make_divisor(uint32_t d) {
    int l = 0;
    while ((1u << l) < d) ++l;
    if (d == 1) return Divisor{0u, 1u, ~0u, 0};
    return Divisor{(uint32_t)(((uint64_t(1) << (31 + l)) + d - 1) / d), d, 0u, l - 1};
}
__device__ __forceinline__ uint32_t div_by(uint32_t n, const Divisor& v) {
    return (__umulhi(n, v.m) >> v.sh) + (n & v.one);
}

// Voxel coordinates of a linear index and squared distances between them.
struct Vox {
    int x, y, z;
};
__device__ __forceinline__ Vox vox_of(uint32_t lin, const Divisor& n0, const Divisor& n1) {
    const uint32_t q = div_by(lin, n0), z = div_by(q, n1);
    return Vox{(int)(lin - q * n0.d), (int)(q - z * n1.d), (int)z};
}
// A list entry's coordinates and linear index.
template <bool PACKED>
__device__ __forceinline__ Vox entry_vox(uint32_t w, const Divisor& n0, const Divisor& n1) {
    if constexpr (PACKED) return Vox{(int)(w & 2047u), (int)((w >> 11) & 2047u), (int)(w >> 22)};
    else return vox_of(w, n0, n1);
}
template <bool PACKED>
__device__ __forceinline__ uint32_t entry_lin(uint32_t w, const Divisor& n0, const Divisor& n1) {
    if constexpr (PACKED) return (w & 2047u) + n0.d * (((w >> 11) & 2047u) + n1.d * (w >> 22));
    else return w;
}
__device__ __forceinline__ uint32_t dist2(const Vox& a, const Vox& b) {
    const int dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;    // |d| < 2^12: 24-bit products are exact
    return (uint32_t)(__mul24(dx, dx) + __mul24(dy, dy) + __mul24(dz, dz));
}

// Picks level l's digit (w bits, at shift sh) from its histogram; every
// thread of the block returns the same state. The digit is the bin holding
// the need-th entry; a bin taken whole ends the search.
__device__ Pick block_pick(Pick s, const uint32_t* __restrict__ hist, int ncopy, int w, int sh) {
    __shared__ Pick res;
    if (s.found) return s;                               // uniform
    constexpr int PER = NBIN / ST;                       // bins per thread, in order, held in registers
    uint32_t hb[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) hb[q] = 0;
    for (int c = 0; c < ncopy; ++c) {                    // the copies' sums
        const u32x4h* src = reinterpret_cast<const u32x4h*>(hist + (size_t)c * NBIN + threadIdx.x * PER);
#pragma unroll
        for (int q = 0; q < PER / 4; ++q) {
            const u32x4h v = src[q];
            hb[4 * q] += v[0]; hb[4 * q + 1] += v[1]; hb[4 * q + 2] += v[2]; hb[4 * q + 3] += v[3];
        }
    }
    int sum = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) sum += (int)hb[q];
    int excl;
    block_scan<ST>(sum, excl);
    if (excl < s.need && s.need <= excl + sum) {         // exactly one thread holds the need-th entry
        int64_t below = excl;
        int q = 0;
#pragma unroll
        for (int t = 0; t < PER; ++t)                    // the first bin where the count reaches need
            if (t == q && below + hb[t] < s.need) { below += hb[t]; ++q; }
        Pick r;
        r.prefix = (s.prefix << w) | (uint32_t)(threadIdx.x * PER + q);
        r.need = s.need - below;
        uint32_t cq = 0;
#pragma unroll
        for (int t = 0; t < PER; ++t) cq = t == q ? hb[t] : cq;
        r.found = (int64_t)cq == r.need ? 1 : 0;
        r.dlim = r.found ? (((r.prefix + 1u) << sh) - 1u) : 0u;
        r.pad = 0;
        res = r;
    }
    __syncthreads();
    const Pick r = res;
    __syncthreads();                                     // before res is written again
    return r;
}

// Zeroes a block's LDS histogram (16 bytes per store).
__device__ __forceinline__ void clear_hist(uint32_t* h) {
#pragma unroll
    for (int q = 0; q < NBIN / (4 * ST); ++q) reinterpret_cast<u32x4h*>(h)[threadIdx.x + ST * q] = u32x4h{0u, 0u, 0u, 0u};
}
// Adds the first nbin bins of a block's LDS histogram into a global one
// (16-byte LDS reads, one atomic per non-empty bin).
__device__ __forceinline__ void flush_hist(const uint32_t* h, uint32_t* __restrict__ dst, int nbin) {
    for (int c = threadIdx.x; 4 * c < nbin; c += ST) {
        const u32x4h v = reinterpret_cast<const u32x4h*>(h)[c];
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (v[e]) atomicAdd(&dst[4 * c + e], v[e]);
    }
}

// The contiguous chunk of groups that block b counts in the final digit:
// groups [first / 16, ceil(S / 16)) cut into G equal chunks.
__device__ __forceinline__ void chunk_of(int64_t first, int64_t S, int G, int b, int64_t& cb, int64_t& ce) {
    const int64_t g0 = first >> 4, gend = (S + 15) >> 4, cg = (gend - g0 + G - 1) / G;
    cb = g0 + (int64_t)b * cg;
    cb = cb < gend ? cb : gend;
    ce = cb + cg < gend ? cb + cg : gend;
}

struct StepArgs {
    const int32_t* list;
    const uint32_t* d2cur;      // field k's d^2
    uint32_t* d2nxt;            // field k + 1's, written here
    int64_t S;
    Divisor n0, n1;
    Geom g;
    const FieldSel* cur;        // field k (its digit kernels are complete)
    const uint32_t* hcur;       // its histogram set
    const uint32_t* cnt;        // its final-digit counts per block
    const int32_t* tpos;        // and the positions of each block's first ties
    const int32_t* agt;         // and each block's first entry above the picked prefix
    FieldSel* nxt;              // field k + 1
    uint32_t* hnxt;
    int32_t field;              // k, or -1 before the first field
    int32_t take_all;           // field k takes every entry left
    int32_t has_next;
    int32_t G;                  // blocks of the selection kernels (this grid)
    int64_t s_next;             // size of field k + 1
    int32_t* fmap;
};

// Inclusive prefix over a wave.
__device__ __forceinline__ int wave_scan(int x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    return x;
}

// Settles field k's threshold: entries with d^2 < dlim, or d^2 = dlim at
// list positions up to pos, belong to it. The totals of the final digit
// and the whole matrix of per-block counts are loaded at once; the first
// wave then finds the value of d^2 and the rank r among its ties, and the
// block whose chunk holds the r-th tie with the rank there; one scan of
// that chunk gives its position.
// Its inputs (the state after the histogram levels, this thread's 16 bytes
// of the per-block counts, and for the first wave one total each) are
// loaded by the caller before anything else.
struct SettleIn {
    Pick s;
    u32x4h cv;
    int tv;
    i32x4h tp;
    int32_t ag;
};
__device__ __forceinline__ SettleIn settle_load(const StepArgs& a) {
    static_assert(NFIN * GMAX == 4 * ST, "one 16-byte load of counts per thread");
    SettleIn in;
    in.s = a.cur->lv[a.g.nh];
    in.cv = reinterpret_cast<const u32x4h*>(a.cnt)[threadIdx.x];
    in.tv = threadIdx.x < (1u << a.g.wf) ? (int)a.hcur[HTOT + threadIdx.x] : 0;
    static_assert(NFIN * GMAX * TP == 4 * ST, "one 16-byte load of tie positions per thread");
    in.tp = reinterpret_cast<const i32x4h*>(a.tpos)[threadIdx.x];
    in.ag = threadIdx.x < (unsigned)a.G ? a.agt[threadIdx.x] : 0x7fffffff;
    return in;
}
// Also the anchor of field k + 1 when it follows from the same counts
// (anchor = -1 otherwise): the first entry that field k leaves is the first
// one above the picked prefix, or the first with a larger final digit, or
// the first tie after the cut. When the cut took every tie of its chunk, the
// last is the first tie of a later chunk; otherwise it is unknown, but lies
// after the cut, so the smallest of the others stands when it lies before.
__device__ void settle(const StepArgs& a, const SettleIn& in, int64_t first, uint32_t& dlim, int64_t& pos,
                       int64_t& anchor) {
    __shared__ __attribute__((aligned(16))) uint32_t s_cnt[NFIN * GMAX];
    __shared__ __attribute__((aligned(16))) int32_t s_tp[NFIN * GMAX * TP];
    __shared__ int s_v, s_whole, s_b, s_direct;
    __shared__ int64_t s_need, s_pos, s_anchor;
    __shared__ int s_known;
    const Pick s = in.s;
    const int tv = in.tv;
    anchor = -1;
    if (s.found) { dlim = s.dlim; pos = INT64_MAX; return; }     // uniform
    const u32x4h cv = in.cv;
    reinterpret_cast<u32x4h*>(s_cnt)[threadIdx.x] = cv;
    reinterpret_cast<i32x4h*>(s_tp)[threadIdx.x] = in.tp;
    __syncthreads();
    if (threadIdx.x < 64) {
        const int t = threadIdx.x;
        const int inc = wave_scan(tv);
        const int64_t ex = inc - tv;
        const uint64_t m = __ballot(ex < s.need && s.need <= inc);
        const int v = m ? __ffsll((unsigned long long)m) - 1 : 0;
        const int64_t need = s.need - __shfl((int)ex, v, 64);
        const int whole = need == __shfl(tv, v, 64) ? 1 : 0;
        int b = 0;
        int64_t r = need;
        int direct = 0;
        int64_t p = first;
        if (!whole) {
            const int c = t < a.G ? (int)s_cnt[v * GMAX + t] : 0;
            const int inc2 = wave_scan(c);
            const int64_t ex2 = inc2 - c;
            const uint64_t m2 = __ballot(c > 0 && ex2 < need && need <= inc2);
            b = m2 ? __ffsll((unsigned long long)m2) - 1 : 0;
            r = need - __shfl((int)ex2, b, 64);
            // the chunk's first tie: its position was kept
            if (r >= 1 && r <= TP) {
                const int32_t q = s_tp[(v * GMAX + b) * TP + (int)r - 1];
                if (q >= 0) { direct = 1; p = q; }
            }
        }
        // the next field's anchor (lane t: block t)
        auto wave_min = [](int32_t x) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) x = min(x, __shfl_xor(x, off, 64));
            return x;
        };
        int32_t cand = in.ag;                                   // above the prefix
        if (t < a.G) {
            for (int u = v + 1; u < (1 << a.g.wf); ++u) {      // larger final digit
                const int32_t q = s_tp[u * GMAX + t];
                if (q >= 0) cand = min(cand, q);
            }
        }
        bool known = true;
        if (!whole) {
            const int cb = __shfl(t < a.G ? (int)s_cnt[v * GMAX + t] : 0, b, 64);
            if (r < cb) known = false;                          // another tie of the chunk follows the cut
            else if (t > b && t < a.G) {                        // ties in later chunks
                const int32_t q = s_tp[v * GMAX + t];
                if (q >= 0) cand = min(cand, q);
            }
        }
        cand = wave_min(cand);
        if (t == 0) {
            s_v = v; s_whole = whole; s_b = b; s_need = r; s_pos = p; s_direct = direct;
            s_anchor = cand == 0x7fffffff ? (int64_t)a.S : (int64_t)cand;
            s_known = known ? 1 : 0;
        }
    }
    __syncthreads();
    dlim = (s.prefix << a.g.wf) | (uint32_t)s_v;
    const int64_t other = s_anchor;
    const bool known = s_known;
    anchor = known ? other : -1;
    if (s_whole) { pos = INT64_MAX; return; }                  // uniform
    if (s_direct) {                                            // uniform
        pos = s_pos;
        if (!known && other < pos) anchor = other;
        return;
    }
    int64_t r = s_need;
    int64_t cb, ce;
    chunk_of(first, a.S, a.G, s_b, cb, ce);
    for (int64_t g0 = cb; g0 < ce; g0 += ST) {
        const int64_t g = g0 + threadIdx.x;
        uint32_t d[16];
        int m = 0;
        if (g < ce) {
            load_d2(a.d2cur, g, d);
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int64_t i = 16 * g + e;
                m += (i >= first && i < a.S && d[e] == dlim) ? 1 : 0;
            }
        }
        int ex;
        const int total = block_scan<ST>(m, ex);
        if (m > 0 && ex < r && r <= ex + m) {
            int64_t left = r - ex;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int64_t i = 16 * g + e;
                if (i >= first && i < a.S && d[e] == dlim && --left == 0) s_pos = i;
            }
        }
        __syncthreads();
        if (r <= total) break;                                  // uniform
        r -= total;
    }
    pos = s_pos;
    if (!known && other < pos) anchor = other;
}

// Assigns field k (entries under its threshold, or all that are left),
// finds the anchor of field k + 1 (the first entry neither assigned before
// nor taken by field k), writes field k + 1's d^2 and counts its top digit.
// Field k's own d^2 tells both: SENT marks an entry assigned before, and
// field k takes d^2 < dlim, or d^2 = dlim up to list position pos. Work goes
// in units of 4 entries per thread (one 16-byte load of d^2, one of linear
// indices), PB units per batch; the main pass's first batch is issued
// before the threshold is settled. One unit per batch is fastest (2, 3 and
// 4 hold more registers and were slower), and the anchor search, which
// most fields skip, loads its rounds itself.
template <bool PACKED>
__global__ __launch_bounds__(ST) void k_sel_step(StepArgs a) {
    constexpr int PB = 1;                          // units per batch
    __shared__ __attribute__((aligned(16))) uint32_t h[NBIN];
    __shared__ int hit;
    const bool prev = a.field >= 0;
    const int64_t first = prev ? a.cur->first : 0;
    const int64_t ubeg = (first >> 4) << 2, uend = (a.S + 3) >> 2;
    const int64_t um = ubeg + (int64_t)blockIdx.x * ST + threadIdx.x, ustride = (int64_t)gridDim.x * ST;
    auto ld_d2 = [&](int64_t u) {
        return prev ? *reinterpret_cast<const u32x4h*>(a.d2cur + 4 * u) : u32x4h{0u, 0u, 0u, 0u};
    };
    auto ld_lin = [&](int64_t u) { return *reinterpret_cast<const i32x4h*>(a.list + 4 * u); };
    // loads in the order they are needed (the wait counter completes in
    // issue order): the threshold's inputs, then the first batch of the
    // main pass
    const bool need_settle = prev && !a.take_all;
    SettleIn sin;
    if (need_settle) sin = settle_load(a);
    u32x4h md[PB], ad[PB];
    i32x4h ml[PB];
#pragma unroll
    for (int p = 0; p < PB; ++p) {
        const int64_t u = um + p * ustride;
        if (u < uend) { md[p] = ld_d2(u); ml[p] = ld_lin(u); }
    }
    uint32_t dlim = 0;
    int64_t pos = -1, known_anchor = -1;
    if (prev) {
        if (a.take_all) { dlim = SENT; pos = INT64_MAX; }
        else settle(a, sin, first, dlim, pos, known_anchor);
    }
    // an entry is a candidate of field k + 1 when it is one of field k's
    // candidates (or any entry before the first field) that field k leaves
    auto left_for_next = [&](uint32_t dk, int64_t i) {
        if (i < first || i >= a.S) return false;
        if (!prev) return true;
        return dk != SENT && !(dk < dlim || (dk == dlim && i <= pos));
    };
    // The anchor search: rounds of PB ST units (4 PB consecutive entries per
    // thread); field k's d^2 is read-only here.
    static_assert(4 * PB <= 32, "one live bit per entry of a thread's round");
    int64_t nfirst = a.S;
    if (a.has_next && known_anchor >= 0) nfirst = known_anchor;  // uniform
    else if (a.has_next) {
        for (int r = 0; ubeg + (int64_t)PB * ST * r < uend; ++r) {
            const int64_t u0 = ubeg + (int64_t)PB * ST * r + PB * threadIdx.x;
#pragma unroll
            for (int p = 0; p < PB; ++p)
                if (u0 + p < uend) ad[p] = ld_d2(u0 + p);
            if (threadIdx.x == 0) hit = 0x7fffffff;
            __syncthreads();
            uint32_t live = 0;
#pragma unroll
            for (int p = 0; p < PB; ++p)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    live |= (uint32_t)(u0 + p < uend && left_for_next(ad[p][e], 4 * (u0 + p) + e)) << (4 * p + e);
            // one atomic per wave: its first lane with a live entry holds the
            // wave's smallest one
            const uint64_t bm = __ballot(live != 0);
            if (bm && (int)(threadIdx.x & 63) == __ffsll((unsigned long long)bm) - 1)
                atomicMin(&hit, 4 * PB * (int)threadIdx.x + __builtin_ctz(live));
            __syncthreads();
            const int hh = hit;
            __syncthreads();
            if (hh != 0x7fffffff) { nfirst = 4 * (ubeg + (int64_t)PB * ST * r) + hh; break; }
        }
    }
    const bool next = a.has_next && nfirst < a.S;
    Vox na{0, 0, 0};
    if (next) {
        const uint32_t an = (uint32_t)a.list[nfirst];
        na = entry_vox<PACKED>(an, a.n0, a.n1);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            a.nxt->first = (int32_t)nfirst;
            a.nxt->anchor = (int32_t)entry_lin<PACKED>(an, a.n0, a.n1);
            Pick p0;
            p0.prefix = 0; p0.dlim = 0; p0.need = a.s_next; p0.found = 0; p0.pad = 0;
            a.nxt->lv[0] = p0;
        }
    }
    clear_hist(h);
    __syncthreads();
    const int sh0 = a.g.sh[0];
    for (int64_t ub = um; ub < uend; ub += PB * ustride) {
        if (ub != um) {
#pragma unroll
            for (int p = 0; p < PB; ++p) {
                const int64_t u = ub + p * ustride;
                if (u < uend) { md[p] = ld_d2(u); ml[p] = ld_lin(u); }
            }
        }
#pragma unroll
        for (int p = 0; p < PB; ++p) {
            const int64_t u = ub + p * ustride;
            if (u >= uend) break;
            // straight-line over the unit, then the stores and counts
            uint32_t d[4];
            uint32_t lv = 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t i = 4 * u + e;
                const uint32_t dk = md[p][e];
                const bool in = i >= first && i < a.S && (!prev || dk != SENT);
                const bool l = left_for_next(dk, i) && next;
                lv |= (uint32_t)l << e;
                d[e] = l ? dist2(entry_vox<PACKED>((uint32_t)ml[p][e], a.n0, a.n1), na) : SENT;
                if (in && prev && !left_for_next(dk, i)) a.fmap[entry_lin<PACKED>((uint32_t)ml[p][e], a.n0, a.n1)] = a.field;
            }
            // neighbouring entries often share a bin: one LDS add per run
            uint32_t rb = 0, rn = 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (!((lv >> e) & 1u)) continue;
                const uint32_t bn = d[e] >> sh0;
                if (rn && bn != rb) { atomicAdd(&h[rb], rn); rn = 0; }
                rb = bn;
                ++rn;
            }
            if (rn) atomicAdd(&h[rb], rn);
            if (next) *reinterpret_cast<u32x4h*>(a.d2nxt + 4 * u) = u32x4h{d[0], d[1], d[2], d[3]};
        }
    }
    __syncthreads();
    if (next) flush_hist(h, a.hnxt + (size_t)(blockIdx.x % NCOPY) * NBIN, 1 << a.g.w[0]);
}

// Histogram level l >= 1 of field k's select: picks level l - 1 (block 0
// stores it), then counts level l's digit of the entries inside the picked
// prefix. The first digit kernel of a field also clears the other set for
// field k + 1.
__global__ __launch_bounds__(ST) void k_sel_level(FieldSel* sel, uint32_t* __restrict__ hset,
                                                   uint32_t* __restrict__ hother, const uint32_t* __restrict__ d2,
                                                   int64_t S, Geom g, int level) {
    __shared__ __attribute__((aligned(16))) uint32_t h[NBIN];
    if (level == 1)
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < HSET; i += (int64_t)gridDim.x * blockDim.x)
            hother[i] = 0;
    const Pick s = block_pick(sel->lv[level - 1], hset + lv_off(level - 1), lv_copies(level - 1), g.w[level - 1],
                              g.sh[level - 1]);
    if (blockIdx.x == 0 && threadIdx.x == 0) sel->lv[level] = s;
    if (s.found) return;                                 // uniform
    clear_hist(h);
    __syncthreads();
    const int sh = g.sh[level], top = sh + g.w[level];
    const uint32_t mask = (1u << g.w[level]) - 1u;
    const int64_t first = sel->first;
    for (int64_t q = (first >> 4) + (int64_t)blockIdx.x * ST + threadIdx.x; 16 * q < S; q += (int64_t)gridDim.x * ST) {
        uint32_t d[16];
        load_d2(d2, q, d);
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int64_t i = 16 * q + e;
            if (i >= first && i < S && d[e] != SENT && (d[e] >> top) == s.prefix) atomicAdd(&h[(d[e] >> sh) & mask], 1u);
        }
    }
    __syncthreads();
    flush_hist(h, hset + lv_off(level), 1 << g.w[level]);
}

// The final digit of field k's select: picks the last histogram level
// (block 0 stores it), then each block counts the final digit of the
// entries inside the picked prefix over its own chunk of the list, storing
// the counts per block and adding them into the totals. Clears the other
// set when it is the field's first digit kernel.
__global__ __launch_bounds__(ST) void k_sel_final(FieldSel* sel, uint32_t* __restrict__ hset,
                                                   uint32_t* __restrict__ hother, const uint32_t* __restrict__ d2,
                                                   uint32_t* __restrict__ cnt, int32_t* __restrict__ tpos,
                                                   int32_t* __restrict__ agt, int64_t S, Geom g) {
    __shared__ uint32_t c[NFIN];
    __shared__ int32_t tf[NFIN];
    __shared__ int32_t above;
    const int64_t first = sel->first;
    int64_t cb, ce;
    chunk_of(first, S, gridDim.x, blockIdx.x, cb, ce);
    const int64_t ub = 4 * cb, ue = 4 * ce;              // units of 4 entries
    u32x4h d = u32x4h{SENT, SENT, SENT, SENT};           // this thread's first unit, loaded before the pick
    if (ub + threadIdx.x < ue) d = *reinterpret_cast<const u32x4h*>(d2 + 4 * (ub + threadIdx.x));
    if (g.nh == 1)
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < HSET; i += (int64_t)gridDim.x * blockDim.x)
            hother[i] = 0;
    const int L = g.nh - 1;
    const Pick s = block_pick(sel->lv[L], hset + lv_off(L), lv_copies(L), g.w[L], g.sh[L]);
    if (blockIdx.x == 0 && threadIdx.x == 0) sel->lv[g.nh] = s;
    if (s.found) return;                                 // uniform
    if (threadIdx.x < NFIN) { c[threadIdx.x] = 0; tf[threadIdx.x] = 0x7fffffff; }
    if (threadIdx.x == 0) above = 0x7fffffff;
    __syncthreads();
    int32_t ab = 0x7fffffff;                                // this thread's first entry above the prefix
    const int wf = g.wf;
    const uint32_t mask = (1u << wf) - 1u;
    for (int64_t u = ub + threadIdx.x; u < ue; u += ST) {
        if (u != ub + threadIdx.x) d = *reinterpret_cast<const u32x4h*>(d2 + 4 * u);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t i = 4 * u + e;
            if (i >= first && i < S && d[e] != SENT && (d[e] >> wf) == s.prefix) {
                atomicAdd(&c[d[e] & mask], 1u);
                atomicMin(&tf[d[e] & mask], (int32_t)i);    // the chunk's first tie of this value
            }
            if (i >= first && i < S && d[e] != SENT && (d[e] >> wf) > s.prefix) ab = min(ab, (int32_t)i);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ab = min(ab, __shfl_xor(ab, off, 64));
    if ((threadIdx.x & 63) == 0 && ab != 0x7fffffff) atomicMin(&above, ab);
    __syncthreads();
    if (threadIdx.x == 0) agt[blockIdx.x] = above;
    if (threadIdx.x < (1 << wf)) {
        const uint32_t v = c[threadIdx.x];
        cnt[threadIdx.x * GMAX + blockIdx.x] = v;
        if (v) atomicAdd(&hset[HTOT + threadIdx.x], v);
        tpos[threadIdx.x * GMAX + blockIdx.x] = v ? tf[threadIdx.x] : -1;
    }
}

// ---- uniform blocks ----------------------------------------------------------
struct UniArgs {
    const float* occ;
    float thr;
    int n0, n1, n2, b0, b1, b2;
    int64_t nvox;
    int32_t* flag;     // [nb] 1 where a block holds an occupied voxel, then its field id or -1
    int32_t* fmap;
    int32_t* total;
};

__device__ __forceinline__ int block_of(const UniArgs& a, int64_t v) {
    const int x = (int)(v % a.n0), y = (int)((v / a.n0) % a.n1), z = (int)(v / ((int64_t)a.n0 * a.n1));
    const int bx = (int)((int64_t)x * a.b0 / a.n0), by = (int)((int64_t)y * a.b1 / a.n1);
    const int bz = (int)((int64_t)z * a.b2 / a.n2);
    return bx + a.b0 * (by + a.b1 * bz);
}

__global__ __launch_bounds__(256) void k_uni_mark(UniArgs a) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < a.nvox; v += (int64_t)gridDim.x * blockDim.x)
        if (a.occ[v] > a.thr) a.flag[block_of(a, v)] = 1;
}

__global__ __launch_bounds__(256) void k_uni_number(UniArgs a, int64_t nb) {
    int carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += 256) {
        const int64_t b = b0 + threadIdx.x;
        const int f = b < nb ? a.flag[b] : 0;
        int excl;
        const int tot = block_scan256(f, excl);
        if (b < nb) a.flag[b] = f ? carry + excl : -1;
        carry += tot;
    }
    if (threadIdx.x == 0) *a.total = carry;
}

__global__ __launch_bounds__(256) void k_uni_label(UniArgs a) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < a.nvox; v += (int64_t)gridDim.x * blockDim.x)
        a.fmap[v] = a.occ[v] > a.thr ? a.flag[block_of(a, v)] : -1;
}

// ---- per-field encoding frames ----------------------------------------------
// Box of the voxels labelled f: per axis the extreme voxel indices (atomic
// min / max, order-independent), box_lo = fma(imin, voxel, lo), box_hi =
// fma(imax + 1, voxel, lo), centre (box_lo + box_hi) * 0.5, half extent the
// largest (box_hi - box_lo) * 0.5 over the axes; a field without voxels gets
// centre 0 and half extent 1.
__global__ __launch_bounds__(256) void k_ff_init(int32_t* __restrict__ mm, int F) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 6 * F) mm[i] = i < 3 * F ? 0x7fffffff : -1;
}

__global__ __launch_bounds__(256) void k_ff_scan(const int32_t* __restrict__ fmap, int n0, int n1, int64_t nvox, int F,
                                                 int32_t* __restrict__ mm) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nvox; v += (int64_t)gridDim.x * blockDim.x) {
        const int f = fmap[v];
        if (f < 0 || f >= F) continue;
        const int idx[3] = {(int)(v % n0), (int)((v / n0) % n1), (int)(v / ((int64_t)n0 * n1))};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            atomicMin(mm + 3 * f + a, idx[a]);
            atomicMax(mm + 3 * F + 3 * f + a, idx[a]);
        }
    }
}

__global__ __launch_bounds__(256) void k_ff_final(const int32_t* __restrict__ mm, int F, float lo0, float lo1, float lo2,
                                                  float voxel, float* __restrict__ centers, float* __restrict__ halves) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    if (mm[3 * F + 3 * f] < 0) {
        centers[3 * f] = centers[3 * f + 1] = centers[3 * f + 2] = 0.0f;
        halves[f] = 1.0f;
        return;
    }
    const float lo[3] = {lo0, lo1, lo2};
    float h = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float blo = __builtin_fmaf((float)mm[3 * f + a], voxel, lo[a]);
        const float bhi = __builtin_fmaf((float)(mm[3 * F + 3 * f + a] + 1), voxel, lo[a]);
        centers[3 * f + a] = (blo + bhi) * 0.5f;
        const float ha = (bhi - blo) * 0.5f;
        h = h < ha ? ha : h;
    }
    halves[f] = h;
}

__global__ __launch_bounds__(256) void k_pack_frames(const float* __restrict__ centers, const float* __restrict__ halves,
                                                     int F, float* __restrict__ frames) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    frames[4 * f] = centers[3 * f];
    frames[4 * f + 1] = centers[3 * f + 1];
    frames[4 * f + 2] = centers[3 * f + 2];
    frames[4 * f + 3] = 1.0f / halves[f];
}

unsigned grid_for(int64_t n, int64_t cap = 2048) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, cap));
}

}  // namespace

size_t assign_workspace_bytes(int64_t nvox) { return assign_bytes(nvox); }
size_t uniform_workspace_bytes(int64_t nblocks) { return up256(nblocks * 4) + up256(4); }

hipError_t launch_assign_fields(const int32_t n[3], const float* occ, float thr, int32_t n_fields, int32_t* fmap,
                                int64_t* S_out, void* ws, hipStream_t st) {
    const int64_t nvox = (int64_t)n[0] * n[1] * n[2];
    const int64_t nb = (nvox + CB - 1) / CB;
    AssignWs w = carve_assign(ws, nvox);
    hipLaunchKernelGGL(k_fill, dim3(grid_for(nvox)), dim3(256), 0, st, fmap, nvox, -1);
    hipLaunchKernelGGL(k_occ_count, dim3((unsigned)nb), dim3(256), 0, st, occ, thr, nvox, w.bcount);
    hipLaunchKernelGGL(k_block_offsets, dim3(1), dim3(256), 0, st, w.bcount, nb, w.total);
    const bool packed = n[0] <= 2048 && n[1] <= 2048 && n[2] <= 1024;
    if (packed)
        hipLaunchKernelGGL(k_occ_scatter<true>, dim3((unsigned)nb), dim3(256), 0, st, occ, thr, nvox, n[0], n[1], w.bcount, w.list);
    else
        hipLaunchKernelGGL(k_occ_scatter<false>, dim3((unsigned)nb), dim3(256), 0, st, occ, thr, nvox, n[0], n[1], w.bcount, w.list);
    hipLaunchKernelGGL(k_fill, dim3(64), dim3(256), 0, st, reinterpret_cast<int32_t*>(w.hist), (int64_t)2 * HSET, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int32_t S32 = 0;
    if ((e = hipMemcpyAsync(&S32, w.total, 4, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    const int64_t S = S32;
    if (S_out) *S_out = S;
    if (S == 0) return hipSuccess;
    // digits of d^2: bit width of the largest squared distance in the grid
    auto bits = [](uint64_t v) { int b = 0; while (v) { ++b; v >>= 1; } return b; };
    const uint64_t d2max = (uint64_t)(n[0] - 1) * (n[0] - 1) + (uint64_t)(n[1] - 1) * (n[1] - 1) +
                           (uint64_t)(n[2] - 1) * (n[2] - 1);
    const int dbits = std::max(1, bits(d2max));
    Geom g{};
    g.wf = std::min(FW, dbits - 1);
    const int rest = dbits - g.wf;
    g.nh = (rest + DIG - 1) / DIG;
    if (g.nh > HLMAX || dbits > 31) return hipErrorInvalidValue;
    for (int l = 0; l < g.nh; ++l) g.w[l] = l == 0 ? rest - DIG * (g.nh - 1) : DIG;
    for (int l = 0, top = dbits; l < g.nh; ++l) { top -= g.w[l]; g.sh[l] = top; }
    const int G = (int)sel_grid(S);
    auto launch_step = [&](const StepArgs& sa) {
        if (packed) hipLaunchKernelGGL(k_sel_step<true>, dim3(G), dim3(ST), 0, st, sa);
        else hipLaunchKernelGGL(k_sel_step<false>, dim3(G), dim3(ST), 0, st, sa);
    };
    const int64_t base = S / n_fields, rem = S % n_fields;
    auto size_of = [&](int32_t k) { return base + (k < rem ? 1 : 0); };
    StepArgs sa{};
    sa.list = w.list; sa.S = S; sa.g = g;
    sa.n0 = make_divisor((uint32_t)n[0]); sa.n1 = make_divisor((uint32_t)n[1]);
    sa.cnt = w.cnt; sa.tpos = w.tpos; sa.agt = w.agt; sa.G = G; sa.fmap = fmap;
    // the step before field 0 only finds its anchor and d^2 (set 0)
    int32_t k = 0;
    while (k < n_fields && size_of(k) == 0) ++k;
    sa.field = -1; sa.take_all = 0; sa.has_next = 1; sa.s_next = size_of(k);
    sa.cur = w.sel + 1; sa.hcur = w.hist + HSET; sa.d2cur = w.d2[1];
    sa.nxt = w.sel; sa.hnxt = w.hist; sa.d2nxt = w.d2[0];
    launch_step(sa);
    int64_t left = S;
    int set = 0;
    while (k < n_fields && left > 0) {
        FieldSel* sel = w.sel + set;
        uint32_t* hset = w.hist + (size_t)set * HSET;
        uint32_t* hother = w.hist + (size_t)(set ^ 1) * HSET;
        const int64_t sk = size_of(k);
        const int take_all = sk >= left ? 1 : 0;
        if (!take_all) {
            for (int lv = 1; lv < g.nh; ++lv)
                hipLaunchKernelGGL(k_sel_level, dim3(G), dim3(ST), 0, st, sel, hset, hother, w.d2[set], S, g, lv);
            hipLaunchKernelGGL(k_sel_final, dim3(G), dim3(ST), 0, st, sel, hset, hother, w.d2[set], w.cnt, w.tpos, w.agt, S,
                               g);
        }
        left -= sk;
        int32_t k2 = k + 1;
        while (k2 < n_fields && size_of(k2) == 0) ++k2;
        sa.field = k; sa.take_all = take_all;
        sa.has_next = (left > 0 && k2 < n_fields) ? 1 : 0;
        sa.s_next = sa.has_next ? size_of(k2) : 0;
        sa.cur = sel; sa.hcur = hset; sa.d2cur = w.d2[set];
        sa.nxt = w.sel + (set ^ 1); sa.hnxt = hother; sa.d2nxt = w.d2[set ^ 1];
        launch_step(sa);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        k = k2;
        set ^= 1;
    }
    return hipSuccess;
}

hipError_t launch_field_frames(const r360_grid_desc* g, const int32_t* fmap, int F, float* centers, float* halves,
                               void* ws, hipStream_t st) {
    int32_t* mm = static_cast<int32_t*>(ws);
    const int64_t nvox = (int64_t)g->n[0] * g->n[1] * g->n[2];
    hipLaunchKernelGGL(k_ff_init, dim3((6 * F + 255) / 256), dim3(256), 0, st, mm, F);
    hipLaunchKernelGGL(k_ff_scan, dim3(grid_for(nvox)), dim3(256), 0, st, fmap, g->n[0], g->n[1], nvox, F, mm);
    hipLaunchKernelGGL(k_ff_final, dim3((F + 255) / 256), dim3(256), 0, st, mm, F, g->lo[0], g->lo[1], g->lo[2], g->voxel,
                       centers, halves);
    return hipGetLastError();
}

hipError_t launch_pack_frames(const float* centers, const float* halves, int F, float* frames, hipStream_t st) {
    hipLaunchKernelGGL(k_pack_frames, dim3((F + 255) / 256), dim3(256), 0, st, centers, halves, F, frames);
    return hipGetLastError();
}

hipError_t launch_assign_uniform(const int32_t n[3], const float* occ, float thr, const int32_t b[3], int32_t* fmap,
                                 int32_t* count_out, void* ws, hipStream_t st) {
    UniArgs a;
    a.occ = occ; a.thr = thr;
    a.n0 = n[0]; a.n1 = n[1]; a.n2 = n[2];
    a.b0 = b[0]; a.b1 = b[1]; a.b2 = b[2];
    a.nvox = (int64_t)n[0] * n[1] * n[2];
    const int64_t nb = (int64_t)b[0] * b[1] * b[2];
    a.flag = static_cast<int32_t*>(ws);
    a.total = reinterpret_cast<int32_t*>(static_cast<char*>(ws) + up256(nb * 4));
    a.fmap = fmap;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(nb)), dim3(256), 0, st, a.flag, nb, 0);
    hipLaunchKernelGGL(k_uni_mark, dim3(grid_for(a.nvox)), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_uni_number, dim3(1), dim3(256), 0, st, a, nb);
    hipLaunchKernelGGL(k_uni_label, dim3(grid_for(a.nvox)), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int32_t c = 0;
    if ((e = hipMemcpyAsync(&c, a.total, 4, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    if (count_out) *count_out = c;
    return hipSuccess;
}

}  // namespace r360
