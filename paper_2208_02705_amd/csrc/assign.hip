// Stage II of Alg.1 (Sec. 4.2): adaptive assignment of the occupied voxels
// to n local fields, and the uniform block decomposition (the 360Roam-u
// variant of Sec. 6).
//
// Adaptive assignment. S voxels are occupied (occ > threshold); field k
// receives s_k = floor(S/n) + (k < S mod n) of them. For k = 0, 1, ...: the
// anchor is the unassigned occupied voxel of smallest linear index (the
// minimum coordinate, z then y then x) and the field takes the s_k
// unassigned voxels nearest to it (squared distance between voxel indices,
// ties to the smaller linear index). Each voxel's rank is the unique key
// (d^2 << LB) | lin (LB the bit width of the linear index; at most 57 bits
// for grids of up to 4096^3 voxels), so field k is exactly the keys up to
// the s_k-th smallest; that key is found by a radix select over 12-bit
// digits from the top (LV levels, 4 for the 128^3 and 256^3 grids), one
// histogram per level, stopping as soon as a whole bin is taken. (Wider
// digits save a level but every block clears, flushes and scans its whole
// histogram: at 14 bits those fixed costs took most of each launch.)
//
// Launches per field: one kernel that assigns the previous field, finds
// this field's anchor, writes its keys and counts their top digits, then
// one histogram kernel per further level. A level's digit is picked from
// the previous level's histogram by every block of the kernel that needs it
// (the same deterministic scan in each; block 0 stores the result for the
// kernels after it), so no launch is spent on picks. Fields alternate
// between two histogram sets: the one a field reads is cleared by the next
// field's first histogram kernel.
//
// Layout: the occupied voxels in increasing linear index (a stable
// compaction), a done byte and a key per list entry; the walk over the list
// starts at the first unassigned entry, which only moves forward.
// Every step is a deterministic function of the keys (the histogram atomics
// only count), so the field map is reproducible bit for bit.
#include "r360_internal.h"

namespace r360 {

namespace {

constexpr int CB = 4096;            // voxels per compaction block (256 threads x 16)
constexpr int DIG = 12;             // digit width of the radix select
constexpr int NBIN = 1 << DIG;      // histogram bins per level
constexpr int LVMAX = 5;            // 57-bit keys
constexpr uint64_t NOKEY = ~uint64_t(0);
// Blocks of the selection kernels (each holds a 16 KB histogram and pays its
// fixed costs): one per 1024 occupied voxels, between 64 and 256 (256 for
// the large grid, 128 for the room scene, the measured best of 64/128/256).
inline unsigned sel_grid(int64_t S) { return (unsigned)std::min<int64_t>(256, std::max<int64_t>(64, S / 1024)); }

// Radix-select state after some levels: keys <= threshold join the field
// once found; otherwise the s_k-th key lies among the keys whose top digits
// equal prefix, at rank `need` there.
struct Pick {
    uint64_t prefix;
    uint64_t threshold;
    int64_t need;
    int32_t found;
    int32_t pad;
};
struct FieldSel {
    int32_t first;        // first list entry not assigned before this field
    int32_t anchor;       // its linear index
    int32_t pad[2];
    Pick lv[LVMAX + 1];   // lv[0]: before any level; lv[l + 1]: after picking level l
};

struct AssignWs {
    int32_t* list;        // [nvox] occupied voxels, increasing linear index
    uint8_t* done;        // [nvox]
    uint64_t* key;        // [nvox]
    int32_t* bcount;      // [blocks] occupied voxels per compaction block, then their offsets
    uint32_t* hist;       // [2][LVMAX][NBIN] two histogram sets
    FieldSel* sel;        // [2]
    int32_t* total;       // S
};

size_t up256(size_t b) { return (b + 255) & ~size_t(255); }

AssignWs carve_assign(void* base, int64_t nvox) {
    AssignWs w;
    char* p = static_cast<char*>(base);
    size_t off = 0;
    auto take = [&](size_t bytes) { char* q = p + off; off += up256(bytes); return q; };
    const int64_t nb = (nvox + CB - 1) / CB;
    w.list = reinterpret_cast<int32_t*>(take(nvox * 4));
    w.done = reinterpret_cast<uint8_t*>(take(nvox));
    w.key = reinterpret_cast<uint64_t*>(take(nvox * 8));
    w.bcount = reinterpret_cast<int32_t*>(take(nb * 4));
    w.hist = reinterpret_cast<uint32_t*>(take((size_t)2 * LVMAX * NBIN * 4));
    w.sel = reinterpret_cast<FieldSel*>(take(2 * sizeof(FieldSel)));
    w.total = reinterpret_cast<int32_t*>(take(4));
    return w;
}

size_t assign_bytes(int64_t nvox) {
    const int64_t nb = (nvox + CB - 1) / CB;
    return up256(nvox * 4) + up256(nvox) + up256(nvox * 8) + up256(nb * 4) + up256((size_t)2 * LVMAX * NBIN * 4) +
           up256(2 * sizeof(FieldSel)) + up256(4);
}

// Exclusive prefix over a block of 256 threads; returns the block total.
__device__ int block_scan256(int v, int& excl) {
    __shared__ int wsum[4];
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
    for (int q = 0; q < 4; ++q) {
        before += q < wv ? wsum[q] : 0;
        tot += wsum[q];
    }
    excl = before + inc - v;
    __syncthreads();
    return tot;
}

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

__global__ __launch_bounds__(256) void k_occ_scatter(const float* __restrict__ occ, float thr, int64_t nvox,
                                                     const int32_t* __restrict__ boff, int32_t* __restrict__ list,
                                                     uint8_t* __restrict__ done) {
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
            list[pos] = (int32_t)(v0 + j);
            done[pos] = 0;
            ++pos;
        }
}

// Key geometry: LB bits of linear index under the squared distance; LV
// levels of DIG bits cover the key from the top (level l: bits
// [DIG (LV - 1 - l), DIG (LV - l))).
struct KeyGeom {
    int LB, LV;
};
__device__ __forceinline__ int lv_shift(const KeyGeom& kg, int l) { return DIG * (kg.LV - 1 - l); }

// Picks level l's digit from its histogram (every thread of the block
// returns the same state). The digit is the bin holding the need-th key;
// a bin taken whole ends the search.
__device__ Pick block_pick(Pick s, const uint32_t* __restrict__ hist, int shift) {
    __shared__ Pick res;
    if (s.found) return s;                               // uniform
    constexpr int PER = NBIN / 256;                      // bins per thread, in order, held in registers
    typedef __attribute__((ext_vector_type(4))) unsigned u32x4_;
    uint32_t hb[PER];
    const u32x4_* src = reinterpret_cast<const u32x4_*>(hist + threadIdx.x * PER);
#pragma unroll
    for (int q = 0; q < PER / 4; ++q) {
        const u32x4_ v = src[q];
        hb[4 * q] = v[0]; hb[4 * q + 1] = v[1]; hb[4 * q + 2] = v[2]; hb[4 * q + 3] = v[3];
    }
    int sum = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) sum += (int)hb[q];
    int excl;
    block_scan256(sum, excl);
    if (excl < s.need && s.need <= excl + sum) {         // exactly one thread holds the need-th key
        int64_t below = excl;
        int q = 0;
#pragma unroll
        for (int t = 0; t < PER; ++t)                    // the first bin where the count reaches need
            if (t == q && below + hb[t] < s.need) { below += hb[t]; ++q; }
        Pick r;
        r.prefix = (s.prefix << DIG) | (uint64_t)(threadIdx.x * PER + q);
        r.need = s.need - below;
        uint32_t cq = 0;
#pragma unroll
        for (int t = 0; t < PER; ++t) cq = t == q ? hb[t] : cq;
        r.found = (int64_t)cq == r.need ? 1 : 0;
        r.threshold = r.found ? ((r.prefix << shift) | ((uint64_t(1) << shift) - 1)) : 0;
        r.pad = 0;
        res = r;
    }
    __syncthreads();
    const Pick r = res;
    __syncthreads();                                     // before res is written again
    return r;
}

typedef __attribute__((ext_vector_type(4))) unsigned u32x4h;
// Zeroes a block's LDS histogram (16 bytes per store).
__device__ __forceinline__ void clear_hist(uint32_t* h) {
#pragma unroll
    for (int q = 0; q < NBIN / 1024; ++q) reinterpret_cast<u32x4h*>(h)[threadIdx.x + 256 * q] = u32x4h{0u, 0u, 0u, 0u};
}
// Adds a block's LDS histogram into a global one (16-byte LDS reads, one
// atomic per non-empty bin).
__device__ __forceinline__ void flush_hist(const uint32_t* h, uint32_t* __restrict__ dst) {
#pragma unroll
    for (int q = 0; q < NBIN / 1024; ++q) {
        const int b = 4 * (threadIdx.x + 256 * q);
        const u32x4h v = reinterpret_cast<const u32x4h*>(h)[threadIdx.x + 256 * q];
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (v[e]) atomicAdd(&dst[b + e], v[e]);
    }
}

struct StepArgs {
    const int32_t* list;
    uint8_t* done;
    uint64_t* key;
    int64_t S;
    int n0, n1;
    KeyGeom kg;
    const FieldSel* cur;        // field k (its keys and histograms are complete)
    const uint32_t* hcur;       // its histogram set
    FieldSel* nxt;              // field k + 1
    uint32_t* hnxt;
    int32_t field;              // k, or -1 before the first field
    int32_t take_all;           // field k takes every entry left
    int32_t has_next;
    int64_t s_next;             // size of field k + 1
    int32_t* fmap;
};

// Assigns field k (keys <= its threshold, or all that are left), finds the
// anchor of field k + 1 (the first entry neither assigned before nor taken
// by field k), writes field k + 1's keys and counts their top digit.
__global__ __launch_bounds__(256) void k_sel_step(StepArgs a) {
    __shared__ __attribute__((aligned(16))) uint32_t h[NBIN];
    __shared__ int hit;
    const int64_t first = a.field >= 0 ? a.cur->first : 0;
    uint64_t th = 0;
    if (a.field >= 0 && !a.take_all)
        th = block_pick(a.cur->lv[a.kg.LV - 1], a.hcur + (size_t)(a.kg.LV - 1) * NBIN, lv_shift(a.kg, a.kg.LV - 1))
                 .threshold;
    auto key_of = [&](int l, int ax, int ay, int az) {
        const int64_t dx = l % a.n0 - ax, dy = (l / a.n0) % a.n1 - ay, dz = l / (a.n0 * a.n1) - az;
        return ((uint64_t)(dx * dx + dy * dy + dz * dz) << a.kg.LB) | (uint64_t)l;
    };
    // field k's own entry (its key was written by the step before this one;
    // only this thread touches it here)
    auto taken = [&](int64_t i) { return a.field >= 0 && (a.take_all || a.key[i] <= th); };
    int64_t nfirst = a.S;
    if (a.has_next) {
        // The anchor search reads entries other blocks are assigning and
        // re-keying meanwhile: it recomputes field k's keys from its anchor
        // instead of reading them, and a done byte seen either before or
        // after another block sets it gives the same answer.
        int kx = 0, ky = 0, kz = 0;
        if (a.field >= 0) {
            const int ka = a.cur->anchor;
            kx = ka % a.n0; ky = (ka / a.n0) % a.n1; kz = ka / (a.n0 * a.n1);
        }
        auto taken_k = [&](int64_t i) {
            return a.field >= 0 && (a.take_all || key_of(a.list[i], kx, ky, kz) <= th);
        };
        for (int64_t i0 = first;; i0 += 256) {
            if (threadIdx.x == 0) hit = 256;
            __syncthreads();
            const int64_t i = i0 + threadIdx.x;
            if (i < a.S && !a.done[i] && !taken_k(i)) atomicMin(&hit, (int)threadIdx.x);
            __syncthreads();
            const int hh = hit;
            __syncthreads();
            if (hh < 256) { nfirst = i0 + hh; break; }
            if (i0 + 256 >= a.S) break;
        }
    }
    const bool next = a.has_next && nfirst < a.S;
    int ax = 0, ay = 0, az = 0;
    if (next) {
        const int an = a.list[nfirst];
        ax = an % a.n0; ay = (an / a.n0) % a.n1; az = an / (a.n0 * a.n1);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            a.nxt->first = (int32_t)nfirst;
            a.nxt->anchor = an;
            Pick p0;
            p0.prefix = 0; p0.threshold = 0; p0.need = a.s_next; p0.found = 0; p0.pad = 0;
            a.nxt->lv[0] = p0;
        }
    }
    clear_hist(h);
    __syncthreads();
    const int sh0 = lv_shift(a.kg, 0);
    for (int64_t i = first + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.S;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (a.done[i]) continue;
        if (taken(i)) {
            a.done[i] = 1;
            a.key[i] = NOKEY;
            a.fmap[a.list[i]] = a.field;
            continue;
        }
        if (!next) continue;
        const uint64_t k = key_of(a.list[i], ax, ay, az);
        a.key[i] = k;
        atomicAdd(&h[k >> sh0], 1u);
    }
    __syncthreads();
    if (next) flush_hist(h, a.hnxt);
}

// Level l >= 1 of field k's select: picks level l - 1 (block 0 stores it),
// then counts the digit of the keys inside the picked prefix. Level 1 also
// clears the other histogram set for field k + 1.
__global__ __launch_bounds__(256) void k_sel_level(FieldSel* sel, uint32_t* __restrict__ hset,
                                                   uint32_t* __restrict__ hother, const uint64_t* __restrict__ key,
                                                   int64_t S, KeyGeom kg, int level) {
    __shared__ __attribute__((aligned(16))) uint32_t h[NBIN];
    if (level == 1)
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)LVMAX * NBIN;
             i += (int64_t)gridDim.x * blockDim.x)
            hother[i] = 0;
    const Pick s = block_pick(sel->lv[level - 1], hset + (size_t)(level - 1) * NBIN, lv_shift(kg, level - 1));
    if (blockIdx.x == 0 && threadIdx.x == 0) sel->lv[level] = s;
    if (s.found) return;                                 // uniform
    clear_hist(h);
    __syncthreads();
    const int sh = lv_shift(kg, level);
    for (int64_t i = sel->first + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < S;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = key[i];
        if (k != NOKEY && (k >> (sh + DIG)) == s.prefix) atomicAdd(&h[(k >> sh) & (NBIN - 1)], 1u);
    }
    __syncthreads();
    flush_hist(h, hset + (size_t)level * NBIN);
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
    hipLaunchKernelGGL(k_occ_scatter, dim3((unsigned)nb), dim3(256), 0, st, occ, thr, nvox, w.bcount, w.list, w.done);
    hipLaunchKernelGGL(k_fill, dim3(64), dim3(256), 0, st, reinterpret_cast<int32_t*>(w.hist),
                       (int64_t)2 * LVMAX * NBIN, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int32_t S32 = 0;
    if ((e = hipMemcpyAsync(&S32, w.total, 4, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    const int64_t S = S32;
    if (S_out) *S_out = S;
    if (S == 0) return hipSuccess;
    // key geometry: bit widths of the largest linear index and squared distance
    auto bits = [](uint64_t v) { int b = 0; while (v) { ++b; v >>= 1; } return b; };
    const uint64_t d2max = (uint64_t)(n[0] - 1) * (n[0] - 1) + (uint64_t)(n[1] - 1) * (n[1] - 1) +
                           (uint64_t)(n[2] - 1) * (n[2] - 1);
    KeyGeom kg;
    kg.LB = std::max(1, bits((uint64_t)(nvox - 1)));
    kg.LV = std::max(2, (bits(d2max) + kg.LB + DIG - 1) / DIG);
    if (kg.LV > LVMAX) return hipErrorInvalidValue;
    const int64_t base = S / n_fields, rem = S % n_fields;
    auto size_of = [&](int32_t k) { return base + (k < rem ? 1 : 0); };
    StepArgs sa{};
    sa.list = w.list; sa.done = w.done; sa.key = w.key; sa.S = S; sa.n0 = n[0]; sa.n1 = n[1]; sa.kg = kg;
    sa.fmap = fmap;
    // the step before field 0 only finds its anchor and keys
    int32_t k = 0;
    while (k < n_fields && size_of(k) == 0) ++k;
    sa.field = -1; sa.take_all = 0; sa.has_next = 1; sa.s_next = size_of(k);
    sa.cur = w.sel + 1; sa.hcur = w.hist + (size_t)LVMAX * NBIN;
    sa.nxt = w.sel; sa.hnxt = w.hist;
    hipLaunchKernelGGL(k_sel_step, dim3(sel_grid(S)), dim3(256), 0, st, sa);
    int64_t left = S;
    while (k < n_fields && left > 0) {
        const int set = k & 1;
        FieldSel* sel = w.sel + set;
        uint32_t* hset = w.hist + (size_t)set * LVMAX * NBIN;
        uint32_t* hother = w.hist + (size_t)(set ^ 1) * LVMAX * NBIN;
        const int64_t sk = size_of(k);
        const int take_all = sk >= left ? 1 : 0;
        if (!take_all)
            for (int lv = 1; lv < kg.LV; ++lv)
                hipLaunchKernelGGL(k_sel_level, dim3(sel_grid(S)), dim3(256), 0, st, sel, hset, hother, w.key, S, kg, lv);
        left -= sk;
        int32_t k2 = k + 1;
        while (k2 < n_fields && size_of(k2) == 0) ++k2;
        sa.field = k; sa.take_all = take_all;
        sa.has_next = (left > 0 && k2 < n_fields) ? 1 : 0;
        sa.s_next = sa.has_next ? size_of(k2) : 0;
        sa.cur = sel; sa.hcur = hset;
        sa.nxt = w.sel + (set ^ 1); sa.hnxt = hother;
        hipLaunchKernelGGL(k_sel_step, dim3(sel_grid(S)), dim3(256), 0, st, sa);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        k = k2;
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
