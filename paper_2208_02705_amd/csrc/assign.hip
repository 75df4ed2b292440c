// Stage II of Alg.1 (Sec. 4.2): adaptive assignment of the occupied voxels
// to n local fields, and the uniform block decomposition (the 360Roam-u
// variant of Sec. 6).
//
// Adaptive assignment. S voxels are occupied (occ > threshold); field k
// receives s_k = floor(S/n) + (k < S mod n) of them. For k = 0, 1, ...: the
// anchor is the unassigned occupied voxel of smallest linear index (the
// minimum coordinate, z then y then x) and the field takes the s_k
// unassigned voxels nearest to it (squared distance between voxel indices,
// ties to the smaller linear index). Each voxel's rank is the unique 57-bit
// key (d^2 << 31) | lin, so field k is exactly the keys up to the s_k-th
// smallest; that key is found by a five-level radix select (12-bit digits
// from the top, a block-privatised histogram per level, one pick block that
// narrows the prefix and stops as soon as a whole bin is taken).
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
constexpr int HB = 4096;            // histogram bins (12-bit digits)
constexpr int LEVELS = 5;        // digits of the 57-bit key: bits 45-56, 33-44, 21-32, 9-20, 0-8
__device__ __forceinline__ int level_shift(int lv) { return lv < 4 ? 45 - 12 * lv : 0; }
__device__ __forceinline__ int level_width(int lv) { return lv < 4 ? 12 : 9; }
constexpr uint64_t NOKEY = ~uint64_t(0);

struct SelState {
    uint64_t prefix;      // top digits of the s_k-th key found so far
    uint64_t threshold;   // keys <= threshold join the field
    int64_t need;         // rank still to find inside the current prefix
    int32_t found;
    int32_t first;        // first unassigned list entry
    int32_t anchor;       // its linear index
    int32_t pad;
};

struct AssignWs {
    int32_t* list;        // [nvox] occupied voxels, increasing linear index
    uint8_t* done;        // [nvox]
    uint64_t* key;        // [nvox]
    int32_t* bcount;      // [blocks] occupied voxels per compaction block, then their offsets
    uint32_t* hist;       // [HB]
    SelState* st;
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
    w.hist = reinterpret_cast<uint32_t*>(take(HB * 4));
    w.st = reinterpret_cast<SelState*>(take(sizeof(SelState)));
    w.total = reinterpret_cast<int32_t*>(take(4));
    return w;
}

size_t assign_bytes(int64_t nvox) {
    const int64_t nb = (nvox + CB - 1) / CB;
    return up256(nvox * 4) + up256(nvox) + up256(nvox * 8) + up256(nb * 4) + up256(HB * 4) +
           up256(sizeof(SelState)) + up256(4);
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

__global__ void k_sel_init(SelState* st) {
    st->first = 0;
}

// key = (d^2 << 31) | lin for unassigned entries, NOKEY for assigned ones;
// the anchor is the first unassigned entry. Block 0 also resets the
// selection for this field (read only by the kernels launched after this
// one).
__global__ __launch_bounds__(256) void k_sel_keys(SelState* st, const int32_t* __restrict__ list,
                                                  const uint8_t* __restrict__ done, uint64_t* __restrict__ key,
                                                  int64_t S, int n0, int n1, int64_t sk) {
    const int first = st->first, a = list[first];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->anchor = a;
        st->prefix = 0;
        st->need = sk;
        st->found = 0;
        st->threshold = 0;
    }
    const int ax = a % n0, ay = (a / n0) % n1, az = a / (n0 * n1);
    for (int64_t i = first + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < S;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (done[i]) { key[i] = NOKEY; continue; }
        const int l = list[i];
        const int64_t dx = l % n0 - ax, dy = (l / n0) % n1 - ay, dz = l / (n0 * n1) - az;
        key[i] = ((uint64_t)(dx * dx + dy * dy + dz * dz) << 31) | (uint64_t)l;
    }
}

// Histogram of the level's digit over the keys inside the current prefix.
__global__ __launch_bounds__(256) void k_sel_hist(const SelState* st, const uint64_t* __restrict__ key, int64_t S,
                                                  int level, uint32_t* __restrict__ hist) {
    if (st->found) return;
    __shared__ uint32_t h[HB];
    for (int b = threadIdx.x; b < HB; b += 256) h[b] = 0;
    __syncthreads();
    const int sh = level_shift(level), wd = level_width(level);
    const uint64_t pre = st->prefix;
    const uint64_t mask = (uint64_t(1) << wd) - 1;
    for (int64_t i = st->first + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < S;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = key[i];
        if ((k >> (sh + wd)) == pre) atomicAdd(&h[(k >> sh) & mask], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < HB; b += 256)
        if (h[b]) atomicAdd(&hist[b], h[b]);
}

// One block of 256 threads: the digit whose bin holds the need-th key; the
// prefix grows by it; a bin taken whole ends the search. Clears the
// histogram for the next level.
__global__ __launch_bounds__(256) void k_sel_pick(SelState* st, uint32_t* __restrict__ hist, int level) {
    if (st->found) return;                               // uniform: every thread reads the same word
    const int t = threadIdx.x;
    constexpr int PER = HB / 256;                        // 16 bins per thread, in order
    uint32_t c[PER];
    int sum = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        c[j] = hist[t * PER + j];
        sum += (int)c[j];
    }
    int excl;
    block_scan256(sum, excl);
    const int64_t need = st->need;
    __syncthreads();                                     // every thread has read `need` before it changes
    if (excl < need && need <= excl + sum) {             // exactly one thread holds the need-th key
        int64_t below = excl;
        int j = 0;
        while (below + c[j] < need) below += c[j++];
        const int sh = level_shift(level), wd = level_width(level);
        const uint64_t pre = (st->prefix << wd) | (uint64_t)(t * PER + j);
        const int64_t left = need - below;
        st->prefix = pre;
        st->need = left;
        if ((int64_t)c[j] == left) {                    // the whole bin joins: done
            st->found = 1;
            st->threshold = (pre << sh) | ((uint64_t(1) << sh) - 1);
        }
    }
#pragma unroll
    for (int j = 0; j < PER; ++j) hist[t * PER + j] = 0;
}

__global__ __launch_bounds__(256) void k_sel_assign(const SelState* st, const int32_t* __restrict__ list,
                                                    uint8_t* __restrict__ done, const uint64_t* __restrict__ key,
                                                    int64_t S, int take_all, int32_t field, int32_t* __restrict__ fmap) {
    const uint64_t th = st->threshold;
    for (int64_t i = st->first + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < S;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (done[i]) continue;
        if (take_all || key[i] <= th) {
            done[i] = 1;
            fmap[list[i]] = field;
        }
    }
}

// Moves `first` to the next unassigned entry (one block, 256 entries a round).
__global__ __launch_bounds__(256) void k_sel_advance(SelState* st, const uint8_t* __restrict__ done, int64_t S) {
    __shared__ int hit;
    int64_t f = st->first;
    __syncthreads();
    for (;;) {
        if (threadIdx.x == 0) hit = 256;
        __syncthreads();
        const int64_t i = f + threadIdx.x;
        if (i < S && !done[i]) atomicMin(&hit, (int)threadIdx.x);
        __syncthreads();
        const int h = hit;
        if (h < 256 || f + 256 >= S) {
            if (threadIdx.x == 0) st->first = (int32_t)(h < 256 ? f + h : S);
            return;
        }
        f += 256;
        __syncthreads();
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
    hipLaunchKernelGGL(k_occ_scatter, dim3((unsigned)nb), dim3(256), 0, st, occ, thr, nvox, w.bcount, w.list, w.done);
    hipLaunchKernelGGL(k_fill, dim3(16), dim3(256), 0, st, reinterpret_cast<int32_t*>(w.hist), (int64_t)HB, 0);
    hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(1), 0, st, w.st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int32_t S32 = 0;
    if ((e = hipMemcpyAsync(&S32, w.total, 4, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    const int64_t S = S32;
    if (S_out) *S_out = S;
    if (S == 0) return hipSuccess;
    const int64_t base = S / n_fields, rem = S % n_fields;
    int64_t left = S;
    for (int32_t k = 0; k < n_fields && left > 0; ++k) {
        const int64_t sk = base + (k < rem ? 1 : 0);
        if (sk == 0) continue;
        const unsigned g = grid_for(left);
        const int take_all = sk >= left ? 1 : 0;
        if (!take_all) {
            hipLaunchKernelGGL(k_sel_keys, dim3(g), dim3(256), 0, st, w.st, w.list, w.done, w.key, S, n[0], n[1],
                               sk);
            for (int lv = 0; lv < LEVELS; ++lv) {
                hipLaunchKernelGGL(k_sel_hist, dim3(std::min(g, 512u)), dim3(256), 0, st, w.st, w.key, S, lv,
                                   w.hist);
                hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(256), 0, st, w.st, w.hist, lv);
            }
        }
        hipLaunchKernelGGL(k_sel_assign, dim3(g), dim3(256), 0, st, w.st, w.list, w.done, w.key, S, take_all, k, fmap);
        left -= sk;
        if (left > 0) hipLaunchKernelGGL(k_sel_advance, dim3(1), dim3(256), 0, st, w.st, w.done, S);
        if ((e = hipGetLastError()) != hipSuccess) return e;
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
