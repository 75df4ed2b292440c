// Routing of samples to the local field that owns their voxel (Sec. 5:
// each occupied voxel is labelled with its tiny MLP; the labels come from
// Alg.1 Stage II). A stable counting sort by field id over the samples in
// slot layout (sample k of ray r at slot (r - r % 64) S + 64 k + r % 64):
//   1. every wave takes a contiguous run of 64-ray blocks and counts the
//      field ids of their samples (block by block, k by k, lane = ray); the
//      render path gathers the same counts during the traversal instead
//      (sample.hip), and this pass is then skipped;
//   2. per field, an exclusive scan over the waves' counts; then a scan over
//      the fields gives each field's first sorted position (start[F] = total);
//   3. every wave walks its blocks again in the same order and places each
//      sample at field_start + (earlier waves' count) + (rank among equal ids
//      so far), the rank within 64 lanes coming from one ballot per distinct
//      field id among the lanes.
// perm[sorted position] = slot; the order inside each field is the fixed
// walk order, so the sort is deterministic.
#include "r360_internal.h"

namespace r360 {

namespace {

// The 64-ray blocks [beg, end) and sample levels [klo, khi) of route wave
// w (RouteMap).
__device__ __forceinline__ void unit_of(int64_t N, RouteMap m, int w, int& beg, int& end, int& klo, int& khi) {
    const int nblk = (int)((N + 63) / 64);
    if (m.lr == 1) {
        beg = min(nblk, w * m.per);
        end = min(nblk, beg + m.per);
        klo = 0;
        khi = m.ls;
    } else {
        beg = min(nblk, w / m.lr);
        end = min(nblk, beg + 1);
        klo = (w % m.lr) * m.ls;
        khi = klo + m.ls;
    }
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) v = max(v, __shfl_xor(v, s, 64));
    return v;
}

// Field ids of sample levels k0 .. k0+RB-1 of this lane's ray in block blk
// (-1 past the ray's count); the loads are issued together.
constexpr int RB = 16;
__device__ __forceinline__ void load_levels(const int32_t* __restrict__ field, int slot0, int k0, int c, int fv[RB]) {
#pragma unroll
    for (int u = 0; u < RB; ++u) {
        const int k = k0 + u < c ? k0 + u : (c > 0 ? c - 1 : 0);
        const int v = field[slot0 + 64 * k];
        fv[u] = k0 + u < c ? v : -1;
    }
}

template <int WPB>
__global__ __launch_bounds__(WPB * 64) void k_hist(const int32_t* __restrict__ field, const int32_t* __restrict__ cnt,
                                                   int64_t N, int smax, int F, int rw, RouteMap m,
                                                   int32_t* __restrict__ hist) {
    extern __shared__ int32_t lds[];
    const int wl = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int32_t* h = lds + wl * F;
    for (int f = lane; f < F; f += 64) h[f] = 0;
    const int w = blockIdx.x * WPB + wl;
    int beg, end, klo, khi;
    unit_of(N, m, w, beg, end, klo, khi);
    int c_next = 0;
    if (beg < end) { const int64_t r = (int64_t)beg * 64 + lane; c_next = r < N ? cnt[r] : 0; }
    for (int blk = beg; blk < end; ++blk) {
        const int c = c_next;
        if (blk + 1 < end) { const int64_t r = (int64_t)(blk + 1) * 64 + lane; c_next = r < N ? cnt[r] : 0; }
        const int kmax = min(wave_max(c), khi);
        const int cu = min(c, khi);
        const int slot0 = blk * 64 * smax + lane;
        for (int k0 = klo; k0 < kmax; k0 += RB) {
            int fv[RB];
            load_levels(field, slot0, k0, cu, fv);
#pragma unroll
            for (int u = 0; u < RB; ++u)
                if (fv[u] >= 0) atomicAdd(&h[fv[u]], 1);
        }
    }
    __syncthreads();
    for (int f = lane; f < F; f += 64) hist[(int64_t)f * rw + w] = h[f];
}

__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        const int t = __shfl_up(v, s, 64);
        if (lane >= s) v += t;
    }
    return v;
}

__device__ __forceinline__ int block_excl_scan(int v, int* total) {
    __shared__ int wsum[16];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int inc = wave_incl_scan(v);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    if (w == 0) {
        int x = lane < 16 ? wsum[lane] : 0;
        x = wave_incl_scan(x);
        if (lane < 16) wsum[lane] = x;
    }
    __syncthreads();
    const int before = w > 0 ? wsum[w - 1] : 0;
    *total = wsum[15];
    __syncthreads();
    return before + inc - v;
}

// One block per field: exclusive scan over the waves' counts (in place);
// the field's total goes to cnt[f].
__global__ __launch_bounds__(1024) void k_rows(int32_t* __restrict__ hist, int rw, int32_t* __restrict__ cnt) {
    const int f = blockIdx.x;
    int32_t* row = hist + (int64_t)f * rw;
    int carry = 0;
    for (int base = 0; base < rw; base += 4096) {
        int v[4], s = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = base + threadIdx.x * 4 + k;
            v[k] = i < rw ? row[i] : 0;
            s += v[k];
        }
        int tot;
        int ex = carry + block_excl_scan(s, &tot);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = base + threadIdx.x * 4 + k;
            if (i < rw) row[i] = ex;
            ex += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) cnt[f] = carry;
}

// Exclusive scan over the fields' totals (in place); start[F] = total.
__global__ __launch_bounds__(1024) void k_fields(int32_t* __restrict__ start, int F) {
    int carry = 0;
    for (int base = 0; base < F; base += 1024) {
        const int i = base + threadIdx.x;
        const int v = i < F ? start[i] : 0;
        int tot;
        const int ex = block_excl_scan(v, &tot);
        if (i < F) start[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) start[F] = carry;
}

template <int WPB>
__global__ __launch_bounds__(WPB * 64) void k_scatter(const int32_t* __restrict__ field, const int32_t* __restrict__ cnt,
                                                      int64_t N, int smax, int F, int rw, RouteMap m,
                                                      const int32_t* __restrict__ hist, const int32_t* __restrict__ start,
                                                      int32_t* __restrict__ perm) {
    extern __shared__ int32_t lds[];
    const int wl = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int32_t* run = lds + wl * F;
    const int w = blockIdx.x * WPB + wl;
    int beg, end, klo, khi;
    unit_of(N, m, w, beg, end, klo, khi);
    if (beg < end)
        for (int f = lane; f < F; f += 64) run[f] = start[f] + hist[(int64_t)f * rw + w];
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int c_next = 0;
    if (beg < end) { const int64_t r = (int64_t)beg * 64 + lane; c_next = r < N ? cnt[r] : 0; }
    for (int blk = beg; blk < end; ++blk) {
        const int c = c_next;
        if (blk + 1 < end) { const int64_t r = (int64_t)(blk + 1) * 64 + lane; c_next = r < N ? cnt[r] : 0; }
        const int kmax = min(wave_max(c), khi);
        const int cu = min(c, khi);
        const int slot0 = blk * 64 * smax + lane;
        for (int k0 = klo; k0 < kmax; k0 += RB) {
            int fv[RB];
            load_levels(field, slot0, k0, cu, fv);
#pragma unroll
            for (int u = 0; u < RB; ++u) {
                if (k0 + u >= kmax) break;                  // wave-uniform
                const bool valid = fv[u] >= 0;
                const int f = fv[u];   // -1 when not valid
                // the lanes sharing this lane's field: peel one field per
                // round (the first lane not yet grouped names it); the 64
                // rays of a block are neighbours, so a level holds few fields
                uint64_t rest = __ballot(valid), peers = 0;
                while (rest) {
                    const int fl = __builtin_amdgcn_readlane(f, (int)__builtin_ctzll(rest));
                    const uint64_t m = __ballot(f == fl);
                    peers = f == fl ? m : peers;
                    rest &= ~m;
                }
                if (valid) {
                    const int rank = __popcll(peers & lt);
                    const int n = __popcll(peers);
                    const int pos = run[f] + rank;
                    perm[pos] = slot0 + 64 * (k0 + u);
                    if (rank == n - 1) run[f] = pos + 1;
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
    }
}

}  // namespace

int route_waves(int F) {
    int rw = ROUTE_WAVES;
    while (rw > 256 && (int64_t)rw * F > (4 << 20)) rw >>= 1;
    return rw;
}

// Level ranges only when blocks are fewer than waves, at most eight per
// block, each of at least RB levels, and at most 1024 counters per wave for
// the walk-time counting (4 lr F ints of LDS per traversal block).
RouteMap route_map(int64_t N, int smax, int F) {
    const int rw = route_waves(F);
    const int64_t nblk = (N + 63) / 64;
    if (nblk >= rw || smax <= RB) return RouteMap{(int)std::max<int64_t>(1, (nblk + rw - 1) / rw), 1, smax};
    int64_t lr = std::min<int64_t>(rw / std::max<int64_t>(nblk, 1), (smax + RB - 1) / RB);
    lr = std::min<int64_t>(lr, 8);
    lr = std::min<int64_t>(lr, std::max(1, 1024 / std::max(F, 1)));
    if (lr <= 1) return RouteMap{1, 1, smax};
    const int ls = (int)((smax + lr - 1) / lr);
    return RouteMap{1, (int)((smax + ls - 1) / ls), ls};
}

hipError_t launch_route(const Workspace& w, int F, bool counted, hipStream_t st) {
    const int rw = route_waves(F);
    const int64_t N = w.N;
    const int smax = w.slots.smax;
    const RouteMap m = route_map(N, smax, F);
    if (counted) {
        // step 1 was done during the traversal
    } else if (F <= 4096) {
        const size_t lds = 4 * F * sizeof(int32_t);
        hipLaunchKernelGGL(k_hist<4>, dim3(rw / 4), dim3(256), lds, st, w.field, w.ray_off, N, smax, F, rw, m, w.hist);
    } else {
        const size_t lds = F * sizeof(int32_t);
        hipLaunchKernelGGL(k_hist<1>, dim3(rw), dim3(64), lds, st, w.field, w.ray_off, N, smax, F, rw, m, w.hist);
    }
    hipLaunchKernelGGL(k_rows, dim3(F), dim3(1024), 0, st, w.hist, rw, w.field_start);
    hipLaunchKernelGGL(k_fields, dim3(1), dim3(1024), 0, st, w.field_start, F);
    if (F <= 4096) {
        const size_t lds = 4 * F * sizeof(int32_t);
        hipLaunchKernelGGL(k_scatter<4>, dim3(rw / 4), dim3(256), lds, st, w.field, w.ray_off, N, smax, F, rw, m,
                           w.hist, w.field_start, w.perm);
    } else {
        const size_t lds = F * sizeof(int32_t);
        hipLaunchKernelGGL(k_scatter<1>, dim3(rw), dim3(64), lds, st, w.field, w.ray_off, N, smax, F, rw, m,
                           w.hist, w.field_start, w.perm);
    }
    return hipGetLastError();
}

}  // namespace r360
