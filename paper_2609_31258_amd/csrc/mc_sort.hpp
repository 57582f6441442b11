// mc_sort.hpp -- reordering of the pack slots by species and cell (gfx950).
//
// Every sort_every steps the active packs are put in the order of their key
// (species tag, then the lower-left node of their CIC cell) and the slots of
// terminal packs are dropped.  A wavefront then holds packs of one species
// at nearly the same place: their collision rates lambda dt are alike (a
// wavefront runs until its pack with the most candidates is done, so mixed
// species leave most lanes idle), their field gathers read the same table
// records, and the CIC deposit meets long runs of one cell.
//
// The reordering is a stable least-significant-digit radix sort of
// (key, slot) pairs with 8-bit digits: per pass a digit histogram per tile
// of 4096 pairs, one exclusive scan over (digit, tile), and a stable
// scatter in which each pair's rank among equal digits of its tile comes
// from wavefront ballots on the digit's bits.  Stable and free of atomics
// in the ordering, so the resulting slot order is the same on every run.
// The packs are then gathered into a second set of arrays (k_sort_permute)
// and the two sets swap roles.  Slot order changes no pack's arithmetic:
// random streams are keyed by pack id and step, and tallies are integer.
#pragma once
#include "mc_kernels.hpp"

namespace mc {

constexpr int kSortThreads = 256, kSortItems = 16;
constexpr int64_t kSortTile = (int64_t)kSortThreads * kSortItems;  // pairs per tile
constexpr int kRadixBins = 256;
// The scan of the (digit, tile) table covers at most kSortTile blocks of
// kSortTile entries: 65536 tiles, 2^28 slots.
constexpr int64_t kSortMaxSlots = (int64_t)1 << 28;

// Number of 8-bit digits that hold every key below n_keys plus the key of a
// dropped slot (all ones over those digits).
inline int sort_passes(int64_t n_keys) {
    int p = 1;
    while (p < 4 && ((int64_t)1 << (8 * p)) - 1 <= n_keys) ++p;
    return p;
}

// Key of slot s: tag * nn + (j * nr + i) for an active pack, (i, j) the
// lower-left node of its CIC cell clamped to the grid as the deposit clamps
// it; dead_key for a terminal slot.  Per block, the number of active packs
// (partial[3 b]) and the survival-yield term W (1 - exp(-H)) of the
// terminal packs whose slots the sort drops (partial[3 b + 2]), for k_retire.
template <class T>
__global__ __launch_bounds__(256) void k_sort_keys(PackPtrs<T> p, int64_t n, int32_t nr, int32_t nz, double inv_dr,
                                                   double inv_dz, int64_t nn, uint32_t dead_key, uint32_t *keys,
                                                   uint32_t *idx, double *partial) {
    __shared__ double red[2][256];
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool act = false;
    double retire = 0.0;
    if (s < n) {
        uint32_t key = dead_key;
        if (p.status[s] == ST_ACTIVE) {
#pragma clang fp contract(off)
            double X = p.x[s], Y = p.y[s], Z = p.z[s];
            if constexpr (sizeof(T) == 4) {
                X += (double)p.xl[s];
                Y += (double)p.yl[s];
                Z += (double)p.zl[s];
            }
            int64_t cell = 0;
            if (isfinite(X) && isfinite(Y) && isfinite(Z)) {
                double fi = floor(sqrt(X * X + Y * Y) * inv_dr), fj = floor(Z * inv_dz);
                fi = fi > (double)(nr - 2) ? (double)(nr - 2) : fi;
                fj = fj > (double)(nz - 2) ? (double)(nz - 2) : (fj < 0.0 ? 0.0 : fj);
                cell = (int64_t)fj * nr + (int64_t)fi;
            }
            key = (uint32_t)((int64_t)p.tag[s] * nn + cell);
            act = true;
        } else {
            retire = p.w[s] * (-expm1(-(double)p.h[s]));
        }
        keys[s] = key;
        idx[s] = (uint32_t)s;
    }
    red[0][threadIdx.x] = act ? 1.0 : 0.0;
    red[1][threadIdx.x] = retire;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            red[0][threadIdx.x] += red[0][threadIdx.x + o];
            red[1][threadIdx.x] += red[1][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[3 * (int64_t)blockIdx.x] = red[0][0];
        partial[3 * (int64_t)blockIdx.x + 2] = red[1][0];
    }
}

// From the nb blocks' partials, in a fixed order: the active count (exact:
// integers below 2^53) and retired += the dropped packs' survival-yield sum.
static __global__ __launch_bounds__(256) void k_retire(const double *partial, int64_t nb,
                                                       unsigned long long *n_active, double *retired) {
    __shared__ double red[2][256];
    double c = 0.0, a = 0.0;
    for (int64_t b = threadIdx.x; b < nb; b += blockDim.x) {
        c += partial[3 * b];
        a += partial[3 * b + 2];
    }
    red[0][threadIdx.x] = c;
    red[1][threadIdx.x] = a;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            red[0][threadIdx.x] += red[0][threadIdx.x + o];
            red[1][threadIdx.x] += red[1][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *n_active = (unsigned long long)red[0][0];
        *retired += red[1][0];
    }
}

// Digit histogram of each tile, stored digit-major: hist[d * n_tiles + tile].
static __global__ __launch_bounds__(kSortThreads) void k_radix_count(const uint32_t *keys, int64_t n, int32_t shift,
                                                                     uint32_t *hist, int64_t n_tiles) {
    __shared__ uint32_t cnt[kRadixBins];
    cnt[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    uint32_t d[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {  // every load of the tile in flight at once
        const int64_t e = base + (int64_t)r * kSortThreads + threadIdx.x;
        d[r] = e < n ? (keys[e] >> shift) & 255u : 256u;
    }
    // a wavefront whose 64 items share a digit (sorted input) adds them at once
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const uint32_t d0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)d[r]);
        if (__ballot(d[r] == d0) == ~0ull) {
            if (lane == 0 && d0 < 256u) atomicAdd(&cnt[d0], 64u);
        } else if (d[r] < 256u) {
            atomicAdd(&cnt[d[r]], 1u);
        }
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * n_tiles + blockIdx.x] = cnt[threadIdx.x];
}

// Exclusive prefix over a block's 256 thread totals (in LDS), returned per
// thread; *total receives the block's sum.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *lds, uint32_t *total) {
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < kSortThreads; o <<= 1) {
        const uint32_t add = threadIdx.x >= (unsigned)o ? lds[threadIdx.x - o] : 0u;
        __syncthreads();
        lds[threadIdx.x] += add;
        __syncthreads();
    }
    const uint32_t incl = lds[threadIdx.x];
    *total = lds[kSortThreads - 1];
    __syncthreads();
    return incl - v;
}

// In-place exclusive scan of each block's kSortTile consecutive entries;
// tot[block] receives the block's sum.
static __global__ __launch_bounds__(kSortThreads) void k_scan_tiles(uint32_t *h, int64_t len, uint32_t *tot) {
    __shared__ uint32_t lds[kSortThreads];
    const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)threadIdx.x * kSortItems;
    uint32_t v[kSortItems], sum = 0u;
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        v[i] = base + i < len ? h[base + i] : 0u;
        sum += v[i];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(sum, lds, &total);
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        if (base + i < len) h[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == 0) tot[blockIdx.x] = total;
}

// Exclusive scan of the block sums in place (one block; at most kSortTile of them).
static __global__ __launch_bounds__(kSortThreads) void k_scan_totals(uint32_t *tot, int64_t len) {
    __shared__ uint32_t lds[kSortThreads];
    const int64_t base = (int64_t)threadIdx.x * kSortItems;
    uint32_t v[kSortItems], sum = 0u;
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        v[i] = base + i < len ? tot[base + i] : 0u;
        sum += v[i];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(sum, lds, &total);
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        if (base + i < len) tot[base + i] = run;
        run += v[i];
    }
}

// Stable scatter of one pass.  The tile's items are taken in 16 rounds of
// 256 (item r * 256 + t of the tile in round r); within a round an item's
// destination is the digit's running base for this tile, plus the items of
// lower wavefronts with its digit, plus the lower lanes of its own
// wavefront with its digit (found from ballots on the digit's eight bits).
static __global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const uint32_t *kin, const uint32_t *iin,
                                                                       uint32_t *kout, uint32_t *iout, int64_t n,
                                                                       int32_t shift, const uint32_t *hist,
                                                                       const uint32_t *tot, int64_t n_tiles) {
    __shared__ uint32_t base[kRadixBins];
    __shared__ uint32_t wcnt[kSortThreads / 64][kRadixBins];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    {
        const int64_t e = (int64_t)threadIdx.x * n_tiles + blockIdx.x;
        base[threadIdx.x] = hist[e] + tot[e / kSortTile];
    }
#pragma unroll
    for (int k = 0; k < kSortThreads / 64; ++k) wcnt[k][threadIdx.x] = 0u;
    __syncthreads();
    const uint64_t lower = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int64_t t0 = (int64_t)blockIdx.x * kSortTile;
    // the whole tile's pairs are read first (one memory latency per tile)
    uint32_t keyv[kSortItems], idv[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t e = t0 + (int64_t)r * kSortThreads + threadIdx.x;
        keyv[r] = e < n ? kin[e] : 0u;
        idv[r] = e < n ? iin[e] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t e = t0 + (int64_t)r * kSortThreads + threadIdx.x;
        const bool valid = e < n;
        const uint32_t key = keyv[r], id = idv[r];
        const uint32_t d = (key >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lower);
        if (valid && (peers & lower) == 0ull) wcnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t dst = base[d] + rank;
            for (int k = 0; k < w; ++k) dst += wcnt[k][d];
            kout[dst] = key;
            iout[dst] = id;
        }
        __syncthreads();
        uint32_t add = 0u;
#pragma unroll
        for (int k = 0; k < kSortThreads / 64; ++k) {
            add += wcnt[k][threadIdx.x];
            wcnt[k][threadIdx.x] = 0u;
        }
        base[threadIdx.x] += add;
        __syncthreads();
    }
}

// Gather of the sorted packs into the other set of arrays: destination d <
// n_active takes slot idx[d] (the active packs come first in key order).
template <class T>
__global__ __launch_bounds__(256) void k_sort_permute(PackPtrs<T> src, PackPtrs<T> dst, const uint32_t *idx,
                                                      int64_t n, const unsigned long long *n_active) {
    const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= n || d >= (int64_t)*n_active) return;
    const int64_t s = idx[d];
    dst.x[d] = src.x[s];
    dst.y[d] = src.y[s];
    dst.z[d] = src.z[s];
    if constexpr (sizeof(T) == 4) {
        dst.xl[d] = src.xl[s];
        dst.yl[d] = src.yl[s];
        dst.zl[d] = src.zl[s];
        dst.el[d] = src.el[s];
    }
    dst.vx[d] = src.vx[s];
    dst.vy[d] = src.vy[s];
    dst.vz[d] = src.vz[s];
    dst.e[d] = src.e[s];
    dst.h[d] = src.h[s];
    dst.w[d] = src.w[s];
    dst.id[d] = src.id[s];
    dst.q[d] = src.q[s];
    dst.tag[d] = src.tag[s];
    dst.status[d] = ST_ACTIVE;
}

}  // namespace mc
