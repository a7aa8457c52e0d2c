// ff_scan.h — the scans of a counting sort by tile, shared by the density
// histogram and the tiled particle image.  A count pass writes, for every
// count/scatter block b and tile t, counts[t * nblk + b] = entries of block b
// that fall in tile t; these kernels turn that into
//   counts[t * nblk + b]  -> exclusive prefix of block b within tile t,
//   tile_start[t]         -> first entry of tile t in the sorted array
//                            (tile_start[ntiles] = all entries),
//   chunk_start[t]        -> first accumulate chunk of tile t, with tile t
//                            split into ceil(entries / chunk) chunks
//                            (chunk_start[ntiles] = all chunks).
// Each translation unit gets its own copy (internal linkage).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace ff {
namespace {

// Exclusive scan over a block of 1024 threads (16 wavefronts of 64):
// returns the exclusive prefix of v and writes the block total to *total.
__device__ __forceinline__ uint32_t block_scan_1024(uint32_t v, uint32_t* wsum, uint32_t* total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t inc = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(inc, off, 64);
        if (lane >= off) inc += t;
    }
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();
    if (wv == 0) {
        uint32_t s = lane < 16 ? wsum[lane] : 0u;
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
            const uint32_t t = __shfl_up(s, off, 64);
            if (lane >= off) s += t;
        }
        if (lane < 16) wsum[16 + lane] = s;  // inclusive scan of wave sums
    }
    __syncthreads();
    const uint32_t before = wv ? wsum[16 + wv - 1] : 0u;
    *total = wsum[16 + 15];
    __syncthreads();
    return before + inc - v;
}

// Per-tile scan over the count blocks (one block of 1024 threads per tile).
__global__ void __launch_bounds__(1024) k_scan_blocks(uint32_t* counts, int nblk, uint32_t* tile_total) {
    __shared__ uint32_t wsum[32];
    uint32_t* row = counts + (int64_t)blockIdx.x * nblk;
    uint32_t carry = 0;
    for (int base = 0; base < nblk; base += 1024) {
        const int b = base + threadIdx.x;
        const uint32_t v = b < nblk ? row[b] : 0u;
        uint32_t tot;
        const uint32_t ex = block_scan_1024(v, wsum, &tot);
        if (b < nblk) row[b] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) tile_total[blockIdx.x] = carry;
}

// Scan over tiles (one block of 1024 threads): entry and chunk offsets.
__global__ void __launch_bounds__(1024) k_scan_tiles(const uint32_t* tile_total, int ntiles, uint32_t chunk,
                                                     uint32_t* tile_start, uint32_t* chunk_start) {
    __shared__ uint32_t wsum[32];
    uint32_t carry = 0, ccarry = 0;
    for (int base = 0; base < ntiles; base += 1024) {
        const int t = base + threadIdx.x;
        const uint32_t v = t < ntiles ? tile_total[t] : 0u;
        const uint32_t c = (v + chunk - 1) / chunk;
        uint32_t tot, ctot;
        const uint32_t ex = block_scan_1024(v, wsum, &tot);
        const uint32_t cex = block_scan_1024(c, wsum, &ctot);
        if (t < ntiles) {
            tile_start[t] = carry + ex;
            chunk_start[t] = ccarry + cex;
        }
        carry += tot;
        ccarry += ctot;
    }
    if (threadIdx.x == 0) {
        tile_start[ntiles] = carry;
        chunk_start[ntiles] = ccarry;
    }
}

// The tile of accumulate chunk g: the largest t with chunk_start[t] <= g
// (g < chunk_start[ntiles]).
__device__ __forceinline__ int tile_of_chunk(const uint32_t* chunk_start, int ntiles, uint32_t g) {
    int lo = 0, hi = ntiles;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (chunk_start[mid] <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

}  // namespace
}  // namespace ff
