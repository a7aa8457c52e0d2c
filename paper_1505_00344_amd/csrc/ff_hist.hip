// ff_hist.hip — 2D density projection (Appendix A "Render Technique" and
// Appendix A.1: each particle is a unit-weight point added into the pixel it
// projects to), as exact uint32 counts.
//
// Binning, in double precision whatever the state precision (float values
// convert exactly): vx = (a - x_lo) * sx with sx = nx / (x_hi - x_lo) formed
// on the host; kept iff 0 <= vx < nx and 0 <= vy < ny (NaN fails); bin =
// floor(vy) * nx + floor(vx).
//
// The grids of interest (512^2 and 1024^2 uint32 = 1-4 MB) are far larger
// than one CU's 160 KB of LDS, and particle order in memory is random with
// respect to bins, so privatising the whole grid per block is impossible and
// privatising a tile per block would re-read every particle once per tile.
// The large-grid path therefore partitions by tile first (a counting sort on
// the tile index), then accumulates each tile in LDS and merges it into the
// global grid with one atomic per non-zero bin per block:
//   1. count:   bin of every particle -> binbuf; per-block tile counts; drops
//   2. scan:    exclusive scan of each tile's per-block counts (one block
//               per tile), then of the tile totals (one block)
//   3. scatter: local bin index (uint16) of every kept particle -> its tile's
//               segment of `sorted`
//   4. accum:   block = (tile, chunk of <= 8192 entries): LDS histogram of
//               the 16384-bin tile, then atomicAdd of the non-zero bins.
// Grids of at most 16384 bins skip 1-3 (one LDS histogram per block over a
// stride of particles).  Algorithmic HBM traffic of the large path per kept
// particle: read 2 coordinates, write+read 4 B bin, write+read 2 B local bin;
// plus the grid (clear + merge).
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "ff_internal.h"
#include "ff_scan.h"

namespace ff {

namespace {

constexpr int kTileBits = 14;
constexpr uint32_t kTile = 1u << kTileBits;      // bins per LDS tile (64 KB)
constexpr int kBlock = 256;
constexpr int kPerThread = 16;
constexpr int64_t kChunk = (int64_t)kBlock * kPerThread;  // particles per count/scatter block
constexpr int64_t kAccChunk = 8192;                     // sorted entries per accumulate block
constexpr int kMaxTiles = 4096;                         // grids up to 64M bins
constexpr uint32_t kNone = 0xFFFFFFFFu;

struct Geom {
    double xlo, ylo, sx, sy;
    int nx, ny;
};

template <typename R>
__device__ __forceinline__ uint32_t bin_of(R a, R b, const Geom& g) {
    const double vx = ((double)a - g.xlo) * g.sx;
    const double vy = ((double)b - g.ylo) * g.sy;
    const bool ok = (vx >= 0.0) && (vx < (double)g.nx) && (vy >= 0.0) && (vy < (double)g.ny);
    const int ix = (int)(ok ? vx : 0.0);
    const int iy = (int)(ok ? vy : 0.0);
    return ok ? (uint32_t)iy * (uint32_t)g.nx + (uint32_t)ix : kNone;
}

__global__ void k_fill(uint32_t* hist, int64_t nbins, unsigned long long* dropped) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = i; k < nbins; k += stride) hist[k] = 0u;
    if (i == 0 && dropped) *dropped = 0ull;
}

__device__ __forceinline__ void add_drops(unsigned long long* dropped, unsigned int mine,
                                          unsigned int* s_drop) {
    if (!dropped) return;
    if (mine) atomicAdd(s_drop, mine);
    __syncthreads();
    if (threadIdx.x == 0 && *s_drop) atomicAdd(dropped, (unsigned long long)*s_drop);
}

// Grids of <= kTile bins: LDS histogram per block, grid-stride over particles.
template <typename R>
__global__ void __launch_bounds__(kBlock) k_hist_small(const R* ax, const R* ay, int64_t n, Geom g,
                                                       uint32_t* hist, unsigned long long* dropped) {
    __shared__ uint32_t s[kTile];
    __shared__ unsigned int s_drop;
    const uint32_t nbins = (uint32_t)g.nx * (uint32_t)g.ny;
    for (uint32_t k = threadIdx.x; k < nbins; k += blockDim.x) s[k] = 0u;
    if (threadIdx.x == 0) s_drop = 0u;
    __syncthreads();
    unsigned int drops = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t b = bin_of<R>(ax[i], ay[i], g);
        if (b != kNone) atomicAdd(&s[b], 1u);
        else ++drops;
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < nbins; k += blockDim.x)
        if (s[k]) atomicAdd(&hist[k], s[k]);
    add_drops(dropped, drops, &s_drop);
}

// 1. count
template <typename R>
__global__ void __launch_bounds__(kBlock) k_hist_count(const R* ax, const R* ay, int64_t n, Geom g,
                                                       int ntiles, uint32_t* binbuf, uint32_t* counts,
                                                       unsigned long long* dropped) {
    __shared__ uint32_t cnt[kMaxTiles];
    __shared__ unsigned int s_drop;
    const int nblk = gridDim.x;
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x) cnt[t] = 0u;
    if (threadIdx.x == 0) s_drop = 0u;
    __syncthreads();
    const int64_t lo = (int64_t)blockIdx.x * kChunk;
    const int64_t hi = lo + kChunk < n ? lo + kChunk : n;
    unsigned int drops = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const uint32_t b = bin_of<R>(ax[i], ay[i], g);
        binbuf[i] = b;
        if (b != kNone) atomicAdd(&cnt[b >> kTileBits], 1u);
        else ++drops;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x) counts[(int64_t)t * nblk + blockIdx.x] = cnt[t];
    add_drops(dropped, drops, &s_drop);
}

// 3. scatter
__global__ void __launch_bounds__(kBlock) k_hist_scatter(const uint32_t* binbuf, int64_t n, int ntiles,
                                                         const uint32_t* offsets, const uint32_t* tile_start,
                                                         uint16_t* sorted) {
    __shared__ uint32_t cur[kMaxTiles];
    const int nblk = gridDim.x;
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x)
        cur[t] = tile_start[t] + offsets[(int64_t)t * nblk + blockIdx.x];
    __syncthreads();
    const int64_t lo = (int64_t)blockIdx.x * kChunk;
    const int64_t hi = lo + kChunk < n ? lo + kChunk : n;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const uint32_t b = binbuf[i];
        if (b == kNone) continue;
        const uint32_t pos = atomicAdd(&cur[b >> kTileBits], 1u);
        sorted[pos] = (uint16_t)(b & (kTile - 1));
    }
}

// 4. accumulate one (tile, chunk) in LDS and merge
__global__ void __launch_bounds__(kBlock) k_hist_accum(const uint16_t* sorted, int ntiles,
                                                       const uint32_t* tile_start,
                                                       const uint32_t* chunk_start, uint32_t* hist) {
    __shared__ uint32_t s[kTile];
    const uint32_t g = blockIdx.x;
    if (g >= chunk_start[ntiles]) return;  // uniform: more blocks than chunks were launched
    const int t = tile_of_chunk(chunk_start, ntiles, g);
    const int64_t lo = (int64_t)tile_start[t] + (int64_t)(g - chunk_start[t]) * kAccChunk;
    const int64_t end = tile_start[t + 1];
    const int64_t hi = lo + kAccChunk < end ? lo + kAccChunk : end;
    for (uint32_t k = threadIdx.x; k < kTile; k += blockDim.x) s[k] = 0u;
    __syncthreads();
    for (int64_t j = lo + threadIdx.x; j < hi; j += blockDim.x) atomicAdd(&s[sorted[j]], 1u);
    __syncthreads();
    uint32_t* dst = hist + (int64_t)t * kTile;
    for (uint32_t k = threadIdx.x; k < kTile; k += blockDim.x)
        if (s[k]) atomicAdd(&dst[k], s[k]);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct WsLayout {
    size_t binbuf, sorted, counts, tile_total, tile_start, chunk_start, total;
};

WsLayout layout(int64_t n, int64_t nbins) {
    WsLayout L{};
    if (nbins <= (int64_t)kTile) return L;
    const int64_t ntiles = (nbins + kTile - 1) / kTile;
    const int64_t nblk = (n + kChunk - 1) / kChunk;
    size_t off = 0;
    L.binbuf = off;
    off += align256((size_t)n * 4);
    L.sorted = off;
    off += align256((size_t)n * 2);
    L.counts = off;
    off += align256((size_t)ntiles * (size_t)nblk * 4);
    L.tile_total = off;
    off += align256((size_t)ntiles * 4);
    L.tile_start = off;
    off += align256((size_t)(ntiles + 1) * 4);
    L.chunk_start = off;
    off += align256((size_t)(ntiles + 1) * 4);
    L.total = off;
    return L;
}

template <typename R>
hipError_t run_hist(const R* ax, const R* ay, int64_t n, const Geom& g, uint32_t* hist,
                    unsigned long long* dropped, bool accumulate, char* ws, hipStream_t st) {
    const int64_t nbins = (int64_t)g.nx * g.ny;
    if (!accumulate) {
        const int64_t blocks = std::min<int64_t>((nbins + 1023) / 1024, 2048);
        hipLaunchKernelGGL(k_fill, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(1024), 0, st, hist,
                           nbins, dropped);
        if (hipError_t e = hipGetLastError()) return e;
    }
    if (n == 0) return hipSuccess;
    if (nbins <= (int64_t)kTile) {
        const int64_t blocks = std::min<int64_t>((n + kChunk - 1) / kChunk, 1024);
        hipLaunchKernelGGL((k_hist_small<R>), dim3((unsigned)blocks), dim3(kBlock), 0, st, ax, ay, n, g, hist,
                           dropped);
        return hipGetLastError();
    }
    const WsLayout L = layout(n, nbins);
    const int ntiles = (int)((nbins + kTile - 1) / kTile);
    const int nblk = (int)((n + kChunk - 1) / kChunk);
    uint32_t* binbuf = (uint32_t*)(ws + L.binbuf);
    uint16_t* sorted = (uint16_t*)(ws + L.sorted);
    uint32_t* counts = (uint32_t*)(ws + L.counts);
    uint32_t* ttotal = (uint32_t*)(ws + L.tile_total);
    uint32_t* tstart = (uint32_t*)(ws + L.tile_start);
    uint32_t* cstart = (uint32_t*)(ws + L.chunk_start);
    hipLaunchKernelGGL((k_hist_count<R>), dim3(nblk), dim3(kBlock), 0, st, ax, ay, n, g, ntiles, binbuf, counts,
                       dropped);
    if (hipError_t e = hipGetLastError()) return e;
    hipLaunchKernelGGL(k_scan_blocks, dim3(ntiles), dim3(1024), 0, st, counts, nblk, ttotal);
    if (hipError_t e = hipGetLastError()) return e;
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, st, ttotal, ntiles, (uint32_t)kAccChunk, tstart,
                       cstart);
    if (hipError_t e = hipGetLastError()) return e;
    hipLaunchKernelGGL(k_hist_scatter, dim3(nblk), dim3(kBlock), 0, st, binbuf, n, ntiles, counts, tstart, sorted);
    if (hipError_t e = hipGetLastError()) return e;
    const int64_t acc_blocks = (n + kAccChunk - 1) / kAccChunk + ntiles;
    hipLaunchKernelGGL(k_hist_accum, dim3((unsigned)acc_blocks), dim3(kBlock), 0, st, sorted, ntiles, tstart,
                       cstart, hist);
    return hipGetLastError();
}

}  // namespace

namespace {

// A validated projection request: the geometry and the two axis columns.
struct Projection {
    Geom g;
    const void* ax;
    const void* ay;
    int64_t n;
    bool f64;
};

ff_status check_projection(const ff_system_s* sys, const ff_batch* b, int32_t axis_x, int32_t axis_y,
                           double x_lo, double x_hi, double y_lo, double y_hi, int32_t nx, int32_t ny,
                           const uint32_t* hist, Projection* out) {
    if (ff_status s = check_system(sys)) return s;
    if (ff_status s = check_batch(sys, b, false)) return s;
    if (b->n > 0 && !b->state) return fail(FF_E_INVALID, "batch.state is NULL");
    auto axis_ok = [&](int a) { return (a >= 0 && a < sys->dim) || (a < 0 && -1 - a < b->n_pp); };
    if (!axis_ok(axis_x) || !axis_ok(axis_y))
        return fail(FF_E_INVALID, "axis must be a state component (>= 0) or -1 - k for a per-particle parameter k");
    if (nx <= 0 || ny <= 0) return fail(FF_E_INVALID, "nx and ny must be positive");
    if ((int64_t)nx * ny > (int64_t)kMaxTiles * kTile) return fail(FF_E_UNSUPPORTED, "grid larger than 64M bins");
    if (!std::isfinite(x_lo) || !std::isfinite(x_hi) || !std::isfinite(y_lo) || !std::isfinite(y_hi) ||
        !(x_hi > x_lo) || !(y_hi > y_lo))
        return fail(FF_E_INVALID, "ranges must be finite with hi > lo");
    if (!hist) return fail(FF_E_INVALID, "hist is NULL");
    if (b->n > 0x7fffffffLL) return fail(FF_E_UNSUPPORTED, "more than 2^31 - 1 particles in one projection");
    Geom g;
    g.xlo = x_lo;
    g.ylo = y_lo;
    g.sx = (double)nx / (x_hi - x_lo);
    g.sy = (double)ny / (y_hi - y_lo);
    if (!std::isfinite(g.sx) || !std::isfinite(g.sy)) return fail(FF_E_INVALID, "range too small");
    g.nx = nx;
    g.ny = ny;
    const size_t esz = prec_size(b->prec);
    auto col = [&](int a) -> const void* {
        return a >= 0 ? (const char*)b->state + (size_t)a * b->ld * esz
                      : (const char*)b->pparams + (size_t)(-1 - a) * b->ld * esz;
    };
    out->g = g;
    out->ax = col(axis_x);
    out->ay = col(axis_y);
    out->n = b->n;
    out->f64 = b->prec == FF_FP64;
    return FF_OK;
}

hipError_t run_projection(const Projection& P, uint32_t* hist, unsigned long long* dropped, bool accumulate,
                          char* ws, hipStream_t st) {
    if (P.f64)
        return run_hist<double>((const double*)P.ax, (const double*)P.ay, P.n, P.g, hist, dropped, accumulate, ws,
                                st);
    return run_hist<float>((const float*)P.ax, (const float*)P.ay, P.n, P.g, hist, dropped, accumulate, ws, st);
}

}  // namespace

// Scratch of ff_project_histogram_noalloc: a file-scope device array, one
// copy per GPU (at its own address), held from the library's load on that
// GPU until the process ends.  Every buffer in it is written before it is
// read within one call, so nothing needs clearing between calls.  Host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in): the per-device address comes from hipGetSymbolAddress.
constexpr size_t kNoAllocBytes = (size_t)FF_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up on the first
// call on that device (no allocation, now or later).
ff_status noalloc_scratch(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return device_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(FF_E_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return device_fail(e, "hipGetSymbolAddress of the histogram's static scratch");
        if (!p) return fail(FF_E_DEVICE, "hipGetSymbolAddress returned a null address for the static scratch");
        g_noalloc_ptr[dev] = p;
    }
    *out = g_noalloc_ptr[dev];
    return FF_OK;
}

}  // namespace

namespace {
// Library-owned scratch per device and use (grown on demand, kept for the
// process).
struct Scratch {
    void* ptr = nullptr;
    size_t bytes = 0;
};
std::mutex g_scratch_mu;
std::vector<Scratch> g_scratch[kScratchUses];
}  // namespace

ff_status library_scratch(int use, size_t need, hipStream_t stream, void** out) {
    static const char* const kWhat[kScratchUses] = {"histogram", "render"};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return device_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    std::vector<Scratch>& per_dev = g_scratch[use];
    if ((int)per_dev.size() <= dev) per_dev.resize(dev + 1);
    Scratch& s = per_dev[dev];
    if (s.bytes < need) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
            return fail(FF_E_NOMEM, std::string(kWhat[use]) + " scratch must be passed as `workspace` under stream capture");
        if (s.ptr) {
            e = hipStreamSynchronize(stream);
            if (e != hipSuccess) return device_fail(e, "hipStreamSynchronize");
            (void)hipFree(s.ptr);
            s.ptr = nullptr;
            s.bytes = 0;
        }
        e = hipMalloc(&s.ptr, need);
        if (e != hipSuccess) {
            s.ptr = nullptr;
            return fail(FF_E_NOMEM, std::string("hipMalloc of ") + kWhat[use] + " scratch: " + hipGetErrorString(e));
        }
        s.bytes = need;
    }
    *out = s.ptr;
    return FF_OK;
}

}  // namespace ff

using namespace ff;

extern "C" {

ff_status ff_histogram_workspace_size(int64_t n, int32_t nx, int32_t ny, size_t* bytes) {
    set_error("");
    if (!bytes) return fail(FF_E_INVALID, "bytes is NULL");
    if (n < 0 || nx <= 0 || ny <= 0) return fail(FF_E_INVALID, "n < 0 or grid size <= 0");
    const int64_t nbins = (int64_t)nx * ny;
    if (nbins > (int64_t)kMaxTiles * kTile) return fail(FF_E_UNSUPPORTED, "grid larger than 64M bins");
    *bytes = layout(n, nbins).total;
    return FF_OK;
}

ff_status ff_project_histogram(ff_system_t sys, const ff_batch* b, int32_t axis_x, int32_t axis_y,
                               double x_lo, double x_hi, double y_lo, double y_hi, int32_t nx,
                               int32_t ny, uint32_t* hist, uint64_t* n_dropped, int32_t accumulate,
                               void* workspace, size_t workspace_bytes, void* stream) {
    set_error("");
    Projection P;
    if (ff_status s = check_projection(sys, b, axis_x, axis_y, x_lo, x_hi, y_lo, y_hi, nx, ny, hist, &P))
        return s;
    hipStream_t st = (hipStream_t)stream;
    const size_t need = layout(b->n, (int64_t)nx * ny).total;
    char* ws = nullptr;
    if (need > 0 && b->n > 0) {
        if (workspace) {
            if (workspace_bytes < need)
                return fail(FF_E_NOMEM, "histogram workspace too small: need " + std::to_string(need) + " bytes");
            ws = (char*)workspace;
        } else {
            void* p = nullptr;
            if (ff_status s = library_scratch(kScratchHistogram, need, st, &p)) return s;
            ws = (char*)p;
        }
    }
    const hipError_t e = run_projection(P, hist, (unsigned long long*)n_dropped, accumulate != 0, ws, st);
    if (e != hipSuccess) return device_fail(e, "ff_project_histogram launch");
    return FF_OK;
}

ff_status ff_project_histogram_noalloc(ff_system_t sys, const ff_batch* b, int32_t axis_x, int32_t axis_y,
                                       double x_lo, double x_hi, double y_lo, double y_hi, int32_t nx,
                                       int32_t ny, uint32_t* hist, uint64_t* n_dropped, int32_t accumulate,
                                       void* stream) {
    set_error("");
    Projection P;
    if (ff_status s = check_projection(sys, b, axis_x, axis_y, x_lo, x_hi, y_lo, y_hi, nx, ny, hist, &P))
        return s;
    const size_t need = layout(b->n, (int64_t)nx * ny).total;
    char* ws = nullptr;
    if (need > 0 && b->n > 0) {
        if (need > kNoAllocBytes)
            return fail(FF_E_NOMEM, "ff_project_histogram_noalloc: this projection needs " + std::to_string(need) +
                                        " bytes of scratch, more than the " + std::to_string(kNoAllocBytes) +
                                        " bytes its static buffer holds; use ff_project_histogram with a workspace");
        void* p = nullptr;
        if (ff_status s = noalloc_scratch(&p)) return s;
        ws = (char*)p;
    }
    const hipError_t e = run_projection(P, hist, (unsigned long long*)n_dropped, accumulate != 0, ws,
                                        (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "ff_project_histogram_noalloc launch");
    return FF_OK;
}

}  // extern "C"
