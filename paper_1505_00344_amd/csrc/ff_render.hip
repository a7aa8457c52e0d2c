// ff_render.hip — particle image (Appendix A "Render Technique"; Appendix A.1:
// the vertex shader applies the model-view matrix, the geometry shader the
// view-projection matrix — orthographic for 2D, perspective for 3D — and
// emits a square sprite; the fragment shader gives each covered pixel an
// intensity that falls off with the distance from the sprite's centre and a
// colour that is fixed or linear in the particle's position; blending adds
// source*alpha into the pixel).
//
// Per particle, all geometry in double precision:
//   c = M (a0, a1, a2, 1) with M = projection * view * model (row-major 4x4);
//   culled if c3 <= 0 or some c_i / c3 (i < 3) is outside [-1, 1] or NaN;
//   px = (c0/c3 + 1) W / 2, py = (1 - c1/c3) H / 2;
//   rgb_k = clamp(base_k + sum_i grad[k][i] (a_i - origin_i), 0, 1);
//   radius 0: pixel (floor px, floor py) gets w = weight; radius R: pixels
//   floor(px - R - 1) .. floor(px + R + 1) (and in y) whose centre is at
//   distance d < R + 1 get w = weight (1 - d / (R + 1))^2;
//   img[(iy W + ix) 3 + k] += rint(256 w rgb_k)   (uint32, modulo 2^32).
// Fixed-point integer accumulation makes the image exact and independent of
// the order in which particles are added, so the two paths below give the
// same image bit for bit.
//
// Tiled path (sprites of radius <= 8, images of <= 4096 tiles of 64 x 32
// pixels, at most 2^29 particles).  Particles projected onto an attractor
// pile onto few pixels, and one global atomic per pixel hit serialises there.
// Instead the particles are counting-sorted by the tiles their sprite touches
// (at most 2 x 2):
//   1. count:   project every particle; code of its tile range -> `code`;
//               per-block tile counts; culled count
//   2. scan:    per tile over blocks, then over tiles (entry and chunk offsets)
//   3. scatter: particle index -> the segment of every tile it touches
//   4. accum:   block = (tile, chunk of <= 1024 entries), grid-stride: project
//               each entry's particle again (same code, same result), add its
//               pixels inside the tile into a 24 KB LDS tile, then merge the
//               non-zero pixels with one global atomic each.
// Larger sprites or images use the direct path: one thread per particle,
// global atomics per pixel.
#include <algorithm>
#include <cmath>

#include "ff_internal.h"
#include "ff_scan.h"

namespace ff {

namespace {

struct RenderArgs {
    int axis[3];
    double mvp[16];
    int width, height;
    double base[3], grad[9], origin[3];
    double weight;
    int radius;
};

constexpr int kRTileW = 64, kRTileH = 32;
constexpr int kRTilePx = kRTileW * kRTileH;       // 2048 pixels, 24 KB of uint32 RGB
constexpr int kRMaxRadius = 8;                    // sprite <= 19 pixels: <= 2 x 2 tiles
constexpr int kRMaxTiles = 4096;                  // images up to 8M pixels (4K UHD fits)
constexpr int kRBlock = 256;
constexpr int64_t kRChunk = (int64_t)kRBlock * 16;  // particles per count / scatter block
constexpr uint32_t kRAccChunk = 1024;             // entries per accumulate chunk
constexpr int64_t kRMaxCounts = (int64_t)1 << 26;  // tiles x count blocks
constexpr int64_t kRMaxN = (int64_t)1 << 29;       // 4 n entries stay below 2^31 (uint32 offsets)
constexpr uint32_t kRNone = 0xFFFFFFFFu;

struct Point {
    bool keep;
    double px, py;
    double rgb[3];
};

template <typename R>
__device__ __forceinline__ Point project(R a0, R a1, R a2, const RenderArgs& r) {
    Point P;
    const double a[3] = {(double)a0, (double)a1, (double)a2};
    double c[4];
#pragma unroll
    for (int row = 0; row < 4; ++row) {
        const double* m = r.mvp + 4 * row;
        c[row] = m[0] * a[0] + m[1] * a[1] + m[2] * a[2] + m[3];
    }
    bool keep = c[3] > 0.0;
    double ndc[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        ndc[k] = c[k] / c[3];
        keep = keep && ndc[k] >= -1.0 && ndc[k] <= 1.0;
    }
    P.keep = keep;
    P.px = (ndc[0] + 1.0) * (double)r.width / 2.0;
    P.py = (1.0 - ndc[1]) * (double)r.height / 2.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double v = r.base[k];
#pragma unroll
        for (int j = 0; j < 3; ++j) v += r.grad[3 * k + j] * (a[j] - r.origin[j]);
        P.rgb[k] = fmin(fmax(v, 0.0), 1.0);
    }
    return P;
}

// Pixel box of a kept particle's sprite (before clipping to the image).
__device__ __forceinline__ void sprite_box(const Point& P, int radius, int64_t& x0, int64_t& x1, int64_t& y0,
                                           int64_t& y1) {
    const double reach = radius + 1.0;
    x0 = (int64_t)floor(P.px);
    x1 = x0;
    y0 = (int64_t)floor(P.py);
    y1 = y0;
    if (radius > 0) {
        x0 = (int64_t)floor(P.px - reach);
        x1 = (int64_t)floor(P.px + reach);
        y0 = (int64_t)floor(P.py - reach);
        y1 = (int64_t)floor(P.py + reach);
    }
}

// The sprite's weight at pixel (ix, iy) of its box; false outside the disc.
__device__ __forceinline__ bool pixel_weight(const Point& P, int64_t ix, int64_t iy, const RenderArgs& r,
                                             double& w) {
    w = r.weight;
    if (r.radius > 0) {
        const double reach = r.radius + 1.0;
        const double dx = ((double)ix + 0.5) - P.px, dy = ((double)iy + 0.5) - P.py;
        const double d = sqrt(dx * dx + dy * dy);
        if (!(d < reach)) return false;
        const double f = 1.0 - d / reach;
        w = r.weight * (f * f);
    }
    return true;
}

__device__ __forceinline__ uint32_t quantise(double w, double rgb) { return (uint32_t)rint(256.0 * (w * rgb)); }

// ---------------------------------------------------------------- direct path
template <typename R>
__global__ void __launch_bounds__(256) k_render(const R* a0p, const R* a1p, const R* a2p, int64_t n, RenderArgs r,
                                                uint32_t* img, unsigned long long* culled) {
    __shared__ unsigned int s_cull;
    if (threadIdx.x == 0) s_cull = 0u;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const Point P = project<R>(a0p[i], a1p[i], a2p[i], r);
        if (!P.keep) {
            atomicAdd(&s_cull, 1u);
        } else {
            const int64_t W = r.width, H = r.height;
            int64_t x0, x1, y0, y1;
            sprite_box(P, r.radius, x0, x1, y0, y1);
            for (int64_t iy = y0; iy <= y1; ++iy) {
                for (int64_t ix = x0; ix <= x1; ++ix) {
                    if (ix < 0 || ix >= W || iy < 0 || iy >= H) continue;
                    double w;
                    if (!pixel_weight(P, ix, iy, r, w)) continue;
                    uint32_t* pix = img + (iy * W + ix) * 3;
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const uint32_t q = quantise(w, P.rgb[k]);
                        if (q) atomicAdd(pix + k, q);
                    }
                }
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && culled && s_cull) atomicAdd(culled, (unsigned long long)s_cull);
}

__global__ void k_clear_img(uint32_t* img, int64_t len, unsigned long long* culled) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = i; k < len; k += stride) img[k] = 0u;
    if (i == 0 && culled) *culled = 0ull;
}

// ---------------------------------------------------------------- tiled path
// Tile range of a kept particle, clipped to the image: first tile t0 in bits
// 2.., one more tile to the right in bit 0, one more below in bit 1.
__device__ __forceinline__ uint32_t tile_code(const Point& P, const RenderArgs& r, int ntx) {
    int64_t x0, x1, y0, y1;
    sprite_box(P, r.radius, x0, x1, y0, y1);
    x0 = x0 > 0 ? x0 : 0;
    y0 = y0 > 0 ? y0 : 0;
    x1 = x1 < r.width - 1 ? x1 : r.width - 1;
    y1 = y1 < r.height - 1 ? y1 : r.height - 1;
    if (x0 > x1 || y0 > y1) return kRNone;
    const uint32_t tx0 = (uint32_t)(x0 / kRTileW), tx1 = (uint32_t)(x1 / kRTileW);
    const uint32_t ty0 = (uint32_t)(y0 / kRTileH), ty1 = (uint32_t)(y1 / kRTileH);
    return ((ty0 * (uint32_t)ntx + tx0) << 2) | ((ty1 - ty0) << 1) | (tx1 - tx0);
}

template <typename R>
__global__ void __launch_bounds__(kRBlock) k_render_count(const R* a0p, const R* a1p, const R* a2p, int64_t n,
                                                          RenderArgs r, int ntx, int ntiles, uint32_t* code,
                                                          uint32_t* counts, unsigned long long* culled) {
    __shared__ uint32_t cnt[kRMaxTiles];
    __shared__ unsigned int s_cull;
    const int nblk = gridDim.x;
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x) cnt[t] = 0u;
    if (threadIdx.x == 0) s_cull = 0u;
    __syncthreads();
    const int64_t lo = (int64_t)blockIdx.x * kRChunk;
    const int64_t hi = lo + kRChunk < n ? lo + kRChunk : n;
    unsigned int cull = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const Point P = project<R>(a0p[i], a1p[i], a2p[i], r);
        uint32_t cd = kRNone;
        if (!P.keep) {
            ++cull;
        } else {
            cd = tile_code(P, r, ntx);
            if (cd != kRNone) {
                const uint32_t t0 = cd >> 2, dx = cd & 1u, dy = (cd >> 1) & 1u;
                for (uint32_t yy = 0; yy <= dy; ++yy)
                    for (uint32_t xx = 0; xx <= dx; ++xx) atomicAdd(&cnt[t0 + yy * (uint32_t)ntx + xx], 1u);
            }
        }
        code[i] = cd;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x) counts[(int64_t)t * nblk + blockIdx.x] = cnt[t];
    if (culled) {
        if (cull) atomicAdd(&s_cull, cull);
        __syncthreads();
        if (threadIdx.x == 0 && s_cull) atomicAdd(culled, (unsigned long long)s_cull);
    }
}

__global__ void __launch_bounds__(kRBlock) k_render_scatter(const uint32_t* code, int64_t n, int ntx, int ntiles,
                                                            const uint32_t* offsets, const uint32_t* tile_start,
                                                            uint32_t* entries) {
    __shared__ uint32_t cur[kRMaxTiles];
    const int nblk = gridDim.x;
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x)
        cur[t] = tile_start[t] + offsets[(int64_t)t * nblk + blockIdx.x];
    __syncthreads();
    const int64_t lo = (int64_t)blockIdx.x * kRChunk;
    const int64_t hi = lo + kRChunk < n ? lo + kRChunk : n;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const uint32_t cd = code[i];
        if (cd == kRNone) continue;
        const uint32_t t0 = cd >> 2, dx = cd & 1u, dy = (cd >> 1) & 1u;
        for (uint32_t yy = 0; yy <= dy; ++yy)
            for (uint32_t xx = 0; xx <= dx; ++xx) {
                const uint32_t pos = atomicAdd(&cur[t0 + yy * (uint32_t)ntx + xx], 1u);
                entries[pos] = (uint32_t)i;
            }
    }
}

template <typename R>
__global__ void __launch_bounds__(kRBlock) k_render_accum(const R* a0p, const R* a1p, const R* a2p, RenderArgs r,
                                                          int ntx, int ntiles, const uint32_t* entries,
                                                          const uint32_t* tile_start, const uint32_t* chunk_start,
                                                          uint32_t* img) {
    __shared__ uint32_t s[kRTilePx * 3];
    const uint32_t nchunks = chunk_start[ntiles];
    const int64_t W = r.width, H = r.height;
    for (uint32_t g = blockIdx.x; g < nchunks; g += gridDim.x) {  // uniform over the block
        const int t = tile_of_chunk(chunk_start, ntiles, g);
        const int64_t X0 = (int64_t)(t % ntx) * kRTileW, Y0 = (int64_t)(t / ntx) * kRTileH;
        const int64_t Xe = X0 + kRTileW < W ? X0 + kRTileW : W;  // exclusive ends, inside the image
        const int64_t Ye = Y0 + kRTileH < H ? Y0 + kRTileH : H;
        const int64_t lo = (int64_t)tile_start[t] + (int64_t)(g - chunk_start[t]) * kRAccChunk;
        const int64_t end = tile_start[t + 1];
        const int64_t hi = lo + kRAccChunk < end ? lo + kRAccChunk : end;
        for (int k = threadIdx.x; k < kRTilePx * 3; k += blockDim.x) s[k] = 0u;
        __syncthreads();
        for (int64_t j = lo + threadIdx.x; j < hi; j += blockDim.x) {
            const uint32_t i = entries[j];
            const Point P = project<R>(a0p[i], a1p[i], a2p[i], r);
            if (!P.keep) continue;
            int64_t x0, x1, y0, y1;
            sprite_box(P, r.radius, x0, x1, y0, y1);
            x0 = x0 > X0 ? x0 : X0;
            y0 = y0 > Y0 ? y0 : Y0;
            x1 = x1 < Xe - 1 ? x1 : Xe - 1;
            y1 = y1 < Ye - 1 ? y1 : Ye - 1;
            for (int64_t iy = y0; iy <= y1; ++iy)
                for (int64_t ix = x0; ix <= x1; ++ix) {
                    double w;
                    if (!pixel_weight(P, ix, iy, r, w)) continue;
                    uint32_t* px = s + ((iy - Y0) * kRTileW + (ix - X0)) * 3;
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const uint32_t q = quantise(w, P.rgb[k]);
                        if (q) atomicAdd(px + k, q);
                    }
                }
        }
        __syncthreads();
        for (int k = threadIdx.x; k < kRTilePx * 3; k += blockDim.x) {
            const uint32_t v = s[k];
            if (!v) continue;
            const int p = k / 3, ch = k - 3 * p;
            const int64_t ix = X0 + (p & (kRTileW - 1)), iy = Y0 + p / kRTileW;
            if (ix < W && iy < H) atomicAdd(img + (iy * W + ix) * 3 + ch, v);
        }
        __syncthreads();
    }
}

struct RLayout {
    bool tiled;
    int ntx, ntiles, nblk;
    size_t code, counts, tile_total, tile_start, chunk_start, entries, total;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

RLayout rlayout(int64_t n, int width, int height, int radius) {
    RLayout L{};
    const int64_t ntx = (width + kRTileW - 1) / kRTileW, nty = (height + kRTileH - 1) / kRTileH;
    const int64_t nblk = (n + kRChunk - 1) / kRChunk;
    L.tiled = n > 0 && n <= kRMaxN && radius <= kRMaxRadius && ntx * nty <= kRMaxTiles &&
              ntx * nty * nblk <= kRMaxCounts;
    if (!L.tiled) return L;
    L.ntx = (int)ntx;
    L.ntiles = (int)(ntx * nty);
    L.nblk = (int)nblk;
    const int64_t per = radius == 0 ? 1 : 4;  // tiles one sprite can touch
    size_t off = 0;
    L.code = off;
    off += align256((size_t)n * 4);
    L.counts = off;
    off += align256((size_t)L.ntiles * (size_t)nblk * 4);
    L.tile_total = off;
    off += align256((size_t)L.ntiles * 4);
    L.tile_start = off;
    off += align256((size_t)(L.ntiles + 1) * 4);
    L.chunk_start = off;
    off += align256((size_t)(L.ntiles + 1) * 4);
    L.entries = off;
    off += align256((size_t)(per * n) * 4);
    L.total = off;
    return L;
}

template <typename R>
hipError_t run_render(const R* a0, const R* a1, const R* a2, int64_t n, const RenderArgs& r, const RLayout& L,
                      char* ws, uint32_t* img, unsigned long long* culled, hipStream_t st) {
    if (!L.tiled) {
        const unsigned grid = (unsigned)((n + 255) / 256);
        hipLaunchKernelGGL((k_render<R>), dim3(grid), dim3(256), 0, st, a0, a1, a2, n, r, img, culled);
        return hipGetLastError();
    }
    uint32_t* code = (uint32_t*)(ws + L.code);
    uint32_t* counts = (uint32_t*)(ws + L.counts);
    uint32_t* ttotal = (uint32_t*)(ws + L.tile_total);
    uint32_t* tstart = (uint32_t*)(ws + L.tile_start);
    uint32_t* cstart = (uint32_t*)(ws + L.chunk_start);
    uint32_t* entries = (uint32_t*)(ws + L.entries);
    hipLaunchKernelGGL((k_render_count<R>), dim3(L.nblk), dim3(kRBlock), 0, st, a0, a1, a2, n, r, L.ntx, L.ntiles,
                       code, counts, culled);
    if (hipError_t e = hipGetLastError()) return e;
    hipLaunchKernelGGL(k_scan_blocks, dim3(L.ntiles), dim3(1024), 0, st, counts, L.nblk, ttotal);
    if (hipError_t e = hipGetLastError()) return e;
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, st, ttotal, L.ntiles, kRAccChunk, tstart, cstart);
    if (hipError_t e = hipGetLastError()) return e;
    hipLaunchKernelGGL(k_render_scatter, dim3(L.nblk), dim3(kRBlock), 0, st, code, n, L.ntx, L.ntiles, counts,
                       tstart, entries);
    if (hipError_t e = hipGetLastError()) return e;
    const int64_t per = r.radius == 0 ? 1 : 4;
    const int64_t bound = (per * n + kRAccChunk - 1) / kRAccChunk + L.ntiles;
    const unsigned acc_blocks = (unsigned)std::min<int64_t>(bound, 8192);
    hipLaunchKernelGGL((k_render_accum<R>), dim3(acc_blocks), dim3(kRBlock), 0, st, a0, a1, a2, r, L.ntx, L.ntiles,
                       entries, tstart, cstart, img);
    return hipGetLastError();
}

ff_status check_render(const ff_render* r) {
    if (!r) return fail(FF_E_INVALID, "render description is NULL");
    if (r->width <= 0 || r->height <= 0) return fail(FF_E_INVALID, "image size must be positive");
    if ((int64_t)r->width * r->height > (int64_t)1 << 28) return fail(FF_E_UNSUPPORTED, "image larger than 2^28 pixels");
    if (r->radius < 0 || r->radius > 64) return fail(FF_E_INVALID, "sprite radius must be in [0, 64]");
    return FF_OK;
}

}  // namespace

}  // namespace ff

using namespace ff;

extern "C" {

ff_status ff_render_workspace_size(int64_t n, const ff_render* r, size_t* bytes) {
    set_error("");
    if (!bytes) return fail(FF_E_INVALID, "bytes is NULL");
    if (n < 0) return fail(FF_E_INVALID, "n < 0");
    if (ff_status s = check_render(r)) return s;
    const RLayout L = rlayout(n, r->width, r->height, r->radius);
    *bytes = L.tiled ? L.total : 0;
    return FF_OK;
}

ff_status ff_render_image(ff_system_t sys, const ff_batch* b, const ff_render* r, uint32_t* img,
                          uint64_t* n_culled, int32_t accumulate, void* workspace, size_t workspace_bytes,
                          void* stream) {
    set_error("");
    if (ff_status s = check_system(sys)) return s;
    if (ff_status s = check_batch(sys, b, false)) return s;
    if (ff_status s = check_render(r)) return s;
    if (b->n > 0 && !b->state) return fail(FF_E_INVALID, "batch.state is NULL");
    auto axis_ok = [&](int a) { return (a >= 0 && a < sys->dim) || (a < 0 && -1 - a < b->n_pp); };
    for (int i = 0; i < 3; ++i)
        if (!axis_ok(r->axis[i])) return fail(FF_E_INVALID, "render axis must be a state component or -1 - k");
    for (int k = 0; k < 16; ++k)
        if (!std::isfinite(r->mvp[k])) return fail(FF_E_INVALID, "matrix entries must be finite");
    if (!std::isfinite(r->weight) || r->weight < 0.0) return fail(FF_E_INVALID, "weight must be finite and >= 0");
    if (!img) return fail(FF_E_INVALID, "img is NULL");
    hipStream_t st = (hipStream_t)stream;
    RenderArgs a;
    for (int i = 0; i < 3; ++i) a.axis[i] = r->axis[i];
    for (int k = 0; k < 16; ++k) a.mvp[k] = r->mvp[k];
    a.width = r->width;
    a.height = r->height;
    for (int k = 0; k < 3; ++k) {
        a.base[k] = r->base[k];
        a.origin[k] = r->origin[k];
    }
    for (int k = 0; k < 9; ++k) a.grad[k] = r->grad[k];
    a.weight = r->weight;
    a.radius = r->radius;
    const RLayout L = rlayout(b->n, r->width, r->height, r->radius);
    char* ws = nullptr;
    if (L.tiled) {
        if (workspace) {
            if (workspace_bytes < L.total)
                return fail(FF_E_NOMEM, "render workspace too small: need " + std::to_string(L.total) + " bytes");
            ws = (char*)workspace;
        } else {
            void* p = nullptr;
            if (ff_status s = library_scratch(kScratchRender, L.total, st, &p)) return s;
            ws = (char*)p;
        }
    }
    unsigned long long* cu = (unsigned long long*)n_culled;
    if (!accumulate) {
        const int64_t len = (int64_t)r->width * r->height * 3;
        const int64_t blocks = std::min<int64_t>((len + 1023) / 1024, 2048);
        hipLaunchKernelGGL(k_clear_img, dim3((unsigned)blocks), dim3(1024), 0, st, img, len, cu);
        if (hipError_t e = hipGetLastError()) return device_fail(e, "ff_render_image clear");
    }
    if (b->n == 0) return FF_OK;
    const size_t esz = prec_size(b->prec);
    auto col = [&](int ax) -> const char* {
        return ax >= 0 ? (const char*)b->state + (size_t)ax * b->ld * esz
                       : (const char*)b->pparams + (size_t)(-1 - ax) * b->ld * esz;
    };
    hipError_t e;
    if (b->prec == FF_FP64)
        e = run_render<double>((const double*)col(r->axis[0]), (const double*)col(r->axis[1]),
                               (const double*)col(r->axis[2]), b->n, a, L, ws, img, cu, st);
    else
        e = run_render<float>((const float*)col(r->axis[0]), (const float*)col(r->axis[1]),
                              (const float*)col(r->axis[2]), b->n, a, L, ws, img, cu, st);
    if (e != hipSuccess) return device_fail(e, "ff_render_image launch");
    return FF_OK;
}

}  // extern "C"
