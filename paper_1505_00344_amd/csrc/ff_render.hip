// ff_render.hip — particle image (Appendix A "Render Technique"; Appendix A.1:
// the vertex shader applies the model-view matrix, the geometry shader the
// view-projection matrix — orthographic for 2D, perspective for 3D — and
// emits a square sprite; the fragment shader gives each covered pixel an
// intensity that falls off with the distance from the sprite's centre and a
// colour that is fixed or linear in the particle's position; blending adds
// source*alpha into the pixel).
//
// One thread per particle, all geometry in double precision:
//   c = M (a0, a1, a2, 1) with M = projection * view * model (row-major 4x4);
//   culled if c3 <= 0 or some c_i / c3 (i < 3) is outside [-1, 1] or NaN;
//   px = (c0/c3 + 1) W / 2, py = (1 - c1/c3) H / 2;
//   rgb_k = clamp(base_k + sum_i grad[k][i] (a_i - origin_i), 0, 1);
//   radius 0: pixel (floor px, floor py) gets w = weight; radius R: pixels
//   floor(px - R - 1) .. floor(px + R + 1) (and in y) whose centre is at
//   distance d < R + 1 get w = weight (1 - d / (R + 1))^2;
//   img[(iy W + ix) 3 + k] += rint(256 w rgb_k)   (uint32 atomics).
// Fixed-point integer accumulation makes the image exact and independent of
// the order in which particles are added.
#include <algorithm>
#include <cmath>

#include "ff_internal.h"

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

template <typename R>
__global__ void __launch_bounds__(256) k_render(const R* a0p, const R* a1p, const R* a2p, int64_t n, RenderArgs r,
                                                uint32_t* img, unsigned long long* culled) {
    __shared__ unsigned int s_cull;
    if (threadIdx.x == 0) s_cull = 0u;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const double a[3] = {(double)a0p[i], (double)a1p[i], (double)a2p[i]};
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
        if (!keep) {
            atomicAdd(&s_cull, 1u);
        } else {
            const int64_t W = r.width, H = r.height;
            const double px = (ndc[0] + 1.0) * (double)W / 2.0;
            const double py = (1.0 - ndc[1]) * (double)H / 2.0;
            double rgb[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                double v = r.base[k];
#pragma unroll
                for (int j = 0; j < 3; ++j) v += r.grad[3 * k + j] * (a[j] - r.origin[j]);
                rgb[k] = fmin(fmax(v, 0.0), 1.0);
            }
            const double reach = r.radius + 1.0;
            int64_t x0 = (int64_t)floor(px), x1 = x0, y0 = (int64_t)floor(py), y1 = y0;
            if (r.radius > 0) {
                x0 = (int64_t)floor(px - reach);
                x1 = (int64_t)floor(px + reach);
                y0 = (int64_t)floor(py - reach);
                y1 = (int64_t)floor(py + reach);
            }
            for (int64_t iy = y0; iy <= y1; ++iy) {
                for (int64_t ix = x0; ix <= x1; ++ix) {
                    if (ix < 0 || ix >= W || iy < 0 || iy >= H) continue;
                    double w = r.weight;
                    if (r.radius > 0) {
                        const double dx = ((double)ix + 0.5) - px, dy = ((double)iy + 0.5) - py;
                        const double d = sqrt(dx * dx + dy * dy);
                        if (!(d < reach)) continue;
                        const double f = 1.0 - d / reach;
                        w = r.weight * (f * f);
                    }
                    uint32_t* pix = img + (iy * W + ix) * 3;
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const uint32_t q = (uint32_t)rint(256.0 * (w * rgb[k]));
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

}  // namespace

}  // namespace ff

using namespace ff;

extern "C" ff_status ff_render_image(ff_system_t sys, const ff_batch* b, const ff_render* r, uint32_t* img,
                                     uint64_t* n_culled, int32_t accumulate, void* stream) {
    set_error("");
    if (ff_status s = check_system(sys)) return s;
    if (ff_status s = check_batch(sys, b, false)) return s;
    if (!r) return fail(FF_E_INVALID, "render description is NULL");
    if (b->n > 0 && !b->state) return fail(FF_E_INVALID, "batch.state is NULL");
    auto axis_ok = [&](int a) { return (a >= 0 && a < sys->dim) || (a < 0 && -1 - a < b->n_pp); };
    for (int i = 0; i < 3; ++i)
        if (!axis_ok(r->axis[i])) return fail(FF_E_INVALID, "render axis must be a state component or -1 - k");
    if (r->width <= 0 || r->height <= 0) return fail(FF_E_INVALID, "image size must be positive");
    if ((int64_t)r->width * r->height > (int64_t)1 << 28) return fail(FF_E_UNSUPPORTED, "image larger than 2^28 pixels");
    if (r->radius < 0 || r->radius > 64) return fail(FF_E_INVALID, "sprite radius must be in [0, 64]");
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
    const unsigned grid = (unsigned)((b->n + 255) / 256);
    if (b->prec == FF_FP64)
        hipLaunchKernelGGL((k_render<double>), dim3(grid), dim3(256), 0, st, (const double*)col(r->axis[0]),
                           (const double*)col(r->axis[1]), (const double*)col(r->axis[2]), b->n, a, img, cu);
    else
        hipLaunchKernelGGL((k_render<float>), dim3(grid), dim3(256), 0, st, (const float*)col(r->axis[0]),
                           (const float*)col(r->axis[1]), (const float*)col(r->axis[2]), b->n, a, img, cu);
    if (hipError_t e = hipGetLastError()) return device_fail(e, "ff_render_image launch");
    return FF_OK;
}
