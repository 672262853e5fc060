// Loss gradient of the full training step (gfx950): per view, the mean
// absolute error of the RGB and semantic channels against seeded targets plus
// lambda_u times the mean rendered uncertainty (Sec. 3.4.2 Eq. 11 regulariser
// L_u = sum R_u / (H W)). Writes dL/d(out) for every element and accumulates
// the loss value; one pass over out and target (HBM-bound).
#include "legs_internal.h"

namespace {

__global__ void __launch_bounds__(256)
k_l1(const float *__restrict__ out, const float *__restrict__ tgt, const legs_view *__restrict__ views,
     int n_views, int C, int n_fit, float lambda_u, int64_t total, float *__restrict__ d_out,
     float *__restrict__ loss)
{
    float lsum = 0.0f;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        // view holding element e: last v with C * pixel_offset(v) <= e
        int lo = 0, hi = n_views - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if ((int64_t)C * views[mid].pixel_offset <= e) lo = mid; else hi = mid - 1;
        }
        const int64_t hw = (int64_t)views[lo].cam.width * views[lo].cam.height;
        const int64_t local = e - (int64_t)C * views[lo].pixel_offset;
        const int c = (int)(local / hw);
        const float o = out[e];
        float g, l;
        if (c < n_fit) {
            const float inv = 1.0f / (float)((int64_t)n_fit * hw);
            const float d = o - tgt[e];
            g = d > 0.0f ? inv : (d < 0.0f ? -inv : 0.0f);
            l = fabsf(d) * inv;
        } else {
            const float inv = lambda_u / (float)hw;
            g = inv;
            l = o * inv;
        }
        d_out[e] = g;
        lsum += l;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, LEGS_WAVE);
    __shared__ float s_w[4];
    if (legs_lane() == 0) s_w[threadIdx.x / LEGS_WAVE] = lsum;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(loss, s_w[0] + s_w[1] + s_w[2] + s_w[3]);
}

__global__ void k_zero1(float *p) { *p = 0.0f; }

// Zero n 32-bit words (16-byte stores where aligned; a kernel, so it records
// as a kernel node under graph capture).
__global__ void __launch_bounds__(256)
k_clear(uint32_t *__restrict__ p, int64_t n)
{
    const int64_t n4 = (reinterpret_cast<uintptr_t>(p) & 15) == 0 ? n / 4 : 0;
    uint4 *q = reinterpret_cast<uint4 *>(p);
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += stride) q[i] = make_uint4(0, 0, 0, 0);
    for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) p[i] = 0u;
}

} // namespace

int32_t legs_launch_clear(legs_ctx *ctx, void *dev, int64_t words, hipStream_t s)
{
    if (words <= 0) return LEGS_OK;
    int64_t g = (words / 4 + 255) / 256;
    const int64_t cap = (int64_t)ctx->num_cus * 8;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_clear, dim3((unsigned)g), dim3(256), 0, s, static_cast<uint32_t *>(dev), words);
    LEGS_CHECK_LAUNCH(ctx);
    return LEGS_OK;
}

int32_t legs_launch_l1_loss_grad(legs_ctx *ctx, const float *out, const float *target,
                                 const legs_view *views, int32_t n_views, int64_t total_pixels,
                                 int32_t C, int32_t n_fit, float lambda_u, float *d_out,
                                 float *loss, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero1, dim3(1), dim3(1), 0, s, loss);
    const int64_t total = (int64_t)C * total_pixels;
    if (total > 0) {
        int64_t g = (total + 255) / 256;
        const int64_t cap = (int64_t)ctx->num_cus * 16;
        if (g > cap) g = cap;
        hipLaunchKernelGGL(k_l1, dim3((unsigned)g), dim3(256), 0, s, out, target, views, n_views, C,
                           n_fit, lambda_u, total, d_out, loss);
    }
    LEGS_CHECK_LAUNCH(ctx);
    return LEGS_OK;
}
