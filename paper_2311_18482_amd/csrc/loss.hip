// Loss gradient of the full training step (gfx950): per view, the mean
// absolute error of the RGB and semantic channels against seeded targets plus
// lambda_u times the mean rendered uncertainty (Sec. 3.4.2 Eq. 11 regulariser
// L_u = sum R_u / (H W)). Writes dL/d(out) for every element and accumulates
// the loss value; one pass over out and target (HBM-bound).
#include "legs_internal.h"

namespace {

// Grid: y walks the (view, channel) planes, each contiguous in out, tgt and
// d_out, so the view, the channel, the weight and the kind of term are
// wave-uniform; x strides within a plane, four neighbouring elements per
// step where the plane and the three buffers are 16-byte aligned (vec), one
// at a time otherwise and for the plane's tail.
__device__ __forceinline__ float l1_grad(float d, float inv, float &lsum)
{
    lsum = fmaf(fabsf(d), inv, lsum);
    return d > 0.0f ? inv : (d < 0.0f ? -inv : 0.0f);
}

__global__ void __launch_bounds__(256)
k_l1(const float *__restrict__ out, const float *__restrict__ tgt, const legs_view *__restrict__ views,
     int n_views, int C, int n_fit, float lambda_u, int vec, float *__restrict__ d_out,
     float *__restrict__ loss)
{
    float lsum = 0.0f;
    const int64_t planes = (int64_t)n_views * C;
    const int64_t t0 = (int64_t)blockIdx.x * 256 + threadIdx.x, stride = (int64_t)gridDim.x * 256;
    for (int64_t pl = blockIdx.y; pl < planes; pl += gridDim.y) {
        const int v = (int)(pl / C), c = (int)(pl % C);
        const int64_t hw = (int64_t)views[v].cam.width * views[v].cam.height;
        const int64_t base = (int64_t)C * views[v].pixel_offset + (int64_t)c * hw;
        const float *o = out + base, *t = tgt + base;
        float *g = d_out + base;
        const int64_t n4 = vec && (base & 3) == 0 ? hw / 4 : 0;
        if (c < n_fit) {   // mean absolute error of a fitted channel
            const float inv = 1.0f / (float)((int64_t)n_fit * hw);
            for (int64_t i = t0; i < n4; i += stride) {
                const float4 a = reinterpret_cast<const float4 *>(o)[i];
                const float4 b = reinterpret_cast<const float4 *>(t)[i];
                float4 r;
                r.x = l1_grad(a.x - b.x, inv, lsum);
                r.y = l1_grad(a.y - b.y, inv, lsum);
                r.z = l1_grad(a.z - b.z, inv, lsum);
                r.w = l1_grad(a.w - b.w, inv, lsum);
                reinterpret_cast<float4 *>(g)[i] = r;
            }
            for (int64_t i = 4 * n4 + t0; i < hw; i += stride) g[i] = l1_grad(o[i] - t[i], inv, lsum);
        } else {           // lambda_u times the mean rendered uncertainty
            const float inv = lambda_u / (float)hw;
            for (int64_t i = t0; i < n4; i += stride) {
                const float4 a = reinterpret_cast<const float4 *>(o)[i];
                lsum = fmaf(a.x, inv, lsum);
                lsum = fmaf(a.y, inv, lsum);
                lsum = fmaf(a.z, inv, lsum);
                lsum = fmaf(a.w, inv, lsum);
                reinterpret_cast<float4 *>(g)[i] = make_float4(inv, inv, inv, inv);
            }
            for (int64_t i = 4 * n4 + t0; i < hw; i += stride) {
                lsum = fmaf(o[i], inv, lsum);
                g[i] = inv;
            }
        }
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
    if (total > 0 && n_views > 0 && C > 0) {
        // about 16 workgroups per CU in all (one loss atomic each), spread over
        // the planes; a plane's workgroups stride over it
        const int64_t planes = (int64_t)n_views * C;
        const int64_t gy = planes < 65535 ? planes : 65535;
        int64_t gx = ((total_pixels / n_views) / 4 + 255) / 256;
        const int64_t cap = (int64_t)ctx->num_cus * 16 / gy;
        if (gx > cap) gx = cap;
        if (gx < 1) gx = 1;
        const int vec = ((reinterpret_cast<uintptr_t>(out) | reinterpret_cast<uintptr_t>(target) |
                          reinterpret_cast<uintptr_t>(d_out)) & 15) == 0;
        hipLaunchKernelGGL(k_l1, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, s, out, target, views, n_views,
                           C, n_fit, lambda_u, vec, d_out, loss);
    }
    LEGS_CHECK_LAUNCH(ctx);
    return LEGS_OK;
}
