// EWA projection of Gaussians into every view and its derivative (gfx950).
//
// Forward (Sec. 3.1, Eq. 1 inputs p and Sigma): camera transform, 3D
// covariance Sigma = R S S^T R^T from the quaternion and exp(log_scale), the
// pinhole Jacobian J at the guard-band clamped mean, 2D covariance
// J W Sigma W^T J^T + lowpass I, conic, 2D mean, 3-sigma integer pixel box,
// tile rectangle and depth key. Everything runs in float64: the box and the
// depth key decide the tile lists bit for bit, and the kernel is HBM-bound
// (about 44 bytes read and 44 written per G-view against ~300 FP64 flops),
// so the double-rate cost of FP64 on CDNA4 is hidden behind memory.
//
// Layout: one thread per (Gaussian, view); grid (ceil(n / 256), n_views) so a
// block never straddles views and the per-block instance count written here
// is exactly what the emission kernel re-derives.
#include "legs_internal.h"

namespace {

struct ProjInter {
    double tx, ty, tz;
    double qn[4], qnorm;
    double Rq[3][3], s[3], M[3][3], Sig[3][3];
    double ux, uy;      // x/z and y/z after the guard-band clamp
    bool clx, cly;
    double J00, J02, J11, J12;
    double T[2][3];     // J * W
    double a, b, c;     // 2D covariance incl. low-pass
};

// Returns false when the Gaussian is culled before the 2D covariance exists.
__device__ __forceinline__ bool proj_core(const float *__restrict__ mean,
                                          const float *__restrict__ log_scale,
                                          const float *__restrict__ quat, int64_t g,
                                          const legs_camera &cam, const legs_opts &o,
                                          ProjInter &I)
{
    const double m0 = mean[3 * g + 0], m1 = mean[3 * g + 1], m2 = mean[3 * g + 2];
    const double *W = cam.R;
    I.tx = W[0] * m0 + W[1] * m1 + W[2] * m2 + cam.t[0];
    I.ty = W[3] * m0 + W[4] * m1 + W[5] * m2 + cam.t[1];
    I.tz = W[6] * m0 + W[7] * m1 + W[8] * m2 + cam.t[2];
    if (!(I.tz > o.z_near)) return false;
    const double q0 = quat[4 * g + 0], q1 = quat[4 * g + 1], q2 = quat[4 * g + 2],
                 q3 = quat[4 * g + 3];
    const double nn = q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3;
    if (!(nn > 0.0) || !isfinite(nn)) return false;
    const double l0 = log_scale[3 * g + 0], l1 = log_scale[3 * g + 1], l2 = log_scale[3 * g + 2];
    if (!isfinite(l0) || !isfinite(l1) || !isfinite(l2)) return false;
    I.qnorm = sqrt(nn);
    const double w = q0 / I.qnorm, x = q1 / I.qnorm, y = q2 / I.qnorm, z = q3 / I.qnorm;
    I.qn[0] = w; I.qn[1] = x; I.qn[2] = y; I.qn[3] = z;
    // rotation of a unit quaternion (w, x, y, z)
    I.Rq[0][0] = 1.0 - 2.0 * (y * y + z * z);
    I.Rq[0][1] = 2.0 * (x * y - w * z);
    I.Rq[0][2] = 2.0 * (x * z + w * y);
    I.Rq[1][0] = 2.0 * (x * y + w * z);
    I.Rq[1][1] = 1.0 - 2.0 * (x * x + z * z);
    I.Rq[1][2] = 2.0 * (y * z - w * x);
    I.Rq[2][0] = 2.0 * (x * z - w * y);
    I.Rq[2][1] = 2.0 * (y * z + w * x);
    I.Rq[2][2] = 1.0 - 2.0 * (x * x + y * y);
    I.s[0] = exp(l0); I.s[1] = exp(l1); I.s[2] = exp(l2);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) I.M[i][j] = I.Rq[i][j] * I.s[j];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            I.Sig[i][j] = I.M[i][0] * I.M[j][0] + I.M[i][1] * I.M[j][1] + I.M[i][2] * I.M[j][2];
    const double limx = o.guard * (0.5 * cam.width / cam.fx);
    const double limy = o.guard * (0.5 * cam.height / cam.fy);
    const double u = I.tx / I.tz, v = I.ty / I.tz;
    I.ux = u; I.uy = v; I.clx = false; I.cly = false;
    if (u < -limx) { I.ux = -limx; I.clx = true; } else if (u > limx) { I.ux = limx; I.clx = true; }
    if (v < -limy) { I.uy = -limy; I.cly = true; } else if (v > limy) { I.uy = limy; I.cly = true; }
    const double tz2 = I.tz * I.tz;
    I.J00 = cam.fx / I.tz;
    I.J02 = -cam.fx * (I.ux * I.tz) / tz2;
    I.J11 = cam.fy / I.tz;
    I.J12 = -cam.fy * (I.uy * I.tz) / tz2;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        I.T[0][k] = I.J00 * W[k] + I.J02 * W[6 + k];
        I.T[1][k] = I.J11 * W[3 + k] + I.J12 * W[6 + k];
    }
    double TS[2][3];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k)
            TS[r][k] = I.T[r][0] * I.Sig[0][k] + I.T[r][1] * I.Sig[1][k] + I.T[r][2] * I.Sig[2][k];
    const double s00 = TS[0][0] * I.T[0][0] + TS[0][1] * I.T[0][1] + TS[0][2] * I.T[0][2];
    const double s01 = TS[0][0] * I.T[1][0] + TS[0][1] * I.T[1][1] + TS[0][2] * I.T[1][2];
    const double s11 = TS[1][0] * I.T[1][0] + TS[1][1] * I.T[1][1] + TS[1][2] * I.T[1][2];
    I.a = s00 + o.lowpass;
    I.b = s01;
    I.c = s11 + o.lowpass;
    return true;
}

struct ProjOut {
    double mx, my;
    double A, B, C, sig;
    int x0, x1, y0, y1;
    uint32_t ntiles;
    float depth;
};

__device__ __forceinline__ bool proj_finish(const ProjInter &I, float omega,
                                            const legs_camera &cam, const legs_opts &o,
                                            ProjOut &P)
{
    const double det = I.a * I.c - I.b * I.b;
    if (!(det > 0.0) || !isfinite(det)) return false;
    P.A = I.c / det;
    P.B = -I.b / det;
    P.C = I.a / det;
    P.mx = cam.fx * I.tx / I.tz + cam.cx;
    P.my = cam.fy * I.ty / I.tz + cam.cy;
    const double half = 0.5 * (I.a - I.c);
    const double lam = 0.5 * (I.a + I.c) + sqrt(half * half + I.b * I.b);
    if (!isfinite(lam) || !isfinite(P.mx) || !isfinite(P.my)) return false;
    const double r = ceil(3.0 * sqrt(lam));
    double x0 = ceil(P.mx - r - 0.5), x1 = floor(P.mx + r - 0.5);
    double y0 = ceil(P.my - r - 0.5), y1 = floor(P.my + r - 0.5);
    x0 = x0 < 0.0 ? 0.0 : x0;
    y0 = y0 < 0.0 ? 0.0 : y0;
    x1 = x1 > (double)(cam.width - 1) ? (double)(cam.width - 1) : x1;
    y1 = y1 > (double)(cam.height - 1) ? (double)(cam.height - 1) : y1;
    if (!(x0 <= x1) || !(y0 <= y1)) return false;
    P.x0 = (int)x0; P.x1 = (int)x1; P.y0 = (int)y0; P.y1 = (int)y1;
    const int T = o.tile;
    P.ntiles = (uint32_t)((P.x1 / T - P.x0 / T + 1) * (P.y1 / T - P.y0 / T + 1));
    P.sig = 1.0 / (1.0 + exp(-(double)omega));
    P.depth = (float)I.tz;
    return true;
}

__global__ void __launch_bounds__(LEGS_PROJ_BLOCK)
k_project(const float *__restrict__ mean, const float *__restrict__ log_scale,
          const float *__restrict__ quat, const float *__restrict__ omega, int64_t n,
          const legs_view *__restrict__ views, legs_opts o, double2 *__restrict__ mean2d,
          float4 *__restrict__ conic, int4 *__restrict__ box, float *__restrict__ depth,
          uint32_t *__restrict__ ntiles, uint64_t *__restrict__ block_counts)
{
    const int v = blockIdx.y;
    const int64_t g = (int64_t)blockIdx.x * LEGS_PROJ_BLOCK + threadIdx.x;
    uint32_t cnt = 0;
    if (g < n) {
        const legs_camera cam = views[v].cam;
        const int64_t gv = (int64_t)v * n + g;
        ProjInter I;
        ProjOut P;
        if (proj_core(mean, log_scale, quat, g, cam, o, I) && proj_finish(I, omega[g], cam, o, P)) {
            mean2d[gv] = make_double2(P.mx, P.my);
            conic[gv] = make_float4((float)P.A, (float)P.B, (float)P.C, (float)P.sig);
            box[gv] = make_int4(P.x0, P.x1, P.y0, P.y1);
            depth[gv] = P.depth;
            ntiles[gv] = P.ntiles;
            cnt = P.ntiles;
        } else {
            mean2d[gv] = make_double2(0.0, 0.0);
            conic[gv] = make_float4(0.f, 0.f, 0.f, 0.f);
            box[gv] = make_int4(0, -1, 0, -1);
            depth[gv] = 0.f;
            ntiles[gv] = 0;
        }
    }
    // block total of tile counts (the instance scan's first level)
    __shared__ uint64_t s_part[LEGS_PROJ_BLOCK / LEGS_WAVE];
    uint64_t c = cnt;
#pragma unroll
    for (int off = LEGS_WAVE / 2; off > 0; off >>= 1) c += __shfl_down(c, off, LEGS_WAVE);
    if (legs_lane() == 0) s_part[threadIdx.x / LEGS_WAVE] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int w = 0; w < LEGS_PROJ_BLOCK / LEGS_WAVE; ++w) t += s_part[w];
        block_counts[(int64_t)v * gridDim.x + blockIdx.x] = t;
    }
}

// ---- backward ---------------------------------------------------------------

// Whether view v of Gaussian g received a gradient (it has tiles and a
// non-zero screen-space gradient); the chain rule skips the other views.
__device__ __forceinline__ bool view_has_grad(const uint32_t *__restrict__ ntiles,
                                              const float *__restrict__ grad2d, int64_t gv)
{
    if (ntiles[gv] == 0) return false;
    const float4 ga = *reinterpret_cast<const float4 *>(grad2d + 8 * gv);
    const float2 gb = *reinterpret_cast<const float2 *>(grad2d + 8 * gv + 4);
    return !(ga.x == 0.0f && ga.y == 0.0f && ga.z == 0.0f && ga.w == 0.0f && gb.x == 0.0f && gb.y == 0.0f);
}

// Chain rule of one Gaussian, summed over its views.
__device__ __forceinline__ void project_backward_one(
    const float *__restrict__ mean, const float *__restrict__ log_scale, const float *__restrict__ quat,
    const float *__restrict__ omega, int64_t n, const legs_view *__restrict__ views, int32_t n_views,
    const legs_opts &o, const uint32_t *__restrict__ ntiles, const float *__restrict__ grad2d,
    float *__restrict__ d_mean, float *__restrict__ d_log_scale, float *__restrict__ d_quat,
    float *__restrict__ d_omega, int64_t g)
{
    double dmu[3] = {0, 0, 0}, dls[3] = {0, 0, 0}, dq[4] = {0, 0, 0, 0}, dom = 0.0;
    bool any = false;
    for (int v = 0; v < n_views; ++v) {
        const int64_t gv = (int64_t)v * n + g;
        if (ntiles[gv] == 0) continue;
        const float4 ga = *reinterpret_cast<const float4 *>(grad2d + 8 * gv);
        const float2 gb = *reinterpret_cast<const float2 *>(grad2d + 8 * gv + 4);
        const double gmx = ga.x, gmy = ga.y, gA = ga.z, gB = ga.w, gC = gb.x, gsig = gb.y;
        if (gmx == 0.0 && gmy == 0.0 && gA == 0.0 && gB == 0.0 && gC == 0.0 && gsig == 0.0)
            continue;
        const legs_camera cam = views[v].cam;
        ProjInter I;
        if (!proj_core(mean, log_scale, quat, g, cam, o, I)) continue;
        any = true;
        // opacity = sigmoid(omega)
        const double sg = 1.0 / (1.0 + exp(-(double)omega[g]));
        dom += gsig * sg * (1.0 - sg);
        // conic = inverse of (a b; b c)
        const double a = I.a, b = I.b, c = I.c;
        const double det = a * c - b * b, id = 1.0 / det, id2 = id * id;
        const double da = -gA * c * c * id2 + gB * b * c * id2 + gC * (id - a * c * id2);
        const double db = 2.0 * gA * b * c * id2 - gB * (id + 2.0 * b * b * id2) + 2.0 * gC * a * b * id2;
        const double dc = gA * (id - a * c * id2) + gB * a * b * id2 - gC * a * a * id2;
        // symmetric gradient of the 2D covariance
        const double G00 = da, G01 = 0.5 * db, G11 = dc;
        // Sigma' = T Sigma T^T: dT = 2 G T Sigma; dSigma = T^T G T
        double TS[2][3];
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int k = 0; k < 3; ++k)
                TS[r][k] = I.T[r][0] * I.Sig[0][k] + I.T[r][1] * I.Sig[1][k] + I.T[r][2] * I.Sig[2][k];
        double dT[2][3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            dT[0][k] = 2.0 * (G00 * TS[0][k] + G01 * TS[1][k]);
            dT[1][k] = 2.0 * (G01 * TS[0][k] + G11 * TS[1][k]);
        }
        double GT[2][3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            GT[0][k] = G00 * I.T[0][k] + G01 * I.T[1][k];
            GT[1][k] = G01 * I.T[0][k] + G11 * I.T[1][k];
        }
        double dS[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int k = 0; k < 3; ++k) dS[i][k] = I.T[0][i] * GT[0][k] + I.T[1][i] * GT[1][k];
        // T = J W, J = [[J00, 0, J02], [0, J11, J12]]
        const double *W = cam.R;
        const double dJ00 = dT[0][0] * W[0] + dT[0][1] * W[1] + dT[0][2] * W[2];
        const double dJ02 = dT[0][0] * W[6] + dT[0][1] * W[7] + dT[0][2] * W[8];
        const double dJ11 = dT[1][0] * W[3] + dT[1][1] * W[4] + dT[1][2] * W[5];
        const double dJ12 = dT[1][0] * W[6] + dT[1][1] * W[7] + dT[1][2] * W[8];
        const double tz = I.tz, tz2 = tz * tz, tz3 = tz2 * tz;
        double dtx = 0.0, dty = 0.0, dtz = 0.0;
        dtz -= dJ00 * cam.fx / tz2 + dJ11 * cam.fy / tz2;
        if (I.clx) dtz += dJ02 * cam.fx * I.ux / tz2;
        else { dtx -= dJ02 * cam.fx / tz2; dtz += dJ02 * 2.0 * cam.fx * I.tx / tz3; }
        if (I.cly) dtz += dJ12 * cam.fy * I.uy / tz2;
        else { dty -= dJ12 * cam.fy / tz2; dtz += dJ12 * 2.0 * cam.fy * I.ty / tz3; }
        // 2D mean
        dtx += gmx * cam.fx / tz;
        dty += gmy * cam.fy / tz;
        dtz -= (gmx * cam.fx * I.tx + gmy * cam.fy * I.ty) / tz2;
#pragma unroll
        for (int k = 0; k < 3; ++k) dmu[k] += W[k] * dtx + W[3 + k] * dty + W[6 + k] * dtz;
        // Sigma = M M^T, M = Rq diag(s)
        double dR[3][3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double dsj = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double dM = 2.0 * (dS[i][0] * I.M[0][j] + dS[i][1] * I.M[1][j] + dS[i][2] * I.M[2][j]);
                dR[i][j] = dM * I.s[j];
                dsj += dM * I.Rq[i][j];
            }
            dls[j] += dsj * I.s[j];
        }
        const double w = I.qn[0], x = I.qn[1], y = I.qn[2], z = I.qn[3];
        const double r01 = dR[0][1], r02 = dR[0][2], r10 = dR[1][0], r12 = dR[1][2],
                     r20 = dR[2][0], r21 = dR[2][1];
        double gq[4];
        gq[0] = 2.0 * (x * (r21 - r12) + y * (r02 - r20) + z * (r10 - r01));
        gq[1] = 2.0 * (y * (r01 + r10) + z * (r02 + r20) + w * (r21 - r12)) - 4.0 * x * (dR[1][1] + dR[2][2]);
        gq[2] = 2.0 * (x * (r01 + r10) + z * (r12 + r21) + w * (r02 - r20)) - 4.0 * y * (dR[0][0] + dR[2][2]);
        gq[3] = 2.0 * (x * (r02 + r20) + y * (r12 + r21) + w * (r10 - r01)) - 4.0 * z * (dR[0][0] + dR[1][1]);
        const double dot = w * gq[0] + x * gq[1] + y * gq[2] + z * gq[3];
#pragma unroll
        for (int k = 0; k < 4; ++k) dq[k] += (gq[k] - I.qn[k] * dot) / I.qnorm;
    }
    if (!any) return;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        d_mean[3 * g + k] += (float)dmu[k];
        d_log_scale[3 * g + k] += (float)dls[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) d_quat[4 * g + k] += (float)dq[k];
    d_omega[g] += (float)dom;
}

constexpr int PB_PER_THREAD = 8;   // Gaussians checked per thread

// Most Gaussians of a dense scene receive no gradient (culled or hidden), so
// each workgroup first queues, in LDS, those of its 256 x PB_PER_THREAD that
// have a view with a gradient (one ballot and one LDS atomic per wave), then
// runs the chain rule over the queue with every lane busy.
__global__ void __launch_bounds__(256)
k_project_backward(const float *__restrict__ mean, const float *__restrict__ log_scale,
                   const float *__restrict__ quat, const float *__restrict__ omega, int64_t n,
                   const legs_view *__restrict__ views, int32_t n_views, legs_opts o,
                   const uint32_t *__restrict__ ntiles, const float *__restrict__ grad2d,
                   float *__restrict__ d_mean, float *__restrict__ d_log_scale,
                   float *__restrict__ d_quat, float *__restrict__ d_omega)
{
    __shared__ uint32_t s_q[256 * PB_PER_THREAD];
    __shared__ uint32_t s_n;
    const int tid = threadIdx.x, lane = legs_lane();
    if (tid == 0) s_n = 0;
    __syncthreads();
    const int64_t g0 = (int64_t)blockIdx.x * 256 * PB_PER_THREAD;
#pragma unroll
    for (int i = 0; i < PB_PER_THREAD; ++i) {
        const int64_t g = g0 + (int64_t)i * 256 + tid;
        bool act = false;
        if (g < n)
            for (int v = 0; v < n_views && !act; ++v) act = view_has_grad(ntiles, grad2d, (int64_t)v * n + g);
        const uint64_t bal = legs_ballot(act);
        uint32_t base = 0;
        if (lane == 0 && bal) base = atomicAdd(&s_n, (uint32_t)__popcll(bal));
        base = (uint32_t)__shfl((int)base, 0, LEGS_WAVE);
        if (act)
            s_q[base + __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u))] =
                (uint32_t)(g - g0);
    }
    __syncthreads();
    const uint32_t cnt = s_n;
    for (uint32_t k = tid; k < cnt; k += 256)
        project_backward_one(mean, log_scale, quat, omega, n, views, n_views, o, ntiles, grad2d, d_mean,
                             d_log_scale, d_quat, d_omega, g0 + s_q[k]);
}

} // namespace

int32_t legs_launch_project(legs_ctx *ctx, const float *mean, const float *log_scale,
                            const float *quat, const float *opacity_logit, int64_t n,
                            const legs_view *views, int32_t n_views, const legs_opts *o,
                            legs_projected *out, hipStream_t s)
{
    if (n == 0) return LEGS_OK;
    const int64_t bx = (n + LEGS_PROJ_BLOCK - 1) / LEGS_PROJ_BLOCK;
    if (bx > 0x7fffffffLL || n_views > 65535)
        return legs_set_error(ctx, LEGS_ERR_ARG, "legs_project: grid too large");
    dim3 grid((unsigned)bx, (unsigned)n_views);
    hipLaunchKernelGGL(k_project, grid, dim3(LEGS_PROJ_BLOCK), 0, s, mean, log_scale, quat,
                       opacity_logit, n, views, *o, reinterpret_cast<double2 *>(out->mean2d),
                       reinterpret_cast<float4 *>(out->conic), reinterpret_cast<int4 *>(out->box),
                       out->depth, out->ntiles, out->block_offsets);
    LEGS_CHECK_LAUNCH(ctx);
    return LEGS_OK;
}

int32_t legs_launch_project_backward(legs_ctx *ctx, const float *mean, const float *log_scale,
                                     const float *quat, const float *opacity_logit, int64_t n,
                                     const legs_view *views, int32_t n_views, const legs_opts *o,
                                     const legs_projected *proj, const float *grad2d,
                                     float *d_mean, float *d_log_scale, float *d_quat,
                                     float *d_opacity_logit, hipStream_t s)
{
    if (n == 0) return LEGS_OK;
    const int64_t blocks = (n + 256 * PB_PER_THREAD - 1) / (256 * PB_PER_THREAD);
    hipLaunchKernelGGL(k_project_backward, dim3((unsigned)blocks), dim3(256), 0, s, mean,
                       log_scale, quat, opacity_logit, n, views, n_views, *o, proj->ntiles, grad2d,
                       d_mean, d_log_scale, d_quat, d_opacity_logit);
    LEGS_CHECK_LAUNCH(ctx);
    return LEGS_OK;
}
