/*
 * legs_oracle.c -- plain FP64 CPU oracle for the splatting path of
 * Language Embedded 3D Gaussians (arXiv 2311.18482).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, includes or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark load it. It shares no header, helper or constant with the HIP
 * path: every formula below is written out again from its definition.
 *
 * What it computes (all arithmetic in double on float inputs promoted exactly):
 *   - the renderer I = R(p, Sigma, c, alpha; p_cam) of Sec. 3.1, Eq. 1, with the
 *     extra blended channels of Sec. 3.4.1 (compact semantic feature s_G, the
 *     map R_s of Eq. 8) and Sec. 3.4.2 (uncertainty u, the map R_u of Eq. 10/11);
 *   - the tile overlap lists (tile, depth, id) used by a tile rasteriser;
 *   - the gradient of a loss sum(G * out) with respect to every per-Gaussian
 *     parameter, for the "differentiable rendering and gradient descent" of
 *     Sec. 3.1.
 * The paper gives the renderer only as Eq. 1 ("rasterization and alpha
 * blending", Sec. 3.4.1). Projection, footprint, thresholds and the
 * parameterisation below are the readings listed in the design notes
 * (EWA projection with a screen-space low-pass, 3-sigma integer pixel box,
 * alpha = min(0.99, sigmoid(omega) * exp(power)), skip alpha < 1/255,
 * stop when T * (1 - alpha) < 1e-4 without blending, background 0).
 *
 * Parity pins: see tests/test_oracle_pins.py (closed forms, brute force over
 * all Gaussians, finite differences, invariants).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- plain structs (mirrored by ctypes in oracle/oracle.py) ---------------- */

typedef struct {
    int32_t W, H;
    double fx, fy, cx, cy;
    double R[9]; /* world -> camera rotation, row-major */
    double t[3];
} ocam_t;

typedef struct {
    double lowpass;   /* h added to the diagonal of the 2D covariance (px^2) */
    double z_near;    /* cull when camera-space z <= z_near */
    double guard;     /* guard-band factor for the Jacobian clamp */
    double alpha_max; /* 0.99 */
    double alpha_min; /* 1/255 */
    double t_min;     /* 1e-4 */
    double eps_alpha; /* relative margin below which a skip decision is ambiguous */
    double eps_t;     /* relative margin below which a stop decision is ambiguous */
    double eps_alpha_mag; /* added to eps_alpha per unit of the exponent's magnitude sum
                             (0.5 |A dx^2| + |B dx dy| + 0.5 |C dy^2|): rounding the
                             terms of a strongly cancelling exponent moves alpha by
                             that sum times a few ulps, not by |power| times them */
    int32_t tile;     /* tile edge in pixels */
    int32_t pad;
} oopts_t;

typedef struct {
    int64_t ntiles;           /* tiles touched (0 when culled) */
    double tx, ty, tz;        /* camera-space mean */
    double mx, my;            /* 2D mean, pixels */
    double a, b, c;           /* 2D covariance incl. low-pass */
    double A, B, C;           /* conic = inverse of (a b; b c) */
    double sig;               /* opacity sigmoid(omega) */
    double lam, radius;       /* largest eigenvalue, ceil(3 sqrt(lam)) */
    int32_t valid;
    int32_t clampx, clampy;   /* guard-band clamp active on x / y */
    int32_t x0, x1, y0, y1;   /* inclusive pixel box */
    int32_t tx0, tx1, ty0, ty1; /* inclusive tile rectangle */
    float depth32;            /* tz rounded to float (sort key) */
} oproj_t;

/* ---- projection (Eq. 1 inputs p and Sigma to the screen) -------------------- */

static void quat_to_rot(const double q[4], double Rq[3][3])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    Rq[0][0] = 1.0 - 2.0 * (y * y + z * z);
    Rq[0][1] = 2.0 * (x * y - w * z);
    Rq[0][2] = 2.0 * (x * z + w * y);
    Rq[1][0] = 2.0 * (x * y + w * z);
    Rq[1][1] = 1.0 - 2.0 * (x * x + z * z);
    Rq[1][2] = 2.0 * (y * z - w * x);
    Rq[2][0] = 2.0 * (x * z - w * y);
    Rq[2][1] = 2.0 * (y * z + w * x);
    Rq[2][2] = 1.0 - 2.0 * (x * x + y * y);
}

/* Intermediates shared by the forward projection and its derivative. */
typedef struct {
    int ok;
    double tx, ty, tz;
    double qn[4], qnorm;
    double Rq[3][3], s[3], M[3][3], Sig[3][3];
    double limx, limy, ux, uy;  /* clamped tx/tz, ty/tz */
    int clx, cly;
    double J00, J02, J11, J12;
    double T[2][3];             /* J * W */
    double a, b, c;
} oproj_int_t;

static void project_intermediates(const double mu[3], const double ls[3], const double q[4],
                                  const ocam_t *cam, const oopts_t *o, oproj_int_t *I)
{
    const double *R = cam->R, *tv = cam->t;
    memset(I, 0, sizeof *I);
    I->tx = R[0] * mu[0] + R[1] * mu[1] + R[2] * mu[2] + tv[0];
    I->ty = R[3] * mu[0] + R[4] * mu[1] + R[5] * mu[2] + tv[1];
    I->tz = R[6] * mu[0] + R[7] * mu[1] + R[8] * mu[2] + tv[2];
    if (!(I->tz > o->z_near)) return;
    double n2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    if (!(n2 > 0.0) || !isfinite(n2)) return;
    if (!isfinite(ls[0]) || !isfinite(ls[1]) || !isfinite(ls[2])) return;
    I->qnorm = sqrt(n2);
    for (int k = 0; k < 4; ++k) I->qn[k] = q[k] / I->qnorm;
    quat_to_rot(I->qn, I->Rq);
    for (int j = 0; j < 3; ++j) I->s[j] = exp(ls[j]);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) I->M[i][j] = I->Rq[i][j] * I->s[j];
    /* Sigma = M M^T = R S S^T R^T */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            I->Sig[i][j] = I->M[i][0] * I->M[j][0] + I->M[i][1] * I->M[j][1] + I->M[i][2] * I->M[j][2];
    /* Jacobian of the pinhole map at the (guard-band clamped) mean */
    I->limx = o->guard * (0.5 * cam->W / cam->fx);
    I->limy = o->guard * (0.5 * cam->H / cam->fy);
    double u = I->tx / I->tz, v = I->ty / I->tz;
    I->ux = u; I->uy = v;
    if (u < -I->limx) { I->ux = -I->limx; I->clx = 1; }
    else if (u > I->limx) { I->ux = I->limx; I->clx = 1; }
    if (v < -I->limy) { I->uy = -I->limy; I->cly = 1; }
    else if (v > I->limy) { I->uy = I->limy; I->cly = 1; }
    const double txc = I->ux * I->tz, tyc = I->uy * I->tz;
    const double tz2 = I->tz * I->tz;
    I->J00 = cam->fx / I->tz;
    I->J02 = -cam->fx * txc / tz2;
    I->J11 = cam->fy / I->tz;
    I->J12 = -cam->fy * tyc / tz2;
    for (int k = 0; k < 3; ++k) {
        I->T[0][k] = I->J00 * R[0 * 3 + k] + I->J02 * R[2 * 3 + k];
        I->T[1][k] = I->J11 * R[1 * 3 + k] + I->J12 * R[2 * 3 + k];
    }
    /* Sigma' = T Sigma T^T + h I */
    double S2[2][2];
    for (int r = 0; r < 2; ++r)
        for (int cc = 0; cc < 2; ++cc) {
            double acc = 0.0;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) acc += I->T[r][i] * I->Sig[i][j] * I->T[cc][j];
            S2[r][cc] = acc;
        }
    I->a = S2[0][0] + o->lowpass;
    I->b = 0.5 * (S2[0][1] + S2[1][0]);
    I->c = S2[1][1] + o->lowpass;
    I->ok = 1;
}

static void project_one(const double mu[3], const double ls[3], const double q[4], double omega,
                        const ocam_t *cam, const oopts_t *o, oproj_t *p)
{
    oproj_int_t I;
    memset(p, 0, sizeof *p);
    project_intermediates(mu, ls, q, cam, o, &I);
    p->tx = I.tx; p->ty = I.ty; p->tz = I.tz;
    if (!I.ok) return;
    const double a = I.a, b = I.b, c = I.c;
    const double det = a * c - b * b;
    if (!(det > 0.0) || !isfinite(det)) return;
    p->a = a; p->b = b; p->c = c;
    p->A = c / det; p->B = -b / det; p->C = a / det;
    p->mx = cam->fx * I.tx / I.tz + cam->cx;
    p->my = cam->fy * I.ty / I.tz + cam->cy;
    const double half = 0.5 * (a - c);
    p->lam = 0.5 * (a + c) + sqrt(half * half + b * b);
    if (!isfinite(p->lam) || !isfinite(p->mx) || !isfinite(p->my)) return;
    p->radius = ceil(3.0 * sqrt(p->lam));
    /* pixel i is inside iff |i + 1/2 - mx| <= radius */
    double x0 = ceil(p->mx - p->radius - 0.5), x1 = floor(p->mx + p->radius - 0.5);
    double y0 = ceil(p->my - p->radius - 0.5), y1 = floor(p->my + p->radius - 0.5);
    if (x0 < 0.0) x0 = 0.0;
    if (y0 < 0.0) y0 = 0.0;
    if (x1 > cam->W - 1) x1 = cam->W - 1;
    if (y1 > cam->H - 1) y1 = cam->H - 1;
    if (!(x0 <= x1) || !(y0 <= y1)) return;
    p->x0 = (int32_t)x0; p->x1 = (int32_t)x1; p->y0 = (int32_t)y0; p->y1 = (int32_t)y1;
    p->tx0 = p->x0 / o->tile; p->tx1 = p->x1 / o->tile;
    p->ty0 = p->y0 / o->tile; p->ty1 = p->y1 / o->tile;
    p->ntiles = (int64_t)(p->tx1 - p->tx0 + 1) * (int64_t)(p->ty1 - p->ty0 + 1);
    p->sig = 1.0 / (1.0 + exp(-omega));
    p->depth32 = (float)I.tz;
    p->clampx = I.clx; p->clampy = I.cly;
    p->valid = 1;
}

void oracle_project(int64_t n, const double *mean, const double *log_scale, const double *quat,
                    const double *omega, const ocam_t *cam, const oopts_t *o, oproj_t *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < n; ++g)
        project_one(mean + 3 * g, log_scale + 3 * g, quat + 4 * g, omega[g], cam, o, out + g);
}

/* ---- tile lists ------------------------------------------------------------- */

typedef struct { uint64_t key; uint32_t id; uint32_t pad; } oinst_t;

static int cmp_inst(const void *x, const void *y)
{
    const oinst_t *a = (const oinst_t *)x, *b = (const oinst_t *)y;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->id != b->id) return a->id < b->id ? -1 : 1;
    return 0;
}

int64_t oracle_count(int64_t m, const oproj_t *proj)
{
    int64_t tot = 0;
    for (int64_t i = 0; i < m; ++i) tot += proj[i].valid ? proj[i].ntiles : 0;
    return tot;
}

static uint32_t f32_bits(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }

/* Every (tile, Gaussian) pair whose tile lies in the Gaussian's tile rectangle,
 * keyed (global_tile << 32) | bits(depth32), ordered by (key, id).
 * proj is [n_views][n]; ranges[2 t], ranges[2 t + 1] = [start, end) of tile t. */
void oracle_bin(int32_t n_views, int64_t n, const oproj_t *proj, const int64_t *tile_offset,
                const int32_t *tiles_x, int64_t total_tiles, int64_t total,
                uint64_t *keys, uint32_t *ids, uint32_t *ranges)
{
    oinst_t *v = (oinst_t *)malloc(sizeof(oinst_t) * (size_t)(total > 0 ? total : 1));
    int64_t k = 0;
    for (int32_t view = 0; view < n_views; ++view)
        for (int64_t g = 0; g < n; ++g) {
            const oproj_t *p = proj + (int64_t)view * n + g;
            if (!p->valid) continue;
            for (int32_t ty = p->ty0; ty <= p->ty1; ++ty)
                for (int32_t tx = p->tx0; tx <= p->tx1; ++tx) {
                    uint64_t tile = (uint64_t)(tile_offset[view] + (int64_t)ty * tiles_x[view] + tx);
                    v[k].key = (tile << 32) | (uint64_t)f32_bits(p->depth32);
                    v[k].id = (uint32_t)g;
                    v[k].pad = 0;
                    ++k;
                }
        }
    qsort(v, (size_t)k, sizeof(oinst_t), cmp_inst);
    for (int64_t t = 0; t < 2 * total_tiles; ++t) ranges[t] = 0;
    for (int64_t i = 0; i < k; ++i) {
        keys[i] = v[i].key;
        ids[i] = v[i].id;
        uint64_t tile = v[i].key >> 32;
        if (i == 0 || (v[i - 1].key >> 32) != tile) ranges[2 * tile] = (uint32_t)i;
        if (i == k - 1 || (v[i + 1].key >> 32) != tile) ranges[2 * tile + 1] = (uint32_t)(i + 1);
    }
    free(v);
}

/* ---- per-pixel front-to-back blending --------------------------------------- */

typedef struct {
    int64_t pos;   /* position in the list */
    uint32_t g;
    double alpha, T, ep, dx, dy;
    int clamped;
} oblend_t;

enum { DEC_BOX = 0, DEC_SKIP = 1, DEC_BLEND = 2, DEC_BLEND_CLAMP = 3, DEC_STOP = 4 };

static inline uint64_t fnv(uint64_t h, uint64_t v)
{
    for (int i = 0; i < 8; ++i) { h ^= (v >> (8 * i)) & 0xff; h *= 1099511628211ULL; }
    return h;
}

/* Blend pixel (i, j) over `list` (Gaussian ids in order). Decisions whose
 * relative margin to the 1/255 skip or the 1e-4 stop threshold is below eps are
 * counted as ambiguous events (for the skip, eps grows with the magnitude sum
 * of the exponent's terms: eps_alpha_mag); bit e of flip_mask inverts the
 * e-th such event.
 * rec (optional, capacity len) receives the blended entries in order. */
static void blend_pixel(int i, int j, const uint32_t *list, int64_t len, const oproj_t *P,
                        const double *ch, int C, const oopts_t *o, uint32_t flip_mask,
                        double *acc, double *T_out, int64_t *last_out, int32_t *n_amb,
                        double *min_margin, oblend_t *rec, int64_t *n_rec, uint64_t *hash)
{
    double T = 1.0;
    int64_t last = 0, nr = 0;
    int32_t ev = 0;
    double mm = INFINITY;
    for (int cc = 0; cc < C; ++cc) acc[cc] = 0.0;
    const double px = i + 0.5, py = j + 0.5;
    for (int64_t k = 0; k < len; ++k) {
        const uint32_t g = list[k];
        const oproj_t *p = P + g;
        if (!p->valid || i < p->x0 || i > p->x1 || j < p->y0 || j > p->y1) continue;
        const double dx = p->mx - px, dy = p->my - py;
        double power = -0.5 * (p->A * dx * dx + p->C * dy * dy) - p->B * dx * dy;
        if (power > 0.0) power = 0.0;
        const double ep = exp(power);
        const double raw = p->sig * ep;
        const int clamped = raw > o->alpha_max;
        const double alpha = clamped ? o->alpha_max : raw;
        /* skip decision */
        int skip = alpha < o->alpha_min;
        double m = fabs(alpha - o->alpha_min) / o->alpha_min;
        if (m < mm) mm = m;
        const double mag = 0.5 * (fabs(p->A * dx * dx) + fabs(p->C * dy * dy)) + fabs(p->B * dx * dy);
        if (m < o->eps_alpha + o->eps_alpha_mag * mag) {
            if (ev < 32 && ((flip_mask >> ev) & 1u)) skip = !skip;
            ++ev;
        }
        if (skip) {
            if (hash) *hash = fnv(fnv(*hash, g), DEC_SKIP);
            continue;
        }
        /* stop decision (tested before blending; the stopping Gaussian is not blended) */
        const double Tn = T * (1.0 - alpha);
        int stop = Tn < o->t_min;
        m = fabs(Tn - o->t_min) / o->t_min;
        if (m < mm) mm = m;
        if (m < o->eps_t) {
            if (ev < 32 && ((flip_mask >> ev) & 1u)) stop = !stop;
            ++ev;
        }
        if (stop) {
            if (hash) *hash = fnv(fnv(*hash, g), DEC_STOP);
            break;
        }
        const double w = alpha * T;
        const double *cg = ch + (int64_t)g * C;
        for (int cc = 0; cc < C; ++cc) acc[cc] += w * cg[cc];
        if (rec) {
            rec[nr].pos = k; rec[nr].g = g; rec[nr].alpha = alpha; rec[nr].T = T;
            rec[nr].ep = ep; rec[nr].dx = dx; rec[nr].dy = dy; rec[nr].clamped = clamped;
        }
        ++nr;
        if (hash) *hash = fnv(fnv(*hash, g), clamped ? DEC_BLEND_CLAMP : DEC_BLEND);
        T = Tn;
        last = k + 1;
    }
    *T_out = T;
    *last_out = last;
    if (n_amb) *n_amb = ev;
    if (min_margin) *min_margin = mm;
    if (n_rec) *n_rec = nr;
}

static inline const uint32_t *tile_list(int i, int j, const ocam_t *cam, const oopts_t *o,
                                        const uint32_t *ids, const uint32_t *ranges,
                                        int64_t tile_offset, int64_t *len)
{
    const int tiles_x = (cam->W + o->tile - 1) / o->tile;
    const int64_t t = tile_offset + (int64_t)(j / o->tile) * tiles_x + (i / o->tile);
    const uint32_t s = ranges[2 * t], e = ranges[2 * t + 1];
    *len = (int64_t)e - (int64_t)s;
    return ids + s;
}

/* Render pixels of one view from its tile lists. pix == NULL renders every
 * pixel (outputs planar [C][H*W]); otherwise npix listed linear pixel indices
 * (outputs [C][npix]). flip_mask (optional) per output pixel. */
void oracle_render(const oproj_t *pv, const ocam_t *cam, const oopts_t *o, const double *ch,
                   int32_t C, const uint32_t *ids, const uint32_t *ranges, int64_t tile_offset,
                   int64_t npix, const int64_t *pix, const uint32_t *flip_mask,
                   double *out, double *T_final, int64_t *last, int32_t *n_amb, double *margin)
{
    const int64_t HW = (int64_t)cam->W * cam->H;
    const int64_t cnt = pix ? npix : HW;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t q = 0; q < cnt; ++q) {
        const int64_t lin = pix ? pix[q] : q;
        const int i = (int)(lin % cam->W), j = (int)(lin / cam->W);
        int64_t len;
        const uint32_t *list = tile_list(i, j, cam, o, ids, ranges, tile_offset, &len);
        double acc[64];
        double T; int64_t l; int32_t na; double mm;
        blend_pixel(i, j, list, len, pv, ch, C, o, flip_mask ? flip_mask[q] : 0u, acc, &T, &l,
                    &na, &mm, NULL, NULL, NULL);
        for (int cc = 0; cc < C; ++cc) out[(int64_t)cc * cnt + q] = acc[cc];
        T_final[q] = T;
        last[q] = l;
        if (n_amb) n_amb[q] = na;
        if (margin) margin[q] = mm;
    }
}

/* ---- tile-free rendering of a rectangle (for brute-force checks and FD) ------ */

typedef struct { uint32_t bits; uint32_t id; } ocand_t;

static int cmp_cand(const void *x, const void *y)
{
    const ocand_t *a = (const ocand_t *)x, *b = (const ocand_t *)y;
    if (a->bits != b->bits) return a->bits < b->bits ? -1 : 1;
    if (a->id != b->id) return a->id < b->id ? -1 : 1;
    return 0;
}

/* Render the rectangle [x0, x0+w) x [y0, y0+h) directly from the definition:
 * for each pixel, every valid Gaussian whose pixel box contains it, ordered by
 * (depth32 bits, id). Candidates are those whose box meets the rectangle; each
 * 8x8 cell of the rectangle keeps, in that order, the candidates whose box
 * meets the cell (a superset of every pixel's list there, in the same order,
 * so the result equals a scan over all candidates). Returns sum(G * out) when
 * G != NULL, and a hash of every skip / blend / clamp / stop decision. */
double oracle_render_region(int64_t n, const oproj_t *pv, const ocam_t *cam, const oopts_t *o,
                            const double *ch, int32_t C, int32_t x0, int32_t y0, int32_t w,
                            int32_t h, const double *G, double *out, double *T_out,
                            uint64_t *hash_out)
{
    (void)cam;
    int64_t m = 0;
    for (int64_t g = 0; g < n; ++g) {
        const oproj_t *p = pv + g;
        if (p->valid && p->x1 >= x0 && p->x0 < x0 + w && p->y1 >= y0 && p->y0 < y0 + h) ++m;
    }
    ocand_t *cand = (ocand_t *)malloc(sizeof(ocand_t) * (size_t)(m > 0 ? m : 1));
    m = 0;
    for (int64_t g = 0; g < n; ++g) {
        const oproj_t *p = pv + g;
        if (p->valid && p->x1 >= x0 && p->x0 < x0 + w && p->y1 >= y0 && p->y0 < y0 + h) {
            cand[m].bits = f32_bits(p->depth32);
            cand[m].id = (uint32_t)g;
            ++m;
        }
    }
    qsort(cand, (size_t)m, sizeof(ocand_t), cmp_cand);
    /* per-cell candidate lists (CSR) */
    const int cw = (w + 7) / 8, chh = (h + 7) / 8, ncell = cw * chh;
    int64_t *cstart = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    for (int64_t k = 0; k < m; ++k) {
        const oproj_t *p = pv + cand[k].id;
        const int cx0 = (p->x0 > x0 ? p->x0 - x0 : 0) / 8, cx1 = (p->x1 - x0 < w - 1 ? p->x1 - x0 : w - 1) / 8;
        const int cy0 = (p->y0 > y0 ? p->y0 - y0 : 0) / 8, cy1 = (p->y1 - y0 < h - 1 ? p->y1 - y0 : h - 1) / 8;
        for (int cy = cy0; cy <= cy1; ++cy)
            for (int cx = cx0; cx <= cx1; ++cx) cstart[cy * cw + cx + 1]++;
    }
    for (int c = 0; c < ncell; ++c) cstart[c + 1] += cstart[c];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncell > 0 ? ncell : 1));
    for (int c = 0; c < ncell; ++c) fill[c] = cstart[c];
    uint32_t *lists = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(cstart[ncell] > 0 ? cstart[ncell] : 1));
    for (int64_t k = 0; k < m; ++k) {
        const oproj_t *p = pv + cand[k].id;
        const int cx0 = (p->x0 > x0 ? p->x0 - x0 : 0) / 8, cx1 = (p->x1 - x0 < w - 1 ? p->x1 - x0 : w - 1) / 8;
        const int cy0 = (p->y0 > y0 ? p->y0 - y0 : 0) / 8, cy1 = (p->y1 - y0 < h - 1 ? p->y1 - y0 : h - 1) / 8;
        for (int cy = cy0; cy <= cy1; ++cy)
            for (int cx = cx0; cx <= cx1; ++cx) lists[fill[cy * cw + cx]++] = cand[k].id;
    }
    free(cand);
    free(fill);
    const int64_t hw = (int64_t)w * h;
    uint64_t *phash = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(hw > 0 ? hw : 1));
    double *ploss = (double *)malloc(sizeof(double) * (size_t)(hw > 0 ? hw : 1));
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t q = 0; q < hw; ++q) {
        const int32_t jj = (int32_t)(q / w), ii = (int32_t)(q % w);
        const int cell = (jj / 8) * cw + ii / 8;
        double acc[64];
        double T; int64_t l;
        uint64_t hh = 1469598103934665603ULL;
        blend_pixel(x0 + ii, y0 + jj, lists + cstart[cell], cstart[cell + 1] - cstart[cell], pv, ch,
                    C, o, 0u, acc, &T, &l, NULL, NULL, NULL, NULL, &hh);
        double lq = 0.0;
        for (int cc = 0; cc < C; ++cc) {
            if (out) out[(int64_t)cc * hw + q] = acc[cc];
            if (G) lq += G[(int64_t)cc * hw + q] * acc[cc];
        }
        if (T_out) T_out[q] = T;
        phash[q] = hh;
        ploss[q] = lq;
    }
    double loss = 0.0;
    uint64_t hash = 1469598103934665603ULL;
    for (int64_t q = 0; q < hw; ++q) {
        hash = fnv(hash, phash[q]);
        loss += ploss[q];
    }
    free(phash);
    free(ploss);
    free(lists);
    free(cstart);
    if (hash_out) *hash_out = hash;
    return loss;
}

/* ---- backward of the blend --------------------------------------------------- */

/* For one view: given G = dL/d(out) planar [C][H*W], accumulate per-Gaussian
 * screen-space gradients grad2d[n][6] = d(mx, my, A, B, C, sig) for this view
 * and channel gradients dch[n][C] (summed over views by repeated calls).
 * out_c = sum_k alpha_k T_k ch_kc with T_k = prod_{j<k} (1 - alpha_j), so
 * d out_c / d alpha_k = T_k ch_kc - (sum_{j>k} alpha_j T_j ch_jc) / (1 - alpha_k). */
/* mag2d [n][6] and magch [n][C] (optional, accumulated like grad2d and dch):
 * the same sums with every term replaced by its magnitude (|G_c|, |ch| and the
 * absolute values of the power's derivatives), i.e. sum |term| for each
 * gradient: the scale of the rounding error of any floating-point evaluation
 * of these sums. Every term of a pixel is weighted by 1 + mag_cond * S with
 * S = sum over the pixel's blended entries of 1 / (1 - alpha): a rounding
 * error e in alpha changes 1 - alpha by the relative amount
 * e alpha / (1 - alpha), and the transmittance T = prod (1 - alpha) and the
 * suffix behind an entry, which every term of the pixel uses, collect these
 * relative errors over the list, so S is the condition number of the
 * pixel's terms with respect to the rounding of its alphas. */
void oracle_render_backward(int64_t n, const oproj_t *pv, const ocam_t *cam, const oopts_t *o,
                            const double *ch, int32_t C, const uint32_t *ids,
                            const uint32_t *ranges, int64_t tile_offset, const double *G,
                            const uint32_t *flip_mask, double *grad2d, double *dch,
                            double *mag2d, double *magch, double mag_cond)
{
    const int64_t HW = (int64_t)cam->W * cam->H;
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    const int want_mag = mag2d != NULL && magch != NULL;
    double *priv2 = (double *)calloc((size_t)nth * (size_t)n * 6 * (want_mag ? 2 : 1), sizeof(double));
    double *privc = (double *)calloc((size_t)nth * (size_t)n * (size_t)C * (want_mag ? 2 : 1), sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *g2 = priv2 + (size_t)tid * (size_t)n * 6;
        double *gc = privc + (size_t)tid * (size_t)n * (size_t)C;
        double *m2 = want_mag ? priv2 + ((size_t)nth + (size_t)tid) * (size_t)n * 6 : NULL;
        double *mc = want_mag ? privc + ((size_t)nth + (size_t)tid) * (size_t)n * (size_t)C : NULL;
        int64_t cap = 0;
        oblend_t *rec = NULL;
        double *suffix = NULL, *suffix_abs = NULL;
#pragma omp for schedule(dynamic, 256)
        for (int64_t q = 0; q < HW; ++q) {
            const int i = (int)(q % cam->W), j = (int)(q / cam->W);
            int64_t len;
            const uint32_t *list = tile_list(i, j, cam, o, ids, ranges, tile_offset, &len);
            if (len > cap) {
                cap = len;
                rec = (oblend_t *)realloc(rec, sizeof(oblend_t) * (size_t)cap);
                suffix = (double *)realloc(suffix, sizeof(double) * (size_t)cap * (size_t)C);
                if (want_mag) suffix_abs = (double *)realloc(suffix_abs, sizeof(double) * (size_t)cap * (size_t)C);
            }
            double acc[64];
            double T; int64_t l, nr;
            blend_pixel(i, j, list, len, pv, ch, C, o, flip_mask ? flip_mask[q] : 0u, acc, &T,
                        &l, NULL, NULL, rec, &nr, NULL);
            if (nr == 0) continue;
            /* suffix sums S_k = sum_{j>k} alpha_j T_j ch_j */
            for (int cc = 0; cc < C; ++cc) suffix[(nr - 1) * C + cc] = 0.0;
            for (int64_t k = nr - 2; k >= 0; --k) {
                const oblend_t *e = rec + k + 1;
                const double *cg = ch + (int64_t)e->g * C;
                for (int cc = 0; cc < C; ++cc)
                    suffix[k * C + cc] = suffix[(k + 1) * C + cc] + e->alpha * e->T * cg[cc];
            }
            double wmag = 1.0;
            if (want_mag) {
                double S = 0.0;
                for (int64_t k = 0; k < nr; ++k) S += 1.0 / (1.0 - rec[k].alpha);
                wmag = 1.0 + mag_cond * S;
                for (int cc = 0; cc < C; ++cc) suffix_abs[(nr - 1) * C + cc] = 0.0;
                for (int64_t k = nr - 2; k >= 0; --k) {
                    const oblend_t *e = rec + k + 1;
                    const double *cg = ch + (int64_t)e->g * C;
                    for (int cc = 0; cc < C; ++cc)
                        suffix_abs[k * C + cc] = suffix_abs[(k + 1) * C + cc] + e->alpha * e->T * fabs(cg[cc]);
                }
            }
            for (int64_t k = 0; k < nr; ++k) {
                const oblend_t *e = rec + k;
                const oproj_t *p = pv + e->g;
                const double *cg = ch + (int64_t)e->g * C;
                double dalpha = 0.0, dalpha_abs = 0.0;
                for (int cc = 0; cc < C; ++cc) {
                    const double Gc = G[(int64_t)cc * HW + q];
                    gc[(int64_t)e->g * C + cc] += e->alpha * e->T * Gc;
                    dalpha += Gc * (e->T * cg[cc] - suffix[k * C + cc] / (1.0 - e->alpha));
                    if (want_mag) {
                        mc[(int64_t)e->g * C + cc] += wmag * e->alpha * e->T * fabs(Gc);
                        dalpha_abs += wmag * fabs(Gc) * (e->T * fabs(cg[cc]) + suffix_abs[k * C + cc] / (1.0 - e->alpha));
                    }
                }
                if (e->clamped) continue;
                double *d = g2 + (int64_t)e->g * 6;
                d[5] += dalpha * e->ep;                 /* d sig */
                const double dpow = dalpha * p->sig * e->ep;
                const double dx = e->dx, dy = e->dy;
                const double raw = -0.5 * (p->A * dx * dx + p->C * dy * dy) - p->B * dx * dy;
                if (want_mag) m2[(int64_t)e->g * 6 + 5] += dalpha_abs * e->ep;
                if (raw > 0.0) continue;                /* power clamped at 0 */
                d[0] += dpow * (-(p->A * dx + p->B * dy));
                d[1] += dpow * (-(p->B * dx + p->C * dy));
                d[2] += dpow * (-0.5 * dx * dx);
                d[3] += dpow * (-dx * dy);
                d[4] += dpow * (-0.5 * dy * dy);
                if (want_mag) {
                    double *mm = m2 + (int64_t)e->g * 6;
                    const double ap = dalpha_abs * p->sig * e->ep;
                    mm[0] += ap * (fabs(p->A * dx) + fabs(p->B * dy));
                    mm[1] += ap * (fabs(p->B * dx) + fabs(p->C * dy));
                    mm[2] += ap * 0.5 * dx * dx;
                    mm[3] += ap * fabs(dx * dy);
                    mm[4] += ap * 0.5 * dy * dy;
                }
            }
        }
        free(rec);
        free(suffix);
        free(suffix_abs);
    }
    for (int t = 0; t < nth; ++t) {
        const double *g2 = priv2 + (size_t)t * (size_t)n * 6;
        const double *gc = privc + (size_t)t * (size_t)n * (size_t)C;
        for (int64_t x = 0; x < n * 6; ++x) grad2d[x] += g2[x];
        for (int64_t x = 0; x < n * C; ++x) dch[x] += gc[x];
        if (want_mag) {
            const double *m2 = priv2 + ((size_t)nth + (size_t)t) * (size_t)n * 6;
            const double *mc = privc + ((size_t)nth + (size_t)t) * (size_t)n * (size_t)C;
            for (int64_t x = 0; x < n * 6; ++x) mag2d[x] += m2[x];
            for (int64_t x = 0; x < n * C; ++x) magch[x] += mc[x];
        }
    }
    free(priv2);
    free(privc);
}

/* ---- backward of the projection ------------------------------------------- */

/* Chain rule from d(mx, my, A, B, C, sig) of one view back to the mean,
 * log-scale, (unnormalised) quaternion and opacity logit; accumulates. */
static void project_one_backward(const double mu[3], const double ls[3], const double q[4],
                                 double omega, const ocam_t *cam, const oopts_t *o,
                                 const double g[6], double dmu[3], double dls[3], double dq[4],
                                 double *domega)
{
    oproj_t p;
    project_one(mu, ls, q, omega, cam, o, &p);
    if (!p.valid) return;
    oproj_int_t I;
    project_intermediates(mu, ls, q, cam, o, &I);
    const double *R = cam->R;
    const double a = I.a, b = I.b, c = I.c;
    const double det = a * c - b * b, id = 1.0 / det, id2 = id * id;
    const double gA = g[2], gB = g[3], gC = g[4];
    /* opacity */
    const double sg = p.sig;
    *domega += g[5] * sg * (1.0 - sg);
    /* conic (A, B, C) = (c, -b, a) / det  ->  (a, b, c) */
    const double da = gA * (-c * c * id2) + gB * (b * c * id2) + gC * (id - a * c * id2);
    const double db = gA * (2.0 * b * c * id2) + gB * (-id - 2.0 * b * b * id2) + gC * (2.0 * a * b * id2);
    const double dc = gA * (id - a * c * id2) + gB * (a * b * id2) + gC * (-a * a * id2);
    const double Gp[2][2] = {{da, 0.5 * db}, {0.5 * db, dc}};
    /* Sigma' = T Sigma T^T: dT = 2 G' T Sigma, dSigma = T^T G' T */
    double TS[2][3], dT[2][3], dSig[3][3];
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 3; ++k) {
            double acc = 0.0;
            for (int i = 0; i < 3; ++i) acc += I.T[r][i] * I.Sig[i][k];
            TS[r][k] = acc;
        }
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 3; ++k) dT[r][k] = 2.0 * (Gp[r][0] * TS[0][k] + Gp[r][1] * TS[1][k]);
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) {
            double acc = 0.0;
            for (int r = 0; r < 2; ++r)
                for (int s = 0; s < 2; ++s) acc += I.T[r][i] * Gp[r][s] * I.T[s][k];
            dSig[i][k] = acc;
        }
    /* T = J W: dJ = dT W^T */
    double dJ[2][3];
    for (int r = 0; r < 2; ++r)
        for (int cc = 0; cc < 3; ++cc) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += dT[r][k] * R[3 * cc + k];
            dJ[r][cc] = acc;
        }
    const double tx = I.tx, ty = I.ty, tz = I.tz, fx = cam->fx, fy = cam->fy;
    const double tz2 = tz * tz, tz3 = tz2 * tz;
    double dtx = 0.0, dty = 0.0, dtz = 0.0;
    dtz += dJ[0][0] * (-fx / tz2);
    dtz += dJ[1][1] * (-fy / tz2);
    if (!I.clx) { dtx += dJ[0][2] * (-fx / tz2); dtz += dJ[0][2] * (2.0 * fx * tx / tz3); }
    else { dtz += dJ[0][2] * (fx * I.ux / tz2); }
    if (!I.cly) { dty += dJ[1][2] * (-fy / tz2); dtz += dJ[1][2] * (2.0 * fy * ty / tz3); }
    else { dtz += dJ[1][2] * (fy * I.uy / tz2); }
    /* 2D mean */
    dtx += g[0] * fx / tz;
    dtz += -g[0] * fx * tx / tz2;
    dty += g[1] * fy / tz;
    dtz += -g[1] * fy * ty / tz2;
    /* t = W mu + t_v */
    for (int k = 0; k < 3; ++k) dmu[k] += R[k] * dtx + R[3 + k] * dty + R[6 + k] * dtz;
    /* Sigma = M M^T: dM = 2 dSigma M */
    double dM[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            dM[i][j] = 2.0 * (dSig[i][0] * I.M[0][j] + dSig[i][1] * I.M[1][j] + dSig[i][2] * I.M[2][j]);
    /* M = Rq diag(s) */
    double dR[3][3];
    for (int j = 0; j < 3; ++j) {
        double dsj = 0.0;
        for (int i = 0; i < 3; ++i) { dR[i][j] = dM[i][j] * I.s[j]; dsj += dM[i][j] * I.Rq[i][j]; }
        dls[j] += dsj * I.s[j];
    }
    /* rotation of the normalised quaternion (w, x, y, z) */
    const double w = I.qn[0], x = I.qn[1], y = I.qn[2], z = I.qn[3];
    double dqn[4];
    dqn[0] = 2.0 * (-z * dR[0][1] + y * dR[0][2] + z * dR[1][0] - x * dR[1][2] - y * dR[2][0] + x * dR[2][1]);
    dqn[1] = 2.0 * (y * dR[0][1] + z * dR[0][2] + y * dR[1][0] - w * dR[1][2] + z * dR[2][0] + w * dR[2][1])
             - 4.0 * x * (dR[1][1] + dR[2][2]);
    dqn[2] = 2.0 * (x * dR[0][1] + w * dR[0][2] + x * dR[1][0] + z * dR[1][2] - w * dR[2][0] + z * dR[2][1])
             - 4.0 * y * (dR[0][0] + dR[2][2]);
    dqn[3] = 2.0 * (-w * dR[0][1] + x * dR[0][2] + w * dR[1][0] + y * dR[1][2] + x * dR[2][0] + y * dR[2][1])
             - 4.0 * z * (dR[0][0] + dR[1][1]);
    const double dot = w * dqn[0] + x * dqn[1] + y * dqn[2] + z * dqn[3];
    for (int k = 0; k < 4; ++k) dq[k] += (dqn[k] - I.qn[k] * dot) / I.qnorm;
}

void oracle_project_backward(int64_t n, const double *mean, const double *log_scale,
                             const double *quat, const double *omega, const ocam_t *cam,
                             const oopts_t *o, const double *grad2d, double *dmean, double *dls,
                             double *dquat, double *domega)
{
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < n; ++g)
        project_one_backward(mean + 3 * g, log_scale + 3 * g, quat + 4 * g, omega[g], cam, o,
                             grad2d + 6 * g, dmean + 3 * g, dls + 3 * g, dquat + 4 * g, domega + g);
}

int32_t oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads used by the parallel loops above from now on (timing runs only). */
void oracle_set_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
