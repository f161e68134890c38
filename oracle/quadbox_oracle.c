/*
 * QuadBox CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct reference for the rasterizer hot path of
 * "QuadBox: Accelerating 3D Gaussian Splatting with Geometry-Aware Boxes"
 * (arXiv 2605.04844).  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load this library; the GPU path never links or calls it,
 * and it shares no code, header or table with the GPU path.
 *
 * Precision.  Every floating-point value that decides an integer result (a tile
 * set, a depth key, the alpha-cutoff decision of the render) is computed in
 * IEEE binary32 with a fixed operation order (no contraction: build with
 * -ffp-contract=off; `fmaf` appears only where the order says so), with `/`
 * and `sqrtf` correctly rounded, and with every transcendental evaluated in
 * binary64 and rounded once to binary32.  The one exception is the chain
 * Sigma3D -> Sigma2D -> conic, formed with binary64 +, -, *, / from the
 * binary32 scales, unit quaternion and projected mean, each result rounded
 * once to binary32 (a nearly singular Sigma2D loses its conic to cancellation
 * in binary32).  Everything that only feeds the image (colour, blending
 * weights, accumulation) is binary64.
 *
 * Parity status per function (see the tests that pin each one):
 *   oc_project        pinned: closed forms (Eqs. 5, 6, 9, 11, 12), textbook
 *                     isotropic projection, support-function brute force (Eq. 8)
 *   oc_sh_basis       pinned: complex spherical harmonics of scipy
 *   oc_tile_set       pinned: brute-force conservativeness, set inclusions
 *   oc_pairs          pinned: library sort (qsort of chunks, merged) +
 *                     uniqueness/inclusion tests, a single qsort of the list
 *   oc_ranges         pinned: binary search definition vs linear scan
 *   oc_render         pinned: Eq. (2) closed forms for one and two Gaussians,
 *                     tile-free brute-force render
 *   oc_pixel_boxes    3-sigma square pinned: radius against numpy's eigvalsh
 *                     (isotropic closed form in the floored regime), tile set
 *                     against pixel-sample enumeration
 *   oc_project64,     pinned: agreement with the binary32 projection and the
 *   oc_forward64      binary32 tiled render, both pinned on their own
 *   oc_backward64     pinned: central finite differences of oc_forward64
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OC_TILE 16

enum { OC_BOX_3SIGMA = 0, OC_BOX_ADR = 1, OC_BOX_QUADBOX = 2, OC_BOX_DUALBOX = 3 };
/* Flag added to an opacity-aware mode: each sub-box's tile rect is
 * intersected with the tile rect of the 3-sigma square (the reading that
 * keeps every tile set inside the 3-sigma baseline's, Sec. 2 vs Sec. 3.1). */
enum { OC_CLIP_3SIGMA = 16 };

/* Camera: world->camera rotation R (row-major) and translation t, pinhole
 * intrinsics; x right, y down, z forward; pixel (i, j) samples the point (i, j). */
typedef struct {
    int32_t W, H;
    float fx, fy, cx, cy, near_plane;
    float R[9];
    float t[3];
    float campos[3];
} oc_camera;

/* Per-Gaussian projected values (all binary32 except rgb). */
typedef struct {
    float u, v, depth;       /* mean2D and view depth                                 */
    float A, B, C;           /* Sigma2D entries incl. the 0.3 low-pass on A and C     */
    float a, b, c;           /* conic Lambda = inverse(Sigma2D) = [a b; b c]           */
    float opacity, gamma;    /* o and gamma = 2 ln(o / alpha_min)                      */
    int32_t visible;         /* 0 when culled                                         */
    int32_t nrect;           /* number of tile rectangles whose union is the tile set */
    int32_t rect[4][4];      /* tile rects: tx0, tx1, ty0, ty1 (inclusive)             */
    double rgb[3];
} oc_gauss;

/* ------------------------------------------------------------------------- */
/* Real spherical harmonics, degree <= 3, index k = l*l + l + m.              */
/* Basis: complex SH with the Condon-Shortley phase, made real by              */
/*   m > 0: sqrt2 Re Y_l^m,  m < 0: sqrt2 Im Y_l^|m|,  m = 0: Y_l^0,            */
/* written out as polynomials of the unit direction (x, y, z).                  */
/* ------------------------------------------------------------------------- */
void oc_sh_basis(double x, double y, double z, double out[16])
{
    const double pi = 3.14159265358979323846;
    const double k00 = 0.5 * sqrt(1.0 / pi);
    const double k1 = sqrt(3.0 / (4.0 * pi));
    const double k2a = 0.5 * sqrt(15.0 / pi);
    const double k2b = 0.25 * sqrt(5.0 / pi);
    const double k2c = 0.25 * sqrt(15.0 / pi);
    const double k3a = 0.25 * sqrt(35.0 / (2.0 * pi));
    const double k3b = 0.5 * sqrt(105.0 / pi);
    const double k3c = 0.25 * sqrt(21.0 / (2.0 * pi));
    const double k3d = 0.25 * sqrt(7.0 / pi);
    const double k3e = 0.25 * sqrt(105.0 / pi);
    double xx = x * x, yy = y * y, zz = z * z;
    out[0] = k00;
    out[1] = -k1 * y;
    out[2] = k1 * z;
    out[3] = -k1 * x;
    out[4] = k2a * x * y;
    out[5] = -k2a * y * z;
    out[6] = k2b * (2.0 * zz - xx - yy);
    out[7] = -k2a * x * z;
    out[8] = k2c * (xx - yy);
    out[9] = -k3a * y * (3.0 * xx - yy);
    out[10] = k3b * x * y * z;
    out[11] = -k3c * y * (4.0 * zz - xx - yy);
    out[12] = k3d * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
    out[13] = -k3c * x * (4.0 * zz - xx - yy);
    out[14] = k3e * z * (xx - yy);
    out[15] = -k3a * x * (xx - 3.0 * yy);
}

/* ------------------------------------------------------------------------- */
/* Tile mapping of a closed pixel-coordinate interval [x0, x1] on an axis of   */
/* `n` pixels: the tiles holding the integer samples that lie in it (the       */
/* tile-space bounds of Sec. 3.2).  Returns 0 when no sample lies inside.       */
/* ------------------------------------------------------------------------- */
static int oc_axis_tiles(float x0, float x1, int n, int* t0, int* t1)
{
    float hi = (float)(n - 1);
    if (!(x1 >= 0.0f) || !(x0 <= hi)) return 0;
    float lo_c = x0 > 0.0f ? x0 : 0.0f;
    float hi_c = x1 < hi ? x1 : hi;
    int p0 = (int)ceilf(lo_c);
    int p1 = (int)floorf(hi_c);
    if (p0 > p1) return 0;
    *t0 = p0 / OC_TILE;
    *t1 = p1 / OC_TILE;
    return 1;
}

/* A pixel-coordinate box [x0,x1]x[y0,y1] -> tile rect; 0 when empty. */
static int oc_box_rect(float x0, float x1, float y0, float y1, int W, int H, int32_t r[4])
{
    int a, b, c, d;
    if (!oc_axis_tiles(x0, x1, W, &a, &b)) return 0;
    if (!oc_axis_tiles(y0, y1, H, &c, &d)) return 0;
    r[0] = a; r[1] = b; r[2] = c; r[3] = d;
    return 1;
}

/* Pixel-space boxes of one projected Gaussian (Sec. 2 for the 3-sigma square,
 * Sec. 3.1 for AdR-AABB, DualBox and QuadBox).  Each box is the closed region
 * [x0, x1] x [y0, y1]; returns how many boxes were written (1, 2 or 4). */
int oc_pixel_boxes(const oc_gauss* g, int mode, float box[4][4])
{
    float u = g->u, v = g->v, A = g->A, B = g->B, C = g->C, gam = g->gamma;
    mode &= ~OC_CLIP_3SIGMA;   /* the clip acts on tile rects (oc_build_boxes) */
    if (mode == OC_BOX_3SIGMA) {
        /* square of side 6 sqrt(lambda_max) (Sec. 2), radius rounded up to a
         * whole pixel, discriminant floored at 0.1 */
        float det = A * C - B * B;
        float mid = 0.5f * (A + C);
        float disc = mid * mid - det;
        if (disc < 0.1f) disc = 0.1f;
        float lam = mid + sqrtf(disc);
        float r = ceilf(3.0f * sqrtf(lam));
        box[0][0] = u - r; box[0][1] = u + r; box[0][2] = v - r; box[0][3] = v + r;
        return 1;
    }
    /* half extents from the support function, Eqs. (9)/(11) in Sigma2D entries */
    float xm = sqrtf(gam * A);
    float ym = sqrtf(gam * C);
    if (mode == OC_BOX_ADR) {
        box[0][0] = u - xm; box[0][1] = u + xm; box[0][2] = v - ym; box[0][3] = v + ym;
        return 1;
    }
    /* stretching factor, Eq. (12): b^2/(ac) = B^2/(AC) */
    float ratio = (B * B) / (A * C);
    float fs = 1.0f - ratio;
    if (fs < 0.0f) fs = 0.0f;
    float f = sqrtf(fs);
    /* quadrants holding the major axis: (+,+),(-,-) when B > 0, else (+,-),(-,+) */
    int maj_same = B > 0.0f;
    int nb = 0;
    for (int q = 0; q < 4; q++) {
        int sx = (q & 1) ? 1 : -1;
        int sy = (q & 2) ? 1 : -1;
        int major = maj_same ? (sx == sy) : (sx != sy);
        float w, h;
        if (major) {
            w = xm; h = ym;
        } else {
            if (mode == OC_BOX_DUALBOX) continue;
            w = f * xm; h = f * ym;
        }
        box[nb][0] = sx > 0 ? u : u - w;
        box[nb][1] = sx > 0 ? u + w : u;
        box[nb][2] = sy > 0 ? v : v - h;
        box[nb][3] = sy > 0 ? v + h : v;
        nb++;
    }
    return nb;
}

/* Tile rects of the boxes; empty ones are dropped.  Fills g->rect / g->nrect.
 * With OC_CLIP_3SIGMA each rect is cut to the 3-sigma square's tile rect. */
void oc_build_boxes(oc_gauss* g, int mode, int W, int H)
{
    float box[4][4];
    int nb = oc_pixel_boxes(g, mode & ~OC_CLIP_3SIGMA, box);
    int32_t sq[4];
    int have_sq = 1;
    if (mode & OC_CLIP_3SIGMA) {
        float b3[4][4];
        oc_pixel_boxes(g, OC_BOX_3SIGMA, b3);
        have_sq = oc_box_rect(b3[0][0], b3[0][1], b3[0][2], b3[0][3], W, H, sq);
    }
    g->nrect = 0;
    for (int k = 0; k < nb; k++) {
        int32_t* r = g->rect[g->nrect];
        if (!oc_box_rect(box[k][0], box[k][1], box[k][2], box[k][3], W, H, r)) continue;
        if (mode & OC_CLIP_3SIGMA) {
            if (!have_sq) continue;
            if (r[0] < sq[0]) r[0] = sq[0];
            if (r[1] > sq[1]) r[1] = sq[1];
            if (r[2] < sq[2]) r[2] = sq[2];
            if (r[3] > sq[3]) r[3] = sq[3];
            if (r[0] > r[1] || r[2] > r[3]) continue;
        }
        g->nrect++;
    }
}

/* ------------------------------------------------------------------------- */
/* The activations, each evaluated in binary64 and rounded once to binary32:
 * scale s = exp(log_scale), opacity o = sigmoid(logit) = 1 / (1 + exp(-logit)),
 * and gamma = 2 ln(o / alpha_min) with alpha_min = 1/255 (Eq. (3)). */
static float oc_act_scale(float l) { return (float)exp((double)l); }
static float oc_act_opacity(float x) { return (float)(1.0 / (1.0 + exp(-(double)x))); }
static float oc_act_gamma(float o) { return (float)(2.0 * log(255.0 * (double)o)); }

/* out[i] = activation `which` (0 scale, 1 opacity, 2 gamma) of x[i]. */
void oc_activations(int64_t n, const float* x, int which, float* out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++)
        out[i] = which == 0 ? oc_act_scale(x[i]) : which == 1 ? oc_act_opacity(x[i]) : oc_act_gamma(x[i]);
}

/* ------------------------------------------------------------------------- */
/* EWA projection of one Gaussian (Sec. 2, Eq. (1); Eqs. (3), (4) for gamma).  */
void oc_project_one(const oc_camera* cam, const float mean[3], const float lscale[3],
                    const float quat[4], float logit, const float* sh, int64_t n, int64_t i,
                    int sh_degree, int mode, oc_gauss* g)
{
    memset(g, 0, sizeof(*g));
    const float* R = cam->R;
    /* view transform */
    float px = ((R[0] * mean[0] + R[1] * mean[1]) + R[2] * mean[2]) + cam->t[0];
    float py = ((R[3] * mean[0] + R[4] * mean[1]) + R[5] * mean[2]) + cam->t[1];
    float pz = ((R[6] * mean[0] + R[7] * mean[1]) + R[8] * mean[2]) + cam->t[2];
    g->depth = pz;
    if (!(pz > cam->near_plane) || !isfinite(px) || !isfinite(py) || !isfinite(pz)) return;

    /* activations: evaluated in binary64, rounded once */
    float s0 = oc_act_scale(lscale[0]);
    float s1 = oc_act_scale(lscale[1]);
    float s2 = oc_act_scale(lscale[2]);
    float o = oc_act_opacity(logit);
    g->opacity = o;
    g->gamma = oc_act_gamma(o);

    /* unit quaternion (w, x, y, z) -> rotation */
    float n2 = ((quat[0] * quat[0] + quat[1] * quat[1]) + quat[2] * quat[2]) + quat[3] * quat[3];
    if (!(n2 > 0.0f) || !isfinite(n2)) return;
    float nr = sqrtf(n2);
    float w = quat[0] / nr, x = quat[1] / nr, y = quat[2] / nr, z = quat[3] / nr;
    /* From here to the conic the arithmetic is binary64 on the binary32
     * values above, and each result is rounded once to binary32: Sigma2D of
     * a needle-like Gaussian is nearly singular, and binary32 entries would
     * lose a large part of A C - B^2 to cancellation. */
    double dw = w, dx = x, dy = y, dz = z;
    double Rq[9];
    Rq[0] = 1.0 - 2.0 * (dy * dy + dz * dz);
    Rq[1] = 2.0 * (dx * dy - dw * dz);
    Rq[2] = 2.0 * (dx * dz + dw * dy);
    Rq[3] = 2.0 * (dx * dy + dw * dz);
    Rq[4] = 1.0 - 2.0 * (dx * dx + dz * dz);
    Rq[5] = 2.0 * (dy * dz - dw * dx);
    Rq[6] = 2.0 * (dx * dz - dw * dy);
    Rq[7] = 2.0 * (dy * dz + dw * dx);
    Rq[8] = 1.0 - 2.0 * (dx * dx + dy * dy);

    /* Sigma3D = M M^T with M = Rq diag(s) */
    double sc[3] = {s0, s1, s2};
    double M[9];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) M[r * 3 + c] = Rq[r * 3 + c] * sc[c];
    double S[9];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++)
            S[r * 3 + c] = (M[r * 3 + 0] * M[c * 3 + 0] + M[r * 3 + 1] * M[c * 3 + 1]) +
                           M[r * 3 + 2] * M[c * 3 + 2];

    /* local affine approximation of the projection (EWA), evaluated at the
     * view-space mean with its image-plane slope clamped to 1.3x the half fov
     * (slope in binary32, Jacobian in binary64) */
    float limx = 1.3f * (0.5f * (float)cam->W / cam->fx);
    float limy = 1.3f * (0.5f * (float)cam->H / cam->fy);
    float xs = px / pz, ys = py / pz;
    if (xs < -limx) xs = -limx;
    if (xs > limx) xs = limx;
    if (ys < -limy) ys = -limy;
    if (ys > limy) ys = limy;
    float tx = xs * pz, ty = ys * pz;
    double z64 = pz, zz = z64 * z64;
    double J00 = (double)cam->fx / z64, J02 = -((double)cam->fx * (double)tx) / zz;
    double J11 = (double)cam->fy / z64, J12 = -((double)cam->fy * (double)ty) / zz;
    /* T = J * R (2x3) */
    double T[6];
    for (int c = 0; c < 3; c++) {
        T[c] = J00 * (double)R[c] + J02 * (double)R[6 + c];
        T[3 + c] = J11 * (double)R[3 + c] + J12 * (double)R[6 + c];
    }
    /* U = T Sigma3D (2x3); Sigma2D = U T^T plus the 0.3 low-pass */
    double U[6];
    for (int r = 0; r < 2; r++)
        for (int c = 0; c < 3; c++)
            U[r * 3 + c] = (T[r * 3 + 0] * S[0 * 3 + c] + T[r * 3 + 1] * S[1 * 3 + c]) +
                           T[r * 3 + 2] * S[2 * 3 + c];
    double A = ((U[0] * T[0] + U[1] * T[1]) + U[2] * T[2]) + 0.3;
    double B = (U[0] * T[3] + U[1] * T[4]) + U[2] * T[5];
    double C = ((U[3] * T[3] + U[4] * T[4]) + U[5] * T[5]) + 0.3;

    /* image-plane mean */
    g->u = cam->fx * (px / pz) + cam->cx;
    g->v = cam->fy * (py / pz) + cam->cy;

    /* conic = inverse of Sigma2D */
    double det = A * C - B * B;
    if (!(det > 0.0)) return;
    g->A = (float)A; g->B = (float)B; g->C = (float)C;
    g->a = (float)(C / det);
    g->b = (float)(-(B / det));
    g->c = (float)(A / det);
    if (!isfinite(g->A) || !isfinite(g->B) || !isfinite(g->C) || !isfinite(g->a) || !isfinite(g->b) ||
        !isfinite(g->c) || !isfinite(g->u) || !isfinite(g->v))
        return;

    /* opacity-aware modes drop Gaussians that can never reach alpha_min */
    if ((mode & ~OC_CLIP_3SIGMA) != OC_BOX_3SIGMA && !(g->gamma > 0.0f)) return;

    /* view-dependent colour from SH, binary64 */
    {
        double dx = (double)mean[0] - (double)cam->campos[0];
        double dy = (double)mean[1] - (double)cam->campos[1];
        double dz = (double)mean[2] - (double)cam->campos[2];
        double nn = sqrt(dx * dx + dy * dy + dz * dz);
        double Y[16];
        if (nn > 0) { dx /= nn; dy /= nn; dz /= nn; }
        oc_sh_basis(dx, dy, dz, Y);
        int K = (sh_degree + 1) * (sh_degree + 1);
        for (int ch = 0; ch < 3; ch++) {
            double acc = 0.5;
            for (int k = 0; k < K; k++) acc += Y[k] * (double)sh[(int64_t)(k * 3 + ch) * n + i];
            g->rgb[ch] = acc > 0.0 ? acc : 0.0;
        }
    }

    oc_build_boxes(g, mode, cam->W, cam->H);
    g->visible = 1;
}

/* Project every Gaussian; SoA inputs as in the public interface. */
void oc_project(const oc_camera* cam, int64_t n, const float* means, const float* log_scales,
                const float* quats, const float* logits, const float* sh, int sh_degree,
                int mode, oc_gauss* out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        float m[3] = {means[i], means[n + i], means[2 * n + i]};
        float l[3] = {log_scales[i], log_scales[n + i], log_scales[2 * n + i]};
        float q[4] = {quats[i], quats[n + i], quats[2 * n + i], quats[3 * n + i]};
        oc_project_one(cam, m, l, q, logits[i], sh, n, i, sh_degree, mode, &out[i]);
    }
}

/* ------------------------------------------------------------------------- */
/* Tile set of one Gaussian: the plain union of its tile rects (Sec. 3.2).     */
/* ------------------------------------------------------------------------- */
static int oc_in_rects(const oc_gauss* g, int tx, int ty)
{
    for (int r = 0; r < g->nrect; r++)
        if (tx >= g->rect[r][0] && tx <= g->rect[r][1] && ty >= g->rect[r][2] && ty <= g->rect[r][3])
            return 1;
    return 0;
}

/* Writes the tile ids of the union (ascending) into out (may be NULL);
 * returns the count. */
int64_t oc_tile_set(const oc_gauss* g, int tiles_x, int64_t* out)
{
    if (!g->visible || g->nrect == 0) return 0;
    int x0 = g->rect[0][0], x1 = g->rect[0][1], y0 = g->rect[0][2], y1 = g->rect[0][3];
    for (int r = 1; r < g->nrect; r++) {
        if (g->rect[r][0] < x0) x0 = g->rect[r][0];
        if (g->rect[r][1] > x1) x1 = g->rect[r][1];
        if (g->rect[r][2] < y0) y0 = g->rect[r][2];
        if (g->rect[r][3] > y1) y1 = g->rect[r][3];
    }
    int64_t cnt = 0;
    for (int ty = y0; ty <= y1; ty++)
        for (int tx = x0; tx <= x1; tx++)
            if (oc_in_rects(g, tx, ty)) {
                if (out) out[cnt] = (int64_t)ty * tiles_x + tx;
                cnt++;
            }
    return cnt;
}

void oc_tile_counts(const oc_gauss* g, int64_t n, int tiles_x, int64_t* counts)
{
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; i++) counts[i] = oc_tile_set(&g[i], tiles_x, NULL);
}

/* ------------------------------------------------------------------------- */
/* Keys and sort (Sec. 2 DuplicateWithKeys / SortPairs): key = tile << 32 |    */
/* bits(depth); ascending by key, equal keys ascending by Gaussian id.         */
/* ------------------------------------------------------------------------- */
typedef struct { uint64_t key; uint32_t id; uint32_t pad; } oc_pair;

static int oc_pair_cmp(const void* pa, const void* pb)
{
    const oc_pair* a = (const oc_pair*)pa;
    const oc_pair* b = (const oc_pair*)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->id != b->id) return a->id < b->id ? -1 : 1;
    return 0;
}

static uint64_t oc_depth_bits(float d)
{
    uint32_t u;
    memcpy(&u, &d, 4);
    return (uint64_t)u;
}

/* Sorts the pairs ascending by (key, id): chunks sorted with qsort in
 * parallel, then merged pairwise, round by round.  The comparator is a total
 * order (no two pairs share key and id), so the result is the one a single
 * qsort of the whole list gives. */
static void oc_sort_pairs(oc_pair* pr, int64_t total)
{
    const int64_t min_chunk = 1 << 16;
    int64_t chunks = 1;
    while (chunks < 64 && total / (chunks * 2) >= min_chunk) chunks *= 2;
    if (chunks == 1) {
        qsort(pr, (size_t)total, sizeof(oc_pair), oc_pair_cmp);
        return;
    }
    int64_t step = (total + chunks - 1) / chunks;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < chunks; c++) {
        int64_t lo = c * step, hi = lo + step < total ? lo + step : total;
        if (hi > lo) qsort(pr + lo, (size_t)(hi - lo), sizeof(oc_pair), oc_pair_cmp);
    }
    oc_pair* tmp = (oc_pair*)malloc(sizeof(oc_pair) * (size_t)total);
    oc_pair *src = pr, *dst = tmp;
    for (int64_t width = step; width < total; width *= 2) {
        int64_t merges = (total + 2 * width - 1) / (2 * width);
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t m = 0; m < merges; m++) {
            int64_t lo = m * 2 * width;
            int64_t mid = lo + width < total ? lo + width : total;
            int64_t hi = lo + 2 * width < total ? lo + 2 * width : total;
            int64_t a = lo, b = mid, o = lo;
            while (a < mid && b < hi) dst[o++] = oc_pair_cmp(&src[b], &src[a]) < 0 ? src[b++] : src[a++];
            while (a < mid) dst[o++] = src[a++];
            while (b < hi) dst[o++] = src[b++];
        }
        oc_pair* t = src;
        src = dst;
        dst = t;
    }
    if (src != pr) memcpy(pr, src, sizeof(oc_pair) * (size_t)total);
    free(tmp);
}

/* Emits and sorts every pair; returns P (or -1 when P > capacity). */
int64_t oc_pairs(const oc_gauss* g, int64_t n, int tiles_x, int64_t capacity, uint64_t* keys,
                 uint32_t* ids)
{
    int64_t* cnt = (int64_t*)malloc(sizeof(int64_t) * (n + 1));
    oc_tile_counts(g, n, tiles_x, cnt);
    int64_t total = 0;
    for (int64_t i = 0; i < n; i++) {
        int64_t c = cnt[i];
        cnt[i] = total;
        total += c;
    }
    cnt[n] = total;
    if (total > capacity) { free(cnt); return -1; }
    oc_pair* pr = (oc_pair*)malloc(sizeof(oc_pair) * (total > 0 ? total : 1));
#pragma omp parallel
    {
        int64_t* tl = (int64_t*)malloc(sizeof(int64_t) * 65536);
#pragma omp for schedule(dynamic, 1024)
        for (int64_t i = 0; i < n; i++) {
            int64_t m = cnt[i + 1] - cnt[i];
            if (m == 0) continue;
            int64_t* buf = m <= 65536 ? tl : (int64_t*)malloc(sizeof(int64_t) * m);
            oc_tile_set(&g[i], tiles_x, buf);
            for (int64_t k = 0; k < m; k++) {
                pr[cnt[i] + k].key = ((uint64_t)buf[k] << 32) | oc_depth_bits(g[i].depth);
                pr[cnt[i] + k].id = (uint32_t)i;
                pr[cnt[i] + k].pad = 0;
            }
            if (buf != tl) free(buf);
        }
        free(tl);
    }
    oc_sort_pairs(pr, total);
    for (int64_t k = 0; k < total; k++) {
        keys[k] = pr[k].key;
        ids[k] = pr[k].id;
    }
    free(pr);
    free(cnt);
    return total;
}

/* Per-tile ranges [start, end) of the sorted list: lower bounds of t<<32 and
 * (t+1)<<32. */
static int64_t oc_lower_bound(const uint64_t* keys, int64_t P, uint64_t k)
{
    int64_t lo = 0, hi = P;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (keys[mid] < k) lo = mid + 1; else hi = mid;
    }
    return lo;
}

void oc_ranges(const uint64_t* keys, int64_t P, int num_tiles, uint32_t* ranges)
{
    for (int t = 0; t < num_tiles; t++) {
        ranges[2 * t] = (uint32_t)oc_lower_bound(keys, P, (uint64_t)t << 32);
        ranges[2 * t + 1] = (uint32_t)oc_lower_bound(keys, P, (uint64_t)(t + 1) << 32);
    }
}

/* Sorted (depth, id) list of the Gaussians whose tile set holds `tile`:
 * one tile's slice of the sorted pair list, computed on its own. */
int64_t oc_tile_list(const oc_gauss* g, int64_t n, int tiles_x, int64_t tile, uint32_t* out)
{
    int tx = (int)(tile % tiles_x), ty = (int)(tile / tiles_x);
    int64_t m = 0;
    for (int64_t i = 0; i < n; i++)
        if (g[i].visible && oc_in_rects(&g[i], tx, ty)) out[m++] = (uint32_t)i;
    /* order by (depth bits, id) with the same comparator as the pair sort */
    oc_pair* pr = (oc_pair*)malloc(sizeof(oc_pair) * (m > 0 ? m : 1));
    for (int64_t k = 0; k < m; k++) {
        pr[k].key = oc_depth_bits(g[out[k]].depth);
        pr[k].id = out[k];
        pr[k].pad = 0;
    }
    qsort(pr, (size_t)m, sizeof(oc_pair), oc_pair_cmp);
    for (int64_t k = 0; k < m; k++) out[k] = pr[k].id;
    free(pr);
    return m;
}

/* ------------------------------------------------------------------------- */
/* Render, Eq. (2): front-to-back compositing of one pixel over a depth-      */
/* ordered list.  The alpha_min test is taken in its exact log form            */
/* (power >= -gamma/2, i.e. Eq. (4)), in binary32; alpha, T and the colour     */
/* are binary64.  alpha is capped at 0.99; compositing stops before the first  */
/* Gaussian that would push T below 1e-4.                                      */
/* Returns the count of list entries up to and including the last one that    */
/* contributed; *near flags a pixel whose stopping test came within `band`     */
/* (relative) of the 1e-4 threshold.                                           */
/* ------------------------------------------------------------------------- */
float oc_power(const oc_gauss* gi, float pxf, float pyf)
{
    float dx = gi->u - pxf;
    float dy = gi->v - pyf;
    float ha = -0.5f * gi->a, hc = -0.5f * gi->c, nb = -gi->b;
    return fmaf(fmaf(ha, dx, nb * dy), dx, (hc * dy) * dy);
}

uint32_t oc_render_pixel(const oc_gauss* g, const uint32_t* list, int64_t m, int px, int py,
                         const double bg[3], double band, double out_rgb[3], double* out_T,
                         int* near)
{
    double T = 1.0, acc[3] = {0, 0, 0};
    uint32_t last = 0;
    *near = 0;
    for (int64_t k = 0; k < m; k++) {
        const oc_gauss* gi = &g[list[k]];
        float power = oc_power(gi, (float)px, (float)py);
        if (power > 0.0f) continue;
        if (power < -0.5f * gi->gamma) continue;
        double alpha = (double)gi->opacity * exp((double)power);
        if (alpha > 0.99) alpha = 0.99;
        double test_T = T * (1.0 - alpha);
        if (fabs(test_T - 1e-4) <= band * 1e-4) *near = 1;
        if (test_T < 1e-4) break;
        for (int ch = 0; ch < 3; ch++) acc[ch] += gi->rgb[ch] * alpha * T;
        T = test_T;
        last = (uint32_t)(k + 1);
    }
    for (int ch = 0; ch < 3; ch++) out_rgb[ch] = acc[ch] + T * bg[ch];
    *out_T = T;
    return last;
}

/* Full tiled render over the sorted list and ranges. */
void oc_render(const oc_gauss* g, int W, int H, const uint32_t* ranges, const uint32_t* ids,
               const double bg[3], double band, double* image, double* final_T,
               uint32_t* n_contrib, uint8_t* near_mask)
{
    int tiles_x = (W + OC_TILE - 1) / OC_TILE;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < (int64_t)W * H; p++) {
        int px = (int)(p % W), py = (int)(p / W);
        int tile = (py / OC_TILE) * tiles_x + px / OC_TILE;
        uint32_t s = ranges[2 * tile], e = ranges[2 * tile + 1];
        double rgb[3], T;
        int near;
        uint32_t last = oc_render_pixel(g, ids + s, (int64_t)e - s, px, py, bg, band, rgb, &T, &near);
        for (int ch = 0; ch < 3; ch++) image[(int64_t)ch * W * H + p] = rgb[ch];
        final_T[p] = T;
        n_contrib[p] = last;
        near_mask[p] = (uint8_t)near;
    }
}

/* Render of selected pixels only, each from its own tile list computed from
 * the Gaussians directly (no pair list): for parity at full size. */
void oc_render_pixels(const oc_gauss* g, int64_t n, int W, int64_t npix, const int32_t* pix,
                      const double bg[3], double band, double* rgb_out, double* T_out,
                      uint32_t* contrib_out, uint8_t* near_out)
{
    int tiles_x = (W + OC_TILE - 1) / OC_TILE;
#pragma omp parallel
    {
        uint32_t* list = (uint32_t*)malloc(sizeof(uint32_t) * (n > 0 ? n : 1));
#pragma omp for schedule(dynamic, 1)
        for (int64_t k = 0; k < npix; k++) {
            int px = pix[2 * k], py = pix[2 * k + 1];
            int64_t tile = (int64_t)(py / OC_TILE) * tiles_x + px / OC_TILE;
            int64_t m = oc_tile_list(g, n, tiles_x, tile, list);
            int near;
            contrib_out[k] = oc_render_pixel(g, list, m, px, py, bg, band, rgb_out + 3 * k, &T_out[k], &near);
            near_out[k] = (uint8_t)near;
        }
        free(list);
    }
}

/* Tile-free render: every visible Gaussian, in (depth, id) order, at every
 * pixel.  Differs from the tiled render only where a box misses a pixel. */
void oc_render_brute(const oc_gauss* g, int64_t n, int W, int H, const double bg[3], double band,
                     double* image, double* final_T, uint32_t* n_contrib, uint8_t* near_mask)
{
    oc_pair* pr = (oc_pair*)malloc(sizeof(oc_pair) * (n > 0 ? n : 1));
    int64_t m = 0;
    for (int64_t i = 0; i < n; i++)
        if (g[i].visible) {
            pr[m].key = oc_depth_bits(g[i].depth);
            pr[m].id = (uint32_t)i;
            pr[m].pad = 0;
            m++;
        }
    qsort(pr, (size_t)m, sizeof(oc_pair), oc_pair_cmp);
    uint32_t* list = (uint32_t*)malloc(sizeof(uint32_t) * (m > 0 ? m : 1));
    for (int64_t k = 0; k < m; k++) list[k] = pr[k].id;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < (int64_t)W * H; p++) {
        int px = (int)(p % W), py = (int)(p / W);
        double rgb[3], T;
        int near;
        uint32_t last = oc_render_pixel(g, list, m, px, py, bg, band, rgb, &T, &near);
        for (int ch = 0; ch < 3; ch++) image[(int64_t)ch * W * H + p] = rgb[ch];
        final_T[p] = T;
        n_contrib[p] = last;
        near_mask[p] = (uint8_t)near;
    }
    free(list);
    free(pr);
}

/* ------------------------------------------------------------------------- */
/* Coverage audit (the paper's conservativeness claim, Sec. 1 and Sec. 3):     */
/* every tile holding a pixel sample p with q(p) <= gamma * s^2 must be in the  */
/* tile set, where q is the binary64 quadratic form of the stored Sigma2D and  */
/* s = 1 - margin / r_min shrinks the ellipse by `margin` pixels to absorb the */
/* binary32 rounding of the box extents.  Also counts the exact-sample pairs   */
/* (tiles with a sample at q <= gamma) and reports QuadBox-not-in-box events.  */
/* Returns the number of missed (tile, Gaussian) pairs.                        */
/* ------------------------------------------------------------------------- */
int64_t oc_coverage_audit(const oc_gauss* g, int64_t n, int W, int H, double margin,
                          int64_t* exact_pairs, int64_t* missed_ids, int64_t max_missed)
{
    int tiles_x = (W + OC_TILE - 1) / OC_TILE, tiles_y = (H + OC_TILE - 1) / OC_TILE;
    int64_t missed = 0, exact = 0;
    for (int64_t i = 0; i < n; i++) {
        const oc_gauss* gi = &g[i];
        if (!gi->visible || !(gi->gamma > 0.0f)) continue;
        double A = gi->A, B = gi->B, C = gi->C, gam = gi->gamma;
        double det = A * C - B * B;
        double ia = C / det, ib = -B / det, ic = A / det; /* inverse in binary64 */
        /* smallest semi-axis: sqrt(gamma * lambda_min(Sigma2D)) */
        double mid = 0.5 * (A + C), rad = sqrt(0.25 * (A - C) * (A - C) + B * B);
        double lmin = mid - rad;
        double rmin = sqrt(gam * (lmin > 0 ? lmin : 0));
        double s = rmin > 0 ? 1.0 - margin / rmin : 0.0;
        if (s < 0) s = 0;
        double xr = sqrt(gam * A) + 1.0, yr = sqrt(gam * C) + 1.0;
        int tx0 = (int)floor((gi->u - xr) / OC_TILE), tx1 = (int)floor((gi->u + xr) / OC_TILE);
        int ty0 = (int)floor((gi->v - yr) / OC_TILE), ty1 = (int)floor((gi->v + yr) / OC_TILE);
        if (tx0 < 0) tx0 = 0;
        if (ty0 < 0) ty0 = 0;
        if (tx1 > tiles_x - 1) tx1 = tiles_x - 1;
        if (ty1 > tiles_y - 1) ty1 = tiles_y - 1;
        for (int ty = ty0; ty <= ty1; ty++)
            for (int tx = tx0; tx <= tx1; tx++) {
                int need = 0, any = 0;
                for (int py = ty * OC_TILE; py < ty * OC_TILE + OC_TILE && py < H; py++)
                    for (int px = tx * OC_TILE; px < tx * OC_TILE + OC_TILE && px < W; px++) {
                        double dx = (double)px - gi->u, dy = (double)py - gi->v;
                        double q = ia * dx * dx + 2.0 * ib * dx * dy + ic * dy * dy;
                        if (q <= gam) any = 1;
                        if (q <= gam * s * s) need = 1;
                    }
                exact += any;
                if (need && !oc_in_rects(gi, tx, ty)) {
                    if (missed < max_missed && missed_ids) missed_ids[missed] = i;
                    missed++;
                }
            }
    }
    if (exact_pairs) *exact_pairs = exact;
    return missed;
}

/* Worker threads of the parallel loops (the CPU baseline times the oracle
 * on all cores and on one). */
#ifdef _OPENMP
#include <omp.h>
void oc_set_threads(int32_t t) { omp_set_num_threads(t > 0 ? t : 1); }
int32_t oc_threads(void) { return (int32_t)omp_get_max_threads(); }
#else
void oc_set_threads(int32_t t) { (void)t; }
int32_t oc_threads(void) { return 1; }
#endif

/* Struct layout, so the Python side can check its view of oc_gauss. */
#include <stddef.h>
void oc_layout(int64_t* out)
{
    out[0] = (int64_t)sizeof(oc_gauss);
    out[1] = (int64_t)offsetof(oc_gauss, visible);
    out[2] = (int64_t)offsetof(oc_gauss, nrect);
    out[3] = (int64_t)offsetof(oc_gauss, rect);
    out[4] = (int64_t)offsetof(oc_gauss, rgb);
    out[5] = (int64_t)sizeof(oc_camera);
}

/* ========================================================================= */
/* Binary64 forward and its gradient (the rasterizer is differentiable: the  */
/* paper trains through it, Sec. 4.1).  This is a plain binary64 evaluation  */
/* of the same function -- projection (Sec. 2, Eq. 1), the 1/255 cutoff     */
/* (Eq. 4) and Eq. (2) over every visible Gaussian in (depth, id) order, no  */
/* tiles -- and its reverse-mode derivative, written out by hand.  Order,   */
/* visibility and the cutoff are the rasterizer's binary32 decisions         */
/* (oc_decide32); the rest is binary64.                                      */
/* ========================================================================= */

typedef struct {
    int visible;
    double p[3], s[3], o, qn[4], qnorm, Rq[9], M[9], S[9];
    double limx, limy, xs, ys, clampx, clampy;  /* clamp flags: 0 free, +-1 clamped */
    double J00, J02, J11, J12, T[6];
    double A, B, C, det, a, b, c, u, v, gamma;
    double dir[3], dnorm, rgb_raw[3], rgb[3];
} oc_g64;

static void oc_project64_one(const oc_camera* cam, const double mean[3], const double ls[3],
                             const double q[4], double logit, const double* shc, int K, oc_g64* g)
{
    memset(g, 0, sizeof(*g));
    const float* Rc = cam->R;
    for (int r = 0; r < 3; r++)
        g->p[r] = (double)Rc[3 * r] * mean[0] + (double)Rc[3 * r + 1] * mean[1] + (double)Rc[3 * r + 2] * mean[2] +
                  (double)cam->t[r];
    double pz = g->p[2];
    if (!(pz > (double)cam->near_plane)) return;
    for (int k = 0; k < 3; k++) g->s[k] = exp(ls[k]);
    g->o = 1.0 / (1.0 + exp(-logit));
    g->gamma = 2.0 * log(255.0 * g->o);
    double n2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    if (!(n2 > 0)) return;
    g->qnorm = sqrt(n2);
    for (int k = 0; k < 4; k++) g->qn[k] = q[k] / g->qnorm;
    double w = g->qn[0], x = g->qn[1], y = g->qn[2], z = g->qn[3];
    double* R = g->Rq;
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) g->M[3 * r + c] = R[3 * r + c] * g->s[c];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++)
            g->S[3 * r + c] = g->M[3 * r] * g->M[3 * c] + g->M[3 * r + 1] * g->M[3 * c + 1] + g->M[3 * r + 2] * g->M[3 * c + 2];
    g->limx = 1.3 * (0.5 * cam->W / (double)cam->fx);
    g->limy = 1.3 * (0.5 * cam->H / (double)cam->fy);
    double xs = g->p[0] / pz, ys = g->p[1] / pz;
    g->clampx = xs < -g->limx ? -1 : (xs > g->limx ? 1 : 0);
    g->clampy = ys < -g->limy ? -1 : (ys > g->limy ? 1 : 0);
    if (g->clampx) xs = g->clampx * g->limx;
    if (g->clampy) ys = g->clampy * g->limy;
    g->xs = xs; g->ys = ys;
    double tx = xs * pz, ty = ys * pz;
    g->J00 = cam->fx / pz; g->J02 = -cam->fx * tx / (pz * pz);
    g->J11 = cam->fy / pz; g->J12 = -cam->fy * ty / (pz * pz);
    for (int c = 0; c < 3; c++) {
        g->T[c] = g->J00 * Rc[c] + g->J02 * Rc[6 + c];
        g->T[3 + c] = g->J11 * Rc[3 + c] + g->J12 * Rc[6 + c];
    }
    double U[6];
    for (int r = 0; r < 2; r++)
        for (int c = 0; c < 3; c++)
            U[3 * r + c] = g->T[3 * r] * g->S[c] + g->T[3 * r + 1] * g->S[3 + c] + g->T[3 * r + 2] * g->S[6 + c];
    g->A = U[0] * g->T[0] + U[1] * g->T[1] + U[2] * g->T[2] + 0.3;
    g->B = U[0] * g->T[3] + U[1] * g->T[4] + U[2] * g->T[5];
    g->C = U[3] * g->T[3] + U[4] * g->T[4] + U[5] * g->T[5] + 0.3;
    g->u = cam->fx * (g->p[0] / pz) + cam->cx;
    g->v = cam->fy * (g->p[1] / pz) + cam->cy;
    g->det = g->A * g->C - g->B * g->B;
    if (!(g->det > 0)) return;
    g->a = g->C / g->det; g->b = -g->B / g->det; g->c = g->A / g->det;
    if (!(g->gamma > 0)) return;
    double d[3];
    for (int k = 0; k < 3; k++) d[k] = mean[k] - (double)cam->campos[k];
    g->dnorm = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int k = 0; k < 3; k++) g->dir[k] = d[k] / g->dnorm;
    double Y[16];
    oc_sh_basis(g->dir[0], g->dir[1], g->dir[2], Y);
    for (int ch = 0; ch < 3; ch++) {
        double acc = 0.5;
        for (int k = 0; k < K; k++) acc += Y[k] * shc[k * 3 + ch];
        g->rgb_raw[ch] = acc;
        g->rgb[ch] = acc > 0 ? acc : 0;
    }
    g->visible = 1;
}

/* Gradient of the SH basis polynomials with respect to (x, y, z). */
static void oc_sh_basis_grad(double x, double y, double z, double G[16][3])
{
    const double pi = 3.14159265358979323846;
    const double k1 = sqrt(3.0 / (4.0 * pi));
    const double k2a = 0.5 * sqrt(15.0 / pi), k2b = 0.25 * sqrt(5.0 / pi), k2c = 0.25 * sqrt(15.0 / pi);
    const double k3a = 0.25 * sqrt(35.0 / (2.0 * pi)), k3b = 0.5 * sqrt(105.0 / pi);
    const double k3c = 0.25 * sqrt(21.0 / (2.0 * pi)), k3d = 0.25 * sqrt(7.0 / pi), k3e = 0.25 * sqrt(105.0 / pi);
    double xx = x * x, yy = y * y, zz = z * z;
    double t[16][3] = {
        {0, 0, 0},
        {0, -k1, 0},
        {0, 0, k1},
        {-k1, 0, 0},
        {k2a * y, k2a * x, 0},
        {0, -k2a * z, -k2a * y},
        {-2 * k2b * x, -2 * k2b * y, 4 * k2b * z},
        {-k2a * z, 0, -k2a * x},
        {2 * k2c * x, -2 * k2c * y, 0},
        {-6 * k3a * x * y, -k3a * (3 * xx - 3 * yy), 0},
        {k3b * y * z, k3b * x * z, k3b * x * y},
        {2 * k3c * x * y, -k3c * (4 * zz - xx - 3 * yy), -8 * k3c * y * z},
        {-6 * k3d * x * z, -6 * k3d * y * z, k3d * (6 * zz - 3 * xx - 3 * yy)},
        {-k3c * (4 * zz - 3 * xx - yy), 2 * k3c * x * y, -8 * k3c * x * z},
        {2 * k3e * x * z, -2 * k3e * y * z, k3e * (xx - yy)},
        {-k3a * (3 * xx - 3 * yy), 6 * k3a * x * y, 0},
    };
    memcpy(G, t, sizeof(t));
}

typedef struct { uint64_t key; uint32_t id; uint32_t pad; } oc_dpair;

static int oc_dpair_cmp(const void* pa, const void* pb)
{
    const oc_dpair* a = (const oc_dpair*)pa;
    const oc_dpair* b = (const oc_dpair*)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return a->id < b->id ? -1 : (a->id > b->id);
}

/* The decisions of the rasterized image, taken in binary32 exactly as the
 * rasterizer takes them (the depth sort key and the alpha cutoff of Eq. (4)
 * are binary32 quantities), once, from the unperturbed parameters:
 *   - which Gaussians are visible, from the binary32 projection;
 *   - their order: binary32 depth bits, ties by id (the depth part of the
 *     sort key);
 *   - per pixel, whether an entry passes the cutoff: its binary32 power lies
 *     in [-gamma/2, 0] (oc_power).
 * On that fixed decision set the image is a smooth function of the parameters
 * (up to the 0.99 cap and the stop at T < 1e-4, taken in binary64), which
 * oc_forward64 evaluates and oc_backward64 differentiates. */
static oc_gauss* oc_decide32(const oc_camera* cam, int64_t n, const float* means, const float* ls,
                             const float* quats, const float* logits, const float* sh, int sh_degree,
                             uint32_t* order, int64_t* m_out)
{
    oc_gauss* d = (oc_gauss*)malloc(sizeof(oc_gauss) * (n > 0 ? n : 1));
    oc_project(cam, n, means, ls, quats, logits, sh, sh_degree, OC_BOX_QUADBOX, d);
    oc_dpair* pr = (oc_dpair*)malloc(sizeof(oc_dpair) * (n > 0 ? n : 1));
    int64_t m = 0;
    for (int64_t i = 0; i < n; i++)
        if (d[i].visible) {
            uint32_t bits;
            memcpy(&bits, &d[i].depth, 4);
            pr[m].key = bits; pr[m].id = (uint32_t)i; pr[m].pad = 0; m++;
        }
    qsort(pr, (size_t)m, sizeof(oc_dpair), oc_dpair_cmp);
    for (int64_t k = 0; k < m; k++) order[k] = pr[k].id;
    free(pr);
    *m_out = m;
    return d;
}

/* Cutoff decision of one entry at pixel (px, py), Eq. (4) in binary32. */
static int oc_passes32(const oc_gauss* d, int px, int py)
{
    float power = oc_power(d, (float)px, (float)py);
    return !(power > 0.0f) && !(power < -0.5f * d->gamma);
}

static void oc_unpack(const float* means, const float* ls, const float* quats, const float* logits,
                      const float* sh, int64_t n, int64_t i, int K, const double* delta, double m[3],
                      double l[3], double q[4], double* x, double shc[48])
{
    /* parameter vector of Gaussian i: mean(3) lscale(3) quat(4) logit(1) sh(K*3) */
    const double* dd = delta;
    for (int k = 0; k < 3; k++) m[k] = means[k * n + i] + (dd ? dd[k] : 0);
    for (int k = 0; k < 3; k++) l[k] = ls[k * n + i] + (dd ? dd[3 + k] : 0);
    for (int k = 0; k < 4; k++) q[k] = quats[k * n + i] + (dd ? dd[6 + k] : 0);
    *x = logits[i] + (dd ? dd[10] : 0);
    for (int k = 0; k < K * 3; k++) shc[k] = sh[(int64_t)k * n + i] + (dd ? dd[11 + k] : 0);
}

/* The binary64 projection of every Gaussian (no perturbation), 16 doubles
 * each: visible, u, v, depth, A, B, C, a, b, c, o, gamma, r, g, b, 0.
 * Exposed so that the binary64 path can be checked against the binary32
 * projection (oc_project), which is pinned on its own. */
void oc_project64(const oc_camera* cam, int64_t n, const float* means, const float* ls, const float* quats,
                  const float* logits, const float* sh, int sh_degree, double* out)
{
    int K = (sh_degree + 1) * (sh_degree + 1);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        double m[3], l[3], q[4], x, shc[48];
        oc_g64 g;
        oc_unpack(means, ls, quats, logits, sh, n, i, K, NULL, m, l, q, &x, shc);
        oc_project64_one(cam, m, l, q, x, shc, K, &g);
        double* o = out + 16 * i;
        o[0] = g.visible; o[1] = g.u; o[2] = g.v; o[3] = g.p[2];
        o[4] = g.A; o[5] = g.B; o[6] = g.C; o[7] = g.a; o[8] = g.b; o[9] = g.c;
        o[10] = g.o; o[11] = g.gamma; o[12] = g.rgb[0]; o[13] = g.rgb[1]; o[14] = g.rgb[2]; o[15] = 0.0;
    }
}

/* Binary64 render of all pixels; optional perturbation of one parameter of
 * one Gaussian (for finite differences).  Returns the image [3][H][W]. */
void oc_forward64(const oc_camera* cam, int64_t n, const float* means, const float* ls, const float* quats,
                  const float* logits, const float* sh, int sh_degree, const double bg[3], int64_t pert_id,
                  int pert_param, double pert_h, double* image)
{
    int K = (sh_degree + 1) * (sh_degree + 1);
    oc_g64* g = (oc_g64*)malloc(sizeof(oc_g64) * (n > 0 ? n : 1));
    for (int64_t i = 0; i < n; i++) {
        double delta[59] = {0};
        if (i == pert_id) delta[pert_param] = pert_h;
        double m[3], l[3], q[4], x, shc[48];
        oc_unpack(means, ls, quats, logits, sh, n, i, K, delta, m, l, q, &x, shc);
        oc_project64_one(cam, m, l, q, x, shc, K, &g[i]);
    }
    uint32_t* order = (uint32_t*)malloc(sizeof(uint32_t) * (n > 0 ? n : 1));
    int64_t m;
    oc_gauss* d = oc_decide32(cam, n, means, ls, quats, logits, sh, sh_degree, order, &m);
    int W = cam->W, H = cam->H;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t pidx = 0; pidx < (int64_t)W * H; pidx++) {
        double px = (double)(pidx % W), py = (double)(pidx / W);
        double T = 1, acc[3] = {0, 0, 0};
        for (int64_t k = 0; k < m; k++) {
            const oc_g64* gi = &g[order[k]];
            if (!gi->visible || !oc_passes32(&d[order[k]], (int)px, (int)py)) continue;
            double dx = gi->u - px, dy = gi->v - py;
            double power = -0.5 * (gi->a * dx * dx + gi->c * dy * dy) - gi->b * dx * dy;
            double alpha = gi->o * exp(power);
            if (alpha > 0.99) alpha = 0.99;
            double tT = T * (1 - alpha);
            if (tT < 1e-4) break;
            for (int ch = 0; ch < 3; ch++) acc[ch] += gi->rgb[ch] * alpha * T;
            T = tT;
        }
        for (int ch = 0; ch < 3; ch++) image[(int64_t)ch * W * H + pidx] = acc[ch] + T * bg[ch];
    }
    free(d);
    free(order);
    free(g);
}

/* Reverse mode of oc_forward64: given dL/dimage [3][H][W], the gradient with
 * respect to every parameter, written per Gaussian as 59 doubles:
 * mean(3) log_scale(3) quat(4) logit(1) sh(48, coefficient k*3+ch). */
void oc_backward64(const oc_camera* cam, int64_t n, const float* means, const float* ls, const float* quats,
                   const float* logits, const float* sh, int sh_degree, const double bg[3], const double* dL_dimg,
                   double band, uint8_t* near, double* grad, double* grad2d)
{
    int K = (sh_degree + 1) * (sh_degree + 1);
    int W = cam->W, H = cam->H;
    oc_g64* g = (oc_g64*)malloc(sizeof(oc_g64) * (n > 0 ? n : 1));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        double m[3], l[3], q[4], x, shc[48];
        oc_unpack(means, ls, quats, logits, sh, n, i, K, NULL, m, l, q, &x, shc);
        oc_project64_one(cam, m, l, q, x, shc, K, &g[i]);
    }
    uint32_t* order = (uint32_t*)malloc(sizeof(uint32_t) * (n > 0 ? n : 1));
    int64_t m;
    oc_gauss* d = oc_decide32(cam, n, means, ls, quats, logits, sh, sh_degree, order, &m);
    if (near) memset(near, 0, (size_t)W * H);
    /* per-Gaussian 2D gradients: u v a b c o r g b */
    double* g2 = (double*)calloc((size_t)(n > 0 ? n : 1) * 9, sizeof(double));
#pragma omp parallel
    {
        int64_t* list = (int64_t*)malloc(sizeof(int64_t) * (m > 0 ? m : 1));
        double* al = (double*)malloc(sizeof(double) * (m > 0 ? m : 1));
        double* Ts = (double*)malloc(sizeof(double) * (m > 0 ? m : 1));
#pragma omp for schedule(dynamic, 8)
        for (int64_t pidx = 0; pidx < (int64_t)W * H; pidx++) {
            double dC[3], rest[3];
            for (int ch = 0; ch < 3; ch++) dC[ch] = dL_dimg[(int64_t)ch * W * H + pidx];
            if (dC[0] == 0 && dC[1] == 0 && dC[2] == 0) continue;   /* contributes nothing */
            double px = (double)(pidx % W), py = (double)(pidx / W);
            double T = 1;
            int64_t cnt = 0;
            int close = 0;
            for (int64_t k = 0; k < m; k++) {
                const oc_g64* gi = &g[order[k]];
                if (!gi->visible || !oc_passes32(&d[order[k]], (int)px, (int)py)) continue;
                double dx = gi->u - px, dy = gi->v - py;
                double power = -0.5 * (gi->a * dx * dx + gi->c * dy * dy) - gi->b * dx * dy;
                double alpha = gi->o * exp(power);
                if (fabs(alpha - 0.99) <= band * 0.99) close = 1;
                if (alpha > 0.99) alpha = 0.99;
                double tT = T * (1 - alpha);
                if (fabs(tT - 1e-4) <= band * 1e-4) close = 1;
                if (tT < 1e-4) break;
                list[cnt] = order[k]; al[cnt] = alpha; Ts[cnt] = T; cnt++;
                T = tT;
            }
            if (near) near[pidx] = (uint8_t)close;
            for (int ch = 0; ch < 3; ch++) rest[ch] = T * bg[ch];   /* what lies behind */
            for (int64_t k = cnt - 1; k >= 0; k--) {
                int64_t i = list[k];
                const oc_g64* gi = &g[i];
                double alpha = al[k], Ti = Ts[k];
                double dalpha = 0;
                for (int ch = 0; ch < 3; ch++) {
                    double v = alpha * Ti * dC[ch];
#pragma omp atomic
                    g2[9 * i + 6 + ch] += v;
                    dalpha += dC[ch] * (gi->rgb[ch] * Ti - rest[ch] / (1 - alpha));
                    rest[ch] += gi->rgb[ch] * alpha * Ti;
                }
                double dx = gi->u - px, dy = gi->v - py;
                double power = -0.5 * (gi->a * dx * dx + gi->c * dy * dy) - gi->b * dx * dy;
                double e = exp(power);
                if (gi->o * e > 0.99) continue;    /* capped: alpha is constant */
                double dpower = dalpha * alpha;
                double v[6] = {dpower * -(gi->a * dx + gi->b * dy), dpower * -(gi->c * dy + gi->b * dx),
                               dpower * -0.5 * dx * dx, dpower * -dx * dy, dpower * -0.5 * dy * dy, dalpha * e};
                for (int c = 0; c < 6; c++) {
#pragma omp atomic
                    g2[9 * i + c] += v[c];
                }
            }
        }
        free(Ts); free(al); free(list);
    }
    memset(grad, 0, sizeof(double) * 59 * (size_t)n);
    const float* Rc = cam->R;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        const oc_g64* gi = &g[i];
        if (!gi->visible) continue;
        double* out = grad + 59 * i;
        const double* d2 = g2 + 9 * i;
        /* colour: clamp, SH coefficients, view direction */
        double Y[16], GY[16][3], drgb[3];
        oc_sh_basis(gi->dir[0], gi->dir[1], gi->dir[2], Y);
        oc_sh_basis_grad(gi->dir[0], gi->dir[1], gi->dir[2], GY);
        double ddir[3] = {0, 0, 0};
        double m_[3], l_[3], q_[4], x_, shc[48];
        oc_unpack(means, ls, quats, logits, sh, n, i, K, NULL, m_, l_, q_, &x_, shc);
        for (int ch = 0; ch < 3; ch++) {
            drgb[ch] = gi->rgb_raw[ch] > 0 ? d2[6 + ch] : 0;
            for (int k = 0; k < K; k++) {
                out[11 + k * 3 + ch] = Y[k] * drgb[ch];
                for (int c = 0; c < 3; c++) ddir[c] += GY[k][c] * shc[k * 3 + ch] * drgb[ch];
            }
        }
        double dd = ddir[0] * gi->dir[0] + ddir[1] * gi->dir[1] + ddir[2] * gi->dir[2];
        for (int c = 0; c < 3; c++) out[c] += (ddir[c] - gi->dir[c] * dd) / gi->dnorm;
        /* opacity */
        out[10] = d2[5] * gi->o * (1 - gi->o);
        /* conic (a, b, c) -> Sigma2D (A, B, C) */
        double det2 = gi->det * gi->det, A = gi->A, B = gi->B, C = gi->C;
        double da = d2[2], db = d2[3], dc = d2[4];
        double dA = da * (-C * C / det2) + db * (B * C / det2) + dc * (-B * B / det2);
        double dB = da * (2 * B * C / det2) + db * (-1 / gi->det - 2 * B * B / det2) + dc * (2 * A * B / det2);
        double dCc = da * (-B * B / det2) + db * (B * A / det2) + dc * (-A * A / det2);
        /* Sigma2D = T Sigma T^T: symmetric cotangent G */
        double G[2][2] = {{dA, 0.5 * dB}, {0.5 * dB, dCc}};
        const double* T = gi->T;
        double dS[9];  /* T^T G T */
        for (int r = 0; r < 3; r++)
            for (int c = 0; c < 3; c++) {
                double acc = 0;
                for (int p = 0; p < 2; p++)
                    for (int q2 = 0; q2 < 2; q2++) acc += T[3 * p + r] * G[p][q2] * T[3 * q2 + c];
                dS[3 * r + c] = acc;
            }
        double dT[6];  /* 2 G T S */
        for (int p = 0; p < 2; p++)
            for (int c = 0; c < 3; c++) {
                double acc = 0;
                for (int q2 = 0; q2 < 2; q2++)
                    for (int k = 0; k < 3; k++) acc += G[p][q2] * T[3 * q2 + k] * gi->S[3 * k + c];
                dT[3 * p + c] = 2 * acc;
            }
        /* T = J R: J00, J02 act on rows 0 and 2 of R; J11, J12 on rows 1 and 2 */
        double dJ00 = 0, dJ02 = 0, dJ11 = 0, dJ12 = 0;
        for (int c = 0; c < 3; c++) {
            dJ00 += dT[c] * Rc[c];
            dJ02 += dT[c] * Rc[6 + c];
            dJ11 += dT[3 + c] * Rc[3 + c];
            dJ12 += dT[3 + c] * Rc[6 + c];
        }
        double pz = gi->p[2], fx = cam->fx, fy = cam->fy;
        double tx = gi->xs * pz, ty = gi->ys * pz;
        double dp[3] = {0, 0, 0};
        /* J00 = fx/pz, J11 = fy/pz, J02 = -fx tx/pz^2, J12 = -fy ty/pz^2 */
        dp[2] += dJ00 * (-fx / (pz * pz)) + dJ11 * (-fy / (pz * pz));
        double dtx = dJ02 * (-fx / (pz * pz)), dty = dJ12 * (-fy / (pz * pz));
        dp[2] += dJ02 * (2 * fx * tx / (pz * pz * pz)) + dJ12 * (2 * fy * ty / (pz * pz * pz));
        if (gi->clampx == 0) dp[0] += dtx; else dp[2] += dtx * gi->clampx * gi->limx;
        if (gi->clampy == 0) dp[1] += dty; else dp[2] += dty * gi->clampy * gi->limy;
        /* mean2D */
        dp[0] += d2[0] * fx / pz;
        dp[2] += d2[0] * (-fx * gi->p[0] / (pz * pz));
        dp[1] += d2[1] * fy / pz;
        dp[2] += d2[1] * (-fy * gi->p[1] / (pz * pz));
        for (int c = 0; c < 3; c++) out[c] += Rc[c] * dp[0] + Rc[3 + c] * dp[1] + Rc[6 + c] * dp[2];
        /* Sigma = M M^T, M = R diag(s) */
        double dM[9];
        for (int r = 0; r < 3; r++)
            for (int c = 0; c < 3; c++)
                dM[3 * r + c] = 2 * (dS[3 * r] * gi->M[c] + dS[3 * r + 1] * gi->M[3 + c] + dS[3 * r + 2] * gi->M[6 + c]);
        double dR[9];
        for (int r = 0; r < 3; r++)
            for (int c = 0; c < 3; c++) dR[3 * r + c] = dM[3 * r + c] * gi->s[c];
        for (int c = 0; c < 3; c++) {
            double dsc = dM[c] * gi->Rq[c] + dM[3 + c] * gi->Rq[3 + c] + dM[6 + c] * gi->Rq[6 + c];
            out[3 + c] = dsc * gi->s[c];
        }
        double w = gi->qn[0], x = gi->qn[1], y = gi->qn[2], z = gi->qn[3];
        double dq[4];
        dq[0] = 2 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
        dq[1] = 2 * (y * dR[1] + z * dR[2] + y * dR[3] - 2 * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] - 2 * x * dR[8]);
        dq[2] = 2 * (-2 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] - 2 * y * dR[8]);
        dq[3] = 2 * (-2 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2 * z * dR[4] + y * dR[5] + x * dR[6] + y * dR[7]);
        double qd = w * dq[0] + x * dq[1] + y * dq[2] + z * dq[3];
        for (int k = 0; k < 4; k++) out[6 + k] = (dq[k] - gi->qn[k] * qd) / gi->qnorm;
    }
    if (grad2d) memcpy(grad2d, g2, sizeof(double) * 9 * (size_t)n);
    free(g2); free(d); free(order); free(g);
}
