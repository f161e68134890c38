// qb_project: Gaussian-parallel preprocess (Sec. 2: EWA projection of Eq. (1)
// Gaussians; Sec. 3.1: box construction; Sec. 3.2: tile-space bounds and the
// QPass tile count).
//
// One lane per Gaussian; inputs are structure-of-arrays so every plane is read
// with coalesced 256-byte wave accesses, outputs are 48-byte records and
// 32-byte rect sets written as 16-byte vectors (qb_project_ex also writes
// each Gaussian's 4-byte depth-sort key).  The work is HBM-bound (236 B
// read per SH3 Gaussian), so the arithmetic follows the fixed binary32
// operation order that makes keys reproducible: no contraction (the library is
// built with -ffp-contract=off), correctly rounded divide/sqrt, and the three
// transcendentals in binary64 rounded once.
#include "qb_common.h"

namespace {

struct ProjCam {
    int W, H, tiles_x, tiles_y;
    float fx, fy, cx, cy, near_plane;
    float R[9], t[3], campos[3];
    float limx, limy;
};

// Tile range of the integer pixel samples in the closed interval [x0, x1] of
// an axis with n pixels; false when none lies inside.
__device__ __forceinline__ bool axis_tiles(float x0, float x1, int n, int* t0, int* t1)
{
    float hi = (float)(n - 1);
    if (!(x1 >= 0.0f) || !(x0 <= hi)) return false;
    float lo_c = x0 > 0.0f ? x0 : 0.0f;
    float hi_c = x1 < hi ? x1 : hi;
    int p0 = (int)ceilf(lo_c);
    int p1 = (int)floorf(hi_c);
    if (p0 > p1) return false;
    *t0 = p0 / QB_TILE;
    *t1 = p1 / QB_TILE;
    return true;
}

__device__ __forceinline__ QRect box_rect(float x0, float x1, float y0, float y1, int W, int H)
{
    QRect r{1, 0, 1, 0};
    int a, b, c, d;
    if (axis_tiles(x0, x1, W, &a, &b) && axis_tiles(y0, y1, H, &c, &d)) r = QRect{a, b, c, d};
    return r;
}

// SH coefficients of one Gaussian, (DEG+1)^2 x 3 (plane k*3 + ch of sh).
template <int DEG>
struct ShCoef {
    static constexpr int K = (DEG + 1) * (DEG + 1);
    float c[K * 3];
};

template <int DEG>
__device__ __forceinline__ void sh_load(const float* __restrict__ sh, int64_t n, int64_t i, ShCoef<DEG>& s)
{
#pragma unroll
    for (int k = 0; k < ShCoef<DEG>::K * 3; ++k) s.c[k] = __ldg(sh + (int64_t)k * n + i);
}

// Real SH basis of degree <= 3 (Condon-Shortley phase, index l*l + l + m).
template <int DEG>
__device__ __forceinline__ void sh_colour(const ShCoef<DEG>& s, float x, float y, float z, float rgb[3])
{
    constexpr int deg = DEG;
    const float k00 = 0.28209479177387814f;   // 1 / (2 sqrt(pi))
    const float k1 = 0.48860251190291992f;    // sqrt(3 / (4 pi))
    const float k2a = 1.0925484305920792f;    // sqrt(15 / pi) / 2
    const float k2b = 0.31539156525252005f;   // sqrt(5 / pi) / 4
    const float k2c = 0.54627421529603959f;   // sqrt(15 / pi) / 4
    const float k3a = 0.59004358992664352f;   // sqrt(35 / (2 pi)) / 4
    const float k3b = 2.8906114426405538f;    // sqrt(105 / pi) / 2
    const float k3c = 0.45704579946446572f;   // sqrt(21 / (2 pi)) / 4
    const float k3d = 0.3731763325901154f;    // sqrt(7 / pi) / 4
    const float k3e = 1.4453057213202769f;    // sqrt(105 / pi) / 4
    float Y[16];
    float xx = x * x, yy = y * y, zz = z * z;
    Y[0] = k00;
    constexpr int K = ShCoef<DEG>::K;
    if (deg >= 1) {
        Y[1] = -k1 * y;
        Y[2] = k1 * z;
        Y[3] = -k1 * x;
    }
    if (deg >= 2) {
        Y[4] = k2a * x * y;
        Y[5] = -k2a * y * z;
        Y[6] = k2b * (2.0f * zz - xx - yy);
        Y[7] = -k2a * x * z;
        Y[8] = k2c * (xx - yy);
    }
    if (deg >= 3) {
        Y[9] = -k3a * y * (3.0f * xx - yy);
        Y[10] = k3b * x * y * z;
        Y[11] = -k3c * y * (4.0f * zz - xx - yy);
        Y[12] = k3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
        Y[13] = -k3c * x * (4.0f * zz - xx - yy);
        Y[14] = k3e * z * (xx - yy);
        Y[15] = -k3a * x * (xx - 3.0f * yy);
    }
    float acc[3] = {0.5f, 0.5f, 0.5f};
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) acc[ch] = fmaf(Y[k], s.c[k * 3 + ch], acc[ch]);
    }
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) rgb[ch] = acc[ch] > 0.0f ? acc[ch] : 0.0f;
}

// The activations (Eq. (3) for gamma), each evaluated in binary64 and
// rounded once to binary32: scale s = exp(log_scale), opacity o =
// sigmoid(logit), gamma = 2 ln(o / (1/255)).
__device__ __forceinline__ float act_scale(float l) { return (float)exp((double)l); }
__device__ __forceinline__ float act_opacity(float x) { return (float)(1.0 / (1.0 + exp(-(double)x))); }
__device__ __forceinline__ float act_gamma(float o) { return (float)(2.0 * log(255.0 * (double)o)); }

// View-independent part of one Gaussian: the activations, the unit
// quaternion (binary32) and Sigma3D = M M^T with
// M = R(q) diag(s) in binary64 (6 unique entries: S00 S01 S02 S11 S12 S22).
struct GaussPre {
    float o, gam;
    double S[6];
    bool ok;   // false for a zero or non-finite quaternion: culled in every view
};

__device__ __forceinline__ void gauss_pre(int64_t i, int64_t n, const float* __restrict__ log_scales,
                                          const float* __restrict__ quats, const float* __restrict__ logits,
                                          GaussPre& g)
{
    float sx = act_scale(log_scales[i]);
    float sy = act_scale(log_scales[n + i]);
    float sz = act_scale(log_scales[2 * n + i]);
    g.o = act_opacity(logits[i]);
    g.gam = act_gamma(g.o);
    float qw = quats[i], qx = quats[n + i], qy = quats[2 * n + i], qz = quats[3 * n + i];
    float n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
    g.ok = n2 > 0.0f && isfinite(n2);
    if (!g.ok) return;
    float nr = sqrtf(n2);
    float w = qw / nr, x = qx / nr, y = qy / nr, z = qz / nr;
    // Sigma3D, the EWA projection and the conic in binary64, each result
    // rounded once to binary32: for needle-like Gaussians Sigma2D is nearly
    // singular (condition up to ~1e6), and binary32 entries would lose up to
    // a percent of the conic to cancellation in A C - B^2.
    double dw = w, dxq = x, dyq = y, dzq = z;
    double Rq[9];
    Rq[0] = 1.0 - 2.0 * (dyq * dyq + dzq * dzq);
    Rq[1] = 2.0 * (dxq * dyq - dw * dzq);
    Rq[2] = 2.0 * (dxq * dzq + dw * dyq);
    Rq[3] = 2.0 * (dxq * dyq + dw * dzq);
    Rq[4] = 1.0 - 2.0 * (dxq * dxq + dzq * dzq);
    Rq[5] = 2.0 * (dyq * dzq - dw * dxq);
    Rq[6] = 2.0 * (dxq * dzq - dw * dyq);
    Rq[7] = 2.0 * (dyq * dzq + dw * dxq);
    Rq[8] = 1.0 - 2.0 * (dxq * dxq + dyq * dyq);
    double M[9];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        M[r * 3 + 0] = Rq[r * 3 + 0] * (double)sx;
        M[r * 3 + 1] = Rq[r * 3 + 1] * (double)sy;
        M[r * 3 + 2] = Rq[r * 3 + 2] * (double)sz;
    }
    int k = 0;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = r; c < 3; ++c)
            g.S[k++] = (M[r * 3 + 0] * M[c * 3 + 0] + M[r * 3 + 1] * M[c * 3 + 1]) + M[r * 3 + 2] * M[c * 3 + 2];
}

// Sigma3D entry (r, c) from the 6 stored (symmetric: the products of (r, c)
// and (c, r) are the same, summed in the same order).
__device__ __forceinline__ double s3(const GaussPre& g, int r, int c)
{
    int lo = r < c ? r : c, hi = r < c ? c : r;
    return g.S[lo == 0 ? hi : (lo == 1 ? 2 + hi : 5)];
}

// Projects Gaussian i (mean mx, my, mz; view-independent part g) for one
// camera and writes its splat, rects and count.  The SH coefficients come
// from `pre` when given (loaded once for several views), else they are
// loaded here, only for a Gaussian that survives the culls before its colour.
template <int DEG>
__device__ __forceinline__ void project_view(int64_t i, int64_t n, float mx, float my, float mz, const GaussPre& g,
                                             const float* __restrict__ sh, const ShCoef<DEG>* pre,
                                             const ProjCam& cam, int mode_arg, float4* __restrict__ out_splat,
                                             int4* __restrict__ out_rects, int32_t* __restrict__ out_count,
                                             uint32_t* __restrict__ out_key)
{
    const int mode = mode_arg & ~QB_CLIP_3SIGMA;
    const bool clip = (mode_arg & QB_CLIP_3SIGMA) != 0;
    const float* R = cam.R;
    float px = ((R[0] * mx + R[1] * my) + R[2] * mz) + cam.t[0];
    float py = ((R[3] * mx + R[4] * my) + R[5] * mz) + cam.t[1];
    float pz = ((R[6] * mx + R[7] * my) + R[8] * mz) + cam.t[2];

    float4 s0 = make_float4(0.f, 0.f, pz, 0.f), s1 = make_float4(0.f, 0.f, 0.f, 0.f),
           s2 = make_float4(0.f, 0.f, 0.f, 0.f);
    QRect rr[4] = {{1, 0, 1, 0}, {1, 0, 1, 0}, {1, 0, 1, 0}, {1, 0, 1, 0}};
    int count = 0;

    do {
        if (!(pz > cam.near_plane) || !isfinite(px) || !isfinite(py) || !isfinite(pz)) break;
        if (!g.ok) break;
        float o = g.o, gam = g.gam;

        // Jacobian at the view-space mean with its image-plane slope clamped
        // to 1.3x the half field of view (binary32 slope, binary64 Jacobian)
        float xs = px / pz, ys = py / pz;
        xs = xs < -cam.limx ? -cam.limx : (xs > cam.limx ? cam.limx : xs);
        ys = ys < -cam.limy ? -cam.limy : (ys > cam.limy ? cam.limy : ys);
        float tx = xs * pz, ty = ys * pz;
        double dpz = pz, zz = dpz * dpz;
        double J00 = (double)cam.fx / dpz, J02 = -((double)cam.fx * (double)tx) / zz;
        double J11 = (double)cam.fy / dpz, J12 = -((double)cam.fy * (double)ty) / zz;
        double T[6];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T[c] = J00 * (double)R[c] + J02 * (double)R[6 + c];
            T[3 + c] = J11 * (double)R[3 + c] + J12 * (double)R[6 + c];
        }
        double U[6];
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                U[r * 3 + c] = (T[r * 3 + 0] * s3(g, 0, c) + T[r * 3 + 1] * s3(g, 1, c)) + T[r * 3 + 2] * s3(g, 2, c);
        double A64 = ((U[0] * T[0] + U[1] * T[1]) + U[2] * T[2]) + 0.3;
        double B64 = (U[0] * T[3] + U[1] * T[4]) + U[2] * T[5];
        double C64 = ((U[3] * T[3] + U[4] * T[4]) + U[5] * T[5]) + 0.3;
        double det64 = A64 * C64 - B64 * B64;
        if (!(det64 > 0.0)) break;
        float A = (float)A64, B = (float)B64, C = (float)C64;
        float ca = (float)(C64 / det64), cb = (float)(-(B64 / det64)), cc = (float)(A64 / det64);
        float det = A * C - B * B;  // binary32, for the 3-sigma radius only

        float u = cam.fx * (px / pz) + cam.cx;
        float v = cam.fy * (py / pz) + cam.cy;
        if (!isfinite(A) || !isfinite(B) || !isfinite(C) || !isfinite(ca) || !isfinite(cb) || !isfinite(cc) ||
            !isfinite(u) || !isfinite(v))
            break;
        if (mode != QB_BOX_3SIGMA && !(gam > 0.0f)) break;

        float rgb[3];
        {
            float dx = mx - cam.campos[0], dy = my - cam.campos[1], dz = mz - cam.campos[2];
            float nn = sqrtf(dx * dx + dy * dy + dz * dz);
            if (nn > 0.0f) { dx /= nn; dy /= nn; dz /= nn; }
            if (pre) {
                sh_colour<DEG>(*pre, dx, dy, dz, rgb);
            } else {
                ShCoef<DEG> c;
                sh_load<DEG>(sh, n, i, c);
                sh_colour<DEG>(c, dx, dy, dz, rgb);
            }
        }

        // the 3-sigma square (Sec. 2): the 3SIGMA mode's box, and the rect the
        // sub-boxes are cut to under QB_CLIP_3SIGMA
        auto square = [&]() {
            float mid = 0.5f * (A + C);
            float disc = mid * mid - det;
            if (disc < 0.1f) disc = 0.1f;
            float lam = mid + sqrtf(disc);
            float r = ceilf(3.0f * sqrtf(lam));
            return box_rect(u - r, u + r, v - r, v + r, cam.W, cam.H);
        };
        if (mode == QB_BOX_3SIGMA) {
            rr[0] = square();
        } else {
            float xm = sqrtf(gam * A);
            float ym = sqrtf(gam * C);
            if (mode == QB_BOX_ADR) {
                rr[0] = box_rect(u - xm, u + xm, v - ym, v + ym, cam.W, cam.H);
            } else {
                // stretching factor f = sqrt(1 - b^2/(ac)) = sqrt(1 - B^2/(AC)), Eq. (12)
                float ratio = (B * B) / (A * C);
                float fs = 1.0f - ratio;
                if (fs < 0.0f) fs = 0.0f;
                float f = sqrtf(fs);
                float fw = f * xm, fh = f * ym;
                bool maj_same = B > 0.0f;  // major axis through (+,+) and (-,-)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    int qsx = (q & 1) ? 1 : -1;
                    int qsy = (q & 2) ? 1 : -1;
                    bool major = maj_same ? (qsx == qsy) : (qsx != qsy);
                    if (!major && mode == QB_BOX_DUALBOX) continue;
                    float bw = major ? xm : fw;
                    float bh = major ? ym : fh;
                    float x0 = qsx > 0 ? u : u - bw;
                    float x1 = qsx > 0 ? u + bw : u;
                    float y0 = qsy > 0 ? v : v - bh;
                    float y1 = qsy > 0 ? v + bh : v;
                    rr[q] = box_rect(x0, x1, y0, y1, cam.W, cam.H);
                }
            }
        }
        if (clip && mode != QB_BOX_3SIGMA) {
            // cut each sub-box's tile rect to the square's (an empty square
            // empties them all; a cut rect keeps the centre tile, so the union
            // stays one interval per scanline for QPass)
            QRect sq = square();
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                QRect& c = rr[q];
                if (c.x0 > c.x1 || c.y0 > c.y1) continue;
                c.x0 = max(c.x0, sq.x0);
                c.x1 = min(c.x1, sq.x1);
                c.y0 = max(c.y0, sq.y0);
                c.y1 = min(c.y1, sq.y1);
                if (c.x0 > c.x1 || c.y0 > c.y1) c = QRect{1, 0, 1, 0};
            }
        }
        if (mode == QB_BOX_QUADBOX_NAIVE) {
            count = naive_walk(rr, [](int, int, int) {});
        } else {
            QRuns runs;
            qpass_runs(rr, runs);
            count = runs.total;
        }
        s0 = make_float4(u, v, pz, o);
        s1 = make_float4(ca, cb, cc, gam);
        s2 = make_float4(rgb[0], rgb[1], rgb[2], 1.0f);
    } while (0);

    out_splat[3 * i + 0] = s0;
    out_splat[3 * i + 1] = s1;
    out_splat[3 * i + 2] = s2;
    int4 p0, p1;
    p0.x = (rr[0].x0 & 0xFFFF) | (rr[0].x1 << 16);
    p0.y = (rr[0].y0 & 0xFFFF) | (rr[0].y1 << 16);
    p0.z = (rr[1].x0 & 0xFFFF) | (rr[1].x1 << 16);
    p0.w = (rr[1].y0 & 0xFFFF) | (rr[1].y1 << 16);
    p1.x = (rr[2].x0 & 0xFFFF) | (rr[2].x1 << 16);
    p1.y = (rr[2].y0 & 0xFFFF) | (rr[2].y1 << 16);
    p1.z = (rr[3].x0 & 0xFFFF) | (rr[3].x1 << 16);
    p1.w = (rr[3].y0 & 0xFFFF) | (rr[3].y1 << 16);
    out_rects[2 * i + 0] = p0;
    out_rects[2 * i + 1] = p1;
    out_count[i] = count;
    // the depth sort's key: the depth's bits where the Gaussian has tiles,
    // else the largest key (those Gaussians emit nothing)
    if (out_key) out_key[i] = count > 0 ? __float_as_uint(s0.z) : 0xFFFFFFFFu;
}

template <int DEG>
__global__ __launch_bounds__(QB_BLOCK) void k_project(
    int64_t n, const float* __restrict__ means, const float* __restrict__ log_scales,
    const float* __restrict__ quats, const float* __restrict__ logits,
    const float* __restrict__ sh, ProjCam cam, int mode,
    float4* __restrict__ out_splat, int4* __restrict__ out_rects, int32_t* __restrict__ out_count,
    uint32_t* __restrict__ out_key)
{
    int64_t i = (int64_t)blockIdx.x * QB_BLOCK + threadIdx.x;
    if (i >= n) return;
    GaussPre g;
    gauss_pre(i, n, log_scales, quats, logits, g);
    project_view<DEG>(i, n, means[i], means[n + i], means[2 * n + i], g, sh, (const ShCoef<DEG>*)nullptr, cam, mode,
                      out_splat, out_rects, out_count, out_key);
}

// Cameras of a batched call, by value as a kernel argument (3.3 KB at
// QB_MAX_VIEWS).
struct ProjCamTable {
    ProjCam cam[QB_MAX_VIEWS];
};

// One lane per Gaussian: the view-independent part (activations, Sigma3D
// and the SH coefficients) once, then every view (view v writes the block of
// records starting at v*n).  Per view the same arithmetic as k_project, so
// the records are identical.
template <int DEG>
__global__ __launch_bounds__(QB_BLOCK) void k_project_views(
    int64_t n, int nv, const float* __restrict__ means, const float* __restrict__ log_scales,
    const float* __restrict__ quats, const float* __restrict__ logits,
    const float* __restrict__ sh, ProjCamTable cams, int mode,
    float4* __restrict__ out_splat, int4* __restrict__ out_rects, int32_t* __restrict__ out_count,
    uint32_t* __restrict__ out_key)
{
    int64_t i = (int64_t)blockIdx.x * QB_BLOCK + threadIdx.x;
    if (i >= n) return;
    GaussPre g;
    gauss_pre(i, n, log_scales, quats, logits, g);
    ShCoef<DEG> c;
    sh_load<DEG>(sh, n, i, c);
    float mx = means[i], my = means[n + i], mz = means[2 * n + i];
    for (int v = 0; v < nv; ++v)
        project_view<DEG>(i, n, mx, my, mz, g, sh, &c, cams.cam[v], mode, out_splat + 3 * (int64_t)v * n,
                          out_rects + 2 * (int64_t)v * n, out_count + (int64_t)v * n,
                          out_key ? out_key + (int64_t)v * n : nullptr);
}

// Launches kernel template K for the SH degree (0..3).
#define QB_LAUNCH_DEG(K, deg, grid, ...)                                                  \
    do {                                                                                  \
        switch (deg) {                                                                    \
        case 0: QB_LAUNCH(K<0>, grid, QB_BLOCK, 0, __VA_ARGS__); break;                   \
        case 1: QB_LAUNCH(K<1>, grid, QB_BLOCK, 0, __VA_ARGS__); break;                   \
        case 2: QB_LAUNCH(K<2>, grid, QB_BLOCK, 0, __VA_ARGS__); break;                   \
        default: QB_LAUNCH(K<3>, grid, QB_BLOCK, 0, __VA_ARGS__); break;                  \
        }                                                                                 \
    } while (0)

}  // namespace

namespace {

void make_proj_cam(const qb_camera& cam, ProjCam* pc)
{
    pc->W = cam.width;
    pc->H = cam.height;
    pc->tiles_x = (int)qb_div_up(cam.width, QB_TILE);
    pc->tiles_y = (int)qb_div_up(cam.height, QB_TILE);
    pc->fx = cam.fx; pc->fy = cam.fy; pc->cx = cam.cx; pc->cy = cam.cy;
    pc->near_plane = cam.near_plane;
    for (int k = 0; k < 9; ++k) pc->R[k] = cam.R[k];
    for (int k = 0; k < 3; ++k) { pc->t[k] = cam.t[k]; pc->campos[k] = cam.campos[k]; }
    // 1.3 x tan(half fov), in the same binary32 order as the oracle
    volatile float hx = 0.5f * (float)cam.width;
    volatile float hy = 0.5f * (float)cam.height;
    pc->limx = 1.3f * (hx / cam.fx);
    pc->limy = 1.3f * (hy / cam.fy);
}

}  // namespace

// One activation of qb_project on each input (which: qb_activation).
__global__ __launch_bounds__(QB_BLOCK) void k_activations(int64_t n, const float* x, int which,
                                                          float* out)
{
    for (int64_t i = (int64_t)blockIdx.x * QB_BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * QB_BLOCK) {
        float v = x[i];
        out[i] = which == QB_ACT_SCALE ? act_scale(v) : which == QB_ACT_OPACITY ? act_opacity(v) : act_gamma(v);
    }
}

extern "C" qb_status qb_activations(int64_t n, const float* x, int32_t which, float* out, qb_stream_t stream)
{
    if (n < 0 || which < QB_ACT_SCALE || which > QB_ACT_GAMMA) return QB_ERR_INVALID_ARG;
    if (n == 0) return QB_OK;
    if (!x || !out) return QB_ERR_INVALID_ARG;
    int64_t grid = qb_div_up(n, QB_BLOCK);
    if (grid > 16384) grid = 16384;
    QB_LAUNCH(k_activations, grid, QB_BLOCK, 0, qb_hip_stream(stream), n, x, (int)which, out);
    return QB_OK;
}

extern "C" qb_status qb_project_ex(int64_t n, const float* means, const float* log_scales,
                                   const float* quats, const float* opacity_logits, const float* sh,
                                   int32_t sh_degree, const qb_camera* cam, int32_t mode,
                                   qb_splat* out_splats, qb_rects* out_rects, int32_t* out_counts,
                                   uint32_t* out_depth_keys, qb_stream_t stream)
{
    if (n < 0 || n >= (int64_t)1 << 31 || !cam || sh_degree < 0 || sh_degree > 3) return QB_ERR_INVALID_ARG;
    if (!qb_valid_mode(mode)) return QB_ERR_INVALID_ARG;
    if (!qb_valid_camera(*cam)) return QB_ERR_INVALID_ARG;
    if (n == 0) return QB_OK;
    if (!means || !log_scales || !quats || !opacity_logits || !sh || !out_splats || !out_rects ||
        !out_counts)
        return QB_ERR_INVALID_ARG;
    ProjCam pc;
    make_proj_cam(*cam, &pc);
    int64_t grid = qb_div_up(n, QB_BLOCK);
    QB_LAUNCH_DEG(k_project, sh_degree, grid, qb_hip_stream(stream), n, means, log_scales, quats, opacity_logits, sh,
                  pc, (int)mode, reinterpret_cast<float4*>(out_splats), reinterpret_cast<int4*>(out_rects),
                  out_counts, out_depth_keys);
    return QB_OK;
}

extern "C" qb_status qb_project(int64_t n, const float* means, const float* log_scales,
                                const float* quats, const float* opacity_logits, const float* sh,
                                int32_t sh_degree, const qb_camera* cam, int32_t mode,
                                qb_splat* out_splats, qb_rects* out_rects, int32_t* out_counts,
                                qb_stream_t stream)
{
    return qb_project_ex(n, means, log_scales, quats, opacity_logits, sh, sh_degree, cam, mode, out_splats,
                         out_rects, out_counts, nullptr, stream);
}

extern "C" qb_status qb_project_views_ex(int64_t n, const float* means, const float* log_scales,
                                         const float* quats, const float* opacity_logits, const float* sh,
                                         int32_t sh_degree, const qb_camera* cams, int32_t num_views, int32_t mode,
                                         qb_splat* out_splats, qb_rects* out_rects, int32_t* out_counts,
                                         uint32_t* out_depth_keys, qb_stream_t stream)
{
    if (n < 0 || n >= (int64_t)1 << 31 || !cams || sh_degree < 0 || sh_degree > 3 || num_views < 1 ||
        num_views > QB_MAX_VIEWS)
        return QB_ERR_INVALID_ARG;
    if (!qb_valid_mode(mode)) return QB_ERR_INVALID_ARG;
    ProjCamTable ct;
    for (int v = 0; v < num_views; ++v) {
        if (!qb_valid_camera(cams[v])) return QB_ERR_INVALID_ARG;
        make_proj_cam(cams[v], &ct.cam[v]);
    }
    if (n == 0) return QB_OK;
    if (!means || !log_scales || !quats || !opacity_logits || !sh || !out_splats || !out_rects ||
        !out_counts)
        return QB_ERR_INVALID_ARG;
    QB_LAUNCH_DEG(k_project_views, sh_degree, qb_div_up(n, QB_BLOCK), qb_hip_stream(stream), n, (int)num_views,
                  means, log_scales, quats, opacity_logits, sh, ct, (int)mode,
                  reinterpret_cast<float4*>(out_splats), reinterpret_cast<int4*>(out_rects), out_counts,
                  out_depth_keys);
    return QB_OK;
}

extern "C" qb_status qb_project_views(int64_t n, const float* means, const float* log_scales,
                                      const float* quats, const float* opacity_logits, const float* sh,
                                      int32_t sh_degree, const qb_camera* cams, int32_t num_views, int32_t mode,
                                      qb_splat* out_splats, qb_rects* out_rects, int32_t* out_counts,
                                      qb_stream_t stream)
{
    return qb_project_views_ex(n, means, log_scales, quats, opacity_logits, sh, sh_degree, cams, num_views, mode,
                               out_splats, out_rects, out_counts, nullptr, stream);
}
