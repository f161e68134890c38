// Gradients of the forward rasterizer (the paper trains through it, Sec. 4.1).
//
// qb_render_backward: per 16x16 tile, one workgroup (1, 2 or 4 pixels per
//   lane) walks the tile's list back to front, starting at each pixel's last
//   contributor.  Each step re-evaluates the forward's binary32 power, 1/255
//   cutoff and alpha exactly, recovers the transmittance in front of the
//   Gaussian by dividing out (1 - alpha), and forms the pixel's share of
//   dL/d(u, v, conic, opacity, rgb) of Eq. (2).  The shares are summed over a
//   lane's pixels, then across each wave64 (DPP row sums and two permlane
//   swap folds, skipped when no lane of the wave takes part), and nine lanes
//   per wave add them to the Gaussian's 2D
//   gradient with global float atomics; the order of those additions is not
//   fixed, so the result is deterministic only up to float reassociation.
//
// qb_project_backward: one lane per Gaussian; recomputes the projection's
//   intermediates and applies the chain rule through the conic inverse, the
//   EWA covariance J W Sigma W^T J^T (with the clamped Jacobian), the mean
//   projection, Sigma = R S S^T R^T, the quaternion normalisation, the scale
//   and opacity activations (k_geometry_backward, binary64 like the
//   forward's covariance chain), then the SH colour and its view direction
//   (k_sh_backward, a lighter kernel at higher occupancy).
#include "qb_common.h"

namespace {

// v + the value of v in another lane of the same row of 16 (DPP): step 0
// pairs neighbours, 1 pairs of neighbours, 2 the half-row mirror, 3 the row
// mirror; after the four steps every lane of a row holds the row's sum.
// Every lane of the wave must be active.
__device__ __forceinline__ float dpp_add(float v, int step)
{
    int x = __float_as_int(v);
    int y;
    switch (step) {
    case 0: y = __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false); break;   // quad_perm [1,0,3,2]
    case 1: y = __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false); break;   // quad_perm [2,3,0,1]
    case 2: y = __builtin_amdgcn_update_dpp(0, x, 0x141, 0xF, 0xF, false); break;  // row_half_mirror
    default: y = __builtin_amdgcn_update_dpp(0, x, 0x140, 0xF, 0xF, false); break; // row_mirror
    }
    return v + __int_as_float(y);
}

// x + x of lane ^ 32, and x + x of lane ^ 16: the gfx950 permlane swaps
// exchange the two halves of the wave (32) or the rows of each half (16)
// between two registers; with x in both, the two results at a lane are x
// there and x at the partner lane, whichever way round.
__device__ __forceinline__ float fold_lanes32(float x)
{
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float fold_lanes16(float x)
{
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Adds the wave totals of v[0..8] to g[0..8].  The nine row reductions run
// interleaved, step by step (independent DPP chains, no wait states); lane
// 16 r + j of row r then keeps row r's sum of value j, and two swap folds add
// the four rows' sums of that one value, so lanes 0..8 hold the nine totals
// and issue one atomic instruction over 36 contiguous bytes.  Every lane of
// the wave must be active.
__device__ __forceinline__ void wave_add9(float v[9], float* g, int lane)
{
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int j = 0; j < 9; ++j) v[j] = dpp_add(v[j], s);
    int j = lane & 15;
    float mine = v[0];
#pragma unroll
    for (int t = 1; t < 9; ++t) mine = j == t ? v[t] : mine;
    mine = fold_lanes16(fold_lanes32(mine));
    if (lane < 9) atomicAdd(g + lane, mine);
}

// Backward of one tile of one image: 256 / PPL lanes, each owning PPL pixels
// of one tile row, 16 / PPL apart.  The list is walked back to front from the
// furthest last contributor of the tile, in batches of one record per lane
// staged in LDS.  Per entry, a lane sums its pixels' shares, the wave sums
// its lanes (wave_add9), and lanes 0..8 add the nine totals to grad2d in one
// atomic instruction (float atomics: order-dependent rounding).
template <int PPL>
__device__ __forceinline__ void render_backward_tile(
    int tile, int W, int H, int tiles_x, const uint2* __restrict__ ranges, const uint32_t* __restrict__ ids,
    const float4* __restrict__ splats, float bg0, float bg1, float bg2, const float* __restrict__ final_T,
    const uint32_t* __restrict__ n_contrib, const float* __restrict__ dL_dimg, float* __restrict__ grad2d)
{
    constexpr int NT = 256 / PPL;
    constexpr int LX = QB_TILE / PPL;
    __shared__ float4 s_geo[NT];   // u, v, -a/2, -b
    __shared__ float4 s_opa[NT];   // -c/2, log2(o), -gamma/2, a
    __shared__ float4 s_col[NT];   // r, g, b, b
    __shared__ float2 s_c[NT];     // c, 1/o
    __shared__ uint32_t s_id[NT];
    __shared__ int s_rows[NT];     // tile rows that can pass the cutoff (entry_rows)
    __shared__ uint32_t s_maxlast;

    constexpr int kRowsPerWave = 64 / LX;   // tile rows a wave covers
    int tx = tile % tiles_x, ty = tile / tiles_x;
    int lx = threadIdx.x % LX, ly = threadIdx.x / LX;
    int py = ty * QB_TILE + ly;
    int wrow0 = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64) * kRowsPerWave);
    float fy = (float)py;
    constexpr float kLog2e = 1.44269504088896341f;
    int lane = threadIdx.x & 63;
    int64_t plane = (int64_t)W * H;

    // per pixel: T in front of the current entry, dL/dC, and
    // R = sum_c dL/dC_c * (colour of everything behind the current entry,
    // background included), so that dL/dalpha = T_i (dC . rgb) - R / (1 - alpha)
    float fxp[PPL], T[PPL], dC[PPL][3], R[PPL];
    uint32_t last[PPL];
    uint32_t lmax = 0;
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
        int px = tx * QB_TILE + lx + q * LX;
        bool inside = px < W && py < H;
        int64_t pix = (int64_t)py * W + px;
        fxp[q] = (float)px;
        last[q] = inside ? n_contrib[pix] : 0u;
        T[q] = inside ? final_T[pix] : 1.0f;
        dC[q][0] = inside ? dL_dimg[pix] : 0.f;
        dC[q][1] = inside ? dL_dimg[plane + pix] : 0.f;
        dC[q][2] = inside ? dL_dimg[2 * plane + pix] : 0.f;
        R[q] = T[q] * ((dC[q][0] * bg0 + dC[q][1] * bg1) + dC[q][2] * bg2);
        lmax = max(lmax, last[q]);
    }

    uint2 rg = ranges[tile];
    int64_t start = rg.x;
    if (threadIdx.x == 0) s_maxlast = 0;
    __syncthreads();
    if (lmax) atomicMax(&s_maxlast, lmax);
    __syncthreads();
    int64_t hi = (int64_t)s_maxlast;  // entries [0, hi) of the tile list matter

    for (int64_t b1 = hi; b1 > 0; b1 -= NT) {
        int64_t b0 = b1 - NT > 0 ? b1 - NT : 0;
        int64_t j = b0 + threadIdx.x;
        __syncthreads();
        if (j < b1) {
            uint32_t id = ids[start + j];
            float4 a = splats[3 * (int64_t)id + 0];
            float4 b = splats[3 * (int64_t)id + 1];
            float4 c = splats[3 * (int64_t)id + 2];
            s_geo[threadIdx.x] = make_float4(a.x, a.y, -0.5f * b.x, -b.y);
            s_opa[threadIdx.x] = make_float4(-0.5f * b.z, __log2f(a.w), -0.5f * b.w, b.x);
            s_col[threadIdx.x] = make_float4(c.x, c.y, c.z, b.y);
            s_c[threadIdx.x] = make_float2(b.z, __builtin_amdgcn_rcpf(a.w));
            s_id[threadIdx.x] = id;
            if (kRowsPerWave < QB_TILE) s_rows[threadIdx.x] = entry_rows(a.y, b.x, b.y, b.z, b.w, ty);
        }
        __syncthreads();
        // entries of this batch whose ellipse can reach this wave's rows, one
        // bit each (uniform masks), walked from the back
        constexpr int NM = NT / 64;
        int cnt = (int)(b1 - b0);
        uint64_t mask[NM];
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            int kk = m * 64 + lane;
            bool rel = kk < cnt;
            if (kRowsPerWave < QB_TILE && rel) {
                int rr = s_rows[kk];
                int r0 = (int)(int16_t)(rr & 0xFFFF), r1 = rr >> 16;
                rel = !(r1 < wrow0 || r0 > wrow0 + kRowsPerWave - 1);
            }
            mask[m] = __ballot(rel);
        }
#pragma unroll
        for (int m = NM - 1; m >= 0; --m) {
          uint64_t bits = mask[m];
          while (bits) {
            int hb = 63 - (int)__builtin_clzll(bits);
            bits &= ~(1ull << hb);
            int k = m * 64 + hb;
            uint32_t idx = (uint32_t)(b0 + k);  // list index of this entry
            float4 g = s_geo[k];
            float4 o = s_opa[k];
            float dy = g.y - fy;
            float nbdy = g.w * dy;
            float hcdy2 = (o.x * dy) * dy;
            float dx[PPL], power[PPL];
            bool act[PPL];
            bool any = false;
#pragma unroll
            for (int q = 0; q < PPL; ++q) {
                dx[q] = g.x - fxp[q];
                power[q] = fmaf(fmaf(g.z, dx[q], nbdy), dx[q], hcdy2);
                act[q] = idx < last[q] && !(power[q] > 0.0f || power[q] < o.z);
                any = any || act[q];
            }
            if (!__any(any)) continue;
            float4 col = s_col[k];
            float2 ci = s_c[k];
            float cc = ci.x;
            // per pixel: A = dL/dC . rgb of this entry; the geometric shares
            // are summed over the lane's pixels as P = sum dpow,
            // S1 = sum dpow dx and Q = sum dpow dx^2 (the pixels share the
            // row offset dy), and turned into (u, v, a, b, c) once per lane
            float P = 0.f, S1 = 0.f, Q = 0.f, go = 0.f, gr = 0.f, gg = 0.f, gbl = 0.f;
#pragma unroll
            for (int q = 0; q < PPL; ++q) {
                if (act[q]) {
                    // o e^power as the forward evaluates it: one exp2 of
                    // power log2(e) + log2(o), so alpha matches the forward's
                    float raw = __builtin_amdgcn_exp2f(fmaf(power[q], kLog2e, o.y));
                    float alpha = fminf(0.99f, raw);
                    // 1 / (1 - alpha) by the hardware reciprocal (1 ulp; 1 - alpha >= 0.01):
                    // the transmittance in front of this Gaussian is T / (1 - alpha)
                    float inv = __builtin_amdgcn_rcpf(1.0f - alpha);
                    float Ti = T[q] * inv;
                    float w = alpha * Ti;
                    gr = fmaf(w, dC[q][0], gr);
                    gg = fmaf(w, dC[q][1], gg);
                    gbl = fmaf(w, dC[q][2], gbl);
                    float A = fmaf(dC[q][2], col.z, fmaf(dC[q][1], col.y, dC[q][0] * col.x));
                    float dalpha = Ti * A - R[q] * inv;
                    R[q] = fmaf(w, A, R[q]);
                    T[q] = Ti;
                    if (raw <= 0.99f) {
                        float dpow = dalpha * alpha;
                        go = fmaf(dalpha, raw, go);   // times 1/o below: dalpha/do = e^power
                        float t = dpow * dx[q];
                        P += dpow;
                        S1 += t;
                        Q = fmaf(t, dx[q], Q);
                    }
                }
            }
            // power = -(a dx^2 + 2 b dx dy + c dy^2) / 2 with dx = u - x, dy = v - y
            float a = o.w, b = col.w, dyP = dy * P;
            float gu = -fmaf(a, S1, b * dyP), gv = -fmaf(b, S1, cc * dyP);
            float ga = -0.5f * Q, gb = -(dy * S1), gc = -0.5f * (dy * dyP);
            // an entry some lane composites has gamma >= 0, so o >= 1/255
            float v9[9] = {gu, gv, ga, gb, gc, go * ci.y, gr, gg, gbl};
            wave_add9(v9, grad2d + 9 * (int64_t)s_id[k], lane);
          }
        }
    }
}

template <int PPL>
__global__ __launch_bounds__(256 / PPL) void k_render_backward(
    int W, int H, int tiles_x, const uint2* __restrict__ ranges, const uint32_t* __restrict__ ids,
    const float4* __restrict__ splats, float bg0, float bg1, float bg2, const float* __restrict__ final_T,
    const uint32_t* __restrict__ n_contrib, const float* __restrict__ dL_dimg, float* __restrict__ grad2d,
    const uint32_t* __restrict__ order)
{
    // workgroup i takes tile order[i] (qb_tile_order) or tile i
    uint32_t tile = order ? order[blockIdx.x] : blockIdx.x;
    if (tile >= gridDim.x) return;
    render_backward_tile<PPL>((int)tile, W, H, tiles_x, ranges, ids, splats, bg0, bg1, bg2, final_T, n_contrib,
                              dL_dimg, grad2d);
}

// Every tile of every view in one launch (global tile order[i] or i).
template <int PPL>
__global__ __launch_bounds__(256 / PPL) void k_render_backward_views(QbViewTable vt,
                                                                     const uint32_t* __restrict__ order, float bg0,
                                                                     float bg1, float bg2)
{
    uint32_t g = order ? order[blockIdx.x] : blockIdx.x;
    if (g >= gridDim.x) return;
    int b = (int)g;
    int v = qb_view_of(vt, b);
    const qb_view& w = vt.view[v];
    render_backward_tile<PPL>(b - vt.tile_start[v], w.width, w.height, vt.tiles_x[v],
                              reinterpret_cast<const uint2*>(w.ranges), w.ids,
                              reinterpret_cast<const float4*>(w.splats), bg0, bg1, bg2, w.final_T, w.n_contrib,
                              w.dL_dimage, w.grad2d);
}

// Clears grad2d of every view: blockIdx.y is the view.
__global__ void k_zero_views(QbViewTable vt, int64_t count)
{
    float* p = vt.view[blockIdx.y].grad2d;
    for (int64_t i = (int64_t)blockIdx.x * QB_BLOCK + threadIdx.x; i < count; i += (int64_t)gridDim.x * QB_BLOCK)
        p[i] = 0.0f;
}

struct BwdCam {
    int W, H;
    float fx, fy, cx, cy, near_plane;
    float R[9], t[3], campos[3];
    float limx, limy;
};

// Cameras of a batched call, by value as a kernel argument (3 KB at
// QB_MAX_VIEWS).
struct BwdCamTable {
    BwdCam cam[QB_MAX_VIEWS];
};

// Real SH basis Y_k of degree <= 3 at the unit direction (x, y, z) and its
// gradient, dY_k = G[k][0] dx + G[k][1] dy + G[k][2] dz.
__device__ __forceinline__ void sh_basis_and_grad(float x, float y, float z, float Y[16], float G[16][3])
{
    const float k00 = 0.28209479177387814f, k1 = 0.48860251190291992f;
    const float k2a = 1.0925484305920792f, k2b = 0.31539156525252005f, k2c = 0.54627421529603959f;
    const float k3a = 0.59004358992664352f, k3b = 2.8906114426405538f, k3c = 0.45704579946446572f;
    const float k3d = 0.3731763325901154f, k3e = 1.4453057213202769f;
    float xx = x * x, yy = y * y, zz = z * z;
    Y[0] = k00; G[0][0] = 0.f; G[0][1] = 0.f; G[0][2] = 0.f;
    Y[1] = -k1 * y; G[1][0] = 0.f; G[1][1] = -k1; G[1][2] = 0.f;
    Y[2] = k1 * z; G[2][0] = 0.f; G[2][1] = 0.f; G[2][2] = k1;
    Y[3] = -k1 * x; G[3][0] = -k1; G[3][1] = 0.f; G[3][2] = 0.f;
    Y[4] = k2a * x * y; G[4][0] = k2a * y; G[4][1] = k2a * x; G[4][2] = 0.f;
    Y[5] = -k2a * y * z; G[5][0] = 0.f; G[5][1] = -k2a * z; G[5][2] = -k2a * y;
    Y[6] = k2b * (2.f * zz - xx - yy); G[6][0] = -2.f * k2b * x; G[6][1] = -2.f * k2b * y; G[6][2] = 4.f * k2b * z;
    Y[7] = -k2a * x * z; G[7][0] = -k2a * z; G[7][1] = 0.f; G[7][2] = -k2a * x;
    Y[8] = k2c * (xx - yy); G[8][0] = 2.f * k2c * x; G[8][1] = -2.f * k2c * y; G[8][2] = 0.f;
    Y[9] = -k3a * y * (3.f * xx - yy); G[9][0] = -6.f * k3a * x * y; G[9][1] = -k3a * (3.f * xx - 3.f * yy); G[9][2] = 0.f;
    Y[10] = k3b * x * y * z; G[10][0] = k3b * y * z; G[10][1] = k3b * x * z; G[10][2] = k3b * x * y;
    Y[11] = -k3c * y * (4.f * zz - xx - yy); G[11][0] = 2.f * k3c * x * y; G[11][1] = -k3c * (4.f * zz - xx - 3.f * yy);
    G[11][2] = -8.f * k3c * y * z;
    Y[12] = k3d * z * (2.f * zz - 3.f * xx - 3.f * yy); G[12][0] = -6.f * k3d * x * z; G[12][1] = -6.f * k3d * y * z;
    G[12][2] = k3d * (6.f * zz - 3.f * xx - 3.f * yy);
    Y[13] = -k3c * x * (4.f * zz - xx - yy); G[13][0] = -k3c * (4.f * zz - 3.f * xx - yy); G[13][1] = 2.f * k3c * x * y;
    G[13][2] = -8.f * k3c * x * z;
    Y[14] = k3e * z * (xx - yy); G[14][0] = 2.f * k3e * x * z; G[14][1] = -2.f * k3e * y * z; G[14][2] = k3e * (xx - yy);
    Y[15] = -k3a * x * (xx - 3.f * yy); G[15][0] = -k3a * (3.f * xx - 3.f * yy); G[15][1] = 6.f * k3a * x * y; G[15][2] = 0.f;
}

// Single view: writes d_sh of Gaussian i and returns dL/d(direction).
__device__ __forceinline__ void sh_colour_backward(const float* __restrict__ sh, int64_t n, int64_t i, int deg,
                                                   float x, float y, float z, const float drgb[3],
                                                   float* __restrict__ d_sh, float ddir[3])
{
    float Y[16], G[16][3];
    sh_basis_and_grad(x, y, z, Y, G);
    int K = (deg + 1) * (deg + 1);
    ddir[0] = ddir[1] = ddir[2] = 0.f;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (k < K) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                int64_t off = (int64_t)(k * 3 + ch) * n + i;
                d_sh[off] = Y[k] * drgb[ch];
                float cw = sh[off] * drgb[ch];
                ddir[0] = fmaf(G[k][0], cw, ddir[0]);
                ddir[1] = fmaf(G[k][1], cw, ddir[1]);
                ddir[2] = fmaf(G[k][2], cw, ddir[2]);
            }
        }
    }
}

// Chain rule of one Gaussian from its grad2d rows to the mean (through the
// projection), log-scales, quaternion and opacity logit, in three parts:
// geometry_prep forms what every view shares (M = R(q) diag(s)), geometry_view
// takes one camera's row and ADDS its shares to dm, to dM = dL/dM and to
// dL/do, and geometry_finish turns the summed dM and dL/do into the scale,
// quaternion and logit gradients (linear in them, so one pass serves every
// view).  The forward forms Sigma3D, Sigma2D and the conic in binary64 from
// its binary32 inputs; their derivatives are taken the same way.  The
// colour's share of the mean gradient is left to the SH part.
struct GeoPrep {
    float mx, my, mz;
    double M[9];
};

// The rotation of the normalised quaternion of Gaussian i (binary64 from the
// binary32 norm, as the forward), its unit quaternion (w, x, y, z) and norm.
__device__ __forceinline__ void geometry_rotation(int64_t i, int64_t n, const float* __restrict__ quats,
                                                  double Rq[9], double qn[4], double& nr)
{
    float q4[4] = {quats[i], quats[n + i], quats[2 * n + i], quats[3 * n + i]};
    float n2 = ((q4[0] * q4[0] + q4[1] * q4[1]) + q4[2] * q4[2]) + q4[3] * q4[3];
    float nrf = sqrtf(n2);
    nr = nrf;
    double w = q4[0] / nrf, x = q4[1] / nrf, y = q4[2] / nrf, z = q4[3] / nrf;
    qn[0] = w; qn[1] = x; qn[2] = y; qn[3] = z;
    Rq[0] = 1.0 - 2.0 * (y * y + z * z); Rq[1] = 2.0 * (x * y - w * z); Rq[2] = 2.0 * (x * z + w * y);
    Rq[3] = 2.0 * (x * y + w * z); Rq[4] = 1.0 - 2.0 * (x * x + z * z); Rq[5] = 2.0 * (y * z - w * x);
    Rq[6] = 2.0 * (x * z - w * y); Rq[7] = 2.0 * (y * z + w * x); Rq[8] = 1.0 - 2.0 * (x * x + y * y);
}

__device__ __forceinline__ void geometry_scales(int64_t i, int64_t n, const float* __restrict__ log_scales,
                                                double s[3])
{
    for (int k = 0; k < 3; ++k) s[k] = (double)(float)exp((double)log_scales[k * n + i]);
}

__device__ __forceinline__ void geometry_prep(int64_t i, int64_t n, const float* __restrict__ means,
                                              const float* __restrict__ log_scales,
                                              const float* __restrict__ quats, GeoPrep& g)
{
    g.mx = means[i];
    g.my = means[n + i];
    g.mz = means[2 * n + i];
    double s[3], Rq[9], qn[4], nr;
    geometry_scales(i, n, log_scales, s);
    geometry_rotation(i, n, quats, Rq, qn, nr);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) g.M[r * 3 + c] = Rq[r * 3 + c] * s[c];
}

__device__ __forceinline__ bool geometry_view(const GeoPrep& g, const BwdCam& cam, const float* __restrict__ g2,
                                              double dm[3], double dMs[9], float& dop_sum)
{
    float r0 = g2[0], r1 = g2[1], r2 = g2[2], r3 = g2[3], r4 = g2[4], r5 = g2[5];
    // a zero row adds nothing (culled Gaussians and views a Gaussian does
    // not reach in any pixel have one), so the splat's visibility is not
    // read; returns whether the row added anything
    if (r0 == 0.f && r1 == 0.f && r2 == 0.f && r3 == 0.f && r4 == 0.f && r5 == 0.f) return false;
    double du = r0, dv = r1, da = r2, db = r3, dc = r4;
    dop_sum += r5;
    const double* M = g.M;
    const float* R = cam.R;
    float px = ((R[0] * g.mx + R[1] * g.my) + R[2] * g.mz) + cam.t[0];
    float py = ((R[3] * g.mx + R[4] * g.my) + R[5] * g.mz) + cam.t[1];
    float pz = ((R[6] * g.mx + R[7] * g.my) + R[8] * g.mz) + cam.t[2];
    float xs = px / pz, ys = py / pz;
    float clx = xs < -cam.limx ? -1.f : (xs > cam.limx ? 1.f : 0.f);
    float cly = ys < -cam.limy ? -1.f : (ys > cam.limy ? 1.f : 0.f);
    if (clx != 0.f) xs = clx * cam.limx;
    if (cly != 0.f) ys = cly * cam.limy;
    float txf = xs * pz, tyf = ys * pz;
    double fx = cam.fx, fy = cam.fy, tx = txf, ty = tyf, z1 = pz, z2 = z1 * z1, z3 = z2 * z1;
    double J00 = fx / z1, J02 = -(fx * tx) / z2;
    double J11 = fy / z1, J12 = -(fy * ty) / z2;
    double T[6];
    for (int c = 0; c < 3; ++c) {
        T[c] = J00 * (double)R[c] + J02 * (double)R[6 + c];
        T[3 + c] = J11 * (double)R[3 + c] + J12 * (double)R[6 + c];
    }
    // Sigma2D = V V^T + 0.3 I with V = T M (2x3): the backward never needs
    // Sigma3D itself (binary64 throughout; the rounding differs from the
    // forward's T Sigma3D T^T only at the 1e-16 level)
    double V[6];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c)
            V[r * 3 + c] = (T[r * 3 + 0] * M[c] + T[r * 3 + 1] * M[3 + c]) + T[r * 3 + 2] * M[6 + c];
    double A = ((V[0] * V[0] + V[1] * V[1]) + V[2] * V[2]) + 0.3;
    double B = (V[0] * V[3] + V[1] * V[4]) + V[2] * V[5];
    double C = ((V[3] * V[3] + V[4] * V[4]) + V[5] * V[5]) + 0.3;
    double det = A * C - B * B;
    double id2 = 1.0 / (det * det);
    // conic (a, b, c) = (C, -B, A) / det
    double dA = (da * (-C * C) + db * (B * C) + dc * (-B * B)) * id2;
    double dB = da * (2.0 * B * C) * id2 + db * (-1.0 / det - 2.0 * B * B * id2) + dc * (2.0 * A * B) * id2;
    double dCc = (da * (-B * B) + db * (B * A) + dc * (-A * A)) * id2;
    // Sigma2D = T Sigma T^T with symmetric cotangent G
    double G00 = dA, G01 = 0.5 * dB, G11 = dCc;
    double GV[6];  // G V (2x3)
    for (int c = 0; c < 3; ++c) {
        GV[c] = G00 * V[c] + G01 * V[3 + c];
        GV[3 + c] = G01 * V[c] + G11 * V[3 + c];
    }
    double dT[6];  // 2 G T Sigma3D = 2 (G V) M^T
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c)
            dT[r * 3 + c] = 2.0 * (GV[r * 3 + 0] * M[c * 3 + 0] + GV[r * 3 + 1] * M[c * 3 + 1] + GV[r * 3 + 2] * M[c * 3 + 2]);
    double dJ00 = 0.0, dJ02 = 0.0, dJ11 = 0.0, dJ12 = 0.0;
    for (int c = 0; c < 3; ++c) {
        dJ00 += dT[c] * (double)R[c];
        dJ02 += dT[c] * (double)R[6 + c];
        dJ11 += dT[3 + c] * (double)R[3 + c];
        dJ12 += dT[3 + c] * (double)R[6 + c];
    }
    double dp[3] = {0.0, 0.0, 0.0};
    dp[2] += dJ00 * (-fx / z2) + dJ11 * (-fy / z2);
    double dtx = dJ02 * (-fx / z2), dty = dJ12 * (-fy / z2);
    dp[2] += dJ02 * (2.0 * fx * tx / z3) + dJ12 * (2.0 * fy * ty / z3);
    if (clx == 0.f) dp[0] += dtx; else dp[2] += dtx * clx * cam.limx;
    if (cly == 0.f) dp[1] += dty; else dp[2] += dty * cly * cam.limy;
    double dpx = px, dpy = py;
    dp[0] += du * fx / z1;
    dp[2] += du * (-fx * dpx / z2);
    dp[1] += dv * fy / z1;
    dp[2] += dv * (-fy * dpy / z2);
    for (int c = 0; c < 3; ++c)
        dm[c] += (double)R[c] * dp[0] + (double)R[3 + c] * dp[1] + (double)R[6 + c] * dp[2];
    // Sigma = M M^T, M = R diag(s): dL/dM = 2 T^T G T M = 2 T^T (G V)
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) dMs[r * 3 + c] += 2.0 * (T[r] * GV[c] + T[3 + r] * GV[3 + c]);
    return true;
}

__device__ __forceinline__ void geometry_finish(int64_t i, int64_t n, const float* __restrict__ log_scales,
                                                const float* __restrict__ quats, const float* __restrict__ logits,
                                                const double dM[9], float dop, double dls[3], double dq[4],
                                                float& dlogit)
{
    double s[3], Rq[9], qn[4], nr;
    geometry_scales(i, n, log_scales, s);
    geometry_rotation(i, n, quats, Rq, qn, nr);
    double w = qn[0], x = qn[1], y = qn[2], z = qn[3];
    double dR[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) dR[r * 3 + c] = dM[r * 3 + c] * s[c];
    for (int c = 0; c < 3; ++c)
        dls[c] += (dM[c] * Rq[c] + dM[3 + c] * Rq[3 + c] + dM[6 + c] * Rq[6 + c]) * s[c];
    double gq[4];
    gq[0] = 2.0 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    gq[1] = 2.0 * (y * dR[1] + z * dR[2] + y * dR[3] - 2.0 * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] -
                   2.0 * x * dR[8]);
    gq[2] = 2.0 * (-2.0 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] -
                   2.0 * y * dR[8]);
    gq[3] = 2.0 * (-2.0 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.0 * z * dR[4] + y * dR[5] + x * dR[6] +
                   y * dR[7]);
    double qd = w * gq[0] + x * gq[1] + y * gq[2] + z * gq[3];
    for (int k = 0; k < 4; ++k) dq[k] += (gq[k] - qn[k] * qd) / nr;
    float o = (float)(1.0 / (1.0 + exp(-(double)logits[i])));
    dlogit += dop * o * (1.0f - o);
}

// dL/drgb of one view: the forward clamps rgb at 0, so no gradient where the
// clamp was active (s2 = the splat's colour record).
__device__ __forceinline__ void colour_grad(const float4& s2, const float* __restrict__ g2, float drgb[3])
{
    drgb[0] = s2.x > 0.0f ? g2[6] : 0.0f;
    drgb[1] = s2.y > 0.0f ? g2[7] : 0.0f;
    drgb[2] = s2.z > 0.0f ? g2[8] : 0.0f;
}

// Unit view direction from a camera centre to the mean; returns its length.
__device__ __forceinline__ float view_dir(float mx, float my, float mz, const float campos[3], float dir[3])
{
    float dxw = mx - campos[0], dyw = my - campos[1], dzw = mz - campos[2];
    float dn = sqrtf(dxw * dxw + dyw * dyw + dzw * dzw);
    dir[0] = dxw; dir[1] = dyw; dir[2] = dzw;
    if (dn > 0.0f) { dir[0] /= dn; dir[1] /= dn; dir[2] /= dn; }
    return dn;
}

// Single view, geometry: the mean (through the projection), log-scales,
// quaternion and logit (the colour's share of the mean gradient follows in
// k_sh_backward).  Invisible Gaussians get zero gradients.
__global__ __launch_bounds__(QB_BLOCK) void k_geometry_backward(
    int64_t n, const float* __restrict__ means, const float* __restrict__ log_scales,
    const float* __restrict__ quats, const float* __restrict__ logits, BwdCam cam,
    const float* __restrict__ grad2d, float* __restrict__ d_means,
    float* __restrict__ d_log_scales, float* __restrict__ d_quats, float* __restrict__ d_logits)
{
    int64_t i = (int64_t)blockIdx.x * QB_BLOCK + threadIdx.x;
    if (i >= n) return;
    double dm[3] = {0.0, 0.0, 0.0}, dls[3] = {0.0, 0.0, 0.0}, dq[4] = {0.0, 0.0, 0.0, 0.0};
    float dlogit = 0.f;
    const float* g2 = grad2d + 9 * i;
    if (g2[0] != 0.f || g2[1] != 0.f || g2[2] != 0.f || g2[3] != 0.f || g2[4] != 0.f || g2[5] != 0.f) {
        GeoPrep g;
        geometry_prep(i, n, means, log_scales, quats, g);
        double dM[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        float dop = 0.f;
        geometry_view(g, cam, g2, dm, dM, dop);
        geometry_finish(i, n, log_scales, quats, logits, dM, dop, dls, dq, dlogit);
    }
    for (int c = 0; c < 3; ++c) {
        d_means[c * n + i] = (float)dm[c];
        d_log_scales[c * n + i] = (float)dls[c];
    }
    for (int c = 0; c < 4; ++c) d_quats[c * n + i] = (float)dq[c];
    d_logits[i] = dlogit;
}

// Single view, colour: SH coefficients, and the colour's share of the mean
// gradient (through the view direction) added to d_means.
template <int DEG>
__global__ __launch_bounds__(QB_BLOCK) void k_sh_backward(
    int64_t n, const float* __restrict__ means, const float* __restrict__ sh, BwdCam cam,
    const float4* __restrict__ splats, const float* __restrict__ grad2d, float* __restrict__ d_means,
    float* __restrict__ d_sh)
{
    constexpr int K = (DEG + 1) * (DEG + 1);
    int64_t i = (int64_t)blockIdx.x * QB_BLOCK + threadIdx.x;
    if (i >= n) return;
    float4 s2 = splats[3 * i + 2];
    if (s2.w != 1.0f) {
#pragma unroll
        for (int k = 0; k < K * 3; ++k) d_sh[(int64_t)k * n + i] = 0.f;
        return;
    }
    float dir[3], drgb[3], ddir[3];
    float dn = view_dir(means[i], means[n + i], means[2 * n + i], cam.campos, dir);
    colour_grad(s2, grad2d + 9 * i, drgb);
    sh_colour_backward(sh, n, i, DEG, dir[0], dir[1], dir[2], drgb, d_sh, ddir);
    if (dn > 0.0f) {
        float dd = ddir[0] * dir[0] + ddir[1] * dir[1] + ddir[2] * dir[2];
        for (int c = 0; c < 3; ++c) d_means[c * n + i] += (ddir[c] - dir[c] * dd) / dn;
    }
}

// Views: the geometry part summed over views (the colour's share of the
// mean gradient follows in k_sh_backward_views).  Three waves per SIMD are
// asked for (178 -> 168 VGPRs at the price of 44 bytes of spills): 0.14 ms
// less over 32 views of 2M Gaussians than at two.
// CLEAR: the SH kernel ran first (it stored d_means), this one adds to
// d_means and then zeroes every nonzero grad2d row it read, so that the next
// step's render backward can add into grad2d without clearing it.
template <bool CLEAR>
__global__ __launch_bounds__(QB_BLOCK, 3) void k_geometry_backward_views(
    int64_t n, int nv, const float* __restrict__ means, const float* __restrict__ log_scales,
    const float* __restrict__ quats, const float* __restrict__ logits, BwdCamTable cams,
    float* __restrict__ grad2d, float* __restrict__ d_means,
    float* __restrict__ d_log_scales, float* __restrict__ d_quats, float* __restrict__ d_logits)
{
    int64_t i = (int64_t)blockIdx.x * QB_BLOCK + threadIdx.x;
    if (i >= n) return;
    double dm[3] = {0.0, 0.0, 0.0}, dls[3] = {0.0, 0.0, 0.0}, dq[4] = {0.0, 0.0, 0.0, 0.0};
    float dlogit = 0.f;
    GeoPrep g;
    geometry_prep(i, n, means, log_scales, quats, g);
    double dM[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    float dop = 0.f;
    bool any = false;
    for (int v = 0; v < nv; ++v) {
        float* g2 = grad2d + 9 * ((int64_t)v * n + i);
        bool used = geometry_view(g, cams.cam[v], g2, dm, dM, dop);
        any |= used;
        if (CLEAR && (used || g2[6] != 0.f || g2[7] != 0.f || g2[8] != 0.f))
#pragma unroll
            for (int k = 0; k < 9; ++k) g2[k] = 0.f;
    }
    // (a culled Gaussian, whose rows are all zero, may have no valid rotation)
    if (any) geometry_finish(i, n, log_scales, quats, logits, dM, dop, dls, dq, dlogit);
    for (int c = 0; c < 3; ++c) {
        if (CLEAR) d_means[c * n + i] += (float)dm[c];
        else d_means[c * n + i] = (float)dm[c];
        d_log_scales[c * n + i] = (float)dls[c];
    }
    for (int c = 0; c < 4; ++c) d_quats[c * n + i] = (float)dq[c];
    d_logits[i] = dlogit;
}

// Views: SH coefficients and the colour's share of the mean gradient, summed
// over views in registers.  FIRST: runs before k_geometry_backward_views and
// stores its share of d_means, which that kernel then adds to; otherwise it
// runs after it and adds its share.
template <int DEG, bool FIRST>
__global__ __launch_bounds__(QB_BLOCK) void k_sh_backward_views(
    int64_t n, int nv, const float* __restrict__ means, const float* __restrict__ sh, BwdCamTable cams,
    const float4* __restrict__ splats, const float* __restrict__ grad2d, float* __restrict__ d_means,
    float* __restrict__ d_sh)
{
    constexpr int K = (DEG + 1) * (DEG + 1);
    int64_t i = (int64_t)blockIdx.x * QB_BLOCK + threadIdx.x;
    if (i >= n) return;
    float coef[K * 3], acc[K * 3];
#pragma unroll
    for (int k = 0; k < K * 3; ++k) {
        coef[k] = sh[(int64_t)k * n + i];
        acc[k] = 0.0f;
    }
    float mx = means[i], my = means[n + i], mz = means[2 * n + i];
    float dmx = 0.f, dmy = 0.f, dmz = 0.f;
    for (int v = 0; v < nv; ++v) {
        int64_t vi = (int64_t)v * n + i;
        // a zero colour row adds nothing (culled Gaussians, and views where
        // no pixel composites the Gaussian): only the others read the splat
        const float* g2 = grad2d + 9 * vi;
        if (g2[6] == 0.f && g2[7] == 0.f && g2[8] == 0.f) continue;
        float4 s2 = splats[3 * vi + 2];
        if (s2.w != 1.0f) continue;
        float dir[3], drgb[3];
        float dn = view_dir(mx, my, mz, cams.cam[v].campos, dir);
        colour_grad(s2, g2, drgb);
        float Y[16], G[16][3];
        sh_basis_and_grad(dir[0], dir[1], dir[2], Y, G);
        float ddir[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < K; ++k) {
            // dL/dY_k = sum over the channels of coef * drgb
            float cw = fmaf(coef[k * 3 + 2], drgb[2], fmaf(coef[k * 3 + 1], drgb[1], coef[k * 3] * drgb[0]));
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) acc[k * 3 + ch] = fmaf(Y[k], drgb[ch], acc[k * 3 + ch]);
            ddir[0] = fmaf(G[k][0], cw, ddir[0]);
            ddir[1] = fmaf(G[k][1], cw, ddir[1]);
            ddir[2] = fmaf(G[k][2], cw, ddir[2]);
        }
        if (dn > 0.0f) {
            float dd = ddir[0] * dir[0] + ddir[1] * dir[1] + ddir[2] * dir[2];
            dmx += (ddir[0] - dir[0] * dd) / dn;
            dmy += (ddir[1] - dir[1] * dd) / dn;
            dmz += (ddir[2] - dir[2] * dd) / dn;
        }
    }
#pragma unroll
    for (int k = 0; k < K * 3; ++k) d_sh[(int64_t)k * n + i] = acc[k];
    if (FIRST) {
        d_means[i] = dmx;
        d_means[n + i] = dmy;
        d_means[2 * n + i] = dmz;
    } else {
        d_means[i] += dmx;
        d_means[n + i] += dmy;
        d_means[2 * n + i] += dmz;
    }
}

// qb_l1_grad: the items of one launch, by value as a kernel argument.  Item v
// takes workgroups [wg0[v], wg0[v + 1]); each lane handles 4 consecutive
// elements (one 16-byte load of each input where the item allows it).
struct L1Table {
    const float* image[QB_MAX_VIEWS];
    const float* target[QB_MAX_VIEWS];
    float* grad[QB_MAX_VIEWS];
    int64_t count[QB_MAX_VIEWS];
    float scale[QB_MAX_VIEWS];
    int64_t wg0[QB_MAX_VIEWS + 1];
    int vec[QB_MAX_VIEWS];  // count % 4 == 0 and 16-byte aligned pointers
    int num;
};

__device__ __forceinline__ float l1_sign_scaled(float a, float b, float s)
{
    float d = a - b;  // its sign is that of a - b: rounding keeps signs and zero
    return d > 0.0f ? s : (d < 0.0f ? -s : 0.0f);
}

__global__ __launch_bounds__(QB_BLOCK) void k_l1_grad(L1Table t)
{
    int64_t b = blockIdx.x;
    int v = 0;
    while (v + 1 < t.num && t.wg0[v + 1] <= b) ++v;
    int64_t i = ((b - t.wg0[v]) * QB_BLOCK + threadIdx.x) * 4;
    int64_t cnt = t.count[v];
    if (i >= cnt) return;
    const float* img = t.image[v];
    const float* tgt = t.target[v];
    float* g = t.grad[v];
    float s = t.scale[v];
    if (t.vec[v]) {
        float4 x = *reinterpret_cast<const float4*>(img + i), y = *reinterpret_cast<const float4*>(tgt + i);
        *reinterpret_cast<float4*>(g + i) = make_float4(l1_sign_scaled(x.x, y.x, s), l1_sign_scaled(x.y, y.y, s),
                                                        l1_sign_scaled(x.z, y.z, s), l1_sign_scaled(x.w, y.w, s));
    } else {
        for (int64_t k = i; k < i + 4 && k < cnt; ++k) g[k] = l1_sign_scaled(img[k], tgt[k], s);
    }
}

__global__ void k_zero(float* __restrict__ p, int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * QB_BLOCK + threadIdx.x; i < count; i += (int64_t)gridDim.x * QB_BLOCK)
        p[i] = 0.0f;
}

}  // namespace

namespace {

// Camera constants of the backward; lim = 1.3 * (0.5 W / fx) as the forward.
void make_bwd_cam(const qb_camera& cam, BwdCam* bc)
{
    bc->W = cam.width;
    bc->H = cam.height;
    bc->fx = cam.fx; bc->fy = cam.fy; bc->cx = cam.cx; bc->cy = cam.cy;
    bc->near_plane = cam.near_plane;
    for (int k = 0; k < 9; ++k) bc->R[k] = cam.R[k];
    for (int k = 0; k < 3; ++k) { bc->t[k] = cam.t[k]; bc->campos[k] = cam.campos[k]; }
    volatile float hx = 0.5f * (float)cam.width;
    volatile float hy = 0.5f * (float)cam.height;
    bc->limx = 1.3f * (hx / cam.fx);
    bc->limy = 1.3f * (hy / cam.fy);
}

}  // namespace

extern "C" qb_status qb_render_backward_ex(int32_t width, int32_t height, const uint32_t* ranges,
                                           const uint32_t* ids, const qb_splat* splats, const float* bg,
                                           const float* final_T, const uint32_t* n_contrib, const float* dL_dimage,
                                           int64_t n, float* grad2d, int32_t variant, const uint32_t* tile_order,
                                           qb_stream_t stream)
{
    if (width <= 0 || height <= 0 || width > 32767 * QB_TILE || height > 32767 * QB_TILE || !ranges || !bg ||
        !final_T || !n_contrib || !dL_dimage || n < 0 || (n > 0 && (!grad2d || !splats)) || variant < 0 ||
        variant > QB_RENDER_4PX)
        return QB_ERR_INVALID_ARG;
    int tiles_x = (int)qb_div_up(width, QB_TILE);
    int64_t tiles = (int64_t)tiles_x * qb_div_up(height, QB_TILE);
    if (tiles > (1 << 24)) return QB_ERR_INVALID_ARG;
    hipStream_t s = qb_hip_stream(stream);
    if (n > 0) {
        int64_t g = qb_div_up(9 * n, QB_BLOCK);
        QB_LAUNCH(k_zero, g > 4096 ? 4096 : g, QB_BLOCK, 0, s, grad2d, 9 * n);
    }
    const uint2* rg = reinterpret_cast<const uint2*>(ranges);
    const float4* sp = reinterpret_cast<const float4*>(splats);
    switch (variant) {
    case QB_RENDER_2PX:
        QB_LAUNCH(k_render_backward<2>, tiles, 128, 0, s, (int)width, (int)height, tiles_x, rg, ids, sp, bg[0],
                  bg[1], bg[2], final_T, n_contrib, dL_dimage, grad2d, tile_order);
        break;
    case QB_RENDER_1PX:
        QB_LAUNCH(k_render_backward<1>, tiles, 256, 0, s, (int)width, (int)height, tiles_x, rg, ids, sp, bg[0],
                  bg[1], bg[2], final_T, n_contrib, dL_dimage, grad2d, tile_order);
        break;
    default:
        QB_LAUNCH(k_render_backward<4>, tiles, 64, 0, s, (int)width, (int)height, tiles_x, rg, ids, sp, bg[0],
                  bg[1], bg[2], final_T, n_contrib, dL_dimage, grad2d, tile_order);
        break;
    }
    return QB_OK;
}

extern "C" qb_status qb_render_backward(int32_t width, int32_t height, const uint32_t* ranges, const uint32_t* ids,
                                        const qb_splat* splats, const float* bg, const float* final_T,
                                        const uint32_t* n_contrib, const float* dL_dimage, int64_t n,
                                        float* grad2d, qb_stream_t stream)
{
    return qb_render_backward_ex(width, height, ranges, ids, splats, bg, final_T, n_contrib, dL_dimage, n, grad2d,
                                 QB_RENDER_2PX, nullptr, stream);
}

extern "C" qb_status qb_project_backward(int64_t n, const float* means, const float* log_scales,
                                         const float* quats, const float* opacity_logits, const float* sh,
                                         int32_t sh_degree, const qb_camera* cam, const qb_splat* splats,
                                         const float* grad2d, float* d_means, float* d_log_scales, float* d_quats,
                                         float* d_opacity_logits, float* d_sh, qb_stream_t stream)
{
    if (n < 0 || n >= (int64_t)1 << 31 || !cam || sh_degree < 0 || sh_degree > 3) return QB_ERR_INVALID_ARG;
    if (!qb_valid_camera(*cam)) return QB_ERR_INVALID_ARG;
    if (n == 0) return QB_OK;
    if (!means || !log_scales || !quats || !opacity_logits || !sh || !splats || !grad2d || !d_means ||
        !d_log_scales || !d_quats || !d_opacity_logits || !d_sh)
        return QB_ERR_INVALID_ARG;
    BwdCam bc;
    make_bwd_cam(*cam, &bc);
    hipStream_t s = qb_hip_stream(stream);
    int64_t grid = qb_div_up(n, QB_BLOCK);
    const float4* sp = reinterpret_cast<const float4*>(splats);
    QB_LAUNCH(k_geometry_backward, grid, QB_BLOCK, 0, s, n, means, log_scales, quats, opacity_logits, bc, grad2d,
              d_means, d_log_scales, d_quats, d_opacity_logits);
    switch (sh_degree) {
    case 0: QB_LAUNCH(k_sh_backward<0>, grid, QB_BLOCK, 0, s, n, means, sh, bc, sp, grad2d, d_means, d_sh); break;
    case 1: QB_LAUNCH(k_sh_backward<1>, grid, QB_BLOCK, 0, s, n, means, sh, bc, sp, grad2d, d_means, d_sh); break;
    case 2: QB_LAUNCH(k_sh_backward<2>, grid, QB_BLOCK, 0, s, n, means, sh, bc, sp, grad2d, d_means, d_sh); break;
    default: QB_LAUNCH(k_sh_backward<3>, grid, QB_BLOCK, 0, s, n, means, sh, bc, sp, grad2d, d_means, d_sh); break;
    }
    return QB_OK;
}

// The batched render backward; clear: zero every view's grad2d first, else
// add to what it holds.
static qb_status render_backward_views(int32_t num_views, const qb_view* views, const float* bg, int64_t n,
                                       int32_t variant, const uint32_t* tile_order, bool clear, qb_stream_t stream)
{
    if (!bg || n < 0 || variant < 0 || variant > QB_RENDER_4PX) return QB_ERR_INVALID_ARG;
    QbViewTable vt;
    qb_status st = qb_make_view_table(num_views, views, true, &vt);
    if (st != QB_OK) return st;
    hipStream_t s = qb_hip_stream(stream);
    if (n > 0 && clear) {
        int64_t g = qb_div_up(9 * n, QB_BLOCK);
        QB_LAUNCH(k_zero_views, dim3(g > 1024 ? 1024 : (unsigned)g, num_views), QB_BLOCK, 0, s, vt, 9 * n);
    }
    int tiles = vt.tile_start[num_views];
    if (tiles == 0) return QB_OK;
    switch (variant) {
    case QB_RENDER_2PX: QB_LAUNCH(k_render_backward_views<2>, tiles, 128, 0, s, vt, tile_order, bg[0], bg[1], bg[2]); break;
    case QB_RENDER_1PX: QB_LAUNCH(k_render_backward_views<1>, tiles, 256, 0, s, vt, tile_order, bg[0], bg[1], bg[2]); break;
    default: QB_LAUNCH(k_render_backward_views<4>, tiles, 64, 0, s, vt, tile_order, bg[0], bg[1], bg[2]); break;
    }
    return QB_OK;
}

extern "C" qb_status qb_render_backward_views_ex(int32_t num_views, const qb_view* views, const float* bg,
                                                 int64_t n, int32_t variant, const uint32_t* tile_order,
                                                 qb_stream_t stream)
{
    return render_backward_views(num_views, views, bg, n, variant, tile_order, true, stream);
}

extern "C" qb_status qb_render_backward_views_acc(int32_t num_views, const qb_view* views, const float* bg,
                                                  int64_t n, int32_t variant, const uint32_t* tile_order,
                                                  qb_stream_t stream)
{
    return render_backward_views(num_views, views, bg, n, variant, tile_order, false, stream);
}

extern "C" qb_status qb_render_backward_views(int32_t num_views, const qb_view* views, const float* bg, int64_t n,
                                              qb_stream_t stream)
{
    return qb_render_backward_views_ex(num_views, views, bg, n, QB_RENDER_2PX, nullptr, stream);
}

// The batched projection backward; clear: the SH kernel first, then the
// geometry kernel, which zeroes the grad2d rows it has read.
static qb_status project_backward_views(int64_t n, const float* means, const float* log_scales, const float* quats,
                                        const float* opacity_logits, const float* sh, int32_t sh_degree,
                                        const qb_camera* cams, int32_t num_views, const qb_splat* splats,
                                        float* grad2d, float* d_means, float* d_log_scales, float* d_quats,
                                        float* d_opacity_logits, float* d_sh, bool clear, qb_stream_t stream)
{
    if (n < 0 || n >= (int64_t)1 << 31 || !cams || sh_degree < 0 || sh_degree > 3 || num_views < 1 ||
        num_views > QB_MAX_VIEWS)
        return QB_ERR_INVALID_ARG;
    BwdCamTable ct;
    for (int v = 0; v < num_views; ++v) {
        const qb_camera& c = cams[v];
        if (!qb_valid_camera(c)) return QB_ERR_INVALID_ARG;
        make_bwd_cam(c, &ct.cam[v]);
    }
    if (n == 0) return QB_OK;
    if (!means || !log_scales || !quats || !opacity_logits || !sh || !splats || !grad2d || !d_means ||
        !d_log_scales || !d_quats || !d_opacity_logits || !d_sh)
        return QB_ERR_INVALID_ARG;
    hipStream_t s = qb_hip_stream(stream);
    int64_t grid = qb_div_up(n, QB_BLOCK);
    const float4* sp = reinterpret_cast<const float4*>(splats);
#define QB_SH_VIEWS(FIRST)                                                                                     \
    switch (sh_degree) {                                                                                       \
    case 0: QB_LAUNCH((k_sh_backward_views<0, FIRST>), grid, QB_BLOCK, 0, s, n, (int)num_views, means, sh, ct, sp, \
                      grad2d, d_means, d_sh); break;                                                           \
    case 1: QB_LAUNCH((k_sh_backward_views<1, FIRST>), grid, QB_BLOCK, 0, s, n, (int)num_views, means, sh, ct, sp, \
                      grad2d, d_means, d_sh); break;                                                           \
    case 2: QB_LAUNCH((k_sh_backward_views<2, FIRST>), grid, QB_BLOCK, 0, s, n, (int)num_views, means, sh, ct, sp, \
                      grad2d, d_means, d_sh); break;                                                           \
    default: QB_LAUNCH((k_sh_backward_views<3, FIRST>), grid, QB_BLOCK, 0, s, n, (int)num_views, means, sh, ct,   \
                       sp, grad2d, d_means, d_sh); break;                                                      \
    }
    if (clear) {
        QB_SH_VIEWS(true);
        QB_LAUNCH((k_geometry_backward_views<true>), grid, QB_BLOCK, 0, s, n, (int)num_views, means, log_scales, quats,
                  opacity_logits, ct, grad2d, d_means, d_log_scales, d_quats, d_opacity_logits);
    } else {
        QB_LAUNCH((k_geometry_backward_views<false>), grid, QB_BLOCK, 0, s, n, (int)num_views, means, log_scales,
                  quats, opacity_logits, ct, grad2d, d_means, d_log_scales, d_quats, d_opacity_logits);
        QB_SH_VIEWS(false);
    }
#undef QB_SH_VIEWS
    return QB_OK;
}

extern "C" qb_status qb_project_backward_views(int64_t n, const float* means, const float* log_scales,
                                               const float* quats, const float* opacity_logits, const float* sh,
                                               int32_t sh_degree, const qb_camera* cams, int32_t num_views,
                                               const qb_splat* splats, const float* grad2d, float* d_means,
                                               float* d_log_scales, float* d_quats, float* d_opacity_logits,
                                               float* d_sh, qb_stream_t stream)
{
    // without clearing, grad2d is only read
    return project_backward_views(n, means, log_scales, quats, opacity_logits, sh, sh_degree, cams, num_views,
                                  splats, const_cast<float*>(grad2d), d_means, d_log_scales, d_quats,
                                  d_opacity_logits, d_sh, false, stream);
}

extern "C" qb_status qb_project_backward_views_ex(int64_t n, const float* means, const float* log_scales,
                                                  const float* quats, const float* opacity_logits, const float* sh,
                                                  int32_t sh_degree, const qb_camera* cams, int32_t num_views,
                                                  const qb_splat* splats, float* grad2d, float* d_means,
                                                  float* d_log_scales, float* d_quats, float* d_opacity_logits,
                                                  float* d_sh, int32_t clear_grad2d, qb_stream_t stream)
{
    if (clear_grad2d != 0 && clear_grad2d != 1) return QB_ERR_INVALID_ARG;
    return project_backward_views(n, means, log_scales, quats, opacity_logits, sh, sh_degree, cams, num_views,
                                  splats, grad2d, d_means, d_log_scales, d_quats, d_opacity_logits, d_sh,
                                  clear_grad2d != 0, stream);
}

extern "C" qb_status qb_l1_grad(int32_t num_items, const qb_l1_item* items, qb_stream_t stream)
{
    if (num_items < 0 || num_items > QB_MAX_VIEWS || (num_items > 0 && !items)) return QB_ERR_INVALID_ARG;
    L1Table t;
    t.num = num_items;
    t.wg0[0] = 0;
    constexpr int64_t kPerBlock = 4 * QB_BLOCK;
    for (int v = 0; v < num_items; ++v) {
        const qb_l1_item& it = items[v];
        if (it.count < 0 || (it.count > 0 && (!it.image || !it.target || !it.grad))) return QB_ERR_INVALID_ARG;
        t.image[v] = it.image;
        t.target[v] = it.target;
        t.grad[v] = it.grad;
        t.count[v] = it.count;
        t.scale[v] = it.scale;
        t.vec[v] = (it.count % 4 == 0) && (((uintptr_t)it.image | (uintptr_t)it.target | (uintptr_t)it.grad) & 15u) == 0;
        t.wg0[v + 1] = t.wg0[v] + qb_div_up(it.count, kPerBlock);
    }
    int64_t grid = num_items > 0 ? t.wg0[num_items] : 0;
    if (grid == 0) return QB_OK;
    if (grid > 0x7FFFFFFF) return QB_ERR_INVALID_ARG;
    QB_LAUNCH(k_l1_grad, grid, QB_BLOCK, 0, qb_hip_stream(stream), t);
    return QB_OK;
}
