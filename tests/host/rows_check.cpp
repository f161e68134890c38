// Host-side check of entry_rows (the per-entry row range the render and its
// backward use to let a wave skip entries): every pixel of a tile whose
// binary32 power passes the cutoff (power in [-gamma/2, 0], the render's
// exact decision) lies in the rows [r0, r1] it returns.  Random Gaussians
// with eigenvalues of Sigma2D from 0.3 to 1e6 (needles up to condition 1e6),
// random orientation, centre and opacity.  Prints "cases N bad M".
#include "../../paper_2605_04844_amd/csrc/qb_common.h"

#include <cmath>
#include <cstdio>
#include <random>

int main()
{
    std::mt19937 rng(777);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    long cases = 0, bad = 0;
    for (int it = 0; it < 20000; ++it) {
        double l1 = 0.3 + std::pow(10.0, 6.0 * U(rng)), l2 = 0.3 + std::pow(10.0, 6.0 * U(rng)) * (U(rng) < 0.3 ? 1e-6 : 1.0);
        double th = 2.0 * M_PI * U(rng), cs = std::cos(th), sn = std::sin(th);
        double A = l1 * cs * cs + l2 * sn * sn, B = (l1 - l2) * cs * sn, C = l1 * sn * sn + l2 * cs * cs;
        double det = A * C - B * B;
        if (!(det > 0)) continue;
        float a = (float)(C / det), b = (float)(-B / det), c = (float)(A / det);
        float o = (float)(1.0 / 255.0 + (1.0 - 1.0 / 255.0) * U(rng));
        float gamma = (float)(2.0 * std::log(255.0 * (double)o));
        if (!(gamma > 0.0f)) continue;
        int ty = (int)(U(rng) * 40);
        float u = (float)(U(rng) * 640.0), v = (float)(ty * 16 + (U(rng) * 400.0 - 200.0));
        int rr = entry_rows(v, a, b, c, gamma, ty);
        int r0 = (int)(int16_t)(rr & 0xFFFF), r1 = rr >> 16;
        // brute force over the tile's 16 rows and a window of columns
        double hx = std::sqrt((double)gamma * C) + 2.0;
        int x0 = (int)std::floor(u - hx), x1 = (int)std::ceil(u + hx);
        if (x1 - x0 > 4000) { x0 = (int)u - 2000; x1 = (int)u + 2000; }
        ++cases;
        for (int r = 0; r < 16; ++r) {
            float py = (float)(ty * 16 + r), dy = v - py;
            for (int px = x0; px <= x1; ++px) {
                float dx = u - (float)px;
                float p = std::fmaf(std::fmaf(-0.5f * a, dx, (-b) * dy), dx, ((-0.5f * c) * dy) * dy);
                bool pass = !(p > 0.0f || p < -0.5f * gamma);
                if (pass && (r < r0 || r > r1)) {
                    if (bad < 5) printf("miss: case %d row %d not in [%d, %d]\n", it, r, r0, r1);
                    ++bad;
                    r = 16;
                    break;
                }
            }
        }
    }
    printf("cases %ld bad %ld\n", cases, bad);
    return bad != 0;
}
