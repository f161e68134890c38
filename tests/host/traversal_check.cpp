// Host-side check of the two tile traversals of a QuadBox (Sec. 3.2): QPass
// runs (qpass_runs) and the naive nested-loop walk (naive_walk) must each
// visit every tile of the union of the sub-box rects exactly once, and report
// its size.  The rects are quadrant boxes around one centre, as QuadBox and
// DualBox build them (QPass's per-scanline min/max relies on that shape),
// with random extents, empty and dropped sub-boxes, clipped to the image, and
// in half of the cases cut to a common square around the centre.
// Prints "cases N bad M" and exits non-zero on any mismatch.
#include "../../paper_2605_04844_amd/csrc/qb_common.h"

#include <cmath>
#include <cstdio>
#include <random>
#include <set>
#include <vector>

// Tile range of the pixel samples in [a0, a1] on an axis of n pixels.
static bool axis_tiles(float a0, float a1, int n, int* t0, int* t1)
{
    float hi = (float)(n - 1);
    if (!(a1 >= 0.0f) || !(a0 <= hi)) return false;
    int p0 = (int)std::ceil(a0 > 0.0f ? a0 : 0.0f), p1 = (int)std::floor(a1 < hi ? a1 : hi);
    if (p0 > p1) return false;
    *t0 = p0 / QB_TILE;
    *t1 = p1 / QB_TILE;
    return true;
}

// Four quadrant boxes around a common centre (u, v), as a QuadBox has,
// with random extents (some zero) on a random image, clipped to it.
static void quadrant_rects(std::mt19937& rng, QRect r[4])
{
    int W = 1 + (int)(rng() % 400), H = 1 + (int)(rng() % 400);
    float u = (float)((int)(rng() % 6000) - 1000) / 10.0f, v = (float)((int)(rng() % 6000) - 1000) / 10.0f;
    for (int q = 0; q < 4; ++q) {
        int sx = (q & 1) ? 1 : -1, sy = (q & 2) ? 1 : -1;
        float w = (rng() % 7 == 0) ? 0.0f : (float)(rng() % 12000) / 100.0f;
        float h = (rng() % 7 == 0) ? 0.0f : (float)(rng() % 12000) / 100.0f;
        float x0 = sx > 0 ? u : u - w, x1 = sx > 0 ? u + w : u;
        float y0 = sy > 0 ? v : v - h, y1 = sy > 0 ? v + h : v;
        int a, b, c, d;
        r[q] = QRect{1, 0, 1, 0};
        if (axis_tiles(x0, x1, W, &a, &b) && axis_tiles(y0, y1, H, &c, &d)) r[q] = QRect{a, b, c, d};
        if (rng() % 9 == 0) r[q] = QRect{1, 0, 1, 0};  // a sub-box dropped (DualBox)
    }
    // every other case: all rects cut to the tile rect of a square around the
    // same centre (the 3-sigma clip), as k_project applies it
    if (rng() % 2 == 0) {
        float rad = (float)(rng() % 15000) / 100.0f;
        int a, b, c, d;
        bool sq = axis_tiles(u - rad, u + rad, W, &a, &b) && axis_tiles(v - rad, v + rad, H, &c, &d);
        for (int q = 0; q < 4; ++q) {
            QRect& k = r[q];
            if (k.x0 > k.x1 || k.y0 > k.y1) continue;
            if (!sq) { k = QRect{1, 0, 1, 0}; continue; }
            k.x0 = k.x0 > a ? k.x0 : a;
            k.x1 = k.x1 < b ? k.x1 : b;
            k.y0 = k.y0 > c ? k.y0 : c;
            k.y1 = k.y1 < d ? k.y1 : d;
            if (k.x0 > k.x1 || k.y0 > k.y1) k = QRect{1, 0, 1, 0};
        }
    }
}

int main()
{
    std::mt19937 rng(12345);
    long cases = 0, bad = 0;
    for (int it = 0; it < 200000; ++it) {
        QRect r[4];
        quadrant_rects(rng, r);
        std::set<int> want;
        for (int k = 0; k < 4; ++k)
            for (int y = r[k].y0; y <= r[k].y1; ++y)
                for (int x = r[k].x0; x <= r[k].x1; ++x) want.insert(y * 1024 + x);

        QRuns q;
        qpass_runs(r, q);
        std::multiset<int> got_q;
        for (int s = 0; s < QB_MAX_SEG; ++s)
            for (long j = 0; j < (long)q.n[s] * q.len[s]; ++j) {
                int sl = q.s0[s] + (int)(j / q.len[s]), ot = q.lo[s] + (int)(j % q.len[s]);
                int x = q.axis == 0 ? sl : ot, y = q.axis == 0 ? ot : sl;
                got_q.insert(y * 1024 + x);
            }
        std::vector<int> got_n;
        int seq_ok = 1;
        int cnt = naive_walk(r, [&](int x, int y, int c) {
            if (c != (int)got_n.size()) seq_ok = 0;
            got_n.push_back(y * 1024 + x);
        });
        std::set<int> set_q(got_q.begin(), got_q.end()), set_n(got_n.begin(), got_n.end());
        ++cases;
        bool ok = q.total == (int)want.size() && got_q.size() == want.size() && set_q == want &&
                  cnt == (int)want.size() && got_n.size() == want.size() && set_n == want && seq_ok;
        if (!ok) {
            if (bad < 5) printf("mismatch at case %d: union %zu qpass %d naive %d\n", it, want.size(), q.total, cnt);
            ++bad;
        }
    }
    printf("cases %ld bad %ld\n", cases, bad);
    return bad != 0;
}
