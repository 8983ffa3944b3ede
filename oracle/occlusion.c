/*
 * Segment any-hit against a triangle soup, FP64, for the CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle/__init__.py): this file is compiled
 * into a small shared library loaded by oracle/occlusion.py; the GPU library
 * neither includes nor links it.
 *
 * The visibility steps U^i, U^r and U of Eqs. (1)-(2) are 1 when a path's
 * straight segments miss every occluder.  Here a segment P0 -> P1 is blocked
 * if some triangle is crossed at a parameter t with eps < t < 1 - eps.  The
 * intersection is the Moller-Trumbore test (1997) in double precision; the
 * only acceleration is a uniform grid walked cell by cell along the segment
 * (Amanatides and Woo 1987), with every triangle stored in each cell its
 * bounding box overlaps.  brute != 0 skips the grid and tests every triangle.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int seg_tri(const double *p0, const double *d, const double *tri, double eps) {
    const double *v0 = tri, *v1 = tri + 3, *v2 = tri + 6;
    double e1[3], e2[3], pv[3], tv[3], qv[3];
    for (int i = 0; i < 3; ++i) { e1[i] = v1[i] - v0[i]; e2[i] = v2[i] - v0[i]; }
    pv[0] = d[1] * e2[2] - d[2] * e2[1];
    pv[1] = d[2] * e2[0] - d[0] * e2[2];
    pv[2] = d[0] * e2[1] - d[1] * e2[0];
    double det = e1[0] * pv[0] + e1[1] * pv[1] + e1[2] * pv[2];
    if (det == 0.0) return 0;
    double inv = 1.0 / det;
    for (int i = 0; i < 3; ++i) tv[i] = p0[i] - v0[i];
    double u = (tv[0] * pv[0] + tv[1] * pv[1] + tv[2] * pv[2]) * inv;
    if (u < 0.0 || u > 1.0) return 0;
    qv[0] = tv[1] * e1[2] - tv[2] * e1[1];
    qv[1] = tv[2] * e1[0] - tv[0] * e1[2];
    qv[2] = tv[0] * e1[1] - tv[1] * e1[0];
    double v = (d[0] * qv[0] + d[1] * qv[1] + d[2] * qv[2]) * inv;
    if (v < 0.0 || u + v > 1.0) return 0;
    double t = (e2[0] * qv[0] + e2[1] * qv[1] + e2[2] * qv[2]) * inv;
    return t > eps && t < 1.0 - eps;
}

typedef struct {
    double lo[3], cell[3];
    int res[3];
    int64_t *start; /* res[0]*res[1]*res[2] + 1 */
    int64_t *items;
} grid_t;

static int64_t cidx(const grid_t *g, int x, int y, int z) {
    return ((int64_t)z * g->res[1] + y) * g->res[0] + x;
}

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

static void tri_cells(const grid_t *g, const double *t, int lo[3], int hi[3]) {
    for (int a = 0; a < 3; ++a) {
        double mn = fmin(t[a], fmin(t[3 + a], t[6 + a]));
        double mx = fmax(t[a], fmax(t[3 + a], t[6 + a]));
        lo[a] = clampi((int)floor((mn - g->lo[a]) / g->cell[a]), 0, g->res[a] - 1);
        hi[a] = clampi((int)floor((mx - g->lo[a]) / g->cell[a]), 0, g->res[a] - 1);
    }
}

static int build_grid(grid_t *g, const double *tri, int64_t n) {
    double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = 0; i < n * 3; ++i)
        for (int a = 0; a < 3; ++a) {
            mn[a] = fmin(mn[a], tri[i * 3 + a]);
            mx[a] = fmax(mx[a], tri[i * 3 + a]);
        }
    double ext[3], vol = 1.0;
    for (int a = 0; a < 3; ++a) {
        double pad = 1e-6 * (mx[a] - mn[a]) + 1e-9;
        mn[a] -= pad; mx[a] += pad;
        ext[a] = mx[a] - mn[a];
        vol *= ext[a];
    }
    double target = 2.0 * (double)n;
    double h = cbrt(vol / target);
    for (int a = 0; a < 3; ++a) {
        int r = (int)ceil(ext[a] / h);
        g->res[a] = r < 1 ? 1 : (r > 512 ? 512 : r);
        g->lo[a] = mn[a];
        g->cell[a] = ext[a] / g->res[a];
    }
    int64_t nc = (int64_t)g->res[0] * g->res[1] * g->res[2];
    int64_t *cnt = calloc(nc + 1, sizeof(int64_t));
    if (!cnt) return -1;
    for (int64_t i = 0; i < n; ++i) {
        int lo[3], hi[3];
        tri_cells(g, tri + 9 * i, lo, hi);
        for (int z = lo[2]; z <= hi[2]; ++z)
            for (int y = lo[1]; y <= hi[1]; ++y)
                for (int x = lo[0]; x <= hi[0]; ++x) cnt[cidx(g, x, y, z) + 1]++;
    }
    for (int64_t c = 0; c < nc; ++c) cnt[c + 1] += cnt[c];
    g->start = cnt;
    g->items = malloc(sizeof(int64_t) * (cnt[nc] > 0 ? cnt[nc] : 1));
    int64_t *fill = malloc(sizeof(int64_t) * nc);
    if (!g->items || !fill) return -1;
    memcpy(fill, cnt, sizeof(int64_t) * nc);
    for (int64_t i = 0; i < n; ++i) {
        int lo[3], hi[3];
        tri_cells(g, tri + 9 * i, lo, hi);
        for (int z = lo[2]; z <= hi[2]; ++z)
            for (int y = lo[1]; y <= hi[1]; ++y)
                for (int x = lo[0]; x <= hi[0]; ++x) g->items[fill[cidx(g, x, y, z)]++] = i;
    }
    free(fill);
    return 0;
}

/* Walk the cells the segment passes (clipped to the grid box). */
static int walk(const grid_t *g, const double *tri, const double *p0, const double *d, double eps) {
    double t0 = 0.0, t1 = 1.0;
    for (int a = 0; a < 3; ++a) {
        double hi = g->lo[a] + g->cell[a] * g->res[a];
        if (d[a] == 0.0) {
            if (p0[a] < g->lo[a] || p0[a] > hi) return 0;
        } else {
            double ta = (g->lo[a] - p0[a]) / d[a], tb = (hi - p0[a]) / d[a];
            if (ta > tb) { double s = ta; ta = tb; tb = s; }
            t0 = fmax(t0, ta);
            t1 = fmin(t1, tb);
        }
    }
    if (t0 > t1) return 0;
    int c[3], step[3];
    double tmax[3], tdelta[3];
    for (int a = 0; a < 3; ++a) {
        double p = p0[a] + t0 * d[a];
        c[a] = clampi((int)floor((p - g->lo[a]) / g->cell[a]), 0, g->res[a] - 1);
        if (d[a] > 0) {
            step[a] = 1;
            tmax[a] = (g->lo[a] + (c[a] + 1) * g->cell[a] - p0[a]) / d[a];
            tdelta[a] = g->cell[a] / d[a];
        } else if (d[a] < 0) {
            step[a] = -1;
            tmax[a] = (g->lo[a] + c[a] * g->cell[a] - p0[a]) / d[a];
            tdelta[a] = -g->cell[a] / d[a];
        } else {
            step[a] = 0;
            tmax[a] = INFINITY;
            tdelta[a] = INFINITY;
        }
    }
    for (;;) {
        int64_t id = cidx(g, c[0], c[1], c[2]);
        for (int64_t k = g->start[id]; k < g->start[id + 1]; ++k)
            if (seg_tri(p0, d, tri + 9 * g->items[k], eps)) return 1;
        int a = 0;
        if (tmax[1] < tmax[a]) a = 1;
        if (tmax[2] < tmax[a]) a = 2;
        if (tmax[a] > t1) return 0;
        c[a] += step[a];
        if (c[a] < 0 || c[a] >= g->res[a]) return 0;
        tmax[a] += tdelta[a];
    }
}

int oracle_occlude(const double *tri, int64_t ntri, const double *p0, const double *p1,
                   int64_t nseg, double eps, int brute, uint8_t *hit) {
    if (ntri <= 0) {
        memset(hit, 0, (size_t)nseg);
        return 0;
    }
    grid_t g;
    memset(&g, 0, sizeof g);
    if (!brute && build_grid(&g, tri, ntri) != 0) return -1;
    for (int64_t s = 0; s < nseg; ++s) {
        double d[3] = {p1[3 * s] - p0[3 * s], p1[3 * s + 1] - p0[3 * s + 1], p1[3 * s + 2] - p0[3 * s + 2]};
        int h = 0;
        if (brute) {
            for (int64_t i = 0; i < ntri && !h; ++i) h = seg_tri(p0 + 3 * s, d, tri + 9 * i, eps);
        } else {
            h = walk(&g, tri, p0 + 3 * s, d, eps);
        }
        hit[s] = (uint8_t)h;
    }
    free(g.start);
    free(g.items);
    return 0;
}
