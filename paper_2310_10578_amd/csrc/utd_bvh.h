// Segment visibility for the Heaviside steps U of Eqs. (1)-(2): any-hit of a
// straight segment against the triangle BVH (FP32, watertight test of Woop,
// Benthin and Wald, JCGT 2013) and against the solid spheres and finite
// vertical cylinders of the scene (closed form, FP64).
#pragma once

#include "utd_device.h"

namespace utd {

constexpr float kSegEps = 1e-6f;   // open parameter interval (eps, 1 - eps)
constexpr int kStackDepth = 24;    // per-lane traversal stack (LDS); the builder caps the depth below

// Node: two child boxes and their references, 64 bytes:
//   q0 = (lo0.x, lo0.y, lo0.z, hi0.x)  q1 = (hi0.y, hi0.z, lo1.x, lo1.y)
//   q2 = (lo1.z, hi1.x, hi1.y, hi1.z)  q3 = (c0, n0, c1, n1) as int bits
// child i: n_i > 0 -> leaf holding triangles [c_i, c_i + n_i);
//          n_i == 0 -> inner node c_i; c_i < 0 -> empty.
// Triangles: three float4 per triangle (v0, v1, v2; w unused).

struct SegRay {
    float ox, oy, oz;
    float dx, dy, dz;          // P1 - P0 (segment parameter 0..1)
    float ix, iy, iz;          // 1/d (finite)
    int kx, ky, kz;            // watertight permutation
    float Sx, Sy, Sz;          // shear
};

__device__ __forceinline__ float comp(float x, float y, float z, int k) { return k == 0 ? x : (k == 1 ? y : z); }

__device__ __forceinline__ SegRay make_ray(d3 P0, d3 P1) {
    SegRay r;
    r.ox = (float)P0.x; r.oy = (float)P0.y; r.oz = (float)P0.z;
    r.dx = (float)(P1.x - P0.x); r.dy = (float)(P1.y - P0.y); r.dz = (float)(P1.z - P0.z);
    const float tiny = 1e-30f;
    r.ix = 1.0f / (fabsf(r.dx) > tiny ? r.dx : copysignf(tiny, r.dx));
    r.iy = 1.0f / (fabsf(r.dy) > tiny ? r.dy : copysignf(tiny, r.dy));
    r.iz = 1.0f / (fabsf(r.dz) > tiny ? r.dz : copysignf(tiny, r.dz));
    float ax = fabsf(r.dx), ay = fabsf(r.dy), az = fabsf(r.dz);
    int kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
    int kx = kz + 1 == 3 ? 0 : kz + 1;
    int ky = kx + 1 == 3 ? 0 : kx + 1;
    if (comp(r.dx, r.dy, r.dz, kz) < 0.0f) { int t = kx; kx = ky; ky = t; }
    r.kx = kx; r.ky = ky; r.kz = kz;
    float dkz = comp(r.dx, r.dy, r.dz, kz);
    r.Sx = comp(r.dx, r.dy, r.dz, kx) / dkz;
    r.Sy = comp(r.dx, r.dy, r.dz, ky) / dkz;
    r.Sz = 1.0f / dkz;
    return r;
}

// Segment parameter at which the segment enters the box, or +inf if it
// misses it (conservative by 2 ulp).
__device__ __forceinline__ float box_entry(const SegRay& r, float lx, float ly, float lz, float hx, float hy,
                                           float hz) {
    float t0x = (lx - r.ox) * r.ix, t1x = (hx - r.ox) * r.ix;
    float t0y = (ly - r.oy) * r.iy, t1y = (hy - r.oy) * r.iy;
    float t0z = (lz - r.oz) * r.iz, t1z = (hz - r.oz) * r.iz;
    float tmin = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), 0.0f));
    float tmax = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), 1.0f));
    return tmin <= tmax * 1.00000024f ? tmin : INFINITY;
}

__device__ __forceinline__ bool box_hit(const SegRay& r, float lx, float ly, float lz, float hx, float hy, float hz) {
    return box_entry(r, lx, ly, lz, hx, hy, hz) != INFINITY;
}

// Watertight ray/triangle test restricted to the open segment.
__device__ __forceinline__ bool tri_hit(const SegRay& r, float4 a, float4 b, float4 c) {
    float Ax = comp(a.x, a.y, a.z, r.kx) - comp(r.ox, r.oy, r.oz, r.kx);
    float Ay = comp(a.x, a.y, a.z, r.ky) - comp(r.ox, r.oy, r.oz, r.ky);
    float Az = comp(a.x, a.y, a.z, r.kz) - comp(r.ox, r.oy, r.oz, r.kz);
    float Bx = comp(b.x, b.y, b.z, r.kx) - comp(r.ox, r.oy, r.oz, r.kx);
    float By = comp(b.x, b.y, b.z, r.ky) - comp(r.ox, r.oy, r.oz, r.ky);
    float Bz = comp(b.x, b.y, b.z, r.kz) - comp(r.ox, r.oy, r.oz, r.kz);
    float Cx = comp(c.x, c.y, c.z, r.kx) - comp(r.ox, r.oy, r.oz, r.kx);
    float Cy = comp(c.x, c.y, c.z, r.ky) - comp(r.ox, r.oy, r.oz, r.ky);
    float Cz = comp(c.x, c.y, c.z, r.kz) - comp(r.ox, r.oy, r.oz, r.kz);
    float ax = Ax - r.Sx * Az, ay = Ay - r.Sy * Az;
    float bx = Bx - r.Sx * Bz, by = By - r.Sy * Bz;
    float cx = Cx - r.Sx * Cz, cy = Cy - r.Sy * Cz;
    float U = cx * by - cy * bx;
    float V = ax * cy - ay * cx;
    float W = bx * ay - by * ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        // edge functions exactly zero: recompute in FP64 (as the method prescribes)
        U = (float)((double)cx * by - (double)cy * bx);
        V = (float)((double)ax * cy - (double)ay * cx);
        W = (float)((double)bx * ay - (double)by * ax);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
    float det = U + V + W;
    if (det == 0.0f) return false;
    float T = U * (r.Sz * Az) + V * (r.Sz * Bz) + W * (r.Sz * Cz);
    float lo = kSegEps * det, hi = (1.0f - kSegEps) * det;
    return det > 0.0f ? (T > lo && T < hi) : (T < lo && T > hi);
}

// Any-hit walk of the tree rooted at node `root`.  Of two inner children
// that the segment enters, the one it enters first is walked first (a
// blocked segment then tends to meet its blocker sooner: 5 % of the batched
// crowd's time); the decision does not depend on the order.
__device__ __forceinline__ bool bvh_anyhit(const float4* __restrict__ nodes, const float4* __restrict__ tris,
                                           const SegRay& r, int* stack, int stride, int root = 0) {
    if (!nodes) return false;
    int sp = 0;
    int node = root;
    for (;;) {
        float4 q0 = nodes[4 * node + 0];
        float4 q1 = nodes[4 * node + 1];
        float4 q2 = nodes[4 * node + 2];
        int4 q3 = *reinterpret_cast<const int4*>(&nodes[4 * node + 3]);
        const float e0 = q3.x >= 0 ? box_entry(r, q0.x, q0.y, q0.z, q0.w, q1.x, q1.y) : INFINITY;
        const float e1 = q3.z >= 0 ? box_entry(r, q1.z, q1.w, q2.x, q2.y, q2.z, q2.w) : INFINITY;
        const bool h0 = e0 != INFINITY, h1 = e1 != INFINITY;
        int next = -1;
        if (h0) {
            if (q3.y > 0) {
                for (int t = q3.x; t < q3.x + q3.y; ++t)
                    if (tri_hit(r, tris[3 * t], tris[3 * t + 1], tris[3 * t + 2])) return true;
            } else {
                next = q3.x;
            }
        }
        if (h1) {
            if (q3.w > 0) {
                for (int t = q3.z; t < q3.z + q3.w; ++t)
                    if (tri_hit(r, tris[3 * t], tris[3 * t + 1], tris[3 * t + 2])) return true;
            } else if (next < 0) {
                next = q3.z;
            } else if (sp < kStackDepth) {
                // the host builder caps the tree depth below kStackDepth, so
                // this bound never drops a subtree; it only guards the LDS
                const bool swap = e1 < e0;
                stack[stride * sp++] = swap ? next : q3.z;
                if (swap) next = q3.z;
            }
        }
        if (next >= 0) {
            node = next;
        } else if (sp > 0) {
            node = stack[stride * --sp];
        } else {
            return false;
        }
    }
}

// Conservative FP32 reject: the closest approach of the segment to the
// point (axis) C is farther than a by more than the rounding error of the
// computation (bounded by tol = 4e-6 (|w|^2 + |d|^2), with w = P0 - C and
// d = P1 - P0), so the exact FP64 test below would also say "not crossed".
// Most bodies are far from most segments; this skips their FP64 solve.
// The segment's FP32 form (origin, direction, |d|^2 and its reciprocal) is
// set up once per segment and shared by all bodies.
struct SegF {
    float ox, oy, oz, dx, dy, dz;
    float dd3, id3;     // |d|^2 and 1/|d|^2 (0 for a point)
    float dd2, id2;     // the same in the xy plane
};
__device__ __forceinline__ SegF make_segf(d3 P0, d3 P1) {
    SegF f;
    f.ox = (float)P0.x; f.oy = (float)P0.y; f.oz = (float)P0.z;
    f.dx = (float)(P1.x - P0.x); f.dy = (float)(P1.y - P0.y); f.dz = (float)(P1.z - P0.z);
    f.dd2 = f.dx * f.dx + f.dy * f.dy;
    f.dd3 = f.dd2 + f.dz * f.dz;
    f.id2 = f.dd2 > 0.0f ? 1.0f / f.dd2 : 0.0f;
    f.id3 = f.dd3 > 0.0f ? 1.0f / f.dd3 : 0.0f;
    return f;
}
__device__ __forceinline__ bool far_from(float wx, float wy, float wz, float dx, float dy, float dz, float dd,
                                         float idd, float a) {
    float wd = wx * dx + wy * dy + wz * dz;
    float ww = wx * wx + wy * wy + wz * wz;
    float t = __builtin_amdgcn_fmed3f(-wd * idd, 0.0f, 1.0f);
    float qx = wx + t * dx, qy = wy + t * dy, qz = wz + t * dz;
    float dist2 = qx * qx + qy * qy + qz * qz;
    return dist2 > a * a + 4e-6f * (ww + dd);
}

// Solid sphere (cx, cy, cz, a) crossed strictly inside the segment.
__device__ __forceinline__ bool seg_sphere(d3 P0, d3 P1, const SegF& f, const float* s) {
    if (far_from(f.ox - s[0], f.oy - s[1], f.oz - s[2], f.dx, f.dy, f.dz, f.dd3, f.id3, s[3])) return false;
    d3 d = P1 - P0;
    d3 w = P0 - mk(s[0], s[1], s[2]);
    double a = s[3];
    double A = dot(d, d), B = dot(d, w), C = dot(w, w) - a * a;
    double disc = B * B - A * C;
    if (!(disc > 0) || !(A > 0)) return false;
    double sq = sqrt(disc);
    double t0 = (-B - sq) / A, t1 = (-B + sq) / A;
    return fmax(t0, (double)kSegEps) < fmin(t1, 1.0 - kSegEps);
}

// Solid finite vertical cylinder (cx, cy, z0, h, a).
__device__ __forceinline__ bool seg_cylinder(d3 P0, d3 P1, const SegF& f, const float* c) {
    if (far_from(f.ox - c[0], f.oy - c[1], 0.0f, f.dx, f.dy, 0.0f, f.dd2, f.id2, c[4])) return false;
    d3 d = P1 - P0;
    double wx = P0.x - c[0], wy = P0.y - c[1];
    double a = c[4];
    double A = d.x * d.x + d.y * d.y;
    double B = d.x * wx + d.y * wy;
    double C = wx * wx + wy * wy - a * a;
    double lo, hi;
    if (A > 0) {
        double disc = B * B - A * C;
        if (!(disc > 0)) return false;
        double sq = sqrt(disc);
        lo = (-B - sq) / A;
        hi = (-B + sq) / A;
    } else {
        if (C > 0) return false;
        lo = -1e300; hi = 1e300;
    }
    double z0 = c[2], z1 = (double)c[2] + (double)c[3];
    if (d.z != 0) {
        double ta = (z0 - P0.z) / d.z, tb = (z1 - P0.z) / d.z;
        lo = fmax(lo, fmin(ta, tb));
        hi = fmin(hi, fmax(ta, tb));
    } else if (P0.z < z0 || P0.z > z1) {
        return false;
    }
    return fmax(lo, (double)kSegEps) < fmin(hi, 1.0 - kSegEps);
}


// Grid of the bodies' footprints in the horizontal plane: 16 x 16 cells over
// the box of the bodies' discs (a sphere's and a cylinder's footprint is the
// disc of its radius about its axis), each cell with the bit mask of the
// bodies whose disc, widened by 2 kGridPad, meets it (at most 64 bodies,
// spheres first).  A segment then runs the exact body test only on the
// bodies of the cells its horizontal projection crosses: the grid's rows,
// the segment's x range within each row widened by kGridPad (the cell
// coordinates are FP32, good to about 1e-5 m here).  A body the segment
// meets has a point of the segment inside its disc, in some crossed cell,
// so the subset holds every body that can block and the decision is that of
// the plain loop over all bodies.
constexpr int kGridN = 16;
constexpr float kGridPad = 1e-3f;
struct BodyGrid {
    float x0, y0, sx, sy;        // origin and cells per metre
    int ok;                      // ok = 0: test every body
    int fflags;                  // batched frames: the frame's uniform receiver flags (k_batch_grid)
    int pad[2];
    unsigned long long m[kGridN * kGridN];
};

__device__ __forceinline__ void body_disc(const float* sph, int n_sph, const float* cyl, int j, float* x, float* y,
                                          float* r) {
    if (j < n_sph) {
        const float* q = sph + 4 * j;
        *x = q[0]; *y = q[1]; *r = q[3];
    } else {
        const float* q = cyl + 5 * (j - n_sph);
        *x = q[0]; *y = q[1]; *r = q[4];
    }
}

// The grid of nb = n_sph + n_cyl bodies, built by one block of kGridN^2
// threads (thread = cell); s_box: 4 floats of LDS.  Contains barriers: all
// threads of the block call it with the same arguments.
__device__ __forceinline__ void grid_build_block(BodyGrid* G, const float* sph, int n_sph, const float* cyl,
                                                 int64_t n_cyl, float* s_box) {
    const int t = threadIdx.x;
    const int64_t nb = n_sph + n_cyl;
    if (nb > 64 || nb <= 0) {
        if (t == 0) G->ok = 0;
        return;
    }
    if (t == 0) {
        float x0 = INFINITY, y0 = INFINITY, x1 = -INFINITY, y1 = -INFINITY;
        for (int j = 0; j < (int)nb; ++j) {
            float x, y, r;
            body_disc(sph, n_sph, cyl, j, &x, &y, &r);
            x0 = fminf(x0, x - r); x1 = fmaxf(x1, x + r);
            y0 = fminf(y0, y - r); y1 = fmaxf(y1, y + r);
        }
        // non-finite bodies (flagged elsewhere) keep the plain loop
        const bool fin = isfinite(x0) && isfinite(x1) && isfinite(y0) && isfinite(y1);
        x0 -= kGridPad; y0 -= kGridPad; x1 += kGridPad; y1 += kGridPad;
        s_box[0] = x0; s_box[1] = y0;
        s_box[2] = fin ? (float)kGridN / fmaxf(x1 - x0, 1e-6f) : 0.0f;
        s_box[3] = fin ? (float)kGridN / fmaxf(y1 - y0, 1e-6f) : 0.0f;
        G->x0 = x0; G->y0 = y0; G->sx = s_box[2]; G->sy = s_box[3];
        G->ok = fin ? 1 : 0;
    }
    __syncthreads();
    const int ix = t % kGridN, iy = t / kGridN;
    const float cx0 = s_box[0] + ix / s_box[2], cx1 = s_box[0] + (ix + 1) / s_box[2];
    const float cy0 = s_box[1] + iy / s_box[3], cy1 = s_box[1] + (iy + 1) / s_box[3];
    unsigned long long m = 0ull;
    if (s_box[2] > 0.0f)
        for (int j = 0; j < (int)nb; ++j) {
            float x, y, r;
            body_disc(sph, n_sph, cyl, j, &x, &y, &r);
            const float qx = fminf(fmaxf(x, cx0), cx1), qy = fminf(fmaxf(y, cy0), cy1);
            const float ex = x - qx, ey = y - qy, rr = r + 2.0f * kGridPad;
            if (ex * ex + ey * ey <= rr * rr) m |= 1ull << j;
        }
    G->m[t] = m;
    __syncthreads();
}

// Mask of the bodies a segment P0-P1 may meet.
__device__ __forceinline__ unsigned long long grid_candidates(const BodyGrid* __restrict__ G, int nb, d3 P0, d3 P1) {
    const unsigned long long all = nb >= 64 ? ~0ull : ((1ull << nb) - 1ull);
    if (!G->ok) return all;
    const float x0 = G->x0, y0 = G->y0, sx = G->sx, sy = G->sy;
    const float ax = ((float)P0.x - x0) * sx, ay = ((float)P0.y - y0) * sy;
    const float bx = ((float)P1.x - x0) * sx, by = ((float)P1.y - y0) * sy;
    const float px = kGridPad * sx, py = kGridPad * sy;
    const float ylo = fminf(ay, by) - py, yhi = fmaxf(ay, by) + py;
    const int r0 = (int)fmaxf(floorf(ylo), 0.0f), r1 = (int)fminf(floorf(yhi), (float)(kGridN - 1));
    unsigned long long m = 0ull;
    const float dyb = by - ay;
    for (int r = r0; r <= r1; ++r) {
        // the segment's x range within the row's band [r, r + 1] (widened)
        float t0 = 0.0f, t1 = 1.0f;
        if (fabsf(dyb) > 1e-12f) {
            float ta = ((float)r - py - ay) / dyb, tb = ((float)(r + 1) + py - ay) / dyb;
            if (ta > tb) { const float x = ta; ta = tb; tb = x; }
            t0 = fmaxf(t0, ta);
            t1 = fminf(t1, tb);
        }
        if (t0 > t1) continue;
        const float xa = ax + t0 * (bx - ax), xb = ax + t1 * (bx - ax);
        const int c0 = (int)fmaxf(floorf(fminf(xa, xb) - px), 0.0f);
        const int c1 = (int)fminf(floorf(fmaxf(xa, xb) + px), (float)(kGridN - 1));
        for (int c = c0; c <= c1; ++c) m |= G->m[r * kGridN + c];
    }
    return m;
}

// Any body except `skip` crossed strictly inside the segment, through the
// grid when there is one (G may be NULL) and it holds the bodies.
__device__ __forceinline__ bool blocked_by_grid(d3 P0, d3 P1, const float* sph, int n_sph, const float* cyl,
                                                int n_cyl, int skip, const BodyGrid* G) {
    const int nb = n_sph + n_cyl;
    const SegF f = make_segf(P0, P1);
    if (!G || nb > 64) {
        for (int i = 0; i < nb; ++i) {
            if (i == skip) continue;
            if (i < n_sph ? seg_sphere(P0, P1, f, sph + 4 * i) : seg_cylinder(P0, P1, f, cyl + 5 * (i - n_sph)))
                return true;
        }
        return false;
    }
    unsigned long long m = grid_candidates(G, nb, P0, P1);
    if (skip >= 0 && skip < 64) m &= ~(1ull << skip);
    while (m) {
        const int i = __builtin_ctzll(m);
        m &= m - 1ull;
        if (i < n_sph ? seg_sphere(P0, P1, f, sph + 4 * i) : seg_cylinder(P0, P1, f, cyl + 5 * (i - n_sph)))
            return true;
    }
    return false;
}

}  // namespace utd
