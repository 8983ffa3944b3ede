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

__device__ __forceinline__ bool box_hit(const SegRay& r, float lx, float ly, float lz, float hx, float hy, float hz) {
    float t0x = (lx - r.ox) * r.ix, t1x = (hx - r.ox) * r.ix;
    float t0y = (ly - r.oy) * r.iy, t1y = (hy - r.oy) * r.iy;
    float t0z = (lz - r.oz) * r.iz, t1z = (hz - r.oz) * r.iz;
    float tmin = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), 0.0f));
    float tmax = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), 1.0f));
    return tmin <= tmax * 1.00000024f;   // conservative by 2 ulp
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

// Any-hit walk of the tree rooted at node `root`.
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
        bool h0 = q3.x >= 0 && box_hit(r, q0.x, q0.y, q0.z, q0.w, q1.x, q1.y);
        bool h1 = q3.z >= 0 && box_hit(r, q1.z, q1.w, q2.x, q2.y, q2.z, q2.w);
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
                stack[stride * sp++] = q3.z;
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

}  // namespace utd
