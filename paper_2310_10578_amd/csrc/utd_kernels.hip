// HIP kernels of the smooth-surface UTD field evaluation (gfx950).
//
//   k_paths    per (receiver, body) path validity + visibility bits (the U of
//              Eqs. (1)-(2)) and the frequency-independent constants of every
//              valid path; per receiver inside / line-of-sight flags; it also
//              stores the body and frequency constants used later
//   k_field    per (receiver, frequency chunk) coherent field of Eqs. (1)-(4)
//
// In k_field one lane owns one receiver and a chunk of FC frequencies; it
// walks the bodies in order, reads each valid path's record once and runs the
// Fock-coefficient evaluation for every frequency of the chunk, accumulating E
// in registers.  Frequency constants are uniform across the workgroup (scalar
// loads).  The Fock tables sit in LDS (FP32) or global memory (FP64).
#define FT_QUAL __device__ const
#include "utd_internal.h"
#include "utd_bvh.h"
#include "utd_fock.h"
#include "utd_geom.h"

namespace utd {

// ---------------------------------------------------------------------------
// frequency constants
// ---------------------------------------------------------------------------
__device__ __forceinline__ FreqConst freq_const(double f) {
    double k = kTwoPi * f / kC0;
    double k13 = cbrt(k), k16 = sqrt(k13);
    FreqConst c;
    c.rev_per_m = f / kC0;
    c.kd = k; c.k13d = k13; c.k16d = k16; c.km16d = 1.0 / k16; c.skd = sqrt(k); c.ik13d = 1.0 / k13;
    c.kf = (float)k; c.k13f = (float)k13; c.k16f = (float)k16; c.km16f = (float)(1.0 / k16);
    c.skf = (float)sqrt(k); c.ik13f = (float)(1.0 / k13);
    return c;
}

// Receiver (or source) inside the solid body b.
__device__ __forceinline__ bool inside_raw(const LaunchParams& L, const float* sph, const float* cyl, int b, d3 P) {
    if (b < L.n_sph) {
        const float* s = sph + 4 * b;
        double x = P.x - s[0], y = P.y - s[1], z = P.z - s[2];
        return x * x + y * y + z * z <= (double)s[3] * s[3];
    }
    const float* c = cyl + 5 * (b - L.n_sph);
    double x = P.x - c[0], y = P.y - c[1];
    return x * x + y * y <= (double)c[4] * c[4] && P.z >= c[2] && P.z <= (double)c[2] + c[3];
}

// ---------------------------------------------------------------------------
// visibility
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool blocked_by_bodies(d3 P0, d3 P1, const LaunchParams& L, const float* sph,
                                                  const float* cyl, int skip) {
    for (int i = 0; i < L.n_sph; ++i)
        if (i != skip && seg_sphere(P0, P1, sph + 4 * i)) return true;
    for (int i = 0; i < L.n_cyl; ++i)
        if (L.n_sph + i != skip && seg_cylinder(P0, P1, cyl + 5 * i)) return true;
    return false;
}

__device__ __forceinline__ bool seg_blocked(d3 P0, d3 P1, const LaunchParams& L, const float* sph,
                                            const float* cyl, int skip, bool bodies, const float4* nodes,
                                            const float4* tris, int* stack, int stride) {
    if (bodies && blocked_by_bodies(P0, P1, L, sph, cyl, skip)) return true;
    SegRay r = make_ray(P0, P1);
    return bvh_anyhit(nodes, tris, r, stack, stride);
}

// Path records: the frequency-independent constants of one valid path,
// written by the visibility pass and read by the field kernel.  Slot-major
// layout rec[(body * S + slot) * n_rx + rx] keeps both passes coalesced;
// S = 2 (l_enc + 1) bounds the valid paths of a (receiver, body) pair (one
// side of a lit receiver carries the reflection instead of a creeping path).
// Creeping paths fill slots 0, 1, ... in (ell, side) order; the reflection,
// when present, always sits in slot S - 1 (it then leaves at most S - 1
// creeping paths), so the field kernel can treat the two kinds separately.
template <typename R> struct PathRec;
template <> struct PathRec<float> {          // 64 bytes
    double s_tot;
    int16_t nc;                               // caustic quarter turns
    int16_t refl;
    float xh, uh, qhat;                       // see PathEval
    float4 q0;                                // (ixh, sxh, vs0, vs1)
    float4 q1;                                // (vs2, vh0, vh1, vh2)
    float2 pad;
};
template <> struct PathRec<double> {         // 120 bytes
    double s_tot;
    int32_t nc, refl;
    double v[13];
};

__device__ __forceinline__ void pack(const PathEval<float>& p, PathRec<float>* r) {
    PathRec<float> o;
    o.s_tot = p.s_tot;
    o.nc = (int16_t)p.nc;
    o.refl = (int16_t)p.refl;
    o.xh = p.xh; o.uh = p.uh; o.qhat = p.qhat;
    o.q0 = make_float4(p.ixh, p.sxh, p.vs[0], p.vs[1]);
    o.q1 = make_float4(p.vs[2], p.vh[0], p.vh[1], p.vh[2]);
    o.pad = make_float2(0.0f, 0.0f);
    *r = o;
}
__device__ __forceinline__ void unpack(const PathRec<float>& o, PathEval<float>* p) {
    p->s_tot = o.s_tot;
    p->nc = o.nc;
    p->refl = o.refl;
    p->xh = o.xh; p->uh = o.uh; p->qhat = o.qhat;
    p->ixh = o.q0.x; p->sxh = o.q0.y; p->vs[0] = o.q0.z; p->vs[1] = o.q0.w;
    p->vs[2] = o.q1.x; p->vh[0] = o.q1.y; p->vh[1] = o.q1.z; p->vh[2] = o.q1.w;
}
__device__ __forceinline__ void pack(const PathEval<double>& p, PathRec<double>* r) {
    PathRec<double> o;
    o.s_tot = p.s_tot; o.nc = p.nc; o.refl = p.refl;
    double v[13] = {p.xh, p.uh, p.qhat, p.ixh, p.sxh, p.vs[0], p.vs[1], p.vs[2], p.vh[0], p.vh[1], p.vh[2],
                    0.0, 0.0};
    for (int k = 0; k < 13; ++k) o.v[k] = v[k];
    *r = o;
}
__device__ __forceinline__ void unpack(const PathRec<double>& o, PathEval<double>* p) {
    p->s_tot = o.s_tot; p->nc = o.nc; p->refl = o.refl;
    p->xh = o.v[0]; p->uh = o.v[1]; p->qhat = o.v[2]; p->ixh = o.v[3]; p->sxh = o.v[4];
    p->vs[0] = o.v[5]; p->vs[1] = o.v[6]; p->vs[2] = o.v[7];
    p->vh[0] = o.v[8]; p->vh[1] = o.v[9]; p->vh[2] = o.v[10];
}

// Visibility and path constants.  grid: x over receivers (blockDim 256),
// y over slot = 0 (receiver flags) or 1 + body.  mask[body][rx] gets the path
// bits, flags[rx] the slot-0 bits, rec the constants of each valid path in
// set-bit order.
// The body constants of slot b are computed by every block of the slot (a
// few FP64 operations); the x = 0 block also stores them, and the (0, 0)
// block the frequency constants, for the later kernels of the call.
template <typename R>
__device__ __forceinline__ void paths_body(const LaunchParams& L, const float* __restrict__ rx,
                                           const float* __restrict__ sph, const float* __restrict__ cyl,
                                           const double* __restrict__ freqs, BodyPrep* __restrict__ prep,
                                           FreqConst* __restrict__ fcs, const float4* __restrict__ nodes,
                                           const float4* __restrict__ tris, uint8_t* __restrict__ mask,
                                           PathRec<R>* __restrict__ rec, uint8_t* __restrict__ flags, int* stack) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int slot = blockIdx.y;
    if (slot == 0 && blockIdx.x == 0 && freqs)
        for (int f = threadIdx.x; f < L.n_f; f += blockDim.x) fcs[f] = freq_const(freqs[f]);
    if (i >= L.n_rx) return;
    int* stk = stack + threadIdx.x;
    const int stride = 256;
    d3 R3 = mk(rx[3 * i], rx[3 * i + 1], rx[3 * i + 2]);
    d3 T = mk(L.T[0], L.T[1], L.T[2]);
    int nb = L.n_sph + L.n_cyl;
    if (slot == 0) {
        uint8_t f = 0;
        bool inside = false, tx_inside = false;
        for (int b = 0; b < nb; ++b) {
            inside |= inside_raw(L, sph, cyl, b, R3);
            tx_inside |= inside_raw(L, sph, cyl, b, T);
        }
        if (tx_inside) f |= kFlagTxInside;
        if (inside) f |= kFlagInside;
        if (!inside && !tx_inside && !seg_blocked(T, R3, L, sph, cyl, -1, true, nodes, tris, stk, stride))
            f |= kFlagLos;
        flags[i] = f;
        return;
    }
    int b = slot - 1;
    const BodyPrep P = body_prep(L.T, sph, L.n_sph, cyl, b);
    if (blockIdx.x == 0 && threadIdx.x == 0) prep[b] = P;
    RxGeo g = rx_geo(P, R3);
    uint8_t m = 0;
    int nrec = 0;
    const int S = 2 * (L.l_enc + 1);
    bool bo = L.bodies_occlude != 0;
    for (int ell = 0; ell <= L.l_enc; ++ell) {
        for (int side = 0; side < 2; ++side) {
            int sgn = side == 0 ? 1 : -1;
            PathPts pts;
            bool ok, caus = false;
            if (P.kind == 0)
                ok = sphere_creep<R, double>(P, g, R3, T, L, sgn, ell, &caus, (PathEval<R>*)nullptr, &pts);
            else
                ok = cyl_creep<R, double>(P, g, R3, T, L, sgn, ell, (PathEval<R>*)nullptr, &pts);
            if (caus) m |= (uint8_t)(1u << kBitCaustic);
            if (!ok) continue;
            if (seg_blocked(pts.P0, pts.P1, L, sph, cyl, b, bo, nodes, tris, stk, stride)) continue;
            if (seg_blocked(pts.P2, pts.P3, L, sph, cyl, b, bo, nodes, tris, stk, stride)) continue;
            m |= (uint8_t)(1u << (2 * ell + side));
            PathEval<R> pe;
            bool cz;
            if (P.kind == 0)
                sphere_creep<R, double>(P, g, R3, T, L, sgn, ell, &cz, &pe, nullptr);
            else
                cyl_creep<R, double>(P, g, R3, T, L, sgn, ell, &pe, nullptr);
            if (nrec < S) pack(pe, &rec[((int64_t)b * S + nrec) * L.n_rx + i]);
            ++nrec;
        }
    }
    double th = 0.0;
    if (L.lit_branch && refl_angle(P, g, R3, T, &th)) {
        d3 Q, n;
        refl_point<double>(P, g, R3, T, th, &Q, &n);
        if (!seg_blocked(T, Q, L, sph, cyl, b, bo, nodes, tris, stk, stride) &&
            !seg_blocked(Q, R3, L, sph, cyl, b, bo, nodes, tris, stk, stride)) {
            m |= (uint8_t)(1u << kBitRefl);
            PathEval<R> pe;
            refl_eval<R, double>(P, Q, n, R3, T, L, &pe);
            pack(pe, &rec[((int64_t)b * S + (S - 1)) * L.n_rx + i]);
        }
    }
    mask[(int64_t)b * L.n_rx + i] = m;
}

// Two register budgets of the same pass: the default (no spills, two waves
// per SIMD) for grids that do not fill the chip at that occupancy, and three
// waves per SIMD (168 VGPRs, a few spills), which hides more traversal
// latency on large grids (measured -20% on the room workloads).
template <typename R>
__global__ void __launch_bounds__(256) k_paths(LaunchParams L, const float* __restrict__ rx,
                                               const float* __restrict__ sph, const float* __restrict__ cyl,
                                               const double* __restrict__ freqs, BodyPrep* __restrict__ prep,
                                               FreqConst* __restrict__ fcs, const float4* __restrict__ nodes,
                                               const float4* __restrict__ tris, uint8_t* __restrict__ mask,
                                               PathRec<R>* __restrict__ rec, uint8_t* __restrict__ flags) {
    __shared__ int stack[kStackDepth * 256];
    paths_body<R>(L, rx, sph, cyl, freqs, prep, fcs, nodes, tris, mask, rec, flags, stack);
}

template <typename R>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8)))
k_paths_occ3(LaunchParams L, const float* __restrict__ rx, const float* __restrict__ sph,
             const float* __restrict__ cyl, const double* __restrict__ freqs, BodyPrep* __restrict__ prep,
             FreqConst* __restrict__ fcs, const float4* __restrict__ nodes, const float4* __restrict__ tris,
             uint8_t* __restrict__ mask, PathRec<R>* __restrict__ rec, uint8_t* __restrict__ flags) {
    __shared__ int stack[kStackDepth * 256];
    paths_body<R>(L, rx, sph, cyl, freqs, prep, fcs, nodes, tris, mask, rec, flags, stack);
}

// ---------------------------------------------------------------------------
// field
// ---------------------------------------------------------------------------
template <typename R> struct FreqC;
template <> struct FreqC<float> {
    double rev_per_m;
    float kf, k13, k16, km16, sk, ik13;
    __device__ __forceinline__ FreqC(const FreqConst& c)
        : rev_per_m(c.rev_per_m), kf(c.kf), k13(c.k13f), k16(c.k16f), km16(c.km16f), sk(c.skf), ik13(c.ik13f) {}
};
template <> struct FreqC<double> {
    double rev_per_m;
    double kf, k13, k16, km16, sk, ik13;
    __device__ __forceinline__ FreqC(const FreqConst& c)
        : rev_per_m(c.rev_per_m), kf(c.kd), k13(c.k13d), k16(c.k16d), km16(c.km16d), sk(c.skd), ik13(c.ik13d) {}
};

// One path at one frequency: the Fock arguments scale with powers of k
// (xi ~ k^{1/3}, sqrt(X) ~ k^{1/2}, q ~ k^{1/6}), so they are products of the
// path's constants and the frequency's.  MODE picks the Fock specialisation
// (kCreep, kRefl or kAny for mixed wavefronts); callers branch on
// wave-uniform conditions.
template <typename R, int MODE>
__device__ __forceinline__ void add_path(const PathEval<R>& pe, const Tabs<R>& tb, const FreqC<R>& fc, R* E) {
    FockArgs<R> a;
    a.xi = fc.k13 * pe.xh;
    a.u = fc.sk * pe.uh;
    a.q = fc.k16 * pe.qhat;
    a.ixi = fc.ik13 * pe.ixh;
    a.h = (R)0.5 * fc.k16 * pe.sxh;
    cplx<R> Ks, Kh;
    fock_kernel<R, MODE>(tb, a, pe.refl != 0, &Ks, &Kh);
    cplx<R> ph = phase_rev<R>(fc.rev_per_m * pe.s_tot - 0.25 * pe.nc);
    ph.re *= fc.km16;
    ph.im *= fc.km16;
    cplx<R> cs = cmul(Ks, ph), ch = cmul(Kh, ph);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        E[2 * c] = fma(cs.re, pe.vs[c], E[2 * c]);
        E[2 * c] = fma(ch.re, pe.vh[c], E[2 * c]);
        E[2 * c + 1] = fma(cs.im, pe.vs[c], E[2 * c + 1]);
        E[2 * c + 1] = fma(ch.im, pe.vh[c], E[2 * c + 1]);
    }
}

template <typename R> struct TableStage;

template <> struct TableStage<float> {
    using D = TabDims<float>;
    static constexpr int ROWS = D::ROWS, DEG = D::DEG;
    static constexpr int NREG = (D::NPT + D::NDS + D::NCL) * ROWS * 4;
    static constexpr int NTF = (D::NFA + D::NFH) * ROWS * 2;
    // copy [seg][DEG + 1][W] into [seg][ROWS][W] (padding rows never read)
    template <int W>
    static __device__ __forceinline__ void copy(float* dst, const float* src, int nseg) {
        const int n = nseg * (DEG + 1) * W;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            int sg = i / ((DEG + 1) * W), r = i - sg * (DEG + 1) * W;
            dst[sg * ROWS * W + r] = src[i];
        }
    }
    static __device__ __forceinline__ Tabs<float> stage(float* reg, float* tf) {
        copy<4>(reg, &ft_f32_pt[0][0][0], D::NPT);
        copy<4>(reg + D::NPT * ROWS * 4, &ft_f32_ds[0][0][0], D::NDS);
        copy<4>(reg + (D::NPT + D::NDS) * ROWS * 4, &ft_f32_cl[0][0][0], D::NCL);
        copy<2>(tf, &ft_f32_fa[0][0][0], D::NFA);
        copy<2>(tf + D::NFA * ROWS * 2, &ft_f32_fh[0][0][0], D::NFH);
        __syncthreads();
        return Tabs<float>{reg, tf};
    }
};

// FP64 tables stay in global memory (81 KB; L2 resident).  They are laid out
// back to back in one device array built once at library load.
__device__ double g_f64_reg[(FT_F64_PT_NSEG + FT_F64_DS_NSEG + FT_F64_CL_NSEG) * (FT_F64_PT_DEG + 1) * 4];
__device__ double g_f64_tf[(FT_F64_FA_NSEG + FT_F64_FH_NSEG) * (FT_F64_PT_DEG + 1) * 2];

__global__ void k_pack_f64_tables() {
    constexpr int na = FT_F64_PT_NSEG * (FT_F64_PT_DEG + 1) * 4;
    constexpr int nb = FT_F64_DS_NSEG * (FT_F64_PT_DEG + 1) * 4;
    constexpr int nc = FT_F64_CL_NSEG * (FT_F64_PT_DEG + 1) * 4;
    constexpr int nd = FT_F64_FA_NSEG * (FT_F64_PT_DEG + 1) * 2;
    constexpr int ne = FT_F64_FH_NSEG * (FT_F64_PT_DEG + 1) * 2;
    const double* a = &ft_f64_pt[0][0][0];
    const double* b = &ft_f64_ds[0][0][0];
    const double* c = &ft_f64_cl[0][0][0];
    const double* d = &ft_f64_fa[0][0][0];
    const double* e = &ft_f64_fh[0][0][0];
    for (int i = threadIdx.x; i < na; i += blockDim.x) g_f64_reg[i] = a[i];
    for (int i = threadIdx.x; i < nb; i += blockDim.x) g_f64_reg[na + i] = b[i];
    for (int i = threadIdx.x; i < nc; i += blockDim.x) g_f64_reg[na + nb + i] = c[i];
    for (int i = threadIdx.x; i < nd; i += blockDim.x) g_f64_tf[i] = d[i];
    for (int i = threadIdx.x; i < ne; i += blockDim.x) g_f64_tf[nd + i] = e[i];
}

template <> struct TableStage<double> {
    static constexpr int NREG = 1, NTF = 1;
    static __device__ __forceinline__ Tabs<double> stage(double*, double*) { return Tabs<double>{g_f64_reg, g_f64_tf}; }
};

template <typename R, int FC>
__global__ void __launch_bounds__(256) k_field(LaunchParams L, const float* __restrict__ rx,
                                               const FreqConst* __restrict__ fcs, const uint8_t* __restrict__ mask,
                                               const PathRec<R>* __restrict__ rec, uint8_t* __restrict__ flags,
                                               R* __restrict__ E_out) {
    __shared__ R s_reg[TableStage<R>::NREG];
    __shared__ R s_tf[TableStage<R>::NTF];
    Tabs<R> tb = TableStage<R>::stage(s_reg, s_tf);
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L.n_rx) return;
    const int f0 = blockIdx.y * FC;
    const int nfc = L.n_f - f0 < FC ? L.n_f - f0 : FC;
    const int S = 2 * (L.l_enc + 1);
    R E[FC][6];
#pragma unroll
    for (int j = 0; j < FC; ++j)
#pragma unroll
        for (int c = 0; c < 6; ++c) E[j][c] = (R)0;
    uint8_t fl = flags[i];
    if (!(fl & (kFlagInside | kFlagTxInside))) {
        // direct field, Eq. (1): A (p - (p.s)s) e^{-jks}/s
        if ((fl & kFlagLos) && L.lit_branch) {
            d3 v = mk(rx[3 * i] - L.T[0], rx[3 * i + 1] - L.T[1], rx[3 * i + 2] - L.T[2]);
            double sd = norm(v);
            R isd = (R)(1.0 / sd);
            R shx = (R)v.x * isd, shy = (R)v.y * isd, shz = (R)v.z * isd;
            R px = (R)L.p[0], py = (R)L.p[1], pz = (R)L.p[2];
            R pd = px * shx + py * shy + pz * shz;
            R A = (R)L.amp * isd;
            R e3[3] = {A * (px - pd * shx), A * (py - pd * shy), A * (pz - pd * shz)};
#pragma unroll
            for (int j = 0; j < FC; ++j) {
                if (j < nfc) {
                    cplx<R> ph = phase_rev<R>(fcs[f0 + j].rev_per_m * sd);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        E[j][2 * c] += e3[c] * ph.re;
                        E[j][2 * c + 1] += e3[c] * ph.im;
                    }
                }
            }
        }
        int nb = L.n_sph + L.n_cyl;
        uint8_t caus = 0;
        for (int b = 0; b < nb; ++b) {
            uint8_t m = mask[(int64_t)b * L.n_rx + i];
            caus |= m;
            const bool has_refl = (m >> kBitRefl) & 1u;
            int n = __builtin_popcount(m & 0x3fu);
            n = n < (has_refl ? S - 1 : S) ? n : (has_refl ? S - 1 : S);
            for (int k = 0; k < n; ++k) {
                PathEval<R> pe;
                unpack(rec[((int64_t)b * S + k) * L.n_rx + i], &pe);
#pragma unroll
                for (int j = 0; j < FC; ++j) {
                    if (j < nfc) {
                        FreqC<R> fc(fcs[f0 + j]);
                        add_path<R, kCreep>(pe, tb, fc, E[j]);
                    }
                }
            }
            if (__any(has_refl) && has_refl) {
                PathEval<R> pe;
                unpack(rec[((int64_t)b * S + (S - 1)) * L.n_rx + i], &pe);
#pragma unroll
                for (int j = 0; j < FC; ++j) {
                    if (j < nfc) {
                        FreqC<R> fc(fcs[f0 + j]);
                        add_path<R, kRefl>(pe, tb, fc, E[j]);
                    }
                }
            }
        }
        if (blockIdx.y == 0 && (caus & (1u << kBitCaustic))) flags[i] = fl | kFlagCaustic;
    }
#pragma unroll
    for (int j = 0; j < FC; ++j) {
        if (j < nfc) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                int64_t o = ((int64_t)(f0 + j) * 3 + c) * L.n_rx + i;
                E_out[2 * o] = E[j][2 * c];
                E_out[2 * o + 1] = E[j][2 * c + 1];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// path census: per-bit counts of the masks (integer atomics, deterministic)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_census(int64_t n_mask, const uint8_t* __restrict__ mask, int64_t n_rx,
                                                const uint8_t* __restrict__ flags,
                                                unsigned long long* __restrict__ counts) {
    __shared__ unsigned int part[10];
    if (threadIdx.x < 10) part[threadIdx.x] = 0;
    __syncthreads();
    unsigned int loc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_mask; i += (int64_t)gridDim.x * blockDim.x) {
        uint8_t m = mask[i];
#pragma unroll
        for (int b = 0; b < 8; ++b) loc[b] += (m >> b) & 1u;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_rx; i += (int64_t)gridDim.x * blockDim.x) {
        uint8_t f = flags[i];
        loc[8] += (f & kFlagLos) ? 1u : 0u;
        loc[9] += (f & kFlagInside) ? 1u : 0u;
    }
#pragma unroll
    for (int b = 0; b < 10; ++b) atomicAdd(&part[b], loc[b]);
    __syncthreads();
    if (threadIdx.x < 10) atomicAdd(&counts[threadIdx.x], (unsigned long long)part[threadIdx.x]);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t pack_tables(hipStream_t s) {
    hipLaunchKernelGGL(k_pack_f64_tables, dim3(1), dim3(256), 0, s);
    return hipGetLastError();
}

hipError_t launch_census(int64_t n_mask, const uint8_t* mask, int64_t n_rx, const uint8_t* flags,
                         unsigned long long* counts, hipStream_t s) {
    hipLaunchKernelGGL(k_census, dim3(512), dim3(256), 0, s, n_mask, mask, n_rx, flags, counts);
    return hipGetLastError();
}

template <typename R>
static hipError_t launch_paths_t(const LaunchParams& L, const float* rx, const float* sph, const float* cyl,
                                 const double* freqs, BodyPrep* prep, FreqConst* fcs, const float4* nodes,
                                 const float4* tris, uint8_t* mask, void* rec, uint8_t* flags, hipStream_t s) {
    int nb = L.n_sph + L.n_cyl;
    dim3 grid((unsigned)((L.n_rx + 255) / 256), (unsigned)(nb + 1));
    // waves of the grid against what 256 CUs hold at two waves per SIMD
    const int64_t waves = (int64_t)grid.x * grid.y * 4;
    if (waves > 256 * 4 * 2 * 2)
        hipLaunchKernelGGL((k_paths_occ3<R>), grid, dim3(256), 0, s, L, rx, sph, cyl, freqs, prep, fcs, nodes, tris,
                           mask, (PathRec<R>*)rec, flags);
    else
        hipLaunchKernelGGL((k_paths<R>), grid, dim3(256), 0, s, L, rx, sph, cyl, freqs, prep, fcs, nodes, tris,
                           mask, (PathRec<R>*)rec, flags);
    return hipGetLastError();
}

hipError_t launch_paths(const LaunchParams& L, int precision, const float* rx, const float* sph, const float* cyl,
                        const double* freqs, BodyPrep* prep, FreqConst* fcs, const float4* nodes, const float4* tris,
                        uint8_t* mask, void* rec, uint8_t* flags, hipStream_t s) {
    return precision == 0
               ? launch_paths_t<float>(L, rx, sph, cyl, freqs, prep, fcs, nodes, tris, mask, rec, flags, s)
               : launch_paths_t<double>(L, rx, sph, cyl, freqs, prep, fcs, nodes, tris, mask, rec, flags, s);
}

size_t path_record_bytes(int precision) { return precision == 0 ? sizeof(PathRec<float>) : sizeof(PathRec<double>); }

template <typename R, int FC>
static hipError_t launch_field_fc(const LaunchParams& L, const float* rx, const FreqConst* fcs, const uint8_t* mask,
                                  const void* rec, uint8_t* flags, R* E, hipStream_t s) {
    dim3 grid((unsigned)((L.n_rx + 255) / 256), (unsigned)((L.n_f + FC - 1) / FC));
    hipLaunchKernelGGL((k_field<R, FC>), grid, dim3(256), 0, s, L, rx, fcs, mask, (const PathRec<R>*)rec, flags, E);
    return hipGetLastError();
}

hipError_t launch_field(const LaunchParams& L, int precision, int fc, const float* rx, const FreqConst* fcs,
                        const uint8_t* mask, const void* rec, uint8_t* flags, void* E, hipStream_t s) {
    if (precision == 0) {
        float* e = (float*)E;
        switch (fc) {
            case 1: return launch_field_fc<float, 1>(L, rx, fcs, mask, rec, flags, e, s);
            case 2: return launch_field_fc<float, 2>(L, rx, fcs, mask, rec, flags, e, s);
            default: return launch_field_fc<float, 4>(L, rx, fcs, mask, rec, flags, e, s);
        }
    }
    double* e = (double*)E;
    switch (fc) {
        case 1: return launch_field_fc<double, 1>(L, rx, fcs, mask, rec, flags, e, s);
        default: return launch_field_fc<double, 2>(L, rx, fcs, mask, rec, flags, e, s);
    }
}

}  // namespace utd

#include "utd_adjoint.h"
#include "utd_batched.h"
