// HIP kernels of the smooth-surface UTD field evaluation (gfx950).
//
//   k_prep     per body, source-dependent constants (FP64)
//   k_occlude  per (receiver, body) path validity + visibility bits, and per
//              receiver inside / line-of-sight flags  (the U of Eqs. (1)-(2))
//   k_field    per (receiver, frequency chunk) coherent field of Eqs. (1)-(4)
//
// One lane owns one receiver and a chunk of FC frequencies; it walks the
// bodies in order (uniform across the wavefront, so body data comes through
// scalar loads), rebuilds the frequency-independent path constants once per
// path and then runs the Fock-coefficient evaluation for each frequency of the
// chunk, accumulating E in registers.  The Fock tables sit in LDS (FP32) or
// global memory (FP64).
#define FT_QUAL __device__ const
#include "utd_internal.h"
#include "utd_bvh.h"
#include "utd_fock.h"
#include "utd_geom.h"

namespace utd {

// ---------------------------------------------------------------------------
// body constants
// ---------------------------------------------------------------------------
__global__ void k_prep(LaunchParams L, const float* __restrict__ sph, const float* __restrict__ cyl,
                       BodyPrep* __restrict__ out) {
    int nb = L.n_sph + L.n_cyl;
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += gridDim.x * blockDim.x)
        out[b] = body_prep(L.T, sph, L.n_sph, cyl, b);
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

// grid: x over receivers (blockDim 256), y over slot = 0 (receiver flags) or
// 1 + body.  mask[body][rx] gets the path bits, flags[rx] the slot-0 bits.
__global__ void __launch_bounds__(256) k_occlude(LaunchParams L, const float* __restrict__ rx,
                                                 const float* __restrict__ sph, const float* __restrict__ cyl,
                                                 const BodyPrep* __restrict__ prep, const float4* __restrict__ nodes,
                                                 const float4* __restrict__ tris, uint8_t* __restrict__ mask,
                                                 uint8_t* __restrict__ flags) {
    __shared__ int stack[kStackDepth * 256];
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int slot = blockIdx.y;
    if (i >= L.n_rx) return;
    int* stk = stack + threadIdx.x;
    const int stride = 256;
    d3 R = mk(rx[3 * i], rx[3 * i + 1], rx[3 * i + 2]);
    d3 T = mk(L.T[0], L.T[1], L.T[2]);
    int nb = L.n_sph + L.n_cyl;
    if (slot == 0) {
        uint8_t f = 0;
        bool inside = false, tx_inside = false;
        for (int b = 0; b < nb; ++b) {
            inside |= inside_body(prep[b], R);
            tx_inside |= inside_body(prep[b], T);
        }
        if (tx_inside) f |= kFlagTxInside;
        if (inside) f |= kFlagInside;
        if (!inside && !tx_inside && !seg_blocked(T, R, L, sph, cyl, -1, true, nodes, tris, stk, stride))
            f |= kFlagLos;
        flags[i] = f;
        return;
    }
    int b = slot - 1;
    const BodyPrep& P = prep[b];
    RxGeo g = rx_geo(P, R);
    uint8_t m = 0;
    bool bo = L.bodies_occlude != 0;
    for (int ell = 0; ell <= L.l_enc; ++ell) {
        for (int side = 0; side < 2; ++side) {
            int sgn = side == 0 ? 1 : -1;
            PathPts pts;
            bool ok, caus = false;
            if (P.kind == 0)
                ok = sphere_creep<float>(P, g, R, L, sgn, ell, &caus, (PathEval<float>*)nullptr, &pts);
            else
                ok = cyl_creep<float>(P, g, R, L, sgn, ell, (PathEval<float>*)nullptr, &pts);
            if (caus) m |= (uint8_t)(1u << kBitCaustic);
            if (!ok) continue;
            if (seg_blocked(pts.P0, pts.P1, L, sph, cyl, b, bo, nodes, tris, stk, stride)) continue;
            if (seg_blocked(pts.P2, pts.P3, L, sph, cyl, b, bo, nodes, tris, stk, stride)) continue;
            m |= (uint8_t)(1u << (2 * ell + side));
        }
    }
    if (L.lit_branch) {
        PathPts pts;
        bool ok = P.kind == 0 ? sphere_refl<float>(P, g, R, L, nullptr, &pts)
                              : cyl_refl<float>(P, g, R, L, nullptr, &pts);
        if (ok && !seg_blocked(pts.P0, pts.P1, L, sph, cyl, b, bo, nodes, tris, stk, stride) &&
            !seg_blocked(pts.P2, pts.P3, L, sph, cyl, b, bo, nodes, tris, stk, stride))
            m |= (uint8_t)(1u << kBitRefl);
    }
    mask[(int64_t)b * L.n_rx + i] = m;
}

// ---------------------------------------------------------------------------
// field
// ---------------------------------------------------------------------------
template <typename R> struct FreqC {
    double rev_per_m;   // f / c  (revolutions of phase per metre)
    R kf, k13, k16, km16;
};

template <typename R>
__device__ __forceinline__ FreqC<R> freq_consts(double f) {
    FreqC<R> c;
    double k = kTwoPi * f / kC0;
    c.rev_per_m = f / kC0;
    c.kf = (R)k;
    double k13 = cbrt(k);
    c.k13 = (R)k13;
    double k16 = sqrt(k13);
    c.k16 = (R)k16;
    c.km16 = (R)(1.0 / k16);
    return c;
}

template <typename R>
__device__ __forceinline__ void add_path(const PathEval<R>& pe, const Tabs<R>& tb, const FreqC<R>& fc, R* E) {
    R xi = pe.mhat * fc.k13 * pe.phi_e;
    R X = fc.kf * pe.Lh * pe.phi_e * pe.phi_e;
    R q = fc.k16 * pe.qhat;
    cplx<R> Ks, Kh;
    fock_kernel<R>(tb, xi, X, q, pe.refl != 0, &Ks, &Kh);
    cplx<R> ph = phase_rev<R>(fc.rev_per_m * pe.s_tot + pe.rev0);
    R as = pe.a_s * fc.km16, ah = pe.a_h * fc.km16;
    cplx<R> cs = cmul(Ks, ph), ch = cmul(Kh, ph);
    cs.re *= as; cs.im *= as;
    ch.re *= ah; ch.im *= ah;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        E[2 * c] += cs.re * pe.vs[c] + ch.re * pe.vh[c];
        E[2 * c + 1] += cs.im * pe.vs[c] + ch.im * pe.vh[c];
    }
}

template <typename R> struct TableStage;

template <> struct TableStage<float> {
    static constexpr int NREG = (FT_F32_PT_NSEG + FT_F32_DS_NSEG + FT_F32_CL_NSEG) * (FT_F32_PT_DEG + 1) * 4;
    static constexpr int NTF = (FT_F32_FA_NSEG + FT_F32_FH_NSEG) * (FT_F32_PT_DEG + 1) * 2;
    static __device__ __forceinline__ Tabs<float> stage(float* reg, float* tf) {
        const float* a = &ft_f32_pt[0][0][0];
        const float* b = &ft_f32_ds[0][0][0];
        const float* c = &ft_f32_cl[0][0][0];
        constexpr int na = FT_F32_PT_NSEG * (FT_F32_PT_DEG + 1) * 4;
        constexpr int nb = FT_F32_DS_NSEG * (FT_F32_PT_DEG + 1) * 4;
        constexpr int nc = FT_F32_CL_NSEG * (FT_F32_PT_DEG + 1) * 4;
        for (int i = threadIdx.x; i < na; i += blockDim.x) reg[i] = a[i];
        for (int i = threadIdx.x; i < nb; i += blockDim.x) reg[na + i] = b[i];
        for (int i = threadIdx.x; i < nc; i += blockDim.x) reg[na + nb + i] = c[i];
        const float* d = &ft_f32_fa[0][0][0];
        const float* e = &ft_f32_fh[0][0][0];
        constexpr int nd = FT_F32_FA_NSEG * (FT_F32_PT_DEG + 1) * 2;
        constexpr int ne = FT_F32_FH_NSEG * (FT_F32_PT_DEG + 1) * 2;
        for (int i = threadIdx.x; i < nd; i += blockDim.x) tf[i] = d[i];
        for (int i = threadIdx.x; i < ne; i += blockDim.x) tf[nd + i] = e[i];
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
                                               const double* __restrict__ freqs, const BodyPrep* __restrict__ prep,
                                               const uint8_t* __restrict__ mask, uint8_t* __restrict__ flags,
                                               R* __restrict__ E_out) {
    __shared__ R s_reg[TableStage<R>::NREG];
    __shared__ R s_tf[TableStage<R>::NTF];
    Tabs<R> tb = TableStage<R>::stage(s_reg, s_tf);
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L.n_rx) return;
    int f0 = blockIdx.y * FC;
    int nfc = L.n_f - f0 < FC ? L.n_f - f0 : FC;
    R E[FC][6];
#pragma unroll
    for (int j = 0; j < FC; ++j)
#pragma unroll
        for (int c = 0; c < 6; ++c) E[j][c] = (R)0;
    uint8_t fl = flags[i];
    if (!(fl & (kFlagInside | kFlagTxInside))) {
        FreqC<R> fcs[FC];
#pragma unroll
        for (int j = 0; j < FC; ++j) fcs[j] = freq_consts<R>(freqs[f0 + (j < nfc ? j : 0)]);
        d3 Rp = mk(rx[3 * i], rx[3 * i + 1], rx[3 * i + 2]);
        // direct field, Eq. (1): A (p - (p.s)s) e^{-jks}/s
        if ((fl & kFlagLos) && L.lit_branch) {
            d3 v = Rp - mk(L.T[0], L.T[1], L.T[2]);
            double s = norm(v);
            d3 sh = (1.0 / s) * v;
            d3 p = mk(L.p[0], L.p[1], L.p[2]);
            d3 pp = p - dot(p, sh) * sh;
            double A = L.amp / s;
            R e3[3] = {(R)(A * pp.x), (R)(A * pp.y), (R)(A * pp.z)};
#pragma unroll
            for (int j = 0; j < FC; ++j) {
                cplx<R> ph = phase_rev<R>(fcs[j].rev_per_m * s);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    E[j][2 * c] += e3[c] * ph.re;
                    E[j][2 * c + 1] += e3[c] * ph.im;
                }
            }
        }
        int nb = L.n_sph + L.n_cyl;
        uint8_t caus = 0;
        for (int b = 0; b < nb; ++b) {
            uint8_t m = mask[(int64_t)b * L.n_rx + i];
            caus |= m;
            if (!(m & 0x7f)) continue;
            const BodyPrep P = prep[b];
            RxGeo g = rx_geo(P, Rp);
            for (int bit = 0; bit < 7; ++bit) {
                if (!(m & (1u << bit))) continue;
                PathEval<R> pe;
                bool ok;
                if (bit == kBitRefl) {
                    ok = P.kind == 0 ? sphere_refl<R>(P, g, Rp, L, &pe, nullptr) : cyl_refl<R>(P, g, Rp, L, &pe, nullptr);
                } else {
                    int ell = bit >> 1, sgn = (bit & 1) ? -1 : 1;
                    bool cz;
                    ok = P.kind == 0 ? sphere_creep<R>(P, g, Rp, L, sgn, ell, &cz, &pe, nullptr)
                                     : cyl_creep<R>(P, g, Rp, L, sgn, ell, &pe, nullptr);
                }
                if (!ok) continue;
#pragma unroll
                for (int j = 0; j < FC; ++j)
                    if (j < nfc) add_path<R>(pe, tb, fcs[j], E[j]);
            }
        }
        if (blockIdx.y == 0 && (caus & (1u << kBitCaustic))) flags[i] = fl | kFlagCaustic;
    }
#pragma unroll
    for (int j = 0; j < FC; ++j) {
        if (j >= nfc) break;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            int64_t o = ((int64_t)(f0 + j) * 3 + c) * L.n_rx + i;
            E_out[2 * o] = E[j][2 * c];
            E_out[2 * o + 1] = E[j][2 * c + 1];
        }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t pack_tables(hipStream_t s) {
    hipLaunchKernelGGL(k_pack_f64_tables, dim3(1), dim3(256), 0, s);
    return hipGetLastError();
}

hipError_t launch_prep(const LaunchParams& L, const float* sph, const float* cyl, BodyPrep* prep, hipStream_t s) {
    int nb = L.n_sph + L.n_cyl;
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_prep, dim3((nb + 63) / 64), dim3(64), 0, s, L, sph, cyl, prep);
    return hipGetLastError();
}

hipError_t launch_occlude(const LaunchParams& L, const float* rx, const float* sph, const float* cyl,
                          const BodyPrep* prep, const float4* nodes, const float4* tris, uint8_t* mask,
                          uint8_t* flags, hipStream_t s) {
    int nb = L.n_sph + L.n_cyl;
    dim3 grid((unsigned)((L.n_rx + 255) / 256), (unsigned)(nb + 1));
    hipLaunchKernelGGL(k_occlude, grid, dim3(256), 0, s, L, rx, sph, cyl, prep, nodes, tris, mask, flags);
    return hipGetLastError();
}

template <typename R, int FC>
static hipError_t launch_field_fc(const LaunchParams& L, const float* rx, const double* freqs, const BodyPrep* prep,
                                  const uint8_t* mask, uint8_t* flags, R* E, hipStream_t s) {
    dim3 grid((unsigned)((L.n_rx + 255) / 256), (unsigned)((L.n_f + FC - 1) / FC));
    hipLaunchKernelGGL((k_field<R, FC>), grid, dim3(256), 0, s, L, rx, freqs, prep, mask, flags, E);
    return hipGetLastError();
}

hipError_t launch_field(const LaunchParams& L, int precision, int fc, const float* rx, const double* freqs,
                        const BodyPrep* prep, const uint8_t* mask, uint8_t* flags, void* E, hipStream_t s) {
    if (precision == 0) {
        float* e = (float*)E;
        switch (fc) {
            case 1: return launch_field_fc<float, 1>(L, rx, freqs, prep, mask, flags, e, s);
            case 2: return launch_field_fc<float, 2>(L, rx, freqs, prep, mask, flags, e, s);
            case 4: return launch_field_fc<float, 4>(L, rx, freqs, prep, mask, flags, e, s);
            default: return launch_field_fc<float, 8>(L, rx, freqs, prep, mask, flags, e, s);
        }
    }
    double* e = (double*)E;
    switch (fc) {
        case 1: return launch_field_fc<double, 1>(L, rx, freqs, prep, mask, flags, e, s);
        case 2: return launch_field_fc<double, 2>(L, rx, freqs, prep, mask, flags, e, s);
        default: return launch_field_fc<double, 4>(L, rx, freqs, prep, mask, flags, e, s);
    }
}

}  // namespace utd
