// Adjoint of the field evaluation: gradients of a real loss
// L = Re sum_{f,c,n} conj(g_{f,c,n}) E_{f,c,n} with respect to the source
// position and the body parameters, with the path classification and the
// visibility of the forward evaluation held fixed.  Included by
// utd_kernels.hip after the forward kernels (it reuses their path records,
// table staging and frequency constants).
//
// Per valid path (one lane each, over a compacted list of the paths):
//   1. record adjoint (reverse mode over the frequency loop): lambda_r =
//      dL/dr for every frequency-independent record scalar r (path length,
//      Fock constants xh / uh / qhat, amplitude-weighted polarisation
//      vectors), summed over all frequencies.  The partial derivatives of the Fock
//      coefficients come from the table polynomials evaluated on dual numbers
//      (three directions: xh, uh, qhat).
//   2. geometry tangents (forward mode): the path geometry re-evaluated on
//      dual numbers once per parameter (3 source coordinates, then the
//      body's centre and radius) gives dr/dtheta; dL/dtheta += sum_r lambda_r dr/dtheta.
// The reflection point enters through one Newton step of its stationarity
// condition taken on duals (implicit differentiation).  The direct ray's
// gradient (source only) uses the same two steps.
//
// Reduction: every path writes its 7 FP64 contributions (3 source + up to 4
// body); the paths of a body form one contiguous segment of the list, summed
// by one block in a fixed strided order and a fixed tree; the direct ray's
// source gradient is reduced per block of receivers the same way.  The result
// does not depend on scheduling.
#pragma once

namespace utd {

constexpr int kAdjComp = 8;   // per-block record: 3 source + 4 body + pad

template <typename R> struct RecAdj {
    double s;                  // path length (the phase term dominates)
    R xh, uh, qhat;
    R vs[3], vh[3];
};

// Step 1: lambda for one path from the frequencies' gradients.
template <typename R>
__device__ __forceinline__ void record_adjoint(const PathEval<R>& pe, const Tabs<R>& tb,
                                               const FreqConst* __restrict__ fcs, int n_f,
                                               const R* __restrict__ gE, int64_t n_rx, int64_t i, RecAdj<R>* out) {
    using D = Dual<R>;
    RecAdj<R> l;
    l.s = 0.0;
    l.xh = l.uh = l.qhat = (R)0;
#pragma unroll
    for (int c = 0; c < 3; ++c) l.vs[c] = l.vh[c] = (R)0;
    const bool refl = pe.refl != 0;
    for (int f = 0; f < n_f; ++f) {
        if (!fcs[f].ok) continue;       // an invalid frequency has a zero field
        FreqC<R> fc(fcs[f]);
        cplx<R> g[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            int64_t o = ((int64_t)f * 3 + c) * n_rx + i;
            g[c] = cplx<R>{gE[2 * o], gE[2 * o + 1]};
        }
        // Fock arguments and their derivatives along xh (xi, 1/xi and
        // sqrt(-xi)/2 move together), uh and qhat
        R xi = fc.k13 * pe.xh, u = fc.sk * pe.uh, q = fc.k16 * pe.qhat;
        R ixi = fc.ik13 * pe.ixh, h = (R)0.5 * fc.k16 * pe.sxh;
        R dixi = -fc.ik13 * pe.ixh * pe.ixh;
        R dh = pe.sxh > (R)0 ? (R)-0.25 * fc.k16 / pe.sxh : (R)0;
        cplx<R> Ks, Kh, dKs[3], dKh[3];
#pragma unroll
        for (int dir = 0; dir < 3; ++dir) {
            FockArgs<D> a;
            a.xi = D(xi, dir == 0 ? fc.k13 : (R)0);
            a.u = D(u, dir == 1 ? fc.sk : (R)0);
            a.iu = RT<D>::rcp(u > (R)0 ? a.u : D((R)1));
            a.ixi = D(ixi, dir == 0 ? dixi : (R)0);
            a.h = D(h, dir == 0 ? dh : (R)0);
            a.qc = D(q, dir == 2 ? fc.k16 : (R)0) * D((R)-kC2E4);
            a.xc = a.ixi * D((R)kC2E4);
            cplx<D> ks, kh;
            fock_kernel<D, kAny>(tb, a, refl, &ks, &kh);
            if (dir == 0) {
                Ks = cplx<R>{ks.re.v, ks.im.v};
                Kh = cplx<R>{kh.re.v, kh.im.v};
            }
            dKs[dir] = cplx<R>{ks.re.d, ks.im.d};
            dKh[dir] = cplx<R>{kh.re.d, kh.im.d};
        }
        cplx<R> ph = phase_rev<R>(fc.rev_per_m * pe.s_tot - 0.25 * pe.nc);
        cplx<R> P{ph.re * fc.km16, ph.im * fc.km16};
        // gs = sum_c conj(g_c) vs_c, gh = sum_c conj(g_c) vh_c
        cplx<R> gs{(R)0, (R)0}, gh{(R)0, (R)0};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            gs.re += g[c].re * pe.vs[c]; gs.im -= g[c].im * pe.vs[c];
            gh.re += g[c].re * pe.vh[c]; gh.im -= g[c].im * pe.vh[c];
        }
        cplx<R> Zs = cmul(P, gs), Zh = cmul(P, gh);
        // L_f = Re(K_s Zs + K_h Zh)
        cplx<R> KZs = cmul(Ks, Zs), KZh = cmul(Kh, Zh);
        l.s += kTwoPi * fc.rev_per_m * (double)(KZs.im + KZh.im);
        R dx[3];
#pragma unroll
        for (int dir = 0; dir < 3; ++dir)
            dx[dir] = (dKs[dir].re * Zs.re - dKs[dir].im * Zs.im) + (dKh[dir].re * Zh.re - dKh[dir].im * Zh.im);
        l.xh += dx[0];
        l.uh += dx[1];
        l.qhat += dx[2];
        cplx<R> Ws = cmul(P, Ks), Wh = cmul(P, Kh);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            l.vs[c] += Ws.re * g[c].re + Ws.im * g[c].im;
            l.vh[c] += Wh.re * g[c].re + Wh.im * g[c].im;
        }
    }
    *out = l;
}

// Step 2: sum_r lambda_r dr/dtheta for one tangent.
template <typename R, typename RD, typename GD>
__device__ __forceinline__ double contract(const RecAdj<R>& l, const PathEvalT<RD, GD>& p) {
    R r = l.xh * p.xh.d + l.uh * p.uh.d + l.qhat * p.qhat.d;
#pragma unroll
    for (int c = 0; c < 3; ++c) r += l.vs[c] * p.vs[c].d + l.vh[c] * p.vh[c].d;
    return l.s * p.s_tot.d + (double)r;
}

// Direct ray T -> R: E_c = (amp / s) (p - (p.s) s)_c e^{-j 2 pi (f/c) s}.
template <typename R>
__device__ __forceinline__ void los_adjoint(const LaunchParams& L, d3 R3, const FreqConst* __restrict__ fcs,
                                            const R* __restrict__ gE, int64_t i, double acc[kAdjComp]) {
    using GD = Dual<double>;
    using RD = Dual<R>;
    d3 v0 = mk(R3.x - L.T[0], R3.y - L.T[1], R3.z - L.T[2]);
    double sd0 = norm(v0);
    // amplitude vector in R (as the forward kernel)
    R isd = (R)(1.0 / sd0);
    R shx = (R)v0.x * isd, shy = (R)v0.y * isd, shz = (R)v0.z * isd;
    R px = (R)L.p[0], py = (R)L.p[1], pz = (R)L.p[2];
    R pd = px * shx + py * shy + pz * shz;
    R A = (R)L.amp * isd;
    R e3[3] = {A * (px - pd * shx), A * (py - pd * shy), A * (pz - pd * shz)};
    // lambda of the path length (phase) and of the amplitude vector
    double lsd = 0.0;
    R le[3] = {(R)0, (R)0, (R)0};
    for (int f = 0; f < L.n_f; ++f) {
        if (!fcs[f].ok) continue;
        double rev = fcs[f].rev_per_m;
        cplx<R> ph = phase_rev<R>(rev * sd0);
        R im = (R)0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            int64_t o = ((int64_t)f * 3 + c) * L.n_rx + i;
            R gr = gE[2 * o], gi = gE[2 * o + 1];
            le[c] += gr * ph.re + gi * ph.im;
            im += e3[c] * (gr * ph.im - gi * ph.re);
        }
        lsd += kTwoPi * rev * (double)im;
    }
#pragma unroll 1
    for (int dir = 0; dir < 3; ++dir) {
        V3<GD> v{GD(R3.x - L.T[0], dir == 0 ? -1.0 : 0.0), GD(R3.y - L.T[1], dir == 1 ? -1.0 : 0.0),
                 GD(R3.z - L.T[2], dir == 2 ? -1.0 : 0.0)};
        GD sd = gnorm(v);
        RD is = (RD)(GD(1.0) / sd);
        RD sx = (RD)v.x * is, sy = (RD)v.y * is, sz = (RD)v.z * is;
        RD pdd = px * sx + py * sy + pz * sz;
        RD Ad = (RD)L.amp * is;
        RD ex = Ad * (px - pdd * sx), ey = Ad * (py - pdd * sy), ez = Ad * (pz - pdd * sz);
        acc[dir] += lsd * sd.d + (double)(le[0] * ex.d + le[1] * ey.d + le[2] * ez.d);
    }
}

// ---------------------------------------------------------------------------
// Work list.  Valid paths are sparse over (receiver, body) pairs (a few per
// cent in a furnished room), so the per-path work runs over a compacted list
// instead of one lane per pair: a scan of the per-pair record counts in
// body-major order e = body * n_rx + rx gives every path an entry
// (rx | body << 32 | bit << 48) and every body a contiguous segment of the
// list; per-entry contributions are summed per segment in a fixed order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int pair_records(uint8_t m, uint8_t fl, int S) {
    if (fl & kFlagDead) return 0;
    return __builtin_popcount(m & ((1u << S) - 1u)) + ((m >> kBitRefl) & 1u);
}

constexpr int kScanBlock = 1024;

// Per-block exclusive scan of the record counts: loc[e] (offset inside the
// block) and bsum[block].
__global__ void __launch_bounds__(kScanBlock) k_adj_count(LaunchParams L, const uint8_t* __restrict__ mask,
                                                          const uint8_t* __restrict__ flags, int64_t n_pairs,
                                                          uint16_t* __restrict__ loc, uint32_t* __restrict__ bsum) {
    __shared__ uint32_t sc[kScanBlock];
    const int64_t e = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
    const int S = 2 * (L.l_enc + 1);
    uint32_t c = 0;
    if (e < n_pairs) {
        const int64_t i = e % L.n_rx;
        c = (uint32_t)pair_records(mask[e], flags[i], S);
    }
    sc[threadIdx.x] = c;
    __syncthreads();
    for (int w = 1; w < kScanBlock; w <<= 1) {
        uint32_t v = threadIdx.x >= (unsigned)w ? sc[threadIdx.x - w] : 0u;
        __syncthreads();
        sc[threadIdx.x] += v;
        __syncthreads();
    }
    if (e < n_pairs) loc[e] = (uint16_t)(sc[threadIdx.x] - c);
    if (threadIdx.x == kScanBlock - 1) bsum[blockIdx.x] = sc[threadIdx.x];
}

// One block: exclusive scan of the block sums (boff[nblk] = total entries).
__global__ void __launch_bounds__(kScanBlock) k_adj_scan_top(const uint32_t* __restrict__ bsum, int64_t nblk,
                                                             int64_t* __restrict__ boff) {
    __shared__ int64_t sc[kScanBlock];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nblk; base += kScanBlock) {
        const int64_t j = base + threadIdx.x;
        const int64_t c = j < nblk ? (int64_t)bsum[j] : 0;
        sc[threadIdx.x] = c;
        __syncthreads();
        for (int w = 1; w < kScanBlock; w <<= 1) {
            int64_t v = threadIdx.x >= (unsigned)w ? sc[threadIdx.x - w] : 0;
            __syncthreads();
            sc[threadIdx.x] += v;
            __syncthreads();
        }
        if (j < nblk) boff[j] = carry + sc[threadIdx.x] - c;
        __syncthreads();
        if (threadIdx.x == kScanBlock - 1) carry += sc[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0) boff[nblk] = carry;
}

// Entries of every path and the first entry of every body's segment.
__global__ void __launch_bounds__(kScanBlock) k_adj_emit(LaunchParams L, const uint8_t* __restrict__ mask,
                                                         const uint8_t* __restrict__ flags, int64_t n_pairs,
                                                         const uint16_t* __restrict__ loc,
                                                         const int64_t* __restrict__ boff, uint64_t* __restrict__ ent,
                                                         int64_t* __restrict__ seg) {
    const int64_t e = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
    if (e >= n_pairs) return;
    const int S = 2 * (L.l_enc + 1);
    const int64_t i = e % L.n_rx, b = e / L.n_rx;
    const int64_t base = boff[blockIdx.x] + loc[e];
    if (i == 0) seg[b] = base;
    if (e == 0) seg[n_pairs / L.n_rx] = boff[(n_pairs + kScanBlock - 1) / kScanBlock];   // end of the last segment
    const uint8_t m = mask[e];
    const int n = pair_records(m, flags[i], S);
    if (n == 0) return;
    int k = 0;
    for (int bit = 0; bit < S; ++bit)
        if ((m >> bit) & 1u) ent[base + k++] = (uint64_t)i | ((uint64_t)b << 32) | ((uint64_t)bit << 48);
    if ((m >> kBitRefl) & 1u) ent[base + k] = (uint64_t)i | ((uint64_t)b << 32) | ((uint64_t)kBitRefl << 48);
}

// One path per lane (grid-stride over the entries): record adjoint over all
// frequencies, then the dual-number geometry per parameter; writes the 7
// contributions (3 source + up to 4 body) of the path.
template <typename R>
__global__ void __launch_bounds__(256) k_adj_paths(LaunchParams L, const float* __restrict__ rx,
                                                   const float* __restrict__ sph, const float* __restrict__ cyl,
                                                   const BodyPrep* __restrict__ prep,
                                                   const FreqConst* __restrict__ fcs, const uint8_t* __restrict__ mask,
                                                   const PathRec<R>* __restrict__ rec, const R* __restrict__ gE,
                                                   const uint64_t* __restrict__ ent, const int64_t* __restrict__ ntot,
                                                   double* __restrict__ contrib) {
    using GD = Dual<double>;
    using RD = Dual<R>;
    __shared__ __attribute__((aligned(16))) R s_reg[TableStage<R>::NREG];
    __shared__ __attribute__((aligned(16))) R s_tf[TableStage<R>::NTF];
    Tabs<R> tb = TableStage<R>::template stage<256>(s_reg, s_tf);
    const int64_t total = *ntot;
    const d3 T0 = mk(L.T[0], L.T[1], L.T[2]);
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t en = ent[q];
        const int64_t i = (int64_t)(en & 0xffffffffu);
        const int b = (int)((en >> 32) & 0xffffu);
        const int bit = (int)(en >> 48);
        PathEval<R> pe;
        unpack(rec[((int64_t)b * rec_slots(L) + rec_slot(L, bit)) * L.n_rx + i], &pe);
        RecAdj<R> lam;
        record_adjoint<R>(pe, tb, fcs, L.n_f, gE, L.n_rx, i, &lam);
        const d3 R3 = mk(rx[3 * i], rx[3 * i + 1], rx[3 * i + 2]);
        const bool is_sph = b < L.n_sph;
        double bp[4];
        double z0 = 0.0, hh = 0.0;
        if (is_sph) {
            const float* sp = sph + 4 * b;
            bp[0] = sp[0]; bp[1] = sp[1]; bp[2] = sp[2]; bp[3] = sp[3];
        } else {
            const float* c = cyl + 5 * (b - L.n_sph);
            bp[0] = c[0]; bp[1] = c[1]; bp[2] = c[4]; bp[3] = 0.0;
            z0 = c[2]; hh = c[3];
        }
        const int ndir = is_sph ? 7 : 6;
        const bool refl = bit == kBitRefl;
        const int ell = bit >> 1, sgn = (bit & 1) ? -1 : 1;
        double th = 0.0;
        bool ok0 = true;
        if (refl) {
            const BodyPrep P0 = prep[b];
            RxGeo g0 = rx_geo<double>(P0, R3);
            ok0 = refl_angle(P0, g0, R3, T0, &th);
        }
        V3<GD> Rg{GD(R3.x), GD(R3.y), GD(R3.z)};
        double out[7] = {0, 0, 0, 0, 0, 0, 0};
#pragma unroll 1
        for (int dir = 0; dir < ndir && ok0; ++dir) {
            V3<GD> T{GD(T0.x, dir == 0 ? 1.0 : 0.0), GD(T0.y, dir == 1 ? 1.0 : 0.0), GD(T0.z, dir == 2 ? 1.0 : 0.0)};
            GD p0(bp[0], dir == 3 ? 1.0 : 0.0), p1(bp[1], dir == 4 ? 1.0 : 0.0), p2(bp[2], dir == 5 ? 1.0 : 0.0);
            BodyPrepT<GD> P = is_sph ? prep_sphere<GD>(T, V3<GD>{p0, p1, p2}, GD(bp[3], dir == 6 ? 1.0 : 0.0))
                                     : prep_cylinder<GD>(T, p0, p1, z0, hh, p2);
            RxGeoT<GD> g = rx_geo<GD>(P, Rg);
            PathEvalT<RD, GD> pd;
            bool ok = true;
            if (refl) {
                GD thd = refl_angle_g<GD>(P, g, Rg, T, th);
                V3<GD> Q, n;
                refl_point<GD>(P, g, Rg, T, thd, &Q, &n);
                refl_eval<RD, GD>(P, Q, n, Rg, T, L, &pd);
            } else if (is_sph) {
                bool cz;
                ok = sphere_creep<RD, GD>(P, g, Rg, T, L, sgn, ell, &cz, &pd, nullptr);
            } else {
                ok = cyl_creep<RD, GD>(P, g, Rg, T, L, sgn, ell, &pd, nullptr);
            }
            if (ok) out[dir] = contract(lam, pd);
        }
        // cylinders: parameters (cx, cy, a) go to components 3, 4, 5
#pragma unroll
        for (int d = 0; d < 7; ++d) contrib[q * 8 + d] = out[d];
    }
}

// Direct ray (source gradient only): one lane per receiver, block partials.
template <typename R>
__global__ void __launch_bounds__(256) k_adj_los(LaunchParams L, const float* __restrict__ rx,
                                                 const FreqConst* __restrict__ fcs,
                                                 const uint8_t* __restrict__ flags, const R* __restrict__ gE,
                                                 double* __restrict__ part) {
    __shared__ double s_red[4][4];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc[kAdjComp];
#pragma unroll
    for (int d = 0; d < kAdjComp; ++d) acc[d] = 0.0;
    if (i < L.n_rx) {
        uint8_t fl = flags[i];
        if (!(fl & kFlagDead) && (fl & kFlagLos) && L.lit_branch)
            los_adjoint<R>(L, mk(rx[3 * i], rx[3 * i + 1], rx[3 * i + 2]), fcs, gE, i, acc);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double v = acc[d];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) s_red[wid][d] = v;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        int d = threadIdx.x;
        part[(int64_t)blockIdx.x * 4 + d] = (s_red[0][d] + s_red[1][d]) + (s_red[2][d] + s_red[3][d]);
    }
}

// Block per body (segment sums of the path contributions) plus one block for
// the direct-ray partials; fixed strided order and a fixed tree.
template <typename R>
__global__ void __launch_bounds__(256) k_adj_reduce(const double* __restrict__ contrib, const int64_t* __restrict__ seg,
                                                    const double* __restrict__ los_part, int64_t n_los_blk, int nb,
                                                    int has_paths, int n_sph, R* __restrict__ d_sph,
                                                    R* __restrict__ d_cyl, double* __restrict__ txpart) {
    __shared__ double red[256];
    const int slot = blockIdx.x;            // body, or nb for the direct ray
    const bool los = slot == nb;
    const int64_t lo = los ? 0 : (has_paths ? seg[slot] : 0);
    const int64_t hi = los ? n_los_blk : (has_paths ? seg[slot + 1] : 0);
    const int nd = los ? 3 : 7;
    for (int d = 0; d < nd; ++d) {
        double s = 0.0;
        for (int64_t j = lo + threadIdx.x; j < hi; j += 256) s += los ? los_part[j * 4 + d] : contrib[j * 8 + d];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            double t = red[0];
            if (d < 3) {
                txpart[slot * 3 + d] = t;
            } else {
                if (slot < n_sph) d_sph[slot * 4 + (d - 3)] = (R)t;
                else if (d < 6) d_cyl[(slot - n_sph) * 3 + (d - 3)] = (R)t;
            }
        }
        __syncthreads();
    }
}

template <typename R>
__global__ void k_adjoint_tx(const double* __restrict__ txpart, int nslot, R* __restrict__ d_tx) {
    int d = threadIdx.x;
    if (d < 3) {
        double s = 0.0;
        for (int k = 0; k < nslot; ++k) s += txpart[k * 3 + d];
        d_tx[d] = (R)s;
    }
}

// Scratch of the adjoint beyond the forward workspace, in bytes.
size_t adjoint_scratch_bytes(const LaunchParams& L) {
    const int64_t nb = L.n_sph + L.n_cyl;
    const int64_t n_pairs = nb * L.n_rx;
    const int64_t nblk = (n_pairs + kScanBlock - 1) / kScanBlock;
    const int64_t max_ent = n_pairs * (2 * (L.l_enc + 1) + 1);
    const int64_t nlos = (L.n_rx + 255) / 256;
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    return up(sizeof(uint16_t) * n_pairs) + up(sizeof(uint32_t) * nblk) + up(sizeof(int64_t) * (nblk + 1)) +
           up(sizeof(int64_t) * (nb + 1)) + up(sizeof(uint64_t) * max_ent) + up(sizeof(double) * 8 * max_ent) +
           up(sizeof(double) * 4 * nlos) + up(sizeof(double) * 3 * (nb + 1)) + 256;
}

template <typename R>
static hipError_t launch_adjoint_t(const LaunchParams& L, const float* rx, const float* sph, const float* cyl,
                                   const BodyPrep* prep, const FreqConst* fcs, const uint8_t* mask, const void* rec,
                                   const uint8_t* flags, const void* gE, char* scratch, void* d_sph, void* d_cyl,
                                   void* d_tx, hipStream_t s) {
    const int nb = L.n_sph + L.n_cyl;
    const int64_t n_pairs = (int64_t)nb * L.n_rx;
    const int64_t nblk = (n_pairs + kScanBlock - 1) / kScanBlock;
    const int64_t max_ent = n_pairs * (2 * (L.l_enc + 1) + 1);
    const int64_t nlos = (L.n_rx + 255) / 256;
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    char* p = scratch;
    uint16_t* loc = (uint16_t*)p; p += up(sizeof(uint16_t) * n_pairs);
    uint32_t* bsum = (uint32_t*)p; p += up(sizeof(uint32_t) * nblk);
    int64_t* boff = (int64_t*)p; p += up(sizeof(int64_t) * (nblk + 1));
    int64_t* seg = (int64_t*)p; p += up(sizeof(int64_t) * (nb + 1));
    uint64_t* ent = (uint64_t*)p; p += up(sizeof(uint64_t) * max_ent);
    double* contrib = (double*)p; p += up(sizeof(double) * 8 * max_ent);
    double* los_part = (double*)p; p += up(sizeof(double) * 4 * nlos);
    double* txpart = (double*)p;
    hipError_t e;
    if (n_pairs > 0) {
        hipLaunchKernelGGL(k_adj_count, dim3((unsigned)nblk), dim3(kScanBlock), 0, s, L, mask, flags, n_pairs, loc,
                           bsum);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_adj_scan_top, dim3(1), dim3(kScanBlock), 0, s, bsum, nblk, boff);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_adj_emit, dim3((unsigned)nblk), dim3(kScanBlock), 0, s, L, mask, flags, n_pairs, loc,
                           boff, ent, seg);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        int64_t grid = (max_ent + 255) / 256;
        grid = grid < 1 ? 1 : (grid > 256 * 8 ? 256 * 8 : grid);
        hipLaunchKernelGGL((k_adj_paths<R>), dim3((unsigned)grid), dim3(256), 0, s, L, rx, sph, cyl, prep, fcs, mask,
                           (const PathRec<R>*)rec, (const R*)gE, ent, boff + nblk, contrib);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (nlos > 0) {
        hipLaunchKernelGGL((k_adj_los<R>), dim3((unsigned)nlos), dim3(256), 0, s, L, rx, fcs, flags, (const R*)gE,
                           los_part);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_adj_reduce<R>), dim3(nb + 1), dim3(256), 0, s, contrib, seg, los_part, nlos, nb,
                       n_pairs > 0 ? 1 : 0, L.n_sph, (R*)d_sph, (R*)d_cyl, txpart);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((k_adjoint_tx<R>), dim3(1), dim3(64), 0, s, txpart, nb + 1, (R*)d_tx);
    return hipGetLastError();
}

hipError_t launch_adjoint(const LaunchParams& L, int precision, const float* rx, const float* sph, const float* cyl,
                          const BodyPrep* prep, const FreqConst* fcs, const uint8_t* mask, const void* rec,
                          const uint8_t* flags, const void* gE, char* scratch, void* d_sph, void* d_cyl, void* d_tx,
                          hipStream_t s) {
    return precision == 0 ? launch_adjoint_t<float>(L, rx, sph, cyl, prep, fcs, mask, rec, flags, gE, scratch, d_sph,
                                                    d_cyl, d_tx, s)
                          : launch_adjoint_t<double>(L, rx, sph, cyl, prep, fcs, mask, rec, flags, gE, scratch, d_sph,
                                                     d_cyl, d_tx, s);
}

}  // namespace utd
