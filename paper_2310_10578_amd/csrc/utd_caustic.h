// Uniform field of a sphere's creeping-ray pairs at the axial caustic
// (option caustic_uniform; spheres of the single-frame calls).
//
// Every creeping ray of a sphere lies in a half-plane bounded by the source
// axis.  A receiver sees them in pairs that meet on that axis: at the rear
// axis (the component of R - C along e_T negative) pair ell joins
// (side +, ell) and (side -, ell); at the front axis pair ell >= 1 joins
// (side -, ell - 1) and (side +, ell).  The first of each is the near ray
// (in R's own half-plane), the second the far ray, which crosses the axis
// once more.  Their ray fields grow as 1/sqrt(distance to the axis); the
// pair is summed instead as the integral over the azimuth alpha of the
// half-plane whose stationary points the two rays are:
//
//   phase k s_bar - x cos(alpha),  x = k a eps,  s_bar = (s_near + s_far)/2,
//   eps = angle of R from the axis (pi - theta_R at the rear, theta_R at the front),
//   amplitudes linear in cos(alpha) between the two rays' values,
//   polarisation dyadic (b b soft, n1 n2 hard) turning with alpha exactly,
//
// closed with int cos(n alpha) e^{j x cos alpha} d alpha = 2 pi j^n J_n(x).
// Each ray's amplitude keeps its Fock coefficients (path_coefs, measured
// from s_bar with the near ray's caustic count) and exchanges the
// transverse spreading for its finite limit
//   |S| sqrt(x) = sqrt(k a^2 sin(gamma_T) (eps / sin eps) / (s^d d_R)).
// For large x the Bessel functions' leading forms return the two ray fields
// of Eq. (4); on the axis the field is finite.
//
//   k_pair     per receiver: the pairs of every sphere whose two paths are
//              both visible leave the mask (their bits go to a pair byte per
//              (sphere, receiver)); a path left alone within the axis guard
//              is dropped and the receiver flagged, as without the option
//   k_caustic  per (receiver, 4 frequencies): the pairs' field added into E,
//              after k_field
// The path kernels run with a zero guard under this option (no path is
// dropped before it is paired).
namespace utd {

// sin(pi k / 32), k = 0 .. 16: the trapezoidal nodes below (cos(pi k / 32)
// is entry 16 - k; the nodes beyond pi/2 follow by symmetry)
__device__ const double kNodeSin[17] = {
    0.0, 0.098017140329560604, 0.19509032201612825, 0.29028467725446233,
    0.38268343236508978, 0.47139673682599764, 0.55557023301960218, 0.63439328416364549,
    0.70710678118654752, 0.77301045336273699, 0.83146961230254524, 0.88192126434835494,
    0.92387953251128674, 0.95694033573220894, 0.98078528040323043, 0.99518472667219682, 1.0};

__device__ __forceinline__ void gsincos_r(double x, double* s, double* c) { sincos(x, s, c); }
__device__ __forceinline__ void gsincos_r(float x, float* s, float* c) { sincosf(x, s, c); }

// J_0 .. J_3 at x >= 0 in precision R.  Up to x = x_s the trapezoidal rule
// on Bessel's integral J_n(x) = (1/2 pi) int_0^{2 pi} cos(n t - x sin t) dt
// with M nodes, whose error is the aliased orders M - n and beyond; the
// integrand is even about t = pi, so M/2 + 1 distinct nodes.  FP64: M = 64
// up to x_s = 25 (J_61(25) ~ 3e-16); FP32: M = 32 up to x_s = 12
// (J_29(12) ~ 5e-8).  Beyond: Hankel's asymptotic expansion,
// J_n = sqrt(2/(pi x)) (P cos chi - Q sin chi) with chi = x - (2n + 1) pi/4
// and P, Q the even and odd terms of the series in 1/(8x), 16 terms (below
// 1e-15 relative at x = 25, 1e-9 at x = 12).
template <typename R>
__device__ __forceinline__ void bessel_j03(R x, R J[4]) {
    constexpr bool kF64 = sizeof(R) == 8;
    constexpr int kStep = kF64 ? 1 : 2;          // every node of the 64, or every other one
    if (x <= (kF64 ? (R)25 : (R)12)) {
        R acc[4] = {(R)0, (R)0, (R)0, (R)0};
#pragma unroll 1
        for (int k = 0; k <= 32; k += kStep) {
            const bool lo = k <= 16;
            const R st = (R)kNodeSin[lo ? k : 32 - k];
            const R ct = lo ? (R)kNodeSin[16 - k] : -(R)kNodeSin[k - 16];
            R sx, cx;
            gsincos_r(x * st, &sx, &cx);
            const R w = (k == 0 || k == 32) ? (R)1 : (R)2;
            R cn = (R)1, sn = (R)0;   // cos(n t), sin(n t)
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                acc[n] += w * (cn * cx + sn * sx);
                const R c2 = cn * ct - sn * st;
                sn = sn * ct + cn * st;
                cn = c2;
            }
        }
#pragma unroll
        for (int n = 0; n < 4; ++n) J[n] = acc[n] * (R)(kStep / 64.0);
        return;
    }
    R s, c;
    gsincos_r(x, &s, &c);
    // cos and sin of chi_0 = x - pi/4; each next order turns chi by -pi/2
    R cc = (c + s) * (R)0.70710678118654752, sc = (s - c) * (R)0.70710678118654752;
    const R amp = sqrt((R)2 / ((R)kPi * x)), i8x = (R)1 / ((R)8 * x);
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        const R mu = (R)(4 * n * n);
        R t = (R)1, P = (R)1, Q = (R)0;
#pragma unroll 1
        for (int k = 1; k <= 16; ++k) {
            t *= (mu - (R)((2 * k - 1) * (2 * k - 1))) * i8x / (R)k;
            switch (k & 3) {
                case 1: Q += t; break;
                case 2: P -= t; break;
                case 3: Q -= t; break;
                default: P += t; break;
            }
        }
        J[n] = amp * (P * cc - Q * sc);
        const R c2 = sc;
        sc = -cc;
        cc = c2;
    }
}

// Mask bits of pair ell, near path first (bit 2 ell + 1 is side - of ell).
__device__ __forceinline__ void pair_bits(bool rear, int ell, int* bn, int* bf) {
    if (rear) {
        *bn = 2 * ell;
        *bf = 2 * ell + 1;
    } else {
        *bn = 2 * ell - 1;
        *bf = 2 * ell;
    }
}

// grid ceil(n_rx / 256); pm[sphere][rx]: bit ell set for pair ell.
__global__ void __launch_bounds__(256) k_pair(LaunchParams L, double guard, const float* __restrict__ rx,
                                              const BodyPrep* __restrict__ prep, uint8_t* __restrict__ mask,
                                              uint8_t* __restrict__ pm) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L.n_rx) return;
    const d3 R3 = mk(rx[3 * i], rx[3 * i + 1], rx[3 * i + 2]);
    const uint32_t creep = (1u << (2 * (L.l_enc + 1))) - 1u;
    for (int b = 0; b < L.n_sph; ++b) {
        const int64_t o = (int64_t)b * L.n_rx + i;
        uint32_t m = mask[o];
        uint32_t pb = 0u;
        if (m & creep) {
            const RxGeo g = rx_geo_sphere<double>(prep[b], R3);
            const bool rear = g.along < 0.0;
            for (int ell = rear ? 0 : 1; ell <= L.l_enc; ++ell) {
                int bn, bf;
                pair_bits(rear, ell, &bn, &bf);
                const uint32_t two = (1u << bn) | (1u << bf);
                if ((m & two) == two) {
                    m &= ~two;
                    pb |= 1u << ell;
                }
            }
            if ((m & creep) && g.wn < guard) m = (m & ~creep) | (1u << kBitCaustic);
            mask[o] = (uint8_t)m;
        }
        pm[o] = (uint8_t)pb;
    }
}

template <typename R> __device__ __forceinline__ cplx<R> cx_add(cplx<R> a, cplx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R> __device__ __forceinline__ cplx<R> cx_sub(cplx<R> a, cplx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R> __device__ __forceinline__ cplx<R> cx_scale(cplx<R> a, R s) { return {a.re * s, a.im * s}; }
// s a + j t b for real s, t
template <typename R> __device__ __forceinline__ cplx<R> cx_comb(R s, cplx<R> a, R t, cplx<R> b) {
    return {s * a.re - t * b.im, s * a.im + t * b.re};
}

// Frequencies per thread of k_caustic (grid rows).  With the four-wave cap
// below, per call on the sphere workload with one encirclement (FP32 /
// FP64): 2 per row 0.396 / 1.42 ms, 4 0.402 / 1.38, 8 0.455 / 1.50, 16
// 0.547 / 1.61 (fewer, longer rows recompute the pair geometry less often
// but fill the chip less).
constexpr int kCausticFreqs = 4;

// grid (ceil(n_rx / 256), rows): receiver i at the frequencies of its row,
// kCausticFreqs consecutive ones every rows * kCausticFreqs; adds into
// E [n_f][3][n_rx] complex.
// At most 128 VGPRs (four waves per SIMD; eight frequencies per row): 0.459
// against 0.505 ms (FP32) and 1.49 against 1.67 ms (FP64) with the
// compiler's own choice of 155 and 256; five waves helped FP32 no further
// and cost FP64 40 %.
template <typename R>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_caustic(LaunchParams L, const float* __restrict__ rx, const BodyPrep* __restrict__ prep,
          const FreqConst* __restrict__ fcs, const uint8_t* __restrict__ pm, R* __restrict__ E_out) {
    __shared__ __attribute__((aligned(16))) R s_reg[TableStage<R>::NREG];
    __shared__ __attribute__((aligned(16))) R s_tf[TableStage<R>::NTF];
    const Tabs<R> tb = TableStage<R>::template stage<256>(s_reg, s_tf);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L.n_rx) return;
    const d3 R3 = mk(rx[3 * i], rx[3 * i + 1], rx[3 * i + 2]);
    const d3 T = mk(L.T[0], L.T[1], L.T[2]);
    const d3 p = mk(L.p[0], L.p[1], L.p[2]);
    for (int b = 0; b < L.n_sph; ++b) {
        uint32_t pb = pm[(int64_t)b * L.n_rx + i];
        while (pb) {
            const int ell = __builtin_ctz(pb);
            pb &= pb - 1u;
            const BodyPrep P = prep[b];
            const RxGeo g = rx_geo_sphere<double>(P, R3);
            const bool rear = g.along < 0.0;
            const int sn = rear ? 1 : -1, sf = -sn;
            PathEval<R> pn, pf;
            bool cz;
            sphere_creep<R, double>(P, g, R3, T, L, sn, rear ? ell : ell - 1, &cz, &pn, nullptr);
            sphere_creep<R, double>(P, g, R3, T, L, sf, ell, &cz, &pf, nullptr);
            // both rays measured from s_bar, with the near ray's caustic count
            const double sbar = 0.5 * (pn.s_tot + pf.s_tot);
            pn.s_tot = sbar;
            pf.s_tot = sbar;
            pf.nc = pn.nc;
            const double a = P.a, dR = g.dR, sI = P.sI0, sD = g.sD0;
            const double c1 = a / P.dT, s1 = sI / P.dT;
            const R c2n = (R)(sn > 0 ? g.c2p : g.c2m), s2n = (R)(sn > 0 ? g.s2p : g.s2m);
            const R c2f = (R)(sf > 0 ? g.c2p : g.c2m), s2f = (R)(sf > 0 ? g.s2p : g.s2m);
            const double eps = rear ? atan2(g.wn, -g.along) : atan2(g.wn, g.along);
            const double ratio = g.wn > 0.0 ? eps * dR / g.wn : 1.0;     // eps / sin(eps)
            // amplitude per sqrt(k): source strength, the Fock prefactor
            // -sqrt(2) m/k^{1/3}, |S| sqrt(x / k), 1/sqrt(2 pi) and 1/s^i
            const double W0 = L.amp * (-1.4142135623730951 * cbrt(0.5 * a)) *
                              sqrt(a * a * s1 * ratio / (sD * dR)) / (sI * 2.5066282746310002);
            const d3 u = mk(P.eT[0], P.eT[1], P.eT[2]);
            // near the axis the rounding of R - C leaves eperp a component
            // along u (relative 1e-16 |R - C| / wn): removed, so that
            // p1 e1 + p2 e2 is the transverse dipole whatever e1's direction
            d3 e1 = mk(sn * g.eperp.x, sn * g.eperp.y, sn * g.eperp.z);
            const double e1u = dot(e1, u);
            e1 = mk(e1.x - e1u * u.x, e1.y - e1u * u.y, e1.z - e1u * u.z);
            const double ie1 = 1.0 / sqrt(dot(e1, e1));
            e1 = mk(e1.x * ie1, e1.y * ie1, e1.z * ie1);
            const d3 e2 = cross(u, e1);
            const R pu = (R)dot(p, u), p1 = (R)dot(p, e1), p2 = (R)dot(p, e2);
            const R c1R = (R)c1, s1R = (R)s1;
            const R ux = (R)u.x, uy = (R)u.y, uz = (R)u.z;
            const R e1x = (R)e1.x, e1y = (R)e1.y, e1z = (R)e1.z;
            const R e2x = (R)e2.x, e2y = (R)e2.y, e2z = (R)e2.z;
            // this row's frequencies: kCausticFreqs consecutive ones, every
            // gridDim.y * kCausticFreqs
#pragma unroll 1
            for (int jb = (int)blockIdx.y * kCausticFreqs; jb < L.n_f; jb += (int)gridDim.y * kCausticFreqs)
#pragma unroll 1
            for (int j = jb; j < jb + kCausticFreqs && j < L.n_f; ++j) {
                if (!fcs[j].ok) continue;      // an invalid frequency keeps its zero field
                const FreqC<R> fc(fcs[j]);
                cplx<R> csn, chn, csf, chf;
                path_coefs<R, kCreep>(pn, tb, fc, &csn, &chn);
                path_coefs<R, kCreep>(pf, tb, fc, &csf, &chf);
                const double k = fcs[j].kd;
                R J[4];
                bessel_j03<R>((R)(k * a * eps), J);
                const R pi = (R)kPi;
                const R a0 = (R)2 * pi * J[0], a1 = (R)2 * pi * J[1];
                const R am = pi * (J[0] - J[2]), ap = pi * (J[0] + J[2]);
                const R b3 = (R)0.5 * pi * ((R)3 * J[1] - J[3]), b1 = (R)0.5 * pi * (J[1] + J[3]);
                // W e^{j pi/4} times each coefficient
                const R w = (R)(W0 * sqrt(k) * 0.70710678118654752);
                const cplx<R> wq{w, w};
                const cplx<R> Gsn = cmul(wq, csn), Gsf = cmul(wq, csf);
                const cplx<R> Ghn = cmul(wq, chn), Ghf = cmul(wq, chf);
                const R h = (R)0.5;
                const cplx<R> Gsb = cx_scale(cx_add(Gsn, Gsf), h), dGs = cx_scale(cx_sub(Gsn, Gsf), h);
                const cplx<R> Hun = cx_scale(Ghn, c2n), Huf = cx_scale(Ghf, c2f);
                const cplx<R> Hrn = cx_scale(Ghn, s2n), Hrf = cx_scale(Ghf, s2f);
                const cplx<R> Hub = cx_scale(cx_add(Hun, Huf), h), dHu = cx_scale(cx_sub(Hun, Huf), h);
                const cplx<R> Hrb = cx_scale(cx_add(Hrn, Hrf), h), dHr = cx_scale(cx_sub(Hrn, Hrf), h);
                // the three components along u, e1, e2
                const cplx<R> E_s1 = cx_scale(cx_comb(ap, Gsb, b1, dGs), p1);
                const cplx<R> E_s2 = cx_scale(cx_comb(am, Gsb, b3, dGs), p2);
                const cplx<R> E_u = cx_add(cx_scale(cx_comb(a0, Hub, a1, dHu), c1R * pu),
                                           cx_scale(cx_comb(am, dHu, a1, Hub), s1R * p1));
                const cplx<R> E_1 = cx_add(E_s1, cx_add(cx_scale(cx_comb(am, dHr, a1, Hrb), c1R * pu),
                                                        cx_scale(cx_comb(am, Hrb, b3, dHr), s1R * p1)));
                const cplx<R> E_2 = cx_add(E_s2, cx_scale(cx_comb(ap, Hrb, b1, dHr), s1R * p2));
                const R vx[3] = {ux, uy, uz}, v1[3] = {e1x, e1y, e1z}, v2[3] = {e2x, e2y, e2z};
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int64_t o = ((int64_t)j * 3 + c) * L.n_rx + i;
                    E_out[2 * o] += E_u.re * vx[c] + E_1.re * v1[c] + E_2.re * v2[c];
                    E_out[2 * o + 1] += E_u.im * vx[c] + E_1.im * v1[c] + E_2.im * v2[c];
                }
            }
        }
    }
}

hipError_t launch_pairs(const LaunchParams& L, double guard, const float* rx, const BodyPrep* prep, uint8_t* mask,
                        uint8_t* pm, hipStream_t s) {
    if (L.n_sph == 0 || L.n_rx == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pair, dim3((unsigned)((L.n_rx + 255) / 256)), dim3(256), 0, s, L, guard, rx, prep, mask, pm);
    return hipGetLastError();
}

hipError_t launch_caustic(const LaunchParams& L, int precision, const float* rx, const BodyPrep* prep,
                          const FreqConst* fcs, const uint8_t* pm, void* E, hipStream_t s) {
    if (L.n_sph == 0 || L.n_rx == 0 || L.n_f == 0) return hipSuccess;
    const int rows = (L.n_f + kCausticFreqs - 1) / kCausticFreqs;
    const dim3 grid((unsigned)((L.n_rx + 255) / 256), (unsigned)(rows < 65535 ? rows : 65535));
    if (precision == 0)
        hipLaunchKernelGGL((k_caustic<float>), grid, dim3(256), 0, s, L, rx, prep, fcs, pm, (float*)E);
    else
        hipLaunchKernelGGL((k_caustic<double>), grid, dim3(256), 0, s, L, rx, prep, fcs, pm, (double*)E);
    return hipGetLastError();
}

}  // namespace utd
