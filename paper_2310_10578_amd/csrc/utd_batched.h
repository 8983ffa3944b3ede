// Many frames in one launch (utd_smooth_field_batched): every frame has its
// own cylinders and receivers (CSR offsets), all frames share the scene
// triangles, the source and the frequencies.  Included by utd_kernels.hip.
//
//   k_batch_prep   body constants of every cylinder, frequency constants,
//                  sanitised per-frame offsets, the tile prefix sum and the
//                  work-queue counter reset (one block does the scan)
//   k_batch_sort   per frame, a counting sort of the receivers by spatial
//                  cell (Morton order of a grid over the frame's receivers),
//                  so that the receivers of one tile are neighbours
//   k_batch_grid   per frame, the grid of the cylinders' footprints that
//                  the visibility tests take their candidate bodies from
//   k_batch_fans   per (cylinder, side), the visibility profile of the
//                  source-side legs along the tangent line
//   k_batch_los    per receiver, in the tiles' order, its flags and the
//                  visibility of its direct ray
//   k_batch        persistent: each workgroup takes the next (frame, tile of
//                  TILE receivers in sorted order) from an atomic work queue
//                  until the queue is empty.  A lane owns one receiver: its
//                  flags and direct ray (from k_batch_los); then per group
//                  of the frame's bodies a cull (tile box, then per
//                  receiver), the classification of the surviving
//                  (receiver, body) pairs one per lane into an LDS queue of
//                  candidate paths, the visibility of the candidates one per
//                  lane, and the Fock evaluation of each lane's visible paths
//                  at every frequency, added in place to the lane's column of
//                  the block's field scratch (initialised with the direct
//                  ray), which is copied to the receiver's own place in E
//                  when the tile is done.
//
// Neighbouring receivers have nearly the same paths: their candidate legs
// walk the same BVH nodes and meet the same bodies, so a wavefront of
// neighbours diverges far less than one of receivers scattered over the room
// (the crowd's receivers are uniform random; sorting them halves the time).
// The order changes nothing in any receiver's result: each receiver's field
// is computed by one lane, whatever lane that is.
//
// Fusing visibility and field keeps no per-path records (a 256-frame crowd
// has ~2.4e8 receiver-body pairs).  Each receiver's field is the direct ray,
// then per group of 32 bodies its creeping paths in (body, ell, side) order
// and its reflections in body order, so a frame gives the field of
// utd_smooth_field on that frame up to rounding.
#pragma once

namespace utd {

// One block scans the frames; all threads fill body and frequency constants.
__global__ void __launch_bounds__(1024) k_batch_prep(BatchParams B, const int64_t* __restrict__ body_off,
                                                     const int64_t* __restrict__ rx_off,
                                                     const float* __restrict__ cyl, const double* __restrict__ freqs,
                                                     BodyPrep* __restrict__ prep, FreqConst* __restrict__ fc,
                                                     int64_t* __restrict__ bo, int64_t* __restrict__ ro,
                                                     int64_t* __restrict__ tile_off, unsigned* __restrict__ counter) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nt = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b = tid; b < B.n_cyl; b += nt) prep[b] = body_prep(B.L.T, nullptr, 0, cyl, (int)b);
    for (int64_t f = tid; f < B.L.n_f; f += nt) fc[f] = freq_const(freqs[f]);
    if (blockIdx.x != 0) return;
    // Sanitised offsets: clamped to [0, n] and made non-decreasing, so a
    // malformed frame becomes empty instead of indexing out of bounds.
    __shared__ int64_t s_scan[1024];
    __shared__ int64_t s_carry[3];
    if (threadIdx.x == 0) {
        s_carry[0] = 0;   // tiles
        s_carry[1] = 0;   // running max of body offsets
        s_carry[2] = 0;   // running max of receiver offsets
        tile_off[0] = 0;
        bo[0] = 0;
        ro[0] = 0;
        *counter = 0u;
    }
    __syncthreads();
    for (int64_t base = 0; base < B.n_frames; base += blockDim.x) {
        int64_t f = base + threadIdx.x;
        int64_t b1 = 0, r1 = 0;
        if (f < B.n_frames) {
            b1 = body_off[f + 1];
            r1 = rx_off[f + 1];
            b1 = b1 < 0 ? 0 : (b1 > B.n_cyl ? B.n_cyl : b1);
            r1 = r1 < 0 ? 0 : (r1 > B.n_rx ? B.n_rx : r1);
        }
        // running maxima (prefix max) of the clamped end offsets
        s_scan[threadIdx.x] = b1;
        __syncthreads();
        for (int w = 1; w < (int)blockDim.x; w <<= 1) {
            int64_t v = threadIdx.x >= (unsigned)w ? s_scan[threadIdx.x - w] : 0;
            __syncthreads();
            if (v > s_scan[threadIdx.x]) s_scan[threadIdx.x] = v;
            __syncthreads();
        }
        int64_t bm = s_scan[threadIdx.x] > s_carry[1] ? s_scan[threadIdx.x] : s_carry[1];
        __syncthreads();
        s_scan[threadIdx.x] = r1;
        __syncthreads();
        for (int w = 1; w < (int)blockDim.x; w <<= 1) {
            int64_t v = threadIdx.x >= (unsigned)w ? s_scan[threadIdx.x - w] : 0;
            __syncthreads();
            if (v > s_scan[threadIdx.x]) s_scan[threadIdx.x] = v;
            __syncthreads();
        }
        int64_t rm = s_scan[threadIdx.x] > s_carry[2] ? s_scan[threadIdx.x] : s_carry[2];
        __syncthreads();
        // receivers of frame f: [ro[f], rm); its start is the previous frame's end
        s_scan[threadIdx.x] = rm;
        __syncthreads();
        int64_t r0 = threadIdx.x == 0 ? s_carry[2] : s_scan[threadIdx.x - 1];
        int64_t nt_f = f < B.n_frames ? (rm - r0 + B.tile - 1) / B.tile : 0;
        __syncthreads();
        // tile counts: inclusive prefix sum
        s_scan[threadIdx.x] = nt_f;
        __syncthreads();
        for (int w = 1; w < (int)blockDim.x; w <<= 1) {
            int64_t v = threadIdx.x >= (unsigned)w ? s_scan[threadIdx.x - w] : 0;
            __syncthreads();
            s_scan[threadIdx.x] += v;
            __syncthreads();
        }
        int64_t toff = s_carry[0] + s_scan[threadIdx.x];
        if (f < B.n_frames) {
            tile_off[f + 1] = toff;
            bo[f + 1] = bm;
            ro[f + 1] = rm;
        }
        __syncthreads();
        int last = (int)((B.n_frames - base < (int64_t)blockDim.x ? B.n_frames - base : blockDim.x) - 1);
        if ((int)threadIdx.x == last) {
            s_carry[0] = toff;
            s_carry[1] = bm;
            s_carry[2] = rm;
        }
        __syncthreads();
    }
}

// Spatial counting sort of each frame's receivers (one block of 1024 threads
// per frame, grid-stride over frames): the bounding box of the frame's finite
// receivers gets a grid of at most kSortCells cells, about cubic, with up to
// 2^6 cells per axis (an axis of small extent gets fewer bits, a flat layer
// none); cells are numbered in Morton order; then a counting sort in LDS.
// perm[ro[f] + k] is the frame-local index of the receiver at sorted
// position k.  Non-finite receivers go to cell 0.  The cell of every receiver
// is stored (key) in the counting pass and read back in the scatter pass, so
// the two passes agree exactly and perm is a permutation.
constexpr int kSortCells = 4096;
constexpr int kSortBits = 12;

__global__ void __launch_bounds__(1024) k_batch_sort(BatchParams B, const float* __restrict__ rx,
                                                     const int64_t* __restrict__ ro, uint16_t* __restrict__ key,
                                                     int* __restrict__ perm) {
    __shared__ int hist[kSortCells];
    __shared__ int s_part[1024];
    __shared__ float s_lo[3][16], s_hi[3][16];
    __shared__ float s_org[3], s_scale[3];
    __shared__ int s_bits[3];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int64_t fr = blockIdx.x; fr < B.n_frames; fr += gridDim.x) {
        const int64_t r0 = ro[fr];
        const int n = (int)(ro[fr + 1] - r0);
        // 1. bounding box of the finite receivers
        float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int k = tid; k < n; k += 1024) {
            const float x = rx[3 * (r0 + k)], y = rx[3 * (r0 + k) + 1], z = rx[3 * (r0 + k) + 2];
            if (isfinite(x) && isfinite(y) && isfinite(z)) {
                lo[0] = fminf(lo[0], x); lo[1] = fminf(lo[1], y); lo[2] = fminf(lo[2], z);
                hi[0] = fmaxf(hi[0], x); hi[1] = fmaxf(hi[1], y); hi[2] = fmaxf(hi[2], z);
            }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            for (int o = 32; o > 0; o >>= 1) {
                lo[a] = fminf(lo[a], __shfl_xor(lo[a], o, 64));
                hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], o, 64));
            }
            if (lane == 0) { s_lo[a][wave] = lo[a]; s_hi[a][wave] = hi[a]; }
        }
        for (int k = tid; k < kSortCells; k += 1024) hist[k] = 0;
        __syncthreads();
        if (tid == 0) {
            float ext[3], emax = 0.0f;
            for (int a = 0; a < 3; ++a) {
                float l = s_lo[a][0], h = s_hi[a][0];
                for (int w = 1; w < 16; ++w) { l = fminf(l, s_lo[a][w]); h = fmaxf(h, s_hi[a][w]); }
                if (!(h >= l)) { l = 0.0f; h = 0.0f; }           // no finite receiver
                s_org[a] = l;
                ext[a] = h - l;
                emax = fmaxf(emax, ext[a]);
            }
            int b[3];
            for (int a = 0; a < 3; ++a) {
                b[a] = 0;
                if (emax > 0.0f && ext[a] > 0.0f) {
                    float r = ceilf(log2f(ext[a] / emax * 64.0f));
                    b[a] = r < 0.0f ? 0 : (r > 6.0f ? 6 : (int)r);
                }
            }
            while (b[0] + b[1] + b[2] > kSortBits) {
                int m = b[0] >= b[1] ? (b[0] >= b[2] ? 0 : 2) : (b[1] >= b[2] ? 1 : 2);
                --b[m];
            }
            for (int a = 0; a < 3; ++a) {
                s_bits[a] = b[a];
                s_scale[a] = b[a] > 0 ? (float)(1 << b[a]) / ext[a] : 0.0f;
            }
        }
        __syncthreads();
        // 2. cell of every receiver and the cell counts
        for (int k = tid; k < n; k += 1024) {
            int c[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const float t = (rx[3 * (r0 + k) + a] - s_org[a]) * s_scale[a];
                const int top = (1 << s_bits[a]) - 1;
                c[a] = t >= 1.0f ? (t < (float)top ? (int)t : top) : 0;      // NaN -> 0
            }
            int m = 0, pos = 0;
            for (int bit = 0; bit < 6; ++bit)
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    if (bit < s_bits[a]) m |= ((c[a] >> bit) & 1) << pos++;
            key[r0 + k] = (uint16_t)m;
            atomicAdd(&hist[m], 1);
        }
        __syncthreads();
        // 3. exclusive prefix sum of the counts: four cells per thread, then
        // an inclusive scan of the 1024 partial sums
        int c4[4], sum = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) { c4[q] = hist[4 * tid + q]; sum += c4[q]; }
        s_part[tid] = sum;
        __syncthreads();
        for (int w = 1; w < 1024; w <<= 1) {
            const int v = tid >= w ? s_part[tid - w] : 0;
            __syncthreads();
            s_part[tid] += v;
            __syncthreads();
        }
        int run = s_part[tid] - sum;
#pragma unroll
        for (int q = 0; q < 4; ++q) { hist[4 * tid + q] = run; run += c4[q]; }
        __syncthreads();
        // 4. scatter: the same thread reads back the cells it wrote
        for (int k = tid; k < n; k += 1024) {
            const int pos = atomicAdd(&hist[key[r0 + k]], 1);
            perm[r0 + pos] = k;
        }
        __syncthreads();
    }
}

// Visibility profiles of the source-side legs (the incident segments of
// Eqs. (2) and (4)).  Every creeping path of one (cylinder, side) attaches
// on the same vertical tangent line (the tangent point of the source's
// horizontal tangent; only the height depends on the receiver), so the legs
// from the source to it form a planar fan, and whether a leg is blocked is a
// function of the attachment height alone: computed once per frame for all
// receivers (the reuse of diffraction paths across a local area, Sec. III-A).
//
// Each occluder cuts the fan in a segment (a triangle) or a rectangle (a
// cylinder); the rays from the source through the cut reach the tangent
// line in an interval of heights.  A cut (lo, hi, mlo, mhi) blocks heights
// in (lo + mlo, hi - mhi) for certain and leaves heights within mlo of lo
// and mhi of hi undecided.  The margins are the spatial tolerance ds (40
// FP32 ulps of the scene's largest coordinate) seen from the tangent line
// (ds / t for a crossing at the leg's parameter t), so outside them the
// FP32 segment test of the same leg and the exact body tests decide the same
// way.  A height is blocked if a cut blocks it for certain, else undecided if
// it lies in a cut's margin, else free; the profile stores that
// classification of the line's heights as at most kFanRuns runs.  A run
// boundary, a degenerate cut (a triangle edge in the fan's plane, a
// cylinder tangent to it), more than kFanCuts cuts or runs, a fan reaching
// outside the scene box, or a main tree larger than kFanMaxNodes nodes all
// fall back to testing the leg itself, so the decisions are those of the
// per-segment tests.
constexpr int kFanRuns = 16;
constexpr int kFanCuts = 64;
constexpr int kFanMaxNodes = 4096;
constexpr int kFanFree = 0, kFanBlocked = 1, kFanUndecided = 2;
struct FanProfile {
    int n;                       // runs; -1: no profile (every leg is tested)
    float z0;                    // start of the first run
    float pad[2];
    float2 run[kFanRuns];        // (end height, status)
};

// kFanFree: no occluder blocks the leg ending at height z; kFanBlocked;
// kFanUndecided: test the leg.
__device__ __forceinline__ int fan_lookup(const FanProfile* __restrict__ F, double z) {
    const int n = F->n;
    const float zf = (float)z;
    if (n <= 0 || !(zf > F->z0 + 1e-6f)) return kFanUndecided;
    for (int i = 0; i < n; ++i) {
        const float2 r = F->run[i];
        if (zf < r.x - 1e-6f) return (int)r.y;
        if (zf <= r.x + 1e-6f) return kFanUndecided;      // at a run boundary
    }
    return kFanUndecided;                                  // above the last run
}

// Cuts of one fan (source T, horizontal unit direction (dx, dy) towards the
// tangent line at horizontal distance U), appended to an LDS list.
struct FanGeo {
    double tx, ty, tz, dx, dy, U, ds;
    double zmin, zmax;           // the heights that matter (the line's, widened)
    __device__ double zline(double u, double w) const { return tz + (w - tz) * U / u; }
};

// Appends one cut (unless it lies wholly outside the heights that matter);
// returns false when the list is full.
__device__ __forceinline__ bool fan_put(const FanGeo& F, float4* cuts, int* ncut, double lo, double hi, double mlo,
                                        double mhi) {
    if (hi + mhi < F.zmin || lo - mlo > F.zmax) return true;
    const int k = atomicAdd(ncut, 1);
    if (k >= kFanCuts) return false;
    cuts[k] = make_float4((float)lo, (float)hi, (float)mlo + 1e-6f, (float)mhi + 1e-6f);
    return true;
}

// The segment (ua, wa)-(ub, wb) of the fan's plane inside an occluder; with
// `edge` (a cut along a triangle edge or through a vertex) its whole image
// is undecided.  Returns false on overflow.
__device__ __forceinline__ bool fan_segment(const FanGeo& F, float4* cuts, int* ncut, double ua, double wa,
                                            double ub, double wb, bool edge) {
    const double e0 = 1e-6 * F.U, e1 = (1.0 - 1e-6) * F.U;  // open leg parameter (kSegEps)
    double t0 = 0.0, t1 = 1.0;
    const double du = ub - ua;
    if (du != 0.0) {
        double ta = (e0 - ua) / du, tb = (e1 - ua) / du;
        if (ta > tb) { const double x = ta; ta = tb; tb = x; }
        t0 = fmax(t0, ta);
        t1 = fmin(t1, tb);
    } else if (ua < e0 || ua > e1) {
        return true;
    }
    if (t0 > t1) return true;
    const double u0 = ua + t0 * du, w0 = wa + t0 * (wb - wa);
    const double u1 = ua + t1 * du, w1 = wa + t1 * (wb - wa);
    const double z0 = F.zline(u0, w0), z1 = F.zline(u1, w1);
    const double m0 = F.ds * F.U / u0, m1 = F.ds * F.U / u1;
    const double lo = fmin(z0, z1), hi = fmax(z0, z1);
    const double mlo = z0 <= z1 ? m0 : m1, mhi = z0 <= z1 ? m1 : m0;
    if (edge) {
        const double mid = 0.5 * (lo + hi), half = 0.5 * (hi - lo) + fmax(mlo, mhi);
        return fan_put(F, cuts, ncut, mid, mid, half, half);
    }
    return fan_put(F, cuts, ncut, lo, hi, mlo, mhi);
}

// A scene triangle; returns false on overflow or a degenerate cut.
__device__ __forceinline__ bool fan_triangle(const FanGeo& F, float4* cuts, int* ncut, float4 a, float4 b, float4 c) {
    const double vx[3] = {a.x, b.x, c.x}, vy[3] = {a.y, b.y, c.y}, vz[3] = {a.z, b.z, c.z};
    double sd[3];
    int on = 0, pos = 0, neg = 0;
    const double tol = 1e-12 * (1.0 + fabs(F.tx) + fabs(F.ty) + F.U);
    for (int i = 0; i < 3; ++i) {
        sd[i] = -F.dy * (vx[i] - F.tx) + F.dx * (vy[i] - F.ty);
        if (fabs(sd[i]) <= tol) { sd[i] = 0.0; ++on; }
        else if (sd[i] > 0.0) ++pos;
        else ++neg;
    }
    if (on == 3) return false;                         // in the fan's plane
    if (on == 0 && (pos == 0 || neg == 0)) return true;
    double pu[3], pw[3];
    int np = 0;
    for (int i = 0; i < 3; ++i) {
        const int j = i == 2 ? 0 : i + 1;
        if (sd[i] == 0.0) {
            pu[np] = F.dx * (vx[i] - F.tx) + F.dy * (vy[i] - F.ty);
            pw[np] = vz[i];
            ++np;
        }
        if ((sd[i] < 0.0 && sd[j] > 0.0) || (sd[i] > 0.0 && sd[j] < 0.0)) {
            const double f = sd[i] / (sd[i] - sd[j]);
            const double x = vx[i] + f * (vx[j] - vx[i]), y = vy[i] + f * (vy[j] - vy[i]);
            pu[np] = F.dx * (x - F.tx) + F.dy * (y - F.ty);
            pw[np] = vz[i] + f * (vz[j] - vz[i]);
            ++np;
        }
    }
    if (np < 2) return np == 1 ? fan_segment(F, cuts, ncut, pu[0], pw[0], pu[0], pw[0], true) : true;
    return fan_segment(F, cuts, ncut, pu[0], pw[0], pu[1], pw[1], on >= 2);
}

// Another solid vertical cylinder (cx, cy, z0, h, a); false on overflow or
// a cylinder tangent to the fan's plane.
__device__ __forceinline__ bool fan_cylinder(const FanGeo& F, float4* cuts, int* ncut, const float* cq) {
    const double cx = cq[0], cy = cq[1], cz0 = cq[2], ch = cq[3], ca = cq[4];
    const double dc = -F.dy * (cx - F.tx) + F.dx * (cy - F.ty);
    if (fabs(dc) >= ca + F.ds) return true;
    if (fabs(dc) > ca - F.ds) return false;
    const double hc = sqrt((ca - dc) * (ca + dc));
    const double uc = F.dx * (cx - F.tx) + F.dy * (cy - F.ty);
    const double e0 = 1e-6 * F.U, e1 = (1.0 - 1e-6) * F.U;
    const double u0 = fmax(uc - hc, e0), u1 = fmin(uc + hc, e1);
    if (u0 >= u1) return true;
    const double w0 = cz0, w1 = cz0 + ch;
    const double za = F.zline(u0, w0), zb = F.zline(u0, w1), zc = F.zline(u1, w0), zd = F.zline(u1, w1);
    const double lo = fmin(fmin(za, zb), fmin(zc, zd)), hi = fmax(fmax(za, zb), fmax(zc, zd));
    const double m = F.ds * F.U / u0;                  // the larger of the two columns' margins
    return fan_put(F, cuts, ncut, lo, hi, m, m);
}

// One wavefront per (cylinder, side) of the call, four per workgroup: the
// fan profiles of every frame, from the sanitised body offsets and the body
// constants of k_batch_prep.  Lanes share the cuts: the main tree's nodes
// (n_main of them) and the frame's cylinders are strided over the lanes.
__global__ void __launch_bounds__(256) k_batch_fans(BatchParams B, const float* __restrict__ cyl,
                                                    const BodyPrep* __restrict__ prep,
                                                    const int64_t* __restrict__ bo, const float4* __restrict__ nodes,
                                                    const float4* __restrict__ tris, int n_main,
                                                    FanProfile* __restrict__ fans) {
    __shared__ float4 s_cut[4][kFanCuts];
    __shared__ float s_bp[4][4 * kFanCuts + 2];
    __shared__ float s_srt[4][4 * kFanCuts + 2];
    __shared__ int s_st[4][4 * kFanCuts + 2];
    __shared__ int s_n[4];
    __shared__ int s_bad[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t k = (int64_t)blockIdx.x * 4 + w;          // (cylinder, side) of this wavefront
    if (k >= 2 * B.n_cyl) return;                            // wave-uniform
    FanProfile* out = fans + k;
    const int64_t g = k >> 1;
    const int sgn = (k & 1) ? -1 : 1;
    if (lane == 0) { s_n[w] = 0; s_bad[w] = 0; }
    __builtin_amdgcn_wave_barrier();
    // frame of cylinder g: the last f with bo[f] <= g (empty frames skipped)
    int64_t lo = 0, hi = B.n_frames;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (bo[mid] <= g) lo = mid; else hi = mid;
    }
    const BodyPrep P = prep[g];
    const LaunchParams& L = B.L;
    bool ok = B.n_frames > 0 && bo[lo] <= g && g < bo[lo + 1] && P.ok && n_main <= kFanMaxNodes;
    // the tangent line, as the creeping path computes its attachment point
    const double a = P.a, idT = grcp(P.dT);
    const double cgT = a * idT, sgT = P.sI0 * idT;
    const double c1 = P.eT[0] * cgT - (double)sgn * P.eT[1] * sgT, s1 = P.eT[1] * cgT + (double)sgn * P.eT[0] * sgT;
    const double xt = P.c[0] + a * c1, yt = P.c[1] + a * s1;
    const double zl0 = P.z0, zl1 = P.z0 + P.h;
    FanGeo F;
    F.tx = L.T[0]; F.ty = L.T[1]; F.tz = L.T[2];
    const double hx = xt - F.tx, hy = yt - F.ty;
    F.U = sqrt(hx * hx + hy * hy);
    ok = ok && F.U > 1e-9 && isfinite(F.U);
    F.dx = ok ? hx / F.U : 1.0; F.dy = ok ? hy / F.U : 0.0;
    const double ext = fmax(fmax(fmax(fabs(F.tx), fabs(F.ty)), fmax(fabs(F.tz), fabs(xt))),
                            fmax(fmax(fabs(yt), fabs(zl0)), fabs(zl1)));
    F.ds = 4e-6 * (1.0 + ext);
    F.zmin = zl0 - 1e-3;
    F.zmax = zl1 + 1e-3;
    // segments reaching outside the scene box walk the boundary tree too:
    // those fans are not profiled
    if (ok && nodes && L.broot >= 0) {
        auto inb = [&](double x, double y, double z) {
            const float fx = (float)x, fy = (float)y, fz = (float)z;
            return fx >= L.blo[0] && fx <= L.bhi[0] && fy >= L.blo[1] && fy <= L.bhi[1] && fz >= L.blo[2] &&
                   fz <= L.bhi[2];
        };
        ok = inb(F.tx, F.ty, F.tz) && inb(xt, yt, zl0) && inb(xt, yt, zl1);
    }
    if (!ok) {
        if (lane == 0) out->n = -1;
        return;
    }
    float4* cuts = s_cut[w];
    int* ncut = &s_n[w];
    bool good = true;
    if (nodes) {
        // leaves of the main tree whose boxes meet the fan's box, the nodes
        // strided over the lanes
        const float pad = (float)F.ds;
        const float bx0 = (float)fmin(F.tx, xt) - pad, bx1 = (float)fmax(F.tx, xt) + pad;
        const float by0 = (float)fmin(F.ty, yt) - pad, by1 = (float)fmax(F.ty, yt) + pad;
        const float bz0 = (float)fmin(F.tz, zl0) - pad, bz1 = (float)fmax(F.tz, zl1) + pad;
        for (int nd = lane; nd < n_main && good; nd += 64) {
            const float4 q0 = nodes[4 * nd], q1 = nodes[4 * nd + 1], q2 = nodes[4 * nd + 2];
            const int4 q3 = *reinterpret_cast<const int4*>(&nodes[4 * nd + 3]);
            for (int c = 0; c < 2 && good; ++c) {
                const int first = c ? q3.z : q3.x, cnt = c ? q3.w : q3.y;
                if (first < 0 || cnt <= 0) continue;           // empty or an inner child
                const float lx = c ? q1.z : q0.x, ly = c ? q1.w : q0.y, lz = c ? q2.x : q0.z;
                const float ux = c ? q2.y : q0.w, uy = c ? q2.z : q1.x, uz = c ? q2.w : q1.y;
                if (!(lx <= bx1 && ux >= bx0 && ly <= by1 && uy >= by0 && lz <= bz1 && uz >= bz0)) continue;
                for (int t = first; t < first + cnt && good; ++t)
                    good = fan_triangle(F, cuts, ncut, tris[3 * t], tris[3 * t + 1], tris[3 * t + 2]);
            }
        }
    }
    if (L.bodies_occlude)
        for (int64_t j = bo[lo] + lane; j < bo[lo + 1] && good; j += 64)
            if (j != g) good = fan_cylinder(F, cuts, ncut, cyl + 5 * j);
    if (!good) atomicOr(&s_bad[w], 1);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const int nc = s_n[w];
    if (s_bad[w] || nc > kFanCuts) {
        if (lane == 0) out->n = -1;
        return;
    }
    // breakpoints: the four margin edges of every cut, within the line's
    // heights widened by a little
    const float za = (float)zl0 - 1e-3f, zb = (float)zl1 + 1e-3f;
    float* bp = s_bp[w];
    const int nb = 4 * nc + 2;
    for (int i = lane; i < nb; i += 64) {
        float v;
        if (i >= 4 * nc) {
            v = i == 4 * nc ? za : zb;
        } else {
            const float4 q = cuts[i >> 2];
            const int e = i & 3;
            v = e == 0 ? q.x - q.z : (e == 1 ? q.x + q.z : (e == 2 ? q.y - q.w : q.y + q.w));
        }
        bp[i] = fminf(fmaxf(v, za), zb);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    // sort by rank (ties broken by index)
    float* srt = s_srt[w];
    for (int i = lane; i < nb; i += 64) {
        const float v = bp[i];
        int r = 0;
        for (int j = 0; j < nb; ++j) r += (bp[j] < v || (bp[j] == v && j < i)) ? 1 : 0;
        srt[r] = v;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    // status of every gap between consecutive breakpoints, at its middle
    int* st = s_st[w];
    for (int i = lane; i + 1 < nb; i += 64) {
        const float z = 0.5f * (srt[i] + srt[i + 1]);
        bool blk = false, und = false;
        for (int c = 0; c < nc; ++c) {
            const float4 q = cuts[c];
            blk |= z > q.x + q.z && z < q.y - q.w;
            und |= fabsf(z - q.x) <= q.z || fabsf(z - q.y) <= q.w;
        }
        st[i] = blk ? kFanBlocked : (und ? kFanUndecided : kFanFree);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (lane == 0) {
        // runs: consecutive gaps of one status merged (empty gaps skipped)
        int nr = 0, cur = -1;
        float2 run[kFanRuns];
        bool over = false;
        for (int i = 0; i + 1 < nb; ++i) {
            if (!(srt[i + 1] > srt[i])) continue;
            if (st[i] == cur) {
                run[nr - 1].x = srt[i + 1];
            } else if (nr < kFanRuns) {
                run[nr++] = make_float2(srt[i + 1], (float)st[i]);
                cur = st[i];
            } else {
                over = true;
            }
        }
        if (over || nr == 0) {
            out->n = -1;
        } else {
            out->z0 = srt[0];
            for (int i = 0; i < nr; ++i) out->run[i] = run[i];
            out->n = nr;
        }
    }
}

// One block of kGridN^2 threads per frame (grid-stride): the grid of the
// frame's cylinders (BodyGrid, utd_bvh.h) and the receiver flags that are the
// same for the whole frame (source inside a cylinder, an invalid cylinder),
// with the invalid-body input bit raised for a frame that has receivers.
__global__ void __launch_bounds__(kGridN * kGridN) k_batch_grid(BatchParams B, const float* __restrict__ cyl,
                                                                const int64_t* __restrict__ bo,
                                                                const int64_t* __restrict__ ro,
                                                                BodyGrid* __restrict__ grids) {
    __shared__ float s_box[4];
    __shared__ int s_ff;
    const d3 T = mk(B.L.T[0], B.L.T[1], B.L.T[2]);
    for (int64_t fr = blockIdx.x; fr < B.n_frames; fr += gridDim.x) {
        const int64_t b0 = bo[fr], nb = bo[fr + 1] - b0;
        if (threadIdx.x == 0) s_ff = 0;
        grid_build_block(grids + fr, nullptr, 0, cyl + 5 * b0, nb, s_box);
        __syncthreads();
        LaunchParams L = B.L;
        L.n_sph = 0;
        L.n_cyl = (int)nb;
        int ff = 0;
        for (int64_t j = threadIdx.x; j < nb; j += blockDim.x) {
            if (inside_raw(L, nullptr, cyl + 5 * b0, (int)j, T)) ff |= kFlagTxInside;
            if (body_params_bad(nullptr, 0, cyl + 5 * b0, (int)j)) ff |= kFlagBadBody;
        }
        if (ff) atomicOr(&s_ff, ff);
        __syncthreads();
        if (threadIdx.x == 0) {
            grids[fr].fflags = s_ff;
            report_bad((s_ff & kFlagBadBody) && ro[fr + 1] > ro[fr], kBadBody);
        }
        __syncthreads();   // s_ff is cleared for the next frame
    }
}

// seg_blocked of the batched kernel: the frame's cylinders through its grid.
__device__ __forceinline__ bool seg_blocked_frame(d3 P0, d3 P1, const LaunchParams& L, const float* cyl, int skip,
                                                  bool bodies, const BodyGrid* G, const float4* nodes,
                                                  const float4* tris, int* stack, int stride) {
    if (bodies && blocked_by_grid(P0, P1, nullptr, 0, cyl, L.n_cyl, skip, G)) return true;
    return seg_blocked(P0, P1, L, nullptr, cyl, skip, false, nodes, tris, stack, stride);
}

__device__ __forceinline__ int64_t uniform64(int64_t v) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// One work item = one frame's tile of TILE receivers (one lane each).  Its
// bodies are taken in groups of kBGroup; per group:
//   1. cull: per body, every lane checks whether its receiver's height can
//      see the lateral surface at all; the passing (lane, body) pairs go to
//      an LDS queue, kPGroup bodies at a time;
//   2. candidates: the queued pairs are classified one per lane (which paths
//      exist: geometry and, for the reflection, the FP64 point solve), one
//      key per candidate into a second LDS queue (receiver lane, body in
//      group, path bit); reflection angles go to the work item's scratch;
//   3. visibility: whenever another chunk's candidates might not fit, and
//      after the last one, all lanes drain the candidate queue, one candidate
//      each (legs against the frame's other bodies and the BVH), and set
//      visible bits in the group's LDS masks -- so classification and
//      traversal run with every lane busy however sparse the pairs are;
//   4. field: every lane walks its receiver's visible paths of the group,
//      bodies and paths in order, at every frequency, adding to E in place.
constexpr int kBGroup = 32;
constexpr int kPGroup = 16;   // bodies per cull sub-group (LDS pair queue of kPGroup x TILE)

// The Fock tables are read through the caches here, not staged in LDS: the
// 20 KB of LDS they would take is what lets three workgroups of 256 share a
// CU (measured 9 % faster on the crowd than two with the tables in LDS).
template <typename R> struct GlobalTabs;
template <> struct GlobalTabs<float> {
    static __device__ __forceinline__ Tabs<float> get() { return Tabs<float>{&ft_f32_reg[0][0][0], &ft_f32_tf[0][0][0]}; }
};
template <> struct GlobalTabs<double> {
    static __device__ __forceinline__ Tabs<double> get() {
        return Tabs<double>{&ft_f64_reg[0][0][0], &ft_f64_tf[0][0][0]};
    }
};

// Receiver flags and the direct rays' visibility of every receiver, in the
// persistent kernel's tile order (sorted receivers: neighbouring lanes walk
// the same BVH nodes).  Kept out of k_batch, whose registers are taken by the
// path stages: here the walks run at six waves per SIMD (measured 1.3 ms
// less in k_batch for 0.8 ms here on the crowd).  Each lane writes its
// receiver's flags (inside, source inside, invalid receiver, bad body, bad
// frequency, line of sight) to fl, which k_batch reads.
template <int TILE>
__global__ void __launch_bounds__(TILE) k_batch_los(BatchParams B, const float* __restrict__ rx,
                                                    const float* __restrict__ cyl, const FreqConst* __restrict__ fcs,
                                                    const int64_t* __restrict__ bo, const int64_t* __restrict__ ro,
                                                    const int64_t* __restrict__ tile_off, const int* __restrict__ perm,
                                                    const BodyGrid* __restrict__ grids,
                                                    const float4* __restrict__ nodes, const float4* __restrict__ tris,
                                                    uint8_t* __restrict__ fl) {
    __shared__ int stack[kStackDepth * TILE];
    int* stk = stack + threadIdx.x;
    const int64_t total = tile_off[B.n_frames];
    const d3 T = mk(B.L.T[0], B.L.T[1], B.L.T[2]);
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int64_t lo = 0, hi = B.n_frames;
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if (tile_off[mid] <= t) lo = mid; else hi = mid;
        }
        const int64_t r0 = ro[lo], r1 = ro[lo + 1];
        const int64_t li = (t - tile_off[lo]) * TILE + threadIdx.x;
        if (r0 + li >= r1) continue;
        const int src = perm[r0 + li];
        if (src < 0 || src >= r1 - r0) continue;
        const int64_t i = r0 + src;
        LaunchParams L = B.L;
        L.n_sph = 0;
        L.n_cyl = (int)(bo[lo + 1] - bo[lo]);
        L.n_rx = r1 - r0;
        const float* fcyl = cyl + 5 * bo[lo];
        const d3 R3 = mk(rx[3 * i], rx[3 * i + 1], rx[3 * i + 2]);
        // receiver_flags, with the frame-uniform part from k_batch_grid and
        // the inside test on the cylinders of the receiver's grid cells (all
        // of them without a grid or with an invalid cylinder in the frame)
        const BodyGrid* G = grids + lo;
        uint8_t f = (uint8_t)G->fflags;
        const bool bad_rx = !finite3(R3);
        report_bad(bad_rx, kBadRx);
        bool inside = false;
        if (!bad_rx) {
            if (G->ok && !(f & kFlagBadBody) && L.n_cyl <= 64) {
                uint64_t m = grid_candidates(G, L.n_cyl, R3, R3);
                while (m && !inside) {
                    const int b = __builtin_ctzll(m);
                    m &= m - 1ull;
                    inside = inside_raw(L, nullptr, fcyl, b, R3);
                }
            } else {
                for (int b = 0; b < L.n_cyl && !inside; ++b) inside = inside_raw(L, nullptr, fcyl, b, R3);
            }
        }
        f |= (inside ? kFlagInside : 0) | (bad_rx ? kFlagInvalidRx : 0);
        for (int j = 0; j < L.n_f; ++j)
            if (!fcs[j].ok) f |= kFlagBadFreq;
        if (!(f & kFlagDead) && !seg_blocked_frame(T, R3, L, fcyl, -1, true, grids + lo, nodes, tris, stk, TILE))
            f |= kFlagLos;
        fl[i] = f;
    }
}

template <typename R, int TILE>
__global__ void __launch_bounds__(TILE) __attribute__((amdgpu_waves_per_eu(3, 8))) k_batch(BatchParams B, const float* __restrict__ rx,
                                                const float* __restrict__ cyl, const BodyPrep* __restrict__ prep,
                                                const FreqConst* __restrict__ fcs, const int64_t* __restrict__ bo,
                                                const int64_t* __restrict__ ro, const int64_t* __restrict__ tile_off,
                                                unsigned* __restrict__ counter, const float4* __restrict__ nodes,
                                                const float4* __restrict__ tris, double* __restrict__ th_scratch,
                                                const int* __restrict__ perm, R* __restrict__ ew_scratch,
                                                const FanProfile* __restrict__ fans,
                                                const BodyGrid* __restrict__ grids,
                                                const uint8_t* __restrict__ flw, R* __restrict__ E_out,
                                                uint8_t* __restrict__ flags) {
    static_assert(TILE <= 256, "lane index is stored in 8 bits");
    constexpr int QCAP = 8 * TILE;
    __shared__ int stack[kStackDepth * TILE];
    __shared__ unsigned int s_mask[kBGroup * TILE / 4];   // bytes [body in group][lane]
    __shared__ uint32_t s_q[QCAP];
    __shared__ uint16_t s_pq[kPGroup * TILE];             // queued (lane, body) pairs
    __shared__ int s_qn, s_qr, s_pn;   // creeping / reflection candidates, queued pairs
    __shared__ float s_box[TILE / 64][6];                 // per wavefront: its live receivers' box
    __shared__ uint32_t s_tmask;                          // bodies of the group the tile's box can reach
    __shared__ int64_t s_tile;
    __shared__ float s_rx[3][TILE];                       // the tile's receivers
    const Tabs<R> tb = GlobalTabs<R>::get();
    uint8_t* mask8 = reinterpret_cast<uint8_t*>(s_mask);
    double* thb = th_scratch + (int64_t)blockIdx.x * kBGroup * TILE;
    // the tile's field, [frequency][component][lane] complex, read and
    // written by its own lane only; without scratch (many frequencies) the
    // lane accumulates in place in E
    R* const Ews = ew_scratch ? ew_scratch + (int64_t)blockIdx.x * 2 * 3 * B.L.n_f * TILE : nullptr;
    int* stk = stack + threadIdx.x;
    const int tid = threadIdx.x;
    const int n_creep = 2 * (B.L.l_enc + 1);
    const int per_pair = n_creep + 1;
    const int64_t total = tile_off[B.n_frames];
    const d3 T = mk(B.L.T[0], B.L.T[1], B.L.T[2]);
    for (;;) {
        if (tid == 0) s_tile = (int64_t)atomicAdd(counter, 1u);
        __syncthreads();
        // the tile index is workgroup-uniform: keep it (and everything derived
        // from it: frame, offsets, body constants) in scalar registers
        const int64_t t = uniform64(s_tile);
        __syncthreads();
        if (t >= total) break;
        // frame: the last f with tile_off[f] <= t (empty frames are skipped)
        int64_t lo = 0, hi = B.n_frames;
        while (hi - lo > 1) {
            int64_t mid = (lo + hi) >> 1;
            if (tile_off[mid] <= t) lo = mid; else hi = mid;
        }
        const int64_t fr = lo;
        const int64_t r0 = ro[fr], r1 = ro[fr + 1];
        const int64_t lbase = (t - tile_off[fr]) * TILE;      // first receiver of the tile (in the frame)
        const int64_t li = lbase + tid;                     // sorted position in the frame
        // the receiver at that position (frame-local index); the sort makes
        // perm a permutation of [0, r1 - r0), the check only guards memory
        int src = 0;
        bool act = r0 + li < r1;
        if (act) {
            src = perm[r0 + li];
            act = src >= 0 && src < r1 - r0;
        }
        const int64_t b0 = bo[fr];
        LaunchParams L = B.L;
        L.n_sph = 0;
        L.n_cyl = (int)(bo[fr + 1] - b0);
        L.n_rx = r1 - r0;
        const int nbf = L.n_cyl;
        const float* fcyl = cyl + 5 * b0;
        const BodyPrep* fprep = prep + b0;
        const FanProfile* ffan = fans + 2 * b0;
        const BodyGrid* fgrid = grids + fr;
        R* E = E_out + 2 * 3 * (int64_t)B.L.n_f * r0;
        const int64_t i = r0 + src;
        const float rxx = act ? rx[3 * i] : 0.0f, rxy = act ? rx[3 * i + 1] : 0.0f, rxz = act ? rx[3 * i + 2] : 0.0f;
        const d3 R3 = mk(rxx, rxy, rxz);
        // read by other lanes after the group loop's first barrier; the
        // previous tile's last read was before its last barrier
        s_rx[0][tid] = rxx; s_rx[1][tid] = rxy; s_rx[2][tid] = rxz;
        // field accumulator of this lane: entry jc = 3 j + c at Ew[2 (jc es + ec)]
        R* const Ew = Ews ? Ews : E;
        const int64_t es = Ews ? TILE : L.n_rx, ec = Ews ? tid : src;

        // --- flags and direct ray (from k_batch_los), E initialisation ------
        bool dead = true;
        uint8_t fl = 0;
        if (act) {
            fl = flw[i];
            dead = (fl & kFlagDead) != 0;
            const bool los = (fl & kFlagLos) != 0;
            R e3[3] = {(R)0, (R)0, (R)0};
            double sd = 0.0;
            const bool use_los = los && L.lit_branch;
            if (use_los) {
                d3 v = mk(R3.x - T.x, R3.y - T.y, R3.z - T.z);
                sd = norm(v);
                R isd = (R)(1.0 / sd);
                R shx = (R)v.x * isd, shy = (R)v.y * isd, shz = (R)v.z * isd;
                R px = (R)L.p[0], py = (R)L.p[1], pz = (R)L.p[2];
                R pd = px * shx + py * shy + pz * shz;
                R A = (R)L.amp * isd;
                e3[0] = A * (px - pd * shx); e3[1] = A * (py - pd * shy); e3[2] = A * (pz - pd * shz);
            }
#pragma unroll 1
            for (int j = 0; j < L.n_f; ++j) {
                cplx<R> ph{(R)0, (R)0};
                if (use_los && fcs[j].ok) ph = phase_rev<R>(fcs[j].rev_per_m * sd);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int64_t o = (int64_t)(j * 3 + c) * es + ec;
                    Ew[2 * o] = (R)0 + e3[c] * ph.re;
                    Ew[2 * o + 1] = (R)0 + e3[c] * ph.im;
                }
            }
        }

        // box of the tile's live receivers (for the per-group body cull)
        {
            const bool live = act && !dead;
            float v[6] = {live ? rxx : INFINITY, live ? rxy : INFINITY, live ? rxz : INFINITY,
                          live ? rxx : -INFINITY, live ? rxy : -INFINITY, live ? rxz : -INFINITY};
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    const float o = __shfl_xor(v[k], off);
                    v[k] = k < 3 ? fminf(v[k], o) : fmaxf(v[k], o);
                }
            if ((tid & 63) == 0)
#pragma unroll
                for (int k = 0; k < 6; ++k) s_box[tid >> 6][k] = v[k];
        }
        __syncthreads();

        for (int g0 = 0; g0 < nbf; g0 += kBGroup) {
            const int ng = nbf - g0 < kBGroup ? nbf - g0 : kBGroup;
            for (int k = tid; k < kBGroup * TILE / 4; k += TILE) s_mask[k] = 0u;
            if (tid == 0) { s_qn = 0; s_qr = 0; }
            // the group's bodies that some live receiver of the tile may reach
            if (tid < 64) {
                float blo[3] = {INFINITY, INFINITY, INFINITY}, bhi[3] = {-INFINITY, -INFINITY, -INFINITY};
                for (int w = 0; w < TILE / 64; ++w)
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        blo[k] = fminf(blo[k], s_box[w][k]);
                        bhi[k] = fmaxf(bhi[k], s_box[w][3 + k]);
                    }
                const bool any_live = blo[0] <= bhi[0];
                const bool okb = any_live && tid < ng && cyl_box_possible(fprep[g0 + tid], blo, bhi, T, L);
                const uint64_t bm = __ballot(okb);
                if (tid == 0) s_tmask = (uint32_t)bm;
            }
            __syncthreads();
            // --- 3. visibility: the queued candidates, one per lane (legs
            // against the frame's other bodies and the BVH); visible bits go
            // to the group's LDS masks and the queue is emptied
            // Creeping candidates fill the queue from the front, reflections
            // from the back, so most wavefronts hold one kind (one branch).
            auto drain = [&](int qn, int qr) {
                for (int kq = tid; kq < qn + qr; kq += TILE) {
                    const uint32_t key = s_q[kq < qn ? kq : QCAP - qr + (kq - qn)];
                    const int lane = (int)(key & 0xffu), blk = (int)((key >> 8) & 0x1fu), bit = (int)(key >> 13);
                    const d3 R2 = mk(s_rx[0][lane], s_rx[1][lane], s_rx[2][lane]);
                    const int b = g0 + blk;
                    const BodyPrep P = fprep[b];
                    PathPts pts;
                    if (bit == kBitRefl) {
                        // a cylinder's reflection point needs only the angle
                        // (no receiver geometry)
                        d3 Q, n3;
                        refl_point<double, Kinds::Cylinders>(P, RxGeo{}, R2, T, thb[blk * TILE + lane], &Q, &n3);
                        pts.P0 = T; pts.P1 = Q; pts.P2 = Q; pts.P3 = R2;
                    } else {
                        RxGeo g = rx_geo<double, Kinds::Cylinders>(P, R2);
                        cyl_creep<R, double>(P, g, R2, T, L, (bit & 1) ? -1 : 1, bit >> 1,
                                             (PathEval<R>*)nullptr, &pts);
                    }
                    // a creeping path's source-side leg: the frame's profile of
                    // its (body, side) decides unless the height is undecided
                    bool vis = true;
                    int leg = 0;
                    if (bit != kBitRefl) {
                        const int fv = fan_lookup(ffan + 2 * b + (bit & 1), pts.P1.z);
                        vis = fv != 1;
                        leg = fv == 0 ? 1 : 0;
                    }
                    // a reflection tests its receiver-side leg first (the one
                    // more often blocked on the crowd: 1.5 % faster); the
                    // order does not change the decision
#pragma unroll 1
                    for (; leg < 2 && vis; ++leg) {
                        const int lg = bit == kBitRefl ? 1 - leg : leg;
                        d3 a = lg ? pts.P2 : pts.P0, c = lg ? pts.P3 : pts.P1;
                        vis = !seg_blocked_frame(a, c, L, fcyl, b, L.bodies_occlude != 0, fgrid, nodes, tris,
                                           stk, TILE);
                    }
                    if (vis) {
                        const int mb = blk * TILE + lane;
                        atomicOr(&s_mask[mb >> 2], (1u << bit) << (8 * (mb & 3)));
                    }
                }
                __syncthreads();
                if (tid == 0) { s_qn = 0; s_qr = 0; }
                __syncthreads();
            };
            // --- 1. cull: the (receiver, body) pairs whose heights can reach
            // the lateral surface, queued in LDS a sub-group of bodies at a
            // time, so the classification below runs with every lane busy
#pragma unroll 1
            for (int c0 = 0; c0 < ng; c0 += kPGroup) {
                const int nc = ng - c0 < kPGroup ? ng - c0 : kPGroup;
                if (tid == 0) s_pn = 0;
                __syncthreads();
                for (int bl = c0; bl < c0 + nc; ++bl) {
                    const bool ok = act && !dead && ((s_tmask >> bl) & 1u) && cyl_paths_possible(fprep[g0 + bl], R3, T, L);
                    if (ok) s_pq[atomicAdd(&s_pn, 1)] = (uint16_t)((uint32_t)tid | ((uint32_t)bl << 8));
                }
                __syncthreads();
                const int np = s_pn;
                // --- 2. classification of the queued pairs, TILE at a time:
                // candidate paths (geometry, reflection point) into the
                // candidate queue; drained whenever another chunk might not fit
#pragma unroll 1
                for (int base = 0; base < np; base += TILE) {
                    const int k = base + tid;
                    if (k < np) {
                        const uint32_t pk = s_pq[k];
                        const int lane = (int)(pk & 0xffu), bl = (int)(pk >> 8);
                        const d3 R2 = mk(s_rx[0][lane], s_rx[1][lane], s_rx[2][lane]);
                        const BodyPrep P = fprep[g0 + bl];
                        RxGeo g = rx_geo<double, Kinds::Cylinders>(P, R2);
                        uint32_t cand = 0;
                        for (int bit = 0; bit < n_creep; ++bit) {
                            PathPts pts;
                            if (cyl_creep<R, double>(P, g, R2, T, L, (bit & 1) ? -1 : 1, bit >> 1,
                                                     (PathEval<R>*)nullptr, &pts))
                                cand |= 1u << bit;
                        }
                        double th;
                        if (L.lit_branch && refl_angle<Kinds::Cylinders, (sizeof(R) == 8)>(P, g, R2, T, &th)) {
                            cand |= 1u << kBitRefl;
                            thb[bl * TILE + lane] = th;
                        }
                        const uint32_t key0 = (uint32_t)lane | ((uint32_t)bl << 8);
                        const uint32_t creep = cand & ((1u << kBitRefl) - 1u);
                        if (creep) {
                            int q = atomicAdd(&s_qn, __builtin_popcount(creep));
                            for (int bit = 0; bit < kBitRefl; ++bit)
                                if ((creep >> bit) & 1u) s_q[q++] = key0 | ((uint32_t)bit << 13);
                        }
                        if ((cand >> kBitRefl) & 1u)
                            s_q[QCAP - 1 - atomicAdd(&s_qr, 1)] = key0 | ((uint32_t)kBitRefl << 13);
                    }
                    __syncthreads();
                    // every wave reads the count before any wave appends more,
                    // so the drain decision is workgroup-uniform
                    const int qn = s_qn, qr = s_qr;
                    __syncthreads();
                    if (qn + qr > QCAP - TILE * per_pair) drain(qn, qr);
                }
            }
            // every write of the count was followed by a barrier
            const int qe = s_qn, qf = s_qr;
            if (qe + qf > 0) drain(qe, qf);
            // --- 4. field of this group's visible paths ---------------------
            // Each lane walks its own visible paths (creeping paths in
            // (body, bit) order, then the reflections), so a wavefront runs
            // as many iterations as its busiest lane: walking the bodies and
            // bits in lockstep would evaluate every (body, path kind) that
            // any of the 64 receivers has visible.
            if (act && !dead) {
                const uint32_t creep_sel = (1u << n_creep) - 1u;
#pragma unroll 1
                for (int pass = 0; pass < 2; ++pass) {
                    const uint32_t sel = pass == 0 ? creep_sel : (1u << kBitRefl);
                    int bl = 0;
                    uint32_t mrem = ng > 0 ? (mask8[tid] & sel) : 0u;
#pragma unroll 1
                    for (;;) {
                        while (mrem == 0u && bl < ng) {
                            ++bl;
                            if (bl < ng) mrem = mask8[bl * TILE + tid] & sel;
                        }
                        const bool have = bl < ng;
                        if (!__any(have)) break;
                        if (!have) continue;
                        const int bit = __builtin_ctz(mrem);
                        mrem &= mrem - 1u;
                        const BodyPrep P = fprep[g0 + bl];
                        PathEval<R> pe;
                        if (pass == 1) {
                            d3 Q, n3;
                            refl_point<double, Kinds::Cylinders>(P, RxGeo{}, R3, T, thb[bl * TILE + tid], &Q, &n3);
                            refl_eval<R, double>(P, Q, n3, R3, T, L, &pe);
                        } else {
                            RxGeo g = rx_geo<double, Kinds::Cylinders>(P, R3);
                            cyl_creep<R, double>(P, g, R3, T, L, (bit & 1) ? -1 : 1, bit >> 1, &pe, nullptr);
                        }
                        // Two frequencies per step: both loads first, then
                        // both evaluations, then both stores, so the memory
                        // latency of one overlaps the other's work (four per
                        // step measured slower: registers).  With an odd
                        // count the last step's second slot repeats the
                        // first unchanged and is stored before it.
#pragma unroll 1
                        for (int j = 0; j < L.n_f; j += 2) {
                            const bool two = j + 1 < L.n_f;
                            R e[2][6];
#pragma unroll
                            for (int u = 0; u < 2; ++u)
#pragma unroll
                                for (int c = 0; c < 3; ++c) {
                                    const int64_t o = (int64_t)((j + (two ? u : 0)) * 3 + c) * es + ec;
                                    e[u][2 * c] = Ew[2 * o];
                                    e[u][2 * c + 1] = Ew[2 * o + 1];
                                }
#pragma unroll
                            for (int u = 0; u < 2; ++u) {
                                const int jj = j + (two ? u : 0);
                                // an invalid frequency keeps its zero field
                                if ((u == 0 || two) && fcs[jj].ok) {
                                    FreqC<R> fc(fcs[jj]);
                                    if (pass == 0)
                                        add_path<R, kCreep>(pe, tb, fc, e[u]);
                                    else
                                        add_path<R, kRefl>(pe, tb, fc, e[u]);
                                }
                            }
#pragma unroll
                            for (int u = 1; u >= 0; --u)
#pragma unroll
                                for (int c = 0; c < 3; ++c) {
                                    const int64_t o = (int64_t)((j + (two ? u : 0)) * 3 + c) * es + ec;
                                    Ew[2 * o] = e[u][2 * c];
                                    Ew[2 * o + 1] = e[u][2 * c + 1];
                                }
                        }
                    }
                }
            }
            __syncthreads();      // masks, queue and angle scratch are reused by the next group
        }
        // the finished field and flags go to the receiver's own place
        if (act && Ews) {
#pragma unroll 1
            for (int jc = 0; jc < 3 * L.n_f; ++jc) {
                const int64_t o = (int64_t)jc * TILE + tid;
                const int64_t od = (int64_t)jc * L.n_rx + src;
                E[2 * od] = Ew[2 * o];
                E[2 * od + 1] = Ew[2 * o + 1];
            }
        }
        if (act && flags) flags[i] = fl;
    }
}

// Work-queue launch: the grid is persistent (blocks_per_cu x CUs workgroups).
template <typename R, int TILE>
static hipError_t launch_batch_tile(const BatchParams& B, int n_blocks, const float* rx, const float* cyl,
                                    const BatchWs& w, const float4* nodes, const float4* tris, void* E,
                                    uint8_t* flags, hipStream_t s) {
    hipLaunchKernelGGL((k_batch<R, TILE>), dim3(n_blocks), dim3(TILE), 0, s, B, rx, cyl, w.prep, w.fcs, w.bo, w.ro,
                       w.tile_off, w.counter, nodes, tris, w.th, w.perm, (R*)w.ew, w.fans, w.grids, w.flw, (R*)E,
                       flags);
    return hipGetLastError();
}

// The per-block field scratch is used while it stays below this size (it
// grows with the frequency count); above it the lanes accumulate in E.
constexpr size_t kBatchFieldScratchMax = (size_t)1 << 30;

size_t batch_workspace(const BatchParams& B, int precision, int n_blocks, char* base, BatchWs* ws) {
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t nf1 = (size_t)B.n_frames + 1;
    const size_t real = precision == 0 ? sizeof(float) : sizeof(double);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = up(o + bytes);
        return at;
    };
    const size_t o_prep = take(sizeof(BodyPrep) * (size_t)(B.n_cyl > 0 ? B.n_cyl : 1));
    const size_t o_fc = take(sizeof(FreqConst) * (size_t)(B.L.n_f > 0 ? B.L.n_f : 1));
    const size_t o_bo = take(sizeof(int64_t) * nf1);
    const size_t o_ro = take(sizeof(int64_t) * nf1);
    const size_t o_to = take(sizeof(int64_t) * nf1);
    const size_t o_cnt = take(256);
    const size_t o_key = take(sizeof(uint16_t) * (size_t)B.n_rx);
    const size_t o_perm = take(sizeof(int) * (size_t)B.n_rx);
    const size_t o_th = take(sizeof(double) * (size_t)n_blocks * kBGroup * B.tile);
    const size_t o_fan = take(sizeof(FanProfile) * 2 * (size_t)(B.n_cyl > 0 ? B.n_cyl : 1));
    const size_t o_grid = take(sizeof(BodyGrid) * (size_t)(B.n_frames > 0 ? B.n_frames : 1));
    const size_t o_flw = take((size_t)(B.n_rx > 0 ? B.n_rx : 1));
    const size_t ew_bytes = real * 2 * 3 * (size_t)B.L.n_f * (size_t)n_blocks * B.tile;
    const bool use_ew = ew_bytes <= kBatchFieldScratchMax;
    const size_t o_ew = take(use_ew ? ew_bytes : 0);
    if (base && ws) {
        ws->prep = (BodyPrep*)(base + o_prep);
        ws->fcs = (FreqConst*)(base + o_fc);
        ws->bo = (int64_t*)(base + o_bo);
        ws->ro = (int64_t*)(base + o_ro);
        ws->tile_off = (int64_t*)(base + o_to);
        ws->counter = (unsigned*)(base + o_cnt);
        ws->key = (uint16_t*)(base + o_key);
        ws->perm = (int*)(base + o_perm);
        ws->th = (double*)(base + o_th);
        ws->fans = (FanProfile*)(base + o_fan);
        ws->grids = (BodyGrid*)(base + o_grid);
        ws->flw = (uint8_t*)(base + o_flw);
        ws->ew = use_ew ? base + o_ew : nullptr;
    }
    return o;
}

hipError_t launch_batch(const BatchParams& B, int precision, int n_blocks, const int64_t* body_off,
                        const int64_t* rx_off, const float* rx, const float* cyl, const double* freqs,
                        const BatchWs& w, const float4* nodes, const float4* tris, int n_main, void* E,
                        uint8_t* flags, hipStream_t s, int part) {
    if (part != 2) {
        int64_t nwork = B.n_cyl > B.L.n_f ? B.n_cyl : B.L.n_f;
        int pb = (int)((nwork + 1023) / 1024);
        pb = pb < 1 ? 1 : (pb > 1024 ? 1024 : pb);
        hipLaunchKernelGGL(k_batch_prep, dim3(pb), dim3(1024), 0, s, B, body_off, rx_off, cyl, freqs, w.prep, w.fcs,
                           w.bo, w.ro, w.tile_off, w.counter);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const int sb = (int)(B.n_frames < 4096 ? B.n_frames : 4096);
        hipLaunchKernelGGL(k_batch_sort, dim3(sb), dim3(1024), 0, s, B, rx, w.ro, w.key, w.perm);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        const int gb = (int)(B.n_frames < 4096 ? B.n_frames : 4096);
        hipLaunchKernelGGL(k_batch_grid, dim3(gb), dim3(kGridN * kGridN), 0, s, B, cyl, w.bo, w.ro, w.grids);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (B.n_cyl > 0) {
            const unsigned fb = (unsigned)((2 * B.n_cyl + 3) / 4);
            hipLaunchKernelGGL(k_batch_fans, dim3(fb), dim3(256), 0, s, B, cyl, w.prep, w.bo, nodes, tris,
                               n_main, w.fans);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        // a block per tile up to 16384 blocks (grid-stride beyond): its own
        // occupancy, whatever the persistent kernel's workgroups per CU
        const int64_t ntile = B.n_rx / B.tile + B.n_frames + 1;
        const dim3 lg((unsigned)(ntile < 16384 ? ntile : 16384));
        switch (B.tile) {
            case 64:
                hipLaunchKernelGGL(k_batch_los<64>, lg, dim3(64), 0, s, B, rx, cyl, w.fcs, w.bo, w.ro, w.tile_off,
                                   w.perm, w.grids, nodes, tris, w.flw);
                break;
            case 128:
                hipLaunchKernelGGL(k_batch_los<128>, lg, dim3(128), 0, s, B, rx, cyl, w.fcs, w.bo, w.ro, w.tile_off,
                                   w.perm, w.grids, nodes, tris, w.flw);
                break;
            default:
                hipLaunchKernelGGL(k_batch_los<256>, lg, dim3(256), 0, s, B, rx, cyl, w.fcs, w.bo, w.ro, w.tile_off,
                                   w.perm, w.grids, nodes, tris, w.flw);
        }
        e = hipGetLastError();
        if (e != hipSuccess || part == 1) return e;
    }
    if (precision == 0) {
        switch (B.tile) {
            case 64: return launch_batch_tile<float, 64>(B, n_blocks, rx, cyl, w, nodes, tris, E, flags, s);
            case 128: return launch_batch_tile<float, 128>(B, n_blocks, rx, cyl, w, nodes, tris, E, flags, s);
            default: return launch_batch_tile<float, 256>(B, n_blocks, rx, cyl, w, nodes, tris, E, flags, s);
        }
    }
    switch (B.tile) {
        case 64: return launch_batch_tile<double, 64>(B, n_blocks, rx, cyl, w, nodes, tris, E, flags, s);
        case 128: return launch_batch_tile<double, 128>(B, n_blocks, rx, cyl, w, nodes, tris, E, flags, s);
        default: return launch_batch_tile<double, 256>(B, n_blocks, rx, cyl, w, nodes, tris, E, flags, s);
    }
}

}  // namespace utd
