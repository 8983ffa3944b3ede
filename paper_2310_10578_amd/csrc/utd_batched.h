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
//   k_batch        persistent: each workgroup takes the next (frame, tile of
//                  TILE receivers in sorted order) from an atomic work queue
//                  until the queue is empty.  A lane owns one receiver:
//                  inside / line-of-sight flags, then per body of its frame
//                  the path geometry, the visibility tests, and for each
//                  visible path the Fock evaluation of every frequency, added
//                  in place to the lane's column of the block's field scratch
//                  (initialised with the direct ray), which is copied to the
//                  receiver's own place in E when the tile is done.
//
// Neighbouring receivers have nearly the same paths: their candidate legs
// walk the same BVH nodes and meet the same bodies, so a wavefront of
// neighbours diverges far less than one of receivers scattered over the room
// (the crowd's receivers are uniform random; sorting them halves the time).
// The order changes nothing in any receiver's result: each receiver's field
// is computed by one lane, whatever lane that is.
//
// Fusing visibility and field keeps no per-path records (config-4 sized runs
// have ~2.7e8 receiver-body pairs); the per-receiver accumulation order is
// that of the single-frame kernels (direct ray, then bodies in order, paths
// in (ell, side) order, reflection last), so a frame gives the same field as
// utd_smooth_field on that frame up to floating-point contraction.
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

template <typename R, int TILE>
__global__ void __launch_bounds__(TILE) __attribute__((amdgpu_waves_per_eu(3, 8))) k_batch(BatchParams B, const float* __restrict__ rx,
                                                const float* __restrict__ cyl, const BodyPrep* __restrict__ prep,
                                                const FreqConst* __restrict__ fcs, const int64_t* __restrict__ bo,
                                                const int64_t* __restrict__ ro, const int64_t* __restrict__ tile_off,
                                                unsigned* __restrict__ counter, const float4* __restrict__ nodes,
                                                const float4* __restrict__ tris, double* __restrict__ th_scratch,
                                                const int* __restrict__ perm, R* __restrict__ ew_scratch,
                                                R* __restrict__ E_out, uint8_t* __restrict__ flags) {
    static_assert(TILE <= 256, "lane index is stored in 8 bits");
    constexpr int QCAP = 8 * TILE;
    __shared__ int stack[kStackDepth * TILE];
    __shared__ unsigned int s_mask[kBGroup * TILE / 4];   // bytes [body in group][lane]
    __shared__ uint32_t s_q[QCAP];
    __shared__ uint16_t s_pq[kPGroup * TILE];             // queued (lane, body) pairs
    __shared__ int s_qn, s_pn;
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

        // --- flags, direct ray, E initialisation ---------------------------
        bool dead = true;
        uint8_t fl = 0;
        if (act) {
            fl = receiver_flags(L, nullptr, fcyl, R3, T);
            for (int j = 0; j < L.n_f; ++j)
                if (!fcs[j].ok) fl |= kFlagBadFreq;
            dead = (fl & kFlagDead) != 0;
            const bool los = !dead && !seg_blocked(T, R3, L, nullptr, fcyl, -1, true, nodes, tris, stk, TILE);
            if (los) fl |= kFlagLos;
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

        for (int g0 = 0; g0 < nbf; g0 += kBGroup) {
            const int ng = nbf - g0 < kBGroup ? nbf - g0 : kBGroup;
            for (int k = tid; k < kBGroup * TILE / 4; k += TILE) s_mask[k] = 0u;
            if (tid == 0) s_qn = 0;
            __syncthreads();
            // --- 3. visibility: the queued candidates, one per lane (legs
            // against the frame's other bodies and the BVH); visible bits go
            // to the group's LDS masks and the queue is emptied
            auto drain = [&](int qn) {
                for (int kq = tid; kq < qn; kq += TILE) {
                    const uint32_t key = s_q[kq];
                    const int lane = (int)(key & 0xffu), blk = (int)((key >> 8) & 0x1fu), bit = (int)(key >> 13);
                    const d3 R2 = mk(s_rx[0][lane], s_rx[1][lane], s_rx[2][lane]);
                    const int b = g0 + blk;
                    const BodyPrep P = fprep[b];
                    RxGeo g = rx_geo<double, Kinds::Cylinders>(P, R2);
                    PathPts pts;
                    if (bit == kBitRefl) {
                        d3 Q, n3;
                        refl_point<double, Kinds::Cylinders>(P, g, R2, T, thb[blk * TILE + lane], &Q, &n3);
                        pts.P0 = T; pts.P1 = Q; pts.P2 = Q; pts.P3 = R2;
                    } else {
                        cyl_creep<R, double>(P, g, R2, T, L, (bit & 1) ? -1 : 1, bit >> 1,
                                             (PathEval<R>*)nullptr, &pts);
                    }
                    bool vis = true;
#pragma unroll 1
                    for (int leg = 0; leg < 2 && vis; ++leg) {
                        d3 a = leg ? pts.P2 : pts.P0, c = leg ? pts.P3 : pts.P1;
                        vis = !seg_blocked(a, c, L, nullptr, fcyl, b, L.bodies_occlude != 0, nodes, tris,
                                           stk, TILE);
                    }
                    if (vis) {
                        const int mb = blk * TILE + lane;
                        atomicOr(&s_mask[mb >> 2], (1u << bit) << (8 * (mb & 3)));
                    }
                }
                __syncthreads();
                if (tid == 0) s_qn = 0;
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
                    const bool ok = act && !dead && cyl_paths_possible(fprep[g0 + bl], R3, T, L);
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
                        if (cand) {
                            int q = atomicAdd(&s_qn, __builtin_popcount(cand));
                            for (int bit = 0; bit <= kBitRefl; ++bit)
                                if ((cand >> bit) & 1u)
                                    s_q[q++] = (uint32_t)lane | ((uint32_t)bl << 8) | ((uint32_t)bit << 13);
                        }
                    }
                    __syncthreads();
                    // every wave reads the count before any wave appends more,
                    // so the drain decision is workgroup-uniform
                    const int qn = s_qn;
                    __syncthreads();
                    if (qn > QCAP - TILE * per_pair) drain(qn);
                }
            }
            // every write of the count was followed by a barrier
            const int qe = s_qn;
            if (qe > 0) drain(qe);
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
                        RxGeo g = rx_geo<double, Kinds::Cylinders>(P, R3);
                        PathEval<R> pe;
                        if (pass == 1) {
                            d3 Q, n3;
                            refl_point<double, Kinds::Cylinders>(P, g, R3, T, thb[bl * TILE + tid], &Q, &n3);
                            refl_eval<R, double>(P, Q, n3, R3, T, L, &pe);
                        } else {
                            cyl_creep<R, double>(P, g, R3, T, L, (bit & 1) ? -1 : 1, bit >> 1, &pe, nullptr);
                        }
#pragma unroll 1
                        for (int j = 0; j < L.n_f; ++j) {
                            if (!fcs[j].ok) continue;     // an invalid frequency keeps its zero field
                            R e[6];
#pragma unroll
                            for (int c = 0; c < 3; ++c) {
                                const int64_t o = (int64_t)(j * 3 + c) * es + ec;
                                e[2 * c] = Ew[2 * o];
                                e[2 * c + 1] = Ew[2 * o + 1];
                            }
                            FreqC<R> fc(fcs[j]);
                            if (pass == 0)
                                add_path<R, kCreep>(pe, tb, fc, e);
                            else
                                add_path<R, kRefl>(pe, tb, fc, e);
#pragma unroll
                            for (int c = 0; c < 3; ++c) {
                                const int64_t o = (int64_t)(j * 3 + c) * es + ec;
                                Ew[2 * o] = e[2 * c];
                                Ew[2 * o + 1] = e[2 * c + 1];
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
                       w.tile_off, w.counter, nodes, tris, w.th, w.perm, (R*)w.ew, (R*)E, flags);
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
        ws->ew = use_ew ? base + o_ew : nullptr;
    }
    return o;
}

hipError_t launch_batch(const BatchParams& B, int precision, int n_blocks, const int64_t* body_off,
                        const int64_t* rx_off, const float* rx, const float* cyl, const double* freqs,
                        const BatchWs& w, const float4* nodes, const float4* tris, void* E, uint8_t* flags,
                        hipStream_t s, int part) {
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
