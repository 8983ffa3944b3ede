// HIP kernels of the smooth-surface UTD field evaluation (gfx950).
//
// Visibility and path constants (frequency independent):
//   k_setup / k_cand / k_vis / k_rec   scenes with triangles: candidate
//              paths per (receiver, body), queued; any-hit tests of their
//              legs; records of the visible ones
//   k_paths    scenes of bodies only: the same in one pass without a queue
// Both produce the per (receiver, body) mask bits (the U of Eqs. (1)-(2)),
// one record of frequency-independent constants per visible path, the
// receiver flags, and the body and frequency constants used later.
// Field:
//   k_field    per (receiver, frequency chunk) coherent field of Eqs. (1)-(4)
//   k_census   per-bit counts of the masks (measurement)
// The adjoint (utd_adjoint.h), the batched kernels (utd_batched.h), the
// wall bounce (utd_walls.h) and the uniform sum of a sphere's creeping-ray
// pairs at the axial caustic (utd_caustic.h) are included at the end.
//
// In k_field one lane owns one receiver and a chunk of FC frequencies; it
// walks the bodies in order, reads each valid path's record once and runs the
// Fock-coefficient evaluation for every frequency of the chunk, accumulating E
// in registers.  Frequency constants are uniform across the workgroup (scalar
// loads).  The Fock tables sit in LDS (FP32) or global memory (FP64).
#define FT_QUAL __device__ const __attribute__((aligned(16)))
#include <map>
#include <mutex>

#include "utd_internal.h"
#include "utd_bvh.h"
#include "utd_fock.h"
#include "utd_geom.h"

namespace utd {

// ---------------------------------------------------------------------------
// input status: bits (kBadRx, kBadBody, kBadFreq) raised by any call on this
// device since the host last read them (utd_input_status)
// ---------------------------------------------------------------------------
__device__ unsigned int g_input_status;

// Lanes that found an invalid input raise its bit; a plain read first keeps
// the atomics to the lanes that find the bit still clear.
__device__ __forceinline__ void report_bad(bool bad, unsigned bit) {
    if (bad && !(__atomic_load_n(&g_input_status, __ATOMIC_RELAXED) & bit)) atomicOr(&g_input_status, bit);
}

// ---------------------------------------------------------------------------
// frequency constants (an invalid frequency gets ok = 0 and harmless finite
// constants; its field is written as zero)
// ---------------------------------------------------------------------------
__device__ __forceinline__ FreqConst freq_const(double f_in) {
    const bool ok = isfinite(f_in) && f_in > 0.0;
    report_bad(!ok, kBadFreq);
    const double f = ok ? f_in : 1e9;
    double k = kTwoPi * f / kC0;
    double k13 = cbrt(k), k16 = sqrt(k13);
    FreqConst c;
    c.rev_per_m = f / kC0;
    c.kd = k; c.k13d = k13; c.k16d = k16; c.km16d = 1.0 / k16; c.skd = sqrt(k); c.ik13d = 1.0 / k13;
    c.iskd = 1.0 / c.skd;
    c.kf = (float)k; c.k13f = (float)k13; c.k16f = (float)k16; c.km16f = (float)(1.0 / k16);
    c.skf = (float)sqrt(k); c.ik13f = (float)(1.0 / k13); c.iskf = (float)c.iskd;
    c.ok = ok ? 1 : 0;
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

// Flags of receiver R3 that do not depend on visibility: inside a body,
// source inside a body, non-finite receiver, an invalid body in the call.
// Raises the matching input-status bits.
__device__ __forceinline__ uint8_t receiver_flags(const LaunchParams& L, const float* sph, const float* cyl, d3 R3,
                                                  d3 T) {
    const int nb = L.n_sph + L.n_cyl;
    const bool bad_rx = !finite3(R3);
    bool inside = false, tx_inside = false, bad_body = false;
    for (int k = 0; k < nb; ++k) {
        inside |= inside_raw(L, sph, cyl, k, R3);
        tx_inside |= inside_raw(L, sph, cyl, k, T);
        bad_body |= body_params_bad(sph, L.n_sph, cyl, k);
    }
    report_bad(bad_rx, kBadRx);
    report_bad(bad_body, kBadBody);
    return (uint8_t)((tx_inside ? kFlagTxInside : 0) | (inside ? kFlagInside : 0) | (bad_rx ? kFlagInvalidRx : 0) |
                     (bad_body ? kFlagBadBody : 0));
}

// ---------------------------------------------------------------------------
// visibility
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool blocked_by_bodies(d3 P0, d3 P1, const LaunchParams& L, const float* sph,
                                                  const float* cyl, int skip) {
    const SegF f = make_segf(P0, P1);
    for (int i = 0; i < L.n_sph; ++i)
        if (i != skip && seg_sphere(P0, P1, f, sph + 4 * i)) return true;
    for (int i = 0; i < L.n_cyl; ++i)
        if (L.n_sph + i != skip && seg_cylinder(P0, P1, f, cyl + 5 * i)) return true;
    return false;
}

__device__ __forceinline__ bool seg_blocked(d3 P0, d3 P1, const LaunchParams& L, const float* sph,
                                            const float* cyl, int skip, bool bodies, const float4* nodes,
                                            const float4* tris, int* stack, int stride) {
    if (bodies && blocked_by_bodies(P0, P1, L, sph, cyl, skip)) return true;
    if (!nodes) return false;
    SegRay r = make_ray(P0, P1);
    if (bvh_anyhit(nodes, tris, r, stack, stride)) return true;
    if (L.broot < 0) return false;
    // the boundary triangles lie in the faces of the scene box: a segment
    // with both (FP32) end points inside the closed box can meet them only
    // at an end point, which the open-segment test excludes
    const float ex = (float)P1.x, ey = (float)P1.y, ez = (float)P1.z;
    const bool in0 = r.ox >= L.blo[0] && r.ox <= L.bhi[0] && r.oy >= L.blo[1] && r.oy <= L.bhi[1] &&
                     r.oz >= L.blo[2] && r.oz <= L.bhi[2];
    const bool in1 = ex >= L.blo[0] && ex <= L.bhi[0] && ey >= L.blo[1] && ey <= L.bhi[1] && ez >= L.blo[2] &&
                     ez <= L.bhi[2];
    if (in0 && in1) return false;
    return bvh_anyhit(nodes, tris, r, stack, stride, L.broot);
}

// The same with the bodies through their grid (grid may be NULL).
__device__ __forceinline__ bool seg_blocked_g(d3 P0, d3 P1, const LaunchParams& L, const float* sph,
                                              const float* cyl, int skip, bool bodies, const BodyGrid* grid,
                                              const float4* nodes, const float4* tris, int* stack, int stride) {
    if (bodies && blocked_by_grid(P0, P1, sph, L.n_sph, cyl, L.n_cyl, skip, grid)) return true;
    return seg_blocked(P0, P1, L, sph, cyl, skip, false, nodes, tris, stack, stride);
}

// Path records: the frequency-independent constants of one valid path,
// written by the visibility pass and read by the field kernel.  Slot-major
// layout rec[(body * S + slot) * n_rx + rx] keeps both passes coalesced;
// S = 2 (l_enc + 1) + 1 slots per (receiver, body) pair, one per possible
// path: the creeping path of mask bit 2 ell + side in slot 2 ell + side, the
// reflection in the last slot.  Only the slots of set mask bits are written
// or read.
template <typename R> struct PathRec;
template <> struct PathRec<float> {          // 80 bytes (q0 and q1 aligned to 16)
    double s_tot;
    int16_t nc;                               // caustic quarter turns
    int16_t refl;
    float xh, uh, qhat;                       // see PathEval
    float4 q0;                                // (ixh, sxh, vs0, vs1)
    float4 q1;                                // (vs2, vh0, vh1, vh2)
    float iuh;
    float pad;
};
template <> struct PathRec<double> {         // 120 bytes
    double s_tot;
    int32_t nc, refl;
    double v[13];
};
static_assert(sizeof(PathRec<float>) == 80 && sizeof(PathRec<double>) == 120, "path record sizes");

__device__ __forceinline__ void pack(const PathEval<float>& p, PathRec<float>* r) {
    PathRec<float> o;
    o.s_tot = p.s_tot;
    o.nc = (int16_t)p.nc;
    o.refl = (int16_t)p.refl;
    o.xh = p.xh; o.uh = p.uh; o.qhat = p.qhat;
    o.q0 = make_float4(p.ixh, p.sxh, p.vs[0], p.vs[1]);
    o.q1 = make_float4(p.vs[2], p.vh[0], p.vh[1], p.vh[2]);
    o.iuh = p.iuh;
    o.pad = 0.0f;
    *r = o;
}
// The same with streaming (non-temporal) stores, for the single-pass
// bodies-only kernel: the field kernel that follows reads the record on
// whichever XCD takes its receiver, and lines left dirty in this XCD's L2
// would be written back at the kernel boundary, delaying the next launch.
// (The queue path's k_rec writes scattered records; there ordinary stores
// measured faster.)
__device__ __forceinline__ void pack_stream(const PathEval<float>& p, PathRec<float>* r) {
    PathRec<float> o;
    pack(p, &o);
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    const u32x4* src = reinterpret_cast<const u32x4*>(&o);
    u32x4* dst = reinterpret_cast<u32x4*>(r);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(PathRec<float>) / sizeof(u32x4)); ++k) __builtin_nontemporal_store(src[k], dst + k);
}
__device__ __forceinline__ void unpack(const PathRec<float>& o, PathEval<float>* p) {
    p->s_tot = o.s_tot;
    p->nc = o.nc;
    p->refl = o.refl;
    p->xh = o.xh; p->uh = o.uh; p->qhat = o.qhat;
    p->ixh = o.q0.x; p->sxh = o.q0.y; p->vs[0] = o.q0.z; p->vs[1] = o.q0.w;
    p->vs[2] = o.q1.x; p->vh[0] = o.q1.y; p->vh[1] = o.q1.z; p->vh[2] = o.q1.w;
    p->iuh = o.iuh;
}
__device__ __forceinline__ void pack(const PathEval<double>& p, PathRec<double>* r) {
    PathRec<double> o;
    o.s_tot = p.s_tot; o.nc = p.nc; o.refl = p.refl;
    double v[13] = {p.xh, p.uh, p.qhat, p.ixh, p.sxh, p.vs[0], p.vs[1], p.vs[2], p.vh[0], p.vh[1], p.vh[2],
                    p.iuh, 0.0};
    for (int k = 0; k < 13; ++k) o.v[k] = v[k];
    *r = o;
}
__device__ __forceinline__ void pack_stream(const PathEval<double>& p, PathRec<double>* r) { pack(p, r); }
__device__ __forceinline__ void unpack(const PathRec<double>& o, PathEval<double>* p) {
    p->s_tot = o.s_tot; p->nc = o.nc; p->refl = o.refl;
    p->xh = o.v[0]; p->uh = o.v[1]; p->qhat = o.v[2]; p->ixh = o.v[3]; p->sxh = o.v[4];
    p->vs[0] = o.v[5]; p->vs[1] = o.v[6]; p->vs[2] = o.v[7];
    p->vh[0] = o.v[8]; p->vh[1] = o.v[9]; p->vh[2] = o.v[10];
    p->iuh = o.v[11];
}

// Record slots per (receiver, body): one per possible path, creeping paths at
// their mask bit 2 ell + side, the reflection after them.
__device__ __forceinline__ int rec_slots(const LaunchParams& L) { return 2 * (L.l_enc + 1) + 1; }
__device__ __forceinline__ int rec_slot(const LaunchParams& L, int bit) {
    return bit == kBitRefl ? 2 * (L.l_enc + 1) : bit;
}

// ---------------------------------------------------------------------------
// Visibility in two passes.  Geometric validity is cheap and decided per
// (receiver, body) lane, but only a fraction of the pairs have valid paths
// (in a room with the source above the cylinder tops most helices leave the
// lateral surface), so the BVH traversal, the expensive part, runs over a
// compacted queue of candidate paths with every lane busy:
//   k_setup queue counters and the per-body constants.
//   k_cand  one lane per (receiver, body) pair (slot 0: the receiver's flags
//           and its direct ray): classification, path existence, reflection
//           point; appends one queue entry per candidate path (prefix sum
//           over the workgroup, one atomic per workgroup).
//   k_vis   one lane per queue entry: the path's legs against the other
//           bodies and the BVH; a visible path sets its mask bit and joins
//           the visible list.
//   k_rec   one lane per visible path: its record.
// The queue and list orders vary between runs; the outputs (mask bits,
// records, flags) do not.
// ---------------------------------------------------------------------------
constexpr uint64_t kLosEntry = 0xffffull;   // body field of a direct-ray entry

__device__ __forceinline__ uint64_t make_entry(int64_t i, int64_t b, int bit) {
    return (uint64_t)i | ((uint64_t)b << 32) | ((uint64_t)bit << 48);
}

// Exclusive prefix of cnt over a workgroup of 256 lanes plus one atomic per
// workgroup: wave prefixes, the four wave totals through LDS.  The counter is
// shared by the whole grid, so fewer atomics on it means less serialisation.
// Every lane of the workgroup must call it.
__device__ __forceinline__ int64_t block_append(int cnt, unsigned long long* counter) {
    __shared__ int s_wt[4];
    __shared__ unsigned long long s_base;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int x = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_wt[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int tot = s_wt[0] + s_wt[1] + s_wt[2] + s_wt[3];
        s_base = tot > 0 ? atomicAdd(counter, (unsigned long long)tot) : 0ull;
    }
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wave; ++w) before += s_wt[w];
    return (int64_t)s_base + before + x - cnt;
}

// Set-up of the two-pass visibility: queue and visible-list lengths, and the
// per-body constants (which depend on the source only).
__global__ void __launch_bounds__(256) k_setup(LaunchParams L, const float* __restrict__ sph,
                                               const float* __restrict__ cyl, BodyPrep* __restrict__ prep,
                                               unsigned long long* __restrict__ counter) {
    if (threadIdx.x == 0) {
        counter[0] = 0ull;
        counter[1] = 0ull;
    }
    const int nb = L.n_sph + L.n_cyl;
    for (int b = (int)(blockIdx.x * blockDim.x + threadIdx.x); b < nb; b += (int)(gridDim.x * blockDim.x))
        prep[b] = body_prep(L.T, sph, L.n_sph, cyl, b);
}

// Pass 1.  grid: x over receivers (blockDim 256), y over slot = 0 (receiver
// flags, direct ray) or 1 + body (constants from k_setup); the (0, 0) block
// stores the frequency constants.
template <typename R>
__global__ void __launch_bounds__(256) k_cand(LaunchParams L, const float* __restrict__ rx,
                                              const float* __restrict__ sph, const float* __restrict__ cyl,
                                              const double* __restrict__ freqs, const BodyPrep* __restrict__ prep,
                                              FreqConst* __restrict__ fcs, uint8_t* __restrict__ mask,
                                              uint8_t* __restrict__ flags, uint64_t* __restrict__ ent,
                                              double* __restrict__ ent_th, unsigned long long* __restrict__ counter,
                                              int64_t cap) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int slot = blockIdx.y;
    if (slot == 0 && blockIdx.x == 0 && freqs)
        for (int f = threadIdx.x; f < L.n_f; f += blockDim.x) fcs[f] = freq_const(freqs[f]);
    const bool in_range = i < L.n_rx;
    const d3 R3 = in_range ? mk(rx[3 * i], rx[3 * i + 1], rx[3 * i + 2]) : mk(0.0, 0.0, 0.0);
    const bool act = in_range && finite3(R3);
    const d3 T = mk(L.T[0], L.T[1], L.T[2]);
    const int nb = L.n_sph + L.n_cyl;
    uint8_t cand = 0;            // candidate bits (creeping 2 ell + side, reflection kBitRefl)
    bool los_cand = false;
    double th = 0.0;
    int b = slot - 1;
    if (slot == 0) {
        if (in_range) {
            flags[i] = receiver_flags(L, sph, cyl, R3, T);
            los_cand = !(flags[i] & kFlagDead);
        }
    } else {
        const BodyPrep P = prep[b];
        if (act && (P.kind == 0 || cyl_paths_possible(P, R3, T, L))) {
            RxGeo g = rx_geo(P, R3);
            uint8_t m = 0;
            for (int ell = 0; ell <= L.l_enc; ++ell) {
                for (int side = 0; side < 2; ++side) {
                    const int sgn = side == 0 ? 1 : -1;
                    PathPts pts;
                    bool ok, caus = false;
                    if (P.kind == 0)
                        ok = sphere_creep<R, double>(P, g, R3, T, L, sgn, ell, &caus, (PathEval<R>*)nullptr, &pts);
                    else
                        ok = cyl_creep<R, double>(P, g, R3, T, L, sgn, ell, (PathEval<R>*)nullptr, &pts);
                    if (caus) m |= (uint8_t)(1u << kBitCaustic);
                    if (ok) cand |= (uint8_t)(1u << (2 * ell + side));
                }
            }
            if (L.lit_branch && refl_angle<Kinds::Any, (sizeof(R) == 8)>(P, g, R3, T, &th)) cand |= (uint8_t)(1u << kBitRefl);
            mask[(int64_t)b * L.n_rx + i] = m;     // visible bits are added by k_vis
        } else if (in_range) {
            mask[(int64_t)b * L.n_rx + i] = 0;
        }
    }
    const int cnt = (los_cand ? 1 : 0) + __builtin_popcount(cand);
    int64_t q = block_append(cnt, counter);
    if (los_cand && q < cap) {
        ent[q] = make_entry(i, kLosEntry, 0);
        ent_th[q] = 0.0;
        ++q;
    }
    for (int bit = 0; bit <= kBitRefl; ++bit) {
        if (!((cand >> bit) & 1u)) continue;
        if (q < cap) {
            ent[q] = make_entry(i, b, bit);
            ent_th[q] = bit == kBitRefl ? th : 0.0;
        }
        ++q;
    }
}

// Pass 2: one lane per queue entry (grid-stride): the path's legs against
// the bodies and the BVH.  A visible path ORs its bit into the (rx, body)
// mask and joins the visible list; its record is written by pass 3.  Kept
// free of the record arithmetic so the traversal runs at higher occupancy.
template <typename R>
__device__ __forceinline__ void vis_body(const LaunchParams& L, const float* __restrict__ rx,
                                         const float* __restrict__ sph, const float* __restrict__ cyl,
                                         const BodyPrep* __restrict__ prep, const float4* __restrict__ nodes,
                                         const float4* __restrict__ tris, const uint64_t* __restrict__ ent,
                                         const double* __restrict__ ent_th, unsigned long long* __restrict__ counter,
                                         int64_t cap, uint8_t* __restrict__ mask, uint8_t* __restrict__ flags,
                                         uint64_t* __restrict__ vis_list, const BodyGrid* grid, int* stack,
                                         uint64_t* vbuf) {
    int* stk = stack + threadIdx.x;
    // Visible paths collect in the wavefront's own LDS buffer (vbuf, 128
    // entries) and go to the global list 64 at a time: one atomic on the
    // grid-wide counter per 64 visible paths instead of one per wavefront
    // and iteration.  The loop runs the same trip count on every lane of a
    // wavefront, so all 64 lanes take part in each buffer step.
    const int lane = threadIdx.x & 63;
    int nbuf = 0;                                     // wave-uniform
    const int stride = 256;
    int64_t total = (int64_t)counter[0];
    total = total < cap ? total : cap;
    const d3 T = mk(L.T[0], L.T[1], L.T[2]);
    const bool bo = L.bodies_occlude != 0;
    for (int64_t qw = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); qw < total;
         qw += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = qw + lane;
        bool vis = false;
        if (q < total) {
            const uint64_t en = ent[q];
            const int64_t i = (int64_t)(en & 0xffffffffu);
            const int64_t bb = (int64_t)((en >> 32) & 0xffffu);
            const int bit = (int)(en >> 48);
            const d3 R3 = mk(rx[3 * i], rx[3 * i + 1], rx[3 * i + 2]);
            if (bb == (int64_t)kLosEntry) {
                // the receiver's only entry of this kind: a plain byte update
                if (!seg_blocked_g(T, R3, L, sph, cyl, -1, true, grid, nodes, tris, stk, stride))
                    flags[i] = (uint8_t)(flags[i] | kFlagLos);
            } else {
                const int b = (int)bb;
                const BodyPrep P = prep[b];
                RxGeo g = rx_geo(P, R3);
                PathPts pts;
                if (bit == kBitRefl) {
                    d3 Q, n;
                    refl_point<double>(P, g, R3, T, ent_th[q], &Q, &n);
                    pts.P0 = T; pts.P1 = Q; pts.P2 = Q; pts.P3 = R3;
                } else {
                    const int ell = bit >> 1, sgn = (bit & 1) ? -1 : 1;
                    bool cz;
                    if (P.kind == 0)
                        sphere_creep<R, double>(P, g, R3, T, L, sgn, ell, &cz, (PathEval<R>*)nullptr, &pts);
                    else
                        cyl_creep<R, double>(P, g, R3, T, L, sgn, ell, (PathEval<R>*)nullptr, &pts);
                }
                vis = !seg_blocked_g(pts.P0, pts.P1, L, sph, cyl, b, bo, grid, nodes, tris, stk, stride);
                if (vis) vis = !seg_blocked_g(pts.P2, pts.P3, L, sph, cyl, b, bo, grid, nodes, tris, stk, stride);
                if (vis) {
                    // mask bytes of one pair can be set by concurrent lanes: OR into the word
                    const int64_t mb = (int64_t)b * L.n_rx + i;
                    atomicOr(reinterpret_cast<unsigned int*>(mask + (mb & ~(int64_t)3)),
                             (1u << bit) << (8 * (mb & 3)));
                }
            }
        }
        // all 64 lanes: buffer this iteration's visible paths
        const uint64_t bal = __ballot(vis);
        if (vis) vbuf[nbuf + __popcll(bal & ((1ull << lane) - 1ull))] = (uint64_t)q;
        nbuf += __popcll(bal);
        if (nbuf >= 64) {
            unsigned long long base = 0;
            if (lane == 0) base = atomicAdd(counter + 1, 64ull);
            base = __shfl(base, 0, 64);
            vis_list[base + lane] = vbuf[lane];
            const uint64_t rest = lane + 64 < nbuf ? vbuf[lane + 64] : 0ull;
            __builtin_amdgcn_wave_barrier();
            if (lane + 64 < nbuf) vbuf[lane] = rest;
            nbuf -= 64;
        }
    }
    if (nbuf > 0) {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(counter + 1, (unsigned long long)nbuf);
        base = __shfl(base, 0, 64);
        if (lane < nbuf) vis_list[base + lane] = vbuf[lane];
    }
}

// Four waves per SIMD (128 VGPRs, a few spills): more traversals in flight
// hide more of their memory latency (measured faster than three without
// spills).
template <typename R>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) k_vis(LaunchParams L, const float* __restrict__ rx,
                                             const float* __restrict__ sph, const float* __restrict__ cyl,
                                             const BodyPrep* __restrict__ prep, const float4* __restrict__ nodes,
                                             const float4* __restrict__ tris, const uint64_t* __restrict__ ent,
                                             const double* __restrict__ ent_th,
                                             unsigned long long* __restrict__ counter, int64_t cap,
                                             uint8_t* __restrict__ mask, uint8_t* __restrict__ flags,
                                             uint64_t* __restrict__ vis_list, const BodyGrid* __restrict__ grid) {
    __shared__ int stack[kStackDepth * 256];
    __shared__ uint64_t vbuf[4 * 128];
    vis_body<R>(L, rx, sph, cyl, prep, nodes, tris, ent, ent_th, counter, cap, mask, flags, vis_list, grid, stack,
                vbuf + 128 * (threadIdx.x >> 6));
}

// The grid of the call's bodies (one block; at most 64 bodies).
__global__ void __launch_bounds__(kGridN * kGridN) k_body_grid(LaunchParams L, const float* __restrict__ sph,
                                                               const float* __restrict__ cyl,
                                                               BodyGrid* __restrict__ grid) {
    __shared__ float s_box[4];
    grid_build_block(grid, sph, L.n_sph, cyl, L.n_cyl, s_box);
}

size_t body_grid_bytes() { return sizeof(BodyGrid); }

// Pass 3: one lane per visible path (grid-stride over the visible list): the
// frequency-independent constants of the path, packed into its record slot.
template <typename R>
__global__ void __launch_bounds__(256) k_rec(LaunchParams L, const float* __restrict__ rx,
                                             const BodyPrep* __restrict__ prep, const uint64_t* __restrict__ ent,
                                             const double* __restrict__ ent_th,
                                             const unsigned long long* __restrict__ counter,
                                             const uint64_t* __restrict__ vis_list, PathRec<R>* __restrict__ rec) {
    const int64_t n = (int64_t)counter[1];
    const d3 T = mk(L.T[0], L.T[1], L.T[2]);
    const int NS = rec_slots(L);
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = (int64_t)vis_list[k];
        const uint64_t en = ent[q];
        const int64_t i = (int64_t)(en & 0xffffffffu);
        const int b = (int)((en >> 32) & 0xffffu);
        const int bit = (int)(en >> 48);
        const d3 R3 = mk(rx[3 * i], rx[3 * i + 1], rx[3 * i + 2]);
        const BodyPrep P = prep[b];
        RxGeo g = rx_geo(P, R3);
        PathEval<R> pe;
        if (bit == kBitRefl) {
            d3 Q, n3;
            refl_point<double>(P, g, R3, T, ent_th[q], &Q, &n3);
            refl_eval<R, double>(P, Q, n3, R3, T, L, &pe);
        } else {
            const int ell = bit >> 1, sgn = (bit & 1) ? -1 : 1;
            bool cz;
            if (P.kind == 0)
                sphere_creep<R, double>(P, g, R3, T, L, sgn, ell, &cz, &pe, nullptr);
            else
                cyl_creep<R, double>(P, g, R3, T, L, sgn, ell, &pe, nullptr);
        }
        pack(pe, &rec[((int64_t)b * NS + rec_slot(L, bit)) * L.n_rx + i]);
    }
}

// Scenes of bodies only (no triangles): one pass, no queue.
// grid (ceil(n_rx / 64), max(bodies, 1)), 64 K threads, K = 2 (l_enc + 1) + 1
// path kinds; a workgroup covers 64 receivers of one body.  Wave k takes
// path kind k (creeping (ell, side) = (k >> 1, k & 1), the reflection for
// k = K - 1), so every wavefront runs one kind of path.  Each wave leaves its
// mask bits in its own LDS row; after the one barrier wave 0 merges the rows.
// Wave 0 of the body-0 workgroups (the side-+ creeping wave, which ends
// earliest: its path does not exist for lit receivers) then sets the
// receivers' inside / source-inside flags and tests the direct ray; wave 1 of
// workgroup (0, 0) converts the frequencies.  Every wavefront computes the
// body constants itself (the chains are latency-bound; waiting for one lane
// to share them costs more), after issuing its receiver load.
template <typename R>
__global__ void __launch_bounds__(512) k_paths(LaunchParams L, const float* __restrict__ rx,
                                               const float* __restrict__ sph, const float* __restrict__ cyl,
                                               const double* __restrict__ freqs, BodyPrep* __restrict__ prep,
                                               FreqConst* __restrict__ fcs, uint8_t* __restrict__ mask,
                                               PathRec<R>* __restrict__ rec, uint8_t* __restrict__ flags) {
    __shared__ unsigned s_m[8][64];
    const d3 T = mk(L.T[0], L.T[1], L.T[2]);
    const int nb = L.n_sph + L.n_cyl;
    const int b = blockIdx.y;
    const int lane = threadIdx.x & 63, kind = threadIdx.x >> 6;
    const int K = rec_slots(L);
    const int64_t i = (int64_t)blockIdx.x * 64 + lane;
    const bool have = i < L.n_rx;
    const d3 R3 = have ? mk(rx[3 * i], rx[3 * i + 1], rx[3 * i + 2]) : T;
    unsigned m = 0u;
    if (b < nb) {
        const BodyPrep P = body_prep(L.T, sph, L.n_sph, cyl, b);
        if (blockIdx.x == 0 && threadIdx.x == 0) prep[b] = P;
        const bool bo = L.bodies_occlude != 0;
        if (have && finite3(R3)) {
            RxGeo g = rx_geo(P, R3);
            if (kind < K - 1) {
                const int ell = kind >> 1, sgn = (kind & 1) ? -1 : 1;
                PathPts pts;
                bool ok, caus = false;
                if (P.kind == 0)
                    ok = sphere_creep<R, double>(P, g, R3, T, L, sgn, ell, &caus, (PathEval<R>*)nullptr, &pts);
                else
                    ok = cyl_creep<R, double>(P, g, R3, T, L, sgn, ell, (PathEval<R>*)nullptr, &pts);
                if (caus) m |= 1u << kBitCaustic;
                if (ok && !seg_blocked(pts.P0, pts.P1, L, sph, cyl, b, bo, nullptr, nullptr, nullptr, 0) &&
                    !seg_blocked(pts.P2, pts.P3, L, sph, cyl, b, bo, nullptr, nullptr, nullptr, 0)) {
                    m |= 1u << kind;
                    PathEval<R> pe;
                    bool cz;
                    if (P.kind == 0)
                        sphere_creep<R, double>(P, g, R3, T, L, sgn, ell, &cz, &pe, nullptr);
                    else
                        cyl_creep<R, double>(P, g, R3, T, L, sgn, ell, &pe, nullptr);
                    pack_stream(pe, &rec[((int64_t)b * K + rec_slot(L, kind)) * L.n_rx + i]);
                }
            } else {
                double th = 0.0;
                if (L.lit_branch && refl_angle<Kinds::Any, (sizeof(R) == 8)>(P, g, R3, T, &th)) {
                    d3 Q, n;
                    refl_point<double>(P, g, R3, T, th, &Q, &n);
                    if (!seg_blocked(T, Q, L, sph, cyl, b, bo, nullptr, nullptr, nullptr, 0) &&
                        !seg_blocked(Q, R3, L, sph, cyl, b, bo, nullptr, nullptr, nullptr, 0)) {
                        m |= 1u << kBitRefl;
                        PathEval<R> pe;
                        refl_eval<R, double>(P, Q, n, R3, T, L, &pe);
                        pack_stream(pe, &rec[((int64_t)b * K + rec_slot(L, kBitRefl)) * L.n_rx + i]);
                    }
                }
            }
        }
    }
    if (b == 0 && kind == (K > 1 ? 1 : 0) && blockIdx.x == 0 && freqs)
        for (int f = lane; f < L.n_f; f += 64) fcs[f] = freq_const(freqs[f]);
    if (b == 0 && kind == 0 && have) {
        uint8_t f = receiver_flags(L, sph, cyl, R3, T);
        if (!(f & kFlagDead) && !seg_blocked(T, R3, L, sph, cyl, -1, true, nullptr, nullptr, nullptr, 0))
            f |= kFlagLos;
        flags[i] = f;
    }
    if (b >= nb) return;   // the whole workgroup: no barrier below is skipped by part of it
    s_m[kind][lane] = m;
    __syncthreads();
    if (kind == 0 && have) {
        unsigned mm = 0u;
        for (int k = 0; k < K; ++k) mm |= s_m[k][lane];
        mask[(int64_t)b * L.n_rx + i] = (uint8_t)mm;
    }
}

// ---------------------------------------------------------------------------
template <typename R> struct FreqC;
template <> struct FreqC<float> {
    double rev_per_m;
    float kf, k13, k16, km16, sk, ik13, isk;
    __device__ __forceinline__ FreqC(const FreqConst& c)
        : rev_per_m(c.rev_per_m), kf(c.kf), k13(c.k13f), k16(c.k16f), km16(c.km16f), sk(c.skf), ik13(c.ik13f),
          isk(c.iskf) {}
};
template <> struct FreqC<double> {
    double rev_per_m;
    double kf, k13, k16, km16, sk, ik13, isk;
    __device__ __forceinline__ FreqC(const FreqConst& c)
        : rev_per_m(c.rev_per_m), kf(c.kd), k13(c.k13d), k16(c.k16d), km16(c.km16d), sk(c.skd), ik13(c.ik13d),
          isk(c.iskd) {}
};

// The soft and hard coefficients of one path at one frequency (its Fock
// kernels times its phase).  The Fock arguments scale with powers of k
// (xi ~ k^{1/3}, sqrt(X) ~ k^{1/2}, q ~ k^{1/6}), so they are products of the
// path's constants and the frequency's.  MODE picks the Fock specialisation
// (kCreep, kRefl or kAny for mixed wavefronts); callers branch on
// wave-uniform conditions.  Every diffracted term carries the factor
// k^{-1/6}; with KM16 = false it is left out, for callers that apply it once
// to their sum.
template <typename R, int MODE, bool KM16 = true>
__device__ __forceinline__ void path_coefs(const PathEval<R>& pe, const Tabs<R>& tb, const FreqC<R>& fc,
                                           cplx<R>* cs_out, cplx<R>* ch_out) {
    FockArgs<R> a;
    a.xi = fc.k13 * pe.xh;
    a.u = fc.sk * pe.uh;
    a.iu = fc.isk * pe.iuh;
    a.ixi = fc.ik13 * pe.ixh;
    a.h = (R)0.5 * fc.k16 * pe.sxh;
    // the path factors are the same for every frequency of the lane's chunk
    a.qc = fc.k16 * (pe.qhat * (R)-kC2E4);
    a.xc = fc.ik13 * (pe.ixh * (R)kC2E4);
    cplx<R> Ks, Kh;
    fock_kernel<R, MODE>(tb, a, pe.refl != 0, &Ks, &Kh);
    cplx<R> ph = phase_rev<R>(fc.rev_per_m * pe.s_tot - 0.25 * pe.nc);
    if (KM16) {
        ph.re *= fc.km16;
        ph.im *= fc.km16;
    }
    *cs_out = cmul(Ks, ph);
    *ch_out = cmul(Kh, ph);
}

// The path's field at one frequency: the coefficients times its
// polarisation vectors, accumulated into E[6] (x, y, z; re, im).
template <typename R, int MODE, bool KM16 = true>
__device__ __forceinline__ void add_path(const PathEval<R>& pe, const Tabs<R>& tb, const FreqC<R>& fc, R* E) {
    cplx<R> cs, ch;
    path_coefs<R, MODE, KM16>(pe, tb, fc, &cs, &ch);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        E[2 * c] = fma(cs.re, pe.vs[c], E[2 * c]);
        E[2 * c] = fma(ch.re, pe.vh[c], E[2 * c]);
        E[2 * c + 1] = fma(cs.im, pe.vs[c], E[2 * c + 1]);
        E[2 * c + 1] = fma(ch.im, pe.vh[c], E[2 * c + 1]);
    }
}

// The FP32 tables are copied into LDS once per workgroup: the generated
// arrays already have the LDS layout, so the copy is a straight 16-byte
// vector copy.  NT is the workgroup size the caller is launched with; the
// copy is unrolled to a fixed count per thread so that every lane issues all
// of its loads before the first LDS write (a plain strided loop waits for
// each load in turn, one L2 round trip per iteration).  The FP64 tables stay
// in global memory (L2 resident).
template <typename R> struct TableStage;

template <> struct TableStage<float> {
    using D = TabDims<float>;
    static constexpr int NREG = (D::NCL + D::NPT + D::NDS) * D::ROWS * 4;
    static constexpr int NTF = 2 * D::NT * D::ROWS * 2;
    static_assert(NREG % 4 == 0 && NTF % 4 == 0, "float4 copy");
    static_assert(sizeof(ft_f32_reg) == NREG * sizeof(float) && sizeof(ft_f32_tf) == NTF * sizeof(float),
                  "table layout");
    template <int NT>
    static __device__ __forceinline__ Tabs<float> stage(float* reg, float* tf) {
        constexpr int NA = NREG / 4, NB = NTF / 4;
        constexpr int RA = (NA + NT - 1) / NT, RB = (NB + NT - 1) / NT;
        const float4* a = reinterpret_cast<const float4*>(&ft_f32_reg[0][0][0]);
        const float4* b = reinterpret_cast<const float4*>(&ft_f32_tf[0][0][0]);
        float4* ra = reinterpret_cast<float4*>(reg);
        float4* rb = reinterpret_cast<float4*>(tf);
        const int t = threadIdx.x;
        // no branches (a branch lets the compiler sink each load to its store):
        // indices past the end are clamped to the last entry, so those lanes
        // load and store that entry's own value again
        float4 va[RA], vb[RB];
#pragma unroll
        for (int r = 0; r < RA; ++r) va[r] = a[t + r * NT < NA ? t + r * NT : NA - 1];
#pragma unroll
        for (int r = 0; r < RB; ++r) vb[r] = b[t + r * NT < NB ? t + r * NT : NB - 1];
#pragma unroll
        for (int r = 0; r < RA; ++r) ra[t + r * NT < NA ? t + r * NT : NA - 1] = va[r];
#pragma unroll
        for (int r = 0; r < RB; ++r) rb[t + r * NT < NB ? t + r * NT : NB - 1] = vb[r];
        __syncthreads();
        return Tabs<float>{reg, tf};
    }
};

template <> struct TableStage<double> {
    static constexpr int NREG = 1, NTF = 1;
    template <int NT>
    static __device__ __forceinline__ Tabs<double> stage(double*, double*) {
        return Tabs<double>{&ft_f64_reg[0][0][0], &ft_f64_tf[0][0][0]};
    }
};

// Receiver i at frequencies f0 .. f0 + FC - 1 (those below n_f).
template <typename R, int FC>
__device__ __forceinline__ void field_rx(const LaunchParams& L, const float* __restrict__ rx,
                                         const FreqConst* __restrict__ fcs, const uint8_t* __restrict__ mask,
                                         const PathRec<R>* __restrict__ rec, uint8_t* __restrict__ flags,
                                         R* __restrict__ E_out, const Tabs<R>& tb, int64_t i, int f0) {
    const int nfc = L.n_f - f0 < FC ? L.n_f - f0 : FC;
    const int NS = rec_slots(L);
    R E[FC][6];
#pragma unroll
    for (int j = 0; j < FC; ++j)
#pragma unroll
        for (int c = 0; c < 6; ++c) E[j][c] = (R)0;
    // frequencies of the chunk that are evaluated (an invalid one stays zero)
    bool fok[FC];
#pragma unroll
    for (int j = 0; j < FC; ++j) fok[j] = j < nfc && fcs[f0 + j].ok;
    uint8_t fl = flags[i];
    uint8_t fl_new = fl;
    if (f0 == 0)
        for (int f = 0; f < L.n_f; ++f)
            if (!fcs[f].ok) fl_new |= kFlagBadFreq;
    if (!(fl & kFlagDead)) {
        // diffracted and reflected paths, Eqs. (2)-(4), without their common
        // factor k^{-1/6} (applied once per frequency below)
        int nb = L.n_sph + L.n_cyl;
        uint8_t caus = 0;
        for (int b = 0; b < nb; ++b) {
            uint8_t m = mask[(int64_t)b * L.n_rx + i];
            caus |= m;
            const bool has_refl = (m >> kBitRefl) & 1u;
            // creeping paths in bit order, then the reflection
            uint32_t cb = m & ((1u << (2 * (L.l_enc + 1))) - 1u);
            while (cb) {
                const int k = __builtin_ctz(cb);
                cb &= cb - 1u;
                PathEval<R> pe;
                unpack(rec[((int64_t)b * NS + k) * L.n_rx + i], &pe);
#pragma unroll
                for (int j = 0; j < FC; ++j) {
                    if (fok[j]) {
                        FreqC<R> fc(fcs[f0 + j]);
                        add_path<R, kCreep, false>(pe, tb, fc, E[j]);
                    }
                }
            }
            if (__any(has_refl) && has_refl) {
                PathEval<R> pe;
                unpack(rec[((int64_t)b * NS + rec_slot(L, kBitRefl)) * L.n_rx + i], &pe);
#pragma unroll
                for (int j = 0; j < FC; ++j) {
                    if (fok[j]) {
                        FreqC<R> fc(fcs[f0 + j]);
                        add_path<R, kRefl, false>(pe, tb, fc, E[j]);
                    }
                }
            }
        }
        if (caus & (1u << kBitCaustic)) fl_new |= kFlagCaustic;
#pragma unroll
        for (int j = 0; j < FC; ++j) {
            if (fok[j]) {
                const R km16 = FreqC<R>(fcs[f0 + j]).km16;
#pragma unroll
                for (int c = 0; c < 6; ++c) E[j][c] *= km16;
            }
        }
        // direct field, Eq. (1): A (p - (p.s)s) e^{-jks}/s
        if ((fl & kFlagLos) && L.lit_branch) {
            d3 v = mk(rx[3 * i] - L.T[0], rx[3 * i + 1] - L.T[1], rx[3 * i + 2] - L.T[2]);
            // 1/s from grsqrt and s = |v|^2 / s: within an ulp, without the
            // library square root and a division
            const double d2v = dot(v, v), isd_d = grsqrt(d2v);
            const double sd = d2v * isd_d;
            R isd = (R)isd_d;
            R shx = (R)v.x * isd, shy = (R)v.y * isd, shz = (R)v.z * isd;
            R px = (R)L.p[0], py = (R)L.p[1], pz = (R)L.p[2];
            R pd = px * shx + py * shy + pz * shz;
            R A = (R)L.amp * isd;
            R e3[3] = {A * (px - pd * shx), A * (py - pd * shy), A * (pz - pd * shz)};
#pragma unroll
            for (int j = 0; j < FC; ++j) {
                if (fok[j]) {
                    cplx<R> ph = phase_rev<R>(fcs[f0 + j].rev_per_m * sd);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        E[j][2 * c] += e3[c] * ph.re;
                        E[j][2 * c + 1] += e3[c] * ph.im;
                    }
                }
            }
        }
    }
    if (f0 == 0 && fl_new != fl) flags[i] = fl_new;
#pragma unroll
    for (int j = 0; j < FC; ++j) {
        if (j < nfc) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                int64_t o = ((int64_t)(f0 + j) * 3 + c) * L.n_rx + i;
                // streaming stores: the field is not read again here, and lines
                // left dirty in L2 would be written back at the kernel boundary
                __builtin_nontemporal_store(E[j][2 * c], &E_out[2 * o]);
                __builtin_nontemporal_store(E[j][2 * c + 1], &E_out[2 * o + 1]);
            }
        }
    }
}

// grid (ceil(n_rx / 256), y_big + ceil((n_f - FC y_big) / FS)): rows
// y < y_big take FC frequencies per lane, the rows after them FS = FC / 2
// (at least 1), so the last workgroups of the launch are short and the chip
// drains evenly.
template <typename R, int FC>
__global__ void __launch_bounds__(256) k_field(LaunchParams L, const float* __restrict__ rx,
                                               const FreqConst* __restrict__ fcs, const uint8_t* __restrict__ mask,
                                               const PathRec<R>* __restrict__ rec, uint8_t* __restrict__ flags,
                                               R* __restrict__ E_out, int y_big) {
    __shared__ __attribute__((aligned(16))) R s_reg[TableStage<R>::NREG];
    __shared__ __attribute__((aligned(16))) R s_tf[TableStage<R>::NTF];
    Tabs<R> tb = TableStage<R>::template stage<256>(s_reg, s_tf);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L.n_rx) return;
    const int y = (int)blockIdx.y;
    if constexpr (FC > 1) {
        constexpr int FS = FC > 2 ? FC / 2 : 1;
        if (y >= y_big) {
            field_rx<R, FS>(L, rx, fcs, mask, rec, flags, E_out, tb, i, y_big * FC + FS * (y - y_big));
            return;
        }
    }
    field_rx<R, FC>(L, rx, fcs, mask, rec, flags, E_out, tb, i, y * FC);
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
// Scratch of utd_smooth_field_noalloc: every call on a device shares it
// (calls that overlap on one device race).  Its device address comes from
// hipGetSymbolAddress once per device, with that device current; host code
// uses only that address, never the array's name.
static __device__ __attribute__((aligned(256))) char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(char** out) {
    static std::mutex mu;
    static std::map<int, char*> ptrs;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(mu);
    auto it = ptrs.find(dev);
    if (it == ptrs.end()) {
        char* ptr = nullptr;
        e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        it = ptrs.emplace(dev, ptr).first;
    }
    *out = it->second;
    return hipSuccess;
}

hipError_t read_input_status(unsigned* bits) {
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpyFromSymbol(bits, HIP_SYMBOL(g_input_status), sizeof(unsigned));
    const unsigned zero = 0u;
    if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(g_input_status), &zero, sizeof(unsigned));
    return e;
}

hipError_t launch_census(int64_t n_mask, const uint8_t* mask, int64_t n_rx, const uint8_t* flags,
                         unsigned long long* counts, hipStream_t s) {
    hipLaunchKernelGGL(k_census, dim3(512), dim3(256), 0, s, n_mask, mask, n_rx, flags, counts);
    return hipGetLastError();
}

template <typename R>
static hipError_t launch_paths_t(const LaunchParams& L, const float* rx, const float* sph, const float* cyl,
                                 const double* freqs, BodyPrep* prep, FreqConst* fcs, const float4* nodes,
                                 const float4* tris, uint8_t* mask, void* rec, uint8_t* flags, uint64_t* ent,
                                 double* ent_th, uint64_t* vis_list, unsigned long long* counter, int64_t cap,
                                 hipStream_t s, void* grid_mem) {
    int nb = L.n_sph + L.n_cyl;
    if (!nodes) {
        // one wavefront per path kind and 64 receivers
        const int K = 2 * (L.l_enc + 1) + 1;
        dim3 grid((unsigned)((L.n_rx + 63) / 64), (unsigned)(nb > 0 ? nb : 1));
        hipLaunchKernelGGL((k_paths<R>), grid, dim3(64 * K), 0, s, L, rx, sph, cyl, freqs, prep, fcs, mask,
                           (PathRec<R>*)rec, flags);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_setup, dim3((unsigned)((nb + 255) / 256 > 0 ? (nb + 255) / 256 : 1)), dim3(256), 0, s, L,
                       sph, cyl, prep, counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 grid((unsigned)((L.n_rx + 255) / 256), (unsigned)(nb + 1));
    hipLaunchKernelGGL((k_cand<R>), grid, dim3(256), 0, s, L, rx, sph, cyl, freqs, prep, fcs, mask, flags, ent, ent_th,
                       counter, cap);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // persistent grids over the queue and the visible list: enough
    // workgroups to fill the chip
    int64_t vgrid = (cap + 255) / 256;
    vgrid = vgrid < 1 ? 1 : (vgrid > 256 * 20 ? 256 * 20 : vgrid);
    BodyGrid* bgrid = nullptr;
    if (grid_mem && nb > 0 && nb <= 64) {
        bgrid = (BodyGrid*)grid_mem;
        hipLaunchKernelGGL(k_body_grid, dim3(1), dim3(kGridN * kGridN), 0, s, L, sph, cyl, bgrid);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_vis<R>), dim3((unsigned)vgrid), dim3(256), 0, s, L, rx, sph, cyl, prep, nodes, tris, ent,
                       ent_th, counter, cap, mask, flags, vis_list, bgrid);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int64_t rgrid = vgrid < 256 * 8 ? vgrid : 256 * 8;
    hipLaunchKernelGGL((k_rec<R>), dim3((unsigned)rgrid), dim3(256), 0, s, L, rx, prep, ent, ent_th, counter,
                       vis_list, (PathRec<R>*)rec);
    return hipGetLastError();
}

hipError_t launch_paths(const LaunchParams& L, int precision, const float* rx, const float* sph, const float* cyl,
                        const double* freqs, BodyPrep* prep, FreqConst* fcs, const float4* nodes, const float4* tris,
                        uint8_t* mask, void* rec, uint8_t* flags, uint64_t* ent, double* ent_th,
                        uint64_t* vis_list, unsigned long long* counter, int64_t cap, hipStream_t s,
                        void* grid) {
    return precision == 0 ? launch_paths_t<float>(L, rx, sph, cyl, freqs, prep, fcs, nodes, tris, mask, rec, flags,
                                                  ent, ent_th, vis_list, counter, cap, s, grid)
                          : launch_paths_t<double>(L, rx, sph, cyl, freqs, prep, fcs, nodes, tris, mask, rec, flags,
                                                   ent, ent_th, vis_list, counter, cap, s, grid);
}

size_t path_record_bytes(int precision) { return precision == 0 ? sizeof(PathRec<float>) : sizeof(PathRec<double>); }

template <typename R, int FC>
static hipError_t launch_field_fc(const LaunchParams& L, const float* rx, const FreqConst* fcs, const uint8_t* mask,
                                  const void* rec, uint8_t* flags, R* E, hipStream_t s) {
    // the last frequency chunk as rows of FS frequencies once there are enough full rows
    constexpr int FS = FC > 2 ? FC / 2 : 1;
    const int nch = (L.n_f + FC - 1) / FC;
    const int y_big = (FC > 1 && nch >= 4) ? nch - 1 : nch;
    const int rows = y_big < nch ? y_big + (L.n_f - FC * y_big + FS - 1) / FS : nch;
    dim3 grid((unsigned)((L.n_rx + 255) / 256), (unsigned)rows);
    hipLaunchKernelGGL((k_field<R, FC>), grid, dim3(256), 0, s, L, rx, fcs, mask, (const PathRec<R>*)rec, flags, E,
                       y_big);
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
#include "utd_walls.h"
#include "utd_caustic.h"
