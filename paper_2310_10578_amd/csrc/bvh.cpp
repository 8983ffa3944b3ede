// Host-side BVH builder for the occluder triangles (binned SAH, two children
// per node, leaves of at most 2 triangles).  The visibility steps U of
// Eqs. (1)-(2) are decided by walking these trees on the GPU (utd_bvh.h).
//
// Two trees share the output arrays: the first (root node 0) holds the
// interior triangles, the second (root node `broot`, when there is one) the
// boundary triangles, those lying in a face plane of the scene's bounding
// box (the walls, floor and ceiling of a room).  A segment with both end
// points inside the closed box meets such a triangle at most at an end point,
// which the open-segment test excludes, so the device walks the second tree
// only for segments reaching outside the box.
//
// Output layout (read by the device traversal):
//   node  = 4 float4: (lo0.xyz, hi0.x) (hi0.yz, lo1.xy) (lo1.z, hi1.xyz) (c0, n0, c1, n1)
//           n_i > 0: leaf of n_i triangles starting at c_i; n_i == 0: inner node c_i;
//           c_i < 0: empty child.
//   tris  = 3 float4 per triangle (v0, v1, v2), in leaf order; the w of v0
//           holds the index of the triangle's reflector plane (int bits, -1
//           for a degenerate triangle).
//
// Reflector planes (one specular wall bounce, utd_walls.h): the triangles
// lying in one plane n.x = d form one mirror.  A triangle's unit normal is
// taken with its first component of magnitude above 1e-9 positive;
// triangles whose normal components and offsets agree after rounding to
// multiples of 1e-6 share a plane, planes are ordered by those rounded
// values, and each keeps the normal of its first triangle, the mean offset
// and its triangles' bounding box.
#include <algorithm>
#include <cmath>
#include <map>
#include <tuple>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "utd_internal.h"

namespace utd {

namespace {

struct Box {
    float lo[3] = {INFINITY, INFINITY, INFINITY};
    float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    void grow(const float* p) {
        for (int a = 0; a < 3; ++a) { lo[a] = std::min(lo[a], p[a]); hi[a] = std::max(hi[a], p[a]); }
    }
    void grow(const Box& b) {
        for (int a = 0; a < 3; ++a) { lo[a] = std::min(lo[a], b.lo[a]); hi[a] = std::max(hi[a], b.hi[a]); }
    }
    float area() const {
        float d[3];
        for (int a = 0; a < 3; ++a) d[a] = std::max(hi[a] - lo[a], 0.0f);
        return 2.0f * (d[0] * d[1] + d[1] * d[2] + d[2] * d[0]);
    }
};

struct Prim {
    Box box;
    float c[3];
    int64_t idx;
};

struct Child {
    Box box;
    int ref = -1;
    int count = 0;
};

struct Node {
    Child ch[2];
};

// At most two triangles per leaf and 32 SAH bins: of leaves of 1, 2, 4 and
// 8 triangles and 16, 32 or 64 bins, the fastest for the batched crowd and
// the room's visibility pass (the walks are latency-bound, so a node visit
// that rejects a box costs about what a triangle test does).
constexpr int kLeaf = 2;
constexpr int kBins = 32;

Box range_box(const std::vector<Prim>& P, int64_t b, int64_t e) {
    Box bx;
    for (int64_t i = b; i < e; ++i) bx.grow(P[i].box);
    return bx;
}

// Binned SAH split of P[b, e); returns mid with b < mid < e.
int64_t split(std::vector<Prim>& P, int64_t b, int64_t e) {
    Box cb;
    for (int64_t i = b; i < e; ++i) cb.grow(P[i].c);
    float best = INFINITY;
    int best_axis = -1, best_bin = -1;
    for (int a = 0; a < 3; ++a) {
        float ext = cb.hi[a] - cb.lo[a];
        if (!(ext > 0)) continue;
        Box bb[kBins];
        int64_t cnt[kBins] = {0};
        for (int64_t i = b; i < e; ++i) {
            int k = (int)((P[i].c[a] - cb.lo[a]) / ext * kBins);
            k = std::min(std::max(k, 0), kBins - 1);
            bb[k].grow(P[i].box);
            cnt[k]++;
        }
        float right_area[kBins];
        int64_t right_cnt[kBins];
        Box acc;
        int64_t n = 0;
        for (int k = kBins - 1; k > 0; --k) {
            acc.grow(bb[k]);
            n += cnt[k];
            right_area[k] = acc.area();
            right_cnt[k] = n;
        }
        Box lacc;
        int64_t ln = 0;
        for (int k = 0; k < kBins - 1; ++k) {
            lacc.grow(bb[k]);
            ln += cnt[k];
            if (ln == 0 || right_cnt[k + 1] == 0) continue;
            float cost = lacc.area() * (float)ln + right_area[k + 1] * (float)right_cnt[k + 1];
            if (cost < best) { best = cost; best_axis = a; best_bin = k; }
        }
    }
    int64_t mid;
    if (best_axis >= 0) {
        float ext = cb.hi[best_axis] - cb.lo[best_axis];
        auto it = std::partition(P.begin() + b, P.begin() + e, [&](const Prim& p) {
            int k = (int)((p.c[best_axis] - cb.lo[best_axis]) / ext * kBins);
            k = std::min(std::max(k, 0), kBins - 1);
            return k <= best_bin;
        });
        mid = it - P.begin();
    } else {
        mid = (b + e) / 2;
    }
    if (mid <= b || mid >= e) {
        int a = 0;
        float ext = -1;
        for (int k = 0; k < 3; ++k)
            if (cb.hi[k] - cb.lo[k] > ext) { ext = cb.hi[k] - cb.lo[k]; a = k; }
        mid = (b + e) / 2;
        std::nth_element(P.begin() + b, P.begin() + mid, P.begin() + e,
                         [a](const Prim& x, const Prim& y) { return x.c[a] < y.c[a]; });
    }
    return mid;
}

// Appends the tree over tri[ids] to the output arrays: nodes numbered from
// node_base, triangles from tri_base (references are absolute).  An empty set
// gives one node with two empty children.
// Reflector plane of every triangle (index into *planes, -1 if degenerate).
void group_planes(const float* tri, int64_t n, std::vector<int>* plane_of, std::vector<WallPlane>* planes) {
    typedef std::tuple<long long, long long, long long, long long> Key;
    std::map<Key, std::vector<int64_t>> groups;
    std::vector<double> nd(4 * (size_t)n, 0.0);
    plane_of->assign((size_t)n, -1);
    for (int64_t i = 0; i < n; ++i) {
        const float* t = tri + 9 * i;
        const double e1[3] = {(double)t[3] - t[0], (double)t[4] - t[1], (double)t[5] - t[2]};
        const double e2[3] = {(double)t[6] - t[0], (double)t[7] - t[1], (double)t[8] - t[2]};
        double c[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        const double ln = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        if (!(ln > 0)) continue;
        for (int a = 0; a < 3; ++a) c[a] /= ln;
        for (int a = 0; a < 3; ++a) {
            if (std::fabs(c[a]) > 1e-9) {
                if (c[a] < 0)
                    for (int b = 0; b < 3; ++b) c[b] = -c[b];
                break;
            }
        }
        const double d = c[0] * t[0] + c[1] * t[1] + c[2] * t[2];
        for (int a = 0; a < 3; ++a) nd[4 * i + a] = c[a];
        nd[4 * i + 3] = d;
        // round half to even, as the default floating-point rounding mode does
        Key k{(long long)std::nearbyint(c[0] / 1e-6), (long long)std::nearbyint(c[1] / 1e-6),
              (long long)std::nearbyint(c[2] / 1e-6), (long long)std::nearbyint(d / 1e-6)};
        groups[k].push_back(i);
    }
    planes->clear();
    for (auto& g : groups) {
        WallPlane P;
        const int64_t f = g.second.front();
        for (int a = 0; a < 3; ++a) P.n[a] = nd[4 * f + a];
        double sd = 0.0;
        for (int a = 0; a < 3; ++a) { P.lo[a] = INFINITY; P.hi[a] = -INFINITY; }
        for (int64_t i : g.second) {
            sd += nd[4 * i + 3];
            for (int v = 0; v < 3; ++v)
                for (int a = 0; a < 3; ++a) {
                    P.lo[a] = std::min(P.lo[a], tri[9 * i + 3 * v + a]);
                    P.hi[a] = std::max(P.hi[a], tri[9 * i + 3 * v + a]);
                }
            (*plane_of)[(size_t)i] = (int)planes->size();
        }
        P.d = sd / (double)g.second.size();
        planes->push_back(P);
    }
}

void build_tree(const float* tri, const std::vector<int>& plane_of, const std::vector<int64_t>& ids, int max_depth,
                int node_base, int64_t tri_base,
                std::vector<float>& out_nodes, std::vector<float>& out_tris, int* depth_out) {
    const int64_t n = (int64_t)ids.size();
    std::vector<Prim> P((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        Prim& p = P[(size_t)i];
        for (int v = 0; v < 3; ++v) p.box.grow(tri + 9 * ids[(size_t)i] + 3 * v);
        for (int a = 0; a < 3; ++a) p.c[a] = 0.5f * (p.box.lo[a] + p.box.hi[a]);
        p.idx = ids[(size_t)i];
    }
    std::vector<Node> nodes(1);
    struct Task { int node; int64_t b, e; int depth; };
    std::vector<Task> todo;
    if (n > 0) todo.push_back({0, 0, n, 1});
    int depth_seen = 1;
    while (!todo.empty()) {
        Task t = todo.back();
        todo.pop_back();
        int64_t ranges[2][2];
        if (t.e - t.b <= kLeaf) {
            ranges[0][0] = t.b; ranges[0][1] = t.e;
            ranges[1][0] = t.e; ranges[1][1] = t.e;
        } else {
            int64_t mid = split(P, t.b, t.e);
            ranges[0][0] = t.b; ranges[0][1] = mid;
            ranges[1][0] = mid; ranges[1][1] = t.e;
        }
        for (int c = 0; c < 2; ++c) {
            int64_t b = ranges[c][0], e = ranges[c][1];
            Child ch;
            if (e > b) {
                ch.box = range_box(P, b, e);
                if (e - b <= kLeaf || t.depth + 1 >= max_depth) {
                    ch.ref = (int)b;
                    ch.count = (int)(e - b);
                } else {
                    ch.ref = (int)nodes.size();
                    ch.count = 0;
                    nodes.emplace_back();
                    todo.push_back({ch.ref, b, e, t.depth + 1});
                    depth_seen = std::max(depth_seen, t.depth + 1);
                }
            }
            nodes[(size_t)t.node].ch[c] = ch;
        }
    }
    for (size_t k = 0; k < nodes.size(); ++k) {
        float q[16];
        const Child& a = nodes[k].ch[0];
        const Child& b = nodes[k].ch[1];
        q[0] = a.box.lo[0]; q[1] = a.box.lo[1]; q[2] = a.box.lo[2]; q[3] = a.box.hi[0];
        q[4] = a.box.hi[1]; q[5] = a.box.hi[2]; q[6] = b.box.lo[0]; q[7] = b.box.lo[1];
        q[8] = b.box.lo[2]; q[9] = b.box.hi[0]; q[10] = b.box.hi[1]; q[11] = b.box.hi[2];
        auto absref = [&](const Child& ch) {
            if (ch.ref < 0) return -1;
            return ch.count > 0 ? (int)(ch.ref + tri_base) : ch.ref + node_base;
        };
        int refs[4] = {absref(a), a.count, absref(b), b.count};
        std::memcpy(q + 12, refs, sizeof refs);
        out_nodes.insert(out_nodes.end(), q, q + 16);
    }
    for (int64_t i = 0; i < n; ++i) {
        const float* src = tri + 9 * P[(size_t)i].idx;
        for (int v = 0; v < 3; ++v) {
            out_tris.push_back(src[3 * v + 0]);
            out_tris.push_back(src[3 * v + 1]);
            out_tris.push_back(src[3 * v + 2]);
            float w = 0.0f;
            if (v == 0) {
                const int pid = plane_of[(size_t)P[(size_t)i].idx];
                std::memcpy(&w, &pid, sizeof w);
            }
            out_tris.push_back(w);
        }
    }
    *depth_out = depth_seen;
}

}  // namespace

int build_bvh(const float* tri, int64_t n, int max_depth, HostBvh* out) {
    *out = HostBvh();
    if (n <= 0) return 0;
    Box scene;
    for (int64_t i = 0; i < 3 * n; ++i) scene.grow(tri + 3 * i);
    std::vector<int64_t> inner, bound;
    for (int64_t i = 0; i < n; ++i) {
        const float* t = tri + 9 * i;
        bool on_face = false;
        for (int a = 0; a < 3 && !on_face; ++a)
            on_face = (t[a] == scene.lo[a] && t[3 + a] == scene.lo[a] && t[6 + a] == scene.lo[a]) ||
                      (t[a] == scene.hi[a] && t[3 + a] == scene.hi[a] && t[6 + a] == scene.hi[a]);
        (on_face ? bound : inner).push_back(i);
    }
    std::vector<float> nodes, tris;
    int d0 = 0, d1 = 0;
    std::vector<int> plane_of;
    group_planes(tri, n, &plane_of, &out->planes);
    build_tree(tri, plane_of, inner, max_depth, 0, 0, nodes, tris, &d0);
    out->broot = -1;
    if (!bound.empty()) {
        out->broot = (int64_t)(nodes.size() / 16);
        build_tree(tri, plane_of, bound, max_depth, (int)out->broot, (int64_t)inner.size(), nodes, tris, &d1);
    }
    for (int a = 0; a < 3; ++a) { out->lo[a] = scene.lo[a]; out->hi[a] = scene.hi[a]; }
    out->n_nodes = (int64_t)(nodes.size() / 16);
    out->n_inner_tris = (int64_t)inner.size();
    out->depth = std::max(d0, d1);
    out->nodes = (float*)std::malloc(sizeof(float) * nodes.size());
    out->tris = (float*)std::malloc(sizeof(float) * tris.size());
    if (!out->nodes || !out->tris) { free_bvh(out); return -1; }
    std::memcpy(out->nodes, nodes.data(), sizeof(float) * nodes.size());
    std::memcpy(out->tris, tris.data(), sizeof(float) * tris.size());
    return 0;
}

void free_bvh(HostBvh* b) {
    std::free(b->nodes);
    std::free(b->tris);
    b->nodes = nullptr;
    b->tris = nullptr;
    b->n_nodes = 0;
}

}  // namespace utd
