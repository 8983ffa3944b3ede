// Internal interface between the C ABI (utd_api.cpp) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "utd_device.h"

namespace utd {

struct FanProfile;
struct BodyGrid;

// Frames of a batched call (see utd_batched.h).
struct BatchParams {
    LaunchParams L;          // source, frequency count and options (n_sph = 0)
    int64_t n_frames;
    int64_t n_cyl;           // cylinders in the array (bound for body_off)
    int64_t n_rx;            // receivers in the array (bound for rx_off)
    int tile;                // receivers per work item (= blockDim.x)
};
// Visibility: with triangles (nodes != NULL) through a queue of candidate
// paths (ent, ent_th) and a list of the visible ones (vis_list), each of cap
// entries (n_rx (1 + n_bodies (2 l_enc + 3)) always suffices), with their
// lengths in counter[0] and counter[1]; without triangles in one pass.  Also
// stores the body constants (prep) and, when freqs is not NULL, the
// frequency constants (fcs) for the later kernels of the call.  Record slots
// per (receiver, body): 2 (l_enc + 1) + 1.  `grid` (body_grid_bytes(), or
// NULL): scratch for the grid of the bodies' footprints that the visibility
// tests use.
hipError_t launch_paths(const LaunchParams& L, int precision, const float* rx, const float* sph, const float* cyl,
                        const double* freqs, BodyPrep* prep, FreqConst* fcs, const float4* nodes, const float4* tris,
                        uint8_t* mask, void* rec, uint8_t* flags, uint64_t* ent, double* ent_th,
                        uint64_t* vis_list, unsigned long long* counter, int64_t cap, hipStream_t s,
                        void* grid = nullptr);
// Scratch of the body grid that launch_paths builds (scenes with triangles
// and at most 64 bodies) when given one.
size_t body_grid_bytes();
size_t path_record_bytes(int precision);
hipError_t launch_field(const LaunchParams& L, int precision, int fc, const float* rx, const FreqConst* fcs,
                        const uint8_t* mask, const void* rec, uint8_t* flags, void* E, hipStream_t s);

// Adjoint (utd_adjoint.h): scratch is adjoint_scratch_bytes(L) bytes.
size_t adjoint_scratch_bytes(const LaunchParams& L);
hipError_t launch_adjoint(const LaunchParams& L, int precision, const float* rx, const float* sph, const float* cyl,
                          const BodyPrep* prep, const FreqConst* fcs, const uint8_t* mask, const void* rec,
                          const uint8_t* flags, const void* gE, char* scratch, void* d_sph, void* d_cyl, void* d_tx,
                          hipStream_t s);

// Device workspace of a batched call, carved from one allocation by
// batch_workspace (which returns its size in bytes; base may be NULL to size).
struct BatchWs {
    BodyPrep* prep;          // per cylinder
    FreqConst* fcs;          // per frequency
    int64_t* bo;             // sanitised body offsets (n_frames + 1)
    int64_t* ro;             // sanitised receiver offsets (n_frames + 1)
    int64_t* tile_off;       // tile prefix sum (n_frames + 1)
    unsigned* counter;       // work-queue counter
    uint16_t* key;           // per receiver: spatial cell
    int* perm;               // per receiver: frame-local index at each sorted position
    double* th;              // per block: reflection angles of a body group
    void* ew;                // per block: the tile's field
    struct FanProfile* fans; // per (cylinder, side): source-side leg profile
    struct BodyGrid* grids;  // per frame: grid of the cylinders' footprints
    uint8_t* flw;            // per receiver: its flags and line of sight (k_batch_los)
};
size_t batch_workspace(const BatchParams& B, int precision, int n_blocks, char* base, BatchWs* ws);
// part 0: the whole call; 1: the constants, the receiver order, the body
// grids, the source-side leg profiles and the receivers' flags and direct
// rays only (k_batch_prep, k_batch_sort, k_batch_grid, k_batch_fans,
// k_batch_los); 2: the persistent kernel only.  n_main: nodes of the BVH's
// main (interior-triangle) tree, which come first in `nodes`.
hipError_t launch_batch(const BatchParams& B, int precision, int n_blocks, const int64_t* body_off,
                        const int64_t* rx_off, const float* rx, const float* cyl, const double* freqs,
                        const BatchWs& ws, const float4* nodes, const float4* tris, int n_main, void* E,
                        uint8_t* flags, hipStream_t s, int part = 0);

// Scratch of the allocation-free entry point: a static device array of
// kNoAllocScratchBytes; noalloc_scratch gives its address on the current
// device (taken once per device with hipGetSymbolAddress).
constexpr size_t kNoAllocScratchBytes = (size_t)256 << 20;
hipError_t noalloc_scratch(char** out);

// Waits for the current device, then reads and clears its input-status bits.
hipError_t read_input_status(unsigned* bits);

hipError_t launch_census(int64_t n_mask, const uint8_t* mask, int64_t n_rx, const uint8_t* flags,
                         unsigned long long* counts, hipStream_t s);

// A reflector plane n.x = d of the scene triangles (one specular wall
// bounce) with the bounding box of its triangles.
struct WallPlane {
    double n[3];
    double d;
    float lo[3], hi[3];
};

// Wall material: a slab of relative permittivity eps_r, conductivity sigma
// (S/m) and thickness (m; infinite: a half-space), or a perfect conductor.
struct WallMat {
    double eps_r, sigma, thickness;
    int pec;
};

// Uniform sum of a sphere's creeping-ray pairs at the axial caustic
// (utd_caustic.h): launch_pairs after the path kernels (the pairs with both
// paths visible leave the mask for pm [n_sph][n_rx]; unpaired paths within
// guard of the axis are dropped and flagged), launch_caustic after the
// field kernel (the pairs' field added into E).
hipError_t launch_pairs(const LaunchParams& L, double guard, const float* rx, const BodyPrep* prep, uint8_t* mask,
                        uint8_t* pm, hipStream_t s);
hipError_t launch_caustic(const LaunchParams& L, int precision, const float* rx, const BodyPrep* prep,
                          const FreqConst* fcs, const uint8_t* pm, void* E, hipStream_t s);

// One specular wall bounce (utd_walls.h): body constants of the image
// sources (prep_img, n_planes * bodies entries) then the wall paths of every
// receiver, added to E; wall decisions to wmask ([n_rx][n_planes]) when not
// NULL.
size_t walls_scratch_bytes(const LaunchParams& L, int n_planes);
hipError_t launch_walls(const LaunchParams& L, int precision, const WallMat& M, const float* rx, const float* sph,
                        const float* cyl, const BodyPrep* prep, BodyPrep* prep_img, const WallPlane* planes,
                        int n_planes, const float4* nodes, const float4* tris, const FreqConst* fcs,
                        const double* freqs, uint8_t* flags, void* E, uint64_t* wmask, hipStream_t s);

// host BVH over a triangle soup (bvh.cpp)
struct HostBvh {
    int64_t n_nodes = 0;
    int64_t broot = -1;       // root of the boundary-triangle tree (-1: none)
    int64_t n_inner_tris = 0;
    float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};   // scene bounding box
    int depth = 0;
    float* nodes = nullptr;   // n_nodes * 16 floats (4 float4 per node)
    float* tris = nullptr;    // n_tri * 12 floats (3 float4 per triangle), leaf order
    std::vector<WallPlane> planes;   // reflector planes, ordered as described in bvh.cpp
};
int build_bvh(const float* tri_xyz, int64_t n_tri, int max_depth, HostBvh* out);
void free_bvh(HostBvh* b);

}  // namespace utd
