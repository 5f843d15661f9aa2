// Internal interface between the host-side C-ABI (api.cpp) and the kernels
// of tetrahedral parts (tets.hip), kept apart from the structured-brick
// interface (dpvr_kernels.h) that it builds on.
#pragma once

#include "dpvr_kernels.h"

namespace dpvr {

// Tetrahedral parts (tets.hip).  A part's location tables (built on the host,
// tet_build.h) as the kernels see them, and its share of a frame: the runs
// (maximal stretches of consecutive lattice samples the part holds) of every
// ROI pixel's ray.
constexpr int kMaxTetRuns = 32;
enum : int32_t { kTetGrid = 0, kTetBvh = 1 };
constexpr int kMaxTetParts = 64;
struct TetPartK {
    const double* planes;       // n_tets x 16: per face (nx, ny, nz, c), D = n.p - c >= 0 inside
    const float* vals;          // n_tets x 4: vertex values in vertex order (16-byte aligned)
    const uint32_t* owned;      // n_tets: tie-rule bits
    const int32_t* cell_start;  // grid cells + 1
    const int32_t* cell_tets;
    const int32_t* nbr;         // n_tets x 4: tetrahedron across each face (-1: none in the part)
    const int32_t* bvh_nodes;   // BVH nodes, 8 words each (tet_build.h)
    const int32_t* bvh_tets;    // leaves' tetrahedra
    double lo[3], hi[3];        // closed bounding box
    double glo[3], ginv[3];     // grid origin, cells per world unit
    int32_t gdim[3];
    int32_t n_tets;
    int32_t roi_x0, roi_y0, roi_w, roi_h;
    long long entry0;           // first frame entry of the part (its ROI pixels, row-major, after the previous parts')
    int32_t* rcount;            // roi_h x roi_w: runs of the pixel's ray
    int32_t* rkey;              // max_runs x roi_h x roi_w: first sample index of each run
    float* rcol;                // max_runs x roi_h x roi_w x 4: premultiplied colour, alpha of each run
};

struct TetFrameParams {
    CameraK cam;
    TFK tf;
    double dt;
    const TetPartK* parts;      // device, n
    const int32_t* tile_start;  // device, n + 1: exclusive prefix of tiles (tet_tiles)
    int32_t n, total_tiles, max_runs;
    int32_t width, height;
    float bg[4];
    float* out;                 // height x width x 4
    unsigned long long* samples;  // optional: += samples held by a tetrahedron (primary and shadow)
    int32_t* err;               // device error word
    int32_t locator;            // after the walk: kTetGrid or kTetBvh
    // shadow rays (one directional light): per frame entry the first slot of
    // its held primary samples (offsets[n_entries] = total), per slot the
    // sample index and the shadow transmittance
    long long n_entries, total;
    long long* offsets;
    int32_t* slot_k;
    float* shade;
    double light[3];            // unit direction toward the light
    float ambient;              // a0: emission scaled by a0 + (1 - a0) S
    int32_t step;               // cycle step of a shadow launch
};

// Stages of a tetrahedral frame (bit mask): the plain march into runs, the
// resolve; with shadows: count the held samples per entry, record their
// sample indices, the shadow cycle steps, the shaded march into runs.
enum : int { kTetMarch = 1, kTetResolve = 2, kTetCount = 4, kTetRecord = 8, kTetShadow = 16, kTetShaded = 32 };

constexpr int32_t kErrRuns = 4;   // a ray crossed a part in more than max_runs runs

// Tiles of the tetrahedral march: kTetTile x kTetTile pixels, one workgroup
// of (kTetTile / 8)^2 wavefronts of 8 x 8 rays each.
constexpr int kTetTile = 16;
inline int32_t tet_tiles(int32_t w, int32_t h) {
    return ((w + kTetTile - 1) / kTetTile) * ((h + kTetTile - 1) / kTetTile);
}
// Per tetrahedron its four vertex values: vertex v < n_input from
// vertex_values, a cell centre v >= n_input the mean of its cell's nodes
// (centre_nodes[8 (v - n_input) + i], -1 after the last).
hipError_t launch_tet_values(const float* vertex_values, int32_t n_input, const int32_t* centre_nodes,
                             const int32_t* tets, int32_t n_tets, float* vals, hipStream_t stream);
// stages: a mask of the kTet* stages above, run in the order listed there
hipError_t launch_tet_frame(TetFrameParams p, int stages, hipStream_t stream);

}  // namespace dpvr
