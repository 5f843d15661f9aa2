// Host-side construction of a tetrahedral part's location tables (no HIP
// dependency): the four face planes of every tetrahedron with the tie rule
// folded in, and a uniform grid over the part's bounding box whose cells
// list the tetrahedra that can hold a point of the cell.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace dpvr {

// Fixed direction of the face tie rule: a point on a face belongs to the
// tetrahedron that this direction enters across the face (exact binary
// fractions, so no face normal of a lattice-aligned mesh is orthogonal to it).
constexpr double kTieG[3] = {1.0, 0x1p-10, 0x1p-20};

struct TetTables {
    int32_t n_tets = 0, n_vertices = 0;
    // Face i of tetrahedron e (the face opposite vertex i): planes[16 e + 4 i
    // + (0, 1, 2, 3)] = (nx, ny, nz, c) such that the signed sub-volume of a
    // point p against that face is D_i(p) = (nx px + ny py) + nz pz - c,
    // positive toward vertex i.  The normal is computed from the face's
    // vertices in lexicographic order, so the two tetrahedra sharing a face
    // compute the same D up to sign.
    std::vector<double> planes;
    // bit i: a point with D_i = 0 counts as inside across face i (the tie
    // direction enters the tetrahedron there)
    std::vector<uint32_t> owned;
    std::vector<int32_t> tets;        // 4 vertex indices per tetrahedron (value gather)
    // nbr[4 e + i]: the tetrahedron of the part across face i of e (-1 on the
    // part's boundary), for the walk from one sample's tetrahedron to the next
    std::vector<int32_t> nbr;
    double lo[3], hi[3];              // closed bounding box of the vertices the tetrahedra use
    double glo[3], ginv[3];           // grid origin and cells per world unit
    int32_t gdim[3];
    std::vector<int32_t> cell_start;  // gdim product + 1 (exclusive prefix)
    std::vector<int32_t> cell_tets;   // tetrahedra of each cell, ascending
    // Bounding volume hierarchy over the tetrahedra, nodes in depth-first
    // order (a node's first child follows it), 8 words each: lo x, y, z
    // (float32 bits), skip; hi x, y, z (float32 bits), leaf.  The box is
    // rounded outward, so it holds every float64 point of its tetrahedra's
    // boxes; skip = the node after the subtree (-1: none); leaf = -1 for an
    // inner node, else 8 first + count: the leaf's tetrahedra are
    // bvh_tets[first .. first + count), count <= 4.
    std::vector<int32_t> bvh_nodes;
    std::vector<int32_t> bvh_tets;
};

// Tetrahedra of a part given as mixed cells (host arrays): sizes[c] = 4, 5,
// 6 or 8 nodes (tetrahedron, pyramid, wedge, hexahedron; node orders as in
// dpvr.h), their node indices one cell after another.  Every quadrilateral
// is cut along the diagonal through its node of smallest id (ids: one per
// vertex, NULL = the vertex index), a pyramid is its two base triangles
// joined to its apex, and a wedge or hexahedron gets a centre vertex (the
// sum of its node positions in node order over the node count) joined to
// every triangle of its faces.  Appends the centre vertices to `vertices`
// (a copy of the input first) and, per centre vertex, its cell's nodes to
// `centre_nodes` (8 per centre, -1 after the last).  Returns false with a
// message on invalid input.
bool decompose_cells(const double* vertices, int32_t n_vertices, const int64_t* ids, const uint8_t* sizes,
                     const int32_t* cell_vertices, int32_t n_cells, std::vector<double>& out_vertices,
                     std::vector<int32_t>& out_tets, std::vector<int32_t>& centre_nodes, std::string& err);

// Builds the tables of a part given as host arrays (vertices: n_vertices x 3
// doubles x, y, z; tets: n_tets x 4 indices, either orientation).  Returns
// false with a message on invalid input (index out of range, non-finite
// coordinate, zero-volume tetrahedron, a face of more than two tetrahedra,
// too many grid entries) and throws
// std::bad_alloc when host memory runs out.
bool build_tet_tables(const double* vertices, int32_t n_vertices, const int32_t* tets, int32_t n_tets,
                      TetTables& out, std::string& err);

}  // namespace dpvr
