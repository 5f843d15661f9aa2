// Location tables of a tetrahedral part (host, float64, no contraction: the
// library is compiled with -ffp-contract=off, so every plane is computed
// with plain rounded multiplies and adds).
#include "tet_build.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>

namespace dpvr {
namespace {

bool lex_less(const double* a, const double* b) {
    if (a[0] != b[0]) return a[0] < b[0];
    if (a[1] != b[1]) return a[1] < b[1];
    return a[2] < b[2];
}

// Plane of face i of the tetrahedron with vertex positions v[0..3]; returns
// false for a degenerate tetrahedron (the opposite vertex on the face plane).
bool face_plane(const double* const v[4], int i, double plane[4], bool* owned) {
    const double* f[3];
    int m = 0;
    for (int j = 0; j < 4; ++j)
        if (j != i) f[m++] = v[j];
    std::sort(f, f + 3, lex_less);
    const double e1[3] = {f[1][0] - f[0][0], f[1][1] - f[0][1], f[1][2] - f[0][2]};
    const double e2[3] = {f[2][0] - f[0][0], f[2][1] - f[0][1], f[2][2] - f[0][2]};
    const double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                         e1[0] * e2[1] - e1[1] * e2[0]};
    const double c = (n[0] * f[0][0] + n[1] * f[0][1]) + n[2] * f[0][2];
    const double di = ((n[0] * v[i][0] + n[1] * v[i][1]) + n[2] * v[i][2]) - c;
    if (!(di != 0.0) || !std::isfinite(di)) return false;
    const double s = di > 0.0 ? 1.0 : -1.0;
    for (int a = 0; a < 3; ++a) plane[a] = s * n[a];
    plane[3] = s * c;
    *owned = s * ((n[0] * kTieG[0] + n[1] * kTieG[1]) + n[2] * kTieG[2]) > 0.0;
    return true;
}

// Whether a tetrahedron with these planes can hold a point of the box
// centred at ctr with half extents h: no face has the whole box on its
// outer side (D is affine, so its maximum over the box is D(ctr) + sum |n_a| h_a).
bool may_hold(const double* planes, const double ctr[3], const double h[3]) {
    for (int i = 0; i < 4; ++i) {
        const double* p = planes + 4 * i;
        const double dc = ((p[0] * ctr[0] + p[1] * ctr[1]) + p[2] * ctr[2]) - p[3];
        const double reach = std::fabs(p[0]) * h[0] + std::fabs(p[1]) * h[1] + std::fabs(p[2]) * h[2];
        // slack for rounding: relative to the plane's magnitude at the box
        const double mag = std::fabs(p[0] * ctr[0]) + std::fabs(p[1] * ctr[1]) + std::fabs(p[2] * ctr[2]) +
                           std::fabs(p[3]) + reach;
        if (dc + reach < -1e-12 * mag) return false;
    }
    return true;
}

// BVH over the tetrahedra (median split of the centroids on the longest
// axis of their bounds, leaves of at most kLeaf), nodes in depth-first
// order with skip links, so that a point query needs no stack.
constexpr int kLeaf = 4;

void build_bvh(const double* V, const int32_t* T, int32_t nt, TetTables& out) {
    out.bvh_nodes.clear();
    out.bvh_tets.resize(nt);
    if (nt == 0) return;
    std::vector<double> box((size_t)nt * 6), cen((size_t)nt * 3);
    for (int32_t e = 0; e < nt; ++e) {
        double* b = &box[6 * (size_t)e];
        for (int c = 0; c < 3; ++c) {
            b[c] = INFINITY;
            b[3 + c] = -INFINITY;
        }
        for (int j = 0; j < 4; ++j)
            for (int c = 0; c < 3; ++c) {
                const double x = V[3 * (size_t)T[4 * (size_t)e + j] + c];
                b[c] = std::fmin(b[c], x);
                b[3 + c] = std::fmax(b[3 + c], x);
            }
        for (int c = 0; c < 3; ++c) cen[3 * (size_t)e + c] = 0.5 * (b[c] + b[3 + c]);
        out.bvh_tets[e] = e;
    }
    // float32 bounds that contain the float64 box
    auto down = [](double x) {
        const float f = (float)x;
        return (double)f > x ? std::nextafter(f, -INFINITY) : f;
    };
    auto up = [](double x) {
        const float f = (float)x;
        return (double)f < x ? std::nextafter(f, INFINITY) : f;
    };
    auto bits = [](float f) {
        int32_t i;
        std::memcpy(&i, &f, sizeof i);
        return i;
    };
    std::function<void(int32_t, int32_t)> rec = [&](int32_t first, int32_t count) {
        const size_t node = out.bvh_nodes.size() / 8;
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int32_t i = first; i < first + count; ++i) {
            const int32_t e = out.bvh_tets[i];
            for (int c = 0; c < 3; ++c) {
                lo[c] = std::fmin(lo[c], box[6 * (size_t)e + c]);
                hi[c] = std::fmax(hi[c], box[6 * (size_t)e + 3 + c]);
                clo[c] = std::fmin(clo[c], cen[3 * (size_t)e + c]);
                chi[c] = std::fmax(chi[c], cen[3 * (size_t)e + c]);
            }
        }
        for (int c = 0; c < 3; ++c) out.bvh_nodes.push_back(bits(down(lo[c])));
        out.bvh_nodes.push_back(-1);
        for (int c = 0; c < 3; ++c) out.bvh_nodes.push_back(bits(up(hi[c])));
        out.bvh_nodes.push_back(-1);
        if (count <= kLeaf) {
            out.bvh_nodes[8 * node + 7] = 8 * first + count;
        } else {
            int axis = 0;
            for (int c = 1; c < 3; ++c)
                if (chi[c] - clo[c] > chi[axis] - clo[axis]) axis = c;
            const int32_t half = count / 2;
            std::nth_element(out.bvh_tets.begin() + first, out.bvh_tets.begin() + first + half,
                             out.bvh_tets.begin() + first + count, [&](int32_t a, int32_t b) {
                                 const double ca = cen[3 * (size_t)a + axis], cb = cen[3 * (size_t)b + axis];
                                 return ca < cb || (ca == cb && a < b);
                             });
            rec(first, half);
            rec(first + half, count - half);
        }
        out.bvh_nodes[8 * node + 3] = (int32_t)(out.bvh_nodes.size() / 8);   // the node after the subtree
    };
    rec(0, nt);
    const int32_t n_nodes = (int32_t)(out.bvh_nodes.size() / 8);
    for (int32_t q = 0; q < n_nodes; ++q)
        if (out.bvh_nodes[8 * (size_t)q + 3] >= n_nodes) out.bvh_nodes[8 * (size_t)q + 3] = -1;
}

}  // namespace

bool build_tet_tables(const double* V, int32_t nv, const int32_t* T, int32_t nt, TetTables& out,
                      std::string& err) {
    char buf[256];
    out = TetTables{};
    if (nt >= (1 << 28)) {
        err = "a part of 2^28 or more tetrahedra (split it into smaller parts)";
        return false;
    }
    out.n_tets = nt;
    out.n_vertices = nv;
    out.planes.resize((size_t)nt * 16);
    out.owned.resize(nt);
    out.tets.assign(T, T + (size_t)nt * 4);
    for (int c = 0; c < 3; ++c) {
        out.lo[c] = INFINITY;
        out.hi[c] = -INFINITY;
    }
    for (int32_t e = 0; e < nt; ++e) {
        const double* v[4];
        for (int j = 0; j < 4; ++j) {
            const int32_t q = T[4 * (size_t)e + j];
            if (q < 0 || q >= nv) {
                snprintf(buf, sizeof buf, "tetrahedron %d: vertex index %d outside [0, %d)", e, q, nv);
                err = buf;
                return false;
            }
            v[j] = V + 3 * (size_t)q;
            for (int c = 0; c < 3; ++c) {
                if (!std::isfinite(v[j][c])) {
                    snprintf(buf, sizeof buf, "vertex %d has a non-finite coordinate", q);
                    err = buf;
                    return false;
                }
                out.lo[c] = std::fmin(out.lo[c], v[j][c]);
                out.hi[c] = std::fmax(out.hi[c], v[j][c]);
            }
        }
        uint32_t bits = 0;
        for (int i = 0; i < 4; ++i) {
            bool own = false;
            if (!face_plane(v, i, &out.planes[16 * (size_t)e + 4 * i], &own)) {
                snprintf(buf, sizeof buf, "tetrahedron %d has zero volume", e);
                err = buf;
                return false;
            }
            if (own) bits |= 1u << i;
        }
        out.owned[e] = bits;
    }
    // face neighbours: the faces of all tetrahedra sorted by their vertex
    // triple; two equal neighbours are the tetrahedra sharing that face
    {
        struct Face {
            int32_t v[3];
            int32_t id;   // 4 e + i
        };
        std::vector<Face> faces((size_t)nt * 4);
        for (int32_t e = 0; e < nt; ++e)
            for (int i = 0; i < 4; ++i) {
                Face& f = faces[4 * (size_t)e + i];
                int m = 0;
                for (int j = 0; j < 4; ++j)
                    if (j != i) f.v[m++] = T[4 * (size_t)e + j];
                std::sort(f.v, f.v + 3);
                f.id = 4 * e + i;
            }
        std::sort(faces.begin(), faces.end(), [](const Face& a, const Face& b) {
            if (a.v[0] != b.v[0]) return a.v[0] < b.v[0];
            if (a.v[1] != b.v[1]) return a.v[1] < b.v[1];
            if (a.v[2] != b.v[2]) return a.v[2] < b.v[2];
            return a.id < b.id;
        });
        out.nbr.assign((size_t)nt * 4, -1);
        for (size_t q = 0; q < faces.size();) {
            size_t r = q + 1;
            while (r < faces.size() && faces[r].v[0] == faces[q].v[0] && faces[r].v[1] == faces[q].v[1] &&
                   faces[r].v[2] == faces[q].v[2])
                ++r;
            if (r - q > 2) {
                snprintf(buf, sizeof buf, "a face (vertices %d, %d, %d) is shared by %d tetrahedra", faces[q].v[0],
                         faces[q].v[1], faces[q].v[2], (int)(r - q));
                err = buf;
                return false;
            }
            if (r - q == 2) {
                out.nbr[faces[q].id] = faces[q + 1].id / 4;
                out.nbr[faces[q + 1].id] = faces[q].id / 4;
            }
            q = r;
        }
    }
    if (nt == 0) {
        for (int c = 0; c < 3; ++c) {
            out.lo[c] = out.hi[c] = out.glo[c] = 0.0;
            out.ginv[c] = 1.0;
            out.gdim[c] = 1;
        }
        out.cell_start.assign(2, 0);
        build_bvh(V, T, nt, out);
        return true;
    }
    // Grid: about one cell per tetrahedron, cubic cells, over the box grown
    // by a small margin (so points that round onto the box faces still fall
    // in a cell).
    double ext[3], vol = 1.0, emax = 0.0;
    for (int c = 0; c < 3; ++c) emax = std::fmax(emax, out.hi[c] - out.lo[c]);
    const double margin = 1e-7 * emax;
    for (int c = 0; c < 3; ++c) {
        ext[c] = (out.hi[c] - out.lo[c]) + 2.0 * margin;
        out.glo[c] = out.lo[c] - margin;
        vol *= ext[c];
    }
    const double cell = std::cbrt(vol / (double)nt);
    size_t cells = 1;
    for (int c = 0; c < 3; ++c) {
        const double g = std::ceil(ext[c] / cell);
        out.gdim[c] = (int32_t)std::min(std::max(g, 1.0), 1024.0);
        out.ginv[c] = (double)out.gdim[c] / ext[c];
        cells *= (size_t)out.gdim[c];
    }
    const double cw[3] = {ext[0] / out.gdim[0], ext[1] / out.gdim[1], ext[2] / out.gdim[2]};
    // cells tested for tetrahedron e: those its bounding box touches, widened
    // by a millionth of a cell; each is grown by that much too
    auto range = [&](int32_t e, int32_t r0[3], int32_t r1[3]) {
        double a[3] = {INFINITY, INFINITY, INFINITY}, b[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int j = 0; j < 4; ++j) {
            const double* p = V + 3 * (size_t)T[4 * (size_t)e + j];
            for (int c = 0; c < 3; ++c) {
                a[c] = std::fmin(a[c], p[c]);
                b[c] = std::fmax(b[c], p[c]);
            }
        }
        for (int c = 0; c < 3; ++c) {
            r0[c] = (int32_t)std::max(std::floor((a[c] - out.glo[c]) * out.ginv[c] - 1e-6), 0.0);
            r1[c] = (int32_t)std::min(std::floor((b[c] - out.glo[c]) * out.ginv[c] + 1e-6),
                                      (double)(out.gdim[c] - 1));
        }
    };
    const double h[3] = {0.5 * cw[0] * (1.0 + 2e-6), 0.5 * cw[1] * (1.0 + 2e-6), 0.5 * cw[2] * (1.0 + 2e-6)};
    auto for_cells = [&](int32_t e, auto&& fn) {
        int32_t r0[3], r1[3];
        range(e, r0, r1);
        const double* pl = &out.planes[16 * (size_t)e];
        for (int32_t z = r0[2]; z <= r1[2]; ++z)
            for (int32_t y = r0[1]; y <= r1[1]; ++y)
                for (int32_t x = r0[0]; x <= r1[0]; ++x) {
                    const double ctr[3] = {out.glo[0] + (x + 0.5) * cw[0], out.glo[1] + (y + 0.5) * cw[1],
                                           out.glo[2] + (z + 0.5) * cw[2]};
                    if (may_hold(pl, ctr, h))
                        fn(((size_t)z * out.gdim[1] + y) * out.gdim[0] + x);
                }
    };
    std::vector<int64_t> count(cells + 1, 0);
    for (int32_t e = 0; e < nt; ++e) for_cells(e, [&](size_t q) { ++count[q + 1]; });
    for (size_t q = 0; q < cells; ++q) count[q + 1] += count[q];
    if (count[cells] > INT32_MAX) {
        snprintf(buf, sizeof buf, "location grid of %lld entries exceeds 2^31 - 1", (long long)count[cells]);
        err = buf;
        return false;
    }
    out.cell_start.resize(cells + 1);
    for (size_t q = 0; q <= cells; ++q) out.cell_start[q] = (int32_t)count[q];
    out.cell_tets.resize((size_t)count[cells]);
    std::vector<int32_t> fill(out.cell_start.begin(), out.cell_start.end() - 1);
    for (int32_t e = 0; e < nt; ++e) for_cells(e, [&](size_t q) { out.cell_tets[fill[q]++] = e; });
    build_bvh(V, T, nt, out);
    return true;
}

bool decompose_cells(const double* V, int32_t nv, const int64_t* ids, const uint8_t* sizes, const int32_t* C,
                     int32_t n_cells, std::vector<double>& out_v, std::vector<int32_t>& out_t,
                     std::vector<int32_t>& centre_nodes, std::string& err) {
    char buf[256];
    out_v.assign(V, V + 3 * (size_t)nv);
    out_t.clear();
    centre_nodes.clear();
    auto id = [&](int32_t q) { return ids ? ids[q] : (int64_t)q; };
    auto tet = [&](int32_t a, int32_t b, int32_t c, int32_t d) {
        out_t.push_back(a);
        out_t.push_back(b);
        out_t.push_back(c);
        out_t.push_back(d);
    };
    // the two triangles of quadrilateral (a, b, c, d), cyclic, each joined to apex x
    auto quad = [&](int32_t a, int32_t b, int32_t c, int32_t d, int32_t x) {
        const int32_t q[4] = {a, b, c, d};
        int m = 0;
        for (int i = 1; i < 4; ++i)
            if (id(q[i]) < id(q[m])) m = i;
        if (m == 0 || m == 2) {
            tet(a, b, c, x);
            tet(a, c, d, x);
        } else {
            tet(a, b, d, x);
            tet(b, c, d, x);
        }
    };
    static const int kWedge[5][4] = {{0, 1, 2, -1}, {3, 4, 5, -1}, {0, 1, 4, 3}, {1, 2, 5, 4}, {2, 0, 3, 5}};
    static const int kHex[6][4] = {{0, 1, 2, 3}, {4, 5, 6, 7}, {0, 1, 5, 4}, {1, 2, 6, 5}, {2, 3, 7, 6}, {3, 0, 4, 7}};
    size_t pos = 0;
    for (int32_t c = 0; c < n_cells; ++c) {
        const int n = sizes[c];
        if (n != 4 && n != 5 && n != 6 && n != 8) {
            snprintf(buf, sizeof buf, "cell %d has %d nodes (4, 5, 6 or 8 expected)", c, n);
            err = buf;
            return false;
        }
        const int32_t* q = C + pos;
        pos += (size_t)n;
        for (int i = 0; i < n; ++i)
            if (q[i] < 0 || q[i] >= nv) {
                snprintf(buf, sizeof buf, "cell %d: vertex index %d outside [0, %d)", c, q[i], nv);
                err = buf;
                return false;
            }
        if (n == 4) {
            tet(q[0], q[1], q[2], q[3]);
        } else if (n == 5) {
            quad(q[0], q[1], q[2], q[3], q[4]);
        } else {
            const size_t centre = out_v.size() / 3;
            if (centre > (size_t)INT32_MAX) {
                err = "more than 2^31 - 1 vertices with the cell centres";
                return false;
            }
            double sx = 0.0, sy = 0.0, sz = 0.0;
            for (int i = 0; i < n; ++i) {
                sx += V[3 * (size_t)q[i]];
                sy += V[3 * (size_t)q[i] + 1];
                sz += V[3 * (size_t)q[i] + 2];
            }
            out_v.push_back(sx / n);
            out_v.push_back(sy / n);
            out_v.push_back(sz / n);
            for (int i = 0; i < 8; ++i) centre_nodes.push_back(i < n ? q[i] : -1);
            const int32_t x = (int32_t)centre;
            if (n == 6) {
                for (const auto& f : kWedge) {
                    if (f[3] < 0) tet(q[f[0]], q[f[1]], q[f[2]], x);
                    else quad(q[f[0]], q[f[1]], q[f[2]], q[f[3]], x);
                }
            } else {
                for (const auto& f : kHex) quad(q[f[0]], q[f[1]], q[f[2]], q[f[3]], x);
            }
        }
        if (out_t.size() / 4 > (size_t)INT32_MAX) {
            err = "more than 2^31 - 1 tetrahedra";
            return false;
        }
    }
    return true;
}

}  // namespace dpvr
