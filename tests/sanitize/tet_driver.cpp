// Host check of the tetrahedral location tables (tet_build.cpp), run under
// the sanitizers: on conforming meshes of a box (vertices on a 2^-10 grid),
// every probe point -- random ones, half-step lattice points on vertices,
// edges and faces, and points on the faces of jittered tetrahedra -- is held
// (by the planes and tie bits, the kernels' rule) by exactly one tetrahedron
// inside the box and by none outside its half-open extent, and that
// tetrahedron is listed in the point's grid cell.  (Points within a few
// rounding steps of an edge, where the four rounded face tests need not
// agree, are not probed: a ray sample lands there with probability of order
// 1e-32.)
#include <cmath>
#include <cstdint>
#include <cstring>
#include <cstdio>
#include <vector>

#include "tet_build.h"

using namespace dpvr;

static int g_fail = 0;
#define EXPECT(c)                                                           \
    do {                                                                    \
        if (!(c)) {                                                         \
            ++g_fail;                                                       \
            if (g_fail < 20) std::printf("FAILED %s:%d: %s\n", __FILE__, __LINE__, #c); \
        }                                                                   \
    } while (0)

// splitmix64: seeded coordinates for the jitter and the probe points
static uint64_t g_state = 0x9e3779b97f4a7c15ULL;
static double uniform() {
    uint64_t z = (g_state += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1p-53;
}

static bool holds(const TetTables& t, int e, const double p[3]) {
    for (int i = 0; i < 4; ++i) {
        const double* q = &t.planes[16 * (size_t)e + 4 * i];
        const double d = ((q[0] * p[0] + q[1] * p[1]) + q[2] * p[2]) - q[3];
        if (d < 0.0 || (d == 0.0 && !((t.owned[e] >> i) & 1u))) return false;
    }
    return true;
}

static void mesh(int nx, int ny, int nz, double jitter, std::vector<double>& v, std::vector<int32_t>& t) {
    auto vid = [&](int i, int j, int k) { return (i * (ny + 1) + j) * (nz + 1) + k; };
    v.clear();
    t.clear();
    for (int i = 0; i <= nx; ++i)
        for (int j = 0; j <= ny; ++j)
            for (int k = 0; k <= nz; ++k) {
                const bool in = i > 0 && i < nx && j > 0 && j < ny && k > 0 && k < nz;
                const int c[3] = {i, j, k};
                for (int a = 0; a < 3; ++a) {
                    const double d = in ? jitter * (2.0 * uniform() - 1.0) : 0.0;
                    v.push_back(std::round((c[a] + d) * 1024.0) / 1024.0);
                }
            }
    const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j)
            for (int k = 0; k < nz; ++k)
                for (const auto& pm : perms) {
                    int c[3] = {i, j, k};
                    t.push_back(vid(c[0], c[1], c[2]));
                    for (int a = 0; a < 3; ++a) {
                        ++c[pm[a]];
                        t.push_back(vid(c[0], c[1], c[2]));
                    }
                }
}

static void probe(const TetTables& tab, const int dims[3], const double p[3]) {
    int owners = 0, first = -1;
    for (int e = 0; e < tab.n_tets; ++e)
        if (holds(tab, e, p)) {
            if (owners++ == 0) first = e;
        }
    const bool in = p[0] >= 0 && p[0] < dims[0] && p[1] >= 0 && p[1] < dims[1] && p[2] >= 0 && p[2] < dims[2];
    const bool strictly = p[0] > 1e-9 && p[0] < dims[0] - 1e-9 && p[1] > 1e-9 && p[1] < dims[1] - 1e-9 &&
                          p[2] > 1e-9 && p[2] < dims[2] - 1e-9;
    EXPECT(owners <= 1);
    if (strictly) EXPECT(owners == 1);
    if (!in) EXPECT(owners == 0);
    if (owners == 1) {
        // the kernels' cell of p must list the owner
        double u[3];
        bool inside = true;
        for (int c = 0; c < 3; ++c) {
            u[c] = (p[c] - tab.glo[c]) * tab.ginv[c];
            inside = inside && u[c] >= 0.0 && u[c] < (double)tab.gdim[c];
        }
        EXPECT(inside);
        if (!inside) return;
        const size_t cell = ((size_t)(int)u[2] * tab.gdim[1] + (int)u[1]) * tab.gdim[0] + (int)u[0];
        bool listed = false;
        for (int q = tab.cell_start[cell]; q < tab.cell_start[cell + 1]; ++q) listed = listed || tab.cell_tets[q] == first;
        EXPECT(listed);
    }
    // the BVH walk (boxes entered when they hold p, skip links otherwise)
    // finds the same tetrahedron
    int found = -1, node = tab.n_tets > 0 ? 0 : -1;
    while (node >= 0 && found < 0) {
        const int32_t* nd = &tab.bvh_nodes[8 * (size_t)node];
        float b[6];
        for (int c = 0; c < 3; ++c) {
            std::memcpy(&b[c], &nd[c], 4);
            std::memcpy(&b[3 + c], &nd[4 + c], 4);
        }
        const bool in = p[0] >= b[0] && p[1] >= b[1] && p[2] >= b[2] && p[0] <= b[3] && p[1] <= b[4] && p[2] <= b[5];
        if (!in) {
            node = nd[3];
        } else if (nd[7] >= 0) {
            for (int i = 0; i < (nd[7] & 7) && found < 0; ++i)
                if (holds(tab, tab.bvh_tets[(nd[7] >> 3) + i], p)) found = tab.bvh_tets[(nd[7] >> 3) + i];
            node = nd[3];
        } else {
            node = node + 1;
        }
    }
    EXPECT(found == first);
}

int main() {
    const int cases[3][3] = {{3, 3, 3}, {5, 2, 4}, {4, 4, 2}};
    const double jit[3] = {0.0, 0.2, 0.35};
    for (int m = 0; m < 3; ++m) {
        std::vector<double> v;
        std::vector<int32_t> t;
        mesh(cases[m][0], cases[m][1], cases[m][2], jit[m], v, t);
        TetTables tab;
        std::string err;
        EXPECT(build_tet_tables(v.data(), (int32_t)v.size() / 3, t.data(), (int32_t)t.size() / 4, tab, err));
        EXPECT(tab.cell_start.back() == (int32_t)tab.cell_tets.size());
        const int* d = cases[m];
        // lattice of half steps, one step beyond the box on each side
        for (int i = -1; i <= 2 * d[0] + 1; ++i)
            for (int j = -1; j <= 2 * d[1] + 1; ++j)
                for (int k = -1; k <= 2 * d[2] + 1; ++k) {
                    const double p[3] = {0.5 * i, 0.5 * j, 0.5 * k};
                    probe(tab, d, p);
                }
        for (int s = 0; s < 4000; ++s) {
            const double p[3] = {(d[0] + 0.4) * uniform() - 0.2, (d[1] + 0.4) * uniform() - 0.2,
                                 (d[2] + 0.4) * uniform() - 0.2};
            probe(tab, d, p);
        }
        // points on the faces of the jittered tetrahedra: barycentric
        // combinations of three vertices of a face
        for (int s = 0; s < 2000; ++s) {
            const int e = (int)(uniform() * (tab.n_tets - 1));
            const int skip = (int)(uniform() * 3.999);
            double w[3] = {uniform(), uniform(), uniform()};
            const double ws = w[0] + w[1] + w[2];
            double p[3] = {0, 0, 0};
            int m2 = 0;
            for (int j = 0; j < 4; ++j) {
                if (j == skip) continue;
                for (int c = 0; c < 3; ++c) p[c] += (w[m2] / ws) * v[3 * (size_t)t[4 * (size_t)e + j] + c];
                ++m2;
            }
            probe(tab, d, p);
        }
    }
    // rejected input
    {
        std::vector<double> v = {0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 0};
        std::vector<int32_t> t = {0, 1, 2, 3};
        TetTables tab;
        std::string err;
        EXPECT(!build_tet_tables(v.data(), 4, t.data(), 1, tab, err) && err.find("zero volume") != std::string::npos);
        t[3] = 7;
        EXPECT(!build_tet_tables(v.data(), 4, t.data(), 1, tab, err) && err.find("outside") != std::string::npos);
        EXPECT(build_tet_tables(v.data(), 4, t.data(), 0, tab, err) && tab.cell_start.size() == 2);
    }
    std::printf("%s: %d failed expectations\n", g_fail ? "FAIL" : "OK", g_fail);
    return g_fail ? 1 : 0;
}
