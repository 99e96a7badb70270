// Closed-form index arithmetic of the periodic pyrochlore lattice
// (16-site cubic cell, L^3 cells; Sec. 2 of the paper, Fig. 1).
//
// Geometry, in units of a/4: cell (x,y,z) has index (z*L + y)*L + x; site
// (cell, f, mu) has index 16*cell + 4f + mu and sits at 4(x,y,z) + F_f + B_mu
// with F = (0,0,0),(0,2,2),(2,0,2),(2,2,0) and B = (0,0,0),(0,1,1),(1,0,1),
// (1,1,0).  Because F_mu = 2 B_mu, the "down" tetrahedron {R - B_mu} around
// the FCC point R = 4c + F_f has vertex mu at site (c + D(f,mu), f xor mu,
// mu), where D(f,mu) = floor((F_f - F_mu)/4) is 0 or -1 per axis:
//   D_x = -1 iff f in {0,1} and mu in {2,3}
//   D_y = -1 iff f in {0,2} and mu in {1,3}
//   D_z = -1 iff f in {0,3} and mu in {1,2}
// The "up" tetrahedron {R + B_mu} is (c, f, mu), mu = 0..3, inside the cell.
//
// Bonds: cell c owns 48 bonds, b = 48 c + 6 t + e, t = f (up) or 4 + f
// (down), e = vertex pair (0,1),(0,2),(0,3),(1,2),(1,3),(2,3).  Each bond is
// an edge of exactly one tetrahedron, so the 3N bonds are enumerated once.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pyro {

// Neighbouring cells a down tetrahedron reaches: offsets from the owner.
enum : int { kSelf = 0, kMx = 1, kMy = 2, kMz = 3, kMyMz = 4, kMxMz = 5, kMxMy = 6, kNCellCodes = 7 };

struct SiteRef {
    uint8_t cell;  // one of the cell codes above
    uint8_t site;  // 4*f' + mu within that cell
};

// Down tetrahedron of FCC point f of cell c: vertex mu -> (cell code, site).
__host__ __device__ constexpr SiteRef down_vertex(int f, int mu)
{
    constexpr SiteRef table[4][4] = {
        {{kSelf, 0}, {kMyMz, 5}, {kMxMz, 10}, {kMxMy, 15}},
        {{kSelf, 4}, {kSelf, 1}, {kMx, 14}, {kMx, 11}},
        {{kSelf, 8}, {kMy, 13}, {kSelf, 2}, {kMy, 7}},
        {{kSelf, 12}, {kMz, 9}, {kMz, 6}, {kSelf, 3}},
    };
    return table[f][mu];
}

__host__ __device__ constexpr int pair_a(int e) { return e < 3 ? 0 : (e < 5 ? 1 : 2); }
__host__ __device__ constexpr int pair_b(int e) { return e < 3 ? e + 1 : (e < 5 ? e - 1 : 3); }

// Endpoints of bond j (0..47) of a cell.
__host__ __device__ constexpr SiteRef bond_end_a(int j)
{
    return (j / 6) < 4 ? SiteRef{kSelf, (uint8_t)(4 * (j / 6) + pair_a(j % 6))}
                       : down_vertex(j / 6 - 4, pair_a(j % 6));
}
__host__ __device__ constexpr SiteRef bond_end_b(int j)
{
    return (j / 6) < 4 ? SiteRef{kSelf, (uint8_t)(4 * (j / 6) + pair_b(j % 6))}
                       : down_vertex(j / 6 - 4, pair_b(j % 6));
}

// The seven cells a cell's bonds touch (periodic wrap).
struct CellNbrs {
    int c[kNCellCodes];
};

__host__ __device__ __forceinline__ CellNbrs cell_neighbours(int cell, int L)
{
    const int x = cell % L;
    const int y = (cell / L) % L;
    const int z = cell / (L * L);
    const int xm = x == 0 ? L - 1 : x - 1;
    const int ym = y == 0 ? L - 1 : y - 1;
    const int zm = z == 0 ? L - 1 : z - 1;
    CellNbrs n;
    n.c[kSelf] = cell;
    n.c[kMx] = (z * L + y) * L + xm;
    n.c[kMy] = (z * L + ym) * L + x;
    n.c[kMz] = (zm * L + y) * L + x;
    n.c[kMyMz] = (zm * L + ym) * L + x;
    n.c[kMxMz] = (zm * L + y) * L + xm;
    n.c[kMxMy] = (z * L + ym) * L + xm;
    return n;
}

}  // namespace pyro
