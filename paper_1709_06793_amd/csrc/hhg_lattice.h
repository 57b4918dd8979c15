// hhg_lattice.h -- index arithmetic of one uniformly refined macro tetrahedron.
//
// A macro tet refined l times (n = 2^l) holds the lattice points (i,j,k),
// i,j,k >= 0, i+j+k <= n; (n-i-j-k, i, j, k)/n are the barycentric coordinates
// with respect to the tet's vertices v0..v3.  Bey's refinement (Sec. 2.1)
// splits the tet into n^3 elements of six lattice shapes: the "up" tet at base
// b, {b, b+e1, b+e2, b+e3}; the octahedron over b+{e1,e2,e3,e1+e2,e1+e3,e2+e3}
// cut along its diagonal b+e2 -- b+e1+e3 into four tets; and the "down" tet
// {b+e1+e2, b+e1+e3, b+e2+e3, b+e1+e2+e3}.  Every interior node touches 24
// elements and 14 neighbours (Sec. 2.2, Fig. 1), along +-e1, +-e2, +-e3,
// +-(e1-e2), +-(e1-e3), +-(e2-e3) and +-(e1-e2+e3) (the octahedron diagonal,
// the "gray" edge of Fig. 5).
//
// Storage: points ordered by plane k, then anti-diagonal s = i + j, then i.
// Along an anti-diagonal the +-(e1-e2) neighbours are adjacent slots, and all
// 14 neighbours sit at offsets that depend only on s and the plane.
#pragma once
#include <stdint.h>

#ifdef __HIPCC__
#define HHG_HD __host__ __device__ __forceinline__
#else
#define HHG_HD inline
#endif

namespace hhg {

constexpr int NDIR = 14;   // neighbour directions; index 14 = the centre
// direction d and its opposite d+7
constexpr int DIR[NDIR][3] = {
    {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, -1, 0}, {1, 0, -1}, {0, 1, -1}, {1, -1, 1},
    {-1, 0, 0}, {0, -1, 0}, {0, 0, -1}, {-1, 1, 0}, {-1, 0, 1}, {0, -1, 1}, {-1, 1, -1}};

// six element shapes, vertex offsets from the base point
constexpr int NTYPE = 6;
constexpr int TYPE_OFF[NTYPE][4][3] = {
    {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}},   // up
    {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 0, 1}},   // octahedron pieces sharing
    {{1, 0, 0}, {0, 1, 0}, {1, 1, 0}, {1, 0, 1}},   //   the diagonal e2 -- e1+e3
    {{0, 1, 0}, {0, 0, 1}, {1, 0, 1}, {0, 1, 1}},
    {{0, 1, 0}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}},
    {{1, 1, 0}, {1, 0, 1}, {0, 1, 1}, {1, 1, 1}}};  // down

// index of direction (a,b,c) in DIR, 14 for (0,0,0), -1 otherwise
HHG_HD constexpr int dir_index(int a, int b, int c)
{
    return (a == 0 && b == 0 && c == 0) ? 14
         : (a == 1 && b == 0 && c == 0) ? 0
         : (a == 0 && b == 1 && c == 0) ? 1
         : (a == 0 && b == 0 && c == 1) ? 2
         : (a == 1 && b == -1 && c == 0) ? 3
         : (a == 1 && b == 0 && c == -1) ? 4
         : (a == 0 && b == 1 && c == -1) ? 5
         : (a == 1 && b == -1 && c == 1) ? 6
         : (a == -1 && b == 0 && c == 0) ? 7
         : (a == 0 && b == -1 && c == 0) ? 8
         : (a == 0 && b == 0 && c == -1) ? 9
         : (a == -1 && b == 1 && c == 0) ? 10
         : (a == -1 && b == 0 && c == 1) ? 11
         : (a == 0 && b == -1 && c == 1) ? 12
         : (a == -1 && b == 1 && c == -1) ? 13 : -1;
}

// number of lattice points with i+j+k <= m (m >= -1)
HHG_HD int64_t tet_count(int64_t m) { return (m + 1) * (m + 2) * (m + 3) / 6; }
// number of lattice points with i+j <= m in one plane
HHG_HD int64_t tri_count(int64_t m) { return (m + 1) * (m + 2) / 2; }

// slot of (i,j,k) inside one tet lattice of size n: planes k in turn; inside a
// plane the anti-diagonals s = i + j in turn (positions i = 0..s).  A plane
// with m = n - k holds (m+1)(m+2)/2 points.
HHG_HD int64_t slot_of(int n, int i, int j, int k)
{
    const int64_t s = i + j;
    return tet_count(n) - tet_count(n - k) + s * (s + 1) / 2 + i;
}
// first slot of plane k
HHG_HD int64_t plane_start(int n, int k) { return tet_count(n) - tet_count(n - k); }

// zero pattern of the barycentric weights: bit a set iff weight a is zero.
// 0 = tet interior, one bit = face opposite vertex a, two bits = edge,
// three bits = vertex.  Used as the primitive "kind" (0..14).
HHG_HD int zero_pattern(int n, int i, int j, int k)
{
    return (n - i - j - k == 0 ? 1 : 0) | (i == 0 ? 2 : 0) | (j == 0 ? 4 : 0) | (k == 0 ? 8 : 0);
}

HHG_HD bool in_lattice(int n, int i, int j, int k)
{
    return i >= 0 && j >= 0 && k >= 0 && i + j + k <= n;
}

// packed reference to one copy of a node: tet (16 bits) | kind (4) | i,j,k (14 each)
HHG_HD uint64_t pack_copy(int tet, int kind, int i, int j, int k)
{
    return ((uint64_t)tet << 46) | ((uint64_t)kind << 42) | ((uint64_t)i << 28) |
           ((uint64_t)j << 14) | (uint64_t)k;
}
HHG_HD void unpack_copy(uint64_t c, int &tet, int &kind, int &i, int &j, int &k)
{
    tet = (int)(c >> 46);
    kind = (int)((c >> 42) & 15);
    i = (int)((c >> 28) & 16383);
    j = (int)((c >> 14) & 16383);
    k = (int)(c & 16383);
}

}  // namespace hhg
