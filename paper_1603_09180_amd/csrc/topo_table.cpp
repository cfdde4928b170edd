// topo_table.cpp -- connectivity table of the 3x3 characterisation, generated
// on the host from the definitions of section 2.1 (T+ = #C_n[x, Gamma+],
// T-- = #C_n'[x, Gamma--], destructible <=> T+ = 1 and T-- = 1; for the
// lambda-skeleton also peak points, T+ = 0, and end points, exactly one
// n-neighbour in the section of the point's own level).
//
// The kernels index it by the upper-neighbour mask U (bit p set when ring
// neighbour p has F >= F(x)); the lower set is L = ~U.  The ring positions
// 0..7 are E, NE, N, NW, W, SW, S, SE: even positions are the 4-neighbours of
// the centre, odd positions its corners.  On this cycle two ring pixels are
// 4-adjacent exactly when they are consecutive, and 8-adjacent when they are
// consecutive or when both are 4-neighbours of the centre two steps apart
// (E and N touch diagonally; two corners never do).  A component of a ring
// subset counts for C_m[x, .] when one of its pixels is m-adjacent to the
// centre: any pixel for m = 8, an even position for m = 4.
#include "thin_internal.h"

namespace thin {
namespace {

bool ring_adjacent(int p, int q, int m)
{
    int d = (p - q + 8) % 8;
    if (d > 4) d = 8 - d;
    if (d == 1) return true;
    return m == 8 && d == 2 && (p % 2 == 0) && (q % 2 == 0);
}

int find(int* parent, int a)
{
    while (parent[a] != a) a = parent[a] = parent[parent[a]];
    return a;
}

// Components of `set` (8-bit ring mask) under m-adjacency that touch the
// centre.  Writes their ring masks, ordered by lowest ring position, into
// masks[]; returns their number.
int counted_components(unsigned set, int m, unsigned masks[8])
{
    int parent[8];
    for (int p = 0; p < 8; ++p) parent[p] = p;
    for (int p = 0; p < 8; ++p)
        for (int q = p + 1; q < 8; ++q)
            if ((set >> p & 1) && (set >> q & 1) && ring_adjacent(p, q, m)) {
                int a = find(parent, p), b = find(parent, q);
                if (a != b) parent[b] = a;
            }
    unsigned by_root[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int p = 0; p < 8; ++p)
        if (set >> p & 1) by_root[find(parent, p)] |= 1u << p;
    int n = 0;
    const unsigned touching = (m == 8) ? 0xFFu : 0x55u;  // positions adjacent to the centre
    for (int p = 0; p < 8; ++p) {          // roots visited in ring order
        unsigned comp = 0;
        for (int r = 0; r < 8; ++r)
            if (by_root[r] && (by_root[r] & -by_root[r]) == (1u << p)) comp = by_root[r];
        if (comp && (comp & touching)) masks[n++] = comp;
    }
    return n;
}

}  // namespace

void build_topology_table(int adjacency, int op, TopoEntry out[256])
{
    const int n = adjacency == 0 ? 8 : 4;
    const int nbar = adjacency == 0 ? 4 : 8;
    const unsigned n_neighbours = (n == 8) ? 0xFFu : 0x55u;
    for (unsigned u = 0; u < 256; ++u) {
        unsigned up[8], lo[8];
        const int tplus = counted_components(u, n, up);
        const int tminus = counted_components(~u & 0xFFu, nbar, lo);
        uint32_t comps = 0;
        for (int c = 0; c < tminus && c < 4; ++c) comps |= (uint32_t)lo[c] << (8 * c);
        const uint32_t destructible = (tplus == 1 && tminus == 1) ? 1u : 0u;
        uint32_t flags = destructible | ((uint32_t)tminus << 4) | ((uint32_t)tplus << 8);
        if (op == 1) {
            // peak: T+ = 0; end point: exactly one n-neighbour in Gamma+
            if (tplus == 0) flags |= 2u;
            if (__builtin_popcount(u & n_neighbours) == 1) flags |= 4u;
        }
        out[u].flags = flags;
        out[u].comps = comps;
    }
}

}  // namespace thin
