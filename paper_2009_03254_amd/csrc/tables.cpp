// Marching cubes case table of libbcmc, generated on the host at load time
// (the paper uses Lorensen-Cline marching cubes, Sec. 3.3.3, and prints no
// table).  The construction is this library's own:
//
//   Corner k sits at (k&1, (k>>1)&1, (k>>2)&1); edge e runs along axis e>>2
//   and bits 0/1 of e are its offsets on the other two axes in increasing
//   axis order.  A corner is inside when its value is below the isovalue.
//
//   Face walk: on every cube face, walk its four corners counter-clockwise
//   around the outward normal.  Each maximal run of inside corners is entered
//   through one crossing edge and left through another; the contour segment
//   on that face goes from the entering edge to the leaving edge.  (On a face
//   with two diagonal inside corners this separates them.)  Going from
//   entering to leaving edge with the inside on the walk's left keeps the
//   surface normal pointing toward increasing values.
//
//   The segments form closed polygons.  Polygons are listed by their smallest
//   edge id; walking each from that edge, the fan apex is the first vertex none
//   of whose fan diagonals joins two edges lying in a common face.
//
// Packed form per case: bits 4k..4k+3 hold the k-th edge id of the triangle
// list (15 when unused), bits 60..63 the number of triangles.
#include <stdint.h>

#include "common.h"

namespace bcmc {
namespace {

int corner_of(int x, int y, int z) { return x | (y << 1) | (z << 2); }

// Edge joining two corners that differ along exactly one axis.
int edge_between(int ka, int kb) {
    int diff = ka ^ kb;
    int axis = diff == 1 ? 0 : (diff == 2 ? 1 : 2);
    int lo = (axis == 0) ? 1 : 0;      // the two other axes, increasing
    int hi = (axis == 2) ? 1 : 2;
    int bit_lo = (ka >> lo) & 1, bit_hi = (ka >> hi) & 1;
    return (axis << 2) | bit_lo | (bit_hi << 1);
}

// Offset of edge e along axis f (f must differ from the edge's own axis).
int edge_offset(int e, int f) {
    int axis = e >> 2;
    int lo = (axis == 0) ? 1 : 0;
    return (f == lo) ? (e & 1) : ((e >> 1) & 1);
}

// Closed form: parallel edges share a face when they agree on one offset;
// edges along axes a and b share a face when they agree along the third axis.
bool share_face(int e1, int e2) {
    int a1 = e1 >> 2, a2 = e2 >> 2;
    if (e1 == e2) return true;
    if (a1 == a2) return ((e1 ^ e2) & 1) == 0 || ((e1 ^ e2) & 2) == 0;
    int f = 3 - a1 - a2;
    return edge_offset(e1, f) == edge_offset(e2, f);
}

int build_case(int cs, int *tri) {
    int succ[12];
    for (int e = 0; e < 12; e++) succ[e] = -1;
    for (int f = 0; f < 3; f++) {
        int u = (f + 1) % 3, v = (f + 2) % 3;  // e_u x e_v = e_f
        for (int side = 0; side < 2; side++) {
            // counter-clockwise about the outward normal (+e_f or -e_f)
            static const int ccw[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
            int ring[4];
            for (int i = 0; i < 4; i++) {
                int j = side ? i : (4 - i) % 4;  // reverse the walk for -e_f
                int p[3];
                p[f] = side;
                p[u] = ccw[j][0];
                p[v] = ccw[j][1];
                ring[i] = corner_of(p[0], p[1], p[2]);
            }
            for (int i = 0; i < 4; i++) {
                int prev = ring[(i + 3) % 4], cur = ring[i];
                bool in_prev = (cs >> prev) & 1, in_cur = (cs >> cur) & 1;
                if (!in_cur || in_prev) continue;  // not the start of an inside run
                int j = i;
                while ((cs >> ring[(j + 1) % 4]) & 1) j = (j + 1) % 4;
                int enter = edge_between(prev, cur);
                int leave = edge_between(ring[j], ring[(j + 1) % 4]);
                if (succ[enter] != -1) return -1;
                succ[enter] = leave;
            }
        }
    }
    int n = 0;
    bool seen[12] = {false};
    for (int e = 0; e < 12; e++) {
        if (succ[e] < 0 || seen[e]) continue;
        int poly[12], m = 0;
        for (int c = e; !seen[c]; c = succ[c]) {
            if (succ[c] < 0 || m == 12) return -1;
            seen[c] = true;
            poly[m++] = c;
        }
        int apex = -1;
        for (int a = 0; a < m && apex < 0; a++) {
            bool ok = true;
            for (int d = 2; d + 1 < m; d++)
                if (share_face(poly[a], poly[(a + d) % m])) ok = false;
            if (ok) apex = a;
        }
        if (apex < 0) return -1;
        for (int d = 1; d + 1 < m; d++) {
            if (n == 5) return -1;
            tri[3 * n] = poly[apex];
            tri[3 * n + 1] = poly[(apex + d) % m];
            tri[3 * n + 2] = poly[(apex + d + 1) % m];
            n++;
        }
    }
    return n;
}

struct Table {
    uint64_t packed[256];
    int status = 0;
    Table() {
        for (int cs = 0; cs < 256; cs++) {
            int tri[15];
            int n = build_case(cs, tri);
            if (n < 0) {
                status = -1;
                n = 0;
            }
            uint64_t w = (uint64_t)n << 60;
            for (int k = 0; k < 15; k++)
                w |= (uint64_t)(k < 3 * n ? tri[k] : 15) << (4 * k);
            packed[cs] = w;
        }
    }
};

const Table &table() {
    static const Table t;
    return t;
}

}  // namespace

const uint64_t *mc_table_host() { return table().packed; }
int mc_table_status() { return table().status; }

}  // namespace bcmc
