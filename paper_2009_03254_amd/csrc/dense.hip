// Dense data-parallel marching cubes over an uncompressed field resident in
// device memory: the standard GPU formulation the paper measures as its
// baseline (Sec. 3.3.3, tab:mc_naive_parallel_perf).  Every cell of the
// volume is classified, the cells that hold the surface are compacted by a
// prefix sum, each of them gets its vertex count, a second prefix sum gives
// the output offsets and the total, and a last pass over the compacted cells
// writes the triangle soup.  No blocks, culling or cache: it measures what
// the block-compressed path's culling buys.
//
// Records are the 16-byte vertices of the block path (block-relative float32
// position + block id), computed with the same operations, so the soup is
// the block path's soup with the cells in global row-major order (x fastest)
// instead of block order.
//
// The two prefix sums run over tiles of 4096 cells: a pass classifies every
// cell and counts each tile's cells with triangles and their vertices, one
// workgroup scans the tile counts, and a pass over the stored cases writes
// the compacted cells with their first vertex (the per-cell vertex counts
// and the second prefix sum come with the first, so no pass of their own).
// No same-address atomics: tiles are indexed by workgroup.
#include <stdint.h>

#include <algorithm>

#include "common.h"
#include "mc_device.h"

namespace bcmc {
namespace {

constexpr int DENSE_SEG = 16;   // cells per thread: a segment of one row of cells

struct DenseCtr {
    unsigned int unused[4];
    unsigned long long n_active, n_verts;
};

// A row of cells is split into segments of DENSE_SEG cells; segment s covers
// cells x in [16 k, min(16 k + 16, nx - 1)) of row r = s / segs_per_row
// (r = y + (ny - 1) z), so the segments in order visit the cells in global
// row-major order.  A tile is 256 segments.
struct DenseGeom {
    uint32_t nx, ny, nz;
    uint32_t segs_per_row;
    uint64_t n_segs;      // segs_per_row * (ny - 1) * (nz - 1)
    uint32_t nbx, nby;    // blocks per row / per layer (for the block ids of the records)
};

// Segment s: first sample of its row, first cell x0, number of cells.
__device__ __forceinline__ void dense_segment(const DenseGeom &g, uint64_t s, uint64_t &row_base, uint32_t &x0,
                                              uint32_t &ncell) {
    const uint32_t r = (uint32_t)(s / g.segs_per_row);
    const uint32_t k = (uint32_t)(s - (uint64_t)r * g.segs_per_row);
    const uint32_t y = r % (g.ny - 1), z = r / (g.ny - 1);
    x0 = DENSE_SEG * k;
    ncell = min((uint32_t)DENSE_SEG, g.nx - 1 - x0);
    row_base = ((uint64_t)z * g.ny + y) * g.nx;
}

// Pass 1: the cases of the segment's cells (stored as the segment's 16
// bytes), and the tile's count of cells whose case is not 0 or 255 and of
// their vertices (3 per triangle), as (vertices << 32 | cells).
__global__ __launch_bounds__(256) void k_dense_classify(DenseGeom g, const float *__restrict__ f, float iso,
                                                       const uint64_t *__restrict__ mc_table,
                                                       uint4 *__restrict__ seg_cases,
                                                       uint64_t *__restrict__ tile_cnt) {
    __shared__ uint8_t s_ntri[256];
    __shared__ uint64_t s_w[4];
    s_ntri[threadIdx.x] = (uint8_t)(mc_table[threadIdx.x] >> 60);
    __syncthreads();
    const uint64_t s = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    uint32_t na = 0, nv = 0;
    if (s < g.n_segs) {
        uint64_t row_base;
        uint32_t x0, ncell;
        dense_segment(g, s, row_base, x0, ncell);
        const uint64_t sy = g.nx, sz = (uint64_t)g.nx * g.ny;
        // the four sample rows of the segment, DENSE_SEG + 1 samples each
        float v[4][DENSE_SEG + 1];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const float *p = f + row_base + x0 + (q & 1) * sy + (q >> 1) * sz;
#pragma unroll
            for (int j = 0; j <= DENSE_SEG; j++) v[q][j] = j <= (int)ncell ? p[j] : 0.0f;
        }
        uint32_t cw[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int j = 0; j < DENSE_SEG; j++) {
            uint32_t c = 0;
#pragma unroll
            for (int kk = 0; kk < 8; kk++)
                c |= (v[((kk >> 1) & 1) | ((kk >> 2) << 1)][j + (kk & 1)] < iso ? 1u : 0u) << kk;
            cw[j >> 2] |= c << (8 * (j & 3));
            if (j < (int)ncell && c != 0u && c != 255u) {
                na++;
                nv += 3u * s_ntri[c];
            }
        }
        seg_cases[s] = make_uint4(cw[0], cw[1], cw[2], cw[3]);
    }
    uint64_t x = wave_sum(((uint64_t)nv << 32) | na);
    if (lane() == 0) s_w[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) tile_cnt[blockIdx.x] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

// Pass 2 (one workgroup): exclusive prefix of the tiles' counts, tile_off[2t]
// = cells before tile t, tile_off[2t + 1] = vertices before it; the totals.
__global__ __launch_bounds__(256) void k_dense_scan(const uint64_t *__restrict__ tile_cnt, uint64_t n_tiles,
                                                   uint64_t *__restrict__ tile_off, DenseCtr *ctr) {
    __shared__ uint64_t s_a[4], s_v[4];
    const int w = threadIdx.x >> 6;
    uint64_t ca = 0, cv = 0;   // carries
    for (uint64_t c0 = 0; c0 < n_tiles; c0 += 4096) {
        const uint64_t i0 = c0 + 16u * threadIdx.x;
        uint64_t t[16], sa = 0, sv = 0;
#pragma unroll
        for (int j = 0; j < 16; j++) {
            t[j] = i0 + j < n_tiles ? tile_cnt[i0 + j] : 0ull;
            sa += t[j] & 0xFFFFFFFFull;
            sv += t[j] >> 32;
        }
        const uint64_t ia = wave_incl_scan(sa), iv = wave_incl_scan(sv);
        if (lane() == 63) {
            s_a[w] = ia;
            s_v[w] = iv;
        }
        __syncthreads();
        uint64_t oa = ca + ia - sa, ov = cv + iv - sv, ta = 0, tv = 0;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            if (i < w) {
                oa += s_a[i];
                ov += s_v[i];
            }
            ta += s_a[i];
            tv += s_v[i];
        }
#pragma unroll
        for (int j = 0; j < 16; j++) {
            if (i0 + j < n_tiles) {
                tile_off[2 * (i0 + j)] = oa;
                tile_off[2 * (i0 + j) + 1] = ov;
            }
            oa += t[j] & 0xFFFFFFFFull;
            ov += t[j] >> 32;
        }
        ca += ta;
        cv += tv;
        __syncthreads();   // s_a / s_v are rewritten by the next step
    }
    if (threadIdx.x == 0) {
        ctr->n_active = ca;
        ctr->n_verts = cv;
    }
}

// Pass 3: the cells with triangles, in order: id (index of the cell's lowest
// sample), case, first vertex (the tile's offsets plus a workgroup scan).
__global__ __launch_bounds__(256) void k_dense_compact(DenseGeom g, const uint4 *__restrict__ seg_cases,
                                                      const uint64_t *__restrict__ tile_off,
                                                      const uint64_t *__restrict__ mc_table,
                                                      uint32_t *__restrict__ ids, uint8_t *__restrict__ cases,
                                                      uint64_t *__restrict__ first) {
    __shared__ uint8_t s_ntri[256];
    __shared__ uint32_t s_w[4];
    s_ntri[threadIdx.x] = (uint8_t)(mc_table[threadIdx.x] >> 60);
    __syncthreads();
    const uint64_t s = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    uint32_t cw[4] = {0u, 0u, 0u, 0u}, act = 0, x0 = 0, ncell = 0;
    uint64_t row_base = 0;
    uint32_t na = 0, nv = 0;
    if (s < g.n_segs) {
        dense_segment(g, s, row_base, x0, ncell);
        const uint4 q = seg_cases[s];
        cw[0] = q.x; cw[1] = q.y; cw[2] = q.z; cw[3] = q.w;
#pragma unroll
        for (int j = 0; j < DENSE_SEG; j++) {
            const uint32_t c = (cw[j >> 2] >> (8 * (j & 3))) & 0xFFu;
            if (j < (int)ncell && c != 0u && c != 255u) {
                act |= 1u << j;
                na++;
                nv += 3u * s_ntri[c];
            }
        }
    }
    // per thread na <= 16, nv <= 240; per workgroup na < 2^13, nv < 2^16
    const uint32_t packed = na | (nv << 13);
    const uint32_t incl = wave_incl_scan(packed);
    if (lane() == 63) s_w[threadIdx.x >> 6] = incl;
    __syncthreads();
    uint32_t ex = incl - packed;
#pragma unroll
    for (int i = 0; i < 4; i++)
        if (i < (int)(threadIdx.x >> 6)) ex += s_w[i];
    uint64_t o = tile_off[2 * (uint64_t)blockIdx.x] + (ex & 0x1FFFu);
    uint64_t ov = tile_off[2 * (uint64_t)blockIdx.x + 1] + (ex >> 13);
    for (uint32_t m = act; m; m &= m - 1) {
        const int j = __builtin_ctz(m);
        const uint32_t c = (cw[j >> 2] >> (8 * (j & 3))) & 0xFFu;
        ids[o] = (uint32_t)(row_base + x0 + (uint32_t)j);
        cases[o] = (uint8_t)c;
        first[o] = ov;
        o++;
        ov += 3u * s_ntri[c];
    }
}

// Pass 4: one thread per compacted cell writes its triangles' vertices from
// its first vertex on (records past cap dropped).
__global__ __launch_bounds__(256) void k_dense_emit(DenseGeom g, const float *__restrict__ f, float iso,
                                                   const uint32_t *__restrict__ ids,
                                                   const uint8_t *__restrict__ cases,
                                                   const uint64_t *__restrict__ first,
                                                   const uint64_t *__restrict__ mc_table,
                                                   void *__restrict__ out, uint64_t cap,
                                                   const DenseCtr *ctr) {
    __shared__ uint64_t s_tab[256];
    for (int i = threadIdx.x; i < 256; i += 256) s_tab[i] = mc_table[i];
    __syncthreads();
    const uint64_t n = ctr->n_active;
    const uint64_t sy = g.nx, sz = (uint64_t)g.nx * g.ny;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t id = ids[i];
        const uint32_t x = id % g.nx, r = id / g.nx, y = r % g.ny, z = r / g.ny;
        float v[8];
#pragma unroll
        for (int k = 0; k < 8; k++)
            v[k] = f[id + (k & 1) + ((k >> 1) & 1) * sy + (k >> 2) * sz];
        const uint64_t tb = s_tab[cases[i]];
        const int nv = 3 * (int)(tb >> 60);
        const uint32_t b = (x >> 2) + g.nbx * ((y >> 2) + g.nby * (z >> 2));
        const int cx = (int)(x & 3), cy = (int)(y & 3), cz = (int)(z & 3);
        uint64_t o = first[i];
        for (int j = 0; j < nv; j++, o++) {
            const int e = (int)((tb >> (4 * j)) & 15u);
            const uint32_t d = (uint32_t)(kEdgeGeom >> (5 * e)) & 31u;
            const int axis = (int)(d >> 3);
            const int k0 = (int)(d & 7u);            // first corner (ox | oy << 1 | oz << 2)
            const int k1 = k0 | (1 << axis);
            const float a = v[k0], bv = v[k1];
            const float tt = (iso - a) / (bv - a);
            const float px = (float)(cx + (int)(d & 1u)) + (axis == 0 ? tt : 0.0f);
            const float py = (float)(cy + (int)((d >> 1) & 1u)) + (axis == 1 ? tt : 0.0f);
            const float pz = (float)(cz + (int)((d >> 2) & 1u)) + (axis == 2 ? tt : 0.0f);
            if (o < cap) store_record(out, o, px, py, pz, b);
        }
    }
}

}  // namespace

// 64-bit words of work memory: the segments' cases (2 words each), the
// tiles' counts (1) and offsets (2).
uint64_t dense_work_words(uint32_t nx, uint32_t ny, uint32_t nz) {
    const uint64_t segs = (uint64_t)((nx - 2) / DENSE_SEG + 1) * (ny - 1) * (nz - 1);
    const uint64_t tiles = (segs + 255) / 256;
    return 2 * segs + 3 * tiles;
}

uint64_t dense_counter_bytes() { return sizeof(DenseCtr); }

// ids, cases, first: per cell of the volume at most; work: see above;
// ctr: dense_counter_bytes().  The counters' n_active and n_verts (u64 at
// byte offsets 16 and 24) are valid when the stream reaches the end.
void launch_dense(uint32_t nx, uint32_t ny, uint32_t nz, const float *field, float iso,
                  uint32_t *ids, uint8_t *cases, uint64_t *first, uint64_t *work,
                  void *ctr_mem, const uint64_t *mc_table, void *out, uint64_t cap, hipStream_t s) {
    DenseGeom g;
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.segs_per_row = (nx - 2) / DENSE_SEG + 1;
    g.n_segs = (uint64_t)g.segs_per_row * (ny - 1) * (nz - 1);
    g.nbx = (nx + 3) / 4;
    g.nby = (ny + 3) / 4;
    DenseCtr *ctr = reinterpret_cast<DenseCtr *>(ctr_mem);
    const uint64_t tiles = (g.n_segs + 255) / 256;
    uint4 *seg_cases = reinterpret_cast<uint4 *>(work);
    uint64_t *tile_cnt = work + 2 * g.n_segs, *tile_off = tile_cnt + tiles;
    k_dense_classify<<<(unsigned)tiles, 256, 0, s>>>(g, field, iso, mc_table, seg_cases, tile_cnt);
    k_dense_scan<<<1, 256, 0, s>>>(tile_cnt, tiles, tile_off, ctr);
    k_dense_compact<<<(unsigned)tiles, 256, 0, s>>>(g, seg_cases, tile_off, mc_table, ids, cases, first);
    const uint64_t cells = (uint64_t)(nx - 1) * (ny - 1) * (nz - 1);
    k_dense_emit<<<(unsigned)std::min<uint64_t>((cells + 255) / 256, 8192), 256, 0, s>>>(
        g, field, iso, ids, cases, first, mc_table, out, cap, ctr);
}

}  // namespace bcmc
