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
#include <stdint.h>

#include <algorithm>

#include "common.h"
#include "mc_device.h"

namespace bcmc {
namespace {

constexpr int DENSE_SEG = 16;   // cells per thread: a segment of one row of cells

struct DenseCtr {
    unsigned int tile_cls, tile_cnt;   // tile tickets of the two scans
    unsigned int err;
    unsigned int pad;
    unsigned long long n_active, n_verts;
};

// A row of cells is split into segments of DENSE_SEG cells; segment s covers
// cells x in [16 k, min(16 k + 16, nx - 1)) of row r = s / segs_per_row
// (r = y + (ny - 1) z), so the segments in order visit the cells in global
// row-major order.
struct DenseGeom {
    uint32_t nx, ny, nz;
    uint32_t segs_per_row;
    uint64_t n_segs;      // segs_per_row * (ny - 1) * (nz - 1)
    uint32_t nbx, nby;    // blocks per row / per layer (for the block ids of the records)
};

// Pass 1: classify the cells of a tile (256 segments), and compact the ids
// (index of the cell's lowest sample) and cases of those whose case is not
// 0 or 255, in order, by a single-pass scan with decoupled look-back.
__global__ __launch_bounds__(256) void k_dense_classify(DenseGeom g, const float *__restrict__ f,
                                                       float iso, uint32_t *__restrict__ ids,
                                                       uint8_t *__restrict__ cases, DenseCtr *ctr,
                                                       uint64_t *status) {
    const uint64_t n_tiles = (g.n_segs + 255) / 256;
    const uint32_t t = take_tile(&ctr->tile_cls);
    if (t >= n_tiles) return;
    const uint64_t s = (uint64_t)t * 256 + threadIdx.x;
    uint32_t cs[DENSE_SEG];
    uint32_t act = 0, x0 = 0, ncell = 0;
    uint64_t row_base = 0;
    if (s < g.n_segs) {
        const uint32_t r = (uint32_t)(s / g.segs_per_row);
        const uint32_t k = (uint32_t)(s - (uint64_t)r * g.segs_per_row);
        const uint32_t y = r % (g.ny - 1), z = r / (g.ny - 1);
        x0 = DENSE_SEG * k;
        ncell = min((uint32_t)DENSE_SEG, g.nx - 1 - x0);
        row_base = ((uint64_t)z * g.ny + y) * g.nx;
        const uint64_t sx = 1, sy = g.nx, sz = (uint64_t)g.nx * g.ny;
        // the four sample rows of the segment, DENSE_SEG + 1 samples each
        float v[4][DENSE_SEG + 1];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const float *p = f + row_base + x0 + (q & 1) * sy + (q >> 1) * sz;
#pragma unroll
            for (int j = 0; j <= DENSE_SEG; j++) v[q][j] = j <= (int)ncell ? p[j] : 0.0f;
        }
        (void)sx;
#pragma unroll
        for (int j = 0; j < DENSE_SEG; j++) {
            uint32_t c = 0;
#pragma unroll
            for (int kk = 0; kk < 8; kk++)
                c |= (v[((kk >> 1) & 1) | ((kk >> 2) << 1)][j + (kk & 1)] < iso ? 1u : 0u) << kk;
            cs[j] = c;
            if (j < (int)ncell && c != 0u && c != 255u) act |= 1u << j;
        }
    }
    uint64_t total;
    const uint64_t base = tile_scan_lookback((uint64_t)__popc(act), status, t, &total);
    uint64_t o = base;
    for (uint32_t m = act; m; m &= m - 1) {
        const int j = __builtin_ctz(m);
        ids[o] = (uint32_t)(row_base + x0 + (uint32_t)j);
        cases[o] = (uint8_t)cs[j];
        o++;
    }
    if (t == n_tiles - 1 && threadIdx.x == 0) ctr->n_active = total;
}

// Pass 2: the vertex count of every compacted cell (3 per triangle of its
// case) and their exclusive prefix sum (decoupled look-back): each cell's
// first vertex, and the total.
__global__ __launch_bounds__(256) void k_dense_count(const uint8_t *__restrict__ cases,
                                                    const uint64_t *__restrict__ mc_table,
                                                    uint64_t *__restrict__ first, DenseCtr *ctr,
                                                    uint64_t *status) {
    __shared__ uint8_t s_ntri[256];
    for (int i = threadIdx.x; i < 256; i += 256) s_ntri[i] = (uint8_t)(mc_table[i] >> 60);
    __syncthreads();
    const uint64_t n = ctr->n_active;
    const uint64_t n_tiles = (n + 256 * DENSE_SEG - 1) / (256 * DENSE_SEG);
    const uint32_t t = take_tile(&ctr->tile_cnt);
    if (t >= n_tiles) return;
    const uint64_t i0 = (uint64_t)t * 256 * DENSE_SEG + (uint64_t)threadIdx.x * DENSE_SEG;
    uint32_t c[DENSE_SEG], sum = 0;
#pragma unroll
    for (int j = 0; j < DENSE_SEG; j++) {
        c[j] = i0 + j < n ? 3u * s_ntri[cases[i0 + j]] : 0u;
        sum += c[j];
    }
    uint64_t total;
    uint64_t o = tile_scan_lookback(sum, status, t, &total);
#pragma unroll
    for (int j = 0; j < DENSE_SEG; j++) {
        if (i0 + j < n) first[i0 + j] = o;
        o += c[j];
    }
    if (t == n_tiles - 1 && threadIdx.x == 0) ctr->n_verts = total;
}

// Pass 3: one thread per compacted cell writes its triangles' vertices from
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

__global__ void k_dense_reset(DenseCtr *ctr, uint64_t *status, uint64_t n_status) {
    const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i == 0) *ctr = DenseCtr{};
    for (uint64_t w = i; w < n_status; w += (uint64_t)gridDim.x * blockDim.x) status[w] = 0;
}

}  // namespace

// Look-back status words the two scans need (classification tiles, then
// count tiles: at most one per 4096 cells).
uint64_t dense_status_words(uint32_t nx, uint32_t ny, uint32_t nz) {
    const uint64_t segs = (uint64_t)((nx - 2) / DENSE_SEG + 1) * (ny - 1) * (nz - 1);
    const uint64_t cells = (uint64_t)(nx - 1) * (ny - 1) * (nz - 1);
    return (segs + 255) / 256 + (cells + 256 * DENSE_SEG - 1) / (256 * DENSE_SEG) + 2;
}

uint64_t dense_counter_bytes() { return sizeof(DenseCtr); }

// ids, cases, first: per cell of the volume at most; status: see above;
// ctr: dense_counter_bytes().  The counters' n_active and n_verts (u64 at
// byte offsets 16 and 24) are valid when the stream reaches the end.
void launch_dense(uint32_t nx, uint32_t ny, uint32_t nz, const float *field, float iso,
                  uint32_t *ids, uint8_t *cases, uint64_t *first, uint64_t *status,
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
    const uint64_t n_status = dense_status_words(nx, ny, nz);
    const uint64_t cls_tiles = (g.n_segs + 255) / 256;
    k_dense_reset<<<256, 256, 0, s>>>(ctr, status, n_status);
    k_dense_classify<<<(unsigned)cls_tiles, 256, 0, s>>>(g, field, iso, ids, cases, ctr, status);
    const uint64_t cells = (uint64_t)(nx - 1) * (ny - 1) * (nz - 1);
    const uint64_t cnt_tiles = (cells + 256 * DENSE_SEG - 1) / (256 * DENSE_SEG);
    k_dense_count<<<(unsigned)cnt_tiles, 256, 0, s>>>(cases, mc_table, first, ctr, status + cls_tiles);
    k_dense_emit<<<(unsigned)std::min<uint64_t>((cells + 255) / 256, 8192), 256, 0, s>>>(
        g, field, iso, ids, cases, first, mc_table, out, cap, ctr);
}

}  // namespace bcmc
