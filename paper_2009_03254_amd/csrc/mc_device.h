// Device-side building blocks shared by the extraction kernels: wave64
// primitives, decoupled look-back, and the 5^3 LDS staging of a block with
// its +x/+y/+z halo.  Internal linkage in every includer.
#pragma once

#include <stdint.h>

#include "common.h"

namespace bcmc {
namespace {

__device__ __forceinline__ int lane() { return (int)__lane_id(); }

__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const int l = lane();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T t = __shfl_up(v, d, 64);
        if (l >= d) v += t;
    }
    return v;
}

// 32-bit inclusive scan over the wave with DPP moves (no LDS round trips):
// row_shr 1, 2, 4, 8 scan each row of 16 lanes (lanes shifted in from
// outside the row read 0), row_bcast:15 adds row 0's total to row 1 and row
// 2's to row 3, row_bcast:31 adds the total of rows 0-1 to rows 2 and 3.
template <>
__device__ __forceinline__ uint32_t wave_incl_scan<uint32_t>(uint32_t v) {
    int x = (int)v;
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);   // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);   // row_bcast:31
    return (uint32_t)x;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

__device__ __forceinline__ uint64_t lb_load(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void lb_store(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Decoupled look-back, run by one whole wave: publishes `agg` for tile t and
// returns the exclusive prefix of the tile.  256 predecessors are inspected
// per step (4 status words per lane, all loads in flight together): the
// window is summed up to (and including) the nearest tile that already holds
// an inclusive prefix.  With ~1000 tiles running at once most windows hold
// only aggregates, so the step width sets the latency of the walk.
__device__ uint64_t lookback(uint64_t *status, uint64_t t, uint64_t agg) {
    const int l = lane();
    if (t == 0) {
        if (l == 0) lb_store(&status[0], LB_PRE | agg);
        return 0;
    }
    if (l == 0) lb_store(&status[t], LB_AGG | agg);
    uint64_t excl = 0;
    int64_t j = (int64_t)t - 1;
    for (;;) {
        uint64_t w[4];
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int64_t idx = j - l - 64 * r;   // window position 64 r + l
            w[r] = idx >= 0 ? lb_load(&status[idx]) : LB_PRE;
        }
        // first inclusive prefix in window order, and whether anything before it is missing
        int first = 256;
        bool missing = false;
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const uint64_t flag = w[r] & ~LB_VAL;
            const uint64_t pre = __ballot(flag == LB_PRE);
            const uint64_t notready = __ballot(flag == 0);
            if (first == 256) {
                const int f = pre ? (int)__builtin_ctzll(pre) : 64;
                const uint64_t upto = f >= 63 ? ~0ull : ((2ull << f) - 1);
                if (notready & upto) missing = true;
                if (f < 64) first = 64 * r + f;
            }
        }
        if (missing) {
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        uint64_t v = 0;
#pragma unroll
        for (int r = 0; r < 4; r++)
            if (64 * r + l <= first) v += w[r] & LB_VAL;
        excl += wave_sum(v);
        if (first < 256) break;
        j -= 256;
    }
    if (l == 0) lb_store(&status[t], LB_PRE | (excl + agg));
    return excl;
}

// Workgroup (256 threads = 4 waves) exclusive scan of one value per thread
// followed by the look-back; returns the thread's global exclusive prefix and
// the tile total through *total (inclusive prefix of the tile in *incl_end).
__device__ uint64_t tile_scan_lookback(uint64_t v, uint64_t *status, uint64_t t,
                                       uint64_t *incl_end) {
    __shared__ uint64_t s_w[4];
    __shared__ uint64_t s_excl;
    const int w = threadIdx.x >> 6;
    uint64_t incl = wave_incl_scan(v);
    if (lane() == 63) s_w[w] = incl;
    __syncthreads();
    uint64_t woff = 0, agg = 0;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        if (i < w) woff += s_w[i];
        agg += s_w[i];
    }
    if (w == 0) {
        uint64_t e = lookback(status, t, agg);
        if (lane() == 0) s_excl = e;
    }
    __syncthreads();
    uint64_t e = s_excl;
    *incl_end = e + agg;
    __syncthreads();  // s_w / s_excl are reused by the next tile
    return e + woff + incl - v;
}

// Sum of one value per thread over a 256-thread workgroup, returned to every
// thread (all threads must call it).  Device-wide counters are then bumped
// once per workgroup: same-address atomics from every wave serialise.
__device__ __forceinline__ uint32_t wg_sum_u32(uint32_t v) {
    __shared__ uint32_t s_part[4];
    v = wave_sum(v);
    if (lane() == 0) s_part[threadIdx.x >> 6] = v;
    __syncthreads();
    const uint32_t t = s_part[0] + s_part[1] + s_part[2] + s_part[3];
    __syncthreads();
    return t;
}

__device__ __forceinline__ uint32_t take_tile(unsigned int *ctr) {
    __shared__ uint32_t s_tile;
    if (threadIdx.x == 0) s_tile = atomicAdd(ctr, 1u);
    __syncthreads();
    uint32_t t = s_tile;
    __syncthreads();
    return t;
}

// ---------------------------------------------------------------------------
// Marching cubes over the active blocks (Sec. 4.3-4.5), as the paper's three
// steps: a count pass (per-block vertex count, Sec. 4.4), a device-wide
// exclusive scan of the block counts, and an emission pass (Sec. 4.5).
// One wave64 owns one 4^3 block: lane = dual cell.  The block and its
// +x/+y/+z halo (5^3 samples) are staged in LDS from the cache slots of the
// block and its 7 positive neighbours.  Only blocks flagged "can emit" by the
// cull (the value hull of the block and its positive neighbours contains
// iso) are staged; every other block emits nothing, because a cell's eight
// samples all lie in the block of its lowest corner and that block's positive
// neighbours.
// ---------------------------------------------------------------------------
struct Halo {
    int bad;                // a needed block has no slot (internal error)
    uint32_t bx, by, bz;
    uint32_t nslot[8];      // slots of the block (0) and its + neighbours (mask dx|dy<<1|dz<<2)
};

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void halo_setup(const Geom &g, uint32_t b, const int32_t *__restrict__ I_slot,
                                           int identity, Halo &h) {
    h.bx = b % g.nbx;
    uint32_t r = b / g.nbx;
    h.by = r % g.nby;
    h.bz = r / g.nby;
    h.bad = 0;
#pragma unroll
    for (int m = 0; m < 8; m++) {
        uint32_t x = h.bx + (m & 1), y = h.by + ((m >> 1) & 1), z = h.bz + (m >> 2);
        h.nslot[m] = 0;
        if (x < g.nbx && y < g.nby && z < g.nbz) {
            uint32_t nb = x + g.nbx * (y + g.nby * z);
            if (identity) {
                h.nslot[m] = nb;
            } else {
                int32_t s = I_slot[nb];
                if (s < 0) h.bad = 1;
                h.nslot[m] = s < 0 ? 0u : (uint32_t)s;
            }
        }
    }
}

// LDS index of sample (x,y,z) of the 5^3 tile
__device__ __forceinline__ int tix(int x, int y, int z) { return x + 5 * y + 25 * z; }

// Stage the 125 samples: lane -> own sample, lanes 0..60 -> one halo sample.
__device__ __forceinline__ void stage_tile(const Geom &g, const Halo &h, const float *__restrict__ slots,
                                           float *tile) {
    const int l = lane();
    const int lx = l & 3, ly = (l >> 2) & 3, lz = l >> 4;
    tile[tix(lx, ly, lz)] = slots[(uint64_t)h.nslot[0] * 64 + l];
    if (l < 61) {
        int x, y, z;
        if (l < 16) { x = 4; y = l & 3; z = l >> 2; }
        else if (l < 32) { x = l & 3; y = 4; z = (l >> 2) & 3; }
        else if (l < 48) { x = l & 3; y = (l >> 2) & 3; z = 4; }
        else if (l < 52) { x = 4; y = 4; z = l - 48; }
        else if (l < 56) { x = 4; y = l - 52; z = 4; }
        else if (l < 60) { x = l - 56; y = 4; z = 4; }
        else { x = 4; y = 4; z = 4; }
        int m = (x >> 2) | ((y >> 2) << 1) | ((z >> 2) << 2);
        bool inside = (h.bx + (x >> 2) < g.nbx) && (h.by + (y >> 2) < g.nby) && (h.bz + (z >> 2) < g.nbz);
        float v = 0.0f;
        if (inside) v = slots[(uint64_t)h.nslot[m] * 64 + (x & 3) + 4 * (y & 3) + 16 * (z & 3)];
        tile[tix(x, y, z)] = v;
    }
}

// Case of the lane's cell (corner k at +(k&1, k>>1&1, k>>2&1); bit k set when
// the corner value is below iso) or -1 when the cell lies outside the volume.
__device__ __forceinline__ int cell_case(const Geom &g, const Halo &h, const float *tile, float iso) {
    const int l = lane();
    const int lx = l & 3, ly = (l >> 2) & 3, lz = l >> 4;
    if (4 * h.bx + lx + 1 >= g.nx || 4 * h.by + ly + 1 >= g.ny || 4 * h.bz + lz + 1 >= g.nz) return -1;
    int cs = 0;
#pragma unroll
    for (int k = 0; k < 8; k++)
        if (tile[tix(lx + (k & 1), ly + ((k >> 1) & 1), lz + (k >> 2))] < iso) cs |= 1 << k;
    return cs;
}

// Edge e of a cell: its lower endpoint offset and axis.
__device__ __forceinline__ void edge_geom(int e, int &ox, int &oy, int &oz, int &axis) {
    axis = e >> 2;
    int b0 = e & 1, b1 = (e >> 1) & 1;
    ox = axis == 0 ? 0 : b0;
    oy = axis == 1 ? 0 : (axis == 0 ? b0 : b1);
    oz = axis == 2 ? 0 : b1;
}

// ---- batched staging ------------------------------------------------------
// A wave takes 64 consecutive active blocks at a time (one per lane): each lane
// resolves the cache slots of its block and the block's 7 positive neighbours
// (the "octet"), then the wave stages MC_SB of the selected blocks per memory
// round trip (2 loads per lane per block, all in flight together) and works
// through them from LDS.  Slots of out-of-volume neighbours are 0: what is
// loaded from there only feeds cells outside the volume, which are never used.
constexpr int MC_SB = 8;

struct LaneGeom {            // per-lane constants of the 5^3 staging
    int own_t;               // tile index of the lane's own sample
    int halo_t;              // tile index of the lane's halo sample (lanes < 61)
    int halo_m;              // which + neighbour holds it (dx | dy<<1 | dz<<2)
    int halo_l;              // its index inside that neighbour
};

__device__ __forceinline__ LaneGeom lane_geom() {
    const int l = lane();
    LaneGeom q;
    q.own_t = tix(l & 3, (l >> 2) & 3, l >> 4);
    int x = 0, y = 0, z = 0;
    if (l < 16) { x = 4; y = l & 3; z = l >> 2; }
    else if (l < 32) { x = l & 3; y = 4; z = (l >> 2) & 3; }
    else if (l < 48) { x = l & 3; y = (l >> 2) & 3; z = 4; }
    else if (l < 52) { x = 4; y = 4; z = l - 48; }
    else if (l < 56) { x = 4; y = l - 52; z = 4; }
    else if (l < 60) { x = l - 56; y = 4; z = 4; }
    else { x = 4; y = 4; z = 4; }
    q.halo_t = tix(x, y, z);
    q.halo_m = (x >> 2) | ((y >> 2) << 1) | ((z >> 2) << 2);
    q.halo_l = (x & 3) + 4 * (y & 3) + 16 * (z & 3);
    return q;
}

// Slots of block b and its 7 positive neighbours; false if one is missing.
// The 8 lookups are issued unconditionally (an out-of-volume neighbour reads
// block b's own entry) so that they are in flight together.  Also returns the
// block's coordinates (bx, by, bz), so that the per-block loops broadcast them
// instead of dividing again.
__device__ __forceinline__ bool octet(const Geom &g, uint32_t b, const int32_t *__restrict__ I_slot,
                                      int identity, uint32_t so[8], uint32_t &bx, uint32_t &by,
                                      uint32_t &bz) {
    const uint32_t r = b / g.nbx;
    bx = b - r * g.nbx;
    by = r % g.nby;
    bz = r / g.nby;
    uint32_t nb[8];
    bool in[8];
#pragma unroll
    for (int m = 0; m < 8; m++) {
        const uint32_t x = bx + (m & 1), y = by + ((m >> 1) & 1), z = bz + (m >> 2);
        in[m] = x < g.nbx && y < g.nby && z < g.nbz;
        nb[m] = in[m] ? x + g.nbx * (y + g.nby * z) : b;
    }
    if (identity) {
#pragma unroll
        for (int m = 0; m < 8; m++) so[m] = in[m] ? nb[m] : 0u;
        return true;
    }
    int32_t sl[8];
#pragma unroll
    for (int m = 0; m < 8; m++) sl[m] = I_slot[nb[m]];
    bool ok = true;
#pragma unroll
    for (int m = 0; m < 8; m++) {
        ok = ok && (!in[m] || sl[m] >= 0);
        so[m] = (in[m] && sl[m] >= 0) ? (uint32_t)sl[m] : 0u;
    }
    return ok;
}

__device__ __forceinline__ uint32_t bcast(uint32_t v, int src) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, src);
}

// Stage up to SB blocks (the lanes of `batch`, in lane order blocks
// k < nsb; the rest repeat block 0) into tiles[k].  Their slots pass through
// LDS: each lane of the batch writes its block's 8 slots (the block and its 7
// positive neighbours) to tab[8 k + m], and every lane reads the two it needs,
// its own sample's block and its halo sample's neighbour (per block, 8 lane
// reads and a chain of selects, each select needing a copy, cost more).  Every
// slot is loaded unconditionally, so that all 2 SB loads of a lane are in
// flight before the first tile write.  `tab` holds 8 SB words (8-byte
// aligned) of the wave's LDS that nothing else uses meanwhile.
template <int SB>
__device__ __forceinline__ void stage_batch_tab(const LaneGeom &q, const float *__restrict__ slots,
                                                const uint32_t so[8], uint64_t batch, int nsb,
                                                uint32_t *tab, float (*tiles)[128]) {
    const int l = lane();
    if ((batch >> l) & 1u) {   // 8-byte stores: `tab` is 8-byte aligned
        uint2 *p = reinterpret_cast<uint2 *>(tab + 8 * mbcnt(batch));
        p[0] = make_uint2(so[0], so[1]);
        p[1] = make_uint2(so[2], so[3]);
        p[2] = make_uint2(so[4], so[5]);
        p[3] = make_uint2(so[6], so[7]);
    }
    wave_lds_sync();
    float ov[SB], hv[SB];
#pragma unroll
    for (int k = 0; k < SB; k++) {
        const int kk = k < nsb ? k : 0;
        const uint32_t s_own = tab[8 * kk];
        const uint32_t s_h = tab[8 * kk + q.halo_m];
        ov[k] = slots[(uint64_t)s_own * 64 + l];
        hv[k] = slots[(uint64_t)s_h * 64 + q.halo_l];
    }
#pragma unroll
    for (int k = 0; k < SB; k++) {
        tiles[k][q.own_t] = ov[k];
        if (l < 61) tiles[k][q.halo_t] = hv[k];
    }
}

// Case of the lane's cell in block (bx,by,bz) staged in `tile`, -1 outside.
__device__ __forceinline__ int tile_case(const Geom &g, uint32_t bx, uint32_t by, uint32_t bz,
                                         const float *tile, float iso) {
    const int l = lane();
    const int lx = l & 3, ly = (l >> 2) & 3, lz = l >> 4;
    if (4 * bx + lx + 1 >= g.nx || 4 * by + ly + 1 >= g.ny || 4 * bz + lz + 1 >= g.nz) return -1;
    int cs = 0;
#pragma unroll
    for (int k = 0; k < 8; k++)
        if (tile[tix(lx + (k & 1), ly + ((k >> 1) & 1), lz + (k >> 2))] < iso) cs |= 1 << k;
    return cs;
}

// The chunks of items (mc_chunk_size) a wave of a persistent grid takes.  Workgroups are
// dispatched round-robin over the 8 XCDs (blockIdx % 8): the workgroups of one
// XCD take one contiguous eighth of the chunks, so that blocks whose halos
// overlap are staged through the same L2, and that XCD's waves take its
// chunks in turn (wave r: chunks r, r + W, r + 2 W, ... of the eighth, W its
// waves), so that they all work in one window that moves along the eighth:
// a block's +y and +z neighbours are staged at about the same time as the
// block, and the output is written in a few dense regions instead of one
// stream per wave.  gridDim.x must be a multiple of 8.
// Blocks per chunk for n active blocks on `waves` waves: 64 (one per lane)
// once every wave has at least that many, fewer for small calls, so that
// every wave still gets work.
__host__ __device__ __forceinline__ uint32_t mc_chunk_size(uint64_t n, uint32_t waves) {
    const uint64_t per = (n + waves - 1) / waves;
    return per >= 64 ? 64u : (per < 1 ? 1u : (uint32_t)per);
}
struct ChunkRange {
    uint64_t first, end;
    uint32_t stride;
};
__device__ __forceinline__ ChunkRange xcd_chunks(uint64_t n_chunks) {
    const uint32_t G = gridDim.x, g = blockIdx.x;
    const uint32_t per_xcd = (G / 8u) * MC_WAVES;                  // waves of one XCD
    const uint32_t r = (g / 8u) * MC_WAVES + (threadIdx.x >> 6);  // this wave's rank there
    const uint64_t per = (n_chunks + 7) / 8;
    uint64_t lo = (uint64_t)(g % 8u) * per;
    if (lo > n_chunks) lo = n_chunks;
    const uint64_t hi = lo + per < n_chunks ? lo + per : n_chunks;
    return {lo + r, hi, per_xcd};
}

// Corner masks of the 64 cells of a block from the sign masks of the block
// and its 7 positive neighbours (M[dx | dy<<1 | dz<<2]): bit i of c[k] is the
// sign bit of corner k = (k&1, k>>1&1, k>>2&1) of cell i.  sx / sy / sz give,
// for every cell, the sample one step along x / y / z: from the block itself,
// or from the neighbour for the cells on its far face.
__device__ __forceinline__ uint64_t sx(uint64_t a, uint64_t b) {
    return ((a >> 1) & 0x7777777777777777ull) | ((b << 3) & 0x8888888888888888ull);
}
__device__ __forceinline__ uint64_t sy(uint64_t a, uint64_t b) {
    return ((a >> 4) & 0x0FFF0FFF0FFF0FFFull) | ((b << 12) & 0xF000F000F000F000ull);
}
__device__ __forceinline__ uint64_t sz(uint64_t a, uint64_t b) { return (a >> 16) | (b << 48); }

__device__ __forceinline__ void corner_masks(const uint64_t M[8], uint64_t c[8]) {
    const uint64_t x01 = sx(M[0], M[1]), x23 = sx(M[2], M[3]);
    const uint64_t x45 = sx(M[4], M[5]), x67 = sx(M[6], M[7]);
    c[0] = M[0];
    c[1] = x01;
    c[2] = sy(M[0], M[2]);
    c[3] = sy(x01, x23);
    c[4] = sz(M[0], M[4]);
    c[5] = sz(x01, x45);
    c[6] = sz(c[2], sy(M[4], M[6]));
    c[7] = sz(c[3], sy(x45, x67));
}

// Cells of block (bx, by, bz) whose 8 corners lie in the volume.
__device__ __forceinline__ uint64_t valid_cells(const Geom &g, uint32_t bx, uint32_t by, uint32_t bz) {
    const int vx = min(4, (int)g.nx - 1 - 4 * (int)bx);
    const int vy = min(4, (int)g.ny - 1 - 4 * (int)by);
    const int vz = min(4, (int)g.nz - 1 - 4 * (int)bz);
    if (vx <= 0 || vy <= 0 || vz <= 0) return 0;
    const uint64_t mx = 0x1111111111111111ull * ((1ull << vx) - 1);
    const uint64_t my = 0x0001000100010001ull * ((1ull << (4 * vy)) - 1);
    const uint64_t mz = vz == 4 ? ~0ull : ((1ull << (16 * vz)) - 1);
    return mx & my & mz;
}

// Per-edge lookup, 5 bits per edge id e (0..11), built from edge_geom's
// convention: ox | oy << 1 | oz << 2 | axis << 3 (first corner offset and
// axis).
constexpr uint64_t edge_lut() {
    uint64_t r = 0;
    for (int e = 0; e < 12; e++) {
        const int axis = e >> 2, b0 = e & 1, b1 = (e >> 1) & 1;
        const int ox = axis == 0 ? 0 : b0;
        const int oy = axis == 1 ? 0 : (axis == 0 ? b0 : b1);
        const int oz = axis == 2 ? 0 : b1;
        r |= (uint64_t)(ox | oy << 1 | oz << 2 | axis << 3) << (5 * e);
    }
    return r;
}
constexpr uint64_t kEdgeGeom = edge_lut();

// Vertex records are written once and not read back by the path:
// non-temporal stores.  (Plain stores drain a bare streaming write faster on
// gfx950, but in this kernel the two measured the same within the spread
// that the output buffer's physical placement causes.)
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void store_record(void *out, uint64_t o, uint64_t r) {
    __builtin_nontemporal_store(r, reinterpret_cast<uint64_t *>(out) + o);
}
__device__ __forceinline__ void store_record(void *out, uint64_t o, float x, float y, float z, uint32_t b) {
    u32x4_t v = {__float_as_uint(x), __float_as_uint(y), __float_as_uint(z), b};
    __builtin_nontemporal_store(v, reinterpret_cast<u32x4_t *>(out) + o);
}

constexpr int EMIT_TRIS = 64 * 5;   // a wave's triangle list (one block's maximum)

// Output record formats of the emission.
enum : int { VFMT_F32 = 0, VFMT_EDGE8 = 1, VFMT_Q10 = 2 };
// Not an output format: the emission's pass over the soup of the last
// extract, accumulating the gradient of a loss on the vertex positions
// (GradCtx) instead of writing records.
constexpr int VFMT_GRAD = 3;

// Sec. 4.5's vertex: each block-relative coordinate (in [0, 4]) quantised to
// 10 bits, q = trunc(x * (1023 / 4) + 1/2) (round to nearest, in float32,
// each operation rounded), x in bits 0-9, y in 10-19, z in 20-29.  The
// dequantised coordinate q * 4 / 1023 is within 2 / 1023 voxel of x plus
// float32 rounding.
__host__ __device__ __forceinline__ uint32_t q10_axis(float x) {
    const float t = x * 255.75f;   // 1023 / 4, exact in float32
    const uint32_t q = (uint32_t)(t + 0.5f);
    return q < 1023u ? q : 1023u;
}
__host__ __device__ __forceinline__ uint32_t q10_code(float x, float y, float z) {
    return q10_axis(x) | (q10_axis(y) << 10) | (q10_axis(z) << 20);
}

// Per-edge entry of the emission's LDS edge table: low word the first
// corner's offset in the cell as bytes (x, y, z in bytes 0-2, each 0 or 1)
// plus the tile step along the edge's axis (1, 5 or 25) in byte 3; high word
// the axis as a unit vector of bytes.  Edges 12-15 are unused (zero).
__host__ __device__ constexpr uint64_t edge_entry(int e) {
    if (e >= 12) return 0;
    const uint32_t d = (uint32_t)(kEdgeGeom >> (5 * e)) & 31u;   // ox | oy << 1 | oz << 2 | axis << 3
    const uint32_t axis = d >> 3;
    const uint32_t o = (d & 1u) | ((d >> 1) & 1u) << 8 | ((d >> 2) & 1u) << 16;
    const uint32_t step = axis == 0 ? 1u : (axis == 1 ? 5u : 25u);
    return (uint64_t)(o | step << 24) | (uint64_t)(1u << (8 * axis)) << 32;
}
// Tile index (x + 5 y + 25 z) of a point given as bytes x | y << 8 | z << 16.
__device__ __forceinline__ uint32_t tile_index(uint32_t xyz) {
    return __builtin_amdgcn_udot4(xyz, 0x00190501u, 0u, false);
}
// Tile index of the point one step along the axis whose step is in byte 3.
__device__ __forceinline__ uint32_t tile_index_next(uint32_t xyz_step) {
    return __builtin_amdgcn_udot4(xyz_step, 0x01190501u, 0u, false);
}

// Per-wave LDS of the emission: SB staged tiles, the triangle list of the
// staged blocks and each staged block's id and isovalue.
template <int SB>
struct EmitSharedT {
    uint64_t edge[16];                  // edge_entry(e), read per vertex
    float tiles[MC_WAVES][SB][128];
    uint32_t tri[MC_WAVES][EMIT_TRIS];  // per triangle: its list record (emit_batch)
    uint32_t blk[MC_WAVES][SB];         // block id of each staged block
    float iso[MC_WAVES][SB];            // its isovalue
};
using EmitShared = EmitSharedT<MC_SB>;
// The plain emission stages two blocks fewer and keeps the triangle table in
// LDS (a per-lane lookup per block that global memory serves only after the
// staged slots have evicted it from L1): its LDS then fits 8 workgroups per CU
// (its registers hold it to 7, where it needs no scratch).
constexpr int EMIT_SB = MC_SB - 2;

// The backward's LDS: the plain emission's, and per staged block the
// gradient accumulated at each of its 125 tile samples (added to the field
// once per block instead of once per vertex and corner).
struct EmitSharedGrad {
    uint64_t tab[256];
    uint64_t edge[16];
    float tiles[MC_WAVES][EMIT_SB][128];
    uint32_t tri[MC_WAVES][EMIT_TRIS];
    uint32_t blk[MC_WAVES][EMIT_SB];
    float iso[MC_WAVES][EMIT_SB];
    float acc[MC_WAVES][EMIT_SB][128];
};

// The backward's side of emit_batch<VFMT_GRAD>: dL/dv per vertex (3 floats,
// in the soup's order), the field's gradient in block layout, the staged
// blocks' vertex counts of the forward (a block whose recomputed count
// differs sets ERR_INTERNAL: the field changed), and the lane's share of
// dL/diso.
struct GradCtx {
    const float *gV;
    float *dfield;
    unsigned int *err;
    uint32_t nbx, nbxy;           // blocks per row and per layer
    uint32_t expect[MC_SB];
    float giso;
};
// Index in the block-layout field of the sample at tile position p (bytes
// x | y << 8 | z << 16, 0..4 each) of the staged block b.
__device__ __forceinline__ uint64_t tile_sample(const GradCtx &gc, uint32_t b, uint32_t p) {
    const uint32_t x = p & 0xFFu, y = (p >> 8) & 0xFFu, z = (p >> 16) & 0xFFu;
    const uint64_t blk = (uint64_t)b + (x >> 2) + (uint64_t)gc.nbx * (y >> 2) + (uint64_t)gc.nbxy * (z >> 2);
    return blk * 64 + (x & 3) + 4 * (y & 3) + 16 * (z & 3);
}
struct EmitSharedPlain {
    uint64_t tab[256];
    uint64_t edge[16];
    float tiles[MC_WAVES][EMIT_SB][128];
    uint32_t tri[MC_WAVES][EMIT_TRIS];
    uint32_t blk[MC_WAVES][EMIT_SB];
    float iso[MC_WAVES][EMIT_SB];
};

}  // namespace
}  // namespace bcmc

namespace bcmc {
namespace {

// Emission (Sec. 4.5) of the nsb blocks staged in tiles[0..nsb), whose
// vertex ranges follow each other in the output from `base` on (records past
// `cap` dropped).  Per block: the cases of its cells, an exclusive scan of
// their triangle counts and one record per triangle (cell, 3 edge ids, staged
// block) appended to the wave's list; when the next block would overflow the
// list, and after the last, one lane-per-vertex loop writes the listed
// triangles in canonical order (block, cell, triangle, vertex).
// info(k, g, b, bx, by, bz, iso) gives block k's volume geometry, id, block
// coordinates and isovalue (wave-uniform).
// FMT (VFMT_*): VFMT_F32 16-byte records {f32 x, y, z block-relative; u32
// block}; VFMT_EDGE8 8-byte records block | cell << 32 | edge << 38 | q << 42
// with q = min(trunc(t * 2^22), 2^22 - 1); VFMT_Q10 8-byte records (Sec. 4.5)
// of the block-relative float32 coordinates quantised to 10 bits each
// (q10_code) | block << 32.
template <int FMT, class Info, class SH>
__device__ __forceinline__ void emit_batch(int nsb, const Info &info, float (*tiles)[128],
                                           const uint64_t *__restrict__ mc_table, SH &sh,
                                           int w, uint64_t base, void *__restrict__ out,
                                           uint64_t cap, GradCtx *gc = nullptr) {
    const int l = lane();
    // the lane's cell as bytes x | y << 8 | z << 16
    const uint32_t cell_xyz = (uint32_t)(l & 3) | (uint32_t)((l >> 2) & 3) << 8 | (uint32_t)(l >> 4) << 16;
    uint32_t run = 0;   // triangles listed
    // backward: dL/dv of the lane's next vertex, loaded one pass ahead (the
    // first pass's while the blocks are classified)
    float gpre[3] = {0.0f, 0.0f, 0.0f};
    auto gload = [&](uint64_t o) {
        if constexpr (FMT == VFMT_GRAD) {
            if (o < cap) {
                const float *q = gc->gV + 3 * o;
                gpre[0] = q[0];
                gpre[1] = q[1];
                gpre[2] = q[2];
            }
        }
    };
    gload(base + (uint64_t)l);
    // List record of a triangle: the cell as bytes (bits 0-1, 8-9, 16-17),
    // the staged block in bits 2-4, the 3 edge ids in bits 20-31 (as in the
    // case table).
    auto flush = [&]() {
        wave_lds_sync();
        const int total = 3 * (int)run;
        for (int j = l; j < total; j += 64) {
            const float gcur[3] = {gpre[0], gpre[1], gpre[2]};   // dL/dv of vertex base + j (backward)
            if (j + 64 < total) gload(base + (uint64_t)(j + 64));
            const int t = (j * 43691) >> 17;               // j / 3 for j < 3 * EMIT_TRIS
            const uint32_t rec = sh.tri[w][t];
            const uint32_t e = (rec >> (20 + 4 * (j - 3 * t))) & 15u;
            const uint32_t k = (rec >> 2) & 7u;
            const uint64_t ent = sh.edge[e];
            const uint32_t cxyz = rec & 0x030303u;         // the cell
            const uint32_t p0 = cxyz + (uint32_t)ent;      // the edge's first corner | step << 24
            const float *tile = tiles[k];
            const float a = tile[tile_index(p0)];
            const float bv = tile[tile_index_next(p0)];
            const float iso = sh.iso[w][k];
            const uint32_t b = sh.blk[w][k];
            const float tt = (iso - a) / (bv - a);
            const uint64_t o = base + (uint64_t)j;
            if constexpr (FMT == VFMT_GRAD) {
                // t = (iso - a) / (b - a): dt/da = (t - 1) / (b - a),
                // dt/db = -t / (b - a), dt/diso = 1 / (b - a), times dL/dv
                // along the edge's axis; the corners' shares go to the
                // staged block's LDS accumulators
                (void)b;
                if (o < cap) {
                    const uint32_t u = (uint32_t)(ent >> 32);
                    const uint32_t axis = __builtin_amdgcn_udot4(u, 0x00020100u, 0u, false);
                    const float gt = axis == 0 ? gcur[0] : (axis == 1 ? gcur[1] : gcur[2]);
                    const float inv = 1.0f / (bv - a);
                    const float t2 = (iso - a) * inv;
                    atomicAdd(&sh.acc[w][k][tile_index(p0)], gt * (t2 - 1.0f) * inv);
                    atomicAdd(&sh.acc[w][k][tile_index_next(p0)], -gt * t2 * inv);
                    gc->giso += gt * inv;
                }
            } else if (FMT == VFMT_EDGE8) {
                uint32_t qt = (uint32_t)(tt * 4194304.0f);   // t * 2^22 is exact
                qt = qt < 4194303u ? qt : 4194303u;
                const uint32_t c = __builtin_amdgcn_udot4(cxyz, 0x00100401u, 0u, false);   // x + 4 y + 16 z
                const uint64_t r = (uint64_t)b | ((uint64_t)c << 32) | ((uint64_t)e << 38) | ((uint64_t)qt << 42);
                if (o < cap) store_record(out, o, r);
            } else {
                // the first corner plus t along the edge's axis: t * 1 + x
                // rounds as x + t, and t * 0 + x is x exactly (for finite t)
                const uint32_t u = (uint32_t)(ent >> 32);
                const float x0 = (float)(p0 & 0xFFu), y0 = (float)((p0 >> 8) & 0xFFu),
                            z0 = (float)((p0 >> 16) & 0xFFu);
                const float ux = (float)(u & 0xFFu), uy = (float)((u >> 8) & 0xFFu),
                            uz = (float)((u >> 16) & 0xFFu);
                float px = __builtin_fmaf(tt, ux, x0);
                float py = __builtin_fmaf(tt, uy, y0);
                float pz = __builtin_fmaf(tt, uz, z0);
                if (__builtin_expect(tt != tt, 0)) {
                    // both differences overflowed (inf / inf): NaN on the
                    // axis only, the other two coordinates stay the corner's
                    px = ux != 0.0f ? x0 + tt : x0;
                    py = uy != 0.0f ? y0 + tt : y0;
                    pz = uz != 0.0f ? z0 + tt : z0;
                }
                if (FMT == VFMT_Q10) {
                    if (o < cap) store_record(out, o, (uint64_t)q10_code(px, py, pz) | ((uint64_t)b << 32));
                } else {
                    if (o < cap) store_record(out, o, px, py, pz, b);
                }
            }
        }
        base += (uint64_t)total;
        run = 0;
        gload(base + (uint64_t)l);   // for a further pass over the list
        wave_lds_sync();
    };
    for (int k = 0; k < nsb; k++) {
        Geom g;
        uint32_t b, bx, by, bz;
        float iso;
        info(k, g, b, bx, by, bz, iso);
        const int cs = tile_case(g, bx, by, bz, tiles[k], iso);
        const uint64_t tb = cs < 0 ? 0ull : mc_table[cs];   // 2 KB table (LDS-resident for the callers)
        const uint32_t nt = (uint32_t)(tb >> 60);
        const uint32_t incl = wave_incl_scan(nt);
        const uint32_t tot = __shfl(incl, 63, 64);
        if (FMT == VFMT_GRAD && 3 * tot != gc->expect[k] && l == 0) atomicOr(gc->err, ERR_INTERNAL);
        if (run + tot > (uint32_t)EMIT_TRIS) flush();
        if (l == 0) {
            sh.blk[w][k] = b;
            sh.iso[w][k] = iso;
        }
        const uint32_t rec0 = cell_xyz | (uint32_t)k << 2;
        for (uint32_t t = 0; t < nt; t++)
            sh.tri[w][run + incl - nt + t] = rec0 | (uint32_t)(tb >> (12 * t)) << 20;
        run += tot;
    }
    if (run) flush();
    else wave_lds_sync();   // the caller restages the tiles next
    if constexpr (FMT == VFMT_GRAD) {
        // each staged block's accumulated samples into the field (one
        // atomic per touched sample), the accumulators back to zero
        for (int k = 0; k < nsb; k++) {
            const uint32_t b = sh.blk[w][k];
            for (int i = l; i < 125; i += 64) {
                const float v = sh.acc[w][k][i];
                if (v != 0.0f) {
                    const uint32_t z = (uint32_t)i / 25u, y = ((uint32_t)i - 25u * z) / 5u,
                                   x = (uint32_t)i - 25u * z - 5u * y;
                    atomicAdd(&gc->dfield[tile_sample(*gc, b, x | y << 8 | z << 16)], v);
                    sh.acc[w][k][i] = 0.0f;
                }
            }
        }
        wave_lds_sync();
    }
}

}  // namespace
}  // namespace bcmc
