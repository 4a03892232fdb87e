// Extraction kernels for gfx950 (paper Sec. 4): active-block culling (4.1),
// the GPU-driven LRU cache update (4.2, Alg. 1), and block-wise marching cubes
// (4.3-4.5).  Every count the host does not know is read from device memory,
// so the whole sequence is enqueued without host round-trips.
//
// Shared idioms:
//   * wave64 primitives: ballot / mbcnt compaction, shuffle scans;
//   * single-pass scans with decoupled look-back (Merrill & Garland 2016):
//     each tile publishes its aggregate, then its inclusive prefix, in a
//     64-bit status word (2 flag bits + value); tiles are taken from an atomic
//     counter in order, so a tile only ever waits on tiles already running;
//   * device-scope atomics on one address serialise (~14 ns each), so work
//     without a look-back is spread statically (workgroup w takes items w,
//     w + G, ...) and per-workgroup counts go to arrays, not one counter.
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "common.h"
#include "mc_device.h"
#include "mc_ntri.h"

namespace bcmc {
namespace {
// ---------------------------------------------------------------------------
// Sec. 4.1: active blocks.  Block b is active when its range, or its range
// united with the range of one of its 26 neighbours, contains iso
// (lo < iso <= hi).  With LO / HI the min / max over the 3x3x3 neighbourhood
// that is:  (lo_b < iso <= HI)  or  (LO < iso <= hi_b).
// ---------------------------------------------------------------------------
// Tiled: a workgroup culls a CULL_TX x CULL_TY x CULL_TZ box of blocks.  The
// box's ranges with a one-block halo (+inf / -inf outside the volume) are
// staged in LDS with all loads in flight at once; the 3x3 in-plane min / max
// and the 2x2 positive-quadrant min / max are then combined across z in
// registers, so every range is read about 1.6 times and no load waits inside
// the sweep.
constexpr int CULL_TX = 32, CULL_TY = 8, CULL_TZ = 8;

// Hull of the ranges over a tile's box with its one-block halo (clipped to
// the volume), one workgroup per tile, at load.  When the hull does not
// straddle iso, no block of the tile can be active: every block's
// neighbourhood range lies inside it.
__global__ __launch_bounds__(256) void k_tile_ranges(Geom g, const float2 *__restrict__ ranges,
                                                    float2 *__restrict__ tile_ranges) {
    constexpr int RX = CULL_TX + 2, RY = CULL_TY + 2, RZ = CULL_TZ + 2;
    const uint32_t ntx = (g.nbx + CULL_TX - 1) / CULL_TX, nty = (g.nby + CULL_TY - 1) / CULL_TY;
    uint32_t t = blockIdx.x;
    const uint32_t tx = t % ntx;
    t /= ntx;
    const uint32_t ty = t % nty, tz = t / nty;
    float lo = INFINITY, hi = -INFINITY;
    for (int i = threadIdx.x; i < RX * RY * RZ; i += 256) {
        const int hz = i / (RX * RY), r = i - hz * RX * RY, hy = r / RX, hx = r - hy * RX;
        const int x = (int)(tx * CULL_TX) + hx - 1, y = (int)(ty * CULL_TY) + hy - 1,
                  z = (int)(tz * CULL_TZ) + hz - 1;
        if (x >= 0 && x < (int)g.nbx && y >= 0 && y < (int)g.nby && z >= 0 && z < (int)g.nbz) {
            const float2 q = ranges[((uint64_t)z * g.nby + (uint32_t)y) * g.nbx + (uint32_t)x];
            lo = fminf(lo, q.x);
            hi = fmaxf(hi, q.y);
        }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        lo = fminf(lo, __shfl_xor(lo, d, 64));
        hi = fmaxf(hi, __shfl_xor(hi, d, 64));
    }
    __shared__ float2 s_h[4];
    if (lane() == 0) s_h[threadIdx.x >> 6] = make_float2(lo, hi);
    __syncthreads();
    if (threadIdx.x == 0)
        tile_ranges[blockIdx.x] = make_float2(fminf(fminf(s_h[0].x, s_h[1].x), fminf(s_h[2].x, s_h[3].x)),
                                              fmaxf(fmaxf(s_h[0].y, s_h[1].y), fmaxf(s_h[2].y, s_h[3].y)));
}

// The per-call counters and the look-back status words of the call's scans
// start at zero: cleared first (the cull's tile queue counts in the counters).
__global__ __launch_bounds__(256) void k_call_reset(Counters *ctr, uint64_t n_slots_host, uint64_t *status,
                                                   uint64_t status_words) {
    const uint64_t gid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (gid == 0) {
        Counters c{};
        c.n_slots = n_slots_host;
        c.n_slots_old = n_slots_host;
        c.key_or = 0u;
        c.key_and = ~0u;
        *ctr = c;
    }
    for (uint64_t w = gid; w < status_words; w += (uint64_t)gridDim.x * blockDim.x) status[w] = 0;
}

// Tile queue of the cull: the tiles whose hull straddles iso (live: culled
// block by block) and those whose hull straddled the previous call's isovalue
// only (stale: their flags are cleared), one tile per thread, appended with
// one atomic per wave.  live: n_tiles entries, stale: the n_tiles after.
__global__ __launch_bounds__(256) void k_cull_scan(const float2 *__restrict__ tile_ranges, uint64_t n_tiles,
                                                  float iso, float prev_iso, uint32_t *__restrict__ list,
                                                  Counters *ctr) {
    const uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    bool live = false, stale = false;
    if (t < n_tiles) {
        const float2 hull = tile_ranges[t];
        live = hull.x < iso && iso <= hull.y;
        stale = !live && hull.x < prev_iso && prev_iso <= hull.y;
    }
    const uint64_t lm = __ballot(live), sm = __ballot(stale);
    uint32_t lb = 0, sb = 0;
    if (lane() == 0) {
        if (lm) lb = atomicAdd(&ctr->tile_ctr[TC_CULL_LIVE], (uint32_t)__popcll(lm));
        if (sm) sb = atomicAdd(&ctr->tile_ctr[TC_CULL_STALE], (uint32_t)__popcll(sm));
    }
    lb = __shfl(lb, 0, 64);
    sb = __shfl(sb, 0, 64);
    if (live) list[lb + mbcnt(lm)] = (uint32_t)t;
    if (stale) list[n_tiles + sb + mbcnt(sm)] = (uint32_t)t;
}

// Flags per block: bit 0 active, bit 1 may emit, bit 2 active without a
// slot (new, Alg. 1 MarkNewBlocks; never set for an identity cache).
// The flags are zero outside the tiles the previous call culled, so a tile
// live then and dead now (stale) is cleared here, a live tile is rewritten
// in full, and no other flag is touched.  Persistent: workgroup w takes
// queue entries w, w + G, ... (stale tiles first), so that a surface's live
// tiles spread evenly over the workgroups whatever their layout, with no
// shared counter (same-address atomics serialise, ~14 ns each).
__global__ __launch_bounds__(256) void k_cull(Geom g, const float2 *__restrict__ ranges, float iso,
                                             const uint32_t *__restrict__ list, uint64_t n_tiles,
                                             const int32_t *__restrict__ I_slot, int identity,
                                             uint8_t *__restrict__ active, Counters *ctr,
                                             uint32_t *__restrict__ round_gen, uint32_t gen) {
    constexpr int NL = CULL_TZ + 2, RX = CULL_TX + 2, RY = CULL_TY + 2, SLOTS = RX * RY;
    __shared__ float2 sh[NL][RY][RX];
    const uint32_t ntx = (g.nbx + CULL_TX - 1) / CULL_TX, nty = (g.nby + CULL_TY - 1) / CULL_TY;
    const uint32_t n_live = ctr->tile_ctr[TC_CULL_LIVE], n_stale = ctr->tile_ctr[TC_CULL_STALE];
    const uint32_t n_q = n_stale + n_live;
    const int lx = threadIdx.x % CULL_TX, ly = threadIdx.x / CULL_TX;
    auto tile_of = [&](uint32_t t, uint32_t &tx, uint32_t &ty, uint32_t &tz) {
        tx = t % ntx;
        t /= ntx;
        ty = t % nty;
        tz = t / nty;
    };
    uint32_t q = blockIdx.x;
    for (; q < n_stale; q += gridDim.x) {   // culled last time only: flags cleared
        uint32_t tx, ty, tz;
        tile_of(list[n_tiles + q], tx, ty, tz);
        const int z0 = (int)(tz * CULL_TZ), z1 = min(z0 + CULL_TZ, (int)g.nbz);
        const uint32_t bx = tx * CULL_TX + lx, by = ty * CULL_TY + ly;
        if (bx < g.nbx && by < g.nby)
            for (int z = z0; z < z1; z++) active[((uint64_t)z * g.nby + by) * g.nbx + bx] = 0;
    }
    // live tiles: a box's ranges with their halo, all loads in flight
    // together; the next box's are loaded while this one is culled
    constexpr int PER = (NL * SLOTS + 255) / 256;
    auto load_box = [&](uint32_t qq, float2 (&v)[PER]) {
        uint32_t tx, ty, tz;
        tile_of(list[qq - n_stale], tx, ty, tz);
        const int z0 = (int)(tz * CULL_TZ), z1 = min(z0 + CULL_TZ, (int)g.nbz);
#pragma unroll
        for (int k = 0; k < PER; k++) {
            const int i = (int)threadIdx.x + 256 * k;
            const int li = i / SLOTS, r = i - li * SLOTS;
            const int hy = r / RX, hx = r - hy * RX;
            const int zl = z0 - 1 + li;
            const int x = (int)(tx * CULL_TX) + hx - 1, y = (int)(ty * CULL_TY) + hy - 1;
            v[k] = make_float2(INFINITY, -INFINITY);
            if (i < NL * SLOTS && zl >= 0 && zl < (int)g.nbz && zl <= z1 && x >= 0 && x < (int)g.nbx &&
                y >= 0 && y < (int)g.nby)
                v[k] = ranges[((uint64_t)zl * g.nby + (uint32_t)y) * g.nbx + (uint32_t)x];
        }
    };
    float2 v[PER];
    if (q < n_q) load_box(q, v);
    for (; q < n_q; q += gridDim.x) {
        uint32_t tx, ty, tz;
        tile_of(list[q - n_stale], tx, ty, tz);
        const int z0 = (int)(tz * CULL_TZ), z1 = min(z0 + CULL_TZ, (int)g.nbz);
        const uint32_t bx = tx * CULL_TX + lx, by = ty * CULL_TY + ly;
#pragma unroll
        for (int k = 0; k < PER; k++) {
            const int i = (int)threadIdx.x + 256 * k;
            if (i < NL * SLOTS) (&sh[0][0][0])[i] = v[k];
        }
        __syncthreads();
        if (q + gridDim.x < n_q) load_box(q + gridDim.x, v);
        uint32_t act = 0;   // bit z - z0: block (bx, by, z) is active
        if (bx < g.nbx && by < g.nby) {
            // per layer: 3x3 min / max, 2x2 positive min / max, own range
            float l3a = INFINITY, h3a = -INFINITY;                       // layer zl - 2
            float l3b = INFINITY, h3b = -INFINITY, p2lb = INFINITY, p2hb = -INFINITY;
            float2 ownb = make_float2(INFINITY, -INFINITY);             // layer zl - 1
            uint32_t can = 0;
#pragma unroll
            for (int li = 0; li < NL; li++) {
                float l3 = INFINITY, h3 = -INFINITY, p2l = INFINITY, p2h = -INFINITY;
#pragma unroll
                for (int dy = -1; dy <= 1; dy++)
#pragma unroll
                    for (int dx = -1; dx <= 1; dx++) {
                        const float2 q2 = sh[li][ly + 1 + dy][lx + 1 + dx];
                        l3 = fminf(l3, q2.x);
                        h3 = fmaxf(h3, q2.y);
                        if (dx >= 0 && dy >= 0) {
                            p2l = fminf(p2l, q2.x);
                            p2h = fmaxf(p2h, q2.y);
                        }
                    }
                const float2 own = sh[li][ly + 1][lx + 1];
                if (li >= 2 && z0 - 2 + li < z1) {   // layer z0 - 2 + li has both z neighbours now
                    const float LO = fminf(l3a, fminf(l3b, l3)), HI = fmaxf(h3a, fmaxf(h3b, h3));
                    const float PLO = fminf(p2lb, p2l), PHI = fmaxf(p2hb, p2h);
                    // "can emit": the hull of the 2x2x2 group headed by the block
                    // contains iso (implies act, as that group contains the block)
                    if ((ownb.x < iso && iso <= HI) || (LO < iso && iso <= ownb.y)) act |= 1u << (li - 2);
                    if (PLO < iso && iso <= PHI) can |= 1u << (li - 2);
                }
                l3a = l3b;
                h3a = h3b;
                l3b = l3;
                h3b = h3;
                p2lb = p2l;
                p2hb = p2h;
                ownb = own;
            }
            // the slots of the active blocks (new: none), their loads in flight together
            int32_t sl[CULL_TZ];
#pragma unroll
            for (int z = 0; z < CULL_TZ; z++) {
                sl[z] = 0;
                if (!identity && ((act >> z) & 1u))
                    sl[z] = I_slot[((uint64_t)(z0 + z) * g.nby + by) * g.nbx + bx];
            }
#pragma unroll
            for (int z = 0; z < CULL_TZ; z++) {
                if (z0 + z >= z1) break;
                const bool a = (act >> z) & 1u;
                const uint64_t b = ((uint64_t)(z0 + z) * g.nby + by) * g.nbx + bx;
                active[b] = (a ? 1u : 0u) | (((can >> z) & 1u) ? 2u : 0u) | (a && sl[z] < 0 ? 4u : 0u);
            }
        }
        // mark the 4096-block rounds holding active blocks for the
        // compaction: each half-wave is 32 consecutive blocks of one row, so
        // its first and last active lanes name every round
#pragma unroll
        for (int z = 0; z < CULL_TZ; z++) {
            const bool a = (act >> z) & 1u;
            const uint64_t am = __ballot(a);
            const uint32_t half = (uint32_t)(am >> (lane() & 32));
            const int hl = lane() & 31;
            if (a && (hl == __builtin_ctz(half) || hl == 31 - __builtin_clz(half)))
                round_gen[(((uint64_t)(z0 + z) * g.nby + by) * g.nbx + bx) / BLK_TILE] = gen;
        }
        __syncthreads();   // sh is restaged for the next live tile
    }
}

// I_active (StreamCompactIDs of M_active) and I_new (active blocks without a
// slot, Alg. 1 MarkNewBlocks, flagged by the cull).  The blocks are cut into
// rounds of 4096 consecutive blocks, and the cull stamped every round holding
// an active block with the call's gen (the other rounds' flags are all zero).
// k_round_list lists the live rounds in ascending order; k_round_counts
// counts each one's active and new blocks, k_round_scan turns the counts into
// offsets, and k_compact_blocks writes each round's ids there.  A surface
// makes runs of live rounds: taking them one per workgroup (rounds w, w + G,
// ...) spreads a run over the chip, with no waiting between workgroups and no
// shared counter.  In a round each thread takes 16 consecutive flags (one
// 16-byte load).
// Bit 0 of each byte of w, gathered into bits 0..3: the four bits land on
// bits 21..24 of the product with no carries between them.
__device__ __forceinline__ uint32_t byte_bits(uint32_t w) {
    return (((w & 0x01010101u) * 0x00204081u) >> 21) & 0xFu;
}

__device__ __forceinline__ void flag_bits(uint4 q, uint32_t &actb, uint32_t &newb, uint32_t &cand) {
    actb = newb = 0;
    if ((q.x | q.y | q.z | q.w) == 0) return;   // the common case of a sparse volume
    const uint32_t wds[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int i = 0; i < 4; i++) {   // flags use bits 0..2 of each byte
        const uint32_t w = wds[i];
        actb |= byte_bits(w | (w >> 1) | (w >> 2)) << (4 * i);
        newb |= byte_bits(w >> 2) << (4 * i);
        cand += (uint32_t)__popc(w & 0x02020202u);
    }
}

__device__ __forceinline__ uint4 load_flags16(const uint8_t *__restrict__ active, uint64_t base,
                                              uint64_t nb) {
    if (base + 16 <= nb) return *reinterpret_cast<const uint4 *>(active + base);
    uint32_t wd[4] = {0, 0, 0, 0};
    for (int j = 0; j < 16; j++)
        if (base + j < nb) wd[j >> 2] |= (uint32_t)active[base + j] << (8 * (j & 3));
    return make_uint4(wd[0], wd[1], wd[2], wd[3]);
}


// The live rounds (round_gen == gen) in ascending order: 16 stamps per thread
// (4096 per workgroup), a look-back over the workgroups; the last one writes
// their number.
__global__ __launch_bounds__(256) void k_round_list(const uint32_t *__restrict__ round_gen, uint64_t n_rounds,
                                                   uint32_t gen, uint32_t *__restrict__ list, Counters *ctr,
                                                   uint64_t *status) {
    const uint64_t t = take_tile(&ctr->tile_ctr[TC_ROUNDS]);   // look-back order = start order
    const uint64_t n_tiles = (n_rounds + 4095) / 4096;
    const uint64_t r0 = t * 4096 + 16u * threadIdx.x;
    uint32_t live = 0;   // bit j: round r0 + j
    if (r0 + 16 <= n_rounds) {
        const uint4 *p = reinterpret_cast<const uint4 *>(round_gen + r0);
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const uint4 q = p[k];
            live |= ((q.x == gen ? 1u : 0u) | (q.y == gen ? 2u : 0u) | (q.z == gen ? 4u : 0u) |
                     (q.w == gen ? 8u : 0u)) << (4 * k);
        }
    } else {
        for (int j = 0; j < 16; j++)
            if (r0 + j < n_rounds && round_gen[r0 + j] == gen) live |= 1u << j;
    }
    uint64_t total;
    uint64_t o = tile_scan_lookback((uint64_t)__popc(live), status, t, &total);
    for (uint32_t m = live; m; m &= m - 1) list[o++] = (uint32_t)(r0 + __builtin_ctz(m));
    if (t == n_tiles - 1 && threadIdx.x == 0) ctr->n_live_rounds = total;
}

// Per live round: (active << 32 | new) blocks, and the blocks that may emit.
__global__ __launch_bounds__(256) void k_round_counts(Geom g, const uint8_t *__restrict__ active,
                                                     const uint32_t *__restrict__ round_list,
                                                     uint64_t *__restrict__ round_cnt,
                                                     uint32_t *__restrict__ part_cand, const Counters *ctr) {
    __shared__ uint64_t s_part[4];
    const uint64_t n_live = ctr->n_live_rounds;
    for (uint64_t k = blockIdx.x; k < n_live; k += gridDim.x) {
        const uint64_t base = (uint64_t)round_list[k] * BLK_TILE + 16u * threadIdx.x;
        uint32_t actb, newb, cand = 0;
        flag_bits(load_flags16(active, base, g.nb), actb, newb, cand);
        // three counts of at most 4096 in 21-bit fields
        uint64_t v = (uint64_t)__popc(actb) | ((uint64_t)__popc(newb) << 21) | ((uint64_t)cand << 42);
        v = wave_sum(v);
        if (lane() == 0) s_part[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint64_t t = s_part[0] + s_part[1] + s_part[2] + s_part[3];
            const uint64_t m21 = (1ull << 21) - 1;
            round_cnt[k] = ((t & m21) << 32) | ((t >> 21) & m21);
            part_cand[k] = (uint32_t)(t >> 42);
        }
        __syncthreads();   // s_part is rewritten by the next round
    }
}

// Exclusive prefix of the live rounds' counts, in place; the totals are the
// call's n_act and n_new.  One workgroup, 4096 rounds per step.
__global__ __launch_bounds__(256) void k_round_scan(uint64_t *__restrict__ round_cnt, Counters *ctr) {
    __shared__ uint64_t s_w[4];
    const uint64_t n = ctr->n_live_rounds;
    const int w = threadIdx.x >> 6;
    uint64_t carry = 0;
    for (uint64_t c0 = 0; c0 < n; c0 += 4096) {
        const uint64_t i0 = c0 + 16u * threadIdx.x;
        uint64_t v[16], sum = 0;
#pragma unroll
        for (int j = 0; j < 16; j++) {
            v[j] = i0 + j < n ? round_cnt[i0 + j] : 0ull;
            sum += v[j];
        }
        const uint64_t incl = wave_incl_scan(sum);
        if (lane() == 63) s_w[w] = incl;
        __syncthreads();
        uint64_t o = carry + incl - sum, tot = 0;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            if (i < w) o += s_w[i];
            tot += s_w[i];
        }
#pragma unroll
        for (int j = 0; j < 16; j++) {
            if (i0 + j < n) round_cnt[i0 + j] = o;
            o += v[j];
        }
        carry += tot;
        __syncthreads();   // s_w is rewritten by the next step
    }
    if (threadIdx.x == 0) {
        ctr->n_act = carry >> 32;
        ctr->n_new = carry & 0xFFFFFFFFull;
    }
}

// Each live round's active and new block ids, from its offsets on.  A wave
// takes 1024 consecutive flags of the round (16 per lane, one 16-byte load),
// puts them in LDS and writes the ids 64 blocks at a time: lane l takes block
// 64 j + l, a ballot orders the wave's ids, and each store covers one
// contiguous run of the lists.
__global__ __launch_bounds__(256) void k_compact_blocks(Geom g, const uint8_t *__restrict__ active,
                                                       const uint32_t *__restrict__ round_list,
                                                       const uint64_t *__restrict__ round_off,
                                                       uint32_t *__restrict__ I_active,
                                                       uint32_t *__restrict__ I_new, const Counters *ctr) {
    __shared__ uint32_t s_w[4];
    __shared__ uint4 s_fl[4][64];   // per wave: its 1024 flags in block order
    const uint64_t n_live = ctr->n_live_rounds;
    const int w = threadIdx.x >> 6, l = lane();
    for (uint64_t k = blockIdx.x; k < n_live; k += gridDim.x) {
        const uint64_t wbase = (uint64_t)round_list[k] * BLK_TILE + 1024u * w;
        const uint64_t off = round_off[k];
        const uint4 q = load_flags16(active, wbase + 16u * l, g.nb);
        uint32_t actb, newb, unused = 0;
        flag_bits(q, actb, newb, unused);
        const uint32_t tot = wave_sum(((uint32_t)__popc(actb) << 16) | (uint32_t)__popc(newb));   // < 2^11 each
        if (l == 0) s_w[w] = tot;
        s_fl[w][l] = q;
        __syncthreads();
        uint32_t ex = 0;
#pragma unroll
        for (int i = 0; i < 4; i++)
            if (i < w) ex += s_w[i];
        uint64_t pa = (off >> 32) + (ex >> 16), pn = (off & 0xFFFFFFFFull) + (ex & 0xFFFFu);
        if (tot) {
            const uint8_t *fl = reinterpret_cast<const uint8_t *>(s_fl[w]);
#pragma unroll 4
            for (int j = 0; j < 16; j++) {
                const uint32_t f = fl[64 * j + l];
                const bool a = (f & 7u) != 0, nw = (f & 4u) != 0;   // any flag bit marks an active block
                const uint64_t am = __ballot(a), nm = __ballot(nw);
                const uint32_t blk = (uint32_t)(wbase + 64u * j + (uint32_t)l);
                if (a) I_active[pa + mbcnt(am)] = blk;
                if (nw) I_new[pn + mbcnt(nm)] = blk;
                pa += (uint64_t)__popcll(am);
                pn += (uint64_t)__popcll(nm);
            }
        }
        __syncthreads();   // s_w and s_fl are rewritten by the next round
    }
}

// Alg. 1 IncrementSlotAge + the slot half of MarkNewBlocks, then
// StreamCompactIDs of the available slots (I_avail) and StreamCompact of their
// ages (K_age, stored as ~age so that ascending key = descending age).
__global__ __launch_bounds__(256) void k_slot_pass(const uint8_t *__restrict__ active,
                                                  const int32_t *__restrict__ S_block,
                                                  uint32_t *__restrict__ S_age, uint64_t n_slots,
                                                  uint32_t age_cap, uint32_t *__restrict__ keys,
                                                  uint32_t *__restrict__ vals,
                                                  uint32_t *__restrict__ part_or,
                                                  uint32_t *__restrict__ part_and, Counters *ctr,
                                                  uint64_t *status) {
    const uint64_t n_tiles = (n_slots + SLOT_TILE - 1) / SLOT_TILE;
    // the list of available slots (look-back order = ticket order) is needed
    // only when the call has new blocks; otherwise the tiles just age, in any
    // order, without a shared ticket counter
    const bool need_list = ctr->n_new != 0;
    const uint32_t t = need_list ? take_tile(&ctr->tile_ctr[TC_SLOT]) : blockIdx.x;
    if (t >= n_tiles) return;
    constexpr int PER = SLOT_TILE / 256;   // consecutive slots per thread (16-byte loads)
    static_assert(PER % 4 == 0, "the vector path loads 4 slots at a time");
    const uint64_t base = (uint64_t)t * SLOT_TILE + threadIdx.x * PER;
    uint32_t availb = 0;
    uint32_t age[PER];
    int32_t blk[PER];
    uint32_t kor = 0, kand = ~0u, key[PER];
    const bool full = base + PER <= n_slots;
    if (full) {
#pragma unroll
        for (int j = 0; j < PER; j += 4) {
            const int4 bq = *reinterpret_cast<const int4 *>(S_block + base + j);
            const uint4 aq = *reinterpret_cast<const uint4 *>(S_age + base + j);
            blk[j] = bq.x; blk[j + 1] = bq.y; blk[j + 2] = bq.z; blk[j + 3] = bq.w;
            age[j] = aq.x; age[j + 1] = aq.y; age[j + 2] = aq.z; age[j + 3] = aq.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < PER; j++) {
            blk[j] = base + j < n_slots ? S_block[base + j] : -1;
            age[j] = base + j < n_slots ? S_age[base + j] : 0u;
        }
    }
#pragma unroll
    for (int j = 0; j < PER; j++) {
        key[j] = 0u;
        if (base + j < n_slots) {
            const bool act = blk[j] >= 0 && active[blk[j]];
            uint32_t a = age[j];
            a = act ? 0u : (a == 0xFFFFFFFFu ? a : a + 1u);
            age[j] = a;
            if (!act) {
                availb |= 1u << j;
                // sort key, ascending = oldest first: slots never used (age
                // >= HIGH_AGE, created in slot order) before every used one,
                // used ones by age descending.  age_cap exceeds every used
                // slot's age, so the keys keep the exact order in few digits.
                key[j] = a >= HIGH_AGE ? 0u : age_cap - a;
                kor |= key[j];
                kand &= key[j];
            }
        }
    }
    if (full) {
#pragma unroll
        for (int j = 0; j < PER; j += 4)
            *reinterpret_cast<uint4 *>(S_age + base + j) = make_uint4(age[j], age[j + 1], age[j + 2], age[j + 3]);
    } else {
#pragma unroll
        for (int j = 0; j < PER; j++)
            if (base + j < n_slots) S_age[base + j] = age[j];
    }
    if (!need_list) return;
    uint64_t incl_end;
    uint64_t e = tile_scan_lookback((uint64_t)__popc(availb), status, t, &incl_end);
#pragma unroll
    for (int j = 0; j < PER; j++)
        if ((availb >> j) & 1u) {
            keys[e] = key[j];
            vals[e] = (uint32_t)(base + j);
            e++;
        }
    // OR / AND of the keys (which radix digits vary), one entry per tile
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        kor |= __shfl_xor(kor, d, 64);
        kand &= __shfl_xor(kand, d, 64);
    }
    __shared__ uint32_t s_or[4], s_and[4];
    if (lane() == 0) {
        s_or[threadIdx.x >> 6] = kor;
        s_and[threadIdx.x >> 6] = kand;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part_or[t] = s_or[0] | s_or[1] | s_or[2] | s_or[3];
        part_and[t] = s_and[0] & s_and[1] & s_and[2] & s_and[3];
    }
    if (t == n_tiles - 1 && threadIdx.x == 0) ctr->n_avail_old = incl_end;
}

// Alg. 1's early exit (nothing new) and growth (more new blocks than available
// slots): every workgroup
// derives the same plan from values no kernel of this launch writes; block 0
// publishes it and all threads initialise the appended slots (empty,
// available, age HIGH_AGE) and append them to the available list.
__global__ __launch_bounds__(256) void k_plan_grow(Counters *ctr, uint64_t max_slots,
                                                  int32_t *__restrict__ S_block,
                                                  uint32_t *__restrict__ S_age,
                                                  uint32_t *__restrict__ keys,
                                                  uint32_t *__restrict__ vals,
                                                  const uint32_t *__restrict__ part_or,
                                                  const uint32_t *__restrict__ part_and) {
    const uint64_t n_new = ctr->n_new;
    if (ctr->err || n_new == 0) return;
    const uint64_t na = ctr->n_avail_old, ns = ctr->n_slots_old;
    uint64_t grow = 0;
    if (n_new > na) {
        grow = n_new - na;
        uint64_t half = (ns + 1) / 2;
        if (half > grow) grow = half;
        if (ns + grow > max_slots) grow = max_slots - ns;
    }
    const uint64_t gid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (na + grow < n_new) {
        if (gid == 0) ctr->err |= ERR_CACHE_CAP;
        return;
    }
    if (blockIdx.x == 0) {   // the keys' OR / AND from the slot pass's tiles
        const uint64_t n_tiles = (ns + SLOT_TILE - 1) / SLOT_TILE;
        uint32_t o = 0u, a = ~0u;
        for (uint64_t i = threadIdx.x; i < n_tiles; i += blockDim.x) {
            o |= part_or[i];
            a &= part_and[i];
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            o |= __shfl_xor(o, d, 64);
            a &= __shfl_xor(a, d, 64);
        }
        __shared__ uint32_t s_or[4], s_and[4];
        if (lane() == 0) {
            s_or[threadIdx.x >> 6] = o;
            s_and[threadIdx.x >> 6] = a;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            ctr->key_or = s_or[0] | s_or[1] | s_or[2] | s_or[3];
            ctr->key_and = s_and[0] & s_and[1] & s_and[2] & s_and[3];
        }
    }
    if (gid == 0) {
        uint32_t kor = ctr->key_or, kand = ctr->key_and;
        if (grow) kand = 0u;   // appended slots: key 0
        uint32_t vary = kor ^ kand;
        uint32_t mask = 0;
        for (int p = 0; p < 4; p++)
            if ((vary >> (8 * p)) & 0xFFu) mask |= 1u << p;
        ctr->pass_mask = mask;
        ctr->n_grow = grow;
        ctr->n_slots = ns + grow;
        ctr->n_avail = na + grow;
    }
    for (uint64_t i = gid; i < grow; i += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t s = ns + i;
        S_block[s] = -1;
        S_age[s] = HIGH_AGE;
        keys[na + i] = 0u;
        vals[na + i] = (uint32_t)s;
    }
}

// ---------------------------------------------------------------------------
// Alg. 1 SortByKey: stable LSD radix sort of the available slots by ~age
// (8-bit digits).  Digits on which every key agrees are skipped: a pass over
// such a digit is the identity.  Tiles of 1024 elements are owned by single
// waves, striped as element = tile*1024 + round*64 + lane.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool radix_pass_live(const Counters *ctr, int p) {
    return !ctr->err && ctr->n_new != 0 && ((ctr->pass_mask >> p) & 1u);
}
__device__ __forceinline__ int radix_in_buf(const Counters *ctr, int p) {
    return __popc(ctr->pass_mask & ((1u << p) - 1u)) & 1;
}

__global__ __launch_bounds__(256) void k_radix_hist(Counters *ctr, int p,
                                                   const uint32_t *__restrict__ keys0,
                                                   const uint32_t *__restrict__ keys1,
                                                   uint32_t *__restrict__ hist, uint64_t *status) {
    if (!radix_pass_live(ctr, p)) return;
    const uint32_t *keys = radix_in_buf(ctr, p) ? keys1 : keys0;
    const uint64_t n = ctr->n_avail;
    const uint64_t n_tiles = (n + RADIX_TILE - 1) / RADIX_TILE;
    const uint64_t gid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    const uint64_t gsz = (uint64_t)gridDim.x * blockDim.x;
    // clear the scan's status words and tile counter for this pass
    const uint64_t scan_tiles = (256 * n_tiles + SCAN_TILE - 1) / SCAN_TILE;
    for (uint64_t w = gid; w < scan_tiles; w += gsz) status[w] = 0;
    if (gid == 0) ctr->tile_ctr[TC_SCAN0 + p] = 0;
    __shared__ uint32_t h[4][256];
    const int w = threadIdx.x >> 6;
    const int shift = 8 * p;
    const uint64_t waves = (uint64_t)gridDim.x * 4;
    for (uint64_t tb = blockIdx.x * 4ull; tb < n_tiles; tb += waves) {
        uint64_t tile = tb + w;
        for (int i = lane(); i < 256; i += 64) h[w][i] = 0;
        __syncthreads();
        if (tile < n_tiles) {
            for (int r = 0; r < RADIX_TILE / 64; r++) {
                uint64_t idx = tile * RADIX_TILE + r * 64 + lane();
                if (idx < n) atomicAdd(&h[w][(keys[idx] >> shift) & 0xFFu], 1u);
            }
        }
        __syncthreads();
        if (tile < n_tiles)
            for (int d = lane(); d < 256; d += 64) hist[(uint64_t)d * n_tiles + tile] = h[w][d];
        __syncthreads();
    }
}

// In-place exclusive scan of the digit-major histogram (256 * n_tiles u32).
__global__ __launch_bounds__(256) void k_radix_scan(Counters *ctr, int p, uint32_t *hist,
                                                   uint64_t *status) {
    if (!radix_pass_live(ctr, p)) return;
    const uint64_t n_tiles = (ctr->n_avail + RADIX_TILE - 1) / RADIX_TILE;
    const uint64_t len = 256 * n_tiles;
    const uint64_t scan_tiles = (len + SCAN_TILE - 1) / SCAN_TILE;
    for (;;) {
        const uint32_t t = take_tile(&ctr->tile_ctr[TC_SCAN0 + p]);
        if (t >= scan_tiles) return;
        constexpr int PER = SCAN_TILE / 256;   // consecutive entries per thread
        const uint64_t base = (uint64_t)t * SCAN_TILE + threadIdx.x * PER;
        uint32_t x[PER];
        uint64_t sum = 0;
#pragma unroll
        for (int j = 0; j < PER; j++) {
            x[j] = base + j < len ? hist[base + j] : 0u;
            sum += x[j];
        }
        uint64_t incl_end;
        uint64_t e = tile_scan_lookback(sum, status, t, &incl_end);
#pragma unroll
        for (int j = 0; j < PER; j++) {
            if (base + j < len) hist[base + j] = (uint32_t)e;
            e += x[j];
        }
    }
}

__global__ __launch_bounds__(256) void k_radix_scatter(Counters *ctr, int p,
                                                      uint32_t *keys0, uint32_t *keys1,
                                                      uint32_t *vals0, uint32_t *vals1,
                                                      const uint32_t *__restrict__ hist) {
    if (!radix_pass_live(ctr, p)) return;
    const int in = radix_in_buf(ctr, p);
    const uint32_t *__restrict__ kin = in ? keys1 : keys0;
    const uint32_t *__restrict__ vin = in ? vals1 : vals0;
    uint32_t *__restrict__ kout = in ? keys0 : keys1;
    uint32_t *__restrict__ vout = in ? vals0 : vals1;
    const uint64_t n = ctr->n_avail;
    const uint64_t n_tiles = (n + RADIX_TILE - 1) / RADIX_TILE;
    __shared__ uint32_t off[4][256];
    const int w = threadIdx.x >> 6;
    const int l = lane();
    const int shift = 8 * p;
    const uint64_t lt = (1ull << l) - 1ull;
    const uint64_t waves = (uint64_t)gridDim.x * 4;
    for (uint64_t tile = blockIdx.x * 4ull + w; tile < n_tiles; tile += waves) {
        for (int d = l; d < 256; d += 64) off[w][d] = hist[(uint64_t)d * n_tiles + tile];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int r = 0; r < RADIX_TILE / 64; r++) {
            uint64_t idx = tile * RADIX_TILE + r * 64 + l;
            bool valid = idx < n;
            uint32_t key = valid ? kin[idx] : 0u;
            uint32_t val = valid ? vin[idx] : 0u;
            uint32_t d = (key >> shift) & 0xFFu;
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int bit = 0; bit < 8; bit++) {
                uint64_t m = __ballot((d >> bit) & 1u);
                peers &= ((d >> bit) & 1u) ? m : ~m;
            }
            uint32_t base = off[w][d];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (valid) {
                uint32_t pos = base + (uint32_t)__popcll(peers & lt);
                if (pos < n) {
                    kout[pos] = key;
                    vout[pos] = val;
                } else {
                    atomicOr(&ctr->err, ERR_INTERNAL);
                }
                if ((peers & lt) == 0) off[w][d] = base + (uint32_t)__popcll(peers);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
}

// Sign masks (Sec. 4.4's per-cell classification, one bit per sample): for
// every active block, bit i of masks[slot] is set when sample i of the
// block (x fastest) is below iso.  One lane per block: its 16 float4 loads
// are all in flight before the first compare.
__global__ __launch_bounds__(256) void k_masks(const uint32_t *__restrict__ I_active,
                                              const int32_t *__restrict__ I_slot, int identity,
                                              const float *__restrict__ slots, float iso,
                                              uint64_t *__restrict__ masks,
                                              uint32_t *__restrict__ mask_iso,
                                              const Counters *ctr) {
    if (ctr->err) return;
    const uint64_t n_act = ctr->n_act;
    // every active block was decoded by this call, its mask with it
    if (!identity && ctr->n_new == n_act) return;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n_act;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t b = I_active[i];
        const int32_t s = identity ? (int32_t)b : I_slot[b];
        if (s < 0) continue;
        const uint32_t tag = __float_as_uint(iso);
        if (!identity && mask_iso[s] == tag) continue;   // built for this isovalue already
        const float4 *src = reinterpret_cast<const float4 *>(slots) + (uint64_t)s * 16;
        float4 v[16];
#pragma unroll
        for (int q = 0; q < 16; q++) v[q] = src[q];
        uint64_t m = 0;
#pragma unroll
        for (int q = 0; q < 16; q++) {
            const uint64_t nib = (v[q].x < iso ? 1u : 0u) | (v[q].y < iso ? 2u : 0u) |
                                 (v[q].z < iso ? 4u : 0u) | (v[q].w < iso ? 8u : 0u);
            m |= nib << (4 * q);
        }
        masks[s] = m;
        if (!identity) mask_iso[s] = tag;
    }
}

// Count pass (Sec. 4.4): vertex count of every active block (0 unless it can
// emit), one lane per block, over the chunks of xcd_chunks (mc_chunk_size
// blocks each); each chunk's total goes to chunk_off for k_chunk_scan.  The
// cases of all 64 cells are evaluated at once on the corner masks, and the
// triangle count per case by the bit-sliced diagram of the marching-cubes
// table (mc_ntri_bits, generated at build time).
__global__ __launch_bounds__(256) void k_mc_count(Geom g, const uint32_t *__restrict__ I_active,
                                                 const uint8_t *__restrict__ active,
                                                 const int32_t *__restrict__ I_slot, int identity,
                                                 const uint64_t *__restrict__ masks,
                                                 uint32_t *__restrict__ blk_cnt,
                                                 uint64_t *__restrict__ chunk_off,
                                                 uint32_t *__restrict__ part_occw, uint32_t emit_waves,
                                                 Counters *ctr) {
    if (ctr->err) return;
    const uint64_t n_act = ctr->n_act;
    const uint32_t cs = mc_chunk_size(n_act, emit_waves);   // the emission's chunks
    const ChunkRange cr = xcd_chunks((n_act + cs - 1) / cs);
    uint32_t wocc = 0;
    for (uint64_t c = cr.first; c < cr.end; c += cr.stride) {
        const uint64_t i = c * cs + lane();
        const bool in = lane() < (int)cs && i < n_act;
        uint32_t cnt = 0;
        const uint32_t b = in ? I_active[i] : 0u;
        if (in && (active[b] & 2u)) {
            uint32_t so[8], bx, by, bz;
            if (!octet(g, b, I_slot, identity, so, bx, by, bz)) {
                atomicOr(&ctr->err, ERR_INTERNAL);
            } else {
                uint64_t M[8], cm[8];
#pragma unroll
                for (int m = 0; m < 8; m++) M[m] = masks[so[m]];
                corner_masks(M, cm);
                uint64_t n0, n1, n2;
                mc_ntri_bits(cm, n0, n1, n2);
                const uint64_t V = valid_cells(g, bx, by, bz);
                const uint32_t tris = (uint32_t)__popcll(n0 & V) + 2u * (uint32_t)__popcll(n1 & V) +
                                      4u * (uint32_t)__popcll(n2 & V);
                cnt = 3u * tris;
            }
        }
        if (in) blk_cnt[i] = cnt;
        const uint32_t tot = wave_sum(cnt);   // the chunk's vertices (k_chunk_scan turns them into offsets)
        if (lane() == 0) chunk_off[c] = tot;
        wocc += cnt ? 1u : 0u;
    }
    wocc = wave_sum(wocc);
    if (lane() == 0) part_occw[blockIdx.x * MC_WAVES + (threadIdx.x >> 6)] = wocc;
}

// Sec. 4.4's prefix sum over the block counts, at the granularity of the
// count pass's chunks (up to 64 blocks).  Workgroup x < 8 scans the chunk
// totals of XCD eighth x (the split of xcd_chunks) in place, exclusively, in
// rounds of 16 K chunks (thread t holds chunks t + 1024 j, j < 16: coalesced loads; a
// chunk holds at most 64 * 960 vertices, so a round's sums fit 32 bits), and
// writes the eighth's total to xcd_tot[x] (the emission adds the totals of
// the eighths before its own).  Workgroup 8 forms the call's occupied and
// may-emit block counts.
__global__ __launch_bounds__(1024) void k_chunk_scan(uint64_t *__restrict__ chunk_off,
                                                    uint64_t *__restrict__ xcd_tot,
                                                    const uint32_t *__restrict__ part_occw,
                                                    uint32_t n_waves, uint32_t emit_waves,
                                                    const uint32_t *__restrict__ part_cand,
                                                    Counters *ctr) {
    constexpr int J = 16;
    __shared__ uint32_t s_w[J * 16];   // per (j, wave): the wave's total, then its exclusive prefix
    __shared__ uint32_t s_round;
    __shared__ uint32_t s_occ[16], s_cand[16];
    if (ctr->err) return;
    const int t = threadIdx.x, w = t >> 6, l = lane();
    if (blockIdx.x < 8) {
        const uint32_t cs = mc_chunk_size(ctr->n_act, emit_waves);
        const uint64_t n = (ctr->n_act + cs - 1) / cs, per = (n + 7) / 8;
        uint64_t lo = blockIdx.x * per;
        if (lo > n) lo = n;
        const uint64_t hi = lo + per < n ? lo + per : n;
        uint64_t carry = 0;
        for (uint64_t base = lo; base < hi; base += J * 1024) {
            uint32_t v[J], inc[J];
#pragma unroll
            for (int j = 0; j < J; j++) {
                const uint64_t i = base + 1024 * (uint64_t)j + t;
                v[j] = i < hi ? (uint32_t)chunk_off[i] : 0u;
            }
#pragma unroll
            for (int j = 0; j < J; j++) inc[j] = wave_incl_scan(v[j]);
            if (l == 63) {
#pragma unroll
                for (int j = 0; j < J; j++) s_w[16 * j + w] = inc[j];
            }
            __syncthreads();
            if (w == 0) {   // exclusive scan of the 256 wave totals in chunk order (j, then wave)
                uint32_t e[4], run = 0;
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const uint32_t x = s_w[4 * l + k];
                    e[k] = run;
                    run += x;
                }
                const uint32_t incl = wave_incl_scan(run);
#pragma unroll
                for (int k = 0; k < 4; k++) s_w[4 * l + k] = incl - run + e[k];
                if (l == 63) s_round = incl;
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < J; j++) {
                const uint64_t i = base + 1024 * (uint64_t)j + t;
                if (i < hi) chunk_off[i] = carry + s_w[16 * j + w] + (inc[j] - v[j]);
            }
            carry += s_round;
            __syncthreads();   // s_w and s_round are rewritten next round
        }
        if (t == 0) xcd_tot[blockIdx.x] = carry;
        return;
    }
    // 8 loads in flight per thread (a plain loop waits for each load)
    uint32_t occ = 0, cand = 0;
    for (uint32_t i0 = t; i0 < n_waves; i0 += 8 * 1024) {
        uint32_t x[8];
#pragma unroll
        for (int j = 0; j < 8; j++) x[j] = i0 + 1024u * j < n_waves ? part_occw[i0 + 1024u * j] : 0u;
#pragma unroll
        for (int j = 0; j < 8; j++) occ += x[j];
    }
    const uint64_t n_ct = ctr->n_live_rounds;
    for (uint64_t i0 = t; i0 < n_ct; i0 += 8 * 1024) {
        uint32_t x[8];
#pragma unroll
        for (int j = 0; j < 8; j++) x[j] = i0 + 1024u * j < n_ct ? part_cand[i0 + 1024u * j] : 0u;
#pragma unroll
        for (int j = 0; j < 8; j++) cand += x[j];
    }
    occ = wave_sum(occ);
    cand = wave_sum(cand);
    if (l == 0) {
        s_occ[w] = occ;
        s_cand[w] = cand;
    }
    __syncthreads();
    if (t == 0) {
        uint32_t o = 0, c = 0;
        for (int k = 0; k < 16; k++) {
            o += s_occ[k];
            c += s_cand[k];
        }
        ctr->n_occ = o;
        ctr->n_cand = c;
    }
}


// Emission pass (Sec. 4.5), over the chunks of xcd_chunks (the count pass's
// schedule), each from its scanned offset: the chunk's block offsets by a
// wave scan of the counts, then the occupied blocks restaged a few at a time;
// each block's in-block prefix of its per-cell triangle counts, the
// triangles of the staged blocks listed together and written lane per vertex
// from the first block's offset, in canonical order (block, cell, triangle,
// vertex).
template <int FMT>
__global__ __launch_bounds__(256, FMT == VFMT_GRAD ? 5 : 7) void k_mc_emit(Geom g, const uint32_t *__restrict__ I_active,
                                                const int32_t *__restrict__ I_slot, int identity,
                                                const float *__restrict__ slots,
                                                const uint64_t *__restrict__ mc_table, float iso,
                                                const uint32_t *__restrict__ blk_cnt,
                                                uint64_t *__restrict__ blk_off,
                                                void *__restrict__ out, uint64_t cap,
                                                const uint64_t *__restrict__ chunk_off,
                                                const uint64_t *__restrict__ xcd_tot,
                                                uint32_t chunk_waves, Counters *ctr,
                                                const float *__restrict__ gV = nullptr,
                                                float *__restrict__ dfield = nullptr,
                                                float *__restrict__ part_giso = nullptr) {
    __shared__ std::conditional_t<FMT == VFMT_GRAD, EmitSharedGrad, EmitSharedPlain> sh;
    if (ctr->err) return;
    for (int i = threadIdx.x; i < 256; i += blockDim.x) sh.tab[i] = mc_table[i];
    if (threadIdx.x < 16) sh.edge[threadIdx.x] = edge_entry((int)threadIdx.x);
    if constexpr (FMT == VFMT_GRAD) {
        for (int i = threadIdx.x; i < MC_WAVES * EMIT_SB * 128; i += blockDim.x) (&sh.acc[0][0][0])[i] = 0.0f;
    }
    __syncthreads();
    const uint64_t n_act = ctr->n_act;
    const int w = threadIdx.x >> 6, l = lane();
    const uint32_t cs = mc_chunk_size(n_act, chunk_waves);   // the count pass's chunks
    const ChunkRange cr = xcd_chunks((n_act + cs - 1) / cs);
    GradCtx gc;
    if constexpr (FMT == VFMT_GRAD) {
        gc.gV = gV;
        gc.dfield = dfield;
        gc.err = &ctr->err;
        gc.nbx = g.nbx;
        gc.nbxy = g.nbx * g.nby;
        gc.giso = 0.0f;
    }
    // the vertices of the XCD eighths before this workgroup's (the chunk
    // offsets are local to their eighth); workgroup 0 forms the call's total
    uint64_t xbase = 0, all = 0;
    for (uint32_t x = 0; x < 8; x++) {
        const uint64_t tx = xcd_tot[x];
        xbase += x < blockIdx.x % 8u ? tx : 0ull;
        all += tx;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) ctr->total_verts = all;
    const LaneGeom q = lane_geom();
    for (uint64_t c = cr.first; c < cr.end; c += cr.stride) {
        const uint64_t base = xbase + chunk_off[c];   // the chunk's first vertex (wave-uniform)
        const uint64_t idx = c * cs + l;
        const bool valid = l < (int)cs && idx < n_act;
        const uint32_t cnt = valid ? blk_cnt[idx] : 0u;
        const uint32_t incl = wave_incl_scan(cnt);
        const uint64_t off = base + (incl - cnt);
        if (valid) blk_off[idx] = off;
        const uint32_t b = cnt ? I_active[idx] : 0u;
        const uint64_t boff = off;
        uint32_t so[8], lbx, lby, lbz;
        octet(g, b, I_slot, identity, so, lbx, lby, lbz);
        uint64_t todo = __ballot(cnt != 0);
        while (todo) {
            const uint64_t left = todo;
            int jl[EMIT_SB], nsb = 0;
#pragma unroll
            for (int k = 0; k < EMIT_SB; k++) {
                jl[k] = k ? jl[0] : 0;
                if (todo) {
                    jl[k] = (int)__builtin_ctzll(todo);
                    todo &= todo - 1;
                    nsb++;
                }
            }
            // the triangle list area is empty between batches (emit_batch flushes)
            static_assert(8 * EMIT_SB <= EMIT_TRIS, "slot table fits the triangle list");
            stage_batch_tab<EMIT_SB>(q, slots, so, left & ~todo, nsb, sh.tri[w], sh.tiles[w]);
            wave_lds_sync();
            // the staged blocks are consecutive occupied blocks: their vertex
            // ranges follow each other from the first one's offset, so their
            // triangles are listed together and written by one lane-per-vertex
            // loop (a block's last partial pass of 64 lanes is shared)
            const uint64_t ob = ((uint64_t)bcast((uint32_t)(boff >> 32), jl[0]) << 32) |
                                bcast((uint32_t)boff, jl[0]);
            auto info = [&](int k, Geom &gk, uint32_t &bk, uint32_t &bx, uint32_t &by, uint32_t &bz,
                            float &isok) {
                gk = g;
                bk = bcast(b, jl[k]);
                bx = bcast(lbx, jl[k]);
                by = bcast(lby, jl[k]);
                bz = bcast(lbz, jl[k]);
                isok = iso;
            };
            if constexpr (FMT == VFMT_GRAD) {
#pragma unroll
                for (int k = 0; k < EMIT_SB; k++) gc.expect[k] = bcast(cnt, jl[k]);
            }
            emit_batch<FMT>(nsb, info, sh.tiles[w], sh.tab, sh, w, ob, out, cap, &gc);
        }
    }
    if constexpr (FMT == VFMT_GRAD) {   // the wave's share of dL/diso (summed by k_sum_f32: no
                                        // same-address atomics, a fixed order)
        const float gi = wave_sum(gc.giso);
        if (l == 0) part_giso[blockIdx.x * MC_WAVES + w] = gi;
    }
}

// out = sum of p[0..n) in a fixed order (one workgroup of 1024 threads).
__global__ __launch_bounds__(1024) void k_sum_f32(const float *__restrict__ p, uint32_t n,
                                                 float *__restrict__ out) {
    __shared__ float s_w[16];
    float v = 0.0f;
    for (uint32_t i = threadIdx.x; i < n; i += 1024) v += p[i];
    v = wave_sum(v);
    if (lane() == 0) s_w[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.0f;
        for (int k = 0; k < 16; k++) t += s_w[k];
        *out = t;
    }
}

// Cases of every cell of every active block (0 for cells outside the volume
// or in blocks that cannot emit), [n_act][64].
__global__ __launch_bounds__(256) void k_debug_cases(Geom g, const uint32_t *__restrict__ I_active,
                                                    const uint8_t *__restrict__ active,
                                                    const int32_t *__restrict__ I_slot, int identity,
                                                    const float *__restrict__ slots, float iso,
                                                    uint8_t *__restrict__ cases,
                                                    const Counters *ctr) {
    __shared__ float tiles[MC_WAVES][128];
    if (ctr->err) return;
    const uint64_t n_act = ctr->n_act;
    const int w = threadIdx.x >> 6;
    const uint64_t waves = (uint64_t)gridDim.x * MC_WAVES;
    for (uint64_t i = (uint64_t)blockIdx.x * MC_WAVES + w; i < n_act; i += waves) {
        const uint32_t b = I_active[i];
        int cs = -1;
        if (active[b] & 2u) {
            Halo h;
            halo_setup(g, b, I_slot, identity, h);
            if (!h.bad) {
                stage_tile(g, h, slots, tiles[w]);
                wave_lds_sync();
                cs = cell_case(g, h, tiles[w], iso);
                wave_lds_sync();
            }
        }
        cases[i * 64 + lane()] = (uint8_t)(cs < 0 ? 0 : cs);
    }
}

// Plain streaming copy (16 B per lane per iteration): a known-size reference
// for reading memory-traffic counters.
__global__ __launch_bounds__(256) void k_copy_calibration(uint4 *__restrict__ dst,
                                                         const uint4 *__restrict__ src, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// Ages of the first n slots advanced by k, saturating at 2^32 - 1.
__global__ void k_age_slots(uint32_t *S_age, uint64_t n, uint32_t k) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t a = S_age[i];
        S_age[i] = a > 0xFFFFFFFFu - k ? 0xFFFFFFFFu : a + k;
    }
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_iota_i32(int32_t *p, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = (int32_t)i;
}

unsigned grid_cap(uint64_t n_threads, unsigned cap) {
    uint64_t gsz = (n_threads + 255) / 256;
    if (gsz < 1) gsz = 1;
    return (unsigned)(gsz < cap ? gsz : cap);
}

}  // namespace

// Workgroups of a persistent kernel that are all resident at once (the
// static per-wave shares assume no second round), in whole XCD rounds.
template <typename K>
static unsigned resident_grid(K kernel, uint64_t max_blocks) {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 256;
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    uint64_t g = (uint64_t)per_cu * cus;
    uint64_t need = (max_blocks + MC_WAVES - 1) / MC_WAVES;
    if (need < g) g = need;
    g = g / 8 * 8;
    return (unsigned)(g < 8 ? 8 : g);
}
static unsigned mc_grid(uint64_t max_blocks) {
    uint64_t g = (max_blocks + MC_WAVES - 1) / MC_WAVES;
    g = g < MC_MAX_GRID ? g : MC_MAX_GRID;
    return (unsigned)((g + 7) / 8 * 8);   // whole XCD rounds
}

void launch_cull(const Geom &g, const DevState &d, const StatusLayout &sl, float iso, float prev_iso,
                 uint64_t n_slots_host, int identity_cache, uint32_t gen, hipStream_t s) {
    static unsigned rgrid = 0;
    if (!rgrid) rgrid = resident_grid(k_cull, ~0ull >> 4);
    const uint64_t nt = cull_tiles(g);
    k_call_reset<<<grid_cap(sl.total, 64), 256, 0, s>>>(d.ctr, n_slots_host, d.status, sl.total);
    k_cull_scan<<<(unsigned)((nt + 255) / 256), 256, 0, s>>>(d.tile_ranges, nt, iso, prev_iso, d.cull_list,
                                                             d.ctr);
    k_cull<<<(unsigned)std::min<uint64_t>(nt, rgrid), 256, 0, s>>>(
        g, d.ranges, iso, d.cull_list, nt, d.I_slot, identity_cache, d.active, d.ctr, d.round_gen, gen);
}

uint64_t cull_tiles(const Geom &g) {
    return (uint64_t)((g.nbx + CULL_TX - 1) / CULL_TX) * ((g.nby + CULL_TY - 1) / CULL_TY) *
           ((g.nbz + CULL_TZ - 1) / CULL_TZ);
}

void launch_tile_ranges(const Geom &g, const float2 *ranges, float2 *tile_ranges, hipStream_t s) {
    k_tile_ranges<<<(unsigned)cull_tiles(g), 256, 0, s>>>(g, ranges, tile_ranges);
}

void launch_compact_blocks(const Geom &g, const DevState &d, const StatusLayout &sl, uint32_t gen,
                           hipStream_t s) {
    static unsigned cgrid = 0, wgrid = 0;
    if (!cgrid) cgrid = resident_grid(k_round_counts, ~0ull >> 4);
    if (!wgrid) wgrid = resident_grid(k_compact_blocks, ~0ull >> 4);
    const uint64_t n_rounds = block_rounds(g.nb);
    k_round_list<<<(unsigned)((n_rounds + 4095) / 4096), 256, 0, s>>>(d.round_gen, n_rounds, gen, d.round_list,
                                                                      d.ctr, d.status + sl.rnd);
    k_round_counts<<<(unsigned)std::min<uint64_t>(n_rounds, cgrid), 256, 0, s>>>(
        g, d.active, d.round_list, d.round_cnt, d.part_cand, d.ctr);
    k_round_scan<<<1, 256, 0, s>>>(d.round_cnt, d.ctr);
    k_compact_blocks<<<(unsigned)std::min<uint64_t>(n_rounds, wgrid), 256, 0, s>>>(
        g, d.active, d.round_list, d.round_cnt, d.I_active, d.I_new, d.ctr);
}

void launch_slot_pass(const DevState &d, const StatusLayout &sl, uint64_t n_slots_host,
                      uint32_t age_cap, hipStream_t s) {
    if (n_slots_host == 0) return;
    unsigned tiles = (unsigned)((n_slots_host + SLOT_TILE - 1) / SLOT_TILE);
    k_slot_pass<<<tiles, 256, 0, s>>>(d.active, d.S_block, d.S_age, n_slots_host, age_cap,
                                      d.sort_key[0], d.sort_val[0], d.slot_or, d.slot_and, d.ctr,
                                      d.status + sl.slot);
}

void launch_plan_grow(const DevState &d, uint64_t max_slots, uint64_t grow_bound, hipStream_t s) {
    k_plan_grow<<<grid_cap(grow_bound, 2048), 256, 0, s>>>(d.ctr, max_slots, d.S_block, d.S_age,
                                                          d.sort_key[0], d.sort_val[0], d.slot_or,
                                                          d.slot_and);
}

void launch_radix(const DevState &d, const StatusLayout &sl, uint64_t max_elems, uint32_t age_cap,
                  hipStream_t s) {
    uint64_t tiles = (max_elems + RADIX_TILE - 1) / RADIX_TILE;
    unsigned grid = (unsigned)((tiles + 3) / 4 < 2048 ? (tiles + 3) / 4 : 2048);
    if (grid == 0) grid = 1;
    uint64_t scan_tiles = (256 * tiles + SCAN_TILE - 1) / SCAN_TILE;
    unsigned sgrid = (unsigned)(scan_tiles < 2048 ? scan_tiles : 2048);
    if (sgrid == 0) sgrid = 1;
    for (int p = 0; p < 4 && (p == 0 || (age_cap >> (8 * p)) != 0); p++) {
        k_radix_hist<<<grid, 256, 0, s>>>(d.ctr, p, d.sort_key[0], d.sort_key[1], d.radix_hist,
                                          d.status + sl.scan);
        k_radix_scan<<<sgrid, 256, 0, s>>>(d.ctr, p, d.radix_hist, d.status + sl.scan);
        k_radix_scatter<<<grid, 256, 0, s>>>(d.ctr, p, d.sort_key[0], d.sort_key[1], d.sort_val[0],
                                             d.sort_val[1], d.radix_hist);
    }
}


// Grid of the emission: as many workgroups as are resident at once (their
// waves sweep the chunks of the active list as one window), in whole XCD
// rounds.  Its wave count also sets the chunk size (mc_chunk_size).
static unsigned emit_grid(const Geom &g, int fmt) {
    static unsigned grid[3] = {0, 0, 0};
    if (!grid[0]) grid[0] = resident_grid(k_mc_emit<VFMT_F32>, ~0ull >> 4);
    if (!grid[1]) grid[1] = resident_grid(k_mc_emit<VFMT_EDGE8>, ~0ull >> 4);
    if (!grid[2]) grid[2] = resident_grid(k_mc_emit<VFMT_Q10>, ~0ull >> 4);
    return std::min<unsigned>(grid[fmt >= 0 && fmt < 3 ? fmt : 0], mc_grid(g.nb));
}

void launch_mc_count(const Geom &g, const DevState &d, const float *slots, const int32_t *I_slot,
                     int identity_cache, float iso, int fmt, hipStream_t s) {
    static unsigned mgrid = 0;
    if (!mgrid) mgrid = resident_grid(k_masks, ~0ull >> 4);
    k_masks<<<std::min<unsigned>(mgrid, mc_grid(g.nb / 16 + 1)), 256, 0, s>>>(
        d.I_active, I_slot, identity_cache, slots, iso, d.masks, d.mask_iso, d.ctr);
    // the count pass takes the emission's chunks on a grid of its own (all
    // of it resident)
    static unsigned cres = 0;
    if (!cres) cres = std::min<unsigned>(resident_grid(k_mc_count, ~0ull >> 4), MC_MAX_GRID);
    const unsigned egrid = emit_grid(g, fmt), cgrid = std::min<unsigned>(cres, mc_grid(g.nb));
    k_mc_count<<<cgrid, 256, 0, s>>>(g, d.I_active, d.active, I_slot, identity_cache, d.masks,
                                     d.blk_cnt, d.chunk_off, d.part_occw, egrid * MC_WAVES, d.ctr);
    k_chunk_scan<<<9, 1024, 0, s>>>(d.chunk_off, d.chunk_off + mc_chunk_slots(g.nb), d.part_occw,
                                    cgrid * MC_WAVES, egrid * MC_WAVES, d.part_cand, d.ctr);
}

void launch_mc_emit(const Geom &g, const DevState &d, const float *slots, const int32_t *I_slot,
                    int identity_cache, float iso, void *out, uint64_t cap_verts, int fmt,
                    hipStream_t s) {
    const unsigned n = emit_grid(g, fmt);
#define BCMC_EMIT(F)                                                                          \
    k_mc_emit<F><<<n, 256, 0, s>>>(g, d.I_active, I_slot, identity_cache, slots, d.mc_table, iso, \
                                   d.blk_cnt, d.blk_off, out, cap_verts, d.chunk_off,              \
                                   d.chunk_off + mc_chunk_slots(g.nb), n * MC_WAVES, d.ctr)
    if (fmt == VFMT_EDGE8) BCMC_EMIT(VFMT_EDGE8);
    else if (fmt == VFMT_Q10) BCMC_EMIT(VFMT_Q10);
    else BCMC_EMIT(VFMT_F32);
#undef BCMC_EMIT
}

// 16-byte vertices -> Sec. 4.5's 8-byte records (q10_code | block << 32),
// two vertices per lane per iteration.
__global__ __launch_bounds__(256) void k_vertices_q10(const uint4 *__restrict__ in, uint64_t n,
                                                     uint64_t *__restrict__ out) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint4 v = in[i];
        const uint32_t q = q10_code(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z));
        __builtin_nontemporal_store((uint64_t)q | ((uint64_t)v.w << 32), out + i);
    }
}

void launch_vertices_q10(const void *in, uint64_t n, void *out, hipStream_t s) {
    if (n) k_vertices_q10<<<grid_cap(n, 8192), 256, 0, s>>>(reinterpret_cast<const uint4 *>(in), n,
                                                            reinterpret_cast<uint64_t *>(out));
}

void launch_debug_cases(const Geom &g, const DevState &d, const float *slots,
                        const int32_t *I_slot, int identity_cache, float iso, uint8_t *cases,
                        uint64_t max_act, hipStream_t s) {
    k_debug_cases<<<mc_grid(max_act), 256, 0, s>>>(g, d.I_active, d.active, I_slot, identity_cache,
                                                    slots, iso, cases, d.ctr);
}

// Backward of the vertex positions through t = (iso - a)/(b - a), topology
// fixed: the emission's pass over the last extract's soup (same chunks and
// offsets) in VFMT_GRAD mode, which for a vertex on an edge along axis e
// with g = dL/dv[e] adds g (t - 1)/(b - a) to dL/da, -g t/(b - a) to dL/db
// and g/(b - a) to dL/diso (float atomics into the field through per-block
// LDS sums; dL/diso by per-wave partial sums).  fmt: the extract's vertex
// format (its grid set the chunks).
void launch_backward(const Geom &g, const DevState &d, const float *slots, float iso,
                     const float *gV, uint64_t n_verts, float *dfield, float *diso, int fmt,
                     hipStream_t s) {
    static unsigned grid = 0;
    if (!grid) grid = resident_grid(k_mc_emit<VFMT_GRAD>, ~0ull >> 4);
    const unsigned n = std::min<unsigned>(grid, mc_grid(g.nb));
    k_mc_emit<VFMT_GRAD><<<n, 256, 0, s>>>(g, d.I_active, nullptr, 1, slots, d.mc_table, iso, d.blk_cnt,
                                          d.blk_off, nullptr, n_verts, d.chunk_off,
                                          d.chunk_off + mc_chunk_slots(g.nb),
                                          emit_grid(g, fmt) * MC_WAVES, d.ctr, gV, dfield, d.part_giso);
    k_sum_f32<<<1, 1024, 0, s>>>(d.part_giso, n * MC_WAVES, diso);
}

void launch_copy_calibration(void *dst, const void *src, uint64_t n16, hipStream_t s) {
    if (n16) k_copy_calibration<<<grid_cap(n16, 16384), 256, 0, s>>>(
        reinterpret_cast<uint4 *>(dst), reinterpret_cast<const uint4 *>(src), n16);
}

void launch_age_slots(uint32_t *S_age, uint64_t n, uint32_t k, hipStream_t s) {
    if (n && k) k_age_slots<<<grid_cap(n, 8192), 256, 0, s>>>(S_age, n, k);
}

void launch_fill_u32(uint32_t *p, uint32_t v, uint64_t n, hipStream_t s) {
    if (n) k_fill_u32<<<grid_cap(n, 8192), 256, 0, s>>>(p, v, n);
}

void launch_iota_i32(int32_t *p, uint64_t n, hipStream_t s) {
    if (n) k_iota_i32<<<grid_cap(n, 8192), 256, 0, s>>>(p, n);
}

}  // namespace bcmc
