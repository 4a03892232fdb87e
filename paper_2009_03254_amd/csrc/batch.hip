// Batched extraction: many volumes of uneven size, several isovalues each,
// in ONE persistent cooperative launch (phases separated by grid barriers),
// replayable from a hipGraph.
//
// Each job j = (volume v_j, isovalue iso_j) produces exactly the triangle soup
// a single-volume extract of v_j at iso_j produces (same kernels' arithmetic,
// same canonical order); the jobs' soups are concatenated in job order.
//
// The batch keeps its own decoded-block store: a block needed by any job of
// its volume (the union over the volume's isovalues, Sec. 4.1 rule per job)
// is decoded once, into the next free slot, and stays resident (an
// unbounded cache: nothing is evicted, so later runs decode only blocks no
// earlier run needed).
//
// Phases (grid = all workgroups resident; every thread reaches every barrier):
//   0  reset the run's counters
//   1  per global block: needed by some job of its volume and not yet decoded;
//      per (job, block): the block may emit for that job (2x2x2 hull rule);
//      per-workgroup counts of both
//   2  workgroup 0 scans the per-workgroup counts
//   3  scatter: list of new blocks; list L of (job, block) pairs in job-major,
//      block-ascending order (= the concatenated canonical orders)
//   4  decode the new blocks into slots n_slots + rank
//   5  count pass over L (Sec. 4.4)
//   6  exclusive scan of the counts (reduce, scan partials, distribute)
//   7  emission over L (Sec. 4.5), per-job output offsets
#include <stdint.h>

#include "batch.h"
#include "common.h"
#include "mc_device.h"
#include "zfp_device.h"

namespace bcmc {
namespace {

constexpr int BT = 256;  // threads per workgroup

// Which volume / job an index belongs to: largest i with base[i] <= x.
__device__ __forceinline__ uint32_t find_base(const uint64_t *base, uint32_t n, uint64_t x) {
    uint32_t lo = 0, hi = n;  // base[lo] <= x < base[hi]
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (base[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Index -> segment lookup for increasing indices: caches [lo, hi) of the
// current segment and searches again only when the index leaves it.
struct SegCursor {
    uint32_t seg;
    uint64_t lo, hi;
    __device__ __forceinline__ void reset() { lo = 1; hi = 0; seg = 0; }
    __device__ __forceinline__ uint32_t find(const uint64_t *base, uint32_t n, uint64_t end, uint64_t x) {
        if (x < lo || x >= hi) {
            seg = find_base(base, n, x);
            lo = base[seg];
            hi = seg + 1 < n ? base[seg + 1] : end;
        }
        return seg;
    }
};

// Grid-wide barrier for a grid whose workgroups are all resident: arrival
// counter + generation word (device-scope atomics).  The spin is bounded: on
// timeout it raises ERR_TIMEOUT and returns false, and the caller leaves the
// kernel, so a barrier can never hang the device.
constexpr unsigned BARRIER_SPIN_LIMIT = 1u << 22;

__device__ bool grid_barrier(unsigned int *bar, unsigned int *err) {
    __shared__ int ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        ok = 1;
        __threadfence();
        const unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned arrived = atomicAdd(&bar[0], 1u) + 1u;
        if (arrived == gridDim.x) {
            __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __threadfence();
            atomicAdd(&bar[1], 1u);
        } else {
            unsigned spins = 0;
            while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ERR_TIMEOUT ||
                    ++spins > BARRIER_SPIN_LIMIT) {
                    atomicOr(err, ERR_TIMEOUT);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __threadfence();
    }
    __syncthreads();
    return ok;
}

// Workgroup-wide exclusive scan of one u32 per thread; returns the total.
__device__ uint32_t wg_excl_scan(uint32_t v, uint32_t &excl, uint32_t *sh_w) {
    const int w = threadIdx.x >> 6;
    uint32_t incl = wave_incl_scan(v);
    if (lane() == 63) sh_w[w] = incl;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < BT / 64; i++) {
        if (i < w) off += sh_w[i];
        tot += sh_w[i];
    }
    __syncthreads();
    excl = off + incl - v;
    return tot;
}

// Contiguous share of [0, n) for workgroup g of G.
__device__ __forceinline__ void wg_range(uint64_t n, uint64_t &lo, uint64_t &hi) {
    const uint64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    lo = (uint64_t)blockIdx.x * chunk;
    hi = lo + chunk < n ? lo + chunk : n;
    if (lo > n) lo = n;
}

// Exclusive scan, by workgroup 0, of partial[0..G) in place; returns total.
__device__ uint64_t scan_partials(uint64_t *partial, uint32_t *sh_w) {
    const uint32_t G = gridDim.x;
    uint64_t carry = 0;
    for (uint32_t base = 0; base < G; base += BT) {
        uint32_t i = base + threadIdx.x;
        uint32_t v = i < G ? (uint32_t)partial[i] : 0u;
        uint32_t excl;
        uint32_t tot = wg_excl_scan(v, excl, sh_w);
        if (i < G) partial[i] = carry + excl;
        carry += tot;
    }
    return carry;
}

struct BatchShared {
    EmitShared emit;
    uint32_t w[BT / 64];
    uint32_t ntri[256];
};

// Workgroup 0 stamps the device's constant-rate clock at phase boundaries.
__device__ __forceinline__ void stamp(const BatchParams &p, int k) {
    if (blockIdx.x == 0 && threadIdx.x == 0) p.phase_ts[k] = wall_clock64();
}

template <bool F64, int SB>
__global__ __launch_bounds__(BT) void k_batch(BatchParams p) {
    __shared__ BatchShared sh;
    const int l = lane(), w = threadIdx.x >> 6;
    const uint64_t gtid = blockIdx.x * (uint64_t)BT + threadIdx.x;
    stamp(p, 0);
    for (int i = threadIdx.x; i < 256; i += BT) sh.ntri[i] = 3u * (uint32_t)(p.mc_table[i] >> 60);
    // phase 0
    if (gtid == 0) {
        p.ctr->n_new = 0;
        p.ctr->n_list = 0;
        p.ctr->total_verts = 0;
        p.ctr->err = 0;
    }
    const uint64_t n_slots0 = p.ctr->n_slots;
    if (!grid_barrier(p.bar, &p.ctr->err)) return;
    stamp(p, 1);

    // ---- phase 1: flags and per-workgroup counts ----------------------------
    {
        uint64_t lo, hi;
        wg_range(p.n_gblocks, lo, hi);
        uint32_t cnt = 0;
        SegCursor cur;
        cur.reset();
        for (uint64_t gb = lo + threadIdx.x; gb < hi; gb += BT) {
            const uint32_t v = cur.find(p.vol_gbase, p.n_vols, p.n_gblocks, gb);
            const BatchVol &vol = p.vols[v];
            const Geom &g = vol.g;
            const uint32_t b = (uint32_t)(gb - vol.gbase);
            uint8_t need = 0;
            if (p.I_slot[gb] < 0) {
                const uint32_t bx = b % g.nbx, r = b / g.nbx, by = r % g.nby, bz = r / g.nby;
                const float2 own = vol.ranges[b];
                float LO = own.x, HI = own.y;
                for (int dz = -1; dz <= 1; dz++) {
                    int z = (int)bz + dz;
                    if (z < 0 || z >= (int)g.nbz) continue;
                    for (int dy = -1; dy <= 1; dy++) {
                        int y = (int)by + dy;
                        if (y < 0 || y >= (int)g.nby) continue;
                        const float2 *row = vol.ranges + ((uint64_t)z * g.nby + y) * g.nbx;
                        for (int dx = -1; dx <= 1; dx++) {
                            int x = (int)bx + dx;
                            if (x < 0 || x >= (int)g.nbx) continue;
                            float2 q = row[x];
                            LO = fminf(LO, q.x);
                            HI = fmaxf(HI, q.y);
                        }
                    }
                }
                for (uint32_t j = vol.job_lo; j < vol.job_hi; j++) {
                    const float iso = p.job_iso[p.vol_jobs[j]];
                    if ((own.x < iso && iso <= HI) || (LO < iso && iso <= own.y)) need = 1;
                }
            }
            p.need[gb] = need;
            cnt += need;
        }
        uint32_t excl;
        uint32_t tot = wg_excl_scan(cnt, excl, sh.w);
        if (threadIdx.x == 0) p.part_new[blockIdx.x] = tot;

        wg_range(p.n_jblocks, lo, hi);
        cnt = 0;
        cur.reset();
        for (uint64_t e = lo + threadIdx.x; e < hi; e += BT) {
            const uint32_t j = cur.find(p.job_jbase, p.n_jobs, p.n_jblocks, e);
            const BatchVol &vol = p.vols[p.job_vol[j]];
            const Geom &g = vol.g;
            const uint32_t b = (uint32_t)(e - p.job_jbase[j]);
            const uint32_t bx = b % g.nbx, r = b / g.nbx, by = r % g.nby, bz = r / g.nby;
            const float iso = p.job_iso[j];
            float PLO = INFINITY, PHI = -INFINITY;
#pragma unroll
            for (int m = 0; m < 8; m++) {
                uint32_t x = bx + (m & 1), y = by + ((m >> 1) & 1), z = bz + (m >> 2);
                if (x < g.nbx && y < g.nby && z < g.nbz) {
                    float2 q = vol.ranges[x + g.nbx * (y + g.nby * z)];
                    PLO = fminf(PLO, q.x);
                    PHI = fmaxf(PHI, q.y);
                }
            }
            uint8_t em = (PLO < iso && iso <= PHI) ? 1 : 0;
            p.emit_flag[e] = em;
            cnt += em;
        }
        tot = wg_excl_scan(cnt, excl, sh.w);
        if (threadIdx.x == 0) p.part_list[blockIdx.x] = tot;
    }
    if (!grid_barrier(p.bar, &p.ctr->err)) return;
    stamp(p, 2);

    // ---- phase 2 -------------------------------------------------------------
    if (blockIdx.x == 0) {
        uint64_t tn = scan_partials(p.part_new, sh.w);
        uint64_t tl = scan_partials(p.part_list, sh.w);
        if (threadIdx.x == 0) {
            p.ctr->n_new = tn;
            p.ctr->n_list = tl;
        }
    }
    if (!grid_barrier(p.bar, &p.ctr->err)) return;
    stamp(p, 3);

    // ---- phase 3: ordered scatter of both lists --------------------------------
    {
        uint64_t lo, hi;
        wg_range(p.n_gblocks, lo, hi);
        const uint64_t per = (hi - lo + BT - 1) / BT;    // contiguous items per thread
        uint64_t a = lo + threadIdx.x * per, z = a + per < hi ? a + per : hi;
        uint32_t c = 0;
        for (uint64_t i = a; i < z; i++) c += p.need[i];
        uint32_t excl;
        wg_excl_scan(c, excl, sh.w);
        uint64_t o = p.part_new[blockIdx.x] + excl;
        for (uint64_t i = a; i < z; i++)
            if (p.need[i]) p.new_list[o++] = (uint32_t)i;

        wg_range(p.n_jblocks, lo, hi);
        const uint64_t per2 = (hi - lo + BT - 1) / BT;
        a = lo + threadIdx.x * per2;
        z = a + per2 < hi ? a + per2 : hi;
        c = 0;
        for (uint64_t i = a; i < z; i++) c += p.emit_flag[i];
        wg_excl_scan(c, excl, sh.w);
        o = p.part_list[blockIdx.x] + excl;
        SegCursor cur;
        cur.reset();
        for (uint64_t i = a; i < z; i++)
            if (p.emit_flag[i]) {
                p.list[o] = (uint32_t)i;
                p.list_job[o++] = cur.find(p.job_jbase, p.n_jobs, p.n_jblocks, i);
            }
    }
    if (!grid_barrier(p.bar, &p.ctr->err)) return;
    stamp(p, 4);

    // ---- phase 4: decode the new blocks; first list entry of every job --------
    const uint64_t n_new = p.ctr->n_new;
    const uint64_t n_list = p.ctr->n_list;
    for (uint64_t j = gtid; j < p.n_jobs; j += (uint64_t)gridDim.x * BT) {
        uint64_t lo = 0, hi = n_list;   // first entry with list[i] >= job_jbase[j]
        const uint64_t key = p.job_jbase[j];
        while (lo < hi) {
            uint64_t mid = (lo + hi) >> 1;
            if (p.list[mid] < key) lo = mid + 1;
            else hi = mid;
        }
        p.job_first[j] = lo;
    }
    for (uint64_t i = gtid; i < n_new; i += (uint64_t)gridDim.x * BT) {
        const uint32_t gb = p.new_list[i];
        const BatchVol &vol = p.vols[find_base(p.vol_gbase, p.n_vols, gb)];
        const uint64_t slot = n_slots0 + i;
        if (slot >= p.max_slots) {
            atomicOr(&p.ctr->err, ERR_INTERNAL);
            continue;
        }
        float v[64];
        decode_block<F64>(vol.stream + (uint64_t)(gb - vol.gbase) * vol.rate, (int)vol.rate, v);
        float4 *dst = reinterpret_cast<float4 *>(p.slots + slot * 64);
#pragma unroll
        for (int q = 0; q < 16; q++) dst[q] = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
        p.I_slot[gb] = (int32_t)slot;
    }
    if (!grid_barrier(p.bar, &p.ctr->err)) return;
    stamp(p, 5);

    // ---- phase 5: count pass over L -------------------------------------------------
    const LaneGeom q = lane_geom();
    {
        uint64_t lo, hi;
        xcd_wave_range(n_list, lo, hi);
        for (uint64_t i0 = lo; i0 < hi; i0 += 64) {
            const uint64_t idx = i0 + l;
            const bool valid = idx < hi;
            const uint32_t e = valid ? p.list[idx] : 0u;
            const uint32_t j = valid ? p.list_job[idx] : 0u;
            const BatchVol &vol = p.vols[p.job_vol[j]];
            const uint32_t b = (uint32_t)(e - p.job_jbase[j]);
            uint32_t so[8], lbx, lby, lbz;
            octet(vol.g, b, p.I_slot + vol.gbase, 0, so, lbx, lby, lbz);
            uint64_t todo = __ballot(valid);
            uint32_t mycnt = 0;
            while (todo) {
                int jl[SB], nsb = 0;
#pragma unroll
                for (int k = 0; k < SB; k++) {
                    jl[k] = k ? jl[0] : 0;
                    if (todo) {
                        jl[k] = (int)__builtin_ctzll(todo);
                        todo &= todo - 1;
                        nsb++;
                    }
                }
                stage_batch_n<SB>(q, p.slots, so, jl, sh.emit.tiles[w]);
                wave_lds_sync();
#pragma unroll
                for (int k = 0; k < SB; k++) {
                    if (k < nsb) {
                        const uint32_t vj = bcast(p.job_vol[j], jl[k]);
                        const Geom &g = p.vols[vj].g;
                        const uint32_t bx = bcast(lbx, jl[k]), by = bcast(lby, jl[k]), bz = bcast(lbz, jl[k]);
                        const float iso = __uint_as_float(bcast(__float_as_uint(p.job_iso[j]), jl[k]));
                        const int cs = tile_case(g, bx, by, bz, sh.emit.tiles[w][k], iso);
                        const uint32_t total = wave_sum(cs < 0 ? 0u : sh.ntri[cs]);
                        if (l == jl[k]) mycnt = total;
                    }
                }
                wave_lds_sync();
            }
            if (valid) p.cnt[idx] = mycnt;
        }
    }
    if (!grid_barrier(p.bar, &p.ctr->err)) return;
    stamp(p, 6);

    // ---- phase 6: scan of the counts ------------------------------------------------
    {
        uint64_t lo, hi;
        wg_range(n_list, lo, hi);
        const uint64_t per = (hi - lo + BT - 1) / BT;
        const uint64_t a = lo + threadIdx.x * per, z = a + per < hi ? a + per : hi;
        uint32_t c = 0;
        for (uint64_t i = a; i < z; i++) c += p.cnt[i];
        uint32_t excl;
        uint32_t tot = wg_excl_scan(c, excl, sh.w);
        if (threadIdx.x == 0) p.part_list[blockIdx.x] = tot;
        if (!grid_barrier(p.bar, &p.ctr->err)) return;
        if (blockIdx.x == 0) {
            uint64_t t = scan_partials(p.part_list, sh.w);
            if (threadIdx.x == 0) p.ctr->total_verts = t;
        }
        if (!grid_barrier(p.bar, &p.ctr->err)) return;
        uint64_t o = p.part_list[blockIdx.x] + excl;
        for (uint64_t i = a; i < z; i++) {
            p.off[i] = o;
            o += p.cnt[i];
        }
    }
    if (!grid_barrier(p.bar, &p.ctr->err)) return;
    stamp(p, 7);

    // ---- phase 7: emission and job offsets -----------------------------------------
    const uint64_t total = p.ctr->total_verts;
    for (uint64_t j = gtid; j <= p.n_jobs; j += (uint64_t)gridDim.x * BT) {
        uint64_t f = j < p.n_jobs ? p.job_first[j] : n_list;
        p.job_off[j] = f < n_list ? p.off[f] : total;
    }
    {
        uint64_t lo, hi;
        xcd_wave_range(n_list, lo, hi);
        for (uint64_t i0 = lo; i0 < hi; i0 += 64) {
            const uint64_t idx = i0 + l;
            const bool valid = idx < hi;
            const uint32_t cnt = valid ? p.cnt[idx] : 0u;
            const uint32_t e = cnt ? p.list[idx] : 0u;
            const uint32_t j = cnt ? p.list_job[idx] : 0u;
            const BatchVol &vol = p.vols[p.job_vol[j]];
            const uint32_t b = (uint32_t)(e - p.job_jbase[j]);
            const uint64_t boff = cnt ? p.off[idx] : 0ull;
            uint32_t so[8], lbx, lby, lbz;
            octet(vol.g, b, p.I_slot + vol.gbase, 0, so, lbx, lby, lbz);
            uint64_t todo = __ballot(cnt != 0);
            while (todo) {
                int jl[SB], nsb = 0;
#pragma unroll
                for (int k = 0; k < SB; k++) {
                    jl[k] = k ? jl[0] : 0;
                    if (todo) {
                        jl[k] = (int)__builtin_ctzll(todo);
                        todo &= todo - 1;
                        nsb++;
                    }
                }
                stage_batch_n<SB>(q, p.slots, so, jl, sh.emit.tiles[w]);
                wave_lds_sync();
                for (int k = 0; k < nsb; k++) {
                    const uint32_t vj = bcast(p.job_vol[j], jl[k]);
                    const Geom &g = p.vols[vj].g;
                    const uint32_t bj = bcast(b, jl[k]);
                    const float iso = __uint_as_float(bcast(__float_as_uint(p.job_iso[j]), jl[k]));
                    const uint64_t base = ((uint64_t)bcast((uint32_t)(boff >> 32), jl[k]) << 32) |
                                          bcast((uint32_t)boff, jl[k]);
                    emit_block<false>(g, bj, bcast(lbx, jl[k]), bcast(lby, jl[k]), bcast(lbz, jl[k]),
                               sh.emit.tiles[w][k], iso, p.mc_table, sh.emit, w, base,
                               p.out, p.cap);
                }
            }
        }
    }
    if (!grid_barrier(p.bar, &p.ctr->err)) return;
    stamp(p, 8);
    if (gtid == 0) p.ctr->n_slots = n_slots0 + n_new;
}

}  // namespace

int batch_max_grid(int is_f64, int sb, int *per_cu) {
    int n = 0;
    hipError_t e;
    if (is_f64)
        e = sb == 4 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch<true, 4>, BT, 0)
                    : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch<true, 8>, BT, 0);
    else
        e = sb == 4 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch<false, 4>, BT, 0)
                    : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch<false, 8>, BT, 0);
    if (e != hipSuccess) return -1;
    *per_cu = n;
    return 0;
}

hipError_t launch_batch(const BatchParams &p, int is_f64, int sb, unsigned grid, hipStream_t s,
                        int cooperative) {
    void *args[] = {const_cast<BatchParams *>(&p)};
    const void *fn;
    if (is_f64) fn = sb == 4 ? (const void *)k_batch<true, 4> : (const void *)k_batch<true, 8>;
    else fn = sb == 4 ? (const void *)k_batch<false, 4> : (const void *)k_batch<false, 8>;
    if (cooperative) return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(BT), args, 0, s);
    return hipLaunchKernel(fn, dim3(grid), dim3(BT), args, 0, s);
}

}  // namespace bcmc
