// Batched extraction: many volumes of uneven size, several isovalues each,
// in four launches (the first persistent, its phases separated by grid
// barriers), replayable from a hipGraph.
//
// Each job j = (volume v_j, isovalue iso_j) produces exactly the triangle soup
// a single-volume extract of v_j at iso_j produces (same arithmetic, same
// canonical order); the jobs' soups are concatenated in job order.
//
// The batch keeps its own decoded-block store: a block needed by any job of
// its volume (the union over the volume's isovalues, Sec. 4.1 rule per job)
// is decoded once, into the next free slot, and stays resident (an
// unbounded cache: nothing is evicted, so later runs decode only blocks no
// earlier run needed).
//
// Front kernel (persistent):
//   0  reset the run's counters
//   1  per global block: used by some job of its volume (new or resident)
//      and, per job of its volume, whether it may emit for that job (2x2x2
//      hull rule); per-workgroup counts of new blocks, per-wave counts of
//      the pairs that may emit
//   2  workgroup 0 scans the counts and reserves the new blocks' slots
//   3  scatter: list of new blocks; list L of (job, block) pairs in job-major,
//      block-ascending order (= the concatenated canonical orders)
// Decode kernel (grid-stride; its grid sized by the decoder's registers):
//   4  decode the new blocks into slots slot_base + rank; sign masks of every
//      used block for every job of its volume
// Count kernel (grid autotuned; every wave owns one contiguous share of L):
//   5  count pass over L from the sign masks (Sec. 4.4), per-wave totals
// Back kernel (same grid and shares as the count kernel, no barriers):
//   6  each workgroup sums the per-wave totals before its waves
//   7  emission over L (Sec. 4.5), offsets by a running wave scan of the
//      counts; per-job output offsets
// Every thread of a persistent grid reaches every barrier of its kernel.
#include <stdint.h>

#include "batch.h"
#include "common.h"
#include "mc_device.h"
#include "mc_ntri.h"
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

// Grid-wide barrier for a grid whose workgroups are all resident.  Arrivals
// are counted in two levels: workgroup g in group g % BAR_GROUPS, the last of
// a group in the top-level count, whose last arrival advances the generation.
// Waiters poll the generation with plain device-scope loads and acquire once
// when it moves.  The spin is bounded: on timeout it raises ERR_TIMEOUT and
// returns false, and the caller leaves the kernel, so a barrier can never
// hang the device.
constexpr unsigned BARRIER_SPIN_LIMIT = 1u << 21;

__device__ __forceinline__ unsigned ld_relaxed(const unsigned *a) {
    return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ bool grid_barrier(unsigned int *bar, unsigned int *err) {
    __shared__ int ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        ok = 1;
        const unsigned G = gridDim.x, k = blockIdx.x % BAR_GROUPS;
        const unsigned groups = G < (unsigned)BAR_GROUPS ? G : (unsigned)BAR_GROUPS;
        const unsigned members = G / BAR_GROUPS + (k < G % BAR_GROUPS ? 1u : 0u);
        const unsigned gen = ld_relaxed(&bar[BAR_GEN]);
        __threadfence();   // release this workgroup's writes; gen read before arriving
        bool last = false;
        if (atomicAdd(&bar[BAR_SUB + k * BAR_PAD], 1u) + 1u == members) {
            __hip_atomic_store(&bar[BAR_SUB + k * BAR_PAD], 0u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            __threadfence();
            if (atomicAdd(&bar[BAR_TOP], 1u) + 1u == groups) {
                __hip_atomic_store(&bar[BAR_TOP], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __threadfence();
                atomicAdd(&bar[BAR_GEN], 1u);
                last = true;
            }
        }
        if (!last) {
            unsigned spins = 0;
            while (ld_relaxed(&bar[BAR_GEN]) == gen) {
                if (ld_relaxed(err) & ERR_TIMEOUT || ++spins > BARRIER_SPIN_LIMIT) {
                    atomicOr(err, ERR_TIMEOUT);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(4);
            }
        }
        __threadfence();   // acquire the other workgroups' writes
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

// Exclusive scan, by workgroup 0, of partial[0..n) in place; returns total.
// Each thread takes a contiguous run (its loads all in flight together),
// the runs' sums are scanned across the workgroup.
__device__ uint64_t scan_partials(uint64_t *partial, uint32_t n, uint64_t *sh_w) {
    const int w = threadIdx.x >> 6;
    const uint32_t per = (n + BT - 1) / BT;
    const uint32_t a = threadIdx.x * per, z = a + per < n ? a + per : n;
    uint64_t s = 0;
#pragma unroll 8
    for (uint32_t i = a; i < z; i++) s += partial[i];
    const uint64_t incl = wave_incl_scan(s);
    if (lane() == 63) sh_w[w] = incl;
    __syncthreads();
    uint64_t off = incl - s, tot = 0;
#pragma unroll
    for (int k = 0; k < BT / 64; k++) {
        if (k < w) off += sh_w[k];
        tot += sh_w[k];
    }
    __syncthreads();
#pragma unroll 8
    for (uint32_t i = a; i < z; i++) {
        const uint64_t v = partial[i];
        partial[i] = off;
        off += v;
    }
    return tot;
}

// Sum of part[0..n) over the workgroup (its loads spread over the threads,
// 8 in flight each); with m > 0 also the sum of part[0..m) into *all.  Every
// thread of the workgroup calls it and gets the sums.
__device__ uint64_t sum_before(const uint64_t *part, uint32_t n, uint32_t m, uint64_t *sh_w, uint64_t *all) {
    const uint32_t lim = n > m ? n : m;
    uint64_t s = 0, t = 0;
    for (uint32_t i0 = threadIdx.x; i0 < lim; i0 += 8u * BT) {
        uint64_t v[8];
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const uint32_t i = i0 + (uint32_t)j * BT;
            v[j] = i < lim ? part[i] : 0ull;
        }
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const uint32_t i = i0 + (uint32_t)j * BT;
            if (i < n) s += v[j];
            if (i < m) t += v[j];
        }
    }
    s = wave_sum(s);
    t = wave_sum(t);
    const int w = threadIdx.x >> 6;
    if (lane() == 0) sh_w[w] = s;
    __syncthreads();
    uint64_t S = 0;
#pragma unroll
    for (int k = 0; k < BT / 64; k++) S += sh_w[k];
    __syncthreads();
    if (lane() == 0) sh_w[w] = t;
    __syncthreads();
    uint64_t T = 0;
#pragma unroll
    for (int k = 0; k < BT / 64; k++) T += sh_w[k];
    __syncthreads();
    *all = T;
    return S;
}

// Sign mask of a decoded block for one isovalue: bit i = (sample i < iso),
// the inside test of the per-cell classification (Sec. 4.4).
__device__ __forceinline__ uint64_t sign_mask(const float *v, float iso) {
    uint64_t m = 0;
#pragma unroll
    for (int i = 0; i < 64; i++) m |= (uint64_t)(v[i] < iso ? 1u : 0u) << i;
    return m;
}

// Jobs per volume whose masks the decoder builds in registers.
constexpr int MASK_JOBS = 4;

// The masks of global block gb (block b of volume vol) for every job of its
// volume.
__device__ __forceinline__ void store_masks(const BatchParams &p, const BatchVol &vol, uint32_t b,
                                            const float *v) {
    for (uint32_t k = vol.job_lo; k < vol.job_hi; k++) {
        const uint32_t j = p.vol_jobs[k];
        p.jmask[p.job_jbase[j] + b] = sign_mask(v, p.job_iso[j]);
    }
}

// Clock stamp k by workgroup 0 (after a grid barrier every workgroup has
// passed the previous phase).
__device__ __forceinline__ void stamp(const BatchParams &p, int k) {
    if (blockIdx.x == 0 && threadIdx.x == 0) p.phase_ts[k] = wall_clock64();
}

// Clock stamp k by the last workgroup to finish the kernel.
__device__ __forceinline__ void stamp_last(const BatchParams &p, int k) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&p.bar[BAR_DONE], 1u) + 1u == gridDim.x) {
            p.phase_ts[k] = wall_clock64();
            __hip_atomic_store(&p.bar[BAR_DONE], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Contiguous share [lo, hi) of n items for the calling wave: the workgroups
// of one XCD (blockIdx % 8) take one contiguous eighth of the range, so that
// blocks whose halos overlap are staged through the same L2; returns the
// share's rank in item order.
__device__ __forceinline__ uint32_t wave_share(uint64_t n, uint64_t &lo, uint64_t &hi) {
    const uint32_t G = gridDim.x, g = blockIdx.x;
    const uint32_t logical = (g % 8u) * (G / 8u) + g / 8u;
    const uint64_t waves = (uint64_t)G * (BT / 64);
    const uint32_t wv = logical * (BT / 64) + (threadIdx.x >> 6);
    const uint64_t chunk = (n + waves - 1) / waves;
    lo = wv * chunk;
    if (lo > n) lo = n;
    hi = lo + chunk < n ? lo + chunk : n;
    return wv;
}

// ---- front kernel: phases 0-3 ---------------------------------------------
__global__ __launch_bounds__(BT) void k_batch_front(BatchParams p) {
    __shared__ uint32_t sh_w[BT / 64];
    __shared__ uint64_t sh_w64[BT / 64];
    const uint64_t gtid = blockIdx.x * (uint64_t)BT + threadIdx.x;
    stamp(p, 0);
    // phase 0: reset the run's counters
    if (gtid == 0) {
        p.ctr->n_new = 0;
        p.ctr->n_list = 0;
        p.ctr->total_verts = 0;
        p.ctr->err = 0;
        p.ctr->grid_front = gridDim.x;
    }
    if (!grid_barrier(p.bar, &p.ctr->err)) return;
    stamp(p, 1);

    // ---- phase 1: flags ----------------------------------------------------------
    // Per global block, with its volume uniform over the workgroup's loop: the
    // ranges of its 3x3x3 neighbourhood (indices clamped into the volume: a
    // clamped neighbour is one already in the neighbourhood, so no load is
    // conditional), whether some job of the volume uses it (Sec. 4.1 rule) and,
    // per job, whether it may emit (2x2x2 hull of its octet).
    {
        uint64_t lo, hi;
        wg_range(p.n_gblocks, lo, hi);
        uint32_t cnt = 0;
        for (uint32_t v = lo < hi ? find_base(p.vol_gbase, p.n_vols, lo) : p.n_vols; v < p.n_vols; v++) {
            const BatchVol &vol = p.vols[v];
            if (vol.gbase >= hi) break;
            const Geom g = vol.g;
            const uint64_t s0 = vol.gbase > lo ? vol.gbase : lo;
            const uint64_t s1 = vol.gbase + g.nb < hi ? vol.gbase + g.nb : hi;
            for (uint64_t gb = s0 + threadIdx.x; gb < s1; gb += BT) {
                const uint32_t b = (uint32_t)(gb - vol.gbase);
                const uint32_t r = b / g.nbx, bx = b - r * g.nbx, by = r % g.nby, bz = r / g.nby;
                uint32_t xs[3], ys[3], zs[3];
                xs[0] = bx ? bx - 1 : 0; xs[1] = bx; xs[2] = bx + 1 < g.nbx ? bx + 1 : bx;
                ys[0] = by ? by - 1 : 0; ys[1] = by; ys[2] = by + 1 < g.nby ? by + 1 : by;
                zs[0] = bz ? bz - 1 : 0; zs[1] = bz; zs[2] = bz + 1 < g.nbz ? bz + 1 : bz;
                float2 q[27];
#pragma unroll
                for (int k = 0; k < 27; k++)
                    q[k] = vol.ranges[xs[k % 3] + g.nbx * ((uint64_t)ys[(k / 3) % 3] + (uint64_t)g.nby * zs[k / 9])];
                float LO = q[0].x, HI = q[0].y, PLO = q[13].x, PHI = q[13].y;
#pragma unroll
                for (int k = 1; k < 27; k++) {
                    LO = fminf(LO, q[k].x);
                    HI = fmaxf(HI, q[k].y);
                }
#pragma unroll
                for (int k = 14; k < 27; k++)
                    if (k % 3 != 0 && (k / 3) % 3 != 0) {   // offsets in {0, 1}^3
                        PLO = fminf(PLO, q[k].x);
                        PHI = fmaxf(PHI, q[k].y);
                    }
                const float2 own = q[13];
                bool used = false;
                for (uint32_t k = vol.job_lo; k < vol.job_hi; k++) {
                    const uint32_t j = p.vol_jobs[k];
                    const float iso = p.job_iso[j];
                    if ((own.x < iso && iso <= HI) || (LO < iso && iso <= own.y)) used = true;
                    p.emit_flag[p.job_jbase[j] + b] = (PLO < iso && iso <= PHI) ? 1 : 0;
                }
                const uint8_t need = used ? (p.I_slot[gb] < 0 ? 1 : 2) : 0;
                p.need[gb] = need;
                cnt += need == 1;
            }
        }
        uint32_t excl;
        const uint32_t tot = wg_excl_scan(cnt, excl, sh_w);
        if (threadIdx.x == 0) p.part_new[blockIdx.x] = tot;
    }
    if (!grid_barrier(p.bar, &p.ctr->err)) return;
    // Pairs that may emit, per wave share of the flags (4 flags per word; the
    // flag array is zero-padded to a multiple of 4).
    const uint64_t n_words = (p.n_jblocks + 3) / 4;
    const uint32_t *flag_words = reinterpret_cast<const uint32_t *>(p.emit_flag);
    {
        uint64_t lo, hi;
        const uint32_t wv = wave_share(n_words, lo, hi);
        uint64_t c = 0;
        for (uint64_t i = lo + lane(); i < hi; i += 64) c += __popc(flag_words[i]);
        c = wave_sum(c);
        if (lane() == 0) p.part_list[wv] = c;
    }
    if (!grid_barrier(p.bar, &p.ctr->err)) return;
    stamp(p, 2);

    // ---- phase 2: offsets of the workgroups' new blocks and the waves' pairs ----
    // scan_sched 0: workgroup 0 scans both count arrays in place, then a grid
    // barrier; 1: every workgroup sums the counts before its own (and
    // workgroup 0 all of them for the totals), no barrier.  The autotuner
    // picks one.
    uint64_t new_off, list_off;
    uint32_t wv_list;   // the wave's share of the flag words (index into part_list)
    {
        uint64_t slo, shi;
        wv_list = wave_share(n_words, slo, shi);
    }
    if (p.scan_sched == 0) {
        if (blockIdx.x == 0) {
            uint64_t tn = scan_partials(p.part_new, gridDim.x, sh_w64);
            uint64_t tl = scan_partials(p.part_list, gridDim.x * (BT / 64), sh_w64);
            if (threadIdx.x == 0) {
                const uint64_t n_slots0 = p.ctr->n_slots;
                p.ctr->slot_base = n_slots0;
                p.ctr->n_slots = n_slots0 + tn;
                p.ctr->n_new = tn;
                p.ctr->n_list = tl;
            }
        }
        if (!grid_barrier(p.bar, &p.ctr->err)) return;
        new_off = p.part_new[blockIdx.x];
        list_off = p.part_list[wv_list];
    } else {
        const uint32_t nw = gridDim.x * (BT / 64);
        const bool all = blockIdx.x == 0;
        new_off = sum_before(p.part_new, blockIdx.x, all ? gridDim.x : 0u, sh_w64, &list_off);
        const uint64_t tn = list_off;
        // the waves before this workgroup's first wave, then its own earlier waves
        const uint32_t wv0 = wv_list - (threadIdx.x >> 6);
        uint64_t tl;
        list_off = sum_before(p.part_list, wv0, all ? nw : 0u, sh_w64, &tl);
        for (uint32_t k = wv0; k < wv_list; k++) list_off += p.part_list[k];
        if (all && threadIdx.x == 0) {
            const uint64_t n_slots0 = p.ctr->n_slots;
            p.ctr->slot_base = n_slots0;
            p.ctr->n_slots = n_slots0 + tn;
            p.ctr->n_new = tn;
            p.ctr->n_list = tl;
        }
    }
    stamp(p, 3);

    // ---- phase 3: ordered scatter of both lists --------------------------------
    {
        uint64_t lo, hi;
        wg_range(p.n_gblocks, lo, hi);
        const uint64_t per = (hi - lo + BT - 1) / BT;    // contiguous items per thread
        uint64_t a = lo + threadIdx.x * per, z = a + per < hi ? a + per : hi;
        uint32_t c = 0;
        for (uint64_t i = a; i < z; i++) c += p.need[i] == 1;
        uint32_t excl;
        wg_excl_scan(c, excl, sh_w);
        uint64_t o = new_off + excl;
        for (uint64_t i = a; i < z; i++)
            if (p.need[i] == 1) p.new_list[o++] = (uint32_t)i;

        // L: each wave walks its share of the flag words again, 64 words per
        // step, placing the pairs by a wave scan of the per-word counts.
        wave_share(n_words, lo, hi);
        uint64_t base = list_off;
        SegCursor cur;
        cur.reset();
        for (uint64_t i0 = lo; i0 < hi; i0 += 64) {
            const uint64_t i = i0 + lane();
            const uint32_t fw = i < hi ? flag_words[i] : 0u;
            const uint32_t cw = __popc(fw);
            const uint32_t incl = wave_incl_scan(cw);
            uint64_t o2 = base + incl - cw;
            base += __shfl(incl, 63, 64);
#pragma unroll
            for (int t = 0; t < 4; t++)
                if ((fw >> (8 * t)) & 0xFFu) {
                    const uint64_t e = 4 * i + t;
                    p.list[o2] = (uint32_t)e;
                    p.list_job[o2++] = cur.find(p.job_jbase, p.n_jobs, p.n_jblocks, e);
                }
        }
    }
    stamp_last(p, 4);
}

// ---- decode kernel: phase 4 ---------------------------------------------------
// STAGED: every volume has rate p.uniform_rate <= STAGE_MAX_RATE and each
// wave stages its blocks' words in LDS before decoding (whole waves iterate
// together: the staging is a wave-wide copy).
template <bool F64, bool STAGED>
__global__ __launch_bounds__(BT) void k_batch_decode(BatchParams p) {
    if (p.ctr->err) return;   // the front kernel failed: nothing to do
    const uint64_t gtid = blockIdx.x * (uint64_t)BT + threadIdx.x;
    if (gtid == 0) p.ctr->grid_decode = gridDim.x;
    const uint64_t gstride = (uint64_t)gridDim.x * BT;
    const uint64_t n_slots0 = p.ctr->slot_base;
    const uint64_t n_new = p.ctr->n_new;
    extern __shared__ uint64_t stage_lds[];
    const int urate = (int)p.uniform_rate;
    uint64_t *st = stage_lds + (threadIdx.x >> 6) * (STAGED ? stage_wave_words(urate, F64) : 0u);
    for (uint64_t i0 = gtid & ~63ull; i0 < n_new; i0 += gstride) {
        const uint64_t i = i0 + lane();
        bool valid = i < n_new;
        const uint32_t gb = valid ? p.new_list[i] : 0u;
        const BatchVol &vol = p.vols[find_base(p.vol_gbase, p.n_vols, gb)];
        const uint64_t slot = n_slots0 + i;
        if (valid && slot >= p.max_slots) {   // never expected: report, do not touch memory
            atomicOr(&p.ctr->err, ERR_INTERNAL);
            valid = false;
        }
        const uint32_t b = (uint32_t)(gb - vol.gbase);
        float v[64];
        if (STAGED) {
            stage_words_at(vol.stream + (uint64_t)b * urate, urate, valid, st);
            if (valid) decode_block_staged<F64>(st, urate, v);
            __builtin_amdgcn_wave_barrier();   // st is rewritten by the next round
        } else if (valid) {
            decode_block<F64>(vol.stream + (uint64_t)b * vol.rate, (int)vol.rate, v);
        }
        if (!valid) continue;
        // store the block, building the masks of the volume's first
        // MASK_JOBS jobs on the way
        const uint32_t nj = vol.job_hi - vol.job_lo;
        float iso[MASK_JOBS];
        uint32_t mw[MASK_JOBS][2];
#pragma unroll
        for (int t = 0; t < MASK_JOBS; t++) {
            iso[t] = (uint32_t)t < nj ? p.job_iso[p.vol_jobs[vol.job_lo + t]] : -INFINITY;
            mw[t][0] = mw[t][1] = 0u;
        }
        float4 *dst = reinterpret_cast<float4 *>(p.slots + slot * 64);
#pragma unroll
        for (int q = 0; q < 16; q++) {
            const float4 f = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
            dst[q] = f;
#pragma unroll
            for (int t = 0; t < MASK_JOBS; t++)
                mw[t][q >> 3] |= ((f.x < iso[t] ? 1u : 0u) | (f.y < iso[t] ? 2u : 0u) |
                                  (f.z < iso[t] ? 4u : 0u) | (f.w < iso[t] ? 8u : 0u)) << (4 * (q & 7));
        }
        p.I_slot[gb] = (int32_t)slot;
#pragma unroll
        for (int t = 0; t < MASK_JOBS; t++)
            if ((uint32_t)t < nj)
                p.jmask[p.job_jbase[p.vol_jobs[vol.job_lo + t]] + b] = (uint64_t)mw[t][1] << 32 | mw[t][0];
    }
    if (p.max_vol_jobs > MASK_JOBS) {
        // the remaining jobs' masks; lane i reads back the block it stored above
        for (uint64_t i = gtid; i < n_new; i += gstride) {
            const uint32_t gb = p.new_list[i];
            const BatchVol &vol = p.vols[find_base(p.vol_gbase, p.n_vols, gb)];
            const uint64_t slot = n_slots0 + i;
            if (vol.job_hi - vol.job_lo <= MASK_JOBS || slot >= p.max_slots) continue;
            const float4 *src = reinterpret_cast<const float4 *>(p.slots + slot * 64);
            float w[64];
#pragma unroll
            for (int q = 0; q < 16; q++) {
                const float4 t4 = src[q];
                w[4 * q] = t4.x;
                w[4 * q + 1] = t4.y;
                w[4 * q + 2] = t4.z;
                w[4 * q + 3] = t4.w;
            }
            const uint32_t b = (uint32_t)(gb - vol.gbase);
            for (uint32_t k = vol.job_lo + MASK_JOBS; k < vol.job_hi; k++) {
                const uint32_t j = p.vol_jobs[k];
                p.jmask[p.job_jbase[j] + b] = sign_mask(w, p.job_iso[j]);
            }
        }
    }
    {
        SegCursor cur;
        cur.reset();
        for (uint64_t gb = gtid; gb < p.n_gblocks; gb += gstride) {
            if (p.need[gb] != 2) continue;
            const BatchVol &vol = p.vols[cur.find(p.vol_gbase, p.n_vols, p.n_gblocks, gb)];
            const float4 *src = reinterpret_cast<const float4 *>(p.slots) + (uint64_t)p.I_slot[gb] * 16;
            float v[64];
#pragma unroll
            for (int q = 0; q < 16; q++) {
                const float4 t = src[q];
                v[4 * q] = t.x;
                v[4 * q + 1] = t.y;
                v[4 * q + 2] = t.z;
                v[4 * q + 3] = t.w;
            }
            store_masks(p, vol, (uint32_t)(gb - vol.gbase), v);
        }
    }
    stamp_last(p, 5);
}

// ---- count kernel: phase 5 -----------------------------------------------------
// One lane per (job, block) pair of L, each wave over its share of L (the
// partition the emission uses: same grid): the cases of the block's 64 cells
// from the sign masks of its octet, the triangle count per case by the
// bit-sliced table circuit (Sec. 4.4); per-wave totals.
__global__ __launch_bounds__(BT) void k_batch_count(BatchParams p) {
    const int l = lane();
    if (p.ctr->err) return;   // an earlier kernel failed: nothing to do
    const uint64_t n_list = p.ctr->n_list;
    uint64_t lo, hi;
    const uint32_t wv = wave_share(n_list, lo, hi);
    uint64_t tot = 0;
    for (uint64_t i0 = lo; i0 < hi; i0 += 64) {
        const uint64_t idx = i0 + l;
        uint32_t c = 0;
        if (idx < hi) {
            const uint32_t j = p.list_job[idx];
            const uint64_t jb = p.job_jbase[j];
            const BatchVol &vol = p.vols[p.job_vol[j]];
            const uint32_t b = (uint32_t)(p.list[idx] - jb);
            uint32_t so[8], bx, by, bz;
            octet(vol.g, b, nullptr, 1, so, bx, by, bz);
            uint64_t M[8], cm[8];
#pragma unroll
            for (int m = 0; m < 8; m++) M[m] = p.jmask[jb + so[m]];
            corner_masks(M, cm);
            uint64_t n0, n1, n2;
            mc_ntri_bits(cm, n0, n1, n2);
            const uint64_t V = valid_cells(vol.g, bx, by, bz);
            c = 3u * ((uint32_t)__popcll(n0 & V) + 2u * (uint32_t)__popcll(n1 & V) +
                      4u * (uint32_t)__popcll(n2 & V));
            p.cnt[idx] = c;
        }
        tot += wave_sum(c);
    }
    if (l == 0) p.part_wave[wv] = tot;
    stamp_last(p, 6);
}

// ---- back kernel: phases 6-7 ----------------------------------------------------
struct BackShared {
    EmitShared emit;
    uint64_t tab[256];   // the triangle table (per-lane lookups at LDS latency)
    uint64_t w64[2][BT / 64];
};

template <int SB>
__global__ __launch_bounds__(BT) void k_batch_back(BatchParams p) {
    __shared__ BackShared sh;
    const int l = lane(), w = threadIdx.x >> 6;
    if (p.ctr->err) return;   // an earlier kernel failed: nothing to do
    const uint64_t n_list = p.ctr->n_list;
    uint64_t lo, hi;
    const uint32_t wv = wave_share(n_list, lo, hi);

    // ---- phase 6: each workgroup sums the per-wave totals before its first
    // wave and all of them (no grid barrier: the counts are a kernel earlier)
    for (int i = threadIdx.x; i < 256; i += BT) sh.tab[i] = p.mc_table[i];   // published by the barrier below
    if (threadIdx.x < 16) sh.emit.edge[threadIdx.x] = edge_entry((int)threadIdx.x);
    const uint32_t W = gridDim.x * (BT / 64), wv0 = wv - (uint32_t)w;
    uint64_t before = 0, all = 0;
    for (uint32_t i0 = threadIdx.x; i0 < W; i0 += 8u * BT) {   // 8 loads in flight at a time
        uint64_t v[8];
#pragma unroll
        for (int j = 0; j < 8; j++) v[j] = i0 + (uint32_t)j * BT < W ? p.part_wave[i0 + (uint32_t)j * BT] : 0ull;
#pragma unroll
        for (int j = 0; j < 8; j++) {
            all += v[j];
            if (i0 + (uint32_t)j * BT < wv0) before += v[j];
        }
    }
    before = wave_sum(before);
    all = wave_sum(all);
    if (l == 0) {
        sh.w64[0][w] = before;
        sh.w64[1][w] = all;
    }
    __syncthreads();
    uint64_t base = 0, total = 0;
#pragma unroll
    for (int k = 0; k < BT / 64; k++) {
        base += sh.w64[0][k];
        total += sh.w64[1][k];
    }
    for (uint32_t k = 0; k < (uint32_t)w; k++) base += p.part_wave[wv0 + k];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        p.ctr->total_verts = total;
        p.ctr->grid_back = gridDim.x;
    }
    stamp(p, 7);

    // ---- phase 7: emission (Sec. 4.5) and the jobs' output offsets --------------
    if (n_list == 0 && blockIdx.x == 0)
        for (uint32_t j = threadIdx.x; j <= p.n_jobs; j += BT) p.job_off[j] = 0;
    const LaneGeom q = lane_geom();
    for (uint64_t i0 = lo; i0 < hi; i0 += 64) {
        const uint64_t idx = i0 + l;
        const bool valid = idx < hi;
        const uint32_t c = valid ? p.cnt[idx] : 0u;
        const uint32_t incl = wave_incl_scan(c);
        const uint64_t off = base + incl - c;
        base += __shfl(incl, 63, 64);
        uint32_t j = 0;
        if (valid) {
            j = p.list_job[idx];
            // first entry of its job: it starts the soups of the jobs since the
            // previous entry's job (jobs with no entry have empty soups)
            const uint32_t jp = idx ? p.list_job[idx - 1] : 0u;
            if (idx == 0 || jp != j)
                for (uint32_t k = idx ? jp + 1 : 0u; k <= j; k++) p.job_off[k] = off;
            if (idx + 1 == n_list)
                for (uint32_t k = j + 1; k <= p.n_jobs; k++) p.job_off[k] = total;
        }
        const BatchVol &vol = p.vols[p.job_vol[j]];
        const float liso = p.job_iso[j];
        const uint32_t b = c ? (uint32_t)(p.list[idx] - p.job_jbase[j]) : 0u;
        uint32_t so[8], lbx, lby, lbz;
        octet(vol.g, b, p.I_slot + vol.gbase, 0, so, lbx, lby, lbz);
        uint64_t todo = __ballot(c != 0);
        while (todo) {
            const uint64_t left = todo;
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
            // the triangle list area is empty between batches (emit_batch flushes)
            static_assert(8 * SB <= EMIT_TRIS, "slot table fits the triangle list");
            stage_batch_tab<SB>(q, p.slots, so, left & ~todo, nsb, sh.emit.tri[w], sh.emit.tiles[w]);
            wave_lds_sync();
            // consecutive entries of L with triangles: adjacent vertex ranges
            const uint64_t ob = ((uint64_t)bcast((uint32_t)(off >> 32), jl[0]) << 32) |
                                bcast((uint32_t)off, jl[0]);
            auto info = [&](int k, Geom &gk, uint32_t &bk, uint32_t &bx, uint32_t &by, uint32_t &bz,
                            float &isok) {
                gk.nx = bcast(vol.g.nx, jl[k]);
                gk.ny = bcast(vol.g.ny, jl[k]);
                gk.nz = bcast(vol.g.nz, jl[k]);
                bk = bcast(b, jl[k]);
                bx = bcast(lbx, jl[k]);
                by = bcast(lby, jl[k]);
                bz = bcast(lbz, jl[k]);
                isok = __uint_as_float(bcast(__float_as_uint(liso), jl[k]));
            };
            emit_batch<VFMT_F32>(nsb, info, sh.emit.tiles[w], sh.tab, sh.emit, w, ob, p.out, p.cap);
        }
    }
    stamp_last(p, 8);
}

const void *decode_kernel(int is_f64, int staged) {
    if (is_f64)
        return staged ? (const void *)k_batch_decode<true, true> : (const void *)k_batch_decode<true, false>;
    return staged ? (const void *)k_batch_decode<false, true> : (const void *)k_batch_decode<false, false>;
}

unsigned decode_lds(const BatchParams &p, int is_f64) {
    return p.uniform_rate ? stage_lds_bytes((int)p.uniform_rate, is_f64 != 0) : 0u;
}

}  // namespace

int batch_front_per_cu(int *per_cu) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_front, BT, 0) != hipSuccess) return -1;
    *per_cu = n;
    return 0;
}


int batch_decode_per_cu(const BatchParams &p, int is_f64, int *per_cu) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, decode_kernel(is_f64, p.uniform_rate != 0), BT,
                                                     decode_lds(p, is_f64)) != hipSuccess)
        return -1;
    *per_cu = n;
    return 0;
}

int batch_back_per_cu(int sb, int *per_cu) {
    int n = 0;
    hipError_t e = sb == 4 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_back<4>, BT, 0)
                           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_back<8>, BT, 0);
    if (e != hipSuccess) return -1;
    *per_cu = n;
    return 0;
}

hipError_t launch_batch(const BatchParams &p, int is_f64, int sb, const unsigned grids[3],
                        hipStream_t s, int cooperative) {
    void *args[] = {const_cast<BatchParams *>(&p)};
    const void *decode = decode_kernel(is_f64, p.uniform_rate != 0);
    const void *back = sb == 4 ? (const void *)k_batch_back<4> : (const void *)k_batch_back<8>;
    hipError_t e = cooperative
                       ? hipLaunchCooperativeKernel((const void *)k_batch_front, dim3(grids[0]), dim3(BT),
                                                    args, 0, s)
                       : hipLaunchKernel((const void *)k_batch_front, dim3(grids[0]), dim3(BT), args, 0, s);
    if (e == hipSuccess) e = hipLaunchKernel(decode, dim3(grids[1]), dim3(BT), args, decode_lds(p, is_f64), s);
    // count and back share one grid: they partition L the same way
    if (e == hipSuccess) e = hipLaunchKernel((const void *)k_batch_count, dim3(grids[2]), dim3(BT), args, 0, s);
    if (e == hipSuccess) e = hipLaunchKernel(back, dim3(grids[2]), dim3(BT), args, 0, s);
    return e;
}

}  // namespace bcmc
