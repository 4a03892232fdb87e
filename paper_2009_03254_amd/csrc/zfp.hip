// Fixed-rate ZFP codec for gfx950 (Sec. 3.3.4; on-demand block decode into
// cache slots, Sec. 4.2.1).  One lane owns one 4x4x4 block: the per-block
// bit-plane loop is serial, so 64 blocks per wave keep the SIMDs busy.
//
// Codec (Lindstrom, "Fixed-Rate Compressed Floating-Point Arrays", TVCG 2014,
// as realised by this project):
//   header   1 bit (0 = all-zero block) then emax+bias in 8 (f32) / 11 (f64)
//            bits; emax = largest frexp exponent, clamped so that
//            2^(emax-(P-2)) is a normal number;
//   values   i = trunc(x * 2^(P-2-emax)) as P-bit integers (P = 32 / 64);
//   lifting  separable 4-point decorrelating transform along x, y, z;
//   order    coefficients by ascending i+j+k, ties by ascending index;
//   negabinary, then embedded bit-plane coding with group tests, cut at
//            64*rate bits; bits are LSB-first in little-endian u64 words.
#include <stdint.h>

#include "common.h"
#include "zfp_device.h"

namespace bcmc {
namespace {
// ---- kernels ---------------------------------------------------------------

__device__ __forceinline__ void block_xyz(const Geom &g, uint64_t b, uint32_t &bx, uint32_t &by,
                                          uint32_t &bz) {
    bx = (uint32_t)(b % g.nbx);
    uint64_t r = b / g.nbx;
    by = (uint32_t)(r % g.nby);
    bz = (uint32_t)(r / g.nby);
}

// Decode every block once: value range over the valid samples (Sec. 4.1),
// non-finite detection, and optionally the decoded blocks themselves.
template <bool F64, bool STAGED>
__global__ __launch_bounds__(256) void k_decode_ranges(Geom g, const uint64_t *__restrict__ stream,
                                                      int rate, float2 *__restrict__ ranges,
                                                      float *__restrict__ blocks,
                                                      unsigned int *err) {
    extern __shared__ uint64_t stage_lds[];
    constexpr bool staged = STAGED;
    uint64_t *st = stage_lds + (threadIdx.x >> 6) * (STAGED ? stage_wave_words(rate, F64) : 0u);
    // whole waves iterate together (the staging is a wave-wide copy)
    for (uint64_t b0 = blockIdx.x * (uint64_t)blockDim.x + (threadIdx.x & ~63u); b0 < g.nb;
         b0 += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t b = b0 + __lane_id();
        const bool valid = b < g.nb;
        float v[64];
        if (staged) {
            stage_words(stream, rate, b, valid, st);
            if (valid) decode_block_staged<F64>(st, rate, v);
        } else if (valid) {
            decode_block<F64>(stream + b * rate, rate, v);
        }
        if (staged) __builtin_amdgcn_wave_barrier();   // st is rewritten by the next round
        if (!valid) continue;
        uint32_t bx, by, bz;
        block_xyz(g, b, bx, by, bz);
        uint32_t vx = min(4u, g.nx - 4 * bx), vy = min(4u, g.ny - 4 * by), vz = min(4u, g.nz - 4 * bz);
        float lo = INFINITY, hi = -INFINITY;
        bool finite = true;
#pragma unroll
        for (int i = 0; i < 64; i++) {
            bool valid = (uint32_t)(i & 3) < vx && (uint32_t)((i >> 2) & 3) < vy && (uint32_t)(i >> 4) < vz;
            if (valid) {
                lo = fminf(lo, v[i]);
                hi = fmaxf(hi, v[i]);
                finite = finite && isfinite(v[i]);
            }
        }
        ranges[b] = make_float2(lo, hi);
        if (!finite) atomicOr(err, ERR_NONFINITE);
        if (blocks) {
            float4 *o = reinterpret_cast<float4 *>(blocks + b * 64);
#pragma unroll
            for (int q = 0; q < 16; q++) o[q] = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
        }
    }
}

__global__ __launch_bounds__(256) void k_ranges_from_blocks(Geom g, const float *__restrict__ blocks,
                                                           float2 *__restrict__ ranges,
                                                           unsigned int *err) {
    // a wave takes 64 consecutive blocks at a time, lane l the l-th (its
    // valid extent); the blocks' 16 KB are read 1 KB per load (in step q,
    // lanes 16 m .. 16 m + 15 hold the 16 float4 of block 4 q + m) and
    // reduced over each row of 16 lanes; the rows' results meet in LDS
    __shared__ float2 s_r[4][64];
    const int l = (int)__lane_id(), w = threadIdx.x >> 6;
    const uint64_t waves = (uint64_t)gridDim.x * 4;
    bool finite = true;
    for (uint64_t b0 = (blockIdx.x * 4ull + w) * 64; b0 < g.nb; b0 += waves * 64) {
        uint32_t ext = 0x040404u;   // the lane's block: valid samples per axis, as bytes
        if (b0 + l < g.nb) {
            uint32_t bx, by, bz;
            block_xyz(g, b0 + l, bx, by, bz);
            ext = min(4u, g.nx - 4 * bx) | min(4u, g.ny - 4 * by) << 8 | min(4u, g.nz - 4 * bz) << 16;
        }
        const int part = l & 15;   // float4 part: samples 4 part .. 4 part + 3 (y = part & 3, z = part >> 2)
#pragma unroll 4
        for (int q = 0; q < 16; q++) {
            const int m = l >> 4;
            const uint64_t blk = b0 + 4 * q + m;
            const uint32_t e = (uint32_t)__shfl((int)ext, 4 * q + m, 64);
            float lo = INFINITY, hi = -INFINITY;
            if (blk < g.nb) {
                const float4 f = reinterpret_cast<const float4 *>(blocks + blk * 64)[part];
                const float v[4] = {f.x, f.y, f.z, f.w};
                const bool rowok = (uint32_t)(part & 3) < ((e >> 8) & 0xFFu) && (uint32_t)(part >> 2) < (e >> 16);
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    if (rowok && (uint32_t)j < (e & 0xFFu)) {
                        lo = fminf(lo, v[j]);
                        hi = fmaxf(hi, v[j]);
                        finite = finite && isfinite(v[j]);
                    }
                }
            }
#pragma unroll
            for (int d = 1; d < 16; d <<= 1) {
                lo = fminf(lo, __shfl_xor(lo, d, 64));
                hi = fmaxf(hi, __shfl_xor(hi, d, 64));
            }
            if (part == 0) s_r[w][4 * q + m] = make_float2(lo, hi);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (b0 + l < g.nb) ranges[b0 + l] = s_r[w][l];
        // s_r is rewritten next step
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (__ballot(!finite) && l == 0) atomicOr(err, ERR_NONFINITE);
}

// Set bits of m below the calling lane.
__device__ __forceinline__ uint32_t mbcnt_lo_hi(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Store a decoded block into its slot, with its sign mask for this call's
// isovalue (so the mask pass need not read the freshly decoded slot back).
__device__ __forceinline__ void store_slot(const float *v, uint64_t s, float iso, float *__restrict__ slots,
                                           uint64_t *__restrict__ masks, uint32_t *__restrict__ mask_iso) {
    float4 *o = reinterpret_cast<float4 *>(slots + s * 64);
    uint32_t mw[2] = {0u, 0u};
#pragma unroll
    for (int q = 0; q < 16; q++) {
        const float4 f = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
        o[q] = f;
        mw[q >> 3] |= ((f.x < iso ? 1u : 0u) | (f.y < iso ? 2u : 0u) | (f.z < iso ? 4u : 0u) |
                       (f.w < iso ? 8u : 0u)) << (4 * (q & 7));
    }
    masks[s] = (uint64_t)mw[1] << 32 | mw[0];
    mask_iso[s] = __float_as_uint(iso);
}

// Alg. 1 AssignSlots fused with DecompressBlocks: new block I_new[i] takes the
// i-th slot of the age-sorted available list, evicting its previous owner,
// and is decoded straight into that slot.
// LOW (double precision, staged, low rates): the decode is
// decode_block_staged_low, which holds the kernel to the registers of the
// low-rate decoder (4 waves per SIMD; 5 spills registers and is slower); the
// blocks it hands back (their indices into I_new) are listed in `retry` for
// k_decode_retry.
template <bool F64, bool STAGED, bool LOW = false>
__global__ __launch_bounds__(256, LOW ? 4 : (F64 ? 1 : 4)) void k_assign_decode(Counters *ctr, const uint32_t *__restrict__ I_new,
                                                      const uint32_t *__restrict__ sorted0,
                                                      const uint32_t *__restrict__ sorted1,
                                                      int32_t *S_block, int32_t *I_slot,
                                                      uint32_t *S_age, const uint64_t *__restrict__ stream,
                                                      int rate, float *__restrict__ slots,
                                                      uint64_t n_blocks, float iso,
                                                      uint64_t *__restrict__ masks,
                                                      uint32_t *__restrict__ mask_iso,
                                                      uint32_t *__restrict__ retry = nullptr) {
    if (ctr->err) return;
    const uint64_t n_slots = ctr->n_slots;
    const uint64_t n_new = ctr->n_new;
    if (n_new == 0) return;
    // the radix passes ping-pong; the result is in buffer (#passes run) & 1
    const uint32_t *sorted = (__popc(ctr->pass_mask) & 1) ? sorted1 : sorted0;
    extern __shared__ uint64_t stage_lds[];
    constexpr bool staged = STAGED;
    uint64_t *st = stage_lds + (threadIdx.x >> 6) * (STAGED ? stage_wave_words(rate, F64) : 0u);
    uint32_t evicted = 0;
    // whole waves iterate together (the staging is a wave-wide copy)
    for (uint64_t i0 = blockIdx.x * (uint64_t)blockDim.x + (threadIdx.x & ~63u); i0 < n_new;
         i0 += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t i = i0 + __lane_id();
        bool valid = i < n_new;
        const uint32_t b = valid ? I_new[i] : 0u;
        const uint32_t s = valid ? sorted[i] : 0u;
        if (valid && (b >= n_blocks || s >= n_slots)) {  // never expected: report, do not touch memory
            atomicOr(&ctr->err, ERR_INTERNAL);
            valid = false;
        }
        if (valid) {
            int32_t old = S_block[s];
            if (old >= 0) {
                I_slot[old] = -1;
                evicted++;
            }
            S_block[s] = (int32_t)b;
            I_slot[b] = (int32_t)s;
            S_age[s] = 0;
        }
        float v[64];
        bool done = true;
        if (staged) {
            stage_words(stream, rate, b, valid, st);
            if constexpr (LOW) {
                if (valid) done = decode_block_staged_low(st, rate, v);
            } else {
                if (valid) decode_block_staged<F64>(st, rate, v);
            }
            __builtin_amdgcn_wave_barrier();   // st is rewritten by the next round
        } else if (valid) {
            decode_block<F64>(stream + (uint64_t)b * rate, rate, v);
        }
        if (valid && done) store_slot(v, s, iso, slots, masks, mask_iso);
        if constexpr (LOW) {   // one atomic per wave for the blocks handed back
            const uint64_t back = __ballot(valid && !done);
            if (back) {
                const int first = (int)__builtin_ctzll(back);
                uint32_t base = 0;
                if (__lane_id() == (unsigned)first)
                    base = atomicAdd(&ctr->tile_ctr[TC_RETRY], (uint32_t)__popcll(back));
                base = __shfl(base, first, 64);
                if (valid && !done) retry[base + mbcnt_lo_hi(back)] = (uint32_t)i;
            }
        }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) evicted += __shfl_xor(evicted, d, 64);   // one atomic per wave
    if (__lane_id() == 0 && evicted) atomicAdd(&ctr->n_evicted, (unsigned long long)evicted);
}

template <bool F64>
__global__ __launch_bounds__(256) void k_encode(Geom g, const void *__restrict__ field, int rate,
                                               uint64_t *__restrict__ stream, unsigned int *err) {
    for (uint64_t b = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; b < g.nb;
         b += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t bx, by, bz;
        block_xyz(g, b, bx, by, bz);
        double x[64];
#pragma unroll
        for (int i = 0; i < 64; i++) {
            // partial blocks replicate the last valid sample along each axis
            uint32_t gx = min(4 * bx + (i & 3), g.nx - 1);
            uint32_t gy = min(4 * by + ((i >> 2) & 3), g.ny - 1);
            uint32_t gz = min(4 * bz + (i >> 4), g.nz - 1);
            uint64_t idx = gx + (uint64_t)g.nx * (gy + (uint64_t)g.ny * gz);
            x[i] = F64 ? ((const double *)field)[idx] : (double)((const float *)field)[idx];
        }
        if (!encode_block<F64>(x, rate, stream + b * rate)) atomicOr(err, ERR_NONFINITE);
    }
}

// The blocks the low-rate decoder handed back, decoded with the general
// decoder from global memory into the slots the assignment gave them.
__global__ __launch_bounds__(256) void k_decode_retry(const Counters *ctr, const uint32_t *__restrict__ I_new,
                                                     const uint32_t *__restrict__ sorted0,
                                                     const uint32_t *__restrict__ sorted1,
                                                     const uint64_t *__restrict__ stream, int rate,
                                                     float *__restrict__ slots, float iso,
                                                     uint64_t *__restrict__ masks,
                                                     uint32_t *__restrict__ mask_iso,
                                                     const uint32_t *__restrict__ retry) {
    if (ctr->err) return;
    const uint32_t n = ctr->tile_ctr[TC_RETRY];
    const uint32_t *sorted = (__popc(ctr->pass_mask) & 1) ? sorted1 : sorted0;
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
        const uint32_t i = retry[j];
        const uint32_t b = I_new[i], s = sorted[i];
        float v[64];
        decode_block<true>(stream + (uint64_t)b * rate, rate, v);
        store_slot(v, s, iso, slots, masks, mask_iso);
    }
}

unsigned grid_for(uint64_t n, unsigned cap) {
    uint64_t gsz = (n + 255) / 256;
    if (gsz < 1) gsz = 1;
    return (unsigned)(gsz < cap ? gsz : cap);
}

}  // namespace

// Instantiates a decode kernel for (type, staged) and launches it with the
// staging LDS the rate needs.
#define BCMC_DECODE_LAUNCH(KERNEL, grid, rate, s, ...)                                      \
    do {                                                                                    \
        const unsigned lds_ = stage_lds_bytes((int)(rate), is_f64 != 0);                                 \
        if (is_f64 && lds_) KERNEL<true, true><<<grid, 256, lds_, s>>>(__VA_ARGS__);         \
        else if (is_f64) KERNEL<true, false><<<grid, 256, 0, s>>>(__VA_ARGS__);              \
        else if (lds_) KERNEL<false, true><<<grid, 256, lds_, s>>>(__VA_ARGS__);             \
        else KERNEL<false, false><<<grid, 256, 0, s>>>(__VA_ARGS__);                         \
    } while (0)

void launch_decode_ranges(const Geom &g, const uint64_t *stream, int is_f64, uint32_t rate,
                          float2 *ranges, float *blocks_out, unsigned int *err, hipStream_t s) {
    unsigned grid = grid_for(g.nb, 8192);
    BCMC_DECODE_LAUNCH(k_decode_ranges, grid, rate, s, g, stream, (int)rate, ranges, blocks_out, err);
}

void launch_ranges_from_blocks(const Geom &g, const float *blocks, float2 *ranges,
                               unsigned int *err, hipStream_t s) {
    k_ranges_from_blocks<<<grid_for(g.nb, 8192), 256, 0, s>>>(g, blocks, ranges, err);
}

void launch_assign_decode(const DevState &d, int is_f64, uint32_t rate, uint64_t max_new, float iso,
                          hipStream_t s) {
    unsigned grid = grid_for(max_new, 2048);
    const unsigned lds = stage_lds_bytes((int)rate, is_f64 != 0);
    if (is_f64 && lds && rate <= LOW_RATE_MAX && d.retry) {
        k_assign_decode<true, true, true><<<grid, 256, lds, s>>>(
            d.ctr, d.I_new, d.sort_val[0], d.sort_val[1], d.S_block, d.I_slot, d.S_age, d.stream,
            (int)rate, d.slots, max_new, iso, d.masks, d.mask_iso, d.retry);
        k_decode_retry<<<64, 256, 0, s>>>(d.ctr, d.I_new, d.sort_val[0], d.sort_val[1], d.stream,
                                          (int)rate, d.slots, iso, d.masks, d.mask_iso, d.retry);
        return;
    }
    BCMC_DECODE_LAUNCH(k_assign_decode, grid, rate, s, d.ctr, d.I_new, d.sort_val[0], d.sort_val[1],
                       d.S_block, d.I_slot, d.S_age, d.stream, (int)rate, d.slots, max_new, iso,
                       d.masks, d.mask_iso);
}

void launch_encode(const Geom &g, const void *field, int is_f64, uint32_t rate, uint64_t *stream,
                   unsigned int *err, hipStream_t s) {
    unsigned grid = grid_for(g.nb, 8192);
    if (is_f64)
        k_encode<true><<<grid, 256, 0, s>>>(g, field, (int)rate, stream, err);
    else
        k_encode<false><<<grid, 256, 0, s>>>(g, field, (int)rate, stream, err);
}

}  // namespace bcmc
