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

namespace bcmc {
namespace {

// ---- coefficient order ----------------------------------------------------
struct Order64 {
    unsigned char idx[64];
};
// Coefficients by total sequency level, each level in ascending block index.
constexpr Order64 sequency_order() {
    Order64 o{};
    int r = 0;
    for (int level = 0; level <= 9; level++)
        for (int i = 0; i < 64; i++)
            if ((i & 3) + ((i >> 2) & 3) + (i >> 4) == level) o.idx[r++] = (unsigned char)i;
    return o;
}
static constexpr Order64 kOrder = sequency_order();

template <bool F64>
struct Prec;
template <>
struct Prec<false> {
    using Int = int32_t;
    using UInt = uint32_t;
    static constexpr int P = 32, EBITS = 8, BIAS = 127, EMIN = 30 - 126;
    static constexpr UInt NB = 0xAAAAAAAAu;
};
template <>
struct Prec<true> {
    using Int = int64_t;
    using UInt = uint64_t;
    static constexpr int P = 64, EBITS = 11, BIAS = 1023, EMIN = 62 - 1022;
    static constexpr UInt NB = 0xAAAAAAAAAAAAAAAAull;
};

// ---- integer lifting (wrapping P-bit arithmetic) --------------------------
// Forward: the matrix (1/16)[[4,4,4,4],[5,1,-1,-5],[-4,4,4,-4],[-2,6,-6,2]]
// as five average/difference lifting steps.
template <typename Int>
__device__ __forceinline__ void fwd4(Int &a, Int &b, Int &c, Int &d) {
    using U = typename std::make_unsigned<Int>::type;
    a = (Int)((U)a + (U)d) >> 1; d = (Int)((U)d - (U)a);
    c = (Int)((U)c + (U)b) >> 1; b = (Int)((U)b - (U)c);
    a = (Int)((U)a + (U)c) >> 1; c = (Int)((U)c - (U)a);
    d = (Int)((U)d + (U)b) >> 1; b = (Int)((U)b - (U)d);
    d = (Int)((U)d + (U)(b >> 1)); b = (Int)((U)b - (U)(d >> 1));
}
// Inverse: the same steps undone in reverse order.
template <typename Int>
__device__ __forceinline__ void inv4(Int &a, Int &b, Int &c, Int &d) {
    using U = typename std::make_unsigned<Int>::type;
    b = (Int)((U)b + (U)(d >> 1)); d = (Int)((U)d - (U)(b >> 1));
    b = (Int)((U)b + (U)d); d = (Int)(((U)d << 1) - (U)b);
    c = (Int)((U)c + (U)a); a = (Int)(((U)a << 1) - (U)c);
    b = (Int)((U)b + (U)c); c = (Int)(((U)c << 1) - (U)b);
    d = (Int)((U)d + (U)a); a = (Int)(((U)a << 1) - (U)d);
}

template <typename Int>
__device__ __forceinline__ void fwd_xyz(Int *v) {
#pragma unroll
    for (int i = 0; i < 16; i++) fwd4(v[4 * i], v[4 * i + 1], v[4 * i + 2], v[4 * i + 3]);
#pragma unroll
    for (int z = 0; z < 4; z++)
#pragma unroll
        for (int x = 0; x < 4; x++)
            fwd4(v[x + 16 * z], v[x + 4 + 16 * z], v[x + 8 + 16 * z], v[x + 12 + 16 * z]);
#pragma unroll
    for (int i = 0; i < 16; i++) fwd4(v[i], v[i + 16], v[i + 32], v[i + 48]);
}

template <typename Int>
__device__ __forceinline__ void inv_zyx(Int *v) {
#pragma unroll
    for (int i = 0; i < 16; i++) inv4(v[i], v[i + 16], v[i + 32], v[i + 48]);
#pragma unroll
    for (int z = 0; z < 4; z++)
#pragma unroll
        for (int x = 0; x < 4; x++)
            inv4(v[x + 16 * z], v[x + 4 + 16 * z], v[x + 8 + 16 * z], v[x + 12 + 16 * z]);
#pragma unroll
    for (int i = 0; i < 16; i++) inv4(v[4 * i], v[4 * i + 1], v[4 * i + 2], v[4 * i + 3]);
}

// ---- bit reader over one block's words ------------------------------------
struct BitReader {
    const uint64_t *__restrict__ p;
    uint64_t cur;  // unread bits, LSB first; bits above cnt are zero
    int cnt;

    __device__ __forceinline__ void refill() {
        cur = __builtin_nontemporal_load(p);
        p++;
        cnt = 64;
    }
    __device__ __forceinline__ void skip(int n) {  // n <= cnt
        cur = (n >= 64) ? 0 : (cur >> n);
        cnt -= n;
    }
    __device__ __forceinline__ uint32_t bit() {
        if (cnt == 0) refill();
        uint32_t b = (uint32_t)(cur & 1u);
        cur >>= 1;
        cnt--;
        return b;
    }
    __device__ __forceinline__ uint64_t read(int n) {  // 0 <= n <= 64
        if (n <= cnt) {
            uint64_t v = (n >= 64) ? cur : (cur & ((1ull << n) - 1));
            skip(n);
            return v;
        }
        uint64_t w = __builtin_nontemporal_load(p);
        p++;
        int take = n - cnt;  // 1..64, cnt < 64
        uint64_t v = cur | (w << cnt);
        if (n < 64) v &= (1ull << n) - 1;
        cur = (take >= 64) ? 0 : (w >> take);
        cnt = 64 - take;
        return v;
    }
};

// Decode one block (words of 64*rate bits) into 64 floats in block order.
template <bool F64>
__device__ __forceinline__ void decode_block(const uint64_t *__restrict__ words, int rate,
                                             float *out) {
    using T = Prec<F64>;
    using UInt = typename T::UInt;
    using Int = typename T::Int;
    BitReader br{words, 0, 0};
    if (!br.bit()) {
#pragma unroll
        for (int i = 0; i < 64; i++) out[i] = 0.0f;
        return;
    }
    int emax = (int)br.read(T::EBITS) - T::BIAS;
    int budget = 64 * rate - 1 - T::EBITS;
    UInt c[64];
#pragma unroll
    for (int i = 0; i < 64; i++) c[i] = 0;
    int n = 0;
    for (int k = T::P - 1; k >= 0 && budget > 0; k--) {
        int m = n < budget ? n : budget;
        uint64_t x = br.read(m);
        budget -= m;
        // group tests: is there a 1 at or beyond n in this plane?
        while (n < 64 && budget > 0) {
            budget--;
            if (!br.bit()) break;
            // find it: zeros until the 1, never past coefficient 63 (implied)
            for (;;) {
                int limit = 63 - n < budget ? 63 - n : budget;
                if (limit == 0) break;
                if (br.cnt == 0) br.refill();
                int z = br.cur ? (int)__builtin_ctzll(br.cur) : br.cnt;
                if (z >= limit) {
                    br.skip(limit);
                    n += limit;
                    budget -= limit;
                    break;
                }
                br.skip(z);
                n += z;
                budget -= z;
                if (br.cnt > 0) {  // the 1 is next: consume it
                    br.skip(1);
                    budget--;
                    break;
                }
            }
            x |= 1ull << n;
            n++;
        }
        if (x) {
            if (F64) {
#pragma unroll
                for (int i = 0; i < 64; i++) c[i] |= (UInt)((x >> i) & 1u) << k;
            } else {
                uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
#pragma unroll
                for (int i = 0; i < 32; i++) c[i] |= ((lo >> i) & 1u) << k;
#pragma unroll
                for (int i = 0; i < 32; i++) c[32 + i] |= ((hi >> i) & 1u) << k;
            }
        }
    }
    Int v[64];
#pragma unroll
    for (int r = 0; r < 64; r++) v[kOrder.idx[r]] = (Int)((c[r] ^ T::NB) - T::NB);
    inv_zyx(v);
    if (F64) {
        double s = ldexp(1.0, emax - 62);
#pragma unroll
        for (int i = 0; i < 64; i++) out[i] = (float)((double)v[i] * s);
    } else {
        float s = ldexpf(1.0f, emax - 30);
#pragma unroll
        for (int i = 0; i < 64; i++) out[i] = (float)(int32_t)v[i] * s;
    }
}

// ---- bit writer ------------------------------------------------------------
struct BitWriter {
    uint64_t *__restrict__ out;
    uint64_t acc;
    int na;
    __device__ __forceinline__ void put(uint64_t v, int n) {  // v < 2^n, n <= 64
        if (n == 0) return;
        acc |= (na >= 64) ? 0 : (v << na);
        if (na + n >= 64) {
            *out++ = acc;
            int used = 64 - na;
            acc = (used >= 64) ? 0 : (v >> used);
            na = na + n - 64;
        } else {
            na += n;
        }
    }
};

template <bool F64>
__device__ __forceinline__ bool encode_block(const double *x, int rate, uint64_t *out) {
    using T = Prec<F64>;
    using UInt = typename T::UInt;
    using Int = typename T::Int;
    const int words = rate;
    bool any = false, finite = true;
    int emax = 0;
#pragma unroll
    for (int i = 0; i < 64; i++) {
        if (!isfinite(x[i])) finite = false;
        if (x[i] != 0.0) {
            int e;
            frexp(x[i], &e);
            emax = any ? (e > emax ? e : emax) : e;
            any = true;
        }
    }
    BitWriter bw{out, 0, 0};
    if (!finite || !any) {
        for (int w = 0; w < words; w++) out[w] = 0;
        return finite;
    }
    if (emax < T::EMIN) emax = T::EMIN;
    bw.put(1, 1);
    bw.put((uint64_t)(emax + T::BIAS), T::EBITS);
    Int v[64];
#pragma unroll
    for (int i = 0; i < 64; i++) {
        if (F64) v[i] = (Int)ldexp(x[i], T::P - 2 - emax);
        else v[i] = (Int)ldexpf((float)x[i], T::P - 2 - emax);
    }
    fwd_xyz(v);
    UInt u[64];
#pragma unroll
    for (int r = 0; r < 64; r++) u[r] = ((UInt)v[kOrder.idx[r]] + T::NB) ^ T::NB;
    int budget = 64 * rate - 1 - T::EBITS;
    int n = 0;
    for (int k = T::P - 1; k >= 0 && budget > 0; k--) {
        uint64_t x64 = 0;
#pragma unroll
        for (int i = 0; i < 64; i++) x64 |= (uint64_t)((u[i] >> k) & 1u) << i;
        int m = n < budget ? n : budget;
        bw.put(m >= 64 ? x64 : (x64 & ((1ull << m) - 1)), m);
        budget -= m;
        while (n < 64 && budget > 0) {
            uint64_t rest = x64 >> n;  // n < 64
            budget--;
            bw.put(rest ? 1 : 0, 1);
            if (!rest) break;
            int zeros = (int)__builtin_ctzll(rest);
            int limit = 63 - n < budget ? 63 - n : budget;
            if (zeros >= limit) {
                bw.put(0, limit);
                n += limit;
                budget -= limit;
            } else {
                bw.put(1ull << zeros, zeros + 1);
                budget -= zeros + 1;
                n += zeros;
            }
            n++;
        }
    }
    if (bw.na > 0) *bw.out++ = bw.acc;
    for (uint64_t *e = out + words; bw.out < e;) *bw.out++ = 0;
    return true;
}

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
template <bool F64>
__global__ __launch_bounds__(256) void k_decode_ranges(Geom g, const uint64_t *__restrict__ stream,
                                                      int rate, float2 *__restrict__ ranges,
                                                      float *__restrict__ blocks,
                                                      unsigned int *err) {
    for (uint64_t b = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; b < g.nb;
         b += (uint64_t)gridDim.x * blockDim.x) {
        float v[64];
        decode_block<F64>(stream + b * rate, rate, v);
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
            for (int i = 0; i < 16; i++) o[i] = make_float4(v[4 * i], v[4 * i + 1], v[4 * i + 2], v[4 * i + 3]);
        }
    }
}

__global__ __launch_bounds__(256) void k_ranges_from_blocks(Geom g, const float *__restrict__ blocks,
                                                           float2 *__restrict__ ranges,
                                                           unsigned int *err) {
    for (uint64_t b = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; b < g.nb;
         b += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t bx, by, bz;
        block_xyz(g, b, bx, by, bz);
        uint32_t vx = min(4u, g.nx - 4 * bx), vy = min(4u, g.ny - 4 * by), vz = min(4u, g.nz - 4 * bz);
        const float4 *src = reinterpret_cast<const float4 *>(blocks + b * 64);
        float lo = INFINITY, hi = -INFINITY;
        bool finite = true;
#pragma unroll
        for (int q = 0; q < 16; q++) {
            float4 f = src[q];
            float e[4] = {f.x, f.y, f.z, f.w};
#pragma unroll
            for (int j = 0; j < 4; j++) {
                int i = 4 * q + j;
                bool valid = (uint32_t)(i & 3) < vx && (uint32_t)((i >> 2) & 3) < vy && (uint32_t)(i >> 4) < vz;
                if (valid) {
                    lo = fminf(lo, e[j]);
                    hi = fmaxf(hi, e[j]);
                    finite = finite && isfinite(e[j]);
                }
            }
        }
        ranges[b] = make_float2(lo, hi);
        if (!finite) atomicOr(err, ERR_NONFINITE);
    }
}

// Alg. 1 AssignSlots fused with DecompressBlocks: new block I_new[i] takes the
// i-th slot of the age-sorted available list, evicting its previous owner,
// and is decoded straight into that slot.
template <bool F64>
__global__ __launch_bounds__(256) void k_assign_decode(Counters *ctr, const uint32_t *__restrict__ I_new,
                                                      const uint32_t *__restrict__ sorted0,
                                                      const uint32_t *__restrict__ sorted1,
                                                      int32_t *S_block, int32_t *I_slot,
                                                      uint32_t *S_age, const uint64_t *__restrict__ stream,
                                                      int rate, float *__restrict__ slots,
                                                      uint64_t n_blocks) {
    if (ctr->err) return;
    const uint64_t n_slots = ctr->n_slots;
    const uint64_t n_new = ctr->n_new;
    if (n_new == 0) return;
    // the radix passes ping-pong; the result is in buffer (#passes run) & 1
    const uint32_t *sorted = (__popc(ctr->pass_mask) & 1) ? sorted1 : sorted0;
    uint32_t evicted = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n_new;
         i += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t b = I_new[i];
        uint32_t s = sorted[i];
        if (b >= n_blocks || s >= n_slots) {  // never expected: report, do not touch memory
            atomicOr(&ctr->err, ERR_INTERNAL);
            continue;
        }
        int32_t old = S_block[s];
        if (old >= 0) {
            I_slot[old] = -1;
            evicted++;
        }
        S_block[s] = (int32_t)b;
        I_slot[b] = (int32_t)s;
        S_age[s] = 0;
        float v[64];
        decode_block<F64>(stream + (uint64_t)b * rate, rate, v);
        float4 *o = reinterpret_cast<float4 *>(slots + (uint64_t)s * 64);
#pragma unroll
        for (int q = 0; q < 16; q++) o[q] = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
    }
    if (evicted) atomicAdd(&ctr->n_evicted, (unsigned long long)evicted);
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

unsigned grid_for(uint64_t n, unsigned cap) {
    uint64_t gsz = (n + 255) / 256;
    if (gsz < 1) gsz = 1;
    return (unsigned)(gsz < cap ? gsz : cap);
}

}  // namespace

void launch_decode_ranges(const Geom &g, const uint64_t *stream, int is_f64, uint32_t rate,
                          float2 *ranges, float *blocks_out, unsigned int *err, hipStream_t s) {
    unsigned grid = grid_for(g.nb, 8192);
    if (is_f64)
        k_decode_ranges<true><<<grid, 256, 0, s>>>(g, stream, (int)rate, ranges, blocks_out, err);
    else
        k_decode_ranges<false><<<grid, 256, 0, s>>>(g, stream, (int)rate, ranges, blocks_out, err);
}

void launch_ranges_from_blocks(const Geom &g, const float *blocks, float2 *ranges,
                               unsigned int *err, hipStream_t s) {
    k_ranges_from_blocks<<<grid_for(g.nb, 8192), 256, 0, s>>>(g, blocks, ranges, err);
}

void launch_assign_decode(const DevState &d, int is_f64, uint32_t rate, uint64_t max_new,
                          hipStream_t s) {
    unsigned grid = grid_for(max_new, 2048);
    if (is_f64)
        k_assign_decode<true><<<grid, 256, 0, s>>>(d.ctr, d.I_new, d.sort_val[0], d.sort_val[1],
                                                   d.S_block, d.I_slot, d.S_age, d.stream,
                                                   (int)rate, d.slots, max_new);
    else
        k_assign_decode<false><<<grid, 256, 0, s>>>(d.ctr, d.I_new, d.sort_val[0], d.sort_val[1],
                                                    d.S_block, d.I_slot, d.S_age, d.stream,
                                                    (int)rate, d.slots, max_new);
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
