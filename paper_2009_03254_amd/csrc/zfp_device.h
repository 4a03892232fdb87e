// Device-side fixed-rate ZFP codec shared by the HIP sources (see zfp.hip
// for the description of the codec).  Internal linkage in every includer.
#pragma once

#include <stdint.h>

#include <type_traits>

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

}  // namespace
}  // namespace bcmc
