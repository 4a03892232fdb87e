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
// Inverse: the same steps undone in reverse order.  Each of the last four
// steps, x += y then y = 2 y - x, is the butterfly (x, y) -> (x + y, y - x)
// (2 y - (x + y) = y - x, also modulo 2^P): two operations instead of three.
template <typename Int>
__host__ __device__ __forceinline__ void inv4(Int &a, Int &b, Int &c, Int &d) {
    using U = typename std::make_unsigned<Int>::type;
    b = (Int)((U)b + (U)(d >> 1)); d = (Int)((U)d - (U)(b >> 1));
    U x;
    x = (U)b; b = (Int)(x + (U)d); d = (Int)((U)d - x);
    x = (U)c; c = (Int)(x + (U)a); a = (Int)((U)a - x);
    x = (U)b; b = (Int)(x + (U)c); c = (Int)((U)c - x);
    x = (U)d; d = (Int)(x + (U)a); a = (Int)((U)a - x);
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
__host__ __device__ __forceinline__ void inv_zyx(Int *v) {
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

// Lowest plane at which a double-precision block's stream may end for the
// 32-bit transform of its coefficients' high words (staged_f64_top_planes).
// The coefficients are then multiples of 2^K, K >= WRAP32_KMIN.  Each inverse
// lifting pass lowers the power of two dividing a value by at most 2 (a
// right shift of d, then one of the new b), so every operand of a right
// shift is a multiple of 2^(K - 5) >= 2^34 and every value a multiple of
// 2^(K - 6) >= 2^33.  With the low 32-bit words all zero, additions,
// subtractions and left shifts (wrapping modulo 2^64) act on the high words
// alone (wrapping modulo 2^32), and a right shift moves a zero out of the
// high word: the 64-bit transform is the 32-bit one on the high words, times
// 2^32.  So is the negabinary conversion (u ^ NB) - NB, the low words of
// u ^ NB and NB being equal.  (K >= 38 would do.)
constexpr int WRAP32_KMIN = 39;

// ---- staging layout ---------------------------------------------------------
// A wave's staging area holds word w of lane l's block at st[w * STAGE_STRIDE + l]
// (see stage_words below).
constexpr int STAGE_STRIDE = 65;
constexpr int STAGE_MAX_RATE = 16;   // larger rates decode from global memory

// ---- bit reader over one block's words ------------------------------------
// Word w of the block sits at p[w * STRIDE]: STRIDE = 1 reads the stream in
// global memory, STRIDE = STAGE_STRIDE reads a wave's LDS staging area
// (stage_words below).
template <int STRIDE>
struct BitReader {
    const uint64_t *__restrict__ p;
    uint64_t cur;  // unread bits, LSB first; bits above cnt are zero
    int cnt;

    __host__ __device__ __forceinline__ void refill() {
        cur = *p;
        p += STRIDE;
        cnt = 64;
    }
    __host__ __device__ __forceinline__ void skip(int n) {  // n <= cnt
        cur = (n >= 64) ? 0 : (cur >> n);
        cnt -= n;
    }
    __host__ __device__ __forceinline__ uint32_t bit() {
        if (cnt == 0) refill();
        uint32_t b = (uint32_t)(cur & 1u);
        cur >>= 1;
        cnt--;
        return b;
    }
    __host__ __device__ __forceinline__ uint64_t read(int n) {  // 0 <= n <= 64
        if (n <= cnt) {
            uint64_t v = (n >= 64) ? cur : (cur & ((1ull << n) - 1));
            skip(n);
            return v;
        }
        uint64_t w = *p;
        p += STRIDE;
        int take = n - cnt;  // 1..64, cnt < 64
        uint64_t v = cur | (w << cnt);
        if (n < 64) v &= (1ull << n) - 1;
        cur = (take >= 64) ? 0 : (w >> take);
        cnt = 64 - take;
        return v;
    }
};

// Bytes of the 8-byte value hi:lo picked by the selector bytes of sel (each
// 0..7, byte 0 = the lowest of lo): one v_perm_b32.
__host__ __device__ __forceinline__ uint32_t byte_perm(uint32_t hi, uint32_t lo, uint32_t sel) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_perm(hi, lo, sel);
#else
    const uint64_t v = (uint64_t)hi << 32 | lo;
    uint32_t r = 0;
    for (int i = 0; i < 4; i++) r |= (uint32_t)(v >> (8 * ((sel >> (8 * i)) & 7u)) & 0xFFu) << (8 * i);
    return r;
#endif
}
// The bits of a where m is set, of b elsewhere: one v_bfi_b32 (the compiler
// does not form it from this expression here).
__host__ __device__ __forceinline__ uint32_t bit_select(uint32_t m, uint32_t a, uint32_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
    uint32_t r;
    asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "s"(m), "v"(a), "v"(b));
    return r;
#else
    return (m & a) | (~m & b);
#endif
}

// One stage of an in-place 32x32 bit-matrix transpose (bit i of a[k] is
// element (k, i)): within every 2J x 2J block the two off-diagonal J x J
// blocks trade places.  M selects the bits i with (i & J) == 0.  Two
// instructions per pair of words at J = 16 and 8 (byte permutes), four
// below (a shift and a bit-field select per word).
template <int J, uint32_t M>
__host__ __device__ __forceinline__ void transpose_stage(uint32_t *a) {
#pragma unroll
    for (int k = 0; k < 32; k++) {
        if (k & J) continue;
        const uint32_t x = a[k], y = a[k + J];
        if constexpr (J == 16) {
            a[k] = byte_perm(y, x, 0x05040100u);       // low halves of x, y
            a[k + J] = byte_perm(y, x, 0x07060302u);   // high halves
        } else if constexpr (J == 8) {
            a[k] = byte_perm(y, x, 0x06020400u);       // bytes x0 y0 x2 y2
            a[k + J] = byte_perm(y, x, 0x07030501u);   // bytes x1 y1 x3 y3
        } else {
            a[k] = bit_select(M, x, y << J);
            a[k + J] = bit_select(M, x >> J, y);
        }
    }
}
__host__ __device__ __forceinline__ void transpose32(uint32_t *a) {
    transpose_stage<16, 0x0000FFFFu>(a);
    transpose_stage<8, 0x00FF00FFu>(a);
    transpose_stage<4, 0x0F0F0F0Fu>(a);
    transpose_stage<2, 0x33333333u>(a);
    transpose_stage<1, 0x55555555u>(a);
}

// Decode one block (64*rate bits read through `br`) into 64 floats in block
// order.  The bits of bit plane k are deposited only into the coefficients
// below n (the number of significant coefficients after the plane), in
// groups of 8: higher coefficients have no bit in the plane.
template <bool F64, class BR>
__host__ __device__ __forceinline__ void decode_block_from(BR br, int rate, float *out) {
    using T = Prec<F64>;
    using UInt = typename T::UInt;
    using Int = typename T::Int;
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
        const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
#pragma unroll
        for (int g = 0; g < 8; g++) {
            if (n > 8 * g) {
                const uint32_t wv = g < 4 ? lo : hi;
#pragma unroll
                for (int i = 8 * g; i < 8 * g + 8; i++) c[i] |= (UInt)((wv >> (i & 31)) & 1u) << k;
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

// ---- decoding from a staging area: two passes -------------------------------
// Lanes of a wave decode different blocks, and the group tests of one plane
// take a data-dependent number of steps, so a plane-by-plane decode makes
// every lane wait for the wave's slowest lane in every plane.  Here a lane
// first walks its whole stream on its own (pass 1), one group-test step per
// iteration, recording for each plane only the length of its group-test
// part and how far it advanced n; the coefficients found significant are
// kept as one 64-bit set.  Pass 2 then rebuilds every plane word in
// lockstep: plane k holds the stream bits of its first n_k coefficients,
// read again at the plane's offset, and ones at the found coefficients in
// [n_k, n_{k+1}) (the coefficients its group tests passed over; exactly one
// plane visits each coefficient this way).  Single precision turns its 32
// plane words into the coefficients by two 32x32 bit transposes; double
// precision deposits each plane word into the coefficients below n_{k+1}.
//
// Word w of the lane's block is st[w * STAGE_STRIDE]; rec holds the lane's
// P/2 record words (plane k's record is the low half of word k/2 for even
// k, the high half for odd k: group-test bits in the low byte, the advance
// of n in the high byte; whole words are written, an odd plane's record
// waits for its even neighbour).
template <bool F64>
struct RecLayout {
    static constexpr int STRIDE = Prec<F64>::P / 2 + 1;   // 32-bit words per lane (odd: no bank conflicts)
    static constexpr int WORDS = 64 * STRIDE / 2;          // 64-bit words of record area per wave
};

// The 64 stream bits from bit offset off (< 64 * rate) on.  Reads words
// off/64 and off/64 + 1: the word past the block's last one lies in the
// wave's record area (which follows the staged words), in bounds of the
// wave's LDS; its bits are masked out by every caller.
__host__ __device__ __forceinline__ uint64_t peek_staged(const uint64_t *st, int off) {
    const uint32_t wi = (uint32_t)off >> 6, sh = (uint32_t)off & 63u;
    const uint64_t *p = st + wi * (uint32_t)STAGE_STRIDE;
    const uint64_t w0 = p[0], w1 = p[STAGE_STRIDE];
    return (w0 >> sh) | ((w1 << 1) << (63u - sh));
}

__host__ __device__ __forceinline__ int ctz64(uint64_t x) {   // x != 0
    return (int)__builtin_ctzll(x);
}

// Pass 1 (after a nonzero block header): returns the found set; kend is the
// lowest plane visited, and the records of planes kend..P-1 are written.
// The group tests form one serial chain (each starts where the previous one
// ended), so the words under the read position are held in registers (words
// wb and wb + 1) and fetched again only when the position moves to another
// word: most steps then wait on no memory read.
template <bool F64>
__host__ __device__ __forceinline__ uint64_t staged_pass1(const uint64_t *st, uint32_t *rec, int rate,
                                                          int &kend) {
    using T = Prec<F64>;
    const int end_bits = 64 * rate;
    int off = 1 + T::EBITS, budget = end_bits - off, n = 0, k = T::P - 1;
    int gstart = 0, nstart = 0;
    bool at_start = true;
    uint64_t found = 0;
    uint32_t pend = 0;   // record of the odd plane above, written with its even neighbour
    int wb = 0;
    uint64_t w0 = st[0], w1 = rate > 1 ? st[STAGE_STRIDE] : 0ull;
    while (k >= 0 && budget > 0) {
        if (at_start) {   // skip the bits of the n significant coefficients
            const int m = n < budget ? n : budget;
            off += m;
            budget -= m;
            gstart = off;
            nstart = n;
            at_start = false;
        }
        bool end = true;
        if (n < 64 && budget > 0) {
            // one group test: a 0 ends the plane; a 1 is followed by zeros up
            // to the next significant coefficient, which the run may not
            // pass: coefficient 63 (implied) and the budget (the run stops
            // where the bits end) bound it at lim
            const int wi = off >> 6;   // < rate: budget > 0
            if (wi != wb) {
                wb = wi;
                w0 = st[wi * STAGE_STRIDE];
                w1 = wi + 1 < rate ? st[(wi + 1) * STAGE_STRIDE] : 0ull;
            }
            const uint32_t sh = (uint32_t)off & 63u;
            const uint64_t w = (w0 >> sh) | ((w1 << 1) << (63u - sh));
            const int lim = (63 - n < budget - 1) ? 63 - n : budget - 1;
            const int z = ctz64((w >> 1) | (1ull << lim));
            const bool g = (w & 1u) != 0;
            const int adv = g ? 2 + z - (z == lim ? 1 : 0) : 1;
            off += adv;
            budget -= adv;
            found |= (uint64_t)g << (n + z);
            n += g ? z + 1 : 0;
            end = !g || n == 64 || budget == 0;
            // after a find, a 0 as the next group test (mostly still inside
            // w) ends the plane in this step
            if (!end && adv < 64 && !((w >> adv) & 1u)) {
                off++;
                budget--;
                end = true;
            }
        }
        if (end) {
            const uint32_t r = (uint32_t)(off - gstart) | ((uint32_t)(n - nstart) << 8);
            if (k & 1) pend = r;
            else rec[k >> 1] = r | (pend << 16);
            k--;
            at_start = true;
        }
    }
    kend = k + 1;
    if (kend & 1) rec[kend >> 1] = pend << 16;
    return found;
}

__host__ __device__ __forceinline__ void decode_block_staged_f32(const uint64_t *st, uint32_t *rec,
                                                                 int rate, float *out) {
    using T = Prec<false>;
    const uint64_t head = st[0];
    // an all-zero block takes the same path with no plane visited (see
    // decode_block_staged_f64_low)
    const bool zero = !(head & 1u);
    const int emax = zero ? 0 : (int)((head >> 1) & 0xFFu) - T::BIAS;
    const int end_bits = 64 * rate;
    int kend = T::P;
    uint64_t found = 0;
    if (!zero) found = staged_pass1<false>(st, rec, rate, kend);
    // ---- pass 2: plane words, in lockstep ----
    uint32_t R[16];
#pragma unroll
    for (int j = 0; j < 16; j++) R[j] = rec[j];
    uint32_t lo[32], hi[32];
    int o = 1 + T::EBITS, nn = 0;
    uint64_t below = 0;   // coefficients below nn
#pragma unroll
    for (int kk = T::P - 1; kk >= 0; kk--) {
        uint64_t x = 0;
        if (kk >= kend) {
            const uint32_t rk = (kk & 1) ? (R[kk >> 1] >> 16) : (R[kk >> 1] & 0xFFFFu);
            const int m = nn < end_bits - o ? nn : end_bits - o;
            if (m > 0) x = peek_staged(st, o) & (~0ull >> (64 - m));
            const int nn2 = nn + (int)(rk >> 8);
            const uint64_t below2 = nn2 >= 64 ? ~0ull : ((1ull << nn2) - 1);
            x |= found & below2 & ~below;
            below = below2;
            nn = nn2;
            o += m + (int)(rk & 0xFFu);
        }
        lo[kk] = (uint32_t)x;
        hi[kk] = (uint32_t)(x >> 32);
    }
    transpose32(lo);
    transpose32(hi);
    int32_t v[64];
#pragma unroll
    for (int r = 0; r < 32; r++) {
        v[kOrder.idx[r]] = (int32_t)((lo[r] ^ T::NB) - T::NB);
        v[kOrder.idx[r + 32]] = (int32_t)((hi[r] ^ T::NB) - T::NB);
    }
    inv_zyx(v);
    const float s = ldexpf(1.0f, emax - 30);
#pragma unroll
    for (int i = 0; i < 64; i++) out[i] = (float)v[i] * s;
}

// Pass 2 and the transform of a double-precision block whose stream ends by
// plane WRAP32_KMIN (low rates), on the coefficients' high 32-bit words: the
// visited planes kend..63 are the rows kend - 32..31 of a bit matrix (row r =
// plane 32 + r; the rows below are zero), rebuilt in lockstep and turned into
// the high words by two 32x32 transposes; then negabinary conversion and the
// inverse transform in 32 bits (exact, see WRAP32_KMIN).  The 64-bit value
// is the high word times 2^32, and the double value of the decoded sample
// h * 2^32 * 2^(emax - 62) = h * 2^(emax - 30), |h| < 2^31: for -96 <= emax
// <= 96 that is float(h) * 2^(emax - 30) in single precision, rounded once
// and never subnormal, else it is formed in double as the plain decoder does.
// SINGLE_ONLY: the caller guarantees -96 <= emax <= 96 (no double-precision
// branch, whose results the compiler would merge with register copies).
template <bool SINGLE_ONLY = false>
__host__ __device__ __forceinline__ void staged_f64_top_planes(const uint64_t *st, const uint32_t *rec,
                                                               int rate, uint64_t found, int kend, int emax,
                                                               float *out) {
    using T = Prec<true>;
    const int end_bits = 64 * rate;
    uint32_t lo[32], hi[32];
#pragma unroll
    for (int r = 0; r < WRAP32_KMIN - 32; r++) lo[r] = hi[r] = 0u;
    int o = 1 + T::EBITS, nn = 0;
    uint64_t below = 0;
#pragma unroll
    for (int r = 31; r >= WRAP32_KMIN - 32; r--) {
        const int kk = 32 + r;
        uint64_t x = 0;
        if (kk >= kend) {
            const uint32_t rw = rec[kk >> 1], rk = (kk & 1) ? (rw >> 16) : (rw & 0xFFFFu);
            const int m = nn < end_bits - o ? nn : end_bits - o;
            if (m > 0) x = peek_staged(st, o) & (~0ull >> (64 - m));
            const int nn2 = nn + (int)(rk >> 8);
            const uint64_t below2 = nn2 >= 64 ? ~0ull : ((1ull << nn2) - 1);
            x |= found & below2 & ~below;
            below = below2;
            nn = nn2;
            o += m + (int)(rk & 0xFFu);
        }
        lo[r] = (uint32_t)x;
        hi[r] = (uint32_t)(x >> 32);
    }
    transpose32(lo);
    transpose32(hi);
    constexpr uint32_t NB_HI = (uint32_t)(T::NB >> 32);
    int32_t v[64];
#pragma unroll
    for (int r = 0; r < 32; r++) {
        v[kOrder.idx[r]] = (int32_t)((lo[r] ^ NB_HI) - NB_HI);
        v[kOrder.idx[r + 32]] = (int32_t)((hi[r] ^ NB_HI) - NB_HI);
    }
    inv_zyx(v);
    if (SINGLE_ONLY || (emax >= -96 && emax <= 96)) {
        const float s = ldexpf(1.0f, emax - 30);
#pragma unroll
        for (int i = 0; i < 64; i++) out[i] = (float)v[i] * s;
    } else {
        const double s = ldexp(1.0, emax - 62);
#pragma unroll
        for (int i = 0; i < 64; i++) out[i] = (float)((double)v[i] * 4294967296.0 * s);
    }
}

__host__ __device__ __forceinline__ void decode_block_staged_f64(const uint64_t *st, uint32_t *rec,
                                                                 int rate, float *out) {
    using T = Prec<true>;
    const uint64_t head = st[0];
    if (!(head & 1u)) {
#pragma unroll
        for (int i = 0; i < 64; i++) out[i] = 0.0f;
        return;
    }
    const int emax = (int)((head >> 1) & 0x7FFu) - T::BIAS;
    const int end_bits = 64 * rate;
    int kend;
    const uint64_t found = staged_pass1<true>(st, rec, rate, kend);
    const double s = ldexp(1.0, emax - 62);
    if (kend >= WRAP32_KMIN) {
        staged_f64_top_planes(st, rec, rate, found, kend, emax, out);
        return;
    }
    // ---- pass 2: plane words in lockstep, each deposited into the
    // coefficients below n_{k+1} in groups of 8 ----
    uint64_t c[64];
#pragma unroll
    for (int i = 0; i < 64; i++) c[i] = 0;
    int o = 1 + T::EBITS, nn = 0;
    uint64_t below = 0;
    for (int kk = T::P - 1; kk >= kend; kk--) {
        const uint32_t rw = rec[kk >> 1], rk = (kk & 1) ? (rw >> 16) : (rw & 0xFFFFu);
        const int m = nn < end_bits - o ? nn : end_bits - o;
        uint64_t x = m > 0 ? peek_staged(st, o) & (~0ull >> (64 - m)) : 0ull;
        const int nn2 = nn + (int)(rk >> 8);
        const uint64_t below2 = nn2 >= 64 ? ~0ull : ((1ull << nn2) - 1);
        x |= found & below2 & ~below;
        below = below2;
        nn = nn2;
        o += m + (int)(rk & 0xFFu);
        const uint32_t xl = (uint32_t)x, xh = (uint32_t)(x >> 32);
#pragma unroll
        for (int g = 0; g < 8; g++) {
            if (nn > 8 * g) {
                const uint32_t wv = g < 4 ? xl : xh;
#pragma unroll
                for (int i = 8 * g; i < 8 * g + 8; i++) c[i] |= (uint64_t)((wv >> (i & 31)) & 1u) << kk;
            }
        }
    }
    int64_t v[64];
#pragma unroll
    for (int r = 0; r < 64; r++) v[kOrder.idx[r]] = (int64_t)((c[r] ^ T::NB) - T::NB);
    inv_zyx(v);
#pragma unroll
    for (int i = 0; i < 64; i++) out[i] = (float)((double)v[i] * s);
}

// Low-rate double precision: the block when its stream ends by plane
// WRAP32_KMIN and |emax| <= 96 (pass 1, then staged_f64_top_planes, the same
// values as decode_block_staged_f64) and true; false, with out untouched, for
// a block whose stream goes on below that plane or whose exponent is outside
// that range (the caller decodes it with the general decoder).
__host__ __device__ __forceinline__ bool decode_block_staged_f64_low(const uint64_t *st, uint32_t *rec,
                                                                    int rate, float *out) {
    using T = Prec<true>;
    const uint64_t head = st[0];
    // An all-zero block takes the same path with no plane visited (every
    // coefficient 0, any scale): one path that writes `out`, so that the
    // compiler does not merge the results of several with register copies.
    const bool zero = !(head & 1u);
    const int emax = zero ? 0 : (int)((head >> 1) & 0x7FFu) - T::BIAS;
    if (emax < -96 || emax > 96) return false;   // values formed in double: the general decoder's
    int kend = T::P;
    uint64_t found = 0;
    if (!zero) found = staged_pass1<true>(st, rec, rate, kend);
    if (kend < WRAP32_KMIN) return false;
    staged_f64_top_planes<true>(st, rec, rate, found, kend, emax, out);
    return true;
}

// Decode one block straight from the stream in global memory.
template <bool F64>
__host__ __device__ __forceinline__ void decode_block(const uint64_t *__restrict__ words, int rate,
                                             float *out) {
    decode_block_from<F64>(BitReader<1>{words, 0, 0}, rate, out);
}

// ---- wave-level staging of the compressed words ----------------------------
// The 64 lanes of a wave each decode one block.  Before decoding, the wave
// copies the words of its blocks into LDS, word w of lane l's block at
// st[w * STAGE_STRIDE + l] (the odd row pitch keeps the transposing writes
// free of bank conflicts).  When the wave's blocks are consecutive (lane l
// holds block b0 + l, the usual case: new blocks are listed in ascending
// order) the copy reads one contiguous run of the stream, 512 bytes per
// instruction; otherwise each lane copies its own block's words.

// `words`: lane l's block's first word (rate words follow); the rate is
// uniform over the wave.
__device__ __forceinline__ void stage_words_at(const uint64_t *__restrict__ words, int rate, bool valid,
                                               uint64_t *st) {
    const int l = (int)__lane_id();
    const uint64_t vmask = __ballot(valid);
    const uint64_t a = reinterpret_cast<uint64_t>(words);
    const uint64_t a0 = ((uint64_t)__shfl((uint32_t)(a >> 32), 0, 64) << 32) | __shfl((uint32_t)a, 0, 64);
    const bool prefix = (vmask & (vmask + 1)) == 0;   // valid lanes are 0..nv-1
    const bool consecutive = prefix && (vmask & 1) &&
                             __ballot(valid && a == a0 + 8ull * (uint64_t)rate * (uint64_t)l) == vmask;
    if (consecutive) {
        const uint32_t total = (uint32_t)__popcll(vmask) * (uint32_t)rate;
        // i / rate as (i * ceil(2^32 / rate)) >> 32: exact for i < 2^32 / rate
        const uint64_t magic = ((1ull << 32) + (uint64_t)rate - 1) / (uint64_t)rate;
        const uint64_t *src = reinterpret_cast<const uint64_t *>(a0);
        for (uint32_t i = (uint32_t)l; i < total; i += 64) {
            const uint32_t ln = (uint32_t)(((uint64_t)i * magic) >> 32), wd = i - ln * (uint32_t)rate;
            st[wd * STAGE_STRIDE + ln] = src[i];
        }
    } else if (valid) {
        for (int wd = 0; wd < rate; wd++) st[wd * STAGE_STRIDE + l] = words[wd];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Block b of `stream` for each lane.
__device__ __forceinline__ void stage_words(const uint64_t *__restrict__ stream, int rate, uint64_t b,
                                            bool valid, uint64_t *st) {
    stage_words_at(stream + b * (uint64_t)rate, rate, valid, st);
}

// 64-bit words of LDS one wave uses at `rate`: the staged words, then the
// per-lane plane records of the two-pass decoder.
__host__ __device__ inline unsigned stage_wave_words(int rate, bool f64) {
    return (unsigned)(STAGE_STRIDE * rate + (f64 ? RecLayout<true>::WORDS : RecLayout<false>::WORDS));
}

// Lane l's block from the staging area by decode_block_staged_f64_low.
__device__ __forceinline__ bool decode_block_staged_low(uint64_t *st, int rate, float *out) {
    uint32_t *rec = reinterpret_cast<uint32_t *>(st + STAGE_STRIDE * rate) + __lane_id() * RecLayout<true>::STRIDE;
    return decode_block_staged_f64_low(st + __lane_id(), rec, rate, out);
}

// Decode lane l's block from the staging area (stage_wave_words(rate, F64)
// words per wave) written by stage_words.
template <bool F64>
__device__ __forceinline__ void decode_block_staged(uint64_t *st, int rate, float *out) {
    uint32_t *rec = reinterpret_cast<uint32_t *>(st + STAGE_STRIDE * rate) + __lane_id() * RecLayout<F64>::STRIDE;
    if constexpr (F64) decode_block_staged_f64(st + __lane_id(), rec, rate, out);
    else decode_block_staged_f32(st + __lane_id(), rec, rate, out);
}

// Bytes of dynamic LDS a 256-thread workgroup needs for staging at `rate`
// (0: the rate is decoded from global memory: above STAGE_MAX_RATE, or when
// the staged words and records would pass 64 KB, as double precision does
// at rate 16).
constexpr unsigned STAGE_MAX_LDS = 64u * 1024u;
__host__ __device__ inline unsigned stage_lds_bytes(int rate, bool f64) {
    if (rate < 1 || rate > STAGE_MAX_RATE) return 0u;
    const unsigned b = 4u * stage_wave_words(rate, f64) * 8u;
    return b <= STAGE_MAX_LDS ? b : 0u;
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
