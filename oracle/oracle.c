/*
 * CPU oracle for block-compressed isosurface extraction -- TEST
 * INFRASTRUCTURE ONLY (see oracle.h).  Plain single-threaded C, no HIP, no
 * shared code with the GPU library.  Built with -O2 -ffp-contract=off.
 *
 * Paper: Usher & Pascucci, "Interactive Visualization of Terascale Data in the
 * Browser: Fact or Fiction?" (arXiv 2009.03254).  Citations name the paper's
 * section, algorithm or table.  ZFP internals are not in the paper (it only
 * cites Lindstrom, "Fixed-Rate Compressed Floating-Point Arrays", TVCG 2014);
 * the codec below is written from that publication's description of the
 * method: common block exponent, block floating point, a separable integer
 * lifting transform, sequency ordering, negabinary, embedded bit-plane coding
 * with group tests, truncated at a fixed bit budget.  Its bit layout is this
 * project's own; compatibility with the zfp library bitstream is
 * "parity unpinned" (the library is not available).
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ======================================================================= */
/* geometry                                                                */
/* ======================================================================= */

static uint32_t ceil4(uint32_t n) { return (n + 3u) / 4u; }

uint64_t oracle_num_blocks(uint32_t nx, uint32_t ny, uint32_t nz) {
    return (uint64_t)ceil4(nx) * ceil4(ny) * ceil4(nz);
}

/* ======================================================================= */
/* ZFP fixed-rate codec (Sec. 3.3.4; Sec. 4.2.1 decodes single blocks)     */
/* ======================================================================= */

/* Precision P (bits per integer coefficient), exponent field width and bias. */
static int prec_bits(int is_f64) { return is_f64 ? 64 : 32; }
static int exp_bits(int is_f64) { return is_f64 ? 11 : 8; }
static int exp_bias(int is_f64) { return is_f64 ? 1023 : 127; }
/* Smallest encodable block exponent: keeps 2^(emax - (P-2)) a normal number,
 * so that decoding never produces subnormals from a scale factor. */
static int exp_min(int is_f64) { return is_f64 ? (62 - 1022) : (30 - 126); }

/* Two's-complement arithmetic at the stream precision (wraps mod 2^P). */
static int64_t wrapP(int64_t v, int is_f64) {
    return is_f64 ? v : (int64_t)(int32_t)(uint32_t)(uint64_t)v;
}
static int64_t addP(int64_t a, int64_t b, int f) {
    return wrapP((int64_t)((uint64_t)a + (uint64_t)b), f);
}
static int64_t subP(int64_t a, int64_t b, int f) {
    return wrapP((int64_t)((uint64_t)a - (uint64_t)b), f);
}
static int64_t shl1P(int64_t a, int f) { return wrapP((int64_t)((uint64_t)a << 1), f); }
static int64_t shr1P(int64_t a) { return a >> 1; } /* arithmetic shift */

/*
 * Forward decorrelating transform of 4 values (Lindstrom 2014).  In exact
 * arithmetic it is the matrix
 *     (1/16) [[ 4, 4, 4, 4], [ 5, 1,-1,-5], [-4, 4, 4,-4], [-2, 6,-6, 2]]
 * applied to (v0,v1,v2,v3), realised as five lifting steps that each average
 * or difference a pair (the halvings drop one bit):
 *   1. v0 <- (v0+v3)/2, v3 <- v3-v0      (outer pair: mean, half-difference)
 *   2. v2 <- (v2+v1)/2, v1 <- v1-v2      (inner pair)
 *   3. v0 <- (v0+v2)/2, v2 <- v2-v0      (DC and the even "curvature" term)
 *   4. v3 <- (v3+v1)/2, v1 <- v1-v3      (mix the two odd terms)
 *   5. v3 <- v3 + v1/2, v1 <- v1 - v3/2  (rotate the odd terms)
 * giving (DC, linear, quadratic, cubic) = rows 1..4 of the matrix.
 */
void oracle_fwd_lift(int64_t *v, int f) {
    int64_t a = v[0], b = v[1], c = v[2], d = v[3];
    a = shr1P(addP(a, d, f)); d = subP(d, a, f);
    c = shr1P(addP(c, b, f)); b = subP(b, c, f);
    a = shr1P(addP(a, c, f)); c = subP(c, a, f);
    d = shr1P(addP(d, b, f)); b = subP(b, d, f);
    d = addP(d, shr1P(b), f); b = subP(b, shr1P(d), f);
    v[0] = a; v[1] = b; v[2] = c; v[3] = d;
}

/* Inverse: undo steps 5,4,3,2,1 in that order.  Step 5 is undone exactly;
 * a step "x <- (x+y)/2, y <- y-x" is undone by "y <- y+x, x <- 2x-y". */
void oracle_inv_lift(int64_t *v, int f) {
    int64_t a = v[0], b = v[1], c = v[2], d = v[3];
    b = addP(b, shr1P(d), f); d = subP(d, shr1P(b), f);   /* undo 5 */
    b = addP(b, d, f); d = subP(shl1P(d, f), b, f);        /* undo 4 */
    c = addP(c, a, f); a = subP(shl1P(a, f), c, f);        /* undo 3 */
    b = addP(b, c, f); c = subP(shl1P(c, f), b, f);        /* undo 2 */
    d = addP(d, a, f); a = subP(shl1P(a, f), d, f);        /* undo 1 */
    v[0] = a; v[1] = b; v[2] = c; v[3] = d;
}

/* Apply a 4-point lift along one axis of a 4x4x4 block (stride 1, 4, 16). */
static void lift_axis(int64_t *blk, int stride, int inverse, int f) {
    int s1 = (stride == 1) ? 4 : 1;          /* the two other strides */
    int s2 = (stride == 16) ? 4 : 16;
    for (int j = 0; j < 4; j++)
        for (int i = 0; i < 4; i++) {
            int base = i * s1 + j * s2;
            int64_t t[4];
            for (int k = 0; k < 4; k++) t[k] = blk[base + k * stride];
            if (inverse) oracle_inv_lift(t, f); else oracle_fwd_lift(t, f);
            for (int k = 0; k < 4; k++) blk[base + k * stride] = t[k];
        }
}

/* Coding order of the 64 transform coefficients: ascending total sequency
 * i+j+k, ties broken by ascending block index i + 4j + 16k. */
static int seq_cmp(const void *pa, const void *pb) {
    int a = *(const int *)pa, b = *(const int *)pb;
    int sa = (a & 3) + ((a >> 2) & 3) + (a >> 4);
    int sb = (b & 3) + ((b >> 2) & 3) + (b >> 4);
    if (sa != sb) return sa - sb;
    return a - b;
}

void oracle_sequency_order(int *perm) {
    for (int i = 0; i < 64; i++) perm[i] = i;
    qsort(perm, 64, sizeof(int), seq_cmp);
}

/* Negabinary (base -2) representation: u = (i + M) xor M, M = 0xAA..AA. */
uint64_t oracle_to_negabinary(int64_t i, int f) {
    if (f) {
        const uint64_t M = 0xAAAAAAAAAAAAAAAAull;
        return ((uint64_t)i + M) ^ M;
    }
    const uint32_t M = 0xAAAAAAAAu;
    return (uint64_t)(((uint32_t)(uint64_t)i + M) ^ M);
}

int64_t oracle_from_negabinary(uint64_t u, int f) {
    if (f) {
        const uint64_t M = 0xAAAAAAAAAAAAAAAAull;
        return (int64_t)((u ^ M) - M);
    }
    const uint32_t M = 0xAAAAAAAAu;
    return (int64_t)(int32_t)(((uint32_t)u ^ M) - M);
}

/* Bit i of a little-endian u64 word array, LSB first. */
static void put_bit(uint64_t *w, uint64_t pos, unsigned bit) {
    if (bit) w[pos >> 6] |= (uint64_t)1 << (pos & 63);
}
static unsigned get_bit(const uint64_t *w, uint64_t pos) {
    return (unsigned)((w[pos >> 6] >> (pos & 63)) & 1u);
}

/*
 * Embedded bit-plane coding (Lindstrom 2014), planes from the most
 * significant down, stopping the moment maxbits bits are spent.  n counts the
 * coefficients (in coding order) already known to be significant; they form
 * a prefix.  For each plane:
 *   (a) the plane bits of the first n coefficients are sent verbatim;
 *   (b) group test: one bit telling whether any coefficient at or beyond n
 *       has a 1 in this plane.  If so, the bits of coefficients n, n+1, ...
 *       are sent until a 1 is sent; coefficient 63's bit is never sent (it
 *       must be the 1).  That coefficient and all before it join the
 *       significant prefix, and the group test repeats.
 * If the budget ends during the scan, the coefficient at the scan position
 * is taken as the one holding the 1 (the decoder does the same).
 */
uint64_t oracle_encode_planes(const uint64_t *u, int f, uint64_t maxbits,
                              uint64_t *words) {
    int P = prec_bits(f);
    uint64_t pos = 0;
    int n = 0;
    for (int k = P - 1; k >= 0 && pos < maxbits; k--) {
        for (int i = 0; i < n && pos < maxbits; i++)
            put_bit(words, pos++, (unsigned)((u[i] >> k) & 1u));
        while (n < 64 && pos < maxbits) {
            unsigned any = 0;
            for (int i = n; i < 64; i++) any |= (unsigned)((u[i] >> k) & 1u);
            put_bit(words, pos++, any);
            if (!any) break;
            while (n < 63 && pos < maxbits) {
                unsigned b = (unsigned)((u[n] >> k) & 1u);
                put_bit(words, pos++, b);
                if (b) break;
                n++;
            }
            n++;
        }
    }
    return pos;
}

void oracle_decode_planes(const uint64_t *words, int f, uint64_t maxbits,
                          uint64_t *u) {
    int P = prec_bits(f);
    uint64_t pos = 0;
    int n = 0;
    for (int i = 0; i < 64; i++) u[i] = 0;
    for (int k = P - 1; k >= 0 && pos < maxbits; k--) {
        for (int i = 0; i < n && pos < maxbits; i++)
            u[i] |= (uint64_t)get_bit(words, pos++) << k;
        while (n < 64 && pos < maxbits) {
            unsigned any = get_bit(words, pos++);
            if (!any) break;
            while (n < 63 && pos < maxbits) {
                unsigned b = get_bit(words, pos++);
                if (b) break;
                n++;
            }
            u[n] |= (uint64_t)1 << k;
            n++;
        }
    }
}

/* Encode one block of 64 values (already gathered, block index order). */
static void encode_block(const double *x, int f, uint32_t rate, uint64_t *out) {
    uint64_t maxbits = 64ull * rate;
    int P = prec_bits(f), q = P - 2, EB = exp_bits(f);
    memset(out, 0, sizeof(uint64_t) * rate);
    int emax = INT32_MIN, any = 0;
    for (int i = 0; i < 64; i++)
        if (x[i] != 0.0) {
            int e;
            frexp(x[i], &e);
            if (!any || e > emax) emax = e;
            any = 1;
        }
    if (!any) return; /* header bit 0: all-zero block */
    if (emax < exp_min(f)) emax = exp_min(f);
    /* header: a 1, then emax + bias in EB bits (LSB first) */
    put_bit(out, 0, 1);
    uint32_t E = (uint32_t)(emax + exp_bias(f));
    for (int j = 0; j < EB; j++) put_bit(out, 1 + (uint64_t)j, (E >> j) & 1u);
    /* block floating point: i = trunc(x * 2^(q - emax)); exact scaling */
    int64_t blk[64];
    for (int i = 0; i < 64; i++) {
        if (f) blk[i] = (int64_t)ldexp(x[i], q - emax);
        else blk[i] = (int64_t)(int32_t)ldexpf((float)x[i], q - emax);
    }
    lift_axis(blk, 1, 0, f);
    lift_axis(blk, 4, 0, f);
    lift_axis(blk, 16, 0, f);
    int perm[64];
    oracle_sequency_order(perm);
    uint64_t u[64];
    for (int r = 0; r < 64; r++) u[r] = oracle_to_negabinary(blk[perm[r]], f);
    /* the coefficient bits follow the header in the same word array */
    uint64_t hdr = 1 + (uint64_t)EB;
    uint64_t tmp[64 * 64 / 64 + 2];
    uint64_t words_needed = (maxbits - hdr + 63) / 64 + 1;
    uint64_t *planes = tmp;
    uint64_t *heap = NULL;
    if (words_needed > sizeof(tmp) / sizeof(tmp[0])) {
        heap = (uint64_t *)calloc(words_needed, sizeof(uint64_t));
        planes = heap;
    } else {
        memset(tmp, 0, sizeof(tmp));
    }
    uint64_t used = oracle_encode_planes(u, f, maxbits - hdr, planes);
    for (uint64_t p = 0; p < used; p++)
        put_bit(out, hdr + p, get_bit(planes, p));
    free(heap);
}

/* Decode one block into 64 doubles (exact values of the decoded floats). */
static void decode_block(const uint64_t *in, int f, uint32_t rate, double *x) {
    uint64_t maxbits = 64ull * rate;
    int P = prec_bits(f), q = P - 2, EB = exp_bits(f);
    if (!get_bit(in, 0)) {
        for (int i = 0; i < 64; i++) x[i] = 0.0;
        return;
    }
    uint32_t E = 0;
    for (int j = 0; j < EB; j++) E |= get_bit(in, 1 + (uint64_t)j) << j;
    int emax = (int)E - exp_bias(f);
    uint64_t hdr = 1 + (uint64_t)EB;
    /* copy the coefficient bits to a zero-based word array */
    uint64_t nb = maxbits - hdr;
    uint64_t *planes = (uint64_t *)calloc(nb / 64 + 2, sizeof(uint64_t));
    for (uint64_t p = 0; p < nb; p++) put_bit(planes, p, get_bit(in, hdr + p));
    uint64_t u[64];
    oracle_decode_planes(planes, f, nb, u);
    free(planes);
    int perm[64];
    oracle_sequency_order(perm);
    int64_t blk[64];
    for (int r = 0; r < 64; r++) blk[perm[r]] = oracle_from_negabinary(u[r], f);
    lift_axis(blk, 16, 1, f);
    lift_axis(blk, 4, 1, f);
    lift_axis(blk, 1, 1, f);
    if (f) {
        double s = ldexp(1.0, emax - q);
        for (int i = 0; i < 64; i++) x[i] = (double)blk[i] * s;
    } else {
        float s = ldexpf(1.0f, emax - q);
        for (int i = 0; i < 64; i++) x[i] = (double)((float)(int32_t)blk[i] * s);
    }
}

static int valid_rate(int f, uint32_t rate) {
    return rate >= 1 && rate <= (uint32_t)(f ? 64 : 32);
}

int oracle_zfp_encode(const void *field, int f, uint32_t nx, uint32_t ny,
                      uint32_t nz, uint32_t rate, uint64_t *stream) {
    if (!valid_rate(f, rate) || nx < 1 || ny < 1 || nz < 1) return -1;
    uint32_t nbx = ceil4(nx), nby = ceil4(ny), nbz = ceil4(nz);
    const float *f32 = (const float *)field;
    const double *f64 = (const double *)field;
    uint64_t nvox = (uint64_t)nx * ny * nz;
    for (uint64_t i = 0; i < nvox; i++) {
        double v = f ? f64[i] : (double)f32[i];
        if (!isfinite(v)) return -6;
    }
    for (uint32_t bz = 0; bz < nbz; bz++)
        for (uint32_t by = 0; by < nby; by++)
            for (uint32_t bx = 0; bx < nbx; bx++) {
                double x[64];
                for (int l = 0; l < 64; l++) {
                    /* partial blocks: replicate the last valid sample */
                    uint32_t gx = 4 * bx + (l & 3), gy = 4 * by + ((l >> 2) & 3),
                             gz = 4 * bz + (l >> 4);
                    if (gx >= nx) gx = nx - 1;
                    if (gy >= ny) gy = ny - 1;
                    if (gz >= nz) gz = nz - 1;
                    uint64_t idx = gx + (uint64_t)nx * (gy + (uint64_t)ny * gz);
                    x[l] = f ? f64[idx] : (double)f32[idx];
                }
                uint64_t b = bx + (uint64_t)nbx * (by + (uint64_t)nby * bz);
                encode_block(x, f, rate, stream + b * rate);
            }
    return 0;
}

int oracle_zfp_decode(const uint64_t *stream, int f, uint32_t nx, uint32_t ny,
                      uint32_t nz, uint32_t rate, float *blocks) {
    if (!valid_rate(f, rate)) return -1;
    uint64_t nb = oracle_num_blocks(nx, ny, nz);
    for (uint64_t b = 0; b < nb; b++) {
        double x[64];
        decode_block(stream + b * rate, f, rate, x);
        for (int i = 0; i < 64; i++) blocks[b * 64 + i] = (float)x[i];
    }
    return 0;
}

int oracle_zfp_decode_f64(const uint64_t *stream, uint32_t nx, uint32_t ny,
                          uint32_t nz, uint32_t rate, double *blocks) {
    if (!valid_rate(1, rate)) return -1;
    uint64_t nb = oracle_num_blocks(nx, ny, nz);
    for (uint64_t b = 0; b < nb; b++) decode_block(stream + b * rate, 1, rate, blocks + b * 64);
    return 0;
}

int oracle_zfp_decode_some(const uint64_t *stream, int f, uint32_t rate,
                           const uint32_t *ids, uint64_t n, float *blocks) {
    if (!valid_rate(f, rate)) return -1;
    for (uint64_t i = 0; i < n; i++) {
        double x[64];
        decode_block(stream + (uint64_t)ids[i] * rate, f, rate, x);
        for (int k = 0; k < 64; k++) blocks[i * 64 + k] = (float)x[k];
    }
    return 0;
}

/* ======================================================================= */
/* value ranges and active blocks (Sec. 4.1)                               */
/* ======================================================================= */

void oracle_block_ranges(const float *blocks, uint32_t nx, uint32_t ny,
                         uint32_t nz, float *ranges) {
    uint32_t nbx = ceil4(nx), nby = ceil4(ny), nbz = ceil4(nz);
    for (uint32_t bz = 0; bz < nbz; bz++)
        for (uint32_t by = 0; by < nby; by++)
            for (uint32_t bx = 0; bx < nbx; bx++) {
                uint64_t b = bx + (uint64_t)nbx * (by + (uint64_t)nby * bz);
                float lo = INFINITY, hi = -INFINITY;
                for (int l = 0; l < 64; l++) {
                    uint32_t gx = 4 * bx + (l & 3), gy = 4 * by + ((l >> 2) & 3),
                             gz = 4 * bz + (l >> 4);
                    if (gx >= nx || gy >= ny || gz >= nz) continue; /* padding */
                    float v = blocks[b * 64 + l];
                    if (v < lo) lo = v;
                    if (v > hi) hi = v;
                }
                ranges[2 * b] = lo;
                ranges[2 * b + 1] = hi;
            }
}

/* A range contains the isovalue when lo < iso <= hi, the same side convention as the
 * cell classification (a corner is inside when its value is < iso). */
static int contains(float lo, float hi, float iso) { return lo < iso && iso <= hi; }

/* Sec. 4.1: a block is active if its range, or the union of its range with
 * the range of any of its neighbours (the 26 blocks sharing a face, an edge
 * or a corner with it), contains the isovalue. */
uint64_t oracle_active_blocks(const float *ranges, uint32_t nx, uint32_t ny,
                              uint32_t nz, float iso, uint8_t *active) {
    int64_t nbx = ceil4(nx), nby = ceil4(ny), nbz = ceil4(nz);
    uint64_t count = 0;
    for (int64_t bz = 0; bz < nbz; bz++)
        for (int64_t by = 0; by < nby; by++)
            for (int64_t bx = 0; bx < nbx; bx++) {
                uint64_t b = (uint64_t)(bx + nbx * (by + nby * bz));
                float lo = ranges[2 * b], hi = ranges[2 * b + 1];
                int act = contains(lo, hi, iso);
                for (int dz = -1; dz <= 1 && !act; dz++)
                    for (int dy = -1; dy <= 1 && !act; dy++)
                        for (int dx = -1; dx <= 1 && !act; dx++) {
                            int64_t x = bx + dx, y = by + dy, z = bz + dz;
                            if (x < 0 || y < 0 || z < 0 || x >= nbx || y >= nby || z >= nbz)
                                continue;
                            uint64_t n = (uint64_t)(x + nbx * (y + nby * z));
                            float ulo = ranges[2 * n] < lo ? ranges[2 * n] : lo;
                            float uhi = ranges[2 * n + 1] > hi ? ranges[2 * n + 1] : hi;
                            if (contains(ulo, uhi, iso)) act = 1;
                        }
                active[b] = (uint8_t)act;
                count += (uint64_t)act;
            }
    return count;
}

/* ======================================================================= */
/* marching cubes table, generated (Sec. 3.3.3 uses Lorensen-Cline MC)     */
/* ======================================================================= */
/*
 * Corner k of a cell sits at offset (k&1, (k>>1)&1, (k>>2)&1).  Edge e runs
 * along axis a = e>>2; bits 0 and 1 of e give its offsets along the other
 * two axes, taken in increasing axis order.  A corner is "inside" when its
 * value is below the isovalue (bit k of the case).
 *
 * For each case the surface is built face by face: on a cube face the
 * crossing edges (2 or 4) are joined by segments; with 4 (the ambiguous
 * face) each inside corner is cut off on its own.  The segments close into
 * polygons, each oriented so that its normal (p1-p0)x(p2-p0) points toward
 * increasing values.  Walking each polygon from its smallest edge id, the
 * fan apex is the first vertex none of whose fan diagonals joins two edges
 * of a common face.  Polygons are listed by their smallest edge id.
 */
static void corner_xyz(int k, int p[3]) {
    p[0] = k & 1; p[1] = (k >> 1) & 1; p[2] = (k >> 2) & 1;
}

static void edge_corners(int e, int *k0, int *k1) {
    int a = e >> 2;
    int u = (a == 0) ? 1 : 0, v = (a == 2) ? 1 : 2;
    int p[3] = {0, 0, 0};
    p[u] = e & 1;
    p[v] = (e >> 1) & 1;
    *k0 = p[0] + 2 * p[1] + 4 * p[2];
    p[a] = 1;
    *k1 = p[0] + 2 * p[1] + 4 * p[2];
}

static void edge_mid(int e, double m[3]) {
    int k0, k1, p0[3], p1[3];
    edge_corners(e, &k0, &k1);
    corner_xyz(k0, p0);
    corner_xyz(k1, p1);
    for (int i = 0; i < 3; i++) m[i] = 0.5 * (p0[i] + p1[i]);
}

static void cross3(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Two cube edges lie in a common face iff some face contains both: an edge
 * lies in face (axis f, side s) when it does not run along f and its
 * endpoints have coordinate s along f. */
static int edges_share_face(int e1, int e2) {
    for (int fa = 0; fa < 3; fa++)
        for (int side = 0; side < 2; side++) {
            int k1, k2, tmp, p1[3], p2[3];
            edge_corners(e1, &k1, &tmp);
            edge_corners(e2, &k2, &tmp);
            corner_xyz(k1, p1);
            corner_xyz(k2, p2);
            if ((e1 >> 2) != fa && (e2 >> 2) != fa && p1[fa] == side && p2[fa] == side)
                return 1;
        }
    return 0;
}

static int gen_case(int cs, int *tri_out) {
    int next[12];
    for (int e = 0; e < 12; e++) next[e] = -1;
    int crossing[12];
    for (int e = 0; e < 12; e++) {
        int k0, k1;
        edge_corners(e, &k0, &k1);
        crossing[e] = ((cs >> k0) & 1) != ((cs >> k1) & 1);
    }
    for (int fa = 0; fa < 3; fa++)
        for (int side = 0; side < 2; side++) {
            double nF[3] = {0, 0, 0};
            nF[fa] = side ? 1.0 : -1.0;
            /* corners and crossing edges of this face */
            int fc[4], nfc = 0, fe[4], nfe = 0;
            for (int k = 0; k < 8; k++) {
                int p[3];
                corner_xyz(k, p);
                if (p[fa] == side) fc[nfc++] = k;
            }
            for (int e = 0; e < 12; e++) {
                if ((e >> 2) == fa || !crossing[e]) continue;
                int k0, k1, p[3];
                edge_corners(e, &k0, &k1);
                corner_xyz(k0, p);
                if (p[fa] == side) fe[nfe++] = e;
            }
            int segs[2][2], nseg = 0;
            double g[2][3];
            if (nfe == 2) {
                double cin[3] = {0, 0, 0}, cout[3] = {0, 0, 0};
                int nin = 0, nout = 0;
                for (int i = 0; i < 4; i++) {
                    int p[3];
                    corner_xyz(fc[i], p);
                    if ((cs >> fc[i]) & 1) { for (int d = 0; d < 3; d++) cin[d] += p[d]; nin++; }
                    else { for (int d = 0; d < 3; d++) cout[d] += p[d]; nout++; }
                }
                for (int d = 0; d < 3; d++) g[0][d] = cout[d] / nout - cin[d] / nin;
                segs[0][0] = fe[0];
                segs[0][1] = fe[1];
                nseg = 1;
            } else if (nfe == 4) {
                double ctr[3] = {0.5, 0.5, 0.5};
                ctr[fa] = side;
                for (int i = 0; i < 4; i++) {
                    int k = fc[i];
                    if (!((cs >> k) & 1)) continue;
                    int pk[3], m = 0, pair[2];
                    corner_xyz(k, pk);
                    for (int j = 0; j < 4; j++) {
                        int k0, k1;
                        edge_corners(fe[j], &k0, &k1);
                        if (k0 == k || k1 == k) pair[m++] = fe[j];
                    }
                    if (m != 2) return -1;
                    for (int d = 0; d < 3; d++) g[nseg][d] = ctr[d] - pk[d];
                    segs[nseg][0] = pair[0];
                    segs[nseg][1] = pair[1];
                    nseg++;
                }
                if (nseg != 2) return -1;
            } else if (nfe != 0) {
                return -1;
            }
            for (int s = 0; s < nseg; s++) {
                double d[3], m0[3], m1[3];
                cross3(g[s], nF, d);
                edge_mid(segs[s][0], m0);
                edge_mid(segs[s][1], m1);
                double dot = 0;
                for (int i = 0; i < 3; i++) dot += (m1[i] - m0[i]) * d[i];
                int from = dot > 0 ? segs[s][0] : segs[s][1];
                int to = dot > 0 ? segs[s][1] : segs[s][0];
                if (dot == 0 || next[from] != -1) return -1;
                next[from] = to;
            }
        }
    /* chain the directed segments into polygons and fan-triangulate */
    int used[12] = {0}, nt = 0;
    for (int e = 0; e < 12; e++) {
        if (!crossing[e] || used[e]) continue;
        if (next[e] < 0) return -1;
        int poly[12], np = 0, cur = e;
        do {
            if (used[cur] || np >= 12 || next[cur] < 0) return -1;
            used[cur] = 1;
            poly[np++] = cur;
            cur = next[cur];
        } while (cur != e);
        /* fan apex: the first vertex (from the smallest edge id on) none of
         * whose diagonals lies in a cube face; such a diagonal could also be
         * produced by the neighbouring cell and pinch the surface there */
        int apex = -1;
        for (int a = 0; a < np && apex < 0; a++) {
            int ok = 1;
            for (int i = 2; i + 1 < np && ok; i++)
                if (edges_share_face(poly[a], poly[(a + i) % np])) ok = 0;
            if (ok) apex = a;
        }
        if (apex < 0) return -1;
        for (int i = 1; i + 1 < np; i++) {
            tri_out[3 * nt + 0] = poly[apex];
            tri_out[3 * nt + 1] = poly[(apex + i) % np];
            tri_out[3 * nt + 2] = poly[(apex + i + 1) % np];
            nt++;
        }
    }
    return nt;
}

void oracle_mc_tables(int32_t *num_tris, int32_t *tris, int32_t *edge_mask) {
    for (int cs = 0; cs < 256; cs++) {
        int t[3 * 12];
        int nt = gen_case(cs, t);
        if (nt < 0 || nt > 5) {
            fprintf(stderr, "oracle: MC table generation failed for case %d\n", cs);
            abort();
        }
        num_tris[cs] = nt;
        for (int i = 0; i < 16; i++) tris[cs * 16 + i] = (i < 3 * nt) ? t[i] : -1;
        int mask = 0;
        for (int e = 0; e < 12; e++) {
            int k0, k1;
            edge_corners(e, &k0, &k1);
            if (((cs >> k0) & 1) != ((cs >> k1) & 1)) mask |= 1 << e;
        }
        edge_mask[cs] = mask;
    }
}

/* ======================================================================= */
/* plain marching cubes over the decoded field (Sec. 3.3.3, Sec. 4.4-4.5)  */
/* ======================================================================= */

typedef struct {
    const float *blocks;
    uint32_t nx, ny, nz, nbx, nby;
} field_t;

static float sample(const field_t *F, uint32_t x, uint32_t y, uint32_t z) {
    uint64_t b = (x >> 2) + (uint64_t)F->nbx * ((y >> 2) + (uint64_t)F->nby * (z >> 2));
    return F->blocks[b * 64 + (x & 3) + 4 * (y & 3) + 16 * (z & 3)];
}

static int tables_ready = 0;
static int32_t T_num[256], T_tri[256 * 16], T_mask[256];
static void ensure_tables(void) {
    if (!tables_ready) {
        oracle_mc_tables(T_num, T_tri, T_mask);
        tables_ready = 1;
    }
}

static int cell_case(const field_t *F, uint32_t x, uint32_t y, uint32_t z, float iso,
                     float v[8]) {
    int cs = 0;
    for (int k = 0; k < 8; k++) {
        v[k] = sample(F, x + (k & 1), y + ((k >> 1) & 1), z + ((k >> 2) & 1));
        if (v[k] < iso) cs |= 1 << k;
    }
    return cs;
}

/* Visit the non-trivial cells in canonical order: blocks by ascending id,
 * cells by ascending local index lx + 4ly + 16lz. */
typedef void (*cell_fn)(void *ctx, uint64_t b, int l, uint32_t x, uint32_t y,
                        uint32_t z, int cs, const float v[8]);

static void for_each_cell(const field_t *F, float iso, cell_fn fn, void *ctx) {
    uint32_t nbz = ceil4(F->nz);
    for (uint32_t bz = 0; bz < nbz; bz++)
        for (uint32_t by = 0; by < F->nby; by++)
            for (uint32_t bx = 0; bx < F->nbx; bx++) {
                uint64_t b = bx + (uint64_t)F->nbx * (by + (uint64_t)F->nby * bz);
                for (int l = 0; l < 64; l++) {
                    uint32_t x = 4 * bx + (l & 3), y = 4 * by + ((l >> 2) & 3),
                             z = 4 * bz + (l >> 4);
                    if (x + 1 >= F->nx || y + 1 >= F->ny || z + 1 >= F->nz) continue;
                    float v[8];
                    int cs = cell_case(F, x, y, z, iso, v);
                    if (T_num[cs] == 0) continue;
                    fn(ctx, b, l, x, y, z, cs, v);
                }
            }
}

typedef struct {
    const field_t *F;
    float iso;
    double *verts;
    float *verts32;
    uint32_t *vblock;
    int64_t *vedge;
    uint64_t *cell_keys;
    uint8_t *cases;
    uint64_t nv, nc;
    uint64_t *edge8;
    uint64_t *q10;
} emit_ctx;

/* Sec. 4.5: a block-relative coordinate (in [0, 4]) stored in 10 bits.
 * Reading: the 1024 codes span [0, 4] evenly (code q stands for q * 4/1023)
 * and the coordinate goes to its nearest code, computed in float32 as
 * trunc(x * 1023/4 + 1/2). */
static uint32_t quantise10(float x) {
    float scaled = x * (1023.0f / 4.0f);
    uint32_t q = (uint32_t)(scaled + 0.5f);
    return q > 1023u ? 1023u : q;
}

static void emit_cell(void *vctx, uint64_t b, int l, uint32_t x, uint32_t y,
                      uint32_t z, int cs, const float v[8]) {
    emit_ctx *c = (emit_ctx *)vctx;
    if (c->cell_keys) c->cell_keys[c->nc] = b * 64 + (uint64_t)l;
    if (c->cases) c->cases[c->nc] = (uint8_t)cs;
    c->nc++;
    uint32_t ox = x & ~3u, oy = y & ~3u, oz = z & ~3u; /* block origin */
    for (int j = 0; j < 3 * T_num[cs]; j++) {
        int e = T_tri[cs * 16 + j], k0, k1, p0[3];
        edge_corners(e, &k0, &k1);
        corner_xyz(k0, p0);
        int axis = e >> 2;
        uint32_t g[3] = {x + p0[0], y + p0[1], z + p0[2]};
        uint32_t o[3] = {ox, oy, oz};
        float a = v[k0], bv = v[k1];
        if (c->verts) {
            double t = ((double)c->iso - (double)a) / ((double)bv - (double)a);
            for (int d = 0; d < 3; d++)
                c->verts[3 * c->nv + d] = (double)(g[d] - o[d]) + (d == axis ? t : 0.0);
        }
        if (c->verts32) {
            float t = (c->iso - a) / (bv - a);
            for (int d = 0; d < 3; d++) {
                float base = (float)(g[d] - o[d]);
                c->verts32[3 * c->nv + d] = (d == axis) ? base + t : base;
            }
        }
        if (c->edge8) {
            float t = (c->iso - a) / (bv - a);
            uint32_t q = (uint32_t)(t * 4194304.0f);   /* t * 2^22 is exact */
            if (q > 4194303u) q = 4194303u;
            c->edge8[c->nv] = (uint64_t)b | ((uint64_t)l << 32) | ((uint64_t)e << 38) |
                              ((uint64_t)q << 42);
        }
        if (c->q10) {
            /* the float32 vertex as the 16-byte format computes it, then its
             * three coordinates packed x | y << 10 | z << 20 beside the block id */
            float t = (c->iso - a) / (bv - a);
            uint32_t code = 0;
            for (int d = 0; d < 3; d++) {
                float base = (float)(g[d] - o[d]);
                code |= quantise10(d == axis ? base + t : base) << (10 * d);
            }
            c->q10[c->nv] = (uint64_t)code | ((uint64_t)b << 32);
        }
        if (c->vblock) c->vblock[c->nv] = (uint32_t)b;
        if (c->vedge)
            c->vedge[c->nv] = (int64_t)(g[0] + (uint64_t)c->F->nx *
                                        (g[1] + (uint64_t)c->F->ny * g[2])) * 3 + axis;
        c->nv++;
    }
}

static void count_cell(void *vctx, uint64_t b, int l, uint32_t x, uint32_t y,
                       uint32_t z, int cs, const float v[8]) {
    (void)b; (void)l; (void)x; (void)y; (void)z; (void)v;
    uint64_t *n = (uint64_t *)vctx;
    n[0] += (uint64_t)T_num[cs];
    n[1] += 1;
}

uint64_t oracle_mc_extract(const float *blocks, uint32_t nx, uint32_t ny,
                           uint32_t nz, float iso, double *verts,
                           uint32_t *vblock, int64_t *vedge, uint64_t *cell_keys,
                           uint8_t *cases, uint64_t *n_cells) {
    ensure_tables();
    field_t F = {blocks, nx, ny, nz, ceil4(nx), ceil4(ny)};
    if (!verts && !vblock && !vedge && !cell_keys && !cases) {
        uint64_t n[2] = {0, 0};
        for_each_cell(&F, iso, count_cell, n);
        if (n_cells) *n_cells = n[1];
        return n[0];
    }
    emit_ctx c = {&F, iso, verts, NULL, vblock, vedge, cell_keys, cases, 0, 0, NULL, NULL};
    for_each_cell(&F, iso, emit_cell, &c);
    if (n_cells) *n_cells = c.nc;
    return c.nv / 3;
}

uint64_t oracle_mc_extract_f32(const float *blocks, uint32_t nx, uint32_t ny,
                               uint32_t nz, float iso, float *verts,
                               uint32_t *vblock) {
    ensure_tables();
    field_t F = {blocks, nx, ny, nz, ceil4(nx), ceil4(ny)};
    emit_ctx c = {&F, iso, NULL, verts, vblock, NULL, NULL, NULL, 0, 0, NULL, NULL};
    for_each_cell(&F, iso, emit_cell, &c);
    return c.nv / 3;
}

uint64_t oracle_mc_extract_edge8(const float *blocks, uint32_t nx, uint32_t ny,
                                 uint32_t nz, float iso, uint64_t *records) {
    ensure_tables();
    field_t F = {blocks, nx, ny, nz, ceil4(nx), ceil4(ny)};
    emit_ctx c = {&F, iso, NULL, NULL, NULL, NULL, NULL, NULL, 0, 0, records, NULL};
    for_each_cell(&F, iso, emit_cell, &c);
    return c.nv / 3;
}

uint64_t oracle_mc_extract_q10(const float *blocks, uint32_t nx, uint32_t ny,
                               uint32_t nz, float iso, uint64_t *records) {
    ensure_tables();
    field_t F = {blocks, nx, ny, nz, ceil4(nx), ceil4(ny)};
    emit_ctx c = {&F, iso, NULL, NULL, NULL, NULL, NULL, NULL, 0, 0, NULL, records};
    for_each_cell(&F, iso, emit_cell, &c);
    return c.nv / 3;
}

uint64_t oracle_mc_extract_dense(const float *field, uint32_t nx, uint32_t ny,
                                 uint32_t nz, float iso, float *verts,
                                 uint32_t *vblock) {
    /* plain marching cubes over the dense field, cells in z, y, x order (the
     * order of a global scan over the volume), float32 vertices relative to
     * the origin of the 4^3 block holding the cell's lowest corner */
    ensure_tables();
    uint32_t nbx = ceil4(nx), nby = ceil4(ny);
    uint64_t nv = 0;
    for (uint32_t z = 0; z + 1 < nz; z++)
        for (uint32_t y = 0; y + 1 < ny; y++)
            for (uint32_t x = 0; x + 1 < nx; x++) {
                float v[8];
                int cs = 0;
                for (int k = 0; k < 8; k++) {
                    uint64_t idx = (x + (k & 1)) +
                                   (uint64_t)nx * ((y + ((k >> 1) & 1)) +
                                                   (uint64_t)ny * (z + ((k >> 2) & 1)));
                    v[k] = field[idx];
                    if (v[k] < iso) cs |= 1 << k;
                }
                uint32_t b = (x >> 2) + nbx * ((y >> 2) + nby * (z >> 2));
                uint32_t local[3] = {x & 3u, y & 3u, z & 3u};
                for (int j = 0; j < 3 * T_num[cs]; j++, nv++) {
                    int e = T_tri[cs * 16 + j], k0, k1, p0[3];
                    edge_corners(e, &k0, &k1);
                    corner_xyz(k0, p0);
                    int axis = e >> 2;
                    if (verts) {
                        float t = (iso - v[k0]) / (v[k1] - v[k0]);
                        for (int d = 0; d < 3; d++) {
                            float base = (float)(local[d] + (uint32_t)p0[d]);
                            verts[3 * nv + d] = d == axis ? base + t : base;
                        }
                    }
                    if (vblock) vblock[nv] = b;
                }
            }
    return nv / 3;
}

uint64_t oracle_brute_count(const float *field, uint32_t nx, uint32_t ny,
                            uint32_t nz, float iso) {
    ensure_tables();
    uint64_t T = 0;
    for (uint32_t z = 0; z + 1 < nz; z++)
        for (uint32_t y = 0; y + 1 < ny; y++)
            for (uint32_t x = 0; x + 1 < nx; x++) {
                int cs = 0;
                for (int k = 0; k < 8; k++) {
                    uint64_t idx = (x + (k & 1)) +
                                   (uint64_t)nx * ((y + ((k >> 1) & 1)) +
                                                   (uint64_t)ny * (z + ((k >> 2) & 1)));
                    if (field[idx] < iso) cs |= 1 << k;
                }
                T += (uint64_t)T_num[cs];
            }
    return T;
}

uint64_t oracle_brute_count_blocks(const float *blocks, uint32_t nx, uint32_t ny,
                                   uint32_t nz, float iso) {
    ensure_tables();
    field_t F = {blocks, nx, ny, nz, ceil4(nx), ceil4(ny)};
    uint64_t T = 0;
    for (uint32_t z = 0; z + 1 < nz; z++)
        for (uint32_t y = 0; y + 1 < ny; y++)
            for (uint32_t x = 0; x + 1 < nx; x++) {
                float v[8];
                T += (uint64_t)T_num[cell_case(&F, x, y, z, iso, v)];
            }
    return T;
}

void oracle_block_vertex_counts(const float *blocks, uint32_t nx, uint32_t ny,
                                uint32_t nz, float iso, const uint32_t *ids,
                                uint64_t n, uint32_t *counts) {
    ensure_tables();
    field_t F = {blocks, nx, ny, nz, ceil4(nx), ceil4(ny)};
    for (uint64_t i = 0; i < n; i++) {
        uint64_t b = ids[i];
        uint32_t bx = (uint32_t)(b % F.nbx), by = (uint32_t)((b / F.nbx) % F.nby),
                 bz = (uint32_t)(b / ((uint64_t)F.nbx * F.nby));
        uint32_t cnt = 0;
        for (int l = 0; l < 64; l++) {
            uint32_t x = 4 * bx + (l & 3), y = 4 * by + ((l >> 2) & 3), z = 4 * bz + (l >> 4);
            if (x + 1 >= nx || y + 1 >= ny || z + 1 >= nz) continue;
            float v[8];
            cnt += 3u * (uint32_t)T_num[cell_case(&F, x, y, z, iso, v)];
        }
        counts[i] = cnt;
    }
}

/* ======================================================================= */
/* GPU-driven LRU block cache, serial form of Alg. 1 (Sec. 4.2)            */
/* ======================================================================= */
/*
 * Readings where the paper is silent: slots created empty get the "high age"
 * 2^31; ages saturate at 2^32-1; the cache grows by
 * max(n_new - n_avail, ceil(n_slots/2)) slots, capped at max_slots; the sort
 * of available slots by descending age breaks ties by ascending slot id.
 */
#define HIGH_AGE 0x80000000u

struct oracle_lru {
    uint64_t n_blocks, n_slots, initial, max_slots;
    int32_t *I_slot;   /* per block: slot or -1 */
    int32_t *S_block;  /* per slot: block or -1 */
    uint32_t *S_age;
    uint8_t *M_avail;
};

static void lru_reset(oracle_lru *c) {
    for (uint64_t b = 0; b < c->n_blocks; b++) c->I_slot[b] = -1;
    c->n_slots = c->initial;
    for (uint64_t s = 0; s < c->max_slots; s++) {
        c->S_block[s] = -1;
        c->S_age[s] = HIGH_AGE;
        c->M_avail[s] = 1;
    }
}

oracle_lru *oracle_lru_create(uint64_t n_blocks, uint64_t initial, uint64_t max_slots) {
    if (max_slots < initial) max_slots = initial;
    oracle_lru *c = (oracle_lru *)calloc(1, sizeof(oracle_lru));
    c->n_blocks = n_blocks;
    c->initial = initial;
    c->max_slots = max_slots;
    c->I_slot = (int32_t *)malloc(sizeof(int32_t) * (n_blocks ? n_blocks : 1));
    c->S_block = (int32_t *)malloc(sizeof(int32_t) * (max_slots ? max_slots : 1));
    c->S_age = (uint32_t *)malloc(sizeof(uint32_t) * (max_slots ? max_slots : 1));
    c->M_avail = (uint8_t *)malloc(max_slots ? max_slots : 1);
    lru_reset(c);
    return c;
}

void oracle_lru_free(oracle_lru *c) {
    if (!c) return;
    free(c->I_slot);
    free(c->S_block);
    free(c->S_age);
    free(c->M_avail);
    free(c);
}

uint64_t oracle_lru_n_slots(const oracle_lru *c) { return c->n_slots; }

void oracle_lru_state(const oracle_lru *c, int32_t *I_slot, int32_t *S_block,
                      uint32_t *S_age) {
    if (I_slot) memcpy(I_slot, c->I_slot, sizeof(int32_t) * c->n_blocks);
    if (S_block) memcpy(S_block, c->S_block, sizeof(int32_t) * c->n_slots);
    if (S_age) memcpy(S_age, c->S_age, sizeof(uint32_t) * c->n_slots);
}

typedef struct { uint32_t age, slot; } age_slot;
static int by_age_desc(const void *pa, const void *pb) {
    const age_slot *a = (const age_slot *)pa, *b = (const age_slot *)pb;
    if (a->age != b->age) return a->age > b->age ? -1 : 1;
    return a->slot < b->slot ? -1 : (a->slot > b->slot);
}

int oracle_lru_update(oracle_lru *c, const uint8_t *active, uint32_t *I_new_out,
                      uint64_t *n_new_out, uint64_t *n_evicted_out) {
    /* IncrementSlotAge */
    for (uint64_t s = 0; s < c->n_slots; s++)
        if (c->S_age[s] != 0xFFFFFFFFu) c->S_age[s]++;
    /* MarkNewBlocks */
    uint8_t *M_new = (uint8_t *)calloc(c->n_blocks ? c->n_blocks : 1, 1);
    for (uint64_t b = 0; b < c->n_blocks; b++) {
        int32_t s = c->I_slot[b];
        if (active[b] && s != -1) {
            c->S_age[s] = 0;
            c->M_avail[s] = 0;
            M_new[b] = 0;
        } else if (active[b]) {
            M_new[b] = 1;
        } else if (s != -1) {
            c->M_avail[s] = 1;
        }
    }
    uint64_t n_new = 0, n_avail = 0, n_evicted = 0;
    for (uint64_t b = 0; b < c->n_blocks; b++) n_new += M_new[b];
    if (n_new_out) *n_new_out = n_new;
    if (n_evicted_out) *n_evicted_out = 0;
    if (n_new == 0) {
        free(M_new);
        return 0;
    }
    for (uint64_t s = 0; s < c->n_slots; s++) n_avail += c->M_avail[s];
    if (n_new > n_avail) {
        /* grow: new slots are empty, available and get the high age */
        uint64_t grow = n_new - n_avail;
        uint64_t half = (c->n_slots + 1) / 2;
        if (half > grow) grow = half;
        if (c->n_slots + grow > c->max_slots) grow = c->max_slots - c->n_slots;
        for (uint64_t s = c->n_slots; s < c->n_slots + grow; s++) {
            c->S_block[s] = -1;
            c->S_age[s] = HIGH_AGE;
            c->M_avail[s] = 1;
        }
        c->n_slots += grow;
        n_avail += grow;
        if (n_new > n_avail) {
            lru_reset(c);
            free(M_new);
            return -3;
        }
    }
    /* I_new ascending; I_avail ascending, then sorted by age (descending) */
    uint32_t *I_new = (uint32_t *)malloc(sizeof(uint32_t) * n_new);
    uint64_t j = 0;
    for (uint64_t b = 0; b < c->n_blocks; b++)
        if (M_new[b]) I_new[j++] = (uint32_t)b;
    age_slot *avail = (age_slot *)malloc(sizeof(age_slot) * n_avail);
    j = 0;
    for (uint64_t s = 0; s < c->n_slots; s++)
        if (c->M_avail[s]) {
            avail[j].age = c->S_age[s];
            avail[j].slot = (uint32_t)s;
            j++;
        }
    qsort(avail, n_avail, sizeof(age_slot), by_age_desc);
    /* AssignSlots: evict the previous owner, install the new block */
    for (uint64_t i = 0; i < n_new; i++) {
        uint32_t s = avail[i].slot;
        if (c->S_block[s] != -1) {
            c->I_slot[c->S_block[s]] = -1;
            n_evicted++;
        }
        c->S_block[s] = (int32_t)I_new[i];
        c->I_slot[I_new[i]] = (int32_t)s;
        c->M_avail[s] = 0;
        c->S_age[s] = 0;
    }
    if (I_new_out) memcpy(I_new_out, I_new, sizeof(uint32_t) * n_new);
    if (n_evicted_out) *n_evicted_out = n_evicted;
    free(I_new);
    free(avail);
    free(M_new);
    return 0;
}

void oracle_lru_idle(oracle_lru *c, uint64_t k) {
    /* k calls of Alg. 1 at which no block is active: each increments every
     * slot's age (saturating) and marks every cached block available, and
     * none has a new block, so the update stops there */
    for (uint64_t s = 0; s < c->n_slots; s++) {
        uint64_t a = (uint64_t)c->S_age[s] + k;
        c->S_age[s] = a > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)a;
        if (c->S_block[s] != -1) c->M_avail[s] = 1;
    }
}

/* ======================================================================= */
/* gradient through t = (iso - a) / (b - a), topology fixed (FP64)         */
/* ======================================================================= */

/* Neumaier compensated accumulation. */
static void acc_add(double *sum, double *comp, double v) {
    double t = *sum + v;
    if (fabs(*sum) >= fabs(v)) *comp += (*sum - t) + v;
    else *comp += (v - t) + *sum;
    *sum = t;
}

double oracle_sphere_loss(const double *vg, uint64_t n, const double *c, double R,
                          double *gV) {
    double L = 0, comp = 0;
    for (uint64_t j = 0; j < n; j++) {
        double d[3] = {vg[3 * j] - c[0], vg[3 * j + 1] - c[1], vg[3 * j + 2] - c[2]};
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        acc_add(&L, &comp, (r - R) * (r - R));
        if (gV)
            for (int k = 0; k < 3; k++) gV[3 * j + k] = r > 0 ? 2.0 * (r - R) * d[k] / r : 0.0;
    }
    return L + comp;
}

typedef struct {
    const field_t *F;
    float iso;
    const double *gV;
    double *g, *gc; /* dfield and its compensation */
    double di, dic;
    uint64_t nv;
} back_ctx;

static uint64_t block_index_of(const field_t *F, uint32_t x, uint32_t y, uint32_t z) {
    uint64_t b = (x >> 2) + (uint64_t)F->nbx * ((y >> 2) + (uint64_t)F->nby * (z >> 2));
    return b * 64 + (x & 3) + 4 * (y & 3) + 16 * (z & 3);
}

static void back_cell(void *vctx, uint64_t b, int l, uint32_t x, uint32_t y,
                      uint32_t z, int cs, const float v[8]) {
    (void)b; (void)l;
    back_ctx *c = (back_ctx *)vctx;
    for (int j = 0; j < 3 * T_num[cs]; j++) {
        int e = T_tri[cs * 16 + j], k0, k1, p0[3], p1[3];
        edge_corners(e, &k0, &k1);
        corner_xyz(k0, p0);
        corner_xyz(k1, p1);
        int axis = e >> 2;
        double a = v[k0], bv = v[k1], iso = c->iso;
        double t = (iso - a) / (bv - a);
        double gt = c->gV[3 * c->nv + axis]; /* dv/dt = e_axis */
        uint64_t ia = block_index_of(c->F, x + p0[0], y + p0[1], z + p0[2]);
        uint64_t ib = block_index_of(c->F, x + p1[0], y + p1[1], z + p1[2]);
        acc_add(&c->g[ia], &c->gc[ia], gt * (t - 1.0) / (bv - a));
        acc_add(&c->g[ib], &c->gc[ib], gt * (-t) / (bv - a));
        acc_add(&c->di, &c->dic, gt / (bv - a));
        c->nv++;
    }
}

void oracle_mc_backward(const float *blocks, uint32_t nx, uint32_t ny, uint32_t nz,
                        float iso, const double *gV, double *dfield, double *diso) {
    ensure_tables();
    field_t F = {blocks, nx, ny, nz, ceil4(nx), ceil4(ny)};
    uint64_t n = oracle_num_blocks(nx, ny, nz) * 64;
    double *comp = (double *)calloc(n, sizeof(double));
    memset(dfield, 0, sizeof(double) * n);
    back_ctx c = {&F, iso, gV, dfield, comp, 0, 0, 0};
    for_each_cell(&F, iso, back_cell, &c);
    for (uint64_t i = 0; i < n; i++) dfield[i] += comp[i];
    *diso = c.di + c.dic;
    free(comp);
}

typedef struct {
    const field_t *F;
    const double *fd;
    double iso;
    const double *c;
    double R, L, comp;
} fdloss_ctx;

static void fdloss_cell(void *vctx, uint64_t b, int l, uint32_t x, uint32_t y,
                        uint32_t z, int cs, const float v[8]) {
    (void)b; (void)l; (void)v;
    fdloss_ctx *c = (fdloss_ctx *)vctx;
    for (int j = 0; j < 3 * T_num[cs]; j++) {
        int e = T_tri[cs * 16 + j], k0, k1, p0[3], p1[3];
        edge_corners(e, &k0, &k1);
        corner_xyz(k0, p0);
        corner_xyz(k1, p1);
        int axis = e >> 2;
        double a = c->fd[block_index_of(c->F, x + p0[0], y + p0[1], z + p0[2])];
        double bv = c->fd[block_index_of(c->F, x + p1[0], y + p1[1], z + p1[2])];
        double t = (c->iso - a) / (bv - a);
        double g[3] = {(double)(x + p0[0]), (double)(y + p0[1]), (double)(z + p0[2])};
        g[axis] += t;
        double d[3] = {g[0] - c->c[0], g[1] - c->c[1], g[2] - c->c[2]};
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        acc_add(&c->L, &c->comp, (r - c->R) * (r - c->R));
    }
}

double oracle_sphere_loss_fixed_topology(const double *field_blocks,
                                         const float *blocks_case, uint32_t nx,
                                         uint32_t ny, uint32_t nz, float iso_case,
                                         double iso, const double *c, double R) {
    ensure_tables();
    field_t F = {blocks_case, nx, ny, nz, ceil4(nx), ceil4(ny)};
    fdloss_ctx ctx = {&F, field_blocks, iso, c, R, 0, 0};
    for_each_cell(&F, iso_case, fdloss_cell, &ctx);
    return ctx.L + ctx.comp;
}
