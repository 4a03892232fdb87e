/*
 * CPU oracle for block-compressed isosurface extraction.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, single-threaded, deliberately slow C that
 * defines what the GPU library must compute.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg load it; the product path never
 * does.  It shares no code, header, table or generator with the GPU library.
 *
 * Conventions (all arrays are owned by the caller):
 *   - fields are [nz][ny][nx] with x fastest;
 *   - blocks are 4x4x4; block id b = bx + nbx*(by + nby*bz), nbx = ceil(nx / 4) etc.;
 *   - inside a block, sample (lx,ly,lz) is at index lx + 4*ly + 16*lz;
 *   - a compressed block is 64*rate bits = rate little-endian u64 words and
 *     block b starts at word b*rate (fixed-rate ZFP, Sec. 3.3.4 / Sec. 4).
 *
 * Functions whose result no independent pin covers are marked
 * "parity unpinned" where they are defined.
 */
#ifndef BCMC_ORACLE_H
#define BCMC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- geometry ---------------------------------------------------------- */
uint64_t oracle_num_blocks(uint32_t nx, uint32_t ny, uint32_t nz);

/* ---- ZFP fixed-rate codec (Sec. 3.3.4, Sec. 4.2.1; Lindstrom 2014) ----- */
/* is_f64: 0 = float32 stream (P = 32), 1 = float64 stream (P = 64).
 * Returns 0, or -1 on invalid arguments, -6 on a non-finite input value. */
int oracle_zfp_encode(const void *field, int is_f64, uint32_t nx, uint32_t ny,
                      uint32_t nz, uint32_t rate, uint64_t *stream);
/* Decode every block into blocks[N_b][64] as float32 (f64 streams are decoded
 * in double and rounded to nearest float). */
int oracle_zfp_decode(const uint64_t *stream, int is_f64, uint32_t nx,
                      uint32_t ny, uint32_t nz, uint32_t rate, float *blocks);
/* Decode every block of a float64 stream into double blocks[N_b][64]. */
int oracle_zfp_decode_f64(const uint64_t *stream, uint32_t nx, uint32_t ny,
                          uint32_t nz, uint32_t rate, double *blocks);
/* Decode a list of blocks only (blocks[i][64] for block ids ids[i]). */
int oracle_zfp_decode_some(const uint64_t *stream, int is_f64, uint32_t rate,
                           const uint32_t *ids, uint64_t n, float *blocks);

/* Codec pieces exposed for the pin tests. v points to 4 (or 64) integers. */
void oracle_fwd_lift(int64_t *v, int is_f64);
void oracle_inv_lift(int64_t *v, int is_f64);
void oracle_sequency_order(int *perm);              /* perm[r] = block index */
uint64_t oracle_to_negabinary(int64_t i, int is_f64);
int64_t oracle_from_negabinary(uint64_t u, int is_f64);
/* Embedded coding of 64 already-negabinary coefficients into maxbits bits at
 * bit offset 0 of words[] (which must be zeroed); returns bits used. */
uint64_t oracle_encode_planes(const uint64_t *u, int is_f64, uint64_t maxbits,
                              uint64_t *words);
void oracle_decode_planes(const uint64_t *words, int is_f64, uint64_t maxbits,
                          uint64_t *u);

/* ---- value ranges and active blocks (Sec. 4.1) ------------------------- */
/* ranges[2*b] = min, ranges[2*b+1] = max over the valid samples of block b. */
void oracle_block_ranges(const float *blocks, uint32_t nx, uint32_t ny,
                         uint32_t nz, float *ranges);
/* active[b] = 1 iff block b is active for iso; returns the number active. */
uint64_t oracle_active_blocks(const float *ranges, uint32_t nx, uint32_t ny,
                              uint32_t nz, float iso, uint8_t *active);

/* ---- marching cubes tables (generated, Sec. 3.3.3) --------------------- */
/* num_tris[256], tris[256*16] (edge ids, -1 padded), edge_mask[256]. */
void oracle_mc_tables(int32_t *num_tris, int32_t *tris, int32_t *edge_mask);

/* ---- plain marching cubes over the whole decoded field ----------------- */
/* Number of triangles (two-pass: call with verts NULL to count).  verts are
 * block-local double (x,y,z) triples, vblock the owning block id, vedge the
 * global edge key (p0 sample index * 3 + axis), cell_keys/cases the
 * non-trivial cells in canonical order (block*64 + local).  Any output
 * pointer may be NULL. */
uint64_t oracle_mc_extract(const float *blocks, uint32_t nx, uint32_t ny,
                           uint32_t nz, float iso, double *verts,
                           uint32_t *vblock, int64_t *vedge, uint64_t *cell_keys,
                           uint8_t *cases, uint64_t *n_cells);
/* Same with the interpolation done in float32 in the order
 * t = (iso - a) / (b - a), x = (float)p0 + t. */
uint64_t oracle_mc_extract_f32(const float *blocks, uint32_t nx, uint32_t ny,
                               uint32_t nz, float iso, float *verts,
                               uint32_t *vblock);
/* The same soup with each vertex as one 64-bit edge record: block id (bits
 * 0-31), cell l = lx + 4 ly + 16 lz inside the block (32-37), edge id of the
 * table (38-41), and q = min(trunc(t * 2^22), 2^22 - 1) (42-63) with the
 * float32 t = (iso - a) / (b - a) measured from the edge's first corner. */
uint64_t oracle_mc_extract_edge8(const float *blocks, uint32_t nx, uint32_t ny,
                                 uint32_t nz, float iso, uint64_t *records);
/* The same soup in Sec. 4.5's 8-byte vertex: the float32 vertex (as in
 * oracle_mc_extract_f32) with each block-relative coordinate rounded to the
 * nearest of 1024 even steps over [0, 4] (code q = trunc(x * 1023/4 + 1/2)
 * in float32), packed x | y << 10 | z << 20 in the low 32 bits, block id in
 * the high 32 bits. */
uint64_t oracle_mc_extract_q10(const float *blocks, uint32_t nx, uint32_t ny,
                               uint32_t nz, float iso, uint64_t *records);
/* Plain marching cubes over a dense [nz][ny][nx] field with the cells in
 * global z, y, x order (the dense baseline's order): float32 block-relative
 * vertices as oracle_mc_extract_f32 computes them, with their block ids.
 * Returns T; outputs may be NULL. */
uint64_t oracle_mc_extract_dense(const float *field, uint32_t nx, uint32_t ny,
                                 uint32_t nz, float iso, float *verts,
                                 uint32_t *vblock);
/* Brute force: sum over every valid cell of the number of triangles of its
 * case, visiting the dense field in z,y,x order (no blocks). */
uint64_t oracle_brute_count(const float *field, uint32_t nx, uint32_t ny,
                            uint32_t nz, float iso);
/* Same, with the field given in block layout. */
uint64_t oracle_brute_count_blocks(const float *blocks, uint32_t nx,
                                   uint32_t ny, uint32_t nz, float iso);
/* Per-block vertex counts for the given block ids (3 * triangles each). */
void oracle_block_vertex_counts(const float *blocks, uint32_t nx, uint32_t ny,
                                uint32_t nz, float iso, const uint32_t *ids,
                                uint64_t n, uint32_t *counts);

/* ---- GPU-driven LRU cache (Sec. 4.2, Alg. 1), serial simulator --------- */
typedef struct oracle_lru oracle_lru;
oracle_lru *oracle_lru_create(uint64_t n_blocks, uint64_t initial_slots,
                              uint64_t max_slots);
void oracle_lru_free(oracle_lru *c);
/* One cache update for the active mask.  Outputs (optional): I_new[n_new]
 * (ascending block ids).  Returns 0, or -3 when max_slots cannot hold the
 * active set (the cache is then reset to its initial empty state). */
int oracle_lru_update(oracle_lru *c, const uint8_t *active, uint32_t *I_new,
                      uint64_t *n_new, uint64_t *n_evicted);
/* k updates at which no block is active, at once (ages += k, saturating). */
void oracle_lru_idle(oracle_lru *c, uint64_t k);
uint64_t oracle_lru_n_slots(const oracle_lru *c);
/* Copies of the state: I_slot[n_blocks], S_block[n_slots], S_age[n_slots]. */
void oracle_lru_state(const oracle_lru *c, int32_t *I_slot, int32_t *S_block,
                      uint32_t *S_age);

/* ---- gradient through the edge interpolation (FP64) -------------------- */
/* L = sum_j (|v_j - c| - R)^2 over global vertex positions; gV[3T] = dL/dv. */
double oracle_sphere_loss(const double *verts_global, uint64_t n_verts,
                          const double *c, double R, double *gV);
/* dL/dfield (block layout, double[N_b*64]) and dL/diso from dL/dv of every
 * soup vertex, topology held fixed.  Compensated summation. */
void oracle_mc_backward(const float *blocks, uint32_t nx, uint32_t ny,
                        uint32_t nz, float iso, const double *gV,
                        double *dfield, double *diso);
/* L evaluated with iso and the field given in double (for finite
 * differences); the case of every cell is taken from (blocks, iso_case). */
double oracle_sphere_loss_fixed_topology(const double *field_blocks,
                                         const float *blocks_case,
                                         uint32_t nx, uint32_t ny, uint32_t nz,
                                         float iso_case, double iso,
                                         const double *c, double R);

#ifdef __cplusplus
}
#endif
#endif
