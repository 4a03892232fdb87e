/*
 * bcmc -- block-compressed marching cubes on MI355X (gfx950).
 *
 * C ABI of libbcmc.so.  Implements the GPU-driven isosurface extraction from
 * block-compressed volumes of Usher & Pascucci, "Interactive Visualization of
 * Terascale Data in the Browser: Fact or Fiction?" (arXiv 2009.03254), Sec. 4:
 * fixed-rate ZFP data uploaded once (Sec. 4 intro), active-block culling
 * (Sec. 4.1), a GPU-driven LRU cache of decoded blocks (Sec. 4.2, Alg. 1) fed
 * by on-demand block decoding (Sec. 4.2.1), and block-wise marching cubes
 * with halo loads, per-block vertex counts and a triangle-soup output
 * (Sec. 4.3-4.5).
 *
 * Conventions
 *  - Volumes are nx*ny*nz samples, x fastest; blocks are 4x4x4 samples,
 *    nbx = ceil(nx/4) etc., block id b = bx + nbx*(by + nby*bz) (the paper's
 *    row-major block ids, Sec. 4.5); inside a block, sample (lx,ly,lz) is
 *    element lx + 4*ly + 16*lz.  Dimensions need not be multiples of 4.
 *  - A compressed volume is fixed-rate ZFP: block b occupies 64*rate bits =
 *    `rate` little-endian u64 words starting at word b*rate.
 *  - Pointers documented as "device" are HIP device pointers (e.g. from
 *    torch); "host" pointers are ordinary memory.  `hip_stream` is a
 *    hipStream_t (NULL = default stream); all GPU work is enqueued on it.
 *  - Every function returns BCMC_OK (0) or a negative bcmc_status; on error
 *    bcmc_last_error() describes it.  No C++ exception crosses the ABI.
 *  - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef BCMC_H
#define BCMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define BCMC_API __attribute__((visibility("default")))
#else
#define BCMC_API
#endif

typedef struct bcmc_volume bcmc_volume;

typedef enum {
    BCMC_OK = 0,
    BCMC_E_INVALID = -1,   /* bad argument, size or state */
    BCMC_E_NOMEM = -2,     /* a device allocation failed; nothing leaked */
    BCMC_E_CACHE_CAP = -3, /* the active blocks do not fit the cache cap; cache reset */
    BCMC_E_CAPACITY = -4,  /* the vertex buffer is too small; *n_triangles is set */
    BCMC_E_HIP = -5,       /* a HIP runtime call failed */
    BCMC_E_NONFINITE = -6  /* input (or decoded) data holds NaN or infinity */
} bcmc_status;

typedef enum { BCMC_F32 = 0, BCMC_F64 = 1 } bcmc_scalar;

/* One triangle-soup vertex: position relative to the origin of its block
 * (4*bx, 4*by, 4*bz) in voxel units, and that block's id.  16 bytes. */
typedef struct {
    float x, y, z;
    uint32_t block;
} bcmc_vertex;

/* Record formats bcmc_extract can write (per volume, bcmc_set_vertex_format).
 * BCMC_VERTEX_Q10 is Sec. 4.5's compressed vertex, 8 bytes: one uint64_t per
 * vertex whose low uint32 packs the block-relative coordinates quantised to
 * 10 bits each (x in bits 0-9, y in 10-19, z in 20-29; q = trunc(c * 255.75
 * + 0.5) in float32 from the 16-byte vertex's coordinate c in [0, 4], so c is
 * q * 4 / 1023 within 2/1023 voxel plus float32 rounding) and whose high
 * uint32 is the block id.
 * BCMC_VERTEX_EDGE8 is this library's own 8-byte record, which keeps the
 * size but names the vertex by its edge, precise to 2^-23 voxel: one
 * uint64_t per vertex,
 *     bits  0-31  block id
 *     bits 32-37  cell l = lx + 4*ly + 16*lz inside the block
 *     bits 38-41  edge id e (axis e>>2; bits 0 and 1 of e offset the first
 *                 corner along the other two axes, in increasing axis order)
 *     bits 42-63  q = min(trunc(t * 2^22), 2^22 - 1), t = (iso - a)/(b - a)
 *                 in float32 from the edge's first corner (value a)
 * so the block-relative position is the first corner plus (q + 0.5) / 2^22
 * along the edge axis, within 2^-23 voxel of the float32 vertex. */
typedef enum {
    BCMC_VERTEX_F32 = 0,   /* bcmc_vertex, 16 bytes (default) */
    BCMC_VERTEX_EDGE8 = 1, /* uint64_t edge record, 8 bytes */
    BCMC_VERTEX_Q10 = 2    /* uint64_t 10-bit quantised vertex (Sec. 4.5), 8 bytes */
} bcmc_vertex_format;

/* Statistics of the last bcmc_extract call (Sec. 4.6, tab:mc_benchmark_data
 * and tab:mc_benchmark_table report the same quantities). */
typedef struct {
    uint64_t n_blocks;     /* blocks in the volume */
    uint64_t n_active;     /* active blocks (Sec. 4.1) */
    uint64_t n_new;        /* blocks decoded into the cache by this call */
    uint64_t n_evicted;    /* blocks evicted by this call */
    uint64_t n_occupied;   /* active blocks that emitted triangles (Sec. 4.4) */
    uint64_t n_candidates; /* active blocks whose 2x2x2 group straddles iso (staged) */
    uint64_t n_slots;      /* cache slots after this call */
    uint64_t n_triangles;
    uint64_t calls;        /* extract calls on this handle */
    uint64_t n_general;    /* new blocks of a low-rate double-precision stream
                              whose bits reach below plane 39, decoded by the
                              general decoder after the low-rate one */
    double hit_rate;       /* 1 - n_new / n_active (1 when nothing is active) */
    double alg_bytes;      /* 8*N_b + n_new*(8*rate+256) + 256*n_active + 24*T */
    double stage_ms[8];    /* for the profiled stages (HIP events on the
                              stream; 0 for stages not profiled):
                              [0] cull + active/new compaction,
                              [1] cache update (slot pass, growth, age sort),
                              [2] assign + decode of new blocks,
                              [3] sign masks + marching cubes count pass,
                              [4] empty (the block offsets are formed by the
                              emission pass from the count pass's per-wave
                              totals), [5] emission pass, [6] unused, [7] total
                              (when stages 0 and 5 are both profiled) */
} bcmc_stats;

/* Upload a fixed-rate ZFP stream to the device once (Sec. 4: the compressed
 * volume lives on the GPU) and decode every block once to record its value
 * range over the valid samples (Sec. 4.1: ranges precomputed at load).
 *   stream, nbytes   compressed words; nbytes must equal N_b * 8 * rate.
 *                    Copied: the caller keeps ownership.
 *   stream_is_device 1 when `stream` is a device pointer, 0 for host memory.
 *   type             BCMC_F32 (rate 1..32) or BCMC_F64 (rate 1..64); f64
 *                    blocks are decoded in double and rounded to float.
 * The cache starts empty and unbounded (see bcmc_set_cache_budget).
 * Errors: BCMC_E_INVALID (sizes), BCMC_E_NONFINITE (a decoded value is not
 * finite), BCMC_E_NOMEM, BCMC_E_HIP. */
BCMC_API int bcmc_load_compressed(const void *stream, uint64_t nbytes, int stream_is_device,
                         uint32_t nx, uint32_t ny, uint32_t nz, int type, uint32_t rate,
                         void *hip_stream, bcmc_volume **out);

/* A volume over already-decoded float blocks ([N_b][64], device, caller-owned
 * and kept alive while the handle exists): every block is resident, slot =
 * block id (no cache, no decoding).  Used by the differentiable extract. */
BCMC_API int bcmc_volume_from_blocks(const float *d_blocks, uint32_t nx, uint32_t ny, uint32_t nz,
                            void *hip_stream, bcmc_volume **out);

/* Point a bcmc_volume_from_blocks handle at new decoded blocks (same dims;
 * device, caller-owned) and recompute the block ranges on hip_stream without
 * synchronising.  Non-finite values are not detected here.
 * Errors: BCMC_E_INVALID (not an identity handle). */
BCMC_API int bcmc_rebind_blocks(bcmc_volume *v, const float *d_blocks, void *hip_stream);

/* Cache budget (Sec. 4.2: user-set initial number of slots, grown on demand).
 * initial_bytes/256 slots exist at the start; growth adds
 * max(n_new - n_avail, ceil(n_slots/2)) slots, never beyond max_bytes/256
 * (max_bytes = 0: one slot per block).  Slot memory for the cap is reserved
 * here so growth needs no host round-trip.  Empties the cache.
 * Errors: BCMC_E_INVALID (max below initial, identity volume), BCMC_E_NOMEM. */
BCMC_API int bcmc_set_cache_budget(bcmc_volume *v, uint64_t initial_bytes, uint64_t max_bytes);

/* Empty the cache (every slot empty, age 2^31), keeping the budget. */
BCMC_API int bcmc_reset_cache(bcmc_volume *v, void *hip_stream);

/* Extract the isosurface at `iso` (Sec. 4.1-4.5) into the caller's device
 * buffer d_out of capacity_vertices records (bcmc_vertex, or uint64_t edge
 * records after bcmc_set_vertex_format(v, BCMC_VERTEX_EDGE8)): a triangle soup,
 * 3 vertices per triangle, in canonical order (blocks by id, cells by local
 * index, triangles and vertices in table order).  A cell corner is inside
 * when its value is < iso.  Synchronises hip_stream once to read the count.
 * Errors: BCMC_E_CAPACITY when 3*T > capacity_vertices (*n_triangles = T,
 * the first capacity_vertices records are written, the cache stays valid:
 * enlarge and call again); BCMC_E_CACHE_CAP (cache reset); BCMC_E_HIP. */
BCMC_API int bcmc_extract(bcmc_volume *v, float iso, void *d_out, uint64_t capacity_vertices,
                 uint64_t *n_triangles, void *hip_stream);

/* Sec. 4.5's 8-byte vertices (BCMC_VERTEX_Q10 records) from n 16-byte
 * bcmc_vertex records: d_vertices (device, n * 16 bytes) -> d_out (device,
 * n uint64_t), on hip_stream, without synchronising; the same records the
 * emission writes in that format.  Errors: BCMC_E_INVALID (null pointers
 * with n > 0). */
BCMC_API int bcmc_vertices_to_q10(const void *d_vertices, uint64_t n, void *d_out,
                                  void *hip_stream);

/* Record format of this volume's bcmc_extract output (bcmc_vertex_format;
 * default BCMC_VERTEX_F32).  The order and count of records do not depend on
 * it; bcmc_backward and the batch API (always bcmc_vertex) are unaffected.
 * Errors: BCMC_E_INVALID for an unknown format. */
BCMC_API int bcmc_set_vertex_format(bcmc_volume *v, int format);

/* Backward of the last bcmc_extract of a bcmc_volume_from_blocks handle
 * (same iso), topology held fixed: from d_gV = dL/d(vertex position)
 * ([3T][3] float, device) accumulates dL/d(field) into d_dfield ([N_b][64]
 * float, device, overwritten) and dL/d(iso) into d_diso (one float, device,
 * overwritten), through t = (iso - a)/(b - a).  Float atomics: the
 * summation order is not fixed, so results vary in the last bits from run
 * to run.  Each block's vertex count is recomputed from the bound field and
 * compared with the forward's; synchronises hip_stream once to read that
 * check.
 * Errors: BCMC_E_INVALID (not an identity handle, no extract, n_verts
 * differs from the last extract, or the field changed since the extract so
 * that some block's vertex count differs: the gradient is then not valid and
 * the extract must be repeated). */
BCMC_API int bcmc_backward(bcmc_volume *v, float iso, const float *d_gV, uint64_t n_verts,
                  float *d_dfield, float *d_diso, void *hip_stream);

BCMC_API int bcmc_get_stats(const bcmc_volume *v, bcmc_stats *out);
/* Nonzero: record HIP events around every stage of bcmc_extract
 * (bcmc_stats.stage_ms); 0: none.  Same as bcmc_set_profiling_stages with
 * BCMC_PROFILE_ALL or 0. */
BCMC_API int bcmc_set_profiling(bcmc_volume *v, int on);
/* Record HIP events only around the stages whose bit is set in stage_mask
 * (bit i = stage_ms[i], i < 6).  Each event costs a few microseconds of
 * stream time, so timing one kernel inside a measured loop profiles only
 * its stage.  Errors: BCMC_E_INVALID (bits above 5), BCMC_E_HIP. */
#define BCMC_PROFILE_ALL 0x3Fu
BCMC_API int bcmc_set_profiling_stages(bcmc_volume *v, uint32_t stage_mask);
BCMC_API void bcmc_free(bcmc_volume *v);
/* Message of the last error on this thread (empty when none). */
BCMC_API const char *bcmc_last_error(void);
BCMC_API uint64_t bcmc_num_blocks(uint32_t nx, uint32_t ny, uint32_t nz);

/* Fixed-rate ZFP compression of a device field ([nz][ny][nx], x fastest)
 * into d_stream (N_b*rate u64 words, device, caller-owned).  Partial blocks
 * replicate the last valid sample.  Errors: BCMC_E_INVALID,
 * BCMC_E_NONFINITE. */
BCMC_API int bcmc_encode(const void *d_field, int type, uint32_t nx, uint32_t ny, uint32_t nz,
                uint32_t rate, uint64_t *d_stream, void *hip_stream);

/* Decode every block of a compressed volume into d_blocks ([N_b][64] float,
 * device, caller-owned) with the same decoder the cache uses. */
BCMC_API int bcmc_decode_all(bcmc_volume *v, float *d_blocks, void *hip_stream);

/* The generated marching cubes table: packed[c] holds the edge ids of case c
 * (4 bits each, 15 = unused) and its triangle count in bits 60..63. */
BCMC_API int bcmc_mc_table(uint64_t *packed256);

/* Measurement helper: a plain device-to-device copy of nbytes (a multiple of
 * 16) by the library's own streaming kernel, as a known-size reference when
 * reading hardware traffic counters.  Not part of the extraction. */
BCMC_API int bcmc_copy_calibration(void *d_dst, const void *d_src, uint64_t nbytes,
                                   void *hip_stream);

/* ---- batched extraction: many volumes x isovalues in one launch ------- */
/* A batch of jobs j = (volume job_vol[j], isovalue job_iso[j]) over
 * compressed volumes that share one scalar type (the volumes must outlive
 * the batch; their own caches are not used).  bcmc_batch_run extracts every
 * job in four launches: a persistent front kernel that culls and lists (its
 * phases separated by grid barriers), a decode kernel that decodes the new
 * blocks and builds sign masks, a count kernel, and an emission kernel in
 * which each workgroup sums the count kernel's per-wave totals before it;
 * replayed from a hipGraph when the runtime allows it.  Job j's
 * soup equals, byte for byte, bcmc_extract of its volume at its isovalue,
 * and the jobs' soups are concatenated in job order.  The batch keeps one
 * decoded-block store: a block needed by any job of its volume is decoded
 * once and stays resident (nothing is evicted; 256 B per block reserved). */
typedef struct bcmc_batch bcmc_batch;
typedef struct {
    uint64_t n_volumes, n_jobs;
    uint64_t n_blocks;        /* blocks of all volumes */
    uint64_t n_job_blocks;    /* sum over jobs of their volume's blocks */
    uint64_t n_resident;      /* decoded blocks in the batch store */
    uint64_t n_new;           /* decoded by the last run */
    uint64_t n_pairs;         /* (job, block) pairs of the last run that may emit */
    uint64_t n_vertices;      /* vertices of the last run (all jobs) */
    uint32_t stage_blocks;    /* schedule: blocks staged per memory round trip (4 or 8) */
    uint32_t grid;            /* schedule: workgroups of the back kernel */
    uint32_t workgroups_per_cu;  /* of the back kernel */
    uint32_t front_grid;      /* schedule: workgroups of the front kernel */
    uint32_t scan_schedule;   /* schedule: 0 = workgroup 0 scans the front kernel's
                                 counts, then a grid barrier; 1 = every workgroup
                                 sums the counts before its own */
    uint32_t decode_grid;     /* workgroups of the decode kernel */
    uint32_t ran_front_grid;  /* grids the last run's kernels were launched with, */
    uint32_t ran_decode_grid; /* as each kernel recorded them (0: that kernel */
    uint32_t ran_grid;        /* did not run, e.g. nothing to decode) */
    int32_t graph;            /* 1: the last run replayed a hipGraph */
    int32_t graph_unsupported;/* 1: capturing the cooperative launch failed */
    float last_ms;            /* GPU time of the last run (HIP events) */
    float phase_ms[8];        /* the last run's phases (device clock at the grid
                                 barriers and kernel ends): reset, flags, scan of
                                 the counts of new blocks and pairs, list scatter,
                                 decode and masks, count, the emission kernel's
                                 prefix of the per-wave totals (each of the last
                                 three with the gap before its kernel), emission */
} bcmc_batch_info;

BCMC_API int bcmc_batch_create(bcmc_volume *const *vols, uint32_t n_vols, const uint32_t *job_vol,
                               const float *job_iso, uint32_t n_jobs, void *hip_stream,
                               bcmc_batch **out);
/* New isovalues (host array of n_jobs floats); the captured graph reads them
 * from device memory, so no re-capture is needed. */
BCMC_API int bcmc_batch_set_isos(bcmc_batch *b, const float *job_iso, void *hip_stream);
/* Empty the batch's decoded-block store. */
BCMC_API int bcmc_batch_reset(bcmc_batch *b, void *hip_stream);
/* 1 (default): capture the launch in a hipGraph and replay it; 0: launch directly. */
BCMC_API int bcmc_batch_set_graph(bcmc_batch *b, int on);
/* Run every job into d_out (capacity_vertices bcmc_vertex records, device);
 * h_job_off (host, n_jobs + 1 entries) receives each job's first vertex and
 * the total.  Synchronises once.  BCMC_E_CAPACITY when the total exceeds the
 * capacity (offsets are set; enlarge and run again). */
BCMC_API int bcmc_batch_run(bcmc_batch *b, void *d_out, uint64_t capacity_vertices,
                            uint64_t *h_job_off, void *hip_stream);
/* Set the schedule by hand: stage_blocks (4 or 8) blocks staged per round
 * trip, per_cu workgroups per CU of the back kernel and front_per_cu of the
 * front kernel, each clamped to what stays resident (bcmc_batch_get_info
 * reports the grids), and scan_schedule (0 or 1, see bcmc_batch_info) for the
 * offsets of the front kernel's lists.  The next run captures its graph again.
 * Errors: BCMC_E_INVALID. */
BCMC_API int bcmc_batch_set_schedule(bcmc_batch *b, int stage_blocks, int per_cu,
                                     int front_per_cu, int scan_schedule);
/* Autotune the schedule (blocks staged per round trip, workgroups per CU
 * of the back and the front kernel, the front kernel's scan schedule) by
 * timing cold + warm runs of this batch; the best is kept and appended
 * to cache_path (one JSON object per line, keyed by arch, scalar type and
 * batch shape; NULL: $BCMC_AUTOTUNE_CACHE, or nothing).  Batches created
 * later with a matching key start from the stored schedule.  Empties the
 * batch store. */
BCMC_API int bcmc_batch_tune(bcmc_batch *b, const char *cache_path, void *hip_stream);
BCMC_API int bcmc_batch_get_info(const bcmc_batch *b, bcmc_batch_info *out);
BCMC_API void bcmc_batch_free(bcmc_batch *b);

/* ---- dense baseline (Sec. 3.3.3) --------------------------------------- */
/* The standard data-parallel marching cubes the paper measures as its
 * baseline (Sec. 3.3.3, tab:mc_naive_parallel_perf), over an uncompressed
 * float field resident in device memory: every cell classified, the cells
 * holding the surface compacted by a prefix sum, their vertex counts
 * summed by a second prefix sum, then a pass over the compacted cells
 * writes the soup.  No blocks, culling or cache.  Records are bcmc_vertex
 * (block-relative, computed as bcmc_extract computes them) with the cells in
 * global row-major order (x fastest): the same triangles as bcmc_extract of
 * the same field, in another order.
 * bcmc_dense_create reserves the scratch for an nx*ny*nz field (13 bytes per
 * cell; at most 2^32 - 1 samples).
 * bcmc_dense_extract: d_field ([nz][ny][nx] float, device), output as
 * bcmc_extract (capacity in records, BCMC_E_CAPACITY with *n_triangles set);
 * synchronises hip_stream once.  bcmc_dense_active_cells: cells holding the
 * surface in the last extract.  Errors: BCMC_E_INVALID, BCMC_E_NOMEM,
 * BCMC_E_CAPACITY, BCMC_E_HIP. */
typedef struct bcmc_dense bcmc_dense;
BCMC_API int bcmc_dense_create(uint32_t nx, uint32_t ny, uint32_t nz, bcmc_dense **out);
BCMC_API int bcmc_dense_extract(bcmc_dense *h, const float *d_field, float iso, void *d_out,
                                uint64_t capacity_vertices, uint64_t *n_triangles,
                                void *hip_stream);
BCMC_API int bcmc_dense_active_cells(const bcmc_dense *h, uint64_t *n_active);
BCMC_API void bcmc_dense_free(bcmc_dense *h);

/* ---- extraction without allocation ------------------------------------ */
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * extraction of bcmc_volume_from_blocks + bcmc_extract over caller-owned
 * decoded blocks d_blocks ([N_b][64] float, device), written as bcmc_vertex
 * records into d_out (capacity_vertices records, device), byte for byte the
 * same soup.  Every other buffer (ranges, flags, block lists, counts,
 * offsets, sign masks, scan state, counters, the case table) lives in one
 * static device array of 24 MiB per GPU, held until the process ends, so a
 * volume may have at most about 2^19 blocks (the exact bound depends on the
 * shape); larger volumes are rejected with BCMC_E_INVALID before any work.
 * The function calls no hipMalloc, hipFree or allocating routine.  Every
 * call on a GPU shares that GPU's array: calls that overlap on one GPU (on
 * different streams or host threads) race and must not be issued.  Calls in
 * sequence are independent (each clears what must start at zero).
 * Synchronises hip_stream once to read the triangle count.
 * Errors: BCMC_E_INVALID (dims, size above the scratch, NaN iso),
 * BCMC_E_CAPACITY (*n_triangles set, the first capacity_vertices records
 * written), BCMC_E_NONFINITE, BCMC_E_HIP. */
BCMC_API int bcmc_extract_blocks_noalloc(const float *d_blocks, uint32_t nx, uint32_t ny,
                                         uint32_t nz, float iso, void *d_out,
                                         uint64_t capacity_vertices, uint64_t *n_triangles,
                                         void *hip_stream);

/* ---- inspection of the last extract (host copies; synchronous) -------- */
BCMC_API int bcmc_debug_ranges(const bcmc_volume *v, float *h_ranges /* [N_b][2] */);
/* h_active[b]: bit 0 = active (M_active), bit 1 = may emit (the value hull
 * of b and its +x/+y/+z neighbours contains iso). */
BCMC_API int bcmc_debug_active(const bcmc_volume *v, uint8_t *h_active /* [N_b] */,
                      uint32_t *h_I_active /* [N_b] */, uint64_t *h_n_active);
BCMC_API int bcmc_debug_new(const bcmc_volume *v, uint32_t *h_I_new /* [N_b] */, uint64_t *h_n_new);
BCMC_API int bcmc_debug_cache_state(const bcmc_volume *v, int32_t *h_I_slot /* [N_b] */,
                           int32_t *h_S_block /* [n_slots] */,
                           uint32_t *h_S_age /* [n_slots] */, uint64_t *h_n_slots);
BCMC_API int bcmc_debug_slot_data(const bcmc_volume *v, float *h_slots /* [n_slots][64] */);
/* Advance the cache by k calls at which no block is active, as k
 * bcmc_extract calls at an isovalue outside the data would (Alg. 1's age
 * update: every slot's age += k, saturating at 2^32 - 1; every cached block
 * becomes available), without running them.  The cache's age clock counts
 * at most 2^31 - 1 calls since its reset.  A test hook for the age sort's
 * wide keys.  Errors: BCMC_E_INVALID (identity volume, clock overflow). */
BCMC_API int bcmc_debug_age_cache(bcmc_volume *v, uint32_t k, void *hip_stream);
BCMC_API int bcmc_debug_block_counts(const bcmc_volume *v, uint32_t *h_cnt, uint64_t *h_off,
                            uint64_t n /* <= n_active */);
/* Cases of the 64 cells of every active block of the last extract (which
 * must have used the same iso) into d_cases ([n_active][64], device). */
BCMC_API int bcmc_debug_cases(bcmc_volume *v, float iso, uint8_t *d_cases, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* BCMC_H */
