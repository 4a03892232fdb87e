// Internal definitions shared by the HIP sources of libbcmc (not part of the
// C ABI).  gfx950 only: wave64, one process per GPU.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace bcmc {

// ---- constants ----------------------------------------------------------
constexpr uint32_t HIGH_AGE = 0x80000000u;  // age of a slot created empty
// Tag of a sign mask built for no isovalue: a NaN pattern (isovalues are
// never NaN, so no call's tag equals it).
constexpr uint32_t MASK_NONE = 0x7FC00001u;
constexpr int BLK_TILE = 4096;               // blocks per compaction tile
constexpr int SLOT_TILE = 4096;              // slots per compaction tile (16 per thread)
constexpr int RADIX_TILE = 1024;             // elements per radix tile (1 wave)
constexpr int MC_MAX_GRID = 2048;           // workgroups of the count / emission grid at most
constexpr int SCAN_TILE = 4096;              // u32 per look-back scan tile (16 per thread)
constexpr int MC_WAVES = 4;                  // blocks (one per wave) per MC tile

// look-back status words: 2 flag bits on top, value below
constexpr uint64_t LB_AGG = 1ull << 62;
constexpr uint64_t LB_PRE = 2ull << 62;
constexpr uint64_t LB_VAL = (1ull << 62) - 1;

enum : uint32_t { ERR_CACHE_CAP = 1u, ERR_NONFINITE = 2u, ERR_INTERNAL = 4u, ERR_TIMEOUT = 8u };

// Device-resident scalars of one extract call.  Written only by kernels of
// that call, read back once by the host at its end.
struct Counters {
    unsigned long long n_act;        // active blocks
    unsigned long long n_new;        // active blocks not in the cache
    unsigned long long n_avail;      // available slots (after growth)
    unsigned long long n_slots;      // slots in use by the cache (after growth)
    unsigned long long n_slots_old;  // slots before growth
    unsigned long long n_avail_old;  // available slots before growth
    unsigned long long n_grow;       // slots added this call
    unsigned long long n_evicted;    // blocks evicted this call
    unsigned long long n_occ;        // active blocks that emit triangles
    unsigned long long n_cand;       // active blocks that may emit (staged by the count pass)
    unsigned long long total_verts;  // 3 * triangles
    unsigned long long n_live_rounds;  // 4096-block rounds holding an active block
    unsigned int err;                // ERR_* bits
    unsigned int key_or, key_and;    // OR / AND of the sort keys of available slots
    unsigned int pass_mask;          // radix digits that vary (bit p = digit p)
    unsigned int tile_ctr[16];       // dynamic work counters (tiles / batches)
};
enum { TC_ROUNDS = 0, TC_SLOT = 1, TC_MC = 2, TC_SCAN0 = 3 /* 3..6 per radix pass */,
       TC_MCCOUNT = 7, TC_MCEMIT = 8, TC_RETRY = 9 /* blocks the low-rate decoder handed back */,
       TC_CULL_LIVE = 10, TC_CULL_STALE = 11 /* the cull's queued tiles */ };
// Double-precision streams up to this rate decode with the low-rate decoder
// (and a general pass over the blocks it hands back).
constexpr uint32_t LOW_RATE_MAX = 4;


// Geometry of a volume in blocks.
struct Geom {
    uint32_t nx, ny, nz;
    uint32_t nbx, nby, nbz;
    uint64_t nb;
};

// Device buffers of a volume (all owned by the volume).
struct DevState {
    uint64_t *stream = nullptr;     // fixed-rate ZFP words, block b at b*rate
    float2 *ranges = nullptr;       // per block (min, max) of decoded valid samples
    float2 *tile_ranges = nullptr;  // per cull tile: hull of its blocks' and halo's ranges
    uint32_t *cull_list = nullptr;  // 2 x cull tiles: the call's live tiles, then its stale ones
    uint8_t *active = nullptr;      // M_active
    uint32_t *round_gen = nullptr;  // per 4096-block round: the last call that found an active block in it
    uint32_t *I_active = nullptr;   // ascending active block ids
    uint32_t *I_new = nullptr;      // ascending new block ids
    uint32_t *retry = nullptr;      // low-rate f64 decode: indices into I_new handed back
    int32_t *I_slot = nullptr;      // per block: slot or -1
    // cache (max_slots entries)
    int32_t *S_block = nullptr;
    uint32_t *S_age = nullptr;
    float *slots = nullptr;         // [max_slots][64] decoded blocks
    uint64_t *masks = nullptr;      // [max_slots] per slot: bit i = sample i below iso
    uint32_t *slot_or = nullptr;    // [slot tiles] OR / AND of each tile's sort keys
    uint32_t *slot_and = nullptr;
    uint32_t *mask_iso = nullptr;   // [max_slots] bits of the isovalue masks[] was built for
                                    // (MASK_NONE: none)
    uint32_t *sort_key[2] = {nullptr, nullptr};  // ~age of available slots
    uint32_t *sort_val[2] = {nullptr, nullptr};  // slot ids
    uint32_t *radix_hist = nullptr;              // 256 * radix tiles
    // MC
    uint32_t *blk_cnt = nullptr;    // per active block vertex count
    uint64_t *blk_off = nullptr;    // per active block first vertex
    uint32_t *part_cand = nullptr;  // per live round: blocks that may emit
    uint32_t *round_list = nullptr; // ascending live rounds of the call
    uint64_t *round_cnt = nullptr;  // per live round: (active << 32 | new) blocks, then their offsets
    uint64_t *chunk_off = nullptr;  // per 64-entry chunk of the active list: vertices, then first vertex
                                    // in its XCD eighth; then the 8 eighths' totals
    uint32_t *part_occw = nullptr;  // [4 * max MC grid] per-wave occupied blocks
    float *part_giso = nullptr;     // [4 * max MC grid] per-wave dL/diso of the backward
    uint64_t *status = nullptr;     // look-back status words (all kernels)
    Counters *ctr = nullptr;
    uint64_t *mc_table = nullptr;   // 256 packed cases
};

// Offsets of each kernel's region inside DevState::status.
struct StatusLayout {
    uint64_t rnd, slot, mc, scan, total;
};

// ---- launchers (extract.hip) -------------------------------------------
// prev_iso: the previous cull's isovalue (NaN after the flags were cleared).
// gen: a number that differs from every earlier call's on these buffers
// (rounds of blocks whose round_gen equals it hold this call's active blocks).
void launch_cull(const Geom &g, const DevState &d, const StatusLayout &sl, float iso, float prev_iso,
                 uint64_t n_slots_host, int identity_cache, uint32_t gen, hipStream_t s);
void launch_compact_blocks(const Geom &g, const DevState &d, const StatusLayout &sl, uint32_t gen,
                           hipStream_t s);
inline uint64_t block_rounds(uint64_t nb) { return (nb + BLK_TILE - 1) / BLK_TILE; }
// Chunk entries of the count pass's and emission's chunk totals: a call
// with n_act active blocks on W waves has ceil(n_act / cs) chunks of
// cs = min(64, ceil(n_act / W)) blocks (mc_chunk_size), at most
// max(ceil(nb / 64), W); the 8 XCD totals follow them.
inline uint64_t mc_chunk_slots(uint64_t nb) {
    const uint64_t a = (nb + 63) / 64, b = 4ull * MC_MAX_GRID;
    return a > b ? a : b;
}
// age_cap: exceeds the age of every slot used since the cache was reset.
void launch_slot_pass(const DevState &d, const StatusLayout &sl, uint64_t n_slots_host,
                      uint32_t age_cap, hipStream_t s);
void launch_plan_grow(const DevState &d, uint64_t max_slots, uint64_t grow_bound, hipStream_t s);
// Radix passes over the digits of keys up to age_cap (the others are zero).
void launch_radix(const DevState &d, const StatusLayout &sl, uint64_t max_elems, uint32_t age_cap,
                  hipStream_t s);
void launch_mc_count(const Geom &g, const DevState &d, const float *slots, const int32_t *I_slot,
                     int identity_cache, float iso, int fmt, hipStream_t s);

void launch_mc_emit(const Geom &g, const DevState &d, const float *slots, const int32_t *I_slot,
                    int identity_cache, float iso, void *out, uint64_t cap_verts, int fmt,
                    hipStream_t s);
// fmt: the bcmc_vertex_format codes (0 = 16-byte vertex, 1 = edge record,
// 2 = 10-bit quantised vertex).
void launch_vertices_q10(const void *in, uint64_t n, void *out, hipStream_t s);
void launch_debug_cases(const Geom &g, const DevState &d, const float *slots,
                        const int32_t *I_slot, int identity_cache, float iso, uint8_t *cases,
                        uint64_t max_act, hipStream_t s);
void launch_backward(const Geom &g, const DevState &d, const float *slots, float iso,
                     const float *gV, uint64_t n_verts, float *dfield, float *diso, int fmt,
                     hipStream_t s);
void launch_fill_u32(uint32_t *p, uint32_t v, uint64_t n, hipStream_t s);
void launch_age_slots(uint32_t *S_age, uint64_t n, uint32_t k, hipStream_t s);
void launch_copy_calibration(void *dst, const void *src, uint64_t n16, hipStream_t s);
void launch_iota_i32(int32_t *p, uint64_t n, hipStream_t s);

// ---- launchers (dense.hip): dense marching cubes baseline ---------------
uint64_t dense_work_words(uint32_t nx, uint32_t ny, uint32_t nz);
uint64_t dense_counter_bytes();
void launch_dense(uint32_t nx, uint32_t ny, uint32_t nz, const float *field, float iso,
                  uint32_t *ids, uint8_t *cases, uint64_t *first, uint64_t *work,
                  void *ctr_mem, const uint64_t *mc_table, void *out, uint64_t cap, hipStream_t s);

// ---- launchers (zfp.hip) -----------------------------------------------
void launch_decode_ranges(const Geom &g, const uint64_t *stream, int is_f64, uint32_t rate,
                          float2 *ranges, float *blocks_out, unsigned int *err, hipStream_t s);
// Hull of the ranges over each cull tile and its one-block halo (after every
// change of the ranges).
uint64_t cull_tiles(const Geom &g);
void launch_tile_ranges(const Geom &g, const float2 *ranges, float2 *tile_ranges, hipStream_t s);
void launch_ranges_from_blocks(const Geom &g, const float *blocks, float2 *ranges,
                               unsigned int *err, hipStream_t s);
void launch_assign_decode(const DevState &d, int is_f64, uint32_t rate, uint64_t max_new, float iso,
                          hipStream_t s);
void launch_encode(const Geom &g, const void *field, int is_f64, uint32_t rate,
                   uint64_t *stream, unsigned int *err, hipStream_t s);

// ---- host-side tables (tables.cpp) --------------------------------------
// Packed marching cubes table: bits 4k..4k+3 = k-th edge id (15 = unused),
// bits 60..63 = number of triangles.
const uint64_t *mc_table_host();
int mc_table_status();  // 0 when the generator succeeded

// ---- error reporting (capi.cpp) -----------------------------------------
void set_error(const std::string &msg);

}  // namespace bcmc

#define BCMC_HIP_TRY(expr)                                                  \
    do {                                                                    \
        hipError_t e_ = (expr);                                             \
        if (e_ != hipSuccess) {                                             \
            bcmc::set_error(std::string(#expr) + ": " + hipGetErrorString(e_)); \
            return BCMC_E_HIP;                                              \
        }                                                                   \
    } while (0)
