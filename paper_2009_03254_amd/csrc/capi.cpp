// C ABI of libbcmc: volume handles, buffers, and the stream-ordered
// orchestration of one extract call (paper Sec. 4, Alg. 1).
#include "../../include/bcmc.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>

#include "common.h"

using namespace bcmc;

namespace bcmc {
static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }
}  // namespace bcmc

struct bcmc_volume {
    Geom g{};
    int is_f64 = 0;
    uint32_t rate = 0;
    int identity = 0;              // slots are the caller's decoded blocks
    const float *ext_blocks = nullptr;
    DevState d;
    StatusLayout sl{};
    uint64_t init_slots = 0, max_slots = 0, n_slots = 0;  // host mirror
    Counters *h_ctr = nullptr;     // pinned copy of the device counters
    bcmc_stats stats{};
    uint32_t profiling = 0;   // stage mask (bit i: events around stage i)
    int vertex_format = BCMC_VERTEX_F32;  // output records of bcmc_extract
    uint32_t calls_since_reset = 0;  // bounds the age of every slot used since the reset
    hipEvent_t ev[8] = {};
    hipEvent_t ev_done = nullptr;  // after the counters' readback (polled, not slept on)
    int have_extract = 0;
    float last_iso = 0.0f;
    int last_format = BCMC_VERTEX_F32;   // the last extract's format (its grid set the chunks)
    float cull_iso = NAN;          // isovalue of the last cull (NaN: the flags are all zero)
    uint32_t gen = 0;              // extract calls, as the cull stamps rounds with active blocks
};

namespace bcmc {
const uint64_t *volume_stream(const bcmc_volume *v) { return v->d.stream; }
const float2 *volume_ranges(const bcmc_volume *v) { return v->d.ranges; }
Geom volume_geom(const bcmc_volume *v) { return v->g; }
uint32_t volume_rate(const bcmc_volume *v) { return v->rate; }
int volume_is_f64(const bcmc_volume *v) { return v->is_f64; }
int volume_is_identity(const bcmc_volume *v) { return v->identity; }
}  // namespace bcmc

namespace {

// After the ranges change: all flags zero, no tile culled before.
void clear_flags(bcmc_volume *v, hipStream_t s) {
    launch_fill_u32(reinterpret_cast<uint32_t *>(v->d.active), 0u, (v->g.nb + 3) / 4, s);
    v->cull_iso = NAN;
}

int invalid(const std::string &msg) {
    set_error(msg);
    return BCMC_E_INVALID;
}

template <typename T>
int dev_alloc(T **p, uint64_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)p, sizeof(T) * count);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        set_error("hipMalloc of " + std::to_string(sizeof(T) * count) + " bytes failed: " +
                  hipGetErrorString(e));
        return BCMC_E_NOMEM;
    }
    return BCMC_OK;
}

template <typename T>
void dev_free(T *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

Geom make_geom(uint32_t nx, uint32_t ny, uint32_t nz) {
    Geom g;
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.nbx = (nx + 3) / 4;
    g.nby = (ny + 3) / 4;
    g.nbz = (nz + 3) / 4;
    g.nb = (uint64_t)g.nbx * g.nby * g.nbz;
    return g;
}

int check_dims(uint32_t nx, uint32_t ny, uint32_t nz) {
    if (nx < 2 || ny < 2 || nz < 2) return invalid("every dimension must be at least 2");
    Geom g = make_geom(nx, ny, nz);
    if (g.nb >= (1ull << 31)) return invalid("more than 2^31 - 1 blocks");
    return BCMC_OK;
}

void free_cache(bcmc_volume *v) {
    dev_free(v->d.S_block);
    dev_free(v->d.S_age);
    dev_free(v->d.slots);
    dev_free(v->d.masks);
    dev_free(v->d.mask_iso);
    dev_free(v->d.slot_or);
    dev_free(v->d.slot_and);
    for (int i = 0; i < 2; i++) {
        dev_free(v->d.sort_key[i]);
        dev_free(v->d.sort_val[i]);
    }
    dev_free(v->d.radix_hist);
    dev_free(v->d.status);
}

StatusLayout status_layout(const Geom &g, uint64_t max_slots) {
    StatusLayout s;
    s.rnd = 0;
    s.slot = s.rnd + block_rounds(g.nb) / 4096 + 1;
    s.mc = s.slot + (max_slots + SLOT_TILE - 1) / SLOT_TILE;
    s.scan = s.mc + (g.nb + SCAN_TILE - 1) / SCAN_TILE + 1;
    uint64_t rtiles = (max_slots + RADIX_TILE - 1) / RADIX_TILE;
    s.total = s.scan + (256 * rtiles + SCAN_TILE - 1) / SCAN_TILE + 1;
    return s;
}

void layout_status(bcmc_volume *v) { v->sl = status_layout(v->g, v->max_slots); }

int alloc_common(bcmc_volume *v) {
    int rc;
    if ((rc = dev_alloc(&v->d.ranges, v->g.nb))) return rc;
    if ((rc = dev_alloc(&v->d.tile_ranges, cull_tiles(v->g)))) return rc;
    if ((rc = dev_alloc(&v->d.cull_list, 2 * cull_tiles(v->g)))) return rc;
    if ((rc = dev_alloc(&v->d.active, v->g.nb + 16))) return rc;
    if ((rc = dev_alloc(&v->d.round_gen, block_rounds(v->g.nb)))) return rc;
    BCMC_HIP_TRY(hipMemset(v->d.round_gen, 0, block_rounds(v->g.nb) * sizeof(uint32_t)));
    if ((rc = dev_alloc(&v->d.I_active, v->g.nb))) return rc;
    if ((rc = dev_alloc(&v->d.blk_cnt, v->g.nb))) return rc;
    if ((rc = dev_alloc(&v->d.blk_off, v->g.nb))) return rc;
    if ((rc = dev_alloc(&v->d.part_cand, (v->g.nb + BLK_TILE - 1) / BLK_TILE))) return rc;
    if ((rc = dev_alloc(&v->d.round_list, block_rounds(v->g.nb)))) return rc;
    if ((rc = dev_alloc(&v->d.round_cnt, block_rounds(v->g.nb)))) return rc;
    if ((rc = dev_alloc(&v->d.chunk_off, mc_chunk_slots(v->g.nb) + 8))) return rc;
    if ((rc = dev_alloc(&v->d.part_occw, 4 * MC_MAX_GRID))) return rc;
    if ((rc = dev_alloc(&v->d.part_giso, 4 * MC_MAX_GRID))) return rc;
    if ((rc = dev_alloc(&v->d.ctr, 1))) return rc;
    if ((rc = dev_alloc(&v->d.mc_table, 256))) return rc;
    if (mc_table_status() != 0) return invalid("marching cubes table generation failed");
    BCMC_HIP_TRY(hipMemcpy(v->d.mc_table, mc_table_host(), 256 * sizeof(uint64_t),
                           hipMemcpyHostToDevice));
    BCMC_HIP_TRY(hipHostMalloc((void **)&v->h_ctr, sizeof(Counters), hipHostMallocDefault));
    memset(v->h_ctr, 0, sizeof(Counters));
    v->stats.n_blocks = v->g.nb;
    return BCMC_OK;
}

void destroy(bcmc_volume *v) {
    if (!v) return;
    free_cache(v);
    dev_free(v->d.stream);
    dev_free(v->d.ranges);
    dev_free(v->d.tile_ranges);
    dev_free(v->d.cull_list);
    dev_free(v->d.active);
    dev_free(v->d.round_gen);
    dev_free(v->d.I_active);
    dev_free(v->d.I_new);
    dev_free(v->d.retry);
    dev_free(v->d.I_slot);
    dev_free(v->d.blk_cnt);
    dev_free(v->d.blk_off);
    dev_free(v->d.part_cand);
    dev_free(v->d.round_list);
    dev_free(v->d.round_cnt);
    dev_free(v->d.chunk_off);
    dev_free(v->d.part_occw);
    dev_free(v->d.part_giso);
    dev_free(v->d.ctr);
    dev_free(v->d.mc_table);
    if (v->h_ctr) (void)hipHostFree(v->h_ctr);
    for (auto &e : v->ev)
        if (e) (void)hipEventDestroy(e);
    if (v->ev_done) (void)hipEventDestroy(v->ev_done);
    delete v;
}

int reset_cache_state(bcmc_volume *v, hipStream_t s) {
    launch_fill_u32(reinterpret_cast<uint32_t *>(v->d.I_slot), 0xFFFFFFFFu, v->g.nb, s);
    launch_fill_u32(reinterpret_cast<uint32_t *>(v->d.S_block), 0xFFFFFFFFu, v->max_slots, s);
    launch_fill_u32(v->d.S_age, HIGH_AGE, v->max_slots, s);
    launch_fill_u32(v->d.mask_iso, MASK_NONE, v->max_slots, s);
    BCMC_HIP_TRY(hipGetLastError());
    v->calls_since_reset = 0;
    v->n_slots = v->init_slots;
    v->have_extract = 0;
    return BCMC_OK;
}

int set_budget(bcmc_volume *v, uint64_t initial_bytes, uint64_t max_bytes, hipStream_t s) {
    uint64_t init = initial_bytes / 256;
    uint64_t maxs = max_bytes ? max_bytes / 256 : std::max<uint64_t>(init, v->g.nb);
    if (maxs < init) return invalid("max_bytes is below initial_bytes");
    if (maxs >= (1ull << 31)) return invalid("more than 2^31 - 1 cache slots");
    BCMC_HIP_TRY(hipStreamSynchronize(s));
    free_cache(v);
    v->init_slots = init;
    v->max_slots = maxs;
    layout_status(v);
    int rc;
    if ((rc = dev_alloc(&v->d.S_block, maxs))) return rc;
    if ((rc = dev_alloc(&v->d.S_age, maxs))) return rc;
    if ((rc = dev_alloc(&v->d.slots, maxs * 64))) return rc;
    if ((rc = dev_alloc(&v->d.masks, maxs))) return rc;
    if ((rc = dev_alloc(&v->d.mask_iso, maxs))) return rc;
    if ((rc = dev_alloc(&v->d.slot_or, (maxs + SLOT_TILE - 1) / SLOT_TILE))) return rc;
    if ((rc = dev_alloc(&v->d.slot_and, (maxs + SLOT_TILE - 1) / SLOT_TILE))) return rc;
    for (int i = 0; i < 2; i++) {
        if ((rc = dev_alloc(&v->d.sort_key[i], maxs))) return rc;
        if ((rc = dev_alloc(&v->d.sort_val[i], maxs))) return rc;
    }
    if ((rc = dev_alloc(&v->d.radix_hist, 256 * ((maxs + RADIX_TILE - 1) / RADIX_TILE)))) return rc;
    if ((rc = dev_alloc(&v->d.status, v->sl.total))) return rc;
    BCMC_HIP_TRY(hipMemsetAsync(v->d.status, 0, v->sl.total * sizeof(uint64_t), s));
    return reset_cache_state(v, s);
}

hipStream_t as_stream(void *p) { return reinterpret_cast<hipStream_t>(p); }

// Reads the counters back.  The caller waits for them anyway, so the wait
// polls an event instead of sleeping in the runtime (a sleeping wait adds
// its wake-up latency to every call).
int sync_counters(bcmc_volume *v, hipStream_t s) {
    BCMC_HIP_TRY(hipMemcpyAsync(v->h_ctr, v->d.ctr, sizeof(Counters), hipMemcpyDeviceToHost, s));
    if (!v->ev_done) BCMC_HIP_TRY(hipEventCreateWithFlags(&v->ev_done, hipEventDisableTiming));
    BCMC_HIP_TRY(hipEventRecord(v->ev_done, s));
    hipError_t e;
    while ((e = hipEventQuery(v->ev_done)) == hipErrorNotReady) {
    }
    BCMC_HIP_TRY(e);
    return BCMC_OK;
}

}  // namespace

extern "C" {

const char *bcmc_last_error(void) { return g_last_error.c_str(); }

uint64_t bcmc_num_blocks(uint32_t nx, uint32_t ny, uint32_t nz) { return make_geom(nx, ny, nz).nb; }

int bcmc_mc_table(uint64_t *packed256) {
    if (!packed256) return invalid("null table pointer");
    if (mc_table_status() != 0) return invalid("marching cubes table generation failed");
    memcpy(packed256, mc_table_host(), 256 * sizeof(uint64_t));
    return BCMC_OK;
}

int bcmc_load_compressed(const void *stream, uint64_t nbytes, int stream_is_device, uint32_t nx,
                         uint32_t ny, uint32_t nz, int type, uint32_t rate, void *hip_stream,
                         bcmc_volume **out) {
    if (!out) return invalid("null output handle");
    *out = nullptr;
    if (!stream) return invalid("null stream");
    int rc = check_dims(nx, ny, nz);
    if (rc) return rc;
    if (type != BCMC_F32 && type != BCMC_F64) return invalid("type must be BCMC_F32 or BCMC_F64");
    if (rate < 1 || rate > (type == BCMC_F64 ? 64u : 32u)) return invalid("rate out of range");
    Geom g = make_geom(nx, ny, nz);
    if (nbytes != g.nb * 8ull * rate)
        return invalid("stream size " + std::to_string(nbytes) + " != N_b*8*rate = " +
                       std::to_string(g.nb * 8ull * rate));
    hipStream_t s = as_stream(hip_stream);
    bcmc_volume *v = new (std::nothrow) bcmc_volume();
    if (!v) return BCMC_E_NOMEM;
    v->g = g;
    v->is_f64 = type == BCMC_F64;
    v->rate = rate;
    if ((rc = alloc_common(v)) || (rc = dev_alloc(&v->d.stream, g.nb * rate)) ||
        (rc = dev_alloc(&v->d.I_new, g.nb)) || (rc = dev_alloc(&v->d.I_slot, g.nb)) ||
        (v->is_f64 && rate <= LOW_RATE_MAX && (rc = dev_alloc(&v->d.retry, g.nb)))) {
        destroy(v);
        return rc;
    }
    hipError_t e = hipMemcpyAsync(v->d.stream, stream, nbytes,
                                  stream_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(v->d.ctr, 0, sizeof(Counters), s);
    if (e != hipSuccess) {
        set_error(std::string("upload failed: ") + hipGetErrorString(e));
        destroy(v);
        return BCMC_E_HIP;
    }
    launch_decode_ranges(g, v->d.stream, v->is_f64, rate, v->d.ranges, nullptr, &v->d.ctr->err, s);
    launch_tile_ranges(g, v->d.ranges, v->d.tile_ranges, s);
    clear_flags(v, s);
    if ((rc = sync_counters(v, s))) {
        destroy(v);
        return rc;
    }
    if (v->h_ctr->err & ERR_NONFINITE) {
        set_error("the stream decodes to non-finite values");
        destroy(v);
        return BCMC_E_NONFINITE;
    }
    if ((rc = set_budget(v, 0, 0, s))) {
        destroy(v);
        return rc;
    }
    *out = v;
    return BCMC_OK;
}

int bcmc_volume_from_blocks(const float *d_blocks, uint32_t nx, uint32_t ny, uint32_t nz,
                            void *hip_stream, bcmc_volume **out) {
    if (!out) return invalid("null output handle");
    *out = nullptr;
    if (!d_blocks) return invalid("null blocks");
    int rc = check_dims(nx, ny, nz);
    if (rc) return rc;
    hipStream_t s = as_stream(hip_stream);
    bcmc_volume *v = new (std::nothrow) bcmc_volume();
    if (!v) return BCMC_E_NOMEM;
    v->g = make_geom(nx, ny, nz);
    v->identity = 1;
    v->ext_blocks = d_blocks;
    v->max_slots = 0;
    layout_status(v);
    if ((rc = alloc_common(v)) || (rc = dev_alloc(&v->d.status, v->sl.total)) ||
        (rc = dev_alloc(&v->d.masks, v->g.nb))) {
        destroy(v);
        return rc;
    }
    hipError_t e = hipMemsetAsync(v->d.ctr, 0, sizeof(Counters), s);
    if (e != hipSuccess) {
        set_error(hipGetErrorString(e));
        destroy(v);
        return BCMC_E_HIP;
    }
    launch_ranges_from_blocks(v->g, d_blocks, v->d.ranges, &v->d.ctr->err, s);
    launch_tile_ranges(v->g, v->d.ranges, v->d.tile_ranges, s);
    clear_flags(v, s);
    if ((rc = sync_counters(v, s))) {
        destroy(v);
        return rc;
    }
    if (v->h_ctr->err & ERR_NONFINITE) {
        set_error("the blocks hold non-finite values");
        destroy(v);
        return BCMC_E_NONFINITE;
    }
    v->n_slots = v->g.nb;
    *out = v;
    return BCMC_OK;
}

int bcmc_rebind_blocks(bcmc_volume *v, const float *d_blocks, void *hip_stream) {
    if (!v || !d_blocks) return invalid("null argument");
    if (!v->identity) return invalid("only bcmc_volume_from_blocks handles can be rebound");
    v->ext_blocks = d_blocks;
    v->have_extract = 0;
    launch_ranges_from_blocks(v->g, d_blocks, v->d.ranges, &v->d.ctr->err, as_stream(hip_stream));
    launch_tile_ranges(v->g, v->d.ranges, v->d.tile_ranges, as_stream(hip_stream));
    clear_flags(v, as_stream(hip_stream));
    BCMC_HIP_TRY(hipGetLastError());
    return BCMC_OK;
}

int bcmc_set_cache_budget(bcmc_volume *v, uint64_t initial_bytes, uint64_t max_bytes) {
    if (!v) return invalid("null handle");
    if (v->identity) return invalid("identity volumes have no cache");
    return set_budget(v, initial_bytes, max_bytes, nullptr);
}

int bcmc_reset_cache(bcmc_volume *v, void *hip_stream) {
    if (!v) return invalid("null handle");
    if (v->identity) return BCMC_OK;
    return reset_cache_state(v, as_stream(hip_stream));
}

int bcmc_vertices_to_q10(const void *d_vertices, uint64_t n, void *d_out, void *hip_stream) {
    if (n && (!d_vertices || !d_out)) return invalid("null pointer");
    launch_vertices_q10(d_vertices, n, d_out, as_stream(hip_stream));
    BCMC_HIP_TRY(hipGetLastError());
    return BCMC_OK;
}

int bcmc_debug_age_cache(bcmc_volume *v, uint32_t k, void *hip_stream) {
    if (!v) return invalid("null handle");
    if (v->identity) return invalid("identity volumes have no cache");
    if (k > 0x7FFFFFFFu - v->calls_since_reset)
        return invalid("the age clock would pass 2^31 - 1 calls since the cache reset");
    hipStream_t s = as_stream(hip_stream);
    launch_age_slots(v->d.S_age, v->n_slots, k, s);
    BCMC_HIP_TRY(hipGetLastError());
    v->calls_since_reset += k;
    return BCMC_OK;
}

int bcmc_set_vertex_format(bcmc_volume *v, int format) {
    if (!v) return invalid("null handle");
    if (format != BCMC_VERTEX_F32 && format != BCMC_VERTEX_EDGE8 && format != BCMC_VERTEX_Q10)
        return invalid("unknown vertex format");
    v->vertex_format = format;
    return BCMC_OK;
}

int bcmc_set_profiling_stages(bcmc_volume *v, uint32_t stage_mask) {
    if (!v) return invalid("null handle");
    if (stage_mask & ~BCMC_PROFILE_ALL) return invalid("stage mask has bits beyond stage 5");
    if (stage_mask && !v->ev[0])
        for (auto &e : v->ev) BCMC_HIP_TRY(hipEventCreate(&e));
    v->profiling = stage_mask;
    return BCMC_OK;
}

int bcmc_set_profiling(bcmc_volume *v, int on) {
    return bcmc_set_profiling_stages(v, on ? BCMC_PROFILE_ALL : 0u);
}

int bcmc_extract(bcmc_volume *v, float iso, void *d_out, uint64_t capacity_vertices,
                 uint64_t *n_triangles, void *hip_stream) {
    if (!v || !n_triangles) return invalid("null argument");
    if (!d_out && capacity_vertices) return invalid("null output buffer with nonzero capacity");
    if (iso != iso) return invalid("iso is NaN");
    hipStream_t s = as_stream(hip_stream);
    // event i opens stage i and closes stage i - 1: record it when either is profiled
    const uint32_t prof = v->profiling, marks = prof | (prof << 1);
    auto mark = [&](int i) -> hipError_t {
        return (marks >> i) & 1u ? hipEventRecord(v->ev[i], s) : hipSuccess;
    };
    BCMC_HIP_TRY(mark(0));
    if (++v->gen == 0) {   // the stamps would repeat: start over from all-zero
        launch_fill_u32(v->d.round_gen, 0u, block_rounds(v->g.nb), s);
        v->gen = 1;
    }
    launch_cull(v->g, v->d, v->sl, iso, v->cull_iso, v->n_slots, v->identity, v->gen, s);
    v->cull_iso = iso;
    launch_compact_blocks(v->g, v->d, v->sl, v->gen, s);
    BCMC_HIP_TRY(mark(1));
    if (!v->identity) {
        if (v->calls_since_reset < 0x7FFFFFFFu) v->calls_since_reset++;
        const uint32_t age_cap = v->calls_since_reset;   // used slots are younger
        launch_slot_pass(v->d, v->sl, v->n_slots, age_cap, s);
        launch_plan_grow(v->d, v->max_slots, v->max_slots - v->n_slots, s);
        // the first call after a reset finds every slot unused: all sort keys
        // are 0 and the order is the slot order already
        if (age_cap > 1) launch_radix(v->d, v->sl, v->max_slots, age_cap, s);
    }
    BCMC_HIP_TRY(mark(2));
    if (!v->identity) launch_assign_decode(v->d, v->is_f64, v->rate, v->g.nb, iso, s);
    BCMC_HIP_TRY(mark(3));
    const float *slots = v->identity ? v->ext_blocks : v->d.slots;
    launch_mc_count(v->g, v->d, slots, v->d.I_slot, v->identity, iso, v->vertex_format, s);
    BCMC_HIP_TRY(mark(4));   // the block offsets come with the emission (stage 4 is empty)
    BCMC_HIP_TRY(mark(5));
    launch_mc_emit(v->g, v->d, slots, v->d.I_slot, v->identity, iso, d_out, capacity_vertices,
                   v->vertex_format, s);
    BCMC_HIP_TRY(mark(6));
    if (hipError_t le = hipGetLastError()) {   // a launch failed: the flags are unknown
        clear_flags(v, s);
        set_error(std::string("extract launch: ") + hipGetErrorString(le));
        return BCMC_E_HIP;
    }
    int rc = sync_counters(v, s);
    if (rc) return rc;
    const Counters &c = *v->h_ctr;
    v->stats.calls++;
    if (c.err & ERR_INTERNAL) {
        reset_cache_state(v, s);
        set_error("internal consistency check failed in the cache update; cache reset");
        return BCMC_E_HIP;
    }
    if (c.err & ERR_CACHE_CAP) {
        reset_cache_state(v, s);
        v->stats.n_active = c.n_act;
        v->stats.n_new = v->stats.n_evicted = v->stats.n_occupied = v->stats.n_triangles = 0;
        v->stats.n_candidates = v->stats.n_general = 0;
        v->stats.n_slots = v->n_slots;
        set_error("the active blocks (" + std::to_string(c.n_act) +
                  ") do not fit the cache cap of " + std::to_string(v->max_slots) + " slots");
        return BCMC_E_CACHE_CAP;
    }
    if (!v->identity && c.n_new) v->n_slots = c.n_slots;
    const uint64_t T = c.total_verts / 3;
    *n_triangles = T;
    bcmc_stats &st = v->stats;
    st.n_active = c.n_act;
    st.n_new = v->identity ? 0 : c.n_new;
    st.n_evicted = c.n_evicted;
    st.n_occupied = c.n_occ;
    st.n_candidates = c.n_cand;
    st.n_general = v->identity ? 0 : c.tile_ctr[TC_RETRY];
    st.n_slots = v->n_slots;
    st.n_triangles = T;
    st.hit_rate = c.n_act ? 1.0 - (double)st.n_new / (double)c.n_act : 1.0;
    st.alg_bytes = 8.0 * v->g.nb + (double)st.n_new * (8.0 * v->rate + 256.0) +
                   256.0 * (double)c.n_act + 24.0 * (double)T;
    for (int i = 0; i < 8; i++) st.stage_ms[i] = 0.0;
    for (int i = 0; i < 6; i++) {
        if (!((prof >> i) & 1u)) continue;
        float ms = 0;
        (void)hipEventElapsedTime(&ms, v->ev[i], v->ev[i + 1]);
        st.stage_ms[i] = ms;
    }
    if ((prof & 1u) && (prof & (1u << 5))) {
        float tot = 0;
        (void)hipEventElapsedTime(&tot, v->ev[0], v->ev[6]);
        st.stage_ms[7] = tot;
    }
    v->have_extract = 1;
    v->last_iso = iso;
    v->last_format = v->vertex_format;
    if (c.total_verts > capacity_vertices) {
        set_error("vertex buffer too small: need " + std::to_string(c.total_verts) + " vertices");
        return BCMC_E_CAPACITY;
    }
    return BCMC_OK;
}

int bcmc_backward(bcmc_volume *v, float iso, const float *d_gV, uint64_t n_verts, float *d_dfield,
                  float *d_diso, void *hip_stream) {
    if (!v || !d_dfield || !d_diso) return invalid("null argument");
    if (!v->identity) return invalid("backward needs a bcmc_volume_from_blocks handle");
    if (!v->have_extract || iso != v->last_iso) return invalid("no extract at this iso to differentiate");
    if (n_verts != v->h_ctr->total_verts) return invalid("n_verts differs from the last extract");
    if (n_verts && !d_gV) return invalid("null gradient");
    hipStream_t s = as_stream(hip_stream);
    BCMC_HIP_TRY(hipMemsetAsync(d_dfield, 0, v->g.nb * 64 * sizeof(float), s));
    BCMC_HIP_TRY(hipMemsetAsync(d_diso, 0, sizeof(float), s));
    if (!n_verts) return BCMC_OK;
    BCMC_HIP_TRY(hipMemsetAsync(&v->d.ctr->err, 0, sizeof(unsigned int), s));
    launch_backward(v->g, v->d, v->ext_blocks, iso, d_gV, n_verts, d_dfield, d_diso, v->last_format, s);
    BCMC_HIP_TRY(hipGetLastError());
    // the kernel compares each block's vertex count with the forward's
    BCMC_HIP_TRY(hipMemcpyAsync(&v->h_ctr->err, &v->d.ctr->err, sizeof(unsigned int),
                                hipMemcpyDeviceToHost, s));
    BCMC_HIP_TRY(hipStreamSynchronize(s));
    if (v->h_ctr->err) {
        v->h_ctr->err = 0;
        v->have_extract = 0;
        set_error("the field changed between the forward extract and the backward "
                  "(per-block vertex counts differ)");
        return BCMC_E_INVALID;
    }
    return BCMC_OK;
}

int bcmc_get_stats(const bcmc_volume *v, bcmc_stats *out) {
    if (!v || !out) return invalid("null argument");
    *out = v->stats;
    return BCMC_OK;
}

void bcmc_free(bcmc_volume *v) {
    if (!v) return;
    (void)hipDeviceSynchronize();
    destroy(v);
}

int bcmc_encode(const void *d_field, int type, uint32_t nx, uint32_t ny, uint32_t nz, uint32_t rate,
                uint64_t *d_stream, void *hip_stream) {
    if (!d_field || !d_stream) return invalid("null pointer");
    int rc = check_dims(nx, ny, nz);
    if (rc) return rc;
    if (type != BCMC_F32 && type != BCMC_F64) return invalid("type must be BCMC_F32 or BCMC_F64");
    if (rate < 1 || rate > (type == BCMC_F64 ? 64u : 32u)) return invalid("rate out of range");
    hipStream_t s = as_stream(hip_stream);
    unsigned int *err = nullptr;
    if ((rc = dev_alloc(&err, 1))) return rc;
    BCMC_HIP_TRY(hipMemsetAsync(err, 0, sizeof(unsigned int), s));
    launch_encode(make_geom(nx, ny, nz), d_field, type == BCMC_F64, rate, d_stream, err, s);
    unsigned int h = 0;
    hipError_t e = hipMemcpyAsync(&h, err, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(err);
    if (e != hipSuccess) {
        set_error(hipGetErrorString(e));
        return BCMC_E_HIP;
    }
    if (h & ERR_NONFINITE) {
        set_error("the field holds non-finite values");
        return BCMC_E_NONFINITE;
    }
    return BCMC_OK;
}

int bcmc_decode_all(bcmc_volume *v, float *d_blocks, void *hip_stream) {
    if (!v || !d_blocks) return invalid("null argument");
    if (v->identity) return invalid("identity volumes hold no compressed stream");
    launch_decode_ranges(v->g, v->d.stream, v->is_f64, v->rate, v->d.ranges, d_blocks,
                         &v->d.ctr->err, as_stream(hip_stream));
    launch_tile_ranges(v->g, v->d.ranges, v->d.tile_ranges, as_stream(hip_stream));
    clear_flags(v, as_stream(hip_stream));
    BCMC_HIP_TRY(hipGetLastError());
    return BCMC_OK;
}

int bcmc_copy_calibration(void *d_dst, const void *d_src, uint64_t nbytes, void *hip_stream) {
    if (!d_dst || !d_src || (nbytes & 15)) return invalid("need device pointers and a multiple of 16 bytes");
    launch_copy_calibration(d_dst, d_src, nbytes / 16, as_stream(hip_stream));
    BCMC_HIP_TRY(hipGetLastError());
    return BCMC_OK;
}

int bcmc_debug_ranges(const bcmc_volume *v, float *h_ranges) {
    if (!v || !h_ranges) return invalid("null argument");
    BCMC_HIP_TRY(hipDeviceSynchronize());
    BCMC_HIP_TRY(hipMemcpy(h_ranges, v->d.ranges, v->g.nb * sizeof(float2), hipMemcpyDeviceToHost));
    return BCMC_OK;
}

int bcmc_debug_active(const bcmc_volume *v, uint8_t *h_active, uint32_t *h_I_active,
                      uint64_t *h_n_active) {
    if (!v) return invalid("null handle");
    if (!v->have_extract) return invalid("no extract yet");
    BCMC_HIP_TRY(hipDeviceSynchronize());
    uint64_t n = v->h_ctr->n_act;
    if (h_n_active) *h_n_active = n;
    if (h_active) BCMC_HIP_TRY(hipMemcpy(h_active, v->d.active, v->g.nb, hipMemcpyDeviceToHost));
    if (h_I_active && n)
        BCMC_HIP_TRY(hipMemcpy(h_I_active, v->d.I_active, n * 4, hipMemcpyDeviceToHost));
    return BCMC_OK;
}

int bcmc_debug_new(const bcmc_volume *v, uint32_t *h_I_new, uint64_t *h_n_new) {
    if (!v) return invalid("null handle");
    if (!v->have_extract || v->identity) return invalid("no cached extract yet");
    BCMC_HIP_TRY(hipDeviceSynchronize());
    uint64_t n = v->h_ctr->n_new;
    if (h_n_new) *h_n_new = n;
    if (h_I_new && n) BCMC_HIP_TRY(hipMemcpy(h_I_new, v->d.I_new, n * 4, hipMemcpyDeviceToHost));
    return BCMC_OK;
}

int bcmc_debug_cache_state(const bcmc_volume *v, int32_t *h_I_slot, int32_t *h_S_block,
                           uint32_t *h_S_age, uint64_t *h_n_slots) {
    if (!v) return invalid("null handle");
    if (v->identity) return invalid("identity volumes have no cache");
    BCMC_HIP_TRY(hipDeviceSynchronize());
    if (h_n_slots) *h_n_slots = v->n_slots;
    if (h_I_slot) BCMC_HIP_TRY(hipMemcpy(h_I_slot, v->d.I_slot, v->g.nb * 4, hipMemcpyDeviceToHost));
    if (h_S_block && v->n_slots)
        BCMC_HIP_TRY(hipMemcpy(h_S_block, v->d.S_block, v->n_slots * 4, hipMemcpyDeviceToHost));
    if (h_S_age && v->n_slots)
        BCMC_HIP_TRY(hipMemcpy(h_S_age, v->d.S_age, v->n_slots * 4, hipMemcpyDeviceToHost));
    return BCMC_OK;
}

int bcmc_debug_slot_data(const bcmc_volume *v, float *h_slots) {
    if (!v || !h_slots) return invalid("null argument");
    if (v->identity) return invalid("identity volumes have no cache");
    BCMC_HIP_TRY(hipDeviceSynchronize());
    if (v->n_slots)
        BCMC_HIP_TRY(hipMemcpy(h_slots, v->d.slots, v->n_slots * 256, hipMemcpyDeviceToHost));
    return BCMC_OK;
}

int bcmc_debug_block_counts(const bcmc_volume *v, uint32_t *h_cnt, uint64_t *h_off, uint64_t n) {
    if (!v) return invalid("null handle");
    if (!v->have_extract) return invalid("no extract yet");
    if (n > v->h_ctr->n_act) return invalid("n exceeds the active block count");
    BCMC_HIP_TRY(hipDeviceSynchronize());
    if (h_cnt && n) BCMC_HIP_TRY(hipMemcpy(h_cnt, v->d.blk_cnt, n * 4, hipMemcpyDeviceToHost));
    if (h_off && n) BCMC_HIP_TRY(hipMemcpy(h_off, v->d.blk_off, n * 8, hipMemcpyDeviceToHost));
    return BCMC_OK;
}

int bcmc_debug_cases(bcmc_volume *v, float iso, uint8_t *d_cases, void *hip_stream) {
    if (!v || !d_cases) return invalid("null argument");
    if (!v->have_extract || iso != v->last_iso) return invalid("no extract at this iso");
    const float *slots = v->identity ? v->ext_blocks : v->d.slots;
    launch_debug_cases(v->g, v->d, slots, v->d.I_slot, v->identity, iso, d_cases, v->g.nb,
                       as_stream(hip_stream));
    BCMC_HIP_TRY(hipGetLastError());
    return BCMC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Dense baseline (Sec. 3.3.3): marching cubes over an uncompressed field.
// ---------------------------------------------------------------------------
struct bcmc_dense {
    uint32_t nx = 0, ny = 0, nz = 0;
    uint32_t *ids = nullptr;
    uint8_t *cases = nullptr;
    uint64_t *first = nullptr, *work = nullptr, *mc_table = nullptr;
    void *ctr = nullptr;
    uint64_t *h_ctr = nullptr;   // pinned copy of the counters
};

namespace {
void dense_destroy(bcmc_dense *h) {
    if (!h) return;
    dev_free(h->ids);
    dev_free(h->cases);
    dev_free(h->first);
    dev_free(h->work);
    dev_free(h->mc_table);
    if (h->ctr) (void)hipFree(h->ctr);
    if (h->h_ctr) (void)hipHostFree(h->h_ctr);
    delete h;
}
}  // namespace

extern "C" int bcmc_dense_create(uint32_t nx, uint32_t ny, uint32_t nz, bcmc_dense **out) {
    if (!out) return invalid("null output handle");
    *out = nullptr;
    if (nx < 2 || ny < 2 || nz < 2) return invalid("every dimension must be at least 2");
    if ((uint64_t)nx * ny * nz >= (1ull << 32)) return invalid("at most 2^32 - 1 samples");
    if (mc_table_status() != 0) return invalid("marching cubes table generation failed");
    bcmc_dense *h = new (std::nothrow) bcmc_dense();
    if (!h) return BCMC_E_NOMEM;
    h->nx = nx;
    h->ny = ny;
    h->nz = nz;
    const uint64_t cells = (uint64_t)(nx - 1) * (ny - 1) * (nz - 1);
    int rc;
    if ((rc = dev_alloc(&h->ids, cells)) || (rc = dev_alloc(&h->cases, cells)) ||
        (rc = dev_alloc(&h->first, cells)) ||
        (rc = dev_alloc(&h->work, dense_work_words(nx, ny, nz))) ||
        (rc = dev_alloc(&h->mc_table, 256))) {
        dense_destroy(h);
        return rc;
    }
    if (hipMalloc(&h->ctr, dense_counter_bytes()) != hipSuccess ||
        hipHostMalloc((void **)&h->h_ctr, dense_counter_bytes(), hipHostMallocDefault) != hipSuccess ||
        hipMemcpy(h->mc_table, mc_table_host(), 256 * sizeof(uint64_t), hipMemcpyHostToDevice) !=
            hipSuccess) {
        (void)hipGetLastError();
        dense_destroy(h);
        set_error("dense baseline set-up failed");
        return BCMC_E_NOMEM;
    }
    *out = h;
    return BCMC_OK;
}

extern "C" int bcmc_dense_extract(bcmc_dense *h, const float *d_field, float iso, void *d_out,
                                  uint64_t capacity_vertices, uint64_t *n_triangles,
                                  void *hip_stream) {
    if (!h || !d_field || !n_triangles) return invalid("null argument");
    if (!d_out && capacity_vertices) return invalid("null output buffer with nonzero capacity");
    if (iso != iso) return invalid("iso is NaN");
    hipStream_t s = as_stream(hip_stream);
    launch_dense(h->nx, h->ny, h->nz, d_field, iso, h->ids, h->cases, h->first, h->work, h->ctr,
                 h->mc_table, d_out, capacity_vertices, s);
    BCMC_HIP_TRY(hipGetLastError());
    BCMC_HIP_TRY(hipMemcpyAsync(h->h_ctr, h->ctr, dense_counter_bytes(), hipMemcpyDeviceToHost, s));
    BCMC_HIP_TRY(hipStreamSynchronize(s));
    const uint64_t n_verts = h->h_ctr[3];   // counters: n_active at word 2, n_verts at word 3
    *n_triangles = n_verts / 3;
    if (n_verts > capacity_vertices) {
        set_error("vertex buffer too small: need " + std::to_string(n_verts) + " vertices");
        return BCMC_E_CAPACITY;
    }
    return BCMC_OK;
}

extern "C" int bcmc_dense_active_cells(const bcmc_dense *h, uint64_t *n_active) {
    if (!h || !n_active) return invalid("null argument");
    *n_active = h->h_ctr[2];
    return BCMC_OK;
}

extern "C" void bcmc_dense_free(bcmc_dense *h) {
    if (!h) return;
    (void)hipDeviceSynchronize();
    dense_destroy(h);
}

// ---------------------------------------------------------------------------
// Extraction over caller-owned decoded blocks without any allocation: every
// buffer the kernels need beyond the caller's input and output lives in one
// file-scope device array.  Each GPU holds its own copy of the array (it is
// loaded with the module on that device) until the process ends; host code
// never passes the array's name to a kernel, only the address
// hipGetSymbolAddress returns for the current device.
// ---------------------------------------------------------------------------
namespace {

constexpr uint64_t kScratchBytes = 24ull << 20;   // about 2^19 blocks (a 320^3 volume)
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static void *g_scratch_dev[kMaxDevices] = {};
static std::mutex g_scratch_mu;

// The current device's address of `scratch`, looked up once per device.
int scratch_address(void **out) {
    int dev = 0;
    BCMC_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return invalid("device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return BCMC_E_HIP;
        }
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return BCMC_OK;
}

// Carves the extraction's buffers out of the scratch array (256-byte
// aligned pieces); returns the bytes needed.
uint64_t carve_scratch(const Geom &g, const StatusLayout &sl, uintptr_t base, DevState &d,
                       unsigned int **range_err) {
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        unsigned char *p = reinterpret_cast<unsigned char *>(base + off);
        off += (bytes + 255) / 256 * 256;
        return p;
    };
    d.ctr = reinterpret_cast<Counters *>(take(sizeof(Counters)));
    *range_err = reinterpret_cast<unsigned int *>(take(sizeof(unsigned int)));
    d.mc_table = reinterpret_cast<uint64_t *>(take(256 * sizeof(uint64_t)));
    d.ranges = reinterpret_cast<float2 *>(take(g.nb * sizeof(float2)));
    d.tile_ranges = reinterpret_cast<float2 *>(take(cull_tiles(g) * sizeof(float2)));
    d.cull_list = reinterpret_cast<uint32_t *>(take(2 * cull_tiles(g) * sizeof(uint32_t)));
    d.active = take((g.nb + 16 + 3) / 4 * 4);
    d.round_gen = reinterpret_cast<uint32_t *>(take(block_rounds(g.nb) * sizeof(uint32_t)));
    d.I_active = reinterpret_cast<uint32_t *>(take(g.nb * sizeof(uint32_t)));
    d.blk_cnt = reinterpret_cast<uint32_t *>(take(g.nb * sizeof(uint32_t)));
    d.blk_off = reinterpret_cast<uint64_t *>(take(g.nb * sizeof(uint64_t)));
    d.masks = reinterpret_cast<uint64_t *>(take(g.nb * sizeof(uint64_t)));
    d.part_cand = reinterpret_cast<uint32_t *>(take((g.nb + BLK_TILE - 1) / BLK_TILE * sizeof(uint32_t)));
    d.round_list = reinterpret_cast<uint32_t *>(take(block_rounds(g.nb) * sizeof(uint32_t)));
    d.round_cnt = reinterpret_cast<uint64_t *>(take(block_rounds(g.nb) * sizeof(uint64_t)));
    d.chunk_off = reinterpret_cast<uint64_t *>(take((mc_chunk_slots(g.nb) + 8) * sizeof(uint64_t)));
    d.part_occw = reinterpret_cast<uint32_t *>(take(4 * MC_MAX_GRID * sizeof(uint32_t)));
    d.status = reinterpret_cast<uint64_t *>(take(sl.total * sizeof(uint64_t)));
    return off;
}

}  // namespace

extern "C" int bcmc_extract_blocks_noalloc(const float *d_blocks, uint32_t nx, uint32_t ny,
                                           uint32_t nz, float iso, void *d_out,
                                           uint64_t capacity_vertices, uint64_t *n_triangles,
                                           void *hip_stream) {
    if (!d_blocks || !n_triangles) return invalid("null argument");
    if (!d_out && capacity_vertices) return invalid("null output buffer with nonzero capacity");
    if (iso != iso) return invalid("iso is NaN");
    *n_triangles = 0;
    int rc = check_dims(nx, ny, nz);
    if (rc) return rc;
    if (mc_table_status() != 0) return invalid("marching cubes table generation failed");
    const Geom g = make_geom(nx, ny, nz);
    const StatusLayout sl = status_layout(g, 0);
    DevState d;
    unsigned int *range_err = nullptr;
    const uint64_t need = carve_scratch(g, sl, 0, d, &range_err);   // sizes only
    if (need > kScratchBytes)
        return invalid("volume of " + std::to_string(g.nb) + " blocks needs " + std::to_string(need) +
                       " bytes of scratch; the static scratch holds " + std::to_string(kScratchBytes));
    void *base = nullptr;
    if ((rc = scratch_address(&base))) return rc;
    carve_scratch(g, sl, reinterpret_cast<uintptr_t>(base), d, &range_err);
    hipStream_t s = as_stream(hip_stream);
    const uint32_t gen = 1;   // the round stamps are cleared below, every call
    // the previous call on this device left its own contents: clear what
    // must start at zero (counters, error word, flags), rewrite the table
    launch_fill_u32(reinterpret_cast<uint32_t *>(d.ctr), 0u, sizeof(Counters) / 4, s);
    launch_fill_u32(range_err, 0u, 1, s);
    BCMC_HIP_TRY(hipMemcpyAsync(d.mc_table, mc_table_host(), 256 * sizeof(uint64_t),
                                hipMemcpyHostToDevice, s));
    launch_ranges_from_blocks(g, d_blocks, d.ranges, range_err, s);
    launch_tile_ranges(g, d.ranges, d.tile_ranges, s);
    launch_fill_u32(reinterpret_cast<uint32_t *>(d.active), 0u, (g.nb + 3) / 4, s);
    launch_fill_u32(d.round_gen, 0u, block_rounds(g.nb), s);
    launch_cull(g, d, sl, iso, NAN, 0, 1, gen, s);
    launch_compact_blocks(g, d, sl, gen, s);
    launch_mc_count(g, d, d_blocks, nullptr, 1, iso, 0, s);
    launch_mc_emit(g, d, d_blocks, nullptr, 1, iso, d_out, capacity_vertices, 0, s);
    BCMC_HIP_TRY(hipGetLastError());
    Counters c;
    unsigned int rerr = 0;
    BCMC_HIP_TRY(hipMemcpyAsync(&c, d.ctr, sizeof(Counters), hipMemcpyDeviceToHost, s));
    BCMC_HIP_TRY(hipMemcpyAsync(&rerr, range_err, sizeof(unsigned int), hipMemcpyDeviceToHost, s));
    BCMC_HIP_TRY(hipStreamSynchronize(s));
    if (rerr & ERR_NONFINITE) {
        set_error("the blocks hold non-finite values");
        return BCMC_E_NONFINITE;
    }
    if (c.err) {
        set_error("internal consistency check failed in the extraction");
        return BCMC_E_HIP;
    }
    *n_triangles = c.total_verts / 3;
    if (c.total_verts > capacity_vertices) {
        set_error("vertex buffer too small: need " + std::to_string(c.total_verts) + " vertices");
        return BCMC_E_CAPACITY;
    }
    return BCMC_OK;
}
