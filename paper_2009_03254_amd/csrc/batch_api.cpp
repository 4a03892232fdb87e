// C ABI of the batched extraction (many volumes x isovalues in one persistent
// launch), its hipGraph replay and its schedule autotuner.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "../../include/bcmc.h"
#include "batch.h"
#include "common.h"
#include "zfp_device.h"

using namespace bcmc;

namespace bcmc {
// defined in capi.cpp
const uint64_t *volume_stream(const bcmc_volume *v);
const float2 *volume_ranges(const bcmc_volume *v);
Geom volume_geom(const bcmc_volume *v);
uint32_t volume_rate(const bcmc_volume *v);
int volume_is_f64(const bcmc_volume *v);
int volume_is_identity(const bcmc_volume *v);
}  // namespace bcmc

struct bcmc_batch {
    int is_f64 = 0;
    uint32_t n_vols = 0, n_jobs = 0;
    uint64_t n_gblocks = 0, n_jblocks = 0;
    BatchParams p{};
    std::vector<void *> allocs;
    BatchCounters *h_ctr = nullptr;
    uint64_t *h_job_off = nullptr;
    int sb = 8;
    unsigned grid = 0;          // back kernel (count, scan, emission)
    unsigned front_grid = 0;    // front kernel (flags, lists)
    int front_pc_max = 1;       // its resident workgroups per CU
    unsigned decode_grid = 0;   // decode kernel (decode, sign masks)
    int per_cu_max = 1, cus = 256;
    // graph replay on a private stream
    hipStream_t gstream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_t0 = nullptr, ev_t1 = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void *graph_out = nullptr;
    uint64_t graph_cap = 0;
    int graph_sb = 0;
    unsigned graph_grid = 0, graph_front_grid = 0, graph_decode_grid = 0, graph_scan = 0;
    int use_graph = 1, graph_failed = 0;
    float last_ms = 0.0f;
    unsigned long long *h_ts = nullptr;   // phase clock stamps of the last run
    float phase_ms[8] = {};
    int clock_khz = 0;
    std::string key;
};

namespace {

int binvalid(const std::string &m) {
    set_error(m);
    return BCMC_E_INVALID;
}

template <typename T>
int balloc(bcmc_batch *b, T **p, uint64_t n) {
    *p = nullptr;
    if (!n) n = 1;
    if (hipMalloc((void **)p, sizeof(T) * n) != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipMalloc of " + std::to_string(sizeof(T) * n) + " bytes failed");
        return BCMC_E_NOMEM;
    }
    b->allocs.push_back((void *)*p);
    return BCMC_OK;
}

void drop_graph(bcmc_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

void destroy_batch(bcmc_batch *b) {
    if (!b) return;
    drop_graph(b);
    for (void *p : b->allocs) (void)hipFree(p);
    if (b->h_ctr) (void)hipHostFree(b->h_ctr);
    if (b->h_job_off) (void)hipHostFree(b->h_job_off);
    if (b->h_ts) (void)hipHostFree(b->h_ts);
    for (hipEvent_t e : {b->ev_in, b->ev_out, b->ev_t0, b->ev_t1})
        if (e) (void)hipEventDestroy(e);
    if (b->gstream) (void)hipStreamDestroy(b->gstream);
    delete b;
}

unsigned grid_for(bcmc_batch *b, int per_cu) {
    unsigned g = (unsigned)(per_cu * b->cus) / 8u * 8u;
    return g < 8 ? 8 : g;
}

// Back kernel: `sb` blocks staged per round trip, `per_cu` workgroups per
// CU; front kernel: `front_pc` workgroups per CU (both clamped to what stays
// resident) and `scan` its scan schedule (BatchParams::scan_sched).
int set_schedule(bcmc_batch *b, int sb, int per_cu, int front_pc, int scan) {
    int maxc = 0;
    if (batch_back_per_cu(sb, &maxc) != 0 || maxc < 1)
        return binvalid("the batched kernel cannot be made resident");
    b->sb = sb;
    b->per_cu_max = maxc;
    b->grid = grid_for(b, std::min(std::max(per_cu, 1), maxc));
    b->front_grid = grid_for(b, std::min(std::max(front_pc, 1), b->front_pc_max));
    b->p.scan_sched = scan ? 1u : 0u;
    return BCMC_OK;
}

// One run on the private stream (the caller's stream waits for it).
int run_once(bcmc_batch *b, void *d_out, uint64_t cap, hipStream_t caller) {
    b->p.out = d_out;
    b->p.cap = cap;
    BCMC_HIP_TRY(hipEventRecord(b->ev_in, caller));
    BCMC_HIP_TRY(hipStreamWaitEvent(b->gstream, b->ev_in, 0));
    BCMC_HIP_TRY(hipEventRecord(b->ev_t0, b->gstream));
    bool launched = false;
    if (b->use_graph && !b->graph_failed) {
        // a captured graph holds the launch configuration: capture again when
        // any schedule dimension or the output changes
        if (!b->exec || b->graph_out != d_out || b->graph_cap != cap || b->graph_sb != b->sb ||
            b->graph_grid != b->grid || b->graph_front_grid != b->front_grid ||
            b->graph_decode_grid != b->decode_grid || b->graph_scan != b->p.scan_sched) {
            drop_graph(b);
            hipError_t e = hipStreamBeginCapture(b->gstream, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                const unsigned grids[3] = {b->front_grid, b->decode_grid, b->grid};
                hipError_t le = launch_batch(b->p, b->is_f64, b->sb, grids, b->gstream, 0);
                e = hipStreamEndCapture(b->gstream, &b->graph);
                if (le != hipSuccess) e = le;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                drop_graph(b);
                b->graph_failed = 1;
            } else {
                b->graph_out = d_out;
                b->graph_cap = cap;
                b->graph_sb = b->sb;
                b->graph_grid = b->grid;
                b->graph_front_grid = b->front_grid;
                b->graph_decode_grid = b->decode_grid;
                b->graph_scan = b->p.scan_sched;
            }
        }
        if (b->exec) {
            BCMC_HIP_TRY(hipGraphLaunch(b->exec, b->gstream));
            launched = true;
        }
    }
    if (!launched) {
        const unsigned grids[3] = {b->front_grid, b->decode_grid, b->grid};
        BCMC_HIP_TRY(launch_batch(b->p, b->is_f64, b->sb, grids, b->gstream, 1));
    }
    BCMC_HIP_TRY(hipEventRecord(b->ev_t1, b->gstream));
    BCMC_HIP_TRY(hipMemcpyAsync(b->h_ctr, b->p.ctr, sizeof(BatchCounters), hipMemcpyDeviceToHost,
                                b->gstream));
    BCMC_HIP_TRY(hipMemcpyAsync(b->h_job_off, b->p.job_off, (b->n_jobs + 1) * sizeof(uint64_t),
                                hipMemcpyDeviceToHost, b->gstream));
    BCMC_HIP_TRY(hipMemcpyAsync(b->h_ts, b->p.phase_ts, 9 * sizeof(unsigned long long),
                                hipMemcpyDeviceToHost, b->gstream));
    BCMC_HIP_TRY(hipEventRecord(b->ev_out, b->gstream));
    BCMC_HIP_TRY(hipStreamWaitEvent(caller, b->ev_out, 0));
    BCMC_HIP_TRY(hipEventSynchronize(b->ev_out));
    (void)hipEventElapsedTime(&b->last_ms, b->ev_t0, b->ev_t1);
    for (int k = 0; k < 8; k++)
        b->phase_ms[k] = b->clock_khz > 0 && b->h_ts[k + 1] >= b->h_ts[k]
                             ? (float)((double)(b->h_ts[k + 1] - b->h_ts[k]) / b->clock_khz)
                             : 0.0f;
    if (b->h_ctr->err) {
        const unsigned err = b->h_ctr->err;
        // a failed run may leave the store and the barrier words mid-update
        launch_fill_u32(reinterpret_cast<uint32_t *>(b->p.I_slot), 0xFFFFFFFFu, b->n_gblocks,
                              b->gstream);
        (void)hipMemsetAsync(b->p.ctr, 0, sizeof(BatchCounters), b->gstream);
        (void)hipMemsetAsync(b->p.bar, 0, BAR_WORDS * sizeof(unsigned int), b->gstream);
        (void)hipStreamSynchronize(b->gstream);
        set_error(err & ERR_TIMEOUT ? "a grid barrier of the batched kernel timed out"
                                    : "internal consistency check failed in the batched extraction");
        return BCMC_E_HIP;
    }
    return BCMC_OK;
}

int reset_cache(bcmc_batch *b, hipStream_t s) {
    launch_fill_u32(reinterpret_cast<uint32_t *>(b->p.I_slot), 0xFFFFFFFFu, b->n_gblocks, s);
    BCMC_HIP_TRY(hipMemsetAsync(b->p.ctr, 0, sizeof(BatchCounters), s));
    BCMC_HIP_TRY(hipMemsetAsync(b->p.bar, 0, BAR_WORDS * sizeof(unsigned int), s));
    return BCMC_OK;
}

// ---- schedule cache: one JSON object per line, keyed by arch and shape ----
bool load_schedule(const char *path, const std::string &key, int *sb, int *per_cu, int *front_pc,
                   int *scan) {
    if (!path || !*path) return false;
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        if (!strstr(line, ("\"key\": \"" + key + "\"").c_str())) continue;
        const char *a = strstr(line, "\"sb\": ");
        const char *c = strstr(line, "\"per_cu\": ");
        const char *f = strstr(line, "\"front_per_cu\": ");
        const char *d = strstr(line, "\"scan\": ");
        if (a && c && f && d && sscanf(a, "\"sb\": %d", sb) == 1 && sscanf(c, "\"per_cu\": %d", per_cu) == 1 &&
            sscanf(f, "\"front_per_cu\": %d", front_pc) == 1 && sscanf(d, "\"scan\": %d", scan) == 1)
            found = true;
    }
    fclose(f);
    return found;
}

void save_schedule(const char *path, const std::string &key, int sb, int per_cu, int front_pc,
                   int scan, double ms) {
    if (!path || !*path) return;
    std::vector<std::string> keep;
    if (FILE *f = fopen(path, "r")) {
        char line[512];
        while (fgets(line, sizeof line, f))
            if (!strstr(line, ("\"key\": \"" + key + "\"").c_str())) keep.push_back(line);
        fclose(f);
    }
    if (FILE *f = fopen(path, "w")) {
        for (auto &l : keep) fputs(l.c_str(), f);
        fprintf(f, "{\"key\": \"%s\", \"sb\": %d, \"per_cu\": %d, \"front_per_cu\": %d, \"scan\": %d, "
                   "\"ms\": %.4f}\n", key.c_str(), sb, per_cu, front_pc, scan, ms);
        fclose(f);
    }
}

}  // namespace

extern "C" {

int bcmc_batch_create(bcmc_volume *const *vols, uint32_t n_vols, const uint32_t *job_vol,
                      const float *job_iso, uint32_t n_jobs, void *hip_stream, bcmc_batch **out) {
    if (!out) return binvalid("null output handle");
    *out = nullptr;
    if (!vols || !job_vol || !job_iso || n_vols == 0 || n_jobs == 0)
        return binvalid("need at least one volume and one job");
    const int f64 = volume_is_f64(vols[0]);
    for (uint32_t v = 0; v < n_vols; v++) {
        if (!vols[v] || volume_is_identity(vols[v])) return binvalid("batch volumes must be compressed volumes");
        if (volume_is_f64(vols[v]) != f64) return binvalid("batch volumes must share one scalar type");
    }
    for (uint32_t j = 0; j < n_jobs; j++) {
        if (job_vol[j] >= n_vols) return binvalid("job volume index out of range");
        if (job_iso[j] != job_iso[j]) return binvalid("NaN isovalue");
    }
    bcmc_batch *b = new (std::nothrow) bcmc_batch();
    if (!b) return BCMC_E_NOMEM;
    b->is_f64 = f64;
    b->n_vols = n_vols;
    b->n_jobs = n_jobs;
    std::vector<BatchVol> hv(n_vols);
    std::vector<uint64_t> gbase(n_vols), jbase(n_jobs);
    std::vector<uint32_t> vol_jobs;
    uint64_t gb = 0;
    for (uint32_t v = 0; v < n_vols; v++) {
        hv[v].g = volume_geom(vols[v]);
        hv[v].stream = volume_stream(vols[v]);
        hv[v].ranges = volume_ranges(vols[v]);
        hv[v].rate = volume_rate(vols[v]);
        hv[v].gbase = gbase[v] = gb;
        gb += hv[v].g.nb;
        hv[v].job_lo = (uint32_t)vol_jobs.size();
        for (uint32_t j = 0; j < n_jobs; j++)
            if (job_vol[j] == v) vol_jobs.push_back(j);
        hv[v].job_hi = (uint32_t)vol_jobs.size();
    }
    uint64_t jb = 0;
    for (uint32_t j = 0; j < n_jobs; j++) {
        jbase[j] = jb;
        jb += hv[job_vol[j]].g.nb;
    }
    b->n_gblocks = gb;
    b->n_jblocks = jb;
    if (gb >= (1ull << 31) || jb >= (1ull << 32)) {
        destroy_batch(b);
        return binvalid("batch too large");
    }
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipDeviceGetAttribute(&b->clock_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess)
        b->clock_khz = 0;
    int pc4 = 0, pcf = 0, pcd = 0;
    if (batch_back_per_cu(4, &pc4) != 0) pc4 = 0;
    for (uint32_t v = 0; v < n_vols; v++)
        b->p.max_vol_jobs = std::max(b->p.max_vol_jobs, hv[v].job_hi - hv[v].job_lo);
    b->p.uniform_rate = hv[0].rate;
    for (uint32_t v = 1; v < n_vols; v++)
        if (hv[v].rate != hv[0].rate) b->p.uniform_rate = 0;
    if (stage_lds_bytes((int)b->p.uniform_rate, f64 != 0) == 0) b->p.uniform_rate = 0;   // not staged
    if (batch_front_per_cu(&pcf) != 0 || pcf < 1 || batch_decode_per_cu(b->p, f64, &pcd) != 0 || pcd < 1) {
        destroy_batch(b);
        return binvalid("the batched kernel cannot be made resident");
    }
    b->front_pc_max = pcf;
    b->decode_grid = grid_for(b, pcd);
    int rc = set_schedule(b, 8, 1 << 30, std::max(1, pcf / 2), 0);
    if (rc) {
        destroy_batch(b);
        return rc;
    }
    unsigned max_grid = (unsigned)(std::max(b->per_cu_max, pc4) * b->cus);
    BatchParams &p = b->p;
    BatchVol *d_vols;
    uint64_t *d_gbase, *d_jbase;
    uint32_t *d_vol_jobs, *d_job_vol;
    float *d_iso;
    if ((rc = balloc(b, &d_vols, n_vols)) || (rc = balloc(b, &d_gbase, n_vols)) ||
        (rc = balloc(b, &d_jbase, n_jobs)) || (rc = balloc(b, &d_vol_jobs, n_jobs)) ||
        (rc = balloc(b, &d_job_vol, n_jobs)) || (rc = balloc(b, &d_iso, n_jobs)) ||
        (rc = balloc(b, &p.I_slot, gb)) || (rc = balloc(b, &p.slots, gb * 64)) ||
        (rc = balloc(b, &p.need, gb)) || (rc = balloc(b, &p.emit_flag, (jb + 3) / 4 * 4)) ||
        (rc = balloc(b, &p.jmask, jb)) ||
        (rc = balloc(b, &p.new_list, gb)) || (rc = balloc(b, &p.list, jb)) ||
        (rc = balloc(b, &p.list_job, jb)) || (rc = balloc(b, &p.cnt, jb)) ||
        (rc = balloc(b, &p.part_new, (uint64_t)pcf * b->cus)) ||
        (rc = balloc(b, &p.part_list, 4ull * pcf * b->cus)) ||
        (rc = balloc(b, &p.part_wave, 4ull * max_grid)) ||
        (rc = balloc(b, &p.job_off, n_jobs + 1)) ||
        (rc = balloc(b, &p.ctr, 1)) || (rc = balloc(b, &p.bar, BAR_WORDS)) ||
        (rc = balloc(b, &p.phase_ts, 9))) {
        destroy_batch(b);
        return rc;
    }
    uint64_t *d_table;
    if ((rc = balloc(b, &d_table, 256))) {
        destroy_batch(b);
        return rc;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    auto fail = [&](hipError_t e) {
        set_error(std::string("batch setup: ") + hipGetErrorString(e));
        destroy_batch(b);
        return BCMC_E_HIP;
    };
    hipError_t e;
    if ((e = hipMemcpy(d_vols, hv.data(), sizeof(BatchVol) * n_vols, hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(d_gbase, gbase.data(), 8 * n_vols, hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(d_jbase, jbase.data(), 8 * n_jobs, hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(d_vol_jobs, vol_jobs.data(), 4 * n_jobs, hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(d_job_vol, job_vol, 4 * n_jobs, hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(d_iso, job_iso, 4 * n_jobs, hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(d_table, mc_table_host(), 256 * 8, hipMemcpyHostToDevice)) ||
        (e = hipMemset(p.emit_flag, 0, (jb + 3) / 4 * 4)) ||   // the padding stays zero
        (e = hipHostMalloc((void **)&b->h_ctr, sizeof(BatchCounters), hipHostMallocDefault)) ||
        (e = hipHostMalloc((void **)&b->h_job_off, 8 * (n_jobs + 1), hipHostMallocDefault)) ||
        (e = hipHostMalloc((void **)&b->h_ts, 9 * sizeof(unsigned long long), hipHostMallocDefault)) ||
        (e = hipStreamCreateWithFlags(&b->gstream, hipStreamNonBlocking)) ||
        (e = hipEventCreate(&b->ev_in)) || (e = hipEventCreate(&b->ev_out)) ||
        (e = hipEventCreate(&b->ev_t0)) || (e = hipEventCreate(&b->ev_t1)))
        return fail(e);
    p.vols = d_vols;
    p.n_vols = n_vols;
    p.n_jobs = n_jobs;
    p.vol_gbase = d_gbase;
    p.vol_jobs = d_vol_jobs;
    p.job_vol = d_job_vol;
    p.job_jbase = d_jbase;
    p.job_iso = d_iso;
    p.n_gblocks = gb;
    p.n_jblocks = jb;
    p.max_slots = gb;
    p.mc_table = d_table;
    if ((rc = reset_cache(b, s))) {
        destroy_batch(b);
        return rc;
    }
    if ((e = hipStreamSynchronize(s))) return fail(e);
    char key[160];
    snprintf(key, sizeof key, "gfx950|%s|jobs=%u|vols=%u|blocks~2^%d", f64 ? "f64" : "f32", n_jobs,
             n_vols, 64 - __builtin_clzll(jb));
    b->key = key;
    int sb = 0, per_cu = 0, front_pc = 0, scan = 0;
    if (load_schedule(getenv("BCMC_AUTOTUNE_CACHE"), b->key, &sb, &per_cu, &front_pc, &scan) &&
        (sb == 4 || sb == 8))
        (void)set_schedule(b, sb, per_cu, front_pc, scan);
    *out = b;
    return BCMC_OK;
}

int bcmc_batch_set_isos(bcmc_batch *b, const float *job_iso, void *hip_stream) {
    if (!b || !job_iso) return binvalid("null argument");
    for (uint32_t j = 0; j < b->n_jobs; j++)
        if (job_iso[j] != job_iso[j]) return binvalid("NaN isovalue");
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    BCMC_HIP_TRY(hipMemcpyAsync(const_cast<float *>(b->p.job_iso), job_iso, 4 * b->n_jobs,
                                hipMemcpyHostToDevice, s));
    BCMC_HIP_TRY(hipStreamSynchronize(s));
    return BCMC_OK;
}

int bcmc_batch_reset(bcmc_batch *b, void *hip_stream) {
    if (!b) return binvalid("null handle");
    return reset_cache(b, reinterpret_cast<hipStream_t>(hip_stream));
}

int bcmc_batch_set_graph(bcmc_batch *b, int on) {
    if (!b) return binvalid("null handle");
    b->use_graph = on ? 1 : 0;
    return BCMC_OK;
}

int bcmc_batch_run(bcmc_batch *b, void *d_out, uint64_t capacity_vertices, uint64_t *h_job_off,
                   void *hip_stream) {
    if (!b || !h_job_off) return binvalid("null argument");
    if (!d_out && capacity_vertices) return binvalid("null output with nonzero capacity");
    int rc = run_once(b, d_out, capacity_vertices, reinterpret_cast<hipStream_t>(hip_stream));
    if (rc) return rc;
    memcpy(h_job_off, b->h_job_off, 8 * (b->n_jobs + 1));
    if (b->h_ctr->total_verts > capacity_vertices) {
        set_error("vertex buffer too small: need " + std::to_string(b->h_ctr->total_verts) + " vertices");
        return BCMC_E_CAPACITY;
    }
    return BCMC_OK;
}

int bcmc_batch_set_schedule(bcmc_batch *b, int stage_blocks, int per_cu, int front_per_cu,
                            int scan_schedule) {
    if (!b) return binvalid("null handle");
    if (stage_blocks != 4 && stage_blocks != 8) return binvalid("stage_blocks must be 4 or 8");
    if (per_cu < 1 || front_per_cu < 1) return binvalid("workgroups per CU must be >= 1");
    if (scan_schedule != 0 && scan_schedule != 1) return binvalid("scan_schedule must be 0 or 1");
    return set_schedule(b, stage_blocks, per_cu, front_per_cu, scan_schedule);
}

int bcmc_batch_tune(bcmc_batch *b, const char *cache_path, void *hip_stream) {
    if (!b) return binvalid("null handle");
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    // size a scratch output from one run
    int rc = reset_cache(b, s);
    if (rc) return rc;
    rc = run_once(b, nullptr, 0, s);
    if (rc) return rc;
    uint64_t need = b->h_ctr->total_verts + 64;
    void *buf = nullptr;
    if (hipMalloc(&buf, need * 16) != hipSuccess) {
        (void)hipGetLastError();
        set_error("no memory for the tuning buffer");
        return BCMC_E_NOMEM;
    }
    int best_sb = b->sb, best_pc = b->per_cu_max, best_fpc = b->front_pc_max, best_scan = 0;
    double best = 1e30;
    // the front kernel's barriers cost more with more workgroups: half and
    // a quarter of what stays resident
    std::vector<int> fpcs = {std::max(1, b->front_pc_max / 2), std::max(1, b->front_pc_max / 4)};
    fpcs.erase(std::unique(fpcs.begin(), fpcs.end()), fpcs.end());
    for (int sb : {4, 8}) {
        int maxc = 0;
        if (batch_back_per_cu(sb, &maxc) != 0 || maxc < 1) continue;
        std::vector<int> pcs = {maxc, std::max(1, maxc - 1), std::max(1, maxc / 2)};
        std::sort(pcs.begin(), pcs.end());
        pcs.erase(std::unique(pcs.begin(), pcs.end()), pcs.end());
        for (int pc : pcs) {
            // each front grid with both scan schedules
            for (size_t fs = 0; fs < 2 * fpcs.size(); fs++) {
                const int fpc = fpcs[fs / 2], scan = (int)(fs % 2);
                if ((rc = set_schedule(b, sb, pc, fpc, scan))) break;
                // median over 5 repetitions of a cold run (empty batch
                // store) + a warm run; a first repetition warms up
                std::vector<double> ts;
                for (int rep = 0; rep < 6 && !rc; rep++) {
                    if ((rc = reset_cache(b, s)) || (rc = run_once(b, buf, need, s))) break;
                    double cold = b->last_ms;
                    if ((rc = run_once(b, buf, need, s))) break;
                    if (rep) ts.push_back(cold + b->last_ms);
                }
                if (rc) break;
                std::sort(ts.begin(), ts.end());
                const double t = ts[ts.size() / 2];
                if (t < best) {
                    best = t;
                    best_sb = sb;
                    best_pc = pc;
                    best_fpc = fpc;
                    best_scan = scan;
                }
            }
            if (rc) break;
        }
        if (rc) break;
    }
    (void)hipFree(buf);
    if (rc) return rc;
    rc = set_schedule(b, best_sb, best_pc, best_fpc, best_scan);
    if (rc) return rc;
    save_schedule(cache_path ? cache_path : getenv("BCMC_AUTOTUNE_CACHE"), b->key, best_sb, best_pc,
                  best_fpc, best_scan, best / 2.0);
    return reset_cache(b, s);
}

int bcmc_batch_get_info(const bcmc_batch *b, bcmc_batch_info *out) {
    if (!b || !out) return binvalid("null argument");
    out->n_volumes = b->n_vols;
    out->n_jobs = b->n_jobs;
    out->n_blocks = b->n_gblocks;
    out->n_job_blocks = b->n_jblocks;
    out->n_resident = b->h_ctr ? b->h_ctr->n_slots : 0;
    out->n_new = b->h_ctr ? b->h_ctr->n_new : 0;
    out->n_pairs = b->h_ctr ? b->h_ctr->n_list : 0;
    out->n_vertices = b->h_ctr ? b->h_ctr->total_verts : 0;
    out->stage_blocks = (uint32_t)b->sb;
    out->grid = b->grid;
    out->workgroups_per_cu = b->grid / (unsigned)std::max(b->cus, 1);
    out->front_grid = b->front_grid;
    out->decode_grid = b->decode_grid;
    out->scan_schedule = b->p.scan_sched;
    out->ran_front_grid = b->h_ctr ? b->h_ctr->grid_front : 0;
    out->ran_decode_grid = b->h_ctr ? b->h_ctr->grid_decode : 0;
    out->ran_grid = b->h_ctr ? b->h_ctr->grid_back : 0;
    out->graph = (b->use_graph && !b->graph_failed && b->exec) ? 1 : 0;
    out->graph_unsupported = b->graph_failed;
    out->last_ms = b->last_ms;
    for (int k = 0; k < 8; k++) out->phase_ms[k] = b->phase_ms[k];
    return BCMC_OK;
}

void bcmc_batch_free(bcmc_batch *b) {
    if (!b) return;
    (void)hipDeviceSynchronize();
    destroy_batch(b);
}

}  // extern "C"
