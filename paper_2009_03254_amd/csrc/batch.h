// Device-side description of a batch (volumes x isovalues) for the batched
// persistent extraction kernel.
#pragma once

#include <stdint.h>

#include "common.h"

namespace bcmc {

struct BatchVol {
    Geom g;
    const uint64_t *stream;   // fixed-rate ZFP words of the volume
    const float2 *ranges;     // its block ranges
    uint32_t rate;
    uint32_t job_lo, job_hi;  // its jobs: vol_jobs[job_lo .. job_hi)
    uint64_t gbase;           // first global block id of the volume
};

struct BatchCounters {
    unsigned long long n_slots;      // decoded blocks resident (persists across runs)
    unsigned long long n_new;        // blocks decoded by this run
    unsigned long long n_list;       // (job, block) pairs that may emit
    unsigned long long total_verts;
    unsigned int err;
    unsigned int pad[7];
};

struct BatchParams {
    const BatchVol *vols;
    uint32_t n_vols, n_jobs;
    const uint64_t *vol_gbase;   // [n_vols]
    const uint32_t *vol_jobs;    // jobs grouped by volume
    const uint32_t *job_vol;     // [n_jobs]
    const uint64_t *job_jbase;   // [n_jobs] first (job, block) index of each job
    const float *job_iso;        // [n_jobs] (device, so a captured graph follows updates)
    uint64_t n_gblocks, n_jblocks, max_slots;
    int32_t *I_slot;             // [n_gblocks] slot of each global block or -1
    float *slots;                // [max_slots][64]
    uint8_t *need;               // [n_gblocks]
    uint8_t *emit_flag;          // [n_jblocks]
    uint32_t *new_list;          // [n_gblocks]
    uint32_t *list;              // [n_jblocks] (job-major, block-ascending)
    uint32_t *list_job;          // [n_jblocks] job of each list entry
    uint32_t *cnt;               // [n_jblocks]
    uint64_t *off;               // [n_jblocks]
    uint64_t *part_new, *part_list;  // [grid]
    uint64_t *job_first;         // [n_jobs]
    uint64_t *job_off;           // [n_jobs + 1] vertex offsets of the jobs' soups
    const uint64_t *mc_table;
    void *out;
    uint64_t cap;
    BatchCounters *ctr;
    unsigned int *bar;           // [2] grid barrier: arrivals, generation
    unsigned long long *phase_ts;  // [9] real-time clock at the start and after each phase
};

int batch_max_grid(int is_f64, int sb, int *per_cu);
// cooperative = 1: hipLaunchCooperativeKernel (residency guaranteed by the
// runtime); 0: plain launch (for graph capture; the grid never exceeds the
// resident capacity and the barriers are bounded).
hipError_t launch_batch(const BatchParams &p, int is_f64, int sb, unsigned grid, hipStream_t s,
                        int cooperative);

}  // namespace bcmc
