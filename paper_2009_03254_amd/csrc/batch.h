// Device-side description of a batch (volumes x isovalues) for the batched
// extraction kernels.
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
    unsigned long long slot_base;    // first slot of this run's new blocks
    unsigned int err;
    unsigned int grid_front, grid_decode, grid_back;   // grids the kernels ran with
    unsigned int pad[2];
};

// Grid barrier words (u32 units): the generation, the top-level arrival
// count, the arrival counts of BAR_GROUPS workgroup groups and the finish
// count.  Each word sits on its own 256-byte line so that arrivals on one
// word do not queue behind polls of another.
constexpr int BAR_PAD = 64;
constexpr int BAR_GROUPS = 16;
constexpr int BAR_GEN = 0;
constexpr int BAR_TOP = BAR_PAD;
constexpr int BAR_DONE = 2 * BAR_PAD;
constexpr int BAR_SUB = 3 * BAR_PAD;
constexpr int BAR_WORDS = BAR_SUB + BAR_GROUPS * BAR_PAD;

struct BatchParams {
    const BatchVol *vols;
    uint32_t n_vols, n_jobs;
    const uint64_t *vol_gbase;   // [n_vols]
    const uint32_t *vol_jobs;    // jobs grouped by volume
    const uint32_t *job_vol;     // [n_jobs]
    const uint64_t *job_jbase;   // [n_jobs] first (job, block) index of each job
    const float *job_iso;        // [n_jobs] (device, so a captured graph follows updates)
    uint64_t n_gblocks, n_jblocks, max_slots;
    uint32_t uniform_rate;       // the rate of every volume when they share one <= 16, else 0
    uint32_t max_vol_jobs;       // most jobs of one volume
    uint32_t scan_sched;         // offsets of the front kernel's lists: 0 = workgroup 0 scans the
                                 // counts, then a grid barrier; 1 = every workgroup sums the
                                 // counts before its own (no barrier)
    int32_t *I_slot;             // [n_gblocks] slot of each global block or -1
    float *slots;                // [max_slots][64]
    uint8_t *need;               // [n_gblocks] 0 unused, 1 used and new, 2 used and resident
    uint8_t *emit_flag;          // [n_jblocks rounded up to 4] (padding zero)
    uint64_t *jmask;             // [n_jblocks] sign masks of the used blocks per job
    uint32_t *new_list;          // [n_gblocks]
    uint32_t *list;              // [n_jblocks] (job-major, block-ascending)
    uint32_t *list_job;          // [n_jblocks] job of each list entry
    uint32_t *cnt;               // [n_jblocks] vertex count of each list entry
    uint64_t *part_new;          // [front grid] per-workgroup new blocks, then offsets
    uint64_t *part_list;         // [front grid * 4] per-wave pairs, then offsets
    uint64_t *part_wave;         // [back grid * 4] per-wave vertex counts, then offsets
    uint64_t *job_off;           // [n_jobs + 1] vertex offsets of the jobs' soups
    const uint64_t *mc_table;
    void *out;
    uint64_t cap;
    BatchCounters *ctr;
    unsigned int *bar;           // [BAR_WORDS] grid barrier
    unsigned long long *phase_ts;  // [9] real-time clock at the phase boundaries
};

// Resident workgroups per CU of the front kernel (flags and lists), the
// decode kernel (decode and sign masks) and the back kernel (count, scan,
// emission; `sb` blocks staged per wave round trip).
int batch_front_per_cu(int *per_cu);
int batch_decode_per_cu(const BatchParams &p, int is_f64, int *per_cu);
int batch_back_per_cu(int sb, int *per_cu);
// Launches the three kernels with grids[0..2] workgroups.  cooperative = 1:
// the persistent front and back kernels by hipLaunchCooperativeKernel
// (residency guaranteed by the runtime); 0: plain launches (for graph
// capture; each grid never exceeds the resident capacity and the barriers
// are bounded).
hipError_t launch_batch(const BatchParams &p, int is_f64, int sb, const unsigned grids[3],
                        hipStream_t s, int cooperative);

}  // namespace bcmc
