#!/usr/bin/env python3
"""Benchmark of the block-compressed isosurface extraction path on one MI355X.

Headline workload (the largest configuration that fits one GPU): a
5120 x 3840 x 768 float64 channel-flow-like field (tanh mean profile in y plus
Fourier turbulence of 0.1 relative amplitude, seed 5), generated and
fixed-rate ZFP-encoded at 2 bits/value slab by slab on the GPU (3.8 GB of
compressed words resident in HBM before timing), isovalue 0.5, LRU block cache
capped at 64 GiB of decoded float32.  One step = one cold extraction: cull,
cache update, decode of every needed block, marching cubes count and emission,
triangle-count readback (paper Sec. 4).  Before each step, outside its
timing, the cache is emptied and the 256 MB last-level cache is flushed by a
1 GiB write.  `value` = triangles per second over the timed steps.

Extra keys: the 512^3 turbulence call sequence (cold p50, p90, warm p50,
repeat p50), its 8-byte record variants, the differentiable form, the batched
form, and the oracle timed on a bounded sample on one host core.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E peak, GB/s
RATE = 8                # the 512^3 turbulence workload
FLUSH_BYTES = 1 << 30   # write that evicts the 256 MB last-level cache


# Sources of the single-volume kernels, hashed to tell whether the committed
# traffic counters were taken on the kernels as they are now.
KERNEL_SOURCES = ("common.h", "mc_device.h", "zfp_device.h", "extract.hip", "zfp.hip", "tables.cpp",
                  "gen_ntri.cpp")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "path_channelflow_f64_rate2_hbm_counters.md")
COUNTERS_FILE_512 = os.path.join(ROOT, "profiles", "path_turbulence512_rate8_hbm_counters.md")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2009_03254_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, counters_file=None):
    """HBM bytes per dispatch of `kernel` from a committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (copy-calibrated), or None when there is
    none or the kernel sources changed since it was taken."""
    import re
    try:
        text = open(counters_file or COUNTERS_FILE).read()
    except OSError:
        return None
    m = re.search(rf"^traffic {re.escape(kernel)} bytes_per_dispatch=(\d+) sources_sha256=(\w+)$",
                  text, re.M)
    if not m or m.group(2) != sources_sha256():
        return None
    return int(m.group(1))


def host_cpu():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def flush_last_level_cache(buf):
    """One write of FLUSH_BYTES: evicts the 256 MB last-level cache (and L2)."""
    buf.fill_(float(time.perf_counter_ns() & 0xFFFF))


def cpu_baseline_oracle(words_np, dims, rate, is_f64, iso, sample):
    """The oracle as it stands (decode every block, plain marching cubes over
    every cell), single-threaded, on a bounded sample: the first z-planes of
    the same stream given by `dims`."""
    import oracle
    oracle.build(force=False)
    t0 = time.perf_counter()
    blocks = oracle.zfp_decode(words_np, dims, rate, is_f64)
    r = oracle.mc_extract(blocks, dims, iso, want=("verts", "vblock"))
    dt = time.perf_counter() - t0
    model, nproc = host_cpu()
    return {
        "value": r["T"] / dt,
        "unit": "triangles/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{sample}: decode-all + plain MC of {dims[0]}x{dims[1]}x{dims[2]} "
                  f"({oracle.num_blocks(*dims)} blocks, {r['T']} triangles), {dt:.2f} s",
        "seconds": round(dt, 3),
        "cpu_model": model,
        "nproc": nproc,
    }


# Per-kernel algorithmic bytes (SURVEY-defined per-unit figures, no
# bookkeeping) of the stages that hold one kernel each, from a call's stats:
# stage 2 = assign + decode of the new blocks, stage 5 = emission.
def kernel_defs(rate):
    return {
        "k_assign_decode": (2, lambda st: st["n_new"] * (8.0 * rate + 256.0),
                            lambda st: st["n_new"] > 0),
        "k_mc_emit": (5, lambda st: 256.0 * st["n_occupied"] + 24.0 * st["n_triangles"],
                      lambda st: True),
    }


def kstats(recs, stage, bytes_fn, live_fn):
    """Totals over call records (seconds, stats) of one stage's event times."""
    ms = sum(r[1]["stage_ms"][stage] for r in recs if live_fn(r[1]))
    nbytes = sum(bytes_fn(r[1]) for r in recs if live_fn(r[1]))
    launches = sum(1 for r in recs if live_fn(r[1]))
    return {"total_ms": ms, "bytes": nbytes, "launches": max(launches, 1),
            "avg_ms": ms / max(launches, 1),
            "gbs": nbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0}


def stage_medians(recs):
    import numpy as np
    return [round(float(np.median([r[1]["stage_ms"][i] for r in recs])), 4) for i in range(8)]


def differentiable_bench(steps, warmup):
    """256^3 Gaussian blobs (16 blobs, seed 3), iso 0.5: forward extract and
    forward + backward of L = sum_j (|v_j - c| - 64)^2 (c = grid centre)
    through torch.autograd, against the plain extract of the same field
    compressed at rate 16 with a warm cache.  Medians of `steps` runs."""
    import numpy as np
    import torch

    import paper_2009_03254_amd as bcmc
    from synthetic import fields

    n = 256
    dims = (n, n, n)
    f = torch.from_numpy(fields.gaussian_blobs(n, 16, seed=3)).cuda()
    blocks = bcmc.blocks_from_field(f)
    words = bcmc.encode(f, 16)
    vol = bcmc.Volume(words, dims, "f32", 16)
    iso = 0.5
    c = torch.full((3,), (n - 1) / 2.0, dtype=torch.float64, device="cuda")

    def timed(fn):
        ts = []
        for k in range(warmup + steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            if k >= warmup:
                ts.append(time.perf_counter() - t0)
        return float(np.median(ts)) * 1e3, r

    out = torch.empty((1, 4), dtype=torch.int32, device="cuda")
    _, T = vol.extract_into(iso, out)
    out = torch.empty((3 * T + 64, 4), dtype=torch.int32, device="cuda")
    plain_ms, _ = timed(lambda: vol.extract_into(iso, out))
    # the plain extract of the very field the differentiable form sees
    fv = bcmc.FieldVolume(blocks, dims)
    _, T_field = fv.extract_into(iso, out)
    plain_field_ms, _ = timed(lambda: fv.extract_into(iso, out))
    fv.close()
    bl = blocks.clone().requires_grad_(True)
    iso_t = torch.tensor(iso, device="cuda", requires_grad=True)

    def fwd():
        with torch.no_grad():
            return bcmc.ExtractFn.apply(bl, iso_t, dims)

    def fwd_bwd():
        bl.grad = None
        iso_t.grad = None
        xyz, blk = bcmc.ExtractFn.apply(bl, iso_t, dims)
        g = bcmc.global_positions(xyz, blk, dims, dtype=torch.float64)
        loss = ((g - c).norm(dim=1) - 64.0).pow(2).sum()
        loss.backward()
        return loss

    fwd_ms, _ = timed(fwd)
    fb_ms, _ = timed(fwd_bwd)
    vol.close()
    return {
        "workload": "gaussian blobs 256^3 f32 (16 blobs, seed 3), iso 0.5, "
                    "L = sum (|v - c| - 64)^2 over all soup vertices",
        "triangles": T_field,
        "plain_extract_ms": round(plain_field_ms, 4),
        "plain_extract_compressed_ms": round(plain_ms, 4),
        "fwd_ms": round(fwd_ms, 4),
        "fwd_bwd_ms": round(fb_ms, 4),
        "fwd_vs_plain": round(fwd_ms / plain_field_ms, 3),
        "fwd_bwd_vs_plain": round(fb_ms / plain_field_ms, 3),
        "note": "plain = bcmc_extract of the same uncompressed field (identity cache); "
                "plain_extract_compressed = the field at ZFP rate 16 with a warm cache; fwd / "
                "fwd+bwd through torch.autograd on the field (loss in float64 torch ops "
                "included); medians, host-timed",
    }


def batch_bench(steps, warmup):
    """48 volumes (dims from seed 4, each axis uniform in [32, 256]), each a
    turbulence field (seed 4000 + v, 256 modes) at ZFP rate 8, isovalues at the
    20/40/60/80th percentiles of its field: all 192 (volume, isovalue) jobs in
    one persistent launch replayed from a hipGraph with the autotuned
    schedule, against the same jobs run as 192 plain single-volume extracts.
    Medians of `steps` runs, cold (empty caches) and warm."""
    import numpy as np
    import torch

    import paper_2009_03254_amd as bcmc
    from synthetic import fields

    dims_list = fields.batched_dims(48, seed=4, lo=32, hi=256)
    vols, jobs = [], []
    for v, (nx, ny, nz) in enumerate(dims_list):
        f = fields.turbulence_torch(nx, ny, nz, seed=4000 + v, device="cuda")
        isos = [fields.percentile_iso_torch(f, p) for p in (20, 40, 60, 80)]
        vols.append(bcmc.Volume(bcmc.encode(f, RATE), (nx, ny, nz), "f32", RATE))
        jobs += [(v, float(i)) for i in isos]
        del f
    torch.cuda.empty_cache()
    batch = bcmc.Batch(vols, jobs)
    batch.tune()
    verts, offs = batch.run()
    total_v = int(offs[-1])
    out = torch.empty((total_v + 1024, 4), dtype=torch.int32, device="cuda")

    def timed(fn):
        ts = []
        for k in range(warmup + steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            if k >= warmup:
                ts.append(time.perf_counter() - t0)
        return float(np.median(ts)) * 1e3

    gpu_ms = {"cold": [], "warm": []}
    phases = {"cold": [], "warm": []}

    def batch_run(kind):
        rc, o = batch.run_into(out)
        if rc != 0 or int(o[-1]) != total_v:
            raise bcmc.BcmcError(rc, bcmc.lib().bcmc_last_error().decode())
        inf = batch.info()
        gpu_ms[kind].append(inf["last_ms"])
        phases[kind].append(inf["phase_ms"])

    def batch_cold():
        batch.reset()
        batch_run("cold")

    cold_ms = timed(batch_cold)
    info_cold = batch.info()
    warm_ms = timed(lambda: batch_run("warm"))
    info = batch.info()

    alg = {"cold": 0.0, "warm": 0.0}
    plain_T = {"cold": 0, "warm": 0}

    def plain(kind, collect=False):
        tris, nbytes = 0, 0.0
        for v, vol in enumerate(vols):
            if kind == "cold":
                vol.reset_cache()
            for vi, iso in jobs[4 * v: 4 * v + 4]:
                rc, T = vol.extract_into(iso, out)
                if rc != 0:
                    raise bcmc.BcmcError(rc, bcmc.lib().bcmc_last_error().decode())
                if collect:
                    tris += T
                    nbytes += vol.stats()["alg_bytes"]
        if collect:
            alg[kind], plain_T[kind] = nbytes, tris

    plain("cold", collect=True)
    plain("warm", collect=True)
    plain_cold_ms = timed(lambda: plain("cold"))
    plain_warm_ms = timed(lambda: plain("warm"))
    if 3 * plain_T["cold"] != total_v or 3 * plain_T["warm"] != total_v:
        raise RuntimeError("batched and plain extraction disagree on the vertex count")
    T = total_v // 3
    batch.close()
    for v in vols:
        v.close()
    n_blocks = sum(bcmc.num_blocks(*d) for d in dims_list)
    return {
        "workload": "48 turbulence volumes f32 (dims seed 4, axes U[32,256]; field seed 4000+v), "
                    "ZFP rate 8, iso p20/p40/p60/p80 per volume: 192 jobs",
        "n_blocks": n_blocks, "triangles": T,
        "schedule": {"stage_blocks": info["stage_blocks"], "grid": info["grid"],
                     "workgroups_per_cu": info["workgroups_per_cu"],
                     "front_grid": info["front_grid"], "scan_schedule": info["scan_schedule"],
                     "graph": info["graph"]},
        "cold": {"batch_ms": round(cold_ms, 4),
                 "batch_gpu_ms": round(float(np.median(gpu_ms["cold"])), 4),
                 "phase_ms": [round(float(x), 4) for x in np.median(np.array(phases["cold"]), axis=0)],
                 "plain_ms": round(plain_cold_ms, 4),
                 "speedup_vs_plain": round(plain_cold_ms / cold_ms, 3),
                 "triangles_per_s": round(T / (cold_ms * 1e-3)),
                 "alg_gbs": round(alg["cold"] / (cold_ms * 1e-3) / 1e9, 2),
                 "n_new": info_cold["n_new"]},
        "warm": {"batch_ms": round(warm_ms, 4),
                 "batch_gpu_ms": round(float(np.median(gpu_ms["warm"])), 4),
                 "phase_ms": [round(float(x), 4) for x in np.median(np.array(phases["warm"]), axis=0)],
                 "plain_ms": round(plain_warm_ms, 4),
                 "speedup_vs_plain": round(plain_warm_ms / warm_ms, 3),
                 "triangles_per_s": round(T / (warm_ms * 1e-3)),
                 "alg_gbs": round(alg["warm"] / (warm_ms * 1e-3) / 1e9, 2)},
        "note": "alg_gbs = the algorithmic bytes of the 192 plain calls over the batch's time; "
                "ms are wall-clock per pass including the offsets readback; phase_ms: reset, "
                "flags, counts scan, list scatter, decode, count, count scan, emission",
    }



def channel_flow_volume():
    """The 5120 x 3840 x 768 float64 channel flow, encoded at rate 2 slab by
    slab on the GPU: (Volume, words kept for the CPU sample, seconds)."""
    import torch

    import paper_2009_03254_amd as bcmc
    from synthetic import fields

    rate = 2
    nx, ny, nz = fields.CHANNEL_FLOW_DIMS
    nb = bcmc.num_blocks(nx, ny, nz)
    words = torch.empty(nb * rate, dtype=torch.uint64, device="cuda")
    per_layer = (nx // 4) * (ny // 4)
    t0 = time.perf_counter()
    for z0 in range(0, nz, 32):
        f = fields.channel_flow_slab(z0, min(nz, z0 + 32))
        w = bcmc.encode(f, rate)
        first = (z0 // 4) * per_layer * rate
        words[first: first + w.numel()] = w
        del f, w
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    # the CPU sample: the words of the first two block layers (8 z-planes)
    sample = words[: 2 * per_layer * rate].view(torch.int64).cpu().numpy().view("uint64").copy()
    vol = bcmc.Volume(words, (nx, ny, nz), "f64", rate)
    del words
    torch.cuda.empty_cache()
    vol.set_cache_budget(initial_bytes=0, max_bytes=64 << 30)
    return vol, sample, gen_s


def headline(args):
    """Cold extractions of the channel flow: warm-up, profiled steps (events
    around every stage: the breakdown and the dominant kernel), then the
    timed steps with events around the dominant kernel's stage only."""
    import numpy as np
    import torch

    import paper_2009_03254_amd as bcmc
    from synthetic import fields

    rate = 2
    nx, ny, nz = fields.CHANNEL_FLOW_DIMS
    iso = 0.5
    log(f"[bench] channel flow {nx}x{ny}x{nz} f64: generating and encoding at rate {rate} on the GPU")
    vol, sample_words, gen_s = channel_flow_volume()
    nb = vol.n_blocks
    probe = torch.empty((1, 4), dtype=torch.int32, device="cuda")
    _, T = vol.extract_into(iso, probe)
    out = torch.empty((3 * T + 64, 4), dtype=torch.int32, device="cuda")
    flush_buf = torch.empty(FLUSH_BYTES // 4, dtype=torch.float32, device="cuda")
    bufs = {"f32": out}

    def call(cold, record, fmt="f32"):
        if cold:
            vol.reset_cache()
            flush_last_level_cache(flush_buf)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, T2 = vol.extract_into(iso, bufs[fmt])      # synchronises to read the count
        dt = time.perf_counter() - t0
        if rc != 0 or T2 != T:
            raise bcmc.BcmcError(rc, bcmc.lib().bcmc_last_error().decode())
        record.append((dt, vol.stats()))

    kdefs = kernel_defs(rate)
    for _ in range(args.warmup):
        call(True, [])
    vol.set_profiling(True)
    prof = []
    for _ in range(args.steps):
        call(True, prof)
    vol.set_profiling(False)
    kern = {k: kstats(prof, *d) for k, d in kdefs.items()}
    dom = max(kern, key=lambda k: kern[k]["total_ms"])
    if not args.no_profile_events:
        vol.set_profiling(True, stages=[kdefs[dom][0]])
    recs = []
    torch.cuda.synchronize()
    t_region = time.perf_counter()
    for _ in range(args.steps):
        call(True, recs)
    torch.cuda.synchronize()
    region_s = time.perf_counter() - t_region
    vol.set_profiling(False)
    kd = kstats(recs, *kdefs[dom]) if not args.no_profile_events else kern[dom]

    # the same cold steps writing 8-byte records: the paper's 10-bit vertex
    # (Sec. 4.5) and this library's edge record
    formats = {}
    for fmt in ("q10", "edge8"):
        vol.set_vertex_format(fmt)
        bufs[fmt] = torch.empty(3 * T + 64, dtype=torch.int64, device="cuda")
        for _ in range(args.warmup):
            call(True, [], fmt)
        vol.set_profiling(True, stages=[5])
        r8 = []
        for _ in range(args.steps):
            call(True, r8, fmt)
        vol.set_profiling(False)
        e8 = kstats(r8, *kdefs["k_mc_emit"])
        t8 = sum(r[0] for r in r8)
        formats[fmt] = {"triangles_per_s": round(T * len(r8) / t8), "ms_per_step": round(t8 / len(r8) * 1e3, 4),
                        "k_mc_emit_avg_ms": round(e8["avg_ms"], 5),
                        "k_mc_emit_frac": round(e8["gbs"] / HBM_PEAK_GBS, 4)}
        del bufs[fmt]
    vol.set_vertex_format("f32")

    # warm repeats for context
    call(True, [])
    warm, warm_prof = [], []
    for _ in range(args.steps):
        call(False, warm)
    vol.set_profiling(True)
    for _ in range(args.steps):
        call(False, warm_prof)
    vol.set_profiling(False)
    vol.close()

    ext_s = sum(r[0] for r in recs)
    st = recs[-1][1]
    ms = ext_s / len(recs) * 1e3
    alg = st["alg_bytes"]
    alg_no_rt = alg - 8.0 * nb
    warm_ms = float(np.mean([r[0] for r in warm])) * 1e3
    wst = warm[-1][1]
    gpu_ms = float(np.mean([r[1]["stage_ms"][7] for r in prof]))
    result = {
        "metric": "triangles/sec + HBM GB/s for decompress+extract",
        "value": T * len(recs) / ext_s,
        "unit": "triangles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 stream, f32 decoded",
        "data": "synthetic",
        "config": {
            "workload": f"channel flow {nx}x{ny}x{nz} f64 (tanh profile + 0.1 Fourier "
                        "turbulence, seed 5), ZFP rate 2, iso 0.5, cache cap 64 GiB; "
                        "step = one cold extract",
            "n_blocks": nb, "iso": iso, "parallelism": "single GPU",
        },
        "triangles": T,
        "hbm_gbs_alg": round(alg / (ms * 1e-3) / 1e9, 2),
        "hbm_frac_alg": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "hbm_gbs_alg_without_range_table": round(alg_no_rt / (ms * 1e-3) / 1e9, 2),
        "roofline": {
            "bound": "hbm", "kernel": dom, "achieved": round(kd["gbs"], 2),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(kd["gbs"] / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(dom), "avg_launch_ms": round(kd["avg_ms"], 5),
            "launches": kd["launches"],
            "alg_bytes_per_launch": round(kd["bytes"] / kd["launches"]),
        },
        "kernels": {k: {"avg_ms": round(v["avg_ms"], 5), "alg_gbs": round(v["gbs"], 1),
                        "frac": round(v["gbs"] / HBM_PEAK_GBS, 4),
                        "share_of_gpu_time": round(v["total_ms"] / max(gpu_ms * len(prof), 1e-9), 3)}
                    for k, v in kern.items()},
        "cold": {"n_active": st["n_active"], "n_new": st["n_new"], "n_occupied": st["n_occupied"],
                 "n_candidates": st["n_candidates"], "gpu_ms": round(gpu_ms, 4),
                 "stage_ms": stage_medians(prof),
                 "timed_region_s": round(region_s, 4),
                 "wall_ms_per_step": round(region_s / args.steps * 1e3, 4)},
        "warm": {"ms": round(warm_ms, 4), "triangles_per_s": round(T / (warm_ms * 1e-3)),
                 "alg_gbs": round(wst["alg_bytes"] / (warm_ms * 1e-3) / 1e9, 2),
                 "alg_gbs_without_range_table": round((wst["alg_bytes"] - 8.0 * nb)
                                                      / (warm_ms * 1e-3) / 1e9, 2),
                 "n_new": wst["n_new"], "stage_ms": stage_medians(warm_prof)},
        "formats": dict(formats, note="the same cold steps writing 8-byte records: q10 = the "
                        "paper's vertex (10-bit block-relative coordinates + block id, within "
                        "2/1023 voxel); edge8 = edge records within 2^-23 voxel"),
        "generate_encode_s": round(gen_s, 2),
        "note": "ms_per_step / value: host-timed cold extract calls (count readback included); "
                "the cache reset and the 1 GiB cache flush before each step are outside that "
                "time (wall_ms_per_step includes them); stage_ms: [cull+compaction, cache "
                "update, assign+decode, masks+count, -, emission, -, total] from HIP events "
                "in separate profiled steps",
    }
    return result, sample_words


def turbulence512(args):
    """The 512^3 turbulence call sequence (empty cache -> p50 cold -> p90 ->
    p50 warm -> p50 repeat, initial cache 25% of the blocks), 16-byte
    records, then 8-byte edge records."""
    import numpy as np
    import torch

    import paper_2009_03254_amd as bcmc
    from synthetic import fields

    n = 512
    dims = (n, n, n)
    dev = torch.device("cuda:0")
    log(f"[bench] {n}^3 turbulence: generating and encoding at rate {RATE} on the GPU")
    field = fields.turbulence_torch(n, seed=2, device=dev)
    words = bcmc.encode(field, RATE)
    del field
    vol = bcmc.Volume(words, dims, "f32", RATE)
    nb = vol.n_blocks
    vol.set_cache_budget(initial_bytes=(nb // 4) * 256, max_bytes=0)
    D = vol.decode_all()
    iso50 = fields.percentile_iso_torch(D, 50)
    iso90 = fields.percentile_iso_torch(D, 90)
    del D
    torch.cuda.empty_cache()
    flush_buf = torch.empty(FLUSH_BYTES // 4, dtype=torch.float32, device=dev)
    out = torch.empty((1, 4), dtype=torch.int32, device=dev)
    cap_T = 0
    for iso in (iso50, iso90):
        rc, T = vol.extract_into(float(iso), out)
        cap_T = max(cap_T, T)
    out = torch.empty((3 * cap_T + 1024, 4), dtype=torch.int32, device=dev)
    seq = (("cold_p50", iso50), ("p90", iso90), ("warm_p50", iso50), ("repeat_p50", iso50))

    def step(record, buf=None):
        buf = out if buf is None else buf
        vol.reset_cache()
        flush_last_level_cache(flush_buf)
        for name, iso in seq:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, T = vol.extract_into(float(iso), buf)
            dt = time.perf_counter() - t0
            if rc != 0:
                raise bcmc.BcmcError(rc, bcmc.lib().bcmc_last_error().decode())
            record.append((name, dt, vol.stats()))

    def as2(recs):
        return [(r[1], r[2]) for r in recs]

    kdefs = kernel_defs(RATE)
    for _ in range(args.warmup):
        step([])
    vol.set_profiling(True)
    prof = []
    for _ in range(args.steps):
        step(prof)
    vol.set_profiling(False)
    kern = {k: kstats(as2(prof), *d) for k, d in kdefs.items()}
    dom = max(kern, key=lambda k: kern[k]["total_ms"])
    if not args.no_profile_events:
        vol.set_profiling(True, stages=[kdefs[dom][0]])
    recs = []
    for _ in range(args.steps):
        step(recs)
    vol.set_profiling(False)
    kd = kstats(as2(recs), *kdefs[dom]) if not args.no_profile_events else kern[dom]
    ext_s = sum(r[1] for r in recs)
    tris = sum(r[2]["n_triangles"] for r in recs)
    alg = sum(r[2]["alg_bytes"] for r in recs)
    calls = []
    for name, _ in seq:
        rs = [r for r in recs if r[0] == name]
        ps = [r for r in prof if r[0] == name]
        st = rs[-1][2]
        ms = float(np.median([r[1] for r in rs]) * 1e3)
        calls.append({
            "call": name, "ms": round(ms, 4), "triangles": st["n_triangles"],
            "n_active": st["n_active"], "n_new": st["n_new"], "n_slots": st["n_slots"],
            "n_occupied": st["n_occupied"], "n_candidates": st["n_candidates"],
            "hit_rate": round(st["hit_rate"], 4),
            "alg_gbs": round(st["alg_bytes"] / (ms * 1e-3) / 1e9, 2),
            "stage_ms": stage_medians([(r[1], r[2]) for r in ps]),
        })
    res = {
        "workload": f"turbulence {n}^3 f32 (256 Fourier modes, k^-5/3), ZFP rate {RATE}, iso "
                    "p50/p90, initial cache 25% of blocks; step = cold p50 (after a cache "
                    "flush), p90, warm p50, repeat p50",
        "n_blocks": nb, "iso_p50": float(iso50), "iso_p90": float(iso90),
        "triangles_per_s": round(tris / ext_s), "ms_per_step": round(ext_s / args.steps * 1e3, 4),
        "hbm_gbs_alg": round(alg / ext_s / 1e9, 2),
        "roofline": {"kernel": dom, "achieved": round(kd["gbs"], 2),
                     "frac": round(kd["gbs"] / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(dom, COUNTERS_FILE_512),
                     "avg_launch_ms": round(kd["avg_ms"], 5), "launches": kd["launches"],
                     "alg_bytes_per_launch": round(kd["bytes"] / kd["launches"])},
        "kernels": {k: {"avg_ms": round(v["avg_ms"], 5), "alg_gbs": round(v["gbs"], 1),
                        "frac": round(v["gbs"] / HBM_PEAK_GBS, 4)} for k, v in kern.items()},
        "calls": calls,
    }
    # the same steps with 8-byte edge records
    vol.set_vertex_format("edge8")
    out8 = torch.empty(3 * cap_T + 1024, dtype=torch.int64, device=dev)
    for _ in range(args.warmup):
        step([], out8)
    vol.set_profiling(True, stages=[5])
    rec8 = []
    for _ in range(args.steps):
        step(rec8, out8)
    vol.set_profiling(False)
    vol.set_vertex_format("f32")
    e = kstats(as2(rec8), *kernel_defs(RATE)["k_mc_emit"])
    t8 = sum(r[1] for r in rec8)
    res["edge8"] = {
        "triangles_per_s": round(sum(r[2]["n_triangles"] for r in rec8) / t8),
        "ms_per_step": round(t8 / args.steps * 1e3, 4),
        "k_mc_emit_avg_ms": round(e["avg_ms"], 5), "k_mc_emit_frac": round(e["gbs"] / HBM_PEAK_GBS, 4),
        "note": "8-byte edge records (block, cell, edge, 22-bit t): positions within 2^-23 "
                "voxel of the float32 soup",
    }
    # the same steps with the paper's 10-bit vertices, and their error against
    # the float32 soup of the same call
    vol.set_vertex_format("q10")
    for _ in range(args.warmup):
        step([], out8)
    vol.set_profiling(True, stages=[5])
    rq = []
    for _ in range(args.steps):
        step(rq, out8)
    vol.set_profiling(False)
    e = kstats(as2(rq), *kernel_defs(RATE)["k_mc_emit"])
    tq = sum(r[1] for r in rq)
    rc, Tq = vol.extract_into(float(iso50), out8)
    vol.set_vertex_format("f32")
    rc, T16 = vol.extract_into(float(iso50), out)
    pos, _ = bcmc.q10_positions(out8[: 3 * Tq])
    xyz, _ = bcmc.split_vertices(out[: 3 * T16])
    qerr = float((pos - xyz).abs().max()) if Tq == T16 else None
    res["q10"] = {
        "triangles_per_s": round(sum(r[2]["n_triangles"] for r in rq) / tq),
        "ms_per_step": round(tq / args.steps * 1e3, 4),
        "k_mc_emit_avg_ms": round(e["avg_ms"], 5), "k_mc_emit_frac": round(e["gbs"] / HBM_PEAK_GBS, 4),
        "max_dequantisation_error_voxel": qerr,
        "note": "the paper's 8-byte vertex (Sec. 4.5): 10-bit block-relative coordinates + block "
                "id; error = largest |dequantised - float32 vertex| over the p50 soup",
    }
    del out8
    vol.close()
    return res


def zfp_throughput(reps=10):
    """Whole-volume fixed-rate ZFP throughput on the 512^3 float32 turbulence
    field at rates 2, 4 and 8 (the paper's decompression benchmark, Sec.
    3.3.4): encode (field -> stream) and decode of every block (stream ->
    [N_b][64] float32 + block ranges), each the mean of `reps` runs after one
    untimed run, timed with HIP events on the stream."""
    import torch

    import paper_2009_03254_amd as bcmc
    from synthetic import fields

    n = 512
    dims = (n, n, n)
    field = fields.turbulence_torch(n, seed=2, device="cuda")
    nb = bcmc.num_blocks(*dims)
    blocks = torch.empty((nb, 64), dtype=torch.float32, device="cuda")
    out = {}
    for rate in (2, 4, 8):
        words = bcmc.encode(field, rate)
        vol = bcmc.Volume(words, dims, "f32", rate)

        def timed(fn):
            fn()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            torch.cuda.synchronize()
            ev[0].record()
            for _ in range(reps):
                fn()
            ev[1].record()
            torch.cuda.synchronize()
            return ev[0].elapsed_time(ev[1]) / reps

        dec_ms = timed(lambda: vol.decode_all(blocks))
        enc_ms = timed(lambda: bcmc.encode(field, rate, out=words))
        dec_bytes = nb * (8.0 * rate + 256.0 + 8.0)   # stream read, blocks and ranges written
        enc_bytes = nb * (256.0 + 8.0 * rate)
        out[f"rate{rate}"] = {
            "decode_ms": round(dec_ms, 4),
            "decode_gbs_decompressed": round(nb * 256.0 / (dec_ms * 1e-3) / 1e9, 1),
            "decode_hbm_gbs": round(dec_bytes / (dec_ms * 1e-3) / 1e9, 1),
            "decode_frac": round(dec_bytes / (dec_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "decode_gblocks_per_s": round(nb / (dec_ms * 1e-3) / 1e9, 3),
            "encode_ms": round(enc_ms, 4),
            "encode_gbs_uncompressed": round(nb * 256.0 / (enc_ms * 1e-3) / 1e9, 1),
            "encode_hbm_gbs": round(enc_bytes / (enc_ms * 1e-3) / 1e9, 1),
            "encode_frac": round(enc_bytes / (enc_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        }
        vol.close()
        del words
    del field, blocks
    torch.cuda.empty_cache()
    out["note"] = ("512^3 float32 turbulence, mean of %d runs per figure (HIP events); decode = "
                   "bcmc_decode_all (every block decoded, written as [N_b][64] float32 with its "
                   "range); hbm bytes = stream + decoded blocks + ranges (decode), field + stream "
                   "(encode); decompressed GB/s counts the 256-byte decoded blocks" % reps)
    return out


def dense_bench(steps, warmup, n_random=100):
    """The dense data-parallel marching cubes baseline (Sec. 3.3.3) on the
    512^3 turbulence field decoded from its rate-8 stream (the surface the
    block path extracts), resident uncompressed in HBM: p50 and p90 (mean of
    `steps` calls after `warmup`), and the paper's protocol of 100 random
    isovalues (between p10 and p90, first call discarded), beside the block
    path on the same stream (cold = empty cache after a cache flush, repeat =
    everything cached)."""
    import numpy as np
    import torch

    import paper_2009_03254_amd as bcmc
    from synthetic import fields

    n = 512
    dims = (n, n, n)
    field = fields.turbulence_torch(n, seed=2, device="cuda")
    words = bcmc.encode(field, RATE)
    del field
    vol = bcmc.Volume(words, dims, "f32", RATE)
    D = vol.decode_all()
    nb1 = n // 4
    dense = D.view(nb1, nb1, nb1, 4, 4, 4).permute(0, 3, 1, 4, 2, 5).reshape(n, n, n).contiguous()
    del D
    isos = {p: float(fields.percentile_iso_torch(dense, p)) for p in (10, 50, 90)}
    dm = bcmc.DenseMC(dims)
    flush_buf = torch.empty(FLUSH_BYTES // 4, dtype=torch.float32, device="cuda")
    probe = torch.empty((1, 4), dtype=torch.int32, device="cuda")
    T_max = max(dm.extract_into(dense, isos[p], probe)[1] for p in (10, 50, 90))
    out = torch.empty((3 * T_max + 3 * T_max // 8 + 1024, 4), dtype=torch.int32, device="cuda")

    def host_ms(fn, k, w):
        ts = []
        for i in range(w + k):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            dt = time.perf_counter() - t0
            if i >= w:
                ts.append(dt)
        return float(np.mean(ts)) * 1e3

    def dense_call(iso):
        rc, T = dm.extract_into(dense, iso, out)
        bcmc._capi.check(rc)
        return T

    def block_call(iso, cold):
        if cold:
            vol.reset_cache()
            flush_last_level_cache(flush_buf)
            torch.cuda.synchronize()
        rc, T = vol.extract_into(iso, out)
        bcmc._capi.check(rc)
        return T

    res = {"workload": "512^3 float32 turbulence decoded from its ZFP rate-8 stream, resident "
                       "uncompressed (dense) / compressed (block path)"}
    for p in (50, 90):
        iso = isos[p]
        T = dense_call(iso)
        d_ms = host_ms(lambda: dense_call(iso), steps, warmup)
        n_act = dm.active_cells()

        def cold():
            vol.reset_cache()
            flush_last_level_cache(flush_buf)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            block_call(iso, False)
            return time.perf_counter() - t0
        c_ms = float(np.mean([cold() for _ in range(steps)])) * 1e3
        block_call(iso, False)
        r_ms = host_ms(lambda: block_call(iso, False), steps, warmup)
        res[f"p{p}"] = {"iso": iso, "triangles": T, "dense_active_cells": n_act,
                        "dense_ms": round(d_ms, 4),
                        "dense_triangles_per_s": round(T / (d_ms * 1e-3)),
                        "block_cold_ms": round(c_ms, 4), "block_repeat_ms": round(r_ms, 4),
                        "speedup_block_cold": round(d_ms / c_ms, 3),
                        "speedup_block_repeat": round(d_ms / r_ms, 3)}
    rng = np.random.default_rng(7)
    rand = rng.uniform(isos[10], isos[90], n_random).astype(np.float32)
    ts = []
    for i, iso in enumerate(rand):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dense_call(float(iso))
        if i:
            ts.append(time.perf_counter() - t0)
    res["random100"] = {"range": [isos[10], isos[90]], "dense_mean_ms": round(float(np.mean(ts)) * 1e3, 4)}
    vol.reset_cache()
    ts = []
    for i, iso in enumerate(rand):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        block_call(float(iso), False)
        if i:
            ts.append(time.perf_counter() - t0)
    res["random100"]["block_mean_ms"] = round(float(np.mean(ts)) * 1e3, 4)
    res["note"] = ("dense = classify every cell (with its vertex count) -> prefix sums over "
                   "4096-cell tiles -> compact (ids, cases, first vertices) -> emit, over the "
                   "512 MiB uncompressed field; block = the compressed path (cull, cache, "
                   "decode, block-wise MC) on the 128 MiB stream; host-timed calls with their "
                   "count readback")
    dm.close()
    vol.close()
    del dense, out, flush_buf
    torch.cuda.empty_cache()
    return res


INTERACTION_SETS = {
    # name: (description, iso range)
    "nested_blobs": ("gaussian blobs 256^3 f32 (16 blobs, seed 3), ZFP rate 4", (0.1, 1.1)),
    "turbulent_sheet": ("channel flow 1280x960x192 f64 (tanh profile + 0.1 Fourier turbulence, "
                        "seed 5), ZFP rate 2", (-0.6, 0.6)),
}


def interaction_bench(n_iso=100):
    """The paper's interaction benchmarks (Sec. 4.6.1, tab:mc_benchmark_table)
    on a nested-surface volume and a turbulent-sheet volume: Random (100
    seeded isovalues), Sweep Up and Sweep Down (100 evenly spaced isovalues)
    over each volume's range, each from an empty cache (initial budget 0,
    growable to one slot per block), the first extraction discarded.  A first
    untimed pass sizes the output buffer; the timed pass runs without events
    and a third pass with HIP events around every stage gives the stage
    shares."""
    import torch

    import paper_2009_03254_amd as bcmc
    from paper_2009_03254_amd import interaction
    from synthetic import fields

    res = {}
    for name, (desc, (lo, hi)) in INTERACTION_SETS.items():
        if name == "nested_blobs":
            f = torch.from_numpy(fields.gaussian_blobs(256, 16, seed=3)).cuda()
            dims, typ, rate = (256, 256, 256), "f32", 4
            words = bcmc.encode(f, rate)
            del f
        else:
            dims, typ, rate = (1280, 960, 192), "f64", 2
            nbx, nby = dims[0] // 4, dims[1] // 4
            words = torch.empty(bcmc.num_blocks(*dims) * rate, dtype=torch.uint64, device="cuda")
            for z0 in range(0, dims[2], 32):
                f = fields.channel_flow_slab(z0, min(dims[2], z0 + 32), dims=dims)
                w = bcmc.encode(f, rate)
                first = (z0 // 4) * nbx * nby * rate
                words[first: first + w.numel()] = w
                del f, w
        vol = bcmc.Volume(words, dims, typ, rate)
        del words
        vol.set_cache_budget(initial_bytes=0, max_bytes=0)
        nb = vol.n_blocks
        out = torch.empty((1 << 20, 4), dtype=torch.int32, device="cuda")
        entry = {"workload": desc, "n_blocks": nb, "iso_range": [lo, hi]}
        for kind in interaction.KINDS:
            isos = interaction.isovalues(kind, lo, hi, n_iso, seed=11)
            # sizing pass (untimed): grow the buffer on a capacity error
            vol.reset_cache()
            for iso in isos:
                rc, T = vol.extract_into(float(iso), out)
                if rc == bcmc._capi.E_CAPACITY:
                    out = torch.empty((3 * T + 3 * T // 8 + 1024, 4), dtype=torch.int32, device="cuda")
                    rc, T = vol.extract_into(float(iso), out)
                bcmc._capi.check(rc)
            vol.reset_cache()
            timed = interaction.summarise(interaction.run(vol, isos, out), nb)
            vol.reset_cache()
            prof = interaction.summarise(interaction.run(vol, isos, out, profile=True), nb)
            timed["stage_share"] = prof.get("stage_share")
            timed["stage_mean_ms"] = prof.get("stage_mean_ms")
            entry[kind] = {k: (round(v, 5) if isinstance(v, float) else v) for k, v in timed.items()}
        vol.close()
        del out
        torch.cuda.empty_cache()
        res[name] = entry
    res["note"] = ("per benchmark: mean host-timed extraction per isovalue (count readback "
                   "included) over isovalues 2..%d, mean hit rate 1 - n_new/n_active, share of "
                   "the volume's blocks decoded and active per surface, stage shares of the "
                   "summed HIP-event stage times (cull = cull + compaction)" % n_iso)
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-differentiable", action="store_true",
                    help="skip the fwd / fwd+bwd measurement of the differentiable form")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched (48 volumes x 4 isovalues) measurement")
    ap.add_argument("--no-512", action="store_true", help="skip the 512^3 turbulence sequence")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline channel-flow measurement (no extra keys)")
    ap.add_argument("--only-512", action="store_true",
                    help="only the 512^3 turbulence sequence, printed as its own JSON")
    ap.add_argument("--zfp-only", action="store_true",
                    help="only the whole-volume ZFP encode / decode throughput, as its own JSON")
    ap.add_argument("--no-zfp", action="store_true", help="skip the ZFP throughput measurement")
    ap.add_argument("--dense-only", action="store_true",
                    help="only the dense marching cubes baseline, as its own JSON")
    ap.add_argument("--no-dense", action="store_true", help="skip the dense baseline")
    ap.add_argument("--interaction-only", action="store_true",
                    help="only the Random / Sweep Up / Sweep Down benchmarks, as their own JSON")
    ap.add_argument("--no-interaction", action="store_true",
                    help="skip the Random / Sweep Up / Sweep Down benchmarks")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the batched measurement, printed as its own JSON")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--no-profile-events", action="store_true",
                    help="no HIP events inside the timed steps (the roofline then takes "
                         "the dominant kernel's time from the profiled steps)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for --gpus {args.gpus}): the extraction "
              "path has no multi-GPU form here; a volume would be split into slabs of block "
              "layers, one per GPU", file=sys.stderr)
        sys.exit(2)

    import torch

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.batched_only:
        print(json.dumps({"batched": batch_bench(max(args.steps, 5), args.warmup)}), flush=True)
        return
    if args.copy_calibration:
        # 1 GiB read + 1 GiB written by the library's plain copy kernel: the
        # known-size reference for the traffic counters
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        import paper_2009_03254_amd as bcmc
        bcmc._capi.check(bcmc.lib().bcmc_copy_calibration(
            b.data_ptr(), a.data_ptr(), a.numel() * 4, torch.cuda.current_stream().cuda_stream))
        torch.cuda.synchronize()
        del a, b
    if args.zfp_only:
        print(json.dumps({"zfp_throughput": zfp_throughput()}), flush=True)
        return
    if args.dense_only:
        print(json.dumps({"dense_baseline": dense_bench(max(args.steps, 5), args.warmup)}), flush=True)
        return
    if args.interaction_only:
        print(json.dumps({"interaction": interaction_bench()}), flush=True)
        return
    if args.only_512:
        print(json.dumps({"turbulence512": turbulence512(args)}), flush=True)
        return
    result, sample_words = headline(args)
    torch.cuda.empty_cache()
    if not args.headline_only:
        if not args.no_512:
            result["turbulence512"] = turbulence512(args)
            torch.cuda.empty_cache()
        if not args.no_dense:
            log("[bench] dense marching cubes baseline on the decoded 512^3 field")
            result["dense_baseline"] = dense_bench(max(args.steps, 5), args.warmup)
        if not args.no_interaction:
            log("[bench] interaction benchmarks: Random, Sweep Up, Sweep Down")
            result["interaction"] = interaction_bench()
        if not args.no_zfp:
            log("[bench] whole-volume ZFP encode / decode at rates 2, 4, 8")
            result["zfp_throughput"] = zfp_throughput()
        if not args.no_differentiable:
            log("[bench] differentiable form (256^3 blobs)")
            result["differentiable"] = differentiable_bench(max(args.steps, 5), 2)
        if not args.no_batched:
            log("[bench] batched form (48 volumes x 4 isovalues)")
            result["batched"] = batch_bench(max(args.steps, 5), 2)
    if not args.no_cpu_baseline:
        from synthetic import fields
        nx, ny, _ = fields.CHANNEL_FLOW_DIMS
        log("[bench] CPU oracle baseline on the first 8 z-planes")
        result["cpu_baseline"] = cpu_baseline_oracle(
            sample_words, (nx, ny, 8), 2, True, 0.5,
            "the headline stream's first 2 block layers")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
