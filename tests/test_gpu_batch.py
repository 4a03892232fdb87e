"""GPU parity of the batched extraction: every job's slice of the batched
output equals, byte for byte, the single-volume extract of its volume at its
isovalue (and the oracle's counts / FP32 vertices), across cold and warm runs,
isovalue updates, graph replay on and off, autotuned schedules, and f64."""
import numpy as np
import pytest

from synthetic import fields
from tests.gpu_common import say, torch_cuda, verts_np

pytestmark = pytest.mark.gpu


def _make(orc, dims_list, rate, f64=False, seed0=500):
    streams, decoded = [], []
    for k, (nx, ny, nz) in enumerate(dims_list):
        f = fields.turbulence(nx, ny, nz, seed=seed0 + k, n_modes=32,
                              dtype=np.float64 if f64 else np.float32)
        s = orc.zfp_encode(f, rate)
        streams.append(s)
        decoded.append(orc.zfp_decode(s, (nx, ny, nz), rate, f64))
    return streams, decoded


def _plain(bc, vol, iso):
    import torch
    out = torch.empty((1, 4), dtype=torch.int32, device="cuda")
    rc, T = vol.extract_into(float(iso), out)
    out = torch.empty((3 * T + 8, 4), dtype=torch.int32, device="cuda")
    rc, T = vol.extract_into(float(iso), out)
    assert rc == 0
    return out[: 3 * T].cpu().numpy()


def _check(bc, orc, batch, vols, dims_list, decoded, jobs, plain_vols):
    import torch
    need = sum(3 * orc.mc_count(decoded[vi], dims_list[vi], iso) for vi, iso in jobs)
    out = torch.empty((need + 16, 4), dtype=torch.int32, device="cuda")
    rc, offs = batch.run_into(out)
    assert rc == 0, bc.lib().bcmc_last_error()
    assert int(offs[-1]) == need
    v = out[:need].cpu().numpy()
    assert offs[0] == 0 and np.all(np.diff(offs.astype(np.int64)) >= 0)
    for j, (vi, iso) in enumerate(jobs):
        got = v[int(offs[j]):int(offs[j + 1])]
        ref = _plain(bc, plain_vols[vi], iso)
        assert got.shape == ref.shape, (j, got.shape, ref.shape)
        assert np.array_equal(got, ref), j
        T = orc.mc_count(decoded[vi], dims_list[vi], iso)
        assert got.shape[0] == 3 * T
        if T:
            v32, vb = orc.mc_extract_f32(decoded[vi], dims_list[vi], iso)
            assert np.array_equal(got[:, :3].view(np.float32).view(np.uint32), v32.view(np.uint32))
            assert np.array_equal(got[:, 3].view(np.uint32), vb)
    return offs


def test_batch_equals_plain_extract(orc):
    torch_cuda()
    import paper_2009_03254_amd as bc
    rng = np.random.default_rng(7)
    dims_list = [tuple(int(x) for x in rng.integers(18, 60, 3)) for _ in range(7)]
    say(f"[batch] dims {dims_list}")
    streams, decoded = _make(orc, dims_list, 8)
    vols = [bc.Volume(s, d, "f32", 8) for s, d in zip(streams, dims_list)]
    plain = [bc.Volume(s, d, "f32", 8) for s, d in zip(streams, dims_list)]
    isos = {vi: [fields.percentile_iso(orc.blocks_to_field(decoded[vi], dims_list[vi]), p)
                 for p in (20, 50, 80)] for vi in range(len(vols))}
    jobs = [(vi, isos[vi][k]) for k in range(3) for vi in range(len(vols))]   # interleaved
    batch = bc.Batch(vols, jobs)
    _check(bc, orc, batch, vols, dims_list, decoded, jobs, plain)
    info = batch.info()
    assert info["n_new"] > 0 and info["n_resident"] == info["n_new"]
    say(f"  cold: {info}")
    # warm: nothing new, same output
    _check(bc, orc, batch, vols, dims_list, decoded, jobs, plain)
    assert batch.info()["n_new"] == 0
    # new isovalues through device memory (graph replay without re-capture)
    jobs2 = [(vi, isos[vi][(k + 1) % 3] * 0.5) for k in range(3) for vi in range(len(vols))]
    batch.set_isos([j[1] for j in jobs2])
    _check(bc, orc, batch, vols, dims_list, decoded, jobs2, plain)
    # direct cooperative launch (no graph) gives the same bytes
    batch.set_graph(False)
    batch.reset()
    _check(bc, orc, batch, vols, dims_list, decoded, jobs2, plain)
    assert batch.info()["graph"] == 0
    batch.set_graph(True)
    # autotuned schedule, then the same result again
    batch.tune()
    info = batch.info()
    say(f"  tuned: stage_blocks={info['stage_blocks']} grid={info['grid']} graph={info['graph']} "
        f"unsupported={info['graph_unsupported']}")
    _check(bc, orc, batch, vols, dims_list, decoded, jobs2, plain)
    batch.close()


def test_batch_f64_and_empty_jobs(orc):
    torch_cuda()
    import paper_2009_03254_amd as bc
    dims_list = [(21, 18, 13), (9, 30, 17)]
    streams, decoded = _make(orc, dims_list, 2, f64=True, seed0=900)
    vols = [bc.Volume(s, d, "f64", 2) for s, d in zip(streams, dims_list)]
    plain = [bc.Volume(s, d, "f64", 2) for s, d in zip(streams, dims_list)]
    jobs = [(1, 0.1), (0, 50.0), (0, -0.2), (1, -50.0), (0, 0.3)]    # two jobs without surface
    batch = bc.Batch(vols, jobs)
    offs = _check(bc, orc, batch, vols, dims_list, decoded, jobs, plain)
    assert offs[2] == offs[1] and offs[4] == offs[3]
    batch.close()


def test_batch_capacity_retry(orc):
    torch = torch_cuda()
    import paper_2009_03254_amd as bc
    dims_list = [(40, 33, 27)]
    streams, decoded = _make(orc, dims_list, 8, seed0=950)
    vols = [bc.Volume(streams[0], dims_list[0], "f32", 8)]
    batch = bc.Batch(vols, [(0, 0.0), (0, 0.5)])
    out = torch.empty((8, 4), dtype=torch.int32, device="cuda")
    rc, offs = batch.run_into(out)
    assert rc == bc._capi.E_CAPACITY
    T = orc.mc_count(decoded[0], dims_list[0], 0.0) + orc.mc_count(decoded[0], dims_list[0], 0.5)
    assert offs[-1] == 3 * T
    verts, offs2 = batch.run()
    assert np.array_equal(offs, offs2)
    batch.close()


@pytest.mark.parametrize("rates", [(4, 8, 32), (8, 8, 8)])
def test_batch_mixed_rates_many_jobs(orc, rates):
    """Volumes of different rates (the decoder reads each block's words from
    global memory) or one shared rate (staged through LDS), and a volume with
    more jobs than the decoder builds masks for in registers."""
    torch_cuda()
    import paper_2009_03254_amd as bc
    dims_list = [(37, 29, 22), (26, 41, 19), (18, 18, 33)]
    streams, decoded = [], []
    for k, ((nx, ny, nz), r) in enumerate(zip(dims_list, rates)):
        f = fields.turbulence(nx, ny, nz, seed=1200 + k, n_modes=32, dtype=np.float32)
        s = orc.zfp_encode(f, r)
        streams.append(s)
        decoded.append(orc.zfp_decode(s, (nx, ny, nz), r, False))
    vols = [bc.Volume(s, d, "f32", r) for s, d, r in zip(streams, dims_list, rates)]
    plain = [bc.Volume(s, d, "f32", r) for s, d, r in zip(streams, dims_list, rates)]
    fld = [orc.blocks_to_field(decoded[v], dims_list[v]) for v in range(3)]
    jobs = [(0, fields.percentile_iso(fld[0], p)) for p in (10, 25, 40, 55, 70, 85)]
    jobs += [(1, fields.percentile_iso(fld[1], 50)), (2, fields.percentile_iso(fld[2], 30)),
             (2, fields.percentile_iso(fld[2], 60))]
    say(f"[batch] rates {rates}, {len(jobs)} jobs")
    batch = bc.Batch(vols, jobs)
    _check(bc, orc, batch, vols, dims_list, decoded, jobs, plain)
    assert batch.info()["n_new"] > 0
    _check(bc, orc, batch, vols, dims_list, decoded, jobs, plain)   # warm: masks from the store
    assert batch.info()["n_new"] == 0
    batch.close()


def test_batch_checkerboard_with_turbulence(orc):
    """A sign checkerboard (four triangles in every cell, so the batched
    emission's triangle list flushes before nearly every staged block) in
    one batch with a turbulence volume, at several isovalues: every job's
    slice against the plain extract and the oracle's float32 soup."""
    torch_cuda()
    import paper_2009_03254_amd as bc
    dc = (37, 30, 26)
    z, y, x = np.meshgrid(np.arange(dc[2]), np.arange(dc[1]), np.arange(dc[0]), indexing="ij")
    fc = np.where((x + y + z) % 2 == 0, 1.0, -1.0).astype(np.float32)
    fc += 0.25 * np.sin(0.3 * x + 0.2 * y + 0.1 * z).astype(np.float32)
    sc = orc.zfp_encode(fc, 32)
    dims_list = [dc, (29, 35, 22)]
    streams, decoded = _make(orc, dims_list[1:], 32, seed0=1200)
    streams = [sc] + streams
    decoded = [orc.zfp_decode(sc, dc, 32)] + decoded
    vols = [bc.Volume(s, d, "f32", 32) for s, d in zip(streams, dims_list)]
    plain = [bc.Volume(s, d, "f32", 32) for s, d in zip(streams, dims_list)]
    jobs = [(0, 0.0), (1, 0.0), (0, 0.1), (1, 0.3), (0, -0.1)]
    batch = bc.Batch(vols, jobs)
    offs = _check(bc, orc, batch, vols, dims_list, decoded, jobs, plain)
    cells = (dc[0] - 1) * (dc[1] - 1) * (dc[2] - 1)
    assert int(offs[1] - offs[0]) == 3 * 4 * cells
    batch.close()


def test_batch_schedule_change_recaptures_graph(orc):
    """Changing one schedule dimension at a time (the front kernel's grid
    alone, its scan schedule alone, then the back kernel's grid, then the
    staging) captures the graph again: every kernel records the grid it ran
    with, which must be the grid the schedule reports, and the output stays
    byte-identical."""
    torch_cuda()
    import paper_2009_03254_amd as bc
    dims_list = [(41, 37, 29), (30, 26, 45)]
    streams, decoded = _make(orc, dims_list, 8, seed0=1300)
    vols = [bc.Volume(s, d, "f32", 8) for s, d in zip(streams, dims_list)]
    plain = [bc.Volume(s, d, "f32", 8) for s, d in zip(streams, dims_list)]
    fld = [orc.blocks_to_field(decoded[v], dims_list[v]) for v in range(2)]
    jobs = [(v, fields.percentile_iso(fld[v], p)) for v in range(2) for p in (30, 70)]
    batch = bc.Batch(vols, jobs)
    batch.set_graph(True)
    seen = set()
    for sb, pc, fpc, scan in ((8, 4, 4, 0), (8, 4, 1, 0), (8, 4, 1, 1), (8, 4, 2, 1), (8, 2, 2, 1),
                              (4, 2, 2, 0), (4, 2, 1, 1)):
        batch.set_schedule(sb, pc, fpc, scan)
        batch.reset()                   # cold: the decode kernel runs too
        _check(bc, orc, batch, vols, dims_list, decoded, jobs, plain)
        info = batch.info()
        say(f"  schedule {sb},{pc},{fpc},{scan}: {info['front_grid']} {info['decode_grid']} {info['grid']}"
            f" ran {info['ran_front_grid']} {info['ran_decode_grid']} {info['ran_grid']}"
            f" graph={info['graph']}")
        assert info["stage_blocks"] == sb and info["scan_schedule"] == scan
        assert info["ran_front_grid"] == info["front_grid"]
        assert info["ran_decode_grid"] == info["decode_grid"]
        assert info["ran_grid"] == info["grid"]
        seen.add((info["front_grid"], info["grid"]))
        _check(bc, orc, batch, vols, dims_list, decoded, jobs, plain)    # warm replay
        assert batch.info()["ran_front_grid"] == info["front_grid"]
    assert len(seen) >= 3
    with pytest.raises(bc.BcmcError):
        batch.set_schedule(8, 4, 4, 2)   # scan schedules are 0 and 1
    batch.close()


def test_batch_benchmark_workload_full(orc):
    """The batched workload at its full size, as the benchmark builds it: 48
    turbulence volumes (each axis uniform in [32, 256], dims seed 4, field
    seed 4000 + v) generated and encoded on the GPU at rate 8, isovalues at
    the 20/40/60/80th percentiles of each field, 192 jobs in one autotuned,
    graph-replayed batch.  Each volume's GPU stream equals the oracle
    encoder's output for the host copy of its field; every job's slice equals
    the plain single-volume extract byte for byte and the oracle's plain
    extract of the stream (count, float32 vertices bit for bit), cold and
    warm.  The persistent front kernel runs several tiles per workgroup
    here."""
    torch = torch_cuda()
    from concurrent.futures import ThreadPoolExecutor
    import paper_2009_03254_amd as bc
    dims_list = fields.batched_dims(48, seed=4, lo=32, hi=256)
    vols, plain, jobs, host = [], [], [], []
    for v, (nx, ny, nz) in enumerate(dims_list):
        f = fields.turbulence_torch(nx, ny, nz, seed=4000 + v, device="cuda")
        isos = [float(fields.percentile_iso_torch(f, p)) for p in (20, 40, 60, 80)]
        words = bc.encode(f, 8)
        w = words.view(torch.int64).cpu().numpy().view(np.uint64).copy()
        host.append((f.cpu().numpy(), w))
        vols.append(bc.Volume(words, (nx, ny, nz), "f32", 8))
        plain.append(bc.Volume(words, (nx, ny, nz), "f32", 8))
        jobs += [(v, i) for i in isos]
        del f, words
    nb = sum(orc.num_blocks(*d) for d in dims_list)
    say(f"[batch] benchmark workload: 48 volumes, {nb} blocks, 192 jobs")

    def oracle_volume(v):
        f, w = host[v]
        assert np.array_equal(orc.zfp_encode(f, 8), w), v
        D = orc.zfp_decode(w, dims_list[v], 8)
        return [orc.mc_extract_f32(D, dims_list[v], iso) for _, iso in jobs[4 * v: 4 * v + 4]]

    with ThreadPoolExecutor(16) as ex:
        ref = list(ex.map(oracle_volume, range(48)))
    total = sum(len(vb) for r in ref for _, vb in r)
    say(f"  oracle: {total // 3} triangles")

    batch = bc.Batch(vols, jobs)
    batch.tune()
    info = batch.info()
    say(f"  tuned: stage_blocks={info['stage_blocks']} grid={info['grid']} "
        f"front_grid={info['front_grid']} graph={info['graph']}")
    tiles_per_wg = nb / max(1, info["front_grid"])
    out = torch.empty((total + 1024, 4), dtype=torch.int32, device="cuda")
    pbuf = torch.empty((max(len(vb) for r in ref for _, vb in r) + 16, 4), dtype=torch.int32,
                       device="cuda")
    for kind in ("cold", "warm"):
        if kind == "cold":
            batch.reset()
        rc, offs = batch.run_into(out)
        assert rc == 0, bc.lib().bcmc_last_error()
        assert int(offs[-1]) == total
        inf = batch.info()
        assert inf["ran_front_grid"] == inf["front_grid"] and inf["ran_grid"] == inf["grid"]
        if kind == "cold":
            assert inf["n_new"] > 0
        else:
            assert inf["n_new"] == 0
        got = out[:total].cpu().numpy()
        for j, (v, iso) in enumerate(jobs):
            sl = got[int(offs[j]): int(offs[j + 1])]
            v32, vb = ref[v][j - 4 * v]
            assert sl.shape[0] == len(vb), (kind, j)
            assert np.array_equal(sl[:, 3].view(np.uint32), vb), (kind, j)
            assert np.array_equal(sl[:, :3].view(np.float32).view(np.uint32), v32.view(np.uint32)), (kind, j)
            if kind == "cold":
                rc, T = plain[v].extract_into(iso, pbuf)
                assert rc == 0 and 3 * T == len(vb)
                assert np.array_equal(pbuf[: 3 * T].cpu().numpy(), sl), j
        say(f"  {kind}: all 192 job slices equal the oracle's soup and the plain extract "
            f"({tiles_per_wg:.0f} blocks per front workgroup)")
    batch.close()
