"""GPU parity: the HIP path through the C ABI against the CPU oracle on the
same seeded inputs.  Bit-exact for encoded/decoded values, ranges, active
blocks, cache state, cases, cell lists, counts and block ids; vertices within
1e-5 voxel of the FP64 oracle (and bit-exact against its FP32 mode)."""
import numpy as np
import pytest

from synthetic import fields
from tests.gpu_common import say, to_cuda, torch_cuda, verts_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bc():
    torch_cuda()
    import paper_2009_03254_amd as bcmc
    bcmc.lib()
    return bcmc


ENC_CASES = [
    ("sphere64", lambda: fields.sphere_sdf_noisy(64, 20.0, 0.5, seed=1), 16),
    ("turb_ragged_r8", lambda: fields.turbulence(37, 29, 23, seed=21, n_modes=64), 8),
    ("turb_ragged_r1", lambda: fields.turbulence(13, 9, 6, seed=22, n_modes=16), 1),
    ("turb_r2", lambda: fields.turbulence(24, 24, 24, seed=23, n_modes=32), 2),
    ("turb_r32", lambda: fields.turbulence(16, 12, 8, seed=24, n_modes=16), 32),
    ("f64_r2", lambda: fields.turbulence(21, 18, 10, seed=25, n_modes=32, dtype=np.float64), 2),
    ("f64_r8", lambda: fields.turbulence(16, 16, 16, seed=26, n_modes=32, dtype=np.float64), 8),
    ("f64_r64", lambda: fields.turbulence(8, 8, 8, seed=27, n_modes=8, dtype=np.float64), 64),
]


def _special_field():
    rng = np.random.default_rng(5)
    f = rng.standard_normal((16, 16, 16)).astype(np.float32)
    f[0:4, 0:4, 0:4] = 0.0                       # all-zero block
    f[0:4, 0:4, 4:8] = 1.5                       # constant block
    f[0:4, 4:8, 0:4] = 1e-40                     # subnormal block
    f[4:8, 0:4, 0:4] = 3e38                      # huge block
    f[4:8, 4:8, 4:8] *= 1e-30                    # tiny block
    return f


@pytest.mark.parametrize("name,make,rate", ENC_CASES + [("special_r8", _special_field, 8)])
def test_encode_decode_bitexact(bc, orc, name, make, rate):
    say(f"[encode/decode] {name} rate={rate}")
    f = make()
    nz, ny, nx = f.shape
    is64 = f.dtype == np.float64
    ref = orc.zfp_encode(f, rate)
    got = bc.encode(to_cuda(f), rate).cpu().numpy()
    assert np.array_equal(got, ref), "GPU encoder differs from the oracle encoder"
    vol = bc.Volume(ref, (nx, ny, nz), "f64" if is64 else "f32", rate)
    dec = vol.decode_all().cpu().numpy()
    oref = orc.zfp_decode(ref, (nx, ny, nz), rate, is64)
    assert np.array_equal(dec.view(np.uint32), oref.view(np.uint32))
    assert np.array_equal(vol.ranges(), orc.block_ranges(oref, (nx, ny, nz)))
    vol.close()


RANDOM_STREAMS = [
    (1, False, 0.5), (3, False, 0.2), (5, False, 0.05), (8, False, 0.5), (8, False, 0.02),
    (8, False, 0.9), (16, False, 0.3), (24, False, 0.1), (2, True, 0.5), (8, True, 0.05),
    (12, True, 0.3), (16, True, 0.3),
    # double precision at low rates: the stream ends within the top planes,
    # where pass 2 builds the planes by bit transposes
    (1, True, 0.5), (3, True, 0.9), (4, True, 0.2), (4, True, 0.97),
]


@pytest.mark.parametrize("rate,is64,density", RANDOM_STREAMS)
def test_random_streams_decode_bitexact(bc, orc, rate, is64, density):
    """Random block bits (finite exponents, some all-zero blocks): both GPU
    decoders (the load-time one behind decode_all, and the one extraction
    runs on new blocks) give the oracle's values bit for bit, on bit
    patterns a smooth field rarely produces (long zero runs, budgets ending
    inside a run, the implied last coefficient)."""
    dims = (64, 48, 40)
    say(f"[random stream] rate={rate} f64={is64} density={density}")
    s = fields.random_block_stream(dims, rate, is64, density, seed=100 + rate, zero_every=13)
    vol = bc.Volume(s, dims, "f64" if is64 else "f32", rate)
    dec = vol.decode_all().cpu().numpy()
    D = orc.zfp_decode(s, dims, rate, is64)
    assert np.array_equal(dec.view(np.uint32), D.view(np.uint32))
    # an extraction decodes every active block into the cache
    iso = float(np.median(D))
    T = _extract_and_compare(bc, orc, vol, D, dims, iso, check_cells=False)
    assert T > 0
    st = vol.stats()
    if (rate, is64, density) == (4, True, 0.2):
        # bits reaching below plane 39: the general decoder's second pass ran
        assert 0 < st["n_general"] < st["n_new"], st
    elif not is64 or rate > 4:
        assert st["n_general"] == 0, st
    _, ids = vol.active()
    I_slot, _, _ = vol.cache_state()
    slots = vol.slot_data()
    assert (I_slot[ids] >= 0).all()
    assert np.array_equal(slots[I_slot[ids]].view(np.uint32), D[ids].view(np.uint32))
    vol.close()


@pytest.mark.parametrize("rate,density", [(2, 0.5), (4, 0.2)])
def test_random_streams_wide_exponents(bc, orc, rate, density):
    """Double precision at low rates, block exponents up to +-120 (values
    still finite in single precision): the low-rate decoder takes the blocks
    with |emax| <= 96 and hands the others to the general decoder, which
    forms their values in double; both give the oracle's values bit for bit,
    through decode_all and through an extraction's cache fill."""
    dims = (64, 48, 40)
    say(f"[random stream, wide exponents] rate={rate} density={density}")
    s = fields.random_block_stream(dims, rate, True, density, seed=300 + rate, exp_spread=120,
                                   zero_every=11)
    vol = bc.Volume(s, dims, "f64", rate)
    dec = vol.decode_all().cpu().numpy()
    D = orc.zfp_decode(s, dims, rate, True)
    assert np.array_equal(dec.view(np.uint32), D.view(np.uint32))
    iso = float(np.median(D))
    T = _extract_and_compare(bc, orc, vol, D, dims, iso, check_cells=False)
    assert T > 0
    st = vol.stats()
    assert 0 < st["n_general"] < st["n_new"], st
    _, ids = vol.active()
    I_slot, _, _ = vol.cache_state()
    slots = vol.slot_data()
    assert (I_slot[ids] >= 0).all()
    assert np.array_equal(slots[I_slot[ids]].view(np.uint32), D[ids].view(np.uint32))
    vol.close()


def _extract_and_compare(bc, orc, vol, D, dims, iso, check_cells=True):
    import torch
    r = orc.mc_extract(D, dims, iso, want=("verts", "vblock", "cell_keys", "cases"))
    out = torch.empty((3 * r["T"] + 7, 4), dtype=torch.int32, device="cuda")
    rc, T = vol.extract_into(float(iso), out)
    assert rc == 0, bc.lib().bcmc_last_error()
    verts = out[: 3 * T]
    assert T == r["T"], (T, r["T"])
    xyz, blk = verts_np(verts)
    assert np.array_equal(blk, r["vblock"])
    err = np.abs(xyz.astype(np.float64) - r["verts"]).max() if T else 0.0
    assert err <= 1e-5, err
    v32, vb32 = orc.mc_extract_f32(D, dims, iso)
    assert np.array_equal(xyz.view(np.uint32), v32.view(np.uint32))
    # active blocks == the oracle's culling
    act, ids, can_emit = vol.active(with_flags=True)
    ract = orc.active_blocks(orc.block_ranges(D, dims), dims, iso)
    assert np.array_equal(act, ract)
    assert np.array_equal(ids, np.nonzero(ract)[0].astype(np.uint32))
    # "may emit" implies active, and every block owning a non-trivial cell has it
    assert not (can_emit & (1 - act)).any()
    owners = np.unique((r["cell_keys"] // 64).astype(np.int64))
    assert can_emit[owners].all()
    if check_cells:
        cases = vol.cases(iso).cpu().numpy()
        nt, _ = bc.mc_table()
        nontriv = nt[cases] > 0
        keys = (ids.astype(np.uint64)[:, None] * 64 + np.arange(64, dtype=np.uint64))[nontriv]
        assert np.array_equal(keys, r["cell_keys"])
        assert np.array_equal(cases[nontriv], r["cases"])
        # brute-force triangle count over the whole field
        assert T == orc.brute_count_blocks(D, dims, iso)
    # per-block counts and offsets are an exclusive scan
    cnt, off = vol.block_counts()
    ref_cnt = orc.block_vertex_counts(D, dims, iso, ids)
    assert np.array_equal(cnt, ref_cnt)
    assert np.array_equal(off, np.concatenate([[0], np.cumsum(cnt.astype(np.uint64))[:-1]]).astype(np.uint64)) if len(cnt) else True
    return T


def test_config1_sphere_cold(bc, orc):
    say("[extract] 64^3 noisy sphere, rate 16, iso 0, cold cache")
    f = fields.sphere_sdf_noisy(64, 20.0, 0.5, seed=1)
    s = orc.zfp_encode(f, 16)
    D = orc.zfp_decode(s, (64, 64, 64), 16)
    vol = bc.Volume(s, (64, 64, 64), "f32", 16)
    T = _extract_and_compare(bc, orc, vol, D, (64, 64, 64), np.float32(0.0))
    assert T > 10000
    st = vol.stats()
    assert st["n_new"] == st["n_active"] and st["hit_rate"] == 0.0
    # warm repeat: nothing new, identical output
    T2 = _extract_and_compare(bc, orc, vol, D, (64, 64, 64), np.float32(0.0), check_cells=False)
    st = vol.stats()
    assert T2 == T and st["n_new"] == 0 and st["hit_rate"] == 1.0


@pytest.mark.parametrize("dims,rate,seed", [((70, 61, 53), 8, 31), ((33, 47, 29), 4, 32),
                                            ((130, 66, 40), 2, 33)])
def test_turbulence_ragged_isovalues(bc, orc, dims, rate, seed):
    nx, ny, nz = dims
    say(f"[extract] turbulence {dims} rate {rate}")
    f = fields.turbulence(nx, ny, nz, seed=seed, n_modes=64)
    s = orc.zfp_encode(f, rate)
    D = orc.zfp_decode(s, dims, rate)
    vol = bc.Volume(s, dims, "f32", rate)
    for p in (50, 90, 10, 50):
        iso = fields.percentile_iso(orc.blocks_to_field(D, dims), p)
        _extract_and_compare(bc, orc, vol, D, dims, iso)


def test_lru_cache_matches_simulator(bc, orc):
    dims = (72, 64, 56)
    say(f"[cache] LRU parity {dims}")
    f = fields.turbulence(*dims, seed=41, n_modes=64)
    s = orc.zfp_encode(f, 8)
    D = orc.zfp_decode(s, dims, 8)
    nb = orc.num_blocks(*dims)
    vol = bc.Volume(s, dims, "f32", 8)
    init = nb // 10
    vol.set_cache_budget(initial_bytes=init * 256, max_bytes=nb * 256)
    sim = orc.LRU(nb, init, nb)
    rg = orc.block_ranges(D, dims)
    field = orc.blocks_to_field(D, dims)
    isos = [fields.percentile_iso(field, p) for p in (50, 55, 90, 10, 50, 52, 52, 95, 30)]
    import torch
    cap = 3 * max(orc.mc_count(D, dims, iso) for iso in isos) + 16
    out = torch.empty((cap, 4), dtype=torch.int32, device="cuda")
    for k, iso in enumerate(isos):
        rc, T = vol.extract_into(float(iso), out)
        assert rc == 0, bc.lib().bcmc_last_error()
        act = orc.active_blocks(rg, dims, iso)
        rc, I_new, ev = sim.update(act)
        assert rc == 0
        st = vol.stats()
        say(f"  call {k}: iso={iso:.4f} n_act={st['n_active']} n_new={st['n_new']} slots={st['n_slots']}")
        assert st["n_new"] == len(I_new) and st["n_evicted"] == ev
        if len(I_new):
            assert np.array_equal(vol.new_blocks(), I_new)
        I_slot, S_block, S_age = vol.cache_state()
        sI, sB, sA = sim.state()
        assert st["n_slots"] == sim.n_slots
        assert np.array_equal(I_slot, sI)
        assert np.array_equal(S_block, sB)
        assert np.array_equal(S_age, sA)
        # slot contents are the decoded blocks
        data = vol.slot_data()
        used = S_block >= 0
        assert np.array_equal(data[used].view(np.uint32), D[S_block[used]].view(np.uint32))
        assert T == orc.mc_count(D, dims, iso)


def _lru_step(bc, orc, vol, sim, out, D, dims, rg, iso, check_data=False):
    rc, T = vol.extract_into(float(iso), out)
    assert rc == 0, bc.lib().bcmc_last_error()
    act = orc.active_blocks(rg, dims, iso)
    rc, I_new, ev = sim.update(act)
    assert rc == 0
    st = vol.stats()
    assert st["n_new"] == len(I_new) and st["n_evicted"] == ev
    if len(I_new):
        assert np.array_equal(vol.new_blocks(), I_new)
    I_slot, S_block, S_age = vol.cache_state()
    sI, sB, sA = sim.state()
    assert st["n_slots"] == sim.n_slots
    assert np.array_equal(I_slot, sI)
    assert np.array_equal(S_block, sB)
    assert np.array_equal(S_age, sA)
    if check_data:
        data = vol.slot_data()
        used = S_block >= 0
        assert np.array_equal(data[used].view(np.uint32), D[S_block[used]].view(np.uint32))
    return st, T


def test_lru_long_sequence_wide_age_keys(bc, orc):
    """Hundreds of calls after one reset under eviction pressure, checked
    against the simulator after every call: the age sort's keys (the call of
    each slot's last use) then span two radix digits.  Advancing the age
    clock past 2^16 and then 2^24 calls (as that many calls with nothing
    active would) makes the third and fourth digits vary too, so every
    radix pass and both choices of the sorted buffer (an odd or even number
    of live passes) decide evictions."""
    torch = torch_cuda()
    dims = (48, 48, 48)
    f = fields.gaussian_blobs(48, 6, seed=43)
    s = orc.zfp_encode(f, 8)
    D = orc.zfp_decode(s, dims, 8)
    nb = orc.num_blocks(*dims)
    rg = orc.block_ranges(D, dims)
    field = orc.blocks_to_field(D, dims)
    rng = np.random.default_rng(44)
    isos = [fields.percentile_iso(field, p) for p in rng.uniform(5, 95, 360)]
    n_act = [int(orc.active_blocks(rg, dims, iso).sum()) for iso in isos]
    cap = max(n_act) + 8
    assert cap < 0.8 * nb
    init = 16
    say(f"[cache] long LRU sequence {dims}: {nb} blocks, cap {cap} slots, {len(isos)} calls")
    vol = bc.Volume(s, dims, "f32", 8)
    vol.set_cache_budget(initial_bytes=init * 256, max_bytes=cap * 256)
    sim = orc.LRU(nb, init, cap)
    out = torch.empty((3 * max(orc.mc_count(D, dims, i) for i in isos) + 16, 4),
                      dtype=torch.int32, device="cuda")
    evictions = 0
    for k, iso in enumerate(isos[:300]):
        st, T = _lru_step(bc, orc, vol, sim, out, D, dims, rg, iso, check_data=(k % 50 == 49))
        evictions += st["n_evicted"]
    assert T == orc.mc_count(D, dims, isos[299])
    assert evictions > 1000
    say(f"  300 calls: {evictions} evictions, {vol.stats()['n_slots']} slots")
    for k_idle, span in ((70000, range(300, 330)), (1 << 24, range(330, 360))):
        vol.age_cache(k_idle)
        sim.idle(k_idle)
        ev = 0
        for k in span:
            st, T = _lru_step(bc, orc, vol, sim, out, D, dims, rg, isos[k], check_data=True)
            ev += st["n_evicted"]
        say(f"  after {k_idle} idle calls: {ev} evictions")
        assert ev > 50
        assert T == orc.mc_count(D, dims, isos[span[-1]])


def test_cache_cap_error_and_capacity_retry(bc, orc):
    dims = (40, 40, 40)
    f = fields.turbulence(*dims, seed=51, n_modes=32)
    s = orc.zfp_encode(f, 8)
    D = orc.zfp_decode(s, dims, 8)
    iso = fields.percentile_iso(orc.blocks_to_field(D, dims), 50)
    vol = bc.Volume(s, dims, "f32", 8)
    vol.set_cache_budget(initial_bytes=10 * 256, max_bytes=20 * 256)
    import torch
    out = torch.empty((16, 4), dtype=torch.int32, device="cuda")
    rc, T = vol.extract_into(float(iso), out)
    assert rc == bc._capi.E_CACHE_CAP
    I_slot, S_block, _ = vol.cache_state()
    assert (I_slot == -1).all() and vol.stats()["n_slots"] == 10
    vol.set_cache_budget(0, 0)
    rc, T = vol.extract_into(float(iso), out)
    assert rc == bc._capi.E_CAPACITY and T == orc.mc_count(D, dims, iso)
    verts, T2 = vol.extract(float(iso))      # grows the buffer and retries (warm)
    assert T2 == T and vol.stats()["n_new"] == 0


def test_invalid_arguments(bc, orc):
    s = np.zeros(orc.num_blocks(8, 8, 8) * 4, np.uint64)
    with pytest.raises(bc.BcmcError):
        bc.Volume(s[:-1], (8, 8, 8), "f32", 4)
    with pytest.raises(bc.BcmcError):
        bc.Volume(s, (8, 8, 8), "f32", 40)
    vol = bc.Volume(s, (8, 8, 8), "f32", 4)   # all-zero stream: valid, no surface
    v, T = vol.extract(0.5)
    assert T == 0
    with pytest.raises(bc.BcmcError):
        vol.set_profiling(True, stages=[6])
    with pytest.raises(bc.BcmcError):
        vol.extract(float("nan"))
    # a real field: an infinite isovalue lies outside every (finite) range
    f = fields.sphere_sdf_noisy(16, 5.0, 0.5, seed=3)
    v2 = bc.Volume(orc.zfp_encode(f, 8), (16, 16, 16), "f32", 8)
    assert v2.extract(0.0)[1] > 0
    for iso in (float("inf"), float("-inf")):
        _, T = v2.extract(iso)
        assert T == 0 and v2.stats()["n_active"] == 0


@pytest.mark.parametrize("fmt", ["f32", "edge8", "q10"])
def test_checkerboard_every_cell_full(bc, orc, fmt):
    """Every cell of a sign checkerboard has case 105 or 150 (four
    triangles): 256 per interior block, so the emission's triangle list is
    flushed before nearly every staged block and blocks straddle flushes.
    Ragged dims, rate 32 (signs survive the codec); the output against the
    oracle bit for bit."""
    dims = (45, 38, 41)
    say(f"[extract] checkerboard {dims}, rate 32, {fmt}")
    z, y, x = np.meshgrid(np.arange(dims[2]), np.arange(dims[1]), np.arange(dims[0]), indexing="ij")
    f = np.where((x + y + z) % 2 == 0, 1.0, -1.0).astype(np.float32)
    f += 0.25 * np.sin(0.3 * x + 0.2 * y + 0.1 * z).astype(np.float32)   # distinct edge crossings
    s = orc.zfp_encode(f, 32)
    D = orc.zfp_decode(s, dims, 32)
    vol = bc.Volume(s, dims, "f32", 32)
    if fmt == "f32":
        T = _extract_and_compare(bc, orc, vol, D, dims, np.float32(0.0))
        cells = (dims[0] - 1) * (dims[1] - 1) * (dims[2] - 1)
        assert T == 4 * cells
    else:
        import torch
        vol.set_vertex_format(fmt)
        ref = (orc.mc_extract_edge8 if fmt == "edge8" else orc.mc_extract_q10)(D, dims, np.float32(0.0))
        out = torch.empty(len(ref) + 16, dtype=torch.int64, device="cuda")
        rc, T = vol.extract_into(0.0, out)
        assert rc == 0 and 3 * T == len(ref)
        got = out[: 3 * T].cpu().numpy().view(np.uint64)
        assert np.array_equal(got, np.asarray(ref, dtype=np.uint64))


def test_profiling_stage_mask(bc, orc):
    say("[profile] 48^3 sphere, rate 8: stage mask selects which stage times exist")
    f = fields.sphere_sdf_noisy(48, 15.0, 0.5, seed=4)
    s = orc.zfp_encode(f, 8)
    vol = bc.Volume(s, (48, 48, 48), "f32", 8)
    vol.set_profiling(True)
    v_all, T_all = vol.extract(0.0)
    st = vol.stats()["stage_ms"]
    assert all(st[i] > 0 for i in (0, 2, 3, 5)) and st[7] >= st[5] > 0
    vol.reset_cache()
    vol.set_profiling(True, stages=[5])
    v5, T5 = vol.extract(0.0)
    st = vol.stats()["stage_ms"]
    assert st[5] > 0 and all(st[i] == 0 for i in (0, 1, 2, 3, 4, 6, 7))
    assert T5 == T_all and _same_soup(v5, v_all)
    vol.set_profiling(False)
    vol.reset_cache()
    v0, T0 = vol.extract(0.0)
    assert all(x == 0 for x in vol.stats()["stage_ms"]) and T0 == T_all and _same_soup(v0, v_all)


def _same_soup(a, b):
    """Same triangles as a set (rows of whole triangles, order free)."""
    def rows(v):
        r = v.cpu().numpy().reshape(-1, 12)
        return r[np.lexsort(r.T[::-1])]
    return np.array_equal(rows(a), rows(b))


def test_mc_single_cells_all_cases(bc, orc):
    """Every one of the 256 cube cases on a 2x2x2 volume: the GPU emits
    exactly the table's triangles at the corner configuration."""
    nt, tri = bc.mc_table()
    for cs in range(256):
        f = np.array([[[(-1.0 if (cs >> (x + 2 * y + 4 * z)) & 1 else 1.0) for x in range(2)]
                       for y in range(2)] for z in range(2)], dtype=np.float32)
        B = orc.field_to_blocks(f)
        vol = bc.FieldVolume(to_cuda(B), (2, 2, 2))
        verts, T = vol.extract(0.0)
        assert T == nt[cs], cs
        if T:
            r = orc.mc_extract(B, (2, 2, 2), 0.0, want=("verts", "vblock"))
            xyz, blk = verts_np(verts)
            assert np.abs(xyz - r["verts"]).max() < 1e-6
        vol.close()


@pytest.mark.parametrize("dims,rate,seed", [((70, 61, 53), 8, 34), ((45, 38, 31), 16, 35)])
def test_edge8_records_bitexact(bc, orc, dims, rate, seed):
    """8-byte edge records: bit-exact against the oracle's records over cold,
    warm and repeated calls; decoded positions within 1e-5 of the float64
    soup; the 16-byte output of the same volume still matches; the capacity
    error counts records."""
    torch = bc._torch()
    say(f"[edge8] turbulence {dims} rate {rate}")
    f = fields.turbulence(*dims, seed=seed, n_modes=64)
    s = orc.zfp_encode(f, rate)
    D = orc.zfp_decode(s, dims, rate)
    field = orc.blocks_to_field(D, dims)
    vol = bc.Volume(s, dims, "f32", rate)
    vol.set_vertex_format("edge8")
    small = torch.empty(5, dtype=torch.int64, device="cuda")
    iso0 = fields.percentile_iso(field, 50)
    rc, T = vol.extract_into(float(iso0), small)
    assert rc == bc._capi.E_CAPACITY and T == orc.mc_count(D, dims, iso0)
    for p in (50, 85, 50, 20):
        iso = fields.percentile_iso(field, p)
        ref = orc.mc_extract_edge8(D, dims, iso)
        out = torch.empty(ref.shape[0] + 7, dtype=torch.int64, device="cuda")
        rc, T = vol.extract_into(float(iso), out)
        assert rc == 0 and 3 * T == ref.shape[0]
        got = out[: 3 * T].cpu().numpy().view(np.uint64)
        assert np.array_equal(got, ref), p
        r = orc.mc_extract(D, dims, iso, want=("verts", "vblock"))
        pos, blk = bc.edge8_positions(out[: 3 * T])
        assert np.array_equal(blk.cpu().numpy(), r["vblock"].astype(np.int64))
        assert float((pos.cpu() - torch.from_numpy(r["verts"])).abs().max()) <= 1e-5
    vol.set_vertex_format("f32")
    iso = fields.percentile_iso(field, 85)
    _extract_and_compare(bc, orc, vol, D, dims, iso)
    with pytest.raises(bc.BcmcError):
        vol.set_vertex_format(7)


@pytest.mark.parametrize("dims,rate,seed", [((70, 61, 53), 8, 36), ((45, 38, 31), 16, 37)])
def test_q10_records_bitexact(bc, orc, dims, rate, seed):
    """Sec. 4.5's 8-byte vertices written by the emission: bit-exact against
    the oracle's over cold and warm calls, equal to the conversion kernel's
    records of the 16-byte soup, dequantised within 2/1023 voxel of the
    float64 soup; the capacity error counts records."""
    torch = bc._torch()
    say(f"[q10] turbulence {dims} rate {rate}")
    f = fields.turbulence(*dims, seed=seed, n_modes=64)
    s = orc.zfp_encode(f, rate)
    D = orc.zfp_decode(s, dims, rate)
    field = orc.blocks_to_field(D, dims)
    vol = bc.Volume(s, dims, "f32", rate)
    ref16 = bc.Volume(s, dims, "f32", rate)
    vol.set_vertex_format("q10")
    small = torch.empty(5, dtype=torch.int64, device="cuda")
    iso0 = fields.percentile_iso(field, 50)
    rc, T = vol.extract_into(float(iso0), small)
    assert rc == bc._capi.E_CAPACITY and T == orc.mc_count(D, dims, iso0)
    worst = 0.0
    for p in (50, 85, 50, 20):
        iso = fields.percentile_iso(field, p)
        ref = orc.mc_extract_q10(D, dims, iso)
        out = torch.empty(ref.shape[0] + 7, dtype=torch.int64, device="cuda")
        rc, T = vol.extract_into(float(iso), out)
        assert rc == 0 and 3 * T == ref.shape[0]
        got = out[: 3 * T].cpu().numpy().view(np.uint64)
        assert np.array_equal(got, ref), p
        v16, T16 = ref16.extract(float(iso))
        assert T16 == T
        conv = bc.vertices_to_q10(v16)
        assert torch.equal(conv, out[: 3 * T])
        r = orc.mc_extract(D, dims, iso, want=("verts", "vblock"))
        pos, blk = bc.q10_positions(out[: 3 * T], dtype=torch.float64)
        assert np.array_equal(blk.cpu().numpy(), r["vblock"].astype(np.int64))
        err = float((pos.cpu() - torch.from_numpy(r["verts"])).abs().max())
        assert err <= 2.0 / 1023 + 1e-6
        worst = max(worst, err)
    say(f"  largest dequantisation error {worst:.3e} voxel")
    assert bc.vertices_to_q10(v16[:0]).numel() == 0


def test_flags_follow_tiles_across_isovalues(bc, orc):
    """A ramp along x over three cull tiles: successive isovalues make
    different tiles live, then none; the active flags (written only in live
    tiles, cleared in tiles live the call before) match the oracle every
    time."""
    dims = (260, 70, 38)
    nx, ny, nz = dims
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    f = np.broadcast_to(x + 0.25 * np.sin(0.7 * np.arange(ny))[None, :, None], (nz, ny, nx)).astype(np.float32)
    s = orc.zfp_encode(np.ascontiguousarray(f), 8)
    D = orc.zfp_decode(s, dims, 8)
    vol = bc.Volume(s, dims, "f32", 8)
    say(f"[flags] ramp {dims}")
    for iso in (20.5, 200.5, 250.5, 20.5, -5.0, 130.5, 130.5):
        T = _extract_and_compare(bc, orc, vol, D, dims, np.float32(iso), check_cells=False)
        assert (T > 0) == (iso > 0), (iso, T)


@pytest.mark.parametrize("iso", [1.0, 2.0, 0.5])
def test_isovalue_ties_integer_field(bc, orc, iso):
    """An integer-valued field (0..3) at an integer isovalue puts many
    corners exactly on iso: a corner is inside only when its value is below
    iso, a block's range contains iso only when lo < iso <= hi, and t is
    exactly 0 or 1 on edges ending at iso.  Identity volume (no codec, the
    ties survive) against the oracle bit for bit and the brute-force count
    on the raw field; the compressed path (rate 32) against the oracle's
    decode.  iso 0.5 is the tie-free control."""
    dims = (35, 27, 30)
    say(f"[extract] integer field {dims}, iso {iso}")
    rng = np.random.default_rng(61)
    f = rng.integers(0, 4, size=(dims[2], dims[1], dims[0])).astype(np.float32)
    B = orc.field_to_blocks(f)
    vol = bc.FieldVolume(to_cuda(B), dims)
    verts, T = vol.extract(iso)
    iso32 = np.float32(iso)
    assert T == orc.brute_count(f, iso32) > 0
    v32, vb = orc.mc_extract_f32(B, dims, iso32)
    xyz, blk = verts_np(verts)
    assert np.array_equal(blk, vb)
    assert np.array_equal(xyz.view(np.uint32), v32.view(np.uint32))
    r = orc.mc_extract(B, dims, iso32, want=("verts", "vblock"))
    assert np.abs(xyz.astype(np.float64) - r["verts"]).max() <= 1e-5
    s = orc.zfp_encode(f, 32)
    D = orc.zfp_decode(s, dims, 32)
    vc = bc.Volume(s, dims, "f32", 32)
    _extract_and_compare(bc, orc, vc, D, dims, iso32)
