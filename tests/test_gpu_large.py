"""GPU parity at full size on the large float64 volume: 5120 x 3840 x 768
channel-flow-like field (tanh mean profile plus Fourier turbulence), ZFP
fixed-rate 2 bits/value (3.8 GB on the device), isovalue 0.5, LRU cache
capped at 64 GiB of decoded float32.

The oracle cannot run on 2.4e8 blocks, so the check is on sampled blocks:
the generator's values around each sample are kept while the field is
produced slab by slab, and the oracle (encode, decode, cull rule, plain
marching cubes over the decoded 3x3x3 block neighbourhood) is compared bit
for bit with the GPU's stream words, flags, per-block counts and the block's
slice of the triangle soup.  Most samples are placed on the surface: at 40
seeded (x, z) block columns, the block where the generated field crosses the
isovalue.  Properties that hold at any size (counts, offsets, totals, vertex
bounds) are checked on the whole output."""
import numpy as np
import pytest

from synthetic import fields
from tests.gpu_common import say, torch_cuda

pytestmark = pytest.mark.gpu

RATE = 2
ISO = 0.5
SLAB = 32            # z-planes generated and encoded at a time (multiple of 4)


def _generate(bc, torch, nb, cols, loose):
    """Generate + encode the volume; keep the field on 12-voxel-wide column
    neighbourhoods of `cols` and 12^3 neighbourhoods of `loose`."""
    nx, ny, nz = fields.CHANNEL_FLOW_DIMS
    per_layer = (nx // 4) * (ny // 4)
    words = torch.empty(nb * RATE, dtype=torch.uint64, device="cuda")
    colv = {c: np.empty((12, ny, 12)) for c in cols}
    loosev = {c: np.empty((12, 12, 12)) for c in loose}
    for z0 in range(0, nz, SLAB):
        z1 = min(nz, z0 + SLAB)
        f = fields.channel_flow_slab(z0, z1)
        w = bc.encode(f, RATE)
        first = (z0 // 4) * per_layer
        words[first * RATE: first * RATE + w.numel()] = w
        for store, keys in ((colv, cols), (loosev, loose)):
            for key in keys:
                bx, bz = key[0], key[-1]
                za, zb = max(z0, 4 * bz - 4), min(z1, 4 * bz + 8)
                if za >= zb:
                    continue
                ys = slice(0, ny) if len(key) == 2 else slice(4 * key[1] - 4, 4 * key[1] + 8)
                store[key][za - (4 * bz - 4): zb - (4 * bz - 4)] = \
                    f[za - z0: zb - z0, ys, 4 * bx - 4: 4 * bx + 8].cpu().numpy()
        del f, w
    torch.cuda.synchronize()
    return words, colv, loosev


def test_large_f64_sampled_parity(orc):
    torch = torch_cuda()
    import paper_2009_03254_amd as bc
    nx, ny, nz = fields.CHANNEL_FLOW_DIMS
    nbx, nby, nbz = nx // 4, ny // 4, nz // 4
    nb = nbx * nby * nbz
    rng = np.random.default_rng(55)
    cols = [(int(rng.integers(1, nbx - 1)), int(rng.integers(1, nbz - 1))) for _ in range(40)]
    loose = [(int(rng.integers(1, nbx - 1)), int(rng.integers(1, nby - 1)), int(rng.integers(1, nbz - 1)))
             for _ in range(8)]
    say(f"[large] {nx}x{ny}x{nz} f64, rate {RATE}, {nb} blocks")
    words, colv, loosev = _generate(bc, torch, nb, cols, loose)

    # samples: the surface crossing of each column (middle one if several), + loose blocks
    samples, kept = [], {}
    for (bx, bz) in cols:
        c = colv[(bx, bz)][4:8, :, 4:8]
        lo, hi = c.min(axis=(0, 2)), c.max(axis=(0, 2))
        rows = np.nonzero((lo < ISO) & (ISO <= hi))[0]
        rows = rows[(rows >= 8) & (rows < ny - 8)]
        if len(rows) == 0:
            continue
        by = int(rows[len(rows) // 2]) // 4
        samples.append((bx, by, bz))
        kept[(bx, by, bz)] = np.ascontiguousarray(colv[(bx, bz)][:, 4 * by - 4: 4 * by + 8, :])
    for key in loose:
        samples.append(key)
        kept[key] = loosev[key]
    del colv, loosev
    say(f"  generated and encoded; {len(samples)} samples")

    # stream words of every block around the samples: bit-exact against the
    # oracle encoder
    nbh = [(key, dx, dy, dz) for key in samples for dz in range(3) for dy in range(3) for dx in range(3)]
    ids = np.array([(key[0] + dx - 1) + nbx * ((key[1] + dy - 1) + nby * (key[2] + dz - 1))
                    for (key, dx, dy, dz) in nbh], dtype=np.int64)
    idx = torch.from_numpy((ids[:, None] * RATE + np.arange(RATE)[None, :]).ravel()).cuda()
    gw = words.view(torch.int64)[idx].cpu().numpy().view(np.uint64).reshape(-1, RATE)
    for k, (key, dx, dy, dz) in enumerate(nbh):
        blk = np.ascontiguousarray(kept[key][4 * dz: 4 * dz + 4, 4 * dy: 4 * dy + 4, 4 * dx: 4 * dx + 4])
        ref = orc.zfp_encode(blk, RATE)
        assert np.array_equal(np.asarray(ref, dtype=np.uint64), gw[k]), (key, dx, dy, dz)

    vol = bc.Volume(words, (nx, ny, nz), "f64", RATE)
    del words
    torch.cuda.empty_cache()
    vol.set_cache_budget(initial_bytes=0, max_bytes=64 << 30)
    probe = torch.empty((1, 4), dtype=torch.int32, device="cuda")
    rc, T = vol.extract_into(ISO, probe)                     # cold, sizes the output
    assert rc in (0, bc._capi.E_CAPACITY)
    st_cold = vol.stats()
    assert st_cold["n_new"] == st_cold["n_active"] and st_cold["n_evicted"] == 0
    out = torch.empty((3 * T + 64, 4), dtype=torch.int32, device="cuda")
    vol.reset_cache()
    rc, T1 = vol.extract_into(ISO, out)                      # cold again, into the buffer
    assert rc == 0 and T1 == T
    st = vol.stats()
    say(f"  T={T} n_active={st['n_active']} n_occupied={st['n_occupied']}")

    active, I_active, may = vol.active(with_flags=True)
    cnt, off = vol.block_counts()
    assert len(I_active) == st["n_active"] == int(active.sum())
    assert np.all(np.diff(I_active.astype(np.int64)) > 0)
    assert int(cnt.sum()) == 3 * T
    assert np.array_equal(off[1:], np.cumsum(cnt[:-1], dtype=np.uint64))
    assert off[0] == 0
    occ = cnt > 0
    assert int(occ.sum()) == st["n_occupied"]
    assert int(may[I_active].sum()) == st["n_candidates"]
    assert np.all(cnt % 3 == 0)
    assert np.all(may[I_active[occ]] == 1)

    # whole soup: block ids follow the offsets, coordinates inside the block
    vblk = out[: 3 * T, 3].cpu().numpy().view(np.uint32)
    assert np.array_equal(vblk, np.repeat(I_active[occ], cnt[occ]))
    xyz = out[: 3 * T, :3].view(torch.float32)
    assert float(xyz.min()) >= 0.0 and float(xyz.max()) <= 4.0

    # sampled blocks against the oracle on their decoded neighbourhoods
    n_checked = 0
    for (bx, by, bz) in samples:
        D = orc.zfp_decode(orc.zfp_encode(kept[(bx, by, bz)], RATE), (12, 12, 12), RATE, True)
        rng_sub = orc.block_ranges(D, (12, 12, 12))
        act_sub = orc.active_blocks(rng_sub, (12, 12, 12), ISO)
        b = bx + nbx * (by + nby * bz)
        assert int(active[b]) == int(act_sub[13]), (bx, by, bz)
        group = [13 + dx + 3 * dy + 9 * dz for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)]
        lo = float(rng_sub[group, 0].min())
        hi = float(rng_sub[group, 1].max())
        if active[b]:
            assert int(may[b]) == int(lo < ISO <= hi), (bx, by, bz)
        r = orc.mc_extract(D, (12, 12, 12), ISO, want=("verts", "vblock"))
        ref64 = r["verts"][r["vblock"] == 13]
        v32, vb = orc.mc_extract_f32(D, (12, 12, 12), ISO)
        ref32 = v32[vb == 13]
        if not active[b]:
            assert ref64.shape[0] == 0, (bx, by, bz)
            continue
        i = int(np.searchsorted(I_active, b))
        assert I_active[i] == b
        assert int(cnt[i]) == ref64.shape[0], (bx, by, bz)
        if cnt[i]:
            got = out[int(off[i]): int(off[i]) + int(cnt[i])].cpu().numpy()
            assert np.all(got[:, 3].view(np.uint32) == b)
            g32 = got[:, :3].view(np.float32)
            assert np.array_equal(g32.view(np.uint32), ref32.astype(np.float32).view(np.uint32))
            assert np.max(np.abs(g32.astype(np.float64) - ref64)) <= 1e-5
            n_checked += 1
    say(f"  {n_checked} of {len(samples)} sampled blocks have triangles; all matched the oracle")
    assert n_checked >= 15

    # warm repeat: nothing decoded, same bytes
    before = out[: 3 * T].clone()
    rc, T2 = vol.extract_into(ISO, out)
    assert rc == 0 and T2 == T and vol.stats()["n_new"] == 0
    assert torch.equal(before, out[: 3 * T])
    vol.close()
