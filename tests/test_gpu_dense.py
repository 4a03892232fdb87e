"""GPU parity of the dense data-parallel marching cubes baseline (Sec.
3.3.3): over an uncompressed field, bit for bit against the oracle's dense
scan (cells in global row-major order), the same triangles as the block
path's extract of the same field, and at the 512^3 size the benchmark times
it on, against the oracle run slab by slab."""
import numpy as np
import pytest

from synthetic import fields
from tests.gpu_common import say, to_cuda, torch_cuda

pytestmark = pytest.mark.gpu


def _rows(v):
    """Whole triangles as sorted rows (order-free comparison)."""
    r = v.reshape(-1, 12)
    return r[np.lexsort(r.T[::-1])]


@pytest.mark.parametrize("dims,seed", [((37, 29, 23), 61), ((70, 61, 53), 62), ((2, 5, 3), 63),
                                       ((129, 18, 20), 64)])
def test_dense_equals_oracle(orc, dims, seed):
    torch = torch_cuda()
    import paper_2009_03254_amd as bc
    f = fields.turbulence(*dims, seed=seed, n_modes=32)
    say(f"[dense] turbulence {dims}")
    dm = bc.DenseMC(dims)
    fd = to_cuda(f)
    B = orc.field_to_blocks(f)
    vol = bc.FieldVolume(to_cuda(B), dims)
    for p in (50, 10, 90):
        iso = fields.percentile_iso(f, p)
        verts, T = dm.extract(fd, float(iso))
        v, vb = orc.mc_extract_dense(f, iso)
        assert 3 * T == len(vb) == 3 * orc.brute_count(f, iso)
        got = verts.cpu().numpy()
        assert np.array_equal(got[:, :3].view(np.float32).view(np.uint32), v.view(np.uint32)), p
        assert np.array_equal(got[:, 3].view(np.uint32), vb), p
        cs = np.zeros(np.array(f.shape) - 1, dtype=np.int64)
        for k in range(8):
            dx, dy, dz = k & 1, (k >> 1) & 1, k >> 2
            cs |= (f[dz:dz + f.shape[0] - 1, dy:dy + f.shape[1] - 1, dx:dx + f.shape[2] - 1] < iso) << k
        assert dm.active_cells() == int(np.count_nonzero((cs != 0) & (cs != 255)))
        blk, Tb = vol.extract(float(iso))
        assert Tb == T
        if T:
            assert np.array_equal(_rows(got), _rows(blk.cpu().numpy()))
    # no surface; capacity retry
    verts, T = dm.extract(fd, float(f.max()) + 1.0)
    assert T == 0 and dm.active_cells() == 0
    iso = fields.percentile_iso(f, 50)
    small = torch.empty((4, 4), dtype=torch.int32, device="cuda")
    rc, T = dm.extract_into(fd, float(iso), small)
    assert (rc == bc._capi.E_CAPACITY) == (3 * T > 4)
    dm.close()
    vol.close()


def test_dense_turbulence512_full(orc):
    """The 512^3 float32 turbulence at p50, the size the benchmark times: the
    whole soup against the oracle's dense scan run on host threads by slabs of
    whole block layers."""
    torch = torch_cuda()
    from concurrent.futures import ThreadPoolExecutor
    import paper_2009_03254_amd as bc
    n = 512
    field = fields.turbulence_torch(n, seed=2, device="cuda")
    f = field.cpu().numpy()
    iso = fields.percentile_iso(f.ravel()[::7], 50)
    say(f"[dense] 512^3 turbulence, iso {float(iso):.6f}")
    dm = bc.DenseMC((n, n, n))
    verts, T = dm.extract(field, float(iso))
    got = verts.cpu().numpy()
    nb_layer = (n // 4) ** 2

    def slab(z0):
        z1 = min(z0 + 16, n - 1)                 # cells z0..z1-1 need planes z0..z1
        v, vb = orc.mc_extract_dense(np.ascontiguousarray(f[z0:z1 + 1]), iso)
        return v, vb + np.uint32((z0 // 4) * nb_layer)

    with ThreadPoolExecutor(16) as ex:
        parts = list(ex.map(slab, range(0, n - 1, 16)))
    pos = 0
    for v, vb in parts:
        k = len(vb)
        assert np.array_equal(got[pos:pos + k, 3].view(np.uint32), vb)
        assert np.array_equal(got[pos:pos + k, :3].view(np.float32).view(np.uint32), v.view(np.uint32))
        pos += k
    assert pos == 3 * T > 0
    say(f"  {T} triangles equal the oracle's")
    dm.close()
