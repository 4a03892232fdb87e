"""The allocation-free extraction entry point (bcmc_extract_blocks_noalloc,
all scratch in the library's static device array) against the allocating one
(bcmc_volume_from_blocks + bcmc_extract) on the same decoded blocks: byte
for byte, on two calls in a row with the second smaller, then a larger
first volume again, a capacity retry and a volume beyond the scratch."""
import numpy as np
import pytest

from synthetic import fields
from tests.gpu_common import say, torch_cuda

pytestmark = pytest.mark.gpu


def _reference(bc, blocks, dims, iso):
    vol = bc.FieldVolume(blocks, dims)
    verts, T = vol.extract(float(iso))
    ref = verts[: 3 * T].clone()
    vol.close()
    return ref, T


def _noalloc(bc, torch, blocks, dims, iso, cap):
    out = torch.full((cap, 4), -1, dtype=torch.int32, device="cuda")
    rc, T = bc.extract_blocks_noalloc(blocks, dims, float(iso), out)
    return rc, T, out


def test_noalloc_equals_allocating_extract(orc):
    torch = torch_cuda()
    import paper_2009_03254_amd as bc
    cases = [((150, 133, 97), 4101, 55), ((37, 29, 22), 4102, 40), ((150, 133, 97), 4101, 70)]
    for dims, seed, p in cases:
        nx, ny, nz = dims
        f = fields.turbulence(nx, ny, nz, seed=seed, n_modes=64)
        B = orc.field_to_blocks(f)
        iso = fields.percentile_iso(f, p)
        say(f"[noalloc] {dims} seed {seed} p{p}: {len(B)} blocks")
        blocks = torch.from_numpy(B).cuda()
        ref, T_ref = _reference(bc, blocks, dims, iso)
        assert T_ref == orc.mc_count(B, dims, iso) > 0
        rc, T, out = _noalloc(bc, torch, blocks, dims, iso, 3 * T_ref + 64)
        assert rc == 0 and T == T_ref, (rc, T, T_ref)
        assert torch.equal(out[: 3 * T], ref)
        assert bool((out[3 * T:] == -1).all())          # nothing written past the soup
    # capacity retry: too small a buffer reports T, a second call completes
    dims, seed, p = cases[1]
    f = fields.turbulence(*dims, seed=seed, n_modes=64)
    B = orc.field_to_blocks(f)
    iso = fields.percentile_iso(f, p)
    blocks = torch.from_numpy(B).cuda()
    ref, T_ref = _reference(bc, blocks, dims, iso)
    rc, T, out = _noalloc(bc, torch, blocks, dims, iso, 5)
    assert rc == bc._capi.E_CAPACITY and T == T_ref
    assert torch.equal(out[:5], ref[:5])
    rc, T, out = _noalloc(bc, torch, blocks, dims, iso, 3 * T)
    assert rc == 0 and torch.equal(out, ref)


def test_noalloc_rejects_volume_beyond_scratch():
    torch = torch_cuda()
    import paper_2009_03254_amd as bc
    dims = (512, 512, 512)
    blocks = torch.zeros((bc.num_blocks(*dims), 64), dtype=torch.float32, device="cuda")
    out = torch.empty((16, 4), dtype=torch.int32, device="cuda")
    with pytest.raises(bc.BcmcError, match="scratch"):
        bc.extract_blocks_noalloc(blocks, dims, 0.5, out)
