"""GPU parity of the differentiable extract: forward through
torch.autograd.Function, hand-written backward kernel, against the oracle's
FP64 analytic gradient (itself pinned to finite differences on the CPU) and
the exact shift / scale identities.  Tolerances: ||dG||/||G|| <= 1e-4,
per-entry |dG| <= 1e-3 max|G|, d/diso relative 1e-4 (float32 atomics)."""
import numpy as np
import pytest

from synthetic import fields
from tests.gpu_common import say, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,radius", [(48, 12.0), (67, 16.0)])
def test_backward_matches_oracle(orc, n, radius):
    torch = torch_cuda()
    import paper_2009_03254_amd as bcmc
    say(f"[backward] blobs {n}^3")
    f = fields.gaussian_blobs(n, 8, seed=3 + n)
    dims = (n, n, n)
    B = orc.field_to_blocks(f)
    iso = fields.percentile_iso(f, 60)
    blocks = torch.from_numpy(B).cuda().requires_grad_(True)
    iso_t = torch.tensor(float(iso), device="cuda", requires_grad=True)
    xyz, blk = bcmc.ExtractFn.apply(blocks, iso_t, dims)
    r = orc.mc_extract(B, dims, iso, want=("verts", "vblock"))
    assert xyz.shape[0] == 3 * r["T"] and r["T"] > 100
    assert np.array_equal(blk.cpu().numpy().view(np.uint32), r["vblock"])
    c = np.full(3, (n - 1) / 2.0)
    g = bcmc.global_positions(xyz, blk, dims, dtype=torch.float64)
    loss = ((g - torch.tensor(c, device="cuda")).norm(dim=1) - radius).pow(2).sum()
    loss.backward()
    vg = orc.verts_global(r["verts"], r["vblock"], dims)
    L, gV = orc.sphere_loss(vg, c, radius)
    assert float(loss.detach()) == pytest.approx(L, rel=1e-5)
    df, di = orc.mc_backward(B, dims, iso, gV)
    got = blocks.grad.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(got - df) <= 1e-4 * np.linalg.norm(df)
    assert np.abs(got - df).max() <= 1e-3 * np.abs(df).max()
    assert float(iso_t.grad) == pytest.approx(di, rel=1e-4)
    # shift and scale identities hold for the GPU gradient too
    assert abs(got.sum() + float(iso_t.grad)) <= 1e-4 * (np.abs(got).sum() + abs(di))
    D = B.astype(np.float64)
    assert abs((D * got).sum() + float(iso) * float(iso_t.grad)) <= 1e-4 * (np.abs(D * got).sum() + abs(di))


def test_backward_no_surface(orc):
    torch = torch_cuda()
    import paper_2009_03254_amd as bcmc
    B = np.zeros((8, 64), np.float32)
    blocks = torch.from_numpy(B).cuda().requires_grad_(True)
    iso_t = torch.tensor(1.0, device="cuda", requires_grad=True)
    xyz, blk = bcmc.ExtractFn.apply(blocks, iso_t, (8, 8, 8))
    assert xyz.shape[0] == 0
    (xyz.sum() * 1.0).backward()
    assert float(blocks.grad.abs().sum()) == 0.0 and float(iso_t.grad) == 0.0


def test_forward_without_grad_reuses_volume(orc):
    """A forward under no_grad returns its pooled volume at once: repeated
    calls reuse one handle, give the oracle's soup, and a later forward +
    backward still matches the oracle's gradient sum identity."""
    torch = torch_cuda()
    import paper_2009_03254_amd as bcmc
    n = 40
    f = fields.gaussian_blobs(n, 6, seed=77)
    dims = (n, n, n)
    B = orc.field_to_blocks(f)
    iso = fields.percentile_iso(f, 55)
    blocks = torch.from_numpy(B).cuda().requires_grad_(True)
    iso_t = torch.tensor(float(iso), device="cuda", requires_grad=True)
    r = orc.mc_extract(B, dims, iso, want=("verts", "vblock"))
    v32, vb = orc.mc_extract_f32(B, dims, iso)
    pool = bcmc._POOL.setdefault(dims, [])
    for _ in range(3):
        with torch.no_grad():
            xyz, blk = bcmc.ExtractFn.apply(blocks, iso_t, dims)
        assert len(pool) == 1
        assert xyz.shape[0] == 3 * r["T"]
        assert np.array_equal(xyz.cpu().numpy().view(np.uint32), v32.view(np.uint32))
        assert np.array_equal(blk.cpu().numpy().view(np.uint32), vb)
    xyz, blk = bcmc.ExtractFn.apply(blocks, iso_t, dims)
    assert len(pool) == 0               # held until the backward
    (xyz.sum()).backward()
    assert len(pool) == 1
    got = blocks.grad.cpu().numpy().astype(np.float64)
    assert abs(got.sum() + float(iso_t.grad)) <= 1e-4 * (np.abs(got).sum() + abs(float(iso_t.grad)))


def _loss_backward(torch, bcmc, blocks_np, dims, iso, c, radius):
    blocks = torch.from_numpy(blocks_np).cuda().requires_grad_(True)
    iso_t = torch.tensor(float(iso), device="cuda", requires_grad=True)
    xyz, blk = bcmc.ExtractFn.apply(blocks, iso_t, dims)
    g = bcmc.global_positions(xyz, blk, dims, dtype=torch.float64)
    loss = ((g - torch.tensor(c, device="cuda")).norm(dim=1) - radius).pow(2).sum()
    loss.backward()
    return blocks, iso_t, xyz, blk, loss


def test_backward_config_workload_256(orc):
    """The differentiable workload at its full size, as the benchmark runs it:
    256^3 Gaussian blobs (16 blobs, seed 3), iso 0.5, L = sum (|v - c| - 64)^2
    with c the grid centre, against the oracle's FP64 analytic gradient."""
    torch = torch_cuda()
    import paper_2009_03254_amd as bcmc
    n, radius, iso = 256, 64.0, 0.5
    say("[backward] blobs 256^3, 16 blobs, seed 3, iso 0.5")
    f = fields.gaussian_blobs(n, 16, seed=3)
    dims = (n, n, n)
    B = orc.field_to_blocks(f)
    c = np.full(3, (n - 1) / 2.0)
    blocks, iso_t, xyz, blk, loss = _loss_backward(torch, bcmc, B, dims, iso, c, radius)
    r = orc.mc_extract(B, dims, iso, want=("verts", "vblock"))
    assert xyz.shape[0] == 3 * r["T"] and r["T"] > 100000
    assert np.array_equal(blk.cpu().numpy().view(np.uint32), r["vblock"])
    assert np.abs(xyz.detach().cpu().numpy().astype(np.float64) - r["verts"]).max() <= 1e-5
    vg = orc.verts_global(r["verts"], r["vblock"], dims)
    L, gV = orc.sphere_loss(vg, c, radius)
    assert float(loss.detach()) == pytest.approx(L, rel=1e-5)
    df, di = orc.mc_backward(B, dims, iso, gV)
    got = blocks.grad.cpu().numpy().astype(np.float64)
    say(f"  T={r['T']} rel {np.linalg.norm(got - df) / np.linalg.norm(df):.2e} "
        f"diso {float(iso_t.grad):.6e} vs {di:.6e}")
    assert np.linalg.norm(got - df) <= 1e-4 * np.linalg.norm(df)
    assert np.abs(got - df).max() <= 1e-3 * np.abs(df).max()
    assert float(iso_t.grad) == pytest.approx(di, rel=1e-4)
    assert abs(got.sum() + float(iso_t.grad)) <= 1e-4 * (np.abs(got).sum() + abs(di))
    D = B.astype(np.float64)
    assert abs((D * got).sum() + iso * float(iso_t.grad)) <= 1e-4 * (np.abs(D * got).sum() + abs(di))


def test_inplace_edit_before_backward_raises(orc):
    """Editing the field in place between the forward and the backward is
    refused by autograd's version check on the saved field."""
    torch = torch_cuda()
    import paper_2009_03254_amd as bcmc
    n = 32
    f = fields.gaussian_blobs(n, 4, seed=21)
    dims = (n, n, n)
    B = orc.field_to_blocks(f)
    iso = fields.percentile_iso(f, 50)
    blocks = torch.from_numpy(B).cuda().requires_grad_(True)
    iso_t = torch.tensor(float(iso), device="cuda", requires_grad=True)
    xyz, blk = bcmc.ExtractFn.apply(blocks, iso_t, dims)
    assert xyz.shape[0] > 0
    with torch.no_grad():
        blocks.mul_(-1.0)
    with pytest.raises(RuntimeError):
        xyz.sum().backward()
    # the pooled volume went back: a fresh forward + backward works
    with torch.no_grad():
        blocks.mul_(-1.0)
    blocks.grad = None
    xyz, blk = bcmc.ExtractFn.apply(blocks, iso_t, dims)
    xyz.sum().backward()
    assert blocks.grad is not None


def test_backward_rejects_changed_field(orc):
    """Through the C ABI, without autograd: the field's memory changes after
    the extract (negated, so blocks' vertex counts change); the backward
    reports an error instead of reading outside the forward's vertex ranges."""
    torch = torch_cuda()
    import paper_2009_03254_amd as bcmc
    n = 36
    f = fields.gaussian_blobs(n, 5, seed=22)
    dims = (n, n, n)
    B = orc.field_to_blocks(f)
    iso = float(fields.percentile_iso(f, 40))
    blocks = torch.from_numpy(B).cuda()
    vol = bcmc.FieldVolume(blocks, dims)
    verts, T = vol.extract(iso)
    assert T > 0
    gV = torch.ones((3 * T, 3), dtype=torch.float32, device="cuda")
    vol.backward(iso, gV)                  # unchanged field: fine
    blocks.copy_(torch.from_numpy(orc.field_to_blocks(f[::-1].copy())).cuda())
    with pytest.raises(RuntimeError):
        vol.backward(iso, gV)
    vol.close()


@pytest.mark.parametrize("fmt", ["edge8", "q10"])
def test_backward_after_8byte_extract(orc, fmt):
    """The backward follows the soup of the extract before it whatever that
    extract's record format: after an 8-byte-record extract it gives the same
    gradients (up to float32 summation order) as after a 16-byte one, and the
    oracle's."""
    torch = torch_cuda()
    import paper_2009_03254_amd as bcmc
    n = 40
    say(f"[backward] blobs 40^3 after a {fmt} extract")
    f = fields.gaussian_blobs(n, 6, seed=31)
    dims = (n, n, n)
    B = orc.field_to_blocks(f)
    iso = float(fields.percentile_iso(f, 60))
    blocks = torch.from_numpy(B).cuda()
    vol = bcmc.FieldVolume(blocks, dims)
    verts, T = vol.extract(iso)
    assert T > 1000
    gen = torch.Generator(device="cpu").manual_seed(5)
    gV = torch.randn((3 * T, 3), generator=gen, dtype=torch.float32).cuda()
    df16, di16 = (x.cpu().numpy().astype(np.float64) for x in vol.backward(iso, gV))
    vol.set_vertex_format(fmt)
    rec, T8 = vol.extract(iso)
    assert T8 == T
    df8, di8 = (x.cpu().numpy().astype(np.float64) for x in vol.backward(iso, gV))
    vol.close()
    assert np.linalg.norm(df8 - df16) <= 1e-5 * np.linalg.norm(df16)
    assert float(di8) == pytest.approx(float(di16), rel=1e-5)
    dfo, dio = orc.mc_backward(B, dims, iso, gV.cpu().numpy().astype(np.float64))
    assert np.linalg.norm(df8 - dfo) <= 1e-4 * np.linalg.norm(dfo)
    assert float(di8) == pytest.approx(dio, rel=1e-4)
