"""Helpers shared by the GPU parity tests (inputs come from synthetic/ and the
oracle; nothing here computes any part of the method)."""
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


def to_cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def verts_np(verts):
    """[3T,4] int32 CUDA records -> (float32 [3T,3], uint32 [3T])."""
    v = verts.cpu().numpy()
    return v[:, :3].view(np.float32).copy(), v[:, 3].view(np.uint32).copy()


def oracle_soup_by_slabs(orc, words, dims, rate, iso, is_f64=False, layers=8, workers=8,
                         want64=True):
    """The oracle's plain extract of a compressed volume, computed slab by
    slab of `layers` block layers (each slab decoded from its own words plus
    one halo layer, so that its last cells see the next layer's samples) on a
    thread pool.  Yields, in block order, (first block id, T, float32
    vertices, block ids, float64 vertices or None) per slab: the slabs'
    soups concatenated are the whole volume's canonical soup."""
    from concurrent.futures import ThreadPoolExecutor
    nx, ny, nz = dims
    nbx, nby, nbz = orc.block_dims(nx, ny, nz)
    per = nbx * nby
    words = np.asarray(words, dtype=np.uint64)

    def job(z0):
        z1 = min(z0 + layers, nbz)
        zl = z1 + 1 if z1 < nbz else z1          # decode one halo layer
        sub = words[z0 * per * rate: zl * per * rate]
        D = orc.zfp_decode(sub, (nx, ny, 4 * (zl - z0)), rate, is_f64)
        nzs = 4 * (z1 - z0) + 1 if z1 < nbz else nz - 4 * z0
        v32, vb = orc.mc_extract_f32(D, (nx, ny, nzs), iso)
        v64 = None
        if want64:
            r = orc.mc_extract(D, (nx, ny, nzs), iso, want=("verts",))
            v64 = r["verts"]
        assert np.all(vb < (z1 - z0) * per)
        return z0 * per, len(vb) // 3, v32, vb + np.uint32(z0 * per), v64

    with ThreadPoolExecutor(workers) as ex:
        futs = [ex.submit(job, z0) for z0 in range(0, nbz, layers)]
        for fu in futs:
            yield fu.result()
