"""Pins of the oracle's helper functions that the GPU checks lean on: the
brute-force count over the block layout, the per-block vertex counts and the
decode of a list of blocks.  Each is checked against something other than
itself: the dense-field brute force, the axis-plane closed form, a per-cell
recount written out here in numpy, and the whole-volume decoder."""
import numpy as np

from synthetic import fields


def _blocks(orc, f):
    return orc.field_to_blocks(np.ascontiguousarray(f, dtype=np.float32))


def _cases_dense(f, iso):
    """Case of every cell of a dense [nz][ny][nx] field, written out from the
    corner and case conventions (corner k at (k&1, k>>1&1, k>>2&1); bit k set
    when that corner is < iso)."""
    nz, ny, nx = f.shape
    cs = np.zeros((nz - 1, ny - 1, nx - 1), dtype=np.int64)
    for k in range(8):
        dx, dy, dz = k & 1, (k >> 1) & 1, (k >> 2) & 1
        sub = f[dz:dz + nz - 1, dy:dy + ny - 1, dx:dx + nx - 1]
        cs |= (sub < iso).astype(np.int64) << k
    return cs


CASES = [
    (lambda: fields.turbulence(37, 29, 23, seed=6, n_modes=64), (0.3, -0.2)),
    (lambda: fields.sphere_sdf_noisy(40, 12.0, 0.5, seed=5), (0.0, 1.5)),
    (lambda: fields.gaussian_blobs(21, 3, seed=8)[:, :18, :], (1.2, 1.9)),
]


def test_brute_count_blocks_equals_dense(orc):
    for make, isos in CASES:
        f = make()
        nz, ny, nx = f.shape
        B = _blocks(orc, f)
        for iso in isos:
            T = orc.brute_count(f, iso)
            assert T > 0
            assert orc.brute_count_blocks(B, (nx, ny, nz), iso) == T


def test_brute_counts_axis_plane_closed_form(orc):
    # f = z - 10.3 crosses every column of cells once, in a cell of case 15
    # (two triangles): T = 2 (nx - 1)(ny - 1)
    for nx, ny, nz in ((21, 17, 25), (8, 5, 13)):
        f = fields.plane_z(nx, ny, nz, 10.3 if nz > 12 else 6.3)
        T = 2 * (nx - 1) * (ny - 1)
        assert orc.brute_count(f, 0.0) == T
        assert orc.brute_count_blocks(_blocks(orc, f), (nx, ny, nz), 0.0) == T


def test_block_vertex_counts(orc):
    nt, _, _ = orc.mc_tables()
    rng = np.random.default_rng(11)
    for make, isos in CASES:
        f = make()
        nz, ny, nx = f.shape
        dims = (nx, ny, nz)
        B = _blocks(orc, f)
        nbx, nby, nbz = orc.block_dims(nx, ny, nz)
        nb = nbx * nby * nbz
        for iso in isos:
            ids = np.arange(nb, dtype=np.uint32)
            cnt = orc.block_vertex_counts(B, dims, iso, ids)
            # all blocks together hold every cell once: 3 vertices per triangle
            assert int(cnt.sum(dtype=np.int64)) == 3 * orc.brute_count(f, iso)
            # a recount of sampled blocks (interior and boundary) from the dense field
            ntri = nt[_cases_dense(f, iso)]
            last = [b for b in range(nb) if (b % nbx == nbx - 1 or (b // nbx) % nby == nby - 1
                                             or b // (nbx * nby) == nbz - 1)]
            pick = np.unique(np.concatenate([rng.choice(nb, 24, replace=False),
                                             rng.choice(last, 12, replace=False), [0, nb - 1]]))
            sub = orc.block_vertex_counts(B, dims, iso, pick.astype(np.uint32))
            for b, c in zip(pick, sub):
                bx, by, bz = b % nbx, (b // nbx) % nby, b // (nbx * nby)
                # cells of the block: lowest corner inside it, all 8 corners in the volume
                blk = ntri[4 * bz:min(4 * bz + 4, nz - 1), 4 * by:min(4 * by + 4, ny - 1),
                           4 * bx:min(4 * bx + 4, nx - 1)]
                assert int(c) == 3 * int(blk.sum()), (b, int(c), 3 * int(blk.sum()))
            # ids in any order, repeated
            perm = pick[::-1].copy()
            again = orc.block_vertex_counts(B, dims, iso, np.concatenate([perm, perm]).astype(np.uint32))
            assert np.array_equal(again, np.concatenate([sub[::-1], sub[::-1]]))


def test_decode_some_equals_rows_of_decode_all(orc):
    rng = np.random.default_rng(12)
    for dtype, rates in ((np.float32, (1, 8, 16, 32)), (np.float64, (2, 16, 64))):
        f = fields.turbulence(26, 19, 11, seed=9, n_modes=32, dtype=dtype)
        nz, ny, nx = f.shape
        is64 = dtype == np.float64
        for rate in rates:
            s = orc.zfp_encode(f, rate)
            D = orc.zfp_decode(s, (nx, ny, nz), rate, is_f64=is64)
            nb = len(D)
            ids = np.concatenate([[nb - 1, 0], rng.integers(0, nb, 40), [nb - 1]]).astype(np.uint32)
            got = orc.zfp_decode_some(s, ids, rate, is_f64=is64)
            assert np.array_equal(got.view(np.uint32), D[ids].view(np.uint32)), (dtype, rate)
            # the block's words alone suffice: decode from a copy holding only them
            for b in (0, nb // 2, nb - 1):
                only = np.zeros_like(s)
                only[b * rate:(b + 1) * rate] = s[b * rate:(b + 1) * rate]
                one = orc.zfp_decode_some(only, np.array([b], np.uint32), rate, is_f64=is64)
                assert np.array_equal(one[0].view(np.uint32), D[b].view(np.uint32))
