"""Pins of the oracle's marching cubes (Sec. 3.3.3) and block culling
(Sec. 4.1): exhaustive checks of the generated 256-case table, closed forms
(planes, sphere area and volume convergence), watertightness, a brute-force
triangle count and the exactness of the culling rule."""
import itertools

import numpy as np
import pytest

from synthetic import fields


# ---- cube geometry written out independently of the oracle ----------------
def corner(k):
    return np.array([k & 1, (k >> 1) & 1, (k >> 2) & 1])


def edge_ends(e):
    a = e >> 2
    other = [d for d in range(3) if d != a]
    p = [0, 0, 0]
    p[other[0]] = e & 1
    p[other[1]] = (e >> 1) & 1
    k0 = p[0] + 2 * p[1] + 4 * p[2]
    p[a] = 1
    return k0, p[0] + 2 * p[1] + 4 * p[2]


def edge_mid(e):
    k0, k1 = edge_ends(e)
    return (corner(k0) + corner(k1)) / 2.0


def edge_faces(e):
    """The two cube faces (axis, side) that contain edge e."""
    k0, _ = edge_ends(e)
    p = corner(k0)
    return {(d, int(p[d])) for d in range(3) if d != (e >> 2)}


def crossing(cs):
    return {e for e in range(12)
            if ((cs >> edge_ends(e)[0]) & 1) != ((cs >> edge_ends(e)[1]) & 1)}


def tris_of(tri, nt, cs):
    t = tri[cs][: 3 * nt[cs]]
    return [tuple(t[3 * i: 3 * i + 3]) for i in range(nt[cs])]


@pytest.fixture(scope="module")
def tables(orc):
    return orc.mc_tables()


def test_edge_mask_closed_form(tables):
    nt, tri, em = tables
    for cs in range(256):
        assert {e for e in range(12) if (em[cs] >> e) & 1} == crossing(cs)


def test_vertices_are_exactly_the_crossing_edges(tables):
    nt, tri, em = tables
    assert nt[0] == 0 and nt[255] == 0 and nt.max() <= 5
    for cs in range(256):
        used = set(tri[cs][: 3 * nt[cs]].tolist())
        assert used == crossing(cs), cs
        assert all(v == -1 for v in tri[cs][3 * nt[cs]:])


def test_triangle_sides_face_segments_or_shared_diagonals(tables):
    nt, tri, em = tables
    for cs in range(1, 255):
        directed = {}
        for t in tris_of(tri, nt, cs):
            assert len(set(t)) == 3
            for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])):
                directed[(a, b)] = directed.get((a, b), 0) + 1
        for (a, b), n in directed.items():
            assert n == 1, (cs, a, b)
            if (b, a) not in directed:
                # used once: a boundary segment of the patch, lying in a face
                assert edge_faces(a) & edge_faces(b), (cs, a, b)
            # otherwise an interior diagonal shared by exactly two triangles
            # traversed in opposite directions
        boundary = {(a, b) for (a, b) in directed if (b, a) not in directed}
        # every crossing edge starts exactly one and ends exactly one boundary segment
        assert sorted(a for a, _ in boundary) == sorted(crossing(cs))
        assert sorted(b for _, b in boundary) == sorted(crossing(cs))


def _face_segments(tri, nt, cs, face):
    sides = set()
    for t in tris_of(tri, nt, cs):
        for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])):
            sides.add((a, b))
    return {(a, b) for (a, b) in sides if (b, a) not in sides
            and face in edge_faces(a) and face in edge_faces(b)}


def test_face_consistency(tables):
    """Cases that agree on a face's 4 corners cut that face identically
    (same directed segments), so neighbouring cells never crack."""
    nt, tri, em = tables
    for axis in range(3):
        for side in range(2):
            face = (axis, side)
            fcorners = [k for k in range(8) if corner(k)[axis] == side]
            ref = {}
            for cs in range(256):
                key = tuple((cs >> k) & 1 for k in fcorners)
                segs = _face_segments(tri, nt, cs, face)
                if key in ref:
                    assert ref[key] == segs, (face, cs)
                else:
                    ref[key] = segs


def test_orientation_toward_increasing_values(tables):
    """With inside corners at 0 and outside at 1 (iso 0.5), each triangle's
    normal has a positive component along the trilinear gradient."""
    nt, tri, em = tables
    for cs in range(1, 255):
        vals = np.array([0.0 if (cs >> k) & 1 else 1.0 for k in range(8)])
        for t in tris_of(tri, nt, cs):
            p = [edge_mid(e) for e in t]
            n = np.cross(p[1] - p[0], p[2] - p[0])
            c = sum(p) / 3
            g = np.zeros(3)
            for k in range(8):
                ck = corner(k)
                w = [(c[d] if ck[d] else 1 - c[d]) for d in range(3)]
                for d in range(3):
                    wd = list(w)
                    wd[d] = 1.0 if ck[d] else -1.0
                    g[d] += vals[k] * np.prod(wd)
            assert n @ g > 0, (cs, t)


def _blocks(orc, f):
    return orc.field_to_blocks(f)


def test_axis_plane_closed_form(orc):
    nx, ny, nz = 21, 18, 30
    f = fields.plane_z(nx, ny, nz, 10.3)
    B = _blocks(orc, f)
    r = orc.mc_extract(B, (nx, ny, nz), 0.0, want=("verts", "vblock"))
    assert r["T"] == 2 * (nx - 1) * (ny - 1)
    vg = orc.verts_global(r["verts"], r["vblock"], (nx, ny, nz))
    assert np.abs(vg[:, 2] - 10.3).max() < 1e-6
    tri = vg.reshape(-1, 3, 3)
    area = 0.5 * np.linalg.norm(np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0]), axis=1).sum()
    assert area == pytest.approx((nx - 1) * (ny - 1), rel=1e-9)


def _plane_box_polygon_area(n, d, box):
    """Area of {p : n.p = d} inside [0,box]: intersect the plane with the 12
    box edges, order the points around their centroid, sum the fan."""
    n = np.asarray(n, float)
    pts = []
    for a in range(3):
        o = [x for x in range(3) if x != a]
        for u, v in itertools.product((0, box[o[0]]), (0, box[o[1]])):
            p0 = np.zeros(3)
            p0[o[0]], p0[o[1]] = u, v
            if abs(n[a]) < 1e-15:
                continue
            t = (d - n @ p0) / n[a]
            if 0 <= t <= box[a]:
                q = p0.copy()
                q[a] = t
                pts.append(q)
    pts = np.unique(np.round(np.array(pts), 12), axis=0)
    c = pts.mean(axis=0)
    u = pts[0] - c
    u /= np.linalg.norm(u)
    w = np.cross(n / np.linalg.norm(n), u)
    ang = np.arctan2((pts - c) @ w, (pts - c) @ u)
    pts = pts[np.argsort(ang)]
    area = 0.0
    for i in range(len(pts)):
        area += 0.5 * np.linalg.norm(np.cross(pts[i] - c, pts[(i + 1) % len(pts)] - c))
    return area


def test_tilted_plane_closed_form(orc):
    nx, ny, nz = 23, 19, 17
    n = np.array([0.3, -0.5, 0.8])
    d = 2.0
    f = fields.tilted_plane(nx, ny, nz, n, d, dtype=np.float64)
    B = _blocks(orc, f.astype(np.float32))
    r = orc.mc_extract(B, (nx, ny, nz), 0.0, want=("verts", "vblock"))
    vg = orc.verts_global(r["verts"], r["vblock"], (nx, ny, nz))
    # every vertex on the plane (up to the float32 rounding of the samples)
    assert np.abs(vg @ n - d).max() < 1e-5
    tri = vg.reshape(-1, 3, 3)
    cr = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
    area = 0.5 * np.linalg.norm(cr, axis=1).sum()
    ref = _plane_box_polygon_area(n, d, (nx - 1, ny - 1, nz - 1))
    assert area == pytest.approx(ref, rel=1e-5)
    # normals point toward increasing f, i.e. along +n (zero-area fan
    # triangles of collinear vertices have no direction)
    big = np.linalg.norm(cr, axis=1) > 1e-6
    assert big.sum() > len(cr) // 2
    assert np.all(cr[big] @ n > 0)


def _area_volume(vg):
    tri = vg.reshape(-1, 3, 3)
    cr = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
    area = 0.5 * np.linalg.norm(cr, axis=1).sum()
    vol = np.einsum("ij,ij->i", tri[:, 0], np.cross(tri[:, 1], tri[:, 2])).sum() / 6.0
    return area, vol


def test_sphere_area_volume_converge(orc):
    errs = []
    for N in (32, 64, 128):
        R = 0.3125 * N
        f = fields.sphere_sdf(N, R)
        c = (N - 1) / 2.0
        r = orc.mc_extract(_blocks(orc, f), (N, N, N), 0.0, want=("verts", "vblock"))
        vg = orc.verts_global(r["verts"], r["vblock"], (N, N, N)) - c
        area, vol = _area_volume(vg)
        ea = abs(area / (4 * np.pi * R * R) - 1)
        ev = abs(vol / (4.0 / 3.0 * np.pi * R ** 3) - 1)
        assert vol > 0               # outward normals: inside is f < iso
        errs.append((ea, ev))
    assert errs[0][0] > errs[1][0] > errs[2][0]
    assert errs[0][1] > errs[1][1] > errs[2][1]
    assert errs[2][0] < 5e-3 and errs[2][1] < 5e-3
    # second-order convergence: halving h divides the error by about 4
    assert errs[1][1] / errs[2][1] > 2.5


def _check_watertight(vedge):
    tri = vedge.reshape(-1, 3)
    directed = {}
    for t in tri:
        assert len(set(t.tolist())) == 3
        for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])):
            directed[(int(a), int(b))] = directed.get((int(a), int(b)), 0) + 1
    for (a, b), n in directed.items():
        assert n == 1, (a, b)
        assert directed.get((b, a)) == 1, (a, b)    # shared by exactly 2, opposite


def test_watertight_noisy_sphere(orc):
    f = fields.sphere_sdf_noisy(64, 20.0, 0.5, seed=1)
    s = orc.zfp_encode(f, 16)
    D = orc.zfp_decode(s, (64, 64, 64), 16)
    r = orc.mc_extract(D, (64, 64, 64), 0.0, want=("vedge",))
    assert r["T"] > 10000
    _check_watertight(r["vedge"])


def test_brute_force_count(orc):
    for f, iso in ((fields.sphere_sdf_noisy(40, 12.0, 0.5, seed=5), 0.0),
                   (fields.turbulence(37, 29, 23, seed=6, n_modes=64), 0.3)):
        nz, ny, nx = f.shape
        B = _blocks(orc, f)
        assert orc.mc_count(B, (nx, ny, nz), iso) == orc.brute_count(f, iso)
        r = orc.mc_extract(B, (nx, ny, nz), iso, want=("cases", "cell_keys"))
        nt, _, _ = orc.mc_tables()
        assert int(nt[r["cases"]].sum()) == r["T"]
        assert np.all(np.diff(r["cell_keys"].astype(np.int64)) > 0)   # canonical order


def test_block_ranges(orc):
    f = fields.turbulence(22, 13, 9, seed=7, n_modes=32)
    nz, ny, nx = f.shape
    B = _blocks(orc, f)
    rg = orc.block_ranges(B, (nx, ny, nz))
    nbx, nby, nbz = orc.block_dims(nx, ny, nz)
    for b in range(len(rg)):
        bx, by, bz = b % nbx, (b // nbx) % nby, b // (nbx * nby)
        sub = f[4 * bz:4 * bz + 4, 4 * by:4 * by + 4, 4 * bx:4 * bx + 4]
        assert rg[b, 0] == sub.min() and rg[b, 1] == sub.max()


def _group_rule(rg, dims, iso):
    """Equivalent form of the culling rule: a block is active iff some 2x2x2
    group of blocks containing it has lo < iso <= hi over the group."""
    nbx, nby, nbz = [(n + 3) // 4 for n in dims]
    lo = rg[:, 0].reshape(nbz, nby, nbx)
    hi = rg[:, 1].reshape(nbz, nby, nbx)
    act = np.zeros((nbz, nby, nbx), bool)
    for z0 in range(-1, nbz):
        for y0 in range(-1, nby):
            for x0 in range(-1, nbx):
                zs = slice(max(z0, 0), min(z0 + 2, nbz))
                ys = slice(max(y0, 0), min(y0 + 2, nby))
                xs = slice(max(x0, 0), min(x0 + 2, nbx))
                if lo[zs, ys, xs].min() < iso <= hi[zs, ys, xs].max():
                    act[zs, ys, xs] = True
    return act.ravel()


def test_culling_rule_and_exactness(orc):
    for f, iso in ((fields.turbulence(41, 27, 34, seed=8, n_modes=64), 0.2),
                   (fields.sphere_sdf_noisy(36, 11.0, 0.5, seed=9), 0.0)):
        nz, ny, nx = f.shape
        dims = (nx, ny, nz)
        B = _blocks(orc, f)
        rg = orc.block_ranges(B, dims)
        act = orc.active_blocks(rg, dims, iso)
        assert np.array_equal(act.astype(bool), _group_rule(rg, dims, iso))
        # exact: every cell whose block is inactive is trivial (case 0 or 255)
        r = orc.mc_extract(B, dims, iso, want=("cell_keys",))
        owners = (r["cell_keys"] // 64).astype(np.int64)
        assert act[owners].all()
        # and the active blocks hold every sample any emitting cell reads
        nbx, nby, nbz = orc.block_dims(*dims)
        for key in r["cell_keys"][::7]:
            b, l = int(key) // 64, int(key) % 64
            bx, by, bz = b % nbx, (b // nbx) % nby, b // (nbx * nby)
            x, y, zz = 4 * bx + (l & 3), 4 * by + ((l >> 2) & 3), 4 * bz + (l >> 4)
            for k in range(8):
                cx, cy, cz = x + (k & 1), y + ((k >> 1) & 1), zz + ((k >> 2) & 1)
                nb = cx // 4 + nbx * (cy // 4 + nby * (cz // 4))
                assert act[nb]


def test_face_only_neighbours_would_be_wrong(orc):
    """Only the +x+y+z block holds values >= iso; face neighbours alone miss
    the cells that straddle the shared corner, the 26-neighbourhood does not."""
    f = np.zeros((8, 8, 8), np.float32)
    f[4:, 4:, 4:] = 1.0
    B = _blocks(orc, f)
    rg = orc.block_ranges(B, (8, 8, 8))
    act = orc.active_blocks(rg, (8, 8, 8), 0.5)
    assert act.all()
    r = orc.mc_extract(B, (8, 8, 8), 0.5, want=("cell_keys",))
    assert 0 in set((r["cell_keys"] // 64).tolist())   # block 0 emits the corner cell


def test_f32_mode_matches_f64_mode(orc):
    f = fields.sphere_sdf_noisy(32, 9.0, 0.5, seed=10)
    B = _blocks(orc, f)
    r = orc.mc_extract(B, (32, 32, 32), 0.0, want=("verts", "vblock"))
    v32, vb = orc.mc_extract_f32(B, (32, 32, 32), 0.0)
    assert np.array_equal(vb, r["vblock"])
    assert np.abs(v32 - r["verts"]).max() < 1e-6


def test_edge_records_decode_to_the_soup(orc):
    """64-bit edge records: same blocks and order as the soup, decoded
    positions within 2^-22 of the float64 vertices (the quantisation of t),
    q inside [0, 2^22), and every record's edge joins two corners of its cell
    on opposite sides of iso (checked on the dense field)."""
    dims = (29, 23, 19)
    f = fields.turbulence(*dims, seed=12, n_modes=32)
    blocks = orc.field_to_blocks(f)
    iso = float(fields.percentile_iso(f, 55))
    rec = orc.mc_extract_edge8(blocks, dims, iso)
    r = orc.mc_extract(blocks, dims, iso, want=("verts", "vblock"))
    assert rec.shape[0] == r["verts"].shape[0] > 0
    pos, blk = orc.edge8_positions(rec)
    assert np.array_equal(blk, r["vblock"])
    assert np.max(np.abs(pos - r["verts"])) <= 2.0 ** -22
    assert np.max(np.abs(pos - r["verts"])) <= 1e-5
    q = rec >> np.uint64(42)
    assert np.all(q < (1 << 22))
    nbx, nby = (dims[0] + 3) // 4, (dims[1] + 3) // 4
    org = np.stack([blk % nbx, (blk // nbx) % nby, blk // (nbx * nby)], axis=1).astype(np.int64) * 4
    g = np.floor(pos).astype(np.int64) + org              # first corner of each edge
    e = ((rec >> np.uint64(38)) & np.uint64(15)).astype(np.int64)
    step = np.eye(3, dtype=np.int64)[e >> 2]
    a = f[g[:, 2], g[:, 1], g[:, 0]]
    g1 = g + step
    b = f[g1[:, 2], g1[:, 1], g1[:, 0]]
    assert np.all((a < iso) != (b < iso))


def test_slab_orchestration_equals_whole_volume(orc):
    """The slab-by-slab driver the full-size GPU checks use (each slab decoded
    with one halo layer, block ids offset) gives the whole volume's soup."""
    from tests.gpu_common import oracle_soup_by_slabs
    for dims, layers, rate in (((37, 29, 45), 3, 8), ((24, 20, 32), 2, 4)):
        f = fields.turbulence(*dims, seed=3, n_modes=32)
        s = orc.zfp_encode(f, rate)
        D = orc.zfp_decode(s, dims, rate)
        iso = fields.percentile_iso(f, 50)
        v32, vb = orc.mc_extract_f32(D, dims, iso)
        r = orc.mc_extract(D, dims, iso)
        parts = list(oracle_soup_by_slabs(orc, s, dims, rate, iso, layers=layers, workers=4))
        assert sum(p[1] for p in parts) == len(vb) // 3 > 0
        assert np.array_equal(np.concatenate([p[2] for p in parts]).view(np.uint32), v32.view(np.uint32))
        assert np.array_equal(np.concatenate([p[3] for p in parts]), vb)
        assert np.array_equal(np.concatenate([p[4] for p in parts]), r["verts"])


def test_q10_vertices(orc):
    """Sec. 4.5's 8-byte vertex: 10-bit block-relative coordinates (nearest
    of 1024 even steps over [0, 4]) beside the block id.  Same blocks and
    order as the soup; dequantised positions within 2/1023 voxel (half a
    step) of the float64 vertices, the bound reached (about 2e-3 voxel);
    each code the nearest step to its float32 coordinate."""
    dims = (29, 23, 19)
    f = fields.turbulence(*dims, seed=12, n_modes=32)
    B = orc.field_to_blocks(f)
    iso = float(fields.percentile_iso(f, 45))
    rec = orc.mc_extract_q10(B, dims, iso)
    r = orc.mc_extract(B, dims, iso, want=("verts", "vblock"))
    v32, vb = orc.mc_extract_f32(B, dims, iso)
    assert len(rec) == len(vb) > 0
    pos, blk = orc.q10_positions(rec)
    assert np.array_equal(blk, r["vblock"])
    assert np.all((rec & np.uint64(0xC0000000)) == 0)
    err = np.abs(pos - r["verts"]).max()
    assert 1.5e-3 < err <= 2.0 / 1023 + 1e-6, err
    code = (rec & np.uint64(0xFFFFFFFF)).astype(np.int64)
    q = np.stack([code & 1023, (code >> 10) & 1023, (code >> 20) & 1023], axis=1)
    assert np.abs(q - v32.astype(np.float64) * (1023 / 4)).max() <= 0.5 + 1e-4


def test_q10_axis_plane_hand_worked(orc):
    """f = z - 10.3 on 9x7x13: every vertex at block-relative z = 2.3 (block
    layer 2) with x, y on the integer grid; codes worked out by hand:
    x, y in {0, 1, 2, 3, 4} -> {0, 256, 512, 767, 1023}, z 2.3 -> 588."""
    dims = (9, 7, 13)
    f = fields.plane_z(*dims, 10.3)
    rec = orc.mc_extract_q10(orc.field_to_blocks(f), dims, 0.0)
    assert len(rec) == 3 * 2 * 8 * 6
    code = (rec & np.uint64(0xFFFFFFFF)).astype(np.int64)
    assert set(((code >> 20) & 1023).tolist()) == {588}
    assert set((code & 1023).tolist()) <= {0, 256, 512, 767, 1023}
    assert set(((code >> 10) & 1023).tolist()) <= {0, 256, 512, 767, 1023}
    assert {0, 1023} <= set((code & 1023).tolist())


def test_dense_order_soup_is_the_block_soup_reordered(orc):
    """The dense scan's soup holds the block-order soup's triangles exactly:
    grouped per cell (global key of the cell) both give the same float32
    vertices, cell by cell; the count is the brute force's, and the cells
    come in global row-major order."""
    for dims, seed in (((37, 29, 23), 6), ((20, 33, 17), 8)):
        f = fields.turbulence(*dims, seed=seed, n_modes=32)
        iso = float(fields.percentile_iso(f, 40))
        v, vb = orc.mc_extract_dense(f, iso)
        assert len(vb) == 3 * orc.brute_count(f, iso) > 0
        B = orc.field_to_blocks(f)
        r = orc.mc_extract(B, dims, iso, want=("cell_keys", "cases"))
        v32, vb32 = orc.mc_extract_f32(B, dims, iso)
        nt, _, _ = orc.mc_tables()
        # the block soup's vertices per cell, keyed by global cell coordinates
        nx, ny, nz = dims
        nbx, nby = (nx + 3) // 4, (ny + 3) // 4
        keys = r["cell_keys"].astype(np.int64)
        bid, loc = keys // 64, keys % 64
        gx = 4 * (bid % nbx) + loc % 4
        gy = 4 * ((bid // nbx) % nby) + (loc // 4) % 4
        gz = 4 * (bid // (nbx * nby)) + loc // 16
        gkey = gx + nx * (gy + ny * gz)
        nv = 3 * nt[r["cases"]]
        starts = np.concatenate([[0], np.cumsum(nv)[:-1]])
        order = np.argsort(gkey, kind="stable")
        assert np.all(np.diff(gkey[order]) > 0)
        idx = np.concatenate([np.arange(starts[i], starts[i] + nv[i]) for i in order])
        assert np.array_equal(v.view(np.uint32), v32[idx].view(np.uint32))
        assert np.array_equal(vb, vb32[idx])
