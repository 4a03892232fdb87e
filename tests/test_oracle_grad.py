"""Pins of the oracle's FP64 gradient through the edge interpolation
t = (iso - a) / (b - a) with the topology held fixed: central finite
differences (step 1e-6; local over the edges incident to a sample, global
for the isovalue) and the exact shift and scale identities."""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest

from synthetic import fields


@pytest.fixture(scope="module")
def small_case(orc):
    f = fields.gaussian_blobs(24, 4, seed=13)
    B = orc.field_to_blocks(f)
    dims = (24, 24, 24)
    iso = fields.percentile_iso(f, 50)
    r = orc.mc_extract(B, dims, iso, want=("verts", "vblock"))
    vg = orc.verts_global(r["verts"], r["vblock"], dims)
    c = np.array([11.5, 11.5, 11.5])
    R = 6.0
    L, gV = orc.sphere_loss(vg, c, R)
    df, di = orc.mc_backward(B, dims, iso, gV)
    return dict(B=B, dims=dims, iso=iso, c=c, R=R, L=L, df=df, di=di, T=r["T"])


def test_sphere_loss_gradient_fd(orc):
    rng = np.random.default_rng(0)
    v = rng.uniform(0, 20, (30, 3))
    c = np.array([10.0, 9.0, 11.0])
    L, g = orc.sphere_loss(v, c, 4.0)
    h = 1e-6
    for j in range(30):
        for k in range(3):
            vp, vm = v.copy(), v.copy()
            vp[j, k] += h
            vm[j, k] -= h
            fd = (orc.sphere_loss(vp, c, 4.0)[0] - orc.sphere_loss(vm, c, 4.0)[0]) / (2 * h)
            assert fd == pytest.approx(g[j, k], rel=1e-6, abs=1e-6)


def _local_fd_setup(orc, n=40):
    """A 40^3 blob field with its soup's edge multiplicities and the oracle's
    analytic gradient in dense layout."""
    f = fields.gaussian_blobs(n, 6, seed=13)
    dims = (n, n, n)
    B = orc.field_to_blocks(f)
    iso = fields.percentile_iso(f, 50)
    r = orc.mc_extract(B, dims, iso, want=("verts", "vblock", "vedge"))
    vg = orc.verts_global(r["verts"], r["vblock"], dims)
    c = np.array([(n - 1) / 2.0] * 3)
    R = 12.0
    _, gV = orc.sphere_loss(vg, c, R)
    df, di = orc.mc_backward(B, dims, iso, gV)
    keys, mult = np.unique(r["vedge"], return_counts=True)
    return dict(f=f, n=n, iso=iso, c=c, R=R, G=orc.blocks_to_field(df, dims), di=di,
                edges=dict(zip(keys.tolist(), mult.tolist())), T=r["T"])


def _incident_edges(s, x, y, z):
    """Soup edges with sample u = (x, y, z) as an endpoint: (p0, axis, a, b,
    multiplicity, u is p0).  The edge key is p0's sample index * 3 + axis."""
    n, flat = s["n"], s["f"].ravel()
    idx = lambda p: p[0] + n * (p[1] + n * p[2])
    u = (x, y, z)
    out = []
    for ax in range(3):
        for p0 in (u, tuple(u[d] - (d == ax) for d in range(3))):
            if p0[ax] < 0:
                continue
            m = s["edges"].get(idx(p0) * 3 + ax)
            if m is None:
                continue
            p1 = tuple(p0[d] + (d == ax) for d in range(3))
            out.append((p0, ax, float(flat[idx(p0)]), float(flat[idx(p1)]), m, p0 == u))
    return out


def _vertex_loss(p0, ax, a, b, iso, c, R, sqrt):
    """(|v - c| - R)^2 for the vertex p0 + t e_ax, t = (iso - a) / (b - a)."""
    t = (iso - a) / (b - a)
    q = [p0[d] + (t if d == ax else 0) - c[d] for d in range(3)]
    r = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]) - R
    return r * r


def _pick_samples(s, n_surface=2200, n_zero=200, seed=1):
    G = s["G"]
    rng = np.random.default_rng(seed)
    nz = np.argwhere(G != 0)
    zero = np.argwhere(G == 0)
    return (nz[rng.choice(len(nz), min(n_surface, len(nz)), replace=False)],
            zero[rng.choice(len(zero), n_zero, replace=False)])


def test_field_gradient_local_fd(orc):
    """Local central differences (step 1e-6) of L for one sample D_u: only the
    vertices on the soup edges incident to u move, so only they are summed.
    Evaluated in 40-digit decimal arithmetic (no cancellation floor), the FD
    matches the analytic FP64 gradient to 1e-6 relative; evaluated in float64
    with fsum, to 1e-6 relative plus the FD's own rounding floor.  Samples
    within 1e-5 of iso, or on an edge with |b - a| < 1e-2 (where the FD's
    truncation error h^2 / (b - a)^2 could reach 1e-8), are skipped and
    counted."""
    s = _local_fd_setup(orc)
    getcontext().prec = 40
    Dm = lambda v: Decimal(float(v))
    h, hD = 1e-6, Decimal("1e-6")
    cD, RD, isoD = [Dm(v) for v in s["c"]], Dm(s["R"]), Dm(s["iso"])
    c, R, iso = s["c"], s["R"], float(s["iso"])
    surf, zero = _pick_samples(s)
    checked = skipped = 0
    worst = 0.0
    for z, y, x in surf:
        terms = _incident_edges(s, x, y, z)
        assert terms, (x, y, z)            # a nonzero gradient needs a soup edge
        if (abs(float(s["f"][z, y, x]) - iso) < 1e-5
                or any(abs(b - a) < 1e-2 for _, _, a, b, _, _ in terms)):
            skipped += 1
            continue
        g = float(s["G"][z, y, x])
        # decimal
        Lp = Lm = Decimal(0)
        for p0, ax, a, b, m, isp0 in terms:
            A, B = Dm(a), Dm(b)
            ap, bp, am, bm = (A + hD, B, A - hD, B) if isp0 else (A, B + hD, A, B - hD)
            Lp += m * _vertex_loss(p0, ax, ap, bp, isoD, cD, RD, Decimal.sqrt)
            Lm += m * _vertex_loss(p0, ax, am, bm, isoD, cD, RD, Decimal.sqrt)
        fd = float((Lp - Lm) / (2 * hD))
        assert abs(fd - g) <= 1e-6 * abs(g), (x, y, z, fd, g)
        worst = max(worst, abs(fd - g) / abs(g))
        # float64
        lp, lm = [], []
        for p0, ax, a, b, m, isp0 in terms:
            ap, bp, am, bm = (a + h, b, a - h, b) if isp0 else (a, b + h, a, b - h)
            lp.append(m * _vertex_loss(p0, ax, ap, bp, iso, c, R, math.sqrt))
            lm.append(m * _vertex_loss(p0, ax, am, bm, iso, c, R, math.sqrt))
        fd64 = (math.fsum(lp) - math.fsum(lm)) / (2 * h)
        floor = 8 * np.finfo(np.float64).eps * (math.fsum(lp) + math.fsum(lm)) / h
        assert abs(fd64 - g) <= 1e-6 * abs(g) + floor, (x, y, z, fd64, g)
        checked += 1
    assert checked >= 2000 and skipped <= 0.1 * len(surf), (checked, skipped)
    assert worst < 1e-6
    # samples off the surface: no soup edge touches them, the gradient is exactly 0
    for z, y, x in zero:
        assert not _incident_edges(s, x, y, z)


def test_iso_gradient_fd(orc):
    """Global central difference of L in iso (every vertex moves), summed in
    40-digit decimal over the soup's edges with their multiplicities: 1e-6
    relative."""
    s = _local_fd_setup(orc)
    getcontext().prec = 40
    Dm = lambda v: Decimal(float(v))
    hD = Decimal("1e-6")
    cD, RD, isoD = [Dm(v) for v in s["c"]], Dm(s["R"]), Dm(s["iso"])
    n, flat = s["n"], s["f"].ravel()
    Lp = Lm = Decimal(0)
    for key, m in s["edges"].items():
        ax, i0 = key % 3, key // 3
        p0 = (i0 % n, (i0 // n) % n, i0 // (n * n))
        i1 = i0 + (1, n, n * n)[ax]
        A, B = Dm(flat[i0]), Dm(flat[i1])
        Lp += m * _vertex_loss(p0, ax, A, B, isoD + hD, cD, RD, Decimal.sqrt)
        Lm += m * _vertex_loss(p0, ax, A, B, isoD - hD, cD, RD, Decimal.sqrt)
    fd = float((Lp - Lm) / (2 * hD))
    assert abs(fd - s["di"]) <= 1e-6 * abs(s["di"]), (fd, s["di"])


def test_iso_gradient_fd_fixed_topology_loss(orc, small_case):
    s = small_case
    base = s["B"].astype(np.float64)
    h = 1e-6
    Lp = orc.sphere_loss_fixed_topology(base, s["B"], s["dims"], s["iso"], float(s["iso"]) + h,
                                        s["c"], s["R"])
    Lm = orc.sphere_loss_fixed_topology(base, s["B"], s["dims"], s["iso"], float(s["iso"]) - h,
                                        s["c"], s["R"])
    fd = (Lp - Lm) / (2 * h)
    assert fd == pytest.approx(s["di"], rel=1e-5)


def test_field_gradient_fd_fixed_topology_loss(orc, small_case):
    """Global FD of the oracle's fixed-topology loss (float64, fsum-like
    compensated sum): a cross-check of that loss, which the local FD above
    does not use."""
    s = small_case
    B, dims, iso = s["B"], s["dims"], s["iso"]
    base = B.astype(np.float64)
    h = 1e-6
    nz = np.argwhere(np.abs(s["df"]) > 0)
    rng = np.random.default_rng(1)
    picks = nz[rng.choice(len(nz), min(40, len(nz)), replace=False)]
    checked = 0
    for b, l in picks:
        if abs(base[b, l] - iso) < 10 * h:
            continue
        fp, fm = base.copy(), base.copy()
        fp[b, l] += h
        fm[b, l] -= h
        Lp = orc.sphere_loss_fixed_topology(fp, B, dims, iso, float(iso), s["c"], s["R"])
        Lm = orc.sphere_loss_fixed_topology(fm, B, dims, iso, float(iso), s["c"], s["R"])
        fd = (Lp - Lm) / (2 * h)
        g = s["df"][b, l]
        # the global sum of ~T terms of size |L|/T rounds to about eps * |L| / h
        floor = 8 * np.finfo(np.float64).eps * abs(s["L"]) / h
        assert abs(fd - g) <= 1e-6 * abs(g) + floor, (b, l, fd, g)
        checked += 1
    assert checked >= 30


def test_shift_and_scale_identities(orc, small_case):
    s = small_case
    df, di = s["df"], s["di"]
    D = s["B"].astype(np.float64)
    scale = np.abs(df).sum() + abs(di)
    # t is unchanged when field and iso shift together
    assert abs(df.sum() + di) <= 1e-9 * scale
    # ... or scale together
    assert abs((D * df).sum() + float(s["iso"]) * di) <= 1e-9 * (np.abs(D * df).sum() + abs(di))
