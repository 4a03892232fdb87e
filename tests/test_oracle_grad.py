"""Pins of the oracle's FP64 gradient through the edge interpolation
t = (iso - a) / (b - a) with the topology held fixed: central finite
differences (step 1e-6) and the exact shift and scale identities."""
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


def test_field_gradient_fd(orc, small_case):
    s = small_case
    assert s["T"] > 100
    B, dims, iso = s["B"], s["dims"], s["iso"]
    base = B.astype(np.float64)
    h = 1e-6
    nz = np.argwhere(np.abs(s["df"]) > 0)
    rng = np.random.default_rng(1)
    picks = nz[rng.choice(len(nz), min(60, len(nz)), replace=False)]
    zero = np.argwhere(s["df"] == 0)
    picks = np.concatenate([picks, zero[rng.choice(len(zero), 10, replace=False)]])
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
        assert abs(fd - g) <= 1e-6 * max(1.0, abs(g)) + 1e-5 * max(1.0, abs(g)), (b, l, fd, g)
        checked += 1
    assert checked >= 50


def test_iso_gradient_fd(orc, small_case):
    s = small_case
    base = s["B"].astype(np.float64)
    h = 1e-6
    Lp = orc.sphere_loss_fixed_topology(base, s["B"], s["dims"], s["iso"], float(s["iso"]) + h,
                                        s["c"], s["R"])
    Lm = orc.sphere_loss_fixed_topology(base, s["B"], s["dims"], s["iso"], float(s["iso"]) - h,
                                        s["c"], s["R"])
    fd = (Lp - Lm) / (2 * h)
    assert fd == pytest.approx(s["di"], rel=1e-5)


def test_shift_and_scale_identities(orc, small_case):
    s = small_case
    df, di = s["df"], s["di"]
    D = s["B"].astype(np.float64)
    scale = np.abs(df).sum() + abs(di)
    # t is unchanged when field and iso shift together
    assert abs(df.sum() + di) <= 1e-9 * scale
    # ... or scale together
    assert abs((D * df).sum() + float(s["iso"]) * di) <= 1e-9 * (np.abs(D * df).sum() + abs(di))
