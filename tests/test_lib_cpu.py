"""CPU-side checks of the HIP library (no GPU needed): it loads, exports every
symbol include/bcmc.h declares, its generated marching cubes table equals the
oracle's independently generated one, and argument validation rejects bad
input before any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2009_03254_amd import _capi
    if not os.path.exists(_capi.LIB_PATH):
        from paper_2009_03254_amd import build
        build.build()
    return _capi.lib()


def _declared():
    with open(os.path.join(ROOT, "include", "bcmc.h")) as fh:
        src = fh.read()
    return sorted(set(re.findall(r"BCMC_API\s+[\w\s\*]*?\b(bcmc_\w+)\s*\(", src)))


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    from paper_2009_03254_amd import _capi
    assert set(_capi.SIGNATURES) == set(names)


def test_mc_table_equals_oracle(L, orc):
    import paper_2009_03254_amd as bcmc
    nt, tri = bcmc.mc_table()
    ont, otri, _ = orc.mc_tables()
    assert np.array_equal(nt, ont)
    assert np.array_equal(tri, otri)


def test_num_blocks(L):
    assert L.bcmc_num_blocks(64, 64, 64) == 4096
    assert L.bcmc_num_blocks(5120, 3840, 768) == 1280 * 960 * 192
    assert L.bcmc_num_blocks(5, 6, 7) == 8


def test_validation_before_device_work(L):
    h = C.c_void_p()
    buf = np.zeros(64, np.uint64)
    p = buf.ctypes.data_as(C.c_void_p)
    # wrong size, bad rate, bad type, tiny dims, null pointers
    assert L.bcmc_load_compressed(p, 8 * 63, 0, 4, 4, 4, 0, 8, None, C.byref(h)) == -1
    assert L.bcmc_load_compressed(p, 8 * 64, 0, 4, 4, 4, 0, 33, None, C.byref(h)) == -1
    assert L.bcmc_load_compressed(p, 8 * 64, 0, 4, 4, 4, 2, 8, None, C.byref(h)) == -1
    assert L.bcmc_load_compressed(p, 8 * 64, 0, 1, 4, 4, 0, 8, None, C.byref(h)) == -1
    assert L.bcmc_load_compressed(None, 8, 0, 4, 4, 4, 0, 1, None, C.byref(h)) == -1
    assert b"rate" in L.bcmc_last_error() or len(L.bcmc_last_error()) > 0
    assert L.bcmc_extract(None, C.c_float(0.0), None, 0, None, None) == -1
    assert L.bcmc_encode(None, 0, 4, 4, 4, 8, None, None) == -1
    assert L.bcmc_set_profiling(None, 1) == -1
    assert L.bcmc_set_profiling_stages(None, 0x20) == -1


def test_generated_triangle_count_circuit(L, orc):
    """The build-time bit-sliced triangle count (mc_ntri.h) gives, for every
    one of the 256 cases, the oracle table's triangle count: the 256 cases are
    evaluated at once, case c in bit c of four 64-bit words per corner."""
    from paper_2009_03254_amd import build
    path = os.path.join(build.GEN, "mc_ntri.h")
    if not os.path.exists(path):
        build.build()
    src = open(path).read()
    M = (1 << 64) - 1
    n_ref = orc.mc_tables()[0]

    def py(expr):   # C expression over uint64 -> Python expression on ints
        e = expr.replace("~0ull", "M").replace("0ull", "0")
        return re.sub(r"~(c\[\d\]|n\d+)", r"(M ^ \1)", e)

    for w in range(4):                    # cases 64w .. 64w+63
        c = [0] * 8
        for k in range(8):
            for i in range(64):
                if ((64 * w + i) >> k) & 1:
                    c[k] |= 1 << i
        env = {"c": c}
        for name, expr in re.findall(r"const uint64_t (n\d+) = (.*);", src):
            env[name] = eval(py(expr), {"M": M}, env) & M
        outs = {}
        for b in ("b0", "b1", "b2"):
            expr = re.search(rf"\b{b} = (.*);", src).group(1)
            outs[b] = eval(py(expr), {"M": M}, env) & M
        for i in range(64):
            n = ((outs["b0"] >> i) & 1) | (((outs["b1"] >> i) & 1) << 1) | (((outs["b2"] >> i) & 1) << 2)
            assert n == n_ref[64 * w + i], 64 * w + i
