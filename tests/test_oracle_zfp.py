"""Pins of the oracle's fixed-rate ZFP codec against what the mathematics and
the paper fix (Sec. 3.3.4, Sec. 4.2.1; transform matrix from Lindstrom 2014).

The zfp library itself is not available, so bitstream compatibility with it is
"parity unpinned"; everything below is pinned by definitions, closed forms,
exactness cases, error bounds and the paper's printed compressed sizes."""
import json
import os

import numpy as np
import pytest

from synthetic import fields

HERE = os.path.dirname(os.path.abspath(__file__))

# Lindstrom's forward decorrelating transform and its inverse.
A = np.array([[4, 4, 4, 4], [5, 1, -1, -5], [-4, 4, 4, -4], [-2, 6, -6, 2]], dtype=np.float64) / 16
AINV = np.array([[4, 6, -4, -1], [4, 2, 4, 5], [4, -2, 4, -5], [4, -6, -4, 1]], dtype=np.float64) / 4


def test_matrix_pair_is_inverse():
    assert np.allclose(A @ AINV, np.eye(4))


@pytest.mark.parametrize("is_f64", [False, True])
def test_forward_lift_is_the_published_matrix(orc, is_f64):
    rng = np.random.default_rng(0)
    for _ in range(200):
        v = rng.integers(-2**20, 2**20, 4) * 16       # multiples of 16: no bit is dropped
        got = orc.fwd_lift(v, is_f64)
        assert np.array_equal(got, (A @ v).astype(np.int64)), (v, got)
        # and the inverse lift undoes it exactly, which pins it to A^-1
        back = orc.inv_lift(got, is_f64)
        assert np.array_equal(back, v)
        assert np.array_equal(back, np.rint(AINV @ got).astype(np.int64))


def test_transform_closed_forms(orc):
    # constant -> DC only; linear -> DC + slope; quadratic -> no cubic term
    assert list(orc.fwd_lift([16, 16, 16, 16])) == [16, 0, 0, 0]
    assert list(orc.fwd_lift([0, 16, 32, 48])) == [24, -16, 0, 0]
    assert list(orc.fwd_lift([0, 16, 64, 144])) == [56, -48, -16, 0]


def test_lift_roundtrip_error_small(orc):
    rng = np.random.default_rng(1)
    for _ in range(500):
        v = rng.integers(-2**29, 2**29, 4)
        back = orc.inv_lift(orc.fwd_lift(v))
        assert np.abs(back - v).max() <= 4


def test_negabinary_definition(orc):
    rng = np.random.default_rng(2)
    vals = list(rng.integers(-2**30, 2**30, 300)) + [0, 1, -1, 2, -2, 2**30 - 1, -2**30]
    for i in vals:
        u = orc.to_negabinary(int(i))
        # base -2 digits of u must evaluate to i
        assert sum(((u >> k) & 1) * (-2) ** k for k in range(32)) == int(i)
        assert orc.from_negabinary(u) == int(i)
    for i in list(rng.integers(-2**62, 2**62, 100)):
        u = orc.to_negabinary(int(i), True)
        assert sum(((u >> k) & 1) * (-2) ** k for k in range(64)) == int(i)
        assert orc.from_negabinary(u, True) == int(i)


def test_sequency_order(orc):
    p = orc.sequency_order()
    assert sorted(p.tolist()) == list(range(64))
    seq = [(i & 3) + ((i >> 2) & 3) + (i >> 4) for i in p]
    assert seq == sorted(seq)
    for a, b in zip(p[:-1], p[1:]):
        sa = (a & 3) + ((a >> 2) & 3) + (a >> 4)
        sb = (b & 3) + ((b >> 2) & 3) + (b >> 4)
        assert sa < sb or (sa == sb and a < b)


def _random_coeffs(rng, bits=32):
    # negabinary words with a decaying number of significant bits
    u = np.zeros(64, dtype=np.uint64)
    for i in range(64):
        nb = max(0, bits - int(rng.integers(0, bits)) - i // 4)
        u[i] = np.uint64(int(rng.integers(0, 2**max(nb, 1))) if nb else 0)
    return u


def test_plane_coding_roundtrip_and_prefix(orc):
    rng = np.random.default_rng(3)
    for _ in range(60):
        u = _random_coeffs(rng)
        words, used = orc.encode_planes(u, 1 << 14)
        assert used < (1 << 14)
        assert np.array_equal(orc.decode_planes(words, 1 << 14), u)
        # embedded (progressive) code: a smaller budget gives a prefix of the stream
        for budget in (7, 64, 129, 500, used - 1):
            w2, used2 = orc.encode_planes(u, budget)
            assert used2 == min(budget, used)
            bits_full = np.unpackbits(words.view(np.uint8), bitorder="little")[:used2]
            bits_cut = np.unpackbits(w2.view(np.uint8), bitorder="little")
            assert np.array_equal(bits_full, bits_cut[:used2])
            assert not bits_cut[used2:].any()


def test_plane_coding_truncation_keeps_high_planes(orc):
    # decoding a truncated stream recovers every plane that was sent in full
    rng = np.random.default_rng(4)
    for _ in range(40):
        u = _random_coeffs(rng)
        for budget in (100, 300, 700):
            words, used = orc.encode_planes(u, budget)
            d = orc.decode_planes(words, budget)
            # find the lowest plane k such that decoding is exact on planes >= k
            diff = np.bitwise_xor(d, u)
            top_bad = max((int(x).bit_length() for x in diff), default=0)
            # bits above the partially sent plane agree
            assert all(((int(a) >> top_bad) == (int(b) >> top_bad)) for a, b in zip(d, u))
            assert top_bad <= 32


def _roundtrip(orc, f, rate, is_f64=False):
    nz, ny, nx = f.shape
    s = orc.zfp_encode(f, rate)
    assert s.nbytes == orc.num_blocks(nx, ny, nz) * 8 * rate
    d = orc.zfp_decode(s, (nx, ny, nz), rate, is_f64)
    return s, d


def test_zero_block_exact(orc):
    f = np.zeros((4, 4, 4), np.float32)
    s, d = _roundtrip(orc, f, 2)
    assert not s.any() and not d.any()


def test_header_layout(orc):
    # one block whose largest magnitude is 1.0 = 0.5 * 2^1 -> emax = 1
    f = np.full((4, 4, 4), 0.25, np.float32)
    f[0, 0, 0] = 1.0
    s = orc.zfp_encode(f, 4)
    w = int(s[0])
    assert w & 1 == 1
    assert (w >> 1) & 0xFF == 1 + 127
    s64 = orc.zfp_encode(f.astype(np.float64), 4)
    w = int(s64[0])
    assert w & 1 == 1 and (w >> 1) & 0x7FF == 1 + 1023


@pytest.mark.parametrize("rate", [2, 4, 8, 16])
def test_constant_block_exact(orc, rate):
    rng = np.random.default_rng(5)
    for c in list(rng.standard_normal(20) * 10.0 ** rng.integers(-30, 30, 20)) + [1.0, -3.5]:
        f = np.full((4, 4, 4), c, np.float32)
        _, d = _roundtrip(orc, f, rate)
        assert np.array_equal(d[0], f.ravel()), c
        f64 = np.full((4, 4, 4), c, np.float64)
        s = orc.zfp_encode(f64, rate)
        d64 = orc.zfp_decode_f64(s, (4, 4, 4), rate)
        assert np.array_equal(d64[0], f64.ravel()), c


def test_linear_block_near_exact(orc):
    z, y, x = np.meshgrid(np.arange(4), np.arange(4), np.arange(4), indexing="ij")
    rng = np.random.default_rng(6)
    for _ in range(20):
        a, b, c, d0 = rng.uniform(-1, 1, 4)
        f = (d0 + a * x + b * y + c * z).astype(np.float32)
        _, d = _roundtrip(orc, f, 8)
        emax = np.frexp(np.abs(f).max())[1]
        assert np.abs(d[0] - f.ravel()).max() <= 2.0 ** (emax - 20)


def test_full_rate_error_bound(orc):
    # rate 32 (f32): only the lowest planes are cut; truncation + lifting
    # rounding + those planes stay below 2^10 units of 2^(emax-30)
    rng = np.random.default_rng(7)
    f = (rng.standard_normal((16, 16, 16)) * 10.0 ** rng.uniform(-3, 3)).astype(np.float32)
    _, d = _roundtrip(orc, f, 32)
    B = orc.field_to_blocks(f)
    emax = np.frexp(np.abs(B).max(axis=1))[1]
    err = np.abs(d - B).max(axis=1)
    assert np.all(err <= 2.0 ** (emax - 20.0))
    # f64 at rate 64: 2^(emax-52)
    f64 = rng.standard_normal((8, 8, 8))
    s = orc.zfp_encode(f64, 64)
    d64 = orc.zfp_decode_f64(s, (8, 8, 8), 64)
    B64 = orc.field_to_blocks(f64)
    emax = np.frexp(np.abs(B64).max(axis=1))[1]
    assert np.all(np.abs(d64 - B64).max(axis=1) <= 2.0 ** (emax - 52.0))


def test_error_decreases_with_rate(orc):
    f = fields.turbulence(32, seed=11, n_modes=64)
    B = orc.field_to_blocks(f)
    errs = []
    for rate in (1, 2, 4, 8, 16, 32):
        _, d = _roundtrip(orc, f, rate)
        errs.append(float(np.sqrt(np.mean((d.astype(np.float64) - B) ** 2))))
    assert all(e1 >= e2 for e1, e2 in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-6 and errs[0] > errs[-1] * 100


def test_f64_stream_rounds_to_f32(orc):
    f = fields.turbulence(12, 9, 7, seed=12, n_modes=16, dtype=np.float64)
    s = orc.zfp_encode(f, 2)
    d64 = orc.zfp_decode_f64(s, (12, 9, 7), 2)
    d32 = orc.zfp_decode(s, (12, 9, 7), 2, is_f64=True)
    assert np.array_equal(d64.astype(np.float32), d32)


def test_partial_blocks_replicate_edges(orc):
    rng = np.random.default_rng(8)
    f = rng.standard_normal((7, 6, 5)).astype(np.float32)
    s, d = _roundtrip(orc, f, 32)
    assert s.size == 2 * 2 * 2 * 32
    B = orc.field_to_blocks(f)
    assert np.abs(d - B).max() < 1e-5
    back = orc.blocks_to_field(d, (5, 6, 7))
    assert back.shape == f.shape and np.abs(back - f).max() < 1e-5


def test_nonfinite_rejected(orc):
    f = np.zeros((4, 4, 4), np.float32)
    f[1, 2, 3] = np.nan
    with pytest.raises(ValueError):
        orc.zfp_encode(f, 8)


def test_tiny_and_huge_magnitudes(orc):
    # exponent clamp keeps decoding in the normal range; subnormal inputs
    # decode to zero or to a normal multiple of the clamped scale
    f = np.full((4, 4, 4), 1e-40, np.float32)
    f[0, 0, 0] = 3e-39
    _, d = _roundtrip(orc, f, 16)
    assert np.all(np.isfinite(d)) and np.abs(d - f.ravel()).max() <= 2.0 ** -126
    g = np.full((4, 4, 4), 3e38, np.float32)
    _, d = _roundtrip(orc, g, 16)
    assert np.array_equal(d[0], g.ravel())


def test_stream_size_matches_paper_table(orc):
    with open(os.path.join(HERE, "golden", "paper_compressed_sizes.json")) as fh:
        gold = json.load(fh)
    for e in gold["entries"]:
        nx, ny, nz = e["dims"]
        nbytes = orc.num_blocks(nx, ny, nz) * 8 * e["rate"]
        assert round(nbytes / 1e6, e["decimals"]) == pytest.approx(e["printed_mb"]), e["name"]
    # padding to whole blocks is what makes Kingsnake and Backpack match
    unpadded = 1024 * 1024 * 795 * 2 / 8 / 1e6
    assert round(unpadded) != 209
