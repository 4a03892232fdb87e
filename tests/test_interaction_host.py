"""Host logic of the interaction benchmarks' driver (no GPU): the isovalue
sequences and the averages over a sequence's calls."""
import numpy as np
import pytest

from paper_2009_03254_amd import interaction


def test_isovalue_sequences():
    r = interaction.isovalues("random", 0.2, 0.8, 100, seed=3)
    assert r.dtype == np.float32 and len(r) == 100
    assert np.all((r >= 0.2) & (r <= 0.8))
    assert np.array_equal(r, interaction.isovalues("random", 0.2, 0.8, 100, seed=3))
    up = interaction.isovalues("sweep_up", 0.2, 0.8, 7)
    down = interaction.isovalues("sweep_down", 0.2, 0.8, 7)
    assert np.all(np.diff(up) > 0) and np.array_equal(up[::-1], down)
    assert up[0] == np.float32(0.2) and up[-1] == np.float32(0.8)
    with pytest.raises(ValueError):
        interaction.isovalues("zigzag", 0, 1)


def test_summary_discards_the_first_call():
    def rec(ms, n_new, n_act, T, slots, stages):
        return {"ms": ms, "n_new": n_new, "n_active": n_act, "n_triangles": T,
                "n_slots": slots, "hit_rate": 1.0 - n_new / n_act, "stage_ms": stages}
    z = [0.0] * 8
    recs = [rec(100.0, 50, 50, 9, 50, [5, 5, 5, 5, 0, 5, 0, 25]),
            rec(2.0, 10, 40, 4, 60, [1, 1, 2, 0, 0, 4, 0, 8]),
            rec(4.0, 0, 20, 6, 60, [1, 1, 0, 0, 0, 2, 0, 4])]
    s = interaction.summarise(recs, 100)
    assert s["n_isovalues"] == 2
    assert s["mean_ms"] == pytest.approx(3.0)
    assert s["hit_rate"] == pytest.approx((0.75 + 1.0) / 2)
    assert s["decoded_per_surface"] == pytest.approx(0.05)
    assert s["active_per_surface"] == pytest.approx(0.3)
    assert s["max_slots"] == 60
    want = {"cull": 2 / 12, "cache_update": 2 / 12, "decode": 2 / 12, "mc_count": 0.0, "emit": 6 / 12}
    assert s["stage_share"] == {k: pytest.approx(v, abs=1e-4) for k, v in want.items()}
    s0 = interaction.summarise([dict(r, stage_ms=z) for r in recs], 100)
    assert "stage_share" not in s0
