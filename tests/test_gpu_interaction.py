"""The interaction benchmarks' driver (Random, Sweep Up, Sweep Down over a
value range, Sec. 4.6.1) at reduced size: across each sequence the cache
carries over from surface to surface, and after every call the GPU's LRU
state equals the serial simulator's on the oracle's active blocks, the
triangle count the oracle's, and the reported hit rates the simulator's."""
import numpy as np
import pytest

from synthetic import fields
from tests.gpu_common import say, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["random", "sweep_up", "sweep_down"])
def test_interaction_sequence_matches_simulator(orc, kind):
    torch = torch_cuda()
    import paper_2009_03254_amd as bc
    from paper_2009_03254_amd import interaction
    n, rate = 64, 4
    dims = (n, n, n)
    f = fields.gaussian_blobs(n, 6, seed=71)
    s = orc.zfp_encode(f, rate)
    D = orc.zfp_decode(s, dims, rate)
    nb = orc.num_blocks(*dims)
    rg = orc.block_ranges(D, dims)
    lo, hi = fields.percentile_iso(f, 85), fields.percentile_iso(f, 99.5)
    isos = interaction.isovalues(kind, lo, hi, 40, seed=5)
    say(f"[interaction] {kind}: blobs {dims}, rate {rate}, 40 isovalues in [{lo:.3f}, {hi:.3f}]")
    vol = bc.Volume(s, dims, "f32", rate)
    vol.set_cache_budget(initial_bytes=0, max_bytes=0)
    sim = orc.LRU(nb, 0, nb)
    T_max = max(orc.mc_count(D, dims, float(i)) for i in isos)
    out = torch.empty((3 * T_max + 16, 4), dtype=torch.int32, device="cuda")
    hits = []

    def check(k, st):
        iso = isos[k]
        act = orc.active_blocks(rg, dims, iso)
        rc, I_new, ev = sim.update(act)
        assert rc == 0
        assert st["n_active"] == int(act.sum()) and st["n_new"] == len(I_new), k
        assert st["n_evicted"] == ev and st["n_slots"] == sim.n_slots, k
        I_slot, S_block, S_age = vol.cache_state()
        sI, sB, sA = sim.state()
        assert np.array_equal(I_slot, sI) and np.array_equal(S_block, sB), k
        assert np.array_equal(S_age, sA), k
        assert st["n_triangles"] == orc.mc_count(D, dims, iso), k
        hits.append(1.0 - len(I_new) / max(int(act.sum()), 1) if act.any() else 1.0)

    recs = interaction.run(vol, isos, out, profile=(kind == "random"), on_call=check)
    summ = interaction.summarise(recs, nb)
    say(f"  hit rate {summ['hit_rate']:.4f}, decoded per surface {summ['decoded_per_surface']:.4f}")
    assert summ["n_isovalues"] == 39
    assert summ["hit_rate"] == pytest.approx(float(np.mean(hits[1:])), abs=1e-12)
    if kind == "random":
        assert set(summ["stage_share"]) == set(interaction.STAGES)
        assert sum(summ["stage_share"].values()) == pytest.approx(1.0, abs=1e-3)
    else:
        assert "stage_share" not in summ
    vol.close()
