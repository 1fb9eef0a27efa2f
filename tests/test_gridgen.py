"""The seeded instance generator: its random stream and its feasibility repairs (CPU only)."""
import numpy as np

from paper_2307_16830_amd import gridgen


def test_splitmix64_matches_published_outputs():
    # outputs of the SplitMix64 reference generator (Steele, Lea and Flood 2014; Vigna's reference code)
    assert [int(v) for v in gridgen.SplitMix64(1234567).raw(5)] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423, 4593380528125082431,
        16408922859458223821]
    assert [int(v) for v in gridgen.SplitMix64(0).raw(2)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4]
    u = gridgen.SplitMix64(7).uniform(10000)
    assert u.min() >= 0.0 and u.max() < 1.0 and abs(u.mean() - 0.5) < 0.01


def _dc_flows(g):
    """Branch flows of the DC power flow with generation in proportion to Pmax, solved densely."""
    N = g.nbus
    bl = 1.0 / g.x
    B = np.zeros((N, N))
    np.add.at(B, (g.f, g.f), bl)
    np.add.at(B, (g.t, g.t), bl)
    np.add.at(B, (g.f, g.t), -bl)
    np.add.at(B, (g.t, g.f), -bl)
    p = np.zeros(N)
    np.add.at(p, g.gbus, g.pmax * (g.pd.sum() / g.pmax.sum()))
    p -= g.pd
    th = np.zeros(N)
    th[1:] = np.linalg.solve(B[1:, 1:], p[1:])
    return bl * (th[g.f] - th[g.t])


def test_dc_rating_repair():
    N, E, G, seed = 400, 540, 32, 11
    raw = gridgen.make_grid(N, E, G, seed, repair=False)
    g = gridgen.make_grid(N, E, G, seed, repair="dc")
    lam = min(1.0, 0.75 * raw.pmax.sum() / raw.pd.sum())
    assert np.allclose(g.pd, lam * raw.pd, rtol=1e-15, atol=0)
    assert np.array_equal(g.f, raw.f) and np.array_equal(g.t, raw.t) and np.array_equal(g.x, raw.x)
    need = 1.25 * 1.044 * np.abs(_dc_flows(g))
    assert np.all(g.rate >= need * (1 - 1e-8))
    assert np.all(g.rate >= raw.rate)
    raised = g.rate > raw.rate
    assert np.allclose(g.rate[raised], need[raised], rtol=1e-8)
    assert g.repaired_branches == int(raised.sum())


def test_ac_repair_keeps_generation_above_load():
    g = gridgen.make_grid(300, 405, 60, 5)
    assert g.pd.sum() <= 0.75 * g.pmax.sum() + 1e-9
    assert np.all(g.rate > 0) and np.all(np.isfinite(g.bs))
