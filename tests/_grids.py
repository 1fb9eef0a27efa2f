"""Tiny hand-made grids for oracle pins (input data only)."""
import math

import numpy as np

from paper_2307_16830_amd.gridgen import Grid


def grid_from(nb, branches, gens, pd, qd=None, gs=None, bs=None, vmin=0.94, vmax=1.06):
    """branches: list of (f, t, r, x, b, rate); gens: list of (bus, c2, c1, pmin, pmax, qmin, qmax)."""
    E = len(branches)
    G = len(gens)
    br = np.array(branches, dtype=float).reshape(E, 6) if E else np.zeros((0, 6))
    gn = np.array(gens, dtype=float).reshape(G, 7)
    pd = np.asarray(pd, dtype=float)
    return Grid(
        pd=pd, qd=np.asarray(qd if qd is not None else 0.3 * pd, dtype=float),
        gs=np.asarray(gs if gs is not None else np.zeros(nb), dtype=float),
        bs=np.asarray(bs if bs is not None else np.zeros(nb), dtype=float),
        vmin=np.full(nb, vmin), vmax=np.full(nb, vmax),
        f=br[:, 0].astype(np.int32), t=br[:, 1].astype(np.int32), r=br[:, 2].copy(), x=br[:, 3].copy(),
        b=br[:, 4].copy(), rate=br[:, 5].copy(), angmin=np.full(E, -math.pi / 3), angmax=np.full(E, math.pi / 3),
        gbus=gn[:, 0].astype(np.int32), c2=gn[:, 1].copy(), c1=gn[:, 2].copy(), c0=np.zeros(G),
        pmin=gn[:, 3].copy(), pmax=gn[:, 4].copy(), qmin=gn[:, 5].copy(), qmax=gn[:, 6].copy(),
    )


def random_point(model, rng, spread=0.2):
    """A random interior-ish point: angles in +-spread, vm around 1, flows and gens random."""
    L = model.L
    x = np.zeros(L.n)
    x[L.ova:L.ova + L.N] = rng.uniform(-spread, spread, L.N)
    x[L.ovm:L.ovm + L.N] = rng.uniform(0.95, 1.05, L.N)
    x[L.opg:L.opg + L.G] = rng.uniform(0.1, 1.0, L.G)
    x[L.oqg:L.oqg + L.G] = rng.uniform(-0.5, 0.5, L.G)
    x[L.op:L.op + 2 * L.E] = rng.uniform(-1, 1, 2 * L.E)
    x[L.oq:L.oq + 2 * L.E] = rng.uniform(-1, 1, 2 * L.E)
    return x


_CONFIG_CACHE = {}


def config_grid(name):
    """Generated benchmark grid by configuration name, generated once per test session (the 10k- and 80k-bus
    feasibility repairs take tens of seconds); every call returns a private copy."""
    import copy

    from paper_2307_16830_amd import gridgen
    if name not in _CONFIG_CACHE:
        _CONFIG_CACHE[name] = gridgen.make_config(name)
    return copy.deepcopy(_CONFIG_CACHE[name])
