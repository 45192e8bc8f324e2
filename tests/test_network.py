"""Pore-network drainage assembly: the pore network of a packing (geometry
pins), the reference rules on hand-built networks whose outcome is worked out
by hand, invariants on random networks, and the native implementation
(lbm_network_drain, host code) against the reference."""
import collections

import numpy as np
import pytest

import synth
from oracle import network as ref
from synth import network as net_geo


@pytest.fixture(scope="module")
def net():
    x, r, L, phi, _ = synth.dense_packing(120, seed=9)
    return net_geo.pore_network(x, r, L), L, phi


def test_network_geometry(net):
    nw, L, phi = net
    # the tetrahedra tile the cell and the sphere sectors add up to the
    # spheres, so the void volumes sum to the porosity times the cell
    assert abs(nw["pore_vol"].sum() / L ** 3 - (1.0 - phi)) < 1e-9
    th = nw["throats"]
    n = len(nw["pore_vol"])
    deg = collections.Counter()
    for a, b in th:
        assert a >= 0 or b >= 0
        deg[a] += 1
        deg[b] += 1
    # every pore body is a tetrahedron with four facets
    assert all(deg[p] == 4 for p in range(n))
    assert deg[net_geo.INLET] > 0 and deg[net_geo.OUTLET] > 0
    assert len(nw["facets"]) == len(th) == len(nw["apex"])


def test_chain_by_hand():
    # inlet -(1)- 0 -(2)- 1 -(9)- outlet, volumes 1 and 3
    th = [(-1, 0), (0, 1), (1, -2)]
    sw, inv, st = ref.drain([1.0, 3.0], th, [1.0, 2.0, 9.0], [0.5, 1.5, 2.5, 10.0])
    assert sw == [1.0, 0.75, 0.0, 0.0]
    assert inv == [1, 2] and st == [ref.N, ref.N]


def test_trapping_by_hand():
    # pore 2 reaches the outlet only through pore 1; invading 0 and 1 at
    # p = 2.5 traps it, and it keeps its fluid up to the last pressure
    th = [(-1, 0), (0, 1), (1, 3), (3, -2), (0, 2), (2, 1)]
    pce = [1.0, 2.0, 9.0, 100.0, 5.0, 5.0]
    vol = [1.0, 1.0, 2.0, 4.0]
    sw, inv, st = ref.drain(vol, th, pce, [2.5, 10.0])
    assert st == [ref.N, ref.N, ref.T, ref.N]
    assert inv == [0, 0, -1, 1]
    assert sw == [6.0 / 8.0, 2.0 / 8.0]


def test_order_of_equal_entry_pressures():
    # two candidates at the same entry pressure: the lower throat index goes
    # first, and its invasion traps the other pore before it is reached
    th = [(-1, 0), (-1, 1), (0, -2), (1, 0)]
    sw, inv, st = ref.drain([1.0, 1.0], th, [1.0, 1.0, 50.0, 50.0], [1.0])
    assert st == [ref.N, ref.T] and sw == [0.5]


def _random_pce(nw, seed, ties=False):
    rng = np.random.default_rng(seed)
    k = len(nw["throats"])
    pce = rng.lognormal(0.0, 0.4, k)
    if ties:
        pce = np.round(pce, 1)
    return pce


def _adj(throats, n):
    adj = [[] for _ in range(n)]
    for t, (a, b) in enumerate(throats):
        if a >= 0:
            adj[a].append((int(b), t))
        if b >= 0:
            adj[b].append((int(a), t))
    return adj


@pytest.mark.parametrize("seed", [1, 2])
def test_reference_invariants(net, seed):
    nw, _, _ = net
    pce = _random_pce(nw, seed)
    p = np.quantile(pce, np.linspace(0.05, 0.95, 12))
    sw, inv, st = ref.drain(list(nw["pore_vol"]), nw["throats"].tolist(), list(pce), list(p))
    assert all(a >= b for a, b in zip(sw, sw[1:]))
    n = len(st)
    adj = _adj(nw["throats"], n)
    # every invaded pore was reached through a passable throat from the inlet
    # or from a pore invaded no later than itself
    for v in range(n):
        if st[v] == ref.N:
            assert any((u == -1 or (u >= 0 and st[u] == ref.N and inv[u] <= inv[v]))
                       and pce[t] <= p[inv[v]] for u, t in adj[v])
        else:
            assert inv[v] == -1
    # trapped pores have no wetting path to the outlet, wetting ones do
    reach = set()
    stack = [v for v in range(n) if st[v] == ref.W and any(u == -2 for u, _ in adj[v])]
    reach.update(stack)
    while stack:
        v = stack.pop()
        for u, _ in adj[v]:
            if u >= 0 and st[u] == ref.W and u not in reach:
                reach.add(u)
                stack.append(u)
    assert all((st[v] == ref.W) == (v in reach) for v in range(n) if st[v] != ref.N)


@pytest.mark.parametrize("seed,ties", [(3, False), (4, True)])
def test_native_matches_reference(net, seed, ties):
    from paper_1906_04722_amd import network
    nw, _, _ = net
    pce = _random_pce(nw, seed, ties)
    pce[::17] = np.inf
    p = np.unique(np.quantile(pce[np.isfinite(pce)], np.linspace(0.02, 0.98, 16)))
    sw_r, inv_r, st_r = ref.drain(list(nw["pore_vol"]), nw["throats"].tolist(), list(pce),
                                  list(p))
    sw, inv, st = network.drain(nw["pore_vol"], nw["throats"], pce, p)
    assert np.array_equal(sw, np.array(sw_r))
    assert np.array_equal(inv, inv_r) and np.array_equal(st, st_r)
    assert (st == network.TRAPPED).any() and (st == network.INVADED).any()


def test_native_rejects_bad_input():
    from paper_1906_04722_amd import lbm, network
    with pytest.raises(lbm.LBMError):
        network.drain([1.0], [(-1, 0)], [1.0], [2.0, 1.0])   # pressures not increasing
    with pytest.raises(lbm.LBMError):
        network.drain([1.0], [(-1, 3)], [1.0], [1.0])        # pore index out of range
    with pytest.raises(lbm.LBMError):
        network.drain([1.0], [(-1, 0)], [np.nan], [1.0])     # entry pressure not a number
