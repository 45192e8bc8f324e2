"""Batched drainage on the GPU against the FP64 oracle's drains of the same
throats (values stored by tests/golden/make_drain_golden.py, which calls only
the oracle).  Steady state is |Delta S_w| < 1e-6 over 100 steps and the entry
pressure is bisected to a 0.5 % bracket (Sec. 2.2.2: p_c^e is the largest
capillary pressure held before the non-wetting phase passes the throat).

Bars: the same first invaded ramp point, the saturation at every ramp point
within 1e-3, and the bisected p_c^e midpoints within 1 %."""
import json
import os

import numpy as np
import pytest

from tests.golden import drain_cases

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "drain_oracle.json")


def _stored():
    if not os.path.exists(GOLD):
        pytest.skip("stored oracle drains not written yet (tests/golden/make_drain_golden.py)")
    with open(GOLD) as f:
        g = json.load(f)
    assert g["conv"] == drain_cases.CONV
    return g["cases"]


def test_batched_drains_match_the_oracle():
    from paper_1906_04722_amd import lbm
    stored = _stored()
    names = [n for n in drain_cases.NAMES if n in stored]
    assert len(names) >= 3
    probs, pcs = [], []
    for n in names:
        p, pc = drain_cases.case(n)
        # the ramp the oracle drained (rebuilt here from the same seeds)
        assert np.allclose(pc, stored[n]["pc"], rtol=1e-12, atol=0)
        probs.append(p)
        pcs.append(stored[n]["pc"])
    print("batched drain of", names, flush=True)
    outs, info = lbm.drain_batch(probs, np.array(pcs), **drain_cases.CONV)
    print("batch info", info, flush=True)
    for n, b in zip(names, outs):
        o = stored[n]
        dS = float(np.max(np.abs(np.array(o["S"]) - b["S"])))
        print(f"{n}: invaded at {b['invaded_at']} (oracle {o['invaded_at']}), p_c^e "
              f"{b['pce']:.6g} (oracle {o['pce']:.6g}), max |dS| {dS:.2e}, steps {list(b['steps'])} "
              f"(oracle {o['steps']})", flush=True)
        assert not b["failed"]
        assert b["invaded_at"] == o["invaded_at"] >= 1
        assert dS <= 1e-3
        assert abs(b["pce"] - o["pce"]) <= 0.01 * o["pce"]


@pytest.mark.parametrize("name", ["slit_gap6", "tetra40_s2"])
def test_single_drain_matches_the_oracle(name):
    """lbm_drain_throat (the resumable host ramp run to its end) on a stored
    case: the same bars as the batch."""
    from paper_1906_04722_amd import lbm
    stored = _stored()
    if name not in stored:
        pytest.skip(f"{name} not stored")
    o = stored[name]
    p, _ = drain_cases.case(name)
    t = lbm.Throat(p)
    t.autotune(4)
    b = t.drain(np.array(o["pc"]), **drain_cases.CONV)
    t.close()
    dS = float(np.max(np.abs(np.array(o["S"]) - b["S"])))
    print(f"{name}: invaded at {b['invaded_at']} (oracle {o['invaded_at']}), p_c^e {b['pce']:.6g} "
          f"(oracle {o['pce']:.6g}), max |dS| {dS:.2e}", flush=True)
    assert b["invaded_at"] == o["invaded_at"] >= 1
    assert dS <= 1e-3
    assert abs(b["pce"] - o["pce"]) <= 0.01 * o["pce"]
