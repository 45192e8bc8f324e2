"""Inputs of the stored oracle drains (tests/golden/drain_oracle.json): six
throats rebuilt from seeds, each with its capillary-pressure ramp.  Shared by
the script that writes the stored values and by the GPU tests that compare
with them; it holds no arithmetic of the method (the ramps are equally spaced
multiples of the incircle estimate 2 gamma / r_ins)."""
import numpy as np

import synth

# steady state: |Delta S_w| < 1e-6 over 100 steps (at most 10 000 steps per
# ramp point or bisection run); bisection to a relative bracket of 0.5 %
CONV = dict(tol=1e-6, check_every=100, max_steps=10000, bisect_rel=0.005)

NAMES = ("tetra40_s2", "tetra40_s11", "tetra40_s12", "slit_gap6", "slit_gap5", "slit_gap8")


def case(name):
    """(problem, pc ramp) of a stored drain."""
    if name.startswith("tetra40_s"):
        seed = int(name[len("tetra40_s"):])
        # the 96^3 four-sphere throat's layout at 40^3 (mean radius 13.3 lu)
        p = synth.c2_problem(seed=seed, n=40, mean_r=32.0 * 40 / 96)
        r_ins, _ = synth.throat_incircle(p.spheres)
        return p, synth.pc_ramp(synth.GAMMA_LAPLACE, r_ins, 6, 0.1, 0.9)
    if name.startswith("slit_gap"):
        # the periodic slit throat: gaps of 5, 6 and 8 lu in 20, 20 and 24 lu
        # periods, each with its own seed
        gap = float(name[len("slit_gap"):])
        nx, seed = {5.0: (20, 9), 6.0: (20, 5), 8.0: (24, 7)}[gap]
        p = synth.constriction_problem(nx=nx, gap=gap, seed=seed)
        return p, np.linspace(0.2, 1.4, 6) * 2 * synth.GAMMA_LAPLACE / gap
    raise KeyError(name)
