"""The command-line drain (plain C over lbm_abi.h) against the Python
binding of the same library: the same drainage results bit for bit, and a
drain stopped after one chunk, checkpointed and run again ends where the
uninterrupted one does."""
import os
import subprocess

import numpy as np
import pytest

import synth
from tests.cli_problem import CLI_REL, parse_output, write_problem

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLI = os.path.join(ROOT, CLI_REL)
CONV = dict(tol=1e-5, check_every=100, max_steps=3000, bisect_rel=0.02)


def _problem():
    p = synth.c2_problem(n=40, mean_r=32.0 * 40 / 96, seed=11, amp=0)
    p.rho_init = None          # the library's layered start (nw up to z_front)
    r_ins, _ = synth.throat_incircle(p.spheres)
    return p, synth.pc_ramp(synth.GAMMA_LAPLACE, r_ins, 5, 0.1, 0.9)


def _run(*args):
    print("lbm_drain", *args, flush=True)
    return subprocess.run([CLI, *args], capture_output=True, text=True, timeout=300)


def _same(a, b):
    for k in ("S", "steps", "status", "mass"):
        assert np.array_equal(a[k], b[k]), k
    for k in ("pce", "pce_lo", "pce_hi", "invaded_at", "n_bisect", "total_steps", "S_w"):
        assert a[k] == b[k], k


def test_cli_drain_equals_the_python_binding(tmp_path):
    from paper_1906_04722_amd import lbm
    p, pcs = _problem()
    path = str(tmp_path / "throat.txt")
    write_problem(path, p, pcs, CONV)
    r = _run(path, "--chunk", "700")
    assert r.returncode == 0, r.stderr
    got = parse_output(r.stdout)
    g = lbm.Throat(p)
    ref = g.drain(pcs, **CONV)
    mass, S_w = g.reduce()
    g.close()
    ref = dict(ref, mass=np.asarray(mass), S_w=S_w)
    print("cli", got["S"], got["pce"], "binding", ref["S"], ref["pce"], flush=True)
    assert ref["invaded_at"] >= 1 and ref["n_bisect"] >= 1   # the bisection ran
    assert got["failed"] == 0
    _same(got, ref)


def test_cli_resumes_from_its_checkpoint(tmp_path):
    p, pcs = _problem()
    path = str(tmp_path / "throat.txt")
    write_problem(path, p, pcs, CONV)
    whole = _run(path, "--chunk", "700")
    assert whole.returncode == 0, whole.stderr
    ck = str(tmp_path / "state.lbm")
    first = _run(path, "--chunk", "700", "--checkpoint", ck, "--max-chunks", "2")
    assert first.returncode == 3 and os.path.exists(ck), first.stderr
    rest = _run(path, "--chunk", "700", "--checkpoint", ck)
    assert rest.returncode == 0 and "resumed from" in rest.stderr, rest.stderr
    _same(parse_output(rest.stdout), parse_output(whole.stdout))
