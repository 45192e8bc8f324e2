"""Checkpoint and resume across the C interface (lbm_save / lbm_load) and the
resumable drainage ramp (lbm_drain_begin / _advance / _get): a run stopped,
saved, loaded into a fresh handle and continued ends bit for bit where the
uninterrupted run ends (populations, saturations, steps, the entry-pressure
bracket)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

CONV = dict(tol=1e-5, check_every=100, max_steps=3000, bisect_rel=0.02)


def _throat():
    p = synth.c2_problem(n=40, mean_r=32.0 * 40 / 96, seed=11)
    r_ins, _ = synth.throat_incircle(p.spheres)
    return p, synth.pc_ramp(synth.GAMMA_LAPLACE, r_ins, 5, 0.1, 0.9)


def test_steps_resume_bitwise_after_save_and_load(tmp_path):
    from paper_1906_04722_amd import lbm
    p = synth.c1_problem(seed=1)
    a = lbm.Throat(p)
    a.step(60)
    a.set_rho_in(2.07)
    path = str(tmp_path / "state.lbm")
    a.save(path)
    b = lbm.Throat(p)
    b.set_schedule(lbm.LBM_SCHED_NODE_LIST)   # another launch shape: results are the same
    b.load(path)
    assert np.array_equal(a.f(), b.f())
    a.step(40)
    b.step(40)
    assert np.array_equal(a.f(), b.f())
    assert np.array_equal(a.density(), b.density())
    a.close()
    b.close()


def test_drainage_ramp_resumes_bitwise_after_save_and_load(tmp_path):
    from paper_1906_04722_amd import lbm
    p, pcs = _throat()
    ref_t = lbm.Throat(p)
    ref = ref_t.drain(pcs, **CONV)
    ref_f = ref_t.f()
    ref_t.close()
    print("uninterrupted", ref["S"], ref["steps"], ref["pce"], ref["n_bisect"], flush=True)
    assert ref["invaded_at"] >= 1 and ref["n_bisect"] >= 1
    # stop inside the bisection (after the first invaded point's steps) and
    # inside the ramp, save, resume in a fresh handle
    inv = ref["invaded_at"]
    cut_bisect = int(ref["steps"][:inv + 1].sum()) + 200
    for cut in (300, cut_bisect):
        a = lbm.Throat(p)
        a.drain_begin(pcs, **CONV)
        done = a.drain_advance(cut)
        part = a.drain_get()
        assert not done and part["total_steps"] <= cut
        path = str(tmp_path / f"ramp_{cut}.lbm")
        a.save(path)
        a.close()
        b = lbm.Throat(p)
        b.load(path, n_pc=len(pcs))
        mid = b.drain_get()
        assert np.array_equal(mid["S"], part["S"]) and mid["total_steps"] == part["total_steps"]
        while not b.drain_advance(1000):
            pass
        got = b.drain_get()
        print("resumed after", cut, "steps:", got["S"], got["steps"], got["pce"], flush=True)
        for k in ("S", "steps", "status"):
            assert np.array_equal(got[k], ref[k]), k
        for k in ("pce", "pce_lo", "pce_hi", "invaded_at", "n_bisect", "total_steps"):
            assert got[k] == ref[k], k
        assert got["done"] and not got["failed"]
        assert np.array_equal(b.f(), ref_f)
        b.close()


def test_load_refuses_another_subdomain(tmp_path):
    from paper_1906_04722_amd import lbm
    p, _ = _throat()
    a = lbm.Throat(p)
    a.step(10)
    path = str(tmp_path / "a.lbm")
    a.save(path)
    q = synth.c2_problem(n=40, mean_r=32.0 * 40 / 96, seed=12)   # other geometry
    b = lbm.Throat(q)
    b.step(5)
    before = b.f()
    with pytest.raises(lbm.LBMError) as e:
        b.load(path)
    assert e.value.code == lbm.LBM_EINVAL
    assert np.array_equal(b.f(), before)
    a.close()
    b.close()


def test_load_refuses_a_ramp_with_corrupt_settings(tmp_path):
    """A saved ramp whose convergence settings were damaged (check_every 0)
    is refused with LBM_EINVAL and leaves the handle as it was."""
    import struct
    from paper_1906_04722_amd import lbm
    p, pcs = _throat()
    a = lbm.Throat(p)
    a.drain_begin(pcs, **CONV)
    a.drain_advance(200)
    path = str(tmp_path / "ramp.lbm")
    a.save(path)
    a.close()
    raw = bytearray(open(path, "rb").read())
    # file layout: 112-byte header, inlet density, steps done, then the ramp:
    # phase, point, number of points, tol, check_every, ...
    phase, point, n = struct.unpack_from("<iii", raw, 128)
    tol, every = struct.unpack_from("<di", raw, 140)
    assert (phase, n, tol, every) == (1, len(pcs), CONV["tol"], CONV["check_every"])
    assert 0 <= point < n
    struct.pack_into("<i", raw, 148, 0)
    bad = str(tmp_path / "bad.lbm")
    open(bad, "wb").write(bytes(raw))
    b = lbm.Throat(p)
    b.step(7)
    before = b.f()
    with pytest.raises(lbm.LBMError) as e:
        b.load(bad, n_pc=len(pcs))
    assert e.value.code == lbm.LBM_EINVAL
    assert np.array_equal(b.f(), before)
    b.close()


def test_placement_search_keeps_the_state_bitwise():
    """lbm_place moves the populations into the fastest of several buffer
    pairs: the state is unchanged, and stepping on continues bit for bit as
    in a handle that was never moved."""
    from paper_1906_04722_amd import lbm
    p = synth.c1_problem(seed=2)
    a, b = lbm.Throat(p), lbm.Throat(p)
    a.step(31)                # odd: the state sits in the second buffer
    b.step(31)
    before = a.f()
    ms0, ms1 = a.place(3, 4)
    print("placement", ms0, "->", ms1, flush=True)
    assert 0 < ms1 <= ms0
    assert np.array_equal(a.f(), before)
    a.step(40)
    b.step(40)
    assert np.array_equal(a.f(), b.f())
    a.close()
    b.close()


def test_placement_search_respects_the_memory_budget():
    from paper_1906_04722_amd import lbm
    p = synth.c1_problem(seed=2)
    a = lbm.Throat(p)
    a.step(5)
    before = a.f()
    lbm.set_memory_budget(1 << 20)     # far below one more population buffer
    try:
        with pytest.raises(lbm.LBMError) as e:
            a.place(2, 4)
        assert e.value.code == lbm.LBM_ENOMEM
    finally:
        lbm.set_memory_budget(0)
    assert np.array_equal(a.f(), before)
    a.close()
