"""Benchmark of the Shan-Chen drainage hot path on one MI355X.

Headline workload: the fully resolved 512^3 packed sample (a seeded dense
packing of 1000 polydisperse spheres scaled to fill the box, walls on the
sides, non-wetting bath at z = 0, wetting bath at z = 511), drained
quasi-statically over a 12-point capillary-pressure ramp.  Geometry,
initial state and launch shape are set up before the timed region (inputs
resident in HBM); one timed "step" is one pass of the hot path: 400 lattice
steps of the fused update (moments, cohesion and adhesion forces, velocity
shift, BGK collision, pull streaming with bounce-back, bath re-imposition)
with the FP64 saturation check every 100 steps and the ramp's decisions
(steady state, invasion probe, next pressure or bisection, state copies), as
lbm_drain_advance runs them.  value = fluid-node MLUPS over the timed steps.

Prints one JSON line with the roofline of the fused step kernel (HIP-event
timed launches inside the ramp), the FP64 CPU oracle timed on this host on a
crop of the same sample, and further legs: the batched drainage of 512 pore
throats in one lbm_drain_batch call, the 96^3 single-throat drainage and the
512^3 periodic box.  Progress goes to stderr.
"""
import argparse
import glob
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from paper_1906_04722_amd import lbm  # noqa: E402
from paper_1906_04722_amd import network  # noqa: E402
from paper_1906_04722_amd import surrogate  # noqa: E402

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, vendor figure
BYTES_PER_FLUID_NODE = 304   # 2 components x 19 FP32 populations, read + write
GAMMA = synth.GAMMA_LAPLACE  # interfacial tension of the model (Laplace fit)
# headline: the 512^3 packed sample, 12-point ramp; a timed step advances the
# drainage by STEP_LATTICE lattice steps (checks every 100)
SAMPLE_N, SAMPLE_SPHERES, SAMPLE_NPC = 512, 1000, 12
SAMPLE_CONV = dict(tol=1e-6, check_every=100, max_steps=2000, bisect_rel=0.01)
STEP_LATTICE = 400
# single 96^3 throat: 20-point ramp to steady state, bisection to 0.5 %
N_PC = 20
CONV = dict(tol=1e-6, check_every=100, max_steps=20000, bisect_rel=0.005)
# batched drainage: 512 throats cut from one seeded dense packing (radii
# lognormal, mean 1, log-sd 0.2, porosity 0.38), 32 lu per unit radius, box
# sides 48-128, 16-point ramp, entry pressure bracketed to 1 %, all in one
# lbm_drain_batch call
BATCH_THROATS = 512
BATCH_SINGLES = 4
BATCH_N_PC = 16
BATCH_CONV = dict(tol=1e-6, check_every=100, max_steps=600, bisect_rel=0.01)
SAMPLE_PLACEMENTS = 4   # extra population-buffer pairs tried by lbm_place
PLACEMENT = {}
# learned surrogate: trained on throats of one packing drained by the batched
# LBM, evaluated on throats of another packing against the plain LBM
SG_TEST, SG_INFER = 256, 100000
SG_CFG = {"train": 512}
SG_RES, SG_SIDES = 12.0, (24, 64)
SG_CONV = dict(tol=1e-6, check_every=100, max_steps=1500, bisect_rel=0.01)
SG_FIT = dict(epochs=200, batch=64, lr=1e-3, seed=2)
SG_THRESHOLD = 0.02
# hybrid assembly: pore network of a 40-sphere packing (the paper's sample
# size), each throat's entry pressure from the batched LBM, then the
# network drainage with trapping
HYB_SPHERES = 40
HYB_CONV = dict(tol=1e-6, check_every=100, max_steps=1500, bisect_rel=0.01)
BF16_PEAK_TFLOPS = 2500.0    # MI355X dense BF16 matrix cores, vendor figure
KERNEL_SRC = os.path.join(ROOT, "paper_1906_04722_amd", "csrc", "sc_kernels.hip")
PROFILES = os.path.join(ROOT, "profiles")


def log(msg):
    """Progress line on stderr (the JSON result line is the only stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def kernel_sha():
    from paper_1906_04722_amd.profile_run import kernel_sha as sha
    return sha(KERNEL_SRC)


def read_traffic(prefix, schedule):
    """HBM bytes per step from a committed counter summary (profiles/
    <prefix>*traffic.txt) taken on the current kernel source with the same
    launch shape; else None."""
    want = ",".join(str(int(v)) for v in schedule)
    for path in sorted(glob.glob(os.path.join(PROFILES, prefix + "*traffic.txt"))):
        kv = {}
        for line in open(path):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        if kv.get("kernel_sha") == kernel_sha() and kv.get("schedule") == want:
            try:
                return float(kv["traffic_bytes_per_launch"])
            except (KeyError, ValueError):
                return None
    return None


def step_kernels(schedule):
    """What one timed step launches for this launch shape."""
    if schedule[0] == lbm.LBM_SCHED_NODE_LIST:
        return ("k_dens_list + k_step_list (node-list step: densities of the non-solid nodes, "
                "then fused pull + cohesion/adhesion + BGK); figures per step")
    return (f"k_step<{schedule[0]},{schedule[1]}> lz {schedule[2]} (fused pull + moments + "
            "cohesion/adhesion + BGK)")


def c2_workload():
    p = synth.c2_problem()
    r_ins, _ = synth.throat_incircle(p.spheres)
    pcs = synth.pc_ramp(GAMMA, r_ins, N_PC)
    return p, pcs


def one_drain(p, pcs, schedule=None):
    g = lbm.Throat(p)
    if schedule:
        g.set_schedule(*schedule)
        sched = g.schedule()
    else:
        sched = g.autotune(20)
    g.step_timer(1)
    out = g.drain(pcs, **CONV)
    ms, launches = g.step_timer(-1)
    n_fluid = int((g.types() == lbm.LBM_NODE_FLUID).sum())
    g.close()
    out["schedule"] = sched
    return out, ms, launches, n_fluid


def _cpu_model():
    import subprocess
    try:
        for line in subprocess.run(["lscpu"], capture_output=True, text=True,
                                   timeout=10).stdout.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _omp_threads(n=None):
    """Set (n) or read the OpenMP thread count of this process (the oracle's
    loops run on the process's one OpenMP runtime)."""
    import ctypes
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
    except OSError:
        return None
    if n is not None:
        gomp.omp_set_num_threads(int(n))
    return int(gomp.omp_get_max_threads())


def _sample_crop(p, n=128):
    """A crop of the packed sample: the n^3 window at the box centre with the
    spheres that reach into it, walls on all sides, wetting fluid."""
    S = np.asarray(p.spheres, dtype=np.float64).copy()
    o = np.array([(p.nx - n) // 2, (p.ny - n) // 2, (p.nz - n) // 2], dtype=np.float64)
    S[:, :3] -= o
    keep = np.all((S[:, :3] + S[:, 3:4] > -2) & (S[:, :3] - S[:, 3:4] < n + 1), axis=1)
    rho0 = synth.layered_density(n, n, n, -1, p.rho_major, p.rho_minor)
    return synth.Problem(nx=n, ny=n, nz=n, bc=(synth.BC_WALLS,) * 3, spheres=S[keep],
                         rho_init=rho0, probe=None)


def _timed_oracle(prob, budget_s, batch=2):
    """Whole oracle steps on prob for about budget_s; (fluid nodes, steps, s)."""
    import oracle
    o = oracle.Oracle(prob)
    n_fluid = int((o.types() == oracle.FLUID).sum())
    o.step(1)
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        o.step(batch)
        n += batch
    return n_fluid, n, time.perf_counter() - t0


def cpu_other_configs(budget_s=4.0):
    """The oracle on the other workloads' shapes (all cores, a few seconds
    each): the 40^3 throat, the 96^3 throat, two throats of the batched
    packing; fluid-node MLUPS."""
    out = {}
    probs, _, _ = synth.packing_throats(n_throats=2, seed=3)
    for name, pr in (("throat_40", synth.c1_problem()), ("throat_96", synth.c2_problem()),
                     ("batch_throat_a", probs[0]), ("batch_throat_b", probs[1])):
        nf, n, dt = _timed_oracle(pr, budget_s)
        out[name] = {"nodes": pr.n_nodes, "fluid_nodes": nf, "steps": n, "seconds": round(dt, 2),
                     "fluid_MLUPS": round(nf * n / dt / 1e6, 3)}
    return out


def cpu_baseline(p, budget_s=10.0):
    """The FP64 oracle (test infrastructure, as it stands) on this host: a
    128^3 crop of the packed sample, timed for about budget_s of whole steps
    on all cores and again on one core.  Fluid-node MLUPS (the crop's fluid
    nodes x steps / s), the unit of the headline value."""
    import oracle
    c = _sample_crop(p)
    o = oracle.Oracle(c)
    n_fluid = int((o.types() == oracle.FLUID).sum())
    all_threads = _omp_threads()
    runs = {}
    for label, threads in (("all", all_threads), ("one", 1)):
        if threads is not None:
            _omp_threads(threads)
        o.step(1)
        n = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s:
            o.step(2)
            n += 2
        dt = time.perf_counter() - t0
        runs[label] = dict(threads=_omp_threads() if threads is not None else None,
                           steps=n, seconds=round(dt, 2),
                           fluid_MLUPS=round(n_fluid * n / dt / 1e6, 3),
                           MLUPS=round(c.n_nodes * n / dt / 1e6, 3))
    if all_threads is not None:
        _omp_threads(all_threads)
    return {"value": runs["all"]["fluid_MLUPS"], "unit": "fluid MLUPS",
            "cores": runs["all"]["threads"], "kind": "oracle",
            "sample": f"128^3 crop of the 512^3 packed sample ({n_fluid} fluid nodes), FP64, "
                      f"{runs['all']['steps']} steps on all cores and {runs['one']['steps']} on "
                      "one core, about 10 s each",
            "one_core_fluid_MLUPS": runs["one"]["fluid_MLUPS"], "runs": runs,
            "other_workloads_all_cores": cpu_other_configs(),
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count()}


def batch_leg(n_throats=BATCH_THROATS):
    """Batched drainage of n_throats packing throats in one lbm_drain_batch
    call: throats per second (all, and those with an entry pressure
    bracketed to 1 %) over the call's wall time (subdomain setup, autotuning
    and the whole graph-replayed ramp; the packing and throat geometry are
    generated on the host before it)."""
    t0 = time.perf_counter()
    probs, rins, summ = synth.packing_throats(n_throats=n_throats, seed=3)
    pcs = np.array([synth.pc_ramp(GAMMA, ri, BATCH_N_PC) for ri in rins])
    log(f"batch: {len(probs)} throats generated on the host in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    out, info = lbm.drain_batch(probs, pcs, **BATCH_CONV)
    dt = time.perf_counter() - t0
    log(f"batch: {len(probs)} throats drained in {dt:.1f} s")
    ok = sum(1 for o in out if o["invaded_at"] >= 0 and not o["failed"]
             and (o["pce_hi"] - o["pce_lo"]) <= BATCH_CONV["bisect_rel"] * o["pce_hi"])
    # the plain per-throat path on the same GPU: the first few of the same
    # throats drained one at a time (lbm_drain_throat, autotuned), same results
    t1 = time.perf_counter()
    n_single, same = BATCH_SINGLES, 0
    for k in range(n_single):
        g = lbm.Throat(probs[k])
        g.autotune(6)
        r = g.drain(pcs[k], **BATCH_CONV)
        g.close()
        same += int(np.array_equal(r["S"], out[k]["S"]) and r["total_steps"] == out[k]["total_steps"])
    dt1 = time.perf_counter() - t1
    st = np.concatenate([o["status"] for o in out])
    fl = info["fluid_updates"] / (info["wall_ms"] * 1e-3)
    gbs = fl * BYTES_PER_FLUID_NODE / 1e9
    return {"workload": f"{len(probs)} throats cut from a seeded dense packing "
                        f"({summ['n_spheres']} spheres, radii lognormal mean 1 sigma 0.2, porosity "
                        f"{summ['porosity']:.2f}), 32 lu per unit radius, box sides 48-128, "
                        f"{BATCH_N_PC}-point ramp, |dS_w| < {BATCH_CONV['tol']:g} per 100 steps "
                        f"capped at {BATCH_CONV['max_steps']} steps per point, p_c^e bracket 1 %, "
                        "one lbm_drain_batch call",
            "throats": len(probs), "box_nodes": int(sum(p.n_nodes for p in probs)),
            "wall_s": round(dt, 2), "device_ms": round(info["wall_ms"], 1),
            "throats_per_s": round(len(probs) / dt, 3),
            "invaded_within_ramp": int(sum(1 for o in out if o["invaded_at"] >= 0)),
            "pce_bracketed_1pct": ok, "bracketed_throats_per_s": round(ok / dt, 3),
            "failed": int(sum(o["failed"] for o in out)),
            "points_converged": int((st == lbm.LBM_PT_CONVERGED).sum()),
            "points_capped": int((st == lbm.LBM_PT_NOT_CONVERGED).sum()),
            "fluid_MLUPS": round(fl / 1e6, 1), "achieved_GBps": round(gbs, 1),
            "frac": round(gbs / HBM_PEAK_GBS, 4),
            "frac_note": "fluid-node updates x 304 B over the device time of the whole drain "
                         "(steps, reductions, decisions, checkpoint copies)",
            "schedule": [info["tx"], info["ty"], info["lz"]], "graph_replays": info["replays"],
            "lattice_steps": info["lattice_steps"],
            "single_throat_drains": {"throats": n_single, "throats_per_s": round(n_single / dt1, 3),
                                     "identical_to_batch": same,
                                     "batch_speedup": round((len(probs) / dt) / (n_single / dt1), 2)}}


def surrogate_leg():
    """Train the ensemble on LBM-drained throats, then answer held-out throats
    with surrogate + LBM fallback and compare with the plain batched LBM."""
    def throats(seed, n):
        # the 600-sphere packing holds about 6100 usable throats
        probs, rins, _ = synth.packing_throats(n_throats=n, seed=seed, res=SG_RES,
                                               side_range=SG_SIDES, amp=0)
        return probs, np.array([synth.pc_ramp(GAMMA, r, 16) for r in rins])

    n_train = SG_CFG["train"]
    tr, tr_pc = throats(5, n_train)
    te, te_pc = throats(6, SG_TEST)
    t0 = time.perf_counter()
    drains = []
    for c0 in range(0, len(tr), 1024):  # batches of 1024 throats, each filling the GPU
        d, _ = lbm.drain_batch(tr[c0:c0 + 1024], tr_pc[c0:c0 + 1024], **SG_CONV)
        drains += d
        log(f"surrogate: {len(drains)} of {len(tr)} training throats drained")
    t_data = time.perf_counter() - t0
    log(f"surrogate: training set drained ({len(tr)} throats, {t_data:.1f} s)")
    F, T, _ = surrogate.training_set(tr, drains)
    m = surrogate.Surrogate(members=5, seed=1)
    t0 = time.perf_counter()
    hist = m.train(F, T, **SG_FIT)
    t_train = time.perf_counter() - t0
    steps = SG_FIT["epochs"] * ((len(F) + SG_FIT["batch"] - 1) // SG_FIT["batch"])
    flops = 6.0 * surrogate.NPARAM * m.members * len(F) * SG_FIT["epochs"]
    # held-out throats: plain LBM (reference answers) and surrogate + fallback
    t0 = time.perf_counter()
    ref, _ = lbm.drain_batch(te, te_pc, **SG_CONV)
    t_lbm = time.perf_counter() - t0
    log(f"surrogate: held-out throats drained by the LBM ({t_lbm:.1f} s)")
    t0 = time.perf_counter()
    res, info = m.pce(te, te_pc, threshold=SG_THRESHOLD, **SG_CONV)
    t_sg = time.perf_counter() - t0
    pref = np.array([r["pce"] for r in ref])
    ok = np.isfinite(pref) & np.isfinite(res["pce"])
    err = np.abs(res["pce"][ok] - pref[ok]) / pref[ok]
    acc = ok & ~res["used_fallback"]
    err_acc = np.abs(res["pce"][acc] - pref[acc]) / pref[acc]
    # the network alone (no fallback) and the accept/fallback trade-off at
    # other thresholds (final answer: LBM where flagged, network elsewhere);
    # the no-network estimates are the training means of p_c^e r over r, for
    # r the MS-P radius (the network's target scale) and the opening radius
    from paper_1906_04722_amd import estimators as est
    Fte, r_msp = surrogate.describe(te, with_scale=True)
    ok = ok & np.isfinite(r_msp)
    base = np.abs(T[:, 0].mean() / r_msp[ok] - pref[ok]) / pref[ok]
    circ = lambda probs: [[(s[0], s[1], s[3]) for s in np.asarray(p.spheres)[list(p.prism_ids)]]
                          for p in probs]
    ro_tr = np.array([est.opening_radius(c) for c in circ(tr)])
    ro_te = np.array([est.opening_radius(c) for c in circ(te)])
    pce_tr = np.array([d["pce"] for d in drains])
    fin = np.isfinite(pce_tr) & np.isfinite(ro_tr)
    base_in = np.abs(np.mean(pce_tr[fin] * ro_tr[fin]) / ro_te[ok] - pref[ok]) / pref[ok]
    mean, std = m.predict(Fte)
    raw = mean[:, 0] / r_msp
    err_raw = np.abs(raw[ok] - pref[ok]) / pref[ok]
    trade = []
    for thr in (0.02, 0.05, 0.1, 0.2):
        take = (std[:, 0] <= thr * np.abs(mean[:, 0]))[ok]
        fin_e = np.where(take, err_raw, 0.0)
        trade.append({"threshold": thr, "answered_by_network": round(float(take.mean()), 4),
                      "final_err_median": round(float(np.median(fin_e)), 4),
                      "final_within_1pct": round(float((fin_e <= 0.01).mean()), 4),
                      "network_err_median_where_answered":
                          round(float(np.median(err_raw[take])), 4) if take.any() else None})
    # the calibrated no-LBM estimate of the paper's cheap methods: MS-P on the
    # throat's cross-section, scaled by its median LBM/MS-P ratio on the
    # training throats
    def msp_pc(probs):
        out = []
        for p in probs:
            S = np.asarray(p.spheres)[list(p.prism_ids)]
            out.append(GAMMA / est.msp_general_radius([(s[0], s[1], s[3]) for s in S]))
        return np.array(out)

    t0 = time.perf_counter()
    msp_te = msp_pc(te)
    t_msp = time.perf_counter() - t0
    msp_tr = msp_pc(tr)
    fin = np.isfinite(pce_tr) & np.isfinite(msp_tr)
    k_msp = float(np.median(pce_tr[fin] / msp_tr[fin]))
    ok_m = ok & np.isfinite(msp_te)
    err_msp = np.abs(k_msp * msp_te[ok_m] - pref[ok_m]) / pref[ok_m]
    # inference alone on many descriptor rows (the held-out rows repeated)
    rows = np.tile(Fte, (SG_INFER // len(Fte) + 1, 1))[:SG_INFER]
    m.predict(rows[:4096])
    t0 = time.perf_counter()
    m.predict(rows)
    t_inf = time.perf_counter() - t0
    return {"workload": f"train on {len(F)} drained throats of packing seed 5, test on "
                        f"{SG_TEST} throats of packing seed 6 ({SG_RES:g} lu per unit radius, "
                        f"sides {SG_SIDES[0]}-{SG_SIDES[1]}, 16-point ramp, cap "
                        f"{SG_CONV['max_steps']}); 5 members 80-256-256-256-17, BF16 MFMA",
            "train_data_lbm_s": round(t_data, 2), "train_s": round(t_train, 2),
            "train_steps": steps, "train_loss": [round(float(hist[0]), 4), round(float(hist[-1]), 4)],
            "train_TFLOPs": round(flops / t_train / 1e12, 3),
            "train_frac_bf16_peak": round(flops / t_train / 1e12 / BF16_PEAK_TFLOPS, 6),
            "test_throats": SG_TEST, "fallback": int(info["n_fallback"]),
            "threshold": SG_THRESHOLD,
            "pce_err_median": round(float(np.median(err)), 4),
            "pce_within_1pct": round(float((err <= 0.01).mean()), 4),
            "accepted_err_median": round(float(np.median(err_acc)), 4) if acc.any() else None,
            "baseline_msp_mean_err_median": round(float(np.median(base)), 4),
            "baseline_incircle_mean_err_median": round(float(np.median(base_in)), 4),
            "msp_lbm_ratio_train_median": round(k_msp, 4),
            "msp_calibrated_err_median": round(float(np.median(err_msp)), 4),
            "msp_calibrated_within_5pct": round(float((err_msp <= 0.05).mean()), 4),
            "msp_throats_per_s_host": round(len(te) / t_msp, 1),
            "network_err_median": round(float(np.median(err_raw)), 4),
            "network_within_5pct": round(float((err_raw <= 0.05).mean()), 4),
            "tradeoff": trade,
            "throats_per_s_lbm": round(SG_TEST / t_lbm, 3),
            "throats_per_s_surrogate_with_fallback": round(SG_TEST / t_sg, 3),
            "inference_rows_per_s": round(SG_INFER / t_inf, 1)}


def surrogate_eval_leg(path, n_test=SG_TEST):
    """The surrogate with stored weights (trained by surrogate_data on throats
    drained by the batched LBM) on held-out throats of another packing at the
    same resolution: the network alone, the network with LBM fallback, and
    the plain batched LBM on the same throats, p_c^e error against the LBM."""
    if not 1 <= n_test <= 512:
        raise SystemExit("--sg-test: 1 to 512 held-out throats (one batch)")
    from paper_1906_04722_amd import surrogate_data
    m, meta = surrogate_data.load(path)
    res, sides, conv = meta["lu_per_unit_radius"], tuple(meta["sides"]), meta["conv"]
    te, rins, _ = synth.packing_throats(n_throats=n_test, seed=6, res=res, side_range=sides,
                                        amp=0)
    te_pc = surrogate_data.ramps(rins)
    t0 = time.perf_counter()
    ref, _ = lbm.drain_batch(te, te_pc, **conv)
    t_lbm = time.perf_counter() - t0
    log(f"surrogate: {len(te)} held-out throats drained by the LBM ({t_lbm:.1f} s)")
    t0 = time.perf_counter()
    res_sg, info = m.pce(te, te_pc, threshold=SG_THRESHOLD, **conv)
    t_sg = time.perf_counter() - t0
    pref = np.array([r["pce"] for r in ref])
    Fte, r_msp = surrogate.describe(te, with_scale=True)
    mean, std = m.predict(Fte)
    raw = mean[:, 0] / r_msp
    ok = np.isfinite(pref) & np.isfinite(raw)
    err_raw = np.abs(raw[ok] - pref[ok]) / pref[ok]
    fin = np.isfinite(res_sg["pce"]) & np.isfinite(pref)
    err = np.abs(res_sg["pce"][fin] - pref[fin]) / pref[fin]
    acc = fin & ~res_sg["used_fallback"]
    err_acc = np.abs(res_sg["pce"][acc] - pref[acc]) / pref[acc]
    ok1 = int((err <= 0.01).sum())
    rows = np.tile(Fte, (SG_INFER // len(Fte) + 1, 1))[:SG_INFER]
    m.predict(rows[:4096])
    t0 = time.perf_counter()
    m.predict(rows)
    t_inf = time.perf_counter() - t0
    m.close()
    return {"workload": f"weights trained on {meta['trained_on']} of {meta['throats']} throats "
                        f"of packing seed {meta['packing_seed']} drained by the batched LBM "
                        f"({res:g} lu per unit radius, sides {sides[0]}-{sides[1]}, 16-point ramp, "
                        f"cap {conv['max_steps']}); {len(te)} held-out throats of packing seed 6",
            "recipe": meta, "test_throats": len(te), "threshold": SG_THRESHOLD,
            "network_err_median": round(float(np.median(err_raw)), 4),
            "network_within_1pct": round(float((err_raw <= 0.01).mean()), 4),
            "network_within_5pct": round(float((err_raw <= 0.05).mean()), 4),
            "fallback": int(info["n_fallback"]),
            "fallback_rate": round(info["n_fallback"] / len(te), 4),
            "accepted_err_median": round(float(np.median(err_acc)), 4) if acc.any() else None,
            "final_err_median": round(float(np.median(err)), 4),
            "final_within_1pct": ok1,
            "throats_per_s_lbm": round(len(te) / t_lbm, 3),
            "throats_per_s_surrogate_with_fallback": round(len(te) / t_sg, 3),
            "within_1pct_per_s_surrogate_with_fallback": round(ok1 / t_sg, 3),
            "inference_rows_per_s": round(SG_INFER / t_inf, 1)}


def sample_setup():
    """The 512^3 packed sample on the GPU, its launch shape autotuned, and its
    drainage ramp begun (all before the timed region)."""
    p, summ = synth.packed_sample(SAMPLE_N, SAMPLE_SPHERES, seed=4)
    g = lbm.Throat(p)
    sched = g.autotune(4)
    # the step time depends on where the two population buffers lie in
    # physical memory: keep the fastest of SAMPLE_PLACEMENTS + 1 pairs
    ms0, ms1 = g.place(SAMPLE_PLACEMENTS, 4)
    PLACEMENT.update(tries=SAMPLE_PLACEMENTS, first_pair_ms=round(ms0, 4), kept_pair_ms=round(ms1, 4))
    log(f"placement: {ms0:.3f} ms per step on the first buffer pair, {ms1:.3f} on the kept one")
    n_fluid = int((g.types() == lbm.LBM_NODE_FLUID).sum())
    r_ins = (2.0 / np.sqrt(3.0) - 1.0) * summ["mean_radius_lu"]  # three touching spheres
    pcs = synth.pc_ramp(GAMMA, r_ins, SAMPLE_NPC)
    g.drain_begin(pcs, **SAMPLE_CONV)
    return p, summ, g, sched, n_fluid, pcs


def advance(g, pcs):
    """One bench step: STEP_LATTICE lattice steps of the drainage (a ramp that
    has ended starts over from the state it reached)."""
    if g.drain_advance(STEP_LATTICE):
        g.drain_begin(pcs, **SAMPLE_CONV)


def _hybrid(x, r, L, res, state, name):
    """Hybrid drainage of a periodic packing: throat entry pressures from one
    lbm_drain_batch call, assembled by lbm_network_drain.  Facets whose
    opening lies outside their triangle of centres have no prism subdomain;
    they get the incircle estimate scaled by the median LBM/incircle ratio of
    the solved throats.  Entry pressures are compared in units of the
    interfacial tension per packing length (p_c^e * lu-per-unit / gamma).
    `res`: lattice units per packing length; `state` receives what the fully
    resolved comparison needs."""
    from synth import network as net_geo
    nw = net_geo.pore_network(x, r, L)
    probs, r_lu, scale, r_unit = net_geo.throat_problems(nw, res=res, side_range=SG_SIDES)
    idx = [i for i, p in enumerate(probs) if p is not None]
    pcs = np.array([synth.pc_ramp(GAMMA, r_lu[i], 16) for i in idx])
    t0 = time.perf_counter()
    drains, info = lbm.drain_batch([probs[i] for i in idx], pcs, **HYB_CONV)
    t_lbm = time.perf_counter() - t0
    # the same kind of throat drained one at a time (8 of them), for the
    # batching gain on subdomains too small to fill the GPU
    t0 = time.perf_counter()
    for i, pc in zip(idx[:8], pcs[:8]):
        g = lbm.Throat(probs[i])
        g.drain(pc, **HYB_CONV)
        g.close()
    t_one = (time.perf_counter() - t0) / 8
    k = len(probs)
    pce = np.full(k, np.nan)
    for i, d in zip(idx, drains):
        # not invaded up to the top of its ramp: impassable in this sample
        pce[i] = d["pce"] * scale[i] / GAMMA if np.isfinite(d["pce"]) else np.inf
    solved = np.array(idx)
    fin = solved[np.isfinite(pce[solved])]
    ratio = float(np.median(pce[fin] * r_unit[fin] / 2.0))
    rest = np.setdiff1d(np.arange(k), solved)
    pce[rest] = ratio * 2.0 / r_unit[rest]
    pressures = np.linspace(0.5 * np.min(pce), 1.05 * np.max(pce[np.isfinite(pce)]), 24)
    t0 = time.perf_counter()
    sw, inv, st = network.drain(nw["pore_vol"], nw["throats"], pce, pressures)
    t_net = time.perf_counter() - t0
    state.update(x=x, r=r, L=L, res=res, nw=nw, pressures=pressures, inv=inv, st=st,
                 wall_s=t_lbm + t_net, name=name)
    return {"workload": f"pore network of {name}: {len(nw['pore_vol'])} pores, {k} throats, "
                        f"{len(idx)} solved by the batched LBM ({res:.3g} lu per packing length, "
                        f"16-point ramp, cap {HYB_CONV['max_steps']}), the rest by the scaled "
                        "incircle estimate",
            "throat_lbm_s": round(t_lbm, 2), "throats_per_s": round(len(idx) / t_lbm, 2),
            "throats_per_s_one_at_a_time": round(1.0 / t_one, 3),
            "lbm_fluid_MLUPS": round(info["fluid_updates"] / (info["wall_ms"] * 1e3), 1),
            "schedule": [info["tx"], info["ty"], info["lz"]],
            "network_ms": round(t_net * 1e3, 3), "lbm_over_incircle_median": round(ratio, 4),
            "pressures_per_gamma": [round(float(v), 4) for v in pressures],
            "S_w": [round(float(v), 4) for v in sw],
            "trapped_pores": int((st == network.TRAPPED).sum()),
            "invaded_pores": int((st == network.INVADED).sum())}


def hybrid_leg():
    """The hybrid method on a 40-sphere dense packing (mean radius 1, porosity
    0.38) at 12 lu per unit radius."""
    x, r, L, phi, _ = synth.dense_packing(HYB_SPHERES, seed=7)
    return _hybrid(x, r, L, SG_RES, HYB_STATE,
                   f"a {HYB_SPHERES}-sphere dense packing (seed 7, porosity {1 - phi:.2f})")


THREE_CFG = {"radii": (16.0, 24.0, 32.0)}


def three_sphere_leg():
    """The paper's example throat (three equal touching spheres, prism, no
    fourth sphere): p_c^e in the paper's normalisation p* = 2 p_c R / gamma
    at several sphere radii (lattice units), beside the incircle and MS-P
    estimates, and the p*-V* drainage curve of the largest radius."""
    from paper_1906_04722_amd import estimators as est
    rows, curve = [], None
    for R in THREE_CFG["radii"]:
        p = synth.three_sphere_throat(R)
        r_in = est.incircle_radius(R)
        pcs = synth.pc_ramp(GAMMA, r_in, 20, lo=0.3, hi=1.2)
        g = lbm.Throat(p)
        g.autotune(5)
        t0 = time.perf_counter()
        out = g.drain(pcs, tol=1e-6, check_every=100, max_steps=40000, bisect_rel=0.005)
        dt = time.perf_counter() - t0
        nf = int((g.types() == lbm.LBM_NODE_FLUID).sum())
        g.close()
        rows.append({"R": R, "nodes": p.n_nodes, "pce_star": round(est.pc_star(out["pce"], R, GAMMA), 3),
                     "bracket_star": [round(est.pc_star(out["pce_lo"], R, GAMMA), 3),
                                      round(est.pc_star(out["pce_hi"], R, GAMMA), 3)],
                     "wall_s": round(dt, 2), "lattice_steps": int(out["total_steps"])})
        curve = {"R": R, "p_star": [round(est.pc_star(v, R, GAMMA), 3) for v in pcs],
                 "V_star": [round(est.v_star(s * nf, R), 4) for s in out["S"]],
                 "S_w": [round(float(s), 4) for s in out["S"]]}
    return {"workload": "three equal touching spheres in their prism, no fourth sphere, baths 6 "
                        "planes beyond the spheres; 20-point ramp from 0.3 to 1.2 x the incircle "
                        "estimate, bisection to 0.5 %",
            "incircle_star": round(4.0 / (2.0 / math.sqrt(3.0) - 1.0), 3),
            "msp_star": round(2.0 / est.msp_radius(1.0), 3),
            "radii": rows, "curve": curve}


HYB_STATE = {}
FULL_CONV = dict(tol=1e-5, check_every=200, max_steps=30000)


def _full(H):
    """The packing of a hybrid run fully resolved (Sec. 3's reference
    drainage): the slab between a non-wetting bath and a porous membrane in
    front of the wetting bath, at the resolution of the hybrid's throats,
    ramped through the hybrid's pressures.  Compared with the hybrid: the slab
    saturation, and pore by pore the invaded state (the full LBM's saturation
    within 2 lu of each pore centroid below 1/2, against the network's state)."""
    from paper_1906_04722_amd import sample_drain
    from synth import membrane
    p, info = synth.membrane_sample(H["x"], H["r"], H["L"], res=H["res"])
    pcs = H["pressures"] * GAMMA / info["scale"]
    pts = membrane.lattice_points(H["nw"]["pore_xyz"], info)
    out = sample_drain.drain_sample(p, pcs, info["slab"], info["membrane_z"], points=pts, log=log,
                                    **FULL_CONV)
    Sp = np.array(out["S_points"])
    seen = np.isfinite(Sp[0])
    agree = []
    for i in range(len(pcs)):
        hyb = (H["st"] == network.INVADED) & (H["inv"] >= 0) & (H["inv"] <= i)
        full = Sp[i] < 0.5
        agree.append(float(np.mean(hyb[seen] == full[seen])))
    return {"workload": f"{H['name']} fully resolved: {p.nx} x {p.ny} x {p.nz} lattice "
                        f"({info['scale']:.3g} lu per packing length), periodic in x and y, "
                        f"non-wetting bath, slab planes {info['slab'][0]}-{info['slab'][1]}, "
                        f"membrane of single-node holes at z = {info['membrane_z']}, wetting bath; "
                        f"{len(pcs)} pressures to steady state (|dS| < {FULL_CONV['tol']:g} per "
                        f"{FULL_CONV['check_every']} steps, cap {FULL_CONV['max_steps']})",
            "schedule": out["schedule"], "lattice_steps": out["lattice_steps"],
            "wall_s": round(out["wall_s"], 2), "hybrid_wall_s": round(H["wall_s"], 2),
            "MLUPS": round(p.n_nodes * out["lattice_steps"] / out["wall_s"] / 1e6, 1),
            "pressures_per_gamma": [round(float(v), 4) for v in H["pressures"]],
            "S_slab": [round(v, 4) for v in out["S_slab"]],
            "S_slab_sharp": [round(v, 4) for v in out["S_slab_sharp"]],
            "S_behind_membrane_min": round(min(out["S_outlet"]), 4),
            "converged": [bool(v) for v in out["converged"]],
            "pores_compared": int(seen.sum()),
            "pore_state_agreement": [round(v, 4) for v in agree],
            "pore_state_agreement_mean": round(float(np.mean(agree)), 4)}


def full_leg():
    """The hybrid_40 packing fully resolved, compared with the hybrid."""
    if not HYB_STATE:
        hybrid_leg()
    return _full(HYB_STATE)


PAPER40_STATE = {}


def paper40_leg():
    """A replica of the paper's sample sizes (Sec. 3: 40 polydisperse spheres
    of mean radius 1.26 in a 10-unit cube; log-sd 0.2 assumed, solid fraction
    0.40 follows), periodic like the network: the hybrid and the fully
    resolved drainage at 12 lu per mean radius, compared."""
    x, r, L, phi, _ = synth.dense_packing(40, mean_r=1.26, seed=7, side=10.0)
    hyb = _hybrid(x, r, L, SG_RES / 1.26, PAPER40_STATE,
                  f"a 40-sphere packing in a 10-unit cell (mean radius 1.26, seed 7, solid "
                  f"fraction {phi:.2f})")
    return {"hybrid": hyb, "full": _full(PAPER40_STATE)}


def dense_512(steps=10):
    """The same fused step on a 512^3 periodic fluid box (HBM-bound shape)."""
    n = 512
    p = synth.Problem(nx=n, ny=n, nz=n, bc=(synth.BC_PERIODIC,) * 3, z_front=n // 2,
                      G_ads=(0.0, 0.0))
    g = lbm.Throat(p)
    sched = g.autotune(3)
    ms0, ms1 = g.place(SAMPLE_PLACEMENTS, 3)
    g.step(2)
    g.sync()
    ms = g.time_steps(steps) / steps
    g.close()
    nodes = n ** 3
    gbs = nodes * BYTES_PER_FLUID_NODE / (ms * 1e-3) / 1e9
    return {"workload": "512^3 periodic fluid box", "schedule": list(sched),
            "placement": {"tries": SAMPLE_PLACEMENTS, "first_pair_ms": round(ms0, 4),
                          "kept_pair_ms": round(ms1, 4)},
            "ms_per_step": round(ms, 4),
            "MLUPS": round(nodes / ms / 1e3, 1), "achieved_GBps": round(gbs, 1),
            "peak_GBps": HBM_PEAK_GBS, "frac": round(gbs / HBM_PEAK_GBS, 4)}


def c2_leg(schedule=None):
    """The 96^3 single throat: one drainage ramp of 20 pressures with
    bisection (lbm_drain_throat), launch shape autotuned, each ramp point's
    convergence status reported."""
    p, pcs = c2_workload()
    t0 = time.perf_counter()
    out, ms, launches, n_fluid = one_drain(p, pcs, schedule)
    dt = time.perf_counter() - t0
    avg = ms * 1e-3 / max(launches, 1)
    gbs = n_fluid * BYTES_PER_FLUID_NODE / avg / 1e9
    return {"workload": "96^3 single pore throat: 4 spheres, lognormal radii (mean 32 lu, sigma "
                        "0.15) on a jittered tetrahedron, prism closure, 20-point drainage ramp, "
                        f"|dS_w| < {CONV['tol']:g} per 100 steps capped at {CONV['max_steps']} steps "
                        "per point, bisection of p_c^e to 0.5 %",
            "fluid_nodes": n_fluid, "wall_s": round(dt, 2),
            "lattice_steps": int(out["total_steps"]),
            "MLUPS": round(p.n_nodes * out["total_steps"] / dt / 1e6, 1),
            "fluid_MLUPS": round(n_fluid * out["total_steps"] / dt / 1e6, 1),
            "schedule": list(out["schedule"]), "ms_per_step": round(avg * 1e3, 5),
            "achieved_GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "traffic": read_traffic("k_step_c2_96_", out["schedule"]),
            "kernel": step_kernels(out["schedule"]),
            "pce": lbm.nan_safe(out["pce"]), "pce_bracket": [out["pce_lo"], lbm.nan_safe(out["pce_hi"])],
            "invaded_at": int(out["invaded_at"]),
            "points_converged": int((out["status"] == lbm.LBM_PT_CONVERGED).sum()),
            "points_capped": int((out["status"] == lbm.LBM_PT_NOT_CONVERGED).sum()),
            "status": [int(v) for v in out["status"]],
            "drainage_curve": {"pc": [round(float(x), 6) for x in pcs],
                               "S_w": [round(float(x), 6) for x in out["S"]]}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-c2", action="store_true")
    ap.add_argument("--batch-throats", type=int, default=BATCH_THROATS)
    ap.add_argument("--surrogate", action="store_true",
                    help="also train and evaluate the learned entry-pressure surrogate")
    ap.add_argument("--three", action="store_true",
                    help="also run the three-touching-sphere throat at several radii")
    ap.add_argument("--hybrid", action="store_true",
                    help="also run the hybrid pore-network drainage of a 40-sphere packing")
    ap.add_argument("--full", action="store_true",
                    help="also run that packing fully resolved with the membrane (minutes)")
    ap.add_argument("--paper40", action="store_true",
                    help="also run the replica of the paper's 40-sphere sample (about 2 min)")
    ap.add_argument("--sg-weights", default="",
                    help="stored surrogate weights (surrogate_data train): evaluate them on "
                         "held-out throats instead of training")
    ap.add_argument("--sg-test", type=int, default=SG_TEST,
                    help="held-out throats of the stored-weights evaluation (at most 512: "
                         "they are drained in one batch)")
    ap.add_argument("--sg-train", type=int, default=SG_CFG["train"],
                    help="throats drained to train the surrogate (default 512, at most ~6000)")
    ap.add_argument("--schedule", default="",
                    help="launch shape tx,ty,lz of the 96^3 drain (e.g. --schedule=-1,0,0 for "
                         "the node list) instead of the autotuner's pick")
    ap.add_argument("--three-radii", default=",".join(f"{v:g}" for v in THREE_CFG["radii"]),
                    help="sphere radii (lattice units) of the three-sphere throat leg")
    ap.add_argument("--full-cap", type=int, default=FULL_CONV["max_steps"],
                    help="steps per pressure of the fully resolved ramp (full_40)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {a.gpus} is not supported "
              "(throat batches shard with no communication; see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    # headline: the 512^3 packed sample; setup (voxelize, initial state,
    # autotune, ramp begun) before the timed region
    t0 = time.perf_counter()
    p, summ, g, sched, n_fluid, pcs = sample_setup()
    log(f"512^3 sample ready in {time.perf_counter() - t0:.1f} s, schedule {sched}, "
        f"{n_fluid} fluid nodes")
    for i in range(a.warmup):
        advance(g, pcs)
        log(f"warmup step {i + 1}/{a.warmup} done")
    g.sync()
    g.step_timer(1)
    t0 = time.perf_counter()
    for i in range(a.steps):
        advance(g, pcs)
        log(f"timed step {i + 1}/{a.steps} done")
    g.sync()
    dt = time.perf_counter() - t0
    k_ms, k_launches = g.step_timer(-1)
    g.step_timer(0)
    ramp = g.drain_get()
    g.close()
    lattice = k_launches   # one fused-step launch per lattice step
    fluid_mlups = n_fluid * lattice / dt / 1e6
    avg_launch_s = k_ms * 1e-3 / max(k_launches, 1)
    alg_bytes = n_fluid * BYTES_PER_FLUID_NODE
    achieved = alg_bytes / avg_launch_s / 1e9
    line = {
        "metric": "MLUPS + % HBM roofline (Shan-Chen FP32); throats/sec to p_c^e at \u22641% err",
        "value": round(fluid_mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(dt / max(a.steps, 1) * 1e3, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "storage_dtype": "f32",
        "sum_dtype": "f64",
        "data": "synthetic (seeded)",
        "config": {"workload": f"512^3 fully resolved packed sample: {summ['spheres_in_box']} "
                               f"spheres in the box (dense packing of {SAMPLE_SPHERES}, radii "
                               f"lognormal, mean {summ['mean_radius_lu']:.1f} lu), walls, baths at "
                               f"z = 0 / 511, {SAMPLE_NPC}-point drainage ramp (|dS_w| < "
                               f"{SAMPLE_CONV['tol']:g} per 100 steps, capped at "
                               f"{SAMPLE_CONV['max_steps']} per point, bisection to 1 %); one step "
                               f"= {STEP_LATTICE} lattice steps of the ramp",
                   "nx": p.nx, "ny": p.ny, "nz": p.nz, "fluid_nodes": n_fluid,
                   "lattice_steps_per_step": STEP_LATTICE},
        "value_kind": "fluid-node MLUPS (fluid nodes x lattice steps / wall time of the timed steps)",
        "box_MLUPS": round(p.n_nodes * lattice / dt / 1e6, 1),
        "lattice_steps_timed": int(lattice),
        "schedule": list(sched),
        "placement": dict(PLACEMENT),
        "ramp": {"pc": [round(float(x), 6) for x in pcs],
                 "S_w_so_far": [round(float(x), 6) for x in ramp["S"]],
                 "status_so_far": [int(x) for x in ramp["status"]],
                 "steps_so_far": int(ramp["total_steps"])},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": read_traffic("k_step_sample_512", sched),
                     "kernel": step_kernels(sched),
                     "launches": int(k_launches), "avg_launch_us": round(avg_launch_s * 1e6, 2),
                     "alg_bytes_per_launch": alg_bytes,
                     "alg_bytes_note": "fluid nodes x 304 B (38 FP32 populations read and written)"},
    }
    log(f"headline: {fluid_mlups:.0f} fluid MLUPS, step kernel {avg_launch_s * 1e3:.3f} ms, "
        f"{achieved / HBM_PEAK_GBS:.3f} of 8 TB/s")
    line["copy_probe_GBps"] = round(lbm.bw_probe(4 << 30, 10), 1)
    FULL_CONV["max_steps"] = a.full_cap
    SG_CFG["train"] = a.sg_train
    THREE_CFG["radii"] = tuple(float(v) for v in a.three_radii.split(","))
    fixed = tuple(int(v) for v in a.schedule.split(",")) if a.schedule else None
    legs = [("batch", a.no_batch, lambda: batch_leg(a.batch_throats)),
            ("c2_96", a.no_c2, lambda: c2_leg(fixed)),
            ("dense_512", a.no_dense, dense_512),
            ("surrogate", not a.surrogate or bool(a.sg_weights), surrogate_leg),
            ("surrogate_stored", not a.sg_weights, lambda: surrogate_eval_leg(a.sg_weights, a.sg_test)),
            ("three_sphere", not a.three, three_sphere_leg),
            ("hybrid_40", not (a.hybrid or a.full), hybrid_leg),
            ("full_40", not a.full, full_leg),
            ("paper_40", not a.paper40, paper40_leg),
            ("cpu_baseline", a.no_cpu, lambda: cpu_baseline(p))]
    for name, skip, fn in legs:
        if skip:
            continue
        log(f"{name} ...")
        t1 = time.perf_counter()
        line[name] = fn()
        log(f"{name} done in {time.perf_counter() - t1:.1f} s")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
