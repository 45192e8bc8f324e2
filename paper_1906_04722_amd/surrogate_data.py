"""Training data, training and stored weights of the entry-pressure surrogate.

The surrogate maps a throat's geometry to its entry pressure p_c^e and its
16-point drainage curve (the network and its kernels live in the HIP
library, lbm_surrogate.h).  Its training targets are produced by the batched
lattice Boltzmann drainage itself (lbm_drain_batch, Sec. 2.2.2's ramp with
bisection): throats cut from a seeded dense packing are drained in batches
of `chunk` throats, described, and the ensemble is trained on the GPU.

Stored weights are safetensors files (no pickled objects): one float32
tensor of 156,689 parameters per member, the FP64 feature and target
statistics, and the recipe as metadata.

    python -m paper_1906_04722_amd.surrogate_data train --throats 4096 \\
        --seed 5 --res 32 --out weights.safetensors

A larger set is drained in parts (each a slice of one packing's throat
list, e.g. in separate sessions) and trained on their union:

    python -m paper_1906_04722_amd.surrogate_data drain --throats 20000 \\
        --spheres 2000 --first 0 --count 5000 --out part0.npz
    python -m paper_1906_04722_amd.surrogate_data fit --data part*.npz \\
        --out weights.safetensors
"""
import argparse
import json
import sys
import time

import numpy as np

from . import lbm
from . import surrogate

# a throat's ramp: 16 pressures from 0.1 to 1.5 x the incircle estimate
# 2 gamma / r_ins, gamma the model's interfacial tension (0.190 lattice units)
GAMMA = 0.190
N_PC = 16


def ramps(r_ins):
    return np.array([np.linspace(0.1, 1.5, N_PC) * 2.0 * GAMMA / r for r in r_ins])


def drain_throats(n, seed, res, side_range, conv, chunk=512, log=None, n_spheres=600,
                  first=0, count=None):
    """Throats [first, first + count) of the first n throats of the seed's
    packing of n_spheres spheres (synth.packing_throats), drained by
    lbm_drain_batch in chunks; returns (problems, ramps, drain results)."""
    import synth
    probs, rins, _ = synth.packing_throats(n_throats=n, n_spheres=n_spheres, seed=seed, res=res,
                                           side_range=side_range, amp=0)
    stop = len(probs) if count is None else min(len(probs), first + count)
    probs, rins = probs[first:stop], rins[first:stop]
    pcs = ramps(rins)
    drains = []
    for c0 in range(0, len(probs), chunk):
        d, _ = lbm.drain_batch(probs[c0:c0 + chunk], pcs[c0:c0 + chunk], **conv)
        drains += d
        if log:
            log(f"{len(drains)} of {len(probs)} throats drained")
    return probs, pcs, drains


def save(model, path, meta):
    from safetensors.numpy import save_file
    xmu, xsd, tmu, tsd = model.get_stats()
    t = {f"member{z}": model.get_params(z).astype(np.float32) for z in range(model.members)}
    t.update(xmu=np.asarray(xmu, np.float64), xsd=np.asarray(xsd, np.float64),
             tmu=np.asarray(tmu, np.float64), tsd=np.asarray(tsd, np.float64))
    save_file(t, path, metadata={"recipe": json.dumps(meta)})


def load(path, seed=0):
    """(Surrogate with the stored weights and statistics, recipe dict)."""
    from safetensors import safe_open
    from safetensors.numpy import load_file
    t = load_file(path)
    with safe_open(path, framework="numpy") as f:
        meta = json.loads(f.metadata().get("recipe", "{}"))
    members = sum(1 for k in t if k.startswith("member"))
    m = surrogate.Surrogate(members=members, seed=seed)
    for z in range(members):
        m.set_params(z, t[f"member{z}"])
    m.set_stats(t["xmu"], t["xsd"], t["tmu"], t["tsd"])
    return m, meta


def cmd_drain(a, log):
    """One part of a training set: drained throats' descriptors and targets
    to an .npz (plain arrays and the recipe as JSON text)."""
    if not a.out.endswith(".npz"):
        raise SystemExit("drain --out: the part is an .npz file")
    sides = tuple(int(v) for v in a.sides.split(","))
    conv = dict(tol=1e-6, check_every=100, max_steps=a.cap, bisect_rel=0.01)
    t0 = time.perf_counter()
    probs, pcs, drains = drain_throats(a.throats, a.seed, a.res, sides, conv, a.chunk, log,
                                       a.spheres, a.first, a.count)
    t_lbm = time.perf_counter() - t0
    F, T, ok = surrogate.training_set(probs, drains)
    meta = dict(throats_in_list=a.throats, packing_spheres=a.spheres, packing_seed=a.seed,
                first=a.first, drained=len(probs), usable=int(ok.sum()),
                lu_per_unit_radius=a.res, sides=list(sides), ramp_points=N_PC, conv=conv,
                lbm_seconds=round(t_lbm, 1))
    np.savez(a.out, F=F, T=T, recipe=np.array(json.dumps(meta)))
    log(f"{len(F)} of {len(probs)} throats usable ({t_lbm:.1f} s of batched LBM) -> {a.out}")
    print(json.dumps(meta), flush=True)


def cmd_fit(a, log):
    """Train the ensemble on the union of drained parts and store it."""
    parts = [np.load(f, allow_pickle=False) for f in a.data]
    F = np.concatenate([q["F"] for q in parts])
    T = np.concatenate([q["T"] for q in parts])
    recipes = [json.loads(str(q["recipe"])) for q in parts]
    m = surrogate.Surrogate(members=a.members, seed=1)
    t0 = time.perf_counter()
    hist = m.train(F, T, epochs=a.epochs, batch=a.batch, lr=a.lr, seed=2)
    t_fit = time.perf_counter() - t0
    r0 = recipes[0]
    meta = dict(throats=int(sum(r["drained"] for r in recipes)), trained_on=int(len(F)),
                packing_seed=r0["packing_seed"], packing_spheres=r0["packing_spheres"],
                lu_per_unit_radius=r0["lu_per_unit_radius"], sides=r0["sides"],
                ramp_points=N_PC, conv=r0["conv"], epochs=a.epochs, batch=a.batch, lr=a.lr,
                members=a.members,
                lbm_seconds=round(float(sum(r["lbm_seconds"] for r in recipes)), 1),
                train_seconds=round(t_fit, 1), parts=[[r["first"], r["drained"]] for r in recipes],
                loss_first_last=[float(hist[0]), float(hist[-1])])
    save(m, a.out, meta)
    log(f"trained on {len(F)} rows from {len(parts)} parts -> {a.out}")
    print(json.dumps(meta), flush=True)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    dr = sub.add_parser("drain", help="drain a slice of a packing's throats to an .npz part")
    dr.add_argument("--throats", type=int, required=True, help="length of the throat list")
    dr.add_argument("--spheres", type=int, default=600, help="spheres of the packing")
    dr.add_argument("--first", type=int, default=0)
    dr.add_argument("--count", type=int, default=None)
    dr.add_argument("--seed", type=int, default=5)
    dr.add_argument("--res", type=float, default=32.0)
    dr.add_argument("--sides", default="48,128")
    dr.add_argument("--cap", type=int, default=600)
    dr.add_argument("--chunk", type=int, default=512)
    dr.add_argument("--out", required=True)
    ft = sub.add_parser("fit", help="train on drained .npz parts and store the weights")
    ft.add_argument("--data", nargs="+", required=True)
    ft.add_argument("--epochs", type=int, default=200)
    ft.add_argument("--batch", type=int, default=64)
    ft.add_argument("--lr", type=float, default=1e-3)
    ft.add_argument("--members", type=int, default=5)
    ft.add_argument("--out", required=True)
    tr = sub.add_parser("train")
    tr.add_argument("--throats", type=int, default=4096)
    tr.add_argument("--seed", type=int, default=5)
    tr.add_argument("--res", type=float, default=32.0)
    tr.add_argument("--sides", default="48,128")
    tr.add_argument("--cap", type=int, default=600)
    tr.add_argument("--epochs", type=int, default=200)
    tr.add_argument("--batch", type=int, default=64)
    tr.add_argument("--lr", type=float, default=1e-3)
    tr.add_argument("--members", type=int, default=5)
    tr.add_argument("--chunk", type=int, default=512)
    tr.add_argument("--out", required=True)
    a = ap.parse_args()

    def log(msg):
        print(f"surrogate_data: {msg}", file=sys.stderr, flush=True)

    if a.cmd == "drain":
        return cmd_drain(a, log)
    if a.cmd == "fit":
        return cmd_fit(a, log)

    sides = tuple(int(v) for v in a.sides.split(","))
    conv = dict(tol=1e-6, check_every=100, max_steps=a.cap, bisect_rel=0.01)
    t0 = time.perf_counter()
    probs, pcs, drains = drain_throats(a.throats, a.seed, a.res, sides, conv, a.chunk, log)
    t_lbm = time.perf_counter() - t0
    F, T, ok = surrogate.training_set(probs, drains)
    log(f"{len(F)} of {len(probs)} throats usable for training ({t_lbm:.1f} s of batched LBM)")
    m = surrogate.Surrogate(members=a.members, seed=1)
    t0 = time.perf_counter()
    hist = m.train(F, T, epochs=a.epochs, batch=a.batch, lr=a.lr, seed=2)
    t_fit = time.perf_counter() - t0
    meta = dict(throats=len(probs), trained_on=int(len(F)), packing_seed=a.seed,
                lu_per_unit_radius=a.res, sides=list(sides), ramp_points=N_PC,
                conv=conv, epochs=a.epochs, batch=a.batch, lr=a.lr, members=a.members,
                lbm_seconds=round(t_lbm, 1), train_seconds=round(t_fit, 1),
                loss_first_last=[float(hist[0]), float(hist[-1])])
    save(m, a.out, meta)
    print(json.dumps(meta), flush=True)


if __name__ == "__main__":
    main()
