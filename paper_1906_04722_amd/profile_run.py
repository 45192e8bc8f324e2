"""Profiling driver for rocprofv3 runs of the fused step, and the summary
writer for the counter output.

  python3 -m paper_1906_04722_amd.profile_run run --steps 200 [--autotune 20]
      builds the 96^3 throat (or an N^3 periodic box with --workload N, or the
      512^3 packed sample with --workload sample512; --workload batchN drains N
      packing throats in one batch instead, --steps capping each ramp point), runs
      a 1 GiB copy twice (the counter calibration: 2 GiB moved per launch,
      known exactly) and `steps` fused steps, optionally after autotuning the
      launch shape as the benchmark does.
  python3 -m paper_1906_04722_amd.profile_run trace --trace T.csv --kernel K --last N
      --out profiles/NAME.txt: per-kernel statistics of a kernel trace and the
      average of kernel K's last N dispatches (a benchmark's timed region).
  python3 -m paper_1906_04722_amd.profile_run sq --counters C.csv --stats S.csv
      --kernel K --workload W --schedule S --out profiles/NAME.txt: one row of
      SQ counters (waves, lifetimes, instructions per wave) of kernel K.
  python3 -m paper_1906_04722_amd.profile_run summarize --stats S.csv
      --fetch F.csv --write W.csv --out profiles/NAME.txt --command "..."
      writes the per-step averages of the step kernels (the fused k_step, or
      with --kernels k_dens_list,k_step_list the two passes of the node-list
      step, summed), the copy-kernel calibration factors and the calibrated
      HBM traffic per step.
"""
import argparse
import csv
import hashlib
import os
import re
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
COPY_BYTES = 1 << 30
KERNEL_SRC = os.path.join(PKG, "csrc", "sc_kernels.hip")

_TOKENS = re.compile(r'//[^\n]*|/\*.*?\*/|"(?:\\.|[^"\\])*"|[^\s"/]+|/', re.S)


def kernel_sha(path=KERNEL_SRC):
    """Hash of the kernel source's code: comments dropped, tokens separated by
    single spaces, so that a counter summary stays valid across edits of the
    comments and layout only."""
    code = [t for t in _TOKENS.findall(open(path).read()) if not t.startswith(("//", "/*"))]
    return hashlib.sha256(" ".join(code).encode()).hexdigest()[:16]


def cmd_run(a):
    sys.path.insert(0, ROOT)
    import synth
    from paper_1906_04722_amd import lbm
    lbm.bw_probe(COPY_BYTES, 2)
    if a.workload.startswith("batch"):
        # batched drainage of N packing throats (32 lu per unit radius, sides
        # 48-128), a 16-point ramp capped at --steps steps per point; chunks
        # launched kernel by kernel (--no-graph) for tracers that do not
        # follow graph launches
        import numpy as np
        n = int(a.workload[len("batch"):] or 64)
        probs, rins, _ = synth.packing_throats(n_throats=n, seed=3)
        pcs = np.array([synth.pc_ramp(synth.GAMMA_LAPLACE, r, 16) for r in rins])
        if a.no_graph:
            os.environ["LBM_BATCH_NO_GRAPH"] = "1"
        out, info = lbm.drain_batch(probs, pcs, tol=1e-6, check_every=100, max_steps=a.steps,
                                    bisect_rel=0.01)
        print(f"profile_run: {a.workload}, cap {a.steps} per point, schedule "
              f"{[info['tx'], info['ty'], info['lz']]}, lattice steps {info['lattice_steps']}, "
              f"fluid updates {info['fluid_updates']}, {info['n_tiles']} tiles, graph "
              f"{'off' if a.no_graph else 'on'}", flush=True)
        return
    if a.workload == "c2":
        p = synth.c2_problem()
    elif a.workload == "sample512":
        p, _ = synth.packed_sample(512, 1000, seed=4)
    else:
        n = int(a.workload)
        p = synth.Problem(nx=n, ny=n, nz=n, bc=(synth.BC_PERIODIC,) * 3, z_front=n // 2,
                          G_ads=(0.0, 0.0))
    g = lbm.Throat(p)
    if a.autotune:
        g.autotune(a.autotune)
    if a.schedule:
        g.set_schedule(*[int(v) for v in a.schedule.split(",")])
    g.step(a.steps)
    g.sync()
    print(f"profile_run: {a.workload}, {a.steps} steps, schedule {g.schedule()}", flush=True)


def _per_kernel(path, counter=None):
    out = {}
    for r in csv.DictReader(open(path)):
        if counter and r.get("Counter_Name") != counter:
            continue
        name = r["Kernel_Name"]
        out.setdefault(name, []).append(float(r["Counter_Value"]))
    return out


def cmd_summarize(a):
    stats = list(csv.DictReader(open(a.stats)))
    fetch = _per_kernel(a.fetch, "FETCH_SIZE")
    write = _per_kernel(a.write, "WRITE_SIZE")

    def find(d, key):
        for k, v in d.items():
            if key in k:
                return v
        raise KeyError(key)

    cf = find(fetch, "k_copy")
    cw = find(write, "k_copy")
    # counters are KiB per dispatch; the copy moves COPY_BYTES each way
    f_scale = COPY_BYTES / (sum(cf) / len(cf) * 1024.0)
    w_scale = COPY_BYTES / (sum(cw) / len(cw) * 1024.0)
    fb = wb = 0.0
    counted = []
    for key in [k for k in a.kernels.split(";" if ";" in a.kernels else ",") if k]:
        sf = find(fetch, key)
        sw = find(write, key)
        fb += sum(sf) / len(sf) * 1024.0 * f_scale
        wb += sum(sw) / len(sw) * 1024.0 * w_scale
        counted.append(f"{key} x{len(sf)}")
    lines = [f"# {a.title}", f"# command: {a.command}",
             f"kernel_sha: {kernel_sha()}"]
    if a.schedule:
        lines.append(f"schedule: {a.schedule}")
    lines += [f"copy_fetch_scale: {f_scale:.4f}", f"copy_write_scale: {w_scale:.4f}",
             f"step_launches_counted: {', '.join(counted)}",
             f"fetch_bytes_per_launch: {fb:.0f}", f"write_bytes_per_launch: {wb:.0f}",
             f"traffic_bytes_per_launch: {fb + wb:.0f}"]
    if a.alg_bytes:
        lines.append(f"algorithmic_bytes_per_launch: {a.alg_bytes}")
        lines.append(f"traffic_over_algorithmic: {(fb + wb) / float(a.alg_bytes):.3f}")
    lines.append("# kernel stats (rocprofv3 --kernel-trace --stats):")
    lines.append("# name | calls | avg_ns | min_ns | max_ns | percent")
    for r in stats:
        lines.append(f"# {r['Name'][:70]} | {r['Calls']} | {float(r['AverageNs']):.0f} | "
                     f"{r['MinNs']} | {r['MaxNs']} | {float(r['Percentage']):.2f}")
    open(a.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


SQ_COUNTERS = ("SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAIT_INST_ANY",
               "SQ_INSTS_VALU", "SQ_INSTS_VMEM_RD")


def cmd_sq(a):
    """One row of the SQ-counter table: per-dispatch means of the step
    kernel's wave count, lifetime (SQ_WAVE_CYCLES per wave, counted in units of
    4 cycles at 2.4 GHz), vector ALU and vector-memory-read instructions per
    wave, and the share of SIMD time that issues vector ALU work (one wave64
    instruction taken as 4 cycles, 1024 SIMDs, the step time of a separate
    kernel-trace run)."""
    vals = {c: _per_kernel(a.counters, c) for c in SQ_COUNTERS}
    keys = [k for k in vals["SQ_WAVES"] if a.kernel in k]
    if len(keys) != 1:
        raise SystemExit(f"kernel key {a.kernel!r} matches {keys}")
    k = keys[0]
    mean = {c: sum(vals[c][k]) / len(vals[c][k]) for c in SQ_COUNTERS}
    step_ns = None
    for r in csv.DictReader(open(a.stats)):
        if a.kernel in r["Name"]:
            step_ns = float(r["AverageNs"])
    if step_ns is None:
        raise SystemExit(f"kernel {a.kernel!r} not in {a.stats}")
    waves = mean["SQ_WAVES"]
    life_us = mean["SQ_WAVE_CYCLES"] / waves * 4 / 2.4e3
    valu_share = mean["SQ_INSTS_VALU"] * 4 / (1024 * step_ns * 2.4)
    new = not os.path.exists(a.out)
    with open(a.out, "a") as f:
        if new:
            f.write(f"# {a.title}\n# command: {a.command}\n")
            f.write("# lifetime_us reads SQ_WAVE_CYCLES / SQ_WAVES in units of 4 cycles at 2.4 GHz; "
                    "simd_valu_share is SQ_INSTS_VALU x 4 cycles / (1024 SIMDs x step time), the "
                    "share of SIMD time spent issuing vector ALU instructions (one wave64 "
                    "instruction taken as 4 cycles)\n")
            f.write(f"kernel_sha: {kernel_sha()}\n")
            f.write("# workload | schedule | kernel | waves | lifetime_us | valu_per_wave | "
                    "vmem_rd_per_wave | wait_inst_any_per_wave_cycle | step_us | simd_valu_share\n")
        f.write(f"{a.workload} | {a.schedule} | {k[:40]} | {waves:.0f} | {life_us:.1f} | "
                f"{mean['SQ_INSTS_VALU'] / waves:.0f} | {mean['SQ_INSTS_VMEM_RD'] / waves:.1f} | "
                f"{mean['SQ_WAIT_INST_ANY'] / mean['SQ_WAVE_CYCLES']:.2f} | {step_ns / 1e3:.1f} | "
                f"{valu_share:.2f}\n")
    print(open(a.out).read())


def cmd_trace(a):
    """Summary of a kernel trace: per-kernel statistics, and for one kernel
    the average of its last `last` dispatches (the timed region of a run
    whose earlier dispatches include autotuner trials)."""
    rows = list(csv.DictReader(open(a.trace)))
    per = {}
    for r in rows:
        d = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        per.setdefault(r["Kernel_Name"], []).append((int(r["Start_Timestamp"]), d, r))
    lines = [f"# {a.title}", f"# command: {a.command}", f"kernel_sha: {kernel_sha()}"]
    key = [k for k in per if a.kernel in k]
    if len(key) != 1:
        raise SystemExit(f"kernel key {a.kernel!r} matches {key}")
    ev = sorted(per[key[0]])[-a.last:]
    durs = [d for _, d, _ in ev]
    r0 = ev[-1][2]
    lines += [f"timed_kernel: {key[0]}",
              f"timed_dispatches: {len(durs)} (the last {a.last})",
              f"timed_avg_ns: {sum(durs) / len(durs):.0f}",
              f"timed_min_ns: {min(durs)}", f"timed_max_ns: {max(durs)}",
              f"grid: {r0['Grid_Size_X']} x {r0['Grid_Size_Y']}, workgroup {r0['Workgroup_Size_X']}, "
              f"VGPRs {r0['VGPR_Count']}, SGPRs {r0['SGPR_Count']}, LDS {r0['LDS_Block_Size']} B, "
              f"scratch {r0['Scratch_Size']} B"]
    lines.append("# all kernels of the run: name | calls | avg_ns | min_ns | max_ns")
    for name, v in sorted(per.items(), key=lambda kv: -sum(d for _, d, _ in kv[1])):
        ds = [d for _, d, _ in v]
        lines.append(f"# {name[:70]} | {len(ds)} | {sum(ds) / len(ds):.0f} | {min(ds)} | {max(ds)}")
    open(a.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--steps", type=int, default=200)
    r.add_argument("--workload", default="c2")
    r.add_argument("--autotune", type=int, default=0,
                   help="trial steps of the launch-shape autotuner before the run (0: default shape)")
    r.add_argument("--schedule", default="",
                   help="launch shape tx,ty,lz to run with (e.g. the one the benchmark's autotuner picks)")
    r.add_argument("--no-graph", action="store_true",
                   help="batch workloads: launch each chunk's kernels instead of a graph replay")
    s = sub.add_parser("summarize")
    s.add_argument("--stats", required=True)
    s.add_argument("--fetch", required=True)
    s.add_argument("--write", required=True)
    s.add_argument("--out", required=True)
    s.add_argument("--title", default="fused step")
    s.add_argument("--command", default="")
    s.add_argument("--alg-bytes", type=int, default=0)
    s.add_argument("--kernels", default="k_step",
                   help="kernel-name keys (separated by commas, or by semicolons when a key "
                        "holds a comma) whose per-dispatch counters make one step")
    s.add_argument("--schedule", default="", help="launch shape the run used (recorded)")
    q = sub.add_parser("sq")
    q.add_argument("--counters", required=True, help="counter_collection.csv of a --pmc run of SQ_*")
    q.add_argument("--stats", required=True, help="kernel_stats.csv of a kernel-trace run")
    q.add_argument("--kernel", required=True)
    q.add_argument("--workload", required=True)
    q.add_argument("--schedule", required=True)
    q.add_argument("--out", required=True)
    q.add_argument("--title", default="SQ counters of the fused step")
    q.add_argument("--command", default="")
    t = sub.add_parser("trace")
    t.add_argument("--trace", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--kernel", required=True, help="key of the timed kernel's name")
    t.add_argument("--last", type=int, required=True)
    t.add_argument("--title", default="kernel trace")
    t.add_argument("--command", default="")
    a = ap.parse_args()
    {"run": cmd_run, "summarize": cmd_summarize, "trace": cmd_trace, "sq": cmd_sq}[a.cmd](a)


if __name__ == "__main__":
    main()
