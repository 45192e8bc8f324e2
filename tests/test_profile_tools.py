"""Host logic of the measurement: the kernel hash that keys the committed
counter summaries, and the bench's choice of summary by hash and schedule."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1906_04722_amd.profile_run import kernel_sha  # noqa: E402

CODE = '''#include "a.h"
// a comment
int f(int a, int b) { return a / b; }  /* trailing
   block */
const char *s = "x // not a comment";
'''


def _write(tmp_path, name, text):
    p = tmp_path / name
    p.write_text(text)
    return str(p)


def test_kernel_sha_ignores_comments_and_layout(tmp_path):
    a = kernel_sha(_write(tmp_path, "a.hip", CODE))
    relaid = CODE.replace("// a comment", "// another comment\n\n").replace(
        "{ return a / b; }", "{\n  return a/b;\n}")
    assert kernel_sha(_write(tmp_path, "b.hip", relaid)) == a


def test_kernel_sha_follows_code(tmp_path):
    a = kernel_sha(_write(tmp_path, "a.hip", CODE))
    assert kernel_sha(_write(tmp_path, "b.hip", CODE.replace("a / b", "a * b"))) != a
    # text inside a string literal is code, not a comment
    assert kernel_sha(_write(tmp_path, "c.hip", CODE.replace("x // not", "x // nor"))) != a


def test_traffic_is_taken_by_hash_and_schedule(tmp_path, monkeypatch):
    import bench
    src = _write(tmp_path, "k.hip", CODE)
    monkeypatch.setattr(bench, "KERNEL_SRC", src)
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    sha = kernel_sha(src)
    (tmp_path / "k_step_c2_96_list_traffic.txt").write_text(
        f"# node list\nkernel_sha: {sha}\nschedule: -1,0,0\ntraffic_bytes_per_launch: 123\n")
    (tmp_path / "k_step_c2_96_old_traffic.txt").write_text(
        "# another source\nkernel_sha: 0000000000000000\nschedule: 16,8,1\n"
        "traffic_bytes_per_launch: 456\n")
    assert bench.read_traffic("k_step_c2_96_", (-1, 0, 0)) == 123.0
    assert bench.read_traffic("k_step_c2_96_", (16, 8, 1)) is None   # taken on other code
    assert bench.read_traffic("k_step_c2_96_", (32, 4, 1)) is None   # no summary for this shape
    assert bench.read_traffic("k_step_sample_512", (-1, 0, 0)) is None   # another workload


def test_sq_row_from_counter_and_trace_csv(tmp_path):
    """The SQ summary row: per-dispatch means over the step kernel's
    dispatches only, lifetimes in units of 4 cycles at 2.4 GHz, and the VALU
    share of 1024 SIMDs over the traced step time."""
    import argparse
    from paper_1906_04722_amd import profile_run as pr
    rows = ["Kernel_Name,Counter_Name,Counter_Value"]
    vals = {"SQ_WAVES": (100, 300), "SQ_WAVE_CYCLES": (1.2e6, 3.6e6), "SQ_BUSY_CYCLES": (1, 1),
            "SQ_WAIT_INST_ANY": (0.6e6, 1.8e6), "SQ_INSTS_VALU": (2e5, 4e5),
            "SQ_INSTS_VMEM_RD": (1000, 5000)}
    for c, (v1, v2) in vals.items():
        rows += [f"k_step<32 8>,{c},{v1}", f"k_step<32 8>,{c},{v2}", f"k_copy,{c},7"]
    counters = _write(tmp_path, "c.csv", "\n".join(rows) + "\n")
    stats = _write(tmp_path, "s.csv", "Name,AverageNs\nk_step<32 8>,1000000\nk_copy,5\n")
    out = str(tmp_path / "sq.txt")
    pr.cmd_sq(argparse.Namespace(counters=counters, stats=stats, kernel="k_step", workload="w",
                                 schedule="32,8,16", out=out, title="t", command="c"))
    row = open(out).read().strip().splitlines()[-1].split(" | ")
    assert row[0] == "w" and row[3] == "200"                       # mean waves per dispatch
    assert abs(float(row[4]) - 2.4e6 / 200 * 4 / 2400) < 0.1        # lifetime, us
    assert row[5] == "1500" and row[6] == "15.0"                   # VALU and VMEM per wave
    assert row[7] == "0.50" and row[8] == "1000.0"
    assert abs(float(row[9]) - 3e5 * 4 / (1024 * 1e6 * 2.4)) < 0.006


def test_summarize_scales_counters_by_the_copy_calibration(tmp_path):
    """Traffic per step: each counter's per-dispatch mean (KiB) scaled by the
    factor that maps the copy kernel's reading onto the bytes it moves."""
    import argparse
    from paper_1906_04722_amd import profile_run as pr
    gib = pr.COPY_BYTES / 1024.0                      # KiB the copy moves each way
    rows = ["Kernel_Name,Counter_Name,Counter_Value"]
    rows += [f"k_copy,FETCH_SIZE,{gib / 2}", f"k_copy,FETCH_SIZE,{gib / 2}"]   # reads half
    rows += [f"k_step<32 8>,FETCH_SIZE,100", f"k_step<32 8>,FETCH_SIZE,300"]
    fetch = _write(tmp_path, "f.csv", "\n".join(rows) + "\n")
    rows = ["Kernel_Name,Counter_Name,Counter_Value", f"k_copy,WRITE_SIZE,{gib}",
            "k_step<32 8>,WRITE_SIZE,50", "k_step<32 8>,WRITE_SIZE,50"]
    write = _write(tmp_path, "w.csv", "\n".join(rows) + "\n")
    stats = _write(tmp_path, "s.csv", "Name,Calls,AverageNs,MinNs,MaxNs,Percentage\n"
                                      "k_step<32 8>,2,1000,900,1100,90\n")
    out = str(tmp_path / "t.txt")
    pr.cmd_summarize(argparse.Namespace(stats=stats, fetch=fetch, write=write, out=out,
                                        title="t", command="c", alg_bytes=200 * 1024,
                                        kernels="k_step", schedule="32,8,16"))
    kv = dict(l.split(": ", 1) for l in open(out).read().splitlines() if ": " in l
              and not l.startswith("#"))
    assert float(kv["copy_fetch_scale"]) == 2.0 and float(kv["copy_write_scale"]) == 1.0
    assert float(kv["fetch_bytes_per_launch"]) == 2.0 * 200 * 1024    # mean 200 KiB, x2
    assert float(kv["write_bytes_per_launch"]) == 50 * 1024
    assert float(kv["traffic_over_algorithmic"]) == 2.25


def test_trace_averages_the_last_dispatches_of_one_kernel(tmp_path):
    import argparse
    from paper_1906_04722_amd import profile_run as pr
    cols = ("Kernel_Name,Start_Timestamp,End_Timestamp,Grid_Size_X,Grid_Size_Y,Workgroup_Size_X,"
            "VGPR_Count,SGPR_Count,LDS_Block_Size,Scratch_Size")
    rows = [cols]
    # three autotuner-like early dispatches of 50 ns, then four of 10 ns
    t = 0
    for d in (50, 50, 50, 10, 10, 10, 10):
        rows.append(f"k_step<32 8>,{t},{t + d},256,1,256,160,100,51200,0")
        t += 100
    rows.append(f"k_copy,{t},{t + 7},1,1,256,8,16,0,0")
    trace = _write(tmp_path, "t.csv", "\n".join(rows) + "\n")
    out = str(tmp_path / "o.txt")
    pr.cmd_trace(argparse.Namespace(trace=trace, out=out, kernel="k_step", last=4, title="t",
                                    command="c"))
    text = open(out).read()
    assert "timed_avg_ns: 10\n" in text and "timed_dispatches: 4 (the last 4)" in text


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
