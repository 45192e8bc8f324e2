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
