"""The C boundary from plain C, host side only: every public header compiles
as C99, and the command-line drain (csrc/lbm_drain_cli.c, linked to the
library) reports usage and problem-file errors before it touches a GPU."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLI = os.path.join(ROOT, "paper_1906_04722_amd", "lbm_drain")


@pytest.mark.parametrize("header", sorted(h for h in os.listdir(os.path.join(ROOT, "include"))
                                          if h.endswith(".h")))
def test_header_is_plain_c99(header):
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                        "-fsyntax-only", "-x", "c", os.path.join(ROOT, "include", header)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def _run(*args):
    return subprocess.run([CLI, *args], capture_output=True, text=True, timeout=60)


def test_cli_prints_usage():
    r = _run()
    assert r.returncode == 1 and "usage: lbm_drain" in r.stderr
    assert _run("p.txt", "--chunk", "0").returncode == 1


def test_cli_rejects_malformed_problem_files(tmp_path):
    good = ["size 8 8 8", "pc 0.01 0.02", "conv 1e-6 100 1000 0.01"]
    cases = {"missing_conv": good[:2], "missing_pc": [good[0], good[2]],
             "unknown_key": good + ["colour blue"], "short_size": ["size 8 8"] + good[1:],
             "bad_number": ["size 8 8 8", "pc 0.01", "conv x 100 1000 0.01"]}
    for name, lines in cases.items():
        path = tmp_path / f"{name}.txt"
        path.write_text("\n".join(lines) + "\n")
        r = _run(str(path))
        assert r.returncode == 1, (name, r.stderr)
        assert "lbm_drain:" in r.stderr, name
    r = _run(str(tmp_path / "absent.txt"))
    assert r.returncode == 1 and "cannot open" in r.stderr
