"""Problem files of the command-line drain (paper_1906_04722_amd/lbm_drain):
a synth.Problem and its ramp written in the tool's keyword format, and the
tool's output parsed back."""
import numpy as np

CLI_REL = "paper_1906_04722_amd/lbm_drain"


def write_problem(path, p, pcs, conv):
    if p.rho_init is not None:
        raise ValueError("the problem file states no initial-density array")
    lines = [f"size {p.nx} {p.ny} {p.nz}", "bc {} {} {}".format(*p.bc),
             "tau {!r} {!r}".format(*map(float, p.tau)), f"G {float(p.G)!r}",
             "G_ads {!r} {!r}".format(*map(float, p.G_ads)),
             f"rho {float(p.rho_major)!r} {float(p.rho_minor)!r}",
             f"baths {float(p.rho_in_nw)!r} {float(p.rho_out_w)!r}", f"z_front {p.z_front}"]
    if p.probe is not None:
        lines.append("probe {} {} {}".format(*p.probe))
    if p.prism_ids is not None:
        lines.append("prism {} {} {}".format(*p.prism_ids))
    for s in np.asarray(p.spheres, dtype=np.float64).reshape(-1, 4):
        lines.append("sphere " + " ".join(repr(float(v)) for v in s))
    lines.append("pc " + " ".join(repr(float(v)) for v in pcs))
    lines.append(f"conv {float(conv['tol'])!r} {int(conv['check_every'])} "
                 f"{int(conv['max_steps'])} {float(conv['bisect_rel'])!r}")
    with open(path, "w") as f:
        f.write("# written by tests/cli_problem.py\n" + "\n".join(lines) + "\n")


def parse_output(text):
    out = {}
    for line in text.strip().splitlines():
        k, *v = line.split()
        if k in ("S", "mass"):
            out[k] = np.array([float(x) for x in v])
        elif k in ("steps", "status"):
            out[k] = np.array([int(x) for x in v])
        elif k in ("pce", "pce_lo", "pce_hi", "S_w"):
            out[k] = float(v[0])
        else:
            out[k] = int(v[0])
    return out
