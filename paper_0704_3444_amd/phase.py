"""Phase-equilibrium experiments of Sec. IV on the GPU.

The paper measures binodals by running many short periodic D1Q3 lines (one
per interaction strength, relaxation time or starting composition) until the
profile stops changing and reading the compositions of the two coexisting
phases off it.  Here a set of such runs is stepped by one line group
(lb_lines_* of the C ABI: one wavefront per run, all steps of a call in
registers), and the coexisting compositions are read from each final
profile.  Nothing here computes a theoretical binodal."""
from __future__ import annotations

from typing import Optional

import numpy as np

from .lb import Lines, Simulation


def run_lines(runs, steps: int, *, storage: str = "f64", marks=None) -> list:
    """Step every run of `runs` (a list of (cfg, rho0, ...) with D1Q3 cfgs of
    one N and one line length) for `steps` steps in one line group.  Returns
    one dict per run with the FP64 fields rho [N][L] and mu [N][L], the
    health flag and, if `marks` (increasing step counts below `steps`) is
    given, the densities at those steps in ``history``."""
    sims = [Simulation(r[0], r[1], storage=storage, path="split") for r in runs]
    group = Lines(sims)
    history = [[] for _ in sims]
    done = 0
    for t in list(marks or []) + [steps]:
        if t > done:
            group.step(t - done)
            done = t
        if t < steps:
            for h, s in zip(history, sims):
                h.append((t, s.moments(fields=True, raise_numeric=False)["rho"]))
    out = []
    for h, s in zip(history, sims):
        m = s.moments(fields=True, raise_numeric=False)
        out.append({"rho": m["rho"], "mu": m["mu"], "healthy": m["status"] == 0, "step": m["step"],
                    "history": h})
    group.close()
    for s in sims:
        s.close()
    return out


def _domains(mask: np.ndarray):
    """(start, length) of the runs of True in a periodic boolean line."""
    L = mask.size
    if mask.all():
        return [(0, L)]
    if not mask.any():
        return []
    start = int(np.argmin(mask))  # a False site: runs do not wrap past it
    rolled = np.roll(mask, -start)
    out, i = [], 0
    while i < L:
        if rolled[i]:
            j = i
            while j < L and rolled[j]:
                j += 1
            out.append(((i + start) % L, j - i))
            i = j
        else:
            i += 1
    return out


def coexisting_phases(rho: np.ndarray, min_contrast: float = 0.02) -> Optional[dict]:
    """Compositions of the two phases of a separated periodic line.

    Sites are split by phi^A = rho^A / sum rho above or below the mid value
    (max + min) / 2.  Each phase is represented by the volume fractions at
    the centre of its widest domain; `spread` is the largest range of any
    phi^sigma over the middle half of those two domains (zero for flat
    plateaus), and `domains` counts the domains of the A-rich phase.  None
    when phi^A varies by less than `min_contrast` (no separation)."""
    phi = rho / rho.sum(axis=0)
    a = phi[0]
    if a.max() - a.min() < min_contrast:
        return None
    mid = 0.5 * (a.max() + a.min())
    L = a.size
    res = {}
    spread = 0.0
    for name, mask in (("rich", a > mid), ("poor", a <= mid)):
        doms = _domains(mask)
        s, n = max(doms, key=lambda d: d[1])
        centre = (s + n // 2) % L
        res[name] = phi[:, centre].copy()
        core = [(s + n // 4 + k) % L for k in range(max(1, n // 2))]
        spread = max(spread, float(np.ptp(phi[:, core], axis=1).max()))
        if name == "rich":
            res["domains"] = len(doms)
    res["spread"] = spread
    return res


def main(argv=None) -> None:
    """Run one of the binodal run sets of Sec. IV and print the coexisting
    compositions of every run:  python -m paper_0704_3444_amd.phase
    binary_monomer [--steps N]."""
    import argparse
    import os
    import sys

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import lbinputs

    names = ("binary_monomer", "binary_polymer", "ternary_monomer", "ternary_polymer", "ternary_monomer_plait",
             "ternary_polymer_plait")
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("experiment", choices=names)
    ap.add_argument("--steps", type=int, default=0, help="steps per run (default: the paper's 50 000 or 200 000)")
    ap.add_argument("--storage", default="f64", choices=("f64", "f32"))
    args = ap.parse_args(argv)
    runs = lbinputs.binodal_runs(args.experiment)
    steps = args.steps or (50000 if args.experiment.startswith("binary") else 200000)
    for (cfg, rho0, label), r in zip(runs, run_lines(runs, steps, storage=args.storage)):
        ph = coexisting_phases(r["rho"]) if r["healthy"] else None
        if not r["healthy"]:
            print(f"{label:24s} unstable")
        elif ph is None:
            print(f"{label:24s} not separated")
        else:
            print(f"{label:24s} phi {np.round(ph['rich'], 5)} | {np.round(ph['poor'], 5)}  "
                  f"plateau spread {ph['spread']:.1e}  A-rich domains {ph['domains']}")


if __name__ == "__main__":
    main()
