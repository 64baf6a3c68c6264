"""Rounding-schedule study on the FP64 oracle (not collected by pytest; CPU).

The same workload is stepped by the core-level oracle stepper under each
rounding schedule ("three": eq. 17 as the library computes it; "seven": a
rounding after every shift-operator application as well; "one": only the
update sum rounded, usable on small grids since the Laplacian and c^2 products
are kept exact).  Each checkpoint is compared with the dense FDTD update of
eq. 2 on the same c^2 reconstruction, so the difference is the state
truncation of that schedule alone.

    python tests/schedule_study.py C2 50,100,150,200 three,seven
    python tests/schedule_study.py small 20,40,60 three,seven,one

Prints one JSON line per schedule.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import fdtd as F  # noqa: E402
from oracle import mps as M  # noqa: E402
from oracle import stepper as S  # noqa: E402
import synth  # noqa: E402


def workload(name, steps):
    if name == "small":
        n = 5
        N = 1 << n
        return dict(n=n, chi=8, eps=1e-6, lam=0.5, eps_c=1e-8,
                    c2=synth.layered_fault_velocity(n, dh=40.0) * 1e-8,
                    src=(N // 3, 2), wavelet=synth.ricker(steps, 0.004, 20.0))
    cfg = synth.get_config(name, steps=steps)
    return dict(n=cfg["n"], chi=cfg["chi"], eps=cfg["eps"], lam=cfg["lam"], eps_c=cfg["eps_c"],
                c2=cfg["c2"], src=(cfg["ix"], cfg["iz"]), wavelet=cfg["wavelet_samples"])


def run(name, checkpoints, schedule):
    last = max(checkpoints)
    w = workload(name, last)
    n = w["n"]
    N = 1 << n
    c2m = S.c2_mps(w["c2"], n, w["eps_c"])
    c2r = M.from_sites(M.to_dense(c2m), n)
    st = S.MPSStepper(n, w["lam"], w["eps"], w["chi"], c2m, src=w["src"], wavelet=w["wavelet"],
                      schedule=schedule)
    a, b = np.zeros((N, N)), np.zeros((N, N))
    out = {"workload": name, "n": n, "chi": w["chi"], "eps": w["eps"], "schedule": schedule,
           "checkpoints": []}
    t0 = time.time()
    for k in range(last):
        st.step()
        a, b = b, F.fdtd_step(b, a, c2r, w["lam"], w["wavelet"][k], w["src"], "periodic")
        if k + 1 in checkpoints:
            g = st.dense()
            bonds = M.bonds_of(st.psi)
            out["checkpoints"].append({"step": k + 1, "rel_l2_vs_eq2": float(np.linalg.norm(g - b) / np.linalg.norm(b)),
                                       "max_bond": int(max(bonds)), "sum_bonds": int(sum(bonds))})
    out["seconds"] = round(time.time() - t0, 2)
    out["roundings_per_step"] = {"three": 3, "seven": 3 + 4, "one": 1}[schedule]
    return out


if __name__ == "__main__":
    name = sys.argv[1] if len(sys.argv) > 1 else "small"
    cps = [int(x) for x in (sys.argv[2] if len(sys.argv) > 2 else "20,40,60").split(",")]
    schedules = (sys.argv[3] if len(sys.argv) > 3 else "three,seven,one").split(",")
    for sch in schedules:
        print(json.dumps(run(name, cps, sch)), flush=True)
