"""Site-order study (not collected by pytest; needs a GPU).

The same workload is stepped on the GPU twice, once with the sites in the
register order of eq. 3 (x bits, then z bits) and once interleaved
(x_{n-1} z_{n-1} ... x_0 z_0).  At each checkpoint the field is compared with
the dense FDTD update of eq. 2 on that order's own reconstruction of c^2, so
the difference is the state truncation of that order alone; the bonds, the
largest exact bond of each rounding and the discarded tails are reported too.

    python tests/ordering_study.py C2 250,500,750,1000
    python tests/ordering_study.py C3 250,500,750,1000

Prints one JSON line per order.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import fdtd as F  # noqa: E402
import synth  # noqa: E402


def run(mpsw, name, checkpoints, ordering):
    last = max(checkpoints)
    cfg = synth.get_config(name, steps=last)
    n = cfg["n"]
    N = 1 << n
    order = mpsw.MPSW_INTERLEAVED if ordering == "interleaved" else mpsw.MPSW_SEQUENTIAL
    st = mpsw.State(mpsw.make_config(n, cfg["chi"], cfg["eps"], cfg["lam"], ordering=order))
    st.set_velocity_dense(cfg["c2"], cfg["eps_c"])
    src = (cfg["ix"], cfg["iz"])
    st.set_source(0, src[0], src[1], cfg["wavelet_samples"])
    c2r = st.to_dense(0, 2)
    out = {"workload": name, "n": n, "chi": cfg["chi"], "eps": cfg["eps"], "order": ordering,
           "c2_bonds": st.bonds(0, 2),
           "c2_rel_err": float(np.linalg.norm(c2r - cfg["c2"]) / np.linalg.norm(cfg["c2"])),
           "rows": []}
    a = b = np.zeros((N, N))
    t0 = time.perf_counter()
    for k in range(last):
        st.step(1)
        a, b = b, F.fdtd_step(b, a, c2r, cfg["lam"], cfg["wavelet_samples"][k], src)
        if k + 1 in checkpoints:
            g = st.to_dense(0, 0)
            s = st.stats(0)
            row = {"step": k + 1, "rel_l2_vs_fdtd": float(np.linalg.norm(g - b) / np.linalg.norm(b)),
                   "bonds": st.bonds(0, 0), "max_exact_bond": list(s["max_exact_bond"]),
                   "tail2": [float(x) for x in s["tail2"]], "elapsed_s": time.perf_counter() - t0}
            out["rows"].append(row)
            print(f"{name} {ordering} step {k + 1}: rel-L2 vs dense FDTD {row['rel_l2_vs_fdtd']:.3e}; "
                  f"max bond {max(row['bonds'])}; exact bonds {row['max_exact_bond']}", file=sys.stderr,
                  flush=True)
    st.close()
    return out


def main():
    name = sys.argv[1] if len(sys.argv) > 1 else "C2"
    checkpoints = [int(x) for x in (sys.argv[2] if len(sys.argv) > 2 else "250,500,750,1000").split(",")]
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("a GPU is needed")
    from paper_2609_01904_amd import mpsw
    mpsw.load()
    for ordering in ("sequential", "interleaved"):
        print(json.dumps(run(mpsw, name, checkpoints, ordering)), flush=True)


if __name__ == "__main__":
    main()
