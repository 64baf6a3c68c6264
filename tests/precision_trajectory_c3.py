"""C3 precision trajectory against the FP64 oracle (not collected by pytest:
the oracle needs about 45 minutes of host time for the 2000 steps).

The GPU side runs first, on a GPU machine:

    python bench.py --trajectory 500,1000,1500,2000 --save OUT

which steps one C3 shot from rest with FP64, FP32 and BF16 contractions
together and prints the relative L2 of FP32 and BF16 against FP64 at those
steps, saving the FP64 fields.  This script then runs the dense-detour FP64
oracle stepper over the same workload and compares:

    python tests/precision_trajectory_c3.py OUT [ORACLE_DIR]

It prints, per step, the relative L2 of the GPU FP64 run against the oracle.
Once the truncation rule acts (eps = 1e-6), and more so once the chi cap binds,
two FP64 computations that differ only in rounding order leave each other:
the oracle-vs-GPU-FP64 distance is the sensitivity floor of the workload, the
level against which the FP32 and BF16 distances are read.
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import mps as M          # noqa: E402
from oracle import stepper as S      # noqa: E402
import synth                         # noqa: E402

MARKS = (500, 1000, 1500, 2000)


def oracle_run(out):
    cfg = synth.get_config("C3")
    n = cfg["n"]
    N = 1 << n
    c2r = M.to_dense(S.c2_mps(cfg["c2"], n, cfg["eps_c"])).reshape(N, N)
    ds = S.DenseStepper(n, cfg["lam"], cfg["eps"], cfg["chi"], c2r, src=(cfg["ix"], cfg["iz"]),
                        wavelet=cfg["wavelet_samples"])
    for k in range(1, max(MARKS) + 1):
        ds.step()
        if k in MARKS:
            np.save(os.path.join(out, f"oracle_u{k}.npy"), ds.dense())
        if k % 100 == 0:
            print("oracle step", k, ds.ranks[-1][2], flush=True)


def main():
    gpu = sys.argv[1]
    orc = sys.argv[2] if len(sys.argv) > 2 else gpu
    if not all(os.path.exists(os.path.join(orc, f"oracle_u{k}.npy")) for k in MARKS):
        oracle_run(orc)
    for k in MARKS:
        g = np.load(os.path.join(gpu, f"gpu_fp64_u{k}.npy"))
        o = np.load(os.path.join(orc, f"oracle_u{k}.npy"))
        print(f"step {k}: GPU FP64 vs FP64 oracle rel-L2 {np.linalg.norm(g - o) / np.linalg.norm(o):.3e}")


if __name__ == "__main__":
    main()
