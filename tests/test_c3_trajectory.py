"""The measured workload's long precision trajectory against the FP64 oracle.

C3 (n = 10, chi = 128, eps = 1e-6, layered model, Ricker source at depth
index 1) from rest for 2000 steps, the c^2 operator being the oracle's TT-SVD
of the model in both runs.  The GPU side (FP64, FP32 and BF16 contractions
stepped as one group) runs on a GPU machine:

    python tests/test_c3_trajectory.py c2 C2CORES.npz
    python bench.py --trajectory 500,1000,2000 --velocity-cores C2CORES.npz --save GPU_DIR

The oracle side runs on the host (about 80 minutes each on 4 threads):

    python tests/test_c3_trajectory.py oracle ORACLE_DIR            # the dense-detour stepper
    python tests/test_c3_trajectory.py floor ORACLE_DIR 1e-15 d15   # the same, inputs perturbed by 1e-15
    python tests/test_c3_trajectory.py floor ORACLE_DIR 5.96e-8 u32 # ... by FP32's unit roundoff

and the comparison is this test, with MPSW_C3_GPU and MPSW_C3_ORACLE set to the
two directories (it is skipped without them).  The floor runs give the
sensitivity floor of the workload: the distance at which two computations of
the same truncated trajectory that differ by rounding-sized perturbations
part.  GPU FP64 must lie within 10x the floor at perturbation 1e-15, BF16
within 1e-3 or 10x that floor, FP32 within 1e-6 or 10x its floor at FP32's
unit roundoff.  The summary the benchmark reports is written by

    python tests/test_c3_trajectory.py summary GPU_DIR ORACLE_DIR > profiles/trajectory_C3.json
"""
import json
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

MARKS = (500, 1000, 2000)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _oracle_run(out, delta=0.0, tag="oracle"):
    from oracle import mps as M
    from oracle import stepper as S
    import synth
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import sensitivity
    cfg = synth.get_config("C3")
    n = cfg["n"]
    N = 1 << n
    c2r = M.to_dense(S.c2_mps(cfg["c2"], n, cfg["eps_c"])).reshape(N, N)
    ds = sensitivity.PerturbedStepper(delta, 0, n, cfg["lam"], cfg["eps"], cfg["chi"], c2r,
                                      src=(cfg["ix"], cfg["iz"]), wavelet=cfg["wavelet_samples"])
    ds.keep_log = False
    for k in range(1, max(MARKS) + 1):
        ds.step()
        if k in MARKS:
            np.save(os.path.join(out, f"{tag}_u{k}.npy"), ds.dense())
            if delta == 0.0:
                json.dump({"ranks": ds.ranks, "first_flag": ds.first_flag(),
                           "flags": [(a, b, c, sorted(d)) for a, b, c, d in ds.flags]},
                          open(os.path.join(out, f"{tag}_log.json"), "w"))
        if k % 100 == 0:
            print(tag, "step", k, ds.ranks[-1][2], flush=True)


def summary(gpu, orc):
    rows = []
    log = json.load(open(os.path.join(orc, "oracle_log.json")))
    for k in MARKS:
        o = np.load(os.path.join(orc, f"oracle_u{k}.npy"))
        r = {"step": k, "middle_bond": log["ranks"][k - 1][2][len(log["ranks"][k - 1][2]) // 2]}
        for p in ("fp64", "fp32", "bf16"):
            r[p] = rel(np.load(os.path.join(gpu, f"gpu_{p}_u{k}.npy")).astype(np.float64), o)
        for tag in ("d15", "u32"):
            f = os.path.join(orc, f"{tag}_u{k}.npy")
            if os.path.exists(f):
                r[f"floor_{tag}"] = rel(np.load(f), o)
        rows.append(r)
    return {"workload": "C3: n=10, chi=128, eps=1e-6, 2000 steps from rest", "first_flagged_cut": log["first_flag"],
            "checkpoints": rows}


@pytest.mark.skipif(not (os.environ.get("MPSW_C3_GPU") and os.environ.get("MPSW_C3_ORACLE")),
                    reason="needs the saved GPU and oracle trajectories (see the module docstring)")
def test_c3_trajectory_against_oracle():
    s = summary(os.environ["MPSW_C3_GPU"], os.environ["MPSW_C3_ORACLE"])
    print(json.dumps(s, indent=1))
    for r in s["checkpoints"]:
        floor = r["floor_d15"]
        assert r["fp64"] <= 10.0 * floor, r
        assert r["bf16"] <= max(1e-3, 10.0 * floor), r
        # FP32: the 1e-6 target lies below this workload's floor at FP32's unit
        # roundoff (7.4e-5 at step 500), so FP32 is held to that floor
        assert r["fp32"] <= max(1e-6, 10.0 * max(floor, r.get("floor_u32", 0.0))), r


if __name__ == "__main__":
    what, out = sys.argv[1], sys.argv[2]
    if what == "c2":
        from oracle import mps as M
        from oracle import stepper as S
        import synth
        cfg = synth.get_config("C3")
        ref = S.c2_mps(cfg["c2"], cfg["n"], cfg["eps_c"])
        np.savez(out, bonds=np.array(M.bonds_of(ref)), cores=np.concatenate([c.ravel() for c in ref]))
    elif what == "oracle":
        _oracle_run(out)
    elif what == "floor":
        _oracle_run(out, float(sys.argv[3]), sys.argv[4])
    elif what == "summary":
        print(json.dumps(summary(out, sys.argv[3]), indent=1))
