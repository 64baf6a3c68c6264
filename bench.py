"""Throughput of the quantics-MPS wave step (eq. 17) on one GPU.

One step = the three roundings of the time step (Laplacian MPO, c^2 Hadamard,
MPS sum + source), each an L->R QR sweep plus an R->L truncated SVD sweep
(Sec. 4.3), for every shot of the batch.  The default measures the chosen form
(256 shots advanced together, FP64 throughout, launch shapes autotuned) and,
beside it, the other forms (FP32 contractions, learned rank) and the plain form
(one shot, FP64, exact SVD).  The workload is the n = 10 grid
(1024 x 1024, dh = 10 m, dt = 1 ms) over the seeded layered-fault velocity model
(c^2 MPO cutoff 1e-6), chi_max = 128, eps = 1e-6, Ricker 15 Hz sources at depth
index 1.  Timing starts from a developed wavefield (a seeded superposition of
circular wavefronts, every middle bond at the chi cap), so the timed steps are
steady-state steps at the cap.

Prints ONE JSON line (rank 0).  `value` is shot-steps per second over the
timed steps with all inputs resident on the device.  `roofline` is the dominant
kernel class: its algorithmic flops (counted on the device from the live bond
sizes) over its event-timed launch durations in the same timed region.
`cpu_baseline` times the FP64 CPU oracle (dense-detour stepper) on a bounded
sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# Peaks of one MI355X (published).  FP64 vector: 256 CUs x 4 SIMDs x 16 lanes
# x 2 flop (FMA) x 2.4 GHz = 78.6 TFLOP/s, the same as the FP64 matrix-core peak.
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

KERNEL_SOURCES = {
    0: ["paper_2609_01904_amd/csrc/fact.hip"],
    1: ["paper_2609_01904_amd/csrc/fact.hip"],
    2: ["paper_2609_01904_amd/csrc/kernels.hip"],
    3: ["paper_2609_01904_amd/csrc/fact.hip"],
    4: ["paper_2609_01904_amd/csrc/fact.hip"],
}
KERNEL_NAMES = {0: "k_qrf", 1: "k_jac", 2: "k_gemm", 3: "k_applyq", 4: "k_applyv"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash(kclass):
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[kclass] + ["paper_2609_01904_amd/csrc/mpsw_device.h",
                                         "paper_2609_01904_amd/csrc/mpsw_internal.h"]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(kclass, workload, batch, precision):
    """HBM bytes per launch from a committed counter summary, or None when the
    summary is missing or was taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{KERNEL_NAMES[kclass]}_{workload}_b{batch}_{precision}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.strip().split("=", 1)
                vals[k.strip()] = v.strip()
    if vals.get("SOURCE_HASH") != source_hash(kclass):
        return None
    try:
        return float(vals["HBM_BYTES_PER_LAUNCH"])
    except (KeyError, ValueError):
        return None


def log_rank_data(st, steps, chi, shot=0):
    """Step an exact-rank state `steps` times; for every bond and rounding the
    network input the library forms for the coming step (its rank features)
    and, as the label, the rank the exact rule then kept, divided by chi.
    Returns (X, y) as float32."""
    K = st.K
    X, y, feats = [], [], None
    for _ in range(steps):
        st.step(1)
        ranks = [st.bonds(shot, 3), st.bonds(shot, 4), st.bonds(shot, 0)]   # y, w, psi after the step
        if feats is not None:
            for j in range(3):
                X.append(feats[j])
                y.append(np.asarray(ranks[j][1:K], dtype=np.float64) / chi)
        feats = [st.rank_features(shot, j) for j in range(3)]
    return np.concatenate(X).astype(np.float32), np.concatenate(y).astype(np.float32)


def train_rank_model(mpsw, synth, steps=80):
    """Rank network trained on spectra of an exact run of the n=8, chi=64 workload."""
    cfg = synth.get_config("C2", steps=steps)
    n, chi = cfg["n"], cfg["chi"]
    st = mpsw.State(mpsw.make_config(n, chi, cfg["eps"], cfg["lam"]))
    st.set_velocity_dense(cfg["c2"], cfg["eps_c"])
    up, u = synth.wavefront_fields(n, seed=5)
    st.set_fields(0, up, u)
    st.set_source(0, cfg["ix"], cfg["iz"], cfg["wavelet_samples"])
    X, y = log_rank_data(st, steps, chi)
    st.close()
    w0 = mpsw.mlp_init(seed=1)
    w = mpsw.mlp_train(X, y, w0, epochs=400, lr=2e-3, alpha=4.0)
    return w, len(y)


def make_state(mpsw, synth, workload, batch, precision, rank="exact", model=None, ordering="sequential",
               velocity=None, from_rest=False):
    """State of `batch` shots of a workload from its developed wavefield.  The
    c^2 operator is the device's TT-SVD of the dense model, or the given
    (bonds, cores) of its diagonal in the state's site order."""
    cfg = synth.get_config(workload)
    n = cfg["n"]
    N = 1 << n
    prec = {"fp64": mpsw.MPSW_FP64, "fp32": mpsw.MPSW_FP32, "bf16": mpsw.MPSW_BF16}[precision]
    rmode = {"learned": mpsw.MPSW_RANK_LEARNED, "previous": mpsw.MPSW_RANK_PREVIOUS}.get(rank, mpsw.MPSW_RANK_EXACT)
    order = mpsw.MPSW_INTERLEAVED if ordering == "interleaved" else mpsw.MPSW_SEQUENTIAL
    nd = cfg["ndim"]
    cfgs = [mpsw.make_config(n, cfg["chi"], cfg["eps"], cfg["lam"], precision=prec, rank_mode=rmode, seed=11,
                             ordering=order, ndim=nd)
            for _ in range(batch)]
    st = mpsw.State(cfgs if batch > 1 else cfgs[0])
    if velocity is None:
        st.set_velocity_dense(cfg["c2"], cfg["eps_c"])
    else:
        st.set_velocity_mpo(*velocity)
    if model is not None:
        st.set_rank_model(model)
    fields = []
    if nd == 3:   # the cube: 8 variants of one developed wavefield (x, y swapped and flipped)
        up0, u0 = synth.wavefront_fields_3d(n, seed=0)
        for b in range(batch):
            def sym(f):
                g = f.transpose(1, 0, 2) if b % 2 else f
                g = g[::-1] if (b // 2) % 2 else g
                return np.ascontiguousarray(g[:, ::-1] if (b // 4) % 2 else g)
            up, u = sym(up0), sym(u0)
            st.set_fields(b, up, u)
            ix = (cfg["ix"] + b * (N // max(batch, 1))) % N
            st.set_source_3d(b, ix, cfg["iy"], cfg["iz"], cfg["wavelet_samples"])
            fields.append((up, u, (ix, cfg["iy"], cfg["iz"])))
        return st, cfg, fields
    up0, u0 = (np.zeros((N, N)), np.zeros((N, N))) if from_rest else synth.wavefront_fields(n, seed=0)
    for b in range(batch):
        # shot b starts from one of the 8 symmetries of the square of the same wavefield
        sym = lambda f: np.rot90(f[::-1] if (b // 4) % 2 else f, b % 4).copy()  # noqa: E731
        up, u = sym(up0), sym(u0)
        if not from_rest:
            st.set_fields(b, up, u)
        # distinct source positions along the surface row
        ix = (cfg["ix"] + b * (N // max(batch, 1))) % N
        st.set_source(b, ix, cfg["iz"], cfg["wavelet_samples"])
        fields.append((up, u, (ix, cfg["iz"])))
    return st, cfg, fields


def cpu_baseline(synth, workload, fields, seconds, ordering="sequential"):
    """Steps/s of the FP64 CPU oracle (dense-detour stepper) from shot 0's state."""
    from oracle import mps as OM
    from oracle.stepper import DenseStepper
    try:
        from threadpoolctl import threadpool_info
        cores = max([x.get("num_threads", 1) for x in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    cfg = synth.get_config(workload)
    n = cfg["n"]
    N = 1 << n
    nd = cfg["ndim"]
    c2 = OM.from_sites(OM.to_dense(OM.tt_svd(OM.to_sites(cfg["c2"], ordering), nd * n, cfg["eps_c"],
                                              chi_max=1 << 30)), n, ordering, nd)
    up, u, src = fields[0]
    ds = DenseStepper(n, cfg["lam"], cfg["eps"], cfg["chi"], c2, src=src,
                      wavelet=cfg["wavelet_samples"], ordering=ordering)
    ds.set_fields(up, u)
    steps, t0 = 0, time.perf_counter()
    while True:
        ds.step()
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= 50:
            break
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": steps / el, "unit": "steps/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{steps} steps of the same workload (shot 0, same starting wavefield) with the "
                      f"FP64 dense-detour oracle stepper on the host, {el:.1f} s "
                      f"({model}, {os.cpu_count()} logical CPUs visible)"}


def write_metrics(st, path, steps):
    """Per-step record of shot 0: one JSON line per step."""
    K = st.K
    with open(path, "w") as f:
        for _ in range(steps):
            st.step(1)
            s = st.stats(0)
            rec = {"step": s["step"], "bonds": s["bonds"], "max_exact_bond": s["max_exact_bond"],
                   "tail2": s["tail2"], "max_jacobi_sweeps": s["max_jacobi_sweeps"],
                   "sketches": s["sketches"], "fallbacks": s["fallbacks"],
                   "sigma_middle": [[float(x) for x in st.sigma_log(0, r)[K // 2][:8]] for r in range(3)]}
            f.write(json.dumps(rec) + "\n")
    log(f"per-step metrics of shot 0 for {steps} steps in {path}")


def copy_calibration(torch):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    nbytes = 1 << 30
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 5}))


def make_mixed_states(mpsw, synth, precision, steps, nshots=64, velocity=None):
    """States of the batched-shots workload: the seeded shot list (grids n in
    {8, 9, 10}, chi caps in {32, 64, 128}, Ricker sources), one state per grid
    holding its shots with the layered model of that grid (c^2 operator from
    the device's TT-SVD, or velocity[n] = (bonds, cores)).  Returns (states,
    {n: shots of that state in order}, all shots)."""
    shots = synth.batch_shots(nshots, seed=1, steps=steps)
    prec = {"fp64": mpsw.MPSW_FP64, "fp32": mpsw.MPSW_FP32, "bf16": mpsw.MPSW_BF16}[precision]
    states, groups = [], {}
    for n in sorted(set(sh["n"] for sh in shots)):
        mine = [sh for sh in shots if sh["n"] == n]
        groups[n] = mine
        cfg = synth.get_config("C3", n=n)
        lam = mine[0]["dt"] / mine[0]["dh"]
        st = mpsw.State([mpsw.make_config(n, sh["chi"], sh["eps"], lam, precision=prec) for sh in mine])
        if velocity is None:
            st.set_velocity_dense(cfg["c2"], cfg["eps_c"])
        else:
            st.set_velocity_mpo(*velocity[n])
        for i, sh in enumerate(mine):
            st.set_source(i, sh["ix"], sh["iz"], sh["wavelet_samples"])
        states.append(st)
    return states, groups, shots


def mixed_batch(mpsw, synth, torch, args):
    """The batched-shots workload: 64 shots on grids n in {8, 9, 10} with chi
    caps in {32, 64, 128} (seeded), one state per grid size holding its shots,
    all states stepped by one group graph.  The shots start from rest; the
    first `warmup` steps are untimed, then each state's launch shapes are
    autotuned, then `steps` steps are timed."""
    t0 = time.perf_counter()
    states, groups, shots = make_mixed_states(mpsw, synth, args.precision, args.warmup + args.steps)
    counts = {n: len(g) for n, g in groups.items()}
    grp = mpsw.Group(states)
    done = 0
    while done < args.warmup:
        k = min(100, args.warmup - done)
        grp.step(k)
        torch.cuda.synchronize()
        done += k
        log(f"mixed batch: warm-up step {done}")
    tuned = {}
    if not args.no_tune:
        for st in states:
            tuned[st.K // 2] = st.autotune(2)
        log(f"autotuned (QR workgroups per shot, Jacobi block) per grid n: {tuned}")
    grp.close()
    grp = mpsw.Group(states)   # captured with the tuned shapes
    grp.step(3)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    left = args.steps - 3
    while left > 0:
        k = min(99, left)
        grp.step(k)
        torch.cuda.synchronize()
        left -= k
        log(f"mixed batch: {args.steps - left} of {args.steps} timed steps ({time.perf_counter() - t1:.0f} s)")
    el = time.perf_counter() - t1
    timed = args.steps - 3
    nshot = len(shots)
    out = {
        "metric": "aggregate shot-steps/s, 64 shots on mixed grids in one graph",
        "value": nshot * timed / el, "unit": "shot-steps/s", "n_gpus": 1, "steps": timed,
        "warmup": args.warmup + 3, "ms_per_step": el * 1e3 / timed, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}[args.precision], "data": "synthetic",
        "config": {"workload": "C4: 64 Ricker shots (f0 ~ U[8, 25] Hz, x ~ U, depth 10 m), n ~ U{8, 9, 10}, "
                               "chi ~ U{32, 64, 128}, eps=1e-06, layered-fault c^2 per grid",
                   "shots_per_grid": {str(k): v for k, v in counts.items()},
                   "tuned": {str(k): list(v) for k, v in tuned.items()}, "graph": True},
        "max_bonds": {str(st.K // 2): max(max(st.bonds(b, 0)) for b in range(st.nshots)) for st in states},
        "setup_and_warmup_s": t1 - t0,
    }
    print(json.dumps(out), flush=True)
    grp.close()
    for st in states:
        st.close()


def mixed_trajectory(mpsw, synth, torch, args):
    """The batched-shots workload from rest through the given steps, one group
    graph, in the chosen precision; the first shot of each grid is saved at
    each of those steps (FP32 .npy, enough for distances down to 1e-7) so that
    it can be held against the oracle."""
    marks = sorted(set(int(x) for x in args.trajectory.split(",")))
    velocity = load_velocity_cores_mixed(args.velocity_cores) if args.velocity_cores else None
    states, groups, shots = make_mixed_states(mpsw, synth, args.precision, marks[-1], velocity=velocity)
    first = {}
    for i, sh in enumerate(shots):
        first.setdefault(sh["n"], i)
    grp = mpsw.Group(states)
    if args.save:
        os.makedirs(args.save, exist_ok=True)
    rows, done, t0 = [], 0, time.perf_counter()
    for mark in marks:
        while done < mark:
            k = min(99, mark - done)
            grp.step(k)
            torch.cuda.synchronize()
            done += k
            log(f"mixed trajectory: step {done} ({time.perf_counter() - t0:.0f} s)")
        for st in states:
            n = st.K // 2
            row = {"step": mark, "n": n, "shot": first[n], "bonds": st.bonds(0, 0)}
            rows.append(row)
            if args.save:
                np.save(os.path.join(args.save, f"gpu_s{first[n]}_u{mark}.npy"), st.to_dense(0, 0).astype(np.float32))
    print(json.dumps({"workload": "C4", "precision": args.precision, "trajectory": rows,
                      "seconds": time.perf_counter() - t0}), flush=True)
    grp.close()
    for st in states:
        st.close()


def precision_trajectory(mpsw, synth, torch, args):
    """FP64, FP32 and BF16 contractions on the same shot from rest, stepped
    together as one group; rel-L2 of FP32 and BF16 against FP64 at the given
    steps (the fields can be saved and held against the oracle).  With
    --rank learned a fourth member runs the mixed form: BF16 contractions and
    the learned rank (network trained as for the headline's forms)."""
    cfg = synth.get_config(args.workload)
    n = cfg["n"]
    precs = [("fp64", mpsw.MPSW_FP64), ("fp32", mpsw.MPSW_FP32), ("bf16", mpsw.MPSW_BF16)]
    model = None
    if args.rank == "learned":
        t0 = time.perf_counter()
        model, nrows = train_rank_model(mpsw, synth)
        log(f"rank network trained on {nrows} logged bonds in {time.perf_counter() - t0:.1f} s")
        precs.append(("bf16l", mpsw.MPSW_BF16))
    states = []
    for name, p in precs:
        learned = name == "bf16l"
        st = mpsw.State(mpsw.make_config(n, cfg["chi"], cfg["eps"], cfg["lam"], precision=p, seed=11,
                                         rank_mode=mpsw.MPSW_RANK_LEARNED if learned else mpsw.MPSW_RANK_EXACT))
        if learned:
            st.set_rank_model(model)
        if args.velocity_cores:
            st.set_velocity_mpo(*load_velocity_cores(args.velocity_cores))
        else:
            st.set_velocity_dense(cfg["c2"], cfg["eps_c"])
        st.set_source(0, cfg["ix"], cfg["iz"], cfg["wavelet_samples"])
        states.append(st)
    grp = mpsw.Group(states)
    marks = sorted(set(int(x) for x in args.trajectory.split(",")))
    if args.save:
        os.makedirs(args.save, exist_ok=True)
        if args.save_window <= 0:
            np.save(os.path.join(args.save, "gpu_c2r.npy"), states[0].to_dense(0, 2))
    rows, done, t0 = [], 0, time.perf_counter()
    window = {"outside_norm": {}}
    for mark in marks:
        while done < mark:
            k = min(50, mark - done)
            grp.step(k)
            torch.cuda.synchronize()
            done += k
            log(f"trajectory: step {done} ({time.perf_counter() - t0:.0f} s), bonds {states[0].bonds(0, 0)}")
        u = [st.to_dense(0, 0) for st in states]
        nb = float(np.linalg.norm(u[0]))
        row = {"step": mark, "bonds_fp64": states[0].bonds(0, 0)}
        for (name, _), v in zip(precs[1:], u[1:]):
            row[f"rel_l2_{name}_vs_fp64"] = float(np.linalg.norm(v - u[0])) / nb if nb > 0 else 0.0
        rows.append(row)
        if args.save and args.save_window > 0:
            # every member in FP64 on the W x W window centred on the source
            # (the grid is periodic: the field is rolled so that the source sits
            # at (W/2, W/2)), and the norm of what lies outside it, so the
            # full-field distance can be bounded
            W = min(args.save_window, 1 << n)
            shift = [W // 2 - cfg["ix"], W // 2 - cfg["iz"]]
            window.update({"shift": shift, "W": W})
            for (name, _), v in zip(precs, u):
                win, out = window_split(v, shift, W)
                np.save(os.path.join(args.save, f"gpu_{name}_u{mark}.npy"), win)
                window["outside_norm"][f"{name}_u{mark}"] = out
                if name == "fp64" and out > 1e-14 * float(np.linalg.norm(v)):
                    # the whole FP64 member in FP32 as well: with the window in
                    # FP64 (window_join) its distance is exact to FP32 outside
                    np.save(os.path.join(args.save, f"gpu_fp64_full_u{mark}.npy"), v.astype(np.float32))
        elif args.save:   # FP64 fields in FP64; the others in FP32, enough for their distances
            np.save(os.path.join(args.save, f"gpu_fp64_u{mark}.npy"), u[0])
            for (name, _), v in zip(precs[1:], u[1:]):
                np.save(os.path.join(args.save, f"gpu_{name}_u{mark}.npy"), v.astype(np.float32))
    out = {"workload": args.workload, "trajectory": rows, "seconds": time.perf_counter() - t0}
    if model is not None:
        s = states[-1].stats(0)
        out["learned_rank"] = {"sketches": s["sketches"], "fallbacks": s["fallbacks"]}
    if args.save:
        with open(os.path.join(args.save, "trajectory.json"), "w") as f:
            json.dump(dict(out, window=window if args.save_window > 0 else None), f)
    print(json.dumps(out), flush=True)
    grp.close()
    for st in states:
        st.close()


def load_velocity_cores(path):
    """(bonds, cores) of a c^2 operator saved with numpy.savez(path, bonds=..., cores=<flat>)."""
    with np.load(path) as z:
        bonds = [int(b) for b in z["bonds"]]
        flat = np.asarray(z["cores"], dtype=np.float64)
    cores, o = [], 0
    for k in range(len(bonds) - 1):
        sz = bonds[k] * 2 * bonds[k + 1]
        cores.append(flat[o:o + sz].reshape(bonds[k], 2, bonds[k + 1]))
        o += sz
    return bonds, cores


def window_split(v, shift, W):
    """(W x W window of the periodic field v rolled by shift, norm of the rest).
    The rest's norm is summed directly: a difference of squared norms would
    cancel to noise."""
    rolled = np.roll(v, shift, axis=(0, 1))
    win = rolled[:W, :W].copy()
    rolled[:W, :W] = 0.0
    return win, float(np.linalg.norm(rolled))


def window_join(full, win, shift):
    """The field `full` (any precision) with its window replaced by `win`."""
    W = win.shape[0]
    rolled = np.roll(np.asarray(full, dtype=np.float64), shift, axis=(0, 1))
    rolled[:W, :W] = win
    return np.roll(rolled, (-shift[0], -shift[1]), axis=(0, 1))


def load_velocity_cores_mixed(path):
    """{n: (bonds, cores)} of the c^2 operators of several grids, saved with
    numpy.savez(path, bonds_<n>=..., cores_<n>=<flat>)."""
    out = {}
    with np.load(path) as z:
        for key in z.files:
            if key.startswith("bonds_"):
                n = int(key[6:])
                bonds = [int(b) for b in z[key]]
                flat = np.asarray(z[f"cores_{n}"], dtype=np.float64)
                cores, o = [], 0
                for k in range(len(bonds) - 1):
                    sz = bonds[k] * 2 * bonds[k + 1]
                    cores.append(flat[o:o + sz].reshape(bonds[k], 2, bonds[k + 1]))
                    o += sz
                out[n] = (bonds, cores)
    return out


def accuracy_summary():
    """Relative L2 against the FP64 oracle at the checkpoints of the long
    precision trajectory (a committed measurement summary), or None."""
    path = os.path.join(ROOT, "profiles", "trajectory_C3.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def run_form(mpsw, synth, torch, args, batch, precision, rank, model=None, velocity=None, tune=None, kclass=None):
    """Build a state of `batch` shots, tune it (or take `tune`), warm up, time
    args.steps steps.  With kclass (-1: the class with the most event time in
    one untimed probe step) the launches of that kernel class are timed with
    HIP events on the state's stream during the timed steps.  Returns (state,
    cfg, fields, result, kernel class, its profile)."""
    t0 = time.perf_counter()
    st, cfg, fields = make_state(mpsw, synth, args.workload, batch, precision, rank, model, args.ordering, velocity,
                                 from_rest=args.from_rest)
    if args.from_rest:   # the warm-up grows the bonds first, so the tuner sees the timed steps' sizes
        done = 0
        while done < args.warmup:
            k = min(25, args.warmup - done)
            st.step(k)
            torch.cuda.synchronize()
            done += k
            log(f"warm-up from rest: step {done}, bonds of shot 0 {st.bonds(0, 0)}")
    tuned = tune
    if tune is None and args.shapes:
        tune = tuned = tuple(int(x) for x in args.shapes.split(","))
    if tune is not None:
        st.set_launch_shapes(*tune)
    elif not args.no_tune:
        tuned = st.autotune(2)
    if not args.from_rest:
        st.step(max(args.warmup, 0))
    torch.cuda.synchronize()
    prof = None
    if kclass is not None and kclass < 0:   # the class with the most event time over one probe step (untimed)
        best = None
        for c in range(5):
            st.profile(c)
            st.step(1)
            p = st.profile_read(c)
            log(f"probe class {mpsw.KC_NAMES[c]}: {p['total_ms']:.2f} ms in {p['launches']} launches")
            if best is None or p["total_ms"] > best[1]:
                best = (c, p["total_ms"])
        kclass = best[0]
    if kclass is not None:
        st.profile(kclass)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st.step(args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    if kclass is not None:
        prof = st.profile_read(kclass)
    stats = [st.stats(b) for b in range(batch)]
    res = {"value": batch * args.steps / el, "unit": "shot-steps/s",
           "per_shot_steps_per_s": args.steps / el, "ms_per_step": el * 1e3 / args.steps,
           "shots": batch, "precision": precision,
           "rank": {"exact": "exact SVD", "learned": "learned rank + range finder, exact fallback",
                    "previous": "previous step's rank + range finder, exact fallback"}[rank],
           "tuned": None if tuned is None else {"workgroups_per_shot": tuned[0], "jacobi_block": tuned[1] or "rule"},
           "sketches": int(sum(x["sketches"] for x in stats)), "fallbacks": int(sum(x["fallbacks"] for x in stats)),
           "setup_s": t1 - t0}
    log(f"form {precision}/{rank}/{batch} shots: {res['value']:.1f} shot-steps/s "
        f"({res['ms_per_step']:.1f} ms per step; sketches {res['sketches']}, fallbacks {res['fallbacks']})")
    return st, cfg, fields, res, kclass, prof


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=6)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=256, help="shots advanced together")
    ap.add_argument("--workload", default="C3")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16"],
                    help="contraction arithmetic (factorisations and truncation stay FP64)")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-shape autotuner")
    ap.add_argument("--from-rest", action="store_true",
                    help="start the shots from rest (sources only) instead of the developed wavefield; the "
                         "warm-up steps run before the autotuner")
    ap.add_argument("--shapes", default=None, metavar="Q,B",
                    help="launch shapes (QR workgroups per shot, Jacobi block; 0 = the width rule) instead of "
                         "the autotuner, e.g. the pair it picked in an earlier run")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the single-shot FP64 reference run (plain form, rel-L2 of shot 0)")
    ap.add_argument("--rank", default="exact", choices=["exact", "learned", "previous"],
                    help="learned: rank network (trained here on spectra logged from a short exact run of the "
                         "n=8, chi=64 layered-model workload) + randomized range finder with exact fallback; "
                         "previous: the same range finder at each bond's rank of the previous step, no network")
    ap.add_argument("--graph", action="store_true",
                    help="replay captured HIP graphs (three steps per launch) in the timed region; "
                         "the roofline kernel is then timed over an equal eager region after it")
    ap.add_argument("--kernel-class", type=int, default=-1,
                    help="kernel class for the roofline (-1: the one with most time)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--ordering", default="sequential", choices=["sequential", "interleaved"],
                    help="site order of the quantics MPS: x bits then z bits, or the two interleaved")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--trajectory", default=None, metavar="STEPS",
                    help="precision run instead of the throughput measurement: one shot of the "
                         "workload from rest in FP64, FP32 and BF16 contractions (one group), the "
                         "relative L2 of FP32 and BF16 against FP64 at these comma-separated steps; "
                         "with --workload C4, the 64-shot batch from rest in --precision, the first "
                         "shot of each grid saved at these steps")
    ap.add_argument("--save", default=None, help="directory for the trajectory's fields (.npy)")
    ap.add_argument("--save-window", type=int, default=0, metavar="W",
                    help="save the trajectory's fields on a W x W window centred on the source (periodic "
                         "grid) in FP64, with the norm outside it, instead of whole")
    ap.add_argument("--metrics", default=None, metavar="JSONL",
                    help="after the timed steps, step shot 0 of the headline state --metrics-steps more steps "
                         "one at a time and write one JSON line per step: bonds, largest pre-truncation bond "
                         "and FP64 tail sum per rounding, Jacobi sweeps, sketches and fallbacks, the leading "
                         "singular values of the middle bond (not part of the timed region)")
    ap.add_argument("--metrics-steps", type=int, default=20)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (byte-counter calibration)")
    ap.add_argument("--velocity-cores", default=None, metavar="NPZ",
                    help="c^2 operator as saved cores (bonds, flat cores; for C4 bonds_<n>, cores_<n> per grid) "
                         "instead of the device's TT-SVD of the model")
    ap.add_argument("--forms", default="fp32,learned",
                    help="comma-separated extra forms timed beside the headline one on the same workload and "
                         "batch: fp32, bf16 (contraction precision), learned (rank network + range finder), "
                         "previous (range finder at the previous step's ranks), chosen (all of fp32 + learned), "
                         "bf16l (bf16 + learned); "
                         "empty for none")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(shots are independent and would be partitioned across GPUs by the caller)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration(torch)
        return

    from paper_2609_01904_amd import mpsw
    import synth

    if args.trajectory:
        if args.workload == "C4":
            mixed_trajectory(mpsw, synth, torch, args)
        else:
            precision_trajectory(mpsw, synth, torch, args)
        return
    if args.workload == "C4":
        mixed_batch(mpsw, synth, torch, args)
        return

    velocity = load_velocity_cores(args.velocity_cores) if args.velocity_cores else None
    model = None
    if args.rank == "learned" or any(f in ("learned", "chosen", "bf16l") for f in args.forms.split(",")):
        t0 = time.perf_counter()
        model, nrows = train_rank_model(mpsw, synth)
        log(f"rank network trained on {nrows} logged bonds in {time.perf_counter() - t0:.1f} s")
    st, cfg, fields, head, kclass, prof = run_form(mpsw, synth, torch, args, args.batch, args.precision, args.rank,
                                                   model if args.rank == "learned" else None, velocity,
                                                   kclass=args.kernel_class)
    el_prof = head["ms_per_step"] * args.steps * 1e-3
    if args.metrics:
        write_metrics(st, args.metrics, args.metrics_steps)
    free, total = torch.cuda.mem_get_info()
    log(f"bonds {st.bonds(0, 0)}; c^2 bonds {st.bonds(0, 2)}; "
        f"device memory in use {(total - free) / 2**30:.1f} of {total / 2**30:.0f} GiB")
    if args.graph:   # events cannot sit inside graphs: the eager timed region above carries the roofline
        st.set_graph_mode(True)
        st.step(3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st.step(args.steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        head.update(value=args.batch * args.steps / el, per_shot_steps_per_s=args.steps / el,
                    ms_per_step=el * 1e3 / args.steps)
        st.set_graph_mode(False)
    avg_ms = prof["total_ms"] / max(prof["launches"], 1)
    flops_per_launch = prof["alg_flops"] / max(prof["launches"], 1)
    achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
    # counters were taken on the sequential site order only
    traffic = read_traffic(kclass, args.workload, args.batch, args.precision) if args.ordering == "sequential" else None
    # contractions run on the matrix cores (dense peak of their operand type);
    # the factorisation kernels on the FP64 vector ALUs
    if KERNEL_NAMES[kclass] == "k_gemm":
        bound, peak = "mfma", {"fp64": PEAK_FP64_TFLOPS, "fp32": 157.3, "bf16": 2500.0}[args.precision]
    else:
        bound, peak = "alu", PEAK_FP64_TFLOPS
    roofline = {"bound": bound, "achieved": achieved,
                "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": traffic, "kernel": KERNEL_NAMES[kclass], "launches": prof["launches"],
                "avg_launch_ms": avg_ms, "alg_flops_per_launch": flops_per_launch,
                "share_of_step_time": prof["total_ms"] / (el_prof * 1e3)}
    out = {
        "metric": "MPS FDTD steps/sec at n=10, chi=128 (chosen vs plain FP64) at stated rel-L2 err",
        "value": head["value"], "unit": "shot-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: n={cfg['n']} ({'x'.join([str(1 << cfg['n'])] * cfg['ndim'])}), chi_max={cfg['chi']}, "
                               f"eps={cfg['eps']}, layered-fault c^2 (cutoff {cfg['eps_c']}), "
                               f"start from a developed wavefield at the chi cap",
                   "shots": args.batch, "precision": args.precision, "site_order": args.ordering,
                   "rank": head["rank"], "graph": bool(args.graph), "tuned": head["tuned"]},
        "per_shot_steps_per_s": head["per_shot_steps_per_s"],
        "roofline": roofline,
    }
    st.close()
    forms = {}
    for f in [x for x in args.forms.split(",") if x]:
        prec = {"fp32": "fp32", "bf16": "bf16", "chosen": "fp32", "bf16l": "bf16"}.get(f, args.precision)
        rank = "learned" if f in ("learned", "chosen", "bf16l") else "previous" if f == "previous" else args.rank
        fs, _, _, res, _, _ = run_form(mpsw, synth, torch, args, args.batch, prec, rank,
                                       model if rank == "learned" else None, velocity)
        fs.close()
        forms[f] = res
    if forms:
        out["forms"] = forms
    if not args.no_plain:
        # plain form: one shot, FP64 contractions, exact SVD, from shot 0's start
        pl, _, _, res, _, _ = run_form(mpsw, synth, torch, args, 1, "fp64", "exact", None, velocity)
        pl.close()
        out["plain_fp64"] = res
        out["speedup_vs_plain"] = head["value"] / res["value"]
    acc = accuracy_summary()
    if acc is not None:
        out["rel_l2_vs_fp64_oracle"] = acc
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(synth, args.workload, fields, args.cpu_seconds, args.ordering)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
