"""ctypes binding of libmpsw (argument marshalling only).

Every computation happens in the HIP library; this module converts Python and
NumPy (or torch) arguments into the C ABI declared in include/mpsw.h and turns
error codes into exceptions.  It fails loudly when the library is not built.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpsw.so")

MPSW_FP64, MPSW_FP32, MPSW_BF16 = 0, 1, 2
MPSW_PERIODIC, MPSW_OPEN = 0, 1
MPSW_RANK_EXACT, MPSW_RANK_LEARNED, MPSW_RANK_PREVIOUS = 0, 1, 2
MPSW_SEQUENTIAL, MPSW_INTERLEAVED = 0, 1
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ESTATE", -5: "ECFL", -6: "ENONFINITE"}

EXPORTS = [
    "mpsw_create_state", "mpsw_create_batch", "mpsw_create_batch_ex", "mpsw_get_cores", "mpsw_set_cores", "mpsw_set_velocity_dense", "mpsw_set_velocity_mpo",
    "mpsw_set_source", "mpsw_set_fields", "mpsw_step", "mpsw_to_dense", "mpsw_get_bonds",
    "mpsw_get_stats", "mpsw_get_shape", "mpsw_destroy", "mpsw_last_error", "mpsw_debug_laplacian_mpo",
    "mpsw_debug_factor", "mpsw_profile", "mpsw_profile_read", "mpsw_set_graph_mode",
    "mpsw_group_create", "mpsw_group_step", "mpsw_group_destroy", "mpsw_mlp_grad", "mpsw_mlp_train",
    "mpsw_mlp_forward", "mpsw_mlp_init", "mpsw_mlp_grad_noalloc", "mpsw_rank_model_set", "mpsw_get_rank_features", "mpsw_debug_rank_plan", "mpsw_debug_sketch_normals", "mpsw_debug_sketch", "mpsw_get_sigma_log", "mpsw_autotune", "mpsw_set_launch_shapes", "mpsw_set_source_3d",
]
MLP_NPARAM = 21121
MLP_NIN = 34

KC_QR, KC_JACOBI, KC_GEMM, KC_APPLYQ, KC_APPLYV = 0, 1, 2, 3, 4
KC_NAMES = {KC_QR: "qr", KC_JACOBI: "jacobi", KC_GEMM: "gemm", KC_APPLYQ: "applyq", KC_APPLYV: "applyv"}


class MpswError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class Config(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("chi_max", ctypes.c_int), ("eps", ctypes.c_double),
                ("lambda_", ctypes.c_double), ("precision", ctypes.c_int), ("boundary", ctypes.c_int),
                ("rank_mode", ctypes.c_int), ("seed", ctypes.c_uint64), ("ordering", ctypes.c_int),
                ("ndim", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("nsites", ctypes.c_int), ("bonds", ctypes.c_int * 64),
                ("max_exact_bond", ctypes.c_int * 3), ("tail2", ctypes.c_double * 3),
                ("fallbacks", ctypes.c_int64), ("max_jacobi_sweeps", ctypes.c_int), ("sketches", ctypes.c_int64)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


class TorchAllocator:
    """Device memory for a state from torch's caching allocator: each block the
    library asks for is a uint8 tensor kept alive until the library frees it."""

    def __init__(self, device="cuda"):
        import torch
        self.blocks = {}

        def _alloc(nbytes, ctx):
            try:
                t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
            except RuntimeError:
                return None
            self.blocks[t.data_ptr()] = t
            return t.data_ptr()

        def _free(ptr, nbytes, ctx):
            self.blocks.pop(ptr, None)

        self._fns = (ALLOC_FN(_alloc), FREE_FN(_free))   # the callbacks must outlive the state
        self.struct = Allocator(self._fns[0], self._fns[1], None)

    def bytes_held(self):
        return sum(t.numel() for t in self.blocks.values())


class KProf(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("total_ms", ctypes.c_double), ("alg_flops", ctypes.c_double)]


_lib = None


def load():
    """The loaded library; raises if libmpsw.so has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libmpsw.so not found at {LIB_PATH}: run __graft_entry__.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.mpsw_last_error.restype = ctypes.c_char_p
    sig = {
        "mpsw_create_state": [ctypes.POINTER(Config), P, ctypes.POINTER(P)],
        "mpsw_create_batch": [ctypes.POINTER(Config), I, P, ctypes.POINTER(P)],
        "mpsw_create_batch_ex": [ctypes.POINTER(Config), I, P, ctypes.POINTER(Allocator), ctypes.POINTER(P)],
        "mpsw_get_cores": [P, I, I, P, P, ctypes.c_int64],
        "mpsw_set_cores": [P, I, ctypes.c_int64, P, P, P, P],
        "mpsw_set_velocity_dense": [P, P, D],
        "mpsw_set_velocity_mpo": [P, P, P],
        "mpsw_set_source": [P, I, I, I, I, P],
        "mpsw_set_fields": [P, I, P, P],
        "mpsw_step": [P, I],
        "mpsw_to_dense": [P, I, I, P, I],
        "mpsw_get_bonds": [P, I, I, P],
        "mpsw_get_stats": [P, I, ctypes.POINTER(Stats)],
        "mpsw_get_shape": [P, ctypes.POINTER(I), ctypes.POINTER(I)],
        "mpsw_destroy": [P],
        "mpsw_debug_laplacian_mpo": [I, I, I, I, P, P, ctypes.c_int64],
        "mpsw_set_source_3d": [P, I, I, I, I, I, P],
        "mpsw_debug_factor": [I, I, I, P, P, P],
        "mpsw_profile": [P, I],
        "mpsw_set_graph_mode": [P, I],
        "mpsw_group_create": [ctypes.POINTER(P), I, P, ctypes.POINTER(P)],
        "mpsw_group_step": [P, I],
        "mpsw_group_destroy": [P],
        "mpsw_mlp_grad": [P, P, I, ctypes.c_float, P, P, P],
        "mpsw_mlp_train": [P, P, I, I, ctypes.c_float, ctypes.c_float, P],
        "mpsw_mlp_forward": [P, I, P, P],
        "mpsw_mlp_init": [ctypes.c_uint64, P],
        "mpsw_mlp_grad_noalloc": [P, P, I, ctypes.c_float, P, P, P, P],
        "mpsw_get_rank_features": [P, I, I, P],
        "mpsw_debug_rank_plan": [P, I, I, P, P],
        "mpsw_debug_sketch_normals": [ctypes.c_uint64, I, I, I, I, I, P],
        "mpsw_debug_sketch": [P, I, I, I, D, I, ctypes.c_uint64, I, I, I, P, P, P, P],
        "mpsw_rank_model_set": [P, P, I],
        "mpsw_get_sigma_log": [P, I, I, P],
        "mpsw_autotune": [P, I, ctypes.POINTER(I), ctypes.POINTER(I)],
        "mpsw_set_launch_shapes": [P, I, I],
        "mpsw_profile_read": [P, I, ctypes.POINTER(KProf)],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = I
    _lib = lib
    return lib


def _check(rc):
    if rc < 0:
        msg = load().mpsw_last_error().decode(errors="replace")
        raise MpswError(rc, msg)
    return rc


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def make_config(n, chi_max, eps, lam, precision=MPSW_FP64, boundary=MPSW_PERIODIC,
                rank_mode=MPSW_RANK_EXACT, seed=0, ordering=MPSW_SEQUENTIAL, ndim=2):
    return Config(n, chi_max, eps, lam, precision, boundary, rank_mode, seed, ordering, ndim)


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)   # torch.cuda.Stream


class State:
    """One shot (cfg is a Config) or a batch (cfg is a list of Configs)."""

    def __init__(self, cfg, stream=None, allocator=None):
        lib = load()
        self._h = ctypes.c_void_p()
        self.allocator = allocator   # kept alive as long as the state
        if allocator is not None:
            cfgs = list(cfg) if isinstance(cfg, (list, tuple)) else [cfg]
            arr = (Config * len(cfgs))(*cfgs)
            _check(lib.mpsw_create_batch_ex(arr, len(cfgs), _stream_handle(stream), ctypes.byref(allocator.struct),
                                            ctypes.byref(self._h)))
            self.n, self.ndim = cfgs[0].n, cfgs[0].ndim or 2
        elif isinstance(cfg, (list, tuple)):
            arr = (Config * len(cfg))(*cfg)
            _check(lib.mpsw_create_batch(arr, len(cfg), _stream_handle(stream), ctypes.byref(self._h)))
            self.n, self.ndim = cfg[0].n, cfg[0].ndim or 2
        else:
            _check(lib.mpsw_create_state(ctypes.byref(cfg), _stream_handle(stream), ctypes.byref(self._h)))
            self.n, self.ndim = cfg.n, cfg.ndim or 2
        nshots, nsites = ctypes.c_int(), ctypes.c_int()
        _check(lib.mpsw_get_shape(self._h, ctypes.byref(nshots), ctypes.byref(nsites)))
        self.nshots, self.K = nshots.value, nsites.value

    def close(self):
        if self._h:
            load().mpsw_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_velocity_dense(self, c2, eps_c):
        a, p = _f64(c2)
        _check(load().mpsw_set_velocity_dense(self._h, p, float(eps_c)))

    def set_velocity_mpo(self, bonds, cores):
        b = np.ascontiguousarray(bonds, dtype=np.int32)
        c, p = _f64(np.concatenate([np.ravel(x) for x in cores]))
        _check(load().mpsw_set_velocity_mpo(self._h, b.ctypes.data_as(ctypes.c_void_p), p))

    def set_source(self, shot, ix, iz, wavelet):
        w, p = _f64(wavelet)
        _check(load().mpsw_set_source(self._h, shot, ix, iz, w.size, p))

    def set_source_3d(self, shot, ix, iy, iz, wavelet):
        w, p = _f64(wavelet)
        _check(load().mpsw_set_source_3d(self._h, shot, ix, iy, iz, w.size, p))

    def set_fields(self, shot, u_prev, u_cur):
        args = []
        keep = []
        for u in (u_prev, u_cur):
            if u is None:
                args.append(None)
            else:
                a, p = _f64(u)
                keep.append(a)
                args.append(p)
        _check(load().mpsw_set_fields(self._h, shot, args[0], args[1]))

    def get_cores(self, shot=0, which=0):
        """(bonds, [core_k of shape (b_k, 2, b_{k+1})]) of psi^k (which 0) or psi^{k-1} (1)."""
        lib = load()
        b = np.zeros(self.K + 1, dtype=np.int32)
        tot = _check(lib.mpsw_get_cores(self._h, shot, which, b.ctypes.data_as(ctypes.c_void_p), None, 0))
        buf = np.zeros(max(tot, 1))
        _check(lib.mpsw_get_cores(self._h, shot, which, b.ctypes.data_as(ctypes.c_void_p),
                                  buf.ctypes.data_as(ctypes.c_void_p), buf.size))
        cores, o = [], 0
        for k in range(self.K):
            sz = int(b[k]) * 2 * int(b[k + 1])
            cores.append(buf[o:o + sz].reshape(int(b[k]), 2, int(b[k + 1])))
            o += sz
        return [int(x) for x in b], cores

    def set_cores(self, shot, step, prev, cur):
        """Resume from a checkpoint: prev and cur are (bonds, cores) of psi^{k-1} and psi^k."""
        args = []
        keep = []
        for bonds, cores in (prev, cur):
            bb = np.ascontiguousarray(bonds, dtype=np.int32)
            cc, pc = _f64(np.concatenate([np.ravel(x) for x in cores]))
            keep += [bb, cc]
            args += [bb.ctypes.data_as(ctypes.c_void_p), pc]
        _check(load().mpsw_set_cores(self._h, shot, int(step), *args))

    def step(self, k=1):
        _check(load().mpsw_step(self._h, int(k)))

    def to_dense(self, shot=0, which=0, out=None):
        """Dense field as a (2^n,)*ndim float64 array; `out` may be a CUDA torch tensor."""
        N = 1 << self.n
        if out is not None and hasattr(out, "data_ptr"):
            _check(load().mpsw_to_dense(self._h, shot, which, ctypes.c_void_p(out.data_ptr()), 1))
            return out
        a = np.empty((N,) * self.ndim, dtype=np.float64)
        _check(load().mpsw_to_dense(self._h, shot, which, a.ctypes.data_as(ctypes.c_void_p), 0))
        return a

    def bonds(self, shot=0, which=0):
        b = np.zeros(self.K + 1, dtype=np.int32)
        _check(load().mpsw_get_bonds(self._h, shot, which, b.ctypes.data_as(ctypes.c_void_p)))
        return [int(x) for x in b]

    def stats(self, shot=0):
        s = Stats()
        _check(load().mpsw_get_stats(self._h, shot, ctypes.byref(s)))
        return {"step": s.step, "bonds": list(s.bonds[: self.K + 1]),
                "max_exact_bond": list(s.max_exact_bond), "tail2": list(s.tail2),
                "fallbacks": s.fallbacks, "max_jacobi_sweeps": s.max_jacobi_sweeps, "sketches": s.sketches}


    def set_rank_model(self, w):
        """Parameters of the rank network for the learned-rank rounding."""
        w = np.ascontiguousarray(w, dtype=np.float32)
        _check(load().mpsw_rank_model_set(self._h, w.ctypes.data_as(ctypes.c_void_p), int(w.size)))

    def rank_features(self, shot=0, rounding=0):
        """Rank-network inputs of bonds 1..K-1 of one rounding for the coming step ((K-1) x 34)."""
        out = np.zeros((self.K - 1, MLP_NIN), dtype=np.float32)
        _check(load().mpsw_get_rank_features(self._h, shot, rounding, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def debug_rank_plan(self, shot=0, rounding=0):
        """(network outputs, proposed ranks) of bonds 1..K-1 of one rounding for the coming step."""
        o = np.zeros(self.K - 1, dtype=np.float32)
        r = np.zeros(self.K - 1, dtype=np.int32)
        _check(load().mpsw_debug_rank_plan(self._h, shot, rounding, o.ctypes.data_as(ctypes.c_void_p),
                                           r.ctypes.data_as(ctypes.c_void_p)))
        return o, r

    def sigma_log(self, shot=0, rounding=0):
        """Leading 32 singular values of every bond of one rounding in the last step (K x 32)."""
        out = np.zeros((self.K, 32))
        _check(load().mpsw_get_sigma_log(self._h, shot, rounding, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def autotune(self, steps=2):
        """Pick the launch shapes by timing `steps` steps per candidate; the state is restored."""
        q, b = ctypes.c_int(), ctypes.c_int()
        _check(load().mpsw_autotune(self._h, int(steps), ctypes.byref(q), ctypes.byref(b)))
        return q.value, b.value

    def set_launch_shapes(self, qr_nwg, jac_block):
        """Set the launch shapes autotune chooses (QR workgroups per shot, Jacobi block)."""
        _check(load().mpsw_set_launch_shapes(self._h, int(qr_nwg), int(jac_block)))

    def set_graph_mode(self, on=True):
        """Replay captured HIP graphs (three steps per launch) in step()."""
        _check(load().mpsw_set_graph_mode(self._h, 1 if on else 0))

    def profile(self, kclass=-1):
        """Reset the per-class flop counters; time launches of `kclass` with events."""
        _check(load().mpsw_profile(self._h, int(kclass)))

    def profile_read(self, kclass):
        p = KProf()
        _check(load().mpsw_profile_read(self._h, int(kclass), ctypes.byref(p)))
        return {"launches": int(p.launches), "total_ms": float(p.total_ms), "alg_flops": float(p.alg_flops)}


class Group:
    """Several states (any mix of grids) stepped together by one HIP graph."""

    def __init__(self, states, stream=None):
        lib = load()
        self.states = list(states)   # keep the states alive as long as the group
        arr = (ctypes.c_void_p * len(self.states))(*[s._h.value for s in self.states])
        self._h = ctypes.c_void_p()
        _check(lib.mpsw_group_create(arr, len(self.states), _stream_handle(stream), ctypes.byref(self._h)))

    def step(self, k=1):
        _check(load().mpsw_group_step(self._h, int(k)))

    def close(self):
        if self._h:
            load().mpsw_group_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _f32(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def mlp_grad(X, y, w, alpha):
    """(loss, gradient) of the rank network on the GPU."""
    X, px = _f32(X)
    y, py = _f32(y)
    w, pw = _f32(w)
    g = np.zeros(MLP_NPARAM, dtype=np.float32)
    loss = np.zeros(1, dtype=np.float32)
    _check(load().mpsw_mlp_grad(px, py, X.shape[0], float(alpha), pw, g.ctypes.data_as(ctypes.c_void_p),
                                loss.ctypes.data_as(ctypes.c_void_p)))
    return float(loss[0]), g


def mlp_grad_noalloc(X, y, w, grad, loss, alpha, stream=None):
    """Enqueue the rank network's loss and gradient on device tensors (torch,
    CUDA, float32, contiguous): X (m x 34), y (m), w, grad (MLP_NPARAM), loss (1)."""
    for t in (X, y, w, grad, loss):
        if not (t.is_cuda and t.is_contiguous() and str(t.dtype) == "torch.float32"):
            raise ValueError("device float32 contiguous tensors expected")
    P = ctypes.c_void_p
    _check(load().mpsw_mlp_grad_noalloc(P(X.data_ptr()), P(y.data_ptr()), int(X.shape[0]), float(alpha),
                                        P(w.data_ptr()), P(grad.data_ptr()), P(loss.data_ptr()),
                                        _stream_handle(stream)))


def mlp_train(X, y, w, epochs, lr, alpha):
    """Weights after `epochs` full-batch Adam steps on the GPU."""
    X, px = _f32(X)
    y, py = _f32(y)
    w = np.array(w, dtype=np.float32)
    _check(load().mpsw_mlp_train(px, py, X.shape[0], int(epochs), float(lr), float(alpha),
                                 w.ctypes.data_as(ctypes.c_void_p)))
    return w


def mlp_init(seed=0):
    """He-scaled normal initial parameters of the rank network (the library's generator)."""
    w = np.zeros(MLP_NPARAM, dtype=np.float32)
    _check(load().mpsw_mlp_init(int(seed), w.ctypes.data_as(ctypes.c_void_p)))
    return w


def mlp_forward(X, w):
    X, px = _f32(X)
    w, pw = _f32(w)
    out = np.zeros(X.shape[0], dtype=np.float32)
    _check(load().mpsw_mlp_forward(px, X.shape[0], pw, out.ctypes.data_as(ctypes.c_void_p)))
    return out


def debug_laplacian_mpo(n, boundary=MPSW_PERIODIC, ordering=MPSW_SEQUENTIAL, ndim=2):
    """Host-built fused Laplacian MPO cores (list of [wl, wr, 2, 2] arrays)."""
    lib = load()
    K = ndim * n
    bonds = np.zeros(K + 1, dtype=np.int32)
    total = _check(lib.mpsw_debug_laplacian_mpo(n, boundary, ordering, ndim, bonds.ctypes.data_as(ctypes.c_void_p),
                                                None, 0))
    buf = np.zeros(max(total, 1))
    _check(lib.mpsw_debug_laplacian_mpo(n, boundary, ordering, ndim, bonds.ctypes.data_as(ctypes.c_void_p),
                                        buf.ctypes.data_as(ctypes.c_void_p), buf.size))
    cores, o = [], 0
    for k in range(K):
        sz = bonds[k] * bonds[k + 1] * 4
        cores.append(buf[o:o + sz].reshape(bonds[k], bonds[k + 1], 2, 2))
        o += sz
    return [int(b) for b in bonds], cores


def debug_sketch_normals(seed, step, rounding, site, rows, cols):
    """The library's Gaussian test matrix for one sketch key (rows x cols)."""
    out = np.zeros((rows, cols))
    _check(load().mpsw_debug_sketch_normals(int(seed), int(step), int(rounding), int(site), int(rows), int(cols),
                                            out.ctypes.data_as(ctypes.c_void_p)))
    return out


def debug_sketch(A, l, eps, chi, seed, step, rounding, site):
    """Run the library's sketch of one bond matrix: (sigma of B (32), residual,
    discarded sketched sigma^2, largest sketched sigma, kept rank, accepted)."""
    a, p = _f64(A)
    m, n = a.shape
    sig = np.zeros(32)
    st = np.zeros(3)
    r, ok = ctypes.c_int(), ctypes.c_int()
    _check(load().mpsw_debug_sketch(p, m, n, int(l), float(eps), int(chi), int(seed), int(step), int(rounding),
                                    int(site), sig.ctypes.data_as(ctypes.c_void_p), st.ctypes.data_as(ctypes.c_void_p),
                                    ctypes.byref(r), ctypes.byref(ok)))
    return sig, float(st[0]), float(st[1]), float(st[2]), r.value, bool(ok.value)


def debug_factor(op, A):
    """Run the library's QR (op 0) or SVD (op 1) kernels on one matrix."""
    lib = load()
    a, p = _f64(A)
    m, n = a.shape
    big = max(m, n)
    o1 = np.zeros(big * big + m * n)
    o2 = np.zeros(big * big + m * n)
    q = _check(lib.mpsw_debug_factor(op, m, n, p, o1.ctypes.data_as(ctypes.c_void_p),
                                     o2.ctypes.data_as(ctypes.c_void_p)))
    if op == 0:
        return o1[: m * q].reshape(m, q), o2[: q * n].reshape(q, n)
    return o1[: q * n].reshape(q, n), o2[: m * q].reshape(m, q)
