"""Training data for the truncation-rank network, logged from a running state.

For every bond k of every rounding j at step t, the input row is built from
the leading singular values of the same bond and rounding at step t-1 (as the
device computes them when it predicts): log10(sigma_i / sigma_1) for i < 32
(-30 where absent), k / K and min(t, 10^4) / 1000.  The label is the rank the
exact truncation rule kept at step t, divided by chi_max.
"""
import numpy as np

NIN, NH = 34, 128
NPARAM = NIN * NH + NH + NH * NH + NH + NH + 1


def features(sigma, k, K, step):
    f = np.full(NIN, -30.0, dtype=np.float64)
    s = np.asarray(sigma, dtype=np.float64)[:32]
    if s.size and s[0] > 0:
        with np.errstate(divide="ignore"):
            v = np.log10(np.where(s > 0, s / s[0], 0.0))
        v[~np.isfinite(v)] = -30.0
        f[:s.size] = np.maximum(v, -30.0)
    f[32] = k / K
    f[33] = min(step, 10000) / 1000.0
    return f


def log_run(st, steps, chi, shot=0):
    """Step an exact-rank state `steps` times and return (X, y) as float32."""
    K = st.K
    X, y, prev = [], [], None
    for t in range(steps):
        st.step(1)
        logs = [st.sigma_log(shot, j) for j in range(3)]
        ranks = [st.bonds(shot, 3), st.bonds(shot, 4), st.bonds(shot, 0)]   # y, w, psi after the step
        if prev is not None:
            for j in range(3):
                for k in range(1, K):
                    X.append(features(prev[j][k], k, K, t))
                    y.append(ranks[j][k] / chi)
        prev = logs
    return np.array(X, dtype=np.float32), np.array(y, dtype=np.float32)


def init_params(seed=0):
    """He-scaled normal weights, zero biases (flat, in the library's order)."""
    rng = np.random.default_rng(seed)
    parts = [rng.standard_normal((NIN, NH)) * np.sqrt(2.0 / NIN), np.zeros(NH),
             rng.standard_normal((NH, NH)) * np.sqrt(2.0 / NH), np.zeros(NH),
             rng.standard_normal(NH) * np.sqrt(1.0 / NH), np.zeros(1)]
    return np.concatenate([np.ravel(p) for p in parts]).astype(np.float32)
