"""Sensitivity floor of a truncating run (test helper).

The floor at perturbation size delta is the relative L2 distance between two
FP64 oracle runs of the same workload, one of which multiplies every tensor
entering a rounding by (1 + delta g), g standard normal (seeded).  It measures
how far rounding-sized perturbations move the truncated trajectory: no
arithmetic whose unit roundoff is delta can be expected to land closer to the
oracle than about this distance, since every truncation decision near the
cutoff eps sigma_1 is as sensitive to it.
"""
import numpy as np

from oracle import stepper as S


class PerturbedStepper(S.DenseStepper):
    def __init__(self, delta, seed, *args, **kw):
        super().__init__(*args, **kw)
        self.delta = delta
        self.rng = np.random.default_rng(seed)

    def _round(self, t, which):
        if which >= 0 and self.delta > 0:
            t = t * (1.0 + self.delta * self.rng.standard_normal(t.shape))
        return super()._round(t, which)


def run(n, lam, eps, chi, c2, src, wav, steps, delta=0.0, seed=0):
    ds = PerturbedStepper(delta, seed, n, lam, eps, chi, c2, src=src, wavelet=wav)
    for _ in range(steps):
        ds.step()
    return ds.dense()


def floor(n, lam, eps, chi, c2, src, wav, steps, delta, seeds=(0, 1)):
    """Mean over seeds of rel-L2(perturbed run, unperturbed run)."""
    base = run(n, lam, eps, chi, c2, src, wav, steps)
    nb = np.linalg.norm(base)
    return float(np.mean([np.linalg.norm(run(n, lam, eps, chi, c2, src, wav, steps, delta, s) - base) / nb
                          for s in seeds]))
