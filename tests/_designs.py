"""Small seeded designs used by the oracle pins and the GPU parity tests."""
import numpy as np

import workloads


def tiny(family, T, m, d, order=2, adaptive=False, seed=0, xi=1e-3, profile=True, rank=None):
    rng = np.random.default_rng(seed)
    gen = workloads.random_dseq_gen(rng, d) if family == "dseq" else workloads.random_lattice_gen(rng, d)
    shift = workloads.random_shifts(rng, T, d)
    s = T if rank is None else rank
    theta = dict(tau=rng.normal(size=T), gamma=float(np.exp(rng.uniform(-0.5, 0.5))),
                 eta=np.exp(rng.uniform(np.log(0.3), np.log(3.0), size=d)),
                 b=workloads.adaptive_b(rng) if adaptive else None,
                 xi=xi * np.exp(rng.uniform(-0.5, 0.5, size=T)),
                 B=rng.normal(0, 0.7, size=(T, s)), zeta=np.exp(rng.uniform(-2.5, -1.0, size=T)))
    m = list(m) if hasattr(m, "__len__") else [m] * T
    return workloads.Workload(f"tiny_{family}_T{T}_m{m}_d{d}_o{order}{'a' if adaptive else ''}",
                              family, T, d, m, order, adaptive, gen, shift, theta, profile, seed,
                              "corr_sines", workloads._corr_sine_params(rng, T, d), 1e-4, 64)
