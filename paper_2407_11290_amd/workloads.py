"""Seeded synthetic problem lists shared by the tests and the benchmark.

This module only draws problem descriptions (mode sizes, generating function,
its parameters, seeds, arrival times).  It holds none of the method's
arithmetic, so both the GPU path and the CPU oracle can be driven from it.
"""
from dataclasses import dataclass, field

import numpy as np

FN_HILBERT, FN_BIMAXWELL = 1, 3


@dataclass
class ProblemSpec:
    n: list                 # mode sizes
    fn_id: int
    params: list            # generating-function parameters (C ABI layout)
    eps: float
    seed: int               # the solve's own sample seed
    grid: list = field(default_factory=list)
    arrival_s: float = 0.0  # for served traces

    @property
    def d(self):
        return len(self.n)


def batch_mix(count=512, gen_seed=2024, eps=1e-6, ds=(3, 4, 5, 6), ns=(16, 32, 64, 128)):
    """Mixed batch: d ~ U(ds), one n ~ U(ns) for every mode of a problem.

    Even problems are Hilbert tensors 1/(i_1+..+i_d + c) (1-based i) with
    c ~ U[0, 4]; odd ones are sums of two 3v Maxwellians with rho_m ~ U[0.5, 2],
    u_m ~ U[-2, 2]^3 and T_m ~ U[0.5, 2] (velocity box [-8, 8]).  Problem b uses
    sample seed b.  Modes are split into two subtensor blocks each."""
    rng = np.random.default_rng(gen_seed)
    out = []
    for b in range(count):
        d = int(rng.choice(ds))
        n = int(rng.choice(ns))
        if b % 2 == 0:
            c = float(rng.uniform(0.0, 4.0))
            fn, params = FN_HILBERT, [c]
        else:
            params = []
            for _m in range(2):
                rho = float(rng.uniform(0.5, 2.0))
                u = [float(x) for x in rng.uniform(-2.0, 2.0, 3)]
                T = float(rng.uniform(0.5, 2.0))
                params += [rho, *u, T]
            params.append(8.0)
            fn = FN_BIMAXWELL
        out.append(ProblemSpec(n=[n] * d, fn_id=fn, params=params, eps=eps, seed=b, grid=[2] * d))
    return out


def served_trace(count=2000, trace_seed=7, rate_hz=1000.0, ds=(4, 5, 6), ns=(32, 64, 128, 256),
                 epss=(1e-4, 1e-8)):
    """Served requests with Poisson arrivals at rate_hz: half Hilbert (as in
    batch_mix), half bi-Maxwellian; d ~ U(ds), n ~ U(ns), eps ~ U(epss)."""
    rng = np.random.default_rng(trace_seed)
    t = 0.0
    out = []
    for b in range(count):
        t += float(rng.exponential(1.0 / rate_hz))
        d = int(rng.choice(ds))
        n = int(rng.choice(ns))
        eps = float(rng.choice(epss))
        if rng.uniform() < 0.5:
            fn, params = FN_HILBERT, [float(rng.uniform(0.0, 4.0))]
        else:
            params = []
            for _m in range(2):
                params += [float(rng.uniform(0.5, 2.0)), *[float(x) for x in rng.uniform(-2.0, 2.0, 3)],
                           float(rng.uniform(0.5, 2.0))]
            params.append(8.0)
            fn = FN_BIMAXWELL
        out.append(ProblemSpec(n=[n] * d, fn_id=fn, params=params, eps=eps, seed=b, grid=[2] * d,
                               arrival_s=t))
    return out
