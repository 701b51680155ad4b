"""Seeded batch of Carleman-LBM instances of uneven size (the batched workload).

Instance i draws from numpy.random.default_rng(seed + i): N_x from {8, 16, 32},
N_K from {2, 3, 4}, N_t from {1, 2, 4}, tau ~ U[0.6, 1.2], amplitude ~
U[0.01, 0.1], wavenumber from {1, 2}; u0 = 0 and dt = 0.1.  Qubit counts follow
from the register sizes (21 to 28 qubits).
"""
from __future__ import annotations

import numpy as np

from .carleman_circuit import CarlemanConfig


def batch_configs(count: int = 64, seed: int = 0) -> list[CarlemanConfig]:
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed + i)
        out.append(CarlemanConfig(
            nx=int(rng.choice([8, 16, 32])),
            nk=int(rng.choice([2, 3, 4])),
            nt=int(rng.choice([1, 2, 4])),
            tau=float(rng.uniform(0.6, 1.2)),
            amp=float(rng.uniform(0.01, 0.1)),
            wavenumber=int(rng.choice([1, 2])),
            u0=0.0,
            dt=0.1,
        ))
    return out
