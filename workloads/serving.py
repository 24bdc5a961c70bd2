"""Seeded request stream of the serving workload.

2,000 requests by default; each picks a cubed-sphere resolution E uniformly
from {16, 32, 64, 128, 256, 512} (N = 6 E^2 from 1,536 to 1,572,864), a kernel
uniformly from {Poisson log, Biot-Savart, 1/|x-y|} and a degree p uniformly
from {6, 8}; its field is a random sum of real harmonics of degree <= 8 with
N(0, 1/(n+1)^2) coefficients (seed 5006, one coefficient vector per request),
weights w = f A.  Arrival times are a Poisson process of a given rate (seed
5005).
"""

import numpy as np

E_CHOICES = (16, 32, 64, 128, 256, 512)
KERNELS = (1, 2, 3)
DEGREES = (6, 8)
FIELD_DEGREE = 8


def request_mix(n, seed_mix=5006, e_choices=E_CHOICES, kernels=KERNELS, degrees=DEGREES):
    """[(E, kernel, p, coefficients[(FIELD_DEGREE+1)^2])] for n requests."""
    rng = np.random.default_rng(seed_mix)
    ncoef = (FIELD_DEGREE + 1) ** 2
    sig = np.concatenate([np.full(2 * k + 1, 1.0 / (k + 1)) for k in range(FIELD_DEGREE + 1)])
    out = []
    for _ in range(n):
        E = int(rng.choice(e_choices))
        k = int(rng.choice(kernels))
        p = int(rng.choice(degrees))
        c = rng.standard_normal(ncoef) * sig
        out.append((E, k, p, c))
    return out


def poisson_arrivals(n, rate, seed=5005):
    """Arrival times (seconds from 0) of a Poisson process with the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))
