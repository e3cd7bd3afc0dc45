"""Seeded Poisson request arrivals for the serving workload."""
import numpy as np


def poisson_arrivals(seed, rate_per_s, n):
    """Arrival times in seconds of n requests of a Poisson process."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))
