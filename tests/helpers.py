"""Shared test utilities: seeded random trains and densification."""
import numpy as np

from oracle import qtt as Q


def random_tt(rng, dims, ranks, batch=1):
    """Batch of random complex trains; cores (B, r0, d, r1)."""
    cores = []
    for k, d in enumerate(dims):
        shp = (batch, ranks[k], d, ranks[k + 1])
        cores.append((rng.standard_normal(shp) + 1j * rng.standard_normal(shp)) / np.sqrt(d * ranks[k + 1]))
    return cores


def batch_element(cores, b):
    return [c[b] for c in cores]


def dense(cores, b=0):
    return Q.tt_full(batch_element(cores, b))


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))
