"""Seed discipline for every synthetic input."""
import numpy as np

ROOT_SEED = 10034984
STREAM_ALM, STREAM_PHI, STREAM_SUBSET, STREAM_TARGETS, STREAM_ARRIVALS = 0, 1, 2, 3, 4


def rng(cfg, job, stream):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([ROOT_SEED, cfg, job, stream])))
