"""Shared test helpers: input plumbing between the synthetic generator and the oracle."""
import numpy as np

from paper_2412_01695_amd import synth


def beta_fn(cfg, ik, miller):
    return synth.beta_values(cfg, synth.q_vectors(cfg, ik, miller))


def zero_beta_fn(cfg, ik, miller):
    return np.zeros((cfg.nproj, np.asarray(miller).shape[0]), dtype=np.complex128)


def miller_map(src, dst):
    """Index array p with dst[p[i]] == src[i] (rows are Miller triples)."""
    key = {tuple(int(x) for x in row): i for i, row in enumerate(dst)}
    return np.array([key[tuple(int(x) for x in row)] for row in src], dtype=np.int64)
