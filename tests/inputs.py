"""Seeded synthetic workloads shared by the oracle tests, the GPU parity tests
and bench.py.  This module holds no decoding arithmetic: only the workload
recipes (code, distance, rounds, noise strength, iteration budget, shot
counts) and the seeds.

The paper evaluates on circuits from an external generator (Sec. III.E);
that tool is not available, so every workload is the project's own rotated
surface code (code capacity) or memory-Z circuit at the same sizes and noise
description, and every syndrome is drawn by the sampler from a seed below.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 0x2603053810000000

# (name, kind, d, rounds, p, max_iters, n_shots)
WORKLOADS = {
    # tiny code-capacity case: d=3, 4 X checks, 9 qubits, q = 2p/3
    "cc_d3": ("code_capacity", 3, 1, 0.05, 50, 10_000),
    # code-capacity sweep points
    "cc_d5_p10": ("code_capacity", 5, 1, 0.10, 25, 1_000_000),
    "cc_d15_p10": ("code_capacity", 15, 1, 0.10, 25, 1_000_000),
    # circuit-level memory-Z, d rounds
    "mz_d5_p005": ("memory_z", 5, 5, 0.005, 50, 1_000_000),
    "mz_d13_p005": ("memory_z", 13, 13, 0.005, 50, 1_000_000),
}


def seed_for(config_index: int, d: int, p: float) -> int:
    """Seed of the sampler for one (config, d, p) point."""
    return (SEED_BASE ^ (config_index << 32) ^ (d << 16) ^ int(round(p * 1e5))) & 0xFFFFFFFFFFFFFFFF


def random_llr_instance(rng: np.random.Generator, s: int, lo: float = -12.0, hi: float = 2.0):
    """A symmetric s x s prior matrix (diagonal = boundary) and integer weights
    that decrease with the prior, for tests that exercise BP without a code."""
    a = rng.uniform(lo, hi, size=(s, s))
    L = np.triu(a) + np.triu(a, 1).T
    W = np.round((hi - L) * 2 ** 20).astype(np.int64) + 1
    return L, W
