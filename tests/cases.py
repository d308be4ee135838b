"""Seeded test inputs shared by the GPU parity tests and the host-emulation
tests (inputs only; no processing)."""
import numpy as np

import synth


def tiny_cluster_case(seed):
    """The random event-mode clustering case of a seed: events on a small
    grid with frequent neighbours, repeats and shot boundaries, a radius and a
    time window."""
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(1, 300))
    ev = synth.tiny_events(rng, n, grid=int(rng.integers(2, 12)), t_span=int(rng.integers(0, 800)),
                           n_shots=int(rng.integers(1, 5)), sort_by_shot=bool(seed % 2))
    dxy = int(rng.integers(0, 4))
    dt = int(rng.choice([0, 1, 64, 128, 500]))
    return ev, dxy, dt
