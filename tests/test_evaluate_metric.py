"""The product's error metric (evaluate.displacement_error, Section 5:
relative displacement error and the paper's position error, summed over
recorded steps and particles) against the oracle's accumulator on the same
arrays, plus its invariants.  Runs on CPU tensors (the metric is a host-side
reduction over decoded positions)."""
import numpy as np
import torch

from oracle import rom as OR
from paper_2109_12390_amd import evaluate


def _trajectories(seed, steps=4, P=300, d=3):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0.2, 0.8, size=(P, d)).astype(np.float32)
    fom = [X + 0.05 * k * rng.standard_normal((P, d)).astype(np.float32) for k in range(steps)]
    rom = [x + 1e-3 * rng.standard_normal((P, d)).astype(np.float32) for x in fom]
    return X, fom, rom


def test_displacement_error_matches_oracle_accumulator():
    X, fom, rom = _trajectories(1)
    acc = OR.ErrorAccumulator()
    for a, b in zip(rom, fom):
        acc.add(a, b, X)
    # the product takes (d, P) device-layout tensors
    T = lambda a: torch.tensor(np.ascontiguousarray(a.T))
    e_u, e_pos = evaluate.displacement_error([T(a) for a in rom], [T(b) for b in fom], X)
    np.testing.assert_allclose(e_u, acc.displacement_relative(), rtol=1e-12)
    np.testing.assert_allclose(e_pos, acc.position_percent(), rtol=1e-12)


def test_displacement_error_invariants():
    """Zero for identical trajectories; invariant under a common rescaling
    of all displacements (about the reference positions)."""
    X, fom, rom = _trajectories(2)
    T = lambda a: torch.tensor(np.ascontiguousarray(a.T), dtype=torch.float64)
    e0, p0 = evaluate.displacement_error([T(b) for b in fom], [T(b) for b in fom], X)
    assert e0 == 0.0 and p0 == 0.0
    Xd = X.astype(np.float64)
    e1, _ = evaluate.displacement_error([T(a) for a in rom], [T(b) for b in fom], X)
    e2, _ = evaluate.displacement_error([T(Xd + 3.0 * (a - Xd)) for a in rom],
                                        [T(Xd + 3.0 * (b - Xd)) for b in fom], X)
    np.testing.assert_allclose(e1, e2, rtol=1e-6)
