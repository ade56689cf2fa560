"""Seeded complex test vectors for matrix-vector products."""

from __future__ import annotations

import numpy as np


def random_current(n: int, nrhs: int = 1, seed: int = 7) -> np.ndarray:
    """x = (a + j b)/sqrt(2), a, b ~ N(0, 1), from ``default_rng(seed)``.

    Shape (nrhs, n), complex128 (each row one right-hand side)."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((nrhs, n))
    b = rng.standard_normal((nrhs, n))
    return (a + 1j * b) / np.sqrt(2.0)
