"""Helpers shared by the GPU tests (comparison metrics, samplers)."""
import numpy as np

import synth

SEED = synth.DEFAULT_SEED
FP32_REL_FRO_TOL = 1e-5   # relative Frobenius error bound for float results


def rel_fro(got, ref) -> float:
    ref = np.asarray(ref, dtype=np.float64)
    num = float(np.linalg.norm(np.asarray(got, dtype=np.float64) - ref))
    den = float(np.linalg.norm(ref))
    return num / den if den else num


def sample_entries(n: int, count: int, seed: int = SEED, stream: int = 99):
    """Entries spread over the whole matrix: corners, the ragged last row and
    column, and uniform random positions."""
    g = synth.rng(seed, stream)
    ii = list(g.integers(0, n, count)) + [0, 0, n - 1, n - 1]
    jj = list(g.integers(0, n, count)) + [0, n - 1, 0, n - 1]
    ii += [n - 1] * 8 + list(g.integers(0, n, 8))
    jj += list(g.integers(0, n, 8)) + [n - 1] * 8
    return np.array(ii, dtype=np.int64), np.array(jj, dtype=np.int64)
