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


def tile_samples(m: int, n: int, bm: int, bn: int, count: int, seed: int = SEED, stream: int = 98):
    """At least `count` entries of an m x n result that touch every tile row
    and every tile column of a bm x bn tiling (one random entry inside the
    tile of each pair), plus the four corners."""
    g = synth.rng(seed, stream)
    ntr, ntc = -(-m // bm), -(-n // bn)
    t = np.arange(max(count, ntr, ntc))
    tr, tc = t % ntr, (t + t // ntr) % ntc
    r0, c0 = tr * bm, tc * bn
    ii = r0 + g.integers(0, bm, t.size) % np.maximum(1, np.minimum(bm, m - r0))
    jj = c0 + g.integers(0, bn, t.size) % np.maximum(1, np.minimum(bn, n - c0))
    ii = np.concatenate([ii, [0, 0, m - 1, m - 1]]).astype(np.int64)
    jj = np.concatenate([jj, [0, n - 1, 0, n - 1]]).astype(np.int64)
    return ii, jj
