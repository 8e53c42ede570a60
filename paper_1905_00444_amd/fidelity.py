"""Noisy simulation by partial path sums (paper Sec. III-C).

The slices of a sliced contraction are the paper's paths: for random circuits they are close
to orthogonal and of equal weight, so summing a fraction f of them yields amplitudes a_f whose
fidelity with the exact ones is about f:
    sum_x Re(a_f(x) conj(a(x))) / sum_x |a(x)|^2  ~  f,   sum_x |a_f(x)|^2 / sum_x |a(x)|^2  ~  f.
The cost falls by 1/f.  The alternative the same section gives, exact amplitudes for a fraction
of the target set, simulates sampling of fidelity (fraction of amplitudes) x (their fidelity).

qf_amplitudes adds over any slice range, so a path subset is one call per run of consecutive
slice ids; everything here is host-side bookkeeping around that call.
"""
from __future__ import annotations

import math
from typing import List, Optional, Sequence, Tuple

import numpy as np


def paths_for_fidelity(n_paths: int, f: float) -> int:
    """Number of paths to sum for target fidelity f (at least one, at most all)."""
    if not 0.0 < f <= 1.0:
        raise ValueError("fidelity must be in (0, 1]")
    return min(n_paths, max(1, math.ceil(f * n_paths)))


def slice_runs(slices: Sequence[int]) -> List[Tuple[int, int]]:
    """Half-open ranges [a, b) covering the given slice ids (sorted, duplicates removed)."""
    runs: List[Tuple[int, int]] = []
    for s in sorted(set(int(x) for x in slices)):
        if runs and runs[-1][1] == s:
            runs[-1] = (runs[-1][0], s + 1)
        else:
            runs.append((s, s + 1))
    return runs


def noisy_amplitudes(plan, bits, f: float, paths: Optional[Sequence[int]] = None, out=None):
    """Amplitudes of fidelity about f: the sum over the first paths_for_fidelity(len(paths), f)
    entries of `paths` (default: all slice ids in order; pass the non-vanishing slices of a
    plan with structurally zero slices so that f counts contributing paths)."""
    if paths is None:
        paths = range(plan.info()["n_slices"])
    paths = list(paths)
    chosen = paths[: paths_for_fidelity(len(paths), f)]
    for a, b in slice_runs(chosen):
        out = plan.amplitudes(bits, a, b, out=out)
    return out


def overlap_fidelity(a_f: np.ndarray, a: np.ndarray) -> float:
    """sum Re(a_f conj(a)) / sum |a|^2 over all given amplitudes."""
    a_f = np.asarray(a_f).reshape(-1)
    a = np.asarray(a).reshape(-1)
    return float(np.sum(np.real(a_f * np.conj(a))) / np.sum(np.abs(a) ** 2))


def norm_fidelity(a_f: np.ndarray, a: np.ndarray) -> float:
    """sum |a_f|^2 / sum |a|^2 over all given amplitudes."""
    return float(np.sum(np.abs(np.asarray(a_f)) ** 2) / np.sum(np.abs(np.asarray(a)) ** 2))


def sampling_fidelity(fraction_of_amplitudes: float, amplitude_fidelity: float) -> float:
    """Fidelity of sampling from a fraction of the target amplitudes computed at a given fidelity."""
    return fraction_of_amplitudes * amplitude_fidelity
