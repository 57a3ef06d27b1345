"""Signal extension operators (oracle; test infrastructure only).

Sec. "A few signal extensions": wavelet analysis with a boundary condition is
the zero-boundary analysis of an extended signal, W^dagger = W^dagger_zpd E.
Every extension used here copies samples (each extended sample is one source
sample), so E has 0/1 entries with exactly one 1 per row. Hence

    E^* E = diag(mult),  mult(n) = number of extended samples copied from n,
    E^dagger = diag(1/mult) E^*,   (E^dagger)^* = E diag(1/mult).

That last form is the paper's closed form for the symmetric and periodic
extensions (1/2 on the reflected blocks when N > 2L'), and it yields the 1/3
(and smaller) weights of the N <= 2L' case without special-casing.

Modes (e = extension width on each side, L = filter length, L' = L - 1):
  'zpd'      e = 0: the zero boundary is implicit in the full convolution of
             the zero-boundary core (the software's W_zpd "implicitly contains
             a zero-padded extension"); E = I.
  'sym'      e = L': half-point symmetric, ext[-1-k] = y[k], ext[N+k] = y[N-1-k],
             repeated with period 2N when e > N (block matrix E_sym).
  'per_ext'  e = L': periodic extension ext[i] = y[i mod N] (block matrix E_per).
The critically sampled periodic transform ('per') needs no extension operator;
it is handled in ``oracle.wavelet``.
"""
from __future__ import annotations

import numpy as np

EXT_MODES = ("zpd", "sym", "per_ext")


def ext_width(mode: str, L: int) -> int:
    if mode == "zpd":
        return 0
    if mode in ("sym", "per_ext"):
        return L - 1
    raise ValueError(mode)


def src_index(i: int, N: int, mode: str) -> int:
    """Source sample of extended position i, i in [-e, N+e)."""
    if mode == "sym":
        j = i % (2 * N)
        return j if j < N else 2 * N - 1 - j
    if mode == "per_ext":
        return i % N
    if mode == "zpd":
        if not 0 <= i < N:
            raise IndexError(i)
        return i
    raise ValueError(mode)


def src_map(N: int, e: int, mode: str) -> np.ndarray:
    """src_map[i + e] = source index of extended position i."""
    return np.array([src_index(i, N, mode) for i in range(-e, N + e)], dtype=np.int64)


def multiplicity(N: int, e: int, mode: str) -> np.ndarray:
    """mult(n) = #{i in [-e, N+e) : src(i) = n} = diag(E^* E)."""
    m = np.zeros(N, dtype=np.int64)
    for s in src_map(N, e, mode):
        m[s] += 1
    return m


def matrix(N: int, e: int, mode: str) -> np.ndarray:
    """Explicit (N+2e) x N extension matrix E."""
    E = np.zeros((N + 2 * e, N))
    for row, s in enumerate(src_map(N, e, mode)):
        E[row, s] = 1.0
    return E


def extend(y: np.ndarray, e: int, mode: str, axis: int = -1, weights: str = "ones") -> np.ndarray:
    """E y along ``axis``; with weights='pinv' returns (E^dagger)^* y = E diag(1/mult) y."""
    y = np.moveaxis(np.asarray(y, dtype=np.float64), axis, -1)
    N = y.shape[-1]
    if weights == "pinv":
        y = y / multiplicity(N, e, mode)
    elif weights != "ones":
        raise ValueError(weights)
    out = y[..., src_map(N, e, mode)]
    return np.moveaxis(out, -1, axis)


def fold(v: np.ndarray, N: int, e: int, mode: str, axis: int = -1, weights: str = "pinv") -> np.ndarray:
    """Apply E^* (weights='ones', summing fold) or E^dagger = diag(1/mult) E^*
    (weights='pinv', averaging fold) along ``axis`` to an extended signal."""
    v = np.moveaxis(np.asarray(v, dtype=np.float64), axis, -1)
    if v.shape[-1] != N + 2 * e:
        raise ValueError("extended length mismatch")
    out = np.zeros(v.shape[:-1] + (N,))
    for row, s in enumerate(src_map(N, e, mode)):
        out[..., s] += v[..., row]
    if weights == "pinv":
        out = out / multiplicity(N, e, mode)
    elif weights != "ones":
        raise ValueError(weights)
    return np.moveaxis(out, -1, axis)
