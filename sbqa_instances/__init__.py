"""Seeded synthetic Ising instances and initial states.

This module only draws random numbers and arranges them into arrays. It holds
none of the SBQA arithmetic, so both the FP64 oracle tests and the GPU path can
take their inputs from it without sharing any of the method's code.

Instance families stand in for the paper's (whose data are not available):

* ``sk_pm1``          dense Sherrington-Kirkpatrick couplings J_ij = +-1 (fair coin
                      for i<j), symmetric, zero diagonal; dense all-to-all problems
                      such as the Wishart instance of Sec. II.B.
* ``regular_graph`` + ``gaussian_edges``  random d-regular graphs with N(0,1) edge
                      weights; the sparse, rugged families of Sec. III (cubic
                      lattices have degree 6).
* ``dense_gaussian``  dense J_ij ~ N(0,1), real-valued couplings.

Coupling convention everywhere: J is symmetric with a zero diagonal, stored
row-major as float64 (dense) or as CSR (row_ptr int32[N+1], col int32[nnz]
sorted within each row, val float64[nnz]) with every edge present twice.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "sk_pm1", "dense_gaussian", "regular_graph", "gaussian_edges",
    "edges_to_csr", "csr_to_dense", "dense_to_csr", "gaussian_fields",
    "uniform_state", "spins_pm1",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def sk_pm1(N: int, seed: int) -> np.ndarray:
    """Dense SK couplings: J_ij = J_ji uniform in {-1,+1} for i<j, J_ii = 0."""
    rng = _rng(seed)
    J = np.zeros((N, N), dtype=np.float64)
    iu = np.triu_indices(N, k=1)
    J[iu] = rng.integers(0, 2, size=iu[0].size) * 2.0 - 1.0
    return J + J.T


def dense_gaussian(N: int, seed: int) -> np.ndarray:
    """Dense real couplings: J_ij = J_ji ~ N(0,1) for i<j, J_ii = 0."""
    rng = _rng(seed)
    J = np.zeros((N, N), dtype=np.float64)
    iu = np.triu_indices(N, k=1)
    J[iu] = rng.standard_normal(iu[0].size)
    return J + J.T


def regular_graph(N: int, d: int, seed: int, max_restarts: int = 100) -> np.ndarray:
    """Uniform-ish random simple d-regular graph on N vertices.

    Pairing (configuration) model in the Steger-Wormald form: N*d stubs are
    paired one random pair at a time, pairs that would form a loop or a
    repeated edge are redrawn, and the whole pairing restarts if no valid
    pair remains. Returns an int64 array of shape (N*d/2, 2) with u < v.
    """
    if (N * d) % 2 or d >= N:
        raise ValueError("need N*d even and d < N")
    rng = _rng(seed)
    for _ in range(max_restarts):
        stubs = np.repeat(np.arange(N), d)
        rng.shuffle(stubs)
        stubs = list(stubs)
        adj = [set() for _ in range(N)]
        edges = []
        ok = True
        while stubs:
            placed = False
            for _try in range(64):
                a = int(rng.integers(len(stubs)))
                b = int(rng.integers(len(stubs)))
                if a == b:
                    continue
                u, v = stubs[a], stubs[b]
                if u == v or v in adj[u]:
                    continue
                adj[u].add(v)
                adj[v].add(u)
                edges.append((min(u, v), max(u, v)))
                for idx in sorted((a, b), reverse=True):
                    stubs[idx] = stubs[-1]
                    stubs.pop()
                placed = True
                break
            if not placed:
                # exhaustive check before giving up on this pairing
                found = None
                for a in range(len(stubs)):
                    for b in range(a + 1, len(stubs)):
                        u, v = stubs[a], stubs[b]
                        if u != v and v not in adj[u]:
                            found = (a, b)
                            break
                    if found:
                        break
                if found is None:
                    ok = False
                    break
                a, b = found
                u, v = stubs[a], stubs[b]
                adj[u].add(v)
                adj[v].add(u)
                edges.append((min(u, v), max(u, v)))
                for idx in (b, a):
                    stubs[idx] = stubs[-1]
                    stubs.pop()
        if ok:
            return np.asarray(sorted(edges), dtype=np.int64)
    raise RuntimeError("could not build a simple regular graph")


def gaussian_edges(n_edges: int, seed: int) -> np.ndarray:
    """Edge weights J_e ~ N(0,1)."""
    return _rng(seed).standard_normal(n_edges)


def edges_to_csr(N: int, edges: np.ndarray, w: np.ndarray):
    """Symmetric CSR (both directions stored), columns ascending per row."""
    u = np.concatenate([edges[:, 0], edges[:, 1]])
    v = np.concatenate([edges[:, 1], edges[:, 0]])
    ww = np.concatenate([w, w]).astype(np.float64)
    order = np.lexsort((v, u))
    u, v, ww = u[order], v[order], ww[order]
    row_ptr = np.zeros(N + 1, dtype=np.int32)
    np.add.at(row_ptr, u + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    return row_ptr, v.astype(np.int32), ww


def csr_to_dense(N: int, row_ptr, col, val) -> np.ndarray:
    J = np.zeros((N, N), dtype=np.float64)
    for i in range(N):
        for p in range(row_ptr[i], row_ptr[i + 1]):
            J[i, col[p]] += val[p]
    return J


def dense_to_csr(J: np.ndarray):
    N = J.shape[0]
    row_ptr = np.zeros(N + 1, dtype=np.int32)
    cols, vals = [], []
    for i in range(N):
        nz = np.nonzero(J[i])[0]
        cols.append(nz)
        vals.append(J[i, nz])
        row_ptr[i + 1] = row_ptr[i] + nz.size
    col = np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, np.int32)
    val = np.concatenate(vals).astype(np.float64) if vals else np.zeros(0)
    return row_ptr, col, val


def gaussian_fields(N: int, sigma: float, seed: int) -> np.ndarray:
    """h_i ~ N(0, sigma^2)."""
    return _rng(seed).standard_normal(N) * sigma


def uniform_state(N: int, C: int, amp: float, seed: int):
    """Initial positions and momenta X, Y ~ U[-amp, amp], float32, shape (N, C).

    Column c = r*R + k holds replica k of run r. Values are drawn in float64
    and rounded once to float32 so that both sides start from identical bits.
    """
    rng = _rng(seed)
    X = rng.uniform(-amp, amp, size=(N, C)).astype(np.float32)
    Y = rng.uniform(-amp, amp, size=(N, C)).astype(np.float32)
    return X, Y


def spins_pm1(count: int, N: int, seed: int) -> np.ndarray:
    """Random spin configurations in {-1,+1}, int8, shape (count, N)."""
    return (_rng(seed).integers(0, 2, size=(count, N)) * 2 - 1).astype(np.int8)
