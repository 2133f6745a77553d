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
* ``sidon28_dense``   dense couplings drawn from the Sidon28 set of the QAC
                      benchmarks of Sec. III, scaled by 28 to the integers
                      {+-8, +-13, +-19, +-28}.
* ``square_lattice``, ``cubic_lattice``  periodic lattices (degree 4 and 6) for
                      the large sparse lattice instances of Sec. III.
* ``planted_square``  square-lattice instances with a planted ground state of
                      known energy (frustrated plaquettes, hidden by a gauge), for
                      optimality gaps and time-to-epsilon without a reference
                      solver.
* ``heavy_hex`` + ``hubo_heavy_hex``  native higher-order (3-body) instances on a
                      heavy-hexagon graph, shaped like the HUBO benchmark of
                      Sec. III.B: one set of vertex-disjoint 2-body edges and
                      several sets of vertex-disjoint 3-body paths, weights from
                      a normal, Cauchy or symmetrised Pareto law (the SWAP layers
                      of the original construction are not reproduced).
* ``random_hubo``     small random 2-body + 3-body instances with integer
                      weights (exhaustive checks).

Coupling convention everywhere: J is symmetric with a zero diagonal, stored
row-major as float64 (dense) or as CSR (row_ptr int32[N+1], col int32[nnz]
sorted within each row, val float64[nnz]) with every edge present twice.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "sk_pm1", "dense_gaussian", "sidon28_dense", "SIDON28", "regular_graph", "gaussian_edges",
    "edges_to_csr", "csr_to_dense", "dense_to_csr", "gaussian_fields",
    "uniform_state", "spins_pm1", "square_lattice", "cubic_lattice", "planted_square",
    "heavy_hex", "hubo_heavy_hex", "random_hubo",
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


# Magnitudes of the Sidon28 couplings {8/28, 13/28, 19/28, 1}, times 28.
SIDON28 = (8, 13, 19, 28)


def sidon28_dense(N: int, seed: int) -> np.ndarray:
    """Dense integer couplings: J_ij = J_ji uniform over {+-8, +-13, +-19, +-28}
    for i<j, J_ii = 0 (28 x the Sidon28 set)."""
    rng = _rng(seed)
    J = np.zeros((N, N), dtype=np.float64)
    iu = np.triu_indices(N, k=1)
    mag = np.asarray(SIDON28, dtype=np.float64)[rng.integers(0, 4, size=iu[0].size)]
    J[iu] = mag * (rng.integers(0, 2, size=iu[0].size) * 2.0 - 1.0)
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


def square_lattice(L: int) -> np.ndarray:
    """Edges (u < v) of the periodic L x L square lattice, site x + L*y, L >= 3."""
    if L < 3:
        raise ValueError("periodic square lattice needs L >= 3")
    x, y = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    site = (x + L * y).ravel()
    right = (((x + 1) % L) + L * y).ravel()
    up = (x + L * ((y + 1) % L)).ravel()
    E = np.concatenate([np.stack([site, right], 1), np.stack([site, up], 1)])
    return np.sort(E, axis=1).astype(np.int64)


def cubic_lattice(L: int) -> np.ndarray:
    """Edges (u < v) of the periodic L x L x L simple cubic lattice, site
    x + L*y + L*L*z, L >= 3."""
    if L < 3:
        raise ValueError("periodic cubic lattice needs L >= 3")
    x, y, z = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    site = (x + L * y + L * L * z).ravel()
    nb = [(((x + 1) % L) + L * y + L * L * z).ravel(),
          (x + L * ((y + 1) % L) + L * L * z).ravel(),
          (x + L * y + L * L * ((z + 1) % L)).ravel()]
    E = np.concatenate([np.stack([site, n], 1) for n in nb])
    return np.sort(E, axis=1).astype(np.int64)


def planted_square(L: int, seed: int, p_frustrated: float = 0.5):
    """Periodic L x L square lattice (L even, >= 4) with a planted ground state.

    The faces with x + y even (a checkerboard) cover every bond exactly once.
    Each such plaquette gets integer bond magnitudes in {1, 2, 3}; with
    probability p_frustrated its weakest bond (first minimum) is made
    antiferromagnetic. A frustrated 4-cycle must violate at least one bond and
    at best violates only its weakest one, which is what the all-up state does,
    so all-up minimises every plaquette at once and is a ground state of the
    sum. A random gauge s* (J_uv -> s*_u s*_v J_uv) then hides it.

    Returns (edges (n, 2) int64 with u < v, weights float64, planted spins s*
    int8, E0): E0 is the energy -sum_edges J_uv s_u s_v of s* (Eq. 2 at the
    corners with h = 0), the sum of the plaquette minima."""
    if L < 4 or L % 2:
        raise ValueError("planted_square needs an even L >= 4")
    rng = _rng(seed)
    edges, w = [], []
    E0 = 0.0
    for x in range(L):
        for y in range(L):
            if (x + y) % 2:
                continue
            a, b = x + L * y, (x + 1) % L + L * y
            c, d = (x + 1) % L + L * ((y + 1) % L), x + L * ((y + 1) % L)
            mags = rng.integers(1, 4, size=4).astype(np.float64)
            J = mags.copy()
            if rng.random() < p_frustrated:
                J[int(np.argmin(mags))] *= -1.0
            E0 += -J.sum()
            for (u, v), j in zip(((a, b), (b, c), (c, d), (d, a)), J):
                edges.append((min(u, v), max(u, v)))
                w.append(j)
    edges = np.asarray(edges, dtype=np.int64)
    w = np.asarray(w)
    s = (rng.integers(0, 2, size=L * L) * 2 - 1).astype(np.int8)
    w = w * s[edges[:, 0]] * s[edges[:, 1]]
    return edges, w, s, float(E0)


def heavy_hex(rows: int, cols: int) -> tuple:
    """Heavy-hexagon graph: a brick-wall honeycomb of rows x cols degree-<=3
    sites (horizontal bonds along each row, vertical bonds where row + column
    is even) with one extra degree-2 site on every bond. Returns (N, edges
    (n, 2) int64 with u < v); honeycomb site (i, j) is i*cols + j, the bond
    sites follow in bond order."""
    if rows < 2 or cols < 2:
        raise ValueError("heavy_hex needs rows, cols >= 2")
    site = lambda i, j: i * cols + j
    bonds = [(site(i, j), site(i, j + 1)) for i in range(rows) for j in range(cols - 1)]
    bonds += [(site(i, j), site(i + 1, j)) for i in range(rows - 1) for j in range(cols) if (i + j) % 2 == 0]
    n0 = rows * cols
    E = []
    for q, (u, v) in enumerate(bonds):
        m = n0 + q
        E.append((u, m))
        E.append((v, m))
    E = np.sort(np.asarray(E, dtype=np.int64), axis=1)
    return n0 + len(bonds), E


def _weights(rng, n: int, dist: str) -> np.ndarray:
    if dist == "normal":
        return rng.standard_normal(n)
    if dist == "cauchy":
        return rng.standard_cauchy(n)
    if dist == "pareto":   # symmetrised Pareto: shape 2, scale 1, random sign
        return (1.0 + rng.pareto(2.0, n)) * (rng.integers(0, 2, n) * 2.0 - 1.0)
    if dist == "int":      # integers in {-5..-1, 1..5}
        return rng.integers(1, 6, n) * (rng.integers(0, 2, n) * 2.0 - 1.0)
    raise ValueError("unknown weight law " + dist)


def hubo_heavy_hex(rows: int, cols: int, seed: int, dist: str = "normal", n2_sets: int = 1, n3_sets: int = 6):
    """Native 3-body instance on heavy_hex(rows, cols).

    2-body terms: n2_sets greedy maximal matchings of the edges (each a set of
    vertex-disjoint pairs, drawn in random edge order, later sets among the
    edges not yet taken). 3-body terms: n3_sets sets of vertex-disjoint paths
    l - m - n (m adjacent to both), each set a greedy maximal selection in
    random order, a path used at most once. Weights from `dist` (normal,
    cauchy, pareto, int), one per term.

    Returns (N, edges (n2, 2), w2 (n2,), triples (n3, 3) int64 sorted within
    each triple, K (n3,)); the energy is -sum w2 s_u s_v - sum K s_l s_m s_n
    (the library's sign convention)."""
    rng = _rng(seed)
    N, E = heavy_hex(rows, cols)
    adj = [[] for _ in range(N)]
    for u, v in E:
        adj[u].append(int(v))
        adj[v].append(int(u))
    taken = np.zeros(len(E), dtype=bool)
    pairs = []
    for _ in range(n2_sets):
        used = np.zeros(N, dtype=bool)
        for q in rng.permutation(len(E)):
            u, v = E[q]
            if taken[q] or used[u] or used[v]:
                continue
            taken[q] = used[u] = used[v] = True
            pairs.append((u, v))
    paths = [(a, m, b) for m in range(N) for x, a in enumerate(adj[m]) for b in adj[m][x + 1:]]
    ptaken = np.zeros(len(paths), dtype=bool)
    tris = []
    for _ in range(n3_sets):
        used = np.zeros(N, dtype=bool)
        for q in rng.permutation(len(paths)):
            t = paths[q]
            if ptaken[q] or used[t[0]] or used[t[1]] or used[t[2]]:
                continue
            ptaken[q] = True
            used[list(t)] = True
            tris.append(sorted(t))
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    tris = np.asarray(tris, dtype=np.int64).reshape(-1, 3)
    return N, pairs, _weights(rng, len(pairs), dist), tris, _weights(rng, len(tris), dist)


def random_hubo(N: int, n2: int, n3: int, seed: int):
    """Random instance on N spins: n2 distinct pairs and n3 distinct triples
    (uniform), integer weights in {-5..-1, 1..5}, and integer h in [-2, 2].
    Returns (edges (n2, 2), w2, triples (n3, 3), K, h)."""
    rng = _rng(seed)
    allp = [(u, v) for u in range(N) for v in range(u + 1, N)]
    allt = [(a, b, c) for a in range(N) for b in range(a + 1, N) for c in range(b + 1, N)]
    P = np.asarray([allp[q] for q in rng.choice(len(allp), n2, replace=False)], dtype=np.int64).reshape(-1, 2)
    T = np.asarray([allt[q] for q in rng.choice(len(allt), n3, replace=False)], dtype=np.int64).reshape(-1, 3)
    return P, _weights(rng, n2, "int"), T, _weights(rng, n3, "int"), rng.integers(-2, 3, N).astype(np.float64)
