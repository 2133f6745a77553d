"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it checks (arXiv 2604.01050). None of them
re-types the oracle's update formula: they check hand-computed values,
exhaustive enumeration, Hamilton's equations of the Eq. 4 Hamiltonian, the
transfer matrix behind Eq. S12, special cases that reduce to Eq. 3, exact
symmetries and closed-form linear maps.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import sbqa_instances as inst

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------- energy
def test_energy_hand_fixtures(orc):
    """Hand-computed energies (Eq. 2 at the corners / Eq. S1)."""
    with open(os.path.join(GOLD, "energy_hand.json")) as f:
        cases = json.load(f)["cases"]
    for case in cases:
        J = np.array(case["J"], dtype=float)
        h = np.array(case["h"], dtype=float)
        s = np.array(case["spins"], dtype=np.int8)
        E = orc.energy(s, J=J, h=h)
        assert np.array_equal(E, np.array(case["E"], dtype=float)), case["name"]
        Eg, sg = orc.bruteforce(J, h)
        assert Eg == case["ground_E"], case["name"]
        assert orc.energy(sg[None], J=J, h=h)[0] == Eg


def test_energy_single_flip_identity(orc):
    """Flipping s_i changes E by 2 s_i (sum_j J_ij s_j + h_i): the local-field
    form of the same energy. A dropped 1/2, a wrong sign of h or a transposed
    J all break it."""
    N = 23
    J = inst.dense_gaussian(N, 11)
    J[3, 7] += 0.5  # deliberately asymmetric copy to check row/col handling below
    J = 0.5 * (J + J.T)
    h = inst.gaussian_fields(N, 0.7, 12)
    s = inst.spins_pm1(40, N, 13)
    E0 = orc.energy(s, J=J, h=h)
    for i in (0, 5, N - 1):
        t = s.copy()
        t[:, i] = -t[:, i]
        E1 = orc.energy(t, J=J, h=h)
        local = J[i] @ s.T.astype(float) + h[i]
        np.testing.assert_allclose(E1 - E0, 2.0 * s[:, i] * local, rtol=1e-12, atol=1e-12)


def test_energy_symmetries_and_csr(orc):
    """h = 0: E(s) = E(-s). The linear term is exactly -h.s. Dense == CSR."""
    N = 40
    J = inst.sk_pm1(N, 3)
    s = inst.spins_pm1(16, N, 4)
    assert np.array_equal(orc.energy(s, J=J), orc.energy(-s, J=J))
    h = np.arange(N, dtype=float) - 7.0
    assert np.array_equal(orc.energy(s, J=J, h=h) - orc.energy(s, J=J), -(s.astype(float) @ h))
    csr = inst.dense_to_csr(J)
    assert np.array_equal(orc.energy(s, J=J, h=h), orc.energy(s, csr=csr, h=h))


def test_bruteforce_matches_enumeration(orc):
    """Gray-code search equals a direct enumeration of all 2^N states."""
    for N, seed in ((8, 1), (11, 2)):
        J = inst.dense_gaussian(N, seed)
        h = inst.gaussian_fields(N, 0.3, seed + 100)
        allS = np.array(list(itertools.product((-1, 1), repeat=N)), dtype=np.int8)
        Sf = allS.astype(float)
        Eall = -0.5 * np.einsum("mi,ij,mj->m", Sf, J, Sf) - Sf @ h
        Eg, sg = orc.bruteforce(J, h)
        assert abs(Eg - Eall.min()) < 1e-10
        assert abs(orc.energy(sg[None], J=J, h=h)[0] - Eg) < 1e-10


# ------------------------------------------------------------------ schedule
def test_jperp_transfer_matrix(orc):
    """Eq. S12 from its derivation: with theta = beta Gamma_x / R the single-site
    transfer matrix exp(theta sigma_x) has entries cosh and sinh, and
    exp(a + b s s') reproduces them with b = beta J_perp."""
    scipy_linalg = pytest.importorskip("scipy.linalg")
    sx = np.array([[0.0, 1.0], [1.0, 0.0]])
    for beta, gR in ((0.5, 0.3), (1.0, 1.0), (1.5, 0.01), (0.7, 2.5)):
        theta = beta * gR
        M = scipy_linalg.expm(theta * sx)
        jp = orc.jperp(beta, gR)
        b = beta * jp
        a = 0.5 * math.log(M[0, 0] * M[0, 1])
        # <s|e^{theta sx}|s'> = exp(a + b s s')
        assert math.isclose(math.exp(a + b), M[0, 0], rel_tol=1e-12)
        assert math.isclose(math.exp(a - b), M[0, 1], rel_tol=1e-12)
        # the two printed forms of Eq. S12 agree: ln coth = -ln tanh
        assert math.isclose(jp, math.log(1.0 / math.tanh(theta)) / (2 * beta), rel_tol=1e-12)


def test_jperp_asymptotics_and_invariance(orc):
    """Large theta: J_perp -> exp(-2 theta)/beta; small theta: -ln(theta)/(2 beta).
    Only beta*Gamma_x/R enters, so (Gamma_x(0), R) -> (l Gamma_x(0), l R) is a no-op."""
    beta = 1.3
    th = 6.0   # ln coth = 2 e^{-2th} + O(e^{-6th}); log(tanh) cancels ~1e-16/e^{-12}
    assert math.isclose(orc.jperp(beta, th / beta), math.exp(-2 * th) / beta, rel_tol=1e-8)
    th = 1e-7
    assert math.isclose(orc.jperp(beta, th / beta), -math.log(th) / (2 * beta), rel_tol=1e-6)
    S = 97
    t1 = orc.jperp_paper_table(1.0, 0.8, 8.0 / 8.0, S)       # Gamma_x(0) = 8, R = 8
    t2 = orc.jperp_paper_table(1.0, 0.8, 1.0 / 1.0, S)       # Gamma_x(0) = 1, R = 1
    assert np.array_equal(t1, t2)


def test_gamma_x_regulariser(orc):
    """Eq. 5: Gamma_x(0)[(1 - t/T)^alpha + 1e-5]; finite at t = T, linear for alpha = 1,
    monotone decreasing, so J_perp ramps up during the anneal (Sec. II.B)."""
    assert orc.gamma_x(2.0, 0.7, 1.0) == pytest.approx(2e-5, rel=1e-12)
    assert orc.gamma_x(2.0, 0.7, 0.0) == pytest.approx(2.0 * (1 + 1e-5), rel=1e-15)
    assert orc.gamma_x(1.0, 1.0, 0.25) == pytest.approx(0.75 + 1e-5, rel=1e-15)
    tab = orc.jperp_paper_table(1.0, 0.5, 1.0, 200)
    assert np.all(np.diff(tab) > 0) and np.all(np.isfinite(tab))
    assert orc.pump(0, 10) == 0.0 and orc.pump(5, 10) == 0.5
    # Eq. 8 threshold, delta_max = 0.7, decision precision binary32
    assert orc.delta32(0.7, 5, 10) == np.float32(0.35)
    lin = orc.jperp_linear_table(0.5, 0.0, 4)
    assert np.array_equal(lin, [0.5, 0.375, 0.25, 0.125])


def test_auto_c0_closed_forms(orc):
    """c0 = 0.5/(sqrt(N) std J): SK +-1 has rms 1, so c0 = 0.5/sqrt(N)."""
    assert orc.auto_c0(J=inst.sk_pm1(64, 5)) == pytest.approx(0.0625, rel=1e-15)
    N, d = 512, 6
    E = inst.regular_graph(N, d, 7)
    w = np.full(len(E), 2.0)
    csr = inst.edges_to_csr(N, E, w)
    # rms over N(N-1) off-diagonal entries: sqrt(N d 4 / (N (N-1)))
    assert orc.auto_c0(csr=csr) == pytest.approx(0.5 / (math.sqrt(N) * math.sqrt(4 * d / (N - 1))), rel=1e-14)


# ------------------------------------------------------------- nonlinearity
def test_f_variants(orc):
    """Eq. 8 ternary (0 inside |x| <= Delta, sign outside), dSB sign, bSB identity."""
    x = np.array([-0.9, -0.35, -0.2, 0.0, 0.2, 0.35, 0.3500001, 0.9])
    g = orc.apply_f(orc.F_TERNARY, np.float32(0.35), x)
    assert np.array_equal(g, [-1, 0, 0, 0, 0, 0, 1, 1])
    g = orc.apply_f(orc.F_SIGN, 0.35, x)
    assert np.array_equal(g, [-1, -1, -1, 0, 1, 1, 1, 1])
    assert np.array_equal(orc.apply_f(orc.F_BALLISTIC, 0.35, x), x)


# ------------------------------------------------------------------ dynamics
def _hamiltonian_eq4(J, h, X, Y, a, a0, c0, R, jp):
    """Eq. 4 written out term by term, per run. X, Y are (N, runs*R)."""
    N, C = X.shape
    runs = C // R
    H = np.zeros(runs)
    for r in range(runs):
        q = X[:, r * R:(r + 1) * R]
        p = Y[:, r * R:(r + 1) * R]
        kin = (a0 / (2 * R)) * np.sum(p * p)
        pot = ((a0 - a) / (2 * R)) * np.sum(q * q)
        ising = -(c0 / R) * (np.sum(h[:, None] * q) + 0.5 * np.einsum("ik,ij,jk->", q, J, q))
        ring = -jp[r] * sum(np.sum(q[:, k] * q[:, (k + 1) % R]) for k in range(R))
        H[r] = kin + pot + ising + ring
    return H


@pytest.mark.parametrize("R", [1, 2, 3, 5])
def test_eom_is_hamiltons_equations_of_eq4(orc, R):
    """With f(x) = x (bSB) Eq. 7 must be Hamilton's equations of Eq. 4:
    q' = dH/dp and p' = -dH/dq. The oracle's kick from Y = 0 gives the force
    F = Y'/dt; its drift gives q' = (x' - x)/dt. H is quadratic, so central
    differences are exact up to rounding. Checks every sign, the 1/R factors,
    the 1/2 on the symmetric J sum and the ring (including R <= 2)."""
    N, runs = 6, 2
    rng = np.random.default_rng(R)
    J = inst.dense_gaussian(N, 30 + R)
    h = rng.normal(size=N)
    a0, c0, a, dt = 1.0, 0.37, 0.31, 1e-3
    jp = np.array([0.23, 0.61])
    P = orc.Problem(N, R, runs, J=J, h=h, dt=dt, a0=a0, c0=c0, fmode=orc.F_BALLISTIC)
    X = rng.uniform(-0.2, 0.2, size=(N, R * runs))
    Y0 = np.zeros_like(X)
    X1, Y1 = P.step(X, Y0, a, 0.0, jp)
    force = Y1 / dt
    eps = 1e-4
    grad = np.zeros_like(X)
    for i in range(N):
        for c in range(R * runs):
            Xp, Xm = X.copy(), X.copy()
            Xp[i, c] += eps
            Xm[i, c] -= eps
            r = c // R
            Hp = _hamiltonian_eq4(J, h, Xp, Y0, a, a0, c0, R, jp)[r]
            Hm = _hamiltonian_eq4(J, h, Xm, Y0, a, a0, c0, R, jp)[r]
            grad[i, c] = (Hp - Hm) / (2 * eps)
    np.testing.assert_allclose(force, -grad, rtol=1e-7, atol=1e-9)
    # dH/dp = (a0/R) p: the drift uses the new momentum
    np.testing.assert_allclose((X1 - X) / dt, (a0 / R) * Y1, rtol=1e-9, atol=1e-12)


def test_energy_bounded_without_drift(orc):
    """Frozen a and J_perp, f(x) = x, no wall contact: symplectic Euler keeps the
    Eq. 4 Hamiltonian within O(dt) of its start over 10^4 steps (no secular drift)."""
    N, R, runs = 5, 4, 1
    J = inst.dense_gaussian(N, 77) * 0.3
    h = np.zeros(N)
    a0, c0, a, dt = 1.0, 0.2, 0.2, 0.05
    jp = np.array([0.03])   # stiffness (a0-a)/R - 2 J_perp - c0 |J|/R stays positive
    P = orc.Problem(N, R, runs, J=J, h=h, dt=dt, a0=a0, c0=c0, fmode=orc.F_BALLISTIC)
    rng = np.random.default_rng(5)
    X = rng.uniform(-0.1, 0.1, size=(N, R))
    Y = rng.uniform(-0.1, 0.1, size=(N, R))
    H0 = _hamiltonian_eq4(J, h, X, Y, a, a0, c0, R, jp)[0]
    Hs = []
    for n in range(10000):
        X, Y = P.step(X, Y, a, 0.0, jp)
        assert np.max(np.abs(X)) < 1.0
        if n % 10 == 0:
            Hs.append(_hamiltonian_eq4(J, h, X, Y, a, a0, c0, R, jp)[0])
    Hs = np.array(Hs)
    scale = abs(H0) + np.sum(X * X)
    assert np.max(np.abs(Hs - H0)) < 0.1 * scale
    first, last = Hs[: len(Hs) // 10].mean(), Hs[-len(Hs) // 10:].mean()
    assert abs(last - first) < 0.02 * scale


def test_free_particle_closed_form(orc):
    """N = 1, J = 0, h = 0, J_perp = 0: each step is the linear map
    M_n = [[1 - dt^2 (a0/R)(a0 - a_n)/R, dt a0/R], [-dt (a0 - a_n)/R, 1]],
    det M_n = 1 (symplectic)."""
    for R in (1, 4):
        S, dt, a0 = 300, 0.5, 1.0
        P = orc.Problem(1, R, 1, J=np.zeros((1, 1)), dt=dt, a0=a0, c0=0.1, fmode=orc.F_TERNARY)
        X = np.full((1, R), 0.01)
        Y = np.linspace(-0.01, 0.01, R)[None, :]
        v = np.stack([X[0], Y[0]])
        res = P.run(X, Y, S, np.zeros((1, S)))
        for n in range(S):
            an = n / S
            M = np.array([[1 - dt * dt * (a0 / R) * (a0 - an) / R, dt * a0 / R],
                          [-dt * (a0 - an) / R, 1.0]])
            assert abs(np.linalg.det(M) - 1.0) < 1e-14
            v = M @ v
        assert np.max(np.abs(v[0])) < 1.0
        np.testing.assert_allclose(res["X"][0], v[0], rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(res["Y"][0], v[1], rtol=1e-12, atol=1e-14)


def _sbm_step_eq3(J, h, x, y, a, dt, a0, c0, g):
    """SBM (Eq. 3) for one trajectory, kick then drift then wall; J +-1 so the
    coupling sum is an exact integer whatever the summation order."""
    phi = J @ g
    y = y + dt * (-(a0 - a) * x + c0 * (phi + h))
    x = x + dt * a0 * y
    out = np.abs(x.astype(np.float32)) > 1.0
    x = np.where(out, np.sign(x), x)
    y = np.where(out, 0.0, y)
    return x, y


def test_reduces_to_sbm_when_uncoupled(orc):
    """J_perp = 0 and R = 1: SBQA is SBM Eq. 3 bit-for-bit. With R a power of two
    each column is SBM with the step dt/R (Eqs. 6-7 are Eq. 3 in time t/R), also
    bit-for-bit, since scaling by 2^-m is exact."""
    N, S, dt, a0 = 24, 60, 0.5, 1.0
    J = inst.sk_pm1(N, 21)
    h = np.round(inst.gaussian_fields(N, 1.0, 22) * 8) / 8  # dyadic fields keep phi+h exact
    c0 = 0.5 / math.sqrt(N)
    for R in (1, 4):
        runs = 2
        P = orc.Problem(N, R, runs, J=J, h=h, dt=dt, a0=a0, c0=c0, fmode=orc.F_TERNARY)
        X0, Y0 = inst.uniform_state(N, R * runs, 0.1, 23)
        X, Y = X0.astype(float), Y0.astype(float)
        xs = [X[:, c].copy() for c in range(R * runs)]
        ys = [Y[:, c].copy() for c in range(R * runs)]
        for n in range(S):
            an, dn = orc.pump(n, S), orc.delta32(0.7, n, S)
            X, Y = P.step(X, Y, an, dn, np.zeros(runs))
            for c in range(R * runs):
                g = orc.apply_f(orc.F_TERNARY, dn, xs[c])
                xs[c], ys[c] = _sbm_step_eq3(J, h, xs[c], ys[c], an, dt / R, a0, c0, g)
        for c in range(R * runs):
            assert np.array_equal(X[:, c], xs[c]), (R, c)
            assert np.array_equal(Y[:, c], ys[c]), (R, c)


def test_symmetries_exact(orc):
    """h = 0: negating the start negates the trajectory (f and the wall are odd).
    A cyclic shift or a reflection of replica indices inside a run permutes the
    trajectory (the periodic ring of S1 is symmetric). Permuting runs (with their
    J_perp) permutes results."""
    N, R, runs, S = 20, 5, 3, 40
    J = inst.dense_gaussian(N, 8)
    P = orc.Problem(N, R, runs, J=J, dt=0.5, a0=1.0, c0=0.1, fmode=orc.F_TERNARY)
    X0, Y0 = inst.uniform_state(N, R * runs, 0.1, 9)
    jt = np.stack([orc.jperp_linear_table(0.5, 0.0, S), orc.jperp_paper_table(1.0, 0.7, 1.0, S),
                   orc.jperp_paper_table(0.6, 1.0, 0.5, S)])
    base = P.run(X0, Y0, S, jt)
    neg = P.run(-X0, -Y0, S, jt)
    assert np.array_equal(neg["X"], -base["X"]) and np.array_equal(neg["Y"], -base["Y"])
    assert np.array_equal(neg["best_E"], base["best_E"])
    perm = []
    for r in range(runs):
        perm += [r * R + (k + 2) % R for k in range(R)]      # cyclic shift by 2
    sh = P.run(X0[:, perm], Y0[:, perm], S, jt)
    assert np.array_equal(sh["X"], base["X"][:, perm])
    refl = []
    for r in range(runs):
        refl += [r * R + (R - 1 - k) for k in range(R)]
    rf = P.run(X0[:, refl], Y0[:, refl], S, jt)
    assert np.array_equal(rf["X"], base["X"][:, refl])
    rp = [2, 0, 1]
    cols = [rp[c // R] * R + c % R for c in range(R * runs)]
    pr = P.run(X0[:, cols], Y0[:, cols], S, jt[rp])
    assert np.array_equal(pr["X"], base["X"][:, cols])
    assert np.array_equal(pr["best_E"], base["best_E"][rp])


def test_wall_invariant(orc):
    """After each step |x| <= 1, and every element clamped in that step has y = 0
    (the wall of Sec. II.A)."""
    N, R, runs, S = 32, 4, 2, 200
    J = inst.sk_pm1(N, 2)
    P = orc.Problem(N, R, runs, J=J, dt=0.5, a0=1.0, c0=None, fmode=orc.F_TERNARY)
    X, Y = inst.uniform_state(N, R * runs, 0.1, 3)
    X, Y = X.astype(float), Y.astype(float)
    clamped_total = 0
    for n in range(S):
        Xn, Yn = P.step(X, Y, orc.pump(n, S), orc.delta32(0.7, n, S), np.full(runs, 0.2))
        assert np.max(np.abs(Xn)) <= 1.0
        at_wall = np.abs(Xn) == 1.0
        assert np.all(Yn[at_wall] == 0.0)
        clamped_total += int(at_wall.sum())
        X, Y = Xn, Yn
    assert clamped_total > 0


def test_worked_fixture(orc):
    """Regression fixture for the documented readings (not a value printed in the
    paper). Step 0 of element (i=0, k=0) by hand: G = sign(X0) (Delta_0 = 0),
    Phi_00 = J_01 G_10 = -1, ring = 2 x_{0,1} = -0.04, force = -(1/2)(0.05)
    + (0.5/2)(-1 + 0.5) + 0.1(-0.04) = -0.154, y = 0.01 + 0.5(-0.154) = -0.067,
    x = 0.05 + 0.5(1/2)(-0.067) = 0.03325."""
    with open(os.path.join(GOLD, "worked_fixture.json")) as f:
        fx = json.load(f)
    P = orc.Problem(2, 2, 1, J=np.array(fx["J"]), h=np.array(fx["h"]), dt=fx["dt"],
                    a0=fx["a0"], c0=fx["c0"], fmode=orc.F_TERNARY)
    X0, Y0 = np.array(fx["X0"]), np.array(fx["Y0"])
    S = fx["S"]
    jt = np.full((1, S), fx["jperp"])
    X1, Y1 = P.step(X0, Y0, orc.pump(0, S), orc.delta32(0.7, 0, S), jt[:, 0])
    assert X1[0, 0] == pytest.approx(0.03325, abs=1e-15)
    assert Y1[0, 0] == pytest.approx(-0.067, abs=1e-15)
    np.testing.assert_allclose(X1, fx["X_after_step0"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(Y1, fx["Y_after_step0"], rtol=0, atol=1e-15)
    res = P.run(X0, Y0, S, jt)
    np.testing.assert_allclose(res["X"], fx["X_final"], rtol=0, atol=1e-14)
    assert res["best_E"][0] == fx["best_E"]


@pytest.mark.parametrize("kind", ["sk", "gauss_csr"])
def test_reaches_bruteforce_ground_state(orc, kind):
    """The SBQA iteration (Sec. II.A with the auto-tuned J_perp of Sec. II.B)
    finds the exhaustive ground state of small instances."""
    N, R, runs, S = 14, 8, 16, 600
    if kind == "sk":
        J = inst.sk_pm1(N, 101)
        csr, h = None, np.zeros(N)
    else:
        E = inst.regular_graph(N, 3, 102)
        csr = inst.edges_to_csr(N, E, inst.gaussian_edges(len(E), 103))
        J = inst.csr_to_dense(N, *csr)
        h = inst.gaussian_fields(N, 0.1, 104)
    Eg, _ = orc.bruteforce(J, h)
    P = orc.Problem(N, R, runs, J=None if csr else J, csr=csr, h=h, dt=0.5, a0=1.0,
                    fmode=orc.F_TERNARY)
    rng = np.random.default_rng(105)
    betas, alphas = rng.uniform(0.5, 1.5, runs), rng.uniform(0.5, 1.0, runs)
    jt = np.stack([orc.jperp_paper_table(b, a, 1.0, S) for b, a in zip(betas, alphas)])
    X0, Y0 = inst.uniform_state(N, R * runs, 0.1, 106)
    res = P.run(X0, Y0, S, jt)
    assert res["best_E"].min() == pytest.approx(Eg, abs=1e-9)
    for r in range(runs):
        assert orc.energy(res["best_s"][r][None], J=J, h=h)[0] == pytest.approx(res["best_E"][r], abs=1e-12)


def test_energy_tracking_ties_and_best_step(orc):
    """energy_every = K evaluates after every K-th step and at the end; the best
    per run is the minimum over its replicas and evaluations (Sec. II.B)."""
    N, R, runs, S = 16, 4, 2, 30
    J = inst.sk_pm1(N, 41)
    P = orc.Problem(N, R, runs, J=J, dt=0.5, a0=1.0, fmode=orc.F_TERNARY)
    X0, Y0 = inst.uniform_state(N, R * runs, 0.1, 42)
    jt = np.full((runs, S), 0.3)
    a = P.run(X0, Y0, S, jt, energy_every=0)
    b = P.run(X0, Y0, S, jt, energy_every=5)
    assert np.all(b["best_E"] <= a["best_E"])
    assert np.all(b["best_step"] % 5 == 0)
    # recompute the tracked minimum by stepping manually
    X, Y = X0.astype(float), Y0.astype(float)
    best = np.full(runs, np.inf)
    for n in range(S):
        X, Y = P.step(X, Y, orc.pump(n, S), orc.delta32(0.7, n, S), jt[:, n])
        if (n + 1) % 5 == 0:
            s = np.where(X >= 0, 1, -1).astype(np.int8).T
            E = orc.energy(s, J=J)
            best = np.minimum(best, E.reshape(runs, R).min(axis=1))
    assert np.array_equal(best, b["best_E"])


def test_regular_graph_generator():
    """Input recipe check: simple, exactly d-regular, symmetric CSR."""
    N, d = 200, 6
    E = inst.regular_graph(N, d, 1)
    assert len(E) == N * d // 2
    assert len({tuple(e) for e in E}) == len(E) and np.all(E[:, 0] < E[:, 1])
    rp, col, val = inst.edges_to_csr(N, E, inst.gaussian_edges(len(E), 2))
    assert np.all(np.diff(rp) == d)
    D = inst.csr_to_dense(N, rp, col, val)
    assert np.array_equal(D, D.T) and np.all(np.diag(D) == 0)


# ------------------------------------------------- three-body terms (HUBO)
def _hubo_csr(N, pairs, w2):
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    return inst.edges_to_csr(N, pairs, np.asarray(w2, dtype=float))


def test_hubo_energy_hand_fixture(orc):
    """Hand-computed energies with native three-body terms (Eq. 11 in the sign
    convention of Eq. 2); dense and CSR two-body parts agree; exhaustive
    minimum where given."""
    with open(os.path.join(GOLD, "hubo_hand.json")) as f:
        cases = json.load(f)["cases"]
    for case in cases:
        N = case["N"]
        csr = _hubo_csr(N, case["pairs"], case["w2"])
        J = inst.csr_to_dense(N, *csr)
        h = np.array(case["h"], dtype=float)
        T, K = np.array(case["triples"]), np.array(case["K"], dtype=float)
        s = np.array(case["spins"], dtype=np.int8)
        want = np.array(case["E"], dtype=float)
        assert np.array_equal(orc.energy(s, csr=csr, h=h, tri=T, K=K), want), case["name"]
        assert np.array_equal(orc.energy(s, J=J, h=h, tri=T, K=K), want), case["name"]
        if "ground_E" in case:
            assert orc.bruteforce_hubo(J, h, T, K)[0] == case["ground_E"]


def test_hubo_flip_identity_pins_three_body_fields(orc):
    """The energy is linear in each s_i, so flipping s_i changes it by
    2 s_i (phi_i + h_i), phi the coupling sum at f = s. With three-body terms
    this pins the oracle's three-body coupling sum (each triple feeds all three
    members with the product of the other two) against its energy."""
    N = 14
    P, w2, T, K, h = inst.random_hubo(N, 20, 30, 61)
    K = K + 0.25 * inst.gaussian_fields(len(K), 1.0, 62)   # non-integer weights too
    csr = _hubo_csr(N, P, w2)
    s = inst.spins_pm1(25, N, 63)
    phi = orc.fields(s.T.astype(float), csr=csr, tri=T, K=K)          # (N, count)
    E0 = orc.energy(s, csr=csr, h=h, tri=T, K=K)
    for i in range(N):
        t = s.copy()
        t[:, i] = -t[:, i]
        dE = orc.energy(t, csr=csr, h=h, tri=T, K=K) - E0
        np.testing.assert_allclose(dE, 2.0 * s[:, i] * (phi[i] + h[i]), rtol=1e-12, atol=1e-12)


def test_hubo_bruteforce_cross_checks(orc):
    """Plain enumeration (bruteforce_hubo) equals the Gray-code search without
    triples, and a numpy enumeration over all 2^N states with triples."""
    N = 11
    P, w2, T, K, h = inst.random_hubo(N, 18, 25, 71)
    J = inst.csr_to_dense(N, *_hubo_csr(N, P, w2))
    Eg, _ = orc.bruteforce(J, h)
    assert orc.bruteforce_hubo(J, h)[0] == Eg
    states = np.array(list(itertools.product([1, -1], repeat=N)), dtype=np.int8)
    Sd = states.astype(float)
    E_all = -0.5 * np.einsum("ci,ij,cj->c", Sd, J, Sd) - Sd @ h - (Sd[:, T[:, 0]] * Sd[:, T[:, 1]] * Sd[:, T[:, 2]]) @ K
    Eh, sh = orc.bruteforce_hubo(J, h, T, K)
    assert Eh == E_all.min()
    assert orc.energy(sh[None], J=J, h=h, tri=T, K=K)[0] == Eh


def test_hubo_special_cases(orc):
    """No triples: the three-body run is bit-identical to the Ising run.
    Reordering the triple list or the members inside a triple changes nothing
    (integer weights, ternary f: exact sums). c0 with triples follows the
    field-variance rule and reduces to the two-body rule."""
    N, R, runs, S = 16, 4, 3, 120
    P, w2, T, K, h = inst.random_hubo(N, 24, 30, 81)
    csr = _hubo_csr(N, P, w2)
    X0, Y0 = inst.uniform_state(N, R * runs, 0.2, 82)
    jt = np.tile(orc.jperp_linear_table(0.5, 0.0, S), (runs, 1))
    c0 = 0.07
    a = orc.Problem(N, R, runs, csr=csr, h=h, c0=c0).run(X0, Y0, S, jt)
    b = orc.Problem(N, R, runs, csr=csr, h=h, c0=c0, tri=T[:0], K=K[:0]).run(X0, Y0, S, jt)
    assert np.array_equal(a["X"], b["X"]) and np.array_equal(a["best_E"], b["best_E"])
    perm = np.random.default_rng(83).permutation(len(K))
    T2 = T[perm][:, [2, 0, 1]]
    r1 = orc.Problem(N, R, runs, csr=csr, h=h, c0=c0, tri=T, K=K).run(X0, Y0, S, jt)
    r2 = orc.Problem(N, R, runs, csr=csr, h=h, c0=c0, tri=T2, K=K[perm]).run(X0, Y0, S, jt)
    assert np.array_equal(r1["X"], r2["X"]) and np.array_equal(r1["best_E"], r2["best_E"])
    assert not np.array_equal(r1["X"], a["X"])
    # c0: 0.5 / sqrt((sum_{i!=j} J_ij^2 + 3 sum K^2) / (N - 1))
    ss = 2.0 * np.sum(w2 ** 2) + 3.0 * np.sum(K ** 2)
    assert orc.auto_c0(csr=csr, K=K) == pytest.approx(0.5 / math.sqrt(ss / (N - 1)), rel=1e-14)
    assert orc.auto_c0(csr=csr, K=K[:0]) == orc.auto_c0(csr=csr)


def test_hubo_reaches_bruteforce_ground_state(orc):
    """The SBQA iteration with native three-body coupling sums (ternary f,
    auto-tuned J_perp of Sec. II.B) finds the exhaustive minimum of small
    random instances."""
    N, R, runs, S = 14, 8, 16, 800
    for seed in (91, 92):
        P, w2, T, K, h = inst.random_hubo(N, 20, 24, seed)
        csr = _hubo_csr(N, P, w2)
        J = inst.csr_to_dense(N, *csr)
        Eg, _ = orc.bruteforce_hubo(J, h, T, K)
        Pb = orc.Problem(N, R, runs, csr=csr, h=h, tri=T, K=K, fmode=orc.F_TERNARY)
        rng = np.random.default_rng(seed + 100)
        betas, alphas = rng.uniform(0.5, 1.5, runs), rng.uniform(0.5, 1.0, runs)
        jt = np.stack([orc.jperp_paper_table(b, a, 1.0, S) for b, a in zip(betas, alphas)])
        X0, Y0 = inst.uniform_state(N, R * runs, 0.1, seed + 200)
        res = Pb.run(X0, Y0, S, jt)
        assert res["best_E"].min() == Eg, (seed, res["best_E"].min(), Eg)
        for r in range(runs):
            assert orc.energy(res["best_s"][r][None], csr=csr, h=h, tri=T, K=K)[0] == res["best_E"][r]


def test_heavy_hex_generator():
    """Heavy-hex graph: honeycomb sites of degree <= 3, bond sites of degree 2,
    bipartite between the two; HUBO terms are vertex-disjoint inside each set
    and every triple is a path of the graph."""
    N, E = inst.heavy_hex(6, 7)
    n0 = 42
    deg = np.bincount(E.ravel(), minlength=N)
    assert np.all(deg[n0:] == 2) and np.all(deg[:n0] <= 3) and np.all(deg[:n0] >= 2)
    assert np.all((E[:, 0] < n0) & (E[:, 1] >= n0))
    N2, P, w2, T, K = inst.hubo_heavy_hex(6, 7, 5, n2_sets=1, n3_sets=6)
    assert N2 == N and len(set(map(tuple, P))) == len(P) and len(set(map(tuple, T))) == len(T)
    assert len(np.unique(P.ravel())) == P.size          # one matching
    es = set(map(tuple, E))
    for a, b, c in T:
        links = sum((min(u, v), max(u, v)) in es for u, v in ((a, b), (b, c), (a, c)))
        assert links == 2                                # a path l - m - n


# ------------------------------------------- checkers used by the GPU tests
@pytest.mark.parametrize("kind", ["dense", "csr", "csr3"])
@pytest.mark.parametrize("fmode", [0, 1, 2])
def test_step_rows_equals_full_step(orc, kind, fmode):
    """The row-sampled step (the checker of every full-size GPU test) is the
    full step of Eqs. 6-7 restricted to the given rows, bit for bit: fields,
    positions and momenta. With three-body terms (Eq. 11) this pins its
    per-row three-body sum against the whole-list sum, which the single-flip
    identity above pins against the energy."""
    N, R, runs = 37, 4, 3
    rng = np.random.default_rng(101 + fmode)
    tri = K = None
    if kind == "dense":
        J, csr = inst.dense_gaussian(N, 102), None
    else:
        P2, w2, T, Kt, _ = inst.random_hubo(N, 60, 45, 103)
        csr = _hubo_csr(N, P2, w2)
        J = None
        if kind == "csr3":
            tri, K = T, Kt + 0.5 * inst.gaussian_fields(len(Kt), 1.0, 104)
    h = inst.gaussian_fields(N, 0.3, 105)
    P = orc.Problem(N, R, runs, J=J, csr=csr, h=h, dt=0.5, c0=0.21, fmode=fmode, tri=tri, K=K)
    X, Y = inst.uniform_state(N, R * runs, 0.6, 106)
    jr = np.array([0.11, 0.37, 0.02])
    an, dn = 0.43, np.float32(0.29)
    Xf, Yf, Pf = P.step(X, Y, an, dn, jr, want_phi=True)
    for rows in (np.arange(N), rng.permutation(N)[:9], np.array([N - 1, 0, 5, 5])):
        Xo, Yo, Po = P.step_rows(X, Y, an, dn, jr, rows)
        assert np.array_equal(Po, Pf[rows]), (kind, fmode)
        assert np.array_equal(Xo, Xf[rows]) and np.array_equal(Yo, Yf[rows]), (kind, fmode)


def test_jperp_paper_table_closed_form_values(orc):
    """Eq. 5 / Eq. S12 tabulated per step: entry n is J_perp at s = n/S with
    Gamma_x(t) = Gamma_x(0)[(1 - s)^alpha + 1e-5]. Values of
    (1/(2 beta)) ln coth(beta Gamma_x / R) worked out independently to ten
    digits, at s = 0 and 0.5 (table entries 0 and S/2) and s = 1 (the end of
    the anneal, one step past the table)."""
    S = 1000
    cases = [  # beta, alpha, Gamma_x(0), R, values at s = 0, 0.5, 1
        (1.0, 1.0, 1.0, 1, (0.1361679773, 0.3859599074, 5.7564627325)),
        (0.5, 0.5, 1.0, 16, (3.4660513560, 3.8124580975, 14.9786613678)),
        (1.5, 1.0, 1.0, 32, (1.0203309520, 1.2511936883, 4.8577320866)),
    ]
    for beta, alpha, g0, R, want in cases:
        tab = orc.jperp_paper_table(beta, alpha, g0 / R, S)
        assert tab[0] == pytest.approx(want[0], rel=2e-10, abs=0)
        assert tab[S // 2] == pytest.approx(want[1], rel=2e-10, abs=0)
        end = orc.jperp(beta, orc.gamma_x(g0 / R, alpha, 1.0))
        assert end == pytest.approx(want[2], rel=2e-10, abs=0)
        assert tab[-1] < end


def test_fields_dense_exact_and_equal_to_csr(orc):
    """The dense coupling sum Phi = J G of Eq. 7 for integer J and an operand
    in {-1, 0, +1}: every sum is an exact integer, so it must equal the exact
    int64 product bit for bit (J deliberately asymmetric, so a transposed
    operand fails), and the CSR form of the same J."""
    N, C = 45, 13
    rng = np.random.default_rng(111)
    J = rng.integers(-5, 6, size=(N, N)).astype(float)
    np.fill_diagonal(J, 0.0)
    G = rng.integers(-1, 2, size=(N, C)).astype(float)
    want = (J.astype(np.int64) @ G.astype(np.int64)).astype(float)
    Phi = orc.fields(G, J=J)
    assert np.array_equal(Phi, want)
    nz = np.nonzero(J)
    rp = np.concatenate([[0], np.cumsum(np.bincount(nz[0], minlength=N))]).astype(np.int32)
    assert np.array_equal(orc.fields(G, csr=(rp, nz[1].astype(np.int32), J[nz])), want)
    # one hand-sized case: row 0 of [[0, 2], [-3, 0]] . [[1, -1], [0, 1]]
    assert np.array_equal(orc.fields(np.array([[1.0, -1.0], [0.0, 1.0]]), J=np.array([[0.0, 2.0], [-3.0, 0.0]])),
                          [[0.0, 2.0], [-3.0, 3.0]])
