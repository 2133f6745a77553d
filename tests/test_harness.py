"""Instance generators of the benchmark families and the time-to-epsilon
harness (Sec. III): lattice structure, the planted ground state checked
against the oracle's energy and exhaustive enumeration, and the TT_eps
formula's closed-form values. The GPU runs of the harness are marked gpu."""
import math

import numpy as np
import pytest

import sbqa_instances as inst


@pytest.mark.parametrize("L", [3, 4, 7])
def test_lattices(L):
    """Periodic square (degree 4, 2L^2 bonds) and cubic (degree 6, 3L^3 bonds)
    lattices: every bond once, u < v, all sites of full degree."""
    for E, n_sites, deg in ((inst.square_lattice(L), L * L, 4), (inst.cubic_lattice(L), L ** 3, 6)):
        assert E.shape == (n_sites * deg // 2, 2)
        assert np.all(E[:, 0] < E[:, 1])
        assert len({tuple(e) for e in E}) == len(E)
        assert np.all(np.bincount(E.ravel(), minlength=n_sites) == deg)


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_planted_square_ground_state(orc, seed):
    """The planted state has energy E0 (oracle energy, Eq. 2 at the corners)
    and no configuration is lower (exhaustive search at L = 4, N = 16); the
    gauge hides it (not a constant configuration); bonds are the square
    lattice's."""
    L = 4
    E, w, s, E0 = inst.planted_square(L, seed)
    N = L * L
    assert sorted(map(tuple, E)) == sorted(map(tuple, inst.square_lattice(L)))
    csr = inst.edges_to_csr(N, E, w)
    assert orc.energy(s[None, :], csr=csr)[0] == E0
    J = inst.csr_to_dense(N, *csr)
    Emin, _ = orc.bruteforce(J)
    assert Emin == E0
    assert 0 < int(np.sum(s > 0)) < N


def test_planted_square_larger_is_consistent(orc):
    """At L = 32 the planted energy still equals the oracle's energy of the
    planted spins, and single flips never lower it (a local-minimum check)."""
    L = 32
    E, w, s, E0 = inst.planted_square(L, 11)
    N = L * L
    csr = inst.edges_to_csr(N, E, w)
    assert orc.energy(s[None, :], csr=csr)[0] == E0
    flips = np.repeat(s[None, :], 64, axis=0)
    idx = np.random.default_rng(12).choice(N, 64, replace=False)
    flips[np.arange(64), idx] *= -1
    assert np.all(orc.energy(flips, csr=csr) >= E0)


def test_tt_epsilon_formula():
    """TT_eps = tau log(1 - p_target) / log(1 - p_success) (Sec. III)."""
    from paper_2604_01050_amd.harness import optimality_gap, tt_epsilon
    assert math.isclose(tt_epsilon(2.0, 0.5), 2.0 * math.log(0.01) / math.log(0.5), rel_tol=1e-15)
    assert math.isclose(tt_epsilon(1.0, 0.9, 0.99), 2.0, rel_tol=1e-12)   # 0.1^2 = 0.01
    assert tt_epsilon(3.0, 0.995) == 3.0
    assert tt_epsilon(3.0, 0.0) == math.inf
    with pytest.raises(ValueError):
        tt_epsilon(1.0, 0.5, 1.0)
    assert np.allclose(optimality_gap([-90.0, -100.0], -100.0), [0.1, 0.0])


@pytest.mark.gpu
def test_harness_on_planted_lattice():
    """GPU: SBQA and the SBM baseline on a planted 16 x 16 lattice never return
    an energy below the planted ground state, return spins whose energy is
    the reported one, and the TT_eps study and per-step timing are finite."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    oracle.build()
    from paper_2604_01050_amd import harness as H
    E, w, s, E0 = inst.planted_square(16, 21)
    N = 256
    csr = inst.edges_to_csr(N, E, w)
    for sbm in (False, True):
        r = H.solve(csr=csr, R=16, runs=8, steps=800, seed=5, sbm=sbm)
        assert r["best"] >= E0
        assert oracle.energy(r["spins"][None, :], csr=csr)[0] == r["best"]
        assert np.all(r["per_run"] >= E0)
    st = H.tte_study(E0, [0.0, 0.02], [200, 800], seeds=[1, 2, 3], csr=csr, R=16, runs=8)
    assert len(st["rows"]) == 2 and all(0.0 <= p <= 1.0 for row in st["rows"] for p in row["p_success"])
    t_q = H.step_time(csr=csr, R=16, runs=8, steps=100)
    t_m = H.step_time(csr=csr, R=16, runs=8, steps=100, sbm=True)
    assert 0.0 < t_q < 1e-2 and 0.0 < t_m < 1e-2
