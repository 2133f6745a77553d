"""GPU parity of the SBQA library (through the C ABI) against the FP64 oracle.

Bars (see the readings of arXiv 2604.01050 documented with the oracle):
  * energies of given spins: bit-exact for integer J and h, 1e-12 relative otherwise;
  * one step from an identical float32 state: fields and x', y' within
    TOL = 1e-5 of the magnitude of the terms that make them (mixed bound),
    fp8 fields (J in {-1,0,1}) bit-exact, bf16 hi+lo fields within the derived
    bound BF16X3_TOL;
  * whole trajectories are chaotic: compared as best-energy statistics over
    256 seeds.
"""
import math
import os
import subprocess
import sys

import numpy as np
import pytest

import sbqa_instances as inst

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

TOL = 1e-5
# split bf16: J = J_hi + J_lo + e_J with |e_J| <= 2^-17 |J| (two 8-bit mantissas),
# same for x; the dropped J_lo x_lo is <= 2^-18 |J x|. Per product <= 2^-15.4 ~ 2.4e-5,
# plus fp32 accumulation; bound 4e-5 of sum_j |J_ij x_j|.
BF16X3_TOL = 4e-5


@pytest.fixture(scope="module")
def sb():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_01050_amd as p
    return p


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build()
    return oracle


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# ------------------------------------------------------------------ helpers
def _ctx(sb, J=None, csr=None, h=None, R=4, runs=3, steps=50, **kw):
    kw.setdefault("jp_kind", sb.JP_LINEAR)
    kw.setdefault("jp_start", 0.5)
    kw.setdefault("jp_end", 0.0)
    return sb.sbqa_create(J=J, csr=csr, h=h, R=R, runs=runs, steps=steps, **kw)


def _orc_problem(orc, sb, ctx, J=None, csr=None, h=None, fmode=0, dt=0.5, a0=1.0, tri=None, K=None):
    info = sb.sbqa_info(ctx)
    return orc.Problem(ctx.N, ctx.R, ctx.runs, J=J, csr=csr, h=h, dt=dt, a0=a0, c0=info["c0"], fmode=fmode,
                       tri=tri, K=K)


def _check_step(orc, P, ctx, sb, X, Y, n, S, jp_r, xg, yg, J=None, csr=None, h=None, rows=None,
                field_tol=TOL, delta_max=0.7, tri=None, K=None):
    """Compare the GPU's one step (xg, yg) from float32 (X, Y) with the oracle
    (all rows, or the sampled rows). Returns the number of wall-boundary
    elements excluded."""
    an, dn = orc.pump(n, S), orc.delta32(delta_max, n, S)
    if rows is None:
        xo, yo, phi = P.step(X, Y, an, dn, jp_r, want_phi=True)
        rows = np.arange(P.N)
    else:
        xo, yo, phi = P.step_rows(X, Y, an, dn, jp_r, rows)
        xg, yg = xg[rows], yg[rows]
    # magnitude of the coupling sum: sum_j |J_ij f_j| (+ sum |K f_a f_b|)
    G = orc.apply_f(P.fmode, dn, X.astype(np.float64))
    if csr is not None:
        absP = orc.Problem(P.N, P.R, P.runs, csr=(csr[0], csr[1], np.abs(csr[2])), c0=1.0, fmode=2, tri=tri,
                           K=None if K is None else np.abs(K))
    else:
        absP = orc.Problem(P.N, P.R, P.runs, J=np.abs(J), c0=1.0, fmode=2)
    _, _, phi_abs = absP.step_rows(np.abs(G), np.zeros_like(G), 0.0, 0.0, np.zeros(P.runs), rows)
    R = P.R
    hv = np.zeros(P.N) if h is None else np.asarray(h)
    Xr = X[rows].astype(np.float64)
    C = P.C
    kk = np.arange(C) % R
    rr = np.arange(C) // R
    left = rr * R + (kk + R - 1) % R
    right = rr * R + (kk + 1) % R
    jpc = np.asarray(jp_r)[rr]
    scale_y = np.abs(Y[rows]) + P.dt * (abs((P.a0 - an) / R) * np.abs(Xr)
                                         + (P.c0 / R) * (phi_abs + np.abs(hv[rows])[:, None])
                                         + np.abs(jpc) * (np.abs(Xr[:, left]) + np.abs(Xr[:, right])))
    tol_y = field_tol * scale_y + 1e-30
    tol_x = TOL * np.abs(Xr) + P.dt * (P.a0 / R) * tol_y + 1e-30
    at_wall = (np.abs(xg) >= 1.0 - 1e-5) | (np.abs(xo) >= 1.0 - 1e-5)
    clamp_mismatch = (np.abs(xg) == 1.0) != (np.abs(xo) == 1.0)
    excluded = at_wall & clamp_mismatch
    ok_x = (np.abs(xg - xo) <= tol_x) | excluded
    ok_y = (np.abs(yg - yo) <= tol_y) | excluded
    bad = ~(ok_x & ok_y)
    assert not bad.any(), "step %d: %d elements off; worst x %.3g (tol %.3g) y %.3g (tol %.3g)" % (
        n, bad.sum(), np.max(np.abs(xg - xo)), tol_x.ravel()[np.argmax(np.abs(xg - xo))],
        np.max(np.abs(yg - yo)), tol_y.ravel()[np.argmax(np.abs(yg - yo))])
    assert excluded.sum() <= max(2, 1e-3 * excluded.size)
    return int(excluded.sum()), phi, phi_abs


# ------------------------------------------------------------------ energies
@pytest.mark.parametrize("kind", ["sk_dense", "int_dense_h", "int_csr_h", "gauss_dense", "gauss_csr",
                                  "int_hubo_h", "normal_hubo"])
def test_energy_of_given_spins(sb, orc, kind):
    """Ising energy (Eq. 2 at the corners; with three-body terms the cubic part
    of Eq. 11) of given spins: bit-exact for integer J, K, h."""
    N = 300
    _log("energy parity %s N=%d" % (kind, N))
    csr = J = h = T = K = None
    if kind.endswith("hubo_h") or kind.endswith("hubo"):
        N, P2, w2, T, K = inst.hubo_heavy_hex(9, 10, 15, dist="int" if kind.startswith("int") else "normal")
        csr = inst.edges_to_csr(N, P2, w2)
        h = np.random.default_rng(16).integers(-2, 3, size=N).astype(float) if kind.endswith("_h") else None
    elif kind == "sk_dense":
        J = inst.sk_pm1(N, 1)
    elif kind == "int_dense_h":
        rng = np.random.default_rng(2)
        J = np.triu(rng.integers(-3, 4, size=(N, N)).astype(float), 1)
        J = J + J.T
        h = rng.integers(-5, 6, size=N).astype(float)
    elif kind == "int_csr_h":
        E = inst.regular_graph(N, 5, 3)
        w = np.random.default_rng(4).integers(-4, 5, size=len(E)).astype(float)
        csr = inst.edges_to_csr(N, E, w)
        h = np.random.default_rng(5).integers(-2, 3, size=N).astype(float)
    elif kind == "gauss_dense":
        J = inst.dense_gaussian(N, 6)
        h = inst.gaussian_fields(N, 0.3, 7)
    else:
        E = inst.regular_graph(N, 6, 8)
        csr = inst.edges_to_csr(N, E, inst.gaussian_edges(len(E), 9))
        h = inst.gaussian_fields(N, 0.1, 10)
    ctx = _ctx(sb, J=J, csr=csr, h=h, R=2, runs=3, precision=sb.PREC_FP32 if J is not None else 0, tri=T, K=K)
    s = inst.spins_pm1(70, N, 11)
    Eg = sb.sbqa_energy(ctx, s)
    Eo = orc.energy(s, J=J, h=h, csr=csr, tri=T, K=K)
    if kind.startswith(("sk", "int")):
        assert np.array_equal(Eg, Eo)
        assert sb.sbqa_info(ctx)["j_integral"]
    else:
        np.testing.assert_allclose(Eg, Eo, rtol=1e-12, atol=1e-9)


# ------------------------------------------------------- single-step parity
CASES = [
    # name, precision, fmode, coupling
    ("fp32_ternary", "PREC_FP32", 0, "gauss"),
    ("fp32_sign", "PREC_FP32", 1, "gauss"),
    ("fp32_ballistic", "PREC_FP32", 2, "gauss"),
    ("fp8_ternary", "PREC_FP8", 0, "sk"),
    ("fp8_sign", "PREC_FP8", 1, "sk"),
    ("fp8_bytes_ternary", "PREC_FP8", 0, "sk"),
    ("fp8_ternary_zeros", "PREC_FP8", 0, "sk0"),
    ("fp4_ternary", "PREC_FP4", 0, "sk"),
    ("fp4_bytes_sign", "PREC_FP4", 1, "sk"),
    ("fp4_ternary_zeros", "PREC_FP4", 0, "sk0"),
    ("int8_ternary", "PREC_INT8", 0, "sidon"),
    ("int8_sign", "PREC_INT8", 1, "sidon"),
    ("bf16x3_ballistic", "PREC_BF16X3", 2, "gauss"),
    ("bf16x3_ternary", "PREC_BF16X3", 0, "gauss"),
    ("csr_ternary", None, 0, "csr"),
    ("csr_sign", None, 1, "csr"),
    ("csr_ballistic", None, 2, "csr"),
    ("csr_ternary_r8", None, 0, "csr"),
    ("csr_ballistic_r8", None, 2, "csr"),
    # small dense loop (one workgroup per run, many steps per launch; here K = 1)
    ("small_fp32_ternary", "PREC_FP32", 0, "gauss_small"),
    ("small_fp32_ballistic", "PREC_FP32", 2, "gauss_small"),
    ("small_fp8_sign", "PREC_FP8", 1, "sk_small"),
    ("small_int8_ternary", "PREC_INT8", 0, "sidon_small"),
]


@pytest.mark.parametrize("name,prec,fmode,coup", CASES)
def test_single_step_parity(sb, orc, name, prec, fmode, coup):
    """One step of Eqs. 6-7 from identical float32 states at several step
    indices along a GPU trajectory (N = 300 / 1001 with ragged tiles; R = 5,
    runs = 7, C = 35 not a multiple of 4 or of the 128-column tile; R = 8 takes
    the CSR path whose ring neighbours come from adjacent lanes)."""
    R, runs, S = (8 if name.endswith("_r8") else 5), 7, 40
    csr = J = None
    small = coup.endswith("_small")
    if coup.startswith("sk"):
        N = 100 if small else 300
        J = inst.sk_pm1(N, 21)
        if coup == "sk0":   # J in {-1, 0, +1}: one byte per coupling
            keep = np.triu(np.random.default_rng(20).random((N, N)) < 0.6, 1)
            J = J * (keep | keep.T)
        h = np.round(inst.gaussian_fields(N, 1.0, 22))
    elif coup.startswith("sidon"):
        N = 100 if small else 300
        J = inst.sidon28_dense(N, 21)
        h = np.round(inst.gaussian_fields(N, 20.0, 22))
    elif coup.startswith("gauss"):
        N = 100 if small else 300
        J = inst.dense_gaussian(N, 23)
        h = inst.gaussian_fields(N, 0.2, 24)
    else:
        N = 1001
        E = inst.regular_graph(N - 1, 6, 25)
        E = np.vstack([E, [[3, N - 1], [N - 1, 500]]])  # ragged degree
        E = np.sort(E, axis=1)
        csr = inst.edges_to_csr(N, E, inst.gaussian_edges(len(E), 26))
        h = inst.gaussian_fields(N, 0.1, 27)
    _log("single-step parity %s N=%d R=%d runs=%d" % (name, N, R, runs))
    kw = {} if prec is None else {"precision": getattr(sb, prec)}
    kw["loop_kernel"] = sb.LOOP_RESIDENT if small else sb.LOOP_STREAM
    if "_bytes" in name:
        kw["j_packing"] = sb.JPACK_BYTES
    rng = np.random.default_rng(28)
    beta, alpha = rng.uniform(0.5, 1.5, runs), rng.uniform(0.5, 1.0, runs)
    ctx = _ctx(sb, J=J, csr=csr, h=h, R=R, runs=runs, steps=S, fmode=fmode, jp_kind=sb.JP_PAPER,
               beta=beta, alpha=alpha, gamma0_over_R=0.7, **kw)
    info = sb.sbqa_info(ctx)
    assert info["resident"] == small
    if prec in ("PREC_FP8", "PREC_FP4") and not small:
        base = "dense_fp8" if prec == "PREC_FP8" else "dense_fp4"
        assert info["path"] == (base + "_packed" if coup == "sk" and "_bytes" not in name else base)
    P = _orc_problem(orc, sb, ctx, J=J, csr=csr, h=h, fmode=fmode)
    jt = np.stack([orc.jperp_paper_table(b, a, 0.7, S) for b, a in zip(beta, alpha)])
    # schedule table of the library equals the oracle's, rounded to float32
    assert np.array_equal(sb.sbqa_jperp_table(ctx), jt.astype(np.float32))
    X0, Y0 = inst.uniform_state(N, R * runs, 0.3, 29)
    sb.sbqa_set_state(ctx, X0, Y0)
    excluded = 0
    for n in range(S):
        X, Y = sb.sbqa_get_state(ctx)
        if n in (0, 1, 7, 20, 39):
            phi_g = sb.sbqa_fields(ctx)
        sb.sbqa_step(ctx, 1)
        xg, yg = sb.sbqa_get_state(ctx)
        if n in (0, 1, 7, 20, 39):
            jr = jt[:, n].astype(np.float32).astype(np.float64)
            ex, phi_o, phi_abs = _check_step(orc, P, ctx, sb, X, Y, n, S, jr, xg, yg, J=J, csr=csr, h=h,
                                             field_tol=BF16X3_TOL if prec == "PREC_BF16X3" else TOL)
            excluded += ex
            if prec in ("PREC_FP8", "PREC_FP4", "PREC_INT8") or coup.startswith(("sk", "sidon")):
                assert np.array_equal(phi_g, phi_o.astype(np.float32)), "integer-J fields must be exact"
            else:
                ftol = BF16X3_TOL if prec == "PREC_BF16X3" else TOL
                err = np.abs(phi_g - phi_o)
                assert np.all(err <= ftol * phi_abs + 1e-30), "fields off: %g" % np.max(err / (phi_abs + 1e-30))
                if prec == "PREC_BF16X3" and fmode == 2:
                    rel = np.linalg.norm(phi_g - phi_o) / np.linalg.norm(phi_o)
                    _log("  bf16x3 normwise field error at step %d: %.3e" % (n, rel))
    _log("  %s: wall-boundary elements excluded: %d" % (name, excluded))


@pytest.mark.parametrize("prec,fmode,coup", [("PREC_FP32", 2, "gauss"), ("PREC_BF16X3", 2, "gauss"),
                                              ("PREC_FP8", 0, "sk"), ("PREC_FP8", 0, "sk_bytes"),
                                              ("PREC_INT8", 1, "sidon"), ("PREC_FP4", 0, "sk"),
                                              ("PREC_FP4", 1, "sk_bytes")])
def test_dense_tiles_identical(sb, prec, fmode, coup):
    """Every dense workgroup tile (64, 128 or 256 replica columns; the
    autotuner picks one) sums each field in the same K order, so trajectories
    agree bit-for-bit, real-valued couplings included."""
    N, R, runs, S = 300, 8, 20, 30
    J = {"gauss": inst.dense_gaussian, "sidon": inst.sidon28_dense}.get(coup, inst.sk_pm1)(N, 41)
    pk = {"j_packing": sb.JPACK_BYTES} if coup == "sk_bytes" else {}
    h = inst.gaussian_fields(N, 0.3, 42)
    _log("dense tiles %s N=%d C=%d" % (prec, N, R * runs))
    X0, Y0 = inst.uniform_state(N, R * runs, 0.2, 43)
    out = []
    for tile in (64, 128, 256, 0):
        ctx = _ctx(sb, J=J, h=h, R=R, runs=runs, steps=S, fmode=fmode, precision=getattr(sb, prec), dense_tile=tile,
                   loop_kernel=sb.LOOP_STREAM, **pk)
        info = sb.sbqa_info(ctx)
        assert info["tile_cols"] == tile or (tile == 0 and info["tile_cols"] in (64, 128, 256))
        sb.sbqa_set_state(ctx, X0, Y0)
        sb.sbqa_step(ctx, S)
        out.append(sb.sbqa_get_state(ctx) + (sb.sbqa_fields(ctx),))
    for other in out[1:]:
        for a, b in zip(out[0], other):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("prec,fmode", [("PREC_FP8", 0), ("PREC_FP8", 1), ("PREC_FP4", 0)])
def test_dense_split_k_identical(sb, orc, prec, fmode):
    """Bit-packed +-1 J with N = 2000 (K in 16 fp8 / 8 fp4 chunks): the
    128-column tile runs as the split-K kernel (two K halves added through
    LDS), the 64- and 256-column tiles in one pass; the integer-valued fields,
    trajectories, readout energies and best spins agree bit-for-bit, and the
    energies equal the oracle's."""
    N, R, runs, S = 2000, 8, 32, 25
    J = inst.sk_pm1(N, 51)
    h = inst.gaussian_fields(N, 1.0, 52).round()
    X0, Y0 = inst.uniform_state(N, R * runs, 0.2, 53)
    _log("dense split-K %s fmode %d N=%d C=%d" % (prec, fmode, N, R * runs))
    out = []
    for tile in (128, 64, 256):
        ctx = _ctx(sb, J=J, h=h, R=R, runs=runs, steps=S, fmode=fmode, precision=getattr(sb, prec), dense_tile=tile,
                   loop_kernel=sb.LOOP_STREAM)
        assert sb.sbqa_info(ctx)["tile_cols"] == tile
        sb.sbqa_set_state(ctx, X0, Y0)
        sb.sbqa_step(ctx, S)
        Eb, sp = sb.sbqa_best(ctx)
        out.append(sb.sbqa_get_state(ctx) + (sb.sbqa_fields(ctx), Eb, sp))
    for other in out[1:]:
        for a, b in zip(out[0], other):
            assert np.array_equal(a, b)
    np.testing.assert_array_equal(orc.energy(out[0][-1], J=J, h=h), out[0][-2])


def test_fp8_and_fp32_trajectories_identical(sb):
    """J in {-1,+1} with ternary f: fields are exact integers in fp8 and fp4
    (J bit-packed, or as e4m3 bytes / e2m1 nibbles) and fp32, so whole
    trajectories agree bit-for-bit."""
    N, R, runs, S = 700, 8, 6, 150
    J = inst.sk_pm1(N, 31)
    _log("fp8 vs fp32 trajectory N=%d S=%d" % (N, S))
    X0, Y0 = inst.uniform_state(N, R * runs, 0.1, 32)
    out = []
    for prec, pk, path in ((sb.PREC_FP8, sb.JPACK_AUTO, "dense_fp8_packed"), (sb.PREC_FP8, sb.JPACK_BYTES, "dense_fp8"),
                           (sb.PREC_FP4, sb.JPACK_AUTO, "dense_fp4_packed"), (sb.PREC_FP4, sb.JPACK_BYTES, "dense_fp4"),
                           (sb.PREC_AUTO, sb.JPACK_AUTO, "dense_fp4_packed"),
                           (sb.PREC_FP32, sb.JPACK_AUTO, "dense_fp32")):
        ctx = _ctx(sb, J=J, R=R, runs=runs, steps=S, precision=prec, j_packing=pk, loop_kernel=sb.LOOP_STREAM)
        assert sb.sbqa_info(ctx)["path"] == path
        sb.sbqa_set_state(ctx, X0, Y0)
        sb.sbqa_step(ctx, S)
        out.append(sb.sbqa_get_state(ctx) + sb.sbqa_best(ctx))
    for other in out[1:]:
        for a, b in zip(out[0], other):
            assert np.array_equal(a, b)


def test_int8_and_fp32_trajectories_identical(sb):
    """Integer J from the Sidon28 set (x 28) with ternary f: the int8 path's
    int32 sums and the fp32 path's sums are the same exact integers (|field| <
    2^24), so whole trajectories agree bit-for-bit; AUTO picks int8."""
    N, R, runs, S = 700, 8, 6, 150
    J = inst.sidon28_dense(N, 31)
    h = np.round(inst.gaussian_fields(N, 30.0, 30))
    _log("int8 vs fp32 trajectory N=%d S=%d" % (N, S))
    X0, Y0 = inst.uniform_state(N, R * runs, 0.1, 32)
    out = []
    for prec in (sb.PREC_AUTO, sb.PREC_FP32):
        ctx = _ctx(sb, J=J, h=h, R=R, runs=runs, steps=S, precision=prec, loop_kernel=sb.LOOP_STREAM)
        assert sb.sbqa_info(ctx)["path"] == ("dense_int8" if prec == sb.PREC_AUTO else "dense_fp32")
        sb.sbqa_set_state(ctx, X0, Y0)
        sb.sbqa_step(ctx, S)
        out.append(sb.sbqa_get_state(ctx) + sb.sbqa_best(ctx))
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("prec,coup,packing", [("PREC_FP8", "sk", "auto"), ("PREC_FP8", "sk", "bytes"),
                                               ("PREC_FP8", "sk0", "auto"), ("PREC_INT8", "sidon", "auto"),
                                               ("PREC_FP4", "sk", "auto"), ("PREC_FP4", "sk0", "auto")])
def test_integer_j_energies_on_mfma(sb, orc, prec, coup, packing):
    """Integer J on the fp8 / int8 paths: the readout energies come from the
    MFMA contraction of sign(x) (exact integers), and equal the oracle's
    float64 energies of the same spins bit for bit (N = 300 ragged, integer h)."""
    N, R, runs, S = 300, 4, 5, 37
    J = inst.sidon28_dense(N, 71) if coup == "sidon" else inst.sk_pm1(N, 71)
    if coup == "sk0":
        keep = np.triu(np.random.default_rng(72).random((N, N)) < 0.5, 1)
        J = J * (keep | keep.T)
    h = np.round(inst.gaussian_fields(N, 3.0, 73))
    ctx = _ctx(sb, J=J, h=h, R=R, runs=runs, steps=S, precision=getattr(sb, prec), loop_kernel=sb.LOOP_STREAM,
               j_packing=sb.JPACK_BYTES if packing == "bytes" else sb.JPACK_AUTO)
    sb.sbqa_step(ctx, S)
    X, _ = sb.sbqa_get_state(ctx)
    spins = np.where(X >= 0, 1, -1).astype(np.int8).T          # (C, N)
    Eo = orc.energy(spins, J=J, h=h).reshape(runs, R)
    Eb, sp = sb.sbqa_best(ctx)
    assert np.array_equal(Eb, Eo.min(axis=1))
    assert np.array_equal(orc.energy(sp, J=J, h=h), Eb)


# ----------------------------------------------- native three-body (HUBO) terms
@pytest.mark.parametrize("fmode,law,R", [(0, "int", 5), (1, "int", 8), (2, "normal", 5), (0, "normal", 8),
                                         (0, "cauchy", 5)])
def test_hubo_single_step_parity(sb, orc, fmode, law, R):
    """Heavy-hex instance with native three-body terms (Eq. 11): one step of
    Eqs. 6-7 from identical float32 states at several step indices; integer
    weights with ternary or sign f give exact fields; c0 follows the
    field-variance rule (R = 5: ring from memory, C = 35 ragged; R = 8: ring
    by lane reads)."""
    runs, S = 7, 40
    N, P2, w2, T, K = inst.hubo_heavy_hex(7, 8, 51, dist=law)
    csr = inst.edges_to_csr(N, P2, w2)
    h = np.round(inst.gaussian_fields(N, 1.0, 52)) if law == "int" else inst.gaussian_fields(N, 0.2, 52)
    _log("hubo single-step parity f=%d %s N=%d triples=%d R=%d" % (fmode, law, N, len(K), R))
    rng = np.random.default_rng(53)
    beta, alpha = rng.uniform(0.5, 1.5, runs), rng.uniform(0.5, 1.0, runs)
    ctx = _ctx(sb, csr=csr, h=h, tri=T, K=K, R=R, runs=runs, steps=S, fmode=fmode, jp_kind=sb.JP_PAPER,
               beta=beta, alpha=alpha, gamma0_over_R=0.7)
    info = sb.sbqa_info(ctx)
    assert info["path"] == "csr_fp32" and not info["resident"]
    assert info["c0"] == pytest.approx(orc.auto_c0(csr=csr, K=K), rel=1e-12)
    P = _orc_problem(orc, sb, ctx, csr=csr, h=h, fmode=fmode, tri=T, K=K)
    jt = np.stack([orc.jperp_paper_table(b, a, 0.7, S) for b, a in zip(beta, alpha)])
    X0, Y0 = inst.uniform_state(N, R * runs, 0.3, 54)
    sb.sbqa_set_state(ctx, X0, Y0)
    for n in range(S):
        X, Y = sb.sbqa_get_state(ctx)
        if n in (0, 1, 7, 20, 39):
            phi_g = sb.sbqa_fields(ctx)
        sb.sbqa_step(ctx, 1)
        xg, yg = sb.sbqa_get_state(ctx)
        if n in (0, 1, 7, 20, 39):
            jr = jt[:, n].astype(np.float32).astype(np.float64)
            _, phi_o, phi_abs = _check_step(orc, P, ctx, sb, X, Y, n, S, jr, xg, yg, csr=csr, h=h, tri=T, K=K)
            if law == "int" and fmode != 2:
                assert np.array_equal(phi_g, phi_o.astype(np.float32)), "integer three-body fields must be exact"
            else:
                assert np.all(np.abs(phi_g - phi_o) <= TOL * phi_abs + 1e-30)


def test_hubo_reaches_bruteforce_minimum(sb, orc):
    """End to end on the GPU: small random instances with three-body terms
    reach the exhaustive minimum of the oracle, and the returned energies are
    the oracle's energies of the returned spins (bit-exact, integer weights)."""
    N, R, runs, S = 14, 8, 16, 800
    for seed in (91, 92, 93):
        P2, w2, T, K, h = inst.random_hubo(N, 20, 24, seed)
        csr = inst.edges_to_csr(N, P2, w2)
        Eg, _ = orc.bruteforce_hubo(inst.csr_to_dense(N, *csr), h, T, K)
        ctx = _ctx(sb, csr=csr, h=h, tri=T, K=K, R=R, runs=runs, steps=S, jp_kind=sb.JP_PAPER, seed=seed)
        sb.sbqa_step(ctx, S)
        Eb, sp = sb.sbqa_best(ctx)
        assert np.array_equal(orc.energy(sp, csr=csr, h=h, tri=T, K=K), Eb)
        assert Eb.min() == Eg, (seed, Eb.min(), Eg)


def test_hubo_large_heavy_hex(sb, orc):
    """Heavy-hex HUBO with about 1e5 spins (200 x 200 honeycomb, one matching
    of 2-body terms, six sets of 3-body paths), R = 16 x 8 runs: sampled rows
    of one step, and the energies of the returned spins."""
    N, P2, w2, T, K = inst.hubo_heavy_hex(200, 200, 61, dist="normal")
    csr = inst.edges_to_csr(N, P2, w2)
    R, runs = 16, 8
    _log("large heavy-hex hubo N=%d triples=%d" % (N, len(K)))
    _full_size_step(sb, orc, csr=csr, N=N, R=R, runs=runs, nrows=48, S=1000, tri=T, K=K)
    ctx = _ctx(sb, csr=csr, tri=T, K=K, R=R, runs=runs, steps=100, seed=3)
    assert sb.sbqa_info(ctx)["reordered"]          # vertex and bond sites far apart: relabelled (AUTO)
    sb.sbqa_step(ctx, 100)
    Eb, sp = sb.sbqa_best(ctx)
    np.testing.assert_allclose(orc.energy(sp, csr=csr, tri=T, K=K), Eb, rtol=1e-12, atol=1e-9)


# --------------------------------------------------------------- edge cases
def _edge_instance(kind):
    """Degenerate shapes: a single spin, one run of one replica, isolated
    spins, no couplings at all, three-body terms only."""
    rng = np.random.default_rng(90)
    if kind == "dense_n1":
        return dict(J=np.zeros((1, 1)), h=np.array([0.5]), R=3, runs=2, precision="PREC_FP32")
    if kind == "dense_n2_fp4_c1":
        return dict(J=np.array([[0.0, -1.0], [-1.0, 0.0]]), h=np.array([1.0, 0.0]), R=1, runs=1, precision="PREC_FP4")
    if kind == "dense_n2_fp8_bytes":
        return dict(J=np.array([[0.0, 1.0], [1.0, 0.0]]), h=None, R=2, runs=1, precision="PREC_FP8",
                    j_packing="JPACK_BYTES")
    if kind == "csr_isolated":
        N = 37
        E = np.array([[0, 1], [1, 2], [2, 3], [5, 9], [9, 30], [30, 36], [0, 36]])
        return dict(csr=inst.edges_to_csr(N, E, rng.integers(-3, 4, len(E)).astype(float)),
                    h=rng.integers(-1, 2, N).astype(float), R=1, runs=3)
    if kind == "csr_empty":
        N = 10
        return dict(csr=(np.zeros(N + 1, np.int32), np.zeros(0, np.int32), np.zeros(0)),
                    h=rng.integers(-2, 3, N).astype(float), R=4, runs=2)
    if kind == "hubo_pure":
        N = 12
        P2, w2, T, K, h = inst.random_hubo(N, 0, 15, 91)
        return dict(csr=(np.zeros(N + 1, np.int32), np.zeros(0, np.int32), np.zeros(0)), tri=T, K=K, h=h, R=4, runs=2)
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["dense_n1", "dense_n2_fp4_c1", "dense_n2_fp8_bytes", "csr_isolated", "csr_empty",
                                  "hubo_pure"])
def test_edge_instances_step_parity(sb, orc, kind):
    """Degenerate instances step for step against the oracle (one step from
    the GPU's own state, 12 steps, streaming kernels), and the energies of
    the returned spins."""
    d = _edge_instance(kind)
    J, csr, h = d.get("J"), d.get("csr"), d.get("h")
    R, runs, S = d["R"], d["runs"], 12
    kw = {}
    if "precision" in d:
        kw["precision"] = getattr(sb, d["precision"])
    if "j_packing" in d:
        kw["j_packing"] = getattr(sb, d["j_packing"])
    ctx = _ctx(sb, J=J, csr=csr, h=h, R=R, runs=runs, steps=S, tri=d.get("tri"), K=d.get("K"),
               loop_kernel=sb.LOOP_STREAM, jp_kind=sb.JP_PAPER, **kw)
    P = _orc_problem(orc, sb, ctx, J=J, csr=csr, h=h, tri=d.get("tri"), K=d.get("K"))
    N = ctx.N
    X0, Y0 = inst.uniform_state(N, R * runs, 0.6, 92)
    sb.sbqa_set_state(ctx, X0, Y0)
    jt = sb.sbqa_jperp_table(ctx)
    for n in range(S):
        X, Y = sb.sbqa_get_state(ctx)
        sb.sbqa_step(ctx, 1)
        xg, yg = sb.sbqa_get_state(ctx)
        _check_step(orc, P, ctx, sb, X, Y, n, S, jt[:, n].astype(np.float64), xg, yg, J=J, csr=csr, h=h,
                    tri=d.get("tri"), K=d.get("K"))
    Eb, sp = sb.sbqa_best(ctx)
    np.testing.assert_allclose(orc.energy(sp, J=J, csr=csr, h=h, tri=d.get("tri"), K=d.get("K")), Eb,
                               rtol=1e-12, atol=1e-12)


def test_negation_symmetry_and_column_independence(sb):
    """h = 0: negated start -> negated trajectory (bit-exact). With J_perp = 0
    a run alone equals the same run inside a batch (CSR path: per-element
    arithmetic independent of the batch)."""
    N, R, runs, S = 500, 4, 5, 60
    E = inst.regular_graph(N, 4, 33)
    csr = inst.edges_to_csr(N, E, inst.gaussian_edges(len(E), 34))
    X0, Y0 = inst.uniform_state(N, R * runs, 0.1, 35)
    res = []
    for sgn in (1, -1):
        ctx = _ctx(sb, csr=csr, R=R, runs=runs, steps=S)
        sb.sbqa_set_state(ctx, sgn * X0, sgn * Y0)
        sb.sbqa_step(ctx, S)
        res.append(sb.sbqa_get_state(ctx))
    assert np.array_equal(res[0][0], -res[1][0]) and np.array_equal(res[0][1], -res[1][1])
    J = inst.sk_pm1(200, 36)
    X0, Y0 = inst.uniform_state(200, R * runs, 0.1, 37)
    full = _ctx(sb, J=J, R=R, runs=runs, steps=S, jp_start=0.0, jp_end=0.0)
    sb.sbqa_set_state(full, X0, Y0)
    sb.sbqa_step(full, S)
    xf, _ = sb.sbqa_get_state(full)
    one = _ctx(sb, J=J, R=R, runs=1, steps=S, jp_start=0.0, jp_end=0.0)
    sb.sbqa_set_state(one, X0[:, 2 * R:3 * R], Y0[:, 2 * R:3 * R])
    sb.sbqa_step(one, S)
    x1, _ = sb.sbqa_get_state(one)
    assert np.array_equal(x1, xf[:, 2 * R:3 * R])


def _philox4x32_10(ctr, key):
    """Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), vectorised numpy."""
    M0, M1, W0, W1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57), 0x9E3779B9, 0xBB67AE85
    c = [np.asarray(v, dtype=np.uint64) for v in ctr]
    k0, k1 = np.uint64(key[0]), np.uint64(key[1])
    mask = np.uint64(0xFFFFFFFF)
    for rnd in range(10):
        if rnd:
            k0 = np.uint64((int(k0) + W0) & 0xFFFFFFFF)
            k1 = np.uint64((int(k1) + W1) & 0xFFFFFFFF)
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        c = [((p1 >> np.uint64(32)) ^ c[1] ^ k0) & mask, p1 & mask,
             ((p0 >> np.uint64(32)) ^ c[3] ^ k1) & mask, p0 & mask]
    return c


def test_init_state_is_philox(sb):
    """Library's initial state x, y ~ U[-amp, amp] from Philox4x32-10 keyed by
    the seed with counter (i, c, 0, 0)."""
    z = _philox4x32_10([0, 0, 0, 0], (0, 0))
    assert [int(v) for v in z] == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]  # published KAT
    N, R, runs, seed, amp = 130, 3, 5, 0x123456789ABCDEF, 0.1
    for J, csr in ((inst.sk_pm1(N, 40), None), (None, inst.edges_to_csr(N, inst.regular_graph(N, 4, 41), np.ones(N * 2)))):
        ctx = _ctx(sb, J=J, csr=csr, R=R, runs=runs, seed=seed, init_amp=amp)
        x, y = sb.sbqa_get_state(ctx)
        i, c = np.meshgrid(np.arange(N), np.arange(R * runs), indexing="ij")
        r = _philox4x32_10([i.ravel(), c.ravel(), 0, 0], (seed & 0xFFFFFFFF, seed >> 32))
        ux = (r[0] >> np.uint64(8)).astype(np.float64) / 16777216.0
        uy = (r[1] >> np.uint64(8)).astype(np.float64) / 16777216.0
        assert np.array_equal(x.ravel(), (amp * (2 * ux - 1)).astype(np.float32))
        assert np.array_equal(y.ravel(), (amp * (2 * uy - 1)).astype(np.float32))


def test_best_and_step_errors(sb, orc):
    """sbqa_best returns per run the minimum over replicas of E(sign x) and the
    spins that reach it; stepping past the schedule is ESTATE."""
    N, R, runs, S = 180, 6, 4, 100
    J = inst.sk_pm1(N, 50)
    ctx = _ctx(sb, J=J, R=R, runs=runs, steps=S)
    sb.sbqa_step(ctx, S)
    E, s = sb.sbqa_best(ctx)
    assert np.array_equal(orc.energy(s, J=J), E)
    x, _ = sb.sbqa_get_state(ctx)
    allE = orc.energy(np.where(x >= 0, 1, -1).astype(np.int8).T, J=J).reshape(runs, R)
    assert np.array_equal(allE.min(axis=1), E)
    with pytest.raises(sb.SbqaError) as ei:
        sb.sbqa_step(ctx, 1)
    assert ei.value.status == sb.ESTATE


def test_energy_tracking_matches_oracle(sb, orc):
    """energy_every = K: best over evaluations after every K-th step (CSR with
    integer J: trajectories identical in this short window, energies exact)."""
    N, R, runs, S, K = 256, 4, 3, 30, 5
    E = inst.regular_graph(N, 3, 60)
    csr = inst.edges_to_csr(N, E, np.ones(len(E)))
    ctx = _ctx(sb, csr=csr, R=R, runs=runs, steps=S, energy_every=K)
    X0, Y0 = inst.uniform_state(N, R * runs, 0.1, 61)
    sb.sbqa_set_state(ctx, X0, Y0)
    sb.sbqa_step(ctx, S)
    Eg, sg = sb.sbqa_best(ctx)
    st = sb.sbqa_best_step(ctx)
    assert np.all(st % K == 0)
    assert np.array_equal(orc.energy(sg, csr=csr), Eg)


# ----------------------------------------------------- full-size, sampled rows
def _full_size_step(sb, orc, J=None, csr=None, h=None, N=None, R=None, runs=None, prec=None, fmode=0,
                    nrows=48, steps_before=3, S=1000, field_tol=TOL, exact_fields=False, **extra):
    kw = {} if prec is None else {"precision": prec}
    kw.update(extra)
    tri, K = extra.get("tri"), extra.get("K")
    ctx = _ctx(sb, J=J, csr=csr, h=h, R=R, runs=runs, steps=S, fmode=fmode, seed=7, **kw)
    sb.sbqa_step(ctx, steps_before)
    X, Y = sb.sbqa_get_state(ctx)
    phi_g = sb.sbqa_fields(ctx)
    sb.sbqa_step(ctx, 1)
    xg, yg = sb.sbqa_get_state(ctx)
    P = _orc_problem(orc, sb, ctx, J=J, csr=csr, h=h, fmode=fmode, tri=tri, K=K)
    rows = np.sort(np.random.default_rng(3).choice(N, nrows, replace=False))
    rows[-1] = N - 1
    jr = sb.sbqa_jperp_table(ctx)[:, steps_before].astype(np.float64)
    ex, phi_o, phi_abs = _check_step(orc, P, ctx, sb, X, Y, steps_before, S, jr, xg, yg, J=J, csr=csr, h=h,
                                     rows=rows, field_tol=field_tol, tri=tri, K=K)
    if exact_fields:
        assert np.array_equal(phi_g[rows], phi_o.astype(np.float32))
    else:
        assert np.all(np.abs(phi_g[rows] - phi_o) <= field_tol * phi_abs + 1e-30)
    return phi_g[rows], phi_o, phi_abs


def test_full_size_sparse_regular(sb, orc):
    """Random 6-regular N = 4096, Gaussian J, h ~ N(0, 0.1^2), R = 32 x 64 runs:
    the bench workload, checked on every row for one step."""
    N, d, R, runs = 4096, 6, 32, 64
    _log("full-size sparse N=%d R=%d runs=%d" % (N, R, runs))
    E = inst.regular_graph(N, d, 2001)
    csr = inst.edges_to_csr(N, E, inst.gaussian_edges(len(E), 2002))
    h = inst.gaussian_fields(N, 0.1, 2003)
    _full_size_step(sb, orc, csr=csr, h=h, N=N, R=R, runs=runs, nrows=N, S=5000)


def test_large_cubic_lattice(sb, orc):
    """Periodic cubic lattice L = 64 (N = 262144, degree 6), Gaussian bonds,
    R = 16 x 8 runs: the large-lattice regime of Sec. III on the streaming CSR
    kernel, sampled rows (the last row included); energies of the returned
    spins agree with the oracle's."""
    L, R, runs = 64, 16, 8
    N = L ** 3
    _log("large cubic lattice N=%d R=%d runs=%d" % (N, R, runs))
    E = inst.cubic_lattice(L)
    csr = inst.edges_to_csr(N, E, inst.gaussian_edges(len(E), 2201))
    h = inst.gaussian_fields(N, 0.1, 2202)
    _full_size_step(sb, orc, csr=csr, h=h, N=N, R=R, runs=runs, nrows=48, S=1000)
    ctx = _ctx(sb, csr=csr, h=h, R=R, runs=runs, steps=200, seed=9)
    assert not sb.sbqa_info(ctx)["reordered"]      # lattice order is already local (REORDER_AUTO)
    sb.sbqa_step(ctx, 200)
    Eb, sp = sb.sbqa_best(ctx)
    np.testing.assert_allclose(orc.energy(sp, csr=csr, h=h), Eb, rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("prec,packing", [("PREC_FP8", "packed"), ("PREC_FP8", "bytes"), ("PREC_FP4", "packed")])
def test_full_size_fp8_sk(sb, orc, prec, packing):
    """SK N = 16384, J = +-1 bit-packed or as e4m3 bytes (fp8), bit-packed
    (fp4), R = 16 x 16 runs: sampled rows, fields exact."""
    N, R, runs = 16384, 16, 16
    _log("full-size %s SK N=%d J %s" % (prec, N, packing))
    J = inst.sk_pm1(N, 3001)
    _full_size_step(sb, orc, J=J, N=N, R=R, runs=runs, prec=getattr(sb, prec), S=10000, exact_fields=True, nrows=24,
                    j_packing=sb.JPACK_AUTO if packing == "packed" else sb.JPACK_BYTES)


def test_full_size_int8_sidon(sb, orc):
    """N = 16384, integer J from the Sidon28 set (x 28) as int8, R = 16 x 16
    runs: sampled rows, fields exact."""
    N, R, runs = 16384, 16, 16
    _log("full-size int8 Sidon28 N=%d" % N)
    J = inst.sidon28_dense(N, 3101)
    _full_size_step(sb, orc, J=J, N=N, R=R, runs=runs, prec=sb.PREC_INT8, S=10000, exact_fields=True, nrows=24)


def test_full_size_bf16x3_gaussian(sb, orc):
    """N = 8192 Gaussian J, ballistic f, bf16 hi+lo, R = 16 x 32 runs: sampled rows
    within the derived split-bf16 bound; normwise error reported."""
    N, R, runs = 8192, 16, 32
    _log("full-size bf16x3 N=%d" % N)
    J = inst.dense_gaussian(N, 4001)
    pg, po, pa = _full_size_step(sb, orc, J=J, N=N, R=R, runs=runs, prec=sb.PREC_BF16X3, fmode=2, S=5000,
                                 field_tol=BF16X3_TOL, nrows=24)
    _log("  bf16x3 N=8192 normwise field error %.3e, max elementwise/|J||x| %.3e" % (
        np.linalg.norm(pg - po) / np.linalg.norm(po), np.max(np.abs(pg - po) / pa)))


# ---------------------------------------------------------------- statistics
def test_best_energy_statistics_256_seeds(sb, orc):
    """SK N = 64 +-1, h = 0, R = 8, 4 runs, 1000 steps, dt = 0.5, J_perp linear
    0.5 -> 0, ternary f (256 seeds): per-seed best energy from the GPU and from
    the oracle agree within 3 sigma of the mean difference and pass a KS test."""
    stats = pytest.importorskip("scipy.stats")
    N, R, runs_per_seed, seeds, S = 64, 8, 4, 256, 1000
    runs = runs_per_seed * seeds
    J = inst.sk_pm1(N, 1001)
    X0, Y0 = inst.uniform_state(N, R * runs, 0.1, 1002)
    _log("statistics: %d seeds x %d runs, S=%d" % (seeds, runs_per_seed, S))
    ctx = _ctx(sb, J=J, R=R, runs=runs, steps=S, precision=sb.PREC_FP32)
    sb.sbqa_set_state(ctx, X0, Y0)
    sb.sbqa_step(ctx, S)
    Eg, _ = sb.sbqa_best(ctx)
    P = orc.Problem(N, R, runs, J=J, dt=0.5, a0=1.0, c0=sb.sbqa_info(ctx)["c0"], fmode=0)
    res = P.run(X0, Y0, S, np.tile(orc.jperp_linear_table(0.5, 0.0, S), (runs, 1)))
    Eo = res["best_E"]
    g = Eg.reshape(seeds, runs_per_seed).min(axis=1)
    o = Eo.reshape(seeds, runs_per_seed).min(axis=1)
    se = math.sqrt(g.var() / seeds + o.var() / seeds)
    _log("  GPU mean %.3f min %.0f | oracle mean %.3f min %.0f | se %.3f" % (g.mean(), g.min(), o.mean(), o.min(), se))
    assert abs(g.mean() - o.mean()) <= 3 * se + 1e-12
    assert stats.ks_2samp(g, o).pvalue > 0.01


def test_bf16x3_matches_fp32_statistics_256_seeds(sb):
    """Real-valued couplings (the Gaussian dense configuration at a smaller
    N): J ~ N(0,1) symmetric, h = 0, ballistic f, R = 16, 2 runs per seed,
    256 seeds, 1000 steps, J_perp linear 0.5 -> 0, from identical initial
    states. The split-bf16 contraction (hi+lo products, float32 sums) and the
    plain float32 one follow different rounding, so the chaotic trajectories
    part; their per-seed best energies must still agree in distribution: mean
    difference within 3 sigma and two-sample KS p > 0.01."""
    stats = pytest.importorskip("scipy.stats")
    N, R, runs_per_seed, seeds, S = 256, 16, 2, 256, 1000
    runs = runs_per_seed * seeds
    J = inst.dense_gaussian(N, 1101)
    X0, Y0 = inst.uniform_state(N, R * runs, 0.1, 1102)
    best = {}
    for name, prec in (("bf16x3", sb.PREC_BF16X3), ("fp32", sb.PREC_FP32)):
        _log("statistics bf16x3 vs fp32: %s, %d seeds x %d runs, N=%d, S=%d" % (name, seeds, runs_per_seed, N, S))
        ctx = _ctx(sb, J=J, R=R, runs=runs, steps=S, precision=prec, fmode=sb.F_BALLISTIC)
        sb.sbqa_set_state(ctx, X0, Y0)
        sb.sbqa_step(ctx, S)
        E, _ = sb.sbqa_best(ctx)
        best[name] = E.reshape(seeds, runs_per_seed).min(axis=1)
        sb.sbqa_destroy(ctx)
    g, f = best["bf16x3"], best["fp32"]
    se = math.sqrt(g.var() / seeds + f.var() / seeds)
    _log("  bf16x3 mean %.4f min %.4f | fp32 mean %.4f min %.4f | se %.4f | identical seeds %d"
         % (g.mean(), g.min(), f.mean(), f.min(), se, int(np.sum(g == f))))
    assert abs(g.mean() - f.mean()) <= 3 * se + 1e-12
    assert stats.ks_2samp(g, f).pvalue > 0.01


# -------------------------------------------------------------------- serving
def test_serving_graph_blocks_alone_equals_mix(sb):
    """Longer schedules (several full step blocks, replayed from a captured
    graph while membership changes as instances finish at different steps,
    plus partial blocks and energy tracking; fp8, int8, CSR and three-body CSR
    instances): every result equals the instance's standalone run bit-for-bit."""
    rng = np.random.default_rng(80)
    items = []
    for q in range(7):
        N = int(rng.choice([200, 300, 512]))
        steps = int(rng.choice([150, 200, 333]))
        ee = 0 if q % 3 else 50
        extra = {}
        if q % 2 == 0:   # q = 6: integer Sidon28 couplings (int8 path); q = 2: fp4
            J, csr = (inst.sidon28_dense if q == 6 else inst.sk_pm1)(N, 800 + q), None
            if q == 2:
                extra = dict(precision=sb.PREC_FP4)
        elif q == 5:     # native three-body terms on a heavy-hex graph
            Nh, P2, w2, T, K = inst.hubo_heavy_hex(8, 9, 815, dist="normal")
            J, csr = None, inst.edges_to_csr(Nh, P2, w2)
            extra = dict(tri=T, K=K)
        else:
            N -= N % 2
            E = inst.regular_graph(N, int(rng.integers(3, 7)), 810 + q)
            J, csr = None, inst.edges_to_csr(N, E, inst.gaussian_edges(len(E), 820 + q))
        items.append((J, csr, dict(R=8, runs=2, steps=steps, seed=830 + q, jp_kind=sb.JP_PAPER, energy_every=ee,
                                   **extra)))
    alone = []
    for J, csr, kw in items:
        ctx = sb.sbqa_create(J=J, csr=csr, loop_kernel=sb.LOOP_STREAM, **kw)
        sb.sbqa_step(ctx, kw["steps"])
        alone.append(sb.sbqa_best(ctx))
        sb.sbqa_destroy(ctx)
    srv = sb.sbqa_server_create(1 << 30, 4)
    import time
    for rep in range(2):      # the second round replays the graphs captured in the first
        tickets = [sb.sbqa_submit(srv, J=J, csr=csr, **kw) for J, csr, kw in items]
        got = {}
        t0 = time.time()
        while len(got) < len(tickets) and time.time() - t0 < 120:
            for t in tickets:
                if t not in got:
                    r = sb.sbqa_poll(srv, t)
                    if r is not None:
                        got[t] = r
            time.sleep(0.005)
        assert len(got) == len(tickets)
        for t, (Ea, sa) in zip(tickets, alone):
            Em, sm, _ = got[t]
            assert np.array_equal(Ea, Em) and np.array_equal(sa, sm)
    sb.sbqa_server_destroy(srv)


def test_serving_alone_equals_mix_stream_sizes(sb):
    """The serving configuration's shapes: R = 16 x 8 runs (C = 128), a dense
    SK +-1 instance of N = 8192 (bit-packed fp8, built from sign bits on the
    server), a sparse d-regular Gaussian instance of N = 8000, and smaller ones
    of both kinds, one dense instance on the fp4 contraction (the stream's
    --serve-dense fp4 form); served results equal the standalone runs bit for
    bit."""
    rng = np.random.default_rng(71)
    specs = [("dense", 8192), ("sparse", 8000), ("dense", 1536), ("sparse", 700), ("dense", 300),
             ("dense_fp4", 4096)]
    items = []
    for q, (kind, N) in enumerate(specs):
        kw = dict(R=16, runs=8, steps=100, seed=740 + q, jp_kind=sb.JP_LINEAR, jp_start=0.5, jp_end=0.0)
        if kind.startswith("dense"):
            prec = sb.PREC_FP4 if kind == "dense_fp4" else sb.PREC_FP8
            items.append((inst.sk_pm1(N, 750 + q), None, dict(kw, precision=prec)))
        else:
            d = int(rng.integers(3, 13))
            E = inst.regular_graph(N, d, 760 + q)
            items.append((None, inst.edges_to_csr(N, E, inst.gaussian_edges(len(E), 770 + q)), kw))
    _log("serving at stream sizes: %s" % specs)
    alone = []
    for J, csr, kw in items:
        ctx = sb.sbqa_create(J=J, csr=csr, **kw)
        sb.sbqa_step(ctx, kw["steps"])
        alone.append(sb.sbqa_best(ctx))
        sb.sbqa_destroy(ctx)
    srv = sb.sbqa_server_create(8 << 30, 3)
    tickets = [sb.sbqa_submit(srv, J=J, csr=csr, **kw) for J, csr, kw in items]
    import time
    got = {}
    t0 = time.time()
    while len(got) < len(tickets) and time.time() - t0 < 120:
        for t in tickets:
            if t not in got:
                r = sb.sbqa_poll(srv, t)
                if r is not None:
                    got[t] = r
        time.sleep(0.005)
    assert len(got) == len(tickets)
    for t, (Ea, sa), (kind, N) in zip(tickets, alone, specs):
        Em, sm, _ = got[t]
        assert np.array_equal(Ea, Em) and np.array_equal(sa, sm), (kind, N)
    sb.sbqa_server_destroy(srv)


def test_serving_alone_equals_mix(sb):
    """Continuous batching: instances of mixed size and density submitted to a
    server (small budget, 3 slots, so some wait) give exactly the results they
    give alone; an instance larger than the budget is EBUDGET."""
    rng = np.random.default_rng(70)
    items = []
    for q in range(6):
        N = int(rng.choice([256, 384, 512, 1000]))
        if q % 2 == 0:
            J, csr = inst.sk_pm1(N, 700 + q), None
        else:
            d = int(rng.integers(3, 9))
            N -= N % 2
            E = inst.regular_graph(N, d, 710 + q)
            J, csr = None, inst.edges_to_csr(N, E, inst.gaussian_edges(len(E), 720 + q))
        items.append((J, csr, dict(R=8, runs=4, steps=120, seed=730 + q, jp_kind=sb.JP_PAPER)))
    alone = []
    for J, csr, kw in items:
        ctx = sb.sbqa_create(J=J, csr=csr, **kw)
        sb.sbqa_step(ctx, kw["steps"])
        alone.append(sb.sbqa_best(ctx))
        sb.sbqa_destroy(ctx)
    srv = sb.sbqa_server_create(96 << 20, 3)
    tickets = [sb.sbqa_submit(srv, J=J, csr=csr, **kw) for J, csr, kw in items]
    with pytest.raises(sb.SbqaError) as ei:   # real-valued J: float32 + float64 copies, 192 MiB
        sb.sbqa_submit(srv, J=inst.dense_gaussian(4096, 1), R=8, runs=4, steps=10, fmode=sb.F_BALLISTIC)
    assert ei.value.status == sb.EBUDGET
    import time
    got = {}
    t0 = time.time()
    while len(got) < len(tickets) and time.time() - t0 < 120:
        for t in tickets:
            if t not in got:
                r = sb.sbqa_poll(srv, t)
                if r is not None:
                    got[t] = r
        time.sleep(0.01)
    assert len(got) == len(tickets)
    lat = []
    for t, (Ea, sa) in zip(tickets, alone):
        Em, sm, l = got[t]
        assert np.array_equal(Ea, Em) and np.array_equal(sa, sm)
        lat.append(l)
    st = sb.sbqa_server_stats(srv)
    assert st["completed"] == len(items)
    _log("  serving latencies p50 %.3f s, max %.3f s" % (np.median(lat), np.max(lat)))
    sb.sbqa_server_destroy(srv)


def test_torch_stream_interop(sb):
    """The context can issue its work on a PyTorch stream."""
    import torch
    J = inst.sk_pm1(128, 80)
    X0, Y0 = inst.uniform_state(128, 8, 0.1, 81)
    outs = []
    for use in (False, True):
        ctx = _ctx(sb, J=J, R=4, runs=2, steps=20)
        if use:
            s = torch.cuda.Stream()
            sb.sbqa_set_stream(ctx, s)
        sb.sbqa_set_state(ctx, X0, Y0)
        sb.sbqa_step(ctx, 20)
        outs.append(sb.sbqa_get_state(ctx)[0])
    assert np.array_equal(outs[0], outs[1])


# ------------------------------------------------------------ resident loop
RESIDENT_CASES = [
    # name, N, degree, R, runs, fmode, energy_every
    ("bench_shape", 4096, 6, 32, 64, 0, 0),
    ("one_block_per_run", 1001, 6, 8, 7, 0, 0),
    ("two_blocks_sign", 700, 5, 16, 5, 1, 0),
    ("three_blocks_deg12_tracking", 2000, 12, 24, 3, 0, 7),
    ("small_ring_tracking", 333, 3, 8, 2, 0, 5),
    ("deg8_readout_row_pairs", 1500, 8, 8, 3, 0, 0),
    ("deg16_sign_tracking", 902, 16, 16, 2, 1, 9),
]


@pytest.mark.parametrize("name,N,d,R,runs,fmode,ee", RESIDENT_CASES)
def test_resident_loop_matches_streaming(sb, orc, name, N, d, R, runs, fmode, ee):
    """The register-resident CSR loop (many steps per launch, state in
    registers, ring edges exchanged between workgroups) computes exactly the
    bits of the one-launch-per-step kernel, over several launches, with energy
    tracking and a state overwrite in between; and one of its steps matches the
    oracle."""
    if d % 2 and N % 2:
        N += 1
    _log("resident vs streaming %s N=%d d=%d R=%d runs=%d" % (name, N, d, R, runs))
    E = inst.regular_graph(N, d, 5001)
    csr = inst.edges_to_csr(N, E, inst.gaussian_edges(len(E), 5002))
    h = inst.gaussian_fields(N, 0.1, 5003)
    S = 120
    out = {}
    for kern in (sb.LOOP_STREAM, sb.LOOP_RESIDENT):
        ctx = _ctx(sb, csr=csr, h=h, R=R, runs=runs, steps=S, fmode=fmode, loop_kernel=kern, seed=5004,
                   energy_every=ee, jp_kind=sb.JP_PAPER)
        assert sb.sbqa_info(ctx)["resident"] == (kern == sb.LOOP_RESIDENT)
        sb.sbqa_step(ctx, 37)
        mid = sb.sbqa_get_state(ctx)
        phi_mid = sb.sbqa_fields(ctx)
        sb.sbqa_step(ctx, 1)
        one = sb.sbqa_get_state(ctx)
        x, y = one
        sb.sbqa_set_state(ctx, x, y)
        best_set = sb.sbqa_best(ctx)       # signs from the state just written
        sb.sbqa_step(ctx, 50)
        sb.sbqa_step(ctx, S - 88)
        fin = sb.sbqa_get_state(ctx)
        best = sb.sbqa_best(ctx)           # signs the resident loop left
        out[kern] = (mid, one, fin, best, sb.sbqa_best_step(ctx), sb.sbqa_info(ctx)["c0"], phi_mid, best_set)
    a, b = out[sb.LOOP_STREAM], out[sb.LOOP_RESIDENT]
    assert np.array_equal(a[7][0], b[7][0]) and np.array_equal(a[7][1], b[7][1])
    for u, v in zip(a[:3], b[:3]):
        assert np.array_equal(u[0], v[0]) and np.array_equal(u[1], v[1])
    assert np.array_equal(a[3][0], b[3][0]) and np.array_equal(a[3][1], b[3][1])
    assert np.array_equal(a[4], b[4])
    assert np.array_equal(a[6], b[6])      # fields hook from the column-block state
    # one resident step (37 -> 38) against the oracle
    (X, Y), (xg, yg) = b[0], b[1]
    P = orc.Problem(N, R, runs, csr=csr, h=h, dt=0.5, a0=1.0, c0=b[5], fmode=fmode)
    ctx = _ctx(sb, csr=csr, h=h, R=R, runs=runs, steps=S, fmode=fmode, loop_kernel=sb.LOOP_RESIDENT, seed=5004,
               jp_kind=sb.JP_PAPER)
    jr = sb.sbqa_jperp_table(ctx)[:, 37].astype(np.float64)
    _check_step(orc, P, ctx, sb, X, Y, 37, S, jr, xg, yg, csr=csr, h=h)


SMALL_CASES = [
    # name, N, R, runs, fmode, energy_every
    ("sk64_cfg_shape", 64, 8, 4, 0, 0),
    ("sk100_sign_tracking", 100, 5, 3, 1, 7),
    ("sk128_max_elems", 128, 32, 2, 0, 13),
    ("sk1_degenerate", 1, 3, 2, 0, 0),
    # J in {-1, 0, +1}: the bit-mask coupling sum (the cases above take it
    # too: N = 100 and 128 with two waves per replica), except with more than
    # 8 replicas per thread (the last case: the float32 loop)
    ("bits32_partial_halfwaves", 32, 40, 2, 1, 9),
    ("bits20_padded_rows", 20, 100, 2, 0, 7),
    ("bits50_padded_rows_zeros", 50, 20, 3, 1, 0),
    ("bits32_max_elems", 32, 128, 1, 0, 0),
    ("bits64_max_elems_zeros", 64, 64, 2, 0, 11),
    ("bits64_ring_of_one", 64, 1, 3, 1, 0),
    ("bits90_two_waves_zeros", 90, 12, 2, 0, 6),
    ("fma20_many_replicas", 20, 200, 1, 0, 5),
]


@pytest.mark.parametrize("name,N,R,runs,fmode,ee", SMALL_CASES)
def test_small_dense_loop_matches_streaming(sb, orc, name, N, R, runs, fmode, ee):
    """The small dense loop (one workgroup per run, J and the run state in
    LDS, many steps per launch) against the one-launch-per-step MFMA kernel:
    with J in {-1,0,+1} and a ternary or sign operand both sum exact integers,
    so states, tracked best energies and best spins agree bit-for-bit; the
    first step also matches the oracle."""
    S = 60
    J = inst.sk_pm1(N, 5201) if N > 1 else np.zeros((1, 1))
    if name.endswith("_zeros"):     # ternary J: about half of the couplings 0
        keep = np.triu(np.random.default_rng(5205).random((N, N)) < 0.5, 1)
        J = J * (keep | keep.T)
    h = np.round(inst.gaussian_fields(N, 1.0, 5202))
    _log("small dense loop vs streaming %s N=%d R=%d runs=%d ee=%d" % (name, N, R, runs, ee))
    X0, Y0 = inst.uniform_state(N, R * runs, 0.2, 5203)
    out = {}
    for kern in (sb.LOOP_STREAM, sb.LOOP_RESIDENT):
        ctx = _ctx(sb, J=J, h=h, R=R, runs=runs, steps=S, fmode=fmode, precision=sb.PREC_FP8,
                   loop_kernel=kern, energy_every=ee)
        assert sb.sbqa_info(ctx)["resident"] == (kern == sb.LOOP_RESIDENT)
        sb.sbqa_set_state(ctx, X0, Y0)
        sb.sbqa_step(ctx, 1)
        first = sb.sbqa_get_state(ctx)
        sb.sbqa_step(ctx, 23)          # launches split at the energy_every boundaries
        sb.sbqa_step(ctx, S - 24)
        out[kern] = first + sb.sbqa_get_state(ctx) + sb.sbqa_best(ctx) + (sb.sbqa_best_step(ctx),)
    for a, b in zip(out[sb.LOOP_STREAM], out[sb.LOOP_RESIDENT]):
        assert np.array_equal(a, b)
    P = _orc_problem(orc, sb, ctx, J=J, h=h, fmode=fmode)
    jr = np.full(runs, 0.5)     # linear J_perp at step 0, exact in float32
    _check_step(orc, P, ctx, sb, X0, Y0, 0, S, jr, out[sb.LOOP_RESIDENT][0], out[sb.LOOP_RESIDENT][1], J=J, h=h)


_TILE_PROBE = """
import sys
sys.path.insert(0, %r)
import paper_2604_01050_amd as sb
import sbqa_instances as inst
ctx = sb.sbqa_create(J=inst.sk_pm1(1024, 5), R=16, runs=12, steps=10, precision=sb.PREC_FP8)
print("tile", sb.sbqa_info(ctx)["tile_cols"])
"""


def test_tile_choices_persist_across_processes(tmp_path):
    """The autotuned dense tile (C = 192: candidates of 64, 128 and 256
    columns) is appended to the tile file named by SBQA_TUNE_CACHE; the next
    process reads it back instead of timing again (nothing appended), uses an
    edited choice as long as it is one of the key's candidates, and skips
    malformed lines."""
    f = tmp_path / "tiles.txt"
    env = dict(os.environ, SBQA_TUNE_CACHE=str(f))

    def run():
        r = subprocess.run([sys.executable, "-c", _TILE_PROBE % ROOT], env=env, capture_output=True, text=True,
                           timeout=120)
        assert r.returncode == 0, r.stderr[-2000:]
        return int(r.stdout.split()[-1])

    _log("tile file across processes: %s" % f)
    t1 = run()
    lines = f.read_text().splitlines()
    assert len(lines) == 1 and lines[0].startswith("sbqa-tile-v1 ") and int(lines[0].split()[-1]) * 64 == t1
    assert run() == t1 and f.read_text().splitlines() == lines
    fields = lines[0].split()
    other = 1 if int(fields[-1]) != 1 else 4
    f.write_text("garbage\nsbqa-tile-v1 gfx950\n" + " ".join(fields[:-1] + [str(other)]) + "\n")
    assert run() == 64 * other
    f.write_text(" ".join(fields[:-1] + ["3"]) + "\n")     # not a candidate: timed again and appended
    assert run() in (64, 128, 256) and len(f.read_text().splitlines()) == 2


def test_resident_rejects_unfit_instances(sb):
    """LOOP_RESIDENT on an instance no resident loop can hold is EINVAL with a reason;
    AUTO then falls back to the streaming kernel."""
    E = inst.regular_graph(300, 4, 5101)
    csr = inst.edges_to_csr(300, E, inst.gaussian_edges(len(E), 5102))
    tri3 = dict(tri=np.array([[0, 1, 2], [5, 9, 200]]), K=np.array([1.0, -0.5]))
    for kw, why in ((dict(R=5, runs=4), "multiple of 8"), (dict(R=8, runs=2, fmode=sb.F_BALLISTIC), "ballistic"),
                    (dict(R=8, runs=2, **tri3), "three-body")):
        with pytest.raises(sb.SbqaError) as ei:
            _ctx(sb, csr=csr, loop_kernel=sb.LOOP_RESIDENT, **kw)
        assert ei.value.status == sb.EINVAL and why in ei.value.message
        ctx = _ctx(sb, csr=csr, **kw)
        assert not sb.sbqa_info(ctx)["resident"]
    # dense: the small loop holds N <= 128 and R*N <= 4096 in float32 only
    for J, kw, why in ((inst.sk_pm1(129, 5103), dict(R=4, runs=2), "N is above"),
                       (inst.sk_pm1(100, 5104), dict(R=41, runs=1), "R*N"),
                       (inst.dense_gaussian(64, 5105), dict(R=4, runs=2, fmode=sb.F_BALLISTIC,
                                                            precision=sb.PREC_BF16X3), "float32")):
        with pytest.raises(sb.SbqaError) as ei:
            _ctx(sb, J=J, loop_kernel=sb.LOOP_RESIDENT, **kw)
        assert ei.value.status == sb.EINVAL and why in ei.value.message, ei.value.message
        ctx = _ctx(sb, J=J, **kw)
        assert not sb.sbqa_info(ctx)["resident"]


def test_resident_wait_timeout_is_reported(sb):
    """Failure path of the resident sparse loop, forced from the host: with
    the device error word set as a ring-neighbour wait timeout sets it, the
    next launch runs through without waiting (every kernel ends normally) and
    the readout reports EDEVICE; a streaming context rejects the hook."""
    N = 512
    E = inst.regular_graph(N, 6, 9101)
    csr = inst.edges_to_csr(N, E, inst.gaussian_edges(len(E), 9102))
    ctx = _ctx(sb, csr=csr, R=8, runs=2, steps=40, loop_kernel=sb.LOOP_RESIDENT)
    _log("resident wait timeout injected: N=%d" % N)
    sb.sbqa_step(ctx, 5)
    sb.sbqa_best(ctx)                     # a healthy readout first
    sb.sbqa_inject_wait_timeout(ctx)
    sb.sbqa_step(ctx, 5)
    with pytest.raises(sb.SbqaError) as ei:
        sb.sbqa_best(ctx)
    assert ei.value.status == sb.EDEVICE and "timed out" in ei.value.message
    with pytest.raises(sb.SbqaError) as ei:
        sb.sbqa_sync(ctx)
    assert ei.value.status == sb.EDEVICE
    sb.sbqa_destroy(ctx)
    stream = _ctx(sb, csr=csr, R=8, runs=2, steps=40, loop_kernel=sb.LOOP_STREAM)
    with pytest.raises(sb.SbqaError) as ei:
        sb.sbqa_inject_wait_timeout(stream)
    assert ei.value.status == sb.EINVAL


def test_package_imported_before_torch_keeps_one_runtime(sb):
    """Imported before PyTorch, the binding still leaves one HIP runtime in
    the process (PyTorch's): in a fresh process that imports the package
    first, the benchmark's sparse shape runs the resident loop on a PyTorch
    stream and reads out."""
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = "\n".join([
        "import paper_2604_01050_amd as sb",
        "import torch",
        "import sbqa_instances as inst",
        "N = 4096",
        "E = inst.regular_graph(N, 6, 9001)",
        "csr = inst.edges_to_csr(N, E, inst.gaussian_edges(len(E), 9002))",
        "c = sb.sbqa_create(csr=csr, R=32, runs=64, steps=50, loop_kernel=sb.LOOP_RESIDENT)",
        "st = torch.cuda.Stream()",
        "sb.sbqa_set_stream(c, st)",
        "sb.sbqa_step(c, 5)",
        "E0, _ = sb.sbqa_best(c)",
        "print('resident', sb.sbqa_info(c)['resident'], bool(abs(E0[0]) < 1e12))",
        "sb.sbqa_destroy(c)"])
    _log("package imported before torch: fresh process, resident sparse N=4096")
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=110)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "resident True True" in r.stdout, r.stdout


# ------------------------------------------------------------ internal spin relabelling
@pytest.mark.gpu
@pytest.mark.parametrize("case", ["hubo_int", "ising_resident", "ising_stream"])
def test_internal_relabelling_is_invisible(sb, orc, case):
    """CSR spins relabelled internally (reverse Cuthill-McKee, REORDER_ON)
    against the given order (REORDER_OFF): the seeded initial state, the state
    after any number of steps, the fields and (integer weights) the best
    energies and spins are the same bit for bit, in the caller's spin order;
    real weights: best energies to 1e-12 (their FP64 sums run in another row
    order). sbqa_energy of given spins agrees with the oracle either way."""
    if case == "hubo_int":
        N, P2, w2, T, K = inst.hubo_heavy_hex(12, 12, 71, dist="int")
        csr = inst.edges_to_csr(N, P2, w2)
        h = np.round(inst.gaussian_fields(N, 2.0, 72))
        extra = dict(tri=T, K=K)
        R, runs = 8, 3
    else:
        N = 600
        E = inst.regular_graph(N, 3, 73)
        csr = inst.edges_to_csr(N, E, inst.gaussian_edges(len(E), 74))
        h = inst.gaussian_fields(N, 0.1, 75)
        extra = dict(loop_kernel=sb.LOOP_RESIDENT if case == "ising_resident" else sb.LOOP_STREAM)
        T = K = None
        R, runs = 8, 4
    S = 90
    _log("relabelling %s N=%d" % (case, N))
    out = {}
    for mode in (sb.REORDER_OFF, sb.REORDER_ON):
        ctx = _ctx(sb, csr=csr, h=h, R=R, runs=runs, steps=S, seed=7, energy_every=15, reorder=mode, **extra)
        assert sb.sbqa_info(ctx)["reordered"] == (mode == sb.REORDER_ON)
        r = [sb.sbqa_get_state(ctx)]
        sb.sbqa_step(ctx, 31)
        r += [sb.sbqa_get_state(ctx), sb.sbqa_fields(ctx)]
        sb.sbqa_step(ctx, S - 31)
        r += [sb.sbqa_get_state(ctx)]
        E, sp = sb.sbqa_best(ctx)
        spins = np.where(r[-1][0].T >= 0, 1, -1).astype(np.int8)[:5]
        out[mode] = (r, E, sp, sb.sbqa_energy(ctx, spins), spins)
        sb.sbqa_destroy(ctx)
    (ra, Ea, sa, ea, spins), (rb, Eb, sbest, eb, _) = out[sb.REORDER_OFF], out[sb.REORDER_ON]
    for u, v in zip(ra, rb):
        for a, b in zip(u if isinstance(u, tuple) else (u,), v if isinstance(v, tuple) else (v,)):
            assert np.array_equal(a, b)
    eo = orc.energy(spins, csr=csr, h=h, tri=T, K=K)
    if case == "hubo_int":
        assert np.array_equal(Ea, Eb) and np.array_equal(sa, sbest)
        assert np.array_equal(ea, eo) and np.array_equal(eb, eo)
    else:
        np.testing.assert_allclose(Eb, Ea, rtol=1e-12, atol=1e-12)
        assert np.array_equal(sa, sbest)
        np.testing.assert_allclose(ea, eo, rtol=1e-12)
        np.testing.assert_allclose(eb, eo, rtol=1e-12)
    # the served result of a relabelled instance equals the standalone one
    if case == "hubo_int":
        srv = sb.sbqa_server_create(1 << 28, 2)
        t = sb.sbqa_submit(srv, csr=csr, h=h, R=R, runs=runs, steps=S, seed=7, jp_kind=sb.JP_LINEAR, jp_start=0.5,
                           jp_end=0.0, energy_every=15, reorder=sb.REORDER_ON, tri=T, K=K)
        import time
        t0 = time.time()
        res = None
        while res is None and time.time() - t0 < 60:
            res = sb.sbqa_poll(srv, t)
            time.sleep(0.005)
        assert res is not None
        assert np.array_equal(res[0], Eb) and np.array_equal(res[1], sbest)
        sb.sbqa_server_destroy(srv)
