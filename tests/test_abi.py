"""C-ABI checks that need no GPU: the library loads, exports every entry point
that include/sbqa.h declares, and rejects invalid instances with EINVAL and a
message (validation runs before any device call)."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

import sbqa_instances as inst

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def abi():
    lib_path = os.path.join(ROOT, "paper_2604_01050_amd", "libsbqa.so")
    if not os.path.exists(lib_path):
        import importlib.util
        spec = importlib.util.spec_from_file_location("sbqa_build", os.path.join(ROOT, "paper_2604_01050_amd", "build.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.build()
    import paper_2604_01050_amd as p
    return p


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "sbqa.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sbqa_[a-z_]+)\s*\(", src)))


def test_header_symbols_exported(abi):
    names = _declared_functions()
    assert len(names) >= 20
    lib = ct.CDLL(abi.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    # the binding keeps the C names
    for n in names:
        assert hasattr(abi, n), n


def test_schedule_default_matches_paper_ranges(abi):
    s = abi.lib.sbqa_schedule_default()
    assert s.delta_max == 0.7                        # Eq. 8
    assert (s.beta_lo, s.beta_hi) == (0.5, 1.5)      # Sec. II.B
    assert (s.alpha_lo, s.alpha_hi) == (0.5, 1.0)
    assert s.jp_kind == abi.JP_PAPER and s.fmode == abi.F_TERNARY
    assert s.loop_kernel == abi.LOOP_AUTO and s.dense_tile == 0   # resident loops and tiles chosen by the library
    assert s.reorder == abi.REORDER_AUTO and s.j_packing == abi.JPACK_AUTO


def _expect(abi, status, **kw):
    with pytest.raises(abi.SbqaError) as ei:
        abi.sbqa_create(**kw)
    assert ei.value.status == status, ei.value
    assert ei.value.message
    return ei.value.message


def test_validation_errors(abi):
    J = inst.sk_pm1(16, 1)
    bad = J.copy()
    bad[2, 5] = 3.0
    assert "symmetric" in _expect(abi, abi.EINVAL, J=bad, R=2, runs=2)
    bad = J.copy()
    bad[3, 3] = 1.0
    assert "diagonal" in _expect(abi, abi.EINVAL, J=bad, R=2, runs=2)
    bad = J.copy()
    bad[1, 2] = bad[2, 1] = np.nan
    assert "finite" in _expect(abi, abi.EINVAL, J=bad, R=2, runs=2)
    _expect(abi, abi.EINVAL, J=J, R=0, runs=2)
    _expect(abi, abi.EINVAL, J=J, R=2, runs=2, steps=0)
    _expect(abi, abi.EINVAL, J=J, R=2, runs=2, dt=-1.0)
    # FP8 needs J in {-1,0,1} and a discrete f
    _expect(abi, abi.EINVAL, J=J * 2, R=2, runs=2, precision=abi.PREC_FP8)
    _expect(abi, abi.EINVAL, J=J, R=2, runs=2, precision=abi.PREC_FP8, fmode=abi.F_BALLISTIC)
    _expect(abi, abi.EINVAL, J=J * 0.5, R=2, runs=2, precision=abi.PREC_INT8)
    assert "FP4" in _expect(abi, abi.EINVAL, J=J * 2, R=2, runs=2, precision=abi.PREC_FP4)
    _expect(abi, abi.EINVAL, J=J, R=2, runs=2, precision=abi.PREC_FP4, fmode=abi.F_BALLISTIC)
    assert "127" in _expect(abi, abi.EINVAL, J=J * 128, R=2, runs=2, precision=abi.PREC_INT8)
    _expect(abi, abi.EINVAL, J=J * 28, R=2, runs=2, precision=abi.PREC_INT8, fmode=abi.F_BALLISTIC)
    assert "precision" in _expect(abi, abi.EINVAL, J=J, R=2, runs=2, precision=6)
    assert "dense_tile" in _expect(abi, abi.EINVAL, J=J, R=2, runs=2, dense_tile=96)
    assert "loop_kernel" in _expect(abi, abi.EINVAL, J=J, R=2, runs=2, loop_kernel=7)
    assert "j_packing" in _expect(abi, abi.EINVAL, J=J, R=2, runs=2, j_packing=2)
    assert "reorder" in _expect(abi, abi.EINVAL, J=J, R=2, runs=2, reorder=3)
    # CSR: asymmetric, out of range, unsorted, bf16 precision
    E = inst.regular_graph(20, 3, 2)
    rp, col, val = inst.edges_to_csr(20, E, inst.gaussian_edges(len(E), 3))
    v2 = val.copy()
    v2[0] += 1.0
    assert "symmetric" in _expect(abi, abi.EINVAL, csr=(rp, col, v2), R=2, runs=2)
    c2 = col.copy()
    c2[0] = 99
    _expect(abi, abi.EINVAL, csr=(rp, c2, val), R=2, runs=2)
    c3 = col.copy()
    c3[0], c3[1] = c3[1], c3[0]
    _expect(abi, abi.EINVAL, csr=(rp, c3, val), R=2, runs=2)
    _expect(abi, abi.EINVAL, csr=(rp, col, val), R=2, runs=2, precision=abi.PREC_BF16X3)
    # an interior row_ptr entry past nnz (later entries decrease again): rejected before
    # any col or val entry outside the caller's nnz-long arrays is read
    bad_rp = np.array([0, 100, 5], dtype=np.int32)
    assert "row_ptr" in _expect(abi, abi.EINVAL, csr=(bad_rp, np.array([1, 1, 1, 0, 0], dtype=np.int32),
                                                      np.ones(5)), R=2, runs=2)
    assert "row_ptr" in _expect(abi, abi.EINVAL, csr=(np.array([0, -2, 2], dtype=np.int32),
                                                      np.array([1, 0], dtype=np.int32), np.ones(2)), R=2, runs=2)
    # three-body terms: CSR only, indices in range and distinct, finite weights
    T = np.array([[0, 1, 2], [3, 4, 5]])
    Kw = np.array([1.0, -2.0])
    assert "CSR" in _expect(abi, abi.EINVAL, J=J, R=2, runs=2, tri=T, K=Kw)
    assert "range" in _expect(abi, abi.EINVAL, csr=(rp, col, val), R=2, runs=2, tri=T + 17, K=Kw)
    assert "repeats" in _expect(abi, abi.EINVAL, csr=(rp, col, val), R=2, runs=2, tri=[[0, 1, 1]], K=[1.0])
    assert "finite" in _expect(abi, abi.EINVAL, csr=(rp, col, val), R=2, runs=2, tri=T, K=[1.0, np.inf])
    # schedule table must be given for JP_TABLE
    _expect(abi, abi.EINVAL, J=J, R=2, runs=2, jp_kind=abi.JP_TABLE)


def test_noalloc_energy_argument_errors(abi):
    """The allocation-free energy entry point checks its arguments before any
    device work."""
    assert abi.lib.sbqa_energy_noalloc(None, None, 1, None) == abi.EINVAL
    assert abi.lib.sbqa_energy_noalloc(None, None, 0, None) == abi.EINVAL
    assert "NULL" in abi.sbqa_last_error()


def test_inject_wait_timeout_argument_errors(abi):
    """The failure-path hook rejects a NULL context before any device work."""
    assert abi.lib.sbqa_inject_wait_timeout(None) == abi.EINVAL
    assert "NULL" in abi.sbqa_last_error()


def test_server_argument_errors(abi):
    with pytest.raises(abi.SbqaError):
        abi.sbqa_server_create(0, 4)
    with pytest.raises(abi.SbqaError):
        abi.sbqa_server_create(1 << 20, 0)
