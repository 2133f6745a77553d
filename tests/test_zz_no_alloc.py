"""sbqa_energy_noalloc, the allocation-free variant of sbqa_energy, through
the C ABI: device input and output buffers, scratch in the library's static
per-GPU array. Its energies must equal sbqa_energy's bit for bit (the same
kernels in the same order) on two calls in a row, the second one smaller, so
that whatever the first call left in the shared scratch cannot leak into the
second; and sizes above the scratch limit or host pointers are rejected."""
import numpy as np
import pytest

import sbqa_instances as inst

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)
    import paper_2604_01050_amd as sb
    return sb


def _log(msg):
    print(msg, flush=True)


def _instance(sb, case, N):
    if case == "dense_pm1_fp8":
        return dict(J=inst.sk_pm1(N, 9101), h=None, precision=sb.PREC_FP8)
    if case == "dense_gauss_fp32":
        return dict(J=inst.dense_gaussian(N, 9102), h=inst.gaussian_fields(N, 0.3, 9103), precision=sb.PREC_FP32,
                    fmode=sb.F_BALLISTIC)
    if case == "csr_gauss":
        E = inst.regular_graph(N, 5, 9104)
        return dict(csr=inst.edges_to_csr(N, E, inst.gaussian_edges(len(E), 9105)), h=inst.gaussian_fields(N, 0.1, 9106))
    if case == "csr_hubo_relabelled":
        n, P2, w2, T, K = inst.hubo_heavy_hex(N, N, 9107, dist="normal")
        return dict(csr=inst.edges_to_csr(n, P2, w2), tri=T, K=K, h=None, reorder=sb.REORDER_ON)
    raise ValueError(case)


def _run(sb, ctx, spins):
    import torch
    ds = torch.from_numpy(np.ascontiguousarray(spins)).cuda()
    out = torch.full((spins.shape[0],), float("nan"), dtype=torch.float64, device="cuda")
    sb.sbqa_energy_noalloc(ctx, ds.data_ptr(), spins.shape[0], out.data_ptr())
    torch.cuda.synchronize()
    return out.cpu().numpy()


# case, (N first context, count first call), (N second context, count second call)
CASES = [
    ("dense_pm1_fp8", (1000, 70), (300, 3)),
    ("dense_gauss_fp32", (1500, 130), (1500, 9)),
    ("csr_gauss", (2000, 64), (500, 2)),
    ("csr_hubo_relabelled", (14, 40), (9, 5)),
]


@pytest.mark.parametrize("case,first,second", CASES)
def test_noalloc_energy_equals_sbqa_energy(sb, case, first, second):
    import torch
    results = []
    for q, (N, count) in enumerate((first, second)):
        kw = _instance(sb, case, N)
        _log("noalloc energy %s call %d N=%d count=%d" % (case, q, N, count))
        ctx = sb.sbqa_create(R=8, runs=2, steps=10, jp_kind=sb.JP_LINEAR, jp_start=0.5, jp_end=0.0, **kw)
        if case == "csr_hubo_relabelled":
            assert sb.sbqa_info(ctx)["reordered"]
        sb.sbqa_set_stream(ctx, torch.cuda.current_stream())
        spins = inst.spins_pm1(count, ctx.N, 9200 + q)
        got = _run(sb, ctx, spins)
        want = sb.sbqa_energy(ctx, spins)
        assert np.array_equal(got, want), (case, q, np.max(np.abs(got - want)))
        results.append(got)
        sb.sbqa_destroy(ctx)
    assert len(results[1]) < len(results[0])


def test_noalloc_energy_rejects_oversize_and_host_pointers(sb):
    import torch
    N = 2048
    ctx = sb.sbqa_create(J=inst.sk_pm1(N, 9301), R=8, runs=1, steps=10, precision=sb.PREC_FP8)
    sb.sbqa_set_stream(ctx, torch.cuda.current_stream())
    count = 4200          # float64 spin matrix and GEMM partials above the scratch limit
    ds = torch.ones((count, N), dtype=torch.int8, device="cuda")
    out = torch.empty(count, dtype=torch.float64, device="cuda")
    with pytest.raises(sb.SbqaError) as ei:
        sb.sbqa_energy_noalloc(ctx, ds.data_ptr(), count, out.data_ptr())
    assert ei.value.status == sb.EINVAL and "scratch" in ei.value.message
    host = np.ones((2, N), dtype=np.int8)
    with pytest.raises(sb.SbqaError) as ei:
        sb.sbqa_energy_noalloc(ctx, host.ctypes.data, 2, out.data_ptr())
    assert ei.value.status == sb.EINVAL and "device memory" in ei.value.message
    # a call that fits still works after the rejected ones
    spins = inst.spins_pm1(3, N, 9302)
    assert np.array_equal(_run(sb, ctx, spins), sb.sbqa_energy(ctx, spins))
    sb.sbqa_destroy(ctx)
