"""Host-side logic of bench.py (no GPU): the one-GPU contract, the algorithmic
work the roofline figures are computed from, and the committed counter
summaries being used only for the kernel source they were measured on."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    """--gpus N > 1 exits with status 2 and a message, before touching a GPU."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_sparse_algorithmic_bytes_and_ops():
    """Random 6-regular N = 4096, R = 32 x 64 runs: per step the streaming
    kernel must read and write x and y (fp32) and write and read the int8
    operand once (18 B per replica-spin), plus the CSR arrays and h; the
    resident loop must do one FMA per neighbour and 13 more operations per
    update."""
    import bench
    w = bench.make_workload("sparse6")
    N, C = 4096, 32 * 64
    nnz = N * 6
    assert len(w["csr"][1]) == nnz
    expect = N * C * 18 + 4 * (N + 1) + 8 * nnz + 4 * N
    assert bench.algorithmic_bytes(w, {"path": "csr_fp32"}) == expect == 151224324
    assert bench.resident_ops_per_step(w) == nnz * C + 13 * N * C


def test_dense_algorithmic_flops():
    import bench
    w = {"N": 1000, "R": 4, "runs": 3}
    assert bench.algorithmic_flops(w) == 2.0 * 1000 * 1000 * 12


def test_committed_traffic_used_only_for_its_source(tmp_path, monkeypatch):
    """Every committed traffic summary names the source hash it was measured
    on; bench.py reports its bytes while the hash matches and null once the
    kernel source differs (checked on a copy with a changed source)."""
    import bench
    seen = 0
    for name in sorted(os.listdir(os.path.join(ROOT, "profiles"))):
        if not name.startswith("traffic_"):
            continue
        kv = {}
        for line in open(os.path.join(ROOT, "profiles", name)):
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
        srcs = kv["source"].split()
        path = [p for p, files in bench.KERNEL_SOURCES.items() if files == srcs][0]
        workload = name[len("traffic_"):-len(".txt")]
        got = bench.measured_traffic(workload, path)
        if kv["source_sha256_16"] != bench.source_hash(srcs):
            assert got is None          # measured on another source: reported as null
            continue
        assert got == float(kv.get("hbm_bytes_per_launch", kv.get("hbm_bytes_per_step")))
        seen += 1
    assert seen >= 1
    # a changed kernel source invalidates the summary
    fake = tmp_path / "repo"
    shutil.copytree(os.path.join(ROOT, "profiles"), fake / "profiles")
    src = fake / "paper_2604_01050_amd" / "csrc"
    src.mkdir(parents=True)
    for f in bench.KERNEL_SOURCES["csr_resident"]:
        data = open(os.path.join(ROOT, f), "rb").read()
        (fake / f).write_bytes(data + b"\n// changed\n")
    monkeypatch.setattr(bench, "ROOT", str(fake))
    assert bench.measured_traffic("sparse6_resident", "csr_resident") is None


def test_dense_kernel_name():
    """Bit-packed J at the 128-column tile runs split-K when the K chunks
    split into two even halves (the library's launch rule)."""
    import bench
    base = {"N": 16384, "path": "dense_fp4_packed", "tile_cols": 128}
    assert bench.dense_kernel_name(base) == "k_dense_step_sk"
    assert bench.dense_kernel_name(dict(base, path="dense_fp8_packed", N=2000)) == "k_dense_step_sk"
    assert bench.dense_kernel_name(dict(base, N=1500)) == "k_dense_step"       # fp4: 6 chunks of 256
    assert bench.dense_kernel_name(dict(base, path="dense_fp8_packed", N=300)) == "k_dense_step_sk"   # 4 of 128
    assert bench.dense_kernel_name(dict(base, tile_cols=256)) == "k_dense_step"
    assert bench.dense_kernel_name(dict(base, path="dense_int8")) == "k_dense_step"
    # two J planes (bf16 hi+lo) at the 128-column tile: two column groups per
    # workgroup when the padded columns make whole 256-column pairs
    bf = {"N": 8192, "path": "dense_bf16x3", "tile_cols": 128, "R": 16, "runs": 32}
    assert bench.dense_kernel_name(bf) == "k_dense_step_cg2"
    assert bench.dense_kernel_name(dict(bf, runs=8)) == "k_dense_step"          # C = 128: one chunk
    assert bench.dense_kernel_name(dict(bf, runs=12)) == "k_dense_step_cg2"     # C = 192 -> 256
    assert bench.dense_kernel_name(dict(bf, tile_cols=64)) == "k_dense_step"


def test_small_kernel_name():
    """The small dense loop counts bits for J in {-1, 0, +1} with a ternary or
    sign operand and at most 8 replicas per thread; else it sums floats."""
    import numpy as np
    import bench
    w = bench.make_workload("sk64")
    assert bench.small_kernel_name(w) == "k_dense_small_bits"
    assert bench.small_kernel_name(dict(w, fmode=2)) == "k_dense_small"         # ballistic operand
    J2 = w["J"].copy()
    J2[0, 1] = J2[1, 0] = 2.0
    assert bench.small_kernel_name(dict(w, J=J2)) == "k_dense_small"            # |J| = 2
    assert bench.small_kernel_name(dict(w, R=64)) == "k_dense_small_bits"       # 8 per thread
    assert bench.small_kernel_name(dict(w, R=65)) == "k_dense_small"            # 9 per thread
    w20 = dict(w, N=20, J=np.zeros((20, 20)))
    assert bench.small_kernel_name(dict(w20, R=128)) == "k_dense_small_bits"    # 16 per 512 threads
    assert bench.small_kernel_name(dict(w20, R=129)) == "k_dense_small"


def test_dense_traffic_summaries_name_the_launched_kernel():
    """The committed counter summaries of the SK N = 16384 packed-J workloads
    and of the Gaussian N = 8192 bf16 hi+lo workload (taken at the 128-column
    tile) name the kernel the launch rule selects."""
    import bench
    for workload, info in (("sk_fp8", {"N": 16384, "path": "dense_fp8_packed", "R": 16, "runs": 16}),
                           ("sk_fp4", {"N": 16384, "path": "dense_fp4_packed", "R": 16, "runs": 16}),
                           ("gauss_bf16x3", {"N": 8192, "path": "dense_bf16x3", "R": 16, "runs": 32})):
        kv = {}
        for line in open(os.path.join(ROOT, "profiles", "traffic_%s.txt" % workload)):
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
        assert kv["kernel"] == bench.dense_kernel_name(dict(info, tile_cols=128))


def test_unknown_workload_is_rejected():
    import bench
    with pytest.raises(SystemExit):
        bench.make_workload("no_such_workload")
