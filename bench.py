"""Benchmark of the SBQA time-stepping loop on one MI355X.

Default workload (the configuration the replica-spin-update metric is quoted
on): random 6-regular graph, N = 4096, J_e ~ N(0,1) on the edges,
h_i ~ N(0, 0.1^2), R = 32 replicas x 64 runs (C = 2048 columns), 5000 steps,
dt = 0.5, a0 = 1, c0 = 0.5/(sqrt(N) rms J), ternary f (Eq. 8), J_perp linear
0.5 -> 0, x, y ~ U[-0.1, 0.1]; fp32 CSR contraction fused with the update.

A bench "step" is one SBQA time step over all runs and replicas (operand,
contraction, update). The timed region is K steps of a fresh solve followed by
the readout (energies of all replicas and the best per run). value =
N*R*runs*K / seconds. The dominant kernel's average duration comes from one
HIP event pair around the K steps on the context's stream (each step is one
launch of that kernel, or all K steps are one resident launch); its roofline uses the
algorithmic bytes (HBM-bound kernels) or operations (MFMA and VALU-bound
kernels) per launch computed below.

The default line also carries "configs", the other configurations measured
on the same GPU in the same run, each with its own step count, step time,
roofline and readout: SK N = 64 (small resident loop), SK N = 16384 on the fp8
and fp4 paths (bit-packed J) against the plain fp32 path, Gaussian N = 8192 on
the split-bf16 path against fp32 with the single-step field error of both
against the float64 product on sampled rows, and the mixed serving stream of
512 instances (Poisson arrivals at 0.8 of the measured service rate) with its
p50/p99 solve latency, the second half of the metric.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                       [--no-cpu-baseline] [--no-configs] [--no-serve]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PEAK = {"fp4": 10060.0, "fp8": 5030.0, "int8": 5030.0, "bf16": 2520.0, "fp32": 157.3, "fp64": 78.6}  # T(FL)OP/s dense MFMA


_CACHE = {}


def _cached(key, fn):
    """Large generated matrices shared by several workloads of one run."""
    if key not in _CACHE:
        _CACHE[key] = fn()
    return _CACHE[key]


def make_workload(name: str):
    import sbqa_instances as inst
    if name == "sparse6":
        N, d, R, runs, S = 4096, 6, 32, 64, 5000
        E = inst.regular_graph(N, d, 2001)
        csr = inst.edges_to_csr(N, E, inst.gaussian_edges(len(E), 2002))
        h = inst.gaussian_fields(N, 0.1, 2003)
        desc = ("random 6-regular N=4096, J~N(0,1) on edges, h~N(0,0.1^2), R=32 x 64 runs, "
                "5000 steps, dt=0.5, ternary f, J_perp linear 0.5->0, fp32 CSR")
        return dict(csr=csr, h=h, N=N, R=R, runs=runs, S=S, prec=None, fmode=0, desc=desc, d=d, dtype="f32")
    if name in ("sk_fp4", "sk_fp4_bytes"):
        N, R, runs, S = 16384, 16, 16, 10000
        packed = name == "sk_fp4"
        return dict(J=_cached("sk16384", lambda: inst.sk_pm1(N, 3001)), h=None, N=N, R=R, runs=runs, S=S, prec="PREC_FP4", fmode=0,
                    j_packing=None if packed else "JPACK_BYTES",
                    desc="SK N=16384 J=+-1 (%s), R=16 x 16 runs, 10000 steps, ternary f"
                         % ("1 bit per coupling, e2m1 fp4 MFMA" if packed else "e2m1 nibbles"), dtype="fp4")
    if name in ("sk_fp8", "sk_fp8_bytes"):
        N, R, runs, S = 16384, 16, 16, 10000
        packed = name == "sk_fp8"
        return dict(J=_cached("sk16384", lambda: inst.sk_pm1(N, 3001)), h=None, N=N, R=R, runs=runs, S=S, prec="PREC_FP8", fmode=0,
                    j_packing=None if packed else "JPACK_BYTES",
                    desc="SK N=16384 J=+-1 (%s), R=16 x 16 runs, 10000 steps, ternary f"
                         % ("1 bit per coupling, e4m3 MFMA" if packed else "e4m3 bytes"), dtype="fp8")
    if name in ("sidon_i8", "sidon_fp32"):
        # integer couplings of the QAC benchmarks (Sidon28 set x 28), dense at the SK size
        N, R, runs, S = 16384, 16, 16, 10000
        i8 = name == "sidon_i8"
        return dict(J=inst.sidon28_dense(N, 3101), h=None, N=N, R=R, runs=runs, S=S,
                    prec="PREC_INT8" if i8 else "PREC_FP32", fmode=0,
                    desc="dense N=16384 J in 28 x Sidon28 = {+-8,+-13,+-19,+-28} (%s), R=16 x 16 runs, "
                         "10000 steps, ternary f" % ("int8" if i8 else "fp32 path"), dtype="int8" if i8 else "f32")
    if name == "sk_fp32":
        N, R, runs, S = 16384, 16, 16, 10000
        return dict(J=_cached("sk16384", lambda: inst.sk_pm1(N, 3001)), h=None, N=N, R=R, runs=runs, S=S, prec="PREC_FP32", fmode=0,
                    desc="SK N=16384 J=+-1 (fp32 path), R=16 x 16 runs, 10000 steps, ternary f", dtype="f32")
    if name == "gauss_bf16x3":
        N, R, runs, S = 8192, 16, 32, 5000
        return dict(J=_cached("gauss8192", lambda: inst.dense_gaussian(N, 4001)), h=None, N=N, R=R, runs=runs, S=S, prec="PREC_BF16X3",
                    fmode=2, desc="dense N=8192 J~N(0,1), ballistic, bf16 hi+lo, R=16 x 32 runs, 5000 steps",
                    dtype="bf16x3")
    if name == "gauss_fp32":
        N, R, runs, S = 8192, 16, 32, 5000
        return dict(J=_cached("gauss8192", lambda: inst.dense_gaussian(N, 4001)), h=None, N=N, R=R, runs=runs, S=S, prec="PREC_FP32",
                    fmode=2, desc="dense N=8192 J~N(0,1), ballistic, fp32, R=16 x 32 runs, 5000 steps",
                    dtype="f32")
    if name in ("cubic88", "square800"):
        # large sparse lattices (Sec. III: cubic and square lattice families up to ~7e5 spins),
        # many runs batched; Gaussian couplings on the bonds, h ~ N(0, 0.1^2)
        L = 88 if name == "cubic88" else 800
        E = inst.cubic_lattice(L) if name == "cubic88" else inst.square_lattice(L)
        N = L ** 3 if name == "cubic88" else L * L
        csr = inst.edges_to_csr(N, E, inst.gaussian_edges(len(E), 2101))
        h = inst.gaussian_fields(N, 0.1, 2102)
        R, runs, S = 16, 8, 1000
        desc = ("%s lattice L=%d (N=%d), J~N(0,1) on bonds, h~N(0,0.1^2), R=16 x 8 runs, 1000 steps, "
                "ternary f, fp32 CSR" % ("cubic" if name == "cubic88" else "square", L, N))
        return dict(csr=csr, h=h, N=N, R=R, runs=runs, S=S, prec=None, fmode=0, desc=desc,
                    d=6 if name == "cubic88" else 4, dtype="f32")
    if name == "hubo_hh":
        # native three-body instance on a heavy-hex graph (Sec. III.B HUBO family, scaled up):
        # 200 x 200 honeycomb with a site on every bond, one matching of 2-body terms and six
        # sets of vertex-disjoint 3-body paths, N(0,1) weights
        N, P2, w2, T, K = inst.hubo_heavy_hex(200, 200, 2301, dist="normal")
        R, runs, S = 16, 8, 1000
        desc = ("heavy-hex HUBO N=%d (%d 2-body, %d 3-body terms, N(0,1)), R=16 x 8 runs, 1000 steps, "
                "ternary f, fp32 CSR + 3-body lists" % (N, len(P2), len(T)))
        return dict(csr=inst.edges_to_csr(N, P2, w2), tri=T, K=K, h=None, N=N, R=R, runs=runs, S=S, prec=None,
                    fmode=0, desc=desc, d=2, dtype="f32")
    if name == "sk64":
        N, R, runs, S = 64, 8, 4, 1000
        return dict(J=inst.sk_pm1(N, 1001), h=None, N=N, R=R, runs=runs, S=S, prec="PREC_FP32", fmode=0,
                    desc="SK N=64, R=8 x 4 runs, 1000 steps, fp32", dtype="f32")
    raise SystemExit("unknown workload " + name)


def create(sb, w, seed, loop_kernel="auto"):
    kw = dict(R=w["R"], runs=w["runs"], steps=w["S"], dt=0.5, a0=1.0, fmode=w["fmode"],
              jp_kind=sb.JP_LINEAR, jp_start=0.5, jp_end=0.0, seed=seed, init_amp=0.1,
              loop_kernel={"auto": sb.LOOP_AUTO, "stream": sb.LOOP_STREAM, "resident": sb.LOOP_RESIDENT}[loop_kernel])
    if w["prec"]:
        kw["precision"] = getattr(sb, w["prec"])
    if w.get("j_packing"):
        kw["j_packing"] = getattr(sb, w["j_packing"])
    if w.get("dense_tile"):
        kw["dense_tile"] = w["dense_tile"]
    return sb.sbqa_create(J=w.get("J"), csr=w.get("csr"), h=w.get("h"), tri=w.get("tri"), K=w.get("K"), **kw)


def algorithmic_bytes(w, info):
    """Bytes the dominant kernel must move per launch (one step)."""
    N, C = w["N"], w["R"] * w["runs"]
    if info["path"] == "csr_fp32":
        nnz = len(w["csr"][1])
        # x, y read + write (fp32) + int8 operand written once and read once
        b = N * C * (16 + 2) + 4 * (N + 1) + 8 * nnz + 4 * N
        if w.get("K") is not None:   # three-body lists: per member entry two indices and a weight
            b += 4 * (N + 1) + 3 * len(w["K"]) * 12
        return b
    eb = {"dense_fp8": 1, "dense_fp8_packed": 1, "dense_int8": 1, "dense_fp4": 0.5, "dense_fp4_packed": 0.5,
          "dense_fp32": 4, "dense_bf16x3": 4}[info["path"]]
    jb = N * N / 8 if info["path"].endswith("_packed") else N * N * eb
    # GEMM: J streamed once + operand read once + fp32 field partial written
    return jb + C * N * eb + C * N * 4


# VALU peak of MI355X in fp32 lane operations: 256 CUs x 4 SIMDs x 16 lanes x
# 2.4 GHz = 39.3 Tops/s, one operation per lane per cycle (the 157.3 TFLOP/s
# fp32 vector figure counts an FMA as two flops and needs packed fp32, which
# the library is compiled without).
PEAK_VALU_OPS = 256 * 4 * 16 * 2.4e9 / 1e12


def resident_ops_per_step(w):
    """VALU lane operations one step of a resident loop must perform per
    replica-spin update: one FMA per coupling of the row (d for a sparse row,
    N for the small dense loop; the operand -1/0/+1 is read by the FMA in a
    format it takes directly, no conversion), 7 for the kick and drift, 3 for
    the wall, 3 for the ternary decision of Eq. 8: d + 13 (or N + 13). The
    peak counts one lane operation per lane per cycle, an FMA being one. The
    count is the algorithmic unit: the bit-mask small loop forms the N-term
    sum with about a dozen bit operations and still counts N."""
    N, C = w["N"], w["R"] * w["runs"]
    nnz = len(w["csr"][1]) if "csr" in w else N * N
    return 1.0 * nnz * C + 13.0 * N * C


def small_kernel_name(w):
    """The small dense loop's kernel (the library's launch rule): the
    bit-mask form for J in {-1, 0, +1} and a ternary or sign operand when the
    replicas fill at most 8 groups of N rounded up to 32, 64 or 128 lanes per
    thread, else the float32 form."""
    J, N = w.get("J"), w["N"]
    lanes = 32 if N <= 32 else 64 if N <= 64 else 128
    per_thread = -(-w["R"] // (512 // lanes))
    bits = (J is not None and w.get("fmode", 0) != 2 and per_thread <= 8
            and bool(np.isin(J, (-1.0, 0.0, 1.0)).all()))
    return "k_dense_small_bits" if bits else "k_dense_small"


def dense_kernel_name(info):
    """The dense step kernel the library launches: bit-packed +-1 J at the
    128-column tile runs as the split-K kernel when the K chunks (128 spins
    each in fp8, 256 in fp4; spins padded to a multiple of 512) split into
    two halves of an even count."""
    Np = -(-info["N"] // 512) * 512
    nkc = {"dense_fp8_packed": Np // 128, "dense_fp4_packed": Np // 256}.get(info["path"], 1)
    split = info["path"] in ("dense_fp8_packed", "dense_fp4_packed") and info["tile_cols"] == 128 and nkc % 4 == 0
    if split:
        return "k_dense_step_sk"
    # two J planes at the 128-column tile: two column groups per workgroup
    # when the padded columns make whole pairs of 128-column chunks
    if info["path"] == "dense_bf16x3" and info["tile_cols"] == 128:
        cg = -(-(info["R"] * info["runs"]) // 128) * 128
        if cg % 256 == 0:
            return "k_dense_step_cg2"
    return "k_dense_step"


def algorithmic_flops(w):
    N, C = w["N"], w["R"] * w["runs"]
    return 2.0 * N * N * C


_CS = "paper_2604_01050_amd/csrc/"
# Source files that hold each dominant kernel's code (the kernel file and the
# device helpers it includes); counter summaries record their hash.
KERNEL_SOURCES = {"csr_fp32": [_CS + "kernels_csr.hip", _CS + "csr_common.h"],
                  "csr_resident": [_CS + "kernels_resident.hip", _CS + "csr_common.h"]}
for _p in ("dense_fp8", "dense_fp8_packed", "dense_int8", "dense_fp4", "dense_fp4_packed", "dense_fp32",
           "dense_bf16x3"):
    KERNEL_SOURCES[_p] = [_CS + "kernels_dense.hip"]


def source_hash(paths):
    """First 16 hex digits of the sha256 of the concatenated files."""
    import hashlib
    h = hashlib.sha256()
    for path in paths:
        with open(os.path.join(ROOT, path), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, path):
    """HBM bytes per launch (or per step, for the many-step resident loop) of
    the dominant kernel from the committed counter summary (rocprofv3
    FETCH_SIZE + WRITE_SIZE, scaled by a copy kernel of known size); None when
    absent or taken on a different kernel source."""
    f = os.path.join(ROOT, "profiles", "traffic_%s.txt" % workload)
    if not os.path.exists(f):
        return None
    kv = {}
    for line in open(f):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256_16") != source_hash(KERNEL_SOURCES[path]):
        return None
    try:
        return float(kv.get("hbm_bytes_per_launch", kv.get("hbm_bytes_per_step")))
    except (TypeError, ValueError):
        return None


def copy_calibration():
    """A plain copy of known size (256 MiB read + 256 MiB written), three times,
    for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copy calibration: 3 x copy of %d bytes" % (a.numel() * 4), flush=True)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, window_s=5.0, windows=3, single_s=4.0):
    """The FP64 oracle on the host cores over the first steps of the same
    workload (inputs from the shared generators, c0 and J_perp from the
    oracle): the median rate of three consecutive windows on all threads, then
    a shorter window on one thread."""
    import oracle
    import sbqa_instances as inst
    oracle.build()
    N, R, runs, S = w["N"], w["R"], w["runs"], w["S"]
    P = oracle.Problem(N, R, runs, J=w.get("J"), csr=w.get("csr"), h=w.get("h"), dt=0.5, a0=1.0, c0=None,
                       fmode=w["fmode"], tri=w.get("tri"), K=w.get("K"))
    jt = oracle.jperp_linear_table(0.5, 0.0, S)
    X0, Y0 = inst.uniform_state(N, R * runs, 0.1, 99)
    X, Y = X0.astype(np.float64), Y0.astype(np.float64)
    n, rates, counts = 0, [], []
    for _ in range(windows):
        t0, k = time.perf_counter(), 0
        while n < S and (time.perf_counter() - t0) < window_s:
            X, Y = P.step(X, Y, oracle.pump(n, S), oracle.delta32(0.7, n, S), np.full(runs, jt[n]))
            n += 1
            k += 1
        if k:
            rates.append(N * R * runs * k / (time.perf_counter() - t0))
            counts.append(k)
    cores = oracle.num_threads()
    # one thread, continuing from the state reached
    oracle.set_threads(1)
    t1, n1 = time.perf_counter(), 0
    while n + n1 < S and (time.perf_counter() - t1) < single_s:
        X, Y = P.step(X, Y, oracle.pump(n + n1, S), oracle.delta32(0.7, n + n1, S), np.full(runs, jt[n + n1]))
        n1 += 1
    d1 = time.perf_counter() - t1
    oracle.set_threads(cores)
    out = {"value": float(np.median(rates)), "unit": "replica-spin updates/s", "cores": cores,
           "kind": "oracle",
           "sample": "the first %d of %d steps of the same workload in %d consecutive window%s of about %.0f s "
                     "(%s steps), median rate (FP64 C oracle, OpenMP)"
                     % (n, S, len(rates), "s" if len(rates) != 1 else "", window_s,
                        "/".join(str(c) for c in counts)),
           "windows": rates, "cpu_model": _cpu_model(), "compile_flags": " ".join(oracle.CFLAGS)}
    if n1:
        out["single_thread"] = {"value": N * R * runs * n1 / d1, "sample": "the next %d steps on one thread" % n1}
    return out


# ------------------------------------------------------------------ serving
def serve_instances(n, seed):
    """Mixed stream of the serving configuration: N log-uniform in
    [256, 8192] (even), half dense SK +-1 (FP8 path, h = 0), half random
    d-regular graphs with d ~ U{3..12} and J ~ N(0,1) (h = 0); R = 16, 8 runs,
    2000 steps. Dense instances are principal submatrices of one SK +-1 matrix
    of order 8192 (any principal submatrix of an i.i.d. +-1 matrix is itself an
    SK instance), so no per-instance N x N generation is needed."""
    import sbqa_instances as inst
    rng = np.random.default_rng(seed)
    Ns = np.exp(rng.uniform(np.log(256), np.log(8192), n)).astype(int)
    Ns -= Ns % 2
    dense = rng.permutation(np.arange(n) % 2 == 0)
    big = inst.sk_pm1(8192, seed + 1) if dense.any() else None
    out = []
    for q in range(n):
        N = int(Ns[q])
        if dense[q]:
            off = int(rng.integers(0, 8192 - N + 1))
            out.append(dict(kind="dense", N=N, J=big[off:off + N, off:off + N], csr=None))
        else:
            d = int(rng.integers(3, 13))
            E = inst.regular_graph(N, d, seed + 100 + q)
            out.append(dict(kind="sparse", N=N, J=None, d=d,
                            csr=inst.edges_to_csr(N, E, inst.gaussian_edges(len(E), seed + 10000 + q))))
    return out


def serve_run(sb, srv, items, arrivals, R, runs, S, seed, workers=8, dense_prec="fp8"):
    """Submit items at their arrival times (seconds from start) from a pool of
    client threads (a submission validates and copies the instance, so one
    client thread would delay later arrivals), poll until all are done.
    Returns per-item latency (completion - arrival time), the makespan and the
    library's own latencies (submit call -> result)."""
    from concurrent.futures import ThreadPoolExecutor

    def submit(q):
        it = items[q]
        prec = dict(precision=sb.PREC_FP8 if dense_prec == "fp8" else sb.PREC_FP4) if it["kind"] == "dense" else {}
        return sb.sbqa_submit(srv, J=it["J"], csr=it["csr"], R=R, runs=runs, steps=S, fmode=0,
                              jp_kind=sb.JP_LINEAR, jp_start=0.5, jp_end=0.0, seed=seed + q, **prec)

    pool = ThreadPoolExecutor(max_workers=workers)
    futs, done, lib_lat = {}, {}, {}
    t0 = time.perf_counter()
    nxt, n = 0, len(items)
    try:
        while len(done) < n:
            now = time.perf_counter() - t0
            while nxt < n and arrivals[nxt] <= now:
                futs[nxt] = pool.submit(submit, nxt)
                nxt += 1
            for q, f in list(futs.items()):
                if q in done or not f.done():
                    continue
                r = sb.sbqa_poll(srv, f.result())
                if r is not None:
                    done[q] = time.perf_counter() - t0 - arrivals[q]
                    lib_lat[q] = r[2]
            time.sleep(0.0005)
    finally:
        pool.shutdown(wait=True)
    makespan = time.perf_counter() - t0
    lat = np.array([done[q] for q in range(n)])
    return lat, makespan, np.array([lib_lat[q] for q in range(n)])


def serve_main(a):
    print(json.dumps(serve_measure(a, a.serve_instances)), flush=True)


def serve_measure(a, n):
    """The mixed serving stream of n instances: calibration burst, then
    Poisson arrivals at rho x the measured service rate; returns the result
    line (throughput, latency percentiles)."""
    import paper_2604_01050_amd as sb
    R, runs, S = 16, 8, 2000
    items = serve_instances(n, 5001)
    updates = float(sum(it["N"] for it in items)) * R * runs * S
    budget = int(a.serve_budget_gib * (1 << 30))
    # service rate: a burst of the first n_cal instances, all arriving at t = 0
    n_cal = min(n, max(8, n // 4))
    srv = sb.sbqa_server_create(budget, a.serve_slots)
    _, t_cal, _ = serve_run(sb, srv, items[:n_cal], np.zeros(n_cal), R, runs, S, 7000, dense_prec=a.serve_dense)
    sb.sbqa_server_destroy(srv)
    mu = n_cal / t_cal
    lam = a.serve_rho * mu
    arrivals = np.cumsum(np.random.default_rng(5002).exponential(1.0 / lam, n))
    arrivals -= arrivals[0]
    srv = sb.sbqa_server_create(budget, a.serve_slots)
    lat, makespan, lib_lat = serve_run(sb, srv, items, arrivals, R, runs, S, 8000, dense_prec=a.serve_dense)
    st = sb.sbqa_server_stats(srv)
    sb.sbqa_server_destroy(srv)
    kinds = np.array([it["kind"] == "dense" for it in items])
    out = {
        "metric": "replica-spin updates/s (N*R*runs*steps/s); p99 solve latency, mixed stream",
        "value": updates / makespan, "unit": "replica-spin updates/s", "n_gpus": 1, "steps": S, "warmup": 0,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "%s (dense) / f32 (sparse)" % a.serve_dense, "data": "synthetic",
        "config": {"workload": "serving stream: %d instances, Poisson arrivals at %.2f x the measured service "
                               "rate, N log-uniform in [256, 8192], half dense SK +-1 (%s), half d-regular "
                               "d~U{3..12} Gaussian (CSR), R=16 x 8 runs, 2000 steps"
                               % (n, a.serve_rho, a.serve_dense.upper()),
                   "instances": n, "rho": a.serve_rho, "hbm_budget_gib": a.serve_budget_gib,
                   "slots": a.serve_slots},
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                      "max": float(lat.max()), "mean": float(lat.mean()),
                      "p50_dense": float(np.percentile(lat[kinds], 50)) if kinds.any() else None,
                      "p50_sparse": float(np.percentile(lat[~kinds], 50)) if (~kinds).any() else None,
                      "library_p99": float(np.percentile(lib_lat, 99))},
        "service_rate_per_s": mu, "arrival_rate_per_s": lam, "makespan_s": makespan,
        "gpu_busy_fraction": st["busy_s"] / makespan,
        "calibration": {"instances": n_cal, "seconds": t_cal},
    }
    return out


# ------------------------------------------------- time-to-epsilon, SBQA vs SBM
def tte_main(a):
    """Planted square lattices (known ground energy): optimality gaps and
    time-to-epsilon of SBQA and of the SBM baseline (same trajectory count,
    no ring), and the per-step device time of both with the same kernel."""
    import sbqa_instances as inst
    from paper_2604_01050_amd import harness as H
    import paper_2604_01050_amd as sb
    eps = [0.0, 0.002, 0.005, 0.01]
    steps_list = [int(x) for x in a.tte_steps.split(",")]
    seeds = list(range(1, a.tte_seeds + 1))
    sizes = []
    for L in [int(x) for x in a.tte_sizes.split(",")]:
        E, w, _, E0 = inst.planted_square(L, 600 + L)
        N = L * L
        csr = inst.edges_to_csr(N, E, w)
        row = {"L": L, "N": N, "E0": E0}
        # Gamma_x(0)/R is not given in the paper: SBQA is minimised over it as well. SBQA
        # runs at dt = R * 0.5: its per-replica terms carry 1/R (Eqs. 6-7), so each
        # replica then advances on the SBM time grid (dt 0.5) of the baseline.
        studies = {g0: H.tte_study(E0, eps, steps_list, seeds, csr=csr, R=16, runs=8, gamma0_over_R=g0, dt=8.0)
                   for g0 in (4.0, 16.0, 64.0)}
        best = []
        for q in range(len(eps)):
            g0 = min(studies, key=lambda k: studies[k]["best"][q]["tte_s"])
            best.append(dict(studies[g0]["best"][q], gamma0_over_R=g0))
        row["sbqa"] = {"best": best, "by_gamma0_over_R": {str(k): v for k, v in studies.items()}}
        row["sbm"] = H.tte_study(E0, eps, steps_list, seeds, csr=csr, R=16, runs=8, sbm=True)
        t_q = H.step_time(csr=csr, R=16, runs=8, steps=500, loop_kernel=sb.LOOP_STREAM)
        t_m = H.step_time(csr=csr, R=16, runs=8, steps=500, sbm=True, loop_kernel=sb.LOOP_STREAM)
        t_r = H.step_time(csr=csr, R=16, runs=8, steps=500)
        row["step_us"] = {"sbqa_stream": t_q * 1e6, "sbm_stream": t_m * 1e6, "sbqa_auto": t_r * 1e6,
                          "sbqa_over_sbm": t_q / t_m}
        sizes.append(row)
        print(json.dumps({"L": L, "N": N, "step_us": row["step_us"],
                          "best": {m: row[m]["best"] for m in ("sbqa", "sbm")}}), file=sys.stderr, flush=True)
    out = {"metric": "time-to-epsilon (s), planted square lattices; SBQA vs SBM", "value": None,
           "unit": "s", "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
           "config": {"workload": "planted periodic square lattices (known ground state), R=16 x 8 runs "
                                  "(SBM: 128 independent trajectories), steps %s, %d seeds; SBQA also minimised "
                                  "over Gamma_x(0)/R in {4, 16, 64}; SBQA dt = 8 (= R x 0.5), SBM dt = 0.5"
                                  % (steps_list, len(seeds)),
                      "eps": eps},
           "sizes": sizes}
    print(json.dumps(out), flush=True)


def measure(sb, w, K, warmup, stream, loop_kernel="auto", events=True, workload=None):
    """One timed solve of workload w: a warmup solve of `warmup` steps, then K
    steps of a fresh context and the readout, timed on the host clock; the
    dominant kernel's average launch comes from one HIP event pair around the
    K steps on the context's stream. The warmup also records the two events
    once (the runtime creates an event at its first record) and reads the
    fresh context out once at step 0 (each readout evaluates the current
    state anew and discards the previous best, so this changes no result; it
    leaves the first-use costs of the context's readout buffers outside the
    timed region). Returns the result fields and the context's readout."""
    import torch
    wctx = create(sb, w, seed=1, loop_kernel=loop_kernel)
    sb.sbqa_set_stream(wctx, stream)
    torch.cuda.synchronize()
    t_create = time.perf_counter()
    ctx = create(sb, w, seed=2, loop_kernel=loop_kernel)
    sb.sbqa_set_stream(ctx, stream)
    info = sb.sbqa_info(ctx)
    torch.cuda.synchronize()
    create_s = time.perf_counter() - t_create
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) if events else None
    # warmup: a separate solve, right before the timed one
    if ev:
        ev[0].record(stream)
    sb.sbqa_step(wctx, min(max(warmup, 1), w["S"]))
    if ev:
        ev[1].record(stream)
    sb.sbqa_best(wctx)
    sb.sbqa_destroy(wctx)
    sb.sbqa_best(ctx)
    torch.cuda.synchronize()
    resident = info["resident"]
    t0 = time.perf_counter()
    if ev:
        ev[0].record(stream)
    if resident:
        sb.sbqa_step(ctx, K)
    else:
        for q in range(K):
            sb.sbqa_step(ctx, 1)
    if ev:
        ev[1].record(stream)
    E, spins = sb.sbqa_best(ctx)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    N, R, runs = w["N"], w["R"], w["runs"]
    out = {
        "value": N * R * runs * K / t, "steps": K, "ms_per_step": 1e3 * t / K,
        "path": info["path"] + ("_resident" if resident else ""),
        "best_energy": {"mean": float(np.mean(E)), "min": float(np.min(E))},
        "end_to_end": {"seconds": create_s + t, "create_s": create_s,
                       "updates_per_s": N * R * runs * K / (create_s + t)},
    }
    if ev:
        launches = 1 if resident else K
        avg_s = ev[0].elapsed_time(ev[1]) * 1e-3 / launches
        out["readout_ms"] = 1e3 * t - ev[0].elapsed_time(ev[1])
        if resident:
            ops = K * resident_ops_per_step(w)
            sparse = "csr" in w
            tr = measured_traffic((workload or "") + "_resident", "csr_resident") if sparse and workload else None
            out["roofline"] = {"bound": "alu", "achieved": ops / avg_s / 1e12, "peak": PEAK_VALU_OPS,
                               "unit": "Tops/s (fp32 VALU lane ops)", "frac": ops / avg_s / 1e12 / PEAK_VALU_OPS,
                               "traffic": None if tr is None else tr * K,
                               "kernel": "k_csr_resident" if sparse else small_kernel_name(w),
                               "avg_launch_us": avg_s * 1e6, "steps_per_launch": K,
                               "algorithmic_ops_per_launch": ops}
        elif info["path"] == "csr_fp32":
            ab = algorithmic_bytes(w, info)
            out["roofline"] = {"bound": "hbm", "achieved": ab / avg_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": ab / avg_s / 1e9 / HBM_PEAK_GBS,
                               "traffic": measured_traffic(workload, info["path"]) if workload else None,
                               "kernel": "k_csr_step", "avg_launch_us": avg_s * 1e6,
                               "algorithmic_bytes_per_launch": ab}
        else:
            fl = algorithmic_flops(w)
            peak = PEAK[{"dense_fp8": "fp8", "dense_fp8_packed": "fp8", "dense_int8": "int8", "dense_fp4": "fp4",
                         "dense_fp4_packed": "fp4", "dense_fp32": "fp32",
                         "dense_bf16x3": "bf16"}[info["path"]]]
            unit = "TOP/s" if info["path"] == "dense_int8" else "TFLOP/s"
            out["roofline"] = {"bound": "mfma", "achieved": fl / avg_s / 1e12, "peak": peak, "unit": unit,
                               "frac": fl / avg_s / 1e12 / peak,
                               "traffic": measured_traffic(workload, info["path"]) if workload else None,
                               "kernel": dense_kernel_name(info), "avg_step_us": avg_s * 1e6,
                               "algorithmic_flops_per_step": fl}
    return out, ctx


def field_error(sb, ctx, w, rows):
    """Single-step field error of a dense context against the float64 product
    J . f(X) on sampled rows (ballistic f: the operand is the float32 state):
    normwise ||phi - phi64|| / ||phi64|| and the largest element error over
    the sum of magnitudes of the terms that form it."""
    x, _ = sb.sbqa_get_state(ctx)
    phi = sb.sbqa_fields(ctx)[rows].astype(np.float64)
    J = w["J"][rows]
    G = x.astype(np.float64)
    ref = J @ G
    mag = np.abs(J) @ np.abs(G)
    err = np.abs(phi - ref)
    return {"rows": len(rows), "normwise": float(np.linalg.norm(err) / np.linalg.norm(ref)),
            "max_over_term_magnitude": float(np.max(err / np.maximum(mag, 1e-300)))}


def dense_configs(sb, stream, K, cpu=True):
    """Dense configurations on the same GPU: SK N = 16384 (fp8 and fp4 with
    bit-packed J against the plain fp32 path) and Gaussian N = 8192 (split
    bf16 hi+lo against fp32, with the single-step field error of both); with
    cpu, each also beside the FP64 oracle on the host cores over its first
    steps (one window of about 5 s, at least one step)."""
    import torch
    res = {}
    sk = {}
    for name, key in (("sk_fp8", "fp8"), ("sk_fp4", "fp4"), ("sk_fp32", "fp32")):
        w = make_workload(name)
        r, ctx = measure(sb, w, K, K, stream, workload=name)
        sb.sbqa_destroy(ctx)
        r["workload"] = w["desc"]
        sk[key] = r
        print("dense %s: %.3f ms/step" % (name, r["roofline"]["avg_step_us"] / 1e3), file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    for key in ("fp8", "fp4"):
        sk[key + "_over_fp32"] = sk[key]["value"] / sk["fp32"]["value"]
    # +-1 couplings with a ternary operand: every field is an exact integer on all three paths,
    # so their trajectories and best energies agree exactly
    sk["best_energies_equal"] = sk["fp8"]["best_energy"] == sk["fp32"]["best_energy"] == sk["fp4"]["best_energy"]
    if cpu:
        sk["cpu_baseline"] = cpu_baseline(w, window_s=5.0, windows=1, single_s=0.0)
    res["sk_N16384_C256"] = sk
    g = {}
    rows = np.random.default_rng(77).choice(8192, 24, replace=False)
    for name, key in (("gauss_bf16x3", "bf16x3"), ("gauss_fp32", "fp32")):
        w = make_workload(name)
        r, ctx = measure(sb, w, K, K, stream, workload=name)
        r["field_error"] = field_error(sb, ctx, w, rows)
        sb.sbqa_destroy(ctx)
        r["workload"] = w["desc"]
        g[key] = r
        print("dense %s: %.3f ms/step" % (name, r["roofline"]["avg_step_us"] / 1e3), file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    g["bf16x3_over_fp32"] = g["bf16x3"]["value"] / g["fp32"]["value"]
    if cpu:
        g["cpu_baseline"] = cpu_baseline(w, window_s=5.0, windows=1, single_s=0.0)
    res["gauss_N8192_C512"] = g
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="sparse6")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true",
                    help="default workload: skip the mixed serving stream (p50/p99 solve latency)")
    ap.add_argument("--no-configs", action="store_true",
                    help="default workload: skip the other configurations (dense paths, serving stream)")
    ap.add_argument("--dense-steps", type=int, default=200,
                    help="default workload: timed steps of each dense configuration")
    ap.add_argument("--no-events", action="store_true", help="no events in the timed region")
    ap.add_argument("--calibrate", action="store_true", help="also run a copy kernel of known size (counter scaling)")
    ap.add_argument("--dense-tile", type=int, default=0,
                    help="dense workloads: replica columns per workgroup tile (64/128/256; 0 = autotuned), "
                         "e.g. to hold the tile fixed in counter runs")
    ap.add_argument("--loop-kernel", default="auto", choices=["auto", "stream", "resident"],
                    help="step loop: one launch per step (stream) or many steps per launch (resident)")
    ap.add_argument("--serve-instances", type=int, default=512, help="serve workload: number of instances")
    ap.add_argument("--serve-rho", type=float, default=0.8, help="serve workload: arrival rate / service rate")
    ap.add_argument("--serve-budget-gib", type=float, default=64.0, help="serve workload: HBM budget")
    ap.add_argument("--serve-slots", type=int, default=16, help="serve workload: resident instances at most")
    ap.add_argument("--serve-dense", default="fp8", choices=["fp8", "fp4"],
                    help="serve workload: contraction of the dense SK instances (both exact)")
    ap.add_argument("--tte-sizes", default="32,64,128", help="tte workload: lattice sizes L (N = L*L)")
    ap.add_argument("--tte-steps", default="250,1000,4000", help="tte workload: step counts")
    ap.add_argument("--tte-seeds", type=int, default=8, help="tte workload: solves per point")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU only: the SBQA runs of one instance are independent and the "
              "library has no multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2604_01050_amd as sb
    torch.cuda.set_device(0)
    if a.workload == "serve":
        serve_main(a)
        return
    if a.workload == "tte":
        tte_main(a)
        return
    if a.calibrate:
        copy_calibration()
    w = make_workload(a.workload)
    if a.dense_tile:
        w["dense_tile"] = a.dense_tile
    K = a.steps if a.steps is not None else w["S"]
    if K < 1 or K > w["S"]:
        raise SystemExit("--steps must be in [1, %d] (one solve of the schedule)" % w["S"])
    stream = torch.cuda.Stream()
    r, ctx = measure(sb, w, K, a.warmup, stream, loop_kernel=a.loop_kernel, events=not a.no_events,
                     workload=a.workload)
    sb.sbqa_destroy(ctx)
    N, R, runs = w["N"], w["R"], w["runs"]
    out = {
        "metric": "replica-spin updates/s (N*R*runs*steps/s)",
        "value": r["value"], "unit": "replica-spin updates/s", "n_gpus": 1, "steps": K, "warmup": a.warmup,
        "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": w["dtype"], "data": "synthetic",
        "config": {"workload": w["desc"], "N": N, "R": R, "runs": runs, "schedule_steps": w["S"], "path": r["path"]},
        "best_energy": r["best_energy"],
        "end_to_end": dict(r["end_to_end"], includes="sbqa_create from host arrays (validation, upload, initial "
                                                     "state), the K steps and the readout"),
    }
    if "roofline" in r:
        out["roofline"] = r["roofline"]
        out["readout_ms"] = r["readout_ms"]
    if a.workload == "sparse6" and not a.no_configs:
        # the other configurations, measured on the same GPU in the same run: the small
        # dense instance, the dense fp8 / fp4 / split-bf16 paths against fp32, and the
        # mixed serving stream (the p50/p99 half of the metric)
        cfg = {}
        try:
            w1 = make_workload("sk64")
            r1, c1 = measure(sb, w1, 1000, 200, stream, workload="sk64")
            sb.sbqa_destroy(c1)
            r1["workload"] = w1["desc"]
            # the same solve with one launch per step (the MFMA step kernel)
            r2, c2 = measure(sb, w1, 1000, 200, stream, loop_kernel="stream", workload="sk64")
            sb.sbqa_destroy(c2)
            r1["one_launch_per_step"] = {"value": r2["value"], "ms_per_step": r2["ms_per_step"],
                                         "avg_step_us": r2.get("roofline", {}).get("avg_step_us"),
                                         "path": r2["path"]}
            cfg["sk_N64_C32"] = r1
        except Exception as e:   # reported, never hides the main line
            cfg["sk_N64_C32"] = {"error": repr(e)}
        try:
            cfg.update(dense_configs(sb, stream, a.dense_steps, cpu=not a.no_cpu_baseline))
        except Exception as e:
            cfg["dense"] = {"error": repr(e)}
        if not a.no_serve:
            try:
                sv = serve_measure(a, a.serve_instances)
                cfg["serving"] = {"instances": a.serve_instances, "updates_per_s": sv["value"],
                                  "latency_s": sv["latency_s"], "workload": sv["config"]["workload"],
                                  "service_rate_per_s": sv["service_rate_per_s"],
                                  "gpu_busy_fraction": sv["gpu_busy_fraction"], "makespan_s": sv["makespan_s"]}
            except Exception as e:
                cfg["serving"] = {"error": repr(e)}
        out["configs"] = cfg
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
