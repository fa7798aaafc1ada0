"""SpMV sweep benchmark on one MI355X, plus the solver measurements.

One step = one FP64 SpMV (y = A x) in every storage format on both matrices
of the sweep workload: the 3D 27-point stencil on a 128^3 grid (n = 2,097,152,
nnz = 55,742,968) and a random matrix with n = 1,000,000, lognormal row
lengths (mean 16, longest row 10,000) and uniform columns.  ELL on the random
matrix is infeasible (width 10,000) and is skipped.  The two matrices'
SpMVs alternate so the random matrix (213 MB, small enough for the 256 MB
last-level cache) never runs right after itself.  Inputs are synthetic and
seeded, resident in HBM before timing starts.

value = algorithmic bytes of all SpMVs of a step / step time (GB/s).
Algorithmic bytes per SpMV (value size s, beta = 0; x read once, y written once):
  CSR, CSR_MERGE: nnz (s+4) + (n+1) 4 + n_cols s + n s
  COO:            nnz (s+8) + n_cols s + n s
  ELL:            n K (s+4) + n_cols s + n s
  HYBRID:         n K (s+4) + tail (s+8) + n_cols s + n s (+ n s when a tail exists)
The paper's own model (Sec. 6.1) counts only the matrix entries: 12 bytes per
CSR entry and 16 per COO entry.  The padded formats count their stored slots,
padding included, although their kernels stop at a row's first padding slot;
per_kernel reports those unread bytes beside the figure (on the stencil
10.6 MB, 1.5% of ELL's bytes: the shorter rows at the grid's faces).

After the timed sweep (outside it): CG on the 2D 5-point Laplacian 64x64
(to 1e-10), and block-Jacobi PCG on the 3D 7-point Poisson 256^3 in FP64 and
in mixed precision (FP32 inner solve, FP64 refinement), each to 1e-10, the
10,000-system batched CG and the learned format selector.

The CPU baseline is the oracle, one host core per run: the sweep's SpMVs, the
solves of both CG workloads, the per-system batch loop and the selector's
features.  The two Poisson 256^3 oracle solves (minutes of serial work) run
in child processes started before the GPU is touched, on other host cores
while the GPU legs run; their solutions also give each GPU solve's error
against the FP64 oracle.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published
METRIC = "SpMV GB/s (% HBM peak); CG s to 1e-10, FP64 vs mixed; batch solves/s"


def spmv_bytes(desc, s=8):
    n, m, nnz = desc.n_rows, desc.n_cols, desc.nnz
    f = desc.format
    if f in ("csr", "csr_merge"):
        return nnz * (s + 4) + (n + 1) * 4 + m * s + n * s
    if f == "coo":
        return nnz * (s + 8) + m * s + n * s
    if f == "ell":
        return n * desc.ell_width * (s + 4) + m * s + n * s
    if f == "hybrid":
        b = n * desc.ell_width * (s + 4) + desc.coo_nnz * (s + 8) + m * s + n * s
        return b + (n * s if desc.coo_nnz else 0)
    if f == "sellp":
        return desc.sellp_slots * (s + 4) + (desc.sellp_slices + 1) * 8 + m * s + n * s
    raise ValueError(f)


def padding_bytes(desc, s=8):
    """Bytes of the padding slots that the algorithmic bytes of ELL, HYB and
    SELL-P count (the stored slots) but their kernels never read: a row stops
    at its first padding slot."""
    f = desc.format
    if f == "ell":
        return (desc.n_rows * desc.ell_width - desc.nnz) * (s + 4)
    if f == "hybrid":
        return (desc.n_rows * desc.ell_width - (desc.nnz - desc.coo_nnz)) * (s + 4)
    if f == "sellp":
        return (desc.sellp_slots - desc.nnz) * (s + 4)
    return 0


def csr_bytes(n, m, nnz, s=8):
    return nnz * (s + 4) + (n + 1) * 4 + m * s + n * s


def kernel_source_hash():
    """sha256 over the HIP sources: counters taken on other sources do not apply."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2011_08879_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp", ".cpp")):
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def measured_traffic(key):
    """HBM bytes per launch of one sweep SpMV from the committed rocprofv3 counter
    summary (32 x the L2's DRAM-bound 32-byte read and write request counts, which
    reproduce a 1 GiB copy without a scale factor), or None when the kernels
    changed since."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_sha256") != kernel_source_hash() or key not in t.get("kernels", {}):
        return None
    return t["kernels"][key]["traffic_bytes"]


def log(msg):
    sys.stderr.write("[bench] %s\n" % msg)
    sys.stderr.flush()


def build_sweep(g, gen, torch):
    mats = []
    t0 = time.time()
    st = gen.stencil27(128)
    log("stencil27 128^3 generated (%.1fs)" % (time.time() - t0))
    t0 = time.time()
    rnd = gen.random_lognormal(4, 1_000_000, mean=16.0, sigma=1.56, max_len=10000)
    log("lognormal 1M generated (%.1fs)" % (time.time() - t0))
    inputs = {"stencil27_128": st, "lognormal_1M": rnd}
    xs = {name: torch.from_numpy(gen.uniform(3 if name.startswith("st") else 5,
                                              len(A[0]) - 1)).cuda() for name, A in inputs.items()}
    base = {name: g.Matrix.from_csr(*A) for name, A in inputs.items()}
    order = [("stencil27_128", "csr"), ("lognormal_1M", "csr"),
             ("stencil27_128", "csr_merge"), ("lognormal_1M", "csr_merge"),
             ("stencil27_128", "coo"), ("lognormal_1M", "coo"),
             ("stencil27_128", "ell"), ("stencil27_128", "hybrid"), ("lognormal_1M", "hybrid")]
    for name, fmt in order:
        M = base[name].clone().convert(fmt)
        d = M.describe()
        y = torch.empty(d.n_rows, dtype=torch.float64, device="cuda")
        mats.append({"matrix": name, "format": fmt, "M": M, "x": xs[name], "y": y, "desc": d,
                     "bytes": spmv_bytes(d), "useful_bytes": csr_bytes(d.n_rows, d.n_cols, d.nnz),
                     "flops": 2 * d.nnz})
    skipped = [{"matrix": "lognormal_1M", "format": "ell", "reason": "unsupported: width 10000"}]
    try:
        base["lognormal_1M"].clone().convert("ell")
        skipped = []
    except g.GkoError as e:
        assert e.status == g.ERR_UNSUPPORTED
    return mats, skipped, inputs, base


def host_info():
    """The host CPU the oracle ran on: model name and core counts."""
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count(),
            "cpus_available": len(os.sched_getaffinity(0))}


def cpu_solver_baselines(keep, gpu_solvers, selector_lat, n_feature_matrices=12):
    """The oracle, serial, on the solver, batch and selector workloads: config-1
    CG seconds and iterations, the per-system batch loop in FP64 and FP32
    (refined) storage, and the selector's 32 features per corpus matrix."""
    import gen
    import oracle
    out = {}
    if "cg_laplace2d_64" in keep:
        A, b = keep["cg_laplace2d_64"]
        best = None
        for _ in range(5):
            t0 = time.perf_counter()
            rc, x, info = oracle.cg(A, b, tol=1e-10)
            el = time.perf_counter() - t0
            best = el if best is None else min(best, el)
        out["cg_laplace2d_64"] = {"seconds": round(best, 6), "iterations": info["iters"],
                                  "true_rel_residual": float(info["true_relres"])}
        if gpu_solvers:
            out["cg_laplace2d_64"]["gpu_seconds"] = gpu_solvers["cg_laplace2d_64"]["seconds"]
    if "batch" in keep:
        Bk = keep["batch"]
        B = Bk["B"]
        res = {}
        for label, fn, vals in (("fp64", oracle.batch_cg, B.val),
                                ("fp32", oracle.batch_ir_cg,
                                 B.val.astype(np.float32).astype(np.float64))):
            t0 = time.perf_counter()
            rc, x, it, rr = fn(B.row_off, B.nnz_off, B.row_ptr, B.col, vals, Bk[label], tol=1e-10)
            el = time.perf_counter() - t0
            res[label] = {"seconds": round(el, 4), "solves_per_s": round(B.nsys / el, 1),
                          "iters_mean": round(float(it.mean()), 1),
                          "max_true_rel_residual": float(rr.max())}
            if gpu_solvers:
                res[label]["gpu_solves_per_s"] = gpu_solvers["batch_cg_10k"][label]["solves_per_s"]
        out["batch_cg_10k"] = res
    if selector_lat is not None:
        secs, rows = [], []
        for i in range(n_feature_matrices):
            A = gen.corpus_matrix(gen.corpus_spec(i))
            t0 = time.perf_counter()
            oracle.features(A)
            secs.append(time.perf_counter() - t0)
            rows.append(len(A[0]) - 1)
        out["selector_features"] = {"matrices": n_feature_matrices,
                                    "seconds_per_matrix": round(float(np.mean(secs)), 5),
                                    "mean_rows": int(np.mean(rows)),
                                    "gpu_seconds_per_matrix_corpus":
                                        round(selector_lat["features_s_mean"], 5)}
    return out


def cpu_baseline(inputs, step_alg_bytes, budget_s=15.0):
    """The oracle (serial FP64 CSR SpMV, one host core) on the sweep's two
    matrices, alternating until the time budget is spent.  The oracle computes
    every format's product by CSR, so one sweep step is 5 stencil and 4 random
    products; the value is the step's algorithmic bytes over that CPU time."""
    import oracle
    if not os.path.exists(oracle._LIB):
        oracle.build()
    rng = np.random.default_rng(0)
    mats = {name: (A, rng.uniform(-1, 1, len(A[0]) - 1)) for name, A in inputs.items()}
    for A, x in mats.values():
        oracle.spmv(A, x)  # warm the pages
    secs = {name: [] for name in mats}
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        for name, (A, x) in mats.items():
            t = time.perf_counter()
            oracle.spmv(A, x)
            secs[name].append(time.perf_counter() - t)
    per = {name: float(np.median(v)) for name, v in secs.items()}
    step = 5 * per["stencil27_128"] + 4 * per["lognormal_1M"]
    st = inputs["stencil27_128"]
    n = len(st[0]) - 1
    return {"value": round(step_alg_bytes / step / 1e9, 3), "unit": "GB/s", "cores": 1,
            "kind": "oracle",
            "sample": "%d + %d serial FP64 CSR SpMVs of the 27-point 128^3 stencil and the "
                      "lognormal 1e6 matrix (%.1f s); a sweep step = 5 stencil + 4 random "
                      "products over the step's algorithmic bytes" %
                      (len(secs["stencil27_128"]), len(secs["lognormal_1M"]),
                       time.perf_counter() - t0),
            "seconds_per_step": round(step, 4),
            "stencil_csr_GB/s": round(csr_bytes(n, n, len(st[1])) / per["stencil27_128"] / 1e9, 3),
            "seconds_per_spmv": {k: round(v, 4) for k, v in per.items()}}


def stream_probe(g, torch, n=1 << 27, reps=10):
    """Achievable HBM bandwidth: the library's COPY and TRIAD kernels on 1 GiB
    FP64 arrays (the measured-bandwidth reference the paper takes from
    BabelStream, Sec. 6).  Mean over reps after one warm-up."""
    a = torch.rand(n, dtype=torch.float64, device="cuda")
    b = torch.rand(n, dtype=torch.float64, device="cuda")
    c = torch.empty_like(a)
    out = {"n": n, "bytes_per_array": n * 8}
    for name, op, nbytes in (("copy", g.STREAM_COPY, 16 * n), ("triad", g.STREAM_TRIAD, 24 * n)):
        g.stream(op, a, c, b, 0.5)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            g.stream(op, a, c, b, 0.5)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name + "_GB/s"] = round(nbytes / (ms * 1e-3) / 1e9, 1)
    del a, b, c
    out["gather"] = gather_probe(g, torch)
    torch.cuda.empty_cache()
    return out


def gather_probe(g, torch, n=16_000_000, m=1_000_000, reps=10):
    """The random-gather ceiling: y[i] = x[idx[i]] with 16M indices uniform over
    an 8 MB x (the random sweep matrix's x and entry count), index and output
    streamed.  Reported as gathers per second and as the streamed bytes
    (4 + 8 per gather, plus x once) per second; the L2's fetch for it comes
    from the profiles' DRAM request counters."""
    rng = np.random.default_rng(41)
    idx = torch.from_numpy(rng.integers(0, m, n).astype(np.int32)).cuda()
    x = torch.rand(m, dtype=torch.float64, device="cuda")
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    g.gather_probe(x, idx, y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        g.gather_probe(x, idx, y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nb = n * 12 + m * 8
    return {"n": n, "x_bytes": m * 8, "ms": round(ms, 5),
            "gathers_per_s": round(n / (ms * 1e-3), 1),
            "streamed_GB/s": round(nb / (ms * 1e-3) / 1e9, 1)}


def poisson256_inputs(gen):
    """Config-3 inputs: the 3D 7-point Poisson matrix on 256^3, x* ~ U[-1,1]
    (seed 5), b = A x* by scipy (neither the oracle nor the library)."""
    import scipy.sparse as sp
    A = gen.laplace3d(256)
    n = 256 ** 3
    S = sp.csr_matrix((A[2], A[1], A[0]), shape=(n, n))
    xs = gen.uniform(5, n)
    return A, S, xs, S @ xs


def kappa_laplace3d(N):
    """Condition number of the 3D 7-point Dirichlet Laplacian on N^3."""
    c = math.cos(math.pi / (N + 1))
    return (6 + 6 * c) / (6 - 6 * c)


def oracle_poisson_worker(outdir, mode):
    """Child process: the oracle's FP64 block-Jacobi PCG ("fp64") or its
    mixed-precision refinement ("mixed") on the config-3 system, serial.
    Writes <mode>.json (timings, counts) and <mode>_x.npy.  Never touches
    the GPU."""
    import hashlib

    import gen
    import oracle
    if not os.path.exists(oracle._LIB):
        raise SystemExit("oracle library missing")
    A, S, xs, bh = poisson256_inputs(gen)
    del S
    t0 = time.perf_counter()
    rc, inv = oracle.bj_invert(A, 8)
    setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    if mode == "fp64":
        rc, x, info = oracle.cg(A, bh, tol=1e-10, maxit=20000, bj_inv=inv)
        it = {"iterations": info["iters"], "restarts": info["restarts"]}
        relres = info["true_relres"]
    else:
        rc, x, info = oracle.ir_cg(A, bh, tol=1e-10, inner_tol=1e-5, bj_inv=inv)
        it = {"iterations": info["inner_iters"], "outer_iterations": info["outer_iters"]}
        relres = info["true_relres"]
    el = time.perf_counter() - t0
    np.save(os.path.join(outdir, mode + "_x.npy"), x)
    res = dict(it, status=int(rc), seconds=round(el, 3), setup_seconds=round(setup, 3),
               seconds_per_iteration=round(el / max(it["iterations"], 1), 5),
               true_rel_residual=float(relres),
               b_sha256=hashlib.sha256(np.ascontiguousarray(bh).tobytes()).hexdigest())
    with open(os.path.join(outdir, mode + ".json"), "w") as fh:
        json.dump(res, fh)


def start_oracle_workers():
    """Start both config-3 oracle solves as child processes (before this
    process initialises the GPU)."""
    outdir = tempfile.mkdtemp(prefix="gko_oracle_")
    procs = {}
    for mode in ("fp64", "mixed"):
        procs[mode] = subprocess.Popen(
            [sys.executable, os.path.abspath(__file__), "--oracle-poisson-worker", mode,
             "--worker-dir", outdir], stdout=subprocess.DEVNULL,
            stderr=open(os.path.join(outdir, mode + ".err"), "w"))
    return {"dir": outdir, "procs": procs, "t0": time.time()}


def finish_oracle_workers(w, gpu, deadline_s):
    """Wait (up to deadline_s after the start) for the oracle solves; report
    their timings and each GPU solution's error against the FP64 oracle's."""
    out = {}
    for mode, p in w["procs"].items():
        try:
            p.wait(timeout=max(1.0, deadline_s - (time.time() - w["t0"])))
        except subprocess.TimeoutExpired:
            p.kill()
            p.wait()
            out[mode] = {"unfinished": "killed after %.0f s" % (time.time() - w["t0"])}
            continue
        path = os.path.join(w["dir"], mode + ".json")
        if p.returncode != 0 or not os.path.exists(path):
            with open(os.path.join(w["dir"], mode + ".err")) as fh:
                out[mode] = {"failed": "rc %d: %s" % (p.returncode, fh.read()[-300:])}
            continue
        with open(path) as fh:
            out[mode] = json.load(fh)
    errs = {}
    if "seconds" in out.get("fp64", {}) and gpu is not None:
        xo = np.load(os.path.join(w["dir"], "fp64_x.npy"))
        same_b = out["fp64"].pop("b_sha256") == gpu["b_sha256"]
        no = np.linalg.norm(xo)
        for label in ("fp64", "mixed"):
            errs["gpu_" + label] = float(np.linalg.norm(gpu[label] - xo) / no)
        if "seconds" in out.get("mixed", {}):
            xm = np.load(os.path.join(w["dir"], "mixed_x.npy"))
            errs["oracle_mixed"] = float(np.linalg.norm(xm - xo) / no)
            out["mixed"].pop("b_sha256", None)
        errs["same_b"] = same_b
        errs["bound_2kappa_tol"] = 2 * kappa_laplace3d(256) * 1e-10
    for f in os.listdir(w["dir"]):
        os.remove(os.path.join(w["dir"], f))
    os.rmdir(w["dir"])
    return out, errs


def run_solvers(g, gen, torch, keep):
    import scipy.sparse as sp
    out = {}
    ctx = g.default_context()
    # config 1: 2D 5-point Laplacian 64x64, unpreconditioned FP64 CG to 1e-10
    A = gen.laplace2d(64)
    n = 4096
    S = sp.csr_matrix((A[2], A[1], A[0]), shape=(n, n))
    xs = gen.uniform(2, n)
    b = torch.from_numpy(S @ xs).cuda()
    M = g.Matrix.from_csr(*A)
    # one-workgroup single-launch CG (the default at this size) and the
    # multi-kernel path
    res1 = {}
    for label, single in (("single_workgroup", 1), ("multi_kernel", 0)):
        ctx.set_solver_opts(single_workgroup=single)
        best = None
        for _ in range(5):
            x = torch.zeros(n, dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = g.cg(M, b, x, tol=1e-10)
            el = time.perf_counter() - t0
            best = el if best is None else min(best, el)
        xh = x.cpu().numpy()
        res1[label] = {"seconds": round(best, 5), "iterations": info["iterations"],
                       "true_rel_residual": info["true_rel_residual"],
                       "rel_error_vs_xstar": float(np.linalg.norm(xh - xs) / np.linalg.norm(xs)),
                       "status": info["status_name"]}
        log("config-1 CG (%s): %.2f ms, %d it" % (label, best * 1e3, info["iterations"]))
    ctx.set_solver_opts()
    res1["seconds"] = min(res1["single_workgroup"]["seconds"], res1["multi_kernel"]["seconds"])
    out["cg_laplace2d_64"] = res1
    keep["cg_laplace2d_64"] = (A, S @ xs)
    # config 3: 3D 7-point Poisson 256^3, block-Jacobi(8), FP64 PCG vs mixed IR
    t0 = time.time()
    A, S, xs, bh = poisson256_inputs(gen)
    n = 256 ** 3
    log("poisson 256^3 ready (%.1fs)" % (time.time() - t0))
    b = torch.from_numpy(bh).cuda()
    M = g.Matrix.from_csr(*A)
    del A
    M.convert("auto")   # the library times every format and keeps the fastest SpMV
    res = {"format": M.describe().format}
    log("config-3 matrix stored as %s" % res["format"])
    for label, prec in (("fp64", g.PREC_FP64), ("mixed", g.PREC_MIXED_IR)):
        ctx.set_solver_opts(precision=prec, precond=g.PRECOND_BLOCK_JACOBI, block_size=8,
                            inner_tol=1e-5)
        runs = []
        for rep in range(2):
            M2 = M.clone()   # fresh handle: the preconditioner setup is part of the solve
            x = torch.zeros(n, dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = g.cg(M2, b, x, tol=1e-10, maxit=20000)
            el = time.perf_counter() - t0
            runs.append(el)
            M2.close()
        xh = x.cpu().numpy()
        r = bh - S @ xh
        res[label] = {"seconds": round(min(runs), 4), "iterations": info["iterations"],
                      "outer_iterations": info["outer_iterations"],
                      "setup_seconds": round(info["setup_seconds"], 4),
                      "true_rel_residual": float(np.linalg.norm(r) / np.linalg.norm(bh)),
                      "rel_error_vs_xstar": float(np.linalg.norm(xh - xs) / np.linalg.norm(xs)),
                      "status": info["status_name"]}
        res[label + "_x"] = xh
        log("config-3 %s: %.3f s, %d it (%d outer)" % (label, min(runs), info["iterations"],
                                                      info["outer_iterations"]))
    res["krylov_fixed_iterations"] = run_krylov(g, torch, ctx, M, b, n)
    x64, xmx = res.pop("fp64_x"), res.pop("mixed_x")
    res["mixed"]["rel_diff_vs_fp64_solution"] = float(np.linalg.norm(xmx - x64) / np.linalg.norm(x64))
    import hashlib
    keep["poisson256"] = {"fp64": x64, "mixed": xmx,
                          "b_sha256": hashlib.sha256(np.ascontiguousarray(bh).tobytes()).hexdigest()}
    res["speedup_mixed_over_fp64"] = round(res["fp64"]["seconds"] / res["mixed"]["seconds"], 3)
    out["pcg_bj8_poisson3d_256"] = res
    ctx.set_solver_opts()
    del M, b, S
    torch.cuda.empty_cache()
    out["batch_cg_10k"] = run_batch(g, gen, torch, keep)
    return out


def krylov_bytes(name, S, n, iters, m=30):
    """Algorithmic bytes of `iters` FP64 iterations (S: one SpMV's bytes, n rows).
    Per iteration: CG and FCG S + 9 vector passes (fused product with p.q;
    x, r update with the sums; p update); pipelined CG S + 13 (one update
    kernel reading n, z, s, p, x, r, w and writing all but n); BiCGSTAB
    2S + 15 (rhat read by the fused v = A p; s = r - alpha v; t.s and t.t
    formed in t = A s; x, r update reading x, p, s, t, rhat; p update);
    CGS 2S + 16 (rhat read by the fused t = A p);
    GMRES Arnoldi step j: S + (2j + 7) passes with one Gram-Schmidt round
    (dot over j+1 basis vectors and w, update reading them and writing w,
    normalisation), plus per cycle the residual (S + 5 passes) and
    x += V y (m + 2 passes).  A vector pass is 8n bytes."""
    vp = 8.0 * n
    if name in ("cg", "fcg"):
        return iters * (S + 9 * vp)
    if name == "pipecg":
        return iters * (S + 13 * vp)
    if name == "bicgstab":
        return iters * (2 * S + 15 * vp)
    if name == "cgs":
        return iters * (2 * S + 16 * vp)
    if name == "gmres":
        cycles, rest = divmod(iters, m)
        steps = [j for _ in range(cycles) for j in range(m)] + list(range(rest))
        per_cycle = S + 5 * vp + (m + 2) * vp
        return sum(S + (2 * j + 7) * vp for j in steps) + (cycles + (rest > 0)) * per_cycle
    raise ValueError(name)


def run_krylov(g, torch, ctx, M, b, n):
    """Every Krylov solver for a fixed number of FP64 iterations on the same
    matrix (unpreconditioned, tolerance out of reach): time per iteration and
    algorithmic bytes per second, as the paper's solver benchmark measures
    bandwidth-bound solvers over a fixed iteration count."""
    d = M.describe()
    S = spmv_bytes(d)
    out = {"format": d.format, "n": n, "spmv_alg_bytes": int(S)}
    runs = (("cg", g.cg, 300), ("fcg", g.fcg, 300), ("pipecg", g.pipecg, 300),
            ("bicgstab", g.bicgstab, 150), ("cgs", g.cgs, 150), ("gmres", g.gmres, 300))
    for name, fn, iters in runs:
        ctx.set_solver_opts(single_workgroup=0, krylov_dim=30)
        best = None
        for _ in range(2):
            x = torch.zeros(n, dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = fn(M, b, x, tol=1e-30, maxit=iters)
            el = time.perf_counter() - t0
            best = el if best is None else min(best, el)
        it = info["iterations"]
        nb = krylov_bytes(name, S, n, it)
        out[name] = {"iterations": it, "seconds": round(best, 4),
                     "ms_per_iteration": round(best / max(it, 1) * 1e3, 4),
                     "alg_GB/s": round(nb / best / 1e9, 1),
                     "frac_hbm_peak": round(nb / best / 1e9 / HBM_PEAK_GBS, 4),
                     "status": info["status_name"]}
        if name == "gmres":
            out[name]["reorthogonalized_steps"] = info["reorthogonalized"]
        log("krylov %-8s %4d it  %.3f ms/it  %.0f GB/s" % (name, it, out[name]["ms_per_iteration"],
                                                         out[name]["alg_GB/s"]))
    ctx.set_solver_opts()
    out["cg_vs_pipecg_by_size"] = cg_vs_pipecg(g, torch, ctx)
    out["gmres_small_systems"] = gmres_small(g, torch, ctx)
    return out


def gmres_small(g, torch, ctx):
    """GMRES(30) on small 3D Poisson matrices (CSR), the whole solve on one
    workgroup against the multi-kernel path: us per Arnoldi step over 300
    steps (tol 1e-30, so every step runs; restarts included)."""
    import gen
    res = {}
    for N in (12, 16):   # 1,728 and 4,096 rows (the one-workgroup solve takes up to 4,096)
        A = gen.laplace3d(N)
        n = N ** 3
        M = g.Matrix.from_csr(*A)
        b = torch.from_numpy(gen.uniform(5, n)).cuda()
        row = {}
        for label, single in (("one_workgroup", 1), ("multi_kernel", 0)):
            ctx.set_solver_opts(krylov_dim=30, single_workgroup=single)
            best = None
            for _ in range(3):
                x = torch.zeros(n, dtype=torch.float64, device="cuda")
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                info = g.gmres(M, b, x, tol=1e-30, maxit=300)
                el = time.perf_counter() - t0
                best = el if best is None else min(best, el)
            row[label + "_us_per_step"] = round(best / info["iterations"] * 1e6, 2)
        ctx.set_solver_opts()
        res["poisson3d_%d" % N] = row
        log("gmres(30) n=%d: one workgroup %.1f, multi-kernel %.1f us per step" %
            (n, row["one_workgroup_us_per_step"], row["multi_kernel_us_per_step"]))
    return res


def cg_vs_pipecg(g, torch, ctx):
    """CG (three kernels and two reductions per iteration) against pipelined
    CG (two kernels, one reduction, more vector traffic) on 3D Poisson
    matrices from latency-bound to bandwidth-bound sizes: us per iteration."""
    import gen
    res = {}
    for N in (16, 32, 64, 128):
        A = gen.laplace3d(N)
        n = N ** 3
        M = g.Matrix.from_csr(*A)
        M.convert("sellp")
        b = torch.from_numpy(gen.uniform(5, n)).cuda()
        row = {}
        for name, fn in (("cg", g.cg), ("pipecg", g.pipecg)):
            ctx.set_solver_opts(single_workgroup=0)
            best = None
            for _ in range(3):
                x = torch.zeros(n, dtype=torch.float64, device="cuda")
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                info = fn(M, b, x, tol=1e-30, maxit=200)
                el = time.perf_counter() - t0
                best = el if best is None else min(best, el)
            row[name + "_us_per_iteration"] = round(best / info["iterations"] * 1e6, 2)
        res["poisson3d_%d" % N] = row
        log("cg vs pipecg n=%d: %.1f / %.1f us per iteration" %
            (n, row["cg_us_per_iteration"], row["pipecg_us_per_iteration"]))
        M.close()
    ctx.set_solver_opts()
    return res


def run_batch(g, gen, torch, keep, nsys=10000, reps=3):
    """10,000 SPD systems (3-/5-point, 32..1024 rows, shift U[0.1, 2]) to 1e-10 each,
    one persistent launch per solve; FP64 and FP32 storage (FP32 CG inside FP64
    refinement).  The workgroup size is autotuned first.  A secondary line
    runs the FP32 batch to 1e-5, which FP32 iterations reach on their own: the
    kernel's first inner solve then meets the tolerance and its FP64 residual
    check ends the solve without a refinement step."""
    import scipy.sparse as sp
    B = gen.batch_systems(nsys, master_seed=6)
    # b = A x* from a block-diagonal assembly of all systems (scipy, not the library)
    rows = np.repeat(np.arange(B.row_off[-1]), np.concatenate(
        [np.diff(B.system(i)[0]) for i in range(nsys)]))
    sys_of_entry = np.repeat(np.arange(nsys), np.diff(B.nnz_off))
    cols = B.col.astype(np.int64) + B.row_off[:-1][sys_of_entry]
    out = {"nsys": nsys, "rows": int(B.row_off[-1]), "nnz": int(B.nnz_off[-1])}
    keep["batch"] = {"B": B}
    for label, vals, tdt, tol in (("fp64", B.val, torch.float64, 1e-10),
                                  ("fp32", B.val.astype(np.float32), torch.float32, 1e-10),
                                  ("fp32_only_tol1e-5", B.val.astype(np.float32), torch.float32,
                                   1e-5)):
        S = sp.csr_matrix((vals.astype(np.float64), (rows, cols)), shape=(out["rows"], out["rows"]))
        bh = S @ B.xstar
        keep["batch"][label] = bh
        b = torch.from_numpy(bh).cuda()
        G = g.Batch(B.row_off, B.nnz_off, B.row_ptr, B.col, vals, dtype=tdt)
        x = torch.zeros(out["rows"], dtype=torch.float64, device="cuda")
        blk, times = G.autotune(b, x, tol=tol, maxit=1000)
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, it, rr = G.solve(b, x, tol=tol, maxit=1000)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            best = el if best is None else min(best, el)
        it, rr, xh = it.cpu().numpy(), rr.cpu().numpy(), x.cpu().numpy()
        err = np.abs(xh - B.xstar).max() / np.abs(B.xstar).max()
        # HBM floor: one read of every system (local row_ptr, col, val, the two
        # int64 offset arrays), of b and of the initial x, one write of x
        vs = 8 if label == "fp64" else 4
        floor_bytes = ((out["rows"] + nsys) * 4 + out["nnz"] * (4 + vs) + 2 * (nsys + 1) * 8
                       + 3 * out["rows"] * 8)
        out[label] = {"solves_per_s": round(nsys / best, 1), "seconds": round(best, 5), "tol": tol,
                      "hbm_floor_bytes": int(floor_bytes),
                      "hbm_floor_seconds": round(floor_bytes / (HBM_PEAK_GBS * 1e9), 7),
                      "block": blk, "lds_mode": G.lds_mode,
                      "autotune_ms": {"%d/%s" % k: (round(v, 3) if np.isfinite(v) else None)
                                      for k, v in times.items()},
                      "status": g.status_string(st), "iters_mean": round(float(it.mean()), 1),
                      "iters_max": int(it.max()), "max_true_rel_residual": float(rr.max()),
                      "max_abs_err_rel_to_max_xstar": float(err)}
        if label == "fp64":
            out[label]["bound"] = batch_bound(g, torch, B, vals, bh, G, it, best, floor_bytes)
        log("batch %s: %.0f solves/s (%.2f ms, block %d, mean %.1f it, max relres %.1e)" %
            (label, nsys / best, best * 1e3, blk, it.mean(), rr.max()))
        G.close()
    return out


WAVE_ROWS = 256   # largest system a wavefront solves alone in the batch's wavefront mode
LDS_PEAK_GBS = 256 * 128 * 2.4   # 256 CUs x 128 B/clk x 2.4 GHz


def batch_bound(g, torch, B, vals, bh, G, its, measured_s, floor_bytes):
    """Lower bounds on the batched solve's time and the fraction achieved.

    * HBM: one read of every system, b and x0, one write of x.
    * LDS: per system and iteration the p gathers of its entries and one p
      store per row (8 bytes each), against 256 CUs x 128 B/clk.
    * latency: an iteration cannot take less than on a workgroup (or, for the
      small systems of the wavefront mode, a wavefront) alone on the GPU.
      t_iter(m) is measured on one-system batches in the batch's workgroup
      size and mode (the smallest and the largest system, and in the
      wavefront mode also the largest system a wavefront takes and the
      smallest one above it; kernel time of the full solve minus a
      one-iteration solve) and interpolated in m within each kind; with R
      workgroups resident, each running one system or, in the wavefront
      mode, block / 64 small ones at a time, the batch needs at least
      max(sum_s its_s t_iter(m_s) / (R slots_s), max_s its_s t_iter(m_s)).
    fraction = the largest bound / the measured time."""
    m = np.diff(B.row_off)
    nz = np.diff(B.nnz_off)
    resident, lds_bytes = G.launch_info()
    waves = G.lds_mode == "waves"
    small = (m <= WAVE_ROWS) if waves else np.zeros(len(m), bool)
    probes = {int(np.argmin(m)), int(np.argmax(m))}
    if waves and small.any() and (~small).any():
        probes |= {int(np.flatnonzero(small)[np.argmax(m[small])]),
                   int(np.flatnonzero(~small)[np.argmin(m[~small])])}
    t_iter = {}
    for sid in sorted(probes):
        rp, c, _ = B.system(sid)
        k0, k1 = int(B.nnz_off[sid]), int(B.nnz_off[sid + 1])
        r0, r1 = int(B.row_off[sid]), int(B.row_off[sid + 1])
        one = g.Batch(np.array([0, r1 - r0], np.int64), np.array([0, k1 - k0], np.int64),
                      np.ascontiguousarray(rp), np.ascontiguousarray(c), vals[k0:k1],
                      dtype=torch.float64)
        b1 = torch.from_numpy(np.ascontiguousarray(bh[r0:r1])).cuda()
        x1 = torch.zeros(r1 - r0, dtype=torch.float64, device="cuda")
        one.block = G.block
        one.lds_mode = G.lds_mode
        ts = {}
        for mi in (1, 1000):
            best = None
            for _ in range(5):
                st, it1, _ = one.solve(b1, x1, tol=1e-10, maxit=mi)
                a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                one.solve(b1, x1, tol=1e-10, maxit=mi)
                e.record()
                torch.cuda.synchronize()
                ms = a.elapsed_time(e)
                best = ms if best is None else min(best, ms)
            ts[mi] = (best * 1e-3, int(it1.cpu()[0]))
        one.close()
        t_iter[int(m[sid])] = (ts[1000][0] - ts[1][0]) / max(ts[1000][1] - 1, 1)
    tm = np.empty(len(m))
    for kind in (True, False):
        sel = small == kind
        if not sel.any():
            continue
        pts = sorted((k, v) for k, v in t_iter.items() if (k <= WAVE_ROWS if waves else False) == kind)
        tm[sel] = np.interp(m[sel], [k for k, _ in pts], [v for _, v in pts])
    slots = np.where(small, G.block // 64, 1)
    work = its.astype(np.float64) * tm
    latency_s = max(float((work / slots).sum()) / resident, float(work.max()))
    lds_s = float((its.astype(np.float64) * (nz + m) * 8).sum()) / (LDS_PEAK_GBS * 1e9)
    hbm_s = floor_bytes / (HBM_PEAK_GBS * 1e9)
    bound = max(latency_s, lds_s, hbm_s)
    return {"resident_workgroups": resident, "lds_bytes_per_workgroup": lds_bytes,
            "mode": G.lds_mode,
            "t_iter_lone_us": {str(k): round(v * 1e6, 3) for k, v in t_iter.items()},
            "latency_floor_s": round(latency_s, 7), "lds_floor_s": round(lds_s, 7),
            "hbm_floor_s": round(hbm_s, 7), "bound": "latency" if bound == latency_s else
            ("lds" if bound == lds_s else "hbm"),
            "frac": round(bound / measured_s, 4)}


def run_sweep(args, g, gen, torch, result):
    mats, skipped, inputs, base = build_sweep(g, gen, torch)
    log("sweep matrices on device: %d SpMV kernels per step" % len(mats))

    def step(events=None):
        for k, e in enumerate(mats):
            if events is not None:
                events[k][0].record()
            g.spmv(e["M"], 1.0, e["x"], 0.0, e["y"])
            if events is not None:
                events[k][1].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in mats] for _ in range(args.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record()
    for s in range(args.steps):
        step(ev[s])
    t_end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t_start.elapsed_time(t_end)
    ms_per_step = total_ms / args.steps
    step_bytes = sum(e["bytes"] for e in mats)
    value = step_bytes / (ms_per_step * 1e-3) / 1e9

    per_kernel = []
    for k, e in enumerate(mats):
        ms = float(np.mean([ev[s][k][0].elapsed_time(ev[s][k][1]) for s in range(args.steps)]))
        per_kernel.append({"matrix": e["matrix"], "format": e["format"], "ms": round(ms, 5),
                           "GB/s": round(e["bytes"] / (ms * 1e-3) / 1e9, 1),
                           "useful_GB/s": round(e["useful_bytes"] / (ms * 1e-3) / 1e9, 1),
                           "GFLOP/s": round(e["flops"] / (ms * 1e-3) / 1e9, 1),
                           "frac_hbm_peak": round(e["bytes"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                           "alg_bytes": int(e["bytes"]),
                           "unread_padding_bytes": int(padding_bytes(e["desc"]))})
    dom = max(range(len(mats)), key=lambda k: per_kernel[k]["ms"])
    d = per_kernel[dom]
    achieved = d["alg_bytes"] / (d["ms"] * 1e-3) / 1e9
    traffic = measured_traffic("%s/%s" % (d["matrix"], d["format"]))
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "kernel": "spmv %s on %s" % (d["format"], d["matrix"]),
                "alg_bytes_per_launch": d["alg_bytes"]}
    if traffic:
        # bytes the L2 exchanged with the fabric (Infinity Cache hits included)
        # per second: above the algorithmic rate when x gathers miss the L2
        roofline["traffic_GB/s"] = round(traffic / (d["ms"] * 1e-3) / 1e9, 1)

    result.update({
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "FP64 SpMV sweep, formats csr/csr_merge/coo/ell/hybrid: 27-point "
                               "stencil 128^3 (n=2097152, nnz=55742968) and lognormal random "
                               "n=1e6 (mean 16, max 10000); one SpMV per format and matrix per step",
                   "frac_hbm_peak": round(value / HBM_PEAK_GBS, 4),
                   "step_alg_bytes": int(step_bytes),
                   "wall_s_timed": round(wall, 4),
                   "skipped": skipped},
        "roofline": roofline,
        "per_kernel": per_kernel,
    })
    log("sweep: %.1f GB/s aggregate (%.1f%% of 8 TB/s), %.3f ms/step" %
        (value, 100 * value / HBM_PEAK_GBS, ms_per_step))
    for p in per_kernel:
        log("  %-14s %-10s %8.4f ms %8.1f GB/s" % (p["matrix"], p["format"], p["ms"], p["GB/s"]))
    if args.calib_copy_mib:
        # one library COPY kernel of known size: reads and writes calib bytes
        nel = (args.calib_copy_mib << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        g.stream(g.STREAM_COPY, src, dst)
        torch.cuda.synchronize()
        result["calib_copy_bytes"] = nel * 8
        del src, dst
    result["stream"] = stream_probe(g, torch)
    log("stream probe: copy %.0f GB/s, triad %.0f GB/s; gather probe %.3f ms" %
        (result["stream"]["copy_GB/s"], result["stream"]["triad_GB/s"],
         result["stream"]["gather"]["ms"]))
    roofline["frac_of_stream_copy"] = round(achieved / result["stream"]["copy_GB/s"], 4)
    result["config"]["frac_of_stream_copy"] = round(value / result["stream"]["copy_GB/s"], 4)
    result["sellp"] = run_sellp(args, g, torch, base, mats, per_kernel)
    result["cache_protocol"] = cache_protocol(g, torch, mats)
    for e in mats:
        e["M"].close()
    for M in base.values():
        M.close()
    del mats
    torch.cuda.empty_cache()

    return result, inputs


def profile_sweep(args, g, gen, torch):
    """Launch sequence for rocprofv3 runs: every sweep SpMV (and SELL-P on the
    stencil) `reps` times in a group of its own, then the random-gather probe,
    each group opened by a small library COPY of 512 (k+1) doubles (grid
    256 (k+1) threads) that marks group k, and a 1 GiB COPY last (group
    "copy_1GiB") as the counters' calibration transfer.  Returns the groups."""
    mats, skipped, inputs, base = build_sweep(g, gen, torch)
    st = base["stencil27_128"].clone().convert("sellp")
    d = st.describe()
    mats.append({"matrix": "stencil27_128", "format": "sellp", "M": st,
                 "x": mats[0]["x"], "y": torch.empty(d.n_rows, dtype=torch.float64, device="cuda"),
                 "desc": d, "bytes": spmv_bytes(d)})
    sep_src = torch.zeros(512 * (len(mats) + 3), dtype=torch.float64, device="cuda")
    sep_dst = torch.empty_like(sep_src)
    rng = np.random.default_rng(41)
    gn, gm = 16_000_000, 1_000_000
    gidx = torch.from_numpy(rng.integers(0, gm, gn).astype(np.int32)).cuda()
    gx = torch.rand(gm, dtype=torch.float64, device="cuda")
    gy = torch.empty(gn, dtype=torch.float64, device="cuda")
    groups = []
    for k, e in enumerate(mats):
        g.stream(g.STREAM_COPY, sep_src[:512 * (k + 1)], sep_dst)
        for _ in range(args.steps):
            g.spmv(e["M"], 1.0, e["x"], 0.0, e["y"])
        groups.append({"name": "%s/%s" % (e["matrix"], e["format"]), "launches": args.steps,
                       "alg_bytes": int(e["bytes"])})
    # the random-gather probe as a group of its own
    k = len(mats)
    g.stream(g.STREAM_COPY, sep_src[:512 * (k + 1)], sep_dst)
    for _ in range(args.steps):
        g.gather_probe(gx, gidx, gy)
    groups.append({"name": "gather_probe/16M_of_8MB", "launches": args.steps,
                   "alg_bytes": gn * 12 + gm * 8})
    g.stream(g.STREAM_COPY, sep_src[:512 * (k + 2)], sep_dst)
    nel = (1 << 30) // 8
    src = torch.ones(nel, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    g.stream(g.STREAM_COPY, src, dst)
    groups.append({"name": "copy_1GiB", "launches": 1, "alg_bytes": 2 * nel * 8})
    torch.cuda.synchronize()
    return groups


def cache_protocol(g, torch, mats, reps=20, warmup=5, scratch_mib=1024):
    """Each sweep SpMV alone, outside the timed step: the median of `reps`
    single-launch event timings, warm (launches back to back, so a matrix that
    fits the 256 MB Infinity Cache is served from it) and cold (a 1 GiB fill
    of a scratch buffer before every launch evicts the L2s and the Infinity
    Cache).  The timed sweep sits between the two: its SpMVs alternate
    matrices, so the random matrix never runs right after itself."""
    scratch = torch.empty((scratch_mib << 20) // 8, dtype=torch.float64, device="cuda")
    out = []
    for e in mats:
        row = {"matrix": e["matrix"], "format": e["format"]}
        for mode in ("warm", "cold"):
            for _ in range(warmup):
                g.spmv(e["M"], 1.0, e["x"], 0.0, e["y"])
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(reps)]
            for k, (a, b) in enumerate(ev):
                if mode == "cold":
                    scratch.fill_(float(k))
                a.record()
                g.spmv(e["M"], 1.0, e["x"], 0.0, e["y"])
                b.record()
            torch.cuda.synchronize()
            ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
            row[mode + "_ms"] = round(ms, 5)
            row[mode + "_GB/s"] = round(e["bytes"] / (ms * 1e-3) / 1e9, 1)
        out.append(row)
        log("  %-14s %-10s warm %8.4f ms  cold %8.4f ms" % (row["matrix"], row["format"],
                                                          row["warm_ms"], row["cold_ms"]))
    del scratch
    return {"reps": reps, "scratch_bytes": scratch_mib << 20, "kernels": out}


def run_sellp(args, g, torch, base, mats, per_kernel):
    """SELL-P (sliced ELL, 64-row slices, not sorted) on the sweep matrices, next to
    ELL on the same matrix; outside the sweep aggregate, whose formats are fixed."""
    out = {}
    ell_ms = {p["matrix"]: p["ms"] for p in per_kernel if p["format"] == "ell"}
    for name, M0 in base.items():
        try:
            M = M0.clone().convert("sellp")
        except g.GkoError as e:
            assert e.status == g.ERR_UNSUPPORTED
            out[name] = {"skipped": "unsupported: SELL-P slots above 4x the CSR storage"}
            continue
        d = M.describe()
        x = next(e["x"] for e in mats if e["matrix"] == name)
        y = torch.empty(d.n_rows, dtype=torch.float64, device="cuda")
        for _ in range(args.warmup):
            g.spmv(M, 1.0, x, 0.0, y)
        reps = max(args.steps, 10)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(reps):
            g.spmv(M, 1.0, x, 0.0, y)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        nb = spmv_bytes(d)
        out[name] = {"ms": round(ms, 5), "GB/s": round(nb / (ms * 1e-3) / 1e9, 1),
                     "frac_hbm_peak": round(nb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "alg_bytes": int(nb), "unread_padding_bytes": int(padding_bytes(d)),
                     "slots": d.sellp_slots,
                     "padding_ratio": round(d.sellp_slots / max(d.nnz, 1), 4)}
        if name in ell_ms:
            out[name]["ell_ms_in_sweep"] = ell_ms[name]
        log("sellp %-14s %8.4f ms %8.1f GB/s (slots/nnz %.4f)" %
            (name, ms, out[name]["GB/s"], out[name]["padding_ratio"]))
        M.close()
    out["lognormal_sigma05_1M"] = sellp_mild_irregular(args, g, torch)
    return out


def time_spmv(g, torch, M, x, y, warmup, reps):
    for _ in range(warmup):
        g.spmv(M, 1.0, x, 0.0, y)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        g.spmv(M, 1.0, x, 0.0, y)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def sellp_mild_irregular(args, g, torch):
    """Lognormal rows with sigma 0.5 (mean 16, n = 10^6): irregular enough that
    ELL pads to the longest row, mild enough for 64-row slices.  Every format's
    SpMV time (ms) and its storage relative to CSR."""
    import gen
    A = gen.random_lognormal(9, 1_000_000, mean=16.0, sigma=0.5, max_len=10000)
    n = len(A[0]) - 1
    x = torch.from_numpy(gen.uniform(10, n)).cuda()
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    base = g.Matrix.from_csr(*A)
    csr_stored = base.describe().stored_bytes
    res = {"n": n, "nnz": int(len(A[1])), "max_row_len": int(np.diff(A[0]).max())}
    for fmt in ("csr", "csr_merge", "coo", "ell", "hybrid", "sellp"):
        try:
            M = base.clone().convert(fmt)
        except g.GkoError as e:
            assert e.status == g.ERR_UNSUPPORTED
            res[fmt] = {"skipped": "unsupported: padding above 4x the CSR storage"}
            continue
        d = M.describe()
        ms = time_spmv(g, torch, M, x, y, args.warmup, max(args.steps, 10))
        res[fmt] = {"ms": round(ms, 5), "storage_vs_csr": round(d.stored_bytes / csr_stored, 3)}
        M.close()
    base.close()
    log("sellp vs formats, lognormal sigma 0.5: " +
        ", ".join("%s %s" % (f, res[f].get("ms", "-")) for f in
                  ("csr", "csr_merge", "coo", "ell", "hybrid", "sellp")))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-solvers", action="store_true", help="skip the solver measurements")
    ap.add_argument("--selector-matrices", type=int, default=2000,
                    help="corpus size of the learned-selector leg (0 skips it)")
    ap.add_argument("--profile-sweep", default="",
                    help="only launch the sweep SpMVs in marked groups (--steps launches "
                         "each) for rocprofv3, and write the group list to this JSON file")
    ap.add_argument("--oracle-poisson-worker", choices=("fp64", "mixed"), default=None,
                    help=argparse.SUPPRESS)
    ap.add_argument("--worker-dir", default="", help=argparse.SUPPRESS)
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the SpMV sweep (profiling the solvers alone)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the sweep, copy this many MiB device-to-device (a transfer of "
                         "known size for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.oracle_poisson_worker:
        oracle_poisson_worker(args.worker_dir, args.oracle_poisson_worker)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import gen
    if not os.path.exists(gen._LIB):
        gen.build()
    # the config-3 oracle solves start first, before anything touches the GPU
    workers = None
    if not args.no_cpu and not args.no_solvers and not args.profile_sweep:
        import oracle
        if not os.path.exists(oracle._LIB):
            oracle.build()
        workers = start_oracle_workers()

    import torch

    import paper_2011_08879_amd as g

    torch.cuda.set_device(0)
    g.default_context()
    if args.profile_sweep:
        groups = profile_sweep(args, g, gen, torch)
        with open(args.profile_sweep, "w") as fh:
            json.dump({"groups": groups, "marker": "stream_copy_kernel",
                       "source_sha256": kernel_source_hash()}, fh, indent=1)
        log("profile groups written: %d" % len(groups))
        return
    result = {"metric": METRIC, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
              "dtype": "f64", "data": "synthetic"}
    inputs = None
    if not args.no_sweep:
        result, inputs = run_sweep(args, g, gen, torch, result)

    keep = {}
    if not args.no_solvers:
        result["solvers"] = run_solvers(g, gen, torch, keep)
    poisson = None
    if workers is not None:
        # the oracle solves finish before the selector leg loads the host cores
        log("waiting for the oracle's Poisson 256^3 solves ...")
        poisson, errs = finish_oracle_workers(workers, keep.get("poisson256"), deadline_s=420.0)
        keep.pop("poisson256", None)
        pc = result["solvers"]["pcg_bj8_poisson3d_256"]
        for label in ("fp64", "mixed"):
            if "gpu_" + label in errs:
                pc[label]["rel_error_vs_oracle_fp64"] = errs["gpu_" + label]
        pc["oracle_check"] = errs
        log("poisson oracle: %s; errors vs oracle FP64 x: %s" %
            ({k: v.get("seconds", v) for k, v in poisson.items()}, errs))
    sel_lat = None
    if args.selector_matrices > 0:
        import paper_2011_08879_amd.selector as sel
        t0 = time.time()
        res, model = sel.run(n_matrices=args.selector_matrices, n_lo=1e4, n_hi=1e6, steps=3000,
                             lr=3e-3, workers=8, log=log, retimed=True, five_class=True)
        res["wall_s"] = round(time.time() - t0, 1)
        result["selector"] = res
        sel_lat = res["latency"]
        log("selector (%d matrices): test regret %.3f (CSR alone %.3f), gain vs CSR %.3f" %
            (args.selector_matrices, res["test"]["regret_total"], res["test"]["csr_regret_total"],
             res["test"]["gain_vs_csr_total"]))
        model.close()
    if not args.no_cpu and inputs is not None:
        log("cpu baseline (oracle, 1 core) ...")
        cb = cpu_baseline(inputs, result["config"]["step_alg_bytes"])
        cb["host"] = host_info()
        cb.update(cpu_solver_baselines(keep, result.get("solvers"), sel_lat))
        if poisson is not None:
            cb["pcg_bj8_poisson3d_256"] = dict(
                poisson, note="each solve serial on its own host core, run beside the GPU legs")
            for label in ("fp64", "mixed"):
                if "seconds" in poisson.get(label, {}):
                    poisson[label]["gpu_seconds"] = \
                        result["solvers"]["pcg_bj8_poisson3d_256"][label]["seconds"]
        result["cpu_baseline"] = cb
        log("cpu baseline: %.2f GB/s" % result["cpu_baseline"]["value"])
    print(json.dumps(result))


if __name__ == "__main__":
    main()
