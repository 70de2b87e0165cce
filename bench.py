"""Benchmark: forward Maxwell solves per second on one MI355X.

Workload (default): the synthetic imaging chamber -- cylinder R = 0.15 m,
H = 0.28 m meshed as a 5-block O-grid (22 x 11 radial x 27 layers of cells,
Kuhn-split), degree-2 edge elements (1,477,926 unknowns after removing the
metallic wall and bottom), background eps = 44+20i with a seeded head
(40+15i) and a +-20 % inclusion, 1 GHz, 1,728 block-aligned core subdomains
(3 x 3 x 3 cells each), 2 face layers of overlap (n_s <= 3,474), 32
z-polarised dipoles on the 0.14 m ring solved together by block FGMRES(50),
complex-FP32 local LU and solves, everything else in FP64.  A step is one
complete forward solve of the 32 sources: FP64 element matrices with this
step's medium, CSR assembly of A, dense local matrices A_s, batched LU of
every A_s, right-hand sides, and ORAS-preconditioned block FGMRES to a true
relative residual of 1e-8 for every source.  The per-mesh host setup
(entity numbering, CSR pattern, overlapping subdomains), its device copy and
the problem's device buffers are built once before the timed region
(reported separately); each step redoes all medium-dependent work in those
buffers, as an imaging loop does when only the permittivity changes.

After the steps, the plain path is timed on the same chamber and medium
(FP64 local factors, one dipole, 3,465 subdomains of 2 x 2 x 3 cells: a
whole forward solve from the medium), and the oracle's timing, run on the
host cores in a process of its own beside the GPU steps, is collected.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import atexit
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "forward Maxwell solves/s on 1 GPU at rel. residual 1e-8; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash(name):
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_1605_04521_amd", "csrc", name), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


KERNEL_SOURCES = {"lu": "lu_kernels.hip", "local_solve": "solve_kernels.hip", "spmv": "solve_kernels.hip",
                  "local_solve_multi": "multi_solve.hip"}


def measured_traffic(kernel, precision, nrhs, nsub="2x2x3"):
    """HBM bytes per launch from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by a copy of known size), if it was taken
    on this partition with the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    rec = data.get(f"{kernel}|{precision}|{nrhs}|{nsub}")
    if rec is None and nsub == "2x2x3":
        rec = data.get(f"{kernel}|{precision}|{nrhs}")
    if not rec or rec.get("source_hash") != kernel_source_hash(KERNEL_SOURCES[kernel]):
        return None
    return rec.get("bytes_per_launch")


# ---------------------------------------------------------------------------
# CPU baseline: the oracle on the host cores, in a process of its own that is
# started before anything touches the GPU and runs beside the GPU steps
# ---------------------------------------------------------------------------
def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_ORC = {}


def _oracle_local_job(s):
    """Oracle local setup (A_s assembly with the transmission term + SuperLU)
    and one solve of the block's columns, for subdomain s (in a worker)."""
    import scipy.sparse.linalg as spla
    from oracle.schwarz import Subdomain, grow_overlap, local_matrix
    d, part, own, layers, X = _ORC["d"], _ORC["part"], _ORC["own"], _ORC["layers"], _ORC["X"]
    t0 = time.perf_counter()
    tets = grow_overlap(d, part, int(s), layers)
    in_s = np.zeros(d.topo.n_tets, dtype=bool)
    in_s[tets] = True
    dd = d.dofs.tet_dofs[tets].ravel()
    dofs = np.unique(dd[dd >= 0])
    iface = []
    for t in tets:
        for lf, f in enumerate(d.topo.tet_faces[t]):
            other = [u for u in d.topo.face_tets[f] if u >= 0 and u != t]
            if other and not in_s[other[0]]:
                iface.append((int(t), lf, d.k0 * np.sqrt(d.eps[t].real)))
    sub = Subdomain(int(s), tets, dofs, (own[dofs] == s).astype(np.uint8), iface)
    lu = spla.splu(local_matrix(d, sub))
    t1 = time.perf_counter()
    lu.solve(np.ascontiguousarray(X[sub.dofs]))
    t2 = time.perf_counter()
    return t1 - t0, t2 - t1


def _oracle_rows_job(job):
    """One worker's share of the rows: the product of A's rows with the
    block's columns, or the oracle's block MGS of one step (q previous
    blocks of the block's width) on `rows` rows of random data."""
    kind, lo, hi, q = job
    A, X = _ORC["A"], _ORC["X"]
    t0 = time.perf_counter()
    if kind == "spmm":
        A[lo:hi] @ X
    else:
        rng = np.random.default_rng(lo)
        p = X.shape[1]
        V = [rng.standard_normal((hi - lo, p)) + 1j * rng.standard_normal((hi - lo, p)) for _ in range(q)]
        W = rng.standard_normal((hi - lo, p)) + 1j * rng.standard_normal((hi - lo, p))
        t0 = time.perf_counter()
        for Vi in V:
            H = Vi.conj().T @ W
            W -= Vi @ H
    return time.perf_counter() - t0


def cpu_baseline_worker(args):
    """The oracle timed on a bounded sample of the benchmark's workload, on
    up to `cpu_workers` host processes; prints one JSON line.

    Every process runs single-threaded BLAS.  Timed in full: the oracle's
    global setup (entities, numbering, element matrices, global matrix,
    owners; one process) and one product of A with the block's columns (rows
    split over the pool).  Sampled: the local setup (A_s with its
    transmission term + SuperLU) and one solve of the block's columns for
    cpu_sample random subdomains on the pool, the pool's wall time per
    subdomain scaled to all subdomains; the oracle's block MGS of one block
    step against the mean basis size of a cycle, on 100k rows per process,
    scaled to all rows.  One solve of the block = setup + steps x (ORAS
    application + product with A + orthogonalisation), with the block step
    count the GPU run reports."""
    import multiprocessing as mp
    import signal
    from oracle.assemble import Discretization
    from oracle.schwarz import owners
    from paper_1605_04521_amd import gen

    # stopped by the benchmark (SIGTERM): leave through the normal exit path,
    # whose pool cleanup also ends the pool's workers (they keep the default
    # action, set by the pool's initializer)
    signal.signal(signal.SIGTERM, lambda *_: sys.exit(1))
    nsub = tuple(int(q) for q in args.nsub.split("x")) if "x" in args.nsub else int(args.nsub)
    prob = gen.chamber_problem(n=args.n, nz=args.nz, degree=args.degree, n_sub=nsub, overlap=args.overlap,
                               seed=args.seed, n_sources=max(args.nrhs, 1))
    m = prob.mesh
    t0 = time.perf_counter()
    d = Discretization(m.xyz, m.tets, prob.eps, m.bfaces, m.bface_kind, prob.k0, prob.degree)
    A = d.global_matrix()
    own = owners(d, prob.part)
    t_global = time.perf_counter() - t0
    rng = np.random.default_rng(args.seed)
    p = max(args.nrhs, 1)
    X = rng.standard_normal((d.ndof, p)) + 1j * rng.standard_normal((d.ndof, p))
    _ORC.update(d=d, A=A, part=prob.part, own=own, layers=prob.overlap, X=X)
    picks = rng.choice(prob.n_sub, size=min(args.cpu_sample, prob.n_sub), replace=False)
    workers = max(1, min(args.cpu_workers, os.cpu_count() or 1))
    q = max(1, (args.restart + 1) // 2)        # mean number of previous blocks in a cycle
    rows = min(d.ndof // workers, 100000)
    bounds = np.linspace(0, d.ndof, workers + 1).astype(np.int64)
    ctx = mp.get_context("fork")
    with ctx.Pool(workers, initializer=signal.signal, initargs=(signal.SIGTERM, signal.SIG_DFL)) as pool:
        t0 = time.perf_counter()
        pool.map(_oracle_rows_job, [("spmm", int(bounds[w]), int(bounds[w + 1]), 0) for w in range(workers)],
                 chunksize=1)
        t_spmm = time.perf_counter() - t0
        t0 = time.perf_counter()
        pool.map(_oracle_rows_job, [("mgs", w * rows, (w + 1) * rows, q) for w in range(workers)], chunksize=1)
        t_orth = (time.perf_counter() - t0) * d.ndof / (rows * workers)
        t0 = time.perf_counter()
        res = pool.map(_oracle_local_job, list(picks), chunksize=1)
        wall = time.perf_counter() - t0
    ts = np.array(res)
    share_setup = ts[:, 0].sum() / ts.sum()
    per_sub = wall / len(picks)
    t_setup_all = prob.n_sub * per_sub * share_setup
    t_apply = prob.n_sub * per_sub * (1 - share_setup)
    out = {"t_global": t_global, "t_spmm": t_spmm, "t_orth": t_orth, "t_setup_all": t_setup_all,
           "t_apply": t_apply, "workers": workers, "sample": len(picks), "n_sub": prob.n_sub, "nrhs": p,
           "mean_setup_s": float(ts[:, 0].mean()), "mean_solve_s": float(ts[:, 1].mean()), "pool_wall_s": wall,
           "cpu_model": _cpu_model(), "host_cpus": os.cpu_count()}
    print(json.dumps(out), flush=True)


def start_cpu_baseline(args):
    """Starts the oracle's timing in a child process (before any GPU work)."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline-worker", "--n", str(args.n), "--nz",
           str(args.nz), "--degree", str(args.degree), "--nsub", args.nsub, "--overlap", str(args.overlap),
           "--nrhs", str(args.nrhs), "--restart", str(args.restart), "--seed", str(args.seed),
           "--cpu-sample", str(args.cpu_sample), "--cpu-workers", str(args.cpu_workers)]
    env = dict(os.environ, HIP_VISIBLE_DEVICES="", CUDA_VISIBLE_DEVICES="", OMP_NUM_THREADS="1",
               OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    return subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=env)


def stop_child(proc):
    """Ends the oracle's timing child if it still runs: SIGTERM first (the
    child then leaves through its process pool's cleanup), SIGKILL after 10 s."""
    import subprocess
    if proc.poll() is None:
        proc.terminate()
        try:
            proc.communicate(timeout=10)
        except subprocess.TimeoutExpired:
            proc.kill()
            proc.communicate()


def finish_cpu_baseline(proc, steps, timeout):
    """Collects the child's timings and forms solves/s for a solve of the
    block that takes `steps` block steps."""
    try:
        out, err = proc.communicate(timeout=timeout)
    except Exception:
        proc.kill()
        proc.communicate()
        return None
    lines = [l for l in out.splitlines() if l.startswith("{")]
    if proc.returncode != 0 or not lines:
        log(f"[bench] oracle timing failed: {err[-500:]}")
        return None
    r = json.loads(lines[-1])
    per_solve = r["t_global"] + r["t_setup_all"] + steps * (r["t_apply"] + r["t_spmm"] + r["t_orth"])
    return {
        "value": r["nrhs"] / per_solve, "unit": "solves/s", "cores": r["workers"], "kind": "oracle",
        "cpu_model": r["cpu_model"], "host_cpus": r["host_cpus"],
        "sample": (f"oracle (NumPy/SciPy FP64) on the same chamber and partition: global setup and one product "
                   f"of A with the {r['nrhs']} columns timed in full ({r['t_global']:.1f} s, {r['t_spmm']:.2f} s); "
                   f"local setup (A_s + SuperLU) and one {r['nrhs']}-column local solve for {r['sample']} random "
                   f"of {r['n_sub']} subdomains on {r['workers']} processes ({r['pool_wall_s']:.1f} s wall, "
                   f"{r['mean_setup_s'] * 1e3:.0f} / {r['mean_solve_s'] * 1e3:.1f} ms each), scaled to every "
                   f"subdomain; block MGS of one step at the mean basis size of a cycle timed on 100k rows per "
                   f"process and scaled to all rows ({r['t_orth']:.2f} s); {steps} block steps as on the GPU; "
                   f"single-threaded BLAS in every process"),
        "seconds_per_solve_of_block": per_solve,
    }


def build_workload(args):
    """The seeded problem and its host layout (entities, CSR pattern,
    overlapping subdomains), built once per mesh."""
    from paper_1605_04521_amd import gen
    from paper_1605_04521_amd.api import Layout
    t0 = time.perf_counter()
    if args.workload == "cube":
        prob = gen.cube_planewave_problem(n=args.n, degree=args.degree, seed=args.seed, n_sources=args.nrhs)
        wl = f"unit cube {args.n}^3 Kuhn, r={args.degree}, plane wave, 2x2x2 boxes"
    else:
        nsub = tuple(int(q) for q in args.nsub.split("x")) if "x" in args.nsub else int(args.nsub)
        prob = gen.chamber_problem(n=args.n, nz=args.nz, degree=args.degree, n_sub=nsub, overlap=args.overlap,
                                   seed=args.seed, n_sources=max(args.nrhs, args.nsources))
        kind = f"{args.nsub}-cell block-aligned" if "x" in args.nsub else "RCB"
        srcs = f"{max(args.nrhs, args.nsources)} dipole(s)"
        if args.ports:
            width = min(0.03, 0.8 * 2.0 * np.pi * 0.1 / args.ports)   # neighbours do not overlap
            prob.sources = gen.top_ports(args.ports, ring=0.1, width=width, narrow=0.5 * width)
            srcs = (f"{args.ports} TE10 ports on the top ({100 * width:.2f} x {50 * width:.2f} cm, ring r = 10 cm) "
                    f"and their S-matrix")
        wl = (f"imaging chamber cylinder R=0.15 m H=0.28 m, O-grid {args.n}x{args.n // 2}x{args.nz}, "
              f"r={args.degree}, {prob.n_sub} {kind} subdomains, {args.overlap} face layers, "
              f"{srcs}, eps 44+20i / head 40+15i / inclusion")
    lay = Layout.from_problem(prob)
    info = lay.info()
    t_mesh = time.perf_counter() - t0
    log(f"[bench] {wl}: ndof={info.ndof} nnz={info.nnz} n_sub={info.n_sub} max_ns={info.max_ns} "
        f"sum_ns2={info.sum_ns2:.3e} host setup {t_mesh:.1f}s")
    return prob, lay, info, wl, t_mesh


def kernel_rooflines(info, precision, nrhs):
    """Per-kernel achieved rates from the in-dispatch HIP-event timers:
    algorithmic bytes or flops per launch / average launch duration."""
    from paper_1605_04521_amd import _lib as B
    from paper_1605_04521_amd.api import kernel_time
    ktimes = {}
    for name in ("lu", "local_solve", "local_solve_multi", "spmv"):
        ktimes[name] = kernel_time(name)
    rsz = 8 if precision == B.MXW_FP64 else 4
    mfma_peak = FP64_PEAK_TFLOPS if precision == B.MXW_FP64 else FP32_PEAK_TFLOPS
    lu_flops = 8.0 / 3.0 * info.sum_ns3            # complex LU: 8 n^3 / 3 real flops
    # one column: every factor entry once (2 planes), restrict + prolong vectors
    solve_bytes = 2 * rsz * info.sum_ns2 + 16 * info.sum_ns * 2 + 16 * info.ndof * 2
    kern = {}

    def add(name, bound, amount, peak, unit, **extra):
        ms, n = ktimes[name]
        if not n:
            return
        avg = ms / n / 1e3
        kern[name] = dict(bound=bound, achieved=amount / avg / (1e12 if unit == "TFLOP/s" else 1e9), peak=peak,
                          unit=unit, avg_ms=avg * 1e3, launches=n, total_ms=ms, **extra)

    add("lu", "mfma", lu_flops, mfma_peak, "TFLOP/s")
    add("local_solve", "hbm", nrhs * solve_bytes, HBM_PEAK_GBS, "GB/s")
    # all columns of a 32-column chunk per factor read: MFMA-bound at 32 columns
    add("local_solve_multi", "mfma", 8.0 * info.sum_ns2 * nrhs, mfma_peak, "TFLOP/s")
    if "local_solve_multi" in kern:
        k = kern["local_solve_multi"]
        k["factor_GBps"] = 2 * rsz * info.sum_ns2 / (k["avg_ms"] / 1e3) / 1e9
    # matrix once (16 B value + 4 B index per entry, row pointers), x read and y written per column
    add("spmv", "hbm", 20 * info.nnz + 8 * (info.ndof + 1) + 32 * info.ndof * nrhs, HBM_PEAK_GBS, "GB/s")
    for v in kern.values():
        v["frac"] = v["achieved"] / v["peak"]
    return kern


def kernels_probe(args):
    """Each hot kernel launched a few times on the chamber workload (no
    solve): the LU of every A_s once, then --steps applications of ORAS and
    of A to --nrhs random columns; then a 1 GiB device copy, whose counter
    readings calibrate FETCH_SIZE / WRITE_SIZE.  Meant to run under
    rocprofv3; prints one JSON line with the HIP-event kernel timings."""
    import torch
    from paper_1605_04521_amd import _lib as B
    from paper_1605_04521_amd.api import Problem, reset_timing, timing
    precision = B.MXW_FP64 if args.precision == "fp64" else B.MXW_MIXED
    prob, lay, info, wl, _ = build_workload(args)
    timing(True)
    reset_timing()
    P = Problem.from_layout(lay, eps=prob.eps, k0=prob.k0, precision=precision)
    g = torch.Generator(device="cuda").manual_seed(args.seed)
    V = torch.complex(torch.randn(args.nrhs, info.ndof, dtype=torch.float64, device="cuda", generator=g),
                      torch.randn(args.nrhs, info.ndof, dtype=torch.float64, device="cuda", generator=g))
    for i in range(args.steps):
        P.apply_prec(V)
        P.apply_A(V)
        log(f"[kernels] application {i} done")
    torch.cuda.synchronize()
    timing(False)
    x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    out = {"workload": "kernels", "config": wl, "precision": args.precision, "nrhs": args.nrhs,
           "applications": args.steps, "copy_bytes": 1 << 30,
           "kernels": kernel_rooflines(info, precision, args.nrhs),
           "source_hash": {k: kernel_source_hash(v) for k, v in KERNEL_SOURCES.items()}}
    print(json.dumps(out), flush=True)


SERVE_CATALOGUE = {
    # key: (centre cells n, layers nz, degree, core cells), O-grid chamber, 2 face layers; the core
    # cells keep the largest subdomain at 1.9k-4k unknowns (at r = 1, 2x2x3 cells give subdomains
    # of at most 443 unknowns and one-level ORAS then needs thousands of iterations)
    "r1-0.27M": (22, 27, 1, (4, 4, 6)),
    "r1-1.2M": (36, 44, 1, (4, 4, 6)),
    "r2-0.23M": (12, 14, 2, (2, 2, 3)),
    "r2-1.48M": (22, 27, 2, (3, 3, 3)),
    "r3-0.21M": (8, 10, 3, (1, 2, 2)),
    "r3-0.71M": (12, 15, 3, (2, 2, 2)),
}


def serve_bench(args):
    """Serving: a Poisson stream (4 requests/s) of forward solves on a
    catalogue of chamber meshes (r = 1, 2, 3; 0.2 M to 1.5 M unknowns), each
    request with its own seeded head and inclusion (a new medium every time)
    and 1-32 ring dipoles; mixed precision, block GMRES per request,
    continuous batching over 4 slots; per-subdomain factor residency (a
    resident problem on the request's mesh keeps the factors of subdomains
    whose elements the new medium leaves unchanged).  Run for --duration
    seconds of arrivals (or --requests requests).  Compared with the plain
    path on the same stream: FP64 factors, one source at a time, every
    subdomain factorised for every request, with its per-mesh factorisation
    and single-source solve times measured once per mesh."""
    import torch
    from paper_1605_04521_amd import _lib as B
    from paper_1605_04521_amd import gen
    from paper_1605_04521_amd.api import Problem
    from paper_1605_04521_amd.serve import GpuBackend, Request, Server, latency_stats, poisson_arrivals

    keys = list(SERVE_CATALOGUE)
    catalogue = {k: gen.chamber_problem(n=n, nz=nz, degree=r, n_sub=blk, overlap=2)
                 for k, (n, nz, r, blk) in SERVE_CATALOGUE.items()}
    ring = [s for z in (0.084, 0.140, 0.196) for s in gen.ring_dipoles(32, 0.14, z)]
    rng = np.random.default_rng(args.seed)
    arrivals = poisson_arrivals(args.requests, 4.0, args.seed)
    reqs = []
    for i in range(args.requests):
        key = keys[int(rng.integers(len(keys)))]
        nsrc = int(rng.integers(1, 33))
        pick = rng.choice(len(ring), size=nsrc, replace=False)
        eps = gen.chamber_eps(catalogue[key].mesh, 1000 + i)[0]        # the request's own head
        reqs.append(Request(rid=i, arrival=float(arrivals[i]), mesh=key, eps=eps,
                            sources=[ring[j] for j in sorted(pick)], precision=B.MXW_MIXED))
    budget = int(args.budget_gb * 1e9)
    backend = GpuBackend(catalogue, budget=budget, slots=4)
    sizes = {k: backend.layouts[k].info().ndof for k in keys}
    log("[serve] catalogue: " + ", ".join(f"{k}: {sizes[k]} unknowns" for k in keys))
    # warm-up (untimed): device copies of every mesh and one resident problem each
    warm = [Request(rid=-1 - j, arrival=0.0, mesh=k, eps=catalogue[k].eps, sources=ring[:1], precision=B.MXW_MIXED)
            for j, k in enumerate(keys)]
    Server(backend, budget=budget, slots=4).run(warm, realtime=False)
    def finished(r):   # one line per completed request (the run's progress)
        state = f"failed: {r.error[:300]}" if r.error else f"{len(r.sources)} sources, {r.reused}"
        log(f"[serve] request {r.rid} on {r.mesh} done at {r.finish:.1f}s ({state})")

    server = Server(backend, budget=budget, slots=4, on_finish=finished)
    wall = server.run(reqs, realtime=True, deadline=args.duration or None)
    done = [r for r in reqs if r.error is None and r.finish is not None]
    bad = [r for r in done if r.relres is None or np.max(r.relres) > 1e-8]
    st = latency_stats(done)
    refac = sum(r.refactored[0] for r in done if r.refactored)
    total_sub = sum(r.refactored[1] for r in done if r.refactored)
    log(f"[serve] {len(done)} of {len(reqs)} requests served, {sum(len(r.sources) for r in done)} solves in "
        f"{wall:.1f}s; p50 {st['p50_s']:.2f}s p99 {st['p99_s']:.2f}s; subdomains re-factorised "
        f"{refac} of {total_sub}")
    # plain path, per mesh: one full factorisation and one single-source solve
    per_mesh = {}
    for k in sorted({r.mesh for r in done}):
        for e in list(backend.idle):
            e.problem.close()
        backend.idle.clear()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        base = catalogue[k]
        P = Problem.from_layout(backend.layouts[k], eps=base.eps, k0=base.k0, precision=B.MXW_FP64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.forget_factors()
        P.set_medium(base.eps, base.k0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x, it, rr, _ = P.solve(ring[:1])
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        P.close()
        per_mesh[k] = {"factor_s": t1 - t0, "solve_s": t2 - t1, "iterations": int(it[0])}
        log(f"[serve] plain FP64 on {k}: factorisation {t1 - t0:.2f}s, one source {t2 - t1:.2f}s ({it[0]} its)")
    nsol = sum(len(r.sources) for r in done)
    t_plain = sum(per_mesh[r.mesh]["factor_s"] + len(r.sources) * per_mesh[r.mesh]["solve_s"] for r in done)
    base_rate = nsol / t_plain
    out = {
        "metric": METRIC, "value": st["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": len(done),
        "warmup": len(warm), "ms_per_step": 1e3 * wall / max(1, len(done)), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "serving: Poisson 4 req/s, chamber meshes " +
                   ", ".join(f"{k} ({sizes[k]} unknowns)" for k in keys) +
                   ", a new seeded head per request, 1-32 dipoles per request, mixed precision, block GMRES, "
                   "4 slots, per-subdomain factor residency",
                   "requests_arrived": len(reqs), "requests_served": len(done),
                   "requests_not_started_by_the_end": sum(1 for r in reqs if r.start is None),
                   "failed_or_unconverged": sum(1 for r in reqs if r.start is not None and r.error) + len(bad),
                   "duration_s": args.duration or None,
                   "budget_gb": args.budget_gb},
        "latency_s": {"p50": st["p50_s"], "p99": st["p99_s"]},
        "reuse": {"factors_kept_fraction": 1.0 - refac / max(1, total_sub),
                  "requests": {k: sum(1 for r in done if r.reused == k) for k in ("factors", "partial", "new")}},
        "plain_fp64_single_rhs": {"value": base_rate, "unit": "solves/s", "per_mesh": per_mesh,
                                  "note": "the same served requests, one source at a time, FP64 factors, every "
                                          "subdomain factorised per request; per-mesh times measured once"},
        "speedup_vs_plain": st["solves_per_s"] / base_rate,
        "memory": {"admission_max_gb": backend.max_allocated / 1e9, "context_peak_gb":
                   backend.ctx.usage()["peak"] / 1e9},
    }
    print(json.dumps(out), flush=True)


def plain_fp64_rate(args, prob, lay_target):
    """The plain path on the same chamber and medium: FP64 local factors, one
    dipole, on the partition the FP64 factors fit best (block-aligned 2x2x3
    cells); one forward solve timed from the medium (assembly + LU of every
    subdomain) to the converged field."""
    import torch
    from paper_1605_04521_amd import _lib as B
    from paper_1605_04521_amd import gen
    from paper_1605_04521_amd.api import Layout, Problem
    if args.nsub == "2x2x3" and args.overlap == 2:
        lay = lay_target
        ref = prob
    else:
        ref = gen.chamber_problem(n=args.n, nz=args.nz, degree=args.degree, n_sub=(2, 2, 3), overlap=2,
                                  seed=args.seed, n_sources=1)
        lay = Layout.from_problem(ref)
    P = Problem.from_layout(lay, eps=ref.eps, k0=ref.k0, precision=B.MXW_FP64)   # device copy, untimed
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.forget_factors()
    P.set_medium(ref.eps, ref.k0)
    x, it, rr, st = P.solve(ref.sources[:1])
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    P.close()
    del P
    torch.cuda.empty_cache()
    assert rr[0] <= 1e-8
    return {"value": 1.0 / t, "unit": "solves/s", "seconds_per_solve": t, "iterations": int(it[0]),
            "config": f"FP64 local factors, 1 dipole, pseudo-block FGMRES({args.restart}), "
                      f"{lay.info().n_sub} block-aligned 2x2x3-cell subdomains, 2 face layers, same chamber and medium"}


def main():
    t_program = time.perf_counter()
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="chamber", choices=["chamber", "cube", "serve", "kernels"])
    ap.add_argument("--requests", type=int, default=24)
    ap.add_argument("--duration", type=float, default=0.0,
                    help="serving: stop submitting after this many seconds (0: all requests)")
    ap.add_argument("--budget-gb", type=float, default=250.0)
    ap.add_argument("--n", type=int, default=22)
    ap.add_argument("--nz", type=int, default=27)
    ap.add_argument("--degree", type=int, default=2)
    ap.add_argument("--nsub", default="3x3x3",
                    help="RCB subdomain count, or AxBxC cells per block-aligned core subdomain")
    ap.add_argument("--overlap", type=int, default=2)
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed"])
    ap.add_argument("--nrhs", type=int, default=32, help="right-hand sides per solve (one block)")
    ap.add_argument("--nsources", type=int, default=0,
                    help="sources per step, solved nrhs at a time (default: nrhs)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=96, help="subdomains the oracle's local setup is timed on")
    ap.add_argument("--cpu-workers", type=int, default=12, help="host processes of the oracle timing")
    ap.add_argument("--cpu-baseline-worker", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain FP64 single-source solve timed after the steps")
    ap.add_argument("--time-budget", type=float, default=560.0,
                    help="seconds after which the optional legs (plain FP64 solve, oracle timing) are skipped")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--restart", type=int, default=50)
    ap.add_argument("--variant", default="oras", choices=["oras", "oas", "ras", "oras_mult"],
                    help="Schwarz variant: Robin (ORAS), no partition of unity (OAS), Dirichlet (RAS), "
                         "Robin with the multiplicity partition of unity (ORAS_MULT)")
    ap.add_argument("--krylov", default="block", choices=["pseudo", "block"],
                    help="pseudo-block (one Krylov space per source) or block GMRES (one shared space)")
    ap.add_argument("--keep-factors", action="store_true",
                    help="let a step keep the factors of subdomains whose local data did not change "
                         "(default: every step factorises every subdomain)")
    ap.add_argument("--ports", type=int, default=0,
                    help="excite this many synthetic TE10 ports (one solve each) and form their S-matrix per step")
    ap.add_argument("--sequence", action="store_true",
                    help="slowly varying media: step i scales eps by 1 + 0.01 i (an imaging-loop sequence)")
    ap.add_argument("--recycle", type=int, default=0,
                    help="solve with GCRO-DR, recycling a space of this many vectors from system to system "
                         "(Block GCRO-DR with --krylov block and 2..16 sources per block)")
    ap.add_argument("--e-error", action="store_true",
                    help="mixed precision: after the timed steps, solve the last step's sources again with FP64 "
                         "factors and report each source's relative E-field difference")
    ap.add_argument("--tune", action="store_true",
                    help="after the warm-up, time the tile choices on the problem and keep the fastest")
    ap.add_argument("--graph", action="store_true",
                    help="replay each Arnoldi step as a captured HIP graph (kernel timers are off inside graphs)")
    args = ap.parse_args()

    if args.cpu_baseline_worker:
        cpu_baseline_worker(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU: --gpus must be 1 (sharding over several "
                                   "GPUs is not implemented)", "n_gpus": args.gpus}))
        sys.exit(2)
    # the oracle's timing runs on the host cores beside the GPU work; started
    # before anything touches the GPU
    cpu_proc = None
    if args.workload == "chamber" and not args.no_cpu_baseline:
        cpu_proc = start_cpu_baseline(args)
        log(f"[bench] oracle timing started in process {cpu_proc.pid}")
        # whatever ends this process (no GPU, an error) also ends the child;
        # after a normal run it has already been collected
        atexit.register(stop_child, cpu_proc)

    import torch
    from paper_1605_04521_amd import _lib as B
    from paper_1605_04521_amd import gen
    from paper_1605_04521_amd.api import Layout, Problem, kernel_time, reset_timing, timing

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    torch.cuda.init()
    if args.workload == "serve":
        serve_bench(args)
        return
    if args.workload == "kernels":
        kernels_probe(args)
        return
    precision = B.MXW_FP64 if args.precision == "fp64" else B.MXW_MIXED
    krylov = B.MXW_KRYLOV_BLOCK if args.krylov == "block" else B.MXW_KRYLOV_PSEUDOBLOCK
    nsources = args.nsources if args.nsources > 0 else args.nrhs
    if args.ports:
        nsources = args.ports

    prob, lay, info, wl, t_mesh = build_workload(args)
    footprint = lay.footprint(precision, args.nrhs, restart=args.restart, krylov=krylov)
    log(f"[bench] device footprint {footprint/1e9:.1f} GB")

    phases = []
    # device buffers of the problem are allocated once (untimed); every step
    # redoes all medium-dependent work in them: element matrices, CSR values,
    # dense A_s, batched LU of every subdomain, right-hand sides and the solve
    holder = {}

    def one_step():
        t0 = time.perf_counter()
        eps = prob.eps
        if args.sequence:
            eps = prob.eps * (1.0 + 0.01 * holder.get("seq", 0))
            holder["seq"] = holder.get("seq", 0) + 1
        if "P" not in holder:
            variant = {"oras": B.MXW_PREC_ORAS, "oas": B.MXW_PREC_OAS, "ras": B.MXW_PREC_RAS,
                       "oras_mult": B.MXW_PREC_ORAS_MULT}[args.variant]
            holder["P"] = Problem.from_layout(lay, eps=eps, k0=prob.k0, precision=precision, variant=variant)
        else:
            if not args.keep_factors:
                holder["P"].forget_factors()
            holder["P"].set_medium(eps, prob.k0)
        P = holder["P"]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        # all sources of the step, nrhs at a time (one block each)
        its, rrs, xs = [], [], []
        for c0 in range(0, nsources, args.nrhs):
            if args.recycle:
                b = P.rhs(prob.sources[c0:c0 + args.nrhs])
                # Block GCRO-DR for blocks of 2..16 sources, else one source after another
                x, it, rr, st = P.solve_recycle(b, k=args.recycle, restart=args.restart,
                                                block=args.krylov == "block" and 2 <= b.shape[0] <= 16)
            else:
                x, it, rr, st = P.solve(prob.sources[c0:c0 + args.nrhs], use_graph=int(args.graph),
                                        krylov=krylov, restart=args.restart)
            its.append(it)
            rrs.append(rr)
            if args.ports or args.e_error:
                xs.append(x)
        if args.ports:   # S-matrix of every port's field on every port (eq. (5))
            holder["S"] = P.smatrix(prob.sources, torch.cat(xs))
        if args.e_error:
            holder["X"], holder["eps"] = torch.cat(xs), eps
        it, rr = np.concatenate(its), np.concatenate(rrs)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        phases.append((t1 - t0, t2 - t1))
        log(f"[bench]   assemble+factor {t1-t0:.2f}s solve {t2-t1:.2f}s")
        return it, rr

    # first call also builds the layout's device copy (per-mesh, untimed)
    t0 = time.perf_counter()
    for w in range(args.warmup):
        it, rr = one_step()
        log(f"[bench] warmup {w}: iters={it.tolist()} relres={rr.tolist()} {time.perf_counter()-t0:.2f}s")
        t0 = time.perf_counter()

    tiles = None
    if args.tune:
        if "P" not in holder:
            one_step()  # untimed: creates and factors the problem
        tiles = holder["P"].tune(args.nrhs)
        log(f"[bench] tuned tiles {tiles}")

    timing(not args.no_kernel_timing)
    reset_timing()
    torch.cuda.synchronize()
    lat = []
    iters = []
    t_start = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        it, rr = one_step()
        lat.append(time.perf_counter() - ts)
        iters.append(int(np.max(it)))
        log(f"[bench] step {k}: {lat[-1]:.3f}s iters={it.tolist()} relres={[f'{v:.2e}' for v in rr]}")
        assert np.all(rr <= 1e-8), "solve did not reach the tolerance"
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    timing(False)

    kern = kernel_rooflines(info, precision, args.nrhs)
    dom = max(kern, key=lambda k: kern[k]["total_ms"]) if kern else None
    roof = None
    if dom:
        kd = kern[dom]
        roof = {"kernel": dom, "bound": kd["bound"], "achieved": kd["achieved"], "peak": kd["peak"],
                "unit": kd["unit"], "frac": kd["achieved"] / kd["peak"],
                "traffic": measured_traffic(dom, args.precision, args.nrhs, args.nsub)}
    ms_per_step = 1e3 * elapsed / args.steps
    value = nsources * args.steps / elapsed
    out = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if precision == B.MXW_FP64 else "f32+f64", "data": "synthetic",
        "config": {"workload": wl, "ndof": int(info.ndof), "nnz": int(info.nnz), "n_sub": int(info.n_sub),
                   "max_ns": int(info.max_ns), "nrhs": args.nrhs, "sources_per_step": nsources, "precision": args.precision,
                   "iterations": iters, "restart": args.restart, "tol": 1e-8, "variant": args.variant, "graph": bool(args.graph),
                   "krylov": (("block gcro-dr k=%d" if args.krylov == "block" and 2 <= args.nrhs <= 16 else
                               "gcro-dr k=%d") % args.recycle) if args.recycle else args.krylov,
                   "factorisation": "kept where the local data did not change" if args.keep_factors
                   else "every subdomain, every step",
                   "medium": "scaled by 1 + 0.01 i at step i" if args.sequence else "fixed"},
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "mesh_setup_s": t_mesh,
        "phase_s": {"assemble_factor": float(np.median([p[0] for p in phases[-args.steps:]])),
                    "solve": float(np.median([p[1] for p in phases[-args.steps:]]))},
        "roofline": roof,
        "kernels": kern,
        "tiles": tiles,
    }
    need64 = lay.footprint(B.MXW_FP64, args.nrhs, restart=args.restart, krylov=krylov) if args.e_error else 0
    total = torch.cuda.get_device_properties(0).total_memory
    if args.e_error and precision == B.MXW_MIXED and need64 > total:
        out["e_error_vs_fp64"] = {"skipped": f"FP64 factors and Krylov space need {need64 / 1e9:.1f} GB, above the "
                                             f"device's {total / 1e9:.1f} GB"}
        log(f"[bench] E-field check against FP64 factors skipped: {need64 / 1e9:.1f} GB needed")
    elif args.e_error and precision == B.MXW_MIXED:
        # the same sources with FP64 factors (untimed; the mixed problem is
        # released first so that both sets of factors never share the HBM)
        Xm = holder.pop("X")
        torch.cuda.synchronize()
        holder.pop("P").close()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        P64 = Problem.from_layout(lay, eps=holder["eps"], k0=prob.k0, precision=B.MXW_FP64)
        errs = []
        for c0 in range(0, nsources, args.nrhs):
            x64, _, _, _ = P64.solve(prob.sources[c0:c0 + args.nrhs], krylov=krylov, restart=args.restart)
            d = torch.linalg.vector_norm(Xm[c0:c0 + args.nrhs] - x64, dim=1)
            errs += (d / torch.linalg.vector_norm(x64, dim=1)).tolist()
        P64.close()
        out["e_error_vs_fp64"] = {"per_source": errs, "max": max(errs),
                                  "note": "relative l2 difference of E between FP32 and FP64 local factors, "
                                          "both solved to a true relative residual of 1e-8"}
        log(f"[bench] E-field difference mixed vs FP64 factors: max {max(errs):.2e}")
    if args.ports:
        S = holder["S"].cpu().numpy()
        out["smatrix"] = {"nports": args.ports, "max_abs": float(np.abs(S).max()),
                          "reciprocity": float(np.abs(S - S.T).max() / np.abs(S).max()),
                          "diag_mean": [float(np.mean(np.diag(S)).real), float(np.mean(np.diag(S)).imag)]}
    # the plain path (FP64 factors, one source at a time) on the same chamber,
    # if the run's time allows it (about 25 s)
    if "P" in holder:
        holder.pop("P").close()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    spent = time.perf_counter() - t_program
    if args.no_plain or precision == B.MXW_FP64 and args.nrhs == 1:
        out["plain_fp64_single_rhs"] = None
    elif spent + 40.0 < args.time_budget:
        log("[bench] timing the plain FP64 single-source path")
        plain = plain_fp64_rate(args, prob, lay)
        out["plain_fp64_single_rhs"] = plain
        out["speedup_vs_plain"] = value / plain["value"]
        log(f"[bench] plain FP64 single source: {plain['seconds_per_solve']:.2f} s per solve; "
            f"speedup {out['speedup_vs_plain']:.2f}x")
    else:
        out["plain_fp64_single_rhs"] = {"skipped": f"time budget: {spent:.0f} s spent of {args.time_budget:.0f} s"}
    if cpu_proc is not None:
        spent = time.perf_counter() - t_program
        log("[bench] collecting the oracle's timing (CPU)")
        cb = finish_cpu_baseline(cpu_proc, int(np.median(iters)), timeout=max(5.0, args.time_budget - spent))
        out["cpu_baseline"] = cb if cb is not None else {"skipped": "oracle timing did not finish in the time budget"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
