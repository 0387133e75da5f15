"""Benchmark: one RLOBPCG solve per step on one MI355X.

Workload (default): the complex null-space problem at 10^6 x 1000, k = 10
(complex128): A = U diag(sigma) V^H plus i.i.d. complex Gaussian noise of std
1e-14, sigma_1..sigma_990 log-spaced from 1 to 1e-4 and the last 10 zero,
sketch d = 3n = 3000 with 8 nonzeros per column, block b = k = 10.  A is drawn
on the device (torch RNG, Cholesky-QR2 for U) and is resident in HBM before
the timed region.  One step = one full solve (sketch, QR, preconditioner,
start block, LOBPCG to the stopping rule or max_iter, outputs).  Its pass
runs the products with A on the FP64 matrix cores with plain sums (see
the design doc for why the compensated sums are not the default there).  The other
workloads (--workload) are the real 10^6 x 200 (k = 1), 2*10^6 x 500 (k = 5)
and 4000 x 50 (k = 1) problems, with compensated (Dot2) products, and the
block-size study's 10^6 x 2000 clustered problem (k = 1, --block 1, 3, 5 or
10; plain sums on the matrix cores, the only pass past n = 1024).

The JSON line reports solves/s as ``value``; time-to-solution as
``ms_per_step``; the dominant kernel against its roofline (the Gram
contraction A^* [A_V A_X A_W] against the FP64 matrix-core peak for the
complex workload, the fused one-read pass against HBM for the real ones),
timed with HIP events around each launch on the solve's stream, plus the
whole pass against max(bytes / HBM peak, flops / FP64 peak); and the CPU
oracle timed on a row sample of the same input with all host cores and with
one thread, scaled to the full solve.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "time-to-solution & A-stream HBM GB/s at resid≤1e-12‖A‖; solves/s + p99 served"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6
DEFAULT_WORKLOAD = "tall-1e6x1000c-k10"
# products with A per workload: compensated (Dot2) sums, or plain sums (the
# complex null-space workload, whose pass then runs on the matrix cores)
DEFAULT_DOT2 = {"tall-1e6x1000c-k10": False, "clustered-1e6x2000-k1": False}

WORKLOADS = {
    # name: (m, n, k, d, zeta, complex, data seed, sketch seed, spectrum)
    "tall-1e6x200-k1": (1_000_000, 200, 1, 800, 8, False, 1002, 2002, ("gap", 1e-12, 10.0)),
    "tall-4000x50-k1": (4000, 50, 1, 200, 8, False, 1001, 2001, ("tail", 1e-3, 1e-6)),
    "tall-2e6x500-k5": (2_000_000, 500, 5, 2000, 8, False, 1004, 2004, ("gap", 1e-10, 100.0)),
    # complex nullspace: rank n-k plus complex Gaussian noise of std 1e-14
    "tall-1e6x1000c-k10": (1_000_000, 1000, 10, 3000, 8, True, 1003, 2003, ("null", 1e-4, 1e-14)),
    # the block-size study (Sec. 5.2): clustered spectrum, exponent 1/256, condition 1e10;
    # real n = 2000 runs plain sums on the matrix cores (the only pass past n = 1024)
    "clustered-1e6x2000-k1": (1_000_000, 2000, 1, 8000, 8, False, 1005, 2005, ("clustered", 1.0 / 256.0, 1e10)),
}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def spectrum(n, k, spec):
    from workloads import spectrum_clustered, spectrum_gap, spectrum_logspace_tail, spectrum_nullspace
    if spec[0] == "clustered":
        return spectrum_clustered(n, spec[1], spec[2])
    if spec[0] == "gap":
        return spectrum_gap(n, k, spec[1], spec[2])
    if spec[0] == "null":
        return spectrum_nullspace(n, k, spec[1])
    return spectrum_logspace_tail(n, spec[1], spec[2])


def astream_kernel(cplx: bool, n: int, b: int, dot2: bool = True) -> str:
    """The pass kernel(s) the library launches for this shape (the dispatch
    rule of launch_astream, for a dense A with 16-byte aligned rows)."""
    if cplx:
        if 256 < n <= 1024 and not dot2:
            return ("k_zm_aw + k_zm_g (A W, then after the Rayleigh-Ritz A^* A_{V_{i+1}}, both on the FP64 "
                    "matrix cores: two reads of A)")
        if 256 < n <= 1024:
            return "k_c2_rows + k_c2_cols (A W, then A^* [A_V A_X A_W]: two reads of A)"
        if n <= 1024:
            return "k_astream_ccs (A W and A^* [A_V A_X A_W] in one read of A)"
        return "k_astream<cd> (A W and A^* [A_V A_X A_W] in one read of A)"
    if 1024 < n <= 2048 and n % 2 == 0 and not dot2:
        return ("k_zm_aw + k_zm_g (A W, then after the Rayleigh-Ritz A^* A_{V_{i+1}}, both on the FP64 "
                "matrix cores: two reads of A)")
    if n % 2 == 0 and n <= 256 and b <= 2:
        return "k_astream_r2 (A W and A^* [A_V A_X A_W] in one read of A)"
    if n <= 1024 and b <= 10:
        return "k_astream_cs (A W and A^* [A_V A_X A_W] in one read of A)"
    return "k_astream<double> (A W and A^* [A_V A_X A_W] in one read of A)"


def measured_traffic(workload: str):
    """HBM bytes per A-stream launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a copy kernel of known size),
    or None when there is none for this workload or the kernel sources have
    changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"astream_traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\s*(\{.*?\})\s*```", open(path).read(), re.S)
    if not m:
        return None
    data = json.loads(m.group(1))
    h = hashlib.sha256()
    for f in data["sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != data["source_sha256"]:
        return None
    return int(data["traffic_bytes_per_launch"])


def _oracle_sample_times(A, k, seed, d, zeta, dot2, threads, extra=5):
    """Times of the oracle on the row sample A with the given thread count
    (BLAS and the compensated products): setup (sketch, SVD of S*A, start),
    the SVD of S*A alone, and one LOBPCG iteration (from runs of 1 and
    1 + extra iterations, after an untimed warm-up run)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import eft, rlobpcg, sparsestack
    eft.set_threads(threads)
    with threadpool_limits(limits=threads):
        rlobpcg(A, k, seed=seed, d=d, zeta=zeta, max_iter=0, rule="none", dot2=dot2, refresh=False)

        def run(iters):
            t0 = time.perf_counter()
            rlobpcg(A, k, seed=seed, d=d, zeta=zeta, max_iter=iters, rule="none", dot2=dot2, refresh=False)
            return time.perf_counter() - t0
        t_a = run(1)
        t_b = run(1 + extra)
        t_iter = max(t_b - t_a, 1e-9) / extra
        SA = sparsestack.sketch(A, d, zeta, seed)
        t0 = time.perf_counter()
        np.linalg.svd(SA, full_matrices=False)
        t_svd = time.perf_counter() - t0
    return max(t_a - t_iter, t_svd), t_svd, t_iter


def cpu_baseline(A_dev, k, seed, d, zeta, gpu_iters, dot2, sample_rows):
    """The oracle timed on this host on a bounded sample: its first
    sample_rows rows, run with all host cores and with one thread; every
    cost that grows with m (the sketch, the products with A, the tall
    Rayleigh-Ritz) is scaled by m / sample_rows, the SVD of the d x n sketch
    is counted once, and the iteration count is the GPU's."""
    m, n = A_dev.shape
    ms = int(min(m, max(sample_rows, d + 1, n + 1)))
    A = A_dev[:ms].cpu().numpy()
    f = m / ms
    cores = len(os.sched_getaffinity(0))
    res = {}
    for thr in (cores, 1):
        t_setup, t_svd, t_iter = _oracle_sample_times(A, k, seed, d, zeta, dot2, thr)
        t_solve = t_svd + (t_setup - t_svd) * f + gpu_iters * t_iter * f
        res[thr] = (t_solve, t_setup, t_svd, t_iter)
    del A
    tN, t1 = res[cores], res[1]
    return {
        "value": 1.0 / tN[0],
        "unit": "solves/s",
        "cores": cores,
        "kind": "oracle",
        "value_1thread": 1.0 / t1[0],
        "sample": (f"oracle (compensated products {'on' if dot2 else 'off'}, as the GPU run) on the first {ms} of "
                   f"{m} rows: setup and LOBPCG iterations timed (runs of 1 and 6 iterations after a warm-up), "
                   f"the m-proportional parts scaled by "
                   f"{f:.1f}, the SVD of the {d}x{n} sketch counted once, {gpu_iters} iterations as on the GPU; "
                   f"{cores} threads: setup {tN[1]:.2f} s (SVD {tN[2]:.2f} s), {tN[3]:.4f} s/iteration on the "
                   f"sample; 1 thread: setup {t1[1]:.2f} s (SVD {t1[2]:.2f} s), {t1[3]:.4f} s/iteration; the refresh "
                   f"pass (one more product) is not counted"),
    }


def served(args):
    """The served stream: 256 requests of different shapes, Poisson arrivals,
    continuous admission under an HBM budget (rl_server_*)."""
    import numpy as np
    import torch

    import paper_2602_16797_amd as rl
    from workloads import planted_torch, request_spectrum, served_requests

    reqs = served_requests(count=args.served_count)
    log(f"staging {len(reqs)} requests in HBM")
    staged = []
    t0 = time.perf_counter()
    for q in reqs:
        sig = request_spectrum(q)
        A, _, _ = planted_torch(q.m, q.n, sig, q.data_seed, device="cuda")
        if q.n % 2:  # even leading dimension keeps every row 16-byte aligned
            P = torch.zeros((q.m, q.n + 1), dtype=torch.float64, device="cuda")
            P[:, :q.n] = A
            A = P[:, :q.n]
        staged.append(A)
    torch.cuda.synchronize()
    gb = sum(q.m * q.n * 8 for q in reqs) / 1e9
    log(f"staged {gb:.1f} GB in {time.perf_counter() - t0:.1f} s")
    budget = int(args.served_budget_gb * (1 << 30))
    kw = dict(sketch_prec=args.sketch_prec, lock=args.lock)

    def run(srv, arrivals):
        tickets = []
        t_start = time.perf_counter()
        for q, A, at in zip(reqs, staged, arrivals):
            now = time.perf_counter() - t_start
            if at > now:
                time.sleep(at - now)
            tickets.append(srv.submit(A, q.k, seed=q.sketch_seed, want_u=True, **kw))
        res = [srv.wait(t) for t in tickets]
        return res, time.perf_counter() - t_start

    # sequential (one slot) and saturated (all submitted at once)
    with rl.Server(budget, max_inflight=1) as srv:
        seq, t_seq = run(srv, [0.0] * len(reqs))
    with rl.Server(budget, max_inflight=args.served_slots) as srv:
        sat, t_sat = run(srv, [0.0] * len(reqs))
    cap = len(reqs) / t_sat
    lam = 0.8 * cap
    # the stream's Poisson arrivals were drawn at 100/s; rescale them to rate lam
    arr = np.array([q.arrival_s for q in reqs]) * (100.0 / lam)
    with rl.Server(budget, max_inflight=args.served_slots) as srv:
        paced, t_paced = run(srv, list(arr))
    lat = np.array([r.latency_us for r in paced]) / 1e3
    # gates: residual of every served triplet (||A|| = 1 for the planted spectra)
    worst = 0.0
    statuses = {}
    for q, A, r in zip(reqs, staged, paced):
        statuses[r.status] = statuses.get(r.status, 0) + 1
        with torch.no_grad():
            R = A @ r.V - r.U * r.sigma[None, :]
            worst = max(worst, torch.linalg.norm(R, dim=0).max().item())
    same = all(torch.equal(a.sigma, b.sigma) and torch.equal(a.V, b.V) for a, b in zip(seq, paced))
    line = {
        "metric": "served solves/s with p50/p99 latency (continuous batching)",
        "value": round(len(reqs) / t_paced, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "served-256-poisson", "requests": len(reqs), "slots": args.served_slots,
                   "hbm_budget_gb": args.served_budget_gb, "sketch_prec": args.sketch_prec, "lock": args.lock,
                   "a_bytes_gb": round(gb, 2)},
        "lambda_per_s": round(lam, 3),
        "p50_ms": round(float(np.percentile(lat, 50)), 3),
        "p99_ms": round(float(np.percentile(lat, 99)), 3),
        "saturated_solves_per_s": round(cap, 3),
        "sequential_solves_per_s": round(len(reqs) / t_seq, 3),
        "statuses": {str(k): v for k, v in statuses.items()},
        "resid_max": worst,
        "resid_gate": 1e-12,
        "bitwise_same_as_sequential": same,
    }
    print(json.dumps(line), flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--block", type=int, default=0, help="block size b >= k (default k)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sketch-prec", default="f64", choices=["f64", "f32", "bf16"],
                    help="precision of the sketch and its QR (the rest stays FP64)")
    ap.add_argument("--dot2", default="auto", choices=["auto", "on", "off"],
                    help="compensated (Dot2) products with A; auto: off for the complex null-space workload "
                         "(its pass then runs on the matrix cores), on for the others")
    ap.add_argument("--no-dot2", action="store_true", help="same as --dot2 off")
    ap.add_argument("--cpu-sample-rows", type=int, default=0,
                    help="rows of A in the oracle's timed sample (default: about 15 s of oracle work)")
    ap.add_argument("--lock", action="store_true",
                    help="locking of converged columns (Sec. 2.3; off in the paper's runs): a column whose residual "
                         "meets the tolerance gets no more search directions, and the solve ends once all are locked")
    ap.add_argument("--orth", default="cgs2", choices=["cgs2", "svqb"],
                    help="Orth of the new search block after its block projections: CGS2 (the method) or SVQB")
    ap.add_argument("--loop-precond", default="sketch", choices=["sketch", "diag", "none"],
                    help="preconditioner of the LOBPCG loop: the sketch's (the method) or the diagonal / no "
                         "preconditioner of the paper's comparison methods (same sketch-and-solve start)")
    ap.add_argument("--vs-fp64", action="store_true",
                    help="after timing, solve once with the FP64 sketch and Dot2 products and report the "
                         "difference of the timed variant's sigma and subspace from it")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the solves, copy a 1.6 GB device buffer three times (a plain copy kernel of "
                         "known size, the reference for the HBM byte counters)")
    ap.add_argument("--served", action="store_true",
                    help="run the served stream (continuous batching) instead of the single-solve workload")
    ap.add_argument("--served-count", type=int, default=256)
    ap.add_argument("--served-slots", type=int, default=8)
    ap.add_argument("--served-budget-gb", type=float, default=16.0)
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(json.dumps({"error": "one process drives one GPU here; --gpus above 1 is not supported (the row-sharded multi-GPU path is a design, not code)",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.served:
        served(args)
        return

    import numpy as np
    import torch

    import paper_2602_16797_amd as rl
    from workloads import planted_torch

    m, n, k, d, zeta, cplx, dseed, sseed, spec = WORKLOADS[args.workload]
    if args.no_dot2:
        args.dot2 = "off"
    dot2 = DEFAULT_DOT2.get(args.workload, True) if args.dot2 == "auto" else args.dot2 == "on"
    sig = spectrum(n, k, spec)
    log(f"drawing {args.workload}: {m}x{n} on cuda:0")
    noise = spec[2] if spec[0] == "null" else 0.0
    t_draw = time.perf_counter()
    A, Vp, s = planted_torch(m, n, sig, dseed, device="cuda", is_complex=cplx, noise_std=noise)
    torch.cuda.synchronize()
    log(f"drew A in {time.perf_counter() - t_draw:.1f} s")
    es = 16 if cplx else 8
    kw = dict(seed=sseed, d=d, zeta=zeta, sketch_prec=args.sketch_prec, dot2=dot2,
              loop_precond=args.loop_precond, orth=args.orth, lock=args.lock)
    if args.block:
        kw["block"] = args.block

    for w in range(args.warmup):
        r = rl.rl_svds_smallest(A, k, **kw)
        torch.cuda.synchronize()
        log(f"warmup {w}: iters {r.iters} status {r.status} sigma {r.sigma.tolist()}")

    results = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        results.append(rl.rl_svds_smallest(A, k, profile=True, **kw))
        log(f"solve {i}: iters {results[-1].iters} status {results[-1].status}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    last = results[-1]
    log(f"timed {args.steps} solves: {ms_per_step:.3f} ms/solve; iters {last.iters}; "
        f"setup {last.t_setup_us / 1e3:.3f} ms, loop {last.t_iter_us / 1e3:.3f} ms")

    # gates on the last solve: residual and sigma against the planted value
    with torch.no_grad():
        Av = A @ last.V
        res = torch.linalg.norm(Av - last.U * last.sigma[None, :], dim=0).max().item()
    sig_err = float(np.max(np.abs(last.sigma.cpu().numpy() - np.sort(sig)[:k])))
    # with noise the planted values are not the singular values of A; the
    # noise moves the null space's sigma to about noise * sqrt(m)
    sig_tol = 1e-12 * sig[0] if not noise else 10.0 * noise * math.sqrt(m)
    gates = {"resid_max": res, "resid_gate": 1e-12 * float(sig[0]), "sigma_err_vs_planted": sig_err,
             "sigma_gate": sig_tol, "passed": bool(res <= 1e-12 * sig[0] and sig_err <= sig_tol)}
    if not noise:
        # the angle to the planted right singular vectors of the k smallest values
        with torch.no_grad():
            order = torch.from_numpy(np.argsort(sig)[:k].copy()).to(Vp.device)
            P = Vp[:, order]
            Qa, _ = torch.linalg.qr(last.V)
            gates["sin_angle_vs_planted"] = torch.linalg.matrix_norm(P - Qa @ (Qa.conj().T @ P), ord=2).item()
    log(f"gates: {gates}")
    if args.vs_fp64:
        ref = rl.rl_svds_smallest(A, k, seed=sseed, d=d, zeta=zeta)
        with torch.no_grad():
            Qa, _ = torch.linalg.qr(last.V)
            Qb, _ = torch.linalg.qr(ref.V)
            sin = torch.linalg.matrix_norm(Qb - Qa @ (Qa.conj().T @ Qb), ord=2).item()
        gates["vs_fp64_dot2"] = {"sin_angle": sin,
                                 "sigma_diff": float((last.sigma - ref.sigma).abs().max().item()),
                                 "fp64_iters": ref.iters}
        log(f"vs FP64 Dot2 solve: {gates['vs_fp64_dot2']}")

    # The A-stream pass, its kernels timed per launch with HIP events on the
    # solve's stream (the reduction of the per-workgroup partial sums is
    # excluded).  Algorithmic bytes of each launch: A once, W, the A_W write,
    # and the panel reads the fused form needs (A_V from the first loop pass
    # on, A_X from the second); the start pass reads neither.  b is the
    # solve's block size.
    n_as = sum(r.n_astream for r in results)
    t_as = sum(r.t_astream_us for r in results)
    avg_us = t_as / max(n_as, 1)
    bb = last.block
    base = m * n * es + m * bb * es + n * bb * es
    mv = m * bb * es
    tot_bytes = 0
    for r in results:
        it = r.n_astream - 1
        tot_bytes += (1 + it) * base + it * mv + max(it - 1, 0) * mv
    bytes_launch = tot_bytes / max(n_as, 1)
    # flops of the two products of an iteration in the paper's form (A W and
    # A^* A_V): 2 x 8 m n b real flops for complex data, 2 x 2 m n b for real
    cflop = 8 if cplx else 2
    pass_flops = 2 * cflop * m * n * bb
    bound_us = 1e6 * max(bytes_launch / (HBM_PEAK_GBS * 1e9), pass_flops / (FP64_PEAK_TFS * 1e12))
    pass_line = {"avg_launch_us": round(avg_us, 2), "algorithmic_bytes": round(bytes_launch),
                 "flops": pass_flops, "bound_us": round(bound_us, 2), "frac": round(bound_us / avg_us, 4),
                 "bound_rule": "max(bytes / 8 TB/s, flops / 78.6 TFLOP/s)"}
    n_g = sum(r.n_pass_g for r in results)
    traffic = (measured_traffic(args.workload)
               if (args.sketch_prec == "f64" and dot2 == DEFAULT_DOT2.get(args.workload, True)
                   and args.loop_precond == "sketch" and args.orth == "cgs2" and not args.block
                   and not args.lock) else None)
    if n_g > 0:
        # the second kernel of the two-read passes is the Gram contraction on
        # the matrix cores; in a solve it forms one m x b block per launch
        # (A^* A_W of the start pass, then the loop's late residual
        # A^* A_{V_{i+1}}): cflop m n b flops, A once plus that block
        t_g = sum(r.t_pass_g_us for r in results)
        g_us = t_g / n_g
        g_flops_launch = cflop * m * n * bb
        g_bytes_launch = m * n * es + m * bb * es
        common = {"kernel": "k_zm_g (A^* A_V on the FP64 matrix cores)", "avg_launch_us": round(g_us, 2),
                  "launches": n_g, "algorithmic_flops_per_launch": round(g_flops_launch),
                  "algorithmic_bytes_per_launch": round(g_bytes_launch),
                  "pass": astream_kernel(cplx, n, bb, dot2), "pass_roofline": pass_line}
        # the bound is whichever of the flops and the bytes takes longer at peak
        if g_flops_launch / (FP64_PEAK_TFS * 1e12) >= g_bytes_launch / (HBM_PEAK_GBS * 1e9):
            achieved = g_flops_launch / (g_us * 1e-6) / 1e12
            roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                        "frac": round(achieved / FP64_PEAK_TFS, 4), "traffic": traffic, **common}
        else:
            achieved = g_bytes_launch / (g_us * 1e-6) / 1e9
            roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, **common}
    else:
        achieved = bytes_launch / (avg_us * 1e-6) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "kernel": astream_kernel(cplx, n, bb, dot2), "avg_launch_us": round(avg_us, 2),
                    "launches": n_as, "algorithmic_bytes_per_launch": round(bytes_launch),
                    "pass_roofline": pass_line}

    if args.copy_calibration:
        src = torch.empty(200_000_000, dtype=torch.float64, device="cuda")
        src.fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 copies of 1.6e9 bytes")
        del src, dst

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        # about 15 s of oracle work on all cores: the products with A cost
        # about 50 (real) or 200 (complex) flops per element and vector
        rows = args.cpu_sample_rows or int(min(m, max(2 * d, 3e10 / (n * bb * (200 if cplx else 50)))))
        cpu = cpu_baseline(A, k, sseed, d, zeta, last.iters, dot2, rows)
        log(f"cpu baseline: {cpu}")

    line = {
        "metric": METRIC,
        "value": round(args.steps / elapsed, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128" if cplx else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "m": m, "n": n, "k": k, "block": last.block, "d": d, "zeta": zeta,
                   "spectrum": list(spec), "stop_rule": "paper", "dot2": dot2,
                   "sketch_prec": args.sketch_prec, "loop_precond": args.loop_precond, "orth": args.orth,
                   "lock": args.lock},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": {"iters": last.iters, "a_passes": last.a_passes, "matvecs": last.a_passes * last.block,
                   "status": last.status,
                   "t_setup_ms": round(last.t_setup_us / 1e3, 4), "t_loop_ms": round(last.t_iter_us / 1e3, 4),
                   "t_final_ms": round(last.t_final_us / 1e3, 4),
                   "a_stream_gbs_whole_solve": round(last.bytes_a / (ms_per_step * 1e-3) / 1e9, 1),
                   "gates": gates},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
