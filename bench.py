"""Benchmark: GenEO setup + PCG to a 1e-10 residual reduction on one MI355X.

A step is one pass of the whole path over one synthetic problem already
resident in HBM (the per-element coefficient field): device Q1 assembly of
the global and local matrices, the GenEO setup (local factors, shifted
factors, eigen sweeps, coarse basis, Galerkin product, coarse factor) and
the graph-captured PCG solve, then the release of the operator.

The headline workload is the largest single-GPU one: 3D Darcy on a 96^3 Q1
grid (912,673 dofs), 8^3 subdomains of 12^3 elements with one-element
overlap, z-layers of random thickness 2-6 alternating k = 1 and
k = 10^U(4,6), 12 eigenvectors per subdomain, FP32 local factors with FP64
eigen, coarse and PCG.  The same JSON line also carries, as nested objects,
the FP64 form of the same workload, the 512^2 Darcy workload, the
serendipity laminate (20-node bricks, 23,175 dofs) and the serving
stream's p50/p99 latency.

Prints one JSON line.  `--gpus N` with N > 1 exits: the library maps all
subdomains onto one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_MFMA_PEAK_TFLOPS = 157.3
GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")
# workloads reported as nested objects of the headline line
NESTED = ("grf_512", "laminate_s20_32x8x6")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="layers_96",
                    choices=["channels_64", "grf_512", "layers_96", "laminate_128x32x24",
                             "laminate_s20_32x8x6"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-form", action="store_true")
    ap.add_argument("--no-nested", action="store_true",
                    help="skip the nested workloads and the serving object")
    ap.add_argument("--cpu-budget-s", type=float, default=20.0)
    ap.add_argument("--opt", action="append", default=[], metavar="NAME=VALUE",
                    help="further setup option (geneo_opts_t field, integer or float)")
    ap.add_argument("--eig-tol", type=float, default=None,
                    help="eigen residual tolerance (default: the library's)")
    ap.add_argument("--serve", action="store_true",
                    help="only the serving benchmark: a seeded Poisson stream of new problems "
                         "and repeat solves through serve.Server; prints one JSON line with "
                         "p50/p99 latency")
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-budget-gb", type=float, default=200.0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (elementwise x*1): the "
                         "reference kernel for scaling HBM traffic counters")
    return ap.parse_args()


def log(msg):
    """Progress on stderr (the JSON line alone goes to stdout)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def copy_probe():
    """A plain elementwise copy of known size (reads and writes 1 GiB each)."""
    import torch
    n = 1 << 27
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe": {"read_bytes": 8 * n, "write_bytes": 8 * n,
                                     "launches": 3}}))


def make_problem(name, seed):
    import synth
    return synth.CONFIGS[name](seed=seed)


class Runner:
    """Holds the resident input and runs steps through the C ABI."""

    def __init__(self, prob, **extra):
        import torch
        from paper_1906_10944_amd import geneo as G
        self.G = G
        self.prob = prob
        self.extra = extra   # further setup options
        self.grid = G.grid_from_problem(prob)
        self.coeff = torch.as_tensor(prob.coeff, dtype=torch.float64).cuda().contiguous()
        self.xbuf = None
        self.last = None
        torch.cuda.synchronize()

    def step(self, precision):
        import torch
        G = self.G
        sysm = G.geneo_assemble_q1(self.grid, self.coeff)
        opts = G.opts_from_problem(self.prob, precision=precision, **self.extra)
        h = G.geneo_setup(sysm.csr(), sysm.subdomains(), sysm.neumann(), sysm.overlap(), opts)
        # the solution vector is the caller's: one buffer for all steps,
        # zeroed (x0 = 0) at the start of each
        if self.xbuf is None or self.xbuf.shape != sysm.b.shape:
            self.xbuf = torch.empty_like(sysm.b)
        x = self.xbuf
        x.zero_()
        info = G.pcg_solve(sysm.csr(), h, sysm.b, x, rtol=self.prob.rtol, maxit=self.prob.maxit)
        sinfo = G.geneo_get_setup_info(h)
        out = {"iters": info["iters"], "converged": info["converged"], "relres": info["relres"],
               "kappa_est": info["kappa_est"], "t_solve_ms": info["t_solve_ms"],
               "t_setup_ms": sinfo["t_setup_ms"], "nc": sinfo["nc"],
               "eig_sweeps": sinfo["eig_sweeps"], "fallback_fp64": sinfo["fallback_fp64"],
               "eig_stalled": sinfo["eig_stalled"], "eig_max_resid": sinfo["eig_max_resid"],
               "symv_tiles": sinfo["symv_tiles"], "eig_block": sinfo["eig_block"],
               "eig_solve": sinfo["eig_solve"], "eig_split": sinfo["eig_split"],
               "local_solve": sinfo["local_solve"], "eig_solve_split": sinfo["eig_solve_split"],
               "t_phase_ms": sinfo["t_phase_ms"]}
        self.last = (sysm, h, x)
        return out

    def true_residual(self):
        import torch
        sysm, h, x = self.last
        y = torch.empty_like(x)
        self.G.geneo_spmv(sysm.csr(), x, y)
        torch.cuda.synchronize()
        return float(torch.linalg.norm(sysm.b - y) / torch.linalg.norm(sysm.b))

    def solution(self):
        import torch
        torch.cuda.synchronize()
        return self.last[2].cpu().numpy()

    def release(self):
        if self.last is not None:
            self.last[1].close()
        self.last = None


def timed(runner, precision, steps, warmup):
    import torch
    for _ in range(warmup):
        runner.step(precision)
        runner.release()
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for k in range(steps):
        infos.append(runner.step(precision))
        if k + 1 < steps:
            runner.release()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) * 1e3 / steps, infos


def err_vs_oracle(prob, seed, x, iters):
    """Error of a device solution against the FP64 oracle's whole run of the
    same workload (stored by tests/golden/make_fullsize_golden.py, which
    calls only the oracle), or None where no stored run exists."""
    import numpy as np
    path = os.path.join(GOLDEN_DIR, "fullsize_%s_seed%d.npz" % (prob.name, seed))
    if not os.path.exists(path):
        return None
    g = np.load(path)
    xr, xo = g["x_ref"], g["x"]
    if xo.shape != x.shape:
        return None
    return {"rel_l2": float(np.linalg.norm(x - xr) / np.linalg.norm(xr)),
            "rel_max_abs": float(np.abs(x - xr).max() / np.abs(xr).max()),
            "rel_l2_vs_oracle_pcg": float(np.linalg.norm(x - xo) / np.linalg.norm(xo)),
            "reference": "the oracle's PCG solution refined twice with extended-precision "
                         "residuals (rel_l2_vs_oracle_pcg: against its plain PCG solution)",
            "iters": iters, "oracle_iters": int(g["iters"]),
            "oracle_kappa": float(g["kappa"]), "oracle_nc": int(g["nc"])}


def prof_query(G, name):
    import ctypes as C
    L = G.lib()
    L.geneo_prof_query.argtypes = [C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int),
                                   C.POINTER(C.c_double), C.POINTER(C.c_double)]
    t, n, by, fl = C.c_double(), C.c_int(), C.c_double(), C.c_double()
    rc = L.geneo_prof_query(name.encode(), C.byref(t), C.byref(n), C.byref(by), C.byref(fl))
    if rc:
        raise RuntimeError("geneo_prof_query failed")
    return {"ms": t.value, "launches": n.value, "bytes": by.value, "flops": fl.value}


PROF_KERNELS = ["densify_dirichlet", "chol_dirichlet_f32", "chol_dirichlet_f64",
                "trtri_dirichlet", "densify_shifted", "chol_shifted_f64", "trsm_bwd",
                "trsm_fwd", "trsm_bwd_split", "trsm_fwd_split", "bapply", "rayleigh_ritz",
                "orth", "coarse_chol", "lauum_dirichlet", "local_solve", "symv", "symv_cols",
                "cheb_combine"]


def kernel_profile(runner, precision):
    """One extra step with the library's event timing on (each timed launch
    has an event pair on the stream it runs on), plus eager applies (the PCG
    iterations themselves run inside a captured graph)."""
    import torch
    G = runner.G
    L = G.lib()
    L.geneo_prof_enable(1)
    runner.step(precision)
    sysm, h, x = runner.last
    r = torch.ones_like(x)
    z = torch.empty_like(x)
    for _ in range(10):
        G.geneo_apply(h, r, z)
    torch.cuda.synchronize()
    prof = {k: prof_query(G, k) for k in PROF_KERNELS}
    L.geneo_prof_enable(0)
    runner.release()
    return prof


# kernel symbol of each event-timed launch site (as rocprofv3 names it)
PROF_SYMBOL = {"densify_dirichlet": "k_densify_dirichlet", "chol_dirichlet_f32": "k_potrf_local_f32",
               "chol_dirichlet_f64": "k_potrf_local_f64", "trtri_dirichlet": "k_trtri_win<float, 2>",
               "lauum_dirichlet": "k_lauum<float>",
               "densify_shifted": "k_densify_shifted", "chol_shifted_f64": "k_potrf_shifted_f64",
               "bapply": "k_bapply", "rayleigh_ritz": "rayleigh-ritz kernels",
               "orth": "orthonormalisation kernels", "cheb_combine": "k_cheb",
               "coarse_chol": "tile-column step kernels", "local_solve": "k_local_solve_f32",
               "symv": "k_symv_rows", "symv_cols": "k_symv_cols"}
COMPUTE_BOUND = ("chol_dirichlet_f32", "chol_dirichlet_f64", "chol_shifted_f64", "trtri_dirichlet",
                 "lauum_dirichlet", "coarse_chol")


def prof_symbol(name, info):
    """The kernel a launch site ran, where it depends on the setup: the eigen
    block width picks the solve kernel, the number of FP64 refactors their
    factorisation."""
    if name in ("trsm_fwd", "trsm_bwd", "trsm_fwd_split", "trsm_bwd_split"):
        # the kernel the setup's tuning chose (1, 2: 8 wavefronts; 3, 4: 4;
        # 1, 3 two tile rows per wavefront, 2, 4 one), unsplit or on
        # 16-column blocks
        split = name.endswith("split")
        b = info.get("eig_block", 32)
        bwd = "true" if name.startswith("trsm_bwd") else "false"
        v = info.get("eig_solve_split" if split else "eig_solve", 1)
        if b > 48:
            return "k_trsm_bwd" if bwd == "true" else "k_trsm_fwd"
        ncq = 1 if split else b // 16
        nw = 8 if v in (1, 2) else 4
        if v in (2, 4) or (ncq, b) == (3, 48):
            ad, bp = {(1, 16): (2, "true"), (2, 32): (1, "true"), (3, 48): (1, "false"),
                      (1, 32): (2, "true"), (1, 48): (2, "true")}[(ncq, b)]
            return "k_trsm_w1<%d, %s, %d, %s, %d, %d>" % (ncq, bwd, ad, bp, b, nw)
        return "k_trsm_win<%d, %s, %d, %d>" % (ncq, bwd, b, nw)
    if name == "chol_dirichlet_f64" and 0 < info.get("fallback_fp64", 0) <= 32:
        return "tile-column step kernels"
    if name == "chol_shifted_f64" and info.get("nsub", 0) <= 32:
        return "tile-column step kernels"
    if name == "local_solve" and info.get("fallback_fp64", 0) >= info.get("nsub", 1):
        return "k_local_solve_f64"
    return PROF_SYMBOL.get(name, name)


APPLY_KERNELS = ("local_solve", "symv", "symv_cols")


def measured_traffic(symbol, workload):
    """HBM bytes per launch from the committed counter summary of this
    workload (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy), or None when
    there is none or the kernel sources have changed since the counters
    were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic_%s.json" % workload)
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    h = hashlib.sha256()
    for f in rec.get("sources", []):
        try:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        except OSError:
            return None
    if h.hexdigest() != rec.get("source_sha256"):
        return None
    k = rec.get("kernels", {}).get(symbol)
    if not k:
        return None
    return k["fetch_bytes"] + k["write_bytes"]


def roofline(prof, iters, info, workload):
    """The kernel with the largest time per step, against its bound.

    Per-step time: average launch time x launches per step.  The apply
    kernels run once per PCG iteration (inside the captured graph, where
    launches are not event-timed: their average comes from eager applies);
    the setup kernels run as often as in the profiled step."""
    per_step = {}
    for k, p in prof.items():
        if not p["launches"]:
            continue
        avg = p["ms"] / p["launches"]
        n = iters + 1 if k in APPLY_KERNELS else p["launches"]
        per_step[k] = avg * n
    cand = {k: v for k, v in per_step.items() if prof[k]["bytes"] > 0 or prof[k]["flops"] > 0}
    name = max(cand, key=cand.get)
    p = prof[name]
    avg_ms = p["ms"] / p["launches"]
    if name in COMPUTE_BOUND:
        peak = FP32_MFMA_PEAK_TFLOPS if name.endswith("f32") else FP64_PEAK_TFLOPS
        if name in ("trtri_dirichlet", "lauum_dirichlet") and info.get("fallback_fp64", 0) < info.get("nsub", 1):
            peak = FP32_MFMA_PEAK_TFLOPS
        achieved = p["flops"] / p["launches"] / (avg_ms * 1e-3) / 1e12
        rf = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s"}
    else:
        achieved = p["bytes"] / p["launches"] / (avg_ms * 1e-3) / 1e9
        rf = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    rf["frac"] = rf["achieved"] / rf["peak"]
    sym = prof_symbol(name, info)
    rf["traffic"] = measured_traffic(sym, workload)
    rf["kernel"] = sym
    rf["launches_per_step"] = p["launches"] if name not in APPLY_KERNELS else iters + 1
    rf["avg_launch_ms"] = avg_ms
    rf["algorithmic_bytes_per_launch"] = p["bytes"] / p["launches"]
    rf["algorithmic_flops_per_launch"] = p["flops"] / p["launches"]
    rf["per_step_ms_estimate"] = {k: round(v, 3) for k, v in sorted(per_step.items(),
                                                                      key=lambda kv: -kv[1])}
    return rf


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        n = [i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"]
        return max(n) if n else 1
    except Exception:
        return 1


def cpu_baseline(prob, gpu_iters, budget_s):
    """The oracle timed on a bounded SAMPLE of the same workload, extrapolated.

    Timed in full: global assembly and decomposition, one SpMV.  Timed on an
    evenly spaced sample of subdomains until the time budget is used: the
    whole per-subdomain setup step of the oracle (Dirichlet matrix and its
    Cholesky factor, Neumann/overlap matrices, the shift-and-invert
    eigensolve, basis) and one local solve.  The estimate scales the sample
    to all subdomains and to the GPU's iteration count; the coarse problem
    is left out, so it is a lower bound on a full oracle run."""
    import numpy as np
    import scipy.linalg as sla
    from oracle import decomp, fem, geneo
    t0 = time.perf_counter()
    A, b = fem.assemble(prob)
    subs, _ = decomp.build(prob)
    t_asm = time.perf_counter() - t0
    nev, tau, nev_max = prob.nev, prob.tau, prob.nev_max
    if tau is not None:
        nev = None
    setup_t, solve_t = [], []
    stride = max(1, len(subs) // 32)
    for j in range(0, len(subs), stride):
        s = subs[j]
        t1 = time.perf_counter()
        L, lam, mj, _, _ = geneo.local_setup(prob, A, s, nev, tau, nev_max, True, False, "auto")
        t2 = time.perf_counter()
        r = np.ones(L.shape[0])
        sla.cho_solve((L, True), r)
        t3 = time.perf_counter()
        setup_t.append(t2 - t1)
        solve_t.append(t3 - t2)
        if sum(setup_t) + sum(solve_t) > budget_s:
            break
    x = np.ones(prob.ndof)
    t4 = time.perf_counter()
    for _ in range(3):
        A @ x
    t_spmv = (time.perf_counter() - t4) / 3
    nsub = len(subs)
    est = (t_asm + nsub * float(np.mean(setup_t))
           + gpu_iters * (t_spmv + nsub * float(np.mean(solve_t))))
    return {"value": prob.ndof / est, "unit": "DOF/s", "cores": blas_threads(), "kind": "oracle",
            "sample": "SAMPLE, not a full run: global assembly, decomposition and one SpMV "
                      "timed in full; the oracle's per-subdomain setup step and one local "
                      "solve timed on %d of %d subdomains (%.2f s setup each); extrapolated "
                      "to %d subdomains and %d PCG iterations; coarse problem not counted" %
                      (len(setup_t), nsub, float(np.mean(setup_t)), nsub, gpu_iters),
            "sample_cpu_s": t_asm + sum(setup_t) + sum(solve_t) + 3 * t_spmv,
            "est_total_s": est}


def serve_bench(requests, slots, budget_gb, seed):
    """p50/p99 latency of the serving loop on a seeded stream (2D Darcy of
    128^2..1024^2 and 3D layered 48^3..96^3 new problems, repeat solves with
    8 random right-hand sides).  The arrival rate is 0.8 x the single-slot
    capacity measured first on a closed-loop prefix of the same stream."""
    from paper_1906_10944_amd import serve as S
    budget = int(budget_gb * (1 << 30))
    probe = S.make_stream(seed=seed, count=8, rate=1e9)
    srv = S.Server(budget, slots=1)
    t0 = time.perf_counter()
    srv.run(probe)
    mean_service = (time.perf_counter() - t0) / len(probe)
    srv.close()
    rate = 0.8 / mean_service
    reqs = S.make_stream(seed=seed, count=requests, rate=rate)
    srv = S.Server(budget, slots=slots)
    st = srv.run(reqs)
    srv.close()
    kinds = {}
    for r in reqs:
        kinds[r.kind] = kinds.get(r.kind, 0) + 1
    return {"metric": "GenEO serving latency (setup+solve or repeat solve per request)",
            "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "unit": "ms",
            "requests": st["requests"], "errors": st["errors"], "kinds": kinds,
            "arrival_rate_per_s": rate, "single_slot_mean_service_ms": mean_service * 1e3,
            "solves_per_s": st["solves_per_s"], "dof_per_s": st["dof_per_s"],
            "slots": slots, "peak_bytes": st["peak_bytes"], "budget_bytes": budget,
            "workload": "serving stream (2D GRF 128^2-1024^2, 3D layers 48^3-96^3, repeats "
                        "with 8 right-hand sides), seed %d" % seed}


def setup_options(args):
    extra = {"eig_tol": args.eig_tol} if args.eig_tol else {}
    for kv in args.opt:
        k, v = kv.split("=", 1)
        extra[k] = float(v) if any(c in v for c in ".eE") else int(v)
    return extra


def workload_line(prob, args, steps, warmup, full):
    """Timed steps of one workload (mixed form, the bench's options), with
    the FP64 form, the error against the oracle's stored run and, if `full`,
    the per-kernel roofline."""
    runner = Runner(prob, **setup_options(args))
    mixed = 1 if prob.precision == "mixed" else 0
    log("%s: %d warmup + %d timed steps" % (prob.name, warmup, steps))
    ms, infos = timed(runner, mixed, steps, warmup)
    log("%s: %.1f ms/step" % (prob.name, ms))
    tres = runner.true_residual()
    last = infos[-1]
    err = err_vs_oracle(prob, args.seed, runner.solution(), last["iters"])
    runner.release()
    out = {
        "value": prob.ndof / (ms * 1e-3), "unit": "DOF/s", "ms_per_step": ms,
        "steps": steps, "warmup": warmup,
        "config": {"workload": prob.name, "ndof": prob.ndof, "nsub": prob.nsub,
                   "form": "mixed" if mixed else "fp64", "rtol": prob.rtol, "seed": args.seed},
        "iters": last["iters"], "converged": bool(last["converged"]),
        "relres": last["relres"], "true_relres": tres, "kappa_est": last["kappa_est"],
        "err_vs_oracle": err,
        "nc": last["nc"], "eig_sweeps": last["eig_sweeps"], "eig_stalled": last["eig_stalled"],
        "eig_max_resid": last["eig_max_resid"], "eig_block": last["eig_block"],
        "symv_tiles": last["symv_tiles"], "eig_solve": last["eig_solve"],
        "eig_split": last["eig_split"], "fallback_fp64": last["fallback_fp64"],
        "local_solve": {1: "triangular", 2: "inverse"}.get(last["local_solve"], "?"),
        "eig_solve_split": last["eig_solve_split"],
        "setup_ms": last["t_setup_ms"], "solve_ms": last["t_solve_ms"],
        "setup_phase_ms": last["t_phase_ms"][:6],
    }
    if mixed and not args.no_fp64_form:
        ms64, inf64 = timed(runner, 0, 1, 1)
        log("%s: FP64 form %.1f ms/step" % (prob.name, ms64))
        tres64 = runner.true_residual()
        err64 = err_vs_oracle(prob, args.seed, runner.solution(), inf64[-1]["iters"])
        runner.release()
        out["fp64_form"] = {"ms_per_step": ms64, "value": prob.ndof / (ms64 * 1e-3),
                            "iters": inf64[-1]["iters"], "setup_ms": inf64[-1]["t_setup_ms"],
                            "solve_ms": inf64[-1]["t_solve_ms"], "true_relres": tres64,
                            "relres": inf64[-1]["relres"], "err_vs_oracle": err64}
        out["speedup_vs_fp64_form"] = ms64 / ms
    if full:
        prof = kernel_profile(runner, mixed)
        log("%s: per-kernel profile step done" % prob.name)
        last["nsub"] = prob.nsub
        out["roofline"] = roofline(prof, last["iters"], last, prob.name)
        out["kernels_ms"] = {k: round(v["ms"], 3) for k, v in prof.items() if v["launches"]}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library maps all subdomains onto one GPU; --gpus %d "
                          "is not supported" % args.gpus}))
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return
    if args.serve:
        out = serve_bench(args.serve_requests, args.serve_slots, args.serve_budget_gb, args.seed)
        out.update({"higher_is_better": False, "n_gpus": 1, "data": "synthetic"})
        print(json.dumps(out))
        return
    import torch  # noqa: F401  (before the library: one HIP runtime in the process)
    from paper_1906_10944_amd import geneo as G
    G.lib()
    prob = make_problem(args.config, args.seed)
    head = workload_line(prob, args, args.steps, args.warmup, True)
    mixed = head["config"]["form"] == "mixed"
    out = {
        "metric": "GenEO setup+PCG DOF/s to 1e-10 residual reduction (one GPU)",
        "value": head.pop("value"), "unit": head.pop("unit"),
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head.pop("ms_per_step"),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 local factors + f64" if mixed else "f64",
        "data": "synthetic",
    }
    head.pop("steps")
    head.pop("warmup")
    out.update(head)
    for name in ([] if args.no_nested else NESTED):
        if name != args.config:
            p2 = make_problem(name, args.seed)
            out[name] = workload_line(p2, args, max(1, min(args.steps, 10)), 2, False)
    if not args.no_cpu_baseline:
        log("oracle baseline on a sample of %s" % prob.name)
        out["cpu_baseline"] = cpu_baseline(prob, out["iters"], args.cpu_budget_s)
    if not args.no_nested:
        log("serving stream, %d requests" % args.serve_requests)
        out["serving"] = serve_bench(args.serve_requests, args.serve_slots,
                                     args.serve_budget_gb, args.seed)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
