"""Benchmark: time-to-solve (setup + PCG to relative residual 1e-8) and
preconditioner applies/s of the two-level Schwarz preconditioner on one
MI355X, mixed precision (FP32 local / FP64 outer and coarse) against plain
FP64 on the same GPU.

Workload (default): 2D high-contrast finite-volume diffusion on a 1024x1024
grid (n = 1,048,576), coefficient log-uniform in [1, 1e6] plus 20 channels at
1e6, 256 subdomains from randomised recursive coordinate bisection (cut ratio
uniform in [0.3, 0.7]), overlap 2, 16 coarse vectors per subdomain, b ~ N(0,1),
all seeded and synthetic. A step is one pass of the whole hot path: setup
(overlap, local matrices, batched factorization, coarse basis, A_0 and its
factor, and for SPD matrices the explicit inverses of the local matrices and
of A_0) plus the PCG solve. Inputs are resident in HBM before timing starts.
Other configurations (--config 1..5), the RAS + deflated composition
(--composition 1, FGMRES) and local solves by substitution
(--local-inverse 0) are options.

Prints ONE JSON line. Usage: python bench.py [--steps K] [--warmup W] [--gpus 1]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "time-to-solve (rel res 1e-8) + precond applies/s: mixed/batched vs plain FP64"
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}
# HBM bytes per launch of the dominant kernel (the forward substitution on
# the default workload) from two rocprofv3 counter runs (FETCH_SIZE, then
# WRITE_SIZE, KiB per dispatch), scaled by what the same counters read for a
# 1 GiB read + 1 GiB write elementwise copy (--copy-probe). Keyed by the
# block rows per substitution task, i.e. by the kernel the autotuner picked
# (1 -> k_trsv, 2..4 -> k_trsv_sr<float, FWD_L, rows>); None for a kernel
# without counters, and whenever that kernel has changed since they were
# taken.
TRAFFIC = {3: 1759144898, 2: 1763033267}
# The same for k_symv<float, 8> (explicit local inverses, taken on cfg2 when
# they were its default) and for the SpMV k_spmv<1280>.
TRAFFIC_SYMV = 16347116314
TRAFFIC_SPMV = 86755960


SOLVE_ROWS = 0  # --solve-rows


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def local_lower_bytes(info, w):
    """Algorithmic bytes of ONE triangular-solve launch (forward or
    backward) over all subdomains: the lower triangle of each local factor,
    m_i (m_i + 1) / 2 words of w bytes, read once:
    w * (sum m^2 + sum m) / 2. The vector traffic (2 m_i words) is left out."""
    return float(w) * (float(info["local_sum_m2"]) + float(info["local_sum_m"])) / 2.0


WORKLOADS = {
    1: "2D 5-point Poisson 64x64, 16 boxes, overlap 1, nev 8",
    2: "2D high-contrast FV diffusion 1024x1024, 256 RCB parts, overlap 2, nev 16",
    3: "3D lognormal FV diffusion 128^3, 1024 RCB parts, overlap 1, nev 12",
    4: "3D layered Q1 elasticity 48^3 nodes, 512 boxes, overlap 1, nev 20",
    5: "2D upwind convection-diffusion 1024x1024, 256 boxes, overlap 2, nev 16 (Section 6 basis, LU)",
    6: "2D Stokes lid-driven cavity, MAC 694x694 cells (1,443,520 unknowns, saddle point), 256 boxes, overlap 6, "
       "nev 16 (Section 6 basis, LU)",
}


def workload_name(cfg, prob, scale, composition, restart):
    base = WORKLOADS[cfg] if scale is None else f"{WORKLOADS[cfg]} shrunk to side {scale} ({prob.n_parts} parts)"
    if composition == 1:
        krylov = f"RAS + deflated coarse correction, FGMRES({restart})"
    else:
        krylov = "additive, " + ("PCG" if prob.spd else f"FGMRES({restart})")
    return f"cfg{cfg}: {base}; {krylov} to 1e-8"


def factor_flops(ctx, n_parts, spd=True):
    """Algorithmic flops of the batched factorization over the overlapping
    subdomain sizes m_i = #Omega_i (from the library's export): Cholesky
    sum_i m_i^3 / 3, LU sum_i 2 m_i^3 / 3."""
    import paper_2401_03915_amd as tls
    sp = np.zeros(n_parts + 1, dtype=np.int32)
    tls.tls_export(ctx, sub_ptr=sp)
    m = np.diff(sp).astype(np.float64)
    return float((m ** 3).sum() / 3.0) * (1.0 if spd else 2.0)


def run_mode(prob, dev_in, precision, steps, warmup, n_applies, use_graph, tune_cache, composition=0, restart=30,
             local_inverse=0, tol=1e-8, local_refine=0):
    import torch

    import paper_2401_03915_amd as tls
    rp, ci, val, part, b = dev_in
    A = prob.A
    n, nnz = A.shape[0], A.nnz
    stream = torch.cuda.current_stream()

    def make_opt(profile=0):
        opt = tls.tls_default_options()
        opt.precision = precision
        opt.matrix_kind = 0 if prob.spd else 1
        opt.composition = composition
        opt.restart = restart
        opt.local_inverse = local_inverse
        opt.local_refine = local_refine
        opt.solve_rows = SOLVE_ROWS
        opt.use_graph = use_graph
        opt.profile = profile
        # the first setup times the solve launch shapes and records the pick in
        # the cache; every later setup reads it back without timing
        opt.autotune = 1
        opt.tune_cache = tune_cache.encode()
        opt.stream = stream.cuda_stream or None
        return opt

    def step(opt):
        ctx = tls.tls_setup(n, nnz, rp.data_ptr(), ci.data_ptr(), val.data_ptr(), part.data_ptr(), prob.n_parts,
                            prob.overlap, prob.nev, opt)
        x = torch.empty_like(b)
        st, it, rr = tls.tls_solve(ctx, b.data_ptr(), x.data_ptr(), tol)
        return ctx, x, st, it, rr

    for w in range(max(warmup, 1)):
        log(f"precision {precision}: warmup {w}")
        ctx, x, st, it, rr = step(make_opt())
        tls.tls_destroy(ctx)
    torch.cuda.synchronize()
    # each step frees the previous step's preconditioner before building its
    # own (as an application replacing it would); holding several of them at
    # once would make later steps map fresh device memory
    prev = None
    t0 = time.perf_counter()
    for k in range(steps):
        if prev is not None:
            tls.tls_destroy(prev)
        ctx, x, st, it, rr = step(make_opt())
        prev = ctx
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / steps
    info = tls.tls_info(ctx)
    fflops = factor_flops(ctx, prob.n_parts, prob.spd)
    log(f"precision {precision}: {ms_per_step:.1f} ms/step, {it} iterations, relres {rr:.2e}, status {st}")
    # applies/s on the last context (plain launches, events on the stream)
    r = torch.randn(n, dtype=torch.float64, device=b.device, generator=torch.Generator(device=b.device).manual_seed(7))
    z = torch.empty_like(r)
    for _ in range(3):
        tls.tls_apply(ctx, r.data_ptr(), z.data_ptr())
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(n_applies):
        tls.tls_apply(ctx, r.data_ptr(), z.data_ptr())
    e1.record(stream)
    torch.cuda.synchronize()
    apply_ms = e0.elapsed_time(e1) / n_applies
    tls.tls_destroy(ctx)
    # kernel-level timing of the local triangular solves (HIP events inside the library)
    ctxp = tls.tls_setup(n, nnz, rp.data_ptr(), ci.data_ptr(), val.data_ptr(), part.data_ptr(), prob.n_parts,
                         prob.overlap, prob.nev, make_opt(profile=1))
    for _ in range(n_applies):
        tls.tls_apply(ctxp, r.data_ptr(), z.data_ptr())
    torch.cuda.synchronize()
    pinfo = tls.tls_info(ctxp)
    tls.tls_destroy(ctxp)
    return {
        "ms_per_step": ms_per_step,
        "iters": it,
        "relres": rr,
        "status": st,
        "apply_ms": apply_ms,
        "applies_per_s": 1e3 / apply_ms,
        "local_solve_ms": pinfo["t_local_solve_ms"],
        "local_fwd_ms": pinfo["t_local_fwd_ms"],
        "n_profiled": pinfo["n_profiled"],
        "solve_wgs": pinfo["solve_wgs"],
        "solve_order": pinfo["solve_order"],
        "solve_order_bwd": pinfo["solve_order_bwd"],
        "solve_rows": pinfo["solve_rows"],
        "tuned": pinfo["tuned"],
        "apply_ms_profiled": pinfo["t_apply_ms"],
        "info": info,
        "factor_flops": fflops,
        "z": z,
    }


GOLDEN = os.path.join(ROOT, "tests", "golden", "oracle_fullsize.json")


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(prob, cfg, composition=0, contexts=(), sample_iters=30):
    """The FP64 oracle (oracle.pool: its per-subdomain work in one worker
    process per host core, at most 16) on the same workload, and the apply
    parity of the timed GPU contexts against it.

    Timed: the oracle's full setup (overlap layers, A_ii, sparse LU, the
    eq. gevpsvd / Section 6 coarse blocks of every subdomain, A_00 and its
    factor) and `sample_iters` iterations of its own Krylov solve; the
    solve time is scaled to the oracle's own iteration count on this
    workload, read from tests/golden/oracle_fullsize.json (written by the
    oracle alone), or to the measured count when the sample converges.

    Then, for each (name, Preconditioner) in `contexts`: the library's own
    coarse basis is imported into the oracle and the relative apply error
    ||z_gpu - z_oracle|| / ||z_oracle|| is measured over three seeded r."""
    import torch

    from oracle import pool
    t0 = time.perf_counter()
    pl = pool.Pool(prob.A, prob.part, prob.overlap, prob.nev, spd=prob.spd)
    t_setup = time.perf_counter() - t0
    nc_oracle = pl.n_coarse
    comp = "ras_deflated" if composition == 1 else "additive"
    t0 = time.perf_counter()
    _, it_s, rr_s = pl.solve(prob.b, 1e-8, maxit=sample_iters, composition=comp)
    t_it = (time.perf_counter() - t0) / max(it_s, 1)
    gold = None
    if os.path.exists(GOLDEN) and prob.A.shape[0] == json.load(open(GOLDEN))["configs"].get(str(cfg), {}).get("n"):
        gold = json.load(open(GOLDEN))["configs"][str(cfg)]
    if rr_s <= 1e-8:
        its, src = it_s, "converged within the sample"
    elif gold is not None:
        its, src = gold["iterations"], "the oracle's own full run (tests/golden/oracle_fullsize.json)"
    else:
        its, src = None, "unknown"
    errors = {}
    for name, pc in contexts:
        pl.with_basis(pc.z_sparse())
        worst = 0.0
        for sd in (101, 102, 103):
            r = np.random.default_rng(sd).standard_normal(prob.A.shape[0])
            z = pc.apply(torch.as_tensor(r, device=pc.device))
            torch.cuda.synchronize()
            z_ref = pl.apply(r, comp)
            worst = max(worst, float(np.linalg.norm(z.cpu().numpy() - z_ref) / np.linalg.norm(z_ref)))
        errors[name] = worst
    workers = pl.workers
    pl.close()
    value = round(t_setup + t_it * its, 2) if its is not None else None
    return {
        "value": value,
        "unit": "s",
        "cores": workers,
        "kind": "oracle",
        "cpu": cpu_model(),
        "sample": (f"full oracle setup of all {prob.n_parts} subdomains (coarse space n_C = {nc_oracle}) on "
                   f"{workers} worker processes: {t_setup:.1f} s; {it_s} of its Krylov iterations: "
                   f"{t_it * 1e3:.0f} ms each, scaled to {its} iterations ({src})"),
        "oracle_iters": its,
    }, errors


WEAK_TAU2 = 0.41  # eq. gevpsvd threshold on lambda^2 (about 12 vectors per part at N = 2)
WEAK_CAP = 40
WEAK_TAU_SVD = 0.83  # Section 6 variant on the same matrices: sigma > tau (about 12 per part at N = 2)
WEAK_SVD_MAX_N = 512


def weak_scaling(N, steps, warmup, local_inverse):
    """Single-GPU analog of the weak-scaling study of Section 7 (Table
    diffusion-3d), one subdomain count N: the constant-coefficient 3D
    Poisson problem with about 15k unknowns per subdomain, the grid growing
    with N, delta = 1, rtol 1e-10, mixed precision. Returns the two-level
    iterations (threshold selection), the one-level iterations, n_C, GC, OC
    and the time to solve (set-up + PCG, inputs resident in HBM)."""
    import torch

    import paper_2401_03915_amd as tls
    from workloads import weak_scaling_poisson_3d
    dev = torch.device("cuda:0")
    log(f"weak scaling: N={N}")
    p = weak_scaling_poisson_3d(N)
    b = torch.as_tensor(p.b, device=dev)

    def run(nev, **kw):
        li = kw.pop("local_inverse", local_inverse)
        pc = tls.Preconditioner(p.A, p.part, p.overlap, nev, precision=1, local_inverse=li, **kw)
        x, it, rr, st = pc.solve(b, 1e-10)
        torch.cuda.synchronize()
        inf = pc.info()
        pc.close()
        log(f"  setup {inf['t_setup'][7]:.1f} ms (factor {inf['t_setup'][2]:.1f}, basis {inf['t_setup'][3]:.1f}), "
            f"solve {inf['t_solve']:.1f} ms, {it} its")
        return it, rr, st, inf

    tau = float(np.sqrt(WEAK_TAU2))
    for _ in range(warmup):
        run(WEAK_CAP, tau=tau)
    t0 = time.perf_counter()
    for _ in range(steps):
        it, rr, st, inf = run(WEAK_CAP, tau=tau)
    t = (time.perf_counter() - t0) / steps
    it1, rr1, st1, _ = run(0)
    log(f"  two-level {it} its (n_C {inf['n_coarse']}, GC {inf['gc']:.4f}) in {t:.2f} s; one-level {it1}")
    svd = None
    if N <= WEAK_SVD_MAX_N:
        t0 = time.perf_counter()
        try:
            its, rrs, sts, infs = run(WEAK_CAP, tau=WEAK_TAU_SVD, matrix_kind=1, local_inverse=0)
        except tls.TlsError as ex:
            if ex.status != tls._lib.TLS_E_NOMEM:
                raise
            svd = {"error": str(ex)}
            log(f"  Section 6 variant does not fit: {ex}")
        else:
            svd = {"iters": its, "status": sts, "n_coarse": infs["n_coarse"], "gc": round(infs["gc"], 4),
                   "oc": round(infs["oc"], 4), "time_to_solve_s": round(time.perf_counter() - t0, 3)}
            log(f"  Section 6 variant (LU, FGMRES(30)): {its} its (n_C {infs['n_coarse']})")
    ts = inf["t_setup"]
    return {"N": N, "n": int(p.A.shape[0]), "grid": list(p.meta["grid"]), "iters": it, "status": st,
            "relres": float(f"{rr:.3e}"), "n_coarse": inf["n_coarse"], "gc": round(inf["gc"], 4),
            "oc": round(inf["oc"], 4), "time_to_solve_s": round(t, 3), "setup_ms": round(ts[7], 1),
            "setup_split_ms": {"overlap": round(ts[0], 1), "gather": round(ts[1], 1), "factor": round(ts[2], 1),
                               "basis": round(ts[3], 1), "coarse": round(ts[5], 1),
                               "inverse": round(inf["t_inverse_ms"], 1)},
            "solve_ms": round(inf["t_solve"], 1), "one_level_iters": it1, "one_level_status": st1,
            "section6_variant": svd}


def weak_summary(rows, steps, warmup, local_inverse):
    t_last = rows[-1]["time_to_solve_s"]
    return {
        "metric": "weak scaling, 3D Poisson with ~15k unknowns per subdomain (rel res 1e-10): time-to-solve at the "
                  "largest N; two-level and one-level PCG iterations per N",
        "value": t_last, "unit": "s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": round(t_last * 1e3, 1), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 local / f64 outer", "data": "synthetic",
        "config": {"workload": f"3D Poisson weak scaling, N = {rows[0]['N']}..{rows[-1]['N']}, delta 1, "
                               f"tau^2 {WEAK_TAU2} (at most {WEAK_CAP} per part); Section 6 variant with sigma > "
                               f"{WEAK_TAU_SVD} up to N = {WEAK_SVD_MAX_N}",
                   "local_solves": "explicit inverse" if local_inverse else "substitution"},
        "table": rows,
    }


def decay_study():
    """Section 7, Fig. 1 at N = 256: the leading values of eq. gevpsvd
    (lambda, for a 3D lognormal diffusion of 80^3 cells in 256 RCB parts)
    and of the Section 6 variant (sigma, for the MAC Stokes cavity of
    config 6, 256 boxes) for delta = 1, 3, 5, each normalized by the
    subdomain's first value, for the subdomains 0, 64, 128 and 192 (the
    paper plots subdomains 1, 65, 129 and 193, counted from 1). At most 40
    values per subdomain are computed (the first 200 in the paper)."""
    import torch

    import paper_2401_03915_amd as tls
    from workloads import fv_diffusion_3d, lognormal_kappa_3d, make_config, rcb_partition
    rng = np.random.default_rng(0)
    A3 = fv_diffusion_3d(lognormal_kappa_3d(80, rng))
    part3 = rcb_partition((80, 80, 80), 8, rng, (0.45, 0.55))
    st = make_config(6)
    picks = (0, 64, 128, 192)
    out = {}
    for name, A, part, kind in (("diffusion_3d", A3, part3, 0), ("stokes_2d", st.A, st.part, 1)):
        out[name] = {}
        for delta in (1, 3, 5):
            log(f"decay study: {name}, delta {delta}")
            t0 = time.perf_counter()
            pc = tls.Preconditioner(A, part, delta, 40, precision=1, matrix_kind=kind)
            ex = pc.export()
            torch.cuda.synchronize()
            pc.close()
            zc, ev = ex["zcol_ptr"], ex["eigvals"]
            curves = {}
            for i in picks:
                v = np.asarray(ev[zc[i]:zc[i + 1]], dtype=np.float64)
                v = np.sqrt(v) if kind == 0 else v  # lambda from lambda^2; sigma as is
                curves[str(i)] = [float(f"{x:.4e}") for x in v / v[0]] if v.size else []
            allv = [np.asarray(ev[zc[i]:zc[i + 1]]) for i in range(len(zc) - 1)]
            norm = [np.sqrt(v / v[0]) if kind == 0 else v / v[0] for v in allv if v.size]
            out[name][f"delta{delta}"] = {
                "curves": curves,
                "median_at": {str(j + 1): round(float(np.median([v[j] for v in norm if v.size > j])), 4)
                              for j in (4, 9, 19, 39)},
                "setup_s": round(time.perf_counter() - t0, 2)}
    return {"metric": "decay of the eq. gevpsvd eigenvalues and Section 6 singular values vs overlap (Fig. 1 analog, "
                      "N = 256)", "value": None, "unit": None, "n_gpus": 1, "data": "synthetic",
            "config": {"workload": "3D lognormal FV diffusion 80^3, 256 RCB parts; MAC Stokes cavity 694^2, 256 "
                                   "boxes; delta 1, 3, 5; first 40 values"}, "decay": out}


def warm_start_study(steps, warmup, precision):
    """The learned warm start on config 4 (layered Q1 elasticity, 48^3 nodes,
    512 boxes, overlap 1, nev 20) against the random start, each setup with
    the benchmark's settings: the coarse-basis phase of the set-up (its
    eigensolves and orthonormalization, and the network's inference when the
    network is used), the subspace iterations, the eigen-residuals, the
    whole set-up and the final PCG iterations. Times are medians over
    `steps` setups after `warmup`."""
    import torch

    import paper_2401_03915_amd as tls
    from paper_2401_03915_amd.gnn_train import TRAINED, load_weights
    from workloads import make_config
    w, c_out = load_weights(TRAINED)
    p = make_config(4)
    b = torch.as_tensor(p.b, device="cuda:0")
    rows = {}
    for name, kw in (("random_start", {}), ("learned_warm_start", {"gnn_weights": w})):
        basis, infer, setup = [], [], []
        for k in range(warmup + steps):
            log(f"warm start study: {name} {k}")
            pc = tls.Preconditioner(p.A, p.part, p.overlap, p.nev, precision=precision, local_inverse=1,
                                    use_graph=1, **kw)
            inf = pc.info()
            if k >= warmup:
                basis.append(inf["t_setup"][3])
                infer.append(inf["t_setup"][4])
                setup.append(inf["t_setup"][7])
            if k == warmup + steps - 1:
                _, it, rr, st = pc.solve(b, 1e-8)
                torch.cuda.synchronize()
                rows[name] = {"basis_phase_ms": round(float(np.median(basis)), 2),
                              "inference_ms": round(float(np.median(infer)), 2),
                              "setup_ms": round(float(np.median(setup)), 2),
                              "eig_iters_mean": round(inf["eig_iters_mean"], 2), "eig_iters_max": inf["eig_iters_max"],
                              "eig_resid_max": inf["eig_resid_max"], "pcg_iters": it, "relres": rr, "status": st}
            pc.close()
    r0, r1 = rows["random_start"], rows["learned_warm_start"]
    return {"metric": "coarse-basis phase of the set-up with the learned warm start vs random start (cfg4)",
            "value": r1["basis_phase_ms"], "unit": "ms", "n_gpus": 1, "steps": steps, "warmup": warmup,
            "higher_is_better": False, "data": "synthetic (seeded)",
            "dtype": "f32-local/f64-outer" if precision == 1 else "f64",
            "config": {"workload": WORKLOADS[4] + "; network 4 layers, hidden 32, "
                                                  f"{c_out} output columns, trained on seeds 100-103"},
            "random_start": r0, "learned_warm_start": r1,
            "basis_phase_gain_ms": round(r0["basis_phase_ms"] - r1["basis_phase_ms"], 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--scale", type=int, default=None, help="smaller grid side (testing only)")
    ap.add_argument("--applies", type=int, default=20)
    ap.add_argument("--graph", type=int, default=1)
    ap.add_argument("--restart", type=int, default=30, help="FGMRES restart length")
    ap.add_argument("--local-inverse", type=int, default=None,
                    help="2 (default for SPD): the library chooses; 1: local solves through the explicit A_ii^{-1} "
                         "(SPD only); 0: substitutions")
    ap.add_argument("--solve-rows", type=int, default=0,
                    help="block rows per substitution task (1 or 2; 0: autotuned)")
    ap.add_argument("--composition", type=int, default=None,
                    help="0: additive one-level + coarse (PCG for SPD); 1: RAS + deflated coarse correction (FGMRES); "
                         "default 1 for the saddle-point config 6, else 0")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (CPU baseline and the apply errors against the oracle)")
    ap.add_argument("--no-refined", action="store_true",
                    help="skip the mixed-precision run with one local refinement step")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run z = 1.0 * x over 1 GiB (reads 1 GiB, writes 1 GiB): the plain copy kernel "
                         "whose HBM counters scale those of the solve kernels")
    ap.add_argument("--weak-scaling", type=str, default=None,
                    help="comma-separated subdomain counts (powers of two): run the weak-scaling analog instead, "
                         "each count in a process of its own")
    ap.add_argument("--weak-scaling-one", type=int, default=None, help=argparse.SUPPRESS)
    ap.add_argument("--warm-start", action="store_true",
                    help="run the learned warm start against the random start on config 4 instead")
    ap.add_argument("--decay", action="store_true",
                    help="run the eigenvalue / singular value decay study against the overlap instead")
    args = ap.parse_args()
    global SOLVE_ROWS
    SOLVE_ROWS = args.solve_rows
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested); the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    # substitutions by default in the weak-scaling study: at ~30-40 iterations
    # the explicit inverses (twice the factorization's flops) do not pay
    li = 0 if args.local_inverse is None else args.local_inverse
    if args.weak_scaling:
        # one process per N, as separate jobs would run: a process that has
        # held the previous N's buffers would free and map them again
        import subprocess
        rows = []
        for N in [int(a) for a in args.weak_scaling.split(",")]:
            r = subprocess.run([sys.executable, os.path.abspath(__file__), "--weak-scaling-one", str(N), "--steps",
                                str(args.steps), "--warmup", str(args.warmup), "--local-inverse", str(li)],
                               stdout=subprocess.PIPE, text=True)
            if r.returncode != 0:
                log(f"weak scaling N={N} failed with status {r.returncode}")
                sys.exit(r.returncode)
            rows.append(json.loads(r.stdout.strip().splitlines()[-1]))
        out = weak_summary(rows, args.steps, args.warmup, li)
        print(json.dumps(out), flush=True)
        return
    import torch

    from workloads import make_config
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    if args.weak_scaling_one:
        print(json.dumps(weak_scaling(args.weak_scaling_one, args.steps, args.warmup, li)), flush=True)
        return
    if args.decay:
        print(json.dumps(decay_study()), flush=True)
        return
    if args.warm_start:
        print(json.dumps(warm_start_study(max(args.steps, 3), args.warmup, 1)), flush=True)
        return
    log("generating workload")
    prob = make_config(args.config, seed=0, scale=args.scale)
    if args.composition is None:
        args.composition = 1 if args.config == 6 else 0
    A = prob.A
    dev = torch.device("cuda:0")
    dev_in = (torch.as_tensor(A.indptr.astype(np.int32), device=dev),
              torch.as_tensor(A.indices.astype(np.int32), device=dev),
              torch.as_tensor(A.data.astype(np.float64), device=dev),
              torch.as_tensor(prob.part.astype(np.int32), device=dev),
              torch.as_tensor(prob.b, device=dev))
    torch.cuda.synchronize()
    log(f"n={A.shape[0]} nnz={A.nnz} parts={prob.n_parts} overlap={prob.overlap} nev={prob.nev}")
    if args.copy_probe:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    import tempfile
    tune_cache = os.path.join(tempfile.mkdtemp(prefix="tls_tune_"), "tune.txt")
    if args.local_inverse is None:
        # SPD: the library chooses (explicit inverses only when the
        # substitutions inside the tile profiles would read more than half
        # of what the product reads)
        args.local_inverse = 2 if prob.spd else 0
    mixed = run_mode(prob, dev_in, 1, args.steps, args.warmup, args.applies, args.graph, tune_cache,
                     args.composition, args.restart, args.local_inverse)
    plain = None
    if not args.no_fp64:
        plain = run_mode(prob, dev_in, 0, args.steps, args.warmup, args.applies, args.graph, tune_cache,
                         args.composition, args.restart, args.local_inverse)
    refined = None
    if not args.no_refined:
        refined = run_mode(prob, dev_in, 1, min(args.steps, 2), 1, args.applies, args.graph, tune_cache,
                           args.composition, args.restart, args.local_inverse, local_refine=1)
    import paper_2401_03915_amd as tls

    def measured_ctx(precision, refine=0):
        """A context with the timed run's options, for the SpMV timing and
        the apply errors against the oracle."""
        return tls.Preconditioner(A, prob.part, prob.overlap, prob.nev, precision=precision,
                                  matrix_kind=0 if prob.spd else 1, composition=args.composition,
                                  restart=args.restart, local_inverse=args.local_inverse, local_refine=refine,
                                  use_graph=args.graph, autotune=1, tune_cache=tune_cache.encode())
    # SpMV (one per Krylov iteration): launch time from events on the stream it runs on
    pcm = measured_ctx(1)
    xs = torch.randn(A.shape[0], dtype=torch.float64, device=dev, generator=torch.Generator(device=dev).manual_seed(3))
    ys = torch.empty_like(xs)
    for _ in range(5):
        pcm.spmv(xs, ys)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(pcm.stream)
    n_spmv = 200
    for _ in range(n_spmv):
        pcm.spmv(xs, ys)
    e1.record(pcm.stream)
    torch.cuda.synchronize()
    spmv_us = e0.elapsed_time(e1) * 1e3 / n_spmv
    spmv_bytes = 12.0 * A.nnz + 4.0 * (A.shape[0] + 1) + 16.0 * A.shape[0]
    spmv = {"kernel": "k_spmv (y = A x, CSR, FP64)", "bytes_per_launch": spmv_bytes,
            "launch_us": round(spmv_us, 2), "launches_timed": n_spmv,
            "achieved": round(spmv_bytes / (spmv_us * 1e-6) / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(spmv_bytes / (spmv_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": TRAFFIC_SPMV if (args.config == 2 and args.scale is None) else None}
    log(f"spmv {spmv_us:.2f} us, {spmv['achieved']} GB/s")
    info = mixed["info"]
    # dominant kernel: the forward persistent triangular solve of the FP32
    # local factors (the backward one reads the same bytes in about the same
    # time); its launch duration comes from HIP events recorded by the library
    # on the stream the kernel runs on
    inverse = bool(info["local_inverse"])
    # the product reads the lower triangles; a substitution reads the tiles
    # inside the profiles (FP32, 64 x 64 tiles)
    bytes_launch = local_lower_bytes(info, 4) if inverse else 4.0 * 4096.0 * float(info["solve_tiles_fwd"])
    t_fwd = mixed["local_fwd_ms"]
    t_bwd = mixed["local_solve_ms"] - t_fwd
    achieved = bytes_launch / (t_fwd * 1e-3) / 1e9 if t_fwd > 0 else 0.0
    default_workload = args.config == 2 and args.scale is None
    if inverse:
        roof = {"bound": "hbm",
                "kernel": "k_symv<float, 8> (product with the explicit local inverses of one apply, all subdomains)",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": TRAFFIC_SYMV if default_workload else None,
                "bytes_per_launch": bytes_launch, "launch_ms": round(t_fwd, 4),
                "launches_timed": mixed["n_profiled"], "reduce_launch_ms": round(t_bwd, 4)}
    else:
        mode_name = "FWD_L" if prob.spd else "FWD_UL"
        rows = mixed["solve_rows"]
        fwd_kernel = f"k_trsv_sr<float, {mode_name}, {rows}>" if rows > 1 else f"k_trsv<float, {mode_name}>"
        roof = {"bound": "hbm", "kernel": f"{fwd_kernel} (forward local solves of one apply, all subdomains)",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": TRAFFIC.get(rows) if default_workload else None,
                "bytes_per_launch": bytes_launch, "launch_ms": round(t_fwd, 4),
                "launches_timed": mixed["n_profiled"], "backward_launch_ms": round(t_bwd, 4),
                "backward_bytes": 4.0 * 4096.0 * float(info["solve_tiles_bwd"]),
                "backward_GBps": round(4.0 * 4096.0 * float(info["solve_tiles_bwd"]) / (t_bwd * 1e-3) / 1e9, 1)
                if t_bwd > 0 else None,
                "solve_wgs": mixed["solve_wgs"], "solve_order": mixed["solve_order"],
                "solve_order_bwd": mixed["solve_order_bwd"],
                "solve_rows": mixed["solve_rows"]}
    def mfma(mode, dt):
        # flops: the library's count of what it ran (SPD: the tiles inside
        # each local matrix's profile); dense_flops: sum_i m_i^3 / 3 (x2 LU),
        # the dense factorization of the same matrices
        t = mode["info"]["t_setup"][6] * 1e-3  # batched factorization (+ diagonal-tile inverses), ms -> s
        fl = mode["info"]["factor_flops"] or mode["factor_flops"]
        ach = fl / t / 1e12
        kern = ("batched tiled Cholesky inside the tile profile (k_potrf/k_trsm/k_update_blk)" if prob.spd
                else "batched tiled LU (k_getrf/k_trsm_lu/k_update_lu)")
        return {"kernel": kern, "flops": fl, "dense_flops": mode["factor_flops"],
                "ms": round(t * 1e3, 2), "achieved": round(ach, 2), "peak": MFMA_PEAK_TFLOPS[dt], "unit": "TFLOP/s",
                "frac": round(ach / MFMA_PEAK_TFLOPS[dt], 4)}
    def inverse_mfma(mode, dt):
        t = mode["info"]["t_inverse_ms"] * 1e-3
        if t <= 0:
            return None
        fl = mode["info"]["inverse_flops"] or 2.0 * mode["factor_flops"]
        return {"kernel": "explicit local inverses (k_tinv_row + k_sinv_row with the profile, "
                          "else k_tinv_row/k_tinv_update/k_tinv_lauum)", "flops": fl,
                "dense_flops": 2.0 * mode["factor_flops"],
                "ms": round(t * 1e3, 2), "achieved": round(fl / t / 1e12, 2), "peak": MFMA_PEAK_TFLOPS[dt],
                "unit": "TFLOP/s", "frac": round(fl / t / 1e12 / MFMA_PEAK_TFLOPS[dt], 4)}
    apply_err = None
    if plain is not None:
        z32, z64 = mixed["z"], plain["z"]
        apply_err = float(torch.linalg.norm(z32 - z64) / torch.linalg.norm(z64))
    out = {
        "metric": METRIC,
        "value": round(mixed["ms_per_step"] / 1e3, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(mixed["ms_per_step"], 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-local/f64-outer",
        "data": "synthetic (seeded), inputs resident in HBM",
        "config": {"workload": workload_name(args.config, prob, args.scale, args.composition, args.restart),
                   "n": int(A.shape[0]), "nnz": int(A.nnz), "parts": prob.n_parts, "overlap": prob.overlap,
                   "nev": prob.nev, "scale": args.scale, "graph": args.graph,
                   "composition": ["additive", "ras_deflated"][args.composition],
                   "local_solves": "explicit inverse" if inverse else "substitution"},
        "applies_per_s": round(mixed["applies_per_s"], 2),
        "mixed": {"time_to_solve_s": round(mixed["ms_per_step"] / 1e3, 4), "iters": mixed["iters"],
                  "relres": mixed["relres"], "applies_per_s": round(mixed["applies_per_s"], 2),
                  "setup_ms": [round(t, 2) for t in info["t_setup"]], "solve_ms": round(info["t_solve"], 2),
                  "n_coarse": info["n_coarse"], "gc": info["gc"], "oc": info["oc"],
                  "eig_resid_max": info["eig_resid_max"], "eig_iters_max": info["eig_iters_max"]},
        "roofline": roof,
        "setup_mfma": mfma(mixed, "f32"),
    }
    if inverse:
        out["setup_inverse_mfma"] = inverse_mfma(mixed, "f32")
    if plain is not None:
        pinf = plain["info"]
        b64 = (1.0 if inverse else 2.0) * local_lower_bytes(pinf, 8)
        ach64 = b64 / (plain["local_solve_ms"] * 1e-3) / 1e9 if plain["local_solve_ms"] > 0 else 0.0
        out["plain_fp64"] = {"time_to_solve_s": round(plain["ms_per_step"] / 1e3, 4), "iters": plain["iters"],
                             "relres": plain["relres"], "applies_per_s": round(plain["applies_per_s"], 2),
                             "setup_ms": [round(t, 2) for t in pinf["t_setup"]], "solve_ms": round(pinf["t_solve"], 2),
                             "n_coarse": pinf["n_coarse"], "local_solve_GBps": round(ach64, 1),
                             "local_solve_frac": round(ach64 / HBM_PEAK_GBS, 4),
                             "setup_mfma": mfma(plain, "f64")}
        if inverse:
            out["plain_fp64"]["setup_inverse_mfma"] = inverse_mfma(plain, "f64")
        out["speedup_mixed_vs_fp64"] = round(plain["ms_per_step"] / mixed["ms_per_step"], 3)
        out["apply_rel_diff_mixed_vs_fp64_own_bases"] = apply_err
    if refined is not None:
        out["mixed_refined"] = {"local_refine": 1, "time_to_solve_s": round(refined["ms_per_step"] / 1e3, 4),
                                "iters": refined["iters"], "relres": refined["relres"],
                                "applies_per_s": round(refined["applies_per_s"], 2)}
    out["spmv"] = spmv
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) and apply errors against the oracle")
        ctxs = [("mixed", pcm)]
        if plain is not None:
            ctxs.append(("plain_fp64", measured_ctx(0)))
        if refined is not None:
            ctxs.append(("mixed_refined", measured_ctx(1, 1)))
        out["cpu_baseline"], errs = cpu_baseline(prob, args.config, args.composition, ctxs)
        for name, _ in ctxs:
            out[name]["apply_error_vs_oracle"] = errs[name]
        for name, pc in ctxs[1:]:
            pc.close()
    pcm.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
