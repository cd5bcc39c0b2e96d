"""Benchmark: lambda-path fit time of the GD-PG solver on one MI355X.

Workload: Gaussian 3-D GLAM, n = (100, 100, 1000), p = (30, 30, 200) clamped
cubic B-spline factors, smooth spatio-temporal signal + N(0,1) noise, a
100-value log-spaced lambda path down to 1e-4 lambda_max, every model fitted to
an FP64 KKT residual <= 1e-6.  One "step" is one whole path fit (all rows of the
hot path: rho chains, family update, prox, Armijo, KKT, warm starts).

Prints one JSON line.  The timed form is the inner-chain dtype --dtype (default
bf16); the other forms (f32, f64) are run once each, untimed, for the
speed-up at equal accuracy.  The dominant kernel (the fused slab kernel of the
inner iteration) is timed live with HIP events on the fit's stream.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {  # MI355X published dense peaks
    "f64": 78.6e12, "f32": 157.3e12, "bf16": 2.5e15, "hbm": 8.0e12,
}
METRIC = "lambda-path fit time & rho-transform TFLOP/s at KKT<=1e-6, BF16/FP32 vs FP64"


def flop_model(n, p):
    """Algorithmic flops of one inner iteration in the executed mode order
    (mode 3 first forward, last adjoint): slab_fwd, fused slab chain, slab_adj."""
    n1, n2, n3 = n
    p1, p2, p3 = p
    fwd3 = 2 * p1 * p2 * p3 * n3
    chain = 4 * p1 * n2 * (p2 + n1) * n3       # T2, eta, S1, S2 for every slab
    adj3 = 2 * p1 * p2 * n3 * p3
    return fwd3, chain, adj3


def chain_bytes(n, p, dt_bytes, poisson=False):
    """Algorithmic HBM bytes of one fused slab-chain launch: read T1, write S2
    (p1 p2 n3 each, chain dtype), read the factors once (and V for Poisson)."""
    n1, n2, n3 = n
    p1, p2, p3 = p
    b = 2 * p1 * p2 * n3 * dt_bytes + (n1 * p1 + n2 * p2) * dt_bytes
    if poisson:
        b += n1 * n2 * n3 * 4
    return b


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(d, total_inner_f64, outer_f64, budget_s=15.0):
    """The oracle (plain NumPy FP64, never tuned) on the host cores: seconds per
    inner PG iteration at this workload's size, measured on a bounded sample,
    extrapolated to the full path with the FP64 GPU form's iteration counts."""
    import oracle.glam_oracle as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    n = d.Y.size
    lm = O.lambda_max("gaussian", d.X, d.Y)
    lam = lm * (1e-4) ** (1.0 / 99.0)
    V = np.ones_like(d.Y)
    cz = O.G(d.X, d.Y) / n
    theta0 = np.zeros(d.p)
    s_prod = float(np.prod(O.spectral_radii(d.X)))
    delta = n / s_prod
    t0 = time.perf_counter()
    iters = 0
    while time.perf_counter() - t0 < budget_s and iters < 200:
        O.inner_pg(d.X, V, cz, theta0, lam, delta, None, -1.0, lm, 1)
        iters += 1
    per_iter = (time.perf_counter() - t0) / iters
    # one oracle inner iteration evaluates grad h twice (at y and at x^{l+1}); the
    # GPU evaluates it once, so the per-gradient cost is the fair unit
    per_grad = per_iter / 2.0
    est = per_grad * (total_inner_f64 + 3 * outer_f64)
    return {
        "value": est, "unit": "s", "cores": int(threads), "kind": "oracle", "cpu_model": cpu_model(),
        "host_logical_cpus": os.cpu_count(),
        "sample": (f"{iters} oracle inner PG iterations at lambda_1 of the same workload "
                   f"({per_grad*1e3:.1f} ms per gradient evaluation), extrapolated to the full path with "
                   f"the FP64 GPU form's {total_inner_f64} inner iterations and {outer_f64} outer steps"),
        "extrapolated": True,
    }


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "inner_kernels_gaussian_100x100x1000_bf16_hbm_traffic.txt")
STATS_FILE = os.path.join(ROOT, "profiles", "gaussian_path_100x100x1000_bf16_kernel_stats.txt")
MFMA_FILE = os.path.join(ROOT, "profiles", "inner_kernels_gaussian_100x100x1000_bf16_mfma_counters.txt")
INNER_KERNELS = ("slab_fwd", "slab_chain", "slab_adj")


def kernel_source_hash():
    """sha256[:16] over every library source (csrc/*, in name order) and include/glam.h: a profile
    summary taken on any other source is stale."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1510_03298_amd", "csrc")
    files = [os.path.join(csrc, f) for f in sorted(os.listdir(csrc))] + [os.path.join(ROOT, "include", "glam.h")]
    for f in files:
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def committed_record(path, dtype=None):
    """The machine-readable line of a committed profile summary, or None when it is missing or was
    taken on a different library source (or dtype)."""
    try:
        with open(path) as fh:
            rec = json.loads([ln for ln in fh if ln.startswith("{")][-1])
    except (OSError, IndexError, ValueError):
        return None
    if rec.get("source_sha256_16") != kernel_source_hash():
        return None
    if dtype is not None and rec.get("dtype") != dtype:
        return None
    return rec


def inner_kernel_models(n, p, dt_bytes, family="gaussian"):
    """Algorithmic work of the three kernels of one inner iteration (executed mode order, mode 3
    first forward and last adjoint): flops and HBM bytes per launch.
      slab_fwd  : T1 = inc^T X3 (read the increment and X3, write T1)
      slab_chain: per slab T2, eta, R, S1, S2 (read T1 and the X1, X2 factors, write S2; V for Poisson)
      slab_adj  : S2^T X3 + the proximal step on the FP32 increment state (read S2, X3; per
                  coefficient read grad h(theta_ref) and theta_ref (FP64), d^l, d^{l-1}, q (FP32),
                  write d^{l+1}, q (FP32) and the next increment (chain dtype))."""
    n1, n2, n3 = n
    p1, p2, p3 = p
    P12, P = p1 * p2, p1 * p2 * p3
    kb3 = -(-p3 // 16) * 16
    kbn3 = -(-n3 // 16) * 16
    fwd3, chain, adj3 = flop_model(n, p)
    b_fwd = (kb3 * P12 + kb3 * n3 + n3 * P12) * dt_bytes
    b_chain = chain_bytes(n, p, dt_bytes, poisson=family != "gaussian")
    b_adj = (kbn3 * P12 + kbn3 * p3) * dt_bytes + P * (8 + 8 + 4 + 4 + 4 + 4 + 4 + dt_bytes)
    return {"slab_fwd": (fwd3, b_fwd), "slab_chain": (chain, b_chain), "slab_adj": (adj3, b_adj)}


def copy_calibration(torch, dev, mib):
    """A plain device-to-device copy of known size: its FETCH_SIZE / WRITE_SIZE
    counter readings give the scale from counter units to bytes."""
    src = torch.ones(mib << 18, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": mib << 20, "copy_calibration_bytes_written": mib << 20}))


def gram_path(glam, torch, d, Xd, Yd, stream, nlambda, chain_seconds):
    """The same Gaussian path with the inner gradient from the Kronecker Gram factors
    X_j^T X_j (Sec. 6.2, exact for identity weights): p-sized inner products only, the
    FP64 outer steps still through the rho chain."""
    out = {"workload": "gaussian_path_n100x100x1000_p30x30x200_100lambda_kkt1e-6_gram_inner"}
    for dt, name in ((glam.BF16, "bf16"), (glam.F64, "f64")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = glam.fit_path(Xd, Yd, d.n, d.p, "gaussian", nlambda=nlambda, lambda_min_ratio=1e-4, dtype=dt,
                          kkt_tol=1e-6, stream=stream, raise_on_error=False, inner="gram")
        torch.cuda.synchronize()
        out[name] = {"seconds": time.perf_counter() - t0, "converged": r.code == 0 and r.n_done == nlambda,
                     "max_kkt": float(np.max(r.kkt[:r.n_done])) if r.n_done else None,
                     "inner": int(r.inner_total), "outer": int(r.iters_outer.sum())}
    out["speedup_vs_chain_bf16"] = chain_seconds / out["bf16"]["seconds"]
    return out


def c1_single_lambda(glam, inputs, torch, stream, reps=20):
    """Gaussian n = (20, 20, 20), p = (8, 8, 8), plain FP64 method, one lambda = 0.1 lambda_max, KKT <= 1e-6:
    wall time per fit (median of reps after one warm-up; launch-bound, no roofline claim)."""
    d = inputs.config_c1()
    Xd = [glam.to_device_colmajor(X, glam.F64) for X in d.X]
    Yd = glam.to_device_colmajor(d.Y, glam.F64)
    kw = dict(nlambda=1, dtype=glam.F64, kkt_tol=1e-6, stream=stream, raise_on_error=False)
    first = glam.fit_path(Xd, Yd, d.n, d.p, "gaussian", lambdas=None, **kw)   # lambda_max (warm-up)
    lam = 0.1 * first.lambda_max
    times, r = [], None
    for _ in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = glam.fit_path(Xd, Yd, d.n, d.p, "gaussian", lambdas=[lam], **kw)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    times = times[1:]
    return {"workload": "gaussian_c1_n20x20x20_p8x8x8_single_lambda0.1_kkt1e-6", "dtype": "f64",
            "seconds_median": float(np.median(times)), "seconds_min": float(np.min(times)), "reps": reps,
            "converged": r.code == 0, "kkt": float(r.kkt[0]), "inner": int(r.inner_total),
            "outer": int(r.iters_outer.sum())}


def progress(msg):
    """One progress line on stderr (the JSON result is the only stdout line)."""
    print(f"bench.py: {msg}", file=sys.stderr, flush=True)


def sim65_path(glam, inputs, torch, stream, family, forms=("bf16", "f64")):
    """Section 6.5's simulated design at the largest size the slab kernel takes (r = 3,
    q = 0.5, kappa = 0.25; modes (60, 30, 180), p = (30, 15, 90)): the default
    100-lambda path to 1e-4 lambda_max, KKT <= 1e-6, BF16 and FP64 inner chains."""
    d = inputs.config_sim(r=3, q=0.5, family=family, kappa=0.25)
    Xd = [glam.to_device_colmajor(X, glam.F64) for X in d.X]
    Yd = glam.to_device_colmajor(d.Y, glam.F64)
    out = {"workload": f"sec6.5_simulated_{family}_r3_q0.5_kappa0.25_n{d.n[0]}x{d.n[1]}x{d.n[2]}"
                       f"_p{d.p[0]}x{d.p[1]}x{d.p[2]}_100lambda_kkt1e-6"}
    for dt, name in ((glam.BF16, "bf16"), (glam.F64, "f64")):
        if name not in forms:
            continue
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = glam.fit_path(Xd, Yd, d.n, d.p, family, nlambda=100, lambda_min_ratio=1e-4, dtype=dt, kkt_tol=1e-6,
                          stream=stream, raise_on_error=False)
        torch.cuda.synchronize()
        out[name] = {"seconds": time.perf_counter() - t0, "models": int(r.n_done),
                     "converged": r.code == 0 and r.n_done == 100,
                     "max_kkt": float(np.max(r.kkt[:r.n_done])) if r.n_done else None,
                     "inner": int(r.inner_total), "outer": int(r.iters_outer.sum()),
                     "fp64_from_model": int(r.escalated_at)}
    return out


def sim65_q3_path(glam, inputs, torch, stream):
    """Section 6.5's p > n designs (q = 3, kappa = 0, Gaussian), which run on the generic-GEMM
    path: r = 1 (n = 12,000, p = 324,000), the default 100-lambda path to 1e-4 lambda_max, and
    r = 2 (n = 96,000, p = 2.59 million), 50 lambdas to 1e-2 lambda_max; KKT <= 1e-6, BF16 chain."""
    out = {}
    for r, nl, ratio in ((1, 100, 1e-4), (2, 50, 1e-2)):
        d = inputs.config_sim(r=r, q=3, family="gaussian", kappa=0.0)
        Xd = [glam.to_device_colmajor(X, glam.F64) for X in d.X]
        Yd = glam.to_device_colmajor(d.Y, glam.F64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = glam.fit_path(Xd, Yd, d.n, d.p, "gaussian", nlambda=nl, lambda_min_ratio=ratio, dtype=glam.BF16,
                            kkt_tol=1e-6, stream=stream, raise_on_error=False)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        out[f"r{r}"] = {"workload": f"sec6.5_simulated_gaussian_r{r}_q3_kappa0_n{d.n[0]}x{d.n[1]}x{d.n[2]}"
                                    f"_p{d.p[0]}x{d.p[1]}x{d.p[2]}_{nl}lambda_to_{ratio:g}_kkt1e-6",
                        "seconds": sec, "models": int(res.n_done), "converged": res.code == 0 and res.n_done == nl,
                        "max_kkt": float(np.max(res.kkt[:res.n_done])) if res.n_done else None,
                        "inner": int(res.inner_total), "outer": int(res.iters_outer.sum()),
                        "us_per_inner_iteration": 1e6 * sec / max(1, int(res.inner_total))}
    return out


def components_path(glam, inputs, torch, stream):
    """A model of c = 2 tensor components (Sec. 2), n = (100, 100, 100), component sizes (20, 20, 20)
    and (8, 8, 40), Gaussian, 50 lambdas to 1e-3 lambda_max, KKT <= 1e-6, on the generic-GEMM path."""
    d = inputs.random_components_problem((100, 100, 100), [(20, 20, 20), (8, 8, 40)], family="gaussian", seed=3,
                                         sparsity=0.05)
    comps = [([glam.to_device_colmajor(X, glam.F64) for X in Xs], tuple(X.shape[1] for X in Xs)) for Xs in d.comps]
    Yd = glam.to_device_colmajor(d.Y, glam.F64)
    out = {"workload": "gaussian_c2_components_n100x100x100_p20x20x20+8x8x40_50lambda_kkt1e-6"}
    for dt, name in ((glam.BF16, "bf16"), (glam.F64, "f64")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = glam.fit_path_multi(comps, Yd, d.n, "gaussian", nlambda=50, lambda_min_ratio=1e-3, dtype=dt, kkt_tol=1e-6,
                                stream=stream, raise_on_error=False)
        torch.cuda.synchronize()
        out[name] = {"seconds": time.perf_counter() - t0, "models": int(r.n_done), "converged": r.code == 0,
                     "max_kkt": float(np.max(r.kkt[:r.n_done])) if r.n_done else None,
                     "inner": int(r.inner_total), "outer": int(r.iters_outer.sum())}
    return out


def poisson_path_kron(glam, inputs, torch, stream):
    """The Poisson path n = (64, 64, 365), p = (24, 24, 120) with Sec. 6.2's tensor-product
    weights: p-sized inner iterations on reweighted Gram factors (exact gradient, approximate
    curvature), same FP64 KKT."""
    d = inputs.config_c3()
    Xd = [glam.to_device_colmajor(X, glam.F64) for X in d.X]
    Yd = glam.to_device_colmajor(d.Y, glam.F64)
    out = {"workload": "poisson_path_n64x64x365_p24x24x120_50lambda_kkt1e-6_kron_weights"}
    for dt, name, step in ((glam.F32, "f32", "prop1"), (glam.F64, "f64", "prop1"), (glam.F32, "f32_exact_L", "exact")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = glam.fit_path(Xd, Yd, d.n, d.p, "poisson", nlambda=d.nlambda, lambda_min_ratio=d.lambda_min_ratio,
                          dtype=dt, kkt_tol=1e-6, stream=stream, raise_on_error=False, inner="kron", max_outer=400,
                          kron_step=step)
        torch.cuda.synchronize()
        out[name] = {"seconds": time.perf_counter() - t0, "models": int(r.n_done),
                     "converged": r.code == 0 and r.n_done == d.nlambda,
                     "max_kkt": float(np.max(r.kkt[:r.n_done])) if r.n_done else None,
                     "inner": int(r.inner_total), "outer": int(r.iters_outer.sum())}
    return out


def poisson_path(glam, inputs, torch, stream):
    """Poisson counts, n = (64, 64, 365), p = (24, 24, 120), 50-lambda log grid to
    1e-4 lambda_max, KKT <= 1e-6, BF16 inner chain (FP64 Armijo, KKT and anchors)."""
    d = inputs.config_c3()
    Xd = [glam.to_device_colmajor(X, glam.F64) for X in d.X]
    Yd = glam.to_device_colmajor(d.Y, glam.F64)
    out = {"workload": "poisson_path_n64x64x365_p24x24x120_50lambda_kkt1e-6", "dtype": "bf16"}
    for dt, name in ((glam.BF16, "bf16"), (glam.F64, "f64")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = glam.fit_path(Xd, Yd, d.n, d.p, "poisson", nlambda=d.nlambda, lambda_min_ratio=d.lambda_min_ratio,
                          dtype=dt, kkt_tol=1e-6, stream=stream, raise_on_error=False)
        torch.cuda.synchronize()
        out[name] = {"seconds": time.perf_counter() - t0, "converged": r.code == 0 and r.n_done == d.nlambda,
                     "max_kkt": float(np.max(r.kkt[:r.n_done])) if r.n_done else None,
                     "inner": int(r.inner_total), "outer": int(r.iters_outer.sum())}
    out["speedup_bf16_vs_f64"] = out["f64"]["seconds"] / out["bf16"]["seconds"]
    return out


def batched(glam, inputs, torch, stream):
    """256 independent GLAMs, n_ij ~ U{16..96}, p_ij = round(n_ij / 4), even
    Gaussian / odd Poisson, lambda_i = 0.1 lambda_max_i, FP32 inner chain, all to
    KKT <= 1e-6 (three batched launches per proximal step of all unconverged problems)."""
    probs = inputs.config_c4()
    ups = [{"X": [glam.to_device_colmajor(X, glam.F64) for X in q.X], "Y": glam.to_device_colmajor(q.Y, glam.F64),
            "n": q.n, "p": q.p, "family": q.family} for q in probs]
    # warm-up on the whole batch: module load, and the tuner times the slab-phase variants of each
    # shape class once (kept for the process); the timed call then reuses those choices
    rw = glam.fit_batched(ups, lambda_ratio=0.1, dtype=glam.F32, stream=stream, raise_on_error=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = glam.fit_batched(ups, lambda_ratio=0.1, dtype=glam.F32, kkt_tol=1e-6, stream=stream, raise_on_error=False)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rf = glam.fit_batched(ups, lambda_ratio=0.1, dtype=glam.F32, kkt_tol=1e-6, stream=stream, raise_on_error=False,
                          tuning="fixed", graph=False)
    torch.cuda.synchronize()
    sec_fixed = time.perf_counter() - t0
    return {"workload": "batched_256_uneven_n16-96_kkt1e-6", "dtype": "f32", "seconds": sec,
            "converged": bool(r.code == 0 and np.all(r.status == 0)), "max_kkt": float(np.max(r.kkt)),
            "batched_steps": r.steps, "proximal_steps": r.problem_steps,
            "proximal_steps_per_s": r.problem_steps / sec,
            "graph_replays": r.graph_replays, "tuning_seconds_in_warmup": rw.tune_seconds,
            "tuning_seconds_timed": r.tune_seconds,
            "seconds_fixed_heuristics_stream_launches": sec_fixed,
            "sum_n": int(sum(np.prod(q.n) for q in probs)), "sum_p": int(sum(np.prod(q.p) for q in probs))}


def nll(glam, inputs, torch, stream, reps=50):
    """Poisson NLL L(beta) = (1/n) sum(exp(eta) - y eta) and its gradient at
    n = (128, 128, 256), p = (32, 32, 64), BF16 chain: HIP-event time per call, for the
    one-shot entry points (the factors packed inside every call) and for the packed ones
    (X and Y packed once, only the beta-dependent work per call)."""
    d = inputs.config_c5()
    Yd = glam.to_device_colmajor(d.Y, glam.F64)
    out = {"workload": "poisson_nll_n128x128x256_p32x32x64", "dtype": "bf16"}
    beta = glam.to_device_colmajor(d.extra["beta"], glam.BF16)
    ws = torch.empty(glam.nll_workspace_size(d.n, d.p, glam.BF16), dtype=torch.uint8, device=Yd.device)
    one = torch.ones(1, dtype=torch.float64, device=Yd.device)
    fwd3, chain, adj3 = flop_model(d.n, d.p)
    flops_f = fwd3 + chain // 2          # forward chain only
    flops_b = fwd3 + chain + adj3        # recomputed forward + adjoint
    Xb = [glam.to_device_colmajor(X, glam.BF16) for X in d.X]
    packed = glam.PackedPoissonNLL(Xb, Yd, d.n, d.p, glam.BF16, stream=stream)   # X and Y packed once
    loss_buf = torch.empty(1, dtype=torch.float64, device=Yd.device)            # outputs reused across calls
    grad_buf = torch.empty(int(np.prod(d.p)), dtype=torch.float32, device=Yd.device)
    calls = (("forward", lambda: glam.poisson_nll_forward(Xb, beta, Yd, d.n, d.p, glam.BF16, ws, stream, out=loss_buf),
              flops_f),
             ("backward", lambda: glam.poisson_nll_backward(Xb, beta, Yd, one, d.n, d.p, glam.BF16, ws, stream,
                                                            out=grad_buf), flops_b),
             ("forward_packed", lambda: packed.forward(beta, out=loss_buf), flops_f),
             ("backward_packed", lambda: packed.backward(beta, one, out=grad_buf), flops_b))
    for kind, fn, fl in calls:
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        us = e0.elapsed_time(e1) / reps * 1e3
        out[kind] = {"us_per_call": us, "tflops": fl / (us * 1e-6) / 1e12, "flops_per_call": fl}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dtype", default="bf16", choices=["f64", "f32", "bf16"])
    ap.add_argument("--nlambda", type=int, default=100)
    ap.add_argument("--no-compare", action="store_true", help="skip the untimed runs of the other forms")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--profile-every", type=int, default=800,
                    help="time one inner iteration in this many with HIP events (those blocks run un-captured)")
    ap.add_argument("--lambda-min-ratio", type=float, default=1e-4)
    ap.add_argument("--eager", action="store_true", help="launch every inner iteration eagerly (no HIP graphs)")
    ap.add_argument("--extrapolation", default="restarted", choices=["restarted", "plain"],
                    help="inner-loop extrapolation sequence of the timed form (the other is timed beside it)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the secondary workloads (Poisson path, 256-problem batch, Poisson NLL)")
    ap.add_argument("--only", default=None, metavar="NAME",
                    help="run only this secondary workload (its JSON on one line), e.g. batched_c4 or poisson_nll_c5; "
                         "for profiling one workload's kernels")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB 5 times (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); "
              "the lambda path is sequential and the multi-GPU split is a design note, not a run.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1510_03298_amd import glam, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        copy_calibration(torch, dev, args.copy_calibration)
        return
    if args.only:
        stream = torch.cuda.current_stream(dev)
        only = {"batched_c4": lambda: batched(glam, inputs, torch, stream),
                "poisson_nll_c5": lambda: nll(glam, inputs, torch, stream),
                "poisson_path_c3": lambda: poisson_path(glam, inputs, torch, stream),
                "gaussian_c1": lambda: c1_single_lambda(glam, inputs, torch, stream),
                "poisson_path_c3_kron": lambda: poisson_path_kron(glam, inputs, torch, stream),
                "sim65_gaussian": lambda: sim65_path(glam, inputs, torch, stream, "gaussian"),
                "sim65_poisson": lambda: sim65_path(glam, inputs, torch, stream, "poisson", forms=("bf16",)),
                "sim65_q3_gaussian": lambda: sim65_q3_path(glam, inputs, torch, stream),
                "components_c2": lambda: components_path(glam, inputs, torch, stream)}
        if args.only not in only:
            print(f"bench.py: --only takes one of {sorted(only)}", file=sys.stderr)
            sys.exit(2)
        progress(f"workload {args.only} alone")
        print(json.dumps({args.only: only[args.only]()}), flush=True)
        return
    d = inputs.config_c2(nlambda=args.nlambda)
    n, p = d.n, d.p
    Xd = [glam.to_device_colmajor(X, glam.F64) for X in d.X]
    Yd = glam.to_device_colmajor(d.Y, glam.F64)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    dts = {"f64": glam.F64, "f32": glam.F32, "bf16": glam.BF16}

    def fit(dt, profile_every=0, extrapolation=None):
        return glam.fit_path(Xd, Yd, n, p, "gaussian", nlambda=args.nlambda, lambda_min_ratio=args.lambda_min_ratio,
                             dtype=dts[dt], kkt_tol=1e-6, check_every=8, stream=stream,
                             profile_every=profile_every, raise_on_error=False, graph=not args.eager,
                             extrapolation=extrapolation or args.extrapolation)

    progress(f"Gaussian 100x100x1000 path, {args.warmup} warmup + {args.steps} timed steps ({args.dtype})")
    for _ in range(args.warmup):
        fit(args.dtype)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for _ in range(args.steps):
        results.append(fit(args.dtype, args.profile_every))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ok = all(r.code == 0 and r.n_done == args.nlambda and float(np.max(r.kkt)) <= 1e-6 for r in results)
    sec = elapsed / args.steps

    # the same path with its host-device copies inside the clock (X, Y up from host memory, the
    # theta path back down): reported beside the device-resident time, never as the value
    progress("Gaussian 100x100x1000 path with the host-device copies")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Xc = [glam.to_device_colmajor(X, glam.F64) for X in d.X]
    Yc = glam.to_device_colmajor(d.Y, glam.F64)
    rc = glam.fit_path(Xc, Yc, n, p, "gaussian", nlambda=args.nlambda, lambda_min_ratio=args.lambda_min_ratio,
                       dtype=dts[args.dtype], kkt_tol=1e-6, check_every=8, stream=stream, raise_on_error=False,
                       graph=not args.eager)
    theta_host = rc.theta.cpu().numpy()
    with_copies = {"seconds": time.perf_counter() - t0,
                   "bytes_to_device": int(d.Y.nbytes + sum(X.nbytes for X in d.X)),
                   "bytes_to_host": int(theta_host.nbytes),
                   "converged": rc.code == 0 and rc.n_done == args.nlambda}
    del Xc, Yc, rc, theta_host

    fwd3, chain, adj3 = flop_model(n, p)
    dtb = {"f64": 8, "f32": 4, "bf16": 2}[args.dtype]
    samples = sum(r.chain_samples for r in results)
    avg_iter = sum(r.iter_ms for r in results) / max(samples, 1) * 1e-3
    live_us = {"slab_chain": sum(r.chain_ms for r in results) / max(samples, 1) * 1e3,
               "slab_adj": sum(r.adj_ms for r in results) / max(samples, 1) * 1e3,
               "slab_fwd": sum(r.fwd_ms for r in results) / max(samples, 1) * 1e3}
    models = inner_kernel_models(n, p, dtb)
    stats = committed_record(STATS_FILE) if args.dtype == "bf16" else None
    traffic = committed_record(TRAFFIC_FILE, args.dtype)
    mfma = committed_record(MFMA_FILE, args.dtype)
    peak_mfma = PEAKS[args.dtype]
    kernels = {}
    for k in INNER_KERNELS:
        fl, by = models[k]
        us = live_us[k] if samples and live_us[k] > 0 else None
        ai = fl / by
        entry = {"flops_per_launch": fl, "algorithmic_bytes_per_launch": by, "arithmetic_intensity": ai,
                 "live_avg_launch_us": us,
                 "tflops": fl / (us * 1e-6) / 1e12 if us else None,
                 "gbs": by / (us * 1e-6) / 1e9 if us else None,
                 "frac_of_mfma_peak": fl / (us * 1e-6) / peak_mfma if us else None,
                 "attainable_tflops": min(peak_mfma, ai * PEAKS["hbm"]) / 1e12,
                 "bound": "mfma" if ai * PEAKS["hbm"] >= peak_mfma else "hbm",
                 "hbm_bytes_per_launch": None, "mfma_util_pct": None}
        if traffic and k in traffic.get("kernels", {}):
            entry["hbm_bytes_per_launch"] = traffic["kernels"][k]["hbm_bytes_per_launch"]
        if mfma and k in mfma.get("kernels", {}):
            entry["mfma_util_pct"] = mfma["kernels"][k].get("mfma_util_pct")
            entry["mfma_flops_counted_per_launch"] = mfma["kernels"][k].get("mfma_flops_per_launch")
        if stats and k in stats.get("kernels", {}):
            entry["rocprof_in_path_avg_us"] = stats["kernels"][k]["in_path_avg_us"]
            entry["rocprof_sampled_avg_us"] = stats["kernels"][k].get("sampled_avg_us")
            entry["rocprof_in_path_total_ms"] = stats["kernels"][k]["in_path_total_ms"]
        kernels[k] = entry
    # the dominant kernel: the largest in-path total of the committed trace of this source, else
    # the largest live per-launch time (the three run once per inner iteration)
    if stats and all(k in stats.get("kernels", {}) for k in INNER_KERNELS):
        dom = max(INNER_KERNELS, key=lambda k: stats["kernels"][k]["in_path_total_ms"])
    else:
        dom = max(INNER_KERNELS, key=lambda k: live_us[k])
    e = kernels[dom]
    if e["bound"] == "mfma":
        ach, pk, unit = (e["tflops"], peak_mfma / 1e12, "TFLOP/s")
    else:
        ach, pk, unit = (e["gbs"], PEAKS["hbm"] / 1e9, "GB/s")
    roofline = {
        "kernel": dom, "bound": e["bound"], "achieved": ach, "peak": pk, "unit": unit,
        "frac": ach / pk if ach else None, "traffic": e["hbm_bytes_per_launch"],
        "timing": ("HIP events on the fit's stream around 8 back-to-back re-launches of each inner-loop kernel on "
                   "a sampled iteration's own inputs (one sample per profile_every inner iterations; the adjoint "
                   "step kernel writes its re-run outputs to scratch); the committed rocprofv3 trace of the same "
                   "command gives the launches inside the path (rocprof_in_path_avg_us)"),
        "kernel_source_sha256_16": kernel_source_hash(), "launches_sampled": samples,
        "avg_launch_us": e["live_avg_launch_us"], "flops_per_launch": e["flops_per_launch"],
        "algorithmic_bytes_per_launch": e["algorithmic_bytes_per_launch"],
        "frac_of_mfma_peak": e["frac_of_mfma_peak"],
        "inner_iteration_us": avg_iter * 1e6,
        "inner_iteration_tflops": (fwd3 + chain + adj3) / avg_iter / 1e12 if samples else None,
        "kernels": kernels,
    }
    forms = {args.dtype: {"seconds": sec, "inner": int(np.mean([r.inner_total for r in results])),
                          "outer": int(np.mean([r.iters_outer.sum() for r in results])),
                          "max_kkt": float(max(np.max(r.kkt) for r in results)), "ok": ok}}
    if not args.no_compare:
        for dt in ["f64", "f32", "bf16"]:
            if dt in forms:
                continue
            # timed like the headline form: the same number of steps (the kernels are already loaded
            # and warm from the timed form, so no separate warm-up), mean wall time per path
            progress(f"Gaussian 100x100x1000 path, {dt} form ({args.steps} timed steps)")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rs = [fit(dt) for _ in range(args.steps)]
            torch.cuda.synchronize()
            forms[dt] = {"seconds": (time.perf_counter() - t0) / args.steps, "steps": args.steps,
                         "inner": int(np.mean([r.inner_total for r in rs])),
                         "outer": int(np.mean([r.iters_outer.sum() for r in rs])),
                         "max_kkt": float(max(np.max(r.kkt) for r in rs)),
                         "ok": all(r.code == 0 and r.n_done == args.nlambda for r in rs)}
        for dt in forms:
            forms[dt]["speedup_vs_f64"] = forms["f64"]["seconds"] / forms[dt]["seconds"]
        # the timed dtype with the other extrapolation sequence (same steps)
        other = "plain" if args.extrapolation == "restarted" else "restarted"
        progress(f"Gaussian 100x100x1000 path, {args.dtype} form with the {other} extrapolation sequence")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rs = [fit(args.dtype, extrapolation=other) for _ in range(args.steps)]
        torch.cuda.synchronize()
        forms[args.dtype + "_" + other + "_extrapolation"] = {
            "seconds": (time.perf_counter() - t0) / args.steps, "steps": args.steps,
            "inner": int(np.mean([r.inner_total for r in rs])), "outer": int(np.mean([r.iters_outer.sum() for r in rs])),
            "max_kkt": float(max(np.max(r.kkt) for r in rs)),
            "ok": all(r.code == 0 and r.n_done == args.nlambda for r in rs)}
    cpu = None
    if not args.no_cpu and "f64" in forms:
        progress("oracle CPU baseline (bounded sample)")
        cpu = cpu_baseline(d, forms["f64"]["inner"], forms["f64"]["outer"])
    extra = None
    if not args.no_extra:
        jobs = [("gaussian_c1", lambda: c1_single_lambda(glam, inputs, torch, stream)),
                ("gaussian_path_c2_gram", lambda: gram_path(glam, torch, d, Xd, Yd, stream, args.nlambda, sec)),
                ("poisson_path_c3", lambda: poisson_path(glam, inputs, torch, stream)),
                ("poisson_path_c3_kron", lambda: poisson_path_kron(glam, inputs, torch, stream)),
                ("batched_c4", lambda: batched(glam, inputs, torch, stream)),
                ("poisson_nll_c5", lambda: nll(glam, inputs, torch, stream)),
                ("sim65_gaussian", lambda: sim65_path(glam, inputs, torch, stream, "gaussian")),
                # BF16 only: its FP64 form takes ~46 s (1.97M launch-bound inner iterations at n = 324k)
                ("sim65_poisson", lambda: sim65_path(glam, inputs, torch, stream, "poisson", forms=("bf16",))),
                ("sim65_q3_gaussian", lambda: sim65_q3_path(glam, inputs, torch, stream)),
                ("components_c2", lambda: components_path(glam, inputs, torch, stream))]
        extra = {}
        for name, job in jobs:
            progress(f"workload {name}")
            extra[name] = job()
    out = {
        "metric": METRIC, "value": sec, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sec * 1e3, "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": "gaussian_path_n100x100x1000_p30x30x200_100lambda_kkt1e-6",
                   "n": list(n), "p": list(p), "nlambda": args.nlambda, "lambda_min_ratio": args.lambda_min_ratio,
                   "kkt_tol": 1e-6, "family": "gaussian", "graphs": not args.eager,
                   "extrapolation": args.extrapolation},
        "all_models_converged": ok,
        "path_with_host_copies": with_copies,
        "forms": forms,
        "flops_per_inner_iteration": fwd3 + chain + adj3,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "other_workloads": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
