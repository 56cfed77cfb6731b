#!/usr/bin/env python3
"""Throughput of the Helmholtz hot path on one MI355X.

Workload (one "step"): the 401 x 401 layered-model configuration with five
frequencies (1.5, 2.25, 3, 4.5, 6 Hz at 25 m spacing), 64 point sources per
frequency: factor the five systems A(m, w) (block chains batched in shared
launches) and solve all 5 x 64 right-hand sides to a relative residual
<= 1e-10.  The headline form factors in complex64 on the matrix cores and
refines in FP64; the plain FP64 form is timed beside it.

Metric: right-hand-side solves per second (5 x 64 per step / step time),
with p50/p99 step latency.  Inputs are seeded synthetic layered models
resident in HBM before the timed region.

Schedule: the K timed steps run as a pipeline of independent batches
(paper_2301_10762_amd.pipeline): the factorisations of the next F steps run
side by side, each on a stream of its own (F = --factor-streams, default 2:
three batches in flight), while step k is solved on another stream; every step
is still factored and solved in full, with the same kernels.  The serial schedule (one step at a time) is timed first and reported
beside it, with the per-step latency percentiles and the per-kernel timings
that the roofline figure uses.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Helmholtz RHS solves/s at 401^2 (rel. residual<=1e-10) vs FP64 plain; p50/p99 ms"
TOL = 1e-10
PEAK = {"fp64": 78.6, "fp32_ir": 157.3}           # dense matrix-core TFLOP/s (MI355X)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_factor_step_401x401_5freq_64src_fp32ir_traffic.txt")
KERNEL_SRCS = [os.path.join(ROOT, "paper_2301_10762_amd", "csrc", f)
               for f in ("helm_factor.hip", "helm_device.h", "helm_internal.h")]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--precision", default="fp32_ir", choices=["fp32_ir", "fp64"])
    p.add_argument("--fp64-steps", type=int, default=None, help="timed steps of the FP64 comparison (0 = skip)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--schedule", default="both", choices=["both", "serial"],
                   help="both: serial steps (kernel timings, latency) then the headline with batches in "
                        "flight; serial: the serial steps only (value = their throughput)")
    p.add_argument("--factor-streams", type=int, default=2,
                   help="factorisations side by side in the pipelined schedule (2: three batches in flight)")
    p.add_argument("--fp64-factor-streams", type=int, default=1,
                   help="the same for plain complex128 factors, whose heavier steps gain nothing from a second "
                        "factorisation beside the first (1: two batches in flight)")
    p.add_argument("--no-extras", action="store_true",
                   help="skip the factor-only, forward+adjoint (misfit and gradient) and Gauss-Newton timings")
    p.add_argument("--profile-copy", action="store_true",
                   help="only run a plain device copy of known size (counter calibration) and exit")
    p.add_argument("--misfit-only", action="store_true",
                   help="only run phi + grad phi (forward + adjoint + gradient assembly) at the 401^2 workload")
    p.add_argument("--hessian-only", action="store_true",
                   help="only run the full-Hessian, PCG, upper-level gradient and FWI measurements at 201^2")
    p.add_argument("--oracle-worker", action="store_true",
                   help="internal: time the CPU oracle on one 401^2 frequency and print one JSON line "
                        "(the single-core leg of the CPU baseline, run as a child process)")
    return p.parse_args()


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def src_sha():
    """Digest of the sources the factorisation-step kernel is compiled from."""
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def read_traffic(prec):
    """HBM bytes per k_factor_step launch from the committed counter summary
    (lines "key: value"), or None when it is missing, was taken for another
    precision, or the kernel's sources changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if ":" in line and not line.startswith((" ", "#", "|", "`")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_sources_sha256") != src_sha() or kv.get("precision") != prec:
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model():
    """The host CPU's model name and the cores this process may use."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return name, len(os.sched_getaffinity(0))


def oracle_worker():
    """Single-core leg of the CPU baseline (run with OMP_NUM_THREADS=1 as a
    child process): the oracle's banded-LU factor and all 64 source solves of
    the 6 Hz system of the 401^2 workload."""
    import oracle
    from paper_2301_10762_amd import inputs as I
    w = I.config_c3()
    g = oracle.Grid.of(w)
    t0 = time.perf_counter()
    F = oracle.Factor(g, w.m, w.omegas[-1])
    F.solve(oracle.unit_sources(g, w.sources))
    t = time.perf_counter() - t0
    F.close()
    print(json.dumps({"seconds": t, "threads": oracle.num_threads(), "solves": len(w.sources)}), flush=True)


def start_single_core_oracle():
    """Start the single-core oracle timing in a child process (one of the
    host's cores; it runs after the GPU measurements, before the all-core
    run)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    return subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-worker"], env=env,
                            stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)


def cpu_baseline(w, X_gpu, proc1):
    """The CPU oracle on the whole 401^2 workload with all host cores: the
    banded-LU factor of each of the five systems and all 64 source solves,
    timed per frequency.  Its solutions also give the error of the GPU's
    solutions (X_gpu: precision -> five [S][N] arrays) per frequency: the
    relative 2-norm error of every column, the worst over the 64 sources,
    and the same in the max-norm.  proc1: the single-core child process."""
    import numpy as np
    import oracle
    # the single-core child first: a busy core would slow the all-core run
    one = None
    if proc1 is not None:
        out, errtxt = proc1.communicate(timeout=1800)
        if proc1.returncode == 0 and out.strip():
            r = json.loads(out.strip().splitlines()[-1])
            one = {"value": round(r["solves"] / r["seconds"], 3), "seconds": round(r["seconds"], 2),
                   "threads": r["threads"]}
        else:
            one = {"error": (errtxt or "")[-300:]}
    g = oracle.Grid.of(w)
    E = oracle.unit_sources(g, w.sources)
    S = len(w.sources)
    per, err = [], {}
    total = 0.0
    worst_rr = 0.0
    for iw, om in enumerate(w.omegas):
        t0 = time.perf_counter()
        F = oracle.Factor(g, w.m, om)
        Xo = F.solve(E)
        tc = time.perf_counter() - t0
        F.close()
        total += tc
        worst_rr = max(worst_rr, float(oracle.relres(g, w.m, om, Xo[:4], E[:4]).max()))
        key = f"{om / (2 * math.pi):.2f}Hz"
        per.append({"frequency": key, "seconds": round(tc, 2)})
        err[key] = {}
        for prec, Xs in X_gpu.items():
            d = Xs[iw] - Xo
            e2 = np.linalg.norm(d, axis=1) / np.linalg.norm(Xo, axis=1)
            ei = np.abs(d).max(axis=1) / np.abs(Xo).max(axis=1)
            err[key][prec] = {"max_over_sources": float(e2.max()), "max_norm": float(ei.max())}
    name, avail = cpu_model()
    n_omega = len(w.omegas)
    base = {"value": round(n_omega * S / total, 3), "unit": "solves/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"the whole 401^2 workload: banded-LU factor + all {S} source solves of each of the "
                      f"{n_omega} frequencies, {total:.1f} s in all; rel. residual <= {worst_rr:.1e}",
            "per_frequency": per, "cpu_model": name, "cores_available": avail}
    if one is not None:
        base["cores_1_value"] = one.get("value")
        base["cores_1_sample"] = ("one frequency (6 Hz) of the 401^2 workload, factor + 64 solves, "
                                  f"{one.get('seconds')} s on {one.get('threads')} thread(s), timed after the "
                                  "GPU part of the benchmark") if "value" in one else one.get("error")
    worst = {p: max(err[k][p]["max_over_sources"] for k in err) for p in X_gpu}
    return base, {"per_frequency": err, "worst": worst,
                  "definition": "per frequency: max over the 64 sources of ||x_s - x_s^oracle|| / "
                                "||x_s^oracle|| (and of the max-norm form), x from the GPU's serial step"}


def per_omega_latency(helm, w, G, m_dev, E, prec, reps=20, warm=3):
    """Latency of one frequency alone (factor + all S solves to the
    tolerance) at the 401^2 workload: p50 / p99 over `reps` repeats after
    `warm` warm-ups, per frequency."""
    import torch
    out = {}
    for om in w.omegas:
        lat = []
        for r in range(warm + reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            F = helm.factor(G, m_dev, om, prec)
            _, info = F.solve(E, tol=TOL)
            F.close()
            torch.cuda.synchronize()
            if r >= warm:
                lat.append(time.perf_counter() - t0)
        f_hz = om / (2 * math.pi)
        out[f"{f_hz:.2f}Hz"] = {"p50_ms": round(percentile(lat, 0.5) * 1e3, 3),
                               "p99_ms": round(percentile(lat, 0.99) * 1e3, 3), "max_relres": info.max_relres}
    return out


def misfit_extra(helm, I, w, G, m_dev, E, prec, reps=2):
    """phi and grad phi (forward + adjoint solves, gradient assembly) at the
    401^2 workload with 200 receivers on the surface; the observations are
    this library's own forward data at the true model (an input for timing,
    not a check)."""
    import numpy as np
    import torch
    n_omega, S = len(w.omegas), len(w.sources)
    rec = w.receivers
    Fs = helm.factor_batch([G] * n_omega, [torch.as_tensor(w.m_true, device="cuda")] * n_omega, w.omegas, "fp64")
    Xt, _ = helm.solve_batch(Fs, [E] * n_omega, tol=TOL)
    for F in Fs:
        F.close()
    ridx = torch.as_tensor(np.asarray(rec, dtype=np.int64), device="cuda")
    d_obs = torch.stack([x[:, ridx] for x in Xt]).contiguous()
    del Xt
    helm.misfit_grad(G, m_dev, w.omegas, d_obs, w.sources, rec, precision=prec, tol=TOL)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        phi, grad, ginfo = helm.misfit_grad(G, m_dev, w.omegas, d_obs, w.sources, rec, precision=prec, tol=TOL)
    torch.cuda.synchronize()
    tg = (time.perf_counter() - t0) / reps
    return {"ms": round(tg * 1e3, 3), "solves_per_s": round(2 * n_omega * S / tg, 2), "solves": 2 * n_omega * S,
            "max_relres": ginfo.max_relres}


def hessian_extra(helm, I, w4, G4, dirs, alpha=1e-4, mu=1e-8, precisions=("fp64", "fp32_ir")):
    """Full-Hessian product (8 directions) and PCG with P2 = Gamma(alpha, mu)
    at 201^2, for each precision of the context's factors."""
    import numpy as np
    import torch
    n_omega, S4 = len(w4.omegas), len(w4.sources)
    E4 = torch.as_tensor(I.point_sources(G4.N, w4.sources), device="cuda")
    Fs = helm.factor_batch([G4] * n_omega, [torch.as_tensor(w4.m_true, device="cuda")] * n_omega, w4.omegas,
                           "fp64")
    Xt, _ = helm.solve_batch(Fs, [E4] * n_omega, tol=TOL)
    for F in Fs:
        F.close()
    ridx = torch.as_tensor(np.asarray(w4.receivers, dtype=np.int64), device="cuda")
    d4 = torch.stack([x[:, ridx] for x in Xt]).contiguous()
    del Xt, E4
    m_fwi = w4.m_true + 0.1 * (w4.m - w4.m_true)
    b = w4.m_true - m_fwi
    out = {"alpha": alpha, "mu": mu, "model": "m_true + 0.1 (m0 - m_true)", "rhs": "m_true - m",
           "pcg_rtol": 1e-6}
    for prec in precisions:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        H = helm.Hessian(G4, m_fwi, w4.omegas, w4.sources, w4.receivers, d4, alpha, mu, precision=prec, tol=TOL)
        torch.cuda.synchronize()
        tc = time.perf_counter() - t0
        try:
            H.apply(dirs)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            hv, hi = H.apply(dirs)
            torch.cuda.synchronize()
            ta = time.perf_counter() - t0
            n_prod = n_omega * S4 * 2 * len(w4.directions)
            t0 = time.perf_counter()
            x, it, rr, pi = H.pcg(b, prec_alpha=alpha, prec_mu=mu, rtol=1e-6, maxit=200)
            torch.cuda.synchronize()
            tp = time.perf_counter() - t0
            plain = None
            if prec == precisions[0]:
                t0 = time.perf_counter()
                _, it0, rr0, _ = H.pcg(b, rtol=1e-6, maxit=4 * it, strict=False)
                torch.cuda.synchronize()
                t_plain = time.perf_counter() - t0
                plain = {"iterations": it0, "relres": rr0, "ms": round(t_plain * 1e3, 3),
                         "converged": bool(rr0 <= 1e-6)}
        finally:
            H.close()
        out[prec] = {"context_ms": round(tc * 1e3, 3),
                     "product": {"ms": round(ta * 1e3, 3), "directions": len(w4.directions), "solves": n_prod,
                                 "solves_per_s": round(n_prod / ta, 2), "max_relres": hi.max_relres},
                     "pcg_p2": {"iterations": it, "relres": rr, "ms": round(tp * 1e3, 3),
                                "ms_per_iteration": round(tp * 1e3 / max(it, 1), 3),
                                "solves_per_s": round(2 * n_omega * S4 * (it + 1) / tp, 2)}}
        if plain:
            out[prec]["cg_plain"] = plain
    return out


def bilevel_extra(helm, I, w4, G4, alpha=1e-4, mu=1e-8, precision="fp64"):
    """One upper-level gradient (Algorithm "Derivative of psi") for one
    training model at 201^2: the training wavefield and its data at 100
    sensors between nodes, the context at the FWI stand-in, PCG with P2 for
    rho, then tau and the derivatives."""
    import numpy as np
    import torch
    n_omega, S4 = len(w4.omegas), len(w4.sources)
    X = (G4.nx - 1) * G4.hx
    P = np.column_stack([np.linspace(0.02 * X, 0.98 * X, 100) + 0.37 * G4.hx, np.full(100, 2.5 * G4.hz)])
    P[:, 0] = np.minimum(P[:, 0], X)
    m_fwi = w4.m_true + 0.1 * (w4.m - w4.m_true)
    E4 = torch.as_tensor(I.point_sources(G4.N, w4.sources), device="cuda")
    out = {"sensors": len(P), "precision": precision, "alpha": alpha, "mu": mu, "pcg_rtol": 1e-6}
    for rep in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Fs = helm.factor_batch([G4] * n_omega, [torch.as_tensor(w4.m_true, device="cuda")] * n_omega, w4.omegas,
                               precision)
        Ut, _ = helm.solve_batch(Fs, [E4] * n_omega, tol=TOL)
        for F in Fs:
            F.close()
        d = torch.stack([helm.restrict(G4, P, U, 0) for U in Ut])
        dd = torch.stack([torch.stack([helm.restrict(G4, P, U, 1), helm.restrict(G4, P, U, 2)], dim=-1) for U in Ut])
        del Ut
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        H = helm.Hessian(G4, m_fwi, w4.omegas, w4.sources, P, d, alpha, mu, precision=precision, tol=TOL)
        try:
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            rho, it, rr, _ = H.pcg(w4.m_true - m_fwi, prec_alpha=alpha, prec_mu=mu, rtol=1e-6, maxit=300)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            dp, da, _ = H.upper_grad(rho, dd)
            torch.cuda.synchronize()
            t4 = time.perf_counter()
        finally:
            H.close()
    # solves: training wavefields, u and lambda, two per PCG product (one
    # more for r_0), tau
    solves = n_omega * S4 * (1 + 2 + 2 * (it + 1) + 1)
    out.update({"data_ms": round((t1 - t0) * 1e3, 3), "context_ms": round((t2 - t1) * 1e3, 3),
                "pcg": {"iterations": it, "relres": rr, "ms": round((t3 - t2) * 1e3, 3)},
                "upper_grad_ms": round((t4 - t3) * 1e3, 3), "total_ms": round((t4 - t0) * 1e3, 3),
                "solves": solves, "solves_per_s": round(solves / (t4 - t0), 2),
                "dpsi_dalpha": da, "dpsi_dp_norm": float(np.linalg.norm(dp))})
    return out


def pcg_batch_extra(helm, I, w4, G4, alpha=1e-3, mu=1e-8, counts=(1, 2, 4)):
    """PCG with P2 for several training models in lockstep (one Hessian
    system each, FP64 contexts), against the same systems one after another."""
    import numpy as np
    import torch
    n_omega = len(w4.omegas)
    E4 = torch.as_tensor(I.point_sources(G4.N, w4.sources), device="cuda")
    ridx = torch.as_tensor(np.asarray(w4.receivers, dtype=np.int64), device="cuda")
    ctx, bs = [], []
    try:
        for k in range(max(counts)):
            wk = I.config_c4(seed=2 + k)
            Fs = helm.factor_batch([G4] * n_omega, [torch.as_tensor(wk.m_true, device="cuda")] * n_omega,
                                   wk.omegas, "fp64")
            Xt, _ = helm.solve_batch(Fs, [E4] * n_omega, tol=TOL)
            for F in Fs:
                F.close()
            d = torch.stack([x[:, ridx] for x in Xt]).contiguous()
            del Xt
            m_fwi = wk.m_true + 0.1 * (wk.m - wk.m_true)
            ctx.append(helm.Hessian(G4, m_fwi, wk.omegas, wk.sources, wk.receivers, d, alpha, mu, precision="fp64",
                                    tol=TOL))
            bs.append(wk.m_true - m_fwi)
        out = {"alpha": alpha, "mu": mu, "pcg_rtol": 1e-6}
        # one untimed run first: the first PCG of a process allocates its
        # scratch, which would be charged to the first timed schedule
        helm.pcg_batch(ctx[:1], bs[:1], prec_alpha=alpha, prec_mu=mu, rtol=1e-6, maxit=300)
        for K in counts:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, its, _, sts, _ = helm.pcg_batch(ctx[:K], bs[:K], prec_alpha=alpha, prec_mu=mu, rtol=1e-6, maxit=300)
            torch.cuda.synchronize()
            tb = time.perf_counter() - t0
            t0 = time.perf_counter()
            for c in range(K):
                helm.pcg_batch(ctx[c:c + 1], bs[c:c + 1], prec_alpha=alpha, prec_mu=mu, rtol=1e-6, maxit=300)
            torch.cuda.synchronize()
            ts = time.perf_counter() - t0
            solves = sum(2 * n_omega * len(w4.sources) * (i + 1) for i in its)
            out[f"models_{K}"] = {"iterations": its, "status": sts, "lockstep_ms": round(tb * 1e3, 3),
                                  "one_after_another_ms": round(ts * 1e3, 3), "speedup": round(ts / tb, 3),
                                  "solves_per_s": round(solves / tb, 2)}
        return out
    finally:
        for H in ctx:
            H.close()


def fwi_extra(helm, I, precision="fp64", max_iters=20, n_data=301):
    """Lower-level FWI by L-BFGS at the 201^2 configuration (3 frequencies,
    30 sources, 100 receivers) from the smoothed starting model.  The data
    come from a second, non-nested grid (n_data^2 over the same domain, the
    true model resampled onto it), where the sources and receivers fall
    between nodes: the inverse-crime-free practice of the paper."""
    import numpy as np
    import torch
    w = I.config_c2()
    G = helm.Grid.of(w)
    n_omega = len(w.omegas)
    X = (G.nx - 1) * G.hx
    Gd = helm.Grid(n_data, n_data, X / (n_data - 1), X / (n_data - 1))
    m_d = I.resample(w.m_true, (G.nx, G.nz, G.hx, G.hz), (Gd.nx, Gd.nz, Gd.hx, Gd.hz))
    src = np.array([[(k % G.nx) * G.hx, (k // G.nx) * G.hz] for k in w.sources])
    rec = np.array([[(k % G.nx) * G.hx, (k // G.nx) * G.hz] for k in w.receivers])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B = helm.point_sources(Gd, src)
    Fs = helm.factor_batch([Gd] * n_omega, [torch.as_tensor(m_d, device="cuda")] * n_omega, w.omegas, "fp64")
    Xt, _ = helm.solve_batch(Fs, [B] * n_omega, tol=TOL)
    for F in Fs:
        F.close()
    d = torch.stack([helm.restrict(Gd, rec, x, 0) for x in Xt]).contiguous()
    del Xt, B
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    t0 = time.perf_counter()
    m, info = helm.fwi(G, w.m, w.omegas, d, w.sources, w.receivers, 1e-6, 1e-8, precision=precision, tol=TOL,
                       memory=5, max_iters=max_iters, gtol=1e-8)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    err0 = float(np.linalg.norm(w.m - w.m_true))
    err = float(np.linalg.norm(m.cpu().numpy() - w.m_true))
    return {"workload": f"c2_layered_201 (3 frequencies, 30 sources, 100 receivers), alpha 1e-6, mu 1e-8; data "
                        f"from a {n_data}^2 grid (sources and receivers between its nodes)",
            "precision": precision, "data_ms": round(t_data * 1e3, 3), "iterations": info["iterations"],
            "evals": info["evals"], "status": info["status"], "phi_ratio": info["phi"] / info["phi0"],
            "model_error_ratio": err / err0, "ms": round(t * 1e3, 3),
            "ms_per_eval": round(t * 1e3 / info["evals"], 3), "solves": info["solves"],
            "solves_per_s": round(info["solves"] / t, 2)}


def main():
    args = parse()
    if args.oracle_worker:
        oracle_worker()
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the systems of this workload are independent per "
              "frequency and each factorisation fits one MI355X; running on several GPUs is not supported.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2301_10762_amd import helm
    from paper_2301_10762_amd import inputs as I

    torch.cuda.set_device(0)
    if args.profile_copy:
        n = 64 << 20                                 # 64 Mi doubles = 512 MiB read + 512 MiB written
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 3}))
        return

    if args.hessian_only:
        w4 = I.config_c4()
        G4 = helm.Grid.of(w4)
        dirs = torch.as_tensor(np.stack(w4.directions), device="cuda")
        print(json.dumps({"hessian_201": hessian_extra(helm, I, w4, G4, dirs),
                          "upper_grad_201": bilevel_extra(helm, I, w4, G4), "fwi_201": fwi_extra(helm, I),
                          "fwi_201_fp32ir": fwi_extra(helm, I, precision="fp32_ir"),
                          "pcg_batch_201": pcg_batch_extra(helm, I, w4, G4)}),
              flush=True)
        return

    w = I.config_c3()
    G = helm.Grid.of(w)
    n_omega, S = len(w.omegas), len(w.sources)
    m_dev = torch.as_tensor(w.m, dtype=torch.float64, device="cuda")
    E = torch.as_tensor(I.point_sources(G.N, w.sources), device="cuda")
    if args.misfit_only:
        print(json.dumps({"misfit_grad": misfit_extra(helm, I, w, G, m_dev, E, args.precision)}), flush=True)
        return
    X = [torch.empty_like(E) for _ in range(n_omega)]
    torch.cuda.synchronize()
    X_gpu = {}

    def step(precision):
        Fs = helm.factor_batch([G] * n_omega, [m_dev] * n_omega, w.omegas, precision)
        _, infos = helm.solve_batch(Fs, [E] * n_omega, tol=TOL, out=X)
        for F in Fs:
            F.close()
        worst = max(i.max_relres for i in infos)
        if not worst <= TOL:
            raise RuntimeError(f"relative residual {worst} above {TOL}")
        return infos

    def run(precision, warmup, steps, timing):
        for _ in range(warmup):
            step(precision)
        torch.cuda.synchronize()
        if timing:
            helm.kernel_timing(True)
        lat, infos = [], None
        t0 = time.perf_counter()
        for _ in range(steps):
            ts = time.perf_counter()
            infos = step(precision)
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - ts) * 1e3)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        kt = {}
        if timing:
            for kind in ("factor_step", "factor_init", "sweep"):
                kt[kind] = helm.kernel_time(kind)
            helm.kernel_timing(False)
        return total, lat, infos, kt

    def run_pipelined(precision, warmup, steps, nf):
        """The same steps as a pipeline: the next nf batches are factored side
        by side (one stream each) while batch k is solved
        (paper_2301_10762_amd.pipeline); at most nf + 1 batches hold factors."""
        from paper_2301_10762_amd.pipeline import Batch, Pipeline
        nf = max(1, nf)
        pipe = Pipeline(factor_streams=nf)
        outs = [[torch.empty_like(E) for _ in range(n_omega)] for _ in range(nf + 1)]

        def batches(k):
            return [Batch([G] * n_omega, [m_dev] * n_omega, w.omegas, [E] * n_omega, precision, TOL,
                          outs[q % (nf + 1)]) for q in range(k)]
        if warmup:
            pipe.run(batches(max(warmup + 1, nf + 1)))   # every factor stream and output set used once
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = pipe.run(batches(steps))
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        worst = max(i.max_relres for _, infos in res for i in infos)
        if not worst <= TOL:
            raise RuntimeError(f"relative residual {worst} above {TOL}")
        return total, res[-1][1]

    prec = args.precision
    nf_head = args.factor_streams if prec == "fp32_ir" else args.fp64_factor_streams
    # serial schedule (one batch at a time), with the per-kernel timing
    total_s, lat, infos, kt = run(prec, args.warmup, args.steps, True)
    solves = n_omega * S * args.steps
    serial = {"value": round(solves / total_s, 2), "ms_per_step": round(total_s / args.steps * 1e3, 3),
              "p50_ms": round(percentile(lat, 0.5), 3), "p99_ms": round(percentile(lat, 0.99), 3)}
    if not args.no_cpu_baseline:
        X_gpu["c64_ir" if prec == "fp32_ir" else "c128"] = [x.cpu().numpy() for x in X]
    # headline: the pipelined schedule
    if args.schedule == "both":
        total, infos_p = run_pipelined(prec, args.warmup, args.steps, nf_head)
    else:
        total = total_s
    value = solves / total
    ms_per_step = total / args.steps * 1e3

    # roofline of the dominant kernel: the factorisation (one k_factor_step
    # launch per panel step of all the systems of a group).  Algorithmic work: the block factorisation's
    # canonical count 8 * (4/3) * n_z * n_x^3 flops per frequency; the timed
    # region factors all five frequencies once per step.
    nx, nz = w.nx, w.nz
    factor_flops = args.steps * n_omega * 8.0 * (4.0 / 3.0) * nz * nx ** 3
    upd_ms, upd_n = kt.get("factor_step", (0.0, 0))
    flops_per_launch = factor_flops / upd_n if upd_n else float("nan")
    avg_upd_s = upd_ms / upd_n * 1e-3 if upd_n else float("nan")
    achieved = flops_per_launch / avg_upd_s / 1e12
    traffic = read_traffic(prec)
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK[prec], "unit": "TFLOP/s",
                "frac": round(achieved / PEAK[prec], 4), "traffic": traffic,
                "kernel": "k_factor_step (one launch per panel step of the five factorisations), timed over "
                          "the serial steps",
                "avg_launch_us": round(avg_upd_s * 1e6, 2), "timed_launches": upd_n,
                "flops_per_launch": flops_per_launch}
    kernels = {}
    for kind, (ms, cnt) in kt.items():
        kernels[kind] = {"avg_us": round(ms / cnt * 1e3, 2) if cnt else None, "timed_launches": cnt}

    # plain FP64 method beside it
    fp64 = None
    fsteps = args.fp64_steps if args.fp64_steps is not None else args.steps
    if prec != "fp64" and fsteps > 0:
        t64, lat64, inf64, _ = run("fp64", 1, fsteps, False)
        if not args.no_cpu_baseline:
            X_gpu["c128"] = [x.cpu().numpy() for x in X]
        tp64 = run_pipelined("fp64", 1, fsteps, args.fp64_factor_streams)[0] if args.schedule == "both" else t64
        v64 = n_omega * S * fsteps / tp64
        fp64 = {"value": round(v64, 2), "ms_per_step": round(tp64 / fsteps * 1e3, 3),
                "serial_value": round(n_omega * S * fsteps / t64, 2),
                "p50_ms": round(percentile(lat64, 0.5), 3), "p99_ms": round(percentile(lat64, 0.99), 3),
                "max_relres": max(i.max_relres for i in inf64), "speedup_of_headline": round(value / v64, 3)}

    extras = None
    if not args.no_extras:
        extras = {}
        # factor-only time of the five systems (headline precision)
        tf = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Fs = helm.factor_batch([G] * n_omega, [m_dev] * n_omega, w.omegas, prec)
            torch.cuda.synchronize()
            tf.append(time.perf_counter() - t0)
            for F in Fs:
                F.close()
        extras["factor_ms"] = round(min(tf) * 1e3, 3)
        # one frequency alone: factor + 64 solves, p50 / p99 over 20 repeats
        extras["per_omega_latency"] = per_omega_latency(helm, w, G, m_dev, E, prec)
        # forward + adjoint: phi and grad phi at the same workload
        extras["misfit_grad"] = misfit_extra(helm, I, w, G, m_dev, E, prec)
        # Gauss-Newton Hessian-vector products: 201^2, 4 frequencies, 32
        # sources, 100 receivers, 8 directions
        w4 = I.config_c4()
        G4 = helm.Grid.of(w4)
        m4 = torch.as_tensor(w4.m, device="cuda")
        dirs = torch.as_tensor(np.stack(w4.directions), device="cuda")
        helm.gn_hvp(G4, m4, w4.omegas, w4.sources, w4.receivers, dirs, precision=prec, tol=TOL)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hv, hinfo = helm.gn_hvp(G4, m4, w4.omegas, w4.sources, w4.receivers, dirs, precision=prec, tol=TOL)
        torch.cuda.synchronize()
        th = time.perf_counter() - t0
        n_solves = len(w4.omegas) * len(w4.sources) * (2 + 2 * len(w4.directions))
        extras["gn_hvp_201"] = {"ms": round(th * 1e3, 3), "directions": len(w4.directions),
                                "solves": n_solves, "solves_per_s": round(n_solves / th, 2),
                                "max_relres": hinfo.max_relres}
        # Full Hessian H1 + H2 + Gamma and the Hessian system H rho = m' - m
        # at the same 201^2 workload.  The model stands in for an FWI result
        # (m_true + 0.1 (m0 - m_true)); the data are this library's forward
        # data at the true model.  One context (factors, u, lambda) serves
        # the 8-direction product and every PCG iteration.
        extras["hessian_201"] = hessian_extra(helm, I, w4, G4, dirs)
        # the upper-level gradient of one training model with 100 sensors
        # between nodes (Algorithm "Derivative of psi")
        extras["upper_grad_201"] = bilevel_extra(helm, I, w4, G4)
        # the lower-level FWI (L-BFGS) at the 201^2 configuration, both
        # precisions of the factors
        extras["fwi_201"] = fwi_extra(helm, I)
        extras["fwi_201_fp32ir"] = fwi_extra(helm, I, precision="fp32_ir")
        # the Hessian systems of several training models in lockstep
        extras["pcg_batch_201"] = pcg_batch_extra(helm, I, w4, G4)
        # the serving workload: 384 Poisson arrivals at 200 requests/s, four
        # batches side by side (lanes), at most 8 requests per batch (one
        # factorisation group); the same stream with plain complex128 factors
        # (the FP64 method served); and the lanes at 150 requests/s
        from paper_2301_10762_amd import serving as SV
        extras["serving_c5"] = SV.run_c5(requests=384, rate=200.0, precision=prec, lanes=4, max_chains=8)
        extras["serving_c5_fp64"] = SV.run_c5(requests=384, rate=200.0, precision="fp64", lanes=4, max_chains=8)
        extras["serving_150"] = SV.run_c5(requests=384, rate=150.0, precision=prec, lanes=4, max_chains=8)
        # above the configured load: the capacity of each precision on the same stream
        extras["serving_250"] = SV.run_c5(requests=384, rate=250.0, precision=prec, lanes=4, max_chains=8)
        extras["serving_250_fp64"] = SV.run_c5(requests=384, rate=250.0, precision="fp64", lanes=4, max_chains=8)

    cpu, oracle_err = None, None
    if not args.no_cpu_baseline:
        # after the GPU part: host work beside it disturbed its timings
        cpu, oracle_err = cpu_baseline(w, X_gpu, start_single_core_oracle())

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 factor + c128 refinement" if prec == "fp32_ir" else "c128",
        "data": "synthetic (seeded layered model + 5% Gaussian random field; Marmousi not available)",
        "config": {"workload": "c3_layered_401: 401x401 grid (25 m), 5 frequencies 1.5-6 Hz, 64 point sources "
                               "per frequency, all solved to rel. residual <= 1e-10",
                   "grid": [nx, nz], "n_omega": n_omega, "sources": S, "parallelism": "single GPU",
                   "precision": prec},
        "schedule": (f"pipelined: the factorisations of the next {max(1, nf_head)} batches run side by "
                     "side (one stream each) while batch k is solved on another stream (each batch = the five "
                     "systems factored and all 5 x 64 right-hand sides solved)")
                    if args.schedule == "both" else "serial: one batch at a time",
        "serial": serial,
        "p50_ms": serial["p50_ms"], "p99_ms": serial["p99_ms"],
        "ir_iters": max(i.ir_iters for i in infos), "max_relres": max(i.max_relres for i in infos),
        "fp64_plain": fp64, "error_vs_oracle": oracle_err, "extras": extras, "roofline": roofline,
        "kernels": kernels, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
