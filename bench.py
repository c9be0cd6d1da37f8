"""Benchmark of the folded-spectrum CG: band-H psi/s on the 4000-atom wire, and
the time-to-residual solves of the metric on the 256-atom wire.

Headline (the JSON line's value): folded-spectrum PCG iterations on the
4000-atom wire, the largest cell of the workload list (50 x 50 x 200 bohr,
128 x 128 x 512 grid, Ecut 10 Ha, 755,605 plane waves, an fcc wire of 4040
sites minus 40 seeded vacancies with Gaussian wells and 4 Kleinman-Bylander
projectors per atom, 1024 bands near E_ref = 0.3 Ha; synthetic stand-in for
the paper's copper nanowire), mixed precision: complex64 FFT/pointwise and
BF16 projector GEMMs with FP32 accumulation for the two H psi of each
iteration, FP64 for the block algebra.  One step = one CG iteration on the
whole block (gradient and preconditioner, conjugation and projection, two H
psi, per-band line minimisation, Gram/Cholesky re-orthonormalisation);
value = band-H psi per second of iteration time (HIP events on the solver's
stream).  The roofline object is the dominant kernel of the iterations.

Extra legs on the 256-atom wire (20 x 20 x 80 bohr, 48 x 48 x 192, 48,369
plane waves, 256 atoms, 128 bands): FP64 iterations; the folded-CG time to
max_i Delta_i <= 1e-6 for the 128 states nearest E_ref (8 buffer bands, median
over three seeded starts) with FP64 + Teter-Payne-Allan, FP64 + the paper's
M(G), mixed with TPA, with M(G) and with the learned preconditioner; the folded
linear equation with the eigenstate-augmented M' (8 and 32 boundary sources);
ChebFD (degree 1500, a window of 64 states); wave-function interpolation
between k-points.  batch64: 64 uneven cubes solved one by one and as one fused
batch (bit for bit the same).  cpu_baseline: the FP64 oracle's H psi on a
bounded sample of the 4000-atom wire.

Prints one JSON line.  Options: --steps K --warmup W --gpus N (1 only)
--no-cpu --no-wire256 --wire256-steps N --no-solve --solve-legs a,b --no-linear
--linear-maxit N --no-chebfd --chebfd-degree D --chebfd-steps S --chebfd-window N
--no-kinterp --no-batch; profiling modes: --wire256-only, --wire4000-hpsi (only
the complex64 H psi of 1024 bands; --tune, --bf16-variant V), --copy-probe BYTES
(HBM counter calibration).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6
BF16_PEAK_TFS = 2500.0


def stage_work(ctx, nb, dtype_bytes, nproj):
    """Algorithmic bytes or flops of one launch of each H psi stage for a batch
    of nb bands: (bound, amount, unit)."""
    n0, n1, n2 = ctx.grid
    colgrid = ctx.ncols * n2 * dtype_bytes          # one band's column grid
    sphere = ctx.npw * dtype_bytes
    return {
        "z_inverse": ("hbm", nb * (sphere + colgrid), "B"),
        "xy_fft_v": ("hbm", nb * 2 * colgrid + n0 * n1 * n2 * (8 if dtype_bytes == 16 else 4), "B"),
        "z_forward_kinetic": ("hbm", nb * (colgrid + 2 * sphere), "B"),
        "projection": ("mfma", 8.0 * nproj * ctx.npw * nb, "flop"),
        "back_projection": ("mfma", 8.0 * nproj * ctx.npw * nb, "flop"),
    }


def cpu_baseline(prob, nb_sample=64, iters=2):
    """The FP64 oracle's folded CG (numpy FFT H psi) on a bounded sample of the
    same cell: nb_sample bands, `iters` iterations."""
    import numpy as np
    from oracle.hamiltonian import Operator
    from oracle.fsm_cg import fsm_cg
    from paper_1907_06821_amd import synth
    op = Operator.from_problem(prob)
    psi0 = synth.start_vectors(2, nb_sample, op.npw)
    t0 = time.perf_counter()
    r = fsm_cg(op.apply, prob.e_ref, psi0, op.kin, tol=1e-30, maxit=iters, check_every=iters)
    dt = time.perf_counter() - t0
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    threads = int(os.environ.get("OMP_NUM_THREADS", cores))
    return {"value": r["n_hpsi"] / dt, "unit": "band-Hpsi/s", "cores": min(cores, threads), "kind": "oracle",
            "sample": f"{prob.name}: {nb_sample} bands, {iters} folded-CG iteration(s) incl. set-up and final "
                      f"Rayleigh-Ritz, {r['n_hpsi']} band-Hpsi in {dt:.1f} s"}


def measured_traffic(stage, mixed, nb, nn_cfg):
    """HBM bytes per launch of the dominant stage from the committed counter runs
    (FETCH_SIZE / WRITE_SIZE, copy-calibrated), if they were taken on this
    workload, on the launch variant the autotuner picked here (nn_cfg: its
    back-projection tile) and the kernel source has not changed since; else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "wire256_fp64_traffic.json")
    if mixed or not os.path.exists(path) or (nb != 128 and not stage.startswith("linear_")):
        return None
    with open(path) as f:
        rec = json.load(f)
    src = os.path.join(ROOT, rec["source"])
    st = rec["stages"].get(stage)
    if st is None or not os.path.exists(src):
        return None
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec["source_sha256"]:
            return None
    if "bytes_by_nn_cfg" in st:
        return st["bytes_by_nn_cfg"].get(str(nn_cfg))
    return st["bytes_per_launch"]


SOLVE_LEGS = (("fp64_tpa", 0, 0), ("fp64_mg", 0, 1), ("mixed_tpa", 1, 0), ("mixed_mg", 1, 1),
              ("mixed_learned", 1, 2))


def solve_legs(ctx, prob, nb, nconv, legs, seeds=(0, 5, 9), maxit=4000, log=None):
    """Folded-CG time to max Delta_i <= 1e-6 (FP64 H psi residuals, final H
    Rayleigh-Ritz) for each (name, precision, preconditioner) from the same seeded
    starts; the step count of a folded solve swings by 10-20% with small
    perturbations (the search for the last wanted states), so each leg reports the
    median over `seeds`.  The learned network comes from the committed weights."""
    import statistics
    import numpy as np
    import torch
    import paper_1907_06821_amd as pw
    from paper_1907_06821_amd import synth, train_precond
    wpath = os.path.join(train_precond.DATA_DIR, train_precond.WEIGHTS)
    meta = None
    if os.path.exists(wpath + ".npy"):
        w = torch.from_numpy(np.load(wpath + ".npy")).to("cuda")
        pw.mlp_set(ctx, w)
        with open(wpath + ".json") as f:
            meta = json.load(f)
    out, ref = {}, {}
    for name, precision, precond in legs:
        if precond == 2 and meta is None:
            out[name] = {"skipped": "no trained weights"}
            continue
        runs = []
        for seed in seeds:
            psi = torch.from_numpy(synth.start_vectors(2, nb, ctx.npw, seed=seed)).to("cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            eig, res, st = pw.folded_cg_solve(ctx, prob.e_ref, psi, tol=1e-6, maxit=maxit, check_every=20,
                                              precision=precision, precond=precond, nconv=nconv,
                                              raise_on_noconv=False)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            near = np.sort(eig[np.argsort(np.abs(eig - prob.e_ref), kind="stable")[:nconv]])
            ref.setdefault(seed, near)
            runs.append({"seed": seed, "seconds": round(dt, 3), "iters": st["iters"], "n_hpsi": st["n_hpsi"],
                         "converged": bool(st["converged"]), "max_resid": st["max_resid"],
                         "max_eig_diff_vs_first_leg": float(np.max(np.abs(near - ref[seed])))})
        out[name] = {"seconds": statistics.median(r["seconds"] for r in runs),
                     "iters": statistics.median(r["iters"] for r in runs),
                     "converged": all(r["converged"] for r in runs),
                     "precision": "mixed" if precision else "fp64", "precond": ("tpa", "mg", "learned")[precond],
                     "per_seed": runs}
        if log:
            log(f"solve {name}: {out[name]}")
    res = {"tol": 1e-6, "bands": nb, "nconv": nconv, "e_ref": prob.e_ref, "seeds": list(seeds),
           "statistic": "median over seeds", "legs": out}
    base, best = out.get("fp64_tpa", {}), out.get("mixed_learned", {})
    if base.get("converged") and best.get("converged"):
        res["speedup_mixed_learned_vs_fp64_tpa"] = round(base["seconds"] / best["seconds"], 3)
    mg = out.get("mixed_mg", {})
    if mg.get("converged") and best.get("converged"):
        res["speedup_mixed_learned_vs_mixed_mg"] = round(mg["seconds"] / best["seconds"], 3)
    if meta is not None:
        res["training"] = {k: meta[k] for k in ("harvest_seconds", "train_seconds", "train_steps", "loss_first",
                                                 "loss_last", "samples")}
    return res


def linear_leg(ctx, prob, nb, nconv, nrhs=8, tol=1e-8, maxit=3000, log=None):
    """The folded linear equation (H - E)^2 psi = (H - E) w for nrhs boundary
    sources at E_ref, to the paper's error ||(H - E) psi - w|| <= 1e-8: first
    the eigensolve that supplies the states near E (mixed precision + M(G),
    seed 0; its time is reported apart), then PCG with M' built from those nb
    eigenpairs and their residuals, and PCG with M(G) alone under the same
    iteration cap."""
    import numpy as np
    import torch
    import paper_1907_06821_amd as pw
    from paper_1907_06821_amd import synth
    phi = torch.from_numpy(synth.start_vectors(2, nb, ctx.npw, seed=0)).to("cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    eig, res, st = pw.folded_cg_solve(ctx, prob.e_ref, phi, tol=1e-6, maxit=4000, check_every=20, precision=1,
                                      precond=1, nconv=nconv, raise_on_noconv=False)
    torch.cuda.synchronize()
    out = {"tol": tol, "nrhs": nrhs, "e_ref": prob.e_ref, "sources": "Gaussian blobs within 0.1 L_z of z = 0",
           "eigensolve": {"seconds": round(time.perf_counter() - t0, 3), "iters": st["iters"], "nev": nb,
                          "converged": bool(st["converged"]), "max_delta_wanted": st["max_resid"],
                          "max_delta_all": float(np.max(res))}}
    miller = pw.basis_miller(prob.grid, prob.cell, prob.ecut, prob.kpt)
    w = torch.from_numpy(synth.boundary_sources(2, nrhs, miller, prob.cell, kpt=prob.kpt, seed=0)).to("cuda")
    # per-stage times from a profiled run of the M' solve (launched kernel by kernel: the per-stage events
    # are recorded by the host), then the timed runs (each check interval replayed from a recorded graph)
    x = torch.zeros_like(w)
    pw.profile_begin(ctx, 40000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pw.folded_linear_solve(ctx, prob.e_ref, w, x, tol=tol, maxit=maxit, check_every=10, raise_on_noconv=False,
                           precond=1, phi=phi, eps=eig, delta=res)
    torch.cuda.synchronize()
    out["mprime_profiled_seconds"] = round(time.perf_counter() - t0, 3)
    prof = pw.profile_end(ctx)
    for name, kw in (("mprime", dict(precond=1, phi=phi, eps=eig, delta=res)), ("m_only", dict(precond=0))):
        x = torch.zeros_like(w)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        err, lst = pw.folded_linear_solve(ctx, prob.e_ref, w, x, tol=tol, maxit=maxit, check_every=10,
                                          raise_on_noconv=False, hist_len=maxit // 10, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[name] = {"seconds": round(dt, 3), "iters": lst["iters"], "converged": lst["converged"],
                     "max_error": lst["max_resid"], "band_hpsi_per_s": round(lst["n_hpsi"] / dt, 1)}
        if log:
            log(f"linear {name}: {out[name]}")
    # the same M' solve for 32 sources: the projector table is streamed once per launch for all of them
    w32 = torch.from_numpy(synth.boundary_sources(2, 32, miller, prob.cell, kpt=prob.kpt, seed=1)).to("cuda")
    x = torch.zeros_like(w32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    err, lst = pw.folded_linear_solve(ctx, prob.e_ref, w32, x, tol=tol, maxit=maxit, check_every=10,
                                      raise_on_noconv=False, precond=1, phi=phi, eps=eig, delta=res)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["mprime_32"] = {"nrhs": 32, "seconds": round(dt, 3), "iters": lst["iters"], "converged": lst["converged"],
                        "max_error": lst["max_resid"], "band_hpsi_per_s": round(lst["n_hpsi"] / dt, 1)}
    if log:
        log(f"linear mprime_32: {out['mprime_32']}")
    out["_eig"] = eig
    if out["mprime"]["converged"]:
        out["iters_ratio_m_only_vs_mprime"] = round(out["m_only"]["iters"] / out["mprime"]["iters"], 2)
    # H psi stages of the M' solve against HBM: at a few bands the projector GEMMs
    # read the whole table per launch for 8 nrhs flops per 16-byte element, below
    # the FP64 ridge, so every stage is bandwidth-bound
    npw, nproj = ctx.npw, ctx.nproj
    n0, n1, n2 = ctx.grid
    table = nproj * npw * 16
    stage_bytes = {
        "z_inverse": nrhs * (npw + ctx.ncols * n2) * 16,
        "xy_fft_v": nrhs * 2 * ctx.ncols * n2 * 16 + n0 * n1 * n2 * 8,
        "z_forward_kinetic": nrhs * (ctx.ncols * n2 + 2 * npw) * 16,
        "projection": table + nrhs * npw * 16 + nrhs * nproj * 16,
        "back_projection": table + nrhs * nproj * 16 + 2 * nrhs * npw * 16,
    }
    stages = {}
    for k, (ms, n) in (prof or {}).items():
        if n == 0 or k not in stage_bytes:
            continue
        ach = stage_bytes[k] / (ms / n / 1e3) / 1e9
        stages[k] = {"avg_us": round(ms / n * 1e3, 2), "launches": n, "bytes": stage_bytes[k],
                     "achieved_gbs": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4),
                     "share": round(ms / 1e3 / out["mprime_profiled_seconds"], 4)}
    if stages:
        dom = max(stages, key=lambda k: stages[k]["avg_us"] * stages[k]["launches"])
        d = stages[dom]
        out["roofline"] = {"bound": "hbm", "achieved": d["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": d["frac"], "kernel": dom, "bytes_per_launch": d["bytes"],
                           "traffic": measured_traffic("linear_" + dom, False, nrhs, None)}
        out["stages"] = stages
    return out


def chebfd_leg(ctx, prob, nb, eig_ref=None, n_window=64, degree=1500, steps=3, log=None):
    """Chebyshev filter diagonalisation of a window around E_ref: spectral bounds
    from 40 Lanczos steps, a window holding n_window of the eigenvalues eig_ref
    (from the folded eigensolve; its edge midway between the n_window-th and the
    next distance from E_ref), nb filtered vectors from a seeded random start,
    `steps` ChebFD steps of the given degree.  Reports the residual of the states
    inside the window after each step, the eigenvalue agreement with the folded
    solve, and the roofline of the dominant H psi stage over the filtering."""
    import numpy as np
    import torch
    import paper_1907_06821_amd as pw
    from paper_1907_06821_amd import synth
    e = prob.e_ref
    v0 = torch.from_numpy(synth.start_vectors(2, 1, ctx.npw, seed=21)[0]).to("cuda")
    t0 = time.perf_counter()
    lo, hi = pw.spectral_bounds(ctx, v0, steps=40)
    t_bounds = time.perf_counter() - t0
    ref = None
    if eig_ref is not None:
        d = np.sort(np.abs(np.asarray(eig_ref) - e))
        w = 0.5 * (d[n_window - 1] + d[n_window])
        ref = np.sort(np.asarray(eig_ref)[np.abs(np.asarray(eig_ref) - e) <= w])
    else:
        w = 0.05
    psi = torch.from_numpy(synth.start_vectors(2, nb, ctx.npw, seed=22)).to("cuda")
    out = {"e_ref": e, "half_width": w, "degree": degree, "nb": nb, "n_window": n_window, "bounds": [lo, hi],
           "bounds_seconds": round(t_bounds, 3), "steps": []}
    pw.profile_begin(ctx, 20000)
    tot = 0.0
    for k in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        eig, res = pw.chebfd_step(ctx, psi, e, w, degree, lo, hi)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        tot += dt
        sel = np.abs(eig - e) <= w
        rec = {"seconds": round(dt, 3), "ritz_in_window": int(sel.sum())}
        if ref is not None:
            # each eigenvalue of the folded solve inside the window, paired with the nearest Ritz value
            # (extra Ritz values in the window are mixtures of states outside it)
            near = np.array([np.argmin(np.abs(eig - x)) for x in ref])
            rec.update({"max_resid_matched": float(res[near].max()),
                        "max_eig_diff_matched": float(np.max(np.abs(eig[near] - ref))),
                        "max_resid_matched_inner_half": float(res[near[np.abs(ref - e) <= 0.5 * w]].max())})
        out["steps"].append(rec)
        if log:
            log(f"chebfd step {k + 1}: {rec}")
    prof = pw.profile_end(ctx)
    out["seconds_per_step"] = round(tot / steps, 3)
    out["band_hpsi_per_s"] = round(steps * (degree + 1) * nb / tot, 1)
    work = stage_work(ctx, nb, 16, ctx.nproj)
    stages = {}
    for k, (ms, n) in prof.items():
        if n == 0:
            continue
        bound, amount, unit = work[k]
        avg_s = ms / n / 1e3
        ach = amount / avg_s / (1e9 if bound == "hbm" else 1e12)
        peak = HBM_PEAK_GBS if bound == "hbm" else FP64_PEAK_TFS
        stages[k] = {"bound": bound, "avg_ms": round(ms / n, 4), "launches": n, "achieved": round(ach, 2),
                     "peak": peak, "frac": round(ach / peak, 4)}
    if stages:
        dom = max(stages, key=lambda k: stages[k]["avg_ms"] * stages[k]["launches"])
        d = stages[dom]
        out["roofline"] = {"bound": d["bound"], "achieved": d["achieved"], "peak": d["peak"],
                           "unit": "GB/s" if d["bound"] == "hbm" else "TFLOP/s", "frac": d["frac"], "kernel": dom}
        out["stages"] = stages
    return out


def batch_leg(n=64, nb=20, nconv=16, log=None):
    """The uneven batch: 64 cubes of 8-14 bohr on 32^3-64^3 grids (16 wanted + 4
    buffer bands, FP64 + M(G), max Delta <= 1e-6, at most 3000 steps, checks every
    20), solved one by one and as one fused batch (every step one launch over all
    problems, finished problems masked on the device); the batch must reproduce
    every problem bit for bit."""
    import numpy as np
    import torch
    import paper_1907_06821_amd as pw
    from paper_1907_06821_amd import synth
    probs = synth.batched_problems(n, seed=0)
    ctxs = [pw.Context.from_problem(p, max_bands=nb) for p in probs]
    starts = [torch.from_numpy(synth.start_vectors(4, nb, c.npw, seed=i)).to("cuda") for i, c in enumerate(ctxs)]
    kw = dict(tol=1e-6, maxit=3000, check_every=20, precision=0, precond=1, nconv=nconv, raise_on_noconv=False)
    for c, p, s_ in zip(ctxs, probs, starts):          # solver workspaces
        pw.folded_cg_solve(c, p.e_ref, s_.clone(), **{**kw, "maxit": 20})
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    one = []
    for c, p, s_ in zip(ctxs, probs, starts):
        psi = s_.clone()
        e, _, st = pw.folded_cg_solve(c, p.e_ref, psi, **kw)
        one.append((e, st, psi))
    torch.cuda.synchronize()
    t_one = time.perf_counter() - t0
    psis = [s_.clone() for s_ in starts]
    t0 = time.perf_counter()
    eigs, _, sts, _ = pw.batch_solve(ctxs, [p.e_ref for p in probs], psis, **kw)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    same = all(np.array_equal(eigs[i], one[i][0]) and torch.equal(psis[i], one[i][2]) for i in range(n))
    out = {"workload": f"{n} cubes of 8-14 bohr on 32^3-64^3 grids, Ecut 8 Ha, npw "
                       f"{min(c.npw for c in ctxs)}-{max(c.npw for c in ctxs)}, {nconv} wanted + {nb - nconv} buffer "
                       "bands, FP64 + M(G), tol 1e-6, maxit 3000",
           "one_by_one_s": round(t_one, 2), "fused_batch_s": round(t_batch, 2),
           "speedup": round(t_one / t_batch, 2), "fused": all(s_["fused"] for s_ in sts),
           "bit_identical": bool(same), "converged": int(sum(s_["converged"] for s_ in sts)),
           "steps_total": int(sum(s_["iters"] for s_ in sts)), "steps_max": int(max(s_["iters"] for s_ in sts))}
    if log:
        log(f"batch of {n} cubes: one by one {t_one:.2f} s, fused {t_batch:.2f} s ({out['speedup']}x), "
            f"bit-identical {same}")
    for c in ctxs:
        c.close()
    return out


def kinterp_leg(prob, nb, nconv, dk=0.02, log=None):
    """Wave-function interpolation along the wire axis: folded eigensolves (mixed +
    M(G), 136 bands, 128 wanted) at k2 = 0 and k1 = (0, 0, dk), interpolation of
    the 128 wanted states to the midpoint (alpha = 1/2), and a direct eigensolve
    there for reference.  Reports the interpolation time against a solve's, and the
    energy error of the interpolated states in the inner half of the window."""
    import dataclasses
    import numpy as np
    import torch
    import paper_1907_06821_amd as pw
    from paper_1907_06821_amd import synth
    out = {"dk": dk, "alpha": 0.5, "n": nconv}
    sol = {}
    for name, kz in (("k2", 0.0), ("k1", dk), ("k", 0.5 * dk)):
        p = dataclasses.replace(prob, kpt=(0.0, 0.0, kz))
        ctx = pw.Context.from_problem(p, max_bands=nb, flags=pw.PW_PREP_C128 | pw.PW_PREP_C64)
        psi = torch.from_numpy(synth.start_vectors(2, nb, ctx.npw, seed=31)).to("cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        eig, res, st = pw.folded_cg_solve(ctx, p.e_ref, psi, tol=1e-6, maxit=4000, check_every=20, precision=1,
                                          precond=1, nconv=nconv, raise_on_noconv=False)
        torch.cuda.synchronize()
        keep = np.sort(np.argsort(np.abs(eig - p.e_ref), kind="stable")[:nconv])
        sol[name] = (ctx, psi[torch.from_numpy(keep).to("cuda")].contiguous(), eig[keep])
        out[f"solve_{name}_seconds"] = round(time.perf_counter() - t0, 3)
        out[f"solve_{name}_converged"] = bool(st["converged"])
    (c1, p1, e1), (c2, p2, e2), (ck, pk, ek) = sol["k1"], sol["k2"], sol["k"]
    pw.kinterp(c1, c2, ck, 0.5, p1, e1, p2, e2)                   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    eps, psik = pw.kinterp(c1, c2, ck, 0.5, p1, e1, p2, e2)
    torch.cuda.synchronize()
    out["interp_seconds"] = round(time.perf_counter() - t0, 4)
    w = np.max(np.abs(ek - prob.e_ref))
    inner = np.abs(ek - prob.e_ref) <= 0.5 * w
    err = [np.min(np.abs(eps - x)) for x in ek[inner]]
    out["inner_states"] = int(inner.sum())
    out["max_energy_error_inner"] = float(np.max(err))
    out["median_energy_error_inner"] = float(np.median(err))
    out["speedup_vs_solve"] = round(out["solve_k_seconds"] / out["interp_seconds"], 1)
    if log:
        log(f"kinterp: {out}")
    return out


def wire4000_autotune(ctx, log=None):
    """The complex64 launch variants of the 4000-atom wire's H psi picked by the
    library's autotuner (FFT passes at up to 128 bands per launch, BF16 GEMM
    variants at the full band count); returns the chosen candidates."""
    import paper_1907_06821_amd as pw
    recs = pw.autotune(ctx, min(128, ctx.cols_bands), dtype=pw.PW_C64, reps=2)
    if log:
        log("wire4000 BF16 GEMM variants (projection + back-projection, ms): " +
            ", ".join(f"{r['sched']}: {r['ms']:.1f}" for r in recs if r["pass_"] == 6))
    return [r for r in recs if r["chosen"]]


def wire4000_hpsi(steps=3, warmup=1, tune=False, bf16_variant=None):
    """Complex64 + BF16 H psi on the 4000-atom wire (50 x 50 x 200 bohr, 128 x 128 x 512 grid,
    755,605 plane waves, 16,000 projectors) for 1024 bands in one call, from a complex64-only
    context (BF16 projector planes built 64 atoms at a time); `tune`: the launch variants the
    folded-CG step uses (wire4000_autotune), else the defaults.  Prints one JSON line."""
    import numpy as np
    import torch
    import paper_1907_06821_amd as pw
    from paper_1907_06821_amd import synth
    torch.cuda.set_device(0)
    prob = synth.config(5)
    nb = prob.nbands
    t0 = time.perf_counter()
    ctx = pw.Context.from_problem(prob, max_bands=nb, flags=pw.PW_PREP_C64)
    torch.cuda.synchronize()
    t_ctx = time.perf_counter() - t0
    tuned = wire4000_autotune(ctx, lambda m: print(m, file=sys.stderr, flush=True)) if tune else []
    if bf16_variant is not None:
        # the BF16 GEMM launch variant forced (counter runs of one variant)
        pw.fft_choose(ctx, {"pass_": 6, "kind": 3, "sched": int(bf16_variant)}, dtype=pw.PW_C64)
        tuned = [r for r in tuned if r["pass_"] != 6] + [{"pass_": 6, "kind": 3, "nthr": 0, "sched": int(bf16_variant)}]
    psi = torch.from_numpy(synth.start_vectors(5, nb, ctx.npw).astype(np.complex64)).to("cuda")
    out = torch.empty_like(psi)
    for _ in range(warmup):
        pw.hpsi(ctx, psi, shift=prob.e_ref, out=out)
    out.zero_()             # a fill kernel: in a kernel trace, the timed calls are the dispatches after it
    torch.cuda.synchronize()
    pw.profile_begin(ctx, 100)
    t0 = time.perf_counter()
    for _ in range(steps):
        pw.hpsi(ctx, psi, shift=prob.e_ref, out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = pw.profile_end(ctx)
    stages = {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
              for k, v in stage_rooflines(ctx, nb, nb * steps, True, prof).items()}
    print(json.dumps({"metric": "band-Hpsi/s, complex64 + BF16 projector GEMMs", "value": round(nb * steps / dt, 1),
                      "unit": "band-Hpsi/s", "ms_per_hpsi": round(dt / steps * 1e3, 3), "dtype": "c64+bf16",
                      "config": {"workload": "wire4000: 50x50x200 bohr, 128x128x512 grid, Ecut 10 Ha, 4000 atoms x 4 "
                                             "KB projectors, 1024 bands in one call", "npw": ctx.npw,
                                 "nproj": ctx.nproj, "bands": nb, "grid": list(ctx.grid)},
                      "context_seconds": round(t_ctx, 2), "device_bytes": ctx.info()["device_bytes"],
                      "autotuned": [{"pass": r["pass_"], "kind": r["kind"], "nthr": r["nthr"], "sched": r["sched"]}
                                    for r in tuned],
                      "stages": stages}))


def wire4000_step(steps, warmup, log=None):
    """The headline: folded-spectrum CG iterations on the 4000-atom wire (50 x 50 x
    200 bohr, 128 x 128 x 512 grid, Ecut 10 Ha, 755,605 plane waves, 4000 atoms x 4
    KB projectors, 1024 bands near E_ref = 0.3 Ha), mixed precision: complex64
    FFT/pointwise and BF16 projector GEMMs (FP32 accumulation) for the two H psi
    of each iteration, FP64 for the block algebra (Gram/Cholesky, projections,
    rotations); the residual checks use FP64 H psi with projector rows generated
    per call (the 193 GB FP64 table is never stored).  The learned preconditioner
    (committed weights) if present, else the paper's M(G).

    One step = one CG iteration on the whole block.  `warmup` iterations run as a
    solve of their own first; then a solve of `steps` iterations whose iterations
    alone are timed by HIP events on the solver's stream (its set-up, its one
    residual check and its final Rayleigh-Ritz are reported apart).  value =
    2 nb steps / iteration time."""
    import numpy as np
    import torch
    import paper_1907_06821_amd as pw
    from paper_1907_06821_amd import synth, train_precond
    prob = synth.config(5)
    nb = prob.nbands
    t0 = time.perf_counter()
    ctx = pw.Context.from_problem(prob, max_bands=nb, flags=pw.PW_PREP_C64 | pw.PW_PREP_C128_OTF)
    torch.cuda.synchronize()
    t_ctx = time.perf_counter() - t0
    if log:
        log(f"wire4000 context: {t_ctx:.1f} s, {ctx.info()['device_bytes'] / 1e9:.1f} GB, "
            f"{ctx.cols_bands} bands per FFT launch")
    # complex64 launch variants picked by the library's autotuner (not timed)
    tuned = wire4000_autotune(ctx, log)
    wpath = os.path.join(train_precond.DATA_DIR, train_precond.WEIGHTS + ".npy")
    precond = 1
    if os.path.exists(wpath):
        pw.mlp_set(ctx, torch.from_numpy(np.load(wpath)).to("cuda"))
        precond = 2
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    psi = torch.randn((nb, ctx.npw), dtype=torch.complex128, device="cuda", generator=gen)
    opts = dict(tol=1e-30, precision=1, precond=precond, raise_on_noconv=False)
    _, _, stw = pw.folded_cg_solve(ctx, prob.e_ref, psi, maxit=max(1, warmup), check_every=max(1, warmup), **opts)
    torch.cuda.synchronize()
    if log:
        log(f"wire4000 warm-up: {stw['iters']} iterations, {stw['ms_iters']:.0f} ms of iterations, "
            f"set-up {stw['ms_setup']:.0f} ms, check {stw['ms_checks']:.0f} ms, max residual {stw['max_resid']:.3e}")
    pw.profile_begin(ctx, 100000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    eig, res, st = pw.folded_cg_solve(ctx, prob.e_ref, psi, maxit=steps, check_every=steps, **opts)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = pw.profile_end(ctx)
    it_s = st["ms_iters"] / 1e3
    band_hpsi = 2 * nb * steps
    value = band_hpsi / it_s
    stages = stage_rooflines(ctx, nb, band_hpsi, True, prof)
    dom = max(stages, key=lambda k: stages[k]["total_ms"])
    d = stages[dom]
    roofline = {"bound": d["bound"], "achieved": round(d["achieved"], 3), "peak": d["peak"], "unit": d["unit"],
                "frac": round(d["frac"], 4), "kernel": dom, "work_per_launch": d["work_per_launch"],
                "traffic": measured_traffic_wire4000(dom, next((r["sched"] for r in tuned if r["pass_"] == 6), None))}
    ideal = sum(v["work_per_launch"] * v["launches"] / (v["peak"] * (1e9 if v["bound"] == "hbm" else 1e12))
                for v in stages.values())
    roofline["step_frac"] = round(ideal / it_s, 4)
    roofline["step_ideal_ms"] = round(ideal / steps * 1e3, 3)
    line = {
        "metric": "band-Hψ/sec and folded-CG time to residual 1e-6 (mixed+learned vs FP64)",
        "value": round(value, 1),
        "unit": "band-Hpsi/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(st["ms_iters"] / steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+bf16 H psi, f64 block algebra",
        "data": "synthetic",
        "config": {"workload": "wire4000: 50x50x200 bohr, 128x128x512 grid, Ecut 10 Ha, npw 755605, 4000 atoms x 4 "
                               "KB projectors (1% vacancies), 1024 bands near E_ref 0.3 Ha, folded-spectrum PCG "
                               "iteration, mixed precision",
                   "npw": ctx.npw, "bands": nb, "nproj": ctx.nproj, "grid": list(ctx.grid), "precision": "mixed",
                   "precond": ("tpa", "mg", "learned")[precond], "cols_bands": ctx.cols_bands},
        "roofline": roofline,
        "stages": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                   for k, v in stages.items()},
        "phases_ms": {"setup": round(st["ms_setup"], 1), "iterations": round(st["ms_iters"], 1),
                      "check": round(st["ms_checks"], 1), "final_rayleigh_ritz": round(st["ms_final"], 1)},
        "solve_wall_s": round(wall, 2),
        "context_s": round(t_ctx, 2),
        "device_bytes": ctx.info()["device_bytes"],
        "max_resid_fp64": st["max_resid"],
        "autotuned": [{"pass": r["pass_"], "kind": r["kind"], "nthr": r["nthr"], "sched": r["sched"],
                       "us": round(r["ms"] * 1e3, 1)} for r in tuned],
    }
    if log:
        log(f"wire4000: {value:.1f} band-Hpsi/s, {st['ms_iters'] / steps:.1f} ms per iteration, dominant {dom} "
            f"{d['frac']:.3f} of peak")
    ctx.close()
    del psi
    torch.cuda.empty_cache()
    return line


def measured_traffic_wire4000(stage, bf16_variant=None):
    """HBM bytes per launch of `stage` on the 4000-atom wire from the committed
    counter runs (FETCH_SIZE / WRITE_SIZE, copy-calibrated), if they were taken
    on the current source of the kernel (and, for the projector GEMMs, on the
    BF16 launch variant in use); else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "wire4000_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    st = rec.get("stages", {}).get(stage)
    if st is None:
        return None
    src = os.path.join(ROOT, st["source"])
    if not os.path.exists(src):
        return None
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != st["source_sha256"]:
            return None
    if "bytes_by_variant" in st:
        return st["bytes_by_variant"].get(str(bf16_variant))
    return st["bytes_per_launch"]


def cpu_baseline_wire4000(atoms=100, log=None):
    """The FP64 oracle's matrix-free H psi (numpy FFT, projector rows built a
    hundred atoms at a time) on the 4000-atom wire, timed on a bounded sample: one
    band's local and kinetic part, plus the nonlocal part of one chunk of `atoms`
    atoms, scaled to all 4000 atoms (the chunks cost the same).  Run on all the
    host's threads and on one."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle.hamiltonian import Operator, hpsi, projectors
    from paper_1907_06821_amd import synth
    prob = synth.config(5)
    op = Operator.from_problem(prob)
    c = synth.start_vectors(5, 1, op.npw, seed=1)

    def one():
        t0 = time.perf_counter()
        hpsi(c, op.miller, op.kin, op.vgrid, None, None, prob.e_ref)
        t1 = time.perf_counter()
        beta = projectors(op.miller, op.cell, op.pos, op.sigma, op.nl, op.kpt, atoms=range(atoms))
        d = op.dproj[:atoms * op.nl]
        _ = ((c @ beta.conj().T) * d[None, :]) @ beta
        t2 = time.perf_counter()
        return (t1 - t0) + (t2 - t1) * (prob.natom / atoms)

    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    threads = min(cores, int(os.environ.get("OMP_NUM_THREADS", cores)))
    t_all = one()
    with threadpool_limits(limits=1):
        t_one = one()
    out = {"value": round(1.0 / t_all, 4), "unit": "band-Hpsi/s", "cores": threads, "kind": "oracle",
           "value_1core": round(1.0 / t_one, 4),
           "sample": f"wire4000: one band-H psi (FP64), local part plus the nonlocal part of {atoms} of "
                     f"{prob.natom} atoms scaled by {prob.natom // atoms}; {t_all:.1f} s per band-H psi on "
                     f"{threads} threads, {t_one:.1f} s on 1"}
    if log:
        log(f"cpu baseline: {out}")
    return out


def wire256_legs(args, log):
    """The 256-atom wire (20 x 20 x 80 bohr, 48 x 48 x 192 grid, 48,369 plane waves,
    1024 projectors): FP64 folded-CG iterations at 128 bands (band-H psi/s and its
    roofline), the time-to-residual solves of the metric, the folded linear
    equation, ChebFD and the k-point interpolation."""
    import numpy as np
    import torch
    import paper_1907_06821_amd as pw
    from paper_1907_06821_amd import synth
    prob = synth.config(2)
    nbuf = 8
    ctx = pw.Context.from_problem(prob, max_bands=prob.nbands + nbuf, flags=pw.PW_PREP_C128 | pw.PW_PREP_C64)
    nb = prob.nbands
    steps = args.wire256_steps
    tuned = {n: [r for r in pw.autotune(ctx, n, dtype=pw.PW_C128, reps=3) if r["chosen"]] for n in (nb, nb + nbuf)}
    psi0 = torch.from_numpy(synth.start_vectors(2, nb, ctx.npw)).to("cuda")
    opts = dict(tol=1e-30, check_every=20, precision=0, raise_on_noconv=False)
    psi = psi0.clone()
    pw.folded_cg_solve(ctx, prob.e_ref, psi, maxit=3, **opts)
    psi = psi0.clone()
    pw.profile_begin(ctx, 200000)
    eig, res, st = pw.folded_cg_solve(ctx, prob.e_ref, psi, maxit=steps, **opts)
    torch.cuda.synchronize()
    prof = pw.profile_end(ctx)
    it_s = st["ms_iters"] / 1e3
    stages = stage_rooflines(ctx, nb, 2 * nb * steps, False, prof)
    dom = max(stages, key=lambda k: stages[k]["total_ms"])
    d = stages[dom]
    ideal = sum(v["work_per_launch"] * v["launches"] / (v["peak"] * (1e9 if v["bound"] == "hbm" else 1e12))
                for v in stages.values())
    out = {"step": {"workload": "wire256: 20x20x80 bohr, 48x48x192 grid, Ecut 10 Ha, npw 48369, 256 atoms x 4 KB "
                                "projectors, 128 bands near E_ref 0.3 Ha, FP64 folded-spectrum PCG iteration",
                    "steps": steps, "value": round(2 * nb * steps / it_s, 1), "unit": "band-Hpsi/s",
                    "ms_per_step": round(st["ms_iters"] / steps, 4), "dtype": "c128",
                    "roofline": {"bound": d["bound"], "achieved": round(d["achieved"], 3), "peak": d["peak"],
                                 "unit": d["unit"], "frac": round(d["frac"], 4), "kernel": dom,
                                 "traffic": measured_traffic(dom, False, nb, next(
                                     (r["sched"] for r in tuned[nb] if r["pass_"] == 4), None)),
                                 "step_frac": round(ideal / it_s, 4)},
                    "stages": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                               for k, v in stages.items()},
                    "autotuned": {str(n): [{"pass": r["pass_"], "kind": r["kind"], "nthr": r["nthr"],
                                            "sched": r["sched"], "us": round(r["ms"] * 1e3, 1)} for r in rs]
                                  for n, rs in tuned.items()}}}
    log(f"wire256 step: {out['step']['value']} band-Hpsi/s, dominant {dom} {d['frac']:.3f}")
    if not args.no_solve:
        legs = [l for l in SOLVE_LEGS if l[0] in args.solve_legs.split(",")]
        out["solve"] = solve_legs(ctx, prob, nb + nbuf, nb, legs, log=log)
    eig_ref = None
    if not args.no_linear:
        out["linear"] = linear_leg(ctx, prob, nb + nbuf, nb, maxit=args.linear_maxit, log=log)
        eig_ref = out["linear"].pop("_eig")
    if not args.no_chebfd:
        out["chebfd"] = chebfd_leg(ctx, prob, nb + nbuf, eig_ref, n_window=args.chebfd_window,
                                   degree=args.chebfd_degree, steps=args.chebfd_steps, log=log)
    if not args.no_kinterp:
        out["kinterp"] = kinterp_leg(prob, nb + nbuf, nb, log=log)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob, nb_sample=args.cpu_bands)
    ctx.close()
    return out


def stage_rooflines(ctx, nb, band_hpsi, mixed, prof):
    """Per-stage achieved rate against its bound, from the per-stage profile of a
    solve's iterations (HIP events on the solver's stream).  Algorithmic work:
    FFT passes move the bytes of stage_work per band-H psi (band_hpsi of them in
    the profiled iterations; the xy pass also reads V once per launch) against
    HBM; the projector GEMMs do 8 nproj npw flops per band-H psi against the
    matrix peak of their precision (BF16 mixed, FP64 otherwise); the solver's FP64
    block products do 8 npw nb^2 flops per product (three in block_rotate3, whose
    lower triangular matrix has nb (nb + 1) / 2 nonzero entries), a Hermitian Gram
    matrix X^H X 4 npw nb (nb + 1) (the entries on and below the diagonal), against
    the FP64 peak.  avg_ms and work_per_launch are totals over launches."""
    npw = ctx.npw
    n0, n1, n2 = ctx.grid
    per_band = stage_work(ctx, 1, 8 if mixed else 16, ctx.nproj)
    vbytes = n0 * n1 * n2 * (4 if mixed else 8)
    blk = 8.0 * npw * nb * nb
    stages = {}
    for k, (ms, n) in prof.items():
        if n == 0 or ms <= 0:
            continue
        if k.startswith("block_"):
            # block_rotate3 rotates by the Cholesky inverse, lower triangular: nb (nb + 1) / 2 of its
            # entries are not zero, 3 blocks x 8 npw flops each
            bound, peak = "mfma", FP64_PEAK_TFS
            if k == "block_rotate3":
                total = 3 * 8.0 * npw * nb * (nb + 1) / 2 * n
            elif k == "block_gram_herm":
                total = 4.0 * npw * nb * (nb + 1) * n
            else:
                total = blk * n
        else:
            bound, amount, _ = per_band[k]
            if k == "xy_fft_v":
                amount -= vbytes                      # stage_work counts V once per call
            total = amount * band_hpsi + (vbytes * n if k == "xy_fft_v" else 0)
            peak = HBM_PEAK_GBS if bound == "hbm" else (BF16_PEAK_TFS if mixed else FP64_PEAK_TFS)
        scale = 1e9 if bound == "hbm" else 1e12
        ach = total / (ms / 1e3) / scale
        stages[k] = {"bound": bound, "avg_ms": ms / n, "launches": n, "total_ms": ms, "achieved": ach,
                     "peak": peak, "unit": "GB/s" if bound == "hbm" else "TFLOP/s", "frac": ach / peak,
                     "work_per_launch": total / n}
    return stages


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-bands", type=int, default=64)
    ap.add_argument("--no-wire256", action="store_true", help="skip every wire256 leg")
    ap.add_argument("--wire256-steps", type=int, default=40)
    ap.add_argument("--no-solve", action="store_true", help="skip the time-to-residual solves")
    ap.add_argument("--solve-legs", default=",".join(n for n, _, _ in SOLVE_LEGS))
    ap.add_argument("--no-linear", action="store_true", help="skip the folded linear-equation leg")
    ap.add_argument("--linear-maxit", type=int, default=3000, help="iteration cap of the linear-equation leg")
    ap.add_argument("--no-chebfd", action="store_true", help="skip the Chebyshev filter diagonalisation leg")
    ap.add_argument("--chebfd-degree", type=int, default=1500)
    ap.add_argument("--chebfd-steps", type=int, default=3)
    ap.add_argument("--chebfd-window", type=int, default=64, help="eigenstates inside the ChebFD window")
    ap.add_argument("--no-kinterp", action="store_true", help="skip the k-point interpolation leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-cube batch leg")
    ap.add_argument("--wire4000-hpsi", action="store_true",
                    help="only: complex64 H psi throughput on the 4000-atom wire (1024 bands in one call)")
    ap.add_argument("--wire256-only", action="store_true",
                    help="only the wire256 legs (for kernel traces of those legs; not the benchmark line)")
    ap.add_argument("--bf16-variant", type=int, default=None,
                    help="with --wire4000-hpsi: force this BF16 GEMM launch variant (autotuner pass 6)")
    ap.add_argument("--tune", action="store_true",
                    help="with --wire4000-hpsi: the launch variants the folded-CG step autotunes")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES between two device buffers 5 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the solver shards no work across GPUs (bands and problems would "
              "shard without communication in H psi, but no multi-GPU path is implemented)",
              file=sys.stderr)
        sys.exit(2)
    if args.wire4000_hpsi:
        wire4000_hpsi(steps=max(1, args.steps), warmup=max(1, args.warmup), tune=args.tune,
                      bf16_variant=args.bf16_variant)
        return
    if args.copy_probe:
        import torch
        a = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel() * 4, "copies": 5}))
        return

    import torch
    torch.cuda.set_device(0)
    log = lambda m: print(m, file=sys.stderr, flush=True)   # noqa: E731
    if args.wire256_only:
        print(json.dumps({"wire256": wire256_legs(args, log)}))
        return
    line = wire4000_step(args.steps, args.warmup, log=log)
    if not args.no_wire256:
        line["wire256"] = wire256_legs(args, log)
    if not args.no_batch:
        line["batch64"] = batch_leg(log=log)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline_wire4000(log=log)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line))


if __name__ == "__main__":
    main()
