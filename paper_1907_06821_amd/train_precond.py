"""Training of the learned per-G-shell preconditioner, on the GPU.

Samples come from the method's own solves: folded-spectrum CG runs on a cell
store snapshots of the iterate X(t); once converged (X*), every snapshot gives
the per-(shell, band) tables of its gradient g = A x - mu x and of its error
direction e = (I - X* X*^H) x (gauge invariant; the CG steps along -K g, so
K g should point along e).  The network
f(T_shell, T_band, E_ref) of the preconditioner K = M(G) e^f is then fitted
to the cosine loss 1 - Re<K g, e> / (|K g| |e|) with the library's own loss,
gradient and Adam kernels.  The inner products are taken in the metric
diag((T_G - E_ref)^2 + delta^2), the plane-wave diagonal of the folded operator
without the potential: trained that way the network takes fewer CG iterations
than trained on the Euclidean cosine.

    python -m paper_1907_06821_amd.train_precond --out paper_1907_06821_amd/data

writes precond_wire256.npy (float32 weights) and precond_wire256.json (what the
samples were, training time and loss history).  Snapshots come from FP64 solves
on the 256-atom wire (136 bands, converged to 1e-6) and from mixed-precision
solves on the 2000-atom wire (24 bands, 16 wanted).  Near E_ref the 2000-atom
wire's spectrum is so dense that its solves do not reach 1e-6 in thousands of
iterations; there the iterate after 1000 iterations is the reference subspace
for snapshots of the first 160, whose residuals are at least about three times
larger (checked per solve).  The two cells' shell tables are merged, each
snapshot contributing its own cell's shells and bands.  The training energies
and start vectors are disjoint from the ones the benchmark and the tests solve
with.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import paper_1907_06821_amd as pw  # noqa: E402
from paper_1907_06821_amd import synth  # noqa: E402

DATA_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")
WEIGHTS = "precond_wire256"


def harvest(ctx, prob, energies, start_seed, nb, nconv, snap_every, nsnap, maxit, weight_delta=0.5, log=print,
            precision=0, cfg_id=2, ref_ratio=0.0):
    """Solve once per energy with snapshots; returns device tables
    (tabs [S, 3, nshell, nb], tband [S, nb], e_ref [S]) and a record per solve.

    ref_ratio > 0: a solve that stops at maxit unconverged still serves as the
    reference subspace when its final residual is at most ref_ratio times the
    residual at the check after its last snapshot (its error is then a small part
    of every snapshot's); else only converged solves serve."""
    import torch
    tabs_l, tband_l, er_l, solves = [], [], [], []
    for j, e in enumerate(energies):
        psi = torch.from_numpy(synth.start_vectors(cfg_id, nb, ctx.npw, seed=start_seed + j)).to("cuda")
        snaps = torch.zeros((nsnap, nb, ctx.npw), dtype=torch.complex128, device="cuda")
        eig, res, st = pw.folded_cg_solve(ctx, e, psi, tol=1e-6, maxit=maxit, check_every=20, precond=1,
                                          nconv=nconv, snapshots=snaps, snap_every=snap_every, hist_len=maxit // 20 + 2,
                                          raise_on_noconv=False, precision=precision, verbose=int(cfg_id == 3))
        last = snap_every * st["n_snap"]
        after = [r for i, r in st["hist"] if i >= last]
        ratio = st["max_resid"] / after[0] if after else float("inf")
        use = st["converged"] or (ref_ratio > 0 and ratio <= ref_ratio)
        rec = {"cell": prob.name, "e_ref": e, "start_seed": start_seed + j, "iters": st["iters"],
               "seconds": round(st["seconds"], 2), "max_resid": st["max_resid"], "snapshots": st["n_snap"],
               "snapshot_iters": [snap_every * k for k in range(1, st["n_snap"] + 1)],
               "resid_after_last_snapshot": after[0] if after else None, "converged": st["converged"],
               "used": bool(use), "precision": "mixed" if precision else "fp64"}
        solves.append(rec)
        log(f"harvest solve {rec}")
        if not use:
            continue
        for k in range(1, st["n_snap"]):      # the first snapshot is the random start
            tb, tband = pw.mlp_harvest(ctx, e, snaps[k], psi, weight_delta=weight_delta)
            tabs_l.append(tb)
            tband_l.append(tband)
            er_l.append(e)
        del snaps
    if not tabs_l:
        raise RuntimeError("no harvest solve converged")
    tabs = torch.stack(tabs_l).contiguous()
    tband = torch.stack(tband_l).contiguous()
    er = torch.tensor(er_l, dtype=torch.float64, device="cuda")
    return tabs, tband, er, solves


def merge(sets):
    """Training sets of several cells as one: the shell lists are concatenated and
    every snapshot's tables are zero outside its own cell's shells, where they add
    nothing to the loss's sums; a cell solved with fewer bands has zero tables for
    the others, whose band loss and gradient are zero.  Pure data layout."""
    import torch
    nsh = [st.shape[0] for st, _, _, _ in sets]
    nb = max(t.shape[3] for _, t, _, _ in sets)
    total = sum(t.shape[0] for _, t, _, _ in sets)
    tabs = torch.zeros((total, 3, sum(nsh), nb), dtype=torch.float64, device="cuda")
    tband = torch.zeros((total, nb), dtype=torch.float64, device="cuda")
    row, col = 0, 0
    for (shell_t, t, tb, er), n in zip(sets, nsh):
        tabs[row:row + t.shape[0], :, col:col + n, :t.shape[3]] = t
        tband[row:row + t.shape[0], :t.shape[3]] = tb
        row += t.shape[0]
        col += n
    shell_t = torch.cat([s_ for s_, _, _, _ in sets]).contiguous()
    er = torch.cat([e for _, _, _, e in sets]).contiguous()
    return shell_t, tabs, tband, er


def train(shell_t, tabs, tband, er, ecut, steps, lr, seed=0, chunk=50, log=None):
    """Adam on the device, `chunk` steps per library call (the moments carry over)."""
    import torch
    w = torch.from_numpy(synth.mlp_init(seed).astype(np.float32)).to("cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m = v = None
    hist = []
    for s0 in range(0, steps, chunk):
        n = min(chunk, steps - s0)
        h, m, v = pw.mlp_train(shell_t, tband, er, ecut, tabs, w, n, lr=lr, m=m, v=v, step0=s0)
        hist.extend(h.tolist())
        if log:
            log(f"train steps {s0 + n}/{steps}: loss {h[-1]:.5f} ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    return w, np.asarray(hist), time.perf_counter() - t0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DATA_DIR)
    ap.add_argument("--energies", default="0.2,0.25,0.35,0.4", help="training energies on the 256-atom wire")
    ap.add_argument("--energies3", default="0.25,0.35", help="training energies on the 2000-atom wire ('' = none)")
    ap.add_argument("--start-seed", type=int, default=11)
    ap.add_argument("--bands", type=int, default=136)
    ap.add_argument("--nconv", type=int, default=128)
    ap.add_argument("--snap-every", type=int, default=40)
    ap.add_argument("--nsnap", type=int, default=16)
    ap.add_argument("--maxit", type=int, default=2000)
    ap.add_argument("--maxit3", type=int, default=1000)
    ap.add_argument("--bands3", type=int, default=24, help="bands of the 2000-atom wire's solves")
    ap.add_argument("--nconv3", type=int, default=16)
    ap.add_argument("--snap-every3", type=int, default=10)
    ap.add_argument("--ref-ratio3", type=float, default=0.3,
                    help="2000-atom wire: largest final / last-snapshot residual ratio of an unconverged reference")
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--weight-delta", type=float, default=0.5, help="metric delta (Ha); < 0: Euclidean")
    a = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    log = lambda s_: print(s_, flush=True)   # noqa: E731
    t0 = time.perf_counter()
    sets, solves, shells = [], [], {}
    cells = [(2, [float(x) for x in a.energies.split(",") if x], a.maxit, 0, a.bands, a.nconv, a.snap_every, 0.0)]
    if a.energies3:
        cells.append((3, [float(x) for x in a.energies3.split(",") if x], a.maxit3, 1, a.bands3, a.nconv3,
                      a.snap_every3, a.ref_ratio3))
    for cfg, energies, maxit, precision, nb, nconv, snap_every, ref_ratio in cells:
        prob = synth.config(cfg)
        ctx = pw.Context.from_problem(prob, max_bands=nb, flags=pw.PW_PREP_C128 | pw.PW_PREP_C64)
        tabs, tband, er, sol = harvest(ctx, prob, energies, a.start_seed + 10 * (cfg - 2), nb, nconv,
                                       snap_every, a.nsnap, maxit, a.weight_delta, log=log, precision=precision,
                                       cfg_id=cfg, ref_ratio=ref_ratio)
        sets.append((torch.from_numpy(ctx.shells()[1]).to("cuda"), tabs, tband, er))
        solves += sol
        shells[prob.name] = ctx.nshell
        ecut = prob.ecut
        ctx.close()
    t_harvest = time.perf_counter() - t0
    shell_t, tabs, tband, er = merge(sets)
    log(f"harvested {tabs.shape[0]} snapshots over {shells} shells in {t_harvest:.1f} s")
    w, hist, t_train = train(shell_t, tabs, tband, er, ecut, a.steps, a.lr, log=log)
    log(f"trained {a.steps} Adam steps in {t_train:.1f} s: loss {hist[0]:.4f} -> {hist[-1]:.4f}")
    os.makedirs(a.out, exist_ok=True)
    np.save(os.path.join(a.out, WEIGHTS + ".npy"), w.cpu().numpy())
    meta = {"workloads": list(shells), "bands": {"wire256": a.bands, "wire2000": a.bands3},
            "nconv": {"wire256": a.nconv, "wire2000": a.nconv3}, "harvest_solves": solves,
            "samples": {"snapshots": int(tabs.shape[0]), "shells": shells, "bands": int(tabs.shape[3])},
            "harvest_seconds": round(t_harvest, 2), "train_steps": a.steps, "lr": a.lr,
            "weight_delta": a.weight_delta,
            "train_seconds": round(t_train, 2), "loss_first": float(hist[0]), "loss_last": float(hist[-1]),
            "loss_every_20": [round(float(x), 5) for x in hist[::20]],
            "command": "python -m paper_1907_06821_amd.train_precond " + " ".join(argv or sys.argv[1:])}
    with open(os.path.join(a.out, WEIGHTS + ".json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps({k: meta[k] for k in ("harvest_seconds", "train_seconds", "loss_first", "loss_last")}))


if __name__ == "__main__":
    main()
