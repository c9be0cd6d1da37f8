"""Writes tests/golden/wire256_nearest.json: the eigenvalues of the 256-atom wire
cell nearest E_ref = 0.3 Ha, from the CPU oracle only.

Route (oracle.shift_invert): the dense FP64 H (48,369 plane waves, 37 GB) is
written into one host array; H - E I is factored in place (LDL^H); Lanczos on
(H - E I)^{-1} gives the K eigenpairs nearest E; their Rayleigh quotients and
residuals come from the matrix-free H psi.  Completeness: with r halfway
between the 128th and the 129th distance |lambda - E|, two more factorisations
count the eigenvalues below E - r and below E + r (Sylvester inertia); their
difference must be 128, so the 128 values are exactly the 128 nearest.

Needs about 40 GB of host memory and roughly an hour on 8 cores.  The inputs
(synthetic, seeded) are hashed into the file so a test can tell whether they
still match.  Usage: python tests/golden/make_wire256_nearest.py
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from paper_1907_06821_amd import synth  # noqa: E402  (seeded inputs only)
from oracle.hamiltonian import Operator  # noqa: E402
from oracle.shift_invert import count_below, nearest_by_shift_invert, work_matrix  # noqa: E402

NWANT = 128
K = 140
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "wire256_nearest.json")


def input_hash(prob, vgrid):
    h = hashlib.sha256()
    for a in (vgrid, prob.pos, prob.dproj, np.asarray(prob.cell), np.asarray(prob.grid, dtype=np.float64)):
        h.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    h.update(repr((prob.ecut, prob.width, prob.sigma, prob.nl, prob.e_ref)).encode())
    return h.hexdigest()


def main():
    t0 = time.perf_counter()

    def log(msg):
        print(f"[{time.perf_counter() - t0:8.1f} s] {msg}", flush=True)

    prob = synth.config(2)
    vgrid = prob.vgrid()
    op = Operator.from_problem(prob, vgrid=vgrid)
    e = prob.e_ref
    log(f"wire256: npw {op.npw}, {op.beta.shape[0]} projectors")
    work = work_matrix(op.npw)
    r = nearest_by_shift_invert(op, e, K, work=work, log=log)
    lam = r["lam"]
    order = np.lexsort((lam, np.abs(lam - e)))
    dist = np.abs(lam[order] - e)
    radius = 0.5 * (dist[NWANT - 1] + dist[NWANT])
    log(f"Lanczos: {r['solves']} solves, max residual {r['resid'].max():.2e}; window radius {radius:.6f} Ha")
    lo = count_below(op, e - radius, work=work)
    log(f"below E - r: {lo}")
    hi = count_below(op, e + radius, work=work)
    log(f"below E + r: {hi}")
    nearest = np.sort(lam[order[:NWANT]])
    out = {
        "cell": "wire256 (synth.config(2))",
        "input_sha256": input_hash(prob, vgrid),
        "e_ref": e,
        "npw": int(op.npw),
        "k_lanczos": K,
        "lanczos_solves": int(r["solves"]),
        "eigenvalues_k": lam.tolist(),
        "residuals_k": r["resid"].tolist(),
        "nearest": nearest.tolist(),
        "nwant": NWANT,
        "dist_nwant": float(dist[NWANT - 1]),
        "dist_next": float(dist[NWANT]),
        "window_radius": float(radius),
        "count_below_e": int(r["below"]),
        "count_below_e_minus_r": int(lo),
        "count_below_e_plus_r": int(hi),
        "count_in_window": int(hi - lo),
        "complete": bool(hi - lo == NWANT),
        "seconds": round(time.perf_counter() - t0, 1),
        "source": "oracle.shift_invert: in-place LDL^H of the dense FP64 H, Lanczos on (H - E)^-1, "
                  "Sylvester inertia at E +- r",
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    log(f"wrote {OUT}: complete = {out['complete']}")


if __name__ == "__main__":
    main()
