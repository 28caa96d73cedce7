"""Write the reference interval and eigenvalues for the 3D 7-point workload.

Workload: 7-point Laplacian on a 100^3 Dirichlet grid plus a diagonal
potential V_i ~ U[0,1) (PCG64 seed 240915053 + 2), block r = 8.  The
interval holds the lowest ~100 eigenvalues; its upper end is put at the
midpoint of the widest gap among eigenvalues 95..105 (endpoints must sit
well away from eigenvalues).  Everything here is computed by the CPU
oracle only:

    python tests/golden/make_c2_reference.py [N]

writes tests/golden/c2_lap3d7_<N>_U01.json.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import flp_oracle as O  # noqa: E402
from paper_2409_15053_amd import inputs as I  # noqa: E402


def main():
    N = int(sys.argv[1]) if len(sys.argv) > 1 else 100
    target = 100
    w = I.workload_c2(N)
    A = w["A"]
    t0 = time.time()
    g = np.random.Generator(np.random.PCG64(w["seed"]))
    lmin, lmax = O.spectrum_bounds(A, g.standard_normal(A.n))
    print(f"n={A.n} nnz={A.nnz} bounds=[{lmin:.6f}, {lmax:.6f}] ({time.time() - t0:.1f}s)", flush=True)
    # pre-pass: a generous low-end window
    beta0 = 0.56
    res = O.flp_solve(A, 0.0, beta0, block=w["block"], degree=60, seed=w["seed"], bounds=(lmin, lmax))
    ev = np.sort(res.evals)
    print(f"pre-pass: {len(ev)} eigenvalues in [0, {beta0}] iters={res.iters} "
          f"max resid={res.resid.max():.2e} ({time.time() - t0:.1f}s)", flush=True)
    assert len(ev) > target + 6, "widen the pre-pass window"
    idx = np.arange(target - 6, target + 5)  # gaps after eigenvalue 95..105 (1-based)
    gaps = ev[idx + 1] - ev[idx]
    k = int(idx[np.argmax(gaps)])
    beta = 0.5 * (ev[k] + ev[k + 1])
    alpha = 0.0
    count = k + 1
    # final run on the chosen interval, reference eigenvalues
    res2 = O.flp_solve(A, alpha, beta, block=w["block"], degree=100, seed=w["seed"] + 1, bounds=(lmin, lmax))
    ev2 = np.sort(res2.evals)
    assert len(ev2) == count, (len(ev2), count)
    assert np.max(np.abs(ev2 - ev[:count]) / ev[:count]) < 1e-10
    out = dict(
        workload=w["name"], n=A.n, nnz=A.nnz, block=w["block"], seed=w["seed"],
        alpha=alpha, beta=beta, count=count, gap_at_beta=float(ev[k + 1] - ev[k]),
        lmin_oracle=lmin, lmax_oracle=lmax, evals=ev2.tolist(),
        max_resid=float(res2.resid.max()), oracle_iters=res2.iters, degree=100,
        made_by="tests/golden/make_c2_reference.py (CPU oracle only)",
    )
    path = os.path.join(HERE, f"c2_lap3d7_{N}_U01.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path}: count={count} beta={beta:.9f} ({time.time() - t0:.1f}s)", flush=True)


if __name__ == "__main__":
    main()
