"""Write step_nl_1024_2000.json: the oracle's state after 2000 step attempts
of the nonlinear 2D model on the 1024^2 synthetic basin (seed 2) under the
variable time-step rule (desired Courant number 0.9, attempts above 1.0
rejected and retried with dt * 0.9 / cfl, no output time), from the initial
state of the 1 m elliptical source and the first step dt0.

Stored: accepted and rejected counts, the final time and next dt (exact
hex), a SHA-256 of each final plane (h, hu, hv as little-endian float64,
row-major), each plane's largest magnitude, and 1024 sampled cells (seeded
positions) with their exact values.  Calls only the oracle; takes several
minutes on a few cores.  Run from the repository root:
    python tests/golden/make_step_nl_1024_2000.py
"""
import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O                      # noqa: E402
from paper_1605_05320_amd import inputs as I        # noqa: E402

N, SEED, ATTEMPTS, N_SAMPLES = 1024, 2, 2000, 1024
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "step_nl_1024_2000.json")


def main():
    b = I.basin(N, SEED)
    g = O.Grid(N, N, b.grid.dx, b.grid.dy)
    p = O.Params()
    q = O.init_state(g, p, O.NONLINEAR, b.B, b.eta0)
    dt = O.dt0(g, p, O.NONLINEAR, b.B, *q)
    t, acc, rej = 0.0, 0, 0
    for a in range(ATTEMPTS):
        h, hu, hv, cfl, _ = O.swe_step(g, p, b.B, *q, dt)
        if cfl > p.cfl_max:
            rej += 1
            dt = dt * p.cfl_desired / cfl
            continue
        acc += 1
        q = [h, hu, hv]
        t = t + dt
        if cfl > 0.0:
            dt = dt * p.cfl_desired / cfl
        if (a + 1) % 100 == 0:
            print(f"{a + 1} attempts, t = {t:.3f} s", flush=True)
    rng = np.random.default_rng(7)
    jj = rng.integers(0, N, N_SAMPLES)
    ii = rng.integers(0, N, N_SAMPLES)
    out = {
        "workload": "nonlinear 2D step, 1024x1024 basin seed 2, 2000 controlled attempts from the initial state",
        "accepted": acc, "rejected": rej, "t": t.hex(), "dt_next": dt.hex(),
        "sha256": [hashlib.sha256(np.ascontiguousarray(x, dtype="<f8").tobytes()).hexdigest() for x in q],
        "max_abs": [float(np.abs(x).max()).hex() for x in q],
        "max_abs_eta": float(np.abs(q[0] + b.B).max()).hex(),
        "samples": {"j": jj.tolist(), "i": ii.tolist(),
                    "values": [[float(x[j, i]).hex() for j, i in zip(jj, ii)] for x in q]},
    }
    with open(OUT, "w") as f:
        json.dump(out, f)
    print(f"wrote {OUT}: {acc} accepted, {rej} rejected, t = {t}")


if __name__ == "__main__":
    main()
