"""Write the oracle fixture of the 32^3 pasta slab box (640 n + 160 p).

Runs only the FP64 oracle (oracle/) on the seeded trial states of
paper_1610_07522_amd.inputs (workload "slab32") and stores, after
iterations 1, 10 and 100 of Fig. 1 steps 2-5, the energy parts, Delta-eps
(Eq. convergence), the ascending subspace eigenvalues of both species and
the densities rho, tau of both species on a fixed sample of grid points.

    python tests/golden/make_slab32.py [max_iter]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import Grid  # noqa: E402
from oracle import solver as so  # noqa: E402
from paper_1610_07522_amd import inputs  # noqa: E402

KEEP = (1, 10, 100)


def sample_points(n, count=256, seed=5):
    rng = np.random.default_rng(seed)
    return rng.integers(0, n, size=(count, 3))


def main():
    max_iter = int(sys.argv[1]) if len(sys.argv) > 1 else max(KEEP)
    w = inputs.WORKLOADS["slab32"]
    rn, rp = inputs.raw_states(w)
    g = Grid(w.n, w.dx)
    st = so.initial_state(rn, rp, g, w.params, w.damp_x0, w.damp_e0)
    pts = sample_points(w.n)
    out = dict(workload="slab32", points=pts.tolist(), iterations={})
    path = os.path.join(HERE, "slab32_oracle.json")
    t0 = time.time()
    for it in range(1, max_iter + 1):
        rep = so.iterate(st)
        print(f"iteration {it}: de={rep.de:.6e} E={rep.E['total']:.12f} "
              f"({time.time() - t0:.0f} s)", flush=True)
        if it in KEEP:
            z, y, x = pts[:, 2], pts[:, 1], pts[:, 0]
            out["iterations"][str(it)] = dict(
                de=rep.de, energy=rep.E,
                ritz=[r.tolist() for r in rep.ritz],
                rho=[d.rho[z, y, x].tolist() for d in st.dens],
                tau=[d.tau[z, y, x].tolist() for d in st.dens])
            with open(path, "w") as f:
                json.dump(out, f, separators=(",", ":"))


if __name__ == "__main__":
    main()
