"""Long oracle run of a 16^3 pasta slab box (80 n + 20 p), with or without
extra unoccupied states: the record behind the residual plateau of the
damped-gradient iteration on pasta starts.  Test infrastructure, like the
rest of this package; it runs the FP64 oracle only.

    python -m oracle.run_plateau EXTRA ITERATIONS

prints every 25th iteration: iteration, Delta-eps, total energy, seconds.
"""
import sys
import time

from oracle import Grid
from oracle import solver as so
from paper_1610_07522_amd import inputs


def main():
    extra = int(sys.argv[1])
    iters = int(sys.argv[2])
    w = inputs.Workload("slab16", 16, 1.0, 80, 20, "slab", seed=1, extra_n=extra,
                        extra_p=extra)
    rn, rp = inputs.raw_states(w)
    g = Grid(16, 1.0)
    st = so.initial_state(rn, rp, g, w.params, w.damp_x0, w.damp_e0, nocc=(80, 20))
    t0 = time.time()
    for it in range(1, iters + 1):
        rep = so.iterate(st)
        if it % 25 == 0 or rep.de < 1e-6:
            print(it, f"{rep.de:.4e}", f"{rep.E['total']:.10f}", f"{time.time() - t0:.0f}s",
                  flush=True)
        if rep.de < 1e-7:
            break


if __name__ == "__main__":
    main()
