"""Write grad_c5_L512.txt: the oracle's 3-round area loss on the L = 512,
50-region synthetic map (seeded, see synth.WORKLOADS["c5_L512"]) with
blur widths 4, 2, 1, its adaptive step schedules, and the central-difference
gradient (h = 1e-4) of the loss with respect to the 50 region densities,
schedules frozen.  Calls only the oracle and the input generator.

    python tests/golden/make_grad_c5.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "grad_c5_L512.txt")


def main():
    oracle.build(force=False)
    m = synth.workload("c5_L512")
    sigmas = [oracle.default_sigma(k) for k in range(3)]
    t0 = time.time()
    ref = oracle.rounds(m, m.density, sigmas)
    g = oracle.fd_gradient(m, m.density, sigmas, ref.schedules, step=1e-4)
    with open(OUT, "w") as f:
        f.write("# oracle (FP64) 3-round area loss on c5_L512, sigmas 4 2 1, adaptive\n")
        f.write("# schedules (tol 1e-3, h0 1e-2, safety 0.9, fac 0.2..5), and the central\n")
        f.write("# difference (h = 1e-4) gradient w.r.t. the region densities with the\n")
        f.write("# schedules frozen; written by tests/golden/make_grad_c5.py\n")
        f.write(f"regions {m.n_regions}\n")
        f.write(f"loss {ref.loss:.17e}\n")
        for k, s in enumerate(ref.schedules):
            f.write(f"schedule {k} " + " ".join(f"{h:.17e}" for h in s) + "\n")
        f.write("gradient " + " ".join(f"{v:.17e}" for v in g) + "\n")
    print(f"wrote {OUT} in {time.time() - t0:.1f} s")


if __name__ == "__main__":
    main()
