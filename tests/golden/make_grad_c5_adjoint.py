"""Write grad_c5_L512_adjoint.txt: the reverse-mode (FP64) gradient of the
oracle's 3-round area loss on the L = 512, 50-region synthetic map with blur
widths 4, 2, 1, with respect to the region densities, at the oracle's own
adaptive step schedules (the ones stored in grad_c5_L512.txt; this script
recomputes them and checks that they agree).  Calls only the oracle and the
input generator.

    python tests/golden/make_grad_c5_adjoint.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

import oracle  # noqa: E402
import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "grad_c5_L512_adjoint.txt")


def stored_schedules():
    sched = {}
    with open(os.path.join(HERE, "grad_c5_L512.txt")) as f:
        for line in f:
            t = line.split()
            if t and t[0] == "schedule":
                sched[int(t[1])] = np.array([float(x) for x in t[2:]])
    return [sched[k] for k in sorted(sched)]


def main():
    oracle.build(force=False)
    m = synth.workload("c5_L512")
    sigmas = [oracle.default_sigma(k) for k in range(3)]
    t0 = time.time()
    ref = oracle.rounds(m, m.density, sigmas)
    for a, b in zip(ref.schedules, stored_schedules()):
        assert np.array_equal(a, b), "schedules differ from grad_c5_L512.txt"
    loss, g = oracle.adjoint_gradient(m, m.density, sigmas, ref.schedules)
    assert loss == ref.loss
    with open(OUT, "w") as f:
        f.write("# oracle (FP64) 3-round area loss on c5_L512, sigmas 4 2 1, at the adaptive\n")
        f.write("# schedules of grad_c5_L512.txt, and its reverse-mode gradient w.r.t. the\n")
        f.write("# region densities (steps frozen); written by\n")
        f.write("# tests/golden/make_grad_c5_adjoint.py\n")
        f.write(f"regions {m.n_regions}\n")
        f.write(f"loss {loss:.17e}\n")
        f.write("gradient " + " ".join(f"{v:.17e}" for v in g) + "\n")
    print(f"wrote {OUT} in {time.time() - t0:.1f} s")


if __name__ == "__main__":
    main()
