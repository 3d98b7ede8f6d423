"""Write the dense-oracle reference eigenvalues of the larger workloads.

Calls only ``synth`` (seeded inputs) and ``oracle.dense`` (the structure-
preserving dense eigensolver, pinned by tests/test_oracle_pins.py).  The
files hold the nev smallest positive eigenvalues of H, one per line, with
17 significant digits:

    python tests/golden/make_dense_reference.py 1 3
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from synth import config_problem  # noqa: E402
from oracle import dense  # noqa: E402


def main(cfgs):
    for c in cfgs:
        p = config_problem(int(c), seed=0)
        t = time.time()
        lam, _ = dense.dense_ph_eig(p.A, p.B)
        out = os.path.join(HERE, f"dense_evals_config{c}_seed0.txt")
        with open(out, "w") as f:
            f.write(f"# {p.name}: m={p.m}, nev={p.nev}; nev+nex+8 smallest positive eigenvalues of H\n")
            f.write("# written by tests/golden/make_dense_reference.py (oracle.dense.dense_ph_eig)\n")
            for v in lam[: p.nev + p.nex + 8]:
                f.write(f"{v:.17e}\n")
        print(out, f"{time.time() - t:.1f}s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["1", "3"])
