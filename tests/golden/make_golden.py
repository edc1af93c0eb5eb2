"""Write the expected values of the full-length two-transmon CNOT workload.

Calls only the CPU oracle (and the seeded input generator); nothing here
touches the HIP library.  Run from the repository root:

    python tests/golden/make_golden.py

Output: tests/golden/c2_cnot_full.npz with rho(T) of the 16 basis states,
the objective G and its gradient (shape [Q, Ns, Nf, 2]).  Takes a few
minutes on one core.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import make_config  # noqa: E402


def main():
    p = make_config(2)
    s = p.systems[0]
    t0 = time.time()
    G, grad, rhoT = oracle.value_and_gradient(s, p.alpha[0], p.rho0[0], p.rhotar[0], p.beta[0],
                                              p.kind, p.gamma2, return_final=True)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_cnot_full.npz")
    np.savez_compressed(out, rhoT=rhoT, G=np.array(G), grad=grad,
                        seed=np.array(20211020 + 2), NT=np.array(s.NT))
    print(f"wrote {out}: G={G:.16e} |grad|max={np.abs(grad).max():.6e} in {time.time() - t0:.1f}s")


if __name__ == "__main__":
    main()
