"""Write the stored residual histories under tests/golden/ (calls only the oracle).

    python tests/golden/make_golden.py

Each file holds one case: a header line naming it, then rho_0 .. rho_k, the
FP64 L2 residual norms after each V(2,2) cycle.
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import inputs  # noqa: E402
import oracle  # noqa: E402

CASES = {
    # 129 x 129 sine problem, RBGS V(2,2), u0 = 0, ten cycles (the paper's Application runs ten)
    "poisson2d_129_sine_rbgs_10cycles": dict(dim=2, n=129, rhs="sine", smoother=0, omega=1.0, cycles=10),
    "poisson2d_129_sine_jacobi_10cycles": dict(dim=2, n=129, rhs="sine", smoother=1, omega=0.8, cycles=10),
    "poisson3d_33_uniform7_rbgs_10cycles": dict(dim=3, n=33, rhs=("uniform", 7), smoother=0, omega=1.0, cycles=10),
}


def rhs(c):
    if c["rhs"] == "sine":
        return inputs.sine_rhs(c["dim"], c["n"])
    return inputs.uniform_rhs(c["dim"], c["n"], c["rhs"][1])


def history(c):
    f = rhs(c)
    _, hist, _ = oracle.solve(np.zeros_like(f), f, tol=0.0, max_cycles=c["cycles"],
                              smoother=c["smoother"], omega=c["omega"])
    return hist


def main():
    for name, c in CASES.items():
        h = history(c)
        with open(os.path.join(HERE, name + ".txt"), "w") as fh:
            fh.write(f"# {name}: FP64 L2 residual after each V(2,2) cycle, written by make_golden.py (oracle only)\n")
            for v in h:
                fh.write(f"{v:.17e}\n")


if __name__ == "__main__":
    main()
