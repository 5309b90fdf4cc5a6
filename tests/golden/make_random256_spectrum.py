"""Writes random256_d8_spectrum_edge.txt: the 20 eigenvalues of the random dense Lindbladian
(n = 256, d = 8, seed 0) nearest the shift mu = -0.67, computed by the oracle's own Algorithm
"Low-lying spectrum via shift-invert Arnoldi" (oracle.krylov.low_spectrum: ARPACK on
(mu - L~_eta)^{-1}, each application a right-preconditioned GMRES solve), with each pair's
eigen-residual.  Calls only oracle/ and lind_inputs (seeded input); run from the repository root:

    python tests/golden/make_random256_spectrum.py

The shift sits about 0.1 to the right of the spectrum's edge (rightmost eigenvalue near -0.769):
there the low edge of this family is a dense cluster (|lambda| within 1e-2 of each other), which a
shift at 0 cannot separate in reasonable time; the eigenvalues nearest this shift include the ten
of smallest modulus."""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import lind_inputs as li  # noqa: E402
from oracle import krylov as ok  # noqa: E402

N, D, SEED, K, MU = 256, 8, 0, 20, -0.67


def main():
    H, Ls = li.random_dense(N, D, SEED)
    t0 = time.time()
    lam, vecs = ok.low_spectrum(H, Ls, K, mu=MU, tol=1e-10, inner_tol=1e-11)
    res = [ok.eigen_residual(H, Ls, l, v) for l, v in zip(lam, vecs)]
    order = np.argsort(np.abs(lam - MU))
    lam = lam[order]
    res = np.array(res)[order]
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "random256_d8_spectrum_edge.txt")
    with open(out, "w") as f:
        f.write("# Random dense Lindbladian n = 256, d = 8, seed 0 (lind_inputs.random_dense): the 20\n")
        f.write("# eigenvalues nearest mu = -0.67 by the oracle's shift-invert Arnoldi (Algorithm\n")
        f.write("# \"Low-lying spectrum via shift-invert Arnoldi\", Section 4.2), ordered by |lambda - mu|;\n")
        f.write("# written by tests/golden/make_random256_spectrum.py (oracle only).\n")
        f.write(f"# oracle time {time.time() - t0:.0f} s; max eigen-residual (max-norm) {max(res):.2e}\n")
        f.write(f"mu = {MU}\n")
        f.write("eigs_re = " + " ".join(f"{z.real:.15e}" for z in lam) + "\n")
        f.write("eigs_im = " + " ".join(f"{z.imag:.15e}" for z in lam) + "\n")
        f.write("residual_max = " + " ".join(f"{r:.3e}" for r in res) + "\n")
    print("wrote", out)


if __name__ == "__main__":
    main()
