"""Writes hw_spectra.json: the extreme |eigenvalues| of H_W = g5 D_W(-rho) for
the seeded synthetic gauge fields the overlap GPU tests use, computed by the
FP64 oracle alone (ARPACK on H_W^2, oracle.overlap.hw_extremes).  The GPU
tests take their Chebyshev interval [0.9 lmin^2, 1.1 lmax^2] from here, so it
comes from the oracle's spectrum, not from the library's own Lanczos.

    python tests/golden/make_hw_spectra.py      (about six minutes on one core)
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import overlap as OV  # noqa: E402

# (extents, link spread eps, gauge seed, rho)
CASES = [((4, 4, 4, 4), 0.2, 311, 1.5), ((4, 4, 4, 6), 0.2, 321, 1.5), ((8, 8, 8, 8), 0.2, 301, 1.5)]


def key(L, eps, seed, rho):
    return f"{'x'.join(map(str, L))}_eps{eps}_seed{seed}_rho{rho}"


def main():
    out = {"_source": "oracle.overlap.hw_extremes (ARPACK, tol 1e-8) on synth.su3_field(L, eps, seed)"}
    for L, eps, seed, rho in CASES:
        U = synth.su3_field(L, eps, seed)
        lo, hi = OV.hw_extremes(U, rho, tol=1e-8)
        out[key(L, eps, seed, rho)] = {"L": list(L), "eps": eps, "seed": seed, "rho": rho, "lmin": lo, "lmax": hi}
        print(key(L, eps, seed, rho), lo, hi, flush=True)
    with open(os.path.join(HERE, "hw_spectra.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
