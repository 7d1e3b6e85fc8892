"""Write tests/golden/scf_small.json: converged closed-shell HF energies and orbital energies
of the synthetic two-nucleus system ``synth.scf_small()``, computed by the FP64 oracle only
(states mixing alpha = 0.3, relative density error below 1e-10).

    python tests/golden/make_scf_golden.py
"""

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import scf  # noqa: E402


def main():
    s = synth.scf_small()
    phi, e, hist = scf.scf(s.guess, s.v_ext, s.h, alpha=0.3, tol=1e-10, max_iter=400)
    out = {"source": "oracle.scf.scf on synth.scf_small(), alpha 0.3, tol 1e-10",
           "n": s.n, "h": s.h, "iterations": len(hist),
           "density_error": hist[-1]["density_error"],
           "eigenvalues": [float(x) for x in hist[-1]["eigenvalues"]],
           "energy": e}
    with open(os.path.join(HERE, "scf_small.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
