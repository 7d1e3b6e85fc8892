"""Write tests/golden/c4_ace.json: the oracle's ACE build of every system of the uneven
64-molecule workload (``synth.config4()``, seed 104; box edges 32-64, h 0.25, 2-16 complex
orbitals): per system the exchange energy E_x = 1/2 tr M, the Hermitised M = dV Phi^H W
(Sec. 3.1, the steps after Eq. (11)), and xi = W L^{-H} (Eq. (12)) at eight seeded grid
points of every orbital.

Computed by ``oracle.exchange`` only (FP64, numpy/scipy FFTs); takes a few minutes.

    python tests/golden/make_c4_golden.py
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import exchange, poisson  # noqa: E402

SAMPLES = 8


def sample_points(index, ng):
    """Grid points (flat indices) at which xi is stored for system ``index``."""
    return np.random.default_rng(7000 + index).integers(0, ng, size=SAMPLES)


def main():
    t0 = time.time()
    mols = synth.config4()
    khats = {}
    systems = []
    for i, m in enumerate(mols):
        if m.n not in khats:
            khats[m.n] = poisson.kernel_hat(m.n, m.h)
        xi, mm, _, ex = exchange.ace_build(m.phi, m.h, khats[m.n])
        pts = sample_points(i, m.n ** 3)
        xs = xi.reshape(xi.shape[0], -1)[:, pts]
        systems.append({"index": i, "n": m.n, "h": m.h, "norb": int(m.phi.shape[0]), "ex": ex,
                        "m_re": mm.real.tolist(), "m_im": mm.imag.tolist(),
                        "points": [int(p) for p in pts],
                        "xi_re": xs.real.tolist(), "xi_im": xs.imag.tolist()})
        print(i, m.n, m.phi.shape[0], "%.12f" % ex, "%.0f s" % (time.time() - t0), flush=True)
    out = {"source": "oracle.exchange.ace_build on synth.config4()", "systems": systems,
           "seconds": time.time() - t0}
    with open(os.path.join(HERE, "c4_ace.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
