"""Write the oracle's full Tamm-Dancoff coupling block of the 64^3 workload (16 occupied + 32
virtual real orbitals, ``synth.config3()``, seed 103):

* tests/golden/c3_coupling_singlet.npy -- C_{ia,jb} = 2 (ai|jb) - (ab|ji) (Eq. (7) without the
  diagonal), 512 x 512 float64, row ia = i * 32 + a;
* tests/golden/c3_eigen.json           -- the eigenvalues of A = diag(eps_a - eps_i) + C
  (Sec. 2, A X = omega X), ascending, in hartree.

Computed by ``oracle.tda`` only (FP64, numpy/scipy FFTs); takes a few minutes.

    python tests/golden/make_c3_golden.py
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import poisson, tda  # noqa: E402


def main():
    t0 = time.time()
    m = synth.config3()
    khat = poisson.kernel_hat(m.n, m.h)
    c = tda.coupling_block(m.phi, m.phi_virt, m.h, 2, khat)
    a = tda.tda_matrix(c, m.eps_occ, m.eps_virt)
    w, _ = tda.excitations(a)
    np.save(os.path.join(HERE, "c3_coupling_singlet.npy"), np.ascontiguousarray(c))
    out = {"source": "oracle.tda.coupling_block / tda_matrix / excitations on synth.config3()",
           "n": m.n, "h": m.h, "n_occ": int(m.phi.shape[0]), "n_virt": int(m.phi_virt.shape[0]),
           "delta_M": 2, "eigenvalues_ha": [float(x) for x in w],
           "ipa_ha": [float(x) for x in tda.ipa_excitations(m.eps_occ, m.eps_virt)],
           "seconds": time.time() - t0}
    with open(os.path.join(HERE, "c3_eigen.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("lowest", out["eigenvalues_ha"][:4], "max |C|", float(np.max(np.abs(c))),
          "%.0f s" % out["seconds"])


if __name__ == "__main__":
    main()
