"""Writes adjoint_crop_48x32x256.json: the FP64 oracle's loss and adjoint
gradient on the adjoint correctness crop (tests/adjoint_case.py, CROP), and
central finite differences of the oracle's forward loss (relative step 1e-4
of the bin's own modulus) for four of its parameters.  Calls only the
oracle; takes about 15 minutes on 8 host threads.

    python tests/golden/make_adjoint_crop.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import adjoint_case as C  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "adjoint_crop_48x32x256.json")
# (modulus, bin) pairs checked by central differences: the two largest
# shear sensitivities near the top and mid-ramp, two bulk ones
FD_PARAMS = (("mu", 1), ("mu", 17), ("K", 2), ("K", 8))
REL_STEP = 1e-4


def main():
    case = C.CROP
    t0 = time.time()
    o, dt = C.oracle_sim(C.medium(case=case), case=case)
    L, gm, gk = o.gradient(case.steps, case.window, case.region)
    del o
    print("gradient: %.1f s, loss %.17g" % (time.time() - t0, L), flush=True)
    mu_b, K_b = C.bin_moduli(case)
    nb = case.region[3]

    def loss(dmu, dK):
        o, _ = C.oracle_sim(C.medium(dmu, dK, case=case), dt, case=case)
        tr = o.run(case.steps)
        return float((tr[:, case.window[0]:case.window[1]] ** 2).sum())

    fds = []
    for name, b in FD_PARAMS:
        e = np.zeros(nb)
        z = np.zeros(nb)
        e[b] = REL_STEP * (mu_b[b] if name == "mu" else K_b[b])
        if name == "mu":
            lp, lm = loss(e, z), loss(-e, z)
        else:
            lp, lm = loss(z, e), loss(z, -e)
        fd = (lp - lm) / (2.0 * e[b])
        fds.append({"modulus": name, "bin": b, "step": e[b], "loss_plus": lp, "loss_minus": lm, "fd": fd})
        print("%s bin %d: fd %.10e adjoint %.10e" % (name, b, fd, (gm if name == "mu" else gk)[b]), flush=True)
    doc = {
        "what": "FP64 oracle on the adjoint correctness crop: loss = sum over steps n in the window and the "
                "axis pressure receivers of p(t_{n+1})^2; dL/dmu and dL/dK (K = lambda + 2 mu / 3) of the "
                "64 one-row bins of the cement annulus below the top; central differences of the oracle's "
                "forward loss with a step of 1e-4 of the bin's own modulus",
        "written_by": "tests/golden/make_adjoint_crop.py (calls only the oracle)",
        "case": {"shape": list(case.shape), "h": case.h, "radii": list(case.radii), "ktop": case.ktop,
                 "ramp": case.ramp, "steps": case.steps, "window": list(case.window),
                 "region": list(case.region), "npml": case.npml, "f0": case.f0, "src_k": case.src_k,
                 "rec_k": list(case.rec_k)},
        "dt": dt,
        "loss": L,
        "dL_dmu": list(gm),
        "dL_dK": list(gk),
        "bin_mu": list(mu_b),
        "bin_K": list(K_b),
        "finite_differences": fds,
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote %s in %.0f s" % (OUT, time.time() - t0))


if __name__ == "__main__":
    main()
