"""Write config2_trajectory.json: the FP64 oracle's KL trajectories on the full
N=1024 T=8192 R=64 workload (Gamma(0.5) factors, 30%-dense H0, Poisson counts
at mean 5; data seed 1302, init seed 2302).

  dna_floor / dna_nofloor: eq. (1) after each of 200 DNA iterations (Algorithm 1,
      step 1 first), with the float32 value floor FLT_MIN on every updated entry
      and without it (the paper's method on the positive reals);
  mu_floor: eq. (1) after each of 1000 MU iterations (the MU-labelled steps of
      Algorithm 1) with the value floor; its last value is the target KL the
      benchmark's time-to-target figure uses.

Only oracle/ and the seeded input recipe are called; nothing here touches the
HIP path.  Run from the repository root:

    python tests/golden/make_config2_trajectory.py [dna|mu|all]

(about 15 minutes per part on 8 cores; the parts can run in parallel and merge
into the same file).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1301_3389_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config2_trajectory.json")
FLOOR32 = float(np.finfo(np.float32).tiny)


def _merge(update):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    data.update(update)
    data["what"] = ("FP64 oracle KL trajectories on the N=1024 T=8192 R=64 workload "
                    "(data seed 1302, init seed 2302)")
    data["citation"] = ("eq. (1) cost after each iteration of Algorithm 1 (DNA: steps 1-29; "
                        "MU: its MU-labelled steps), Sec. 4 parameters eps = 0.01, alpha = 4")
    data["generator"] = "tests/golden/make_config2_trajectory.py (calls oracle.fit_dna / oracle.fit_mu only)"
    with open(OUT + ".tmp", "w") as f:
        json.dump(data, f, indent=1)
    os.replace(OUT + ".tmp", OUT)


def main(part):
    w = synth.config2()
    if part in ("dna", "all"):
        t = time.time()
        a = oracle.fit_dna(w.V, w.W, w.H, 200, value_floor=FLOOR32)
        b = oracle.fit_dna(w.V, w.W, w.H, 200, value_floor=0.0)
        _merge({"dna_floor": [float(x) for x in a.kl], "dna_nofloor": [float(x) for x in b.kl],
                "dna_newton_frac_h": [float(x) for x in a.newton_frac_h],
                "dna_seconds": time.time() - t})
    if part in ("mu", "all"):
        t = time.time()
        m = oracle.fit_mu(w.V, w.W, w.H, 1000, value_floor=FLOOR32)
        _merge({"mu_floor": [float(x) for x in m.kl], "mu_seconds": time.time() - t})


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "all")
