"""Writes dalitz_fits.json: the oracle's fits of the Dalitz-amplitude model
and of the time-dependent Dalitz model (x = 0, and with x free) to 10^5 seeded events each,
from the models' start values (every coefficient's magnitude and phase
moved from the truth by 10 % and 10 degrees, seed 7).  Calls only the
oracle and the seeded input generators; the GPU tests fit the same events
and compare.

    python tests/golden/make_dalitz_fits.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

from helpers import gen_data, oracle_model  # noqa: E402

# (workload, events, seed of the events)
FITS = [("c3", 100_000, 31), ("c4", 100_000, 41), ("c4x", 100_000, 43)]


def main():
    out = {"citation": "Fits of the paper's Dalitz-plot workload class (section 'Results': Dalitz fits "
                       "with a coherent sum of Breit-Wigner amplitudes, and the time-dependent fit), "
                       "done by the oracle (plain FP64, scipy L-BFGS-B then Newton polishing to "
                       "EDM < 1e-12) on seeded synthetic events; theta and errors = sqrt(diag(H^-1)).",
           "fits": {}}
    for name, n, seed in FITS:
        t0 = time.time()
        om = oracle_model(name)
        data = gen_data(name, n, seed)
        r = om.fit(data)
        out["fits"][name] = {"n_events": n, "seed": seed, "theta": r["theta"].tolist(),
                             "errors": r["errors"].tolist(), "nll": r["nll"], "edm": r["edm"],
                             "start": om.theta().tolist()}
        print(f"{name}: nll {r['nll']:.10f} edm {r['edm']:.2e} in {time.time() - t0:.1f} s", flush=True)
    with open(os.path.join(HERE, "dalitz_fits.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
