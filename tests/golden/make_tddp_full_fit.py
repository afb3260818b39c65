"""Writes tddp_full_fit.json: the oracle's fit of the full time-dependent
model (16 complex amplitudes, tau, y, x, complex q/p, the masses and widths
of two resonances: 39 parameters; the test-size variant of helpers.
full_fit_spec) to 5 x 10^4 seeded accept-reject events from its start
values.  Calls only the oracle and the seeded input generators; the GPU
test fits the same events and compares.

    python tests/golden/make_tddp_full_fit.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

from helpers import gen_data, oracle_model, spec  # noqa: E402

NAME, N_EVENTS, SEED = "c4f_fit", 50_000, 47


def main():
    t0 = time.time()
    om = oracle_model(NAME)
    data = gen_data(NAME, N_EVENTS, SEED)
    print(f"generated {N_EVENTS} events in {time.time() - t0:.1f} s", flush=True)
    r = om.fit(data)
    out = {"citation": "Fit of the full time-dependent model of section 'Results' (the mixing fit's "
                       "16 complex amplitudes, mixing parameters, complex q/p and floating resonance "
                       "shapes) done by the oracle (plain FP64, scipy L-BFGS-B then Newton polishing "
                       "to EDM < 1e-12) on seeded synthetic events; errors = sqrt(diag(H^-1)).",
           "fit": {"name": NAME, "n_events": N_EVENTS, "seed": SEED, "theta": r["theta"].tolist(),
                   "errors": r["errors"].tolist(), "nll": r["nll"], "edm": r["edm"],
                   "start": om.theta().tolist(), "par_names": [p[0] for p in spec(NAME)["params"]]}}
    print(f"nll {r['nll']:.10f} edm {r['edm']:.2e} in {time.time() - t0:.1f} s", flush=True)
    with open(os.path.join(HERE, "tddp_full_fit.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
