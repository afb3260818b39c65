"""Statistical pins of the oracle's fit: parameter recovery and pulls on
seeded toys (the method is a maximum-likelihood estimator, so pulls must be
standard normal up to O(1/sqrt(n)) corrections)."""
import numpy as np

import synthgen as S


def test_c1_toy_pulls(oracle_mod):
    m = oracle_mod.Model(S.C1)
    pulls = []
    for i in range(200):
        d = S.gen_c1(n=2000, seed=1000 + i)
        r = m.fit(d)
        pulls.append((r["theta"][0] - S.C1["truth"]["alpha"]) / r["errors"][0])
    pulls = np.array(pulls)
    assert abs(pulls.mean()) < 3 / np.sqrt(200)
    assert abs(pulls.std() - 1) < 0.15


def test_c2_recovers_truth(oracle_mod):
    m = oracle_mod.Model(S.C2)
    d = S.gen_c2(n=200_000, seed=77)
    r = m.fit(d)
    tr = m.theta(S.C2["truth"])
    pull = (r["theta"] - tr) / r["errors"]
    assert np.all(np.abs(pull) < 4), pull
    assert r["edm"] < 1e-8
