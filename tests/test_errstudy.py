"""The error-study harness's variance formulas (host only): identities the paper's expressions
must satisfy, and agreement with the oracle's replica variance on a small graph."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import brute
from paper_1811_09136_amd import errstudy


def test_variance_identities():
    tau, eta = 1000.0, 50000.0
    for m in (2, 5, 10):
        # c = m: Theorem 3 reduces to tau (m - 1); c = c1 m: tau (m - 1) / c1 (Section III-B)
        assert errstudy.variance_rept(tau, eta, m, m) == pytest.approx(tau * (m - 1))
        assert errstudy.variance_rept(tau, eta, m, 3 * m) == pytest.approx(tau * (m - 1) / 3)
        # one processor: REPT and MASCOT are the same sampler
        assert errstudy.variance_rept(tau, eta, m, 1) == pytest.approx(errstudy.variance_mascot(tau, eta, m, 1))
        # the covariance term makes parallel MASCOT worse at c = m (Section III-C)
        assert errstudy.variance_mascot(tau, eta, m, m) > errstudy.variance_rept(tau, eta, m, m)
        # c2 != 0: the combination is below both of its parts
        v = errstudy.variance_rept(tau, eta, m, m + 1)
        v1 = tau * (m - 1)
        v2 = (tau * (m * m - 1) + 2 * eta * (m - 1)) / 1
        assert v == pytest.approx(v1 * v2 / (v1 + v2)) and v < min(v1, v2)
    assert errstudy.variance_rept(tau, eta, 1, 1) == 0.0 and errstudy.variance_mascot(tau, eta, 1, 4) == 0.0
    assert errstudy.nrmse(np.array([9.0, 11.0]), 10.0) == pytest.approx(0.1)


@pytest.mark.parametrize("m,c", [(3, 2), (3, 5)])
def test_variance_matches_oracle_replicas(m, c):
    """The harness's formulas against the empirical variance of the oracle's estimators over
    hash seeds (REPT with c <= m and with c mod m != 0, and parallel MASCOT)."""
    n = 30
    e = synth.shuffled(synth.er(n, 160, 41, 42), 43)
    tau, _ = brute.exact_counts(e, n)
    eta = brute.eta(e, n)
    R = 1200
    seeds = errstudy.replica_seeds(5, R)
    rep, mas = np.empty(R), np.empty(R)
    for r, s in enumerate(seeds):
        g, _ = oracle.rept(e, n, m, c, s)
        if c > m:
            et = int(oracle.rept2_eta(e, n, m, c, s)[0].sum())
            rep[r] = oracle.estimate2(n, m, c, g, None, et, None)[0]
        else:
            rep[r] = oracle.estimate(n, m, c, g)[0]
        gm, _ = oracle.mascot(e, n, m, c, s)
        mas[r] = oracle.estimate_mascot(n, m, c, gm)[0]
    vr = errstudy.variance_rept(tau, eta, m, c)
    vm = errstudy.variance_mascot(tau, eta, m, c)
    # the combined estimator's weights are estimated, so its variance sits a little above the
    # ideal combination's
    hi = 1.25 if c <= m else 1.45
    assert 0.8 < np.mean((rep - tau) ** 2) / vr < hi
    assert 0.8 < np.mean((mas - tau) ** 2) / vm < 1.25
    assert abs(mas.mean() - tau) < 4 * math.sqrt(vm / R)
