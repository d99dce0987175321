"""The seeded input recipe against the ranges the paper prints (Table I, Sec.
III A), stored in tests/golden/table1_priors.json.  psi is drawn in [0, pi):
the antenna patterns have period pi in psi, so this is the same distribution
of F+ and Fx as Table I's [0, 2 pi]."""
import json
import math
import os

import numpy as np
from scipy import stats

from paper_2508_04172_amd import workloads as wl

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1_priors.json")))


def _within(v, rng):
    return np.all(v >= rng[0]) and np.all(v <= rng[1])


def test_event_generator_masses_and_spins():
    ev = wl.ragged_events(64)
    m1 = np.array([e.inj_phys[0] for e in ev])
    m2 = np.array([e.inj_phys[1] for e in ev])
    c1 = np.array([e.inj_phys[2] for e in ev])
    c2 = np.array([e.inj_phys[3] for e in ev])
    mc = (m1 * m2) ** 0.6 / (m1 + m2) ** 0.2
    assert _within(m1, GOLDEN["m1_msun"]) and _within(m2, GOLDEN["m2_msun"])
    assert _within(mc, GOLDEN["chirp_mass_msun"])
    assert _within(m1 / m2, GOLDEN["mass_ratio"])
    assert _within(c1, GOLDEN["chi1z"]) and _within(c2, GOLDEN["chi2z"])
    assert len({e.seg_len for e in ev}) > 20          # uneven events


def test_query_extrinsics_follow_table1():
    q = wl.queries(wl.CFG2, n=100000)
    alpha, dec, psi, iota, phi = q.ext.T
    assert _within(alpha, GOLDEN["alpha"]["range"]) and _within(phi, GOLDEN["phi_c"]["range"])
    assert _within(dec, GOLDEN["dec"]["range"]) and _within(iota, GOLDEN["iota"]["range"])
    assert _within(psi, [0.0, math.pi])
    two_pi = 2 * math.pi
    for v, cdf in ((alpha / two_pi, "uniform"), (phi / two_pi, "uniform"), (psi / math.pi, "uniform"),
                   ((np.sin(dec) + 1) / 2, "uniform"), ((np.cos(iota) + 1) / 2, "uniform")):
        assert stats.kstest(v, cdf).pvalue > 1e-3
    # distance uniform in volume: (d/d_ref)^3 uniform over [1/8, 8]
    r3 = q.dist_ratio ** 3
    assert stats.kstest((r3 - 0.125) / (8.0 - 0.125), "uniform").pvalue > 1e-3
