"""The router's error-budget arithmetic on the CPU: the running error
statistics of a family against numpy on the same samples, and the admitted
set against a brute-force search over the prefixes of the families ordered
by their error bound."""
import itertools
import math

import numpy as np
import pytest

pytest.importorskip("torch")
from paper_2301_08343_amd.router import FamilyError, admit  # noqa: E402


def test_family_error_pools_prior_statistics_and_audits():
    rng = np.random.default_rng(3)
    prior = rng.gamma(0.7, 30.0, size=101)
    audits = rng.gamma(0.7, 40.0, size=37)
    e = FamilyError(n=len(prior), mean=prior.mean(), sd=prior.std())
    for a in audits:
        e.add(float(a))
    both = np.concatenate([prior, audits])
    assert e.n == len(both)
    assert math.isclose(e.mean(), both.mean(), rel_tol=1e-12)
    z = 1.645
    assert math.isclose(e.upper(z), both.mean() + z * both.std() / math.sqrt(len(both)), rel_tol=1e-10)
    # no samples: unknown error, never admitted
    assert FamilyError().upper(z) == math.inf
    assert admit({0: math.inf, 1: 1.0}, {0: 0.5, 1: 0.5}, 25.0) == {1}


def brute_force(bounds, shares, limit_sq):
    order = sorted(bounds, key=lambda f: (bounds[f], f))
    best = set()
    for k in range(len(order) + 1):
        run = order[:k]
        w = sum(shares[f] for f in run)
        if any(not math.isfinite(bounds[f]) for f in run):
            break
        if w > 0 and sum(shares[f] * bounds[f] for f in run) > limit_sq * w:
            break
        best = set(run)
    return best


@pytest.mark.parametrize("seed", range(40))
def test_admitted_set_is_the_longest_prefix_within_the_budget(seed):
    rng = np.random.default_rng(seed)
    nf = int(rng.integers(1, 7))
    bounds = {f: float(rng.gamma(0.8, 30.0)) for f in range(nf)}
    shares = rng.dirichlet(np.ones(nf))
    shares = {f: float(shares[f]) for f in range(nf)}
    got = admit(bounds, shares, 25.0)
    assert got == brute_force(bounds, shares, 25.0)
    if got:
        w = sum(shares[f] for f in got)
        assert sum(shares[f] * bounds[f] for f in got) <= 25.0 * w * (1 + 1e-12)
    # every admitted family's bound is below every excluded one's
    for a, b in itertools.product(got, set(bounds) - got):
        assert bounds[a] <= bounds[b]


def test_budget_of_the_committed_families():
    """Held-out bounds shaped like the committed network's (sphere and cone
    under 1 um^2, cylinder and edge near 30, the textured plate far above):
    the first four fit the 5 um budget together, the plate does not."""
    bounds = {0: 0.6, 1: 31.0, 2: 0.4, 3: 34.0, 4: 560.0}
    shares = {f: 0.2 for f in bounds}
    assert admit(bounds, shares, 25.0) == {0, 1, 2, 3}
    # a smaller budget drops the larger of the two middle bounds first
    assert admit(bounds, shares, 16.0) == {0, 1, 2}


def test_query_class_splits_families_by_depth():
    """Classes are the family alone without edges; with edges, family *
    (bins) + the bin of the press depth (a depth on an edge falls in the
    upper bin)."""
    from paper_2301_08343_amd.router import query_class
    q = lambda fam, depth: {"cfg": {"shape": fam}, "depth": depth}  # noqa: E731
    edges = (0.6e-3, 1.0e-3)
    assert query_class(q(3, 0.9e-3)) == 3
    assert [query_class(q(0, d), edges) for d in (0.2e-3, 0.6e-3 - 1e-9, 0.6e-3, 1.2e-3)] == [0, 0, 1, 2]
    assert query_class(q(4, 1.5e-3), edges) == 14
    assert query_class(q(2, 0.7e-3), edges) == 7
