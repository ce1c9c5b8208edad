"""The data -> training -> router pipeline end to end at a coarse spacing
(0.5 mm lattice, 12,800 particles per contact): it runs, the loss falls, the
router's report is consistent, and the circuit breaker hands everything to
the MPM when its limit cannot be met."""
import json

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_pipeline_small(gpu, tmp_path):
    from paper_2301_08343_amd import surrogate_pipeline as SP
    rc = SP.main(["--train", "512", "--heldout", "64", "--epochs", "6", "--batch", "128", "--queries", "300",
                  "--plain-sample", "64", "--h", "0.5e-3", "--out", str(tmp_path)])
    assert rc == 0
    rep = json.load(open(tmp_path / "report.json"))
    print(json.dumps({k: rep[k] for k in ("data", "heldout", "router", "plain_mpm")}, indent=1))
    assert rep["train"]["loss_curve"][-1] < rep["train"]["loss_curve"][0]
    r = rep["router"]
    assert r["queries"] == 300
    assert r["mpm_fallbacks"] == r["ood"] + r["audited"] + r["breaker_routed"] + r["breaker_rerouted_in_batch"]
    assert r["served_by_surrogate"] + r["mpm_fallbacks"] == 300
    # the served answers' error is measured on a sample spread over the stream
    assert rep["served_sample"]["queries"] >= 32 and rep["served_sample"]["last_index"] >= 200
    # 2% of 300 draws are audited, unless the few-epoch network's held-out
    # error already closes every class (family and depth bin) at the start
    # (then nothing is served by it)
    assert r["audited"] >= 1 or (r["served_by_surrogate"] == 0
                                 and set(r["breaker_tripped_at_start"]) == {int(k) for k in r["per_class"]})
    assert (tmp_path / "surrogate.safetensors").exists()


def test_breaker_routes_everything_to_mpm(gpu, tmp_path):
    """An unreachable accuracy limit trips the breaker at the first audit;
    every later batch goes to the MPM."""
    from paper_2301_08343_amd import dataset as D
    from paper_2301_08343_amd import router as RT
    from paper_2301_08343_amd.surrogate import Net
    net = Net(batch=64, seed=1)
    train = D.contacts_for(range(64), 0.5e-3)
    ftr = RT.features(D.inputs(train))
    qs = D.contacts_for(range(1000, 1096), 0.5e-3)
    r = RT.Router(net, ftr, threshold=1e9, audit_rate=0.5, rmse_limit_um=1e-6, per_class=False)
    ans, rep, route = r.serve(qs, batch=32)
    assert rep["breaker_tripped"] == [0]
    assert rep["breaker_routed"] == 64  # batches 2 and 3
    # audits act in stream order: after the first audit of batch 1 no
    # surrogate answer is served
    first = int(np.nonzero(route == RT.Router.AUDIT)[0][0])
    assert first < 32
    assert not np.any(route[first + 1:] == RT.Router.SURROGATE)
    assert rep["breaker_rerouted_in_batch"] == int(np.sum(route[first + 1:32] == RT.Router.BREAKER_IN_BATCH))
    ym = D.solve(qs[first + 1:])
    assert torch.allclose(ans[first + 1:], ym, rtol=0, atol=1e-4)  # 10 nm: the answers are the MPM's
    # one breaker per indenter family: a family trips at its first audit
    r = RT.Router(net, ftr, threshold=1e9, audit_rate=0.5, rmse_limit_um=1e-6, per_class=True)
    _, rep, route = r.serve(qs, batch=32)
    for k, pc in rep["per_class"].items():
        assert pc["tripped"] == (pc["audits"] > 0)
    assert rep["breaker_routed"] > 0
    assert sum(pc["queries"] for pc in rep["per_class"].values()) == 96


def test_breaker_starts_tripped_from_the_heldout_error(gpu):
    """A family whose held-out error is above the limit never gets a surrogate
    answer; the others start open."""
    from paper_2301_08343_amd import dataset as D
    from paper_2301_08343_amd import router as RT
    from paper_2301_08343_amd.surrogate import Net
    net = Net(batch=64, seed=1)
    ftr = RT.features(D.inputs(D.contacts_for(range(64), 0.5e-3)))
    qs = D.contacts_for(range(2000, 2064), 0.5e-3)
    fam = np.array([c["cfg"]["shape"] for c in qs])
    prior = {0: 1.0, 1: 7.5, 2: 2.0, 3: 6.0, 4: 1.0}
    r = RT.Router(net, ftr, threshold=1e9, audit_rate=0.0, rmse_limit_um=5.0, per_class=True, prior_rmse_um=prior)
    ans, rep, route = r.serve(qs, batch=32)
    assert rep["breaker_tripped_at_start"] == [1, 3]
    bad = np.isin(fam, [1, 3])
    assert np.all(route[bad] == RT.Router.BREAKER)
    assert np.all(route[~bad] == RT.Router.SURROGATE)
    idx = np.nonzero(bad)[0]
    ym = D.solve([qs[i] for i in idx])
    assert torch.allclose(ans[torch.tensor(idx, device="cuda")], ym, rtol=0, atol=1e-4)


def test_budget_admits_families_by_their_error_bound(gpu):
    """Error-budget policy without audits: the families whose held-out bounds
    fit the budget together get surrogate answers, the rest the MPM's."""
    from paper_2301_08343_amd import dataset as D
    from paper_2301_08343_amd import router as RT
    from paper_2301_08343_amd.surrogate import Net
    net = Net(batch=64, seed=1)
    ftr = RT.features(D.inputs(D.contacts_for(range(64), 0.5e-3)))
    qs = D.contacts_for(range(2000, 2064), 0.5e-3)
    fam = np.array([c["cfg"]["shape"] for c in qs])
    stats = {0: {"n": 100, "mean": 0.5, "sd": 0.5}, 1: {"n": 100, "mean": 30.0, "sd": 30.0},
             2: {"n": 100, "mean": 0.4, "sd": 0.4}, 3: {"n": 100, "mean": 33.0, "sd": 30.0},
             4: {"n": 100, "mean": 500.0, "sd": 400.0}}
    r = RT.Router(net, ftr, threshold=1e9, audit_rate=0.0, rmse_limit_um=5.0, policy="budget", prior_stats=stats)
    ans, rep, route = r.serve(qs, batch=32)
    shares = {f: float((fam == f).mean()) for f in range(5)}
    want = RT.admit({f: RT.FamilyError(**stats[f]).upper(1.645) for f in range(5)}, shares, 25.0)
    assert 4 not in want and {0, 2} <= want
    assert rep["budget"]["admitted_at_end"] == sorted(want)
    ok = np.isin(fam, sorted(want))
    assert np.all(route[ok] == RT.Router.SURROGATE)
    assert np.all(route[~ok] == RT.Router.BREAKER)
    idx = np.nonzero(~ok)[0]
    ym = D.solve([qs[i] for i in idx])
    assert torch.allclose(ans[torch.tensor(idx, device="cuda")], ym, rtol=0, atol=1e-4)


def test_budget_closes_a_family_at_its_first_bad_audit(gpu):
    """An untrained network with priors claiming 1 um RMSE and a 1.2 um limit
    (all families admitted at the start): each family's first audit shows an
    error of tens of micrometres, which alone lifts the share-weighted mean
    bound past the limit, so that family closes; no surrogate answer of a
    family is served after its first audit."""
    from paper_2301_08343_amd import dataset as D
    from paper_2301_08343_amd import router as RT
    from paper_2301_08343_amd.surrogate import Net
    net = Net(batch=64, seed=1)
    ftr = RT.features(D.inputs(D.contacts_for(range(64), 0.5e-3)))
    qs = D.contacts_for(range(1000, 1096), 0.5e-3)
    fam = np.array([c["cfg"]["shape"] for c in qs])
    stats = {f: {"n": 2, "mean": 1.0, "sd": 0.0} for f in range(5)}
    r = RT.Router(net, ftr, threshold=1e9, audit_rate=0.5, rmse_limit_um=1.2, policy="budget", prior_stats=stats)
    ans, rep, route = r.serve(qs, batch=32)
    assert rep["breaker_tripped_at_start"] == []
    for f in range(5):
        aud = np.nonzero((fam == f) & (route == RT.Router.AUDIT))[0]
        if len(aud):
            later = np.arange(len(qs)) > aud[0]
            assert not np.any(route[later & (fam == f)] == RT.Router.SURROGATE), f
            assert rep["per_class"][str(f)]["tripped"]
    assert rep["breaker_rerouted_in_batch"] + rep["breaker_routed"] > 0
    assert rep["mpm_fallbacks"] == rep["ood"] + rep["audited"] + rep["breaker_routed"] + rep["breaker_rerouted_in_batch"]


def test_budget_admits_classes_by_family_and_depth(gpu):
    """With depth edges the budget's classes are (family, depth bin): a
    family whose shallow presses have a small error bound and whose deep
    ones a large one gets surrogate answers for the shallow ones only."""
    from paper_2301_08343_amd import dataset as D
    from paper_2301_08343_amd import router as RT
    from paper_2301_08343_amd.surrogate import Net
    net = Net(batch=64, seed=1)
    ftr = RT.features(D.inputs(D.contacts_for(range(64), 0.5e-3)))
    qs = D.contacts_for(range(3000, 3096), 0.5e-3)
    edges = (0.2e-3 + 1.3e-3 / 3, 0.2e-3 + 2.6e-3 / 3)
    cls = np.array([RT.query_class(c, edges) for c in qs])
    # every family's first two depth bins cheap, the deepest bin expensive
    stats = {k: {"n": 50, "mean": (900.0 if k % 3 == 2 else 1.0), "sd": 1.0} for k in range(15)}
    r = RT.Router(net, ftr, threshold=1e9, audit_rate=0.0, rmse_limit_um=5.0, policy="budget", prior_stats=stats,
                  depth_edges=edges)
    ans, rep, route = r.serve(qs, batch=32)
    deep = cls % 3 == 2
    assert deep.any() and (~deep).any()
    assert np.all(route[~deep] == RT.Router.SURROGATE)
    assert np.all(route[deep] == RT.Router.BREAKER)
    assert rep["depth_edges_m"] == list(edges)
    assert set(rep["budget"]["admitted_at_end"]) == {k for k in range(15) if k % 3 != 2}
