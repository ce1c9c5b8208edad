"""The data -> training -> router pipeline end to end at a coarse spacing
(0.5 mm lattice, 12,800 particles per contact): it runs, the loss falls, the
router's report is consistent, and the circuit breaker hands everything to
the MPM when its limit cannot be met."""
import json

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
    assert r["mpm_fallbacks"] == r["ood"] + r["audited"] + r["breaker_routed"]
    assert r["audited"] >= 1  # 2% of 300 draws
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
    ans, rep = r.serve(qs, batch=32)
    assert rep["breaker_tripped"] == [0]
    assert rep["breaker_routed"] == 64  # batches 2 and 3
    ym = D.solve(qs[32:])
    assert torch.allclose(ans[32:], ym, rtol=0, atol=1e-4)  # 10 nm: the answers are the MPM's
    # one breaker per indenter family: a family trips once it has an audit
    r = RT.Router(net, ftr, threshold=1e9, audit_rate=0.5, rmse_limit_um=1e-6, per_class=True)
    _, rep = r.serve(qs, batch=32)
    for k, pc in rep["per_class"].items():
        assert pc["tripped"] == (pc["audits"] > 0)
    assert rep["breaker_routed"] > 0
    assert sum(pc["queries"] for pc in rep["per_class"].values()) == 96
