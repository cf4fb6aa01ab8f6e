"""Full-size parity: the production workloads in the configuration bench.py
times, against values stored by tests/golden/make_golden.py (CPU oracle,
RCM + banded LAPACK Cholesky) -- log-determinants, f_obj, the conditional
mean and the marginal variances at seeded sample positions (every fixed
effect included)."""
import json
import os

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_06938_amd import dalia
    dalia.lib()
    return dalia


@pytest.mark.parametrize("splitk", [False, True])
@pytest.mark.parametrize("name,make", [
    ("c1", W.config1), ("c2", W.config2),
    ("c1_diffusion", lambda: W.config1(model="diffusion"))])
def test_fullsize_against_banded_oracle(D, name, make, splitk):
    path = os.path.join(GOLD, f"{name}_golden.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    g = json.load(open(path))
    wl = make()
    model = D.Model.from_workload(wl)
    ws = D.Workspace(model, selinv=True, splitk=splitk)
    f, parts, info = ws.fobj(np.asarray(g["theta"]))
    mu = ws.mean()
    var = ws.selinv()
    torch.cuda.synchronize()
    p = parts.cpu().numpy()[0]
    assert info.cpu().tolist() == [[0, 0]]
    assert abs(p[1] - g["logdet_p"]) <= 1e-10 * abs(g["logdet_p"])
    assert abs(p[2] - g["logdet_c"]) <= 1e-10 * abs(g["logdet_c"])
    scale = abs(g["logdet_p"]) + abs(g["logdet_c"])
    assert abs(p[0] - g["f"]) <= 1e-10 * scale
    mu_s = mu.cpu().numpy()[np.asarray(g["mu_index_bta"])]
    want = np.asarray(g["mu"])
    assert np.max(np.abs(mu_s - want)) <= 1e-9 * np.max(np.abs(want))
    v_s = var.cpu().numpy()[np.asarray(g["var_index_bta"])]
    np.testing.assert_allclose(v_s, np.asarray(g["var"]), rtol=1e-9)
    # every variance is positive and finite
    v = var.cpu().numpy()
    assert np.all(np.isfinite(v)) and np.all(v > 0)
    del ws
