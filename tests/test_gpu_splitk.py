"""Split-k workspaces (DL_WS_SPLITK): the long inner dimensions of the FP64
block products are cut at absolute multiples of 512 and the pieces summed
in k order by a second launch.  Checked against the CPU oracle and against
the unsplit workspace, at block sizes where products really split (bp > 512,
ragged tails), and for independence of the tile size (bit for bit)."""
import numpy as np
import pytest

import workloads as W
from oracle import fobj as OF

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [
    # name, nx, nt, nv, nr, m_per: b = nv * nx^2
    ("uni_b676", 26, 4, 1, 2, 300),     # bp = 704: two pieces, ragged tail
    ("tri_b1200", 20, 3, 3, 2, 250),    # bp = 1216: three pieces
]


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_06938_amd import dalia
    dalia.lib()
    return dalia


@pytest.mark.parametrize("name,nx,nt,nv,nr,m_per", CASES)
def test_splitk_against_oracle_and_unsplit(D, name, nx, nt, nv, nr, m_per):
    wl = W.scaled(name, nx, nt, nv, nr, m_per, seed=21)
    theta = W.random_theta_near(wl.theta, 0.1, seed=4)
    print(f"case {name} N={wl.N} b={wl.b}", flush=True)
    model = D.Model.from_workload(wl)
    out = {}
    for split in (False, True):
        ws = D.Workspace(model, selinv=True, splitk=split)
        f, parts, info = ws.fobj(theta)
        mu = ws.mean().cpu().numpy()
        var = ws.selinv().cpu().numpy()
        torch.cuda.synchronize()
        assert info.cpu().tolist() == [[0, 0]]
        out[split] = (parts.cpu().numpy()[0], mu, var)
        del ws
    ref = OF.fobj_parts(wl, theta, method="dense")
    for split in (False, True):
        p, mu, var = out[split]
        assert abs(p[1] - ref["logdet_p"]) <= 1e-10 * abs(ref["logdet_p"])
        assert abs(p[2] - ref["logdet_c"]) <= 1e-10 * abs(ref["logdet_c"])
        assert abs(p[0] - ref["f"]) <= 1e-10 * (abs(ref["logdet_p"]) + abs(ref["logdet_c"]))
    # split and unsplit differ by rounding only
    (p0, mu0, v0), (p1, mu1, v1) = out[False], out[True]
    assert abs(p1[2] - p0[2]) <= 1e-13 * abs(p0[2])
    assert np.max(np.abs(mu1 - mu0)) <= 1e-11 * np.max(np.abs(mu0))
    np.testing.assert_allclose(v1, v0, rtol=1e-11)


def test_splitk_independent_of_tile_size(D):
    """Pieces start at absolute multiples of 512, so 64- and 128-wide tiles
    sum every output over the same pieces: bit-identical results."""
    wl = W.scaled("tiles_b784", 28, 3, 1, 2, 200, seed=5)
    model = D.Model.from_workload(wl)
    res = []
    for tile in (64, 128):
        ws = D.Workspace(model, selinv=True, splitk=True)
        ws.force_tile(tile)
        assert ws.tile_counts()[f"tile{tile}"] > 0
        f, parts, _ = ws.fobj(wl.theta)
        var = ws.selinv().cpu().numpy()
        torch.cuda.synchronize()
        res.append((parts.cpu().numpy()[0].copy(), var))
        del ws
    assert np.array_equal(res[0][0], res[1][0])
    assert np.array_equal(res[0][1], res[1][1])


def test_split_piece_length_256_against_unsplit(D):
    """Pieces of 256 (what the tuner may choose for launches with short k):
    agree with the unsplit workspace to rounding and with the oracle, and
    are again independent of the tile size."""
    wl = W.scaled("pieces_b784", 28, 3, 1, 2, 200, seed=6)
    model = D.Model.from_workload(wl)
    res = {}
    for key, ks, tile in (("unsplit", 0, 64), ("s256_64", 256, 64), ("s256_128", 256, 128)):
        ws = D.Workspace(model, selinv=True)
        ws.force_tile(tile)
        ws.force_split(ks)
        f, parts, info = ws.fobj(wl.theta)
        var = ws.selinv().cpu().numpy()
        torch.cuda.synchronize()
        assert info.cpu().tolist() == [[0, 0]]
        res[key] = (parts.cpu().numpy()[0].copy(), var)
        del ws
    ref = OF.fobj_parts(wl, wl.theta, method="dense")
    p, v = res["s256_64"]
    assert abs(p[2] - ref["logdet_c"]) <= 1e-10 * abs(ref["logdet_c"])
    assert abs(p[2] - res["unsplit"][0][2]) <= 1e-13 * abs(p[2])
    np.testing.assert_allclose(v, res["unsplit"][1], rtol=1e-11)
    assert np.array_equal(res["s256_64"][0], res["s256_128"][0])
    assert np.array_equal(res["s256_64"][1], res["s256_128"][1])
