"""The C-ABI library loads and exports every function include/dalia.h
declares (no GPU needed: nothing is called that touches a device)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dalia.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(
        r"^\s*(?:dl_status|void|int32_t|size_t|const char\*)\s+(\w+)\s*\(",
        src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("bta_assemble", "bta_factor", "bta_solve", "bta_selinv",
                 "fobj_eval", "dl_model_create", "dl_ws_create"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2507_06938_amd import build as B
    if not os.path.exists(B.LIB):
        B.build(verbose=False)
    lib = ctypes.CDLL(B.LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert lib.dl_theta_dim(1) == 4 and lib.dl_theta_dim(3) == 15


def test_model_create_rejects_bad_family_before_any_device_call():
    """Argument checks of dl_model_create run on the host before any HIP
    call: an unknown model family, and the diffusion-based family with a
    single time step (its temporal FEM needs two nodes), give DL_EINVAL."""
    import numpy as np
    from paper_2507_06938_amd import build as B
    from paper_2507_06938_amd import dalia as D
    if not os.path.exists(B.LIB):
        B.build(verbose=False)
    L = D.lib()
    pm = np.zeros(4)
    for family, nt in ((7, 3), (-1, 3), (D.MODEL_FAMILIES["diffusion"], 1)):
        d = D._Desc()
        d.nx, d.nt, d.nv, d.nr = 4, nt, 1, 1
        d.theta_prior_mean = pm.ctypes.data
        d.theta_prior_sd = 1.0
        d.prior_fixed = 1e-3
        d.family = family
        h = ctypes.c_void_p()
        assert L.dl_model_create(ctypes.byref(d), ctypes.byref(h)) == 1  # DL_EINVAL
        assert not h.value
    # dl_model_desc: 4 int32, 3 int64, 16 pointers, 2 doubles, int32 family
    # and int32 likelihood
    assert ctypes.sizeof(D._Desc) == 16 + 24 + 128 + 16 + 8


def test_model_create_rejects_bad_likelihood_and_counts_before_any_device_call():
    """An unknown likelihood, and for the Poisson likelihood a negative or
    non-integer count, give DL_EINVAL from the host-side checks; the theta
    dimension drops the noise precisions."""
    import numpy as np
    from paper_2507_06938_amd import build as B
    from paper_2507_06938_amd import dalia as D
    if not os.path.exists(B.LIB):
        B.build(verbose=False)
    L = D.lib()
    assert L.dl_theta_dim_lik(1, 0) == 4 and L.dl_theta_dim_lik(3, 0) == 15
    assert L.dl_theta_dim_lik(1, 1) == 3 and L.dl_theta_dim_lik(3, 1) == 12
    assert L.dl_theta_dim_lik(2, 1) == 7 and L.dl_theta_dim_lik(1, 9) == -1
    pm = np.zeros(4)
    t = np.zeros(2, np.int32)
    nodes = np.array([0, 1, 4, 1, 4, 5], np.int32)
    w = np.full(6, 1.0 / 3.0)
    X = np.ones(2)
    for lik, yv in ((5, (1.0, 2.0)), (-1, (1.0, 2.0)), (1, (1.0, -1.0)), (1, (0.5, 2.0)),
                    (1, (np.nan, 2.0))):
        y = np.array(yv)
        d = D._Desc()
        d.nx, d.nt, d.nv, d.nr = 4, 3, 1, 1
        d.m[0] = 2
        d.obs_t[0], d.obs_nodes[0], d.obs_w[0] = t.ctypes.data, nodes.ctypes.data, w.ctypes.data
        d.obs_x[0], d.y[0] = X.ctypes.data, y.ctypes.data
        d.theta_prior_mean = pm.ctypes.data
        d.theta_prior_sd = 1.0
        d.prior_fixed = 1e-3
        d.likelihood = lik
        h = ctypes.c_void_p()
        assert L.dl_model_create(ctypes.byref(d), ctypes.byref(h)) == 1, (lik, yv)
        assert not h.value


def test_model_create_rejects_blocks_beyond_the_lds_column_buffer():
    """The assembly keeps a column of a diagonal and a sub-diagonal block
    (2 bp + 64 doubles) in 160 KiB of LDS: one response on a 101 x 101
    mesh (bp = 10240) or three on 59 x 59 (bp = 10496) are rejected on the
    host; 100 x 100 and 3 x 58 x 58 are the largest accepted sizes."""
    import numpy as np
    from paper_2507_06938_amd import build as B
    from paper_2507_06938_amd import dalia as D
    if not os.path.exists(B.LIB):
        B.build(verbose=False)
    L = D.lib()
    for nx, nv in ((101, 1), (59, 3)):
        pm = np.zeros(L.dl_theta_dim(nv))
        d = D._Desc()
        d.nx, d.nt, d.nv, d.nr = nx, 3, nv, 1
        d.theta_prior_mean = pm.ctypes.data
        d.theta_prior_sd = 1.0
        d.prior_fixed = 1e-3
        h = ctypes.c_void_p()
        assert L.dl_model_create(ctypes.byref(d), ctypes.byref(h)) == 1, (nx, nv)
        assert not h.value
    for nx, nv in ((100, 1), (58, 3)):
        bp = (nv * nx * nx + 63) // 64 * 64
        assert (2 * bp + 64) * 8 <= 160 * 1024


def test_binding_constants_match_the_header():
    """The flag, likelihood and family values the Python binding passes are
    the ones include/dalia.h defines (read from the header text)."""
    import re
    from paper_2507_06938_amd import dalia as D
    text = open(os.path.join(ROOT, "include", "dalia.h")).read()
    vals = {m.group(1): int(m.group(2))
            for m in re.finditer(r"\b(DL_[A-Z0-9_]+)\s*=\s*(\d+)", text)}
    for name in ("DL_WS_SELINV", "DL_WS_KEEP_QP", "DL_WS_GRAPH", "DL_WS_MIXED",
                 "DL_WS_SPLITK", "DL_WS_TWOSIDED", "DL_WS_FOLD_INV", "DL_WS_WARM_START",
                 "DL_QP", "DL_QC", "DL_BOTH"):
        assert getattr(D, name) == vals[name], name
    assert D.LIKELIHOODS == {"gaussian": vals["DL_LIK_GAUSSIAN"],
                             "poisson": vals["DL_LIK_POISSON"]}
    assert D.MODEL_FAMILIES == {"separable": vals["DL_MODEL_SEPARABLE"],
                                "diffusion": vals["DL_MODEL_DIFFUSION"]}


def test_dpotrf_noalloc_rejects_sizes_on_the_host():
    """dl_dpotrf_noalloc checks n against its static scratch before any
    device call: n above DL_DPOTRF_NOALLOC_MAX_N, n not a multiple of 64 and
    NULL outputs give DL_EINVAL (1)."""
    from paper_2507_06938_amd import build as B
    from paper_2507_06938_amd import dalia as D
    if not os.path.exists(B.LIB):
        B.build(verbose=False)
    L = D.lib()
    hdr = open(HEADER).read()
    max_n = int(re.search(r"#define DL_DPOTRF_NOALLOC_MAX_N (\d+)", hdr).group(1))
    assert max_n == D.DPOTRF_NOALLOC_MAX_N
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: rejected first
    for n in (max_n + 64, 100, 0, -64):
        assert L.dl_dpotrf_noalloc(n, fake, max(n, 1), 0, fake, fake, None) == 1
    assert L.dl_dpotrf_noalloc(64, fake, 64, 0, None, fake, None) == 1
    assert L.dl_dpotrf_noalloc(64, fake, 32, 0, fake, fake, None) == 1
