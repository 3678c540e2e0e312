"""hsn_fhr_step (the whole FHR path in one C call) against the same entry
points called one after the other: the same kernels in the same order, so
V, D, x, x^h and the NMF statistics must agree bit for bit."""
import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import show, to_dev

pytestmark = pytest.mark.gpu


def _scan():
    sc = synth.config_scan("tiny")
    return sc, to_dev(sc.y), to_dev(sc.yo)


@pytest.mark.parametrize("learned", [True, False])
def test_fhr_step_equals_the_calls_in_sequence(hsn, learned):
    sc, y, yo = _scan()
    n_k, K = sc.n_bins, sc.n_mat
    g = np.random.Generator(np.random.PCG64(3))
    V0 = torch.from_numpy(g.uniform(0.1, 1.0, (sc.n_p, K)).astype(np.float32)).cuda()
    D0 = torch.from_numpy(g.uniform(0.1, 1.0, (n_k, K)).astype(np.float32)).cuda()
    if learned:
        m = hsn.hsn_mlp_create(K, hsn.PREC_BF16)
        kw = dict(init=hsn.INIT_MLP, mlp=m, max_iter=0, check_every=1, polish_rounds=4, polish_algo=hsn.ALGO_ANLS)
    else:
        kw = dict(init=hsn.INIT_USER, algo=hsn.ALGO_MU, max_iter=12, check_every=4, polish_rounds=3,
                  polish_algo=hsn.ALGO_ANLS)
    n_x = sc.n_rows * sc.n_cols * sc.n_cols
    show("fhr step vs sequence", learned=learned)
    # the calls one after the other
    V1, D1 = V0.clone(), D0.clone()
    if learned:
        p, _, pooled, _, _ = hsn.hsn_normalize_pooled(y, yo, m.precision)
        s1 = hsn.hsn_subspace_nmf(p, None, n_k, V1, D1, mlp_pooled=pooled, **kw)
    else:
        p, _, _, _ = hsn.hsn_normalize(y, yo)
        s1 = hsn.hsn_subspace_nmf(p, None, n_k, V1, D1, **kw)
    x1 = hsn.hsn_cgls(V1.view(sc.n_views, sc.n_rows, sc.n_cols, K), 6)
    xh1 = hsn.hsn_rehydrate(x1.view(-1, K), D1, vox=(100, n_x - 50), bins=(3, n_k - 7))
    # one call
    V2, D2 = V0.clone(), D0.clone()
    x2, xh2, s2 = hsn.hsn_fhr_step(y, yo, V2, D2, 6, vox=(100, n_x - 50), bins=(3, n_k - 7), **kw)
    assert torch.equal(V1, V2) and torch.equal(D1, D2)
    assert torch.equal(x1, x2) and torch.equal(xh1, xh2)
    assert s1["history"] == s2["history"] and s1["polish_done"] == s2["polish_done"]


def test_fhr_step_stop_test_and_errors(hsn):
    # With a stop test the statistics come back with the convergence read-back.
    sc, y, yo = _scan()
    n_k, K = sc.n_bins, sc.n_mat
    g = np.random.Generator(np.random.PCG64(4))
    V0 = torch.from_numpy(g.uniform(0.1, 1.0, (sc.n_p, K)).astype(np.float32)).cuda()
    D0 = torch.from_numpy(g.uniform(0.1, 1.0, (n_k, K)).astype(np.float32)).cuda()
    kw = dict(init=hsn.INIT_USER, algo=hsn.ALGO_MU, max_iter=20, check_every=5, polish_rounds=200,
              polish_algo=hsn.ALGO_ANLS)
    V, D = V0.clone(), D0.clone()
    _, _, ref = hsn.hsn_fhr_step(y, yo, V, D, 2, **kw)
    f_ref = ref["objective"] * 0.999
    V, D = V0.clone(), D0.clone()
    _, _, st = hsn.hsn_fhr_step(y, yo, V, D, 2, f_ref=f_ref, rel_obj_tol=0.01, **kw)
    show("fhr step stop", rounds=st["polish_done"], rel=st["rel_obj"])
    assert st["rel_obj"] <= 0.01 and st["polish_done"] < 200
    assert len(st["history"]) >= 1 and st["history"][-1] == st["objective"]
    with pytest.raises(hsn.HsnError):     # learned start without a network
        hsn.hsn_fhr_step(y, yo, V, D, 2, init=hsn.INIT_MLP, max_iter=0, polish_rounds=1, polish_algo=hsn.ALGO_ANLS)
