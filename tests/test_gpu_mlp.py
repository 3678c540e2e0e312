"""GPU parity of the warm-start network (pooling, forward, loss gradient,
Adam) and of the canonical form against the FP64 oracle.

FP32 network: float32 weights and activations on the f32 MFMA, float32
accumulation over at most 256 terms per output: forward and gradients are
held to 1e-5 relative (Frobenius, per parameter block).
BF16 network: the oracle runs on the same bfloat16-rounded inputs and
weights in FP64; the kernels also round h1, h2 and the back-propagated dz to
bfloat16 (relative 2^-9 each), so outputs are held to 1e-2 and gradients to
3e-2 relative, with cosine similarity >= 0.999."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import mlp as omlp
from oracle.metrics import canonical
from oracle.nnls import nnls_rows
from tests.gpu_util import bf16_rne, rel_fro, show

pytestmark = pytest.mark.gpu


def _params(k, seed):
    th = synth.mlp_init(k, seed)
    g = np.random.Generator(np.random.PCG64(seed + 1))
    # non-zero biases so that every term of the model is exercised
    for (lo, n) in _bias_slices(k):
        th[lo:lo + n] = g.uniform(-0.3, 0.3, n)
    return th.astype(np.float32)


def _bias_slices(k):
    out, o = [], 0
    for s in omlp.param_shapes(k):
        n = int(np.prod(s))
        if len(s) == 1:
            out.append((o, n))
        o += n
    return out


def _x(n, seed, scale=1.0):
    g = np.random.Generator(np.random.PCG64(seed))
    return (g.uniform(0.0, 2.0, (n, omlp.N_IN)) * scale).astype(np.float32)


def _bits_to_f32(bits):
    return (bits.astype(np.uint32) << 16).view(np.float32)


def _round_bf16(a):
    return _bits_to_f32(bf16_rne(np.asarray(a, np.float32)))


def _blocks(flat, k):
    return omlp.unflatten(np.asarray(flat, np.float64), k)


@pytest.mark.parametrize("n_k", [256, 1024, 1000, 100, 2048])
def test_pool_matches_oracle(hsn, n_k):
    n_p = 300
    g = np.random.Generator(np.random.PCG64(n_k))
    p = g.uniform(0, 2, (n_p, n_k)).astype(np.float32)
    ldb = (n_k + 31) // 32 * 32
    bits = np.zeros((n_p, ldb), np.uint16)
    bits[:, :n_k] = bf16_rne(p)
    ref = omlp.pool(_bits_to_f32(bits[:, :n_k]).astype(np.float64))
    pb = torch.from_numpy(bits.view(np.int16)).cuda()
    show("pool", n_k=n_k)
    x32 = hsn.hsn_mlp_pool(pb, n_k, hsn.PREC_FP32).cpu().numpy()
    assert np.max(np.abs(x32 - ref) / np.maximum(np.abs(ref), 1e-30)) <= 2e-6
    xb = hsn.hsn_mlp_pool(pb, n_k, hsn.PREC_BF16).cpu().numpy().view(np.uint16)
    assert np.array_equal(xb, bf16_rne(x32))


@pytest.mark.parametrize("k,n", [(4, 1000), (1, 64), (8, 333), (5, 4096)])
def test_fp32_forward_and_grad(hsn, k, n):
    th = _params(k, 10 + k)
    x = _x(n, 20 + k)
    g = np.random.Generator(np.random.PCG64(30 + k))
    t = g.uniform(0, 3, (n, k)).astype(np.float32)
    P = _blocks(th, k)
    y_ref, _ = omlp.forward(P, x.astype(np.float64))
    l_ref, g_ref = omlp.loss_and_grad(P, x.astype(np.float64), t.astype(np.float64))
    m = hsn.hsn_mlp_create(k, hsn.PREC_FP32, th)
    xd = torch.from_numpy(x).cuda()
    show("fp32 mlp", k=k, n=n)
    y = hsn.hsn_mlp_forward(m, xd).cpu().numpy()
    show("  forward", err=rel_fro(y, y_ref))
    assert rel_fro(y, y_ref) <= 1e-5
    loss, grad = hsn.hsn_mlp_loss_grad(m, xd, torch.from_numpy(t).cuda())
    gb = _blocks(grad.cpu().numpy(), k)
    errs = [rel_fro(a, b) for a, b in zip(gb, g_ref)]
    show("  grad", loss=abs(loss.item() - l_ref) / l_ref, blocks=errs)
    assert abs(loss.item() - l_ref) <= 1e-5 * l_ref
    assert max(errs) <= 1e-5


@pytest.mark.parametrize("k,n", [(4, 1000), (3, 4096)])
def test_bf16_forward_and_grad(hsn, k, n):
    th = _params(k, 40 + k)
    x = _x(n, 50 + k)
    g = np.random.Generator(np.random.PCG64(60 + k))
    t = g.uniform(0, 3, (n, k)).astype(np.float32)
    # the oracle on the bfloat16 weights and inputs (biases stay float32)
    thq = th.copy()
    bias = np.zeros(th.size, bool)
    for lo, nb in _bias_slices(k):
        bias[lo:lo + nb] = True
    thq[~bias] = _round_bf16(th[~bias])
    xq = _round_bf16(x)
    P = _blocks(thq, k)
    y_ref, _ = omlp.forward(P, xq.astype(np.float64))
    l_ref, g_ref = omlp.loss_and_grad(P, xq.astype(np.float64), t.astype(np.float64))
    m = hsn.hsn_mlp_create(k, hsn.PREC_BF16, th)
    xd = torch.from_numpy(bf16_rne(x).view(np.int16)).cuda()
    show("bf16 mlp", k=k, n=n)
    y = hsn.hsn_mlp_forward(m, xd).cpu().numpy()
    show("  forward", err=rel_fro(y, y_ref))
    assert rel_fro(y, y_ref) <= 1e-2
    loss, grad = hsn.hsn_mlp_loss_grad(m, xd, torch.from_numpy(t).cuda())
    gb = _blocks(grad.cpu().numpy(), k)
    errs = [rel_fro(a, b) for a, b in zip(gb, g_ref)]
    cos = float(np.dot(grad.cpu().numpy(), omlp.flatten(g_ref)) /
                (np.linalg.norm(grad.cpu().numpy()) * np.linalg.norm(omlp.flatten(g_ref))))
    show("  grad", loss=abs(loss.item() - l_ref) / l_ref, blocks=errs, cos=cos)
    assert abs(loss.item() - l_ref) <= 1e-2 * l_ref
    assert max(errs) <= 3e-2 and cos >= 0.999


def test_adam_steps_match_oracle(hsn):
    # Two epochs of one full batch each: two Adam steps from zero moments.
    k, n = 4, 512
    th = _params(k, 70)
    x = _x(n, 71)
    t = np.random.Generator(np.random.PCG64(72)).uniform(0, 3, (n, k)).astype(np.float32)
    ref = th.astype(np.float64)
    mm = np.zeros_like(ref)
    vv = np.zeros_like(ref)
    for step in (1, 2):
        _, g = omlp.loss_and_grad(_blocks(ref, k), x.astype(np.float64), t.astype(np.float64))
        ref, mm, vv = omlp.adam_step(ref, omlp.flatten(g), mm, vv, step)
    m = hsn.hsn_mlp_create(k, hsn.PREC_FP32, th)
    show("adam two steps")
    hist = hsn.hsn_mlp_train(m, torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda(), epochs=2, batch=n, seed=5)
    got = m.get_params()
    show("  err", theta=rel_fro(got - th, ref - th), loss=hist)
    # compare the update itself (the change of the parameters)
    assert rel_fro(got - th, ref - th) <= 1e-4
    assert rel_fro(got, ref) <= 1e-6


def test_training_reduces_loss_and_is_deterministic(hsn):
    # Targets from a fixed random teacher network; ragged last batch.
    k, n = 3, 20000
    x = _x(n, 80, scale=0.5)
    teacher = _params(k, 81)
    y_t, _ = omlp.forward(_blocks(teacher, k), _round_bf16(x).astype(np.float64))
    xd = torch.from_numpy(bf16_rne(x).view(np.int16)).cuda()
    td = torch.from_numpy(y_t.astype(np.float32)).cuda()
    runs = []
    for _ in range(2):
        m = hsn.hsn_mlp_create(k, hsn.PREC_BF16, synth.mlp_init(k, 82).astype(np.float32))
        hist = hsn.hsn_mlp_train(m, xd, td, epochs=6, batch=1024, lr=2e-3, seed=9)
        runs.append((hist, m.get_params()))
    show("train", loss=runs[0][0])
    assert runs[0][0][-1] <= 0.2 * runs[0][0][0]
    assert runs[0][0] == runs[1][0] and np.array_equal(runs[0][1], runs[1][1])


def test_save_load_roundtrip(hsn, tmp_path):
    k = 5
    m = hsn.hsn_mlp_create(k, hsn.PREC_BF16, _params(k, 90))
    x = torch.from_numpy(bf16_rne(_x(200, 91)).view(np.int16)).cuda()
    t = torch.ones((200, k), device="cuda")
    hsn.hsn_mlp_train(m, x, t, epochs=1, batch=64)
    f = str(tmp_path / "net.bin")
    hsn.hsn_mlp_save(m, f)
    m2 = hsn.hsn_mlp_load(f)
    assert m2.k == k and m2.precision == hsn.PREC_BF16
    assert np.array_equal(m.get_params(), m2.get_params())
    assert torch.equal(hsn.hsn_mlp_forward(m, x), hsn.hsn_mlp_forward(m2, x))
    # resumed training continues identically (moments and step count restored)
    hsn.hsn_mlp_train(m, x, t, epochs=1, batch=64, seed=3)
    hsn.hsn_mlp_train(m2, x, t, epochs=1, batch=64, seed=3)
    assert np.array_equal(m.get_params(), m2.get_params())


def test_infer_is_pool_then_forward(hsn):
    k, n_p, n_k = 4, 777, 1024
    m = hsn.hsn_mlp_create(k, hsn.PREC_BF16, _params(k, 95))
    g = np.random.Generator(np.random.PCG64(96))
    bits = np.zeros((n_p, n_k), np.uint16)
    bits[:] = bf16_rne(g.uniform(0, 2, (n_p, n_k)).astype(np.float32))
    pb = torch.from_numpy(bits.view(np.int16)).cuda()
    show("infer")
    v0 = hsn.hsn_mlp_infer(m, pb, n_k)
    v1 = hsn.hsn_mlp_forward(m, hsn.hsn_mlp_pool(pb, n_k, hsn.PREC_BF16))
    assert torch.equal(v0, v1)
    assert bool((v0 > 0).all())


@pytest.mark.parametrize("k,lib", [(4, True), (3, False), (6, True), (1, True)])
def test_canonicalize_matches_oracle(hsn, k, lib):
    n_p, n_k = 1000, 300
    g = np.random.Generator(np.random.PCG64(100 + k))
    L = g.uniform(0.1, 1, (n_k, k))
    perm = g.permutation(k)
    D = (L[:, perm] * g.uniform(0.5, 3, k) + 0.05 * g.uniform(0, 1, (n_k, k))).astype(np.float32)
    V = (g.uniform(0, 1, (n_p, k)) * g.uniform(0.1, 5, k)).astype(np.float32)
    Vr, Dr = canonical(V.astype(np.float64), D.astype(np.float64), library=L if lib else None)
    Vd, Dd = torch.from_numpy(V).cuda(), torch.from_numpy(D).cuda()
    show("canonical", k=k, lib=lib)
    hsn.hsn_canonicalize(Vd, Dd, torch.from_numpy(L.astype(np.float32)).cuda() if lib else None)
    assert rel_fro(Vd.cpu().numpy(), Vr) <= 1e-6
    assert rel_fro(Dd.cpu().numpy(), Dr) <= 1e-6


def test_nmf_learned_start(hsn):
    # init = MLP with max_iter = 0: V0 is the network's output, D0 the exact
    # row-wise NNLS solution for V0 with zeros set to 1e-6 mean(D0).
    sc = synth.config_scan("tiny")
    y = torch.from_numpy(sc.y.view(np.int16)).cuda()
    yo = torch.from_numpy(sc.yo.view(np.int16)).cuda()
    p, pb, _, _ = hsn.hsn_normalize(y, yo, want_bf16=True)
    n_p, n_k, k = sc.n_p, sc.n_bins, 3
    m = hsn.hsn_mlp_create(k, hsn.PREC_BF16, _params(k, 110))
    V = torch.zeros((n_p, k), device="cuda")
    D = torch.zeros((n_k, k), device="cuda")
    show("nmf learned start")
    hsn.hsn_subspace_nmf(p, pb, n_k, V, D, init=hsn.INIT_MLP, mlp=m, max_iter=0)
    v0 = hsn.hsn_mlp_infer(m, pb, n_k)
    assert torch.equal(V, v0)
    V0 = v0.cpu().numpy().astype(np.float64)
    P = p[:, :n_k].cpu().numpy().astype(np.float64)
    Dr = nnls_rows(V0.T @ V0, P.T @ V0)
    Dr[Dr == 0] = 1e-6 * Dr.mean()
    tol = max(1e-5, np.linalg.cond(V0.T @ V0) * 2.0 ** -23)
    show("  D0", err=rel_fro(D.cpu().numpy(), Dr), tol=tol)
    assert rel_fro(D.cpu().numpy(), Dr) <= tol
    # the same start from rows pooled in the normalisation pass (no p_bf16)
    _, _, pooled, _, _ = hsn.hsn_normalize_pooled(y, yo, hsn.PREC_BF16, want_f32=False)
    V2 = torch.zeros_like(V)
    D2 = torch.zeros_like(D)
    hsn.hsn_subspace_nmf(p, None, n_k, V2, D2, init=hsn.INIT_MLP, mlp=m, max_iter=0, mlp_pooled=pooled)
    assert torch.equal(V2, V) and torch.equal(D2, D)
    # first rounds on p_bf16: D0 comes from the bfloat16 pass (N_D = P_bf16^T V0),
    # then one bfloat16 ANLS round; against the oracle on the bfloat16-rounded p,
    # at the cond(G) 2^-16 bound of the split products
    V3 = torch.zeros_like(V)
    D3 = torch.zeros_like(D)
    hsn.hsn_subspace_nmf(p, pb, n_k, V3, D3, init=hsn.INIT_MLP, mlp=m, max_iter=0, polish_rounds=1,
                         polish_bf16_rounds=1, polish_algo=hsn.ALGO_ANLS)
    Pq = hsn.bf16_bits_to_float(pb[:, :n_k]).cpu().numpy().astype(np.float64)
    Dq = nnls_rows(V0.T @ V0, Pq.T @ V0)
    Dq[Dq == 0] = 1e-6 * Dq.mean()
    V1r = nnls_rows(Dq.T @ Dq, Pq @ Dq)
    D1r = nnls_rows(V1r.T @ V1r, Pq.T @ V1r)
    tv = max(2e-5, np.linalg.cond(Dq.T @ Dq) * np.linalg.cond(V0.T @ V0) * 2.0 ** -16)
    td = max(2e-5, np.linalg.cond(V1r.T @ V1r) * 2.0 ** -16 + tv)
    show("  bf16 D0 + round", V=rel_fro(V3.cpu().numpy(), V1r), D=rel_fro(D3.cpu().numpy(), D1r), tv=tv, td=td)
    assert rel_fro(V3.cpu().numpy(), V1r) <= tv and rel_fro(D3.cpu().numpy(), D1r) <= td
    # rejected: missing network, mismatched k, neither p_bf16 nor pooled rows
    with pytest.raises(hsn.HsnError):
        hsn.hsn_subspace_nmf(p, None, n_k, V, D, init=hsn.INIT_MLP, mlp=m, max_iter=0)
    with pytest.raises(hsn.HsnError):
        hsn.hsn_subspace_nmf(p, pb, n_k, V, D, init=hsn.INIT_MLP, max_iter=0)
    m4 = hsn.hsn_mlp_create(4, hsn.PREC_BF16, None)
    with pytest.raises(hsn.HsnError):
        hsn.hsn_subspace_nmf(p, pb, n_k, V, D, init=hsn.INIT_MLP, mlp=m4, max_iter=0)


def test_learned_start_falls_back_to_nndsvda(hsn):
    # A learned start whose first objective is too far above f_ref (here an
    # untrained network and a threshold no start meets) is replaced by
    # NNDSVDa: the run then equals, bit for bit, the same schedule started
    # from NNDSVDa directly, and reports fell_back.  With a loose threshold
    # the learned start is kept.
    sc = synth.config_scan("tiny")
    y = torch.from_numpy(sc.y.view(np.int16)).cuda()
    yo = torch.from_numpy(sc.yo.view(np.int16)).cuda()
    p, pb, _, _, bias = hsn.hsn_normalize(y, yo, want_bf16=True, want_bias=True)
    n_p, n_k, k = sc.n_p, sc.n_bins, 3
    kw = dict(max_iter=0, polish_rounds=24, polish_bf16_rounds=16, polish_algo=hsn.ALGO_ANLS, bf16_bias=bias)
    Vr = torch.zeros((n_p, k), device="cuda")
    Dr = torch.zeros((n_k, k), device="cuda")
    ref = hsn.hsn_subspace_nmf(p, pb, n_k, Vr, Dr, init=hsn.INIT_NNDSVDA, max_iter=0, polish_rounds=60,
                               polish_algo=hsn.ALGO_ANLS)
    f_ref = min(ref["history"])
    kw.update(rel_obj_tol=1e-3, f_ref=f_ref)
    V1 = torch.zeros((n_p, k), device="cuda")
    D1 = torch.zeros((n_k, k), device="cuda")
    st1 = hsn.hsn_subspace_nmf(p, pb, n_k, V1, D1, init=hsn.INIT_NNDSVDA, **kw)
    m = hsn.hsn_mlp_create(k, hsn.PREC_BF16, _params(k, 120))
    V2 = torch.zeros_like(V1)
    D2 = torch.zeros_like(D1)
    show("learned start fallback")
    st2 = hsn.hsn_subspace_nmf(p, pb, n_k, V2, D2, init=hsn.INIT_MLP, mlp=m, mlp_fallback_rel=1e-12, **kw)
    assert st2["fell_back"] and not st1["fell_back"]
    assert torch.equal(V2, V1) and torch.equal(D2, D1)
    for key in ("polish_done", "polish_bf16_done", "history"):
        assert st2[key] == st1[key]
    V3 = torch.zeros_like(V1)
    D3 = torch.zeros_like(D1)
    st3 = hsn.hsn_subspace_nmf(p, pb, n_k, V3, D3, init=hsn.INIT_MLP, mlp=m, mlp_fallback_rel=1e12, **kw)
    assert not st3["fell_back"]
