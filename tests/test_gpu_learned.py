"""Learned estimator on the GPU vs the FP64 reference (oracle/mlp_ref.py).

Features are bit-exact (same FP64 divisions rounded once to FP32).  The
network output y = ln(1 + n) agrees within 1e-4 |y| + 2e-3: the GPU
accumulates in FP32 on the matrix cores where the reference uses FP64, and a
first-layer activation sitting on a bf16 rounding boundary may round the
other way (one bf16 ulp, 2^-8 relative, times a weight).  Gradients of one
batch agree within 1e-3 relative (FP32 accumulation over the batch and the
network), the Adam update to 1e-6 absolute.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def V():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_13132_amd import vbdr
    vbdr.lib()
    return vbdr


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    return oracle


@pytest.fixture(scope="module")
def M():
    from oracle import mlp_ref
    return mlp_ref


def _build(V, O, m, g, k, seed, layout="fast", n_slices=4, n_pairs=60000, n_aip=600):
    rng = np.random.default_rng(seed)
    aips = rng.integers(0, 2**32, n_aip, dtype=np.uint64).astype(np.uint32)
    sk = V.Sketch(m, g, k, seed, layout)
    osk = O.Sketch(m, g, k, seed, O.GFAST if layout == "fast" else O.GSMALL)
    for _ in range(n_slices):
        sizes = rng.zipf(1.3, n_aip).clip(1, 5000)
        a = np.repeat(aips, sizes)
        b = rng.integers(0, 2**32, len(a), dtype=np.uint64).astype(np.uint32)
        pairs = np.stack([a, b], 1)[rng.permutation(len(a))][:n_pairs].astype(np.uint32)
        sk.scan_slice(V.to_device_u32(pairs.reshape(-1)))
        osk.scan(pairs)
        sk.advance_slice()
        osk.advance()
    hosts = np.concatenate([aips, rng.integers(0, 2**32, 37, dtype=np.uint64).astype(np.uint32)])
    return sk, osk, hosts


def _random_params(M, seed):
    p = M.init_params(seed)
    p[M.N_PARAMS - 1] = 5.0  # output bias: ln(1 + n) around e^5
    return p


@pytest.mark.parametrize("m,g,layout", [(20011, 64, "fast"), ((1 << 22) + 5, 256, "small")])
def test_features_bit_exact(V, O, M, m, g, layout):
    sk, osk, hosts = _build(V, O, m, g, 3, 7, layout)
    f = sk.features(V.to_device_u32(hosts)).cpu().numpy()
    _, hist = osk.estimate(hosts, with_hist=True)
    ref = M.features(hist, osk.state()["hist"], g, m).astype(np.float32)
    assert np.array_equal(f, ref)


@pytest.mark.parametrize("m,g,layout", [(20011, 64, "fast"), (50021, 256, "small"), ((1 << 22) + 5, 256, "fast")])
def test_learned_inference_matches_fp64(V, O, M, m, g, layout):
    sk, osk, hosts = _build(V, O, m, g, 3, 11, layout)
    params = _random_params(M, 3)
    mlp = V.MLP(params)
    hd = V.to_device_u32(hosts)
    out, fb = sk.estimate_learned(mlp, hd, with_fallback=True)
    out, fb = out.cpu().numpy(), fb.cpu().numpy()
    assert not fb.any()
    _, hist = osk.estimate(hosts, with_hist=True)
    feats = M.features(hist, osk.state()["hist"], g, m)
    y = M.infer(params, feats)
    y_gpu = np.log1p(out.astype(np.float64))
    ok = np.abs(y_gpu - y) <= 1e-4 * np.abs(y) + 2e-3
    ok |= (out == 0) & (np.expm1(y) <= 1e-3)  # clamped at 0
    assert ok.all(), (y_gpu[~ok][:5], y[~ok][:5])


def test_learned_fallback_is_the_plain_estimate(V, O, M):
    sk, osk, hosts = _build(V, O, 30011, 128, 4, 5)
    params = _random_params(M, 4)
    lo = np.full(67, -1e30, np.float32)
    hi = np.full(67, 1e30, np.float32)
    hi[66] = -100.0  # ln(g/m) outside the envelope: every host falls back
    mlp = V.MLP(params, lo, hi)
    hd = V.to_device_u32(hosts)
    out, fb = sk.estimate_learned(mlp, hd, with_fallback=True)
    assert fb.cpu().numpy().all()
    assert torch.equal(out, sk.estimate(hd))
    wide = V.MLP(params, lo, np.full(67, 1e30, np.float32))
    _, fb2 = sk.estimate_learned(wide, hd, with_fallback=True)
    assert not fb2.cpu().numpy().any()


@pytest.mark.parametrize("m,layout", [(30011, "fast"), ((1 << 22) + 5, "small")])
def test_learned_plain_above_keeps_large_counts(V, O, M, m, layout):
    """With a threshold, hosts whose plain estimate reaches it keep the plain
    estimate bit for bit (flag 2) and the others keep the network's output
    (flag 0); no threshold (inf) gives the network's output everywhere.  The
    second case takes the partitioned histogram path of large pools."""
    sk, osk, hosts = _build(V, O, m, 128, 4, 5, layout)
    params = _random_params(M, 4)
    hd = V.to_device_u32(hosts)
    plain = sk.estimate(hd)
    out0, fb0 = sk.estimate_learned(V.MLP(params), hd, with_fallback=True)
    assert not fb0.any()
    thr = float(torch.quantile(plain.double(), 0.6))
    cut = V.MLP(params, plain_above=thr)
    out1, fb1 = sk.estimate_learned(cut, hd, with_fallback=True)
    big = plain >= thr
    assert 0 < int(big.sum()) < len(hosts)
    assert torch.equal(fb1 == 2, big) and not (fb1 == 1).any()
    assert torch.equal(out1[big], plain[big]) and torch.equal(out1[~big], out0[~big])
    with pytest.raises(V.VbdrError):
        cut.set_plain_above(0.0)
    cut.set_plain_above(float("inf"))
    out2, fb2 = sk.estimate_learned(cut, hd, with_fallback=True)
    assert torch.equal(out2, out0) and not fb2.any()


def test_train_gradient_matches_fp64(V, M):
    rng = np.random.default_rng(0)
    params = _random_params(M, 9)
    feats = rng.uniform(0, 1, (300, 67)).astype(np.float32)
    feats[:, 66] = -6.0
    targets = rng.uniform(0, 9, 300).astype(np.float32)
    tr = V.Trainer(params, 1e-3)
    g, loss = tr.grad(torch.from_numpy(feats).cuda(), torch.from_numpy(targets).cuda())
    ref_loss, ref_g = M.loss_and_grad(params.astype(np.float64), feats.astype(np.float64), targets.astype(np.float64))
    g = g.cpu().numpy().astype(np.float64)
    assert abs(float(loss.cpu()[0]) - ref_loss) <= 1e-4 * ref_loss
    scale = np.abs(ref_g).max()
    np.testing.assert_allclose(g, ref_g, rtol=1e-3, atol=1e-4 * scale)


def test_train_step_is_adam(V, M):
    rng = np.random.default_rng(1)
    params = _random_params(M, 10)
    feats = rng.uniform(0, 1, (128, 67)).astype(np.float32)
    targets = rng.uniform(0, 9, 128).astype(np.float32)
    tr = V.Trainer(params, 1e-3)
    fd, td = torch.from_numpy(feats).cuda(), torch.from_numpy(targets).cuda()
    g, _ = tr.grad(fd, td)
    tr.step(fd, td)
    ref, _, _ = M.adam_step(params.astype(np.float64), np.zeros(M.N_PARAMS), np.zeros(M.N_PARAMS),
                            g.cpu().numpy().astype(np.float64), 1, lr=1e-3)
    np.testing.assert_allclose(tr.params(), ref, rtol=0, atol=1e-6)


def test_training_reduces_loss(V, M):
    rng = np.random.default_rng(2)
    feats = rng.uniform(0, 1, (4096, 67)).astype(np.float32)
    targets = (3 * feats[:, 0] + np.sin(4 * feats[:, 1]) + 2).astype(np.float32)
    fd, td = torch.from_numpy(feats).cuda(), torch.from_numpy(targets).cuda()
    tr = V.Trainer(M.init_params(1), 3e-3)
    first = float(tr.grad(fd, td)[1].cpu()[0])
    for _ in range(300):
        tr.step(fd, td)
    last = float(tr.grad(fd, td)[1].cpu()[0])
    assert last < 0.05 * first
