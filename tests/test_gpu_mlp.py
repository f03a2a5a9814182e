"""GPU tests of the warm-start network kernels against the float64 oracle
network, and of what the trained network gains over uniform starts."""
import numpy as np
import pytest
import torch

from oracle import mlp as omlp
from synth import scenes as sc

from gpu_helpers import TOL_F32, lib, oracle_pi, run_batched, split

pytestmark = pytest.mark.gpu


def bf16_bits(x):
    """float32 array -> (int16 bit tensor, float64 values) rounded to nearest even."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    vals = (r.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return torch.from_numpy(r.view(np.int16).copy()), vals


@pytest.mark.parametrize("shape", [(70, 130, 40), (200, 136, 208)])
@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
def test_gemm_bf16_matches_float64(ta, tb, shape):
    """Ragged against the 64 x 64 output tiles and the 64-deep K stages; the
    second shape has every leading dimension a multiple of 8 elements, so
    that most tile loads take the 16-byte path and the edges the element
    path."""
    from paper_2509_20500_amd.warmstart import gemm_bf16
    lib()
    rng = np.random.default_rng(3)
    M, N, K = shape
    a = rng.normal(size=(K, M) if ta else (M, K)).astype(np.float32)
    b = rng.normal(size=(N, K) if tb else (K, N)).astype(np.float32)
    A, av = bf16_bits(a)
    B, bv = bf16_bits(b)
    C = gemm_bf16(A.cuda(), B.cuda(), ta, tb).cpu().numpy()
    ref = (av.T if ta else av) @ (bv.T if tb else bv)
    assert np.max(np.abs(C - ref)) <= 1e-5 * np.max(np.abs(ref))


def _net(seed=0, max_batch=64):
    from paper_2509_20500_amd.warmstart import WarmStartMLP
    lib()
    return WarmStartMLP(max_batch=max_batch, seed=seed)


def _oracle_params(net):
    """The GPU network's weights as the GEMMs see them (bfloat16 values)."""
    t = net.tensors(net.params.detach().cpu())
    p = {}
    for k, v in t.items():
        x = v.numpy()
        p[k] = bf16_bits(x)[1].reshape(x.shape) if k.startswith("W") else x.astype(np.float64)
    p["W1"] = p["W1"][:omlp.IN]
    return p


def test_features_match_oracle():
    """Features to float32 rounding; the pulse bins exactly (both sides
    divide in float64), including a pulse on a bin edge."""
    net = _net()
    scenes = np.concatenate([sc.batched_uniform(20, seed=7), sc.batched_uneven(20, seed=8),
                             sc.scene(period=50.0, center=25.0), sc.scene(period=100.0, center=0.0)])
    f, k = net.features(scenes)
    ref = np.stack([omlp.features(s) for s in scenes])
    assert np.max(np.abs(f.cpu().numpy() - ref)) < 1e-6
    assert np.array_equal(k.cpu().numpy(), [omlp.pulse_bin(s) for s in scenes])


def test_flux_prior_matches_oracle():
    net = _net()
    scenes = np.concatenate([sc.batched_uniform(16, seed=7), sc.batched_uneven(16, seed=8),
                             sc.scene(signal=0.0, background=0.4), sc.scene(signal=2.0, background=0.0)])
    g = net.flux_prior(scenes).cpu().numpy().astype(np.float64)
    with np.errstate(divide="ignore"):
        ref = np.stack([omlp.flux_prior(s) for s in scenes])
    # the oracle forms lambda itself, which loses digits below the smallest
    # normal double (a log below about -708) and underflows to zero (log
    # -inf) more than about 38 sigma from a pulse without background; the
    # kernel works in the log domain and keeps those logits finite and far
    # below
    ok = ref > -700.0
    assert np.all(np.abs(g[ok] - ref[ok]) <= 1e-6 * np.maximum(1.0, np.abs(ref[ok])))
    assert np.all(np.isfinite(g)) and np.all(g[~ok] < -690.0)


@pytest.mark.parametrize("with_prior,with_shift", [(False, False), (True, False), (True, True)])
def test_forward_and_gradients_match_oracle(with_prior, with_shift):
    """Batch 300: the weight gradients split the batch over blocks (K = 300
    in chunks of 64 to 128 rows) and add the partial products; with the
    pulse-bin rotation, each bin's error goes back to the output it took."""
    net = _net(seed=1, max_batch=300)
    rng = np.random.default_rng(2)
    B = 300
    scenes = sc.batched_uniform(B, seed=9)
    feat, shift = net.features(scenes)
    prior = net.flux_prior(scenes) if with_prior else None
    shift = shift if with_shift else None
    T = rng.uniform(size=(B, omlp.OUT)).astype(np.float32)
    T /= T.sum(axis=1, keepdims=True)
    target = torch.from_numpy(T).cuda()
    q = net.predict(feat, prior, shift).cpu().numpy()
    P = _oracle_params(net)
    X = bf16_bits(feat.cpu().numpy())[1]
    po = None if prior is None else prior.cpu().numpy().astype(np.float64)
    ko = None if shift is None else shift.cpu().numpy()
    Qo, _ = omlp.forward(P, X, po, ko)
    assert np.max(np.abs(q - Qo)) <= 2e-2 * np.max(Qo)
    assert np.allclose(q.sum(axis=1), 1.0, atol=1e-5)
    loss = torch.empty(B, dtype=torch.float32, device="cuda")
    net.backward(feat, target, loss, prior=prior, shift=shift)
    torch.cuda.synchronize()
    lo = -(T * np.log(Qo)).sum(axis=1)
    assert np.max(np.abs(loss.cpu().numpy() - lo)) <= 1e-2 * np.max(np.abs(lo))
    G = net.tensors(net.grads.detach().cpu())
    Go = omlp.grads(P, X, T.astype(np.float64), po, ko)
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        g = G[k].numpy().astype(np.float64)
        if k == "W1":
            assert np.all(g[omlp.IN:] == 0)  # padded inputs get no gradient
            g = g[:omlp.IN]
        rel = np.linalg.norm(g - Go[k]) / np.linalg.norm(Go[k])
        assert rel < 3e-2, (k, rel)


def test_backward_reads_shuffled_rows_in_place():
    """A mini-batch named by row indices gives the same loss and gradients,
    bit for bit, as the same rows gathered beforehand."""
    net = _net(seed=4, max_batch=256)
    scenes = sc.batched_uniform(600, seed=12)
    feat, shift = net.features(scenes)
    prior = net.flux_prior(scenes)
    rng = np.random.default_rng(3)
    T = rng.uniform(size=(600, omlp.OUT)).astype(np.float32)
    T /= T.sum(axis=1, keepdims=True)
    target = torch.from_numpy(T).cuda()
    idx = torch.from_numpy(rng.permutation(600)[:256].astype(np.int32)).cuda()
    loss_a = torch.empty(256, dtype=torch.float32, device="cuda")
    net.backward(feat, target, loss_a, prior=prior, shift=shift, rows=idx)
    torch.cuda.synchronize()
    ga = net.grads.detach().clone()
    il = idx.long()
    loss_b = torch.empty(256, dtype=torch.float32, device="cuda")
    net.backward(feat[il].contiguous(), target[il].contiguous(), loss_b, prior=prior[il].contiguous(),
                 shift=shift[il].contiguous())
    torch.cuda.synchronize()
    assert torch.equal(loss_a, loss_b)
    assert torch.equal(ga, net.grads)


def test_adam_step_matches_formula():
    net = _net(seed=2)
    scenes = sc.batched_uniform(32, seed=10)
    feat, _ = net.features(scenes)
    T = torch.full((32, omlp.OUT), 1.0 / omlp.OUT, device="cuda")
    w0 = net.params.detach().cpu().numpy().astype(np.float64)
    net.backward(feat, T)
    g = net.grads.detach().cpu().numpy().astype(np.float64)
    net.adam(1e-3)
    torch.cuda.synchronize()
    w1 = net.params.detach().cpu().numpy().astype(np.float64)
    m = 0.1 * g
    v = 0.001 * g * g
    ref = w0 - 1e-3 * (m / 0.1) / (np.sqrt(v / 0.001) + 1e-8)
    assert np.max(np.abs(w1 - ref)) < 1e-6


def test_checkpoint_round_trip(tmp_path):
    net = _net(seed=3)
    feat, _ = net.features(sc.batched_uniform(64, seed=11))
    T = torch.full((64, omlp.OUT), 1.0 / omlp.OUT, device="cuda")
    for _ in range(3):
        net.backward(feat, T)
        net.adam(1e-3)
    path = tmp_path / "ckpt.pt"
    torch.save(net.state_dict(), path)
    other = _net(seed=99)
    other.load_state_dict(torch.load(path, weights_only=True))
    assert torch.equal(other.predict(feat), net.predict(feat))
    # resuming continues bit for bit
    for n in (net, other):
        n.backward(feat, T)
        n.adam(1e-3)
    assert torch.equal(other.params, net.params)


def test_trained_warm_start_saves_sweeps():
    """Train on PDFs the solver itself produces (uniform-workload sampling),
    the network correcting the flux start (its logits, in the frame of the
    pulse bin, added to the log of lambda / sum(lambda)), then solve held-out
    pixels from the network's prediction: fewer sweeps than from the flux
    start (the method's own start without the network) and than from
    uniform, same accuracy against the oracle."""
    d = lib()
    from paper_2509_20500_amd.warmstart import WarmStartMLP
    train = sc.warm_start_train(n_pixels=16384, seed=5)
    pi_t, info_t, _ = run_batched(train, "f32")
    assert np.all(info_t["status"] == 0)
    targets = torch.from_numpy(pi_t.astype(np.float32).reshape(-1, omlp.OUT)).cuda()
    targets /= targets.sum(dim=1, keepdim=True)
    net = WarmStartMLP(max_batch=1024, seed=0, zero_output=True)
    feat, shift = net.features(train)
    prior = net.flux_prior(train)
    hist = net.fit(feat, targets, epochs=30, lr=2e-3, prior=prior, shift=shift)
    assert hist[-1] < hist[0]
    held = sc.warm_start_eval(n_pixels=512, seed=6)
    feat_h, shift_h = net.features(held)
    x0 = net.predict(feat_h, net.flux_prior(held), shift_h).reshape(-1)
    flux = d.opts(tol=1e-6)
    flux.flags |= d.DTM_FLAG_START_FLUX
    pi_u, info_u, off = run_batched(held, "f32")
    pi_f, info_f, _ = run_batched(held, "f32", solve_opts=flux)
    pi_w, info_w, _ = run_batched(held, "f32", x0=x0)
    assert np.all(info_w["status"] == 0) and np.all(info_f["status"] == 0)
    assert not np.any(info_w["flags"] & (d.DTM_INFO_WARM_REJECTED | d.DTM_INFO_RESTARTED))
    x0n = x0.cpu().numpy().astype(np.float64)
    l1_start = np.mean([np.abs(x0n[off[p]:off[p + 1]] - split(pi_u, off)[p]).sum() for p in range(len(held))])
    print("mean sweeps uniform %.3f flux %.3f warm %.3f; mean L1(x0, pi) %.4f; loss %.4f -> %.4f"
          % (info_u["iterations"].mean(), info_f["iterations"].mean(), info_w["iterations"].mean(), l1_start,
             hist[0], hist[-1]))
    assert info_w["iterations"].mean() < info_f["iterations"].mean() < info_u["iterations"].mean()
    rng = np.random.default_rng(0)
    for p in rng.choice(len(held), 24, replace=False):
        assert np.abs(split(pi_w, off)[p] - oracle_pi(held[p])).sum() <= TOL_F32
