"""Learned-start network: bf16 GPU kernels against the FP64 CPU oracle of the same network."""
import numpy as np
import pytest

from paper_1709_08803_amd import workloads as W
from oracle import learned as OL

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def bim():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    from paper_1709_08803_amd import bim as B
    B.lib()
    return B


def _bf16_tensor(x):
    """float array -> int16 tensor of bf16 bits (round to nearest even, as the kernels do)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    return torch.as_tensor(u.view(np.int16).copy(), device="cuda")


def _net_and_params(bim, N, M, B, seed, in_linear=1):
    net = bim.LearnedNet(N, M, seed=seed, max_batch=B, C1=8, C2=16, D3=64, in_linear=in_linear)
    params = []
    for l in range(4):
        Wf, b, _, _ = net.get(l)
        a = net.arch
        fan_out = [a.C1, a.C2, a.D3, 2 * M * N][l]
        b = np.random.default_rng(seed + l).normal(0, 0.05, b.shape).astype(np.float32)
        net.set(l, None, b)
        params.append((Wf.reshape(-1, fan_out).astype(np.float64), b.astype(np.float64)))
    return net, params


def _inputs(N, M, B, seed, C=4):
    rng = np.random.default_rng(seed)
    X = rng.normal(0, 1, (B, M, N, C)).astype(np.float32)
    f = rng.normal(0, 1, B).astype(np.float32)
    T = rng.normal(0, 1, (B, 2 * M * N)).astype(np.float32)
    return X, f, T


@pytest.mark.parametrize("N,M,B,lin", [(21, 9, 3, 0), (33, 15, 5, 1)])
def test_forward_matches_fp64_oracle(bim, N, M, B, lin):
    net, params = _net_and_params(bim, N, M, B, 1, lin)
    X, f, _ = _inputs(N, M, B, 2, net.in_channels)
    Y = net.forward(_bf16_tensor(X), torch.as_tensor(f, device="cuda")).cpu().numpy()
    Yref, _ = OL.forward(params, X, f)
    err = np.abs(Y - Yref).max() / np.abs(Yref).max()
    print("forward rel err", err)
    assert err < 2e-3


@pytest.mark.parametrize("N,M,B,lin", [(21, 9, 3, 0), (33, 15, 5, 1)])
def test_gradients_match_fp64_oracle(bim, N, M, B, lin):
    net, params = _net_and_params(bim, N, M, B, 3, lin)
    X, f, T = _inputs(N, M, B, 4, net.in_channels)
    loss = net.train_step(_bf16_tensor(X), torch.as_tensor(f, device="cuda"), torch.as_tensor(T, device="cuda"),
                          lr=0.0, update=False)
    Y, cache = OL.forward(params, X, f)
    lref, dY = OL.loss_and_grad_out(Y, T)
    grads = OL.backward(params, cache, dY)
    assert abs(loss - lref) < 1e-3 * lref
    for l in range(4):
        _, _, gw, gb = net.get(l)
        rw = grads[l][0].reshape(-1)
        rb = grads[l][1]
        ew = np.abs(gw - rw).max() / (np.abs(rw).max() + 1e-30)
        eb = np.abs(gb - rb).max() / (np.abs(rb).max() + 1e-30)
        print("layer", l, "grad rel err", ew, eb)
        assert ew < 2e-2 and eb < 2e-2


def test_training_reduces_loss(bim):
    N, M, B = 21, 9, 8
    net = bim.LearnedNet(N, M, seed=5, max_batch=B, C1=8, C2=16, D3=64)
    X, f, T = _inputs(N, M, B, 6, net.in_channels)
    T = 0.1 * np.tanh(T).astype(np.float32)
    Xd, fd, Td = _bf16_tensor(X), torch.as_tensor(f, device="cuda"), torch.as_tensor(T, device="cuda")
    first = net.train_step(Xd, fd, Td, lr=1e-3)
    for _ in range(200):
        last = net.train_step(Xd, fd, Td, lr=1e-3)
    print("loss", first, "->", last)
    assert last < 0.2 * first


def test_learned_start_is_linear_start_plus_correction(bim):
    p = W.tiny(0.8)
    dp = bim.DeviceProblem(p)
    net = bim.LearnedNet(p.N, p.M, seed=7, max_batch=1, C1=8, C2=16, D3=32)
    uld = bim.linear_start(dp)
    ul = uld.cpu().numpy()
    u = net.infer_start(dp).cpu().numpy()
    X0, f = net.make_input(dp, uld)
    # the input holds the topography, F and the linear start's x-derivative planes
    Xh = X0.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    Xh = Xh.view(np.float32).reshape(p.M, p.N, 4)
    nb = (p.N + 1) * p.M
    zx = ul[:nb].reshape(p.M, p.N + 1)[:, 1:]
    assert np.allclose(Xh[..., 0], (p.beta + 1) / 0.3, rtol=1e-2, atol=1e-3)
    assert np.allclose(Xh[..., 2], zx / 0.2, rtol=1e-2, atol=1e-3)
    Y = net.forward(X0, f).cpu().numpy()[0] * net.arch.out_scale
    for fld in range(2):
        blk = (u - ul)[fld * nb:(fld + 1) * nb].reshape(p.M, p.N + 1)
        assert np.allclose(blk[:, 1:], Y[fld * p.N * p.M:(fld + 1) * p.N * p.M].reshape(p.M, p.N), atol=1e-12)
        assert np.all(blk[:, 0] == 0.0)  # upstream values stay the linear start's
    assert np.array_equal(u[2 * nb:], ul[2 * nb:])


@pytest.mark.timeout(600)
def test_trained_network_reduces_newton_iterations(bim):
    # End to end on a family of 31 x 11 problems (Gaussian and two-bump bottoms,
    # F in [0.8, 1.8]): the method's own converged solutions (batched FP64 JFNK)
    # train the network on the GPU; on held-out problems Newton from the learned
    # start needs fewer iterations on average than from the linear start, and
    # both starts reach the same discrete solution.
    from paper_1709_08803_amd import learned_start as LS
    fam = dict(kinds=(0, 2), froude=(0.8, 1.8), height=(0.1, 0.3), width=(0.7, 1.5), fixed_n=31,
               domain=(-15.0, 15.0, 10.0))
    train_p = W.sweep_instances(768, seed=51, **fam)
    test_p = W.sweep_instances(48, seed=52, **fam)
    net = bim.LearnedNet(31, 11, seed=1, max_batch=64, C1=16, C2=32, D3=512, in_linear=1)
    data = LS.generate(train_p, net, batch=64, log=None)
    print("converged training solutions", len(data))
    assert len(data) >= 500
    hist = LS.train(net, data, epochs=600, batch=32, lr=1e-3, log=None)
    print("loss", hist[0], "->", hist[-1])
    assert hist[-1] < 0.05 * hist[0]
    ev = LS.evaluate(net, test_p)
    s = ev["summary"]
    print(s)
    assert s["both_converged"] >= 36
    assert s["learned_newton_mean"] < s["linear_newton_mean"]
    assert s["max_dx_between_solutions"] <= 1e-8


@pytest.mark.timeout(600)
def test_learned_start_solutions_at_121x41_match_the_oracle(bim):
    # The learned-start configuration (121 x 41, the sweep distribution): a network
    # trained on the GPU on the method's own solutions of seeded sweep problems; on
    # held-out problems of the experiment's test set, Newton from the learned start
    # (falling back to the linear start after 8 steps, as the experiment does) must
    # reach the FP64 oracle's own converged solution (tests/golden/
    # make_learned_heldout.py, oracle/ only).
    import os
    from oracle import residual as R
    from paper_1709_08803_amd import learned_start as LS
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "learned_heldout_121x41.npz"))
    net = bim.LearnedNet(121, 41, seed=0, max_batch=32, D3=256)
    data = LS.generate(W.sweep_instances(96, seed=1, fixed_n=121), net, batch=32, log=None)
    assert len(data) >= 32
    LS.train(net, data, epochs=40, batch=32, log=None)
    probs = W.sweep_instances(8, seed=2, fixed_n=121)
    for i, F, uref in zip(g["index"], g["froude"], g["u"]):
        p = probs[int(i)]
        assert p.froude == F
        dp = bim.DeviceProblem(p)
        P = bim.Preconditioner(dp)
        u = net.infer_start(dp, P)
        rep = bim.solve(dp, u, P, ftol=1e-11, max_newton=8, check=False)
        fallback = rep["status"] != 0
        if fallback:
            u = bim.linear_start(dp, P)
            rep = bim.solve(dp, u, P, ftol=1e-11)
        P.close()
        uh = u.cpu().numpy()
        z, zr = R.reconstruct(p, uh), R.reconstruct(p, uref)
        dz = np.abs(z.zeta - zr.zeta).max()
        print(f"held-out {int(i)} F = {F:.3f}: Newton {rep['newton_iters']} fallback {fallback} max|dzeta| {dz:.2e}")
        assert rep["status"] == 0 and dz <= 1e-9
        assert np.abs(R.residual(p, uh)).max() <= 1e-10  # a root of the oracle's discrete system


# The kernels keep inputs, weights, activations and the gradients fed to products
# in bf16 (8 significant bits, unit roundoff u = 2^-8 relative to the spacing),
# with FP32 accumulation.  Against the plain FP64 network (no rounding at all)
# each layer's operands carry relative errors of order u, so the output differs
# by a few u in the 2-norm: bound 4u.  The gradient of the linear output layer
# follows the output error (4u); the three layers before it sit behind ReLUs
# whose activation pattern flips where rounding moves a pre-activation across
# zero, so their bound is on direction (cosine >= 0.98) and on a 2-norm error
# of 0.25.  (The plain FP64 network under the same rounding, computed on the
# CPU, stays within these bounds: forward 4-6e-3, output layer 4-5e-3, the
# others 4e-3 to 0.14; on the GPU the ReLU layers measured 5e-3 to 4e-2.)
BF16_U = 2.0 ** -8


@pytest.mark.parametrize("N,M,B,lin", [(21, 9, 3, 0), (33, 15, 5, 1), (121, 41, 4, 1)])
def test_network_within_bf16_bound_of_plain_fp64(bim, N, M, B, lin):
    net, params = _net_and_params(bim, N, M, B, 11, lin)
    X, f, T = _inputs(N, M, B, 12, net.in_channels)
    Xd, fd = _bf16_tensor(X), torch.as_tensor(f, device="cuda")
    Y = net.forward(Xd, fd).cpu().numpy().astype(np.float64)
    Yref, cache = OL.forward(params, X, f, bf=False)
    ef = np.linalg.norm(Y - Yref) / np.linalg.norm(Yref)
    print("forward 2-norm rel err vs plain FP64", ef)
    assert ef <= 4 * BF16_U
    net.train_step(Xd, fd, torch.as_tensor(T, device="cuda"), lr=0.0, update=False)
    _, dY = OL.loss_and_grad_out(Yref, T)
    grads = OL.backward(params, cache, dY, bf=False)
    for l in range(4):
        _, _, gw, gb = net.get(l)
        g = np.concatenate([gw.astype(np.float64), gb.astype(np.float64)])
        r = np.concatenate([grads[l][0].reshape(-1), grads[l][1]])
        e = np.linalg.norm(g - r) / np.linalg.norm(r)
        cos = float(g @ r / (np.linalg.norm(g) * np.linalg.norm(r)))
        print("layer", l, "grad 2-norm rel err", e, "cos", cos)
        if l == 3:
            assert e <= 4 * BF16_U
        else:
            assert cos >= 0.98 and e <= 0.25
