"""The oracle network's backward pass equals finite differences of its forward pass (FP64)."""
import numpy as np

from oracle import learned as OL


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    B, H, Wd, C1, C2, D3 = 2, 7, 9, 3, 4, 5
    H1, W1 = OL.out_hw(H), OL.out_hw(Wd)
    H2, W2 = OL.out_hw(H1), OL.out_hw(W1)
    D2 = H2 * W2 * C2
    n_out = 2 * H * Wd
    shapes = [(18, C1), (9 * C1, C2), (D2 + 1, D3), (D3, n_out)]
    params = [(rng.normal(0, 0.5, s), rng.normal(0, 0.1, s[1])) for s in shapes]
    X = rng.normal(0, 1, (B, H, Wd, 2))
    f = rng.normal(0, 1, B)
    T = rng.normal(0, 1, (B, n_out))

    def loss(ps):
        Y, _ = OL.forward(ps, X, f, bf=False)
        return OL.loss_and_grad_out(Y, T)[0]

    Y, cache = OL.forward(params, X, f, bf=False)
    _, dY = OL.loss_and_grad_out(Y, T)
    grads = OL.backward(params, cache, dY, bf=False)
    h = 1e-6
    for l in range(4):
        for which in (0, 1):
            P = params[l][which]
            idx = [tuple(rng.integers(0, s) for s in P.shape) for _ in range(4)]
            for ix in idx:
                plus = [(w.copy(), b.copy()) for w, b in params]
                minus = [(w.copy(), b.copy()) for w, b in params]
                plus[l][which][ix] += h
                minus[l][which][ix] -= h
                fd = (loss(plus) - loss(minus)) / (2 * h)
                assert abs(fd - grads[l][which][ix]) <= 1e-6 * (1 + abs(fd)), (l, which, ix)


def test_bf16_rounding_is_round_to_nearest_even():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.0e38])
    r = OL.bf16(x)
    assert r[0] == 1.0
    assert r[1] == 1.0            # tie -> even
    assert r[2] == 1.0 + 2 ** -7  # above the tie -> up
    assert r[3] == -2.5
