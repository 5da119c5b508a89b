"""Pins of the FP64 network reference: gradients vs central differences,
window geometry vs direct indexing, bf16 rounding vs known values."""
import numpy as np

from oracle import net_ref


def small_params(rng, K=20, H=7, N=5, m=3):
    return {"W1": rng.normal(size=(K, H)), "b1": rng.normal(size=H) * 0.1,
            "W2": rng.normal(size=(H, H)) * 0.5, "b2": rng.normal(size=H) * 0.1,
            "W3": rng.normal(size=(H, H)) * 0.5, "b3": rng.normal(size=H) * 0.1,
            "W4": rng.normal(size=(H, N)), "b4": rng.normal(size=N) * 0.1,
            "Ws": rng.normal(size=(m, K, N)) * 0.2}


def test_backward_matches_central_differences():
    rng = np.random.default_rng(0)
    p = small_params(rng)
    X = rng.normal(size=(9, 20)); T = rng.normal(size=(9, 5))
    Xs = X + 0.1 * rng.normal(size=X.shape)      # the linear map may read other rows
    Y, cache = net_ref.forward(p, X, Xs)
    g = net_ref.backward(p, cache, Y, T)
    eps = 1e-6
    for k, w in p.items():
        fd = np.zeros_like(w)
        for idx in np.ndindex(w.shape):
            old = w[idx]
            w[idx] = old + eps; lp = net_ref.mse(net_ref.forward(p, X, Xs)[0], T)
            w[idx] = old - eps; lm = net_ref.mse(net_ref.forward(p, X, Xs)[0], T)
            w[idx] = old
            fd[idx] = (lp - lm) / (2 * eps)
        assert np.abs(fd - g[k]).max() <= 1e-6 * max(1.0, np.abs(fd).max()), k


def test_features_geometry():
    ns, L, win = 64, 4, 32
    rng = np.random.default_rng(1)
    x0 = rng.uniform(0, 0.2, (2, ns * ns)); xr = rng.uniform(-0.3, 0.3, (2, ns * ns))
    W = net_ref.features(x0, xr, ns, L, win, planes=5)
    ww = win * win
    assert W.shape == (32, 5 * ww + 16)
    # actuator p = 5 (row 1, col 1): window starts at node (16 - 8, 16 - 8)
    b, p = 1, 5
    row = W[b * 16 + p]
    img = x0[b].reshape(ns, ns); ref = xr[b].reshape(ns, ns)
    xt = img[8, 8] / 0.1 - 1.0; rt = ref[8, 8] / 0.3
    assert row[0] == xt and row[ww] == rt
    assert row[2 * ww] == xt * xt - 1.0 / 3.0 and row[3 * ww] == xt * rt
    assert row[4 * ww] == rt * rt - 1.0 / 3.0
    assert row[win - 1] == img[8, 8 + win - 1] / 0.1 - 1.0
    assert row[ww + win] == ref[9, 8] / 0.3
    # actuator 0's window starts 8 nodes outside the grid: every plane is zero there
    for c in range(5):
        assert W[0, c * ww] == 0.0
    assert W[0, 8 * win + 8] == x0[0].reshape(ns, ns)[0, 0] / 0.1 - 1.0
    assert W[b * 16 + p, 5 * ww + p] == 1.0 and W[b * 16 + p, 5 * ww:].sum() == 1.0
    # two planes: the first two of the five
    W2 = net_ref.features(x0, xr, ns, L, win, planes=2)
    np.testing.assert_array_equal(W2[:, :2 * ww], W[:, :2 * ww])


def test_linear_map_uses_each_rows_actuator():
    rng = np.random.default_rng(2)
    Ws = rng.normal(size=(4, 6, 3)); X = rng.normal(size=(8, 6))
    Y = net_ref.skip(Ws, X)
    for r in range(8):
        np.testing.assert_allclose(Y[r], X[r] @ Ws[r % 4], rtol=1e-14)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2**-8, 1.0 + 2**-7 + 2**-9, 3.14159265, -2.5e-3,
                     1.0 + 2**-7 + 3 * 2**-9, 1.0 + 3 * 2**-8])
    r = net_ref.bf16_round(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                      # tie to even (down)
    assert r[2] == 1.0 + 2**-7              # quarter ulp: down
    assert r[5] == 1.0 + 2 * 2**-7          # three quarters: up
    assert r[6] == 1.0 + 2 * 2**-7          # tie to even (up)
    assert abs(r[3] - 3.140625) < 1e-12
    assert abs(r[4] / vals[4] - 1) < 2**-8
