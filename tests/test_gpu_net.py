"""GPU tests of the warm-start network kernels against the FP64 reference."""
import numpy as np
import pytest

from nmpc_inputs import make_batch, make_problem

from oracle import net_ref

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ws():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2004_02484_amd import warmstart
    return warmstart


def bf16_bits(a):
    r = net_ref.bf16_round(a).astype(np.float32)
    return (r.view(np.uint32) >> 16).astype(np.uint16).view(np.int16), r.astype(np.float64)


@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("M,N,K", [(77, 45, 83), (128, 64, 64), (5, 130, 200)])
def test_gemm_layouts(ws, ta, tb, M, N, K):
    import torch
    rng = np.random.default_rng(M * 1000 + N + K)
    A = rng.normal(size=(K, M) if ta else (M, K)); Bm = rng.normal(size=(N, K) if tb else (K, N))
    Ab, Af = bf16_bits(A); Bb, Bf = bf16_bits(Bm)
    bias = rng.normal(size=N)
    C0 = rng.normal(size=(M, N))
    ref = (Af.T if ta else Af) @ (Bf.T if tb else Bf)
    dA = torch.tensor(Ab, device="cuda"); dB = torch.tensor(Bb, device="cuda")
    C = torch.tensor(C0.astype(np.float32), device="cuda")
    dbias = torch.tensor(bias.astype(np.float32), device="cuda")
    Cb = torch.empty((M, N), dtype=torch.int16, device="cuda")
    ws.gemm(dA, dB, M, N, K, ta=ta, tb=tb, C=C, beta=0.5, bias=dbias, relu=True, Cb=Cb)
    torch.cuda.synchronize()
    want = np.maximum(ref + 0.5 * C0.astype(np.float32) + bias.astype(np.float32), 0.0)
    got = C.cpu().numpy().astype(np.float64)
    scale = np.abs(Af).max() * np.abs(Bf).max() * K
    assert np.abs(got - want).max() <= 2e-6 * scale
    np.testing.assert_allclose(ws.bf16_to_float(Cb), net_ref.bf16_round(got), rtol=0, atol=0)


@pytest.mark.parametrize("ta", [0, 1])
@pytest.mark.parametrize("M,N,K,G,S", [(77, 45, 83, 1, 1), (130, 40, 200, 3, 1), (5, 70, 33, 2, 1),
                                       (130, 40, 200, 3, 4), (77, 45, 83, 2, 7)])
def test_gemm_f32_groups(ws, ta, M, N, K, G, S):
    """Grouped fp32 products against float64 products of the same float32 operands,
    with the operands of each group interleaved the way the network stores rows."""
    import torch
    rng = np.random.default_rng(M * 100 + N + K + G)
    # group g: rows g, g + G, ... of a row-interleaved A; B blocks consecutive; C interleaved
    rowsA = (K if ta else M) * G
    wA = M if ta else K
    A = rng.normal(size=(rowsA, wA)).astype(np.float32)
    Bm = rng.normal(size=(G, K, N)).astype(np.float32)
    C0 = rng.normal(size=(M * G, N)).astype(np.float32)
    dA = torch.tensor(A, device="cuda"); dB = torch.tensor(Bm, device="cuda")
    C = torch.tensor(C0, device="cuda")
    work = torch.empty(G * S * M * N, dtype=torch.float32, device="cuda") if S > 1 else None
    ws.gemm_f32(dA, dB, M, N, K, C, ta=ta, lda=G * wA, ldb=N, ldc=G * N, sa=wA, sb=K * N, sc=N,
                groups=G, beta=0.5, ksplit=S, work=work)
    torch.cuda.synchronize()
    got = C.cpu().numpy().astype(np.float64)
    for g in range(G):
        Ag = A[g::G].astype(np.float64)
        opA = Ag.T if ta else Ag
        want = opA @ Bm[g].astype(np.float64) + 0.5 * C0[g::G].astype(np.float64)
        scale = np.abs(opA).max() * np.abs(Bm[g]).max() * np.sqrt(K)
        assert np.abs(got[g::G] - want).max() <= 1e-6 * scale


@pytest.mark.parametrize("ta", [0, 1])
def test_gemm_f64_and_acc64_groups(ws, ta):
    """fp64 grouped products (alpha, beta, separate Cin) and fp32-operand products
    with fp64 sums, against float64 numpy on the same operands."""
    import torch
    rng = np.random.default_rng(11 + ta)
    M, N, K, G = 70, 66, 90, 3
    wA = M if ta else K
    A = rng.normal(size=((K if ta else M) * G, wA))
    Bm = rng.normal(size=(G, K, N))
    Cin = rng.normal(size=(M * G, N))
    dA = torch.tensor(A, device="cuda"); dB = torch.tensor(Bm, device="cuda")
    dCin = torch.tensor(Cin, device="cuda"); C = torch.empty_like(dCin)
    ws.gemm_f64(dA, dB, M, N, K, C, ta=ta, lda=G * wA, ldb=N, ldc=G * N, sa=wA, sb=K * N, sc=N,
                groups=G, alpha=-1.5, beta=2.0, Cin=dCin)
    A32, B32 = A.astype(np.float32), Bm.astype(np.float32)
    C2 = torch.tensor(Cin, device="cuda")
    ws.gemm_f32_acc64(torch.tensor(A32, device="cuda"), torch.tensor(B32, device="cuda"), M, N, K,
                      C2, ta=ta, lda=G * wA, ldb=N, ldc=G * N, sa=wA, sb=K * N, sc=N, groups=G,
                      beta=1.0)
    torch.cuda.synchronize()
    got, got2 = C.cpu().numpy(), C2.cpu().numpy()
    for g in range(G):
        opA = A[g::G].T if ta else A[g::G]
        want = -1.5 * opA @ Bm[g] + 2.0 * Cin[g::G]
        np.testing.assert_allclose(got[g::G], want, rtol=0, atol=1e-12 * np.abs(want).max())
        opA32 = (A32[g::G].T if ta else A32[g::G]).astype(np.float64)
        want2 = opA32 @ B32[g].astype(np.float64) + Cin[g::G]
        np.testing.assert_allclose(got2[g::G], want2, rtol=0, atol=1e-12 * np.abs(want2).max())


def test_linear_fit_matches_ridge_solution(ws):
    """The per-actuator normal-equation fit on a small lattice against numpy's
    solve of the same ridge-regularized normal equations (predictions compared:
    the weights themselves are ill-determined along the reference's few modes)."""
    import torch
    from nmpc_inputs import make_problem as mk
    P = mk("grid", ns=16, N=5, lattice=2)
    x0, xr = make_batch(P, range(600))
    rng = np.random.default_rng(3)
    u = rng.normal(size=(600, 5, 4))
    net = ws.PatchNet(N=5, ns=16, lattice=2, win=12, hidden=32)
    dx0, dxr = torch.tensor(x0, device="cuda"), torch.tensor(xr, device="cuda")
    du = torch.tensor(u, device="cuda")
    res = net.fit_linear(dx0, dxr, du, batch=256, ridge_rel=1e-6, iters=45)
    assert max(res) < 1e-3
    Ws = net.get("Ws").astype(np.float64)
    X = net_ref.features(x0, xr, 16, 2, 12, 5, net.K0p).astype(np.float32).astype(np.float64)
    T = (u / ws.U_SCALE).transpose(0, 2, 1).reshape(-1, 5)
    for p in range(4):
        Xp, Tp = X[p::4], T[p::4]
        G = Xp.T @ Xp
        G += 1e-6 * np.trace(G) / G.shape[0] * np.eye(G.shape[0])
        Wr = np.linalg.solve(G, Xp.T @ Tp)
        pr, prr = Xp @ Ws[p], Xp @ Wr
        assert np.abs(pr - prr).max() <= 1e-5 * np.abs(prr).max()


def test_features_match_reference(ws):
    import torch
    from paper_2004_02484_amd.warmstart import _lib, _p, _stream
    P = make_problem("c1")
    x0, xr = make_batch(P, [3, 4])
    net = ws.PatchNet(hidden=32)
    ld = net.K0p
    Xf = torch.full((32, ld), 7.0, dtype=torch.float32, device="cuda")
    Xb = torch.empty((32, ld), dtype=torch.int16, device="cuda")
    dx0, dxr = torch.tensor(x0, device="cuda"), torch.tensor(xr, device="cuda")   # keep alive
    rc = _lib().nmpc_net_features(_p(dx0), _p(dxr), 2, 64, 4, 32, 5, _p(Xf), _p(Xb), ld, _stream())
    assert rc == 0
    torch.cuda.synchronize()
    full = net_ref.features(x0, xr, 64, 4, 32, 5, ld)
    got = Xf.cpu().numpy().astype(np.float64)
    # fp32 rounding of the fp64 feature values (products rounded once in fp64 first)
    np.testing.assert_allclose(got, full.astype(np.float32).astype(np.float64), rtol=2**-23, atol=0)
    np.testing.assert_array_equal(ws.bf16_to_float(Xb), net_ref.bf16_round(got))
    # the two-plane layout is a prefix of the five-plane one (bf16 only)
    ld2 = 2 * 32 * 32 + 16
    Xb2 = torch.empty((32, ld2), dtype=torch.int16, device="cuda")
    rc = _lib().nmpc_net_features(_p(dx0), _p(dxr), 2, 64, 4, 32, 2, None, _p(Xb2), ld2, _stream())
    assert rc == 0
    torch.cuda.synchronize()
    want2 = net_ref.bf16_round(net_ref.features(x0, xr, 64, 4, 32, 2, ld2).astype(np.float32))
    np.testing.assert_array_equal(ws.bf16_to_float(Xb2), want2)


def _net_case(ws, hidden=64, seed=3, seeds=(7, 8, 9)):
    import torch
    P = make_problem("c1")
    x0, xr = make_batch(P, list(seeds))
    net = ws.PatchNet(hidden=hidden, seed=seed, max_count=8)
    rng = np.random.default_rng(5)
    net.set_param("Ws", rng.normal(size=net.shape("Ws")).astype(np.float32) * 0.02)
    u_t = rng.normal(size=(len(seeds), 40, 16))
    dev = [torch.tensor(a, device="cuda") for a in (x0, xr, u_t)]
    return net, x0, xr, u_t, dev


def test_forward_and_gradients_match_reference(ws):
    """Whole-network output, loss and gradients against the FP64 reference
    network on the GPU's parameters (bf16 rounding of the layer operands is
    the only model difference, so the bar is a few 1e-3 relative)."""
    net, x0, xr, u_t, (dx0, dxr, du) = _net_case(ws)
    loss = net.backward(dx0, dxr, du)
    Y = net.get("Y").astype(np.float64)
    p = {k: v.astype(np.float64) for k, v in net.state().items()}
    for k in list(p):
        if k.startswith("W") and k != "Ws":
            p[k] = net_ref.bf16_round(p[k])
    X = net_ref.features(x0, xr, 64, 4, 32, 5, net.K0p).astype(np.float32).astype(np.float64)
    # hidden layers see bf16 inputs; the per-actuator map reads the fp32 rows
    Yr, cache = net_ref.forward(p, net_ref.bf16_round(X), X)
    T = (u_t / ws.U_SCALE).transpose(0, 2, 1).reshape(-1, 40)
    gr = net_ref.backward(p, cache, Yr, T)
    assert np.linalg.norm(Y - Yr) <= 2e-2 * np.linalg.norm(Yr)
    assert abs(loss - net_ref.mse(Yr, T)) <= 2e-2 * net_ref.mse(Yr, T)
    # the bf16 copies of activations and gradients (2^-9 relative each) and the
    # ReLU masks they flip near zero leave a few percent norm-wise two layers
    # down; each layer alone is held to the fp32 accumulation bound element by
    # element in test_network_layers_elementwise
    rel = {k: np.linalg.norm(net.grad(k).astype(np.float64) - v) / (np.linalg.norm(v) + 1e-30)
           for k, v in gr.items()}
    print({k: f"{r:.1e}" for k, r in rel.items()})
    assert all(r <= 1e-1 for r in rel.values()), rel
    assert all(rel[k] <= 2e-2 for k in ("W4", "b4", "Ws")), rel
    # the fp32 map alone (hidden path switched off): about fp32 accuracy
    p0 = dict(p); p0["W4"] = np.zeros_like(p["W4"]); p0["b4"] = np.zeros_like(p["b4"])
    net.set_param("W4", np.zeros(net.shape("W4"), np.float32))
    net.set_param("b4", np.zeros(net.shape("b4"), np.float32))
    u0 = net.predict(dx0, dxr).cpu().numpy()
    Yr0, _ = net_ref.forward(p0, net_ref.bf16_round(X), X)
    want = ws.U_SCALE * Yr0.reshape(3, 16, 40).transpose(0, 2, 1)
    assert np.abs(u0 - want).max() <= 1e-5 * np.abs(want).max()


U24 = 2.0 ** -24      # unit roundoff of fp32


def _dot_bound(A, W, K, extra=0.0):
    """Elementwise bound of an fp32-accumulated product A W (+ a term of size
    extra): any summation order of K products, each exact (bf16 operands) or
    rounded once (fp32 operands), stays within (K + 2) u sum_k |a_k| |w_k|."""
    return (K + 2) * U24 * (np.abs(A) @ np.abs(W) + np.abs(extra)) + 1e-30


@pytest.mark.parametrize("ns,L,win,planes,count,N", [
    (64, 4, 32, 5, 3, 40),     # the committed network's shape, a partial instance tile
    (64, 4, 32, 5, 70, 40),    # two instance tiles
    (48, 4, 24, 2, 5, 17),     # window of 576 pixels: a partial last chunk
    (32, 2, 20, 5, 2, 48),     # 48 output columns, the kernel's limit
    (16, 8, 6, 5, 1, 3),       # 8 x 8 lattice, windows past the grid edge
])
def test_map_forward_elementwise(ws, ns, L, win, planes, count, N):
    """The forward pass of a network without hidden path is the per-actuator
    map with its features gathered inside the product (no feature rows in
    HBM): every output against the fp64 product of the fp32 feature rows of
    the definition (rounded once from fp64) with Ws, within the fp32
    accumulation bound of K0 + 8 terms (the split-K parts and the one-hot
    row); the returned inputs are 4 Y, transposed to [count][N][L^2]."""
    import torch
    rng = np.random.default_rng(ns + L + win + count)
    cls = type("Net", (ws.PatchNet,), {"PLANES": planes})   # the object takes 2 or 5 planes
    net = cls(N=N, ns=ns, lattice=L, win=win, hidden=0, max_count=count)
    Ws = rng.normal(size=net.shape("Ws")).astype(np.float32) * 0.05
    net.set_param("Ws", Ws)
    x0 = 0.1 + 0.05 * rng.standard_normal((count, ns * ns))
    xr = 0.3 * rng.random((count, ns * ns))
    dx0, dxr = torch.tensor(x0, device="cuda"), torch.tensor(xr, device="cuda")
    u = net.predict(dx0, dxr).cpu().numpy()
    rows, m = count * L * L, L * L
    Y = net.get("Y", rows=rows).astype(np.float64)
    X32 = net_ref.features(x0, xr, ns, L, win, planes, net.K0p).astype(np.float32).astype(np.float64)
    want = net_ref.skip(Ws.astype(np.float64), X32)
    bound = (net.K0p + 8) * U24 * net_ref.skip(np.abs(Ws).astype(np.float64), np.abs(X32)) + 1e-30
    assert np.all(np.abs(Y - want) <= bound)
    np.testing.assert_array_equal(u, 4.0 * Y.astype(np.float32).astype(np.float64)
                                  .reshape(count, m, N).transpose(0, 2, 1))


def test_network_layers_elementwise(ws):
    """Each layer of the GPU pass against its own definition evaluated in
    float64 on the GPU's inputs to that layer: every element within the fp32
    accumulation bound, the bf16 copies equal to the nearest-even rounding of
    the fp32 values, the elementwise steps (dY, the ReLU mask, the bias sums
    in their fixed order) bit-exact."""
    net, x0, xr, u_t, (dx0, dxr, du) = _net_case(ws)
    loss = net.backward(dx0, dxr, du)
    rows, m, N, H, K0 = 3 * 16, 16, 40, 64, net.K0p
    f = lambda name: net.get(name, rows=rows).astype(np.float64)
    Xf, X = f("Xf"), f("X")
    # features: fp32 rounding of the fp64 values, bf16 copy of that
    want = net_ref.features(x0, xr, 64, 4, 32, 5, K0)
    np.testing.assert_allclose(Xf, want.astype(np.float32).astype(np.float64), rtol=2**-23, atol=0)
    np.testing.assert_array_equal(X, net_ref.bf16_round(Xf))
    W = {k: net.get(k).astype(np.float64) for k in ws.PARAMS}
    Wb = {}
    for l in (1, 2, 3, 4):
        Wb[l] = net.get(f"Wb{l}").astype(np.float64)
        np.testing.assert_array_equal(Wb[l], net_ref.bf16_round(W[f"W{l}"]))
    # hidden layers: H_l = relu(A_l Wb_l + b_l), A_1 = X, A_l = bf16 copy of H_{l-1}
    A = X
    Hs, Ab = [], [X]
    for l in (1, 2, 3):
        Z = A @ Wb[l] + W[f"b{l}"]
        Hl, Hlb = f(f"H{l}"), f(f"H{l}b")
        kin = K0 if l == 1 else H
        assert np.all(np.abs(Hl - np.maximum(Z, 0)) <= _dot_bound(A, Wb[l], kin, W[f"b{l}"])), l
        np.testing.assert_array_equal(Hlb, net_ref.bf16_round(Hl))
        Hs.append(Hl)
        A = Hlb
        Ab.append(Hlb)
    # output: Y = H3b Wb4 + b4 + Xf Ws[p]
    Y = f("Y")
    Yw = A @ Wb[4] + W["b4"] + net_ref.skip(W["Ws"], Xf)
    # two accumulations (the bf16 layer, then the map added onto it)
    bound = (H + K0 + 4) * U24 * (np.abs(A) @ np.abs(Wb[4]) + np.abs(W["b4"]) +
                                  net_ref.skip(np.abs(W["Ws"]), np.abs(Xf)))
    assert np.all(np.abs(Y - Yw) <= bound)
    # targets, the error gradient and the loss
    T = f("T")
    np.testing.assert_array_equal(T, (u_t * 0.25).astype(np.float32).transpose(0, 2, 1)
                                  .reshape(rows, N).astype(np.float64))
    scale = np.float32(2.0) / (np.float32(rows) * np.float32(N))
    dY32 = scale * (net.get("Y", rows=rows) - net.get("T", rows=rows))
    dY = f("dY")
    np.testing.assert_array_equal(dY, dY32.astype(np.float64))
    dYb = f("dYb")
    np.testing.assert_array_equal(dYb, net_ref.bf16_round(dY))
    assert abs(loss - np.mean((Y - T) ** 2)) <= 1e-5 * np.mean((Y - T) ** 2)
    # gradients of the output layer and of the map
    colsum = lambda D: np.cumsum(D.astype(np.float32), axis=0, dtype=np.float32)[-1].astype(np.float64)
    g = {k: net.grad(k).astype(np.float64) for k in ws.PARAMS}
    assert np.all(np.abs(g["W4"] - A.T @ dYb) <= _dot_bound(A.T, dYb, rows))
    np.testing.assert_array_equal(g["b4"], colsum(dY))
    for p in range(m):
        gw = Xf[p::m].T @ dY[p::m]
        assert np.all(np.abs(g["Ws"][p] - gw) <= _dot_bound(Xf[p::m].T, dY[p::m], 3)), p
    # back through the hidden layers: dH_l = (dH_{l+1}b Wb_{l+1}^T) masked by H_l > 0
    up, upb = dY, dYb
    for l in (3, 2, 1):
        pre = upb @ Wb[l + 1].T
        mask = Hs[l - 1] > 0
        dH, dHb = f(f"dH{l}"), f(f"dH{l}b")
        kin = N if l == 3 else H
        assert np.all(np.abs(dH - pre * mask) <= _dot_bound(upb, np.abs(Wb[l + 1].T), kin) * mask), l
        assert np.all(dH[~mask] == 0.0), l
        np.testing.assert_array_equal(dHb, net_ref.bf16_round(dH))
        assert np.all(np.abs(g[f"W{l}"] - Ab[l - 1].T @ dHb) <= _dot_bound(Ab[l - 1].T, dHb, rows)), l
        np.testing.assert_array_equal(g[f"b{l}"], colsum(dH))
        up, upb = dH, dHb


def test_adam_step_elementwise(ws):
    """The first Adam step from zero moments moves each unfrozen weight by
    lr g / (|g| + eps) (bias-corrected moments) after the decoupled decay;
    frozen parameters keep every bit."""
    net, x0, xr, u_t, (dx0, dxr, du) = _net_case(ws, hidden=32)
    net.backward(dx0, dxr, du)
    before = net.state()
    g = {k: net.grad(k).astype(np.float64) for k in ws.PARAMS}
    lr, wd = 1e-3, 1e-2
    rc = ws._net_lib().nmpc_net_adam_step(net.hd, lr, 0.9, 0.999, 1e-8, wd,
                                          1 << ws.PARAMS.index("W2"), ws._stream())
    assert rc == 0
    after = net.state()
    np.testing.assert_array_equal(after["W2"], before["W2"])
    for k in ws.PARAMS:
        if k == "W2" or not before[k].size:
            continue
        w0 = before[k].astype(np.float64)
        decay = wd if k.startswith("W") and k != "Ws" else 0.0
        want = w0 * (1 - lr * decay) - lr * g[k] / (np.abs(g[k]) + 1e-8)
        # fp32 evaluation of the same few operations
        tol = 16 * 2.0 ** -24 * (np.abs(w0) + lr) + lr * (np.abs(g[k]) < 1e-12)
        assert np.all(np.abs(after[k] - want) <= tol), k
    # the bf16 copies follow the updated weights
    np.testing.assert_array_equal(net.get("Wb1").astype(np.float64),
                                  net_ref.bf16_round(after["W1"].astype(np.float64)))


def test_weight_file_round_trip(ws, tmp_path):
    """nmpc_net_save / nmpc_net_load: a network of another seed takes every bit
    of the parameters and predicts the same inputs; a file of another
    configuration is refused."""
    net, x0, xr, u_t, (dx0, dxr, du) = _net_case(ws, hidden=32)
    path = str(tmp_path / "w.bin")
    net.save_bin(path)
    other = ws.PatchNet(hidden=32, seed=11, max_count=8)
    assert not np.array_equal(other.get("W1"), net.get("W1"))
    other.load_bin(path)
    for k in ws.PARAMS:
        np.testing.assert_array_equal(other.get(k), net.get(k))
    np.testing.assert_array_equal(other.predict(dx0, dxr).cpu().numpy(),
                                  net.predict(dx0, dxr).cpu().numpy())
    wrong = ws.PatchNet(hidden=16, seed=0, max_count=8)
    with pytest.raises(RuntimeError):
        wrong.load_bin(path)
    # the npz checkpoint holds the same values
    net.save(str(tmp_path / "w.npz"))
    back = ws.PatchNet.load(str(tmp_path / "w.npz"), max_count=8)
    for k in ws.PARAMS:
        np.testing.assert_array_equal(back.get(k), net.get(k))


def test_training_steps_reduce_the_loss(ws):
    import torch
    P = make_problem("c1")
    x0, xr = make_batch(P, range(8))
    rng = np.random.default_rng(1)
    u_t = torch.tensor(rng.normal(size=(8, 40, 16)) * 2.0, device="cuda")
    net = ws.PatchNet(hidden=64, seed=0, max_count=8)
    dx0, dxr = torch.tensor(x0, device="cuda"), torch.tensor(xr, device="cuda")
    first = net.backward(dx0, dxr, u_t)
    for _ in range(60):
        loss = net.train_step(dx0, dxr, u_t, lr=2e-3)
    assert loss < 0.2 * first


def test_trained_network_cuts_iterations_without_moving_the_solution(ws):
    """The committed network on unseen instances: the learned start needs far
    fewer upper iterations than the cold start, is never replaced by the
    fallback, and the converged inputs agree with the cold-start solution and
    with the oracle's exact solution."""
    import os
    import torch
    import paper_2004_02484_amd as nm
    import oracle
    path = os.path.join(os.path.dirname(ws.__file__), "weights", "c1_patchnet.npz")
    net = ws.PatchNet.load(path)
    P = make_problem("c1")
    seeds = list(range(2_000_000, 2_000_016))          # disjoint from the training seeds
    x0, xr = make_batch(P, seeds)
    dx0, dxr = torch.tensor(x0, device="cuda"), torch.tensor(xr, device="cuda")
    s = nm.Solver(P, max_batch=len(seeds), precision=nm.NMPC_FP32_SWEEP, fallback=1)
    rc_c, Xc, Uc, Lc, ic = s.solve_batch(dx0, dxr)
    up = net.predict(dx0, dxr)
    rc_l, Xl, Ul, Ll, il = s.solve_batch(dx0, dxr, warm=(None, up, None))
    assert rc_c == nm.NMPC_OK and rc_l == nm.NMPC_OK
    itc = np.array([i["iters"] for i in ic]); itl = np.array([i["iters"] for i in il])
    pred = ((up - Uc).abs().amax(dim=(1, 2)) / Uc.abs().amax(dim=(1, 2))).cpu().numpy()
    print(f"cold iterations {itc.mean():.1f}, learned {itl.mean():.1f} "
          f"(min {itl.min()}, max {itl.max()}); prediction error median {np.median(pred):.2e}")
    assert all(i["start_used"] == 2 for i in il)
    assert np.median(pred) <= 1e-3
    assert itl.mean() <= 0.25 * itc.mean()
    du = ((Ul - Uc).abs().amax(dim=(1, 2)) / Uc.abs().amax(dim=(1, 2))).max().item()
    assert du <= 1e-4
    ex = oracle.solve(P, x0[0], xr[0], tol=1e-11, max_iter=20000)
    assert ex["status"] == "converged"
    err = np.abs(Ul[0].cpu().numpy() - ex["U"]).max() / np.abs(ex["U"]).max()
    assert err <= 1e-4


def test_map_only_network_is_the_full_network_without_its_hidden_output(ws):
    """PatchNet.load(mlp=False) builds the committed network with hidden = 0:
    its prediction is the per-actuator map alone, bit for bit the full
    network's prediction once the hidden path's output layer (W4, b4) is
    zero; the committed hidden path moves the prediction by far less than the
    map's own error."""
    import os
    import torch
    path = os.path.join(os.path.dirname(ws.__file__), "weights", "c1_patchnet.npz")
    full = ws.PatchNet.load(path, max_count=8)
    lin = ws.PatchNet.load(path, max_count=8, mlp=False)
    assert lin.H == 0 and full.H > 0
    P = make_problem("c1")
    x0, xr = make_batch(P, list(range(2_100_000, 2_100_008)))
    dx0, dxr = torch.tensor(x0, device="cuda"), torch.tensor(xr, device="cuda")
    u_full = full.predict(dx0, dxr).clone()
    u_lin = lin.predict(dx0, dxr).clone()
    full.set_param("W4", np.zeros(full.shape("W4"), np.float32))
    full.set_param("b4", np.zeros(full.shape("b4"), np.float32))
    u_zero = full.predict(dx0, dxr)
    assert torch.equal(u_lin, u_zero)
    rel = ((u_full - u_lin).abs().amax(dim=(1, 2)) / u_lin.abs().amax(dim=(1, 2))).max().item()
    print(f"hidden path's share of the prediction: {rel:.2e} (relative, max over instances)")
    assert 0.0 < rel <= 1e-4


def test_full_batch_in_the_benchmark_configuration(ws):
    """The benchmark's launch configuration at its full size: 256 unseen
    64 x 64, N = 40 instances, learned start (the committed network's
    per-actuator map, as the benchmark runs it) with the fallback check, 10
    state and 14 costate rollout sweeps, FP32 sweeps with the final FP64
    correction, tol 1e-6.
    Every instance reports convergence; on sampled instances the oracle's
    residual of the returned trajectory meets the tolerance and the inputs
    meet the FP32-sweep bar against the oracle's exact solution."""
    import os
    import torch
    import paper_2004_02484_amd as nm
    import oracle
    path = os.path.join(os.path.dirname(ws.__file__), "weights", "c1_patchnet.npz")
    net = ws.PatchNet.load(path, mlp=False)
    P = make_problem("c1")
    B = 256
    x0, xr = make_batch(P, list(range(3_000_000, 3_000_000 + B)))
    dx0, dxr = torch.tensor(x0, device="cuda"), torch.tensor(xr, device="cuda")
    s = nm.Solver(P, max_batch=B, precision=nm.NMPC_FP32_SWEEP, tol=1e-6, max_iter=5000,
                  check_every=16, fallback=1, warm_sweeps=10, warm_sweeps_lambda=14)
    up = net.predict(dx0, dxr)
    rc, X, U, L, infos = s.solve_batch(dx0, dxr, warm=(None, up, None))
    assert rc == nm.NMPC_OK
    assert all(i["status"] == nm.NMPC_OK and i["r_scaled"] <= 1e-6 for i in infos)
    its = np.array([i["iters"] for i in infos])
    for b in (0, 97, 255):
        Xb, Ub, Lb = X[b].cpu().numpy(), U[b].cpu().numpy(), L[b].cpu().numpy()
        rs, _ = oracle.residual(P, x0[b], xr[b], Xb, Ub, Lb)
        ex = oracle.solve(P, x0[b], xr[b], tol=1e-11, max_iter=20000)
        err = np.abs(Ub - ex["U"]).max() / np.abs(ex["U"]).max()
        print(f"instance {b}: {its[b]} iterations, oracle residual {rs:.2e}, "
              f"control rel. error vs exact {err:.2e}")
        # the two residuals differ by the rounding of differently ordered sums
        assert rs <= 1e-6 and abs(rs - infos[b]["r_scaled"]) <= 1e-12
        assert err <= 1e-4
    print(f"iterations mean {its.mean():.1f}, max {its.max()}")
