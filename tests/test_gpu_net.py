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
    Ws = net.params["Ws"].cpu().numpy().astype(np.float64)
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


def test_forward_and_gradients_match_reference(ws):
    import torch
    P = make_problem("c1")
    x0, xr = make_batch(P, [7, 8, 9])
    net = ws.PatchNet(hidden=64, seed=3)
    rng = np.random.default_rng(5)
    net.params["Ws"] = torch.tensor(rng.normal(size=(16, net.K0p, 40)).astype(np.float32) * 0.02,
                                    device="cuda")
    net.load_state(net.state())
    u_t = rng.normal(size=(3, 40, 16))
    dx0, dxr = torch.tensor(x0, device="cuda"), torch.tensor(xr, device="cuda")
    loss, g = net.loss_and_grads(dx0, dxr, torch.tensor(u_t, device="cuda"))
    Y = net._buf["Y"].cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    p = {k: v.astype(np.float64) for k, v in net.state().items()}
    for k in list(p):
        if k.startswith("W") and k != "Ws":
            p[k] = net_ref.bf16_round(p[k])
    X = net_ref.features(x0, xr, 64, 4, 32, 5, net.K0p).astype(np.float32).astype(np.float64)
    # hidden layers see bf16 inputs; the per-actuator map reads the fp32 rows
    Yr, cache = net_ref.forward(p, net_ref.bf16_round(X), X)
    T = (u_t / ws.U_SCALE).transpose(0, 2, 1).reshape(-1, 40)
    gr = net_ref.backward(p, cache, Yr, T)
    # bf16 activations between layers: a few 1e-3 relative
    assert np.linalg.norm(Y - Yr) <= 2e-2 * np.linalg.norm(Yr)
    assert abs(loss - net_ref.mse(Yr, T)) <= 2e-2 * net_ref.mse(Yr, T)
    for k, v in gr.items():
        got = g[k].cpu().numpy().astype(np.float64)
        assert np.linalg.norm(got - v) <= 5e-2 * np.linalg.norm(v) + 1e-12, k
    # the fp32 map alone (hidden path switched off): about fp32 accuracy
    p0 = dict(p); p0["W4"] = np.zeros_like(p["W4"]); p0["b4"] = np.zeros_like(p["b4"])
    net.params["W4"].zero_(); net.params["b4"].zero_(); net.load_state(net.state())
    Y0 = net.forward_rows(dx0, dxr).cpu().numpy().astype(np.float64)
    Yr0, _ = net_ref.forward(p0, net_ref.bf16_round(X), X)
    assert np.abs(Y0 - Yr0).max() <= 1e-5 * np.abs(Yr0).max()


def test_training_steps_reduce_the_loss(ws):
    import torch
    P = make_problem("c1")
    x0, xr = make_batch(P, range(8))
    rng = np.random.default_rng(1)
    u_t = torch.tensor(rng.normal(size=(8, 40, 16)) * 2.0, device="cuda")
    net = ws.PatchNet(hidden=64, seed=0)
    dx0, dxr = torch.tensor(x0, device="cuda"), torch.tensor(xr, device="cuda")
    first, _ = net.loss_and_grads(dx0, dxr, u_t)
    for _ in range(60):
        loss, g = net.loss_and_grads(dx0, dxr, u_t)
        net.adam_step(g, lr=2e-3)
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


def test_full_batch_in_the_benchmark_configuration(ws):
    """The benchmark's launch configuration at its full size: 256 unseen
    64 x 64, N = 40 instances, learned start with the fallback check, 14
    rollout sweeps, FP32 sweeps with the final FP64 correction, tol 1e-6.
    Every instance reports convergence; on sampled instances the oracle's
    residual of the returned trajectory meets the tolerance and the inputs
    meet the FP32-sweep bar against the oracle's exact solution."""
    import os
    import torch
    import paper_2004_02484_amd as nm
    import oracle
    path = os.path.join(os.path.dirname(ws.__file__), "weights", "c1_patchnet.npz")
    net = ws.PatchNet.load(path)
    P = make_problem("c1")
    B = 256
    x0, xr = make_batch(P, list(range(3_000_000, 3_000_000 + B)))
    dx0, dxr = torch.tensor(x0, device="cuda"), torch.tensor(xr, device="cuda")
    s = nm.Solver(P, max_batch=B, precision=nm.NMPC_FP32_SWEEP, tol=1e-6, max_iter=5000,
                  check_every=16, fallback=1, warm_sweeps=14)
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
