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


def test_windows_match_reference(ws):
    import torch
    from paper_2004_02484_amd.warmstart import _lib, _p, _stream
    P = make_problem("c1")
    x0, xr = make_batch(P, [3, 4])
    net = ws.PatchNet(hidden=32)
    out = torch.empty((32, net.K0p), dtype=torch.int16, device="cuda")
    dx0, dxr = torch.tensor(x0, device="cuda"), torch.tensor(xr, device="cuda")   # keep alive
    lo = torch.empty_like(out)
    rc = _lib().nmpc_net_windows(_p(dx0), _p(dxr), 2, 64, 4, 24, _p(out), _p(lo), net.K0p, _stream())
    assert rc == 0
    torch.cuda.synchronize()
    full = net_ref.windows(x0, xr, 64, 4, 24, net.K0p).astype(np.float32).astype(np.float64)
    want = net_ref.bf16_round(full)
    np.testing.assert_array_equal(ws.bf16_to_float(out), want)
    np.testing.assert_array_equal(ws.bf16_to_float(lo), net_ref.bf16_round(full - want))


def test_forward_and_gradients_match_reference(ws):
    import torch
    P = make_problem("c1")
    x0, xr = make_batch(P, [7, 8, 9])
    net = ws.PatchNet(hidden=64, seed=3)
    rng = np.random.default_rng(5)
    net.params["Ws"] = torch.tensor(rng.normal(size=(net.K0p, 40)).astype(np.float32) * 0.02,
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
    X = net_ref.windows(x0, xr, 64, 4, 24, net.K0p)
    # layers see bf16 inputs; the skip path uses split operands (about fp32)
    Xb = net_ref.bf16_round(X)
    Yr, cache = net_ref.forward(p, Xb)
    Yr = Yr + (X - Xb) @ p["Ws"]
    T = (u_t / ws.U_SCALE).transpose(0, 2, 1).reshape(-1, 40)
    gr = net_ref.backward(p, cache, Yr, T)
    # bf16 activations between layers: a few 1e-3 relative
    assert np.linalg.norm(Y - Yr) <= 2e-2 * np.linalg.norm(Yr)
    assert abs(loss - net_ref.mse(Yr, T)) <= 2e-2 * net_ref.mse(Yr, T)
    for k, v in gr.items():
        got = g[k].cpu().numpy().astype(np.float64)
        assert np.linalg.norm(got - v) <= 5e-2 * np.linalg.norm(v) + 1e-12, k


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
    assert np.median(pred) <= 1e-2
    assert itl.mean() <= 0.6 * itc.mean()
    du = ((Ul - Uc).abs().amax(dim=(1, 2)) / Uc.abs().amax(dim=(1, 2))).max().item()
    assert du <= 1e-4
    ex = oracle.solve(P, x0[0], xr[0], tol=1e-11, max_iter=20000)
    assert ex["status"] == "converged"
    err = np.abs(Ul[0].cpu().numpy() - ex["U"]).max() / np.abs(ex["U"]).max()
    assert err <= 1e-4
