"""Train the warm-start network on solutions computed by the solver itself.

    python -m paper_2004_02484_amd.train_warmstart --samples 81920 --epochs 40 \
        --out paper_2004_02484_amd/weights/c1_patchnet.npz

Data: instances of the 64x64, N=40 workload (seeds 0..samples-1) solved on the
GPU to r_scaled <= 1e-9; the last `--val` instances are held out. Training, all
compute in the library's kernels: first the per-actuator linear map, the
exact minimizer of the squared error of the scaled input trajectories (normal
equations with fp64 sums and a relative ridge, solved by Newton-Schulz
iteration on the matrix cores); then Adam on the hidden layers for what the
linear map leaves, the map held fixed; the state with the smallest held-out
error is kept.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np


def generate(P, seeds, batch=256, tol=1e-9):
    import torch
    import paper_2004_02484_amd as nm
    from nmpc_inputs import make_batch
    s = nm.Solver(P, max_batch=batch, tol=tol, max_iter=5000, precision=nm.NMPC_FP32_SWEEP)
    X0, XR, U = [], [], []
    for k in range(0, len(seeds), batch):
        sd = seeds[k:k + batch]
        x0, xr = make_batch(P, sd)
        dx0 = torch.tensor(x0, device="cuda"); dxr = torch.tensor(xr, device="cuda")
        rc, X, Uo, L, inf = s.solve_batch(dx0, dxr)
        if rc != nm.NMPC_OK:
            raise RuntimeError(f"label solve failed: {nm.nmpc_strerror(rc)}")
        X0.append(dx0); XR.append(dxr); U.append(Uo.clone())
    s.close()
    return torch.cat(X0), torch.cat(XR), torch.cat(U)


def rel_errors(net, x0, xr, u, batch=256):
    import torch
    errs = []
    for k in range(0, x0.shape[0], batch):
        up = net.predict(x0[k:k + batch], xr[k:k + batch])
        ut = u[k:k + batch]
        e = (up - ut).abs().amax(dim=(1, 2)) / ut.abs().amax(dim=(1, 2))
        errs.append(e.cpu().numpy())
    return np.concatenate(errs)


def train(samples=81920, val=1024, epochs=40, batch=256, lr=3e-4, wd=1e-5, hidden=128, seed=0,
          ridge=1e-6, log=print):
    import torch
    from nmpc_inputs import make_problem
    from .warmstart import PatchNet
    P = make_problem("c1")
    t0 = time.time()
    x0, xr, u = generate(P, list(range(samples)))
    log(f"labels: {samples} solves in {time.time() - t0:.1f} s")
    ntr = samples - val
    net = PatchNet(N=P.N, ns=P.nsx, lattice=P.lx, hidden=hidden, seed=seed)
    net.set_param("W4", np.zeros(net.shape("W4"), np.float32))
    net.set_param("b4", np.zeros(net.shape("b4"), np.float32))
    # 1. the per-actuator linear map: exact minimizer of the squared error
    t1 = time.time()
    res = net.fit_linear(x0[:ntr], xr[:ntr], u[:ntr], batch=batch, ridge_rel=ridge)
    e = rel_errors(net, x0[ntr:], xr[ntr:], u[ntr:])
    lin = (float(np.median(e)), float(np.percentile(e, 90)))
    log(f"linear map: |I - G X| max {max(res):.1e}, held-out input error median {lin[0]:.2e} "
        f"p90 {lin[1]:.2e} ({time.time() - t1:.1f} s)")
    # 2. the hidden layers on what the linear map leaves, the map held fixed
    g = torch.Generator(device="cpu").manual_seed(seed)
    steps_per_epoch = ntr // batch
    total = epochs * steps_per_epoch
    best, best_state = lin[0], net.state()
    t2 = time.time()
    for ep in range(epochs):
        perm = torch.randperm(ntr, generator=g).to("cuda")
        xs, rs, us = x0[perm], xr[perm], u[perm]
        run = 0.0
        for k in range(steps_per_epoch):
            step = ep * steps_per_epoch + k
            lr_t = lr * 0.5 * (1.0 + np.cos(np.pi * step / total)) + 1e-7
            sl = slice(k * batch, (k + 1) * batch)
            run += net.train_step(xs[sl], rs[sl], us[sl], lr=lr_t, wd=wd, frozen=("Ws",))
        if ep % 5 == 4 or ep == epochs - 1:
            e = rel_errors(net, x0[ntr:], xr[ntr:], u[ntr:])
            med = float(np.median(e))
            log(f"epoch {ep + 1}: train mse {run / steps_per_epoch:.3e}, held-out input error "
                f"median {med:.2e} p90 {np.percentile(e, 90):.2e} ({time.time() - t2:.1f} s)")
            if med < best:
                best, best_state = med, net.state()
    net.load_state(best_state)
    e = rel_errors(net, x0[ntr:], xr[ntr:], u[ntr:])
    meta = {"samples": samples, "val": val, "epochs": epochs, "batch": batch, "lr": lr, "wd": wd,
            "ridge_rel": ridge, "label_tol": 1e-9, "seeds": [0, samples - 1],
            "linear_val_rel_err_median": lin[0],
            "val_rel_err_median": float(np.median(e)), "val_rel_err_p90": float(np.percentile(e, 90)),
            "train_seconds": time.time() - t1}
    return net, meta


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--samples", type=int, default=81920)
    ap.add_argument("--val", type=int, default=1024)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--hidden", type=int, default=128)
    ap.add_argument("--lr", type=float, default=3e-4)
    ap.add_argument("--ridge", type=float, default=1e-6)
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    net, meta = train(samples=args.samples, val=args.val, epochs=args.epochs, hidden=args.hidden,
                      lr=args.lr, ridge=args.ridge, log=lambda s: print(s, flush=True))
    net.save(args.out, meta)
    print(json.dumps(meta), flush=True)


if __name__ == "__main__":
    main()
