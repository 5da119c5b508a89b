"""The allocation-free split-K fp32 GEMM (static device scratch) against the
entry point that takes a caller workspace, through the C ABI: equal results
bit for bit on two calls in a row, the second one smaller (the scratch keeps
the first call's partials, which must not leak into the second), and a clear
error beyond the scratch's size."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2004_02484_amd import _binding as B
    L = B._load()
    vp, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    L.nmpc_gemm_f32.argtypes = [i32, i32, i32, i32, vp, i32, i64, vp, i32, i64, f32, vp, i32,
                                i64, i32, i32, vp, vp]
    L.nmpc_gemm_f32.restype = ctypes.c_int
    L.nmpc_gemm_f32_noalloc.argtypes = [i32, i32, i32, i32, vp, i32, i64, vp, i32, i64, f32, vp,
                                        i32, i64, i32, i32, vp]
    L.nmpc_gemm_f32_noalloc.restype = ctypes.c_int
    return L


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _grouped(lib, rng, M, N, K, groups, ksplit, beta):
    """Both entry points on the same grouped operands (rows of a group
    interleaved like the network's per-actuator map); returns both results."""
    import torch
    dev = "cuda"
    A = torch.tensor(rng.normal(size=(M * groups, K)).astype(np.float32), device=dev)
    Bm = torch.tensor(rng.normal(size=(groups, K, N)).astype(np.float32), device=dev)
    C0 = torch.tensor(rng.normal(size=(M * groups, N)).astype(np.float32), device=dev)
    Cw, Cs = C0.clone(), C0.clone()
    work = torch.empty(groups * ksplit * M * N, dtype=torch.float32, device=dev)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    args = (0, M, N, K, _p(A), groups * K, K, _p(Bm), N, K * N, beta)
    rc = lib.nmpc_gemm_f32(*args, _p(Cw), groups * N, N, groups, ksplit, _p(work), s)
    assert rc == 0
    rc = lib.nmpc_gemm_f32_noalloc(*args, _p(Cs), groups * N, N, groups, ksplit, s)
    assert rc == 0
    torch.cuda.synchronize()
    ref = np.einsum("mgk,gkn->mgn", A.cpu().numpy().astype(np.float64).reshape(M, groups, K),
                    Bm.cpu().numpy().astype(np.float64)).reshape(M * groups, N)
    ref = ref + beta * C0.cpu().numpy().astype(np.float64)
    return Cw, Cs, ref


def test_noalloc_gemm_equals_workspace_gemm_twice(lib):
    import torch
    rng = np.random.default_rng(0)
    # the benchmark's per-actuator map at batch 256 (16 groups, K = 5152, 8 parts)
    Cw, Cs, ref = _grouped(lib, rng, 256, 40, 5152, 16, 8, 1.0)
    assert torch.equal(Cw, Cs)
    err = np.abs(Cs.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err <= 1e-5, err
    # a smaller second call: fewer parts and rows, ragged tiles
    Cw, Cs, ref = _grouped(lib, rng, 37, 19, 301, 3, 5, 0.0)
    assert torch.equal(Cw, Cs)
    err = np.abs(Cs.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err <= 1e-5, err
    # no split: no scratch used
    Cw, Cs, ref = _grouped(lib, rng, 20, 8, 64, 2, 1, 0.5)
    assert torch.equal(Cw, Cs)


def test_noalloc_gemm_rejects_sizes_beyond_the_scratch(lib):
    import torch
    A = torch.zeros((4, 4), dtype=torch.float32, device="cuda")
    C = torch.zeros((4, 4), dtype=torch.float32, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    # groups * ksplit * M * N = 16 * 8 * 4096 * 40 > 2^21: refused before any launch
    rc = lib.nmpc_gemm_f32_noalloc(0, 4096, 40, 5152, _p(A), 5152, 0, _p(A), 40, 0, 0.0, _p(C),
                                   40, 0, 16, 8, s)
    assert rc == 1   # NMPC_E_ARG
    msg = lib.nmpc_last_error().decode()
    assert "static scratch" in msg
