"""C-ABI library checks that need no GPU: exported symbols and argument
validation (both happen before any device call)."""
import ctypes
import re

import numpy as np
import pytest

from nmpc_inputs import make_problem

import paper_2004_02484_amd as nm
from paper_2004_02484_amd import _binding


def declared_functions():
    src = open(_binding.library_path().replace("paper_2004_02484_amd/libnmpc.so",
                                               "include/nmpc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nmpc_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_binding.library_path())
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name


def test_default_options_are_the_papers_lower_layer():
    o = nm.nmpc_default_options()
    assert (o.n_sweep, o.n_schur, o.precision) == (2, 2, nm.NMPC_FP64)
    assert o.upper == nm.NMPC_UPPER_JACOBI
    assert o.tol == 1e-6 and o.check_every >= 1


@pytest.mark.parametrize("field,value", [("dim", 3), ("nsx", 0), ("N", 0), ("h", 0.0),
                                         ("r", 0.0), ("gamma", -1.0), ("q", -1.0),
                                         ("h", float("nan"))])
def test_invalid_problem_rejected(field, value):
    p = make_problem("c0")
    setattr(p, field, value)
    with pytest.raises(nm.NmpcError) as e:
        nm.nmpc_create(p, nm.nmpc_default_options(), 1)
    assert e.value.code == nm.NMPC_E_ARG


def test_1d_needs_single_row():
    p = make_problem("c0").with_(nsy=2, gy=np.ones((1, 2)))
    with pytest.raises(nm.NmpcError) as e:
        nm.nmpc_create(p, nm.nmpc_default_options(), 1)
    assert e.value.code == nm.NMPC_E_ARG


def test_unsupported_shapes_reported():
    fused = nm.nmpc_default_options(path=nm.NMPC_PATH_FUSED)
    p = make_problem("grid", ns=100, N=4)   # wider than 16 lanes x 6 columns
    with pytest.raises(nm.NmpcError) as e:
        nm.nmpc_create(p, fused, 1)
    assert e.value.code == nm.NMPC_E_UNSUPPORTED
    p = make_problem("grid", ns=16, N=4, lattice=3)   # no fused kernel for a 3x3 lattice
    with pytest.raises(nm.NmpcError) as e:
        nm.nmpc_create(p, fused, 1)
    assert e.value.code == nm.NMPC_E_UNSUPPORTED
    p = make_problem("grid", ns=16, N=4, lattice=9)   # more than 64 inputs: no path
    with pytest.raises(nm.NmpcError) as e:
        nm.nmpc_create(p, nm.nmpc_default_options(), 1)
    assert e.value.code == nm.NMPC_E_UNSUPPORTED
    # the streaming path (any width) runs the Jacobi upper layer only
    o = nm.nmpc_default_options(path=nm.NMPC_PATH_STREAM, upper=nm.NMPC_UPPER_SGS)
    with pytest.raises(nm.NmpcError) as e:
        nm.nmpc_create(make_problem("grid", ns=100, N=4), o, 1)
    assert e.value.code == nm.NMPC_E_UNSUPPORTED


@pytest.mark.parametrize("field,value", [("n_sweep", 0), ("n_sweep", 17), ("n_schur", -1),
                                         ("precision", 7), ("check_every", 0),
                                         ("max_iter", -1), ("tol", -1.0), ("tile_rows", -1),
                                         ("tile_rows", 17), ("upper", 4), ("upper", -1),
                                         ("path", 3), ("omega", 0.0), ("omega", 2.0),
                                         ("omega", 1.2), ("fp32_finish", 2),
                                         ("warm_sweeps", -1), ("warm_sweeps", 1001),
                                         ("warm_sweeps_lambda", -1), ("warm_sweeps_lambda", 1001)])
def test_invalid_options_rejected(field, value):
    o = nm.nmpc_default_options(**{field: value})
    with pytest.raises(nm.NmpcError) as e:
        nm.nmpc_create(make_problem("c0"), o, 1)
    assert e.value.code == nm.NMPC_E_ARG


def test_null_handle_calls():
    lib = ctypes.CDLL(_binding.library_path())
    lib.nmpc_destroy(None)
    assert lib.nmpc_kernel_config(None, None, None, None) == nm.NMPC_E_ARG
    lib.nmpc_strerror.restype = ctypes.c_char_p
    assert b"argument" in lib.nmpc_strerror(1)


def test_fp32_finish_needs_the_fused_path():
    o = nm.nmpc_default_options(fp32_finish=1, path=nm.NMPC_PATH_STREAM)
    with pytest.raises(nm.NmpcError) as e:
        nm.nmpc_create(make_problem("c1"), o, 1)
    assert e.value.code == nm.NMPC_E_UNSUPPORTED


def test_unknown_tile_height_is_unsupported():
    o = nm.nmpc_default_options(tile_rows=3)
    with pytest.raises(nm.NmpcError) as e:
        nm.nmpc_create(make_problem("c1"), o, 1)
    assert e.value.code == nm.NMPC_E_UNSUPPORTED


def _grid(ns, N, lattice=4):
    return make_problem("grid", ns=ns, N=N, lattice=lattice)


@pytest.mark.parametrize("classes,opts,code", [
    ([], {}, nm.NMPC_E_ARG),                                             # no class
    ([("grid", 32, 4, 2)], {}, nm.NMPC_E_UNSUPPORTED),                   # 2x2 lattice
    ([("grid", 100, 4, 4)], {}, nm.NMPC_E_UNSUPPORTED),                  # wider than 96
    ([("c0",)], {}, nm.NMPC_E_UNSUPPORTED),                              # 1D class
    ([("grid", 32, 4, 4)], {"xref_per_stage": 1}, nm.NMPC_E_UNSUPPORTED),
    ([("grid", 32, 4, 4)], {"n_sweep": 0}, nm.NMPC_E_ARG),
    ([("grid", 32, 0, 4)], {}, nm.NMPC_E_ARG),                           # horizon 0
    ([("grid", 32, 4, 4)], {"upper": 3}, nm.NMPC_E_UNSUPPORTED),         # SGS not ragged
    ([("grid", 32, 4, 4)], {"fp32_finish": 1}, nm.NMPC_E_UNSUPPORTED),   # FP64 correction kept
])
def test_ragged_create_validates_before_any_device_call(classes, opts, code):
    cl = [make_problem("c0") if c[0] == "c0" else _grid(c[1], c[2], c[3]) for c in classes]
    if not cl:
        o = nm.nmpc_default_options()
        lib = _binding._load()
        hd = ctypes.c_void_p()
        assert lib.nmpc_ragged_create(None, 0, ctypes.byref(o), 4, ctypes.byref(hd)) == code
        return
    with pytest.raises(nm.NmpcError) as e:
        nm.nmpc_ragged_create(cl, nm.nmpc_default_options(**opts), 4)
    assert e.value.code == code


def test_ragged_null_handle_calls():
    lib = _binding._load()
    lib.nmpc_ragged_destroy(None)
    c = (ctypes.c_int32 * 1)(0)
    w = ctypes.c_int32()
    assert lib.nmpc_ragged_config(None, 1, c, ctypes.byref(w)) == nm.NMPC_E_ARG
    assert lib.nmpc_ragged_timing_enable(None, 1) == nm.NMPC_E_ARG
    ev = ctypes.c_int64()
    assert lib.nmpc_ragged_timing_read_eval(None, ctypes.byref(ev)) == nm.NMPC_E_ARG
    assert lib.nmpc_timing_read_eval(None, ctypes.byref(ev)) == nm.NMPC_E_ARG
    assert lib.nmpc_ragged_solve(None, 1, c, None, None, None, None, None, None, None, None,
                                 None, None) == nm.NMPC_E_ARG
    assert lib.nmpc_autotune(None, 1, None, None, 4, None, None) == nm.NMPC_E_ARG


def test_loop_helpers_reject_a_null_handle():
    lib = _binding._load()
    assert lib.nmpc_shift_batch(None, 1, None, None, None, None, None, None, None) == nm.NMPC_E_ARG
    assert lib.nmpc_plant_step_batch(None, 1, None, None, 1, 0.1, None, None) == nm.NMPC_E_ARG


def test_input_box_arguments_checked():
    """An input box needs finite u_lo < 0 < u_hi (the cold start inside) and tau >= 0;
    the checks run before any device work."""
    base = make_problem("c0")
    for bad in (base.with_(tau=0.1, u_lo=0.1, u_hi=1.0), base.with_(tau=0.1, u_lo=-1.0, u_hi=-0.1),
                base.with_(tau=-1.0)):
        with pytest.raises(nm.NmpcError) as e:
            nm.Solver(bad)
        assert e.value.code == nm.NMPC_E_ARG


def test_ragged_box_arguments_checked():
    """Ragged classes with an input box need u_lo < 0 < u_hi (the cold start
    inside); checked before any device work."""
    bad = _grid(32, 4, 4).with_(tau=0.1, u_lo=0.1, u_hi=1.0)
    with pytest.raises(nm.NmpcError) as e:
        nm.nmpc_ragged_create([bad], nm.nmpc_default_options(), 4)
    assert e.value.code == nm.NMPC_E_ARG


def test_network_object_arguments_checked():
    """nmpc_net_create rejects an inconsistent configuration (lattice not
    dividing the grid, a window narrower than an actuator cell or of the wrong
    parity, a feature plane count other than 2 or 5, a negative hidden width,
    no instances) before any device call, and leaves *out NULL; every other
    entry point rejects a NULL network."""
    from paper_2004_02484_amd import warmstart as ws
    lib = ws._net_lib()
    good = dict(N=40, ns=64, lattice=4, win=32, hidden=64, planes=5)
    bad = [dict(ns=63), dict(win=8), dict(win=31), dict(planes=3), dict(hidden=-1), dict(N=0),
           dict(lattice=0)]
    for b in bad:
        cfg = ws.nmpc_net_config(**{**good, **b})
        out = ctypes.c_void_p(1234)
        assert lib.nmpc_net_create(ctypes.byref(cfg), 0, 4, ctypes.byref(out)) == nm.NMPC_E_ARG, b
        assert out.value is None
    cfg = ws.nmpc_net_config(**good)
    out = ctypes.c_void_p()
    assert lib.nmpc_net_create(ctypes.byref(cfg), 0, 0, ctypes.byref(out)) == nm.NMPC_E_ARG
    assert lib.nmpc_net_create(None, 0, 4, ctypes.byref(out)) == nm.NMPC_E_ARG
    assert lib.nmpc_net_create(ctypes.byref(cfg), 0, 4, None) == nm.NMPC_E_ARG
    for b in (dict(N=49), dict(ns=72, lattice=9, win=8)):   # beyond the map kernel
        cfg = ws.nmpc_net_config(**{**good, **b})
        out = ctypes.c_void_p(1234)
        assert lib.nmpc_net_create(ctypes.byref(cfg), 0, 4, ctypes.byref(out)) == nm.NMPC_E_UNSUPPORTED, b
        assert out.value is None
    assert lib.nmpc_net_forward(None, 1, None, None, None, None) == nm.NMPC_E_ARG
    assert lib.nmpc_net_backward(None, 1, None, None, None, None, None) == nm.NMPC_E_ARG
    assert lib.nmpc_net_adam_step(None, 1e-3, 0.9, 0.999, 1e-8, 0.0, 0, None) == nm.NMPC_E_ARG
    assert lib.nmpc_net_get(None, b"W1", None, 0) == nm.NMPC_E_ARG
    assert lib.nmpc_net_set(None, b"W1", None, 0, 0, None) == nm.NMPC_E_ARG
    assert lib.nmpc_net_save(None, b"/nonexistent") == nm.NMPC_E_ARG
    assert lib.nmpc_net_load(None, b"/nonexistent") == nm.NMPC_E_ARG
    assert lib.nmpc_net_num_params(None) == 0
    lib.nmpc_net_destroy(None)
