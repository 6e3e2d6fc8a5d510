"""C-ABI checks that need no GPU: the library loads, exports every symbol include/qs.h
declares, rejects invalid arguments on the host before touching the device, and evaluates
the same SplitMix64 stream as the oracle (two independent implementations)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2607_24234_amd import build, qs
    if not os.path.exists(qs.LIB_PATH):
        build.build()
    return qs, qs.lib()


def declared_functions():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(qs_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_every_declared_symbol_is_exported():
    qs, L = _lib()
    names = declared_functions()
    assert "qs_init" in names and "qs_step_tau" in names
    for n in names:
        assert hasattr(L, n), "libqs.so does not export " + n
    assert set(names) <= set(qs.EXPORTS)


def test_abi_version():
    qs, L = _lib()
    assert L.qs_abi_version() == 1


def _inst(**kw):
    from paper_2607_24234_amd import inputs
    d = inputs.slab(n_modes=4, n_xi=16, n_steps=1)
    d.update(kw)
    return d


@pytest.mark.parametrize("bad,needle", [
    (dict(gamma=0.5), "gamma_b"),
    (dict(length=-1.0), "length"),
    (dict(n_xi=0), "n_xi"),
    (dict(d_tau=0.0), "d_tau"),
    (dict(d_tau=float("nan")), "d_tau"),
    (dict(species=[(-1.0, 0.0, 0.01)]), "m > 0"),
    (dict(species=[(-1.0, 1.0, -0.01)]), "nb_over_np"),
    (dict(kx=np.array([0.1, float("inf")])), "wavenumber"),
    (dict(seed_kind=9), "seed_kind"),
    (dict(flags=64), "flag"),
    (dict(seed_kind=2, kx=np.array([0.0, 1.0])), "k != 0"),
])
def test_invalid_arguments_rejected_on_host(bad, needle):
    qs, L = _lib()
    insts = [qs._Instance(_inst(**bad), qs.QS_FP64)]
    arr = (qs.QSParams * 1)(*[x.p for x in insts])
    assert L.qs_workspace_size(arr, 1) == 0
    ctx = ctypes.c_void_p()
    st = L.qs_init(arr, 1, None, None, 0, ctypes.byref(ctx))
    assert st == qs.QS_ERR_ARG
    assert ctx.value is None
    assert needle in L.qs_last_error().decode()


def _grid_inst(**kw):
    from paper_2607_24234_amd import inputs
    d = inputs.finite_width(nx=16, ny=8, n_xi=32, n_steps=2)
    d.update(kw)
    return d


def test_transverse_grid_arguments():
    qs, L = _lib()
    ok = qs._Instance(_grid_inst(geometry=qs.GEOM_TRANSVERSE_GRID), qs.QS_FP32)
    arr = (qs.QSParams * 1)(ok.p)
    # state (4 x 3 FP32 fields) + fields scratch: at least 19 floats per point
    assert L.qs_workspace_size(arr, 1) >= 16 * 8 * 32 * 4 * 19
    cases = [(dict(nx=12), qs.QS_ERR_ARG, "powers of two"), (dict(lx=0.0), qs.QS_ERR_ARG, "lx"),
             (dict(sigma_r=-1.0), qs.QS_ERR_ARG, "sigma_r"), (dict(flags=4), qs.QS_ERR_UNSUPPORTED, "STEADY"),
             (dict(seed_kind=2), qs.QS_ERR_UNSUPPORTED, "spectral only")]
    for kw, status, needle in cases:
        inst = qs._Instance(_grid_inst(geometry=qs.GEOM_TRANSVERSE_GRID, **kw), qs.QS_FP32)
        arr = (qs.QSParams * 1)(inst.p)
        ctx = ctypes.c_void_p()
        assert L.qs_init(arr, 1, None, None, 0, ctypes.byref(ctx)) == status, kw
        assert needle in L.qs_last_error().decode(), kw
    # FP64 is not offered on the grid; a grid instance cannot share a context
    inst = qs._Instance(_grid_inst(geometry=qs.GEOM_TRANSVERSE_GRID), qs.QS_FP64)
    arr = (qs.QSParams * 1)(inst.p)
    assert L.qs_init(arr, 1, None, None, 0, ctypes.byref(ctypes.c_void_p())) == qs.QS_ERR_UNSUPPORTED
    two = (qs.QSParams * 2)(ok.p, ok.p)
    assert L.qs_init(two, 2, None, None, 0, ctypes.byref(ctypes.c_void_p())) == qs.QS_ERR_ARG
    spec = qs._Instance(_inst(), qs.QS_FP32)
    mixed = (qs.QSParams * 2)(spec.p, ok.p)
    assert L.qs_init(mixed, 2, None, None, 0, ctypes.byref(ctypes.c_void_p())) == qs.QS_ERR_ARG
    # the centroid seed needs the grid
    bad = qs._Instance(_inst(seed_kind=3), qs.QS_FP32)
    arr = (qs.QSParams * 1)(bad.p)
    assert L.qs_init(arr, 1, None, None, 0, ctypes.byref(ctypes.c_void_p())) == qs.QS_ERR_UNSUPPORTED


def test_mixed_precision_rejected():
    qs, L = _lib()
    a = qs._Instance(_inst(), qs.QS_FP64)
    b = qs._Instance(_inst(), qs.QS_FP32)
    arr = (qs.QSParams * 2)(a.p, b.p)
    ctx = ctypes.c_void_p()
    assert L.qs_init(arr, 2, None, None, 0, ctypes.byref(ctx)) == qs.QS_ERR_ARG


def test_workspace_size_scales_with_problem():
    qs, L = _lib()
    s1 = qs.workspace_size([_inst(n_xi=64)], qs.QS_FP32)
    s2 = qs.workspace_size([_inst(n_xi=128)], qs.QS_FP32)
    s3 = qs.workspace_size([_inst(n_xi=64)], qs.QS_FP64)
    assert 0 < s1 < s2 and s1 < s3
    # state of 4 modes padded to one 64-lane block: 64 lanes x 3 values x n_xi
    assert s2 - s1 >= 64 * 3 * 64 * 4


def test_null_arguments():
    qs, L = _lib()
    assert L.qs_step_tau(None, 1, 1, None, None, None) == qs.QS_ERR_ARG
    assert L.qs_sync_check(None) == qs.QS_ERR_ARG
    assert L.qs_steps_done(None) == -1
    L.qs_free(None)
    assert L.qs_init(None, 1, None, None, 0, None) == qs.QS_ERR_ARG


def test_regime_map_arguments_rejected_on_host():
    """qs_regime_map checks its arguments before any device work (host pointers stand in for
    device ones: nothing is launched on these paths)."""
    import ctypes
    qs, L = _lib()
    buf = (ctypes.c_double * 16)()
    p = ctypes.cast(buf, ctypes.c_void_p)
    assert L.qs_regime_map(p, p, 0, 4, 1, qs.QS_FP64, p, None, None) == qs.QS_ERR_ARG       # no modes
    assert L.qs_regime_map(p, p, 4, 0, 1, qs.QS_FP64, p, None, None) == qs.QS_ERR_ARG       # no cells
    assert L.qs_regime_map(p, p, 4, 4, -1, qs.QS_FP64, p, None, None) == qs.QS_ERR_ARG      # negative window
    assert L.qs_regime_map(p, p, 4, 4, 1, 9, p, None, None) == qs.QS_ERR_ARG                # precision
    assert L.qs_regime_map(None, p, 4, 4, 1, qs.QS_FP32, p, None, None) == qs.QS_ERR_ARG    # input
    assert L.qs_regime_map(p, p, 4, 4, 1, qs.QS_FP32, None, None, None) == qs.QS_ERR_ARG    # no output
    assert b"log_ratio" in L.qs_last_error()


def test_device_generator_equals_oracle_generator(oracle):
    qs, L = _lib()
    for seed in (0, 1, 0xDEADBEEF, 2**64 - 1):
        for i in (0, 1, 2, 12345, 2**40 + 7):
            assert L.qs_debug_splitmix64(seed, i) == oracle.splitmix64(seed, i)


def test_failure_handling_entry_points_reject_null_context():
    """qs_set_rollback and the wait-budget hook check their context on the host."""
    qs, L = _lib()
    assert L.qs_set_rollback(None, 1) == qs.QS_ERR_ARG
    assert L.qs_debug_set_wait_budget(None, 0.0) == qs.QS_ERR_ARG
    assert L.qs_sync_check(None) == qs.QS_ERR_ARG


def test_training_gemm_configurations_hold_the_kernel_invariants():
    """Host only: the arguments of every matrix-core GEMM of a training step, at the buffer
    offsets of a real network, against what the GEMM kernel assumes (the same check runs
    before each launch), over the batch sizes qs_mlp_grads accepts, including the 8192 rows
    the surrogate trains with and batches whose row count divides into few splits."""
    import ctypes
    from paper_2607_24234_amd import qs
    L = qs.lib()
    buf = ctypes.create_string_buffer(256)
    for max_batch in (128, 8192, 65536):
        for batch in sorted({128, 384, 640, 1152, 4096, 8192, 8320, 65536}):
            if batch > max_batch:
                continue
            rc = L.qs_debug_mlp_gemm_check(max_batch, batch, buf, 256)
            assert rc == 0, (max_batch, batch, buf.value)
    assert L.qs_debug_mlp_gemm_check(8192, 8192, buf, 256) == 0 and b"16 row splits" in buf.value
    assert L.qs_debug_mlp_gemm_check(8192, 100, buf, 256) == -1
    assert L.qs_debug_mlp_gemm_check(1024, 2048, buf, 256) == -1
