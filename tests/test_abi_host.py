"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/qsv.h declares, has the documented struct layout, and
rejects invalid arguments before touching the device."""
import ctypes

import numpy as np

import pytest

from paper_1807_07914_amd import qsv


def test_library_exports_every_header_function():
    names = qsv.header_functions()
    assert "qsv_alloc_state" in names and "qsv_sample" in names
    L = qsv.lib()
    missing = [f for f in names if not hasattr(L, f)]
    assert not missing, missing


def test_plan_opts_layout():
    assert ctypes.sizeof(qsv.QsvPlanOpts) == 32
    assert qsv.QsvPlanOpts.state_is_output.offset == 8 and qsv.QsvPlanOpts.graph.offset == 12
    assert qsv.QsvPlanOpts.race_check.offset == 16 and qsv.QsvPlanOpts.reserved.offset == 20


def test_op_struct_is_64_bytes():
    assert ctypes.sizeof(qsv.QsvOp) == 64
    assert qsv.QsvOp.mat.offset == 56 and qsv.QsvOp.p.offset == 32


@pytest.mark.parametrize("n,dt", [(0, 1), (41, 1), (-3, 2), (10, 0), (10, 3)])
def test_alloc_rejects_bad_arguments(n, dt):
    h = ctypes.c_void_p()
    rc = qsv.lib().qsv_alloc_state(n, dt, None, 0, None, ctypes.byref(h))
    assert rc == qsv.QSV_ERR_ARG
    assert h.value is None
    assert qsv.lib().qsv_last_error()


def test_foreign_handles_rejected():
    L = qsv.lib()
    bogus = ctypes.c_void_p(0x1234)
    assert L.qsv_free_state(None) == qsv.QSV_OK
    assert L.qsv_free_state(bogus) == qsv.QSV_ERR_STATE
    assert L.qsv_state_info(bogus, None, None, None) == qsv.QSV_ERR_STATE
    assert L.qsv_set_basis(bogus, 0) == qsv.QSV_ERR_STATE
    out = ctypes.c_double()
    assert L.qsv_norm(bogus, ctypes.byref(out)) == qsv.QSV_ERR_STATE
    assert b"invalid" in L.qsv_last_error()


@pytest.mark.parametrize("n,chi,cut", [(0, 4, 1e-4), (1025, 4, 1e-4), (8, 0, 1e-4), (8, 65, 1e-4),
                                       (8, 4, -1.0), (8, 4, float("nan")), (8, 4, float("inf"))])
def test_mps_alloc_rejects_bad_arguments(n, chi, cut):
    # argument checks come before any device call, so they run without a GPU
    h = ctypes.c_void_p()
    rc = qsv.lib().qsv_mps_alloc(n, chi, cut, None, ctypes.byref(h))
    assert rc == qsv.QSV_ERR_ARG and h.value is None
    assert qsv.lib().qsv_last_error()


def test_mps_foreign_handles_rejected():
    L = qsv.lib()
    bogus = ctypes.c_void_p(0x1234)
    assert L.qsv_mps_free(None) == qsv.QSV_OK
    assert L.qsv_mps_free(bogus) == qsv.QSV_ERR_STATE
    assert L.qsv_mps_apply_circuit(bogus, None, 0) == qsv.QSV_ERR_STATE
    dims = (ctypes.c_int32 * 4)()
    assert L.qsv_mps_bonds(bogus, dims, None) == qsv.QSV_ERR_STATE
    assert L.qsv_mps_info(bogus, None, None) == qsv.QSV_ERR_STATE
    assert b"invalid" in L.qsv_last_error()


def test_pauli_mask_encoding():
    x, z, c = qsv.pauli_masks([(0.5, (("X", 0), ("Y", 2), ("Z", 3)))])
    assert int(x[0]) == 0b0101 and int(z[0]) == 0b1100 and c[0] == 0.5
    with pytest.raises(ValueError):
        qsv.pauli_masks([(1.0, (("X", 1), ("Z", 1)))])


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_launch_geometry_up_to_the_largest_register(dtype):
    # every per-gate launch covers its whole range with a grid whose
    # dimensions each stay below 2^32 work-items, up to 2^35 complex64 /
    # 2^34 complex128 amplitudes (256 GiB); larger registers are refused
    import ctypes
    from paper_1807_07914_amd import qsv
    fn = qsv.lib().qsv_debug_launch_dims
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]
    dt = qsv.QSV_C64 if dtype == "c64" else qsv.QSV_C128
    top = 35 if dtype == "c64" else 34
    out = np.zeros(44, dtype=np.int64)
    ptr = out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    for n in range(7, top + 1):
        assert fn(dt, n, ptr) == 0
        rows = out.reshape(11, 4)
        for gx, gy, threads, need in rows:
            assert 1 <= gx <= 65536 and gy >= 1
            assert gx * threads < 2 ** 32 and gy < 2 ** 32
            assert gx * gy >= need and gx * (gy - 1) < need  # covers the range, one row at most overhangs
    assert fn(dt, top + 1, ptr) != 0
    assert qsv.lib().qsv_alloc_state(top + 1, dt, None, 0, None, ctypes.byref(ctypes.c_void_p())) != 0


def test_noalloc_expval_checks_arguments_on_the_host():
    # argument errors are reported before any device work
    import ctypes
    L = qsv.lib()
    z = np.zeros(1, dtype=np.uint64)
    c = np.ones(1)
    u64 = ctypes.POINTER(ctypes.c_uint64)
    dp = ctypes.POINTER(ctypes.c_double)
    tot = ctypes.c_double()
    args = (z.ctypes.data_as(u64), z.ctypes.data_as(u64), c.ctypes.data_as(dp))
    assert L.qsv_expval_noalloc(None, 10, qsv.QSV_C64, *args, 1, None, ctypes.byref(tot), None) == qsv.QSV_ERR_ARG
    assert L.qsv_expval_noalloc(ctypes.c_void_p(256), 10, 7, *args, 1, None, ctypes.byref(tot), None) == qsv.QSV_ERR_ARG
    assert L.qsv_expval_noalloc(ctypes.c_void_p(256), 36, qsv.QSV_C64, *args, 1, None, ctypes.byref(tot),
                                None) == qsv.QSV_ERR_ARG
    assert L.qsv_expval_noalloc(ctypes.c_void_p(256), 10, qsv.QSV_C64, *args, 40000, None, ctypes.byref(tot),
                                None) == qsv.QSV_ERR_ARG
    assert L.qsv_expval_noalloc(ctypes.c_void_p(8), 10, qsv.QSV_C64, *args, 1, None, ctypes.byref(tot),
                                None) == qsv.QSV_ERR_ARG  # misaligned
