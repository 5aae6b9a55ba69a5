"""Host-side behaviour of the C ABI that needs no GPU: argument validation returns
TF_EINVAL (with a message) before any device call, and the solver choice falls back to
its documented heuristic when nothing has been tuned."""
import ctypes as C
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1806_10550_amd", "libthinfilm.so")
TF_EINVAL = 1

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libthinfilm.so not built")


@pytest.fixture(scope="module")
def L():
    lib = C.CDLL(LIB)
    lib.tf_last_error.restype = C.c_char_p
    lib.tf_create.argtypes = [C.c_int, C.c_int, C.c_double, C.c_void_p, C.POINTER(C.c_void_p)]
    lib.tf_ensemble_create.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                       C.c_double, C.c_double, C.c_void_p, C.POINTER(C.c_void_p)]
    lib.tf_penta_solve.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int,
                                   C.c_void_p]
    lib.tf_autotune.argtypes = [C.c_int, C.c_int, C.c_int, C.c_char_p]
    lib.tf_autotune_load.argtypes = [C.c_char_p]
    lib.tf_autotune_choice.argtypes = [C.c_int, C.c_int, C.c_int]
    lib.tf_set_model.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double]
    lib.tf_step.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    lib.tf_adjoint_step.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p,
                                    C.c_double, C.c_int, C.c_void_p]
    lib.tf_adjoint_steps.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p,
                                     C.c_double, C.c_int, C.c_void_p]
    lib.tf_advance_keep.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
    return lib


def test_create_rejects_bad_geometry(L):
    out = C.c_void_p(1)
    assert L.tf_create(3, 8, 0.5, None, C.byref(out)) == TF_EINVAL
    assert out.value is None
    assert b"nx and ny" in L.tf_last_error()
    assert L.tf_create(8, 8, 0.0, None, C.byref(out)) == TF_EINVAL
    assert L.tf_create(8, 8, float("inf"), None, C.byref(out)) == TF_EINVAL
    assert L.tf_create(8, 8, 0.5, None, None) == TF_EINVAL


def test_ensemble_create_rejects_bad_model(L):
    out = C.c_void_p(1)
    nx = (C.c_int * 1)(64)
    ds = (C.c_double * 1)(0.5)
    assert L.tf_ensemble_create(0, nx, nx, ds, ds, 0.1, 3.0, 2.0, None, C.byref(out)) == TF_EINVAL
    assert L.tf_ensemble_create(1, nx, nx, ds, ds, 0.1, 2.5, 2.0, None, C.byref(out)) == TF_EINVAL
    assert L.tf_ensemble_create(1, nx, nx, ds, ds, 0.1, 2.0, 3.0, None, C.byref(out)) == TF_EINVAL
    assert L.tf_ensemble_create(1, nx, nx, ds, ds, -0.1, 3.0, 2.0, None, C.byref(out)) == TF_EINVAL
    assert b"exponents" in L.tf_last_error()


def test_null_handles(L):
    assert L.tf_set_model(None, 10.0, 0.1, 3.0, 2.0) == TF_EINVAL
    assert L.tf_step(None, None, None) == TF_EINVAL
    assert L.tf_adjoint_step(None, None, None, 0.1, None, None, 1e-10, 10, None) == TF_EINVAL
    assert L.tf_adjoint_steps(None, 1, None, 0.1, None, None, 1e-10, 10, None) == TF_EINVAL
    assert L.tf_advance_keep(None, 1, None, None, None) == TF_EINVAL


def test_penta_solve_validates_before_allocating(L):
    p = C.c_void_p(16)  # never dereferenced: validation fails first
    assert L.tf_penta_solve(0, 8, p, p, p, 0, 0, None) == TF_EINVAL
    assert L.tf_penta_solve(4, 1, p, p, p, 0, 0, None) == TF_EINVAL
    assert L.tf_penta_solve(4, 8, p, p, p, 0, 4, None) == TF_EINVAL
    assert L.tf_penta_solve(4, 4096, p, p, p, 0, 2, None) == TF_EINVAL
    assert b"2048" in L.tf_last_error()
    # the whole-line variant takes lines of 4 ..= 4096 cells
    assert L.tf_penta_solve(4, 3, p, p, p, 1, 3, None) == TF_EINVAL
    assert L.tf_penta_solve(4, 4097, p, p, p, 1, 3, None) == TF_EINVAL
    assert b"4096" in L.tf_last_error()
    assert L.tf_penta_solve_noalloc(4, 4097, p, p, p, 1, 3, None) == TF_EINVAL


def test_autotune_arguments_and_default_choice(L, tmp_path):
    assert L.tf_autotune(1, 16, 0, None) == TF_EINVAL
    assert L.tf_autotune(128, 0, 1, None) == TF_EINVAL
    assert L.tf_autotune_load(None) == TF_EINVAL
    assert L.tf_autotune_load(str(tmp_path / "missing.jsonl").encode()) == TF_EINVAL
    # nothing tuned in this process: partitioned below 65536 lines, Thomas from there on
    assert L.tf_autotune_choice(512, 512, 1) == 0
    assert L.tf_autotune_choice(128, 65536, 0) == 1


def test_clock_arguments(L):
    L.tf_set_clock.argtypes = [C.c_void_p, C.c_double, C.c_int]
    L.tf_get_clock.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    assert L.tf_set_clock(None, 0.0, 0) == TF_EINVAL
    assert L.tf_get_clock(None, None, None) == TF_EINVAL


def test_model_entry_points_reject_null_handles(L):
    D = C.c_double
    L.tf_set_model_linear.argtypes = [C.c_void_p, D, D]
    L.tf_set_model_nlc.argtypes = [C.c_void_p, D, D, D, D, D, D]
    L.tf_set_model_polymer.argtypes = [C.c_void_p, D, D, D, D, D]
    L.tf_ensemble_set_model_nlc.argtypes = [C.c_void_p, D, D, D, D, D, D]
    L.tf_ensemble_set_model_polymer.argtypes = [C.c_void_p, D, D, D, D, D]
    L.tf_ensemble_set_model_linear.argtypes = [C.c_void_p, D, D]
    L.tf_model_coeffs.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]
    assert L.tf_set_model_linear(None, 1.0, 1.0) == TF_EINVAL
    assert L.tf_set_model_nlc(None, 0.0857, 36.0, 1.67, 1.0, 0.05, 0.01) == TF_EINVAL
    assert L.tf_set_model_polymer(None, 0.00581, 1.181, 41.25, -243.75, 191.0) == TF_EINVAL
    assert L.tf_ensemble_set_model_linear(None, 1.0, 1.0) == TF_EINVAL
    assert L.tf_ensemble_set_model_nlc(None, 0.0857, 36.0, 1.67, 1.0, 0.05, 0.01) == TF_EINVAL
    assert L.tf_ensemble_set_model_polymer(None, 0.00581, 1.181, 41.25, -243.75, 191.0) == TF_EINVAL
    assert L.tf_model_coeffs(None, None, 1, None) == TF_EINVAL


def test_radial_spectrum_validates_before_any_device_work(L):
    D = C.c_double
    L.tf_radial_spectrum.argtypes = [C.c_void_p, C.c_int, D, D, D, D, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_int, C.c_void_p]
    n = C.c_int(0)
    p = C.c_void_p(16)  # never dereferenced: validation fails first
    assert L.tf_radial_spectrum(None, 64, 0.1, 1.0, 1.0, 1.0, None, None, None, None, 0, C.byref(n)) == TF_EINVAL
    assert L.tf_radial_spectrum(p, 2, 0.1, 1.0, 1.0, 1.0, None, None, None, None, 0, C.byref(n)) == TF_EINVAL
    assert L.tf_radial_spectrum(p, 64, -0.1, 1.0, 1.0, 1.0, None, None, None, None, 0, C.byref(n)) == TF_EINVAL
    assert L.tf_radial_spectrum(p, 64, 0.1, 1.0, -1.0, 1.0, None, None, None, None, 0, C.byref(n)) == TF_EINVAL
    assert L.tf_radial_spectrum(p, 64, 0.1, 1.0, 1.0, float("nan"), None, None, None, None, 0, C.byref(n)) == TF_EINVAL


def test_binding_checks_field_shapes_before_any_device_call():
    """The C calls take bare pointers to (ny, nx) fields; the Python binding rejects a
    field of another shape before it reaches the library."""
    import torch

    from paper_1806_10550_amd.lib import Grid
    g = object.__new__(Grid)        # no device handle: the check must fire first
    g._h, g.nx, g.ny = None, 8, 6
    good = torch.zeros((6, 8), dtype=torch.float64)
    bad = torch.zeros((8, 6), dtype=torch.float64)
    with pytest.raises(ValueError):
        g.newton_iteration(good, good, bad, 0.1)
    with pytest.raises(ValueError):
        g.flux_divergence(bad, good)
    with pytest.raises(ValueError):
        g.adjoint_step(good, bad, 0.1, good)
    with pytest.raises(ValueError):
        g.jacobian_apply_t(good, good, torch.zeros(48, dtype=torch.float64))
