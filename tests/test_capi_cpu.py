"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, validates arguments before touching the device, and its
host-side reference element agrees with the oracle."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import oracle as O
import paper_2504_00998_amd as fe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fe.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fe_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert "fe_cheb_filter" in names and "fe_hx_apply" in names and len(names) >= 14
    L = fe.lib()
    for n in names:
        assert hasattr(L, n), n


def _desc(L=(4.0, 4.0, 4.0), ncell=(2, 2, 2), p=3, bc=(0, 0, 0), rule=0):
    return fe._Desc((C.c_double * 3)(*L), (C.c_int32 * 3)(*ncell), p, (C.c_int32 * 3)(*bc), rule)


@pytest.mark.parametrize("kw,msg", [
    (dict(p=0), "p must"), (dict(p=8), "p must"), (dict(ncell=(0, 2, 2)), "ncell"),
    (dict(L=(0.0, 4.0, 4.0)), "L must"), (dict(L=(4.0, 4.0, 5.0)), "cubes"),
    (dict(bc=(1, 0, 0), ncell=(1, 1, 1), L=(2.0, 2.0, 2.0)), "periodic"), (dict(bc=(3, 0, 0)), "boundary"),
    (dict(rule=2), "rule")])
def test_mesh_create_rejects_bad_descriptors_before_device_use(kw, msg):
    h = C.c_void_p()
    st = fe.lib().fe_mesh_create(C.byref(_desc(**kw)), C.byref(h))
    assert st == fe.FE_EINVAL
    assert msg in fe.lib().fe_last_error().decode()
    assert not h.value


def test_null_mesh_is_rejected_everywhere():
    L = fe.lib()
    assert L.fe_hx_apply(None, None, None, 1, 1, 0, None) == fe.FE_EINVAL
    assert L.fe_hx_apply_noalloc(None, None, None, 1, 1, 0, None) == fe.FE_EINVAL
    assert L.fe_cheb_filter(None, None, None, 1, 1, 3, 0.0, 1.0, math.nan, 0, None, 0, None) == fe.FE_EINVAL
    assert L.fe_set_potential(None, None, 0.0, 0.0, None) == fe.FE_EINVAL
    assert L.fe_mesh_info(None, None, None, None) == fe.FE_EINVAL
    assert L.fe_mesh_destroy(None) == fe.FE_OK
    assert L.fe_mesh_create(None, None) == fe.FE_EINVAL


@pytest.mark.parametrize("p", range(1, 8))
@pytest.mark.parametrize("rule", [0, 1])
def test_library_reference_element_matches_oracle(p, rule):
    h = 0.9
    xi, w, A = fe.reference_cell(p, rule, h)
    xo, wo = O.gll(p)
    np.testing.assert_allclose(xi, xo, atol=1e-15)
    np.testing.assert_allclose(w, wo, rtol=1e-14)
    Ko = O.cell_stiffness(p, rule, h)
    assert np.abs(2.0 * A - Ko).max() < 1e-14 * np.abs(Ko).max()


def test_reference_cell_argument_errors():
    L = fe.lib()
    assert L.fe_reference_cell(0, 0, 1.0, None, None, None) == fe.FE_EINVAL
    assert L.fe_reference_cell(3, 0, -1.0, None, None, None) == fe.FE_EINVAL
    assert L.fe_reference_cell(3, 5, 1.0, None, None, None) == fe.FE_EINVAL
    assert L.fe_reference_cell(3, 1, 1.0, None, None, None) == fe.FE_OK


def test_density_entry_points_reject_null_without_a_device():
    import paper_2504_00998_amd as fe
    L = fe.lib()
    assert L.fe_density(None, None, 4, 4, None, None, None) == fe.FE_EINVAL
    assert L.fe_planar_average(None, None, 0, None, None) == fe.FE_EINVAL
    assert L.fe_bare_potential_planar(None, None, None, None, None, None) == fe.FE_EINVAL


def test_poisson_entry_points_reject_null_without_a_device():
    import paper_2504_00998_amd as fe
    L = fe.lib()
    assert L.fe_poisson_work_bytes(None) == 0
    assert L.fe_poisson_solve(None, None, None, 1e-8, 10, None, 0, None, None, None) == fe.FE_EINVAL
    assert L.fe_poisson_solve_cpd(None, None, None, 1.0, 2.0, 0.1, None, 1e-8, 10, None, 0, None, None,
                                  None) == fe.FE_EINVAL


def test_bloch_entry_points_reject_null_without_a_device():
    import paper_2504_00998_amd as fe
    L = fe.lib()
    assert L.fe_set_kpoint(None, 0.1, 0.2) == fe.FE_EINVAL
    assert L.fe_get_kpoint(None, None) == fe.FE_EINVAL
    assert L.fe_hx_apply_k(None, None, None, 4, 4, None) == fe.FE_EINVAL
    assert L.fe_cheb_filter_k(None, None, None, 4, 4, 5, 1.0, 2.0, float("nan"), None, 0, None) == fe.FE_EINVAL
    assert L.fe_cholqr2_k(None, None, 4, 4, None) == fe.FE_EINVAL
    assert L.fe_rayleigh_ritz_k(None, None, None, None, 4, 4, None, None) == fe.FE_EINVAL


def test_header_compiles_as_c(tmp_path):
    """include/fe.h is a C header: a C11 translation unit that includes it and
    calls an entry point compiles warning-free."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("needs gcc")
    src = tmp_path / "use_fe.c"
    src.write_text('#include "fe.h"\nint main(void) { fe_mesh *m = 0; return (int)fe_mesh_destroy(m); }\n')
    r = subprocess.run(["gcc", "-std=c11", "-Wall", "-Wextra", "-Werror", "-fsyntax-only",
                        "-I" + os.path.join(ROOT, "include"), "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__",
                        str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
