"""The C-ABI library loads and exports every symbol the header declares (CPU;
no compute calls), plus host-side error paths that need no device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import mts_inputs as mi
import paper_2403_03605_amd as mts
from paper_2403_03605_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mtspd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mts_[a-z_]+)\s*\(", src)))


def test_header_declares_binding_exports():
    assert _declared() == sorted(_lib.EXPORTS)


def test_library_exports_every_symbol():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    lib = C.CDLL(_lib.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_struct_layout_matches_header(tmp_path):
    """sizeof/offsetof of the C structs, as the host C compiler lays them out,
    equal the ctypes mirrors used by the binding."""
    checks = []
    for cname, cls in (("mts_problem", _lib.Problem), ("mts_info", _lib.Info), ("mts_plan_info", _lib.PlanInfo),
                      ("mts_pool_info", _lib.PoolInfo), ("mts_energy_info", _lib.EnergyInfo)):
        checks.append((f"sizeof({cname})", C.sizeof(cls)))
        for fname, _ in cls._fields_:
            checks.append((f"offsetof({cname}, {fname})", getattr(cls, fname).offset))
    body = "\n".join(f'  printf("%zu\\n", (size_t){e});' for e, _ in checks)
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "mtspd.h"\nint main(void){\n' + body + "\n  return 0;\n}\n")
    exe = tmp_path / "layout"
    import subprocess
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert got == [v for _, v in checks]


def test_plan_and_validation_on_host():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    inst = mi.config(0)
    pl = mts.plan(inst)
    assert pl["n_pd"] == 1000
    assert pl["nnz_estimate"] >= 25516
    assert pl["device_bytes_estimate"] > 0
    bad = dict(inst, m=0)
    with pytest.raises(mts.MtsError) as e:
        mts.plan(bad)
    assert e.value.status == _lib.EINVAL
    bad = dict(inst, dt_pd=-1.0)
    with pytest.raises(mts.MtsError):
        mts.plan(bad)
    bad = dict(inst, dim=4)
    with pytest.raises(mts.MtsError):
        mts.plan(bad)
    lib = _lib.load()
    assert lib.mts_status_str(_lib.EINVAL) == b"invalid argument"
    lib.mts_destroy(None)
    h = C.c_void_p()
    assert lib.mts_create(None, None, C.byref(h)) == _lib.EINVAL
    assert h.value is None


def _create_status(inst):
    lib = _lib.load()
    p, _pos = _lib.make_problem(inst)
    h = C.c_void_p()
    st = lib.mts_create(C.byref(p), None, C.byref(h))
    return st, h.value


@pytest.mark.parametrize("bad", [
    dict(m=0), dict(dt_pd=0.0), dict(horizon_factor=0.5), dict(dim=1),
    dict(pos=np.zeros((0, 2))),                      # empty lattice
    dict(fe_beta=0.5),                               # only explicit or average acceleration
    dict(clamp_x0=True, vel_bc=1.0),                 # a clamped face moves with no velocity
    dict(mode="pure_pd", traction_x=1e6),            # end traction acts on the FE mesh
    dict(pd_beta=0.25),                              # the implicit PD step runs in pure-PD mode only
    dict(mode="pure_pd", pd_beta=0.25, precision="mixed"),  # ... and in FP64
    dict(mode="pure_pd", pd_beta=0.5),               # only explicit or average acceleration
])
def test_create_rejects_bad_descriptions_before_device_use(bad):
    """Degenerate or inconsistent descriptions are rejected with MTS_EINVAL by
    host-side validation (no device call happens, so this runs on the CPU)."""
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    inst = dict(mi.config(0), **bad)
    st, h = _create_status(inst)
    assert st == _lib.EINVAL and not h
    assert len(_lib.load().mts_last_error()) > 0


def test_pool_rejects_bad_arguments_on_host():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    lib = _lib.load()
    h = C.c_void_p()
    for args in ((0, 4, 2, 1), (1 << 20, 0, 2, 1), (1 << 20, 4, 5, 1), (1 << 20, 4, 2, 7)):
        assert lib.mts_pool_create(args[0], args[1], args[2], args[3], 1, None, C.byref(h)) == _lib.EINVAL
        assert not h.value
    lib.mts_pool_destroy(None)
    assert lib.mts_pool_step(None, None, None, 0, None) == _lib.EINVAL
