"""C-ABI entry points beyond the parity path: the device-memory read gives the
same values as the host read, for every quantity, in both modes."""
import numpy as np
import pytest

import mts_inputs as mi
from paper_2403_03605_amd import _lib

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mts():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_03605_amd as m
    m.load()
    return m


@pytest.mark.parametrize("mode", ["coupled", "pure_pd"])
def test_read_device_equals_read(mts, mode):
    import torch
    inst = mi.config(0) if mode == "coupled" else mi.plate2d(30, 2, 4, 1e-8, perturb=1e-6, seed=13,
                                                             mode="pure_pd", name="pure30")
    print("case", inst["name"], flush=True)
    s = mts.Solver(inst)
    s.advance(10)
    qs = [mts.PD_U, mts.PD_V, mts.PD_A, mts.DAMAGE, mts.PD_ALPHA, mts.PD_MASS]
    if mode == "coupled":
        qs += [mts.FE_U, mts.FE_V, mts.FE_A, mts.FE_X, mts.FE_MASS, mts.LAMBDA, mts.CONSTRAINT_NODES, mts.H]
    for q in qs:
        host = s.read(q)
        dev = s.read_device(q)
        s.sync()
        assert np.array_equal(dev.cpu().numpy(), host), q
    # a too small output is rejected before anything is written
    small = torch.zeros(3, dtype=torch.float64, device="cuda")
    with pytest.raises(mts.MtsError):
        s.read_device(mts.PD_U, small)
    s.close()


@pytest.mark.parametrize("which", ["plate", "block"])
def test_caller_arena(mts, which):
    """mts_create_in: the solver lives in a caller-owned torch tensor of the
    planned size and computes exactly what a self-allocating solver computes;
    a region that is too small fails cleanly with MTS_ENOMEM."""
    import torch
    inst = mi.config(0) if which == "plate" else mi.block3d(12, 12, 6, 4, 80, 5e-8, perturb=1e-6, seed=42,
                                                             name="block12")
    print("case", inst["name"], flush=True)
    est = mts.plan(inst)["device_bytes_estimate"]
    ref = mts.Solver(inst)
    used = ref.query()["device_bytes"]
    print("  planned", est, "allocated", used, flush=True)
    assert est >= used
    arena = torch.empty(est, dtype=torch.uint8, device="cuda")
    s = mts.Solver(inst, arena=arena)
    for x in (ref, s):
        x.advance(20)
    for q in (mts.PD_U, mts.PD_V, mts.DAMAGE, mts.FE_U, mts.LAMBDA):
        assert np.array_equal(s.read(q), ref.read(q)), q
    s.close()
    ref.close()
    small = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    with pytest.raises(mts.MtsError) as e:
        mts.Solver(inst, arena=small)
    assert e.value.status == _lib.ENOMEM
