"""The bond-pass variants (LDS staging with four- or eight-wavefront
workgroups, direct gathers, tile-ordered or canonical rows, chunk lengths)
compute the same sums in the same order, so with the lanes per row fixed they
give bit-identical trajectories and bond states, including ragged tiles at the
lattice edges and bonds that break."""
import os

import numpy as np
import pytest

import mts_inputs as mi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mts():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_03605_amd as m
    m.load()
    return m


KNOBS = ("MTS_LANES", "MTS_HALO", "MTS_HALO_WAVES", "MTS_TILE", "MTS_PD_VARIANT", "MTS_SUBCYCLE", "MTS_SPIN_LIMIT",
         "MTS_SYM_FORM", "MTS_BUILD_STREAMS")


def _run(mts, inst, n_macro, env):
    saved = {k: os.environ.get(k) for k in KNOBS}
    try:
        for k in KNOBS:
            os.environ.pop(k, None)
        os.environ.update(env)
        s = mts.Solver(inst)  # the knobs are read when the solver is created
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    mu0 = s.bonds()[2]
    s.advance(n_macro)
    out = {q: s.read(q) for q in (mts.PD_U, mts.PD_V, mts.DAMAGE, mts.FE_U)}
    out["mu"] = s.bonds()[2]
    s.close()
    return out, int(((mu0 == 1) & (out["mu"] == 0)).sum())  # bonds broken during the run


def _same(a, b):
    for k in a:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_3d_variants_bit_identical(mts, precision):
    # 12 x 12 x 6 nodes: 8 x 4 x 4 and 4 x 4 x 4 tiles are ragged in x and z
    inst = mi.block3d(12, 12, 6, 4, 80, 5e-8, perturb=1e-6, seed=42, precision=precision,
                      name="block12 " + precision)
    print("case", inst["name"], flush=True)
    ref, nb = _run(mts, inst, 20, {"MTS_LANES": "4"})
    assert nb > 0
    for env in ({"MTS_LANES": "4", "MTS_HALO_WAVES": "8"}, {"MTS_LANES": "4", "MTS_HALO_WAVES": "4"},
                {"MTS_LANES": "4", "MTS_HALO": "0"}, {"MTS_LANES": "4", "MTS_TILE": "0"}):
        print("  variant", env, flush=True)
        got, _ = _run(mts, inst, 20, env)
        _same(ref, got)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_2d_variants_bit_identical(mts, precision):
    inst = dict(mi.config(0, precision=precision), name="plate50 " + precision)
    print("case", inst["name"], flush=True)
    ref, nb = _run(mts, inst, 50, {"MTS_LANES": "2"})
    assert nb > 0
    for env in ({"MTS_LANES": "2", "MTS_HALO": "0"}, {"MTS_LANES": "2", "MTS_HALO": "0", "MTS_PD_VARIANT": "1"},
                {"MTS_LANES": "2", "MTS_HALO": "0", "MTS_PD_VARIANT": "2"}, {"MTS_LANES": "2", "MTS_HALO_WAVES": "8"},
                {"MTS_LANES": "2", "MTS_TILE": "0"}):
        print("  variant", env, flush=True)
        got, _ = _run(mts, inst, 50, env)
        _same(ref, got)
    # four lanes per row: 7 iterations, so the mixed staged pass's last paired
    # slot record is half empty
    ref4, _ = _run(mts, inst, 50, {"MTS_LANES": "4"})
    print("  variant lanes 4, staged vs direct", flush=True)
    got, _ = _run(mts, inst, 50, {"MTS_LANES": "4", "MTS_HALO": "0"})
    _same(ref4, got)


@pytest.mark.parametrize("dim", [2, 3])
def test_fe_passes_in_link_launches_bit_identical(mts, dim):
    """Within one mts_advance call the next macro step's FE free step runs as
    extra workgroups of the link launches (2D); one macro step per call runs it
    on its own launches.  Both orders compute the same values."""
    if dim == 2:
        inst = dict(mi.config(0), name="plate50 fp64")
    else:
        inst = mi.block3d(12, 12, 6, 4, 80, 5e-8, perturb=1e-6, seed=43, name="block12 fp64")
    print("case", inst["name"], flush=True)
    n = 12
    a = mts.Solver(inst)
    a.advance(n)
    b = mts.Solver(inst)
    for _ in range(n):
        b.advance(1)
    for q in (mts.PD_U, mts.PD_V, mts.FE_U, mts.FE_V, mts.FE_A, mts.LAMBDA, mts.DAMAGE):
        assert np.array_equal(a.read(q), b.read(q)), q
    a.close()
    b.close()


@pytest.mark.parametrize("case", ["plate50 fp64", "plate50 mixed", "block12 fp64", "block12 mixed"])
def test_subcycle_launch_bit_identical(mts, case):
    """The m substeps of a macro step as one launch (the opt-in subcycle
    kernel: workgroups resident for the whole subcycle, each waiting only for
    the tiles it shares nodes with) give the same trajectories and bond
    states, bit for bit, as one launch per substep, through breaks."""
    name, prec = case.split()
    if name == "plate50":
        inst = dict(mi.config(0, precision=prec), name=case)
        n = 50
    else:
        inst = mi.block3d(12, 12, 6, 4, 80, 5e-8, perturb=1e-6, seed=42, precision=prec, name=case)
        n = 20
    print("case", inst["name"], flush=True)
    ref, nb = _run(mts, inst, n, {"MTS_SUBCYCLE": "0"})
    assert nb > 0
    got, _ = _run(mts, inst, n, {"MTS_SUBCYCLE": "1"})
    _same(ref, got)


def test_subcycle_wait_gives_up_cleanly(mts):
    """With the poll limit forced to zero the subcycle kernel's waits give up
    at once: the kernel still ends, and the solver reports MTS_EDEVICE (sticky)
    instead of results."""
    inst = dict(mi.config(0), name="plate50 give-up")
    saved = {k: os.environ.get(k) for k in KNOBS}
    try:
        for k in KNOBS:
            os.environ.pop(k, None)
        os.environ.update({"MTS_SUBCYCLE": "1", "MTS_SPIN_LIMIT": "0"})
        s = mts.Solver(inst)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    with pytest.raises(mts.MtsError) as e:
        s.advance(6)
        s.sync()
    assert e.value.status == 3  # MTS_EDEVICE
    with pytest.raises(mts.MtsError):
        s.advance(1)
    s.close()


@pytest.mark.parametrize("nx", [200, 400])
def test_inverse_tile_pruning(mts, nx):
    """The multiplier solve skips the tiles of the inverse of H whose entries
    are below 1e-18 of the largest: the multipliers and the PD/FE state stay
    within 1e-13 (max relative) of the solve that reads every tile, and fewer
    bytes are read."""
    inst = mi.plate2d(nx, 10, 10 * 20, 6e-9 * 400 / nx, perturb=1e-6, seed=91, name=f"plate {nx} m=10")
    print("case", inst["name"], flush=True)
    out = {}
    for drop in ("1", "0"):
        saved = os.environ.get("MTS_INV_DROP")
        os.environ["MTS_INV_DROP"] = drop
        try:
            s = mts.Solver(inst)
        finally:
            if saved is None:
                os.environ.pop("MTS_INV_DROP", None)
            else:
                os.environ["MTS_INV_DROP"] = saved
        s.advance(20)
        out[drop] = ({q: s.read(q) for q in (mts.LAMBDA, mts.PD_U, mts.PD_V, mts.FE_V)}, s.query()["inverse_bytes"])
        s.close()
    (a, ba), (b, bb) = out["1"], out["0"]
    print("  inverse bytes read", ba, "of", bb, flush=True)
    assert ba < bb
    for q in a:
        w = np.abs(b[q]).max()
        assert w > 0
        assert np.abs(a[q] - b[q]).max() <= 1e-13 * w, q


def _rebuild_cases():
    c1 = mi.config(0)
    c1i = dict(mi.config(0), fe_beta=0.25, name="plate 50x20 m=4 implicit FE")
    br = mi.branching2d(80)
    br["n_macro"] = 60
    blk = mi.block3d(12, 12, 6, 4, 160, 5e-8, perturb=1e-6, seed=42, name="block12 glass")
    return [c1, c1i, br, blk]


@pytest.mark.parametrize("inst", _rebuild_cases(), ids=lambda i: i["name"])
def test_incremental_rebuild_bit_identical(mts, inst):
    """A rebuild recomputes only the unit-load columns whose response reach
    holds a node with a changed bond; the rest would come out bit for bit the
    same, so every state, the multipliers and the bond states equal those of
    rebuilds that recompute every column (MTS_FULL_REBUILD=1)."""
    print("case", inst["name"], flush=True)
    out = {}
    for full in ("0", "1"):
        saved = os.environ.get("MTS_FULL_REBUILD")
        os.environ["MTS_FULL_REBUILD"] = full
        try:
            s = mts.Solver(inst)
        finally:
            if saved is None:
                os.environ.pop("MTS_FULL_REBUILD", None)
            else:
                os.environ["MTS_FULL_REBUILD"] = saved
        for _ in range(0, inst["n_macro"], 5):
            s.advance(5)
        q = s.query()
        st = {k: s.read(k) for k in (mts.PD_U, mts.PD_V, mts.DAMAGE, mts.FE_U, mts.FE_V, mts.LAMBDA)}
        st["mu"] = s.bonds()[2]
        out[full] = (st, q["n_rebuilds"], q["n_rebuild_columns"], q["n_constraints"])
        s.close()
    (a, na, ca, nc), (b, nb, cb, _) = out["0"], out["1"]
    print(f"  rebuilds {na}, columns recomputed {ca} of {nb * nc}", flush=True)
    assert na == nb and na > 0
    assert cb == nb * nc and 0 < ca <= cb
    _same(a, b)


@pytest.mark.parametrize("inst", _rebuild_cases(), ids=lambda i: i["name"])
def test_multiplier_solve_forms_bit_identical(mts, inst):
    """The multiplier solve's two forms (every load of a tile at once with
    per-wavefront lists of kept partial sums, MTS_SYM_FORM=1; quarters of a
    tile streamed with a reduction over every tile, MTS_SYM_FORM=2) give the
    same bits, through rebuilds of the unit-load responses and the inverse."""
    print("case", inst["name"], flush=True)
    a, nb = _run(mts, inst, inst["n_macro"], {"MTS_SYM_FORM": "1"})
    b, _ = _run(mts, inst, inst["n_macro"], {"MTS_SYM_FORM": "2"})
    assert nb > 0
    _same(a, b)


@pytest.mark.parametrize("inst", _rebuild_cases(), ids=lambda i: i["name"])
def test_build_streams_bit_identical(mts, inst):
    """The colour batches of a build (setup and every rebuild) run on four
    streams at once, each batch with its own response buffers and its own
    columns of H; one stream (MTS_BUILD_STREAMS=1) gives the same bits."""
    print("case", inst["name"], flush=True)
    a, nb = _run(mts, inst, inst["n_macro"], {"MTS_BUILD_STREAMS": "1"})
    b, _ = _run(mts, inst, inst["n_macro"], {"MTS_BUILD_STREAMS": "4"})
    assert nb > 0
    _same(a, b)
