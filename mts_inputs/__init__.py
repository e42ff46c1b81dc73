"""Seeded synthetic problem instances for the multi-time-step PD/FE fracture solver.

This module is shared by the oracle (test infrastructure) and the HIP library's
callers.  It holds no arithmetic of the method itself: it only lays out node
positions on a lattice, draws the seeded perturbation, and records the plain
problem parameters (geometry, material, loads, step ratio, step count).  Every
quantity the method derives from these (horizon, micromodulus, critical stretch,
Arlequin weights, masses, neighbour lists, multipliers) is computed separately
by each side.

Instances stand in for the paper's plate workloads (Sec. 3.3 efficiency study and
Sec. 4.1 crack branching: a 100 x 40 mm plate with an edge notch, PD placed
around the crack, Q4 elements elsewhere, step ratios 2..20).  The paper uses no
public dataset; all inputs here are synthetic.
"""
from __future__ import annotations

import math
from typing import Dict, Iterator, List, Optional

import numpy as np

MASK64 = (1 << 64) - 1
SEED_BASE = 240303605
SERVING_SEED = 240303700


# ---------------------------------------------------------------------------
# SplitMix64 (Vigna, "Further scramblings of Marsaglia's xorshift generators",
# the seeding generator of xoroshiro).  Written from its published definition.
# ---------------------------------------------------------------------------
class SplitMix64:
    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        """Uniform double in [0, 1) with 53 random bits."""
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)


def splitmix64_uniforms(seed: int, count: int) -> np.ndarray:
    """`count` consecutive SplitMix64 uniforms, vectorised (same stream as the class)."""
    golden = np.uint64(0x9E3779B97F4A7C15)
    with np.errstate(over="ignore"):
        k = np.arange(1, count + 1, dtype=np.uint64)
        z = np.uint64(seed & MASK64) + k * golden
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def lattice_positions(n, lo, dx: float, perturb: float = 0.0, seed: int = SEED_BASE) -> np.ndarray:
    """Cell-centred lattice of n[0] x n[1] (x n[2]) nodes starting at `lo`.

    Node id = (iz * ny + iy) * nx + ix.  Each coordinate gets (2u - 1) * perturb * dx
    with u drawn from SplitMix64(seed) in node-id order, x then y (then z).
    Returns an (N, dim) float64 array.
    """
    dim = len(n)
    axes = [lo[a] + (np.arange(n[a], dtype=np.float64) + 0.5) * dx for a in range(dim)]
    if dim == 2:
        yy, xx = np.meshgrid(axes[1], axes[0], indexing="ij")
        pos = np.stack([xx.ravel(), yy.ravel()], axis=1)
    else:
        zz, yy, xx = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
        pos = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    pos = np.ascontiguousarray(pos)
    if perturb > 0.0:
        u = splitmix64_uniforms(seed, pos.size).reshape(pos.shape)
        pos = pos + (2.0 * u - 1.0) * (perturb * dx)
    return pos


# ---------------------------------------------------------------------------
# Instances
# ---------------------------------------------------------------------------
GLASS = dict(E=72e9, rho=2440.0, G0=3.8)
# steel of the paper's impact example (Sec. 4.2): critical stretch given directly
STEEL = dict(E=191e9, rho=8000.0, G0=0.0, s_crit=0.01)


def plate2d(nx: int, m: int, n_pd_steps: int, dt_pd: float, *, perturb: float = 0.0,
            seed: int = SEED_BASE, precision: str = "fp64", traction: float = 1e6,
            notch: Optional[float] = None, crack_y: Optional[float] = None,
            mode: str = "coupled", breaking: bool = True, weight: str = "cubic",
            kernel: str = "pmb", name: str = "plate2d") -> Dict:
    """2D plane-stress plate 0.1 x 0.04 m with an edge notch along y = crack_y.

    PD lattice nx x (0.4 nx) nodes of spacing dx = 0.05 / nx covering the strip
    x in [a - 0.01, a + 0.04], y in [0.01, 0.03] (for the default notch a = 0.05),
    Q4 elements of size 4 dx over the whole plate, overlap 3 dx, traction on the
    edges y = 0 and y = 0.04.
    """
    assert nx % 2 == 0 and (2 * nx) % 5 == 0
    ny = (2 * nx) // 5
    dx = 0.05 / nx
    L, Hh = 0.1, 0.04
    a = 0.05 if notch is None else notch
    yc = 0.02 if crack_y is None else crack_y
    x0 = a - 0.2 * 0.05
    y0 = yc - 0.5 * ny * dx
    fe_h = 4.0 * dx
    pd_lo = (x0, y0)
    pd_hi = (x0 + nx * dx, y0 + ny * dx)
    inst = dict(
        name=name, dim=2, mode=mode, precision=precision, breaking=breaking,
        pd_n=(nx, ny, 1), pd_lo=pd_lo, pd_hi=pd_hi, dx=dx, horizon_factor=3.015,
        perturb=perturb, seed=seed,
        dom_lo=(0.0, 0.0), dom_hi=(L, Hh),
        fe_n=(int(round(L / fe_h)), int(round(Hh / fe_h)), 1), fe_h=fe_h,
        overlap=3.0 * dx, weight=weight,
        cracks=[(yc, 0.0, a)],
        thickness=1.0, kernel=kernel, l_over_delta=0.1,
        traction=traction, vel_bc=0.0,
        m=m, dt_pd=dt_pd, n_macro=n_pd_steps // m, **GLASS,
    )
    if mode == "pure_pd":
        inst.update(dom_lo=pd_lo, dom_hi=pd_hi, fe_n=(0, 0, 0))
    inst["pos"] = lattice_positions((nx, ny), pd_lo, dx, perturb, seed)
    return inst


def block3d(nx: int, ny: int, nz: int, m: int, n_pd_steps: int, dt_pd: float, *,
            perturb: float = 0.0, seed: int = SEED_BASE, precision: str = "fp64",
            vel_bc: float = 20.0, mode: str = "coupled", breaking: bool = True,
            material: str = "glass", name: str = "block3d") -> Dict:
    """3D PD block nx x ny x nz (dx = 1 mm scale: dx = 0.02 / nz) spanning the full
    width and thickness of a hex8 bar 2 nx dx long, centred along x; prescribed
    velocity vel_bc on the bar face x = 0.  material: "glass" or "steel"."""
    dx = 0.02 / nz
    Lx, Ly, Lz = 2.0 * nx * dx, ny * dx, nz * dx
    pd_lo = (0.5 * nx * dx, 0.0, 0.0)
    pd_hi = (1.5 * nx * dx, Ly, Lz)
    fe_h = 2.0 * dx
    inst = dict(
        name=name, dim=3, mode=mode, precision=precision, breaking=breaking,
        pd_n=(nx, ny, nz), pd_lo=pd_lo, pd_hi=pd_hi, dx=dx, horizon_factor=3.015,
        perturb=perturb, seed=seed,
        dom_lo=(0.0, 0.0, 0.0), dom_hi=(Lx, Ly, Lz),
        fe_n=(int(round(Lx / fe_h)), int(round(Ly / fe_h)), int(round(Lz / fe_h))), fe_h=fe_h,
        overlap=3.0 * dx, weight="cubic", cracks=[],
        thickness=1.0, kernel="pmb", l_over_delta=1.0 / 16.0,
        traction=0.0, vel_bc=vel_bc,
        m=m, dt_pd=dt_pd, n_macro=n_pd_steps // m, **(STEEL if material == "steel" else GLASS),
    )
    if mode == "pure_pd":
        inst.update(dom_lo=pd_lo, dom_hi=pd_hi, fe_n=(0, 0, 0))
    inst["pos"] = lattice_positions((nx, ny, nz), pd_lo, dx, perturb, seed)
    return inst


# Duran glass of the paper's crack-branching example (Sec. 4.1): critical
# stretch given directly
DURAN = dict(E=65e9, rho=2235.0, G0=0.0, s_crit=0.002689)


def branching2d(nx: int = 400, mode: str = "coupled", *, m: int = 10, t_end: float = 6e-5,
                precision: str = "fp64", perturb: float = 0.0, seed: int = SEED_BASE + 4,
                traction: float = 12e6, name: Optional[str] = None) -> Dict:
    """The crack-branching plate of the paper's Sec. 4.1: a 100 x 40 mm glass
    plate with a 50 mm edge notch along y = 20 mm, traction on the upper and
    lower edges, dx = 0.1 / nx (0.25 mm at nx = 400).

    mode "pure_pd": PD nodes over the whole plate (nx x 0.4 nx), the traction
    as a body force over a layer of width delta.  mode "coupled": a PD box of
    55 x 30 mm (41.25 % of the plate) at x in [45, 100] mm, y in [5, 35] mm,
    reaching the right edge, with an overlap band of 3 dx on its faces inside
    the plate, and Q4 elements of 4 dx over the plate.  The PD step is 1e-8 s at
    nx = 400 (scaled with dx), the FE step m times that; the run covers t_end."""
    assert nx % 20 == 0
    dx = 0.1 / nx
    L, Hh = 0.1, 0.04
    dt = 1e-8 * (400.0 / nx)
    if mode == "pure_pd":
        pd_lo, pd_hi = (0.0, 0.0), (L, Hh)
        n = (nx, (2 * nx) // 5)
        m_eff = 1
    else:
        pd_lo, pd_hi = (0.045, 0.005), (L, 0.035)
        n = ((11 * nx) // 20, (3 * nx) // 10)
        m_eff = m
    fe_h = 4.0 * dx
    n_pd_steps = int(round(t_end / dt))
    inst = dict(
        name=name or f"branching {n[0]}x{n[1]} {'pure PD' if mode == 'pure_pd' else f'm={m}'} {precision}",
        dim=2, mode=mode, precision=precision, breaking=True,
        pd_n=(n[0], n[1], 1), pd_lo=pd_lo, pd_hi=pd_hi, dx=dx, horizon_factor=3.015,
        perturb=perturb, seed=seed, dom_lo=(0.0, 0.0), dom_hi=(L, Hh),
        fe_n=(int(round(L / fe_h)), int(round(Hh / fe_h)), 1) if mode != "pure_pd" else (0, 0, 0),
        fe_h=fe_h, overlap=3.0 * dx, weight="cubic", cracks=[(0.02, 0.0, 0.05)],
        thickness=1.0, kernel="pmb", l_over_delta=0.1, traction=traction, vel_bc=0.0,
        m=m_eff, dt_pd=dt, n_macro=n_pd_steps // m_eff, **DURAN,
    )
    inst["pos"] = lattice_positions(n, pd_lo, dx, perturb, seed)
    return inst


def efficiency2d(dx: float = 5e-4, *, pd_frac: float = 0.1, m: int = 2, fe_beta: float = 0.25,
                 pd_beta: float = 0.0, n_macro: int = 100, precision: str = "fp64", perturb: float = 0.0,
                 seed: int = SEED_BASE + 6, name: Optional[str] = None) -> Dict:
    """The mode-I plate of the paper's efficiency study (Sec. 3.3, Table 2),
    turned by 90 degrees so that the notch is horizontal: a 40 x 100 mm plate
    (x by y) with a 10 mm edge notch along y = 50 mm from x = 0, 16 MPa on the
    faces y = 0 and y = 100 mm, E = 72 GPa, rho = 2235 kg/m^3, G0 = 204 J/m^2,
    exponential micromodulus with l = delta / 10, PD step 5e-9 s.  pd_frac:
    0.1 (a 20 x 20 mm PD box at the notch), 0.2 (a 40 x 20 mm strip across the
    plate) or 1.0 (pure PD over the plate, the traction as a body force within
    delta of the loaded faces).  Q4 elements of 4 dx, implicit FE step by
    default (the paper's choice for this study); pd_beta = 1/4 makes the PD
    step implicit (pure PD only, the study's case 1)."""
    W, H = 0.04, 0.1
    pure = pd_frac >= 1.0
    if pure:
        pd_lo, pd_hi = (0.0, 0.0), (W, H)
    elif abs(pd_frac - 0.2) < 1e-9:
        pd_lo, pd_hi = (0.0, 0.04), (W, 0.06)
    elif abs(pd_frac - 0.1) < 1e-9:
        pd_lo, pd_hi = (0.0, 0.04), (0.02, 0.06)
    else:
        raise ValueError(pd_frac)
    n = (int(round((pd_hi[0] - pd_lo[0]) / dx)), int(round((pd_hi[1] - pd_lo[1]) / dx)))
    fe_h = 4.0 * dx
    inst = dict(
        name=name or (f"efficiency plate {n[0]}x{n[1]} pure PD{' implicit' if pd_beta else ''} {precision}" if pure else
                      f"efficiency plate PD {int(round(100 * pd_frac))}% m={m} {precision}"),
        dim=2, mode="pure_pd" if pure else "coupled", precision=precision, breaking=True,
        pd_n=(n[0], n[1], 1), pd_lo=pd_lo, pd_hi=pd_hi, dx=dx, horizon_factor=3.015,
        perturb=perturb, seed=seed, dom_lo=pd_lo if pure else (0.0, 0.0), dom_hi=pd_hi if pure else (W, H),
        fe_n=(0, 0, 0) if pure else (int(round(W / fe_h)), int(round(H / fe_h)), 1), fe_h=fe_h,
        overlap=3.0 * dx, weight="cubic", cracks=[(0.05, 0.0, 0.01)],
        thickness=1.0, kernel="exp", l_over_delta=0.1, traction=16e6, vel_bc=0.0,
        fe_beta=0.0 if pure else fe_beta, pd_beta=pd_beta if pure else 0.0, m=1 if pure else m, dt_pd=5e-9,
        n_macro=n_macro,
        E=72e9, rho=2235.0, G0=204.0,
    )
    inst["pos"] = lattice_positions(n, pd_lo, dx, perturb, seed)
    return inst


# Elastic beam of the paper's error study (Sec. 3.2): E = 6.5 GPa, rho = 2235,
# no breaking (the critical stretch is nominal).
BEAM = dict(E=6.5e9, rho=2235.0, G0=0.0, s_crit=1.0)


def beam3d(dx: float = 0.05, *, weight: str = "cubic", overlap_cells: int = 3, m: int = 1,
           dt_fe: float = 2.5e-5, t_end: float = 0.025, fe_beta: float = 0.0, mode: str = "coupled",
           precision: str = "fp64", traction: float = 4e6, name: Optional[str] = None) -> Dict:
    """The 1 x 1 x 10 m beam of the paper's Sec. 3.2: fixed at x = 0, a uniform
    traction (+x) on the end x = 10 m, Hex8 elements of size dx over the beam,
    PD nodes (cell-centred, spacing dx) over 4 < x < 6 with an overlap of
    overlap_cells * dx on the two faces inside the beam, horizon 3.03 dx,
    exponential micromodulus with l = delta / 16.  The FE step is dt_fe, the
    PD step dt_fe / m; the run covers t_end.  mode "pure_fe": the undecomposed
    FE model (no PD nodes), the paper's reference.  The tracked point A is the
    FE node at the centre of the loaded end (`beam_node_a`)."""
    L, W = 10.0, 1.0
    n_len, n_w, n_pd = int(round(L / dx)), int(round(W / dx)), int(round(2.0 / dx))
    assert n_w % 2 == 0 and abs(n_len * dx - L) < 1e-9 * L
    pd_lo, pd_hi = (4.0, 0.0, 0.0), (6.0, W, W)
    inst = dict(
        name=name or f"beam {n_len}x{n_w}x{n_w} {weight} lO={overlap_cells}dx m={m} "
                     f"{'implicit' if fe_beta else 'explicit'} FE {precision}",
        dim=3, mode=mode, precision=precision, breaking=False,
        pd_n=(n_pd, n_w, n_w), pd_lo=pd_lo, pd_hi=pd_hi, dx=dx, horizon_factor=3.03,
        perturb=0.0, seed=SEED_BASE + 5, dom_lo=(0.0, 0.0, 0.0), dom_hi=(L, W, W),
        fe_n=(n_len, n_w, n_w), fe_h=dx, overlap=overlap_cells * dx, weight=weight, cracks=[],
        thickness=1.0, kernel="exp", l_over_delta=1.0 / 16.0, traction=0.0, vel_bc=0.0,
        traction_x=traction, clamp_x0=True, fe_beta=fe_beta,
        m=m, dt_pd=dt_fe / m, n_macro=int(round(t_end / dt_fe)), **BEAM,
    )
    if mode == "pure_fe":
        inst["pos"] = np.zeros((0, 3))
    else:
        inst["pos"] = lattice_positions((n_pd, n_w, n_w), pd_lo, dx)
    return inst


def beam_node_a(inst: Dict) -> int:
    """FE node id of the beam's tracked point A, the centre of the loaded end
    (grid node ids run x fastest, then y, then z)."""
    nx, ny, nz = inst["fe_n"]
    return ((nz // 2) * (ny + 1) + ny // 2) * (nx + 1) + nx


# Step sizes (s): at most 0.8 of the smaller of the PD stability bound and the
# explicit-FE bound divided by m, and below the Gershgorin FE bound / m.  The
# bounds scale with dx for these layouts; the test suite re-derives them.
DT = {
    "plate50": 1.0e-7,
    "plate400": 6.0e-9,
    "plate1000": 2.4e-9,
    "block100": 2.5e-8,
}


def config(k: int, **over) -> Dict:
    """The five workloads: 0 small 2D, 1 plain FP64 2D, 2 mixed 2D, 3 mixed 3D.
    An overridden precision is reflected in the name."""
    inst = _config(k, **over)
    if "precision" in over and "name" not in over:
        base, _, last = inst["name"].rpartition(" ")
        if last in ("fp64", "mixed"):
            inst["name"] = f"{base} {inst['precision']}"
    return inst


def _config(k: int, **over) -> Dict:
    if k == 0:
        kw = dict(nx=50, m=4, n_pd_steps=200, dt_pd=DT["plate50"], perturb=0.0, seed=SEED_BASE,
                  precision="fp64", name="plate 50x20 m=4 fp64")
        kw.update(over)
        return plate2d(**kw)
    if k == 1:
        kw = dict(nx=400, m=10, n_pd_steps=4000, dt_pd=DT["plate400"], perturb=1e-6,
                  seed=SEED_BASE + 1, precision="fp64", name="plate 400x160 m=10 fp64")
        kw.update(over)
        return plate2d(**kw)
    if k == 2:
        kw = dict(nx=1000, m=10, n_pd_steps=5000, dt_pd=DT["plate1000"], perturb=1e-6,
                  seed=SEED_BASE + 2, precision="mixed", name="plate 1000x400 m=10 mixed")
        kw.update(over)
        return plate2d(**kw)
    if k == 3:
        kw = dict(nx=100, ny=100, nz=20, m=8, n_pd_steps=2000, dt_pd=DT["block100"], perturb=1e-6,
                  seed=SEED_BASE + 3, precision="mixed", material="steel",
                  name="block 100x100x20 m=8 mixed")
        kw.update(over)
        return block3d(**kw)
    raise ValueError(k)


def serving_stream(n_requests: int = 256, rate: float = 20.0, seed: int = SERVING_SEED,
                   t_end: float = 1e-5, nx_choices=None) -> List[Dict]:
    """Request stream: Poisson arrivals, plate sizes 100x40 .. 800x320, notch length
    and position in [0.2, 0.6] of the plate's width/height, traction 0.5..2 MPa,
    step ratio in {4, 8, 10}.  Draw order per request: inter-arrival, nx, notch
    length, notch height, traction, m, perturbation seed."""
    rng = SplitMix64(seed)
    if nx_choices is None:
        nx_choices = list(range(100, 801, 20))
    t = 0.0
    out = []
    for r in range(n_requests):
        t += -math.log(1.0 - rng.uniform()) / rate
        nx = nx_choices[min(int(rng.uniform() * len(nx_choices)), len(nx_choices) - 1)]
        a = (0.2 + 0.4 * rng.uniform()) * 0.1
        yc = (0.2 + 0.4 * rng.uniform()) * 0.04
        T = (0.5 + 1.5 * rng.uniform()) * 1e6
        m = (4, 8, 10)[min(int(rng.uniform() * 3), 2)]
        pseed = rng.next_u64()
        out.append(dict(arrival=t, nx=nx, notch=a, crack_y=yc, traction=T, m=m, seed=pseed,
                        t_end=t_end))
    return out


def serving_instance(req: Dict, precision: str = "mixed") -> Dict:
    """The plate solve of one serving request.

    Notch length and height are snapped to the FE node lines (spacing 4 dx) and
    clamped so that the PD strip [a - 10 mm, a + 40 mm] x [y_c - 10 mm, y_c + 10 mm]
    stays at least one element inside the plate.  The PD step follows the
    400 x 160 workload (6e-9 s at dx = 0.125 mm, m = 10) scaled with dx and 1/m,
    which keeps the same fraction of the PD and FE stability bounds; the request
    runs ceil(t_end / (m dt)) macro steps.  Returns the instance with
    "n_macro" and "bond_updates_per_macro" left to the caller (the latter needs
    the bond count)."""
    nx, m = int(req["nx"]), int(req["m"])
    dx = 0.05 / nx
    fe_h = 4.0 * dx
    a = round(req["notch"] / fe_h) * fe_h
    a = min(max(a, 0.01 + fe_h), 0.06 - fe_h)
    yc = round(req["crack_y"] / fe_h) * fe_h
    yc = min(max(yc, 0.01 + fe_h), 0.03 - fe_h)
    dt = 6.0e-9 * (dx / 0.125e-3) * (10.0 / m)
    n_macro = int(math.ceil(req["t_end"] / (m * dt) - 1e-9))
    inst = plate2d(nx, m, n_macro * m, dt, perturb=1e-6, seed=int(req["seed"]) & 0x7FFFFFFFFFFFFFFF,
                   precision=precision, traction=float(req["traction"]), notch=a, crack_y=yc,
                   name=f"serve {nx}x{2 * nx // 5} m={m}")
    inst["n_macro"] = n_macro
    return inst
