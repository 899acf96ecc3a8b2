"""A seeded sweep of small configurations, GPU against the FP64 oracle.

Each case draws a lattice (D2Q9 or D3Q19), sizes around the wavefront and
row-segment widths, which axes are periodic, possibly moving walls, a
penalization strength, the sub-step count K, gravity, and one to four
bodies placed without overlap; both sides start from the same random state
and run 15 steps.  Every case must meet the 1e-12 bar of the other parity
tests (positions, velocities, populations, fields, indicator).  The draws
are fixed by the seed, so a failure names its case.

The first draws run again in FP32, FP16 and BF16 storage, whose 2D two-byte
kernels take their own code path: there the bound is the storage's rounding
(velocities on the nodes both sides give the same owner, relative to the
largest velocity; body centres in lattice units), far below the O(1) error of
a wrong index or a missed tail.

The first 24 draws also run through the hand-written adjoint (K = 1, from a
uniform flow along the first periodic axis), against the complex-step oracle.

The first 24 draws run again with the fractional indicator (an extension;
ellipses become disks of their major semi-axis): the forward step within the
same 1e-12 bar, and the first 12 through the adjoint with the gradient in the
initial centres, against the complex-step oracle.
"""
import numpy as np
import pytest

from gpu_common import banner, pair
from paper_2511_01629_amd.workloads import place, random_state
from test_gpu_adjoint import _check, gpu_gradient, oracle_gradient
from test_gpu_adjoint_positions import gpu_gradient as gpu_gradient_x
from test_gpu_adjoint_positions import oracle_gradient as oracle_gradient_x
from test_gpu_fractional import _compare as _compare_fractional
from test_gpu_parity import _compare_run

pytestmark = pytest.mark.gpu

SEEDS = list(range(48))
STEPS = 15


def draw(seed):
    rng = np.random.default_rng(1000 + seed)
    lattice = "D2Q9" if seed % 3 != 2 else "D3Q19"
    d = 2 if lattice == "D2Q9" else 3
    sizes = [9, 17, 31, 40, 63, 64, 65, 70] if d == 2 else [9, 12, 16, 19, 24]
    n = [int(rng.choice(sizes)) for _ in range(d)] + ([1] if d == 2 else [])
    periodic = [int(rng.random() < 0.5) for _ in range(d)] + ([0] if d == 2 else [])
    cfg = dict(lattice=lattice, n=tuple(n), periodic=tuple(periodic), tau=float(rng.uniform(0.55, 1.2)),
               eps_p=2.0, eps_w=1.0, delta=1.0, K=int(rng.choice([1, 1, 1, 2])))
    if rng.random() < 0.3:
        cfg["alpha"] = float(rng.uniform(0.4, 0.99)) / cfg["tau"]
    # moving walls where allowed: one axis (y, or z in 3D), every other axis periodic
    axis = int(rng.integers(1, d))
    if rng.random() < 0.35 and n[axis] >= 9:
        per = [1] * 3
        per[axis] = 0
        per[2] = per[2] if d == 3 else 0
        cfg["periodic"] = tuple(per)
        w = np.zeros((3, 2, 3))
        for s in range(2):
            for j in range(d):
                if j != axis:
                    w[axis, s, j] = float(rng.uniform(-0.03, 0.03))
        cfg["wall_velocity"] = w.tolist()
    g = np.zeros(3)
    g[int(rng.integers(0, d))] = float(rng.choice([-1, 1])) * float(rng.uniform(1e-4, 6e-4))
    cfg["g"] = tuple(g)
    # bodies: radii that fit the smallest axis, placed without overlap
    nb = int(rng.integers(1, 5))
    rmax = max(2.0, min(n[:d]) / 2.0 - 2.5)
    kinds = []
    for _ in range(nb):
        r = float(rng.uniform(2.0, min(5.0, rmax)))
        if d == 2 and rng.random() < 0.3 and r >= 3.0:
            kinds.append(("ellipse", r, max(1.5, r * float(rng.uniform(0.5, 0.9)))))
        else:
            kinds.append(("sphere" if d == 3 else "disk", r, r))
    try:
        parts = place(tuple(n[:d]), kinds, 2000 + seed, (1.1, 1.8), upper_axis=d - 1, gap=1.0, margin=2.0,
                      max_tries=20000)
    except RuntimeError:  # four bodies do not fit: keep the first
        parts = place(tuple(n[:d]), kinds[:1], 2000 + seed, (1.1, 1.8), upper_axis=d - 1, gap=1.0, margin=2.0,
                      max_tries=20000)
    for p in parts:  # some bodies neutrally buoyant
        if rng.random() < 0.2:
            p["rho_s"] = 1.0
    return cfg, parts


def start(seed, storage="f64"):
    cfg, parts = draw(seed)
    banner(f"random config {seed} {storage}: {cfg['lattice']} n={cfg['n']} periodic={cfg['periodic']} "
           f"tau={cfg['tau']:.3f} K={cfg['K']} alpha={cfg.get('alpha', 'default')} "
           f"walls={'moving' if 'wall_velocity' in cfg else 'fixed'} bodies={len(parts)}")
    n = cfg["n"]
    Q = 9 if cfg["lattice"] == "D2Q9" else 19
    f0 = random_state((n[2], n[1], n[0]), Q, 1e-3, seed=3000 + seed)
    return cfg, parts, f0


@pytest.mark.parametrize("seed", SEEDS)
def test_random_config(seed):
    cfg, parts, f0 = start(seed)
    _compare_run(cfg, parts, STEPS, f0=f0)


# storage: (velocity max-norm / max|u| on nodes of equal owner, max centre
# error in l.u., owner flips), about twice the largest values measured on
# MI355X over these draws: f32 5.3e-7 / 1.8e-9, f16 7.3e-4 / 3.3e-6, bf16
# 4.9e-3 / 2.9e-5, no flips
STORAGE_BOUNDS = {"f32": (1.1e-6, 4e-9, 2), "f16": (1.5e-3, 7e-6, 2), "bf16": (1e-2, 6e-5, 2)}


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("seed", SEEDS[:16])
def test_random_config_storage(seed, storage):
    cfg, parts, f0 = start(seed, storage)
    sim, ora = pair(cfg, parts, storage=storage, f0=f0)
    rg = sim.step_record(STEPS)
    ro = ora.step(STEPS, record=True)
    ug, _, og = sim.fields()
    uo, _, oo = ora.fields()
    sim.close()
    same = og == oo
    flips = int((~same).sum())
    eu = float(np.abs(ug - uo)[same].max() / np.abs(uo).max())
    ex = float(np.abs(rg[:, :, 0:3] - ro[:, :, 0:3]).max())
    print(f"[measured] seed={seed} storage={storage} u_rel={eu:.3e} X_abs={ex:.3e} flips={flips}", flush=True)
    bu, bx, bf = STORAGE_BOUNDS[storage]
    assert eu < bu and ex < bx and flips <= bf


@pytest.mark.parametrize("seed", SEEDS[:24])
def test_random_config_adjoint(seed):
    """The gradient of a seeded weighting of the final centres with respect to
    every rho_s, tau and |g|, checkpoints every 1, 4 or 15 steps: within 1e-8
    of the complex-step oracle (FP64 storage, as the other adjoint tests)."""
    cfg, parts = draw(seed)
    cfg["K"] = 1
    per = cfg["periodic"]
    if any(per):
        u0 = [0.0] * 3
        u0[per.index(1)] = 0.01
        cfg["u0"] = tuple(u0)
    d = 2 if cfg["lattice"] == "D2Q9" else 3
    rng = np.random.default_rng(4000 + seed)
    w = rng.normal(size=(len(parts), 3))
    w[:, d:] = 0.0
    every = int(rng.choice([1, 4, STEPS]))
    banner(f"random config {seed} adjoint every={every}: {cfg['lattice']} n={cfg['n']} periodic={per} "
           f"alpha={cfg.get('alpha', 'default')} walls={'moving' if 'wall_velocity' in cfg else 'fixed'} "
           f"bodies={len(parts)}")
    go = oracle_gradient(cfg, parts, STEPS, w)
    ga = gpu_gradient(cfg, parts, STEPS, every, w)
    _check(ga, go, 1e-8)


@pytest.mark.parametrize("seed", SEEDS[:12])
def test_random_config_adjoint_two_byte(seed):
    """The first adjoint draws in FP16 storage (FP32 lattice arithmetic, FP64
    particle adjoint), whose checkpoint frames of Q N 2 bytes are odd-sized on
    most of these lattices: the gradient within a relative bound of the
    complex-step oracle (1e-3: twice the largest error measured on MI355X
    over these draws, 5.0e-4; FP16 rounding of the random starting state)."""
    cfg, parts = draw(seed)
    cfg["K"] = 1
    per = cfg["periodic"]
    if any(per):
        u0 = [0.0] * 3
        u0[per.index(1)] = 0.01
        cfg["u0"] = tuple(u0)
    d = 2 if cfg["lattice"] == "D2Q9" else 3
    rng = np.random.default_rng(4000 + seed)
    w = rng.normal(size=(len(parts), 3))
    w[:, d:] = 0.0
    every = int(rng.choice([1, 4, STEPS]))
    banner(f"random config {seed} adjoint f16 every={every}: {cfg['lattice']} n={cfg['n']} periodic={per} "
           f"bodies={len(parts)}")
    go = oracle_gradient(cfg, parts, STEPS, w)
    ga = gpu_gradient(cfg, parts, STEPS, every, w, storage="f16")
    _check(ga, go, 1e-3)


def fractional(cfg, parts):
    """The draw with the fractional indicator: disks and spheres only."""
    return dict(cfg, fractional=1), [dict(p, shape=("sphere" if p["shape"] == "sphere" else "disk"), b=p["a"])
                                     for p in parts]


@pytest.mark.parametrize("seed", SEEDS[:24])
def test_random_config_fractional(seed):
    cfg, parts, f0 = start(seed)
    cfg, parts = fractional(cfg, parts)
    _compare_fractional(cfg, parts, STEPS, f0=f0)


@pytest.mark.parametrize("seed", SEEDS[:12])
def test_random_config_fractional_gradient(seed):
    """The gradient with respect to every rho_s, tau, |g| and every initial
    centre coordinate with the fractional indicator: within 1e-10 of the
    complex-step oracle (FP64 storage; measured on MI355X: at most 5.1e-14)."""
    cfg, parts = fractional(*draw(seed))
    cfg["K"] = 1
    per = cfg["periodic"]
    if any(per):
        u0 = [0.0] * 3
        u0[per.index(1)] = 0.01
        cfg["u0"] = tuple(u0)
    d = 2 if cfg["lattice"] == "D2Q9" else 3
    rng = np.random.default_rng(5000 + seed)
    w = rng.normal(size=(len(parts), 3))
    w[:, d:] = 0.0
    every = int(rng.choice([1, 4, STEPS]))
    banner(f"random config {seed} fractional gradient every={every}: {cfg['lattice']} n={cfg['n']} "
           f"periodic={per} walls={'moving' if 'wall_velocity' in cfg else 'fixed'} bodies={len(parts)}")
    go = oracle_gradient_x(cfg, parts, STEPS, w, d)
    ga = gpu_gradient_x(cfg, parts, STEPS, every, w, d)
    _check(ga, go, 1e-10)
