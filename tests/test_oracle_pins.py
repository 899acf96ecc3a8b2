"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage of Millet & Liberge (arXiv 2511.01629) it pins.
None of them re-types an oracle formula: they check moment identities, closed
forms, exact special cases, textbook flows, brute force on tiny lattices, and
the complex-step derivative against finite differences.
"""
import math

import numpy as np
import pytest

from oracle import brute
from oracle import oracle as O

CS2 = 1.0 / 3.0
RNG = np.random.default_rng(12345)
KINDS = ["D2Q9", "D3Q19"]


def _lat(kind):
    c, w, opp = O.lattice(kind)
    return c.astype(float), w, opp


# ------------------------------------------------------------ lattice tables

@pytest.mark.parametrize("kind", KINDS)
def test_lattice_isotropy(kind):
    """Weights by speed (velocity-set figure of sec. 2.2) give the isotropic
    moments the Chapman-Enskog expansion needs; the printed index rule would
    not (it gives an anisotropic second moment for D2Q9)."""
    c, w, opp = _lat(kind)
    d = 2 if kind == "D2Q9" else 3
    assert abs(w.sum() - 1) < 1e-15
    assert np.abs(w @ c).max() < 1e-15
    M2 = np.einsum("a,ai,aj->ij", w, c, c)
    assert np.allclose(M2[:d, :d], CS2 * np.eye(d), atol=1e-15)
    M4 = np.einsum("a,ai,aj,ak,al->ijkl", w, c, c, c, c)[:d, :d, :d, :d]
    I = np.eye(d)
    iso = CS2 ** 2 * (np.einsum("ij,kl->ijkl", I, I) + np.einsum("ik,jl->ijkl", I, I) + np.einsum("il,jk->ijkl", I, I))
    assert np.allclose(M4, iso, atol=1e-15)
    assert np.all(c[opp] == -c)
    if kind == "D2Q9":
        # numbering of the velocity-set figure: 1..4 axes counter-clockwise from +x, 5..8 diagonals
        assert c[1, :2].tolist() == [1, 0] and c[2, :2].tolist() == [0, 1]
        assert c[5, :2].tolist() == [1, 1] and c[8, :2].tolist() == [1, -1]
        # the printed rule (1/9 on 1,3,5,7) is anisotropic -- the reason for the reading
        wp = np.array([4 / 9, 1 / 9, 1 / 36, 1 / 9, 1 / 36, 1 / 9, 1 / 36, 1 / 9, 1 / 36])
        M2p = np.einsum("a,ai,aj->ij", wp, c, c)[:2, :2]
        assert abs(M2p[0, 1]) > 0.1


# ---------------------------------------------------------- equilibrium, eq. 12-13

@pytest.mark.parametrize("kind", KINDS)
def test_feq_moments(kind):
    """eq. (12): sum f^eq = 0, sum f^eq c = u, sum f^eq c c = u u + p I."""
    c, w, _ = _lat(kind)
    d = 2 if kind == "D2Q9" else 3
    for _ in range(20):
        p = RNG.normal(0, 0.01)
        u = np.zeros(3)
        u[:d] = RNG.normal(0, 0.05, d)
        fe = O.feq(kind, p, u)
        assert abs(fe.sum()) < 1e-15
        assert np.abs(fe @ c - u).max() < 1e-15
        Pi = np.einsum("a,ai,aj->ij", fe, c, c)[:d, :d]
        assert np.abs(Pi - (np.outer(u[:d], u[:d]) + p * np.eye(d))).max() < 1e-15


@pytest.mark.parametrize("kind", KINDS)
def test_feq_rest_state_is_zero(kind):
    """Velocity-based model: the rest state p = 0, u = 0 has f^eq = 0 (eq. 13),
    which is why populations are stored as deviations directly."""
    assert np.all(O.feq(kind, 0.0, [0, 0, 0]) == 0.0)


@pytest.mark.parametrize("kind", KINDS)
def test_macro_roundtrip(kind):
    """eq. (15a-b) inverts eq. (13): u(f^eq(p,u)) = u and p(f^eq(p,u)) = p (a = 0);
    with a force, u = sum f c + a/2."""
    d = 2 if kind == "D2Q9" else 3
    for _ in range(20):
        p = RNG.normal(0, 0.01)
        u = np.zeros(3)
        u[:d] = RNG.normal(0, 0.05, d)
        uu, pp = O.macro(kind, O.feq(kind, p, u))
        assert np.abs(uu - u).max() < 1e-15 and abs(pp - p) < 1e-15
        a = np.zeros(3)
        a[:d] = RNG.normal(0, 1e-3, d)
        ua, _ = O.macro(kind, O.feq(kind, p, u), a)
        assert np.abs(ua - u - a / 2).max() < 1e-16


# ---------------------------------------------------------- Guo force, eq. 14

@pytest.mark.parametrize("kind", KINDS)
def test_guo_moments(kind):
    """eq. (14): sum F = 0, sum F c = (1 - 1/2tau) a, sum F c c = (1 - 1/2tau)(u a + a u)."""
    c, _, _ = _lat(kind)
    d = 2 if kind == "D2Q9" else 3
    for tau in (0.55, 0.8, 1.3):
        u = np.zeros(3)
        a = np.zeros(3)
        u[:d] = RNG.normal(0, 0.05, d)
        a[:d] = RNG.normal(0, 1e-3, d)
        F = O.guo(kind, tau, u, a)
        k = 1 - 1 / (2 * tau)
        assert abs(F.sum()) < 1e-17
        assert np.abs(F @ c - k * a).max() < 1e-17
        M2 = np.einsum("a,ai,aj->ij", F, c, c)
        assert np.abs(M2 - k * (np.outer(u, a) + np.outer(a, u))).max() < 1e-17


# ---------------------------------------------------------- penalization, eq. 17

@pytest.mark.parametrize("kind", KINDS)
def test_penalization_moments(kind):
    """eq. (17): S carries no mass and no momentum, and its second moment is E = alpha Pi^neq."""
    c, _, _ = _lat(kind)
    d = 2 if kind == "D2Q9" else 3
    for _ in range(10):
        f = RNG.normal(0, 1e-2, len(c))
        p = RNG.normal(0, 1e-2)
        u = np.zeros(3)
        u[:d] = RNG.normal(0, 0.05, d)
        fe = O.feq(kind, p, u)
        alpha = RNG.uniform(0.2, 1.5)
        S = O.penal(kind, alpha, f, fe)
        Pi = np.einsum("a,ai,aj->ij", f - fe, c, c)
        assert abs(S.sum()) < 1e-16
        assert np.abs(S @ c).max() < 1e-16
        assert np.abs(np.einsum("a,ai,aj->ij", S, c, c) - alpha * Pi).max() < 1e-15


@pytest.mark.parametrize("kind", KINDS)
def test_collision_identities(kind):
    """Right side of eq. (10): with alpha = 1/tau (the value of every run, sec. 3) the
    non-equilibrium stress passes through the collision unrelaxed; the
    post-collision momentum is u + a/2; the node sum relaxes by (1 - 1/tau)."""
    c, _, _ = _lat(kind)
    d = 2 if kind == "D2Q9" else 3
    for tau in (0.55, 0.8):
        f = RNG.normal(0, 1e-2, len(c))
        a = np.zeros(3)
        a[:d] = RNG.normal(0, 1e-4, d)
        u, p = O.macro(kind, f, a)
        fe = O.feq(kind, p, u)
        ft = O.collide(kind, tau, 1 / tau, True, f, a)
        Pi = np.einsum("a,ai,aj->ij", f - fe, c, c)
        Pit = np.einsum("a,ai,aj->ij", ft - fe, c, c)
        k = 1 - 1 / (2 * tau)
        assert np.abs(Pit - Pi - k * (np.outer(u, a) + np.outer(a, u))).max() < 1e-16
        assert np.abs(ft @ c - (u + a / 2)).max() < 1e-16
        assert abs(ft.sum() - (1 - 1 / tau) * f.sum()) < 1e-16
        # fluid node: the stress relaxes at rate 1/tau
        ftf = O.collide(kind, tau, 1 / tau, False, f, [0, 0, 0])
        uf, pf = O.macro(kind, f)
        fef = O.feq(kind, pf, uf)
        Pif = np.einsum("a,ai,aj->ij", f - fef, c, c)
        assert np.abs(np.einsum("a,ai,aj->ij", ftf - fef, c, c) - (1 - 1 / tau) * Pif).max() < 1e-16


# ---------------------------------------------------------- indicator, eq. 9

def _brute_owner(kind, n, periodic, parts):
    st = brute.initial_state(kind, n, periodic, 0.8, 0.0, 1.0, (0, 0, 0), (0, 0, 0), parts)
    nxt = brute.step(st)
    own = np.full((n[2], n[1], n[0]), -1, dtype=np.int32)
    for (x, y, z), i in nxt["owner"].items():
        own[z, y, x] = i
    return own


def test_indicator_vs_whole_lattice_scan():
    """eq. (9) with the closed set, lowest id on shared nodes, minimum image: the
    oracle's bounding-box rasteriser agrees bit for bit with a scan of every node
    against every particle, including the exact ties of an integer centre."""
    n = (30, 26, 1)
    parts = [
        dict(shape="disk", rho_s=1.2, a=5.0, x=(3.0, 12.0)),          # wraps across x = 0; ties at (3,4)
        dict(shape="disk", rho_s=1.2, a=4.0, x=(9.5, 12.25)),         # overlaps particle 0
        dict(shape="ellipse", rho_s=1.3, a=6.0, b=3.0, x=(20.3, 6.7), theta=0.7),
        dict(shape="disk", rho_s=1.1, a=3.0, x=(20.0, 19.0)),
    ]
    o = O.Oracle(dict(lattice="D2Q9", n=n, periodic=(1, 0, 0), tau=0.8), parts)
    _, _, own = o.fields()
    ref = _brute_owner("D2Q9", n, (1, 0, 0), parts)
    assert np.array_equal(own, ref)
    assert (own == 0).sum() > 0 and (own == 1).sum() > 0
    # the 12 exact-distance nodes of the integer centre are inside (closed set)
    assert own[0, 12 + 4, 3 + 3] == 0 and own[0, 12 + 5, 3] == 0 and own[0, 12, (3 - 5) % 30] == 0


def test_indicator_3d():
    n = (12, 11, 13)
    parts = [dict(shape="sphere", rho_s=1.5, a=3.0, x=(5.0, 5.0, 6.0)),
             dict(shape="sphere", rho_s=1.5, a=2.5, x=(8.4, 6.1, 7.7))]
    o = O.Oracle(dict(lattice="D3Q19", n=n, periodic=(0, 1, 0), tau=0.8), parts)
    _, _, own = o.fields()
    assert np.array_equal(own, _brute_owner("D3Q19", n, (0, 1, 0), parts))
    # a sphere of radius 3 at an integer centre holds 123 nodes
    assert (own == 0).sum() == 123


# ---------------------------------------------------------- reductions, eq. 22

def test_reduction_rigid_field_2d():
    """eq. (22a-b) on a rigid field u = U0 + omega0 z x r over a symmetric disk:
    the discrete sums return U0 and omega0 exactly (sum r = 0)."""
    n = (40, 36, 1)
    X = np.array([20.0, 17.0])
    U0 = np.array([0.013, -0.007])
    w0 = 2.3e-3
    o = O.Oracle(dict(lattice="D2Q9", n=n, tau=0.8), [dict(shape="disk", rho_s=1.0, a=7.0, x=tuple(X))])
    f = np.zeros((1, n[1], n[0], 9))
    for y in range(n[1]):
        for x in range(n[0]):
            r = np.array([x, y]) - X
            u = U0 + w0 * np.array([-r[1], r[0]])
            f[0, y, x] = O.feq("D2Q9", 0.0, u)
    o.set_f(f)
    P = o.particles()
    assert P["N"][0] == 149
    assert np.abs(P["U"][0, :2] - U0).max() < 1e-16
    assert abs(P["omega"][0, 2] - w0) < 1e-16


def test_reduction_rigid_field_3d():
    n = (16, 15, 14)
    X = np.array([8.0, 7.0, 6.0])
    U0 = np.array([0.01, -0.02, 0.005])
    W0 = np.array([1e-3, -2e-3, 3e-3])
    o = O.Oracle(dict(lattice="D3Q19", n=n, tau=0.8), [dict(shape="sphere", rho_s=1.0, a=4.0, x=tuple(X))])
    f = np.zeros((n[2], n[1], n[0], 19))
    for z in range(n[2]):
        for y in range(n[1]):
            for x in range(n[0]):
                r = np.array([x, y, z]) - X
                f[z, y, x] = O.feq("D3Q19", 0.0, U0 + np.cross(W0, r))
    o.set_f(f)
    P = o.particles()
    assert np.abs(P["U"][0] - U0).max() < 1e-16
    assert np.abs(P["omega"][0] - W0).max() < 1e-15


# ---------------------------------------------------------- Algorithm 1, sec. 2.3-2.4

def test_algorithm1_free_flight():
    """Algorithm 1 with no contact and K = 1: X^{n+1} = X^n + (U^n + U^{n-1})/2 and
    A^{n+1} = 0 exactly (A is taken from the correction displacements, not from
    a difference of absolute positions)."""
    cfg = dict(lattice="D2Q9", n=(60, 50), periodic=(1, 1, 0), tau=0.8, u0=(0.02, -0.01))
    o = O.Oracle(cfg, [dict(shape="disk", rho_s=1.0, a=6.0, x=(30.25, 24.5))])
    rec = o.step(3, record=True)
    X, U, A = rec[:, 0, 0:3], rec[:, 0, 4:7], rec[:, 0, 10:13]
    # uniform flow is an exact fixed point: U^n = u0, and with no contact A = 0 exactly
    assert np.abs(U[:, :2] - [0.02, -0.01]).max() < 1e-16
    assert np.all(X[1, :2] == X[0, :2] + U[0, :2])
    assert np.all(A == 0.0)


def _pair(d_centres, rho=(1.5, 1.5), a=(5.0, 5.0), form=0):
    cfg = dict(lattice="D2Q9", n=(80, 60), periodic=(1, 1, 0), tau=0.8, g=(0, -1e-4), eps_p=2.0, delta=1.0,
               collision_form=form)
    parts = [dict(shape="disk", rho_s=rho[0], a=a[0], x=(40.0, 30.0)),
             dict(shape="disk", rho_s=rho[1], a=a[1], x=(40.0 + d_centres[0], 30.0 + d_centres[1]))]
    return O.Oracle(cfg, parts).collision_forces()


def test_collision_force_pair():
    """Particle-particle force of sec. 2.3 (eq. 19): zero beyond R_i + R_j + delta,
    equal and opposite for equal particles, along the centre line, with the
    quadratic profile; continuous with a continuous slope at the cut-off."""
    F = _pair((7.0, 6.0))
    assert np.abs(F[0] + F[1]).max() < 1e-18
    dvec = np.array([-7.0, -6.0])
    assert abs(F[0, 0] * dvec[1] - F[0, 1] * dvec[0]) < 1e-18
    d = math.hypot(7, 6)
    C = (1.5 - 1.0) * 1e-4 * math.pi * 25
    mag = C / 2.0 * ((10 + 1 - d) / 1.0) ** 2
    assert abs(np.linalg.norm(F[0]) - mag) < 1e-15
    assert np.all(_pair((11.0001, 0.0)) == 0)
    # C1 at the cut-off: force and its slope vanish like (11 - d)^2
    e = 1e-4
    f1 = np.linalg.norm(_pair((11.0 - e, 0.0))[0])
    f2 = np.linalg.norm(_pair((11.0 - 2 * e, 0.0))[0])
    assert f1 < 1e-10 and abs(f2 / f1 - 4.0) < 1e-6
    # the printed form uses the raw centre difference and C = (rho_s - rho_f)|g|
    Fl = _pair((7.0, 6.0), form=1)
    assert abs(np.linalg.norm(Fl[0]) - 0.5e-4 / 2.0 * (11 - d) ** 2 * d) < 1e-18


def test_collision_force_wall():
    """Particle-wall force of sec. 2.3 (eq. 20) through the mirror particle across
    a wall at -0.5: active when 2(Y + 0.5) <= 2R + delta, pointing into the box."""
    cfg = dict(lattice="D2Q9", n=(40, 60), periodic=(1, 0, 0), tau=0.8, g=(0, -1e-4), eps_w=1.0, delta=1.0)
    o = O.Oracle(cfg, [dict(shape="disk", rho_s=2.0, a=5.0, x=(20.0, 4.8))])
    F = o.collision_forces()[0]
    dprime = 2 * (4.8 + 0.5)
    C = 1.0 * 1e-4 * math.pi * 25
    assert F[0] == 0 and abs(F[1] - C * ((10 + 1 - dprime) / 1.0) ** 2) < 1e-15
    o2 = O.Oracle(cfg, [dict(shape="disk", rho_s=2.0, a=5.0, x=(20.0, 5.1))])
    assert np.all(o2.collision_forces() == 0)


# ---------------------------------------------------------- whole step vs brute force

def _compare_with_brute(kind, n, periodic, parts, g, steps, seed, K=1, beta=0.0, no_stress_penalty=False,
                        fractional=False):
    cfg = dict(lattice=kind, n=n, periodic=periodic, tau=0.7, g=g, eps_p=2.0, eps_w=1.0, delta=1.0, K=K,
               rigid_beta=beta, no_stress_penalty=int(no_stress_penalty), fractional=int(fractional))
    o = O.Oracle(cfg, parts)
    Q = 9 if kind == "D2Q9" else 19
    shp = (n[2] if kind == "D3Q19" else 1, n[1], n[0])
    f0 = RNG.normal(0, 2e-3, shp + (Q,))
    o.set_f(f0)
    o.reset_particles(parts)
    st = brute.initial_state(kind, n if len(n) == 3 else tuple(n) + (1,), periodic, 0.7, 0.0, 1.0, g, (0, 0, 0),
                             parts, K=K, beta=beta, no_stress_penalty=no_stress_penalty, fractional=fractional)
    for nd in st["f"]:
        x, y, z = nd
        st["f"][nd] = list(f0[z, y, x])
    # U^{-1} = U^0 measured on the random initial field
    probe = brute.step(dict(st, eps_p=1e300, eps_w=1e300))
    for q, qn in zip(st["parts"], probe["parts"]):
        q["Uprev"], q["Wprev"] = list(qn["Uprev"]), list(qn["Wprev"])
    for _ in range(steps):
        st = brute.step(st)
    o.step(steps)
    fo = o.f()
    fb = np.zeros_like(fo)
    for (x, y, z), v in st["f"].items():
        fb[z, y, x] = v
    assert np.abs(fo - fb).max() < 1e-15 * max(1.0, np.abs(fb).max()) * 50
    P = o.particles()
    for i, q in enumerate(st["parts"]):
        assert np.abs(P["X"][i] - np.array(q["X"])).max() < 1e-12
        assert np.abs(P["A"][i] - np.array(q["A"])).max() < 1e-13
        assert np.abs(P["U_prev"][i] - np.array(q["Uprev"])).max() < 1e-15
        assert np.abs(P["omega_prev"][i] - np.array(q["Wprev"])).max() < 1e-14
        assert abs(P["theta"][i] - q["theta"]) < 1e-14
    return st


def test_oracle_vs_brute_d2q9():
    """The whole step (S1-S7) against the independent pure-Python transcription
    on a 9x8 lattice, x periodic, y walls, two bodies in repulsive contact."""
    parts = [dict(shape="disk", rho_s=1.6, a=2.2, x=(3.1, 3.2)),
             dict(shape="ellipse", rho_s=1.3, a=2.5, b=1.2, x=(7.6, 4.4), theta=0.4)]
    st = _compare_with_brute("D2Q9", (9, 8, 1), (1, 0, 0), parts, (0.0, -1e-3, 0.0), 3, 1)
    assert any(abs(a) > 1e-8 for q in st["parts"] for a in q["A"])  # contact forces active


def test_oracle_vs_brute_d3q19():
    parts = [dict(shape="sphere", rho_s=1.6, a=1.6, x=(2.0, 2.1, 2.3)),
             dict(shape="sphere", rho_s=1.4, a=1.4, x=(3.4, 3.0, 3.9))]
    _compare_with_brute("D3Q19", (5, 5, 6), (0, 1, 0), parts, (0.0, 0.0, -1e-3), 2, 2)


@pytest.mark.parametrize("K", [2, 3])
def test_oracle_vs_brute_substeps_d2q9(K):
    """Algorithm 1 with K sub-steps (sec. 2.4): the prediction by U_bar/K, the
    correction with (1/K)^2 and the forces at Y^{k-1} and Y*, over three whole
    steps against the brute-force transcription, bodies in contact."""
    parts = [dict(shape="disk", rho_s=1.6, a=2.2, x=(3.1, 3.2)),
             dict(shape="ellipse", rho_s=1.3, a=2.5, b=1.2, x=(7.6, 4.4), theta=0.4)]
    st = _compare_with_brute("D2Q9", (9, 8, 1), (1, 0, 0), parts, (0.0, -1e-3, 0.0), 3, 1, K=K)
    assert any(abs(a) > 1e-8 for q in st["parts"] for a in q["A"])


@pytest.mark.parametrize("K", [2, 3])
def test_oracle_vs_brute_substeps_d3q19(K):
    parts = [dict(shape="sphere", rho_s=1.6, a=1.6, x=(2.0, 2.1, 2.3)),
             dict(shape="sphere", rho_s=1.4, a=1.4, x=(3.4, 3.0, 3.9))]
    st = _compare_with_brute("D3Q19", (5, 5, 6), (0, 1, 0), parts, (0.0, 0.0, -1e-3), 2, 2, K=K)
    assert any(abs(a) > 1e-8 for q in st["parts"] for a in q["A"])


@pytest.mark.parametrize("K", [1, 3])
def test_algorithm1_literal_collision_acceleration(K):
    """Algorithm 1 defines A^{n+1} = 2(X^{n+1} - X^n - U_bar) with
    U_bar = (U^n + U^{n-1})/2.  The oracle takes the bracket as the summed
    correction displacements; here the literal difference of the recorded
    positions must give the same A to round-off of the positions, in a run
    where the contact forces are strong."""
    kinds = [("disk", 5.0, 5.0)] * 5 + [("ellipse", 6.0, 3.0)] * 3
    from paper_2511_01629_amd.workloads import place

    parts = place((64, 96), kinds, seed=7, rho_range=(1.2, 1.8), upper_axis=1, gap=0.3, margin=0.3)
    cfg = dict(lattice="D2Q9", n=(64, 96, 1), periodic=(0, 0, 0), tau=0.6, g=(0.0, -2e-4, 0.0), K=K)
    o = O.Oracle(cfg, parts)
    U_init = o.particles()["U"].copy()  # U^{-1} = U^0
    rec = o.step(60, record=True)  # per step n: X^n theta U^n omega A^n N
    X, U, A = rec[:, :, 0:3], rec[:, :, 4:7], rec[:, :, 10:13]
    Uprev = np.concatenate([U_init[None], U[:-1]])
    Ubar = 0.5 * (U + Uprev)
    A_lit = 2.0 * (X[1:] - X[:-1] - Ubar[:-1])
    ulp = np.spacing(np.abs(X).max())
    assert np.abs(A[1:] - A_lit).max() <= 8 * K * ulp
    assert np.abs(A[1:]).max() > 1e4 * ulp  # contacts act: the pin is not trivially 0 = 0
    assert np.all(A[0] == 0.0)


def test_algorithm1_free_flight_substeps():
    """With no contact, K = 3 sub-steps move by U_bar/3 three times:
    X^{n+1} = X^n + U_bar to round-off, and A^{n+1} = 0 exactly (every
    correction is zero)."""
    cfg = dict(lattice="D2Q9", n=(60, 50), periodic=(1, 1, 0), tau=0.8, u0=(0.02, -0.01), K=3)
    o = O.Oracle(cfg, [dict(shape="disk", rho_s=1.0, a=6.0, x=(30.25, 24.5))])
    rec = o.step(4, record=True)
    X, U, A = rec[:, 0, 0:3], rec[:, 0, 4:7], rec[:, 0, 10:13]
    assert np.abs(U[:, :2] - [0.02, -0.01]).max() < 1e-16
    assert np.abs(X[1:, :2] - X[:-1, :2] - U[:-1, :2]).max() <= 4 * np.spacing(30.0)
    assert np.all(A == 0.0)


@pytest.mark.parametrize("gravity_form,expect", [(0, 1.0 - 1.0 / 1.5), (1, 1.5 - 1.0)])
def test_gravity_form_momentum(gravity_form, expect):
    """The solid-node acceleration of sec. 2.1 (eq. 5-8): a = (1 - rho_f/rho_s) g
    (the default reading) or (rho_s/rho_f - 1) g (gravity_form = 1).  The
    collision with the Guo force leaves the momentum sum f~ c = sum f c + a at
    every node (eq. 14-15; the penalization carries none), so from rest (f = 0)
    in a fully periodic box, where streaming is a permutation, the lattice
    momentum after one step is N_i b g with b the form's factor."""
    g = (0.0, -3e-4, 0.0)
    cfg = dict(lattice="D2Q9", n=(40, 36), periodic=(1, 1, 0), tau=0.7, g=g, gravity_form=gravity_form)
    o = O.Oracle(cfg, [dict(shape="disk", rho_s=1.5, a=6.0, x=(20.0, 18.0))])
    N = int(o.particles()["N"][0])
    o.step(1)
    c, _, _ = _lat("D2Q9")
    P = np.einsum("zyxa,ak->k", o.f(), c)
    assert N > 100
    assert abs(P[1] - N * expect * g[1]) <= 1e-12 * abs(N * expect * g[1])
    assert abs(P[0]) < 1e-17


# ------------------------------------- rigid-velocity forcing (an extension)

@pytest.mark.parametrize("kind,beta,nopen", [("D2Q9", 0.6, False), ("D2Q9", 1.0, True), ("D3Q19", 0.5, False)])
def test_rigid_forcing_vs_brute(kind, beta, nopen):
    """The optional forcing toward the rigid motion U_i + omega_i x r (with and
    without the stress penalization) over whole steps, bodies in contact,
    against the independent brute-force transcription."""
    if kind == "D2Q9":
        parts = [dict(shape="disk", rho_s=1.6, a=2.2, x=(3.1, 3.2)),
                 dict(shape="ellipse", rho_s=1.3, a=2.5, b=1.2, x=(7.6, 4.4), theta=0.4)]
        _compare_with_brute("D2Q9", (9, 8, 1), (1, 0, 0), parts, (0.0, -1e-3, 0.0), 3, 1, beta=beta,
                            no_stress_penalty=nopen)
    else:
        parts = [dict(shape="sphere", rho_s=1.6, a=1.6, x=(2.0, 2.1, 2.3)),
                 dict(shape="sphere", rho_s=1.4, a=1.4, x=(3.4, 3.0, 3.9))]
        _compare_with_brute("D3Q19", (5, 5, 6), (0, 1, 0), parts, (0.0, 0.0, -1e-3), 2, 2, beta=beta)


def test_rigid_forcing_fixed_point():
    """A body whose nodes already move rigidly (u = U0 + omega0 x r on a disk
    centred on a node, so that the momentum sums return U0 and omega0
    exactly) is a fixed point of the forcing: with beta = 1 the step equals
    the unforced one to round-off."""
    n = (40, 36, 1)
    X = np.array([20.0, 17.0])
    U0 = np.array([0.013, -0.007])
    w0 = 2.3e-3
    f = np.zeros((1, n[1], n[0], 9))
    for y in range(n[1]):
        for x in range(n[0]):
            r = np.array([x, y]) - X
            f[0, y, x] = O.feq("D2Q9", 0.0, U0 + w0 * np.array([-r[1], r[0]]))
    out = []
    for beta in (0.0, 1.0):
        o = O.Oracle(dict(lattice="D2Q9", n=n, periodic=(1, 1, 0), tau=0.8, rigid_beta=beta),
                     [dict(shape="disk", rho_s=1.0, a=7.0, x=tuple(X))])
        o.set_f(f)
        o.reset_particles([dict(shape="disk", rho_s=1.0, a=7.0, x=tuple(X))])
        o.step(1)
        out.append(o.f())
    assert np.abs(out[1] - out[0]).max() < 1e-17 * 1e2


@pytest.mark.parametrize("X,beta", [((20.0, 17.0), 0.7), ((20.3, 16.6), 0.7), ((20.3, 16.6), 0.25)])
def test_rigid_forcing_momentum_and_torque(X, beta):
    """What the forcing adds to the lattice over one step, against the
    unforced step from the same state (periodic box, a random field confined
    near the body, so streaming keeps the total momentum and the angular
    momentum about X exactly): the added momentum is the sum of
    2 beta (U + omega x r - u) over the body, which the sums of eq. (22)
    reduce to 2 beta omega z x sum r, and the added angular momentum is
    2 beta (sum r) x U; both vanish for a body centred on a node.  U and
    omega are this step's sums (not the previous step's, which the state
    holds as U_prev and differ here)."""
    n = (48, 40, 1)
    X = np.array(X)
    rng = np.random.default_rng(3)
    f = np.zeros((1, n[1], n[0], 9))
    yy, xx = np.mgrid[0:n[1], 0:n[0]]
    near = (xx - X[0]) ** 2 + (yy - X[1]) ** 2 <= 10.0 ** 2
    f[0][near] = rng.normal(0, 2e-3, (near.sum(), 9))
    body = [dict(shape="disk", rho_s=1.4, a=7.0, x=tuple(X))]
    res = []
    for b in (0.0, beta):
        cfg = dict(lattice="D2Q9", n=n, periodic=(1, 1, 0), tau=0.8, g=(0.0, -1e-4, 0.0), rigid_beta=b)
        o = O.Oracle(cfg, body)
        o.set_f(f)
        o.reset_particles(body)
        P = o.particles()
        raw = P["raw"].copy()
        raw[:, 10:13] = [[0.004, -0.002, 0.0]]  # U^{n-1} unlike U^n
        o.load_particles(raw, 0)
        P = o.particles()
        _, _, own = o.fields()
        o.step(1)
        fn = o.f()[0]
        c, _, _ = _lat("D2Q9")
        j = np.einsum("yxa,ak->yxk", fn, c)[..., :2]
        M = j.reshape(-1, 2).sum(axis=0)
        L = ((xx - X[0]) * j[..., 1] - (yy - X[1]) * j[..., 0]).sum()
        res.append((M, L, P, own[0]))
    (M0, L0, P, own), (M1, L1, _, _) = res
    sel = own == 0
    rs = np.stack([xx[sel] - X[0], yy[sel] - X[1]], axis=1).sum(axis=0)
    U, w = P["U"][0, :2], P["omega"][0, 2]
    dM_expect = 2 * beta * w * np.array([-rs[1], rs[0]])
    dL_expect = 2 * beta * (rs[0] * U[1] - rs[1] * U[0])
    scale = 2 * beta * sel.sum() * np.abs(U).max()
    assert np.abs((M1 - M0) - dM_expect).max() <= 1e-12 * scale
    assert abs((L1 - L0) - dL_expect) <= 1e-12 * scale * 7.0
    if X[0] == int(X[0]) and X[1] == int(X[1]):
        assert np.abs(rs).max() == 0.0
    else:
        assert np.abs(dM_expect).max() > 1e-6 * scale  # the centroid offset makes the pin non-trivial


# ---------------------------------------------------------- conservation and textbook flows

def test_mass_round_off():
    """Collision relaxes the node sum by (1 - 1/tau) (eq. 10, 12, 14, 17 carry no
    mass), streaming with bounce-back permutes: from equilibrium at p = 0 the
    total sum stays at round-off."""
    cfg = dict(lattice="D2Q9", n=(48, 64), tau=0.6, g=(0, -1e-4))
    parts = [dict(shape="disk", rho_s=1.5, a=6.0, x=(20.3, 40.2)),
             dict(shape="ellipse", rho_s=1.2, a=7.0, b=3.5, x=(31.0, 20.0), theta=1.0)]
    o = O.Oracle(cfg, parts)
    f0 = o.f()
    o.step(200)
    f = o.f()
    assert abs(f.sum()) < 1e-13
    assert np.abs(f - f0).max() > 1e-6  # the flow did develop
    # a random start: the sum decays exactly by (1 - 1/tau) per step
    o2 = O.Oracle(dict(cfg, n=(20, 16)), [])
    fr = RNG.normal(0, 1e-2, (1, 16, 20, 9))
    o2.set_f(fr)
    o2.step(1)
    assert abs(o2.f().sum() - (1 - 1 / 0.6) * fr.sum()) < 1e-14


def _shear_wave(tau, alpha=0.0, penalize_all=0, L=64, t1=100, t2=600):
    cfg = dict(lattice="D2Q9", n=(4, L), periodic=(1, 1, 0), tau=tau, alpha=alpha, penalize_all=penalize_all)
    o = O.Oracle(cfg, [])
    U0 = 1e-3
    f = np.zeros((1, L, 4, 9))
    for y in range(L):
        f[0, y, :] = O.feq("D2Q9", 0.0, [U0 * math.sin(2 * math.pi * y / L), 0.0])
    o.set_f(f)
    s = np.sin(2 * math.pi * np.arange(L) / L)

    def amp():
        u, _, _ = o.fields()
        return 2.0 / L * (u[0, :, 0, 0] * s).sum()

    o.step(t1)
    a1 = amp()
    o.step(t2 - t1)
    a2 = amp()
    k = 2 * math.pi / L
    return -math.log(a2 / a1) / (k * k * (t2 - t1))


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.0])
def test_shear_wave_viscosity(tau):
    """Chapman-Enskog viscosity nu = cs^2 (tau - 1/2) (sec. 2.2): a sinusoidal shear
    wave decays at nu k^2 (within 1 % at L = 64)."""
    nu = _shear_wave(tau)
    assert abs(nu / (CS2 * (tau - 0.5)) - 1) < 0.01


@pytest.mark.parametrize("tau,at,L", [(0.8, 0.5, 64), (0.8, 0.8, 256), (0.6, 0.5, 64)])
def test_penalized_viscosity(tau, at, L):
    """Penalization on every node with alpha tau < 1 (sec. 2.2, effective viscosity):
    the source re-injects alpha Pi^neq, so the stress relaxes at 1/tau - alpha and
    nu_eff = cs^2 (tau/(1 - alpha tau) - 1/2).  The printed nu/(1 - alpha tau)
    omits the lattice -1/2 term; the test shows which one the scheme follows.
    (At alpha tau = 0.8 the effective relaxation time is 4 and the k^2 error
    term needs L = 256 to drop under 1 %; it converges at second order.)"""
    alpha = at / tau
    nu = _shear_wave(tau, alpha=alpha, penalize_all=1, L=L, t1=100, t2=100 + 500 * (L // 64) ** 2 // 4 + 400)
    expected = CS2 * (tau / (1 - at) - 0.5)
    printed = CS2 * (tau - 0.5) / (1 - at)
    assert abs(nu / expected - 1) < 0.01
    assert abs(nu / printed - 1) > 0.05


# the channel of the rigidity pins: a neutrally buoyant disk carried and
# turned by a force-driven flow between walls
ALPHA_CHANNEL = dict(lattice="D2Q9", n=(64, 48, 1), periodic=(1, 0, 0), tau=0.8, fluid_accel=(2e-6, 0.0, 0.0))
ALPHA_DISK = [dict(shape="disk", rho_s=1.0, a=8.0, x=(32.0, 16.5, 0.0))]


def test_rigidity_grows_with_penalization():
    """Sec. 2.2 (the penalization source and its bound alpha < 1/tau, with
    alpha = 1/tau used in sec. 3): the source drives the velocity inside a
    solid toward rigid motion, the more so the larger alpha, since it removes
    alpha Pi^neq of the stress.  A disk carried and turned by a channel flow:
    the residual max |u - (U + omega x r)| over its nodes falls strictly as
    alpha tau goes 0.5 -> 0.9 -> 0.99 -> 1, by more than 5x overall, while the
    disk's own motion barely changes (U within 3 %)."""
    from measures import rigidity_residual

    res, Us = [], []
    for at in (0.5, 0.9, 0.99, 1.0):
        cfg = dict(ALPHA_CHANNEL, alpha=at / ALPHA_CHANNEL["tau"])
        o = O.Oracle(cfg, ALPHA_DISK)
        o.step(3000)
        u, _, own = o.fields()
        P = o.particles()
        r, umax = rigidity_residual(u, own, P, cfg["periodic"])
        res.append(r / umax)
        Us.append(P["U"][0][0])
    assert all(a > b for a, b in zip(res, res[1:])), res
    assert res[0] > 5 * res[-1], res
    assert max(Us) / min(Us) - 1 < 0.03, Us


def couette_walls(U, axis=1, direction=(1.0, 0.0, 0.0)):
    """wall_velocity of a plane Couette flow: the walls normal to `axis` move at
    -U/2 and +U/2 along `direction`."""
    w = np.zeros((3, 2, 3))
    w[axis, 0] = -0.5 * U * np.asarray(direction)
    w[axis, 1] = 0.5 * U * np.asarray(direction)
    return w.tolist()


@pytest.mark.parametrize("tau", [0.6, 1.0, 1.7])
def test_couette_exact_2d(tau):
    """Halfway bounce-back off walls moving at -U/2 and +U/2 (the Couette
    benchmark of sec. 3.1): the steady profile is the linear one of the walls
    at y = -1/2 and H - 1/2, to round-off, with no normal velocity and a
    uniform pressure (a linear shear is an exact steady state of BGK, and the
    halfway wall adds no slip to it)."""
    H, U = 16, 0.02
    cfg = dict(lattice="D2Q9", n=(3, H), periodic=(1, 0, 0), tau=tau, wall_velocity=couette_walls(U))
    o = O.Oracle(cfg, [])
    o.step(int(40 * H * H / (CS2 * (tau - 0.5))))
    u, p, _ = o.fields()
    exact = -U / 2 + U * (np.arange(H) + 0.5) / H
    assert np.abs(u[0, :, :, 0] - exact[:, None]).max() < 1e-13 * U
    assert np.abs(u[..., 1]).max() < 1e-15 and np.ptp(p) < 1e-15


def test_couette_exact_3d():
    """The same in D3Q19 with the walls normal to z moving along (1, 2, 0)/sqrt 5."""
    H, U, tau = 12, 0.02, 0.9
    d = np.array([1.0, 2.0, 0.0]) / math.sqrt(5.0)
    cfg = dict(lattice="D3Q19", n=(3, 3, H), periodic=(1, 1, 0), tau=tau, wall_velocity=couette_walls(U, 2, d))
    o = O.Oracle(cfg, [])
    o.step(int(40 * H * H / (CS2 * (tau - 0.5))))
    u, _, _ = o.fields()
    prof = -U / 2 + U * (np.arange(H) + 0.5) / H
    for k in range(2):
        assert np.abs(u[..., k] - (prof * d[k])[:, None, None]).max() < 1e-13 * U
    assert np.abs(u[..., 2]).max() < 1e-15


def test_couette_start_keeps_zero_momentum():
    """Impulsively started Couette flow between walls at -U/2 and +U/2: the
    flow is odd about the mid-plane at every step, so the total momentum stays
    zero to round-off while the profile builds up (a wrong sign or side of
    either wall term breaks it)."""
    H, U = 20, 0.04
    cfg = dict(lattice="D2Q9", n=(5, H), periodic=(1, 0, 0), tau=0.7, wall_velocity=couette_walls(U))
    o = O.Oracle(cfg, [])
    for _ in range(5):
        o.step(37)
        u, _, _ = o.fields()
        assert abs(u[..., 0].sum()) < 1e-15 * u[..., 0].size
        assert np.abs(u[0, :, :, 0] + u[0, ::-1, :, 0]).max() < 1e-16
        assert u[0, -1, 0, 0] > 0.1 * U


@pytest.mark.parametrize("bad", [
    dict(periodic=(1, 1, 0)),                                    # moving wall on a periodic axis
    dict(wall_velocity=[[(0, 0, 0)] * 2, [(0, 0.01, 0), (0, 0, 0)], [(0, 0, 0)] * 2]),  # normal motion
    dict(periodic=(0, 1, 0), wall_velocity=[[(0, 0.01, 0), (0, 0, 0)], [(0, 0, 0)] * 2, [(0, 0, 0)] * 2]),  # x walls
    dict(periodic=(0, 0, 0)),                                    # another axis with walls
])
def test_moving_wall_limits(bad):
    """Moving walls are accepted on the y (or z) axis only, tangential, with
    every other axis periodic (a population crossing two walls would have no
    single wall velocity)."""
    cfg = dict(lattice="D2Q9", n=(6, 8), periodic=(1, 0, 0), tau=0.8, wall_velocity=couette_walls(0.01))
    cfg.update(bad)
    with pytest.raises(Exception):
        O.Oracle(cfg, [])


def _poiseuille(tau, H, a=1e-6, steps=None):
    cfg = dict(lattice="D2Q9", n=(3, H), periodic=(1, 0, 0), tau=tau, fluid_accel=(a, 0.0))
    o = O.Oracle(cfg, [])
    nu = CS2 * (tau - 0.5)
    o.step(steps or int(8 * H * H / nu))
    u, _, _ = o.fields()
    y = np.arange(H)
    exact = a / (2 * nu) * (y + 0.5) * (H - 0.5 - y)
    return u[0, :, 1, 0], exact


def test_poiseuille_profile():
    """Force-driven channel between halfway bounce-back walls (walls at -0.5 and
    H - 0.5) with the Guo force and half-force velocity of eq. (14-15): the
    profile is parabolic; the wall slip vanishes at (tau - 1/2)^2 = 3/16 and is
    second order in 1/H otherwise."""
    tau_m = 0.5 + math.sqrt(3.0 / 16.0)
    num, ex = _poiseuille(tau_m, 16)
    assert np.abs(num - ex).max() / ex.max() < 1e-6
    e1 = [np.abs(n_ - e_).max() / e_.max() for n_, e_ in (_poiseuille(0.8, H) for H in (8, 16))]
    assert e1[0] < 0.05 and 3.5 < e1[0] / e1[1] < 4.5


def test_floating_disk_periodic_exact():
    """sec. 3.1 setting, reduced: a neutrally buoyant disk in fully periodic
    uniform flow is an exact fixed point (f = f^eq, so Pi^neq = 0, S = 0, a = 0);
    the disk moves at u0: X^n = X^0 + n u0."""
    cfg = dict(lattice="D2Q9", n=(64, 48), periodic=(1, 1, 0), tau=0.8, u0=(0.02, 0.005))
    o = O.Oracle(cfg, [dict(shape="disk", rho_s=1.0, a=8.0, x=(20.0, 24.0))])
    o.step(300)
    X = o.particles()["X"][0]
    assert abs(X[0] - (20.0 + 300 * 0.02 - 64)) < 1e-10 or abs(X[0] - (20.0 + 300 * 0.02)) < 1e-10
    assert abs(X[1] - (24.0 + 300 * 0.005)) < 1e-10


@pytest.mark.slow
def test_floating_disk_walls():
    """The 200x400 floating-disk workload (x periodic, y walls 190 l.u. from the
    disk): over 2000 steps the disk keeps |U - u0| <= 1e-3 u0."""
    cfg = dict(lattice="D2Q9", n=(200, 400), periodic=(1, 0, 0), tau=0.8, u0=(0.02, 0.0))
    o = O.Oracle(cfg, [dict(shape="disk", rho_s=1.0, a=10.0, x=(100.0, 200.0))])
    rec = o.step(2000, record=True)
    U = rec[:, 0, 4:6]
    assert np.abs(U - [0.02, 0.0]).max() <= 1e-3 * 0.02
    assert rec[0, 0, 13] == 317  # N of the disk at the integer centre


def test_centred_disk_falls_straight_to_a_terminal_velocity():
    """Settling sanity (sec. 3): a disk centred between two walls falls along
    the mid-line -- the step commutes with the mirror x -> n_x - 1 - x (halfway
    walls at -1/2 and n_x - 1/2, a symmetric indicator), so X_x stays on the
    centre line and omega at zero to round-off -- and, started from rest,
    accelerates (|U_y| at step 50 below half its final value) to a terminal
    velocity: over the last two thirds of 3000 steps U_y stays within 5 % of
    its mean (the wobble left is the binary indicator crossing nodes)."""
    cfg = dict(lattice="D2Q9", n=(41, 200), tau=0.8, g=(0.0, -2e-5), eps_p=2.0, eps_w=1.0, delta=1.0)
    o = O.Oracle(cfg, [dict(shape="disk", rho_s=1.5, a=5.0, x=(20.0, 170.0))])
    rec = o.step(3000, record=True)
    X, U, W = rec[:, 0, 0:2], rec[:, 0, 4:6], rec[:, 0, 9]
    Umax = np.abs(U[:, 1]).max()
    assert np.abs(X[:, 0] - 20.0).max() < 1e-12
    assert np.abs(U[:, 0]).max() < 1e-12 * Umax and np.abs(W).max() * 5.0 < 1e-12 * Umax
    late = U[1000:, 1]
    assert late.mean() < 0 and np.abs(late - late.mean()).max() < 0.05 * abs(late.mean())
    assert abs(U[50, 1]) < 0.5 * abs(late.mean())
    assert X[0, 1] - X[-1, 1] > 0.5  # it fell


# ---------------------------------------------------------- complex step vs finite differences

def _small_settling():
    cfg = dict(lattice="D2Q9", n=(24, 40), tau=0.7, g=(0.0, -2e-4), eps_p=2.0, eps_w=1.0, delta=1.0)
    parts = [dict(shape="disk", rho_s=1.5, a=3.0, x=(10.0, 26.0)),
             dict(shape="disk", rho_s=1.3, a=3.0, x=(15.2, 19.5))]
    return cfg, parts


def _loss(cfg, parts, steps, replay=None, cs=None):
    o = O.Oracle(cfg, parts, complex_step=cs)
    if replay is not None:
        o.set_replay(0, replay[0], replay[1])
    o.step(steps)
    P = o.particles()
    if cs is not None:
        Pi = o.particles(imag=True)
        return P["X"][:, 1].mean(), Pi["X"][:, 1].mean() / cs["h"]
    return P["X"][:, 1].mean()


def test_complex_step_matches_finite_differences():
    """The complex-step build differentiates the step map with the indicator
    frozen; central differences with the indicator replayed from the base run
    give the same derivative (rho_s of body 0, tau and |g|)."""
    cfg, parts = _small_settling()
    steps = 60
    base = O.Oracle(cfg, parts)
    rec = base.step(steps, record=True)
    replay = (rec[:, :, 0:3], rec[:, :, 3])
    L0, dL_rho = _loss(cfg, parts, steps, cs=dict(d_rho_s=[1.0, 0.0], h=1e-30))
    _, dL_tau = _loss(cfg, parts, steps, cs=dict(d_tau=1.0, h=1e-30))
    _, dL_g = _loss(cfg, parts, steps, cs=dict(d_gmag=1.0, h=1e-30))
    assert abs(L0 - base.particles()["X"][:, 1].mean()) < 1e-12

    def fd(mod, h):
        cp, pp = mod(+h)
        cm, pm = mod(-h)
        return (_loss(cp, pp, steps, replay) - _loss(cm, pm, steps, replay)) / (2 * h)

    def m_rho(h):
        p2 = [dict(q) for q in parts]
        p2[0]["rho_s"] += h
        return cfg, p2

    def m_tau(h):
        return dict(cfg, tau=cfg["tau"] + h), parts

    def m_g(h):
        return dict(cfg, g=(0.0, cfg["g"][1] - h)), parts

    for dl, mod, h in ((dL_rho, m_rho, 1e-6 * 1.5), (dL_tau, m_tau, 1e-6 * 0.7), (dL_g, m_g, 1e-6 * 2e-4)):
        ref = fd(mod, h)
        assert abs(dl) > 0
        assert abs(dl - ref) <= 1e-5 * abs(ref), (dl, ref)


def test_stored_gradient_complex_step_vs_central_differences():
    """The stored oracle gradient of the differentiated workload (5000 steps,
    tests/golden/adjoint_512x1024_grad.json, written by the script beside it):
    the complex-step derivative agrees with the central differences of the
    replayed oracle for all 18 parameters, to the differences' own accuracy:
    (L(theta + h) - L(theta - h)) / 2h carries the rounding difference of the
    two perturbed 5000-step runs' losses over 2h, a few units in the last
    place of L (at most 10.2 measured); the bound is 32 of them, with
    h = 1e-6 |theta_k| (truncation, of order h^2, is far below it)."""
    import json
    import os

    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "adjoint_512x1024_grad.json")
    gold = json.load(open(path))
    cs, fd = np.asarray(gold["grad_complex_step"]), gold["grad_central_diff"]
    assert len(fd) == 18 and all(v is not None for v in fd)
    h = gold["fd_rel_step"] * np.abs(np.asarray(gold["values"]))
    ulp = np.finfo(float).eps * abs(gold["loss_value"]) / (2 * h)
    for k in range(18):
        assert abs(cs[k] - fd[k]) <= 32 * ulp[k], (gold["params"][k], cs[k], fd[k])


# ---------------------------------------------------------- fractional indicator (an extension)
#
# chi_i(x) = min(1, R_i + 1/2 - |x - X_i|) on the band |x - X_i| < R_i + 1/2
# (disks and spheres), every use of the indicator weighted by chi.  The
# integral of chi over the plane is pi (R^2 + 1/12) (a disk; the linear ramp of
# width one across the circle of radius R adds pi/12 to pi R^2), over space
# (4/3) pi (R^3 + R/4) (a sphere); averaged over the position of the centre
# within a lattice cell, the lattice sum of chi equals that integral exactly.

FRAC_RNG = np.random.default_rng(2511)


@pytest.mark.parametrize("R", [3.3, 8.0])
def test_fractional_area_disk(R):
    vals = []
    for _ in range(200):
        X = (20.0 + FRAC_RNG.uniform(0, 1), 20.0 + FRAC_RNG.uniform(0, 1))
        o = O.Oracle(dict(lattice="D2Q9", n=(40, 40), tau=0.8, fractional=1), [dict(shape="disk", rho_s=1.0, a=R, x=X)])
        vals.append(o.particles()["Nw"][0])
    vals = np.array(vals)
    se = vals.std() / np.sqrt(len(vals))
    exact = np.pi * (R * R + 1.0 / 12.0)
    assert abs(vals.mean() - exact) < 5 * se
    # a binary area (pi R^2) or a ramp ending at R (pi (R^2 - R + 1/3)) is far outside
    assert abs(vals.mean() - np.pi * R * R) > 10 * se
    assert abs(vals.mean() - np.pi * (R * R - R + 1.0 / 3.0)) > 100 * se


def test_fractional_volume_sphere():
    R = 4.0
    vals = []
    for _ in range(80):
        X = tuple(8.0 + FRAC_RNG.uniform(0, 1, 3))
        o = O.Oracle(dict(lattice="D3Q19", n=(16, 16, 16), tau=0.8, fractional=1),
                     [dict(shape="sphere", rho_s=1.0, a=R, x=X)])
        vals.append(o.particles()["Nw"][0])
    vals = np.array(vals)
    se = vals.std() / np.sqrt(len(vals))
    assert abs(vals.mean() - 4.0 / 3.0 * np.pi * (R ** 3 + R / 4.0)) < 5 * se
    assert abs(vals.mean() - 4.0 / 3.0 * np.pi * R ** 3) > 10 * se


def test_fractional_rigid_field_2d():
    """The chi-weighted sums of a rigid field u = U0 + omega0 z x r over a disk
    centred on a node (the weights are symmetric, so sum chi r = 0) return U0
    and omega0; the weight sum is that of the ramp over the disk's nodes."""
    n = (40, 36, 1)
    X = np.array([20.0, 17.0])
    U0 = np.array([0.013, -0.007])
    w0 = 2.3e-3
    o = O.Oracle(dict(lattice="D2Q9", n=n, tau=0.8, fractional=1), [dict(shape="disk", rho_s=1.0, a=7.0, x=tuple(X))])
    f = np.zeros((1, n[1], n[0], 9))
    for y in range(n[1]):
        for x in range(n[0]):
            r = np.array([x, y]) - X
            f[0, y, x] = O.feq("D2Q9", 0.0, U0 + w0 * np.array([-r[1], r[0]]))
    o.set_f(f)
    P = o.particles()
    _, _, own = o.fields()
    ys, xs = np.nonzero(own[0] == 0)
    d = np.hypot(xs - X[0], ys - X[1])
    assert d.max() < 7.5 and np.sum((np.hypot(*np.meshgrid(np.arange(40) - 20.0, np.arange(36) - 17.0)) < 7.5)) == len(d)
    assert abs(P["Nw"][0] - np.minimum(1.0, 7.5 - d).sum()) < 1e-12
    assert np.abs(P["U"][0, :2] - U0).max() < 1e-16
    assert abs(P["omega"][0, 2] - w0) < 1e-16


def test_fractional_rigid_field_3d():
    n = (16, 15, 14)
    X = np.array([8.0, 7.0, 6.0])
    U0 = np.array([0.01, -0.02, 0.005])
    W0 = np.array([1e-3, -2e-3, 3e-3])
    o = O.Oracle(dict(lattice="D3Q19", n=n, tau=0.8, fractional=1), [dict(shape="sphere", rho_s=1.0, a=4.0, x=tuple(X))])
    f = np.zeros((n[2], n[1], n[0], 19))
    for z in range(n[2]):
        for y in range(n[1]):
            for x in range(n[0]):
                r = np.array([x, y, z]) - X
                f[z, y, x] = O.feq("D3Q19", 0.0, U0 + np.cross(W0, r))
    o.set_f(f)
    P = o.particles()
    assert np.abs(P["U"][0] - U0).max() < 1e-16
    assert np.abs(P["omega"][0] - W0).max() < 1e-15


def test_fractional_vs_brute_d2q9():
    """The whole step with the fractional indicator against the brute-force
    transcription: two disks whose bands meet (the lower id owns the shared
    nodes), one across the periodic x axis, contact forces active."""
    parts = [dict(shape="disk", rho_s=1.6, a=2.2, x=(0.7, 3.2)),
             dict(shape="disk", rho_s=1.3, a=2.0, x=(5.1, 4.4))]
    st = _compare_with_brute("D2Q9", (9, 8, 1), (1, 0, 0), parts, (0.0, -1e-3, 0.0), 3, 3, fractional=True)
    assert any(abs(a) > 1e-8 for q in st["parts"] for a in q["A"])
    assert any(0.0 < abs(st["parts"][0]["N"] - k) for k in range(200))  # a weight sum, not a count


def test_fractional_vs_brute_d3q19():
    parts = [dict(shape="sphere", rho_s=1.6, a=1.6, x=(2.0, 2.1, 2.3)),
             dict(shape="sphere", rho_s=1.4, a=1.4, x=(3.4, 3.0, 3.9))]
    _compare_with_brute("D3Q19", (5, 5, 6), (0, 1, 0), parts, (0.0, 0.0, -1e-3), 2, 4, fractional=True)


def test_fractional_velocity_has_no_node_crossing_jumps():
    """What the weights are for (reading 24): a disk settling across about
    six nodes.  With the binary indicator U = sum u / N jumps whenever a node
    enters or leaves (N changes by one): the largest step-to-step change of
    U_y over steps 1000-2500 exceeds 2e-3 of its mean.  With the fractional
    indicator the weights, and so U, move continuously: that change stays
    below 1e-3, and below a fifth of the binary run's."""
    jumps = []
    for frac in (0, 1):
        cfg = dict(lattice="D2Q9", n=(41, 240), tau=0.8, g=(0.0, -2e-4), eps_p=2.0, eps_w=1.0, delta=1.0,
                   fractional=frac)
        o = O.Oracle(cfg, [dict(shape="disk", rho_s=1.5, a=5.0, x=(20.0, 200.0))])
        rec = o.step(2500, record=True)
        late = rec[1000:, 0, 5]
        assert rec[0, 0, 1] - rec[-1, 0, 1] > 5.0  # it crossed several nodes
        jumps.append(np.abs(np.diff(late)).max() / abs(late.mean()))
    assert jumps[0] > 2e-3 and jumps[1] < 1e-3 and jumps[1] < 0.2 * jumps[0], jumps


def test_fractional_rejects_ellipses():
    with pytest.raises(ValueError):
        O.Oracle(dict(lattice="D2Q9", n=(20, 20), tau=0.8, fractional=1),
                 [dict(shape="ellipse", rho_s=1.2, a=4.0, b=2.0, x=(10.0, 10.0), theta=0.3)])


def test_fractional_position_gradient():
    """With the fractional indicator the loss is differentiable in the initial
    centres: the complex-step derivative (the step map with nothing frozen)
    equals central differences of plain runs, with no replay of the indicator.
    With the binary indicator the same differences do not converge (the
    indicator jumps between the +h and -h runs)."""
    cfg, parts = _small_settling()
    steps = 60
    cfg_f = dict(cfg, fractional=1)

    def loss(c, p):
        o = O.Oracle(c, p)
        o.step(steps)
        return o.particles()["X"][:, 1].mean()

    def moved(i, k, h):
        p2 = [dict(q) for q in parts]
        x = list(p2[i]["x"]) + [0.0]
        x[k] += h
        p2[i]["x"] = tuple(x[:2])
        return p2

    h = 1e-4
    for i, k in ((0, 0), (0, 1), (1, 0)):
        dX = np.zeros((2, 3))
        dX[i, k] = 1.0
        _, dcs = _loss(cfg_f, parts, steps, cs=dict(d_X=dX, h=1e-30))
        fd = (loss(cfg_f, moved(i, k, h)) - loss(cfg_f, moved(i, k, -h))) / (2 * h)
        assert abs(dcs - fd) <= 1e-6 * max(abs(fd), 1e-3), (i, k, dcs, fd)
    fd_b = [(loss(cfg, moved(0, 0, hb)) - loss(cfg, moved(0, 0, -hb))) / (2 * hb) for hb in (1e-4, 1e-5)]
    assert abs(fd_b[0] - fd_b[1]) > 10 * abs(fd_b[0]) * 1e-2
