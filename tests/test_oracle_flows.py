"""Pins of the oracle's update (no GPU): closed-form flows and invariants.

Every check here is fixed by something other than the oracle's code:
* rest state: a uniform fluid at rest with boundary data at rest stays put;
* sealed bounce-back box: total mass is conserved exactly (up to rounding);
* write coverage: with a symmetric neighbour table the push update writes
  every population slot exactly once per step;
* shear wave: the decay rate matches the eigenvalue of the linearised D3Q19
  BGK operator built here from the lattice definition, and the viscosity of
  eq. (8) to leading order;
* plane Couette flow between a bounce-back wall and a Ladd velocity lid:
  exact linear profile (pins the sign and factor of the Ladd term);
* pressure-driven square duct: textbook Fourier-series profile (pins the
  ghost-density pressure iolet and eq. (8)), converging at second order
  when the cross-section doubles;
* the straight-pipe configuration: Poiseuille profile, pressure drop, flux
  and wall shear stress (pins the wall shear stress definition's scale);
* porous walls: a box whose walls all leak to the reservoir reaches the
  reservoir state (rho0, at rest) exactly; with a small porosity the box
  stays well mixed and its mean density relaxes exponentially at the rate
  phi * (sum of the weights of its wall links) / (number of sites);
* permutation invariance of the site numbering.
"""
import math

import numpy as np
import pytest

from paper_2202_11770_amd import geometry as G


def _macros(P, f):
    return P.macros(f)


def test_rest_state_all_boundary_kinds(orc):
    g = G.cylinder(u_max=0.0, rho_out=1.0)
    P = orc.Problem(g, 0.8)
    f = P.init()
    _, w, _ = orc.lattice()
    P.run(f, 0, 1000)
    assert np.abs(f - w[None, :]).max() <= 1e-15


@pytest.mark.parametrize("tau", [0.6, 1.3])
def test_sealed_box_mass(orc, tau):
    g = G.sealed_box(24)
    rng = np.random.default_rng(7)
    rho = 1.0 + rng.uniform(-0.01, 0.01, g.n)
    u = rng.uniform(-1, 1, (g.n, 3))
    u *= (0.02 * rng.uniform(0, 1, g.n) / np.linalg.norm(u, axis=1))[:, None]
    P = orc.Problem(g, tau)
    f = P.init(rho, u)
    m0 = P.mass(f)
    flux = 0.0
    eps = 2.0 ** -53
    for chunk in range(4):
        flux += P.run(f, 500 * chunk, 500)
        assert flux == 0.0
        # exact conservation up to rounding: each collision can shift a site's
        # mass by the rounding error of its 19-term density sum (<= 19 eps
        # relative), relaxed by 1/tau; a wrong bounce-back slot would move
        # O(1e-3) per step instead
        steps = 500 * (chunk + 1)
        assert abs(P.mass(f) - m0) / m0 <= steps * 19 * eps / tau


@pytest.mark.parametrize("name", ["cylinder", "tree", "sealed", "couette"])
def test_write_coverage(orc, name):
    g = {"cylinder": lambda: G.cylinder(),
         "tree": lambda: G.tree(seed=3, generations=3, target_sites=20000),
         "sealed": lambda: G.sealed_box(5, 6, 7),
         "couette": lambda: G.couette_column(6)}[name]()
    P = orc.Problem(g, 0.7)
    f = P.init()
    F, _, wc = P.step(f, 0, write_count=True)
    assert (wc == 1).all()
    assert np.isfinite(F).all()


def _linear_bgk_eigs(tau, k):
    """Eigen-decomposition of the D3Q19 BGK update linearised about rest,
    for a Fourier mode exp(i k z): streaming phase times the relaxation
    towards the linearised equilibrium w_i (drho + 3 c_i . dj)."""
    c = G.C.astype(float)
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    E = w[:, None] * (1.0 + 3.0 * c @ c.T)  # d feq_i / d f_j
    om = 1.0 / tau
    Col = np.eye(19) - om * (np.eye(19) - E)
    S = np.diag(np.exp(-1j * k * c[:, 2]))
    return np.linalg.eig(S @ Col), c


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.0])
def test_shear_wave_decay(orc, tau):
    L = 64
    k = 2 * math.pi / L
    (lam, vec), c = _linear_bgk_eigs(tau, k)
    # the shear mode carries x-momentum
    jx = np.abs(vec.T @ c[:, 0])
    lam_shear = lam[np.argmax(jx * (np.abs(lam) > 0.5))]
    assert abs(lam_shear.imag) < 1e-12
    lam_shear = lam_shear.real
    nu = (tau - 0.5) / 3.0
    g = G.periodic_box(1, 1, L)
    z = g.coords[:, 2].astype(float)
    A = 1e-5  # linear regime: nonlinear terms enter the k-mode at O(A^3)
    u = np.zeros((g.n, 3))
    u[:, 0] = A * np.sin(k * z)
    P = orc.Problem(g, tau)
    f = P.init(np.ones(g.n), u)
    P.run(f, 0, 200)  # non-hydrodynamic modes decay like (1 - 1/tau)^t
    amp = []
    span = 2000  # rate over many steps so that rounding of f does not dominate
    for s in range(2):
        _, uu, _ = P.macros(f)
        amp.append(2.0 / L * np.sum(uu[:, 0] * np.sin(k * z)))
        P.run(f, 200 + s * span, span)
    rate_meas = math.log(amp[0] / amp[1]) / span
    rate_eig = -math.log(lam_shear)
    assert abs(rate_meas - rate_eig) <= 1e-8 * rate_eig
    # eq. (8): nu = cs^2 (tau - 1/2) recovered to leading order in k^2
    assert abs(rate_eig / (nu * k * k) - 1.0) < 2e-3


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.3])
def test_couette_ladd(orc, tau):
    H, U = 8, 0.01
    g = G.couette_column(H, U)
    P = orc.Problem(g, tau)
    f = P.init()
    P.run(f, 0, 20000)
    rho, u, _ = P.macros(f)
    z = g.coords[:, 2].astype(float)
    exact = U * (z + 0.5) / H
    assert np.abs(u[:, 0] - exact).max() <= 1e-10 * U
    assert np.abs(u[:, 1:]).max() <= 1e-14
    assert np.abs(rho - 1.0).max() <= 1e-10


@pytest.mark.parametrize("local", [False, True], ids=["rho0", "rho_local"])
def test_couette_ladd_density(orc, local):
    """The Ladd lid in a fluid whose density differs from rho0 (uniform
    rho = 1.2, rho0 = 1): its momentum term carries rho0 (Sec. 2.3.2 read as
    a fixed reference density), so the lid acts as one moving at
    U rho0 / rho, and the steady profile is the linear one scaled by
    rho0 / rho; with the site's own density in the term (the local-density
    reading) the lid moves at U and the profile is exactly U (z + 1/2) / H.
    Either way the closed form holds to the convergence of the run."""
    H, U, tau, rho = 8, 0.01, 0.8, 1.2
    g = G.couette_column(H, U)
    P = orc.Problem(g, tau, rho0=1.0, ladd_rho_local=local)
    f = P.init(np.full(g.n, rho), None)
    P.run(f, 0, 40000)
    r, u, _ = P.macros(f)
    z = g.coords[:, 2].astype(float)
    exact = U * (z + 0.5) / H * (1.0 if local else 1.0 / rho)
    assert np.abs(u[:, 0] - exact).max() <= 1e-10 * U
    assert np.abs(r - rho).max() <= 1e-10
    if local:
        with pytest.raises(ValueError):
            P.adjoint(P.init(), 0, 2, 0, 2)


def _duct_series(y, z, a, b, G_, eta, nterms=201):
    """Steady velocity in the rectangular duct |y| <= a, |z| <= b under a
    pressure gradient -G_ (textbook Fourier series)."""
    s = 0.0
    for n in range(1, nterms + 1, 2):
        s += ((-1) ** ((n - 1) // 2) * (1 - np.cosh(n * np.pi * z / (2 * a)) / np.cosh(n * np.pi * b / (2 * a)))
              * np.cos(n * np.pi * y / (2 * a)) / n ** 3)
    return 16 * a * a * G_ / (eta * np.pi ** 3) * s


@pytest.mark.parametrize("tau,steps", [(0.6, 6000), (0.8, 4000)])
def test_duct_pressure_poiseuille(orc, tau, steps):
    nu = (tau - 0.5) / 3.0
    rho_in, rho_out = 1.006, 1.0
    g = G.duct(16, 16, 64, rho_in=rho_in, rho_out=rho_out)
    P = orc.Problem(g, tau)
    f = P.init()
    P.run(f, 0, steps)
    rho, u, wss = P.macros(f)
    x, y, z = (g.coords[:, a] for a in range(3))
    # pressure gradient from the interior density profile (p = rho/3, eq. (7))
    zs = np.arange(16, 48)
    rz = np.array([rho[z == k].mean() for k in zs])
    fit = np.polyfit(zs, rz, 1)
    slope = fit[0]
    Gp = -slope / 3.0
    assert Gp > 0
    # the linear density profile meets the ghost densities at the iolet planes
    drho = rho_in - rho_out
    assert abs(np.polyval(fit, -0.5) - rho_in) <= 0.1 * drho
    assert abs(np.polyval(fit, 63.5) - rho_out) <= 0.1 * drho
    mid = z == 32
    rmid = rho[mid].mean()
    eta = rmid * nu
    yy = x[mid] - 7.5
    zz = y[mid] - 7.5
    exact = _duct_series(yy, zz, 8.0, 8.0, Gp, eta)
    got = u[mid, 2]
    err = np.linalg.norm(got - exact) / np.linalg.norm(exact)
    assert err <= 0.01
    # wall shear stress at the face-centre wall sites (half a spacing from the
    # wall) vs eta du/dn of the series there; pins the (1 - 1/(2 tau)) factor
    h = 1e-4
    for yc in (7, 8):
        sel = mid & (x == 0) & (y == yc)
        zc = yc - 7.5
        dudn = (_duct_series(-7.5 + h, zc, 8.0, 8.0, Gp, eta) - _duct_series(-7.5 - h, zc, 8.0, 8.0, Gp, eta)) / (2 * h)
        assert abs(wss[sel][0] / (eta * dudn) - 1.0) <= 0.02
    # equal iolet densities keep the fluid at rest
    g2 = G.duct(8, 8, 16, rho_in=1.0, rho_out=1.0)
    P2 = orc.Problem(g2, tau)
    f2 = P2.init()
    P2.run(f2, 0, 300)
    _, u2, _ = P2.macros(f2)
    assert np.abs(u2).max() <= 1e-15


def test_duct_second_order_convergence(orc):
    """Doubling the duct's cross-section (8x8 -> 16x16, length with it, the
    run long enough to converge in both) cuts the profile error against the
    series about fourfold: second-order accuracy of the bulk scheme with
    mid-link bounce-back and the ghost-density iolets at fixed tau."""
    tau = 0.8
    nu = (tau - 0.5) / 3.0
    errs = []
    for w, L, steps in ((8, 32, 2000), (16, 64, 8000)):
        g = G.duct(w, w, L, rho_in=1.006, rho_out=1.0)
        P = orc.Problem(g, tau)
        f = P.init()
        P.run(f, 0, steps)
        rho, u, _ = P.macros(f)
        x, y, z = (g.coords[:, a] for a in range(3))
        zs = np.arange(L // 4, 3 * L // 4)
        Gp = -np.polyfit(zs, np.array([rho[z == k].mean() for k in zs]), 1)[0] / 3.0
        mid = z == L // 2
        c = (w - 1) / 2
        exact = _duct_series(x[mid] - c, y[mid] - c, w / 2, w / 2, Gp, rho[mid].mean() * nu)
        errs.append(np.linalg.norm(u[mid, 2] - exact) / np.linalg.norm(exact))
    print(f"L2 errors {errs[0]:.3e} (8x8), {errs[1]:.3e} (16x16), ratio {errs[0] / errs[1]:.2f}")
    assert errs[1] <= 0.005
    assert errs[0] / errs[1] >= 3.0


def test_cylinder_poiseuille(orc):
    """Straight pipe, radius 8, tau 0.8, parabolic Ladd inlet u_max = 0.01."""
    tau, R, umax = 0.8, 8.0, 0.01
    nu = (tau - 0.5) / 3.0
    g = G.cylinder()
    P = orc.Problem(g, tau)
    f = P.init()
    m0 = P.mass(f)
    flux = P.run(f, 0, 2000)
    rho, u, wss = P.macros(f)
    # mass bookkeeping: M(t) - M(0) equals the summed boundary flux, up to
    # the per-collision rounding of the density sum (see the sealed box)
    assert abs(P.mass(f) - m0 - flux) / m0 <= 2000 * 19 * 2.0 ** -53 / tau
    x, y, z = (g.coords[:, a].astype(float) for a in range(3))
    r2 = (x - 9.5) ** 2 + (y - 9.5) ** 2
    sl = z == 32
    exact = umax * (1 - r2[sl] / R ** 2)
    err = np.linalg.norm(u[sl, 2] - exact) / np.linalg.norm(exact)
    assert err <= 0.05
    zs = np.arange(16, 49)
    rz = np.array([rho[z == k].mean() for k in zs])
    slope = np.polyfit(zs, rz, 1)[0]
    want = -12.0 * nu * umax / R ** 2
    assert abs(slope / want - 1.0) <= 0.05
    Q = u[sl, 2].sum()
    assert abs(Q / (math.pi * R ** 2 * umax / 2) - 1.0) <= 0.05
    # wall shear stress at the wall sites of the mid slice vs eta * du/dr at r = R
    wsites = sl & (g.types == G.SITE_WALL)
    want_w = 2 * nu * umax / R
    ratio = wss[wsites].mean() / want_w
    assert abs(ratio - 1.0) <= 0.15


def test_permutation_invariance(orc):
    g = G.cylinder()
    rng = np.random.default_rng(11)
    perm = rng.permutation(g.n)
    gp = G.permute(g, perm)
    P, Pp = orc.Problem(g, 0.8), orc.Problem(gp, 0.8)
    f, fp = P.init(), Pp.init()
    P.run(f, 0, 50)
    Pp.run(fp, 0, 50)
    assert np.array_equal(f[perm], fp)


def test_porous_box_relaxes_to_reservoir(orc):
    g = G.sealed_box(8)
    ws = g.wall_sites()
    rho0 = 0.99
    # every wall link leaks completely: the only steady state is the reservoir's
    phi = np.zeros(g.n)
    phi[ws] = 1.0
    P = orc.Problem(g, 0.8, rho0=rho0, phi=phi)
    rng = np.random.default_rng(1)
    f = P.init(1.0 + 0.01 * rng.uniform(-1, 1, g.n), 0.01 * rng.uniform(-1, 1, (g.n, 3)))
    P.run(f, 0, 400)
    rho, u, _ = P.macros(f)
    assert np.abs(rho - rho0).max() <= 1e-13 and np.abs(u).max() <= 1e-13
    # a slow leak: the box mixes much faster than it drains, so its mean
    # density follows rho0 + (rho_1 - rho0) exp(-kappa t) with kappa = phi *
    # (sum over wall links of w_i) / N, up to O(phi) mixing corrections
    _, w, _ = orc.lattice()
    ph = 1e-3
    phi[ws] = ph
    P = orc.Problem(g, 0.8, rho0=rho0, phi=phi)
    f = P.init(np.ones(g.n), None)
    links = g.nbr[:, 1:] == G.LINK_WALL
    kappa = ph * float((links * w[None, 1:]).sum()) / g.n
    T = 3000
    P.run(f, 0, T)
    mean = P.mass(f) / g.n
    pred = rho0 + (1.0 - rho0) * math.exp(-kappa * T)
    print(f"mean density {mean:.12f}, well-mixed prediction {pred:.12f}")
    assert abs((mean - rho0) / (pred - rho0) - 1.0) <= 1e-3
