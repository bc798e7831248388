"""GPU adjoint with the iolet-flux objective (hlb_set_objective).

J = sum over t in the window of sum_k w_k Q_k(t), Q_k(t) the net outflow
through iolet k during the update t-1 -> t.  Checked against
  * the oracle's reference adjoint (J, per-step amplitude and ghost-density
    derivatives, porosity derivatives);
  * mass conservation: with unit weights and no porosity J is the mass the
    GPU forward run loses over the window;
  * central finite differences through torch.autograd on the tortuous vessel.
"""
import time

import numpy as np
import pytest

import oracle
from paper_2202_11770_amd import geometry as G
from paper_2202_11770_amd import hlb

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def _small_case(nsteps=60, seed=4):
    g = G.tortuous(radius=4.0, length=32, amplitude=4.0, period=32.0)
    rng = np.random.default_rng(seed)
    s = np.arange(nsteps)
    a = rng.uniform(-1, 1, 4) * 0.002 / np.arange(1, 5)
    b = rng.uniform(-1, 1, 4) * 0.002 / np.arange(1, 5)
    A = 0.01 + sum(a[k] * np.cos(2 * np.pi * (k + 1) * s / nsteps) + b[k] * np.sin(2 * np.pi * (k + 1) * s / nsteps)
                   for k in range(4))
    R = 1.0 + 0.001 * np.sin(2 * np.pi * s / nsteps)
    tables = [A if io.kind == G.VELOCITY else R.copy() for io in g.iolets]
    phi = np.zeros(g.n)
    ws = g.wall_sites()
    phi[ws] = np.random.default_rng(40).uniform(0, 1, ws.size)
    return g, tables, phi, ws


@pytest.mark.parametrize("porous", [True, False], ids=["porous", "no_porosity"])
def test_flux_adjoint_matches_oracle_small(porous):
    nsteps, w0, w1, tau = 60, 30, 60, 0.8
    g, tables, phi, ws = _small_case(nsteps)
    if not porous:
        phi = None
    w = np.array([1.0 if io.kind == G.PRESSURE else 0.5 for io in g.iolets])
    say(f"case: small tortuous {g.n} sites, {nsteps} steps, window ({w0},{w1}], weights {w}, porous {porous}")
    P = oracle.Problem(g, tau, tables=tables, phi=phi)
    Jr, dTr, dphir = P.adjoint(P.init(), 0, nsteps, w0, w1, weights=w)
    sim = hlb.Simulation.create(g, tau, tables=tables, adjoint=True)
    if porous:
        hlb.hlb_set_porosity(sim.ctx, phi)
    hlb.hlb_set_objective(sim.ctx, hlb.HLB_OBJ_IOLET_FLUX, w)
    J, dT, dphi, fw = hlb.hlb_adjoint_run(sim.ctx, nsteps, w0, w1, 4)
    say(f"flux adjoint: J {J:.9e} vs {Jr:.9e}; table rows rel {rel(dT, dTr):.2e}; dphi rel {rel(dphi, dphir):.2e}")
    assert abs(J - Jr) <= 1e-12 * abs(Jr)
    for k, io in enumerate(g.iolets):
        e = rel(dT[k], dTr[k])
        say(f"  iolet {k} ({'velocity' if io.kind == G.VELOCITY else 'pressure'}): rel {e:.2e}")
        assert e <= 1e-10
    assert rel(dphi, dphir) <= 1e-10
    # argument checks
    for kind, wts, match in ((7, w, "unknown objective"), (hlb.HLB_OBJ_IOLET_FLUX, None, "needs weights"),
                             (hlb.HLB_OBJ_IOLET_FLUX, np.array([1.0, np.nan]), "not finite")):
        with pytest.raises(hlb.HLBError, match=match):
            hlb.hlb_set_objective(sim.ctx, kind, wts)
    # back to the WSS objective: the earlier result comes back
    hlb.hlb_set_objective(sim.ctx, hlb.HLB_OBJ_WSS)
    Jw, _, _, _ = hlb.hlb_adjoint_run(sim.ctx, nsteps, w0, w1, 4)
    Jw_r, _, _ = P.adjoint(P.init(), 0, nsteps, w0, w1)
    assert abs(Jw - Jw_r) <= 1e-12 * abs(Jw_r)
    sim.close()


def test_unit_weight_flux_is_gpu_mass_loss():
    nsteps, w0, w1, tau = 200, 50, 200, 0.8
    g, tables, _, _ = _small_case(nsteps)
    say(f"case: small tortuous {g.n} sites, unit weights, window ({w0},{w1}]")
    sim = hlb.Simulation.create(g, tau, tables=tables, adjoint=True)
    hlb.hlb_set_objective(sim.ctx, hlb.HLB_OBJ_IOLET_FLUX, np.ones(len(g.iolets)))
    J, _, _, _ = hlb.hlb_adjoint_run(sim.ctx, nsteps, w0, w1, 8)
    sim.step(w0)
    m0, _ = hlb.hlb_mass_balance(sim.ctx)
    sim.step(w1 - w0)
    m1, _ = hlb.hlb_mass_balance(sim.ctx)
    say(f"J {J:.12e}  mass loss {m0 - m1:.12e}")
    assert abs(J) > 1e-3
    assert abs(J - (m0 - m1)) <= 1e-12 * m0
    sim.close()


def test_flux_autograd_vs_fd_tortuous():
    """Tortuous vessel (~1.25e5 sites), tau 0.8, 1000 steps, window (800, 1000],
    J = outflow through the pressure outlet; gradients through
    IoletFluxObjective for 8 Fourier inlet coefficients, the per-step outlet
    ghost densities and the wall porosity, against central FD of the GPU
    objective.  The objective is summed with atomics (run-to-run rounding
    ~1e-13 relative), so the steps are 1e-5 (Fourier coefficients) and 1e-4
    (ghost densities, porosity); J is close to linear in all three."""
    import torch
    from paper_2202_11770_amd.autograd import IoletFluxObjective, fourier_inlet
    g = G.tortuous()
    n, w0, w1, tau, n_snap = 1000, 800, 1000, 0.8, 10
    rng = np.random.default_rng(4)
    k = np.arange(1, 5)
    theta0 = np.concatenate([rng.uniform(-1, 1, 4) * 0.001 / k, rng.uniform(-1, 1, 4) * 0.001 / k])
    R0 = 1.0 + 0.0005 * np.cos(2 * np.pi * np.arange(n) / n)
    phi0 = np.zeros(g.n)
    ws = g.wall_sites()
    phi0[ws] = np.random.default_rng(40).uniform(0.01, 0.2, ws.size)  # FD stays in [0, 1]
    kinds = [io.kind for io in g.iolets]
    w = np.array([1.0 if kk == G.PRESSURE else 0.0 for kk in kinds])
    say(f"case: tortuous {g.n} sites, {n} steps, window ({w0},{w1}], outlet flux, {n_snap} snapshots")
    sim = hlb.Simulation.create(g, tau, adjoint=True)
    theta = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
    R = torch.tensor(R0[None, :], dtype=torch.float64, requires_grad=True)
    phi = torch.tensor(phi0, dtype=torch.float64, requires_grad=True)
    t = time.time()
    A = fourier_inlet(theta, n, period=float(n))[None, :]
    J = IoletFluxObjective.apply(A, R, phi, sim, n, w0, w1, n_snap, w)
    J.backward()
    say(f"adjoint: J = {J.item():.10e} in {time.time() - t:.2f}s")
    g_theta, g_R, g_phi = theta.grad.numpy().copy(), R.grad.numpy()[0].copy(), phi.grad.numpy().copy()
    vel, pres = kinds.index(G.VELOCITY), kinds.index(G.PRESSURE)

    def J_of(th, Rt, ph):
        A_ = fourier_inlet(torch.tensor(th, dtype=torch.float64), n, period=float(n)).numpy()
        hlb.hlb_set_iolet_table(sim.ctx, vel, A_)
        hlb.hlb_set_iolet_table(sim.ctx, pres, Rt)
        hlb.hlb_set_porosity(sim.ctx, ph)
        hlb.hlb_set_objective(sim.ctx, hlb.HLB_OBJ_IOLET_FLUX, w)
        return hlb.hlb_adjoint_run(sim.ctx, n, w0, w1, n_snap, want_dA=False, want_dphi=False)[0]

    assert abs(J_of(theta0, R0, phi0) - J.item()) <= 1e-12 * abs(J.item())
    h = 1e-5
    fd = []
    for j in range(theta0.size):
        e = np.zeros(theta0.size)
        e[j] = h
        fd.append((J_of(theta0 + e, R0, phi0) - J_of(theta0 - e, R0, phi0)) / (2 * h))
    e_theta = rel(g_theta, fd)
    steps = [0, 150, 420, 799, 800, 801, 900, 998]
    hr = 1e-4
    fdr = []
    for s in steps:
        e = np.zeros(n)
        e[s] = hr
        fdr.append((J_of(theta0, R0 + e, phi0) - J_of(theta0, R0 - e, phi0)) / (2 * hr))
    e_R = rel(g_R[steps], fdr)
    hp = 1e-4
    e_dir = []
    prng = np.random.default_rng(3)
    for _ in range(3):
        v = np.zeros(g.n)
        v[ws] = prng.uniform(-1, 1, ws.size)
        v /= np.abs(v).max()
        fdv = (J_of(theta0, R0, phi0 + hp * v) - J_of(theta0, R0, phi0 - hp * v)) / (2 * hp)
        e_dir.append(abs(float(g_phi @ v) - fdv) / abs(fdv))
    say(f"FD: theta rel {e_theta:.2e}; ghost densities rel {e_R:.2e}; porosity directions "
        f"{['%.2e' % x for x in e_dir]}")
    assert e_theta <= 1e-6 and e_R <= 1e-6 and max(e_dir) <= 1e-6
    sim.close()
