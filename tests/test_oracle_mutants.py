"""Mutation tests of the oracle's pins (no GPU).

Each case plants one plausible mistake in a copy of the oracle's sources (a
dropped term, a wrong sign, index or operand order), builds that copy in a
temporary directory, and runs the pin tests that should catch it against it,
in a separate process.  The case passes when those pins fail.  The unaltered
copy must pass the same pins, so the harness itself is checked too.

The mistakes are made in the copy only; the oracle under oracle/ is never
changed.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")

ALG = "tests/test_oracle_algebra.py"
FLOWS = "tests/test_oracle_flows.py"
ADJ = "tests/test_oracle_adjoint.py"
TAN = "tests/test_oracle_tangent.py"
REST = FLOWS + "::test_rest_state_all_boundary_kinds"
COUETTE = FLOWS + "::test_couette_ladd"
COUETTE_RHO = FLOWS + "::test_couette_ladd_density"
PIPE = FLOWS + "::test_cylinder_poiseuille"
DUCT = FLOWS + "::test_duct_pressure_poiseuille"
POROUS = FLOWS + "::test_porous_box_relaxes_to_reservoir"
WKADJ = "tests/test_oracle_windkessel_adjoint.py"
DOT = TAN + "::test_dot_product_identity"
TLFD = TAN + "::test_tangent_vs_central_differences"

# (name, source file, original text, planted text, pin tests expected to fail)
MUTANTS = [
    # equilibrium eq. (4) as printed, without the 1/2 on the (c.u)^2 term
    ("feq_no_half", "oracle.c", "(cu * cu) / (2.0 * CS2 * CS2)", "(cu * cu) / (CS2 * CS2)", [ALG]),
    # a weight of the wrong shell
    ("weight_shell", "oracle.c", "1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,",
     "1.0 / 18.0, 1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0,", [ALG]),
    # momentum picks up the wrong component
    ("momentum_component", "oracle.c", "jy += f[i] * C[i][1];", "jy += f[i] * C[i][2];", [ALG]),
    # collision relaxes away from equilibrium
    ("collision_sign", "oracle.c", "fp[i] = fx[i] - (fx[i] - feq[i]) / tau;", "fp[i] = fx[i] + (fx[i] - feq[i]) / tau;",
     [REST]),
    # bounce-back into the same direction instead of the opposite one
    ("bounce_back_slot", "oracle.c", "slot = ORC_Q * x + OPP[i];\n          val = (1.0 - ph)",
     "slot = ORC_Q * x + i;\n          val = (1.0 - ph)", [REST]),
    # Ladd term with the wrong sign, and with the wrong factor
    ("ladd_sign", "oracle.c", "return fp[i] - 2.0 * W[i] * rw * cdot(i, U) / CS2;",
     "return fp[i] + 2.0 * W[i] * rw * cdot(i, U) / CS2;", [COUETTE]),
    ("ladd_factor", "oracle.c", "return fp[i] - 2.0 * W[i] * rw * cdot(i, U) / CS2;",
     "return fp[i] - 1.0 * W[i] * rw * cdot(i, U) / CS2;", [COUETTE]),
    # Ladd density: the local-density option ignored, or taken in both modes
    ("ladd_density_ignored", "oracle.c", "const double rw = K->rho_local ? rho_x : rho0;",
     "const double rw = rho0;", [COUETTE_RHO]),
    ("ladd_density_always_local", "oracle.c", "const double rw = K->rho_local ? rho_x : rho0;",
     "const double rw = rho_x;", [COUETTE_RHO]),
    # ghost-density rule returns the equilibrium of the outgoing direction
    ("pressure_direction", "oracle.c", "return fg[OPP[i]];", "return fg[i];", [PIPE, DUCT]),
    # ghost velocity reversed
    ("pressure_velocity_sign", "oracle.c", "const double ug[3] = {un * nk[0], un * nk[1], un * nk[2]};",
     "const double ug[3] = {-un * nk[0], -un * nk[1], -un * nk[2]};", [PIPE, DUCT]),
    # porous wall leaks to density 1 instead of the reservoir density rho0
    ("porosity_reservoir", "oracle.c", "val = (1.0 - ph) * fp[i] + ph * W[i] * rho0;",
     "val = (1.0 - ph) * fp[i] + ph * W[i];", [POROUS]),
    # porous wall leaks twice as fast
    ("porosity_factor", "oracle.c", "val = (1.0 - ph) * fp[i] + ph * W[i] * rho0;",
     "val = (1.0 - 2.0 * ph) * fp[i] + 2.0 * ph * W[i] * rho0;", [POROUS]),
    # wall shear stress without the (1 - 1/(2 tau)) factor
    ("wss_factor", "oracle.c", "const double fac = -(1.0 - 1.0 / (2.0 * tau));", "const double fac = -1.0;", [PIPE, DUCT]),
    # adjoint: the pressure rule's dependence on the site velocity dropped
    ("adj_pressure_term", "oracle_adjoint.c", "mu_out[ORC_Q * x + j] = v + dpre[j];", "mu_out[ORC_Q * x + j] = v;",
     [DOT, ADJ]),
    # adjoint: wall link reads the adjoint of the wrong slot
    ("adj_wall_slot", "oracle_adjoint.c", "const double m = mu_next[ORC_Q * x + LOPP[i]];\n          const double ph",
     "const double m = mu_next[ORC_Q * x + i];\n          const double ph", [DOT, ADJ]),
    # adjoint: collision Jacobian not transposed
    ("adj_transpose", "oracle_adjoint.c", "v += a[i] * D[i][j] / tau;", "v += a[i] * D[j][i] / tau;", [DOT, ADJ]),
    # adjoint: porosity derivative with the wrong sign
    ("adj_porosity_sign", "oracle_adjoint.c", "dJ_dphi[x] += m * (LW[i] * rho0 - fp[i]);",
     "dJ_dphi[x] += m * (fp[i] - LW[i] * rho0);", [DOT, ADJ]),
    # adjoint: wall shear stress gradient without its factor
    ("adj_wss_factor", "oracle_adjoint.c", "wd[i] = fac * cn * ce;", "wd[i] = cn * ce;", [DOT, ADJ]),
    # adjoint: the outflow's direct term at Ladd links with the wrong sign
    ("adj_flux_ladd", "oracle_adjoint.c", "myA[k] += (m - wk) * (-2.0 * LW[i]", "myA[k] += (m + wk) * (-2.0 * LW[i]",
     [DOT, ADJ]),
    # adjoint through a Windkessel outlet: the capacitor's 1/C dropped from
    # dX(s+1)/dQ(s); the leak's decay of X taken with the wrong sign
    ("adj_wk_capacitance", "oracle_adjoint.c", "(P[2] > 0.0 ? 1.0 / P[2] : P[3]) * LX[k]",
     "(P[2] > 0.0 ? 1.0 : P[3]) * LX[k]", [WKADJ]),
    ("adj_wk_leak_sign", "oracle_adjoint.c", "1.0 - (P[3] > 0.0 ? 1.0 / (P[3] * P[2]) : 0.0)",
     "1.0 + (P[3] > 0.0 ? 1.0 / (P[3] * P[2]) : 0.0)", [WKADJ]),
    # tangent: velocity derivative without the density term
    ("tan_velocity", "oracle_tangent.c", "du[a] = (dj[a] - dr * u[a]) / r;", "du[a] = dj[a] / r;", [TLFD]),
    # tangent: porous-wall derivative with the wrong sign
    ("tan_porosity_sign", "oracle_tangent.c", "(1.0 - ph) * dfp[i] - dph * fp[i] + dph * TW[i] * rho0;",
     "(1.0 - ph) * dfp[i] + dph * fp[i] + dph * TW[i] * rho0;", [TLFD]),
]


def _run_pins(tmp_path, edit, pins):
    src = tmp_path / "src"
    src.mkdir()
    for name in os.listdir(ORACLE):
        if name.endswith((".c", ".h")):
            shutil.copy(os.path.join(ORACLE, name), src / name)
    if edit is not None:
        fname, old, new = edit
        text = (src / fname).read_text()
        assert text.count(old) == 1, f"mutation site not unique in {fname}: {old!r}"
        (src / fname).write_text(text.replace(old, new))
    env = dict(os.environ, HLB_ORACLE_SRC=str(src), HLB_ORACLE_LIB=str(tmp_path / "liboracle_mutant.so"),
               PYTHONDONTWRITEBYTECODE="1", OMP_NUM_THREADS=os.environ.get("OMP_NUM_THREADS", "4"))
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu", *pins]
    return subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


def test_unaltered_copy_passes_the_pins(tmp_path):
    r = _run_pins(tmp_path, None, [ALG, FLOWS, ADJ, TAN, WKADJ])
    print(r.stdout[-2000:])
    assert r.returncode == 0


@pytest.mark.parametrize("name,fname,old,new,pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(tmp_path, name, fname, old, new, pins):
    r = _run_pins(tmp_path, (fname, old, new), pins)
    failed = [ln for ln in r.stdout.splitlines() if ln.startswith("FAILED")]
    print(name, "->", failed[:3] if failed else r.stdout[-800:])
    # exit status 1: tests ran and at least one failed (not a collection or
    # build error, which would exit differently)
    assert r.returncode == 1 and failed
