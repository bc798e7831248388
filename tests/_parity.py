"""Error metrics of GPU results against the FP64 oracle (shared by the tests)."""
import numpy as np


def errors(rho, u, wss, rho_r, u_r, wss_r, rho0=1.0):
    """e_rho = max|rho - rho_ref| / rho0
    e_u   = max ||u - u_ref|| / max ||u_ref||
    e_wss = max |wss - wss_ref| / max wss_ref   (None if the reference has no wall stress)
    plus the RMS variants."""
    out = {}
    out["e_rho"] = float(np.abs(rho - rho_r).max() / rho0)
    out["rms_rho"] = float(np.sqrt(np.mean((rho - rho_r) ** 2)) / rho0)
    un = np.linalg.norm(u_r, axis=1)
    scale = un.max() if un.max() > 0 else 1.0
    du = np.linalg.norm(u - u_r, axis=1)
    out["e_u"] = float(du.max() / scale)
    out["rms_u"] = float(np.sqrt(np.mean(du ** 2)) / scale)
    if wss is not None and wss_r is not None and wss_r.max() > 0:
        out["e_wss"] = float(np.abs(wss - wss_r).max() / wss_r.max())
        out["rms_wss"] = float(np.sqrt(np.mean((wss - wss_r) ** 2)) / wss_r.max())
    else:
        out["e_wss"] = None
    return out


def fmt(e):
    return " ".join(f"{k}={v:.3e}" for k, v in e.items() if v is not None)
