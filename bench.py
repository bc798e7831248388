"""Throughput of the sparse D3Q19 LBGK update on one MI355X.

Workload (default): the seeded bifurcating tree of ~2.0e8 fluid sites (seed
2, 8 branching generations, Murray radii, 30-60 deg branch angles, lengths of
6-10 radii), tau = 0.6, one Ladd velocity inlet with
A(s) = 0.02 * (1 - cos(2 pi s / 2000)) / 2 and 256 pressure outlets at
rho = 1, FP64 storage; the same geometry is also run with the shifted FP32
and FP16 storages.  A step is one full LB update of every site (all groups),
i.e. one pass of the hot path.

Error of each storage, stated beside its throughput:
  - against the FP64 oracle on the error subtree of the same tree (the
    first-child branch of the generation whose subtree has about 2e6 sites,
    at the same lattice spacing, with its own Ladd inlet and rho = 1
    leaves), every site after 1000 steps from rest;
  - FP32 and FP16 against the FP64 GPU run on the full tree, every site
    after the same number of steps (compared on the device).

Prints ONE JSON line:
  value       MLUPS of the FP64 run (eq. (9): sites x steps / (s x 1e6))
  roofline    the step kernel (the only kernel of a step) against 8 TB/s:
              algorithmic bytes per launch (38 population loads/stores +
              the pull-table bytes per site, times all sites) over its mean
              launch duration from HIP events on its stream
  cpu_baseline  the FP64 oracle on the host cores, timed on its error
              reference run over the subtree (a bounded sample of the
              workload)
  storages    MLUPS, step-kernel GB/s and fraction of peak for f64/f32/f16
  errors_vs_oracle, errors_vs_f64_gpu   the errors above
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_GBS = 8000.0  # MI355X HBM3E


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Geometry scales that give the stated site counts (found by the generators'
# own scale iteration; recorded so that the large cases are voxelised once).
TREE_SCALE_200M = 2.446148147624885   # seed 2, 8 generations: 200,030,189 sites
FOREST_SCALE_600M = 1.0722357994557143  # seed 5, 8x8 trees of 4 generations: 600,343,441 sites

WORKLOADS = {
    # name: (tau, default steps, storages, description)
    "tree20m": (0.6, 1000, "f64,f32,f16", "bifurcating tree, seed 2, 8 generations, ~2.0e7 sites, "
                "1 Ladd inlet + 256 pressure outlets"),
    "tree200m": (0.6, 200, "f64,f32,f16", "bifurcating tree, seed 2, 8 generations, ~2.0e8 sites, "
                 "1 Ladd inlet + 256 pressure outlets"),
    "forest600m": (0.55, 500, "f32", "forest of 64 trees (seed 5, 4 generations), ~6.0e8 sites, "
                   "64 Ladd inlets + 1024 pressure outlets"),
}


def inlet_table():
    """A(s) = u_max (1 - cos(2 pi s / T)) / 2, u_max = 0.02, T = 2000 steps."""
    import numpy as np
    s = np.arange(2000)
    return 0.02 * 0.5 * (1.0 - np.cos(2.0 * np.pi * s / 2000.0))


def tree_workload(target=20_000_000, seed=2, generations=8, scale=None, verbose=False):
    import numpy as np
    from paper_2202_11770_amd import geometry as G
    g = G.tree(seed=seed, generations=generations, target_sites=target, scale=scale, verbose=verbose)
    tables = [inlet_table() if io.kind == G.VELOCITY else np.array([1.0]) for io in g.iolets]
    return g, tables


def workload(name):
    import numpy as np
    from paper_2202_11770_amd import geometry as G
    if name == "tree20m":
        return tree_workload()
    if name == "tree200m":
        return tree_workload(scale=TREE_SCALE_200M, verbose=True)
    if name == "forest600m":
        g = G.forest(scale=FOREST_SCALE_600M, verbose=True)
        tables = [inlet_table() if io.kind == G.VELOCITY else np.array([1.0]) for io in g.iolets]
        return g, tables
    raise ValueError(name)


def kernel_source_hash():
    """Hash of the code (comments and blank space removed) of the sources the
    step kernel is compiled from: a comment edit leaves measured counters
    valid, any code change invalidates them."""
    import re
    h = hashlib.sha256()
    for name in ("hlb_device.h", "hlb_kernels.hip", "hlb_internal.h"):
        text = open(os.path.join(ROOT, "paper_2202_11770_amd", "csrc", name)).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def order_tag(order, block):
    """Site order as recorded with the counters: "bands7", "columns6", "lex", ..."""
    return f"{order}{block}" if order in ("bands", "columns") else order


def stored_traffic(storage, n_sites, order):
    """HBM bytes per step-kernel launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source, workload and site
    order (an order_tag); else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    sha = kernel_source_hash()
    for e in json.load(open(p)).get("entries", []):
        if (e.get("storage") == storage and e.get("n_sites") == n_sites and e.get("kernel_sha") == sha
                and e.get("order") == order):
            return e.get("bytes_per_launch")
    return None


ORDER = (None, 0)  # site order of the timed runs and its block width (None, 0: the library's defaults)


def run_storage(g, tables, tau, storage, steps, warmup, scheme="pull", windkessel=None, sites_per_thread=0):
    import torch
    from paper_2202_11770_amd import hlb
    t0 = time.time()
    sim = hlb.Simulation.create(g, tau, storage=storage, tables=tables, scheme=scheme,
                                sites_per_thread=sites_per_thread, order_block=ORDER[1],
                                **({"order": ORDER[0]} if ORDER[0] else {}))
    for k, m in (windkessel or {}).items():
        hlb.hlb_set_windkessel(sim.ctx, k, m)
    info = sim.info()
    log(f"{storage}: context created in {time.time() - t0:.1f}s, {info['device_bytes'] / 2**30:.1f} GiB on the device")
    sim.step(warmup)
    hlb.hlb_sync(sim.ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    hlb.hlb_sync(sim.ctx)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # second pass with HIP events around every launch on the library's stream
    hlb.hlb_set_timing(sim.ctx, True)
    sim.step(steps)
    st = hlb.hlb_stats(sim.ctx)
    hlb.hlb_set_timing(sim.ctx, False)
    m, r = hlb.hlb_mass_balance(sim.ctx)
    sim.close()
    n = info["n_sites"]
    bpl = info["bytes_per_lup"]
    mlups = n * steps / dt / 1e6
    # one step kernel updates every site of every group
    achieved = bpl * n / (st["kernel_ms"] * 1e-3) / 1e9
    order = {v: k for k, v in hlb.ORDER.items()}[info["order"]]
    order_block = ORDER[1] or hlb.hlb_default_options().order_block
    return dict(storage=storage, n_sites=n, bytes_per_lup=bpl, ms_per_step=dt / steps * 1e3, order=order,
                order_block=order_block if order in ("bands", "columns") else None,
                xcd_remap=info["xcd_remap"],
                mlups=mlups, alg_gbs=bpl * n * steps / dt / 1e9, kernel_ms=st["kernel_ms"],
                event_step_ms=st["step_ms"], kernel_gbs=achieved,
                frac=achieved / PEAK_GBS, mass=m, mass_residual_rel=r / m)


def device_macros(g, tables, tau, storage, steps):
    """rho, u, wss (device, FP64) after `steps` steps from rest."""
    import torch
    from paper_2202_11770_amd import hlb
    sim = hlb.Simulation.create(g, tau, storage=storage, tables=tables)
    log(f"{storage}: {steps} steps from rest for the error comparison")
    sim.step(steps)
    rho = torch.empty(g.n, dtype=torch.float64, device="cuda")
    u = torch.empty(g.n, 3, dtype=torch.float64, device="cuda")
    wss = torch.empty(g.n, dtype=torch.float64, device="cuda")
    hlb.hlb_macros_device(sim.ctx, rho, u, wss)
    hlb.hlb_sync(sim.ctx)
    m, r = hlb.hlb_mass_balance(sim.ctx)
    sim.close()
    return rho, u, wss, m


def storage_errors(a, ref, rho0=1.0):
    """Max and RMS errors of (rho, u, wss) against a reference run: rho
    relative to rho0, u relative to max |u_ref|, wss relative to max wss_ref."""
    rho, u, wss = a[:3]
    rr, ur, wr = ref[:3]
    du = (u - ur).norm(dim=1)
    us = float(ur.norm(dim=1).max())
    ws = float(wr.max())
    return {"e_rho": float((rho - rr).abs().max()) / rho0,
            "rms_rho": float((rho - rr).pow(2).mean().sqrt()) / rho0,
            "e_u": float(du.max()) / us, "rms_u": float(du.pow(2).mean().sqrt()) / us,
            "e_wss": float((wss - wr).abs().max()) / ws,
            "rms_wss": float((wss - wr).pow(2).mean().sqrt()) / ws,
            "mass_rel": (a[3] - ref[3]) / ref[3]}


def compare_storages(g, tables, tau, storages, steps):
    """Errors of each reduced-precision storage against the FP64 GPU run over
    the same steps from rest, every site compared on the device."""
    import torch
    ref = device_macros(g, tables, tau, "f64", steps)
    out = {}
    for st in storages:
        if st == "f64":
            continue
        a = device_macros(g, tables, tau, st, steps)
        out[st] = {k: float(f"{v:.4g}") for k, v in storage_errors(a, ref).items()}
        log(f"{st} vs f64-GPU after {steps} steps: {out[st]}")
        del a
        torch.cuda.empty_cache()
    return out


def run_split(g, tables, tau, storage, steps, warmup, nparts, exchange="direct"):
    """The same workload as nparts partitions on this GPU with the halo
    exchange overlapped (the one-GPU emulation of a domain split)."""
    import torch
    from paper_2202_11770_amd import halo
    t0 = time.time()
    sp = halo.SplitSimulation(g, tau, storage=storage, tables=tables, nparts=nparts, exchange=exchange)
    log(f"split {storage} ({exchange} exchange): {nparts} parts created in {time.time() - t0:.1f}s")
    sp.step(warmup)
    sp.synchronize()
    t0 = time.perf_counter()
    sp.step(steps)
    sp.synchronize()
    dt = time.perf_counter() - t0
    n_halo = sum(int(v[0].size) for P in sp.parts for v in P.send.values())
    ghosts = sum(P.glob.size - P.n_owned for P in sp.parts)
    sp.close()
    return {"parts": nparts, "exchange": exchange, "mlups": round(g.n * steps / dt / 1e6, 1),
            "ms_per_step": round(dt / steps * 1e3, 4),
            "halo_values_per_step": n_halo, "ghost_sites": int(ghosts)}


def run_split_fresh(workload_name, storage, steps, warmup, nparts, exchange):
    """run_split in a process of its own.  The split's streams map onto the
    GPU's few hardware queues in an order that depends on what the process
    ran before: in one process a split run after another one measured up to
    40% slower than the same run first, so every split run starts fresh."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--workload", workload_name, "--steps", str(steps),
           "--warmup", str(warmup), "--split-one", f"{storage},{exchange},{nparts}"]
    out = subprocess.run(cmd, capture_output=True, text=True, check=True).stdout
    return json.loads([l for l in out.splitlines() if l.startswith("{")][-1])


def oracle_rate(g, tables, tau, budget_s):
    """Oracle MLUPS on a bounded sample: steps (after one untimed) until about
    budget_s of work.  Returns (mlups, steps)."""
    import oracle
    P = oracle.Problem(g, tau, tables=tables)
    f = P.init()
    t0 = time.perf_counter()
    P.run(f, 0, 1)
    one = time.perf_counter() - t0
    k = max(1, min(2000, int(budget_s / max(one, 1e-4))))
    t0 = time.perf_counter()
    P.run(f, 1, k)
    dt = time.perf_counter() - t0
    return g.n * k / dt / 1e6, k


def gpu_rate(g, tables, tau, storage, steps):
    from paper_2202_11770_amd import hlb
    sim = hlb.Simulation.create(g, tau, storage=storage, tables=tables)
    sim.step(20)
    hlb.hlb_sync(sim.ctx)
    t0 = time.perf_counter()
    sim.step(steps)
    hlb.hlb_sync(sim.ctx)
    dt = time.perf_counter() - t0
    sim.close()
    return g.n * steps / dt / 1e6


def oracle_table(g20, tables20, budget_s=4.0):
    """The oracle with all host threads and with one, beside the GPU, on the
    pipe, the benchmark tree, the error subtree of the 2e8-site tree and the
    tortuous vessel (the sizes where the oracle is practical)."""
    import oracle
    import numpy as np
    from paper_2202_11770_amd import geometry as G
    seg = G.tree_segments(2, 8, scale=TREE_SCALE_200M, origin=(0.5, 0.5, -0.5))
    sub = G.subtree(segments=seg, scale=TREE_SCALE_200M, target_sites=2_000_000)
    tort = G.tortuous()
    s = np.arange(3000)
    tort_tab = [0.01 + 0.001 * np.sin(2 * np.pi * s / 3000) if io.kind == G.VELOCITY else np.array([1.0])
                for io in tort.iolets]
    cases = [("pipe (13,312 sites)", G.cylinder(), None, 0.8),
             (f"tree20m ({g20.n} sites)", g20, tables20, 0.6),
             (f"error subtree of tree200m ({sub.n} sites)", sub,
              [inlet_table() if io.kind == G.VELOCITY else np.array([1.0]) for io in sub.iolets], 0.6),
             (f"tortuous vessel ({tort.n} sites)", tort, tort_tab, 0.8)]
    nmax = oracle.threads()
    rows = []
    for name, g, tabs, tau in cases:
        row = {"case": name, "n_sites": int(g.n)}
        for nt in (nmax, 1):
            oracle.set_threads(nt)
            mlups, k = oracle_rate(g, tabs, tau, budget_s)
            row[f"oracle_{nt}t_mlups"] = round(mlups, 3)
            row[f"oracle_{nt}t_steps"] = k
        oracle.set_threads(nmax)
        for st in ("f64", "f32", "f16"):
            row[f"gpu_{st}_mlups"] = round(gpu_rate(g, tabs, tau, st, 500 if g.n < 1e6 else 200), 1)
        row["gpu_f64_vs_oracle_1t"] = round(row["gpu_f64_mlups"] / row["oracle_1t_mlups"], 1)
        log(f"oracle table: {row}")
        rows.append(row)
    return {"threads": nmax, "rows": rows}


def run_adjoint(g, tables, tau, n=40, n_snap=10):
    """hlb_adjoint_run on the workload (FP64, WSS objective over the last
    half of n steps; also timed with every step inside the window and with
    none, and the mean for the differentiation protocol's window, the last
    sixth of the steps): the reverse step's kernels timed with HIP events
    and set against their algorithmic bytes per site:
      k_adj_collide: gather of s (19 x 8 + the pull table), mu read, nu
                     written (19 x 8 each), porosity derivative read and
                     written (16), order (4);
      k_adj_stream:  order (4), the pull table again (its entry opp(i) names
                     the site that pulled population i), nu gathered and mu
                     written (19 x 8 each)."""
    from paper_2202_11770_amd import hlb
    sim = hlb.Simulation.create(g, tau, tables=tables, adjoint=True)
    info = sim.info()

    def timed(w0, w1):
        hlb.hlb_set_timing(sim.ctx, True)
        t0 = time.perf_counter()
        J, _, _, fw = hlb.hlb_adjoint_run(sim.ctx, n, w0, w1, n_snap)
        wall = time.perf_counter() - t0
        return J, fw, wall, hlb.hlb_stats(sim.ctx)["adj_ms"]

    J, fw, wall, adj_ms = timed(n // 2, n)
    # reverse steps inside the objective window (the boundary kernel also
    # takes every wall site) and outside it (iolet sites only)
    in_ms = timed(0, n)[3]
    out_ms = timed(n, n)[3]
    # the forward step kernel in the same context (its site order)
    hlb.hlb_set_timing(sim.ctx, True)
    sim.step(20)
    fwd_ms = hlb.hlb_stats(sim.ctx)["kernel_ms"]
    sim.close()
    bps = 5 * 19 * 8 + 2 * info["table_bytes_per_site"] + 16 + 4 + 4
    gbs = lambda ms: bps * info["n_sites"] / (ms * 1e-3) / 1e9
    c4_ms = (500 * in_ms + 2500 * out_ms) / 3000  # the protocol's window: the last 500 of 3000 steps
    return {"steps": n, "snapshots": n_snap, "window": [n // 2, n], "forward_steps": fw, "wall_s": round(wall, 3),
            "reverse_step_ms": round(adj_ms, 4), "bytes_per_site": round(bps, 2),
            "achieved_gbs": round(gbs(adj_ms), 1), "frac": round(gbs(adj_ms) / PEAK_GBS, 4),
            "reverse_mlups": round(info["n_sites"] / adj_ms / 1e3, 1),
            "reverse_step_in_window_ms": round(in_ms, 4), "frac_in_window": round(gbs(in_ms) / PEAK_GBS, 4),
            "reverse_step_outside_window_ms": round(out_ms, 4),
            "frac_outside_window": round(gbs(out_ms) / PEAK_GBS, 4),
            "reverse_step_ms_window_last_sixth": round(c4_ms, 4),
            "frac_window_last_sixth": round(gbs(c4_ms) / PEAK_GBS, 4),
            "forward_step_ms": round(fwd_ms, 4), "J": J}


def copy_ceiling(nbytes=4 << 30, reps=20):
    """A plain HIP device-to-device copy (in libhlb): the practical HBM ceiling."""
    from paper_2202_11770_amd import hlb
    return hlb.hlb_copy_bandwidth(nbytes, reps)


def error_subtree(target=2_000_000):
    """The error subtree of the 2e8-site tree: cut from the segment list at
    the 2e8 tree's lattice spacing, so the full tree is never voxelised for
    it.  Its Ladd inlet takes the benchmark's A(s), its leaves rho = 1."""
    import numpy as np
    from paper_2202_11770_amd import geometry as G
    seg = G.tree_segments(2, 8, scale=TREE_SCALE_200M, origin=(0.5, 0.5, -0.5))
    sub = G.subtree(segments=seg, scale=TREE_SCALE_200M, target_sites=target)
    tabs = [inlet_table() if io.kind == G.VELOCITY else np.array([1.0]) for io in sub.iolets]
    return sub, tabs


def errors_vs_oracle(storages, tau, steps=1000):
    """Every storage against the FP64 oracle on the error subtree, every site
    after `steps` steps from rest.  The oracle run is timed: it is the CPU
    baseline (a bounded sample of the workload's own geometry)."""
    import numpy as np
    import oracle
    from paper_2202_11770_amd import hlb
    sub, tabs = error_subtree()
    log(f"error subtree: {sub.n} sites, {len(sub.iolets)} iolets; oracle {steps} steps")
    P = oracle.Problem(sub, tau, tables=tabs)
    f = P.init()
    t0 = time.perf_counter()
    P.run(f, 0, steps)
    dt = time.perf_counter() - t0
    rr, ur, wr = P.macros(f)
    cores = oracle.threads()
    cpu = {"value": round(sub.n * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
           "sample": f"{steps} steps from rest of the {sub.n}-site error subtree of the 2e8-site tree (same "
                     f"lattice spacing and physics), FP64 AoS push oracle, OpenMP over {cores} threads; "
                     f"the run that the storages' errors are measured against"}
    log(f"oracle: {cpu['value']} MLUPS over {dt:.1f}s")
    un = np.linalg.norm(ur, axis=1).max()
    out = {"case": f"error subtree of the 2e8-site tree, {sub.n} sites, {steps} steps from rest",
           "n_sites": int(sub.n), "steps": steps,
           "metrics": "e_rho = max|rho - rho_ref| / rho0; e_u = max|u - u_ref| / max|u_ref|; "
                      "e_wss = max|wss - wss_ref| / max wss_ref; rms_u the RMS of |u - u_ref| / max|u_ref|"}
    for st in storages:
        sim = hlb.Simulation.create(sub, tau, storage=st, tables=tabs)
        sim.step(steps)
        rho, u, wss = sim.macros()
        sim.close()
        du = np.linalg.norm(u - ur, axis=1)
        e = {"e_rho": float(np.abs(rho - rr).max()), "e_u": float(du.max() / un),
             "e_wss": float(np.abs(wss - wr).max() / wr.max()),
             "rms_u": float(np.sqrt(np.mean(du ** 2)) / un)}
        out[st] = {k: float(f"{v:.3g}") for k, v in e.items()}
        log(f"{st} vs oracle on the subtree: {out[st]}")
    return out, cpu


def cpu_baseline(g, tables, tau, budget_s=15.0):
    import oracle
    P = oracle.Problem(g, tau, tables=tables)
    f = P.init()
    t0 = time.perf_counter()
    P.run(f, 0, 1)
    one = time.perf_counter() - t0
    k = max(1, min(50, int(budget_s / max(one, 1e-3))))
    t0 = time.perf_counter()
    P.run(f, 1, k)
    dt = time.perf_counter() - t0
    cores = oracle.threads()
    return {"value": round(g.n * k / dt / 1e6, 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{k} steps (after 1 untimed) of the full {g.n}-site tree, FP64, AoS push oracle, "
                      f"OpenMP over {cores} threads"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="tree200m", choices=sorted(WORKLOADS))
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--storages", default=None)
    ap.add_argument("--order", default=None, help="site order of the timed runs (default: the library's)")
    ap.add_argument("--order-block", type=int, default=0, help="log2 band/column width of the bands/columns orders")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-copy", action="store_true")
    ap.add_argument("--schemes", default="pull",
                    help="update orders to time: pull (the headline), and push for the A/B")
    ap.add_argument("--sites-per-thread", default="0",
                    help="bulk sites per GPU thread, comma-separated: the first value is timed as the headline "
                         "(0: the library's default per storage), the others as an A/B")
    ap.add_argument("--adjoint", action="store_true",
                    help="also time the adjoint's reverse step on the workload (FP64)")
    ap.add_argument("--oracle-table", action="store_true",
                    help="also time the oracle (all threads and one) beside the GPU on four configurations")
    ap.add_argument("--windkessel", action="store_true",
                    help="also time the workload with every pressure outlet a three-element Windkessel")
    ap.add_argument("--split-one", default=None, help=argparse.SUPPRESS)  # storage,exchange,parts (run_split_fresh)
    ap.add_argument("--split", type=int, default=0,
                    help="also time the workload as this many partitions with the halo exchange (one GPU)")
    ap.add_argument("--compare-steps", type=int, default=None,
                    help="run every storage for this many steps from rest and report the FP32/FP16 errors "
                         "against the FP64 GPU run (default: 1000 on tree200m, else 0)")
    ap.add_argument("--error-steps", type=int, default=None,
                    help="steps of the per-storage comparison with the oracle on the error subtree "
                         "(default: 1000 on tree200m, else 0)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "decomposition is a design, not an implementation", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(int(os.environ.get("LOCAL_RANK", "0")))
    tau, def_steps, def_storages, desc = WORKLOADS[args.workload]
    if args.split_one:
        st, ex, nparts = args.split_one.split(",")
        g, tables = workload(args.workload)
        print(json.dumps(run_split(g, tables, tau, st, args.steps or def_steps, args.warmup, int(nparts), exchange=ex)))
        return
    args.steps = args.steps or def_steps
    args.storages = args.storages or def_storages
    global ORDER
    if args.order:
        ORDER = (args.order, args.order_block)
    big = args.workload == "tree200m"
    if args.compare_steps is None:
        args.compare_steps = 1000 if big else 0
    if args.error_steps is None:
        args.error_steps = 1000 if big else 0
    t0 = time.time()
    g, tables = workload(args.workload)
    log(f"workload: {args.workload}: {g.n} sites, {len(g.iolets)} iolets, fill {g.meta['fill']:.4f}, "
        f"generated in {time.time() - t0:.1f}s")
    spts = [int(x) for x in args.sites_per_thread.split(",") if x]
    results = {}
    for st in args.storages.split(","):
        t1 = time.time()
        results[st] = run_storage(g, tables, tau, st, args.steps, args.warmup, sites_per_thread=spts[0])
        r = results[st]
        log(f"{st}: {r['mlups']:.0f} MLUPS, {r['ms_per_step']:.3f} ms/step, step kernel {r['kernel_ms']:.3f} ms "
            f"= {r['kernel_gbs']:.0f} GB/s ({100 * r['frac']:.1f}% of 8 TB/s), mass residual {r['mass_residual_rel']:.2e} "
            f"({time.time() - t1:.1f}s)")
    main_st = args.storages.split(",")[0]
    R = results[main_st]
    ab = {}
    for sch in [x for x in args.schemes.split(",") if x and x != "pull"]:
        ab[sch] = {}
        for st in args.storages.split(","):
            r = run_storage(g, tables, tau, st, args.steps, args.warmup, scheme=sch)
            ab[sch][st] = {"mlups": round(r["mlups"], 1), "kernel_ms": round(r["kernel_ms"], 5),
                           "kernel_gbs": round(r["kernel_gbs"], 1), "frac": round(r["frac"], 4),
                           "vs_pull": round(r["mlups"] / results[st]["mlups"], 3),
                           "mass_residual_rel": r["mass_residual_rel"]}
            log(f"{sch} {st}: {r['mlups']:.0f} MLUPS, step kernel {r['kernel_ms']:.3f} ms = {r['kernel_gbs']:.0f} GB/s "
                f"({100 * r['frac']:.1f}%), {ab[sch][st]['vs_pull']:.3f}x pull")
    spt_ab = {}
    for spt in spts[1:]:
        spt_ab[str(spt)] = {}
        for st in args.storages.split(","):
            r = run_storage(g, tables, tau, st, args.steps, args.warmup, sites_per_thread=spt)
            spt_ab[str(spt)][st] = {"mlups": round(r["mlups"], 1), "kernel_ms": round(r["kernel_ms"], 5),
                                    "kernel_gbs": round(r["kernel_gbs"], 1), "frac": round(r["frac"], 4),
                                    "vs_headline": round(r["mlups"] / results[st]["mlups"], 3)}
            log(f"sites_per_thread {spt} {st}: {r['mlups']:.0f} MLUPS, step kernel {r['kernel_ms']:.3f} ms = "
                f"{r['kernel_gbs']:.0f} GB/s ({100 * r['frac']:.1f}%), {spt_ab[str(spt)][st]['vs_headline']:.3f}x")
    copy_gbs = None if args.no_copy else round(copy_ceiling(), 1)
    if copy_gbs:
        log(f"plain copy: {copy_gbs:.0f} GB/s")
    cpu = None
    err_or = None
    if args.error_steps > 0:
        err_or, cpu_sub = errors_vs_oracle(args.storages.split(","), tau, args.error_steps)
        if not args.no_cpu_baseline:
            cpu = cpu_sub
    if cpu is None and not args.no_cpu_baseline and args.workload == "tree20m":
        cpu = cpu_baseline(g, tables, tau)
    if cpu is not None:
        log(f"cpu baseline: {cpu}")
    adj = None
    if args.adjoint:
        adj = run_adjoint(g, tables, tau)
        log(f"adjoint: {adj}")
    otab = None
    if args.oracle_table:
        otab = oracle_table(g, tables)
    wk = {}
    if args.windkessel:
        from paper_2202_11770_amd import geometry as G
        models = {k: (1.0, 0.01, 2000.0, 0.02, 0.0) for k, io in enumerate(g.iolets) if io.kind == G.PRESSURE}
        for st in args.storages.split(","):
            r = run_storage(g, tables, tau, st, args.steps, args.warmup, windkessel=models)
            wk[st] = {"outlets": len(models), "mlups": round(r["mlups"], 1), "ms_per_step": round(r["ms_per_step"], 4),
                      "overhead_vs_fixed": round(results[st]["mlups"] / r["mlups"] - 1.0, 4)}
            log(f"windkessel {st}: {wk[st]}")
    split = {}
    if args.split > 1:
        for st in args.storages.split(","):
            split[st] = {}
            for ex in ("direct", "copy"):
                r = run_split_fresh(args.workload, st, args.steps, args.warmup, args.split, ex)
                r["overhead_vs_single"] = round(results[st]["mlups"] / r["mlups"] - 1.0, 4)
                split[st][ex] = r
                log(f"split {st}: {r}")
    compare = None
    if args.compare_steps > 0:
        compare = compare_storages(g, tables, tau, args.storages.split(","), args.compare_steps)
    traffic = stored_traffic(main_st, R["n_sites"], order_tag(R["order"], R["order_block"]))
    out = {
        "metric": "MLUPS & achieved HBM GB/s, FP64 vs FP32/FP16 storage at stated error",
        "value": round(R["mlups"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(R["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32-storage", "f16": "f16-storage"}[main_st],
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}; {g.n} fluid sites, tau {tau}, storage {main_st}",
                   "n_sites": g.n, "storage": main_st, "order": R["order"], "order_block": R["order_block"],
                   "xcd_remap": R["xcd_remap"],
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(R["kernel_gbs"], 1), "peak": PEAK_GBS, "unit": "GB/s",
                     "frac": round(R["frac"], 4), "traffic": traffic,
                     "kernel": "k_step (all site groups, one launch per step)",
                     "bytes_per_site": R["bytes_per_lup"], "sites_per_launch": R["n_sites"],
                     "mean_launch_ms": round(R["kernel_ms"], 5)},
        "cpu_baseline": cpu,
        "copy_ceiling_gbs": copy_gbs,
        "storages": {k: {"mlups": round(v["mlups"], 1), "ms_per_step": round(v["ms_per_step"], 4),
                         "kernel_ms": round(v["kernel_ms"], 5),
                         "kernel_gbs": round(v["kernel_gbs"], 1), "frac": round(v["frac"], 4),
                         "bytes_per_lup": v["bytes_per_lup"],
                         "gain_vs_f64": round(v["mlups"] / results[main_st]["mlups"], 3),
                         "mass_residual_rel": v["mass_residual_rel"]} for k, v in results.items()},
    }
    if err_or is not None:
        out["errors_vs_oracle"] = err_or
    if compare is not None:
        out["errors_vs_f64_gpu"] = {"case": f"the full {g.n}-site workload, every site", "steps": args.compare_steps,
                                    **compare}
    if ab:
        out["schemes"] = ab
    if spt_ab:
        out["sites_per_thread_ab"] = spt_ab
    if split:
        out["split"] = split
    if wk:
        out["windkessel"] = wk
    if otab:
        out["oracle_table"] = otab
    if adj:
        out["adjoint"] = adj
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
