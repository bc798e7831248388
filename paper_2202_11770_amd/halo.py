"""One-GPU emulation of the domain split (Sec. 3.1's edge / mid-domain
update with the halo exchange of Sec. 3.2.3), on the pull update.

``partition(geom, nparts)`` cuts a geometry's site list into ``nparts`` slabs
of about equal site counts along z (whole planes) and builds, per part, the
input of ``hlb_create_part``: its owned sites, then ghost copies of the other
parts' sites its owned sites pull from; roles (MID / EDGE / GHOST); and the
exchange lists.  Element (z, i) -- population i of site z after collision --
travels from z's part to the part of the site at z + c_i whenever the two
differ; every list is ordered by (global site, direction), so sender and
receiver agree without negotiation.

``SplitSimulation`` runs one context per part on one GPU, each on its own
stream.  Per step every part updates its edge sites (``hlb_step_edge``) and
then its mid-domain sites (``hlb_step_mid``), which overlap the exchange.
With the direct exchange the mid step runs on a second stream of its part
(``hlb_set_mid_stream``), so that it also overlaps the part's edge step: a
part's edge step waits for its previous mid step (which wrote sites the
edge step reads, and read the buffer it writes), and its mid step for its
previous edge step.  Two exchanges are built:

* ``exchange="direct"`` (default): the edge step writes each exchanged
  value straight into the ghost slot of the peer's population buffer that
  the peer's next step pulls from (``hlb_halo_ghost_slots``,
  ``hlb_halo_add_peer``): no receive buffer, no transfer, no unpack.  A
  part's edge step waits only for its peers' previous edge steps (the last
  readers of the ghost slots it overwrites, and the writers of the ones it
  reads).  Between GPUs the peer buffer would be mapped over xGMI.
* ``exchange="copy"``: the edge step packs into a send buffer, a device copy
  on a transfer stream moves it into the peer's receive buffer, and the
  peer unpacks it into its ghost slots after its mid-domain update (the
  shape of an RCCL send/recv of the same buffers).

All of the update, pack and unpack runs in libhlb; torch provides the
buffers, streams and events.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import hlb

Q = 19


@dataclass
class Part:
    coords: np.ndarray        # [n_local, 3]
    types: np.ndarray         # [n_local]
    nbr: np.ndarray           # [n_local, 19] local ids
    iolets: list
    role: np.ndarray          # [n_local] HLB_PART_*
    glob: np.ndarray          # [n_local] global id of each local site
    n_owned: int
    send: dict = field(default_factory=dict)  # peer -> (local sites, directions)
    recv: dict = field(default_factory=dict)  # peer -> (local sites, directions)


def partition(geom, nparts: int = 2):
    coords, nbr, types = geom.coords, geom.nbr, geom.types
    n = coords.shape[0]
    z = coords[:, 2]
    zs = np.sort(z, kind="stable")
    cuts = np.array([zs[(k * n) // nparts] for k in range(1, nparts)])
    owner = np.searchsorted(cuts, z, side="right").astype(np.int32)
    # exchanged elements: (site z, direction i) with the site at z + c_i in
    # another part, which pulls population i of z
    zz, ii = np.nonzero(nbr[:, 1:] >= 0)
    ii = ii + 1
    xx = nbr[zz, ii]
    cross = owner[xx] != owner[zz]
    zz, ii, xx = zz[cross], ii[cross], xx[cross]
    src, dst = owner[zz], owner[xx]
    key = zz.astype(np.int64) * Q + ii
    o = np.argsort(key, kind="stable")
    zz, ii, src, dst = zz[o], ii[o], src[o], dst[o]
    parts = []
    for r in range(nparts):
        owned = np.nonzero(owner == r)[0]
        ghosts = np.unique(zz[dst == r])
        glob = np.concatenate([owned, ghosts])
        local = np.full(n, -1, dtype=np.int64)
        local[glob] = np.arange(glob.size)
        nl = glob.size
        nb = np.full((nl, Q), hlb.HLB_LINK_WALL, dtype=np.int32)
        on = nbr[owned]
        mapped = np.where(on >= 0, local[np.maximum(on, 0)], on)
        if np.any((on >= 0) & (mapped < 0)):
            raise AssertionError("an owned site links to a site that is neither owned nor a ghost")
        nb[: owned.size] = mapped
        nb[owned.size:, 0] = np.arange(owned.size, nl)
        role = np.full(nl, hlb.HLB_PART_MID, dtype=np.uint8)
        role[owned.size:] = hlb.HLB_PART_GHOST
        sends = zz[src == r]
        role[local[np.unique(sends)]] = hlb.HLB_PART_EDGE
        P = Part(coords=coords[glob], types=types[glob], nbr=nb, iolets=list(geom.iolets), role=role, glob=glob,
                 n_owned=int(owned.size))
        for q in range(nparts):
            if q == r:
                continue
            m = (src == r) & (dst == q)
            if m.any():
                P.send[q] = (local[zz[m]].astype(np.int32), ii[m].astype(np.int32))
            m = (src == q) & (dst == r)
            if m.any():
                P.recv[q] = (local[zz[m]].astype(np.int32), ii[m].astype(np.int32))
        parts.append(P)
    return parts


_DTYPE = {"f64": "float64", "f32": "float32", "f16": "float16"}

# Per part index, the part's two streams (its update stream, and the mid step's
# stream of the direct exchange or the transfer stream of the copy exchange),
# shared by every SplitSimulation of the process.  The GPU maps streams onto
# a few hardware queues, and two streams that share one serialise: with new
# streams per simulation the second simulation of a process measured up to
# 40% slower than the first.  With these streams a repeated run of one
# exchange runs as the first; a copy-exchange run after a direct-exchange
# run of the same process still measured 33% slower (its transfer stream
# was the mid stream before), so measurements start a process per run.
_STREAMS = []


def _part_streams(torch, r):
    while len(_STREAMS) <= r:
        _STREAMS.append((torch.cuda.Stream(), torch.cuda.Stream()))
    return _STREAMS[r]


class SplitSimulation:
    """One context per part on one GPU; see the module docstring."""

    def __init__(self, geom, tau: float, storage: str = "f64", tables=None, nparts: int = 2, xcd_remap: int = -1,
                 shared_stream: bool = False, exchange: str = "direct"):
        """shared_stream: all parts' updates on one stream (their kernels run
        back to back) instead of one stream per part (they may overlap); the
        transfers of the copy exchange have their own streams either way.
        exchange: "direct" or "copy" (module docstring)."""
        import torch
        if exchange not in ("direct", "copy"):
            raise ValueError(f"exchange must be 'direct' or 'copy', not {exchange!r}")
        self.torch = torch
        self.direct = exchange == "direct"
        self.n = int(geom.types.shape[0])
        self.parts = partition(geom, nparts)
        dt = getattr(torch, _DTYPE[storage])
        opt = hlb.hlb_default_options()
        opt.storage = hlb.STORAGE[storage]
        opt.xcd_remap = int(xcd_remap)
        self.ctx, self.s, self.m, self.c, self.send, self.recv = [], [], [], [], [], []
        common = torch.cuda.Stream() if shared_stream else None
        self.send_slice, self.recv_slice = [], []
        for P in self.parts:
            ctx = hlb.hlb_create_part(P.coords, P.types, P.nbr, tau, P.iolets, P.role, opt)
            for k, io in enumerate(P.iolets):
                tab = tables[k] if tables is not None and tables[k] is not None else getattr(io, "table", None)
                if tab is not None:
                    hlb.hlb_set_iolet_table(ctx, k, tab)
            peers_s = sorted(P.send)
            peers_r = sorted(P.recv)
            ss = np.concatenate([P.send[q][0] for q in peers_s]) if peers_s else np.zeros(0, np.int32)
            sd = np.concatenate([P.send[q][1] for q in peers_s]) if peers_s else np.zeros(0, np.int32)
            rs = np.concatenate([P.recv[q][0] for q in peers_r]) if peers_r else np.zeros(0, np.int32)
            rd = np.concatenate([P.recv[q][1] for q in peers_r]) if peers_r else np.zeros(0, np.int32)
            if self.direct:  # no buffers: the peers are wired below
                sb = torch.empty(0, dtype=dt, device="cuda")
                rb = torch.empty(0, dtype=dt, device="cuda")
            else:
                sb = torch.empty(max(ss.size, 1), dtype=dt, device="cuda")
                rb = torch.empty(max(rs.size, 1), dtype=dt, device="cuda")
                hlb.hlb_halo_set(ctx, ss, sd, sb, rs, rd, rb)
            off, sl = 0, {}
            for q in peers_s:
                sl[q] = slice(off, off + P.send[q][0].size)
                off += P.send[q][0].size
            self.send_slice.append(sl)
            off, sl = 0, {}
            for q in peers_r:
                sl[q] = slice(off, off + P.recv[q][0].size)
                off += P.recv[q][0].size
            self.recv_slice.append(sl)
            s, x = _part_streams(torch, len(self.ctx))
            if common is not None:
                s = common
            hlb.hlb_set_stream(ctx, s.cuda_stream)
            m = None
            if common is None and self.direct:
                m = x
                hlb.hlb_set_mid_stream(ctx, m.cuda_stream)
            self.ctx.append(ctx)
            self.s.append(s)
            self.m.append(m)
            self.c.append(None if self.direct else x)
            self.send.append(sb)
            self.recv.append(rb)
        self.unpacked = [None] * len(self.parts)
        # direct exchange: each part writes its send list into the peers'
        # ghost slots; the peer's receive list names the same (site,
        # direction) pairs in the same order
        self.nb = [sorted(set(P.send) | set(P.recv)) for P in self.parts]
        if self.direct:
            for r, P in enumerate(self.parts):
                for q in sorted(P.send):
                    sites, dirs = P.send[q]
                    rs, rd = self.parts[q].recv[r]
                    elem, bufs = hlb.hlb_halo_ghost_slots(self.ctx[q], rs, rd)
                    hlb.hlb_halo_add_peer(self.ctx[r], sites, dirs, bufs[0], bufs[1], elem)
        self.edge_done = [None] * len(self.parts)
        self.mid_done = [None] * len(self.parts)  # each part's last mid step (mid stream)
        self.exchange()

    def _transfer(self, packed):
        """Move every part's received values; returns the per-part 'arrived' events."""
        torch = self.torch
        arrived = []
        for r in range(len(self.parts)):
            with torch.cuda.stream(self.c[r]):
                for q in self.recv_slice[r]:
                    self.c[r].wait_event(packed[q])
                if self.unpacked[r] is not None:
                    self.c[r].wait_event(self.unpacked[r])  # the last unpack has read recv[r]
                for q, sl in self.recv_slice[r].items():
                    self.recv[r][sl].copy_(self.send[q][self.send_slice[q][r]])
                e = torch.cuda.Event()
                e.record(self.c[r])
            arrived.append(e)
        return arrived

    def _unpack(self, arrived):
        torch = self.torch
        for r, ctx in enumerate(self.ctx):
            self.s[r].wait_event(arrived[r])
            for q in self.send_slice[r]:
                self.s[r].wait_event(arrived[q])  # peers have copied send[r]: it may be overwritten
            hlb.hlb_halo_unpack(ctx)
            e = torch.cuda.Event()
            e.record(self.s[r])
            self.unpacked[r] = e

    def _join(self):
        """Order later work on each part's stream after its mid steps."""
        for s, m in zip(self.s, self.m):
            if m is not None:
                s.wait_stream(m)

    def exchange(self):
        """Fill every ghost from its owner's current state (after creation,
        init or set_state)."""
        torch = self.torch
        self._join()
        if self.direct:
            torch.cuda.synchronize()  # every part's state is settled before any peer writes its ghosts
            for r, ctx in enumerate(self.ctx):
                hlb.hlb_halo_pack(ctx)
                e = torch.cuda.Event()
                e.record(self.s[r])
                self.edge_done[r] = e
            return
        packed = []
        for r, ctx in enumerate(self.ctx):
            hlb.hlb_halo_pack(ctx)
            e = torch.cuda.Event()
            e.record(self.s[r])
            packed.append(e)
        self._unpack(self._transfer(packed))

    def init_equilibrium(self, rho=None, u=None, t0: int = 0):
        """Every part to f^eq(rho, u) (global [n] and [n][3] host arrays, or
        None for rest) at time t0, then the ghosts from their owners."""
        self.synchronize()
        for P, ctx in zip(self.parts, self.ctx):
            r = None if rho is None else np.ascontiguousarray(np.asarray(rho, np.float64)[P.glob])
            v = None if u is None else np.ascontiguousarray(np.asarray(u, np.float64)[P.glob])
            hlb.hlb_init_equilibrium(ctx, r, v, t0)
        self.exchange()

    def step(self, n: int = 1):
        torch = self.torch
        if self.direct:
            for _ in range(n):
                done, before = [], []
                for r, ctx in enumerate(self.ctx):
                    m = self.m[r]
                    if m is not None:
                        # everything on the part's stream so far (its previous
                        # edge step and exchange, any set-up), recorded before
                        # the wait on the previous mid step, so that the next
                        # mid step does not wait for it a second time through
                        # this stream
                        e = torch.cuda.Event()
                        e.record(self.s[r])
                        before.append(e)
                        if self.mid_done[r] is not None:
                            self.s[r].wait_event(self.mid_done[r])
                    else:
                        before.append(None)
                    # the peers' previous edge steps wrote the ghosts this one
                    # reads and were the last to read the ghosts it writes
                    for q in self.nb[r]:
                        self.s[r].wait_event(self.edge_done[q])
                    hlb.hlb_step_edge(ctx)
                    e = torch.cuda.Event()
                    e.record(self.s[r])
                    done.append(e)
                for r, ctx in enumerate(self.ctx):
                    m = self.m[r]
                    if m is not None:
                        m.wait_event(before[r])
                    hlb.hlb_step_mid(ctx)
                    if m is not None:
                        e = torch.cuda.Event()
                        e.record(m)
                        self.mid_done[r] = e
                self.edge_done = done
            return
        for _ in range(n):
            packed = []
            for r, ctx in enumerate(self.ctx):
                hlb.hlb_step_edge(ctx)
                e = torch.cuda.Event()
                e.record(self.s[r])
                packed.append(e)
            arrived = self._transfer(packed)
            for ctx in self.ctx:
                hlb.hlb_step_mid(ctx)
            self._unpack(arrived)

    def synchronize(self):
        self.torch.cuda.synchronize()

    def macros(self):
        self._join()
        rho = np.empty(self.n)
        u = np.empty((self.n, 3))
        wss = np.empty(self.n)
        for P, ctx in zip(self.parts, self.ctx):
            r, v, w = hlb.hlb_macros(ctx)
            o = P.glob[: P.n_owned]
            rho[o], u[o], wss[o] = r[: P.n_owned], v[: P.n_owned], w[: P.n_owned]
        return rho, u, wss

    def mass(self) -> float:
        self._join()
        return float(sum(hlb.hlb_mass_balance(ctx)[0] for ctx in self.ctx))

    def close(self):
        self.synchronize()
        for ctx in self.ctx:
            hlb.hlb_destroy(ctx)
        self.ctx = []
