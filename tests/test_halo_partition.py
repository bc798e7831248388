"""Host logic of the domain split (paper_2202_11770_amd/halo.py): the
partition tables against a brute-force reading of the global neighbour
table (no GPU)."""
import numpy as np
import pytest

from paper_2202_11770_amd import geometry as G
from paper_2202_11770_amd import halo, hlb


@pytest.fixture(scope="module", params=["tree", "cylinder", "tree3"])
def case(request):
    if request.param == "cylinder":
        g, k = G.cylinder(), 2
    elif request.param == "tree":
        g, k = G.tree(seed=3, generations=3, target_sites=30000), 2
    else:
        g, k = G.tree(seed=5, generations=4, target_sites=60000), 3
    return g, halo.partition(g, k)


def test_owned_sets_cover_the_domain(case):
    g, parts = case
    owned = np.concatenate([P.glob[: P.n_owned] for P in parts])
    assert np.array_equal(np.sort(owned), np.arange(g.n))


def test_local_tables(case):
    g, parts = case
    for P in parts:
        n_loc = P.glob.size
        own = P.nbr[: P.n_owned]
        # every fluid link of an owned site maps to the same global site
        m = own >= 0
        gl = np.where(m, P.glob[np.maximum(own, 0)], own)
        assert np.array_equal(gl, g.nbr[P.glob[: P.n_owned]])
        assert np.all(own[m] < n_loc)
        assert np.array_equal(P.nbr[:, 0], np.arange(n_loc))
        assert np.all(P.role[P.n_owned:] == hlb.HLB_PART_GHOST)
        assert np.all(P.role[: P.n_owned] != hlb.HLB_PART_GHOST)


def test_exchange_lists_brute_force(case):
    g, parts = case
    owner = np.empty(g.n, dtype=int)
    for r, P in enumerate(parts):
        owner[P.glob[: P.n_owned]] = r
    want = {}
    for z in range(g.n):
        for i in range(1, 19):
            x = g.nbr[z, i]
            if x >= 0 and owner[x] != owner[z]:
                want.setdefault((owner[z], owner[x]), []).append((z, i))
    for (r, q), elems in want.items():
        s_site, s_dir = parts[r].send[q]
        r_site, r_dir = parts[q].recv[r]
        sent = list(zip(parts[r].glob[s_site].tolist(), s_dir.tolist()))
        got = list(zip(parts[q].glob[r_site].tolist(), r_dir.tolist()))
        assert sent == elems and got == elems
        assert np.all(parts[r].role[s_site] == hlb.HLB_PART_EDGE)
        assert np.all(parts[q].role[r_site] == hlb.HLB_PART_GHOST)
    # exactly the sending sites are edge sites
    for r, P in enumerate(parts):
        senders = set()
        for q, (s_site, _) in P.send.items():
            senders |= set(s_site.tolist())
        assert senders == set(np.nonzero(P.role == hlb.HLB_PART_EDGE)[0].tolist())
        assert set(P.send) == {q for (a, q) in want if a == r}
