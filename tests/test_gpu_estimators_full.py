"""The TRK and RTB estimators at the bench workload's full size
(mid-chunglu-n50k: n = 50,000, |E| = 2,000,000, bursty ticks), on outputs the
oracle can give one by one and on properties that hold at any size.

TRK (pairs 0..7 of the bench's pair stream): records equal the oracle's pair
records; the drawn walk is a chain of temporal edges from s to z at strictly
increasing times, every edge and internal node of it lies on an optimal walk
(its oracle count N is positive), it has one internal visit fewer than edges
(at most that for fm, whose walks may pass through s or z again), and for sh
and sfm exactly the pair's hop count of edges.

RTB (the first sources of the same stream): the reached-target count equals
the number of nodes the oracle's distances reach (fm sources, whose walk
counts over the whole span pass 2^64, are void: flagged, with no f); for sh
and sfm, where every optimal walk to z has d(s, z) hops,
(n - 1) * sum_v f(v|s) equals sum_z (d(s, z) - 1) and (n - 1) * sum_e f(e|s)
equals sum_z d(s, z).
"""
import numpy as np
import pytest

import oracle
from oracle import distances as odist
from synthgen import workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mid(request):
    import torch
    assert torch.cuda.is_available(), "GPU tests need the MI355X"
    import paper_2304_08356_amd as pk
    G = workload("mid-chunglu-n50k")
    return G, pk.Graph.of(G), oracle.Graph.of(G)


@pytest.mark.parametrize("opt", ["sh", "fm", "sfm", "pfm"])
def test_trk_walks_full_size(mid, opt):
    G, gg, og = mid
    S, Z = oracle.draw_pairs(2002, oracle.STREAM_PAIR, G.n, 0, 8)
    rec, nf, ef = gg.sample_paths(opt, S, Z, seed=2002)
    for q in range(len(S)):
        s, z = int(S[q]), int(Z[q])
        want, nN, eN = oracle.pair(og, opt, s, z, mode=1)
        c = (opt, q, s, z)
        assert (int(rec["reachable"][q]), int(rec["t_arr"][q]), int(rec["hops"][q]), int(rec["sigma"][q])) == (
            want["reachable"], want["t_arr"], want["hops"], want["sigma"]), (c, rec[q], want)
        assert int(rec["flags"][q]) & 2 == 0, c
        if not want["reachable"] or int(rec["flags"][q]) & 1:
            assert not nf[q].any() and not ef[q].any(), c
            continue
        used = np.nonzero(ef[q])[0]
        assert np.all(ef[q][used] == 1.0), c  # strictly increasing times: no edge twice
        order = used[np.argsort(G.t[used], kind="stable")]
        src, dst, t = G.src[order], G.dst[order], G.t[order]
        assert src[0] == s and dst[-1] == z, c
        assert np.all(dst[:-1] == src[1:]) and np.all(np.diff(t) > 0), c
        assert np.all(eN[used] > 0), c
        visited = np.nonzero(nf[q])[0]
        assert np.all(nN[visited] > 0), c
        if opt == "fm":
            # a foremost walk may pass through s or z again, which are not counted
            assert nf[q].sum() <= len(used) - 1, c
        else:
            assert nf[q].sum() == len(used) - 1, c
        if opt in ("sh", "sfm"):
            assert len(used) == want["hops"], c


@pytest.mark.parametrize("opt", ["sh", "fm", "sfm", "pfm"])
def test_rtb_sources_full_size(mid, opt):
    G, gg, og = mid
    S = oracle.draw_pairs(2002, oracle.STREAM_PAIR, G.n, 0, 3)[0]
    rec, nf, ef = gg.source_dependencies(opt, S)
    hops = odist.source_hops(og, opt, S)
    for q, s in enumerate(S):
        d = hops[q][hops[q] >= 0].astype(np.int64)
        c = (opt, q, int(s))
        assert int(rec["flags"][q]) & 2 == 0, c
        if int(rec["flags"][q]) & 1:
            # fm walk counts over the whole span pass 2^64: the source is void
            assert opt == "fm" and not nf[q].any() and not ef[q].any(), c
            continue
        assert int(rec["sigma"][q]) == len(d) and int(rec["reachable"][q]) == (1 if len(d) else 0), c
        if opt in ("sh", "sfm"):
            want_v, want_e = float(np.sum(d - 1)), float(np.sum(d))
            got_v, got_e = nf[q].sum() * (G.n - 1), ef[q].sum() * (G.n - 1)
            assert abs(got_v - want_v) <= 1e-9 * max(want_v, 1.0), (c, got_v, want_v)
            assert abs(got_e - want_e) <= 1e-9 * max(want_e, 1.0), (c, got_e, want_e)
