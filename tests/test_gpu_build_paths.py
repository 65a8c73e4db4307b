"""Build paths that the workload generators never reach, checked on the GPU.

* Adjacency segments of more than 4096 entries (sorted in global memory by a radix sort): the
  complete graph K_4100, whose lowest-ranked nodes own out-lists of 4099, 4098 and 4097 entries,
  and a clique with one extra node adjacent to 4098 of it.  Their counts at m = c = 1 are closed
  forms (every triangle is counted once); at m = 10 windows of the stream are checked against the
  oracle's per-edge updates.  A repeated pair inside such a segment is EDUP (Section II: the
  stream is a simple graph).
* Node ids spread over [0, 2^26) (more than 2^25 ids: the build places entries with global
  cursors instead of per-slice LDS cursors), counted against the oracle.
"""
from math import comb

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def _clique_plus_hub(k: int, spokes: int) -> np.ndarray:
    """Nodes 1..k form a clique; node 0 is joined to nodes 1..spokes (spokes < k).  Node 0 has the
    lowest rank (its degree `spokes` is below every clique node's), so its out-list holds all of
    its `spokes` edges."""
    cl = synth.complete(k) + 1
    hub = np.stack([np.zeros(spokes, np.uint32), np.arange(1, spokes + 1, dtype=np.uint32)], axis=1)
    return np.concatenate([hub, cl]).astype(np.uint32)


@pytest.mark.timeout(300)
def test_complete_graph_with_segments_over_4096(cuda):
    import torch
    from paper_1811_09136_amd import rept
    n = 4100
    e = synth.shuffled(synth.complete(n), 41, flip_seed=42)
    _say(f"K_{n}: {len(e)} edges, build")
    g = rept.Graph(rept.to_device_edges(e, cuda), n)
    assert g.info.max_out_degree == n - 1  # node 0's list: all of its neighbours
    _say(f"K_{n}: m = c = 1 count")
    glob, loc = g.count(rept.Params(1, 1, 7))
    torch.cuda.synchronize()
    assert int(glob[0]) == comb(n, 3)
    assert torch.all(loc[0] == comb(n - 1, 2)).item()
    # m = 10, two groups: the last stream edges, against the oracle's per-edge updates
    P = rept.Params(10, 20, 11)
    E = len(e)
    out = g.outputs(P)
    out[0].zero_()
    out[1].zero_()
    t0 = E - 400
    _say(f"K_{n}: m = 10, c = 20, window [{t0}, {E})")
    g.count_range(P, t0, E, out)
    torch.cuda.synchronize()
    og, ol = oracle.edge_updates(e, n, 10, 20, 11, np.arange(t0, E))
    assert og.sum() > 0
    assert np.array_equal(out[0].cpu().numpy(), og)
    assert np.array_equal(out[1].cpu().numpy(), ol)
    g.close()


@pytest.mark.timeout(300)
def test_hub_segment_over_4096_closed_form_and_duplicate(cuda):
    import torch
    from paper_1811_09136_amd import rept
    k, spokes = 4100, 4098
    n = k + 1
    e = synth.shuffled(_clique_plus_hub(k, spokes), 43, flip_seed=44)
    _say(f"clique K_{k} + node of degree {spokes}: {len(e)} edges")
    g = rept.Graph(rept.to_device_edges(e, cuda), n)
    glob, loc = g.count(rept.Params(1, 1, 3))
    torch.cuda.synchronize()
    # triangles: those of the clique, and node 0 with any two of its (pairwise adjacent) neighbours
    assert int(glob[0]) == comb(k, 3) + comb(spokes, 2)
    lo = loc[0].cpu().numpy()
    assert lo[0] == comb(spokes, 2)
    assert np.all(lo[1:spokes + 1] == comb(k - 1, 2) + spokes - 1)
    assert np.all(lo[spokes + 1:] == comb(k - 1, 2))
    g.close()
    # the same stream with one hub edge repeated (reversed, in the middle of the stream): node 0's
    # segment of 4099 entries then holds the pair twice
    for where in (len(e) // 2, len(e)):
        dup = np.insert(e, where, np.array([[1, 0]], np.uint32), axis=0)
        assert oracle.validate(n, dup) == oracle.EDUP
        _say(f"duplicate hub edge at t = {where}")
        with pytest.raises(rept.ReptError) as ei:
            rept.Graph(rept.to_device_edges(dup, cuda), n)
        assert ei.value.code == rept.REPT_EDUP


@pytest.mark.timeout(300)
def test_ids_spread_over_two_to_the_26(cuda):
    import torch
    from paper_1811_09136_amd import rept
    e0, n0 = synth.scaled_chung_lu(150_000, 61)
    n = 1 << 26
    # an injective spread of the node ids: x -> (a x + b) mod 2^26 with a odd
    a, b = 40_503 * 2 + 1, 12_345_678
    ids = ((a * np.arange(n0, dtype=np.uint64) + b) % n).astype(np.uint32)
    e = ids[e0]
    for m, c, per_proc in [(4, 8, False), (3, 3, True)]:
        P = rept.Params(m, c, 21 + m, per_proc=per_proc)
        _say(f"n = 2^26, E = {len(e)}, m = {m}, c = {c}, per_proc = {per_proc}")
        g = rept.Graph(rept.to_device_edges(e, cuda), n)
        glob, loc = g.count(P)
        torch.cuda.synchronize()
        og, ol = oracle.rept_threads(e, n, m, c, P.seed, per_proc=per_proc, workers=4)
        assert og.sum() > 0
        assert np.array_equal(glob.cpu().numpy(), og)
        assert np.array_equal(loc.cpu().numpy(), ol)
        g.close()
        del glob, loc, og, ol
