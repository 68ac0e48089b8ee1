"""Independent checks of a converted graph.

None of these routines shares code with the oracle or with the HIP path:
brute force over Python sets, a numpy/scipy route, and invariants that
hold at any size (computed with numpy on the host or torch on the device).
"""
from __future__ import annotations

import numpy as np

FIELDS = ("node_ids", "out_offsets", "out_nbrs", "in_offsets", "in_nbrs")


def brute_force(src, dst):
    """Straight from the definition with Python sets and dicts (tiny inputs)."""
    src = [int(x) for x in src]
    dst = [int(x) for x in dst]
    nodes = sorted(set(src) | set(dst))
    pos = {x: i for i, x in enumerate(nodes)}
    edges = sorted({(pos[s], pos[d]) for s, d in zip(src, dst)})
    V = len(nodes)
    out_nbrs = [d for _, d in edges]
    out_offsets = [sum(1 for s, _ in edges if s < v) for v in range(V + 1)]
    tr = sorted((d, s) for s, d in edges)
    in_nbrs = [s for _, s in tr]
    in_offsets = [sum(1 for d, _ in tr if d < v) for v in range(V + 1)]
    return {"node_ids": np.array(nodes, dtype=np.int64), "out_offsets": np.array(out_offsets, dtype=np.int64),
            "out_nbrs": np.array(out_nbrs, dtype=np.int32), "in_offsets": np.array(in_offsets, dtype=np.int64),
            "in_nbrs": np.array(in_nbrs, dtype=np.int32)}


def scipy_route(src, dst):
    """numpy.unique for the node list and positions; scipy.sparse CSR/CSC
    (with duplicates summed and indices sorted) for the two adjacencies."""
    import scipy.sparse as sp
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    nodes, inv = np.unique(np.concatenate([src, dst]), return_inverse=True)
    n = src.size
    V = nodes.size
    s, d = inv[:n], inv[n:]
    m = sp.coo_matrix((np.ones(n, dtype=np.int64), (s, d)), shape=(V, V))
    csr = m.tocsr()
    csr.sum_duplicates()
    csr.sort_indices()
    csc = m.tocsc()
    csc.sum_duplicates()
    csc.sort_indices()
    return {"node_ids": nodes.astype(np.int64), "out_offsets": csr.indptr.astype(np.int64),
            "out_nbrs": csr.indices.astype(np.int32), "in_offsets": csc.indptr.astype(np.int64),
            "in_nbrs": csc.indices.astype(np.int32)}


def as_dict(g):
    if isinstance(g, dict):
        return g
    out = {}
    for f in FIELDS:
        v = getattr(g, f)
        if hasattr(v, "cpu"):
            v = v.cpu().numpy()
        out[f] = np.asarray(v)
    return out


def assert_same(got, want, what=""):
    got, want = as_dict(got), as_dict(want)
    for f in FIELDS:
        a, b = np.asarray(got[f]), np.asarray(want[f])
        assert a.shape == b.shape, f"{what}{f}: shape {a.shape} != {b.shape}"
        if not np.array_equal(a.astype(np.int64), b.astype(np.int64)):
            bad = np.flatnonzero(a.astype(np.int64) != b.astype(np.int64))
            raise AssertionError(f"{what}{f}: {bad.size} mismatches, first at {bad[0]}: {a[bad[0]]} != {b[bad[0]]}")
        assert a.dtype == b.dtype or f in ("node_ids",), f"{what}{f}: dtype {a.dtype} != {b.dtype}"


def check_invariants(g, src, dst):
    """Invariants of the conversion that pin the result completely:
    node list = sorted distinct identifiers; out-lists strictly increasing;
    every row present as an edge; E = number of distinct rows; in-CSR is the
    transpose of out-CSR."""
    g = as_dict(g)
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    nodes = g["node_ids"]
    V = nodes.size
    oo, on, io, inn = g["out_offsets"], g["out_nbrs"].astype(np.int64), g["in_offsets"], g["in_nbrs"].astype(np.int64)
    E = on.size
    assert oo.size == V + 1 and io.size == V + 1
    assert oo[0] == 0 and io[0] == 0 and oo[-1] == E and io[-1] == E and inn.size == E
    assert np.all(np.diff(oo) >= 0) and np.all(np.diff(io) >= 0)
    assert np.all(nodes[1:] > nodes[:-1]), "node ids strictly increasing"
    allv = np.concatenate([src, dst])
    assert V == np.unique(allv).size
    if src.size == 0:
        assert V == 0 and E == 0
        return
    pos = np.searchsorted(nodes, allv)
    assert np.all(pos < V) and np.array_equal(nodes[pos], allv), "every identifier listed"
    # sources of the out-edges
    osrc = np.repeat(np.arange(V, dtype=np.int64), np.diff(oo))
    okey = osrc * V + on
    assert np.all((on >= 0) & (on < V))
    assert np.all(np.diff(okey) > 0), "out-lists strictly increasing, no duplicate edge"
    rkey = pos[:src.size] * V + pos[src.size:]
    assert E == np.unique(rkey).size, "E = distinct rows"
    k = np.searchsorted(okey, rkey)
    assert np.all(k < E) and np.array_equal(okey[k], rkey), "every row is an edge"
    idst = np.repeat(np.arange(V, dtype=np.int64), np.diff(io))
    ikey = idst * V + inn
    assert np.all(np.diff(ikey) > 0), "in-lists strictly increasing"
    assert np.array_equal(np.sort(on * V + osrc), ikey), "in-CSR is the transpose"
    deg = np.diff(oo) + np.diff(io)
    assert np.all(deg >= 1), "no isolated node"


def check_invariants_torch(g, src, dst):
    """Same invariants as check_invariants, with torch on the device (for
    tables too large for the host checks).  Uses only torch's own sort,
    unique and searchsorted.  The library's idle cached blocks go back to
    the device first, for torch's temporaries."""
    import torch
    from paper_1503_07881_amd import ringo
    torch.cuda.synchronize()
    ringo.release_cached()
    nodes = g.node_ids
    V = nodes.numel()
    oo, io = g.out_offsets, g.in_offsets
    on, inn = g.out_nbrs.long(), g.in_nbrs.long()
    E = on.numel()
    assert oo.numel() == V + 1 and io.numel() == V + 1 and inn.numel() == E
    assert int(oo[0]) == 0 and int(io[0]) == 0 and int(oo[-1]) == E and int(io[-1]) == E
    assert bool((oo[1:] >= oo[:-1]).all()) and bool((io[1:] >= io[:-1]).all())
    assert bool((nodes[1:] > nodes[:-1]).all())
    n = src.numel()
    # node set: every row identifier is listed, and V equals the distinct count
    pos_s = torch.searchsorted(nodes, src)
    pos_d = torch.searchsorted(nodes, dst)
    assert bool((pos_s < V).all()) and bool((pos_d < V).all())
    assert bool((nodes[pos_s] == src).all()) and bool((nodes[pos_d] == dst).all())
    del pos_s, pos_d
    # (torch.unique takes fewer than 2^31 elements: unique each column first)
    uniq_v = torch.unique(torch.cat([torch.unique(src), torch.unique(dst)])).numel()
    assert V == uniq_v, f"V {V} != distinct identifiers {uniq_v}"
    ar = torch.arange(V, device=nodes.device, dtype=torch.int64)
    osrc = torch.repeat_interleave(ar, oo[1:] - oo[:-1])
    okey = osrc * V + on
    del osrc
    assert bool((okey[1:] > okey[:-1]).all()), "out-lists strictly increasing"
    # rows -> packed keys in chunks (bounded memory)
    uniq_rows = []
    chunk = 1 << 28
    for lo in range(0, n, chunk):
        s = torch.searchsorted(nodes, src[lo:lo + chunk])
        d = torch.searchsorted(nodes, dst[lo:lo + chunk])
        rk = s * V + d
        del s, d
        k = torch.searchsorted(okey, rk)
        assert bool((k < E).all()) and bool((okey[k] == rk).all()), "every row is an edge"
        uniq_rows.append(torch.unique(rk))
        del rk, k
    assert E == torch.unique(torch.cat(uniq_rows)).numel(), "E = distinct rows"
    del uniq_rows
    idst = torch.repeat_interleave(ar, io[1:] - io[:-1])
    ikey = idst * V + inn
    del idst
    assert bool((ikey[1:] > ikey[:-1]).all()), "in-lists strictly increasing"
    tr = torch.sort(on * V + torch.div(okey - on, V, rounding_mode="floor"))[0]
    assert bool((tr == ikey).all()), "in-CSR is the transpose"
    deg = (oo[1:] - oo[:-1]) + (io[1:] - io[:-1])
    assert bool((deg >= 1).all())


def check_sampled(g, src, dst, num_samples=256, seed=0):
    """Exact out- and in-lists of sampled nodes, computed on the host from the
    rows that touch them (the definition, one node at a time)."""
    import torch
    V = g.num_nodes
    rng = np.random.default_rng(seed)
    pick = torch.from_numpy(np.unique(rng.integers(0, V, size=num_samples))).to(g.node_ids.device)
    ids = g.node_ids[pick]
    m = torch.isin(src, ids) | torch.isin(dst, ids)
    rs, rd = src[m].cpu().numpy(), dst[m].cpu().numpy()
    nodes = g.node_ids
    oo, io = g.out_offsets.cpu().numpy(), g.in_offsets.cpu().numpy()
    for v, x in zip(pick.cpu().numpy().tolist(), ids.cpu().numpy().tolist()):
        want_out = np.unique(rd[rs == x])
        want_in = np.unique(rs[rd == x])
        got_out = nodes[g.out_nbrs[oo[v]:oo[v + 1]].long()].cpu().numpy()
        got_in = nodes[g.in_nbrs[io[v]:io[v + 1]].long()].cpu().numpy()
        assert np.array_equal(got_out, want_out), f"out-list of node {x}"
        assert np.array_equal(got_in, want_in), f"in-list of node {x}"
