"""The C-ABI library on the host: it loads, exports every symbol of
include/spand.h, and its symbolic analysis (host C++) equals the oracle's
partition bit for bit: levels, paths, elimination permutation, the clusters of
every step, their adjacency with symbolic fill, children and colours."""
import os
import re

import numpy as np
import pytest

from synthetic import laplacian_2d, laplacian_3d, fv_diffusion_3d
from oracle import nd

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                      "spand.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(spand_[a-z_]+)\s*\(", txt)))


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert "spand_analyze" in names and "spand_pcg" in names
    for name in names:
        assert hasattr(lib, name), name
    from paper_2007_00789_amd import spand
    assert set(names) == set(spand.SIGNATURES)


CASES = [
    ("lap2d_64", lambda: laplacian_2d(64), 6, 4),
    ("lap2d_ragged", lambda: laplacian_2d(37, 23), 7, 2),
    ("lap3d_16", lambda: laplacian_3d(16), 6, 4),
    ("lap3d_box", lambda: laplacian_3d(5, shape=(11, 6, 9)), 7, 0),
    ("fv3d_12", lambda: fv_diffusion_3d(12, 3.0, 1002), 5, 1),
    ("lap3d_32", lambda: laplacian_3d(32), 9, 4),
]


def _two_grids():
    a, b = laplacian_2d(20, 9), laplacian_3d(7)
    rowptr = np.concatenate([a.rowptr, a.rowptr[-1] + b.rowptr[1:]])
    colind = np.concatenate([a.colind, b.colind + a.n])

    class P:
        pass
    p = P()
    p.n, p.rowptr, p.colind, p.nnz, p.coords = a.n + b.n, rowptr, colind, colind.size, None
    return p


# coordinate-free analysis (coords withheld): landmark hop distances
FREE = [
    ("free_lap2d_ragged", lambda: laplacian_2d(37, 23), 7, 2),
    ("free_lap3d_16", lambda: laplacian_3d(16), 6, 4),
    ("free_fv3d_12", lambda: fv_diffusion_3d(12, 3.0, 1002), 5, 1),
    ("free_disconnected", _two_grids, 5, 1),
]


@pytest.mark.parametrize("name,make,depth,skip", CASES + FREE, ids=[c[0] for c in CASES + FREE])
def test_analyze_matches_oracle(lib, name, make, depth, skip):
    from paper_2007_00789_amd import spand
    p = make()
    coords = None if name.startswith("free_") else p.coords
    ref = nd.analyze(p.rowptr, p.colind, coords, depth, skip)
    plan = spand.analyze(p.n, p.rowptr, p.colind, coords, spand.make_opts(depth=depth, skip=skip))
    assert plan.depth == depth and plan.n == p.n and plan.nnz == p.nnz
    lvl, path, perm = plan.vertices()
    assert np.array_equal(lvl, ref.lvl)
    assert np.array_equal(path, ref.path)
    assert np.array_equal(perm, ref.perm)
    for l in range(depth, -1, -1):
        st = ref.steps[l]
        got = plan.step(l)
        assert got["n_clusters"] == st.n_clusters and got["n_interior"] == st.n_interior
        assert got["sparsified"] == st.sparsified
        assert [(0 if i < st.n_interior else 1, int(a), int(b))
                for i, (a, b) in enumerate(zip(got["key_lvl"], got["key_prefix"]))] == st.keys
        adj = [got["adj"][got["adj_ptr"][c]:got["adj_ptr"][c + 1]] for c in range(st.n_clusters)]
        for c in range(st.n_clusters):
            assert np.array_equal(adj[c], st.adj[c]), (l, c)
        assert np.array_equal(got["colour"], st.colour)
        if st.children is not None:
            ch = [list(got["child"][got["child_ptr"][c]:got["child_ptr"][c + 1]])
                  for c in range(st.n_clusters)]
            assert ch == st.children


def test_default_depth_is_log2_n_over_64(lib):
    from paper_2007_00789_amd import spand
    p = laplacian_2d(64)
    plan = spand.analyze(p.n, p.rowptr, p.colind, p.coords, spand.make_opts(depth=0))
    assert plan.depth == 6


def test_error_paths(lib):
    from paper_2007_00789_amd import spand
    p = laplacian_2d(8)
    ci = p.colind.copy()
    ci[3] = (ci[3] + 5) % p.n          # breaks the symmetry of the pattern
    with pytest.raises(spand.SpandError) as e:
        spand.analyze(p.n, p.rowptr, ci, p.coords, spand.make_opts(depth=3))
    assert e.value.status == -2
    with pytest.raises(spand.SpandError) as e:
        spand.analyze(p.n, p.rowptr, p.colind, p.coords, spand.make_opts(depth=3, eps=1.5))
    assert e.value.status == -1
    with pytest.raises(spand.SpandError) as e:
        spand.analyze(p.n, p.rowptr, p.colind, p.coords, spand.make_opts(depth=3, scheme=7))
    assert e.value.status == -1


def test_opts_validation_on_the_host(lib):
    """spand_analyze checks the options without a device: negative
    top_fp64_levels or hbm_budget_bytes, unknown precisions and a
    qr_single_launch other than 0 or 1 are rejected; the defaults written by
    spand_default_opts land in the binding's fields (same layout)."""
    from paper_2007_00789_amd import spand
    p = laplacian_2d(16)
    o = spand.make_opts(depth=2, skip=0)
    assert o.top_fp64_levels == 3 and o.hbm_budget_bytes == 0 and o.qr_single_launch == 1
    spand.analyze(p.n, p.rowptr, p.colind, p.coords, o).close()
    for field, bad in (("top_fp64_levels", -1), ("hbm_budget_bytes", -5), ("precision", 7),
                       ("qr_single_launch", 2)):
        o2 = spand.make_opts(depth=2, skip=0)
        setattr(o2, field, bad)
        with pytest.raises(spand.SpandError) as e:
            spand.analyze(p.n, p.rowptr, p.colind, p.coords, o2)
        assert e.value.status == -1, field
