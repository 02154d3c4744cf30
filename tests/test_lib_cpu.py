"""Library checks that need no GPU: the shared library loads and exports
every symbol of include/hlu.h; host-side assembly and the integer cluster /
block structure are bit-exact against the oracle; argument errors."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle.assemble import Discretisation
from oracle.cluster import Structure

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2211_11303_amd", "libhlu.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libhlu.so not built")


def _header_symbols():
    txt = open(os.path.join(ROOT, "include", "hlu.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hlu_[a-z_]+|gmres_[a-z_]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    syms = _header_symbols()
    assert "hlu_factor" in syms and "gmres_solve" in syms and len(syms) >= 18
    for s in syms:
        assert hasattr(lib, s), s


@pytest.mark.parametrize("n,kappa", [(1, 1.0), (2, 3.0), (4, 2.0), (8, 8.0)])
def test_assembly_matches_oracle(n, kappa):
    from paper_2211_11303_amd import hlu
    rp, ci, va, mid = hlu.hlu_kuhn_assemble(n, kappa)
    d = Discretisation(n, kappa)
    assert np.array_equal(rp, d.A.indptr) and np.array_equal(ci, d.A.indices)
    assert np.abs(va - d.A.data).max() <= 1e-14 * np.abs(d.A.data).max()
    assert np.array_equal(mid, d.mesh.midpoints2())
    assert hlu.hlu_kuhn_sizes(n) == (7 * n ** 3 - 9 * n ** 2 + 3 * n, len(ci))


@pytest.mark.parametrize("n", [1, 2, 4, 8])
def test_load_matches_oracle(n):
    """hlu_kuhn_load against the oracle's load (itself pinned by the exact
    reproduction of constant fields and G^T b = 0)."""
    from paper_2211_11303_amd import hlu
    d = Discretisation(n, 1.0)
    for J in ((0.0, 0.0, 1.0), (0.3, -1.2, 0.7)):
        b = hlu.hlu_kuhn_load(n, J)
        ref = d.load(J)
        assert b.shape == ref.shape
        assert np.abs(b - ref).max() <= 1e-14 * max(1e-300, np.abs(ref).max())


@pytest.mark.parametrize("n,leaf", [(4, 32), (4, 8), (5, 20), (8, 64), (8, 17)])
def test_structure_bit_exact(n, leaf):
    from paper_2211_11303_amd import hlu
    rp, ci, va, mid = hlu.hlu_kuhn_assemble(n, 2.0)
    h = hlu.HLU(rp, ci, va, mid, 2.0, leaf)
    st = h.hlu_export_structure()
    s = Structure(mid, leaf, 2.0)
    assert np.array_equal(st["perm"], s.perm)
    assert np.array_equal(st["begin"], [c.begin for c in s.clusters])
    assert np.array_equal(st["end"], [c.end for c in s.clusters])
    assert np.array_equal(st["level"], [c.level for c in s.clusters])
    assert np.array_equal(st["son0"], [c.sons[0].id if c.sons else -1 for c in s.clusters])
    assert np.array_equal(st["son1"], [c.sons[1].id if c.sons else -1 for c in s.clusters])
    assert np.array_equal(st["brow"], [b.row.id for b in s.block_leaves])
    assert np.array_equal(st["bcol"], [b.col.id for b in s.block_leaves])
    assert np.array_equal(st["bkind"], [b.kind for b in s.block_leaves])
    stats = h.hlu_get_stats()
    sm = s.summary()
    assert stats["num_admissible"] == sm["admissible"] and stats["num_dense"] == sm["dense"]
    assert stats["dense_entries"] == sm["dense_entries"] and stats["depth"] == sm["depth"]


@pytest.mark.slow
def test_structure_bit_exact_16():
    from paper_2211_11303_amd import hlu
    rp, ci, va, mid = hlu.hlu_kuhn_assemble(16, 4.0)
    h = hlu.HLU(rp, ci, va, mid, 2.0, 64)
    st = h.hlu_export_structure()
    s = Structure(mid, 64, 2.0)
    assert np.array_equal(st["perm"], s.perm)
    assert np.array_equal(st["bkind"], [b.kind for b in s.block_leaves])
    assert np.array_equal(st["brow"], [b.row.id for b in s.block_leaves])


def test_argument_errors():
    from paper_2211_11303_amd import _lib as L
    from paper_2211_11303_amd import hlu
    rp, ci, va, mid = hlu.hlu_kuhn_assemble(2, 1.0)
    bad = ci.copy()
    bad[0] = len(rp) + 5                      # column out of range
    with pytest.raises(L.HluError) as e:
        hlu.HLU(rp, bad, va, mid, 2.0, 8)
    assert e.value.status == -1
    unsorted = ci.copy()
    unsorted[[0, 1]] = unsorted[[1, 0]]
    with pytest.raises(L.HluError):
        hlu.HLU(rp, unsorted, va, mid, 2.0, 8)
    with pytest.raises(L.HluError):
        hlu.HLU(rp, ci, va, mid, 2.0, 0)     # leaf size 0
    h = hlu.HLU(rp, ci, va, mid, 2.0, 8)
    with pytest.raises(L.HluError):
        h.hlu_workspace_bytes(-1.0)          # negative eps
    with pytest.raises(L.HluError) as e:
        L.check(L.lib().hlu_solve(h.handle, ctypes.c_void_p(8), ctypes.c_void_p(8), 1, h.n, None))
    assert e.value.status == -6              # not factored


def test_plan_sizes_reported():
    from paper_2211_11303_amd import hlu
    rp, ci, va, mid = hlu.hlu_kuhn_assemble(4, 2.0)
    h = hlu.HLU(rp, ci, va, mid, 2.0, 32)
    b64 = h.hlu_workspace_bytes(1e-6, prec="fp64")
    b32 = h.hlu_workspace_bytes(1e-6, prec="fp32")
    assert b32 < b64
    # FP32 storage whatever the arithmetic of the dense tasks
    assert h.hlu_workspace_bytes(1e-6, prec="fp32-acc64") == b32
    st = h.hlu_get_stats()
    assert st["factor_waves"] > 0 and st["factor_tasks"] > 0 and st["solve_waves"] > 0


def test_build_shared_pattern_rules():
    """hlu_build_shared accepts another kappa on the same mesh (same plans,
    same structure) and rejects a different pattern."""
    from paper_2211_11303_amd import _lib as L
    from paper_2211_11303_amd import hlu
    rp, ci, va, mid = hlu.hlu_kuhn_assemble(4, 2.0)
    proto = hlu.HLU(rp, ci, va, mid, 2.0, 32)
    rp2, ci2, va2, _ = hlu.hlu_kuhn_assemble(4, 7.0)
    h2 = hlu.HLU(rp2, ci2, va2, share=proto)
    a, b = proto.hlu_export_structure(), h2.hlu_export_structure()
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    assert h2.hlu_workspace_bytes(1e-6) == proto.hlu_workspace_bytes(1e-6)
    rp3, ci3, va3, _ = hlu.hlu_kuhn_assemble(5, 2.0)
    with pytest.raises(L.HluError) as e:
        hlu.HLU(rp3, ci3, va3, share=proto)
    assert e.value.status == -1
    moved = ci2.copy()
    moved[3] = moved[3] - 1 if moved[3] - 1 != moved[2] else moved[3]
    if not np.array_equal(moved, ci2):
        with pytest.raises(L.HluError):
            hlu.HLU(rp2, moved, va2, share=proto)


def test_server_rejects_bad_refinement_options():
    """Refinement options are checked before any device work."""
    from paper_2211_11303_amd import _lib as L
    from paper_2211_11303_amd import hlu
    for kw in (dict(refine_iters=-1), dict(refine_iters=10, refine_eps_factor=1.0),
               dict(refine_iters=10, refine_eps_factor=0.0), dict(refine_iters=10, max_refines=-1)):
        with pytest.raises(L.HluError) as e:
            hlu.Server(**kw)
        assert e.value.status == L.STATUS_CODES["HLU_ERR_INVALID_ARG"], kw


def test_autotune_rejects_bad_arguments():
    """hlu_autotune_leaf checks its arguments before any device work."""
    from paper_2211_11303_amd import _lib as L
    fo = L.FactorOpts(1e-3, 0, L.HLU_FP32)
    go = L.GmresOpts(50, 100, 1e-8)
    secs = (ctypes.c_double * 4)()
    best = ctypes.c_int32()
    for cand, count, nrhs in (([0], 1, 1), ([129], 1, 1), ([32], 0, 1), ([32], 1, 0), ([32], 1, 33)):
        arr = (ctypes.c_int32 * max(1, len(cand)))(*cand)
        st = L.lib().hlu_autotune_leaf(4, 2.0, 2.0, arr, count, ctypes.byref(fo), ctypes.byref(go), nrhs, secs,
                                       ctypes.byref(best), None)
        assert st == L.STATUS_CODES["HLU_ERR_INVALID_ARG"], (cand, count, nrhs, st)


@pytest.mark.parametrize("n,leaf", [(12, 64), (12, 32)])
def test_planning_mid_size(n, leaf):
    """Host planning of a mid-size mesh: the factor plan and the persistent
    solve schedule are built (the schedule builder checks that every
    T-product is formed exactly once, by a leaf task or by one T-product
    task) and the sizes are consistent."""
    from paper_2211_11303_amd import hlu
    rp, ci, va, mid = hlu.hlu_kuhn_assemble(n, 8.0)
    h = hlu.HLU(rp, ci, va, mid, 2.0, leaf)
    b32 = h.hlu_workspace_bytes(1e-3, prec="fp32")
    st = h.hlu_get_stats()
    assert b32 > 0 and st["factor_waves"] > 0 and st["factor_tasks"] > st["factor_waves"]
    assert st["num_leaf_clusters"] * 2 - 1 == st["num_clusters"]


@pytest.mark.parametrize("n,leaf", [(8, 32), (16, 64)])
def test_truncation_rounds_terminate(n, leaf):
    """Host replay of the truncation rounds of the factor plan (the same
    round code as the device kernel) with every rank forced: at rank 64 a
    block already holds a whole round's columns while parts remain (the
    case that once looped), and every op still finishes within its bound;
    the total rounds grow with the forced rank."""
    from paper_2211_11303_amd import hlu
    rp, ci, va, mid = hlu.hlu_kuhn_assemble(n, 8.0)
    H = hlu.HLU(rp, ci, va, mid, eta=2.0, leaf=leaf)
    prev = 0
    for forced in (0, 4, 48, 64, 200):
        r = H.hlu_check_trunc_rounds(1e-3, forced)
        assert r["ops"] > 0 and r["unfinished"] == 0, (forced, r)
        assert r["rounds"] >= prev
        prev = r["rounds"]
        if forced >= 64:
            assert r["stalled_rounds"] > 0, r
        if forced <= 48:
            assert r["stalled_rounds"] == 0, r
    # a capacity cap below the round limit never stalls
    r = H.hlu_check_trunc_rounds(1e-3, 200, max_rank=32)
    assert r["unfinished"] == 0 and r["stalled_rounds"] == 0, r


@pytest.mark.parametrize("n,box,beta", [(2, (0, 0, 0, 1, 2, 1), 10.0), (4, (1, 1, 1, 3, 3, 3), 100.0),
                                        (8, (0, 2, 3, 8, 5, 6), 0.1)])
def test_coefficient_box_matches_oracle(n, box, beta):
    from paper_2211_11303_amd import hlu
    rp, ci, va, mid = hlu.hlu_kuhn_assemble_beta(n, 3.0, box, beta)
    d = Discretisation(n, 3.0, box, beta)
    assert np.array_equal(rp, d.A.indptr) and np.array_equal(ci, d.A.indices)
    assert np.abs(va - d.A.data).max() <= 1e-14 * np.abs(d.A.data).max()
    assert np.array_equal(mid, d.mesh.midpoints2())


@pytest.mark.parametrize("n", [1, 3, 8])
def test_support_boxes_match_oracle(n):
    from paper_2211_11303_amd import hlu
    from oracle.mesh import KuhnMesh
    lo, hi = hlu.hlu_kuhn_support_boxes(n)
    olo, ohi = KuhnMesh(n).support_boxes2()
    assert np.array_equal(lo, olo) and np.array_equal(hi, ohi)


@pytest.mark.parametrize("n,leaf", [(4, 8), (6, 16), (8, 64)])
def test_support_box_structure_bit_exact(n, leaf):
    from paper_2211_11303_amd import hlu
    rp, ci, va, mid = hlu.hlu_kuhn_assemble(n, 2.0)
    boxes = hlu.hlu_kuhn_support_boxes(n)
    h = hlu.HLU(rp, ci, va, mid, 2.0, leaf, boxes=boxes)
    st = h.hlu_export_structure()
    s = Structure(mid, leaf, 2.0, boxes=boxes)
    assert np.array_equal(st["perm"], s.perm)
    assert np.array_equal(st["brow"], [b.row.id for b in s.block_leaves])
    assert np.array_equal(st["bcol"], [b.col.id for b in s.block_leaves])
    assert np.array_equal(st["bkind"], [b.kind for b in s.block_leaves])
    assert h.hlu_get_stats()["dense_entries"] == s.summary()["dense_entries"]


def test_box_arguments_rejected():
    from paper_2211_11303_amd import hlu
    from paper_2211_11303_amd import _lib as L
    rp, ci, va, mid = hlu.hlu_kuhn_assemble(3, 2.0)
    lo, hi = hlu.hlu_kuhn_support_boxes(3)
    bad = lo.copy()
    bad[5, 1] = mid[5, 1] + 1           # box no longer contains its midpoint
    with pytest.raises(L.HluError):
        hlu.HLU(rp, ci, va, mid, 2.0, 16, boxes=(bad, hi))
    with pytest.raises(L.HluError):
        hlu.hlu_kuhn_assemble_beta(3, 2.0, (0, 0, 0, 1, 1, 1), -1.0)


def test_fit_ranks_needs_a_factorisation():
    """hlu_fit_ranks reads the ranks of the handle's last factorisation; before
    one it is a state error (no device work is started)."""
    from paper_2211_11303_amd import hlu
    from paper_2211_11303_amd import _lib as L
    rp, ci, va, mid = hlu.hlu_kuhn_assemble(3, 2.0)
    h = hlu.HLU(rp, ci, va, mid, 2.0, 16)
    with pytest.raises(L.HluError) as e:
        h.hlu_fit_ranks(1e-4, margin=2)
    assert L.STATUS.get(e.value.status) == "HLU_ERR_STATE"
    # dropping a fit that was never made gives back the uniform workspace
    assert h.hlu_fit_ranks(1e-4, margin=-1) == h.hlu_workspace_bytes(1e-4)


@pytest.mark.parametrize("mm", [1, 2])
def test_two_box_domain_matches_oracle(mm):
    """hlu_kuhn_*_domain on the two-box domain against the oracle (which finds
    the boundary from the triangles of exactly one tetrahedron, the library
    from the lattice faces): pattern, midpoints and support boxes bit-exact,
    values and load to 1e-14."""
    from paper_2211_11303_amd import hlu
    from paper_2211_11303_amd.inputs import two_box_mask
    n, mask = two_box_mask(mm)
    rp, ci, va, mid = hlu.hlu_kuhn_assemble_domain(n, 3.0, mask, beta_box=(0, 0, 0, n, n // 2, n), beta_in=5.0)
    d = Discretisation(n, 3.0, (0, 0, 0, n, n // 2, n), 5.0, mask=mask)
    assert np.array_equal(rp, d.A.indptr) and np.array_equal(ci, d.A.indices)
    assert np.abs(va - d.A.data).max() <= 1e-14 * np.abs(d.A.data).max()
    assert np.array_equal(mid, d.mesh.midpoints2())
    b = hlu.hlu_kuhn_load_domain(n, mask, (1.0, 1.0, 1.0))
    ref = d.load((1.0, 1.0, 1.0))
    assert np.abs(b - ref).max() <= 1e-14 * np.abs(ref).max()
    lo, hi = hlu.hlu_kuhn_domain_support_boxes(n, mask)
    olo, ohi = d.mesh.support_boxes2()
    assert np.array_equal(lo, olo) and np.array_equal(hi, ohi)
    assert hlu.hlu_kuhn_domain_sizes(n, np.ones(n ** 3, np.uint8)) == hlu.hlu_kuhn_sizes(n)


def test_empty_domain_rejected():
    from paper_2211_11303_amd import hlu
    from paper_2211_11303_amd import _lib as L
    mask = np.zeros(27, np.uint8)
    assert hlu.hlu_kuhn_domain_sizes(3, mask) == (0, 0)
    with pytest.raises(L.HluError):
        hlu.hlu_kuhn_assemble_domain(3, 1.0, mask)
    lo = np.empty((1, 3), np.int32)
    b = np.empty(1)
    J = np.ones(3)
    m8 = mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    assert L.STATUS.get(L.lib().hlu_kuhn_domain_support_boxes(3, m8, lo.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                                              lo.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))) == \
        "HLU_ERR_INVALID_ARG"
    assert L.STATUS.get(L.lib().hlu_kuhn_load_domain(3, m8, J.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                     b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))) == \
        "HLU_ERR_INVALID_ARG"
    mask[13] = 1                      # one cube: only its body diagonal is off the boundary
    assert hlu.hlu_kuhn_domain_sizes(3, mask)[0] == 1


def test_gmres_refined_arguments():
    """gmres_solve_refined: workspace sizes, and NULL arguments rejected
    before any device work (the options are checked on the GPU tests)."""
    import ctypes
    from paper_2211_11303_amd import _lib as L
    lib = L.lib()
    assert lib.gmres_refined_workspace_bytes(100, 2, 30) > lib.gmres_workspace_bytes(100, 2, 30)
    assert lib.gmres_refined_workspace_bytes(0, 2, 30) == 0
    o = L.GmresOpts(30, 100, 1e-8)
    r = L.RefineOpts(10, 1, 0.1)
    info = (L.GmresInfo * 1)()
    ref = (ctypes.c_int32 * 1)()
    st = lib.gmres_solve_refined(None, None, None, 1, 10, None, ctypes.byref(o), ctypes.byref(r), info, ref,
                                 None, 0, None)
    assert L.STATUS.get(st) == "HLU_ERR_INVALID_ARG"
