"""The C-ABI library loads and exports every symbol the header declares.

Host-only entry points (argument validation that fails before any device
call, the Chebyshev order rule) are exercised without a GPU.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "procmv.h")).read()
    return sorted(set(re.findall(r"\b(procmv_[a-z_]+)\s*\(", text)))


def test_header_matches_binding_list():
    from paper_2606_31598_amd import procmv
    assert sorted(procmv.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    from paper_2606_31598_amd import procmv
    L = procmv.load()
    for name in _declared():
        assert hasattr(L, name), name


def test_cheb_order_matches_oracle():
    from paper_2606_31598_amd import procmv
    from oracle import chebyshev as ch
    for x in [0.125, 1.0, 7.3, 141.37, 4000.0, 82792.0]:
        for tol in [1e-7, 1e-10]:
            assert procmv.cheb_order(x, tol) == ch.cheb_order(x, tol)


def test_invalid_arguments_rejected_on_host():
    from paper_2606_31598_amd import procmv
    L = procmv.load()
    h = ctypes.c_void_p()
    assert L.procmv_create_operator(7, 1, 16, None, ctypes.byref(h)) == 1
    assert L.procmv_create_operator(0, 1, 0, None, ctypes.byref(h)) == 1
    assert L.procmv_create_operator(0, 1, 1 << 31, None, ctypes.byref(h)) == 1
    assert b"outside" in L.procmv_last_error()
    assert L.procmv_create_operator(0, 1, 100, None, None) == 1
    # a Philox-GUE operator is host state only until it is planned
    assert L.procmv_create_operator(0, 1, 100, None, ctypes.byref(h)) == 0
    assert L.procmv_plan(h, 100, 0, 0.0, 0, None) == 1         # not a multiple of 64
    assert L.procmv_plan(h, 64, 9, 0.0, 0, None) == 1          # unknown strategy
    assert L.procmv_plan(h, 64, 1, 1.5, 0, None) == 1          # fraction outside [0, 1]
    assert L.procmv_plan(h, 64, 0, 0.0, 2, None) == 1          # compensated: sinc-DVR only
    assert b"sinc-DVR" in L.procmv_last_error()
    assert L.procmv_plan(h, 64, 0, 0.0, 3, None) == 1          # unknown precision
    x = ctypes.c_void_p(16)
    assert L.procmv_apply(h, x, 100, x, 100, 1, None) == 4     # not planned
    info = procmv.PlanInfo()
    assert L.procmv_plan_info(h, ctypes.byref(info)) == 4
    assert L.procmv_get_entries(h, 90, 0, 20, 1, x, None) == 1  # window outside
    L.procmv_destroy(h)
    L.procmv_destroy(None)


def test_planner_memory_model_matches_paper_formulas():
    """Cache bytes of a plan are Eq. planner_partial_cache over canonical pairs
    (Eq. partial_cache_pairs); the memory test is Eq. planner_memory_constraint."""
    from paper_2606_31598_amd import procmv as pm
    from oracle import planner as opl
    D, b = 262144, 512
    nb = D // b
    for st, f in ((1, 0.25), (2, 1.0), (0, 0.0)):
        x, mt, fe = pm.plan_features(D, 16, 256e9, 1, 0, b, st, f)
        p = {0: 0, 1: int(f * opl.n_pair(nb)), 2: opl.n_pair(nb)}[st]
        m_op = opl.mem_partial(p, b)
        # workspace (Eq. planner_workspace, r arrays of D x R complex64): the
        # partial slots (one per 256-row band + 1, R = 16 per block of vectors)
        # plus input and output
        m_work = opl.mem_work(D // 256 + 1, D, 16) + opl.mem_work(2, D, 16)
        assert mt == m_op + m_work
        assert fe == opl.feasible(mt, [256e9], alpha=0.9)
        assert abs(x[7] - mt / 256e9) < 1e-6
    # a GUE full cache at D = 2^18 does not fit 256 GB
    _, _, fe = pm.plan_features(D, 1, 256e9, 1, 0, b, 2, 1.0)
    assert not fe


def test_analytic_planner_prefers_cache_with_reuse():
    from paper_2606_31598_amd import procmv as pm
    mm = pm.MachineModel()
    mm.gen_rate[0], mm.gen_rate[1] = 2.7e11, 5e11
    mm.dvr_rate, mm.cache_bw, mm.flop_rate, mm.launch_s = 1.4e13, 4e12, 1e14, 2e-5
    c = pm.plan_candidates()
    q1, _ = pm.plan_choose(0, 32768, 1, 256e9, 1, 0, mm=mm)
    q500, _ = pm.plan_choose(0, 32768, 1, 256e9, 500, 0, mm=mm)
    assert c[q1][1] == pm.PROCEDURAL        # one product: filling a cache never pays
    assert c[q500][1] == pm.FULL            # many products: the full cache does
    import pytest as _pt
    with _pt.raises(pm.ProcmvError) as e:
        pm.plan_choose(0, 262144, 64, 1e6, 1, 0, mm=mm)
    assert e.value.status == 3


def test_filter_order_matches_oracle():
    """Host-side order rule of the imaginary-time filter (no GPU needed)."""
    from paper_2606_31598_amd import procmv
    from oracle import chebyshev as ch
    for z in (0.0, 0.5, 3.0, 40.0, 713.0 * 2.0, 5000.0):
        for tol in (1e-7, 1e-10, 1e-13):
            assert procmv.filter_order(z, tol) == ch.filter_order(z, tol)
    assert procmv.filter_order(-1.0, 1e-10) == -1


def test_tile_shape_fit_keeps_cached_tiles_in_their_slot():
    """Tile rows 4 RW must fit the super-tile edge and divide a cached block
    size: one vector at shape 2 has 128-row tiles, allowed at D = 12000
    (256-row super-tiles) only for block sizes that 128 divides."""
    from paper_2606_31598_amd import procmv as pm
    assert pm.tile_shape_fit(1, 2, 12000, 0) == 2
    assert pm.tile_shape_fit(1, 2, 12000, 256) == 2
    assert pm.tile_shape_fit(1, 2, 12000, 192) == 1
    assert pm.tile_shape_fit(1, 2, 12000, 64) == 1
    assert pm.tile_shape_fit(1, 1, 12000, 64) == 1      # 64-row tiles fit a 64 block
    assert pm.tile_shape_fit(1, 2, 5000, 0) == 1        # 64-row super-tiles: 64-row tiles
    assert pm.tile_shape_fit(1, 2, 8000, 0) == 2        # 128-row super-tiles
    for nv in (2, 4, 8):                                # at most 64 rows: every block fits
        for b in (64, 192, 320):
            assert pm.tile_shape_fit(nv, 2, 12000, b) == 2
    for D in range(1, 20000, 997):
        for nv in (1, 2, 4, 8):
            for sh in (0, 1, 2):
                for b in (0, 64, 128, 192, 256, 448, 512):
                    got = pm.tile_shape_fit(nv, sh, D, b)
                    tr = 4 * (16 << got) // (2 * nv)
                    edge = 256 if (D + 255) // 256 >= 45 else 128 if (D + 127) // 128 >= 45 else 64
                    assert 0 <= got <= sh
                    assert got == 0 or (tr <= edge and (b == 0 or b % tr == 0))
    assert pm.tile_shape_fit(3, 0, 100, 0) == -1
    assert pm.tile_shape_fit(1, 3, 100, 0) == -1
    assert pm.tile_shape_fit(1, 0, 100, 100) == -1
