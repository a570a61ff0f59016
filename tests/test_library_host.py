"""CPU checks of libpic.so: it loads, exports the C ABI, builds the same tree
tables as the oracle (host code only, no GPU needed) and rejects bad
arguments before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import workloads as W
import paper_1508_02435_amd as pic
from paper_1508_02435_amd import _capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

TREES = [W.regular_tree(2, 3), W.regular_tree(3, 2), W.disc_tree(2, 2, 4), W.disc_tree(3, 1, 3),
         W.disc_tree(2, 1, 3, radius=(1, 3)), W.regular_tree(2, 0), W.disc_tree(2, 4, 6)]


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "pic.h")).read()
    declared = set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(pic_\w+)\s*\(", header, re.M))
    assert declared == set(_capi.EXPORTS)
    L = C.CDLL(_capi.LIB_PATH)
    for name in declared:
        assert hasattr(L, name), name


@pytest.mark.parametrize("spec", TREES, ids=lambda s: f"d{s.dim}L{s.max_level}")
def test_tree_tables_equal_oracle(spec):
    o = oracle.OracleTree(spec)
    t = pic.Tree(spec)
    assert (t.n_leaves, t.n_vertices, t.n_pidt) == (o.n_leaves, o.n_vertices, o.n_pidt)
    a, b = t.leaf_table(), o.leaves()
    for k in ("key", "level", "coord", "vtx", "pidt"):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(t.vertex_table(), o.vertex_positions())
    pa, pb = t.pidt_table(), o.pidt_bins()
    for k in ("key", "level", "b"):
        assert np.array_equal(pa[k], pb[k]), k
    assert t.regular == all(lv == spec.max_level for lv in b["level"])


def test_forest_tables_concatenate_instances():
    specs = [W.regular_tree(2, 3), W.disc_tree(2, 2, 4), W.regular_tree(2, 2)]
    t = pic.Tree(specs)
    assert t.n_inst == 3 and not t.regular
    lt = t.leaf_table()
    off = 0
    voff = 0
    poff = 0
    for i, s in enumerate(specs):
        o = oracle.OracleTree(s)
        ii = t.instance(i)
        assert (ii.leaf_offset, ii.vertex_offset, ii.pidt_offset) == (off, voff, poff)
        ol = o.leaves()
        assert np.array_equal(lt["key"][off:off + o.n_leaves], ol["key"])
        assert np.array_equal(lt["vtx"][off:off + o.n_leaves], ol["vtx"] + voff)
        assert np.array_equal(lt["pidt"][off:off + o.n_leaves], ol["pidt"] + poff)
        off += o.n_leaves
        voff += o.n_vertices
        poff += o.n_pidt
    assert (t.n_leaves, t.n_vertices, t.n_pidt) == (off, voff, poff)


def test_division_magic_is_exact():
    """floor(n M / 2^k) == floor(n / 3^e) for n < 2^30 (Granlund-Montgomery bound)."""
    for e in range(0, 20):
        d = 3 ** e
        k = 30 + (d - 1).bit_length()
        M = (2 ** k + d - 1) // d
        assert 2 ** k <= M * d <= 2 ** k + 2 ** (k - 30)
        assert M * (2 ** 30) < 2 ** 64
        for n in [0, 1, d - 1, d, d + 1, 2 ** 30 - 1, (2 ** 30 // d) * d, (2 ** 30 // d) * d - 1]:
            if 0 <= n < 2 ** 30:
                assert (n * M) >> k == n // d


def _tree_handle(spec):
    return pic.Tree(spec)


def test_bad_tree_arguments_are_rejected():
    L = _capi.lib()
    h = C.c_void_p()
    lv = (C.c_int32 * 1)(3)
    assert L.pic_tree_create(4, 1, lv, None, C.byref(h)) == _capi.PIC_E_ARG
    assert L.pic_tree_create(2, 0, lv, None, C.byref(h)) == _capi.PIC_E_ARG
    assert L.pic_tree_create(2, 1, lv, None, C.byref(h)) == _capi.PIC_E_ARG     # masks missing
    lv19 = (C.c_int32 * 1)(19)
    assert L.pic_tree_create(2, 1, lv19, None, C.byref(h)) == _capi.PIC_E_ARG
    lv13 = (C.c_int32 * 1)(13)
    assert L.pic_tree_create(3, 1, lv13, None, C.byref(h)) == _capi.PIC_E_ARG   # 3^(3*13)*64 > 2^64
    assert L.pic_tree_create(2, 1, lv, None, None) == _capi.PIC_E_ARG


def test_calls_check_arguments_before_the_device():
    t = pic.Tree(W.regular_tree(2, 2))
    L = _capi.lib()
    P = _capi.Particles()
    P.n = 10
    # no coordinate pointers
    assert L.pic_gather_push(t.handle, 0, 0, C.byref(P), None, 0.0, 0.0, None, None, None, None, None) \
        == _capi.PIC_E_ARG
    assert L.pic_locate(t.handle, 5, 0, C.byref(P), None, None, None) == _capi.PIC_E_ARG
    # positions alone are enough for locate and deposit (no velocities needed)
    P.x[0], P.x[1] = 0x1000, 0x2000
    assert L.pic_locate(t.handle, 0, 0, C.byref(P), None, C.c_void_p(0x3000), None) == _capi.PIC_E_STATE
    # ... but gather_push needs velocities
    E = (C.c_void_p * 3)(0x4000, 0x5000, None)
    assert L.pic_gather_push(t.handle, 0, 0, C.byref(P), E, 0.0, 0.0, None, None, C.c_void_p(0x3000), None,
                             None) == _capi.PIC_E_ARG
    P.v[0], P.v[1] = 0x6000, 0x7000
    assert L.pic_gather_push(t.handle, 0, 0, C.byref(P), E, 0.0, 0.0, None, None, C.c_void_p(0x3000), None,
                             None) == _capi.PIC_E_STATE
    P.n = 0
    # nothing uploaded yet: valid arguments report the state error
    assert L.pic_locate(t.handle, 0, 0, C.byref(P), None, None, None) == _capi.PIC_E_STATE
    # undersized scratch is reported
    need = pic.scratch_bytes(t, 1000, pic.PIT)
    assert need > 0
    fake = C.c_void_p(0x1000)
    start = C.c_void_p(0x2000)
    nb = C.c_void_p(0x3000)
    assert L.pic_rebin(t.handle, 0, 1000, nb, None, 0, None, None, None, start, fake, need - 1, None, None) \
        == _capi.PIC_E_SCRATCH
    # statistics need the old offsets (a sorted input)
    assert L.pic_rebin(t.handle, 0, 1000, nb, None, 0, None, None, None, start, fake, need, C.c_void_p(0x6000),
                       None) == _capi.PIC_E_ARG
    # bad column width
    cols = (C.c_void_p * 1)(0x4000)
    outs = (C.c_void_p * 1)(0x5000)
    w = (C.c_int32 * 1)(2)
    assert L.pic_rebin(t.handle, 0, 1000, nb, None, 1, cols, outs, w, start, fake, need, None, None) \
        == _capi.PIC_E_ARG
    # aliasing columns
    w8 = (C.c_int32 * 1)(8)
    assert L.pic_rebin(t.handle, 0, 1000, nb, None, 1, cols, cols, w8, start, fake, need, None, None) \
        == _capi.PIC_E_ARG
    assert L.pic_status_sync(t.handle, None) == _capi.PIC_E_STATE
    assert _capi.status_string(_capi.PIC_E_SCRATCH) == "scratch buffer too small"


def test_tuning_knobs_accept_only_listed_values():
    before = pic.tuning()
    try:
        for name, values in pic.TUNING_KNOBS.items():
            for v in values:
                pic.tune(name, v)
                assert pic.tuning()[name] == v
            with pytest.raises(pic.PicError):
                pic.tune(name, 12345)
        with pytest.raises(pic.PicError):
            pic.tune("no_such_knob", 1)
        assert _capi.lib().pic_tune_get(b"no_such_knob") == -1
    finally:
        for k, v in before.items():
            pic.tune(k, v)


def test_output_sets_must_hold_every_particle():
    """The output set of a step states its capacity in n: one smaller (or
    larger) than the input is rejected before anything is enqueued."""
    t = pic.Tree(W.regular_tree(2, 2))
    L = _capi.lib()
    P, Q = _capi.Particles(), _capi.Particles()
    P.n, Q.n = 100, 99
    P.x[0], P.x[1], P.v[0], P.v[1] = 0x1000, 0x2000, 0x3000, 0x4000
    Q.x[0], Q.x[1], Q.v[0], Q.v[1] = 0x5000, 0x6000, 0x7000, 0x8000
    E = (C.c_void_p * 3)(0x9000, 0xa000, None)
    ptr = C.c_void_p
    need = pic.scratch_bytes(t, 100, pic.PIT)
    for qn, want in ((99, _capi.PIC_E_ARG), (101, _capi.PIC_E_ARG), (100, _capi.PIC_E_STATE)):
        Q.n = qn
        assert L.pic_step(t.handle, 0, 0, C.byref(P), ptr(0xb000), E, 0.0, 0.0, None, 0, None, None, None, -1,
                          0.0, C.byref(Q), ptr(0xc000), ptr(0xd000), ptr(0xe000), need, None, None) == want
        assert L.pic_stream_step(t.handle, 0, C.byref(P), ptr(0xb000), 0.1, _capi.REFLECTING, 0, 0, None, None,
                                 None, C.byref(Q), ptr(0xc000), ptr(0xe000), need, None, None) == want


def test_knobs_are_per_tree():
    """A tree copies the process defaults when it is created; changing one
    tree's knobs changes neither the defaults nor another tree's."""
    before = pic.tuning()
    try:
        pic.tune("step_tile", 1024)
        a = pic.Tree(W.regular_tree(2, 2))
        pic.tune("step_tile", 2048)
        b = pic.Tree(W.regular_tree(2, 2))
        assert pic.tuning(a)["step_tile"] == 1024 and pic.tuning(b)["step_tile"] == 2048
        pic.tune("emit_threads", 512, a)
        assert pic.tuning(a)["emit_threads"] == 512
        assert pic.tuning(b)["emit_threads"] == pic.tuning()["emit_threads"] == before["emit_threads"]
        with pytest.raises(pic.PicError):
            pic.tune("emit_threads", 256, a)
        with pytest.raises(pic.PicError):                 # read only when a tree is created
            pic.tune("regular_tables", 0, a)
        assert "regular_tables" not in pic.tuning(a)
    finally:
        for k, v in before.items():
            pic.tune(k, v)


def test_fp32_form_needs_regular_trees_with_tables():
    L = _capi.lib()
    adaptive = pic.Tree(W.disc_tree(2, 2, 4))
    regular = pic.Tree(W.regular_tree(2, 3))
    assert pic.scratch_bytes(adaptive, 1000, pic.PIT, pic.F32_OFFSET) == 0
    assert pic.scratch_bytes(regular, 1000, pic.PIT, pic.F32_OFFSET) > pic.scratch_bytes(regular, 1000, pic.PIT)
    P = _capi.Particles()
    P.n = 10
    P.off[0], P.off[1], P.u[0], P.u[1] = 0x1000, 0x2000, 0x3000, 0x4000
    E = (C.c_void_p * 3)(0x5000, 0x6000, None)
    nb = C.c_void_p(0x7000)
    start = C.c_void_p(0x8000)
    assert L.pic_gather_push(adaptive.handle, 0, 1, C.byref(P), E, 0.0, 0.0, None, start, nb, None, None) \
        == _capi.PIC_E_ARG
    # FP32 needs the segment offsets (its cell is implicit in the bin) and produces no E_p
    assert L.pic_gather_push(regular.handle, 0, 1, C.byref(P), E, 0.0, 0.0, None, None, nb, None, None) \
        == _capi.PIC_E_ARG
    assert L.pic_gather_push(regular.handle, 0, 1, C.byref(P), E, 0.0, 0.0, None, start, nb,
                             C.c_void_p(0x9000), None) == _capi.PIC_E_ARG
    assert L.pic_gather_push(regular.handle, 0, 1, C.byref(P), E, 0.0, 0.0, None, start, nb, None, None) \
        == _capi.PIC_E_STATE                                   # arguments fine, nothing uploaded
    # conversion needs both forms' pointers and a positive dt
    assert L.pic_convert(regular.handle, 0, 1, C.byref(P), 0.5, None, None, nb, None) == _capi.PIC_E_ARG
    P.x[0], P.x[1], P.v[0], P.v[1] = 0xa000, 0xb000, 0xc000, 0xd000
    assert L.pic_convert(regular.handle, 0, 1, C.byref(P), 0.0, None, None, nb, None) == _capi.PIC_E_ARG
    assert L.pic_convert(regular.handle, 0, 1, C.byref(P), 0.5, None, None, nb, None) == _capi.PIC_E_STATE
    assert L.pic_convert(adaptive.handle, 0, 1, C.byref(P), 0.5, None, None, nb, None) == _capi.PIC_E_ARG


def test_tables_off_gives_no_fp32_form():
    before = pic.tuning()["regular_tables"]
    pic.tune("regular_tables", 0)
    try:
        t = pic.Tree(W.regular_tree(2, 3))
    finally:
        pic.tune("regular_tables", before)
    assert pic.scratch_bytes(t, 1000, pic.PIT, pic.F32_OFFSET) == 0
    assert pic.scratch_bytes(t, 1000, pic.PIT) > 0


def _adapt_cases():
    rng = np.random.default_rng(21)
    out = []
    for spec, start, n, ppc, cap in [(W.regular_tree(2, 1), 1.0, 2000, 50, 5), (W.regular_tree(2, 2), 0.1, 3000, 30, 5),
                                     (W.disc_tree(2, 1, 3), 1.0, 1500, 8, 4), (W.regular_tree(3, 1), 0.1, 1200, 20, 3),
                                     (W.disc_tree(3, 1, 2), 1.0, 800, 4, 3), (W.regular_tree(2, 3), 0.3, 400, 6, 3),
                                     (W.regular_tree(2, 0), 1.0, 50, 10, 2)]:
        out.append((spec, rng.random((spec.dim, n)) * start, ppc, cap))
    return out


@pytest.mark.parametrize("case", range(7))
def test_tree_adapt_equals_oracle_rule(case):
    """pic_tree_adapt (host code of the library) against the oracle's rule,
    applied repeatedly until the tree stops changing: the masks agree byte
    for byte at every application."""
    spec, x, ppc, cap = _adapt_cases()[case]
    for _ in range(8):
        o = oracle.OracleTree(spec)
        t = pic.Tree(spec)
        counts = np.bincount(o.bin_of(x, oracle.PIT), minlength=o.n_leaves)
        got = pic.adapt(t, counts, ppc, cap)
        want = oracle.adapt(spec, x, ppc, cap)
        same = want.max_level == spec.max_level and np.array_equal(want.masks_concat(), spec.masks_concat())
        if same:
            assert got is None
            break
        assert got is not None and got.max_level == want.max_level
        assert np.array_equal(got.masks_concat(), want.masks_concat())
        spec = want


def test_tree_adapt_rejects_bad_arguments():
    t = pic.Tree(W.regular_tree(2, 1))
    cnt = np.zeros(9, np.int64)
    ln, nl = C.c_size_t(0), C.c_int32(0)
    L = _capi.lib()
    assert L.pic_tree_adapt(t.handle, cnt.ctypes.data, -1, 3, None, 0, C.byref(ln), C.byref(nl)) == _capi.PIC_E_ARG
    assert L.pic_tree_adapt(t.handle, cnt.ctypes.data, 5, 19, None, 0, C.byref(ln), C.byref(nl)) == _capi.PIC_E_ARG
    bad = cnt.copy()
    bad[3] = -2
    assert L.pic_tree_adapt(t.handle, bad.ctypes.data, 5, 3, None, 0, C.byref(ln), C.byref(nl)) == _capi.PIC_E_ARG
    cnt[4] = 10
    assert L.pic_tree_adapt(t.handle, cnt.ctypes.data, 5, 3, None, 0, C.byref(ln), C.byref(nl)) == _capi.PIC_E_CAPACITY
    assert (ln.value, nl.value) == (1 + 9, 2)
    forest = pic.Tree([W.regular_tree(2, 1), W.regular_tree(2, 1)])
    cnt2 = np.zeros(18, np.int64)
    assert L.pic_tree_adapt(forest.handle, cnt2.ctypes.data, 5, 3, None, 0, C.byref(ln), C.byref(nl)) == _capi.PIC_E_ARG


def test_free_stream_rejects_bad_arguments():
    t = pic.Tree(W.regular_tree(2, 1))
    L = _capi.lib()
    P = _capi.Particles()
    for boundary, flops in ((2, 0), (-1, 0), (1, 3), (1, -2), (0, (1 << 20) + 2)):
        assert L.pic_free_stream(t.handle, 0, 0, C.byref(P), 0.1, None, boundary, flops, None, None) == _capi.PIC_E_ARG
    assert L.pic_free_stream(t.handle, 0, 1, C.byref(P), 0.1, None, 1, 0, None, None) == _capi.PIC_E_ARG
