"""pic_deposit_noalloc: the deposit for callers that cannot allocate.

The entry point keeps the per-bin partials in a device-resident array the
library holds instead of a caller buffer.  Through the C ABI it must give the
charge pic_deposit gives (the same kernels in the same order: bit for bit,
which is inside the 1e-12 per-vertex bound), call after call: here two calls
in a row, the second on a smaller tree with fewer particles, so it reads only
what it wrote itself and nothing the first call left behind.  Trees whose
partials exceed the array are refused before anything is enqueued.
"""
import ctypes as C

import numpy as np
import pytest

import oracle
import workloads as W
import paper_1508_02435_amd as pic
from paper_1508_02435_amd import _capi

torch = pytest.importorskip("torch")


def _deposit_both(t, scheme, st, f32=False):
    """rho from pic_deposit (caller scratch) and from pic_deposit_noalloc."""
    L = _capi.lib()
    if f32:
        P = pic._particles(st.n, off=st.off, u=st.u, inst_start=st.inst_start)
        prec = pic.F32_OFFSET
    else:
        P = pic._particles(st.n, x=st.x, v=st.v, inst_start=st.inst_start)
        prec = pic.F64
    q = C.c_void_p(st.q.data_ptr()) if st.q is not None else None
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    ref = torch.full((t.n_vertices,), np.nan, dtype=torch.float64, device=st.start.device)
    got = torch.full_like(ref, np.nan)
    qu = -1.0 / st.n
    pic.check(L.pic_deposit(t.handle, scheme, prec, C.byref(P), C.c_void_p(st.start.data_ptr()), q, qu,
                            C.c_void_p(ref.data_ptr()), C.c_void_p(st.scratch.data_ptr()),
                            st.scratch.numel() * st.scratch.element_size(), s), "pic_deposit")
    pic.check(L.pic_deposit_noalloc(t.handle, scheme, prec, C.byref(P), C.c_void_p(st.start.data_ptr()), q, qu,
                                    C.c_void_p(got.data_ptr()), s), "pic_deposit_noalloc")
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


def _stepped(spec, x, v, scheme, q=None, f32=False, dt=0.5):
    t = pic.Tree(spec).upload()
    if f32:
        st = pic.Stepper32(t, scheme, x, v, dt=dt, q=q)
    else:
        st = pic.Stepper(t, scheme, x, v, q=q)
        st.initial_sort()
    E = torch.tensor(W.random_field(np.random.default_rng(4), spec.dim, t.n_vertices, 0.3), device="cuda")
    st.step_fused(E, -0.5, dt, q_uniform=-1.0 / st.n)
    torch.cuda.synchronize()
    return t, st


@pytest.mark.gpu
@pytest.mark.parametrize("scheme", [pic.PIT, pic.PIDT])
def test_noalloc_deposit_equals_deposit_on_consecutive_calls(scheme):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    print(f"[no_alloc] scheme {scheme}", flush=True)
    big = W.config1()
    t1, s1 = _stepped(big.tree, big.x, big.v, scheme)
    rng = np.random.default_rng(9)
    t2, s2 = _stepped(W.regular_tree(2, 2), rng.random((2, 500)), 0.05 * rng.standard_normal((2, 500)), scheme)
    for t, st in ((t1, s1), (t2, s2)):
        ref, got = _deposit_both(t, scheme, st)
        assert np.isfinite(ref).all()
        assert np.array_equal(ref.view(np.uint64), got.view(np.uint64))
        assert t.status_sync() == 0
    # the charge also meets the oracle bound for the second (smaller) set
    o = oracle.OracleTree(W.regular_tree(2, 2))
    rho_o = o.deposit(s2.x.cpu().numpy(), None, -1.0 / s2.n)
    assert (np.abs(got - rho_o) <= 1e-12 * np.abs(rho_o) + 1e-300).all()


@pytest.mark.gpu
@pytest.mark.parametrize("scheme", [pic.PIT, pic.PIDT])
def test_noalloc_deposit_fp32_and_charges(scheme):
    """The FP32 form and per-particle charges go through the same array."""
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    print(f"[no_alloc] fp32/q scheme {scheme}", flush=True)
    wl = W.small_adaptive()
    t, st = _stepped(wl.tree, wl.x, wl.v, scheme, q=wl.q)
    ref, got = _deposit_both(t, scheme, st)
    assert np.array_equal(ref.view(np.uint64), got.view(np.uint64))
    c1 = W.config1()
    t32, s32 = _stepped(c1.tree, c1.x, c1.v, scheme, f32=True)
    ref, got = _deposit_both(t32, scheme, s32, f32=True)
    assert np.array_equal(ref.view(np.uint64), got.view(np.uint64))
    assert t.status_sync() == 0 and t32.status_sync() == 0


def test_noalloc_deposit_refuses_trees_beyond_its_array():
    """A 3D depth-4 tree's PIDT partials (531441 bins x 27 slots x 8 bytes)
    exceed the array: PIC_E_SCRATCH, checked on the host before the device
    is touched; its PIT partials fit (the tree is not uploaded, so the call
    then reports the missing upload)."""
    t = pic.Tree(W.regular_tree(3, 4))
    P = _capi.Particles()
    P.n = 10
    P.x[0], P.x[1], P.x[2] = 0x1000, 0x2000, 0x3000
    L = _capi.lib()
    start, rho = C.c_void_p(0x4000), C.c_void_p(0x5000)
    assert 531441 * 27 * 8 > _capi.NOALLOC_SCRATCH_BYTES >= 531441 * 8 * 8
    assert L.pic_deposit_noalloc(t.handle, pic.PIDT, pic.F64, C.byref(P), start, None, -1.0, rho, None) \
        == _capi.PIC_E_SCRATCH
    assert L.pic_deposit_noalloc(t.handle, pic.PIT, pic.F64, C.byref(P), start, None, -1.0, rho, None) \
        == _capi.PIC_E_STATE
    assert L.pic_deposit_noalloc(t.handle, pic.PIT, pic.F64, C.byref(P), None, None, -1.0, rho, None) \
        == _capi.PIC_E_ARG
