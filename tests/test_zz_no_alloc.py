"""pd_energy_noalloc, the entry point for callers that cannot allocate,
against pd_energy through the C ABI: the same bits on two calls in a row,
the second on a smaller problem, and the row limit of its fixed array."""

import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from pd_inputs import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


def test_energy_noalloc_equals_pd_energy():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_11273_amd.solver import Context, Solver
    ctx = Context(0)
    big = W.impact3d(nx=72, ny=72, nz=9, dt=2.6e-7, steps=80)
    small = W.plate2d(nx=48, ny=24, dt=1.347e-7, sigma=12e6, notch_row=11, notch_tip=23.37, steps=80)
    sizes = []
    for w in (big, small):
        s = Solver(w, ctx=ctx)
        s.step(80, precision="fp64", report=False)
        out = torch.full((2,), np.nan, dtype=torch.float64, device=s.dev)
        s.energy_noalloc(out)
        torch.cuda.synchronize()
        got = tuple(out.cpu().numpy().tolist())
        ref = s.energy()
        assert got == ref, (w.name, got, ref)
        assert ref[0] > 0.0 and ref[1] > 0.0
        sizes.append(s.n_pad)
    assert sizes[1] < sizes[0]


def test_energy_noalloc_rejects_rows_beyond_its_array():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_11273_amd import _abi as A
    from paper_2309_11273_amd.solver import Context, Solver
    ctx = Context(0)
    w = W.plate2d(nx=24, ny=12, dt=1.0e-7, notch_row=5, notch_tip=10.37, steps=10)
    s = Solver(w, ctx=ctx)
    P = A.pd_problem_dev()
    C.memmove(C.byref(P), C.byref(s.P), C.sizeof(P))
    P.n_pad = (1 << 24) + 64  # one slice past the limit; checked on the host only
    P.n_slices = P.n_pad // 64
    out = torch.zeros(2, dtype=torch.float64, device=s.dev)
    st = A.load().pd_energy_noalloc(ctx.h, C.byref(P), C.byref(s.S), C.c_void_p(out.data_ptr()))
    assert st == -2
    assert b"exceeds" in A.load().pd_last_error(ctx.h)
