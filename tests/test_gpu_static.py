"""Static equilibrium on the GPU (preconditioned conjugate gradients with
the assembled block-sparse stiffness of Eq. 2.14), through the C ABI,
against the CPU reference's direct sparse solve of the same equations.

Bar: |u - u_ref| / |u_ref| <= max(1e-10, 10 cond(K_ff) |r| / |r0|), the
error bound of a linear solve stopped at relative residual |r| / |r0|
(cond from the reference's dense K on the small cases; the cylinder uses
the residual it reaches, 1e-13, and a bound of 1e-8)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import Oracle, dense  # noqa: E402
from pd_inputs import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_11273_amd.solver import Context
    return Context(0)


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def static_solver(w, ctx, u0=None):
    from paper_2309_11273_amd.solver import Solver
    s = Solver(w, ctx=ctx, u0=u0)
    s.build_K(fp32=False)
    s.assemble_K()
    return s


def clamped_plate():
    """The notched plate with its left edge clamped (static problem with a
    unique solution); the traction on the long edges stays."""
    w = W.plate2d(nx=48, ny=24, dt=1.347e-7, sigma=1e6, notch_row=11, notch_tip=23.37)
    w.bc = w.bc.copy()
    w.bc[w.lat[:, 0] == 0] = 3
    return w


@pytest.mark.parametrize("op", ["stored_K", "matrix_free", "no_K"])
@pytest.mark.parametrize("name", ["cantilever", "plate_clamped"])
def test_static_solution_matches_direct_solve(ctx, name, op):
    w = W.cantilever3d() if name == "cantilever" else clamped_plate()
    o = Oracle(w)
    ref = dense.static_solution(w, o, rho_bond=o.rho())
    L, _ = dense.internal_force_operator(w, rho_bond=o.rho())
    free = dense.free_dofs(w)
    ev = np.linalg.eigvalsh(-L[np.ix_(free, free)])
    cond = ev[-1] / ev[0]
    s = static_solver(w, ctx)
    rep = s.static_solve(tol=1e-13, max_iter=20000, matrix_free=op != "stored_K", use_K=op != "no_K")
    assert rep["converged"], rep
    u, _ = s.read()
    assert rel(u, ref) <= max(1e-10, 10 * cond * rep["rel_residual"]), (rel(u, ref), cond, rep)


@pytest.mark.parametrize("op", ["stored_K", "matrix_free", "no_K"])
def test_cylinder_torsion_static(ctx, op):
    """Small cylinder (dx = 5 mm) with its end layers turned by a prescribed
    rotation: the interior equilibrium against the direct solve."""
    w = W.cylinder3d(dx=5e-3, dt=2.4e-7, twist_rate=8.0, steps=10)
    u0 = w.v0 * 1e-4
    o = Oracle(w)
    ref = dense.static_solution(w, o, u0=u0, rho_bond=o.rho())
    s = static_solver(w, ctx, u0=u0)
    rep = s.static_solve(tol=1e-13, max_iter=50000, matrix_free=op != "stored_K", use_K=op != "no_K")
    assert rep["converged"], rep
    u, _ = s.read()
    assert rel(u, ref) <= 1e-8, (rel(u, ref), rep)
    # prescribed components untouched, and a second solve from the solution
    # changes it only by its remaining residual
    pres = np.asarray(w.bc) != 0
    assert np.array_equal(u[pres], u0[pres])
    s.static_solve(tol=1e-6, max_iter=200, check_every=1)
    u2, _ = s.read()
    assert rel(u2, u) <= 1e-8


def test_static_solve_is_deterministic(ctx):
    w = clamped_plate()
    outs = []
    for _ in range(2):
        s = static_solver(w, ctx)
        s.static_solve(tol=1e-12)
        outs.append(s.read()[0])
    assert np.array_equal(outs[0], outs[1])


def test_static_solve_checks(ctx):
    from paper_2309_11273_amd import _abi as A
    w = W.cantilever3d()
    from paper_2309_11273_amd.solver import Solver
    s = Solver(w, ctx=ctx)
    s.build_K(fp32=True)
    s.assemble_K()
    with pytest.raises(A.PDError):
        s.static_solve()
    s.build_K(fp32=False)
    with pytest.raises(A.PDError):  # not assembled
        s.static_solve()


@pytest.mark.parametrize("name", ["cantilever", "plate_broken"])
def test_diagonal_from_bonds_equals_stored_K(ctx, name):
    """The block-Jacobi diagonal summed from the bonds (no stored K) equals
    the one taken from the assembled K, block inverses compared entry by
    entry, with broken bonds in the plate."""
    import torch
    if name == "cantilever":
        w = W.cantilever3d()
    else:
        w = W.plate2d(nx=48, ny=24, dt=1.347e-7, sigma=12e6, notch_row=11, notch_tip=23.37, steps=300)
    s = static_solver(w, ctx)
    if name == "plate_broken":
        s.step(200, precision="fp64", form="bsr")  # breaks bonds and re-assembles K
        st = s.bond_status()[2]
        assert 0 < (st == 0).sum() < st.size
    n = s.n_pad
    s.static_solve(tol=1e-3, max_iter=1)
    d_k = s._cg_work[20 * n:32 * n].clone()
    s.static_solve(tol=1e-3, max_iter=1, matrix_free=True, use_K=False)
    d_b = s._cg_work[20 * n:32 * n].clone()
    torch.cuda.synchronize()
    a, b = d_k.cpu().numpy(), d_b.cpu().numpy()
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max(), np.abs(a - b).max() / np.abs(a).max()
