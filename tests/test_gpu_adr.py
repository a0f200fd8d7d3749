"""Parity of the adaptive dynamic relaxation (the quasi-static solver of the
paper's Example 4) on the GPU, through the C ABI, with the FP64 CPU
reference: the fictitious density, the iterates (u, v), the adaptive
damping and the broken-bond set, and the cantilever's static solution."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import Oracle, dense  # noqa: E402
from pd_inputs import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_11273_amd.solver import Context
    return Context(0)


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def relax_solver(w, ctx, dt=1.0):
    from paper_2309_11273_amd.solver import Solver
    s = Solver(w, ctx=ctx)
    s.adr_setup(dt)
    return s


def ramped_plate():
    """Notched plate whose 12 MPa traction rises over 400 iterations: bonds
    break progressively while the relaxation follows the load."""
    w = W.plate2d(nx=48, ny=24, dt=1.347e-7, sigma=12e6, notch_row=11, notch_tip=23.37, steps=450)
    w.ramp_steps = 400
    return w


def cases():
    r2 = W.impact3d(nx=36, ny=36, nz=9, dt=1.6e-7, steps=200)
    r2.delta = 2.015 * r2.dx
    return {
        "cantilever": W.cantilever3d(),
        "plate_notched": W.plate2d(nx=48, ny=24, dt=1.347e-7, sigma=12e6, notch_row=11, notch_tip=23.37),
        "impact": W.impact3d(nx=36, ny=36, nz=9, dt=2.6e-7, steps=200),
        "impact_r2": r2,
        "cylinder": W.cylinder3d(dx=2.5e-3, dt=2.4e-7, twist_rate=8.0, steps=200),
        "batch": W.batch2d(n_plates=3, steps=200, dt=np.array([1.0e-7, 1.1e-7, 0.9e-7])),
    }


@pytest.mark.parametrize("name", ["cantilever", "plate_notched", "impact", "impact_r2", "cylinder", "batch"])
def test_density_matches_reference(ctx, name):
    w = cases()[name]
    s = relax_solver(w, ctx, dt=0.8)
    lam = s.adr_lambda()
    lo = Oracle(w).adr_density(0.8)
    if w.dim == 2:
        lam, lo = lam[:, :2], lo[:, :2]
    assert np.abs(lam - lo).max() <= 1e-13 * np.abs(lo).max()


@pytest.mark.parametrize("kernel", ["tiled", "gather"])
def test_cantilever_relaxation(ctx, kernel):
    """The first iterations follow the reference (u, v, damping); the
    relaxed state equals the reference's and the direct solution of
    K u = F_ext.  Iterates in between are not compared: the damping divides
    force differences by velocities that pass through zero, which amplifies
    a change of summation order (the reference disagrees with itself under
    another reduction order, tests/test_oracle_pins.py)."""
    w = W.cantilever3d()
    o = Oracle(w)
    st = o.adr_start()
    s = relax_solver(w, ctx)
    done = 0
    for target in (1, 2, 5, 10, 20):
        s.adr_step(target - done, kernel=kernel)
        o.adr_run(target - done, st)
        done = target
        u, v = s.read()
        assert rel(u, st["u"]) <= FP64_TOL, (target, rel(u, st["u"]))
        assert rel(v, st["v"]) <= FP64_TOL, (target, rel(v, st["v"]))
        g = s.adr_stats()
        assert g["iterations"] == target
        assert g["c"] == pytest.approx(st["stats"][0], rel=1e-10, abs=1e-300)
        assert g["uu"] == pytest.approx(st["stats"][2], rel=1e-10)
        assert g["res2"] == pytest.approx(st["stats"][3], rel=1e-10)
    s.adr_step(3000 - done, kernel=kernel)
    o.adr_run(3000 - done, st)
    u, _ = s.read()
    assert rel(u, st["u"]) <= FP64_TOL
    L, _ = dense.internal_force_operator(w)
    free = dense.free_dofs(w)
    F = np.asarray(w.fext).reshape(-1)
    us = np.zeros(3 * w.n)
    us[free] = np.linalg.solve(-L[np.ix_(free, free)], F[free])
    assert rel(u.reshape(-1), us) <= FP64_TOL


def test_relaxation_with_breaking(ctx):
    """A 12 MPa traction applied at once on the notched plate: about a
    thousand bonds break during the first fifteen iterations; iterates and
    broken-bond sets follow the reference through them."""
    w = W.plate2d(nx=48, ny=24, dt=1.347e-7, sigma=12e6, notch_row=11, notch_tip=23.37, steps=20)
    o = Oracle(w)
    st = o.adr_start()
    s = relax_solver(w, ctx)
    n0 = int(o.rho().sum())
    done = 0
    for target in (3, 5, 8, 10, 15, 20):
        s.adr_step(target - done)
        o.adr_run(target - done, st)
        done = target
        u, _ = s.read()
        assert rel(u, st["u"]) <= FP64_TOL, (target, rel(u, st["u"]))
        _, _, bs = s.bond_status()
        assert np.array_equal(bs, o.rho()), (target, int((bs != o.rho()).sum()))
    assert n0 - int(o.rho().sum()) > 500


def test_graph_replay_equals_eager(ctx):
    w = ramped_plate()
    a = relax_solver(w, ctx)
    b = relax_solver(w, ctx)
    a.adr_step(240)
    for _ in range(3):
        b.adr_step(80, graph_chunk=20)
    assert np.array_equal(a.read()[0], b.read()[0])
    assert np.array_equal(a.mask_host(), b.mask_host())
    assert a.adr_stats() == b.adr_stats()


def test_restart_by_density(ctx):
    """pd_adr_density restarts the relaxation: the first iteration rule
    applies again."""
    w = W.cantilever3d()
    s = relax_solver(w, ctx)
    s.adr_step(10)
    s.reset()
    s.adr_setup()
    s.adr_step(1)
    g = s.adr_stats()
    assert g["first"] == 1.0 and g["iterations"] == 1


def test_full_size_cylinder_short_run(ctx):
    """The full cylinder (911,319 nodes) for a few relaxation iterations in
    the launch configuration the benchmark times (graph replay)."""
    w = W.workload("cylinder3d")
    s = relax_solver(w, ctx)
    s.adr_step(4, graph_chunk=2)
    u, _ = s.read()
    o = Oracle(w)
    st = o.adr_start()
    o.adr_run(4, st)
    assert rel(u, st["u"]) <= FP64_TOL
    assert np.array_equal(s.bond_status()[2], o.rho())
