"""GPU checks of the solver's other behaviours through the C ABI: batching,
resume, graph replay of every path, energies, the stable time step, damage,
failure detection and full-size short runs against the CPU reference."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import Oracle  # noqa: E402
from pd_inputs import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_11273_amd.solver import Context
    return Context(0)


def solver(w, ctx, **kw):
    from paper_2309_11273_amd.solver import Solver
    return Solver(w, ctx=ctx, **kw)


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def test_batch_member_equals_single_specimen(ctx):
    """Plate k of a batch advances exactly as the same plate alone (double
    path, bitwise): specimens share no bonds and each row's sum order depends
    only on its own family."""
    dts = np.array([1.0e-7, 1.1e-7, 0.9e-7])
    wb = W.batch2d(n_plates=3, steps=150, dt=dts)
    sb = solver(wb, ctx)
    sb.step(150, precision="fp64")
    ub, _ = sb.read()
    for k in range(3):
        w1 = W.batch2d(n_plates=1, first=k, steps=150, dt=dts[k:k + 1])
        s1 = solver(w1, ctx)
        s1.step(150, precision="fp64")
        u1, _ = s1.read()
        uk = ub[wb.specimen == k]
        assert np.array_equal(uk[:, :2], u1[:, :2]), k


def test_resume_equals_uninterrupted(ctx):
    """Stopping after n1 steps and restarting a new state from (u, v, bond
    status, step counter) gives bitwise the uninterrupted trajectory."""
    w = W.plate2d(nx=48, ny=24, dt=1.347e-7, sigma=12e6, notch_row=11, notch_tip=23.37, steps=200)
    a = solver(w, ctx)
    a.step(200, precision="fp64")
    ua, va = a.read()
    b = solver(w, ctx)
    b.step(120, precision="fp64")
    u1, v1 = b.read()
    m1 = b.mask_host()
    c = solver(w, ctx, u0=u1)
    c.reset(u0=u1, v0=v1, start_step=120, mask=m1)
    c.step(80, precision="fp64")
    uc, vc = c.read()
    assert np.array_equal(ua, uc)
    assert np.array_equal(va, vc)
    assert np.array_equal(a.mask_host(), c.mask_host())
    assert c.step_count() == 200


@pytest.mark.parametrize("precision,form", [("fp32", "mf"), ("fp64", "bsr")])
def test_graph_replay_equals_eager_all_paths(ctx, precision, form):
    w = W.impact3d(nx=36, ny=36, nz=9, dt=2.6e-7, steps=120)
    a = solver(w, ctx)
    b = solver(w, ctx)
    if form == "bsr":
        for s in (a, b):
            s.build_K(fp32=False)
            s.assemble_K()
    a.step(120, precision=precision, form=form)
    for _ in range(3):
        b.step(40, precision=precision, form=form, graph_chunk=10)
    ua, _ = a.read()
    ub, _ = b.read()
    # the FP32 path keeps its shadow, scale and D_i between calls: the same bits
    assert np.array_equal(ua, ub)
    assert np.array_equal(a.mask_host(), b.mask_host())


@pytest.mark.parametrize("kernel", ["tiled", "gather", "super", "super3d"])
def test_fp32_split_calls_equal_one_call(ctx, kernel):
    """An FP32 trajectory is the same bits however its steps are split into
    calls (1 + 7 + 30 + 62 eager steps against 100 in one call), on a plate
    that breaks bonds (super3d: the cracking-free impact plate with its
    16.5 m/s edge)."""
    if kernel == "super3d":
        kernel = "super"
        w = W.impact3d(nx=36, ny=36, nz=9, dt=2.6e-7, steps=100)
    else:
        w = W.plate2d(nx=48, ny=24, dt=1.347e-7, sigma=12e6, notch_row=11, notch_tip=23.37, steps=100)
    a = solver(w, ctx)
    b = solver(w, ctx)
    a.step(100, precision="fp32", kernel=kernel)
    for n in (1, 7, 30, 62):
        b.step(n, precision="fp32", kernel=kernel)
    assert np.array_equal(a.read()[0], b.read()[0])
    assert np.array_equal(a.mask_host(), b.mask_host())
    assert b.bond_status()[2].size and int((b.bond_status()[2] == 0).sum()) > 0
    if kernel == "super":
        assert a.fam.st_tiles is not None


def test_fp32_shadow_rebuilt_after_other_paths(ctx):
    """A step of another path in between invalidates the kept shadow: FP64
    steps, then FP32 steps, equal a fresh state resumed from the FP64 state
    (where the set-up runs anyway)."""
    w = W.impact3d(nx=36, ny=36, nz=9, dt=2.6e-7, steps=60)
    a = solver(w, ctx)
    a.step(20, precision="fp32")
    a.step(20, precision="fp64")
    u1, v1 = a.read()
    m1 = a.mask_host()
    a.step(20, precision="fp32")
    b = solver(w, ctx)
    b.reset(u0=u1, v0=v1, start_step=40, mask=m1)
    b.step(20, precision="fp32")
    assert np.array_equal(a.read()[0], b.read()[0])


@pytest.mark.parametrize("order", [("tiled", "gather", "tiled"), ("gather", "tiled", "gather"),
                                   ("super", "tiled", "super")])
def test_fp32_kernel_kinds_in_turn(ctx, order):
    """FP32 steps of the tile, super-tile and gather kernels in turn on one
    state (the shadow rebuilt at every change of kind, its maximum kept in the
    word and in the tile kernels' slots) follow the reference on a plate that
    breaks bonds: rel-L2 <= 1e-4 and identical broken sets."""
    w = W.plate2d(nx=48, ny=24, dt=1.347e-7, sigma=12e6, notch_row=11, notch_tip=23.37, steps=300)
    s = solver(w, ctx)
    if "super" in order and s.fam.st_tiles is None:
        pytest.skip("no super-tiles for this family")
    o = Oracle(w)
    uo, vo = o.initial_state()
    cut0 = int((o.rho() == 0).sum())  # notch cuts
    for kern in order:
        s.step(100, precision="fp32", kernel=kern)
    o.run(300, uo, vo)
    u, _ = s.read()
    assert rel(u, uo) <= 1e-4
    assert int((o.rho() == 0).sum()) > cut0  # bonds broke
    assert np.array_equal(s.bond_status()[2], o.rho())
    assert s.step_count() == 300


def test_graph_cache_with_two_problems_on_one_context(ctx):
    """Captured step graphs are keyed on every launch parameter: problems of
    different shape and size stepped in turn on one context with graph
    replay each follow the reference, also after a solver is freed and a new
    one may land on the old addresses."""
    wa = W.plate2d(nx=48, ny=24, dt=1.347e-7, sigma=12e6, notch_row=11, notch_tip=23.37, steps=120)
    wb = W.impact3d(nx=36, ny=36, nz=9, dt=2.6e-7, steps=120)
    wc = W.plate2d(nx=40, ny=24, dt=1.2e-7, sigma=8e6, notch_row=10, notch_tip=19.37, steps=120)
    oa, ob, oc = Oracle(wa), Oracle(wb), Oracle(wc)
    sa, sb = solver(wa, ctx), solver(wb, ctx)
    ua, va = oa.initial_state()
    ub, vb = ob.initial_state()
    for _ in range(3):
        sa.step(40, precision="fp64", graph_chunk=20)
        oa.run(40, ua, va)
        sb.step(40, precision="fp64", graph_chunk=20)
        ob.run(40, ub, vb)
        assert rel(sa.read()[0], ua) <= 1e-10
        assert rel(sb.read()[0], ub) <= 1e-10
    assert np.array_equal(sa.bond_status()[2], oa.rho())
    del sa
    torch.cuda.synchronize()
    sc = solver(wc, ctx)
    uc, vc = oc.initial_state()
    for _ in range(3):
        sc.step(40, precision="fp64", graph_chunk=20)
        oc.run(40, uc, vc)
        assert rel(sc.read()[0], uc) <= 1e-10
    assert np.array_equal(sc.bond_status()[2], oc.rho())


def test_energy_matches_reference(ctx):
    w = W.cantilever3d(steps=300)
    s = solver(w, ctx)
    o = Oracle(w)
    s.step(300, precision="fp64")
    u, v = s.read()
    kin, strain = s.energy()
    rho = w.materials[0].rho
    kin_ref = 0.5 * (rho * w.vol[:, None] * v * v).sum()
    strain_ref = o.strain_energy(u)
    assert kin == pytest.approx(kin_ref, rel=1e-12)
    assert strain == pytest.approx(strain_ref, rel=1e-10)


def test_energies_are_repeatable_and_match_reference(ctx):
    """pd_energy (Eq. 1.20, fixed-order sums) gives the same bits on every
    call and agrees with the reference's energy; the step's energy check
    reports the same numbers."""
    w = W.plate2d(nx=48, ny=24, dt=1.347e-7, sigma=12e6, notch_row=11, notch_tip=23.37, steps=150)
    s = solver(w, ctx)
    rep = s.step(150, precision="fp64", energy_check=True)
    u, v = s.read()
    e1, e2 = s.energy(), s.energy()
    assert e1 == e2
    o = Oracle(w)
    o.set_rho(s.bond_status()[2])
    rho = w.materials[0].rho
    assert e1[0] == pytest.approx(0.5 * (rho * w.vol[:, None] * v * v).sum(), rel=1e-12)
    assert e1[1] == pytest.approx(o.strain_energy(u), rel=1e-12)
    assert (rep["kinetic"], rep["strain"]) == e1
    assert rep["energy_step"] == 150
    assert rep["min_margin"] == float("inf")  # the FP64 path rechecks nothing


def test_energy_growth_is_reported_as_unstable(ctx):
    """A step beyond the stability limit (1.3 x 2/omega_max on the
    cantilever) makes the energy grow geometrically; the energy check stops
    the run with PD_ERR_UNSTABLE while the state is still finite, long before
    a non-finite value appears.  Every kernel exits normally."""
    from paper_2309_11273_amd._abi import PDError
    w = W.cantilever3d(steps=400, dt=1.3 * 2.814e-7)
    s = solver(w, ctx)
    for prec in ("fp64", "fp32"):
        s.reset()
        with pytest.raises(PDError) as ei:
            s.step(400, precision=prec, check_every=10, energy_check=True)
        assert ei.value.status == -4 and "energy grew" in str(ei.value), prec
        u, _ = s.read()
        assert np.all(np.isfinite(u)), prec
    # the stable step runs through with the same checks
    s2 = solver(W.cantilever3d(steps=400), ctx)
    rep = s2.step(400, precision="fp64", check_every=10, energy_check=True)
    assert rep["energy_step"] == 400 and rep["kinetic"] > 0


def test_fp32_reports_min_recheck_margin(ctx):
    """The FP32 path reports the smallest breaking margin among the bonds it
    decided in double; the reference saw a margin at least as small over all
    bonds (up to the single-precision error of the state)."""
    w = W.plate2d(nx=48, ny=24, dt=1.347e-7, sigma=12e6, notch_row=11, notch_tip=23.37, steps=300)
    s = solver(w, ctx)
    rep = s.step(300, precision="fp32")
    o = Oracle(w)
    uo, vo = o.initial_state()
    o.run(300, uo, vo)
    assert rep["rechecks"] > 0
    assert np.isfinite(rep["min_margin"]) and rep["min_margin"] >= 0.0
    assert rep["min_margin"] >= o.min_margin() - 1e-4


def test_stable_dt_matches_reference(ctx):
    """pd_stable_dt (power iteration on the GPU operator) agrees with the
    CPU reference's power iteration and the dense eigenvalue."""
    w = W.cantilever3d()
    s = solver(w, ctx)
    dt_gpu = s.stable_dt(iters=500, seed=0)
    o = Oracle(w, apply_cuts=False)
    lam = o.lambda_max(500, 0)
    assert dt_gpu == pytest.approx(2 / np.sqrt(lam), rel=1e-6)
    assert w.dt[0] < 0.8 * dt_gpu * 1.0001


def test_nonfinite_state_is_reported(ctx):
    """A non-finite displacement is caught at the next check and reported
    as PD_ERR_UNSTABLE (forced from the host: NaN in the initial state)."""
    from paper_2309_11273_amd._abi import PDError
    w = W.plate2d(nx=24, ny=12, dt=1.0e-7, notch_row=5, notch_tip=10.37, steps=20)
    u0 = np.zeros((w.n, 3))
    u0[7, 0] = np.nan
    s = solver(w, ctx, u0=u0)
    with pytest.raises(PDError) as ei:
        s.step(10, precision="fp64", check_every=5)
    assert ei.value.status == -4


def test_wrong_uniform_volume_is_reported(ctx):
    """A vol_uniform that differs from the node volumes is caught by the FP32
    tile pass 1, which checks every node it stages, and fails the report
    with PD_ERR_ARG (forced from the host: the problem's constant altered)."""
    from paper_2309_11273_amd._abi import PDError
    w = W.impact3d(nx=24, ny=24, nz=9, dt=2.4e-7, steps=20)
    s = solver(w, ctx)
    assert s.P.vol_uniform == np.float32(w.dx ** 3)
    s.step(2, precision="fp32", kernel="tiled")  # the constant as the family gives it
    s.P.vol_uniform = float(np.float32(w.dx ** 3)) * 1.5
    with pytest.raises(PDError) as ei:
        s.step(2, precision="fp32", kernel="tiled", report=True)
    assert ei.value.status == -1


def test_damage_matches_reference(ctx):
    w = W.plate2d(nx=48, ny=24, dt=1.347e-7, sigma=12e6, notch_row=11, notch_tip=23.37, steps=250)
    s = solver(w, ctx)
    o = Oracle(w)
    s.step(250, precision="fp64")
    uo, vo = o.initial_state()
    o.run(250, uo, vo)
    phi = s.damage()
    np.testing.assert_allclose(phi, o.damage(), rtol=0, atol=1e-15)
    assert phi.max() > 0.3


@pytest.mark.parametrize("name,steps", [("impact3d", 6), ("cylinder3d", 4), ("batch2d", 6)])
def test_full_size_short_run(ctx, name, steps):
    """The full workloads in the launch configuration the benchmark times
    (FP32 force path, graph replay) for a few steps: displacement within the
    FP32 bar of the CPU reference, broken-bond set identical."""
    w = W.workload(name)
    s = solver(w, ctx)
    s.step(steps, precision="fp32", graph_chunk=2)
    u, _ = s.read()
    o = Oracle(w)
    uo, vo = o.initial_state()
    o.run(steps, uo, vo)
    assert rel(u, uo) <= 1e-4
    assert np.array_equal(s.bond_status()[2], o.rho())


def test_autotune_picks_a_measured_candidate(ctx, tmp_path):
    w = W.impact3d(nx=36, ny=36, nz=9, dt=2.6e-7, steps=50)
    s = solver(w, ctx)
    cache = str(tmp_path / "tune.json")
    r = s.autotune("fp32", trial_steps=5, cache=cache)
    ms = [c["ms"] for c in r["candidates"]]
    # tile kernels, super-tile kernels, gather at 64/128/256
    assert len(ms) == 5 and min(ms) == r["ms_per_step"]
    assert r["kernel"] in ("tiled", "super", "gather")
    # 2D: the tile kernels with one tile per wave and with one per workgroup
    w2 = W.plate2d(nx=48, ny=24, dt=1.347e-7, sigma=12e6, notch_row=11, notch_tip=23.37, steps=50)
    s2 = solver(w2, ctx)
    r2 = s2.autotune("fp32", trial_steps=5)
    assert sorted(c["kernel"] for c in r2["candidates"]) == [1, 1, 1, 2, 3, 4]
    assert r2["kernel"] in ("tiled", "super", "gather", "tiled1")
    # cached result is reused and the state was reset
    assert s.autotune("fp32", trial_steps=5, cache=cache) == r
    assert s.step_count() == 0
    r64 = s.autotune("fp64", trial_steps=5)
    assert len(r64["candidates"]) == 4 and min(c["ms"] for c in r64["candidates"]) == r64["ms_per_step"]
    assert (r64["kernel"], r64["block"]) in [("tiled", 0), ("gather", 64), ("gather", 128), ("gather", 256)]
