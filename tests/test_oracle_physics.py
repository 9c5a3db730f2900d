"""Whole-run pins of the oracle: single-level reduction to textbook BGK,
conservation, invariance of uniform states on refined meshes, the sound speed
and viscosity closed forms, symmetry, the shared-equilibrium identity at
co-located nodes, and agreement with a uniform-fine run.  CPU only."""
import numpy as np
import pytest

import oracle as O
from paper_2004_14887_amd import workloads as W

CS2 = 1.0 / 3.0


def make(wl, plant_R=None):
    o = O.Oracle(wl.lattice, wl.n0, wl.boxes, wl.tau0, wl.coupling, wl.eq_order, wl.probes,
                 probe_capacity=max(1, wl.steps))
    if plant_R is not None:
        o.plant_R(plant_R)
    for l in range(wl.n_levels):
        rho, u = W.initial_fields(wl, l)
        o.init(l, rho, u)
    return o


def macros(o, l):
    xi, _ = O.lattice_table(o.lattice)
    f = o.f(l)
    rho = f.sum(0)
    u = (xi[:, :o.D].T.astype(float) @ f) / rho
    return rho, u


# ------------------------------------------------------------------ textbook BGK
def _textbook_bgk(f, xi, w, tau, steps, dims):
    """Standard periodic stream-and-collide (the state is post-collision) with the usual
    textbook equilibrium
    w rho (1 + 3 e.u + 9/2 (e.u)^2 - 3/2 u.u), written independently."""
    D = len(dims)
    f = f.reshape((len(w),) + tuple(reversed(dims)))
    for _ in range(steps):
        for i in range(len(w)):
            shift = tuple(int(xi[i, a]) for a in reversed(range(D)))
            f[i] = np.roll(f[i], shift, axis=tuple(range(D)))
        rho = f.sum(0)
        u = [np.tensordot(xi[:, a].astype(float), f, axes=1) / rho for a in range(D)]
        uu = sum(c * c for c in u)
        for i in range(len(w)):
            eu = sum(xi[i, a] * u[a] for a in range(D))
            feq = w[i] * rho * (1 + 3 * eu + 4.5 * eu * eu - 1.5 * uu)
            f[i] = f[i] - (f[i] - feq) / tau
    return f.reshape(len(w), -1)


@pytest.mark.parametrize("lat,n0", [("D2Q9", (24, 20)), ("D3Q19", (10, 12, 8))])
def test_single_level_is_textbook_bgk(lat, n0):
    rng = np.random.default_rng(1)
    wl = W.Workload("t", lat, n0, [], 0.57, 12)
    o = O.Oracle(lat, n0, [], tau0=0.57)
    n = int(np.prod(n0))
    D = len(n0)
    rho = 1 + 1e-2 * rng.normal(size=n)
    u = 0.03 * rng.normal(size=(D, n))
    o.init(0, rho, u)
    f_init = o.f(0)
    o.run(12)
    xi, w = O.lattice_table(lat)
    ref = _textbook_bgk(f_init.copy(), xi[:, :D], w, 0.57, 12, n0)
    assert np.abs(o.f(0) - ref).max() < 1e-14
    assert wl.n_levels == 1


@pytest.mark.parametrize("lat,n0", [("D2Q9", (32, 24)), ("D3Q19", (12, 10, 8))])
def test_single_level_conserves_mass_and_momentum(lat, n0):
    rng = np.random.default_rng(2)
    o = O.Oracle(lat, n0, [], tau0=0.53)
    n = int(np.prod(n0))
    D = len(n0)
    o.init(0, 1 + 1e-2 * rng.normal(size=n), 0.05 * rng.normal(size=(D, n)))
    b0 = o.balance()
    o.run(30)
    b1 = o.balance()
    assert abs(b1[0] - b0[0]) < 1e-12 * b0[0]
    assert np.abs(b1[1:1 + D] - b0[1:1 + D]).max() < 1e-12 * b0[0]


# ------------------------------------------------------------------ uniform states on refined meshes
@pytest.mark.parametrize("coupling", [1, 2])
@pytest.mark.parametrize("eq_order", [2, 3])
@pytest.mark.parametrize("case", ["2d3", "3d2"])
def test_uniform_states_stay_exact_on_refined_meshes(coupling, eq_order, case):
    if case == "2d3":
        lat, n0, boxes, steps = "D2Q9", (32, 32), [((8, 8), (24, 24)), ((8, 8), (24, 24))], 6
    else:
        lat, n0, boxes, steps = "D3Q19", (16, 16, 16), [((4, 4, 4), (12, 12, 12))], 3
    D = len(n0)
    for u0 in [(0.0, 0.0, 0.0), (0.05, -0.03, 0.02)]:
        wl = W.uniform_state(lat, n0, boxes, u0=u0[:D], coupling=coupling)
        wl.eq_order = eq_order
        o = make(wl)
        f0 = [o.f(l) for l in range(wl.n_levels)]
        o.run(steps)
        for l in range(wl.n_levels):
            assert np.nanmax(np.abs(o.f(l) - f0[l])) < 2e-15, (l, u0)


# ------------------------------------------------------------------ closed forms
def test_sound_speed_is_one_over_root_three():
    # a plane Gaussian pulse splits into two waves travelling at c_s = 1/sqrt(3)
    n0 = (512, 8)
    wl = W.Workload("p", "D2Q9", n0, [], 0.51, 1)
    o = O.Oracle("D2Q9", n0, [], tau0=0.51)
    pos = W.node_positions(wl, 0)
    rho = 1 + 1e-4 * np.exp(-((pos[0] - 256.0) ** 2) / (2 * 8.0 ** 2))
    o.init(0, rho, np.zeros((2, pos.shape[1])))
    T = 150
    o.run(T)
    r = macros(o, 0)[0].reshape(8, 512)[0] - 1
    k = 256 + int(np.argmax(r[256:]))
    a, b, c = r[k - 1], r[k], r[k + 1]
    peak = k + 0.5 * (a - c) / (a - 2 * b + c)
    cs = (peak - 256.0) / T
    assert cs == pytest.approx(np.sqrt(CS2), rel=5e-3)


def test_shear_wave_decays_at_nu_equal_cs2_tau_minus_half():
    # Eq.(linkTauNu): nu = c_s^2 (tau - 1/2)
    n0 = (64, 8)
    tau = 0.8
    o = O.Oracle("D2Q9", n0, [], tau0=tau)
    wl = W.Workload("s", "D2Q9", n0, [], tau, 1)
    pos = W.node_positions(wl, 0)
    k = 2 * np.pi / 64
    u = np.zeros((2, pos.shape[1]))
    u[1] = 1e-4 * np.sin(k * pos[0])
    o.init(0, np.ones(pos.shape[1]), u)
    T = 400
    o.run(T)
    uy = macros(o, 0)[1][1]
    amp = 2 * (uy * np.sin(k * pos[0])).mean()
    nu = -np.log(amp / 1e-4) / (k * k * T)
    assert nu == pytest.approx(CS2 * (tau - 0.5), rel=2e-3)


def _refined_shear(coupling, plant_R=None, n0=64, steps=200, tau0=0.55):
    q = n0 // 4
    wl = W.Workload("s", "D2Q9", (n0, n0), [((q, q), (3 * q, 3 * q))], tau0, steps, coupling=coupling)
    o = O.Oracle("D2Q9", (n0, n0), wl.boxes, tau0, coupling)
    if plant_R is not None:
        o.plant_R(plant_R)
    k, A = 2 * np.pi / n0, 1e-3
    for l in range(2):
        pos = W.node_positions(wl, l)
        u = np.zeros((2, pos.shape[1]))
        u[1] = A * np.sin(k * pos[0])
        o.init(l, np.ones(pos.shape[1]), u)
    o.run(steps)
    nu = CS2 * (tau0 - 0.5)   # coarse units; Eq.(rescNu) makes it the same physical viscosity
    err = 0.0
    for l in range(2):
        pos = W.node_positions(wl, l)
        uy = macros(o, l)[1][1]
        exact = A * np.sin(k * pos[0]) * np.exp(-nu * k * k * steps)
        err = max(err, np.nanmax(np.abs(uy - exact)))
    return err / A


@pytest.mark.parametrize("coupling", [1, 2])
def test_refined_shear_wave_follows_closed_form(coupling):
    """A shear wave crossing both faces of a refined patch decays at the one
    physical viscosity (Eq.(rescNu), Eq.(rescTau)); the off-equilibrium
    rescaling of Eq.(fneqResc) is what keeps the stress continuous."""
    assert _refined_shear(coupling) < 2e-3


def test_refined_shear_wave_detects_a_wrong_rescaling_factor():
    # planted mistake in the oracle: R forced to 1 (no off-equilibrium rescaling)
    assert _refined_shear(2, plant_R=1.0) > 4e-3


# ------------------------------------------------------------------ coupling identities
@pytest.mark.parametrize("coupling", [1, 2])
def test_completed_moments_equal_shared_equilibrium(coupling):
    """After the reconstruction (Eq.(rescff)) the completed fine populations
    carry exactly the Newton root X: sum Phi (f - f0(X)) = F(X) = 0."""
    wl = W.vortex_2level(n0=64, steps=3, coupling=coupling)
    o = make(wl)
    o.run(3)
    xi, _ = O.lattice_table("D2Q9")
    pre, X = o.pre(1), o.X(1)
    tf = ~np.isnan(X[0])
    assert tf.sum() == 4 * 32          # co-located nodes on the perimeter of the 65^2 patch
    rho = pre[:, tf].sum(0)
    j = xi[:, :2].T.astype(float) @ pre[:, tf]
    assert np.abs(rho - X[0, tf]).max() < 1e-14
    assert np.abs(j / rho - X[1:3, tf]).max() < 1e-14


def test_centred_pulse_keeps_square_symmetry():
    wl = W.Workload("p", "D2Q9", (64, 64), [((16, 16), (48, 48))], 0.55, 30,
                    pulses=[dict(c=(32.0, 32.0, 0.0), A=1e-3, Rc=4.0)])
    o = make(wl)
    o.run(30)
    r0 = macros(o, 0)[0].reshape(64, 64)
    mirror0 = np.roll(r0[:, ::-1], 1, axis=1)          # x -> 64 - x (periodic)
    m = ~np.isnan(r0)
    assert np.abs(r0 - mirror0)[m].max() < 1e-13
    assert np.abs(r0 - r0.T)[m].max() < 1e-13
    r1 = macros(o, 1)[0].reshape(65, 65)
    assert np.abs(r1 - r1[:, ::-1]).max() < 1e-13
    assert np.abs(r1 - r1.T).max() < 1e-13


@pytest.mark.slow
@pytest.mark.parametrize("coupling", [1, 2])
def test_refined_run_no_worse_than_coarse_against_uniform_fine(coupling):
    """Sec. 4 methodology: a uniform fine run is the reference.  The coupled
    run's velocity error is at most that of the uniform coarse run."""
    steps = 80
    base = W.vortex_2level(n0=128, steps=steps, coupling=coupling)
    dc = make(base)
    dc.run(steps)
    fine = W.Workload("f", "D2Q9", (256, 256), [], 0.6, 2 * steps, background=base.background,
                      vortices=[dict(xc=2 * v["xc"], yc=2 * v["yc"], eps=v["eps"], Rc=2 * v["Rc"])
                                for v in base.vortices])
    of = make(fine)
    of.run(2 * steps)
    coarse = W.Workload("c", "D2Q9", (128, 128), [], 0.55, steps, background=base.background,
                        vortices=base.vortices)
    oc = make(coarse)
    oc.run(steps)
    uf = macros(of, 0)[1].reshape(2, 256, 256)[:, ::2, ::2]
    u0 = macros(dc, 0)[1].reshape(2, 128, 128)
    uc = macros(oc, 0)[1].reshape(2, 128, 128)
    m = ~np.isnan(u0[0])
    e_dc = np.abs(u0 - uf)[:, m].max()
    e_c = np.abs(uc - uf)[:, m].max()
    assert e_dc <= 1.1 * e_c
    u1 = macros(dc, 1)[1].reshape(2, 129, 129)
    assert np.abs(u1 - macros(of, 0)[1].reshape(2, 256, 256)[:, 64:193, 64:193]).max() <= 1.1 * e_c


def test_newton_iterations_in_a_vortex_run():
    # Sec. 3.2: fewer than three iterations, i.e. at most two updates plus the converged check
    wl = W.vortex_2level(n0=128, steps=40)
    o = make(wl)
    o.run(40)
    calls, worst, hist = o.newton_stats()
    assert calls == 40 * 2 * 256
    assert worst <= 3


def test_newton_failure_is_reported():
    wl = W.vortex_2level(n0=64, steps=2)
    o = make(wl)
    o.set_newton(1e-30, 2)
    with pytest.raises(RuntimeError):
        o.run(1)


def test_3d_refined_pulse_keeps_cubic_symmetry():
    wl = W.Workload("p3", "D3Q19", (16, 16, 16), [((4, 4, 4), (12, 12, 12))], 0.6, 6,
                    pulses=[dict(c=(8.0, 8.0, 8.0), A=1e-3, Rc=2.0)])
    o = make(wl)
    o.run(6)
    r1 = macros(o, 1)[0].reshape(17, 17, 17)
    for perm in [(1, 0, 2), (2, 1, 0), (0, 2, 1)]:
        assert np.abs(r1 - r1.transpose(perm)).max() < 1e-13
    assert np.abs(r1 - r1[::-1]).max() < 1e-13


def test_probes_read_finest_level():
    wl = W.vortex_2level(n0=64, steps=4)
    o = make(wl)
    o.run(4)
    p = o.probes()
    assert p.shape == (4, 16)
    r0 = macros(o, 0)[0].reshape(64, 64)
    r1 = macros(o, 1)[0].reshape(65, 65)
    for k, (x, y) in enumerate(wl.probes):
        if 16 <= x <= 48 and 16 <= y <= 48:
            ref = r1[2 * (y - 16), 2 * (x - 16)]
        else:
            ref = r0[y, x]
        assert p[-1, k] == pytest.approx(CS2 * (ref - 1), abs=1e-18)
