"""Pins of the oracle's H-RR collision (Sec. 2, App. A) on one periodic
level, each against a fact fixed by the definitions or by the physics
(CPU only):

* a uniform state (rest or uniform flow) is a fixed point for every sigma;
* the collision conserves mass and momentum node by node;
* with sigma = 1 and no cubic correction the regularised off-equilibrium
  keeps the second-order non-equilibrium moment scaled by (1 - 1/tau), and in
  D2Q9 its third-order moments are the recursive a_1^(3) of Eq.(a13RR);
* shear waves decay at nu k^2 with nu = c_s^2 (tau - 1/2) for sigma = 1,
  0.98 and 0 (the finite-difference part converging as k^2);
* the cubic Mach correction makes that decay Galilean invariant: with a
  mean flow normal to the wave vector, D3Q19 without the correction loses
  about 3/2 U^2 / c_s^2 of its viscosity (the lattice's missing
  third-order moment rho u_y u_z^2 / 2), and with it does not;
* the regularisation leaves no off-equilibrium part in the moments outside
  the Hermite basis it keeps (BGK keeps 1 - 1/tau of them).
"""
import numpy as np
import pytest

import oracle as O
from paper_2004_14887_amd import workloads as W

CS2 = 1.0 / 3.0


def hrr(lat, dims, tau, sigma=0.98, psi=True, eq_order=3):
    o = O.Oracle(lat, dims, [], tau0=tau, eq_order=eq_order)
    if sigma is not None:
        o.set_collision("hrr", sigma, psi)
    return o


def moments(lat, f):
    xi, _ = O.lattice_table(lat)
    rho = f.sum(0)
    j = xi.T.astype(float) @ f
    return rho, j, xi


@pytest.mark.parametrize("lat,dims", [("D2Q9", (16, 12)), ("D3Q19", (10, 9, 8))])
@pytest.mark.parametrize("sigma", [1.0, 0.98, 0.0])
def test_uniform_state_is_a_fixed_point(lat, dims, sigma):
    D = len(dims)
    n = int(np.prod(dims))
    u0 = np.array([0.08, -0.05, 0.03][:D])
    o = hrr(lat, dims, 0.5 + 1e-4, sigma)
    o.init(0, np.full(n, 1.013), np.tile(u0[:, None], (1, n)))
    f0 = o.f(0)
    o.run(5)
    assert np.abs(o.f(0) - f0).max() <= 1e-15


@pytest.mark.parametrize("lat,dims", [("D2Q9", (16, 12)), ("D3Q19", (10, 9, 8))])
def test_collision_conserves_mass_and_momentum_per_node(lat, dims):
    rng = np.random.default_rng(7)
    D = len(dims)
    n = int(np.prod(dims))
    o = hrr(lat, dims, 0.51, 0.98)
    o.init(0, 1 + 1e-2 * rng.normal(size=n), 0.05 * rng.normal(size=(D, n)))
    o.run(3)
    rp, jp, _ = moments(lat, o.pre(0))
    rf, jf, _ = moments(lat, o.f(0))
    assert np.abs(rf - rp).max() <= 1e-15
    assert np.abs(jf - jp).max() <= 1e-15


@pytest.mark.parametrize("lat,dims", [("D2Q9", (16, 12)), ("D3Q19", (10, 9, 8))])
def test_projected_part_keeps_second_moment_scaled(lat, dims):
    """sigma = 1, no correction: sum xi xi (f* - f0) = (1 - 1/tau) sum xi xi (pre - f0)."""
    rng = np.random.default_rng(8)
    D = len(dims)
    n = int(np.prod(dims))
    tau = 0.57
    o = hrr(lat, dims, tau, 1.0, psi=False)
    o.init(0, 1 + 1e-2 * rng.normal(size=n), 0.05 * rng.normal(size=(D, n)))
    o.run(2)
    pre, post = o.pre(0), o.f(0)
    rho, j, xi = moments(lat, pre)
    u = j[:D] / rho
    f0 = np.stack([O.feq(lat, rho[q], u[:, q], eq_order=3) for q in range(n)], 1)
    for a in range(D):
        for b in range(D):
            m_pre = (xi[:, a] * xi[:, b]) @ (pre - f0)
            m_post = (xi[:, a] * xi[:, b]) @ (post - f0)
            assert np.abs(m_post - (1 - 1 / tau) * m_pre).max() <= 1e-15
            if lat == "D2Q9" and a != b:
                # third order: sum xi_a^2 xi_b (f* - f0) = (1 - 1/tau) (2 u_a a1_ab + u_b a1_aa)
                a1_ab = m_pre
                a1_aa = (xi[:, a] * xi[:, a]) @ (pre - f0)
                m3 = (xi[:, a] ** 2 * xi[:, b]) @ (post - f0)
                assert np.abs(m3 - (1 - 1 / tau) * (2 * u[a] * a1_ab + u[b] * a1_aa)).max() <= 1e-15


def shear_rate(lat, n, tau, sigma, psi=True, U=(0.0, 0.0, 0.0), steps=200, A=1e-4):
    """Decay rate of a shear wave u_y = A sin(2 pi x / n) (plus a mean flow U)
    relative to nu k^2."""
    D = 2 if lat == "D2Q9" else 3
    dims = (n, 8) if D == 2 else (n, 8, 8)
    o = hrr(lat, dims, tau, sigma, psi)
    N = int(np.prod(dims))
    x = np.arange(N) % n
    k = 2 * np.pi / n
    u = np.zeros((D, N))
    for a in range(D):
        u[a] += U[a]
    u[1] += A * np.sin(k * x)
    o.init(0, np.ones(N), u)
    xi, _ = O.lattice_table(lat)
    amps = []
    for _ in range(steps):
        o.run(1)
        f = o.f(0)
        uy = (xi[:, 1].astype(float) @ f) / f.sum(0) - U[1]
        amps.append(2 * np.mean(uy * np.sin(k * x)))
    t = np.arange(1, steps + 1)
    rate = -np.polyfit(t[20:], np.log(np.abs(np.array(amps[20:]))), 1)[0]
    return rate / (CS2 * (tau - 0.5) * k * k)


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
@pytest.mark.parametrize("sigma,n,tol", [(1.0, 32, 0.005), (0.98, 32, 0.005), (0.0, 64, 0.012)])
def test_shear_wave_decays_at_nu(lat, sigma, n, tol):
    r = shear_rate(lat, n, 0.6, sigma, steps=200 if n == 32 else 400)
    assert abs(r - 1.0) <= tol, r


def test_finite_difference_part_converges_as_k_squared():
    e32 = shear_rate("D2Q9", 32, 0.6, 0.0) - 1.0
    e64 = shear_rate("D2Q9", 64, 0.6, 0.0, steps=400) - 1.0
    assert 3.0 <= e32 / e64 <= 5.0


@pytest.mark.parametrize("U", [0.1, 0.2])
def test_cubic_correction_makes_shear_decay_galilean_invariant(U):
    rest = shear_rate("D3Q19", 32, 0.6, 0.98)
    on = shear_rate("D3Q19", 32, 0.6, 0.98, True, U=(0.0, 0.0, U))
    off = shear_rate("D3Q19", 32, 0.6, 0.98, False, U=(0.0, 0.0, U))
    assert abs(on - rest) <= 1e-3
    # without it the apparent viscosity drops by U^2 / (2 c_s^2): the lattice
    # lacks rho u_y u_z^2 / 2 of the third-order moment xxy
    expected = U * U / (2 * CS2)
    assert abs((rest - off) / rest - expected) <= 0.2 * expected


@pytest.mark.parametrize("lat,dims", [("D2Q9", (16, 12)), ("D3Q19", (10, 9, 8))])
@pytest.mark.parametrize("sigma,psi", [(1.0, False), (0.98, True), (0.0, True)])
def test_regularised_off_equilibrium_lies_in_its_hermite_span(lat, dims, sigma, psi):
    """After an H-RR collision f* - f0 is a combination of w_i H2_{i,ab} and
    of the kept w_i H3_{i,aab} (psi lies in the w H2 span too): nothing of the
    other (non-hydrodynamic) directions of population space survives, while
    BGK keeps 1 - 1/tau of them."""
    rng = np.random.default_rng(9)
    D = len(dims)
    n = int(np.prod(dims))
    tau = 0.52
    xi, w = O.lattice_table(lat)
    xi = xi[:, :D].astype(float)
    basis = []
    for a in range(D):
        for b in range(a, D):
            basis.append(w * (xi[:, a] * xi[:, b] - (CS2 if a == b else 0.0)))
    for a in range(D):
        for b in range(D):
            if a != b:
                basis.append(w * (xi[:, a] ** 2 * xi[:, b] - CS2 * xi[:, b]))
    B = np.stack(basis, 1)
    rho0 = 1 + 1e-2 * rng.normal(size=n)
    u0 = 0.05 * rng.normal(size=(D, n))
    res = {}
    for kind in ("hrr", "bgk"):
        o = hrr(lat, dims, tau, sigma if kind == "hrr" else None, psi)
        o.init(0, rho0, u0)
        o.run(3)
        pre, post = o.pre(0), o.f(0)
        rho, j, _ = moments(lat, pre)
        f0 = np.stack([O.feq(lat, rho[q], j[:D, q] / rho[q], eq_order=3) for q in range(n)], 1)
        d = post - f0
        coef, *_ = np.linalg.lstsq(B, d, rcond=None)
        res[kind] = (np.abs(d - B @ coef).max(), np.abs(d).max())
    assert res["hrr"][0] <= 1e-15 * res["hrr"][1] * 100
    assert res["bgk"][0] > 1e-3 * res["bgk"][1]


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
@pytest.mark.parametrize("sigma", [0.98, 0.0])
def test_centred_gradients_keep_the_shear_wave_in_place(lat, sigma):
    """u_y = A sin(k x) is odd about x = 0, and centred finite differences
    (Eq.(a1FD_scheme), Eq.(PSI_FD)) on the symmetric lattice keep it odd: no
    cos(k x) component may appear (a one-sided stencil would shift it)."""
    D = 2 if lat == "D2Q9" else 3
    n = 32
    dims = (n, 8) if D == 2 else (n, 8, 8)
    o = hrr(lat, dims, 0.55, sigma)
    N = int(np.prod(dims))
    x = np.arange(N) % n
    k = 2 * np.pi / n
    u = np.zeros((D, N))
    u[1] = 1e-3 * np.sin(k * x)
    o.init(0, np.ones(N), u)
    o.run(60)
    f = o.f(0)
    xi, _ = O.lattice_table(lat)
    uy = (xi[:, 1].astype(float) @ f) / f.sum(0)
    s, c = np.mean(uy * np.sin(k * x)), np.mean(uy * np.cos(k * x))
    assert abs(c) <= 1e-12 * abs(s)
