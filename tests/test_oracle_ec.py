"""Pins of the oracle's electronic-conductivity routines (EC section):
geometry, the current operator J = i[H, X], the EC correlation of Eq. dc_corr
(EC-Sequential and EC-Concurrent-M) and the conductivity integral of Eq. DC.

- bond vectors equal position differences on open lattices, unit length;
- J equals the dense commutator i(HX - XH) on open lattices, the
  nearest-image form on periodic chains and squares, and the open-lattice
  J away from the boundary on periodic honeycombs; J is Hermitian;
- an explicit matrix with coordinates gives the stencil lattice's J;
- the correlation equals exact diagonalisation, with and without a
  spectral centre, and the moment form equals the sequential form;
- the time integral reproduces closed forms within the trapezoid bound.
"""
import math

import numpy as np
import pytest

import csp_inputs as ci
import oracle as o

SPECS = [
    ("chain", 13, 1, dict(t=1.0, W=1.0, disorder_seed=1)),
    ("square", 6, 5, dict(t=-1.0, W=0.7, disorder_seed=2)),
    ("honeycomb", 5, 4, dict(t=-2.7, W=1.0, disorder_seed=3)),
]


def lat_open(kind, Lx, Ly, kw):
    return o.Lattice(kind, Lx, Ly, periodic_x=False, periodic_y=False, **kw)


@pytest.mark.parametrize("kind,Lx,Ly,kw", SPECS)
def test_bond_vectors_are_position_differences(kind, Lx, Ly, kw):
    lat = lat_open(kind, Lx, Ly, kw)
    pos = o.positions(lat)
    v = o.bond_vectors(lat)
    d = pos[lat.bond_b] - pos[lat.bond_a]
    assert np.max(np.abs(d - v)) < 1e-12
    assert np.max(np.abs(np.linalg.norm(v, axis=1) - 1.0)) < 1e-12


@pytest.mark.parametrize("kind,Lx,Ly,kw", SPECS)
@pytest.mark.parametrize("alpha", [0, 1])
def test_current_is_the_commutator_on_open_lattices(kind, Lx, Ly, kw, alpha):
    lat = lat_open(kind, Lx, Ly, kw)
    H = lat.dense()
    X = np.diag(o.positions(lat)[:, alpha])
    J = 1j * (H @ X - X @ H)
    psi = np.random.default_rng(4).normal(size=(lat.N, 3)) * (1 + 0.5j)
    assert np.max(np.abs(o.current(lat, alpha, psi) - J @ psi)) < 1e-12
    assert np.max(np.abs(J - J.conj().T)) < 1e-14          # Hermitian


@pytest.mark.parametrize("kind,Lx,Ly", [("chain", 9, 1), ("square", 6, 5)])
def test_current_nearest_image_on_periodic_lattices(kind, Lx, Ly):
    lat = o.Lattice(kind, Lx, Ly, t=1.3, W=0.4, disorder_seed=5)
    H = lat.dense()
    pos = o.positions(lat)
    for alpha, box in ((0, Lx), (1, Ly)):
        d = pos[:, alpha][None, :] - pos[:, alpha][:, None]       # x_j - x_i
        d -= box * np.rint(d / box)
        J = 1j * H * d
        psi = np.random.default_rng(alpha).normal(size=lat.N) + 1j
        assert np.max(np.abs(o.current(lat, alpha, psi) - J @ psi)) < 1e-12


def test_periodic_honeycomb_current_matches_open_away_from_the_boundary():
    kw = dict(t=-2.7, W=0.5, disorder_seed=6)
    per = o.Lattice("honeycomb", 7, 6, **kw)
    opn = lat_open("honeycomb", 7, 6, kw)
    psi = np.zeros(per.N, dtype=np.complex128)
    rng = np.random.default_rng(7)
    for iy in range(2, 4):
        for ix in range(2, 5):
            A = 2 * (iy * 7 + ix)
            psi[A:A + 2] = rng.normal(size=2) + 1j * rng.normal(size=2)
    for alpha in (0, 1):
        assert np.max(np.abs(o.current(per, alpha, psi) - o.current(opn, alpha, psi))) < 1e-13
    # clean periodic honeycomb: the three bond vectors of a site sum to zero
    clean = o.Lattice("honeycomb", 5, 4, t=-2.7)
    for alpha in (0, 1):
        assert np.max(np.abs(o.current(clean, alpha, np.ones(clean.N)))) < 1e-12


def test_current_hermitian_periodic():
    lat = o.Lattice("honeycomb", 6, 5, t=-2.7, W=1.0, disorder_seed=2)
    rng = np.random.default_rng(3)
    a = rng.normal(size=lat.N) + 1j * rng.normal(size=lat.N)
    b = rng.normal(size=lat.N) + 1j * rng.normal(size=lat.N)
    for alpha in (0, 1):
        lhs = np.vdot(a, o.current(lat, alpha, b))
        rhs = np.conj(np.vdot(b, o.current(lat, alpha, a)))
        assert abs(lhs - rhs) < 1e-12


def test_explicit_matrix_current_matches_stencil():
    lat = o.Lattice("square", 7, 6, t=-1.0, W=0.8, disorder_seed=9)
    cnt = np.diff(lat.rowptr)
    D = int(cnt.max())
    col = np.full((lat.N, D), -1, np.int64)
    val = np.zeros((lat.N, D))
    for s in range(lat.N):
        k = cnt[s]
        col[s, :k] = lat.col[lat.rowptr[s]:lat.rowptr[s + 1]]
        val[s, :k] = lat.val[lat.rowptr[s]:lat.rowptr[s + 1]]
    sp = o.SparseLattice(col, val, pos=o.positions(lat), box=(7.0, 6.0))
    psi = np.random.default_rng(1).normal(size=(lat.N, 2)) * (1 - 0.3j)
    for alpha in (0, 1):
        assert np.max(np.abs(o.current(sp, alpha, psi) - o.current(lat, alpha, psi))) < 1e-13


def test_long_range_current_and_correlation():
    # explicit matrix with coordinates: J is the nearest-image commutator and
    # the EC correlation matches exact diagonalisation
    col, val = ci.long_range_square(8, 2.3, t0=-1.0, decay=1.5, W=0.6, seed=3)
    pos, box = ci.long_range_square_positions(8)
    lat = o.SparseLattice(col, val, pos=pos, box=box)
    H = lat.dense()
    psi = o.random_phase_states(lat.N, 2, 8)
    for alpha in (0, 1):
        d = pos[:, alpha][None, :] - pos[:, alpha][:, None]
        d -= 8.0 * np.rint(d / 8.0)
        assert np.max(np.abs(o.current(lat, alpha, psi) - (1j * H * d) @ psi)) < 1e-12
    Hn = lat.halfwidth()
    qe, _ = o.quasi_eigenstates(lat, psi, 10, [-0.8, 0.5], Hn=Hn)
    got, _ = o.ec_correlation(lat, psi, qe, 20, 1, Hn=Hn)
    ref = _ed_corr(lat, psi, qe, 20, 1, Hn)
    assert np.max(np.abs(got - ref)) < 1e-10 * max(1.0, np.max(np.abs(ref)))


def _ed_corr(lat, psi, qe, Nt, alpha, Hn, H0=0.0):
    w, V = np.linalg.eigh(lat.dense())
    Jpsi = o.current(lat, alpha, psi)
    out = np.zeros((qe.shape[0], Nt + 1, psi.shape[1]), dtype=np.complex128)
    tp = math.pi / Hn
    for e in range(qe.shape[0]):
        X = o.current(lat, alpha, qe[e])
        nrm = np.abs(np.einsum("sr,sr->r", psi.conj(), qe[e]))
        a = V.conj().T @ Jpsi
        b = V.conj().T @ X
        for j in range(Nt + 1):
            out[e, j] = np.einsum("kr,k,kr->r", a.conj(), np.exp(1j * w * j * tp), b) / nrm
    return out


@pytest.mark.parametrize("kind,Lx,Ly,kw", [SPECS[1], SPECS[2]])
def test_ec_correlation_matches_exact_diagonalisation(kind, Lx, Ly, kw):
    lat = o.Lattice(kind, Lx, Ly, **kw)
    Hn = lat.halfwidth()
    psi = o.random_phase_states(lat.N, 2, 11)
    E = [-1.1, 0.4]
    qe, _ = o.quasi_eigenstates(lat, psi, 12, E, Hn=Hn)
    Nt = 25
    for alpha in (0, 1):
        got, cnt = o.ec_correlation(lat, psi, qe, Nt, alpha, Hn=Hn)
        ref = _ed_corr(lat, psi, qe, Nt, alpha, Hn)
        assert np.max(np.abs(got - ref)) < 1e-10 * max(1.0, np.max(np.abs(ref)))
    # EC-Sequential counts (Tab. cost): Nt N(tau) amxsy and (Nt + 1) n_E dots per state
    assert cnt["amxsy"] == 2 * Nt * o.truncation(math.pi)
    assert cnt["dot"] == 2 * (Nt + 1) * len(E)


def test_ec_correlation_with_spectral_centre():
    lat = o.Lattice("square", 5, 4, t=1.0, W=1.5, disorder_seed=4)
    H0, Hn = 0.35, 5.3
    psi = o.random_phase_states(lat.N, 1, 3)
    qe, _ = o.quasi_eigenstates(lat, psi, 10, [0.2], Hn=Hn, H0=H0)
    got, _ = o.ec_correlation(lat, psi, qe, 20, 0, Hn=Hn, H0=H0)
    ref = _ed_corr(lat, psi, qe, 20, 0, Hn)
    assert np.max(np.abs(got - ref)) < 1e-10 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("kind,Lx,Ly,kw", SPECS)
def test_ec_moment_form_equals_sequential(kind, Lx, Ly, kw):
    lat = o.Lattice(kind, Lx, Ly, **kw)
    Hn = lat.halfwidth()
    psi = o.random_phase_states(lat.N, 2, 5)
    E = [-0.5, 0.3, 1.2]
    qe, _ = o.quasi_eigenstates(lat, psi, 15, E, Hn=Hn)
    seq, _ = o.ec_correlation(lat, psi, qe, 40, 0, Hn=Hn)
    mom, m = o.ec_moments(lat, psi, qe, 40, 0, Hn=Hn)
    assert m.shape[0] == o.truncation(40 * math.pi) + 1
    assert np.max(np.abs(mom - seq)) < 1e-11 * max(1.0, np.max(np.abs(seq)))


def test_sigma_integral():
    Hn, Nt = 4.1, 400
    tp = math.pi / Hn
    t = np.arange(Nt + 1) * tp
    E = np.array([-0.7, 0.9])
    a = np.array([[0.3, -1.2], [2.0, 0.5]])                # [nE][R]
    # C = a e^{iEt}: the integrand is the constant a
    corr = a[:, None, :] * np.exp(1j * E[:, None, None] * t[None, :, None])
    s = o.ec_sigma(corr, E, Hn, dos_over_area=[2.0, 0.5])
    ref = np.array([2.0, 0.5])[:, None] * a * Nt * tp
    assert np.max(np.abs(s - ref)) < 1e-13 * np.max(np.abs(ref))
    # C = e^{iEt - t/T}: integral T (1 - e^{-t_max/T}) within the trapezoid error
    T = 7.0
    corr = np.exp((1j * E[:, None, None] - 1.0 / T) * t[None, :, None]) * np.ones((1, 1, 2))
    s = o.ec_sigma(corr, E, Hn)
    exact = T * (1 - math.exp(-t[-1] / T))
    bound = t[-1] * tp ** 2 / (12 * T ** 2)
    assert np.max(np.abs(s - exact)) <= bound
