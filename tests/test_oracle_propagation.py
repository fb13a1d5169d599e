"""Pins for the oracle's propagation and DOS.

Against: exact diagonalisation; Bloch closed forms of clean periodic
lattices; the chain's return amplitude J_0(2|t|t) and its DOS
1/(pi sqrt(4t^2 - E^2)); the eigenvector identity T_n(cos th) = cos(n th);
norm conservation; the discrete DOS sum rule; the brute-force DFT;
agreement of the concurrent and sequential forms (Sec. III accuracy scale);
and the operation counts of Tab. (cost).
"""
import math

import numpy as np
import pytest
from scipy.special import jv

import oracle as o


def exact_corr(lat, psi0, Nt, Hn):
    """C_r(t_j) = sum_k |<v_k|psi_r>|^2 exp(-i E_k t_j) by eigh."""
    E, V = np.linalg.eigh(lat.dense())
    wts = np.abs(V.conj().T @ psi0) ** 2
    t = np.arange(Nt + 1) * math.pi / Hn
    return np.exp(-1j * np.outer(t, E)) @ wts


SMALL = [
    ("square", 6, 5, 1.0, 1.3, True, True),
    ("square", 7, 4, -1.0, 0.0, False, True),
    ("honeycomb", 4, 3, -2.7, 1.0, True, True),
    ("honeycomb", 3, 5, -2.7, 0.5, False, False),
    ("chain", 17, 1, 1.0, 2.0, True, True),
    ("chain", 12, 1, 0.8, 0.0, False, False),
]


@pytest.mark.parametrize("kind,Lx,Ly,t,W,px,py", SMALL)
@pytest.mark.parametrize("b", [0, 1, 3, 60])
def test_propagation_matches_exact_diagonalisation(kind, Lx, Ly, t, W, px, py, b):
    lat = o.Lattice(kind, Lx, Ly, t=t, W=W, disorder_seed=5, periodic_x=px, periodic_y=py)
    Hn = lat.halfwidth()
    psi = o.random_phase_states(lat.N, 2, 9)
    Nt = 60
    corr, _ = o.propagate(lat, psi, Nt, b=b, Hn=Hn)
    assert np.max(np.abs(corr - exact_corr(lat, psi, Nt, Hn))) < 1e-10


def test_exact_diagonalisation_config1_size():
    # 64 x 64 square, t = 1, |H| = 4.1, one random state, 1024 time points
    lat = o.Lattice("square", 64, 64, t=1.0)
    psi = o.random_phase_states_fast(lat.N, 1, 1)
    Nt = 1024
    corr, _ = o.propagate(lat, psi, Nt, b=32, Hn=4.1)
    assert np.max(np.abs(corr - exact_corr(lat, psi, Nt, 4.1))) < 1e-10


def test_square_bloch_closed_form():
    Lx, Ly = 40, 36
    lat = o.Lattice("square", Lx, Ly, t=1.0)
    psi = o.random_phase_states_fast(lat.N, 1, 2)[:, 0]
    Hn = lat.halfwidth()
    Nt = 200
    corr, _ = o.propagate(lat, psi, Nt, b=16, Hn=Hn)
    ph = np.fft.fft2(psi.reshape(Ly, Lx)) / math.sqrt(lat.N)
    kx = 2 * np.pi * np.arange(Lx) / Lx
    ky = 2 * np.pi * np.arange(Ly) / Ly
    E = 2 * (np.cos(kx)[None, :] + np.cos(ky)[:, None])
    t = np.arange(Nt + 1) * math.pi / Hn
    ref = np.exp(-1j * np.outer(t, E.ravel())) @ (np.abs(ph.ravel()) ** 2)
    assert np.max(np.abs(corr[:, 0] - ref)) < 1e-10


def test_honeycomb_bloch_closed_form():
    Lx, Ly = 24, 21          # 21 divisible by 3: Dirac points are on the grid
    lat = o.Lattice("honeycomb", Lx, Ly, t=-2.7)
    psi = o.random_phase_states_fast(lat.N, 1, 3)[:, 0]
    Hn = lat.halfwidth()
    Nt = 150
    corr, _ = o.propagate(lat, psi, Nt, b=8, Hn=Hn)
    ref = o.bloch_corr("honeycomb", Lx, Ly, -2.7, psi, np.arange(Nt + 1) * math.pi / Hn)
    assert np.max(np.abs(corr[:, 0] - ref[:, 0])) < 1e-10


@pytest.mark.parametrize("kind,Lx,Ly,t", [("square", 7, 5, 1.0), ("square", 6, 6, -0.8),
                                          ("honeycomb", 5, 4, -2.7), ("honeycomb", 6, 3, 1.0),
                                          ("chain", 13, 1, 0.7)])
def test_bloch_closed_form_equals_exact_diagonalisation(kind, Lx, Ly, t):
    # the k-space closed form against eigh of the real-space matrix, also
    # with localized columns (the LDOS states)
    lat = o.Lattice(kind, Lx, Ly, t=t)
    psi = np.concatenate([o.random_phase_states_fast(lat.N, 2, 8),
                          o.site_states(lat.N, [0, lat.N - 1])], axis=1)
    Hn = lat.halfwidth()
    Nt = 40
    ref = exact_corr(lat, psi, Nt, Hn)
    got = o.bloch_corr(kind, Lx, Ly, t, psi, np.arange(Nt + 1) * math.pi / Hn)
    assert np.max(np.abs(got - ref)) < 1e-12


@pytest.mark.parametrize("kind,Lx,Ly,t", [("square", 6, 5, 1.0), ("honeycomb", 5, 4, -2.7),
                                          ("chain", 11, 1, 0.9)])
def test_bloch_uniform_and_return_amplitude_equal_exact_diagonalisation(kind, Lx, Ly, t):
    lat = o.Lattice(kind, Lx, Ly, t=t)
    Hn = lat.halfwidth()
    Nt = 50
    tau = math.pi / Hn
    psi = np.concatenate([o.random_phase_states_fast(lat.N, 2, 4),
                          o.site_states(lat.N, [1])], axis=1)
    got = o.bloch_corr_uniform(kind, Lx, Ly, t, psi, tau, Nt + 1)
    assert np.max(np.abs(got - exact_corr(lat, psi, Nt, Hn))) < 1e-12
    ret = o.bloch_return_amplitude(kind, Lx, Ly, t, tau, Nt + 1)
    for site in (0, 1, lat.N // 2, lat.N - 1):
        ref = exact_corr(lat, o.site_states(lat.N, [site]), Nt, Hn)[:, 0]
        assert np.max(np.abs(ret - ref)) < 1e-12


def test_bloch_uniform_long_times_match_direct():
    # block products against direct cos/sin over thousands of steps
    lat = o.Lattice("honeycomb", 30, 24, t=-2.7)
    psi = o.random_phase_states_fast(lat.N, 2, 6)
    tau = math.pi / lat.halfwidth()
    u = o.bloch_corr_uniform("honeycomb", 30, 24, -2.7, psi, tau, 4097)
    sel = np.array([0, 1, 17, 1000, 2047, 4096])
    d = o.bloch_corr("honeycomb", 30, 24, -2.7, psi, sel * tau)
    assert np.max(np.abs(u[sel] - d)) < 1e-12


def test_chain_return_amplitude_is_bessel_j0():
    # periodic chain long enough that no wave wraps round within t_tot:
    # <0|exp(-iHt)|0> = J_0(2|t| t) for the infinite chain
    L, tt, Nt = 1400, 1.0, 200
    lat = o.Lattice("chain", L, t=tt)
    Hn = lat.halfwidth()
    corr, _ = o.propagate(lat, o.site_states(L, [0]), Nt, b=20, Hn=Hn)
    t = np.arange(Nt + 1) * math.pi / Hn
    assert np.max(np.abs(corr[:, 0] - jv(0, 2 * abs(tt) * t))) < 1e-12


def test_chain_dos_closed_form():
    # DOS of the infinite chain, 1/(pi sqrt(4t^2 - E^2)), from the windowed
    # transform of the exact return amplitude at many time points
    tt, Nt = 1.0, 4096
    Hn = 1.025 * 2 * tt
    t = np.arange(Nt + 1) * math.pi / Hn
    E, D, im = o.dos(jv(0, 2 * t)[:, None], Hn)
    inner = np.abs(E) < 1.5 * tt
    ref = 1.0 / (math.pi * np.sqrt(4 * tt**2 - E[inner] ** 2))
    assert np.max(np.abs(D[inner, 0] / ref - 1.0)) < 1e-3
    assert im < 1e-12


def test_chain_dos_from_propagation():
    L, tt, Nt = 1400, 1.0, 200
    lat = o.Lattice("chain", L, t=tt)
    Hn = lat.halfwidth()
    corr, _ = o.propagate(lat, o.site_states(L, [5]), Nt, b=50, Hn=Hn)
    t = np.arange(Nt + 1) * math.pi / Hn
    _, D, _ = o.dos(corr, Hn)
    _, Dref, _ = o.dos(jv(0, 2 * t)[:, None], Hn)
    assert np.max(np.abs(D - Dref)) < 1e-10


def test_chebyshev_vectors_on_eigenvector():
    lat = o.Lattice("honeycomb", 3, 3, t=-1.0, W=0.7, disorder_seed=2)
    Hn = lat.halfwidth()
    E, V = np.linalg.eigh(lat.dense())
    for k in (0, 5, lat.N - 1):
        th = math.acos(E[k] / Hn)
        vecs = o.chebyshev_vectors(lat, V[:, k].astype(np.complex128), 30, Hn)
        for n in range(31):
            assert np.max(np.abs(vecs[n] - math.cos(n * th) * V[:, k])) < 1e-12


@pytest.mark.parametrize("b", [0, 7])
def test_norm_conservation(b):
    lat = o.Lattice("honeycomb", 10, 9, t=-2.7, W=1.0, disorder_seed=4)
    psi = o.random_phase_states_fast(lat.N, 2, 5)
    _, _, fin = o.propagate(lat, psi, 100, b=b, return_final=True)
    assert np.max(np.abs(np.linalg.norm(fin, axis=0) - 1.0)) < 1e-12


def test_dos_sum_rule_and_direct_dft():
    lat = o.Lattice("square", 8, 7, t=1.0, W=1.0, disorder_seed=3)
    Hn = lat.halfwidth()
    psi = o.random_phase_states(lat.N, 2, 4)
    Nt = 24
    corr, _ = o.propagate(lat, psi, Nt, b=5, Hn=Hn)
    E, D, im = o.dos(corr, Hn)
    dE = Hn / Nt
    assert np.allclose(D.sum(axis=0) * dE, corr[0].real, atol=1e-14)
    assert im < 1e-13
    E2, D2 = o.dos_direct(corr, Hn)
    assert np.allclose(E, E2, atol=1e-15)
    assert np.max(np.abs(D - D2.real)) < 1e-13
    assert np.max(np.abs(D2.imag)) < 1e-13


def test_dos_of_exact_spectrum():
    # DOS from exact correlations equals the window kernel placed on each level
    lat = o.Lattice("chain", 9, t=1.0, W=1.0, disorder_seed=1)
    Hn = lat.halfwidth()
    psi = o.random_phase_states(lat.N, 1, 2)
    Nt = 32
    E, D, _ = o.dos(exact_corr(lat, psi, Nt, Hn), Hn)
    lev, V = np.linalg.eigh(lat.dense())
    wts = np.abs(V.conj().T @ psi[:, 0]) ** 2
    tau = math.pi / Hn
    j = np.arange(-Nt, Nt)
    w = 0.5 * (1 + np.cos(np.pi * j / Nt))
    for ik in (0, 13, 32, 50):
        kern = [(tau / (2 * math.pi)) * np.sum(w * np.cos((E[ik] - e) * j * tau)) for e in lev]
        assert D[ik, 0] == pytest.approx(float(np.dot(wts, kern)), abs=1e-12)


def test_dos_with_spectral_centre_on_exact_spectrum():
    # with H~ = (H - H0)/|H| the correlations carry exp(-i (H - H0) t), and
    # the DOS placed at H0 + E_k is the window kernel on each true level
    # (a spectrum that is not centred on 0: on-site energies shifted by +0.9)
    lat = o.Lattice("chain", 11, t=1.0, W=1.0, disorder_seed=5)
    H = lat.dense() + 0.9 * np.eye(lat.N)
    shifted = o.SparseLattice(*_ell_of_dense(H))
    lev, V = np.linalg.eigh(H)
    H0 = 0.5 * (lev[0] + lev[-1])
    Hn = 1.025 * 0.5 * (lev[-1] - lev[0])
    psi = o.random_phase_states(lat.N, 1, 3)
    Nt = 40
    corr, _ = o.propagate(shifted, psi, Nt, b=0, Hn=Hn, H0=H0)
    E, D, _ = o.dos(corr, Hn, H0=H0)
    assert E[Nt] == H0 and E[0] == pytest.approx(H0 - Hn, abs=1e-14)
    wts = np.abs(V.conj().T @ psi[:, 0]) ** 2
    tau = math.pi / Hn
    j = np.arange(-Nt, Nt)
    w = 0.5 * (1 + np.cos(np.pi * j / Nt))
    for ik in (3, 25, Nt, 61):
        kern = [(tau / (2 * math.pi)) * np.sum(w * np.cos((E[ik] - e) * j * tau)) for e in lev]
        assert D[ik, 0] == pytest.approx(float(np.dot(wts, kern)), abs=1e-12)
    # the density peaks inside the true band [lev[0], lev[-1]], not around 0
    assert lev[0] - 0.3 < E[int(np.argmax(D[:, 0]))] < lev[-1] + 0.3
    E2, D2 = o.dos_direct(corr, Hn, H0=H0)
    assert np.allclose(E, E2, atol=1e-15) and np.max(np.abs(D - D2.real)) < 1e-13


def _ell_of_dense(H):
    N = H.shape[0]
    D = int(max(np.count_nonzero(H[s]) for s in range(N)))
    col = -np.ones((N, D), dtype=np.int64)
    val = np.zeros((N, D))
    for s in range(N):
        nz = np.nonzero(H[s])[0]
        col[s, :len(nz)] = nz
        val[s, :len(nz)] = H[s, nz]
    return col, val


@pytest.mark.parametrize("b", [2, 16, 32, 40, 256])
def test_concurrent_equals_sequential(b, golden):
    scale = float(golden("dos_accuracy.txt")["eps_inf_correlation"])
    lat = o.Lattice("honeycomb", 24, 24, t=-2.7, W=1.0, disorder_seed=4)
    Hn = lat.halfwidth()
    psi = o.random_phase_states_fast(lat.N, 1, 5)
    Nt = 256
    c_seq, _ = o.propagate(lat, psi, Nt, b=0, Hn=Hn)
    c_con, _ = o.propagate(lat, psi, Nt, b=b, Hn=Hn)
    eps_c = np.max(np.abs(c_con - c_seq))
    assert eps_c < 1e-12
    assert eps_c < 100 * scale
    _, D1, _ = o.dos(c_seq, Hn)
    _, D2, _ = o.dos(c_con, Hn)
    assert np.max(np.abs(D1 - D2)) < 1e-12


@pytest.mark.parametrize("Nt,b", [(64, 1), (64, 8), (64, 32), (50, 8), (50, 64)])
def test_operation_counts_match_cost_table(Nt, b):
    """Tab. (cost): DOS-Sequential has Nt*N(pi) amxsy and axpy and Nt dot;
    the state-based concurrent form has t_tot*R(t_b) = N_b*N(b*pi) amxsy and
    N_b*sum_j N(j*pi) axpy.  Where b does not divide Nt the last block is
    shorter and contributes its own terms."""
    lat = o.Lattice("chain", 10, t=1.0)
    psi = o.random_phase_states(lat.N, 1, 1)
    Npi = o.truncation(math.pi)
    _, cs = o.propagate(lat, psi, Nt, b=0)
    assert cs["amxsy"] == Nt * Npi and cs["axpy"] == Nt * Npi and cs["dot"] == Nt
    _, cc = o.propagate(lat, psi, Nt, b=b)
    blocks = [min(b, Nt - k) for k in range(0, Nt, b)]
    if Nt % b == 0:
        Nb = Nt // b
        tt_tot = Nt * math.pi
        R_tb = o.truncation(b * math.pi) / (b * math.pi)
        assert cc["amxsy"] == round(tt_tot * R_tb)
        assert cc["axpy"] == Nb * sum(o.truncation(j * math.pi) for j in range(1, b + 1))
    assert cc["amxsy"] == sum(o.truncation(bk * math.pi) for bk in blocks)
    assert cc["axpy"] == sum(sum(o.truncation(j * math.pi) for j in range(1, bk + 1))
                             for bk in blocks)
    assert cc["dot"] == Nt


def test_spectral_centre_shift():
    # with H~ = (H - H0)/|H| the propagator is exp(-i (H - H0) t), so the
    # correlation picks up the phase exp(+i H0 t) relative to exact H
    lat = o.Lattice("square", 5, 4, t=1.0, W=2.0, disorder_seed=6)
    H0, Hn = 0.4, lat.halfwidth() + 0.5
    psi = o.random_phase_states(lat.N, 1, 3)
    Nt = 40
    for b in (0, 9):
        corr, _ = o.propagate(lat, psi, Nt, b=b, Hn=Hn, H0=H0)
        t = np.arange(Nt + 1) * math.pi / Hn
        ref = exact_corr(lat, psi, Nt, Hn)[:, 0] * np.exp(1j * H0 * t)
        assert np.max(np.abs(corr[:, 0] - ref)) < 1e-10


def test_graphene_dos_features():
    # textbook features of the clean graphene DOS (Sec. III's lattice family):
    # linear vanishing at the Dirac point, van Hove peaks at +-|t|, band edges
    # at +-3|t|, one state per orbital; from the Bloch closed form of the
    # propagation (all cells, random-phase state) on a large periodic lattice
    tt, L, Nt = -2.7, 256, 2048
    psi = o.random_phase_states_fast(2 * L * L, 1, 4)
    Hn = 1.025 * 3 * abs(tt)
    corr = o.bloch_corr_uniform("honeycomb", L, L, tt, psi, math.pi / Hn, Nt + 1)
    E, D, _ = o.dos(corr, Hn)
    D = D[:, 0]
    dE = E[1] - E[0]
    assert abs(np.sum(D) * dE - 1.0) < 1e-6
    # peaks of the two halves at +-|t| (within the resolution of the window)
    for sgn in (-1, 1):
        half = (sgn * E > 0.3 * abs(tt)) & (sgn * E < 2.5 * abs(tt))
        Ep = E[half][np.argmax(D[half])]
        assert abs(abs(Ep) - abs(tt)) < 0.1 * abs(tt)
    # Dirac point: far below the van Hove peak, and rising linearly near it
    d0 = D[np.argmin(np.abs(E))]
    assert d0 < 0.1 * np.max(D)
    small = (np.abs(E) > 0.2 * abs(tt)) & (np.abs(E) < 0.5 * abs(tt))
    slope = np.polyfit(np.abs(E[small]), D[small], 1)[0]
    assert slope > 0
    # outside the band (|E| > 3|t| plus a few window widths, up to the grid
    # edge |H| = 1.025 x 3|t|) the DOS vanishes
    outside = np.abs(E) > 3 * abs(tt) * 1.01
    assert np.count_nonzero(outside) > 10
    assert np.max(np.abs(D[outside])) < 1e-3 * np.max(D)
