"""Pins of the quasi-eigenstate oracle (QE section, Eq. QE / Eq. QE_coeff).

With the eigen-decomposition H v_k = E_k v_k, psi(t) = sum_k e^{-i E_k t}
<v_k|psi0> v_k, so the discretised time integral of Eq. QE is a filter of
the spectrum:
  Psi(E) = sum_k g(E - E_k) <v_k|psi0> v_k,
  g(w) = tau_p [1 + 2 sum_{j=1}^{Nt} cos(w t_j)],  t_j = j tau_p.
This closed form (exact diagonalisation) pins the forward and backward
propagation, their coefficients c_n(-x) = conj(c_n(x)) and the weights
(2 - delta_j0)/2; the projection <psi0|Psi(E)> is pinned against the
correlations of the sequential propagation, a separate code path.
"""
import math

import numpy as np
import pytest

import oracle as o


def dense(lat):
    H = np.zeros((lat.N, lat.N))
    for s in range(lat.N):
        for p in range(lat.rowptr[s], lat.rowptr[s + 1]):
            H[s, lat.col[p]] += lat.val[p]
    return H


def exact_qe(lat, psi, Nt, energies, Hn):
    w, V = np.linalg.eigh(dense(lat))
    tp = math.pi / Hn
    j = np.arange(1, Nt + 1)
    amp = V.conj().T @ psi                          # [k][R]
    out = []
    for E in energies:
        g = tp * (1.0 + 2.0 * np.cos(np.outer(E - w, j * tp)).sum(1))
        out.append(V @ (g[:, None] * amp))
    return np.array(out)


@pytest.mark.parametrize("spec", [
    dict(kind="square", Lx=6, Ly=5, t=1.0, W=0.7, disorder_seed=3),
    dict(kind="honeycomb", Lx=4, Ly=3, t=-2.7, W=0.4, disorder_seed=5),
    dict(kind="chain", Lx=17, t=1.0, W=0.0, periodic_x=False),
])
def test_qe_matches_exact_diagonalisation(spec):
    kind = spec.pop("kind")
    lat = o.Lattice(kind, **spec)
    psi = o.random_phase_states_fast(lat.N, 2, 7)
    Hn = lat.halfwidth(1.025)
    E = [-1.3, 0.0, 0.45, 2.1]
    Nt = 60
    got, cnt = o.quasi_eigenstates(lat, psi, Nt, E, Hn=Hn)
    ref = exact_qe(lat, psi, Nt, E, Hn)
    assert got.shape == (len(E), lat.N, 2)
    assert np.max(np.abs(got - ref)) < 1e-10 * np.max(np.abs(ref))
    # forward and backward: 2 N(pi) recursion steps per time step and column
    assert cnt["amxsy"] == 2 * 2 * Nt * o.truncation(math.pi)


def test_qe_shift_of_the_spectral_centre():
    # H~ = (H - H0)/|H| with H0 != 0: the filter still selects E_k = E
    lat = o.Lattice("square", 5, 5, t=1.0, W=1.0, disorder_seed=2)
    psi = o.random_phase_states_fast(lat.N, 1, 3)
    H0 = 0.4
    Hn = lat.halfwidth(1.025) + abs(H0)
    E = [-0.8, 1.1]
    got, _ = o.quasi_eigenstates(lat, psi, 40, E, Hn=Hn, H0=H0)
    ref = exact_qe(lat, psi, 40, E, Hn)
    assert np.max(np.abs(got - ref)) < 1e-10 * np.max(np.abs(ref))


def test_qe_projection_equals_correlation_transform():
    # <psi0|Psi(E)> = tau_p [C_0 + 2 sum_j Re(e^{iE t_j} C_j)] with C_j from the
    # sequential propagation (C_{-j} = conj(C_j) for Hermitian H)
    lat = o.Lattice("honeycomb", 6, 4, t=-2.7, W=1.0, disorder_seed=8)
    psi = o.random_phase_states_fast(lat.N, 1, 9)
    Hn = lat.halfwidth(1.025)
    Nt = 50
    E = [-3.0, 0.7]
    q, _ = o.quasi_eigenstates(lat, psi, Nt, E, Hn=Hn)
    C, _ = o.propagate(lat, psi, Nt, b=0, Hn=Hn)
    tp = math.pi / Hn
    t = np.arange(1, Nt + 1) * tp
    for e, En in enumerate(E):
        proj = np.vdot(psi[:, 0], q[e, :, 0])
        want = tp * (C[0, 0] + 2.0 * np.real(np.exp(1j * En * t) * C[1:, 0]).sum())
        assert abs(proj - want) < 1e-11 * abs(want) + 1e-13
        assert abs(proj.imag) < 1e-10 * abs(proj)     # the filter is real
