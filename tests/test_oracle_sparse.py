"""Pins of the oracle for Hamiltonians given explicitly (ELL form, any matrix
density D_H of Sec. II.B): the same matrix as a stencil lattice gives the
same propagation, exact diagonalisation on a long-range lattice, and the
Gershgorin bound."""
import math

import numpy as np
import pytest

import csp_inputs as ci
import oracle as o


def ell_from_lattice(lat):
    D = int(np.max(np.diff(lat.rowptr)))
    col = -np.ones((lat.N, D), dtype=np.int64)
    val = np.zeros((lat.N, D))
    for s in range(lat.N):
        a, b = lat.rowptr[s], lat.rowptr[s + 1]
        col[s, :b - a] = lat.col[a:b]
        val[s, :b - a] = lat.val[a:b]
    return col, val


def test_stencil_matrix_as_ell_propagates_identically():
    lat = o.Lattice("honeycomb", 7, 5, t=-2.7, W=1.0, disorder_seed=4)
    sp = o.SparseLattice(*ell_from_lattice(lat))
    psi = o.random_phase_states_fast(lat.N, 2, 3)
    Hn = lat.halfwidth(1.025)
    assert np.array_equal(sp.rowptr, lat.rowptr) and np.array_equal(sp.col, lat.col)
    assert np.array_equal(sp.val, lat.val)
    a, _ = o.propagate(lat, psi, 30, b=8, Hn=Hn)
    b, _ = o.propagate(sp, psi, 30, b=8, Hn=Hn)
    # same matrix; the threaded dot products may combine in another order
    assert np.max(np.abs(a - b)) < 1e-14


def test_long_range_lattice_recipe():
    col, val = ci.long_range_square(12, 3.2, t0=1.0, decay=1.5, W=0.8, seed=5)
    # 1 + lattice vectors with 0 < |v| <= 3.2
    want = 1 + sum(1 for dx in range(-3, 4) for dy in range(-3, 4)
                   if 0 < dx * dx + dy * dy <= 3.2 * 3.2)
    assert col.shape == (144, want)
    H = o.SparseLattice(col, val).dense()
    assert np.array_equal(H, H.T)                   # Hermitian (real symmetric)


def test_long_range_propagation_matches_exact_diagonalisation():
    col, val = ci.long_range_square(10, 2.9, t0=-1.0, decay=1.2, W=0.5, seed=2)
    sp = o.SparseLattice(col, val)
    Hn = sp.halfwidth(1.025)
    w, V = np.linalg.eigh(sp.dense())
    assert np.max(np.abs(w)) <= Hn / 1.025 * (1 + 1e-12)     # Gershgorin encloses
    psi = o.random_phase_states_fast(sp.N, 1, 6)
    Nt = 40
    C, _ = o.propagate(sp, psi, Nt, b=0, Hn=Hn)
    t = np.arange(Nt + 1) * math.pi / Hn
    amp = np.abs(V.T @ psi[:, 0]) ** 2
    ref = (amp[None, :] * np.exp(-1j * np.outer(t, w))).sum(1)
    assert np.max(np.abs(C[:, 0] - ref)) < 1e-10
    Cm, _ = o.propagate_moments(sp, psi, Nt, Hn=Hn)
    assert np.max(np.abs(Cm[:, 0] - ref)) < 1e-10
