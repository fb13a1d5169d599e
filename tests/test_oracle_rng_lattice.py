"""Pins for the oracle's generator, lattices and spectral bound.

Each test checks the oracle against something other than itself: published
generator outputs, closed-form band structures, counting identities and
Gershgorin's theorem checked by exact diagonalisation.
"""
import math

import numpy as np
import pytest

import oracle as o


# ------------------------------------------------------------------ generator
def test_splitmix64_published_outputs(golden):
    g = golden("splitmix64.txt")
    for k in range(3):
        assert o.splitmix64(0, k) == int(g["seed0_out%d" % k], 16)


def test_splitmix64_counter_equals_stateful_stream():
    for seed in (0, 1, 12345, 2**63 + 17):
        s = o.splitmix64_stream(seed, 50)
        for k in (0, 1, 7, 49):
            assert int(s[k]) == o.splitmix64(seed, k)


def test_draw_stream_layout():
    # stream r, index s is counter r*2^40 + s of the same generator
    assert o.draw(9, 3, 5) == o.splitmix64(9, (3 << 40) + 5)


def test_u01_uniform_chi_square():
    n, bins = 20000, 20
    u = np.array([o.u01(o.draw(77, 0, i)) for i in range(n)])
    assert u.min() >= 0.0 and u.max() < 1.0
    h, _ = np.histogram(u, bins=bins, range=(0, 1))
    chi2 = float(np.sum((h - n / bins) ** 2 / (n / bins)))
    # 19 degrees of freedom: P(chi2 > 45) ~ 7e-4
    assert chi2 < 45.0


def test_below_range_and_extremes():
    assert o.below(0, 10) == 0
    assert o.below(2**64 - 1, 10) == 9
    assert o.below(2**63, 10) == 5
    vals = [o.below(o.draw(5, 0, i), 7) for i in range(7000)]
    counts = np.bincount(vals, minlength=7)
    assert counts.min() > 850 and counts.max() < 1150


def test_fast_phase_states_match_loop():
    a = o.random_phase_states(50, 3, 11)
    b = o.random_phase_states_fast(50, 3, 11)
    assert np.array_equal(a, b)
    assert np.allclose(np.linalg.norm(a, axis=0), 1.0, atol=1e-14)
    assert np.allclose(np.abs(a), 1.0 / math.sqrt(50), atol=1e-15)


def test_ldos_sites_distinct_and_deterministic():
    s1 = o.ldos_sites(1000, 64, 3)
    s2 = o.ldos_sites(1000, 64, 3)
    assert np.array_equal(s1, s2)
    assert len(set(s1.tolist())) == 64
    assert s1.min() >= 0 and s1.max() < 1000
    # all sites of a tiny lattice: a permutation
    assert sorted(o.ldos_sites(5, 5, 1).tolist()) == [0, 1, 2, 3, 4]


# ------------------------------------------------------------------ lattices
@pytest.mark.parametrize("kind,Lx,Ly,nb_per_cell", [
    ("chain", 9, 1, 1), ("square", 5, 4, 2), ("honeycomb", 4, 3, 3)])
def test_bond_counts_periodic(kind, Lx, Ly, nb_per_cell):
    lat = o.Lattice(kind, Lx, Ly)
    cells = Lx * (Ly if kind != "chain" else 1)
    assert lat.nbonds == nb_per_cell * cells
    deg = {"chain": 2, "square": 4, "honeycomb": 3}[kind]
    assert np.all(lat.degree() == deg)


def test_bond_counts_open():
    # open square Lx x Ly: (Lx-1)Ly + Lx(Ly-1) bonds
    lat = o.Lattice("square", 5, 4, periodic_x=False, periodic_y=False)
    assert lat.nbonds == 4 * 4 + 5 * 3
    # open honeycomb: Lx*Ly + (Lx-1)*Ly + Lx*(Ly-1)
    lat = o.Lattice("honeycomb", 4, 3, periodic_x=False, periodic_y=False)
    assert lat.nbonds == 12 + 9 + 8
    lat = o.Lattice("chain", 6, periodic_x=False)
    assert lat.nbonds == 5


def test_hamiltonian_symmetric_and_onsite():
    lat = o.Lattice("honeycomb", 3, 4, t=-2.7, W=1.0, disorder_seed=4)
    H = lat.dense()
    assert np.array_equal(H, H.T)
    assert np.array_equal(np.diag(H), lat.eps)
    assert np.all(np.abs(lat.eps) <= 0.5)


def test_onsite_uniform_distribution():
    lat = o.Lattice("square", 100, 100, W=2.0, disorder_seed=8)
    from scipy import stats
    p = stats.kstest((lat.eps + 1.0) / 2.0, "uniform").pvalue
    assert p > 1e-3


def _square_bloch(Lx, Ly, t):
    kx = 2 * np.pi * np.arange(Lx) / Lx
    ky = 2 * np.pi * np.arange(Ly) / Ly
    return (2 * t * (np.cos(kx)[None, :] + np.cos(ky)[:, None])).ravel()


def _honeycomb_bloch(Lx, Ly, t):
    k1 = 2 * np.pi * np.arange(Lx) / Lx
    k2 = 2 * np.pi * np.arange(Ly) / Ly
    f = 1 + np.exp(-1j * k1)[None, :] + np.exp(-1j * k2)[:, None]
    e = np.abs(t * f).ravel()
    return np.concatenate([e, -e])


def test_square_spectrum_is_bloch_band():
    lat = o.Lattice("square", 6, 5, t=1.0)
    ev = np.linalg.eigvalsh(lat.dense())
    assert np.allclose(np.sort(ev), np.sort(_square_bloch(6, 5, 1.0)), atol=1e-12)


def test_honeycomb_spectrum_is_bloch_band():
    lat = o.Lattice("honeycomb", 5, 4, t=-2.7)
    ev = np.linalg.eigvalsh(lat.dense())
    assert np.allclose(np.sort(ev), np.sort(_honeycomb_bloch(5, 4, -2.7)), atol=1e-12)


def test_chain_spectrum_and_small_periodic_repeats():
    lat = o.Lattice("chain", 11, t=0.7)
    ev = np.linalg.eigvalsh(lat.dense())
    ref = 2 * 0.7 * np.cos(2 * np.pi * np.arange(11) / 11)
    assert np.allclose(np.sort(ev), np.sort(ref), atol=1e-12)
    # L = 2 periodic square: both x-bonds join the same pair, H_ab = 2t
    lat2 = o.Lattice("square", 2, 3, t=1.0)
    ev2 = np.linalg.eigvalsh(lat2.dense())
    assert np.allclose(np.sort(ev2), np.sort(_square_bloch(2, 3, 1.0)), atol=1e-12)


def test_gershgorin_halfwidth_values():
    # config values: square t=1 -> 4.1; graphene t=-2.7 -> 8.3025
    assert o.Lattice("square", 8, 8, t=1.0).halfwidth() == pytest.approx(4.1, abs=1e-15)
    assert o.Lattice("honeycomb", 6, 6, t=-2.7).halfwidth() == pytest.approx(8.3025, abs=1e-14)


@pytest.mark.parametrize("kind", ["chain", "square", "honeycomb"])
def test_gershgorin_encloses_spectrum(kind):
    lat = o.Lattice(kind, 7, 6, t=-1.3, W=2.5, disorder_seed=21,
                    periodic_x=True, periodic_y=False)
    ev = np.linalg.eigvalsh(lat.dense())
    hw = lat.halfwidth(margin=1.0)
    assert np.max(np.abs(ev)) <= hw + 1e-12
