"""Pins for the oracle's moment-based form (Sec. II.A moment-based
implementation; Sec. III DOS-Concurrent-M with the halving of
Eq. cheby_prod).

Against: the sequential form and exact diagonalisation; the Chebyshev
product identity on explicit Chebyshev vectors (which also fixes the
factor 2 that Eq. cheby-moment omits); the operation counts of Tab. (cost);
the final state of the sequential form.
"""
import math

import numpy as np
import pytest

import oracle as o
from test_oracle_propagation import exact_corr

LATS = [("honeycomb", 8, 7, -2.7, 1.0), ("square", 9, 6, 1.0, 0.7), ("chain", 40, 1, 1.0, 1.5)]


@pytest.mark.parametrize("kind,Lx,Ly,t,W", LATS)
@pytest.mark.parametrize("b,halving", [(None, True), (None, False), (1, False), (9, False)])
def test_moments_equal_exact_diagonalisation(kind, Lx, Ly, t, W, b, halving):
    lat = o.Lattice(kind, Lx, Ly, t=t, W=W, disorder_seed=3)
    Hn = lat.halfwidth()
    psi = np.concatenate([o.random_phase_states_fast(lat.N, 2, 7),
                          o.site_states(lat.N, [3])], axis=1)
    Nt = 90
    corr, _ = o.propagate_moments(lat, psi, Nt, b=b, halving=halving)
    assert np.max(np.abs(corr - exact_corr(lat, psi, Nt, Hn))) < 1e-11


def test_moments_equal_sequential_long_run(golden):
    scale = float(golden("dos_accuracy.txt")["eps_inf_correlation"])
    lat = o.Lattice("honeycomb", 20, 18, t=-2.7, W=1.0, disorder_seed=4)
    psi = o.random_phase_states_fast(lat.N, 1, 5)
    Nt = 1024
    seq, _ = o.propagate(lat, psi, Nt, b=0)
    mom, _ = o.propagate_moments(lat, psi, Nt, b=None, halving=True)
    assert np.max(np.abs(mom - seq)) < 100 * scale


def test_doubling_identity_needs_the_factor_two():
    # 2 T_k T_k = T_2k + T_0 and 2 T_{k+1} T_k = T_{2k+1} + T_1: with T_n
    # Hermitian, <phi_k|phi_k> = (mu_2k + mu_0)/2 and
    # <phi_{k+1}|phi_k> = (mu_{2k+1} + mu_1)/2.  The printed form without the
    # factor 2 on the inner product is off by O(1).
    lat = o.Lattice("square", 7, 6, t=1.0, W=1.0, disorder_seed=2)
    Hn = lat.halfwidth()
    psi = o.random_phase_states_fast(lat.N, 1, 3)[:, 0]
    K = 30
    phi = o.chebyshev_vectors(lat, psi, 2 * K + 1, Hn)
    mu = phi.conj() @ psi          # <phi_n|psi> = <psi|T_n|psi>^* (real here)
    mu = np.conj(mu)
    for k in range(1, K):
        self_k = np.vdot(phi[k], phi[k])
        cross = np.vdot(phi[k + 1], phi[k])
        assert abs(2 * self_k - mu[0] - mu[2 * k]) < 1e-12
        assert abs(2 * cross - mu[1] - mu[2 * k + 1]) < 1e-12
    assert abs((np.vdot(phi[5], phi[5]) - mu[0]) - mu[10]) > 0.1


@pytest.mark.parametrize("Nt", [64, 50, 1000])
def test_moment_operation_counts_match_cost_table(Nt):
    """Tab. (cost), DOS-Concurrent-M: t_tot R(t_tot)/2 = N(t_tot)/2
    recursion steps (rounded up: orders 1..ceil(N/2) are generated), no axpy,
    N(t_tot) moments from inner products, 3 states."""
    lat = o.Lattice("chain", 10, t=1.0)
    psi = o.random_phase_states(lat.N, 1, 1)
    N = o.truncation(Nt * math.pi)
    _, c = o.propagate_moments(lat, psi, Nt, b=None, halving=True)
    assert c["amxsy"] == (N + 1) // 2 and c["axpy"] == 0 and c["dot"] == N
    _, c = o.propagate_moments(lat, psi, Nt, b=None, halving=False)
    assert c["amxsy"] == N and c["dot"] == N
    # blocks: the recursion count of the state-based form, one carry axpy per order
    b = 16
    blocks = [min(b, Nt - k) for k in range(0, Nt, b)]
    _, c = o.propagate_moments(lat, psi, Nt, b=b, halving=False)
    tot = sum(o.truncation(bk * math.pi) for bk in blocks)
    assert c["amxsy"] == tot and c["axpy"] == tot and c["dot"] == tot


def test_block_moments_final_state_equals_sequential():
    lat = o.Lattice("honeycomb", 9, 8, t=-2.7, W=0.8, disorder_seed=6)
    psi = o.random_phase_states_fast(lat.N, 2, 2)
    _, _, f_seq = o.propagate(lat, psi, 70, b=0, return_final=True)
    for b in (8, 70):
        _, _, f_mom = o.propagate_moments(lat, psi, 70, b=b, halving=False, return_final=True)
        assert np.max(np.abs(f_mom - f_seq)) < 1e-12
    with pytest.raises(RuntimeError):
        o.propagate_moments(lat, psi, 70, b=8, halving=True)
