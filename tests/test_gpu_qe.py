"""GPU parity of the quasi-eigenstates (QE section, QE-Concurrent-E) against
the oracle's sequential form QE-Sequential (forward and backward propagation
and the sum of Eq. QE_coeff over the propagated states).

Tolerances relative to max |Psi|: complex128 1e-10; complex64 (split-bf16
MFMA accumulation) 1e-4.  Cases span one and several contraction chunks,
ragged tiles, several column groups, 1..32 energies and every lattice kind.
"""
import math

import numpy as np
import pytest

import oracle as o

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def csp():
    import paper_2510_17432_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(csp):
    c = csp.Context(0)
    yield c
    c.close()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def pair(csp, ctx, spec):
    g = csp.Lattice(ctx, **spec)
    s = dict(spec)
    kind = s.pop("kind")
    Lx = s.pop("Lx")
    Ly = s.pop("Ly", 1)
    return g, o.Lattice(kind, Lx, Ly, **s)


CASES = [
    # spec, R, energies, Nt
    (dict(kind="square", Lx=23, Ly=19, t=1.0, W=1.0, disorder_seed=3), 1, [0.35], 40),
    (dict(kind="honeycomb", Lx=15, Ly=11, t=-2.7, W=0.5, disorder_seed=4), 3,
     [-6.0, -2.7, 0.0, 1.1, 4.2], 60),
    (dict(kind="chain", Lx=301, t=1.0, W=0.0, periodic_x=False), 2, [-1.5, 0.2, 1.9], 200),
    (dict(kind="square", Lx=17, Ly=13, t=-1.0, W=0.3, disorder_seed=9, periodic_y=False), 1,
     list(np.linspace(-4.0, 4.0, 16)), 100),
]


@pytest.mark.parametrize("mode", ["fp64_conc", "fp32_conc"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_quasi_eigenstates_match_oracle(csp, ctx, mode, case):
    spec, R, E, Nt = CASES[case]
    print("[gpu] quasi-eigenstates %s case %d" % (mode, case), flush=True)
    g, c = pair(csp, ctx, spec)
    psi = o.random_phase_states_fast(c.N, R, 13)
    ref, cnt = o.quasi_eigenstates(c, psi, Nt, E, Hn=g.halfwidth)
    dt = torch.complex128 if mode == "fp64_conc" else torch.complex64
    p = torch.from_numpy(psi).to("cuda:0").to(dt)
    params = csp.make_params(Nt, mode=mode)
    q, rep = csp.csp_quasi_eigenstates(ctx, g, p, params, E)
    got = host(q)
    assert got.shape == (len(E), c.N, R)
    scale = np.max(np.abs(ref))
    err = np.max(np.abs(got - ref)) / scale
    print("[gpu]   max rel error %.2e, orders %d, chunks %d" % (err, rep.amxsy,
                                                                rep.contract_launches), flush=True)
    assert err < (1e-10 if mode == "fp64_conc" else 1e-4)
    assert rep.amxsy == o.truncation(Nt * math.pi)


def test_quasi_eigenstates_32_energies_and_chunks(csp, ctx):
    # complex64 with the most energies and several contraction chunks
    spec = dict(kind="honeycomb", Lx=21, Ly=9, t=-2.7, W=1.0, disorder_seed=6)
    g, c = pair(csp, ctx, spec)
    psi = o.random_phase_states_fast(c.N, 5, 17)
    E = list(np.linspace(-8.0, 8.0, 32))
    Nt = 180
    ref, _ = o.quasi_eigenstates(c, psi, Nt, E, Hn=g.halfwidth)
    p = torch.from_numpy(psi).to("cuda:0").to(torch.complex64)
    q, rep = csp.csp_quasi_eigenstates(ctx, g, p, csp.make_params(Nt, mode="fp32_conc"), E)
    assert rep.contract_launches >= 2 and rep.n_groups == 2
    assert np.max(np.abs(host(q) - ref)) < 1e-4 * np.max(np.abs(ref))


@pytest.mark.parametrize("mode,nE", [("fp32_conc", 49), ("fp64_conc", 37)])
def test_quasi_eigenstates_energy_tiles(csp, ctx, mode, nE):
    # several tiles of energies (32 per tile in complex64, 16 in complex128)
    spec = dict(kind="honeycomb", Lx=13, Ly=9, t=-2.7, W=1.0, disorder_seed=7)
    g, c = pair(csp, ctx, spec)
    psi = o.random_phase_states_fast(c.N, 3, 23)
    E = list(np.linspace(-8.0, 8.0, nE))
    ref, _ = o.quasi_eigenstates(c, psi, 40, E, Hn=g.halfwidth)
    dt = torch.complex128 if mode == "fp64_conc" else torch.complex64
    p = torch.from_numpy(psi).to("cuda:0").to(dt)
    q, rep = csp.csp_quasi_eigenstates(ctx, g, p, csp.make_params(40, mode=mode), E)
    err = np.max(np.abs(host(q) - ref)) / np.max(np.abs(ref))
    assert err < (1e-10 if mode == "fp64_conc" else 1e-4)


def test_quasi_eigenstates_errors(csp, ctx):
    g = csp.Lattice(ctx, "square", 8, 8)
    p = torch.zeros((64, 1), dtype=torch.complex64, device="cuda:0")
    for kw, E in ((dict(mode="fp64_seq"), [0.0]), (dict(mode="fp32_conc"), [0.0] * 129),
                  (dict(mode="fp32_conc"), [])):
        with pytest.raises(csp.CspError) as e:
            csp.csp_quasi_eigenstates(ctx, g, p, csp.make_params(10, **kw), E)
        assert e.value.status == csp.CSP_EINVAL
    with pytest.raises(csp.CspError) as e:
        csp.csp_quasi_eigenstates(ctx, g, p, csp.make_params(0, mode="fp32_conc"), [0.0])
    assert e.value.status == csp.CSP_EINVAL


# ---------------------------------------------------------------- QE-Concurrent-S
QES_CASES = [
    # spec, R, energies, Nt, b
    (dict(kind="square", Lx=23, Ly=19, t=1.0, W=1.0, disorder_seed=3), 1, [0.35], 40, 1),
    (dict(kind="honeycomb", Lx=15, Ly=11, t=-2.7, W=0.5, disorder_seed=4), 5,
     [-6.0, -2.7, 0.0, 1.1, 4.2], 60, 7),
    (dict(kind="chain", Lx=301, t=1.0, W=0.0, periodic_x=False), 2, [-1.5, 0.2, 1.9], 200, 32),
    (dict(kind="square", Lx=17, Ly=13, t=-1.0, W=0.3, disorder_seed=9, periodic_y=False), 3,
     list(np.linspace(-4.0, 4.0, 15)), 100, 64),
    (dict(kind="honeycomb", Lx=9, Ly=8, t=-2.7, W=1.0, disorder_seed=2), 2, [0.5, -1.0], 30, 30),
    (dict(kind="square", Lx=21, Ly=13, t=1.0, W=0.8, disorder_seed=11), 7, [0.1, 1.9], 25, 10),
]


@pytest.mark.parametrize("mode", ["fp64_conc", "fp32_conc"])
@pytest.mark.parametrize("case", range(len(QES_CASES)))
def test_quasi_eigenstates_state_based(csp, ctx, mode, case):
    spec, R, E, Nt, b = QES_CASES[case]
    print("[gpu] QE-Concurrent-S %s case %d (b = %d)" % (mode, case, b), flush=True)
    g, c = pair(csp, ctx, spec)
    psi = o.random_phase_states_fast(c.N, R, 19)
    ref, _ = o.quasi_eigenstates(c, psi, Nt, E, Hn=g.halfwidth)
    dt = torch.complex128 if mode == "fp64_conc" else torch.complex64
    p = torch.from_numpy(psi).to("cuda:0").to(dt)
    q, rep = csp.csp_quasi_eigenstates(ctx, g, p, csp.make_params(Nt, mode=mode, block_b=b), E)
    got = host(q)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print("[gpu]   max rel error %.2e, blocks %d, chunks %d" % (err, rep.n_blocks,
                                                               rep.contract_launches), flush=True)
    assert err < (1e-10 if mode == "fp64_conc" else 1e-4)
    bb = min(b, Nt)
    nb = -(-Nt // bb)
    assert rep.block_b == bb and rep.n_blocks == nb
    Nks = [o.truncation(min(bb, Nt - k * bb) * math.pi) for k in range(nb)]
    assert rep.amxsy == 2 * sum(Nks)


def test_quasi_eigenstates_state_based_largest_and_errors(csp, ctx):
    spec = dict(kind="honeycomb", Lx=11, Ly=9, t=-2.7, W=1.0, disorder_seed=6)
    g, c = pair(csp, ctx, spec)
    psi = o.random_phase_states_fast(c.N, 3, 17)
    E = list(np.linspace(-8.0, 8.0, 31))
    ref, _ = o.quasi_eigenstates(c, psi, 50, E, Hn=g.halfwidth)
    p = torch.from_numpy(psi).to("cuda:0").to(torch.complex64)
    q, _ = csp.csp_quasi_eigenstates(ctx, g, p, csp.make_params(50, mode="fp32_conc", block_b=16), E)
    assert np.max(np.abs(host(q) - ref)) < 1e-4 * np.max(np.abs(ref))
    # the energy-based and the state-based forms agree
    qe_e, _ = csp.csp_quasi_eigenstates(ctx, g, p, csp.make_params(50, mode="fp32_conc"), E)
    assert np.max(np.abs(host(q) - host(qe_e))) < 1e-4 * np.max(np.abs(ref))
    for mode, nE in (("fp32_conc", 32), ("fp64_conc", 16)):
        with pytest.raises(csp.CspError) as e:
            csp.csp_quasi_eigenstates(ctx, g, p if mode == "fp32_conc" else p.to(torch.complex128),
                                      csp.make_params(10, mode=mode, block_b=4), [0.0] * nE)
        assert e.value.status == csp.CSP_EINVAL
