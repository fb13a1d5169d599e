"""GPU parity of the electronic-conductivity correlation (EC section,
EC-Concurrent-M) against the oracle's EC-Sequential form (sequential
propagation of J psi, Eq. dc_corr), and of the conductivity integral of
Eq. DC.

Both sides take the same quasi-eigenstates (the oracle's, QE-Sequential) so
that the comparison isolates the conductivity path.  Tolerances relative to
max |C|: complex128 1e-10; complex64 (split-bf16 MFMA moments, FP32
recursion) 1e-4.  Cases: periodic and open square, honeycomb and chain
lattices, an explicit long-range matrix with coordinates, one and several
column groups, one and several chunks of 128 orders, 1..49 energies (one and
several energy tiles), both
directions, a spectral centre H0 != 0.
"""
import math

import numpy as np
import pytest

import csp_inputs as ci
import oracle as o

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def csp():
    import paper_2510_17432_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(csp):
    print("[gpu] creating context", flush=True)
    c = csp.Context(0)
    yield c
    c.close()


def dev(a, dt):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0").to(dt)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def pair(csp, ctx, spec, **extra):
    g = csp.Lattice(ctx, **spec, **extra)
    s = dict(spec)
    kind = s.pop("kind")
    Lx = s.pop("Lx")
    Ly = s.pop("Ly", 1)
    return g, o.Lattice(kind, Lx, Ly, **s)


def sparse_pair(csp, ctx, L, r_cut, seed):
    col, val = ci.long_range_square(L, r_cut, t0=-1.0, decay=1.5, W=0.7, seed=seed)
    pos, box = ci.long_range_square_positions(L)
    g = csp.Lattice.sparse(ctx, col, val)
    g.set_positions(pos, box)
    return g, o.SparseLattice(col, val, pos=pos, box=box)


CASES = [
    # spec, R, energies, Nt (qe), Nt (EC)
    (dict(kind="square", Lx=23, Ly=19, t=1.0, W=1.0, disorder_seed=3), 2, [-1.2, 0.3, 2.0], 20, 40),
    (dict(kind="honeycomb", Lx=15, Ly=11, t=-2.7, W=0.5, disorder_seed=4), 3,
     [-6.0, -2.7, 0.0, 1.1, 4.2], 20, 60),
    (dict(kind="honeycomb", Lx=9, Ly=7, t=-2.7, W=1.0, disorder_seed=5, periodic_x=False), 1,
     [0.4], 15, 50),
    (dict(kind="chain", Lx=301, t=1.0, W=0.5, disorder_seed=6), 2, [-1.0, 0.5], 30, 200),
]


def check(csp, ctx, g, c, R, E, nt_qe, Nt, alpha, mode, seed=13, H0=0.0):
    psi = o.random_phase_states_fast(c.N, R, seed)
    qe, _ = o.quasi_eigenstates(c, psi, nt_qe, E, Hn=g.halfwidth, H0=H0)
    ref, _ = o.ec_correlation(c, psi, qe, Nt, alpha, Hn=g.halfwidth, H0=H0)
    dt = torch.complex128 if mode == "fp64_conc" else torch.complex64
    corr, rep = csp.csp_ec_correlation(ctx, g, alpha, dev(psi, dt), dev(qe, dt),
                                       csp.make_params(Nt, mode=mode))
    got = host(corr)
    assert got.shape == (len(E), Nt + 1, R)
    scale = np.max(np.abs(ref))
    err = np.max(np.abs(got - ref)) / scale
    print("[gpu]   %s alpha=%d: max rel error %.2e (scale %.3g), orders %d, chunks %d" % (
        mode, alpha, err, scale, rep.amxsy, rep.contract_launches), flush=True)
    assert err < (1e-10 if mode == "fp64_conc" else 1e-4)
    assert rep.amxsy == o.truncation(Nt * math.pi)
    assert rep.dot == (rep.amxsy + 1) * len(E)
    return got, ref


@pytest.mark.parametrize("mode", ["fp64_conc", "fp32_conc"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_ec_correlation_matches_oracle(csp, ctx, mode, case):
    spec, R, E, nt_qe, Nt = CASES[case]
    print("[gpu] EC %s case %d" % (mode, case), flush=True)
    g, c = pair(csp, ctx, spec)
    for alpha in ((0, 1) if spec["kind"] != "chain" else (0,)):
        check(csp, ctx, g, c, R, E, nt_qe, Nt, alpha, mode)


@pytest.mark.parametrize("mode", ["fp64_conc", "fp32_conc"])
def test_ec_explicit_matrix(csp, ctx, mode):
    g, c = sparse_pair(csp, ctx, 14, 3.0, 2)
    for alpha in (0, 1):
        # 5 energies x 3 columns (waves of 2 + 1): the current operator over
        # two tiles of 8 bras
        check(csp, ctx, g, c, 3, [-2.0, -0.7, 0.1, 0.9, 1.5], 15, 45, alpha, mode)


def test_ec_spectral_centre(csp, ctx):
    spec = dict(kind="square", Lx=13, Ly=11, t=1.0, W=1.2, disorder_seed=7)
    g, c = pair(csp, ctx, spec, halfwidth_override=5.3, center=0.35)
    assert g.info.H0 == 0.35
    check(csp, ctx, g, c, 1, [0.2, -0.9], 12, 30, 0, "fp64_conc", H0=0.35)


def test_ec_many_energies(csp, ctx):
    # one and several energy tiles (32 per tile in complex64; in complex128 16,
    # or up to 24 with more than 16 energies)
    spec = dict(kind="honeycomb", Lx=12, Ly=10, t=-2.7, W=1.0, disorder_seed=8)
    g, c = pair(csp, ctx, spec)
    check(csp, ctx, g, c, 2, list(np.linspace(-7.0, 7.0, 32)), 10, 30, 1, "fp32_conc")
    check(csp, ctx, g, c, 2, list(np.linspace(-7.0, 7.0, 49)), 10, 30, 0, "fp32_conc")
    check(csp, ctx, g, c, 1, list(np.linspace(-7.0, 7.0, 16)), 10, 30, 0, "fp64_conc")
    check(csp, ctx, g, c, 1, list(np.linspace(-7.0, 7.0, 37)), 10, 30, 1, "fp64_conc")
    # complex128 tiles of up to 24 energies: one of 17, three of 17 + 16 + 16
    check(csp, ctx, g, c, 1, list(np.linspace(-7.0, 7.0, 17)), 10, 30, 0, "fp64_conc")
    check(csp, ctx, g, c, 2, list(np.linspace(-7.0, 7.0, 49)), 10, 30, 1, "fp64_conc")


@pytest.mark.parametrize("mode", ["fp64_conc", "fp32_conc"])
def test_ec_three_groups_and_one_step(csp, ctx, mode):
    # 7 columns (groups 4 + 2 + 1), Nt = 1 (one chunk of N(pi) + 1 orders), ragged N
    spec = dict(kind="square", Lx=21, Ly=13, t=-1.0, W=0.8, disorder_seed=10)
    g, c = pair(csp, ctx, spec)
    check(csp, ctx, g, c, 7, [-0.5, 1.3], 8, 1, 1, mode)
    check(csp, ctx, g, c, 7, [0.2], 8, 33, 0, mode)


def test_ec_sigma_matches_oracle(csp, ctx):
    spec = CASES[0][0]
    g, c = pair(csp, ctx, spec)
    E = CASES[0][2]
    got, ref = check(csp, ctx, g, c, 2, E, 20, 40, 0, "fp64_conc")
    dA = [0.3, 1.0, 2.5]
    s = host(csp.csp_ec_sigma(ctx, torch.from_numpy(got).to("cuda:0"), g.halfwidth, E,
                              dos_over_area=dA))
    s_ref = o.ec_sigma(got, E, g.halfwidth, dos_over_area=dA)
    assert np.max(np.abs(s - s_ref)) < 1e-12 * max(1.0, np.max(np.abs(s_ref)))
    # and against the oracle's correlations, at the correlation tolerance
    s_seq = o.ec_sigma(ref, E, g.halfwidth, dos_over_area=dA)
    assert np.max(np.abs(s - s_seq)) < 1e-9 * max(1.0, np.max(np.abs(s_seq)))


def test_ec_with_gpu_quasi_eigenstates(csp, ctx):
    # the composed path: quasi-eigenstates and conductivity both on the GPU
    spec = CASES[1][0]
    g, c = pair(csp, ctx, spec)
    psi = o.random_phase_states_fast(c.N, 2, 21)
    E = [-2.7, 0.5]
    qe_ref, _ = o.quasi_eigenstates(c, psi, 20, E, Hn=g.halfwidth)
    ref, _ = o.ec_correlation(c, psi, qe_ref, 50, 1, Hn=g.halfwidth)
    p = dev(psi, torch.complex128)
    qe, _ = csp.csp_quasi_eigenstates(ctx, g, p, csp.make_params(20, mode="fp64_conc"), E)
    corr, _ = csp.csp_ec_correlation(ctx, g, 1, p, qe, csp.make_params(50, mode="fp64_conc"))
    assert np.max(np.abs(host(corr) - ref)) < 1e-10 * np.max(np.abs(ref))


def test_ec_errors(csp, ctx):
    g = csp.Lattice(ctx, "square", 8, 8)
    p = torch.zeros((64, 1), dtype=torch.complex64, device="cuda:0")
    q = torch.zeros((1, 64, 1), dtype=torch.complex64, device="cuda:0")
    for alpha, kw, qq in ((0, dict(mode="fp64_seq"), q), (2, dict(mode="fp32_conc"), q),
                          (0, dict(mode="fp32_conc"), q.repeat(129, 1, 1))):
        with pytest.raises(csp.CspError) as e:
            csp.csp_ec_correlation(ctx, g, alpha, p, qq, csp.make_params(10, **kw))
        assert e.value.status == csp.CSP_EINVAL
    with pytest.raises(csp.CspError) as e:
        g.set_positions(np.zeros((64, 2)))
    assert e.value.status == csp.CSP_EUNSUPPORTED
    col, val = ci.long_range_square(6, 1.5, seed=1)
    gs = csp.Lattice.sparse(ctx, col, val)
    p36 = torch.zeros((36, 1), dtype=torch.complex64, device="cuda:0")
    q36 = torch.zeros((1, 36, 1), dtype=torch.complex64, device="cuda:0")
    with pytest.raises(csp.CspError) as e:
        csp.csp_ec_correlation(ctx, gs, 0, p36, q36, csp.make_params(10, mode="fp32_conc"))
    assert e.value.status == csp.CSP_EINVAL
    with pytest.raises(csp.CspError) as e:
        gs.set_positions(np.full((36, 2), np.nan))
    assert e.value.status == csp.CSP_EINVAL
