"""GPU parity for Hamiltonians given explicitly in ELL form (general matrices
of any density D_H, Sec. II.B) against the FP64 oracle on the same matrix.

Bit-exact: the Gershgorin half-width (max row sum of |H_sk| in entry order,
times the margin).  FP64 paths: 1e-10 on correlations and quasi-eigenstates
(1e-13 relative for single steps).  FP32 concurrent path: correlations within
2e-5 absolute and DOS within 1e-4 relative, as for the stencil lattices.
Matrices: the long-range square lattice (every row D = 29 or 49 entries,
no padding) and random symmetric matrices with irregular rows (padding).
All but the largest random matrix run the LDS-staged (windowed) recursion;
that one, the stencil written out in ELL form, and the slices of the
overflow matrix whose windows exceed the LDS budget gather from global
memory.
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


MATS = {
    "lr3": lambda: ci.long_range_square(16, 3.0, t0=-1.0, decay=1.5, W=1.0, seed=2),
    "lr4": lambda: ci.long_range_square(19, 4.0, t0=1.0, decay=1.0, W=0.5, seed=5),
    "rand": lambda: ci.random_symmetric_ell(700, 2500, seed=3),
    "rand_nodiag": lambda: ci.random_symmetric_ell(301, 400, seed=4, diag=False),
    "rand_big": lambda: ci.random_symmetric_ell(6000, 20000, seed=9),
}


def pair(csp, ctx, name, margin=0.0):
    col, val = MATS[name]()
    return csp.Lattice.sparse(ctx, col, val, margin=margin), o.SparseLattice(col, val)


def rel_dos_err(c32, c64, Hn):
    _, D32, _ = o.dos(c32, Hn)
    _, D64, _ = o.dos(c64, Hn)
    return np.max(np.abs(D32.mean(1) - D64.mean(1))) / np.max(np.abs(D64.mean(1)))


@pytest.mark.parametrize("name", sorted(MATS))
@pytest.mark.parametrize("margin", [0.0, 1.1])
def test_halfwidth_bit_exact_and_info(csp, ctx, name, margin):
    g, c = pair(csp, ctx, name, margin)
    assert g.halfwidth == c.halfwidth(margin if margin > 0 else 1.025)
    assert g.info.n_orb == c.N and g.info.max_degree == c.D
    assert g.info.H0 == 0.0 and g.info.has_onsite == 0
    for f in (g.onsite, g.neighbors):
        with pytest.raises(csp.CspError) as e:
            f()
        assert e.value.status == csp.CSP_EUNSUPPORTED


def test_windowed_layout_in_use(csp, ctx):
    # lattices whose slices of 128 neighbouring rows name few columns, and
    # matrices small enough that a slice's window is most of the vector, run
    # the LDS-staged recursion; a large random matrix (every slice names
    # about as many columns as it has entries) keeps the slice layout
    for name, want in (("lr3", 1), ("lr4", 1), ("rand", 1), ("rand_nodiag", 1),
                       ("rand_big", 0)):
        g, c = pair(csp, ctx, name)
        assert g.info.ell_windowed == want, name
        if want:
            assert 0 < g.info.ell_max_window <= c.N


@pytest.mark.parametrize("mode,b,R", [("fp32_conc", 16, 5), ("fp64_conc", 8, 3),
                                      ("fp32_conc", 0, 2), ("fp64_seq", 0, 1)])
def test_windows_that_overflow_the_lds(csp, ctx, mode, b, R):
    # most slices stage their window, the slices holding the rows with far
    # entries (windows above the LDS budget of 8 or 4 columns) gather from
    # global memory, in the same launch
    print("[gpu] sparse windows overflow %s b=%d R=%d" % (mode, b, R), flush=True)
    col, val = ci.long_range_with_far_pairs()
    g = csp.Lattice.sparse(ctx, col, val)
    c = o.SparseLattice(col, val)
    assert g.info.ell_windowed == 1 and g.info.ell_max_window > 2048
    psi = o.random_phase_states_fast(c.N, R, 17)
    Nt = 60
    ref, _ = o.propagate(c, psi, Nt, b=0, Hn=g.halfwidth)
    got, _, _ = run(csp, ctx, g, psi, Nt, mode, b=b)
    tol = 2e-5 if mode == "fp32_conc" else 1e-10
    assert np.max(np.abs(got - ref)) < tol
    if mode != "fp64_seq":
        mref, _ = o.propagate_moments(c, psi, Nt, b=None, halving=True, Hn=g.halfwidth)
        mgot, _, _ = run(csp, ctx, g, psi, Nt, mode, assembly=csp.CSP_ASSEMBLE_MOMENTS)
        assert np.max(np.abs(mgot - mref)) < tol


def test_creation_errors(csp, ctx):
    col, val = ci.random_symmetric_ell(50, 60, seed=1)
    bad = col.copy()
    bad[3, 0] = 50
    nan = val.copy()
    nan[4, 0] = np.nan
    for cc, vv in ((bad, val), (col, nan), (col, np.zeros_like(val)),
                   (np.zeros((0, 3), np.int32), np.zeros((0, 3)))):
        with pytest.raises(csp.CspError) as e:
            csp.Lattice.sparse(ctx, cc, vv)
        assert e.value.status == csp.CSP_EINVAL


@pytest.mark.parametrize("name", ["lr3", "rand"])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_chebyshev_step(csp, ctx, name, dtype):
    g, c = pair(csp, ctx, name)
    R = 3
    rng = np.random.default_rng(7)
    x = rng.normal(size=(c.N, R)) + 1j * rng.normal(size=(c.N, R))
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    xd = dev(x).to(tdt)
    y1 = torch.zeros_like(xd)
    csp.csp_chebyshev_step(ctx, g, xd, y1, first=True)
    y2 = xd.clone()
    csp.csp_chebyshev_step(ctx, g, y1, y2, first=False)
    ref = np.stack([o.chebyshev_vectors(c, x[:, r], 2, g.halfwidth) for r in range(R)], -1)
    tol = 1e-13 if dtype == "c128" else 2e-6
    scale = np.max(np.abs(x))
    assert np.max(np.abs(host(y1) - ref[1])) < tol * scale
    assert np.max(np.abs(host(y2) - ref[2])) < tol * 3 * scale


def run(csp, ctx, g, psi, Nt, mode, b=0, assembly=None, final=False):
    tdt = torch.complex128 if mode != "fp32_conc" else torch.complex64
    p = dev(psi).to(tdt)
    kw = {} if assembly is None else dict(assembly=assembly)
    params = csp.make_params(Nt, mode=mode, block_b=b, **kw)
    fin = torch.zeros_like(p) if final else None
    corr, rep = csp.csp_propagate(ctx, g, p, params, final=fin)
    return host(corr), rep, (host(fin) if final else None)


@pytest.mark.parametrize("name", ["lr3", "rand", "rand_nodiag", "rand_big"])
@pytest.mark.parametrize("mode,b", [("fp64_seq", 0), ("fp64_conc", 13), ("fp32_conc", 32),
                                    ("fp32_conc", 7)])
def test_state_assembly_matches_oracle(csp, ctx, name, mode, b):
    print("[gpu] sparse %s %s b=%d" % (name, mode, b), flush=True)
    g, c = pair(csp, ctx, name)
    # one group of 5 columns: waves of 4 + 1
    psi = o.random_phase_states_fast(c.N, 5, 5)
    Nt = 120
    ref, cnt = o.propagate(c, psi, Nt, b=0, Hn=g.halfwidth)
    got, rep, _ = run(csp, ctx, g, psi, Nt, mode, b=b)
    assert rep.spmm_steps == 1
    if mode.startswith("fp64"):
        assert np.max(np.abs(got - ref)) < 1e-10
        if mode == "fp64_seq":
            assert rep.amxsy * 5 == cnt["amxsy"]
    else:
        assert np.max(np.abs(got - ref)) < 2e-5
        assert rel_dos_err(got, ref, g.halfwidth) < 1e-4


@pytest.mark.parametrize("mode", ["fp64_seq", "fp64_conc", "fp32_conc"])
def test_matrix_smaller_than_one_slice(csp, ctx, mode):
    # N = 50 < the 128 rows of one slice (rows past N padded), irregular rows;
    # one and several columns, one time step and several blocks
    col, val = ci.random_symmetric_ell(50, 120, seed=8)
    g = csp.Lattice.sparse(ctx, col, val)
    c = o.SparseLattice(col, val)
    for R, Nt, b in ((1, 1, 0), (2, 1, 0), (2, 9, 4), (3, 9, 0)):
        b = 0 if mode == "fp64_seq" else b
        psi = o.random_phase_states_fast(c.N, R, 40 + R)
        ref, _ = o.propagate(c, psi, Nt, b=0, Hn=g.halfwidth)
        got, _, _ = run(csp, ctx, g, psi, Nt, mode, b=b)
        assert np.max(np.abs(got - ref)) < (2e-5 if mode == "fp32_conc" else 1e-12), (R, Nt, b)


@pytest.mark.parametrize("mode", ["fp64_conc", "fp32_conc"])
def test_odd_column_counts(csp, ctx, mode):
    # column groups of an explicit matrix: 3 (waves of 2 + 1), 7 (waves of
    # 4 + 3), 10 and 17 (windowed tiles of 5 + 5 and 6 + 6 + 5) and 33
    # (groups of 32 and 1)
    g, c = pair(csp, ctx, "rand")
    for R, seed in ((3, 31), (7, 32), (10, 34), (17, 35), (33, 33)):
        print("[gpu] sparse %s R=%d" % (mode, R), flush=True)
        psi = o.random_phase_states_fast(c.N, R, seed)
        ref, _ = o.propagate(c, psi, 50, b=0, Hn=g.halfwidth)
        got, _, _ = run(csp, ctx, g, psi, 50, mode, b=16)
        assert np.max(np.abs(got - ref)) < (1e-10 if mode == "fp64_conc" else 2e-5)
        mref, _ = o.propagate_moments(c, psi, 50, b=8, halving=False, Hn=g.halfwidth)
        mgot, _, _ = run(csp, ctx, g, psi, 50, mode, b=8, assembly=csp.CSP_ASSEMBLE_MOMENTS)
        assert np.max(np.abs(mgot - mref)) < (1e-10 if mode == "fp64_conc" else 2e-5)
    # released workspace and orbital-major copies are rebuilt by the next call
    ctx.trim()
    again, _, _ = run(csp, ctx, g, psi, 50, mode, b=16)
    assert np.array_equal(again, got)


@pytest.mark.parametrize("name", ["lr4", "rand"])
@pytest.mark.parametrize("mode", ["fp64_conc", "fp32_conc"])
@pytest.mark.parametrize("b", [0, 16])
def test_moment_assembly_matches_oracle(csp, ctx, name, mode, b):
    print("[gpu] sparse moments %s %s b=%d" % (name, mode, b), flush=True)
    g, c = pair(csp, ctx, name)
    psi = np.concatenate([o.random_phase_states_fast(c.N, 3, 5),
                          o.site_states(c.N, o.ldos_sites(c.N, 2, 3))], axis=1)
    Nt = 150
    ref, cnt = o.propagate_moments(c, psi, Nt, b=(None if b == 0 else b), halving=b == 0,
                                   Hn=g.halfwidth)
    got, rep, _ = run(csp, ctx, g, psi, Nt, mode, b=b, assembly=csp.CSP_ASSEMBLE_MOMENTS)
    R = psi.shape[1]
    assert rep.amxsy * R == cnt["amxsy"] and rep.dot * R == cnt["dot"]
    if mode == "fp64_conc":
        assert np.max(np.abs(got - ref)) < 1e-10
    else:
        assert np.max(np.abs(got - ref)) < 2e-5
        assert rel_dos_err(got, ref, g.halfwidth) < 1e-4


def test_moments_final_state(csp, ctx):
    # one block with a final state: the carried sum over every order
    g, c = pair(csp, ctx, "rand")
    psi = o.random_phase_states_fast(c.N, 2, 4)
    ref, _, fin_ref = o.propagate(c, psi, 40, b=0, Hn=g.halfwidth, return_final=True)
    got, _, fin = run(csp, ctx, g, psi, 40, "fp64_conc", assembly=csp.CSP_ASSEMBLE_MOMENTS,
                      final=True)
    assert np.max(np.abs(got - ref)) < 1e-10
    assert np.max(np.abs(fin - fin_ref)) < 1e-10


@pytest.mark.parametrize("mode", ["fp64_conc", "fp32_conc"])
def test_quasi_eigenstates(csp, ctx, mode):
    g, c = pair(csp, ctx, "lr3")
    psi = o.random_phase_states_fast(c.N, 3, 13)      # waves of 2 + 1 columns
    E = [-3.0, -0.4, 0.0, 1.7]
    Nt = 60
    ref, _ = o.quasi_eigenstates(c, psi, Nt, E, Hn=g.halfwidth)
    dt = torch.complex128 if mode == "fp64_conc" else torch.complex64
    for b in (0, 8):                                  # energy-based, then state-based
        q, rep = csp.csp_quasi_eigenstates(ctx, g, dev(psi).to(dt),
                                           csp.make_params(Nt, mode=mode, block_b=b), E)
        err = np.max(np.abs(host(q) - ref)) / np.max(np.abs(ref))
        assert err < (1e-10 if mode == "fp64_conc" else 1e-4)


def test_stencil_matrix_as_ell_matches_stencil_path(csp, ctx):
    # the same honeycomb Hamiltonian through the stencil kernel and through
    # the explicit-matrix kernel (rows padded to the largest degree)
    spec = dict(kind="honeycomb", Lx=12, Ly=10, t=-2.7, W=1.0, disorder_seed=3,
                periodic_x=False)
    gs = csp.Lattice(ctx, **spec)
    c = o.Lattice("honeycomb", 12, 10, t=-2.7, W=1.0, disorder_seed=3, periodic_x=False)
    cnt = np.diff(c.rowptr)
    D = int(cnt.max())
    col = np.full((c.N, D), -1, np.int32)
    val = np.zeros((c.N, D))
    for s in range(c.N):
        k = c.rowptr[s + 1] - c.rowptr[s]
        col[s, :k] = c.col[c.rowptr[s]:c.rowptr[s + 1]]
        val[s, :k] = c.val[c.rowptr[s]:c.rowptr[s + 1]]
    ge = csp.Lattice.sparse(ctx, col, val)
    assert ge.halfwidth == pytest.approx(gs.halfwidth, rel=1e-14)
    psi = o.random_phase_states_fast(c.N, 3, 2)
    a, _, _ = run(csp, ctx, gs, psi, 80, "fp64_conc", b=16)
    b, _, _ = run(csp, ctx, ge, psi, 80, "fp64_conc", b=16)
    ref, _ = o.propagate(c, psi, 80, b=0)
    assert np.max(np.abs(a - b)) < 1e-11
    assert np.max(np.abs(b - ref)) < 1e-10


def test_batch_mixes_stencil_and_explicit(csp, ctx):
    gs = csp.Lattice(ctx, "square", 20, 18, t=1.0, W=1.5, disorder_seed=1)
    cs = o.Lattice("square", 20, 18, t=1.0, W=1.5, disorder_seed=1)
    ge, ce = pair(csp, ctx, "lr3")
    Nt = 64
    psis, refs = [], []
    for c, R, seed in ((cs, 3, 11), (ce, 2, 12)):
        psi = o.random_phase_states_fast(c.N, R, seed)
        psis.append(dev(psi).to(torch.complex64))
        refs.append(o.propagate(c, psi, Nt, b=0)[0])
    params = csp.make_params(Nt, mode="fp32_conc", block_b=16)
    corrs, rep = csp.csp_propagate_batch(ctx, [gs, ge], psis, params)
    for corr, ref in zip(corrs, refs):
        assert np.max(np.abs(host(corr) - ref)) < 2e-5


def test_batch_of_two_explicit_matrices(csp, ctx):
    # two complex64 explicit instances of different sizes and column counts
    # (each with its own orbital-major copies) beside a stencil lattice, in
    # several time blocks
    ga, ca = pair(csp, ctx, "rand")
    gb, cb = pair(csp, ctx, "lr4")
    gs = csp.Lattice(ctx, "square", 17, 15, t=1.0, W=1.0, disorder_seed=2)
    cs = o.Lattice("square", 17, 15, t=1.0, W=1.0, disorder_seed=2)
    Nt = 40
    psis, refs = [], []
    for c, R, seed, Hn in ((ca, 3, 21, ga.halfwidth), (cs, 2, 22, gs.halfwidth),
                           (cb, 6, 23, gb.halfwidth)):
        psi = o.random_phase_states_fast(c.N, R, seed)
        psis.append(dev(psi).to(torch.complex64))
        refs.append(o.propagate(c, psi, Nt, b=0, Hn=Hn)[0])
    for b in (8, 0):
        params = csp.make_params(Nt, mode="fp32_conc", block_b=b)
        corrs, _ = csp.csp_propagate_batch(ctx, [ga, gs, gb], psis, params)
        for corr, ref in zip(corrs, refs):
            assert np.max(np.abs(host(corr) - ref)) < 2e-5


def test_autotune_explicit_matrix(csp, ctx):
    g, c = pair(csp, ctx, "lr4")
    params = csp.make_params(256, mode="fp32_conc")
    t = csp.csp_autotune(ctx, [g], [4], params)
    assert t.spmm_steps == 1 and t.block_b >= 1
    psi = o.random_phase_states_fast(c.N, 4, 1)
    ref, _ = o.propagate(c, psi, 256, b=0, Hn=g.halfwidth)
    got, rep, _ = run(csp, ctx, g, psi, 256, "fp32_conc")
    assert rep.block_b == t.block_b
    assert np.max(np.abs(got - ref)) < 2e-5
