"""GPU parity: every HIP entry point against the FP64 CPU oracle.

Bit-exact: on-site energies, neighbour tables, localized sites, the
spectral half-width.  FP64 paths: 1e-10 on correlations (1e-13 for single
steps and coefficients).  FP32 concurrent path: correlations within 2e-5
absolute and DOS within 1e-4 relative (max |D32 - D64| / max |D64|).
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
    print("[gpu] creating context", flush=True)
    c = csp.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


LATS = [
    dict(kind="square", Lx=37, Ly=23, t=1.0, W=1.3, disorder_seed=5),
    dict(kind="square", Lx=17, Ly=9, t=-0.7, W=0.0, periodic_x=False, periodic_y=True),
    dict(kind="honeycomb", Lx=16, Ly=9, t=-2.7, W=1.0, disorder_seed=2),
    dict(kind="honeycomb", Lx=5, Ly=4, t=-2.7, W=0.5, disorder_seed=3, periodic_x=False,
         periodic_y=False),
    dict(kind="chain", Lx=301, t=1.0, W=2.0, disorder_seed=9),
    dict(kind="chain", Lx=50, t=0.5, W=0.0, periodic_x=False),
]


def pair(csp, ctx, spec):
    g = csp.Lattice(ctx, **spec)
    spec2 = dict(spec)
    kind = spec2.pop("kind")
    Lx = spec2.pop("Lx")
    Ly = spec2.pop("Ly", 1)
    return g, o.Lattice(kind, Lx, Ly, **spec2)


@pytest.mark.parametrize("spec", LATS)
def test_lattice_onsite_and_bound_bit_exact(csp, ctx, spec):
    print("[gpu] lattice", spec, flush=True)
    g, c = pair(csp, ctx, spec)
    assert g.N == c.N
    assert np.array_equal(host(g.onsite()), c.eps)
    assert g.halfwidth == c.halfwidth()


@pytest.mark.parametrize("spec", LATS)
def test_neighbour_table_matches_bonds(csp, ctx, spec):
    g, c = pair(csp, ctx, spec)
    nb = host(g.neighbors())
    for s in range(c.N):
        cols = c.col[c.rowptr[s] + 1:c.rowptr[s + 1]]          # off-diagonal entries
        mine = nb[s][nb[s] >= 0]
        assert sorted(mine.tolist()) == sorted(cols.tolist()), s


def test_random_phase_states(csp, ctx):
    N, R, ld, col0, seed = 1000, 3, 5, 1, 77
    ref = o.random_phase_states_fast(N, R, seed)
    p64 = torch.zeros((N, ld), dtype=torch.complex128, device="cuda:0")
    csp.csp_states_random_phase(ctx, p64, R, seed, col0=col0)
    got = host(p64)
    assert np.max(np.abs(got[:, col0:col0 + R] - ref)) < 1e-15
    assert np.all(got[:, :col0] == 0) and np.all(got[:, col0 + R:] == 0)
    p32 = torch.zeros((N, ld), dtype=torch.complex64, device="cuda:0")
    csp.csp_states_random_phase(ctx, p32, R, seed, col0=col0)
    assert np.max(np.abs(host(p32)[:, col0:col0 + R] - ref)) < 1e-7


def test_ldos_sites_and_site_states(csp, ctx):
    sites = host(csp.csp_ldos_sites(ctx, 5000, 64, 3))
    assert np.array_equal(sites, o.ldos_sites(5000, 64, 3))
    psi = torch.full((5000, 66), 7.0, dtype=torch.complex64, device="cuda:0")
    csp.csp_states_sites(ctx, psi, dev(sites), col0=2)
    got = host(psi)
    assert np.array_equal(got[:, 2:], o.site_states(5000, sites).astype(np.complex64))
    assert np.all(got[:, :2] == 7.0)


@pytest.mark.parametrize("x", [math.pi, 10 * math.pi, 32 * math.pi, 64 * math.pi])
def test_chebyshev_coefficients(csp, ctx, x):
    n_ref = o.truncation(x)
    c, n = csp.csp_chebyshev_coefficients(ctx, x, n_ref + 5)
    assert n == n_ref
    assert np.max(np.abs(host(c) - o.cheb_coeffs(x, n_ref + 5))) < 1e-13


STEP_LATS = LATS + [
    dict(kind="square", Lx=40, Ly=100, t=1.0, W=0.8, disorder_seed=4),   # several row segments
    dict(kind="square", Lx=600, Ly=5, t=1.0, W=0.0),                     # several strips
    dict(kind="honeycomb", Lx=300, Ly=40, t=-2.7, W=1.0, disorder_seed=6),
    dict(kind="square", Lx=1, Ly=7, t=1.0, W=0.0),                       # self-bonds
    dict(kind="honeycomb", Lx=2, Ly=2, t=1.0, W=0.2, disorder_seed=1),   # repeated bonds
]


@pytest.mark.parametrize("spec", STEP_LATS)
@pytest.mark.parametrize("R", [1, 3, 4])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_chebyshev_step(csp, ctx, spec, R, dtype):
    g, c = pair(csp, ctx, spec)
    Hn = g.halfwidth
    rng = np.random.default_rng(R)
    x = rng.normal(size=(c.N, R)) + 1j * rng.normal(size=(c.N, R))
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    xd = dev(x).to(tdt)
    y1 = torch.zeros_like(xd)
    csp.csp_chebyshev_step(ctx, g, xd, y1, first=True)
    y2 = xd.clone()
    csp.csp_chebyshev_step(ctx, g, y1, y2, first=False)
    ref = np.stack([o.chebyshev_vectors(c, x[:, r], 2, Hn) for r in range(R)], axis=-1)
    tol = 1e-13 if dtype == "c128" else 2e-6
    scale = np.max(np.abs(x))
    assert np.max(np.abs(host(y1) - ref[1])) < tol * scale
    assert np.max(np.abs(host(y2) - ref[2])) < tol * 3 * scale


def test_chebyshev_step_spectral_centre(csp, ctx):
    spec = dict(kind="honeycomb", Lx=7, Ly=6, t=-1.0, W=1.0, disorder_seed=8)
    g = csp.Lattice(ctx, halfwidth_override=4.5, center=0.3, **spec)
    c = o.Lattice("honeycomb", 7, 6, t=-1.0, W=1.0, disorder_seed=8)
    x = np.random.default_rng(0).normal(size=(c.N, 2)).astype(np.complex128)
    xd = dev(x)
    y = torch.zeros_like(xd)
    csp.csp_chebyshev_step(ctx, g, xd, y, first=True)
    ref = np.stack([o.chebyshev_vectors(c, x[:, r], 1, 4.5, H0=0.3)[1] for r in range(2)], -1)
    assert np.max(np.abs(host(y) - ref)) < 1e-13


def run_gpu(csp, ctx, g, psi, Nt, mode, b=0, K=0, final=False):
    tdt = torch.complex128 if mode != "fp32_conc" else torch.complex64
    p = dev(psi).to(tdt)
    params = csp.make_params(Nt, mode=mode, block_b=b, chunk_K=K)
    fin = torch.zeros_like(p) if final else None
    corr, rep = csp.csp_propagate(ctx, g, p, params, final=fin)
    return host(corr), rep, (host(fin) if final else None)


def test_fp64_sequential_config1(csp, ctx):
    # 64 x 64 square, t = 1, |H| = 4.1, one random state (seed 1), 1024 steps
    print("[gpu] config-1 fp64 sequential", flush=True)
    g = csp.Lattice(ctx, "square", 64, 64, t=1.0)
    assert g.halfwidth == pytest.approx(4.1, abs=1e-15)
    c = o.Lattice("square", 64, 64, t=1.0)
    psi = o.random_phase_states_fast(c.N, 1, 1)
    ref, _ = o.propagate(c, psi, 1024, b=0, Hn=4.1)
    got, rep, _ = run_gpu(csp, ctx, g, psi, 1024, "fp64_seq")
    assert np.max(np.abs(got - ref)) < 1e-10
    assert rep.amxsy == 1024 * 20 and rep.dot == 1024


@pytest.mark.parametrize("b", [1, 4, 13, 16])
def test_fp64_concurrent(csp, ctx, b):
    spec = dict(kind="honeycomb", Lx=20, Ly=12, t=-2.7, W=1.0, disorder_seed=4)
    g, c = pair(csp, ctx, spec)
    psi = o.random_phase_states_fast(c.N, 3, 5)
    Nt = 100
    ref, cnt = o.propagate(c, psi, Nt, b=b)
    got, rep, _ = run_gpu(csp, ctx, g, psi, Nt, "fp64_conc", b=b)
    assert np.max(np.abs(got - ref)) < 1e-10
    assert rep.amxsy * 3 == cnt["amxsy"] and rep.axpy * 3 == cnt["axpy"]


@pytest.mark.parametrize("mode", ["fp64_seq", "fp64_conc", "fp32_conc"])
def test_smallest_lattices(csp, ctx, mode):
    # side 3 (the smallest without doubled bonds), periodic and open, one time
    # step and several blocks; a strip of 64 V values covers the whole row
    print("[gpu] smallest lattices %s" % mode, flush=True)
    for spec in (dict(kind="chain", Lx=3, t=1.0, W=0.5, disorder_seed=1),
                 dict(kind="square", Lx=3, Ly=3, t=-1.0, W=1.0, disorder_seed=2),
                 dict(kind="honeycomb", Lx=3, Ly=3, t=-2.7, W=0.3, disorder_seed=3),
                 dict(kind="square", Lx=3, Ly=4, t=1.0, periodic_x=False, periodic_y=False)):
        g, c = pair(csp, ctx, spec)
        for Nt, b in ((1, 0), (9, 4)):
            b = 0 if mode == "fp64_seq" else b
            psi = o.random_phase_states_fast(c.N, 2, 6)
            ref, _ = o.propagate(c, psi, Nt, b=0)
            got, _, _ = run_gpu(csp, ctx, g, psi, Nt, mode, b=b)
            assert np.max(np.abs(got - ref)) < (2e-5 if mode == "fp32_conc" else 1e-12), spec


def rel_dos_err(c32, c64, Hn):
    _, D32, _ = o.dos(c32, Hn)
    _, D64, _ = o.dos(c64, Hn)
    return np.max(np.abs(D32.mean(1) - D64.mean(1))) / np.max(np.abs(D64.mean(1)))


@pytest.mark.parametrize("b,K", [(1, 0), (7, 0), (32, 0), (64, 0), (32, 16), (40, 32)])
def test_fp32_concurrent(csp, ctx, b, K):
    print("[gpu] fp32 concurrent b=%d K=%d" % (b, K), flush=True)
    spec = dict(kind="honeycomb", Lx=24, Ly=24, t=-2.7, W=1.0, disorder_seed=4)
    g, c = pair(csp, ctx, spec)
    psi = o.random_phase_states_fast(c.N, 5, 5)       # groups of 4 + 1 columns
    Nt = 200
    ref, _ = o.propagate(c, psi, Nt, b=0)
    got, rep, _ = run_gpu(csp, ctx, g, psi, Nt, "fp32_conc", b=b, K=K)
    assert rep.block_b == b
    assert np.max(np.abs(got - ref)) < 2e-5
    assert rel_dos_err(got, ref, g.halfwidth) < 1e-4


def test_fp32_concurrent_ldos_columns(csp, ctx):
    # random columns and localized columns in one block, as the LDOS workload
    g, c = pair(csp, ctx, dict(kind="honeycomb", Lx=32, Ly=32, t=-2.7, W=0.0))
    sites = o.ldos_sites(c.N, 6, 3)
    psi = np.concatenate([o.random_phase_states_fast(c.N, 4, 2), o.site_states(c.N, sites)], 1)
    Nt = 96
    ref, _ = o.propagate(c, psi, Nt, b=0)
    got, rep, _ = run_gpu(csp, ctx, g, psi, Nt, "fp32_conc", b=32)
    assert rep.n_groups == 2                     # 8 + 2 columns
    assert np.max(np.abs(got - ref)) < 2e-5
    assert rel_dos_err(got[:, 4:], ref[:, 4:], g.halfwidth) < 1e-4


def test_final_state_and_norm(csp, ctx):
    g, c = pair(csp, ctx, dict(kind="square", Lx=30, Ly=20, t=1.0, W=1.0, disorder_seed=1))
    psi = o.random_phase_states_fast(c.N, 2, 4)
    ref, _, fin_ref = o.propagate(c, psi, 50, b=0, return_final=True)
    got, _, fin = run_gpu(csp, ctx, g, psi, 50, "fp64_seq", final=True)
    assert np.max(np.abs(fin - fin_ref)) < 1e-10
    _, _, fin32 = run_gpu(csp, ctx, g, psi, 50, "fp32_conc", b=16, final=True)
    assert np.max(np.abs(np.linalg.norm(fin32, axis=0) - 1.0)) < 1e-5


def test_dos_kernel(csp, ctx):
    g, c = pair(csp, ctx, dict(kind="square", Lx=12, Ly=11, t=1.0, W=1.0, disorder_seed=2))
    psi = o.random_phase_states_fast(c.N, 3, 1)
    ref, _ = o.propagate(c, psi, 128, b=8)
    for window, wcode in (("hann", csp.CSP_WINDOW_HANN), ("none", csp.CSP_WINDOW_NONE)):
        E, D, Dm = csp.csp_dos(ctx, dev(ref), g.halfwidth, window=wcode)
        Er, Dr, _ = o.dos(ref, g.halfwidth, window=window)
        assert np.max(np.abs(host(E) - Er)) < 1e-12
        assert np.max(np.abs(host(D) - Dr)) < 1e-12
        assert np.max(np.abs(host(Dm) - Dr.mean(1))) < 1e-12


def test_dos_with_spectral_centre(csp, ctx):
    # a lattice with H0 != 0: the propagation carries exp(-i (H - H0) t) on
    # both sides, and csp_dos places the density on center + E_k
    spec = dict(kind="honeycomb", Lx=9, Ly=8, t=-1.0, W=1.2, disorder_seed=3)
    g = csp.Lattice(ctx, halfwidth_override=4.2, center=0.35, **spec)
    c = o.Lattice("honeycomb", 9, 8, t=-1.0, W=1.2, disorder_seed=3)
    assert g.info.H0 == 0.35 and g.halfwidth == 4.2
    psi = o.random_phase_states_fast(c.N, 2, 7)
    Nt = 96
    ref, _ = o.propagate(c, psi, Nt, b=0, Hn=4.2, H0=0.35)
    corr, _ = csp.csp_propagate(ctx, g, dev(psi), csp.make_params(Nt, mode="fp64_conc",
                                                                  block_b=16))
    assert np.max(np.abs(host(corr) - ref)) < 1e-10
    E, D, Dm = csp.csp_dos(ctx, corr, g.halfwidth, center=g.info.H0)
    Er, Dr, _ = o.dos(ref, 4.2, H0=0.35)
    assert np.max(np.abs(host(E) - Er)) < 1e-12
    assert host(E)[Nt] == 0.35
    assert np.max(np.abs(host(D) - Dr)) < 1e-10
    assert np.max(np.abs(host(Dm) - Dr.mean(1))) < 1e-10


def test_batch_matches_oracle(csp, ctx):
    specs = [dict(kind="square", Lx=20, Ly=18, t=1.0, W=1.5, disorder_seed=1),
             dict(kind="honeycomb", Lx=9, Ly=14, t=-2.7, W=0.5, disorder_seed=2),
             dict(kind="chain", Lx=400, t=1.0, W=0.0)]
    Rs = [1, 3, 2]
    Nt = 64
    gl, psis, refs = [], [], []
    for spec, R in zip(specs, Rs):
        g, c = pair(csp, ctx, spec)
        psi = o.random_phase_states_fast(c.N, R, 11)
        gl.append(g)
        psis.append(dev(psi).to(torch.complex64))
        refs.append(o.propagate(c, psi, Nt, b=0)[0])
    params = csp.make_params(Nt, mode="fp32_conc", block_b=16)
    corrs, rep = csp.csp_propagate_batch(ctx, gl, psis, params)
    for corr, ref in zip(corrs, refs):
        assert np.max(np.abs(host(corr) - ref)) < 2e-5


def test_error_paths(csp, ctx):
    g = csp.Lattice(ctx, "square", 8, 8)
    psi = torch.zeros((64, 1), dtype=torch.complex64, device="cuda:0")
    with pytest.raises(csp.CspError) as e:
        csp.csp_propagate(ctx, g, psi, csp.make_params(10, mode="fp32_conc", block_b=65))
    assert e.value.status == csp.CSP_EUNSUPPORTED
    with pytest.raises(csp.CspError) as e:
        csp.csp_propagate(ctx, g, psi, csp.make_params(10, mode=7))
    assert e.value.status == csp.CSP_EINVAL
    with pytest.raises(csp.CspError) as e:
        csp.csp_propagate(ctx, g, psi, csp.make_params(10, mode="fp32_conc", block_b=8,
                                                       mem_cap_bytes=1 << 20))
    assert e.value.status == csp.CSP_ENOMEM
    with pytest.raises(csp.CspError):
        csp.Lattice(ctx, "square", 0, 8)
    # Nt = 0: only the t = 0 correlation
    psi[0, 0] = 1.0
    corr, _ = csp.csp_propagate(ctx, g, psi, csp.make_params(0, mode="fp32_conc", block_b=4))
    assert host(corr).shape == (1, 1) and host(corr)[0, 0] == 1.0


# ---------------------------------------------------------------- moment form
def run_gpu_moments(csp, ctx, g, psi, Nt, mode, b=0, final=False):
    tdt = torch.complex128 if mode != "fp32_conc" else torch.complex64
    p = dev(psi).to(tdt)
    params = csp.make_params(Nt, mode=mode, block_b=b, assembly=csp.CSP_ASSEMBLE_MOMENTS)
    fin = torch.zeros_like(p) if final else None
    corr, rep = csp.csp_propagate(ctx, g, p, params, final=fin)
    return host(corr), rep, (host(fin) if final else None)


@pytest.mark.parametrize("mode", ["fp64_conc", "fp32_conc"])
@pytest.mark.parametrize("b", [0, 16, 7, 200])
def test_moments_match_oracle(csp, ctx, mode, b):
    print("[gpu] moments %s b=%d" % (mode, b), flush=True)
    spec = dict(kind="honeycomb", Lx=24, Ly=20, t=-2.7, W=1.0, disorder_seed=4)
    g, c = pair(csp, ctx, spec)
    psi = np.concatenate([o.random_phase_states_fast(c.N, 3, 5),
                          o.site_states(c.N, o.ldos_sites(c.N, 2, 3))], axis=1)   # groups 4 + 1
    Nt = 200
    ref, cnt = o.propagate_moments(c, psi, Nt, b=(None if b in (0, 200) else b),
                                   halving=b in (0, 200))
    seq, _ = o.propagate(c, psi, Nt, b=0)
    assert np.max(np.abs(ref - seq)) < 1e-12
    got, rep, _ = run_gpu_moments(csp, ctx, g, psi, Nt, mode, b=b)
    R = psi.shape[1]
    assert rep.amxsy * R == cnt["amxsy"] and rep.dot * R == cnt["dot"]
    if mode == "fp64_conc":
        assert np.max(np.abs(got - ref)) < 1e-10
    else:
        assert np.max(np.abs(got - ref)) < 2e-5
        assert rel_dos_err(got, ref, g.halfwidth) < 1e-4


def test_moments_sequential_mode_and_final_state(csp, ctx):
    g, c = pair(csp, ctx, dict(kind="square", Lx=30, Ly=20, t=1.0, W=1.0, disorder_seed=1))
    psi = o.random_phase_states_fast(c.N, 2, 4)
    ref, _, fin_ref = o.propagate(c, psi, 50, b=0, return_final=True)
    got, rep, fin = run_gpu_moments(csp, ctx, g, psi, 50, "fp64_seq", final=True)
    assert rep.block_b == 1 and rep.amxsy == 50 * 20
    assert np.max(np.abs(got - ref)) < 1e-10
    assert np.max(np.abs(fin - fin_ref)) < 1e-10
    # one block with a final state: no halving, carry over all orders
    got, rep, fin = run_gpu_moments(csp, ctx, g, psi, 50, "fp64_conc", final=True)
    assert rep.amxsy == o.truncation(50 * math.pi)
    assert np.max(np.abs(got - ref)) < 1e-10
    assert np.max(np.abs(fin - fin_ref)) < 1e-10


@pytest.mark.parametrize("mode,tol", [("fp64_conc", 1e-12), ("fp32_conc", 2e-5)])
def test_state_and_moment_assembly_agree(csp, ctx, mode, tol):
    # the reduction <psi0|.> commutes with the block contraction: assembling
    # the states on MFMA and contracting the block moments give the same
    # correlations up to rounding
    g, c = pair(csp, ctx, dict(kind="square", Lx=41, Ly=33, t=1.0, W=0.5, disorder_seed=7))
    psi = o.random_phase_states_fast(c.N, 4, 9)
    Nt = 160
    b = 16
    s_corr, _, _ = run_gpu(csp, ctx, g, psi, Nt, mode, b=b)
    m_corr, _, _ = run_gpu_moments(csp, ctx, g, psi, Nt, mode, b=b)
    assert np.max(np.abs(s_corr - m_corr)) < tol


# ---------------------------------------------------------------- norm guard
@pytest.mark.parametrize("mode,assembly,b", [("fp32_conc", 0, 16), ("fp32_conc", 1, 16),
                                             ("fp32_conc", 1, 0), ("fp64_seq", 0, 1)])
def test_norm_guard(csp, ctx, mode, assembly, b):
    g, c = pair(csp, ctx, dict(kind="honeycomb", Lx=16, Ly=12, t=-2.7, W=1.0, disorder_seed=2))
    psi = o.random_phase_states_fast(c.N, 3, 1)
    tdt = torch.complex128 if mode != "fp32_conc" else torch.complex64
    Nt = 64
    ok = csp.make_params(Nt, mode=mode, block_b=b, assembly=assembly, check_norm=True)
    corr, _ = csp.csp_propagate(ctx, g, dev(psi).to(tdt), ok)
    ref, _ = o.propagate(c, psi, Nt, b=0)
    assert np.max(np.abs(host(corr) - ref)) < 2e-5
    # a non-finite input value is caught after the first block
    bad = psi.copy()
    bad[7, 1] = np.nan
    with pytest.raises(csp.CspError) as e:
        csp.csp_propagate(ctx, g, dev(bad).to(tdt), ok)
    assert e.value.status == csp.CSP_ENUMERIC and "block 0" in str(e.value)
    # a tolerance below the rounding of the path trips the guard too (forced
    # from the host; the kernels run normally)
    if mode == "fp32_conc" and b > 0:
        tight = csp.make_params(Nt, mode=mode, block_b=b, assembly=assembly, check_norm=True,
                                norm_tol=1e-14)
        with pytest.raises(csp.CspError) as e:
            csp.csp_propagate(ctx, g, dev(psi).to(tdt), tight)
        assert e.value.status == csp.CSP_ENUMERIC


# ---------------------------------------------------------------- autotuner
def test_autotune_and_block_selection(csp, ctx):
    print("[gpu] autotune", flush=True)
    spec = dict(kind="honeycomb", Lx=96, Ly=64, t=-2.7, W=1.0, disorder_seed=4)
    g, c = pair(csp, ctx, spec)
    R, Nt = 5, 256
    params = csp.make_params(Nt, mode="fp32_conc", block_b=0)
    T = csp.csp_autotune(ctx, [g], [R], params)
    assert T.n_candidates >= 10 and T.spmm_vec in (1, 2, 4) and T.spmm_seg_rows >= 2
    assert T.contract_wg_per_cu in (2, 4, 8) and T.t_amxsy_us > 0 and T.t_order_us[0] > 0
    assert 1 <= T.block_b <= 64
    costs = list(T.model_cost_ms)
    assert costs[0] > 0 and all(x > 0 for x in costs[:7])      # b = 1..64 allowed
    assert costs[7] == -1.0                                     # b = 128 above the MFMA limit
    b_sel, rep_sel = csp.csp_select_block(ctx, g, R, params)
    assert b_sel == T.block_b
    # a propagation of the same shape uses the tuned launch shapes and b
    psi = o.random_phase_states_fast(c.N, R, 3)
    got, rep, _ = run_gpu(csp, ctx, g, psi, Nt, "fp32_conc", b=0)
    assert rep.block_b == T.block_b
    ref, _ = o.propagate(c, psi, Nt, b=0)
    assert np.max(np.abs(got - ref)) < 2e-5
    # moment assembly: recursion shapes only, one block
    pm = csp.make_params(Nt, mode="fp32_conc", assembly=csp.CSP_ASSEMBLE_MOMENTS)
    Tm = csp.csp_autotune(ctx, [g], [R], pm)
    assert Tm.block_b == 0 and Tm.t_amxsy_us > 0
    gotm, _, _ = run_gpu_moments(csp, ctx, g, psi, Nt, "fp32_conc")
    assert np.max(np.abs(gotm - ref)) < 2e-5


def test_autotune_fp64_and_memory_cap(csp, ctx):
    g, c = pair(csp, ctx, dict(kind="square", Lx=80, Ly=70, t=1.0, W=0.5, disorder_seed=2))
    T = csp.csp_autotune(ctx, [g], [3], csp.make_params(64, mode="fp64_conc"))
    assert 1 <= T.block_b <= 16 and T.t_order_us[1] == -1.0
    psi = o.random_phase_states_fast(c.N, 3, 8)
    got, rep, _ = run_gpu(csp, ctx, g, psi, 64, "fp64_conc", b=0)
    assert rep.block_b == T.block_b
    ref, _ = o.propagate(c, psi, 64, b=0)
    assert np.max(np.abs(got - ref)) < 1e-10
    with pytest.raises(csp.CspError) as e:
        csp.csp_autotune(ctx, [g], [3], csp.make_params(64, mode="fp64_conc", mem_cap_bytes=4096))
    assert e.value.status == csp.CSP_ENOMEM


# ---------------------------------------------------------------- HIP graphs
def _batch_inputs(csp, ctx, Nt):
    specs = [dict(kind="square", Lx=33, Ly=21, t=1.0, W=1.5, disorder_seed=1),
             dict(kind="honeycomb", Lx=17, Ly=14, t=-2.7, W=0.5, disorder_seed=2),
             dict(kind="chain", Lx=900, t=1.0, W=0.3, disorder_seed=3)]
    Rs = [1, 6, 3]
    gl, psis, refs = [], [], []
    for spec, R in zip(specs, Rs):
        g, c = pair(csp, ctx, spec)
        psi = o.random_phase_states_fast(c.N, R, 13)
        gl.append(g)
        psis.append(dev(psi).to(torch.complex64))
        refs.append(o.propagate(c, psi, Nt, b=0)[0])
    return gl, psis, refs


def test_graph_replay_equals_direct_launches(csp, ctx):
    print("[gpu] graph replay", flush=True)
    Nt, b = 100, 16                                     # 6 full blocks + 1 of 4 steps
    gl, psis, refs = _batch_inputs(csp, ctx, Nt)
    direct, rep_d = csp.csp_propagate_batch(ctx, gl, psis, csp.make_params(Nt, block_b=b, graph=-1))
    assert rep_d.graph_blocks == 0
    direct = [host(x) for x in direct]
    for ref, d in zip(refs, direct):
        assert np.max(np.abs(d - ref)) < 2e-5
    # several graph-mode calls with eager work in between: every replay is
    # bit-identical to the direct launches
    for rep_i in range(3):
        got, rep_g = csp.csp_propagate_batch(ctx, gl, psis, csp.make_params(Nt, block_b=b))
        assert rep_g.graph_blocks == 6
        for d, x in zip(direct, got):
            assert np.array_equal(host(x), d)
        _ = (psis[0] * 2).sum().item()
    # single-lattice call with the graph switched on
    single, rep_s = csp.csp_propagate(ctx, gl[1], psis[1], csp.make_params(Nt, block_b=b, graph=1))
    assert rep_s.graph_blocks == 6 and np.array_equal(host(single), direct[1])


def test_graph_capture_failure_falls_back(csp, ctx, monkeypatch):
    Nt, b = 64, 16
    gl, psis, refs = _batch_inputs(csp, ctx, Nt)
    monkeypatch.setenv("CSP_FORCE_GRAPH_FAILURE", "1")
    got, rep = csp.csp_propagate_batch(ctx, gl, psis, csp.make_params(Nt, block_b=b, graph=1))
    assert rep.graph_blocks == 0
    for ref, x in zip(refs, got):
        assert np.max(np.abs(host(x) - ref)) < 2e-5


def test_graph_replay_with_norm_guard(csp, ctx):
    Nt, b = 64, 8
    gl, psis, refs = _batch_inputs(csp, ctx, Nt)
    params = csp.make_params(Nt, block_b=b, graph=1, check_norm=True)
    got, rep = csp.csp_propagate_batch(ctx, gl, psis, params)
    assert rep.graph_blocks == 8
    bad = [p.clone() for p in psis]
    bad[2][5, 1] = float("nan")
    with pytest.raises(csp.CspError) as e:
        csp.csp_propagate_batch(ctx, gl, bad, params)
    assert e.value.status == csp.CSP_ENUMERIC and "block 0" in str(e.value)


# ---------------------------------------------------------------- memory cap
@pytest.mark.parametrize("assembly", [0, 1])
def test_column_windows_under_memory_cap(csp, ctx, assembly):
    # all 8 columns at once exceed the cap: the library runs windows of
    # fewer columns one after another, with the same results
    print("[gpu] column windows assembly=%d" % assembly, flush=True)
    g, c = pair(csp, ctx, dict(kind="honeycomb", Lx=128, Ly=128, t=-2.7, W=1.0, disorder_seed=3))
    R, Nt = 8, 48
    psi = o.random_phase_states_fast(c.N, R, 21)
    ref, _ = o.propagate(c, psi, Nt, b=0)
    cap = 96 * 2**20 + 18 * c.N * 4 * 8 + 2**20     # room for 4 columns, not 8
    if assembly == 1:
        cap = 96 * 2**20 + 6 * c.N * 4 * 8 + 2**20
    params = csp.make_params(Nt, mode="fp32_conc", block_b=16, assembly=assembly,
                             mem_cap_bytes=cap)
    corr, rep = csp.csp_propagate(ctx, g, dev(psi).to(torch.complex64), params)
    assert rep.n_passes == 2
    assert np.max(np.abs(host(corr) - ref)) < 2e-5
    full, rep1 = csp.csp_propagate(ctx, g, dev(psi).to(torch.complex64),
                                   csp.make_params(Nt, mode="fp32_conc", block_b=16,
                                                   assembly=assembly))
    assert rep1.n_passes == 1
    assert np.max(np.abs(host(full) - host(corr))) < 1e-6


def test_bandwidth_probe(csp, ctx):
    r, w, rw = csp.csp_bandwidth_probe(ctx, 256 << 20)
    print("[gpu] streaming GB/s read %.0f write %.0f 2r1w %.0f" % (r, w, rw), flush=True)
    for x in (r, w, rw):
        assert 500.0 < x < 8000.0 * 1.05      # below the published HBM peak
    with pytest.raises(csp.CspError):
        csp.csp_bandwidth_probe(ctx, 1000)


# ---------------------------------------------------------------- launch shapes
SHAPE_LATS = [
    dict(kind="honeycomb", Lx=80, Ly=20, t=-2.7, W=1.0, disorder_seed=6),
    dict(kind="honeycomb", Lx=70, Ly=11, t=-2.7, W=0.0, periodic_x=False, periodic_y=False),
    dict(kind="square", Lx=150, Ly=13, t=1.0, W=0.7, disorder_seed=2, periodic_x=False),
    dict(kind="square", Lx=45, Ly=17, t=-1.0, W=0.0, periodic_y=False),
    dict(kind="chain", Lx=301, t=1.0, W=1.0, disorder_seed=3),
]
SHAPES = {("fp32_conc", 0): [(v, k) for v in (2, 4) for k in (1, 2, 4, 8)],
          ("fp32_conc", 1): [(v, k) for v in (2, 4) for k in (1, 2, 4)] + [(2, 8)],
          ("fp64_conc", 0): [(2, 1), (2, 2), (2, 4)],
          ("fp64_conc", 1): [(2, 1), (2, 2), (2, 4)]}


@pytest.mark.parametrize("spec", SHAPE_LATS)
def test_every_recursion_shape_matches_oracle(csp, ctx, spec):
    # every compiled recursion kernel (values per lane, steps per launch),
    # with short row segments so strips, segments and their ragged ends all
    # occur, in both assemblies and both precisions
    print("[gpu] launch shapes %s %dx%d" % (spec["kind"], spec["Lx"], spec.get("Ly", 1)),
          flush=True)
    g, c = pair(csp, ctx, spec)
    psi = o.random_phase_states_fast(c.N, 3, 21)
    Nt = 40
    ref, _ = o.propagate(c, psi, Nt, b=0)
    for (mode, assembly), shapes in SHAPES.items():
        tdt = torch.complex128 if mode == "fp64_conc" else torch.complex64
        tol = 1e-10 if mode == "fp64_conc" else 2e-5
        for b in ((8,) if assembly == 0 else (0, 8)):
            params = csp.make_params(Nt, mode=mode, block_b=b, assembly=assembly)
            for (v, k) in shapes:
                T = csp.Tuning()
                T.spmm_vec, T.spmm_steps, T.spmm_seg_rows = v, k, 8
                T.contract_wg_per_cu, T.block_b = 4, 8
                csp.csp_set_tuning(ctx, [g], [psi.shape[1]], params, T)
                corr, rep = csp.csp_propagate(ctx, g, dev(psi).to(tdt), params)
                got = host(corr)
                assert rep.spmm_steps == k, (mode, assembly, b, v, k)
                err = np.max(np.abs(got - ref))
                assert err < tol, (mode, assembly, b, v, k, err)


def test_set_tuning_rejects_missing_shapes(csp, ctx):
    g = csp.Lattice(ctx, "square", 16, 16)
    T = csp.Tuning()
    T.spmm_vec, T.spmm_steps, T.spmm_seg_rows, T.contract_wg_per_cu = 3, 4, 8, 4
    params = csp.make_params(10, mode="fp32_conc", block_b=4)
    with pytest.raises(csp.CspError) as e:
        csp.csp_set_tuning(ctx, [g], [1], params, T)
    assert e.value.status == csp.CSP_EINVAL
    T.spmm_vec, T.spmm_steps = 4, 8
    pm = csp.make_params(10, mode="fp32_conc", assembly=csp.CSP_ASSEMBLE_MOMENTS)
    with pytest.raises(csp.CspError) as e:          # no moment kernel with 4 values x 8 steps
        csp.csp_set_tuning(ctx, [g], [1], pm, T)
    assert e.value.status == csp.CSP_EINVAL
    T.spmm_vec = 2
    csp.csp_set_tuning(ctx, [g], [1], pm, T)
    csp.csp_set_tuning(ctx, [g], [1], params, T)
