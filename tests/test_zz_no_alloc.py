"""The allocation-free DOS entry point, csp_dos_noalloc, through the C ABI:
its results equal those of csp_dos (the same kernels, with the twiddle
table in the library's static device scratch instead of a per-call
allocation) and the oracle's transform, on two calls in a row, the second
with a smaller input (the scratch keeps the first call's table, which the
second call overwrites before reading); and an Nt above the scratch's limit
is rejected before any work is enqueued."""
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


def _case(csp, ctx, Nt, R, seed, center):
    """Correlations of the oracle (complex128) on a small disordered
    lattice, and both transforms of them on the GPU."""
    lat = o.Lattice("square", 11, 9, t=1.0, W=1.0, disorder_seed=seed)
    Hn = lat.halfwidth() + abs(center)
    psi = o.random_phase_states_fast(lat.N, R, seed + 1)
    corr, _ = o.propagate(lat, psi, Nt, b=0, Hn=Hn, H0=center)
    dcorr = torch.from_numpy(corr).to("cuda:0")
    E, D, Dm = csp.csp_dos(ctx, dcorr, Hn, center=center)
    En = torch.full((2 * Nt,), np.nan, dtype=torch.float64, device="cuda:0")
    Dn = torch.full((2 * Nt, R), np.nan, dtype=torch.float64, device="cuda:0")
    Dmn = torch.full((2 * Nt,), np.nan, dtype=torch.float64, device="cuda:0")
    print("[no-alloc] csp_dos_noalloc Nt=%d R=%d center=%g" % (Nt, R, center), flush=True)
    csp.csp_dos_noalloc(ctx, dcorr, Hn, En, Dn, Dmn, center=center)
    torch.cuda.synchronize()
    Er, Dr, _ = o.dos(corr, Hn, H0=center)
    return (E.cpu().numpy(), D.cpu().numpy(), Dm.cpu().numpy()), \
        (En.cpu().numpy(), Dn.cpu().numpy(), Dmn.cpu().numpy()), (Er, Dr)


def test_noalloc_equals_allocating_entry_point_twice(csp, ctx):
    for Nt, R, seed, center in ((300, 3, 4, 0.25), (64, 2, 8, 0.0)):
        (E, D, Dm), (En, Dn, Dmn), (Er, Dr) = _case(csp, ctx, Nt, R, seed, center)
        assert np.array_equal(En, E) and np.array_equal(Dn, D) and np.array_equal(Dmn, Dm)
        assert np.max(np.abs(En - Er)) < 1e-12
        assert np.max(np.abs(Dn - Dr)) < 1e-12
        assert np.max(np.abs(Dmn - Dr.mean(1))) < 1e-12


def test_noalloc_rejects_nt_above_its_scratch(csp, ctx):
    Nt = 262144 + 1
    corr = torch.zeros((2, 1), dtype=torch.complex128, device="cuda:0")
    E = torch.zeros(2, dtype=torch.float64, device="cuda:0")
    D = torch.zeros((2, 1), dtype=torch.float64, device="cuda:0")
    # the shape check comes from Nt alone; the pointers are never used
    with pytest.raises(csp.CspError) as ei:
        csp._check(csp._lib.csp_dos_noalloc(ctx.handle, csp._ptr(corr), Nt, 1, 4.0, 0.0, 3.14,
                                            csp.CSP_WINDOW_HANN, csp._ptr(E), csp._ptr(D), None))
    assert ei.value.status == csp.CSP_EINVAL
    assert "262144" in str(ei.value)
