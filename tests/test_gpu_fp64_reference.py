"""GPU parity at full size against the complex128 reference, for the two
workloads whose full runs the oracle cannot finish:

  - the 1e9-orbital square lattice (31623^2 sites, W = 0.5, seed 6; 4
    random-phase columns, seed 7; 4096 time steps): the complex64 moment
    form (DOS-Concurrent-M, one block, halving) on all 4 columns, and the
    complex64 state assembly (Eq. TE, time blocks of the selection rule's
    size, one column) over all 4096 steps;
  - disordered graphene (honeycomb 4096^2 cells, W = 1 eV, seed 4; 16
    columns, seed 5; 2048 time steps): the complex64 state assembly with the
    autotuned block size over all 2048 steps.

The reference is the complex128 moment form on the GPU at the same size.
It is checked against the FP64 oracle element by element on lattices the
oracle can run (tests/test_gpu_parity.py, test_gpu_configs.py), and at
full size it must obey the properties that hold at any size (C_0 = 1,
|C_j| <= C_0, the discrete DOS sum rule).  The accuracy measure is that of
the Sec. III accuracy paragraph: eps_inf = max |C32 - C64| over every time
and column (printed), and the relative DOS error
max_k |D32 - D64| / max_k |D64| of the column mean, which must stay below
1e-4; each column's own DOS error is held to the same bound, and eps_inf to
2e-5 (the complex64 tolerance of the other parity tests).

Each test prints what it runs before it starts; the reference of the large
lattice is computed one column per test (about half a minute each).
"""
import numpy as np
import pytest

import csp_inputs as ci
import oracle as o

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DOS_TOL = 1e-4
EPS_TOL = 2e-5

# complex128 reference correlations of the large square lattice, per column
_REF = {}


@pytest.fixture(scope="module")
def csp():
    import paper_2510_17432_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(csp):
    c = csp.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def big(csp, ctx):
    w = ci.SQUARE31623
    print("[gpu-ref] square 31623^2 lattice", flush=True)
    lat = csp.Lattice(ctx, w["kind"], w["Lx"], w["Ly"], t=w["t"], W=w["W"],
                      disorder_seed=w["disorder_seed"])
    assert lat.N == 31623 * 31623
    yield lat
    lat.close()


@pytest.fixture(autouse=True)
def release_memory(ctx):
    yield
    ctx.trim()
    torch.cuda.empty_cache()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def dos_mean(c, Hn):
    _, D, im = o.dos(c, Hn)
    assert im < 1e-10
    return D.mean(1)


def rel_dos(c_test, c_ref, Hn):
    d, r = dos_mean(c_test, Hn), dos_mean(c_ref, Hn)
    return float(np.max(np.abs(d - r)) / np.max(np.abs(r)))


def check_properties(c, Hn, tol):
    assert np.max(np.abs(c[0] - 1.0)) < 1e-6                      # C_0 = <psi0|psi0> = 1
    assert np.max(np.abs(c)) < 1.0 + tol                           # |C_j| <= C_0
    _, D, _ = o.dos(c, Hn)
    dE = Hn / (c.shape[0] - 1)
    assert np.max(np.abs(D.sum(axis=0) * dE - c[0].real)) < 1e-10   # discrete sum rule


def compare(name, c32, c64, Hn):
    eps = float(np.max(np.abs(c32 - c64)))
    per_col = [rel_dos(c32[:, k:k + 1], c64[:, k:k + 1], Hn) for k in range(c64.shape[1])]
    rel = rel_dos(c32, c64, Hn)
    print("[gpu-ref] %s: eps_inf %.3e, relative DOS error %.3e (columns %s)" %
          (name, eps, rel, ", ".join("%.2e" % x for x in per_col)), flush=True)
    assert rel < DOS_TOL
    assert max(per_col) < DOS_TOL
    assert eps < EPS_TOL


# ------------------------------------------------- 1e9-orbital square lattice
@pytest.mark.parametrize("col", [0, 1, 2, 3])
def test_square31623_complex128_reference(csp, ctx, big, col):
    w = ci.SQUARE31623
    print("[gpu-ref] complex128 moment form, column %d of 4, %d steps" % (col, w["Nt"]),
          flush=True)
    psi = torch.empty((big.N, w["R"]), dtype=torch.complex128, device="cuda:0")
    csp.csp_states_random_phase(ctx, psi, w["R"], w["seed_states"])
    p = psi[:, col:col + 1].contiguous()
    del psi
    corr, rep = csp.csp_propagate(ctx, big, p, csp.make_params(
        w["Nt"], mode="fp64_conc", assembly=csp.CSP_ASSEMBLE_MOMENTS))
    c = host(corr)
    print("[gpu-ref] column %d: %d recursion steps, %.1f s" % (col, rep.amxsy, rep.ms_total / 1e3),
          flush=True)
    assert rep.amxsy == (o.truncation(w["Nt"] * np.pi) + 1) // 2
    check_properties(c, big.halfwidth, 1e-12)
    _REF[col] = c


def _reference(R):
    if len(_REF) < R:
        pytest.skip("the complex128 reference columns did not run")
    return np.concatenate([_REF[k] for k in range(R)], axis=1)


def test_square31623_complex64_moments_full_run(csp, ctx, big):
    w = ci.SQUARE31623
    ref = _reference(w["R"])
    print("[gpu-ref] complex64 moment form, 4 columns, %d steps" % w["Nt"], flush=True)
    psi = torch.empty((big.N, w["R"]), dtype=torch.complex64, device="cuda:0")
    csp.csp_states_random_phase(ctx, psi, w["R"], w["seed_states"])
    corr, rep = csp.csp_propagate(ctx, big, psi, csp.make_params(
        w["Nt"], mode="fp32_conc", assembly=csp.CSP_ASSEMBLE_MOMENTS))
    c = host(corr)
    del psi
    print("[gpu-ref] %.1f s, %d passes" % (rep.ms_total / 1e3, rep.n_passes), flush=True)
    check_properties(c, big.halfwidth, EPS_TOL)
    compare("1e9 orbitals, complex64 moments", c, ref, big.halfwidth)


def test_square31623_complex64_state_assembly_full_run(csp, ctx, big):
    # one column (the ring of one 8 GB column fills most of the memory), the
    # block size of the selection rule under the memory cap, all 4096 steps
    w = ci.SQUARE31623
    ref = _reference(w["R"])[:, :1]
    psi = torch.empty((big.N, 1), dtype=torch.complex64, device="cuda:0")
    csp.csp_states_random_phase(ctx, psi, 1, w["seed_states"])    # stream 0 = column 0
    params = csp.make_params(w["Nt"], mode="fp32_conc", block_b=0)
    print("[gpu-ref] complex64 state assembly, column 0, %d steps" % w["Nt"], flush=True)
    corr, rep = csp.csp_propagate(ctx, big, psi, params)
    c = host(corr)
    del psi
    print("[gpu-ref] b = %d, K = %d, %d blocks, %.1f s" % (rep.block_b, rep.chunk_K,
                                                           rep.n_blocks, rep.ms_total / 1e3),
          flush=True)
    assert rep.block_b > 1 and rep.chunk_K < o.truncation(rep.block_b * np.pi) + 1
    check_properties(c, big.halfwidth, EPS_TOL)
    compare("1e9 orbitals, complex64 state assembly (column 0)", c, ref, big.halfwidth)


# ------------------------------------------------- disordered graphene 4096^2
def test_disordered_graphene_state_assembly_full_run(csp, ctx):
    w = ci.DISORDERED_GRAPHENE4096
    print("[gpu-ref] disordered graphene 4096^2, R = 16, %d steps" % w["Nt"], flush=True)
    g = csp.Lattice(ctx, w["kind"], w["Lx"], w["Ly"], t=w["t"], W=w["W"],
                    disorder_seed=w["disorder_seed"])
    psi64 = torch.empty((g.N, w["R"]), dtype=torch.complex128, device="cuda:0")
    csp.csp_states_random_phase(ctx, psi64, w["R"], w["seed_states"])
    ref, rref = csp.csp_propagate(ctx, g, psi64, csp.make_params(
        w["Nt"], mode="fp64_conc", assembly=csp.CSP_ASSEMBLE_MOMENTS))
    ref = host(ref)
    print("[gpu-ref] complex128 moment form: %.1f s" % (rref.ms_total / 1e3), flush=True)
    check_properties(ref, g.halfwidth, 1e-12)
    psi = psi64.to(torch.complex64)
    del psi64
    ctx.trim()
    params = csp.make_params(w["Nt"], mode="fp32_conc", block_b=0)
    T = csp.csp_autotune(ctx, [g], [w["R"]], params)
    corr, rep = csp.csp_propagate(ctx, g, psi, params)
    c = host(corr)
    print("[gpu-ref] complex64 state assembly: tuned b = %d, K = %d, %.1f s" %
          (rep.block_b, rep.chunk_K, rep.ms_total / 1e3), flush=True)
    assert rep.block_b == T.block_b
    check_properties(c, g.halfwidth, EPS_TOL)
    compare("disordered graphene, complex64 state assembly", c, ref, g.halfwidth)
    del psi
    g.close()
