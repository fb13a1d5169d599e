"""GPU: the propagation forms keep their vectors with rows padded to a
multiple of 16 values (128-byte aligned rows); callers pass and receive
packed [N][R] blocks.  Lattices whose rows are not such a multiple (and one
whose rows are) run the state assembly and the moment form with time
blocks, the norm guard (which reads whole padded vectors) and a final state,
against the FP64 oracle."""
import numpy as np
import pytest

import oracle as o

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LATS = [
    dict(kind="square", Lx=37, Ly=23, t=1.0, W=1.3, disorder_seed=5),       # rows of 37
    dict(kind="honeycomb", Lx=19, Ly=21, t=-2.7, W=0.5, disorder_seed=2),   # rows of 38
    dict(kind="chain", Lx=301, t=1.0, W=2.0, disorder_seed=9),              # one row of 301
    dict(kind="square", Lx=13, Ly=29, t=-1.0, W=0.0, periodic_x=False),     # open rows of 13
    dict(kind="square", Lx=32, Ly=9, t=1.0, W=0.7, disorder_seed=3),        # rows of 32: unpadded
]


@pytest.fixture(scope="module")
def csp():
    import paper_2510_17432_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(csp):
    c = csp.Context(0)
    yield c
    c.close()


def pair(csp, ctx, spec):
    g = csp.Lattice(ctx, **spec)
    spec2 = dict(spec)
    kind = spec2.pop("kind")
    Lx = spec2.pop("Lx")
    Ly = spec2.pop("Ly", 1)
    return g, o.Lattice(kind, Lx, Ly, **spec2)


@pytest.mark.parametrize("spec", LATS)
def test_padded_rows_against_oracle(csp, ctx, spec):
    print("[gpu] padded layout %s %dx%d" % (spec["kind"], spec["Lx"], spec.get("Ly", 1)),
          flush=True)
    g, c = pair(csp, ctx, spec)
    R, Nt, b = 3, 40, 8
    psi = o.random_phase_states_fast(c.N, R, 11)
    ref, _, fin_ref = o.propagate(c, psi, Nt, b=0, return_final=True)
    cases = [("fp64_conc", csp.CSP_ASSEMBLE_STATES, torch.complex128, 1e-10, 1e-10),
             ("fp32_conc", csp.CSP_ASSEMBLE_STATES, torch.complex64, 2e-5, 1e-4),
             ("fp64_conc", csp.CSP_ASSEMBLE_MOMENTS, torch.complex128, 1e-10, 1e-10),
             ("fp32_conc", csp.CSP_ASSEMBLE_MOMENTS, torch.complex64, 2e-5, 1e-4)]
    for mode, assembly, dt, tol_c, tol_f in cases:
        p = torch.from_numpy(np.ascontiguousarray(psi)).to("cuda:0").to(dt)
        fin = torch.zeros_like(p)
        params = csp.make_params(Nt, mode=mode, block_b=b, assembly=assembly, check_norm=True)
        corr, rep = csp.csp_propagate(ctx, g, p, params, final=fin)
        torch.cuda.synchronize()
        got, fgot = corr.cpu().numpy(), fin.cpu().numpy()
        assert fgot.shape == (c.N, R)
        assert np.max(np.abs(got - ref)) < tol_c, (mode, assembly)
        assert np.max(np.abs(fgot - fin_ref)) < tol_f, (mode, assembly)
    g.close()
