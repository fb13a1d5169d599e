"""GPU parity at full size: graphene, honeycomb 1024 x 1024 cells
(2 097 152 orbitals), periodic, t = -2.7 eV, 4 random-phase columns (seed 2)
and 64 LDOS sites (seed 3), 2048 time steps, in the launch configuration
of the graphene leg that bench.py times (complex64, b = 32, split-bf16 MFMA
contraction).

The reference is the oracle's band-structure closed form of the clean
periodic lattice, valid at any size: every correlation at every time
point, for the random columns and for the localized columns (whose return
amplitude is the same for every site).  Tolerances: complex64 path 2e-5
absolute on correlations, 1e-4 relative on the DOS and on the LDOS;
complex128 sequential form 1e-10 on correlations.
"""
import math

import numpy as np
import pytest

import oracle as o

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LX = LY = 1024
T_HOP = -2.7
NT = 2048
R_RAND, N_SITES = 4, 64
SEED_STATES, SEED_SITES = 2, 3


@pytest.fixture(scope="module")
def csp():
    import paper_2510_17432_amd as m
    return m


@pytest.fixture(scope="module")
def setup(csp):
    print("[gpu-full] context + lattice", flush=True)
    ctx = csp.Context(0)
    lat = csp.Lattice(ctx, "honeycomb", LX, LY, t=T_HOP)
    N = lat.N
    psi = torch.empty((N, R_RAND + N_SITES), dtype=torch.complex64, device="cuda:0")
    csp.csp_states_random_phase(ctx, psi, R_RAND, SEED_STATES, col0=0)
    sites = csp.csp_ldos_sites(ctx, N, N_SITES, SEED_SITES)
    csp.csp_states_sites(ctx, psi, sites, col0=R_RAND)
    torch.cuda.synchronize()
    # reference: closed form for the random columns and one unit column
    print("[gpu-full] oracle closed form", flush=True)
    rnd = o.random_phase_states_fast(N, R_RAND, SEED_STATES)
    unit = np.zeros((N, 1), dtype=np.complex128)
    unit[0, 0] = 1.0
    tau = math.pi / lat.halfwidth
    ref = o.bloch_corr_uniform("honeycomb", LX, LY, T_HOP, np.concatenate([rnd, unit], 1), tau,
                               NT + 1)
    yield dict(ctx=ctx, lat=lat, psi=psi, sites=sites, rnd=rnd, ref_rand=ref[:, :R_RAND],
               ref_ldos=ref[:, R_RAND])
    del psi
    ctx.close()


def rel_dos_err(c_test, c_ref, Hn):
    _, Dt, _ = o.dos(c_test, Hn)
    _, Dr, _ = o.dos(c_ref, Hn)
    return float(np.max(np.abs(Dt.mean(1) - Dr.mean(1))) / np.max(np.abs(Dr.mean(1))))


def test_states_and_sites_match_oracle_generator(setup):
    lat, psi = setup["lat"], setup["psi"]
    assert lat.halfwidth == o.Lattice("honeycomb", 4, 4, t=T_HOP).halfwidth()
    rows = np.random.default_rng(0).choice(lat.N, 4096, replace=False)
    got = psi[torch.from_numpy(rows).to("cuda:0")].cpu().numpy()
    assert np.max(np.abs(got[:, :R_RAND] - setup["rnd"][rows])) < 1e-7
    sites = setup["sites"].cpu().numpy()
    assert np.array_equal(sites, o.ldos_sites(lat.N, N_SITES, SEED_SITES))
    assert np.array_equal(got[:, R_RAND:], o.site_states(lat.N, sites)[rows].astype(np.complex64))


def test_fp32_concurrent_bench_configuration(csp, setup):
    print("[gpu-full] complex64 concurrent, b = 32, R = 68", flush=True)
    ctx, lat, psi = setup["ctx"], setup["lat"], setup["psi"]
    params = csp.make_params(NT, mode="fp32_conc", block_b=32)
    corr, rep = csp.csp_propagate(ctx, lat, psi, params)
    torch.cuda.synchronize()
    assert rep.block_b == 32 and rep.n_groups == 3 and rep.amxsy == 64 * 148
    c = corr.cpu().numpy()
    err_rand = np.max(np.abs(c[:, :R_RAND] - setup["ref_rand"]))
    err_ldos = np.max(np.abs(c[:, R_RAND:] - setup["ref_ldos"][:, None]))
    print("[gpu-full] eps_inf random %.3e, ldos %.3e" % (err_rand, err_ldos), flush=True)
    assert err_rand < 2e-5 and err_ldos < 2e-5
    e_dos = rel_dos_err(c[:, :R_RAND], setup["ref_rand"], lat.halfwidth)
    e_ldos = rel_dos_err(c[:, R_RAND:], np.repeat(setup["ref_ldos"][:, None], N_SITES, 1),
                         lat.halfwidth)
    print("[gpu-full] relative DOS error %.3e, LDOS %.3e" % (e_dos, e_ldos), flush=True)
    assert e_dos < 1e-4 and e_ldos < 1e-4
    # the GPU transform of the same correlations equals the oracle transform
    E, D, Dm = csp.csp_dos(ctx, corr[:, :R_RAND].contiguous(), lat.halfwidth)
    Er, Dr, _ = o.dos(c[:, :R_RAND], lat.halfwidth)
    assert np.max(np.abs(Dm.cpu().numpy() - Dr.mean(1))) < 1e-12


def test_fp64_sequential_full_size(csp, setup):
    print("[gpu-full] complex128 sequential, R = 4", flush=True)
    ctx, lat = setup["ctx"], setup["lat"]
    p64 = torch.from_numpy(setup["rnd"]).to("cuda:0")
    corr, rep = csp.csp_propagate(ctx, lat, p64, csp.make_params(NT, mode="fp64_seq"))
    torch.cuda.synchronize()
    assert rep.amxsy == NT * 20
    err = np.max(np.abs(corr.cpu().numpy() - setup["ref_rand"]))
    print("[gpu-full] eps_inf %.3e" % err, flush=True)
    assert err < 1e-10


def test_fp32_moments_single_block_full_size(csp, setup):
    # DOS-Concurrent-M of Sec. III: one block of 2048 steps, halving
    print("[gpu-full] complex64 moments, one block, halving, R = 68", flush=True)
    ctx, lat, psi = setup["ctx"], setup["lat"], setup["psi"]
    params = csp.make_params(NT, mode="fp32_conc", block_b=0, assembly=csp.CSP_ASSEMBLE_MOMENTS)
    corr, rep = csp.csp_propagate(ctx, lat, psi, params)
    torch.cuda.synchronize()
    Nfull = o.truncation(NT * math.pi)
    assert rep.amxsy == (Nfull + 1) // 2 and rep.dot == Nfull
    c = corr.cpu().numpy()
    err_rand = np.max(np.abs(c[:, :R_RAND] - setup["ref_rand"]))
    err_ldos = np.max(np.abs(c[:, R_RAND:] - setup["ref_ldos"][:, None]))
    print("[gpu-full] moments eps_inf random %.3e, ldos %.3e" % (err_rand, err_ldos), flush=True)
    assert err_rand < 2e-5 and err_ldos < 2e-5
    e_dos = rel_dos_err(c[:, :R_RAND], setup["ref_rand"], lat.halfwidth)
    e_ldos = rel_dos_err(c[:, R_RAND:], np.repeat(setup["ref_ldos"][:, None], N_SITES, 1),
                         lat.halfwidth)
    print("[gpu-full] moments relative DOS error %.3e, LDOS %.3e" % (e_dos, e_ldos), flush=True)
    assert e_dos < 1e-4 and e_ldos < 1e-4
