"""Fig. 3 ingredients on the GPU, through the C ABI: spin-1 chains (d = 3,
mpo_build lattice 5) against the oracle and exact diagonalisation, and the
merge prediction infidelity reported by sweep against the oracle's."""
import numpy as np
import pytest

from helpers import pl, synth, say, mpo_site
from oracle import models, mpo as M, dmrg

pytestmark = pytest.mark.gpu
Q1 = models.SPIN_ONE_Q
OPS1 = models.OPS_S1


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = pl.Context(0)
    yield c
    c.close()


def sector_ground_energy(H, N, d, q_of, q_target=0):
    idx = np.arange(d ** N)
    q = np.zeros(d ** N, dtype=np.int64)
    for site in range(N):
        q += np.array(q_of)[(idx // d ** (N - 1 - site)) % d]
    sel = np.nonzero(q == q_target)[0]
    return float(np.linalg.eigvalsh(H[np.ix_(sel, sel)])[0])


def test_spin_one_mpo_matches_oracle(ctx):
    N = 10
    mpo = pl.Mpo("chain_s1", N, 1, (1.0, 0.8))
    assert mpo.d == 3 and mpo.phys_q == Q1
    omp = M.build_mpo(models.xxz_terms(models.chain_bonds(N), 1.0, 0.8), N, OPS1, Q1)
    ompo = pl.Mpo(sites=[mpo_site(omp, i) for i in range(N)])
    bonds, sites = synth.random_mps(N, 20, 91, phys_q=Q1)
    mps = pl.Mps(ctx, bonds, sites, Q1, 0)
    e1, e2 = mps.energy(mpo), mps.energy(ompo)
    say("spin-1 MPO energies", e1, e2)
    assert abs(e1 - e2) < 1e-12 * max(1.0, abs(e2))
    mps.free()


def test_spin_one_chain_reaches_ed(ctx):
    N = 6
    terms = models.heisenberg_terms(models.chain_bonds(N))
    E_ed = sector_ground_energy(M.terms_to_dense(terms, N, OPS1), N, 3, Q1)
    mpo = pl.Mpo("chain_s1", N, 1, (1.0, 1.0))
    bonds, sites = synth.random_mps(N, 27, 93, phys_q=Q1)
    mps = pl.Mps(ctx, bonds, sites, Q1, 0)
    for k in range(4):
        rep = mps.sweep(mpo, 64, 1 if k < 1 else 2, dav=pl.dav_params(30, 10, 1e-12),
                        dav_shared=pl.dav_params(40, 10, 1e-12))
    say("spin-1 N=6 gpu", rep["energy"], "ED", E_ed)
    assert abs(rep["energy"] - E_ed) < 1e-10 * abs(E_ed)
    mps.free()


def test_spin_one_chain_matches_oracle_sweeps(ctx):
    N = 12
    bonds, sites = synth.random_mps(N, 24, 95, phys_q=Q1)
    sched = [32, 48, 64, 64]
    omp = M.build_mpo(models.heisenberg_terms(models.chain_bonds(N)), N, OPS1, Q1)
    p = dmrg.SweepParams(schedule=sched, n_warmup=1, n_regions=2, dav=dmrg.DavidsonParams(10, 1e-10, 8),
                         dav_shared=dmrg.DavidsonParams(40, 1e-10, 8))
    st, Eo = dmrg.run_dmrg(omp, bonds, sites, 0, p)
    mpo = pl.Mpo("chain_s1", N, 1, (1.0, 1.0))
    mps = pl.Mps(ctx, bonds, sites, Q1, 0)
    Eg = [mps.sweep(mpo, m, 1 if k < 1 else 2, dav=pl.dav_params(10, 8, 1e-10),
                    dav_shared=pl.dav_params(40, 8, 1e-10))["energy"] for k, m in enumerate(sched)]
    say("spin-1 N=12 gpu", Eg, "oracle", Eo)
    # the first sweep truncates a random state to m = 32 through degenerate
    # SU(2) multiplets of the spin-1 spectrum, where rounding decides which
    # states stay (the truncation reading of ties); the sweeps after it agree
    assert abs(Eg[0] - Eo[0]) <= 1e-4 * abs(Eo[0])
    for a, b in zip(Eg[1:], Eo[1:]):
        assert abs(a - b) <= 1e-9 * abs(b)
    mps.free()


def test_merge_infidelity_matches_oracle(ctx):
    """Chain N = 16, 2 regions, no warm-up, 4 matvecs per interior bond: the
    per-sweep merge infidelity of the GPU sweep equals the oracle's (one merge
    per sweep) and decays to rounding."""
    N = 16
    bonds, sites = synth.random_mps(N, 16, 1)
    sched = [16, 32, 64, 64, 64, 64]
    omp = M.build_mpo(models.heisenberg_terms(models.chain_bonds(N)), N, models.OPS, models.SPIN_HALF_Q)
    p = dmrg.SweepParams(schedule=sched, n_warmup=0, n_regions=2, dav=dmrg.DavidsonParams(4, 1e-11, 8),
                         dav_shared=dmrg.DavidsonParams(60, 1e-12, 10))
    st, Eo = dmrg.run_dmrg(omp, bonds, sites, 0, p)
    io = [e["infidelity"] for e in st.log if e["kind"] == "merge"]
    mpo = pl.Mpo("chain", N, 1, (1.0, 1.0))
    mps = pl.Mps(ctx, bonds, sites)
    ig = [mps.sweep(mpo, m, 2, dav=pl.dav_params(4, 8, 1e-11), dav_shared=pl.dav_params(60, 10, 1e-12))
          ["max_infidelity"] for m in sched]
    say("merge infidelity gpu", ["%.3e" % v for v in ig], "oracle", ["%.3e" % v for v in io])
    assert len(io) == len(ig)
    for a, b in zip(ig, io):
        assert abs(a - b) <= max(1e-6 * b, 1e-12), (a, b)
    assert ig[0] > 1e-2 and max(ig[-2:]) < 1e-12
    mps.free()
