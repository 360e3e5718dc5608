"""Pins of the Fig. 3 ingredients in the oracle: spin-1 chains (d = 3) and the
prediction infidelity 1 - |<Psi'|Psi>| of the merged state."""
import numpy as np
import pytest

from oracle import models, mpo as M, dmrg
from paper_1301_3494_amd import synth

OPS1 = models.OPS_S1
Q1 = models.SPIN_ONE_Q


def sector_ground_energy(H, N, d, q_of, q_target=0):
    idx = np.arange(d ** N)
    q = np.zeros(d ** N, dtype=np.int64)
    for site in range(N):
        digit = (idx // d ** (N - 1 - site)) % d      # site 0 is the leading Kronecker factor
        q += np.array(q_of)[digit]
    sel = np.nonzero(q == q_target)[0]
    return float(np.linalg.eigvalsh(H[np.ix_(sel, sel)])[0])


def test_spin_one_operators():
    """Spin-1 algebra: [S+, S-] = 2 Sz, S^2 = S(S+1) = 2."""
    Sz, Sp, Sm = OPS1["Sz"], OPS1["Sp"], OPS1["Sm"]
    assert np.allclose(Sp @ Sm - Sm @ Sp, 2 * Sz)
    S2 = Sz @ Sz + 0.5 * (Sp @ Sm + Sm @ Sp)
    assert np.allclose(S2, 2.0 * np.eye(3))


def test_spin_one_mpo_equals_kronecker_sum():
    N = 5
    terms = models.heisenberg_terms(models.chain_bonds(N))
    mpo = M.build_mpo(terms, N, OPS1, Q1)
    assert np.abs(M.mpo_to_dense(mpo) - M.terms_to_dense(terms, N, OPS1)).max() < 1e-13


def test_spin_one_dmrg_reaches_ed():
    N = 6
    terms = models.heisenberg_terms(models.chain_bonds(N))
    E_ed = sector_ground_energy(M.terms_to_dense(terms, N, OPS1), N, 3, Q1)
    mpo = M.build_mpo(terms, N, OPS1, Q1)
    bonds, sites = synth.random_mps(N, 27, 3, phys_q=Q1)
    st, E = dmrg.run_dmrg(mpo, bonds, sites, 0, dmrg.SweepParams(schedule=[64] * 4,
                                                                   dav=dmrg.DavidsonParams(30, 1e-12, 10)))
    assert abs(E[-1] - E_ed) < 1e-10 * abs(E_ed)


def test_prediction_infidelity_formula():
    rng = np.random.default_rng(1)
    a = {(0, 0, 1): rng.standard_normal((3, 4)), (1, 1, 0): rng.standard_normal((2, 2))}
    perp = {k: rng.standard_normal(v.shape) for k, v in a.items()}
    # make perp orthogonal to a, then mix at a known angle
    na2 = sum(float(np.sum(v * v)) for v in a.values())
    ov = sum(float(np.sum(a[k] * perp[k])) for k in a)
    perp = {k: perp[k] - ov / na2 * a[k] for k in a}
    np2 = sum(float(np.sum(v * v)) for v in perp.values())
    th = 0.3
    b = {k: np.cos(th) * a[k] / np.sqrt(na2) + np.sin(th) * perp[k] / np.sqrt(np2) for k in a}
    assert abs(dmrg.prediction_infidelity(a, b) - (1 - np.cos(th))) < 1e-14
    assert dmrg.prediction_infidelity(a, {k: -3 * v for k, v in a.items()}) < 1e-15


def test_merge_prediction_improves_to_convergence():
    """Parallel sweeps (2 regions, no warm-up, 4 matvecs per interior bond) of
    the N = 16 chain: every merge records an infidelity in [0, 1); it falls
    from O(1) at the first merge by orders of magnitude per sweep to the
    rounding level once the state has converged (the behaviour Fig. 3
    reports)."""
    N = 16
    mpo = M.build_mpo(models.heisenberg_terms(models.chain_bonds(N)), N, models.OPS, models.SPIN_HALF_Q)
    bonds, sites = synth.random_mps(N, 16, 1)
    p = dmrg.SweepParams(schedule=[16, 32, 64, 64, 64, 64], n_warmup=0, n_regions=2,
                         dav=dmrg.DavidsonParams(4, 1e-11, 8), dav_shared=dmrg.DavidsonParams(60, 1e-12, 10))
    st, E = dmrg.run_dmrg(mpo, bonds, sites, 0, p)
    inf = [e["infidelity"] for e in st.log if e["kind"] == "merge"]
    assert inf and all(0.0 <= v < 1.0 for v in inf)
    assert inf[0] > 1e-2 and inf[0] > inf[1] > inf[2]
    assert max(inf[-2:]) < 1e-12
