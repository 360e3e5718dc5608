"""Pins of the oracle's inverse canonical gauge and local measurements
(Sec. IV) against brute force on the dense state vector and against exact
diagonalisation."""
import numpy as np
import pytest

from oracle import models, mpo as M, exact, dmrg, gauge
from oracle.blocks import Bond
from paper_1301_3494_amd import synth

from helpers import dense_state, dense_sz, dense_exchange

PQ = models.SPIN_HALF_Q
OPS = models.OPS


def _random_ic(N=8, m=6, seed=3, q_target=0):
    bonds, sites = synth.random_mps(N, m, seed, q_target=q_target)
    mpo = M.build_mpo(models.heisenberg_terms(models.chain_bonds(N)), N, OPS, PQ)
    ic = gauge.inverse_canonical(mpo, bonds, sites, q_target)
    ref = dense_state(sites, [Bond(b) for b in bonds], N)
    return ic, ref / np.linalg.norm(ref)


def test_inverse_canonical_is_the_same_state():
    """psi_0 V_1 psi_1 ... V_{N-1} psi_{N-1} reproduces the input state."""
    ic, ref = _random_ic()
    back = dense_state(ic.psi, ic.bonds, ic.N, ic.V)
    s = np.sign(back @ ref)
    assert np.max(np.abs(back - s * ref)) < 1e-12
    assert abs(abs(back @ ref) - 1.0) < 1e-12


def test_every_site_is_an_orthogonality_centre():
    """psi_j^T psi_j = Lambda_{j+1}^2 over the right index and psi_j psi_j^T =
    Lambda_j^2 over the left index, on every site; V Lambda = 1."""
    ic, _ = _random_ic(N=10, m=8, seed=5)
    assert max(gauge.oc_residuals(ic)) < 1e-13
    for b in range(1, ic.N):
        for q in ic.lam[b]:
            assert np.allclose(ic.V[b][q] * ic.lam[b][q], 1.0, rtol=0, atol=1e-12)
    assert ic.n_floored == 0
    # a deliberately broken centre (one psi replaced by its left-orthonormal
    # factor) fails the residual check
    bad = gauge.InverseCanonical(ic.bonds, list(ic.psi), ic.V, ic.lam, ic.phys_q, 0)
    j = 4
    bad.psi[j] = {k: v * ic.V[j + 1][k[0] + PQ[k[1]]][None, :] for k, v in ic.psi[j].items()}
    assert gauge.oc_residuals(bad)[j] > 1e-3


@pytest.mark.parametrize("q_target", [0, 2])
def test_site_expectations_match_dense_state(q_target):
    ic, ref = _random_ic(N=8, m=6, seed=7, q_target=q_target)
    for j in range(ic.N):
        assert abs(gauge.expect_site(ic, j, OPS["Sz"]) - dense_sz(ref, ic.N, j)) < 1e-12
    tot = sum(gauge.expect_site(ic, j, OPS["Sz"]) for j in range(ic.N))
    assert abs(tot - q_target / 2) < 1e-12
    # an identity "measurement" is the norm of each centre
    for j in range(ic.N):
        assert abs(gauge.expect_site(ic, j, OPS["I"]) - 1.0) < 1e-12


def test_correlators_match_dense_state():
    ic, ref = _random_ic(N=8, m=6, seed=9)
    terms = gauge.heisenberg_exchange(OPS)
    for (i, k) in [(0, 1), (2, 3), (1, 4), (0, 7), (3, 6), (6, 7)]:
        got = gauge.correlator(ic, i, k, terms)
        assert abs(got - dense_exchange(ref, ic.N, i, k)) < 1e-12, (i, k)
    # a single term: <Sz_i Sz_k>
    zz = gauge.correlator(ic, 2, 5, [(1.0, OPS["Sz"], OPS["Sz"])])
    idx = np.arange(ref.size)
    want = np.sum(ref ** 2 * np.where(((idx >> 2) & 1) == ((idx >> 5) & 1), 0.25, -0.25))
    assert abs(zz - want) < 1e-12


def test_ground_state_bond_energies_sum_to_ed_energy():
    """Converged DMRG ground state of the open Heisenberg chain (N = 10): the
    nearest-neighbour exchanges from the centres match exact diagonalisation
    one by one, and sum to E_ED; in the sector 2 S^z = 2 (two regions, V on
    the shared bond folded into its left neighbour first) the S^z profile
    matches ED and sums to 1."""
    N = 10
    for q_target in (0, 2):
        bonds_h = models.chain_bonds(N)
        terms = models.heisenberg_terms(bonds_h)
        mpo = M.build_mpo(terms, N, OPS, PQ)
        bonds, sites = synth.random_mps(N, 16, 11, q_target=q_target)
        # the second case ends with V on the shared bond of two regions
        nreg = 1 if q_target == 0 else 2
        p = dmrg.SweepParams(schedule=[32] * 5, n_warmup=1, n_regions=nreg,
                             dav=dmrg.DavidsonParams(30, 1e-11, 10), dav_shared=dmrg.DavidsonParams(40, 1e-12, 10))
        st, E = dmrg.run_dmrg(mpo, bonds, sites, q_target, p)
        assert bool(st.V) == (nreg > 1)
        w, v, basis = exact.ground_state(terms, N, q_target)
        ic = gauge.inverse_canonical(mpo, st.bonds, gauge.plain_sites(st), q_target)
        ex = gauge.heisenberg_exchange(OPS)
        tot = 0.0
        for (i, k) in bonds_h:
            H1, _ = exact.sparse_hamiltonian(models.heisenberg_terms([(i, k)]), N, q_target)
            want = float(v[:, 0] @ (H1 @ v[:, 0]))
            got = gauge.correlator(ic, i, k, ex)
            assert abs(got - want) < 1e-7, (q_target, i, k, got, want)
            tot += got
        assert abs(tot - w[0]) < 1e-9 * abs(w[0])
        sz = [gauge.expect_site(ic, j, OPS["Sz"]) for j in range(N)]
        assert abs(sum(sz) - q_target / 2) < 1e-12
        for j in range(N):
            Hz, _ = exact.sparse_hamiltonian([(1.0, ((j, "Sz"),))], N, q_target)
            assert abs(sz[j] - float(v[:, 0] @ (Hz @ v[:, 0]))) < 1e-7


def test_correlator_detects_planted_sign_error():
    """A wrong sign on the flip terms (a plausible slip) breaks the match."""
    ic, ref = _random_ic(N=6, m=4, seed=13)
    bad = [(1.0, OPS["Sz"], OPS["Sz"]), (-0.5, OPS["Sp"], OPS["Sm"]), (-0.5, OPS["Sm"], OPS["Sp"])]
    i, k = 1, 3
    assert abs(gauge.correlator(ic, i, k, bad) - dense_exchange(ref, ic.N, i, k)) > 1e-3
