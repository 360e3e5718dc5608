"""Pins of the Sec. III pinning terms and order parameters (D_x of the J-Q2
study, M_z of the triangular study) as the oracle computes them from the
orthogonality centres: against exact diagonalisation of small cylinders."""
import numpy as np
import pytest

from oracle import models, mpo as M, exact, dmrg, gauge
from paper_1301_3494_amd import synth

PQ = models.SPIN_HALF_Q
OPS = models.OPS


def ed_expect(terms_obs, N, v, q=0):
    H1, _ = exact.sparse_hamiltonian(terms_obs, N, q)
    return float(v @ (H1 @ v))


def ed_dx(Lx, Ly, v):
    xc = Lx // 2 - 1

    def bond(x, y):
        a, b = models.snake_site(x, y, Ly), models.snake_site(x + 1, y, Ly)
        return ed_expect(models.heisenberg_terms([(min(a, b), max(a, b))]), Lx * Ly, v)
    return sum(bond(xc, y) - 0.5 * bond(xc - 1, y) - 0.5 * bond(xc + 1, y) for y in range(Ly)) / Ly


def ed_mz(Lx, Ly, v):
    xc = (Lx - 1) // 2
    vals = [ed_expect([(1.0, ((models.snake_site(xc, y, Ly), "Sz"),))], Lx * Ly, v)
            for y in range(Ly) if models.tri_sublattice(xc, y) == 0]
    return sum(vals) / len(vals)


def _ground(terms, N, seed, m=64, sweeps=5):
    mpo = M.build_mpo(terms, N, OPS, PQ)
    bonds, sites = synth.random_mps(N, 16, seed)
    p = dmrg.SweepParams(schedule=[m] * sweeps, dav=dmrg.DavidsonParams(30, 1e-11, 10))
    st, E = dmrg.run_dmrg(mpo, bonds, sites, 0, p)
    ic = gauge.inverse_canonical(mpo, st.bonds, gauge.plain_sites(st), 0)
    return ic, E[-1]


def test_three_colouring_of_the_triangular_cylinder():
    for x, y in [(0, 0), (3, 4), (5, 5)]:
        for dx, dy in [(0, 1), (1, 0), (1, -1)]:
            assert models.tri_sublattice(x, y) != models.tri_sublattice(x + dx, (y + dy) % 6)


def test_jq2_pinned_dx_matches_ed():
    """Pure-Q2 plus a weak J on the pinned 4x3 cylinder: D_x from the centres
    of the converged DMRG state against D_x of the ED ground state; pinning
    changes D_x (it is not a no-op)."""
    Lx, Ly, N = 4, 3, 12
    terms = models.jq2_terms(Lx, Ly, 0.2, 1.0, pin=1.0)
    w, v, _ = exact.ground_state(terms, N, 0)
    ic, E = _ground(terms, N, 3)
    assert abs(E - w[0]) < 1e-9 * abs(w[0])
    dx = gauge.order_dx(ic, Lx, Ly, OPS, models.snake_site)
    want = ed_dx(Lx, Ly, v[:, 0])
    assert abs(dx - want) < 1e-7, (dx, want)
    w0, v0, _ = exact.ground_state(models.jq2_terms(Lx, Ly, 0.2, 1.0), N, 0)
    assert abs(ed_dx(Lx, Ly, v0[:, 0]) - want) > 1e-3


def test_triangular_pinned_mz_matches_ed():
    """Triangular 4x3 cylinder with the edge field h = J/2 on sublattice 0:
    M_z of the centre column from the centres against ED, and nonzero."""
    Lx, Ly, N = 4, 3, 12
    terms = models.heisenberg_terms(models.triangular_cylinder_bonds(Lx, Ly)) + \
        models.triangular_pin_terms(Lx, Ly, 0.5)
    w, v, _ = exact.ground_state(terms, N, 0)
    ic, E = _ground(terms, N, 5)
    assert abs(E - w[0]) < 1e-9 * abs(w[0])
    mz = gauge.order_mz(ic, Lx, Ly, OPS, models.snake_site, models.tri_sublattice)
    want = ed_mz(Lx, Ly, v[:, 0])
    assert abs(mz - want) < 1e-7, (mz, want)
    assert abs(want) > 1e-3
