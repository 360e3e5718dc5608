"""Inverse canonical gauge and local measurements (Sec. IV) on the GPU,
through the C ABI, against the oracle, brute force on dense states and exact
diagonalisation; full-size checks at the 8x4, m = 1024 cylinder."""
import numpy as np
import pytest

from helpers import pl, synth, say, dense_state, dense_sz, dense_exchange
from oracle import models, mpo as M, dmrg, exact, gauge
from oracle.blocks import Bond

pytestmark = pytest.mark.gpu
OPS = models.OPS
PQ = models.SPIN_HALF_Q
EXCHANGE = gauge.heisenberg_exchange(OPS)


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = pl.Context(0)
    yield c
    c.close()


def gpu_ic(mps):
    """The GPU's converted state as an oracle InverseCanonical (read back)."""
    bonds = [Bond(mps.bond(b)) for b in range(mps.N + 1)]
    psi = [mps.site_blocks(j) for j in range(mps.N)]
    V = {b: mps.get_v(b) for b in range(1, mps.N)}
    lam = {b: {q: 1.0 / v for q, v in V[b].items()} for b in V}
    return gauge.InverseCanonical(bonds, psi, V, lam, PQ, 0)


def _random(N, m, seed, q_target=0):
    bonds, sites = synth.random_mps(N, m, seed, q_target=q_target)
    omp = M.build_mpo(models.heisenberg_terms(models.chain_bonds(N)), N, OPS, PQ)
    return bonds, sites, omp


@pytest.mark.parametrize("q_target", [0, 2])
def test_conversion_matches_oracle(ctx, q_target):
    N, m = 10, 12
    bonds, sites, omp = _random(N, m, 21 + q_target, q_target)
    mps = pl.Mps(ctx, bonds, sites, PQ, q_target)
    nfl = mps.inverse_canonical()
    ic_o = gauge.inverse_canonical(omp, bonds, sites, q_target)
    ic_g = gpu_ic(mps)
    assert nfl == 0 and ic_o.n_floored == 0
    for b in range(N + 1):
        assert ic_g.bonds[b] == ic_o.bonds[b], b
    # Schmidt values are unique (random state: no degeneracy)
    err_v = max(float(np.max(np.abs(ic_g.V[b][q] / ic_o.V[b][q] - 1.0))) for b in range(1, N) for q in ic_o.V[b])
    # every site an orthogonality centre, the state unchanged
    res = max(gauge.oc_residuals(ic_g))
    ref = dense_state(sites, [Bond(b) for b in bonds], N)
    ref /= np.linalg.norm(ref)
    back = dense_state(ic_g.psi, ic_g.bonds, N, ic_g.V)
    ov = abs(float(back @ ref))
    say("icmps conversion q", q_target, "V rel", err_v, "OC residual", res, "overlap-1", ov - 1.0)
    assert err_v < 1e-10
    assert res < 1e-12
    assert abs(ov - 1.0) < 1e-12
    mps.free()


def test_site_expectations(ctx):
    N, m = 10, 12
    for q_target in (0, 2):
        bonds, sites, omp = _random(N, m, 31, q_target)
        mps = pl.Mps(ctx, bonds, sites, PQ, q_target)
        mps.inverse_canonical()
        ic_o = gauge.inverse_canonical(omp, bonds, sites, q_target)
        ref = dense_state(sites, [Bond(b) for b in bonds], N)
        ref /= np.linalg.norm(ref)
        sz = mps.expect_site(OPS["Sz"])
        want = np.array([gauge.expect_site(ic_o, j, OPS["Sz"]) for j in range(N)])
        assert np.max(np.abs(sz - want)) < 1e-12
        assert np.max(np.abs(sz - [dense_sz(ref, N, j) for j in range(N)])) < 1e-12
        assert abs(sz.sum() - q_target / 2) < 1e-12
        assert np.max(np.abs(mps.expect_site(OPS["I"]) - 1.0)) < 1e-12
        O = np.diag([0.3, -1.1])
        got = mps.expect_site(O)
        assert np.max(np.abs(got - [gauge.expect_site(ic_o, j, O) for j in range(N)])) < 1e-12
        # charge-changing entries cannot contribute in a U(1) eigenstate
        assert np.max(np.abs(mps.expect_site(OPS["Sx"]))) == 0.0
        mps.free()


def test_pair_correlators(ctx):
    N, m = 10, 12
    bonds, sites, omp = _random(N, m, 41)
    mps = pl.Mps(ctx, bonds, sites, PQ, 0)
    mps.inverse_canonical()
    ic_o = gauge.inverse_canonical(omp, bonds, sites, 0)
    ref = dense_state(sites, [Bond(b) for b in bonds], N)
    ref /= np.linalg.norm(ref)
    pairs = [(0, 1), (2, 5), (0, 9), (3, 4), (6, 8), (8, 9), (1, 7)]
    got = mps.expect_pairs(EXCHANGE, pairs, concurrent=True)
    seq = mps.expect_pairs(EXCHANGE, pairs, concurrent=False)
    assert np.array_equal(got, seq), "concurrent and sequential differ"
    want = np.array([gauge.correlator(ic_o, i, k, EXCHANGE) for i, k in pairs])
    dense = np.array([dense_exchange(ref, N, i, k) for i, k in pairs])
    say("pairs gpu-oracle", np.max(np.abs(got - want)), "gpu-dense", np.max(np.abs(got - dense)))
    assert np.max(np.abs(got - want)) < 1e-12
    assert np.max(np.abs(got - dense)) < 1e-12
    zz = mps.expect_pairs([(1.0, OPS["Sz"], OPS["Sz"])], [(2, 6)])
    assert abs(zz[0] - gauge.correlator(ic_o, 2, 6, [(1.0, OPS["Sz"], OPS["Sz"])])) < 1e-12
    mps.free()


def test_errors(ctx):
    bonds, sites, _ = _random(8, 6, 51)
    mps = pl.Mps(ctx, bonds, sites, PQ, 0)
    with pytest.raises(pl.PdmrgError):
        mps.expect_site(OPS["Sz"])          # not in the inverse canonical gauge yet
    mps.inverse_canonical()
    with pytest.raises(pl.PdmrgError):
        mps.expect_pairs(EXCHANGE, [(3, 3)])
    with pytest.raises(pl.PdmrgError):
        mps.expect_pairs(EXCHANGE, [(4, 2)])
    with pytest.raises(pl.PdmrgError):
        mps.expect_pairs([(1.0, OPS["Sz"] + OPS["Sp"], OPS["Sz"])], [(1, 2)])   # no definite charge
    with pytest.raises(pl.PdmrgError):
        mps.expect_pairs([(1.0, OPS["Sp"], OPS["Sp"])], [(1, 2)])               # charges do not cancel
    with pytest.raises(pl.PdmrgError):
        mps.get_v(0)                                                           # outer bond: no V
    mps.free()


@pytest.mark.parametrize("n_regions", [1, 2])
def test_ground_state_bonds_match_ed(ctx, n_regions):
    """4x3 cylinder ground state by GPU sweeps (two regions leave V on the
    shared bond, folded back by the conversion): every Hamiltonian bond's
    <S_i.S_k> against exact diagonalisation, their sum against E_ED and
    mps_energy; a sweep after the conversion keeps the energy."""
    Lx, Ly = 4, 3
    N = Lx * Ly
    hb = models.square_cylinder_bonds(Lx, Ly)
    terms = models.heisenberg_terms(hb)
    w, v, basis = exact.ground_state(terms, N, 0)
    mpo = pl.Mpo("square", Lx, Ly, (1.0, 1.0))
    bonds, sites = synth.random_mps(N, 16, 61)
    mps = pl.Mps(ctx, bonds, sites, PQ, 0)
    dav = pl.dav_params(30, 10, 1e-11)
    davs = pl.dav_params(40, 10, 1e-12)
    for k in range(6):
        mps.sweep(mpo, 64, 1 if k < 2 else n_regions, dav=dav, dav_shared=davs)
    E_before = mps.energy(mpo)
    mps.inverse_canonical()
    assert abs(mps.energy(mpo) - E_before) < 1e-11 * abs(E_before)
    pairs = [(min(i, k), max(i, k)) for i, k in hb]
    got = mps.expect_pairs(EXCHANGE, pairs)
    for (i, k), g in zip(pairs, got):
        H1, _ = exact.sparse_hamiltonian(models.heisenberg_terms([(i, k)]), N, 0)
        assert abs(g - float(v[:, 0] @ (H1 @ v[:, 0]))) < 1e-7, (i, k)
    say("4x3 regions", n_regions, "sum bonds", got.sum(), "E_ED", w[0], "E mps", E_before)
    assert abs(got.sum() - w[0]) < 1e-9 * abs(w[0])
    assert abs(got.sum() - E_before) < 1e-10 * abs(E_before)
    sz = mps.expect_site(OPS["Sz"])
    assert np.max(np.abs(sz)) < 1e-7          # S^z = 0 sector, spin-flip symmetric ground state
    rep = mps.sweep(mpo, 64, 1, dav=dav, dav_shared=davs)
    assert abs(rep["energy"] - w[0]) < 1e-9 * abs(w[0])
    mps.free()


def test_full_size_cylinder_8x4_m1024(ctx):
    """Random state on the 8x4 cylinder's binomial bonds at m = 1024: the
    conversion keeps the energy and leaves sampled sites orthogonality
    centres; site values against the oracle on the GPU's tensors; the
    D_x-type exchanges of the centre column (snake distance up to 2 Ly - 1)
    against the oracle on the GPU's tensors; the sum over all Hamiltonian
    bonds equals the energy."""
    Lx, Ly = 8, 4
    N = Lx * Ly
    bonds, sites = synth.random_mps(N, 1024, 71)
    mpo = pl.Mpo("square", Lx, Ly, (1.0, 1.0))
    mps = pl.Mps(ctx, bonds, sites, PQ, 0)
    E0 = mps.energy(mpo)
    mps.inverse_canonical()
    E1 = mps.energy(mpo)
    assert abs(E1 - E0) < 1e-10 * max(1.0, abs(E0))
    ic_g = gpu_ic(mps)
    res = gauge.oc_residuals(ic_g)
    say("8x4 m1024 OC residual max", max(res), "E", E0, E1)
    assert max(res) < 1e-10
    sz = mps.expect_site(OPS["Sz"])
    want = np.array([gauge.expect_site(ic_g, j, OPS["Sz"]) for j in range(N)])
    assert np.max(np.abs(sz - want)) < 1e-12
    x = Lx // 2
    sample = [(models.snake_site(x, y, Ly), models.snake_site(x + 1, y, Ly)) for y in (0, Ly - 1)]
    sample = [(min(a, b), max(a, b)) for a, b in sample]
    got = mps.expect_pairs(EXCHANGE, sample)
    for (i, k), g in zip(sample, got):
        o = gauge.correlator(ic_g, i, k, EXCHANGE)
        say("8x4 pair", (i, k), g, o)
        assert abs(g - o) < 1e-11
    hb = [(min(i, k), max(i, k)) for i, k in models.square_cylinder_bonds(Lx, Ly)]
    tot = mps.expect_pairs(EXCHANGE, hb).sum()
    say("8x4 sum over bonds", tot, "energy", E1)
    assert abs(tot - E1) < 1e-10 * max(1.0, abs(E1))
    mps.free()
