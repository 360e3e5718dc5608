"""Backward kernel: dE/dW at fixed state (grad_site, grad_mpo) against the
oracle's site gradient, exact Hellmann-Feynman values from exact
diagonalisation, the TFIM closed form, homogeneity, and the torch.autograd
route."""
import numpy as np
import pytest

from helpers import pl, synth, say, dev, host, blocks_to_flat
from oracle import models, mpo as M, exact, grad as ograd

pytestmark = pytest.mark.gpu
PQ = synth.SPIN_HALF_Q


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = pl.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("m,i,seed", [(40, 5, 11), (150, 7, 12)])
def test_grad_site_matches_oracle(ctx, m, i, seed):
    say("grad_site m", m, "site", i)
    Lx, Ly = 4, 4
    N = Lx * Ly
    mpo = M.build_mpo(models.heisenberg_terms(models.square_cylinder_bonds(Lx, Ly)), N, models.OPS, PQ)
    bonds = synth.binomial_bonds(N, m)
    bl, br = bonds[i], bonds[i + 1]
    rng = np.random.default_rng(seed)
    psi = synth.random_site_blocks(bl, br, PQ, rng)
    L = synth.random_env_blocks(bl, mpo.deltas[i], rng)
    R = synth.random_env_blocks(br, mpo.deltas[i + 1], rng)
    ref = ograd.site_gradient(L, R, psi, PQ, mpo.deltas[i], mpo.deltas[i + 1])
    B1, B2, P = pl.Bond(bl), pl.Bond(br), pl.Phys(PQ)
    tS, nS = pl.layout(pl.SITE, B1, B2, P)
    tL, nL = pl.layout(pl.ENV_L, B1, deltas=mpo.deltas[i])
    tR, nR = pl.layout(pl.ENV_R, B2, deltas=mpo.deltas[i + 1])
    W = pl.MpoSite(mpo.W[i], mpo.deltas[i], mpo.deltas[i + 1])
    G = pl.grad_site(ctx, B1, B2, P, W, dev(blocks_to_flat(L, tL, nL, pl.ENV_L)),
                     dev(blocks_to_flat(psi, tS, nS, pl.SITE)), dev(blocks_to_flat(R, tR, nR, pl.ENV_R)))
    got = host(G)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
    # entries the charges forbid are exactly zero on both sides
    assert np.array_equal(got == 0.0, ref == 0.0)
    # deterministic: a second call gives the same bits
    assert np.array_equal(host(pl.grad_site(ctx, B1, B2, P, W, dev(blocks_to_flat(L, tL, nL, pl.ENV_L)),
                                            dev(blocks_to_flat(psi, tS, nS, pl.SITE)),
                                            dev(blocks_to_flat(R, tR, nR, pl.ENV_R)))), got)


def _converged(ctx, lattice, Lx, Ly, couplings, m, sweeps, phys=PQ, q=0, n_regions=1, seed=1):
    N = Lx * Ly
    bonds, sites = synth.random_mps(N, min(m, 16), seed, phys_q=phys, q_target=q)
    mpo = pl.Mpo(lattice, Lx, Ly, couplings)
    mps = pl.Mps(ctx, bonds, sites, phys, q)
    for k in range(sweeps):
        nreg = 1 if k < 2 else n_regions
        rep = mps.sweep(mpo, m, nreg, dav=pl.dav_params(30, 8, 1e-11), dav_shared=pl.dav_params(40, 8, 1e-11))
    return mps, mpo, rep["energy"]


def test_grad_mpo_xxz_hellmann_feynman_vs_ed(ctx):
    N, Delta = 10, 0.9
    mps, mpo, E = _converged(ctx, "chain", N, 1, (1.0, Delta), 64, 5)
    Eg, (gJ, gD) = pl.dE_dcouplings(mps, mpo)
    terms = models.xxz_terms(models.chain_bonds(N), 1.0, Delta)
    e, v, _ = exact.ground_state(terms, N, 0)
    Hd, _ = exact.sparse_hamiltonian([(1.0, ((i, "Sz"), (j, "Sz"))) for i, j in models.chain_bonds(N)], N, 0)
    hf = float(v[:, 0] @ (Hd @ v[:, 0]))
    say("xxz dE/dDelta gpu", gD, "ED", hf, "E", Eg, e[0])
    assert abs(Eg - e[0]) <= 1e-9 * abs(e[0])
    assert abs(gD - hf) <= 1e-9 * max(1.0, abs(hf))
    # homogeneity of the XXZ energy in J at fixed Delta: J dE/dJ = E
    assert abs(1.0 * gJ - Eg) <= 1e-9 * abs(Eg)


def test_grad_mpo_tfim_closed_form(ctx):
    N, h = 10, 0.8
    mps, mpo, E = _converged(ctx, "tfim", N, 1, (1.0, h), 64, 5, phys=synth.TRIVIAL_Q)
    Eg, (gJ, gh) = pl.dE_dcouplings(mps, mpo)
    ref = exact.tfim_chain_dE_dh(N, 1.0, h)
    say("tfim dE/dh gpu", gh, "closed form", ref)
    assert abs(Eg - exact.tfim_chain_energy(N, 1.0, h)) <= 1e-9 * abs(Eg)
    assert abs(gh - ref) <= 1e-8 * max(1.0, abs(ref))
    assert abs(gJ * 1.0 + gh * h - Eg) <= 1e-8 * abs(Eg)


def test_grad_mpo_after_parallel_sweeps_homogeneity(ctx):
    """Heisenberg J = 1.3 on a 12-site chain swept with 2 regions (V on the
    shared bond): dE/dJ = E/J."""
    N, J = 12, 1.3
    mps, mpo, E = _converged(ctx, "chain", N, 1, (J, 1.0), 64, 5, n_regions=2)
    Eg, (gJ, gD) = pl.dE_dcouplings(mps, mpo)
    say("homogeneity E", Eg, "J dE/dJ", J * gJ)
    assert abs(Eg - E) <= 1e-10 * abs(E)
    assert abs(J * gJ - Eg) <= 1e-9 * abs(Eg)
    # SU(2) point: the S^z S^z part carries one third of the energy
    assert abs(gD - Eg / 3.0) <= 1e-7 * abs(Eg)


def test_autograd_function_matches_grad_mpo(ctx):
    import torch
    N = 8
    mps, mpo, E = _converged(ctx, "chain", N, 1, (1.0, 1.0), 16, 4)
    W = [torch.tensor(w, dtype=torch.float64, requires_grad=True) for w in mpo.W]
    Et = pl.mpo_energy(mps, mpo.deltas, W)
    Et.backward()
    _, G = mps.gradients(mpo)
    assert abs(float(Et.detach()) - E) <= 1e-10 * abs(E)
    for w, g in zip(W, G):
        assert torch.allclose(w.grad, g.cpu(), rtol=1e-11, atol=1e-13)
    # each site's G contracted with its own W gives the energy
    assert abs(float(np.sum(W[3].grad.numpy() * mpo.W[3])) - E) <= 1e-10 * abs(E)


def test_triangular_xxz_dE_dDelta_vs_ed_and_finite_difference(ctx):
    """Triangular-lattice XXZ cylinder (the backward kernel's workload, at a
    size exact diagonalisation covers): grad_mpo's dE/dDelta against the exact
    Hellmann-Feynman value and against central differences of converged GPU
    energies (h = 1e-4)."""
    Lx, Ly, Delta, h = 4, 3, 0.9, 1e-4
    N = Lx * Ly
    mps, mpo, E = _converged(ctx, "triangular", Lx, Ly, (1.0, Delta), 200, 6)
    Eg, (gJ, gD) = pl.dE_dcouplings(mps, mpo)
    bonds = models.triangular_cylinder_bonds(Lx, Ly)
    e, v, _ = exact.ground_state(models.xxz_terms(bonds, 1.0, Delta), N, 0)
    Hzz, _ = exact.sparse_hamiltonian([(1.0, ((i, "Sz"), (j, "Sz"))) for i, j in bonds], N, 0)
    hf = float(v[:, 0] @ (Hzz @ v[:, 0]))
    Ep = _converged(ctx, "triangular", Lx, Ly, (1.0, Delta + h), 200, 6)[2]
    Em = _converged(ctx, "triangular", Lx, Ly, (1.0, Delta - h), 200, 6)[2]
    fd = (Ep - Em) / (2 * h)
    say("triangular dE/dDelta grad", gD, "ED", hf, "FD", fd, "E", Eg, e[0])
    assert abs(Eg - e[0]) <= 1e-9 * abs(e[0])
    assert abs(gD - hf) <= 1e-8 * max(1.0, abs(hf))
    assert abs(gD - fd) <= 1e-6 * max(1.0, abs(fd))
    assert abs(gJ - Eg) <= 1e-8 * abs(Eg)        # E is linear in J at fixed Delta


def test_jq2_homogeneity_on_gpu(ctx):
    """J-Q2 cylinder: J dE/dJ + Q dE/dQ = E (degree-1 homogeneity), with E
    equal to exact diagonalisation."""
    Lx, Ly, J, Q = 3, 3, 1.0, 0.6
    N = Lx * Ly
    mps, mpo, E = _converged(ctx, "jq2", Lx, Ly, (J, Q), 200, 6, q=1)
    Eg, (gJ, gQ) = pl.dE_dcouplings(mps, mpo)
    e = exact.ground_state(models.jq2_terms(Lx, Ly, J, Q), N, 1)[0][0]
    say("jq2 E", Eg, "ED", e, "J gJ + Q gQ", J * gJ + Q * gQ)
    assert abs(Eg - e) <= 1e-9 * abs(e)
    assert abs(J * gJ + Q * gQ - Eg) <= 1e-9 * abs(Eg)


def test_triangular_12x6_su2_identity_and_finite_difference(ctx):
    """The triangular study's cylinder at its own size (12 x 6, D = 23) at
    reduced bond dimension (m ramped to 512, 8 sweeps).  At Delta = 1 the
    Hamiltonian is SU(2) invariant and a singlet ground state carries a third
    of its energy in the S^z S^z part, dE/dDelta = E/3; the truncated MPS
    breaks the symmetry slightly (measured 8e-4 relative at m = 512, 2.4e-3 at
    m = 256), so the identity is held to 2e-3.  grad_couplings' dE/dDelta
    against (a) the central difference (h = 1e-4) of <Psi|H(Delta +- h)|Psi>
    on the same state, which the Hellmann-Feynman value must equal up to
    rounding (E is linear in Delta at fixed state: 1e-8 relative), and (b) the
    central difference of the energies after three more sweeps at
    Delta = 1 +- h from device copies of the state, the envelope-theorem check,
    limited by how far the m = 512 sweeps still move the state (measured
    1.8e-4 relative after four sweeps at m = 512, 6e-6 after nine; held to
    5e-4)."""
    Lx, Ly, h = 12, 6, 1e-4
    N = Lx * Ly
    bonds, sites = synth.random_mps(N, 16, 5)
    mpo = pl.Mpo("triangular", Lx, Ly, (1.0, 1.0))
    mps = pl.Mps(ctx, bonds, sites)
    dav, davs = pl.dav_params(30, 8, 1e-11), pl.dav_params(40, 8, 1e-11)
    for m in (64, 128, 256, 256, 512, 512, 512, 512):
        E = mps.sweep(mpo, m, 1, dav=dav, dav_shared=davs)["energy"]
    base = mps.copy()
    Eg, (gJ, gD) = pl.dE_dcouplings(mps, mpo)
    Es = []
    for sgn in (+1, -1):
        st = base.copy()
        mh = pl.Mpo("triangular", Lx, Ly, (1.0, 1.0 + sgn * h))
        for _ in range(3):
            e = st.sweep(mh, 512, 1, dav=dav, dav_shared=davs)["energy"]
        Es.append(e)
        st.free()
        mh.free()
    base.free()
    fd = (Es[0] - Es[1]) / (2 * h)
    Ef = []
    for sgn in (+1, -1):
        mh = pl.Mpo("triangular", Lx, Ly, (1.0, 1.0 + sgn * h))
        Ef.append(mps.energy(mh))
        mh.free()
    fd_fixed = (Ef[0] - Ef[1]) / (2 * h)
    say("tri 12x6 m=512 E", Eg, "dE/dDelta", gD, "E/3", Eg / 3, "FD fixed state", fd_fixed, "FD converged", fd,
        "dE/dJ", gJ)
    assert abs(Eg - E) <= 1e-10 * abs(E)
    assert abs(gD - Eg / 3.0) <= 2e-3 * abs(Eg)
    assert abs(gD - fd_fixed) <= 1e-8 * abs(gD)
    assert abs(gD - fd) <= 5e-4 * abs(fd)
    assert abs(gJ - Eg) <= 1e-9 * abs(Eg)        # E is linear in J at fixed Delta
    mps.free()


def test_grad_couplings_rejects_mpo_without_tables(ctx):
    """An MPO from caller tensors (mpo_from_sites) carries no coupling
    tables: grad_couplings reports PDMRG_EINVAL."""
    mps, mpo, E = _converged(ctx, "chain", 6, 1, (1.0, 1.0), 16, 2)
    raw = pl.Mpo(sites=[mpo.site(i) for i in range(mpo.N)])
    raw.ncouplings = 2
    with pytest.raises(pl.PdmrgError):
        pl.dE_dcouplings(mps, raw)


def test_grad_per_site_identity_past_one_grid(ctx):
    """J-Q2 16 x 8 at m = 1200 (binomial bonds, seeded random state, D = 110):
    at the bonds next to the edges the measurement's block dot products take
    more tiles than one launch's grid (about 1.3e6 > 2^20), so the dot kernel
    walks them with a grid stride.  E is linear in every W_i, so each
    <G_i, W_i> equals E; a dropped or stale tile breaks it at that site."""
    Lx, Ly, m = 16, 8, 1200
    N = Lx * Ly
    mpo = pl.Mpo("jq2", Lx, Ly, (1.0, 1.0))
    bonds, sites = synth.random_mps(N, m, 6)
    mps = pl.Mps(ctx, bonds, sites)
    _, G = mps.gradients(mpo)
    E = mps.energy(mpo)   # of the re-gauged state (the random one's norm can overflow)
    gw = np.array([float(np.sum(G[i].cpu().numpy() * mpo.W[i])) for i in range(N)])
    bad = np.nonzero(np.abs(gw - E) > 1e-8 * abs(E))[0]
    say("E", E, "worst <G_i,W_i> rel", np.max(np.abs(gw - E)) / abs(E), "bad sites", bad[:8])
    assert len(bad) == 0
    mps.free()
