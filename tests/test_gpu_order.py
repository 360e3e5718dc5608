"""Sec. III pinning terms of mpo_build and the order parameters D_x and M_z
(mps_order_parameter) on the GPU, through the C ABI: the pinned MPOs give the
energies of the oracle's pinned term lists, and the order parameters of GPU
ground states match exact diagonalisation and the oracle evaluated on the
GPU's tensors."""
import numpy as np
import pytest

from helpers import pl, synth, say, mpo_site
from oracle import models, mpo as M, exact, gauge
from oracle.blocks import Bond

pytestmark = pytest.mark.gpu
OPS = models.OPS
PQ = models.SPIN_HALF_Q


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = pl.Context(0)
    yield c
    c.close()


def gpu_ic(mps):
    bonds = [Bond(mps.bond(b)) for b in range(mps.N + 1)]
    psi = [mps.site_blocks(j) for j in range(mps.N)]
    V = {b: mps.get_v(b) for b in range(1, mps.N)}
    lam = {b: {q: 1.0 / v for q, v in V[b].items()} for b in V}
    return gauge.InverseCanonical(bonds, psi, V, lam, PQ, 0)


def _ed_expect(obs, N, v):
    H1, _ = exact.sparse_hamiltonian(obs, N, 0)
    return float(v @ (H1 @ v))


CASES = {
    "jq2": dict(lattice="jq2", Lx=4, Ly=3, couplings=(0.2, 1.0, 1.0),
                terms=lambda: models.jq2_terms(4, 3, 0.2, 1.0, pin=1.0)),
    "tri": dict(lattice="triangular", Lx=4, Ly=3, couplings=(1.0, 1.0, 0.5),
                terms=lambda: models.heisenberg_terms(models.triangular_cylinder_bonds(4, 3))
                + models.triangular_pin_terms(4, 3, 0.5)),
}


@pytest.mark.parametrize("name", ["jq2", "tri"])
def test_pinned_mpo_matches_oracle_terms(ctx, name):
    c = CASES[name]
    N = c["Lx"] * c["Ly"]
    mpo = pl.Mpo(c["lattice"], c["Lx"], c["Ly"], c["couplings"])
    omp = M.build_mpo(c["terms"](), N, OPS, PQ)
    ompo = pl.Mpo(sites=[mpo_site(omp, i) for i in range(N)])
    bonds, sites = synth.random_mps(N, 12, 81)
    mps = pl.Mps(ctx, bonds, sites, PQ, 0)
    e1, e2 = mps.energy(mpo), mps.energy(ompo)
    say(name, "pinned MPO energies", e1, e2)
    assert abs(e1 - e2) < 1e-12 * max(1.0, abs(e2))
    mps.free()


@pytest.mark.parametrize("name", ["jq2", "tri"])
def test_order_parameter_of_ground_state(ctx, name):
    c = CASES[name]
    Lx, Ly = c["Lx"], c["Ly"]
    N = Lx * Ly
    w, v, _ = exact.ground_state(c["terms"](), N, 0)
    mpo = pl.Mpo(c["lattice"], Lx, Ly, c["couplings"])
    bonds, sites = synth.random_mps(N, 16, 83)
    mps = pl.Mps(ctx, bonds, sites, PQ, 0)
    dav = pl.dav_params(30, 10, 1e-11)
    for k in range(6):
        rep = mps.sweep(mpo, 64, 1 if k < 2 else 2, dav=dav, dav_shared=pl.dav_params(40, 10, 1e-12))
    assert abs(rep["energy"] - w[0]) < 1e-9 * abs(w[0])
    mps.inverse_canonical()
    ic = gpu_ic(mps)
    if name == "jq2":
        got = mps.order_parameter("Dx", Lx, Ly)
        orc = gauge.order_dx(ic, Lx, Ly, OPS, models.snake_site)
        xc = Lx // 2 - 1

        def bond(x, y):
            a, b = models.snake_site(x, y, Ly), models.snake_site(x + 1, y, Ly)
            return _ed_expect(models.heisenberg_terms([(min(a, b), max(a, b))]), N, v[:, 0])
        ed = sum(bond(xc, y) - 0.5 * bond(xc - 1, y) - 0.5 * bond(xc + 1, y) for y in range(Ly)) / Ly
    else:
        got = mps.order_parameter("Mz", Lx, Ly)
        orc = gauge.order_mz(ic, Lx, Ly, OPS, models.snake_site, models.tri_sublattice)
        xc = (Lx - 1) // 2
        vals = [_ed_expect([(1.0, ((models.snake_site(xc, y, Ly), "Sz"),))], N, v[:, 0])
                for y in range(Ly) if models.tri_sublattice(xc, y) == 0]
        ed = sum(vals) / len(vals)
    say(name, "order parameter gpu", got, "oracle on gpu tensors", orc, "ED", ed)
    assert abs(got - orc) < 1e-12
    assert abs(got - ed) < 1e-7
    mps.free()


def test_order_parameter_errors(ctx):
    bonds, sites = synth.random_mps(12, 8, 85)
    mps = pl.Mps(ctx, bonds, sites, PQ, 0)
    mps.inverse_canonical()
    with pytest.raises(pl.PdmrgError):
        mps.order_parameter("Dx", 3, 4)     # Lx < 4
    with pytest.raises(pl.PdmrgError):
        mps.order_parameter("Mz", 6, 2)     # Ly not a multiple of 3
    with pytest.raises(pl.PdmrgError):
        mps.order_parameter("Dx", 5, 3)     # Lx * Ly != N
    with pytest.raises(pl.PdmrgError):
        mps.order_parameter(7, 4, 3)
    with pytest.raises(pl.PdmrgError):
        pl.Mpo("triangular", 4, 4, (1.0, 1.0, 0.5))   # pinning needs Ly % 3 == 0
    mps.free()
