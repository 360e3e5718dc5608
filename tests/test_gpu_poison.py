"""The library with every device buffer NaN-filled as it is handed out
(pdmrg_set_alloc_poison): a kernel that reads memory nothing wrote would
turn the results below into NaN.  Davidson (FP64 and mixed precision),
serial and region-parallel sweeps, the inverse canonical gauge with local
measurements and an H_eff product, each against exact or oracle values."""
import numpy as np
import pytest

from helpers import pl, synth, say, golden, dense_state, dense_exchange
from oracle import models, mpo as M, gauge
from oracle.blocks import Bond

pytestmark = pytest.mark.gpu
E_ED_CHAIN16 = golden("heisenberg_chain_N16_J1_E0")


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    pl.set_alloc_poison(True)
    c = pl.Context(0)
    yield c
    c.close()
    pl.set_alloc_poison(False)


@pytest.mark.parametrize("prec,nreg", [(pl.F64, 1), (pl.F64, 2), (pl.F32, 2)])
def test_sweeps_reach_ed_with_poisoned_memory(ctx, prec, nreg):
    N = 16
    bonds, sites = synth.random_mps(N, 16, 1)
    mpo = pl.Mpo("chain", N, 1, (1.0, 1.0))
    mps = pl.Mps(ctx, bonds, sites, (-1, 1), 0)
    E = []
    for k in range(5):
        rep = mps.sweep(mpo, 64, 1 if k == 0 else nreg, prec=prec, dav=pl.dav_params(30, 8, 1e-11),
                        dav_shared=pl.dav_params(40, 8, 1e-11))
        E.append(rep["energy"])
    mps.free()
    say("poisoned sweeps prec", prec, "regions", nreg, E)
    assert np.all(np.isfinite(E))
    assert abs(E[-1] - E_ED_CHAIN16) <= 1e-9 * abs(E_ED_CHAIN16)


def test_gauge_measurements_with_poisoned_memory(ctx):
    N, m = 10, 12
    PQ = models.SPIN_HALF_Q
    bonds, sites = synth.random_mps(N, m, 41)
    omp = M.build_mpo(models.heisenberg_terms(models.chain_bonds(N)), N, models.OPS, PQ)
    mps = pl.Mps(ctx, bonds, sites, PQ, 0)
    assert mps.inverse_canonical() == 0
    ic_o = gauge.inverse_canonical(omp, bonds, sites, 0)
    ref = dense_state(sites, [Bond(b) for b in bonds], N)
    ref /= np.linalg.norm(ref)
    pairs = [(0, 1), (2, 5), (0, 9), (6, 8)]
    got = mps.expect_pairs(gauge.heisenberg_exchange(models.OPS), pairs)
    dense = np.array([dense_exchange(ref, N, i, k) for i, k in pairs])
    sz = mps.expect_site(models.OPS["Sz"])
    want = np.array([gauge.expect_site(ic_o, j, models.OPS["Sz"]) for j in range(N)])
    mps.free()
    assert np.max(np.abs(got - dense)) < 1e-12
    assert np.max(np.abs(sz - want)) < 1e-12
