"""Tile-shape autotuning of H_eff plans (grouped-GEMM shapes and split-K
chosen by timing): results stay those of the cost-model plan."""
import numpy as np
import pytest

from helpers import dev, say

pytestmark = pytest.mark.gpu


def _apply(pl, torch, level, prec, case):
    ctx = pl.Context(0)
    pl.set_autotune(ctx, level)
    B1, B2, P, W1, W2, L, R, x = case
    op = pl.Heff(ctx, B1, B2, P, W1, W2, L, R, prec)
    y = torch.empty_like(x)
    op.apply(x, y)
    op.apply(x, y)          # second apply reuses the tuned plan
    torch.cuda.synchronize()
    op.free()
    ctx.close()
    return y.cpu().numpy()


@pytest.fixture(scope="module")
def case():
    import torch
    from paper_1301_3494_amd import _lib as pl, synth
    rng = np.random.default_rng(7)
    PQ = (-1, 1)
    mpo = pl.Mpo("square", 4, 4, (1.0, 1.0))
    bonds = synth.binomial_bonds(16, 96)
    c = 7
    B1, B2, P = pl.Bond(bonds[c]), pl.Bond(bonds[c + 2]), pl.Phys(PQ)
    W1, W2 = mpo.site(c), mpo.site(c + 1)
    _, nL = pl.layout(pl.ENV_L, B1, deltas=mpo.deltas[c])
    _, nR = pl.layout(pl.ENV_R, B2, deltas=mpo.deltas[c + 2])
    _, nX = pl.layout(pl.TWO_SITE, B1, B2, P)
    L = dev(rng.standard_normal(nL) / np.sqrt(nL) * 30)
    R = dev(rng.standard_normal(nR) / np.sqrt(nR) * 30)
    x = dev(rng.standard_normal(nX))
    return (B1, B2, P, W1, W2, L, R, x)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
def test_autotuned_heff_matches_model_plan(case, prec):
    import torch
    from paper_1301_3494_amd import _lib as pl
    say(f"autotune heff prec={prec}")
    p = pl.PREC_NAMES[prec]
    y0 = _apply(pl, torch, 0, pl.PREC_NAMES["f64"], case)
    y1 = _apply(pl, torch, 1, p, case)
    y2 = _apply(pl, torch, 1, p, case)     # cache hit: same shapes, same bits
    assert np.array_equal(y1, y2)
    tol = {"f64": 1e-12, "f32": 1e-5, "bf16x3": 1e-5}[prec]
    assert np.linalg.norm(y1 - y0) <= tol * np.linalg.norm(y0)
