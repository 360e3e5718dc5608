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


@pytest.mark.parametrize("shape", [8, 9, 10])
def test_bf16x3_every_tile_shape(case, shape, tmp_path):
    """Each tile shape of the BF16x3 path (the LDS-DMA shapes 128x32, 64x64,
    32x128 on split operands), forced through an imported tuning entry, against
    the FP64 product."""
    import torch
    from paper_1301_3494_amd import _lib as pl
    B1, B2, P, W1, W2, L, R, x = case
    y0 = _apply(pl, torch, 0, pl.F64, case)
    ctx = pl.Context(0)
    pl.set_autotune(ctx, 1)
    pl.Heff(ctx, B1, B2, P, W1, W2, L, R, pl.BF16X3).free()      # creates this operator's entry
    f = tmp_path / "plans.tsv"
    pl.autotune_export(str(f))
    rows = [r.split("\t") for r in f.read_text().splitlines() if r]
    mine = [r[0] for r in rows if r[0].split("|")[1] == str(pl.BF16X3)]
    assert mine
    f.write_text("".join("%s\t%d\t%d\t%d\n" % (k, shape, shape, 2) for k in mine))
    pl.autotune_import(str(f))
    op = pl.Heff(ctx, B1, B2, P, W1, W2, L, R, pl.BF16X3)
    info = op.info()
    names = SHAPES
    say(f"bf16x3 forced shape {names[shape]}: plan {info['shape_Lpsi']} / {info['shape_R']}, parts {info['splitk_parts']}")
    assert info["shape_Lpsi"] == names[shape] and info["shape_R"] == names[shape]
    y = torch.empty_like(x)
    op.apply(x, y)
    torch.cuda.synchronize()
    y = y.cpu().numpy()
    op.free()
    ctx.close()
    err = np.linalg.norm(y - y0) / np.linalg.norm(y0)
    say(f"bf16x3 shape {names[shape]} rel err {err:.3e}")
    assert err <= 1e-5


SHAPES = ["64x64", "128x32", "32x128", "128x128", "64x64k16", "128x32k16", "64x64k8", "128x32k8",
          "128x32dma", "64x64dma", "32x128dma"]


@pytest.mark.parametrize("parts", [1, 3])
@pytest.mark.parametrize("shape", list(range(len(SHAPES))))
def test_f32_every_tile_shape(case, shape, parts, tmp_path):
    """Each FP32 tile shape (register-staged K steps of 32, 16 and 8; LDS-DMA
    pipelined steps of 16) for both stages, forced through an imported tuning
    entry, with and without split-K, against the FP64 product."""
    import torch
    from paper_1301_3494_amd import _lib as pl
    B1, B2, P, W1, W2, L, R, x = case
    y0 = _apply(pl, torch, 0, pl.F64, case)
    ctx = pl.Context(0)
    pl.set_autotune(ctx, 1)
    pl.Heff(ctx, B1, B2, P, W1, W2, L, R, pl.F32).free()      # creates this operator's entry
    f = tmp_path / "plans.tsv"
    pl.autotune_export(str(f))
    rows = [r.split("\t") for r in f.read_text().splitlines() if r]
    mine = [r[0] for r in rows if r[0].split("|")[1] == str(pl.F32)]
    assert mine
    f.write_text("".join("%s\t%d\t%d\t%d\n" % (k, shape, shape, parts) for k in mine))
    pl.autotune_import(str(f))
    op = pl.Heff(ctx, B1, B2, P, W1, W2, L, R, pl.F32)
    info = op.info()
    assert info["shape_Lpsi"] == SHAPES[shape] and info["shape_R"] == SHAPES[shape]
    y = torch.empty_like(x)
    op.apply(x, y)
    y1 = torch.empty_like(x)
    op.apply(x, y1)
    torch.cuda.synchronize()
    y, y1 = y.cpu().numpy(), y1.cpu().numpy()
    op.free()
    ctx.close()
    err = np.linalg.norm(y - y0) / np.linalg.norm(y0)
    say(f"f32 shape {SHAPES[shape]} parts {parts}: tiles {info['tiles_Lpsi']} / {info['tiles_R']}, rel err {err:.3e}")
    assert np.array_equal(y, y1)
    assert err <= 1e-5


@pytest.mark.parametrize("parts", [1, 3])
@pytest.mark.parametrize("shape", [8, 9, 10])
def test_f64_lds_dma_tile_shapes(case, shape, parts, tmp_path):
    """The LDS-DMA tile shapes in FP64, forced for both stages, against the
    cost-model FP64 plan (register-staged kernel) to 1e-12."""
    import torch
    from paper_1301_3494_amd import _lib as pl
    B1, B2, P, W1, W2, L, R, x = case
    y0 = _apply(pl, torch, 0, pl.F64, case)
    ctx = pl.Context(0)
    pl.set_autotune(ctx, 1)
    pl.Heff(ctx, B1, B2, P, W1, W2, L, R, pl.F64).free()
    f = tmp_path / "plans.tsv"
    pl.autotune_export(str(f))
    rows = [r.split("\t") for r in f.read_text().splitlines() if r]
    mine = [r[0] for r in rows if r[0].split("|")[1] == str(pl.F64)]
    assert mine
    f.write_text("".join("%s\t%d\t%d\t%d\n" % (k, shape, shape, parts) for k in mine))
    pl.autotune_import(str(f))
    op = pl.Heff(ctx, B1, B2, P, W1, W2, L, R, pl.F64)
    info = op.info()
    assert info["shape_Lpsi"] == SHAPES[shape] and info["shape_R"] == SHAPES[shape]
    y = torch.empty_like(x)
    op.apply(x, y)
    torch.cuda.synchronize()
    y = y.cpu().numpy()
    op.free()
    ctx.close()
    err = np.linalg.norm(y - y0) / np.linalg.norm(y0)
    say(f"f64 shape {SHAPES[shape]} parts {parts}: rel err {err:.3e}")
    assert err <= 1e-12
    assert np.max(np.abs(y - y0)) <= 1e-12 * np.max(np.abs(y0))
