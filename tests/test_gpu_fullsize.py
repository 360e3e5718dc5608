"""Parity at the full size of the metric's bond (8 x 4 cylinder, m = 1024,
sites 15 and 16, D = 14, 586,150 psi elements) in the configuration the
benchmark times (autotuned tile shapes and split-K), all three precisions,
against the oracle's complete H_eff product."""
import numpy as np
import pytest

from helpers import pl, synth, say, dev, host, blocks_to_flat, flat_to_blocks, tables, mpo_site, rel_err
from oracle import models, mpo as M, dmrg
from oracle.blocks import Bond, two_site_keys, two_site_shape, flatten

pytestmark = pytest.mark.gpu
PQ = synth.SPIN_HALF_Q


@pytest.fixture(scope="module")
def problem():
    Lx, Ly, m, c, seed = 8, 4, 1024, 15, 2
    N = Lx * Ly
    mpo = M.build_mpo(models.heisenberg_terms(models.square_cylinder_bonds(Lx, Ly)), N, models.OPS, PQ)
    bonds = synth.binomial_bonds(N, m)
    rng = np.random.default_rng(seed)
    L = synth.random_env_blocks(bonds[c], mpo.deltas[c], rng)
    R = synth.random_env_blocks(bonds[c + 2], mpo.deltas[c + 2], rng)
    psi = synth.random_two_site_blocks(bonds[c], bonds[c + 2], PQ, rng)
    bl, br = Bond(bonds[c]), Bond(bonds[c + 2])
    yref = dmrg.heff_apply(L, R, mpo.W[c], mpo.W[c + 1], psi, bl, br, PQ, mpo.deltas[c], mpo.deltas[c + 2])
    keys = two_site_keys(bl, br, PQ)
    shapes = [two_site_shape(k, bl, br, PQ) for k in keys]
    return dict(mpo=mpo, bonds=bonds, c=c, L=L, R=R, psi=psi, yref=flatten(yref, keys, shapes), keys=keys,
                shapes=shapes)


@pytest.fixture(scope="module")
def ctx():
    c = pl.Context(0)
    pl.set_autotune(c, 1)
    yield c
    c.close()


@pytest.mark.parametrize("prec,tol", [(pl.F64, 1e-12), (pl.F32, 1e-5), (pl.BF16X3, 1e-4)])
def test_full_size_heff_matches_oracle(ctx, problem, prec, tol):
    P = problem
    mpo, bonds, c = P["mpo"], P["bonds"], P["c"]
    say("full-size heff prec", prec)
    t, (B1, B2, Ph) = tables(bonds[c], bonds[c + 2], PQ, mpo.deltas[c], mpo.deltas[c + 2])
    Ld = dev(blocks_to_flat(P["L"], t["L"][0], t["L"][1], pl.ENV_L))
    Rd = dev(blocks_to_flat(P["R"], t["R"][0], t["R"][1], pl.ENV_R))
    op = pl.Heff(ctx, B1, B2, Ph, mpo_site(mpo, c), mpo_site(mpo, c + 1), Ld, Rd, prec)
    info = op.info()
    assert info["n_psi"] == 586150
    x = dev(blocks_to_flat(P["psi"], t["x"][0], t["x"][1], pl.TWO_SITE))
    y = dev(np.full(t["x"][1], np.nan))
    op.apply(x, y)
    a = flatten(flat_to_blocks(host(y), t["x"][0], pl.TWO_SITE), P["keys"], P["shapes"])
    b = P["yref"]
    err = rel_err(a, b)
    say("  plan", {k: info[k] for k in ("shape_Lpsi", "shape_R", "splitk_parts")}, "rel err", err)
    assert np.all(np.isfinite(a))
    assert err <= tol
    if prec == pl.F64:
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))
    # repeated application gives the same bits
    y2 = dev(np.full(t["x"][1], np.nan))
    op.apply(x, y2)
    assert np.array_equal(host(y), host(y2))
    op.free()


@pytest.mark.parametrize("prec,tol", [(pl.F32, 1e-5), (pl.F64, 1e-12)])
@pytest.mark.parametrize("shape", [8, 9, 10])
def test_full_size_lds_dma_shapes(ctx, problem, shape, prec, tol, tmp_path):
    """The LDS-DMA tiles (128x32, 64x64, 32x128) in FP32 and FP64, forced for
    both stages with 8 K parts at the full-size bond, against the oracle."""
    P = problem
    mpo, bonds, c = P["mpo"], P["bonds"], P["c"]
    t, (B1, B2, Ph) = tables(bonds[c], bonds[c + 2], PQ, mpo.deltas[c], mpo.deltas[c + 2])
    Ld = dev(blocks_to_flat(P["L"], t["L"][0], t["L"][1], pl.ENV_L))
    Rd = dev(blocks_to_flat(P["R"], t["R"][0], t["R"][1], pl.ENV_R))
    W1, W2 = mpo_site(mpo, c), mpo_site(mpo, c + 1)
    pl.Heff(ctx, B1, B2, Ph, W1, W2, Ld, Rd, prec).free()      # this operator's tuning entry
    f0, f = tmp_path / "tuned.tsv", tmp_path / "plans.tsv"
    pl.autotune_export(str(f0))
    keys = [r.split("\t")[0] for r in f0.read_text().splitlines() if r and r.split("|")[1] == str(prec)]
    f.write_text("".join("%s\t%d\t%d\t8\n" % (k, shape, shape) for k in keys))
    pl.autotune_import(str(f))
    op = pl.Heff(ctx, B1, B2, Ph, W1, W2, Ld, Rd, prec)
    info = op.info()
    assert info["shape_Lpsi"] == info["shape_R"] and info["shape_R"].endswith("dma")
    x = dev(blocks_to_flat(P["psi"], t["x"][0], t["x"][1], pl.TWO_SITE))
    y = dev(np.full(t["x"][1], np.nan))
    op.apply(x, y)
    a = flatten(flat_to_blocks(host(y), t["x"][0], pl.TWO_SITE), P["keys"], P["shapes"])
    err = rel_err(a, P["yref"])
    say("  forced", info["shape_R"], "prec", prec, "parts", info["splitk_parts"], "rel err", err)
    assert np.all(np.isfinite(a))
    assert err <= tol
    if prec == pl.F64:
        assert np.max(np.abs(a - P["yref"])) <= 1e-12 * np.max(np.abs(P["yref"]))
    op.free()
    pl.autotune_import(str(f0))   # the tuned plans again


CONFIGS = {
    # name: (lattice for mpo_build, oracle terms, Lx, Ly, couplings, m)
    "cyl24x8_m2000": ("square", lambda: models.heisenberg_terms(models.square_cylinder_bonds(24, 8)), 24, 8,
                      (1.0, 1.0), 2000),
    "tri12x6_m3000": ("triangular", lambda: models.xxz_terms(models.triangular_cylinder_bonds(12, 6), 1.0, 1.0),
                      12, 6, (1.0, 1.0), 3000),
    "jq2_16x8_m4000": ("jq2", lambda: models.jq2_terms(16, 8, 1.0, 1.0), 16, 8, (1.0, 1.0), 4000),
}


@pytest.mark.parametrize("name", list(CONFIGS))
def test_large_config_heff_sampled_rows(name):
    """H_eff at the centre bond of the larger configurations (24 x 8 cylinder
    m = 2000, triangular 12 x 6 m = 3000, J-Q2 16 x 8 m = 4000), FP64 and FP32,
    with the plans sweeps use (cost model): sampled output rows against the
    oracle computed row by row."""
    import torch
    lattice, terms_fn, Lx, Ly, couplings, m = CONFIGS[name]
    N = Lx * Ly
    c = N // 2 - 1
    say("large config", name)
    omp = M.build_mpo(terms_fn(), N, models.OPS, PQ)
    # the library's own MPO has the same bond dimensions (its channel order
    # may differ); both sides contract the oracle's W with the same inputs
    gmp = pl.Mpo(lattice, Lx, Ly, couplings)
    assert [w.shape for w in gmp.W] == [w.shape for w in omp.W]
    gmp.free()
    bonds = synth.binomial_bonds(N, m)
    rng = np.random.default_rng(3)
    L = synth.random_env_blocks(bonds[c], omp.deltas[c], rng)
    R = synth.random_env_blocks(bonds[c + 2], omp.deltas[c + 2], rng)
    psi = synth.random_two_site_blocks(bonds[c], bonds[c + 2], PQ, rng)
    t, (B1, B2, P) = tables(bonds[c], bonds[c + 2], PQ, omp.deltas[c], omp.deltas[c + 2])
    Ld = dev(blocks_to_flat(L, t["L"][0], t["L"][1], pl.ENV_L))
    Rd = dev(blocks_to_flat(R, t["R"][0], t["R"][1], pl.ENV_R))
    x = dev(blocks_to_flat(psi, t["x"][0], t["x"][1], pl.TWO_SITE))
    bl, br = Bond(bonds[c]), Bond(bonds[c + 2])
    keys = sorted(psi, key=lambda k: -psi[k].size)[:2] + [sorted(psi, key=lambda k: psi[k].size)[0]]
    table = {k: (off, rows, cols, ld) for k, off, rows, cols, ld in t["x"][0]}
    ref = {}
    for k in keys:
        rows = sorted({0, psi[k].shape[0] // 2, psi[k].shape[0] - 1})
        ref[k] = (rows, dmrg.heff_apply_rows(L, R, omp.W[c], omp.W[c + 1], psi, bl, br, PQ, omp.deltas[c],
                                             omp.deltas[c + 2], k, rows))
    ctx = pl.Context(0)
    for prec, tol in ((pl.F64, 1e-12), (pl.F32, 1e-5), (pl.BF16X3, 1e-4)):
        op = pl.Heff(ctx, B1, B2, P, mpo_site(omp, c), mpo_site(omp, c + 1), Ld, Rd, prec)
        y = torch.full_like(x, float("nan"))
        op.apply(x, y)
        yh = host(y)
        num = den = 0.0
        for k in keys:
            off, rows_k, cols, ld = table[k]
            rows, want = ref[k]
            got = np.stack([yh[off + r * ld: off + r * ld + cols] for r in rows])
            assert np.all(np.isfinite(got))
            num += float(np.sum((got - want) ** 2))
            den += float(np.sum(want ** 2))
        err = np.sqrt(num / den)
        say("  prec", prec, "sampled rel err", err, "flops", op.info()["flops"])
        assert err <= tol
        assert np.all(np.isfinite(yh))
        op.free()
    ctx.close()
