"""Degenerate and boundary cases on the GPU: H_eff at the outer bonds of a
chain (one-state boundary bonds, tiny ragged blocks) in every precision and
in the forced LDS-DMA tile shapes against the oracle; sweeps of a two-site
chain (the singlet), of the fully polarised sector (one state per bond) and
of a sector with nonzero total S^z, against closed forms and exact
diagonalisation."""
import numpy as np
import pytest

from helpers import (pl, synth, tables, blocks_to_flat, flat_to_blocks, mpo_site, rel_err, dev, host, say)
from oracle import models, mpo as M, dmrg, exact
from oracle.blocks import Bond, two_site_keys, two_site_shape, flatten

pytestmark = pytest.mark.gpu
PQ = (-1, 1)


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = pl.Context(0)
    yield c
    c.close()


def _force_shape(ctx, make_op, prec, shape, parts, tmp_path):
    """Build the operator once to create its tuning entry, then force `shape`
    for both stages with `parts` K parts through an imported entry."""
    pl.set_autotune(ctx, 1)
    make_op().free()
    f0, f = tmp_path / "tuned.tsv", tmp_path / "forced.tsv"
    pl.autotune_export(str(f0))
    keys = [r.split("\t")[0] for r in f0.read_text().splitlines() if r and r.split("|")[1] == str(prec)]
    f.write_text("".join("%s\t%d\t%d\t%d\n" % (k, shape, shape, parts) for k in keys))
    pl.autotune_import(str(f))
    op = make_op()
    pl.autotune_import(str(f0))
    pl.set_autotune(ctx, 0)
    return op


@pytest.mark.parametrize("prec,tol", [(pl.F64, 1e-12), (pl.F32, 1e-5), (pl.BF16X3, 1e-4)])
@pytest.mark.parametrize("where", ["left", "right", "next_to_left"])
@pytest.mark.parametrize("shape", [None, 9])
def test_heff_at_chain_edges(ctx, prec, tol, where, shape, tmp_path):
    N, m, seed = 10, 16, 3
    mpo = M.build_mpo(models.heisenberg_terms(models.chain_bonds(N)), N, models.OPS, PQ)
    bonds = synth.binomial_bonds(N, m)
    i = {"left": 0, "right": N - 2, "next_to_left": 1}[where]
    rng = np.random.default_rng(seed + i)
    L = synth.random_env_blocks(bonds[i], mpo.deltas[i], rng)
    R = synth.random_env_blocks(bonds[i + 2], mpo.deltas[i + 2], rng)
    psi = synth.random_two_site_blocks(bonds[i], bonds[i + 2], PQ, rng)
    bl, br = Bond(bonds[i]), Bond(bonds[i + 2])
    yref = dmrg.heff_apply(L, R, mpo.W[i], mpo.W[i + 1], psi, bl, br, PQ, mpo.deltas[i], mpo.deltas[i + 2])
    t, (B1, B2, P) = tables(bonds[i], bonds[i + 2], PQ, mpo.deltas[i], mpo.deltas[i + 2])
    Ld = dev(blocks_to_flat(L, t["L"][0], t["L"][1], pl.ENV_L))
    Rd = dev(blocks_to_flat(R, t["R"][0], t["R"][1], pl.ENV_R))
    make = lambda: pl.Heff(ctx, B1, B2, P, mpo_site(mpo, i), mpo_site(mpo, i + 1), Ld, Rd, prec)
    op = make() if shape is None else _force_shape(ctx, make, prec, shape, 3, tmp_path)
    info = op.info()
    x = dev(blocks_to_flat(psi, t["x"][0], t["x"][1], pl.TWO_SITE))
    y = dev(np.full(t["x"][1], np.nan))
    op.apply(x, y)
    keys = two_site_keys(bl, br, PQ)
    shapes = [two_site_shape(k, bl, br, PQ) for k in keys]
    a = flatten(flat_to_blocks(host(y), t["x"][0], pl.TWO_SITE), keys, shapes)
    b = flatten(yref, keys, shapes)
    err = rel_err(a, b)
    say("edge heff", where, "prec", prec, "plan", info["shape_Lpsi"], info["shape_R"], "n", len(a), "rel err", err)
    op.free()
    assert np.all(np.isfinite(a))
    assert err <= tol


def test_two_site_chain_is_the_singlet(ctx):
    """N = 2: one two-site update holds the whole state; E = -3/4."""
    mpo = pl.Mpo("chain", 2, 1, (1.0, 1.0))
    bonds, sites = synth.random_mps(2, 4, 1)
    mps = pl.Mps(ctx, bonds, sites, PQ, 0)
    E = [mps.sweep(mpo, 4, 1)["energy"] for _ in range(2)]
    mps.free()
    say("two-site chain", E)
    assert abs(E[-1] + 0.75) < 1e-12


@pytest.mark.parametrize("n_regions", [1, 2])
def test_fully_polarised_sector(ctx, n_regions):
    """2 S^z = N: a single basis state, every bond one state; E = (N - 1)/4
    for the open Heisenberg chain."""
    N = 12
    mpo = pl.Mpo("chain", N, 1, (1.0, 1.0))
    bonds, sites = synth.random_mps(N, 8, 2, q_target=N)
    assert all(sum(b.values()) == 1 for b in bonds)
    mps = pl.Mps(ctx, bonds, sites, PQ, N)
    E = [mps.sweep(mpo, 8, 1 if k == 0 else n_regions)["energy"] for k in range(3)]
    mps.free()
    say("polarised", n_regions, E)
    assert abs(E[-1] - (N - 1) / 4) < 1e-12


def test_nonzero_sector_matches_ed(ctx):
    """2 S^z = 4 on the open chain of 14 sites, two regions: the sector's
    ground-state energy by exact diagonalisation."""
    N, q = 14, 4
    mpo = pl.Mpo("chain", N, 1, (1.0, 1.0))
    w, _, _ = exact.ground_state(models.heisenberg_terms(models.chain_bonds(N)), N, q)
    bonds, sites = synth.random_mps(N, 16, 3, q_target=q)
    mps = pl.Mps(ctx, bonds, sites, PQ, q)
    dav, davs = pl.dav_params(30, 8, 1e-11), pl.dav_params(40, 8, 1e-11)
    E = [mps.sweep(mpo, 64, 1 if k == 0 else 2, dav=dav, dav_shared=davs)["energy"] for k in range(5)]
    mps.free()
    say("sector q=4", E, "ED", w[0])
    assert abs(E[-1] - w[0]) < 1e-9 * abs(w[0])
