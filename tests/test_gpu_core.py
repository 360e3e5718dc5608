"""GPU parity of the HIP hot path against the CPU oracle: H_eff (three
precisions), environment updates, merge and Davidson, on seeded inputs that
span several 64 x 64 tiles with ragged tails."""
import numpy as np
import pytest

from helpers import (pl, synth, tables, blocks_to_flat, flat_to_blocks, mpo_site, rel_err, dev, host, say)
from oracle import models, mpo as M, dmrg
from oracle.blocks import Bond, two_site_keys, two_site_shape, flatten, unflatten

pytestmark = pytest.mark.gpu
PQ = (-1, 1)


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = pl.Context(0)
    yield c
    c.close()


def _cylinder_problem(Lx, Ly, m, seed, center=None):
    N = Lx * Ly
    mpo = M.build_mpo(models.heisenberg_terms(models.square_cylinder_bonds(Lx, Ly)), N, models.OPS, PQ)
    bonds = synth.binomial_bonds(N, m)
    i = N // 2 - 1 if center is None else center
    rng = np.random.default_rng(seed)
    L = synth.random_env_blocks(bonds[i], mpo.deltas[i], rng)
    R = synth.random_env_blocks(bonds[i + 2], mpo.deltas[i + 2], rng)
    psi = synth.random_two_site_blocks(bonds[i], bonds[i + 2], PQ, rng)
    return mpo, bonds, i, L, R, psi


def _heff_setup(ctx, mpo, bonds, i, L, R, prec):
    bl, br = bonds[i], bonds[i + 2]
    t, (B1, B2, P) = tables(bl, br, PQ, mpo.deltas[i], mpo.deltas[i + 2])
    Ld = dev(blocks_to_flat(L, t["L"][0], t["L"][1], pl.ENV_L))
    Rd = dev(blocks_to_flat(R, t["R"][0], t["R"][1], pl.ENV_R))
    op = pl.Heff(ctx, B1, B2, P, mpo_site(mpo, i), mpo_site(mpo, i + 1), Ld, Rd, prec)
    return op, t


@pytest.mark.parametrize("prec,tol", [(pl.F64, 1e-12), (pl.F32, 1e-5), (pl.BF16X3, 1e-4)])
@pytest.mark.parametrize("shape", [(4, 4, 200, 11), (3, 4, 64, 12), (5, 2, 40, 13)])
def test_heff_apply_matches_oracle(ctx, prec, tol, shape):
    Lx, Ly, m, seed = shape
    say("heff parity", shape, "prec", prec)
    mpo, bonds, i, L, R, psi = _cylinder_problem(Lx, Ly, m, seed)
    bl, br = Bond(bonds[i]), Bond(bonds[i + 2])
    yref = dmrg.heff_apply(L, R, mpo.W[i], mpo.W[i + 1], psi, bl, br, PQ, mpo.deltas[i], mpo.deltas[i + 2])
    op, t = _heff_setup(ctx, mpo, bonds, i, L, R, prec)
    x = dev(blocks_to_flat(psi, t["x"][0], t["x"][1], pl.TWO_SITE))
    y = dev(np.full(t["x"][1], np.nan))
    op.apply(x, y)
    ygot = flat_to_blocks(host(y), t["x"][0], pl.TWO_SITE)
    keys = two_site_keys(bl, br, PQ)
    shapes = [two_site_shape(k, bl, br, PQ) for k in keys]
    a, b = flatten(ygot, keys, shapes), flatten(yref, keys, shapes)
    err = rel_err(a, b)
    say("  rel err", err, "n", len(a), "flops", op.info()["flops"])
    assert np.all(np.isfinite(a))
    assert err <= tol
    if prec == pl.F64:
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


def test_heff_diag_matches_oracle(ctx):
    mpo, bonds, i, L, R, psi = _cylinder_problem(4, 4, 120, 21)
    bl, br = Bond(bonds[i]), Bond(bonds[i + 2])
    dref = dmrg.heff_diag(L, R, mpo.W[i], mpo.W[i + 1], bl, br, PQ, mpo.deltas[i], mpo.deltas[i + 2])
    op, t = _heff_setup(ctx, mpo, bonds, i, L, R, pl.F64)
    out = dev(np.full(t["x"][1], np.nan))
    op.diag(out)
    got = flat_to_blocks(host(out), t["x"][0], pl.TWO_SITE)
    for k, v in dref.items():
        assert np.allclose(got[k], v, rtol=1e-13, atol=1e-13 * np.abs(v).max())


def test_heff_repeated_calls_bitwise_identical(ctx):
    mpo, bonds, i, L, R, psi = _cylinder_problem(4, 4, 200, 5)
    op, t = _heff_setup(ctx, mpo, bonds, i, L, R, pl.F64)
    x = dev(blocks_to_flat(psi, t["x"][0], t["x"][1], pl.TWO_SITE))
    y1, y2 = dev(np.zeros(t["x"][1])), dev(np.ones(t["x"][1]))
    op.apply(x, y1)
    op.apply(x, y2)
    assert np.array_equal(host(y1), host(y2))


def _site_tables(bl, br):
    return pl.layout(pl.SITE, pl.Bond(bl), pl.Bond(br), pl.Phys(PQ))


@pytest.mark.parametrize("direction", [1, -1])
def test_env_update_matches_oracle(ctx, direction):
    Lx, Ly, m, seed = 4, 4, 180, 31
    say("env parity dir", direction)
    N = Lx * Ly
    mpo = M.build_mpo(models.heisenberg_terms(models.square_cylinder_bonds(Lx, Ly)), N, models.OPS, PQ)
    bonds = synth.binomial_bonds(N, m)
    i = 7
    rng = np.random.default_rng(seed)
    A = synth.random_site_blocks(bonds[i], bonds[i + 1], PQ, rng)
    bl, br = bonds[i], bonds[i + 1]
    tA, nA = _site_tables(bl, br)
    Ad = dev(blocks_to_flat(A, tA, nA, pl.SITE))
    if direction == 1:
        Ein = synth.random_env_blocks(bl, mpo.deltas[i], rng)
        tin, nin = pl.layout(pl.ENV_L, pl.Bond(bl), deltas=mpo.deltas[i])
        tout, nout = pl.layout(pl.ENV_L, pl.Bond(br), deltas=mpo.deltas[i + 1])
        ref = dmrg.update_L(Ein, A, mpo.W[i], PQ, mpo.deltas[i], mpo.deltas[i + 1])
        kind = pl.ENV_L
    else:
        Ein = synth.random_env_blocks(br, mpo.deltas[i + 1], rng)
        tin, nin = pl.layout(pl.ENV_R, pl.Bond(br), deltas=mpo.deltas[i + 1])
        tout, nout = pl.layout(pl.ENV_R, pl.Bond(bl), deltas=mpo.deltas[i])
        ref = dmrg.update_R(Ein, A, mpo.W[i], PQ, mpo.deltas[i], mpo.deltas[i + 1])
        kind = pl.ENV_R
    Ed = dev(blocks_to_flat(Ein, tin, nin, kind))
    out = dev(np.full(nout, np.nan))
    pl.env_update(ctx, direction, pl.Bond(bl), pl.Bond(br), pl.Phys(PQ), mpo_site(mpo, i), Ed, Ad, out)
    got = flat_to_blocks(host(out), tout, kind)
    num = sum(float(np.sum((got[k] - ref.get(k, 0.0)) ** 2)) for k in got)
    den = sum(float(np.sum(v ** 2)) for v in ref.values())
    assert set(ref) <= set(got)
    assert np.sqrt(num / den) <= 1e-12


def test_merge_matches_oracle(ctx):
    rng = np.random.default_rng(41)
    N = 20
    bonds = synth.binomial_bonds(N, 150)
    j = 9
    bl, bm, br = bonds[j], bonds[j + 1], bonds[j + 2]
    psiL = synth.random_site_blocks(bl, bm, PQ, rng)
    psiR = synth.random_site_blocks(bm, br, PQ, rng)
    Bm = Bond(bm)
    V = {q: 1.0 / rng.uniform(1e-6, 1.0, Bm.dim(q)) for q in Bm.qs}
    ref = dmrg.merge(psiL, V, psiR, PQ)
    tL, nL = _site_tables(bl, bm)
    tR, nR = _site_tables(bm, br)
    tx, nx = pl.layout(pl.TWO_SITE, pl.Bond(bl), pl.Bond(br), pl.Phys(PQ))
    Vflat = np.concatenate([V[q] for q in Bm.qs])
    out = dev(np.full(nx, np.nan))
    pl.merge_regions(ctx, pl.Bond(bl), pl.Bond(bm), pl.Bond(br), pl.Phys(PQ), dev(blocks_to_flat(psiL, tL, nL, pl.SITE)),
                     dev(Vflat), dev(blocks_to_flat(psiR, tR, nR, pl.SITE)), out)
    got = flat_to_blocks(host(out), tx, pl.TWO_SITE)
    keys = two_site_keys(Bond(bl), Bond(br), PQ)
    shapes = [two_site_shape(k, Bond(bl), Bond(br), PQ) for k in keys]
    assert rel_err(flatten(got, keys, shapes), flatten(ref, keys, shapes)) <= 1e-13


def _hermitian_problem(ctx, N, m, seed, center):
    """L, R built by both sides from the same random MPS (so H_eff is
    symmetric): the oracle with update_L/R, the GPU with env_update."""
    mpo = M.build_mpo(models.heisenberg_terms(models.chain_bonds(N)), N, models.OPS, PQ)
    bonds, sites = synth.random_mps(N, m, seed)
    sites = synth.isometric_scale(sites, bonds, PQ, center)
    Lo, Ro = dmrg.left_boundary(), dmrg.right_boundary(0)
    Ph = pl.Phys(PQ)
    Lg = dev(np.ones(1))
    for i in range(center):
        Lo = dmrg.update_L(Lo, sites[i], mpo.W[i], PQ, mpo.deltas[i], mpo.deltas[i + 1])
        tA, nA = _site_tables(bonds[i], bonds[i + 1])
        tout, nout = pl.layout(pl.ENV_L, pl.Bond(bonds[i + 1]), deltas=mpo.deltas[i + 1])
        out = dev(np.zeros(nout))
        pl.env_update(ctx, 1, pl.Bond(bonds[i]), pl.Bond(bonds[i + 1]), Ph, mpo_site(mpo, i), Lg,
                      dev(blocks_to_flat(sites[i], tA, nA, pl.SITE)), out)
        Lg = out
    Rg = dev(np.ones(1))
    for i in range(N - 1, center + 1, -1):
        Ro = dmrg.update_R(Ro, sites[i], mpo.W[i], PQ, mpo.deltas[i], mpo.deltas[i + 1])
        tA, nA = _site_tables(bonds[i], bonds[i + 1])
        tout, nout = pl.layout(pl.ENV_R, pl.Bond(bonds[i]), deltas=mpo.deltas[i])
        out = dev(np.zeros(nout))
        pl.env_update(ctx, -1, pl.Bond(bonds[i]), pl.Bond(bonds[i + 1]), Ph, mpo_site(mpo, i), Rg,
                      dev(blocks_to_flat(sites[i], tA, nA, pl.SITE)), out)
        Rg = out
    rng = np.random.default_rng(seed + 7)
    psi = synth.random_two_site_blocks(bonds[center], bonds[center + 2], PQ, rng)
    return mpo, bonds, Lo, Ro, Lg, Rg, psi


@pytest.mark.parametrize("prec", [pl.F64, pl.F32, pl.BF16X3])
def test_davidson_matches_oracle(ctx, prec):
    N, m, seed, c = 14, 60, 3, 6
    say("davidson parity prec", prec)
    mpo, bonds, Lo, Ro, Lg, Rg, psi = _hermitian_problem(ctx, N, m, seed, c)
    bl, br = Bond(bonds[c]), Bond(bonds[c + 2])
    keys = two_site_keys(bl, br, PQ)
    shapes = [two_site_shape(k, bl, br, PQ) for k in keys]
    mv = lambda v: flatten(dmrg.heff_apply(Lo, Ro, mpo.W[c], mpo.W[c + 1], unflatten(v, keys, shapes),
                                           bl, br, PQ, mpo.deltas[c], mpo.deltas[c + 2]), keys, shapes)
    diag = flatten(dmrg.heff_diag(Lo, Ro, mpo.W[c], mpo.W[c + 1], bl, br, PQ, mpo.deltas[c], mpo.deltas[c + 2]),
                   keys, shapes)
    x0 = flatten(psi, keys, shapes)
    Eo, xo, rno, nmvo = dmrg.davidson(mv, x0, diag, dmrg.DavidsonParams(200, 1e-9, 8))
    t, (B1, B2, P) = tables(bonds[c], bonds[c + 2], PQ, mpo.deltas[c], mpo.deltas[c + 2])
    W1, W2 = mpo_site(mpo, c), mpo_site(mpo, c + 1)
    op = pl.Heff(ctx, B1, B2, P, W1, W2, Lg, Rg, prec)
    op64 = pl.Heff(ctx, B1, B2, P, W1, W2, Lg, Rg, pl.F64) if prec != pl.F64 else None
    x = dev(blocks_to_flat(psi, t["x"][0], t["x"][1], pl.TWO_SITE))
    E, rn, nmv, code = pl.davidson_step(ctx, op, x, max_matvec=200, max_sub=8, tol=1e-9, op64=op64)
    say("  E_gpu", E, "E_oracle", Eo, "resid", rn, "nmv", nmv, "oracle nmv", nmvo)
    assert code == 0
    assert abs(E - Eo) <= 1e-9 * abs(Eo)
    xg = flatten(flat_to_blocks(host(x), t["x"][0], pl.TWO_SITE), keys, shapes)
    assert abs(abs(xg @ xo) - 1.0) <= 1e-6


def test_davidson_mixed_vs_f64_at_m2000_bond(ctx):
    """One bond at the sweep workload's scale: width-8 Heisenberg cylinder
    (6 x 8, D = 26, the 24 x 8 workload's MPO width) at m = 2000, environments
    built by both sides from the same seeded isometric MPS.  Davidson to a
    residual of 1e-8 (energy error ~ residual^2 / gap) in FP64 and in the
    mixed mode (FP32 products, FP64 refinement) against the oracle's Davidson
    on its own environments: both within 1e-9 relative, and the mixed energy
    is not the FP64 one bit for bit (the check sees the FP32 products).
    From the random start the first 70-90 products (the number varies with
    rounding) find the ground state; then the residual falls by about 0.6 per
    restart cycle of 8 products, so 500 products leave a margin."""
    Lx, Ly, m, seed = 6, 8, 2000, 12
    N = Lx * Ly
    c = N // 2 - 1
    mpo = M.build_mpo(models.heisenberg_terms(models.square_cylinder_bonds(Lx, Ly)), N, models.OPS, PQ)
    bonds, sites = synth.random_mps(N, m, seed)
    sites = synth.isometric_scale(sites, bonds, PQ, c)
    Ph = pl.Phys(PQ)
    Lo, Ro = dmrg.left_boundary(), dmrg.right_boundary(0)
    Lg, Rg = dev(np.ones(1)), dev(np.ones(1))
    for i in range(c):
        Lo = dmrg.update_L(Lo, sites[i], mpo.W[i], PQ, mpo.deltas[i], mpo.deltas[i + 1])
        tA, nA = _site_tables(bonds[i], bonds[i + 1])
        _, nout = pl.layout(pl.ENV_L, pl.Bond(bonds[i + 1]), deltas=mpo.deltas[i + 1])
        out = dev(np.zeros(nout))
        pl.env_update(ctx, 1, pl.Bond(bonds[i]), pl.Bond(bonds[i + 1]), Ph, mpo_site(mpo, i), Lg,
                      dev(blocks_to_flat(sites[i], tA, nA, pl.SITE)), out)
        Lg = out
    for i in range(N - 1, c + 1, -1):
        Ro = dmrg.update_R(Ro, sites[i], mpo.W[i], PQ, mpo.deltas[i], mpo.deltas[i + 1])
        tA, nA = _site_tables(bonds[i], bonds[i + 1])
        _, nout = pl.layout(pl.ENV_R, pl.Bond(bonds[i]), deltas=mpo.deltas[i])
        out = dev(np.zeros(nout))
        pl.env_update(ctx, -1, pl.Bond(bonds[i]), pl.Bond(bonds[i + 1]), Ph, mpo_site(mpo, i), Rg,
                      dev(blocks_to_flat(sites[i], tA, nA, pl.SITE)), out)
        Rg = out
    psi = synth.random_two_site_blocks(bonds[c], bonds[c + 2], PQ, np.random.default_rng(seed + 7))
    bl, br = Bond(bonds[c]), Bond(bonds[c + 2])
    keys = two_site_keys(bl, br, PQ)
    shapes = [two_site_shape(k, bl, br, PQ) for k in keys]
    mv = lambda v: flatten(dmrg.heff_apply(Lo, Ro, mpo.W[c], mpo.W[c + 1], unflatten(v, keys, shapes),
                                           bl, br, PQ, mpo.deltas[c], mpo.deltas[c + 2]), keys, shapes)
    diag = flatten(dmrg.heff_diag(Lo, Ro, mpo.W[c], mpo.W[c + 1], bl, br, PQ, mpo.deltas[c], mpo.deltas[c + 2]),
                   keys, shapes)
    Eo, _, rno, nmvo = dmrg.davidson(mv, flatten(psi, keys, shapes), diag, dmrg.DavidsonParams(300, 1e-8, 8))
    t, (B1, B2, P) = tables(bonds[c], bonds[c + 2], PQ, mpo.deltas[c], mpo.deltas[c + 2])
    W1, W2 = mpo_site(mpo, c), mpo_site(mpo, c + 1)
    x0 = blocks_to_flat(psi, t["x"][0], t["x"][1], pl.TWO_SITE)
    E = {}
    for name, prec in (("f64", pl.F64), ("mixed", pl.F32)):
        op = pl.Heff(ctx, B1, B2, P, W1, W2, Lg, Rg, prec)
        op64 = pl.Heff(ctx, B1, B2, P, W1, W2, Lg, Rg, pl.F64) if prec != pl.F64 else None
        x = dev(x0)
        E[name], rn, nmv, code = pl.davidson_step(ctx, op, x, max_matvec=500, max_sub=8, tol=1e-8, op64=op64)
        say("  m=2000 bond", name, "E", E[name], "resid", rn, "nmv", nmv)
        assert rn <= 5e-7, name
        op.free()
        if op64 is not None:
            op64.free()
    say("  oracle E", Eo, "resid", rno, "nmv", nmvo, "n_psi", t["x"][1], "mixed - f64", E["mixed"] - E["f64"])
    for name in E:
        assert abs(E[name] - Eo) <= 1e-9 * abs(Eo), name
    assert E["mixed"] != E["f64"]
