"""heff_apply replayed from captured HIP graphs gives the bits of the eager
launches: several replays with eager work and synchronisations between them,
several (x, y) pairs, and a Davidson solve."""
import numpy as np
import pytest

from helpers import pl, synth, say, dev, host, blocks_to_flat, tables, mpo_site
from oracle import models, mpo as M

pytestmark = pytest.mark.gpu
PQ = synth.SPIN_HALF_Q


@pytest.fixture(scope="module")
def setup():
    import torch
    rng = np.random.default_rng(61)
    Lx, Ly, m, i = 4, 4, 96, 7
    N = Lx * Ly
    mpo = M.build_mpo(models.heisenberg_terms(models.square_cylinder_bonds(Lx, Ly)), N, models.OPS, PQ)
    bonds = synth.binomial_bonds(N, m)
    t, (B1, B2, P) = tables(bonds[i], bonds[i + 2], PQ, mpo.deltas[i], mpo.deltas[i + 2])
    L = synth.random_env_blocks(bonds[i], mpo.deltas[i], rng)
    R = synth.random_env_blocks(bonds[i + 2], mpo.deltas[i + 2], rng)
    # Hermitian operator for the Davidson check: symmetrise the blocks pairwise
    Ld = dev(blocks_to_flat(L, t["L"][0], t["L"][1], pl.ENV_L))
    Rd = dev(blocks_to_flat(R, t["R"][0], t["R"][1], pl.ENV_R))
    xs = [dev(rng.standard_normal(t["x"][1])) for _ in range(3)]
    return dict(mpo=mpo, i=i, B=(B1, B2, P), Ld=Ld, Rd=Rd, xs=xs, n=t["x"][1])


@pytest.mark.parametrize("prec", [pl.F64, pl.F32])
def test_graph_replay_bitwise_equals_eager(setup, prec):
    import torch
    S = setup
    B1, B2, P = S["B"]
    ctx = pl.Context(0)
    op = pl.Heff(ctx, B1, B2, P, mpo_site(S["mpo"], S["i"]), mpo_site(S["mpo"], S["i"] + 1), S["Ld"], S["Rd"], prec)
    eager = []
    for x in S["xs"]:
        y = torch.empty_like(x)
        op.apply(x, y)
        torch.cuda.synchronize()
        eager.append(host(y))
    pl.set_graphs(ctx, True)
    ys = [torch.full_like(x, float("nan")) for x in S["xs"]]
    scratch = torch.zeros(1 << 20, dtype=torch.float64, device="cuda")
    for rep in range(4):
        for k, x in enumerate(S["xs"]):
            ys[k].fill_(float("nan"))
            op.apply(x, ys[k])                 # first pass captures, later ones replay
            scratch.mul_(1.5).add_(rep)        # eager work between replays
            torch.cuda.synchronize()
            assert np.array_equal(host(ys[k]), eager[k]), (rep, k)
    say("graph replay prec", prec, "ok")
    op.free()
    ctx.close()


def test_davidson_with_graphs_bitwise_equals_eager(setup):
    import torch
    S = setup
    B1, B2, P = S["B"]
    out = []
    for graphs in (False, True):
        ctx = pl.Context(0)
        pl.set_graphs(ctx, graphs)
        op = pl.Heff(ctx, B1, B2, P, mpo_site(S["mpo"], S["i"]), mpo_site(S["mpo"], S["i"] + 1), S["Ld"], S["Rd"],
                     pl.F64)
        psi = S["xs"][0].clone()
        E, r, n, code = pl.davidson_step(ctx, op, psi, max_matvec=12, max_sub=6, tol=1e-12)
        torch.cuda.synchronize()
        out.append((E, r, n, host(psi)))
        op.free()
        ctx.close()
    say("davidson eager", out[0][:3], "graphs", out[1][:3])
    assert out[0][:3] == out[1][:3]
    assert np.array_equal(out[0][3], out[1][3])
