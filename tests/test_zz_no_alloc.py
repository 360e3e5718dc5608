"""env_update_noalloc (the environment update that allocates no device
memory) against env_update on the same inputs: two calls in a row, the
second on a smaller bond, both directions; and the size limit."""
import numpy as np
import pytest

from helpers import pl, synth, blocks_to_flat, dev, host, say, mpo_site
from oracle import models, mpo as M

pytestmark = pytest.mark.gpu
PQ = (-1, 1)


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = pl.Context(0)
    yield c
    c.close()


def _problem(Lx, Ly, m, i, seed, direction):
    N = Lx * Ly
    mpo = M.build_mpo(models.heisenberg_terms(models.square_cylinder_bonds(Lx, Ly)), N, models.OPS, PQ)
    bonds = synth.binomial_bonds(N, m)
    rng = np.random.default_rng(seed)
    bl, br = bonds[i], bonds[i + 1]
    A = synth.random_site_blocks(bl, br, PQ, rng)
    tA, nA = pl.layout(pl.SITE, pl.Bond(bl), pl.Bond(br), pl.Phys(PQ))
    if direction == 1:
        Ein = synth.random_env_blocks(bl, mpo.deltas[i], rng)
        tin, nin = pl.layout(pl.ENV_L, pl.Bond(bl), deltas=mpo.deltas[i])
        _, nout = pl.layout(pl.ENV_L, pl.Bond(br), deltas=mpo.deltas[i + 1])
        kind = pl.ENV_L
    else:
        Ein = synth.random_env_blocks(br, mpo.deltas[i + 1], rng)
        tin, nin = pl.layout(pl.ENV_R, pl.Bond(br), deltas=mpo.deltas[i + 1])
        _, nout = pl.layout(pl.ENV_R, pl.Bond(bl), deltas=mpo.deltas[i])
        kind = pl.ENV_R
    args = (pl.Bond(bl), pl.Bond(br), pl.Phys(PQ), mpo_site(mpo, i),
            dev(blocks_to_flat(Ein, tin, nin, kind)), dev(blocks_to_flat(A, tA, nA, pl.SITE)))
    return args, nout


@pytest.mark.parametrize("direction", [1, -1])
def test_noalloc_equals_env_update_twice(ctx, direction):
    """Same bits as env_update on a 4x4 cylinder bond at m = 180, then on a
    smaller bond (m = 60) right after it (the scratch keeps the first call's
    contents), the outputs NaN-filled before each call."""
    for (m, i, seed) in ((180, 7, 31), (60, 5, 32)):
        say("noalloc dir", direction, "m", m)
        args, nout = _problem(4, 4, m, i, seed, direction)
        ref = dev(np.full(nout, np.nan))
        got = dev(np.full(nout, np.nan))
        pl.env_update(ctx, direction, *args, ref)
        pl.env_update_noalloc(ctx, direction, *args, got)
        a, b = host(got), host(ref)
        assert np.all(np.isfinite(a)) and np.array_equal(a, b)


def test_noalloc_rejects_updates_beyond_its_scratch(ctx):
    """A 24x8 cylinder bond at m = 2000 (D = 26) needs more than the 64 MiB
    scratch: PDMRG_EINVAL with a message, nothing launched (the device
    buffers are never read)."""
    N = 24 * 8
    mpo = M.build_mpo(models.heisenberg_terms(models.square_cylinder_bonds(24, 8)), N, models.OPS, PQ)
    bonds = synth.binomial_bonds(N, 2000)
    i = N // 2
    dummy = dev(np.zeros(4))
    with pytest.raises(pl.PdmrgError, match="scratch"):
        pl.env_update_noalloc(ctx, 1, pl.Bond(bonds[i]), pl.Bond(bonds[i + 1]), pl.Phys(PQ), mpo_site(mpo, i),
                              dummy, dummy, dummy)
