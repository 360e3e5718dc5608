"""End-to-end DMRG sweeps on the GPU against the oracle and exact references:
serial and real-space parallel sweeps (Sec. II, Fig. 4), FP64 and mixed
precision with FP64 refinement, U(1) and no-symmetry models."""
import numpy as np
import pytest

from helpers import pl, synth, say, golden
from oracle import models, mpo as M, dmrg, exact

pytestmark = pytest.mark.gpu
E_ED_CHAIN16 = golden("heisenberg_chain_N16_J1_E0")


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = pl.Context(0)
    yield c
    c.close()


def _oracle_run(terms, N, phys, bonds, sites, schedule, n_regions, n_warmup, dav, dav_shared, q=0):
    mpo = M.build_mpo(terms, N, models.OPS, phys)
    p = dmrg.SweepParams(schedule=schedule, n_warmup=n_warmup, n_regions=n_regions,
                         dav=dmrg.DavidsonParams(max_matvec=dav[0], max_sub=dav[1], tol=dav[2]),
                         dav_shared=dmrg.DavidsonParams(max_matvec=dav_shared[0], max_sub=dav_shared[1],
                                                        tol=dav_shared[2]))
    return dmrg.run_dmrg(mpo, bonds, sites, q, p)[1]


def _gpu_run(ctx, mpo, bonds, sites, schedule, n_regions, n_warmup, dav, dav_shared, prec=pl.F64, phys=(-1, 1), q=0):
    mps = pl.Mps(ctx, bonds, sites, phys, q)
    out = []
    for k, m in enumerate(schedule):
        nreg = 1 if k < n_warmup else n_regions
        rep = mps.sweep(mpo, m, nreg, prec=prec, dav=pl.dav_params(*dav), dav_shared=pl.dav_params(*dav_shared))
        out.append(rep)
    mps.free()
    return out


def test_chain16_serial_matches_ed_and_oracle(ctx):
    N = 16
    bonds, sites = synth.random_mps(N, 16, 1)
    mpo = pl.Mpo("chain", N, 1, (1.0, 1.0))
    dav, davs = (20, 8, 1e-10), (40, 8, 1e-10)
    reps = _gpu_run(ctx, mpo, bonds, sites, [64] * 4, 1, 0, dav, davs)
    Eo = _oracle_run(models.heisenberg_terms(models.chain_bonds(N)), N, (-1, 1), bonds, sites, [64] * 4, 1, 0, dav, davs)
    Eg = [r["energy"] for r in reps]
    say("chain16 gpu", Eg, "oracle", Eo, "s/sweep", [round(r["seconds"], 3) for r in reps])
    assert abs(Eg[-1] - E_ED_CHAIN16) <= 1e-9 * abs(E_ED_CHAIN16)
    for a, b in zip(Eg, Eo):
        assert abs(a - b) <= 1e-9 * abs(b)


@pytest.mark.parametrize("n_regions", [2, 4])
def test_chain16_parallel_regions(ctx, n_regions):
    N = 16
    bonds, sites = synth.random_mps(N, 16, 1)
    mpo = pl.Mpo("chain", N, 1, (1.0, 1.0))
    sched = [32, 32, 64, 64, 64]
    dav, davs = (10, 8, 1e-10), (40, 8, 1e-10)
    reps = _gpu_run(ctx, mpo, bonds, sites, sched, n_regions, 2, dav, davs)
    Eo = _oracle_run(models.heisenberg_terms(models.chain_bonds(N)), N, (-1, 1), bonds, sites, sched, n_regions, 2,
                     dav, davs)
    Eg = [r["energy"] for r in reps]
    say("regions", n_regions, "gpu", Eg, "oracle", Eo)
    assert abs(Eg[-1] - E_ED_CHAIN16) <= 1e-9 * abs(E_ED_CHAIN16)
    assert abs(Eo[-1] - E_ED_CHAIN16) <= 1e-9 * abs(E_ED_CHAIN16)
    for a, b in zip(Eg, Eo):
        assert abs(a - b) <= 1e-8 * abs(b)


@pytest.mark.parametrize("prec", [pl.F32, pl.BF16X3])
def test_chain16_mixed_precision_reaches_ed(ctx, prec):
    N = 16
    bonds, sites = synth.random_mps(N, 16, 1)
    mpo = pl.Mpo("chain", N, 1, (1.0, 1.0))
    reps = _gpu_run(ctx, mpo, bonds, sites, [64] * 4, 1, 0, (30, 8, 1e-10), (40, 8, 1e-10), prec=prec)
    say("mixed", prec, [r["energy"] for r in reps])
    assert abs(reps[-1]["energy"] - E_ED_CHAIN16) <= 1e-9 * abs(E_ED_CHAIN16)


def test_tfim_no_symmetry_closed_form(ctx):
    N, h = 12, 0.8
    bonds, sites = synth.random_mps(N, 16, 4, phys_q=synth.TRIVIAL_Q)
    mpo = pl.Mpo("tfim", N, 1, (1.0, h))
    reps = _gpu_run(ctx, mpo, bonds, sites, [64] * 4, 1, 0, (30, 8, 1e-10), (40, 8, 1e-10), phys=synth.TRIVIAL_Q)
    e = exact.tfim_chain_energy(N, 1.0, h)
    say("tfim", reps[-1]["energy"], e)
    assert abs(reps[-1]["energy"] - e) <= 1e-9 * abs(e)


def test_xx_chain_closed_form_two_regions(ctx):
    N = 16
    bonds, sites = synth.random_mps(N, 16, 6)
    mpo = pl.Mpo("chain", N, 1, (1.0, 0.0))
    reps = _gpu_run(ctx, mpo, bonds, sites, [32, 64, 64, 64, 64, 64], 2, 1, (20, 8, 1e-10), (40, 8, 1e-11))
    e = exact.xx_chain_energy(N)
    say("xx", reps[-1]["energy"], e)
    assert abs(reps[-1]["energy"] - e) <= 1e-9 * abs(e)


def test_concurrent_regions_bitwise_equal_to_sequential(ctx):
    """Regions on their own streams and host threads, and regions in lockstep
    with the truncation SVDs of each step in one batch (concurrent = 2), give
    the same bits as one after the other (no data crosses regions between
    merges, and a block's Jacobi iteration does not depend on its batch)."""
    N = 16
    bonds, sites = synth.random_mps(N, 16, 5)
    mpo = pl.Mpo("chain", N, 1, (1.0, 1.0))
    out = {}
    for conc in (False, True, 2):
        mps = pl.Mps(ctx, bonds, sites)
        es = []
        for k, m in enumerate([32, 48, 48, 64]):
            rep = mps.sweep(mpo, m, 1 if k == 0 else 4, dav=pl.dav_params(6, 8, 1e-9),
                            dav_shared=pl.dav_params(40, 8, 1e-10), concurrent=conc)
            es.append(rep["energy"])
        tens = []
        for i in range(N):
            B1, B2 = pl.Bond(mps.bond(i)), pl.Bond(mps.bond(i + 1))
            _, n = pl.layout(pl.SITE, B1, B2, pl.Phys((-1, 1)))
            buf = np.zeros(n)
            pl.check(pl.lib().mps_get_site(mps.h, i, buf.ctypes.data_as(pl.POINTER(pl.c_double)), n))
            tens.append(buf)
        out[conc] = (es, tens)
        mps.free()
    say("sequential", out[False][0], "concurrent", out[True][0], "lockstep", out[2][0])
    for conc in (True, 2):
        assert out[False][0] == out[conc][0]
        for a, b in zip(out[False][1], out[conc][1]):
            assert np.array_equal(a, b)
    assert abs(out[True][0][-1] - E_ED_CHAIN16) <= 1e-6 * abs(E_ED_CHAIN16)


@pytest.mark.parametrize("n_regions,concurrent", [(1, False), (2, False), (4, True)])
def test_env_recompute_stride_same_bits_less_memory(ctx, n_regions, concurrent):
    """Environment recompute (stride 3): the sweeps give the same bits as
    with every environment kept, the measurement sweep the same gradient,
    and the allocator's peak of device memory in use is lower."""
    N, m = 24, 48
    mpo = pl.Mpo("chain", N, 1, (1.0, 1.0))
    bonds, sites = synth.random_mps(N, 16, 11)
    out = {}
    for stride in (0, 3):
        pl.set_env_stride(ctx, stride)
        mps = pl.Mps(ctx, bonds, sites)
        pl.memory_stats(reset_peak=True)
        in0 = pl.memory_stats()[0]
        E = [mps.sweep(mpo, m, 1 if k == 0 else n_regions, concurrent=concurrent)["energy"] for k in range(3)]
        peak = pl.memory_stats()[1] - in0
        _, G = mps.gradients(mpo)
        out[stride] = (E, [g.cpu().numpy() for g in G], peak)
        mps.free()
    pl.set_env_stride(ctx, 0)
    say("stride energies", out[0][0], out[3][0], "peak bytes", out[0][2], out[3][2])
    assert out[0][0] == out[3][0]
    assert all(np.array_equal(a, b) for a, b in zip(out[0][1], out[3][1]))
    assert out[3][2] < out[0][2]


def test_sweep_schedule_is_fig4(ctx):
    """The library's region-parallel sweep follows Fig. 4 (reading R5) step by
    step: with the progress log on and the regions one after the other, a
    12-site chain in 3 regions optimises bonds 0, 1, 2 (region 1 right),
    6, 5, 4 (region 2 left), 8, 9, 10 (region 3 right), merges at sites 3|4,
    then moves every region back and merges at 7|8 -- the order the oracle's
    schedule pin fixes."""
    import os
    import sys
    import tempfile
    N, m = 12, 8
    mpo = pl.Mpo("chain", N, 1, (1.0, 1.0))
    bonds, sites = synth.random_mps(N, m, 5)
    mps = pl.Mps(ctx, bonds, sites)
    mps.sweep(mpo, m, 3)   # canonical form, split, one parallel sweep
    tmp = tempfile.TemporaryFile(mode="w+b")
    saved = os.dup(2)
    pl.set_verbose(ctx, 1)
    try:
        sys.stderr.flush()
        os.dup2(tmp.fileno(), 2)
        mps.sweep(mpo, m, 3, concurrent=False)
    finally:
        os.dup2(saved, 2)
        os.close(saved)
        pl.set_verbose(ctx, 0)
    tmp.seek(0)
    got = []
    for line in tmp.read().decode().splitlines():
        f = line.split()
        if len(f) > 2 and f[0] == "pdmrg:" and f[1] in ("bond", "merge"):
            got.append((f[1], int(f[2].split("|")[0])))
    half_a = [0, 1, 2, 6, 5, 4, 8, 9, 10]
    half_b = [2, 1, 0, 4, 5, 6, 10, 9, 8]
    want = [("bond", i) for i in half_a] + [("merge", 3)] + [("bond", i) for i in half_b] + [("merge", 7)]
    say("schedule", got)
    assert got == want
    mps.free()
    mpo.free()
