"""GPU parity of svd_truncate (Eq. eqn:svd with the Appendix recursion)
against the oracle: singular values (including graded spectra down to
1e-12 lambda_1), reconstruction, orthonormality, truncation bookkeeping and
the split / merge round trip (Eqs. eqn:inverse, eqn:isvd, eqn:merge)."""
import numpy as np
import pytest

from helpers import pl, synth, blocks_to_flat, flat_to_blocks, dev, host, say
from oracle import dmrg
from test_oracle_pins import tie_psi, TIE_CASES
from oracle.blocks import Bond, two_site_keys, two_site_shape, flatten

pytestmark = pytest.mark.gpu
PQ = (-1, 1)


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = pl.Context(0)
    yield c
    c.close()


def _graded_psi(bl, br, seed, smin):
    """Two-site blocks whose middle-charge blocks have log-spaced singular
    values from 1 down to smin (random orthogonal factors)."""
    rng = np.random.default_rng(seed)
    Bl, Br = Bond(bl), Bond(br)
    psi = {}
    mids = sorted({q + s for q in Bl.qs for s in PQ})
    for qm in mids:
        rows = [(s1, qm - PQ[s1]) for s1 in range(2) if Bl.has(qm - PQ[s1])]
        cols = [(s2, qm + PQ[s2]) for s2 in range(2) if Br.has(qm + PQ[s2])]
        nr = sum(Bl.dim(q) for _, q in rows)
        nc = sum(Br.dim(q) for _, q in cols)
        if not rows or not cols:
            continue
        k = min(nr, nc)
        U, _ = np.linalg.qr(rng.standard_normal((nr, k)))
        V, _ = np.linalg.qr(rng.standard_normal((nc, k)))
        s = np.logspace(0, np.log10(smin), k) * rng.uniform(0.5, 1.0)
        M = (U * s) @ V.T
        r0 = 0
        for s1, qa in rows:
            c0 = 0
            for s2, qb in cols:
                psi[(qa, s1, s2)] = M[r0:r0 + Bl.dim(qa), c0:c0 + Br.dim(qb)].copy()
                c0 += Br.dim(qb)
            r0 += Bl.dim(qa)
    nrm = np.sqrt(sum(float(np.sum(v * v)) for v in psi.values()))
    return {k: v / nrm for k, v in psi.items()}


CASES = [
    ("binomial", synth.binomial_bond(24, 11, 90), synth.binomial_bond(24, 13, 90), 1),
    ("tall-wide", {-2: 40, 0: 70, 2: 12}, {-2: 9, 0: 30, 2: 50}, 2),
    ("tiny", {0: 1}, {0: 1, 2: 1}, 3),
]


@pytest.mark.parametrize("name,bl,br,seed", CASES)
def test_svd_values_and_reconstruction(ctx, name, bl, br, seed):
    say("svd", name)
    psi = _graded_psi(bl, br, seed, 1e-12)
    B1, B2, P = pl.Bond(bl), pl.Bond(br), pl.Phys(PQ)
    tx, nx = pl.layout(pl.TWO_SITE, B1, B2, P)
    x = dev(blocks_to_flat(psi, tx, nx, pl.TWO_SITE))
    res = pl.SvdResult(ctx, B1, B2, P, x, 10 ** 6, cutoff=0.0, eps=1e-4, mode=pl.ABSORB_RIGHT)
    ref = dmrg.svd_truncate(psi, Bond(bl), Bond(br), PQ, 10 ** 6, "right", cutoff=0.0, eps=1e-4)
    assert res.bond == dict(zip(ref.bond.qs, ref.bond.dims))
    lam_ref = np.concatenate([ref.lam[q] for q in ref.bond.qs])
    l1 = lam_ref.max()
    assert np.max(np.abs(res.lam - lam_ref)) <= 1e-13 * l1
    big = lam_ref > 1e-8 * l1
    assert np.max(np.abs(res.lam[big] - lam_ref[big]) / lam_ref[big]) <= 1e-6
    # A Lambda B rebuilds Psi
    Bn = pl.Bond(res.bond)
    ta, na = pl.layout(pl.SITE, B1, Bn, P)
    tb, nb = pl.layout(pl.SITE, Bn, B2, P)
    A = flat_to_blocks(host(res.A)[:na], ta, pl.SITE)
    R = flat_to_blocks(host(res.right)[:nb], tb, pl.SITE)
    back = dmrg.contract_two(A, R, PQ)
    keys = two_site_keys(Bond(bl), Bond(br), PQ)
    shapes = [two_site_shape(k, Bond(bl), Bond(br), PQ) for k in keys]
    err = np.linalg.norm(flatten(back, keys, shapes) - flatten(psi, keys, shapes))
    say("  reconstruction", err, "max lam err", np.max(np.abs(res.lam - lam_ref)) / l1)
    assert err <= 1e-13
    # orthonormality: A^T A = 1 per right sector, B B^T = 1 per left sector
    Bb = flat_to_blocks(host(res.B)[:nb], tb, pl.SITE)
    for q, n in res.bond.items():
        Ga = sum(A[(qa, s)].T @ A[(qa, s)] for (qa, s) in A if qa + PQ[s] == q)
        Gb = sum(Bb[(q2, s)] @ Bb[(q2, s)].T for (q2, s) in Bb if q2 == q)
        assert np.abs(Ga - np.eye(n)).max() <= 1e-12
        assert np.abs(Gb - np.eye(n)).max() <= 1e-12


def test_svd_truncation_matches_oracle(ctx):
    bl, br = synth.binomial_bond(30, 14, 160), synth.binomial_bond(30, 16, 160)
    rng = np.random.default_rng(5)
    psi = synth.random_two_site_blocks(bl, br, PQ, rng)
    nrm = np.sqrt(sum(float(np.sum(v * v)) for v in psi.values()))
    psi = {k: v / nrm for k, v in psi.items()}
    B1, B2, P = pl.Bond(bl), pl.Bond(br), pl.Phys(PQ)
    tx, nx = pl.layout(pl.TWO_SITE, B1, B2, P)
    x = dev(blocks_to_flat(psi, tx, nx, pl.TWO_SITE))
    for m in (1, 7, 60, 159):
        res = pl.SvdResult(ctx, B1, B2, P, x, m, mode=pl.ABSORB_LEFT)
        ref = dmrg.svd_truncate(psi, Bond(bl), Bond(br), PQ, m, "left")
        assert res.bond == dict(zip(ref.bond.qs, ref.bond.dims)), m      # bit-exact bookkeeping
        assert abs(res.discarded - ref.discarded) <= 1e-12
        lam_ref = np.concatenate([ref.lam[q] for q in ref.bond.qs])
        assert np.max(np.abs(res.lam - lam_ref)) <= 1e-12


def test_split_then_merge_round_trip(ctx):
    bl, br = synth.binomial_bond(20, 9, 70), synth.binomial_bond(20, 11, 70)
    psi = _graded_psi(bl, br, 9, 1e-6)
    B1, B2, P = pl.Bond(bl), pl.Bond(br), pl.Phys(PQ)
    tx, nx = pl.layout(pl.TWO_SITE, B1, B2, P)
    x = dev(blocks_to_flat(psi, tx, nx, pl.TWO_SITE))
    res = pl.SvdResult(ctx, B1, B2, P, x, 10 ** 6, cutoff=0.0, mode=pl.SPLIT)
    assert np.allclose(res.V * res.lam, 1.0, rtol=1e-15)
    out = dev(np.zeros(nx))
    pl.merge_regions(ctx, B1, pl.Bond(res.bond), B2, P, res.left, dev(res.V), res.right, out)
    err = np.linalg.norm(host(out) - host(x))
    say("  split/merge round trip", err)
    assert err <= 1e-12


def _middle_blocks(psi, bl, br):
    """The middle-charge blocks of Psi as dense matrices (rows (s1, a), columns
    (s2, b)), keyed by charge."""
    Bl, Br = Bond(bl), Bond(br)
    out = {}
    for qm in sorted({q + s for q in Bl.qs for s in PQ}):
        rows = [(s1, qm - PQ[s1]) for s1 in range(2) if Bl.has(qm - PQ[s1])]
        cols = [(s2, qm + PQ[s2]) for s2 in range(2) if Br.has(qm + PQ[s2])]
        if rows and cols:
            out[qm] = np.block([[psi[(qa, s1, s2)] for (s2, qb) in cols] for (s1, qa) in rows])
    return out


def _mp_singular_values(M, dps=40):
    import mpmath
    mpmath.mp.dps = dps
    s = mpmath.svd_r(mpmath.matrix(M.tolist()), compute_uv=False)
    return np.array(sorted((float(v) for v in s), reverse=True))


@pytest.fixture(scope="module")
def mp_ref():
    bl, br = {-1: 24, 1: 24}, {-1: 28, 1: 28}
    psi = _graded_psi(bl, br, 11, 1e-12)
    ref = np.concatenate([_mp_singular_values(M_) for q, M_ in sorted(_middle_blocks(psi, bl, br).items())])
    return bl, br, psi, ref / np.sqrt(np.sum(ref ** 2))


@pytest.mark.parametrize("pre", [0, 2])
@pytest.mark.parametrize("mode", [pl.ABSORB_RIGHT, pl.ABSORB_LEFT, pl.SPLIT])
def test_svd_small_values_relative_accuracy(ctx, mp_ref, mode, pre):
    """Appendix accuracy on the GPU: graded blocks (24 x 28, 48 x 56, 24 x 28,
    singular values from 1 down to 1e-12 with random orthogonal factors)
    against 40-digit singular values of the same FP64 blocks (mpmath): every
    lambda, and V = 1/lambda where it is not floored, to 1e-5 relative down to
    1e-12 lambda_1, in all three modes, with the Jacobi iteration on the
    blocks themselves (pre 0) and on their QR factors (pre 2)."""
    bl, br, psi, ref = mp_ref
    B1, B2, P = pl.Bond(bl), pl.Bond(br), pl.Phys(PQ)
    tx, nx = pl.layout(pl.TWO_SITE, B1, B2, P)
    x = dev(blocks_to_flat(psi, tx, nx, pl.TWO_SITE))
    pl.set_svd_precondition(ctx, pre)
    try:
        res = pl.SvdResult(ctx, B1, B2, P, x, 10 ** 6, cutoff=0.0, eps=1e-4, mode=mode)
    finally:
        pl.set_svd_precondition(ctx, 1)
    assert res.lam.size == ref.size
    lmax = ref.max()
    ok = ref >= 1e-12 * lmax
    rel = np.abs(res.lam - ref) / ref
    say("  mode", mode, "smallest lambda/lambda_1 %.2e" % (ref.min() / lmax),
        "max rel err %.2e" % rel[ok].max())
    assert rel[ok].max() <= 1e-5
    if mode == pl.SPLIT:
        lam_max = res.lam.max()
        unfl = res.lam >= 1e-12 * lam_max
        assert np.abs(res.V[unfl] * ref[unfl] - 1.0).max() <= 1e-5
        assert np.allclose(res.V[~unfl], 1.0 / (1e-12 * lam_max), rtol=1e-15)


@pytest.mark.parametrize("max_m", sorted(TIE_CASES))
def test_svd_truncation_tie_break(ctx, max_m):
    """Exactly degenerate singular values in the q = -2 and q = +2 sectors with
    max_m cutting the multiplet (R1): the GPU keeps the smaller charge, and its
    bond table equals the oracle's bit for bit."""
    bl, br, psi = tie_psi()
    B1, B2, P = pl.Bond(bl), pl.Bond(br), pl.Phys(PQ)
    tx, nx = pl.layout(pl.TWO_SITE, B1, B2, P)
    x = dev(blocks_to_flat(psi, tx, nx, pl.TWO_SITE))
    ref = dmrg.svd_truncate(psi, Bond(bl), Bond(br), PQ, max_m, "right", cutoff=0.0)
    for mode in (pl.ABSORB_RIGHT, pl.ABSORB_LEFT, pl.SPLIT):
        res = pl.SvdResult(ctx, B1, B2, P, x, max_m, cutoff=0.0, mode=mode)
        assert res.bond == dict(zip(ref.bond.qs, ref.bond.dims)) == TIE_CASES[max_m]


def _dmrg_graded_psi(bl, br, seed, rate):
    """Two-site blocks graded the way a DMRG state's are: within each
    (s, sector) segment of rows and of columns the weights fall like a Schmidt
    spectrum, exp(-rate sqrt(k)), around a random Gaussian core."""
    rng = np.random.default_rng(seed)
    Bl, Br = Bond(bl), Bond(br)
    psi = {}
    for qa in Bl.qs:
        for s1 in range(2):
            for s2 in range(2):
                qb = qa + PQ[s1] + PQ[s2]
                if not Br.has(qb):
                    continue
                wr = np.exp(-rate * np.sqrt(np.arange(Bl.dim(qa)) + 0.3 * s1))
                wc = np.exp(-rate * np.sqrt(np.arange(Br.dim(qb)) + 0.3 * s2))
                psi[(qa, s1, s2)] = (wr[:, None] * rng.standard_normal((Bl.dim(qa), Br.dim(qb)))) * wc[None, :]
    nrm = np.sqrt(sum(float(np.sum(v * v)) for v in psi.values()))
    return {k: v / nrm for k, v in psi.items()}


@pytest.mark.parametrize("shape", ["wide", "tall"])
def test_svd_qr_preconditioned_large_blocks(ctx, shape):
    """Middle-charge blocks of 300 x 500, 700 x 1100 and 400 x 600 (or their
    transposes), graded like a DMRG state's: the QR-preconditioned Jacobi
    iteration (several chunks and panels, the longest panel rows) gives the
    singular values of LAPACK's SVD of the same blocks to 1e-13 lambda_1 and
    those of the plain iteration to 1e-6 relative above 1e-8 lambda_1, and its
    factors rebuild Psi and are orthonormal."""
    import time
    import torch
    a, b = {-1: 300, 1: 400}, {-1: 500, 1: 600}
    bl, br = (a, b) if shape == "wide" else (b, a)
    psi = _dmrg_graded_psi(bl, br, 21, 0.9)
    ref = np.sort(np.concatenate([np.linalg.svd(M_, compute_uv=False)
                                  for M_ in _middle_blocks(psi, bl, br).values()]))[::-1]
    B1, B2, P = pl.Bond(bl), pl.Bond(br), pl.Phys(PQ)
    tx, nx = pl.layout(pl.TWO_SITE, B1, B2, P)
    x = dev(blocks_to_flat(psi, tx, nx, pl.TWO_SITE))
    out = {}
    for pre in (0, 1):
        pl.set_svd_precondition(ctx, pre)
        try:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = pl.SvdResult(ctx, B1, B2, P, x, 10 ** 6, cutoff=0.0, eps=1e-4, mode=pl.ABSORB_RIGHT)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        finally:
            pl.set_svd_precondition(ctx, 1)
        assert res.code == 0, "Jacobi iteration did not converge"
        out[pre] = res
        lam = np.sort(res.lam)[::-1]
        say("  pre", pre, "seconds %.4f" % dt, "max |lam - lapack| / lam_1 %.2e" % (np.abs(lam - ref).max() / ref[0]))
        assert lam.size == ref.size
        assert np.abs(lam - ref).max() <= 1e-13 * ref[0]
    l0, l1 = np.sort(out[0].lam)[::-1], np.sort(out[1].lam)[::-1]
    big = l0 > 1e-8 * l0[0]
    assert (np.abs(l1[big] - l0[big]) / l0[big]).max() <= 1e-6
    assert out[1].bond == out[0].bond
    res = out[1]
    Bn = pl.Bond(res.bond)
    ta, na = pl.layout(pl.SITE, B1, Bn, P)
    tb, nb = pl.layout(pl.SITE, Bn, B2, P)
    A = flat_to_blocks(host(res.A)[:na], ta, pl.SITE)
    R = flat_to_blocks(host(res.right)[:nb], tb, pl.SITE)
    back = dmrg.contract_two(A, R, PQ)
    keys = two_site_keys(Bond(bl), Bond(br), PQ)
    shapes = [two_site_shape(k, Bond(bl), Bond(br), PQ) for k in keys]
    err = np.linalg.norm(flatten(back, keys, shapes) - flatten(psi, keys, shapes))
    say("  reconstruction", err)
    assert err <= 1e-13
    Bb = flat_to_blocks(host(res.B)[:nb], tb, pl.SITE)
    for q, n in res.bond.items():
        Ga = sum(A[(qa, s)].T @ A[(qa, s)] for (qa, s) in A if qa + PQ[s] == q)
        Gb = sum(Bb[(q2, s)] @ Bb[(q2, s)].T for (q2, s) in Bb if q2 == q)
        assert np.abs(Ga - np.eye(n)).max() <= 1e-12
        assert np.abs(Gb - np.eye(n)).max() <= 1e-12
