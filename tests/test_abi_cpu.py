"""Host-only checks of the C-ABI library (no GPU needed): it loads, exports
every declared entry point, its block bookkeeping equals the oracle's bit for
bit, and its MPO builder reproduces the Hamiltonians."""
import ctypes
import os
import re
from ctypes import POINTER, byref, c_double, c_int32, c_void_p

import numpy as np
import pytest

from helpers import ROOT, pl, synth
from oracle import models, mpo as M, dmrg
from oracle.blocks import Bond, two_site_keys, two_site_shape, site_keys, site_shape, env_keys


def _lib():
    return pl.lib()


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "pdmrg.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    names = set(re.findall(r"^\s*(?:const\s+)?(?:int|void|char)\s*\*?\s*(\w+)\s*\(", hdr, flags=re.M))
    assert len(names) >= 30
    L = _lib()
    for n in sorted(names):
        assert hasattr(L, n), n
    assert set(pl.EXPORTS) == names


def _bonds():
    return [({-3: 2, -1: 5, 1: 4, 3: 1}, {-2: 3, 0: 6, 2: 2, 4: 1}),
            ({0: 1}, {-1: 1, 1: 1}),
            (synth.binomial_bond(20, 9, 70), synth.binomial_bond(20, 11, 70))]


@pytest.mark.parametrize("case", range(3))
def test_two_site_layout_matches_oracle_bookkeeping(case):
    bl, br = _bonds()[case]
    PQ = (-1, 1)
    blocks, n = pl.layout(pl.TWO_SITE, pl.Bond(bl), pl.Bond(br), pl.Phys(PQ))
    keys = two_site_keys(Bond(bl), Bond(br), PQ)
    assert [b[0] for b in blocks] == keys          # same blocks, same order
    for (key, off, rows, cols, ld), k in zip(blocks, keys):
        assert (rows, cols) == two_site_shape(k, Bond(bl), Bond(br), PQ)
    assert n == sum(r * c for _, _, r, c, _ in blocks)
    # no two blocks overlap
    cover = np.zeros(n, int)
    for key, off, rows, cols, ld in blocks:
        for r in range(rows):
            cover[off + r * ld: off + r * ld + cols] += 1
    assert np.all(cover == 1)


@pytest.mark.parametrize("case", range(3))
def test_site_layout_matches_oracle_bookkeeping(case):
    bl, br = _bonds()[case]
    bl2 = {q + 1: n for q, n in br.items()}          # a bond one site to the right
    for (a, b) in ((bl, {q + 1: n for q, n in bl.items()}), (br, bl2)):
        blocks, n = pl.layout(pl.SITE, pl.Bond(a), pl.Bond(b), pl.Phys((-1, 1)))
        keys = site_keys(Bond(a), Bond(b), (-1, 1))
        assert [(bk[0][0], bk[0][1]) for bk in blocks] == keys
        for (key, off, rows, cols, ld), k in zip(blocks, keys):
            assert (rows, cols) == site_shape(k, Bond(a), Bond(b), (-1, 1))


@pytest.mark.parametrize("kind", [pl.ENV_L, pl.ENV_R])
def test_env_layout_matches_oracle_bookkeeping(kind):
    bond = {-4: 2, -2: 3, 0: 5, 2: 4, 4: 1}
    deltas = [0, 2, -2, 0, 0]
    blocks, n = pl.layout(kind, pl.Bond(bond), deltas=deltas)
    keys = set(env_keys(Bond(bond), deltas))
    assert set(b[0][:2] for b in blocks) == keys and len(blocks) == len(keys)
    B = Bond(bond)
    for key, off, rows, cols, ld in blocks:
        q, w = key[:2]
        shape = (B.dim(q), B.dim(q - deltas[w]))
        assert (rows, cols) == (shape if kind == pl.ENV_L else shape[::-1])
    cover = np.zeros(n, int)
    for key, off, rows, cols, ld in blocks:
        for r in range(rows):
            cover[off + r * ld: off + r * ld + cols] += 1
    assert np.all(cover == 1)


def _lib_mpo(lattice, Lx, Ly, c):
    L = _lib()
    h = c_void_p()
    cc = (c_double * 2)(*c)
    pl.check(L.mpo_build(lattice, Lx, Ly, cc, 2, byref(h)))
    n, d = c_int32(), c_int32()
    pl.check(L.mpo_info(h, byref(n), byref(d), None, None))
    D = np.zeros(n.value + 1, np.int32)
    pq = np.zeros(d.value, np.int32)
    pl.check(L.mpo_info(h, None, None, pq.ctypes.data_as(POINTER(c_int32)), D.ctypes.data_as(POINTER(c_int32))))
    Ws, deltas = [], []
    for i in range(n.value):
        W = np.zeros((D[i], d.value, d.value, D[i + 1]))
        dl = np.zeros(D[i], np.int32)
        dr = np.zeros(D[i + 1], np.int32)
        pl.check(L.mpo_get_site(h, i, W.ctypes.data_as(POINTER(c_double)), dl.ctypes.data_as(POINTER(c_int32)),
                                dr.ctypes.data_as(POINTER(c_int32))))
        Ws.append(W)
        deltas.append(dl)
    deltas.append(dr)
    L.mpo_free(h)
    return M.MPO(Ws, [list(range(len(x))) for x in deltas], deltas, tuple(pq)), D


@pytest.mark.parametrize("lattice,Lx,Ly,c,terms", [
    (0, 8, 1, (1.0, 0.8), lambda: models.xxz_terms(models.chain_bonds(8), 1.0, 0.8)),
    (1, 3, 3, (1.0, 1.0), lambda: models.heisenberg_terms(models.square_cylinder_bonds(3, 3))),
    (2, 3, 3, (0.9, 1.1), lambda: models.xxz_terms(models.triangular_cylinder_bonds(3, 3), 0.9, 1.1)),
    (3, 3, 3, (1.0, 0.7), lambda: models.jq2_terms(3, 3, 1.0, 0.7)),
    (4, 7, 1, (1.0, 0.6), lambda: models.tfim_terms(7, 1.0, 0.6)),
])
def test_library_mpo_builder_reproduces_hamiltonian(lattice, Lx, Ly, c, terms):
    mpo, D = _lib_mpo(lattice, Lx, Ly, c)
    N = mpo.N
    H = M.mpo_to_dense(mpo)
    Href = M.terms_to_dense(terms(), N, models.OPS)
    assert np.abs(H - Href).max() <= 1e-13 * np.abs(Href).max()
    # same channel structure as the oracle's builder: D and channel-charge multisets
    phys = (0, 0) if lattice == 4 else (-1, 1)
    ref = M.build_mpo(terms(), N, models.OPS, phys)
    assert [ref.D(b) for b in range(N + 1)] == list(D)
    for b in range(N + 1):
        assert sorted(ref.deltas[b]) == sorted(mpo.deltas[b])
    for i, W in enumerate(mpo.W):
        for wl, s, t, wr in zip(*np.nonzero(W)):
            assert mpo.deltas[i][wl] + phys[s] - phys[t] == mpo.deltas[i + 1][wr]


def test_mpo_bulk_dimension_of_benchmark_lattices():
    _, D2 = _lib_mpo(1, 8, 4, (1.0, 1.0))
    assert D2.max() == 14                       # 3 Ly + 2
    _, D3 = _lib_mpo(1, 24, 8, (1.0, 1.0))
    assert D3.max() == 26
    _, D4 = _lib_mpo(2, 12, 6, (1.0, 1.0))
    assert D4.max() == 23                       # 3 (Ly + 1) + 2


def test_jq2_mpo_of_the_16x8_cylinder_against_operator_schmidt_ranks():
    """The library's J-Q2 MPO on the 16 x 8 cylinder (the m = 4000 workload):
    D is never below the operator-Schmidt rank of the Hamiltonian across any
    cut and equals it, 98 = 2 + 3 Ly + 9 Ly, at every bulk column cut (the
    largest rank of the lattice); inside a column the prefix machine keeps
    110 channels where the rank is 80."""
    from test_oracle_pins import product_basis_rank
    Lx, Ly = 16, 8
    N = Lx * Ly
    _, D = _lib_mpo(3, Lx, Ly, (1.0, 0.7))
    terms = models.jq2_terms(Lx, Ly, 1.0, 0.7)
    ranks = [product_basis_rank(terms, c) for c in range(1, N)]
    assert all(D[c] >= ranks[c - 1] for c in range(1, N))
    for x in range(2, Lx - 1):
        assert D[x * Ly] == ranks[x * Ly - 1] == 2 + 12 * Ly
    assert max(ranks) == 98 and D.max() == 110
    assert ranks[Ly * Lx // 2 + 2] == 80


def test_errors_are_reported_not_raised():
    L = _lib()
    h = c_void_p()
    cc = (c_double * 2)(1.0, 1.0)
    assert L.mpo_build(99, 4, 1, cc, 2, byref(h)) == -1
    assert b"unknown lattice" in L.pdmrg_last_error()
    # a bond with descending charges is rejected by the bookkeeping
    q = np.array([2, 0], np.int32)
    d = np.array([1, 1], np.int32)
    b = pl.CBond(2, q.ctypes.data_as(POINTER(c_int32)), d.ctypes.data_as(POINTER(c_int32)))
    n, nb = ctypes.c_int64(), ctypes.c_int32()
    P = pl.Phys((-1, 1))
    assert L.pdmrg_layout_size(pl.TWO_SITE, byref(b), byref(b), P.ref, None, 0, byref(n), byref(nb)) == -1


def test_autotune_cache_file_round_trip(tmp_path):
    """The tuning cache file format: an empty export, an import of a
    hand-written entry, re-export, and rejection of malformed lines."""
    from helpers import pl
    p = tmp_path / "tune.txt"
    n0 = pl.autotune_export(p)
    p.write_text("sig-a\t1\t5\t4\n")
    assert pl.autotune_import(p) == 1
    q = tmp_path / "tune2.txt"
    assert pl.autotune_export(q) == n0 + 1
    assert "sig-a\t1\t5\t4" in q.read_text()
    bad = tmp_path / "bad.txt"
    bad.write_text("sig-b\t1\t99\t4\n")
    with pytest.raises(pl.PdmrgError):
        pl.autotune_import(bad)
    with pytest.raises(pl.PdmrgError):
        pl.autotune_import(tmp_path / "missing.txt")


def test_sweep_concurrency_field_mapping():
    """The binding passes the sweep's region mode as the C field expects:
    False / 0 one after the other, True / 1 own streams, 2 lockstep with
    batched SVDs; anything else is refused before reaching the library."""
    assert pl._concurrency(False) == 0 and pl._concurrency(0) == 0
    assert pl._concurrency(True) == 1 and pl._concurrency(1) == 1
    assert pl._concurrency(np.bool_(True)) == 1
    assert pl._concurrency(2) == 2
    for bad in (3, -1, "2"):
        with pytest.raises(ValueError):
            pl._concurrency(bad)
