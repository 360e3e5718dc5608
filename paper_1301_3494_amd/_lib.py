"""ctypes binding of libpdmrg.so (include/pdmrg.h): argument marshalling only.

Every computation happens inside the HIP library; this module converts Python
bond / MPO descriptions into the C structs and device tensors into pointers.
It raises immediately if the library has not been built.
"""
import ctypes
import os
from ctypes import POINTER, Structure, byref, c_char_p, c_double, c_int, c_int32, c_int64, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpdmrg.so")

F64, F32, BF16X3 = 0, 1, 2
SITE, TWO_SITE, ENV_L, ENV_R = 0, 1, 2, 3
ABSORB_RIGHT, ABSORB_LEFT, SPLIT = 0, 1, 2
WARN_NOT_CONVERGED, WARN_V_FLOORED = 1, 2
PREC_NAMES = {"f64": F64, "f32": F32, "bf16x3": BF16X3}


class CBond(Structure):
    _fields_ = [("nsec", c_int32), ("q", POINTER(c_int32)), ("dim", POINTER(c_int32))]


class CPhys(Structure):
    _fields_ = [("d", c_int32), ("q", POINTER(c_int32))]


class CMpoSite(Structure):
    _fields_ = [("Dl", c_int32), ("Dr", c_int32), ("d", c_int32), ("W", POINTER(c_double)),
                ("dl", POINTER(c_int32)), ("dr", POINTER(c_int32))]


class CDavParams(Structure):
    _fields_ = [("max_matvec", c_int32), ("max_sub", c_int32), ("tol", c_double)]


class CSweepParams(Structure):
    _fields_ = [("max_m", c_int32), ("n_regions", c_int32), ("prec", c_int32), ("refine", c_int32),
                ("dav", CDavParams), ("dav_shared", CDavParams), ("cutoff", c_double), ("eps", c_double),
                ("concurrent", c_int32), ("pad_", c_int32)]


class CSweepReport(Structure):
    _fields_ = [("energy", c_double), ("max_trunc", c_double), ("seconds", c_double),
                ("seconds_heff", c_double), ("n_matvec", c_int64), ("n_floored", c_int32),
                ("max_bond", c_int32), ("max_infidelity", c_double),
                ("n_svd_unconverged", c_int32), ("pad_", c_int32), ("seconds_svd", c_double),
                ("seconds_env", c_double)]


class PdmrgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("pdmrg error %d: %s" % (code, msg))
        self.code = code


_lib = None


def lib():
    """Load libpdmrg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpdmrg.so not built: run paper_1301_3494_amd/build.py (or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        _declare(L)
        _lib = L
    return _lib


EXPORTS = [
    "pdmrg_last_error", "pdmrg_version", "pdmrg_ctx_create", "pdmrg_ctx_destroy", "pdmrg_ctx_set_timing",
    "pdmrg_ctx_timing", "pdmrg_ctx_set_autotune", "pdmrg_set_alloc_poison", "pdmrg_ctx_set_env_stride",
    "pdmrg_ctx_set_verbose",
    "pdmrg_ctx_set_svd_precondition",
    "pdmrg_memory_stats", "pdmrg_ctx_set_graphs", "pdmrg_autotune_export", "pdmrg_autotune_import", "pdmrg_layout_size", "pdmrg_layout_blocks", "mpo_build", "mpo_from_sites",
    "mpo_info", "mpo_get_site", "mpo_free", "heff_create", "heff_apply", "heff_info", "heff_plan_info", "heff_diag",
    "heff_free", "env_update", "env_update_noalloc", "env_update_info", "davidson_step", "svd_truncate", "svd_result_bond", "svd_result_copy",
    "svd_free", "merge_regions", "mps_alloc", "mps_set_site", "mps_bond", "mps_get_site", "sweep",
    "mps_energy", "mps_copy", "mps_free", "grad_site", "grad_mpo", "grad_couplings", "mps_inverse_canonical", "mps_get_v", "mps_expect_site",
    "mps_expect_pairs", "mps_order_parameter",
]


def _declare(L):
    P = c_void_p
    pb, pp, pm = POINTER(CBond), POINTER(CPhys), POINTER(CMpoSite)
    pi32, pi64, pd = POINTER(c_int32), POINTER(c_int64), POINTER(c_double)
    sig = {
        "pdmrg_last_error": (c_char_p, []),
        "pdmrg_version": (c_char_p, []),
        "pdmrg_ctx_create": (c_int, [c_int, P, POINTER(P)]),
        "pdmrg_ctx_destroy": (c_int, [P]),
        "pdmrg_ctx_set_timing": (c_int, [P, c_int]),
        "pdmrg_ctx_timing": (c_int, [P, pd, pi64]),
        "pdmrg_ctx_set_autotune": (c_int, [P, c_int]),
        "pdmrg_ctx_set_graphs": (c_int, [P, c_int]),
        "pdmrg_autotune_export": (c_int, [c_char_p, pi32]),
        "pdmrg_set_alloc_poison": (c_int, [c_int]),
        "pdmrg_ctx_set_env_stride": (c_int, [P, c_int]),
        "pdmrg_ctx_set_verbose": (c_int, [P, c_int]),
        "pdmrg_ctx_set_svd_precondition": (c_int, [P, c_int]),
        "pdmrg_memory_stats": (c_int, [pi64, pi64, pi64, c_int]),
        "pdmrg_autotune_import": (c_int, [c_char_p, pi32]),
        "pdmrg_layout_size": (c_int, [c_int, pb, pb, pp, pi32, c_int32, pi64, pi32]),
        "pdmrg_layout_blocks": (c_int, [c_int, pb, pb, pp, pi32, c_int32, pi32, pi64, pi32, pi32, pi32]),
        "mpo_build": (c_int, [c_int, c_int, c_int, pd, c_int, POINTER(P)]),
        "mpo_from_sites": (c_int, [c_int, pm, POINTER(P)]),
        "mpo_info": (c_int, [P, pi32, pi32, pi32, pi32]),
        "mpo_get_site": (c_int, [P, c_int, pd, pi32, pi32]),
        "mpo_free": (None, [P]),
        "heff_create": (c_int, [P, pb, pb, pp, pm, pm, P, P, c_int, POINTER(P)]),
        "heff_apply": (c_int, [P, P, P, P]),
        "heff_info": (c_int, [P, pd, pd, pd, pi64, pi64, pi64, pi64, pi64]),
        "heff_diag": (c_int, [P, P, P]),
        "heff_plan_info": (c_int, [P, pi32, pi32, pi32, pi32, pi32]),
        "heff_free": (None, [P]),
        "env_update": (c_int, [P, c_int, pb, pb, pp, pm, P, P, P, c_int]),
        "env_update_noalloc": (c_int, [P, c_int, pb, pb, pp, pm, P, P, P, c_int]),
        "env_update_info": (c_int, [c_int, pb, pb, pp, pm, pd, pi64]),
        "davidson_step": (c_int, [P, P, P, P, POINTER(CDavParams), pd, pd, pi32]),
        "svd_truncate": (c_int, [P, pb, pb, pp, P, c_int32, c_double, c_double, c_int, POINTER(P)]),
        "svd_result_bond": (c_int, [P, pi32, pi32, pi32, c_int32, pd, pi32]),
        "svd_result_copy": (c_int, [P, P, P, P, P, P, pd, pd]),
        "svd_free": (None, [P]),
        "merge_regions": (c_int, [P, pb, pb, pb, pp, P, P, P, P]),
        "mps_alloc": (c_int, [P, c_int, pp, c_int32, pb, POINTER(P)]),
        "mps_set_site": (c_int, [P, c_int, pd, c_int64]),
        "mps_bond": (c_int, [P, c_int, pi32, pi32, pi32, c_int32]),
        "mps_get_site": (c_int, [P, c_int, pd, c_int64]),
        "sweep": (c_int, [P, P, P, POINTER(CSweepParams), POINTER(CSweepReport)]),
        "mps_copy": (c_int, [P, P, POINTER(c_void_p)]),
        "mps_energy": (c_int, [P, P, P, pd]),
        "mps_free": (None, [P]),
        "grad_site": (c_int, [P, pb, pb, pp, pm, P, P, P, P]),
        "grad_mpo": (c_int, [P, P, P, P, c_int64, pd]),
        "grad_couplings": (c_int, [P, P, P, pd, c_int32, pd]),
        "mps_inverse_canonical": (c_int, [P, P, c_double, c_double, pi32]),
        "mps_get_v": (c_int, [P, c_int, pd, c_int64]),
        "mps_expect_site": (c_int, [P, P, pd, pd]),
        "mps_expect_pairs": (c_int, [P, P, c_int, pd, pd, pd, c_int, pi32, pi32, c_int, pd]),
        "mps_order_parameter": (c_int, [P, P, c_int, c_int, c_int, pd]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args


def check(code, allow_warn=False):
    if code < 0 or (code > 0 and not allow_warn):
        msg = lib().pdmrg_last_error()
        raise PdmrgError(code, msg.decode() if msg else "")
    return code


# ---------------------------------------------------------------- marshalling
class Bond:
    """Host bond descriptor {charge: dim}; keeps the arrays alive."""

    def __init__(self, sectors):
        items = sorted((int(q), int(n)) for q, n in dict(sectors).items() if int(n) > 0)
        self.sectors = dict(items)
        self.q = np.array([q for q, _ in items], dtype=np.int32)
        self.dim = np.array([n for _, n in items], dtype=np.int32)
        self.c = CBond(len(items), self.q.ctypes.data_as(POINTER(c_int32)),
                       self.dim.ctypes.data_as(POINTER(c_int32)))

    @property
    def ref(self):
        return byref(self.c)


class Phys:
    def __init__(self, qs):
        self.q = np.array(qs, dtype=np.int32)
        self.c = CPhys(len(qs), self.q.ctypes.data_as(POINTER(c_int32)))

    @property
    def ref(self):
        return byref(self.c)


class MpoSite:
    def __init__(self, W, dl, dr):
        self.W = np.ascontiguousarray(W, dtype=np.float64)
        self.dl = np.ascontiguousarray(dl, dtype=np.int32)
        self.dr = np.ascontiguousarray(dr, dtype=np.int32)
        Dl, d, _, Dr = self.W.shape
        self.c = CMpoSite(Dl, Dr, d, self.W.ctypes.data_as(POINTER(c_double)),
                          self.dl.ctypes.data_as(POINTER(c_int32)), self.dr.ctypes.data_as(POINTER(c_int32)))

    @property
    def ref(self):
        return byref(self.c)


def layout(kind, b1, b2=None, phys=None, deltas=None):
    """Block table of a layout: list of (key tuple, offset, rows, cols, ld) and
    the total element count."""
    L = lib()
    dl = None if deltas is None else np.ascontiguousarray(deltas, dtype=np.int32)
    dptr = None if dl is None else dl.ctypes.data_as(POINTER(c_int32))
    nd = 0 if dl is None else len(dl)
    b2r = None if b2 is None else b2.ref
    pr = None if phys is None else phys.ref
    n, nb = c_int64(), c_int32()
    check(L.pdmrg_layout_size(kind, b1.ref, b2r, pr, dptr, nd, byref(n), byref(nb)))
    k = np.zeros((max(nb.value, 1), 3), np.int32)
    off = np.zeros(max(nb.value, 1), np.int64)
    r = np.zeros(max(nb.value, 1), np.int32)
    c = np.zeros(max(nb.value, 1), np.int32)
    ld = np.zeros(max(nb.value, 1), np.int32)
    check(L.pdmrg_layout_blocks(kind, b1.ref, b2r, pr, dptr, nd,
                                k.ctypes.data_as(POINTER(c_int32)), off.ctypes.data_as(POINTER(c_int64)),
                                r.ctypes.data_as(POINTER(c_int32)), c.ctypes.data_as(POINTER(c_int32)),
                                ld.ctypes.data_as(POINTER(c_int32))))
    blocks = [(tuple(int(v) for v in k[i]), int(off[i]), int(r[i]), int(c[i]), int(ld[i]))
              for i in range(nb.value)]
    return blocks, n.value


def ptr(t):
    """Device pointer of a torch tensor (or None)."""
    return None if t is None else c_void_p(t.data_ptr())


class Context:
    """pdmrg context bound to a torch CUDA (HIP) device and stream."""

    def __init__(self, device=0, stream=None):
        import torch
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = c_void_p()
        check(lib().pdmrg_ctx_create(device, c_void_p(self.stream.cuda_stream), byref(h)))
        self.h = h

    def close(self):
        if self.h:
            lib().pdmrg_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- operations
class Heff:
    """heff_create / heff_apply / heff_info / heff_diag / heff_free."""

    def __init__(self, ctx, bl, br, phys, W1, W2, L, R, prec=F64):
        self.ctx = ctx
        self._keep = (bl, br, phys, W1, W2)
        h = c_void_p()
        check(lib().heff_create(ctx.h, bl.ref, br.ref, phys.ref, W1.ref, W2.ref, ptr(L), ptr(R), int(prec),
                                byref(h)))
        self.h = h

    def apply(self, x, y):
        check(lib().heff_apply(self.ctx.h, self.h, ptr(x), ptr(y)))

    def info(self):
        f = [c_double() for _ in range(3)]
        n = [c_int64() for _ in range(5)]
        check(lib().heff_info(self.h, *[byref(v) for v in f], *[byref(v) for v in n]))
        keys = ["n_psi", "n_L", "n_R", "n_T1", "n_T2"]
        out = dict(flops_Lpsi=f[0].value, flops_W=f[1].value, flops_R=f[2].value)
        out.update({k: v.value for k, v in zip(keys, n)})
        out["flops"] = out["flops_Lpsi"] + out["flops_W"] + out["flops_R"]
        v = [c_int32() for _ in range(5)]
        check(lib().heff_plan_info(self.h, *[byref(x) for x in v]))
        names = ["64x64", "128x32", "32x128", "128x128", "64x64k16", "128x32k16", "64x64k8", "128x32k8",
                 "128x32dma", "64x64dma", "32x128dma"]
        out.update(shape_Lpsi=names[v[0].value], shape_R=names[v[1].value], tiles_Lpsi=v[2].value,
                   tiles_R=v[3].value, splitk_parts=v[4].value)
        return out

    def diag(self, out):
        check(lib().heff_diag(self.ctx.h, self.h, ptr(out)))

    def free(self):
        if self.h:
            lib().heff_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def env_update(ctx, direction, bl, br, phys, W, env_in, site, env_out, prec=F64):
    check(lib().env_update(ctx.h, int(direction), bl.ref, br.ref, phys.ref, W.ref, ptr(env_in), ptr(site),
                           ptr(env_out), int(prec)))


def env_update_noalloc(ctx, direction, bl, br, phys, W, env_in, site, env_out, prec=F64):
    """env_update through the entry point that allocates no device memory."""
    check(lib().env_update_noalloc(ctx.h, int(direction), bl.ref, br.ref, phys.ref, W.ref, ptr(env_in), ptr(site),
                                   ptr(env_out), int(prec)))


def env_update_info(direction, bl, br, phys, W):
    """(algorithmic flops, output elements) of env_update (host only)."""
    f, n = c_double(), c_int64()
    check(lib().env_update_info(int(direction), bl.ref, br.ref, phys.ref, W.ref, byref(f), byref(n)))
    return f.value, n.value


def davidson_step(ctx, op, psi, max_matvec=20, max_sub=8, tol=1e-10, op64=None):
    p = CDavParams(int(max_matvec), int(max_sub), float(tol))
    E, r, n = c_double(), c_double(), c_int32()
    code = check(lib().davidson_step(ctx.h, op.h, None if op64 is None else op64.h, ptr(psi), byref(p),
                                     byref(E), byref(r), byref(n)), allow_warn=True)
    return E.value, r.value, n.value, code


def merge_regions(ctx, bl, bm, br, phys, psiL, V, psiR, out):
    check(lib().merge_regions(ctx.h, bl.ref, bm.ref, br.ref, phys.ref, ptr(psiL), ptr(V), ptr(psiR), ptr(out)))


def timing(ctx, enable=None):
    if enable is not None:
        check(lib().pdmrg_ctx_set_timing(ctx.h, int(bool(enable))))
        return None
    ms = (c_double * 5)()
    n = c_int64()
    check(lib().pdmrg_ctx_timing(ctx.h, ms, byref(n)))
    return list(ms), n.value


def set_alloc_poison(on):
    """Debugging aid: NaN-fill every device buffer the library hands out."""
    check(lib().pdmrg_set_alloc_poison(1 if on else 0))


def autotune_export(path):
    n = c_int32()
    check(lib().pdmrg_autotune_export(str(path).encode(), byref(n)))
    return n.value


def autotune_import(path):
    n = c_int32()
    check(lib().pdmrg_autotune_import(str(path).encode(), byref(n)))
    return n.value


def set_graphs(ctx, enable):
    """heff_apply through captured HIP graphs (one per (x, y) pair)."""
    check(lib().pdmrg_ctx_set_graphs(ctx.h, int(bool(enable))))


def set_autotune(ctx, level):
    """Tile-shape selection of H_eff plans built afterwards on ctx: 0 cost
    model, 1 timed and cached per block signature, 2 = 1 with a log line."""
    check(lib().pdmrg_ctx_set_autotune(ctx.h, int(level)))


LATTICES = {"chain": 0, "square": 1, "triangular": 2, "jq2": 3, "tfim": 4, "chain_s1": 5}


class Mpo:
    """mpo_build (or mpo_from_sites) handle with its site tensors exported."""

    def __init__(self, lattice=None, Lx=None, Ly=1, couplings=(1.0, 1.0), sites=None):
        L = lib()
        h = c_void_p()
        if sites is not None:
            arr = (CMpoSite * len(sites))(*[s.c for s in sites])
            self._keep = sites
            check(L.mpo_from_sites(len(sites), arr, byref(h)))
        else:
            cc = (c_double * len(couplings))(*couplings)
            check(L.mpo_build(LATTICES.get(lattice, lattice), int(Lx), int(Ly), cc, len(couplings), byref(h)))
        self.ncouplings = 0 if sites is not None else len(couplings)
        self.h = h
        n, d = c_int32(), c_int32()
        check(L.mpo_info(h, byref(n), byref(d), None, None))
        self.N, self.d = n.value, d.value
        D = np.zeros(self.N + 1, np.int32)
        pq = np.zeros(self.d, np.int32)
        check(L.mpo_info(h, None, None, pq.ctypes.data_as(POINTER(c_int32)), D.ctypes.data_as(POINTER(c_int32))))
        self.D, self.phys_q = D, tuple(int(v) for v in pq)
        self.W, self.deltas = [], []
        for i in range(self.N):
            W = np.zeros((D[i], self.d, self.d, D[i + 1]))
            dl = np.zeros(D[i], np.int32)
            dr = np.zeros(D[i + 1], np.int32)
            check(L.mpo_get_site(h, i, W.ctypes.data_as(POINTER(c_double)), dl.ctypes.data_as(POINTER(c_int32)),
                                 dr.ctypes.data_as(POINTER(c_int32))))
            self.W.append(W)
            self.deltas.append(dl)
        self.deltas.append(dr)

    def site(self, i):
        return MpoSite(self.W[i], self.deltas[i], self.deltas[i + 1])

    def free(self):
        if self.h:
            lib().mpo_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class SvdResult:
    """svd_truncate handle: new bond, discarded weight, and output tensors."""

    def __init__(self, ctx, bl, br, phys, psi, max_m, cutoff=1e-12, eps=1e-4, mode=ABSORB_RIGHT):
        import torch
        self.ctx = ctx
        h = c_void_p()
        self.code = check(lib().svd_truncate(ctx.h, bl.ref, br.ref, phys.ref, ptr(psi), int(max_m), float(cutoff),
                                             float(eps), int(mode), byref(h)), allow_warn=True)
        self.h = h
        n = c_int32()
        disc, nf = c_double(), c_int32()
        check(lib().svd_result_bond(h, byref(n), None, None, 0, byref(disc), byref(nf)))
        q = np.zeros(max(n.value, 1), np.int32)
        d = np.zeros(max(n.value, 1), np.int32)
        check(lib().svd_result_bond(h, None, q.ctypes.data_as(POINTER(c_int32)), d.ctypes.data_as(POINTER(c_int32)),
                                    n.value, None, None))
        self.bond = {int(a): int(b) for a, b in zip(q[:n.value], d[:n.value])}
        self.discarded, self.n_floored = disc.value, nf.value
        B = Bond(self.bond)
        _, na = layout(SITE, bl, B, phys)
        _, nb = layout(SITE, B, br, phys)
        mk = lambda k: torch.empty(max(k, 1), dtype=torch.float64, device="cuda")
        self.A, self.B, self.left, self.right = mk(na), mk(nb), mk(na), mk(nb)
        m = sum(self.bond.values())
        self.lam = np.zeros(max(m, 1))
        self.V = np.zeros(max(m, 1))
        check(lib().svd_result_copy(ctx.h, h, ptr(self.A), ptr(self.B), ptr(self.left), ptr(self.right),
                                    self.lam.ctypes.data_as(POINTER(c_double)), self.V.ctypes.data_as(POINTER(c_double))))
        self.lam, self.V = self.lam[:m], self.V[:m]
        lib().svd_free(h)
        self.h = None


def dav_params(max_matvec=4, max_sub=8, tol=1e-8):
    return CDavParams(int(max_matvec), int(max_sub), float(tol))


class Mps:
    """mps_alloc / mps_set_site / sweep / mps_energy on a context."""

    def __init__(self, ctx, bonds, sites, phys_q=(-1, 1), q_target=0):
        self.ctx = ctx
        self.phys = Phys(phys_q)
        self.B = [Bond(b) for b in bonds]
        arr = (CBond * len(self.B))(*[b.c for b in self.B])
        h = c_void_p()
        check(lib().mps_alloc(ctx.h, len(sites), self.phys.ref, int(q_target), arr, byref(h)))
        self.h = h
        self.N = len(sites)
        for i, s in enumerate(sites):
            table, n = layout(SITE, self.B[i], self.B[i + 1], self.phys)
            flat = np.zeros(n)
            for key, off, rows, cols, ld in table:
                b = s[key[:2]]
                for r in range(rows):
                    flat[off + r * ld: off + r * ld + cols] = b[r]
            check(lib().mps_set_site(h, i, flat.ctypes.data_as(POINTER(c_double)), n))

    def copy(self):
        """Deep device copy (mps_copy)."""
        other = Mps.__new__(Mps)
        other.ctx, other.phys, other.B, other.N = self.ctx, self.phys, list(self.B), self.N
        h = c_void_p()
        check(lib().mps_copy(self.ctx.h, self.h, byref(h)))
        other.h = h
        return other

    def sweep(self, mpo, max_m, n_regions=1, prec=F64, refine=True, dav=None, dav_shared=None,
              cutoff=1e-12, eps=1e-4, concurrent=False):
        p = CSweepParams(int(max_m), int(n_regions), int(prec), int(bool(refine)),
                         dav or dav_params(4, 8, 1e-8), dav_shared or dav_params(40, 8, 1e-10),
                         float(cutoff), float(eps), _concurrency(concurrent), 0)
        rep = CSweepReport()
        check(lib().sweep(self.ctx.h, self.h, mpo.h, byref(p), byref(rep)))
        return {f: getattr(rep, f) for f, _ in CSweepReport._fields_}

    def energy(self, mpo):
        e = c_double()
        check(lib().mps_energy(self.ctx.h, self.h, mpo.h, byref(e)))
        return e.value

    def gradients(self, mpo):
        """grad_mpo: (E, [G_i]) with G_i = dE/dW_i at fixed state, torch
        tensors [Dl, d, d, Dr] on the device.  Leaves the MPS unsplit."""
        import torch
        shapes = [w.shape for w in mpo.W]
        n = sum(int(np.prod(sh)) for sh in shapes)
        G = torch.empty(max(n, 1), dtype=torch.float64, device="cuda")
        e = c_double()
        check(lib().grad_mpo(self.ctx.h, self.h, mpo.h, ptr(G), n, byref(e)))
        out, o = [], 0
        for sh in shapes:
            k = int(np.prod(sh))
            out.append(G[o:o + k].view(*sh))
            o += k
        return e.value, out

    def site_blocks(self, i):
        """mps_get_site: the site tensor as {(q_left, s): array}."""
        B = [Bond(self.bond(i)), Bond(self.bond(i + 1))]
        table, n = layout(SITE, B[0], B[1], self.phys)
        flat = np.zeros(max(n, 1))
        check(lib().mps_get_site(self.h, i, flat.ctypes.data_as(POINTER(c_double)), n))
        out = {}
        for key, off, rows, cols, ld in table:
            out[key[:2]] = np.array([flat[off + r * ld: off + r * ld + cols] for r in range(rows)]).reshape(rows, cols)
        return out

    def inverse_canonical(self, cutoff=1e-14, eps=1e-4):
        """mps_inverse_canonical: in place; returns the number of floored V entries."""
        nf = c_int32()
        check(lib().mps_inverse_canonical(self.ctx.h, self.h, float(cutoff), float(eps), byref(nf)))
        return nf.value

    def get_v(self, b):
        """mps_get_v: {q: V on the sector} of bond b."""
        bd = self.bond(b)
        tot = sum(bd.values())
        v = np.zeros(max(tot, 1))
        check(lib().mps_get_v(self.h, b, v.ctypes.data_as(POINTER(c_double)), tot))
        out, o = {}, 0
        for q in sorted(bd):
            out[q] = v[o:o + bd[q]].copy()
            o += bd[q]
        return out

    def expect_site(self, op):
        """mps_expect_site: <O_j> for every site j."""
        op = np.ascontiguousarray(op, dtype=np.float64)
        out = np.zeros(self.N)
        check(lib().mps_expect_site(self.ctx.h, self.h, op.ctypes.data_as(POINTER(c_double)),
                                    out.ctypes.data_as(POINTER(c_double))))
        return out

    def expect_pairs(self, terms, pairs, concurrent=False):
        """mps_expect_pairs: sum_t c_t <A_t(i) B_t(k)> for each (i, k) in pairs;
        terms = [(c, A, B), ...] with d x d operators."""
        c = np.ascontiguousarray([t[0] for t in terms], dtype=np.float64)
        A = np.ascontiguousarray(np.stack([t[1] for t in terms]), dtype=np.float64)
        Bm = np.ascontiguousarray(np.stack([t[2] for t in terms]), dtype=np.float64)
        i = np.ascontiguousarray([p[0] for p in pairs], dtype=np.int32)
        k = np.ascontiguousarray([p[1] for p in pairs], dtype=np.int32)
        out = np.zeros(max(len(pairs), 1))
        pd_ = lambda a: a.ctypes.data_as(POINTER(c_double))
        check(lib().mps_expect_pairs(self.ctx.h, self.h, len(terms), pd_(c), pd_(A), pd_(Bm), len(pairs),
                                     i.ctypes.data_as(POINTER(c_int32)), k.ctypes.data_as(POINTER(c_int32)),
                                     int(bool(concurrent)), pd_(out)))
        return out[:len(pairs)]

    def order_parameter(self, kind, Lx, Ly):
        """mps_order_parameter: kind "Dx" (0) or "Mz" (1)."""
        v = c_double()
        k = {"Dx": 0, "Mz": 1}.get(kind, kind)
        check(lib().mps_order_parameter(self.ctx.h, self.h, int(k), int(Lx), int(Ly), byref(v)))
        return v.value

    def bond(self, b):
        n = c_int32()
        check(lib().mps_bond(self.h, b, byref(n), None, None, 0))
        q = np.zeros(max(n.value, 1), np.int32)
        d = np.zeros(max(n.value, 1), np.int32)
        check(lib().mps_bond(self.h, b, None, q.ctypes.data_as(POINTER(c_int32)), d.ctypes.data_as(POINTER(c_int32)),
                             n.value))
        return {int(a): int(c) for a, c in zip(q[:n.value], d[:n.value])}

    def free(self):
        if self.h:
            lib().mps_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ---------------------------------------------------------------- gradients
def grad_site(ctx, bl, br, phys, W, L, psi, R):
    """grad_site: G[w, s, t, w'] (torch, device) for a single-site centre."""
    import torch
    G = torch.empty(W.W.size, dtype=torch.float64, device="cuda")
    check(lib().grad_site(ctx.h, bl.ref, br.ref, phys.ref, W.ref, ptr(L), ptr(psi), ptr(R), ptr(G)))
    return G.view(*W.W.shape)


def _energy_function():
    import torch

    class MpoEnergy(torch.autograd.Function):
        """E(W_0..W_{N-1}) = <Psi|H(W)|Psi>/<Psi|Psi> at a fixed MPS; the
        backward pass is the grad_mpo measurement sweep (G_i = dE/dW_i)."""

        @staticmethod
        def forward(fctx, mps, deltas, *W):
            sites = [MpoSite(w.detach().cpu().numpy(), deltas[i], deltas[i + 1]) for i, w in enumerate(W)]
            mpo = Mpo(sites=sites)
            fctx.mps, fctx.mpo = mps, mpo
            fctx.devices = [w.device for w in W]
            return torch.tensor(mps.energy(mpo), dtype=torch.float64)

        @staticmethod
        def backward(fctx, gE):
            _, G = fctx.mps.gradients(fctx.mpo)
            fctx.mpo.free()
            return (None, None) + tuple((gE.to(g.device) * g).to(dev) for g, dev in zip(G, fctx.devices))

    return MpoEnergy


def mpo_energy(mps, deltas, W):
    """Differentiable E(W) at fixed state (torch.autograd); W: list of
    [Dl, d, d, Dr] tensors, deltas: channel charges of bonds 0..N."""
    return _energy_function().apply(mps, deltas, *W)


def set_env_stride(ctx, stride):
    """Environment recompute stride of sweeps / measurement sweeps on ctx."""
    check(lib().pdmrg_ctx_set_env_stride(ctx.h, int(stride)))


def set_verbose(ctx, level):
    """Progress lines (one per optimised bond / gauge move) on stderr."""
    check(lib().pdmrg_ctx_set_verbose(ctx.h, int(level)))


def _concurrency(c):
    """sweep's concurrent field: False / 0 one after the other, True / 1 own
    streams, 2 lockstep with batched SVDs."""
    if isinstance(c, bool) or c in (0, 1):
        return int(bool(c))
    if c == 2:
        return 2
    raise ValueError("concurrent must be False, True or 2")


def set_svd_precondition(ctx, mode):
    """QR preconditioning of the truncation SVD: 0 off, 1 blocks of >= 64
    rows (default), 2 every block."""
    check(lib().pdmrg_ctx_set_svd_precondition(ctx.h, int(mode)))


def memory_stats(reset_peak=False):
    """(in_use, peak, cached) device bytes of the library's allocator."""
    a, b, c = c_int64(), c_int64(), c_int64()
    check(lib().pdmrg_memory_stats(byref(a), byref(b), byref(c), int(bool(reset_peak))))
    return a.value, b.value, c.value


def dE_dcouplings(mps, mpo):
    """(E, [dE/dtheta_k]) for the couplings mpo_build was given: grad_couplings
    (one measurement sweep and the device contraction with the MPO's
    coefficient-derivative tables)."""
    n = mpo.ncouplings
    dE = np.zeros(max(n, 1))
    E = c_double()
    check(lib().grad_couplings(mps.ctx.h, mps.h, mpo.h, dE.ctypes.data_as(POINTER(c_double)), n, byref(E)))
    return E.value, [float(v) for v in dE[:n]]
