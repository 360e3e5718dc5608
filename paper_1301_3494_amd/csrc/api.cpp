// extern "C" entry points of include/pdmrg.h: argument checking, handle
// management and error translation.  No C++ exception crosses the ABI.
#include "internal.hpp"

#include <cmath>

using namespace pdmrg;

namespace pdmrg {
const char *last_error_cstr();
}

#define API_BEGIN try {
#define API_END                                                  \
    }                                                            \
    catch (const pdmrg::Error &e) {                              \
        pdmrg::set_last_error(e.what());                         \
        return e.code;                                           \
    }                                                            \
    catch (const std::bad_alloc &) {                             \
        pdmrg::set_last_error("host allocation failed");         \
        return PDMRG_ENOMEM;                                     \
    }                                                            \
    catch (const std::exception &e) {                            \
        pdmrg::set_last_error(e.what());                         \
        return PDMRG_EINVAL;                                     \
    }                                                            \
    return PDMRG_OK;

extern "C" {

const char *pdmrg_last_error(void) { return last_error_cstr(); }
const char *pdmrg_version(void) { return "pdmrg 0.1 (gfx950)"; }

int pdmrg_ctx_create(int device, void *stream, pdmrg_ctx **out) {
    API_BEGIN
    PD_REQUIRE(out != nullptr, PDMRG_EINVAL, "ctx_create: null out");
    int n = 0;
    HIP_OK(hipGetDeviceCount(&n));
    PD_REQUIRE(device >= 0 && device < n, PDMRG_EINVAL, "ctx_create: no such device");
    HIP_OK(hipSetDevice(device));
    pdmrg::noalloc_init(device);
    auto *c = new pdmrg_ctx();
    c->device = device;
    c->stream = static_cast<hipStream_t>(stream);
    *out = c;
    API_END
}

int pdmrg_ctx_destroy(pdmrg_ctx *ctx) {
    API_BEGIN
    if (!ctx) return PDMRG_OK;
    ctx->pool.reset();   // joins the idle worker threads
    (void)hipStreamSynchronize(ctx->stream);
    for (pdmrg_ctx *c : ctx->sub) {
        (void)hipStreamSynchronize(c->stream);
        for (auto &e : c->ev_pool) (void)hipEventDestroy(e);
        if (c->owns_stream) (void)hipStreamDestroy(c->stream);
        if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
        delete c;
    }
    for (auto &e : ctx->ev_pool) (void)hipEventDestroy(e);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    delete ctx;
    API_END
}

int pdmrg_ctx_set_graphs(pdmrg_ctx *ctx, int enable) {
    API_BEGIN
    PD_REQUIRE(ctx, PDMRG_EINVAL, "null ctx");
    ctx->graphs = enable != 0;
    API_END
}

int pdmrg_ctx_set_timing(pdmrg_ctx *ctx, int enable) {
    API_BEGIN
    PD_REQUIRE(ctx, PDMRG_EINVAL, "null ctx");
    ctx->timing = enable != 0;
    ctx->n_timed = 0;
    API_END
}

int pdmrg_ctx_set_autotune(pdmrg_ctx *ctx, int level) {
    API_BEGIN
    PD_REQUIRE(ctx, PDMRG_EINVAL, "null ctx");
    PD_REQUIRE(level >= 0 && level <= 2, PDMRG_EINVAL, "autotune level must be 0, 1 or 2");
    ctx->autotune = level;
    API_END
}

int pdmrg_ctx_set_env_stride(pdmrg_ctx *ctx, int stride) {
    API_BEGIN
    PD_REQUIRE(ctx && stride >= 0, PDMRG_EINVAL, "set_env_stride: bad arguments");
    ctx->env_stride = stride;
    API_END
}

int pdmrg_ctx_set_verbose(pdmrg_ctx *ctx, int level) {
    API_BEGIN
    PD_REQUIRE(ctx && level >= 0, PDMRG_EINVAL, "set_verbose: bad arguments");
    ctx->verbose = level;
    API_END
}

int pdmrg_ctx_set_svd_precondition(pdmrg_ctx *ctx, int mode) {
    API_BEGIN
    PD_REQUIRE(ctx && mode >= 0 && mode <= 2, PDMRG_EINVAL, "set_svd_precondition: bad arguments");
    ctx->svd_precond = mode;
    API_END
}

int pdmrg_memory_stats(int64_t *in_use, int64_t *peak, int64_t *cached, int reset_peak) {
    API_BEGIN
    pdmrg::alloc_stats(in_use, peak, cached);
    if (reset_peak) pdmrg::alloc_reset_peak();
    API_END
}

int pdmrg_set_alloc_poison(int on) {
    API_BEGIN
    pdmrg::g_alloc_poison.store(on != 0);
    API_END
}

int pdmrg_autotune_export(const char *path, int32_t *n_entries) {
    API_BEGIN
    PD_REQUIRE(path, PDMRG_EINVAL, "autotune export: null path");
    const int n = tune_export(path);
    if (n_entries) *n_entries = n;
    API_END
}

int pdmrg_autotune_import(const char *path, int32_t *n_entries) {
    API_BEGIN
    PD_REQUIRE(path, PDMRG_EINVAL, "autotune import: null path");
    const int n = tune_import(path);
    if (n_entries) *n_entries = n;
    API_END
}

int pdmrg_ctx_timing(pdmrg_ctx *ctx, double *ms_stage, int64_t *n_calls) {
    API_BEGIN
    PD_REQUIRE(ctx && ms_stage && n_calls, PDMRG_EINVAL, "null argument");
    constexpr int NS = kTimingEvents - 1;
    double acc[NS + 1] = {};
    if (ctx->n_timed > 0) {
        HIP_OK(hipEventSynchronize(ctx->ev_pool[(size_t)ctx->n_timed * kTimingEvents - 1]));
        for (int64_t c = 0; c < ctx->n_timed; ++c) {
            hipEvent_t *e = &ctx->ev_pool[(size_t)c * kTimingEvents];
            for (int k = 0; k < NS; ++k) {
                float ms = 0.f;
                HIP_OK(hipEventElapsedTime(&ms, e[k], e[k + 1]));
                acc[k] += ms;
                acc[NS] += ms;
            }
        }
    }
    *n_calls = ctx->n_timed;
    for (int i = 0; i <= NS; ++i) ms_stage[i] = ctx->n_timed ? acc[i] / ctx->n_timed : 0.0;
    API_END
}

// ------------------------------------------------------------------ layouts
static void layout_common(int kind, const pdmrg_bond *b1, const pdmrg_bond *b2, const pdmrg_phys *phys,
                          const int32_t *deltas, int32_t ndelta, std::vector<int32_t> *keys,
                          std::vector<int64_t> *offs, std::vector<int32_t> *rows, std::vector<int32_t> *cols,
                          std::vector<int32_t> *lds, int64_t *n_elems) {
    if (kind == PDMRG_SITE || kind == PDMRG_TWO_SITE) {
        const Bond bl = Bond::from(b1), br = Bond::from(b2);
        const Phys p = Phys::from(phys);
        const bool two = kind == PDMRG_TWO_SITE;
        const SiteLayout L = two ? two_site_layout(bl, br, p) : site_layout(bl, br, p);
        const int d = p.d();
        for (int i = 0; i < bl.nsec(); ++i)
            for (int s = 0; s < L.nphys; ++s) {
                const int co = L.colo[(size_t)i * L.nphys + s];
                if (co < 0) continue;
                keys->push_back(bl.q[i]);
                keys->push_back(two ? s / d : s);
                keys->push_back(two ? s % d : 0);
                offs->push_back(L.base[i] + co);
                rows->push_back(bl.dim[i]);
                cols->push_back(L.width[(size_t)i * L.nphys + s]);
                lds->push_back(L.cols[i]);
            }
        *n_elems = L.size;
    } else if (kind == PDMRG_ENV_L || kind == PDMRG_ENV_R) {
        const Bond b = Bond::from(b1);
        PD_REQUIRE(deltas && ndelta > 0, PDMRG_EINVAL, "layout: env needs channel charges");
        const std::vector<int> dv(deltas, deltas + ndelta);
        const bool isL = kind == PDMRG_ENV_L;
        const EnvLayout E = isL ? env_l_layout(b, dv) : env_r_layout(b, dv);
        // list blocks keyed by (bra sector, w)
        for (int qb = 0; qb < b.nsec(); ++qb)
            for (int w = 0; w < E.D; ++w) {
                const int qk = b.find(b.q[qb] - dv[w]);   // ket sector
                if (qk < 0) continue;
                if (isL) {
                    const int ro = E.rowo[(size_t)qk * E.D + w];
                    keys->push_back(b.q[qb]);
                    keys->push_back(w);
                    keys->push_back(0);
                    offs->push_back(E.base[qk] + (int64_t)ro * b.dim[qk]);
                    rows->push_back(b.dim[qb]);
                    cols->push_back(b.dim[qk]);
                    lds->push_back(b.dim[qk]);
                } else {
                    const int ro = E.rowo[(size_t)qb * E.D + w];
                    keys->push_back(b.q[qb]);
                    keys->push_back(w);
                    keys->push_back(0);
                    offs->push_back(E.base[qb] + (int64_t)ro * b.dim[qb]);
                    rows->push_back(b.dim[qk]);   // stored transposed: rows = ket
                    cols->push_back(b.dim[qb]);
                    lds->push_back(b.dim[qb]);
                }
            }
        *n_elems = E.size;
    } else {
        throw Error(PDMRG_EINVAL, "layout: unknown kind");
    }
}

int pdmrg_layout_size(int kind, const pdmrg_bond *b1, const pdmrg_bond *b2, const pdmrg_phys *phys,
                      const int32_t *deltas, int32_t ndelta, int64_t *n_elems, int32_t *n_blocks) {
    API_BEGIN
    PD_REQUIRE(n_elems && n_blocks, PDMRG_EINVAL, "layout_size: null outputs");
    std::vector<int32_t> k, r, c, l;
    std::vector<int64_t> o;
    layout_common(kind, b1, b2, phys, deltas, ndelta, &k, &o, &r, &c, &l, n_elems);
    *n_blocks = (int32_t)o.size();
    API_END
}

int pdmrg_layout_blocks(int kind, const pdmrg_bond *b1, const pdmrg_bond *b2, const pdmrg_phys *phys,
                        const int32_t *deltas, int32_t ndelta, int32_t *keys, int64_t *offsets,
                        int32_t *rows, int32_t *cols, int32_t *ld) {
    API_BEGIN
    std::vector<int32_t> k, r, c, l;
    std::vector<int64_t> o;
    int64_t n = 0;
    layout_common(kind, b1, b2, phys, deltas, ndelta, &k, &o, &r, &c, &l, &n);
    if (keys) std::copy(k.begin(), k.end(), keys);
    if (offsets) std::copy(o.begin(), o.end(), offsets);
    if (rows) std::copy(r.begin(), r.end(), rows);
    if (cols) std::copy(c.begin(), c.end(), cols);
    if (ld) std::copy(l.begin(), l.end(), ld);
    API_END
}

// ------------------------------------------------------------------ MPO
int mpo_from_sites(int nsites, const pdmrg_mpo_site *sites, pdmrg_mpo **out) {
    API_BEGIN
    PD_REQUIRE(nsites > 0 && sites && out, PDMRG_EINVAL, "mpo_from_sites: bad arguments");
    auto m = std::make_unique<pdmrg_mpo>();
    m->N = nsites;
    for (int i = 0; i < nsites; ++i) {
        m->W.push_back(MpoSite::from(&sites[i]));
        if (i > 0) {
            PD_REQUIRE(m->W[i].Dl == m->W[i - 1].Dr && m->W[i].dl == m->W[i - 1].dr, PDMRG_ESHAPE,
                       "mpo_from_sites: channel mismatch between sites");
            PD_REQUIRE(m->W[i].d == m->W[0].d, PDMRG_ESHAPE, "mpo_from_sites: local dimension mismatch");
        }
    }
    PD_REQUIRE(m->W[0].Dl == 1 && m->W[nsites - 1].Dr == 1, PDMRG_ESHAPE,
               "mpo_from_sites: boundary MPO bonds must have one channel");
    m->d = m->W[0].d;
    *out = m.release();
    API_END
}

int mpo_info(const pdmrg_mpo *mpo, int32_t *nsites, int32_t *d, int32_t *phys_q, int32_t *D) {
    API_BEGIN
    PD_REQUIRE(mpo, PDMRG_EINVAL, "null mpo");
    if (nsites) *nsites = mpo->N;
    if (d) *d = mpo->d;
    if (phys_q)
        for (size_t i = 0; i < mpo->phys_q.size(); ++i) phys_q[i] = mpo->phys_q[i];
    if (D) {
        for (int i = 0; i < mpo->N; ++i) D[i] = mpo->W[i].Dl;
        D[mpo->N] = mpo->W[mpo->N - 1].Dr;
    }
    API_END
}

int mpo_get_site(const pdmrg_mpo *mpo, int site, double *W, int32_t *dl, int32_t *dr) {
    API_BEGIN
    PD_REQUIRE(mpo && site >= 0 && site < mpo->N, PDMRG_EINVAL, "mpo_get_site: bad site");
    const MpoSite &m = mpo->W[site];
    if (W) std::copy(m.W.begin(), m.W.end(), W);
    if (dl) std::copy(m.dl.begin(), m.dl.end(), dl);
    if (dr) std::copy(m.dr.begin(), m.dr.end(), dr);
    API_END
}

void mpo_free(pdmrg_mpo *mpo) { delete mpo; }

// ------------------------------------------------------------------ H_eff
int heff_create(pdmrg_ctx *ctx, const pdmrg_bond *bl, const pdmrg_bond *br, const pdmrg_phys *phys,
                const pdmrg_mpo_site *W1, const pdmrg_mpo_site *W2, const double *L_dev, const double *R_dev,
                int prec, pdmrg_heff **out) {
    API_BEGIN
    PD_REQUIRE(ctx && out && L_dev && R_dev, PDMRG_EINVAL, "heff_create: null argument");
    auto op = std::make_unique<pdmrg_heff>();
    heff_build(ctx, op.get(), Bond::from(bl), Bond::from(br), Phys::from(phys), MpoSite::from(W1),
               MpoSite::from(W2), L_dev, R_dev, prec);
    HIP_OK(hipStreamSynchronize(ctx->stream));
    *out = op.release();
    API_END
}

int heff_apply(pdmrg_ctx *ctx, pdmrg_heff *op, const double *x_dev, double *y_dev) {
    API_BEGIN
    PD_REQUIRE(ctx && op && x_dev && y_dev, PDMRG_EINVAL, "heff_apply: null argument");
    heff_run(ctx, op, x_dev, y_dev);
    API_END
}

int heff_info(const pdmrg_heff *op, double *flops_Lpsi, double *flops_W, double *flops_R, int64_t *n_psi,
              int64_t *n_L, int64_t *n_R, int64_t *n_T1, int64_t *n_T2) {
    API_BEGIN
    PD_REQUIRE(op, PDMRG_EINVAL, "null op");
    if (flops_Lpsi) *flops_Lpsi = op->plan.g1.flops;
    if (flops_W) *flops_W = op->plan.w.flops;
    if (flops_R) *flops_R = op->plan.g3.flops;
    if (n_psi) *n_psi = op->nX;
    if (n_L) *n_L = op->nL;
    if (n_R) *n_R = op->nR;
    if (n_T1) *n_T1 = op->plan.nT1;
    if (n_T2) *n_T2 = op->plan.nT2;
    API_END
}

int heff_plan_info(const pdmrg_heff *op, int32_t *shape_Lpsi, int32_t *shape_R, int32_t *tiles_Lpsi,
                   int32_t *tiles_R, int32_t *splitk_parts) {
    API_BEGIN
    PD_REQUIRE(op, PDMRG_EINVAL, "heff_plan_info: null operator");
    const HeffPlan &pl = op->plan;
    if (shape_Lpsi) *shape_Lpsi = (int32_t)pl.g1.shape;
    if (shape_R) *shape_R = (int32_t)pl.g3.shape;
    if (tiles_Lpsi) *tiles_Lpsi = (int32_t)pl.g1.ntiles_real;
    if (tiles_R) *tiles_R = (int32_t)pl.g3.ntiles_real;
    if (splitk_parts) *splitk_parts = pl.parts3;
    API_END
}

int heff_diag(pdmrg_ctx *ctx, pdmrg_heff *op, double *diag_dev) {
    API_BEGIN
    PD_REQUIRE(ctx && op && diag_dev, PDMRG_EINVAL, "heff_diag: null argument");
    if (op->nX)
        HIP_OK(hipMemcpyAsync(diag_dev, op->diag.ptr, op->nX * sizeof(double), hipMemcpyDeviceToDevice,
                              ctx->stream));
    API_END
}

void heff_free(pdmrg_heff *op) { delete op; }

// ------------------------------------------------------------------ environments
int env_update(pdmrg_ctx *ctx, int dir, const pdmrg_bond *bl, const pdmrg_bond *br, const pdmrg_phys *phys,
               const pdmrg_mpo_site *W, const double *env_in_dev, const double *site_dev, double *env_out_dev,
               int prec) {
    API_BEGIN
    PD_REQUIRE(ctx && env_in_dev && site_dev && env_out_dev, PDMRG_EINVAL, "env_update: null argument");
    PD_REQUIRE(dir == 1 || dir == -1, PDMRG_EINVAL, "env_update: dir must be +1 or -1");
    PD_REQUIRE(prec == PDMRG_F64, PDMRG_EINVAL, "env_update: only FP64 environments are supported");
    EnvPlan plan;
    plan.build(dir, Bond::from(bl), Bond::from(br), Phys::from(phys), MpoSite::from(W), ctx->stream);
    const size_t need = (size_t)(std::max<int64_t>(plan.nU1, 1) + std::max<int64_t>(plan.nU2, 1)) * sizeof(double);
    ctx->ws_env.ensure(need);
    double *U1 = ctx->ws_env.as<double>();
    double *U2 = U1 + std::max<int64_t>(plan.nU1, 1);
    plan.run(GemmPrec::F64, env_in_dev, site_dev, env_out_dev, U1, U2, ctx->stream);
    HIP_OK(hipStreamSynchronize(ctx->stream));
    API_END
}

// ------------------------------------------------------------------ gradient

int grad_site(pdmrg_ctx *ctx, const pdmrg_bond *bl, const pdmrg_bond *br, const pdmrg_phys *phys,
              const pdmrg_mpo_site *W, const double *L_dev, const double *psi_dev, const double *R_dev,
              double *G_dev) {
    API_BEGIN
    PD_REQUIRE(ctx && L_dev && psi_dev && R_dev && G_dev, PDMRG_EINVAL, "grad_site: null argument");
    GradPlan plan;
    plan.build(Bond::from(bl), Bond::from(br), Phys::from(phys), MpoSite::from(W), ctx->stream);
    grad_site_run(ctx, plan, L_dev, psi_dev, R_dev, G_dev);
    HIP_OK(hipStreamSynchronize(ctx->stream));
    API_END
}

int env_update_info(int dir, const pdmrg_bond *bl, const pdmrg_bond *br, const pdmrg_phys *phys,
                    const pdmrg_mpo_site *W, double *flops, int64_t *n_out) {
    API_BEGIN
    PD_REQUIRE(dir == 1 || dir == -1, PDMRG_EINVAL, "env_update_info: dir must be +1 or -1");
    EnvPlan plan;
    plan.build(dir, Bond::from(bl), Bond::from(br), Phys::from(phys), MpoSite::from(W), nullptr, false);
    if (flops) *flops = plan.g1.flops + plan.w.flops + plan.g3.flops;
    if (n_out) *n_out = plan.Eout.size;
    API_END
}

// ------------------------------------------------------------------ Davidson
int davidson_step(pdmrg_ctx *ctx, pdmrg_heff *op, pdmrg_heff *op64, double *psi_dev, const pdmrg_dav_params *p,
                  double *energy, double *resid, int32_t *n_matvec) {
    API_BEGIN
    PD_REQUIRE(ctx && op && psi_dev && p, PDMRG_EINVAL, "davidson_step: null argument");
    DavResult r = davidson_run(ctx, op, op64, psi_dev, *p);
    if (energy) *energy = r.energy;
    if (resid) *resid = r.resid;
    if (n_matvec) *n_matvec = r.nmv;
    if (!r.converged) {
        pdmrg::set_last_error("davidson: residual above tolerance after the matvec budget");
        return PDMRG_WARN_NOT_CONVERGED;
    }
    API_END
}

// ------------------------------------------------------------------ merge
int merge_regions(pdmrg_ctx *ctx, const pdmrg_bond *bl, const pdmrg_bond *bm, const pdmrg_bond *br,
                  const pdmrg_phys *phys, const double *psiL_dev, const double *V_dev, const double *psiR_dev,
                  double *psi2_dev) {
    API_BEGIN
    PD_REQUIRE(ctx && psiL_dev && V_dev && psiR_dev && psi2_dev, PDMRG_EINVAL, "merge_regions: null argument");
    MergePlan plan;
    plan.build(Bond::from(bl), Bond::from(bm), Bond::from(br), Phys::from(phys), ctx->stream);
    ctx->ws_merge.ensure(std::max<int64_t>(plan.SR.size, 1) * sizeof(double));
    plan.run(psiL_dev, V_dev, psiR_dev, psi2_dev, ctx->ws_merge.as<double>(), ctx->stream);
    HIP_OK(hipStreamSynchronize(ctx->stream));
    API_END
}

}  // extern "C"

// ------------------------------------------------------------------ SVD
extern "C" {

int svd_truncate(pdmrg_ctx *ctx, const pdmrg_bond *bl, const pdmrg_bond *br, const pdmrg_phys *phys,
                 const double *psi_dev, int32_t max_m, double cutoff, double eps, int mode, pdmrg_svd **out) {
    API_BEGIN
    PD_REQUIRE(ctx && psi_dev && out, PDMRG_EINVAL, "svd_truncate: null argument");
    PD_REQUIRE(cutoff >= 0.0 && eps >= 0.0 && eps < 1.0, PDMRG_EINVAL, "svd_truncate: bad cutoff / eps");
    auto r = std::make_unique<pdmrg_svd>();
    svd_truncate_run(ctx, Bond::from(bl), Bond::from(br), Phys::from(phys), psi_dev, max_m, cutoff, eps, mode, r->r);
    const bool floored = mode == PDMRG_SPLIT && r->r.n_floored > 0;
    const int unconv = r->r.n_unconverged;
    *out = r.release();
    if (unconv > 0) {
        pdmrg::set_last_error("svd_truncate: " + std::to_string(unconv) +
                              " block(s) of the Jacobi SVD ran out of sweeps (absolute accuracy only)");
        return PDMRG_WARN_NOT_CONVERGED;
    }
    if (floored) {
        pdmrg::set_last_error("svd_truncate: some V entries were floored");
        return PDMRG_WARN_V_FLOORED;
    }
    API_END
}

int svd_result_bond(const pdmrg_svd *res, int32_t *nsec, int32_t *q, int32_t *dim, int32_t nsec_max,
                    double *discarded, int32_t *n_floored) {
    API_BEGIN
    PD_REQUIRE(res, PDMRG_EINVAL, "svd_result_bond: null result");
    const Bond &b = res->r.bnew;
    if (nsec) *nsec = b.nsec();
    if (q || dim) {
        PD_REQUIRE(nsec_max >= b.nsec(), PDMRG_EINVAL, "svd_result_bond: capacity too small");
        for (int k = 0; k < b.nsec(); ++k) {
            if (q) q[k] = b.q[k];
            if (dim) dim[k] = b.dim[k];
        }
    }
    if (discarded) *discarded = res->r.discarded;
    if (n_floored) *n_floored = res->r.n_floored;
    API_END
}

int svd_result_copy(pdmrg_ctx *ctx, const pdmrg_svd *res, double *A_dev, double *B_dev, double *left_dev,
                    double *right_dev, double *lam_host, double *V_host) {
    API_BEGIN
    PD_REQUIRE(ctx && res, PDMRG_EINVAL, "svd_result_copy: null argument");
    const SvdOut &r = res->r;
    const int64_t na = site_layout(r.bl, r.bnew, r.p).size, nb = site_layout(r.bnew, r.br, r.p).size;
    auto cp = [&](double *dst, const DevBuf &src, int64_t n) {
        if (dst && n) HIP_OK(hipMemcpyAsync(dst, src.ptr, n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    };
    cp(A_dev, r.A, na);
    cp(B_dev, r.B, nb);
    cp(left_dev, r.mode == PDMRG_ABSORB_RIGHT ? r.A : r.left, na);
    cp(right_dev, r.mode == PDMRG_ABSORB_LEFT ? r.B : r.right, nb);
    if (lam_host) std::copy(r.lam.begin(), r.lam.end(), lam_host);
    if (V_host) std::copy(r.V.begin(), r.V.end(), V_host);
    HIP_OK(hipStreamSynchronize(ctx->stream));
    API_END
}

void svd_free(pdmrg_svd *res) { delete res; }

}  // extern "C"
