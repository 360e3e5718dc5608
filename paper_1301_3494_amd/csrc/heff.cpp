// Two-site effective Hamiltonian operator (Sec. II): plan + environments in
// the compute precision + intermediates.
#include "internal.hpp"

namespace pdmrg {

GemmPrec gemm_prec(int prec) {
    switch (prec) {
        case PDMRG_F64: return GemmPrec::F64;
        case PDMRG_F32: return GemmPrec::F32;
        case PDMRG_BF16X3: return GemmPrec::BF16X3;
    }
    throw Error(PDMRG_EINVAL, "unknown precision " + std::to_string(prec));
}

void heff_build(pdmrg_ctx *ctx, pdmrg_heff *op, const Bond &bl, const Bond &br, const Phys &p,
                const MpoSite &W1, const MpoSite &W2, const double *L, const double *R, int prec) {
    hipStream_t s = ctx->stream;
    (void)gemm_prec(prec);
    op->prec = prec;
    op->plan.build(bl, br, p, W1, W2, prec, s);
    HeffPlan &pl = op->plan;
    op->nX = pl.X.size;
    op->nL = pl.Lt.size;
    op->nR = pl.Rt.size;
    // diagonal preconditioner from the FP64 environments
    op->diag.ensure(std::max<int64_t>(op->nX, 1) * sizeof(double));
    upload(op->diag_terms, pl.diag_terms, s);
    upload(op->diag_groups, pl.diag_groups, s);
    {
        Slots sl{};
        sl.p[0] = op->diag.ptr;
        sl.p[1] = L;
        sl.p[2] = R;
        launch_diag_terms(sl, op->diag_terms.as<DiagTerm>(), op->diag_groups.as<int32_t>(),
                          (int)pl.diag_groups.size() - 1, pl.diag_max_rows, s);
    }
    const size_t es = prec == PDMRG_F64 ? sizeof(double) : sizeof(float);
    op->L.ensure(std::max<int64_t>(op->nL, 1) * es);
    op->R.ensure(std::max<int64_t>(op->nR, 1) * es);
    if (prec == PDMRG_F64) {
        if (op->nL) HIP_OK(hipMemcpyAsync(op->L.ptr, L, op->nL * es, hipMemcpyDeviceToDevice, s));
        if (op->nR) HIP_OK(hipMemcpyAsync(op->R.ptr, R, op->nR * es, hipMemcpyDeviceToDevice, s));
    } else {
        launch_convert_f64_f32(L, op->L.as<float>(), op->nL, s);
        launch_convert_f64_f32(R, op->R.as<float>(), op->nR, s);
        op->xs.ensure(std::max<int64_t>(op->nX, 1) * sizeof(float));
    }
    op->T1.ensure(std::max<int64_t>(pl.nT1, 1) * es);
    op->T2.ensure(std::max<int64_t>(pl.nT2, 1) * es);
    op->P.ensure(std::max<int64_t>(pl.nP, 1) * sizeof(double));
}

void heff_run(pdmrg_ctx *ctx, pdmrg_heff *op, const double *x, double *y) {
    hipStream_t s = ctx->stream;
    const HeffPlan &pl = op->plan;
    const GemmPrec gp = gemm_prec(op->prec);
    const bool f64 = op->prec == PDMRG_F64;
    Slots sl{};
    if (f64) {
        sl.p[0] = x;
    } else {
        launch_convert_f64_f32(x, op->xs.as<float>(), op->nX, s);
        sl.p[0] = op->xs.ptr;
    }
    sl.p[1] = y;
    sl.p[2] = op->L.ptr;
    sl.p[3] = op->R.ptr;
    sl.p[4] = op->T1.ptr;
    sl.p[5] = op->T2.ptr;
    sl.p[6] = op->P.ptr;
    hipEvent_t *ev = nullptr;
    if (ctx->timing) {
        const size_t need = (size_t)(ctx->n_timed + 1) * 4;
        while (ctx->ev_pool.size() < need) {
            hipEvent_t e;
            HIP_OK(hipEventCreate(&e));
            ctx->ev_pool.push_back(e);
        }
        ev = &ctx->ev_pool[(size_t)ctx->n_timed * 4];
        ctx->n_timed += 1;
        HIP_OK(hipEventRecord(ev[0], s));
    }
    pl.g1.launch(gp, f64, sl, s);
    if (ev) HIP_OK(hipEventRecord(ev[1], s));
    pl.w.launch(f64, sl, s);
    if (ev) HIP_OK(hipEventRecord(ev[2], s));
    pl.g3.launch(gp, true, sl, s);
    pl.r3.launch(true, sl, s);
    if (ev) HIP_OK(hipEventRecord(ev[3], s));
}

}  // namespace pdmrg
