// Davidson eigensolver for the lowest eigenpair of H_eff (Sec. II: "a few
// Lanczos or Davidson steps" per bond), FP64 vectors on the device.
//
// Per iteration: Rayleigh-Ritz on the orthonormal basis V (projected matrix
// G = V^T H V, lowest pair by a one-wave Jacobi kernel), Ritz vector x and
// residual r = H x - theta x, diagonal-preconditioned correction
// t = r / (diag - theta) orthogonalised twice against V (classical
// Gram-Schmidt), restart to x when V holds max_sub vectors.  The Ritz vector
// is signed so that its overlap with the first basis vector is >= 0.
//
// Mixed precision (operator in FP32 / BF16x3 with an FP64 operator op64):
// the first basis vector's product H x is always taken in FP64 and every
// restart recomputes it; the coupling of x to the correction directions
// t_k is taken from that exact product (t_k . H x), so the low-precision
// error enters only through the t_k . H~ t_j block, whose weight in the Ritz
// vector shrinks quadratically with the correction.  Convergence is declared
// on the FP64 residual of the restarted vector.
#include "internal.hpp"

#include <cmath>

namespace pdmrg {

namespace {
struct DavWs {
    double *V, *HV, *X, *HX, *r, *t;
    double *G;        // [ks][ks]
    double *c;        // [ks]
    double *dots;     // [ks]
    double *scal;     // [kScal]: 0 theta, 1 rr, 2 tn2, 3 nrm2; the fused
                      // passes reduce [rr, V_0.t, ..] into 1 .. k + 1
    double *partial;  // [nblk][ks]
};
constexpr int kBlk = 1024;   // blocks of the reduction passes (4 per CU: memory parallelism)
constexpr int kScal = 8 + kDavFused + 2;
}  // namespace

DavResult davidson_run(pdmrg_ctx *ctx, pdmrg_heff *op, pdmrg_heff *op64, double *psi,
                       const pdmrg_dav_params &p) {
    hipStream_t s = ctx->stream;
    const int64_t n = op->nX;
    const int ks = std::max(2, (int)p.max_sub);
    PD_REQUIRE(ks <= 64, PDMRG_EINVAL, "davidson: max_sub must be <= 64");
    PD_REQUIRE(p.max_matvec >= 1, PDMRG_EINVAL, "davidson: max_matvec must be >= 1");
    const bool refine = op->prec != PDMRG_F64 && op64 != nullptr;
    if (refine) PD_REQUIRE(op64->nX == n && op64->prec == PDMRG_F64, PDMRG_ESHAPE, "davidson: op64 mismatch");

    // workspace (owned by the context, grown on demand)
    DevBuf &ws = ctx->ws_dav;
    const size_t nvec = (size_t)2 * ks + 4;
    const size_t ndots = std::max(ks, 2 * kDavFused + 2);
    const size_t small = (size_t)ks * ks + ks + ndots + kScal + (size_t)kBlk * (2 * std::max(ks, kDavFused) + 2);
    ws.ensure((nvec * n + small) * sizeof(double));
    DavWs w;
    double *b = ws.as<double>();
    w.V = b; b += (size_t)ks * n;
    w.HV = b; b += (size_t)ks * n;
    w.X = b; b += n;
    w.HX = b; b += n;
    w.r = b; b += n;
    w.t = b; b += n;
    w.G = b; b += (size_t)ks * ks;
    w.c = b; b += ks;
    w.dots = b; b += ndots;
    w.scal = b; b += kScal;
    w.partial = b;
    // subspaces of up to kDavFused vectors take the fused passes (one read of
    // each vector per pass, fewer launches); larger ones the separate kernels
    const bool fused = ks <= kDavFused;

    auto dot_into = [&](const double *U, int nv, const double *x, double *out, int stride = 1) {
        launch_multidot(U, n, nv, x, n, w.partial, kBlk, s);
        launch_reduce_partials(w.partial, kBlk, nv, out, stride, s);
    };
    auto cgs2 = [&](int k, double *t) {
        for (int pass = 0; pass < 2; ++pass) {
            dot_into(w.V, k, t, w.dots);
            launch_subtract_combine(w.V, n, k, w.dots, t, n, s);
        }
    };
    const double *diag = op->diag.as<double>();
    int nmv = 0;
    auto matvec = [&](pdmrg_heff *o, const double *x, double *y) {
        heff_run(ctx, o, x, y);
        ++nmv;
    };
    // G column/row for vector k: G[i][k] = V_i . HV_k, G[k][i] = V_k . HV_i
    auto extend_G = [&](int k) {
        if (fused) {
            launch_dav_ext_gram(w.V, w.HV, n, k, n, w.partial, kBlk, s);
            launch_reduce_partials(w.partial, kBlk, 2 * dav_ext_gram_width(k) + 1, w.dots, 1, s);
            launch_dav_g_scatter(w.G, ks, k, w.dots, refine, s);
            return;
        }
        dot_into(w.V, k + 1, w.HV + (size_t)k * n, w.G + k, ks);          // column k
        if (k > 0) dot_into(w.HV, k, w.V + (size_t)k * n, w.G + (size_t)k * ks);   // row k
        // Mixed precision: G[0][k] = x . H~ t_k carries the low-precision error
        // ~eps |H| whatever the size of the correction, while G[k][0] = t_k . H x
        // uses the exact FP64 product; take the exact one for both.
        if (refine && k > 0)
            HIP_OK(hipMemcpyAsync(w.G + k, w.G + (size_t)k * ks, sizeof(double), hipMemcpyDeviceToDevice, s));
    };

    // Ritz pair of the k-vector basis, residual r (|r|^2 -> scal[1]),
    // preconditioned correction t orthogonalised twice against V
    // (|t|^2 -> scal[2]); theta -> scal[0], x, hx
    auto ritz_step = [&](int k) {
        launch_small_eig(w.G, k, ks, w.scal + 0, w.c, s);
        if (fused) {
            launch_dav_ritz(w.V, w.HV, n, k, w.c, w.scal + 0, diag, w.X, w.HX, w.r, w.t, n, w.partial, kBlk, s);
            launch_reduce_partials(w.partial, kBlk, k + 1, w.scal + 1, 1, s);   // rr, first projections
            launch_dav_sub_dot(w.V, n, k, w.scal + 2, w.t, n, true, w.partial, kBlk, s);
            launch_reduce_partials(w.partial, kBlk, k, w.dots, 1, s);           // second projections
            launch_dav_sub_dot(w.V, n, k, w.dots, w.t, n, false, w.partial, kBlk, s);
            launch_reduce_partials(w.partial, kBlk, 1, w.scal + 2, 1, s);       // |t|^2
            return;
        }
        launch_combine(w.V, n, k, w.c, w.X, n, 0.0, s);
        launch_combine(w.HV, n, k, w.c, w.HX, n, 0.0, s);
        launch_residual(w.HX, w.X, w.scal + 0, w.r, n, s);
        dot_into(w.r, 1, w.r, w.scal + 1);
        launch_precond(w.r, diag, w.scal + 0, w.t, n, s);
        cgs2(k, w.t);
        dot_into(w.t, 1, w.t, w.scal + 2);
    };

    // V0 = psi / |psi|
    dot_into(psi, 1, psi, w.scal + 3);
    launch_scale_by_inv_sqrt(psi, w.scal + 3, w.V, n, s);
    matvec(refine ? op64 : op, w.V, w.HV);
    int k = 1;
    extend_G(0);

    double host[3] = {0, 0, 0};
    double theta = 0, rn = 0;
    bool converged = false;
    while (true) {
        ritz_step(k);
        HIP_OK(hipMemcpyAsync(host, w.scal, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        theta = host[0];
        rn = std::sqrt(std::max(0.0, host[1]));
        PD_REQUIRE(std::isfinite(theta) && std::isfinite(rn), PDMRG_ENUMERIC, "davidson: NaN/Inf in H_eff");
        const bool small_r = rn <= p.tol;
        const bool budget = nmv >= p.max_matvec;
        if (!refine) {
            if (small_r) { converged = true; break; }
            if (budget) break;
            if (std::sqrt(std::max(0.0, host[2])) < 1e-14) break;
            if (k >= ks) {
                // restart: V0 = x/|x|, HV0 = hx/|x|
                dot_into(w.X, 1, w.X, w.scal + 3);
                launch_scale_by_inv_sqrt(w.X, w.scal + 3, w.V, n, s);
                launch_scale_by_inv_sqrt(w.HX, w.scal + 3, w.HV, n, s);
                k = 1;
                extend_G(0);
            }
        } else {
            if (small_r || budget || k >= ks || std::sqrt(std::max(0.0, host[2])) < 1e-14) {
                // FP64 restart at the Ritz vector
                dot_into(w.X, 1, w.X, w.scal + 3);
                launch_scale_by_inv_sqrt(w.X, w.scal + 3, w.V, n, s);
                matvec(op64, w.V, w.HV);
                k = 1;
                extend_G(0);
                ritz_step(1);   // x = V0 (c = 1), hx = HV0
                HIP_OK(hipMemcpyAsync(host, w.scal, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
                HIP_OK(hipStreamSynchronize(s));
                theta = host[0];
                rn = std::sqrt(std::max(0.0, host[1]));
                HIP_OK(hipMemcpyAsync(w.X, w.V, n * sizeof(double), hipMemcpyDeviceToDevice, s));
                if (rn <= p.tol) { converged = true; break; }
                if (nmv >= p.max_matvec) break;
                if (std::sqrt(std::max(0.0, host[2])) < 1e-14) break;
            }
        }
        // append t / |t|
        launch_scale_by_inv_sqrt(w.t, w.scal + 2, w.V + (size_t)k * n, n, s);
        matvec(op, w.V + (size_t)k * n, w.HV + (size_t)k * n);
        extend_G(k);
        ++k;
    }
    // psi <- x / |x|
    dot_into(w.X, 1, w.X, w.scal + 3);
    launch_scale_by_inv_sqrt(w.X, w.scal + 3, psi, n, s);
    HIP_OK(hipStreamSynchronize(s));
    DavResult res;
    res.energy = theta;
    res.resid = rn;
    res.nmv = nmv;
    res.converged = converged;
    return res;
}

}  // namespace pdmrg
