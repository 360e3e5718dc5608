// Internal objects behind the opaque handles of include/pdmrg.h.
#pragma once
#include "plans.hpp"

struct pdmrg_heff {
    pdmrg::HeffPlan plan;
    int prec = PDMRG_F64;
    pdmrg::DevBuf L, R;            // environments in the operator's precision
    pdmrg::DevBuf T1, T2, xs;      // intermediates, low-precision copy of x
    pdmrg::DevBuf P;               // split-K partials of stage 3 (FP64)
    pdmrg::DevBuf diag;            // diag(H_eff), FP64
    pdmrg::DevBuf diag_terms, diag_groups;
    // buffers the launches use: the owned ones above, or the caller's FP64
    // environments (borrowed) and another operator's intermediates (shared)
    const void *lp = nullptr, *rp = nullptr;
    void *t1 = nullptr, *t2 = nullptr, *pp = nullptr;
    int64_t nX = 0, nL = 0, nR = 0;
    // captured kernel sequences of heff_apply, one per (x, y) pair
    struct Graph {
        const double *x = nullptr;
        double *y = nullptr;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
    };
    static constexpr size_t kMaxGraphs = 16;
    std::vector<Graph> graphs;
    ~pdmrg_heff() {
        for (auto &g : graphs) {
            if (g.exec) (void)hipGraphExecDestroy(g.exec);
            if (g.graph) (void)hipGraphDestroy(g.graph);
        }
    }
};

struct pdmrg_mpo {
    int N = 0, d = 0;
    std::vector<int> phys_q;
    std::vector<pdmrg::MpoSite> W;   // W[i]: Dl = D(i), Dr = D(i+1)
    // mpo_build only: per coupling k, dW_i/dtheta_k of every site
    // concatenated in site order (the grad_mpo layout); empty where the
    // channel structure depends on that coupling
    std::vector<std::vector<double>> dW;
};

namespace pdmrg {

GemmPrec gemm_prec(int prec);
// may_time: with ctx->autotune >= 1, time the candidate plans on a cache
// miss (false: a miss takes the cost model, as inside sweeps where bond
// shapes rarely repeat).
// borrow_env (FP64 only): the operator reads L and R in place (the caller
// keeps them alive and unchanged while it is used) instead of copying them.
// ws_from: an operator of the same bond whose intermediates (T1, T2, split-K
// partials) this one reuses where they are large enough; the two must not be
// applied at the same time.
void heff_build(pdmrg_ctx *ctx, pdmrg_heff *op, const Bond &bl, const Bond &br, const Phys &p,
                const MpoSite &W1, const MpoSite &W2, const double *L, const double *R, int prec,
                bool may_time = true, bool borrow_env = false, const pdmrg_heff *ws_from = nullptr);
void heff_run(pdmrg_ctx *ctx, pdmrg_heff *op, const double *x, double *y);

struct DavResult {
    double energy = 0, resid = 0;
    int nmv = 0;
    bool converged = false;
};
DavResult davidson_run(pdmrg_ctx *ctx, pdmrg_heff *op, pdmrg_heff *op64, double *psi,
                       const pdmrg_dav_params &p);

// Truncated SVD of a two-site tensor (svd.cpp).
struct SvdOut {
    Bond bl, br, bnew;
    Phys p;
    int mode = 0;
    DevBuf A, B, left, right;      // SITE layouts: A, left on (bl, bnew); B, right on (bnew, br)
    std::vector<double> lam, V;    // in new-bond order
    double discarded = 0;
    int n_floored = 0;
    int n_unconverged = 0;         // Jacobi blocks that ran out of sweeps
};
// Process-wide tuning cache to / from a text file (one line per signature).
// Cylinder geometry of the Sec. III lattices: site (x, y) in the snake order
// (column by column, alternating direction) and the three-colouring of the
// triangular cylinder's bonds (x,y)-(x,y+1), (x,y)-(x+1,y), (x,y)-(x+1,y-1).
inline int lattice_snake(int x, int y, int Ly) { return x * Ly + ((x % 2 == 0) ? y : Ly - 1 - y); }
inline int tri_sublattice(int x, int y) { return ((x - y) % 3 + 3) % 3; }

// Resolves the device address of env_update_noalloc's scratch array on the
// current device (noalloc.hip); called when a context is created.
void noalloc_init(int device);

int tune_export(const char *path);
int tune_import(const char *path);
void grad_site_run(pdmrg_ctx *ctx, const GradPlan &plan, const double *L, const double *psi, const double *R,
                   double *G);
void svd_truncate_run(pdmrg_ctx *ctx, const Bond &bl, const Bond &br, const Phys &p, const double *psi,
                      int max_m, double cutoff, double eps, int mode, SvdOut &out);
// Several truncated SVDs in one batch: the sector blocks of all problems
// share the Jacobi launches (each block on its own tolerance); each problem
// is truncated on its own.  The results equal separate svd_truncate_run calls.
struct SvdProblem {
    const Bond *bl, *br;
    const Phys *p;
    const double *psi;
    int max_m;
    double cutoff;
    int mode;
};
void svd_truncate_multi(pdmrg_ctx *ctx, const std::vector<SvdProblem> &probs, double eps,
                        std::vector<SvdOut> &outs);

}  // namespace pdmrg

struct pdmrg_svd {
    pdmrg::SvdOut r;
};
