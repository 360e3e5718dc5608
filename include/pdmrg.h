/*
 * pdmrg.h -- C ABI of the MI355X (gfx950) hot path of real-space parallel
 * DMRG (E. M. Stoudenmire and S. R. White, "Real-Space Parallel Density
 * Matrix Renormalization Group").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Status: every function returns int.  0 = OK; > 0 = warning
 * (PDMRG_WARN_NOT_CONVERGED, PDMRG_WARN_V_FLOORED); < 0 = error (see the
 * PDMRG_E* codes).  pdmrg_last_error() returns a thread-local message for the
 * last non-zero status.  No C++ exception crosses the ABI.
 *
 * Charges: integers q = 2 S^z.  Bond charges are left-accumulated: a bond
 * state's charge is the total charge of the sites to its left, so every MPS
 * tensor satisfies q_left + q_phys = q_right; bond 0 is {q = 0, dim 1} and bond
 * N is {q = target, dim 1}.  A bond is a list of sectors with strictly
 * ascending charge and positive dimension; within a sector, states are ordered
 * as produced by the SVD (descending singular value).
 *
 * Memory: pointers named *_dev are device pointers (HIP device memory of the
 * context's device, e.g. torch tensors); every other pointer is host memory.
 * The library never frees caller memory.  Device data is FP64 unless an
 * argument says otherwise; layouts are row-major.
 *
 * Layouts (block-sparse, U(1) allowed blocks only), all blocks concatenated in
 * ascending order of their leading sector:
 *  PDMRG_SITE     A[a, s, b] on bonds (bl, br): for each left sector q_a, a
 *                 row-major block of dim(q_a) rows and sum_s dim_br(q_a + q_s)
 *                 columns, the column segments ordered by s ascending (absent
 *                 right sectors skipped).
 *  PDMRG_TWO_SITE Psi[a, s1, s2, b] on (bl, br): as SITE with the column
 *                 segments ordered by (s1, s2) lexicographically (Eq. eqn:wf).
 *  PDMRG_ENV_L    left environment L[a, w, a'] on a bond (a = bra, a' = ket):
 *                 for each ket sector q', a row-major block whose rows run over
 *                 the MPO channels w ascending and, within w, the bra states of
 *                 sector q' + delta_w; columns are the ket states of q'.
 *  PDMRG_ENV_R    right environment R[b, w, b'] (b = bra): for each bra sector
 *                 q, a row-major block whose rows run over w ascending and,
 *                 within w, the ket states of sector q - delta_w; columns are
 *                 the bra states of q.  (R is stored with its ket index on the
 *                 rows.)
 * pdmrg_layout_blocks() lists every block with its offset, shape and leading
 * dimension, so callers can move data in and out.
 *
 * MPO tensors W_i[wl, s, s', wr] (<s|O|s'> for channel wl -> wr) are host
 * arrays; channel charges delta_w satisfy delta_wl + q_s - q_s' = delta_wr.
 * The environment of bond 0 is L = [[1]] on MPO channel 0 and that of bond N
 * is R = [[1]] on the last bond's single channel.
 */
#ifndef PDMRG_H
#define PDMRG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
#define PDMRG_OK 0
#define PDMRG_WARN_NOT_CONVERGED 1
#define PDMRG_WARN_V_FLOORED 2
#define PDMRG_EINVAL (-1)     /* bad argument                              */
#define PDMRG_ESHAPE (-2)     /* sector / charge structure mismatch         */
#define PDMRG_ENOMEM (-3)     /* device or host allocation failed           */
#define PDMRG_EHIP (-4)       /* HIP runtime error                          */
#define PDMRG_ENUMERIC (-5)   /* NaN / Inf detected                         */

/* --------------------------------------------------------------- precision */
#define PDMRG_F64 0           /* FP64 MFMA, FP64 storage                     */
#define PDMRG_F32 1           /* FP32 MFMA, FP32 storage, FP32 accumulation  */
#define PDMRG_BF16X3 2        /* split-BF16 x3 MFMA (hi*hi + hi*lo + lo*hi),
                                 FP32 storage and accumulation              */

/* ----------------------------------------------------------------- layouts */
#define PDMRG_SITE 0
#define PDMRG_TWO_SITE 1
#define PDMRG_ENV_L 2
#define PDMRG_ENV_R 3

typedef struct {
    int32_t nsec;             /* number of sectors                          */
    const int32_t *q;         /* [nsec] charges, strictly ascending         */
    const int32_t *dim;       /* [nsec] dimensions, > 0                     */
} pdmrg_bond;

typedef struct {
    int32_t d;                /* local dimension                            */
    const int32_t *q;         /* [d] charges of the local states            */
} pdmrg_phys;

typedef struct {
    int32_t Dl, Dr, d;
    const double *W;          /* [Dl][d][d][Dr], row-major                   */
    const int32_t *dl;        /* [Dl] channel charges of the left MPO bond   */
    const int32_t *dr;        /* [Dr] channel charges of the right MPO bond  */
} pdmrg_mpo_site;

typedef struct pdmrg_ctx pdmrg_ctx;
typedef struct pdmrg_mpo pdmrg_mpo;
typedef struct pdmrg_heff pdmrg_heff;
typedef struct pdmrg_svd pdmrg_svd;
typedef struct pdmrg_mps pdmrg_mps;

const char *pdmrg_last_error(void);
const char *pdmrg_version(void);

/* Context on one device.  stream: a hipStream_t (NULL = default stream) on
 * which every kernel of this context is launched, in order.  Not thread-safe:
 * one context per host thread. */
int pdmrg_ctx_create(int device, void *stream, pdmrg_ctx **out);
int pdmrg_ctx_destroy(pdmrg_ctx *ctx);
/* H_eff stage timing: while enabled, every heff_apply records HIP events on
 * the context's stream around its three stages (no synchronisation);
 * pdmrg_ctx_timing waits for the last one and returns the average duration
 * (ms) of stage 1 (L psi), 2 (W), 3 (. R) and their sum over the calls since
 * timing was enabled. */
int pdmrg_ctx_set_timing(pdmrg_ctx *ctx, int enable);
/* Tile-shape selection of the grouped GEMMs of every H_eff built afterwards
 * on this context (the contraction order of Sec. II is unchanged):
 *   0  (default) a cost model of padded MFMA work and device fill;
 *   1  each allowed shape of stage 1 and stage 3 is timed on the operator's
 *      own buffers when it is created by heff_create (a few ms), and the
 *      fastest is kept in a process-wide cache keyed by device, precision,
 *      bond sectors and MPO widths, so later operators of the same shape are
 *      not re-timed (sweep() uses cached plans but never times candidates);
 *   2  as 1, with one line per tuned signature on stderr.
 * Every shape computes the same product; the summation order follows the
 * tile shape and the K split, so results can differ in the last bits (FP64:
 * about 1e-15 relative).  A given plan is bitwise reproducible.
 * Returns PDMRG_EINVAL for another level. */
int pdmrg_ctx_set_autotune(pdmrg_ctx *ctx, int level);
/* Environment recompute (memory for time) for sweep, grad_mpo and
 * grad_couplings on this context: with stride k >= 2, a pass keeps the
 * environments of every k-th bond and of the region boundaries and drops the
 * others once it has moved past them; a pass that needs a dropped one
 * rebuilds it (and the ones between) from the nearest kept environment with
 * env_update steps on the current site tensors, so results are the same bits
 * as with every environment kept.  Memory: about N/k + k environments per
 * region instead of N + 1; cost: about one extra environment update per bond.
 * k <= 1 (the default 0): every environment is kept. */
int pdmrg_ctx_set_env_stride(pdmrg_ctx *ctx, int stride);
/* Progress log of sweep, grad_mpo and grad_couplings on this context: with
 * level 1 every optimised bond (bond, kept m, energy, Davidson and SVD
 * seconds) and every gauge move prints one line on stderr; level 2 also one
 * line per level of each truncation SVD (blocks, preconditioned blocks,
 * largest block, Jacobi sweeps and launched rounds); 0 (the default): silent.  PDMRG_EINVAL for a
 * negative level. */
int pdmrg_ctx_set_verbose(pdmrg_ctx *ctx, int level);
/* Preconditioning of the truncation SVD (svd_truncate, and every SVD of
 * sweep, split, gauge conversion and grad passes on this context; Eq. eqn:svd
 * and the Appendix): with mode 1 (the default) each middle-charge block of at
 * least 64 rows (of the smaller dimension) and at most 2048 columns is
 * factored by Householder QR after ordering its rows by decreasing norm, and
 * the one-sided Jacobi iteration runs on the triangular factor, which needs
 * about half the sweeps on the graded blocks of a DMRG state; 2 does this for
 * every block up to 2048 columns, 0 never.  The factors are those of the same
 * block to rounding (not the same bits as mode 0); the Appendix recursion
 * runs on top unchanged.  PDMRG_EINVAL for another mode. */
int pdmrg_ctx_set_svd_precondition(pdmrg_ctx *ctx, int mode);
/* Device memory of the library's caching allocator (all contexts of the
 * process, bytes): in_use = handed out and not released, peak = largest
 * in_use since the last reset, cached = released blocks held for reuse.
 * reset_peak != 0 sets peak to the current in_use afterwards.  Outputs
 * optional. */
int pdmrg_memory_stats(int64_t *in_use, int64_t *peak, int64_t *cached, int reset_peak);
/* Debugging aid, process-wide: on != 0 fills every device buffer the library
 * allocates or takes from its cache (workspaces, plans, MPS storage) with
 * 0xFF bytes, a NaN in FP64 and FP32, before first use, so that a kernel
 * reading memory nothing wrote shows up as NaN instead of as whatever an
 * earlier call left there.  Synchronises the device at each allocation (slow;
 * not for use during stream capture).  on = 0 (the default) turns it off. */
int pdmrg_set_alloc_poison(int on);
/* enable = 1: heff_apply (and the Davidson matvecs on this context) replay a
 * HIP graph of the operator's kernel sequence, captured on the first call for
 * each (x, y) pair (up to 16 pairs per operator; further pairs run
 * eagerly); the graph holds kernel nodes only.  Saves the per-kernel launch
 * cost when the products are short.  Bypassed while stage timing is on.  The
 * graphs are destroyed with the operator. */
int pdmrg_ctx_set_graphs(pdmrg_ctx *ctx, int enable);
/* The process-wide tuning cache as a text file (one line per signature: key,
 * stage-1 shape, stage-3 shape, stage-3 K parts, tab-separated).  Export
 * writes every entry; import adds / replaces entries, so operators built
 * afterwards with autotune >= 1 take the stored plans without timing (the
 * same plans in another process).  n_entries (optional) receives the count.
 * PDMRG_EINVAL if the file cannot be opened or a line is malformed. */
int pdmrg_autotune_export(const char *path, int32_t *n_entries);
int pdmrg_autotune_import(const char *path, int32_t *n_entries);
int pdmrg_ctx_timing(pdmrg_ctx *ctx, double *ms_stage /*[4]: L.psi, W, .R, total*/,
                     int64_t *n_calls);

/* Host-only layout bookkeeping (no device needed).  kind = PDMRG_SITE /
 * TWO_SITE use (b1 = left bond, b2 = right bond, phys); ENV_L / ENV_R use
 * (b1 = the bond, deltas[ndelta] = MPO channel charges of that bond).
 * pdmrg_layout_size gives the element count and block count; blocks lists
 * per block: key[3] (SITE: q_left, s, -; TWO_SITE: q_left, s1, s2; ENV: q_bra, w, -),
 * offset, rows, cols, ld.  For ENV_R the stored block is the transpose of
 * R[b, w, b'] restricted to the sectors (rows = ket b', cols = bra b). */
int pdmrg_layout_size(int kind, const pdmrg_bond *b1, const pdmrg_bond *b2,
                      const pdmrg_phys *phys, const int32_t *deltas, int32_t ndelta,
                      int64_t *n_elems, int32_t *n_blocks);
int pdmrg_layout_blocks(int kind, const pdmrg_bond *b1, const pdmrg_bond *b2,
                        const pdmrg_phys *phys, const int32_t *deltas, int32_t ndelta,
                        int32_t *keys /*[nb][3]*/, int64_t *offsets, int32_t *rows,
                        int32_t *cols, int32_t *ld);

/* ------------------------------------------------------------------- MPO
 * mpo_build: MPO of a lattice Hamiltonian (Sec. III models) from a finite
 * state machine over term prefixes (channels 'start', shared operator
 * prefixes, 'done'; the coupling sits on each term's last operator).
 * Host-only.  lattice: 0 = open chain (Lx sites), 1 = square cylinder
 * Lx x Ly (open x, periodic y, snake order), 2 = triangular cylinder,
 * 3 = J-Q2 square cylinder, 4 = transverse-field Ising chain (no symmetry:
 * all charges 0), 5 = open S = 1 chain (d = 3, local charges q = 2 S^z =
 * -2, 0, 2; the Fig. 3 study).  couplings[]: chain/square/S = 1 chain
 * {J, Delta}; triangular
 * {J, Delta} or {J, Delta, h}; J-Q2 {J, Q} or {J, Q, pin}; TFIM {J, h}.
 * Edge pinning of Sec. III (optional third coupling, 0 = off): J-Q2 adds
 * pin * (Q/4)(S_r . S_{r+y} - 1/4) on every vertical bond of the columns
 * x = 0 and x = Lx - 1 (the paper's strong-pinning term at pin = 1);
 * triangular adds the field -h S^z on the sites of those two columns that
 * belong to sublattice (x - y) mod 3 = 0 (the paper uses h = J/2; needs
 * Ly % 3 == 0). */
int mpo_build(int lattice, int Lx, int Ly, const double *couplings, int ncouplings,
              pdmrg_mpo **out);
/* MPO from caller tensors (copied). */
int mpo_from_sites(int nsites, const pdmrg_mpo_site *sites, pdmrg_mpo **out);
int mpo_info(const pdmrg_mpo *mpo, int32_t *nsites, int32_t *d, int32_t *phys_q /*[d]*/,
             int32_t *D /*[nsites+1]*/);
int mpo_get_site(const pdmrg_mpo *mpo, int site, double *W /*[Dl*d*d*Dr]*/,
                 int32_t *dl, int32_t *dr);
void mpo_free(pdmrg_mpo *mpo);

/* ------------------------------------------------------------------ H_eff
 * Two-site effective Hamiltonian of Sec. II: y = (L x W1 W2 x R) x,
 * y[a,s1,s2,b] = sum L[a,w,a'] W1[w,s1,t1,c] W2[c,s2,t2,w2] R[b,w2,b'] x[a',t1,t2,b'].
 * heff_create builds the contraction plan for the bonds (bl, br) and copies
 * L (ENV_L on bl with W1's left channels) and R (ENV_R on br with W2's right
 * channels) into the precision `prec` (the caller may free L, R afterwards).
 * heff_apply: x_dev, y_dev in TWO_SITE layout, FP64. */
int heff_create(pdmrg_ctx *ctx, const pdmrg_bond *bl, const pdmrg_bond *br,
                const pdmrg_phys *phys, const pdmrg_mpo_site *W1, const pdmrg_mpo_site *W2,
                const double *L_dev, const double *R_dev, int prec, pdmrg_heff **out);
int heff_apply(pdmrg_ctx *ctx, pdmrg_heff *op, const double *x_dev, double *y_dev);
/* Algorithmic flop count of one heff_apply (U(1)-allowed blocks, nonzero MPO
 * entries only, 2 flops per multiply-add) and element counts. */
int heff_info(const pdmrg_heff *op, double *flops_Lpsi, double *flops_W, double *flops_R,
              int64_t *n_psi, int64_t *n_L, int64_t *n_R, int64_t *n_T1, int64_t *n_T2);
/* Plan of an operator: tile shape of the stage-1 and stage-3 grouped GEMMs
 * (0: 64x64, 1: 128x32, 2: 32x128, 3: 128x128; 4: 64x64 and 5: 128x32 with
 * half-depth, 6: 64x64 and 7: 128x32 with quarter-depth K steps; 8: 128x32,
 * 9: 64x64, 10: 32x128 with K steps of 16 staged by direct-to-LDS loads, FP32
 * and FP64 only), their tile counts (without the idle padding of the launch
 * order), and the number of K parts of the longest stage-3 item (the other
 * items are cut into ranges of about the same length).  Outputs optional. */
int heff_plan_info(const pdmrg_heff *op, int32_t *shape_Lpsi, int32_t *shape_R, int32_t *tiles_Lpsi,
                   int32_t *tiles_R, int32_t *splitk_parts);
/* diag(H_eff) into diag_dev (TWO_SITE layout, FP64). */
int heff_diag(pdmrg_ctx *ctx, pdmrg_heff *op, double *diag_dev);
void heff_free(pdmrg_heff *op);

/* ------------------------------------------------------------- gradient
 * Hellmann-Feynman derivative of <psi|H|psi> with respect to one MPO tensor
 * at fixed state (not part of the paper; its Sec. III motivates scans over
 * large coupling spaces).  For a single-site centre psi (SITE layout on
 * (bl, br), FP64, device) between L (ENV_L on bl, deltas W->dl) and R (ENV_R
 * on br, deltas W->dr):
 *   G[w, s, t, w'] = sum L[a,w,a'] psi[a,s,b] psi[a',t,b'] R[b,w',b'],
 * written to G_dev (device, W->Dl * d * d * W->Dr doubles, row-major, every
 * entry overwritten).  Not normalised by <psi|psi>.  Deterministic (fixed
 * summation order).  Synchronises the context stream. */
int grad_site(pdmrg_ctx *ctx, const pdmrg_bond *bl, const pdmrg_bond *br, const pdmrg_phys *phys,
              const pdmrg_mpo_site *W, const double *L_dev, const double *psi_dev, const double *R_dev,
              double *G_dev);

/* ------------------------------------------------------------- environments
 * dir = +1: L_out (ENV_L on br) from L_in (ENV_L on bl) and the site tensor
 *           A (SITE on (bl, br)): L'[b,w',b'] = sum A[a,s,b] L[a,w,a'] W[w,s,s',w'] A[a',s',b'].
 * dir = -1: R_out (ENV_R on bl) from R_in (ENV_R on br) and B:
 *           R'[a,w,a'] = sum B[a,s,b] W[w,s,s',w'] R[b,w',b'] B[a',s',b'].
 * (Sec. II, transformation of the projected operators while sweeping.) */
/* Host-only: algorithmic flops of env_update with these arguments (allowed
 * blocks and nonzero MPO entries only, 2 per multiply-add) and the element
 * count of its output layout. */
int env_update_info(int dir, const pdmrg_bond *bl, const pdmrg_bond *br, const pdmrg_phys *phys,
                    const pdmrg_mpo_site *W, double *flops, int64_t *n_out);
int env_update(pdmrg_ctx *ctx, int dir, const pdmrg_bond *bl, const pdmrg_bond *br,
               const pdmrg_phys *phys, const pdmrg_mpo_site *W, const double *env_in_dev,
               const double *site_dev, double *env_out_dev, int prec);
/* env_update_noalloc: the same update for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  It calls no hipMalloc / hipFree: the two intermediates
 * and the device copies of the work lists live in a file-scope device array
 * of 64 MiB per GPU, set up when a context is created on that GPU and held
 * until the process ends.  Arguments, layouts and results are those of
 * env_update (same kernels, same bits).  An update whose intermediates and
 * lists need more than 64 MiB is rejected with PDMRG_EINVAL before anything
 * is launched.  Every call on a GPU shares that GPU's array (each call
 * overwrites what the last one left; nothing needs to start at zero), so
 * calls that overlap on one GPU, from several threads or streams, race.
 * Synchronises the context stream. */
int env_update_noalloc(pdmrg_ctx *ctx, int dir, const pdmrg_bond *bl, const pdmrg_bond *br,
                       const pdmrg_phys *phys, const pdmrg_mpo_site *W, const double *env_in_dev,
                       const double *site_dev, double *env_out_dev, int prec);

/* ---------------------------------------------------------------- Davidson
 * Lowest eigenpair of H_eff by Davidson (Rayleigh-Ritz on an orthonormal
 * basis, FP64 classical Gram-Schmidt twice, diagonal preconditioner, restart
 * to the Ritz vector at max_sub vectors; Sec. II "a few Davidson steps").
 * psi_dev: initial guess in, normalised eigenvector out.  If `op` is not FP64,
 * op64 (FP64 operator of the same bond, may be NULL for no refinement) is
 * used for outer FP64 refinement: each restart recomputes H x in FP64, so the
 * low-precision error enters only through the correction directions. */
typedef struct {
    int32_t max_matvec;       /* total matvec budget (low + high precision) */
    int32_t max_sub;          /* basis size before restart                  */
    double tol;               /* stop when ||H x - E x|| <= tol (FP64 residual) */
} pdmrg_dav_params;
int davidson_step(pdmrg_ctx *ctx, pdmrg_heff *op, pdmrg_heff *op64, double *psi_dev,
                  const pdmrg_dav_params *p, double *energy, double *resid, int32_t *n_matvec);

/* -------------------------------------------------------------------- SVD
 * Truncated SVD of the two-site Psi (Eq. eqn:svd) as the (m d) x (d m) matrix,
 * block-diagonal in the middle charge; per block a one-sided block-Jacobi SVD
 * followed by the Appendix recursion on singular values below eps * lambda_1
 * of that block.  Keeps the max_m largest singular values over all blocks
 * (ties: larger lambda, then smaller charge, then smaller index), dropping
 * lambda < cutoff * lambda_max, renormalised to sum lambda^2 = 1.
 * mode 0 = ABSORB_RIGHT (A kept, centre Lambda B), 1 = ABSORB_LEFT (B kept,
 * centre A Lambda), 2 = SPLIT (A Lambda and Lambda B, plus V = 1/Lambda
 * floored at 1/(1e-12 lambda_max); Eqs. eqn:inverse, eqn:isvd).
 * Returns a result handle (status PDMRG_WARN_NOT_CONVERGED if a block's
 * Jacobi iteration met its tolerance in none of 60 sweeps: the result is then
 * an exact rotation of the block with absolute, not relative, accuracy; else
 * PDMRG_WARN_V_FLOORED if SPLIT floored a V entry); read the new bond with
 * svd_result_bond, then copy
 * tensors into caller buffers with svd_result_copy (SITE layouts on
 * (bl, new) and (new, br); lam / V in bond order). */
#define PDMRG_ABSORB_RIGHT 0
#define PDMRG_ABSORB_LEFT 1
#define PDMRG_SPLIT 2
int svd_truncate(pdmrg_ctx *ctx, const pdmrg_bond *bl, const pdmrg_bond *br,
                 const pdmrg_phys *phys, const double *psi_dev, int32_t max_m, double cutoff,
                 double eps, int mode, pdmrg_svd **out);
int svd_result_bond(const pdmrg_svd *res, int32_t *nsec, int32_t *q /*cap nsec_max*/,
                    int32_t *dim, int32_t nsec_max, double *discarded, int32_t *n_floored);
/* Any device pointer may be NULL.  left_dev: A (ABSORB_RIGHT) or A Lambda
 * (ABSORB_LEFT, SPLIT); right_dev: Lambda B (ABSORB_RIGHT, SPLIT) or B
 * (ABSORB_LEFT); A_dev / B_dev: the orthonormal factors. */
int svd_result_copy(pdmrg_ctx *ctx, const pdmrg_svd *res, double *A_dev, double *B_dev,
                    double *left_dev, double *right_dev, double *lam_host, double *V_host);
void svd_free(pdmrg_svd *res);

/* -------------------------------------------------------------------- merge
 * Psi'[a,s3,s4,b] = sum_alpha psiL[a,s3,alpha] V[alpha] psiR[alpha,s4,b]
 * (Eq. eqn:merge).  psiL: SITE on (bl, bm); psiR: SITE on (bm, br);
 * V_dev: FP64 of length total(bm) in bond order; out: TWO_SITE on (bl, br). */
int merge_regions(pdmrg_ctx *ctx, const pdmrg_bond *bl, const pdmrg_bond *bm,
                  const pdmrg_bond *br, const pdmrg_phys *phys, const double *psiL_dev,
                  const double *V_dev, const double *psiR_dev, double *psi2_dev);

/* ---------------------------------------------------------------- MPS, sweep
 * mps_alloc: MPS of nsites sites with the given bond sector tables
 * (nsites+1 bonds); site data (SITE layouts, FP64, host) via mps_set_site.
 * sweep: one full sweep.  The first call brings the MPS to right-canonical
 * form with its centre on site 0 and builds the environments.  With
 * n_regions = 1 it is the standard two-site sweep (right, then back).  With
 * n_regions > 1 the first such call splits the chain into n contiguous
 * regions (V = Lambda^{-1} on every shared bond, odd regions centred at their
 * left end, even ones at their right end) and every call runs the staggered
 * pattern of Fig. 4: half-sweep A (odd regions right, even left), merge and
 * re-split at shared bonds 1|2, 3|4, ...; half-sweep B, merges at 2|3, ...
 * The regions of a half-sweep share no data (and neither do the merges of
 * one merge phase): with concurrent = 1 each region runs on its own HIP
 * stream, driven by its own host thread, with its own work space (the
 * paper's one process per region, on one device); with concurrent = 0 they
 * run one after the other on the context's stream; with concurrent = 2 the
 * regions run in lockstep, one bond of every region per step (their
 * eigensolvers as with 1, then the truncation SVDs of all the step's bonds
 * as one batch whose sector blocks share the Jacobi launches, then their
 * environment updates), and the merges of a phase form one step.  The
 * result is the same bits in all three modes.  energy: <Psi|H|Psi>/<Psi|Psi> of the whole MPS after the
 * sweep (V applied on the shared bonds). */
typedef struct {
    int32_t max_m;
    int32_t n_regions;
    int32_t prec;                     /* precision of bulk H_eff contractions */
    int32_t refine;                   /* 1: FP64 refinement when prec != F64  */
    pdmrg_dav_params dav;             /* interior bonds                       */
    pdmrg_dav_params dav_shared;      /* shared (merge) bonds                 */
    double cutoff, eps;
    int32_t concurrent;               /* 1: regions on their own streams;
                                         2: in lockstep, SVDs batched        */
    int32_t pad_;
} pdmrg_sweep_params;
typedef struct {
    double energy;                    /* full <H> after the sweep             */
    double max_trunc;                 /* largest discarded weight             */
    double seconds;                   /* wall time of the sweep               */
    double seconds_heff;              /* time inside Davidson (H_eff matvecs and the
                                         eigensolver's vector work); these three
                                         times add up over concurrent regions   */
    int64_t n_matvec;
    int32_t n_floored;
    int32_t max_bond;
    double max_infidelity;            /* largest 1 - |<Psi'|Psi>| over the merges:
                                         Psi' = psi_L V psi_R (Eq. eqn:merge), Psi the
                                         shared-bond eigenvector (Fig. 3); 0 without merges */
    int32_t n_svd_unconverged;        /* SVD blocks whose Jacobi iteration ran out of
                                         sweeps (kept with absolute accuracy)   */
    int32_t pad_;
    double seconds_svd;               /* time inside truncated SVDs           */
    double seconds_env;               /* time inside environment updates      */
} pdmrg_sweep_report;
int mps_alloc(pdmrg_ctx *ctx, int nsites, const pdmrg_phys *phys, int32_t q_target,
              const pdmrg_bond *bonds, pdmrg_mps **out);
int mps_set_site(pdmrg_mps *mps, int site, const double *host_data, int64_t n);
int mps_bond(const pdmrg_mps *mps, int b, int32_t *nsec, int32_t *q, int32_t *dim, int32_t cap);
int mps_get_site(pdmrg_mps *mps, int site, double *host_data, int64_t cap);
int sweep(pdmrg_ctx *ctx, pdmrg_mps *mps, const pdmrg_mpo *mpo, const pdmrg_sweep_params *p,
          pdmrg_sweep_report *rep);
int mps_energy(pdmrg_ctx *ctx, pdmrg_mps *mps, const pdmrg_mpo *mpo, double *energy);
/* Deep copy on the device (site tensors, environments, V of every bond, the
 * region split): the copy sweeps on exactly as the source would.  Owned by
 * the caller (mps_free). */
int mps_copy(pdmrg_ctx *ctx, const pdmrg_mps *src, pdmrg_mps **out);
/* Measurement sweep for dE/dW of E = <Psi|H|Psi>/<Psi|Psi> at fixed Psi:
 * G_dev (device, n_G doubles) receives G_0, ..., G_{N-1} concatenated, G_i
 * of shape [Dl_i][d][d][Dr_i] (mpo_get_site sizes), each the grad_site value
 * at centre i divided by <Psi|Psi>.  For couplings theta entering W affinely,
 * dE/dtheta = sum_i <G_i, dW_i/dtheta> (= <Psi| dH/dtheta |Psi>).  The MPS is
 * left unsplit (V folded into the left neighbour of each shared bond; the
 * re-canonicalisation drops only singular values below 1e-14 of the
 * largest) with the centre on the last site; the next sweep re-canonicalises
 * and re-splits it.  *energy (optional) receives E
 * before the gauge changes.  PDMRG_ESHAPE if n_G is not the total size. */
int grad_mpo(pdmrg_ctx *ctx, pdmrg_mps *mps, const pdmrg_mpo *mpo, double *G_dev, int64_t n_G, double *energy);
/* dE/dtheta_k for the couplings theta given to mpo_build (e.g. J and Delta,
 * J and Q, J and h; the same order and count): the measurement sweep of
 * grad_mpo (same effect on the MPS) followed, on the device, by
 * dE/dtheta_k = sum_i <G_i, dW_i/dtheta_k> with dW_i/dtheta_k taken from
 * tables mpo_build keeps for every coupling (each coefficient of its models
 * is affine in each coupling when the others are fixed).  Hellmann-Feynman
 * derivative at fixed state: the derivative of the ground-state energy when
 * the state is converged.  dE: host, ncouplings doubles; energy (optional)
 * receives E.  PDMRG_EINVAL if the MPO was not made by mpo_build, ncouplings
 * differs from the build's count, or the MPO's channel structure depends on
 * a coupling (no table for it). */
int grad_couplings(pdmrg_ctx *ctx, pdmrg_mps *mps, const pdmrg_mpo *mpo, double *dE, int32_t ncouplings,
                   double *energy);

/* ---------------------------------------------------------------------------
 * Inverse canonical gauge and local measurements (Sec. IV, Figs. imps_step
 * and inversecmps).  In this gauge every site tensor is an orthogonality
 * centre, psi_j = Lambda_j Gamma_j Lambda_{j+1}, and every inner bond b
 * carries V_b = Lambda_b^{-1}:  |Psi> = psi_0 V_1 psi_1 ... V_{N-1} psi_{N-1}.
 *
 * mps_inverse_canonical converts the MPS in place (same state, normalised):
 * any V of a region split is folded back, the MPS is brought to
 * right-canonical form with its centre on site 0, then the split of
 * Eqs. eqn:inverse, eqn:isvd is applied at bonds 1..N-1 in order, each
 * Lambda multiplied into both neighbours and V stored on the bond.  Singular
 * values below cutoff * lambda_max are dropped (bond dimensions can only
 * shrink); V is floored as in the sweep's split (1/max(lambda, 1e-12
 * lambda_max)), *n_floored (optional) counts the floored entries; eps is the
 * Appendix recursion threshold of the SVDs.  Afterwards mps_get_site returns
 * psi_j, mps_get_v returns V_b, mps_energy works unchanged, and the next
 * sweep or grad_mpo folds V back and re-canonicalises first.  No MPO needed.
 *
 * mps_get_v: V on bond b (host, bond order = sectors ascending in charge,
 * mps_bond dims) into V[0 .. total); PDMRG_EINVAL if the bond carries none
 * or cap is too small.
 *
 * mps_expect_site: out[j] = <Psi|O_j|Psi> for every site j (host, N doubles)
 * from the centres alone, sum psi_j[a,s,b] O[s][t] psi_j[a,t,b]; op is the
 * host d x d matrix <s|O|t> (row-major, local basis order of the MPS).  Only
 * charge-conserving entries can contribute.  One device launch covers all
 * sites.  PDMRG_EINVAL unless the MPS is in the inverse canonical gauge.
 *
 * mps_expect_pairs: out[p] = sum_t coef[t] <Psi| A_t(i_p) B_t(k_p) |Psi> for
 * npairs site pairs 0 <= i_p < k_p < N (host arrays).  opA / opB: nterms
 * host d x d matrices each (row-major <s|O|t>); every A_t must carry one
 * definite charge and B_t the opposite one (else PDMRG_EINVAL).  Needs only
 * the tensors on sites i..k: the left transfer starts from the identity on
 * bond i, passes psi_i and then V_j psi_j for j = i+1..k, and closes with the
 * trace on bond k+1 (F64 environment updates, one channel per term).
 * concurrent = 1 spreads the pairs over up to 8 host threads with their own
 * HIP streams (default priority); results are the same bits either way.
 * Example: S_i . S_k is {1, Sz, Sz}, {1/2, S+, S-}, {1/2, S-, S+}.
 * PDMRG_EINVAL unless the MPS is in the inverse canonical gauge. */
int mps_inverse_canonical(pdmrg_ctx *ctx, pdmrg_mps *mps, double cutoff, double eps, int32_t *n_floored);
int mps_get_v(const pdmrg_mps *mps, int bond, double *V, int64_t cap);
int mps_expect_site(pdmrg_ctx *ctx, pdmrg_mps *mps, const double *op, double *out);
int mps_expect_pairs(pdmrg_ctx *ctx, pdmrg_mps *mps, int nterms, const double *coef, const double *opA,
                     const double *opB, int npairs, const int32_t *site_i, const int32_t *site_k, int concurrent,
                     double *out);
/* Order parameters of Sec. III from the centres (MPS in the inverse canonical
 * gauge, spin-1/2 sites, N = Lx * Ly in the snake order of mpo_build; host
 * scalar *value):
 *   kind 0: columnar dimer order of the J-Q2 study,
 *     D_x = (1/Ly) sum_y <S_r.S_{r+x}> - <S_{r-x}.S_r>/2 - <S_{r+x}.S_{r+2x}>/2,
 *     r = (Lx/2 - 1, y) zero-based (the centre bond of an even-length
 *     cylinder); needs Lx >= 4;
 *   kind 1: sublattice magnetisation of the triangular study,
 *     M_z = <S^z> averaged over the sites (xc, y) of sublattice
 *     (x - y) mod 3 = 0 (the one mpo_build pins), xc = (Lx - 1)/2 zero-based;
 *     needs Ly % 3 == 0.
 * The pair values come from mps_expect_pairs (pairs one after the other), the site
 * values from mps_expect_site.  PDMRG_EINVAL on a gauge, size or kind
 * mismatch. */
int mps_order_parameter(pdmrg_ctx *ctx, pdmrg_mps *mps, int kind, int Lx, int Ly, double *value);

void mps_free(pdmrg_mps *mps);

#ifdef __cplusplus
}
#endif
#endif /* PDMRG_H */
