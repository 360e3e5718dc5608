// Records and launchers of the batched Jacobi SVD kernels (svd.hip).
#pragma once
#include "kernels.hpp"

namespace pdmrg {

// One matrix: nv rows of length len (W), rotation accumulator Z (nv x nv);
// a pair needs a rotation while its relative off-diagonal exceeds tol.
struct JacItem {
    double *W, *Z;
    double tol;
    int32_t nv, len;
};

// One block pair (blocks of 8 rows) of one matrix in a Jacobi round.
struct JacPair {
    int32_t item, bi, bj, pad_;
};

struct RowRef {
    const double *p;
    int32_t len, pad_;
};

// dst[r][c] = (trans ? src[c'][r'] : src[r'][c']) * rscale[r] * cscale[c]
// with r' = ridx ? ridx[r] : r, c' = cidx ? cidx[c] : c (scales and index
// maps optional).
struct CopyTask {
    const double *src;
    double *dst;
    const double *rscale, *cscale;
    int32_t rows, cols, sld, dld, trans, pad_;
    const int32_t *ridx, *cidx;
};

// Householder QR of a matrix stored as nv rows of length len (row p of A is
// column p of the factored len x nv matrix X = A^T), in panels of 16
// reflectors.  After panel j0: rows j0 .. j0+15 hold R[0..p-1][p] at
// positions < p, R[p][p] at position p and the reflector's tail (its entry p
// is 1) after it; T is the panel's upper-triangular compact-WY factor
// (H_j0 ... H_j0+15 = I - V T V^T).
constexpr int kQrPanel = 16;
constexpr int kQrMaxLen = 2048;   // longest row the panel kernel holds in registers
struct QrPanel {
    double *A;
    double *T;
    int32_t nv, len, j0, pad_;
};
// Applies the panel's reflectors (rows j0.. of V = A + j0 len) to up to 16
// target rows (row stride len) at positions j0 .. len-1: with d_j = v_j . y,
// y -= sum_j c_j v_j, c = T^T d (trans: the QR's trailing update, Q^T y) or
// c = T d (the product with Q from the right, y Q^T, panels taken last first).
struct QrApply {
    const double *V, *T;
    double *Y;
    int32_t nb, ntgt, len, j0, trans, pad_;
};
// Per matrix: R rows (nv x nv) from the factored A; Y = [Z, 0] (nv x len).
struct QrItem {
    const double *A, *Z;
    double *R, *Y;
    int32_t nv, len;
};

void launch_jac_round(const JacItem *items, const JacPair *pairs, int npairs, const int32_t *active,
                      unsigned long long *offmax, hipStream_t s);
void launch_identity(const JacItem *items, int nitems, int max_nv, hipStream_t s);
void launch_row_norms(const RowRef *rows, int nrows, double *out, hipStream_t s);
void launch_copies(const CopyTask *tasks, int ntasks, int64_t max_elems, hipStream_t s);
void launch_qr_panels(const QrPanel *tasks, int ntasks, int max_span, hipStream_t s);
void launch_qr_apply(const QrApply *tasks, int ntasks, hipStream_t s);
void launch_qr_extract_r(const QrItem *items, int nitems, int max_nv, hipStream_t s);
void launch_qr_embed_z(const QrItem *items, int nitems, int64_t max_elems, hipStream_t s);

}  // namespace pdmrg
