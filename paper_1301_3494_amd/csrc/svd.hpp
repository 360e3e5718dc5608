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

// dst[r][c] = (trans ? src[c][r] : src[r][c]) * rscale[r] * cscale[c]
// (scales optional).
struct CopyTask {
    const double *src;
    double *dst;
    const double *rscale, *cscale;
    int32_t rows, cols, sld, dld, trans, pad_;
};

void launch_jac_round(const JacItem *items, const JacPair *pairs, int npairs, const int32_t *active,
                      unsigned long long *offmax, hipStream_t s);
void launch_identity(const JacItem *items, int nitems, int max_nv, hipStream_t s);
void launch_row_norms(const RowRef *rows, int nrows, double *out, hipStream_t s);
void launch_copies(const CopyTask *tasks, int ntasks, int64_t max_elems, hipStream_t s);

}  // namespace pdmrg
