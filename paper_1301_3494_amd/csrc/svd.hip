// Batched one-sided block-Jacobi SVD kernels (FP64) for the truncation step.
//
// Each matrix is stored as nv row vectors of length len (W, row-major).  One
// Jacobi round rotates disjoint pairs of 8-row blocks: a workgroup forms the
// 16 x 16 Gram matrix of its two blocks, diagonalises it with cyclic Jacobi
// in LDS and replaces the rows by the eigenvector combinations, making all
// 16 rows mutually orthogonal; the same rotation is applied to the
// accumulator Z (nv x nv, starts at I).  Rounds follow the circle schedule,
// so every block pair meets once per sweep.  When no pair of a sweep needed a
// rotation (relative off-diagonal |G_ij| / sqrt(G_ii G_jj) <= tol) the rows
// are orthogonal: W = Z M, row norms are the singular values.
#include "svd.hpp"

namespace pdmrg {

constexpr int JB = 8, J2 = 16, JCH = 256;

// Threads per block pair: the row streaming (Gram, rotation) needs several
// waves for latency hiding; the 16 x 16 eigensolver is short.
constexpr int JT = 256;

__device__ void sym_eig16(double (*A)[J2 + 1], double (*Q)[J2 + 1], double *red, int *rp, int *rq, double *rc,
                          double *rs) {
    const int tid = threadIdx.x;
    for (int e = tid; e < J2 * J2; e += JT) Q[e / J2][e % J2] = (e / J2 == e % J2) ? 1.0 : 0.0;
    __syncthreads();
    // Relative skipping rule |a_pq| <= tol sqrt(|a_pp a_qq|), so that small
    // eigenvalues of a graded Gram matrix are resolved in relative terms (a
    // norm-wide rule would never rotate them).  Only a few sweeps: the outer
    // block-Jacobi iteration re-measures orthogonality on fresh Gram matrices,
    // so a partial diagonalisation (still an exact rotation of the rows) is
    // enough and convergence is decided there.
    for (int sweep = 0; sweep < 3; ++sweep) {
        double off = 0.0;
        for (int e = tid; e < J2 * J2; e += JT) {
            const int i = e / J2, j = e % J2;
            if (i >= j) continue;
            const double v = fabs(A[i][j]);
            if (v == 0.0) continue;
            const double dd = sqrt(fabs(A[i][i] * A[j][j]));
            off = fmax(off, dd > 0.0 ? v / dd : 1.0);
        }
        red[tid] = off;
        __syncthreads();
        for (int w = JT / 2; w > 0; w >>= 1) {
            if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
            __syncthreads();
        }
        const double roff = red[0];
        __syncthreads();
        if (roff <= 1e-15) break;
        for (int r = 0; r < J2 - 1; ++r) {
            if (tid < J2 / 2) {
                int p = (tid == 0) ? J2 - 1 : (r + tid) % (J2 - 1);
                int q = (r - tid + (J2 - 1)) % (J2 - 1);
                if (p > q) { const int t = p; p = q; q = t; }
                double c = 1.0, s = 0.0;
                const double apq = A[p][q];
                if (apq != 0.0 && fabs(apq) > 1e-16 * sqrt(fabs(A[p][p] * A[q][q]))) {
                    const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
                    const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + t * t);
                    s = t * c;
                }
                rp[tid] = p; rq[tid] = q; rc[tid] = c; rs[tid] = s;
            }
            __syncthreads();
            for (int e = tid; e < (J2 / 2) * J2; e += JT) {
                const int pr = e / J2, i = e % J2;
                const int p = rp[pr], q = rq[pr];
                const double c = rc[pr], s = rs[pr];
                if (s == 0.0) continue;
                const double ap = A[i][p], aq = A[i][q];
                A[i][p] = c * ap - s * aq;
                A[i][q] = s * ap + c * aq;
                const double qp = Q[i][p], qq = Q[i][q];
                Q[i][p] = c * qp - s * qq;
                Q[i][q] = s * qp + c * qq;
            }
            __syncthreads();
            for (int e = tid; e < (J2 / 2) * J2; e += JT) {
                const int pr = e / J2, j = e % J2;
                const int p = rp[pr], q = rq[pr];
                const double c = rc[pr], s = rs[pr];
                if (s == 0.0) continue;
                const double ap = A[p][j], aq = A[q][j];
                A[p][j] = c * ap - s * aq;
                A[q][j] = s * ap + c * aq;
            }
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(JT) void jac_pair_kernel(const JacItem *__restrict__ items,
                                                      const JacPair *__restrict__ pairs,
                                                      const int32_t *__restrict__ active,
                                                      unsigned long long *__restrict__ offmax, double tol) {
    const JacPair pr = pairs[blockIdx.x];
    if (!active[pr.item]) return;
    const JacItem it = items[pr.item];
    __shared__ double chunk[J2][JCH + 1];
    __shared__ double G[J2][J2 + 1];
    __shared__ double Q[J2][J2 + 1];
    __shared__ double red[JT];
    __shared__ double rc[J2 / 2], rs[J2 / 2];
    __shared__ int rp[J2 / 2], rq[J2 / 2];
    __shared__ int rowid[J2], ev[J2], vp[J2];
    __shared__ int nvalid;
    const int tid = threadIdx.x;
    if (tid < J2) {
        const int r = tid < JB ? pr.bi * JB + tid : pr.bj * JB + (tid - JB);
        rowid[tid] = r < it.nv ? r : -1;
    }
    __syncthreads();
    // Gram matrix of the 16 rows: 136 (r <= s) entries, up to 3 per lane
    constexpr int NG = J2 * (J2 + 1) / 2;
    int gr[3], gs[3];
    double acc[3] = {0.0, 0.0, 0.0};
    for (int u = 0; u < 3; ++u) {
        int t = tid + u * JT, r = 0;
        gr[u] = gs[u] = -1;
        if (t < NG) {
            while (t >= J2 - r) { t -= J2 - r; ++r; }
            gr[u] = r;
            gs[u] = r + t;
        }
    }
    for (int c0 = 0; c0 < it.len; c0 += JCH) {
        for (int e = tid; e < J2 * JCH; e += JT) {
            const int r = e / JCH, c = e % JCH, gc = c0 + c;
            chunk[r][c] = (rowid[r] >= 0 && gc < it.len) ? it.W[(int64_t)rowid[r] * it.len + gc] : 0.0;
        }
        __syncthreads();
        for (int u = 0; u < 3; ++u)
            if (gr[u] >= 0)
                for (int c = 0; c < JCH; ++c) acc[u] += chunk[gr[u]][c] * chunk[gs[u]][c];
        __syncthreads();
    }
    double off = 0.0;
    for (int u = 0; u < 3; ++u)
        if (gr[u] >= 0) {
            G[gr[u]][gs[u]] = acc[u];
            G[gs[u]][gr[u]] = acc[u];
        }
    __syncthreads();
    // relative off-diagonal of this pair
    for (int u = 0; u < 3; ++u)
        if (gr[u] >= 0 && gr[u] != gs[u] && rowid[gr[u]] >= 0 && rowid[gs[u]] >= 0) {
            const double dd = G[gr[u]][gr[u]] * G[gs[u]][gs[u]];
            if (dd > 0.0) off = fmax(off, fabs(G[gr[u]][gs[u]]) / sqrt(dd));
        }
    red[tid] = off;
    __syncthreads();
    for (int w = JT / 2; w > 0; w >>= 1) {
        if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
        __syncthreads();
    }
    const double poff = red[0];
    __syncthreads();
    if (tid == 0) atomicMax(&offmax[pr.item], (unsigned long long)__double_as_longlong(poff));
    if (poff <= tol) return;
    // rows absent from the matrix: isolated with eigenvalue -1 (never rotated)
    if (tid < J2 && rowid[tid] < 0)
        for (int j = 0; j < J2; ++j) G[tid][j] = (j == tid) ? -1.0 : 0.0;
    __syncthreads();
    if (tid < J2 && rowid[tid] < 0)
        for (int j = 0; j < J2; ++j)
            if (j != tid) G[j][tid] = 0.0;
    __syncthreads();
    sym_eig16(G, Q, red, rp, rq, rc, rs);
    if (tid == 0) {
        // valid positions in order; valid eigenvectors sorted by descending eigenvalue
        int n = 0;
        for (int j = 0; j < J2; ++j)
            if (rowid[j] >= 0) { vp[n] = j; ev[n] = j; ++n; }
        for (int a = 0; a < n; ++a) {
            int best = a;
            for (int b = a + 1; b < n; ++b)
                if (G[ev[b]][ev[b]] > G[ev[best]][ev[best]]) best = b;
            const int t = ev[a]; ev[a] = ev[best]; ev[best] = t;
        }
        nvalid = n;
    }
    __syncthreads();
    const int n = nvalid;
    // rotate W rows and Z rows: new row vp[j] = sum_s Q[s][ev[j]] old row s
    for (int pass = 0; pass < 2; ++pass) {
        double *M = pass == 0 ? it.W : it.Z;
        const int len = pass == 0 ? it.len : it.nv;
        for (int c0 = 0; c0 < len; c0 += JCH) {
            for (int e = tid; e < J2 * JCH; e += JT) {
                const int r = e / JCH, c = e % JCH, gc = c0 + c;
                chunk[r][c] = (rowid[r] >= 0 && gc < len) ? M[(int64_t)rowid[r] * len + gc] : 0.0;
            }
            __syncthreads();
            for (int e = tid; e < n * JCH; e += JT) {
                const int j = e / JCH, c = e % JCH, gc = c0 + c;
                if (gc >= len) continue;
                const int col = ev[j];
                double v = 0.0;
                for (int s = 0; s < J2; ++s) v += Q[s][col] * chunk[s][c];
                M[(int64_t)rowid[vp[j]] * len + gc] = v;
            }
            __syncthreads();
        }
    }
}

void launch_jac_round(const JacItem *items, const JacPair *pairs, int npairs, const int32_t *active,
                      unsigned long long *offmax, double tol, hipStream_t s) {
    if (npairs <= 0) return;
    hipLaunchKernelGGL(jac_pair_kernel, dim3(npairs), dim3(JT), 0, s, items, pairs, active, offmax, tol);
}

__global__ void identity_kernel(const JacItem *items) {
    const JacItem it = items[blockIdx.y];
    const int64_t n = (int64_t)it.nv * it.nv;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        it.Z[e] = (e / it.nv == e % it.nv) ? 1.0 : 0.0;
}

void launch_identity(const JacItem *items, int nitems, int max_nv, hipStream_t s) {
    if (nitems <= 0 || max_nv <= 0) return;
    const int g = std::min(1024, (max_nv * max_nv + 255) / 256);
    hipLaunchKernelGGL(identity_kernel, dim3(g, nitems), dim3(256), 0, s, items);
}

__global__ __launch_bounds__(256) void row_norm_kernel(const RowRef *rows, double *out) {
    __shared__ double sh[256];
    const RowRef r = rows[blockIdx.x];
    double acc = 0.0;
    for (int c = threadIdx.x; c < r.len; c += 256) acc += r.p[c] * r.p[c];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sqrt(sh[0]);
}

void launch_row_norms(const RowRef *rows, int nrows, double *out, hipStream_t s) {
    if (nrows > 0) hipLaunchKernelGGL(row_norm_kernel, dim3(nrows), dim3(256), 0, s, rows, out);
}

__global__ __launch_bounds__(256) void copy_kernel(const CopyTask *tasks) {
    const CopyTask t = tasks[blockIdx.y];
    const int64_t n = (int64_t)t.rows * t.cols;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / t.cols), c = (int)(e % t.cols);
        double v = t.trans ? t.src[(int64_t)c * t.sld + r] : t.src[(int64_t)r * t.sld + c];
        if (t.rscale) v *= t.rscale[r];
        if (t.cscale) v *= t.cscale[c];
        t.dst[(int64_t)r * t.dld + c] = v;
    }
}

void launch_copies(const CopyTask *tasks, int ntasks, int64_t max_elems, hipStream_t s) {
    if (ntasks <= 0 || max_elems <= 0) return;
    const int g = (int)std::min<int64_t>(256, (max_elems + 255) / 256);
    hipLaunchKernelGGL(copy_kernel, dim3(g, ntasks), dim3(256), 0, s, tasks);
}

}  // namespace pdmrg
