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
//
// The 16 rows are staged through LDS in 512-column chunks (coalesced, all
// loads in flight together); the Gram matrix and the row rotations are
// 16 x 16 x K products on the FP64 matrix cores (v_mfma_f64_16x16x4, 4 waves
// over disjoint K / column ranges).
// The 16 x 16 eigenproblem runs in LDS with one matrix entry per thread: a
// round's 8 disjoint rotations J are applied as A <- J^T A J, Q <- Q J from
// the previous round's copy (double buffer), two barriers per round.
#include "svd.hpp"

namespace pdmrg {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int JB = 8, J2 = 16;
constexpr int JT = 256;   // 4 waves; one 16 x 16 entry per thread in the eigensolver
constexpr int JCH = 512;  // columns of the 16 rows staged in LDS at a time

__device__ __forceinline__ d4 mfma_f64(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__global__ __launch_bounds__(JT) void jac_pair_kernel(const JacItem *__restrict__ items,
                                                      const JacPair *__restrict__ pairs,
                                                      const int32_t *__restrict__ active,
                                                      unsigned long long *__restrict__ offmax, double tol) {
    const JacPair pr = pairs[blockIdx.x];
    if (!active[pr.item]) return;
    const JacItem it = items[pr.item];
    __shared__ double rows[J2][JCH + 1];
    __shared__ double Gp[4][J2][J2 + 1];
    __shared__ double A[2][J2][J2 + 1];
    __shared__ double Q[2][J2][J2 + 1];
    __shared__ double cself[J2], cother[J2];
    __shared__ int partner[J2];
    __shared__ int rowid[J2], ev[J2], vp[J2];
    __shared__ int nvalid;
    __shared__ double wred[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, g = lane >> 4;
    if (tid < J2) {
        const int r = tid < JB ? pr.bi * JB + tid : pr.bj * JB + (tid - JB);
        rowid[tid] = r < it.nv ? r : -1;
    }
    __syncthreads();

    // Stage the 16 rows through LDS in chunks of JCH columns (coalesced
    // loads, all in flight together); rows absent from the matrix read as 0.
    auto stage = [&](const double *M, int len, int c0) {
        constexpr int U = J2 * JCH / JT;
        const int w = min(JCH, len - c0);
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = tid + u * JT, r = e / JCH, c = e % JCH;
            v[u] = (rowid[r] >= 0 && c < w) ? M[(int64_t)rowid[r] * len + c0 + c] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = tid + u * JT;
            rows[e / JCH][e % JCH] = v[u];
        }
    };

    // ---- Gram matrix G = Wp Wp^T (Wp: the 16 rows).  MFMA j of a 16-wide K
    // chunk takes k = kk + 4 g + j from lane group g; A and B operands are the
    // same element Wp[r16][k].
    {
        d4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int c0 = 0; c0 < it.len; c0 += JCH) {
            stage(it.W, it.len, c0);
            __syncthreads();
            const int w = min(JCH, it.len - c0);
            for (int kk = wave * 16; kk < w; kk += 64) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const double v = rows[r16][kk + 4 * g + j];
                    acc = mfma_f64(v, v, acc);
                }
            }
            __syncthreads();
        }
        // v_mfma_f64_16x16x4 result: register r of lane l is row 4 r + l / 16, column l % 16
#pragma unroll
        for (int r = 0; r < 4; ++r) Gp[wave][4 * r + g][r16] = acc[r];
    }
    __syncthreads();
    const int ei = tid / J2, ej = tid % J2;   // this thread's entry of the 16 x 16 matrices
    const double gij = ((Gp[0][ei][ej] + Gp[1][ei][ej]) + Gp[2][ei][ej]) + Gp[3][ei][ej];
    A[0][ei][ej] = gij;
    __syncthreads();
    // ---- relative off-diagonal of this pair
    double off = 0.0;
    if (ei < ej && rowid[ei] >= 0 && rowid[ej] >= 0) {
        const double dd = A[0][ei][ei] * A[0][ej][ej];
        if (dd > 0.0) off = fabs(gij) / sqrt(dd);
    }
    for (int w = 32; w > 0; w >>= 1) off = fmax(off, __shfl_xor(off, w));
    if (lane == 0) wred[wave] = off;
    __syncthreads();
    const double poff = fmax(fmax(wred[0], wred[1]), fmax(wred[2], wred[3]));
    if (tid == 0) atomicMax(&offmax[pr.item], (unsigned long long)__double_as_longlong(poff));
    if (poff <= tol) return;
    // rows absent from the matrix: isolated with eigenvalue -1 (never rotated)
    {
        double v = gij;
        if (rowid[ei] < 0 || rowid[ej] < 0) v = (ei == ej) ? -1.0 : 0.0;
        A[0][ei][ej] = v;
        Q[0][ei][ej] = (ei == ej) ? 1.0 : 0.0;
    }
    __syncthreads();

    // ---- 16 x 16 cyclic Jacobi, at most 3 sweeps.  Relative skipping rule
    // |a_pq| <= 1e-16 sqrt(|a_pp a_qq|), so the small eigenvalues of a graded
    // Gram matrix are resolved in relative terms.  A partial
    // diagonalisation is still an exact rotation of the rows; the outer
    // iteration measures orthogonality on fresh Gram matrices.
    int cur = 0;
    for (int sweep = 0; sweep < 3; ++sweep) {
        if (sweep > 0) {
            // stop once every off-diagonal entry is below 1e-15 of sqrt(a_ii a_jj)
            double o = 0.0;
            if (ei != ej) {
                const double v = fabs(A[cur][ei][ej]);
                if (v != 0.0) {
                    const double dd = sqrt(fabs(A[cur][ei][ei] * A[cur][ej][ej]));
                    o = dd > 0.0 ? v / dd : 1.0;
                }
            }
            for (int w = 32; w > 0; w >>= 1) o = fmax(o, __shfl_xor(o, w));
            if (lane == 0) wred[wave] = o;
            __syncthreads();
            const double ro = fmax(fmax(wred[0], wred[1]), fmax(wred[2], wred[3]));
            __syncthreads();
            if (ro <= 1e-15) break;
        }
        for (int r = 0; r < J2 - 1; ++r) {
            if (tid < J2 / 2) {
                int p = (tid == 0) ? J2 - 1 : (r + tid) % (J2 - 1);
                int q = (r - tid + (J2 - 1)) % (J2 - 1);
                if (p > q) { const int t = p; p = q; q = t; }
                double c = 1.0, sn = 0.0;
                const double apq = A[cur][p][q];
                const double app = A[cur][p][p], aqq = A[cur][q][q];
                if (apq != 0.0 && fabs(apq) > 1e-16 * sqrt(fabs(app * aqq))) {
                    const double tau = (aqq - app) / (2.0 * apq);
                    const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + t * t);
                    sn = t * c;
                }
                // new column p = c col_p - s col_q, new column q = s col_p + c col_q
                partner[p] = q; cself[p] = c; cother[p] = -sn;
                partner[q] = p; cself[q] = c; cother[q] = sn;
            }
            __syncthreads();
            {
                const int pi = partner[ei], pj = partner[ej];
                const double si = cself[ei], oi = cother[ei], sj = cself[ej], oj = cother[ej];
                const double (*Ac)[J2 + 1] = A[cur];
                const double v = si * (sj * Ac[ei][ej] + oj * Ac[ei][pj]) + oi * (sj * Ac[pi][ej] + oj * Ac[pi][pj]);
                A[cur ^ 1][ei][ej] = v;
                Q[cur ^ 1][ei][ej] = sj * Q[cur][ei][ej] + oj * Q[cur][ei][pj];
            }
            __syncthreads();
            cur ^= 1;
        }
    }
    if (tid == 0) {
        // valid positions in order; valid eigenvectors sorted by descending eigenvalue
        int n = 0;
        for (int j = 0; j < J2; ++j)
            if (rowid[j] >= 0) { vp[n] = j; ev[n] = j; ++n; }
        for (int a = 0; a < n; ++a) {
            int best = a;
            for (int b = a + 1; b < n; ++b)
                if (A[cur][ev[b]][ev[b]] > A[cur][ev[best]][ev[best]]) best = b;
            const int t = ev[a]; ev[a] = ev[best]; ev[best] = t;
        }
        nvalid = n;
    }
    __syncthreads();
    const int n = nvalid;

    // ---- rotate the W rows and Z rows: new row vp[o] = sum_k Q[k][ev[o]] old row k,
    // as (16 x 16) x (16 x JCH) MFMA products from the staged rows; every
    // chunk is staged completely before any of its columns is written.
    const double qa[4] = {r16 < n ? Q[cur][g][ev[r16]] : 0.0, r16 < n ? Q[cur][4 + g][ev[r16]] : 0.0,
                          r16 < n ? Q[cur][8 + g][ev[r16]] : 0.0, r16 < n ? Q[cur][12 + g][ev[r16]] : 0.0};
    int dst[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) dst[r] = (4 * r + g) < n ? rowid[vp[4 * r + g]] : -1;
    for (int pass = 0; pass < 2; ++pass) {
        double *M = pass == 0 ? it.W : it.Z;
        const int len = pass == 0 ? it.len : it.nv;
        // W rows are still staged when they fit in one chunk
        const bool staged = pass == 0 && it.len <= JCH;
        for (int c0 = 0; c0 < len; c0 += JCH) {
            if (!staged) {
                __syncthreads();
                stage(M, len, c0);
            }
            __syncthreads();
            const int w = min(JCH, len - c0);
            for (int n0 = wave * 16; n0 < w; n0 += 64) {
                const int col = n0 + r16;
                d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int j = 0; j < 4; ++j) acc = mfma_f64(qa[j], rows[4 * j + g][col], acc);
                if (col < w)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (dst[r] >= 0) M[(int64_t)dst[r] * len + c0 + col] = acc[r];
            }
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
