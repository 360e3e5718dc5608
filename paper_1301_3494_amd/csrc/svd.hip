// Batched one-sided block-Jacobi SVD kernels (FP64) for the truncation step.
//
// Each matrix is stored as nv row vectors of length len (W, row-major).  One
// Jacobi round rotates disjoint pairs of 8-row blocks: a workgroup forms the
// 16 x 16 Gram matrix of its two blocks, applies one cyclic Jacobi sweep to it
// in LDS and replaces the rows by the resulting combinations, sorted by
// decreasing norm; the same rotation is applied to the accumulator Z (nv x nv,
// starts at I).  Rounds follow the circle schedule, so every block pair meets
// once per sweep.  When no pair of a sweep needed a rotation (relative
// off-diagonal |G_ij| / sqrt(G_ii G_jj) <= tol) the rows are orthogonal:
// W = Z M, row norms are the singular values.
//
// Rows of W and Z are staged in LDS in 512-column chunks, both first chunks
// fetched at entry with all loads in flight; global accesses are raw buffer
// operations whose out-of-range offsets read zero / drop the store, so rows
// absent from the matrix need no branches.  The Gram matrix and the row
// rotations are 16 x 16 x K products on the FP64 matrix cores
// (v_mfma_f64_16x16x4).  A round of the inner sweep applies its 8 disjoint
// rotations J as A <- J^T A J, Q <- Q J from the previous round's copy
// (double buffer), one barrier per round: every wave computes the 8 angles
// itself (one pair per lane) and hands them to the lanes that use them by
// cross-lane shuffles while the operands of the update are already being
// read, since a round's partner indices follow from the schedule alone.
//
// Measured alternatives: 16-row blocks (32 x 32 inner problem) halve the
// rounds per sweep but cost more than twice as much per round; up to three
// inner sweeps per meeting save fewer outer rounds than they cost; 8 waves
// (W and Z rotated by separate halves at once) and the inner sweep in one
// wave without workgroup barriers are no faster.
//
// Also here: the Householder QR that preconditions the iteration (panel and
// reflector-application kernels, below) and the copy / norm helpers.
#include "svd.hpp"

#include <algorithm>
#include <stdexcept>

namespace pdmrg {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef unsigned u2 __attribute__((ext_vector_type(2)));

constexpr int JB = 8;            // rows per block
constexpr int J2 = 2 * JB;       // rows of a pair
constexpr int M = J2 - 1;        // circle schedule modulus
constexpr int JT = 256;          // 4 waves; one 16 x 16 entry per thread
constexpr int CH = 512;          // columns staged in LDS at a time
constexpr int U = J2 * CH / JT;  // staged elements per thread and chunk
static_assert(J2 * CH % JT == 0 && CH % 16 == 0, "chunk must split evenly over the threads and 16-column steps");
constexpr unsigned kOut = 0x80000000u;   // buffer offset past every record

__device__ __forceinline__ d4 mfma_f64(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Raw buffer descriptor over the n doubles at p (p is the same in every lane).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rows_rsrc(const double *p, int64_t n) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    void *q = reinterpret_cast<void *>(((uint64_t)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(q, 0, (int)(n * 8), 0x00020000);
}
__device__ __forceinline__ double bload(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, unsigned off, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, off, 0, 0);
}

// Circle schedule on J2 = M + 1 positions, round r: position M meets r, every
// other position i meets (2 r - i) mod M.  Pair l (0 <= l < J2 / 2) is
// {M, r} for l = 0 and {(r + l) mod M, (r - l) mod M} otherwise.
__device__ __forceinline__ int sched_partner(int i, int r) {
    if (i == M) return r;
    if (i == r) return M;
    return (2 * r - i + 2 * M) % M;
}
__device__ __forceinline__ int sched_pair(int i, int r) {
    if (i == M || i == r) return 0;
    const int d = (i - r + M) % M;
    return d <= M / 2 ? d : M - d;
}

// Rotation that zeroes a_pq of the symmetric 2 x 2 block (app, apq, aqq),
// p < q: column p becomes c col_p - s col_q, column q becomes s col_p + c col_q,
// with t = tan(angle) = 2 a_pq / (d + sign(d) sqrt(d^2 + 4 a_pq^2)),
// d = a_qq - a_pp (the root of smaller magnitude, |t| <= 1), c = 1 / sqrt(1 + t^2),
// s = t c.  d and 2 a_pq are first scaled by a power of two so the larger
// magnitude lies in [1/2, 1); then u = d^2 + 4 a_pq^2 lies in [1/4, 2],
// |d| + sqrt(u) in [1/2, 3] and 1 + t^2 in [1, 2], so hardware reciprocal and
// reciprocal square root estimates refined by Newton-type steps give full
// precision without range handling.
// The angle only decides how well a_pq is annihilated; the rotation is
// orthogonal to working precision whatever t is, because c and s follow from
// t.  Skipped (c = 1, s = 0) when a_pq^2 <= 1e-32 |a_pp a_qq| (the relative
// rule that resolves the small eigenvalues of a graded Gram matrix).
__device__ __forceinline__ void jacobi_angle(double app, double apq, double aqq, double &c, double &s) {
    const double d0 = aqq - app;
    const double big = fmax(fabs(d0), fabs(2.0 * apq));
    const int e = big > 0.0 ? __builtin_amdgcn_frexp_exp(big) : 0;
    const double d = __builtin_amdgcn_ldexp(d0, -e), a2 = __builtin_amdgcn_ldexp(2.0 * apq, -e);
    // h = sqrt(u): Goldschmidt iteration from the reciprocal square root estimate
    const double u = fma(d, d, a2 * a2);
    const double y0 = __builtin_amdgcn_rsq(u);
    double g = u * y0, hh = 0.5 * y0;
    const double r = fma(-hh, g, 0.5);
    g = fma(g, r, g);
    hh = fma(hh, r, hh);
    const double h = fma(fma(-g, g, u), hh, g);
    // t = a2 / den: reciprocal estimate and two Newton steps
    const double den = d >= 0.0 ? d + h : d - h;
    double q = __builtin_amdgcn_rcp(den);
    q = fma(q, fma(-den, q, 1.0), q);
    q = fma(q, fma(-den, q, 1.0), q);
    const double t = a2 * q;
    // c = (1 + t^2)^(-1/2): estimate y, w = 1 - v y^2, c = y (1 + w / 2 + 3 w^2 / 8)
    const double v = fma(t, t, 1.0);
    const double y = __builtin_amdgcn_rsq(v);
    const double w = fma(-v * y, y, 1.0);
    const double ct = fma(y * w, fma(w, 0.375, 0.5), y);
    const bool skip = apq == 0.0 || apq * apq <= 1e-32 * fabs(app * aqq);
    c = skip ? 1.0 : ct;
    s = skip ? 0.0 : t * ct;
}

__global__ __launch_bounds__(JT) void jac_pair_kernel(const JacItem *__restrict__ items,
                                                      const JacPair *__restrict__ pairs,
                                                      const int32_t *__restrict__ active,
                                                      unsigned long long *__restrict__ offmax) {
    const JacPair pr = pairs[blockIdx.x];
    const JacItem it = items[pr.item];
    if (!active[pr.item]) return;
    __shared__ double wrows[J2][CH + 1];   // W rows, current chunk
    __shared__ double zrows[J2][CH + 1];   // Z rows, current chunk
    __shared__ double Gp[4][J2][J2 + 1];
    __shared__ double A[2][J2][J2 + 1];
    __shared__ double Q[2][J2][J2 + 1];
    __shared__ int ev[J2];
    __shared__ double wred[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, g = lane >> 4;
    if (tid < J2) ev[tid] = tid;
    // rows of the pair present in the matrix form a prefix 0..n-1 (only the
    // last block of a matrix is partial, and a pair never holds two blocks
    // past it)
    const int n = min(max(it.nv - pr.bi * JB, 0), JB) + min(max(it.nv - pr.bj * JB, 0), JB);
    auto grow = [&](int r) { return r < JB ? pr.bi * JB + r : pr.bj * JB + (r - JB); };
    const __amdgpu_buffer_rsrc_t rW = rows_rsrc(it.W, (int64_t)it.nv * it.len);
    const __amdgpu_buffer_rsrc_t rZ = rows_rsrc(it.Z, (int64_t)it.nv * it.nv);

    // Element u of this thread in a chunk: flat index e = u JT + tid of the
    // J2 x CH chunk, row e / CH, column e % CH (consecutive threads take
    // consecutive columns of one row).
    auto load_chunk = [&](__amdgpu_buffer_rsrc_t rs, int len, int c0, double (&v)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = u * JT + tid, r = e / CH, c = c0 + e % CH;
            const unsigned off = (r < n && c < len) ? (unsigned)(((int64_t)grow(r) * len + c) * 8) : kOut;
            v[u] = bload(rs, off);
        }
    };
    auto store_chunk = [&](double (*dst)[CH + 1], const double (&v)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = u * JT + tid;
            dst[e / CH][e % CH] = v[u];
        }
    };
    {
        double v[U], z[U];
        load_chunk(rW, it.len, 0, v);
        load_chunk(rZ, it.nv, 0, z);
        store_chunk(wrows, v);
        store_chunk(zrows, z);
    }

    // ---- Gram matrix G = Wp Wp^T (Wp: the 16 rows).  MFMA j of a 16-wide K
    // step takes k = kk + 4 g + j from lane group g; A and B operands are the
    // same element Wp[r16][k]; the four waves split K and their partial tiles
    // are summed in a fixed order.
    const int nch = (it.len + CH - 1) / CH;
    {
        d4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int ch = 0; ch < nch; ++ch) {
            const int c0 = ch * CH;
            if (ch > 0) {
                double v[U];
                load_chunk(rW, it.len, c0, v);
                __syncthreads();
                store_chunk(wrows, v);
            }
            __syncthreads();
            const int w = min(CH, it.len - c0);
            for (int kk = wave * 16; kk < w; kk += 64) {
                double v[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) v[j] = wrows[r16][kk + 4 * g + j];
#pragma unroll
                for (int j = 0; j < 4; ++j) acc = mfma_f64(v[j], v[j], acc);
            }
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
    if (ei < ej && ej < n) {
        const double dd = A[0][ei][ei] * A[0][ej][ej];
        if (dd > 0.0) off = fabs(gij) / sqrt(dd);
    }
    for (int w = 32; w > 0; w >>= 1) off = fmax(off, __shfl_xor(off, w));
    if (lane == 0) wred[wave] = off;
    __syncthreads();
    const double poff = fmax(fmax(wred[0], wred[1]), fmax(wred[2], wred[3]));
    if (tid == 0) atomicMax(&offmax[pr.item], (unsigned long long)__double_as_longlong(poff));
    if (poff <= it.tol) return;
    // rows absent from the matrix: isolated with eigenvalue -1 (never rotated)
    A[0][ei][ej] = (ei >= n || ej >= n) ? (ei == ej ? -1.0 : 0.0) : gij;
    Q[0][ei][ej] = ei == ej ? 1.0 : 0.0;
    __syncthreads();

    // ---- one cyclic Jacobi sweep on the 16 x 16 Gram matrix.  A partial
    // diagonalisation is still an exact rotation of the rows; the outer
    // iteration measures orthogonality on fresh Gram matrices.
    int cur = 0;
    const int lp = lane % (J2 / 2);   // the pair whose angle this lane computes
    for (int r = 0; r < M; ++r) {
        const double(*Ac)[J2 + 1] = A[cur];
        const double(*Qc)[J2 + 1] = Q[cur];
        const int pa = lp == 0 ? M : (r + lp) % M, pb = (r - lp + M) % M;
        const int lo = min(pa, pb), hi = max(pa, pb);
        const double app = Ac[lo][lo], apq = Ac[lo][hi], aqq = Ac[hi][hi];
        const int pi = sched_partner(ei, r), pj = sched_partner(ej, r);
        const double a0 = Ac[ei][ej], a1 = Ac[ei][pj], a2 = Ac[pi][ej], a3 = Ac[pi][pj];
        const double q0 = Qc[ei][ej], q1 = Qc[ei][pj];
        double c, s;
        jacobi_angle(app, apq, aqq, c, s);
        // the lower index of a pair takes -s, the upper +s
        const int li = sched_pair(ei, r), lj = sched_pair(ej, r);
        const double ci = __shfl(c, li), si = __shfl(s, li);
        const double cj = __shfl(c, lj), sj = __shfl(s, lj);
        const double oi = ei < pi ? -si : si, oj = ej < pj ? -sj : sj;
        A[cur ^ 1][ei][ej] = ci * (cj * a0 + oj * a1) + oi * (cj * a2 + oj * a3);
        Q[cur ^ 1][ei][ej] = cj * q0 + oj * q1;
        __syncthreads();
        cur ^= 1;
    }
    // rank of each present row's eigenvalue, descending (ties: lower index first)
    if (tid < n) {
        const double di = A[cur][tid][tid];
        int rank = 0;
#pragma unroll
        for (int j = 0; j < J2; ++j) {
            const double dj = A[cur][j][j];
            rank += (j < n && (dj > di || (dj == di && j < tid))) ? 1 : 0;
        }
        ev[rank] = tid;
    }
    __syncthreads();

    // ---- new row o = sum_k Q[k][ev[o]] old row k, stored at row o of the
    // pair, as (16 x 16) x (16 x CH) MFMA products from the staged rows.
    double qa[4];
    unsigned dbase[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) qa[j] = r16 < n ? Q[cur][4 * j + g][ev[r16]] : 0.0;
    for (int pass = 0; pass < 2; ++pass) {
        const __amdgpu_buffer_rsrc_t rs = pass == 0 ? rW : rZ;
        double(*src)[CH + 1] = pass == 0 ? wrows : zrows;
        const int len = pass == 0 ? it.len : it.nv;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = 4 * r + g;
            dbase[r] = o < n ? (unsigned)((int64_t)grow(o) * len) : kOut;
        }
        // W: the last chunk of the Gram pass is still staged, so go backwards;
        // Z: chunk 0 is staged
        const int nc = (len + CH - 1) / CH;
        for (int i = 0; i < nc; ++i) {
            const int ch = pass == 0 ? nc - 1 - i : i;
            const int c0 = ch * CH;
            if (i > 0) {
                double v[U];
                load_chunk(rs, len, c0, v);
                __syncthreads();
                store_chunk(src, v);
            }
            __syncthreads();
            const int w = min(CH, len - c0);
            for (int n0 = wave * 16; n0 < w; n0 += 64) {
                const int col = n0 + r16;
                double b[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) b[j] = src[4 * j + g][col];
                d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int j = 0; j < 4; ++j) acc = mfma_f64(qa[j], b[j], acc);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const unsigned offr = (dbase[r] != kOut && col < w) ? (dbase[r] + c0 + col) * 8u : kOut;
                    bstore(rs, offr, acc[r]);
                }
            }
        }
    }
}

void launch_jac_round(const JacItem *items, const JacPair *pairs, int npairs, const int32_t *active,
                      unsigned long long *offmax, hipStream_t s) {
    if (npairs <= 0) return;
    hipLaunchKernelGGL(jac_pair_kernel, dim3(npairs), dim3(JT), 0, s, items, pairs, active, offmax);
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
        const int rs = t.ridx ? t.ridx[r] : r, cs = t.cidx ? t.cidx[c] : c;
        double v = t.trans ? t.src[(int64_t)cs * t.sld + rs] : t.src[(int64_t)rs * t.sld + cs];
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


// ---------------------------------------------------------------------------
// Householder QR preconditioning of the one-sided Jacobi iteration.
//
// Panel kernel: one workgroup of NT threads factors the 16 rows of a panel.
// Thread t holds positions j0 + t + NT u (u < UQ) of all 16 rows in
// registers.  Reflector j (pivot position p = j0 + j) needs one block
// reduction of 16 sums C_k = sum_{q > p} x_j[q] x_k[q] (C_j is the squared
// norm below the pivot) and the pivot-row entries E_k = x_k[p] (E_j is the
// pivot), which thread j publishes.  With beta = -sign(E_j) sqrt(E_j^2 + C_j),
// tau = (beta - E_j) / beta and v = x_j / (E_j - beta) below p (v_p = 1), the
// dot of v with row k is E_k + C_k / (E_j - beta): for later rows it gives
// their update, for earlier rows (which hold their reflectors there) the new
// column of T.  The sums are a reduce-scatter butterfly within each wave and
// a fixed-order sum over the waves, so every thread reads identical scalars
// and the result is reproducible.
template <int NT>
__device__ __forceinline__ void qr_sum16(double (&v)[16], double (*red)[16], double *res, int tid) {
    const int lane = tid & 63, wave = tid >> 6;
    double h8[8], h4[4], h2[2];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const bool up = lane & 16;
        h8[i] = (up ? v[8 + i] : v[i]) + __shfl_xor(up ? v[i] : v[8 + i], 16);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const bool up = lane & 8;
        h4[i] = (up ? h8[4 + i] : h8[i]) + __shfl_xor(up ? h8[i] : h8[4 + i], 8);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const bool up = lane & 4;
        h2[i] = (up ? h4[2 + i] : h4[i]) + __shfl_xor(up ? h4[i] : h4[2 + i], 4);
    }
    const bool up = lane & 2;
    double one = (up ? h2[1] : h2[0]) + __shfl_xor(up ? h2[0] : h2[1], 2);
    one += __shfl_xor(one, 1);
    one += __shfl_xor(one, 32);
    // lane bits 4..1 chose the halves: the lane holds value (lane >> 1) & 15
    if ((lane & 33) == 0) red[wave][(lane >> 1) & 15] = one;
    __syncthreads();
    if (tid < 16) {
        double a = red[0][tid];
#pragma unroll
        for (int w = 1; w < NT / 64; ++w) a += red[w][tid];
        res[tid] = a;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = res[i];
}

template <int NT, int UQ>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(1, 2))) void qr_panel_kernel(
    const QrPanel *tasks) {
    const QrPanel tk = tasks[blockIdx.x];
    const int nb = min(kQrPanel, tk.nv - tk.j0);
    const int tid = threadIdx.x;
    __shared__ double red[NT / 64][16];
    __shared__ double res[16];
    __shared__ double piv[2][kQrPanel];   // E of alternate steps: written before a step's first barrier
    __shared__ double Ts[kQrPanel][kQrPanel];
    if (tid < kQrPanel * kQrPanel) Ts[tid / kQrPanel][tid % kQrPanel] = 0.0;
    double x[kQrPanel][UQ];
#pragma unroll
    for (int r = 0; r < kQrPanel; ++r)
#pragma unroll
        for (int u = 0; u < UQ; ++u) {
            const int q = tk.j0 + tid + NT * u;
            x[r][u] = (r < nb && q < tk.len) ? tk.A[(int64_t)(tk.j0 + r) * tk.len + q] : 0.0;
        }
    // j runs as a loop; rows are picked and written back by selects, so every
    // register index is a constant
    for (int j = 0; j < nb; ++j) {   // nb is uniform over the workgroup
        const int p = tk.j0 + j;
        double xj[UQ];
#pragma unroll
        for (int u = 0; u < UQ; ++u) {
            double t = x[0][u];
#pragma unroll
            for (int r = 1; r < kQrPanel; ++r) t = r == j ? x[r][u] : t;
            const int q = tk.j0 + tid + NT * u;
            xj[u] = q > p ? t : 0.0;   // below the pivot only
        }
        double cs[kQrPanel];
#pragma unroll
        for (int k = 0; k < kQrPanel; ++k) {
            double t = 0.0;
#pragma unroll
            for (int u = 0; u < UQ; ++u) t = fma(xj[u], x[k][u], t);
            cs[k] = t;
        }
        double *E = piv[j & 1];
        if (tid == j)   // position p is thread j's u = 0
#pragma unroll
            for (int k = 0; k < kQrPanel; ++k) E[k] = x[k][0];
        qr_sum16<NT>(cs, red, res, tid);
        double sig = cs[0], alpha = E[0];
#pragma unroll
        for (int k = 1; k < kQrPanel; ++k) {
            sig = k == j ? cs[k] : sig;
            alpha = k == j ? E[k] : alpha;
        }
        double tau = 0.0, beta = alpha, inv = 0.0;
        if (sig > 0.0) {
            const double nrm = sqrt(fma(alpha, alpha, sig));
            beta = alpha >= 0.0 ? -nrm : nrm;
            tau = (beta - alpha) / beta;
            inv = 1.0 / (alpha - beta);
        }
        // reflector v: 0 before p, 1 at p, x * inv after; row j keeps beta at p
        double v[UQ];
#pragma unroll
        for (int u = 0; u < UQ; ++u) {
            const int q = tk.j0 + tid + NT * u;
            v[u] = q > p ? xj[u] * inv : (q == p ? 1.0 : 0.0);
            const bool keep = q < p;
#pragma unroll
            for (int r = 0; r < kQrPanel; ++r) x[r][u] = (r == j && !keep) ? (q == p ? beta : v[u]) : x[r][u];
        }
        // d_k = v . x_k (row k after the earlier steps)
        double d[kQrPanel];
#pragma unroll
        for (int k = 0; k < kQrPanel; ++k) d[k] = fma(cs[k], inv, E[k]);
#pragma unroll
        for (int k = 0; k < kQrPanel; ++k) {
            const double f = (k > j && k < nb) ? tau * d[k] : 0.0;
#pragma unroll
            for (int u = 0; u < UQ; ++u) x[k][u] = fma(-f, v[u], x[k][u]);
        }
        // T[0:j][j] = -tau T[0:j][0:j] (V[:, 0:j]^T v); T[j][j] = tau.  Thread i
        // only reads row i of T, which it wrote itself.
        if (tid < j) {
            double t = 0.0;
#pragma unroll
            for (int l = 0; l < kQrPanel; ++l)
                if (l >= tid && l < j) t = fma(Ts[tid][l], d[l], t);
            Ts[tid][j] = -tau * t;
        }
        if (tid == j) Ts[j][j] = tau;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kQrPanel; ++r)
#pragma unroll
        for (int u = 0; u < UQ; ++u) {
            const int q = tk.j0 + tid + NT * u;
            if (r < nb && q < tk.len) tk.A[(int64_t)(tk.j0 + r) * tk.len + q] = x[r][u];
        }
    if (tid < kQrPanel * kQrPanel) tk.T[tid] = Ts[tid / kQrPanel][tid % kQrPanel];
}

void launch_qr_panels(const QrPanel *tasks, int ntasks, int max_span, hipStream_t s) {
    if (ntasks <= 0) return;
    if (max_span <= 512)
        hipLaunchKernelGGL((qr_panel_kernel<256, 2>), dim3(ntasks), dim3(256), 0, s, tasks);
    else if (max_span <= 1024)
        hipLaunchKernelGGL((qr_panel_kernel<256, 4>), dim3(ntasks), dim3(256), 0, s, tasks);
    else if (max_span <= 2048)
        hipLaunchKernelGGL((qr_panel_kernel<512, 4>), dim3(ntasks), dim3(512), 0, s, tasks);
    else
        throw std::invalid_argument("qr panel: rows longer than the panel kernel holds");
}
static_assert(kQrMaxLen == 2048, "panel kernel reach");

// Apply kernel: one workgroup of 4 waves per (panel, group of 16 target rows).
// D = V Y^T over positions j0.. (FP64 MFMA, reflector rows masked to their
// support with the unit entry), C = T^T D or T D, then Y -= C^T V (FP64 MFMA),
// both through the same 512-position chunks staged in LDS as the Jacobi
// kernel uses.
__global__ __launch_bounds__(JT) void qr_apply_kernel(const QrApply *tasks) {
    const QrApply tk = tasks[blockIdx.x];
    __shared__ double vrows[J2][CH + 1];
    __shared__ double yrows[J2][CH + 1];
    __shared__ double Dp[4][J2][J2 + 1];
    __shared__ double Cs[J2][J2 + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, g = lane >> 4;
    const __amdgpu_buffer_rsrc_t rV = rows_rsrc(tk.V, (int64_t)tk.nb * tk.len);
    const __amdgpu_buffer_rsrc_t rY = rows_rsrc(tk.Y, (int64_t)tk.ntgt * tk.len);
    const int span = tk.len - tk.j0;
    const int nch = (span + CH - 1) / CH;
    auto stage = [&](int c0) {
        double a[U], b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = u * JT + tid, r = e / CH, q = tk.j0 + c0 + e % CH;
            const bool in = q < tk.len;
            const unsigned ov = (r < tk.nb && in && q > tk.j0 + r) ? (unsigned)(((int64_t)r * tk.len + q) * 8) : kOut;
            const unsigned oy = (r < tk.ntgt && in) ? (unsigned)(((int64_t)r * tk.len + q) * 8) : kOut;
            a[u] = (r < tk.nb && q == tk.j0 + r) ? 1.0 : bload(rV, ov);
            b[u] = bload(rY, oy);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = u * JT + tid;
            vrows[e / CH][e % CH] = a[u];
            yrows[e / CH][e % CH] = b[u];
        }
        __syncthreads();
    };
    {
        d4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int ch = 0; ch < nch; ++ch) {
            const int c0 = ch * CH;
            stage(c0);
            const int w = min(CH, span - c0);
            for (int kk = wave * 16; kk < w; kk += 64) {
                double a[4], b[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    a[j] = vrows[r16][kk + 4 * g + j];
                    b[j] = yrows[r16][kk + 4 * g + j];
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) acc = mfma_f64(a[j], b[j], acc);
            }
        }
        // D[i][c] = v_i . y_c; register r of lane l: row 4 r + l / 16, column l % 16
#pragma unroll
        for (int r = 0; r < 4; ++r) Dp[wave][4 * r + g][r16] = acc[r];
    }
    __syncthreads();
    {
        const int ei = tid / J2, ej = tid % J2;
        double c = 0.0;
#pragma unroll
        for (int i = 0; i < J2; ++i) {
            const double t = tk.trans ? tk.T[i * J2 + ei] : tk.T[ei * J2 + i];
            const double dij = ((Dp[0][i][ej] + Dp[1][i][ej]) + Dp[2][i][ej]) + Dp[3][i][ej];
            c = fma(t, dij, c);
        }
        Cs[ei][ej] = c;   // coefficient of reflector ei in target row ej
    }
    __syncthreads();
    double qa[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) qa[j] = Cs[4 * j + g][r16];
    unsigned dbase[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int o = 4 * r + g;
        dbase[r] = o < tk.ntgt ? (unsigned)((int64_t)o * tk.len) : kOut;
    }
    // the last chunk is still staged: go backwards
    for (int i = 0; i < nch; ++i) {
        const int ch = nch - 1 - i;
        const int c0 = ch * CH;
        if (i > 0) stage(c0);
        const int w = min(CH, span - c0);
        for (int n0 = wave * 16; n0 < w; n0 += 64) {
            const int col = n0 + r16;
            double b[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = vrows[4 * j + g][col];
            d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int j = 0; j < 4; ++j) acc = mfma_f64(qa[j], b[j], acc);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int o = 4 * r + g;
                const unsigned offr =
                    (dbase[r] != kOut && col < w) ? (dbase[r] + tk.j0 + c0 + col) * 8u : kOut;
                bstore(rY, offr, yrows[o][col] - acc[r]);
            }
        }
        __syncthreads();   // before the next chunk overwrites the staged rows
    }
}

void launch_qr_apply(const QrApply *tasks, int ntasks, hipStream_t s) {
    if (ntasks > 0) hipLaunchKernelGGL(qr_apply_kernel, dim3(ntasks), dim3(JT), 0, s, tasks);
}

// R[i][j] = A[j][i] for j >= i (the factor's upper triangle as rows), else 0.
__global__ void qr_extract_r_kernel(const QrItem *items) {
    const QrItem it = items[blockIdx.y];
    const int64_t n = (int64_t)it.nv * it.nv;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / it.nv), j = (int)(e % it.nv);
        it.R[e] = j >= i ? it.A[(int64_t)j * it.len + i] : 0.0;
    }
}

void launch_qr_extract_r(const QrItem *items, int nitems, int max_nv, hipStream_t s) {
    if (nitems <= 0 || max_nv <= 0) return;
    const int g = std::min(1024, (max_nv * max_nv + 255) / 256);
    hipLaunchKernelGGL(qr_extract_r_kernel, dim3(g, nitems), dim3(256), 0, s, items);
}

// Y[r][c] = Z[r][c] for c < nv, 0 after (Y: nv x len).
__global__ void qr_embed_z_kernel(const QrItem *items) {
    const QrItem it = items[blockIdx.y];
    const int64_t n = (int64_t)it.nv * it.len;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / it.len), c = (int)(e % it.len);
        it.Y[e] = c < it.nv ? it.Z[(int64_t)r * it.nv + c] : 0.0;
    }
}

void launch_qr_embed_z(const QrItem *items, int nitems, int64_t max_elems, hipStream_t s) {
    if (nitems <= 0 || max_elems <= 0) return;
    const int g = (int)std::min<int64_t>(1024, (max_elems + 255) / 256);
    hipLaunchKernelGGL(qr_embed_z_kernel, dim3(g, nitems), dim3(256), 0, s, items);
}

}  // namespace pdmrg
