// Single-workgroup tile operations: Cholesky of a diagonal tile (POTRF) and
// inverse of a lower-triangular tile (the "TRSM(L_ii^T, I)" of Phase 1,
// i.e. TRTRI).  One workgroup of 256 threads works on one tile held in global
// memory (it stays in L2 while the workgroup runs); 16 x 16 sub-blocks go
// through LDS and registers, and the rank-16 trailing updates run on the
// FP64 matrix cores.
#pragma once
#include "common.hpp"

#define TO_LDD 17   // LDS leading dimension of 16-wide panels

// Lower-triangle tile index t -> (I, J), J <= I.
__device__ inline void tri_decode(int t, int& I, int& J) {
    int i = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (i * (i + 1) / 2 > t) --i;
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    I = i;
    J = t - i * (i + 1) / 2;
}

__device__ inline void neumaier(double& s, double& c, double x) {
    double t = s + x;
    if (fabs(s) >= fabs(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
}

// LDS needed by potrf_tile for a tile of order m (m <= 256).
__host__ __device__ inline int potrf_smem_doubles(int m) { return 16 * TO_LDD + 16 + (m - 16) * TO_LDD; }

// In-place Cholesky of the m x m lower triangle of M (column-major, leading
// dimension ld), m a multiple of 16, m <= 256.  Right-looking, 16-column
// panels: the 16 x 16 diagonal block is factored in the registers of
// wavefront 0, the panel below it is solved row by row, and the trailing
// lower triangle is updated with MFMA.  The strict upper triangle is set to 0.
// On return (all threads): *fail = first local column whose pivot was not
// positive (or NaN), -1 if none; ld_sum + ld_comp = sum of 2 log(L_jj)
// (Neumaier-compensated), valid in thread 0.
__device__ __forceinline__ void potrf_tile(double* M, int64_t ld, int m, double* smem, int* fail,
                                  double* ld_sum, double* ld_comp) {
    double* sD = smem;                 // 16 x 17
    double* sR = smem + 16 * TO_LDD;   // 16 reciprocals of the pivots
    double* sP = sR + 16;              // (m-16) x 17 panel
    __shared__ int s_fail;
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wv = t >> 6;
    double lsum = 0.0, lcomp = 0.0;
    if (t == 0) s_fail = -1;
    __syncthreads();

    for (int p = 0; p < m; p += 16) {
        {   // 1. load the diagonal block
            const int i = t & 15, j = t >> 4;
            sD[i * TO_LDD + j] = M[(p + i) + (int64_t)(p + j) * ld];
        }
        __syncthreads();
        // 2. factor it in the registers of wavefront 0:
        //    lane = (row i, column group g) holds D[i][4g .. 4g+3]
        if (wv == 0) {
            const int i = lane & 15, g = lane >> 4;
            double d[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) d[q] = sD[i * TO_LDD + 4 * g + q];
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const int cg = c >> 2, cq = c & 3;
                const double piv = __shfl(d[cq], c + 16 * cg);
                const double dd = sqrt(piv);
                const double rinv = 1.0 / dd;
                if (g == cg) {
                    if (i > c) d[cq] *= rinv;
                    else if (i == c) d[cq] = dd;
                }
                const double lic = __shfl(d[cq], i + 16 * cg);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int k = 4 * g + q;
                    const double lkc = __shfl(d[cq], k + 16 * cg);
                    if (k > c && k <= i) d[q] -= lic * lkc;
                }
                if (lane == 0) {
                    if (!(piv > 0.0) && s_fail < 0) s_fail = p + c;
                    neumaier(lsum, lcomp, 2.0 * log(dd));
                    sR[c] = rinv;
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = 4 * g + q;
                sD[i * TO_LDD + k] = (k <= i) ? d[q] : 0.0;
            }
        }
        __syncthreads();
        {   // write the factored block (upper part zero)
            const int i = t & 15, j = t >> 4;
            M[(p + i) + (int64_t)(p + j) * ld] = sD[i * TO_LDD + j];
        }
        const int rows = m - p - 16;
        // 3. panel below: x * D^T = row  (rows independent)
        if (t < rows) {
            const int r = p + 16 + t;
            double x[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) x[c] = M[r + (int64_t)(p + c) * ld];
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                double s = x[c];
#pragma unroll
                for (int k = 0; k < c; ++k) s -= x[k] * sD[c * TO_LDD + k];
                x[c] = s * sR[c];
            }
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                M[r + (int64_t)(p + c) * ld] = x[c];
                sP[t * TO_LDD + c] = x[c];
            }
        }
        __syncthreads();
        // 4. trailing lower triangle -= P P^T, 16 x 16 tiles on MFMA
        const int q = rows / 16;
        const int ntile = q * (q + 1) / 2;
        for (int tt = wv; tt < ntile; tt += 4) {
            int I, J;
            tri_decode(tt, I, J);
            const int r0 = p + 16 + 16 * I, c0 = p + 16 + 16 * J;
            const int li = lane & 15, lk = lane >> 4;
            dbl4 acc;
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[r] = M[(r0 + 4 * r + lk) + (int64_t)(c0 + li) * ld];
#pragma unroll
            for (int kk = 0; kk < 16; kk += 4) {
                const double av = -sP[(16 * I + li) * TO_LDD + kk + lk];
                const double bv = sP[(16 * J + li) * TO_LDD + kk + lk];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) M[(r0 + 4 * r + lk) + (int64_t)(c0 + li) * ld] = acc[r];
        }
        __syncthreads();
    }
    // zero the strict upper triangle outside the diagonal 16 x 16 blocks
    for (int idx = t; idx < m * m; idx += 256) {
        const int i = idx % m, j = idx / m;
        if ((j >> 4) > (i >> 4)) M[i + (int64_t)j * ld] = 0.0;
    }
    __syncthreads();
    *fail = s_fail;
    if (t == 0) { *ld_sum = lsum; *ld_comp = lcomp; }
}

// LDS needed by trtri_tile (per-wavefront 16 x 16 scratch).
#define TRTRI_SMEM_DOUBLES (4 * 16 * TO_LDD)

// X = L^{-1} for the m x m lower-triangular L (column-major, leading dimension
// ldl), m a multiple of 16, m <= 512.  X is written whole (upper part 0).
// Diagonal 16 x 16 blocks are inverted by forward substitution, then the block
// diagonals d = 1, 2, ... follow from X_IJ = -X_II sum_{K=J}^{I-1} L_IK X_KJ,
// every block of one diagonal in parallel.  Returns 1 in *bad (all threads) if
// a diagonal entry of L is not positive or is NaN.
__device__ __forceinline__ void trtri_tile(const double* L, int64_t ldl, double* X, int64_t ldx, int m,
                                  double* smem, int* bad) {
    __shared__ int s_bad;
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wv = t >> 6;
    const int nblk = m / 16;
    if (t == 0) s_bad = 0;
    __syncthreads();
    // zero the blocks above the block diagonal
    for (int idx = t; idx < m * m; idx += 256) {
        const int i = idx % m, j = idx / m;
        if ((j >> 4) > (i >> 4)) X[i + (int64_t)j * ldx] = 0.0;
    }
    // 1. diagonal blocks, one column per lane
    for (int base = 0; base < nblk; base += 4) {
        const int blk = base + wv;
        if (blk < nblk && lane < 16) {
            const int o = 16 * blk;
            const int j = lane;
            double x[16];
            bool badl = false;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                double s = (i == j) ? 1.0 : 0.0;
#pragma unroll
                for (int k = 0; k < i; ++k) s -= L[(o + i) + (int64_t)(o + k) * ldl] * x[k];
                const double lii = L[(o + i) + (int64_t)(o + i) * ldl];
                if (!(lii > 0.0)) badl = true;
                x[i] = (i >= j) ? s / lii : 0.0;
            }
#pragma unroll
            for (int i = 0; i < 16; ++i) X[(o + i) + (int64_t)(o + j) * ldx] = x[i];
            if (badl) s_bad = 1;
        }
    }
    __syncthreads();
    // 2. block diagonals
    double* sT = smem + wv * 16 * TO_LDD;
    const int li = lane & 15, lk = lane >> 4;
    for (int dlt = 1; dlt < nblk; ++dlt) {
        const int ntask = nblk - dlt;
        for (int base = 0; base < ntask; base += 4) {
            const int J = base + wv;
            const bool act = J < ntask;
            const int I = J + dlt;
            dbl4 acc = {0.0, 0.0, 0.0, 0.0};
            if (act) {
                for (int K = J; K < I; ++K) {
#pragma unroll
                    for (int kk = 0; kk < 16; kk += 4) {
                        const double av = L[(16 * I + li) + (int64_t)(16 * K + kk + lk) * ldl];
                        const double bv = X[(16 * K + kk + lk) + (int64_t)(16 * J + li) * ldx];
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
                    }
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) sT[li * TO_LDD + 4 * r + lk] = acc[r];
            }
            __syncthreads();
            if (act) {
                dbl4 out = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kk = 0; kk < 16; kk += 4) {
                    const double av = -X[(16 * I + li) + (int64_t)(16 * I + kk + lk) * ldx];
                    const double bv = sT[li * TO_LDD + kk + lk];
                    out = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, out, 0, 0, 0);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    X[(16 * I + 4 * r + lk) + (int64_t)(16 * J + li) * ldx] = out[r];
            }
            __syncthreads();
        }
    }
    *bad = s_bad;
}

