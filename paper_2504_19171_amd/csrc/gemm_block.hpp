// 64 x 64 output block of an FP64 matrix product on one workgroup of 256
// threads (4 wavefronts of 64 lanes), using the CDNA3/CDNA4 matrix core
// instruction v_mfma_f64_16x16x4_f64.
//
// Each wavefront owns a 32 x 32 quadrant of the block (2 x 2 MFMA tiles of
// 16 x 16, four double4 accumulators per lane).  The reduction dimension is
// streamed in chunks of 16 through LDS: every thread fetches 4 doubles of each
// operand per chunk straight from column-major global memory (coalesced along
// the contiguous dimension, transposed on the write into LDS), the next chunk
// is fetched into registers while the current one feeds the MFMAs.
//
// MFMA lane layout (16x16x4, FP64), lane l in [0, 64):
//   A operand  A[i][k]  with i = l % 16, k = l / 16
//   B operand  B[k][j]  with j = l % 16, k = l / 16
//   D (double4) element r holds D[4*r + l/16][l % 16]  (rows interleaved;
//   measured on gfx950 with one-hot inputs)
#pragma once
#include "common.hpp"

#define GB_M 64
#define GB_KC 16
#define GB_LDA 65   // padded LDS leading dimension (doubles)
#define GB_LDC 65

// One operand of C += A * B.
//   A(i, k) = trans ? p[k + i*ld] : p[i + k*ld]   rows i >= valid read as 0
//   B(k, j) = trans ? p[j + k*ld] : p[k + j*ld]   cols j >= valid read as 0
struct Opnd {
    const double* p;
    int64_t ld;
    int trans;
    int valid;
};

__device__ inline Opnd opnd(const double* p, int64_t ld, int trans, int valid = 64) {
    Opnd o;
    o.p = p; o.ld = ld; o.trans = trans; o.valid = valid;
    return o;
}

// LDS needed by gemm_block: A and B chunks, later reused as the 64x64 output
// staging area.
#define GB_SMEM_DOUBLES (GB_M * GB_LDC)

struct GAcc {
    dbl4 c[2][2];
};

__device__ inline void gacc_zero(GAcc& g) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) g.c[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
}

// Fetch 4 doubles of chunk k0 of operand "A-like" (x = output row index) into r.
// trans == 0: element (x, k) at p[x + k*ld]; trans == 1: at p[k + x*ld].
// The loads are unconditional (a row x >= valid reads row valid-1, inside the
// operand) and gb_stash zeroes those rows: a load guarded by a branch, or
// whose value is selected right away, makes the compiler wait for every load
// in flight there, and the next chunk's loads would no longer overlap the
// products of the current one.
__device__ inline void gb_fetch(const Opnd& o, int k0, double r[4], bool a_side) {
    const int t = threadIdx.x;
    // For the B operand the roles of "normal" and "transposed" swap: B(k, j)
    // normal is p[k + j*ld], i.e. contiguous along k like a transposed A.
    const int contig_x = a_side ? !o.trans : o.trans;
    // offsets stay inside one operand tile (< 2^29 doubles)
    const double* b = uniform_ptr(o.p);
    const int ldi = (int)o.ld;
    const int last = (o.valid > 0 ? o.valid : 1) - 1;
    if (contig_x) {
        const int x = imin_(t & 63, last);
        const uint32_t off = (uint32_t)(x + (k0 + (t >> 6)) * ldi);
#pragma unroll
        for (int q = 0; q < 4; ++q) r[q] = ld_s(b, off + (uint32_t)(4 * q * ldi));
    } else {
        const int k = t & 15;
        const int x0 = t >> 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) r[q] = ld_s(b, (uint32_t)((k0 + k) + imin_(x0 + 16 * q, last) * ldi));
    }
}

// Store the fetched values as s[k][x] (leading dimension GB_LDA), rows x >=
// valid as 0.
__device__ inline void gb_stash(const Opnd& o, double* s, const double r[4], bool a_side) {
    const int t = threadIdx.x;
    const int contig_x = a_side ? !o.trans : o.trans;
    if (contig_x) {
        const int x = t & 63;
        const bool ok = x < o.valid;
#pragma unroll
        for (int q = 0; q < 4; ++q) s[((t >> 6) + 4 * q) * GB_LDA + x] = ok ? r[q] : 0.0;
    } else {
        const int k = t & 15;
#pragma unroll
        for (int q = 0; q < 4; ++q) s[k * GB_LDA + (t >> 4) + 16 * q] = ((t >> 4) + 16 * q < o.valid) ? r[q] : 0.0;
    }
}

__device__ inline void gb_mma_chunk(const double* sA, const double* sB, GAcc& g) {
    const int l = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    const int li = l & 15, lk = l >> 4;
#pragma unroll
    for (int kk = 0; kk < GB_KC; kk += 4) {
        const double* ra = sA + (kk + lk) * GB_LDA + wr + li;
        const double* rb = sB + (kk + lk) * GB_LDA + wc + li;
        double a0 = ra[0], a1 = ra[16];
        double b0 = rb[0], b1 = rb[16];
        g.c[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, g.c[0][0], 0, 0, 0);
        g.c[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, g.c[0][1], 0, 0, 0);
        g.c[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, g.c[1][0], 0, 0, 0);
        g.c[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, g.c[1][1], 0, 0, 0);
    }
}

// g += A(0:64, 0:K) * B(0:K, 0:64); K must be a multiple of 16.
// smem must hold 2 * GB_KC * GB_LDA doubles.  Ends with a barrier so smem can
// be reused right after.
__device__ inline void gemm_acc(GAcc& g, const Opnd& A, const Opnd& B, int K, double* smem) {
    if (K <= 0) return;
    double* sA = smem;
    double* sB = smem + GB_KC * GB_LDA;
    double ra[4], rb[4];
    gb_fetch(A, 0, ra, true);
    gb_fetch(B, 0, rb, false);
    for (int k0 = 0; k0 < K; k0 += GB_KC) {
        __syncthreads();
        gb_stash(A, sA, ra, true);
        gb_stash(B, sB, rb, false);
        __syncthreads();
        if (k0 + GB_KC < K) {
            gb_fetch(A, k0 + GB_KC, ra, true);
            gb_fetch(B, k0 + GB_KC, rb, false);
        }
        gb_mma_chunk(sA, sB, g);
    }
    __syncthreads();
}

// Write the accumulators into LDS as a column-major 64 x 64 block sC[j*GB_LDC + i].
__device__ inline void gacc_to_lds(const GAcc& g, double* sC) {
    const int l = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = wr + ti * 16 + 4 * r + (l >> 4);
                const int j = wc + tj * 16 + (l & 15);
                sC[j * GB_LDC + i] = g.c[ti][tj][r];
            }
}

// Epilogue: out(i, j) = alpha * acc(i, j) + beta * in(i, j) for i < mv, j < nv.
// `in` may equal `out` (each element is read before it is written by the same
// thread).  Both column-major with leading dimensions ldi / ldo.
__device__ inline void gemm_store(const GAcc& g, double* smem, double alpha, double beta,
                                  const double* in, int64_t ldi, double* out, int64_t ldo,
                                  int mv, int nv) {
    gacc_to_lds(g, smem);
    __syncthreads();
    const int t = threadIdx.x;
    const int i = t & 63;
    if (i < mv) {
        for (int j = t >> 6; j < nv; j += 4) {
            double v = alpha * smem[j * GB_LDC + i];
            if (beta != 0.0) v += beta * in[i + (int64_t)j * ldi];
            out[i + (int64_t)j * ldo] = v;
        }
    }
    __syncthreads();
}

// Symmetric epilogue for a block on or below the diagonal of a symmetric
// matrix stored full: value(i, j) = alpha*acc(i, j) + beta*in(i, j), for
// i < mv, j < nv.
//   diag == 1: a diagonal block (mv == nv); the lower triangle of value is
//              written to both triangles of out_lo (mirrored).
//   diag == 0: value is written to out_lo(i, j) and to out_up(j, i).
// All of `in` is read before any write.
__device__ inline void gemm_store_sym(const GAcc& g, double* smem, double alpha, double beta,
                                      const double* in, int64_t ldi, double* out_lo,
                                      double* out_up, int64_t ldo, int diag, int mv, int nv) {
    gacc_to_lds(g, smem);
    __syncthreads();
    const int t = threadIdx.x;
    {
        const int i = t & 63;
        if (i < mv) {
            for (int j = t >> 6; j < nv; j += 4) {
                if (diag && i < j) continue;
                double v = alpha * smem[j * GB_LDC + i];
                if (beta != 0.0) v += beta * in[i + (int64_t)j * ldi];
                smem[j * GB_LDC + i] = v;
            }
        }
    }
    __syncthreads();
    {
        const int i = t & 63;
        if (i < mv) {
            for (int j = t >> 6; j < nv; j += 4) {
                double v = (diag && i < j) ? smem[i * GB_LDC + j] : smem[j * GB_LDC + i];
                out_lo[i + (int64_t)j * ldo] = v;
            }
        }
        if (!diag) {
            // out_up(j, i) = value(i, j): thread handles row j = t & 63 of out_up.
            const int jj = t & 63;
            if (jj < nv) {
                for (int ii = t >> 6; ii < mv; ii += 4)
                    out_up[jj + (int64_t)ii * ldo] = smem[jj * GB_LDC + ii];
            }
        }
    }
    __syncthreads();
}
