// Cholesky of one diagonal tile (m <= 256, m a multiple of 64) by one
// workgroup of 4 wavefronts, left-looking over 16-column panels with a
// one-panel lookahead:
//   - every wavefront owns the 16 x 16 row tiles I = w, w+4, ... of the
//     current panel and keeps them in registers in transposed MFMA form
//     (lane (i, k) holds C[16I + i][c0 + 4r + k], the layout the matrix cores
//     take as the B operand, so the panel solve needs no shuffle);
//   - the diagonal 16 x 16 block is factored by wavefront 0 (two 8 x 8
//     Cholesky factorizations and inverses kept in registers, redundantly in
//     every lane, joined by an 8 x 8 TRSM and SYRK), while the other
//     wavefronts already reduce the next panel over every older panel;
//   - the panel below is solved with the inverse of the diagonal block on the
//     matrix cores, L_Ip^T = Y_pp C_Ip^T, and the last product of the next
//     panel (this panel's contribution) follows from LDS.
// Also returns the inverses of the 64 x 64 diagonal blocks of L (for the
// panel TRSM below the tile) and the Neumaier pair of sum 2 log L_jj.
#pragma once
#include "common.hpp"
#include "tile_ops.hpp"

#define P3_LD 17
#define P3_SLOTS 6   // row tiles per wavefront: ceil(16 / 3)

struct P3Smem {
    double D[16 * P3_LD];          // diagonal block of the current panel, D(i, j) at D[j * P3_LD + i]
    double Y[16 * P3_LD];          // Y = L_pp^{-1}, Y(i, j) at Y[i * P3_LD + j]
    double L21[8 * 9];             // factor16 scratch: L21(i, j) at L21[i * 9 + j]
    double S22[8 * 9];             // factor16 scratch: S(i, j) at S22[i * 9 + j]
    double Y21[8 * 9];             // Y21(i, j) at Y21[i * 9 + j]
    double T[8 * 9];               // T = L21 Y11, T(i, j) at T[i * 9 + j]
    double Pk[4][36];              // packed L11, Y11, L22, Y22 (P8 order)
    double Pn[16][256];            // L tiles of the last solved panel: L[16I + i][c0 + j] at Pn[I][j * 16 + i]
    double lsum, lcomp;
    int fail;
};

// Packed lower triangle of an 8 x 8 matrix, by columns.
#define P8(i, j) ((j) * 8 - ((j) * ((j) - 1)) / 2 + ((i) - (j)))

// sqrt(x) and 1/sqrt(x) from the hardware reciprocal square root and two
// Goldschmidt steps (a few ulp; the pivot decides nothing else).
__device__ inline void p3_sqrt_rsqrt(double x, double& s, double& r) {
    const double r0 = __builtin_amdgcn_rsq(x);
    double g = x * r0, h = 0.5 * r0;
    double e = fma(-g, h, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    e = fma(-g, h, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    s = g;
    r = 2.0 * h;
}

// In-register Cholesky of the packed 8 x 8 lower triangle a; rinv[j] = 1/L_jj.
// *fail gets the first local column (base + j) whose pivot is not positive.
__device__ inline void p3_chol8(double (&a)[36], double (&rinv)[8], int base, int& fail, double& ls, double& lc) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const double piv = a[P8(j, j)];
        if (!(piv > 0.0) && fail < 0) fail = base + j;
        double s, r;
        p3_sqrt_rsqrt(piv, s, r);
        a[P8(j, j)] = s;
        rinv[j] = r;
        neumaier(ls, lc, 2.0 * log(s));
#pragma unroll
        for (int i = j + 1; i < 8; ++i) a[P8(i, j)] *= r;
#pragma unroll
        for (int k = j + 1; k < 8; ++k)
#pragma unroll
            for (int i = k; i < 8; ++i) a[P8(i, k)] = fma(-a[P8(i, j)], a[P8(k, j)], a[P8(i, k)]);
    }
}

// In place: the packed 8 x 8 lower-triangular L becomes L^{-1} (rinv = 1/L_jj).
// Column j is done top down; y_ij needs L_ik (k >= j, columns not yet
// replaced, and L_ij itself still in place) and y_kj (k < i, already there).
__device__ inline void p3_inv8(double (&a)[36], const double (&rinv)[8]) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
#pragma unroll
        for (int i = j + 1; i < 8; ++i) {
            double s = a[P8(i, j)] * rinv[j];
#pragma unroll
            for (int k = j + 1; k < i; ++k) s = fma(a[P8(i, k)], a[P8(k, j)], s);
            a[P8(i, j)] = -s * rinv[i];
        }
        a[P8(j, j)] = rinv[j];
    }
}

// Factor the 16 x 16 block in sm.D (lower part) on one wavefront: L_pp back
// into sm.D (lower, [col][row]) and Y = L_pp^{-1} into sm.Y ([row][col]),
// both with zero strict upper parts.  With D = [D11 .; D21 D22] (8 x 8
// blocks): L11 = chol(D11), L21 = D21 L11^{-T} (row by row), S = D22 -
// L21 L21^T, L22 = chol(S), and Y = [Y11 0; -Y22 L21 Y11  Y22].
__device__ inline void p3_wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline void p3_factor16(P3Smem& sm, int base, int& fail, double& ls, double& lc) {
    const int lane = threadIdx.x & 63;
    double a[36], r[8], l21[8];
    // 1. L11 = chol(D11), in every lane; lane i < 8 forms row i of L21
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int i = j; i < 8; ++i) a[P8(i, j)] = sm.D[j * P3_LD + i];
    p3_chol8(a, r, base, fail, ls, lc);
    if (lane == 0) {
#pragma unroll
        for (int e = 0; e < 36; ++e) sm.Pk[0][e] = a[e];
    }
    if (lane < 8) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            double v = sm.D[j * P3_LD + 8 + lane];
#pragma unroll
            for (int k = 0; k < j; ++k) v = fma(-l21[k], a[P8(j, k)], v);
            l21[j] = v * r[j];
            sm.L21[lane * 9 + j] = l21[j];
        }
    }
    // 2. Y11 = L11^{-1}; T = L21 Y11 (row i on lane i < 8)
    p3_inv8(a, r);
    if (lane == 0) {
#pragma unroll
        for (int e = 0; e < 36; ++e) sm.Pk[1][e] = a[e];
    }
    if (lane < 8) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            double v = 0.0;
#pragma unroll
            for (int k = j; k < 8; ++k) v = fma(l21[k], a[P8(k, j)], v);
            sm.T[lane * 9 + j] = v;
        }
    }
    p3_wsync();
    // 3. S = D22 - L21 L21^T, lane (i, j), j <= i
    {
        const int i = lane >> 3, jj = lane & 7;
        if (jj <= i) {
            double v = sm.D[(8 + jj) * P3_LD + 8 + i];
#pragma unroll
            for (int k = 0; k < 8; ++k) v = fma(-sm.L21[i * 9 + k], sm.L21[jj * 9 + k], v);
            sm.S22[i * 9 + jj] = v;
        }
    }
    p3_wsync();
    // 4. L22 = chol(S), Y22 = L22^{-1}, in every lane
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int i = j; i < 8; ++i) a[P8(i, j)] = sm.S22[i * 9 + j];
    p3_chol8(a, r, base + 8, fail, ls, lc);
    if (lane == 0) {
#pragma unroll
        for (int e = 0; e < 36; ++e) sm.Pk[2][e] = a[e];
    }
    p3_inv8(a, r);
    if (lane == 0) {
#pragma unroll
        for (int e = 0; e < 36; ++e) sm.Pk[3][e] = a[e];
    }
    // 5. Y21 = -Y22 T, column j on lane j < 8
    if (lane < 8) {
        double t[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) t[k] = sm.T[k * 9 + lane];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            double v = 0.0;
#pragma unroll
            for (int k = 0; k <= i; ++k) v = fma(a[P8(i, k)], t[k], v);
            sm.Y21[i * 9 + lane] = -v;
        }
    }
    p3_wsync();
    // 6. assemble L_pp ([col][row]) and Y ([row][col]) with zero upper parts
    for (int e = lane; e < 256; e += 64) {
        const int i = e & 15, j = e >> 4;
        double lv = 0.0, yv = 0.0;
        if (j <= i) {
            if (i < 8) {
                const int q = j * 8 - (j * (j - 1)) / 2 + (i - j);
                lv = sm.Pk[0][q];
                yv = sm.Pk[1][q];
            } else if (j >= 8) {
                const int i2 = i - 8, j2 = j - 8;
                const int q = j2 * 8 - (j2 * (j2 - 1)) / 2 + (i2 - j2);
                lv = sm.Pk[2][q];
                yv = sm.Pk[3][q];
            } else {
                lv = sm.L21[(i - 8) * 9 + j];
                yv = sm.Y21[(i - 8) * 9 + j];
            }
        }
        sm.D[j * P3_LD + i] = lv;
        sm.Y[i * P3_LD + j] = yv;
    }
}

// In-place Cholesky of the m x m lower triangle of M (column-major, leading
// dimension ld), m a multiple of 64, m <= 256; the strict upper triangle is
// set to 0.  X64 + q*4096: inverse of the q-th 64 x 64 diagonal block of L
// (column-major, entries above its 16 x 16 block diagonal not written).
// Thread 0 returns the first failing local column (or -1) and the log det
// pair.
__device__ inline void potrf3(double* M, int64_t ld, int m, double* X64, P3Smem& sm, int* fail_out, double* ls_out,
                              double* lc_out) {
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const int np = m / 16;
    const double* Mc = uniform_ptr(M);
    const int ldi = (int)ld;
    int fail = -1;
    double ls = 0.0, lc = 0.0;
    // waves 1..3 own the row tiles I = 3s + w - 1; wave 0 factors the diagonal blocks
    dbl4 cur[P3_SLOTS], nxt[P3_SLOTS];
    // panel 0, transposed: element r = C[16I + li][4r + lk]
#pragma unroll
    for (int s = 0; s < P3_SLOTS; ++s) {
        const int I = (w == 0) ? np : 3 * s + w - 1;
        cur[s] = dbl4{0.0, 0.0, 0.0, 0.0};
        if (I < np) {
#pragma unroll
            for (int r = 0; r < 4; ++r) cur[s][r] = Mc[(16 * I + li) + (4 * r + lk) * ldi];
        }
    }
    for (int p = 0; p < np; ++p) {
        const int c0 = 16 * p;
        // the owner of the diagonal block hands it over
        if (w != 0 && (p % 3) == w - 1) {
#pragma unroll
            for (int s = 0; s < P3_SLOTS; ++s)
                if (3 * s + w - 1 == p)
#pragma unroll
                    for (int r = 0; r < 4; ++r) sm.D[(4 * r + lk) * P3_LD + li] = cur[s][r];
        }
        __syncthreads();
        if (w == 0) p3_factor16(sm, c0, fail, ls, lc);
        // next panel, every older panel but this one (global L is final there)
        if (p + 1 < np) {
            const int c1 = c0 + 16;
#pragma unroll
            for (int s = 0; s < P3_SLOTS; ++s) {
                const int I = (w == 0) ? np : 3 * s + w - 1;
                nxt[s] = dbl4{0.0, 0.0, 0.0, 0.0};
                if (I >= p + 1 && I < np) {
                    dbl4 e0, e1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int r = 0; r < 4; ++r) e0[r] = Mc[(16 * I + li) + (c1 + 4 * r + lk) * ldi];
                    for (int k = 0; k < c0; k += 8) {
                        const double a0 = -Mc[(c1 + li) + (k + lk) * ldi];
                        const double b0 = Mc[(16 * I + li) + (k + lk) * ldi];
                        const double a1 = -Mc[(c1 + li) + (k + 4 + lk) * ldi];
                        const double b1 = Mc[(16 * I + li) + (k + 4 + lk) * ldi];
                        e0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, e0, 0, 0, 0);
                        e1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, e1, 0, 0, 0);
                    }
                    nxt[s] = e0 + e1;
                }
            }
        }
        __syncthreads();   // L_pp, Y ready
        // L_pp to global (lower with zero upper), the upper blocks above it to 0
        for (int e = threadIdx.x; e < 256; e += 256) {
            const int i = e & 15, j = e >> 4;
            M[(c0 + i) + (int64_t)(c0 + j) * ld] = sm.D[j * P3_LD + i];
        }
        for (int e = threadIdx.x; e < c0 * 16; e += 256) {
            const int i = e % c0, j = e / c0;
            M[i + (int64_t)(c0 + j) * ld] = 0.0;
        }
        // panel solve: L_Ip^T = Y C_Ip^T, B operand straight from the registers
#pragma unroll
        for (int s = 0; s < P3_SLOTS; ++s) {
            const int I = (w == 0) ? np : 3 * s + w - 1;
            if (I > p && I < np) {
                dbl4 o = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const double av = sm.Y[li * P3_LD + 4 * r + lk];
                    o = __builtin_amdgcn_mfma_f64_16x16x4f64(av, cur[s][r], o, 0, 0, 0);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    M[(16 * I + li) + (int64_t)(c0 + 4 * r + lk) * ld] = o[r];
                    sm.Pn[I][(4 * r + lk) * 16 + li] = o[r];
                }
            }
        }
        __syncthreads();   // Pn complete
        if (p + 1 < np) {
            // this panel's product into the next panel
#pragma unroll
            for (int s = 0; s < P3_SLOTS; ++s) {
                const int I = (w == 0) ? np : 3 * s + w - 1;
                if (I >= p + 1 && I < np) {
#pragma unroll
                    for (int kk = 0; kk < 16; kk += 4) {
                        const double av = -sm.Pn[p + 1][(kk + lk) * 16 + li];
                        const double bv = sm.Pn[I][(kk + lk) * 16 + li];
                        nxt[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, nxt[s], 0, 0, 0);
                    }
                }
                cur[s] = nxt[s];
            }
        }
        // the diagonal 16 x 16 inverse goes to its 64-block of X64
        if (threadIdx.x < 256) {
            const int i = threadIdx.x & 15, j = threadIdx.x >> 4;
            double* Xg = X64 + (int64_t)(p >> 2) * 4096;
            const int xo = 16 * (p & 3);
            Xg[(xo + i) + (xo + j) * 64] = sm.Y[i * P3_LD + j];
        }
        // (the next iteration's first barrier orders the LDS reuse)
    }
    __syncthreads();
    inv64_rounds(M, ld, X64, m, &sm.Pn[0][0]);
    if (threadIdx.x == 0) {
        *fail_out = fail;
        *ls_out = ls;
        *lc_out = lc;
    }
}
