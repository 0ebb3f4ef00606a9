// Cholesky of one diagonal tile (m <= 256, m a multiple of 64) by one
// workgroup of 4 wavefronts, left-looking over 16-column panels with a
// one-panel lookahead:
//   - wavefronts 1..3 own the 16 x 16 row tiles I = w, w+3, ... of every
//     panel; the reduced current panel sits in LDS in transposed MFMA form
//     (lane (i, k) reads C[16I + i][c0 + 4r + k], the layout the matrix cores
//     take as the B operand, so the panel solve needs no shuffle);
//   - the diagonal 16 x 16 block is factored by wavefront 0 (two 8 x 8
//     Cholesky factorizations and inverses kept in registers, redundantly in
//     every lane, joined by an 8 x 8 TRSM and SYRK), while the other
//     wavefronts reduce the panels ahead of it (see potrf3 below);
//   - the panel below is solved with the inverse of the diagonal block on the
//     matrix cores, L_Ip^T = Y_pp C_Ip^T.
// Also returns the inverses of the 64 x 64 diagonal blocks of L (for the
// panel TRSM below the tile) and the Neumaier pair of sum 2 log L_jj.
#pragma once
#include "common.hpp"
#include "tile_ops.hpp"

#define P3_LD 17
#define P3_SLOTS 5   // row tiles I >= 1 per wavefront: 15 / 3

struct P3Smem {
    double D[16 * P3_LD];          // diagonal block of the current panel, D(i, j) at D[j * P3_LD + i]
    double Y[16 * P3_LD];          // Y = L_pp^{-1}, Y(i, j) at Y[i * P3_LD + j]
    double S22[8 * 9];             // factor16 scratch: S(i, j) at S22[i * 9 + j]
    double T[8 * 9];               // T = L21 Y11, T(i, j) at T[i * 9 + j]
    double Dn[2][16 * P3_LD];      // next diagonal blocks (by parity), reduced up to two panels back
    double Pn[2][16][256];         // L tiles of solved panels by parity: L[16I + i][c0 + j] at Pn[par][I][j * 16 + i]
    double Cp[16][256];            // reduced current panel, transposed MFMA form (r * 64 + lane)
                                   // (Pn and Cp, 48 tiles, are the epilogue's staging area)
    double dg[256];                // diagonal of L, then 2 log L_jj
    double ps[64], pc[64];         // log det partial sums
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
// (The logarithms of the pivots are taken after the sweep, off this chain.)
// *fail gets the first local column (base + j) whose pivot is not positive.
__device__ inline void p3_chol8(double (&a)[36], double (&rinv)[8], int base, int& fail) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const double piv = a[P8(j, j)];
        if (!(piv > 0.0) && fail < 0) fail = base + j;
        double s, r;
        p3_sqrt_rsqrt(piv, s, r);
        a[P8(j, j)] = s;
        rinv[j] = r;
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

// Workgroup barriers that wait only for what the next phase reads: LDS
// (lgkm) always, global stores (vm) only where another wavefront reads them
// back from global memory.  The "memory" clobber keeps the compiler from
// moving accesses across them.
__device__ inline void p3_bar_lds() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }
__device__ inline void p3_bar_all() { asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

__device__ inline void p3_wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Store a packed 8 x 8 lower triangle (identical in every lane) into LDS
// from lane 0, at compile-time addresses.  ToY: into sm.Y ([row][col]) at
// block offset o; otherwise into sm.D ([col][row]), the diagonal also into
// sm.dg.
template <bool ToY>
__device__ inline void p3_put8(P3Smem& sm, const double (&l)[36], int o, int base) {
    if ((threadIdx.x & 63) != 0) return;
#pragma unroll
    for (int jj = 0; jj < 8; ++jj)
#pragma unroll
        for (int ii = jj; ii < 8; ++ii) {
            const int e = P8(ii, jj);
            if (ToY) {
                sm.Y[(o + ii) * P3_LD + o + jj] = l[e];
            } else {
                sm.D[(o + jj) * P3_LD + o + ii] = l[e];
                if (ii == jj) sm.dg[base + o + ii] = l[e];
            }
        }
}

// Factor the 16 x 16 block in sm.D (lower part) on one wavefront: L_pp back
// into the lower part of sm.D ([col][row]; the upper part is left as is) and
// Y = L_pp^{-1} into the lower part of sm.Y ([row][col]; its upper part is
// zero from the start).  With D = [D11 .; D21 D22] (8 x 8 blocks):
// L11 = chol(D11), L21 = D21 L11^{-T} (row by row), S = D22 - L21 L21^T,
// L22 = chol(S), and Y = [Y11 0; -Y22 L21 Y11  Y22].
__device__ inline void p3_factor16(P3Smem& sm, int base, int& fail) {
    const int lane = threadIdx.x & 63;
    double a[36], r[8], l21[8];
    // 1. L11 = chol(D11), in every lane; lane i < 8 forms row i of L21 (in place in sm.D)
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int i = j; i < 8; ++i) a[P8(i, j)] = sm.D[j * P3_LD + i];
    p3_chol8(a, r, base, fail);
    if (lane < 8) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            double v = sm.D[j * P3_LD + 8 + lane];
#pragma unroll
            for (int k = 0; k < j; ++k) v = fma(-l21[k], a[P8(j, k)], v);
            l21[j] = v * r[j];
            sm.D[j * P3_LD + 8 + lane] = l21[j];
        }
    }
    // 2. Y11 = L11^{-1} (in place); T = L21 Y11 (row i on lane i < 8)
    p3_put8<false>(sm, a, 0, base);
    p3_inv8(a, r);
    p3_put8<true>(sm, a, 0, base);
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
            for (int k = 0; k < 8; ++k) v = fma(-sm.D[k * P3_LD + 8 + i], sm.D[k * P3_LD + 8 + jj], v);
            sm.S22[i * 9 + jj] = v;
        }
    }
    p3_wsync();
    // 4. L22 = chol(S), Y22 = L22^{-1}, in every lane
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int i = j; i < 8; ++i) a[P8(i, j)] = sm.S22[i * 9 + j];
    p3_chol8(a, r, base + 8, fail);
    p3_put8<false>(sm, a, 8, base);
    p3_inv8(a, r);
    p3_put8<true>(sm, a, 8, base);
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
            sm.Y[(8 + i) * P3_LD + lane] = -v;
        }
    }
}

// C = A B for 16 x 16 tiles in LDS (column-major, A(i, k) at A[k*16 + i]) on
// one wavefront, added to acc (MFMA D layout: element r = C(4r + lane/16, lane%16)).
__device__ inline void p3_mm16(dbl4& acc, const double* A, const double* B) {
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[(kk + lk) * 16 + li], B[li * 16 + kk + lk], acc, 0, 0, 0);
}
__device__ inline void p3_put16(double* C, const dbl4& acc, double scale) {
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r) C[li * 16 + 4 * r + lk] = scale * acc[r];
}

// Epilogue: wavefront g forms the inverse X of the g-th 64 x 64 diagonal block
// of L from the inverses Y_q of its 16 x 16 diagonal blocks (already in X64)
// and its 16 x 16 blocks L_IJ, staged in LDS (st: 11 tiles per wavefront):
// X_IJ = -Y_I sum_{K=J}^{I-1} L_IK X_KJ, block diagonal by block diagonal.
__device__ inline void p3_inv64(const double* Mc, int ldi, double* X64, int m, double* stage) {
    const int g = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (64 * g >= m) return;
    const int lane = threadIdx.x & 63;
    double* T = stage + g * 11 * 256;   // tiles: Y0..Y3, L10, L20, L21, L30, L31, L32, tmp
    double* Xg = (double*)uniform_ptr(X64 + (int64_t)g * 4096);
    const int Ls[6][2] = {{1, 0}, {2, 0}, {2, 1}, {3, 0}, {3, 1}, {3, 2}};
    double v[40];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = lane + 64 * q, i = e & 15, j = e >> 4;
            v[4 * t + q] = ld_s(Xg, (uint32_t)((16 * t + i) + (16 * t + j) * 64));
        }
#pragma unroll
    for (int t = 0; t < 6; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = lane + 64 * q, i = e & 15, j = e >> 4;
            v[16 + 4 * t + q] = ld_s(Mc, (uint32_t)((64 * g + 16 * Ls[t][0] + i) + (64 * g + 16 * Ls[t][1] + j) * ldi));
        }
#pragma unroll
    for (int t = 0; t < 10; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) T[t * 256 + lane + 64 * q] = v[4 * t + q];
    p3_wsync();
    double* Y[4] = {T, T + 256, T + 512, T + 768};
    double* L10 = T + 4 * 256; double* L20 = T + 5 * 256; double* L21 = T + 6 * 256;
    double* L30 = T + 7 * 256; double* L31 = T + 8 * 256; double* L32 = T + 9 * 256;
    double* tmp = T + 10 * 256;
    // one block X_IJ = -Y_I (sum of the products given), written over slot `dst`
    auto block = [&](int I, int J, double* dst, const double* a0, const double* b0, const double* a1, const double* b1,
                     const double* a2, const double* b2) {
        dbl4 acc = {0.0, 0.0, 0.0, 0.0};
        p3_mm16(acc, a0, b0);
        if (a1) p3_mm16(acc, a1, b1);
        if (a2) p3_mm16(acc, a2, b2);
        p3_put16(tmp, acc, 1.0);
        p3_wsync();
        dbl4 x = {0.0, 0.0, 0.0, 0.0};
        p3_mm16(x, Y[I], tmp);
        p3_wsync();   // tmp read before the next block writes it
        p3_put16(dst, x, -1.0);
        const int li = lane & 15, lk = lane >> 4;
#pragma unroll
        for (int r = 0; r < 4; ++r) st_s(Xg, (uint32_t)((16 * I + 4 * r + lk) + (16 * J + li) * 64), -x[r]);
        p3_wsync();
    };
    // slots are reused once their L block is no longer needed
    block(1, 0, L10, L10, Y[0], nullptr, nullptr, nullptr, nullptr);        // X10
    block(2, 0, L20, L20, Y[0], L21, L10, nullptr, nullptr);                // X20 (L10 holds X10)
    block(2, 1, L21, L21, Y[1], nullptr, nullptr, nullptr, nullptr);        // X21
    block(3, 0, L30, L30, Y[0], L31, L10, L32, L20);                        // X30 (L20 holds X20)
    block(3, 1, L31, L31, Y[1], L32, L21, nullptr, nullptr);                // X31 (L21 holds X21)
    block(3, 2, L32, L32, Y[2], nullptr, nullptr, nullptr, nullptr);        // X32
}

// Tiles I = 3s + w (slots s >= S0) of panel p+2 (columns c0 + 32 ..) reduced
// over the panels < p, read from global memory in 16-column chunks: the
// raw tile values go into nxt, the products are accumulated apart and
// subtracted at the end.  The next chunk is in flight while the current one
// is multiplied; all loads are unconditional (a chunk past the end re-reads
// the last one and is not used) so the waits stay exact.
template <int S0>
__device__ __forceinline__ void p3_reduce_panel(dbl4 (&nxt)[P3_SLOTS], const double* Mc, int ldi, int w, int np,
                                                int c0, int li, int lk) {
    constexpr int NS = P3_SLOTS - S0;
    const int c2 = c0 + 32;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const int I = imin_(3 * (S0 + q) + w, np - 1);
#pragma unroll
        for (int r = 0; r < 4; ++r) nxt[S0 + q][r] = ld_s(Mc, (uint32_t)((16 * I + li) + (c2 + 4 * r + lk) * ldi));
    }
    if (c0 == 0) return;
    dbl4 red[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) red[q] = dbl4{0.0, 0.0, 0.0, 0.0};
    auto fetch = [&](double (&ra)[4], double (&rb)[NS][4], int k0) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) ra[kk] = ld_s(Mc, (uint32_t)((c2 + li) + (k0 + 4 * kk + lk) * ldi));
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const int I = imin_(3 * (S0 + q) + w, np - 1);
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) rb[q][kk] = ld_s(Mc, (uint32_t)((16 * I + li) + (k0 + 4 * kk + lk) * ldi));
        }
    };
    auto mma = [&](const double (&ra)[4], const double (&rb)[NS][4]) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
            for (int q = 0; q < NS; ++q) red[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(ra[kk], rb[q][kk], red[q], 0, 0, 0);
    };
    double ra0[4], ra1[4], rb0[NS][4], rb1[NS][4];
    if (NS <= 3) {
        // two chunks in flight: chunk 3t in buffer 0, 3t+1 in 1, 3t+2 in 2
        double ra2[4], rb2[NS][4];
        fetch(ra0, rb0, 0);
        fetch(ra1, rb1, imin_(16, c0 - 16));
        for (int k0 = 0; k0 < c0; k0 += 48) {
            fetch(ra2, rb2, imin_(k0 + 32, c0 - 16));
            mma(ra0, rb0);
            fetch(ra0, rb0, imin_(k0 + 48, c0 - 16));
            if (k0 + 16 < c0) mma(ra1, rb1);
            fetch(ra1, rb1, imin_(k0 + 64, c0 - 16));
            if (k0 + 32 < c0) mma(ra2, rb2);
        }
    } else {
        // one chunk in flight
        fetch(ra0, rb0, 0);
        for (int k0 = 0; k0 < c0; k0 += 32) {
            fetch(ra1, rb1, imin_(k0 + 16, c0 - 16));
            mma(ra0, rb0);
            fetch(ra0, rb0, imin_(k0 + 32, c0 - 16));
            if (k0 + 16 < c0) mma(ra1, rb1);
        }
    }
#pragma unroll
    for (int q = 0; q < NS; ++q) nxt[S0 + q] -= red[q];
}

// In-place Cholesky of the m x m lower triangle of M (column-major, leading
// dimension ld), m a multiple of 64, m <= 256; the strict upper triangle is
// set to 0.  X64 + q*4096: inverse of the q-th 64 x 64 diagonal block of L
// (column-major, entries above its 16 x 16 block diagonal not written).
// Thread 0 returns the first failing local column (or -1) and the log det
// pair.
//
// Software pipeline over the 16-column panels p, two phases per panel:
//   S(p): L_pp and Y_pp go out; wavefronts 1..3 solve their tiles of panel p
//         (L_Ip = C_Ip Y^T) into LDS (Pn, by parity of p) and global memory;
//   U(p): wavefront 0 forms the next diagonal block D_{p+1} = Dn - L_{p+1,p}
//         L_{p+1,p}^T and factors it (factor16), while wavefronts 1..3 add
//         panel p into the tiles of panel p+1 (-> Cp, read by S(p+1)) and
//         reduce the tiles of panel p+2 over panels 0..p (older panels from
//         global memory, panel p from LDS); the owner of tile p+2 hands its
//         diagonal block to wavefront 0 through Dn (by parity).
// So the chain of diagonal factorizations overlaps all the other work.
__device__ inline void potrf3(double* M, int64_t ld, int m, double* X64, P3Smem& sm, int* fail_out, double* ls_out,
                              double* lc_out) {
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const int np = m / 16;
    const double* Mc = uniform_ptr(M);   // with unsigned 32-bit offsets: scalar base + vector offset loads
    double* Mw = (double*)Mc;
    const int ldi = (int)ld;
    int fail = -1;
    // panel 0 into LDS, transposed MFMA form: Cp[I][r*64 + lane] = C[16I + li][4r + lk];
    // D_0 = tile (0, 0); Y's upper part stays 0 from here on
    {
        double v[16];
        const int q = threadIdx.x, r = q >> 6, ln = q & 63;
#pragma unroll
        for (int I = 0; I < 16; ++I)
            v[I] = ld_s(Mc, (uint32_t)((16 * imin_(I, np - 1) + (ln & 15)) + (4 * r + (ln >> 4)) * ldi));
#pragma unroll
        for (int I = 0; I < 16; ++I)
            if (I < np) sm.Cp[I][q] = v[I];
    }
    {
        const int i = threadIdx.x & 15, j = threadIdx.x >> 4;
        sm.D[j * P3_LD + i] = ld_s(Mc, (uint32_t)(i + j * ldi));
    }
    for (int e = threadIdx.x; e < 16 * P3_LD; e += 256) sm.Y[e] = 0.0;
    // wavefronts 1..3 own the row tiles I = 3s + w >= 1 of every panel
    dbl4 nxt[P3_SLOTS];
    // raw tiles of panel 1 (nothing to reduce yet); tile 1 is owned by
    // wavefront 1, slot 0, and goes to Dn
    if (w != 0) {
#pragma unroll
        for (int s = 0; s < P3_SLOTS; ++s) {
            const int I = imin_(3 * s + w, np - 1);
#pragma unroll
            for (int r = 0; r < 4; ++r) nxt[s][r] = ld_s(Mc, (uint32_t)((16 * I + li) + (16 + 4 * r + lk) * ldi));
        }
        if (w == 1) {
#pragma unroll
            for (int r = 0; r < 4; ++r) sm.Dn[1][(4 * r + lk) * P3_LD + li] = nxt[0][r];
        }
    }
    __syncthreads();
    if (w == 0) p3_factor16(sm, 0, fail);
    p3_bar_lds();
    for (int p = 0; p < np; ++p) {
        const int c0 = 16 * p;
        const int par = p & 1;
        // ---- S(p)
        if (w == 0) {
            double* Xg = (double*)uniform_ptr(X64 + (int64_t)(p >> 2) * 4096);
            const int xo = 16 * (p & 3);
            for (int e = lane; e < 256; e += 64) {
                const int i = e & 15, j = e >> 4;
                st_s(Mw, (uint32_t)((c0 + i) + (c0 + j) * ldi), (j <= i) ? sm.D[j * P3_LD + i] : 0.0);
                st_s(Xg, (uint32_t)((xo + i) + (xo + j) * 64), sm.Y[i * P3_LD + j]);
            }
        } else {
#pragma unroll
            for (int s = 0; s < P3_SLOTS; ++s) {
                const int I = 3 * s + w;
                if (I > p && I < np) {
                    dbl4 o = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const double av = sm.Y[li * P3_LD + 4 * r + lk];
                        o = __builtin_amdgcn_mfma_f64_16x16x4f64(av, sm.Cp[I][r * 64 + lane], o, 0, 0, 0);
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        st_s(Mw, (uint32_t)((16 * I + li) + (c0 + 4 * r + lk) * ldi), o[r]);
                        sm.Pn[par][I][(4 * r + lk) * 16 + li] = o[r];
                    }
                }
            }
        }
        for (int j = 0; j < 16; ++j)
            for (int i = threadIdx.x; i < c0; i += 256) st_s(Mw, (uint32_t)(i + (c0 + j) * ldi), 0.0);
        p3_bar_lds();   // Pn[par] complete (the global stores stay in flight)
        if (p + 1 == np) break;
        // ---- U(p)
        if (w == 0) {
            // D_{p+1} = Dn - L_{p+1,p} L_{p+1,p}^T, then its factorization
            dbl4 acc;
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[r] = sm.Dn[(p + 1) & 1][(4 * r + lk) * P3_LD + li];
#pragma unroll
            for (int kk = 0; kk < 16; kk += 4) {
                const double v = sm.Pn[par][p + 1][(kk + lk) * 16 + li];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-v, v, acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) sm.D[(4 * r + lk) * P3_LD + li] = acc[r];
            p3_wsync();
            p3_factor16(sm, c0 + 16, fail);
        } else {
            // panel p into the tiles I >= p+2 of panel p+1 -> Cp
#pragma unroll
            for (int s = 0; s < P3_SLOTS; ++s) {
                const int I = 3 * s + w;
                if (I >= p + 2 && I < np) {
#pragma unroll
                    for (int kk = 0; kk < 16; kk += 4) {
                        const double av = -sm.Pn[par][p + 1][(kk + lk) * 16 + li];
                        const double bv = sm.Pn[par][I][(kk + lk) * 16 + li];
                        nxt[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, nxt[s], 0, 0, 0);
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) sm.Cp[I][r * 64 + lane] = nxt[s][r];
                }
            }
            // tiles I >= p+2 of panel p+2 over panels 0..p: panels < p from
            // global memory in 16-column chunks (the next one in flight while
            // the current one is multiplied; the rows of tile p+2 are the A
            // operand of every slot), then panel p from LDS
            if (p + 2 < np) {
                // slots s >= s0 hold tiles I >= p+2; only they load and multiply
                const int s0 = imin_(P3_SLOTS - 1, imax_(0, (p + 2 - w + 2) / 3));
                switch (s0) {
                    case 0: p3_reduce_panel<0>(nxt, Mc, ldi, w, np, c0, li, lk); break;
                    case 1: p3_reduce_panel<1>(nxt, Mc, ldi, w, np, c0, li, lk); break;
                    case 2: p3_reduce_panel<2>(nxt, Mc, ldi, w, np, c0, li, lk); break;
                    case 3: p3_reduce_panel<3>(nxt, Mc, ldi, w, np, c0, li, lk); break;
                    default: p3_reduce_panel<4>(nxt, Mc, ldi, w, np, c0, li, lk); break;
                }
#pragma unroll
                for (int s = 0; s < P3_SLOTS; ++s) {
                    const int I = 3 * s + w;
                    if (I >= p + 2 && I < np) {
#pragma unroll
                        for (int kk = 0; kk < 16; kk += 4) {
                            const double av = -sm.Pn[par][p + 2][(kk + lk) * 16 + li];
                            const double bv = sm.Pn[par][I][(kk + lk) * 16 + li];
                            nxt[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, nxt[s], 0, 0, 0);
                        }
                        if (I == p + 2) {
#pragma unroll
                            for (int r = 0; r < 4; ++r) sm.Dn[(p + 2) & 1][(4 * r + lk) * P3_LD + li] = nxt[s][r];
                        }
                    }
                }
            }
        }
        p3_bar_all();   // D, Y of p+1; Cp; Dn; the L of panel p in global memory
    }
    __syncthreads();
    // log det: 2 log L_jj in parallel; the 64-block inverses; then a
    // fixed-order compensated sum (lane l of wavefront 0 sums entries l, l+64,
    // ..., then the lanes are joined pairwise by a butterfly)
    for (int t = threadIdx.x; t < m; t += 256) sm.dg[t] = 2.0 * log(sm.dg[t]);
    p3_inv64(Mc, ldi, X64, m, &sm.Pn[0][0][0]);
    __syncthreads();
    if (w == 0) {
        double ps = 0.0, pc = 0.0;
        for (int t = lane; t < m; t += 64) neumaier(ps, pc, sm.dg[t]);
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const double qs = __shfl_xor(ps, o), qc = __shfl_xor(pc, o);
            // the lower lane of each pair is the left operand, so both lanes agree
            const bool lo = (lane & o) == 0;
            const double a = lo ? ps : qs, b = lo ? qs : ps;
            const double t = a + b;
            const double e = (fabs(a) >= fabs(b)) ? (a - t) + b : (b - t) + a;
            pc = (lo ? pc + qc : qc + pc) + e;
            ps = t;
        }
        if (lane == 0) {
            *fail_out = fail;
            *ls_out = ps;
            *lc_out = pc;
        }
    }
}
